"""bpdc_decode_noalloc (the entry point that allocates nothing: its workspace is the
library's static device scratch) against bpdc_decode with a caller workspace (GPU).

For each kernel family, two calls in a row through the C ABI, the second on a smaller
batch at a shot offset (the scratch keeps the first call's contents, so anything the
kernels fail to clear would show), each compared output by output, bit for bit, with
bpdc_decode on the same shots; and a batch whose workspace exceeds the scratch is
refused before any launch."""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    import paper_2510_08695_amd as P
    P.lib()
    return P


def _syn(code, B, seed):
    import torch
    sh = synth.make_shots(code, B, seed)
    return torch.from_numpy(synth.pack_bits(sh.syndromes).view(np.int64)).cuda()


def _same(a, b):
    for k in ("corr", "flags", "post", "cut", "iters"):
        assert a[k].dtype == b[k].dtype
        x, y = a[k].cpu().numpy(), b[k].cpu().numpy()
        if x.dtype == np.float32:
            x, y = x.view(np.uint32), y.view(np.uint32)
        np.testing.assert_array_equal(x, y, err_msg=k)


@pytest.mark.parametrize("family,B1,B2", [("lane", 20000, 3000), ("group", 4000, 700), ("plain", 3000, 500)])
def test_noalloc_equals_decode_on_two_calls(P, family, B1, B2):
    import torch
    code = synth.bb_code("bb144", p=0.06)
    kid = {"lane": P.KERNEL_LANE, "group": P.KERNEL_GROUP, "plain": P.KERNEL_PLAIN}[family]
    prm = P.Params(max_iter=(60, 60), alpha=0.625, second_pass_prior=P.PRIOR_CHANNEL, seed=17)
    plan = P.Plan([P.Code.from_problem(code)], prm, kernel=kid)
    syn = _syn(code, B1, 901)
    for B, off in ((B1, 0), (B2, 12345)):
        s = syn[:B].contiguous()
        print(f"case noalloc {family} B={B} offset={off}", flush=True)
        a = plan.decode_noalloc(s, shot_offset=off, want_post=True, want_cut=True, want_iters=True)
        b = plan.decode(s, shot_offset=off, want_post=True, want_cut=True, want_iters=True)
        torch.cuda.synchronize()
        assert ((a["flags"] & 2) != 0).sum().item() > 10
        _same(a, b)


def test_noalloc_refuses_a_batch_beyond_the_scratch(P):
    import torch
    code = synth.bb_code("bb144", p=0.06)
    prm = P.Params(max_iter=(20, 20))
    plan = P.Plan([P.Code.from_problem(code)], prm, kernel=P.KERNEL_PLAIN)
    B = 20000      # the plain family needs ~4.7 kB of workspace per BB144 shot: ~94 MB
    syn = torch.zeros((B, 2), dtype=torch.int64, device="cuda")
    with pytest.raises(P.BpdcError, match="static scratch"):
        plan.decode_noalloc(syn)
