"""Parity at the full sizes of the phenomenological and uneven-batch configurations (GPU).

* BB[[288,12,18]] phenomenological noise, T = 18 rounds, p = 0.003 on every column,
  1000 + 1000 iterations (Fig. 5 caption), channel second-pass prior, in both
  time-boundary forms (Sec. IV.C: the paper's, with a final noiseless round,
  2736 x 8064; and the open one, 2592 x 7776): one launch of the group kernel over
  the whole batch (1e5 shots open, 5e4 paper), then three blocks of 400 shots and up
  to 40 more shots that ran DC, each bit-exact with the float32 oracle (corrections,
  flags, iteration counts, cut), and properties of every shot.
* 64 hypergraph-product codes (n from 400 to 6400), Poisson(2000) shots each in a
  seeded random order, p = 0.03, 100 + 100 iterations, in one graph-captured
  multi-code launch: 20 shots of every code plus up to 5 that ran DC, bit-exact with
  the float32 oracle at their global shot index, and properties of every shot.
"""
import numpy as np
import pytest

import oracle
import synth

from gpu_helpers import oracle_params

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    import paper_2510_08695_amd as P
    P.lib()
    return P


def _check_rows(code, syndromes, prm, rows, out, sp="channel"):
    """Oracle (float32) on the listed shots, each at its own global index."""
    rows = np.asarray(sorted(set(int(r) for r in rows)))
    # contiguous runs decode in one oracle call
    starts = np.nonzero(np.diff(np.concatenate([[-2], rows])) != 1)[0]
    ends = np.concatenate([starts[1:], [len(rows)]])
    for a, b in zip(starts, ends):
        lo, hi = rows[a], rows[b - 1] + 1
        ref = oracle.decode(code, syndromes[lo:hi], oracle_params(prm, sp), precision="f32", shot_offset=lo,
                            want_post=False)
        for k in ("ehat", "flags", "iters", "cut"):
            np.testing.assert_array_equal(out[k][lo:hi], ref[k], err_msg=f"{k} shots {lo}:{hi}")
    return len(rows)


def _properties(code, syndromes, out, T1):
    conv = (out["flags"] & 1) != 0
    assert (synth.syndromes_of(out["ehat"][conv], code.H) == syndromes[conv]).all()
    dc = (out["flags"] & 2) != 0
    assert (out["iters"][dc, 0] == T1).all() and (out["iters"][~dc, 1] == 0).all()
    assert not (out["ehat"].astype(bool) & out["cut"].astype(bool)).any()
    assert not out["cut"][~dc].any()
    nc = out["cut"][dc].sum(1)
    assert (nc > 0).all() and (nc <= code.D.rows).all()


@pytest.mark.parametrize("form,B", [("open", 100_000), ("paper", 50_000)])
def test_phenomenological_bb288_T18_full_size(P, form, B):
    import torch
    code = synth.phenomenological_dem(synth.bb_code("bb288"), 18, 0.003, 0.003, form == "paper")
    sh = synth.make_shots(code, B, 3)
    prm = P.Params(max_iter=(1000, 1000), alpha=0.625, second_pass_prior=P.PRIOR_CHANNEL, seed=3)
    plan = P.Plan([P.Code.from_problem(code)], prm, kernel=P.KERNEL_GROUP)
    syn = torch.from_numpy(synth.pack_bits(sh.syndromes).view(np.int64)).cuda()
    print(f"case phenomenological bb288 T=18 {form} {code.H.rows}x{code.n} B={B} group", flush=True)
    o = plan.decode(syn, want_cut=True, want_iters=True)
    torch.cuda.synchronize()
    out = {"ehat": synth.unpack_bits(o["corr"].cpu().numpy().view(np.uint64), code.n),
           "cut": synth.unpack_bits(o["cut"].cpu().numpy().view(np.uint64), code.n),
           "flags": o["flags"].cpu().numpy(), "iters": o["iters"].cpu().numpy().astype(np.int32)}
    _properties(code, sh.syndromes, out, 1000)
    dc = np.nonzero(out["flags"] & 2)[0]
    assert len(dc) > 30     # open form ~1.4 % of shots, paper form ~0.16 %
    rows = list(range(0, 400)) + list(range(B // 2, B // 2 + 400)) + list(range(B - 400, B))
    extra = [int(b) for b in np.random.default_rng(1).permutation(dc) if b not in set(rows)][:40]
    checked = _check_rows(code, sh.syndromes, prm, rows + extra, out)
    print(f"  {checked} shots bit-exact, {len(dc)} of {B} ran DC", flush=True)


def test_hgp64_uneven_batch_graph_launch(P):
    import torch
    codes = synth.hgp_batch_codes(64, 4000, 0.03, with_logicals=False)
    code_of_shot, syn, per = synth.mixed_batch(codes, 2000, 4, 4100)
    B = len(code_of_shot)
    prm = P.Params(max_iter=(100, 100), alpha=0.625, second_pass_prior=P.PRIOR_CHANNEL, seed=4)
    plan = P.Plan([P.Code.from_problem(c) for c in codes], prm, kernel=P.KERNEL_GROUP)
    cos = torch.from_numpy(code_of_shot).cuda()
    so, co, sw, nw = plan.multi_buffers(cos)
    syn_t = torch.from_numpy(syn).cuda()
    corr = torch.full((nw,), -1, dtype=torch.int64, device="cuda")
    flags = torch.zeros(B, dtype=torch.uint8, device="cuda")
    iters = torch.zeros((B, 2), dtype=torch.int16, device="cuda")
    print(f"case hgp64 uneven batch B={B} graph launch", flush=True)
    plan.capture_multi(cos, syn_t, so, corr, co, flags, iters)
    plan.graph_launch()
    torch.cuda.synchronize()
    corr_h, flags_h, iters_h, co_h = (corr.cpu().numpy(), flags.cpu().numpy(), iters.cpu().numpy(),
                                      co.cpu().numpy())
    assert not (flags_h & 0x80).any()
    op = oracle_params(prm, "channel")
    rng = np.random.default_rng(2)
    n_checked, n_dc = 0, 0
    for i, c in enumerate(codes):
        idx, sh = per[i]
        nwi = (c.n + 63) // 64
        words = np.stack([corr_h[co_h[b]:co_h[b] + nwi] for b in idx]).view(np.uint64)
        out = {"ehat": synth.unpack_bits(words, c.n), "flags": flags_h[idx], "iters": iters_h[idx].astype(np.int32)}
        # properties of every shot of the code
        conv = (out["flags"] & 1) != 0
        assert (synth.syndromes_of(out["ehat"][conv], c.H) == sh.syndromes[conv]).all()
        dc = (out["flags"] & 2) != 0
        assert (out["iters"][dc, 0] == 100).all() and (out["iters"][~dc, 1] == 0).all()
        n_dc += int(dc.sum())
        pick = list(range(min(20, len(idx)))) + [int(k) for k in rng.permutation(np.nonzero(dc)[0])[:5]]
        for k in sorted(set(pick)):
            ref = oracle.decode(c, sh.syndromes[k:k + 1], op, precision="f32", shot_offset=int(idx[k]),
                                want_post=False)
            np.testing.assert_array_equal(out["ehat"][k], ref["ehat"][0], err_msg=f"code {i} shot {idx[k]}")
            assert out["flags"][k] == ref["flags"][0], (i, idx[k])
            np.testing.assert_array_equal(out["iters"][k], ref["iters"][0])
            n_checked += 1
    assert n_dc > 50
    print(f"  {n_checked} shots of 64 codes bit-exact; {n_dc} of {B} ran DC", flush=True)
