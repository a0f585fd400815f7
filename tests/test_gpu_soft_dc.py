"""Intermittent soft DC (the extension proposed in Sec. V) on the GPU against the
float32 oracle (needs an MI355X): every K first-pass iterations, while H e != s,
DC's nominees get their prior LLR raised by beta.  Lane, group and plain kernel
families; every output bit-exact with the float32 oracle."""
import numpy as np
import pytest

import oracle
import synth

from gpu_helpers import assert_bit_exact, gpu_decode, oracle_params

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    import paper_2510_08695_amd as P
    P.lib()
    return P


def _code(name, p):
    return synth.toric_code(6, p=p) if name == "toric6" else synth.bb_code(name, p=p)


CASES = [
    # name, p, shots, T, K, beta, stop
    ("bb144", 0.05, 1500, (100, 100), 5, 0.5, True),
    ("bb144", 0.06, 800, (60, 40), 10, 2.0, True),
    ("bb72", 0.06, 800, (40, 40), 3, 0.75, False),
    ("toric6", 0.07, 1000, (50, 50), 4, 1.0, True),
]


@pytest.mark.parametrize("kernel", ["lane", "group", "plain"])
@pytest.mark.parametrize("name,p,shots,T,K,beta,stop", CASES)
def test_soft_dc_bit_exact_vs_float32_oracle(P, kernel, name, p, shots, T, K, beta, stop):
    code = _code(name, p)
    sh = synth.make_shots(code, shots, 9000 + shots)
    sp = P.PRIOR_POSTERIOR if code.second_pass == "posterior" else P.PRIOR_CHANNEL
    prm = P.Params(max_iter=T, alpha=0.625, second_pass_prior=sp, seed=41, stop_on_converge=stop,
                   soft_period=K, soft_shift=beta)
    kid = {"lane": P.KERNEL_LANE, "group": P.KERNEL_GROUP, "plain": P.KERNEL_PLAIN}[kernel]
    plan = P.Plan([P.Code.from_problem(code)], prm, kernel=kid)
    print(f"case {name} p={p} K={K} beta={beta} stop={stop} kernel={kernel}", flush=True)
    g = gpu_decode(plan, code, sh.syndromes, shot_offset=7)
    ref = oracle.decode(code, sh.syndromes, oracle_params(prm, code.second_pass), precision="f32", shot_offset=7)
    assert ((ref["flags"] & 2) != 0).sum() > 0
    assert_bit_exact(g, ref, code.n)
    # soft DC changed the decoding (against BP+DC without it)
    off = oracle.decode(code, sh.syndromes, oracle_params(P.Params(max_iter=T, alpha=0.625, second_pass_prior=sp,
                                                                   seed=41, stop_on_converge=stop),
                                                          code.second_pass), precision="f32", shot_offset=7,
                        want_post=False)
    assert (off["iters"] != ref["iters"]).any()


def test_soft_dc_plans(P):
    code = P.Code.from_problem(synth.bb_code("bb144", p=0.05))
    prm = P.Params(max_iter=(50, 50), soft_period=5, soft_shift=0.5)
    assert P.Plan([code], prm, kernel=P.KERNEL_AUTO).info(0)["kernel"] == P.KERNEL_LANE
    # product-sum with soft DC: the group kernel (rows of at most 8 edges), else plain;
    # the lane family has no product-sum soft variant
    surf = P.Code.from_problem(synth.rotated_surface_code(5, p=0.03))
    ps = P.Params(max_iter=(25, 25), alpha=1.0, second_pass_prior=P.PRIOR_POSTERIOR, rule=P.RULE_PRODUCT_SUM,
                  soft_period=5, soft_shift=0.5)
    assert P.Plan([surf], ps, kernel=P.KERNEL_AUTO).info(0)["kernel"] == P.KERNEL_GROUP
    with pytest.raises(P.BpdcError):
        P.Plan([surf], ps, kernel=P.KERNEL_LANE)
    wide = P.Code.from_problem(synth.hgp_code(synth.random_regular_classical(12, 5, dv=3, dc=6),
                                              with_logicals=False, p=0.03))
    psc = P.Params(max_iter=(25, 25), alpha=1.0, second_pass_prior=P.PRIOR_CHANNEL, rule=P.RULE_PRODUCT_SUM,
                   soft_period=5, soft_shift=0.5)
    assert P.Plan([wide], psc, kernel=P.KERNEL_AUTO).info(0)["kernel"] == P.KERNEL_PLAIN
    for bad in (dict(soft_period=-1), dict(soft_period=5, soft_shift=-1.0), dict(soft_period=5, soft_shift=float("inf"))):
        with pytest.raises(P.BpdcError):
            P.Plan([code], P.Params(max_iter=(50, 50), **bad), kernel=P.KERNEL_GROUP)


def test_soft_dc_multi_code_launch(P):
    """The multi-code group launch runs soft DC too (two codes, mixed shots, each shot
    checked against the float32 oracle at its index in the mixed batch)."""
    from test_gpu_group import _check_multi, _mixed_batch, _run_multi
    codes = [synth.bb_code("bb72", p=0.06), synth.bb_code("bb144", p=0.05)]
    prm = P.Params(max_iter=(60, 60), alpha=0.625, second_pass_prior=P.PRIOR_CHANNEL, seed=5,
                   soft_period=6, soft_shift=1.0)
    plan = P.Plan([P.Code.from_problem(c) for c in codes], prm, kernel=P.KERNEL_GROUP)
    code_of_shot, syn, per_code = _mixed_batch(P, codes, [70, 90], 91)
    outs, corr_off = _run_multi(P, plan, codes, code_of_shot, syn)
    _check_multi(P, prm, codes, per_code, outs[0], corr_off)


def test_soft_dc_lane_full_size_sampled(P):
    """The benchmark configuration (BB144, p = 0.05, 1e6 shots, K = 5, beta = 0.5) on
    the lane kernel in one launch: sampled blocks bit-exact with the float32 oracle,
    and every output equal to the group kernel's on the same shots."""
    import torch
    code = synth.bb_code("bb144", p=0.05)
    B = 1_000_000
    sh = synth.make_shots(code, B, 2005)
    prm = P.Params(max_iter=(100, 100), alpha=0.625, second_pass_prior=P.PRIOR_CHANNEL, seed=1,
                   soft_period=5, soft_shift=0.5)
    syn = torch.from_numpy(synth.pack_bits(sh.syndromes).view(np.int64)).cuda()
    outs = {}
    for kid in (P.KERNEL_LANE, P.KERNEL_GROUP):
        plan = P.Plan([P.Code.from_problem(code)], prm, kernel=kid)
        o = plan.decode(syn, want_cut=True, want_iters=True)
        torch.cuda.synchronize()
        outs[kid] = {k: v.cpu().numpy() for k, v in o.items() if v is not None}
    for k in outs[P.KERNEL_LANE]:
        np.testing.assert_array_equal(outs[P.KERNEL_LANE][k], outs[P.KERNEL_GROUP][k], err_msg=k)
    corr = synth.unpack_bits(outs[P.KERNEL_LANE]["corr"].view(np.uint64), code.n)
    for lo in (0, 500_000, 999_000):
        hi = lo + 1000
        ref = oracle.decode(code, sh.syndromes[lo:hi], oracle_params(prm, "channel"), precision="f32",
                            shot_offset=lo, want_post=False)
        np.testing.assert_array_equal(corr[lo:hi], ref["ehat"])
        np.testing.assert_array_equal(outs[P.KERNEL_LANE]["flags"][lo:hi], ref["flags"])
        np.testing.assert_array_equal(outs[P.KERNEL_LANE]["iters"][lo:hi], ref["iters"])


def test_soft_dc_lane_zero_shift_equals_bpdc(P):
    """beta = 0: the lane kernel's soft-DC variant reproduces the headline lane
    kernel's outputs bit for bit (the nominations run but shift nothing)."""
    code = synth.bb_code("bb144", p=0.05)
    sh = synth.make_shots(code, 3000, 9400)
    base = P.Params(max_iter=(100, 100), alpha=0.625, second_pass_prior=P.PRIOR_CHANNEL, seed=3)
    zero = P.Params(max_iter=(100, 100), alpha=0.625, second_pass_prior=P.PRIOR_CHANNEL, seed=3,
                    soft_period=4, soft_shift=0.0)
    c = P.Code.from_problem(code)
    a = gpu_decode(P.Plan([c], base, kernel=P.KERNEL_LANE), code, sh.syndromes)
    b = gpu_decode(P.Plan([c], zero, kernel=P.KERNEL_LANE), code, sh.syndromes)
    for k in ("flags", "iters", "ehat", "cut"):
        np.testing.assert_array_equal(a[k], b[k])
    np.testing.assert_array_equal(a["post"].view(np.uint32), b["post"].view(np.uint32))


def test_soft_dc_lane_dc_stats_equal_plain(P):
    """DC diagnostics of a soft-DC decode: the lane kernel's soft variant and the
    plain kernel count the same DC shots, cut sizes and spread bins."""
    import torch
    code = synth.bb_code("bb144", p=0.06)
    sh = synth.make_shots(code, 4000, 9500)
    prm = P.Params(max_iter=(60, 60), alpha=0.625, second_pass_prior=P.PRIOR_CHANNEL, seed=8,
                   soft_period=5, soft_shift=0.5)
    stats = []
    for kid in (P.KERNEL_LANE, P.KERNEL_PLAIN):
        plan = P.Plan([P.Code.from_problem(code)], prm, kernel=kid)
        st = torch.zeros(103 + code.n, dtype=torch.int64, device="cuda")
        plan.set_dc_stats(st)
        gpu_decode(plan, code, sh.syndromes, want_post=False)
        stats.append(st.cpu().numpy())
    assert stats[0][101] > 0
    np.testing.assert_array_equal(stats[0], stats[1])
