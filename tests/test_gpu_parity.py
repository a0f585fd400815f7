"""Parity of the HIP decoders with the CPU oracle (needs an MI355X).

Every GPU result is compared element by element with the float32 oracle on
the same seeded shots: corrections, flags, iteration counts, cut sets and the
float32 posteriors bit for bit (both sides take every floating-point decision
in float32, in the same order).  Against the float64 oracle the logical error
rate must agree within statistical error and posteriors of shots without
near-tie decisions within a relative 1e-3 (see the tolerance derivation in
the design doc's parity section).
"""
import numpy as np
import pytest

import oracle
import synth

from gpu_helpers import assert_bit_exact, gpu_decode, ler, oracle_params

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    import paper_2510_08695_amd as P
    P.lib()
    return P


def _code(name, p):
    if name == "toric6":
        return synth.toric_code(6, p=p)
    return synth.bb_code(name, p=p)


def _params(P, code, T=(50, 50), alpha=0.625, **kw):
    sp = P.PRIOR_POSTERIOR if code.second_pass == "posterior" else P.PRIOR_CHANNEL
    return P.Params(max_iter=T, alpha=alpha, second_pass_prior=sp, seed=kw.pop("seed", 17), **kw)


CASES = [
    # name, p, shots, T, kernels
    ("toric6", 0.05, 1000, (50, 50)),
    ("toric6", 0.09, 700, (50, 50)),
    ("bb144", 0.05, 1000, (100, 100)),
    ("bb144", 0.07, 600, (60, 40)),
    ("bb72", 0.06, 500, (40, 40)),
]


@pytest.mark.parametrize("kernel", ["lane", "plain"])
@pytest.mark.parametrize("name,p,shots,T", CASES)
def test_bit_exact_vs_float32_oracle(P, kernel, name, p, shots, T):
    code = _code(name, p)
    sh = synth.make_shots(code, shots, 1000 + shots)
    prm = _params(P, code, T=T)
    kid = P.KERNEL_LANE if kernel == "lane" else P.KERNEL_PLAIN
    c = P.Code.from_problem(code)
    plan = P.Plan([c], prm, kernel=kid)
    print(f"case {name} p={p} shots={shots} kernel={kernel}", flush=True)
    g = gpu_decode(plan, code, sh.syndromes, shot_offset=5)
    ref = oracle.decode(code, sh.syndromes, oracle_params(prm, code.second_pass), precision="f32",
                        shot_offset=5)
    assert ((ref["flags"] & 2) != 0).sum() > 0, "case must exercise DC"
    assert_bit_exact(g, ref, code.n)
    # converged outputs reproduce their syndromes
    conv = (g["flags"] & 1) != 0
    assert (synth.syndromes_of(g["ehat"][conv], code.H) == sh.syndromes[conv]).all()


@pytest.mark.parametrize("name,p,shots,T", [("bb144", 0.05, 3000, (100, 100)), ("toric6", 0.05, 3000, (50, 50))])
def test_float64_oracle_tolerances(P, name, p, shots, T):
    code = _code(name, p)
    sh = synth.make_shots(code, shots, 77)
    prm = _params(P, code, T=T)
    plan = P.Plan([P.Code.from_problem(code)], prm, kernel=P.KERNEL_LANE)
    g = gpu_decode(plan, code, sh.syndromes)
    r64 = oracle.decode(code, sh.syndromes, oracle_params(prm, code.second_pass), precision="f64")
    # logical error rates within statistical error
    a, b = ler(code, sh.errors, g), ler(code, sh.errors, r64)
    se = np.sqrt(max(b * (1 - b), 1.0 / shots) / shots)
    assert abs(a - b) <= 3 * se, (a, b)
    # hard decisions and cut sets agree on shots without near-tie decisions
    ok = r64["margin"] >= 1e-5
    assert ok.mean() > 0.95
    same = (g["ehat"] == r64["ehat"]).all(1) & (g["cut"] == r64["cut"]).all(1)
    assert same[ok].mean() >= 0.999
    # posteriors of unflagged shots that converged in the first pass
    sel = ok & ((r64["flags"] & 2) == 0)
    x, y = g["post"][sel].astype(np.float64), r64["post"][sel]
    rel = np.abs(x - y) / np.maximum(1.0, np.abs(y))
    assert rel.max() < 1e-3, rel.max()


def test_edge_cases(P):
    code = _code("bb144", 0.05)
    prm = _params(P, code, T=(20, 20))
    c = P.Code.from_problem(code)
    plan = P.Plan([c], prm, kernel=P.KERNEL_LANE)
    import torch
    # empty batch is a no-op
    syn0 = torch.zeros((0, 2), dtype=torch.int64, device="cuda")
    out = plan.decode(syn0)
    assert out["corr"].shape == (0, 3)
    # all-zero syndromes converge after one iteration with e_hat = 0
    z = np.zeros((130, code.m), np.uint8)
    g = gpu_decode(plan, code, z)
    assert (g["flags"] == 1).all() and (g["iters"][:, 0] == 1).all() and not g["ehat"].any()
    # single shots and ragged batch sizes agree with one big batch
    sh = synth.make_shots(code, 257, 5)
    full = gpu_decode(plan, code, sh.syndromes)
    for lo, hi in [(0, 1), (1, 65), (65, 257)]:
        part = gpu_decode(plan, code, sh.syndromes[lo:hi], shot_offset=lo)
        for k in ("ehat", "flags", "iters", "cut"):
            np.testing.assert_array_equal(part[k], full[k][lo:hi])


@pytest.mark.parametrize("variant", ["no_stop", "lowest_tie", "T1_is_1", "posterior_bb", "wide_eps"])
def test_parameter_variants_bit_exact(P, variant):
    code = _code("bb144", 0.06)
    sh = synth.make_shots(code, 400, 9)
    kw = {}
    T = (30, 30)
    sp_name = code.second_pass
    if variant == "no_stop":
        kw["stop_on_converge"] = False
    elif variant == "lowest_tie":
        kw["tie_break"] = P.TIE_LOWEST_INDEX
    elif variant == "T1_is_1":
        T = (1, 30)
    elif variant == "wide_eps":
        kw["tie_eps"] = 0.3
    prm = _params(P, code, T=T, **kw)
    if variant == "posterior_bb":
        prm.second_pass_prior = P.PRIOR_POSTERIOR
        sp_name = "posterior"
    for kid in (P.KERNEL_LANE, P.KERNEL_PLAIN):
        plan = P.Plan([P.Code.from_problem(code)], prm, kernel=kid)
        g = gpu_decode(plan, code, sh.syndromes, shot_offset=3)
        ref = oracle.decode(code, sh.syndromes, oracle_params(prm, sp_name), precision="f32", shot_offset=3)
        assert_bit_exact(g, ref, code.n)


def test_full_size_batch_sampled(P):
    """The benchmark workload (1e6 shots of [[144,12,12]] at p = 0.05, one launch):
    sampled contiguous blocks against the float32 oracle."""
    import torch
    code = _code("bb144", 0.05)
    B = 1_000_000
    sh = synth.make_shots(code, B, 2005)
    prm = _params(P, code, T=(100, 100))
    plan = P.Plan([P.Code.from_problem(code)], prm, kernel=P.KERNEL_LANE)
    syn = torch.from_numpy(synth.pack_bits(sh.syndromes).view(np.int64)).cuda()
    out = plan.decode(syn, want_cut=True, want_iters=True)
    torch.cuda.synchronize()
    corr = synth.unpack_bits(out["corr"].cpu().numpy().view(np.uint64), code.n)
    flags = out["flags"].cpu().numpy()
    iters = out["iters"].cpu().numpy()
    cut = synth.unpack_bits(out["cut"].cpu().numpy().view(np.uint64), code.n)
    for lo in (0, 333_333, 999_000):
        hi = lo + 1000
        ref = oracle.decode(code, sh.syndromes[lo:hi], oracle_params(prm, "channel"), precision="f32",
                            shot_offset=lo, want_post=False)
        np.testing.assert_array_equal(corr[lo:hi], ref["ehat"])
        np.testing.assert_array_equal(flags[lo:hi], ref["flags"])
        np.testing.assert_array_equal(iters[lo:hi], ref["iters"])
        np.testing.assert_array_equal(cut[lo:hi], ref["cut"])
    # properties that hold at any size
    conv = (flags & 1) != 0
    assert (synth.syndromes_of(corr[conv][:200000], code.H) == sh.syndromes[conv][:200000]).all()
    dc = (flags & 2) != 0
    assert (iters[dc, 0] == 100).all() and (iters[~dc, 1] == 0).all()
    assert not (corr & cut).any()


@pytest.mark.parametrize("variant", ["soft_lane", "soft_group", "ps_group", "circuit_group"])
def test_edge_cases_other_kernel_modes(P, variant):
    """Empty batches, all-zero syndromes, single shots and ragged sub-batches (with the
    matching shot offsets) on the soft-DC lane variant, soft DC and product-sum on the
    group kernel, and the group kernel's 64-bit check records."""
    import torch
    if variant == "ps_group":
        code = synth.toric_code(6, p=0.05)
        prm = P.Params(max_iter=(30, 30), alpha=1.0, second_pass_prior=P.PRIOR_POSTERIOR, seed=2,
                       rule=P.RULE_PRODUCT_SUM)
    elif variant == "circuit_group":
        code = synth.bb_circuit_dem("bb72", 2, 0.004)
        prm = P.Params(max_iter=(60, 20), alpha=0.625, second_pass_prior=P.PRIOR_CHANNEL, seed=2)
    else:
        code = _code("bb144", 0.06)
        prm = P.Params(max_iter=(40, 20), alpha=0.625, second_pass_prior=P.PRIOR_CHANNEL, seed=2,
                       soft_period=3, soft_shift=1.0)
    kid = P.KERNEL_LANE if variant == "soft_lane" else P.KERNEL_GROUP
    plan = P.Plan([P.Code.from_problem(code)], prm, kernel=kid)
    nw_s, nw_c = (code.m + 63) // 64, (code.n + 63) // 64
    out = plan.decode(torch.zeros((0, nw_s), dtype=torch.int64, device="cuda"))
    assert out["corr"].shape == (0, nw_c)
    z = np.zeros((70, code.m), np.uint8)
    g = gpu_decode(plan, code, z)
    assert (g["flags"] == 1).all() and (g["iters"][:, 0] == 1).all() and not g["ehat"].any()
    sh = synth.make_shots(code, 200, 9)
    off = 10 ** 12
    full = gpu_decode(plan, code, sh.syndromes, shot_offset=off)
    for lo, hi in [(0, 1), (1, 64), (64, 200)]:
        part = gpu_decode(plan, code, sh.syndromes[lo:hi], shot_offset=off + lo)
        for k in ("ehat", "flags", "iters", "cut"):
            np.testing.assert_array_equal(part[k], full[k][lo:hi])
    ps = variant == "ps_group"
    ref = oracle.decode(code, sh.syndromes, oracle_params(prm, "posterior" if ps else "channel"),
                        precision="f64" if ps else "f32", shot_offset=off)
    if not ps:
        assert_bit_exact(full, ref, code.n)
    else:  # product-sum: the float64 oracle's decisions on shots with clear margins
        np.testing.assert_array_equal(full["ehat"][ref["margin"] >= 1e-3], ref["ehat"][ref["margin"] >= 1e-3])
