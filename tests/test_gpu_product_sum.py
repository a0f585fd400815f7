"""Product-sum BP+DC on the GPU against the float64 oracle (needs an MI355X).

The product-sum check rule (Sec. II.C; used by the paper for surface codes),
on the plain kernel family and on the lane family (one lane per shot),
evaluates tanh and atanh, whose float32 implementations on the GPU and in the
host's C library may differ in the last bit; near a saturated product the
difference is amplified, and on shots whose BP does not settle the float32
and float64 trajectories part (the float32 and float64 oracles themselves
disagree on ~3 % of non-converging surface-code shots).  The parity bar is
therefore:
  * on every shot whose float64 decode keeps all decision margins (|q| at sign
    tests, |L| at hard decisions) at or above 1e-3, corrections, flags and
    iteration counts equal the float64 oracle's;
  * the first-pass failure rate and the logical error rate over all shots
    agree with the float64 oracle's within 4 binomial standard deviations;
  * on every shot: a shot flagged converged satisfies H e = s, cut columns
    have correction 0 and posterior +inf, and hard decisions are the signs of
    the posteriors.
"""
import numpy as np
import pytest

import oracle
import synth

from gpu_helpers import gpu_decode, oracle_params

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    import paper_2510_08695_amd as P
    P.lib()
    return P


def _code(name, p):
    if name.startswith("surface"):
        return synth.rotated_surface_code(int(name[7:]), p=p)
    return synth.toric_code(int(name[5:]), p=p)


CASES = [
    # name, p, shots, T (= n for the surface codes, Fig. 2 caption)
    ("surface7", 0.01, 6000, 49),
    ("surface5", 0.03, 4000, 25),
    ("toric6", 0.05, 3000, 50),
]


def _two_prop_ok(a, b, n):
    p = (a + b) / (2 * n)
    sd = np.sqrt(max(p * (1 - p), 1e-12) * 2 / n)
    return abs(a - b) / n <= 4 * sd + 1.0 / n


def _kernels(P, name):
    # the lane family runs product-sum for codes of at most 96 edges (the surface codes here);
    # the group family for rows of at most 8 edges (all of them)
    return [P.KERNEL_PLAIN, P.KERNEL_GROUP] + ([P.KERNEL_LANE] if name.startswith("surface") else [])


@pytest.mark.parametrize("kname", ["plain", "lane", "group"])
@pytest.mark.parametrize("name,p,shots,T", CASES)
def test_product_sum_vs_float64_oracle(P, kname, name, p, shots, T):
    code = _code(name, p)
    kid = {"plain": P.KERNEL_PLAIN, "lane": P.KERNEL_LANE, "group": P.KERNEL_GROUP}[kname]
    if kid not in _kernels(P, name):
        pytest.skip("the lane family runs product-sum for codes of at most 96 edges")
    sh = synth.make_shots(code, shots, 5000 + shots)
    prm = P.Params(max_iter=(T, T), alpha=1.0, second_pass_prior=P.PRIOR_POSTERIOR, seed=23,
                   rule=P.RULE_PRODUCT_SUM)
    plan = P.Plan([P.Code.from_problem(code)], prm, kernel=kid)
    g = gpu_decode(plan, code, sh.syndromes)
    _check_vs_float64_oracle(P, code, sh, prm, g, shots)


def _check_vs_float64_oracle(P, code, sh, prm, g, shots):
    ref = oracle.decode(code, sh.syndromes, oracle_params(prm, "posterior"), precision="f64")
    # decisions on shots with clear margins
    sel = ref["margin"] >= 1e-3
    assert sel.mean() > 0.5
    np.testing.assert_array_equal(g["flags"][sel], ref["flags"][sel])
    np.testing.assert_array_equal(g["iters"][sel], ref["iters"][sel])
    np.testing.assert_array_equal(g["ehat"][sel], ref["ehat"][sel])
    # rates over all shots
    n_dc_g, n_dc_r = int(((g["flags"] & 2) != 0).sum()), int(((ref["flags"] & 2) != 0).sum())
    assert _two_prop_ok(n_dc_g, n_dc_r, shots), (n_dc_g, n_dc_r)

    def fails(out):
        return int((((out["flags"] & 1) == 0) | synth.residual_is_logical(sh.errors ^ out["ehat"], code.O)).sum())
    assert _two_prop_ok(fails(g), fails(ref), shots), (fails(g), fails(ref))
    # invariants on every shot
    H = code.H.to_dense().astype(np.int64)
    conv = (g["flags"] & 1) != 0
    s_hat = (g["ehat"].astype(np.int64) @ H.T) % 2
    assert (s_hat[conv] == sh.syndromes[conv]).all()
    cut = g["cut"].astype(bool)
    assert not (g["ehat"].astype(bool) & cut).any()
    assert np.isinf(g["post"][cut]).all() and (g["post"][cut] > 0).all()
    assert not cut[(g["flags"] & 2) == 0].any()
    np.testing.assert_array_equal(g["ehat"].astype(bool), g["post"] <= 0)
    return ref


@pytest.mark.parametrize("name,p,shots,T", [("surface5", 0.03, 4000, 25), ("toric6", 0.05, 3000, 50)])
def test_product_sum_soft_dc(P, name, p, shots, T):
    """Product-sum with intermittent soft DC (K = 5, beta = 0.5) on the plain and
    group kernels: the float64 oracle's bar above, and the group kernel's outputs
    equal to the plain kernel's bit for bit."""
    code = _code(name, p)
    sh = synth.make_shots(code, shots, 7000 + shots)
    prm = P.Params(max_iter=(T, T), alpha=1.0, second_pass_prior=P.PRIOR_POSTERIOR, seed=31,
                   rule=P.RULE_PRODUCT_SUM, soft_period=5, soft_shift=0.5)
    c = P.Code.from_problem(code)
    print(f"case {name} p={p} product-sum soft DC", flush=True)
    a = gpu_decode(P.Plan([c], prm, kernel=P.KERNEL_PLAIN), code, sh.syndromes)
    ref = _check_vs_float64_oracle(P, code, sh, prm, a, shots)
    assert (((ref["flags"] & 2) != 0) | (ref["iters"][:, 0] > 5)).sum() > 0
    b = gpu_decode(P.Plan([c], prm, kernel=P.KERNEL_GROUP), code, sh.syndromes)
    for k in ("flags", "iters", "ehat", "cut"):
        np.testing.assert_array_equal(a[k], b[k], err_msg=k)
    np.testing.assert_array_equal(a["post"].view(np.uint32), b["post"].view(np.uint32))
    # soft DC changed the decoding
    off = oracle.decode(code, sh.syndromes, oracle_params(P.Params(max_iter=(T, T), alpha=1.0,
                                                                   second_pass_prior=P.PRIOR_POSTERIOR, seed=31,
                                                                   rule=P.RULE_PRODUCT_SUM), "posterior"),
                        precision="f64", want_post=False)
    assert (off["iters"] != ref["iters"]).any()


@pytest.mark.parametrize("name,p,shots,T", CASES)
def test_product_sum_kernels_equal_bit_for_bit(P, name, p, shots, T):
    """The GPU product-sum decoders evaluate tanh and atanh with the same float32
    functions, in the same order (leave-one-out products left to right in column
    order, column sums in ascending check order): every output of the lane (surface
    codes) and group kernels equals the plain kernel's."""
    code = _code(name, p)
    sh = synth.make_shots(code, shots, 6000 + shots)
    prm = P.Params(max_iter=(T, T), alpha=1.0, second_pass_prior=P.PRIOR_POSTERIOR, seed=29,
                   rule=P.RULE_PRODUCT_SUM)
    c = P.Code.from_problem(code)
    a = gpu_decode(P.Plan([c], prm, kernel=P.KERNEL_PLAIN), code, sh.syndromes)
    for kid in _kernels(P, name)[1:]:
        b = gpu_decode(P.Plan([c], prm, kernel=kid), code, sh.syndromes)
        for k in ("flags", "iters", "ehat", "cut"):
            np.testing.assert_array_equal(a[k], b[k], err_msg=f"kernel {kid} {k}")
        np.testing.assert_array_equal(a["post"].view(np.uint32), b["post"].view(np.uint32))


@pytest.mark.parametrize("name,p,shots,T", [("surface5", 0.03, 3000, 25), ("surface7", 0.01, 4000, 49)])
def test_product_sum_low_saturation(P, name, p, shots, T):
    """llr_sat = 8, below the level where float32 tanh(|q| / 2) reaches 1: messages from cut
    columns (posterior +inf) and from columns whose posterior exceeds 8 must be held at 8
    before tanh (q = sat(L - r), Sec. II.C), or they would send tanh = 1 instead of tanh(4).
    The lane (surface codes), group and plain kernels agree bit for bit and meet the float64
    oracle's product-sum bar at this saturation."""
    code = _code(name, p)
    sh = synth.make_shots(code, shots, 8000 + shots)
    prm = P.Params(max_iter=(T, T), alpha=1.0, second_pass_prior=P.PRIOR_POSTERIOR, seed=37,
                   rule=P.RULE_PRODUCT_SUM, llr_sat=8.0)
    c = P.Code.from_problem(code)
    print(f"case {name} p={p} product-sum llr_sat=8", flush=True)
    a = gpu_decode(P.Plan([c], prm, kernel=P.KERNEL_PLAIN), code, sh.syndromes)
    ref = _check_vs_float64_oracle(P, code, sh, prm, a, shots)
    assert ((ref["flags"] & 2) != 0).sum() > 10
    for kid in _kernels(P, name)[1:]:
        b = gpu_decode(P.Plan([c], prm, kernel=kid), code, sh.syndromes)
        for k in ("flags", "iters", "ehat", "cut"):
            np.testing.assert_array_equal(a[k], b[k], err_msg=f"kernel {kid} {k}")
        np.testing.assert_array_equal(a["post"].view(np.uint32), b["post"].view(np.uint32))


def test_product_sum_plans(P):
    prm = P.Params(max_iter=(25, 25), alpha=1.0, second_pass_prior=P.PRIOR_POSTERIOR, rule=P.RULE_PRODUCT_SUM)
    small = P.Code.from_problem(synth.rotated_surface_code(5, p=0.03))
    assert P.Plan([small], prm, kernel=P.KERNEL_AUTO).info(0)["kernel"] == P.KERNEL_LANE
    big = P.Code.from_problem(synth.toric_code(6, p=0.05))  # 144 edges: group kernel
    assert P.Plan([big], prm, kernel=P.KERNEL_AUTO).info(0)["kernel"] == P.KERNEL_GROUP
    with pytest.raises(P.BpdcError):
        P.Plan([big], prm, kernel=P.KERNEL_LANE)
    # rows of 9 to 32 edges: the plain kernel (AUTO), not the group kernel
    wide = P.Code.from_problem(synth.hgp_code(synth.random_regular_classical(12, 5, dv=3, dc=6),
                                              with_logicals=False, p=0.03))
    psc = P.Params(max_iter=(25, 25), alpha=1.0, second_pass_prior=P.PRIOR_CHANNEL, rule=P.RULE_PRODUCT_SUM)
    assert P.Plan([wide], psc, kernel=P.KERNEL_AUTO).info(0)["kernel"] == P.KERNEL_PLAIN
    with pytest.raises(P.BpdcError):
        P.Plan([wide], psc, kernel=P.KERNEL_GROUP)
    # rows above 32 edges (a circuit-level DEM has 35): no product-sum kernel
    circ = P.Code.from_problem(synth.bb_circuit_dem("bb72", 2, 0.002))
    with pytest.raises(P.BpdcError):
        P.Plan([circ], psc, kernel=P.KERNEL_PLAIN)
