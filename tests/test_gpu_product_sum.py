"""Product-sum BP+DC on the GPU against the float64 oracle (needs an MI355X).

The product-sum check rule (Sec. II.C; used by the paper for surface codes) is
evaluated in the log domain by every decoder here, r = phi(sum of phi(|q|)) with
phi(x) = -ln tanh(x/2): the GPU kernels with their own float32 phi (tested below
against float64 on a dense grid), the oracle with the host library's
log1p / expm1.  The parity bar is the float64 tier of the min-sum decoder:
  * on every shot whose float64 decode keeps all decision margins (|q| at sign
    tests, |L| at hard decisions, DC tie gaps) at or above 1e-5 ("unflagged"),
    corrections, flags, iteration counts and cuts equal the float64 oracle's;
  * hard decisions agree on at least 99.99 % of all shots, any disagreeing bit
    with |L64| < 1e-3;
  * posteriors within 1e-4 max(1, |L64|) on unflagged shots whose float64
    posteriors move by at most 2.5e-5 (relative) under a one-ulp change of the
    priors (well-conditioned), and within max(1e-4, 4 x that sensitivity) on
    every unflagged shot;
  * the first-pass failure rate and the logical error rate agree with the
    float64 oracle's within 4 binomial standard deviations;
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
    from test_gpu_fp64_tier import _rel_post_err, sensitivity
    op = oracle_params(prm, "posterior")
    ref = oracle.decode(code, sh.syndromes, op, precision="f64")
    # every output on unflagged shots
    sel = ref["margin"] >= 1e-5
    assert sel.mean() > 0.5
    for k in ("flags", "iters", "ehat", "cut"):
        np.testing.assert_array_equal(g[k][sel], ref[k][sel], err_msg=k)
    # hard decisions over all shots
    same = (g["ehat"] == ref["ehat"]).all(1)
    assert same.mean() >= 0.9999
    dis = g["ehat"] != ref["ehat"]
    if dis.any():
        assert np.abs(ref["post"][dis]).max() < 1e-3
    # posteriors
    sens = sensitivity(code, sh.syndromes, op, ref)
    err = _rel_post_err(g["post"], ref["post"])
    well = sel & (sens <= 2.5e-5)
    assert well.mean() > 0.5
    assert err[well].max() <= 1e-4, err[well].max()
    assert (err[sel] <= np.maximum(1e-4, 4 * sens[sel])).all()
    print(f"  unflagged {sel.mean():.4f}, well-conditioned {well.mean():.4f}, max posterior error there "
          f"{err[well].max():.2e}", flush=True)
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


def test_phi_accuracy_against_float64(P):
    """The library's float32 phi(x) = -ln tanh(x/2) = ln((e^x + 1)/(e^x - 1)) on a dense grid
    from 1e-30 to 88 (and 0, +inf) against float64 log1p(2 / expm1(x)): relative error at most
    8 float32 ulp (2^-23 relative each) where phi(x) >= 1e-30, phi(0) = +inf, phi(+inf) = 0;
    and phi(phi(x)) returns x to 1e-5 relative where phi is well conditioned (0.01 <= x <= 30)."""
    import torch
    xs = np.concatenate([np.logspace(-30, -1, 4000), np.linspace(0.1, 4.0, 20000), np.linspace(4.0, 88.0, 20000),
                         [0.5, 2.0, np.nextafter(np.float32(0.5), np.float32(0)), np.nextafter(np.float32(2.0), np.float32(0))]])
    x32 = xs.astype(np.float32)
    xt = torch.from_numpy(np.concatenate([x32, np.array([0.0, np.inf], np.float32)])).cuda()
    got = P.eval_phi(xt).cpu().numpy()
    assert np.isposinf(got[-2]) and got[-1] == 0.0
    got = got[:-2].astype(np.float64)
    x64 = x32.astype(np.float64)
    with np.errstate(over="ignore"):
        ref = np.log1p(2.0 / np.expm1(x64))
    ok = ref >= 1e-30
    rel = np.abs(got[ok] - ref[ok]) / ref[ok]
    ulp = 2.0 ** -23
    print(f"phi: max relative error {rel.max() / ulp:.2f} ulp over {ok.sum()} points", flush=True)
    assert rel.max() <= 8 * ulp
    inner = (x64 >= 0.01) & (x64 <= 30.0)
    back = P.eval_phi(torch.from_numpy(got[inner].astype(np.float32)).cuda()).cpu().numpy().astype(np.float64)
    assert (np.abs(back - x64[inner]) <= 1e-5 * x64[inner]).all()


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
