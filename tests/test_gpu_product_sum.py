"""Product-sum BP+DC on the GPU against the float64 oracle (needs an MI355X).

The product-sum check rule (Sec. II.C; used by the paper for surface codes)
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


@pytest.mark.parametrize("name,p,shots,T", CASES)
def test_product_sum_vs_float64_oracle(P, name, p, shots, T):
    code = _code(name, p)
    sh = synth.make_shots(code, shots, 5000 + shots)
    prm = P.Params(max_iter=(T, T), alpha=1.0, second_pass_prior=P.PRIOR_POSTERIOR, seed=23,
                   rule=P.RULE_PRODUCT_SUM)
    plan = P.Plan([P.Code.from_problem(code)], prm, kernel=P.KERNEL_PLAIN)
    g = gpu_decode(plan, code, sh.syndromes)
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


def test_product_sum_plans(P):
    code = synth.rotated_surface_code(5, p=0.03)
    prm = P.Params(max_iter=(25, 25), alpha=1.0, second_pass_prior=P.PRIOR_POSTERIOR, rule=P.RULE_PRODUCT_SUM)
    c = P.Code.from_problem(code)
    assert P.Plan([c], prm, kernel=P.KERNEL_AUTO).info(0)["kernel"] == P.KERNEL_PLAIN
    for k in (P.KERNEL_LANE, P.KERNEL_GROUP):
        with pytest.raises(P.BpdcError):
            P.Plan([c], prm, kernel=k)
