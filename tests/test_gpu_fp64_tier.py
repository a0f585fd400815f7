"""The GPU decoder (float32) against the float64 oracle at the benchmark point (GPU).

BB[[144,12,12]], p = 0.05, 1e5 shots, scaled min-sum (alpha = 0.625), 100 + 100
iterations, channel second-pass prior: the lane kernel the benchmark times.  The
float32 outputs are bit-identical to the float32 oracle (the tier-1 tests); this
file measures how far float32 BP+DC is from float64 BP+DC (Alg. 1 / Alg. 2,
Sec. III.A) and holds it to these bars:

* hard decisions agree on at least 99.99 % of all shots, and every disagreeing bit
  has |L64| < 1e-3;
* a shot is *unflagged* when every decision margin of its float64 decode (|q| at
  each sign test, |L| at each hard decision, the gap of each DC candidate to the
  tie threshold relative to max(1, |L_max|)) is at least 1e-5.  For a sign test
  the margin |x| >= 1e-5 is the same as |x| >= 1e-5 max(1, |x|), since the latter
  holds for every |x| > 1;
* min-sum's posteriors are piecewise linear in the priors with coefficients that
  can grow by (column degree - 1) alpha per iteration, so a shot that iterates
  long is ill-conditioned: its float64 posteriors themselves move when the priors
  move by one float32 ulp.  The *sensitivity* of a shot is the largest relative
  change, max over columns of |dL| / max(1, |L64|), of the float64 oracle's
  posteriors over three random sign patterns of a one-ulp (2^-24 relative) change
  of the prior LLRs, and infinite if its cut changes;
* on unflagged shots of sensitivity at most 2.5e-5 (well-conditioned, a quarter of
  the posterior bar): cut, flags, iteration counts and corrections equal the float64
  oracle's, and posteriors are within 1e-4 max(1, |L64|); at least 98 % of the shots
  are well-conditioned;
* on every unflagged shot: posterior error at most max(1e-4, 4 x sensitivity), so
  no deviation exceeds what one float32 rounding of the inputs already causes in
  float64;
* the logical error rates agree within 3 standard errors.
"""
import numpy as np
import pytest

import oracle
import synth

from gpu_helpers import gpu_decode, oracle_params

ULP32 = 2.0 ** -24


def _rel_post_err(a, b):
    """max over columns of |a - b| / max(1, |b|) per shot; +inf columns must match."""
    fin = np.isfinite(a) & np.isfinite(b)
    with np.errstate(invalid="ignore"):
        r = np.where(fin, np.abs(a - b) / np.maximum(1.0, np.abs(b)),
                     np.where(np.isinf(a) == np.isinf(b), 0.0, np.inf))
    return r.max(1)


def sensitivity(code, syndromes, op, ref64, reps=3, seed=5):
    """Per-shot relative change of the float64 oracle's posteriors under one-ulp prior changes."""
    lam = np.log((1.0 - code.priors) / code.priors)
    rng = np.random.default_rng(seed)
    sens = np.zeros(len(syndromes))
    for _ in range(reps):
        u = rng.choice([-1.0, 1.0], size=code.n)
        c = code.with_priors(1.0 / (1.0 + np.exp(lam * (1.0 + u * ULP32))))
        o = oracle.decode(c, syndromes, op, precision="f64")
        s = _rel_post_err(o["post"], ref64["post"])
        s[(o["cut"] != ref64["cut"]).any(1)] = np.inf
        sens = np.maximum(sens, s)
    return sens


def tier2_report(code, errors, out, ref64, sens):
    """Compare float32 outputs `out` with the float64 oracle's; returns counts and the
    masks the assertions use."""
    B = len(errors)
    dec_same = (out["ehat"] == ref64["ehat"]).all(1)
    dis_bits = out["ehat"] != ref64["ehat"]
    max_L_at_dis = np.abs(ref64["post"][dis_bits]).max() if dis_bits.any() else 0.0
    unflagged = ref64["margin"] >= 1e-5
    well = unflagged & (sens <= 2.5e-5)
    err = _rel_post_err(out["post"], ref64["post"])
    exact = ((out["ehat"] == ref64["ehat"]).all(1) & (out["cut"] == ref64["cut"]).all(1) &
             (out["flags"] == ref64["flags"]) & (out["iters"] == ref64["iters"]).all(1))

    def ler(o):
        return float((((o["flags"] & 1) == 0) | synth.residual_is_logical(errors ^ o["ehat"], code.O)).mean())

    return {
        "shots": B, "decisions_agree": float(dec_same.mean()), "max_abs_L64_at_disagreement": float(max_L_at_dis),
        "unflagged": int(unflagged.sum()), "well_conditioned": int(well.sum()),
        "well_not_exact": int((well & ~exact).sum()), "well_max_post_err": float(err[well].max()),
        "unflagged_over_bound": int((unflagged & (err > np.maximum(1e-4, 4 * sens))).sum()),
        "unflagged_post_err_over_1e-4": int((unflagged & (err > 1e-4)).sum()),
        "dc_shots_well_conditioned": int((well & ((ref64["flags"] & 2) != 0)).sum()),
        "ler32": ler(out), "ler64": ler(ref64),
    }


def check_tier2(rep, min_dc_shots=1000):
    assert rep["decisions_agree"] >= 0.9999, rep
    assert rep["max_abs_L64_at_disagreement"] < 1e-3, rep
    assert rep["well_conditioned"] >= 0.98 * rep["shots"], rep
    assert rep["well_not_exact"] == 0, rep
    assert rep["well_max_post_err"] <= 1e-4, rep
    assert rep["unflagged_over_bound"] == 0, rep
    assert rep["dc_shots_well_conditioned"] > min_dc_shots, rep
    se = np.sqrt(rep["ler64"] * (1 - rep["ler64"]) / rep["shots"])
    assert abs(rep["ler32"] - rep["ler64"]) <= 3 * se + 1.0 / rep["shots"], rep


@pytest.mark.gpu
def test_min_sum_bb144_float32_vs_float64_at_1e5_shots():
    import torch
    assert torch.cuda.is_available()
    import paper_2510_08695_amd as P
    code = synth.bb_code("bb144", p=0.05)
    B = 100_000
    sh = synth.make_shots(code, B, 2005)
    prm = P.Params(max_iter=(100, 100), alpha=0.625, second_pass_prior=P.PRIOR_CHANNEL, seed=1)
    plan = P.Plan([P.Code.from_problem(code)], prm, kernel=P.KERNEL_LANE)
    print("case bb144 p=0.05 B=1e5 lane vs float64 oracle", flush=True)
    g = gpu_decode(plan, code, sh.syndromes)
    op = oracle_params(prm, "channel")
    ref64 = oracle.decode(code, sh.syndromes, op, precision="f64")
    sens = sensitivity(code, sh.syndromes, op, ref64)
    rep = tier2_report(code, sh.errors, g, ref64, sens)
    print("float64 tier:", rep, flush=True)
    check_tier2(rep)


def test_float32_arithmetic_meets_the_float64_tier_on_the_cpu():
    """The same bars for the float32 oracle (whose outputs the GPU kernels reproduce bit for
    bit) on 2e4 shots: the float64 tier is a property of float32 BP+DC, not of a kernel."""
    code = synth.bb_code("bb144", p=0.05)
    sh = synth.make_shots(code, 20_000, 77)
    op = oracle.OracleParams(max_iter1=100, max_iter2=100, alpha=0.625, seed=1)
    o32 = oracle.decode(code, sh.syndromes, op, precision="f32")
    ref64 = oracle.decode(code, sh.syndromes, op, precision="f64")
    rep = tier2_report(code, sh.errors, o32, ref64, sensitivity(code, sh.syndromes, op, ref64))
    check_tier2(rep, min_dc_shots=200)
