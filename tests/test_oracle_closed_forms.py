"""Closed-form pins of the oracle's weighted rule, second-pass prior, product-sum
saturation and tie draw (CPU only).

Each expected value here is worked out by hand (or by brute force over a single
check's local configurations) from the paper's definitions and the readings the
oracle documents, never by calling the oracle's own arithmetic:

* per-edge scales (trainable min-sum): the check-to-variable message on edge
  (c, v) is w_cv times the smallest |q| over the check's *other* edges, signed
  by the syndrome bit and the other signs (Sec. II.C's min-sum with one scale
  per edge instead of one per decoder);
* Algorithm 1's second BP run takes the first run's posteriors as its prior
  (Sec. III.A, Sec. III.B for surface-type codes), or the channel prior (BB-type
  codes); the posteriors it takes are the saturated ones DC reads;
* product-sum (Sec. II.C): r = 2 atanh(prod tanh(|q|/2)), in closed form on
  checks of two and three edges, and held at the saturation level when every
  other column is frozen (an empty product);
* DC's random choice among k tied columns is entry floor(h k / 2^64) of the tie
  set in ascending column order, h the 64-bit draw of (seed, shot, row).
"""
import itertools

import numpy as np
import pytest

import oracle
import synth
from synth import Csr


def _p_of_llr(lam):
    """Prior probability whose LLR log((1 - p) / p) is lam."""
    return 1.0 / (1.0 + np.exp(np.asarray(lam, dtype=np.float64)))


def _single_check_extrinsic(lam_others, s_c):
    """Extrinsic max-marginal term of one parity check for one of its columns, by brute force.

    For the check alone, with the other columns' prior LLRs `lam_others`, this is
    min_{x : parity = s_c xor 1} sum lam x  -  min_{x : parity = s_c} sum lam x over
    the configurations x of the other columns: the change in the best cost when the
    column itself flips (its own prior excluded)."""
    best = {0: np.inf, 1: np.inf}
    for x in itertools.product([0, 1], repeat=len(lam_others)):
        par = sum(x) & 1
        best[par] = min(best[par], float(np.dot(lam_others, x)))
    # column = 1 needs the others to carry parity s_c ^ 1; column = 0 needs parity s_c
    return best[s_c ^ 1] - best[s_c]


# --------------------------------------------------------------------------------------
# per-edge scales


@pytest.mark.parametrize("seed", range(4))
def test_weighted_min_sum_one_iteration_distinct_edge_scales(seed):
    """After the first iteration (q = prior on every edge) the posterior is
    L_v = lam_v + sum_{c in N(v)} w_cv * extrinsic_c(v), with extrinsic_c(v) the single-check
    brute-force term above (magnitude: the smallest other |lam|).  Every edge has its own
    scale, and the graph has several checks so that CSR and CSC edge orders differ: a
    scale taken from another edge, or applied inside the minimum, fails."""
    rng = np.random.default_rng(40 + seed)
    m, n = 5, 11
    while True:
        Hd = (rng.random((m, n)) < 0.35).astype(np.uint8)
        if Hd.sum(1).min() >= 2 and Hd.sum(0).min() >= 1:
            break
    H = Csr.from_dense(Hd)
    lam = rng.normal(0.8, 2.0, size=n)
    s = rng.integers(0, 2, size=m).astype(np.uint8)
    w = rng.uniform(0.2, 1.6, size=H.nnz)          # CSR order, all distinct
    assert len(np.unique(w)) == H.nnz
    _, L, it, _ = oracle.bp_once(H, s, lam, T=1, rule=oracle.MIN_SUM, weights=w, lsat=np.inf)
    assert it == 1
    expect = lam.copy()
    for c in range(m):
        cols = H.row(c)
        for k, v in enumerate(cols):
            e = H.row_ptr[c] + k
            others = [lam[u] for u in cols if u != v]
            expect[v] += w[e] * _single_check_extrinsic(others, int(s[c]))
    np.testing.assert_allclose(L, expect, rtol=1e-12, atol=1e-12)


def _two_bit_code(lam):
    """H = D = (1 1): one check on two columns; DC's single row spans both."""
    row = Csr.from_dense([[1, 1]])
    return synth.Code("two-bit", row, row, _p_of_llr(lam))


@pytest.mark.parametrize("second_pass", ["channel", "posterior"])
@pytest.mark.parametrize("case", range(4))
def test_two_bit_code_pass_two_closed_form(second_pass, case):
    """H = D = (1 1), s = 1, priors lam_0, lam_1 > 0, scales w1 = (a0, a1) for the first
    pass and w2 = (b0, b1) for the second, saturation S = 64.

    Pass 1: q_v = lam_v on every iteration (one check: q = L - r = lam), so
    L1_v = lam_v - a_v lam_{1-v} > 0 for both columns: e = 0 never meets s = 1.  DC
    cuts the column of larger L1 (Alg. 1: lowest posterior error probability).  Pass 2
    on the other column u: q_u = prior2_u, the frozen column sends +S, so
    L_u = prior2_u - b_u S < 0 and BP converges at its first iteration with e_u = 1.
    prior2_u is lam_u (channel) or L1_u (posterior), which are different numbers here."""
    S = 64.0
    lam, a, b = {
        0: ((2.9, 2.2), (0.55, 0.4), (0.3, 0.45)),
        1: ((2.2, 2.9), (0.4, 0.55), (0.45, 0.3)),
        2: ((3.5, 3.3), (0.21, 0.93), (0.71, 0.19)),
        3: ((1.7, 4.1), (0.17, 0.35), (0.23, 0.61)),
    }[case]
    lam, a, b = map(np.array, (lam, a, b))
    L1 = np.array([lam[0] - a[0] * lam[1], lam[1] - a[1] * lam[0]])
    assert (L1 > 0).all() and abs(L1[0] - L1[1]) > 0.01
    vstar = int(np.argmax(L1))
    u = 1 - vstar
    prior2 = lam[u] if second_pass == "channel" else L1[u]
    Lu = prior2 - b[u] * S
    assert -S < Lu < 0

    code = _two_bit_code(lam)
    T1, T2 = 7, 5
    prm = oracle.OracleParams(max_iter1=T1, max_iter2=T2, second_pass_prior=second_pass, seed=3)
    w = np.concatenate([a, b])                       # [pass][edge], edges in CSR order
    out = oracle.decode(code, np.ones((3, 1), np.uint8), prm, weights=w, want_post1=True)
    for k in range(3):
        np.testing.assert_allclose(out["post1"][k], L1, rtol=1e-13)
        assert out["cut"][k].tolist() == [int(vstar == 0), int(vstar == 1)]
        assert out["flags"][k] == 3 and out["iters"][k].tolist() == [T1, 1]
        assert out["ehat"][k].tolist() == [int(u == 0), int(u == 1)]
        assert np.isinf(out["post"][k, vstar]) and out["post"][k, vstar] > 0
        np.testing.assert_allclose(out["post"][k, u], Lu, rtol=1e-13)


@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_posterior_second_pass_starts_from_saturated_first_pass(precision):
    """Saturation S = 2.5, lam = (4.0, 3.5), first-pass scales (0.3, 0.2).

    Pass 1: every q is sat(lam) = S, so L1 = (4.0 - 0.3 S, 3.5 - 0.2 S) = (3.25, 3.0),
    both above S: the saturated posteriors DC reads are (S, S), a tie, and the hash
    h = tie_hash(seed, shot, 0) picks column floor(2 h / 2^64) = h >> 63.  Pass 2 on the
    other column u starts from its saturated first-pass posterior S: q_u = S, the frozen
    column sends +S, so L_u = S - b_u S > 0, the pass never converges and the reported
    posterior is S (1 - b_u).  An unsaturated reading would cut column 0 on every shot
    and report 3.0 - 2.5 b_1; the channel prior would report lam_u - 2.5 b_u."""
    S = 2.5
    lam = np.array([4.0, 3.5])
    a = np.array([0.3, 0.2])
    b = np.array([0.6, 0.7])
    code = _two_bit_code(lam)
    T1, T2 = 6, 4
    seed = 21
    prm = oracle.OracleParams(max_iter1=T1, max_iter2=T2, second_pass_prior="posterior", seed=seed,
                              llr_sat=S)
    B = 64
    out = oracle.decode(code, np.ones((B, 1), np.uint8), prm, weights=np.concatenate([a, b]),
                        want_post1=True, precision=precision)
    picks = []
    tol = 1e-6 if precision == "f32" else 1e-13
    for k in range(B):
        vstar = oracle.tie_hash(seed, k, 0) >> 63
        u = 1 - vstar
        picks.append(vstar)
        assert out["post1"][k].tolist() == [S, S]
        assert out["cut"][k].tolist() == [int(vstar == 0), int(vstar == 1)]
        assert out["flags"][k] == 2 and out["iters"][k].tolist() == [T1, T2]
        assert out["ehat"][k].tolist() == [0, 0]
        np.testing.assert_allclose(out["post"][k, u], S * (1 - b[u]), rtol=tol)
    assert 0 < sum(picks) < B            # both columns get cut on some shot


# --------------------------------------------------------------------------------------
# product-sum saturation


@pytest.mark.parametrize("precision", ["f64", "f32"])
@pytest.mark.parametrize("s0", [0, 1])
def test_product_sum_three_edge_check_closed_form(precision, s0):
    """One check on three columns, product-sum, one iteration from prior LLRs (a, b, c), all
    below the saturation level.  The message to the third column is
    2 atanh(tanh(a/2) tanh(b/2)) = ln(cosh((a+b)/2) / cosh((a-b)/2)) (from
    tanh x tanh y = (cosh(x+y) - cosh(x-y)) / (cosh(x+y) + cosh(x-y))), signed by the syndrome
    bit: the posterior is c +- that (saturation far above: nothing is clamped).  Messages up to 60
    are included, where tanh(|q|/2) rounds to 1 in float64 and a product of tanh values would
    saturate."""
    rng = np.random.default_rng(11 + s0)
    H = Csr.from_dense([[1, 1, 1]])
    sign = -1.0 if s0 else 1.0
    tol = 2e-6 if precision == "f32" else 1e-12
    lams = [rng.uniform(0.05, 60.0, size=3) for _ in range(40)] + [np.array([50.0, 50.0, 1.0]),
                                                                   np.array([60.0, 45.0, 2.0])]
    for lam in lams:
        if precision == "f32":
            lam = lam.astype(np.float32).astype(np.float64)
        _, L, it, _ = oracle.bp_once(H, np.array([s0], np.uint8), lam, T=1, rule=oracle.PRODUCT_SUM, alpha=1.0,
                                     lsat=1e6, precision=precision)
        assert it == 1
        for v in range(3):
            a, b = (lam[u] for u in range(3) if u != v)
            r = np.log(np.cosh((a + b) / 2) / np.cosh((a - b) / 2))
            assert abs(L[v] - (lam[v] + sign * r)) <= tol * max(1.0, abs(lam[v] + sign * r)), (lam, v, L[v])


@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_product_sum_two_edge_check_passes_the_message_through(precision):
    """A check of degree 2: 2 atanh(tanh(|q|/2)) = |q|, so each column receives the other's
    prior LLR exactly (for every magnitude up to the saturation level), signed by the syndrome."""
    H = Csr.from_dense([[1, 1]])
    tol = 1e-6 if precision == "f32" else 1e-13
    for a in (1e-3, 0.1, 1.0, 5.0, 20.0, 40.0, 63.0):
        for s0 in (0, 1):
            lam = np.array([a, 2.5])
            _, L, _, _ = oracle.bp_once(H, np.array([s0], np.uint8), lam, T=1, rule=oracle.PRODUCT_SUM, alpha=1.0,
                                        lsat=1e6, precision=precision)
            sign = -1.0 if s0 else 1.0
            assert abs(L[1] - (2.5 + sign * a)) <= tol * max(1.0, a), (a, s0, L)
            assert abs(L[0] - (a + sign * 2.5)) <= tol * max(1.0, a), (a, s0, L)


def test_product_sum_frozen_columns_send_the_saturation_level():
    """Algorithm 2 on product-sum: a frozen column (prior probability 0, LLR +inf) sends
    tanh(+inf) = 1, so two frozen columns leave the third column the message of an empty
    product, 2 atanh(1) = +inf, held at the saturation level S, exactly as the literal deletion
    of both columns (Algorithm 1) does; the third column's posterior is lam_2 -+ S."""
    S = 64.0
    H = Csr.from_dense([[1, 1, 1]])
    lam = np.array([2.0, 3.0, 1.5])
    for s0 in (0, 1):
        _, L, _, _ = oracle.bp_once(H, np.array([s0], np.uint8), lam, T=1, rule=oracle.PRODUCT_SUM,
                                    alpha=1.0, lsat=S, frozen=np.array([1, 1, 0], np.uint8))
        assert L[2] == min(S, 1.5 + (-S if s0 else S))
        assert np.isinf(L[:2]).all()


# --------------------------------------------------------------------------------------
# DC's draw among tied columns


@pytest.mark.parametrize("k_ties", [3, 4])
def test_dc_tie_draw_among_three_and_four_columns(k_ties):
    """H = D = (1 1 1 1), s = 1, scaled min-sum (0.625).  Priors lam_a on the tied columns
    and lam_b < lam_a on column 1 when k = 3: at every iteration q = lam, so
    L1 = lam_v - 0.625 min_{u != v} lam_u, all > 0 (e = 0, s = 1: no convergence).  The
    columns of lam_a share the largest L1 exactly; with k = 3 the tie set is {0, 2, 3}.
    The nominee is entry floor(h k / 2^64) of the tie set, h = tie_hash(seed, shot, 0)."""
    la, lb = np.log(0.95 / 0.05), np.log(0.9 / 0.1)
    lam = np.array([la, lb if k_ties == 3 else la, la, la])
    row = Csr.from_dense([[1, 1, 1, 1]])
    code = synth.Code("four", row, row, _p_of_llr(lam))
    ties = [0, 2, 3] if k_ties == 3 else [0, 1, 2, 3]
    B = 300
    seen = set()
    for seed in (0, 7, 12345):
        prm = oracle.OracleParams(max_iter1=5, max_iter2=5, seed=seed, tie_eps=1e-3)
        out = oracle.decode(code, np.ones((B, 1), np.uint8), prm, shot_offset=1000, want_post1=True)
        for j in range(B):
            h = oracle.tie_hash(seed, 1000 + j, 0)
            pick = ties[(h * k_ties) >> 64]
            seen.add(pick)
            assert out["cut"][j].tolist() == [int(c == pick) for c in range(4)], (seed, j)
            assert len(set(out["post1"][j][ties])) == 1
    assert seen == set(ties)
