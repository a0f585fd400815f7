"""Pins of the CPU oracle against facts fixed outside it (CPU only).

Each test compares the oracle with something it does not compute itself:
brute-force enumeration, the exact max-marginals / marginals that BP reaches
on trees, published generator outputs, closed forms of special cases, and
the invariants the paper states for degeneracy cutting (Sec. III.A).
"""
import itertools
import os

import numpy as np
import pytest

import oracle
import synth
from synth import Csr

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _read_golden(name):
    rows = []
    for line in open(os.path.join(GOLDEN, name)):
        line = line.strip()
        if line and not line.startswith("#"):
            rows.append(line.split())
    return rows


# --------------------------------------------------------------------------------------
# tie-break generator


def test_splitmix64_published_outputs():
    for state, out in _read_golden("splitmix64.txt"):
        assert oracle.splitmix64(int(state)) == int(out)


# --------------------------------------------------------------------------------------
# tree-shaped Tanner graphs: BP is exact there


def random_tree(rng, n_var, max_check_deg=4):
    """Random bipartite tree on n_var variables; every check has degree >= 2."""
    # grow: start with one variable, repeatedly attach a new check to an existing
    # variable and give it 1..max_check_deg-1 fresh variables
    adj = []  # list of checks, each a list of variables
    nv = 1
    while nv < n_var:
        anchor = int(rng.integers(nv))
        k = int(min(rng.integers(1, max_check_deg), n_var - nv))
        adj.append([anchor] + list(range(nv, nv + k)))
        nv += k
    H = np.zeros((len(adj), n_var), dtype=np.uint8)
    for c, vs in enumerate(adj):
        H[c, vs] = 1
    return H


def brute_force_tables(H, s, lam):
    """All e with H e = s, their cost sum(lam * e) and weight exp(-cost)."""
    m, n = H.shape
    E = np.array(list(itertools.product([0, 1], repeat=n)), dtype=np.uint8)
    ok = ((E.astype(np.int64) @ H.T.astype(np.int64)) % 2 == s[None, :]).all(axis=1)
    E = E[ok]
    cost = E.astype(np.float64) @ lam
    return E, cost


@pytest.mark.parametrize("seed", range(6))
def test_min_sum_on_tree_gives_exact_max_marginals(seed):
    rng = np.random.default_rng(100 + seed)
    Hd = random_tree(rng, int(rng.integers(6, 13)))
    H = Csr.from_dense(Hd)
    lam = rng.normal(1.5, 1.5, size=H.cols)
    s = rng.integers(0, 2, size=H.rows).astype(np.uint8)
    E, cost = brute_force_tables(Hd, s, lam)
    _, L, _, _ = oracle.bp_once(H, s, lam, T=2 * H.cols, rule=oracle.MIN_SUM, alpha=1.0)
    for v in range(H.cols):
        mm = cost[E[:, v] == 1].min() - cost[E[:, v] == 0].min()
        assert abs(L[v] - mm) < 1e-9 * max(1.0, abs(mm)), (v, L[v], mm)


@pytest.mark.parametrize("seed", range(6))
def test_product_sum_on_tree_gives_exact_marginals(seed):
    rng = np.random.default_rng(200 + seed)
    Hd = random_tree(rng, int(rng.integers(6, 13)))
    H = Csr.from_dense(Hd)
    lam = rng.normal(1.0, 1.0, size=H.cols)
    s = rng.integers(0, 2, size=H.rows).astype(np.uint8)
    E, cost = brute_force_tables(Hd, s, lam)
    w = np.exp(-(cost - cost.min()))
    _, L, _, _ = oracle.bp_once(H, s, lam, T=2 * H.cols, rule=oracle.PRODUCT_SUM, alpha=1.0)
    for v in range(H.cols):
        exact = np.log(w[E[:, v] == 0].sum() / w[E[:, v] == 1].sum())
        assert abs(L[v] - exact) < 1e-9 * max(1.0, abs(exact)), (v, L[v], exact)


@pytest.mark.parametrize("alpha", [0.625, 0.8])
def test_scaled_min_sum_single_check_one_iteration(alpha):
    """A star (one check): after one iteration L_v = lam_v + alpha * (exact extrinsic term).

    The exact extrinsic max-marginal term comes from brute force with alpha = 1."""
    rng = np.random.default_rng(7)
    for d in range(2, 8):
        Hd = np.ones((1, d), dtype=np.uint8)
        H = Csr.from_dense(Hd)
        lam = rng.normal(1.0, 2.0, size=d)
        for s0 in (0, 1):
            s = np.array([s0], np.uint8)
            E, cost = brute_force_tables(Hd, s, lam)
            _, L, it, _ = oracle.bp_once(H, s, lam, T=1, rule=oracle.MIN_SUM, alpha=alpha)
            assert it == 1
            for v in range(d):
                mm = cost[E[:, v] == 1].min() - cost[E[:, v] == 0].min()
                assert abs(L[v] - (lam[v] + alpha * (mm - lam[v]))) < 1e-12


def test_zero_syndrome_converges_after_one_iteration():
    """s = 0 with positive priors: every message keeps its sign, e_hat = 0 after t = 1 and
    L_v = lam_v + sum over checks of alpha * (smallest other prior) (closed form)."""
    code = synth.bb_code("bb144", p=0.05)
    lam = np.log(0.95 / 0.05)
    _, L, it, conv = oracle.bp_once(code.H, np.zeros(code.m, np.uint8), np.full(code.n, lam),
                                    T=10, alpha=0.625, lsat=64.0, stop_on_converge=True)
    assert conv and it == 1
    np.testing.assert_allclose(L, lam * (1 + 3 * 0.625), rtol=1e-15)


# --------------------------------------------------------------------------------------
# codes (Table I, Sec. II.B, Sec. IV.C)


def test_bb_codes_match_table1():
    for name, n, k, l, m in _read_golden("paper_table1.txt"):
        c = synth.bb_code(name)
        assert c.n == int(n) and c.m == int(n) // 2
        assert c.O.shape[0] == int(k)
        assert set(c.H.row_weights()) == {6} and set(c.H.col_weights()) == {3}
        assert not ((c.H.to_dense().astype(int) @ c.D.to_dense().T.astype(int)) % 2).any()


def test_toric_and_hgp_parameters():
    t = synth.toric_code(6)
    assert (t.m, t.n, t.H.nnz, t.O.shape[0]) == (36, 72, 144, 2)
    assert set(t.H.row_weights()) == {4} and set(t.H.col_weights()) == {2}
    Hc = synth.random_regular_classical(16, 4001)
    assert set(np.diff(Hc.indptr)) == {4} and set(np.bincount(Hc.indices)) == {3}
    h = synth.hgp_code(Hc)
    assert h.n == 16 * 16 + 12 * 12 and h.m == 16 * 12
    assert set(h.H.row_weights()) == {7}
    assert not ((h.H.to_sparse() @ h.D.to_sparse().T).toarray() % 2).any()


@pytest.mark.parametrize("d", [3, 5, 7])
def test_rotated_surface_code_parameters(d):
    """[[d^2, 1, d]] (Sec. II.B): (d^2 - 1) / 2 checks of each type, weights 2 and 4,
    d - 1 weight-2 checks of each type, X and Z checks commute, k = 1."""
    c = synth.rotated_surface_code(d)
    assert (c.n, c.m, c.D.rows) == (d * d, (d * d - 1) // 2, (d * d - 1) // 2)
    for M in (c.H, c.D):
        w = np.asarray(M.row_weights())
        assert set(w) == {2, 4} and (w == 2).sum() == d - 1
    assert not ((c.H.to_dense().astype(int) @ c.D.to_dense().T.astype(int)) % 2).any()
    assert c.n - synth.f2_rank(c.H) - synth.f2_rank(c.D) == 1 and c.O.shape[0] == 1
    # the logical operator has weight >= d (a logical of weight < d would be an error
    # the code cannot detect): check all words of weight < 3 for d = 3 by brute force
    if d == 3:
        import itertools
        H = c.H.to_dense().astype(int)
        for wt in (1, 2):
            for sup in itertools.combinations(range(c.n), wt):
                e = np.zeros((1, c.n), np.uint8)
                e[0, list(sup)] = 1
                if not ((H @ e[0]) % 2).any():
                    assert not synth.residual_is_logical(e, c.O)[0]


@pytest.mark.parametrize("final", [True, False])
def test_phenomenological_dem_structure(final):
    base = synth.bb_code("bb72")
    T = 4
    d = synth.phenomenological_dem(base, T, 0.01, 0.01, final)
    n, mZ = base.n, base.m
    rounds = T + 1 if final else T
    assert d.H.rows == mZ * rounds
    assert d.n == T * (n + mZ) + (n if final else 0)
    assert max(d.H.row_weights()) <= 6 + 2                      # r + 2
    assert max(d.D.row_weights()) <= max(6, 3 + 2)              # max{r, c + 2}
    assert not ((d.D.to_sparse() @ d.H.to_sparse().T).toarray() % 2).any()
    assert not ((d.D.to_dense().astype(np.int64) @ d.O.T.astype(np.int64)) % 2).any()
    # the DCM has the paper's shape for the [[288,12,18]] code at T = 18
    if final:
        big = synth.phenomenological_dem(synth.bb_code("bb288"), 18, 0.003, 0.003, True)
        assert (big.H.rows, big.H.cols, big.D.rows) == (2736, 8064, 7920)
    else:
        big = synth.phenomenological_dem(synth.bb_code("bb288"), 18, 0.003, 0.003, False)
        assert (big.H.rows, big.H.cols) == (2592, 7776)


# --------------------------------------------------------------------------------------
# degeneracy cutting (Sec. III.A)


@pytest.fixture(scope="module")
def bb144_run():
    code = synth.bb_code("bb144", p=0.06)
    shots = synth.make_shots(code, 3000, 123)
    prm = oracle.OracleParams(max_iter1=40, max_iter2=40, seed=99)
    out = oracle.decode(code, shots.syndromes, prm, precision="f64", want_post1=True)
    return code, shots, prm, out


def test_converged_outputs_satisfy_syndrome(bb144_run):
    code, shots, prm, out = bb144_run
    conv = (out["flags"] & 1).astype(bool)
    synd = synth.syndromes_of(out["ehat"], code.H)
    assert (synd[conv] == shots.syndromes[conv]).all()
    assert not (synd[~conv] == shots.syndromes[~conv]).all(axis=1).any()


def test_dc_invariants(bb144_run):
    code, shots, prm, out = bb144_run
    dc = np.nonzero(out["flags"] & 2)[0]
    assert len(dc) > 20
    eps = prm.tie_eps
    for b in dc:
        cut = out["cut"][b].astype(bool)
        L1 = out["post1"][b]
        assert cut.sum() <= code.D.rows
        assert not out["ehat"][b][cut].any()            # padded with zeros
        assert np.isinf(out["post"][b][cut]).all()      # cut variables have p = 0
        for h in range(code.D.rows):
            supp = code.D.row(h)
            lmax = L1[supp].max()
            ties = supp[L1[supp] >= lmax - eps * max(1.0, abs(lmax))]
            # this row's nominee is a cut variable of its tie set
            assert cut[ties].any()
        # every cut variable was nominated by some row for which it was in the tie set
        for v in np.nonzero(cut)[0]:
            rows = [h for h in range(code.D.rows) if v in set(code.D.row(h))]
            assert any(L1[v] >= L1[code.D.row(h)].max() - eps * max(1.0, abs(L1[code.D.row(h)].max()))
                       for h in rows)


def test_dc_runs_only_after_failed_first_pass(bb144_run):
    code, shots, prm, out = bb144_run
    dc = (out["flags"] & 2).astype(bool)
    p1 = oracle.decode(code, shots.syndromes,
                       oracle.OracleParams(max_iter1=prm.max_iter1, skip_dc=True, seed=prm.seed))
    assert (dc == ~(p1["flags"] & 1).astype(bool)).all()
    assert (out["iters"][dc, 0] == prm.max_iter1).all()
    assert (out["iters"][~dc, 1] == 0).all()


@pytest.mark.parametrize("precision", ["f64", "f32"])
@pytest.mark.parametrize("codename", ["bb144", "toric6"])
def test_algorithm1_delete_columns_equals_algorithm2_zero_prior(precision, codename):
    code = synth.bb_code("bb144", p=0.07) if codename == "bb144" else synth.toric_code(6, p=0.08)
    shots = synth.make_shots(code, 800, 321)
    base = dict(max_iter1=30, max_iter2=30, seed=5, second_pass_prior=code.second_pass)
    a = oracle.decode(code, shots.syndromes, oracle.OracleParams(dc_form="zero_prior", **base),
                      precision=precision)
    b = oracle.decode(code, shots.syndromes, oracle.OracleParams(dc_form="delete_columns", **base),
                      precision=precision)
    assert ((a["flags"] & 2) != 0).sum() > 10
    for k in ("ehat", "flags", "iters", "cut"):
        np.testing.assert_array_equal(a[k], b[k])
    np.testing.assert_array_equal(a["post"], b["post"])


def test_dc_independent_of_row_order():
    code = synth.bb_code("bb144", p=0.07)
    shots = synth.make_shots(code, 600, 77)
    prm = oracle.OracleParams(max_iter1=30, max_iter2=30, tie_break="lowest")
    a = oracle.decode(code, shots.syndromes, prm)
    perm = np.random.default_rng(3).permutation(code.D.rows)
    Dd = code.D.to_dense()[perm]
    b = oracle.decode(code, shots.syndromes, prm, D=Csr.from_dense(Dd))
    np.testing.assert_array_equal(a["cut"], b["cut"])
    np.testing.assert_array_equal(a["ehat"], b["ehat"])


def test_tie_break_is_a_function_of_seed_shot_and_row():
    """Decoding a shot range at an offset reproduces the same shots decoded in one batch."""
    code = synth.bb_code("bb144", p=0.07)
    shots = synth.make_shots(code, 400, 78)
    prm = oracle.OracleParams(max_iter1=25, max_iter2=25, seed=11, tie_eps=0.5)
    full = oracle.decode(code, shots.syndromes, prm)
    part = oracle.decode(code, shots.syndromes[150:], prm, shot_offset=150)
    np.testing.assert_array_equal(full["cut"][150:], part["cut"])
    other = oracle.decode(code, shots.syndromes, oracle.OracleParams(max_iter1=25, max_iter2=25,
                                                                      seed=12, tie_eps=0.5))
    assert (other["cut"] != full["cut"]).any()


# --------------------------------------------------------------------------------------
# whole decoder against maximum likelihood on a tiny code


def test_exact_ler_of_bpdc_not_below_maximum_likelihood_toric3():
    code = synth.toric_code(3, p=0.05)
    n, p = code.n, 0.05
    E = np.array(list(itertools.product([0, 1], repeat=n)), dtype=np.uint8)
    w = E.sum(1)
    prob = (p ** w) * ((1 - p) ** (n - w))
    S = synth.syndromes_of(E, code.H)
    cls = (E.astype(np.int64) @ code.O.T.astype(np.int64)) % 2
    skey = S.astype(np.int64) @ (1 << np.arange(code.m))
    ckey = cls @ (1 << np.arange(code.O.shape[0]))
    # exact maximum-likelihood (coset) failure rate
    table = {}
    for sk, ck, pr in zip(skey, ckey, prob):
        table.setdefault(sk, {}).setdefault(ck, 0.0)
        table[sk][ck] += pr
    ler_ml = sum(sum(d.values()) - max(d.values()) for d in table.values())
    # exact BP+DC failure rate: decode every reachable syndrome once
    uniq, first = np.unique(skey, return_index=True)
    for sp in ("posterior", "channel"):
        prm = oracle.OracleParams(max_iter1=18, max_iter2=18, second_pass_prior=sp, seed=1)
        out = oracle.decode(code, S[first], prm)
        dec_cls = (out["ehat"].astype(np.int64) @ code.O.T.astype(np.int64)) % 2 @ (1 << np.arange(2))
        ler = 0.0
        for j, sk in enumerate(uniq):
            conv = out["flags"][j] & 1
            for ck, pr in table[sk].items():
                if not conv or ck != dec_cls[j]:
                    ler += pr
        assert ler >= ler_ml - 1e-15
        assert ler < 0.3
        print(sp, "exact LER", ler, "ML", ler_ml)
    assert 0.03 < ler_ml < 0.1


def test_saturation_level_is_ler_neutral():
    code = synth.bb_code("bb144", p=0.05)
    shots = synth.make_shots(code, 1500, 2005)
    fails = []
    for lsat in (64.0, 1e30):
        out = oracle.decode(code, shots.syndromes,
                            oracle.OracleParams(max_iter1=100, max_iter2=100, llr_sat=lsat))
        res = shots.errors ^ out["ehat"]
        fails.append(((out["flags"] & 1) == 0) | synth.residual_is_logical(res, code.O))
    a, b = fails[0].mean(), fails[1].mean()
    se = np.sqrt(max(a * (1 - a), 1e-4) / len(shots))
    assert abs(a - b) < 4 * se


# --------------------------------------------------------------------------------------
# statistics the paper prints (Appendix A Table III, Appendix B Table IV)


def test_bb144_first_pass_failure_and_flatness_match_tables_3_and_4():
    """[[144,12,12]], code capacity p = 0.01, min-sum with T = n = 144 (Fig. 2 caption),
    channel prior in the second pass (Sec. III.B).

    The paper does not state the min-sum scale; unscaled min-sum (alpha = 1) in double
    precision reproduces its printed counts, so this pin uses alpha = 1.  Loose bounds:
    1e6 shots give ~140 first-pass failures (Poisson sd ~12)."""
    g = _read_golden("paper_table3_4.txt")
    rate = float(g[0][1])
    flat = {float(a): float(b) for a, b in g[1:]}
    code = synth.bb_code("bb144", p=0.01)
    shots = synth.make_shots(code, 1_000_000, 31)
    out = oracle.decode(code, shots.syndromes,
                        oracle.OracleParams(max_iter1=144, max_iter2=144, alpha=1.0, seed=1),
                        want_post=False, want_post1=True)
    dc = (out["flags"] & 2) != 0
    conv = (out["flags"] & 1) != 0
    fail = ~conv | synth.residual_is_logical(shots.errors ^ out["ehat"], code.O)
    n_dc = dc.sum()
    assert 0.7 * rate * len(shots) < n_dc < 1.4 * rate * len(shots)
    # Table III: DC rescued (9073 + 1740) of 13769 first-pass failures (78.5 %)
    rescued = (dc & ~fail).sum() / n_dc
    assert abs(rescued - (9073 + 1740) / 13769) < 0.12
    # Table IV: spread of the posterior error probabilities over each H_X row
    ph = 1.0 / (1.0 + np.exp(out["post1"][dc]))
    rows = [code.D.row(h) for h in range(code.D.rows)]
    spread = np.stack([ph[:, r].max(1) - ph[:, r].min(1) for r in rows], axis=1)
    for eps_gap, frac in flat.items():
        assert abs((spread <= eps_gap).mean() - frac) < 0.08, eps_gap


def test_surface49_first_pass_failure_matches_table_3():
    """[[49,1,7]] rotated surface code, code capacity p = 0.01 (bit flips), product-sum BP
    with T = n = 49 (Fig. 2 caption), posterior prior in the second pass (Sec. III.B).

    Table III counts 11,995,211 first-pass failures in 1e8 shots (0.11995).  2e5 shots
    give a binomial sd of 7.3e-4: the bound is 4 sd.  BP+DC then fails on 4.09e-4 of the
    first-pass failures (3,098 + 1,810 of 11,995,211); on ~24,000 of them that is ~10
    (Poisson), bounded loosely."""
    g = {k: float(v) for k, v in _read_golden("paper_table3_surface49.txt")}
    code = synth.rotated_surface_code(7, p=0.01)
    B = 200_000
    shots = synth.make_shots(code, B, 41)
    out = oracle.decode(code, shots.syndromes,
                        oracle.OracleParams(rule=oracle.PRODUCT_SUM, max_iter1=49, max_iter2=49, alpha=1.0,
                                            second_pass_prior="posterior", seed=1),
                        want_post=False)
    dc = (out["flags"] & 2) != 0
    rate = dc.mean()
    sd = np.sqrt(g["bp_fail_per_shot"] * (1 - g["bp_fail_per_shot"]) / B)
    assert abs(rate - g["bp_fail_per_shot"]) < 4 * sd, rate
    fail = ((out["flags"] & 1) == 0) | synth.residual_is_logical(shots.errors ^ out["ehat"], code.O)
    expect = g["bpdc_fail_given_bp_fail"] * dc.sum()
    assert (fail & dc).sum() <= 3 * expect + 10


def test_surface49_flatness_matches_table_4():
    """Table IV's surface-code row: the fraction of H_X rows with first-pass posterior
    spread <= eps_gap on shots whose first BP step failed ([[49,1,7]], p = 0.01,
    product-sum, T = n).  2e5 shots give ~24,000 failed shots and ~576,000 rows."""
    flat = {float(a): float(b) for a, b in _read_golden("paper_table4_surface49.txt")}
    code = synth.rotated_surface_code(7, p=0.01)
    shots = synth.make_shots(code, 200_000, 43)
    out = oracle.decode(code, shots.syndromes,
                        oracle.OracleParams(rule=oracle.PRODUCT_SUM, max_iter1=49, max_iter2=49, alpha=1.0,
                                            second_pass_prior="posterior", seed=1),
                        want_post=False, want_post1=True)
    dc = (out["flags"] & 2) != 0
    ph = 1.0 / (1.0 + np.exp(out["post1"][dc].astype(np.float64)))
    rows = [code.D.row(h) for h in range(code.D.rows)]
    spread = np.stack([ph[:, r].max(1) - ph[:, r].min(1) for r in rows], axis=1)
    for eps_gap, frac in flat.items():
        assert abs((spread <= eps_gap).mean() - frac) < 0.01, eps_gap


# --------------------------------------------------------------------------------------
# intermittent soft DC (the extension proposed in Sec. V; reading: every K pass-1
# iterations while H e != s, the nominees' prior LLRs rise by beta)


@pytest.mark.parametrize("K,beta", [(3, 2.0), (4, 0.5), (3, 0.3), (5, 0.75)])
@pytest.mark.parametrize("seed", [1, 2, 3, 5, 8])
def test_soft_dc_two_bit_closed_form(K, beta, seed):
    """H = D = (1 1), s = 1, equal priors: scaled min-sum sits at the symmetric fixed
    point L_0 = L_1 = (1 - alpha) lam and never converges.  The first soft application
    (t = K) meets a tie and nominates the column v* drawn by the hash of row
    rows(D) * 1 + 0; afterwards v* holds the larger posterior and is nominated again
    at t = 2K, 3K, ....  After j applications the other column's posterior at iteration
    jK + 2 is lam - alpha (lam + j beta), so BP converges at t = j* K + 2 with
    j* = ceil(lam (1 - alpha) / (alpha beta)), flipping the column that was not nominated."""
    p, alpha = 0.1, 0.625
    lam = np.log((1 - p) / p)
    code = synth.Code("two", Csr.from_dense([[1, 1]]), Csr.from_dense([[1, 1]]), np.full(2, p))
    jstar = int(np.ceil(lam * (1 - alpha) / (alpha * beta)))
    T1 = jstar * K + 10
    prm = oracle.OracleParams(max_iter1=T1, max_iter2=5, alpha=alpha, seed=seed, soft_period=K,
                              soft_shift=beta)
    shots = np.ones((4, 1), np.uint8)
    out = oracle.decode(code, shots, prm, precision="f64", shot_offset=17)
    for b in range(4):
        vstar = oracle.tie_hash(seed, 17 + b, 1) >> 63   # floor(h * 2 / 2^64)
        assert out["flags"][b] == 1
        assert out["iters"][b, 0] == jstar * K + 2
        np.testing.assert_array_equal(out["ehat"][b], [1 - vstar == 0, 1 - vstar == 1])
    # without soft DC the pass never converges and DC runs
    base = oracle.decode(code, shots, oracle.OracleParams(max_iter1=T1, max_iter2=5, alpha=alpha, seed=seed),
                         precision="f64")
    assert (base["flags"] & 2).all() and (base["iters"][:, 0] == T1).all()


@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_soft_dc_reduces_to_bpdc(precision):
    """beta = 0, or a period beyond the first pass, leaves BP+DC unchanged."""
    code = synth.bb_code("bb72", p=0.06)
    shots = synth.make_shots(code, 400, 77)
    base = oracle.OracleParams(max_iter1=40, max_iter2=40, seed=3)
    ref = oracle.decode(code, shots.syndromes, base, precision=precision, want_post1=True)
    for soft in (dict(soft_period=4, soft_shift=0.0), dict(soft_period=40, soft_shift=3.0)):
        o = oracle.decode(code, shots.syndromes, oracle.OracleParams(max_iter1=40, max_iter2=40, seed=3, **soft),
                          precision=precision, want_post1=True)
        for k in ("ehat", "flags", "iters", "cut", "post", "post1"):
            np.testing.assert_array_equal(o[k], ref[k], err_msg=f"{soft} {k}")
    # and a real shift changes the decoding of some shot
    o = oracle.decode(code, shots.syndromes, oracle.OracleParams(max_iter1=40, max_iter2=40, seed=3,
                                                                 soft_period=4, soft_shift=1.0),
                      precision=precision)
    assert (o["iters"] != ref["iters"]).any()
