"""Decoding at the size limits `bpdc_code_create` and `bpdc_plan_create` state
(needs an MI355X): H rows of 64 edges, H columns of 16, D rows of 32, the group
family's rows of 58 (64-bit check records) and 32 (the widest 32-bit records),
product-sum rows of 8 on the group family; one past each limit is refused with
BpdcError; and at the other end codes with checks and columns that have no
edges, or no edge at all.  Min-sum outputs bit-exact with the float32 oracle;
product-sum on the group family bit-identical with the plain family.

The codes are synthetic: every column meets `dv` distinct checks, chosen among
the checks of lowest current degree (random order among equals), so with
n dv = m R every row has exactly R edges; D's rows are random column subsets
of the given weights."""
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


def _balanced(m, n, dv, seed):
    rng = np.random.default_rng(seed)
    deg = np.zeros(m, dtype=np.int64)
    rows, cols = [], []
    for v in rng.permutation(n):
        key = deg * m + rng.permutation(m)  # lowest degree first, random among equals
        for c in np.argsort(key)[:dv]:
            rows.append(c)
            cols.append(v)
            deg[c] += 1
    A = np.zeros((m, n), dtype=np.uint8)
    A[rows, cols] = 1
    return A


def _code(m, R, dv, d_weights, p, seed, second_pass="channel"):
    n = m * R // dv
    assert n * dv == m * R
    H = _balanced(m, n, dv, seed)
    rng = np.random.default_rng(seed + 1)
    D = np.zeros((len(d_weights), n), dtype=np.uint8)
    for i, w in enumerate(d_weights):
        D[i, rng.choice(n, size=w, replace=False)] = 1
    code = synth.Code(f"limit_m{m}_r{R}_dv{dv}", synth.Csr.from_dense(H), synth.Csr.from_dense(D),
                      np.full(n, p), None, second_pass)
    assert code.H.row_weights().max() == R and code.H.col_weights().max() == dv
    return code


def _min_sum(P, T=(40, 40), seed=13):
    return P.Params(max_iter=T, alpha=0.625, second_pass_prior=P.PRIOR_CHANNEL, seed=seed)


def _parity(P, code, kid, shots, seed):
    sh = synth.make_shots(code, shots, seed)
    prm = _min_sum(P)
    plan = P.Plan([P.Code.from_problem(code)], prm, kernel=kid)
    g = gpu_decode(plan, code, sh.syndromes, shot_offset=3)
    ref = oracle.decode(code, sh.syndromes, oracle_params(prm, "channel"), precision="f32", shot_offset=3)
    assert ((ref["flags"] & 2) != 0).sum() > 0, "case must exercise DC"
    assert_bit_exact(g, ref, code.n)


@pytest.mark.parametrize("kernel", ["group", "plain"])
def test_group_row_limit_58(P, kernel):
    """Rows of 58 edges (the group family's limit, 64-bit records) and D rows of 32."""
    code = _code(12, 58, 3, [32, 32, 5, 3, 17, 32], 0.01, 101)
    kid = P.KERNEL_GROUP if kernel == "group" else P.KERNEL_PLAIN
    print(f"case rows 58 kernel={kernel}", flush=True)
    _parity(P, code, kid, 600, 201)
    if kernel == "group":
        assert P.Plan([P.Code.from_problem(code)], _min_sum(P), kernel=P.KERNEL_AUTO).info(0)["kernel"] == \
            P.KERNEL_GROUP


def test_group_row_59_refused_plain_runs(P):
    code = _code(12, 59, 3, [6, 6, 6], 0.01, 102)
    c = P.Code.from_problem(code)
    with pytest.raises(P.BpdcError):
        P.Plan([c], _min_sum(P), kernel=P.KERNEL_GROUP)
    print("case rows 59 plain", flush=True)
    _parity(P, code, P.KERNEL_PLAIN, 600, 202)


def test_h_row_limit_64_plain(P):
    """Rows of 64 edges (bpdc_code_create's limit) on the plain family; 65 refused."""
    code = _code(12, 64, 3, [32, 9, 4], 0.01, 103)
    print("case rows 64 plain", flush=True)
    _parity(P, code, P.KERNEL_PLAIN, 600, 203)
    over = _code(12, 65, 3, [6], 0.01, 104)
    with pytest.raises(P.BpdcError):
        P.Code.from_problem(over)


@pytest.mark.parametrize("kernel", ["group", "plain"])
def test_column_limit_16_rows_32(P, kernel):
    """Columns of 16 edges (bpdc_code_create's limit) with rows of 32 (the group
    family's widest 32-bit check records)."""
    code = _code(32, 32, 16, [32, 32, 8, 2], 0.02, 105)
    kid = P.KERNEL_GROUP if kernel == "group" else P.KERNEL_PLAIN
    print(f"case columns 16 rows 32 kernel={kernel}", flush=True)
    _parity(P, code, kid, 600, 205)


def test_column_17_and_d_row_33_refused(P):
    with pytest.raises(P.BpdcError):
        P.Code.from_problem(_code(34, 32, 17, [4], 0.02, 106))
    with pytest.raises(P.BpdcError):
        P.Code.from_problem(_code(12, 20, 3, [33], 0.02, 107))


def test_product_sum_row_limits(P):
    """Product-sum: rows of 8 on the group family, bit-identical with the plain
    family; rows of 9 refused there and taken by plain under AUTO; plain takes
    rows of 32 and refuses 33."""
    code = _code(24, 8, 2, [4, 4, 3, 8], 0.02, 108, second_pass="posterior")
    sh = synth.make_shots(code, 2000, 208)
    prm = P.Params(max_iter=(30, 30), alpha=1.0, second_pass_prior=P.PRIOR_POSTERIOR, seed=7,
                   rule=P.RULE_PRODUCT_SUM)
    c = P.Code.from_problem(code)
    print("case product-sum rows 8 group vs plain", flush=True)
    a = gpu_decode(P.Plan([c], prm, kernel=P.KERNEL_PLAIN), code, sh.syndromes)
    b = gpu_decode(P.Plan([c], prm, kernel=P.KERNEL_GROUP), code, sh.syndromes)
    assert ((a["flags"] & 2) != 0).sum() > 0
    for k in ("flags", "iters", "ehat", "cut"):
        np.testing.assert_array_equal(a[k], b[k], err_msg=k)
    np.testing.assert_array_equal(a["post"].view(np.uint32), b["post"].view(np.uint32))
    nine = P.Code.from_problem(_code(24, 9, 3, [4], 0.02, 109))
    with pytest.raises(P.BpdcError):
        P.Plan([nine], prm, kernel=P.KERNEL_GROUP)
    assert P.Plan([nine], prm, kernel=P.KERNEL_AUTO).info(0)["kernel"] == P.KERNEL_PLAIN
    wide = P.Code.from_problem(_code(32, 32, 16, [4], 0.02, 110))
    P.Plan([wide], prm, kernel=P.KERNEL_PLAIN)
    over = P.Code.from_problem(_code(12, 33, 3, [4], 0.02, 111))
    with pytest.raises(P.BpdcError):
        P.Plan([over], prm, kernel=P.KERNEL_PLAIN)


def _degenerate(case, seed=5):
    rng = np.random.default_rng(seed)
    if case == "no_edges":
        m, n = 8, 16
        H = np.zeros((m, n), np.uint8)
    else:
        m, n = 24, 40
        H = (rng.random((m, n)) < 0.15).astype(np.uint8)
        H[[0, 5], :] = 0
        H[:, [3, 17, 39]] = 0
    D = np.zeros((10, n), np.uint8)
    for i in range(10):
        D[i, rng.choice(n, size=int(rng.integers(3, 7)), replace=False)] = 1
    return synth.Code(f"degenerate_{case}", synth.Csr.from_dense(H), synth.Csr.from_dense(D), np.full(n, 0.05), None,
                      "channel")


# degenerate codes: checks without edges (unsatisfiable when their syndrome bit is 1, so such shots
# run both passes and DC) and columns without checks (their posterior stays the prior), and an H
# without any edge; random syndromes, every output bit-exact with the float32 oracle
@pytest.mark.parametrize("kernel", ["group", "plain", "lane"])
@pytest.mark.parametrize("case", ["some_empty", "no_edges"])
def test_rows_and_columns_without_edges(P, kernel, case):
    code = _degenerate(case)
    syn = (np.random.default_rng(7).random((300, code.m)) < 0.3).astype(np.uint8)
    prm = _min_sum(P, T=(20, 20), seed=3)
    kid = {"group": P.KERNEL_GROUP, "plain": P.KERNEL_PLAIN, "lane": P.KERNEL_LANE}[kernel]
    plan = P.Plan([P.Code.from_problem(code)], prm, kernel=kid)
    print(f"case degenerate {case} kernel={kernel} tile={plan.info(0)}", flush=True)
    g = gpu_decode(plan, code, syn, shot_offset=2)
    ref = oracle.decode(code, syn, oracle_params(prm, "channel"), precision="f32", shot_offset=2)
    assert ((ref["flags"] & 2) != 0).sum() > 0 and ((ref["flags"] & 1) != 0).sum() > 0
    assert_bit_exact(g, ref, code.n)
