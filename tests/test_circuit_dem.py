"""Pins of the circuit-level detector error model of BB codes (Appendix C):
the matrices written from the paper's block formulas against the mechanisms of
the syndrome circuit, against the paper's stated weights and its weight-3
completeness statement, and the aggregated priors against closed forms.

The two constructions in synth/circuit.py share only the monomials A_i, B_i:
the block formulas are transcribed from Appendix C, the mechanisms come from
propagating the X part of every fault through the eight-step schedule."""
import numpy as np
import pytest
import scipy.sparse as sp

import synth
from synth import circuit as SC


@pytest.mark.parametrize("name,T", [("bb72", 1), ("bb72", 2), ("bb72", 3), ("bb108", 3), ("bb144", 3)])
def test_circuit_mechanisms_are_the_printed_dcm_columns(name, T):
    """Every mechanism of the circuit is one column of the printed H_DCM and every
    column one mechanism (a bijection on detector signatures); columns are distinct
    and nonzero, so no error of weight <= 2 is trivial."""
    code = SC.bb_circuit_dem(name, T, 0.002)
    H = code.H.to_sparse()
    h = H.shape[0] // (T + 1)
    assert H.shape == ((T + 1) * h, T * 10 * h + 2 * h)
    assert (code.H.col_weights() > 0).all()
    assert ((code.priors > 0) & (code.priors < 0.5)).all()


def test_schedule_change_breaks_the_correspondence(monkeypatch):
    """The bijection is sensitive to the circuit: exchanging the CNOT layers of steps
    3 and 4 (the order in which the Z ancillas meet B1^T and B2^T) breaks it."""
    orig = SC.bb_circuit_schedule

    def swapped(name, T):
        slots, h = orig(name, T)
        for t in range(T):
            s3, s4 = 1 + 8 * t + 2, 1 + 8 * t + 3
            slots[s3], slots[s4] = slots[s4], slots[s3]
        return slots, h

    monkeypatch.setattr(SC, "bb_circuit_schedule", swapped)
    with pytest.raises(ValueError):
        SC.bb_circuit_dem("bb72", 2, 0.002)


def test_dcm_shape_and_weights_bb144_T12():
    """Appendix C: H_DCM has row weight 35 and column weight 6; T = d = 12 rounds of
    [[144,12,12]] give (T+1) n/2 = 936 detectors and 5nT + n = 8784 columns."""
    H, D = SC.bb_circuit_matrices("bb144", 12)
    assert (H.rows, H.cols) == (936, 8784)
    assert H.row_weights().max() == 35
    assert H.col_weights().max() == 6
    assert (D.rows, D.cols) == (12 * 11 * 72 + 72, 8784)
    assert set(np.unique(D.row_weights()).tolist()) == {3, 6}


@pytest.mark.parametrize("name,T", [("bb72", 3), ("bb144", 4)])
def test_ddm_annihilates_dcm_and_logicals(name, T):
    """H_DDM H_DCM^T = 0 and H_DDM O^T = 0, with O the logical effect of each column
    from the circuit.  Column weight of the printed formula: 8 on the L data blocks
    of rounds 2..T (5 from round t's rows, 3 from round t-1's), where the text says 7."""
    code = SC.bb_circuit_dem(name, T, 0.002)
    Hd, Dd = code.H.to_sparse(), code.D.to_sparse()
    assert not ((Dd @ Hd.T).toarray() % 2).any()
    assert not ((Dd @ sp.csr_matrix(code.O.astype(np.int64)).T).toarray() % 2).any()
    assert code.D.row_weights().max() == 6
    assert code.D.col_weights().max() == 8


def _trivial_weight3(code):
    """All e of weight 3 with e H^T = 0 and e O^T = 0, by a random linear hash of the
    stacked columns of (H; O) (pairs a < b, the third column looked up), each
    candidate checked exactly."""
    S = np.concatenate([code.H.to_dense(), code.O], axis=0).astype(np.uint8)
    rng = np.random.default_rng(7)
    R = rng.integers(0, 2 ** 62, size=S.shape[0], dtype=np.int64).astype(np.uint64)
    hc = np.zeros(S.shape[1], dtype=np.uint64)
    for r in range(S.shape[0]):
        hc[np.nonzero(S[r])[0]] ^= R[r]
    assert len(np.unique(hc)) == len(hc)      # no trivial error of weight 2
    order = np.argsort(hc)
    hs = hc[order]
    n = len(hc)
    out = set()
    for a in range(n):
        x = hc[a] ^ hc[a + 1:]
        pos = np.minimum(np.searchsorted(hs, x), n - 1)
        for bi in np.nonzero(hs[pos] == x)[0]:
            b, c = a + 1 + bi, int(order[pos[bi]])
            if c > b:
                e = np.zeros(S.shape[1], np.int64)
                e[[a, b, c]] = 1
                assert not ((S.astype(np.int64) @ e) % 2).any()
                out.add((a, b, c))
    return out


@pytest.mark.parametrize("name", ["bb72", "bb108", "bb144"])
def test_weight3_trivial_errors_are_ddm_rows(name):
    """Appendix D: every weight-3 e with e H_DCM^T = 0 and e O^T = 0 is a row of the
    w = 3 H_DDM for the BB codes, [[108,8,10]] only with its extra row block
    (T = 3, one placement of the local window)."""
    T = 3
    code = SC.bb_circuit_dem(name, T, 0.002)
    triv = _trivial_weight3(code)
    rows = {tuple(code.D.row(i).tolist()) for i in range(code.D.rows)}
    rows3 = {r for r in rows if len(r) == 3}
    assert triv == rows3
    if name == "bb108":
        _, D0 = SC.bb_circuit_matrices(name, T, extra_108=False)
        rows0 = {tuple(D0.row(i).tolist()) for i in range(D0.rows)}
        assert len(triv - rows0) > 0


def test_priors_closed_forms():
    """Aggregated priors (odd number of independent merged faults):
      * R data flips between the CNOTs of steps 1 and 2 (fifth column block): the
        control-only X of the step-1 CNOT and the X on both qubits of the step-2 CNOT,
        4p/15 each: 8p/15 - 2 (4p/15)^2 (the merge example of Appendix C);
      * measurement flips (third block): the Z-measurement flip p, the flip of the
        ancilla's preparation p, and the target-only X of its six CNOTs, 4p/15 each."""
    p = 0.004
    q = 4 * p / 15
    T = 3
    code = SC.bb_circuit_dem("bb72", T, p)
    n, h = 72, 36
    for t in range(T):
        base = t * 5 * n
        np.testing.assert_allclose(code.priors[base + 4 * h: base + 5 * h], 2 * q * (1 - q), rtol=1e-12)
        np.testing.assert_allclose(code.priors[base + 2 * h: base + 3 * h],
                                   0.5 * (1 - (1 - 2 * p) ** 2 * (1 - 2 * q) ** 6), rtol=1e-12)
