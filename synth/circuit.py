"""Circuit-level detector error model of a bivariate bicycle code (Appendix C).

Two independent constructions of the same decoding problem:

  * ``bb_circuit_matrices``: the detector check matrix H_DCM and the w = 3
    detector degeneracy matrix H_DDM written out from their block formulas
    (Appendix C, the per-round blocks H'_DCM and H'_DDM, stacked over T noisy
    rounds plus the final noiseless round; for [[108,8,10]] the extra DDM
    row block);
  * ``bb_circuit_mechanisms``: the error mechanisms of the syndrome
    extraction circuit itself (Appendix C's eight-step schedule after the
    initialisation step, repeated T times, then a noiseless Z-syndrome round),
    found by propagating the X component of every fault of the circuit-level
    noise model (Sec. IV.D) through the CNOTs (an X on a control spreads to
    the target; initialisation clears a qubit's frame), and merged by equal
    (detectors, logical effect) with the probability that an odd number of
    the merged faults occur.

``bb_circuit_dem`` takes the matrices from the formulas and the priors (and
the logical effect of every column) from the circuit, after checking that the
circuit's mechanisms and the formula's columns correspond one to one.

Fault model (Sec. IV.D / Appendix C), X components only, since only the
Z-type detectors are decoded: an idle flips its qubit with 2p/3 (X or Y); a
CNOT's 15 two-qubit Paulis give X on the control only, on the target only, or
on both, each with 4p/15 (four Paulis each); a Z-basis initialisation flips
with p; a Z measurement reports the wrong outcome with p; X-basis preparation
and measurement errors leave the X frame alone.  Each (fault location, X
pattern) is one independent event of its probability.
"""
from __future__ import annotations

from typing import Dict, List, Tuple

import numpy as np
import scipy.sparse as sp

from .codes import BB_TABLE, Code, Csr, _mod2, bb_matrices, shift_matrix


def bb_monomials(name: str) -> Dict[str, sp.csr_matrix]:
    """A1, A2, A3, B1, B2, B3 of a code of Table I, in the order the polynomials list them."""
    l, m, A_terms, B_terms = BB_TABLE[name]
    x = sp.kron(shift_matrix(l), sp.identity(m, dtype=np.int64)).tocsr()
    y = sp.kron(sp.identity(l, dtype=np.int64), shift_matrix(m)).tocsr()

    def mono(var, e):
        M = sp.identity(l * m, dtype=np.int64, format="csr")
        for _ in range(e):
            M = M @ (x if var == "x" else y)
        return _mod2(M)

    out = {}
    for k, (v, e) in enumerate(A_terms):
        out[f"A{k + 1}"] = mono(v, e)
    for k, (v, e) in enumerate(B_terms):
        out[f"B{k + 1}"] = mono(v, e)
    return out


# ----------------------------------------------------------------------------------------
# the block formulas

def _dcm_round_blocks(M) -> List[List[sp.csr_matrix]]:
    """H'_DCM as 2 x 10 blocks (rows: detectors of rounds t and t+1)."""
    T_ = lambda X: X.T.tocsr()
    A1, A2, A3, B1, B2, B3 = (M[k] for k in ("A1", "A2", "A3", "B1", "B2", "B3"))
    A, B = A1 + A2 + A3, B1 + B2 + B3
    Ab1, Ab2, Ab3 = A2 + A3, A3 + A1, A1 + A2
    Bb1, Bb2, Bb3 = B2 + B3, B3 + B1, B1 + B2
    h = A.shape[0]
    I = sp.identity(h, dtype=np.int64, format="csr")
    Z = sp.csr_matrix((h, h), dtype=np.int64)
    top = [T_(B), T_(A), I, T_(Bb1), T_(Ab1), T_(B3), T_(A2), T_(A2) @ T_(Bb2), T_(A2) @ T_(B3), Z]
    bot = [Z, Z, I, T_(B1), T_(A1), T_(Bb3), T_(Ab2), T_(Ab2) @ T_(B2), T_(Ab2) @ T_(Bb3), T_(Ab2) @ T_(B)]
    return [[_mod2(b) for b in top], [_mod2(b) for b in bot]]


def _ddm_round_blocks(M, extra_108: bool) -> List[List[sp.csr_matrix]]:
    """H'_DDM as 11 (12 with the [[108,8,10]] block) x 12 blocks."""
    A1, A2, A3, B1, B2, B3 = (M[k] for k in ("A1", "A2", "A3", "B1", "B2", "B3"))
    A, B = A1 + A2 + A3, B1 + B2 + B3
    Ab2 = A3 + A1
    h = A.shape[0]
    I = sp.identity(h, dtype=np.int64, format="csr")
    rows = []

    def row(entries):
        r = [None] * 12
        for k, X in entries.items():
            r[k - 1] = X
        return r

    rows.append(row({1: A, 2: B}))
    rows.append(row({1: I, 3: B1, 4: I}))
    rows.append(row({2: I, 3: A1, 5: I}))
    rows.append(row({3: B2, 4: I, 6: I}))
    rows.append(row({3: A3, 5: I, 7: I}))
    rows.append(row({3: B3, 6: I, 11: I}))
    rows.append(row({3: A2, 7: I, 12: I}))
    rows.append(row({1: A2, 7: B2, 8: I}))
    rows.append(row({7: B1, 8: I, 9: I}))
    rows.append(row({7: B3, 9: I, 10: I}))
    rows.append(row({10: I, 11: Ab2}))
    if extra_108:
        rows.append(row({10: A1 @ A1 @ A3 + A1 @ A3 @ A3 + I}))
    Z = sp.csr_matrix((h, h), dtype=np.int64)
    return [[_mod2(X) if X is not None else Z for X in r] for r in rows]


def bb_circuit_matrices(name: str, T: int, extra_108: bool = None):
    """(H_DCM, H_DDM) of T noisy rounds plus the final noiseless round.

    Columns: for t = 1..T the ten blocks of round t (5n columns: data flips
    before round t on L and R, measurement flips, four data-flip blocks during
    the round, three X-ancilla blocks), then n columns for data flips before
    the final round.  DCM rows: detectors of rounds 1..T+1 (n/2 each).  DDM
    rows: eleven row blocks per round (the last two column blocks of round t's
    H'_DDM are the data blocks of round t+1, or the final columns), then H_X
    on the final data columns.
    """
    M = bb_monomials(name)
    h = M["A1"].shape[0]
    n = 2 * h
    if extra_108 is None:
        extra_108 = name == "bb108"
    ncols = T * 5 * n + n
    dblk = _dcm_round_blocks(M)
    dcm = [[None] * (10 * T + 2) for _ in range(T + 1)]
    for t in range(T):
        for r in range(2):
            for c in range(10):
                dcm[t + r][10 * t + c] = dblk[r][c]
    HX, HZ = bb_matrices(*BB_TABLE[name])
    dcm[T][10 * T] = HZ[:, :h]
    dcm[T][10 * T + 1] = HZ[:, h:]
    DCM = _mod2(sp.bmat(dcm, format="csr", dtype=np.int64))
    assert DCM.shape == ((T + 1) * h, ncols)

    rblk = _ddm_round_blocks(M, extra_108)
    nr = len(rblk)
    ddm = [[None] * (10 * T + 2) for _ in range(nr * T + 1)]
    for t in range(T):
        for r in range(nr):
            for c in range(12):
                ddm[nr * t + r][10 * t + c] = rblk[r][c]
    ddm[nr * T][10 * T] = HX[:, :h]
    ddm[nr * T][10 * T + 1] = HX[:, h:]
    # pad empty block columns so that bmat knows every width
    for c in range(10 * T + 2):
        if all(ddm[r][c] is None for r in range(len(ddm))):
            ddm[0][c] = sp.csr_matrix((h, h), dtype=np.int64)
    DDM = _mod2(sp.bmat(ddm, format="csr", dtype=np.int64))
    assert DDM.shape == ((nr * T + 1) * h, ncols)
    return Csr.from_sparse(DCM), Csr.from_sparse(DDM)


# ----------------------------------------------------------------------------------------
# the circuit

def _perm(P: sp.csr_matrix) -> np.ndarray:
    """j = P(i) when P has its one of row i in column j."""
    P = P.tocsr()
    assert (np.diff(P.indptr) == 1).all()
    return P.indices.astype(np.int64).copy()


def bb_circuit_schedule(name: str, T: int):
    """The syndrome extraction circuit as a list of slots; each slot is a list of
    operations (kind, arrays).  Qubits: L i -> i, R i -> h + i, X i -> 2h + i,
    Z i -> 3h + i."""
    M = bb_monomials(name)
    h = M["A1"].shape[0]
    ar = np.arange(h)
    Lq, Rq, Xq, Zq = ar, h + ar, 2 * h + ar, 3 * h + ar
    p = {k: _perm(v) for k, v in M.items()}
    pT = {k: _perm(v.T) for k, v in M.items()}
    slots = [[("idle", Xq), ("initz", Zq), ("idle", Lq), ("idle", Rq)]]
    for t in range(T):
        slots.append([("initx", Xq), ("cnot", Rq[pT["A1"]], Zq), ("idle", Lq)])
        slots.append([("cnot", Xq, Lq[p["A2"]]), ("cnot", Rq[pT["A3"]], Zq)])
        slots.append([("cnot", Xq, Rq[p["B2"]]), ("cnot", Lq[pT["B1"]], Zq)])
        slots.append([("cnot", Xq, Rq[p["B1"]]), ("cnot", Lq[pT["B2"]], Zq)])
        slots.append([("cnot", Xq, Rq[p["B3"]]), ("cnot", Lq[pT["B3"]], Zq)])
        slots.append([("cnot", Xq, Lq[p["A1"]]), ("cnot", Rq[pT["A2"]], Zq)])
        slots.append([("cnot", Xq, Lq[p["A3"]]), ("measz", Zq, t), ("idle", Rq)])
        slots.append([("measx", Xq), ("initz", Zq), ("idle", Lq), ("idle", Rq)])
    return slots, h


def bb_circuit_mechanisms(name: str, T: int, p: float):
    """Error mechanisms of the circuit: (detector matrix [E, (T+1) h] uint8,
    logical effect [E, k] uint8, probability [E]), merged by equal
    (detectors, logical effect), mechanisms with no effect dropped."""
    from .codes import bb_code
    slots, h = bb_circuit_schedule(name, T)
    n = 2 * h
    nq = 4 * h
    # events: (slot, qubits flipped after the slot's operations, or a measurement flip)
    ev_slot, ev_q1, ev_q2, ev_meas, ev_p = [], [], [], [], []

    def add(s, q1, q2, meas, prob):
        k = len(q1)
        ev_slot.append(np.full(k, s)); ev_q1.append(q1); ev_q2.append(q2)
        ev_meas.append(np.full(k, meas, dtype=bool)); ev_p.append(np.full(k, prob))

    none = lambda a: np.full(len(a), -1)
    for s, ops in enumerate(slots):
        for op in ops:
            kind = op[0]
            if kind == "idle":
                add(s, op[1], none(op[1]), False, 2 * p / 3)
            elif kind == "initz":
                add(s, op[1], none(op[1]), False, p)
            elif kind == "cnot":
                c, t_ = op[1], op[2]
                add(s, c, none(c), False, 4 * p / 15)
                add(s, t_, none(t_), False, 4 * p / 15)
                add(s, c, t_, False, 4 * p / 15)
            elif kind == "measz":
                add(s, op[1], none(op[1]), True, p)
    ev_slot = np.concatenate(ev_slot); ev_q1 = np.concatenate(ev_q1); ev_q2 = np.concatenate(ev_q2)
    ev_meas = np.concatenate(ev_meas); ev_p = np.concatenate(ev_p)
    E = len(ev_slot)
    frame = np.zeros((E, nq), dtype=np.uint8)
    out = np.zeros((E, T, h), dtype=np.uint8)
    rows = np.arange(E)
    for s, ops in enumerate(slots):
        for op in ops:
            kind = op[0]
            if kind == "cnot":
                frame[:, op[2]] ^= frame[:, op[1]]
            elif kind in ("initz", "initx"):
                frame[:, op[1]] = 0
            elif kind == "measz":
                out[:, op[2], :] = frame[:, op[1]]
        sel = ev_slot == s
        a = sel & ~ev_meas
        frame[rows[a], ev_q1[a]] ^= 1
        b = a & (ev_q2 >= 0)
        frame[rows[b], ev_q2[b]] ^= 1
        m = sel & ev_meas
        if m.any():
            t_meas = [op[2] for op in ops if op[0] == "measz"][0]
            out[rows[m], t_meas, ev_q1[m] - 3 * h] ^= 1
    data = frame[:, :n]
    base = bb_code(name)
    HZ = base.H.to_sparse()
    final = (data.astype(np.int64) @ HZ.T.toarray().astype(np.int64)) % 2
    det = np.zeros((E, T + 1, h), dtype=np.uint8)
    det[:, 0] = out[:, 0]
    det[:, 1:T] = out[:, 1:] ^ out[:, :-1]
    det[:, T] = final.astype(np.uint8) ^ out[:, T - 1]
    det = det.reshape(E, -1)
    obs = ((data.astype(np.int64) @ base.O.T.astype(np.int64)) % 2).astype(np.uint8)
    key = np.packbits(np.concatenate([det, obs], axis=1), axis=1)
    live = key.any(axis=1)
    keyv = np.ascontiguousarray(key[live]).view(np.dtype((np.void, key.shape[1]))).ravel()
    uniq, first, inv = np.unique(keyv, return_index=True, return_inverse=True)
    # probability that an odd number of the merged independent events occur
    lg = np.zeros(len(uniq))
    np.add.at(lg, inv, np.log1p(-2.0 * ev_p[live]))
    prob = 0.5 * (1.0 - np.exp(lg))
    idx = np.nonzero(live)[0][first]
    return det[idx], obs[idx], prob, {"events": E, "merged_events": np.bincount(inv)}


def bb_circuit_dem(name: str = "bb144", T: int = 12, p: float = 0.003) -> Code:
    """Decoding problem of T noisy rounds of the circuit: H = H_DCM, D = H_DDM (w = 3),
    priors and logical effects from the circuit's mechanisms (columns matched by
    their detectors; one mechanism per column, checked)."""
    H, D = bb_circuit_matrices(name, T)
    det, obs, prob, _ = bb_circuit_mechanisms(name, T, p)
    Hs = H.to_sparse().tocsc()
    ncols = H.cols
    colkey = np.packbits(Hs.T.toarray().astype(np.uint8), axis=1)
    ck = np.ascontiguousarray(colkey).view(np.dtype((np.void, colkey.shape[1]))).ravel()
    mk = np.ascontiguousarray(np.packbits(det, axis=1)).view(np.dtype((np.void, colkey.shape[1]))).ravel()
    order = np.argsort(ck)
    assert len(np.unique(ck)) == ncols, "formula columns are not distinct"
    pos = np.searchsorted(ck[order], mk)
    pos = np.minimum(pos, ncols - 1)
    col = order[pos]
    if not (ck[col] == mk).all() or len(np.unique(col)) != ncols or len(mk) != ncols:
        raise ValueError("circuit mechanisms and formula columns do not correspond one to one")
    priors = np.empty(ncols)
    priors[col] = prob
    O = np.zeros((obs.shape[1], ncols), dtype=np.uint8)
    O[:, col] = obs.T
    return Code(f"{name}_circuit_T{T}", H, D, priors, O, "channel",
                {"family": "bb_circuit", "T": T, "p": p, "base": name})
