"""Linear algebra over F2, used to build logical operators and to score decodes.

Rows are bit-packed into uint64 words and reduced with vectorised XORs.
Nothing here is part of the decoder; it only scores its outputs: a decode of
error e with estimate e_hat fails when e_hat does not reproduce the syndrome
or the residual e + e_hat anticommutes with a logical operator (Sec. II.C).
"""
from __future__ import annotations

import numpy as np


def _pack_rows(A: np.ndarray) -> np.ndarray:
    A = np.asarray(A, dtype=np.uint8) & 1
    r, c = A.shape
    nb = (c + 63) // 64
    pad = np.zeros((r, nb * 64), dtype=np.uint8)
    pad[:, :c] = A
    return np.packbits(pad, axis=1, bitorder="little").view("<u8").reshape(r, nb).copy()


def _unpack_rows(P: np.ndarray, c: int) -> np.ndarray:
    b = np.unpackbits(P.view(np.uint8).reshape(P.shape[0], -1), axis=1, bitorder="little")
    return b[:, :c].astype(np.uint8)


def _row_reduce(P: np.ndarray, ncols: int):
    """In-place reduced row echelon form of packed rows; returns pivot columns."""
    P = P.copy()
    r = P.shape[0]
    pivots = []
    row = 0
    for col in range(ncols):
        if row >= r:
            break
        w, b = col >> 6, np.uint64(1) << np.uint64(col & 63)
        hits = np.nonzero(P[row:, w] & b)[0]
        if len(hits) == 0:
            continue
        piv = row + hits[0]
        if piv != row:
            P[[row, piv]] = P[[piv, row]]
        mask = (P[:, w] & b) != 0
        mask[row] = False
        P[mask] ^= P[row]
        pivots.append(col)
        row += 1
    return P[:row], pivots


def f2_rank(A) -> int:
    A = _dense(A)
    if A.shape[0] == 0:
        return 0
    _, piv = _row_reduce(_pack_rows(A), A.shape[1])
    return len(piv)


def _dense(A) -> np.ndarray:
    if hasattr(A, "to_dense"):
        return A.to_dense()
    if hasattr(A, "toarray"):
        return (A.toarray() % 2).astype(np.uint8)
    return np.asarray(A, dtype=np.uint8) & 1


def nullspace(A) -> np.ndarray:
    """Basis (rows) of {x : A x^T = 0} over F2."""
    A = _dense(A)
    n = A.shape[1]
    R, piv = _row_reduce(_pack_rows(A), n)
    Rd = _unpack_rows(R, n) if len(piv) else np.zeros((0, n), dtype=np.uint8)
    pivset = set(piv)
    free = np.array([c for c in range(n) if c not in pivset], dtype=np.int64)
    basis = np.zeros((len(free), n), dtype=np.uint8)
    basis[np.arange(len(free)), free] = 1
    if len(piv) and len(free):
        basis[:, np.asarray(piv)] = Rd[:, free].T
    return basis


def _row_ints(A: np.ndarray):
    P = np.packbits(np.asarray(A, dtype=np.uint8), axis=1, bitorder="little")
    return [int.from_bytes(row.tobytes(), "little") for row in P]


def logical_operators(HX, HZ) -> np.ndarray:
    """Z-type logicals O_Z: a basis of ker(H_X) completing rowspace(H_Z).

    A residual r with r H_Z^T = 0 is trivial iff r O_Z^T = 0 (r then lies in
    rowspace(H_X), the orthogonal complement of ker(H_X)).
    """
    HXd, HZd = _dense(HX), _dense(HZ)
    n = HXd.shape[1]
    N = nullspace(HXd)
    basis = {}                      # leading bit -> row (Python int bitset)

    def insert(v: int) -> bool:
        while v:
            top = v.bit_length() - 1
            if top in basis:
                v ^= basis[top]
            else:
                basis[top] = v
                return True
        return False

    for v in _row_ints(HZd):
        insert(v)
    keep = [i for i, v in enumerate(_row_ints(N)) if insert(v)] if len(N) else []
    k = n - f2_rank(HXd) - f2_rank(HZd)
    O = N[keep].astype(np.uint8).reshape(-1, n)
    assert O.shape[0] == k, (O.shape, k)
    return O


def residual_is_logical(residual: np.ndarray, O: np.ndarray) -> np.ndarray:
    """Per row of `residual` (uint8 [B, n]): True iff it flips some logical."""
    R = np.asarray(residual, dtype=np.int64)
    return ((R @ np.asarray(O, dtype=np.int64).T) % 2).any(axis=1)
