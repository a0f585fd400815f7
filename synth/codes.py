"""Parity-check matrices of the codes and detector error models decoded here.

Every matrix is over F2 and is returned in CSR form with sorted, unique
column indices (``Csr``).  A ``Code`` bundles the Tanner-graph matrix ``H``
(H_Z, or the detector check matrix), the degeneracy matrix ``D`` used by
degeneracy cutting (H_X, or the detector degeneracy matrix), per-column prior
error probabilities and the logical-operator matrix used only to score
decodes.

Constructions (paper sections in brackets):
  * toric code of size L as the hypergraph product of the length-L cyclic
    repetition code [Sec. II.B, Kitaev's toric code];
  * rotated surface code of odd distance d, [[d^2, 1, d]] [Sec. II.B];
  * bivariate bicycle codes H_X = (A|B), H_Z = (B^T|A^T) with x = S_l (x) I_m,
    y = I_l (x) S_m [Sec. II.B, Table I];
  * hypergraph products of random (3,4)-regular classical codes (a synthetic
    family of uneven sizes, not from the paper);
  * the phenomenological detector check / degeneracy matrices, a staircase of
    T blocks ((H_Z, I), (0, I)) and ((H_X, 0, 0), (I, H_Z^T, I)) plus a final
    noiseless round [Sec. IV.C, the two block equations there].
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Optional, Sequence, Tuple

import numpy as np
import scipy.sparse as sp


@dataclass
class Csr:
    """Binary sparse matrix: rows x cols, 0-based sorted unique column indices."""
    rows: int
    cols: int
    row_ptr: np.ndarray
    col_idx: np.ndarray

    @staticmethod
    def from_sparse(S) -> "Csr":
        S = sp.csr_matrix(S, dtype=np.int64)
        S.sum_duplicates()
        S.data %= 2
        S.eliminate_zeros()
        S.sort_indices()
        return Csr(S.shape[0], S.shape[1], S.indptr.astype(np.int32).copy(),
                   S.indices.astype(np.int32).copy())

    @staticmethod
    def from_dense(A) -> "Csr":
        return Csr.from_sparse(sp.csr_matrix(np.asarray(A, dtype=np.int64) % 2))

    def to_sparse(self):
        data = np.ones(len(self.col_idx), dtype=np.int64)
        return sp.csr_matrix((data, self.col_idx, self.row_ptr), shape=(self.rows, self.cols))

    def to_dense(self) -> np.ndarray:
        return self.to_sparse().toarray().astype(np.uint8)

    @property
    def nnz(self) -> int:
        return int(self.row_ptr[-1])

    def row_weights(self) -> np.ndarray:
        return np.diff(self.row_ptr)

    def col_weights(self) -> np.ndarray:
        return np.bincount(self.col_idx, minlength=self.cols)

    def row(self, i: int) -> np.ndarray:
        return self.col_idx[self.row_ptr[i]:self.row_ptr[i + 1]]


@dataclass
class Code:
    """One decoding problem: Tanner graph H, degeneracy matrix D, priors, logicals."""
    name: str
    H: Csr
    D: Csr
    priors: np.ndarray                      # float64 [n], each in (0, 1)
    O: Optional[np.ndarray] = None          # uint8 [k, n] logical matrix (scoring only)
    second_pass: str = "channel"            # "channel" (BB, HGP, DEM) or "posterior" (toric)
    meta: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return self.H.cols

    @property
    def m(self) -> int:
        return self.H.rows

    def with_priors(self, p) -> "Code":
        pri = np.broadcast_to(np.asarray(p, dtype=np.float64), (self.n,)).copy()
        return Code(self.name, self.H, self.D, pri, self.O, self.second_pass, dict(self.meta))


# ----------------------------------------------------------------------------------------
# elementary matrices

def shift_matrix(l: int) -> sp.csr_matrix:
    """Cyclic shift S_l with (S_l)_{ij} = 1 iff j = i + 1 mod l."""
    i = np.arange(l)
    return sp.csr_matrix((np.ones(l, dtype=np.int64), (i, (i + 1) % l)), shape=(l, l))


def repetition_cycle(L: int) -> sp.csr_matrix:
    """Parity checks of the length-L cyclic repetition code, I + S_L (L x L)."""
    return (sp.identity(L, dtype=np.int64, format="csr") + shift_matrix(L)).tocsr()


def _mod2(S) -> sp.csr_matrix:
    S = sp.csr_matrix(S, dtype=np.int64)
    S.data %= 2
    S.eliminate_zeros()
    return S


# ----------------------------------------------------------------------------------------
# code families

def hgp_matrices(Hc) -> Tuple[sp.csr_matrix, sp.csr_matrix]:
    """Hypergraph product of a classical check matrix Hc (m_c x n_c) with itself.

    H_X = [Hc (x) I_{n_c} | I_{m_c} (x) Hc^T],  H_Z = [I_{n_c} (x) Hc | Hc^T (x) I_{m_c}],
    n = n_c^2 + m_c^2 qubits, m_X = m_Z = m_c n_c checks, H_X H_Z^T = 0 over F2.
    """
    Hc = sp.csr_matrix(Hc, dtype=np.int64)
    mc, nc = Hc.shape
    In, Im = sp.identity(nc, dtype=np.int64), sp.identity(mc, dtype=np.int64)
    HX = sp.hstack([sp.kron(Hc, In), sp.kron(Im, Hc.T)])
    HZ = sp.hstack([sp.kron(In, Hc), sp.kron(Hc.T, Im)])
    return _mod2(HX), _mod2(HZ)


def hgp_code(Hc, name: str = "hgp", p: float = 0.05, second_pass: str = "channel",
             with_logicals: bool = True) -> Code:
    from .f2 import logical_operators
    HX, HZ = hgp_matrices(Hc)
    H, D = Csr.from_sparse(HZ), Csr.from_sparse(HX)
    O = logical_operators(D, H) if with_logicals else None
    return Code(name, H, D, np.full(H.cols, p), O, second_pass,
                {"family": "hgp", "classical_shape": tuple(sp.csr_matrix(Hc).shape)})


def toric_code(L: int, p: float = 0.05, second_pass: str = "posterior") -> Code:
    """Toric code of size L: hypergraph product of the cyclic repetition code.

    H_Z is L^2 x 2L^2 with row weight 4 and column weight 2; k = 2.
    """
    c = hgp_code(repetition_cycle(L), name=f"toric{L}", p=p, second_pass=second_pass)
    c.meta.update({"family": "toric", "L": L})
    return c


def rotated_surface_matrices(d: int):
    """Rotated surface code of odd distance d on a d x d grid of data qubits.

    Data qubit (r, c) is column r d + c.  Stabilisers sit on the faces (i, j),
    0 <= i, j <= d, between qubits (i-1..i, j-1..j) that exist: X-type where
    i + j is even, Z-type where it is odd; interior faces have weight 4, and
    the weight-2 faces kept are the X-type ones on the top and bottom edges
    (i = 0, d) and the Z-type ones on the left and right edges (j = 0, d).
    Gives (d^2 - 1) / 2 stabilisers of each type and k = 1.
    """
    assert d >= 3 and d % 2 == 1
    xs, zs = [], []
    for i in range(d + 1):
        for j in range(d + 1):
            qs = [r * d + c for r in (i - 1, i) for c in (j - 1, j) if 0 <= r < d and 0 <= c < d]
            xtype = (i + j) % 2 == 0
            edge_tb = i in (0, d)
            edge_lr = j in (0, d)
            if len(qs) == 4 or (len(qs) == 2 and ((xtype and edge_tb) or (not xtype and edge_lr))):
                (xs if xtype else zs).append(sorted(qs))

    def mat(rows):
        M = sp.lil_matrix((len(rows), d * d), dtype=np.int64)
        for k, qs in enumerate(rows):
            for q in qs:
                M[k, q] = 1
        return sp.csr_matrix(M)
    return mat(xs), mat(zs)


def rotated_surface_code(d: int, p: float = 0.01, second_pass: str = "posterior") -> Code:
    """Rotated surface code [[d^2, 1, d]] [Sec. II.B]: H = H_Z (detects bit flips), D = H_X."""
    from .f2 import logical_operators
    HX, HZ = rotated_surface_matrices(d)
    H, D = Csr.from_sparse(HZ), Csr.from_sparse(HX)
    return Code(f"surface{d}", H, D, np.full(H.cols, p), logical_operators(D, H), second_pass,
                {"family": "rotated_surface", "d": d})


def bb_matrices(l: int, m: int, A_terms: Sequence[Tuple[str, int]],
                B_terms: Sequence[Tuple[str, int]]):
    """Bivariate bicycle code: A = sum of monomials, B likewise, H_X=(A|B), H_Z=(B^T|A^T)."""
    x = sp.kron(shift_matrix(l), sp.identity(m, dtype=np.int64)).tocsr()
    y = sp.kron(sp.identity(l, dtype=np.int64), shift_matrix(m)).tocsr()

    def mono(var: str, e: int):
        base = x if var == "x" else y
        M = sp.identity(l * m, dtype=np.int64, format="csr")
        for _ in range(e):
            M = M @ base
        return M

    A = _mod2(sum(mono(v, e) for v, e in A_terms))
    B = _mod2(sum(mono(v, e) for v, e in B_terms))
    HX = _mod2(sp.hstack([A, B]))
    HZ = _mod2(sp.hstack([B.T, A.T]))
    return HX, HZ


BB_TABLE = {
    # name: (l, m, A, B) -- Table I of the paper, plus the distance-18 code (l = m = 12)
    "bb72": (6, 6, [("x", 3), ("y", 1), ("y", 2)], [("y", 3), ("x", 1), ("x", 2)]),
    "bb108": (9, 6, [("x", 3), ("y", 1), ("y", 2)], [("y", 3), ("x", 1), ("x", 2)]),
    "bb144": (12, 6, [("x", 3), ("y", 1), ("y", 2)], [("y", 3), ("x", 1), ("x", 2)]),
    "bb288": (12, 12, [("x", 3), ("y", 2), ("y", 7)], [("y", 3), ("x", 1), ("x", 2)]),
}


def bb_code(name: str = "bb144", p: float = 0.05, second_pass: str = "channel") -> Code:
    from .f2 import logical_operators
    l, m, A, B = BB_TABLE[name]
    HX, HZ = bb_matrices(l, m, A, B)
    H, D = Csr.from_sparse(HZ), Csr.from_sparse(HX)
    return Code(name, H, D, np.full(H.cols, p), logical_operators(D, H), second_pass,
                {"family": "bb", "l": l, "m": m})


def random_regular_classical(n_c: int, seed: int, dv: int = 3, dc: int = 4,
                             max_tries: int = 10000) -> sp.csr_matrix:
    """Random (dv, dc)-regular bipartite graph by the configuration model.

    n_c bits of degree dv, m_c = dv n_c / dc checks of degree dc; the stub
    matching is resampled until no bit meets a check twice.  Returns the
    m_c x n_c check matrix.
    """
    assert (dv * n_c) % dc == 0
    m_c = dv * n_c // dc
    rng = np.random.default_rng(seed)
    var_stubs = np.repeat(np.arange(n_c), dv)
    chk_stubs = np.repeat(np.arange(m_c), dc)
    for _ in range(max_tries):
        perm = rng.permutation(len(chk_stubs))
        pairs = chk_stubs[perm] * n_c + var_stubs
        if len(np.unique(pairs)) == len(pairs):
            M = sp.csr_matrix((np.ones(len(pairs), dtype=np.int64), (chk_stubs[perm], var_stubs)),
                              shape=(m_c, n_c))
            return _mod2(M)
    raise RuntimeError("configuration model did not produce a simple graph")


def hgp_batch_codes(count: int = 64, base_seed: int = 4000, p: float = 0.03,
                    sizes: Sequence[int] = tuple(range(16, 65, 4)),
                    with_logicals: bool = False):
    """The uneven batch: `count` HGP codes of random (3,4)-regular classical codes.

    Code j uses classical size n_c drawn uniformly from `sizes` (seeded by
    base_seed) and graph seed base_seed + j.
    """
    rng = np.random.default_rng(base_seed)
    ncs = rng.choice(np.asarray(sizes), size=count)
    out = []
    for j, nc in enumerate(ncs):
        Hc = random_regular_classical(int(nc), base_seed + 1 + j)
        c = hgp_code(Hc, name=f"hgp{j}_nc{nc}", p=p, with_logicals=with_logicals)
        c.meta.update({"n_c": int(nc), "index": j})
        out.append(c)
    return out


# ----------------------------------------------------------------------------------------
# phenomenological detector error model

def phenomenological_dem(base: Code, T: int, p_data: float, p_meas: float,
                         final_noiseless_round: bool = True) -> Code:
    """Detector check / degeneracy matrices for T noisy rounds of Z-syndrome extraction.

    Column order: for t = 1..T the n data-flip mechanisms before round t, then
    the m_Z measurement flips of round t; with a final noiseless round, n more
    data mechanisms before it.  Detector rows are d_{i,t} for t = 1..T (+1).

    DCM: data_t -> H_Z in detector block t; meas_t -> I in blocks t and t+1.
    DDM: per round, H_X on data_t (stabilizer degeneracy) and (I, H_Z^T, I) on
    (data_t, meas_t, data_{t+1}) (a data flip in two consecutive rounds equals
    flips of its checks' measurements); with the final round, H_X on data_{T+1}.
    Without the final noiseless round the t = T measurement columns have weight 1
    and the (I, H_Z^T, I) block at t = T is omitted (it would flip a logical).
    """
    HZ = base.H.to_sparse().astype(np.int64)
    HX = base.D.to_sparse().astype(np.int64)
    n, mZ, mX = base.n, base.m, base.D.rows
    blk = n + mZ
    ncols = T * blk + (n if final_noiseless_round else 0)
    nrounds = T + 1 if final_noiseless_round else T

    def data_col(t):  # t in 1..T(+1)
        return (t - 1) * blk

    def meas_col(t):
        return (t - 1) * blk + n

    # detector check matrix
    r_i, c_i = [], []
    HZc = HZ.tocoo()
    Im = np.arange(mZ)
    for t in range(1, T + 1):
        r_i.append((t - 1) * mZ + HZc.row); c_i.append(data_col(t) + HZc.col)
        r_i.append((t - 1) * mZ + Im); c_i.append(meas_col(t) + Im)
        if t + 1 <= nrounds:
            r_i.append(t * mZ + Im); c_i.append(meas_col(t) + Im)
    if final_noiseless_round:
        r_i.append(T * mZ + HZc.row); c_i.append(data_col(T + 1) + HZc.col)
    r_i, c_i = np.concatenate(r_i), np.concatenate(c_i)
    DCM = sp.csr_matrix((np.ones(len(r_i), dtype=np.int64), (r_i, c_i)), shape=(nrounds * mZ, ncols))

    # detector degeneracy matrix
    rows, cols = [], []
    HXc = HX.tocoo()
    HZTc = HZ.T.tocoo()
    In = np.arange(n)
    row0 = 0
    for t in range(1, T + 1):
        rows.append(row0 + HXc.row); cols.append(data_col(t) + HXc.col)
        row0 += mX
        if t < T or final_noiseless_round:
            rows.append(row0 + In); cols.append(data_col(t) + In)
            rows.append(row0 + HZTc.row); cols.append(meas_col(t) + HZTc.col)
            rows.append(row0 + In); cols.append(data_col(t + 1) + In)
            row0 += n
    if final_noiseless_round:
        rows.append(row0 + HXc.row); cols.append(data_col(T + 1) + HXc.col)
        row0 += mX
    rows, cols = np.concatenate(rows), np.concatenate(cols)
    DDM = sp.csr_matrix((np.ones(len(rows), dtype=np.int64), (rows, cols)), shape=(row0, ncols))

    priors = np.empty(ncols)
    is_meas = np.zeros(ncols, dtype=bool)
    for t in range(1, T + 1):
        is_meas[meas_col(t):meas_col(t) + mZ] = True
    priors[:] = p_data
    priors[is_meas] = p_meas

    O = None
    if base.O is not None:
        k = base.O.shape[0]
        O = np.zeros((k, ncols), dtype=np.uint8)
        for t in range(1, T + 1 + (1 if final_noiseless_round else 0)):
            O[:, data_col(t):data_col(t) + n] = base.O
    form = "paper" if final_noiseless_round else "open"
    return Code(f"{base.name}_phen_T{T}_{form}", Csr.from_sparse(DCM), Csr.from_sparse(DDM),
                priors, O, "channel",
                {"family": "phenomenological", "T": T, "final_noiseless_round": final_noiseless_round,
                 "base": base.name, "is_meas": is_meas})
