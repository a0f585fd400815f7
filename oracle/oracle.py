"""ctypes wrapper of the CPU oracle ``bpdc_oracle.cpp`` (test infrastructure only).

The oracle takes unpacked byte syndromes and returns unpacked byte
corrections; it does its own prior-LLR conversion and its own tie-break
hash.  Nothing here is imported by the GPU library.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass
from typing import Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "bpdc_oracle.cpp")
LIB = os.path.join(HERE, "liboracle.so")

MIN_SUM, PRODUCT_SUM = 0, 1


def lib_path() -> str:
    return LIB


def build(force: bool = True) -> str:
    """Compile the oracle with g++ (-O2, no FP contraction, no fast-math, OpenMP)."""
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        tmp = LIB + ".tmp"
        subprocess.check_call(["g++", "-std=c++17", "-O2", "-ffp-contract=off", "-fno-fast-math",
                               "-fopenmp", "-fPIC", "-shared", "-Wall", "-o", tmp, SRC])
        os.replace(tmp, LIB)
    return LIB


class _Params(C.Structure):
    _fields_ = [("rule", C.c_int32), ("max_iter1", C.c_int32), ("max_iter2", C.c_int32),
                ("second_pass_prior", C.c_int32), ("stop_on_converge", C.c_int32),
                ("tie_break", C.c_int32), ("dc_form", C.c_int32), ("skip_dc", C.c_int32),
                ("alpha", C.c_double), ("llr_sat", C.c_double), ("tie_eps", C.c_double),
                ("seed", C.c_uint64), ("soft_period", C.c_int32), ("soft_shift", C.c_double)]


@dataclass
class OracleParams:
    rule: int = MIN_SUM
    max_iter1: int = 100
    max_iter2: int = 100
    second_pass_prior: str = "channel"     # or "posterior"
    stop_on_converge: bool = True
    tie_break: str = "hash"                # or "lowest"
    dc_form: str = "zero_prior"            # Alg. 2; or "delete_columns" (Alg. 1)
    skip_dc: bool = False
    alpha: float = 0.625
    llr_sat: float = 64.0
    tie_eps: float = 1e-3
    seed: int = 0
    soft_period: int = 0                   # intermittent soft DC every soft_period pass-1 iterations
    soft_shift: float = 0.0                # prior-LLR increase of each soft nominee

    def to_c(self) -> _Params:
        return _Params(self.rule, self.max_iter1, self.max_iter2,
                       1 if self.second_pass_prior == "posterior" else 0,
                       1 if self.stop_on_converge else 0,
                       1 if self.tie_break == "lowest" else 0,
                       1 if self.dc_form == "delete_columns" else 0,
                       1 if self.skip_dc else 0,
                       float(self.alpha), float(self.llr_sat), float(self.tie_eps),
                       int(self.seed) & 0xFFFFFFFFFFFFFFFF, int(self.soft_period), float(self.soft_shift))


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build(force=False)
        lib = C.CDLL(LIB)
        P = C.c_void_p
        for nm in ("oracle_decode_f64", "oracle_decode_f32"):
            f = getattr(lib, nm)
            f.restype = C.c_int
            f.argtypes = [C.c_int, C.c_int, P, P, C.c_int, P, P, P, P, C.POINTER(_Params),
                          C.c_int64, C.c_int64, P, P, P, P, P, P, P, P, C.c_int]
        for nm in ("oracle_bp_f64", "oracle_bp_f32"):
            f = getattr(lib, nm)
            f.restype = C.c_int
            f.argtypes = [C.c_int, C.c_int, P, P, P, P, P, C.c_double, C.c_int, C.c_int, C.c_int,
                          C.c_double, P, P, P, P]
        lib.oracle_splitmix64.restype = C.c_uint64
        lib.oracle_splitmix64.argtypes = [C.c_uint64]
        lib.oracle_tie_hash.restype = C.c_uint64
        lib.oracle_tie_hash.argtypes = [C.c_uint64, C.c_uint64, C.c_uint64]
        _lib = lib
    return _lib


def _ptr(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def splitmix64(x: int) -> int:
    return int(_load().oracle_splitmix64(C.c_uint64(x & 0xFFFFFFFFFFFFFFFF)))


def tie_hash(seed: int, shot: int, row: int) -> int:
    return int(_load().oracle_tie_hash(C.c_uint64(seed), C.c_uint64(shot), C.c_uint64(row)))


def prior_llr(priors: np.ndarray, precision: str = "f64") -> np.ndarray:
    p = np.asarray(priors, dtype=np.float64)
    lam = np.log((1.0 - p) / p)
    return lam.astype(np.float32).astype(np.float64) if precision == "f32" else lam


def decode(code, syndromes: np.ndarray, params: OracleParams, precision: str = "f64",
           shot_offset: int = 0, weights: Optional[np.ndarray] = None, want_post: bool = True,
           want_post1: bool = False, threads: Optional[int] = None, D=None) -> dict:
    """BP+DC on every row of `syndromes` (uint8 [B, m]).

    Returns a dict with ehat (uint8 [B, n]), flags (uint8 [B]: bit 0 converged,
    bit 1 DC ran), iters (int32 [B, 2]), cut (uint8 [B, n]), margin (float64 [B])
    and, if requested, post / post1 (float64 [B, n]).
    """
    lib = _load()
    H = code.H
    Dm = code.D if D is None else D
    syn = np.ascontiguousarray(syndromes, dtype=np.uint8)
    B = syn.shape[0]
    assert syn.shape[1] == H.rows
    n = H.cols
    hrp, hci = np.ascontiguousarray(H.row_ptr, np.int32), np.ascontiguousarray(H.col_idx, np.int32)
    drp, dci = np.ascontiguousarray(Dm.row_ptr, np.int32), np.ascontiguousarray(Dm.col_idx, np.int32)
    pri = np.ascontiguousarray(code.priors, dtype=np.float64)
    w = None if weights is None else np.ascontiguousarray(weights, dtype=np.float64).reshape(-1)
    if w is not None:
        assert w.size == 2 * H.nnz
    out = {
        "ehat": np.zeros((B, n), np.uint8), "flags": np.zeros(B, np.uint8),
        "iters": np.zeros((B, 2), np.int32), "cut": np.zeros((B, n), np.uint8),
        "margin": np.zeros(B, np.float64),
    }
    post = np.zeros((B, n), np.float64) if want_post else None
    post1 = np.zeros((B, n), np.float64) if want_post1 else None
    prm = params.to_c()
    if threads is None:
        threads = os.cpu_count() or 1
    fn = lib.oracle_decode_f64 if precision == "f64" else lib.oracle_decode_f32
    rc = fn(H.rows, n, _ptr(hrp), _ptr(hci), Dm.rows, _ptr(drp), _ptr(dci), _ptr(pri), _ptr(w),
            C.byref(prm), B, shot_offset, _ptr(syn), _ptr(out["ehat"]), _ptr(post), _ptr(post1),
            _ptr(out["cut"]), _ptr(out["flags"]), _ptr(out["iters"]), _ptr(out["margin"]),
            int(threads))
    if rc != 0:
        raise ValueError(f"oracle rejected the problem (code {rc})")
    if want_post:
        out["post"] = post
    if want_post1:
        out["post1"] = post1
    return out


def bp_once(H, syndrome: np.ndarray, prior_llr_in: np.ndarray, T: int, rule: int = MIN_SUM,
            alpha: float = 1.0, lsat: float = float("inf"), stop_on_converge: bool = False,
            frozen: Optional[np.ndarray] = None, weights: Optional[np.ndarray] = None,
            precision: str = "f64"):
    """One BP_decode run; returns (ehat, posterior LLR, iterations, converged)."""
    lib = _load()
    hrp, hci = np.ascontiguousarray(H.row_ptr, np.int32), np.ascontiguousarray(H.col_idx, np.int32)
    lam = np.ascontiguousarray(prior_llr_in, dtype=np.float64)
    syn = np.ascontiguousarray(syndrome, dtype=np.uint8)
    fz = None if frozen is None else np.ascontiguousarray(frozen, dtype=np.uint8)
    w = None if weights is None else np.ascontiguousarray(weights, dtype=np.float64)
    ehat = np.zeros(H.cols, np.uint8)
    post = np.zeros(H.cols, np.float64)
    it = np.zeros(1, np.int32)
    fn = lib.oracle_bp_f64 if precision == "f64" else lib.oracle_bp_f32
    conv = fn(H.rows, H.cols, _ptr(hrp), _ptr(hci), _ptr(lam), _ptr(fz), _ptr(w), float(alpha),
              int(rule), int(T), 1 if stop_on_converge else 0, float(lsat), _ptr(syn), _ptr(ehat),
              _ptr(post), _ptr(it))
    return ehat, post, int(it[0]), bool(conv)
