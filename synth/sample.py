"""Seeded i.i.d. error sampling, syndromes and bit packing.

Errors are Bernoulli(p_j) per column j drawn from numpy's PCG64 generator
(seeded; drawn in chunks of rows so that the stream does not depend on the
chunk size); the syndrome of error e is s = e H^T over F2 (Sec. II.C).
Bit j of a packed vector is bit (j & 63) of 64-bit word (j >> 6).
"""
from __future__ import annotations

from dataclasses import dataclass
from typing import Optional

import numpy as np

CHUNK = 1 << 16


def sample_errors(rng: np.random.Generator, shots: int, priors: np.ndarray) -> np.ndarray:
    pri = np.asarray(priors, dtype=np.float64)
    out = np.empty((shots, len(pri)), dtype=np.uint8)
    for s0 in range(0, shots, CHUNK):
        s1 = min(shots, s0 + CHUNK)
        out[s0:s1] = rng.random((s1 - s0, len(pri))) < pri
    return out


def syndromes_of(errors: np.ndarray, H) -> np.ndarray:
    """s = e H^T mod 2 for every row of `errors` (uint8 [B, n]) -> uint8 [B, m]."""
    Hs = H.to_sparse().astype(np.int32).tocsr()
    out = np.empty((errors.shape[0], H.rows), dtype=np.uint8)
    for s0 in range(0, errors.shape[0], CHUNK):
        e = errors[s0:s0 + CHUNK].astype(np.int32)
        out[s0:s0 + CHUNK] = ((Hs @ e.T).T & 1).astype(np.uint8)
    return out


def pack_bits(bits: np.ndarray) -> np.ndarray:
    """uint8 0/1 [B, k] -> uint64 [B, ceil(k/64)] (little-endian bit order)."""
    bits = np.asarray(bits, dtype=np.uint8)
    B, k = bits.shape
    nw = (k + 63) // 64
    pad = np.zeros((B, nw * 64), dtype=np.uint8)
    pad[:, :k] = bits
    return np.packbits(pad, axis=1, bitorder="little").view("<u8").reshape(B, nw).copy()


def unpack_bits(words: np.ndarray, k: int) -> np.ndarray:
    """uint64 [B, nw] -> uint8 0/1 [B, k]."""
    w = np.ascontiguousarray(words, dtype="<u8")
    b = np.unpackbits(w.view(np.uint8).reshape(w.shape[0], -1), axis=1, bitorder="little")
    return b[:, :k].astype(np.uint8)


@dataclass
class ShotSet:
    errors: np.ndarray              # uint8 [B, n]
    syndromes: np.ndarray           # uint8 [B, m]
    seed: int

    @property
    def syn_packed(self) -> np.ndarray:
        return pack_bits(self.syndromes)

    def __len__(self):
        return self.syndromes.shape[0]


def make_shots(code, shots: int, seed: int, priors: Optional[np.ndarray] = None) -> ShotSet:
    rng = np.random.default_rng(seed)
    e = sample_errors(rng, shots, code.priors if priors is None else priors)
    return ShotSet(e, syndromes_of(e, code.H), seed)


def mixed_batch(codes, mean_shots: float, seed: int, shot_seed_base: int):
    """A batch of shots over several codes in a seeded random global order.

    Code i gets Poisson(mean_shots) shots (counts drawn from a generator seeded
    with `seed`, which then shuffles the batch order); its shots are drawn with
    seed shot_seed_base + i.  Returns (code_of_shot int32 [B], packed syndromes
    as int64 words concatenated in batch order, per-code list of
    (batch indices, ShotSet))."""
    rng = np.random.default_rng(seed)
    counts = rng.poisson(mean_shots, size=len(codes))
    code_of_shot = np.concatenate([np.full(k, i, np.int32) for i, k in enumerate(counts)])
    rng.shuffle(code_of_shot)
    rows = [None] * len(code_of_shot)
    per = []
    for i, c in enumerate(codes):
        idx = np.nonzero(code_of_shot == i)[0]
        sh = make_shots(c, len(idx), shot_seed_base + i)
        per.append((idx, sh))
        packed = pack_bits(sh.syndromes)
        for k, b in enumerate(idx):
            rows[b] = packed[k]
    syn = np.concatenate(rows).view(np.int64) if rows else np.zeros(0, np.int64)
    return code_of_shot, syn, per
