"""Shared helpers of the GPU parity tests: run the HIP library and the oracle on
the same seeded shots and compare them."""
from __future__ import annotations

import numpy as np

import oracle
import synth


def oracle_params(prm, second_pass: str) -> oracle.OracleParams:
    """Oracle parameters equal to library parameters `prm` (paper_2510_08695_amd.Params)."""
    return oracle.OracleParams(max_iter1=prm.max_iter[0], max_iter2=prm.max_iter[1], alpha=prm.alpha,
                               second_pass_prior=second_pass, stop_on_converge=prm.stop_on_converge,
                               llr_sat=prm.llr_sat, tie_eps=prm.tie_eps,
                               tie_break="lowest" if prm.tie_break == 1 else "hash", seed=prm.seed,
                               rule=getattr(prm, "rule", 0), soft_period=getattr(prm, "soft_period", 0),
                               soft_shift=float(np.float32(getattr(prm, "soft_shift", 0.0))))


def gpu_decode(plan, code, syndromes: np.ndarray, code_index: int = 0, shot_offset: int = 0,
               want_post: bool = True) -> dict:
    """Decode uint8 syndromes [B, m] with `plan`; returns unpacked numpy outputs."""
    import torch
    syn = torch.from_numpy(synth.pack_bits(syndromes).view(np.int64)).cuda()
    out = plan.decode(syn, code=code_index, shot_offset=shot_offset, want_post=want_post,
                      want_cut=True, want_iters=True)
    torch.cuda.synchronize()
    n = code.n
    res = {
        "ehat": synth.unpack_bits(out["corr"].cpu().numpy().view(np.uint64), n),
        "cut": synth.unpack_bits(out["cut"].cpu().numpy().view(np.uint64), n),
        "flags": out["flags"].cpu().numpy(),
        "iters": out["iters"].cpu().numpy().astype(np.int32),
        "corr_words": out["corr"].cpu().numpy().view(np.uint64),
        "cut_words": out["cut"].cpu().numpy().view(np.uint64),
    }
    if want_post:
        res["post"] = out["post"].cpu().numpy()
    return res


def assert_bit_exact(gpu: dict, ref: dict, n: int, check_post: bool = True):
    """GPU (float32) against the float32 oracle: every output identical."""
    np.testing.assert_array_equal(gpu["flags"], ref["flags"])
    np.testing.assert_array_equal(gpu["iters"], ref["iters"])
    np.testing.assert_array_equal(gpu["ehat"], ref["ehat"])
    np.testing.assert_array_equal(gpu["cut"], ref["cut"])
    # padding bits of packed outputs are zero
    nw = (n + 63) // 64
    if n % 64:
        pad = ~np.uint64((1 << (n % 64)) - 1)
        assert not (gpu["corr_words"][:, nw - 1] & pad).any()
        assert not (gpu["cut_words"][:, nw - 1] & pad).any()
    if check_post:
        a = gpu["post"].astype(np.float32)
        b = ref["post"].astype(np.float32)
        np.testing.assert_array_equal(a.view(np.uint32), b.view(np.uint32))


def ler(code, errors: np.ndarray, out: dict) -> float:
    conv = (out["flags"] & 1) != 0
    fail = ~conv | synth.residual_is_logical(errors ^ out["ehat"], code.O)
    return float(fail.mean())
