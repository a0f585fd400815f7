"""CPU oracle for BP+DC decoding (test infrastructure only).

Only the tests, the smoke check and the benchmark's CPU-baseline leg use
this package.  It shares no code with the GPU library ``paper_2510_08695_amd``.
"""
from .oracle import (OracleParams, decode, bp_once, build, lib_path, splitmix64, tie_hash,
                     prior_llr, MIN_SUM, PRODUCT_SUM)

__all__ = ["OracleParams", "decode", "bp_once", "build", "lib_path", "splitmix64", "tie_hash",
           "prior_llr", "MIN_SUM", "PRODUCT_SUM"]
