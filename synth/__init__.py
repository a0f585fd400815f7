"""Seeded synthetic inputs shared by the oracle and the GPU decoder.

This package builds the parity-check matrices of the codes the decoder is
run on (toric, rotated surface, bivariate bicycle, hypergraph product, phenomenological
and circuit-level detector error models) and draws seeded i.i.d. error patterns and their
syndromes.  It contains none of the decoder's arithmetic: no message
passing, no degeneracy cutting.  Both the CPU oracle (``oracle/``) and the
HIP library (``paper_2510_08695_amd``) consume what it produces, and neither
of them is imported here.
"""
from .codes import (Csr, Code, toric_code, bb_code, hgp_code, random_regular_classical,
                    phenomenological_dem, hgp_batch_codes, repetition_cycle, rotated_surface_code,
                    rotated_surface_matrices)
from .sample import (sample_errors, syndromes_of, pack_bits, unpack_bits, ShotSet, make_shots, mixed_batch)
from .f2 import f2_rank, logical_operators, residual_is_logical
from .circuit import bb_circuit_dem, bb_circuit_matrices, bb_circuit_mechanisms

__all__ = [
    "Csr", "Code", "toric_code", "bb_code", "hgp_code", "random_regular_classical",
    "phenomenological_dem", "hgp_batch_codes", "repetition_cycle", "rotated_surface_code",
    "rotated_surface_matrices",
    "sample_errors", "syndromes_of", "pack_bits", "unpack_bits", "ShotSet", "make_shots", "mixed_batch",
    "f2_rank", "logical_operators", "residual_is_logical",
    "bb_circuit_dem", "bb_circuit_matrices", "bb_circuit_mechanisms",
]
