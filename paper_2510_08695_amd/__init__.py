"""MI355X (gfx950) BP+DC decoding: min-sum / product-sum belief propagation + degeneracy cutting.

Thin Python binding of ``libbpdc.so`` (the C ABI in ``include/bpdc.h``).  The
decoder itself runs in the library's HIP kernels; this package only marshals
arguments, with torch tensors supplying device memory and the current stream.
Importing it does not load the library; the first use does, and raises if
the library has not been built.
"""
from ._lib import (BpdcError, Params, Code, Plan, lib, lib_path, lane_precompile, weighted_bpdc, eval_phi,
                   KERNEL_AUTO, KERNEL_PLAIN, KERNEL_LANE, KERNEL_GROUP,
                   PRIOR_CHANNEL, PRIOR_POSTERIOR, TIE_HASH, TIE_LOWEST_INDEX, RULE_MIN_SUM, RULE_PRODUCT_SUM, FLAG_BAD_CODE)

__all__ = ["BpdcError", "Params", "Code", "Plan", "lib", "lib_path", "lane_precompile", "weighted_bpdc", "eval_phi",
           "KERNEL_AUTO", "KERNEL_PLAIN", "KERNEL_LANE", "KERNEL_GROUP",
           "PRIOR_CHANNEL", "PRIOR_POSTERIOR", "TIE_HASH", "TIE_LOWEST_INDEX", "RULE_MIN_SUM", "RULE_PRODUCT_SUM",
           "FLAG_BAD_CODE"]
