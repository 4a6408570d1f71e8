"""MI355X-native fast compressed-sensing SAR imaging with an approximated
observation operator (chirp-scaling G = M^-1 and G^H = M) and iterative
soft thresholding.  The compute path is libcssar.so (HIP, gfx950); this
package is its Python binding."""

from .cssar import (Operator, make_operator, Batch, make_batch, ITAUnrolled, CssarError,
                    supported_length, plan_info, ka_of, params_with_theta, lib, LIB_PATH)

__all__ = ["Operator", "make_operator", "Batch", "make_batch", "ITAUnrolled", "CssarError",
           "supported_length", "plan_info", "ka_of", "params_with_theta", "lib", "LIB_PATH"]
