"""MI355X-native Gamma-only LTMP2: the HIP library libltmp2 and its binding."""
from .ltmp2 import (Context, LTMP2Error, quadrature, supported_grids, load, LIB_PATH,
                    FP64, FP32, BF16X3, QUAD_PLAIN, QUAD_LEARNED, QUAD_GIVEN)

__all__ = ["Context", "LTMP2Error", "quadrature", "supported_grids", "load", "LIB_PATH",
           "FP64", "FP32", "BF16X3", "QUAD_PLAIN", "QUAD_LEARNED", "QUAD_GIVEN"]
