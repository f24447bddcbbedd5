"""MI355X-native Gamma-only LTMP2: the HIP library libltmp2 and its binding."""
from .ltmp2 import (Batch, Context, LTMP2Error, quadrature, supported_grids, load, LIB_PATH,
                    FP64, FP32, BF16X3, QUAD_PLAIN, QUAD_LEARNED, QUAD_GIVEN, quadrature_table,
                    mlp_init, mlp_dataset, mlp_forward, mlp_grad, mlp_train, learned_quadrature,
                    write_mlp_weights, read_mlp_weights, MLP_NPARAM)

__all__ = ["Batch", "Context", "LTMP2Error", "quadrature", "supported_grids", "load", "LIB_PATH",
           "FP64", "FP32", "BF16X3", "QUAD_PLAIN", "QUAD_LEARNED", "QUAD_GIVEN",
           "quadrature_table", "mlp_init", "mlp_dataset", "mlp_forward", "mlp_grad", "mlp_train",
           "learned_quadrature", "write_mlp_weights", "read_mlp_weights", "MLP_NPARAM"]
