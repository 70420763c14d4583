// Transposed hierarchization kernels for float grids (templates in sgh_kernels.inc).
#define SGH_KT float
#define SGH_OPC SGH_OP_ADJOINT
#define SGH_SUFFIX f32_a
#include "sgh_kernels.inc"
