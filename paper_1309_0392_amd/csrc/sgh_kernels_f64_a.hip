// Transposed hierarchization kernels for double grids (templates in sgh_kernels.inc).
#define SGH_KT double
#define SGH_OPC SGH_OP_ADJOINT
#define SGH_SUFFIX f64_a
#include "sgh_kernels.inc"
