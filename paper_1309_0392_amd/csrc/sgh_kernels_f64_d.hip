// Dehierarchization kernels for double grids (templates in sgh_kernels.inc).
#define SGH_KT double
#define SGH_OPC SGH_OP_DEHIERARCHIZE
#define SGH_SUFFIX f64_d
#include "sgh_kernels.inc"
