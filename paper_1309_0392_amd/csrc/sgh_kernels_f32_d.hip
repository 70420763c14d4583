// Dehierarchization kernels for float grids (templates in sgh_kernels.inc).
#define SGH_KT float
#define SGH_OPC SGH_OP_DEHIERARCHIZE
#define SGH_SUFFIX f32_d
#include "sgh_kernels.inc"
