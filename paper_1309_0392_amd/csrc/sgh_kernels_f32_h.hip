// Hierarchization kernels for float grids (templates in sgh_kernels.inc).
#define SGH_KT float
#define SGH_OPC SGH_OP_HIERARCHIZE
#define SGH_SUFFIX f32_h
#include "sgh_kernels.inc"
