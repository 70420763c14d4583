// Hierarchization kernels for float grids (templates in sgh_kernels.inc).
#define SGH_KT float
#define SGH_OPC SGH_OP_HIERARCHIZE
#define SGH_SUFFIX f32_h
#define SGH_DEFINE_COMBI 1
#define SGH_KTNAME f32
#include "sgh_kernels.inc"
