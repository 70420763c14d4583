// Hierarchization kernels for double grids (templates in sgh_kernels.inc).
#define SGH_KT double
#define SGH_OPC SGH_OP_HIERARCHIZE
#define SGH_SUFFIX f64_h
#define SGH_DEFINE_COMMON 1
#define SGH_DEFINE_COMBI 1
#define SGH_KTNAME f64
#include "sgh_kernels.inc"
