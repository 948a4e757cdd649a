// One-lane FP32 stage kernels of orders p = 2, 3 (templates in dg_kernels.h).
// The build compiles this file alone with the max-memory-clause scheduler.
#define DG_DEFINE_STAGE1_F32
#include "dg_kernels.h"

namespace dgk {
DG_STAGE1_F32_ORDER(2)
DG_STAGE1_F32_ORDER(3)
}  // namespace dgk
