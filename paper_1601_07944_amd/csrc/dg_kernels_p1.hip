// Kernels of order p = 1 (templates in dg_kernels.h), including the one-lane
// FP32 stage kernels, which are faster here with the default scheduler.
#define DG_DEFINE_STAGE1_F32
#include "dg_kernels.h"

namespace dgk {
template struct Launch<1>;
DG_STAGE1_F32_ORDER(1)
}
