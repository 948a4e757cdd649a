// Kernels of order p = 5 (templates in dg_kernels.h).
#include "dg_kernels.h"

namespace dgk {
template struct Launch<5>;
}
