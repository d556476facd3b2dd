// Register-resident element and chain kernels instantiated for the thread grids (TS x TS / NB
// register blocks per side) 16x16/7, 16x16/8.
#include "level0_inst.h"

namespace cl {
CL_LEVEL0_INSTANCE(16, 7)
CL_LEVEL0_INSTANCE(16, 8)
}  // namespace cl
