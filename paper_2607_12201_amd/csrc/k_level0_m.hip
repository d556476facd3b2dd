// Register-resident element and chain kernels instantiated for the thread grids (TS x TS / NB
// register blocks per side) 16x16/3, 16x16/4, 16x16/5, 16x16/6.
#include "level0_inst.h"

namespace cl {
CL_LEVEL0_INSTANCE(16, 3)
CL_LEVEL0_INSTANCE(16, 4)
CL_LEVEL0_INSTANCE(16, 5)
CL_LEVEL0_INSTANCE(16, 6)
}  // namespace cl
