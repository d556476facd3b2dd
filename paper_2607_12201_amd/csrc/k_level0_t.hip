// Register-resident element and chain kernels instantiated for the thread grids (TS x TS / NB
// register blocks per side) 16x16/1, 16x16/2, 24x24/2, 24x24/3.
#include "level0_inst.h"

namespace cl {
CL_LEVEL0_INSTANCE(16, 1)
CL_LEVEL0_INSTANCE(16, 2)
CL_LEVEL0_INSTANCE(24, 2)
CL_LEVEL0_INSTANCE(24, 3)
}  // namespace cl
