// Register-resident element and chain kernels instantiated for the thread grids (TS x TS / NB
// register blocks per side) 8x8/1, 8x8/2, 8x8/3, 8x8/4.
#include "level0_inst.h"

namespace cl {
CL_LEVEL0_INSTANCE(8, 1)
CL_LEVEL0_INSTANCE(8, 2)
CL_LEVEL0_INSTANCE(8, 3)
CL_LEVEL0_INSTANCE(8, 4)
}  // namespace cl
