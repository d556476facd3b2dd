// Register-resident element and chain kernels instantiated for the thread grids (TS x TS / NB
// register blocks per side) 20x20/5, 20x20/6, 20x20/7, 20x20/8.
#include "level0_inst.h"

namespace cl {
CL_LEVEL0_INSTANCE(20, 5)
CL_LEVEL0_INSTANCE(20, 6)
CL_LEVEL0_INSTANCE(20, 7)
CL_LEVEL0_INSTANCE(20, 8)
}  // namespace cl
