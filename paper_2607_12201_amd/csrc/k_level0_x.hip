// Register-resident element and chain kernels instantiated for the thread grids (TS x TS / NB
// register blocks per side) 24x24/6, 24x24/7.
#include "level0_inst.h"

namespace cl {
CL_LEVEL0_INSTANCE(24, 6)
CL_LEVEL0_INSTANCE(24, 7)
}  // namespace cl
