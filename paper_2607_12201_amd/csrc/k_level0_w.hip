// Register-resident element and chain kernels instantiated for the thread grids (TS x TS / NB
// register blocks per side) 24x24/4, 24x24/5.
#include "level0_inst.h"

namespace cl {
CL_LEVEL0_INSTANCE(24, 4)
CL_LEVEL0_INSTANCE(24, 5)
}  // namespace cl
