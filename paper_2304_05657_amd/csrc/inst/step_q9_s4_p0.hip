// Explicit instantiation of the step and init kernels for D2Q9, 4 species, precision 0.
#include "../lbfd_kernels.h"

namespace lbfd {
LBFD_INSTANTIATE(9, 4, 0)
}
