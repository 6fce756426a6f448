// Explicit instantiation of the step and init kernels for D2Q9, 4 species, precision 2.
#include "../lbfd_kernels.h"

namespace lbfd {
LBFD_INSTANTIATE(9, 4, 2)
}
