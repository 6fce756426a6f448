// Explicit instantiation of the step and init kernels for D2Q9, 9 species, precision 1.
#include "../lbfd_kernels.h"

namespace lbfd {
LBFD_INSTANTIATE(9, 9, 1)
}
