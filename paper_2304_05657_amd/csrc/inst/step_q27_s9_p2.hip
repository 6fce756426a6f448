// Explicit instantiation of the step and init kernels for D3Q27, 9 species, precision 2.
#include "../lbfd_kernels.h"

namespace lbfd {
LBFD_INSTANTIATE(27, 9, 2)
}
