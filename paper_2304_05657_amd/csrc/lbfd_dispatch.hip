// lbfd_dispatch.hip -- configuration dispatch and the final reduction of
// the diagnostics (the step kernels are instantiated in inst/*.hip).
#include "lbfd_kernels.h"

namespace lbfd {

#define X(q, n, p) \
    extern template hipError_t launch_step_t<q, n, p>(int, const KParams &, const Streams &); \
    extern template hipError_t launch_init_t<q, n, p>(const KParams &, const double *, const double *, dim3, \
                                                      dim3, hipStream_t);
LBFD_FOR_CONFIGS(X)
#undef X

// Deterministic final reduction of the block partials (one block); records
// the first level whose check saw a non-finite value.
__global__ void __launch_bounds__(kBlock) finalize_kernel(const double *partials, int nblocks, double *out,
                                                          long long *first_bad, long long level)
{
    __shared__ double red[kBlock][kNDiag];
    double a[kNDiag];
    diag_identity(a);
    for (int b = threadIdx.x; b < nblocks; b += blockDim.x) diag_combine(a, partials + (long long)b * kNDiag);
#pragma unroll
    for (int s = 0; s < kNDiag; ++s) red[threadIdx.x][s] = a[s];
    __syncthreads();
    for (int stride = blockDim.x / 2; stride >= 1; stride >>= 1) {
        if ((int)threadIdx.x < stride) {
#pragma unroll
            for (int s = 0; s < kNDiag; ++s) a[s] = red[threadIdx.x][s];
            diag_combine(a, red[threadIdx.x + stride]);
#pragma unroll
            for (int s = 0; s < kNDiag; ++s) red[threadIdx.x][s] = a[s];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
#pragma unroll
        for (int s = 0; s < kNDiag; ++s) out[s] = red[0][s];
        if (first_bad && red[0][kNonfinite] > 0.0 && *first_bad < 0) *first_bad = level;
    }
}

bool supported(int Q, int nsp, int prec)
{
#define X(q, n, p) if (Q == q && nsp == n && prec == p) return true;
    LBFD_FOR_CONFIGS(X)
#undef X
    return false;
}

hipError_t launch_step(int Q, int nsp, int prec, int mode, const KParams &kp, const Streams &s)
{
#define X(q, n, p) if (Q == q && nsp == n && prec == p) return launch_step_t<q, n, p>(mode, kp, s);
    LBFD_FOR_CONFIGS(X)
#undef X
    return hipErrorInvalidValue;
}

hipError_t launch_init(int Q, int nsp, int prec, const KParams &kp, const double *u0, const double *Ph0,
                       dim3 grid, dim3 block, hipStream_t s)
{
#define X(q, n, p) if (Q == q && nsp == n && prec == p) return launch_init_t<q, n, p>(kp, u0, Ph0, grid, block, s);
    LBFD_FOR_CONFIGS(X)
#undef X
    return hipErrorInvalidValue;
}

hipError_t launch_finalize(const double *partials, int nblocks, double *out, long long *first_bad,
                           long long level, hipStream_t s)
{
    finalize_kernel<<<1, kBlock, 0, s>>>(partials, nblocks, out, first_bad, level);
    return hipGetLastError();
}

}  // namespace lbfd
