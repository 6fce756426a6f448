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
// the first level whose check saw a non-finite value and, with acc, adds
// coef * out[slot] + shift to *acc.  (A 1024-thread block with wave
// butterflies measured slower: 13.6 against 7.9 us for 1024 partials.)
__global__ void __launch_bounds__(kBlock) finalize_kernel(const double *partials, int nblocks, double *out,
                                                          long long *first_bad, long long level, double *acc,
                                                          int slot, double coef, double shift)
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
        if (acc) *acc += coef * red[0][slot] + shift;
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

// When the inlet profile of x face `face` changes by -du (du = old - new,
// [3][nz][ny]), the stored outgoing population g*_opp of each fluid cell
// next to that face is shifted by 2 w_i rho_in c_i.du for every direction i
// entering through the face: those values are read only by the inlet rule
// of the same cell (they stream out of the box), so the populations
// entering at the current level keep the values the old profile gave them,
// and the new profile applies from the next streaming on.
template <int Q, int PREC>
__global__ void __launch_bounds__(kBlock) inflow_shift_kernel(const KParams P, int face, const double *du)
{
    using L = Lat<Q>;
    using C = typename Prec<PREC>::calc;
    const long long nf = (long long)P.ny * P.nz;
    const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= nf) return;
    const int y = (int)(t % P.ny), z = (int)(t / P.ny);
    const int x = face ? P.nx - 1 : 0, cin = face ? -1 : 1;
    const long long idx = ((long long)z * P.ny + y) * P.nx + x;
    if (P.mask[idx] != LBFD_FLUID) return;
    sfor<0, Q>([&](auto I) {
        constexpr int i = decltype(I)::value;
        constexpr int opp = Q - 1 - i;
        if constexpr (L::cx(i) != 0) {
            if (L::cx(i) == cin) {
                const Nb s = classify(P, x - L::cx(i), y - L::cy(i), z - L::cz(i));
                if (s.kind == kInflow && s.face == face) {
                    const double cdu = L::cx(i) * du[t] + L::cy(i) * du[nf + t] + L::cz(i) * du[2 * nf + t];
                    const C v = pop_load<Q, PREC, opp>(P.pop_in, P.N, idx) + (C)(2.0 * L::w(i) * P.rho_in * cdu);
                    pop_store<Q, PREC, opp>(P.pop_out, P.N, idx, v);
                }
            }
        }
    });
}

hipError_t launch_inflow_shift(int Q, int prec, const KParams &kp, int face, const double *du, hipStream_t s)
{
    const unsigned nb = (unsigned)(((long long)kp.ny * kp.nz + kBlock - 1) / kBlock);
#define SHIFT(q, p)                                                                        \
    if (Q == q && prec == p) {                                                             \
        inflow_shift_kernel<q, p><<<dim3(nb), dim3(kBlock), 0, s>>>(kp, face, du);         \
        return hipGetLastError();                                                          \
    }
    SHIFT(9, 0) SHIFT(9, 1) SHIFT(9, 2) SHIFT(27, 0) SHIFT(27, 1) SHIFT(27, 2)
#undef SHIFT
    return hipErrorInvalidValue;
}

hipError_t launch_finalize(const double *partials, int nblocks, double *out, long long *first_bad,
                           long long level, hipStream_t s, double *acc, int slot, double a, double b)
{
    finalize_kernel<<<1, kBlock, 0, s>>>(partials, nblocks, out, first_bad, level, acc, slot, a, b);
    return hipGetLastError();
}

// Widening copy of single-precision scalars into caller double buffers.
__global__ void __launch_bounds__(kBlock) widen_kernel(const float *src, double *dst, size_t n)
{
    const size_t i = (size_t)blockIdx.x * kBlock + threadIdx.x;
    if (i < n) dst[i] = (double)src[i];
}

hipError_t launch_widen(const float *src, double *dst, size_t n, hipStream_t s)
{
    if (n == 0) return hipSuccess;
    widen_kernel<<<dim3((unsigned)((n + kBlock - 1) / kBlock)), dim3(kBlock), 0, s>>>(src, dst, n);
    return hipGetLastError();
}

}  // namespace lbfd
