#pragma once
// lbfd_kernels.h -- templates of the fused coupled step for gfx950: pull-scheme lattice-Boltzmann streaming
// with boundary conditions, finite-difference advection-diffusion-reaction
// of T and Y_k with ghost nodes, source Xi, central-moment collision, and
// explicit Euler update -- one thread per cell, one kernel per step.
//
// Method: Hosseini & Thevenin, arXiv:2304.05657, Secs. II-III.  The step
// order (all terms at level n) and the readings of the paper's silent or
// garbled passages are those stated in include/lbfd.h and the design notes.
//
// Storage (structure of arrays, x fastest):
//   populations  pop[i][cell]   post-collision values g*_i of the previous
//                               level; FP64: g itself, mixed: g/(w_i cs^2)
//   scalars      sc[0][cell] = T, sc[1+k][cell] = Y_k
//   outlet       post-streaming values of the populations that enter
//                through an outflow face, per face cell (double)
#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>

#include "lbfd_internal.h"
#include "lbfd_math.h"

#include <type_traits>

namespace lbfd {

constexpr double kCs2 = 1.0 / 3.0;

// ---------------------------------------------------------------- lattice
template <int Q>
struct Lat {
    static constexpr int D = (Q == 9) ? 2 : 3;
    __host__ __device__ static constexpr int cx(int i) { return i % 3 - 1; }
    __host__ __device__ static constexpr int cy(int i) { return (i / 3) % 3 - 1; }
    __host__ __device__ static constexpr int cz(int i) { return Q == 9 ? 0 : i / 9 - 1; }
    __host__ __device__ static constexpr int c(int i, int d) { return d == 0 ? cx(i) : d == 1 ? cy(i) : cz(i); }
    __host__ __device__ static constexpr double w(int i)
    {
        // textbook weights by |c|^2
        return Q == 9 ? (cx(i) * cx(i) + cy(i) * cy(i) == 0   ? 4.0 / 9.0
                         : cx(i) * cx(i) + cy(i) * cy(i) == 1 ? 1.0 / 9.0
                                                              : 1.0 / 36.0)
                      : (cx(i) * cx(i) + cy(i) * cy(i) + cz(i) * cz(i) == 0   ? 8.0 / 27.0
                         : cx(i) * cx(i) + cy(i) * cy(i) + cz(i) * cz(i) == 1 ? 2.0 / 27.0
                         : cx(i) * cx(i) + cy(i) * cy(i) + cz(i) * cz(i) == 2 ? 1.0 / 54.0
                                                                              : 1.0 / 216.0);
    }
};

// ------------------------------------------------------------- precision
template <int PREC> struct Prec;
template <> struct Prec<LBFD_FP64> { using calc = double; using pop = double; using scal = double; };
template <> struct Prec<LBFD_MIXED_FP32> { using calc = float; using pop = float; using scal = float; };
template <> struct Prec<LBFD_MIXED_FP16> { using calc = float; using pop = __half; using scal = float; };

// Loads and stores at a 32-bit byte offset from a uniform base pointer
// (base in scalar registers, one 32-bit offset register per access; every
// buffer is below 4 GiB, checked at init).
template <class T>
__device__ __forceinline__ T ldo(const void *base, uint32_t byte_off)
{
    return *(const T *)((const char *)base + byte_off);
}
template <class T>
__device__ __forceinline__ void sto(void *base, uint32_t byte_off, T v)
{
    *(T *)((char *)base + byte_off) = v;
}

// Populations: FP64 stores g; mixed stores g / (w_i cs^2) (deviation from
// the lattice weights, scaled to comparable magnitude across directions).
template <int Q, int PREC, int I>
__device__ __forceinline__ typename Prec<PREC>::calc pop_load(const void *base, long long N, uint32_t idx)
{
    using T = typename Prec<PREC>::pop;
    const char *b = (const char *)base + (size_t)I * (size_t)N * sizeof(T);
    const uint32_t off = idx * (uint32_t)sizeof(T);
    if constexpr (PREC == LBFD_FP64) {
        return ldo<double>(b, off);
    } else if constexpr (PREC == LBFD_MIXED_FP32) {
        constexpr float s = (float)(Lat<Q>::w(I) * kCs2);
        return ldo<float>(b, off) * s;
    } else {
        constexpr float s = (float)(Lat<Q>::w(I) * kCs2);
        return __half2float(ldo<__half>(b, off)) * s;
    }
}

template <int Q, int PREC, int I>
__device__ __forceinline__ void pop_store(void *base, long long N, uint32_t idx, typename Prec<PREC>::calc v)
{
    using T = typename Prec<PREC>::pop;
    char *b = (char *)base + (size_t)I * (size_t)N * sizeof(T);
    const uint32_t off = idx * (uint32_t)sizeof(T);
    if constexpr (PREC == LBFD_FP64) {
        sto<double>(b, off, v);
    } else if constexpr (PREC == LBFD_MIXED_FP32) {
        constexpr float s = (float)(1.0 / (Lat<Q>::w(I) * kCs2));
        sto<float>(b, off, v * s);
    } else {
        constexpr float s = (float)(1.0 / (Lat<Q>::w(I) * kCs2));
        sto<__half>(b, off, __float2half_rn(v * s));
    }
}

// compile-time loop
template <int B, int E, class F>
__device__ __forceinline__ void sfor(F &&f)
{
    if constexpr (B < E) {
        f(std::integral_constant<int, B>{});
        sfor<B + 1, E>(f);
    }
}

// ------------------------------------------------------------- geometry
struct Nb {
    int kind;
    int face;
    long long idx;
    double Tw;
};

__device__ __forceinline__ int wrapc(int v, int n)
{
    if ((unsigned)v < (unsigned)n) return v;
    int r = v % n;
    return r < 0 ? r + n : r;
}

// What sits at (x, y, z): periodic faces wrap; outside any other face the
// point is that face (walls before inflow before outflow, lower axis and
// face first); inside, the mask decides.
__device__ __forceinline__ Nb classify(const KParams &P, int x, int y, int z)
{
    int q[3] = {x, y, z};
    const int n[3] = {P.nx, P.ny, P.nz};
    int best_face = -1, best_rank = 99;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        if ((unsigned)q[d] >= (unsigned)n[d]) {
            int f = 2 * d + (q[d] >= n[d] ? 1 : 0);
            int kind = P.face[f];
            if (kind == LBFD_FACE_PERIODIC) {
                q[d] = wrapc(q[d], n[d]);
            } else {
                int rank = (kind == LBFD_FACE_WALL || kind == LBFD_FACE_WALL_ADIABATIC) ? 0
                         : kind == LBFD_FACE_INFLOW ? 1 : 2;
                if (rank < best_rank) {
                    best_rank = rank;
                    best_face = f;
                }
            }
        }
    }
    Nb r;
    r.idx = 0;
    r.Tw = 0.0;
    r.face = best_face;
    if (best_face >= 0) {
        int kind = P.face[best_face];
        r.kind = kind == LBFD_FACE_WALL ? kIso : kind == LBFD_FACE_WALL_ADIABATIC ? kAdia
               : kind == LBFD_FACE_INFLOW ? kInflow : kOutflow;
        r.Tw = P.face_T[best_face];
        return r;
    }
    r.idx = ((long long)q[2] * P.ny + q[1]) * P.nx + q[0];
    uint8_t m = P.mask[r.idx];
    r.kind = m == LBFD_FLUID ? kFluid : m == LBFD_SOLID_ISOTHERMAL ? kIso : kAdia;
    if (r.kind == kIso) r.Tw = P.wall_T[r.idx];
    return r;
}

__device__ __forceinline__ long long outlet_index(const KParams &P, int face, int i, int Q, int y, int z)
{
    return ((long long)((face & 1) * Q + i) * P.nz + z) * P.ny + y;
}

// c_I . u_in for population I of fluid cell (x, y, z) entering through an
// inflow face (Eq. 31): an x face carries a per-cell inlet profile, indexed
// by the entering cell's (y, z); other faces the uniform inflow velocity.
// (A source beyond an x inflow face and another non-periodic face is the
// wall's, or the x face's: walls rank first, then the lower axis.)
__device__ __forceinline__ double inflow_cu_c(const KParams &P, int cx, int cy, int cz, int x, int y, int z)
{
    const int f = (cx == 1 && x == 0 && P.face[0] == LBFD_FACE_INFLOW)               ? 0
                  : (cx == -1 && x == P.nx - 1 && P.face[1] == LBFD_FACE_INFLOW) ? 1
                                                                                 : -1;
    if (f >= 0) {
        const long long s = (long long)P.ny * P.nz;
        const double *u = P.inflow_u + 3 * s * f + (long long)z * P.ny + y;
        return cx * u[0] + cy * u[s] + cz * u[2 * s];
    }
    return cx * P.u_in[0] + cy * P.u_in[1] + cz * P.u_in[2];
}

template <int Q, int I>
__device__ __forceinline__ double inflow_cu(const KParams &P, int x, int y, int z)
{
    using L = Lat<Q>;
    return inflow_cu_c(P, L::cx(I), L::cy(I), L::cz(I), x, y, z);
}

// Post-streaming population i of fluid cell (x, y, z) at the current level
// from the post-collision buffer: pull from r - c_i; half-way bounce-back
// from a solid or wall; velocity inlet (Eq. 31 in g units:
// g*_opp + 2 w_i rho_in c_i.u_in); outlet value kept in the outlet buffer.
template <int Q, int PREC, int I>
__device__ __forceinline__ typename Prec<PREC>::calc gather(const KParams &P, int x, int y, int z, long long idx)
{
    using C = typename Prec<PREC>::calc;
    using L = Lat<Q>;
    constexpr int OPP = Q - 1 - I;
    if constexpr (I == (Q - 1) / 2) {
        return pop_load<Q, PREC, I>(P.pop_in, P.N, idx);  // rest population
    } else {
        Nb s = classify(P, x - L::cx(I), y - L::cy(I), z - L::cz(I));
        if (s.kind == kFluid) return pop_load<Q, PREC, I>(P.pop_in, P.N, s.idx);
        if (s.kind == kInflow) {
            const double cu = inflow_cu<Q, I>(P, x, y, z);
            return pop_load<Q, PREC, OPP>(P.pop_in, P.N, idx) + (C)(2.0 * L::w(I) * P.rho_in * cu);
        }
        if (s.kind == kOutflow) {
            int sign = (s.face & 1) ? 1 : -1;
            Nb in = classify(P, x - sign, y, z);
            if (in.kind == kFluid) return (C)P.outlet[outlet_index(P, s.face, I, Q, y, z)];
        }
        return pop_load<Q, PREC, OPP>(P.pop_in, P.N, idx);
    }
}

// ------------------------------------------------------------ scalars
template <int NSP, class C>
struct Pt {
    C T, rho;
    C Y[NSP];
};

template <int NSP, class C>
__device__ __forceinline__ C density(const KParams &P, C T, const C *Y)
{
    C s = 0;
#pragma unroll
    for (int k = 0; k < NSP; ++k) s += Y[k] * (C)P.invW[k];
    return (C)P.T_ref_over_W_ref * rcp(T * s);
}

template <int NSP, int PREC>
__device__ __forceinline__ void load_point(const KParams &P, long long idx, Pt<NSP, typename Prec<PREC>::calc> &o)
{
    using S = typename Prec<PREC>::scal;
    const char *sc = (const char *)P.sc_in;
    const size_t fstride = (size_t)P.N * sizeof(S);
    const uint32_t off = (uint32_t)idx * (uint32_t)sizeof(S);
    o.T = ldo<S>(sc, off);
#pragma unroll
    for (int k = 0; k < NSP; ++k) o.Y[k] = ldo<S>(sc + (size_t)(1 + k) * fstride, off);
    o.rho = density<NSP>(P, o.T, o.Y);
}

// Ghost value across the wall `w` from the image point (Sec. III.B):
// Dirichlet 2 phi_B - phi(I) for T at isothermal walls and for T, Y at the
// inlet; Neumann phi(I) otherwise (walls are impermeable); the density
// ghost is reconstructed directly from its wall value.
template <int NSP, class C>
__device__ __forceinline__ void ghost(const KParams &P, const Nb &w, const Pt<NSP, C> &img, Pt<NSP, C> &o)
{
    // selects rather than branches: every field of o is written once
    const bool iso = w.kind == kIso, inf = w.kind == kInflow;
    const C Tw = (C)w.Tw;
    C rho_b = (C)P.rho_in;
    if (iso) rho_b = density<NSP>(P, Tw, img.Y);
    o.T = iso ? (C)2 * Tw - img.T : inf ? (C)2 * (C)P.T_in - img.T : img.T;
#pragma unroll
    for (int k = 0; k < NSP; ++k) o.Y[k] = inf ? (C)2 * (C)P.Y_in[k] - img.Y[k] : img.Y[k];
    o.rho = iso || inf ? (C)2 * rho_b - img.rho : img.rho;
}

// Population I or its opposite (same lattice weight, hence the same scale
// in the mixed forms) of cell idx, the direction chosen per lane.
template <int Q, int PREC, int I>
__device__ __forceinline__ typename Prec<PREC>::calc pop_load_pair(const void *base, long long N, bool opp,
                                                                   uint32_t idx)
{
    using T = typename Prec<PREC>::pop;
    constexpr int OPP = Q - 1 - I;
    static_assert(Lat<Q>::w(I) == Lat<Q>::w(OPP), "opposite directions share a weight");
    const size_t dir = opp ? (size_t)OPP : (size_t)I;
    const char *b = (const char *)base + dir * (size_t)N * sizeof(T);
    const uint32_t off = idx * (uint32_t)sizeof(T);
    if constexpr (PREC == LBFD_FP64) {
        return ldo<double>(b, off);
    } else if constexpr (PREC == LBFD_MIXED_FP32) {
        constexpr float s = (float)(Lat<Q>::w(I) * kCs2);
        return ldo<float>(b, off) * s;
    } else {
        constexpr float s = (float)(Lat<Q>::w(I) * kCs2);
        return __half2float(ldo<__half>(b, off)) * s;
    }
}

// A zero that a lane loads in place of an entry it does not need.
static __constant__ double kZeroEntry[1] = {0.0};

// Boundary cells: pull and stencil from the per-cell descriptors built at
// init (same rules as gather / axis_stencil, resolved once on the host).
// The pull keeps every lane on one path: the source population is one load
// whose direction and cell are selected per lane, and the rarer inlet,
// outlet and interpolated-wall terms are evaluated under wave-uniform
// conditions (some lane of the wave needs them) for every lane, each lane
// keeping its own by selection.  (Per-lane branches here let the register
// allocator of the toolchain place copies of values that live through the
// branch in the join block, where only one side's lanes are active, so
// that the other side's lanes later read stale registers.)
template <int Q, int PREC, int I, bool CW>
__device__ __forceinline__ typename Prec<PREC>::calc desc_pull(const KParams &P, long long t, long long nb,
                                                               long long idx, int x, int y, int z,
                                                               unsigned long long pcode)
{
    using C = typename Prec<PREC>::calc;
    using L = Lat<Q>;
    constexpr int OPP = Q - 1 - I;
    if constexpr (I == (Q - 1) / 2) {
        return pop_load<Q, PREC, I>(P.pop_in, P.N, (uint32_t)idx);
    } else {
        // the source: the full descriptor with curved-wall links (whose
        // rule also reads the opposite direction's), else the compact code
        int src;
        if constexpr (CW) {
            src = P.bsrc[I * nb + t];
        } else {
            const int kind = decode_pull_kind(pcode, I);
            src = kind == kPullFluid    ? (int)cell_at(x, y, z, -L::cx(I), -L::cy(I), -L::cz(I), P.nx, P.ny, P.nz)
                  : kind == kPullBounce ? kSrcBounce
                  : kind == kPullInflow ? kSrcInflow
                                        : kSrcOutlet;
        }
        const bool fluid = src >= 0;
        // the source cell's population I, or this cell's opposite one
        // (half-way bounce-back, and the base of the inlet rule)
        C g = pop_load_pair<Q, PREC, I>(P.pop_in, P.N, !fluid, fluid ? (uint32_t)src : (uint32_t)idx);
        const bool inflow = src == kSrcInflow, outlet = src == kSrcOutlet;
        if (__any(inflow)) {
            // inlet (Eq. 31): + 2 w_I rho_in c_I.u_in; an x face carries the
            // per-cell profile indexed by the cell's (y, z)
            constexpr int cx = L::cx(I), cy = L::cy(I), cz = L::cz(I);
            const int f = (cx == 1 && x == 0 && P.face[0] == LBFD_FACE_INFLOW)               ? 0
                          : (cx == -1 && x == P.nx - 1 && P.face[1] == LBFD_FACE_INFLOW) ? 1
                                                                                         : -1;
            const bool prof = inflow && f >= 0;
            const long long s3 = (long long)P.ny * P.nz;
            const double *ub = prof ? P.inflow_u : kZeroEntry;
            const long long o = prof ? 3 * s3 * f + (long long)z * P.ny + y : 0;
            const double ux = ub[o], uy = ub[prof ? o + s3 : 0], uz = ub[prof ? o + 2 * s3 : 0];
            const double cu = prof ? cx * ux + cy * uy + cz * uz : cx * P.u_in[0] + cy * P.u_in[1] + cz * P.u_in[2];
            g = inflow ? g + (C)(2.0 * L::w(I) * P.rho_in * cu) : g;
        }
        if (__any(outlet)) {
            // outlet value kept in the outlet buffer
            const double *ob = outlet ? P.outlet : kZeroEntry;
            const C ov = (C)ob[outlet ? outlet_index(P, L::cx(I) < 0 ? 1 : 0, I, Q, y, z) : 0];
            g = outlet ? ov : g;
        }
        if constexpr (CW) {
            // linearly interpolated bounce-back (post-collision form) for a
            // wall met at the fraction q of the link toward it (direction OPP)
            if (P.bq != nullptr) {
                const float qraw = P.bq[I * nb + t];
                const float qs = src == kSrcBounce ? qraw : __builtin_nanf("");
                const bool interp = qs == qs;
                if (__any(interp)) {
                    const C q2 = (C)2 * (C)qs;  // weights in the arithmetic precision
                    // q < 1/2: the far node r + c_I is the pull source of
                    // direction OPP (when it is a fluid cell)
                    const int far = P.bsrc[OPP * nb + t];
                    const bool near_half = qs < 0.5f;
                    const bool use_far = interp && near_half && far >= 0;
                    const C gfar = pop_load_pair<Q, PREC, I>(P.pop_in, P.N, true, use_far ? (uint32_t)far : (uint32_t)idx);
                    const C gown = pop_load<Q, PREC, I>(P.pop_in, P.N, (uint32_t)idx);
                    const C lo = q2 * g + ((C)1 - q2) * gfar;
                    const C iq = (C)1 / (interp && !near_half ? q2 : (C)1);
                    const C hi = g * iq + (q2 - (C)1) * iq * gown;
                    g = use_far ? lo : (interp && !near_half) ? hi : g;
                }
            }
        }
        return g;
    }
}

// Values (T, rho, Y_k) at a listed image point, reconstructed for this
// level by image_kernel.
template <int NSP, class C>
__device__ __forceinline__ void image_value(const KParams &P, int li, Pt<NSP, C> &o)
{
    o.T = (C)P.img_val[li];
    o.rho = (C)P.img_val[P.n_img + li];
#pragma unroll
    for (int k = 0; k < NSP; ++k) o.Y[k] = (C)P.img_val[(2 + k) * P.n_img + li];
}

template <int NSP, int PREC, bool DIAG, bool CW = false>
__device__ __forceinline__ void desc_stencil(const KParams &P, long long t, long long nb, int d,
                                             const Pt<NSP, typename Prec<PREC>::calc> &ctr,
                                             Pt<NSP, typename Prec<PREC>::calc> (&st)[5], bool &near, double &wallq)
{
    using C = typename Prec<PREC>::calc;
    st[2] = ctr;
    int pts[4], wks[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        pts[j] = P.bpt[(d * 4 + j) * nb + t];
        wks[j] = P.bwk[(d * 4 + j) * nb + t];
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const int slot = j < 2 ? j : j + 1;
        Pt<NSP, C> img;
        const int li = CW && P.bimg != nullptr ? P.bimg[(d * 4 + j) * nb + t] : -1;
        if (li >= 0)
            image_value<NSP>(P, li, img);
        else
            load_point<NSP, PREC>(P, pts[j], img);
        // a fluid point passes through ghost() unchanged
        Nb w;
        w.kind = wks[j];
        w.face = -1;
        w.idx = 0;
        w.Tw = P.btw[(d * 4 + j) * nb + t];
        near |= w.kind != kFluid;
        ghost<NSP>(P, w, img, st[slot]);
        if constexpr (DIAG) {
            if ((j == 1 || j == 2) && w.kind == kIso)
                wallq += 2.0 * P.alpha * (double)density<NSP>(P, (C)w.Tw, ctr.Y) * ((double)ctr.T - w.Tw);
        }
    }
}

// fourth-order central first and second derivatives (Sec. II.D)
template <class C>
__device__ __forceinline__ C d1(C a, C b, C c, C d, C e)
{
    return ((a - (C)8 * b) + ((C)8 * d - e)) * (C)(1.0 / 12.0);
}
template <class C>
__device__ __forceinline__ C d2(C a, C b, C c, C d, C e)
{
    return ((C)16 * (b + d) - (a + e) - (C)30 * c) * (C)(1.0 / 12.0);
}

// WENO3 convective derivative (Jiang-Shu weights, eps = 1e-6): for u >= 0
// the face values at i+1/2 and i-1/2 are reconstructed from the left; for
// u < 0 the stencil is mirrored and the result negated, which is the
// right-biased reconstruction.  At a face between b and c reconstructed
// from the side of b (a the far upwind point) the value is
// q1 + w0 (q0 - q1), q0 = 3b/2 - a/2, q1 = (b+c)/2, with the normalised
// weight w0 = e1^2 / (e1^2 + 2 e0^2), e0 = eps + (b-a)^2,
// e1 = eps + (c-b)^2; both faces share one division.
template <class C>
__device__ __forceinline__ C weno3(C m2, C m1, C c0, C p1, C p2, C u)
{
    const bool neg = u < (C)0;
    const C A = neg ? p2 : m2, B = neg ? p1 : m1, E = neg ? m1 : p1;
    const C eps = (C)1e-6;
    const C dA = B - A, dB = c0 - B, dE = E - c0;
    const C eA = eps + dA * dA, eB = eps + dB * dB, eE = eps + dE * dE;
    const C eA2 = eA * eA, eB2 = eB * eB, eE2 = eE * eE;
    const C den_p = eE2 + (C)2 * eB2;  // face i+1/2: e0 = eB, e1 = eE
    const C den_m = eB2 + (C)2 * eA2;  // face i-1/2: e0 = eA, e1 = eB
    const C inv = rcp(den_p * den_m);
    const C w_p = eE2 * den_m * inv, w_m = eB2 * den_p * inv;
    const C q0p = (C)1.5 * c0 - (C)0.5 * B, q1p = (C)0.5 * (c0 + E);
    const C q0m = (C)1.5 * B - (C)0.5 * A, q1m = (C)0.5 * (B + c0);
    const C conv = (q1p + w_p * (q0p - q1p)) - (q1m + w_m * (q0m - q1m));
    return neg ? -conv : conv;
}

// The three finite-difference operators of one scalar along one axis from
// its five stencil values, written on the forward differences
// D0 = m1 - m2, D1 = c0 - m1, D2 = p1 - c0, D3 = p2 - p1:
//   D1 (4th order) = (7 (D1 + D2) - (D0 + D3)) / 12,
//   D2 (4th order) = (15 (D2 - D1) - (D3 - D0)) / 12,
//   conv2 = twice the WENO3 convective derivative of weno3() (the caller
//   folds the 1/2 into u): with (a, b, c) = (D0, D1, D2) for u >= 0 and
//   (D3, D2, D1) for u < 0 (the mirrored stencil, whose negation cancels the
//   sign of its differences), conv2 = (b + c) + w+ (b - c) - w- (a - b),
//   w+ = eC^2 / (eC^2 + 2 eB^2), w- = eB^2 / (eB^2 + 2 eA^2), eX = eps + X^2,
//   both weights from one reciprocal; next to walls (near) the centred
//   difference b + c.
template <class C>
__device__ __forceinline__ void axis5(C m2, C m1, C c0, C p1, C p2, C u, bool near, C &d1o, C &d2o, C &conv2)
{
    const C D0 = m1 - m2, D1 = c0 - m1, D2 = p1 - c0, D3 = p2 - p1;
    const C s12 = D1 + D2;
    d1o = ((C)7 * s12 - (D0 + D3)) * (C)(1.0 / 12.0);
    d2o = ((C)15 * (D2 - D1) - (D3 - D0)) * (C)(1.0 / 12.0);
    const bool neg = u < (C)0;
    const C a = neg ? D3 : D0, b = neg ? D2 : D1, c = neg ? D1 : D2;
    const C eps = (C)1e-6;
    const C eA = eps + a * a, eB = eps + b * b, eC = eps + c * c;
    const C eA2 = eA * eA, eB2 = eB * eB, eC2 = eC * eC;
    const C den_p = eC2 + (C)2 * eB2, den_m = eB2 + (C)2 * eA2;
    const C inv = rcp(den_p * den_m);
    const C X = (eC2 * (b - c)) * den_m - (eB2 * (a - b)) * den_p;
    conv2 = near ? s12 : s12 + X * inv;
}

// ------------------------------------------------------------ chemistry
// Arrhenius source over one step in double precision (per reaction
// r = A dt T^b exp(-Ta/T) prod Y_react; species nu_k r, temperature q r):
// one explicit Euler step, or, with chem_substeps_max > 1, N sub-steps
// with N = ceil(max_j k_j / 0.1) capped at chem_substeps_max; a sub-step
// that would consume a mass fraction below zero is scaled down.
// The rate coefficient A dt T^b exp(-Ta/T) is formed from ln T and 1/T
// shared by every reaction as (A dt) exp(b ln T - Ta / T), one exponential
// per reaction (with b = 0 it is A dt exp(-Ta / T)).
__device__ __forceinline__ double rate_coeff_l(const ChemRx &r, double lnT, double invT, const double *tab)
{
    return r.adt * exp_tab(r.b * lnT - r.ta * invT, tab);
}

// The same coefficient divided by the sub-step count N, with ln(A dt) and
// ln N moved into the exponent: exp(b ln T - Ta/T + ln(A dt) - ln N), formed
// in units of ln 2 / 256 (lnNs = ln N 256/ln 2).  Each operation takes one
// per-reaction constant: an instruction reads at most one scalar register
// operand.
__device__ __forceinline__ double rate_coeff_sub(const ChemRx &r, double lnT, double invT, double lnNs,
                                                 const double *tab)
{
    return exp_scaled_tab(fma(r.bs, lnT, fma(-r.tas, invT, -lnNs)) + r.lnadts, tab);
}

// Returns the number of sub-steps taken.  NR: the largest reactant count
// of a reaction (slots past a reaction's own count multiply by 1).
template <int NSP, bool LE = false, int NR = 4>
__device__ __forceinline__ int chemistry(const KParams &P, const double *tab, const double *ltab, double T,
                                         const double (&Y)[NSP],
                                         double &srcT, double (&srcY)[NSP])
{
    // ln T is needed only when a temperature exponent is not zero
    const bool anyb = P.chem_anyb != 0;
    int nsub = 1;
    if (P.chem_substeps_max > 1) {
        const double lnT = anyb ? log(T) : 0.0, invT = rcp(T);
        double kmax = 0.0;
        for (int j = 0; j < P.n_rx; ++j) kmax = fmax(kmax, rate_coeff_l(P.rxk[j], lnT, invT, tab));
        double want = ceil(kmax / 0.1);
        nsub = want < 1.0 ? 1 : want > (double)P.chem_substeps_max ? P.chem_substeps_max : (int)want;
    }
    const double lnNs = nsub == 1 ? 0.0 : log((double)nsub) * 0x1.71547652b82fep+8;  // ln N 256/ln 2
    double dT = 0.0, dY[NSP];
#pragma unroll
    for (int k = 0; k < NSP; ++k) dY[k] = 0.0;
    for (int s = 0; s < nsub; ++s) {
        const double Tc = T + dT;
        // Yc[NSP] = 1 is the factor of the unused reactant slots
        double Yc[NSP + 1];
#pragma unroll
        for (int k = 0; k < NSP; ++k) Yc[k] = Y[k] + dY[k];
        Yc[NSP] = 1.0;
        double incT = 0.0, incY[NSP];
#pragma unroll
        for (int k = 0; k < NSP; ++k) incY[k] = 0.0;
        const double lnTc = anyb ? log_tab(Tc, ltab) : 0.0, invTc = rcp(Tc);
        // one reaction's progress over the sub-step and its increments;
        // the reactant indices are the same for every lane, so Yc is
        // indexed through the register file (no private memory).  The four
        // reactant slots are all multiplied in (the unused ones index the
        // constant 1): a fixed count lets the four indices arrive in one
        // scalar load ahead of the products instead of one dependent load
        // per reactant
        auto apply = [&](const ChemRx &r, double k) {
            double rr = k;
#pragma unroll
            for (int m = 0; m < NR; ++m) rr *= Yc[r.react[m]];
#pragma unroll
            for (int k2 = 0; k2 < NSP; ++k2) incY[k2] += r.nu[k2] * rr;
            incT += r.q * rr;
        };
        // reactions four at a time: the four exponentials are independent
        // and interleave, the increments follow in reaction order
        int j = 0;
        for (; j + 4 <= P.n_rx; j += 4) {
            double k4[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) k4[u] = rate_coeff_sub(P.rxk[j + u], lnTc, invTc, lnNs, tab);
#pragma unroll
            for (int u = 0; u < 4; ++u) apply(P.rxk[j + u], k4[u]);
        }
        for (; j < P.n_rx; ++j) apply(P.rxk[j], rate_coeff_sub(P.rxk[j], lnTc, invTc, lnNs, tab));
        if constexpr (LE) {
            // q_over_cp is the rise at c_p,ref: divide by c_p(Y) / c_p,ref
            // at the sub-step's composition (Eq. 7: omega_T / (rho c_p))
            double cpm = 0.0;
#pragma unroll
            for (int k = 0; k < NSP; ++k) cpm += Yc[k] * P.cpk[k];
            incT *= rcp(cpm);
        }
        // positivity limiter: scale the sub-step so that no mass fraction
        // is consumed below zero (1, i.e. plain Euler, otherwise)
        double lam = 1.0;
#pragma unroll
        for (int k = 0; k < NSP; ++k)
            if (incY[k] < 0.0 && Yc[k] + incY[k] < 0.0) lam = fmin(lam, fmax(Yc[k], 0.0) * rcp(-incY[k]));
        dT += lam * incT;
#pragma unroll
        for (int k = 0; k < NSP; ++k) dY[k] += lam * incY[k];
    }
    srcT = dT;
#pragma unroll
    for (int k = 0; k < NSP; ++k) srcY[k] = dY[k];
    return nsub;
}

// ------------------------------------------------- central-moment transform
// Central moments about u (Sec. II.C, Eq. 21) of the 3 x 3 (x 3) cube of
// populations, one axis at a time.  Along a line with velocities -1, 0, 1
// holding (a, b, d): m0 = a+b+d, m1 = (d-a) - u m0,
// m2 = (a+d) + 2u(a-d) + u^2 m0.  Moment (p, q, r) lands at p + 3q + 9r.
template <class C>
__device__ __forceinline__ void cm_fwd_line(C &a, C &b, C &d, C u)
{
    C m0 = a + b + d;
    C m1 = (d - a) - u * m0;
    C m2 = (a + d) + (C)2 * u * (a - d) + u * u * m0;
    a = m0;
    b = m1;
    d = m2;
}

// exact inverse of cm_fwd_line
template <class C>
__device__ __forceinline__ void cm_inv_line(C &a, C &b, C &d, C u)
{
    C m0 = a, m1 = b, m2 = d;
    C uu = u * u;
    a = (C)0.5 * (m0 * (uu - u) + m1 * ((C)2 * u - (C)1) + m2);
    b = m0 * ((C)1 - uu) - (C)2 * u * m1 - m2;
    d = (C)0.5 * (m0 * (uu + u) + m1 * ((C)2 * u + (C)1) + m2);
}

template <int Q, class C>
__device__ __forceinline__ void central_fwd(C (&h)[Q], const C (&u)[3])
{
#pragma unroll
    for (int l = 0; l < Q / 3; ++l) cm_fwd_line(h[3 * l], h[3 * l + 1], h[3 * l + 2], u[0]);
#pragma unroll
    for (int zp = 0; zp < Q / 9; ++zp)
#pragma unroll
        for (int p = 0; p < 3; ++p) cm_fwd_line(h[9 * zp + p], h[9 * zp + p + 3], h[9 * zp + p + 6], u[1]);
    if constexpr (Q == 27) {
#pragma unroll
        for (int r = 0; r < 9; ++r) cm_fwd_line(h[r], h[r + 9], h[r + 18], u[2]);
    }
}

template <int Q, class C>
__device__ __forceinline__ void central_inv(C (&h)[Q], const C (&u)[3])
{
    if constexpr (Q == 27) {
#pragma unroll
        for (int r = 0; r < 9; ++r) cm_inv_line(h[r], h[r + 9], h[r + 18], u[2]);
    }
#pragma unroll
    for (int zp = 0; zp < Q / 9; ++zp)
#pragma unroll
        for (int p = 0; p < 3; ++p) cm_inv_line(h[9 * zp + p], h[9 * zp + p + 3], h[9 * zp + p + 6], u[1]);
#pragma unroll
    for (int l = 0; l < Q / 3; ++l) cm_inv_line(h[3 * l], h[3 * l + 1], h[3 * l + 2], u[0]);
}

// Relax toward the Maxwellian central moments at temperature cs^2: orders
// 0-1 kept, order 2 at 1/tau, order 3 at omega3, higher at omega4.
template <int Q, class C>
__device__ __forceinline__ void relax(C (&k)[Q], C om2, C om3, C om4)
{
    sfor<0, Q>([&](auto J) {
        constexpr int j = decltype(J)::value;
        constexpr int p = j % 3, q = (j / 3) % 3, r = (Q == 27) ? j / 9 : 0;
        constexpr int order = p + q + r;
        if constexpr (order >= 2) {
            constexpr bool odd = (p == 1) || (q == 1) || (r == 1);
            constexpr int n2 = (p == 2) + (q == 2) + (r == 2);
            constexpr double tgt = odd ? 0.0 : (n2 == 1 ? kCs2 : n2 == 2 ? kCs2 * kCs2 : kCs2 * kCs2 * kCs2);
            C om = order == 2 ? om2 : order == 3 ? om3 : om4;
            k[j] = k[j] - om * (k[j] - (C)tgt);
        }
    });
}

// Relaxation with the orders >= 4 taken as cumulants (the cumulant form of
// the collision, Sec. II.C).  For the unit-mass, zero-mean shifted
// distribution the cumulants of orders 2 and 3 are the central moments;
// those of orders 4-6 on the 3 x 3 (x 3) cube follow from the
// moment-cumulant relation, kappa_a = sum over the set partitions of a's
// index positions into blocks of two or more of the product of the blocks'
// cumulants (first-order blocks vanish), expanded here by hand:
//   order 4: C_xxyy = k_xxyy - k_xx k_yy - 2 k_xy^2,
//            C_xxyz = k_xxyz - k_xx k_yz - 2 k_xy k_xz;
//   order 5: C_xxyyz = k_xxyyz - k_xx k_yyz - k_yy k_xxz - 2 k_xz k_xyy
//                      - 2 k_yz k_xxy - 4 k_xy k_xyz;
//   order 6: C_xxyyzz = k_xxyyzz - (pair x 4-block: 15 terms)
//                       - (two triples: 10) - (three pairs: 15),
// and the inverse with the relaxed cumulants and the post-collision
// orders 2, 3.  Cumulants of order >= 4 relax at om4 toward 0 (those of the
// Maxwellian); orders 2, 3 as in relax().
template <int Q, class C>
__device__ __forceinline__ void relax_cumulants(C (&k)[Q], C om2, C om3, C om4)
{
    auto K = [&](int p, int q, int r) -> C & { return k[p + 3 * q + 9 * r]; };
    const C keep = (C)1 - om4;
    if constexpr (Q == 9) {
        const C c22 = K(2, 2, 0) - K(2, 0, 0) * K(0, 2, 0) - (C)2 * K(1, 1, 0) * K(1, 1, 0);
        relax<Q>(k, om2, om3, (C)0);
        K(2, 2, 0) = keep * c22 + K(2, 0, 0) * K(0, 2, 0) + (C)2 * K(1, 1, 0) * K(1, 1, 0);
    } else {
        // pre-collision second and third orders
        const C a = K(2, 0, 0), b = K(0, 2, 0), c = K(0, 0, 2);          // xx, yy, zz
        const C xy = K(1, 1, 0), xz = K(1, 0, 1), yz = K(0, 1, 1);
        const C xxy = K(2, 1, 0), xxz = K(2, 0, 1), xyy = K(1, 2, 0), yyz = K(0, 2, 1);
        const C xzz = K(1, 0, 2), yzz = K(0, 1, 2), xyz = K(1, 1, 1);
        // pre-collision cumulants of orders 4, 5, 6
        const C c220 = K(2, 2, 0) - a * b - (C)2 * xy * xy;
        const C c202 = K(2, 0, 2) - a * c - (C)2 * xz * xz;
        const C c022 = K(0, 2, 2) - b * c - (C)2 * yz * yz;
        const C c211 = K(2, 1, 1) - a * yz - (C)2 * xy * xz;
        const C c121 = K(1, 2, 1) - b * xz - (C)2 * xy * yz;
        const C c112 = K(1, 1, 2) - c * xy - (C)2 * xz * yz;
        const C c221 = K(2, 2, 1) - a * yyz - b * xxz - (C)2 * xz * xyy - (C)2 * yz * xxy - (C)4 * xy * xyz;
        const C c212 = K(2, 1, 2) - a * yzz - c * xxy - (C)2 * xy * xzz - (C)2 * yz * xxz - (C)4 * xz * xyz;
        const C c122 = K(1, 2, 2) - b * xzz - c * xyy - (C)2 * xy * yzz - (C)2 * xz * yyz - (C)4 * yz * xyz;
        const C s42 = a * c022 + b * c202 + c * c220 + (C)4 * (xy * c112 + xz * c121 + yz * c211);
        const C s33 = (C)2 * (xxy * yzz + xxz * yyz + xyy * xzz) + (C)4 * xyz * xyz;
        const C s222 = a * b * c + (C)2 * (a * yz * yz + b * xz * xz + c * xy * xy) + (C)8 * xy * xz * yz;
        const C c222 = K(2, 2, 2) - s42 - s33 - s222;
        relax<Q>(k, om2, om3, (C)0);
        // post-collision second and third orders, relaxed cumulants
        const C A = K(2, 0, 0), B = K(0, 2, 0), Cc = K(0, 0, 2);
        const C XY = K(1, 1, 0), XZ = K(1, 0, 1), YZ = K(0, 1, 1);
        const C XXY = K(2, 1, 0), XXZ = K(2, 0, 1), XYY = K(1, 2, 0), YYZ = K(0, 2, 1);
        const C XZZ = K(1, 0, 2), YZZ = K(0, 1, 2), XYZ = K(1, 1, 1);
        const C d220 = keep * c220, d202 = keep * c202, d022 = keep * c022;
        const C d211 = keep * c211, d121 = keep * c121, d112 = keep * c112;
        K(2, 2, 0) = d220 + A * B + (C)2 * XY * XY;
        K(2, 0, 2) = d202 + A * Cc + (C)2 * XZ * XZ;
        K(0, 2, 2) = d022 + B * Cc + (C)2 * YZ * YZ;
        K(2, 1, 1) = d211 + A * YZ + (C)2 * XY * XZ;
        K(1, 2, 1) = d121 + B * XZ + (C)2 * XY * YZ;
        K(1, 1, 2) = d112 + Cc * XY + (C)2 * XZ * YZ;
        K(2, 2, 1) = keep * c221 + A * YYZ + B * XXZ + (C)2 * XZ * XYY + (C)2 * YZ * XXY + (C)4 * XY * XYZ;
        K(2, 1, 2) = keep * c212 + A * YZZ + Cc * XXY + (C)2 * XY * XZZ + (C)2 * YZ * XXZ + (C)4 * XZ * XYZ;
        K(1, 2, 2) = keep * c122 + B * XZZ + Cc * XYY + (C)2 * XY * YZZ + (C)2 * XZ * YYZ + (C)4 * YZ * XYZ;
        const C S42 = A * d022 + B * d202 + Cc * d220 + (C)4 * (XY * d112 + XZ * d121 + YZ * d211);
        const C S33 = (C)2 * (XXY * YZZ + XXZ * YYZ + XYY * XZZ) + (C)4 * XYZ * XYZ;
        const C S222 = A * B * Cc + (C)2 * (A * YZ * YZ + B * XZ * XZ + Cc * XY * XY) + (C)8 * XY * XZ * YZ;
        K(2, 2, 2) = keep * c222 + S42 + S33 + S222;
    }
}

// ------------------------------------------------------------ reductions
__device__ __forceinline__ void diag_combine(double (&a)[kNDiag], const double *b)
{
    a[kSumG] += b[kSumG];
    a[kSumXi] += b[kSumXi];
    a[kMomX] += b[kMomX];
    a[kMomY] += b[kMomY];
    a[kMomZ] += b[kMomZ];
    a[kMaxY] = fmax(a[kMaxY], b[kMaxY]);
    a[kNonfinite] += b[kNonfinite];
    a[kTheta] += b[kTheta];
    if (b[kHrrMax] > a[kHrrMax] || (b[kHrrMax] == a[kHrrMax] && b[kHrrIdx] < a[kHrrIdx])) {
        a[kHrrMax] = b[kHrrMax];
        a[kHrrIdx] = b[kHrrIdx];
    }
    a[kWallQ] += b[kWallQ];
    a[kFuel] += b[kFuel];
    a[kFuelMass] += b[kFuelMass];
}

__device__ __forceinline__ void diag_identity(double (&a)[kNDiag])
{
#pragma unroll
    for (int s = 0; s < kNDiag; ++s) a[s] = 0.0;
    a[kHrrMax] = -INFINITY;
    a[kHrrIdx] = 1e300;
}

// Block reduction (wave64 butterflies, then the waves in order) of the
// per-thread diagnostics; thread 0 writes the block's partial.
__device__ __forceinline__ void block_reduce_diag(double (&a)[kNDiag], double *out)
{
    __shared__ double red[kBlock / 64][kNDiag];
    const int tid = threadIdx.x + blockDim.x * (threadIdx.y + blockDim.y * threadIdx.z);
    const int lane = tid & 63, wave = tid >> 6;
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
        double b[kNDiag];
#pragma unroll
        for (int s = 0; s < kNDiag; ++s) b[s] = __shfl_xor(a[s], off, 64);
        diag_combine(a, b);
    }
    if (lane == 0)
#pragma unroll
        for (int s = 0; s < kNDiag; ++s) red[wave][s] = a[s];
    __syncthreads();
    if (tid == 0) {
        const int nw = (blockDim.x * blockDim.y * blockDim.z + 63) / 64;
        for (int w = 1; w < nw; ++w) diag_combine(a, red[w]);
#pragma unroll
        for (int s = 0; s < kNDiag; ++s) out[s] = a[s];
    }
}

// ------------------------------------------------------------ step kernel
// Everything after the finite differences, for one fluid cell: Arrhenius
// source, Lambda (Eq. 6), Euler update, P_h (Eq. 13a), source Xi_i (Eq. 9),
// central-moment collision (Eqs. 14, 19, 21), diagnostics, stores.
// diffT, diffY already carry the factor alpha.
template <int Q, int NSP, int PREC, int MODE, bool LE = false>
__device__ __forceinline__ void finish_cell(const KParams &P, long long idx, const typename Prec<PREC>::calc (&g)[Q],
                                            const Pt<NSP, typename Prec<PREC>::calc> &ctr,
                                            const typename Prec<PREC>::calc (&u)[3],
                                            const typename Prec<PREC>::calc (&m)[3], typename Prec<PREC>::calc sg,
                                            typename Prec<PREC>::calc inv_rc, typename Prec<PREC>::calc diffT,
                                            const typename Prec<PREC>::calc (&diffY)[NSP],
                                            typename Prec<PREC>::calc CT, const typename Prec<PREC>::calc (&CY)[NSP],
                                            const typename Prec<PREC>::calc (&grad)[3], double wallq,
                                            double (&acc)[kNDiag])
{
    using L = Lat<Q>;
    using C = typename Prec<PREC>::calc;
    using S = typename Prec<PREC>::scal;
    constexpr bool DIAG = MODE != kModeStep;
    const C rho = ctr.rho;
    // Arrhenius source (double): computed here, or read back from this
    // step's output scalars where the chemistry launch left it
    double srcT, srcY[NSP];
    if constexpr (chem_pass(NSP)) {
        const char *so = (const char *)P.sc_out;
        const size_t fstride = (size_t)P.N * sizeof(S);
        const uint32_t off = (uint32_t)idx * (uint32_t)sizeof(S);
        srcT = (double)ldo<S>(so, off);
#pragma unroll
        for (int k = 0; k < NSP; ++k) srcY[k] = (double)ldo<S>(so + (size_t)(1 + k) * fstride, off);
    } else {
        double Yd[NSP];
#pragma unroll
        for (int k = 0; k < NSP; ++k) Yd[k] = (double)ctr.Y[k];
        chemistry<NSP, LE>(P, kExp2Tab, kLogTab, (double)ctr.T, Yd, srcT, srcY);
    }

    // material derivatives, Lambda (Eq. 6), Euler update, P_h (Eq. 13a)
    const C DtT = diffT + (C)srcT;
    C DtY[NSP], invW = 0;
#pragma unroll
    for (int k = 0; k < NSP; ++k) {
        DtY[k] = diffY[k] + (C)srcY[k];
        invW += ctr.Y[k] * (C)P.invW[k];
    }
    const C Wm = rcp(invW);
    C Lam = DtT * rcp(ctr.T);
#pragma unroll
    for (int k = 0; k < NSP; ++k) Lam += (Wm * (C)P.invW[k]) * DtY[k];
    const C Tn = ctr.T - CT + DtT;
    C Yn[NSP];
#pragma unroll
    for (int k = 0; k < NSP; ++k) Yn[k] = ctr.Y[k] - CY[k] + DtY[k];
    const C Ph = sg + (C)0.5 * rho * (C)kCs2 * Lam;

    // source Xi_i (Eq. 9) and pre-conditioned populations (Eq. 19)
    const C uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
    C xi[Q], h[Q], pi = 0, sxi = 0;
    const C half_inv = (C)0.5 * inv_rc;
    sfor<0, Q>([&](auto I) {
        constexpr int i = decltype(I)::value;
        constexpr C wi = (C)L::w(i);
        const C cu = (C)L::cx(i) * u[0] + (C)L::cy(i) * u[1] + (C)L::cz(i) * u[2];
        const C feq_r = wi * ((C)1 + (C)3 * cu + (C)4.5 * cu * cu - (C)1.5 * uu);
        const C proj = ((C)L::cx(i) - u[0]) * grad[0] + ((C)L::cy(i) - u[1]) * grad[1] +
                       ((C)L::cz(i) - u[2]) * grad[2];
        xi[i] = (C)kCs2 * (feq_r - wi) * proj + wi * rho * (C)kCs2 * Lam;
        sxi += xi[i];
        h[i] = g[i] * inv_rc + xi[i] * half_inv;
        pi += h[i];
    });
    // unit-mass shift, central-moment relaxation, shift back (Eq. 14)
    const C sh = (C)1 - pi;
    sfor<0, Q>([&](auto I) { h[decltype(I)::value] += (C)L::w(decltype(I)::value) * sh; });
    central_fwd<Q>(h, u);
    if (P.collision == LBFD_CUMULANTS)
        relax_cumulants<Q>(h, (C)P.omega2, (C)P.omega3, (C)P.omega4);
    else
        relax<Q>(h, (C)P.omega2, (C)P.omega3, (C)P.omega4);
    central_inv<Q>(h, u);
    const C rc = rho * (C)kCs2;
    sfor<0, Q>([&](auto I) {
        constexpr int i = decltype(I)::value;
        h[i] = rc * (h[i] - (C)L::w(i) * sh) + (C)0.5 * xi[i];
    });

    if constexpr (DIAG) {
        bool bad = !isfinite((double)ctr.T);
#pragma unroll
        for (int k = 0; k < NSP; ++k) bad |= !isfinite((double)ctr.Y[k]);
#pragma unroll
        for (int i = 0; i < Q; ++i) bad |= !isfinite((double)g[i]);
        if (bad) {
            acc[kNonfinite] = 1.0;
        } else {
            double sy = 0.0;
#pragma unroll
            for (int k = 0; k < NSP; ++k) sy += (double)ctr.Y[k];
            acc[kSumG] = (double)sg;
            acc[kSumXi] = (double)sxi;
            acc[kMomX] = (double)m[0] * 3.0;
            acc[kMomY] = (double)m[1] * 3.0;
            acc[kMomZ] = (double)m[2] * 3.0;
            acc[kMaxY] = fabs(sy - 1.0);
            acc[kTheta] = ((double)ctr.T - P.T_u) / (P.T_b - P.T_u);
            acc[kHrrMax] = srcT;
            acc[kHrrIdx] = (double)idx;
            acc[kWallQ] = wallq;
            acc[kFuel] = -srcY[0];
            acc[kFuelMass] = -srcY[0] * (double)ctr.rho;
        }
    }

    if constexpr (MODE != kModeFields) {
        sfor<0, Q>([&](auto I) { pop_store<Q, PREC, decltype(I)::value>(P.pop_out, P.N, idx, h[decltype(I)::value]); });
        char *so = (char *)P.sc_out;
        const size_t fstride = (size_t)P.N * sizeof(S);
        const uint32_t off = (uint32_t)idx * (uint32_t)sizeof(S);
        sto<S>(so, off, (S)Tn);
#pragma unroll
        for (int k = 0; k < NSP; ++k) sto<S>(so + (size_t)(1 + k) * fstride, off, (S)Yn[k]);
    } else {
        P.fields[idx] = (double)rho;
        P.fields[P.N + idx] = (double)u[0];
        P.fields[2 * P.N + idx] = (double)u[1];
        P.fields[3 * P.N + idx] = (double)u[2];
        P.fields[4 * P.N + idx] = (double)Ph;
    }
}

// Interior tile of one 256-thread block: 64 x 4 cells in 2-D, 64 x 2 x 2
// in 3-D.
template <int D> struct TileShape {
    static constexpr int X = 64, Y = D == 2 ? 4 : 2, Z = D == 2 ? 1 : 2;
};

// One block of the step.
// FAST = true: an interior tile (bx, by, bz) of the box whose threads work
// only on interior fluid cells (every pull source and every finite-difference
// point in the box and fluid), with plain offset loads.
// FAST = false: block bx of the list of the other fluid cells (boundary
// cells), with the general geometry logic.
// (tx, ty, tz): the thread's place in the tile (FAST) or tx in 0..255.
// slot: the block's row of the diagnostics partials.
// CW: boundary cells apply the curved-wall treatments when listed: the
// interpolated bounce-back of P.bq and the Shepard image points of P.bimg (a
// separate instantiation, so that contexts without them keep the registers
// of plain bounce-back and axis-mirror ghosts).
template <int Q, int NSP, int PREC, int MODE, bool FAST, bool CW = false, bool LE = false>
__device__ __forceinline__ void step_block(const KParams &P, int bx, int by, int bz, int tx, int ty, int tz,
                                           long long slot)
{
    using L = Lat<Q>;
    using C = typename Prec<PREC>::calc;
    constexpr int D = L::D;
    constexpr bool DIAG = MODE != kModeStep;
    using TS = TileShape<D>;
    int x, y, z;
    long long idx, tb = 0;
    unsigned long long pcode = 0, scode = 0;  // a boundary cell's compact codes
    bool active, inbox;
    if constexpr (FAST) {
        x = bx * TS::X + tx;
        y = by * TS::Y + ty;
        z = bz * TS::Z + tz;
        inbox = x < P.nx && y < P.ny && z < P.nz;
        idx = inbox ? ((long long)z * P.ny + y) * P.nx + x : 0;
        active = inbox && P.code[idx] == kCodeInterior;
    } else {
        tb = (long long)bx * kBlock + tx;
        inbox = false;
        active = tb < P.n_boundary;
        idx = active ? (long long)P.boundary[tb] : 0;
        if constexpr (!CW) {
            pcode = P.bcode_pull[active ? tb : 0];
            scode = P.bcode_st[active ? tb : 0];
        }
        x = (int)(idx % P.nx);
        y = (int)((idx / P.nx) % P.ny);
        z = (int)(idx / ((long long)P.nx * P.ny));
    }
    const long long sy = P.nx, sz = (long long)P.nx * P.ny;
    double acc[kNDiag];
    if constexpr (DIAG) diag_identity(acc);

    // 2-D interior kernel: T, Y_k and rho of the block's 64 x 4 cells and a
    // 2-cell halo staged once in LDS (field-major planes of 68 x 8 points);
    // every finite-difference point is then an LDS read at a fixed offset.
    // Halo points outside the box hold the nearest in-box point's values and
    // are never read: only interior cells, whose stencils stay inside the
    // box, read the tile.
    constexpr int kTX = 64, kTY = 4, kHX = kTX + 4, kHY = kTY + 4, kNP = kHX * kHY;
    constexpr bool TILE = FAST && D == 2;
    __shared__ C tile[TILE ? (NSP + 2) * kNP : 1];
    C g[Q];
    if constexpr (TILE) {
        // the cell's pull loads go out first, so that their latency overlaps
        // the staging of the tile
        if (active)
            sfor<0, Q>([&](auto I) {
                constexpr int i = decltype(I)::value;
                g[i] = pop_load<Q, PREC, i>(P.pop_in, P.N, idx - (L::cx(i) + sy * L::cy(i)));
            });
        // staging: every thread loads its (at most three) halo points at
        // addresses clamped into the box before storing any, so that all the
        // loads are in flight together (clamped points are never read)
        const int tid = tx + kTX * ty;
        const int gx0 = bx * kTX - 2, gy0 = by * kTY - 2;
        constexpr int kRounds = (kNP + kBlock - 1) / kBlock;
        Pt<NSP, C> pt[kRounds];
#pragma unroll
        for (int r = 0; r < kRounds; ++r) {
            const int i = tid + r * kBlock;
            const int gx = min(max(gx0 + i % kHX, 0), P.nx - 1), gy = min(max(gy0 + i / kHX, 0), P.ny - 1);
            load_point<NSP, PREC>(P, (long long)gy * P.nx + gx, pt[r]);
        }
#pragma unroll
        for (int r = 0; r < kRounds; ++r) {
            const int i = tid + r * kBlock;
            if (i < kNP) {
                tile[i] = pt[r].T;
                tile[kNP + i] = pt[r].rho;
#pragma unroll
                for (int k = 0; k < NSP; ++k) tile[(2 + k) * kNP + i] = pt[r].Y[k];
            }
        }
        __syncthreads();
    }
    auto tile_point = [&](int dx, int dy, Pt<NSP, C> &o) {
        const int i = (ty + 2 + dy) * kHX + tx + 2 + dx;
        o.T = tile[i];
        o.rho = tile[kNP + i];
#pragma unroll
        for (int k = 0; k < NSP; ++k) o.Y[k] = tile[(2 + k) * kNP + i];
    };

    if (active) {
        // streaming with boundary conditions (pull; already issued for tiles)
        if constexpr (!TILE)
            sfor<0, Q>([&](auto I) {
                constexpr int i = decltype(I)::value;
                if constexpr (FAST)
                    g[i] = pop_load<Q, PREC, i>(P.pop_in, P.N, idx - (L::cx(i) + sy * L::cy(i) + sz * L::cz(i)));
                else
                    g[i] = desc_pull<Q, PREC, i, CW>(P, tb, P.n_boundary, idx, x, y, z, pcode);
            });
        Pt<NSP, C> ctr;
        if constexpr (TILE)
            tile_point(0, 0, ctr);
        else
            load_point<NSP, PREC>(P, idx, ctr);
        const C rho = ctr.rho;

        // moments: sum g and sum c g (Eq. 13)
        C sg = 0, m[3] = {0, 0, 0};
        sfor<0, Q>([&](auto I) {
            constexpr int i = decltype(I)::value;
            sg += g[i];
            if constexpr (L::cx(i) == 1) m[0] += g[i];
            if constexpr (L::cx(i) == -1) m[0] -= g[i];
            if constexpr (L::cy(i) == 1) m[1] += g[i];
            if constexpr (L::cy(i) == -1) m[1] -= g[i];
            if constexpr (L::cz(i) == 1) m[2] += g[i];
            if constexpr (L::cz(i) == -1) m[2] -= g[i];
        });
        const C inv_rho = rcp(rho);
        const C inv_rc = (C)3 * inv_rho;  // 1 / (rho cs^2)
        const C u[3] = {m[0] * inv_rc, m[1] * inv_rc, m[2] * inv_rc};

        // finite differences per axis with ghost nodes (Sec. II.D, III.B);
        // one axis at a time, one scalar at a time, to bound register use
        C diffT = 0, CT = 0, grad[3] = {0, 0, 0};
        C diffY[NSP], CY[NSP];
#pragma unroll
        for (int k = 0; k < NSP; ++k) diffY[k] = CY[k] = 0;
        double wallq = 0.0;
        // mixture-averaged transport (Sec. II.A, Eq. 2 and Eq. 7): the cell's
        // 1/W, c_p and their reciprocals; div V_c summed over the axes
        C Mc = 0, cpc = 0, divVc = 0;
        if constexpr (LE) {
#pragma unroll
            for (int k = 0; k < NSP; ++k) {
                Mc += ctr.Y[k] * (C)P.invW[k];
                cpc += ctr.Y[k] * (C)P.cpk[k];
            }
        }
        const C inv_M = LE ? rcp(Mc) : (C)0, inv_cp = LE ? rcp(cpc) : (C)0;
        auto axis_terms = [&](auto &&val, const C (&r5)[5], bool near, C ud) -> C {
            // val(f, m): field f (0 = T, 2 + k = Y_k) at offset m = -2..2
            const C d1r = d1(r5[0], r5[1], r5[2], r5[3], r5[4]);
            const C uh = (C)0.5 * ud;  // the conv2 values are twice the derivatives
            C t1, t2;
            {
                C tc;
                axis5(val(0, -2), val(0, -1), ctr.T, val(0, 1), val(0, 2), ud, near, t1, t2, tc);
                if constexpr (!LE) diffT += t2 + d1r * t1 * inv_rho;
                CT += uh * tc;
            }
            C cY[NSP], sumc = 0, y1[NSP], y2[NSP];
#pragma unroll
            for (int k = 0; k < NSP; ++k) {
                axis5(val(2 + k, -2), val(2 + k, -1), ctr.Y[k], val(2 + k, 1), val(2 + k, 2), ud, near, y1[k], y2[k],
                      cY[k]);
                if constexpr (!LE) diffY[k] += y2[k] + d1r * y1[k] * inv_rho;
                sumc += cY[k];
            }
            if constexpr (LE) {
                // along this axis, in units of alpha: d ln W = l1, d2 ln W = l2
                // (from 1/W = sum Y_k / W_k, linear in Y_k), G_k = (W_k/W) dX_k
                // = dY_k + Y_k l1, V_c = sum D_k G_k, and sum_k c_pk Y_k V_k
                C M1 = 0, M2 = 0, cp1 = 0;
#pragma unroll
                for (int k = 0; k < NSP; ++k) {
                    M1 += y1[k] * (C)P.invW[k];
                    M2 += y2[k] * (C)P.invW[k];
                    cp1 += y1[k] * (C)P.cpk[k];
                }
                const C l1 = -M1 * inv_M;
                const C l2 = l1 * l1 - M2 * inv_M;
                const C rr = d1r * inv_rho;
                C Vc = 0, H = 0;
#pragma unroll
                for (int k = 0; k < NSP; ++k) {
                    const C Dk = (C)P.dk[k];
                    const C G = y1[k] + ctr.Y[k] * l1;
                    const C dG = y2[k] + y1[k] * l1 + ctr.Y[k] * l2;
                    diffY[k] += Dk * (dG + rr * G);
                    Vc += Dk * G;
                    divVc += Dk * dG;
                    H -= (C)P.cpk[k] * Dk * G;
                }
                H += cpc * Vc;
#pragma unroll
                for (int k = 0; k < NSP; ++k) diffY[k] -= Vc * (y1[k] + ctr.Y[k] * rr);
                diffT += t2 + (rr + cp1 * inv_cp) * t1 - H * inv_cp * t1;
            }
            // mass-conserving correction of the convection (Eq. 26)
#pragma unroll
            for (int k = 0; k < NSP; ++k) CY[k] += uh * (cY[k] - ctr.Y[k] * sumc);
            return d1r;
        };
#pragma unroll 1
        for (int d = 0; d < D; ++d) {
            const C ud = d == 0 ? u[0] : d == 1 ? u[1] : u[2];
            C d1r;
            if constexpr (TILE) {
                const int ic = (ty + 2) * kHX + tx + 2;
                const int sd = d == 0 ? 1 : kHX;
                C r5[5];
#pragma unroll
                for (int m = 0; m < 5; ++m) r5[m] = tile[kNP + ic + (m - 2) * sd];
                d1r = axis_terms([&](int f, int m) -> C { return tile[f * kNP + ic + m * sd]; }, r5, false, ud);
            } else if constexpr (FAST) {
                // the four points' T and Y, read once for their densities and
                // kept for the finite differences
                const long long sd = d == 0 ? 1 : d == 1 ? sy : sz;
                Pt<NSP, C> pv[4];
                C r5[5];
                r5[2] = rho;
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    load_point<NSP, PREC>(P, idx + (j < 2 ? j - 2 : j - 1) * sd, pv[j]);
                    r5[j < 2 ? j : j + 1] = pv[j].rho;
                }
                d1r = axis_terms(
                    [&](int f, int m) -> C {
                        const int j = m < 0 ? m + 2 : m + 1;
                        return f == 0 ? pv[j].T : pv[j].Y[f - 2];
                    },
                    r5, false, ud);
            } else if constexpr (D == 2) {
                // boundary cell (2-D): whole stencil points from the descriptors
                Pt<NSP, C> st[5];
                bool near = false;
                desc_stencil<NSP, PREC, DIAG, CW>(P, tb, P.n_boundary, d, ctr, st, near, wallq);
                C r5[5] = {st[0].rho, st[1].rho, st[2].rho, st[3].rho, st[4].rho};
                d1r = axis_terms(
                    [&](int f, int m) -> C { return f == 0 ? st[m + 2].T : st[m + 2].Y[f - 2]; }, r5, near, ud);
            } else {
                // boundary cell (3-D): per offset m = -2, -1, 1, 2 the descriptor
                // gives the point holding the value (or the ghost's image)
                // and the kind of the wall behind a ghost (Sec. III.B)
                // (or the listed image point of a curved wall)
                const long long nbd = P.n_boundary;
                int pts[4], wks[4], lis[4];
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    if constexpr (CW) {
                        pts[j] = P.bpt[(d * 4 + j) * nbd + tb];
                        wks[j] = P.bwk[(d * 4 + j) * nbd + tb];
                        lis[j] = P.bimg != nullptr ? P.bimg[(d * 4 + j) * nbd + tb] : -1;
                    } else {
                        pts[j] = (int)decode_point(scode, d, j, idx, x, y, z, P.nx, P.ny, P.nz);
                        wks[j] = decode_kind(scode, d, j);
                        lis[j] = -1;
                    }
                }
                // the wall temperature behind an isothermal ghost at slot j
                auto wall_temp = [&](int j) -> double {
                    if constexpr (CW)
                        return P.btw[(d * 4 + j) * nbd + tb];
                    else
                        return decode_wall_T(scode, d, j, x, y, z, P.nx, P.ny, P.nz, P.periodic_bits, P.face_Td,
                                             P.wall_T);
                };
                const bool near = (wks[0] | wks[1] | wks[2] | wks[3]) != kFluid;
                C r5[5];
                r5[2] = rho;
                Pt<NSP, C> pv[4];  // the points' (or images') values, kept for the differences
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    const int slot = j < 2 ? j : j + 1;
                    Pt<NSP, C> &pt = pv[j];
                    if (CW && lis[j] >= 0)
                        image_value<NSP>(P, lis[j], pt);
                    else
                        load_point<NSP, PREC>(P, pts[j], pt);
                    r5[slot] = pt.rho;
                    if (wks[j] == kIso) {
                        const C Tw = (C)wall_temp(j);
                        r5[slot] = (C)2 * density<NSP>(P, Tw, pt.Y) - pt.rho;
                        if constexpr (DIAG) {
                            if (j == 1 || j == 2)
                                wallq += 2.0 * P.alpha * (double)density<NSP>(P, Tw, ctr.Y) *
                                         ((double)ctr.T - (double)Tw);
                        }
                    } else if (wks[j] == kInflow) {
                        r5[slot] = (C)2 * (C)P.rho_in - pt.rho;
                    }
                }
                d1r = axis_terms(
                    [&](int f, int m) -> C {
                        const int j = m < 0 ? m + 2 : m + 1;
                        const C v = f == 0 ? pv[j].T : pv[j].Y[f - 2];
                        if (wks[j] == kFluid) return v;
                        if (f == 0) {
                            if (wks[j] == kIso) return (C)2 * (C)wall_temp(j) - v;
                            if (wks[j] == kInflow) return (C)2 * (C)P.T_in - v;
                            return v;
                        }
                        if (wks[j] == kInflow) return (C)2 * (C)P.Y_in[f - 2] - v;
                        return v;
                    },
                    r5, near, ud);
            }
            grad[0] = d == 0 ? d1r : grad[0];
            grad[1] = d == 1 ? d1r : grad[1];
            grad[2] = d == 2 ? d1r : grad[2];
        }
        if constexpr (LE) {
#pragma unroll
            for (int k = 0; k < NSP; ++k) diffY[k] -= ctr.Y[k] * divVc;
        }
        const C alpha = (C)P.alpha;
        diffT *= alpha;
#pragma unroll
        for (int k = 0; k < NSP; ++k) diffY[k] *= alpha;

        finish_cell<Q, NSP, PREC, MODE, LE>(P, idx, g, ctr, u, m, sg, inv_rc, diffT, diffY, CT, CY, grad, wallq, acc);
        if constexpr (MODE != kModeFields) {
            if constexpr (!FAST && D == 2) {
                // outlet (Eq. 32): g_i(r) <- g_i(r-n)(cs - u.n) + g_i(r)(1 - cs + u.n)
                // for the populations entering through the face, with the
                // post-streaming values and velocity of this level
#pragma unroll
                for (int f = 0; f < 2; ++f) {
                    if (P.face[f] != LBFD_FACE_OUTFLOW || x != (f ? P.nx - 1 : 0)) continue;
                    const int sign = f ? 1 : -1;
                    Nb in = classify(P, x - sign, y, z);
                    if (in.kind != kFluid) continue;
                    const C cs = (C)0.57735026918962576451;
                    const C un = (C)sign * u[0];
                    sfor<0, Q>([&](auto I) {
                        constexpr int i = decltype(I)::value;
                        if constexpr (L::cx(i) != 0) {
                            if (L::cx(i) == -sign) {
                                Nb s = classify(P, x - L::cx(i), y - L::cy(i), z - L::cz(i));
                                if (s.kind == kOutflow && s.face == f) {
                                    C G = gather<Q, PREC, i>(P, x - sign, y, z, in.idx);
                                    P.outlet[outlet_index(P, f, i, Q, y, z)] =
                                        (double)(G * (cs - un) + g[i] * ((C)1 - cs + un));
                                }
                            }
                        }
                    });
                }
            } else if constexpr (!FAST) {
                // 3-D: outlet cells hand their outward normal velocity to
                // outlet_kernel, which applies the same update (keeps the
                // nine extra gathers out of this kernel's registers)
#pragma unroll
                for (int f = 0; f < 2; ++f)
                    if (P.face[f] == LBFD_FACE_OUTFLOW && x == (f ? P.nx - 1 : 0))
                        P.outlet_un[(long long)f * P.ny * P.nz + (long long)z * P.ny + y] =
                            (double)(f ? u[0] : -u[0]);
            }
        }
    } else if constexpr (MODE == kModeFields && FAST) {
        if (inbox && P.code[idx] == kCodeSolid)
#pragma unroll
            for (int c = 0; c < 5; ++c) P.fields[c * P.N + idx] = 0.0;
    }

    if constexpr (DIAG) block_reduce_diag(acc, P.partials + slot * kNDiag);
}

// Minimum waves per SIMD asked of the register allocator for a step
// kernel (measured on MI355X).  2-D with up to 4 species: three waves
// (168 VGPRs) in FP64 and four (128) in the mixed forms -- the boundary
// path, which needs more, spills instead of lowering the tiles' occupancy.
// 3-D FP64: two waves (256 VGPRs) for boundary cells with up to 4 species
// and for both parts with 9 species (spills of 132 and 208 bytes per lane;
// the 9-species interior tiles 3 % and boundary cells 13 % faster than at
// the free allocator's one wave).  Otherwise the allocator is left free
// (1): for the launches with diagnostics or fields (MODE != kModeStep),
// which run once per check or read, and for the curved-wall and
// mixture-transport instantiations (CW, LE).  The 2-D FP64 fields launch
// with curved walls and mixture-averaged transport once returned wrong
// velocities at the three-wave budget (spilling) and exact ones without it;
// the assembly check of the build finds no one-sided copy in it, so the
// budget stays off on those paths.
template <int Q, int NSP, int PREC, int PART, int MODE = kModeStep, bool CWLE = false> struct StepWaves {
    static constexpr int value = (MODE != kModeStep || CWLE)                               ? 1
                                 : (Q == 9 && NSP <= 4)                                     ? (PREC == LBFD_FP64 ? 3 : 4)
                                 : (Q == 27 && NSP <= 4 && PART == 2 && PREC == LBFD_FP64) ? 2
                                 : (Q == 27 && NSP == 9 && PREC == LBFD_FP64)              ? 2
                                                                                           : 1;
};

// The step over the block range [block_begin, block_begin + gridDim.x) of
// the list (boundary blocks, then interior tiles).  PART 0: one launch
// covers both kinds -- boundary blocks first, so that their long dependent
// chains of descriptor and neighbour loads start with the launch and the
// interior tiles fill the remaining wave slots (D2Q9).  PART 2 / PART 1:
// boundary blocks / interior tiles only, two launches in stream order
// (D3Q27, where one kernel holding both paths slows the interior tiles).
// Consecutive blocks go to the 8 XCDs in turn, so the interior tiles are
// renumbered to give each XCD one contiguous band of the box;
// boundary_blocks is a multiple of 8, which keeps the XCD of a tile block
// equal to its index modulo 8.
template <int Q, int NSP, int PREC, int MODE, int PART, bool CW = false, bool LE = false>
__global__ void __launch_bounds__(kBlock)
__attribute__((amdgpu_waves_per_eu(StepWaves<Q, NSP, PREC, PART, MODE, CW || LE>::value))) step_kernel(const KParams P)
{
    using TS = TileShape<Lat<Q>::D>;
    const long long b = (long long)blockIdx.x + P.block_begin;
    if constexpr (PART != 1) {
        if (b < P.boundary_blocks) {
            step_block<Q, NSP, PREC, MODE, false, CW, LE>(P, (int)b, 0, 0, (int)threadIdx.x, 0, 0,
                                                  P.interior_blocks + b);
            return;
        }
    }
    if constexpr (PART != 2) {
        const long long t = b - P.boundary_blocks;
        const long long n = P.interior_blocks, q = n >> 3;
        const int xcd = (int)(t & 7), r = (int)(n & 7);
        const long long tile = xcd * q + (xcd < r ? xcd : r) + (t >> 3);
        const int bx = (int)(tile % P.tiles_x);
        const int by = (int)((tile / P.tiles_x) % P.tiles_y);
        const int bz = (int)(tile / ((long long)P.tiles_x * P.tiles_y));
        const int tx = (int)threadIdx.x % TS::X;
        const int ty = ((int)threadIdx.x / TS::X) % TS::Y;
        const int tz = (int)threadIdx.x / (TS::X * TS::Y);
        step_block<Q, NSP, PREC, MODE, true, false, LE>(P, bx, by, bz, tx, ty, tz, tile);
    }
}

// ------------------------------------------------------------ image points
// Shepard reconstruction at the image points of curved-wall ghost nodes
// (Sec. III.B) for the current level: T, rho, Y_k averaged over the listed
// fluid nodes within four cells with the normalised inverse-square-distance
// weights -- a sparse matrix-vector product, one row per image point.  The
// distinct nodes of all rows (the support) are first packed, once each, into
// records of (T, rho, Y_k) (support_kernel), so that a row entry is one
// contiguous record read rather than 1 + N_sp scattered loads and a density
// evaluation.  LPP lanes share a row (chosen at set-up from the mean row
// length), stride over its entries and combine their sums with a butterfly
// inside the group; the result is written before the step launches read it.
template <int NSP, int PREC>
__global__ void __launch_bounds__(kBlock) support_kernel(const KParams P)
{
    using C = typename Prec<PREC>::calc;
    const long long s = (long long)blockIdx.x * kBlock + threadIdx.x;
    if (s >= P.n_sup) return;
    Pt<NSP, C> pt;
    load_point<NSP, PREC>(P, P.sup_idx[s], pt);
    double *rec = P.sup_val + s * (2 + NSP);
    rec[0] = (double)pt.T;
    rec[1] = (double)pt.rho;
#pragma unroll
    for (int k = 0; k < NSP; ++k) rec[2 + k] = (double)pt.Y[k];
}

template <int NSP, int PREC, int LPP>
__global__ void __launch_bounds__(kBlock) image_kernel(const KParams P)
{
    using C = typename Prec<PREC>::calc;
    const long long k = ((long long)blockIdx.x * kBlock + threadIdx.x) / LPP;
    const int lane = (int)threadIdx.x % LPP;
    const bool live = k < P.n_img;  // every lane stays for the butterfly
    const int2 r = live ? P.img_rng[k] : make_int2(0, 0);
    C acc[2 + NSP];
#pragma unroll
    for (int f = 0; f < 2 + NSP; ++f) acc[f] = 0;
#pragma unroll 2
    for (int e = r.x + lane; e < r.x + r.y; e += LPP) {
        const double *rec = P.sup_val + (long long)P.img_idx[e] * (2 + NSP);
        const C w = (C)P.img_w[e];
#pragma unroll
        for (int f = 0; f < 2 + NSP; ++f) acc[f] += w * (C)rec[f];
    }
#pragma unroll
    for (int f = 0; f < 2 + NSP; ++f) {
        C v = acc[f];
#pragma unroll
        for (int o = LPP / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
        if (live && lane == 0) P.img_val[(size_t)f * P.n_img + k] = (double)v;
    }
}

template <int NSP, int PREC>
hipError_t launch_images(const KParams &kp, hipStream_t s)
{
    support_kernel<NSP, PREC><<<dim3((unsigned)((kp.n_sup + kBlock - 1) / kBlock)), dim3(kBlock), 0, s>>>(kp);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int lpp = kp.img_lpp;
    const unsigned nb = (unsigned)((kp.n_img * lpp + kBlock - 1) / kBlock);
    if (lpp == 16)
        image_kernel<NSP, PREC, 16><<<dim3(nb), dim3(kBlock), 0, s>>>(kp);
    else if (lpp == 32)
        image_kernel<NSP, PREC, 32><<<dim3(nb), dim3(kBlock), 0, s>>>(kp);
    else
        image_kernel<NSP, PREC, 64><<<dim3(nb), dim3(kBlock), 0, s>>>(kp);
    return hipGetLastError();
}

// ------------------------------------------------------------ chemistry launch
// Mechanisms of many species (chem_pass): the FP64 Arrhenius source of every
// fluid cell as a launch of its own ahead of the step, one thread per fluid
// cell, written into this step's output scalars (the slots of T and Y_k),
// where the cell's step thread reads it back before overwriting them with
// the cell's new state.  The sub-stepped source then runs at the occupancy
// of its own registers, not of the step's populations and stencils; the
// exponential's table is staged in LDS.  In the mixed forms the stored
// source is rounded to single precision, as the step kernel rounds it when
// it adds it.
//
// A wave takes as long as its lane with the most sub-steps, and the counts
// are bimodal (cold gas 1, burning gas up to the cap), so the cells are
// ordered first (chem_order_kernel): those whose previous source took at
// most kChemLight sub-steps from the front of chem_order, the others from
// the back, runs of the fluid-cell list kept in list order within a wave.
// The previous step's count only decides where a cell goes; every cell's
// source is computed alike wherever it lands, so the results do not depend
// on the order (which the atomics make vary from run to run).
constexpr int kChemChunk = 16;  // fluid-list positions per thread of the ordering

template <int NSP>
__global__ void __launch_bounds__(kBlock) chem_order_kernel(const KParams P)
{
    __shared__ int cnt[2], base[2];
    if (threadIdx.x < 2) cnt[threadIdx.x] = 0;
    __syncthreads();
    const long long n = P.n_fluid;
    const long long t0 = (long long)blockIdx.x * kBlock * kChemChunk;
    const int lane = (int)(threadIdx.x & 63);
    const unsigned long long below = (1ull << lane) - 1ull;
    // this block's light and heavy cells
    int nh = 0, nl = 0;
    for (int r = 0; r < kChemChunk; ++r) {
        const long long t = t0 + (long long)r * kBlock + threadIdx.x;
        if (t < n) {
            const bool h = P.chem_heavy[P.fluid[t]] != 0;
            nh += h;
            nl += !h;
        }
    }
    atomicAdd(&cnt[0], nl);
    atomicAdd(&cnt[1], nh);
    __syncthreads();
    if (threadIdx.x == 0) {
        base[0] = atomicAdd(&P.chem_count[0], cnt[0]);
        base[1] = atomicAdd(&P.chem_count[1], cnt[1]);
        cnt[0] = cnt[1] = 0;
    }
    __syncthreads();
    // places: per round and wave one run per class, in list order
    for (int r = 0; r < kChemChunk; ++r) {
        const long long t = t0 + (long long)r * kBlock + threadIdx.x;
        const bool valid = t < n;
        const int idx = valid ? P.fluid[t] : 0;
        const bool h = valid && P.chem_heavy[idx] != 0;
        const bool l = valid && !h;
        const unsigned long long bh = __ballot(h), bl = __ballot(l);
        int wh = 0, wl = 0;
        if (lane == 0) {
            wh = atomicAdd(&cnt[1], __popcll(bh));
            wl = atomicAdd(&cnt[0], __popcll(bl));
        }
        wh = __shfl(wh, 0, 64);
        wl = __shfl(wl, 0, 64);
        // (the counts of both passes agree, so every place is in [0, n))
        const long long ph = n - 1 - (base[1] + wh + __popcll(bh & below));
        const long long pl = base[0] + wl + __popcll(bl & below);
        if (h && ph >= 0) P.chem_order[ph] = idx;
        if (l && pl < n) P.chem_order[pl] = idx;
    }
}

// The ordering's two counters, cleared ahead of it (a kernel, so that a
// captured step records no memset node).
template <int NSP>
__global__ void chem_count_clear_kernel(int *count)
{
    if (threadIdx.x < 2) count[threadIdx.x] = 0;
}

template <int NSP, int PREC, bool LE, int NR>
__global__ void __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(4))) chem_kernel(const KParams P)
{
    using S = typename Prec<PREC>::scal;
    __shared__ double tab[kExpTabN], ltab[2 * kLogTabN];
    for (int i = (int)threadIdx.x; i < kExpTabN; i += (int)blockDim.x) tab[i] = kExp2Tab[i];
    for (int i = (int)threadIdx.x; i < 2 * kLogTabN; i += (int)blockDim.x) ltab[i] = kLogTab[i];
    __syncthreads();
    const long long t = (long long)blockIdx.x * kBlock + threadIdx.x;
    if (t >= P.n_fluid) return;
    const long long idx = P.chem_order[t];
    const char *si = (const char *)P.sc_in;
    char *so = (char *)P.sc_out;
    const size_t fstride = (size_t)P.N * sizeof(S);
    const uint32_t off = (uint32_t)idx * (uint32_t)sizeof(S);
    double Y[NSP], srcT, srcY[NSP];
    const double T = (double)ldo<S>(si, off);
#pragma unroll
    for (int k = 0; k < NSP; ++k) Y[k] = (double)ldo<S>(si + (size_t)(1 + k) * fstride, off);
    const int nsub = chemistry<NSP, LE, NR>(P, tab, ltab, T, Y, srcT, srcY);
    P.chem_heavy[idx] = nsub > kChemLight;
    sto<S>(so, off, (S)srcT);
#pragma unroll
    for (int k = 0; k < NSP; ++k) sto<S>(so + (size_t)(1 + k) * fstride, off, (S)srcY[k]);
}

template <int NSP, int PREC>
hipError_t launch_chem(const KParams &kp, hipStream_t s)
{
    const unsigned nb = (unsigned)((kp.n_fluid + kBlock - 1) / kBlock);
    if (nb == 0) return hipSuccess;
    const long long per = (long long)kBlock * kChemChunk;
    chem_count_clear_kernel<NSP><<<dim3(1), dim3(64), 0, s>>>(kp.chem_count);
    chem_order_kernel<NSP><<<dim3((unsigned)((kp.n_fluid + per - 1) / per)), dim3(kBlock), 0, s>>>(kp);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    // the kernel specialised to the mechanism's structure when one was
    // compiled for this context (unity-Lewis transport)
    if (kp.chem_jit != nullptr && kp.transport != LBFD_MIXTURE_AVERAGED)
        return launch_chem_jit(kp, nb, sizeof(typename Prec<PREC>::scal), s);
    // mechanisms of at most two reactants per reaction skip the two
    // constant-1 slots
    const bool two = kp.chem_nreact <= 2;
    if (kp.transport == LBFD_MIXTURE_AVERAGED) {
        if (two)
            chem_kernel<NSP, PREC, true, 2><<<dim3(nb), dim3(kBlock), 0, s>>>(kp);
        else
            chem_kernel<NSP, PREC, true, 4><<<dim3(nb), dim3(kBlock), 0, s>>>(kp);
    } else {
        if (two)
            chem_kernel<NSP, PREC, false, 2><<<dim3(nb), dim3(kBlock), 0, s>>>(kp);
        else
            chem_kernel<NSP, PREC, false, 4><<<dim3(nb), dim3(kBlock), 0, s>>>(kp);
    }
    return hipGetLastError();
}

// ------------------------------------------------------------ outlet
// Outlet (Eq. 32): for every fluid cell of an outflow face whose inner
// neighbour is fluid, the populations entering through the face become
// g_i(r) <- g_i(r-n)(cs - u.n) + g_i(r)(1 - cs + u.n), with the
// post-streaming values g_i(r) (the outlet buffer, read by this step) and
// g_i(r-n) (pulled again from the buffer this step read), and u.n of this
// level (written by the boundary blocks).  Runs after them; used for D3Q27
// (D2Q9 applies the update in the boundary blocks).
template <int Q, int PREC>
__global__ void __launch_bounds__(kBlock) outlet_kernel(const KParams P)
{
    using L = Lat<Q>;
    using C = typename Prec<PREC>::calc;
    const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const long long nf = (long long)P.ny * P.nz;
    if (t >= 2 * nf) return;
    const int f = (int)(t / nf);
    const int y = (int)((t % nf) % P.ny), z = (int)((t % nf) / P.ny);
    if (P.face[f] != LBFD_FACE_OUTFLOW) return;
    const int x = f ? P.nx - 1 : 0, sign = f ? 1 : -1;
    const long long idx = ((long long)z * P.ny + y) * P.nx + x;
    if (P.mask[idx] != LBFD_FLUID) return;
    const Nb in = classify(P, x - sign, y, z);
    if (in.kind != kFluid) return;
    const C cs = (C)0.57735026918962576451;
    const C un = (C)P.outlet_un[t];
    sfor<0, Q>([&](auto I) {
        constexpr int i = decltype(I)::value;
        if constexpr (L::cx(i) != 0) {
            if (L::cx(i) == -sign) {
                const Nb s = classify(P, x - L::cx(i), y - L::cy(i), z - L::cz(i));
                if (s.kind == kOutflow && s.face == f) {
                    const C G = gather<Q, PREC, i>(P, x - sign, y, z, in.idx);
                    double &S = P.outlet[outlet_index(P, f, i, Q, y, z)];
                    S = (double)(G * (cs - un) + (C)S * ((C)1 - cs + un));
                }
            }
        }
    });
}

// ------------------------------------------------------------ init kernel
// g^0 = w (P_h0 - rho cs^2) + cs^2 f^eq(rho, u0) (Eq. 12), scattered into
// the post-collision buffer so that the first gather returns it (inverse
// of the pull, the inlet and the bounce-back rules); populations entering
// through an outlet are written to the outlet buffer.
template <int Q, int NSP, int PREC>
__global__ void __launch_bounds__(kBlock) init_kernel(const KParams P, const double *u0, const double *Ph0)
{
    using L = Lat<Q>;
    using S = typename Prec<PREC>::scal;
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    const int y = blockIdx.y * blockDim.y + threadIdx.y;
    const int z = blockIdx.z * blockDim.z + threadIdx.z;
    if (x >= P.nx || y >= P.ny || z >= P.nz) return;
    const long long idx = ((long long)z * P.ny + y) * P.nx + x;
    if (P.mask[idx] != LBFD_FLUID) return;
    const S *sc = (const S *)P.sc_in;
    double T = (double)sc[idx], Y[NSP];
#pragma unroll
    for (int k = 0; k < NSP; ++k) Y[k] = (double)sc[(1 + k) * P.N + idx];
    const double rho = density<NSP>(P, T, Y);
    double u[3] = {0.0, 0.0, 0.0};
    if (u0)
        for (int d = 0; d < L::D; ++d) u[d] = u0[d * P.N + idx];
    const double ph = Ph0 ? Ph0[idx] : 0.0;
    const double uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
    sfor<0, Q>([&](auto I) {
        constexpr int i = decltype(I)::value;
        constexpr int opp = Q - 1 - i;
        const double cu = L::cx(i) * u[0] + L::cy(i) * u[1] + L::cz(i) * u[2];
        const double feq = L::w(i) * rho * (1.0 + cu / kCs2 + cu * cu / (2.0 * kCs2 * kCs2) - uu / (2.0 * kCs2));
        const double g0 = L::w(i) * (ph - rho * kCs2) + kCs2 * feq;
        using C = typename Prec<PREC>::calc;
        if constexpr (i == (Q - 1) / 2) {
            pop_store<Q, PREC, i>(P.pop_out, P.N, idx, (C)g0);
        } else {
            Nb s = classify(P, x - L::cx(i), y - L::cy(i), z - L::cz(i));
            if (s.kind == kFluid) {
                pop_store<Q, PREC, i>(P.pop_out, P.N, s.idx, (C)g0);
            } else if (s.kind == kInflow) {
                const double ci = inflow_cu<Q, i>(P, x, y, z);
                pop_store<Q, PREC, opp>(P.pop_out, P.N, idx, (C)(g0 - 2.0 * L::w(i) * P.rho_in * ci));
            } else if (s.kind == kOutflow) {
                const int sign = (s.face & 1) ? 1 : -1;
                Nb in = classify(P, x - sign, y, z);
                if (in.kind == kFluid)
                    P.outlet[outlet_index(P, s.face, i, Q, y, z)] = g0;
                else
                    pop_store<Q, PREC, opp>(P.pop_out, P.N, idx, (C)g0);
            } else {
                pop_store<Q, PREC, opp>(P.pop_out, P.N, idx, (C)g0);
            }
        }
    });
}

// ------------------------------------------------------------ launchers
// Instantiated once per configuration in inst/*.hip (explicit
// instantiation), declared extern in the dispatcher.
// One step: the boundary blocks and the interior tiles (both read level n
// and write disjoint cells of level n+1), on the context stream, then for
// D3Q27 the outlet update.
template <int Q, int NSP, int PREC, int MODE, int PART, bool LE>
hipError_t launch_range_t(const KParams &kp, long long count, hipStream_t s)
{
    if constexpr (PART != 1) {
        // boundary cells with curved-wall links or image points
        if (kp.bq != nullptr || kp.bimg != nullptr) {
            step_kernel<Q, NSP, PREC, MODE, PART, true, LE><<<dim3((unsigned)count), dim3(kBlock), 0, s>>>(kp);
            return hipGetLastError();
        }
    }
    step_kernel<Q, NSP, PREC, MODE, PART, false, LE><<<dim3((unsigned)count), dim3(kBlock), 0, s>>>(kp);
    return hipGetLastError();
}

template <int Q, int NSP, int PREC, int MODE, int PART>
hipError_t launch_range(const KParams &kp0, long long begin, long long count, hipStream_t s)
{
    if (count <= 0) return hipSuccess;
    KParams kp = kp0;
    kp.block_begin = begin;
    // the mixture-averaged transport is a separate instantiation, so that
    // unity-Lewis steps keep their registers
    if (kp.transport == LBFD_MIXTURE_AVERAGED) return launch_range_t<Q, NSP, PREC, MODE, PART, true>(kp, count, s);
    return launch_range_t<Q, NSP, PREC, MODE, PART, false>(kp, count, s);
}

template <int Q, int NSP, int PREC, int MODE>
hipError_t launch_pair(const KParams &kp, const Streams &st)
{
    // st.part 0: every launch; 1: interior tiles only; 2: boundary blocks,
    // image points and outlet; 3: the chemistry launch only
    const long long nbb = kp.boundary_blocks, nti = kp.interior_blocks;
    hipError_t e = hipSuccess;
    if constexpr (chem_pass(NSP)) {
        if ((st.part == 0 || st.part == 3) && (e = launch_chem<NSP, PREC>(kp, st.main)) != hipSuccess)
            return e;
    }
    if (st.part == 3) return hipSuccess;
    if (kp.bimg != nullptr && kp.n_img > 0 && st.part != 1)
        if ((e = launch_images<NSP, PREC>(kp, st.main)) != hipSuccess) return e;
    if constexpr (fused_step(Q)) {
        const long long begin = st.part == 1 ? nbb : 0;
        const long long count = st.part == 1 ? nti : st.part == 2 ? nbb : nbb + nti;
        if ((e = launch_range<Q, NSP, PREC, MODE, 0>(kp, begin, count, st.main)) != hipSuccess) return e;
    } else {
        if (st.part != 1 && (e = launch_range<Q, NSP, PREC, MODE, 2>(kp, 0, nbb, st.main)) != hipSuccess)
            return e;
        if (st.part != 2 && (e = launch_range<Q, NSP, PREC, MODE, 1>(kp, nbb, nti, st.main)) != hipSuccess)
            return e;
    }
    if (Lat<Q>::D == 3 && MODE != kModeFields && st.part != 1 && kp.n_boundary > 0 &&
        (kp.face[0] == LBFD_FACE_OUTFLOW || kp.face[1] == LBFD_FACE_OUTFLOW)) {
        const unsigned no = (unsigned)((2LL * kp.ny * kp.nz + kBlock - 1) / kBlock);
        outlet_kernel<Q, PREC><<<dim3(no), dim3(kBlock), 0, st.main>>>(kp);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    return hipSuccess;
}

template <int Q, int NSP, int PREC>
hipError_t launch_step_t(int mode, const KParams &kp, const Streams &st)
{
    switch (mode) {
    case kModeStep: return launch_pair<Q, NSP, PREC, kModeStep>(kp, st);
    case kModeStepDiag: return launch_pair<Q, NSP, PREC, kModeStepDiag>(kp, st);
    default: return launch_pair<Q, NSP, PREC, kModeFields>(kp, st);
    }
}

template <int Q, int NSP, int PREC>
hipError_t launch_init_t(const KParams &kp, const double *u0, const double *Ph0, dim3 grid, dim3 block,
                         hipStream_t s)
{
    init_kernel<Q, NSP, PREC><<<grid, block, 0, s>>>(kp, u0, Ph0);
    return hipGetLastError();
}

// (lattice, species, precision) combinations built into the library
#define LBFD_FOR_CONFIGS(X) \
    X(9, 2, 0) X(9, 4, 0) X(9, 9, 0) X(27, 2, 0) X(27, 4, 0) X(27, 9, 0) \
    X(9, 2, 1) X(9, 4, 1) X(9, 9, 1) X(27, 2, 1) X(27, 4, 1) X(27, 9, 1) \
    X(9, 4, 2) X(27, 4, 2) X(27, 9, 2)

#define LBFD_INSTANTIATE(q, n, p) \
    template hipError_t launch_step_t<q, n, p>(int, const KParams &, const Streams &); \
    template hipError_t launch_init_t<q, n, p>(const KParams &, const double *, const double *, dim3, dim3, \
                                               hipStream_t);

}  // namespace lbfd
