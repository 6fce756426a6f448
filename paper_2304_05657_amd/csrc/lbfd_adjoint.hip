// lbfd_adjoint.hip -- derivatives of the FP64 coupled step.
//
// The objective is J = sum_{n = 0}^{N-1} w_n q(s^n), w_n = 1 inside the
// chosen window of levels, with q either the wall heat flux (the sum over
// fluid cells and axis sides whose first neighbour is an isothermal wall of
// 2 alpha rho(T_w, Y)(T - T_w)) or the flame position
// nx - sum_cells (T - T_u)/(T_b - T_u) nx / n_fluid, and the state s^n = (post-collision populations read by step n, T^n, Y^n).
// With s^{n+1} = F(s^n; theta), theta = (wall temperatures, A_j, Ta_j), the
// adjoint recursion is lambda^N = 0,
//   lambda^n = (dF/ds^n)^T lambda^{n+1} + (dq/ds^n)^T,
//   dJ/dtheta = sum_n (dF/dtheta)^T lambda^{n+1} + dq^n/dtheta.
// One thread per fluid cell c gathers the cell's inputs (pull sources,
// the finite-difference stencil's scalars, ghost wall temperatures; at
// interior cells plain offsets, elsewhere neighbours classified on the fly)
// and runs the cell's update forward in FP64, then backward: the reverse of
// every operation, hand-derived, from the adjoint of the cell's outputs to
// those of its inputs, in two kernels (cell_vjp_collision,
// cell_vjp_stencil).  The sub-stepped Arrhenius source is reversed sub-step
// by sub-step, each sub-step's state recomputed from the cell's (chem_vjp).
// Each pulled population is read by exactly one cell, so its adjoint is
// stored; each stencil slot's share of a scalar's adjoint is stored per slot
// and gathered by the slot's cell in a third kernel; the wall temperatures'
// adjoints are added atomically.  Steps are recomputed from checkpoints taken every K steps
// (host side, lbfd_api.hip).
//
// tangent_kernel evaluates the same update in dual numbers with a given
// tangent of every input (the Jacobian-vector product of one step); the
// identity <J dx, lambda> = <dx, J^T lambda> between the two checks the
// reverse sweep.  Both evaluate the forward step's formulas in the general
// geometry path; rate coefficients are formed as in the step's chemistry
// (A dt exp(b ln T - Ta/T) with the step's exponential).
#include <hip/hip_runtime.h>

#include <type_traits>

#include "lbfd_kernels.h"

namespace lbfd {

// ----------------------------------------------------------- dual numbers
// Value and N tangents.
template <int N>
struct DualN {
    double v;
    double d[N];
    __device__ DualN() : v(0.0)
    {
        for (int i = 0; i < N; ++i) d[i] = 0.0;
    }
    __device__ DualN(double x) : v(x)
    {
        for (int i = 0; i < N; ++i) d[i] = 0.0;
    }
    __device__ explicit operator double() const { return v; }
    __device__ DualN &operator+=(const DualN &b)
    {
        v += b.v;
        for (int i = 0; i < N; ++i) d[i] += b.d[i];
        return *this;
    }
    __device__ DualN &operator-=(const DualN &b)
    {
        v -= b.v;
        for (int i = 0; i < N; ++i) d[i] -= b.d[i];
        return *this;
    }
    __device__ DualN &operator*=(const DualN &b)
    {
        for (int i = 0; i < N; ++i) d[i] = d[i] * b.v + v * b.d[i];
        v *= b.v;
        return *this;
    }
};
using Dual = DualN<1>;

template <int N> __device__ inline DualN<N> operator+(DualN<N> a, const DualN<N> &b) { return a += b; }
template <int N> __device__ inline DualN<N> operator-(DualN<N> a, const DualN<N> &b) { return a -= b; }
template <int N> __device__ inline DualN<N> operator*(DualN<N> a, const DualN<N> &b) { return a *= b; }
template <int N> __device__ inline DualN<N> operator-(const DualN<N> &a)
{
    DualN<N> r(-a.v);
    for (int i = 0; i < N; ++i) r.d[i] = -a.d[i];
    return r;
}
// (divisions, not a reciprocal: with b.v subnormal, 1 / b.v overflows and a
// zero numerator would give 0 * inf)
template <int N> __device__ inline DualN<N> operator/(const DualN<N> &a, const DualN<N> &b)
{
    const double q = a.v / b.v;
    DualN<N> r(q);
    for (int i = 0; i < N; ++i) r.d[i] = (a.d[i] - q * b.d[i]) / b.v;
    return r;
}
// f(a) with f(a.v) = fv and f'(a.v) = fd
template <int N> __device__ inline DualN<N> chain(const DualN<N> &a, double fv, double fd)
{
    DualN<N> r(fv);
    for (int i = 0; i < N; ++i) r.d[i] = fd * a.d[i];
    return r;
}
template <int N> __device__ inline DualN<N> rcp(const DualN<N> &a)
{
    const double r = rcp(a.v);
    return chain(a, r, -r * r);
}
template <int N> __device__ inline bool operator<(const DualN<N> &a, const DualN<N> &b) { return a.v < b.v; }
template <int N> __device__ inline bool operator>(const DualN<N> &a, const DualN<N> &b) { return a.v > b.v; }
template <int N> __device__ inline bool operator>=(const DualN<N> &a, const DualN<N> &b) { return a.v >= b.v; }
template <int N> __device__ inline bool operator<=(const DualN<N> &a, const DualN<N> &b) { return a.v <= b.v; }
// the exponential of the forward chemistry (exp_tab; tab: its table, in
// LDS or constant memory)
template <int N> __device__ inline DualN<N> dexp(const DualN<N> &a, const double *tab)
{
    const double e = exp_tab(a.v, tab);
    return chain(a, e, e);
}
__device__ inline double dexp(double a, const double *tab) { return exp_tab(a, tab); }
template <int N> __device__ inline DualN<N> dlog(const DualN<N> &a) { return chain(a, log(a.v), rcp(a.v)); }
__device__ inline double dlog(double a) { return log(a); }
template <int N> __device__ inline double val(const DualN<N> &a) { return a.v; }
__device__ inline double val(double a) { return a; }

// ------------------------------------------------------------ cell inputs
// Stencil slots: 0 = the cell, 1 + 4 d + j for axis d < D and
// m = -2, -1, 1, 2 (j = 0 .. 3).
template <int Q> constexpr int n_slots() { return 1 + 4 * Lat<Q>::D; }

// A ghost's image is a fluid slot: the cell for a first neighbour; the
// cell or one of the axis's two first neighbours (slots img_lo, img_hi) for
// a second neighbour.
constexpr bool second_nb(int s) { return s > 0 && ((s - 1) % 4 == 0 || (s - 1) % 4 == 3); }
constexpr int img_lo(int s) { return second_nb(s) ? s - (s - 1) % 4 + 1 : 0; }
constexpr int img_hi(int s) { return second_nb(s) ? s - (s - 1) % 4 + 2 : 0; }

template <int Q, int NSP>
struct CellIn {
    static constexpr int S = n_slots<Q>();
    double g[Q];          // pulled populations (with the inlet correction)
    int tdir[Q], tcell[Q];  // population entry each pull read
    int cell[S];          // fluid slot: its cell; ghost slot: -1
    int kind[S];          // kFluid or the kind of the wall behind the ghost
    int img[S];           // ghost slot: slot of its image point
    double Tw[S];         // ghost slot: wall temperature
    int wall[S];          // ghost slot behind an isothermal in-box solid: its cell, else -1
};

// PULLS = false: the stencil's slots only.
template <int Q, int NSP, bool PULLS = true>
__device__ void gather_inputs(const KParams &P, int x, int y, int z, long long idx, CellIn<Q, NSP> &in)
{
    using L = Lat<Q>;
    constexpr int D = L::D;
    const double *pop = (const double *)P.pop_in;
    if (P.code[idx] == kCodeInterior) {
        // every pull source and stencil point is an in-box fluid cell
        const long long st[3] = {1, P.nx, (long long)P.nx * P.ny};
#pragma unroll
        for (int i = 0; i < (PULLS ? Q : 0); ++i) {
            in.tdir[i] = i;
            in.tcell[i] = (int)(idx - (L::cx(i) * st[0] + L::cy(i) * st[1] + L::cz(i) * st[2]));
            in.g[i] = pop[(long long)i * P.N + in.tcell[i]];
        }
#pragma unroll
        for (int s = 0; s < n_slots<Q>(); ++s) {
            const int d = s == 0 ? 0 : (s - 1) / 4, j = s == 0 ? 0 : (s - 1) % 4;
            const int mm = j == 0 ? -2 : j == 1 ? -1 : j == 2 ? 1 : 2;
            in.cell[s] = (int)(s == 0 ? idx : idx + mm * st[d]);
            in.kind[s] = kFluid;
            in.img[s] = -1;
            in.Tw[s] = 0.0;
            in.wall[s] = -1;
        }
        return;
    }
#pragma unroll
    for (int i = 0; i < (PULLS ? Q : 0); ++i) {
        const int cx = i % 3 - 1, cy = (i / 3) % 3 - 1, cz = Q == 9 ? 0 : i / 9 - 1;
        const int opp = Q - 1 - i;
        double corr = 0.0;
        if (cx == 0 && cy == 0 && cz == 0) {
            in.tdir[i] = i;
            in.tcell[i] = (int)idx;
        } else {
            const Nb s = classify(P, x - cx, y - cy, z - cz);
            const bool fl = s.kind == kFluid;
            in.tdir[i] = fl ? i : opp;
            in.tcell[i] = fl ? (int)s.idx : (int)idx;
            if (s.kind == kInflow) corr = 2.0 * L::w(i) * P.rho_in * inflow_cu_c(P, cx, cy, cz, x, y, z);
        }
        in.g[i] = pop[(long long)in.tdir[i] * P.N + in.tcell[i]] + corr;
    }
    auto load = [&](int s, long long c) {
        in.cell[s] = (int)c;
        in.kind[s] = kFluid;
        in.img[s] = -1;
        in.Tw[s] = 0.0;
        in.wall[s] = -1;
    };
    auto ghost_slot = [&](int s, const Nb &w, int image) {
        in.cell[s] = -1;
        in.kind[s] = w.kind;
        in.img[s] = image;
        in.Tw[s] = w.Tw;
        in.wall[s] = (w.kind == kIso && w.face < 0) ? (int)w.idx : -1;
    };
    load(0, idx);
#pragma unroll
    for (int d = 0; d < D; ++d) {
#pragma unroll
        for (int sg = -1; sg <= 1; sg += 2) {
            const int j1 = sg < 0 ? 1 : 2, j2 = sg < 0 ? 0 : 3;
            const int s1 = 1 + 4 * d + j1, s2 = 1 + 4 * d + j2, sm = 1 + 4 * d + (sg < 0 ? 2 : 1);
            const int ox = d == 0, oy = d == 1, oz = d == 2;
            const Nb c1 = classify(P, x + sg * ox, y + sg * oy, z + sg * oz);
            if (c1.kind != kFluid) {
                const Nb cm = classify(P, x - sg * ox, y - sg * oy, z - sg * oz);
                ghost_slot(s1, c1, 0);
                ghost_slot(s2, c1, cm.kind == kFluid ? sm : 0);
            } else {
                load(s1, c1.idx);
                const Nb c2 = classify(P, x + 2 * sg * ox, y + 2 * sg * oy, z + 2 * sg * oz);
                if (c2.kind != kFluid)
                    ghost_slot(s2, c2, s1);
                else
                    load(s2, c2.idx);
            }
        }
    }
}

// T and Y of the fluid slots (read from the state; 0 at ghost slots).
template <int Q, int NSP>
__device__ __forceinline__ void slot_scalars(const KParams &P, const CellIn<Q, NSP> &in, double (&T)[n_slots<Q>()],
                                             double (&Y)[n_slots<Q>()][NSP])
{
    const double *sc = (const double *)P.sc_in;
#pragma unroll
    for (int s = 0; s < n_slots<Q>(); ++s) {
        const bool fl = in.kind[s] == kFluid;
        const long long c = fl ? in.cell[s] : in.cell[0];
        T[s] = fl ? sc[c] : 0.0;
#pragma unroll
        for (int k = 0; k < NSP; ++k) Y[s][k] = fl ? sc[(1 + k) * P.N + c] : 0.0;
    }
}

// Input slot numbering of the tangent: [0, Q) pulls; then S x (1 + NSP)
// stencil scalars (T, Y_k); then S ghost wall temperatures; then
// (A_j, Ta_j) per reaction.
template <int Q, int NSP>
struct Slots {
    static constexpr int S = n_slots<Q>();
    static constexpr int pull = 0;
    static constexpr int scal = Q;
    static constexpr int wall = Q + S * (1 + NSP);
    static constexpr int param = wall + S;
};

template <int NSP, class A>
__device__ A density_a(const KParams &P, A T, const A (&Y)[NSP])
{
    A s = 0.0;
    for (int k = 0; k < NSP; ++k) s += Y[k] * A(P.invW[k]);
    return A(P.T_ref_over_W_ref) / (T * s);
}

// Arrhenius source of one cell over the step in the number type A (the
// forward chemistry's sub-stepping, rate coefficients and limiter): from
// the cell's T0, Y0 and the reactions' (A_j, Ta_j) = par(j) to (srcT, srcY).
// The sub-step count and the limiter's choice follow the values.
template <int NSP, class A, class Par>
__device__ void chem_source(const KParams &P, const double *tab, const A &T0, const A (&Y0)[NSP], Par par, A &srcT,
                            A (&srcY)[NSP])
{
    const bool anyb = P.chem_anyb != 0;
    int nsub = 1;
    if (P.chem_substeps_max > 1) {
        const double lnT = anyb ? log(val(T0)) : 0.0, invT = rcp(val(T0));
        double kmax = 0.0;
        for (int j = 0; j < P.n_rx; ++j) kmax = fmax(kmax, rate_coeff_l(P.rxk[j], lnT, invT, tab));
        const double want = ceil(kmax / 0.1);
        nsub = want < 1.0 ? 1 : want > (double)P.chem_substeps_max ? P.chem_substeps_max : (int)want;
    }
    const double inv_nsub = nsub == 1 ? 1.0 : rcp((double)nsub);
    A dT = 0.0, dY[NSP];
    for (int k = 0; k < NSP; ++k) dY[k] = 0.0;
    for (int s = 0; s < nsub; ++s) {
        const A Tc = T0 + dT;
        A Yc[NSP], incT = 0.0, incY[NSP];
        for (int k = 0; k < NSP; ++k) {
            Yc[k] = Y0[k] + dY[k];
            incY[k] = 0.0;
        }
        const A lnTc = anyb ? dlog(Tc) : A(0.0), invTc = rcp(Tc);
        for (int j = 0; j < P.n_rx; ++j) {
            const lbfd_reaction &r = P.rx[j];
            A Aj, Taj;
            par(j, Aj, Taj);
            A rr = Aj * A(P.dt_phys) * dexp(A(r.b) * lnTc - Taj * invTc, tab) * A(inv_nsub);
            // four reactant factors, Y of the reactant or 1 (react[m] = NSP)
#pragma unroll
            for (int mm = 0; mm < 4; ++mm) {
                const int sp = P.rxk[j].react[mm];
                A f = 1.0;
#pragma unroll
                for (int k = 0; k < NSP; ++k) f = sp == k ? Yc[k] : f;
                rr *= f;
            }
            for (int k = 0; k < NSP; ++k) incY[k] += A(r.nu_mass[k]) * rr;
            incT += A(r.q_over_cp) * rr;
        }
        // positivity limiter (value-based choice, differentiable scale)
        A lam = 1.0;
        for (int k = 0; k < NSP; ++k)
            if (val(incY[k]) < 0.0 && val(Yc[k] + incY[k]) < 0.0) {
                const A l = (val(Yc[k]) > 0.0 ? Yc[k] : A(0.0)) / (-incY[k]);
                if (val(l) < val(lam)) lam = l;
            }
        dT += lam * incT;
        for (int k = 0; k < NSP; ++k) dY[k] += lam * incY[k];
    }
    srcT = dT;
    for (int k = 0; k < NSP; ++k) srcY[k] = dY[k];
}

// One sub-step of chem_source in FP64 from the state (Tc, Yc): the
// increments, the limiter's scale lam and the species that set it (kstar,
// -1 when lam = 1), with the same arithmetic as chem_source.
template <int NSP>
__device__ __forceinline__ void chem_substep(const KParams &P, const double *tab, bool anyb, double inv_nsub,
                                             double Tc, const double (&Yc)[NSP], double &incT, double (&incY)[NSP],
                                             double &lam, int &kstar)
{
    const double lnTc = anyb ? log(Tc) : 0.0, invTc = rcp(Tc);
    incT = 0.0;
#pragma unroll
    for (int k = 0; k < NSP; ++k) incY[k] = 0.0;
    for (int j = 0; j < P.n_rx; ++j) {
        const lbfd_reaction &r = P.rx[j];
        double rr = r.A * P.dt_phys * dexp(r.b * lnTc - r.Ta * invTc, tab) * inv_nsub;
#pragma unroll
        for (int mm = 0; mm < 4; ++mm) {
            const int sp = P.rxk[j].react[mm];
            double f = 1.0;
#pragma unroll
            for (int k = 0; k < NSP; ++k) f = sp == k ? Yc[k] : f;
            rr *= f;
        }
#pragma unroll
        for (int k = 0; k < NSP; ++k) incY[k] += r.nu_mass[k] * rr;
        incT += r.q_over_cp * rr;
    }
    lam = 1.0;
    kstar = -1;
#pragma unroll
    for (int k = 0; k < NSP; ++k)
        if (incY[k] < 0.0 && Yc[k] + incY[k] < 0.0) {
            const double l = (Yc[k] > 0.0 ? Yc[k] : 0.0) / (-incY[k]);
            if (l < lam) {
                lam = l;
                kstar = k;
            }
        }
}

// Reverse of chem_source (FP64): given ls, the adjoint of (srcT, srcY),
// adds ls^T d src / d (T0, Y0) to aT0, aY0 and ls^T d src / d (A_j, Ta_j) to
// lam_param[2 j], lam_param[2 j + 1] (LDS).  The sub-steps are reversed
// from the last; the state of each is recomputed from (T0, Y0), so the cost
// grows with the square of the sub-step count (one sub-step: one forward
// and one reverse evaluation).
template <int NSP>
__device__ void chem_vjp(const KParams &P, const double *tab, double T0, const double (&Y0)[NSP],
                         const double (&ls)[1 + NSP], double &aT0, double (&aY0)[NSP], double *lam_param)
{
    const bool anyb = P.chem_anyb != 0;
    int nsub = 1;
    if (P.chem_substeps_max > 1) {
        const double lnT = anyb ? log(T0) : 0.0, invT = rcp(T0);
        double kmax = 0.0;
        for (int j = 0; j < P.n_rx; ++j) kmax = fmax(kmax, rate_coeff_l(P.rxk[j], lnT, invT, tab));
        const double want = ceil(kmax / 0.1);
        nsub = want < 1.0 ? 1 : want > (double)P.chem_substeps_max ? P.chem_substeps_max : (int)want;
    }
    const double inv_nsub = nsub == 1 ? 1.0 : rcp((double)nsub);
    // adjoint of the accumulated increments (dT, dY) after sub-step s
    double LdT = ls[0], LdY[NSP];
#pragma unroll
    for (int k = 0; k < NSP; ++k) LdY[k] = ls[1 + k];
    for (int s = nsub - 1; s >= 0; --s) {
        double dT = 0.0, dY[NSP];
#pragma unroll
        for (int k = 0; k < NSP; ++k) dY[k] = 0.0;
        double Yc[NSP], incT, incY[NSP], lam;
        int kstar;
        for (int t = 0; t < s; ++t) {
#pragma unroll
            for (int k = 0; k < NSP; ++k) Yc[k] = Y0[k] + dY[k];
            chem_substep<NSP>(P, tab, anyb, inv_nsub, T0 + dT, Yc, incT, incY, lam, kstar);
            dT += lam * incT;
#pragma unroll
            for (int k = 0; k < NSP; ++k) dY[k] += lam * incY[k];
        }
        const double Tc = T0 + dT;
#pragma unroll
        for (int k = 0; k < NSP; ++k) Yc[k] = Y0[k] + dY[k];
        chem_substep<NSP>(P, tab, anyb, inv_nsub, Tc, Yc, incT, incY, lam, kstar);
        // (dT, dY) += lam (incT, incY)
        double llam = LdT * incT, lincY[NSP], lYc[NSP];
#pragma unroll
        for (int k = 0; k < NSP; ++k) {
            llam += LdY[k] * incY[k];
            lincY[k] = lam * LdY[k];
            lYc[k] = 0.0;
        }
        const double lincT = lam * LdT;
        // lam = Yc_k / (-incY_k) for the limiting species k (0 if Yc_k <= 0)
#pragma unroll
        for (int k = 0; k < NSP; ++k)
            if (k == kstar && Yc[k] > 0.0) {
                lYc[k] += llam / (-incY[k]);
                lincY[k] += llam * Yc[k] / (incY[k] * incY[k]);
            }
        // the rates rr_j = A_j dt exp(b_j ln Tc - Ta_j / Tc) / nsub prod_m F_jm
        const double lnTc = anyb ? log(Tc) : 0.0, invTc = rcp(Tc);
        double lTc = 0.0;
        for (int j = 0; j < P.n_rx; ++j) {
            const lbfd_reaction &r = P.rx[j];
            const double e = dexp(r.b * lnTc - r.Ta * invTc, tab);
            const double base = r.A * P.dt_phys * e * inv_nsub;
            double F[4];
            int sp[4];
#pragma unroll
            for (int mm = 0; mm < 4; ++mm) {
                sp[mm] = P.rxk[j].react[mm];
                double f = 1.0;
#pragma unroll
                for (int k = 0; k < NSP; ++k) f = sp[mm] == k ? Yc[k] : f;
                F[mm] = f;
            }
            const double pr = F[0] * F[1] * F[2] * F[3];
            const double rr = base * pr;
            double lrr = r.q_over_cp * lincT;
#pragma unroll
            for (int k = 0; k < NSP; ++k) lrr += r.nu_mass[k] * lincY[k];
            lTc += lrr * rr * (r.b * invTc + r.Ta * invTc * invTc);
            atomicAdd(&lam_param[2 * j], lrr * P.dt_phys * e * inv_nsub * pr);
            atomicAdd(&lam_param[2 * j + 1], -lrr * rr * invTc);
            // each factor: the product of the other three
            const double other[4] = {F[1] * F[2] * F[3], F[0] * F[2] * F[3], F[0] * F[1] * F[3], F[0] * F[1] * F[2]};
#pragma unroll
            for (int mm = 0; mm < 4; ++mm) {
                const double g = lrr * base * other[mm];
#pragma unroll
                for (int k = 0; k < NSP; ++k) lYc[k] += sp[mm] == k ? g : 0.0;
            }
        }
        // Tc = T0 + dT, Yc = Y0 + dY
        aT0 += lTc;
        LdT += lTc;
#pragma unroll
        for (int k = 0; k < NSP; ++k) {
            aY0[k] += lYc[k];
            LdY[k] += lYc[k];
        }
    }
}

// The cell's update in dual numbers with the tangent tan[slot] of every
// input slot (Slots numbering): outputs out[0..Q) = g*, out[Q] = T^{n+1},
// out[Q+1+k] = Y_k^{n+1}; *qc = the cell's wall-heat-flux contribution at
// level n.
template <int Q, int NSP>
__device__ void cell_eval(const KParams &P, const CellIn<Q, NSP> &in, const double *tan, Dual (&out)[Q + 1 + NSP],
                          Dual &qc)
{
    using A = Dual;
    using L = Lat<Q>;
    using S = Slots<Q, NSP>;
    constexpr int D = L::D;
    auto mk = [&](double v, int slot) -> A {
        A r(v);
        r.d[0] = tan[slot];
        return r;
    };
    A g[Q];
    for (int i = 0; i < Q; ++i) g[i] = mk(in.g[i], S::pull + i);
    constexpr int NSL = n_slots<Q>();
    double Tv[NSL], Yv[NSL][NSP];
    slot_scalars<Q, NSP>(P, in, Tv, Yv);
    A T[NSL], Y[NSL][NSP], R[NSL], Tw[NSL];
    for (int s = 0; s < NSL; ++s) {
        Tw[s] = mk(in.Tw[s], S::wall + s);
        if (in.kind[s] == kFluid) {
            T[s] = mk(Tv[s], S::scal + s * (1 + NSP));
            A Ys[NSP];
            for (int k = 0; k < NSP; ++k) {
                Y[s][k] = mk(Yv[s][k], S::scal + s * (1 + NSP) + 1 + k);
                Ys[k] = Y[s][k];
            }
            R[s] = density_a<NSP>(P, T[s], Ys);
        }
    }
    // ghosts (Sec. III.B): images are fluid slots
    for (int s = 0; s < NSL; ++s) {
        if (in.kind[s] == kFluid) continue;
        const int im = in.img[s];
        if (in.kind[s] == kIso) {
            T[s] = A(2.0) * Tw[s] - T[im];
            A Ys[NSP];
            for (int k = 0; k < NSP; ++k) {
                Y[s][k] = Y[im][k];
                Ys[k] = Y[im][k];
            }
            R[s] = A(2.0) * density_a<NSP>(P, Tw[s], Ys) - R[im];
        } else if (in.kind[s] == kInflow) {
            T[s] = A(2.0 * P.T_in) - T[im];
            for (int k = 0; k < NSP; ++k) Y[s][k] = A(2.0 * P.Y_in[k]) - Y[im][k];
            R[s] = A(2.0 * P.rho_in) - R[im];
        } else {
            T[s] = T[im];
            for (int k = 0; k < NSP; ++k) Y[s][k] = Y[im][k];
            R[s] = R[im];
        }
    }
    const A rho = R[0];
    A m[3] = {0.0, 0.0, 0.0};
    for (int i = 0; i < Q; ++i) {
        m[0] += A((double)L::cx(i)) * g[i];
        m[1] += A((double)L::cy(i)) * g[i];
        m[2] += A((double)L::cz(i)) * g[i];
    }
    const A inv_rc = A(1.0) / (rho * A(kCs2));
    const A u[3] = {m[0] * inv_rc, m[1] * inv_rc, m[2] * inv_rc};
    const A inv_rho = A(1.0) / rho;
    A diffT = 0.0, CT = 0.0, grad[3] = {0.0, 0.0, 0.0}, diffY[NSP], CY[NSP];
    for (int k = 0; k < NSP; ++k) diffY[k] = CY[k] = 0.0;
    qc = 0.0;
    for (int d = 0; d < D; ++d) {
        const int sl[5] = {1 + 4 * d, 2 + 4 * d, 0, 3 + 4 * d, 4 + 4 * d};
        bool near = false;
        for (int j = 0; j < 5; ++j) near |= in.kind[sl[j]] != kFluid;
        // wall heat flux through the first-neighbour walls
        for (int j = 1; j <= 3; j += 2)
            if (in.kind[sl[j]] == kIso) {
                A Yc[NSP];
                for (int k = 0; k < NSP; ++k) Yc[k] = Y[0][k];
                qc += A(2.0 * P.alpha) * density_a<NSP>(P, Tw[sl[j]], Yc) * (T[0] - Tw[sl[j]]);
            }
        const A ud = u[d];
        const A d1r = d1(R[sl[0]], R[sl[1]], R[sl[2]], R[sl[3]], R[sl[4]]);
        {
            const A a = T[sl[0]], b = T[sl[1]], c = T[sl[2]], e = T[sl[3]], f = T[sl[4]];
            diffT += d2(a, b, c, e, f) + d1r * d1(a, b, c, e, f) * inv_rho;
            CT += ud * (near ? A(0.5) * (e - b) : weno3(a, b, c, e, f, ud));
        }
        A cY[NSP], sumc = 0.0;
        for (int k = 0; k < NSP; ++k) {
            const A a = Y[sl[0]][k], b = Y[sl[1]][k], c = Y[sl[2]][k], e = Y[sl[3]][k], f = Y[sl[4]][k];
            diffY[k] += d2(a, b, c, e, f) + d1r * d1(a, b, c, e, f) * inv_rho;
            cY[k] = near ? A(0.5) * (e - b) : weno3(a, b, c, e, f, ud);
            sumc += cY[k];
        }
        for (int k = 0; k < NSP; ++k) CY[k] += ud * (cY[k] - Y[0][k] * sumc);
        grad[d] = d1r;
    }
    const A alpha = A(P.alpha);
    diffT *= alpha;
    for (int k = 0; k < NSP; ++k) diffY[k] *= alpha;

    A srcT, srcY[NSP], Y0[NSP];
    for (int k = 0; k < NSP; ++k) Y0[k] = Y[0][k];
    chem_source<NSP>(
        P, kExp2Tab, T[0], Y0,
        [&](int j, A &Aj, A &Taj) {
            Aj = mk(P.rx[j].A, S::param + 2 * j);
            Taj = mk(P.rx[j].Ta, S::param + 2 * j + 1);
        },
        srcT, srcY);

    const A DtT = diffT + srcT;
    A DtY[NSP], invW = 0.0;
    for (int k = 0; k < NSP; ++k) {
        DtY[k] = diffY[k] + srcY[k];
        invW += Y[0][k] * A(P.invW[k]);
    }
    const A Wm = A(1.0) / invW;
    A Lam = DtT / T[0];
    for (int k = 0; k < NSP; ++k) Lam += (Wm * A(P.invW[k])) * DtY[k];
    out[Q] = T[0] - CT + DtT;
    for (int k = 0; k < NSP; ++k) out[Q + 1 + k] = Y[0][k] - CY[k] + DtY[k];

    const A uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
    A xi[Q], h[Q], pi = 0.0;
    const A half_inv = A(0.5) * inv_rc;
    for (int i = 0; i < Q; ++i) {
        const A wi = A(L::w(i));
        const A cu = A((double)L::cx(i)) * u[0] + A((double)L::cy(i)) * u[1] + A((double)L::cz(i)) * u[2];
        const A feq_r = wi * (A(1.0) + A(3.0) * cu + A(4.5) * cu * cu - A(1.5) * uu);
        const A proj = (A((double)L::cx(i)) - u[0]) * grad[0] + (A((double)L::cy(i)) - u[1]) * grad[1] +
                       (A((double)L::cz(i)) - u[2]) * grad[2];
        xi[i] = A(kCs2) * (feq_r - wi) * proj + wi * rho * A(kCs2) * Lam;
        h[i] = g[i] * inv_rc + xi[i] * half_inv;
        pi += h[i];
    }
    const A sh = A(1.0) - pi;
    for (int i = 0; i < Q; ++i) h[i] += A(L::w(i)) * sh;
    central_fwd<Q>(h, u);
    relax<Q>(h, A(P.omega2), A(P.omega3), A(P.omega4));
    central_inv<Q>(h, u);
    const A rc = rho * A(kCs2);
    for (int i = 0; i < Q; ++i) out[i] = rc * (h[i] - A(L::w(i)) * sh) + A(0.5) * xi[i];
}

// ------------------------------------------------------- the reverse sweep
// Reverse of cm_fwd_line at the input (a, b, d): (la, lb, ld) holds the
// adjoints of (m0, m1, m2) and receives those of (a, b, d); returns the
// contribution to the adjoint of u.
__device__ __forceinline__ double cm_fwd_line_adj(double a, double b, double d, double u, double &la, double &lb,
                                                  double &ld)
{
    const double m0 = a + b + d;
    const double l0 = la, l1 = lb, l2 = ld;
    la = l0 - (1.0 + u) * l1 + (1.0 + u) * (1.0 + u) * l2;
    lb = l0 - u * l1 + u * u * l2;
    ld = l0 + (1.0 - u) * l1 + (1.0 - u) * (1.0 - u) * l2;
    return -m0 * l1 + (2.0 * (a - d) + 2.0 * u * m0) * l2;
}

// Reverse of cm_inv_line at the input moments (m0, m1, m2).
__device__ __forceinline__ double cm_inv_line_adj(double m0, double m1, double m2, double u, double &la, double &lb,
                                                  double &ld)
{
    const double uu = u * u;
    const double A = la, B = lb, E = ld;
    la = 0.5 * (uu - u) * A + (1.0 - uu) * B + 0.5 * (uu + u) * E;
    lb = 0.5 * (2.0 * u - 1.0) * A - 2.0 * u * B + 0.5 * (2.0 * u + 1.0) * E;
    ld = 0.5 * A - B + 0.5 * E;
    (void)m2;
    return 0.5 * (m0 * (2.0 * u - 1.0) + 2.0 * m1) * A - 2.0 * (u * m0 + m1) * B +
           0.5 * (m0 * (2.0 * u + 1.0) + 2.0 * m1) * E;
}

// Reverse of relax(): the orders >= 2 were scaled by (1 - omega).
template <int Q>
__device__ __forceinline__ void relax_adj(double (&lk)[Q], double om2, double om3, double om4)
{
    sfor<0, Q>([&](auto J) {
        constexpr int j = decltype(J)::value;
        constexpr int p = j % 3, q = (j / 3) % 3, r = (Q == 27) ? j / 9 : 0;
        constexpr int order = p + q + r;
        if constexpr (order >= 2) lk[j] *= 1.0 - (order == 2 ? om2 : order == 3 ? om3 : om4);
    });
}

// Reverse of weno3(m2, m1, c0, p1, p2, u) for the adjoint lam of its
// result: adds the adjoints of the five stencil values to l[0..5) (u
// enters through its sign only).
__device__ __forceinline__ void weno3_adj(double m2, double m1, double c0, double p1, double p2, double u, double lam,
                                          double (&l)[5])
{
    const bool neg = u < 0.0;
    const double A = neg ? p2 : m2, B = neg ? p1 : m1, E = neg ? m1 : p1;
    const double eps = 1e-6;
    const double dA = B - A, dB = c0 - B, dE = E - c0;
    const double eA = eps + dA * dA, eB = eps + dB * dB, eE = eps + dE * dE;
    const double eA2 = eA * eA, eB2 = eB * eB, eE2 = eE * eE;
    const double den_p = eE2 + 2.0 * eB2, den_m = eB2 + 2.0 * eA2;
    const double ip = rcp(den_p), im = rcp(den_m);
    const double w_p = eE2 * ip, w_m = eB2 * im;
    const double q0p = 1.5 * c0 - 0.5 * B, q1p = 0.5 * (c0 + E);
    const double q0m = 1.5 * B - 0.5 * A, q1m = 0.5 * (B + c0);
    const double L = neg ? -lam : lam;
    const double lq1p = L * (1.0 - w_p), lq0p = L * w_p, lw_p = L * (q0p - q1p);
    const double lq1m = -L * (1.0 - w_m), lq0m = -L * w_m, lw_m = -L * (q0m - q1m);
    const double leE2 = lw_p * 2.0 * eB2 * ip * ip;
    const double leB2 = -lw_p * 2.0 * eE2 * ip * ip + lw_m * 2.0 * eA2 * im * im;
    const double leA2 = -lw_m * 2.0 * eB2 * im * im;
    const double ldA = leA2 * 4.0 * eA * dA, ldB = leB2 * 4.0 * eB * dB, ldE = leE2 * 4.0 * eE * dE;
    const double lA = -ldA - 0.5 * lq0m;
    const double lB = ldA - ldB - 0.5 * lq0p + 1.5 * lq0m + 0.5 * lq1m;
    const double lC = ldB - ldE + 1.5 * lq0p + 0.5 * lq1p + 0.5 * lq1m;
    const double lE = ldE + 0.5 * lq1p;
    // selects on the values, not on the destination (an indexed store would
    // put l in scratch memory)
    l[0] += neg ? 0.0 : lA;
    l[1] += neg ? lE : lB;
    l[2] += lC;
    l[3] += neg ? lB : lE;
    l[4] += neg ? lA : 0.0;
}

// The backward step runs as two kernels per level.  The first
// (adjoint_collision_kernel) evaluates the cell's update forward and reverses
// the collision, the moments and the velocity's part of the convection: it
// finishes the adjoints of the pulled populations and leaves, per cell, the
// few adjoints the rest needs (AdjMid).  The second (adjoint_stencil_kernel)
// reverses the finite-difference stencils, the ghosts and densities, and the
// Arrhenius source, and scatters the stencil scalars' adjoints.  Split so
// that each kernel's registers leave room for more than one wave per SIMD.

// Fields of the per-cell state between the two kernels, [field][N]:
// lDtT, lDtY_k (adjoints of the increments Dt), lgrad_d (of d1 rho), u_d,
// aT0, aY0_k (partial adjoints of the cell's own T, Y), lR0 (of its rho).
template <int D, int NSP>
struct AdjMid {
    static constexpr int ls = 0, lgrad = 1 + NSP, u = lgrad + D, aT0 = u + D, aY0 = aT0 + 1,
                         lR0 = aY0 + NSP, n = lR0 + 1;
};

// Where the reverse sweep puts the adjoints of a cell's inputs.
struct AdjOut {
    const double *lo_pop;  // [Q][N] adjoint of the populations the step writes
    const double *lo_sc;   // [1+NSP][N] adjoint of the scalars the step writes
    double *lam_pop;    // [Q][N]: stored (every entry is pulled by one cell)
    double *lam_sc;     // [1+NSP][N]: accumulated atomically
    double *dwallT;     // [N]: accumulated atomically
    double *lam_param;  // [2 n_rx] in LDS: accumulated atomically
    double *mid;        // [AdjMid::n][N]
    double *nb;         // [S - 1][1+NSP][N]: what each stencil slot's cell receives
};

// The stencil's T, Y, rho and sum_k Y_k / W_k, ghosts from their images
// (fluid slots: the cell or a first neighbour).  Reciprocals of these
// positive normal values by rcp() (the divisions here and in the stencil's
// reverse: about one ulp).
template <int Q, int NSP>
__device__ __forceinline__ void fill_stencil(const KParams &P, const CellIn<Q, NSP> &in, double (&T)[n_slots<Q>()],
                                             double (&Y)[n_slots<Q>()][NSP], double (&R)[n_slots<Q>()],
                                             double (&Sw)[n_slots<Q>()])
{
    constexpr int S = n_slots<Q>();
    const double c0 = P.T_ref_over_W_ref;
    slot_scalars<Q, NSP>(P, in, T, Y);
#pragma unroll
    for (int s = 0; s < S; ++s) {
        double sw = 0.0;
#pragma unroll
        for (int k = 0; k < NSP; ++k) sw += Y[s][k] * P.invW[k];
        const bool fl = in.kind[s] == kFluid;
        Sw[s] = fl ? sw : 1.0;
        R[s] = fl ? c0 * rcp(T[s] * Sw[s]) : 0.0;
    }
#pragma unroll
    for (int s = 1; s < S; ++s) {
        const int kd = in.kind[s];
        if (kd == kFluid) continue;
        const int im = in.img[s];
        const int ca = img_lo(s), cb = img_hi(s);
        const bool ia = im == ca, ib = !ia && im == cb;
        // the image's values as an exact 0/1 blend of the three candidates
        // (a select between array elements would become an indexed load and
        // keep the arrays in scratch memory)
        const double fa = ia ? 1.0 : 0.0, fb = ib ? 1.0 : 0.0, f0 = 1.0 - fa - fb;
        auto blend = [&](double va, double vb, double v0) { return fa * va + fb * vb + f0 * v0; };
        const double Ti = blend(T[ca], T[cb], T[0]);
        const double Ri = blend(R[ca], R[cb], R[0]);
        const double Swi = blend(Sw[ca], Sw[cb], Sw[0]);
        double Yi[NSP];
#pragma unroll
        for (int k = 0; k < NSP; ++k) Yi[k] = blend(Y[ca][k], Y[cb][k], Y[0][k]);
        Sw[s] = Swi;
        if (kd == kIso) {
            T[s] = 2.0 * in.Tw[s] - Ti;
#pragma unroll
            for (int k = 0; k < NSP; ++k) Y[s][k] = Yi[k];
            R[s] = 2.0 * (c0 * rcp(in.Tw[s] * Swi)) - Ri;
        } else if (kd == kInflow) {
            T[s] = 2.0 * P.T_in - Ti;
#pragma unroll
            for (int k = 0; k < NSP; ++k) Y[s][k] = 2.0 * P.Y_in[k] - Yi[k];
            R[s] = 2.0 * P.rho_in - Ri;
        } else {
            T[s] = Ti;
#pragma unroll
            for (int k = 0; k < NSP; ++k) Y[s][k] = Yi[k];
            R[s] = Ri;
        }
    }
}

// First half: the cell's update forward in FP64, then the reverse of the
// collision (central moments and their transforms, the forcing Xi, the
// equilibrium), of the scalars' increments up to Dt, of the convection's
// dependence on u and of the moments (u = m / (rho cs2)).  From the adjoint
// of the outputs (g*, T^{n+1}, Y^{n+1}; read from out) and the weight wT0 of
// the cell's own T (the flame position's linear term): the adjoints of the
// pulled populations (stored) and the cell's AdjMid.
template <int Q, int NSP>
__device__ void cell_vjp_collision(const KParams &P, const CellIn<Q, NSP> &in, double wT0, const double *tab,
                                   const AdjOut &out)
{
    using L = Lat<Q>;
    using M = AdjMid<Lat<Q>::D, NSP>;
    constexpr int D = L::D, S = n_slots<Q>(), NS = 1 + NSP;

    // ------------------------------------------------ forward (values)
    double g[Q];
#pragma unroll
    for (int i = 0; i < Q; ++i) g[i] = in.g[i];
    double m[3] = {0.0, 0.0, 0.0};
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        m[0] += L::cx(i) * g[i];
        m[1] += L::cy(i) * g[i];
        m[2] += L::cz(i) * g[i];
    }
    double T0, Y0[NSP], rho;
    double diffT = 0.0, grad[3] = {0.0, 0.0, 0.0}, diffY[NSP];
    double cT[3] = {0.0, 0.0, 0.0}, cY[3][NSP], sumc[3] = {0.0, 0.0, 0.0};
    double u[3], inv_rc, inv_rho;
    {
        double T[S], Y[S][NSP], R[S], Sw[S];
        fill_stencil<Q, NSP>(P, in, T, Y, R, Sw);
        T0 = T[0];
#pragma unroll
        for (int k = 0; k < NSP; ++k) Y0[k] = Y[0][k];
        rho = R[0];
        inv_rc = rcp(rho * kCs2);
#pragma unroll
        for (int d = 0; d < 3; ++d) u[d] = m[d] * inv_rc;
        inv_rho = rcp(rho);
#pragma unroll
        for (int k = 0; k < NSP; ++k) diffY[k] = 0.0;
#pragma unroll
        for (int d = 0; d < D; ++d) {
            const int sl[5] = {1 + 4 * d, 2 + 4 * d, 0, 3 + 4 * d, 4 + 4 * d};
            bool near = false;
#pragma unroll
            for (int j = 0; j < 5; ++j) near |= in.kind[sl[j]] != kFluid;
            const double d1r = d1(R[sl[0]], R[sl[1]], R[sl[2]], R[sl[3]], R[sl[4]]);
            {
                const double p = T[sl[0]], b = T[sl[1]], c = T[sl[2]], e = T[sl[3]], f = T[sl[4]];
                diffT += d2(p, b, c, e, f) + d1r * d1(p, b, c, e, f) * inv_rho;
                cT[d] = near ? 0.5 * (e - b) : weno3(p, b, c, e, f, u[d]);
            }
#pragma unroll
            for (int k = 0; k < NSP; ++k) {
                const double p = Y[sl[0]][k], b = Y[sl[1]][k], c = Y[sl[2]][k], e = Y[sl[3]][k], f = Y[sl[4]][k];
                diffY[k] += d2(p, b, c, e, f) + d1r * d1(p, b, c, e, f) * inv_rho;
                cY[d][k] = near ? 0.5 * (e - b) : weno3(p, b, c, e, f, u[d]);
                sumc[d] += cY[d][k];
            }
            grad[d] = d1r;
        }
    }
    diffT *= P.alpha;
#pragma unroll
    for (int k = 0; k < NSP; ++k) diffY[k] *= P.alpha;
    double srcT, srcY[NSP];
    chem_source<NSP>(
        P, tab, T0, Y0,
        [&](int j, double &Aj, double &Taj) {
            Aj = P.rx[j].A;
            Taj = P.rx[j].Ta;
        },
        srcT, srcY);
    const double DtT = diffT + srcT;
    double DtY[NSP], invWs = 0.0;
#pragma unroll
    for (int k = 0; k < NSP; ++k) {
        DtY[k] = diffY[k] + srcY[k];
        invWs += Y0[k] * P.invW[k];
    }
    const double Wm = rcp(invWs);
    const double inv_T0 = rcp(T0);
    double Lam = DtT * inv_T0;
#pragma unroll
    for (int k = 0; k < NSP; ++k) Lam += (Wm * P.invW[k]) * DtY[k];

    // xi_i = cs2 (feq_i - w_i) proj_i + w_i rho cs2 Lam, feq_i and proj_i
    // from u and grad (recomputed in the reverse)
    const double uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
    auto xi_of = [&](int i, double &feq, double &proj) {
        const double wi = L::w(i);
        const double cu = L::cx(i) * u[0] + L::cy(i) * u[1] + L::cz(i) * u[2];
        feq = wi * (1.0 + 3.0 * cu + 4.5 * cu * cu - 1.5 * uu);
        proj = (L::cx(i) - u[0]) * grad[0] + (L::cy(i) - u[1]) * grad[1] + (L::cz(i) - u[2]) * grad[2];
        return kCs2 * (feq - wi) * proj + wi * rho * kCs2 * Lam;
    };
    const double half_inv = 0.5 * inv_rc;
    double hx[Q], pi = 0.0;
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        double feq, proj;
        hx[i] = g[i] * inv_rc + xi_of(i, feq, proj) * half_inv;
        pi += hx[i];
    }
    const double sh = 1.0 - pi;
#pragma unroll
    for (int i = 0; i < Q; ++i) hx[i] += L::w(i) * sh;
    // moments (kept: kr, the relaxed central moments; the passes' other
    // inputs are recomputed in the reverse)
    double kr[Q];
#pragma unroll
    for (int i = 0; i < Q; ++i) kr[i] = hx[i];
    central_fwd<Q>(kr, u);
    relax<Q>(kr, P.omega2, P.omega3, P.omega4);
    const double rc = rho * kCs2;

    // ------------------------------------------------------ reverse
    const long long c_self = in.cell[0];
    double lo[Q + 1 + NSP];
#pragma unroll
    for (int i = 0; i < Q; ++i) lo[i] = out.lo_pop[(long long)i * P.N + c_self];
#pragma unroll
    for (int k = 0; k < 1 + NSP; ++k) lo[Q + k] = out.lo_sc[(long long)k * P.N + c_self];
    double lu[3] = {0.0, 0.0, 0.0}, lrho = 0.0, linv_rc = 0.0;

    // out_i = rc (h3_i - w_i sh) + xi_i / 2, h3 = central_inv(kr)
    double lh[Q], lrc = 0.0, lsh = 0.0;
    {
        double iz[Q], iy[Q];
#pragma unroll
        for (int i = 0; i < Q; ++i) iz[i] = kr[i];
        if constexpr (Q == 27) {
#pragma unroll
            for (int r = 0; r < 9; ++r) cm_inv_line(iz[r], iz[r + 9], iz[r + 18], u[2]);
        }
#pragma unroll
        for (int i = 0; i < Q; ++i) iy[i] = iz[i];
#pragma unroll
        for (int zp = 0; zp < Q / 9; ++zp)
#pragma unroll
            for (int p = 0; p < 3; ++p) cm_inv_line(iy[9 * zp + p], iy[9 * zp + p + 3], iy[9 * zp + p + 6], u[1]);
        double h3[Q];
#pragma unroll
        for (int i = 0; i < Q; ++i) h3[i] = iy[i];
#pragma unroll
        for (int l = 0; l < Q / 3; ++l) cm_inv_line(h3[3 * l], h3[3 * l + 1], h3[3 * l + 2], u[0]);
#pragma unroll
        for (int i = 0; i < Q; ++i) {
            lh[i] = rc * lo[i];
            lrc += lo[i] * (h3[i] - L::w(i) * sh);
            lsh -= rc * L::w(i) * lo[i];
        }
        // central_inv, reversed
#pragma unroll
        for (int l = 0; l < Q / 3; ++l)
            lu[0] += cm_inv_line_adj(iy[3 * l], iy[3 * l + 1], iy[3 * l + 2], u[0], lh[3 * l], lh[3 * l + 1],
                                     lh[3 * l + 2]);
#pragma unroll
        for (int zp = 0; zp < Q / 9; ++zp)
#pragma unroll
            for (int p = 0; p < 3; ++p) {
                const int i0 = 9 * zp + p, i1 = i0 + 3, i2 = i0 + 6;
                lu[1] += cm_inv_line_adj(iz[i0], iz[i1], iz[i2], u[1], lh[i0], lh[i1], lh[i2]);
            }
        if constexpr (Q == 27) {
#pragma unroll
            for (int r = 0; r < 9; ++r)
                lu[2] += cm_inv_line_adj(kr[r], kr[r + 9], kr[r + 18], u[2], lh[r], lh[r + 9], lh[r + 18]);
        }
    }
    relax_adj<Q>(lh, P.omega2, P.omega3, P.omega4);
    // central_fwd, reversed
    {
        double hy[Q], hz[Q];
#pragma unroll
        for (int i = 0; i < Q; ++i) hy[i] = hx[i];
#pragma unroll
        for (int l = 0; l < Q / 3; ++l) cm_fwd_line(hy[3 * l], hy[3 * l + 1], hy[3 * l + 2], u[0]);
#pragma unroll
        for (int i = 0; i < Q; ++i) hz[i] = hy[i];
#pragma unroll
        for (int zp = 0; zp < Q / 9; ++zp)
#pragma unroll
            for (int p = 0; p < 3; ++p) cm_fwd_line(hz[9 * zp + p], hz[9 * zp + p + 3], hz[9 * zp + p + 6], u[1]);
        if constexpr (Q == 27) {
#pragma unroll
            for (int r = 0; r < 9; ++r)
                lu[2] += cm_fwd_line_adj(hz[r], hz[r + 9], hz[r + 18], u[2], lh[r], lh[r + 9], lh[r + 18]);
        }
#pragma unroll
        for (int zp = 0; zp < Q / 9; ++zp)
#pragma unroll
            for (int p = 0; p < 3; ++p) {
                const int i0 = 9 * zp + p, i1 = i0 + 3, i2 = i0 + 6;
                lu[1] += cm_fwd_line_adj(hy[i0], hy[i1], hy[i2], u[1], lh[i0], lh[i1], lh[i2]);
            }
#pragma unroll
        for (int l = 0; l < Q / 3; ++l)
            lu[0] += cm_fwd_line_adj(hx[3 * l], hx[3 * l + 1], hx[3 * l + 2], u[0], lh[3 * l], lh[3 * l + 1],
                                     lh[3 * l + 2]);
    }
    // hx = h0 + w sh, sh = 1 - sum h0
#pragma unroll
    for (int i = 0; i < Q; ++i) lsh += L::w(i) * lh[i];
    double ag[Q];
    double lLam = 0.0, lgrad[3] = {0.0, 0.0, 0.0}, luu = 0.0;
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        const double lh0 = lh[i] - lsh;
        double feq, proj;
        const double xi = xi_of(i, feq, proj);
        // h0 = g inv_rc + xi inv_rc / 2
        ag[i] = inv_rc * lh0;
        const double lxi = 0.5 * lo[i] + half_inv * lh0;
        linv_rc += lh0 * (g[i] + 0.5 * xi);
        // xi = cs2 (feq - w) proj + w rho cs2 Lam
        const double wi = L::w(i);
        const double lfeq = kCs2 * proj * lxi;
        const double lproj = kCs2 * (feq - wi) * lxi;
        lrho += wi * kCs2 * Lam * lxi;
        lLam += wi * rho * kCs2 * lxi;
        // proj = sum_d (c_d - u_d) grad_d
        const double cd[3] = {(double)L::cx(i), (double)L::cy(i), (double)L::cz(i)};
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            lgrad[d] += lproj * (cd[d] - u[d]);
            lu[d] -= lproj * grad[d];
        }
        // feq = w (1 + 3 cu + 9/2 cu^2 - 3/2 uu)
        const double cu = cd[0] * u[0] + cd[1] * u[1] + cd[2] * u[2];
        const double lcu = wi * (3.0 + 9.0 * cu) * lfeq;
        luu -= 1.5 * wi * lfeq;
#pragma unroll
        for (int d = 0; d < 3; ++d) lu[d] += cd[d] * lcu;
    }
#pragma unroll
    for (int d = 0; d < 3; ++d) lu[d] += 2.0 * u[d] * luu;
    lrho += kCs2 * lrc;

    // scalar outputs: T' = T0 - CT + DtT, Y' = Y0 - CY + DtY
    const double lTo = lo[Q];
    double aT0 = lTo + wT0, aY0[NSP];
    const double lCT = -lTo;
    double lDtT = lTo, lCY[NSP], lDtY[NSP];
#pragma unroll
    for (int k = 0; k < NSP; ++k) {
        aY0[k] = lo[Q + 1 + k];
        lCY[k] = -lo[Q + 1 + k];
        lDtY[k] = lo[Q + 1 + k];
    }
    // Lam = DtT / T0 + sum_k Wm / W_k DtY_k, Wm = 1 / sum_k Y0_k / W_k
    lDtT += lLam * inv_T0;
    aT0 -= lLam * DtT * inv_T0 * inv_T0;
    double lWm = 0.0;
#pragma unroll
    for (int k = 0; k < NSP; ++k) {
        lDtY[k] += lLam * Wm * P.invW[k];
        lWm += lLam * P.invW[k] * DtY[k];
    }
    const double linvWs = -lWm * Wm * Wm;
#pragma unroll
    for (int k = 0; k < NSP; ++k) aY0[k] += linvWs * P.invW[k];
    // the convection's dependence on u (CT = sum_d u_d cT_d, CY_k = sum_d
    // u_d (cY_k - Y0_k sumc)) and on Y0 through sumc's factor
#pragma unroll
    for (int d = 0; d < D; ++d) {
        lu[d] += lCT * cT[d];
#pragma unroll
        for (int k = 0; k < NSP; ++k) {
            lu[d] += lCY[k] * (cY[d][k] - Y0[k] * sumc[d]);
            aY0[k] -= lCY[k] * u[d] * sumc[d];
        }
    }
    // u = m / (rho cs2)
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        const double lm = lu[d] * inv_rc;
        linv_rc += lu[d] * m[d];
#pragma unroll
        for (int i = 0; i < Q; ++i) {
            const int c = d == 0 ? L::cx(i) : d == 1 ? L::cy(i) : L::cz(i);
            if (c != 0) ag[i] += c * lm;
        }
    }
    lrho -= linv_rc * inv_rc * inv_rho;

    // pull streaming reads every population entry at most once (the source
    // cell's, or the cell's own opposite entry behind a wall)
#pragma unroll
    for (int i = 0; i < Q; ++i) out.lam_pop[(long long)in.tdir[i] * P.N + in.tcell[i]] = ag[i];
    // the source, reversed
    {
        double ls[NS];
        ls[0] = lDtT;
#pragma unroll
        for (int k = 0; k < NSP; ++k) ls[1 + k] = lDtY[k];
        chem_vjp<NSP>(P, tab, T0, Y0, ls, aT0, aY0, out.lam_param);
    }
    double *mid = out.mid + c_self;
    mid[(long long)M::ls * P.N] = lDtT;
#pragma unroll
    for (int k = 0; k < NSP; ++k) mid[(long long)(M::ls + 1 + k) * P.N] = lDtY[k];
#pragma unroll
    for (int d = 0; d < D; ++d) {
        mid[(long long)(M::lgrad + d) * P.N] = lgrad[d];
        mid[(long long)(M::u + d) * P.N] = u[d];
    }
    mid[(long long)M::aT0 * P.N] = aT0;
#pragma unroll
    for (int k = 0; k < NSP; ++k) mid[(long long)(M::aY0 + k) * P.N] = aY0[k];
    mid[(long long)M::lR0 * P.N] = lrho;
}

// Second half: the reverse of the finite-difference stencils (diffusion,
// the convection's dependence on the stencil values, d1 rho), the ghosts
// and densities, the wall-heat-flux term (weight wq) and the Arrhenius
// source, from the cell's AdjMid; scatters the adjoints of the stencil's T,
// Y (atomically, per axis as soon as its slots are finished), of the wall
// temperatures and of A_j, Ta_j.
template <int Q, int NSP>
__device__ void cell_vjp_stencil(const KParams &P, const CellIn<Q, NSP> &in, double wq, const AdjOut &out)
{
    using L = Lat<Q>;
    using M = AdjMid<Lat<Q>::D, NSP>;
    constexpr int D = L::D, S = n_slots<Q>(), NS = 1 + NSP;
    constexpr double c1[5] = {1.0 / 12.0, -8.0 / 12.0, 0.0, 8.0 / 12.0, -1.0 / 12.0};
    constexpr double c2[5] = {-1.0 / 12.0, 16.0 / 12.0, -30.0 / 12.0, 16.0 / 12.0, -1.0 / 12.0};
    const double c0 = P.T_ref_over_W_ref;
    const long long c_self = in.cell[0];
    const double *mid = out.mid + c_self;
    double ls[NS], u[3] = {0.0, 0.0, 0.0}, lgrad[3] = {0.0, 0.0, 0.0};
#pragma unroll
    for (int o = 0; o < NS; ++o) ls[o] = mid[(long long)(M::ls + o) * P.N];
#pragma unroll
    for (int d = 0; d < D; ++d) {
        lgrad[d] = mid[(long long)(M::lgrad + d) * P.N];
        u[d] = mid[(long long)(M::u + d) * P.N];
    }
    double aT0 = mid[(long long)M::aT0 * P.N], aY0[NSP];
#pragma unroll
    for (int k = 0; k < NSP; ++k) aY0[k] = mid[(long long)(M::aY0 + k) * P.N];
    double lR0 = mid[(long long)M::lR0 * P.N];
    const double lCT = -out.lo_sc[c_self];
    double lCY[NSP];
#pragma unroll
    for (int k = 0; k < NSP; ++k) lCY[k] = -out.lo_sc[(long long)(1 + k) * P.N + c_self];

    double T[S], Y[S][NSP], R[S], Sw[S];
    fill_stencil<Q, NSP>(P, in, T, Y, R, Sw);
    const double inv_rho = rcp(R[0]);
    const double ldT = P.alpha * ls[0];
    double ldY[NSP];
#pragma unroll
    for (int k = 0; k < NSP; ++k) ldY[k] = P.alpha * ls[1 + k];
    double linv_rho = 0.0;

    // the axes, reversed; each axis's four slots finished and scattered
#pragma unroll
    for (int d = 0; d < D; ++d) {
        const int sl[5] = {1 + 4 * d, 2 + 4 * d, 0, 3 + 4 * d, 4 + 4 * d};
        bool near = false;
#pragma unroll
        for (int j = 0; j < 5; ++j) near |= in.kind[sl[j]] != kFluid;
        // adjoints of the stencil's T, Y, rho (index 2: the cell, accumulated
        // into aT0, aY0, lR0 at the end of the axis)
        double aT[5] = {0.0, 0.0, 0.0, 0.0, 0.0}, aY[5][NSP], lR[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
        double aTw[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int j = 0; j < 5; ++j)
#pragma unroll
            for (int k = 0; k < NSP; ++k) aY[j][k] = 0.0;
        // wall heat flux q += 2 alpha rho(Tw, Y0) (T0 - Tw), rho(Tw, Y0) = c0 / (Tw Sw0)
#pragma unroll
        for (int j = 1; j <= 3; j += 2)
            if (in.kind[sl[j]] == kIso && wq != 0.0) {
                const double Tw = in.Tw[sl[j]], rw = c0 * rcp(Tw * Sw[0]), f = 2.0 * P.alpha * wq;
                aT0 += f * rw;
                aTw[j] += f * (-rw * rcp(Tw) * (T[0] - Tw) - rw);
                const double rwS = rw * rcp(Sw[0]);
#pragma unroll
                for (int k = 0; k < NSP; ++k) aY0[k] += f * (T[0] - Tw) * (-rwS * P.invW[k]);
            }
        const double d1r = d1(R[sl[0]], R[sl[1]], R[sl[2]], R[sl[3]], R[sl[4]]);
        double ld1r = lgrad[d];
        // diffusion: d2(phi) + d1r d1(phi) / rho
        {
            const double dT1 = d1(T[sl[0]], T[sl[1]], T[sl[2]], T[sl[3]], T[sl[4]]);
#pragma unroll
            for (int j = 0; j < 5; ++j) aT[j] += ldT * (c2[j] + d1r * inv_rho * c1[j]);
            ld1r += ldT * dT1 * inv_rho;
            linv_rho += ldT * d1r * dT1;
        }
#pragma unroll
        for (int k = 0; k < NSP; ++k) {
            const double dY1 = d1(Y[sl[0]][k], Y[sl[1]][k], Y[sl[2]][k], Y[sl[3]][k], Y[sl[4]][k]);
#pragma unroll
            for (int j = 0; j < 5; ++j) aY[j][k] += ldY[k] * (c2[j] + d1r * inv_rho * c1[j]);
            ld1r += ldY[k] * dY1 * inv_rho;
            linv_rho += ldY[k] * d1r * dY1;
        }
        // convection of T: CT += u_d cT_d, cT_d from the stencil
        {
            const double lc = lCT * u[d];
            if (near) {
                aT[3] += 0.5 * lc;
                aT[1] -= 0.5 * lc;
            } else {
                weno3_adj(T[sl[0]], T[sl[1]], T[sl[2]], T[sl[3]], T[sl[4]], u[d], lc, aT);
            }
        }
        // convection of Y: CY_k += u_d (cY_k - Y0_k sumc), sumc = sum_k cY_k
        double lsumc = 0.0;
#pragma unroll
        for (int k = 0; k < NSP; ++k) lsumc -= lCY[k] * u[d] * Y[0][k];
#pragma unroll
        for (int k = 0; k < NSP; ++k) {
            const double lc = lCY[k] * u[d] + lsumc;
            if (near) {
                aY[3][k] += 0.5 * lc;
                aY[1][k] -= 0.5 * lc;
            } else {
                double l5[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
                weno3_adj(Y[sl[0]][k], Y[sl[1]][k], Y[sl[2]][k], Y[sl[3]][k], Y[sl[4]][k], u[d], lc, l5);
#pragma unroll
                for (int j = 0; j < 5; ++j) aY[j][k] += l5[j];
            }
        }
        // d1r = d1(R)
#pragma unroll
        for (int j = 0; j < 5; ++j) lR[j] += ld1r * c1[j];

        // ghosts of this axis onto their images (the cell, j = 2, or a first
        // neighbour, j = 1 or 3) and their wall temperatures
#pragma unroll
        for (int j = 0; j < 5; ++j) {
            if (j == 2) continue;
            const int s = sl[j], kd = in.kind[s];
            if (kd == kFluid) continue;
            const int im = in.img[s];
            // local index of the image: slot img_lo(s) is j = 1, img_hi(s) is j = 3
            const bool second = j == 0 || j == 4;
            const bool ia = second && im == img_lo(s), ib = second && !ia && im == img_hi(s);
            const int li = ia ? 1 : ib ? 3 : 2;
            const double fa = ia ? 1.0 : 0.0, fb = ib ? 1.0 : 0.0;
            const double Swi = fa * Sw[sl[1]] + fb * Sw[sl[3]] + (1.0 - fa - fb) * Sw[0];
            double gT, gY[NSP], gR;  // what the image receives
            if (kd == kIso) {
                const double Tw = in.Tw[s], rw = c0 * rcp(Tw * Swi), rwS = rw * rcp(Swi);
                aTw[j] += 2.0 * aT[j] + 2.0 * lR[j] * (-rw * rcp(Tw));
                gT = -aT[j];
#pragma unroll
                for (int k = 0; k < NSP; ++k) gY[k] = aY[j][k] + 2.0 * lR[j] * (-rwS * P.invW[k]);
                gR = -lR[j];
            } else if (kd == kInflow) {
                gT = -aT[j];
#pragma unroll
                for (int k = 0; k < NSP; ++k) gY[k] = -aY[j][k];
                gR = -lR[j];
            } else {
                gT = aT[j];
#pragma unroll
                for (int k = 0; k < NSP; ++k) gY[k] = aY[j][k];
                gR = lR[j];
            }
            aT[1] += li == 1 ? gT : 0.0;
            aT[3] += li == 3 ? gT : 0.0;
            aT[2] += li == 2 ? gT : 0.0;
            lR[1] += li == 1 ? gR : 0.0;
            lR[3] += li == 3 ? gR : 0.0;
            lR[2] += li == 2 ? gR : 0.0;
#pragma unroll
            for (int k = 0; k < NSP; ++k) {
                aY[1][k] += li == 1 ? gY[k] : 0.0;
                aY[3][k] += li == 3 ? gY[k] : 0.0;
                aY[2][k] += li == 2 ? gY[k] : 0.0;
            }
            if (kd == kIso && in.wall[s] >= 0) atomicAdd(&out.dwallT[in.wall[s]], aTw[j]);
        }
        // the axis's fluid slots: densities R = c0 / (T Sw) onto T and Y; what
        // each slot's cell receives, stored for the gather (0 at ghost slots)
#pragma unroll
        for (int j = 0; j < 5; ++j) {
            if (j == 2) continue;
            const int s = sl[j];
            const bool fl = in.kind[s] == kFluid;
            const double rT = fl ? R[s] * rcp(T[s]) : 0.0, rS = fl ? R[s] * rcp(Sw[s]) : 0.0;
            double *nb = out.nb + (long long)(s - 1) * NS * P.N + c_self;
            nb[0] = fl ? aT[j] - lR[j] * rT : 0.0;
#pragma unroll
            for (int k = 0; k < NSP; ++k) nb[(long long)(1 + k) * P.N] = fl ? aY[j][k] - lR[j] * rS * P.invW[k] : 0.0;
        }
        aT0 += aT[2];
        lR0 += lR[2];
#pragma unroll
        for (int k = 0; k < NSP; ++k) aY0[k] += aY[2][k];
    }

    // inv_rho = 1 / rho; the cell's own slot
    lR0 -= linv_rho * inv_rho * inv_rho;
    const double rT0 = R[0] * rcp(T[0]), rS0 = R[0] * rcp(Sw[0]);
    out.lam_sc[c_self] = aT0 - lR0 * rT0;
#pragma unroll
    for (int k = 0; k < NSP; ++k) out.lam_sc[(long long)(1 + k) * P.N + c_self] = aY0[k] - lR0 * rS0 * P.invW[k];
}

struct AdjParams {
    KParams k;              // pop_in / sc_in: the state of level n
    const double *lam_pop_next;  // [Q][N] adjoint of the populations written by step n
    const double *lam_sc_next;   // [1+NSP][N]
    double *lam_pop;        // [Q][N] adjoint of level n (stored at every fluid cell's entries)
    double *lam_sc;         // [1+NSP][N] (stored at every fluid cell)
    double *dwallT;         // [N] dJ/d wall_T (accumulated)
    double *dparam;         // [2 n_rx]: dJ/dA_j, dJ/dTa_j (accumulated)
    double *mid;            // [AdjMid::n][N] between the first two kernels
    double *nb;             // [S - 1][1+NSP][N] from the stencil kernel to the gather
    int obj_kind;           // LBFD_OBJ_*
    double obj_w;           // weight of this level's q (flame position: times dq/dT of a cell)
};

template <int Q, int NSP>
__global__ void __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(2))) adjoint_collision_kernel(const AdjParams AP)
{
    const KParams &P = AP.k;
    const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    __shared__ double red[2 * LBFD_MAX_REACTIONS];
    __shared__ double tab[kExpTabN];
    for (int j = threadIdx.x; j < 2 * LBFD_MAX_REACTIONS; j += blockDim.x) red[j] = 0.0;
    for (int j = threadIdx.x; j < kExpTabN; j += blockDim.x) tab[j] = kExp2Tab[j];
    __syncthreads();
    if (idx < P.N && P.mask[idx] == LBFD_FLUID) {
        const int x = (int)(idx % P.nx), y = (int)((idx / P.nx) % P.ny), z = (int)(idx / ((long long)P.nx * P.ny));
        CellIn<Q, NSP> in;
        gather_inputs<Q, NSP>(P, x, y, z, idx, in);
        const double wT0 = AP.obj_kind == LBFD_OBJ_FLAME_POSITION ? AP.obj_w : 0.0;
        AdjOut o{AP.lam_pop_next, AP.lam_sc_next, AP.lam_pop, AP.lam_sc, AP.dwallT, red, AP.mid, AP.nb};
        cell_vjp_collision<Q, NSP>(P, in, wT0, tab, o);
    }
    __syncthreads();
    for (int j = threadIdx.x; j < 2 * P.n_rx; j += blockDim.x)
        if (red[j] != 0.0) atomicAdd(&AP.dparam[j], red[j]);
}

template <int Q, int NSP>
__global__ void __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(2))) adjoint_stencil_kernel(const AdjParams AP)
{
    const KParams &P = AP.k;
    const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= P.N || P.mask[idx] != LBFD_FLUID) return;
    const int x = (int)(idx % P.nx), y = (int)((idx / P.nx) % P.ny), z = (int)(idx / ((long long)P.nx * P.ny));
    CellIn<Q, NSP> in;
    gather_inputs<Q, NSP, false>(P, x, y, z, idx, in);
    const double wq = AP.obj_kind == LBFD_OBJ_WALL_HEAT_FLUX ? AP.obj_w : 0.0;
    AdjOut o{AP.lam_pop_next, AP.lam_sc_next, AP.lam_pop, AP.lam_sc, AP.dwallT, nullptr, AP.mid, AP.nb};
    cell_vjp_stencil<Q, NSP>(P, in, wq, o);
}

// The stencil scalars' adjoints: each fluid cell adds to its own share (in
// lam_sc) what the cells whose stencils hold it stored for it, slot by slot
// in a fixed order (so the sums do not depend on scheduling).  The cell
// whose slot s (offset m along axis d) is this cell sits at -m along d;
// at a wall or outside the box nothing is added, and a ghost slot stored 0.
template <int Q, int NSP>
__global__ void __launch_bounds__(kBlock) adjoint_gather_kernel(const AdjParams AP)
{
    constexpr int S = n_slots<Q>(), NS = 1 + NSP;
    const KParams &P = AP.k;
    const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= P.N || P.mask[idx] != LBFD_FLUID) return;
    const int x = (int)(idx % P.nx), y = (int)((idx / P.nx) % P.ny), z = (int)(idx / ((long long)P.nx * P.ny));
    const bool interior = P.code[idx] == kCodeInterior;
    const long long st[3] = {1, P.nx, (long long)P.nx * P.ny};
    double acc[NS];
#pragma unroll
    for (int v = 0; v < NS; ++v) acc[v] = AP.lam_sc[(long long)v * P.N + idx];
#pragma unroll
    for (int s = 1; s < S; ++s) {
        const int d = (s - 1) / 4, j = (s - 1) % 4;
        const int mm = j == 0 ? -2 : j == 1 ? -1 : j == 2 ? 1 : 2;
        long long src = idx - mm * st[d];
        bool ok = true;
        if (!interior) {
            const Nb c = classify(P, x - (d == 0 ? mm : 0), y - (d == 1 ? mm : 0), z - (d == 2 ? mm : 0));
            ok = c.kind == kFluid;
            src = ok ? c.idx : idx;
        }
        const double *nb = AP.nb + (long long)(s - 1) * NS * P.N + src;
#pragma unroll
        for (int v = 0; v < NS; ++v) acc[v] += ok ? nb[(long long)v * P.N] : 0.0;
    }
#pragma unroll
    for (int v = 0; v < NS; ++v) AP.lam_sc[(long long)v * P.N + idx] = acc[v];
}

struct TanParams {
    KParams k;               // pop_in / sc_in: the state of level n
    const double *dpop;      // [Q][N] tangent of the populations read by the step
    const double *dsc;       // [1+NSP][N] tangent of T, Y
    const double *dwallT;    // [N] tangent of the wall temperatures
    const double *dparam;    // [2 n_rx] tangents of A_j, Ta_j
    double *dpop_out;        // [Q][N] tangent of the populations written (fluid cells)
    double *dsc_out;         // [1+NSP][N] tangent of T, Y written (fluid cells)
    double *dq;              // tangent of this level's q (accumulated)
    int obj_kind;
    double obj_w;            // flame position: dq/dT of a cell
};

template <int Q, int NSP>
__global__ void __launch_bounds__(kBlock) tangent_kernel(const TanParams TP)
{
    using S = Slots<Q, NSP>;
    const KParams &P = TP.k;
    const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= P.N || P.mask[idx] != LBFD_FLUID) return;
    const int x = (int)(idx % P.nx), y = (int)((idx / P.nx) % P.ny), z = (int)(idx / ((long long)P.nx * P.ny));
    CellIn<Q, NSP> in;
    gather_inputs<Q, NSP>(P, x, y, z, idx, in);
    double tan[S::param + 2 * LBFD_MAX_REACTIONS];
    for (int i = 0; i < Q; ++i) tan[S::pull + i] = TP.dpop[(long long)in.tdir[i] * P.N + in.tcell[i]];
    for (int s = 0; s < S::S; ++s) {
        const bool fl = in.kind[s] == kFluid;
        for (int v = 0; v < 1 + NSP; ++v)
            tan[S::scal + s * (1 + NSP) + v] = fl ? TP.dsc[(long long)v * P.N + in.cell[s]] : 0.0;
        tan[S::wall + s] = (in.kind[s] == kIso && in.wall[s] >= 0) ? TP.dwallT[in.wall[s]] : 0.0;
    }
    for (int j = 0; j < 2 * P.n_rx; ++j) tan[S::param + j] = TP.dparam[j];
    Dual out[Q + 1 + NSP], qc;
    cell_eval<Q, NSP>(P, in, tan, out, qc);
    for (int i = 0; i < Q; ++i) TP.dpop_out[(long long)i * P.N + idx] = out[i].d[0];
    for (int k = 0; k < 1 + NSP; ++k) TP.dsc_out[(long long)k * P.N + idx] = out[Q + k].d[0];
    const double dq = TP.obj_kind == LBFD_OBJ_WALL_HEAT_FLUX ? qc.d[0] : TP.obj_w * tan[S::scal];
    if (dq != 0.0) atomicAdd(TP.dq, dq);
}

bool adjoint_supported(int Q, int nsp) { return (Q == 9 && nsp == 4) || (Q == 27 && nsp == 4); }

int adjoint_mid_fields(int Q, int nsp)
{
    if (nsp != 4) return 0;
    const int mid = Q == 9 ? AdjMid<2, 4>::n : Q == 27 ? AdjMid<3, 4>::n : 0;
    const int nb = Q == 9 ? (n_slots<9>() - 1) * 5 : Q == 27 ? (n_slots<27>() - 1) * 5 : 0;
    return mid + nb;
}

hipError_t launch_adjoint(int Q, int nsp, const KParams &kp, const double *lam_pop_next, const double *lam_sc_next,
                          double *lam_pop, double *lam_sc, double *dwallT, double *dparam, double *mid, int obj_kind,
                          double obj_w, hipStream_t s)
{
    AdjParams ap;
    ap.k = kp;
    ap.lam_pop_next = lam_pop_next;
    ap.lam_sc_next = lam_sc_next;
    ap.lam_pop = lam_pop;
    ap.lam_sc = lam_sc;
    ap.dwallT = dwallT;
    ap.dparam = dparam;
    ap.mid = mid;
    ap.nb = mid + (size_t)(Q == 9 ? AdjMid<2, 4>::n : AdjMid<3, 4>::n) * kp.N;
    ap.obj_kind = obj_kind;
    ap.obj_w = obj_w;
    const unsigned nb = (unsigned)((kp.N + kBlock - 1) / kBlock);
    if (Q == 9 && nsp == 4) {
        adjoint_collision_kernel<9, 4><<<nb, kBlock, 0, s>>>(ap);
        adjoint_stencil_kernel<9, 4><<<nb, kBlock, 0, s>>>(ap);
        adjoint_gather_kernel<9, 4><<<nb, kBlock, 0, s>>>(ap);
    } else if (Q == 27 && nsp == 4) {
        adjoint_collision_kernel<27, 4><<<nb, kBlock, 0, s>>>(ap);
        adjoint_stencil_kernel<27, 4><<<nb, kBlock, 0, s>>>(ap);
        adjoint_gather_kernel<27, 4><<<nb, kBlock, 0, s>>>(ap);
    } else {
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_tangent(int Q, int nsp, const KParams &kp, const double *dpop, const double *dsc,
                          const double *dwallT, const double *dparam, double *dpop_out, double *dsc_out, double *dq,
                          int obj_kind, double obj_w, hipStream_t s)
{
    TanParams tp;
    tp.k = kp;
    tp.dpop = dpop;
    tp.dsc = dsc;
    tp.dwallT = dwallT;
    tp.dparam = dparam;
    tp.dpop_out = dpop_out;
    tp.dsc_out = dsc_out;
    tp.dq = dq;
    tp.obj_kind = obj_kind;
    tp.obj_w = obj_w;
    const unsigned nb = (unsigned)((kp.N + kBlock - 1) / kBlock);
    if (Q == 9 && nsp == 4)
        tangent_kernel<9, 4><<<nb, kBlock, 0, s>>>(tp);
    else if (Q == 27 && nsp == 4)
        tangent_kernel<27, 4><<<nb, kBlock, 0, s>>>(tp);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

__global__ void fill_kernel(double *dst, int n, double v)
{
    const int i = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    if (i < n) dst[i] = v;
}

hipError_t launch_fill(double *dst, int n, double v, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    fill_kernel<<<(n + kBlock - 1) / kBlock, kBlock, 0, s>>>(dst, n, v);
    return hipGetLastError();
}

}  // namespace lbfd
