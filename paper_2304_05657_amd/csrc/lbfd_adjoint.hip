// lbfd_adjoint.hip -- discrete adjoint of the coupled step (FP64).
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
// One thread per fluid cell c evaluates the cell's update (the forward
// step's formulas, in the general geometry path: neighbours classified on
// the fly, each stencil point and density evaluated separately) in dual
// numbers, once per input slot of the cell (pull source,
// stencil scalar, wall temperature, Arrhenius parameter) with a unit tangent
// on that slot; the tangent of the outputs dotted with the cell's output
// adjoint is that slot's contribution, added atomically to the adjoint of
// the variable behind the slot.  Steps are recomputed from checkpoints
// taken every K steps (host side, lbfd_api.hip).
#include <hip/hip_runtime.h>

#include "lbfd_kernels.h"

namespace lbfd {

// ----------------------------------------------------------- dual numbers
struct Dual {
    double v, d;
    __host__ __device__ Dual() : v(0.0), d(0.0) {}
    __host__ __device__ Dual(double x) : v(x), d(0.0) {}
    __host__ __device__ Dual(double x, double dx) : v(x), d(dx) {}
    __host__ __device__ explicit operator double() const { return v; }
    __device__ Dual &operator+=(const Dual &b) { v += b.v; d += b.d; return *this; }
    __device__ Dual &operator-=(const Dual &b) { v -= b.v; d -= b.d; return *this; }
    __device__ Dual &operator*=(const Dual &b) { d = d * b.v + v * b.d; v *= b.v; return *this; }
};
__device__ inline Dual operator+(Dual a, Dual b) { return Dual(a.v + b.v, a.d + b.d); }
__device__ inline Dual operator-(Dual a, Dual b) { return Dual(a.v - b.v, a.d - b.d); }
__device__ inline Dual operator-(Dual a) { return Dual(-a.v, -a.d); }
__device__ inline Dual operator*(Dual a, Dual b) { return Dual(a.v * b.v, a.d * b.v + a.v * b.d); }
__device__ inline Dual operator/(Dual a, Dual b)
{
    const double q = a.v / b.v;
    return Dual(q, (a.d - q * b.d) / b.v);
}
__device__ inline Dual rcp(Dual a)
{
    const double r = rcp(a.v);
    return Dual(r, -a.d * r * r);
}
__device__ inline bool operator<(Dual a, Dual b) { return a.v < b.v; }
__device__ inline bool operator>(Dual a, Dual b) { return a.v > b.v; }
__device__ inline bool operator>=(Dual a, Dual b) { return a.v >= b.v; }
__device__ inline bool operator<=(Dual a, Dual b) { return a.v <= b.v; }
// the exponential of the forward chemistry (exp_tab)
__device__ inline Dual dexp(Dual a)
{
    const double e = exp_tab(a.v, kExp2Tab);
    return Dual(e, e * a.d);
}
__device__ inline double dexp(double a) { return exp_tab(a, kExp2Tab); }
__device__ inline Dual dlog(Dual a) { return Dual(log(a.v), a.d * rcp(a.v)); }
__device__ inline double dlog(double a) { return log(a); }
__device__ inline double val(Dual a) { return a.v; }
__device__ inline double val(double a) { return a; }
__device__ inline double tan_(Dual a) { return a.d; }

// ------------------------------------------------------------ cell inputs
// Stencil slots: 0 = the cell, 1 + 4 d + j for axis d and m = -2, -1, 1, 2.
constexpr int kSlots = 13;

template <int Q, int NSP>
struct CellIn {
    double g[Q];          // pulled populations (without the inlet correction)
    double corr[Q];       // inlet correction added to the pull
    int tdir[Q], tcell[Q];  // population entry each pull read
    double T[kSlots], Y[NSP][kSlots];
    int cell[kSlots];     // fluid slot: its cell; ghost slot: -1
    int kind[kSlots];     // kFluid or the kind of the wall behind the ghost
    int img[kSlots];      // ghost slot: slot of its image point
    double Tw[kSlots];    // ghost slot: wall temperature
    int wall[kSlots];     // ghost slot behind an isothermal in-box solid: its cell, else -1
};

template <int Q, int NSP>
__device__ void gather_inputs(const KParams &P, int x, int y, int z, long long idx, CellIn<Q, NSP> &in)
{
    using L = Lat<Q>;
    constexpr int D = L::D;
    const double *pop = (const double *)P.pop_in;
    const double *sc = (const double *)P.sc_in;
    for (int i = 0; i < Q; ++i) {
        const int cx = i % 3 - 1, cy = (i / 3) % 3 - 1, cz = Q == 9 ? 0 : i / 9 - 1;
        const int opp = Q - 1 - i;
        in.corr[i] = 0.0;
        if (cx == 0 && cy == 0 && cz == 0) {
            in.tdir[i] = i;
            in.tcell[i] = (int)idx;
        } else {
            const Nb s = classify(P, x - cx, y - cy, z - cz);
            if (s.kind == kFluid) {
                in.tdir[i] = i;
                in.tcell[i] = (int)s.idx;
            } else {
                in.tdir[i] = opp;
                in.tcell[i] = (int)idx;
                if (s.kind == kInflow) in.corr[i] = 2.0 * L::w(i) * P.rho_in * inflow_cu_c(P, cx, cy, cz, x, y, z);
            }
        }
        in.g[i] = pop[(long long)in.tdir[i] * P.N + in.tcell[i]];
    }
    auto load = [&](int s, long long c) {
        in.cell[s] = (int)c;
        in.kind[s] = kFluid;
        in.img[s] = -1;
        in.Tw[s] = 0.0;
        in.wall[s] = -1;
        in.T[s] = sc[c];
        for (int k = 0; k < NSP; ++k) in.Y[k][s] = sc[(1 + k) * P.N + c];
    };
    auto ghost_slot = [&](int s, const Nb &w, int image) {
        in.cell[s] = -1;
        in.kind[s] = w.kind;
        in.img[s] = image;
        in.Tw[s] = w.Tw;
        in.wall[s] = (w.kind == kIso && w.face < 0) ? (int)w.idx : -1;
        in.T[s] = 0.0;
        for (int k = 0; k < NSP; ++k) in.Y[k][s] = 0.0;
    };
    load(0, idx);
    for (int d = 0; d < 3; ++d) {
        for (int sg = -1; sg <= 1; sg += 2) {
            const int j1 = sg < 0 ? 1 : 2, j2 = sg < 0 ? 0 : 3;
            const int s1 = 1 + 4 * d + j1, s2 = 1 + 4 * d + j2, sm = 1 + 4 * d + (sg < 0 ? 2 : 1);
            if (d >= D) {
                load(s1, idx);
                load(s2, idx);
                continue;
            }
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

// Input slot numbering for seeding: [0, Q) pulls; then kSlots x (1 + NSP)
// stencil scalars (T, Y_k); then kSlots ghost wall temperatures; then
// (A_j, Ta_j) per reaction.
template <int Q, int NSP>
struct Slots {
    static constexpr int pull = 0;
    static constexpr int scal = Q;
    static constexpr int wall = Q + kSlots * (1 + NSP);
    static constexpr int param = wall + kSlots;
};

template <int NSP, class A>
__device__ A density_a(const KParams &P, A T, const A (&Y)[NSP])
{
    A s = 0.0;
    for (int k = 0; k < NSP; ++k) s += Y[k] * A(P.invW[k]);
    return A(P.T_ref_over_W_ref) / (T * s);
}

// The cell's update in the number type A (double or Dual), seeded at slot
// `seed`: outputs out[0..Q) = g*, out[Q] = T^{n+1}, out[Q+1+k] = Y_k^{n+1};
// *qc = the cell's wall-heat-flux contribution at level n.
template <int Q, int NSP, class A>
__device__ void cell_eval(const KParams &P, const CellIn<Q, NSP> &in, int seed, A (&out)[Q + 1 + NSP], A &qc)
{
    using L = Lat<Q>;
    using S = Slots<Q, NSP>;
    constexpr int D = L::D;
    auto mk = [&](double v, int slot) -> A {
        if constexpr (std::is_same<A, Dual>::value)
            return Dual(v, slot == seed ? 1.0 : 0.0);
        else
            return v;
    };
    A g[Q];
    for (int i = 0; i < Q; ++i) g[i] = mk(in.g[i], S::pull + i) + A(in.corr[i]);
    A T[kSlots], Y[kSlots][NSP], R[kSlots], Tw[kSlots];
    for (int s = 0; s < kSlots; ++s) {
        Tw[s] = mk(in.Tw[s], S::wall + s);
        if (in.kind[s] == kFluid) {
            T[s] = mk(in.T[s], S::scal + s * (1 + NSP));
            A Ys[NSP];
            for (int k = 0; k < NSP; ++k) {
                Y[s][k] = mk(in.Y[k][s], S::scal + s * (1 + NSP) + 1 + k);
                Ys[k] = Y[s][k];
            }
            R[s] = density_a<NSP>(P, T[s], Ys);
        }
    }
    // ghosts (Sec. III.B): images are fluid slots
    for (int s = 0; s < kSlots; ++s) {
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
    A sg = 0.0, m[3] = {0.0, 0.0, 0.0};
    for (int i = 0; i < Q; ++i) {
        sg += g[i];
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

    // Arrhenius source (same sub-stepping and limiter as the forward)
    A srcT = 0.0, srcY[NSP];
    {
        // rate coefficients k_j = A_j dt exp(b_j ln T - Ta_j / T), ln T and
        // 1/T shared by the reactions, as in the forward chemistry()
        const A Tc0 = T[0];
        const bool anyb = P.chem_anyb != 0;
        int nsub = 1;
        if (P.chem_substeps_max > 1) {
            const double lnT = anyb ? log(val(Tc0)) : 0.0, invT = rcp(val(Tc0));
            double kmax = 0.0;
            for (int j = 0; j < P.n_rx; ++j) kmax = fmax(kmax, rate_coeff_l(P.rxk[j], lnT, invT, kExp2Tab));
            const double want = ceil(kmax / 0.1);
            nsub = want < 1.0 ? 1 : want > (double)P.chem_substeps_max ? P.chem_substeps_max : (int)want;
        }
        const double inv_nsub = nsub == 1 ? 1.0 : rcp((double)nsub);
        A dT = 0.0, dY[NSP];
        for (int k = 0; k < NSP; ++k) dY[k] = 0.0;
        for (int s = 0; s < nsub; ++s) {
            const A Tc = Tc0 + dT;
            A Yc[NSP], incT = 0.0, incY[NSP];
            for (int k = 0; k < NSP; ++k) {
                Yc[k] = Y[0][k] + dY[k];
                incY[k] = 0.0;
            }
            const A lnTc = anyb ? dlog(Tc) : A(0.0), invTc = rcp(Tc);
            for (int j = 0; j < P.n_rx; ++j) {
                const lbfd_reaction &r = P.rx[j];
                const A Aj = mk(r.A, S::param + 2 * j), Taj = mk(r.Ta, S::param + 2 * j + 1);
                A rr = Aj * A(P.dt_phys) * dexp(A(r.b) * lnTc - Taj * invTc) * A(inv_nsub);
                for (int mm = 0; mm < r.n_react; ++mm) rr *= Yc[r.react[mm]];
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

struct AdjParams {
    KParams k;              // pop_in / sc_in: the state of level n
    const double *lam_pop_next;  // [Q][N] adjoint of the populations written by step n
    const double *lam_sc_next;   // [1+NSP][N]
    double *lam_pop;        // [Q][N] adjoint of level n (accumulated)
    double *lam_sc;         // [1+NSP][N]
    double *dwallT;         // [N] dJ/d wall_T (accumulated)
    double *dparam;         // [2 n_rx]: dJ/dA_j, dJ/dTa_j (accumulated)
    int obj_kind;           // LBFD_OBJ_*
    double obj_w;           // weight of this level's q (flame position: times dq/dT of a cell)
};

template <int Q, int NSP>
__global__ void __launch_bounds__(kBlock) adjoint_kernel(const AdjParams AP)
{
    using S = Slots<Q, NSP>;
    const KParams &P = AP.k;
    const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    __shared__ double red[2 * LBFD_MAX_REACTIONS];
    for (int j = threadIdx.x; j < 2 * LBFD_MAX_REACTIONS; j += blockDim.x) red[j] = 0.0;
    __syncthreads();
    if (idx < P.N && P.mask[idx] == LBFD_FLUID) {
        const int x = (int)(idx % P.nx), y = (int)((idx / P.nx) % P.ny), z = (int)(idx / ((long long)P.nx * P.ny));
        CellIn<Q, NSP> in;
        gather_inputs<Q, NSP>(P, x, y, z, idx, in);
        double lam_out[Q + 1 + NSP];
        for (int i = 0; i < Q; ++i) lam_out[i] = AP.lam_pop_next[(long long)i * P.N + idx];
        for (int k = 0; k < 1 + NSP; ++k) lam_out[Q + k] = AP.lam_sc_next[(long long)k * P.N + idx];
        const int nslots = S::param + 2 * P.n_rx;
        const int D = Lat<Q>::D;
        for (int seed = 0; seed < nslots; ++seed) {
            // skip slots with no variable behind them
            if (seed >= S::scal && seed < S::wall) {
                const int s = (seed - S::scal) / (1 + NSP);
                if (in.kind[s] != kFluid || (s > 0 && (s - 1) / 4 >= D)) continue;
            } else if (seed >= S::wall && seed < S::param) {
                const int s = seed - S::wall;
                if (in.kind[s] != kIso || in.wall[s] < 0) continue;
            }
            Dual out[Q + 1 + NSP], qc;
            cell_eval<Q, NSP, Dual>(P, in, seed, out, qc);
            // the objective's share: the wall heat flux through this cell's
            // walls, or the flame position's linear term in the cell's own T
            double contrib = AP.obj_kind == LBFD_OBJ_WALL_HEAT_FLUX ? AP.obj_w * qc.d
                             : seed == S::scal                      ? AP.obj_w
                                                                    : 0.0;
            for (int o = 0; o < Q + 1 + NSP; ++o) contrib += lam_out[o] * out[o].d;
            if (seed < S::scal) {
                atomicAdd(&AP.lam_pop[(long long)in.tdir[seed] * P.N + in.tcell[seed]], contrib);
            } else if (seed < S::wall) {
                const int s = (seed - S::scal) / (1 + NSP), var = (seed - S::scal) % (1 + NSP);
                atomicAdd(&AP.lam_sc[(long long)var * P.N + in.cell[s]], contrib);
            } else if (seed < S::param) {
                atomicAdd(&AP.dwallT[in.wall[seed - S::wall]], contrib);
            } else {
                atomicAdd(&red[seed - S::param], contrib);
            }
        }
    }
    __syncthreads();
    for (int j = threadIdx.x; j < 2 * P.n_rx; j += blockDim.x)
        if (red[j] != 0.0) atomicAdd(&AP.dparam[j], red[j]);
}

__global__ void accumulate_kernel(double *acc, const double *diag, int slot, double a, double b)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) *acc += a * diag[slot] + b;
}

bool adjoint_supported(int Q, int nsp) { return (Q == 9 && nsp == 4) || (Q == 27 && nsp == 4); }

hipError_t launch_adjoint(int Q, int nsp, const KParams &kp, const double *lam_pop_next, const double *lam_sc_next,
                          double *lam_pop, double *lam_sc, double *dwallT, double *dparam, int obj_kind,
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
    ap.obj_kind = obj_kind;
    ap.obj_w = obj_w;
    const unsigned nb = (unsigned)((kp.N + kBlock - 1) / kBlock);
    if (Q == 9 && nsp == 4)
        adjoint_kernel<9, 4><<<nb, kBlock, 0, s>>>(ap);
    else if (Q == 27 && nsp == 4)
        adjoint_kernel<27, 4><<<nb, kBlock, 0, s>>>(ap);
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

hipError_t launch_accumulate(double *acc, const double *diag, int slot, double a, double b, hipStream_t s)
{
    accumulate_kernel<<<1, 1, 0, s>>>(acc, diag, slot, a, b);
    return hipGetLastError();
}

}  // namespace lbfd
