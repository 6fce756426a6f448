/*
 * lbfd_oracle.c -- FP64 CPU oracle of the coupled LB / FD time step of
 * Hosseini & Thevenin, arXiv:2304.05657.
 *
 * TEST INFRASTRUCTURE ONLY: a plain, slow, obviously correct statement of
 * the method.  It is loaded by the test suite, the smoke check and the
 * CPU-baseline leg of the benchmark, never by the GPU library, and it
 * shares no code with it.  Where the paper is silent or garbled the
 * readings used here are listed in the repository's design notes; each is
 * also named at the place it is used ("reading: ...").
 *
 * One step n -> n+1 (all terms at level n, explicit Euler, Sec. II.D):
 *   1. density of every cell from T, Y (ideal gas at uniform P_0,
 *      Sec. II.A), in lattice units rho = (T_ref/T)(W/W_ref);
 *   2. per fluid cell: velocity moment (Eq. 13b), ghost-node values of
 *      T, Y_k, rho across walls (Sec. III.B), WENO3 / centred convection,
 *      4th-order central diffusion (Sec. II.D), Arrhenius source,
 *      Lambda (Eq. 6), P_h (Eq. 13a), source Xi_i (Eq. 9), collision in
 *      central-moment space (Sec. II.C), Euler update of T and Y_k;
 *   3. streaming with half-way bounce-back (Eq. 28), velocity inlet
 *      (Eq. 31) and non-reflecting outlet (Eq. 32).
 *
 * The inverse central-moment transform is a Gaussian elimination of the
 * full Q x Q moment matrix built from its definition (Eq. 21); nothing is
 * factorised or fused.
 */
#include "lbfd_oracle.h"

#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define CS2 (1.0 / 3.0)
#define MAXQ 27

/* kinds of the cell a stencil point or a streaming source lands on */
#define K_FLUID 0
#define K_ISO 1     /* isothermal solid or isothermal wall face */
#define K_ADIA 2    /* adiabatic solid or adiabatic wall face */
#define K_INFLOW 3
#define K_OUTFLOW 4

struct lbo_state {
    lbo_params p;
    int D, Q;
    long N;
    int c[MAXQ][3];
    double w[MAXQ];
    uint8_t *mask;
    double *wall_T;
    double *g;      /* post-streaming populations at the current level */
    double *T, *Y;  /* temperature, mass fractions at the current level */
    double *gstar;  /* post-collision populations (scratch) */
    double *Tn, *Yn, *gn;
    double *rho;    /* density of every cell at the current level */
    double *ux;     /* velocity of every fluid cell at the current level */
    long level;
    const uint8_t *active;  /* NULL, or the cells a step / fields call covers */
    double *u_face;         /* NULL, or [2 x faces][3][nz][ny] inlet velocity per face cell */
    double *q_link;         /* NULL, or [Q][N] wall distance of link (cell, i), NAN = half-way */
    long n_img;             /* image points of ghost nodes on curved walls, sorted by key */
    long *img_key;          /* cell * 12 + axis * 4 + j (offset m = -2, -1, 1, 2 for j = 0..3) */
    double *img_x;          /* [n_img][3] lattice coordinates of the image point */
};

/* Whether a fluid cell is covered by the current active set. */
static int covered(const lbo_state *s, long idx)
{
    return s->active == NULL || s->active[idx] != 0;
}

typedef struct {
    int kind;
    long idx;       /* cell index when the point is inside the box */
    double Tw;      /* wall temperature for K_ISO */
    int face;       /* face index for domain faces, else -1 */
} cellref;

/* ------------------------------------------------------------------ */
/* Lattice (Sec. II.B: first-neighbour D2Q9 and D3Q27 stencils).        */
/* Directions in lexicographic order over (c_z, c_y, c_x), x fastest;  */
/* the opposite of direction i is Q-1-i.                               */
/* ------------------------------------------------------------------ */
void lbo_lattice(int Q, int *c, double *w)
{
    int i = 0;
    int zr = (Q == 27) ? 1 : 0;
    for (int cz = -zr; cz <= zr; ++cz)
        for (int cy = -1; cy <= 1; ++cy)
            for (int cx = -1; cx <= 1; ++cx) {
                c[3 * i] = cx;
                c[3 * i + 1] = cy;
                c[3 * i + 2] = cz;
                int n2 = cx * cx + cy * cy + cz * cz;
                if (Q == 9)
                    w[i] = n2 == 0 ? 4.0 / 9.0 : n2 == 1 ? 1.0 / 9.0 : 1.0 / 36.0;
                else
                    w[i] = n2 == 0 ? 8.0 / 27.0
                         : n2 == 1 ? 2.0 / 27.0
                         : n2 == 2 ? 1.0 / 54.0
                                   : 1.0 / 216.0;
                ++i;
            }
}

/* Density equilibrium, Sec. II.B Eq. (10). */
void lbo_feq(int Q, double rho, const double *u, double *feq)
{
    int c[MAXQ * 3];
    double w[MAXQ];
    lbo_lattice(Q, c, w);
    double uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
    for (int i = 0; i < Q; ++i) {
        double cu = c[3 * i] * u[0] + c[3 * i + 1] * u[1] + c[3 * i + 2] * u[2];
        feq[i] = w[i] * rho * (1.0 + cu / CS2 + cu * cu / (2.0 * CS2 * CS2) - uu / (2.0 * CS2));
    }
}

/* Pressure-based equilibrium, Sec. II.B Eq. (12). */
void lbo_geq(int Q, double Ph, double rho, const double *u, double *geq)
{
    int c[MAXQ * 3];
    double w[MAXQ], feq[MAXQ];
    lbo_lattice(Q, c, w);
    lbo_feq(Q, rho, u, feq);
    for (int i = 0; i < Q; ++i)
        geq[i] = w[i] * (Ph - rho * CS2) + CS2 * feq[i];
}

/* Source term, Sec. II.B Eq. (9). */
void lbo_source_xi(int Q, double rho, const double *u, const double *grad_rho,
                   double Lambda, double *xi)
{
    int c[MAXQ * 3];
    double w[MAXQ], feq[MAXQ];
    lbo_lattice(Q, c, w);
    lbo_feq(Q, rho, u, feq);
    for (int i = 0; i < Q; ++i) {
        double proj = 0.0;
        for (int d = 0; d < 3; ++d)
            proj += (c[3 * i + d] - u[d]) * grad_rho[d];
        xi[i] = CS2 * (feq[i] / rho - w[i]) * proj + w[i] * rho * CS2 * Lambda;
    }
}

/* integer power for small non-negative exponents */
static double ipow(double x, int p)
{
    double r = 1.0;
    for (int k = 0; k < p; ++k)
        r *= x;
    return r;
}

/* Moment j has the exponents (c_jx+1, c_jy+1, c_jz+1), one per axis, so */
/* the Q moments enumerate {0,1,2}^D in the direction order.             */
static void moment_matrix(int Q, const double *u, double *M)
{
    int c[MAXQ * 3];
    double w[MAXQ];
    lbo_lattice(Q, c, w);
    for (int j = 0; j < Q; ++j)
        for (int i = 0; i < Q; ++i) {
            double v = 1.0;
            for (int d = 0; d < 3; ++d) {
                int pj = c[3 * j + d] + 1;
                if (Q == 9 && d == 2)
                    pj = 0;
                v *= ipow((double)c[3 * i + d] - u[d], pj);
            }
            M[j * Q + i] = v;
        }
}

/* Central moments of a distribution about u, Sec. II.C Eq. (21). */
void lbo_central_moments(int Q, const double *h, const double *u, double *kap)
{
    double M[MAXQ * MAXQ];
    moment_matrix(Q, u, M);
    for (int j = 0; j < Q; ++j) {
        double s = 0.0;
        for (int i = 0; i < Q; ++i)
            s += M[j * Q + i] * h[i];
        kap[j] = s;
    }
}

/* Solve A x = b in place (b becomes x), Gaussian elimination with      */
/* partial pivoting.                                                    */
static void gauss_solve(int n, double *A, double *b)
{
    for (int k = 0; k < n; ++k) {
        int piv = k;
        for (int r = k + 1; r < n; ++r)
            if (fabs(A[r * n + k]) > fabs(A[piv * n + k]))
                piv = r;
        if (piv != k) {
            for (int cc = 0; cc < n; ++cc) {
                double t = A[k * n + cc];
                A[k * n + cc] = A[piv * n + cc];
                A[piv * n + cc] = t;
            }
            double t = b[k];
            b[k] = b[piv];
            b[piv] = t;
        }
        for (int r = k + 1; r < n; ++r) {
            double f = A[r * n + k] / A[k * n + k];
            for (int cc = k; cc < n; ++cc)
                A[r * n + cc] -= f * A[k * n + cc];
            b[r] -= f * b[k];
        }
    }
    for (int r = n - 1; r >= 0; --r) {
        double s = b[r];
        for (int cc = r + 1; cc < n; ++cc)
            s -= A[r * n + cc] * b[cc];
        b[r] = s / A[r * n + r];
    }
}

/*
 * Collision, Sec. II.C.  Post-collision populations g*_i (Eq. 14) from
 * the pre-conditioned populations f'_i (Eq. 19), relaxed in the space of
 * central moments (Eq. 21) with the diagonal rate matrix of Eq. (16).
 *
 * Readings: the printed Eq. (15) is the identity; the relaxation used is
 * kappa* = kappa - omega (kappa - kappa_eq) with kappa_eq the central
 * moments of the Maxwellian at temperature cs^2 (kappa_0 = 1, each axis
 * with exponent 2 contributes a factor cs^2, any odd exponent gives 0),
 * or of f^eq/rho when eq_discrete is set.  Eq. (18) is the relaxation
 * time tau; every second-order moment relaxes with 1/tau, third-order
 * ones with omega3, higher ones with omega4, orders 0 and 1 are kept.
 * f' carries mass P_h/(rho cs^2) + u.grad(rho)/(2 rho), not 1, so the
 * moments are taken of h = f' + w (1 - sum f'), which has unit mass and
 * mean velocity u; the shift is undone after relaxation.
 */
/* ------------------------------------------------------------------ */
/* Cumulants (Sec. II.C).  The printed cumulant formulas are garbled    */
/* (reading: the multivariate moment-cumulant relation, derived here,   */
/* not transcribed).  A moment index j carries exponents (p, q, r) =     */
/* (c_x + 1, c_y + 1, c_z + 1) of direction j, i.e. j = p + 3q + 9r.    */
/* The multi-index a of (p, q, r) is the multiset of its p x's, q y's    */
/* and r z's; over the set partitions pi of a's positions               */
/*   C_a   = sum_pi (-1)^(|pi|-1) (|pi|-1)! prod_{B in pi} kap_B,         */
/*   kap_a = sum_pi prod_{B in pi} C_B,                                   */
/* with kap_B (C_B) the moment (cumulant) of B's exponents.  Only        */
/* orders >= 2 are transformed; orders 0 and 1 are copied.               */
/* ------------------------------------------------------------------ */
static int order_of(int j) { return j % 3 + (j / 3) % 3 + j / 9; }

/* sum over the set partitions of the first n positions of axis[] (blocks
   numbered by first appearance), each term the product of vals at the
   blocks' exponents, times (-1)^(k-1) (k-1)! for k blocks when signed */
static double partition_sum(int n, const int *axis, int pos, int *blk, int nblk,
                            const double *vals, int signed_terms)
{
    if (pos == n) {
        double prod = 1.0;
        for (int b = 0; b < nblk; ++b) {
            int e[3] = {0, 0, 0};
            for (int i = 0; i < n; ++i)
                if (blk[i] == b)
                    e[axis[i]] += 1;
            prod *= vals[e[0] + 3 * e[1] + 9 * e[2]];
        }
        if (signed_terms) {
            double cf = (nblk % 2 == 1) ? 1.0 : -1.0;
            for (int k = 2; k < nblk; ++k)
                cf *= k;
            prod *= cf;
        }
        return prod;
    }
    double s = 0.0;
    for (int b = 0; b <= nblk; ++b) {
        blk[pos] = b;
        s += partition_sum(n, axis, pos + 1, blk, b == nblk ? nblk + 1 : nblk, vals, signed_terms);
    }
    return s;
}

static double transform_one(int j, const double *vals, int signed_terms)
{
    int axis[6], blk[6], n = 0;
    int e[3] = {j % 3, (j / 3) % 3, j / 9};
    for (int d = 0; d < 3; ++d)
        for (int k = 0; k < e[d]; ++k)
            axis[n++] = d;
    return partition_sum(n, axis, 0, blk, 0, vals, signed_terms);
}

void lbo_cumulants(int Q, const double *kap, double *cum)
{
    for (int j = 0; j < Q; ++j)
        cum[j] = order_of(j) < 2 ? kap[j] : transform_one(j, kap, 1);
}

void lbo_cumulants_inverse(int Q, const double *cum, double *kap)
{
    for (int j = 0; j < Q; ++j)
        kap[j] = order_of(j) < 2 ? cum[j] : transform_one(j, cum, 0);
}

void lbo_collide(const lbo_params *p, const double *g, const double *xi,
                 double rho, const double *u, double *gstar)
{
    int Q = p->Q;
    int c[MAXQ * 3];
    double w[MAXQ], f[MAXQ], h[MAXQ], kap[MAXQ], keq[MAXQ], M[MAXQ * MAXQ];
    lbo_lattice(Q, c, w);
    double pi = 0.0;
    for (int i = 0; i < Q; ++i) {
        f[i] = g[i] / (rho * CS2) + xi[i] / (2.0 * rho * CS2);
        pi += f[i];
    }
    for (int i = 0; i < Q; ++i)
        h[i] = f[i] + w[i] * (1.0 - pi);
    lbo_central_moments(Q, h, u, kap);
    if (p->eq_discrete) {
        double feq[MAXQ];
        lbo_feq(Q, 1.0, u, feq);
        lbo_central_moments(Q, feq, u, keq);
    } else {
        for (int j = 0; j < Q; ++j) {
            double v = 1.0;
            for (int d = 0; d < 3; ++d) {
                int pj = (Q == 9 && d == 2) ? 0 : c[3 * j + d] + 1;
                v *= pj == 0 ? 1.0 : pj == 1 ? 0.0 : CS2;
            }
            keq[j] = v;
        }
    }
    if (p->collision == LBO_CUMULANTS) {
        /* relax cumulants toward those of the targets: orders 2, 3 at 1/tau
           and omega3 (equal to the central moments there), orders >= 4 at
           omega4; then back to central moments */
        double cum[MAXQ], ceq[MAXQ];
        lbo_cumulants(Q, kap, cum);
        lbo_cumulants(Q, keq, ceq);
        for (int j = 0; j < Q; ++j) {
            int order = order_of(j);
            double om = order <= 1 ? 0.0 : order == 2 ? 1.0 / p->tau : order == 3 ? p->omega3 : p->omega4;
            cum[j] = cum[j] - om * (cum[j] - ceq[j]);
        }
        lbo_cumulants_inverse(Q, cum, kap);
    } else {
        for (int j = 0; j < Q; ++j) {
            int order = 0;
            for (int d = 0; d < 3; ++d)
                order += (Q == 9 && d == 2) ? 0 : c[3 * j + d] + 1;
            double om = order <= 1 ? 0.0 : order == 2 ? 1.0 / p->tau : order == 3 ? p->omega3 : p->omega4;
            kap[j] = kap[j] - om * (kap[j] - keq[j]);
        }
    }
    moment_matrix(Q, u, M);
    gauss_solve(Q, M, kap);  /* kap now holds h* */
    for (int i = 0; i < Q; ++i) {
        double fs = kap[i] - w[i] * (1.0 - pi);
        gstar[i] = rho * CS2 * fs + 0.5 * xi[i];
    }
}

/* ------------------------------------------------------------------ */
/* Finite differences, Sec. II.D.                                      */
/* phi5 = {phi_{i-2}, phi_{i-1}, phi_i, phi_{i+1}, phi_{i+2}}.         */
/* ------------------------------------------------------------------ */

/* fourth-order central first derivative */
double lbo_d1(const double *phi5)
{
    return (phi5[0] - 8.0 * phi5[1] + 8.0 * phi5[3] - phi5[4]) / 12.0;
}

/* fourth-order central second derivative */
double lbo_d2(const double *phi5)
{
    return (-phi5[0] + 16.0 * phi5[1] - 30.0 * phi5[2] + 16.0 * phi5[3] - phi5[4]) / 12.0;
}

/* Third-order WENO (Jiang-Shu weights) value at the face between b and */
/* c, reconstructed from the side of b; a is the far upwind point.       */
static double weno_face(double a, double b, double c)
{
    const double eps = 1e-6;
    double q0 = -0.5 * a + 1.5 * b;
    double q1 = 0.5 * b + 0.5 * c;
    double b0 = (b - a) * (b - a);
    double b1 = (c - b) * (c - b);
    double a0 = (1.0 / 3.0) / ((eps + b0) * (eps + b0));
    double a1 = (2.0 / 3.0) / ((eps + b1) * (eps + b1));
    return (a0 * q0 + a1 * q1) / (a0 + a1);
}

/* WENO3 convective derivative d(phi)/dx at node i for the sign of u;  */
/* reading: the u >= 0 branch is taken at u == 0.                      */
double lbo_weno3(const double *phi5, double u)
{
    if (u >= 0.0)
        return weno_face(phi5[1], phi5[2], phi5[3]) - weno_face(phi5[0], phi5[1], phi5[2]);
    return weno_face(phi5[4], phi5[3], phi5[2]) - weno_face(phi5[3], phi5[2], phi5[1]);
}

/* ------------------------------------------------------------------ */
/* Chemistry.  Explicit Arrhenius law on mass fractions per reaction:   */
/* r_j = A_j dt_phys T^b_j exp(-Ta_j/T) prod_reactants Y, the species   */
/* source sum_j nu_jk r_j and the temperature source sum_j q_j r_j, all */
/* per lattice step.  With chem_substeps_max > 1 the source over one    */
/* step is integrated with N explicit sub-steps, N = ceil(max_j k_j/0.1)*/
/* capped at chem_substeps_max (one sub-step is the plain Euler source);*/
/* each sub-step is scaled down if it would drive a Y_k below zero.     */
/* ------------------------------------------------------------------ */
/* k = A dt T^b exp(-Ta/T), with T^b exp(-Ta/T) written as the one        */
/* exponential exp(b ln T - Ta/T) (the form every implementation of the   */
/* step uses; with b = 0 it is exp(-Ta/T) exactly).                       */
static double rate_coeff(const lbo_reaction *r, double dt_phys, double T)
{
    return r->A * dt_phys * exp(r->b * log(T) - r->Ta / T);
}

void lbo_chemistry(const lbo_params *p, double T, const double *Y,
                   double *src_T, double *src_Y)
{
    int ns = p->n_species;
    int nsub = 1;
    if (p->chem_substeps_max > 1) {
        double kmax = 0.0;
        for (int j = 0; j < p->n_reactions; ++j) {
            double k = rate_coeff(&p->rx[j], p->dt_phys, T);
            if (k > kmax)
                kmax = k;
        }
        double want = ceil(kmax / 0.1);
        nsub = want < 1.0 ? 1 : want > p->chem_substeps_max ? p->chem_substeps_max : (int)want;
    }
    double dT = 0.0, dY[LBO_MAXSP];
    for (int k = 0; k < ns; ++k)
        dY[k] = 0.0;
    for (int s = 0; s < nsub; ++s) {
        double Tc = T + dT;
        double Yc[LBO_MAXSP];
        for (int k = 0; k < ns; ++k)
            Yc[k] = Y[k] + dY[k];
        double incT = 0.0, incY[LBO_MAXSP];
        for (int k = 0; k < ns; ++k)
            incY[k] = 0.0;
        for (int j = 0; j < p->n_reactions; ++j) {
            const lbo_reaction *r = &p->rx[j];
            double rr = rate_coeff(r, p->dt_phys, Tc) / nsub;
            for (int m = 0; m < r->n_react; ++m)
                rr *= Yc[r->react[m]];
            for (int k = 0; k < ns; ++k)
                incY[k] += r->nu[k] * rr;
            incT += r->q * rr;
        }
        /* q is the temperature rise per unit mass at c_p,ref; with       */
        /* species heat capacities it is divided by c_p(Y) / c_p,ref      */
        /* (Eq. 7: omega_T / (rho c_p)) at the sub-step's composition     */
        if (p->transport == LBO_MIXTURE_AVERAGED) {
            double cpm = 0.0;
            for (int k = 0; k < ns; ++k)
                cpm += Yc[k] * p->cp[k];
            incT /= cpm;
        }
        /* positivity limiter (reading for stiff mechanisms): scale the    */
        /* sub-step so that no mass fraction is consumed below zero; it is */
        /* 1, i.e. plain explicit Euler, whenever nothing would go negative */
        double lam = 1.0;
        for (int k = 0; k < ns; ++k)
            if (incY[k] < 0.0 && Yc[k] + incY[k] < 0.0) {
                double l = (Yc[k] > 0.0 ? Yc[k] : 0.0) / (-incY[k]);
                if (l < lam)
                    lam = l;
            }
        dT += lam * incT;
        for (int k = 0; k < ns; ++k)
            dY[k] += lam * incY[k];
    }
    *src_T = dT;
    for (int k = 0; k < ns; ++k)
        src_Y[k] = dY[k];
}

/* ------------------------------------------------------------------ */
/* Geometry queries                                                    */
/* ------------------------------------------------------------------ */

/* mixture density in lattice units (ideal gas at uniform P_0) */
static double density(const lbo_params *p, double T, const double *Y)
{
    double s = 0.0;
    for (int k = 0; k < p->n_species; ++k)
        s += Y[k] / p->W[k];
    return (p->T_ref / T) * ((1.0 / s) / p->W_ref);
}

/* What sits at integer coordinates (x, y, z): periodic faces wrap;      */
/* outside any other face the point is that face (walls before inflow,  */
/* inflow before outflow, lower axis and lower face first).             */
static cellref classify(const lbo_state *s, int x, int y, int z)
{
    const lbo_params *p = &s->p;
    int n[3] = {p->nx, p->ny, p->nz};
    int q[3] = {x, y, z};
    int best_face = -1, best_rank = 99;
    for (int d = 0; d < 3; ++d) {
        if (q[d] < 0 || q[d] >= n[d]) {
            int f = 2 * d + (q[d] >= n[d] ? 1 : 0);
            if (p->face[f] == LBO_PERIODIC) {
                q[d] = ((q[d] % n[d]) + n[d]) % n[d];
            } else {
                int rank = (p->face[f] == LBO_WALL || p->face[f] == LBO_WALL_ADIABATIC) ? 0
                         : p->face[f] == LBO_INFLOW ? 1 : 2;
                if (rank < best_rank) {
                    best_rank = rank;
                    best_face = f;
                }
            }
        }
    }
    cellref r;
    r.idx = -1;
    r.Tw = 0.0;
    r.face = -1;
    if (best_face >= 0) {
        r.face = best_face;
        switch (p->face[best_face]) {
        case LBO_WALL: r.kind = K_ISO; r.Tw = p->face_T[best_face]; break;
        case LBO_WALL_ADIABATIC: r.kind = K_ADIA; break;
        case LBO_INFLOW: r.kind = K_INFLOW; break;
        default: r.kind = K_OUTFLOW; break;
        }
        return r;
    }
    r.idx = ((long)q[2] * p->ny + q[1]) * p->nx + q[0];
    uint8_t m = s->mask[r.idx];
    if (m == LBO_FLUID)
        r.kind = K_FLUID;
    else if (m == LBO_SOLID_ISOTHERMAL) {
        r.kind = K_ISO;
        r.Tw = s->wall_T[r.idx];
    } else
        r.kind = K_ADIA;
    return r;
}

/* ------------------------------------------------------------------ */
/* Ghost/image nodes, Sec. III.B.                                       */
/* Reading: the wall lies half-way between the last fluid cell and the  */
/* first non-fluid cell along the axis (as for half-way bounce-back),   */
/* the image point is the axis mirror of the ghost across that plane,   */
/* and an image that is itself non-fluid is clamped to the last fluid   */
/* cell.  Dirichlet values: phi(G) = 2 phi_B - phi(I) (Eq. 34); walls   */
/* are impermeable (Y ghost = Y(I)); adiabatic walls and the outlet use */
/* phi(G) = phi(I).  The density ghost is reconstructed directly from   */
/* its wall value rho_B = rho(T_w, Y(I)) (last paragraph of III.B).     */
/* ------------------------------------------------------------------ */
typedef struct {
    double T, rho;
    double Y[LBO_MAXSP];
} scal;

static void load_scal(const lbo_state *s, long idx, scal *o)
{
    o->T = s->T[idx];
    o->rho = s->rho[idx];
    for (int k = 0; k < s->p.n_species; ++k)
        o->Y[k] = s->Y[k * s->N + idx];
}

static void ghost_value(const lbo_state *s, const cellref *wall, const scal *img, scal *o)
{
    const lbo_params *p = &s->p;
    int ns = p->n_species;
    switch (wall->kind) {
    case K_ISO:
        o->T = 2.0 * wall->Tw - img->T;
        for (int k = 0; k < ns; ++k)
            o->Y[k] = img->Y[k];
        o->rho = 2.0 * density(p, wall->Tw, img->Y) - img->rho;
        break;
    case K_INFLOW:
        o->T = 2.0 * p->T_in - img->T;
        for (int k = 0; k < ns; ++k)
            o->Y[k] = 2.0 * p->Y_in[k] - img->Y[k];
        o->rho = 2.0 * density(p, p->T_in, p->Y_in) - img->rho;
        break;
    default: /* adiabatic walls, outlet */
        *o = *img;
        break;
    }
}

/* Shepard's inverse-distance reconstruction (Sec. III.B): the value at  */
/* the point x is the average of every fluid node r_j with |x - r_j| <= */
/* 4 cells, weighted by |x - r_j|^-2 (p = 2), the weights normalised to */
/* sum to one; a node at distance zero takes the whole weight.  Nodes   */
/* are found through classify (periodic faces wrap; reading: candidate  */
/* points are the integer points of the cube around x, in a D2Q9 box    */
/* those of the plane z = 0).  Returns the number of nodes used.        */
static int shepard(const lbo_state *s, const double *x, scal *o)
{
    int ns = s->p.n_species;
    int lo[3], hi[3];
    for (int d = 0; d < 3; ++d) {
        if (d < s->D) {
            lo[d] = (int)ceil(x[d] - 4.0);
            hi[d] = (int)floor(x[d] + 4.0);
        } else {
            lo[d] = hi[d] = 0;
        }
    }
    double wsum = 0.0, T = 0.0, rho = 0.0, Y[LBO_MAXSP];
    for (int k = 0; k < ns; ++k)
        Y[k] = 0.0;
    int n = 0;
    for (int z = lo[2]; z <= hi[2]; ++z)
        for (int y = lo[1]; y <= hi[1]; ++y)
            for (int xx = lo[0]; xx <= hi[0]; ++xx) {
                double dx = xx - x[0], dy = y - x[1], dz = s->D == 3 ? z - x[2] : 0.0;
                double d2 = dx * dx + dy * dy + dz * dz;
                if (d2 > 16.0)
                    continue;
                cellref c = classify(s, xx, y, z);
                if (c.kind != K_FLUID)
                    continue;
                if (d2 == 0.0) {            /* x is this node */
                    load_scal(s, c.idx, o);
                    return 1;
                }
                double w = 1.0 / d2;
                wsum += w;
                T += w * s->T[c.idx];
                rho += w * s->rho[c.idx];
                for (int k = 0; k < ns; ++k)
                    Y[k] += w * s->Y[k * s->N + c.idx];
                ++n;
            }
    if (n == 0)
        return 0;
    o->T = T / wsum;
    o->rho = rho / wsum;
    for (int k = 0; k < ns; ++k)
        o->Y[k] = Y[k] / wsum;
    return n;
}

/* The image of the ghost node at slot (axis d, offset index j) of cell */
/* idx when one is listed: the Shepard value at that image point.       */
static int listed_image(const lbo_state *s, long idx, int d, int j, scal *o)
{
    if (s->n_img == 0)
        return 0;
    long key = idx * 12 + d * 4 + j, lo = 0, hi = s->n_img - 1;
    while (lo <= hi) {
        long mid = (lo + hi) / 2;
        if (s->img_key[mid] == key)
            return shepard(s, &s->img_x[3 * mid], o) > 0;
        if (s->img_key[mid] < key)
            lo = mid + 1;
        else
            hi = mid - 1;
    }
    return 0;
}

/* Values at p + m e_d, m = -2..2, with ghosts; *near is set when a      */
/* non-fluid point lies within two cells on either side.                 */
static void axis_stencil(const lbo_state *s, const int *pc, long pidx, int d,
                         scal st[5], int *near)
{
    load_scal(s, pidx, &st[2]);
    for (int sg = -1; sg <= 1; sg += 2) {
        int q1[3] = {pc[0], pc[1], pc[2]}, q2[3] = {pc[0], pc[1], pc[2]}, qm[3] = {pc[0], pc[1], pc[2]};
        q1[d] += sg;
        q2[d] += 2 * sg;
        qm[d] -= sg;
        cellref c1 = classify(s, q1[0], q1[1], q1[2]);
        cellref c2 = classify(s, q2[0], q2[1], q2[2]);
        scal *s1 = &st[2 + sg], *s2 = &st[2 + 2 * sg];
        /* offset index j of m = -2, -1, 1, 2 for the listed image points */
        int j1 = sg < 0 ? 1 : 2, j2 = sg < 0 ? 0 : 3;
        scal img;
        if (c1.kind != K_FLUID) {
            *near = 1;
            if (!listed_image(s, pidx, d, j1, &img))
                img = st[2];                             /* image of p+s is p */
            ghost_value(s, &c1, &img, s1);
            if (!listed_image(s, pidx, d, j2, &img)) {
                cellref cm = classify(s, qm[0], qm[1], qm[2]);
                if (cm.kind == K_FLUID)
                    load_scal(s, cm.idx, &img);          /* image of p+2s is p-s */
                else
                    img = st[2];                         /* clamped to p */
            }
            ghost_value(s, &c1, &img, s2);
        } else {
            load_scal(s, c1.idx, s1);
            if (c2.kind != K_FLUID) {
                *near = 1;
                if (!listed_image(s, pidx, d, j2, &img))
                    img = *s1;                           /* image of p+2s is p+s */
                ghost_value(s, &c2, &img, s2);
            } else {
                load_scal(s, c2.idx, s2);
            }
        }
    }
}

/* ------------------------------------------------------------------ */
/* Mixture-averaged transport (Sec. II.A).                             */
/* Species: -(1/rho) div(rho Y_k V_k) with Eq. (2),                    */
/*   Y_k V_k = -D_k G_k + Y_k V_c,  G_k = (W_k/W) grad X_k             */
/*           = grad Y_k + Y_k grad ln W,  V_c = sum_k D_k G_k,         */
/* D_k = alpha / Le_k.  Energy, Eq. (7) over rho c_p with the          */
/* conductivity lambda = rho c_p alpha (constant Prandtl number at the */
/* local c_p = sum_k Y_k c_pk):                                        */
/*   alpha [lap T + (grad rho / rho + grad c_p / c_p) . grad T]        */
/*   - (1/c_p) (sum_k c_pk Y_k V_k) . grad T.                          */
/* Reading (discretisation): the divergences are expanded by the       */
/* product rule, every derivative is the fourth-order central D1 / D2  */
/* along its axis of the ghost-extended stencil values (of Y_k, T, rho,*/
/* M = 1/W = sum_k Y_k / W_k and c_p), and the products are formed at  */
/* the cell: with l1 = -D1(M)/M = d ln W and l2 = -D2(M)/M + l1^2 =    */
/* d2 ln W per axis,                                                   */
/*   div G_k = sum_axes [D2 Y_k + D1 Y_k l1 + Y_k l2],                 */
/*   rhs_k = D_k (div G_k + grad rho . G_k / rho) - V_c . grad Y_k     */
/*           - Y_k (div V_c + V_c . grad rho / rho).                   */
/* With all Le_k = 1 and equal c_pk this is, to rounding, the Fickian  */
/* alpha (lap Y_k + grad rho . grad Y_k / rho) of the unity-Lewis path. */
/* ------------------------------------------------------------------ */
static void mixture_transport(const lbo_params *p, int D, double rho, double T, const double *Y, double alpha,
                              const double *grad_rho, const double *dT1, const double *dT2,
                              double y1[3][LBO_MAXSP], double y2[3][LBO_MAXSP], const double *dM1,
                              const double *dM2, const double *dcp, double *diffT, double *diffY)
{
    (void)T;
    int ns = p->n_species;
    double M = 0.0, cpm = 0.0, Dk[LBO_MAXSP];
    for (int k = 0; k < ns; ++k) {
        M += Y[k] / p->W[k];
        cpm += Y[k] * p->cp[k];
        Dk[k] = alpha / p->lewis[k];
    }
    double G[3][LBO_MAXSP], Vc[3] = {0.0, 0.0, 0.0}, divG[LBO_MAXSP], divVc = 0.0;
    for (int k = 0; k < ns; ++k)
        divG[k] = 0.0;
    for (int d = 0; d < D; ++d) {
        double l1 = -dM1[d] / M;
        double l2 = -dM2[d] / M + l1 * l1;
        for (int k = 0; k < ns; ++k) {
            G[d][k] = y1[d][k] + Y[k] * l1;
            divG[k] += y2[d][k] + y1[d][k] * l1 + Y[k] * l2;
            Vc[d] += Dk[k] * G[d][k];
        }
    }
    for (int k = 0; k < ns; ++k)
        divVc += Dk[k] * divG[k];
    for (int k = 0; k < ns; ++k) {
        double gG = 0.0, vY = 0.0, vR = 0.0;
        for (int d = 0; d < D; ++d) {
            gG += grad_rho[d] * G[d][k];
            vY += Vc[d] * y1[d][k];
            vR += Vc[d] * grad_rho[d];
        }
        diffY[k] = Dk[k] * (divG[k] + gG / rho) - vY - Y[k] * (divVc + vR / rho);
    }
    double cond = 0.0, enth = 0.0;
    for (int d = 0; d < D; ++d) {
        cond += dT2[d] + (grad_rho[d] / rho + dcp[d] / cpm) * dT1[d];
        double flux = 0.0;                       /* sum_k c_pk Y_k V_k along d */
        for (int k = 0; k < ns; ++k)
            flux += p->cp[k] * (-Dk[k] * G[d][k] + Y[k] * Vc[d]);
        enth += flux * dT1[d];
    }
    *diffT = alpha * cond - enth / cpm;
}

/* ------------------------------------------------------------------ */
/* Per-cell evaluation at the current level                            */
/* ------------------------------------------------------------------ */
typedef struct {
    double rho, u[3], Ph, Lambda;
    double gstar[MAXQ];
    double Tn, Yn[LBO_MAXSP];
    double sum_g, sum_xi, mom[3];
    double src_T, src_Y[LBO_MAXSP];
} cell_eval_t;

static void eval_cell(const lbo_state *s, int x, int y, int z, cell_eval_t *o)
{
    const lbo_params *p = &s->p;
    int Q = s->Q, D = s->D, ns = p->n_species;
    long idx = ((long)z * p->ny + y) * p->nx + x;
    int pc[3] = {x, y, z};
    double g[MAXQ];
    for (int i = 0; i < Q; ++i)
        g[i] = s->g[i * s->N + idx];
    double rho = s->rho[idx];
    double T = s->T[idx];
    double Y[LBO_MAXSP];
    for (int k = 0; k < ns; ++k)
        Y[k] = s->Y[k * s->N + idx];

    /* velocity, Eq. (13b); the oracle-only test body force adds F/(2 rho) */
    double u[3] = {0.0, 0.0, 0.0};
    for (int d = 0; d < 3; ++d) {
        double m = 0.0;
        for (int i = 0; i < Q; ++i)
            m += s->c[i][d] * g[i];
        u[d] = m / (rho * CS2) + 0.5 * p->body_force[d] / rho;
    }

    /* finite-difference operators per axis (Sec. II.D) */
    double alpha = CS2 * (p->tau - 0.5) / p->prandtl;
    double diffT = 0.0, diffY[LBO_MAXSP], convT[3], convY[3][LBO_MAXSP], grad_rho[3] = {0.0, 0.0, 0.0};
    /* first and second derivatives per axis for the mixture-averaged form */
    double dT1[3], dT2[3], y1[3][LBO_MAXSP], y2[3][LBO_MAXSP], dM1[3], dM2[3], dcp[3];
    for (int k = 0; k < ns; ++k)
        diffY[k] = 0.0;
    for (int d = 0; d < D; ++d) {
        scal st[5];
        int near = 0;
        axis_stencil(s, pc, idx, d, st, &near);
        double phM[5], phC[5];
        for (int m = 0; m < 5; ++m) {
            phM[m] = 0.0;   /* 1 / W, linear in the Y_k */
            phC[m] = 0.0;   /* c_p / c_p,ref */
            for (int k = 0; k < ns; ++k) {
                phM[m] += st[m].Y[k] / p->W[k];
                phC[m] += st[m].Y[k] * p->cp[k];
            }
        }
        dM1[d] = lbo_d1(phM);
        dM2[d] = lbo_d2(phM);
        dcp[d] = lbo_d1(phC);
        double phT[5], phR[5], phY[5];
        for (int m = 0; m < 5; ++m) {
            phT[m] = st[m].T;
            phR[m] = st[m].rho;
        }
        double d1r = lbo_d1(phR);
        grad_rho[d] = d1r;
        dT1[d] = lbo_d1(phT);
        dT2[d] = lbo_d2(phT);
        diffT += lbo_d2(phT) + d1r * lbo_d1(phT) / rho;
        /* centred second-order convection next to non-fluid points */
        convT[d] = near ? 0.5 * (phT[3] - phT[1]) : lbo_weno3(phT, u[d]);
        for (int k = 0; k < ns; ++k) {
            for (int m = 0; m < 5; ++m)
                phY[m] = st[m].Y[k];
            diffY[k] += lbo_d2(phY) + d1r * lbo_d1(phY) / rho;
            y1[d][k] = lbo_d1(phY);
            y2[d][k] = lbo_d2(phY);
            convY[d][k] = near ? 0.5 * (phY[3] - phY[1]) : lbo_weno3(phY, u[d]);
        }
    }
    diffT *= alpha;
    for (int k = 0; k < ns; ++k)
        diffY[k] *= alpha;
    if (p->transport == LBO_MIXTURE_AVERAGED)
        mixture_transport(p, D, rho, T, Y, alpha, grad_rho, dT1, dT2, y1, y2, dM1, dM2, dcp, &diffT, diffY);

    /* chemistry */
    double srcT, srcY[LBO_MAXSP];
    lbo_chemistry(p, T, Y, &srcT, srcY);

    /* material derivatives (reading: non-convective right-hand side at */
    /* level n) and the expansion source Lambda, Eq. (6)                 */
    double DtT = diffT + srcT, DtY[LBO_MAXSP];
    double invW = 0.0;
    for (int k = 0; k < ns; ++k) {
        DtY[k] = diffY[k] + srcY[k];
        invW += Y[k] / p->W[k];
    }
    double Wmix = 1.0 / invW;
    double Lambda = DtT / T;
    for (int k = 0; k < ns; ++k)
        Lambda += (Wmix / p->W[k]) * DtY[k];

    /* convection with the mass-conserving correction, Eq. (26) */
    double CT = 0.0, CY[LBO_MAXSP];
    for (int k = 0; k < ns; ++k)
        CY[k] = 0.0;
    for (int d = 0; d < D; ++d) {
        CT += u[d] * convT[d];
        double sumc = 0.0;
        for (int k = 0; k < ns; ++k)
            sumc += convY[d][k];
        for (int k = 0; k < ns; ++k)
            CY[k] += u[d] * (convY[d][k] - Y[k] * sumc);
    }

    /* explicit Euler (Sec. II.D) */
    o->Tn = T - CT + DtT;
    for (int k = 0; k < ns; ++k)
        o->Yn[k] = Y[k] - CY[k] + DtY[k];

    /* hydrodynamic pressure, Eq. (13a) */
    double sg = 0.0;
    for (int i = 0; i < Q; ++i)
        sg += g[i];
    double Ph = sg + 0.5 * rho * CS2 * Lambda;

    /* source Xi (Eq. 9) with the discrete density gradient (reading:   */
    /* fourth-order central differences with the density ghosts)        */
    double xi[MAXQ];
    lbo_source_xi(Q, rho, u, grad_rho, Lambda, xi);
    for (int i = 0; i < Q; ++i)
        for (int d = 0; d < 3; ++d)
            xi[i] += s->w[i] * s->c[i][d] * p->body_force[d];

    lbo_collide(p, g, xi, rho, u, o->gstar);

    o->rho = rho;
    for (int d = 0; d < 3; ++d)
        o->u[d] = u[d];
    o->Ph = Ph;
    o->Lambda = Lambda;
    o->sum_g = sg;
    double sx = 0.0;
    for (int i = 0; i < Q; ++i)
        sx += xi[i];
    o->sum_xi = sx;
    for (int d = 0; d < 3; ++d) {
        double m = 0.0;
        for (int i = 0; i < Q; ++i)
            m += s->c[i][d] * g[i];
        o->mom[d] = m / CS2;
    }
    o->src_T = srcT;
    for (int k = 0; k < ns; ++k)
        o->src_Y[k] = srcY[k];
}

static void compute_density(lbo_state *s)
{
    long N = s->N;
    int ns = s->p.n_species;
#pragma omp parallel for schedule(static)
    for (long idx = 0; idx < N; ++idx) {
        if (s->mask[idx] != LBO_FLUID) {
            s->rho[idx] = 0.0;
            continue;
        }
        double Y[LBO_MAXSP];
        for (int k = 0; k < ns; ++k)
            Y[k] = s->Y[k * N + idx];
        s->rho[idx] = density(&s->p, s->T[idx], Y);
    }
}

/* ------------------------------------------------------------------ */
/* Streaming with boundary conditions (Sec. III.A):                     */
/*  - source fluid: g_i(r) = g*_i(r - c_i)  (LB equation, Eq. 8);        */
/*  - source solid or wall face: half-way bounce-back, Eq. (28);         */
/*  - source beyond the inlet: Eq. (31) in g units, i.e. g*_opp(r) +     */
/*    2 w_i rho_in c_i.u_in (g carries the factor cs^2 of Eq. 12);       */
/*  - source beyond the outlet: Eq. (32) read as                          */
/*    g_i(r) <- g_i(r-n)(cs - u.n) + g_i(r)(1 - cs + u.n) with the        */
/*    post-streaming values and velocity of the current level; if r-n    */
/*    is not fluid the link bounces back.                                 */
/* ------------------------------------------------------------------ */
static void stream(lbo_state *s)
{
    const lbo_params *p = &s->p;
    int Q = s->Q;
    long N = s->N;
    double cs = sqrt(CS2);
    double rho_in = density(p, p->T_in, p->Y_in);
#pragma omp parallel for schedule(static) collapse(2)
    for (int z = 0; z < p->nz; ++z)
        for (int y = 0; y < p->ny; ++y)
            for (int x = 0; x < p->nx; ++x) {
                long idx = ((long)z * p->ny + y) * p->nx + x;
                if (s->mask[idx] != LBO_FLUID || !covered(s, idx))
                    continue;
                for (int i = 0; i < Q; ++i) {
                    int opp = Q - 1 - i;
                    cellref src = classify(s, x - s->c[i][0], y - s->c[i][1], z - s->c[i][2]);
                    double v;
                    if (src.kind == K_FLUID) {
                        v = s->gstar[i * N + src.idx];
                    } else if (src.kind == K_INFLOW) {
                        /* an x face may carry a profile: the velocity of the
                           receiving cell's (y, z) on that face */
                        double cu = 0.0;
                        for (int d = 0; d < 3; ++d) {
                            double ud = p->u_in[d];
                            if (s->u_face && (src.face == 0 || src.face == 1))
                                ud = s->u_face[((long)(3 * src.face + d) * p->nz + z) * p->ny + y];
                            cu += s->c[i][d] * ud;
                        }
                        v = s->gstar[opp * N + idx] + 2.0 * s->w[i] * rho_in * cu;
                    } else if (src.kind == K_OUTFLOW) {
                        int d = src.face / 2;
                        int nsign = (src.face % 2) ? 1 : -1;  /* outward normal */
                        int qn[3] = {x, y, z};
                        qn[d] -= nsign;
                        cellref in = classify(s, qn[0], qn[1], qn[2]);
                        if (in.kind == K_FLUID) {
                            double un = nsign * s->ux[d * N + idx];
                            v = s->g[i * N + in.idx] * (cs - un) + s->g[i * N + idx] * (1.0 - cs + un);
                        } else {
                            v = s->gstar[opp * N + idx];
                        }
                    } else {
                        /* bounce-back; with a wall distance q of the link
                           from this cell toward the wall (direction opp),
                           the post-collision form of the linearly
                           interpolated bounce-back (the curved-wall
                           treatment of Sec. III.A) */
                        v = s->gstar[opp * N + idx];
                        double q = s->q_link ? s->q_link[(long)opp * N + idx] : NAN;
                        if (!isnan(q)) {
                            if (q < 0.5) {
                                cellref far = classify(s, x + s->c[i][0], y + s->c[i][1], z + s->c[i][2]);
                                if (far.kind == K_FLUID)
                                    v = 2.0 * q * s->gstar[opp * N + idx] +
                                        (1.0 - 2.0 * q) * s->gstar[opp * N + far.idx];
                            } else {
                                v = s->gstar[opp * N + idx] / (2.0 * q) +
                                    (2.0 * q - 1.0) / (2.0 * q) * s->gstar[i * N + idx];
                            }
                        }
                    }
                    s->gn[i * N + idx] = v;
                }
            }
}

int lbo_step(lbo_state *s, long nsteps)
{
    const lbo_params *p = &s->p;
    long N = s->N;
    int Q = s->Q, ns = p->n_species;
    for (long n = 0; n < nsteps; ++n) {
        compute_density(s);
#pragma omp parallel for schedule(dynamic, 16) collapse(2)
        for (int z = 0; z < p->nz; ++z)
            for (int y = 0; y < p->ny; ++y)
                for (int x = 0; x < p->nx; ++x) {
                    long idx = ((long)z * p->ny + y) * p->nx + x;
                    if (s->mask[idx] != LBO_FLUID || !covered(s, idx))
                        continue;
                    cell_eval_t o;
                    eval_cell(s, x, y, z, &o);
                    for (int i = 0; i < Q; ++i)
                        s->gstar[i * N + idx] = o.gstar[i];
                    s->Tn[idx] = o.Tn;
                    for (int k = 0; k < ns; ++k)
                        s->Yn[k * N + idx] = o.Yn[k];
                    for (int d = 0; d < 3; ++d)
                        s->ux[d * N + idx] = o.u[d];
                }
        stream(s);
        double *t;
        t = s->g; s->g = s->gn; s->gn = t;
        /* solid cells keep their (never used) values in both buffers */
#pragma omp parallel for schedule(static)
        for (long idx = 0; idx < N; ++idx) {
            if (s->mask[idx] != LBO_FLUID || !covered(s, idx))
                continue;
            s->T[idx] = s->Tn[idx];
            for (int k = 0; k < ns; ++k)
                s->Y[k * N + idx] = s->Yn[k * N + idx];
        }
        s->level++;
    }
    return 0;
}

long lbo_level(const lbo_state *s) { return s->level; }

/*
 * Restrict the following lbo_step / lbo_fields calls to the cells with
 * active[idx] != 0 (NULL: every cell).  Cells outside the set are neither
 * updated nor reported (lbo_fields gives NaN there), so after a restricted
 * step only the cells whose whole dependency region was covered hold the
 * values of the full step: a cell's new state reads the previous level
 * within three cells (its pull sources, and their finite-difference
 * stencils of half-width two).  The array is not copied; it must outlive
 * its use.  lbo_diagnostics needs the full set.
 */
void lbo_set_active(lbo_state *s, const uint8_t *active) { s->active = active; }

/*
 * Inlet velocity profile of x face `face` (0: -x, 1: +x): u [3][nz][ny] is
 * imposed (Eq. 31) on the populations entering through that face at the
 * fluid cell (face cell, y, z); NULL restores the uniform u_in.  Returns 0,
 * or -1 for a face that is not 0 or 1.
 */
/*
 * Wall distances of links (interpolated bounce-back): link k runs from
 * fluid cell cell[k] along lattice direction dir[k] toward a solid cell or
 * wall and meets the wall at the fraction q[k] in (0, 1] of the link.  The
 * population entering cell[k] in the opposite direction then takes, for
 * q < 1/2, 2 q g*_i(r) + (1 - 2q) g*_i(r - c_i) (half-way bounce-back when
 * r - c_i is not fluid), and for q >= 1/2,
 * g*_i(r) / (2q) + (2q - 1)/(2q) g*_opp(r), with i = dir[k] and g* the
 * post-collision populations; other links bounce back half-way.  n = 0
 * clears.  Returns 0, or -1 for an entry out of range.
 */
int lbo_set_wall_links(lbo_state *s, long n, const long *cell, const int *dir, const double *q)
{
    long N = s->N;
    int Q = s->Q;
    free(s->q_link);
    s->q_link = NULL;
    if (n <= 0)
        return 0;
    s->q_link = (double *)malloc(sizeof(double) * (size_t)Q * (size_t)N);
    for (long k = 0; k < (long)Q * N; ++k)
        s->q_link[k] = NAN;
    for (long k = 0; k < n; ++k) {
        if (cell[k] < 0 || cell[k] >= N || dir[k] < 0 || dir[k] >= Q || !(q[k] > 0.0 && q[k] <= 1.0))
            return -1;
        s->q_link[(long)dir[k] * N + cell[k]] = q[k];
    }
    return 0;
}

/*
 * Image points of ghost nodes on curved walls (Sec. III.B): for the ghost
 * at offset m = (-2, -1, 1, 2)[j] along axis d of fluid cell cell[k]
 * (slot[k] = 4 d + j), the image point I = 2B - G of the ghost G across
 * the wall point B nearest to it, image[3k..3k+2] in lattice coordinates.
 * The ghost then takes its wall value from the Shepard reconstruction at
 * I instead of the axis mirror.  n = 0 clears.  Returns 0, or -1 for an
 * entry out of range or a repeated (cell, slot).
 */
static int cmp_long(const void *a, const void *b)
{
    long x = *(const long *)a, y = *(const long *)b;
    return x < y ? -1 : x > y;
}

int lbo_set_image_points(lbo_state *s, long n, const long *cell, const int *slot, const double *image)
{
    free(s->img_key);
    free(s->img_x);
    s->img_key = NULL;
    s->img_x = NULL;
    s->n_img = 0;
    if (n <= 0)
        return 0;
    /* sort (key, position) pairs, then gather the coordinates */
    long *pairs = (long *)malloc(sizeof(long) * 2 * (size_t)n);
    for (long k = 0; k < n; ++k) {
        if (cell[k] < 0 || cell[k] >= s->N || slot[k] < 0 || slot[k] >= 4 * s->D) {
            free(pairs);
            return -1;
        }
        pairs[2 * k] = cell[k] * 12 + slot[k];
        pairs[2 * k + 1] = k;
    }
    qsort(pairs, (size_t)n, 2 * sizeof(long), cmp_long);
    s->img_key = (long *)malloc(sizeof(long) * (size_t)n);
    s->img_x = (double *)malloc(sizeof(double) * 3 * (size_t)n);
    for (long k = 0; k < n; ++k) {
        if (k > 0 && pairs[2 * k] == pairs[2 * k - 2]) {
            free(pairs);
            lbo_set_image_points(s, 0, NULL, NULL, NULL);
            return -1;
        }
        s->img_key[k] = pairs[2 * k];
        for (int d = 0; d < 3; ++d)
            s->img_x[3 * k + d] = image[3 * pairs[2 * k + 1] + d];
    }
    s->n_img = n;
    free(pairs);
    return 0;
}

/* Shepard reconstruction of T and Y_k at the point x from the current   */
/* level (pins of the reconstruction); returns the number of nodes.     */
int lbo_image_value(lbo_state *s, const double *x, double *T, double *Y)
{
    scal o;
    int n = shepard(s, x, &o);
    if (n > 0) {
        *T = o.T;
        for (int k = 0; k < s->p.n_species; ++k)
            Y[k] = o.Y[k];
    }
    return n;
}

int lbo_set_inflow(lbo_state *s, int face, const double *u)
{
    const lbo_params *p = &s->p;
    long nf = (long)p->ny * p->nz;
    if (face != 0 && face != 1)
        return -1;
    if (!s->u_face) {
        s->u_face = (double *)malloc(sizeof(double) * 6 * nf);
        for (int f = 0; f < 2; ++f)
            for (int d = 0; d < 3; ++d)
                for (long i = 0; i < nf; ++i)
                    s->u_face[(3 * f + d) * nf + i] = p->u_in[d];
    }
    for (int d = 0; d < 3; ++d)
        for (long i = 0; i < nf; ++i)
            s->u_face[(3 * face + d) * nf + i] = u ? u[d * nf + i] : p->u_in[d];
    return 0;
}

void lbo_set_threads(int n)
{
#ifdef _OPENMP
    if (n > 0)
        omp_set_num_threads(n);
#else
    (void)n;
#endif
}

/* Macroscopic fields at the current level: rho, u (3 x N), T, Y, P_h.   */
/* Non-fluid cells report rho = u = P_h = 0 and their stored T, Y.       */
void lbo_fields(lbo_state *s, double *rho, double *u, double *T, double *Y, double *Ph)
{
    const lbo_params *p = &s->p;
    long N = s->N;
    int ns = p->n_species;
    compute_density(s);
#pragma omp parallel for schedule(dynamic, 16) collapse(2)
    for (int z = 0; z < p->nz; ++z)
        for (int y = 0; y < p->ny; ++y)
            for (int x = 0; x < p->nx; ++x) {
                long idx = ((long)z * p->ny + y) * p->nx + x;
                if (T)
                    T[idx] = s->T[idx];
                if (Y)
                    for (int k = 0; k < ns; ++k)
                        Y[k * N + idx] = s->Y[k * N + idx];
                if (s->mask[idx] == LBO_FLUID && !covered(s, idx)) {
                    if (T) T[idx] = NAN;
                    if (Y)
                        for (int k = 0; k < ns; ++k)
                            Y[k * N + idx] = NAN;
                    if (rho) rho[idx] = NAN;
                    if (Ph) Ph[idx] = NAN;
                    if (u)
                        for (int d = 0; d < 3; ++d)
                            u[d * N + idx] = NAN;
                    continue;
                }
                if (s->mask[idx] != LBO_FLUID) {
                    if (rho) rho[idx] = 0.0;
                    if (Ph) Ph[idx] = 0.0;
                    if (u)
                        for (int d = 0; d < 3; ++d)
                            u[d * N + idx] = 0.0;
                    continue;
                }
                cell_eval_t o;
                eval_cell(s, x, y, z, &o);
                if (rho) rho[idx] = o.rho;
                if (Ph) Ph[idx] = o.Ph;
                if (u)
                    for (int d = 0; d < 3; ++d)
                        u[d * N + idx] = o.u[d];
            }
}

/*
 * Diagnostics of the current level (plain sums over fluid cells, FP64):
 *  [0] sum_i g_i             [1] sum_i Xi_i          [2..4] sum c_i g_i / cs^2
 *  [5] max |sum_k Y_k - 1|   [6] cells with a non-finite T, Y_k or g_i
 *  [7] sum theta, theta = (T - T_u)/(T_b - T_u)
 *  [8] index of the largest temperature source (first in cell order)
 *  [9] that source           [10] wall heat flux: per fluid cell and axis
 *      side whose first neighbour is an isothermal solid or wall face,
 *      2 alpha rho_B (T - T_w), rho_B = rho(T_w, Y) (ghost-consistent)
 *  [11] fuel consumption: sum of -src(Y_0)
 *  [12] fuel mass consumption: sum of -rho src(Y_0)
 *  [13] consumption speed: [12] / (rho(T_in, Y_in) Y_in[0] n_fluid / nx),
 *       cells per step (cells with a non-finite state are not counted)
 */
void lbo_diagnostics(lbo_state *s, double *out)
{
    if (s->active) {
        for (int k = 0; k < LBO_NDIAG; ++k)
            out[k] = NAN;
        return;
    }
    const lbo_params *p = &s->p;
    long N = s->N;
    int Q = s->Q, ns = p->n_species, D = s->D;
    double alpha = CS2 * (p->tau - 0.5) / p->prandtl;
    compute_density(s);
    for (int k = 0; k < LBO_NDIAG; ++k)
        out[k] = 0.0;
    out[8] = -1.0;
    out[9] = -INFINITY;
    long nfluid = 0;
    for (int z = 0; z < p->nz; ++z)
        for (int y = 0; y < p->ny; ++y)
            for (int x = 0; x < p->nx; ++x) {
                long idx = ((long)z * p->ny + y) * p->nx + x;
                if (s->mask[idx] != LBO_FLUID)
                    continue;
                int bad = !isfinite(s->T[idx]);
                double sy = 0.0;
                for (int k = 0; k < ns; ++k) {
                    bad |= !isfinite(s->Y[k * N + idx]);
                    sy += s->Y[k * N + idx];
                }
                for (int i = 0; i < Q; ++i)
                    bad |= !isfinite(s->g[i * N + idx]);
                if (bad) {
                    out[6] += 1.0;
                    continue;
                }
                cell_eval_t o;
                eval_cell(s, x, y, z, &o);
                out[0] += o.sum_g;
                out[1] += o.sum_xi;
                for (int d = 0; d < 3; ++d)
                    out[2 + d] += o.mom[d];
                if (fabs(sy - 1.0) > out[5])
                    out[5] = fabs(sy - 1.0);
                out[7] += (s->T[idx] - p->T_u) / (p->T_b - p->T_u);
                if (o.src_T > out[9]) {
                    out[9] = o.src_T;
                    out[8] = (double)idx;
                }
                out[11] += -o.src_Y[0];
                out[12] += -o.src_Y[0] * o.rho;
                nfluid += 1;
                double Yc[LBO_MAXSP];
                for (int k = 0; k < ns; ++k)
                    Yc[k] = s->Y[k * N + idx];
                int pc[3] = {x, y, z};
                for (int d = 0; d < D; ++d)
                    for (int sg = -1; sg <= 1; sg += 2) {
                        int q[3] = {pc[0], pc[1], pc[2]};
                        q[d] += sg;
                        cellref nb = classify(s, q[0], q[1], q[2]);
                        if (nb.kind == K_ISO)
                            out[10] += 2.0 * alpha * density(p, nb.Tw, Yc) * (s->T[idx] - nb.Tw);
                    }
            }
    /* consumption speed: the fuel mass consumed per step over the fuel mass
       flux of fresh inflow gas through the mean fluid cross-section */
    double fresh = density(p, p->T_in, p->Y_in) * p->Y_in[0] * ((double)nfluid / p->nx);
    out[13] = fresh > 0.0 ? out[12] / fresh : 0.0;
}

void lbo_get_pops(const lbo_state *s, double *g)
{
    memcpy(g, s->g, sizeof(double) * (size_t)s->Q * (size_t)s->N);
}

/* ------------------------------------------------------------------ */
/* Construction: validation and g^0 = g^eq(P_h0, rho0, u0), Eq. (12).  */
/* ------------------------------------------------------------------ */
static void *xcalloc(size_t n, size_t sz)
{
    void *q = calloc(n ? n : 1, sz);
    return q;
}

lbo_state *lbo_create(const lbo_params *p, const uint8_t *mask,
                      const double *wall_T, const double *T0,
                      const double *Y0, const double *u0, const double *Ph0,
                      char *err, int errlen)
{
#define FAIL(msg) do { if (err) snprintf(err, errlen, "%s", msg); return NULL; } while (0)
    if (p->Q != 9 && p->Q != 27) FAIL("Q must be 9 or 27");
    if (p->nx < 1 || p->ny < 1 || p->nz < 1) FAIL("bad grid size");
    if (p->Q == 9 && p->nz != 1) FAIL("D2Q9 needs nz == 1");
    if (p->tau <= 0.5) FAIL("tau must exceed 1/2");
    if (p->n_species < 1 || p->n_species > LBO_MAXSP) FAIL("bad species count");
    if (p->n_reactions < 0 || p->n_reactions > LBO_MAXRX) FAIL("bad reaction count");
    if (p->prandtl <= 0.0) FAIL("prandtl must be positive");
    for (int j = 0; j < p->n_reactions; ++j) {
        double sn = 0.0;
        for (int k = 0; k < p->n_species; ++k)
            sn += p->rx[j].nu[k];
        if (fabs(sn) > 1e-12) FAIL("reaction does not conserve mass");
    }
    int D = p->Q == 9 ? 2 : 3;
    double alpha = CS2 * (p->tau - 0.5) / p->prandtl;
    if (alpha > (D == 2 ? 3.0 / 16.0 : 1.0 / 8.0)) FAIL("diffusivity above the explicit stability bound");
    if (p->transport != LBO_UNITY_LEWIS && p->transport != LBO_MIXTURE_AVERAGED) FAIL("bad transport model");
    if (p->transport == LBO_MIXTURE_AVERAGED)
        for (int k = 0; k < p->n_species; ++k) {
            if (!(p->lewis[k] > 0.0) || !(p->cp[k] > 0.0)) FAIL("Lewis numbers and heat capacities must be positive");
            if (alpha / p->lewis[k] > (D == 2 ? 3.0 / 16.0 : 1.0 / 8.0))
                FAIL("species diffusivity above the explicit stability bound");
        }
    long N = (long)p->nx * p->ny * p->nz;
    long nfluid = 0;
    for (long idx = 0; idx < N; ++idx) {
        if (mask[idx] == LBO_FLUID) {
            ++nfluid;
            double sy = 0.0;
            for (int k = 0; k < p->n_species; ++k)
                sy += Y0[k * N + idx];
            if (fabs(sy - 1.0) > 1e-12) FAIL("initial mass fractions do not sum to 1");
            if (!(T0[idx] > 0.0)) FAIL("initial temperature must be positive");
        } else if (mask[idx] > LBO_SOLID_ADIABATIC) {
            FAIL("bad mask value");
        }
    }
    if (nfluid == 0) FAIL("no fluid cell");

    lbo_state *s = (lbo_state *)xcalloc(1, sizeof(lbo_state));
    s->p = *p;
    s->D = D;
    s->Q = p->Q;
    s->N = N;
    int cc[MAXQ * 3];
    lbo_lattice(p->Q, cc, s->w);
    for (int i = 0; i < p->Q; ++i)
        for (int d = 0; d < 3; ++d)
            s->c[i][d] = cc[3 * i + d];
    int ns = p->n_species;
    s->mask = (uint8_t *)xcalloc(N, 1);
    s->wall_T = (double *)xcalloc(N, sizeof(double));
    s->g = (double *)xcalloc((size_t)p->Q * N, sizeof(double));
    s->gn = (double *)xcalloc((size_t)p->Q * N, sizeof(double));
    s->gstar = (double *)xcalloc((size_t)p->Q * N, sizeof(double));
    s->T = (double *)xcalloc(N, sizeof(double));
    s->Tn = (double *)xcalloc(N, sizeof(double));
    s->Y = (double *)xcalloc((size_t)ns * N, sizeof(double));
    s->Yn = (double *)xcalloc((size_t)ns * N, sizeof(double));
    s->rho = (double *)xcalloc(N, sizeof(double));
    s->ux = (double *)xcalloc(3 * (size_t)N, sizeof(double));
    memcpy(s->mask, mask, N);
    if (wall_T)
        memcpy(s->wall_T, wall_T, sizeof(double) * N);
    memcpy(s->T, T0, sizeof(double) * N);
    memcpy(s->Y, Y0, sizeof(double) * ns * N);
    compute_density(s);
    for (long idx = 0; idx < N; ++idx) {
        if (mask[idx] != LBO_FLUID)
            continue;
        double u[3] = {0.0, 0.0, 0.0};
        if (u0)
            for (int d = 0; d < D; ++d)
                u[d] = u0[d * N + idx];
        double ph = Ph0 ? Ph0[idx] : 0.0;
        double geq[MAXQ];
        lbo_geq(p->Q, ph, s->rho[idx], u, geq);
        for (int i = 0; i < p->Q; ++i)
            s->g[i * N + idx] = geq[i];
    }
    s->level = 0;
    return s;
#undef FAIL
}

void lbo_destroy(lbo_state *s)
{
    if (!s)
        return;
    free(s->mask); free(s->wall_T); free(s->g); free(s->gn); free(s->gstar);
    free(s->T); free(s->Tn); free(s->Y); free(s->Yn); free(s->rho); free(s->ux);
    free(s->u_face);
    free(s->q_link);
    free(s->img_key);
    free(s->img_x);
    free(s);
}
