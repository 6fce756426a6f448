/*
 * lbfd_oracle.h -- FP64 CPU oracle of the coupled lattice-Boltzmann /
 * finite-difference time step of Hosseini & Thevenin, "Towards pore-scale
 * simulation of combustion in porous media using a low-Mach hybrid lattice
 * Boltzmann/finite difference solver" (arXiv:2304.05657).
 *
 * TEST INFRASTRUCTURE ONLY.  This library is a plain, slow, obviously
 * correct restatement of the method, used to check the GPU library.  Only
 * the test suite, the smoke check and the CPU-baseline leg of the benchmark
 * load it.  It shares no code, header, table or helper with the GPU path.
 *
 * Everything is double precision.  Lattice units: dr = dt = 1, cs^2 = 1/3.
 * Grid index of cell (x, y, z): (z*ny + y)*nx + x.  Fields are stored
 * structure-of-arrays: g[i*N + cell], Y[k*N + cell].
 */
#ifndef LBFD_ORACLE_H
#define LBFD_ORACLE_H
#include <stdint.h>

#define LBO_MAXSP 16
#define LBO_MAXRX 32

/* face kinds, order of faces: -x, +x, -y, +y, -z, +z */
#define LBO_PERIODIC 0
#define LBO_WALL 1          /* isothermal no-slip wall at face_T */
#define LBO_INFLOW 2        /* velocity inlet (u_in, T_in, Y_in) */
#define LBO_OUTFLOW 3       /* non-reflecting zero-gradient outlet */
#define LBO_WALL_ADIABATIC 4

/* cell mask values */
#define LBO_FLUID 0
#define LBO_SOLID_ISOTHERMAL 1
#define LBO_SOLID_ADIABATIC 2

typedef struct {
    int n_react;            /* reactant count; rate is the product of their Y */
    int react[4];           /* species indices (a repeated index squares Y) */
    double A;               /* pre-exponential factor [1/s] */
    double b;               /* temperature exponent */
    double Ta;              /* activation temperature Ea/R [K] */
    double nu[LBO_MAXSP];   /* mass stoichiometric coefficients, sum 0 */
    double q;               /* heat release over c_p per unit progress [K] */
} lbo_reaction;

typedef struct {
    int Q;                  /* 9 (D2Q9, nz must be 1) or 27 (D3Q27) */
    int nx, ny, nz;
    int face[6];
    double face_T[6];       /* wall temperature of LBO_WALL faces */
    double tau;             /* BGK relaxation time; nu = cs^2 (tau - 1/2) */
    double prandtl;         /* alpha = D_k = nu / Pr */
    double dt_phys;         /* physical time step for the Arrhenius law [s] */
    double T_ref;           /* density scale: rho = (T_ref/T) (W/W_ref) */
    double W_ref;
    int n_species;
    double W[LBO_MAXSP];    /* molar masses */
    int n_reactions;
    lbo_reaction rx[LBO_MAXRX];
    double u_in[3], T_in, Y_in[LBO_MAXSP];
    double omega3, omega4;  /* rates of 3rd and >=4th order central moments */
    int eq_discrete;        /* 1: targets are central moments of f^eq/rho */
    int chem_substeps_max;  /* 1 = plain explicit Euler source */
    double body_force[3];   /* oracle-only test fixture (0 in every workload) */
    double T_u, T_b;        /* progress-variable temperatures (diagnostics) */
    int collision;          /* LBO_CENTRAL_MOMENTS or LBO_CUMULANTS */
    int transport;          /* LBO_UNITY_LEWIS or LBO_MIXTURE_AVERAGED */
    double lewis[LBO_MAXSP];/* Le_k = alpha / D_k (mixture-averaged transport) */
    double cp[LBO_MAXSP];   /* c_pk / c_p,ref (mixture-averaged transport) */
} lbo_params;

/* Species transport (Sec. II.A): Fick's law with D_k = alpha and equal
   c_pk, or the mixture-averaged diffusion velocities of Eq. (2) with the
   correction velocity, D_k = alpha / Le_k, and the species enthalpy flux of
   Eq. (7) with c_p = sum_k Y_k c_pk. */
#define LBO_UNITY_LEWIS 0
#define LBO_MIXTURE_AVERAGED 1

/* Collision operators (Sec. II.C): relaxation of central moments (every
   order), or of cumulants for the orders >= 4 (orders 2, 3: the two coincide
   for the unit-mass, zero-mean distributions relaxed here). */
#define LBO_CENTRAL_MOMENTS 0
#define LBO_CUMULANTS 1

typedef struct lbo_state lbo_state;

/* Diagnostics of the state at the current level, see lbo_diagnostics. */
#define LBO_NDIAG 14

lbo_state *lbo_create(const lbo_params *p, const uint8_t *mask,
                      const double *wall_T, const double *T0,
                      const double *Y0, const double *u0, const double *Ph0,
                      char *err, int errlen);
void lbo_destroy(lbo_state *s);
int lbo_step(lbo_state *s, long nsteps);
long lbo_level(const lbo_state *s);
void lbo_set_active(lbo_state *s, const uint8_t *active);
int lbo_set_inflow(lbo_state *s, int face, const double *u);
int lbo_set_wall_links(lbo_state *s, long n, const long *cell, const int *dir, const double *q);
int lbo_set_image_points(lbo_state *s, long n, const long *cell, const int *slot, const double *image);
int lbo_image_value(lbo_state *s, const double *x, double *T, double *Y);
void lbo_fields(lbo_state *s, double *rho, double *u, double *T, double *Y,
                double *Ph);
void lbo_diagnostics(lbo_state *s, double *out);
void lbo_get_pops(const lbo_state *s, double *g);
void lbo_set_threads(int n);

/* single-operator entry points used by the oracle's own pins */
void lbo_lattice(int Q, int *c, double *w);
void lbo_feq(int Q, double rho, const double *u, double *feq);
void lbo_geq(int Q, double Ph, double rho, const double *u, double *geq);
void lbo_central_moments(int Q, const double *h, const double *u, double *kap);
void lbo_cumulants(int Q, const double *kap, double *cum);
void lbo_cumulants_inverse(int Q, const double *cum, double *kap);
void lbo_collide(const lbo_params *p, const double *g, const double *xi,
                 double rho, const double *u, double *gstar);
void lbo_source_xi(int Q, double rho, const double *u, const double *grad_rho,
                   double Lambda, double *xi);
double lbo_weno3(const double *phi5, double u);
double lbo_d1(const double *phi5);
double lbo_d2(const double *phi5);
void lbo_chemistry(const lbo_params *p, double T, const double *Y,
                   double *src_T, double *src_Y);

#endif
