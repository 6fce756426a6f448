/*
 * lbfd.h -- C ABI of the MI355X (gfx950) coupled lattice-Boltzmann /
 * finite-difference time step for low-Mach reacting flow, after
 * Hosseini & Thevenin, "Towards pore-scale simulation of combustion in
 * porous media using a low-Mach hybrid lattice Boltzmann/finite difference
 * solver", arXiv:2304.05657.
 *
 * One step advances, on one GPU, the pressure-based lattice-Boltzmann
 * populations g_i (Sec. II.B: LB equation with the source Xi_i, central-
 * moment multiple-relaxation-time collision of Sec. II.C, D2Q9 or D3Q27)
 * and the temperature T and species mass fractions Y_k by explicit Euler
 * finite differences (Sec. II.D: WENO3 convection with the mass-conserving
 * correction, fourth-order central diffusion, Arrhenius sources), with the
 * boundary treatment of Sec. III: half-way bounce-back at walls and
 * obstacles, velocity inlet, non-reflecting outlet, ghost-node isothermal
 * (Dirichlet) or adiabatic (Neumann) walls.
 *
 * Conventions
 *  - Lattice units: dr = dt = 1, cs^2 = 1/3.
 *  - A box of nx * ny * nz cells (nz = 1 for D2Q9); cell (x, y, z) has the
 *    linear index (z*ny + y)*nx + x.  Multi-component host arrays are
 *    component-major: u[d*N + cell], Y[k*N + cell].
 *  - Faces are ordered -x, +x, -y, +y, -z, +z.
 *  - Density in lattice units: rho = (T_ref / T) * (W / W_ref) with the
 *    mixture molar mass W = 1 / sum_k (Y_k / W_k) (ideal gas at uniform
 *    thermodynamic pressure, Sec. II.A).
 *  - alpha = D_k = cs^2 (tau - 1/2) / prandtl (unity Lewis numbers).
 *
 * Ownership: every input pointer is caller-owned and only read during the
 * call (copied to the device).  A context owns all of its device memory
 * until lbfd_destroy.  Output pointers are caller-owned host buffers.
 *
 * Errors: every function returns LBFD_OK (0) or a negative code; nothing
 * aborts or throws across the ABI.  lbfd_last_error() returns a message
 * for the last failure on the calling thread.
 */
#ifndef LBFD_H
#define LBFD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    LBFD_OK = 0,
    LBFD_EINVAL = -1,     /* invalid argument or configuration */
    LBFD_ENOMEM = -2,     /* device or host allocation failed */
    LBFD_EDEVICE = -3,    /* a HIP runtime call failed */
    LBFD_ENONFINITE = -4, /* a periodic check found NaN/Inf in the state */
    LBFD_ESTATE = -5      /* state blob does not match the context */
};

enum { LBFD_D2Q9 = 9, LBFD_D3Q27 = 27 };

/* Storage and arithmetic of the step.
 *  FP64: populations, T, Y stored and computed in double.
 *  MIXED_FP32: populations stored in float as deviations scaled by the
 *    lattice weight, g_i / (w_i cs^2); T, Y stored in float; collision and
 *    finite differences in float; Arrhenius source and reductions in double.
 *  MIXED_FP16: as MIXED_FP32 with the populations stored in IEEE half
 *    (round to nearest even). */
enum { LBFD_FP64 = 0, LBFD_MIXED_FP32 = 1, LBFD_MIXED_FP16 = 2 };

/* Collision (Sec. II.C): every order relaxed as central moments, or the
 * orders >= 4 relaxed as cumulants (for the unit-mass, zero-mean shifted
 * distribution, cumulants and central moments coincide at orders 2 and 3).
 * Orders >= 4 relax at omega4 toward the Maxwellian values (central moments
 * c_s^2 per squared axis; cumulants 0). */
enum { LBFD_CENTRAL_MOMENTS = 0, LBFD_CUMULANTS = 1 };

/* Species transport (Sec. II.A).  UNITY_LEWIS: Fick's law with every D_k
 * equal to the thermal diffusivity alpha = cs^2 (tau - 1/2) / Pr and equal
 * species heat capacities (Eq. 2 then reduces to -D grad Y_k and the species
 * enthalpy flux of Eq. 7 vanishes).  MIXTURE_AVERAGED: the diffusion
 * velocities of Eq. 2 with the correction velocity, D_k = alpha / lewis[k],
 * and Eq. 7 with c_p = sum_k Y_k cp[k] (cp[k] = c_pk / c_p,ref), the
 * conductivity lambda = rho c_p alpha and the species enthalpy flux; the
 * reactions' temperature rise q_over_cp (at c_p,ref) is divided by
 * c_p / c_p,ref.  The divergences are expanded by the product rule with the
 * fourth-order central differences of Y_k, T, rho, 1/W and c_p. */
enum { LBFD_UNITY_LEWIS = 0, LBFD_MIXTURE_AVERAGED = 1 };

/* Face kinds.  WALL: isothermal no-slip wall at face_T (bounce-back, and a
 * Dirichlet ghost for T).  WALL_ADIABATIC: no-slip, Neumann ghost for T.
 * INFLOW: velocity inlet at u_in with Dirichlet T_in, Y_in (Eq. 31).
 * OUTFLOW: non-reflecting zero-gradient outlet (Eq. 32); only the x faces
 * may be OUTFLOW. */
enum {
    LBFD_FACE_PERIODIC = 0,
    LBFD_FACE_WALL = 1,
    LBFD_FACE_INFLOW = 2,
    LBFD_FACE_OUTFLOW = 3,
    LBFD_FACE_WALL_ADIABATIC = 4
};

/* Cell mask values: solids are no-slip obstacles (half-way bounce-back);
 * isothermal solids hold their wall_T, adiabatic ones impose zero normal
 * gradient on T. */
enum { LBFD_FLUID = 0, LBFD_SOLID_ISOTHERMAL = 1, LBFD_SOLID_ADIABATIC = 2 };

#define LBFD_MAX_SPECIES 16
#define LBFD_MAX_REACTIONS 32

/* One irreversible reaction (Arrhenius law on mass fractions):
 * per lattice step the progress is r = A dt_phys T^b exp(-Ta/T) prod Y_r
 * over the n_react reactant indices; species k changes by nu_mass[k] r and
 * T by q_over_cp r.  sum_k nu_mass[k] must be 0 (checked to 1e-12). */
typedef struct {
    int n_react;
    int react[4];
    double A;      /* [1/s] */
    double b;      /* temperature exponent */
    double Ta;     /* activation temperature Ea/R [K] */
    double nu_mass[LBFD_MAX_SPECIES];
    double q_over_cp; /* [K per unit progress] */
} lbfd_reaction;

typedef struct {
    int lattice;             /* LBFD_D2Q9 (nz must be 1) or LBFD_D3Q27 */
    int nx, ny, nz;
    int precision;           /* LBFD_FP64 / LBFD_MIXED_FP32 / LBFD_MIXED_FP16 */
    int face[6];
    double face_T[6];        /* temperature of WALL faces [K] */
    double tau;              /* relaxation time (> 1/2); nu = cs^2 (tau - 1/2) */
    double prandtl;          /* alpha = nu / prandtl */
    double dt_phys;          /* physical time step of the Arrhenius law [s] */
    double T_ref, W_ref;     /* density scale */
    int n_species;           /* 1..LBFD_MAX_SPECIES (builds: 2, 4 and 9) */
    double W[LBFD_MAX_SPECIES];
    int n_reactions;         /* 0..LBFD_MAX_REACTIONS */
    const lbfd_reaction *rxn;
    double u_in[3], T_in, Y_in[LBFD_MAX_SPECIES]; /* INFLOW state */
    double omega3, omega4;   /* rates of 3rd- and >=4th-order central moments */
    int chem_substeps_max;   /* <= 1: one Euler source step; else sub-cycled */
    int check_every;         /* steps between NaN/Inf checks; 0 = never */
    double T_u, T_b;         /* progress variable theta = (T-T_u)/(T_b-T_u) */
    int collision;           /* LBFD_CENTRAL_MOMENTS or LBFD_CUMULANTS */
    int transport;           /* LBFD_UNITY_LEWIS or LBFD_MIXTURE_AVERAGED */
    double lewis[LBFD_MAX_SPECIES]; /* Le_k (MIXTURE_AVERAGED), > 0 */
    double cp[LBFD_MAX_SPECIES];    /* c_pk / c_p,ref (MIXTURE_AVERAGED), > 0 */
} lbfd_params;

/* Diagnostics of the state at one level (plain sums over fluid cells in
 * double precision):
 *  sum_g     sum_i g_i                  sum_xi   sum_i Xi_i
 *  mom       sum_i c_i g_i / cs^2       max_abs_sumY_minus_1
 *  nonfinite fluid cells with a NaN/Inf T, Y_k or g_i (skipped in the rest)
 *  sum_theta sum of the progress variable
 *  hrr_idx, hrr_max  cell (first in index order) and value of the largest
 *            per-step temperature source
 *  wall_q    per fluid cell and axis side whose first neighbour is an
 *            isothermal solid or wall face: 2 alpha rho(T_w, Y) (T - T_w)
 *  fuel_rate sum of the per-step consumption of species 0
 *  step      level the diagnostics refer to
 *  fuel_mass_rate     sum of rho times the per-step consumption of species 0
 *  consumption_speed  fuel_mass_rate / (rho_in Y_in[0] A), A = n_fluid / nx
 *            (mean fluid cross-section): the speed, in cells per step, of a
 *            flat flame consuming fuel at that rate; the ratio of two runs'
 *            values is the normalised consumption speed of Sec. IV.C */
typedef struct {
    double sum_g, sum_xi, mom[3], max_abs_sumY_minus_1;
    int64_t nonfinite;
    double sum_theta;
    int64_t hrr_idx;
    double hrr_max, wall_q, fuel_rate;
    int64_t step;
    double fuel_mass_rate, consumption_speed;
} lbfd_diag;

typedef struct lbfd_ctx lbfd_ctx;

/* Create a context on the current HIP device.  mask [N] (uint8), wall_T
 * [N] (temperature of isothermal solid cells; NULL = 300 K), T0 [N],
 * Y0 [n_species*N] (sum 1 in fluid cells, checked to 1e-12), u0 [dim*N]
 * or NULL (rest), Ph0 [N] or NULL (0).  The initial populations are the
 * pressure-based equilibrium g_i = w_i (P_h - rho cs^2) + cs^2 f_i^eq
 * (Eq. 12).  hip_stream: a hipStream_t on which all work of the context is
 * queued (NULL: the null stream).  On success *out receives the context.
 * Boxes of 2^29 cells or more are rejected (LBFD_EINVAL) before any array
 * is read: every field is addressed with 32-bit byte offsets. */
int lbfd_init(const lbfd_params *p, const uint8_t *mask, const double *wall_T,
              const double *T0, const double *Y0, const double *u0,
              const double *Ph0, void *hip_stream, lbfd_ctx **out);

/* lbfd_init with every array argument a device pointer (same layouts and
 * optional arguments; e.g. the storage of torch tensors).  The arrays are
 * copied to the host for validation and the host-side set-up, then as in
 * lbfd_init; the caller keeps ownership.  Any work queued on hip_stream is
 * waited for first. */
int lbfd_init_dev(const lbfd_params *p, const uint8_t *mask, const double *wall_T,
                  const double *T0, const double *Y0, const double *u0,
                  const double *Ph0, void *hip_stream, lbfd_ctx **out);

/* Queue nsteps coupled steps (asynchronous).  One step n -> n+1, every
 * term at level n: streaming of the lattice-Boltzmann equation with the
 * source Xi_i (Sec. II.B, Eqs. 8-9) and the boundary rules of Sec. III.A
 * (Eqs. 28, 31, 32), the central-moment collision (Sec. II.C, Eqs. 14, 19,
 * 21), the finite-difference advection-diffusion-reaction terms of T and
 * Y_k with ghost nodes (Sec. II.D, Eq. 26; Sec. III.B, Eq. 34), the
 * coupling term Lambda (Eq. 6) and the explicit Euler update of T and Y_k
 * (Sec. II.D).  Every check_every levels the step also reduces the
 * diagnostics; a non-finite value is reported by the next lbfd_sync. */
int lbfd_step(lbfd_ctx *c, int64_t nsteps);

/* Wait for queued work.  Returns LBFD_ENONFINITE if a periodic check saw
 * a non-finite value (lbfd_last_error names the level). */
int lbfd_sync(lbfd_ctx *c);

/* Current level (number of steps taken). */
int64_t lbfd_level(const lbfd_ctx *c);

/* Macroscopic fields at the current level into host buffers (any may be
 * NULL): rho [N], u [dim*N] (Eq. 13b), T [N], Y [n_species*N],
 * Ph [N] (Eq. 13a, including the rho cs^2 Lambda / 2 term).  Always double.
 * Non-fluid cells report rho = u = Ph = 0 and their stored T, Y.
 * Synchronous. */
int lbfd_read_fields(lbfd_ctx *c, double *rho, double *u, double *T,
                     double *Y, double *Ph);

/* lbfd_read_fields into caller-owned device buffers of the same layouts
 * (double; mixed-precision T, Y are widened on the device), queued on the
 * context stream.  Synchronous. */
int lbfd_read_fields_dev(lbfd_ctx *c, double *rho, double *u, double *T,
                         double *Y, double *Ph);

/* Diagnostics of the current level (synchronous): the sums of lbfd_diag.
 * The wall heat flux is the conductive flux through the ghost-node walls of
 * Sec. III.B (Eq. 34) that the heat-loss study of Sec. IV.A measures; the
 * progress-variable sum gives the flame position followed in Secs. IV.A
 * and IV.C (flame position = nx - sum_theta / (n_fluid / nx)); the fuel rate
 * gives the consumption speed of Sec. IV.C. */
int lbfd_diagnostics(lbfd_ctx *c, lbfd_diag *d);

/* Curved walls (interpolated bounce-back, the post-collision form of the
 * linear interpolation cited in Sec. III.A): link k runs from fluid cell
 * cell[k] along lattice direction dir[k] (lattice order: c_z, c_y, c_x
 * lexicographic, x fastest) to a solid cell or wall face, which it meets at
 * the fraction q[k] in (0, 1] of its length.  The population entering
 * cell[k] in the opposite direction then takes, with i = dir[k] and g* the
 * post-collision populations,
 *   q <  1/2:  2 q g*_i(r) + (1 - 2q) g*_i(r - c_i)   (half-way bounce-back
 *              when r - c_i is not a fluid cell),
 *   q >= 1/2:  g*_i(r) / (2q) + (2q - 1)/(2q) g*_opp(r);
 * every other wall link bounces back half-way (q = 1/2).  Replaces the
 * previous set; n = 0 clears it.  q is stored in single precision.
 * LBFD_EINVAL for a link that does not run from a fluid cell to a wall (the
 * previous set is then kept). */
int lbfd_set_wall_links(lbfd_ctx *c, int64_t n, const int64_t *cell, const int32_t *dir, const double *q);

/* Curved walls for the finite differences (image/ghost nodes, Sec. III.B,
 * with Shepard's inverse-distance reconstruction): entry k names the ghost
 * node at offset m = (-2, -1, +1, +2)[j] along axis a of boundary fluid
 * cell cell[k] (slot[k] = 4 a + j, a = 0 x, 1 y, 2 z) -- a point of the
 * cell's finite-difference stencil that lies behind a wall (solid cell) --
 * and image[3k..3k+2] the lattice coordinates (x, y, z; z = 0 for D2Q9;
 * unwrapped across periodic faces) of its image point I = 2B - G, B the
 * wall point nearest to the ghost G.  The ghost's wall value then comes
 * from the value at I reconstructed by inverse-distance weighting over
 * every fluid node r_j with |I - r_j| <= 4 cells, weights |I - r_j|^-2
 * normalised to sum to one (a node at I takes the whole weight), instead
 * of the axis-mirror image; unlisted ghosts keep the axis mirror.  The
 * weights are computed here, once, in double precision and held on the
 * device (4 + 8 bytes per list entry, and (2 + n_species) doubles per
 * distinct node, packed once per step).  Replaces the previous set; n = 0
 * clears.
 * LBFD_EINVAL for a slot that is not a ghost behind a wall, a repeated
 * ghost, or an image point with no fluid node within four cells (the
 * previous set is then kept); LBFD_ENOMEM when the tables do not fit (no
 * image points are then set). */
int lbfd_set_image_points(lbfd_ctx *c, int64_t n, const int64_t *cell, const int32_t *slot, const double *image);

/* Inlet velocity profile of the x face `face` (0: -x, 1: +x), which must
 * be an INFLOW face: u [3][nz][ny] (host, lattice units) is the velocity
 * imposed (Eq. 31) on every population entering the box through that face
 * at the fluid cell (face cell, y, z); NULL restores the uniform u_in of the
 * parameters.  The current state is unchanged: the profile applies to the
 * populations entering from the next step on. */
int lbfd_set_inflow(lbfd_ctx *c, int face, const double *u);

/* Flame holding (Sec. IV.A: the flow rate follows the flame speed so that
 * the front stays in the box): run nsteps steps in cycles of `every`; after
 * each cycle set the inlet velocity of the INFLOW x face (the -x face if
 * both are) to U times the profile's shape (the profile at the call,
 * normalised to a unit mean normal velocity over the face's fluid cells;
 * uniform if that mean is zero), with
 *   U = max(0, consumption_speed - gain (x_f - x_target)),
 * x_f = nx - sum_theta / (n_fluid / nx) (cells from the -x face, as the
 * flame-position objective).  u_mean and x_flame (may be NULL) receive U
 * and x_f of each cycle (nsteps / every entries).  LBFD_ENONFINITE if a
 * cycle ends in a non-finite state. */
int lbfd_hold_flame(lbfd_ctx *c, int64_t nsteps, int every, double x_target, double gain, double *u_mean,
                    double *x_flame);

/* Replace the wall temperature of isothermal solid cells (host [N]): the
 * T_w of the Dirichlet ghost values 2 T_w - T(I) of Sec. III.B (Eq. 34) and
 * of the wall density rho(T_w, Y(I)) of the density ghosts; entries of
 * other cells are ignored.  Takes effect from the next step (the queued
 * work is waited for first). */
int lbfd_set_wall_temperature(lbfd_ctx *c, const double *wall_T);

/* Checkpoint: the whole state (populations, scalars, outlet buffer,
 * level) as an opaque blob of lbfd_state_size bytes.  Restoring it into a
 * context created with the same parameters and geometry resumes the run
 * bit for bit.  LBFD_ESTATE if the blob does not fit the context. */
int lbfd_state_size(const lbfd_ctx *c, size_t *bytes);
int lbfd_save_state(lbfd_ctx *c, void *blob, size_t bytes);
int lbfd_load_state(lbfd_ctx *c, const void *blob, size_t bytes);

/* Measured duration of the step kernels: queue nsteps steps bracketed by
 * HIP events on the context stream, wait, and return the elapsed
 * milliseconds in *ms. */
int lbfd_time_steps(lbfd_ctx *c, int64_t nsteps, double *ms);

/* Replace the Arrhenius parameters of reaction j (A [1/s], b, Ta [K]). */
int lbfd_set_reaction(lbfd_ctx *c, int j, double A, double b, double Ta);

/* Which kernel computes the Arrhenius source of a mechanism of more than
 * four species (Sec. II.A, Eq. 6-7; the launch ahead of the step): 1 when a
 * kernel specialised to this mechanism's structure (its reactant lists and
 * the zero pattern of its mass coefficients, written into HIP source and
 * compiled for the device at lbfd_init) runs, 0 when the generic kernel
 * does (smaller mechanisms, mixture-averaged transport, LBFD_CHEM_JIT=0 in
 * the environment at lbfd_init, or a failed compile).  Both give the same
 * values.  msg (len bytes, may be NULL) receives a NUL-terminated note: the
 * kernel in use and, for the generic one, why.  LBFD_EINVAL for a null
 * context. */
int lbfd_chem_kernel(const lbfd_ctx *c, char *msg, size_t len);

/* Objectives of lbfd_objective / lbfd_adjoint, per level n:
 *   LBFD_OBJ_WALL_HEAT_FLUX  q(n) = wall_q of lbfd_diag (Sec. III.B ghost
 *                            walls: per fluid cell and first-neighbour
 *                            isothermal wall, 2 alpha rho(T_w, Y)(T - T_w));
 *   LBFD_OBJ_FLAME_POSITION  q(n) = x_f = nx - sum_theta / (n_fluid / nx),
 *                            theta = (T - T_u)/(T_b - T_u): the burnt length
 *                            counted back from the +x face, in cells. */
enum { LBFD_OBJ_WALL_HEAT_FLUX = 0, LBFD_OBJ_FLAME_POSITION = 1 };

/* Select the objective of later lbfd_objective / lbfd_adjoint calls: with
 * L the level at which such a call starts, J = sum of q(n) over the levels
 * n = L + t, t_begin <= t < t_end (and t < nsteps).  The default is the wall
 * heat flux over every level (t_begin = 0, t_end = INT64_MAX).  LBFD_EINVAL
 * for an unknown kind, t_begin < 0 or t_end < t_begin. */
int lbfd_set_objective(lbfd_ctx *c, int kind, int64_t t_begin, int64_t t_end);

/* Forward only: run nsteps steps from the current level L and return the
 * objective J selected by lbfd_set_objective over them (the J of
 * lbfd_adjoint). */
int lbfd_objective(lbfd_ctx *c, int64_t nsteps, double *J);

/* lbfd_objective for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the same objective from the same kernels, with the objective's
 * accumulator, the final diagnostics and the per-block partial diagnostics
 * of its steps in a static device array of the library (16 MiB, one per GPU,
 * held until the process ends) instead of library-allocated memory; no
 * hipMalloc, hipFree or allocating library call is made.  The accumulator
 * is cleared by a fill kernel at the start of every call.  Every call on a
 * GPU shares that GPU's array and leaves its contents there: calls that
 * overlap on one GPU (from several threads or streams) race and must be
 * serialised by the caller.  LBFD_EINVAL when the context's step needs more
 * than the array holds (512 + 104 bytes per step block: boxes up to about
 * 161,000 blocks of 256 cells); J is a host pointer; synchronous. */
int lbfd_objective_static(lbfd_ctx *c, int64_t nsteps, double *J);

/* Discrete adjoint of the FP64 step.  Not a method of the paper: the paper
 * has no differentiation; this entry point serves gradient-based uses of
 * the step (sensitivities of wall heat flux and flame position with respect
 * to wall temperatures and Arrhenius parameters).  Starting from the
 * current level L, runs nsteps steps and
 * computes the objective J selected by lbfd_set_objective and its exact
 * derivatives with respect to the
 * wall temperature of every isothermal solid cell (dJ_dwallT [N], host, may
 * be NULL; zero at other cells) and the Arrhenius A and Ta of every reaction
 * (dJ_dA, dJ_dTa [n_reactions], host, may be NULL).  Checkpoints are taken
 * every K steps and each segment is recomputed once during the backward
 * sweep (device memory: about (nsteps/K + K + 8) states).  On return the
 * context is at level L + nsteps, as after lbfd_step(nsteps).  Requires FP64
 * precision, no OUTFLOW face, and a lattice/species combination with an
 * adjoint kernel (D2Q9 or D3Q27 with 4 species); LBFD_EINVAL otherwise.
 * The wall-temperature and Arrhenius derivatives are accumulated with
 * atomic adds, so they may differ in the last bits between runs. */
int lbfd_adjoint(lbfd_ctx *c, int64_t nsteps, int K, double *J, double *dJ_dwallT, double *dJ_dA,
                 double *dJ_dTa);

/* lbfd_adjoint with dJ_dwallT a device pointer ([N] doubles, caller-owned;
 * e.g. a torch tensor's storage); J, dJ_dA, dJ_dTa stay on the host. */
int lbfd_adjoint_dev(lbfd_ctx *c, int64_t nsteps, int K, double *J, double *dJ_dwallT, double *dJ_dA,
                     double *dJ_dTa);

/* The two derivatives of one FP64 step at the current state s^L, for the
 * same contexts as lbfd_adjoint (LBFD_EINVAL otherwise); like lbfd_adjoint
 * they are not methods of the paper.  Neither advances the context.  Host
 * arrays in the state's layout: populations [Q][N] (the post-collision
 * populations the step pulls from), scalars [1 + n_species][N] (T, then
 * Y_k), wall temperatures [N], Arrhenius parameters [n_reactions]; entries
 * of solid cells neither act on nor receive anything.  q is the
 * per-level term of the objective selected by lbfd_set_objective (wall
 * heat flux or flame position at level L).
 *
 * lbfd_step_tangent: the Jacobian-vector product.  Given tangents of the
 * inputs (dpop, dsc; dwallT, dA, dTa may be NULL for zero), returns the
 * tangents of the populations and scalars the step writes (dpop_out,
 * dsc_out; zero at solid cells) and that of q (dq).  Evaluated in dual
 * numbers, cell by cell, from the step's formulas.
 *
 * lbfd_step_adjoint: the vector-Jacobian product, one backward step of
 * lbfd_adjoint.  Given the adjoint of the step's outputs (lam_pop, lam_sc)
 * and a weight wq of q, returns lam_pop_in, lam_sc_in = (dF/ds)^T lam +
 * wq (dq/ds)^T and, if not NULL, the same products for the wall
 * temperatures (dJ_dwallT [N]) and A_j, Ta_j (dJ_dA, dJ_dTa).  For any
 * tangent dx and adjoint lam the two satisfy <J dx, lam> = <dx, J^T lam>
 * up to rounding.  Synchronous. */
int lbfd_step_tangent(lbfd_ctx *c, const double *dpop, const double *dsc, const double *dwallT, const double *dA,
                      const double *dTa, double *dpop_out, double *dsc_out, double *dq);
int lbfd_step_adjoint(lbfd_ctx *c, const double *lam_pop, const double *lam_sc, double wq, double *lam_pop_in,
                      double *lam_sc_in, double *dJ_dwallT, double *dJ_dA, double *dJ_dTa);

/* Per-part timing: queue nsteps steps with their parts launched separately
 * on the context stream, each bracketed by HIP events -- the chemistry
 * launch (mechanisms of more than four species; 0 otherwise), the
 * interior-cell part, and the boundary-cell part (with the image-point and
 * outlet launches) -- wait and return their summed durations in
 * milliseconds (ms_chemistry may be NULL).  The state advances exactly as
 * with lbfd_step. */
int lbfd_time_kernels(lbfd_ctx *c, int64_t nsteps, double *ms_interior, double *ms_boundary,
                      double *ms_chemistry);

/* Cell counts of the context's geometry: fluid cells, and the fluid cells
 * handled by the boundary-cell path (every other fluid cell is interior: all
 * of its pull sources and finite-difference points are fluid cells inside
 * the box). */
int lbfd_cell_counts(const lbfd_ctx *c, int64_t *n_fluid, int64_t *n_boundary);

/* Kernel launches queued by one lbfd_step level without diagnostics: 1 for
 * D2Q9 (one launch covers boundary and interior cells); for D3Q27 the
 * boundary cells, the interior cells and, with an outflow face, the outlet
 * update (Eq. 32) are separate launches; plus three for the chemistry of a
 * mechanism of more than four species (clearing the ordering's counters,
 * ordering the fluid cells by their previous sub-step count, the sources),
 * and two for image points.
 * Negative on a null context. */
int lbfd_step_launches(const lbfd_ctx *c);

void lbfd_destroy(lbfd_ctx *c);

const char *lbfd_strerror(int code);
const char *lbfd_last_error(void);

#ifdef __cplusplus
}
#endif
#endif
