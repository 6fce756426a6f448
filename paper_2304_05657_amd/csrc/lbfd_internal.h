// Internal interface between the C-ABI layer (lbfd_api.hip) and the gfx950
// kernels (lbfd_step.hip).  Not installed, not part of the ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>

#include "../../include/lbfd.h"

namespace lbfd {

constexpr int kMaxSp = LBFD_MAX_SPECIES;
constexpr int kNDiag = 13;  // per-block partial diagnostics, see DiagSlot
constexpr int kBlock = 256;

// Slots of the per-block and final diagnostics arrays (double).
enum DiagSlot {
    kSumG = 0, kSumXi = 1, kMomX = 2, kMomY = 3, kMomZ = 4, kMaxY = 5,
    kNonfinite = 6, kTheta = 7, kHrrMax = 8, kHrrIdx = 9, kWallQ = 10, kFuel = 11, kFuelMass = 12
};

// Per-cell geometry code: solid, interior fluid (every pull source and
// finite-difference point is an in-box fluid cell), boundary fluid.
enum CellCode { kCodeSolid = 0, kCodeInterior = 1, kCodeBoundary = 2 };

// Special pull sources of boundary cells.
enum { kSrcBounce = -1, kSrcInflow = -2, kSrcOutlet = -3 };

// Kind of what a neighbour coordinate lands on.
enum NbKind { kFluid = 0, kIso = 1, kAdia = 2, kInflow = 3, kOutflow = 4 };

// One reaction as the chemistry reads it: A dt_phys (the rate coefficient's
// prefactor per lattice step), b, Ta, the temperature rise q_over_cp, the
// reactant indices and the mass coefficients.
struct ChemRx {
    double adt, b, ta, q;
    // b, Ta and ln(A dt) scaled by 256 / ln 2 (the sub-steps' exponent is
    // formed in units of ln 2 / 256; ln(A dt) is -inf for A = 0)
    double bs, tas, lnadts;
    int n_react, react[4];  // react[m >= n_react] = n_species (a factor 1)
    double nu[kMaxSp];
};

// Mechanisms of more than four species take their FP64 Arrhenius source in
// a launch of its own ahead of the step (chem_kernel), which leaves it in
// the step's output scalars for the step kernel to read back; smaller ones
// evaluate it inside the step kernel.
constexpr bool chem_pass(int nsp) { return nsp > 4; }

// A chemistry cell that took more than kChemLight sub-steps is "heavy": the
// next launch's ordering puts it at the back of the list.
constexpr int kChemLight = 8;

// Compact per-boundary-cell codes, decoded by the kernels and checked
// against the full descriptors on the host when they are built (the same
// functions on both sides).  Pull: 2 bits per direction I (bits 2 I ..);
// the source of a fluid pull is the neighbour x - c_I, wrapped across
// periodic faces.  Stencil: 5 bits per axis d and offset m = -2, -1, 1, 2
// (slot 4 d + j, bits 5 (4 d + j) ..): the point's kind (kFluid, or the kind
// of the wall behind its ghost; 3 bits) and where its value, or its ghost's
// image, sits (2 bits): the point itself, the cell, the first neighbour on
// the other side, the first neighbour on the same side.
enum { kPullFluid = 0, kPullBounce = 1, kPullInflow = 2, kPullOutlet = 3 };
enum { kImgSelf = 0, kImgCell = 1, kImgMirror = 2, kImgSame = 3 };

// v wrapped once into [0, n) (offsets of at most 2 from an in-box point)
__host__ __device__ inline int wrap_once(int v, int n) { return v < 0 ? v + n : v >= n ? v - n : v; }

__host__ __device__ inline long long cell_at(int x, int y, int z, int dx, int dy, int dz, int nx, int ny, int nz)
{
    return ((long long)wrap_once(z + dz, nz) * ny + wrap_once(y + dy, ny)) * nx + wrap_once(x + dx, nx);
}

__host__ __device__ inline int decode_pull_kind(unsigned long long pc, int I) { return (int)(pc >> (2 * I)) & 3; }

__host__ __device__ inline int decode_kind(unsigned long long sc, int d, int j)
{
    return (int)(sc >> (5 * (4 * d + j))) & 7;
}

__host__ __device__ inline int slot_offset(int j) { return j == 0 ? -2 : j == 1 ? -1 : j == 2 ? 1 : 2; }

// The cell holding the value of stencil slot (d, j), or its ghost's image.
__host__ __device__ inline long long decode_point(unsigned long long sc, int d, int j, long long idx, int x, int y,
                                                  int z, int nx, int ny, int nz)
{
    const int img = (int)(sc >> (5 * (4 * d + j) + 3)) & 3;
    const int m = slot_offset(j), sg = m < 0 ? -1 : 1;
    const int o = img == kImgSelf ? m : img == kImgMirror ? -sg : img == kImgSame ? sg : 0;
    if (o == 0) return idx;
    return cell_at(x, y, z, d == 0 ? o : 0, d == 1 ? o : 0, d == 2 ? o : 0, nx, ny, nz);
}

// Temperature of the isothermal wall behind the ghost of slot (d, j): the
// wall is the first non-fluid point from the cell along the slot's side
// (the first neighbour when that is a ghost, else the point itself), an
// in-box solid cell (wrapped across a periodic face) or a domain face.
// periodic_bits has bit f set for a periodic face f; face_T holds the six
// face temperatures (in device memory on the device: a read of the kernel's
// argument block at a computed index would copy the block to scratch).
__host__ __device__ inline double decode_wall_T(unsigned long long sc, int d, int j, int x, int y, int z, int nx,
                                                int ny, int nz, unsigned periodic_bits, const double *face_T,
                                                const double *wall_T)
{
    const int m = slot_offset(j), sg = m < 0 ? -1 : 1;
    const int j1 = sg < 0 ? 1 : 2;
    const int mw = (j == j1 || decode_kind(sc, d, j1) != kFluid) ? sg : m;
    const int c = d == 0 ? x : d == 1 ? y : z, n = d == 0 ? nx : d == 1 ? ny : nz;
    const int f = 2 * d + (mw > 0 ? 1 : 0);
    if ((c + mw < 0 || c + mw >= n) && !((periodic_bits >> f) & 1u)) return face_T[f];
    return wall_T[cell_at(x, y, z, d == 0 ? mw : 0, d == 1 ? mw : 0, d == 2 ? mw : 0, nx, ny, nz)];
}

// Everything a step kernel reads; passed by value (kernarg segment, read
// through the scalar cache).
struct KParams {
    int nx, ny, nz;
    long long N;
    int face[6];
    double face_T[6];
    const uint8_t *mask;
    const uint8_t *code;        // CellCode per cell
    const int *boundary;        // boundary fluid cells, increasing index
    long long n_boundary;
    const int *fluid;           // every fluid cell, increasing index (chemistry launch)
    int *chem_order;            // [n_fluid] fluid cells in the chemistry launch's order: cells whose last
                                //   source took few sub-steps first, the others from the back
    unsigned char *chem_heavy;  // [N] the cell's last source took more than kChemLight sub-steps
    int *chem_count;            // [2] cells placed at the front / back by this step's ordering
    long long n_fluid;
    // per boundary cell t (structure of arrays, stride n_boundary):
    const int *bsrc;            // [Q][nb] pull source index, or kSrcBounce / kSrcInflow / kSrcOutlet
    const int *bpt;             // [3*4][nb] finite-difference point (or ghost image) index, axis-major, m = -2,-1,1,2
    const uint8_t *bwk;         // [3*4][nb] kind of the wall behind a ghost point, kFluid for a plain point
    const double *btw;          // [3*4][nb] wall temperature of isothermal ghost walls
    const unsigned long long *bcode_pull;  // [nb] compact pull codes (decode_pull_kind below)
    const unsigned long long *bcode_st;    // [nb] compact stencil codes (decode_point below)
    const double *face_Td;      // [6] face_T in device memory (read at a computed face index)
    unsigned periodic_bits;     // bit f: face f periodic
    const float *bq;            // [Q][nb] wall distance of the bounced link of population I, NaN: half-way
                                // (nullptr: every link half-way)
    const int *bimg;            // [3*4][nb] a ghost's image point in img_val, -1: axis mirror
                                // (nullptr: every ghost)
    long long n_img;            // image points:
    int img_lpp;                //   lanes per Shepard row (16, 32 or 64)
    const int2 *img_rng;        //   [n_img] {begin, count} of the Shepard list
    const int *img_idx;         //   entries of the lists: positions in the support
    const double *img_w;        //   and their normalised weights
    long long n_sup;            // support: the distinct fluid nodes of the lists,
    const int *sup_idx;         //   [n_sup] their cells
    double *sup_val;            //   [n_sup][2 + n_species] T, rho, Y_k (this level)
    double *img_val;            //   [2 + n_species][n_img] T, rho, Y_k at the image points (this level)
    // block list of a step launch: boundary_blocks (a multiple of 8) blocks
    // of 256 boundary cells, then interior_blocks tiles of tiles_x x tiles_y
    // x (nz / tile depth); a launch covers blocks [block_begin, + gridDim.x)
    long long boundary_blocks, interior_blocks, block_begin;
    int tiles_x, tiles_y;
    const double *wall_T;
    const void *pop_in;   // post-collision populations of the previous level
    void *pop_out;        // post-collision populations of this level
    const void *sc_in;    // [1 + n_species][N]: T then Y_k
    void *sc_out;
    double *outlet;       // [2 x faces][Q][ny*nz] post-streaming outlet populations
    double *outlet_un;    // [2 x faces][ny*nz] outward normal velocity of the face cells (this level)
    double *fields;       // [5][N]: rho, u_x, u_y, u_z, P_h  (fields mode)
    double *partials;     // [interior_blocks + boundary_blocks][kNDiag]  (diagnostics modes)
    const lbfd_reaction *rx;
    const ChemRx *rxk;  // the same reactions as the chemistry reads them
    int n_rx;
    int chem_anyb;      // some reaction has a temperature exponent b != 0
    int chem_nreact;    // the largest reactant count of a reaction (0..4)
    const void *chem_jit;  // host handle of the mechanism-specialised chemistry kernel, or nullptr
    int chem_substeps_max;
    double omega2, omega3, omega4, alpha;
    double dt_phys;
    double T_ref, W_ref, T_ref_over_W_ref;
    double invW[kMaxSp];
    double u_in[3], T_in, Y_in[kMaxSp], rho_in;
    const double *inflow_u;  // [2 x faces][3][nz][ny] inlet velocity of the cells next to an x face
    double T_u, T_b;
    int collision;  // LBFD_CENTRAL_MOMENTS or LBFD_CUMULANTS
    int transport;  // LBFD_UNITY_LEWIS or LBFD_MIXTURE_AVERAGED
    double dk[kMaxSp];   // D_k / alpha = 1 / Le_k (mixture-averaged transport)
    double cpk[kMaxSp];  // c_pk / c_p,ref (mixture-averaged transport)
};

// Launch modes: the step; the step with the reductions of the level; the
// evaluation of the current level (fields and reductions, nothing of the
// state written).
enum { kModeStep = 0, kModeStepDiag = 1, kModeFields = 2 };

// D2Q9 steps are one launch over boundary blocks and interior tiles;
// D3Q27 steps launch them separately (one kernel holding both paths slows
// the 3-D interior tiles), plus the outlet update with an outflow face.
constexpr bool fused_step(int Q) { return Q == 9; }

inline int step_launches(int Q, int nsp, const KParams &kp)
{
    const int images = kp.bimg != nullptr && kp.n_img > 0 ? 2 : 0;
    const int chem = chem_pass(nsp) && kp.n_fluid > 0 ? 3 : 0;  // counter clear, ordering, sources
    if (fused_step(Q)) return (kp.boundary_blocks + kp.interior_blocks > 0 ? 1 : 0) + images + chem;
    const bool outlet = kp.n_boundary > 0 && (kp.face[0] == LBFD_FACE_OUTFLOW || kp.face[1] == LBFD_FACE_OUTFLOW);
    return (kp.boundary_blocks > 0) + (kp.interior_blocks > 0) + (outlet ? 1 : 0) + images + chem;
}

// Where a step is launched: the context stream, and which launches (0: all;
// for per-part timing 1: interior tiles only, 2: boundary blocks, image
// points and outlet, 3: the chemistry launch only).
struct Streams {
    hipStream_t main;
    int part;
};

// Launchers (instantiated in inst/*.hip, dispatched in lbfd_dispatch.hip).
hipError_t launch_step(int Q, int nsp, int prec, int mode, const KParams &kp, const Streams &s);
hipError_t launch_init(int Q, int nsp, int prec, const KParams &kp, const double *u0,
                       const double *Ph0, dim3 grid, dim3 block, hipStream_t s);
// Keep the populations entering through inflow face `face` at the current
// level when its profile changes by -du (lbfd_dispatch.hip).
hipError_t launch_inflow_shift(int Q, int prec, const KParams &kp, int face, const double *du, hipStream_t s);
// The final diagnostics from the per-block partials (one block); with acc,
// also *acc += a * out[slot] + b (an objective's term).
hipError_t launch_finalize(const double *partials, int nblocks, double *out,
                           long long *first_bad, long long level, hipStream_t s, double *acc = nullptr,
                           int slot = 0, double a = 0.0, double b = 0.0);
bool supported(int Q, int nsp, int prec);

// Adjoint (lbfd_adjoint.hip): one backward step of the FP64 coupled step.
bool adjoint_supported(int Q, int nsp);
// The objective's share of one level: kind LBFD_OBJ_*, weight w (0 outside
// the objective's window; for the flame position w carries d x_f / d T of
// one cell, -nx / (n_fluid (T_b - T_u))).
// mid: adjoint_mid_fields(Q, nsp) x N doubles of scratch between the
// backward step's kernels.  lam_sc is written at every fluid cell (its
// entries at solid cells are left as they are).
int adjoint_mid_fields(int Q, int nsp);
hipError_t launch_adjoint(int Q, int nsp, const KParams &kp, const double *lam_pop_next, const double *lam_sc_next,
                          double *lam_pop, double *lam_sc, double *dwallT, double *dparam, double *mid, int obj_kind,
                          double obj_w, hipStream_t s);
// One forward-mode (Jacobian-vector) evaluation of the FP64 step at the
// state kp.pop_in / kp.sc_in: tangents of the inputs in, tangents of the
// outputs at fluid cells out; *dq accumulates the tangent of the level's q.
hipError_t launch_tangent(int Q, int nsp, const KParams &kp, const double *dpop, const double *dsc,
                          const double *dwallT, const double *dparam, double *dpop_out, double *dsc_out, double *dq,
                          int obj_kind, double obj_w, hipStream_t s);
// dst[i] = src[i] for i < n (float to double, on the stream).
hipError_t launch_widen(const float *src, double *dst, size_t n, hipStream_t s);
// dst[i] = v for i < n (a fill kernel, so that callers capturing a graph
// record no memset node).
hipError_t launch_fill(double *dst, int n, double v, hipStream_t s);

// The chemistry kernel specialised to a mechanism's structure
// (lbfd_chemjit.hip): its HIP source, its compile for the current device
// (cached per device and source for the process; *fn the kernel handle, or
// an error text), and its launch over kp's chemistry list (blocks of 256,
// scalars of scal_bytes).
std::string chem_jit_source(const ChemRx *rx, int n_rx, int nsp, bool fp64);
int chem_jit_build(const ChemRx *rx, int n_rx, int nsp, bool fp64, const void **fn, std::string &err);
hipError_t launch_chem_jit(const KParams &kp, unsigned blocks, size_t scal_bytes, hipStream_t s);

}  // namespace lbfd
