// lbfd_api.hip -- host side of the C ABI declared in include/lbfd.h:
// validation, device memory, the step loop on the caller's stream,
// read-back, diagnostics, checkpoints.
#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <limits>
#include <string>
#include <mutex>
#include <thread>
#include <vector>

#include "lbfd_internal.h"

using namespace lbfd;

namespace {

thread_local char g_err[512] = "";

int fail(int code, const char *fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
    return code;
}

#define HIP_TRY(expr)                                                                  \
    do {                                                                               \
        hipError_t e_ = (expr);                                                        \
        if (e_ != hipSuccess)                                                          \
            return fail(LBFD_EDEVICE, "%s failed: %s", #expr, hipGetErrorString(e_));  \
    } while (0)

constexpr double kCs2 = 1.0 / 3.0;
constexpr uint32_t kMagic = 0x4c424644u;  // "LBFD"

// Device memory of lbfd_objective_static, which allocates nothing: the
// objective's accumulator, the final diagnostics and the per-block partial
// diagnostics of its steps.  One copy per GPU, held until the process ends;
// host code reaches it only through the address hipGetSymbolAddress returns
// on that device (the array's name is a host-side stand-in).
constexpr size_t kScratchBytes = (size_t)16 << 20;
constexpr size_t kScratchAcc = 0, kScratchDiag = 256, kScratchPartials = 512;
constexpr int kMaxDevices = 64;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices];

// The scratch array's device address on the current device, looked up once
// per device (called from lbfd_init).
int scratch_address(void **out)
{
    int dev = -1;
    HIP_TRY(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return fail(LBFD_EDEVICE, "device index %d out of range", dev);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr)
            return fail(LBFD_EDEVICE, "hipGetSymbolAddress(scratch) failed: %s", hipGetErrorString(e));
        g_scratch_ptr[dev] = ptr;
    }
    *out = g_scratch_ptr[dev];
    return LBFD_OK;
}

struct StateHeader {
    uint32_t magic;
    int32_t lattice, n_species, precision, nx, ny, nz;
    int64_t level;
    uint64_t pop_bytes, sc_bytes, outlet_bytes;
};

size_t pop_elem_size(int prec) { return prec == LBFD_FP64 ? 8 : prec == LBFD_MIXED_FP32 ? 4 : 2; }
size_t sc_elem_size(int prec) { return prec == LBFD_FP64 ? 8 : 4; }

double mixture_density(const lbfd_params &p, double T, const double *Y)
{
    double s = 0.0;
    for (int k = 0; k < p.n_species; ++k) s += Y[k] / p.W[k];
    return (p.T_ref / T) * ((1.0 / s) / p.W_ref);
}

}  // namespace

struct lbfd_ctx {
    lbfd_params p;
    lbfd_reaction rx[LBFD_MAX_REACTIONS];
    int Q, D, nsp, prec;
    long long N;
    hipStream_t stream;
    Streams streams = {nullptr, 0};
    int obj_kind = LBFD_OBJ_WALL_HEAT_FLUX;  // objective of lbfd_objective / lbfd_adjoint
    int64_t obj_t0 = 0, obj_t1 = INT64_MAX;  // its window of level offsets
    long long n_fluid = 0;
    void *pop[2] = {nullptr, nullptr};
    void *sc[2] = {nullptr, nullptr};
    int cur = 0;
    uint8_t *mask = nullptr;
    uint8_t *code = nullptr;
    int *boundary = nullptr;
    long long n_boundary = 0;
    int *fluid = nullptr;               // fluid-cell list (contexts with a chemistry launch)
    int *chem_order = nullptr;          // its per-step order for the chemistry launch
    unsigned char *chem_heavy = nullptr;
    int *chem_count = nullptr;
    std::vector<int> boundary_host;
    std::vector<uint8_t> mask_host;
    std::vector<double> wall_T_host;
    int *bsrc = nullptr, *bpt = nullptr;
    uint8_t *bwk = nullptr;
    double *btw = nullptr;
    unsigned long long *bcode_pull = nullptr, *bcode_st = nullptr;  // compact codes of the same descriptors
    double *face_Td = nullptr;                                         // face_T in device memory
    char chem_msg[512] = "";  // which chemistry kernel runs, or why the specialised one does not
    int nblocks_interior = 0;
    double *wall_T = nullptr;
    double *outlet = nullptr;
    double *outlet_un = nullptr;
    double *inflow_u = nullptr;         // [2 x faces][3][nz][ny] inlet velocity profiles
    double *inflow_du = nullptr;        // [3][nz][ny] staging of a profile change
    float *bq = nullptr;                // [Q][nb] interpolated bounce-back wall distances (optional)
    int *bimg = nullptr;                // [12][nb] image point of a ghost node, -1 none (optional)
    long long n_img = 0;                // image points:
    int img_lpp = 64;                   //   lanes per Shepard row
    int2 *img_rng = nullptr;            //   Shepard list ranges
    int *img_idx = nullptr;             //   their fluid nodes
    double *img_w = nullptr;            //   and weights
    double *img_val = nullptr;          //   reconstructed values of the current level
    long long n_sup = 0;                //   distinct nodes of the Shepard lists
    int *sup_idx = nullptr;             //   their cells
    double *sup_val = nullptr;          //   and their packed (T, rho, Y_k) of the current level
    std::vector<uint8_t> bwk_host;      // host copy of the ghost kinds of the descriptors
    std::vector<double> inflow_host;   // host copy
    size_t outlet_n = 0;
    double *fields = nullptr;
    double *partials = nullptr;
    int nblocks = 0;
    double *diag_dev = nullptr;
    long long *bad_dev = nullptr;
    lbfd_reaction *rx_dev = nullptr;
    ChemRx *rxk_dev = nullptr;
    unsigned char *scratch = nullptr;   // this device's static scratch (lbfd_objective_static)
    int64_t level = 0;
    dim3 grid, block;
    KParams base;
};

static void free_ctx(lbfd_ctx *c)
{
    if (!c) return;
    void *ptrs[] = {c->pop[0], c->pop[1], c->sc[0], c->sc[1], c->mask, c->code, c->boundary, c->bsrc, c->bpt, c->bwk,
                    c->btw, c->wall_T, c->outlet, c->outlet_un, c->inflow_u, c->inflow_du, c->bq,
                    c->bimg, c->img_rng, c->img_idx, c->img_w, c->img_val, c->sup_idx, c->sup_val,
                    c->fields, c->partials, c->diag_dev, c->bad_dev, c->rx_dev, c->rxk_dev, c->fluid,
                    c->chem_order, c->chem_heavy, c->chem_count, c->bcode_pull, c->bcode_st, c->face_Td};
    for (void *q : ptrs)
        if (q) (void)hipFree(q);
    delete c;
}

static int validate(const lbfd_params *p, const uint8_t *mask, const double *T0, const double *Y0)
{
    if (!p || !mask || !T0 || !Y0) return fail(LBFD_EINVAL, "null argument");
    if (p->lattice != LBFD_D2Q9 && p->lattice != LBFD_D3Q27) return fail(LBFD_EINVAL, "lattice must be 9 or 27");
    if (p->nx < 1 || p->ny < 1 || p->nz < 1) return fail(LBFD_EINVAL, "grid sizes must be positive");
    if ((long long)p->nx * p->ny * p->nz >= (1LL << 29))
        return fail(LBFD_EINVAL, "box too large (at most 2^29 cells: 32-bit byte offsets per field)");
    if (p->lattice == LBFD_D2Q9 && p->nz != 1) return fail(LBFD_EINVAL, "D2Q9 needs nz == 1");
    if (p->precision < LBFD_FP64 || p->precision > LBFD_MIXED_FP16) return fail(LBFD_EINVAL, "bad precision");
    if (p->n_species < 1 || p->n_species > LBFD_MAX_SPECIES) return fail(LBFD_EINVAL, "bad species count");
    if (!supported(p->lattice, p->n_species, p->precision))
        return fail(LBFD_EINVAL, "no kernel built for lattice %d, %d species, precision %d", p->lattice,
                    p->n_species, p->precision);
    if (!(p->tau > 0.5)) return fail(LBFD_EINVAL, "tau must exceed 1/2");
    if (!(p->prandtl > 0.0)) return fail(LBFD_EINVAL, "prandtl must be positive");
    const int D = p->lattice == LBFD_D2Q9 ? 2 : 3;
    const double alpha = kCs2 * (p->tau - 0.5) / p->prandtl;
    if (alpha > (D == 2 ? 3.0 / 16.0 : 1.0 / 8.0))
        return fail(LBFD_EINVAL, "diffusivity %g above the explicit stability bound", alpha);
    for (int f = 0; f < 6; ++f) {
        if (p->face[f] < LBFD_FACE_PERIODIC || p->face[f] > LBFD_FACE_WALL_ADIABATIC)
            return fail(LBFD_EINVAL, "bad face kind on face %d", f);
        if (p->face[f] == LBFD_FACE_OUTFLOW && f >= 2) return fail(LBFD_EINVAL, "only x faces may be OUTFLOW");
        if (D == 2 && f >= 4 && p->face[f] != LBFD_FACE_PERIODIC)
            return fail(LBFD_EINVAL, "z faces of a D2Q9 box must be periodic");
    }
    if (p->n_reactions < 0 || p->n_reactions > LBFD_MAX_REACTIONS) return fail(LBFD_EINVAL, "bad reaction count");
    if (p->n_reactions > 0 && !p->rxn) return fail(LBFD_EINVAL, "null reaction array");
    for (int j = 0; j < p->n_reactions; ++j) {
        const lbfd_reaction &r = p->rxn[j];
        if (r.n_react < 0 || r.n_react > 4) return fail(LBFD_EINVAL, "reaction %d: bad reactant count", j);
        for (int m = 0; m < r.n_react; ++m)
            if (r.react[m] < 0 || r.react[m] >= p->n_species)
                return fail(LBFD_EINVAL, "reaction %d: bad reactant index", j);
        double s = 0.0;
        for (int k = 0; k < p->n_species; ++k) s += r.nu_mass[k];
        if (std::fabs(s) > 1e-12) return fail(LBFD_EINVAL, "reaction %d does not conserve mass", j);
    }
    for (int k = 0; k < p->n_species; ++k)
        if (!(p->W[k] > 0.0)) return fail(LBFD_EINVAL, "molar masses must be positive");
    if (!(p->T_ref > 0.0) || !(p->W_ref > 0.0)) return fail(LBFD_EINVAL, "T_ref, W_ref must be positive");
    if (p->check_every < 0) return fail(LBFD_EINVAL, "check_every must be >= 0");
    if (p->collision != LBFD_CENTRAL_MOMENTS && p->collision != LBFD_CUMULANTS)
        return fail(LBFD_EINVAL, "bad collision kind %d", p->collision);
    if (p->transport != LBFD_UNITY_LEWIS && p->transport != LBFD_MIXTURE_AVERAGED)
        return fail(LBFD_EINVAL, "bad transport model %d", p->transport);
    if (p->transport == LBFD_MIXTURE_AVERAGED)
        for (int k = 0; k < p->n_species; ++k) {
            if (!(p->lewis[k] > 0.0) || !std::isfinite(p->lewis[k]) || !(p->cp[k] > 0.0) || !std::isfinite(p->cp[k]))
                return fail(LBFD_EINVAL, "species %d: Lewis number and heat capacity must be positive", k);
            if (alpha / p->lewis[k] > (D == 2 ? 3.0 / 16.0 : 1.0 / 8.0))
                return fail(LBFD_EINVAL, "species %d: diffusivity %g above the explicit stability bound", k,
                            alpha / p->lewis[k]);
        }
    const long long N = (long long)p->nx * p->ny * p->nz;
    long long nfluid = 0;
    for (long long i = 0; i < N; ++i) {
        if (mask[i] > LBFD_SOLID_ADIABATIC) return fail(LBFD_EINVAL, "bad mask value at cell %lld", i);
        if (mask[i] != LBFD_FLUID) continue;
        ++nfluid;
        double s = 0.0;
        for (int k = 0; k < p->n_species; ++k) s += Y0[k * N + i];
        if (std::fabs(s - 1.0) > 1e-12) return fail(LBFD_EINVAL, "mass fractions do not sum to 1 at cell %lld", i);
        if (!(T0[i] > 0.0)) return fail(LBFD_EINVAL, "temperature must be positive at cell %lld", i);
    }
    if (nfluid == 0) return fail(LBFD_EINVAL, "no fluid cell");
    return LBFD_OK;
}

// Brick shape of the boundary-cell list order (x, y[, z]); 0: cell index
// order.  Measured on MI355X: 16 x 16 bricks shorten the 2-D boundary part,
// 3-D bricks lengthen it.
constexpr int kBrick2D[2] = {16, 16};
constexpr int kBrick3D[3] = {0, 0, 0};

// Cell codes: solid; interior fluid when every pull source (the 3^D - 1
// neighbours) and every finite-difference point (+-1, +-2 along each axis)
// lies inside the box without wrapping and is fluid; boundary fluid
// otherwise.  Returns the boundary cells in the brick order above.
static void classify_cells(const lbfd_params &p, const uint8_t *mask, std::vector<uint8_t> &code,
                           std::vector<int> &boundary)
{
    const int D = p.lattice == LBFD_D2Q9 ? 2 : 3;
    const long long N = (long long)p.nx * p.ny * p.nz;
    const long long sy = p.nx, sz = (long long)p.nx * p.ny;
    code.assign(N, kCodeSolid);
    boundary.clear();
    int off[40][3];
    int no = 0;
    for (int dz = (D == 3 ? -1 : 0); dz <= (D == 3 ? 1 : 0); ++dz)
        for (int dy = -1; dy <= 1; ++dy)
            for (int dx = -1; dx <= 1; ++dx)
                if (dx || dy || dz) {
                    off[no][0] = dx;
                    off[no][1] = dy;
                    off[no][2] = dz;
                    ++no;
                }
    for (int d = 0; d < D; ++d)
        for (int s2 = -2; s2 <= 2; s2 += 4) {
            off[no][0] = off[no][1] = off[no][2] = 0;
            off[no][d] = s2;
            ++no;
        }
    for (int z = 0; z < p.nz; ++z)
        for (int y = 0; y < p.ny; ++y)
            for (int x = 0; x < p.nx; ++x) {
                const long long i = z * sz + y * sy + x;
                if (mask[i] != LBFD_FLUID) continue;
                bool interior = true;
                for (int o = 0; o < no && interior; ++o) {
                    const int qx = x + off[o][0], qy = y + off[o][1], qz = z + off[o][2];
                    if (qx < 0 || qx >= p.nx || qy < 0 || qy >= p.ny || qz < 0 || qz >= p.nz ||
                        mask[qz * sz + qy * sy + qx] != LBFD_FLUID)
                        interior = false;
                }
                code[i] = interior ? kCodeInterior : kCodeBoundary;
                if (!interior) boundary.push_back((int)i);
            }
    // Order of the boundary-cell list (the cell each thread takes): by
    // bricks of the box, cell index within a brick, so that the neighbour
    // gathers of one wave stay in a compact region.  (0: cell index order.)
    const int bx = D == 2 ? kBrick2D[0] : kBrick3D[0], by = D == 2 ? kBrick2D[1] : kBrick3D[1],
              bz = D == 2 ? 1 : kBrick3D[2];
    if (bx > 0) {
        const long long nbx = (p.nx + bx - 1) / bx, nby = (p.ny + by - 1) / by;
        auto brick = [&](int i) {
            const long long x = i % p.nx, y = (i / p.nx) % p.ny, z = i / sz;
            return ((z / bz) * nby + y / by) * nbx + x / bx;
        };
        std::stable_sort(boundary.begin(), boundary.end(), [&](int a, int b) { return brick(a) < brick(b); });
    }
}

// Host copy of the kernels' neighbour rule: periodic faces wrap; outside
// any other face the point is that face (walls before inflow before
// outflow, lower axis and face first); inside, the mask decides.
struct HostNb {
    int kind, face;
    long long idx;
    double Tw;
};

static HostNb host_classify(const lbfd_params &p, const uint8_t *mask, const double *wall_T, int x, int y, int z)
{
    int q[3] = {x, y, z};
    const int n[3] = {p.nx, p.ny, p.nz};
    int best_face = -1, best_rank = 99;
    for (int d = 0; d < 3; ++d) {
        if (q[d] < 0 || q[d] >= n[d]) {
            const int f = 2 * d + (q[d] >= n[d] ? 1 : 0);
            if (p.face[f] == LBFD_FACE_PERIODIC) {
                q[d] = ((q[d] % n[d]) + n[d]) % n[d];
            } else {
                const int rank = (p.face[f] == LBFD_FACE_WALL || p.face[f] == LBFD_FACE_WALL_ADIABATIC) ? 0
                               : p.face[f] == LBFD_FACE_INFLOW ? 1 : 2;
                if (rank < best_rank) {
                    best_rank = rank;
                    best_face = f;
                }
            }
        }
    }
    HostNb r{kFluid, best_face, 0, 0.0};
    if (best_face >= 0) {
        const int kd = p.face[best_face];
        r.kind = kd == LBFD_FACE_WALL ? kIso : kd == LBFD_FACE_WALL_ADIABATIC ? kAdia : kd == LBFD_FACE_INFLOW ? kInflow : kOutflow;
        r.Tw = p.face_T[best_face];
        return r;
    }
    r.idx = ((long long)q[2] * p.ny + q[1]) * p.nx + q[0];
    const uint8_t m = mask[r.idx];
    r.kind = m == LBFD_FLUID ? kFluid : m == LBFD_SOLID_ISOTHERMAL ? kIso : kAdia;
    if (r.kind == kIso) r.Tw = wall_T[r.idx];
    return r;
}

// Per boundary cell: pull source of every direction and, per axis and
// offset m = -2, -1, 1, 2, the index of the value point (or of the ghost's
// image: the cell itself for m = +-1 behind a first-neighbour wall, the
// cell on the other side for m = +-2, clamped to the cell when not fluid,
// or the first neighbour when the wall is the second), the kind of the wall
// behind a ghost and its temperature.
// bit f set for a periodic face f
static unsigned periodic_bits(const lbfd_params &p)
{
    unsigned b = 0;
    for (int f = 0; f < 6; ++f) b |= p.face[f] == LBFD_FACE_PERIODIC ? 1u << f : 0u;
    return b;
}

static int build_descriptors(lbfd_ctx *c)
{
    const lbfd_params &p = c->p;
    const long long nb = c->n_boundary;
    if (nb == 0) return LBFD_OK;
    const int Q = c->Q, D = c->D;
    const uint8_t *mask = c->mask_host.data();
    const double *wT = c->wall_T_host.data();
    std::vector<int> src((size_t)Q * nb, kSrcBounce), pt((size_t)12 * nb, 0);
    std::vector<uint8_t> wk((size_t)12 * nb, kFluid);
    std::vector<double> tw((size_t)12 * nb, 0.0);
    const int zr = Q == 27 ? 1 : 0;
    for (long long t = 0; t < nb; ++t) {
        const long long idx = c->boundary_host[t];
        const int x = (int)(idx % p.nx), y = (int)((idx / p.nx) % p.ny), z = (int)(idx / ((long long)p.nx * p.ny));
        int i = 0;
        for (int cz = -zr; cz <= zr; ++cz)
            for (int cy = -1; cy <= 1; ++cy)
                for (int cx = -1; cx <= 1; ++cx, ++i) {
                    const HostNb s = host_classify(p, mask, wT, x - cx, y - cy, z - cz);
                    int v = kSrcBounce;
                    if (s.kind == kFluid) {
                        v = (int)s.idx;
                    } else if (s.kind == kInflow) {
                        v = kSrcInflow;
                    } else if (s.kind == kOutflow) {
                        const int sign = (s.face & 1) ? 1 : -1;
                        if (host_classify(p, mask, wT, x - sign, y, z).kind == kFluid) v = kSrcOutlet;
                    }
                    src[(size_t)i * nb + t] = v;
                }
        for (int d = 0; d < D; ++d) {
            const int ox = d == 0, oy = d == 1, oz = d == 2;
            for (int sg = -1; sg <= 1; sg += 2) {
                const int j1 = sg < 0 ? 1 : 2, j2 = sg < 0 ? 0 : 3;
                const size_t s1 = (size_t)(d * 4 + j1) * nb + t, s2 = (size_t)(d * 4 + j2) * nb + t;
                const HostNb c1 = host_classify(p, mask, wT, x + sg * ox, y + sg * oy, z + sg * oz);
                if (c1.kind != kFluid) {
                    const HostNb cm = host_classify(p, mask, wT, x - sg * ox, y - sg * oy, z - sg * oz);
                    pt[s1] = (int)idx;
                    wk[s1] = (uint8_t)c1.kind;
                    tw[s1] = c1.Tw;
                    pt[s2] = cm.kind == kFluid ? (int)cm.idx : (int)idx;
                    wk[s2] = (uint8_t)c1.kind;
                    tw[s2] = c1.Tw;
                } else {
                    pt[s1] = (int)c1.idx;
                    const HostNb c2 = host_classify(p, mask, wT, x + 2 * sg * ox, y + 2 * sg * oy, z + 2 * sg * oz);
                    if (c2.kind != kFluid) {
                        pt[s2] = (int)c1.idx;
                        wk[s2] = (uint8_t)c2.kind;
                        tw[s2] = c2.Tw;
                    } else {
                        pt[s2] = (int)c2.idx;
                    }
                }
            }
        }
    }
    // the compact codes of the same descriptors (what the kernels without
    // curved-wall links read), each decoded entry checked against them
    std::vector<unsigned long long> pcode((size_t)nb, 0ull), scode((size_t)nb, 0ull);
    for (long long t = 0; t < nb; ++t) {
        const long long idx = c->boundary_host[t];
        const int x = (int)(idx % p.nx), y = (int)((idx / p.nx) % p.ny), z = (int)(idx / ((long long)p.nx * p.ny));
        unsigned long long pc = 0;
        int i = 0;
        for (int cz = -zr; cz <= zr; ++cz)
            for (int cy = -1; cy <= 1; ++cy)
                for (int cx = -1; cx <= 1; ++cx, ++i) {
                    const int v = src[(size_t)i * nb + t];
                    const int kind = v >= 0 ? kPullFluid : v == kSrcBounce ? kPullBounce
                                   : v == kSrcInflow ? kPullInflow : kPullOutlet;
                    pc |= (unsigned long long)kind << (2 * i);
                    if (kind == kPullFluid && cell_at(x, y, z, -cx, -cy, -cz, p.nx, p.ny, p.nz) != v)
                        return fail(LBFD_EINVAL, "internal: pull code of boundary cell %lld, direction %d", idx, i);
                }
        unsigned long long sc = 0;
        for (int d = 0; d < D; ++d)
            for (int j = 0; j < 4; ++j) {
                const size_t sl = (size_t)(d * 4 + j) * nb + t;
                const int w = wk[sl], w1 = wk[(size_t)(d * 4 + (j < 2 ? 1 : 2)) * nb + t];
                const bool second = j == 0 || j == 3;
                const int img = !second ? (w == kFluid ? kImgSelf : kImgCell)
                              : w1 != kFluid ? (pt[sl] == idx ? kImgCell : kImgMirror)
                              : w != kFluid ? kImgSame : kImgSelf;
                sc |= (unsigned long long)(w | img << 3) << (5 * (4 * d + j));
            }
        for (int d = 0; d < D; ++d)
            for (int j = 0; j < 4; ++j) {
                const size_t sl = (size_t)(d * 4 + j) * nb + t;
                const bool ok = decode_kind(sc, d, j) == wk[sl] &&
                                decode_point(sc, d, j, idx, x, y, z, p.nx, p.ny, p.nz) == pt[sl] &&
                                (wk[sl] != kIso ||
                                 decode_wall_T(sc, d, j, x, y, z, p.nx, p.ny, p.nz, periodic_bits(p), p.face_T, wT) == tw[sl]);
                if (!ok) return fail(LBFD_EINVAL, "internal: stencil code of boundary cell %lld, axis %d, slot %d", idx, d, j);
            }
        pcode[t] = pc;
        scode[t] = sc;
    }
    HIP_TRY(hipMemcpy(c->bcode_pull, pcode.data(), pcode.size() * sizeof(unsigned long long), hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(c->bcode_st, scode.data(), scode.size() * sizeof(unsigned long long), hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(c->face_Td, p.face_T, sizeof(p.face_T), hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(c->bsrc, src.data(), src.size() * sizeof(int), hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(c->bpt, pt.data(), pt.size() * sizeof(int), hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(c->bwk, wk.data(), wk.size(), hipMemcpyHostToDevice));
    c->bwk_host = wk;
    HIP_TRY(hipMemcpy(c->btw, tw.data(), tw.size() * sizeof(double), hipMemcpyHostToDevice));
    return LBFD_OK;
}

static KParams make_kparams(const lbfd_ctx *c)
{
    const lbfd_params &p = c->p;
    KParams k;
    memset(&k, 0, sizeof(k));
    k.nx = p.nx;
    k.ny = p.ny;
    k.nz = p.nz;
    k.N = c->N;
    for (int f = 0; f < 6; ++f) {
        k.face[f] = p.face[f];
        k.face_T[f] = p.face_T[f];
    }
    k.mask = c->mask;
    k.code = c->code;
    k.boundary = c->boundary;
    k.n_boundary = c->n_boundary;
    k.fluid = c->fluid;
    k.n_fluid = c->n_fluid;
    k.chem_order = c->chem_order;
    k.chem_heavy = c->chem_heavy;
    k.chem_count = c->chem_count;
    k.boundary_blocks = c->nblocks - c->nblocks_interior;
    k.interior_blocks = c->nblocks_interior;
    k.block_begin = 0;
    k.tiles_x = (int)c->grid.x;
    k.tiles_y = (int)c->grid.y;
    k.bsrc = c->bsrc;
    k.bcode_pull = c->bcode_pull;
    k.bcode_st = c->bcode_st;
    k.face_Td = c->face_Td;
    k.periodic_bits = periodic_bits(c->p);
    k.bpt = c->bpt;
    k.bwk = c->bwk;
    k.btw = c->btw;
    k.wall_T = c->wall_T;
    k.outlet = c->outlet;
    k.outlet_un = c->outlet_un;
    k.inflow_u = c->inflow_u;
    k.bq = c->bq;
    k.bimg = c->bimg;
    k.n_img = c->n_img;
    k.img_lpp = c->img_lpp;
    k.img_rng = c->img_rng;
    k.img_idx = c->img_idx;
    k.img_w = c->img_w;
    k.img_val = c->img_val;
    k.n_sup = c->n_sup;
    k.sup_idx = c->sup_idx;
    k.sup_val = c->sup_val;
    k.fields = c->fields;
    k.partials = c->partials;
    k.rx = c->rx_dev;
    k.rxk = c->rxk_dev;
    k.n_rx = p.n_reactions;
    k.chem_substeps_max = p.chem_substeps_max;
    k.omega2 = 1.0 / p.tau;
    k.omega3 = p.omega3;
    k.omega4 = p.omega4;
    k.alpha = kCs2 * (p.tau - 0.5) / p.prandtl;
    k.dt_phys = p.dt_phys;
    k.T_ref = p.T_ref;
    k.W_ref = p.W_ref;
    k.T_ref_over_W_ref = p.T_ref / p.W_ref;
    for (int s = 0; s < c->nsp; ++s) {
        k.invW[s] = 1.0 / p.W[s];
        k.Y_in[s] = p.Y_in[s];
    }
    for (int d = 0; d < 3; ++d) k.u_in[d] = p.u_in[d];
    k.T_in = p.T_in;
    k.rho_in = mixture_density(p, p.T_in, p.Y_in);
    k.T_u = p.T_u;
    k.T_b = p.T_b;
    k.collision = p.collision;
    k.transport = p.transport;
    for (int s = 0; s < c->nsp; ++s) {
        k.dk[s] = p.transport == LBFD_MIXTURE_AVERAGED ? 1.0 / p.lewis[s] : 1.0;
        k.cpk[s] = p.transport == LBFD_MIXTURE_AVERAGED ? p.cp[s] : 1.0;
    }
    return k;
}

// The reactions of the context on the device, in both forms the kernels
// read (the ABI struct for the adjoint, ChemRx for the chemistry: A dt_phys
// formed once here), and whether a temperature exponent is in use.
static int upload_reactions(lbfd_ctx *c)
{
    const lbfd_params &p = c->p;
    ChemRx h[LBFD_MAX_REACTIONS];
    memset(h, 0, sizeof(h));
    int anyb = 0, nreact = 0;
    for (int j = 0; j < p.n_reactions; ++j) {
        const lbfd_reaction &r = c->rx[j];
        h[j].adt = r.A * p.dt_phys;
        constexpr double kScale = 0x1.71547652b82fep+8;  // 256 / ln 2
        h[j].bs = r.b * kScale;
        h[j].tas = r.Ta * kScale;
        h[j].lnadts = h[j].adt > 0.0 ? std::log(h[j].adt) * kScale : -HUGE_VAL;
        h[j].b = r.b;
        h[j].ta = r.Ta;
        h[j].q = r.q_over_cp;
        h[j].n_react = r.n_react;
        // unused reactant slots index the chemistry's constant-1 entry
        for (int m = 0; m < 4; ++m) h[j].react[m] = m < r.n_react ? r.react[m] : c->nsp;
        for (int k = 0; k < c->nsp; ++k) h[j].nu[k] = r.nu_mass[k];
        anyb |= r.b != 0.0;
        nreact = std::max(nreact, r.n_react);
    }
    if (p.n_reactions > 0) {
        HIP_TRY(hipMemcpy(c->rx_dev, c->rx, sizeof(lbfd_reaction) * p.n_reactions, hipMemcpyHostToDevice));
        HIP_TRY(hipMemcpy(c->rxk_dev, h, sizeof(ChemRx) * p.n_reactions, hipMemcpyHostToDevice));
    }
    c->base.chem_anyb = anyb;
    c->base.chem_nreact = nreact;
    // the chemistry launch specialised to the mechanism's structure
    // (LBFD_CHEM_JIT=0 in the environment keeps the generic kernel); a
    // failed compile leaves the generic kernel and says why
    c->base.chem_jit = nullptr;
    if (!chem_pass(c->nsp) || p.n_reactions == 0 || p.transport != LBFD_UNITY_LEWIS) {
        snprintf(c->chem_msg, sizeof c->chem_msg, "generic (the chemistry runs inside the step, or "
                 "mixture-averaged transport)");
    } else if (const char *env = getenv("LBFD_CHEM_JIT"); env && strcmp(env, "0") == 0) {
        snprintf(c->chem_msg, sizeof c->chem_msg, "generic (LBFD_CHEM_JIT=0)");
    } else {
        std::string err;
        const void *fn = nullptr;
        if (chem_jit_build(h, p.n_reactions, c->nsp, c->prec == LBFD_FP64, &fn, err) == 0) {
            c->base.chem_jit = fn;
            snprintf(c->chem_msg, sizeof c->chem_msg, "specialised");
        } else {
            snprintf(c->chem_msg, sizeof c->chem_msg, "generic (%s)", err.c_str());
        }
    }
    return LBFD_OK;
}

// Convert and upload a double host array into a device scalar buffer.
static int upload_scalars(lbfd_ctx *c, void *dst, const double *T0, const double *Y0)
{
    const long long N = c->N;
    const size_t n = (size_t)(1 + c->nsp) * N;
    if (c->prec == LBFD_FP64) {
        HIP_TRY(hipMemcpy(dst, T0, N * sizeof(double), hipMemcpyHostToDevice));
        HIP_TRY(hipMemcpy((double *)dst + N, Y0, (size_t)c->nsp * N * sizeof(double), hipMemcpyHostToDevice));
    } else {
        std::vector<float> tmp(n);
        for (long long i = 0; i < N; ++i) tmp[i] = (float)T0[i];
        for (size_t i = 0; i < (size_t)c->nsp * N; ++i) tmp[N + i] = (float)Y0[i];
        HIP_TRY(hipMemcpy(dst, tmp.data(), n * sizeof(float), hipMemcpyHostToDevice));
    }
    return LBFD_OK;
}

extern "C" {

int lbfd_init(const lbfd_params *p, const uint8_t *mask, const double *wall_T, const double *T0,
              const double *Y0, const double *u0, const double *Ph0, void *hip_stream, lbfd_ctx **out)
{
    if (!out) return fail(LBFD_EINVAL, "null output pointer");
    *out = nullptr;
    int rc = validate(p, mask, T0, Y0);
    if (rc) return rc;
    lbfd_ctx *c = new (std::nothrow) lbfd_ctx();
    if (!c) return fail(LBFD_ENOMEM, "host allocation failed");
    c->p = *p;
    for (int j = 0; j < p->n_reactions; ++j) c->rx[j] = p->rxn[j];
    c->p.rxn = nullptr;
    c->Q = p->lattice;
    c->D = p->lattice == LBFD_D2Q9 ? 2 : 3;
    c->nsp = p->n_species;
    c->prec = p->precision;
    c->N = (long long)p->nx * p->ny * p->nz;
    c->stream = (hipStream_t)hip_stream;
    const long long N = c->N;
    const size_t pop_bytes = (size_t)c->Q * N * pop_elem_size(c->prec);
    const size_t sc_bytes = (size_t)(1 + c->nsp) * N * sc_elem_size(c->prec);
    c->outlet_n = (size_t)2 * c->Q * p->ny * p->nz;
    if (c->D == 2) {
        c->block = dim3(64, 4, 1);
    } else {
        c->block = dim3(64, 2, 2);
    }
    c->grid = dim3((p->nx + c->block.x - 1) / c->block.x, (p->ny + c->block.y - 1) / c->block.y,
                   (p->nz + c->block.z - 1) / c->block.z);
    if (c->N >= (1LL << 29)) {
        delete c;
        return fail(LBFD_EINVAL, "box too large (at most 2^29 cells: 32-bit byte offsets per field)");
    }
    std::vector<uint8_t> code;
    std::vector<int> boundary;
    classify_cells(*p, mask, code, boundary);
    c->n_boundary = (long long)boundary.size();
    for (long long i = 0; i < c->N; ++i) c->n_fluid += mask[i] == LBFD_FLUID;
    c->nblocks_interior = c->grid.x * c->grid.y * c->grid.z;
    // boundary blocks padded to a multiple of 8 (one per XCD in turn), so
    // that the interior tiles after them start on XCD 0
    c->nblocks = c->nblocks_interior + (int)(((c->n_boundary + kBlock - 1) / kBlock + 7) / 8 * 8);

#define ALLOC(ptr, bytes)                                                                   \
    do {                                                                                    \
        const hipError_t ea_ = hipMalloc((void **)&(ptr), (bytes));                         \
        if (ea_ != hipSuccess) {                                                            \
            free_ctx(c);                                                                    \
            return fail(LBFD_ENOMEM, "hipMalloc of %zu bytes failed: %s", (size_t)(bytes), \
                        hipGetErrorString(ea_));                                            \
        }                                                                                   \
    } while (0)
    ALLOC(c->pop[0], pop_bytes);
    ALLOC(c->pop[1], pop_bytes);
    ALLOC(c->sc[0], sc_bytes);
    ALLOC(c->sc[1], sc_bytes);
    ALLOC(c->mask, N);
    ALLOC(c->code, N);
    ALLOC(c->boundary, sizeof(int) * (boundary.empty() ? 1 : boundary.size()));
    {
        const size_t nbd = boundary.empty() ? 1 : boundary.size();
        ALLOC(c->bsrc, sizeof(int) * c->Q * nbd);
        ALLOC(c->bpt, sizeof(int) * 12 * nbd);
        ALLOC(c->bwk, 12 * nbd);
        ALLOC(c->btw, sizeof(double) * 12 * nbd);
        ALLOC(c->bcode_pull, sizeof(unsigned long long) * nbd);
        ALLOC(c->bcode_st, sizeof(unsigned long long) * nbd);
        ALLOC(c->face_Td, sizeof(double) * 6);
    }
    ALLOC(c->wall_T, N * sizeof(double));
    ALLOC(c->outlet, c->outlet_n * sizeof(double));
    ALLOC(c->outlet_un, (size_t)2 * p->ny * p->nz * sizeof(double));
    ALLOC(c->inflow_u, (size_t)6 * p->ny * p->nz * sizeof(double));
    ALLOC(c->inflow_du, (size_t)3 * p->ny * p->nz * sizeof(double));
    ALLOC(c->partials, (size_t)c->nblocks * kNDiag * sizeof(double));
    ALLOC(c->diag_dev, kNDiag * sizeof(double));
    ALLOC(c->bad_dev, sizeof(long long));
    ALLOC(c->rx_dev, sizeof(lbfd_reaction) * LBFD_MAX_REACTIONS);
    ALLOC(c->rxk_dev, sizeof(ChemRx) * LBFD_MAX_REACTIONS);
    if (chem_pass(c->nsp)) {
        ALLOC(c->fluid, sizeof(int) * (size_t)c->n_fluid);
        ALLOC(c->chem_order, sizeof(int) * (size_t)c->n_fluid);
        ALLOC(c->chem_heavy, (size_t)N);
        ALLOC(c->chem_count, 2 * sizeof(int));
    }
#undef ALLOC

#define TRY_OR_FREE(expr)            \
    do {                             \
        int r_ = (expr);             \
        if (r_) {                    \
            free_ctx(c);             \
            return r_;               \
        }                            \
    } while (0)
#define HIP_OR_FREE(expr)                                                              \
    do {                                                                               \
        hipError_t e_ = (expr);                                                        \
        if (e_ != hipSuccess) {                                                        \
            free_ctx(c);                                                               \
            return fail(LBFD_EDEVICE, "%s failed: %s", #expr, hipGetErrorString(e_));  \
        }                                                                              \
    } while (0)
    HIP_OR_FREE(hipMemset(c->pop[0], 0, pop_bytes));
    HIP_OR_FREE(hipMemset(c->pop[1], 0, pop_bytes));
    HIP_OR_FREE(hipMemset(c->outlet, 0, c->outlet_n * sizeof(double)));
    {
        // both x faces start with the uniform inflow velocity of the parameters
        const size_t nf = (size_t)p->ny * p->nz;
        c->inflow_host.assign(6 * nf, 0.0);
        for (int f = 0; f < 2; ++f)
            for (int d = 0; d < 3; ++d)
                for (size_t i = 0; i < nf; ++i) c->inflow_host[(3 * f + d) * nf + i] = p->u_in[d];
        HIP_OR_FREE(hipMemcpy(c->inflow_u, c->inflow_host.data(), 6 * nf * sizeof(double), hipMemcpyHostToDevice));
    }
    HIP_OR_FREE(hipMemcpy(c->mask, mask, N, hipMemcpyHostToDevice));
    HIP_OR_FREE(hipMemcpy(c->code, code.data(), N, hipMemcpyHostToDevice));
    if (!boundary.empty())
        HIP_OR_FREE(hipMemcpy(c->boundary, boundary.data(), sizeof(int) * boundary.size(), hipMemcpyHostToDevice));
    c->mask_host.assign(mask, mask + N);
    if (wall_T)
        c->wall_T_host.assign(wall_T, wall_T + N);
    else
        c->wall_T_host.assign(N, 300.0);
    HIP_OR_FREE(hipMemcpy(c->wall_T, c->wall_T_host.data(), N * sizeof(double), hipMemcpyHostToDevice));
    c->boundary_host = boundary;
    if (c->fluid) {
        std::vector<int> fl;
        fl.reserve((size_t)c->n_fluid);
        for (long long i = 0; i < N; ++i)
            if (mask[i] == LBFD_FLUID) fl.push_back((int)i);
        HIP_OR_FREE(hipMemcpy(c->fluid, fl.data(), fl.size() * sizeof(int), hipMemcpyHostToDevice));
        // every cell starts as light (the first step's order is the list's)
        HIP_OR_FREE(hipMemset(c->chem_heavy, 0, (size_t)N));
        HIP_OR_FREE(hipMemset(c->chem_count, 0, 2 * sizeof(int)));
    }
    TRY_OR_FREE(build_descriptors(c));
    long long minus1 = -1;
    HIP_OR_FREE(hipMemcpy(c->bad_dev, &minus1, sizeof(minus1), hipMemcpyHostToDevice));
    TRY_OR_FREE(upload_scalars(c, c->sc[0], T0, Y0));
    TRY_OR_FREE(upload_scalars(c, c->sc[1], T0, Y0));

    c->streams.main = c->stream;
    c->base = make_kparams(c);
    TRY_OR_FREE(upload_reactions(c));
    {
        void *sp = nullptr;
        TRY_OR_FREE(scratch_address(&sp));
        c->scratch = (unsigned char *)sp;
    }
    double *u0_dev = nullptr, *Ph0_dev = nullptr;
    if (u0) {
        HIP_OR_FREE(hipMalloc((void **)&u0_dev, (size_t)c->D * N * sizeof(double)));
        HIP_OR_FREE(hipMemcpy(u0_dev, u0, (size_t)c->D * N * sizeof(double), hipMemcpyHostToDevice));
    }
    if (Ph0) {
        HIP_OR_FREE(hipMalloc((void **)&Ph0_dev, N * sizeof(double)));
        HIP_OR_FREE(hipMemcpy(Ph0_dev, Ph0, N * sizeof(double), hipMemcpyHostToDevice));
    }
    KParams k = c->base;
    k.sc_in = c->sc[0];
    k.pop_out = c->pop[0];
    hipError_t e = launch_init(c->Q, c->nsp, c->prec, k, u0_dev, Ph0_dev, c->grid, c->block, c->stream);
    hipError_t e2 = hipStreamSynchronize(c->stream);
    if (u0_dev) (void)hipFree(u0_dev);
    if (Ph0_dev) (void)hipFree(Ph0_dev);
    if (e != hipSuccess || e2 != hipSuccess) {
        free_ctx(c);
        return fail(LBFD_EDEVICE, "init kernel failed: %s", hipGetErrorString(e != hipSuccess ? e : e2));
    }
#undef TRY_OR_FREE
#undef HIP_OR_FREE
    c->cur = 0;
    c->level = 0;
    *out = c;
    return LBFD_OK;
}

int lbfd_init_dev(const lbfd_params *p, const uint8_t *mask, const double *wall_T, const double *T0,
                  const double *Y0, const double *u0, const double *Ph0, void *hip_stream, lbfd_ctx **out)
{
    if (!out) return fail(LBFD_EINVAL, "null output pointer");
    *out = nullptr;
    if (!p || !mask || !T0 || !Y0) return fail(LBFD_EINVAL, "null argument");
    if (p->nx < 1 || p->ny < 1 || p->nz < 1) return fail(LBFD_EINVAL, "grid sizes must be positive");
    if ((long long)p->nx * p->ny * p->nz >= (1LL << 29))
        return fail(LBFD_EINVAL, "box too large (at most 2^29 cells: 32-bit byte offsets per field)");
    if (p->n_species < 1 || p->n_species > LBFD_MAX_SPECIES) return fail(LBFD_EINVAL, "bad species count");
    if (p->lattice != LBFD_D2Q9 && p->lattice != LBFD_D3Q27) return fail(LBFD_EINVAL, "lattice must be 9 or 27");
    const size_t N = (size_t)p->nx * p->ny * p->nz, D = p->lattice == LBFD_D2Q9 ? 2 : 3;
    // the inputs are validated and laid out on the host: bring them over
    std::vector<uint8_t> hm;
    std::vector<double> hw, hT, hY, hu, hP;
    try {
        hm.resize(N);
        hT.resize(N);
        hY.resize((size_t)p->n_species * N);
        if (wall_T) hw.resize(N);
        if (u0) hu.resize(D * N);
        if (Ph0) hP.resize(N);
    } catch (const std::bad_alloc &) {
        return fail(LBFD_ENOMEM, "host staging of the initial state failed");
    }
    hipStream_t st = (hipStream_t)hip_stream;
    HIP_TRY(hipStreamSynchronize(st));
    HIP_TRY(hipMemcpy(hm.data(), mask, N, hipMemcpyDeviceToHost));
    HIP_TRY(hipMemcpy(hT.data(), T0, N * sizeof(double), hipMemcpyDeviceToHost));
    HIP_TRY(hipMemcpy(hY.data(), Y0, hY.size() * sizeof(double), hipMemcpyDeviceToHost));
    if (wall_T) HIP_TRY(hipMemcpy(hw.data(), wall_T, N * sizeof(double), hipMemcpyDeviceToHost));
    if (u0) HIP_TRY(hipMemcpy(hu.data(), u0, hu.size() * sizeof(double), hipMemcpyDeviceToHost));
    if (Ph0) HIP_TRY(hipMemcpy(hP.data(), Ph0, N * sizeof(double), hipMemcpyDeviceToHost));
    return lbfd_init(p, hm.data(), wall_T ? hw.data() : nullptr, hT.data(), hY.data(), u0 ? hu.data() : nullptr,
                     Ph0 ? hP.data() : nullptr, hip_stream, out);
}

int lbfd_step(lbfd_ctx *c, int64_t nsteps)
{
    if (!c || nsteps < 0) return fail(LBFD_EINVAL, "bad arguments");
    for (int64_t s = 0; s < nsteps; ++s) {
        KParams k = c->base;
        k.pop_in = c->pop[c->cur];
        k.pop_out = c->pop[1 - c->cur];
        k.sc_in = c->sc[c->cur];
        k.sc_out = c->sc[1 - c->cur];
        const bool check = c->p.check_every > 0 && (c->level % c->p.check_every) == 0;
        HIP_TRY(launch_step(c->Q, c->nsp, c->prec, check ? kModeStepDiag : kModeStep, k,
                            c->streams));
        if (check) HIP_TRY(launch_finalize(c->partials, c->nblocks, c->diag_dev, c->bad_dev, c->level, c->stream));
        c->cur ^= 1;
        c->level += 1;
    }
    return LBFD_OK;
}

int lbfd_sync(lbfd_ctx *c)
{
    if (!c) return fail(LBFD_EINVAL, "null context");
    HIP_TRY(hipStreamSynchronize(c->stream));
    long long bad = -1;
    HIP_TRY(hipMemcpy(&bad, c->bad_dev, sizeof(bad), hipMemcpyDeviceToHost));
    if (bad >= 0) return fail(LBFD_ENONFINITE, "non-finite values in the state at level %lld", bad);
    return LBFD_OK;
}

int64_t lbfd_level(const lbfd_ctx *c) { return c ? c->level : -1; }

// Evaluate the current level without advancing it: fields and diagnostics.
static int evaluate(lbfd_ctx *c)
{
    if (!c->fields) {
        if (hipMalloc((void **)&c->fields, (size_t)5 * c->N * sizeof(double)) != hipSuccess) {
            c->fields = nullptr;
            return fail(LBFD_ENOMEM, "hipMalloc of the field buffer failed");
        }
        c->base.fields = c->fields;
    }
    KParams k = c->base;
    k.pop_in = c->pop[c->cur];
    k.sc_in = c->sc[c->cur];
    // the next level's scalar buffer holds the chemistry launch's source
    // (it is overwritten by the next step)
    k.sc_out = c->sc[1 - c->cur];
    HIP_TRY(launch_step(c->Q, c->nsp, c->prec, kModeFields, k, c->streams));
    HIP_TRY(launch_finalize(c->partials, c->nblocks, c->diag_dev, nullptr, c->level, c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
    return LBFD_OK;
}

// Fields of the current level into host (dev = false) or device buffers.
static int read_fields(lbfd_ctx *c, double *rho, double *u, double *T, double *Y, double *Ph, bool dev)
{
    if (!c) return fail(LBFD_EINVAL, "null context");
    int rc = evaluate(c);
    if (rc) return rc;
    const long long N = c->N;
    const hipMemcpyKind kind = dev ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
    if (rho) HIP_TRY(hipMemcpyAsync(rho, c->fields, N * sizeof(double), kind, c->stream));
    if (u) HIP_TRY(hipMemcpyAsync(u, c->fields + N, (size_t)c->D * N * sizeof(double), kind, c->stream));
    if (Ph) HIP_TRY(hipMemcpyAsync(Ph, c->fields + 4 * N, N * sizeof(double), kind, c->stream));
    if (T || Y) {
        const size_t n = (size_t)(1 + c->nsp) * N;
        if (c->prec == LBFD_FP64) {
            if (T) HIP_TRY(hipMemcpyAsync(T, c->sc[c->cur], N * sizeof(double), kind, c->stream));
            if (Y)
                HIP_TRY(hipMemcpyAsync(Y, (double *)c->sc[c->cur] + N, (size_t)c->nsp * N * sizeof(double), kind,
                                       c->stream));
        } else if (dev) {
            // mixed storage: widened to double on the device
            if (T) HIP_TRY(launch_widen((const float *)c->sc[c->cur], T, (size_t)N, c->stream));
            if (Y) HIP_TRY(launch_widen((const float *)c->sc[c->cur] + N, Y, (size_t)c->nsp * N, c->stream));
        } else {
            std::vector<float> tmp(n);
            HIP_TRY(hipMemcpyAsync(tmp.data(), c->sc[c->cur], n * sizeof(float), hipMemcpyDeviceToHost, c->stream));
            HIP_TRY(hipStreamSynchronize(c->stream));
            if (T)
                for (long long i = 0; i < N; ++i) T[i] = tmp[i];
            if (Y)
                for (size_t i = 0; i < (size_t)c->nsp * N; ++i) Y[i] = tmp[N + i];
        }
    }
    HIP_TRY(hipStreamSynchronize(c->stream));
    return LBFD_OK;
}

int lbfd_read_fields(lbfd_ctx *c, double *rho, double *u, double *T, double *Y, double *Ph)
{
    return read_fields(c, rho, u, T, Y, Ph, false);
}

int lbfd_read_fields_dev(lbfd_ctx *c, double *rho, double *u, double *T, double *Y, double *Ph)
{
    return read_fields(c, rho, u, T, Y, Ph, true);
}

int lbfd_diagnostics(lbfd_ctx *c, lbfd_diag *d)
{
    if (!c || !d) return fail(LBFD_EINVAL, "null argument");
    int rc = evaluate(c);
    if (rc) return rc;
    double a[kNDiag];
    HIP_TRY(hipMemcpy(a, c->diag_dev, sizeof(a), hipMemcpyDeviceToHost));
    d->sum_g = a[kSumG];
    d->sum_xi = a[kSumXi];
    d->mom[0] = a[kMomX];
    d->mom[1] = a[kMomY];
    d->mom[2] = a[kMomZ];
    d->max_abs_sumY_minus_1 = a[kMaxY];
    d->nonfinite = (int64_t)a[kNonfinite];
    d->sum_theta = a[kTheta];
    d->hrr_idx = a[kHrrIdx] < 1e299 ? (int64_t)a[kHrrIdx] : -1;
    d->hrr_max = a[kHrrMax];
    d->wall_q = a[kWallQ];
    d->fuel_rate = a[kFuel];
    d->step = c->level;
    d->fuel_mass_rate = a[kFuelMass];
    const double fresh = c->base.rho_in * c->p.Y_in[0] * ((double)c->n_fluid / c->p.nx);
    d->consumption_speed = fresh > 0.0 ? a[kFuelMass] / fresh : 0.0;
    return LBFD_OK;
}

int lbfd_set_wall_links(lbfd_ctx *c, int64_t n, const int64_t *cell, const int32_t *dir, const double *q)
{
    if (!c || n < 0 || (n > 0 && (!cell || !dir || !q))) return fail(LBFD_EINVAL, "bad arguments");
    HIP_TRY(hipStreamSynchronize(c->stream));
    if (n == 0) {
        if (c->bq) (void)hipFree(c->bq);
        c->bq = nullptr;
        c->base.bq = nullptr;
        return LBFD_OK;
    }
    const long long nb = c->n_boundary, N = c->N;
    const int Q = c->Q;
    std::vector<int> slot(N, -1);  // cell -> position in the boundary list
    for (long long t = 0; t < nb; ++t) slot[c->boundary_host[t]] = (int)t;
    std::vector<float> h((size_t)Q * nb, std::numeric_limits<float>::quiet_NaN());
    const lbfd_params &p = c->p;
    for (int64_t k = 0; k < n; ++k) {
        const long long i = cell[k];
        const int d = dir[k];
        if (i < 0 || i >= N || d < 0 || d >= Q || !(q[k] > 0.0 && q[k] <= 1.0))
            return fail(LBFD_EINVAL, "wall link %lld out of range", (long long)k);
        if (c->mask_host[i] != LBFD_FLUID || slot[i] < 0)
            return fail(LBFD_EINVAL, "wall link %lld does not start at a boundary fluid cell", (long long)k);
        const int x = (int)(i % p.nx), y = (int)((i / p.nx) % p.ny), z = (int)(i / ((long long)p.nx * p.ny));
        const int cx = d % 3 - 1, cy = (d / 3) % 3 - 1, cz = Q == 9 ? 0 : d / 9 - 1;
        const HostNb nbr = host_classify(p, c->mask_host.data(), c->wall_T_host.data(), x + cx, y + cy, z + cz);
        if (nbr.kind != kIso && nbr.kind != kAdia)
            return fail(LBFD_EINVAL, "wall link %lld does not end at a wall", (long long)k);
        h[(size_t)(Q - 1 - d) * nb + slot[i]] = (float)q[k];  // stored by the entering direction
    }
    if (!c->bq && hipMalloc((void **)&c->bq, h.size() * sizeof(float)) != hipSuccess) {
        c->bq = nullptr;
        return fail(LBFD_ENOMEM, "hipMalloc of the wall-distance table failed");
    }
    HIP_TRY(hipMemcpy(c->bq, h.data(), h.size() * sizeof(float), hipMemcpyHostToDevice));
    c->base.bq = c->bq;
    return LBFD_OK;
}

static void clear_image_points(lbfd_ctx *c)
{
    void *ptrs[] = {c->bimg, c->img_rng, c->img_idx, c->img_w, c->img_val, c->sup_idx, c->sup_val};
    for (void *q : ptrs)
        if (q) (void)hipFree(q);
    c->sup_idx = nullptr;
    c->sup_val = nullptr;
    c->n_sup = 0;
    c->base.sup_idx = nullptr;
    c->base.sup_val = nullptr;
    c->base.n_sup = 0;
    c->bimg = nullptr;
    c->img_rng = nullptr;
    c->img_idx = nullptr;
    c->img_w = nullptr;
    c->img_val = nullptr;
    c->n_img = 0;
    c->base.bimg = nullptr;
    c->base.n_img = 0;
    c->base.img_rng = nullptr;
    c->base.img_idx = nullptr;
    c->base.img_w = nullptr;
    c->base.img_val = nullptr;
}

int lbfd_set_image_points(lbfd_ctx *c, int64_t n, const int64_t *cell, const int32_t *slot, const double *image)
{
    if (!c || n < 0 || (n > 0 && (!cell || !slot || !image))) return fail(LBFD_EINVAL, "bad arguments");
    HIP_TRY(hipStreamSynchronize(c->stream));
    if (n == 0) {
        clear_image_points(c);
        return LBFD_OK;
    }
    const lbfd_params &p = c->p;
    const long long nb = c->n_boundary, N = c->N;
    const int D = c->D;
    const uint8_t *mask = c->mask_host.data();
    const double *wT = c->wall_T_host.data();
    std::vector<int> pos(N, -1);  // cell -> position in the boundary list
    for (long long t = 0; t < nb; ++t) pos[c->boundary_host[t]] = (int)t;
    if (n > (int64_t)INT32_MAX) return fail(LBFD_EINVAL, "too many image points");
    // validation, in entry order (the first bad entry is the one reported)
    std::vector<int> which((size_t)12 * nb, -1);
    for (int64_t k = 0; k < n; ++k) {
        const long long i = cell[k];
        const int s = slot[k];
        const double *xi = image + 3 * k;
        if (i < 0 || i >= N || s < 0 || s >= 4 * D || !std::isfinite(xi[0]) || !std::isfinite(xi[1]) ||
            !std::isfinite(xi[2]))
            return fail(LBFD_EINVAL, "image point %lld out of range", (long long)k);
        if (mask[i] != LBFD_FLUID || pos[i] < 0)
            return fail(LBFD_EINVAL, "image point %lld does not belong to a boundary fluid cell", (long long)k);
        const size_t r = (size_t)s * nb + pos[i];
        if (c->bwk_host[r] != kIso && c->bwk_host[r] != kAdia)
            return fail(LBFD_EINVAL, "image point %lld: its stencil point is not a ghost node behind a wall",
                        (long long)k);
        if (which[r] >= 0) return fail(LBFD_EINVAL, "image point %lld repeats a ghost node", (long long)k);
        which[r] = (int)k;
    }
    // Shepard weights, on up to 16 host threads over contiguous ranges of
    // entries: every fluid node within four cells of the image point, weight
    // d^-2 normalised; a node at distance zero takes the whole weight
    struct Part {
        std::vector<int> nodes, count;
        std::vector<double> wts;
        int64_t bad = -1;  // first entry of the range without a fluid node
        bool oom = false;
    };
    const int nth = (int)std::max<int64_t>(1, std::min<int64_t>({16, (int64_t)std::thread::hardware_concurrency(),
                                                                 (n + 4095) / 4096}));
    std::vector<Part> parts(nth);
    auto work = [&](int w) {
        Part &pt = parts[w];
        const int64_t k0 = n * w / nth, k1 = n * (w + 1) / nth;
        try {
            pt.count.reserve(k1 - k0);
            for (int64_t k = k0; k < k1; ++k) {
                const double *xi = image + 3 * k;
                int lo[3] = {0, 0, 0}, hi[3] = {0, 0, 0};
                for (int d = 0; d < D; ++d) {
                    lo[d] = (int)std::ceil(xi[d] - 4.0);
                    hi[d] = (int)std::floor(xi[d] + 4.0);
                }
                const size_t begin = pt.nodes.size();
                double wsum = 0.0;
                bool exact = false;
                for (int z = lo[2]; z <= hi[2] && !exact; ++z)
                    for (int y = lo[1]; y <= hi[1] && !exact; ++y)
                        for (int x = lo[0]; x <= hi[0]; ++x) {
                            const double dx = x - xi[0], dy = y - xi[1], dz = D == 3 ? z - xi[2] : 0.0;
                            const double d2 = dx * dx + dy * dy + dz * dz;
                            if (d2 > 16.0) continue;
                            const HostNb h = host_classify(p, mask, wT, x, y, z);
                            if (h.kind != kFluid) continue;
                            if (d2 == 0.0) {
                                pt.nodes.resize(begin);
                                pt.wts.resize(begin);
                                pt.nodes.push_back((int)h.idx);
                                pt.wts.push_back(1.0);
                                exact = true;
                                break;
                            }
                            pt.nodes.push_back((int)h.idx);
                            pt.wts.push_back(1.0 / d2);
                            wsum += 1.0 / d2;
                        }
                if (pt.nodes.size() == begin && pt.bad < 0) pt.bad = k;
                if (!exact)
                    for (size_t e = begin; e < pt.nodes.size(); ++e) pt.wts[e] /= wsum;
                pt.count.push_back((int)(pt.nodes.size() - begin));
            }
        } catch (const std::bad_alloc &) {
            pt.oom = true;
        }
    };
    {
        std::vector<std::thread> pool;
        std::vector<int> here;  // ranges whose thread could not be started
        for (int w = 1; w < nth; ++w) {
            try {
                pool.emplace_back(work, w);
            } catch (...) {
                here.push_back(w);
            }
        }
        work(0);
        for (int w : here) work(w);
        for (std::thread &t : pool) t.join();
    }
    size_t total = 0;
    for (const Part &pt : parts)
        if (pt.oom) return fail(LBFD_ENOMEM, "host memory for the Shepard weights exhausted");
    for (const Part &pt : parts) {
        if (pt.bad >= 0)
            return fail(LBFD_EINVAL, "image point %lld has no fluid node within four cells", (long long)pt.bad);
        total += pt.nodes.size();
    }
    if (total > (size_t)INT32_MAX) return fail(LBFD_EINVAL, "too many Shepard nodes");
    std::vector<int2> range;
    std::vector<int> nodes;
    std::vector<double> wts;
    try {
        range.resize((size_t)n);
        nodes.reserve(total);
        wts.reserve(total);
    } catch (const std::bad_alloc &) {
        return fail(LBFD_ENOMEM, "host memory for the Shepard weights exhausted");
    }
    for (int w = 0; w < nth; ++w) {
        const int64_t k0 = n * w / nth;
        const size_t base = nodes.size();
        size_t off = 0;
        for (size_t q = 0; q < parts[w].count.size(); ++q) {
            range[k0 + q] = make_int2((int)(base + off), parts[w].count[q]);
            off += (size_t)parts[w].count[q];
        }
        nodes.insert(nodes.end(), parts[w].nodes.begin(), parts[w].nodes.end());
        wts.insert(wts.end(), parts[w].wts.begin(), parts[w].wts.end());
        std::vector<int>().swap(parts[w].nodes);  // release as the tables grow
        std::vector<double>().swap(parts[w].wts);
    }
    // the support: distinct nodes in cell order; list entries become
    // positions in it
    std::vector<int> sup;
    try {
        std::vector<int> at((size_t)N, -1);
        for (int v : nodes) at[v] = 0;
        for (long long i = 0; i < N; ++i)
            if (at[i] == 0) {
                at[i] = (int)sup.size();
                sup.push_back((int)i);
            }
        for (int &v : nodes) v = at[v];
    } catch (const std::bad_alloc &) {
        return fail(LBFD_ENOMEM, "host memory for the Shepard support exhausted");
    }
    // everything checked: the new set replaces the previous one
    clear_image_points(c);
    if (hipMalloc((void **)&c->sup_idx, sup.size() * sizeof(int)) != hipSuccess ||
        hipMalloc((void **)&c->sup_val, (size_t)(2 + c->nsp) * sup.size() * sizeof(double)) != hipSuccess ||
        hipMalloc((void **)&c->bimg, which.size() * sizeof(int)) != hipSuccess ||
        hipMalloc((void **)&c->img_rng, range.size() * sizeof(int2)) != hipSuccess ||
        hipMalloc((void **)&c->img_idx, nodes.size() * sizeof(int)) != hipSuccess ||
        hipMalloc((void **)&c->img_w, wts.size() * sizeof(double)) != hipSuccess ||
        hipMalloc((void **)&c->img_val, (size_t)(2 + c->nsp) * n * sizeof(double)) != hipSuccess) {
        clear_image_points(c);
        return fail(LBFD_ENOMEM, "hipMalloc of the image-point tables failed");
    }
    hipError_t e = hipMemcpy(c->bimg, which.data(), which.size() * sizeof(int), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(c->img_rng, range.data(), range.size() * sizeof(int2), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(c->img_idx, nodes.data(), nodes.size() * sizeof(int), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(c->img_w, wts.data(), wts.size() * sizeof(double), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(c->sup_idx, sup.data(), sup.size() * sizeof(int), hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        clear_image_points(c);
        return fail(LBFD_EDEVICE, "upload of the image-point tables failed: %s", hipGetErrorString(e));
    }
    c->n_sup = (long long)sup.size();
    c->base.n_sup = c->n_sup;
    c->base.sup_idx = c->sup_idx;
    c->base.sup_val = c->sup_val;
    // lanes per row: about two nodes per lane on average
    const double mean = (double)nodes.size() / (double)n;
    c->img_lpp = mean <= 32.0 ? 16 : mean <= 64.0 ? 32 : 64;
    c->n_img = n;
    c->base.bimg = c->bimg;
    c->base.n_img = n;
    c->base.img_lpp = c->img_lpp;
    c->base.img_rng = c->img_rng;
    c->base.img_idx = c->img_idx;
    c->base.img_w = c->img_w;
    c->base.img_val = c->img_val;
    return LBFD_OK;
}

int lbfd_set_inflow(lbfd_ctx *c, int face, const double *u)
{
    if (!c) return fail(LBFD_EINVAL, "null context");
    if (face != 0 && face != 1) return fail(LBFD_EINVAL, "inlet profiles are set on x faces (0 or 1)");
    if (c->p.face[face] != LBFD_FACE_INFLOW) return fail(LBFD_EINVAL, "face %d is not an INFLOW face", face);
    const size_t nf = (size_t)c->p.ny * c->p.nz;
    for (size_t i = 0; u && i < 3 * nf; ++i)
        if (!std::isfinite(u[i])) return fail(LBFD_EINVAL, "non-finite inlet velocity");
    HIP_TRY(hipStreamSynchronize(c->stream));
    double *dst = c->inflow_host.data() + 3 * nf * face;
    std::vector<double> du(3 * nf);
    for (int d = 0; d < 3; ++d)
        for (size_t i = 0; i < nf; ++i) {
            const double v = u ? u[d * nf + i] : c->p.u_in[d];
            du[d * nf + i] = dst[d * nf + i] - v;
            dst[d * nf + i] = v;
        }
    // the current level keeps its entering populations; the new profile
    // applies from the next streaming on
    HIP_TRY(hipMemcpy(c->inflow_du, du.data(), 3 * nf * sizeof(double), hipMemcpyHostToDevice));
    KParams k = c->base;
    k.pop_in = c->pop[c->cur];
    k.pop_out = c->pop[c->cur];
    HIP_TRY(launch_inflow_shift(c->Q, c->prec, k, face, c->inflow_du, c->stream));
    HIP_TRY(hipMemcpyAsync(c->inflow_u + 3 * nf * face, dst, 3 * nf * sizeof(double), hipMemcpyHostToDevice,
                           c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
    return LBFD_OK;
}

int lbfd_hold_flame(lbfd_ctx *c, int64_t nsteps, int every, double x_target, double gain, double *u_mean,
                    double *x_flame)
{
    if (!c || nsteps < 0 || every < 1 || !(gain >= 0.0)) return fail(LBFD_EINVAL, "bad arguments");
    const int face = c->p.face[0] == LBFD_FACE_INFLOW ? 0 : c->p.face[1] == LBFD_FACE_INFLOW ? 1 : -1;
    if (face < 0) return fail(LBFD_EINVAL, "flame holding needs an INFLOW x face");
    const int nx = c->p.nx, ny = c->p.ny, nz = c->p.nz;
    const size_t nf = (size_t)ny * nz;
    // shape of the current profile, scaled to a unit mean of the inward
    // normal velocity over the fluid cells next to the face (a uniform
    // inward unit velocity when that mean is zero)
    const int xc = face == 0 ? 0 : nx - 1;
    const double sign = face == 0 ? 1.0 : -1.0;  // inward normal along x
    std::vector<double> shape(c->inflow_host.begin() + 3 * nf * face, c->inflow_host.begin() + 3 * nf * (face + 1));
    double mean = 0.0;
    long long nface = 0;
    for (int z = 0; z < nz; ++z)
        for (int y = 0; y < ny; ++y)
            if (c->mask_host[((size_t)z * ny + y) * nx + xc] == LBFD_FLUID) {
                mean += sign * shape[(size_t)z * ny + y];
                ++nface;
            }
    if (nface == 0) return fail(LBFD_EINVAL, "no fluid cell next to the inflow face");
    mean /= (double)nface;
    if (std::fabs(mean) > 0.0) {
        for (double &v : shape) v /= mean;
    } else {
        std::fill(shape.begin(), shape.end(), 0.0);
        for (size_t i = 0; i < nf; ++i) shape[i] = sign;
    }
    std::vector<double> prof(3 * nf);
    const int64_t ncycle = nsteps / every;
    for (int64_t k = 0; k < ncycle; ++k) {
        int rc = lbfd_step(c, every);
        if (rc) return rc;
        lbfd_diag d;
        rc = lbfd_diagnostics(c, &d);
        if (rc) return rc;
        if (d.nonfinite > 0) return fail(LBFD_ENONFINITE, "non-finite state at level %lld", (long long)c->level);
        const double xf = nx - d.sum_theta / ((double)c->n_fluid / nx);
        double U = d.consumption_speed - gain * (xf - x_target);
        if (U < 0.0) U = 0.0;
        for (size_t i = 0; i < 3 * nf; ++i) prof[i] = U * shape[i];
        rc = lbfd_set_inflow(c, face, prof.data());
        if (rc) return rc;
        if (u_mean) u_mean[k] = U;
        if (x_flame) x_flame[k] = xf;
    }
    return LBFD_OK;
}

int lbfd_set_wall_temperature(lbfd_ctx *c, const double *wall_T)
{
    if (!c || !wall_T) return fail(LBFD_EINVAL, "null argument");
    HIP_TRY(hipStreamSynchronize(c->stream));
    c->wall_T_host.assign(wall_T, wall_T + c->N);
    HIP_TRY(hipMemcpy(c->wall_T, wall_T, c->N * sizeof(double), hipMemcpyHostToDevice));
    return build_descriptors(c);
}

static void state_sizes(const lbfd_ctx *c, size_t *pop, size_t *sc, size_t *outl)
{
    *pop = (size_t)c->Q * c->N * pop_elem_size(c->prec);
    *sc = (size_t)(1 + c->nsp) * c->N * sc_elem_size(c->prec);
    *outl = c->outlet_n * sizeof(double);
}

int lbfd_state_size(const lbfd_ctx *c, size_t *bytes)
{
    if (!c || !bytes) return fail(LBFD_EINVAL, "null argument");
    size_t a, b, o;
    state_sizes(c, &a, &b, &o);
    *bytes = sizeof(StateHeader) + a + b + o;
    return LBFD_OK;
}

int lbfd_save_state(lbfd_ctx *c, void *blob, size_t bytes)
{
    size_t need;
    int rc = lbfd_state_size(c, &need);
    if (rc) return rc;
    if (!blob || bytes < need) return fail(LBFD_EINVAL, "state buffer too small (%zu < %zu)", bytes, need);
    size_t a, b, o;
    state_sizes(c, &a, &b, &o);
    StateHeader h = {kMagic, c->Q, c->nsp, c->prec, c->p.nx, c->p.ny, c->p.nz, c->level, a, b, o};
    HIP_TRY(hipStreamSynchronize(c->stream));
    char *q = (char *)blob;
    memcpy(q, &h, sizeof(h));
    HIP_TRY(hipMemcpy(q + sizeof(h), c->pop[c->cur], a, hipMemcpyDeviceToHost));
    HIP_TRY(hipMemcpy(q + sizeof(h) + a, c->sc[c->cur], b, hipMemcpyDeviceToHost));
    HIP_TRY(hipMemcpy(q + sizeof(h) + a + b, c->outlet, o, hipMemcpyDeviceToHost));
    return LBFD_OK;
}

int lbfd_load_state(lbfd_ctx *c, const void *blob, size_t bytes)
{
    size_t need;
    int rc = lbfd_state_size(c, &need);
    if (rc) return rc;
    if (!blob || bytes < need) return fail(LBFD_ESTATE, "state blob too small");
    StateHeader h;
    memcpy(&h, blob, sizeof(h));
    size_t a, b, o;
    state_sizes(c, &a, &b, &o);
    if (h.magic != kMagic || h.lattice != c->Q || h.n_species != c->nsp || h.precision != c->prec ||
        h.nx != c->p.nx || h.ny != c->p.ny || h.nz != c->p.nz || h.pop_bytes != a || h.sc_bytes != b ||
        h.outlet_bytes != o)
        return fail(LBFD_ESTATE, "state blob does not match this context");
    HIP_TRY(hipStreamSynchronize(c->stream));
    const char *q = (const char *)blob;
    HIP_TRY(hipMemcpy(c->pop[c->cur], q + sizeof(h), a, hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(c->sc[c->cur], q + sizeof(h) + a, b, hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(c->outlet, q + sizeof(h) + a + b, o, hipMemcpyHostToDevice));
    c->level = h.level;
    return LBFD_OK;
}

int lbfd_time_steps(lbfd_ctx *c, int64_t nsteps, double *ms)
{
    if (!c || !ms || nsteps < 0) return fail(LBFD_EINVAL, "bad arguments");
    hipEvent_t a, b;
    HIP_TRY(hipEventCreate(&a));
    HIP_TRY(hipEventCreate(&b));
    HIP_TRY(hipEventRecord(a, c->stream));
    int rc = lbfd_step(c, nsteps);
    HIP_TRY(hipEventRecord(b, c->stream));
    HIP_TRY(hipEventSynchronize(b));
    float t = 0.0f;
    HIP_TRY(hipEventElapsedTime(&t, a, b));
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    *ms = t;
    return rc;
}

int lbfd_time_kernels(lbfd_ctx *c, int64_t nsteps, double *ms_interior, double *ms_boundary,
                      double *ms_chemistry)
{
    if (!c || !ms_interior || !ms_boundary || nsteps < 0) return fail(LBFD_EINVAL, "bad arguments");
    hipEvent_t ev[4];
    for (int i = 0; i < 4; ++i) HIP_TRY(hipEventCreate(&ev[i]));
    double ti = 0.0, tb = 0.0, tc = 0.0;
    for (int64_t s = 0; s < nsteps; ++s) {
        KParams k = c->base;
        k.pop_in = c->pop[c->cur];
        k.pop_out = c->pop[1 - c->cur];
        k.sc_in = c->sc[c->cur];
        k.sc_out = c->sc[1 - c->cur];
        Streams st = c->streams;
        // chemistry launch (if any) first: the step reads its source
        const int parts[3] = {3, 1, 2};
        HIP_TRY(hipEventRecord(ev[0], c->stream));
        for (int i = 0; i < 3; ++i) {
            st.part = parts[i];
            HIP_TRY(launch_step(c->Q, c->nsp, c->prec, kModeStep, k, st));
            HIP_TRY(hipEventRecord(ev[i + 1], c->stream));
        }
        HIP_TRY(hipEventSynchronize(ev[3]));
        float t[3] = {0.0f, 0.0f, 0.0f};
        for (int i = 0; i < 3; ++i) HIP_TRY(hipEventElapsedTime(&t[i], ev[i], ev[i + 1]));
        tc += t[0];
        ti += t[1];
        tb += t[2];
        c->cur ^= 1;
        c->level += 1;
    }
    for (int i = 0; i < 4; ++i) (void)hipEventDestroy(ev[i]);
    *ms_interior = ti;
    *ms_boundary = tb;
    if (ms_chemistry) *ms_chemistry = tc;
    return LBFD_OK;
}

int lbfd_chem_kernel(const lbfd_ctx *c, char *msg, size_t len)
{
    if (!c) return fail(LBFD_EINVAL, "null context");
    if (msg && len) snprintf(msg, len, "%s", c->chem_msg);
    return c->base.chem_jit != nullptr ? 1 : 0;
}

int lbfd_set_reaction(lbfd_ctx *c, int j, double A, double b, double Ta)
{
    if (!c || j < 0 || j >= c->p.n_reactions) return fail(LBFD_EINVAL, "bad reaction index");
    HIP_TRY(hipStreamSynchronize(c->stream));
    c->rx[j].A = A;
    c->rx[j].b = b;
    c->rx[j].Ta = Ta;
    return upload_reactions(c);
}

namespace {
// device buffers owned by one lbfd_adjoint call
struct AdjBuffers {
    std::vector<void *> ptrs;
    ~AdjBuffers()
    {
        for (void *q : ptrs) (void)hipFree(q);
    }
    void *get(size_t bytes)
    {
        void *q = nullptr;
        if (hipMalloc(&q, bytes ? bytes : 1) != hipSuccess) return nullptr;
        ptrs.push_back(q);
        return q;
    }
};
}  // namespace

// The selected objective's share of level offset t: accumulate coefficients
// (*acc += a diag[slot] + b) and the adjoint weight.
struct ObjTerm {
    bool on;
    int slot;
    double a, b, w;
};

static ObjTerm objective_term(const lbfd_ctx *c, int64_t t)
{
    ObjTerm o{t >= c->obj_t0 && t < c->obj_t1, kWallQ, 1.0, 0.0, 1.0};
    if (c->obj_kind == LBFD_OBJ_FLAME_POSITION) {
        const double nx = c->p.nx, per_col = (double)c->n_fluid / nx;
        o.slot = kTheta;
        o.a = -1.0 / per_col;
        o.b = nx;
        o.w = -1.0 / (per_col * (c->p.T_b - c->p.T_u));
    }
    if (!o.on) o.w = 0.0;
    return o;
}

int lbfd_set_objective(lbfd_ctx *c, int kind, int64_t t_begin, int64_t t_end)
{
    if (!c) return fail(LBFD_EINVAL, "null context");
    if (kind != LBFD_OBJ_WALL_HEAT_FLUX && kind != LBFD_OBJ_FLAME_POSITION)
        return fail(LBFD_EINVAL, "unknown objective kind %d", kind);
    if (t_begin < 0 || t_end < t_begin) return fail(LBFD_EINVAL, "bad objective window [%lld, %lld)",
                                                    (long long)t_begin, (long long)t_end);
    if (kind == LBFD_OBJ_FLAME_POSITION && !(c->p.T_b > c->p.T_u))
        return fail(LBFD_EINVAL, "the flame position needs T_b > T_u");
    c->obj_kind = kind;
    c->obj_t0 = t_begin;
    c->obj_t1 = t_end;
    return LBFD_OK;
}

int lbfd_objective(lbfd_ctx *c, int64_t nsteps, double *J)
{
    if (!c || !J || nsteps < 0) return fail(LBFD_EINVAL, "bad arguments");
    double *Jd = nullptr;
    if (hipMalloc((void **)&Jd, sizeof(double)) != hipSuccess) return fail(LBFD_ENOMEM, "hipMalloc failed");
    hipError_t e = hipMemsetAsync(Jd, 0, sizeof(double), c->stream);
    for (int64_t n = 0; n < nsteps && e == hipSuccess; ++n) {
        KParams k = c->base;
        k.pop_in = c->pop[c->cur];
        k.pop_out = c->pop[1 - c->cur];
        k.sc_in = c->sc[c->cur];
        k.sc_out = c->sc[1 - c->cur];
        const ObjTerm o = objective_term(c, n);
        e = launch_step(c->Q, c->nsp, c->prec, o.on ? kModeStepDiag : kModeStep, k, c->streams);
        if (e == hipSuccess && o.on)
            e = launch_finalize(c->partials, c->nblocks, c->diag_dev, c->bad_dev, c->level, c->stream, Jd, o.slot,
                                o.a, o.b);
        c->cur ^= 1;
        c->level += 1;
    }
    // the context stream may be a non-blocking one: copy on it and wait
    if (e == hipSuccess) e = hipMemcpyAsync(J, Jd, sizeof(double), hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    (void)hipFree(Jd);
    if (e != hipSuccess) return fail(LBFD_EDEVICE, "objective: %s", hipGetErrorString(e));
    return LBFD_OK;
}

int lbfd_objective_static(lbfd_ctx *c, int64_t nsteps, double *J)
{
    if (!c || !J || nsteps < 0) return fail(LBFD_EINVAL, "bad arguments");
    const size_t need = kScratchPartials + (size_t)c->nblocks * kNDiag * sizeof(double);
    if (need > kScratchBytes)
        return fail(LBFD_EINVAL, "lbfd_objective_static: this box needs %zu bytes of scratch, the static array "
                    "holds %zu (use lbfd_objective)", need, kScratchBytes);
    double *acc = (double *)(c->scratch + kScratchAcc);
    double *diag = (double *)(c->scratch + kScratchDiag);
    double *partials = (double *)(c->scratch + kScratchPartials);
    hipError_t e = launch_fill(acc, 1, 0.0, c->stream);
    for (int64_t n = 0; n < nsteps && e == hipSuccess; ++n) {
        KParams k = c->base;
        k.pop_in = c->pop[c->cur];
        k.pop_out = c->pop[1 - c->cur];
        k.sc_in = c->sc[c->cur];
        k.sc_out = c->sc[1 - c->cur];
        k.partials = partials;
        const ObjTerm o = objective_term(c, n);
        e = launch_step(c->Q, c->nsp, c->prec, o.on ? kModeStepDiag : kModeStep, k, c->streams);
        if (e == hipSuccess && o.on)
            e = launch_finalize(partials, c->nblocks, diag, c->bad_dev, c->level, c->stream, acc, o.slot, o.a, o.b);
        c->cur ^= 1;
        c->level += 1;
    }
    if (e == hipSuccess) e = hipMemcpyAsync(J, acc, sizeof(double), hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return fail(LBFD_EDEVICE, "objective: %s", hipGetErrorString(e));
    return LBFD_OK;
}

// The contexts the adjoint and the tangent differentiate; LBFD_OK or the
// reason (LBFD_EINVAL).
static int derivative_check(const lbfd_ctx *c)
{
    if (c->prec != LBFD_FP64) return fail(LBFD_EINVAL, "the adjoint needs FP64 precision");
    if (c->p.collision != LBFD_CENTRAL_MOMENTS)
        return fail(LBFD_EINVAL, "the adjoint differentiates the central-moment collision only");
    if (c->p.transport != LBFD_UNITY_LEWIS)
        return fail(LBFD_EINVAL, "the adjoint differentiates the unity-Lewis transport only");
    if (c->bq || c->bimg)
        return fail(LBFD_EINVAL, "the adjoint differentiates half-way bounce-back and axis-mirror ghosts only");
    if (!adjoint_supported(c->Q, c->nsp))
        return fail(LBFD_EINVAL, "no adjoint kernel for lattice %d with %d species", c->Q, c->nsp);
    for (int f = 0; f < 6; ++f)
        if (c->p.face[f] == LBFD_FACE_OUTFLOW) return fail(LBFD_EINVAL, "the adjoint does not support OUTFLOW faces");
    return LBFD_OK;
}

// dq/dT of one fluid cell for the flame position (its objective is linear in
// the cells' T), 1 for the wall heat flux.
static double objective_cell_weight(const lbfd_ctx *c)
{
    if (c->obj_kind != LBFD_OBJ_FLAME_POSITION) return 1.0;
    const double per_col = (double)c->n_fluid / c->p.nx;
    return -1.0 / (per_col * (c->p.T_b - c->p.T_u));
}

int lbfd_step_tangent(lbfd_ctx *c, const double *dpop, const double *dsc, const double *dwallT, const double *dA,
                      const double *dTa, double *dpop_out, double *dsc_out, double *dq)
{
    if (!c || !dpop || !dsc || !dpop_out || !dsc_out || !dq) return fail(LBFD_EINVAL, "null argument");
    const int rc0 = derivative_check(c);
    if (rc0 != LBFD_OK) return rc0;
    HIP_TRY(hipStreamSynchronize(c->stream));
    const long long N = c->N;
    const int nrx = c->p.n_reactions;
    const size_t pop_b = (size_t)c->Q * N * sizeof(double), sc_b = (size_t)(1 + c->nsp) * N * sizeof(double);
    AdjBuffers mem;
    double *d_in = (double *)mem.get(pop_b), *s_in = (double *)mem.get(sc_b);
    double *d_out = (double *)mem.get(pop_b), *s_out = (double *)mem.get(sc_b);
    double *w_in = (double *)mem.get(N * sizeof(double));
    double *p_in = (double *)mem.get(2 * LBFD_MAX_REACTIONS * sizeof(double)), *q = (double *)mem.get(sizeof(double));
    if (!d_in || !s_in || !d_out || !s_out || !w_in || !p_in || !q)
        return fail(LBFD_ENOMEM, "tangent: device allocation failed");
    std::vector<double> hp(2 * LBFD_MAX_REACTIONS, 0.0);
    for (int j = 0; j < nrx; ++j) {
        hp[2 * j] = dA ? dA[j] : 0.0;
        hp[2 * j + 1] = dTa ? dTa[j] : 0.0;
    }
    HIP_TRY(hipMemcpy(d_in, dpop, pop_b, hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(s_in, dsc, sc_b, hipMemcpyHostToDevice));
    if (dwallT)
        HIP_TRY(hipMemcpy(w_in, dwallT, N * sizeof(double), hipMemcpyHostToDevice));
    else
        HIP_TRY(hipMemset(w_in, 0, N * sizeof(double)));
    HIP_TRY(hipMemcpy(p_in, hp.data(), hp.size() * sizeof(double), hipMemcpyHostToDevice));
    HIP_TRY(hipMemset(d_out, 0, pop_b));
    HIP_TRY(hipMemset(s_out, 0, sc_b));
    HIP_TRY(hipMemset(q, 0, sizeof(double)));
    KParams k = c->base;
    k.pop_in = c->pop[c->cur];
    k.sc_in = c->sc[c->cur];
    HIP_TRY(launch_tangent(c->Q, c->nsp, k, d_in, s_in, w_in, p_in, d_out, s_out, q, c->obj_kind,
                           objective_cell_weight(c), c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
    HIP_TRY(hipMemcpy(dpop_out, d_out, pop_b, hipMemcpyDeviceToHost));
    HIP_TRY(hipMemcpy(dsc_out, s_out, sc_b, hipMemcpyDeviceToHost));
    HIP_TRY(hipMemcpy(dq, q, sizeof(double), hipMemcpyDeviceToHost));
    return LBFD_OK;
}

int lbfd_step_adjoint(lbfd_ctx *c, const double *lam_pop, const double *lam_sc, double wq, double *lam_pop_in,
                      double *lam_sc_in, double *dJ_dwallT, double *dJ_dA, double *dJ_dTa)
{
    if (!c || !lam_pop || !lam_sc || !lam_pop_in || !lam_sc_in) return fail(LBFD_EINVAL, "null argument");
    const int rc0 = derivative_check(c);
    if (rc0 != LBFD_OK) return rc0;
    HIP_TRY(hipStreamSynchronize(c->stream));
    const long long N = c->N;
    const int nrx = c->p.n_reactions;
    const size_t pop_b = (size_t)c->Q * N * sizeof(double), sc_b = (size_t)(1 + c->nsp) * N * sizeof(double);
    AdjBuffers mem;
    double *l_next = (double *)mem.get(pop_b), *s_next = (double *)mem.get(sc_b);
    double *l_out = (double *)mem.get(pop_b), *s_out = (double *)mem.get(sc_b);
    double *dW = (double *)mem.get(N * sizeof(double));
    double *dP = (double *)mem.get(2 * LBFD_MAX_REACTIONS * sizeof(double));
    double *mid = (double *)mem.get((size_t)adjoint_mid_fields(c->Q, c->nsp) * N * sizeof(double));
    if (!l_next || !s_next || !l_out || !s_out || !dW || !dP || !mid)
        return fail(LBFD_ENOMEM, "adjoint step: device allocation failed");
    HIP_TRY(hipMemcpy(l_next, lam_pop, pop_b, hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(s_next, lam_sc, sc_b, hipMemcpyHostToDevice));
    HIP_TRY(hipMemset(l_out, 0, pop_b));
    HIP_TRY(hipMemset(s_out, 0, sc_b));
    HIP_TRY(hipMemset(dW, 0, N * sizeof(double)));
    HIP_TRY(hipMemset(dP, 0, 2 * LBFD_MAX_REACTIONS * sizeof(double)));
    KParams k = c->base;
    k.pop_in = c->pop[c->cur];
    k.sc_in = c->sc[c->cur];
    HIP_TRY(launch_adjoint(c->Q, c->nsp, k, l_next, s_next, l_out, s_out, dW, dP, mid, c->obj_kind,
                           wq * objective_cell_weight(c), c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
    HIP_TRY(hipMemcpy(lam_pop_in, l_out, pop_b, hipMemcpyDeviceToHost));
    HIP_TRY(hipMemcpy(lam_sc_in, s_out, sc_b, hipMemcpyDeviceToHost));
    if (dJ_dwallT) HIP_TRY(hipMemcpy(dJ_dwallT, dW, N * sizeof(double), hipMemcpyDeviceToHost));
    double hP[2 * LBFD_MAX_REACTIONS];
    HIP_TRY(hipMemcpy(hP, dP, sizeof(hP), hipMemcpyDeviceToHost));
    for (int j = 0; j < nrx; ++j) {
        if (dJ_dA) dJ_dA[j] = hP[2 * j];
        if (dJ_dTa) dJ_dTa[j] = hP[2 * j + 1];
    }
    return LBFD_OK;
}

static int adjoint_impl(lbfd_ctx *c, int64_t nsteps, int K, double *J, double *dJ_dwallT, double *dJ_dA,
                        double *dJ_dTa, bool wall_dev)
{
    if (!c || nsteps < 1 || K < 1) return fail(LBFD_EINVAL, "bad arguments");
    const int rc0 = derivative_check(c);
    if (rc0 != LBFD_OK) return rc0;
    HIP_TRY(hipStreamSynchronize(c->stream));
    const long long N = c->N;
    const int Q = c->Q, ns = c->nsp, nrx = c->p.n_reactions;
    const size_t pop_b = (size_t)Q * N * sizeof(double), sc_b = (size_t)(1 + ns) * N * sizeof(double);
    const int64_t nseg = (nsteps + K - 1) / K;
    const int kseg = (int)(nsteps < K ? nsteps : K);
    AdjBuffers mem;
    char *ckpt = (char *)mem.get((size_t)nseg * (pop_b + sc_b));
    char *segs = (char *)mem.get((size_t)kseg * (pop_b + sc_b));
    double *lam[2], *lsc[2];
    for (int b = 0; b < 2; ++b) {
        lam[b] = (double *)mem.get(pop_b);
        lsc[b] = (double *)mem.get(sc_b);
    }
    double *dW = (double *)mem.get(N * sizeof(double));
    double *dP = (double *)mem.get(2 * LBFD_MAX_REACTIONS * sizeof(double));
    double *Jd = (double *)mem.get(sizeof(double));
    double *mid = (double *)mem.get((size_t)adjoint_mid_fields(Q, ns) * N * sizeof(double));
    if (!ckpt || !segs || !lam[0] || !lam[1] || !lsc[0] || !lsc[1] || !dW || !dP || !Jd || !mid)
        return fail(LBFD_ENOMEM, "adjoint: device allocation failed");
    auto ck_pop = [&](int64_t s) { return ckpt + (size_t)s * (pop_b + sc_b); };
    auto ck_sc = [&](int64_t s) { return ckpt + (size_t)s * (pop_b + sc_b) + pop_b; };
    auto sg_pop = [&](int64_t s) { return segs + (size_t)s * (pop_b + sc_b); };
    auto sg_sc = [&](int64_t s) { return segs + (size_t)s * (pop_b + sc_b) + pop_b; };

    // forward pass: checkpoints and the objective
    HIP_TRY(hipMemsetAsync(Jd, 0, sizeof(double), c->stream));
    for (int64_t n = 0; n < nsteps; ++n) {
        if (n % K == 0) {
            HIP_TRY(hipMemcpyAsync(ck_pop(n / K), c->pop[c->cur], pop_b, hipMemcpyDeviceToDevice, c->stream));
            HIP_TRY(hipMemcpyAsync(ck_sc(n / K), c->sc[c->cur], sc_b, hipMemcpyDeviceToDevice, c->stream));
        }
        KParams k = c->base;
        k.pop_in = c->pop[c->cur];
        k.pop_out = c->pop[1 - c->cur];
        k.sc_in = c->sc[c->cur];
        k.sc_out = c->sc[1 - c->cur];
        const ObjTerm o = objective_term(c, n);
        HIP_TRY(launch_step(c->Q, c->nsp, c->prec, o.on ? kModeStepDiag : kModeStep, k, c->streams));
        if (o.on) {
            HIP_TRY(launch_finalize(c->partials, c->nblocks, c->diag_dev, c->bad_dev, c->level, c->stream, Jd, o.slot,
                                    o.a, o.b));
        }
        c->cur ^= 1;
        c->level += 1;
    }

    // backward sweep over segments, each recomputed from its checkpoint
    // Every backward step stores the adjoints of every fluid cell's
    // populations and scalars; entries of solid cells are never written and
    // keep the zeros of this clear.
    for (int b = 0; b < 2; ++b) {
        HIP_TRY(hipMemsetAsync(lam[b], 0, pop_b, c->stream));
        HIP_TRY(hipMemsetAsync(lsc[b], 0, sc_b, c->stream));
    }
    HIP_TRY(hipMemsetAsync(dW, 0, N * sizeof(double), c->stream));
    HIP_TRY(hipMemsetAsync(dP, 0, 2 * LBFD_MAX_REACTIONS * sizeof(double), c->stream));
    int nxt = 0;  // lam[nxt], lsc[nxt]: adjoint of level n+1
    for (int64_t seg = nseg - 1; seg >= 0; --seg) {
        const int64_t n0 = seg * K, n1 = (n0 + K < nsteps) ? n0 + K : nsteps;
        HIP_TRY(hipMemcpyAsync(sg_pop(0), ck_pop(seg), pop_b, hipMemcpyDeviceToDevice, c->stream));
        HIP_TRY(hipMemcpyAsync(sg_sc(0), ck_sc(seg), sc_b, hipMemcpyDeviceToDevice, c->stream));
        for (int64_t n = n0; n < n1 - 1; ++n) {
            KParams k = c->base;
            k.pop_in = sg_pop(n - n0);
            k.pop_out = sg_pop(n - n0 + 1);
            k.sc_in = sg_sc(n - n0);
            k.sc_out = sg_sc(n - n0 + 1);
            HIP_TRY(launch_step(c->Q, c->nsp, c->prec, kModeStep, k, c->streams));
        }
        for (int64_t n = n1 - 1; n >= n0; --n) {
            const int cu = 1 - nxt;
            KParams k = c->base;
            k.pop_in = sg_pop(n - n0);
            k.sc_in = sg_sc(n - n0);
            const ObjTerm o = objective_term(c, n);
            HIP_TRY(launch_adjoint(c->Q, c->nsp, k, lam[nxt], lsc[nxt], lam[cu], lsc[cu], dW, dP, mid, c->obj_kind,
                                   o.w, c->stream));
            nxt = cu;
        }
    }
    HIP_TRY(hipStreamSynchronize(c->stream));
    double hP[2 * LBFD_MAX_REACTIONS];
    HIP_TRY(hipMemcpy(hP, dP, sizeof(hP), hipMemcpyDeviceToHost));
    if (J) HIP_TRY(hipMemcpy(J, Jd, sizeof(double), hipMemcpyDeviceToHost));
    if (dJ_dwallT)
        HIP_TRY(hipMemcpy(dJ_dwallT, dW, N * sizeof(double), wall_dev ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost));
    for (int j = 0; j < nrx; ++j) {
        if (dJ_dA) dJ_dA[j] = hP[2 * j];
        if (dJ_dTa) dJ_dTa[j] = hP[2 * j + 1];
    }
    return LBFD_OK;
}

int lbfd_adjoint(lbfd_ctx *c, int64_t nsteps, int K, double *J, double *dJ_dwallT, double *dJ_dA, double *dJ_dTa)
{
    return adjoint_impl(c, nsteps, K, J, dJ_dwallT, dJ_dA, dJ_dTa, false);
}

int lbfd_adjoint_dev(lbfd_ctx *c, int64_t nsteps, int K, double *J, double *dJ_dwallT, double *dJ_dA,
                     double *dJ_dTa)
{
    return adjoint_impl(c, nsteps, K, J, dJ_dwallT, dJ_dA, dJ_dTa, true);
}

int lbfd_cell_counts(const lbfd_ctx *c, int64_t *n_fluid, int64_t *n_boundary)
{
    if (!c || !n_fluid || !n_boundary) return fail(LBFD_EINVAL, "null argument");
    *n_fluid = c->n_fluid;
    *n_boundary = c->n_boundary;
    return LBFD_OK;
}

int lbfd_step_launches(const lbfd_ctx *c)
{
    if (!c) return fail(LBFD_EINVAL, "null context");
    return step_launches(c->Q, c->nsp, c->base);
}

void lbfd_destroy(lbfd_ctx *c)
{
    if (!c) return;
    (void)hipStreamSynchronize(c->stream);
    free_ctx(c);
}

const char *lbfd_strerror(int code)
{
    switch (code) {
    case LBFD_OK: return "ok";
    case LBFD_EINVAL: return "invalid argument";
    case LBFD_ENOMEM: return "out of memory";
    case LBFD_EDEVICE: return "HIP runtime error";
    case LBFD_ENONFINITE: return "non-finite state";
    case LBFD_ESTATE: return "state blob mismatch";
    default: return "unknown error";
    }
}

const char *lbfd_last_error(void) { return g_err; }

}  // extern "C"
