// lbfd_chemjit.hip -- the chemistry launch specialised to one mechanism's
// structure, generated as HIP source at set-up and compiled at run time
// (hiprtc) for gfx950.
//
// The generic chemistry kernel (chem_kernel) reads every reactant through a
// uniform index into the register file (two moves per factor) and adds
// nu_k r into all N_sp species of every reaction, zero coefficients
// included.  The specialised kernel has each reaction's reactant species
// and the species with a nonzero mass coefficient written into its text, so
// a factor is one multiply and a zero coefficient costs nothing, and the
// constants (A dt, b, Ta and their scaled forms, nu, q) are literals of the
// text (exact: hexadecimal floating point), rematerialised where used
// instead of held in scalar registers.  A mechanism whose constants change
// (lbfd_set_reaction) gets a new text and compile; texts already compiled
// in the process are reused.
//
// Arithmetic is that of chemistry() in lbfd_kernels.h, operation for
// operation and in the same order (Arrhenius rates, sub-step count, Euler
// sub-steps, positivity limiter); an omitted term is an exact zero there
// (a factor 1 or a product 0 nu r added to an increment), so both kernels
// give the same bits for finite rates.  Unity-Lewis transport only (the
// mixture-averaged c_p scaling stays in the generic kernel).
#include <hip/hip_runtime.h>
#include <hip/hiprtc.h>

#include <cmath>
#include <cstdio>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "lbfd_internal.h"

namespace lbfd {
namespace {

// the text of lbfd_math.h (written by the build)
const char kMathText[] =
#include "lbfd_math_text.inc"
    ;

struct ChemJitArgs {
    const char *sc_in;
    char *sc_out;
    const int *order;
    unsigned char *heavy;
    long long n_fluid;
    unsigned long long fstride;  // bytes between two scalar fields
    int substeps_max, anyb;
};

// a number as a C++ literal that reads back to the same double
std::string num(double v)
{
    if (std::isinf(v)) return v < 0 ? "(-__builtin_inf())" : "__builtin_inf()";
    char b[64];
    snprintf(b, sizeof b, "%a", v);
    return std::string("(") + b + ")";
}

// reactions whose exponentials are formed together
constexpr int kGroup = 4;

std::string generate(const ChemRx *rx, int n_rx, int nsp, bool fp64)
{
    const char *S = fp64 ? "double" : "float";
    std::string o;
    auto w = [&](const std::string &s) { o += s; o += "\n"; };
    auto f = [&](const char *fmt, auto... v) {
        char b[512];
        snprintf(b, sizeof b, fmt, v...);
        w(b);
    };
    w("#include \"lbfd_math.h\"");
    w("using namespace lbfd;");
    w("struct ChemJitArgs { const char *sc_in; char *sc_out; const int *order; unsigned char *heavy;");
    w("    long long n_fluid; unsigned long long fstride; int substeps_max, anyb; };");
    // three waves per SIMD (168 registers): at four (128) the unrolled
    // text spills (the compiler's schedule keeps more values live than in
    // the generic kernel's loop over reaction groups)
    w("extern \"C\" __global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3)))");
    // (named for its storage type, so that profiles tell the launches apart)
    f("lbfd_chem_jit_%s(const ChemJitArgs a)", fp64 ? "f64" : "f32");
    w("{");
    w("    __shared__ double tab[kExpTabN], ltab[2 * kLogTabN];");
    w("    for (int i = (int)threadIdx.x; i < kExpTabN; i += (int)blockDim.x) tab[i] = kExp2Tab[i];");
    w("    for (int i = (int)threadIdx.x; i < 2 * kLogTabN; i += (int)blockDim.x) ltab[i] = kLogTab[i];");
    w("    __syncthreads();");
    w("    const long long t = (long long)blockIdx.x * 256 + threadIdx.x;");
    w("    if (t >= a.n_fluid) return;");
    w("    const long long idx = a.order[t];");
    f("    const unsigned long long off = (unsigned long long)idx * sizeof(%s);", S);
    f("    const double T = (double)*(const %s *)(a.sc_in + off);", S);
    w("    const bool anyb = a.anyb != 0;");
    w("    int nsub = 1;");
    w("    if (a.substeps_max > 1) {");
    w("        const double lnT = anyb ? log(T) : 0.0, invT = rcp(T);");
    w("        double kmax = 0.0;");
    for (int j = 0; j < n_rx; ++j) {
        f("        kmax = fmax(kmax, %s * exp_tab(%s * lnT - %s * invT, tab));", num(rx[j].adt).c_str(),
          num(rx[j].b).c_str(), num(rx[j].ta).c_str());
    }
    w("        double want = ceil(kmax / 0.1);");
    w("        nsub = want < 1.0 ? 1 : want > (double)a.substeps_max ? a.substeps_max : (int)want;");
    w("    }");
    w("    const double lnNs = nsub == 1 ? 0.0 : log((double)nsub) * 0x1.71547652b82fep+8;");
    w("    double dT = 0.0;");
    for (int k = 0; k < nsp; ++k) f("    double dY%d = 0.0;", k);
    w("    for (int s = 0; s < nsub; ++s) {");
    w("        const double Tc = T + dT;");
    // Y_k is read again at every sub-step (from the cache) instead of being
    // held in registers for the whole loop: the offset passes through an
    // empty asm so that the loads stay in the loop.  Nine fewer register
    // pairs live across the loop cut the spills at three waves per SIMD.
    w("        unsigned long long offv = off;");
    w("        asm volatile(\"\" : \"+v\"(offv));");
    for (int k = 0; k < nsp; ++k)
        f("        const double Yc%d = (double)*(const %s *)(a.sc_in + %d * a.fstride + offv) + dY%d;", k, S, k + 1, k);
    w("        double incT = 0.0;");
    for (int k = 0; k < nsp; ++k) f("        double incY%d = 0.0;", k);
    w("        const double lnTc = anyb ? log_tab(Tc, ltab) : 0.0, invTc = rcp(Tc);");
    // reactions kGroup at a time, the exponentials of a group first, then
    // its increments in reaction order (the generic kernel's order of the
    // increments)
    for (int j0 = 0; j0 < n_rx; j0 += kGroup) {
        const int j1 = n_rx - j0 >= kGroup ? j0 + kGroup : n_rx;
        // (a reaction with A = 0 adds exact zeros in the generic kernel and
        // is left out; the others' arguments are finite, so the exponential
        // needs no clamp)
        for (int j = j0; j < j1; ++j) {
            if (!(rx[j].adt > 0.0)) continue;
            f("        const double k%d = exp_scaled_tab<false>(fma(%s, lnTc, fma(-%s, invTc, -lnNs)) + %s, tab);", j,
              num(rx[j].bs).c_str(), num(rx[j].tas).c_str(), num(rx[j].lnadts).c_str());
        }
        for (int j = j0; j < j1; ++j) {
            if (!(rx[j].adt > 0.0)) continue;
            f("        double r%d = k%d;", j, j);
            for (int m = 0; m < rx[j].n_react; ++m) f("        r%d *= Yc%d;", j, rx[j].react[m]);
            for (int k = 0; k < nsp; ++k)
                if (rx[j].nu[k] != 0.0)
                    f("        incY%d += %s * r%d;", k, num(rx[j].nu[k]).c_str(), j);
            f("        incT += %s * r%d;", num(rx[j].q).c_str(), j);
        }
    }
    w("        double lam = 1.0;");
    for (int k = 0; k < nsp; ++k)
        f("        if (incY%d < 0.0 && Yc%d + incY%d < 0.0) lam = fmin(lam, fmax(Yc%d, 0.0) * rcp(-incY%d));", k, k, k, k,
          k);
    w("        dT += lam * incT;");
    for (int k = 0; k < nsp; ++k) f("        dY%d += lam * incY%d;", k, k);
    w("    }");
    f("    *(%s *)(a.sc_out + off) = (%s)dT;", S, S);
    for (int k = 0; k < nsp; ++k) f("    *(%s *)(a.sc_out + %d * a.fstride + off) = (%s)dY%d;", S, k + 1, S, k);
    f("    a.heavy[idx] = nsub > %d;", kChemLight);
    w("}");
    return o;
}

std::mutex g_mu;
std::map<std::string, hipFunction_t> g_cache;  // (device, source) -> kernel, kept for the process

}  // namespace

std::string chem_jit_source(const ChemRx *rx, int n_rx, int nsp, bool fp64) { return generate(rx, n_rx, nsp, fp64); }

int chem_jit_build(const ChemRx *rx, int n_rx, int nsp, bool fp64, const void **fn, std::string &err)
{
    *fn = nullptr;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) {
        err = "hipGetDevice failed";
        return -1;
    }
    const std::string src = generate(rx, n_rx, nsp, fp64);
    const std::string key = std::to_string(dev) + "\n" + src;
    std::lock_guard<std::mutex> lock(g_mu);
    auto it = g_cache.find(key);
    if (it != g_cache.end()) {
        *fn = (const void *)it->second;
        return 0;
    }
    hiprtcProgram prog;
    const char *hdr[] = {kMathText};
    const char *hdr_name[] = {"lbfd_math.h"};
    if (hiprtcCreateProgram(&prog, src.c_str(), "lbfd_chem_jit.hip", 1, hdr, hdr_name) != HIPRTC_SUCCESS) {
        err = "hiprtcCreateProgram failed";
        return -1;
    }
    // the library's own flags: gfx950, -O3, packed FP32 instructions off
    const char *opts[] = {"--offload-arch=gfx950", "-O3",          "-std=c++17", "-Xclang",
                          "-target-feature",      "-Xclang",      "-packed-fp32-ops"};
    const hiprtcResult rc = hiprtcCompileProgram(prog, (int)(sizeof opts / sizeof opts[0]), opts);
    if (rc != HIPRTC_SUCCESS) {
        size_t n = 0;
        hiprtcGetProgramLogSize(prog, &n);
        std::string log(n, '\0');
        if (n) hiprtcGetProgramLog(prog, &log[0]);
        err = std::string("hiprtc compile failed: ") + hiprtcGetErrorString(rc) + "\n" + log;
        hiprtcDestroyProgram(&prog);
        return -1;
    }
    size_t sz = 0;
    hiprtcGetCodeSize(prog, &sz);
    std::vector<char> code(sz);
    hiprtcGetCode(prog, code.data());
    hiprtcDestroyProgram(&prog);
    hipModule_t mod;
    hipFunction_t f;
    if (hipModuleLoadData(&mod, code.data()) != hipSuccess ||
        hipModuleGetFunction(&f, mod, fp64 ? "lbfd_chem_jit_f64" : "lbfd_chem_jit_f32") != hipSuccess) {
        err = "loading the compiled chemistry kernel failed";
        return -1;
    }
    g_cache[key] = f;
    *fn = (const void *)f;
    return 0;
}

hipError_t launch_chem_jit(const KParams &kp, unsigned blocks, size_t scal_bytes, hipStream_t s)
{
    ChemJitArgs a;
    a.sc_in = (const char *)kp.sc_in;
    a.sc_out = (char *)kp.sc_out;
    a.order = kp.chem_order;
    a.heavy = kp.chem_heavy;
    a.n_fluid = kp.n_fluid;
    a.fstride = (unsigned long long)kp.N * scal_bytes;
    a.substeps_max = kp.chem_substeps_max;
    a.anyb = kp.chem_anyb;
    void *args[] = {&a};
    return hipModuleLaunchKernel((hipFunction_t)kp.chem_jit, blocks, 1, 1, 256, 1, 1, 0, s, args, nullptr);
}

}  // namespace lbfd
