"""The text of the chemistry kernel specialised to a mechanism
(lbfd_chemjit.hip), on the CPU: for the 9-species / 20-reaction synthetic
mechanism of the porous benchmark, the generator writes one reactant
multiply per reactant and one increment per nonzero mass coefficient (and
none for a zero one), every constant as a hexadecimal literal that reads
back to the reaction table's double, and the text compiles with the
run-time compiler (hiprtc, gfx950, the library's flags) from a working
directory other than the repository, for FP64 and FP32 storage.  A small
host program (built here with hipcc, linked against liblbfd.so) calls the
generator and the compiler; no GPU is used."""
import math
import os
import re
import shutil
import subprocess
import tempfile

import pytest

from paper_2304_05657_amd import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PKG = os.path.join(ROOT, "paper_2304_05657_amd")
HIPCC = "/opt/rocm/bin/hipcc"
SCALE = float.fromhex("0x1.71547652b82fep+8")  # 256 / ln 2, as the host scales b, Ta and ln(A dt)

HARNESS = r'''
#include <hip/hip_runtime.h>
#include <hip/hiprtc.h>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <sstream>
#include <string>
#include <vector>
#include "lbfd_internal.h"
struct R { double adt, b, Ta, q; int n; int react[4]; double nu[9]; };
static const R rs[] = { %(rows)s };
int main(int argc, char **argv) {
    const int n = sizeof(rs) / sizeof(rs[0]);
    std::vector<lbfd::ChemRx> h(n);
    memset(h.data(), 0, sizeof(lbfd::ChemRx) * n);
    const double c = 0x1.71547652b82fep+8;
    for (int j = 0; j < n; ++j) {
        h[j].adt = rs[j].adt; h[j].b = rs[j].b; h[j].ta = rs[j].Ta; h[j].q = rs[j].q; h[j].n_react = rs[j].n;
        h[j].bs = h[j].b * c; h[j].tas = h[j].ta * c; h[j].lnadts = std::log(h[j].adt) * c;
        for (int m = 0; m < 4; ++m) h[j].react[m] = rs[j].react[m];
        for (int k = 0; k < 9; ++k) h[j].nu[k] = rs[j].nu[k];
    }
    const bool fp64 = strcmp(argv[1], "f64") == 0;
    const std::string src = lbfd::chem_jit_source(h.data(), n, 9, fp64);
    std::ofstream(argv[2]) << src;
    std::ifstream hf(argv[3]);
    std::stringstream hs; hs << hf.rdbuf();
    const std::string hdr = hs.str();
    hiprtcProgram p;
    const char *hd[] = {hdr.c_str()};
    const char *hn[] = {"lbfd_math.h"};
    if (hiprtcCreateProgram(&p, src.c_str(), "chem.hip", 1, hd, hn) != HIPRTC_SUCCESS) return 3;
    const char *o[] = {"--offload-arch=gfx950", "-O3", "-std=c++17", "-Xclang", "-target-feature", "-Xclang",
                       "-packed-fp32-ops"};
    const hiprtcResult r = hiprtcCompileProgram(p, 7, o);
    size_t ls = 0;
    hiprtcGetProgramLogSize(p, &ls);
    std::string log(ls, '\0');
    if (ls) hiprtcGetProgramLog(p, &log[0]);
    size_t cs = 0;
    if (r == HIPRTC_SUCCESS) hiprtcGetCodeSize(p, &cs);
    printf("rc %%d code %%zu\n%%s\n", (int)r, cs, log.c_str());
    return r == HIPRTC_SUCCESS && cs > 0 ? 0 : 2;
}
'''


@pytest.fixture(scope="module")
def harness():
    lib = os.path.join(PKG, "liblbfd.so")
    if not (os.path.exists(HIPCC) and os.path.exists(lib)):
        pytest.skip("hipcc or the built library is missing")
    prob = W.porous_3d_mech(nx=32, ny=16, nz=16, margin=4, name="mech_src")
    dt = 1e-6
    rows = []
    for r in prob.reactions:
        re_ = list(r.reactants) + [prob.n_species] * (4 - len(r.reactants))
        rows.append("{ %r, %r, %r, %r, %d, {%s}, {%s} }" % (
            r.A * dt, r.b, r.Ta, r.q, len(r.reactants), ",".join(map(str, re_)),
            ", ".join(repr(float(x)) for x in r.nu)))
    d = tempfile.mkdtemp(prefix="lbfd_chem_src_")
    src = os.path.join(d, "h.hip")
    with open(src, "w") as f:
        f.write(HARNESS % {"rows": ",\n".join(rows)})
    exe = os.path.join(d, "h")
    subprocess.run([HIPCC, "-std=c++17", "-I", os.path.join(PKG, "csrc"), src, "-o", exe, "-L" + PKG, "-llbfd",
                    "-L/opt/rocm/lib", "-lhiprtc", "-Wl,-rpath," + PKG + ":/opt/rocm/lib"],
                   check=True, capture_output=True)
    yield prob, dt, exe, d
    shutil.rmtree(d, ignore_errors=True)


@pytest.mark.parametrize("kind", ["f64", "f32"])
def test_generated_text_compiles(harness, kind):
    prob, dt, exe, d = harness
    out = os.path.join(d, "chem_%s.hip" % kind)
    r = subprocess.run([exe, kind, out, os.path.join(PKG, "csrc", "lbfd_math.h")], cwd=d,
                       capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stdout + r.stderr
    text = open(out).read()
    assert ("lbfd_chem_jit_%s(" % kind) in text
    S = "double" if kind == "f64" else "float"
    assert "(const %s *)(a.sc_in" % S in text and "*(%s *)(a.sc_out" % S in text


def test_generated_text_structure(harness):
    prob, dt, exe, d = harness
    out = os.path.join(d, "chem_struct.hip")
    r = subprocess.run([exe, "f64", out, os.path.join(PKG, "csrc", "lbfd_math.h")], cwd=d,
                       capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stdout + r.stderr
    text = open(out).read()
    rx = prob.reactions
    # one multiply per reactant, in the reaction's own order
    for j, rj in enumerate(rx):
        assert re.findall(r"r%d \*= Yc(\d+);" % j, text) == [str(k) for k in rj.reactants]
    # one increment per nonzero mass coefficient, with its exact value
    incs = re.findall(r"incY(\d+) \+= \(([-0-9a-fx.p+]+)\) \* r(\d+);", text)
    want = [(k, j, v) for j, rj in enumerate(rx) for k, v in enumerate(rj.nu) if v != 0.0]
    assert len(incs) == len(want) == 69
    got = sorted((int(k), int(j), float.fromhex(v)) for k, v, j in incs)
    assert got == sorted(want)
    # the rate constants as the host forms them, each read back exactly
    for j, rj in enumerate(rx):
        lit = re.search(r"const double k%d = exp_scaled_tab<false>\(fma\(\(([^)]+)\), lnTc, fma\(-\(([^)]+)\), invTc, "
                        r"-lnNs\)\) \+ \(([^)]+)\), tab\);" % j, text)
        assert lit is not None, j
        assert float.fromhex(lit.group(1)) == rj.b * SCALE
        assert float.fromhex(lit.group(2)) == rj.Ta * SCALE
        assert float.fromhex(lit.group(3)) == math.log(rj.A * dt) * SCALE
