"""Build liblbfd.so (gfx950) in-tree with hipcc.

Every HIP source is compiled to an object under ``_build/`` (in parallel,
one translation unit per kernel configuration) and linked into
``paper_2304_05657_amd/liblbfd.so``.  ``python -m paper_2304_05657_amd.build``
rebuilds what changed; ``--force`` rebuilds everything.
"""
from __future__ import annotations

import concurrent.futures as cf
import glob
import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
BUILD = os.path.join(ROOT, "_build", "lbfd")
LIB = os.path.join(PKG, "liblbfd.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

# Packed FP32 instructions are disabled (-packed-fp32-ops): plain float code
# is kept on the scalar-lane VALU path.
GEN = os.path.join(BUILD, "gen")
FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-Wall",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-I", os.path.join(ROOT, "include"), "-I", GEN]


def sources() -> list[str]:
    return ([os.path.join(CSRC, "lbfd_api.hip"), os.path.join(CSRC, "lbfd_dispatch.hip"),
             os.path.join(CSRC, "lbfd_adjoint.hip"), os.path.join(CSRC, "lbfd_chemjit.hip")]
            + sorted(glob.glob(os.path.join(CSRC, "inst", "*.hip"))))


def _headers() -> list[str]:
    return glob.glob(os.path.join(CSRC, "*.h")) + [os.path.join(ROOT, "include", "lbfd.h")]


def _obj(src: str) -> str:
    rel = os.path.relpath(src, CSRC).replace(os.sep, "_")
    return os.path.join(BUILD, rel + ".o")


def _asm(src: str) -> str:
    """The device assembly the compile of src leaves beside its object."""
    base = os.path.splitext(os.path.basename(src))[0]
    return os.path.join(BUILD, base + "-hip-amdgcn-amd-amdhsa-gfx950.s")


def _compile(src: str) -> tuple[str, int, str]:
    obj = _obj(src)
    tmp = obj + ".tmp%d" % os.getpid()
    # -save-temps=obj keeps the device assembly (for the check below) in
    # the build folder; the other intermediate files are removed
    cmd = [HIPCC] + FLAGS + ["-save-temps=obj", "-c", src, "-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    base = os.path.splitext(os.path.basename(src))[0]
    for f in glob.glob(os.path.join(BUILD, base + "-hip-*")) + glob.glob(os.path.join(BUILD, base + "-host-*")) + \
            glob.glob(os.path.join(BUILD, base + ".hip-hip-*")):
        if f != _asm(src):
            os.remove(f)
    if r.returncode == 0:
        os.replace(tmp, obj)
    out = "\n".join(l for l in (r.stdout + r.stderr).splitlines()
                    if "packed-fp32-ops" not in l and l.strip())
    return src, r.returncode, out


def _gen_math_text() -> None:
    """The text of lbfd_math.h as a C++ raw string literal (the run-time
    compile of the specialised chemistry kernel is given it), rewritten
    only when it changes."""
    os.makedirs(GEN, exist_ok=True)
    with open(os.path.join(CSRC, "lbfd_math.h")) as f:
        text = f.read()
    assert ")LBFDMATH\"" not in text
    out = 'R"LBFDMATH(' + text + ')LBFDMATH"\n'
    path = os.path.join(GEN, "lbfd_math_text.inc")
    if not os.path.exists(path) or open(path).read() != out:
        with open(path, "w") as f:
            f.write(out)


def build(force: bool = False, jobs: int | None = None, verbose: bool = True) -> str:
    os.makedirs(BUILD, exist_ok=True)
    _gen_math_text()
    hdr_mtime = max(os.path.getmtime(h) for h in _headers())
    todo = []
    for s in sources():
        o = _obj(s)
        if force or not os.path.exists(o) or os.path.getmtime(o) < max(os.path.getmtime(s), hdr_mtime):
            todo.append(s)
    jobs = jobs or min(8, os.cpu_count() or 4)
    failed = []
    if todo:
        with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
            for src, rc, out in ex.map(_compile, todo):
                if verbose:
                    print("[lbfd build] %s %s" % ("ok  " if rc == 0 else "FAIL", os.path.relpath(src, ROOT)),
                          flush=True)
                if out and (rc != 0 or verbose):
                    print(out, flush=True)
                if rc != 0:
                    failed.append(src)
    if failed:
        raise RuntimeError("hipcc failed for: " + ", ".join(failed))
    # every kernel's assembly is checked for copies that only some lanes of
    # a divergent branch receive (a miscompilation of the register
    # allocator; see isa_check.py); a library holding one is not linked
    from . import isa_check
    missing = [s for s in sources() if not os.path.exists(_asm(s))]
    if missing:
        raise RuntimeError("device assembly missing for: " + ", ".join(missing) + " (rebuild with force=True)")
    bad = isa_check.check([_asm(s) for s in sources()])
    if bad:
        for path, name, ins in bad[:20]:
            print("[lbfd build] %s: %s: %s" % (os.path.basename(path), name, ins), flush=True)
        raise RuntimeError("%d one-sided register copies in divergent code (isa_check.py); the library is not "
                           "linked" % len(bad))
    if verbose:
        print("[lbfd build] assembly of %d units checked: no one-sided copies" % len(sources()), flush=True)
    objs = [_obj(s) for s in sources()]
    if force or todo or not os.path.exists(LIB) or os.path.getmtime(LIB) < max(os.path.getmtime(o) for o in objs):
        tmp = LIB + ".tmp%d" % os.getpid()
        subprocess.check_call([HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + objs +
                              ["-L/opt/rocm/lib", "-lhiprtc", "-Wl,-rpath,/opt/rocm/lib"])
        os.replace(tmp, LIB)
        if verbose:
            print("[lbfd build] linked %s" % os.path.relpath(LIB, ROOT), flush=True)
    return LIB


if __name__ == "__main__":
    build(force="--force" in sys.argv)
