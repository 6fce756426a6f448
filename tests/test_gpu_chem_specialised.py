"""The chemistry kernel specialised to a mechanism's structure (compiled at
set-up) against the generic kernel: on the 9-species / 20-reaction porous
mechanism workload both give the same bits for T and Y_k after several steps
(FP64 and FP32 storage), the context reports which kernel runs, and a changed
rate constant (lbfd_set_reaction, a new specialised text) still agrees with
the generic kernel bit for bit."""
import os

import numpy as np
import pytest

from paper_2304_05657_amd import workloads as W

from .gpu_util import need_gpu, say

pytestmark = pytest.mark.gpu


def _run(prob, precision, jit, steps, setrx=None):
    from paper_2304_05657_amd.lbfd import Solver
    old = os.environ.get("LBFD_CHEM_JIT")
    os.environ["LBFD_CHEM_JIT"] = "1" if jit else "0"
    try:
        s = Solver(prob, precision=precision)
    finally:
        if old is None:
            del os.environ["LBFD_CHEM_JIT"]
        else:
            os.environ["LBFD_CHEM_JIT"] = old
    if setrx is not None:
        s.set_reaction(*setrx)
    spec, note = s.chem_kernel()
    s.step(steps)
    f = s.fields()
    s.close()
    return spec, note, f


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_specialised_equals_generic(precision):
    need_gpu()
    prob = W.porous_3d_mech(nx=48, ny=24, nz=24, margin=6, name="mech_48x24x24")
    say("case specialised chemistry vs generic, %s, mechanism 48x24x24, 6 steps" % precision)
    spec, note, fj = _run(prob, precision, True, 6)
    say("  specialised: %s (%s)" % (spec, note[:200]))
    assert spec, note
    gen, note_g, fg = _run(prob, precision, False, 6)
    assert not gen and "LBFD_CHEM_JIT=0" in note_g
    fluid = prob.mask == 0
    for key in ("T", "Y"):
        a, b = np.asarray(fj[key]), np.asarray(fg[key])
        assert np.all(np.isfinite(a))
        diff = np.abs(a - b)[..., fluid] if key == "Y" else np.abs(a - b)[fluid]
        say("  %s max |specialised - generic| = %.3e" % (key, float(diff.max())))
        assert np.array_equal(a, b), key


def test_specialised_after_set_reaction():
    need_gpu()
    prob = W.porous_3d_mech(nx=32, ny=16, nz=16, margin=4, name="mech_32x16x16")
    r = prob.reactions[3]
    setrx = (3, r.A * 1.7, r.b + 0.1, r.Ta * 0.95)
    say("case specialised chemistry after lbfd_set_reaction, mechanism 32x16x16, 4 steps")
    spec, note, fj = _run(prob, "fp64", True, 4, setrx)
    assert spec, note
    _, _, fg = _run(prob, "fp64", False, 4, setrx)
    assert np.array_equal(np.asarray(fj["T"]), np.asarray(fg["T"]))
    assert np.array_equal(np.asarray(fj["Y"]), np.asarray(fg["Y"]))
