"""lbfd_objective_static (the objective without device allocation, its
scratch in the library's static per-GPU array) against lbfd_objective on
twin contexts, through the C ABI: two calls in a row, the second on a
smaller box (fewer step blocks, so fewer partials in the shared array),
with the wall-heat-flux and the flame-position objectives."""
import ctypes as C

import numpy as np
import pytest

from paper_2304_05657_amd import workloads as W

from .gpu_util import need_gpu, say

pytestmark = pytest.mark.gpu


def _call_static(s, n):
    J = C.c_double()
    rc = s._lib.lbfd_objective_static(s._h, C.c_int64(n), C.byref(J))
    assert rc == 0, s._lib.lbfd_last_error().decode()
    return J.value


def _call_alloc(s, n):
    J = C.c_double()
    rc = s._lib.lbfd_objective(s._h, C.c_int64(n), C.byref(J))
    assert rc == 0, s._lib.lbfd_last_error().decode()
    return J.value


@pytest.mark.parametrize("kind", ["wall_q", "flame_x"])
def test_objective_static_matches_objective(kind):
    from paper_2304_05657_amd.lbfd import Solver
    need_gpu()
    cases = [(W.channel_flame(nx=256, ny=64, front_x=64.0, name="noalloc_256x64"), 40),
             (W.channel_flame(nx=96, ny=24, front_x=30.0, name="noalloc_96x24"), 25)]
    for prob, n in cases:
        say("case %s, objective %s over %d steps" % (prob.name, kind, n))
        a, b = Solver(prob), Solver(prob)
        for s in (a, b):
            s.set_objective(kind, 3, n - 2)
            s.step(7)
        ja = _call_static(a, n)
        jb = _call_alloc(b, n)
        assert np.isfinite(ja) and ja != 0.0
        assert abs(ja - jb) <= 1e-13 * abs(jb), (ja, jb)
        # the states advanced alike
        fa, fb = a.fields(), b.fields()
        assert np.array_equal(fa["T"], fb["T"]) and np.array_equal(fa["u"], fb["u"])
        a.close()
        b.close()
