"""Every optional treatment at once, through the C ABI against the FP64
oracle: cumulant collision, mixture-averaged transport, interpolated
bounce-back and Shepard image points on the cylinders, and a sheared inlet
profile changed mid-run (the burner at 512 x 128, D2Q9), and the 3-D
counterpart on a sphere packing."""
import numpy as np
import pytest

from paper_2304_05657_amd import workloads as W

from .gpu_util import compare_fields, need_gpu, oracle_threads, say

pytestmark = pytest.mark.gpu
TOL64 = 1e-10


def _setup(prob, precision="fp64"):
    import oracle
    from paper_2304_05657_amd.lbfd import Solver
    need_gpu()
    g = Solver(prob, precision=precision)
    o = oracle.Oracle(prob, threads=oracle_threads())
    cells, dirs, q = W.wall_links(prob)
    g.set_wall_links(cells, dirs, q)
    o.set_wall_links(cells, dirs, q.astype(np.float32).astype(np.float64))
    c, sl, im = W.image_points(prob)
    g.set_image_points(c, sl, im)
    o.set_image_points(c, sl, im)
    say("  %d links, %d image points" % (len(q), len(c)))
    return g, o


def _profile(prob, scale):
    """A sheared inlet profile [3, nz, ny]: u_x varies across the face."""
    y = np.arange(prob.ny, dtype=np.float64)
    u = np.zeros((3, prob.nz, prob.ny))
    u[0] = (prob.u_in[0] * scale * (1.0 + 0.3 * np.sin(2.0 * np.pi * y / prob.ny)))[None, :]
    return u


def _compare(g, o, prob, level):
    e = compare_fields(g.fields(), o.fields(), prob)
    say("  level %d: %s" % (level, " ".join("%s=%.2e" % kv for kv in e.items())))
    for k, v in e.items():
        assert v <= TOL64, (level, k, v)


def test_burner_everything_fp64():
    prob = W.cylinder_burner(nx=512, ny=128, x_begin=128, x_end=384, front_x=256.0, name="all_burner_512x128")
    prob = W.mixture_transport(prob).replace(collision="cumulants")
    say("case %s: cumulants, mixture-averaged transport, curved walls, inlet profile" % prob.name)
    g, o = _setup(prob)
    for p in (g, o):
        p.set_inflow(0, _profile(prob, 1.0))
    g.step(100)
    o.step(100)
    _compare(g, o, prob, 100)
    for p in (g, o):
        p.set_inflow(0, _profile(prob, 0.7))
    g.step(100)
    o.step(100)
    _compare(g, o, prob, 200)


def test_porous_everything_fp64():
    prob = W.porous_3d(nx=48, ny=20, nz=18, porosity=0.85, radius=4.0, margin=8, seed=7, name="all_porous3d")
    prob = W.mixture_transport(prob).replace(collision="cumulants")
    say("case %s: cumulants, mixture-averaged transport, curved walls" % prob.name)
    g, o = _setup(prob)
    g.step(40)
    o.step(40)
    _compare(g, o, prob, 40)


def test_burner_everything_fp16():
    prob = W.cylinder_burner(nx=512, ny=128, x_begin=128, x_end=384, front_x=256.0, name="all_burner_fp16")
    prob = W.mixture_transport(prob).replace(collision="cumulants")
    say("case %s: everything, FP16 populations, 200 steps" % prob.name)
    g, o = _setup(prob, "fp16")
    g.step(200)
    o.step(200)
    gf, of = g.fields(), o.fields()
    fl = prob.mask == 0
    eT = np.abs(gf["T"][fl] - of["T"][fl]).max() / (prob.T_b - prob.T_u)
    eu = np.abs(gf["u"][:2][:, fl] - of["u"][:2][:, fl]).max() / np.abs(of["u"][:2][:, fl]).max()
    say("  T_max_rel %.2e u_max_rel %.2e" % (eT, eu))
    assert eT < 5e-4 and eu < 5e-3
