"""Parity at the full 3-D sizes the benchmark runs (256^3 sphere packing,
4 species; 512 x 256 x 256 packing with 9 species / 20 reactions), on a
sample of cells.

The oracle steps only the dependency cone of the sample (three cells per
level; its CPU pin shows the sample then holds exactly the values of full
steps), from the same seeded initial state as the GPU.  The GPU runs the
whole box in the launch configuration the benchmark times.  FP64 is held to
the 1e-10 parity bar; the mixed-precision storage the benchmark reports for
the workload is held to the accuracy bounds of the small 3-D case.
"""
import numpy as np
import pytest

from paper_2304_05657_amd import workloads as W

from .gpu_util import need_gpu, oracle_threads, say

pytestmark = pytest.mark.gpu
TOL64 = 1e-10
STEPS = 2
N_SAMPLE = 1024
# T error / (T_b - T_u), u error / max |u| over the sample (as for the
# small porous case)
MIXED_BOUNDS = {"fp32": (5e-6, 5e-5), "fp16": (5e-5, 2e-3)}


def _sample(prob, seed):
    """Random fluid cells, plus fluid cells next to the inlet and outlet."""
    rng = np.random.default_rng(seed)
    fluid = prob.mask == 0
    s = np.zeros(fluid.shape, bool)
    s.reshape(-1)[rng.choice(np.flatnonzero(fluid), N_SAMPLE, replace=False)] = True
    rows = s.reshape(-1, prob.nx)
    for x in (0, 1, prob.nx - 2, prob.nx - 1):
        plane = np.flatnonzero(fluid[..., x].reshape(-1))
        rows[rng.choice(plane, min(16, plane.size), replace=False), x] = True
    return s


def _errors(gf, of, sel, prob):
    def rel(a, b):
        scale = np.abs(b).max()
        return float(np.abs(a - b).max() / (scale if scale > 0 else 1.0))

    out = {"u": rel(gf["u"][:, sel], of["u"][:, sel])}
    for k in ("T", "rho", "Ph"):
        out[k] = rel(gf[k][sel], of[k][sel])
    out["Y"] = max(rel(gf["Y"][j][sel], of["Y"][j][sel]) for j in range(of["Y"].shape[0]))
    out["T_abs"] = float(np.abs(gf["T"][sel] - of["T"][sel]).max() / (prob.T_b - prob.T_u))
    return out


def _check(prob, mixed, seed, links=False):
    import oracle
    from paper_2304_05657_amd.lbfd import Solver
    need_gpu()
    say("case %s %dx%dx%d Q%d: oracle cone over %d steps" % (prob.name, prob.nx, prob.ny, prob.nz,
                                                           prob.lattice, STEPS))
    sel = _sample(prob, seed)
    o = oracle.Oracle(prob, threads=oracle_threads())
    wl = W.wall_links(prob) if links else None
    if links:
        say("  %d wall links" % len(wl[0]))
        o.set_wall_links(wl[0], wl[1], wl[2].astype(np.float32).astype(np.float64))
    o.step_sampled(sel, STEPS)
    of = o.fields()
    del o
    assert np.isfinite(of["T"][sel]).all()
    for precision in ("fp64", mixed):
        say("  gpu %s, %d steps, %d sampled cells" % (precision, STEPS, int(sel.sum())))
        g = Solver(prob, precision=precision)
        if links:
            g.set_wall_links(*wl)
        g.step(STEPS)
        gf = g.fields()
        g.close()
        e = _errors(gf, of, sel, prob)
        say("  %s: %s" % (precision, " ".join("%s=%.2e" % kv for kv in e.items())))
        if precision == "fp64":
            for k in ("u", "T", "rho", "Ph", "Y"):
                assert e[k] <= TOL64, (precision, k, e[k])
        else:
            bT, bu = MIXED_BOUNDS[precision]
            assert e["T_abs"] <= bT and e["u"] <= bu, (precision, e)
        del gf


def test_porous_256_cubed_sampled():
    """256^3, D3Q27, 4 species: FP64 and FP16 population storage."""
    _check(W.porous_3d(), "fp16", seed=21)


def test_porous_mechanism_512x256x256_sampled():
    """512 x 256 x 256, D3Q27, 9 species / 20 reactions (sub-cycled FP64
    source): FP64 and FP32 population storage."""
    _check(W.porous_3d_mech(), "fp32", seed=22)


def test_porous_256_cubed_mixture_curved_sampled():
    """256^3, D3Q27, 4 species with mixture-averaged transport and the
    interpolated bounce-back on every link into a sphere: FP64 and FP32."""
    _check(W.mixture_transport(W.porous_3d()), "fp32", seed=23, links=True)
