"""Mixed-precision forms (FP32 / FP16 population storage, FP32 arithmetic,
FP64 Arrhenius source and reductions) against the FP64 oracle.

These are accuracy reports with stated bounds, not bit-parity: the storage
rounding (2^-24 relative for float, 2^-11 for half, on g / (w_i cs^2)) and
float arithmetic (2^-24 per operation) accumulate over the run.  The bounds
below are about twice the errors measured on MI355X for the same runs.
"""
import numpy as np
import pytest

from paper_2304_05657_amd import workloads as W

from .gpu_util import need_gpu, oracle_threads, say

pytestmark = pytest.mark.gpu

# bounds on max |T - T_oracle| / (T_b - T_u), max |u - u_oracle| / max |u_oracle|
# (and max |Y - Y_oracle| for the mechanism) and the flame-position shift in
# cells, at about twice the errors measured on MI355X for the same runs:
# channel 2000 steps fp32 (2.26e-5, 1.23e-4, 1.02e-3 cells), fp16 (7.7e-4,
# 4.64e-2, 4.2e-4); porous 60 steps fp32 (6.3e-7, 8.4e-6), fp16 (6.9e-6,
# 3.46e-4); mechanism 200 steps fp32 (T 3.26e-6, Y 1.39e-6, u 1.84e-5),
# fp16 (T 1.07e-5, Y 1.48e-6, u 5.5e-4).  Both sides are deterministic, so
# the margin covers toolchain-level rounding changes, not run-to-run noise.
CHANNEL_BOUNDS = {"fp32": (5e-5, 2.5e-4, 2.5e-3), "fp16": (1.6e-3, 1e-1, 1e-3)}
POROUS_BOUNDS = {"fp32": (1.3e-6, 1.7e-5), "fp16": (1.4e-5, 7e-4)}
MECH_BOUNDS = {"fp32": (7e-6, 3e-6, 4e-5), "fp16": (2.2e-5, 3e-6, 1.1e-3)}


def _flame_x(d, prob):
    return prob.nx - d["sum_theta"] / (prob.n_fluid / prob.nx)


@pytest.mark.parametrize("precision", ["fp32", "fp16"])
def test_channel_flame_mixed_vs_oracle(precision):
    import oracle
    from paper_2304_05657_amd.lbfd import Solver
    need_gpu()
    prob = W.channel_flame()
    steps = 2000
    say("case channel_flame_256x64 %s steps=%d" % (precision, steps))
    g = Solver(prob, precision=precision)
    o = oracle.Oracle(prob, threads=oracle_threads())
    g.step(steps)
    o.step(steps)
    gf, of = g.fields(), o.fields()
    fl = prob.mask == 0
    eT = np.abs(gf["T"][fl] - of["T"][fl]).max() / (prob.T_b - prob.T_u)
    umax = np.abs(of["u"][:2][:, fl]).max()
    eu = np.abs(gf["u"][:2][:, fl] - of["u"][:2][:, fl]).max() / umax
    dx = abs(_flame_x(g.diagnostics(), prob) - _flame_x(o.diagnostics(), prob))
    say("  %s: T_max_rel=%.3e u_max_rel=%.3e flame_dx=%.3e cells" % (precision, eT, eu, dx))
    bT, bu, bx = CHANNEL_BOUNDS[precision]
    assert eT <= bT and eu <= bu and dx <= bx, (eT, eu, dx)


@pytest.mark.parametrize("precision", ["fp32", "fp16"])
def test_porous_3d_mixed_vs_oracle(precision):
    import oracle
    from paper_2304_05657_amd.lbfd import Solver
    need_gpu()
    prob = W.porous_3d(nx=48, ny=20, nz=18, porosity=0.85, radius=4.0, margin=8, seed=7,
                       name="porous3d_48x20x18")
    steps = 60
    say("case porous3d_48x20x18 %s steps=%d" % (precision, steps))
    g = Solver(prob, precision=precision)
    o = oracle.Oracle(prob, threads=oracle_threads())
    g.step(steps)
    o.step(steps)
    gf, of = g.fields(), o.fields()
    fl = prob.mask == 0
    eT = np.abs(gf["T"][fl] - of["T"][fl]).max() / (prob.T_b - prob.T_u)
    umax = np.abs(of["u"][:, fl]).max()
    eu = np.abs(gf["u"][:, fl] - of["u"][:, fl]).max() / umax
    say("  %s: T_max_rel=%.3e u_max_rel=%.3e" % (precision, eT, eu))
    bT, bu = POROUS_BOUNDS[precision]
    assert eT <= bT and eu <= bu, (eT, eu)


@pytest.mark.parametrize("precision", ["fp32", "fp16"])
def test_porous_mechanism_mixed_vs_oracle(precision):
    """The 9-species / 20-reaction mechanism (FP64 sub-cycled sources, FP32
    arithmetic elsewhere), 200 steps."""
    import oracle
    from paper_2304_05657_amd.lbfd import Solver
    need_gpu()
    prob = W.porous_3d_mech(nx=32, ny=12, nz=12, porosity=0.9, radius=(2.0, 4.0), margin=6,
                            name="porous3d_mech_32x12x12")
    steps = 200
    say("case porous3d_mech_32x12x12 %s steps=%d" % (precision, steps))
    g = Solver(prob, precision=precision)
    o = oracle.Oracle(prob, threads=oracle_threads())
    g.step(steps)
    o.step(steps)
    gf, of = g.fields(), o.fields()
    fl = prob.mask == 0
    eT = np.abs(gf["T"][fl] - of["T"][fl]).max() / (prob.T_b - prob.T_u)
    eY = np.abs(gf["Y"][:, fl] - of["Y"][:, fl]).max()
    umax = np.abs(of["u"][:, fl]).max()
    eu = np.abs(gf["u"][:, fl] - of["u"][:, fl]).max() / umax
    say("  %s: T_max_rel=%.3e Y_max_abs=%.3e u_max_rel=%.3e" % (precision, eT, eY, eu))
    bT, bY, bu = MECH_BOUNDS[precision]
    assert eT <= bT and eY <= bY and eu <= bu, (eT, eY, eu)
