"""Velocity-inlet profiles, the consumption-speed diagnostic and flame
holding (Sec. IV.A: the flow rate follows the flame so that the front stays
in the box; a 2-D Poiseuille inlet), through the C ABI against the FP64
oracle."""
import numpy as np
import pytest

from paper_2304_05657_amd import workloads as W

from .gpu_util import compare_fields, need_gpu, oracle_threads, say

pytestmark = pytest.mark.gpu
TOL64 = 1e-10


def _pair(prob, profile, steps, checkpoints):
    import oracle
    from paper_2304_05657_amd.lbfd import Solver
    need_gpu()
    g = Solver(prob)
    o = oracle.Oracle(prob, threads=oracle_threads())
    g.set_inflow(0, profile)
    o.set_inflow(0, profile)
    done = 0
    for target in checkpoints + [steps]:
        g.step(target - done)
        o.step(target - done)
        done = target
        e = compare_fields(g.fields(), o.fields(), prob)
        say("  level %d: %s" % (done, " ".join("%s=%.2e" % kv for kv in e.items())))
        for k, v in e.items():
            assert v <= TOL64, (done, k, v)
    return g, o


def test_poiseuille_inlet_flame_channel():
    """D2Q9 channel with adiabatic walls, Poiseuille inlet at -x, outflow,
    burning (A = 1e10): fields and the fuel / consumption diagnostics."""
    prob = W.flame_channel(nx=192, ny=18, u_mean=0.004, front_x=96.0, name="flame_channel_192x18")
    say("case %s with a Poiseuille inlet, 400 steps" % prob.name)
    g, o = _pair(prob, W.poiseuille_profile(prob, 0.004), 400, [1, 100])
    dg, do = g.diagnostics(), o.diagnostics()
    for k in ("fuel_rate", "fuel_mass_rate", "consumption_speed", "sum_theta"):
        say("  %s gpu %.15e oracle %.15e" % (k, dg[k], do[k]))
        assert abs(dg[k] - do[k]) <= 1e-10 * abs(do[k]), k


def test_inlet_profile_3d():
    """D3Q27 packing with a profile varying over the inlet face in y and z
    (and a transverse component)."""
    prob = W.porous_3d(nx=48, ny=20, nz=18, porosity=0.85, radius=4.0, margin=8, seed=7,
                       name="porous3d_profile_48x20x18")
    y = np.arange(prob.ny)[None, :]
    z = np.arange(prob.nz)[:, None]
    u = np.zeros((3, prob.nz, prob.ny))
    u[0] = 0.01 * (1.0 + 0.3 * np.sin(2 * np.pi * y / prob.ny) * np.cos(2 * np.pi * z / prob.nz))
    u[2] = 0.002 * np.sin(2 * np.pi * y / prob.ny)
    say("case %s with a y-z inlet profile, 60 steps" % prob.name)
    _pair(prob, u, 60, [1, 10])


def test_flame_holding_matches_oracle_control():
    """lbfd_hold_flame against the same control law driving the oracle:
    per cycle, U = max(0, s_c - gain (x_f - x_target)) times the profile's
    shape; the U and x_f histories agree to 1e-8."""
    import oracle
    from paper_2304_05657_amd.lbfd import Solver
    need_gpu()
    prob = W.flame_channel(nx=256, ny=18, u_mean=0.002, front_x=128.0, name="hold_256x18")
    prof = W.poiseuille_profile(prob, 0.002)
    steps, every, target, gain = 2000, 100, 128.0, 2e-5  # U stays positive (unclamped)
    say("case flame holding vs oracle, %s, %d steps every %d" % (prob.name, steps, every))
    g = Solver(prob)
    g.set_inflow(0, prof)
    U, X = g.hold_flame(steps, every, target, gain)
    o = oracle.Oracle(prob, threads=oracle_threads())
    o.set_inflow(0, prof)
    fl = prob.mask[0, :, 0] == 0
    shape = prof / prof[0, 0, fl].mean()
    for k in range(steps // every):
        o.step(every)
        d = o.diagnostics()
        xf = prob.nx - d["sum_theta"] / (prob.n_fluid / prob.nx)
        Uo = max(0.0, d["consumption_speed"] - gain * (xf - target))
        o.set_inflow(0, Uo * shape)
        assert abs(X[k] - xf) <= 1e-8 * abs(xf), (k, X[k], xf)
        assert Uo > 0.0 and abs(U[k] - Uo) <= 1e-8 * abs(Uo), (k, U[k], Uo)
    say("  last cycle: x_f %.6f (oracle %.6f), U %.6e (oracle %.6e)" % (X[-1], xf, U[-1], Uo))


def test_flame_holding_converges():
    """Held for 1.2e5 steps, the flame settles within 1 cell of the target
    (a proportional law keeps an offset) and its inlet velocity settles to
    the flame speed; an inlet held at the initial velocity lets the flame
    drift far from the target instead."""
    from paper_2304_05657_amd.lbfd import Solver
    need_gpu()
    prob = W.flame_channel(nx=256, ny=18, u_mean=0.002, front_x=128.0, name="hold_256x18")
    prof = W.poiseuille_profile(prob, 0.002)
    say("case flame holding, 120000 steps")
    g = Solver(prob)
    g.set_inflow(0, prof)
    U, X = g.hold_flame(120000, 200, 128.0, 1e-4)
    say("  x_f: %.3f -> %.3f, U: %.6e -> %.6e" % (X[0], X[-1], U[0], U[-1]))
    assert abs(X[-1] - 128.0) < 1.0
    assert np.ptp(X[-20:]) < 0.05 and np.ptp(U[-20:]) < 0.02 * U[-1]
    assert g.diagnostics()["nonfinite"] == 0
    free = Solver(prob)
    free.set_inflow(0, prof)
    free.step(120000)
    d = free.diagnostics()
    xf = prob.nx - d["sum_theta"] / (prob.n_fluid / prob.nx)
    say("  without holding (inlet at u_mean = 0.002): x_f %.3f" % xf)
    assert abs(xf - 128.0) > 10.0
