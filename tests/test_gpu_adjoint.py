"""Discrete adjoint of the FP64 step: gradients of the time-integrated wall
heat flux J (and of the flame position summed over a window of levels)
with respect to the wall temperature field and the Arrhenius A, Ta,
checked against central finite differences of the GPU forward (eps = 1e-6
relative, FP64), against fourth-order central differences of the oracle
(CPU reference gradient, 1e-8 relative plus a round-off floor), and through
torch.autograd.  The one-step identity <J dx, lam> = <dx, J^T lam> is
checked in test_gpu_adjoint_dot.py.

Tolerance: 1e-5 relative (central differences carry O(eps^2) truncation and
~1e-16 J / eps round-off, i.e. < 1e-8 here; the adjoint differs from the
forward kernels only by rounding)."""
import numpy as np
import pytest

from paper_2304_05657_amd import workloads as W

from .gpu_util import need_gpu, oracle_threads, say

pytestmark = pytest.mark.gpu
RTOL = 1e-5


def _fd_params(s, state, prob, nsteps, eps=1e-6):
    r = prob.reactions[0]
    out = []
    for which in ("A", "Ta"):
        vals = []
        for sg in (1, -1):
            s.load_state(state)
            A = r.A * (1 + sg * eps) if which == "A" else r.A
            Ta = r.Ta * (1 + sg * eps) if which == "Ta" else r.Ta
            s.set_reaction(0, A, r.b, Ta)
            vals.append(s.objective(nsteps))
        h = (r.A if which == "A" else r.Ta) * eps
        out.append((vals[0] - vals[1]) / (2 * h))
    s.set_reaction(0, r.A, r.b, r.Ta)
    return out


def _fd_wall(s, state, prob, nsteps, direction, eps_T):
    vals = []
    for sg in (1, -1):
        s.load_state(state)
        s.set_wall_temperature(prob.wall_T + sg * eps_T * direction)
        vals.append(s.objective(nsteps))
    s.set_wall_temperature(prob.wall_T)
    return (vals[0] - vals[1]) / (2 * eps_T)


def _rel(a, b):
    return abs(a - b) / max(abs(b), 1e-300)


def _check_case(prob, nsteps, K, n_cells, n_dirs, seed, objective=("wall_q", 0, None), eps_T=3e-4):
    from paper_2304_05657_amd.lbfd import Solver
    need_gpu()
    s = Solver(prob)
    s.set_objective(*objective)
    state = s.save_state()
    import time
    t0 = time.perf_counter()
    J, gW, gA, gTa = s.adjoint(nsteps, K)
    t_adj = time.perf_counter() - t0
    s.load_state(state)
    J2 = s.objective(nsteps)
    say("  J=%.12e (forward %.12e), adjoint %.2f s" % (J, J2, t_adj))
    assert _rel(J, J2) < 1e-12
    # eps = 1e-6: the FD numerator J(+) - J(-) can be as small as 1e-11 |J|,
    # where the round-off of J (~1e-15 |J| per evaluation) is a 1e-4-level
    # noise; the bound adds that floor.  eps = 1e-4 lowers the floor 100x
    # (truncation O(eps^2) ~ 1e-8) and is held to RTOL alone.
    r = prob.reactions[0]
    for eps in (1e-6, 1e-4):
        fA, fTa = _fd_params(s, state, prob, nsteps, eps)
        say("  eps %.0e: dJ/dA adjoint %.10e fd %.10e rel %.2e" % (eps, gA[0], fA, _rel(gA[0], fA)))
        say("  eps %.0e: dJ/dTa adjoint %.10e fd %.10e rel %.2e" % (eps, gTa[0], fTa, _rel(gTa[0], fTa)))
        floor_A = 4e-15 * abs(J) / (2 * r.A * eps) if eps < 1e-5 else 0.0
        floor_Ta = 4e-15 * abs(J) / (2 * r.Ta * eps) if eps < 1e-5 else 0.0
        assert abs(gA[0] - fA) <= RTOL * abs(fA) + floor_A
        assert abs(gTa[0] - fTa) <= RTOL * abs(fTa) + floor_Ta
    rng = np.random.default_rng(seed)
    walls = np.argwhere(prob.mask == 1)
    nz = [tuple(w) for w in walls if abs(gW[tuple(w)]) > 1e-3 * np.abs(gW).max()]
    pick = [nz[i] for i in rng.choice(len(nz), size=min(n_cells, len(nz)), replace=False)]
    # round-off floor of a wall-temperature difference quotient
    floor_W = 4e-15 * abs(J) / (2 * eps_T)
    for w in pick:
        d = np.zeros_like(prob.wall_T)
        d[w] = 1.0
        fd = _fd_wall(s, state, prob, nsteps, d, eps_T)
        say("  dJ/dTw%s adjoint %.10e fd %.10e rel %.2e" % (w, gW[w], fd, _rel(gW[w], fd)))
        assert abs(gW[w] - fd) <= RTOL * abs(fd) + floor_W
    for _ in range(n_dirs):
        d = np.where(prob.mask == 1, rng.normal(size=prob.wall_T.shape), 0.0)
        fd = _fd_wall(s, state, prob, nsteps, d, eps_T)
        ad = float((gW * d).sum())
        # a random direction sums hundreds of terms of both signs: compare
        # relative to the magnitude of the summed terms
        scale = float(np.abs(gW * d).sum())
        say("  direction: adjoint %.10e fd %.10e diff/sum|terms| %.2e" % (ad, fd, abs(ad - fd) / scale))
        assert abs(ad - fd) < RTOL * scale + floor_W
    # only isothermal wall cells carry a gradient
    assert np.all(gW[prob.mask != 1] == 0.0)
    return J, gW, gA, gTa


def test_adjoint_small_channel_vs_gpu_fd():
    prob = W.channel_flame(nx=96, ny=24, front_x=30.0, name="adj_channel_96x24")
    say("case adjoint channel 96x24, 40 steps, K=8")
    _check_case(prob, 40, 8, 4, 2, seed=1)


def test_adjoint_3d_vs_gpu_fd():
    prob = W.porous_3d(nx=24, ny=12, nz=12, porosity=0.9, radius=3.0, margin=4, front_x=12.0, name="adj_porous")
    prob = prob.replace(faces=("periodic",) * 6)
    say("case adjoint D3Q27 closed porous 24x12x12, 12 steps, K=5")
    _check_case(prob, 12, 5, 3, 1, seed=2)


def _richardson(f, p, h):
    """Fourth-order central difference of f at p: (4 D(h/2) - D(h)) / 3 with
    D(h) = (f(p + h) - f(p - h)) / (2 h); truncation O(h^4)."""
    D = lambda hh: (f(p + hh) - f(p - hh)) / (2 * hh)
    return (4 * D(h / 2) - D(h)) / 3


# Gradient against the oracle: 1e-8 relative plus a round-off floor.  With
# the oracle's J carrying a relative error below 1e-15 per evaluation
# (|dJ| <= 1e-15 |J|), the noise of the fourth-order difference is at most
# (4 * 2 dJ / h + 2 dJ / (2 h)) / 3 = 3 dJ / h.
ORACLE_RTOL = 1e-8


def _oracle_floor(J, h):
    return 3e-15 * abs(J) / h


def test_adjoint_vs_oracle_reference_gradient():
    """CPU reference gradient: fourth-order central differences of the
    oracle's J, held to 1e-8 relative plus the stated round-off floor.
    Steps: 3e-2 A and 1e-3 Ta (the differences at these and at 3x smaller
    steps agree to < 1e-8); 3e-4 K for one wall cell, where the WENO3
    weights (eps = 1e-6) of the nearly uniform cold gas next to the wall
    change over temperature differences of ~sqrt(eps) = 1e-3 K, so larger
    steps do not converge and the floor (~4e-7 of the derivative) bounds
    the check."""
    import oracle
    from paper_2304_05657_amd.lbfd import Solver
    need_gpu()
    prob = W.channel_flame(nx=64, ny=16, front_x=20.0, name="adj_channel_64x16")
    nsteps, K = 30, 7
    say("case adjoint vs oracle, channel 64x16, %d steps, K=%d" % (nsteps, K))
    s = Solver(prob)
    J, gW, gA, gTa = s.adjoint(nsteps, K)
    Jo = oracle.Oracle(prob, threads=oracle_threads()).objective(nsteps)
    assert _rel(J, Jo) < 1e-10, (J, Jo)
    r = prob.reactions[0]
    w = (0, 0, 40)

    def oJ(A=r.A, Ta=r.Ta, dTw=0.0):
        wt = prob.wall_T.copy()
        wt[w] += dTw
        p = prob.replace(reactions=[W.Reaction(r.reactants, A, r.b, Ta, r.nu, r.q)], wall_T=wt)
        return oracle.Oracle(p, threads=oracle_threads()).objective(nsteps)

    hA, hTa, hW = 3e-2 * r.A, 1e-3 * r.Ta, 3e-4
    fA = _richardson(lambda v: oJ(A=v), r.A, hA)
    fTa = _richardson(lambda v: oJ(Ta=v), r.Ta, hTa)
    fW = _richardson(lambda v: oJ(dTw=v), 0.0, hW)
    say("  A: gpu adjoint %.12e oracle fd %.12e rel %.1e; Ta: %.12e / %.12e rel %.1e; Tw%s: %.12e / %.12e rel %.1e" % (
        gA[0], fA, _rel(gA[0], fA), gTa[0], fTa, _rel(gTa[0], fTa), w, gW[w], fW, _rel(gW[w], fW)))
    assert abs(gA[0] - fA) <= ORACLE_RTOL * abs(fA) + _oracle_floor(J, hA)
    assert abs(gTa[0] - fTa) <= ORACLE_RTOL * abs(fTa) + _oracle_floor(J, hTa)
    assert abs(gW[w] - fW) <= ORACLE_RTOL * abs(fW) + _oracle_floor(J, hW)


def test_autograd_function():
    import torch
    from paper_2304_05657_amd.lbfd import Solver, wall_heat_flux_objective
    need_gpu()
    prob = W.channel_flame(nx=64, ny=16, front_x=20.0, name="adj_autograd")
    say("case adjoint through torch.autograd")
    s = Solver(prob)
    state = s.save_state()
    wT = torch.tensor(prob.wall_T, dtype=torch.float32, requires_grad=True)
    A = torch.tensor(prob.reactions[0].A, dtype=torch.float64, requires_grad=True)
    Ta = torch.tensor(prob.reactions[0].Ta, dtype=torch.float64, requires_grad=True)
    J = wall_heat_flux_objective(s, state, 20, 6, wT, A, Ta)
    J.backward()
    s.load_state(state)
    J2, gW, gA, gTa = s.adjoint(20, 6)
    assert abs(J.item() - J2) <= 1e-12 * abs(J2)
    assert abs(A.grad.item() - gA[0]) <= 1e-12 * abs(gA[0])
    assert abs(Ta.grad.item() - gTa[0]) <= 1e-12 * abs(gTa[0])
    assert np.allclose(wT.grad.numpy(), gW.astype(np.float32), rtol=1e-6, atol=0)


def test_adjoint_channel_1024x256_500_steps():
    """The differentiation workload: channel 1024x256, 500 steps, K = 25;
    FD checks on A, Ta, 8 random wall cells and 4 random directions."""
    prob = W.named("channel_adjoint")
    say("case adjoint channel 1024x256, 500 steps, K=25")
    _check_case(prob, 500, 25, 8, 4, seed=3)


def test_adjoint_flame_position_window_vs_gpu_fd():
    """Objective: the flame position summed over levels 10..39 of 40."""
    prob = W.channel_flame(nx=96, ny=24, front_x=30.0, name="adj_flame_96x24")
    say("case adjoint flame position, channel 96x24, levels [10, 40) of 40, K=8")
    _check_case(prob, 40, 8, 4, 2, seed=4, objective=("flame_x", 10, 40), eps_T=1e-3)


def test_adjoint_flame_position_vs_oracle():
    """Flame-position objective over a window: J equals the oracle's, and the
    gradient equals fourth-order central differences of the oracle's J to
    1e-8 relative plus the round-off floor."""
    import oracle
    from paper_2304_05657_amd.lbfd import Solver
    need_gpu()
    prob = W.channel_flame(nx=64, ny=16, front_x=20.0, name="adj_flame_64x16")
    nsteps, K, win = 30, 7, (5, 25)
    say("case adjoint flame position vs oracle, channel 64x16, %d steps, window %s" % (nsteps, win))
    s = Solver(prob)
    s.set_objective("flame_x", *win)
    J, gW, gA, gTa = s.adjoint(nsteps, K)
    r = prob.reactions[0]

    def oJ(A=r.A, Ta=r.Ta):
        p = prob.replace(reactions=[W.Reaction(r.reactants, A, r.b, Ta, r.nu, r.q)])
        return oracle.Oracle(p, threads=oracle_threads()).objective(nsteps, "flame_x", *win)

    Jo = oJ()
    assert _rel(J, Jo) < 1e-10, (J, Jo)
    hA, hTa = 3e-2 * r.A, 1e-3 * r.Ta
    fA = _richardson(lambda v: oJ(A=v), r.A, hA)
    fTa = _richardson(lambda v: oJ(Ta=v), r.Ta, hTa)
    say("  J %.12e oracle %.12e; A: gpu adjoint %.12e oracle fd %.12e rel %.1e; Ta: %.12e / %.12e rel %.1e" % (
        J, Jo, gA[0], fA, _rel(gA[0], fA), gTa[0], fTa, _rel(gTa[0], fTa)))
    assert abs(gA[0] - fA) <= ORACLE_RTOL * abs(fA) + _oracle_floor(J, hA)
    assert abs(gTa[0] - fTa) <= ORACLE_RTOL * abs(fTa) + _oracle_floor(J, hTa)


def test_objective_on_non_default_stream():
    """lbfd_objective and lbfd_objective_static on a context whose stream is
    a non-default torch stream, busy with earlier work when the objective is
    queued: J equals that of a context on the null stream (the entry points
    wait for their stream before reading J)."""
    import torch
    from paper_2304_05657_amd.lbfd import Solver
    need_gpu()
    prob = W.channel_flame(nx=96, ny=24, front_x=30.0, name="stream_channel_96x24")
    say("case objective on a non-default stream, channel 96x24, 40 steps")
    ref = Solver(prob, stream=0)
    state = ref.save_state()
    J0 = ref.objective(40)
    side = torch.cuda.Stream()
    with torch.cuda.stream(side):
        s = Solver(prob)  # takes torch's current stream
        s.load_state(state)
        x = torch.randn(4096, 4096, device="cuda")
        for _ in range(4):
            x = x @ x / 64.0  # earlier work queued on the same stream
        J1 = s.objective(40)
        s.load_state(state)
        for _ in range(4):
            x = x @ x / 64.0
        J2 = s.objective_static(40)
    torch.cuda.synchronize()
    say("  J null stream %.15e, side stream %.15e, static %.15e" % (J0, J1, J2))
    assert J1 == J0 and J2 == J0
