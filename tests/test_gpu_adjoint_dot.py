"""One step's reverse sweep against its forward-mode linearisation: for
random tangents dx of every input block (populations, T and Y, wall
temperatures, Arrhenius A and Ta) and random adjoints lam of every output
block (populations, T and Y, the level's objective term q), the identity
<J dx, lam> = <dx, J^T lam> between lbfd_step_tangent (dual numbers, cell by
cell) and lbfd_step_adjoint (the hand-derived reverse of the cell update,
lbfd_adjoint's backward step) holds to 1e-12 relative, block by block, so
that a missing or mis-signed term of any one path shows.

Cases: a D2Q9 channel flame with isothermal walls (wall heat flux and flame
position objectives), a D2Q9 inflow channel (inflow ghosts, an isothermal
+x face, a temperature exponent b = 0.7 and sub-stepped chemistry) and a
closed D3Q27 porous box."""
import numpy as np
import pytest

from paper_2304_05657_amd import workloads as W

from .gpu_util import need_gpu, say

pytestmark = pytest.mark.gpu
TOL = 1e-12


def _blocks_in(rng, prob, Q, N, nsp):
    fluid = (prob.mask.ravel() == 0)
    nrx = len(prob.reactions)
    A = np.array([r.A for r in prob.reactions])
    Ta = np.array([r.Ta for r in prob.reactions])
    pop = rng.standard_normal((Q, N)) * fluid
    sc = rng.standard_normal((1 + nsp, N)) * fluid
    sc[0] *= 10.0  # T is O(100-2000) K, Y is O(1)
    wall = rng.standard_normal(N) * (prob.mask.ravel() == 1)
    z = lambda *s: np.zeros(s)
    return {
        "pop": (pop, z(1 + nsp, N), None, None, None),
        "scalars": (z(Q, N), sc, None, None, None),
        "wall_T": (z(Q, N), z(1 + nsp, N), wall, None, None),
        "A": (z(Q, N), z(1 + nsp, N), None, A * rng.standard_normal(nrx), None),
        "Ta": (z(Q, N), z(1 + nsp, N), None, None, Ta * rng.standard_normal(nrx)),
    }


def _dot_case(prob, objective, warm, seed):
    from paper_2304_05657_amd.lbfd import Solver
    need_gpu()
    s = Solver(prob)
    s.set_objective(objective)
    s.step(warm)
    Q, N, nsp = prob.lattice, s.N, prob.n_species
    rng = np.random.default_rng(seed)
    fluid = (prob.mask.ravel() == 0)
    lam_blocks = {
        "pop": (rng.standard_normal((Q, N)) * fluid, np.zeros((1 + nsp, N)), 0.0),
        "scalars": (np.zeros((Q, N)), rng.standard_normal((1 + nsp, N)) * fluid, 0.0),
        "q": (np.zeros((Q, N)), np.zeros((1 + nsp, N)), float(rng.standard_normal())),
    }
    adj = {k: s.step_adjoint(*v) for k, v in lam_blocks.items()}
    for v in adj.values():
        assert all(np.all(np.isfinite(a)) for a in v)
    level = s.level
    worst = 0.0
    for name, (dp, ds, dw, dA, dTa) in _blocks_in(rng, prob, Q, N, nsp).items():
        po, so, dq = s.step_tangent(dp, ds, dw, dA, dTa)
        assert np.all(np.isfinite(po)) and np.all(np.isfinite(so)) and np.isfinite(dq)
        for lname, (lp, ls, wq) in lam_blocks.items():
            lhs = float((po * lp).sum() + (so * ls).sum() + wq * dq)
            gp, gs, gW, gA, gTa = adj[lname]
            rhs = float((dp * gp).sum() + (ds * gs).sum())
            if dw is not None:
                rhs += float((dw * gW).sum())
            if dA is not None:
                rhs += float(dA @ gA)
            if dTa is not None:
                rhs += float(dTa @ gTa)
            scale = max(abs(lhs), abs(rhs))
            err = abs(lhs - rhs) / scale if scale > 0 else 0.0
            say("  dx %-8s lam %-8s <J dx, lam> %+.15e <dx, J^T lam> %+.15e rel %.1e" % (name, lname, lhs, rhs, err))
            worst = max(worst, err)
            assert err <= TOL, (name, lname, lhs, rhs)
    assert s.level == level  # neither call advances the context
    return worst


def test_dot_product_channel_wall_heat_flux():
    prob = W.channel_flame(nx=64, ny=16, front_x=20.0, name="dot_channel_64x16")
    say("case dot product, channel 64x16 after 30 steps, wall heat flux")
    _dot_case(prob, "wall_q", 30, seed=11)


def test_dot_product_channel_flame_position():
    prob = W.channel_flame(nx=64, ny=16, front_x=20.0, name="dot_channel_flame_64x16")
    say("case dot product, channel 64x16 after 30 steps, flame position")
    _dot_case(prob, "flame_x", 30, seed=12)


def test_dot_product_channel_limiter_regime():
    """After 300 steps the reactants diffused into the burnt gas are tiny
    negative numbers (~ -1e-150) at some cells: the positivity limiter then
    takes a zero scale, and its derivative divides by a subnormal rate."""
    from paper_2304_05657_amd.lbfd import Solver
    prob = W.channel_flame(nx=256, ny=64, front_x=32.0, name="dot_channel_256x64")
    say("case dot product, channel 256x64 after 300 steps (limiter regime)")
    s = Solver(prob)
    s.step(300)
    Y = s.fields()["Y"][:2][:, prob.mask == 0]
    say("  reactant mass fractions below zero at %d cells" % int((Y < 0).sum()))
    assert (Y < 0).any()
    s.close()
    _dot_case(prob, "wall_q", 300, seed=15)


def test_dot_product_inflow_channel_b_substeps():
    base = W.flame_channel(nx=48, ny=14, u_mean=0.004, front_x=24.0, adiabatic=False, name="dot_inflow_48x14")
    r = base.reactions[0]
    prob = base.replace(faces=("inflow", "wall", "periodic", "periodic", "periodic", "periodic"),
                        reactions=[W.Reaction(r.reactants, r.A * 300.0 ** -0.7, 0.7, r.Ta, r.nu, r.q)],
                        chem_substeps_max=8)
    say("case dot product, inflow channel 48x14 (b = 0.7, up to 8 sub-steps) after 20 steps")
    _dot_case(prob, "wall_q", 20, seed=13)


def test_dot_product_3d_closed_box():
    prob = W.porous_3d(nx=20, ny=10, nz=10, porosity=0.9, radius=3.0, margin=4, front_x=10.0, name="dot_porous")
    prob = prob.replace(faces=("periodic",) * 6)
    say("case dot product, D3Q27 closed porous 20x10x10 after 8 steps")
    _dot_case(prob, "wall_q", 8, seed=14)
