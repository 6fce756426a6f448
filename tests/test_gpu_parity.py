"""GPU parity: the HIP step (through the C ABI) against the FP64 oracle on
the same seeded inputs, element by element on every fluid cell.

FP64 bar: max relative error 1e-10 on u, T, Y_k (and rho, P_h), each
normalised by the field's largest magnitude over fluid cells.  The two
sides differ only by rounding order (fused multiply-adds, the factorised
central-moment transform against a Gaussian elimination, reassociated
WENO weights), i.e. ~1e-16 per operation.
"""
import numpy as np
import pytest

from paper_2304_05657_amd import workloads as W

from .gpu_util import compare_fields, need_gpu, oracle_threads, say

pytestmark = pytest.mark.gpu
TOL64 = 1e-10


def _run_pair(prob, steps, precision="fp64", checkpoints=None, check_every=0):
    import oracle
    from paper_2304_05657_amd.lbfd import Solver
    need_gpu()
    say("case %s %dx%dx%d Q%d %s steps=%d" % (prob.name, prob.nx, prob.ny, prob.nz, prob.lattice,
                                               precision, steps))
    g = Solver(prob, precision=precision, check_every=check_every)
    o = oracle.Oracle(prob, threads=oracle_threads())
    errs = []
    done = 0
    for target in (checkpoints or []) + [steps]:
        g.step(target - done)
        o.step(target - done)
        done = target
        e = compare_fields(g.fields(), o.fields(), prob)
        say("  level %d: %s" % (done, " ".join("%s=%.2e" % kv for kv in e.items())))
        errs.append((done, e))
    return g, o, errs


def _assert_tol(errs, tol):
    for level, e in errs:
        for k, v in e.items():
            assert v <= tol, (level, k, v)


def test_channel_flame_fp64_2000_steps():
    """2-D channel flame, D2Q9, 256x64, isothermal walls, 2000 steps."""
    prob = W.channel_flame()
    g, o, errs = _run_pair(prob, 2000, checkpoints=[1, 10, 200, 1000])
    _assert_tol(errs, TOL64)
    dg, do = g.diagnostics(), o.diagnostics()
    for k in ("sum_g", "sum_xi", "sum_theta", "wall_q", "fuel_rate"):
        assert abs(dg[k] - do[k]) <= 1e-10 * max(abs(do[k]), 1e-30), (k, dg[k], do[k])
    assert np.allclose(dg["mom"], do["mom"], rtol=0, atol=1e-10 * max(1.0, np.abs(do["mom"]).max()))
    assert dg["max_sumY_err"] < 1e-13 and dg["nonfinite"] == 0
    # the channel is mirror-symmetric in y: the largest heat release is a
    # tie between rows y and ny-1-y, so compare the value and accept either
    assert abs(dg["hrr_max"] - do["hrr_max"]) <= 1e-10 * abs(do["hrr_max"])
    ox, oy = do["hrr_idx"] % prob.nx, do["hrr_idx"] // prob.nx
    assert dg["hrr_idx"] in (do["hrr_idx"], (prob.ny - 1 - oy) * prob.nx + ox)


def test_channel_flame_adiabatic_ragged():
    """Adiabatic walls, ragged box (not a multiple of the 64x4 tile)."""
    prob = W.channel_flame(nx=70, ny=37, front_x=20.0, adiabatic=True, name="channel_adiabatic_70x37")
    _, _, errs = _run_pair(prob, 300, checkpoints=[1, 50])
    _assert_tol(errs, TOL64)


def test_wall_faces_and_thin_gaps():
    """Isothermal and adiabatic wall faces instead of mask rows, an obstacle
    with one-cell fluid gaps (ghost image clamping)."""
    prob = W.channel_flame(nx=48, ny=20, front_x=16.0, name="faces_gaps_48x20")
    prob.mask[:] = 0
    prob.mask[0, 5:15, 20] = 1
    prob.mask[0, 5:15, 22] = 2
    prob.mask[0, 10, 30:33] = 1
    prob.wall_T[0, 5:15, 20] = 500.0
    prob = prob.replace(faces=("periodic", "periodic", "wall", "wall_adiabatic", "periodic", "periodic"),
                        face_T=(300.0, 300.0, 350.0, 300.0, 300.0, 300.0))
    _, _, errs = _run_pair(prob, 200, checkpoints=[1, 20])
    _assert_tol(errs, TOL64)


def test_burner_inflow_outflow_fp64():
    """Pseudo 2-D burner (cylinders, inflow at -x, outflow at +x), scaled
    down to 512x128 so that the oracle finishes in seconds."""
    prob = W.cylinder_burner(nx=512, ny=128, x_begin=128, x_end=384, front_x=256.0,
                             name="cylinder_burner_512x128")
    _, _, errs = _run_pair(prob, 300, checkpoints=[1, 30])
    _assert_tol(errs, TOL64)


def test_burner_full_size_500_steps():
    """The 2048x512 burner at full size, in the launch configuration the
    benchmark times: all fields over the first 500 steps (and the level-0
    moments)."""
    prob = W.cylinder_burner()
    _, _, errs = _run_pair(prob, 500, checkpoints=[0, 1, 100])
    _assert_tol(errs, TOL64)


def test_channel_1024x256_500_steps():
    """The 1024x256 channel flame of the gradient runs, forward step only."""
    prob = W.named("channel_adjoint")
    _, _, errs = _run_pair(prob, 500, checkpoints=[1, 50])
    _assert_tol(errs, TOL64)


def test_porous_3d_fp64():
    """D3Q27 random sphere packing with inflow/outflow, 4 species."""
    prob = W.porous_3d(nx=48, ny=20, nz=18, porosity=0.85, radius=4.0, margin=8, seed=7,
                       name="porous3d_48x20x18")
    _, _, errs = _run_pair(prob, 60, checkpoints=[1, 10])
    _assert_tol(errs, TOL64)


def test_porous_3d_mechanism_fp64():
    """D3Q27, 9 species / 20 reactions, sub-cycled FP64 source."""
    prob = W.porous_3d_mech(nx=32, ny=12, nz=12, porosity=0.9, radius=(2.0, 4.0), margin=6,
                            name="porous3d_mech_32x12x12")
    _, _, errs = _run_pair(prob, 40, checkpoints=[1, 10])
    _assert_tol(errs, TOL64)


def test_porous_3d_fp64_500_steps():
    """A longer 3-D horizon: D3Q27 packing 64x32x32 (58,029 fluid cells),
    inflow / outflow, 4 species, 500 FP64 steps with the reductions every
    10 steps, compared at levels 1, 100 and 500."""
    prob = W.porous_3d(nx=64, ny=32, nz=32, porosity=0.85, radius=4.0, margin=8, seed=11,
                       name="porous3d_64x32x32")
    _, _, errs = _run_pair(prob, 500, checkpoints=[1, 100], check_every=10)
    _assert_tol(errs, TOL64)


def test_porous_3d_mechanism_fp64_400_steps():
    """A longer horizon of the stiff mechanism: 9 species / 20 reactions with
    temperature exponents and sub-cycled FP64 sources, 400 steps, compared at
    levels 1, 40, 200 and 400."""
    prob = W.porous_3d_mech(nx=32, ny=12, nz=12, porosity=0.9, radius=(2.0, 4.0), margin=6,
                            name="porous3d_mech_32x12x12")
    _, _, errs = _run_pair(prob, 400, checkpoints=[1, 40, 200], check_every=10)
    _assert_tol(errs, TOL64)


def test_closed_3d_budget_and_diagnostics():
    """D3Q27 closed periodic box with a sphere: GPU diagnostics equal the
    oracle's and the population budget closes."""
    from paper_2304_05657_amd.lbfd import Solver
    import oracle
    need_gpu()
    prob = W.porous_3d(20, 12, 12, porosity=0.95, radius=3.0, margin=4, front_x=10.0, name="closed3d")
    prob = prob.replace(faces=("periodic",) * 6)
    say("case closed3d diagnostics")
    g = Solver(prob)
    o = oracle.Oracle(prob, threads=oracle_threads())
    g.step(5)
    o.step(5)
    d0 = g.diagnostics()
    od = o.diagnostics()
    for k in ("sum_g", "sum_xi", "sum_theta", "wall_q", "fuel_rate"):
        assert abs(d0[k] - od[k]) <= 1e-10 * max(abs(od[k]), 1e-30), (k, d0[k], od[k])
    g.step(1)
    d1 = g.diagnostics()
    assert abs(d1["sum_g"] - d0["sum_g"] - d0["sum_xi"]) <= 1e-12 * (abs(d0["sum_g"]) + abs(d0["sum_xi"]))


def test_restart_is_bitwise_and_deterministic():
    """Checkpoint/restore resumes bit for bit; two runs are identical."""
    from paper_2304_05657_amd.lbfd import Solver
    need_gpu()
    prob = W.cylinder_burner(nx=256, ny=128, x_begin=64, x_end=192, front_x=128.0, name="burner_256x128")
    say("case restart burner_256x128")
    a = Solver(prob)
    a.step(20)
    blob = a.save_state()
    a.step(15)
    fa = a.fields()
    b = Solver(prob)
    b.load_state(blob)
    assert b.level == 20
    b.step(15)
    fb = b.fields()
    c = Solver(prob)
    c.step(35)
    fc = c.fields()
    for k in ("u", "T", "Y", "Ph"):
        assert np.array_equal(fa[k], fb[k]), k
        assert np.array_equal(fa[k], fc[k]), k


def test_nonfinite_check_reports():
    """A NaN planted in a restored state is reported by lbfd_sync."""
    from paper_2304_05657_amd.lbfd import LbfdError, Solver
    need_gpu()
    prob = W.channel_flame(nx=64, ny=16, front_x=20.0, name="nan_probe")
    say("case nonfinite check")
    s = Solver(prob, check_every=1)
    blob = bytearray(s.save_state())
    # header (64 bytes), then populations, then T: plant NaN in T of cell (5, 5)
    hdr = 64
    pop_bytes = 9 * prob.N * 8
    off = hdr + pop_bytes + (5 * prob.nx + 5) * 8
    blob[off:off + 8] = np.array([np.nan]).tobytes()
    s.load_state(bytes(blob))
    s.step(3)
    with pytest.raises(LbfdError) as ei:
        s.sync()
    assert ei.value.code == -4
