"""Degenerate and ragged boxes through the C ABI against the FP64 oracle:
fully periodic boxes without any solid (2-D and 3-D; the cells within two
of a face take the descriptor path, which wraps), no interior cell at all
(every fluid cell next to a wall), and 3-D boxes that fill neither the
64 x 2 x 2 tiles nor the boundary blocks."""
import numpy as np
import pytest

from paper_2304_05657_amd import workloads as W

from .gpu_util import compare_fields, need_gpu, oracle_threads, say

pytestmark = pytest.mark.gpu
TOL64 = 1e-10


def _periodic(nx, ny, nz, lattice, seed):
    """Fully periodic box at rest with smooth T and Y modes and a slow
    one-step reaction, no solid."""
    rng = np.random.default_rng(seed)
    shape = (nz, ny, nx)
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    th = 2 * np.pi * (x / nx + y / ny + (z / nz if nz > 1 else 0.0))
    T = 900.0 + 300.0 * np.sin(th + rng.uniform(0, 6))
    yf = 0.04 + 0.01 * np.cos(th)
    Y0 = np.stack([yf, np.full(shape, 0.2), np.zeros(shape), 0.8 - yf])
    base = W.channel_flame(nx=8, ny=8, front_x=4.0, name="tmp")
    return base.replace(name="periodic_%dx%dx%d_q%d" % (nx, ny, nz, lattice), lattice=lattice, nx=nx, ny=ny,
                        nz=nz, faces=("periodic",) * 6, mask=np.zeros(shape, np.uint8),
                        wall_T=np.full(shape, 300.0), T0=T, Y0=Y0, u0=None, Ph0=None)


def _run(prob, steps, checkpoints=()):
    import oracle
    from paper_2304_05657_amd.lbfd import Solver
    need_gpu()
    g = Solver(prob)
    o = oracle.Oracle(prob, threads=oracle_threads())
    nf, nb = g.cell_counts()
    say("case %s: %d fluid cells, %d on the boundary path" % (prob.name, nf, nb))
    done = 0
    for target in list(checkpoints) + [steps]:
        g.step(target - done)
        o.step(target - done)
        done = target
        e = compare_fields(g.fields(), o.fields(), prob)
        say("  level %d: %s" % (done, " ".join("%s=%.2e" % kv for kv in e.items())))
        for k, v in e.items():
            assert v <= TOL64, (done, k, v)
    return nf, nb


def test_periodic_2d_without_solids():
    nf, nb = _run(_periodic(70, 9, 1, 9, 1), 200, [1])
    assert nf == 70 * 9 and nb == nf - 66 * 5   # all but the cells two or more from every face


def test_periodic_3d_without_solids():
    nf, nb = _run(_periodic(37, 11, 9, 27, 2), 60, [1])
    assert nf == 37 * 11 * 9 and nb == nf - 33 * 7 * 5


def test_channel_without_interior_cell():
    """Two fluid rows between solid rows: every fluid cell has a wall within
    two cells, so the interior tiles have nothing to do."""
    prob = W.channel_flame(nx=40, ny=4, front_x=12.0, name="channel_40x4")
    nf, nb = _run(prob, 200, [1])
    assert nb == nf == 80


def test_ragged_3d_packing():
    prob = W.porous_3d(nx=37, ny=11, nz=9, porosity=0.9, radius=2.5, margin=6, seed=5, name="porous_37x11x9")
    _run(prob, 60, [1])
