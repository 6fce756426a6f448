"""Curved walls: interpolated bounce-back on the links that cross the
analytic cylinders and spheres of the workloads (workloads.wall_links), and
Shepard-reconstructed image points of the finite-difference ghost nodes
inside them (workloads.image_points), through the C ABI against the FP64
oracle."""
import numpy as np
import pytest

from paper_2304_05657_amd import workloads as W

from .gpu_util import compare_fields, need_gpu, oracle_threads, say

pytestmark = pytest.mark.gpu
TOL64 = 1e-10


def _pair(prob, steps, checkpoints, precision="fp64", links=True, images=False):
    import oracle
    from paper_2304_05657_amd.lbfd import Solver
    need_gpu()
    g = Solver(prob, precision=precision)
    o = oracle.Oracle(prob, threads=oracle_threads())
    if links:
        cells, dirs, q = W.wall_links(prob)
        say("  %d wall links, q in [%.3g, %.3g]" % (len(q), q.min(), q.max()))
        g.set_wall_links(cells, dirs, q)
        # the GPU keeps q in single precision: the oracle gets the same values
        o.set_wall_links(cells, dirs, q.astype(np.float32).astype(np.float64))
    if images:
        cells, slots, im = W.image_points(prob)
        say("  %d ghost image points" % len(cells))
        g.set_image_points(cells, slots, im)
        o.set_image_points(cells, slots, im)
    done, errs = 0, []
    for target in checkpoints + [steps]:
        g.step(target - done)
        o.step(target - done)
        done = target
        e = compare_fields(g.fields(), o.fields(), prob)
        say("  level %d: %s" % (done, " ".join("%s=%.2e" % kv for kv in e.items())))
        errs.append((done, e))
    return g, o, errs


def test_burner_cylinders_fp64():
    prob = W.cylinder_burner(nx=512, ny=128, x_begin=128, x_end=384, front_x=256.0, name="walls_burner_512x128")
    say("case %s with interpolated bounce-back, 300 steps" % prob.name)
    _, _, errs = _pair(prob, 300, [1, 30])
    for level, e in errs:
        for k, v in e.items():
            assert v <= TOL64, (level, k, v)


def test_porous_spheres_fp64():
    prob = W.porous_3d(nx=48, ny=20, nz=18, porosity=0.85, radius=4.0, margin=8, seed=7,
                       name="walls_porous3d_48x20x18")
    say("case %s with interpolated bounce-back, 60 steps" % prob.name)
    _, _, errs = _pair(prob, 60, [1, 10])
    for level, e in errs:
        for k, v in e.items():
            assert v <= TOL64, (level, k, v)


def test_burner_cylinders_fp32():
    prob = W.cylinder_burner(nx=512, ny=128, x_begin=128, x_end=384, front_x=256.0, name="walls_burner_fp32")
    say("case %s with interpolated bounce-back, fp32, 300 steps" % prob.name)
    g, o, _ = _pair(prob, 300, [], precision="fp32")
    gf, of = g.fields(), o.fields()
    fl = prob.mask == 0
    eT = np.abs(gf["T"][fl] - of["T"][fl]).max() / (prob.T_b - prob.T_u)
    eu = np.abs(gf["u"][:2][:, fl] - of["u"][:2][:, fl]).max() / np.abs(of["u"][:2][:, fl]).max()
    say("  T_max_rel %.2e u_max_rel %.2e" % (eT, eu))
    assert eT < 1e-4 and eu < 5e-4


def test_links_validation_and_clear():
    """A link must run from a boundary fluid cell to a wall; clearing the
    links restores half-way bounce-back exactly."""
    from paper_2304_05657_amd.lbfd import LbfdError, Solver
    need_gpu()
    prob = W.cylinder_burner(nx=160, ny=64, x_begin=40, x_end=120, front_x=80.0, name="walls_validate")
    cells, dirs, q = W.wall_links(prob)
    s = Solver(prob)
    interior = [c for c in range(prob.N) if prob.mask.reshape(-1)[c] == 0 and c not in set(cells.tolist())]
    with pytest.raises(LbfdError):
        s.set_wall_links([interior[len(interior) // 2]], [4], [0.3])  # rest direction / no wall
    with pytest.raises(LbfdError):
        s.set_wall_links(cells[:1], dirs[:1], [1.5])
    a, b = Solver(prob), Solver(prob)
    b.set_wall_links(cells, dirs, q)
    b.set_wall_links()
    a.step(10)
    b.step(10)
    fa, fb = a.fields(), b.fields()
    for k in ("u", "T", "Ph"):
        assert np.array_equal(fa[k], fb[k]), k


def test_burner_image_points_fp64():
    prob = W.cylinder_burner(nx=512, ny=128, x_begin=128, x_end=384, front_x=256.0, name="images_burner_512x128")
    say("case %s with Shepard image points (and half-way bounce-back), 300 steps" % prob.name)
    _, _, errs = _pair(prob, 300, [1, 30], links=False, images=True)
    for level, e in errs:
        for k, v in e.items():
            assert v <= TOL64, (level, k, v)


def test_burner_curved_walls_fp64():
    prob = W.cylinder_burner(nx=512, ny=128, x_begin=128, x_end=384, front_x=256.0, name="curved_burner_512x128")
    say("case %s with interpolated bounce-back and image points, 300 steps" % prob.name)
    _, _, errs = _pair(prob, 300, [1], links=True, images=True)
    for level, e in errs:
        for k, v in e.items():
            assert v <= TOL64, (level, k, v)


def test_porous_curved_walls_fp64():
    prob = W.porous_3d(nx=48, ny=20, nz=18, porosity=0.85, radius=4.0, margin=8, seed=7,
                       name="curved_porous3d_48x20x18")
    say("case %s with interpolated bounce-back and image points, 60 steps" % prob.name)
    _, _, errs = _pair(prob, 60, [1, 10], links=True, images=True)
    for level, e in errs:
        for k, v in e.items():
            assert v <= TOL64, (level, k, v)


def test_porous_image_points_fp32():
    prob = W.porous_3d(nx=48, ny=20, nz=18, porosity=0.85, radius=4.0, margin=8, seed=7,
                       name="images_porous3d_fp32")
    say("case %s with image points, fp32, 60 steps" % prob.name)
    g, o, _ = _pair(prob, 60, [], precision="fp32", links=False, images=True)
    gf, of = g.fields(), o.fields()
    fl = prob.mask == 0
    eT = np.abs(gf["T"][fl] - of["T"][fl]).max() / (prob.T_b - prob.T_u)
    say("  T_max_rel %.2e" % eT)
    assert eT < 1e-4


def test_image_points_validation_and_clear():
    """An image point must belong to a ghost behind a wall, once, with a
    fluid node within four cells; clearing restores the axis mirror
    exactly."""
    from paper_2304_05657_amd.lbfd import LbfdError, Solver
    need_gpu()
    prob = W.cylinder_burner(nx=160, ny=64, x_begin=40, x_end=120, front_x=80.0, name="images_validate")
    cells, slots, im = W.image_points(prob)
    s = Solver(prob)
    listed = set(zip(cells.tolist(), slots.tolist()))
    # a fluid cell far from any wall: none of its stencil points is a ghost
    free = next(c for c in range(prob.N) if prob.mask.reshape(-1)[c] == 0
                and all((c, k) not in listed for k in range(8)) and 30 < c % prob.nx < 130
                and prob.mask.reshape(-1)[c - 2:c + 3].max() == 0)
    with pytest.raises(LbfdError):
        s.set_image_points([free], [1], [[free % prob.nx, free // prob.nx, 0.0]])
    with pytest.raises(LbfdError):
        s.set_image_points(np.r_[cells[:1], cells[:1]], np.r_[slots[:1], slots[:1]], np.r_[im[:1], im[:1]])
    with pytest.raises(LbfdError):
        s.set_image_points(cells[:1], [9], im[:1])
    a, b = Solver(prob), Solver(prob)
    b.set_image_points(cells, slots, im)
    b.set_image_points()
    a.step(10)
    b.step(10)
    fa, fb = a.fields(), b.fields()
    for k in ("u", "T", "Ph"):
        assert np.array_equal(fa[k], fb[k]), k
    # a rejected set leaves the previous one in place
    c, d = Solver(prob), Solver(prob)
    c.set_image_points(cells, slots, im)
    d.set_image_points(cells, slots, im)
    with pytest.raises(LbfdError):
        d.set_image_points(cells[:1], [9], im[:1])
    c.step(10)
    d.step(10)
    fc, fd = c.fields(), d.fields()
    for k in ("u", "T", "Ph"):
        assert np.array_equal(fc[k], fd[k]), k
    assert not np.array_equal(fc["T"], fa["T"])
