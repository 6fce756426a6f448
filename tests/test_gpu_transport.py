"""Mixture-averaged species transport (non-unity Lewis numbers, species
heat capacities; Eq. 2 with the correction velocity, Eq. 7 with the species
enthalpy flux) through the C ABI against the FP64 oracle."""
import numpy as np
import pytest

from paper_2304_05657_amd import workloads as W

from .gpu_util import compare_fields, need_gpu, oracle_threads, say

pytestmark = pytest.mark.gpu
TOL64 = 1e-10
LE4 = (0.8, 1.1, 1.4, 1.0)      # synthetic Lewis numbers of F, O, P, N
CP4 = (2.0, 0.9, 1.3, 1.0)      # synthetic c_pk / c_p,ref


def _pair(prob, steps, checkpoints, precision="fp64"):
    import oracle
    from paper_2304_05657_amd.lbfd import Solver
    need_gpu()
    g = Solver(prob, precision=precision)
    o = oracle.Oracle(prob, threads=oracle_threads())
    done, errs = 0, []
    for target in checkpoints + [steps]:
        g.step(target - done)
        o.step(target - done)
        done = target
        e = compare_fields(g.fields(), o.fields(), prob)
        say("  level %d: %s" % (done, " ".join("%s=%.2e" % kv for kv in e.items())))
        errs.append((done, e))
    return g, o, errs


def _check(errs, tol=TOL64):
    for level, e in errs:
        for k, v in e.items():
            assert v <= tol, (level, k, v)


def test_burner_mixture_fp64():
    prob = W.cylinder_burner(nx=512, ny=128, x_begin=128, x_end=384, front_x=256.0, name="mix_burner_512x128")
    prob = prob.replace(transport="mixture_averaged", lewis=LE4, cp=CP4)
    say("case %s, mixture-averaged transport, 300 steps" % prob.name)
    _check(_pair(prob, 300, [1, 30])[2])


def test_burner_mixture_curved_walls_fp64():
    import oracle
    from paper_2304_05657_amd.lbfd import Solver
    need_gpu()
    prob = W.cylinder_burner(nx=512, ny=128, x_begin=128, x_end=384, front_x=256.0, name="mix_curved_512x128")
    prob = prob.replace(transport="mixture_averaged", lewis=LE4, cp=CP4)
    say("case %s, mixture-averaged transport with curved walls, 200 steps" % prob.name)
    g = Solver(prob)
    o = oracle.Oracle(prob, threads=oracle_threads())
    cells, dirs, q = W.wall_links(prob)
    g.set_wall_links(cells, dirs, q)
    o.set_wall_links(cells, dirs, q.astype(np.float32).astype(np.float64))
    c, sl, im = W.image_points(prob)
    g.set_image_points(c, sl, im)
    o.set_image_points(c, sl, im)
    g.step(200)
    o.step(200)
    e = compare_fields(g.fields(), o.fields(), prob)
    say("  level 200: %s" % " ".join("%s=%.2e" % kv for kv in e.items()))
    _check([(200, e)])


def test_porous_mixture_fp64():
    prob = W.porous_3d(nx=48, ny=20, nz=18, porosity=0.85, radius=4.0, margin=8, seed=7, name="mix_porous3d")
    prob = prob.replace(transport="mixture_averaged", lewis=LE4, cp=CP4)
    say("case %s, mixture-averaged transport, 60 steps" % prob.name)
    _check(_pair(prob, 60, [1, 10])[2])


def test_porous_mechanism_mixture_fp64():
    """Nine species, twenty stiff reactions with sub-stepping: the heat
    release divided by the sub-step's c_p."""
    prob = W.porous_3d_mech(nx=32, ny=12, nz=12, porosity=0.9, radius=(2.0, 4.0), margin=6, steps=30,
                            name="mix_mech3d")
    rng = np.random.default_rng(11)
    ns = prob.n_species
    prob = prob.replace(transport="mixture_averaged", lewis=tuple(rng.uniform(0.7, 1.6, ns)),
                        cp=tuple(rng.uniform(0.8, 2.2, ns)))
    say("case %s (%d species), mixture-averaged transport, 30 steps" % (prob.name, ns))
    _check(_pair(prob, 30, [1])[2])


def test_burner_mixture_fp32():
    prob = W.cylinder_burner(nx=512, ny=128, x_begin=128, x_end=384, front_x=256.0, name="mix_burner_fp32")
    prob = prob.replace(transport="mixture_averaged", lewis=LE4, cp=CP4)
    say("case %s, mixture-averaged transport, fp32, 300 steps" % prob.name)
    g, o, _ = _pair(prob, 300, [], precision="fp32")
    gf, of = g.fields(), o.fields()
    fl = prob.mask == 0
    eT = np.abs(gf["T"][fl] - of["T"][fl]).max() / (prob.T_b - prob.T_u)
    eY = np.abs(gf["Y"][:, fl] - of["Y"][:, fl]).max()
    say("  T_max_rel %.2e Y_max %.2e" % (eT, eY))
    assert eT < 1e-4 and eY < 1e-5
    s = gf["Y"][:, fl].sum(axis=0)
    assert np.abs(s - 1.0).max() < 1e-5


def test_adjoint_rejects_mixture_transport():
    from paper_2304_05657_amd.lbfd import LbfdError, Solver
    need_gpu()
    prob = W.channel_flame(nx=64, ny=16, front_x=20.0, name="mix_adjoint")
    s = Solver(prob.replace(transport="mixture_averaged", lewis=LE4, cp=CP4))
    with pytest.raises(LbfdError):
        s.adjoint(4, 2)
