"""Every launch mode of the step against the oracle, for every combination
of lattice (D2Q9, D3Q27), species set (4 species / 1 reaction, 9 species /
20 sub-cycled reactions), species transport (unity Lewis, mixture-averaged)
and curved walls (none; interpolated bounce-back with Shepard image points),
in FP64 and in the mixed forms: the step with the reductions at every level
(check_every = 1), the fields and diagnostics launch, and the objective's
diagnostic steps.  Small boxes, few steps: the matrix is meant to catch a
wrong result in any instantiation, not to measure accuracy."""
import numpy as np
import pytest

from paper_2304_05657_amd import workloads as W

from .gpu_util import compare_fields, need_gpu, oracle_threads, say

pytestmark = pytest.mark.gpu
TOL64 = 1e-10
# relative field and diagnostic errors allowed in the mixed forms after a few
# steps (the 9-species mechanism's fast reactions amplify the single-
# precision rounding of T and Y_k, and sums of sources of both signs the
# relative error of the fuel-rate diagnostic)
TOL_MIXED = {"fp32": 5e-3, "fp16": 2e-2}
Y9_LO = (0.05, 0.2) + (0.0,) * 6 + (0.75,)
Y9_HI = (0.0, 0.0) + (0.05, 0.05, 0.05, 0.05, 0.0, 0.05) + (0.75,)


def _problem(dim, nsp, transport):
    if dim == 2:
        prob = W.cylinder_burner(nx=128, ny=64, radius=8.0, pitch=32, x_begin=32, x_end=96, front_x=64.0,
                                 name="modes_burner_128x64")
        if nsp == 9:
            th = 0.5 * (1.0 + np.tanh((np.arange(prob.nx) - 64.0) / 4.0))
            Y0 = np.stack([np.broadcast_to((1 - th) * Y9_LO[k] + th * Y9_HI[k], prob.T0.shape) for k in range(9)])
            prob = prob.replace(W=(28.0,) * 9, reactions=W.synthetic_mechanism(9, 20, 2305), Y0=np.ascontiguousarray(Y0),
                                Y_in=Y9_LO, chem_substeps_max=64, name="modes_burner9_128x64")
    else:
        if nsp == 9:
            prob = W.porous_3d_mech(nx=32, ny=12, nz=12, porosity=0.9, radius=(2.0, 4.0), margin=6,
                                    name="modes_mech_32x12x12")
        else:
            prob = W.porous_3d(nx=32, ny=12, nz=12, porosity=0.9, radius=3.0, margin=6, seed=5,
                               name="modes_porous_32x12x12")
    if transport == "mixture":
        prob = W.mixture_transport(prob)
    return prob


def _walls(prob, g, o):
    cells, dirs, q = W.wall_links(prob)
    g.set_wall_links(cells, dirs, q)
    o.set_wall_links(cells, dirs, q.astype(np.float32).astype(np.float64))
    c, sl, im = W.image_points(prob)
    g.set_image_points(c, sl, im)
    o.set_image_points(c, sl, im)
    return len(cells), len(c)


CASES = [(d, n, t, cw) for d in (2, 3) for n in (4, 9) for t in ("unity", "mixture") for cw in (False, True)]


@pytest.mark.parametrize("dim,nsp,transport,walls", CASES,
                         ids=["%dd-%dsp-%s-%s" % (d, n, t, "cw" if cw else "bb") for d, n, t, cw in CASES])
@pytest.mark.parametrize("precision", ["fp64", "fp32", "fp16"])
def test_modes_against_oracle(dim, nsp, transport, walls, precision):
    import oracle
    from paper_2304_05657_amd.lbfd import Solver
    need_gpu()
    if dim == 2 and nsp == 9 and precision == "fp16":
        pytest.skip("no D2Q9 / 9-species FP16 kernel is built")
    prob = _problem(dim, nsp, transport)
    say("case %s %s %s walls=%s %s" % (prob.name, transport, precision, walls, "check_every=1"))
    g = Solver(prob, precision=precision, check_every=1)
    o = oracle.Oracle(prob, threads=oracle_threads())
    if walls:
        nl, ni = _walls(prob, g, o)
        say("  %d wall links, %d image points" % (nl, ni))
    tol = TOL64 if precision == "fp64" else TOL_MIXED[precision]
    done = 0
    for target in (1, 4):
        g.step(target - done)
        o.step(target - done)
        done = target
        g.sync()
        e = compare_fields(g.fields(), o.fields(), prob)
        say("  level %d: %s" % (done, " ".join("%s=%.2e" % kv for kv in e.items())))
        for k, v in e.items():
            assert v <= tol, (done, k, v)
        dg, do = g.diagnostics(), o.diagnostics()
        assert dg["nonfinite"] == 0
        for k in ("sum_g", "sum_xi", "sum_theta", "wall_q", "fuel_rate"):
            scale = max(abs(do[k]), 1e-12 * abs(do["sum_theta"]), 1e-30)
            assert abs(dg[k] - do[k]) <= max(tol, 1e-9 if precision == "fp64" else tol) * scale, (k, dg[k], do[k])
    # the objective's diagnostic steps (wall heat flux over levels 4..6)
    if precision == "fp64":
        jg = g.objective(3)
        jo = o.objective(3)
        assert abs(jg - jo) <= 1e-9 * max(abs(jo), 1e-30), (jg, jo)
    g.close()


@pytest.mark.parametrize("dim,nsp,transport,walls", CASES,
                         ids=["%dd-%dsp-%s-%s" % (d, n, t, "cw" if cw else "bb") for d, n, t, cw in CASES])
@pytest.mark.parametrize("precision", ["fp64", "fp32", "fp16"])
def test_reductions_leave_the_state_unchanged(dim, nsp, transport, walls, precision):
    """The step with the reductions at every level (check_every = 1) and the
    plain step advance the state alike, and reading fields and diagnostics
    in between changes nothing.  The two are separate instantiations whose
    compiled arithmetic may contract and order operations differently, so
    "alike" is to rounding: 1e-13 in FP64, 5e-6 in the mixed forms (FP32
    arithmetic, 2^-24 per operation, grown over four steps of the stiff
    mechanism; measured up to 1.1e-6)."""
    from paper_2304_05657_amd.lbfd import Solver
    need_gpu()
    if dim == 2 and nsp == 9 and precision == "fp16":
        pytest.skip("no D2Q9 / 9-species FP16 kernel is built")
    prob = _problem(dim, nsp, transport)
    say("case %s %s %s walls=%s: check_every 1 against 0" % (prob.name, transport, precision, walls))
    a = Solver(prob, precision=precision, check_every=1)
    b = Solver(prob, precision=precision, check_every=0)
    if walls:
        for s in (a, b):
            cells, dirs, q = W.wall_links(prob)
            s.set_wall_links(cells, dirs, q)
            s.set_image_points(*W.image_points(prob))
    for n in (1, 3):
        a.step(n)
        a.fields()
        a.diagnostics()
        b.step(n)
    a.sync()
    b.sync()
    same = a.save_state() == b.save_state()
    fa, fb = a.fields(), b.fields()
    e = compare_fields(fa, fb, prob)
    say("  bitwise %s; %s" % (same, " ".join("%s=%.2e" % kv for kv in e.items())))
    for k, v in e.items():
        assert v <= (1e-13 if precision == "fp64" else 5e-6), (k, v)
    a.close()
    b.close()
