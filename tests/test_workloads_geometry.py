"""CPU checks of the curved-wall inputs the workload generators derive from
their analytic shapes (wall-link fractions, ghost image points) on one
cylinder in a periodic box, where every quantity has a closed form."""
import numpy as np

from paper_2304_05657_amd import workloads as W


def _one_cylinder(nx=40, ny=36, cx=19.3, cy=17.6, r=7.4):
    prob = W.channel_flame(nx=nx, ny=ny, front_x=10.0, name="one_cylinder")
    yy, xx = np.mgrid[0:ny, 0:nx]
    mask = np.where((xx - cx) ** 2 + (yy - cy) ** 2 <= r * r, W.SOLID_ISOTHERMAL, W.FLUID).astype(np.uint8)
    prob = prob.replace(mask=mask[None], faces=("periodic",) * 6, notes={"shapes": [(cx, cy, 0.0, r)],
                                                                          "slab": (0, nx)})
    return prob, (cx, cy, r)


def test_image_points_reflect_across_the_circle():
    """Each image point is the ghost node mirrored across the nearest point
    of the circle: on the ray from the centre through the ghost, at radius
    2r - |G - c|; every ghost node inside the cylinder is listed once."""
    prob, (cx, cy, r) = _one_cylinder()
    cells, slots, im = W.image_points(prob)
    assert len(cells) > 50 and len(set(zip(cells.tolist(), slots.tolist()))) == len(cells)
    offs = (-2, -1, 1, 2)
    fluid = prob.mask[0] == W.FLUID
    for c, s, I in zip(cells, slots, im):
        y, x = divmod(int(c), prob.nx)
        a, j = divmod(int(s), 4)
        G = np.array([x, y], float)
        G[a] += offs[j]
        v = G - (cx, cy)
        w = I[:2] - (cx, cy)
        assert abs(I[2]) == 0.0
        assert abs(np.hypot(*w) - (2 * r - np.hypot(*v))) < 1e-12
        assert abs(v[0] * w[1] - v[1] * w[0]) < 1e-9 * (1 + np.hypot(*v) * np.hypot(*w))
        assert v @ w > 0
    # every stencil point of a fluid cell that is a ghost inside the cylinder
    expect = set()
    for y in range(prob.ny):
        for x in range(prob.nx):
            if not fluid[y, x]:
                continue
            for a in (0, 1):
                for sg in (-1, 1):
                    p1 = [x, y]
                    p1[a] += sg
                    p2 = [x, y]
                    p2[a] += 2 * sg
                    f1 = fluid[p1[1] % prob.ny, p1[0] % prob.nx]
                    f2 = fluid[p2[1] % prob.ny, p2[0] % prob.nx]
                    for m, q, ghost in ((sg, p1, not f1), (2 * sg, p2, (not f1) or (not f2))):
                        inside = (q[0] - cx) ** 2 + (q[1] - cy) ** 2 <= r * r
                        if ghost and inside:
                            expect.add((y * prob.nx + x, 4 * a + offs.index(m)))
    assert expect == set(zip(cells.tolist(), slots.tolist()))


def test_wall_links_cut_the_circle():
    """The fraction q of every listed link puts the point r_f + q c_i on the
    circle, and the links are exactly the fluid-to-cylinder links."""
    prob, (cx, cy, r) = _one_cylinder()
    cells, dirs, q = W.wall_links(prob)
    fluid = prob.mask[0] == W.FLUID
    count = 0
    for c, d, qq in zip(cells, dirs, q):
        y, x = divmod(int(c), prob.nx)
        ex, ey = d % 3 - 1, d // 3 - 1
        px, py = x + qq * ex, y + qq * ey
        assert abs(np.hypot(px - cx, py - cy) - r) < 1e-9
        assert 0.0 < qq <= 1.0 and fluid[y, x] and not fluid[(y + ey) % prob.ny, (x + ex) % prob.nx]
        count += 1
    links = sum(1 for y in range(prob.ny) for x in range(prob.nx) if fluid[y, x]
                for d in range(9) if d != 4 and not fluid[(y + d // 3 - 1) % prob.ny, (x + d % 3 - 1) % prob.nx])
    assert count == links


def test_mixture_transport_property_data():
    prob = W.mixture_transport(W.channel_flame(nx=16, ny=8, front_x=4.0, name="m"))
    assert prob.transport == "mixture_averaged" and len(prob.lewis) == 4 and len(prob.cp) == 4
    p9 = W.mixture_transport(W.porous_3d_mech(nx=16, ny=8, nz=8, margin=4, radius=(2.0, 3.0), porosity=0.95,
                                              name="m9"))
    assert len(p9.lewis) == 9 and min(p9.lewis) >= 0.7 and max(p9.cp) <= 2.2
