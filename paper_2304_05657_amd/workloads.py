"""Seeded synthetic workloads: geometry, initial fields and parameters.

This module only builds input data (masks, wall temperatures, initial
temperature / mass-fraction / velocity fields, chemistry parameters).  It
holds none of the method's arithmetic and is shared, as plain data, by the
GPU library's tests and benchmark and by the CPU oracle.

The workloads stand in for the paper's cases (Sec. IV): a 2-D channel flame
(IV.A), a pseudo 2-D burner with staggered cylinders (IV.B) and random 3-D
sphere packings (IV.C).  The paper's own geometry, the BFER-2 mechanism and
Cantera data are not available, so a one-step synthetic mechanism with the
same structure (fuel + oxidiser -> product, inert diluent) is used.
"""
from __future__ import annotations

import dataclasses
from dataclasses import dataclass, field

import numpy as np

FACES = ("periodic", "wall", "inflow", "outflow", "wall_adiabatic")
FLUID, SOLID_ISOTHERMAL, SOLID_ADIABATIC = 0, 1, 2

# Four-species one-step mixture.  Mass stoichiometry F + 4 O -> 5 P, molar
# masses chosen so that moles (and the mixture molar mass) are unchanged by
# reaction; q = 3e4 K per unit fuel mass fraction so that the stoichiometric
# unburnt mixture at 300 K burns to 1800 K.
W4 = (16.0, 32.0, 80.0 / 3.0, 28.0)
Y_UNBURNT_STOICH = (0.05, 0.2, 0.0, 0.75)
Y_BURNT_STOICH = (0.0, 0.0, 0.25, 0.75)
Y_UNBURNT_LEAN = (0.04, 0.2, 0.0, 0.76)
Y_BURNT_LEAN = (0.0, 0.04, 0.2, 0.76)
W_REF = 28.0
DT_PHYS_CHANNEL = 7.5e-8  # s, time step of the channel cases (Sec. IV.A)
DT_PHYS_BURNER = 1.0e-7   # s, time step of the burner / porous cases (Sec. IV.B)


@dataclass
class Reaction:
    reactants: list
    A: float
    b: float
    Ta: float
    nu: list
    q: float


@dataclass
class Problem:
    name: str
    lattice: int
    nx: int
    ny: int
    nz: int
    faces: tuple
    face_T: tuple
    tau: float
    prandtl: float
    dt_phys: float
    T_ref: float
    W_ref: float
    W: tuple
    reactions: list
    u_in: tuple
    T_in: float
    Y_in: tuple
    mask: np.ndarray
    wall_T: np.ndarray
    T0: np.ndarray
    Y0: np.ndarray
    u0: np.ndarray | None = None
    Ph0: np.ndarray | None = None
    omega3: float = 1.0
    omega4: float = 1.0
    eq_discrete: bool = False
    chem_substeps_max: int = 1
    collision: str = "central_moments"  # or "cumulants" (orders >= 4 relaxed as cumulants)
    transport: str = "unity_lewis"  # or "mixture_averaged" (Lewis numbers and heat capacities below)
    lewis: tuple = ()  # Le_k = alpha / D_k per species (empty: all 1)
    cp: tuple = ()  # c_pk / c_p,ref per species (empty: all 1)
    T_u: float = 300.0
    T_b: float = 1800.0
    steps: int = 0
    notes: dict = field(default_factory=dict)

    @property
    def N(self) -> int:
        return self.nx * self.ny * self.nz

    @property
    def n_species(self) -> int:
        return len(self.W)

    @property
    def n_fluid(self) -> int:
        return int(np.count_nonzero(self.mask == FLUID))

    def replace(self, **kw) -> "Problem":
        return dataclasses.replace(self, **kw)


def one_step_reaction(A: float = 1e9, Ta: float = 15000.0, b: float = 0.0) -> Reaction:
    return Reaction(reactants=[0, 1], A=A, b=b, Ta=Ta, nu=[-1.0, -4.0, 5.0, 0.0], q=3.0e4)


def _tanh_blend(x, x0, width, lo, hi):
    th = 0.5 * (1.0 + np.tanh((x - x0) / width))
    return th, lo + (hi - lo) * th


def _front_fields(shape, xcoord, x0, width, T_lo, T_hi, Y_lo, Y_hi):
    """tanh front along x: theta = (1 + tanh((x - x0)/width))/2."""
    th, T = _tanh_blend(xcoord, x0, width, T_lo, T_hi)
    T = np.broadcast_to(T, shape).astype(np.float64).copy()
    th = np.broadcast_to(th, shape)
    Y = np.stack([(1.0 - th) * Y_lo[k] + th * Y_hi[k] for k in range(len(Y_lo))])
    return T, np.ascontiguousarray(Y, dtype=np.float64)


def channel_flame(nx: int = 256, ny: int = 64, steps: int = 2000, front_x: float = 64.0,
                  width: float = 4.0, wall_T: float = 300.0, adiabatic: bool = False,
                  name: str = "channel_flame_256x64") -> Problem:
    """2-D channel flame, D2Q9: rows y=0 and y=ny-1 solid (isothermal at
    wall_T, or adiabatic), periodic in x, fluid at rest, tanh front from
    300 K / unburnt stoichiometric mixture to 1800 K / burnt mixture at
    x = front_x (width 4 cells).  tau = 0.6, Pr = 0.7, A = 1e9 1/s,
    Ta = 15000 K, dt = 7.5e-8 s."""
    shape = (1, ny, nx)
    mask = np.zeros(shape, dtype=np.uint8)
    solid = SOLID_ADIABATIC if adiabatic else SOLID_ISOTHERMAL
    mask[:, 0, :] = solid
    mask[:, ny - 1, :] = solid
    x = np.arange(nx, dtype=np.float64)[None, None, :]
    T0, Y0 = _front_fields(shape, x, front_x, width, 300.0, 1800.0,
                           Y_UNBURNT_STOICH, Y_BURNT_STOICH)
    wT = np.full(shape, wall_T, dtype=np.float64)
    T0[mask != FLUID] = wall_T
    return Problem(
        name=name, lattice=9, nx=nx, ny=ny, nz=1,
        faces=("periodic",) * 6, face_T=(300.0,) * 6,
        tau=0.6, prandtl=0.7, dt_phys=DT_PHYS_CHANNEL, T_ref=300.0, W_ref=W_REF,
        W=W4, reactions=[one_step_reaction()],
        u_in=(0.0, 0.0, 0.0), T_in=300.0, Y_in=Y_UNBURNT_STOICH,
        mask=mask, wall_T=wT, T0=T0, Y0=Y0, steps=steps,
        notes={"wall": "adiabatic" if adiabatic else "isothermal %.1f K" % wall_T},
    )


def poiseuille_profile(prob, u_mean: float):
    """Inlet profile [3, nz, ny] of a D2Q9 channel whose first and last rows
    are solid: the half-way-wall parabola u_x = 6 u_mean s (1 - s),
    s = (y - 1/2) / H, H = ny - 2, on the fluid rows (Sec. IV.A: a 2-D
    Poiseuille inlet with a target flow rate); zero on the solid rows."""
    H = prob.ny - 2
    y = np.arange(prob.ny, dtype=np.float64)
    s = (y - 0.5) / H
    ux = np.where((y >= 1) & (y <= prob.ny - 2), 6.0 * u_mean * s * (1.0 - s), 0.0)
    u = np.zeros((3, prob.nz, prob.ny))
    u[0] = ux[None, :]
    return u


def flame_channel(nx: int = 512, ny: int = 34, u_mean: float = 0.002, front_x: float = 256.0,
                  adiabatic: bool = True, A: float = 1e10, name: str | None = None) -> Problem:
    """Flame-holding channel, D2Q9: rows 0 and ny-1 solid walls (adiabatic,
    or isothermal at 300 K), fresh stoichiometric inflow at 300 K at -x,
    outflow at +x; tanh front at front_x with the burnt state downstream; the
    fresh side starts with the Poiseuille inlet profile of mean u_mean
    (poiseuille_profile), the burnt side at rest.  A = 1e10 1/s (a faster
    flame than the channel flame's 1e9, so that it forms within ~1e4 steps)."""
    base = channel_flame(nx=nx, ny=ny, front_x=front_x, adiabatic=adiabatic, name="tmp")
    r = base.reactions[0]
    prob = base.replace(name=name or "flame_channel_%dx%d" % (nx, ny),
                        faces=("inflow", "outflow", "periodic", "periodic", "periodic", "periodic"),
                        u_in=(u_mean, 0.0, 0.0),
                        reactions=[Reaction(r.reactants, A, r.b, r.Ta, r.nu, r.q)])
    prof = poiseuille_profile(prob, u_mean)
    x = np.arange(nx, dtype=np.float64)
    fresh = (x < front_x)[None, None, :]
    u0 = np.zeros((3, 1, ny, nx))
    u0[0] = np.where(fresh, prof[0][:, :, None], 0.0)
    return prob.replace(u0=u0)


def mixture_transport(prob, seed: int = 2304):
    """The problem with mixture-averaged species transport and synthetic
    property data (no property database is available): for the 4-species
    F / O / P / N set Lewis numbers (0.8, 1.1, 1.4, 1.0) and heat capacities
    c_pk / c_p,ref (2.0, 0.9, 1.3, 1.0), of the order of methane, oxygen,
    combustion products and nitrogen; for other species counts seeded
    values with Le_k in [0.7, 1.6] and c_pk / c_p,ref in [0.8, 2.2]."""
    ns = prob.n_species
    if ns == 4:
        le, cp = (0.8, 1.1, 1.4, 1.0), (2.0, 0.9, 1.3, 1.0)
    else:
        rng = np.random.default_rng(seed)
        le, cp = tuple(rng.uniform(0.7, 1.6, ns)), tuple(rng.uniform(0.8, 2.2, ns))
    return prob.replace(transport="mixture_averaged", lewis=le, cp=cp)


def wall_links(prob):
    """Wall distances of the links that cross the curved walls of the
    problem's shapes (prob.notes["shapes"]: cylinders (cx, cy, 0, r) of a
    D2Q9 box, spheres (cx, cy, cz, r) of a D3Q27 box; solid where the cell
    centre is within r, y and z periodic, x restricted to prob.notes["slab"]),
    as input for an interpolated bounce-back.  For every fluid cell p and
    lattice direction i whose neighbour p + c_i is a solid cell of a shape,
    q is the fraction of the segment from p to p + c_i at which it enters
    the shape (the smallest over the shapes covering p + c_i that do not
    cover p).  Returns (cell [n] int64, dir [n] int32, q [n] float64),
    sorted by cell then direction, directions in the lattice order (c_z,
    c_y, c_x lexicographic, x fastest).  Links into solids of no shape are
    not listed."""
    shapes = prob.notes.get("shapes", [])
    x0, x1 = prob.notes.get("slab", (0, prob.nx))
    D = 2 if prob.lattice == 9 else 3
    nx, ny, nz = prob.nx, prob.ny, prob.nz
    dirs = [(cx, cy, cz) for cz in ((-1, 0, 1) if D == 3 else (0,)) for cy in (-1, 0, 1) for cx in (-1, 0, 1)]
    fluid = prob.mask.reshape(-1) == FLUID
    best = {}
    for (sx, sy, sz, r) in shapes:
        ri = int(np.ceil(r)) + 2
        xs = np.arange(max(0, int(np.floor(sx)) - ri), min(nx, int(np.ceil(sx)) + ri + 1))
        ys = np.arange(int(np.floor(sy)) - ri, int(np.ceil(sy)) + ri + 1)
        zs = np.arange(int(np.floor(sz)) - ri, int(np.ceil(sz)) + ri + 1) if D == 3 else np.zeros(1, int)
        Z, Y, X = np.meshgrid(zs, ys, xs, indexing="ij")
        # positions relative to the centre (the unwrapped image nearest to it)
        px, py, pz = X - sx, Y - sy, (Z - sz if D == 3 else np.zeros_like(X, dtype=float))
        cell = ((Z % nz) * ny + (Y % ny)) * nx + X
        out_p = (px * px + py * py + pz * pz > r * r) | (X < x0) | (X >= x1)
        for i, (cx, cy, cz) in enumerate(dirs):
            if cx == 0 and cy == 0 and cz == 0:
                continue
            qx, qy, qz = px + cx, py + cy, pz + cz
            Xn = X + cx
            in_n = (qx * qx + qy * qy + qz * qz <= r * r) & (Xn >= x0) & (Xn < x1)
            sel = out_p & in_n & fluid[cell]
            if not sel.any():
                continue
            a = float(cx * cx + cy * cy + cz * cz)
            bq = 2.0 * (px * cx + py * cy + pz * cz)
            cq = px * px + py * py + pz * pz - r * r
            disc = np.sqrt(np.maximum(bq * bq - 4.0 * a * cq, 0.0))
            t = (-bq - disc) / (2.0 * a)
            for c, tv in zip(cell[sel].tolist(), t[sel].tolist()):
                key = (c, i)
                if tv > 0.0 and (key not in best or tv < best[key]):
                    best[key] = min(tv, 1.0)
    keys = sorted(best)
    cells = np.array([k[0] for k in keys], dtype=np.int64)
    dirs_out = np.array([k[1] for k in keys], dtype=np.int32)
    q = np.array([best[k] for k in keys], dtype=np.float64)
    return cells, dirs_out, q


def image_points(prob):
    """Image points of the finite-difference ghost nodes that lie inside the
    problem's shapes (the cylinders / spheres of prob.notes["shapes"], as
    for wall_links), as input for a ghost-node treatment of curved walls.
    The ghost nodes of a fluid cell p along axis a are its stencil points
    p + m e_a (m = -2, -1, 1, 2) behind a wall: both points of a side whose
    first neighbour is not fluid, else the second neighbour when that is
    not fluid.  For a ghost G inside a shape (the one of least depth when
    several cover it) with centre c and radius r, B is the nearest point of
    that shape's surface and the image I = 2B - G = G + 2 (r - |v|) v / |v|,
    v = G - c (nearest periodic image).  Returns (cell [n] int64, slot [n]
    int32 = 4 a + j for m = (-2, -1, 1, 2)[j], image [n, 3] float64 in
    lattice coordinates unwrapped from p), sorted by cell then slot.
    Ghosts in solids of no shape are not listed, nor ghosts whose image point
    is not certain to have a fluid node within four cells (where overlapping
    shapes put it deep in solid: |I - g| + the distance from the grid point
    g nearest to I to the nearest fluid cell must not exceed 4); those keep
    the axis mirror."""
    shapes = prob.notes.get("shapes", [])
    x0, x1 = prob.notes.get("slab", (0, prob.nx))
    D = 2 if prob.lattice == 9 else 3
    nx, ny, nz = prob.nx, prob.ny, prob.nz
    n = (nx, ny, nz)
    periodic = [prob.faces[2 * a] == "periodic" for a in range(3)]
    mask = np.asarray(prob.mask).reshape(nz, ny, nx)
    # the shape of least depth covering each cell centre
    label = np.full(mask.shape, -1, np.int64)
    depth = np.full(mask.shape, np.inf)
    for k, (sx, sy, sz, r) in enumerate(shapes):
        ri = int(np.ceil(r)) + 1
        xs = np.arange(max(x0, int(np.floor(sx)) - ri), min(x1, int(np.ceil(sx)) + ri + 1))
        ys = np.arange(int(np.floor(sy)) - ri, int(np.ceil(sy)) + ri + 1)
        zs = np.arange(int(np.floor(sz)) - ri, int(np.ceil(sz)) + ri + 1) if D == 3 else np.zeros(1, int)
        Z, Y, X = np.meshgrid(zs, ys, xs, indexing="ij")
        px, py, pz = X - sx, Y - sy, (Z - sz if D == 3 else np.zeros_like(X, dtype=float))
        dep = r - np.sqrt(px * px + py * py + pz * pz)
        Zw, Yw = Z % nz, Y % ny
        sel = (dep >= 0.0) & (dep < depth[Zw, Yw, X])
        depth[Zw[sel], Yw[sel], X[sel]] = dep[sel]
        label[Zw[sel], Yw[sel], X[sel]] = k
    # distance from every cell centre to the nearest fluid cell centre
    from scipy import ndimage
    pad = [(6, 6) if periodic[2 - ax] and mask.shape[ax] > 1 else (0, 0) for ax in range(3)]
    fd = ndimage.distance_transform_edt(np.pad(mask != FLUID, pad, mode="wrap"))
    fd = fd[tuple(slice(w[0], w[0] + m) for w, m in zip(pad, mask.shape))]
    fz, fy, fx = np.nonzero(mask == FLUID)
    pc = [fx, fy, fz]
    cell = (fz.astype(np.int64) * ny + fy) * nx + fx

    def probe(a, m):
        """(fluid?, shape label, wrapped coords) of p + m e_a per fluid cell."""
        q = [c.copy() for c in pc]
        q[a] = q[a] + m
        inbox = np.ones(len(fx), bool)
        if periodic[a]:
            q[a] %= n[a]
        else:
            inbox = (q[a] >= 0) & (q[a] < n[a])
            q[a] = np.clip(q[a], 0, n[a] - 1)
        fl = inbox & (mask[q[2], q[1], q[0]] == FLUID)
        lab = np.where(inbox, label[q[2], q[1], q[0]], -1)
        return fl, lab

    out_c, out_s, out_i = [], [], []
    cen = np.array([[s[0], s[1], s[2]] for s in shapes], dtype=np.float64).reshape(-1, 3)
    rad = np.array([s[3] for s in shapes], dtype=np.float64)
    for a in range(D):
        for sg in (-1, 1):
            j1, j2 = (1, 0) if sg < 0 else (2, 3)
            f1, l1 = probe(a, sg)
            f2, l2 = probe(a, 2 * sg)
            for m, j, ghost, lab in ((sg, j1, ~f1, l1), (2 * sg, j2, ~f1 | ~f2, l2)):
                sel = ghost & (lab >= 0)
                if not sel.any():
                    continue
                G = np.stack([c[sel].astype(np.float64) for c in pc], axis=1)
                G[:, a] += m
                if D == 2:
                    G[:, 2] = 0.0
                c = cen[lab[sel]]
                v = G - c
                for ax in range(D):
                    if periodic[ax]:
                        v[:, ax] -= n[ax] * np.round(v[:, ax] / n[ax])
                if D == 2:
                    v[:, 2] = 0.0
                dv = np.sqrt((v * v).sum(axis=1))
                ok = dv > 0.0
                img = G + 2.0 * ((rad[lab[sel]] - dv) / np.where(ok, dv, 1.0))[:, None] * v
                # a fluid node within four cells of the image point, for sure
                gi = np.rint(img).astype(np.int64)
                for ax in range(3):
                    gi[:, ax] = gi[:, ax] % n[ax] if periodic[ax] else np.clip(gi[:, ax], 0, n[ax] - 1)
                if D == 2:
                    gi[:, 2] = 0
                gu = img.copy()   # g unwrapped next to the image point
                for ax in range(3):
                    gu[:, ax] = gi[:, ax] + (n[ax] * np.round((img[:, ax] - gi[:, ax]) / n[ax]) if periodic[ax] else 0)
                reach = np.sqrt(((img - gu) ** 2).sum(axis=1)) + fd[gi[:, 2], gi[:, 1], gi[:, 0]]
                ok &= reach <= 4.0
                out_c.append(cell[sel][ok])
                out_s.append(np.full(int(ok.sum()), 4 * a + j, np.int32))
                out_i.append(img[ok])
    if not out_c:
        return np.zeros(0, np.int64), np.zeros(0, np.int32), np.zeros((0, 3))
    c = np.concatenate(out_c)
    sl = np.concatenate(out_s)
    im = np.concatenate(out_i)
    order = np.lexsort((sl, c))
    return c[order], sl[order], im[order]


def wall_layer(T, Y, mask, wall_T, periodic_axes, delta=4.0):
    """Initial thermal layer next to solids: within `delta` cells of a solid
    cell the gas temperature is blended linearly from the nearest wall
    temperature (distance 1) to the front profile (distance delta + 1),
    so that the initial state has no hot-gas / cold-wall jump.  Distances
    are Euclidean between cell centres, periodic along `periodic_axes`
    (axes of the (z, y, x) array).  Y is left unchanged."""
    from scipy import ndimage
    solid = mask != FLUID
    if not solid.any():
        return T
    pad = int(np.ceil(delta)) + 2
    widths = [(pad, pad) if ax in periodic_axes and solid.shape[ax] > 1 else (0, 0) for ax in range(3)]
    sp = np.pad(solid, widths, mode="wrap")
    wp = np.pad(np.where(solid, wall_T, 0.0), widths, mode="wrap")
    dist, inds = ndimage.distance_transform_edt(~sp, return_indices=True)
    Tw_near = wp[tuple(inds)]
    sl = tuple(slice(w[0], w[0] + n) for w, n in zip(widths, solid.shape))
    dist, Tw_near = dist[sl], Tw_near[sl]
    s = np.clip((dist - 1.0) / delta, 0.0, 1.0)
    out = Tw_near + (T - Tw_near) * s
    return np.where(solid, T, out)


def _periodic_delta(a, c, n):
    d = np.abs(a - c)
    return np.minimum(d, n - d)


def cylinder_burner(nx: int = 2048, ny: int = 512, radius: float = 20.0, pitch: int = 64,
                    x_begin: int = 256, x_end: int = 1792, wall_T: float = 400.0,
                    u_in: float = 0.02, front_x: float = 1024.0, steps: int = 20000,
                    name: str | None = None) -> Problem:
    """Pseudo 2-D porous burner, D2Q9: staggered cylinders of `radius` on a
    `pitch` lattice (columns every `pitch` cells over [x_begin, x_end),
    centres y = pitch/2 + pitch*j + (pitch/2)(col mod 2), periodic in y),
    isothermal at wall_T; lean inflow (Y = 0.04/0.2/0/0.76, 300 K, u_in)
    at -x, outflow at +x; fluid at rest with a tanh front at front_x and
    the lean burnt state downstream."""
    shape = (1, ny, nx)
    mask = np.zeros(shape, dtype=np.uint8)
    yy, xx = np.mgrid[0:ny, 0:nx]
    cylinders = []
    for col, cx in enumerate(range(x_begin, x_end, pitch)):
        for j in range(ny // pitch):
            cy = pitch // 2 + pitch * j + (pitch // 2) * (col % 2)
            cy %= ny
            inside = (xx - cx) ** 2 + _periodic_delta(yy, cy, ny) ** 2 <= radius * radius
            mask[0][inside] = SOLID_ISOTHERMAL
            cylinders.append((float(cx), float(cy), 0.0, float(radius)))
    x = np.arange(nx, dtype=np.float64)[None, None, :]
    T0, Y0 = _front_fields(shape, x, front_x, 4.0, 300.0, 1500.0, Y_UNBURNT_LEAN, Y_BURNT_LEAN)
    wT = np.full(shape, wall_T)
    T0 = wall_layer(T0, Y0, mask, wT, periodic_axes=(1,))
    T0[mask != FLUID] = wall_T
    return Problem(
        name=name or "cylinder_burner_%dx%d" % (nx, ny), lattice=9, nx=nx, ny=ny, nz=1,
        faces=("inflow", "outflow", "periodic", "periodic", "periodic", "periodic"),
        face_T=(300.0,) * 6, tau=0.6, prandtl=0.7, dt_phys=DT_PHYS_BURNER, T_ref=300.0,
        W_ref=W_REF, W=W4, reactions=[one_step_reaction()],
        u_in=(u_in, 0.0, 0.0), T_in=300.0, Y_in=Y_UNBURNT_LEAN,
        mask=mask, wall_T=wT, T0=T0, Y0=Y0, steps=steps,
        T_u=300.0, T_b=1500.0,
        notes={"shapes": cylinders, "slab": (0, nx)},
    )


def sphere_packing_mask(nx, ny, nz, porosity, radius_lo, radius_hi, seed, margin=16,
                        max_spheres=1_000_000):
    """Overlapping spheres with centres uniform in x in [margin, nx-margin)
    and over the periodic y, z extent, radii uniform in [radius_lo,
    radius_hi] (a single value when equal), added until the voxel porosity
    of the packed slab x in [margin, nx-margin) is <= porosity.  A cell is
    solid when its centre is within the radius (periodic in y and z, cut
    at the slab ends)."""
    rng = np.random.default_rng(seed)
    solid = np.zeros((nz, ny, nx), dtype=bool)
    x0, x1 = margin, nx - margin
    total = (x1 - x0) * ny * nz
    nsolid = 0
    spheres = []
    for _ in range(max_spheres):
        if 1.0 - nsolid / total <= porosity:
            break
        cx = rng.uniform(x0, x1)
        cy = rng.uniform(0, ny)
        cz = rng.uniform(0, nz)
        r = radius_lo if radius_hi == radius_lo else rng.uniform(radius_lo, radius_hi)
        spheres.append((cx, cy, cz, r))
        ri = int(np.ceil(r))
        xs = np.arange(max(x0, int(np.floor(cx - ri))), min(x1, int(np.ceil(cx + ri)) + 1))
        ys = np.arange(int(np.floor(cy - ri)), int(np.ceil(cy + ri)) + 1)
        zs = np.arange(int(np.floor(cz - ri)), int(np.ceil(cz + ri)) + 1)
        if xs.size == 0:
            continue
        dz = (zs - cz)[:, None, None] ** 2
        dy = (ys - cy)[None, :, None] ** 2
        dx = (xs - cx)[None, None, :] ** 2
        inside = dz + dy + dx <= r * r
        zi = (zs % nz)[:, None, None]
        yi = (ys % ny)[None, :, None]
        xi = xs[None, None, :]
        zi, yi, xi = np.broadcast_arrays(zi, yi, xi)
        zi, yi, xi = zi[inside], yi[inside], xi[inside]
        new = ~solid[zi, yi, xi]
        # repeated (wrapped) coordinates in one sphere are counted once
        lin = np.unique((zi[new] * ny + yi[new]) * nx + xi[new])
        solid.reshape(-1)[lin] = True
        nsolid += lin.size
    return solid, spheres


def _three_d_front(shape, nx, front_x, T_lo, T_hi, Y_lo, Y_hi):
    x = np.arange(nx, dtype=np.float64)[None, None, :]
    return _front_fields(shape, x, front_x, 4.0, T_lo, T_hi, Y_lo, Y_hi)


def porous_3d(nx: int = 256, ny: int = 256, nz: int = 256, porosity: float = 0.80,
              radius: float = 8.0, seed: int = 2304, wall_T: float = 350.0, u_in: float = 0.01,
              front_x: float | None = None, margin: int = 16, steps: int = 5000,
              name: str | None = None) -> Problem:
    """3-D random porous medium, D3Q27: overlapping spheres of `radius`
    (seeded) to `porosity`, solid isothermal at wall_T, stoichiometric
    inflow at -x (u_in, 300 K), outflow at +x, periodic in y and z; tanh
    front at front_x (default nx/2) with burnt gas downstream."""
    shape = (nz, ny, nx)
    solid, spheres = sphere_packing_mask(nx, ny, nz, porosity, radius, radius, seed, margin)
    mask = np.where(solid, SOLID_ISOTHERMAL, FLUID).astype(np.uint8)
    T0, Y0 = _three_d_front(shape, nx, nx / 2 if front_x is None else front_x, 300.0, 1800.0,
                            Y_UNBURNT_STOICH, Y_BURNT_STOICH)
    T0 = wall_layer(T0, Y0, mask, np.full(shape, wall_T), periodic_axes=(0, 1))
    T0[solid] = wall_T
    return Problem(
        name=name or "porous3d_%dx%dx%d" % (nx, ny, nz), lattice=27, nx=nx, ny=ny, nz=nz,
        faces=("inflow", "outflow", "periodic", "periodic", "periodic", "periodic"),
        face_T=(300.0,) * 6, tau=0.6, prandtl=0.7, dt_phys=DT_PHYS_BURNER, T_ref=300.0,
        W_ref=W_REF, W=W4, reactions=[one_step_reaction()],
        u_in=(u_in, 0.0, 0.0), T_in=300.0, Y_in=Y_UNBURNT_STOICH,
        mask=mask, wall_T=np.full(shape, wall_T), T0=T0, Y0=Y0, steps=steps,
        notes={"seed": seed, "porosity_target": porosity, "shapes": spheres, "slab": (margin, nx - margin)},
    )


def synthetic_enthalpies(n_species: int = 9, seed: int = 2305, h_top: float = 2000.0) -> list:
    """Chemical enthalpy levels (K per unit mass fraction) of the synthetic
    mechanism's species: species 0 and 1 (fuel and oxidiser) at h_top, the
    intermediates 2 .. n_species - 2 at seeded levels in (0.05, 0.9) h_top,
    the last species (inert) at 0."""
    rng = np.random.default_rng([seed, 1])
    h = [h_top, h_top] + [float(v) for v in rng.uniform(0.05, 0.9, n_species - 3) * h_top] + [0.0]
    return h


def synthetic_mechanism(n_species: int = 9, n_reactions: int = 20, seed: int = 2305,
                        log10A=(6.0, 13.0), Ta=(5000.0, 25000.0), b=(-1.0, 1.0),
                        h_top: float = 2000.0) -> list:
    """Seeded synthetic mechanism that conserves energy.  Species carry the
    enthalpy levels of `synthetic_enthalpies`; the last species is inert
    and takes part in no reaction.  Per reaction: two distinct reactants and
    one or two distinct products, every product below both reactants in
    enthalpy (the first reaction burns the fuel with the oxidiser); mass
    coefficients: the reactants lose fractions a, 1 - a that sum to 1, the
    products gain the same total; the heat release per unit progress is
    the enthalpy the reaction gives up, q = sum_r a_r h_r - sum_p c_p h_p > 0
    (K).  Then T + sum_k h_k Y_k is invariant under the sources, so no cycle
    of reactions can heat the gas without bound.  Rate parameters: log10 A,
    Ta and b uniform in the given ranges."""
    rng = np.random.default_rng(seed)
    h = synthetic_enthalpies(n_species, seed, h_top)
    reactive = list(range(n_species - 1))
    rx = []
    while len(rx) < n_reactions:
        if not rx:
            reac = [0, 1]
        else:
            reac = [int(v) for v in rng.choice(reactive, 2, replace=False)]
        lo = min(h[reac[0]], h[reac[1]])
        below = [k for k in reactive if h[k] < lo and k not in reac]
        if not below:
            continue
        nprod = min(int(rng.integers(1, 3)), len(below))
        prods = [int(v) for v in rng.choice(below, nprod, replace=False)]
        nu = [0.0] * n_species
        a = float(rng.uniform(0.2, 0.8))
        nu[reac[0]] = -a
        nu[reac[1]] = -(1.0 - a)
        if nprod == 1:
            nu[prods[0]] = 1.0
        else:
            c = float(rng.uniform(0.2, 0.8))
            nu[prods[0]] = c
            nu[prods[1]] = 1.0 - c
        q = -sum(nu[k] * h[k] for k in range(n_species))
        rx.append(Reaction(reactants=reac, A=float(10.0 ** rng.uniform(*log10A)),
                           b=float(rng.uniform(*b)), Ta=float(rng.uniform(*Ta)), nu=nu, q=q))
    return rx


def porous_3d_mech(nx: int = 512, ny: int = 256, nz: int = 256, porosity: float = 0.85,
                   radius=(6.0, 12.0), seed: int = 2306, mech_seed: int = 2305,
                   wall_T: float = 350.0, u_in: float = 0.01, margin: int = 16,
                   steps: int = 2000, substeps_max: int = 64, name: str | None = None) -> Problem:
    """3-D porous medium with a synthetic 9-species / 20-reaction mechanism
    (all molar masses 28, so the mixture molar mass is constant)."""
    ns = 9
    shape = (nz, ny, nx)
    solid, spheres = sphere_packing_mask(nx, ny, nz, porosity, radius[0], radius[1], seed, margin)
    mask = np.where(solid, SOLID_ISOTHERMAL, FLUID).astype(np.uint8)
    Y_lo = (0.05, 0.2) + (0.0,) * 6 + (0.75,)
    Y_hi = (0.0, 0.0) + (0.05, 0.05, 0.05, 0.05, 0.0, 0.05) + (0.75,)
    T0, Y0 = _three_d_front(shape, nx, nx / 2, 300.0, 1800.0, Y_lo, Y_hi)
    T0 = wall_layer(T0, Y0, mask, np.full(shape, wall_T), periodic_axes=(0, 1))
    T0[solid] = wall_T
    return Problem(
        name=name or "porous3d_mech_%dx%dx%d" % (nx, ny, nz), lattice=27, nx=nx, ny=ny, nz=nz,
        faces=("inflow", "outflow", "periodic", "periodic", "periodic", "periodic"),
        face_T=(300.0,) * 6, tau=0.6, prandtl=0.7, dt_phys=DT_PHYS_BURNER, T_ref=300.0,
        W_ref=28.0, W=(28.0,) * ns, reactions=synthetic_mechanism(ns, 20, mech_seed),
        u_in=(u_in, 0.0, 0.0), T_in=300.0, Y_in=Y_lo,
        mask=mask, wall_T=np.full(shape, wall_T), T0=T0, Y0=Y0, steps=steps,
        chem_substeps_max=substeps_max,
        notes={"seed": seed, "mech_seed": mech_seed, "shapes": spheres, "slab": (margin, nx - margin)},
    )


def named(name: str) -> Problem:
    """The five standard workloads by short name."""
    if name == "channel":
        return channel_flame()
    if name == "burner":
        return cylinder_burner()
    if name == "porous":
        return porous_3d()
    if name == "porous_mech":
        return porous_3d_mech()
    if name == "channel_adjoint":
        return channel_flame(nx=1024, ny=256, steps=500, front_x=64.0,
                             name="channel_flame_1024x256")
    raise KeyError(name)
