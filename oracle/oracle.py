"""ctypes wrapper of the FP64 CPU oracle (``lbfd_oracle.c``).

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, ``__graft_entry__.smoke()``
and the ``cpu_baseline`` leg of ``bench.py``; never by the GPU library.

The oracle takes a :class:`paper_2304_05657_amd.workloads.Problem` (plain
input data: geometry, initial fields, parameters) and marshals it into its
own parameter struct.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "lbfd_oracle.c")
_LIB = os.path.join(_HERE, "liblbfd_oracle.so")

MAXSP = 16
MAXRX = 32
NDIAG = 14
FACE_CODES = {"periodic": 0, "wall": 1, "inflow": 2, "outflow": 3, "wall_adiabatic": 4}


class _Reaction(C.Structure):
    _fields_ = [
        ("n_react", C.c_int),
        ("react", C.c_int * 4),
        ("A", C.c_double),
        ("b", C.c_double),
        ("Ta", C.c_double),
        ("nu", C.c_double * MAXSP),
        ("q", C.c_double),
    ]


class _Params(C.Structure):
    _fields_ = [
        ("Q", C.c_int),
        ("nx", C.c_int),
        ("ny", C.c_int),
        ("nz", C.c_int),
        ("face", C.c_int * 6),
        ("face_T", C.c_double * 6),
        ("tau", C.c_double),
        ("prandtl", C.c_double),
        ("dt_phys", C.c_double),
        ("T_ref", C.c_double),
        ("W_ref", C.c_double),
        ("n_species", C.c_int),
        ("W", C.c_double * MAXSP),
        ("n_reactions", C.c_int),
        ("rx", _Reaction * MAXRX),
        ("u_in", C.c_double * 3),
        ("T_in", C.c_double),
        ("Y_in", C.c_double * MAXSP),
        ("omega3", C.c_double),
        ("omega4", C.c_double),
        ("eq_discrete", C.c_int),
        ("chem_substeps_max", C.c_int),
        ("body_force", C.c_double * 3),
        ("T_u", C.c_double),
        ("T_b", C.c_double),
        ("collision", C.c_int),
        ("transport", C.c_int),
        ("lewis", C.c_double * 16),
        ("cp", C.c_double * 16),
    ]


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (OpenMP, -O2, no fast-math)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < max(
        os.path.getmtime(_SRC), os.path.getmtime(os.path.join(_HERE, "lbfd_oracle.h"))
    ):
        tmp = _LIB + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared", "-Wall",
               "-o", tmp, _SRC, "-lm"]
        subprocess.check_call(cmd)
        os.replace(tmp, _LIB)
    return _LIB


def lib_path() -> str:
    return _LIB


_lib = None


def _load():
    global _lib
    if _lib is None:
        build()
        lib = C.CDLL(_LIB)
        dp = C.POINTER(C.c_double)
        lib.lbo_create.restype = C.c_void_p
        lib.lbo_create.argtypes = [C.POINTER(_Params), C.c_void_p, dp, dp, dp, dp, dp,
                                   C.c_char_p, C.c_int]
        lib.lbo_destroy.argtypes = [C.c_void_p]
        lib.lbo_step.argtypes = [C.c_void_p, C.c_long]
        lib.lbo_step.restype = C.c_int
        lib.lbo_level.argtypes = [C.c_void_p]
        lib.lbo_level.restype = C.c_long
        lib.lbo_set_active.argtypes = [C.c_void_p, C.c_void_p]
        lib.lbo_set_inflow.argtypes = [C.c_void_p, C.c_int, dp]
        lib.lbo_set_wall_links.argtypes = [C.c_void_p, C.c_long, C.c_void_p, C.c_void_p, dp]
        lib.lbo_set_wall_links.restype = C.c_int
        lib.lbo_set_image_points.argtypes = [C.c_void_p, C.c_long, C.c_void_p, C.c_void_p, dp]
        lib.lbo_set_image_points.restype = C.c_int
        lib.lbo_image_value.argtypes = [C.c_void_p, dp, dp, dp]
        lib.lbo_image_value.restype = C.c_int
        lib.lbo_set_inflow.restype = C.c_int
        lib.lbo_fields.argtypes = [C.c_void_p, dp, dp, dp, dp, dp]
        lib.lbo_diagnostics.argtypes = [C.c_void_p, dp]
        lib.lbo_get_pops.argtypes = [C.c_void_p, dp]
        lib.lbo_set_threads.argtypes = [C.c_int]
        lib.lbo_lattice.argtypes = [C.c_int, C.POINTER(C.c_int), dp]
        lib.lbo_feq.argtypes = [C.c_int, C.c_double, dp, dp]
        lib.lbo_geq.argtypes = [C.c_int, C.c_double, C.c_double, dp, dp]
        lib.lbo_central_moments.argtypes = [C.c_int, dp, dp, dp]
        lib.lbo_cumulants.argtypes = [C.c_int, dp, dp]
        lib.lbo_cumulants_inverse.argtypes = [C.c_int, dp, dp]
        lib.lbo_collide.argtypes = [C.POINTER(_Params), dp, dp, C.c_double, dp, dp]
        lib.lbo_source_xi.argtypes = [C.c_int, C.c_double, dp, dp, C.c_double, dp]
        lib.lbo_weno3.argtypes = [dp, C.c_double]
        lib.lbo_weno3.restype = C.c_double
        lib.lbo_d1.argtypes = [dp]
        lib.lbo_d1.restype = C.c_double
        lib.lbo_d2.argtypes = [dp]
        lib.lbo_d2.restype = C.c_double
        lib.lbo_chemistry.argtypes = [C.POINTER(_Params), C.c_double, dp, dp, dp]
        _lib = lib
    return _lib


def _dp(a):
    if a is None:
        return None
    return a.ctypes.data_as(C.POINTER(C.c_double))


def make_params(prob, **over) -> _Params:
    """Marshal a Problem into the oracle's parameter struct."""
    p = _Params()
    p.Q = prob.lattice
    p.nx, p.ny, p.nz = prob.nx, prob.ny, prob.nz
    for f in range(6):
        p.face[f] = FACE_CODES[prob.faces[f]]
        p.face_T[f] = prob.face_T[f]
    p.tau = prob.tau
    p.prandtl = prob.prandtl
    p.dt_phys = prob.dt_phys
    p.T_ref = prob.T_ref
    p.W_ref = prob.W_ref
    p.n_species = len(prob.W)
    for k, v in enumerate(prob.W):
        p.W[k] = v
    p.n_reactions = len(prob.reactions)
    for j, r in enumerate(prob.reactions):
        p.rx[j].n_react = len(r.reactants)
        for m, k in enumerate(r.reactants):
            p.rx[j].react[m] = k
        p.rx[j].A, p.rx[j].b, p.rx[j].Ta = r.A, r.b, r.Ta
        for k, v in enumerate(r.nu):
            p.rx[j].nu[k] = v
        p.rx[j].q = r.q
    for d in range(3):
        p.u_in[d] = prob.u_in[d]
    p.T_in = prob.T_in
    for k, v in enumerate(prob.Y_in):
        p.Y_in[k] = v
    p.omega3 = prob.omega3
    p.omega4 = prob.omega4
    p.eq_discrete = int(prob.eq_discrete)
    p.chem_substeps_max = prob.chem_substeps_max
    p.T_u, p.T_b = prob.T_u, prob.T_b
    p.collision = {"central_moments": 0, "cumulants": 1}[getattr(prob, "collision", "central_moments")]
    p.transport = {"unity_lewis": 0, "mixture_averaged": 1}[getattr(prob, "transport", "unity_lewis")]
    le = tuple(getattr(prob, "lewis", ()) or ())
    cp = tuple(getattr(prob, "cp", ()) or ())
    for k in range(len(prob.W)):
        p.lewis[k] = le[k] if k < len(le) else 1.0
        p.cp[k] = cp[k] if k < len(cp) else 1.0
    bf = over.pop("body_force", (0.0, 0.0, 0.0))
    for d in range(3):
        p.body_force[d] = bf[d]
    for k, v in over.items():
        setattr(p, k, v)
    return p


class Oracle:
    """Time-marching FP64 reference: ``Oracle(problem).step(n)``."""

    def __init__(self, prob, threads: int | None = None, **over):
        lib = _load()
        if threads:
            lib.lbo_set_threads(int(threads))
        self.prob = prob
        self.params = make_params(prob, **over)
        N = prob.nx * prob.ny * prob.nz
        self.N = N
        self.nsp = len(prob.W)
        mask = np.ascontiguousarray(prob.mask, dtype=np.uint8).reshape(-1)
        wall_T = np.ascontiguousarray(prob.wall_T, dtype=np.float64).reshape(-1)
        T0 = np.ascontiguousarray(prob.T0, dtype=np.float64).reshape(-1)
        Y0 = np.ascontiguousarray(prob.Y0, dtype=np.float64).reshape(-1)
        u0 = None if prob.u0 is None else np.ascontiguousarray(prob.u0, dtype=np.float64).reshape(-1)
        Ph0 = None if prob.Ph0 is None else np.ascontiguousarray(prob.Ph0, dtype=np.float64).reshape(-1)
        err = C.create_string_buffer(256)
        h = lib.lbo_create(C.byref(self.params), mask.ctypes.data, _dp(wall_T), _dp(T0), _dp(Y0),
                           _dp(u0), _dp(Ph0), err, 256)
        if not h:
            raise ValueError("oracle rejected the problem: " + err.value.decode())
        self._h = h
        self._lib = lib

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            self._lib.lbo_destroy(h)
            self._h = None

    def set_inflow(self, face: int, u=None):
        """Inlet velocity profile u [3, nz, ny] of x face 0 (-x) or 1 (+x);
        None restores the uniform inflow velocity."""
        pr = self.prob
        a = None if u is None else np.ascontiguousarray(u, dtype=np.float64).reshape(3 * pr.nz * pr.ny)
        if self._lib.lbo_set_inflow(self._h, int(face), _dp(a)) != 0:
            raise ValueError("inlet profiles are set on x faces 0 and 1")

    def set_wall_links(self, cell=None, direction=None, q=None):
        """Interpolated bounce-back on the listed links (fluid cell,
        direction toward the wall, wall fraction q); None clears."""
        if cell is None or len(cell) == 0:
            self._lib.lbo_set_wall_links(self._h, 0, None, None, None)
            return
        c = np.ascontiguousarray(cell, dtype=np.int64)
        d = np.ascontiguousarray(direction, dtype=np.int32)
        qq = np.ascontiguousarray(q, dtype=np.float64)
        if self._lib.lbo_set_wall_links(self._h, len(c), c.ctypes.data, d.ctypes.data, _dp(qq)) != 0:
            raise ValueError("wall link out of range")

    def set_image_points(self, cell=None, slot=None, image=None):
        """Shepard-reconstructed image points of the listed ghost nodes
        (fluid cell, slot = 4 axis + j for the offset (-2, -1, 1, 2)[j],
        image point [n, 3] in lattice coordinates); None clears."""
        if cell is None or len(cell) == 0:
            self._lib.lbo_set_image_points(self._h, 0, None, None, None)
            return
        c = np.ascontiguousarray(cell, dtype=np.int64)
        sl = np.ascontiguousarray(slot, dtype=np.int32)
        im = np.ascontiguousarray(image, dtype=np.float64).reshape(-1, 3)
        if len(im) != len(c) or len(sl) != len(c):
            raise ValueError("cell, slot and image lengths differ")
        if self._lib.lbo_set_image_points(self._h, len(c), c.ctypes.data, sl.ctypes.data, _dp(im)) != 0:
            raise ValueError("image point out of range or repeated")

    def image_value(self, x):
        """Shepard reconstruction (T, Y[n_species], nodes used) at the
        point x of the current level."""
        xx = np.ascontiguousarray(np.asarray(x, dtype=np.float64).reshape(3))
        T = np.zeros(1)
        Y = np.zeros(max(1, self.nsp))
        n = self._lib.lbo_image_value(self._h, _dp(xx), _dp(T), _dp(Y))
        return float(T[0]), Y[: self.nsp].copy(), int(n)

    def set_threads(self, n: int):
        """OpenMP threads of the following steps (process-wide)."""
        self._lib.lbo_set_threads(int(n))

    @property
    def level(self) -> int:
        return int(self._lib.lbo_level(self._h))

    def step(self, n: int = 1):
        self._lib.lbo_step(self._h, int(n))

    # A cell's state at level n+1 reads level n within this many cells
    # (pull sources one cell away, their stencils two further).
    CONE_STEP = 3

    def set_active(self, active):
        """Restrict later steps and fields() to the cells where ``active``
        (box-shaped, any dtype) is nonzero; None restores the whole box."""
        if active is None:
            self._active = None
            self._lib.lbo_set_active(self._h, None)
            return
        a = np.ascontiguousarray(np.asarray(active).reshape(-1) != 0, dtype=np.uint8)
        if a.size != self.N:
            raise ValueError("active set must cover the box")
        self._active = a  # kept alive while the C side holds the pointer
        self._lib.lbo_set_active(self._h, a.ctypes.data)

    def step_sampled(self, sample, n: int):
        """Advance n levels computing only the dependency cone of the cells
        where ``sample`` is true: the step to level k covers the cells within
        CONE_STEP (n - k) + 3 of the sample (cube, wrapped across the box),
        which leaves the sample's state -- and the stencil region P_h and u
        need -- equal to that of n full steps.  fields() then reports the
        sample cells (NaN elsewhere)."""
        from scipy.ndimage import maximum_filter
        sample = np.asarray(sample, dtype=bool).reshape(self.prob.nz, self.prob.ny, self.prob.nx)
        flat = self.prob.nz == 1
        for k in range(1, int(n) + 1):
            r = self.CONE_STEP * (int(n) - k) + 3
            size = (1 if flat else 2 * r + 1, 2 * r + 1, 2 * r + 1)
            self.set_active(maximum_filter(sample.astype(np.uint8), size=size, mode="wrap"))
            self.step(1)
        self.set_active(sample)

    def fields(self) -> dict:
        pr = self.prob
        shp = (pr.nz, pr.ny, pr.nx)
        N = self.N
        rho = np.empty(N)
        u = np.empty(3 * N)
        T = np.empty(N)
        Y = np.empty(self.nsp * N)
        Ph = np.empty(N)
        self._lib.lbo_fields(self._h, _dp(rho), _dp(u), _dp(T), _dp(Y), _dp(Ph))
        return {"rho": rho.reshape(shp), "u": u.reshape((3,) + shp), "T": T.reshape(shp),
                "Y": Y.reshape((self.nsp,) + shp), "Ph": Ph.reshape(shp)}

    def diagnostics(self) -> dict:
        out = np.empty(NDIAG)
        self._lib.lbo_diagnostics(self._h, _dp(out))
        return {"sum_g": out[0], "sum_xi": out[1], "mom": out[2:5].copy(),
                "max_sumY_err": out[5], "nonfinite": int(out[6]), "sum_theta": out[7],
                "hrr_idx": int(out[8]), "hrr_max": out[9], "wall_q": out[10],
                "fuel_rate": out[11], "fuel_mass_rate": out[12], "consumption_speed": out[13]}

    def objective(self, nsteps: int, kind: str = "wall_q", t_begin: int = 0, t_end: int | None = None) -> float:
        """Sum over the next nsteps levels, offsets t_begin <= t < t_end, of
        q(level) evaluated before each step: "wall_q" the wall heat flux
        diagnostic, "flame_x" the flame position nx - sum_theta / (fluid cells
        per x column), in cells."""
        pr = self.prob
        J = 0.0
        for t in range(int(nsteps)):
            if t >= t_begin and (t_end is None or t < t_end):
                d = self.diagnostics()
                if kind == "wall_q":
                    J += d["wall_q"]
                elif kind == "flame_x":
                    J += pr.nx - d["sum_theta"] / (pr.n_fluid / pr.nx)
                else:
                    raise ValueError(kind)
            self.step(1)
        return J

    def pops(self) -> np.ndarray:
        pr = self.prob
        g = np.empty(pr.lattice * self.N)
        self._lib.lbo_get_pops(self._h, _dp(g))
        return g.reshape((pr.lattice, pr.nz, pr.ny, pr.nx))


class single:
    """Single-operator entry points of the oracle (for its own pins)."""

    @staticmethod
    def lattice(Q):
        lib = _load()
        c = (C.c_int * (3 * Q))()
        w = np.empty(Q)
        lib.lbo_lattice(Q, c, _dp(w))
        return np.array(list(c), dtype=np.int64).reshape(Q, 3), w

    @staticmethod
    def feq(Q, rho, u):
        out = np.empty(Q)
        _load().lbo_feq(Q, rho, _dp(np.asarray(u, dtype=np.float64)), _dp(out))
        return out

    @staticmethod
    def geq(Q, Ph, rho, u):
        out = np.empty(Q)
        _load().lbo_geq(Q, Ph, rho, _dp(np.asarray(u, dtype=np.float64)), _dp(out))
        return out

    @staticmethod
    def central_moments(Q, h, u):
        out = np.empty(Q)
        _load().lbo_central_moments(Q, _dp(np.ascontiguousarray(h, dtype=np.float64)),
                                     _dp(np.asarray(u, dtype=np.float64)), _dp(out))
        return out

    @staticmethod
    def cumulants(Q, kap):
        out = np.empty(Q)
        _load().lbo_cumulants(Q, _dp(np.ascontiguousarray(kap, dtype=np.float64)), _dp(out))
        return out

    @staticmethod
    def cumulants_inverse(Q, cum):
        out = np.empty(Q)
        _load().lbo_cumulants_inverse(Q, _dp(np.ascontiguousarray(cum, dtype=np.float64)), _dp(out))
        return out

    @staticmethod
    def collide(params, g, xi, rho, u):
        out = np.empty(params.Q)
        _load().lbo_collide(C.byref(params), _dp(np.ascontiguousarray(g, dtype=np.float64)),
                             _dp(np.ascontiguousarray(xi, dtype=np.float64)), rho,
                             _dp(np.asarray(u, dtype=np.float64)), _dp(out))
        return out

    @staticmethod
    def source_xi(Q, rho, u, grad_rho, Lam):
        out = np.empty(Q)
        _load().lbo_source_xi(Q, rho, _dp(np.asarray(u, dtype=np.float64)),
                               _dp(np.asarray(grad_rho, dtype=np.float64)), Lam, _dp(out))
        return out

    @staticmethod
    def weno3(phi5, u):
        return _load().lbo_weno3(_dp(np.ascontiguousarray(phi5, dtype=np.float64)), u)

    @staticmethod
    def d1(phi5):
        return _load().lbo_d1(_dp(np.ascontiguousarray(phi5, dtype=np.float64)))

    @staticmethod
    def d2(phi5):
        return _load().lbo_d2(_dp(np.ascontiguousarray(phi5, dtype=np.float64)))

    @staticmethod
    def chemistry(params, T, Y):
        ns = params.n_species
        sT = C.c_double()
        sY = np.empty(ns)
        _load().lbo_chemistry(C.byref(params), T, _dp(np.ascontiguousarray(Y, dtype=np.float64)),
                               C.byref(sT), _dp(sY))
        return sT.value, sY
