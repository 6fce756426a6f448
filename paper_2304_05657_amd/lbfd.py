"""Thin ctypes binding of ``liblbfd.so`` (C ABI in ``include/lbfd.h``).

Argument marshalling only: every part of the step runs in the library's
HIP kernels.  The library must have been built (``python -m
paper_2304_05657_amd.build``); if it is missing or cannot be loaded the
import of :class:`Solver` fails loudly -- there is no CPU fallback.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "liblbfd.so")

MAX_SPECIES = 16
MAX_REACTIONS = 32
FP64, MIXED_FP32, MIXED_FP16 = 0, 1, 2
PRECISIONS = {"fp64": FP64, "fp32": MIXED_FP32, "fp16": MIXED_FP16}
FACE_CODES = {"periodic": 0, "wall": 1, "inflow": 2, "outflow": 3, "wall_adiabatic": 4}
ERRORS = {0: "LBFD_OK", -1: "LBFD_EINVAL", -2: "LBFD_ENOMEM", -3: "LBFD_EDEVICE",
          -4: "LBFD_ENONFINITE", -5: "LBFD_ESTATE"}

EXPORTS = ("lbfd_init", "lbfd_step", "lbfd_sync", "lbfd_level", "lbfd_read_fields",
           "lbfd_diagnostics", "lbfd_set_wall_temperature", "lbfd_state_size",
           "lbfd_save_state", "lbfd_load_state", "lbfd_time_steps", "lbfd_time_kernels",
           "lbfd_cell_counts", "lbfd_step_launches", "lbfd_set_reaction", "lbfd_chem_kernel", "lbfd_set_objective",
           "lbfd_objective", "lbfd_adjoint", "lbfd_set_inflow", "lbfd_hold_flame", "lbfd_set_wall_links",
           "lbfd_set_image_points", "lbfd_init_dev", "lbfd_read_fields_dev", "lbfd_adjoint_dev",
           "lbfd_objective_static", "lbfd_step_tangent", "lbfd_step_adjoint",
           "lbfd_destroy",
           "lbfd_strerror", "lbfd_last_error")
# species transport models (lbfd_params.transport)
TRANSPORTS = {"unity_lewis": 0, "mixture_averaged": 1}
# collision operators (lbfd_params.collision)
COLLISIONS = {"central_moments": 0, "cumulants": 1}
# objective kinds (lbfd_set_objective)
OBJECTIVES = {"wall_q": 0, "flame_x": 1}


class LbfdError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("%s: %s" % (ERRORS.get(code, code), msg))
        self.code = code


class Reaction(C.Structure):
    _fields_ = [("n_react", C.c_int), ("react", C.c_int * 4), ("A", C.c_double),
                ("b", C.c_double), ("Ta", C.c_double), ("nu_mass", C.c_double * MAX_SPECIES),
                ("q_over_cp", C.c_double)]


class Params(C.Structure):
    _fields_ = [
        ("lattice", C.c_int), ("nx", C.c_int), ("ny", C.c_int), ("nz", C.c_int),
        ("precision", C.c_int), ("face", C.c_int * 6), ("face_T", C.c_double * 6),
        ("tau", C.c_double), ("prandtl", C.c_double), ("dt_phys", C.c_double),
        ("T_ref", C.c_double), ("W_ref", C.c_double), ("n_species", C.c_int),
        ("W", C.c_double * MAX_SPECIES), ("n_reactions", C.c_int),
        ("rxn", C.POINTER(Reaction)), ("u_in", C.c_double * 3), ("T_in", C.c_double),
        ("Y_in", C.c_double * MAX_SPECIES), ("omega3", C.c_double), ("omega4", C.c_double),
        ("chem_substeps_max", C.c_int), ("check_every", C.c_int),
        ("T_u", C.c_double), ("T_b", C.c_double), ("collision", C.c_int),
        ("transport", C.c_int), ("lewis", C.c_double * 16), ("cp", C.c_double * 16),
    ]


class Diag(C.Structure):
    _fields_ = [("sum_g", C.c_double), ("sum_xi", C.c_double), ("mom", C.c_double * 3),
                ("max_abs_sumY_minus_1", C.c_double), ("nonfinite", C.c_int64),
                ("sum_theta", C.c_double), ("hrr_idx", C.c_int64), ("hrr_max", C.c_double),
                ("wall_q", C.c_double), ("fuel_rate", C.c_double), ("step", C.c_int64),
                ("fuel_mass_rate", C.c_double), ("consumption_speed", C.c_double)]


_lib = None


def load_library():
    """Load liblbfd.so; raises if it has not been built.  When torch is
    importable it is imported first, so that the library binds to the HIP
    runtime torch has loaded (one runtime per process: torch's streams and
    the library's allocations then belong to the same one)."""
    global _lib
    if _lib is not None:
        return _lib
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    if not os.path.exists(LIB_PATH):
        raise ImportError("liblbfd.so is not built (run python -m paper_2304_05657_amd.build); "
                          "the GPU library has no CPU fallback")
    lib = C.CDLL(LIB_PATH)
    vp, dp = C.c_void_p, C.POINTER(C.c_double)
    lib.lbfd_init.argtypes = [C.POINTER(Params), vp, dp, dp, dp, dp, dp, vp, C.POINTER(vp)]
    lib.lbfd_step.argtypes = [vp, C.c_int64]
    lib.lbfd_sync.argtypes = [vp]
    lib.lbfd_level.argtypes = [vp]
    lib.lbfd_level.restype = C.c_int64
    lib.lbfd_read_fields.argtypes = [vp, dp, dp, dp, dp, dp]
    lib.lbfd_init_dev.argtypes = [C.POINTER(Params), vp, vp, vp, vp, vp, vp, vp, C.POINTER(vp)]
    lib.lbfd_read_fields_dev.argtypes = [vp, vp, vp, vp, vp, vp]
    lib.lbfd_adjoint_dev.argtypes = [vp, C.c_int64, C.c_int, dp, vp, dp, dp]
    lib.lbfd_diagnostics.argtypes = [vp, C.POINTER(Diag)]
    lib.lbfd_set_wall_temperature.argtypes = [vp, dp]
    lib.lbfd_state_size.argtypes = [vp, C.POINTER(C.c_size_t)]
    lib.lbfd_save_state.argtypes = [vp, vp, C.c_size_t]
    lib.lbfd_load_state.argtypes = [vp, vp, C.c_size_t]
    lib.lbfd_time_steps.argtypes = [vp, C.c_int64, dp]
    lib.lbfd_time_kernels.argtypes = [vp, C.c_int64, dp, dp, dp]
    lib.lbfd_cell_counts.argtypes = [vp, C.POINTER(C.c_int64), C.POINTER(C.c_int64)]
    lib.lbfd_step_launches.argtypes = [vp]
    lib.lbfd_step_launches.restype = C.c_int
    lib.lbfd_set_reaction.argtypes = [vp, C.c_int, C.c_double, C.c_double, C.c_double]
    lib.lbfd_chem_kernel.argtypes = [vp, C.c_char_p, C.c_size_t]
    lib.lbfd_set_objective.argtypes = [vp, C.c_int, C.c_int64, C.c_int64]
    lib.lbfd_set_inflow.argtypes = [vp, C.c_int, dp]
    lib.lbfd_set_wall_links.argtypes = [vp, C.c_int64, vp, vp, dp]
    lib.lbfd_set_image_points.argtypes = [vp, C.c_int64, vp, vp, dp]
    lib.lbfd_hold_flame.argtypes = [vp, C.c_int64, C.c_int, C.c_double, C.c_double, dp, dp]
    lib.lbfd_objective.argtypes = [vp, C.c_int64, dp]
    lib.lbfd_objective_static.argtypes = [vp, C.c_int64, dp]
    lib.lbfd_adjoint.argtypes = [vp, C.c_int64, C.c_int, dp, dp, dp, dp]
    lib.lbfd_step_tangent.argtypes = [vp, dp, dp, dp, dp, dp, dp, dp, dp]
    lib.lbfd_step_adjoint.argtypes = [vp, dp, dp, C.c_double, dp, dp, dp, dp, dp]
    lib.lbfd_destroy.argtypes = [vp]
    lib.lbfd_destroy.restype = None
    lib.lbfd_strerror.argtypes = [C.c_int]
    lib.lbfd_strerror.restype = C.c_char_p
    lib.lbfd_last_error.argtypes = []
    lib.lbfd_last_error.restype = C.c_char_p
    _lib = lib
    return lib


def _check(lib, rc):
    if rc != 0:
        raise LbfdError(rc, lib.lbfd_last_error().decode())


def _dp(a):
    return None if a is None else a.ctypes.data_as(C.POINTER(C.c_double))


def make_params(prob, precision="fp64", check_every: int = 0):
    """Marshal a workloads.Problem into lbfd_params (+ the reaction array
    that must stay alive while the params are used)."""
    p = Params()
    p.lattice = prob.lattice
    p.nx, p.ny, p.nz = prob.nx, prob.ny, prob.nz
    p.precision = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
    for f in range(6):
        p.face[f] = FACE_CODES[prob.faces[f]]
        p.face_T[f] = prob.face_T[f]
    p.tau, p.prandtl, p.dt_phys = prob.tau, prob.prandtl, prob.dt_phys
    p.T_ref, p.W_ref = prob.T_ref, prob.W_ref
    p.n_species = len(prob.W)
    for k, v in enumerate(prob.W):
        p.W[k] = v
    rx = (Reaction * max(1, len(prob.reactions)))()
    for j, r in enumerate(prob.reactions):
        rx[j].n_react = len(r.reactants)
        for m, k in enumerate(r.reactants):
            rx[j].react[m] = k
        rx[j].A, rx[j].b, rx[j].Ta, rx[j].q_over_cp = r.A, r.b, r.Ta, r.q
        for k, v in enumerate(r.nu):
            rx[j].nu_mass[k] = v
    p.n_reactions = len(prob.reactions)
    p.rxn = C.cast(rx, C.POINTER(Reaction))
    for d in range(3):
        p.u_in[d] = prob.u_in[d]
    p.T_in = prob.T_in
    for k, v in enumerate(prob.Y_in):
        p.Y_in[k] = v
    p.omega3, p.omega4 = prob.omega3, prob.omega4
    p.chem_substeps_max = prob.chem_substeps_max
    p.check_every = check_every
    p.T_u, p.T_b = prob.T_u, prob.T_b
    p.collision = COLLISIONS[getattr(prob, "collision", "central_moments")]
    p.transport = TRANSPORTS[getattr(prob, "transport", "unity_lewis")]
    le = tuple(getattr(prob, "lewis", ()) or ())
    cp = tuple(getattr(prob, "cp", ()) or ())
    for k in range(len(prob.W)):
        p.lewis[k] = le[k] if k < len(le) else 1.0
        p.cp[k] = cp[k] if k < len(cp) else 1.0
    if prob.eq_discrete:
        raise ValueError("the GPU library relaxes toward Maxwellian central moments only")
    return p, rx


class Solver:
    """One GPU context: ``Solver(problem, precision='fp64').step(n)``.

    ``stream`` is a raw hipStream_t handle (int); by default the current
    torch stream of the current device is used when torch is importable,
    else the null stream."""

    def __init__(self, prob, precision="fp64", check_every: int = 0, stream=None, from_device: bool = False):
        lib = load_library()
        if stream is None:
            stream = _torch_stream()
        self.prob = prob
        self.precision = precision
        self._params, self._rx = make_params(prob, precision, check_every)
        N = prob.N
        self.N = N
        self.nsp = len(prob.W)
        self.dim = 2 if prob.lattice == 9 else 3
        mask = np.ascontiguousarray(prob.mask, dtype=np.uint8).reshape(-1)
        wall_T = np.ascontiguousarray(prob.wall_T, dtype=np.float64).reshape(-1)
        T0 = np.ascontiguousarray(prob.T0, dtype=np.float64).reshape(-1)
        Y0 = np.ascontiguousarray(prob.Y0, dtype=np.float64).reshape(-1)
        u0 = None if prob.u0 is None else np.ascontiguousarray(
            np.asarray(prob.u0, dtype=np.float64)[: self.dim]).reshape(-1)
        Ph0 = None if prob.Ph0 is None else np.ascontiguousarray(prob.Ph0, dtype=np.float64).reshape(-1)
        h = C.c_void_p()
        if from_device:
            # the same arrays as torch tensors on the current device (lbfd_init_dev)
            import torch
            dev = [None if a is None else torch.from_numpy(a).cuda() for a in (mask, wall_T, T0, Y0, u0, Ph0)]
            ptr = [None if t is None else C.c_void_p(t.data_ptr()) for t in dev]
            rc = lib.lbfd_init_dev(C.byref(self._params), *ptr, C.c_void_p(stream or 0), C.byref(h))
        else:
            rc = lib.lbfd_init(C.byref(self._params), mask.ctypes.data, _dp(wall_T), _dp(T0), _dp(Y0),
                               _dp(u0), _dp(Ph0), C.c_void_p(stream or 0), C.byref(h))
        _check(lib, rc)
        self._h = h
        self._lib = lib

    def close(self):
        h = getattr(self, "_h", None)
        if h:
            self._lib.lbfd_destroy(h)
            self._h = None

    __del__ = close

    @property
    def level(self) -> int:
        return int(self._lib.lbfd_level(self._h))

    def step(self, n: int = 1):
        _check(self._lib, self._lib.lbfd_step(self._h, int(n)))

    def sync(self):
        _check(self._lib, self._lib.lbfd_sync(self._h))

    def time_steps(self, n: int) -> float:
        ms = C.c_double()
        _check(self._lib, self._lib.lbfd_time_steps(self._h, int(n), C.byref(ms)))
        return ms.value

    def time_kernels(self, n: int) -> tuple:
        """(ms interior kernel, ms boundary kernel, ms chemistry launch)
        summed over n serialised steps."""
        a, b, c = C.c_double(), C.c_double(), C.c_double()
        _check(self._lib, self._lib.lbfd_time_kernels(self._h, int(n), C.byref(a), C.byref(b), C.byref(c)))
        return a.value, b.value, c.value

    def cell_counts(self) -> tuple:
        """(fluid cells, cells on the boundary-cell path)."""
        a, b = C.c_int64(), C.c_int64()
        _check(self._lib, self._lib.lbfd_cell_counts(self._h, C.byref(a), C.byref(b)))
        return a.value, b.value

    def step_launches(self) -> int:
        """Kernel launches per step (1: one launch covers every cell)."""
        n = self._lib.lbfd_step_launches(self._h)
        _check(self._lib, min(n, 0))
        return n

    def set_reaction(self, j: int, A: float, b: float, Ta: float):
        _check(self._lib, self._lib.lbfd_set_reaction(self._h, int(j), float(A), float(b), float(Ta)))

    def chem_kernel(self):
        """(specialised, note): whether the Arrhenius source of this
        mechanism runs in the kernel specialised to its structure, and a
        note on the kernel in use (lbfd_chem_kernel)."""
        buf = C.create_string_buffer(512)
        r = self._lib.lbfd_chem_kernel(self._h, buf, len(buf))
        if r < 0:
            _check(self._lib, r)
        return bool(r), buf.value.decode()

    def set_objective(self, kind: str = "wall_q", t_begin: int = 0, t_end: int | None = None):
        """Objective of objective() / adjoint(): the sum of q(level) over the
        level offsets t_begin <= t < t_end of those calls, q = "wall_q" (wall
        heat flux) or "flame_x" (flame position, cells)."""
        t_end = (1 << 63) - 1 if t_end is None else int(t_end)
        _check(self._lib, self._lib.lbfd_set_objective(self._h, OBJECTIVES[kind], int(t_begin), t_end))

    def objective(self, nsteps: int) -> float:
        """The selected objective over the next nsteps levels (forward only)."""
        J = C.c_double()
        _check(self._lib, self._lib.lbfd_objective(self._h, int(nsteps), C.byref(J)))
        return J.value

    def objective_static(self, nsteps: int) -> float:
        """objective() through lbfd_objective_static: no device allocation,
        the library's static per-GPU scratch array instead."""
        J = C.c_double()
        _check(self._lib, self._lib.lbfd_objective_static(self._h, int(nsteps), C.byref(J)))
        return J.value

    def adjoint(self, nsteps: int, K: int, device: bool = False):
        """(J, dJ/dwall_T [nz, ny, nx], dJ/dA [n_rx], dJ/dTa [n_rx]) over the next
        nsteps levels, checkpointing every K steps; device=True returns
        dJ/dwall_T as a torch tensor on the current device (lbfd_adjoint_dev)."""
        pr = self.prob
        J = C.c_double()
        nrx = max(1, len(pr.reactions))
        gA, gTa = np.zeros(nrx), np.zeros(nrx)
        if device:
            import torch
            gW = torch.zeros(self.N, dtype=torch.float64, device="cuda")
            _check(self._lib, self._lib.lbfd_adjoint_dev(self._h, int(nsteps), int(K), C.byref(J),
                                                         C.c_void_p(gW.data_ptr()), _dp(gA), _dp(gTa)))
        else:
            gW = np.zeros(self.N)
            _check(self._lib, self._lib.lbfd_adjoint(self._h, int(nsteps), int(K), C.byref(J), _dp(gW), _dp(gA),
                                                     _dp(gTa)))
        return J.value, gW.reshape((pr.nz, pr.ny, pr.nx)), gA[: len(pr.reactions)], gTa[: len(pr.reactions)]

    def step_tangent(self, dpop, dsc, dwallT=None, dA=None, dTa=None):
        """Jacobian-vector product of one FP64 step at the current level
        (lbfd_step_tangent): tangents dpop [Q, N], dsc [1 + n_species, N]
        (T, Y_k), optional dwallT [N], dA, dTa [n_reactions] -> (dpop_out,
        dsc_out, dq).  The context does not advance."""
        pop = np.ascontiguousarray(dpop, dtype=np.float64)
        sc = np.ascontiguousarray(dsc, dtype=np.float64)
        opt = [None if v is None else np.ascontiguousarray(v, dtype=np.float64) for v in (dwallT, dA, dTa)]
        po, so = np.zeros_like(pop), np.zeros_like(sc)
        dq = C.c_double()
        _check(self._lib, self._lib.lbfd_step_tangent(self._h, _dp(pop), _dp(sc),
                                                      *(None if v is None else _dp(v) for v in opt),
                                                      _dp(po), _dp(so), C.byref(dq)))
        return po, so, dq.value

    def step_adjoint(self, lam_pop, lam_sc, wq: float = 0.0):
        """Vector-Jacobian product of one FP64 step at the current level
        (lbfd_step_adjoint): adjoints of the step's outputs lam_pop [Q, N],
        lam_sc [1 + n_species, N] and the weight wq of the level's objective
        term -> (lam_pop_in, lam_sc_in, dJ/dwall_T [N], dJ/dA, dJ/dTa)."""
        lp = np.ascontiguousarray(lam_pop, dtype=np.float64)
        ls = np.ascontiguousarray(lam_sc, dtype=np.float64)
        nrx = max(1, len(self.prob.reactions))
        po, so, gW = np.zeros_like(lp), np.zeros_like(ls), np.zeros(self.N)
        gA, gTa = np.zeros(nrx), np.zeros(nrx)
        _check(self._lib, self._lib.lbfd_step_adjoint(self._h, _dp(lp), _dp(ls), C.c_double(wq), _dp(po), _dp(so),
                                                      _dp(gW), _dp(gA), _dp(gTa)))
        n = len(self.prob.reactions)
        return po, so, gW, gA[:n], gTa[:n]

    def fields(self, device: bool = False) -> dict:
        """rho, u [3], T, Y [n_species], Ph of the current level (FP64): numpy
        arrays, or with device=True torch tensors on the current device
        (lbfd_read_fields_dev)."""
        pr = self.prob
        shp = (pr.nz, pr.ny, pr.nx)
        N = self.N
        if device:
            import torch
            out = {k: torch.empty(n * N, dtype=torch.float64, device="cuda")
                   for k, n in (("rho", 1), ("u", self.dim), ("T", 1), ("Y", self.nsp), ("Ph", 1))}
            _check(self._lib, self._lib.lbfd_read_fields_dev(self._h, *(C.c_void_p(out[k].data_ptr())
                                                                      for k in ("rho", "u", "T", "Y", "Ph"))))
            u3 = torch.zeros((3,) + shp, dtype=torch.float64, device="cuda")
            u3[: self.dim] = out["u"].reshape((self.dim,) + shp)
            return {"rho": out["rho"].reshape(shp), "u": u3, "T": out["T"].reshape(shp),
                    "Y": out["Y"].reshape((self.nsp,) + shp), "Ph": out["Ph"].reshape(shp)}
        rho, T, Ph = np.empty(N), np.empty(N), np.empty(N)
        u = np.empty(self.dim * N)
        Y = np.empty(self.nsp * N)
        _check(self._lib, self._lib.lbfd_read_fields(self._h, _dp(rho), _dp(u), _dp(T), _dp(Y), _dp(Ph)))
        u3 = np.zeros((3,) + shp)
        u3[: self.dim] = u.reshape((self.dim,) + shp)
        return {"rho": rho.reshape(shp), "u": u3, "T": T.reshape(shp),
                "Y": Y.reshape((self.nsp,) + shp), "Ph": Ph.reshape(shp)}

    def diagnostics(self) -> dict:
        d = Diag()
        _check(self._lib, self._lib.lbfd_diagnostics(self._h, C.byref(d)))
        return {"sum_g": d.sum_g, "sum_xi": d.sum_xi, "mom": np.array(list(d.mom)),
                "max_sumY_err": d.max_abs_sumY_minus_1, "nonfinite": int(d.nonfinite),
                "sum_theta": d.sum_theta, "hrr_idx": int(d.hrr_idx), "hrr_max": d.hrr_max,
                "wall_q": d.wall_q, "fuel_rate": d.fuel_rate, "step": int(d.step),
                "fuel_mass_rate": d.fuel_mass_rate, "consumption_speed": d.consumption_speed}

    def set_wall_links(self, cell=None, direction=None, q=None):
        """Interpolated bounce-back on the listed links (fluid cell, direction
        toward the wall, wall fraction q), e.g. workloads.wall_links(prob);
        None clears."""
        if cell is None or len(cell) == 0:
            _check(self._lib, self._lib.lbfd_set_wall_links(self._h, 0, None, None, None))
            return
        c = np.ascontiguousarray(cell, dtype=np.int64)
        d = np.ascontiguousarray(direction, dtype=np.int32)
        qq = np.ascontiguousarray(q, dtype=np.float64)
        _check(self._lib, self._lib.lbfd_set_wall_links(self._h, len(c), c.ctypes.data, d.ctypes.data, _dp(qq)))

    def set_image_points(self, cell=None, slot=None, image=None):
        """Shepard-reconstructed image points of ghost nodes on curved walls
        (boundary fluid cell, slot = 4 axis + j for the stencil offset
        (-2, -1, 1, 2)[j], image point [n, 3] in lattice coordinates), e.g.
        workloads.image_points(prob); None clears."""
        if cell is None or len(cell) == 0:
            _check(self._lib, self._lib.lbfd_set_image_points(self._h, 0, None, None, None))
            return
        c = np.ascontiguousarray(cell, dtype=np.int64)
        sl = np.ascontiguousarray(slot, dtype=np.int32)
        im = np.ascontiguousarray(image, dtype=np.float64).reshape(-1, 3)
        if len(sl) != len(c) or len(im) != len(c):
            raise ValueError("cell, slot and image lengths differ")
        _check(self._lib, self._lib.lbfd_set_image_points(self._h, len(c), c.ctypes.data, sl.ctypes.data, _dp(im)))

    def set_inflow(self, face: int, u=None):
        """Inlet velocity profile u [3, nz, ny] of x face 0 (-x) or 1 (+x),
        which must be an inflow face; None restores the uniform inflow."""
        pr = self.prob
        a = None if u is None else np.ascontiguousarray(u, dtype=np.float64).reshape(3 * pr.nz * pr.ny)
        _check(self._lib, self._lib.lbfd_set_inflow(self._h, int(face), _dp(a)))

    def hold_flame(self, nsteps: int, every: int, x_target: float, gain: float):
        """Run nsteps steps holding the flame at x_target (cells) by scaling
        the inlet profile after every `every` steps; returns the per-cycle
        (mean inlet velocity, flame position) arrays."""
        n = int(nsteps) // int(every)
        U, X = np.zeros(max(n, 1)), np.zeros(max(n, 1))
        _check(self._lib, self._lib.lbfd_hold_flame(self._h, int(nsteps), int(every), float(x_target), float(gain),
                                                    _dp(U), _dp(X)))
        return U[:n], X[:n]

    def set_wall_temperature(self, wall_T):
        a = np.ascontiguousarray(wall_T, dtype=np.float64).reshape(-1)
        _check(self._lib, self._lib.lbfd_set_wall_temperature(self._h, _dp(a)))

    def save_state(self) -> bytes:
        n = C.c_size_t()
        _check(self._lib, self._lib.lbfd_state_size(self._h, C.byref(n)))
        buf = (C.c_char * n.value)()
        _check(self._lib, self._lib.lbfd_save_state(self._h, buf, n))
        return bytes(buf)

    def load_state(self, blob: bytes):
        buf = C.create_string_buffer(blob, len(blob))
        _check(self._lib, self._lib.lbfd_load_state(self._h, buf, len(blob)))


def _torch_stream():
    try:
        import torch
    except ImportError:
        return 0
    if not torch.cuda.is_available():
        return 0
    return int(torch.cuda.current_stream().cuda_stream)


def wall_heat_flux_objective(solver: Solver, state: bytes, nsteps: int, K: int, wall_T, A, Ta):
    """Differentiable time-integrated wall heat flux J(wall_T, A, Ta) of
    reaction 0 over nsteps steps from the checkpoint `state`, as a torch
    scalar; its backward uses the library's discrete adjoint."""
    import torch

    class _WallHeatFlux(torch.autograd.Function):
        @staticmethod
        def forward(ctx, wall_T, A, Ta):
            solver.load_state(state)
            solver.set_wall_temperature(wall_T.detach().to(torch.float64).cpu().numpy())
            r = solver.prob.reactions[0]
            solver.set_reaction(0, float(A), r.b, float(Ta))
            on_gpu = wall_T.is_cuda
            J, gW, gA, gTa = solver.adjoint(nsteps, K, device=on_gpu)
            gW = gW if on_gpu else torch.from_numpy(gW)
            ctx.save_for_backward(gW.to(wall_T.dtype), torch.tensor(gA[0], dtype=A.dtype),
                                  torch.tensor(gTa[0], dtype=Ta.dtype))
            return torch.tensor(J, dtype=torch.float64)

        @staticmethod
        def backward(ctx, gJ):
            gW, gA, gTa = ctx.saved_tensors
            return gJ.to(gW.dtype) * gW, gJ.to(gA.dtype) * gA, gJ.to(gTa.dtype) * gTa

    return _WallHeatFlux.apply(wall_T, A, Ta)
