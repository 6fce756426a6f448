"""Error contract of the C ABI: lbfd_init rejects an invalid configuration
with LBFD_EINVAL and a message, before any device call, so these run on
the CPU through the real library (the binding raises LbfdError)."""
import numpy as np
import pytest

from paper_2304_05657_amd import workloads as W

EINVAL = -1


def _small():
    return W.channel_flame(nx=32, ny=12, front_x=10.0, name="abi_err")


def _reject(prob, message, precision="fp64"):
    from paper_2304_05657_amd.lbfd import LbfdError, Solver
    with pytest.raises(LbfdError) as e:
        Solver(prob, precision=precision)
    assert e.value.code == EINVAL
    assert message in str(e.value), str(e.value)


def test_tau_at_one_half():
    _reject(_small().replace(tau=0.5), "tau must exceed 1/2")


def test_diffusivity_above_stability_bound():
    # alpha = cs^2 (tau - 1/2) / Pr = 0.333 > 3/16 in 2-D
    _reject(_small().replace(prandtl=0.1), "explicit stability bound")


def test_mass_fractions_must_sum_to_one():
    p = _small()
    Y0 = p.Y0.copy()
    Y0[0, 0, 5, 7] += 1e-9
    _reject(p.replace(Y0=Y0), "do not sum to 1")


def test_reaction_must_conserve_mass():
    p = _small()
    r = p.reactions[0]
    nu = list(r.nu)
    nu[0] += 1e-6
    _reject(p.replace(reactions=[W.Reaction(r.reactants, r.A, r.b, r.Ta, tuple(nu), r.q)]),
            "does not conserve mass")


def test_no_fluid_cell():
    p = _small()
    _reject(p.replace(mask=np.ones_like(p.mask)), "no fluid cell")


def test_bad_mask_value():
    p = _small()
    m = p.mask.copy()
    m[0, 6, 6] = 7
    _reject(p.replace(mask=m), "bad mask value")


def test_nonpositive_temperature():
    p = _small()
    T0 = p.T0.copy()
    T0[0, 6, 6] = 0.0
    _reject(p.replace(T0=T0), "temperature must be positive")


def test_outflow_only_on_x_faces():
    p = _small()
    _reject(p.replace(faces=("periodic", "periodic", "outflow", "wall", "periodic", "periodic")),
            "only x faces may be OUTFLOW")


def test_d2q9_needs_one_layer():
    p = _small()
    _reject(p.replace(nz=2, mask=np.repeat(p.mask, 2, 0), wall_T=np.repeat(p.wall_T, 2, 0),
                      T0=np.repeat(p.T0, 2, 0), Y0=np.repeat(p.Y0, 2, 1)), "D2Q9 needs nz == 1")


def test_configuration_without_a_kernel():
    # FP16 population storage is built for 4 and 9 species (and D3Q27 9), not D2Q9 with 2
    p = _small()
    two = W.Reaction((0, 1), 1e9, 0.0, 15000.0, (-0.2, 0.2), 3.0e4)
    p = p.replace(W=(16.0, 32.0), Y_in=(0.5, 0.5), reactions=[two],
                  Y0=np.stack([np.full(p.mask.shape, 0.5), np.full(p.mask.shape, 0.5)]))
    _reject(p, "no kernel built", precision="fp16")


def test_mixture_transport_parameters():
    p = _small().replace(transport="mixture_averaged", lewis=(1.0, 0.0, 1.0, 1.0))
    _reject(p, "Lewis number and heat capacity must be positive")
    p = _small().replace(transport="mixture_averaged", cp=(1.0, 1.0, -2.0, 1.0))
    _reject(p, "Lewis number and heat capacity must be positive")
    # alpha = 0.0476 at tau 0.6: Le 0.2 puts D_k above 3/16
    p = _small().replace(transport="mixture_averaged", lewis=(0.2, 1.0, 1.0, 1.0))
    _reject(p, "above the explicit stability bound")


def test_box_beyond_the_maximum_size():
    """Boxes of 2^29 cells or more are rejected before any input array is
    read (the arrays passed here are those of a small box)."""
    import ctypes as C
    from paper_2304_05657_amd import lbfd as L
    lib = L.load_library()
    prob = _small()
    p, rx = L.make_params(prob)
    p.lattice, p.nx, p.ny, p.nz = 27, 1024, 512, 1024
    mask = np.zeros(prob.N, np.uint8)
    T0 = np.full(prob.N, 300.0)
    Y0 = np.full(4 * prob.N, 0.25)
    h = C.c_void_p()
    rc = lib.lbfd_init(C.byref(p), mask.ctypes.data, None, L._dp(T0), L._dp(Y0), None, None, None, C.byref(h))
    assert rc == EINVAL and not h.value
    assert "box too large" in lib.lbfd_last_error().decode()
    rc = lib.lbfd_init_dev(C.byref(p), mask.ctypes.data, None, T0.ctypes.data, Y0.ctypes.data, None, None, None,
                           C.byref(h))
    assert rc == EINVAL and not h.value
    assert "box too large" in lib.lbfd_last_error().decode()
