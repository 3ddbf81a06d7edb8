"""ctypes wrapper of the C oracle (test infrastructure only; see __init__)."""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass, fields

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")

COUPLED, ISOTHERMAL, THERMAL_ONLY = 0, 1, 2


class OracleError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"oracle error {code}: {msg}")
        self.code = code


def _stale() -> bool:
    """True when the library is missing or older than a C source or header."""
    if not os.path.exists(_LIB_PATH):
        return True
    t = os.path.getmtime(_LIB_PATH)
    return any(os.path.getmtime(os.path.join(_HERE, n)) > t
               for n in os.listdir(_HERE) if n.endswith((".c", ".h")))


def _load():
    if _stale():
        from . import build as _build

        _build.build()
    return C.CDLL(_LIB_PATH)


lib = _load()

_d = C.c_double
_pd = C.POINTER(C.c_double)
_i64 = C.c_int64


class _CParams(C.Structure):
    _fields_ = [
        ("nx", C.c_int32), ("ny", C.c_int32),
        ("a", _d), ("b", _d), ("R", _d), ("omega", _d), ("Ts_over_Tc", _d),
        ("G", _d), ("sigma", _d),
        ("s_rho", _d), ("s_e", _d), ("s_zeta", _d), ("s_j", _d), ("s_q", _d),
        ("nu_L", _d), ("nu_V", _d), ("rho_L", _d), ("rho_V", _d),
        ("cv", _d), ("cv_chi", _d), ("g", _d), ("Gw_bottom", _d), ("Gw_top", _d),
        ("periodic_y", C.c_int32), ("thermal_mode", C.c_int32), ("ghost_layer", C.c_int32),
    ]


@dataclass
class Params:
    """Model parameters in lattice units (defaults: Sec. 3.1 of the paper,
    a = 2/49 as in the benchmark workloads)."""
    nx: int = 128
    ny: int = 64
    a: float = 2.0 / 49.0
    b: float = 2.0 / 21.0
    R: float = 1.0
    omega: float = 0.344
    Ts_over_Tc: float = 0.86
    G: float = -1.0
    sigma: float = 1.2
    s_rho: float = 1.0
    s_e: float = 0.8
    s_zeta: float = 0.8
    s_j: float = 1.0
    s_q: float = 1.1
    nu_L: float = 0.1
    nu_V: float = 0.5 / 3.0
    rho_L: float = 6.5
    rho_V: float = 0.38
    cv: float = 6.0
    cv_chi: float = 0.028
    g: float = 3e-5
    Gw_bottom: float = 0.0
    Gw_top: float = 0.0
    periodic_y: int = 0
    thermal_mode: int = COUPLED
    ghost_layer: int = 0

    def c(self) -> _CParams:
        return _CParams(**{f.name: getattr(self, f.name) for f in fields(self)})


_P = C.POINTER(_CParams)

for name in ("orc_Tc",):
    getattr(lib, name).restype = _d
    getattr(lib, name).argtypes = [_d, _d, _d]
lib.orc_kappa.restype = _d
lib.orc_kappa.argtypes = [_d]
for name in ("orc_phi", "orc_dphi_dT"):
    getattr(lib, name).restype = _d
    getattr(lib, name).argtypes = [_d, _d, _d]
for name in ("orc_p_eos", "orc_dp_dT", "orc_dp_drho"):
    getattr(lib, name).restype = _d
    getattr(lib, name).argtypes = [_d] * 7
lib.orc_maxwell.restype = C.c_int
lib.orc_maxwell.argtypes = [_d, _d, _d, _d, _d, _pd, _pd, _pd]
lib.orc_lattice.argtypes = [C.POINTER(C.c_int32), C.POINTER(C.c_int32), _pd, _pd, _pd]
lib.orc_feq.argtypes = [_d, _d, _d, _pd]
lib.orc_collide_site.argtypes = [_P, _pd, _d, _d, _d, _d, _d, _d, _pd]
lib.orc_forcing_moments.argtypes = [_P, _d, _d, _d, _d, _d, _pd]
lib.orc_interaction_force.argtypes = [_P, _pd, _pd, _pd, _pd]
lib.orc_thermal_rhs.argtypes = [_P, _pd, _pd, _pd, _pd, _pd]
lib.orc_grad_iso.argtypes = [C.c_int32, C.c_int32, C.c_int32, _pd, _pd, _pd, _pd]
lib.orc_create.restype = C.c_int
lib.orc_create.argtypes = [_P, _pd, _pd, _pd, _pd, _pd, C.POINTER(C.c_void_p)]
lib.orc_destroy.argtypes = [C.c_void_p]
lib.orc_step.restype = C.c_int
lib.orc_step.argtypes = [C.c_void_p, _i64]
lib.orc_time.restype = _i64
lib.orc_time.argtypes = [C.c_void_p]
lib.orc_fields.argtypes = [C.c_void_p, _pd, _pd, _pd, _pd, _pd]
lib.orc_heat_flux.argtypes = [C.c_void_p, _pd, _pd, C.POINTER(_i64), _pd]
lib.orc_reset_average.argtypes = [C.c_void_p]
lib.orc_set_heater.argtypes = [C.c_void_p, _pd]
lib.orc_set_wettability.argtypes = [C.c_void_p, _d]
lib.orc_set_storage_rounding.restype = C.c_int
lib.orc_set_storage_rounding.argtypes = [C.c_void_p, C.c_int]
lib.orc_last_error.restype = C.c_char_p
lib.orc_num_threads.restype = C.c_int
lib.orc_constants.argtypes = [C.c_void_p, _pd, _pd, _pd]
lib.orc_state_size.restype = _i64
lib.orc_state_size.argtypes = [C.c_void_p]
lib.orc_save.argtypes = [C.c_void_p, _pd]
lib.orc_adjoint.restype = C.c_int
lib.orc_adjoint.argtypes = [C.c_void_p, _i64, _i64, _pd, _pd, _pd]
lib.orc_step_vjp.restype = C.c_int
lib.orc_step_vjp.argtypes = [C.c_void_p, _pd, _pd, _pd, _pd, _pd]
lib.orc_load.argtypes = [C.c_void_p, _pd]
lib.orc3_lattice.argtypes = [C.POINTER(C.c_int32), _pd, _pd]
lib.orc3_feq.argtypes = [_d, _pd, _pd]
lib.orc3_collide_site.argtypes = [_P, _pd, _d, _pd, _pd, _d, _pd]
lib.orc3_grad_iso.argtypes = [C.c_int32, C.c_int32, C.c_int32, C.c_int32, _pd, _pd, _pd, _pd, _pd]
lib.orc3_create.restype = C.c_int
lib.orc3_create.argtypes = [_P, C.c_int32, _pd, _pd, _pd, _pd, _pd, _pd, C.POINTER(C.c_void_p)]
lib.orc3_destroy.argtypes = [C.c_void_p]
lib.orc3_step.restype = C.c_int
lib.orc3_step.argtypes = [C.c_void_p, _i64]
lib.orc3_time.restype = _i64
lib.orc3_time.argtypes = [C.c_void_p]
lib.orc3_fields.argtypes = [C.c_void_p, _pd, _pd, _pd, _pd, _pd, _pd]
lib.orc3_heat_flux.argtypes = [C.c_void_p, _pd, _pd, C.POINTER(_i64), _pd]
lib.orc3_reset_average.argtypes = [C.c_void_p]
lib.orc3_set_heater.argtypes = [C.c_void_p, _pd]
lib.orc3_set_storage_rounding.restype = C.c_int
lib.orc3_set_storage_rounding.argtypes = [C.c_void_p, C.c_int]


def _ptr(a):
    if a is None:
        return None
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(_pd)


def _f64(a):
    return None if a is None else np.ascontiguousarray(a, dtype=np.float64)


def num_threads() -> int:
    return lib.orc_num_threads()


def Tc(a, b, R=1.0):
    return lib.orc_Tc(a, b, R)


def kappa(omega):
    return lib.orc_kappa(omega)


def phi(T, Tc_, kap):
    return lib.orc_phi(T, Tc_, kap)


def dphi_dT(T, Tc_, kap):
    return lib.orc_dphi_dT(T, Tc_, kap)


def p_eos(rho, T, a, b, R, Tc_, kap):
    return lib.orc_p_eos(rho, T, a, b, R, Tc_, kap)


def dp_dT(rho, T, a, b, R, Tc_, kap):
    return lib.orc_dp_dT(rho, T, a, b, R, Tc_, kap)


def dp_drho(rho, T, a, b, R, Tc_, kap):
    return lib.orc_dp_drho(rho, T, a, b, R, Tc_, kap)


def maxwell(a, b, R, omega, T):
    """Maxwell equal-area coexistence (rho_V, rho_L, p_sat) at temperature T."""
    rv, rl, ps = _d(), _d(), _d()
    rc = lib.orc_maxwell(a, b, R, omega, T, C.byref(rv), C.byref(rl), C.byref(ps))
    if rc != 0:
        raise OracleError(rc, "maxwell construction failed")
    return rv.value, rl.value, ps.value


def lattice():
    ex = (C.c_int32 * 9)()
    ey = (C.c_int32 * 9)()
    W = np.zeros(9)
    wpsi = np.zeros(9)
    M = np.zeros(81)
    lib.orc_lattice(ex, ey, _ptr(W), _ptr(wpsi), _ptr(M))
    return np.array(ex[:]), np.array(ey[:]), W, wpsi, M.reshape(9, 9)


def feq(rho, ux, uy):
    out = np.zeros(9)
    lib.orc_feq(rho, ux, uy, _ptr(out))
    return out


def forcing_moments(p: Params, vx, vy, Fx, Fy, Q):
    out = np.zeros(9)
    cp = p.c()
    lib.orc_forcing_moments(C.byref(cp), vx, vy, Fx, Fy, Q, _ptr(out))
    return out


def collide_site(p: Params, f, rho, vx, vy, Fx, Fy, Q):
    f = _f64(f)
    out = np.zeros(9)
    cp = p.c()
    lib.orc_collide_site(C.byref(cp), _ptr(f), rho, vx, vy, Fx, Fy, Q, _ptr(out))
    return out


def interaction_force(p: Params, psi):
    psi = _f64(psi)
    Fx, Fy, Q = (np.zeros_like(psi) for _ in range(3))
    cp = p.c()
    lib.orc_interaction_force(C.byref(cp), _ptr(psi), _ptr(Fx), _ptr(Fy), _ptr(Q))
    return Fx, Fy, Q


def thermal_rhs(p: Params, rho, vx, vy, T):
    rho, vx, vy, T = (_f64(x) for x in (rho, vx, vy, T))
    K = np.zeros_like(T)
    cp = p.c()
    lib.orc_thermal_rhs(C.byref(cp), _ptr(rho), _ptr(vx), _ptr(vy), _ptr(T), _ptr(K))
    return K


def grad_iso(phi_field, periodic_y=0):
    phi_field = _f64(phi_field)
    ny, nx = phi_field.shape
    dx, dy, lap = (np.zeros_like(phi_field) for _ in range(3))
    lib.orc_grad_iso(nx, ny, periodic_y, _ptr(phi_field), _ptr(dx), _ptr(dy), _ptr(lap))
    return dx, dy, lap


class State:
    """One lattice evolving under the oracle's time step."""

    def __init__(self, p: Params, rho0, ux0=None, uy0=None, T0=None, T_bottom=None):
        self.p = p
        self._cp = p.c()
        rho0, ux0, uy0, T0, T_bottom = (_f64(x) for x in (rho0, ux0, uy0, T0, T_bottom))
        assert rho0.shape == (p.ny, p.nx)
        h = C.c_void_p()
        rc = lib.orc_create(C.byref(self._cp), _ptr(rho0), _ptr(ux0), _ptr(uy0), _ptr(T0),
                            _ptr(T_bottom), C.byref(h))
        if rc != 0:
            raise OracleError(rc, lib.orc_last_error().decode())
        self._h = h

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            lib.orc_destroy(h)
            self._h = None

    @property
    def t(self) -> int:
        return lib.orc_time(self._h)

    def step(self, n: int = 1):
        rc = lib.orc_step(self._h, int(n))
        if rc != 0:
            raise OracleError(rc, lib.orc_last_error().decode())
        return self

    def constants(self):
        tc, k, ts = _d(), _d(), _d()
        lib.orc_constants(self._h, C.byref(tc), C.byref(k), C.byref(ts))
        return tc.value, k.value, ts.value

    def fields(self):
        ny, nx = self.p.ny, self.p.nx
        rho, ux, uy, T = (np.zeros((ny, nx)) for _ in range(4))
        f = np.zeros((9, ny, nx))
        lib.orc_fields(self._h, _ptr(rho), _ptr(ux), _ptr(uy), _ptr(T), _ptr(f))
        return dict(rho=rho, ux=ux, uy=uy, T=T, f=f)

    def heat_flux(self):
        qn, qs, ns = _d(), _d(), _i64()
        ql = np.zeros(self.p.nx)
        lib.orc_heat_flux(self._h, C.byref(qn), C.byref(qs), C.byref(ns), _ptr(ql))
        n = ns.value
        return dict(q_now=qn.value, q_sum=qs.value, n_samples=n,
                    q_mean=(qs.value / n if n else float("nan")), q_local=ql)

    def reset_average(self):
        lib.orc_reset_average(self._h)

    def set_heater(self, T_bottom):
        T_bottom = _f64(T_bottom)
        lib.orc_set_heater(self._h, _ptr(T_bottom))

    def set_wettability(self, Gw):
        lib.orc_set_wettability(self._h, float(Gw))

    def store_bits(self, bits: int):
        """Rounding model: bits = 24 rounds the post-collision populations to
        FP32 every step (FP32 storage of f); 1..52 rounds the post-collision
        populations, psi and the new T to `bits` significant bits; 0 turns it
        off.  The arithmetic stays FP64."""
        rc = lib.orc_set_storage_rounding(self._h, int(bits))
        if rc != 0:
            raise OracleError(rc, "bits must lie in 0..52")
        return self

    def adjoint(self, n_steps: int, K: int = 0):
        """J = mean of q over n_steps from the current state (unchanged), and
        dJ/dT_b [nx], dJ/dG_w (bottom wall)."""
        J, gGw = _d(), _d()
        gTb = np.zeros(self.p.nx)
        rc = lib.orc_adjoint(self._h, int(n_steps), int(K), C.byref(J), _ptr(gTb), C.byref(gGw))
        if rc != 0:
            raise OracleError(rc, "adjoint failed")
        return J.value, gTb, gGw.value

    def step_vjp(self, lf1, lT1):
        """One step transposed at the current state."""
        lf1, lT1 = _f64(lf1), _f64(lT1)
        lf0, lT0 = np.zeros_like(lf1), np.zeros_like(lT1)
        g = _d(0.0)
        rc = lib.orc_step_vjp(self._h, _ptr(lf1), _ptr(lT1), _ptr(lf0), _ptr(lT0), C.byref(g))
        if rc != 0:
            raise OracleError(rc, "step_vjp failed")
        return lf0, lT0, g.value

    def save(self) -> np.ndarray:
        buf = np.zeros(lib.orc_state_size(self._h))
        lib.orc_save(self._h, _ptr(buf))
        return buf

    def load(self, buf):
        buf = _f64(buf)
        assert buf.size == lib.orc_state_size(self._h)
        lib.orc_load(self._h, _ptr(buf))


# ---- three-dimensional extension (D3Q19) ---------------------------------


def lattice3():
    """D3Q19 velocities e [19, 3], weights W [19] and moment basis M [19, 19]."""
    e = (C.c_int32 * 57)()
    W = np.zeros(19)
    M = np.zeros(361)
    lib.orc3_lattice(e, _ptr(W), _ptr(M))
    return np.array(e[:]).reshape(19, 3), W, M.reshape(19, 19)


def feq3(rho, v):
    out = np.zeros(19)
    v = _f64(np.asarray(v, dtype=float))
    lib.orc3_feq(rho, _ptr(v), _ptr(out))
    return out


def collide_site3(p: Params, f, rho, v, F, Q):
    f, v, F = (_f64(np.asarray(x, dtype=float)) for x in (f, v, F))
    out = np.zeros(19)
    cp = p.c()
    lib.orc3_collide_site(C.byref(cp), _ptr(f), rho, _ptr(v), _ptr(F), Q, _ptr(out))
    return out


def grad_iso3(phi, periodic_y=0):
    """Isotropic D3Q19 stencils of phi [nz, ny, nx]: d_x, d_y, d_z, lap."""
    phi = _f64(phi)
    nz, ny, nx = phi.shape
    outs = [np.zeros_like(phi) for _ in range(4)]
    lib.orc3_grad_iso(nx, ny, nz, periodic_y, _ptr(phi), *(_ptr(o) for o in outs))
    return tuple(outs)


class State3:
    """One three-dimensional lattice (D3Q19) under the oracle's time step.
    Arrays are [nz, ny, nx]; walls at y = 0 and y = ny - 1 unless
    periodic_y; x and z periodic.  T_bottom is [nz, nx]."""

    def __init__(self, p: Params, nz: int, rho0, ux0=None, uy0=None, uz0=None, T0=None, T_bottom=None):
        self.p, self.nz = p, int(nz)
        self._cp = p.c()
        rho0, ux0, uy0, uz0, T0, T_bottom = (_f64(x) for x in (rho0, ux0, uy0, uz0, T0, T_bottom))
        assert rho0.shape == (nz, p.ny, p.nx)
        h = C.c_void_p()
        rc = lib.orc3_create(C.byref(self._cp), self.nz, _ptr(rho0), _ptr(ux0), _ptr(uy0), _ptr(uz0), _ptr(T0),
                             _ptr(T_bottom), C.byref(h))
        if rc != 0:
            raise OracleError(rc, "invalid 3-D parameters or initial state")
        self._h = h

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            lib.orc3_destroy(h)
            self._h = None

    @property
    def t(self) -> int:
        return lib.orc3_time(self._h)

    def step(self, n: int = 1):
        rc = lib.orc3_step(self._h, int(n))
        if rc != 0:
            raise OracleError(rc, "3-D step failed")
        return self

    def store_bits(self, bits: int):
        """Rounding model as State.store_bits."""
        rc = lib.orc3_set_storage_rounding(self._h, int(bits))
        if rc != 0:
            raise OracleError(rc, "bits must lie in 0..52")
        return self

    def fields(self):
        shape = (self.nz, self.p.ny, self.p.nx)
        rho, ux, uy, uz, T = (np.zeros(shape) for _ in range(5))
        f = np.zeros((19,) + shape)
        lib.orc3_fields(self._h, _ptr(rho), _ptr(ux), _ptr(uy), _ptr(uz), _ptr(T), _ptr(f))
        return dict(rho=rho, ux=ux, uy=uy, uz=uz, T=T, f=f)

    def heat_flux(self):
        qn, qs, ns = _d(), _d(), _i64()
        ql = np.zeros((self.nz, self.p.nx))
        lib.orc3_heat_flux(self._h, C.byref(qn), C.byref(qs), C.byref(ns), _ptr(ql))
        n = ns.value
        return dict(q_now=qn.value, q_sum=qs.value, n_samples=n,
                    q_mean=(qs.value / n if n else float("nan")), q_local=ql)

    def reset_average(self):
        lib.orc3_reset_average(self._h)

    def set_heater(self, T_bottom):
        T_bottom = _f64(T_bottom)
        lib.orc3_set_heater(self._h, _ptr(T_bottom))
