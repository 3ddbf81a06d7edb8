"""ctypes binding of the lbboil C-ABI (include/lbboil.h).

Argument marshalling only: every step of the model runs in the gfx950 HIP
kernels of ``liblbboil.so``.  Loading fails loudly when the library has not
been built (``python -m paper_1501_03857_amd.build``); there is no fallback.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass, fields
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liblbboil.so")

LBB_OK, LBB_EINVAL, LBB_ENOMEM, LBB_EDEVICE, LBB_ENONFINITE, LBB_EUNSUPPORTED, LBB_ESTATE = 0, -1, -2, -3, -4, -5, -6
FP64, FP32 = 0, 1
# fields of lbb_read_fields' mask
FIELD_RHO, FIELD_UX, FIELD_UY, FIELD_T, FIELD_F = 1, 2, 4, 8, 16
FIELD_ALL = 31
COUPLED, ISOTHERMAL, THERMAL_ONLY = 0, 1, 2


class LbbError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"lbboil error {code}: {msg}")
        self.code = code


_d = C.c_double
_pd = C.POINTER(C.c_double)
_i32 = C.c_int32
_i64 = C.c_int64
_pi32 = C.POINTER(C.c_int32)


class CParams(C.Structure):
    _fields_ = [
        ("nx", _i32), ("ny", _i32), ("precision", _i32), ("periodic_y", _i32), ("thermal_mode", _i32),
        ("liquid_rows", _i32),
        ("a", _d), ("b", _d), ("R", _d), ("omega", _d), ("Ts_over_Tc", _d),
        ("G", _d), ("sigma", _d),
        ("s_rho", _d), ("s_e", _d), ("s_zeta", _d), ("s_j", _d), ("s_q", _d),
        ("nu_L", _d), ("nu_V", _d), ("rho_L", _d), ("rho_V", _d),
        ("cv", _d), ("cv_chi", _d), ("g", _d), ("Gw_bottom", _d), ("Gw_top", _d),
        ("noise_amp", _d), ("seed", C.c_uint64), ("ghost_layer", _i32), ("reserved", _i32),
    ]


_lib = None


def lib():
    """The loaded library (raises if it is missing: no fallback exists)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing; build it with python -m paper_1501_03857_amd.build")
        # PyTorch ships its own HIP runtime under the same soname as the
        # system one.  Loaded first, it is the one the library binds to, so
        # the process holds a single runtime and torch streams, events and
        # device buffers can be handed to the library; loaded after the
        # library, it would start a second runtime that cannot see the GPU.
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        L = C.CDLL(LIB_PATH)
        _P = C.POINTER(CParams)
        vp = C.c_void_p
        sig = {
            "lbb_default_params": (None, [_P]),
            "lbb_eos_constants": (C.c_int, [_d, _d, _d, _d, _pd, _pd]),
            "lbb_coexistence": (C.c_int, [_d, _d, _d, _d, _d, _pd, _pd]),
            "lbb_eos_pressure": (C.c_int, [_d, _d, _d, _d, _d, _d, _pd]),
            "lbb_init_domain": (C.c_int, [_P, _pd, _pd, C.POINTER(vp)]),
            "lbb_set_fields": (C.c_int, [vp, _pd, _pd, _pd, _pd]),
            "lbb_step": (C.c_int, [vp, _i64]),
            "lbb_step_async": (C.c_int, [vp, _i64]),
            "lbb_sync": (C.c_int, [vp]),
            "lbb_stream": (vp, [vp]),
            "lbb_time_kernels": (C.c_int, [vp, _i64, _pd, _pd, _pd]),
            "lbb_read_fields": (C.c_int, [vp, C.c_uint32, _pd, _pd, _pd, _pd, _pd]),
            "lbb_wall_heat_flux": (C.c_int, [vp, _pd, _pd, _pd, C.POINTER(_i64)]),
            "lbb_reset_average": (C.c_int, [vp]),
            "lbb_set_heater": (C.c_int, [vp, _pd]),
            "lbb_set_wettability": (C.c_int, [vp, _d]),
            "lbb_save_state": (C.c_int, [vp, vp, C.POINTER(C.c_size_t)]),
            "lbb_load_state": (C.c_int, [vp, vp, C.c_size_t]),
            "lbb_info": (C.c_int, [vp, C.POINTER(_i64), C.POINTER(_i32), C.POINTER(_i32), C.POINTER(_i64)]),
            "lbb_destroy": (C.c_int, [vp]),
            "lbb_batch_init": (C.c_int, [_P, C.c_int, C.POINTER(_pd), C.POINTER(_pd), C.POINTER(vp)]),
            "lbb_batch_step": (C.c_int, [vp, _i64]),
            "lbb_batch_step_async": (C.c_int, [vp, _i64]),
            "lbb_batch_sync": (C.c_int, [vp]),
            "lbb_batch_stream": (vp, [vp]),
            "lbb_batch_heat_flux": (C.c_int, [vp, _pd, _pd, C.POINTER(_i64)]),
            "lbb_batch_domain": (vp, [vp, C.c_int]),
            "lbb_batch_size": (C.c_int, [vp]),
            "lbb_batch_destroy": (C.c_int, [vp]),
            "lbb_adjoint": (C.c_int, [vp, _i64, _i64, C.POINTER(C.c_int32), C.c_int32, _pd, _pd, _pd]),
            "lbb_batch_adjoint": (C.c_int, [vp, _i64, _i64, _pd, _pd, _pd]),
            "lbb_read_fields_dev": (C.c_int, [vp, vp, vp, vp, vp, vp, vp]),
            "lbb_set_device_budget": (C.c_int, [_i64]),
            "lbb_device_bytes_held": (_i64, []),
            "lbb_tile_shapes": (C.c_int, [_pi32, _pi32, _pi32, _pi32]),
            "lbb_get_tiles": (C.c_int, [vp, _pi32, _pi32]),
            "lbb_set_tiles": (C.c_int, [vp, C.c_int32, C.c_int32]),
            "lbb_autotune": (C.c_int, [vp, C.c_int32, _pi32, _pi32, _pd, _pd]),
            "lbb_batch_set_tiles": (C.c_int, [vp, C.c_int32, C.c_int32]),
            "lbb_batch_autotune": (C.c_int, [vp, C.c_int32, _pi32, _pi32, _pd, _pd]),
            "lbb_batch_info": (C.c_int, [vp, C.POINTER(_i64)]),
            "lbb_step_noalloc": (C.c_int, [_P, C.POINTER(vp), C.POINTER(vp), vp, vp, vp, _pi32, _i64, vp, vp]),
            "lbb3_init_domain": (C.c_int, [_P, _i32, _pd, _pd, C.POINTER(vp)]),
            "lbb3_set_fields": (C.c_int, [vp, _pd, _pd, _pd]),
            "lbb3_step": (C.c_int, [vp, _i64]),
            "lbb3_step_async": (C.c_int, [vp, _i64]),
            "lbb3_sync": (C.c_int, [vp]),
            "lbb3_stream": (vp, [vp]),
            "lbb3_read_fields": (C.c_int, [vp, _pd, _pd, _pd, _pd]),
            "lbb3_wall_heat_flux": (C.c_int, [vp, _pd, _pd, _pd, C.POINTER(_i64)]),
            "lbb3_reset_average": (C.c_int, [vp]),
            "lbb3_set_heater": (C.c_int, [vp, _pd]),
            "lbb3_info": (C.c_int, [vp, C.POINTER(_i64), C.POINTER(_i64)]),
            "lbb3_destroy": (C.c_int, [vp]),
            "lbb_last_error": (C.c_char_p, []),
        }
        for name, (res, args) in sig.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def _check(rc: int):
    if rc != LBB_OK:
        raise LbbError(rc, lib().lbb_last_error().decode())


def _ptr(a: Optional[np.ndarray]):
    if a is None:
        return None
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(_pd)


def _f64(a):
    return None if a is None else np.ascontiguousarray(a, dtype=np.float64)


@dataclass
class Params:
    """lbb_params with the library's defaults (lbb_default_params)."""
    nx: int = 128
    ny: int = 64
    precision: int = FP64
    periodic_y: int = 0
    thermal_mode: int = COUPLED
    liquid_rows: int = 38
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
    rho_L: float = 0.0
    rho_V: float = 0.0
    cv: float = 6.0
    cv_chi: float = 0.028
    g: float = 3e-5
    Gw_bottom: float = 0.0
    Gw_top: float = 0.0
    noise_amp: float = 1e-3
    seed: int = 1
    ghost_layer: int = 0
    reserved: int = 0

    def c(self) -> CParams:
        return CParams(**{f.name: getattr(self, f.name) for f in fields(self)})


def default_params() -> CParams:
    p = CParams()
    lib().lbb_default_params(C.byref(p))
    return p


def eos_constants(a, b, R, omega):
    tc, k = _d(), _d()
    _check(lib().lbb_eos_constants(a, b, R, omega, C.byref(tc), C.byref(k)))
    return tc.value, k.value


def coexistence(a, b, R, omega, T):
    rv, rl = _d(), _d()
    _check(lib().lbb_coexistence(a, b, R, omega, T, C.byref(rv), C.byref(rl)))
    return rv.value, rl.value


def eos_pressure(a, b, R, omega, rho, T):
    """p_EOS(rho, T) of the Peng-Robinson equation of state (Eq. (21))."""
    p = _d()
    _check(lib().lbb_eos_pressure(a, b, R, omega, float(rho), float(T), C.byref(p)))
    return p.value


class Domain:
    """One lattice on the current GPU (lbb_init_domain ... lbb_destroy)."""

    @classmethod
    def borrowed(cls, handle, p: Params):
        """A view of a lattice owned elsewhere (a batch member); never destroyed here."""
        d = cls.__new__(cls)
        d.p = p
        d._h = C.c_void_p(handle)
        d._owner = False
        return d

    def __init__(self, p: Params, T_bottom=None, rho0=None):
        self.p = p
        self._cp = p.c()
        T_bottom, rho0 = _f64(T_bottom), _f64(rho0)
        if rho0 is not None:
            assert rho0.shape == (p.ny, p.nx)
        if T_bottom is not None:
            assert T_bottom.shape == (p.nx,)
        h = C.c_void_p()
        _check(lib().lbb_init_domain(C.byref(self._cp), _ptr(T_bottom), _ptr(rho0), C.byref(h)))
        self._h = h
        self._owner = True

    def close(self):
        h = getattr(self, "_h", None)
        if h and getattr(self, "_owner", False):
            lib().lbb_destroy(h)
        self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    @property
    def handle(self):
        return self._h

    def set_fields(self, rho, ux=None, uy=None, T=None):
        rho, ux, uy, T = (_f64(x) for x in (rho, ux, uy, T))
        _check(lib().lbb_set_fields(self._h, _ptr(rho), _ptr(ux), _ptr(uy), _ptr(T)))

    def step(self, n: int = 1):
        _check(lib().lbb_step(self._h, int(n)))
        return self

    def step_async(self, n: int):
        _check(lib().lbb_step_async(self._h, int(n)))

    def sync(self):
        _check(lib().lbb_sync(self._h))

    def time_kernels(self, n: int):
        """Mean (LB launch, thermal launch, whole step) durations in ms over n
        single-launch steps, from HIP events on the library stream."""
        a, b, c = _d(), _d(), _d()
        _check(lib().lbb_time_kernels(self._h, int(n), C.byref(a), C.byref(b), C.byref(c)))
        return a.value, b.value, c.value

    @property
    def stream(self) -> int:
        return lib().lbb_stream(self._h)

    @property
    def tiles(self):
        """(LB shape, thermal shape) indices into tile_shapes()."""
        a, b = C.c_int32(), C.c_int32()
        _check(lib().lbb_get_tiles(self._h, C.byref(a), C.byref(b)))
        return a.value, b.value

    def set_tiles(self, shape_lb: int, shape_thermal: int):
        _check(lib().lbb_set_tiles(self._h, int(shape_lb), int(shape_thermal)))
        return self

    def autotune(self, steps: int = 20):
        """Time every tile shape on this lattice, keep the fastest; the state
        is left unchanged.  Returns the choice and the per-shape times (ms)."""
        return _autotune(lib().lbb_autotune, self._h, steps)

    def adjoint(self, n_steps: int, K: int = 0, heater_idx=None):
        """J = mean bottom-wall heat flux over the next n_steps and its
        gradient w.r.t. T_b of the heater nodes heater_idx (None: all nx, in
        order) and G_w; the state is left unchanged."""
        J, gGw = _d(), _d()
        if heater_idx is None:
            idx, n = None, self.p.nx
        else:
            idx = np.ascontiguousarray(heater_idx, dtype=np.int32)
            n = len(idx)
        gTb = np.zeros(n)
        _check(lib().lbb_adjoint(self._h, int(n_steps), int(K),
                                 None if idx is None else idx.ctypes.data_as(C.POINTER(C.c_int32)), n,
                                 C.byref(J), _ptr(gTb), C.byref(gGw)))
        return J.value, gTb, gGw.value

    def fields(self, f: bool = True):
        ny, nx = self.p.ny, self.p.nx
        rho, ux, uy, T = (np.zeros((ny, nx)) for _ in range(4))
        ff = np.zeros((9, ny, nx)) if f else None
        _check(lib().lbb_read_fields(self._h, FIELD_ALL, _ptr(rho), _ptr(ux), _ptr(uy), _ptr(T), _ptr(ff)))
        out = dict(rho=rho, ux=ux, uy=uy, T=T)
        if f:
            out["f"] = ff
        return out

    def read_into(self, rho=0, ux=0, uy=0, T=0, f=0, stream=0):
        """Read the fields into device buffers given by address (FP64; 0 =
        skip), ordered with the caller's `stream` (a hipStream_t address; 0 is
        the null stream, e.g. torch's default stream)."""
        _check(lib().lbb_read_fields_dev(self._h, rho or None, ux or None, uy or None, T or None, f or None,
                                         stream or None))

    def bottom_temperature(self) -> np.ndarray:
        """The current bottom-wall temperatures T_b(x)."""
        T = np.zeros((self.p.ny, self.p.nx))
        _check(lib().lbb_read_fields(self._h, FIELD_T, None, None, None, _ptr(T), None))
        return T[0].copy()

    def heat_flux(self, local: bool = True):
        qn, qm, ns = _d(), _d(), _i64()
        ql = np.zeros(self.p.nx) if local else None
        _check(lib().lbb_wall_heat_flux(self._h, C.byref(qn), C.byref(qm), _ptr(ql), C.byref(ns)))
        return dict(q_now=qn.value, q_mean=qm.value, n_samples=ns.value, q_local=ql)

    def reset_average(self):
        _check(lib().lbb_reset_average(self._h))

    def set_heater(self, T_bottom):
        T_bottom = _f64(T_bottom)
        _check(lib().lbb_set_heater(self._h, _ptr(T_bottom)))

    def set_wettability(self, Gw):
        _check(lib().lbb_set_wettability(self._h, float(Gw)))

    def save(self) -> bytes:
        n = C.c_size_t(0)
        _check(lib().lbb_save_state(self._h, None, C.byref(n)))
        buf = C.create_string_buffer(n.value)
        _check(lib().lbb_save_state(self._h, buf, C.byref(n)))
        return buf.raw[: n.value]

    def load(self, blob: bytes):
        buf = C.create_string_buffer(blob, len(blob))
        _check(lib().lbb_load_state(self._h, buf, len(blob)))

    def info(self):
        t, nx, ny, nb = _i64(), _i32(), _i32(), _i64()
        _check(lib().lbb_info(self._h, C.byref(t), C.byref(nx), C.byref(ny), C.byref(nb)))
        return dict(t=t.value, nx=nx.value, ny=ny.value, device_bytes=nb.value)

    @property
    def t(self) -> int:
        return self.info()["t"]


def set_device_budget(nbytes: int):
    """Cap the device bytes the library may hold (0: no cap)."""
    _check(lib().lbb_set_device_budget(int(nbytes)))


def device_bytes_held() -> int:
    return lib().lbb_device_bytes_held()


def tile_shapes():
    """(lb, thermal): lists of (width, height, waves) of the tile shapes."""
    na, nb = C.c_int32(), C.c_int32()
    _check(lib().lbb_tile_shapes(C.byref(na), C.byref(nb), None, None))
    a, b = (C.c_int32 * (3 * na.value))(), (C.c_int32 * (3 * nb.value))()
    _check(lib().lbb_tile_shapes(None, None, a, b))
    return ([tuple(a[3 * i:3 * i + 3]) for i in range(na.value)],
            [tuple(b[3 * i:3 * i + 3]) for i in range(nb.value)])


def _autotune(fn, h, steps):
    na, nb = len(tile_shapes()[0]), len(tile_shapes()[1])
    sa, sb = C.c_int32(), C.c_int32()
    ma, mb = np.zeros(na), np.zeros(nb)
    _check(fn(h, int(steps), C.byref(sa), C.byref(sb), _ptr(ma), _ptr(mb)))
    return dict(shape_lb=sa.value, shape_thermal=sb.value, ms_lb=ma, ms_thermal=mb)


class Batch:
    """Many lattices advanced together by shared launches (lbb_batch_*)."""

    def __init__(self, params, T_bottoms=None, rho0s=None):
        n = len(params)
        self.params = list(params)
        self._cps = (CParams * n)(*[p.c() for p in params])
        keep = []

        def arr(xs, shape_of):
            if xs is None:
                return None
            out = (_pd * n)()
            for i, x in enumerate(xs):
                if x is None:
                    out[i] = None
                    continue
                a = np.ascontiguousarray(x, dtype=np.float64)
                assert a.shape == shape_of(params[i])
                keep.append(a)
                out[i] = _ptr(a)
            return out

        tb = arr(T_bottoms, lambda p: (p.nx,))
        r0 = arr(rho0s, lambda p: (p.ny, p.nx))
        h = C.c_void_p()
        _check(lib().lbb_batch_init(self._cps, n, tb, r0, C.byref(h)))
        self._h = h

    def close(self):
        h = getattr(self, "_h", None)
        if h:
            lib().lbb_batch_destroy(h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __len__(self):
        return lib().lbb_batch_size(self._h)

    def step(self, n: int = 1):
        _check(lib().lbb_batch_step(self._h, int(n)))
        return self

    def step_async(self, n: int):
        _check(lib().lbb_batch_step_async(self._h, int(n)))

    def sync(self):
        _check(lib().lbb_batch_sync(self._h))

    @property
    def stream(self) -> int:
        return lib().lbb_batch_stream(self._h)

    def heat_flux(self):
        n = len(self)
        qn, qm = np.zeros(n), np.zeros(n)
        ns = (_i64 * n)()
        _check(lib().lbb_batch_heat_flux(self._h, _ptr(qn), _ptr(qm), ns))
        return dict(q_now=qn, q_mean=qm, n_samples=np.array(ns[:]))

    def adjoint(self, n_steps: int, K: int = 0):
        """Per member: J = mean bottom-wall heat flux over the next n_steps and
        its gradient w.r.t. T_b (all nx of the member) and G_w, all members in
        shared launches; every member's state is left unchanged."""
        n = len(self)
        J, gGw = np.zeros(n), np.zeros(n)
        gTb = np.zeros(sum(p.nx for p in self.params))
        _check(lib().lbb_batch_adjoint(self._h, int(n_steps), int(K), _ptr(J), _ptr(gTb), _ptr(gGw)))
        out, off = [], 0
        for p in self.params:
            out.append(gTb[off:off + p.nx])
            off += p.nx
        return J, out, gGw

    def device_bytes(self) -> int:
        v = _i64()
        _check(lib().lbb_batch_info(self._h, C.byref(v)))
        return v.value

    def set_tiles(self, shape_lb: int, shape_thermal: int):
        _check(lib().lbb_batch_set_tiles(self._h, int(shape_lb), int(shape_thermal)))
        return self

    def autotune(self, steps: int = 20):
        """As Domain.autotune, for the batch's shared launches."""
        return _autotune(lib().lbb_batch_autotune, self._h, steps)

    def domain(self, i: int) -> Domain:
        h = lib().lbb_batch_domain(self._h, int(i))
        if not h:
            raise IndexError(i)
        return Domain.borrowed(h, self.params[i])


NOALLOC_SCRATCH_BYTES = 8 << 20


class NoallocResult(C.Structure):
    """lbb_noalloc_result: written to device memory by lbb_step_noalloc."""
    _fields_ = [("q_now", _d), ("q_mean", _d), ("n_samples", _i64), ("err_step", _i64),
                ("err_code", C.c_uint32), ("reserved", C.c_uint32)]


def step_noalloc(p: "Params", f, T, rho, vx, vy, phase, n: int, result: int, stream: int = 0):
    """lbb_step_noalloc on caller-held device buffers (raw device addresses as
    ints): f = (f0, f1), T = (T0, T1), rho, vx, vy; phase = [phase_f,
    phase_T] (a list, updated in place); result = device address of an
    lbb_noalloc_result; stream = hipStream_t as an int (0: null stream)."""
    cp = p.c()
    fa = (C.c_void_p * 2)(int(f[0]), int(f[1]))
    ta = (C.c_void_p * 2)(int(T[0]), int(T[1]))
    ph = (_i32 * 2)(int(phase[0]), int(phase[1]))
    _check(lib().lbb_step_noalloc(C.byref(cp), fa, ta, C.c_void_p(int(rho)), C.c_void_p(int(vx)),
                                  C.c_void_p(int(vy)), ph, int(n), C.c_void_p(int(result)),
                                  C.c_void_p(int(stream)) if stream else None))
    phase[0], phase[1] = ph[0], ph[1]


class Domain3:
    """One three-dimensional (D3Q19) lattice on the current GPU
    (lbb3_init_domain ... lbb3_destroy).  Arrays are [nz, ny, nx]; T_bottom
    is [nz, nx]."""

    def __init__(self, p: Params, nz: int, T_bottom=None, rho0=None):
        self.p, self.nz = p, int(nz)
        self._cp = p.c()
        T_bottom, rho0 = _f64(T_bottom), _f64(rho0)
        if rho0 is not None:
            assert rho0.shape == (nz, p.ny, p.nx)
        if T_bottom is not None:
            assert T_bottom.shape == (nz, p.nx)
        h = C.c_void_p()
        _check(lib().lbb3_init_domain(C.byref(self._cp), self.nz, _ptr(T_bottom), _ptr(rho0), C.byref(h)))
        self._h = h

    def close(self):
        h = getattr(self, "_h", None)
        if h:
            lib().lbb3_destroy(h)
        self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    @property
    def shape(self):
        return (self.nz, self.p.ny, self.p.nx)

    def step(self, n: int = 1):
        _check(lib().lbb3_step(self._h, int(n)))
        return self

    def step_async(self, n: int):
        _check(lib().lbb3_step_async(self._h, int(n)))

    def sync(self):
        _check(lib().lbb3_sync(self._h))

    @property
    def stream(self) -> int:
        return lib().lbb3_stream(self._h) or 0

    @property
    def t(self) -> int:
        t = _i64()
        _check(lib().lbb3_info(self._h, C.byref(t), None))
        return t.value

    def set_fields(self, rho, u=None, T=None):
        rho = _f64(rho)
        u = None if u is None else _f64(np.asarray(u, dtype=float).reshape(3, *self.shape))
        T = _f64(T)
        _check(lib().lbb3_set_fields(self._h, _ptr(rho), _ptr(u), _ptr(T)))

    def fields(self, f: bool = True):
        rho, T = np.zeros(self.shape), np.zeros(self.shape)
        u = np.zeros((3,) + self.shape)
        ff = np.zeros((19,) + self.shape) if f else None
        _check(lib().lbb3_read_fields(self._h, _ptr(rho), _ptr(u), _ptr(T), _ptr(ff)))
        out = dict(rho=rho, ux=u[0], uy=u[1], uz=u[2], T=T)
        if f:
            out["f"] = ff
        return out

    def heat_flux(self, local: bool = True):
        qn, qm, ns = _d(), _d(), _i64()
        ql = np.zeros((self.nz, self.p.nx)) if local else None
        _check(lib().lbb3_wall_heat_flux(self._h, C.byref(qn), C.byref(qm), _ptr(ql), C.byref(ns)))
        return dict(q_now=qn.value, q_mean=qm.value, n_samples=ns.value, q_local=ql)

    def reset_average(self):
        _check(lib().lbb3_reset_average(self._h))

    def set_heater(self, T_bottom):
        T_bottom = _f64(T_bottom)
        assert T_bottom.shape == (self.nz, self.p.nx)
        _check(lib().lbb3_set_heater(self._h, _ptr(T_bottom)))
