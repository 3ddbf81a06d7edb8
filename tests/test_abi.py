"""The C-ABI library loads, exports every symbol its header declares, and its
host-side logic (parameter validation, EOS constants, Maxwell coexistence)
behaves; none of these tests launches a kernel."""
import ctypes as C
import os
import re

import numpy as np
import pytest

import oracle as O
from paper_1501_03857_amd import lbboil as L

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_symbols():
    names = set()
    inc = os.path.join(ROOT, "include")
    for fn in os.listdir(inc):
        if fn.endswith(".h"):
            src = open(os.path.join(inc, fn)).read()
            src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
            names |= set(re.findall(r"\b(lbb3?_[a-z0-9_]+)\s*\(", src))
    return names


def test_library_exports_every_declared_symbol():
    names = _declared_symbols()
    assert len(names) >= 19
    lib = C.CDLL(L.LIB_PATH)
    missing = [n for n in sorted(names) if not hasattr(lib, n)]
    assert not missing, missing


def test_params_struct_size():
    """The binding's lbb_params has the size the library asserts at compile
    time (216 bytes: 6 int32, 22 doubles, a uint64, 2 int32)."""
    assert C.sizeof(L.CParams) == 216


def test_default_params_match_binding_layout():
    """lbb_default_params fills the struct the binding declares (layout check)."""
    p = L.default_params()
    q = L.Params()
    for name, _ in L.CParams._fields_:
        v = getattr(p, name)
        if name in ("liquid_rows",):
            continue
        assert v == pytest.approx(getattr(q, name), rel=1e-15, abs=0), name
    assert p.liquid_rows == int(np.floor(0.6 * p.ny))


@pytest.mark.parametrize("field,value", [
    ("nx", 2), ("ny", 3), ("precision", 7), ("thermal_mode", 3), ("G", 1.0), ("a", -1.0),
    ("s_e", 2.0), ("nu_L", 0.0), ("cv", float("nan")), ("liquid_rows", 65), ("noise_amp", -1.0),
    ("nx", 1 << 16), ("Ts_over_Tc", 0.0), ("ghost_layer", 2), ("ghost_layer", -1), ("reserved", 1),
])
def test_init_rejects_invalid_parameters(field, value):
    p = L.Params()
    setattr(p, field, value)
    if field == "nx" and value == 1 << 16:
        p.ny = 1 << 16  # 2^32 nodes: a field plane of 2^35 bytes
    with pytest.raises(L.LbbError) as e:
        L.Domain(p)
    assert e.value.code == L.LBB_EINVAL


def test_init_rejects_fp64_plane_of_4_gib():
    """2^29 nodes in FP64 make an 8-byte field plane of exactly 2^32 bytes,
    one byte past the 32-bit offsets the kernels use: refused before any
    device memory is touched."""
    p = L.Params(nx=1 << 15, ny=1 << 14, precision=L.FP64)
    with pytest.raises(L.LbbError) as e:
        L.Domain(p)
    assert e.value.code == L.LBB_EINVAL and "2^32" in str(e.value)


def test_init_rejects_bad_initial_density():
    p = L.Params(nx=8, ny=6)
    rho = np.full((6, 8), 2.0)
    rho[2, 3] = 1.0 / p.b  # b rho >= 1
    with pytest.raises(L.LbbError) as e:
        L.Domain(p, rho0=rho)
    assert e.value.code == L.LBB_EINVAL
    rho[2, 3] = -1.0
    with pytest.raises(L.LbbError):
        L.Domain(p, rho0=rho)
    with pytest.raises(L.LbbError):
        L.Domain(p, T_bottom=np.full(8, -0.1))


@pytest.mark.parametrize("a", [2.0 / 49.0, 3.0 / 49.0])
def test_eos_constants_match_oracle(a):
    tc, k = L.eos_constants(a, 2.0 / 21.0, 1.0, 0.344)
    assert tc == pytest.approx(O.Tc(a, 2.0 / 21.0, 1.0), rel=1e-15)
    assert k == pytest.approx(O.kappa(0.344), rel=1e-15)


@pytest.mark.parametrize("a,omega,theta", [(2.0 / 49.0, 0.344, 0.5), (2.0 / 49.0, 0.344, 0.6),
                                           (2.0 / 49.0, 0.344, 0.86), (2.0 / 49.0, 0.344, 0.97),
                                           (2.0 / 49.0, 0.344, 0.995), (3.0 / 49.0, 0.344, 0.86),
                                           (3.0 / 49.0, 0.2, 0.9), (3.0 / 49.0, 0.0, 0.75)])
def test_library_coexistence_matches_oracle(a, omega, theta):
    """The library's coexistence (Newton on the chemical-potential difference)
    against the oracle's (bisection on the equal-area sign): two methods, one
    construction."""
    b = 2.0 / 21.0
    tc = O.Tc(a, b, 1.0)
    rv, rl = L.coexistence(a, b, 1.0, omega, theta * tc)
    orv, orl, _ = O.maxwell(a, b, 1.0, omega, theta * tc)
    assert rv == pytest.approx(orv, rel=1e-9)
    assert rl == pytest.approx(orl, rel=1e-9)


def test_library_coexistence_paper_densities():
    """Sec. 3.1: at T_s = 0.86 T_c the coexistence densities are about 6.5 and 0.38."""
    a, b = 3.0 / 49.0, 2.0 / 21.0
    tc, _ = L.eos_constants(a, b, 1.0, 0.344)
    rv, rl = L.coexistence(a, b, 1.0, 0.344, 0.86 * tc)
    assert abs(rl - 6.5) < 0.01 and abs(rv - 0.38) < 0.005
    pl, pv = L.eos_pressure(a, b, 1.0, 0.344, rl, 0.86 * tc), L.eos_pressure(a, b, 1.0, 0.344, rv, 0.86 * tc)
    assert pl == pytest.approx(pv, rel=1e-10)


def test_coexistence_rejects_supercritical():
    a, b = 2.0 / 49.0, 2.0 / 21.0
    tc, _ = L.eos_constants(a, b, 1.0, 0.344)
    with pytest.raises(L.LbbError):
        L.coexistence(a, b, 1.0, 0.344, 1.01 * tc)


def test_batch_rejects_mixed_precision_and_empty():
    with pytest.raises(L.LbbError) as e:
        L.Batch([L.Params(precision=L.FP64), L.Params(precision=L.FP32)])
    assert e.value.code == L.LBB_EINVAL
    with pytest.raises(L.LbbError):
        L.Batch([])


def test_tile_shape_tables():
    """The tile shapes: each tile plus its halo is one wave64 wide, heights
    split evenly over the waves of the LB launch."""
    lb, th = L.tile_shapes()
    assert len(lb) >= 2 and len(th) >= 2
    for w, h, nw in lb:
        assert w + 2 == 64 and h % nw == 0 and 1 <= nw <= 16
    for w, h, nw in th:
        assert w + 8 == 64 and h >= 1 and 1 <= nw <= 16
    assert lb[0] == (62, 4, 4) and th[0] == (56, 24, 16)


def test_tile_calls_reject_bad_arguments():
    lib = L.lib()
    assert lib.lbb_set_tiles(None, 0, 0) == L.LBB_EINVAL
    assert lib.lbb_get_tiles(None, None, None) == L.LBB_EINVAL
    assert lib.lbb_autotune(None, 5, None, None, None, None) == L.LBB_EINVAL
    assert lib.lbb_batch_set_tiles(None, 0, 0) == L.LBB_EINVAL
    assert lib.lbb_batch_autotune(None, 5, None, None, None, None) == L.LBB_EINVAL


def test_device_budget_refuses_a_domain_before_touching_the_device():
    """ENOMEM from the host-side budget, before any device call (this runs
    on a host without a GPU); a negative budget is EINVAL."""
    lib = L.lib()
    assert lib.lbb_set_device_budget(-1) == L.LBB_EINVAL
    assert lib.lbb_set_device_budget(1 << 20) == L.LBB_OK
    try:
        with pytest.raises(L.LbbError) as e:
            L.Domain(L.Params(nx=512, ny=256))
        assert e.value.code == L.LBB_ENOMEM and "budget" in str(e.value)
        assert lib.lbb_device_bytes_held() == 0
    finally:
        assert lib.lbb_set_device_budget(0) == L.LBB_OK


def test_step_noalloc_argument_checks():
    """lbb_step_noalloc refuses bad arguments before touching the device:
    missing buffers, n < 0, a phase other than 0/1, and a lattice whose
    partial sums would not fit the library's static scratch array (the
    message names the bytes needed)."""
    p = L.Params(nx=64, ny=32)
    fake = [0x1000, 0x2000]
    with pytest.raises(L.LbbError) as e:
        L.step_noalloc(p, [0, 0], fake, 0x3000, 0x4000, 0x5000, [0, 0], 1, 0x6000)
    assert e.value.code == L.LBB_EINVAL
    with pytest.raises(L.LbbError) as e:
        L.step_noalloc(p, fake, fake, 0x3000, 0x4000, 0x5000, [0, 0], -1, 0x6000)
    assert e.value.code == L.LBB_EINVAL
    with pytest.raises(L.LbbError) as e:
        L.step_noalloc(p, fake, fake, 0x3000, 0x4000, 0x5000, [2, 0], 1, 0x6000)
    assert e.value.code == L.LBB_EINVAL
    big = L.Params(nx=8192, ny=8192, precision=L.FP32)
    with pytest.raises(L.LbbError) as e:
        L.step_noalloc(big, fake, fake, 0x3000, 0x4000, 0x5000, [0, 0], 1, 0x6000)
    assert e.value.code == L.LBB_EINVAL and "scratch bytes" in str(e.value)


def test_read_and_adjoint_reject_a_null_domain():
    """The read-back, heat-flux and adjoint calls check their handle before
    touching the device (this runs without a GPU)."""
    lib = L.lib()
    assert lib.lbb_read_fields(None, L.FIELD_ALL, None, None, None, None, None) == L.LBB_EINVAL
    assert lib.lbb_wall_heat_flux(None, None, None, None, None) == L.LBB_EINVAL
    assert lib.lbb_adjoint(None, 10, 0, None, 0, None, None, None) == L.LBB_EINVAL
    assert L.FIELD_ALL == L.FIELD_RHO | L.FIELD_UX | L.FIELD_UY | L.FIELD_T | L.FIELD_F
