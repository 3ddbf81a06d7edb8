"""Every tile shape of the LB and thermal launches against the oracle and
bitwise against the default shapes (the reductions group and order their
partial sums the same way for every tile height, so any difference would be
a race or an indexing error), and the autotuner: it may only change speed,
never the state it was given."""
import itertools

import numpy as np
import pytest

from paper_1501_03857_amd import lbboil as L
from paper_1501_03857_amd import workloads as WL
from parity_utils import compare, make_pair

pytestmark = pytest.mark.gpu

NA, NB = (len(x) for x in L.tile_shapes())
COMBOS = list(itertools.product(range(NA), range(NB)))


def _say(*a):
    print("[gpu-case]", *a, flush=True)


@pytest.fixture(scope="module")
def ragged_walls():
    w = WL.PLAIN_128x64.resized(100, 37, heater=(25, 51), Gw_bottom=0.05)
    o, _, _ = make_pair(w, Gw_top=-0.03)
    o.step(60)
    return w, o


@pytest.fixture(scope="module")
def ragged_periodic():
    w = WL.PLAIN_128x64.resized(70, 37, heater=(10, 30))
    o, _, _ = make_pair(w, periodic_y=1)
    o.step(60)
    return w, o


def _gpu_run(w, shapes, steps, **kw):
    _, d, _ = make_pair(w, **kw)
    d.set_tiles(*shapes)
    assert d.tiles == tuple(shapes)
    d.step(steps)
    return d


@pytest.fixture(scope="module")
def default_walls(ragged_walls):
    w, _ = ragged_walls
    d = _gpu_run(w, (0, 0), 60, Gw_top=-0.03)
    return d.fields(), d.heat_flux()


@pytest.fixture(scope="module")
def default_periodic(ragged_periodic):
    w, _ = ragged_periodic
    return _gpu_run(w, (0, 0), 60, periodic_y=1).fields()


@pytest.fixture(scope="module")
def default_fp32():
    return _gpu_run(WL.PLAIN_128x64, (0, 0), 100, precision=L.FP32).fields()


def _same(a, b):
    for k in ("f", "T", "rho", "ux", "uy"):
        assert np.array_equal(a[k], b[k]), k


@pytest.mark.parametrize("shape_lb,shape_thermal", COMBOS)
def test_every_tile_shape_matches_oracle_walls(ragged_walls, default_walls, shape_lb, shape_thermal):
    _say("tiles walls", shape_lb, shape_thermal)
    w, o = ragged_walls
    d = _gpu_run(w, (shape_lb, shape_thermal), 60, Gw_top=-0.03)
    errs, bad = compare(o, d, 1e-12)
    assert not bad, errs
    _same(d.fields(), default_walls[0])
    hf = d.heat_flux()
    assert hf["q_mean"] == default_walls[1]["q_mean"] and np.array_equal(hf["q_local"], default_walls[1]["q_local"])


@pytest.mark.parametrize("shape_lb,shape_thermal", COMBOS)
def test_every_tile_shape_matches_oracle_periodic(ragged_periodic, default_periodic, shape_lb, shape_thermal):
    _say("tiles periodic", shape_lb, shape_thermal)
    w, o = ragged_periodic
    d = _gpu_run(w, (shape_lb, shape_thermal), 60, periodic_y=1)
    errs, bad = compare(o, d, 1e-12)
    assert not bad, errs
    _same(d.fields(), default_periodic)


@pytest.mark.parametrize("shape_lb,shape_thermal", COMBOS)
def test_tile_shapes_fp32(default_fp32, shape_lb, shape_thermal):
    _say("tiles fp32", shape_lb, shape_thermal)
    o, _, _ = make_pair(WL.PLAIN_128x64, precision=L.FP32)
    d = _gpu_run(WL.PLAIN_128x64, (shape_lb, shape_thermal), 100, precision=L.FP32)
    o.step(100)
    errs, bad = compare(o, d, 1e-5)
    assert not bad, errs
    _same(d.fields(), default_fp32)


def test_autotune_leaves_state_and_keeps_parity():
    _say("autotune domain")
    o, d, _ = make_pair(WL.PLAIN_128x64)
    o.step(40)
    d.step(20)
    before, hf0 = d.fields(), d.heat_flux()
    r = d.autotune(6)
    assert 0 <= r["shape_lb"] < NA and 0 <= r["shape_thermal"] < NB
    assert d.tiles == (r["shape_lb"], r["shape_thermal"])
    assert np.all(r["ms_lb"] > 0) and np.all(r["ms_thermal"] > 0)
    after, hf1 = d.fields(), d.heat_flux()
    for k in ("f", "T", "rho", "ux", "uy"):
        assert np.array_equal(before[k], after[k]), k
    assert hf0["n_samples"] == hf1["n_samples"] == 20 and hf0["q_mean"] == hf1["q_mean"]
    d.step(20)
    errs, bad = compare(o, d, 1e-12)
    assert not bad, errs


def test_batch_tiles_and_autotune():
    _say("batch tiles")
    ws = [WL.PLAIN_128x64, WL.PLAIN_128x64.resized(100, 37, heater=(10, 60), Gw_bottom=0.065, seed=5)]
    pairs = [make_pair(w) for w in ws]
    b = L.Batch([L.Params(nx=w.nx, ny=w.ny, liquid_rows=w.liquid_rows, sigma=w.sigma, g=w.g, Gw_bottom=w.Gw_bottom,
                          rho_L=x[2]["rho_L"], rho_V=x[2]["rho_V"]) for w, x in zip(ws, pairs)],
                [x[2]["Tb"] for x in pairs], [w.density(x[2]["rho_L"], x[2]["rho_V"]) for w, x in zip(ws, pairs)])
    b.set_tiles(2, 3)
    b.step(33)
    for i, (_, d, _) in enumerate(pairs):
        d.set_tiles(2, 3).step(33)
        assert np.array_equal(b.domain(i).fields()["f"], d.fields()["f"]), i
    before = [b.domain(i).fields() for i in range(2)]
    r = b.autotune(4)
    assert 0 <= r["shape_lb"] < NA and 0 <= r["shape_thermal"] < NB
    for i in range(2):
        assert np.array_equal(before[i]["f"], b.domain(i).fields()["f"]), i
    b.step(7)
    for i, (_, d, _) in enumerate(pairs):
        d.set_tiles(r["shape_lb"], r["shape_thermal"]).step(7)
        assert np.array_equal(b.domain(i).fields()["f"], d.fields()["f"]), i


@pytest.mark.parametrize("precision", [L.FP64, L.FP32])
def test_ragged_tail_column_bitwise_across_shapes_and_match_oracle(precision):
    """A 130x41 lattice with walls leaves 6 columns in its last LB tile
    column, and 41 rows put the top wall row in the halo of the band below
    it for the 4-row shapes.  Every LB shape bands the rows differently; the
    state must not depend on it, bit for bit, and must match the oracle at
    the parity bars."""
    w = WL.PLAIN_128x64.resized(130, 41, heater=(30, 90), Gw_bottom=0.05)
    tol = 1e-12 if precision == L.FP64 else 1e-5
    o, _, _ = make_pair(w, precision=precision, Gw_top=-0.03)
    o.step(50)
    ref = None
    for sa in range(NA):
        _say(f"ragged tail 130x41 LB shape {sa} precision {precision}")
        d = _gpu_run(w, (sa, 0), 50, precision=precision, Gw_top=-0.03)
        fl, hf = d.fields(), d.heat_flux()
        if ref is None:
            ref = (fl, hf)
            errs, bad = compare(o, d, tol)
            assert not bad, errs
        else:
            for k in ("rho", "ux", "uy", "T", "f"):
                assert np.array_equal(fl[k], ref[0][k]), (sa, k)
            assert hf["q_now"] == ref[1]["q_now"], sa
        d.close()


@pytest.mark.parametrize("nx,periodic", [(256, 0), (384, 1), (512, 0), (90, 1), (152, 0)])
def test_ragged_tail_column_keeps_an_x_invariant_state_x_invariant(nx, periodic):
    """Lattice widths whose last LB tile column holds 8, 12, 16, 28 and 28
    columns (the sweep's widths among them), with walls and periodic: a
    layered state with no noise, a uniform heater and the same wall strength
    everywhere is the same in every column, so after 60 steps every column
    must still be identical bit for bit, for every LB tile shape."""
    for sa in range(NA):
        _say(f"x-invariance nx={nx} periodic={periodic} LB shape {sa}")
        w = WL.PLAIN_128x64.resized(nx, 48, heater=(0, nx), Gw_bottom=0.05, noise_amp=0.0)
        _, d, _ = make_pair(w, periodic_y=periodic)
        d.set_tiles(sa, 0)
        d.step(60)
        fl = d.fields()
        for k in ("rho", "ux", "uy", "T"):
            a = fl[k]
            assert np.array_equal(a, np.repeat(a[:, :1], nx, axis=1)), (nx, sa, k)
        d.close()


@pytest.mark.parametrize("precision", [L.FP64, L.FP32])
@pytest.mark.parametrize("nx,ny,periodic", [(130, 41, 0), (20, 40, 1), (90, 45, 0), (512, 37, 1), (256, 9, 0)])
def test_graph_replays_match_single_launches_bitwise(precision, nx, ny, periodic):
    """Steps come either from replays of 32-step graphs or from single
    launches; both must reach the same state bit for bit, for every LB tile
    shape, on lattices whose last tile column is 6, 20, 28, 16 and 8 columns
    wide (20x40: one tile column, its halo columns wrapped across the lattice)
    and whose row count leaves ragged last bands; the heat-flux history as
    well."""
    w = WL.PLAIN_128x64.resized(nx, ny, heater=(nx // 5, nx - nx // 5), Gw_bottom=0.05, seed=11)
    for sa in range(NA):
        _say(f"graphs vs single launches {nx}x{ny} periodic={periodic} LB shape {sa} precision {precision}")
        _, dg, _ = make_pair(w, precision=precision, periodic_y=periodic)
        _, ds, _ = make_pair(w, precision=precision, periodic_y=periodic)
        dg.set_tiles(sa, 0)
        ds.set_tiles(sa, 0)
        dg.step(64)
        for _ in range(64):
            ds.step(1)
        a, b = dg.fields(), ds.fields()
        for k in ("f", "T", "rho", "ux", "uy"):
            assert np.array_equal(a[k], b[k]), (sa, k)
        ha, hb = dg.heat_flux(), ds.heat_flux()
        assert ha["q_mean"] == hb["q_mean"] and ha["n_samples"] == hb["n_samples"] == 64, sa
        dg.close()
        ds.close()


def test_single_tile_column_matches_oracle():
    """A lattice of one tile column (20 wide, periodic in y): every tile's
    halo columns wrap across the whole lattice.  After two graph replays it
    must match the oracle at the parity bar."""
    _say("one tile column 20x40 vs oracle")
    w = WL.PLAIN_128x64.resized(20, 40, heater=(4, 16), Gw_bottom=0.05, seed=11)
    o, d, _ = make_pair(w, periodic_y=1)
    o.step(64)
    d.step(64)
    errs, bad = compare(o, d, 1e-12)
    assert not bad, errs
