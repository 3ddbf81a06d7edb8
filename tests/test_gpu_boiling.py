"""The paper's boiling experiments on the batched GPU path (Sec. 3.2, 3.3):
33 pools of 600 x 151 (a = 3/49) at 11 superheats and 3 wall strengths in
one batch, superheat step from 0.0137 at t = 20000, q averaged over
t = 30000..60000.  The paper's curves are not in its text, so the checks are
its stated regimes and trends (parity unpinned: chaotic runs, qualitative
agreement only):
  - no boiling at the lowest superheat, a critical heat flux near
    0.021-0.025 and a large drop towards film boiling at 0.035;
  - the largest heat transfer coefficient at a lower superheat than the
    critical heat flux;
  - a larger contact angle (larger G_w) lowers the critical heat flux,
    starts boiling earlier, and the curves cross;
  - the top-wall-centre pressure rises as vapour collects, more for the
    higher superheat (Fig. 3)."""
import numpy as np
import pytest

from paper_1501_03857_amd import experiments as E

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def curve():
    print("[gpu-case] boiling curves: 33 x 600x151, 60000 steps", flush=True)
    runs, info = E.boiling_curve(probe=[(0.0137, 0.0), (0.0165, 0.0)])
    print(f"[gpu-case] {info}", flush=True)
    reg = E.regimes(runs)
    for Gw, r in reg.items():
        print(f"[gpu-case] G_w {Gw}: " + " ".join(f"{d}:{q:.3e}" for d, q in zip(r["dT"], r["q_mean"])), flush=True)
    return runs, reg


def _q(reg, Gw, dT):
    r = reg[Gw]
    return r["q_mean"][r["dT"].index(dT)]


def test_boiling_curve_regimes(curve):
    """Thresholds leave room for the run-to-run spread of these chaotic runs:
    any change of rounding moves individual bubbles, and near the transition
    a 30000-step average still varies by some 20% (the q at 0.035 over the
    critical heat flux has ranged over 0.33-0.47, 0.47-0.60 and 0.10-0.16 for
    the three walls)."""
    _, reg = curve
    drops = []
    for Gw, r in reg.items():
        chf = r["q_chf"]
        assert _q(reg, Gw, 0.008) < 0.25 * chf, (Gw, "boiling at the lowest superheat")
        assert 0.019 <= r["dT_chf"] <= 0.029, (Gw, r["dT_chf"])
        drops.append(_q(reg, Gw, 0.035) / chf)
        assert drops[-1] < 0.75, (Gw, "no drop towards film boiling")
        assert r["dT_hmax"] < r["dT_chf"], (Gw, r["dT_hmax"], r["dT_chf"])
    assert np.mean(drops) < 0.6, drops


def test_wettability_trends(curve):
    _, reg = curve
    assert reg[0.0]["q_chf"] > reg[0.065]["q_chf"] > reg[0.105]["q_chf"]
    assert _q(reg, 0.105, 0.01) > _q(reg, 0.0, 0.01)     # earlier onset with the larger contact angle
    assert _q(reg, 0.105, 0.029) < _q(reg, 0.0, 0.029)   # the curves cross


def test_top_wall_pressure_rises(curve):
    runs, _ = curve
    p = {r.dT: r for r in runs if r.p_top is not None}
    before = p[0.0137].p_top[p[0.0137].t <= 20000].mean()
    late = {d: r.p_top[r.t > 40000].mean() for d, r in p.items()}
    assert late[0.0137] > before and late[0.0165] > late[0.0137], (before, late)
