"""Host logic of the paper-scale sweep (no GPU): segment plan, checkpoint,
fit and density summaries."""
import json
import math

import pytest

from paper_2507_06579_amd import sweep


def test_segments_cover_and_hit_powers_of_ten():
    for xmax, width in [(10**11, 10**9), (10**8, 10**9), (3 * 10**9 + 7, 10**9)]:
        segs = sweep.segments(xmax, width)
        assert segs[0][0] == 0 and segs[-1][1] == xmax
        assert all(a < b for a, b in segs)
        assert all(segs[i][1] == segs[i + 1][0] for i in range(len(segs) - 1))
        ends = {b for _, b in segs}
        p = 10
        while p <= xmax:
            assert p in ends
            p *= 10
        assert max(b - a for a, b in segs) <= width


def test_fit_recovers_a_planted_coefficient():
    pts = [(x, x / (3 * math.pi ** 2) - 0.031 * x ** (5 / 6)) for x in (10**6, 10**8, 10**10, 10**11)]
    assert sweep.fit_c56(pts) == pytest.approx(-0.031, rel=1e-12)


def test_mean_inv_sixth_root():
    a, b = 10**6, 10**9
    n = 200000
    h = (b - a) / n
    approx = sum((a + (i + 0.5) * h) ** (-1 / 6) for i in range(n)) / n
    assert sweep.mean_inv_sixth_root(a, b) == pytest.approx(approx, rel=1e-6)


def test_checkpoint_round_trip_and_mismatch(tmp_path):
    p = str(tmp_path / "cp.json")
    done = {(0, 10): (1, 0), (10, 100): (10, 3)}
    sweep.save_checkpoint(p, 100, 10**9, done)
    assert sweep.load_checkpoint(p, 100, 10**9) == done
    with pytest.raises(SystemExit):
        sweep.load_checkpoint(p, 1000, 10**9)
    assert json.load(open(p))["segments"][1]["n_eis"] == 3


def test_summary_of_mock_counts():
    done = {(0, 10): (1, 0), (10, 100): (10, 3), (100, 1000): (100, 30)}
    out = sweep.summarise(done, 1000)
    assert out["pi_D"] == 111 and out["pi_E"] == 33
    assert [p["x"] for p in out["powers_of_ten"]] == [10, 100, 1000]
    assert out["powers_of_ten"][-1]["pi_E"] == 33
    assert out["density"][2]["share"] == pytest.approx(0.3)


def test_expint_and_li6_against_quadrature():
    from scipy import integrate, special
    for z in (0.3, 1.0, 5.0, 17.3, 21.1):
        assert sweep.expint_ei(z) == pytest.approx(float(special.expi(z)), rel=1e-13)
    for x in (10.0, 1e4, 1e8):
        ref, _ = integrate.quad(lambda t: t ** (-1 / 6) / math.log(t), 2, x, limit=400)
        assert sweep.li6(x) == pytest.approx(ref, rel=1e-9)
    # li(x) - li(2): the logarithmic integral offset by li(2) = 1.04516378...
    assert sweep.li(1e6) == pytest.approx(78627.549159 - 1.045163780, rel=1e-9)


def test_prime_weighted_mean():
    from scipy import integrate
    a, b = 10**3, 10**6
    num, _ = integrate.quad(lambda t: t ** (-1 / 6) / math.log(t), a, b, limit=400)
    den, _ = integrate.quad(lambda t: 1 / math.log(t), a, b, limit=400)
    assert sweep.prime_mean_inv_sixth_root(a, b) == pytest.approx(num / den, rel=1e-9)
    assert sweep.prime_mean_inv_sixth_root(0, 5) == 0.0


def test_prime_fit_recovers_a_planted_coefficient():
    pts = [(x, x / 40.0, x / 120.0 - 0.041 * sweep.li6(x)) for x in (10**6, 10**8, 10**11)]
    assert sweep.fit_prime_c(pts) == pytest.approx(-0.041, rel=1e-12)


def test_prime_summary_and_checkpoint_set(tmp_path):
    done = {(0, 10): (1, 0), (10, 100): (4, 1), (100, 1000): (36, 12)}
    out = sweep.summarise(done, 1000, "prime")
    assert out["set"] == "prime" and out["pi_DP"] == 41 and out["pi_EP"] == 13
    assert [p["x"] for p in out["powers_of_ten"]] == [10, 100, 1000]
    assert out["density"][2]["share"] == pytest.approx(1 / 3)
    law = out["density"][2]["paper_law"]
    assert law == pytest.approx(1 / 3 - 0.148 * sweep.prime_mean_inv_sixth_root(100, 1000), abs=1e-6)
    p = str(tmp_path / "cp.json")
    sweep.save_checkpoint(p, 1000, 10**9, done, "prime")
    assert sweep.load_checkpoint(p, 1000, 10**9, "prime") == done
    with pytest.raises(SystemExit):
        sweep.load_checkpoint(p, 1000, 10**9, "squarefree")
