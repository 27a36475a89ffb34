"""Host checks of the input generators added for the time-step, verification and
learned-preconditioner work: determinism per seed and the documented structure."""
import numpy as np

import workloads as W


def test_diffusive_lognormal_is_seeded_and_in_range():
    a = W.diffusive_lognormal(n=(64, 32), seed=3)
    b = W.diffusive_lognormal(n=(64, 32), seed=3)
    c = W.diffusive_lognormal(n=(64, 32), seed=4)
    assert np.array_equal(a["sigma"], b["sigma"]) and np.array_equal(a["E"], b["E"])
    assert not np.array_equal(a["sigma"], c["sigma"])
    assert a["sigma"].shape == (32, 64)
    assert a["sigma"].min() >= 3.0 and a["sigma"].max() <= 300.0
    assert a["E"].min() >= 1e-6 and np.all(a["F"] == 0.0)
    assert a["bc"][:4] == ["periodic"] * 4 and a["flux_source"] == "wb" and a["dt"] == 1000.0


def test_beam45_boundary_rows():
    p = W.beam45()
    g = p["ghost"][0]
    on = np.flatnonzero(g[1] > 0)
    assert on.tolist() == list(range(8, 16))                   # y in [-0.875, -0.75] on 128 rows
    assert np.allclose(g[0][on], 1.0) and np.allclose(g[1][on], g[2][on])
    assert np.allclose(np.hypot(g[1][on], g[2][on]), p["c"] * g[0][on])   # reduced flux 1
    off = np.setdiff1d(np.arange(128), on)
    assert np.allclose(g[0][off], 0.3 ** 4) and np.all(g[1][off] == 0)
    assert np.all(p["sigma"] == 0) and p["lambda_floor"] == 0.0
    assert W.beam45(lambda_floor=1.0)["lambda_floor"] == 1.0


def test_one_dimensional_verification_inputs():
    m = W.marshak_1d()
    assert m["n"] == (400, 1) and m["source"] == "coupled_t"
    assert np.all(m["sigma"] * m["dx"] == 25.0) and np.allclose(m["T"], 0.3)
    assert np.allclose(m["E"], 0.3 ** 4) and m["ghost"][0][0, 0] == 1.0
    assert not W.marshak_1d(ap=False)["ap"]
    j = W.opacity_jump_1d()
    s = j["sigma"][0]
    assert np.all(s[:50] == 100.0) and np.all(s[50:] == 0.0)
    assert j["source"] == "none" and W.opacity_jump_1d(flux_source="centered")["flux_source"] == "centered"


def test_ionization_front_velocity_is_solenoidal_and_subrelativistic():
    p = W.ionization_front(n=(32, 32, 32), with_velocity=True)
    v = p["velocity"]
    rms = np.sqrt((v ** 2).sum(0).mean())
    assert np.isclose(rms, 0.5 * 3.3e-5, rtol=1e-12)
    # central-difference divergence of a central-difference curl vanishes on the periodic grid
    def dd(f, ax):
        return 0.5 * (np.roll(f, -1, ax) - np.roll(f, 1, ax))
    div = dd(v[0], 2) + dd(v[1], 1) + dd(v[2], 0)
    assert np.abs(div).max() <= 1e-12 * np.abs(v).max()


def test_window_copies_fields_and_settings():
    p = W.voronoi_opacity(n=(64, 48), nsites=5, seed=3)
    q = W.window(p, (10, 7), (20, 12), ("periodic",) * 4)
    assert q["n"] == (20, 12) and q["sigma"].shape == (12, 20) and q["F"].shape == (2, 12, 20)
    assert np.array_equal(q["sigma"], p["sigma"][7:19, 10:30])
    assert np.array_equal(q["E"], p["E"][7:19, 10:30])
    assert q["dt"] == p["dt"] and q["flux_source"] == p["flux_source"] and q["bc"][:4] == ["periodic"] * 4
    q["E"][0, 0] = -1.0
    assert p["E"][7, 10] != -1.0
