"""Checks of the seeded input generators (harness, no method arithmetic)."""
import math

import numpy as np
import pytest

from paper_2207_06908_amd import scenarios as S


@pytest.mark.parametrize("T1,T2", [(1e-6, 50e-6), (0.5e-6, 10e-6), (1.5e-6, 10e-6), (1e-6, 10e-6)])
def test_double_exponential_front_and_tail(T1, T2):
    """The solved double exponential has peak 1 and reproduces T1 / T2 when the
    10 / 90 / 50 % crossings are measured on a fine sampling of the curve."""
    a, b, k = S.dexp_params(T1, T2)
    dt = T1 / 2000.0
    n = int(3 * T2 / dt)
    w = S.double_exponential(n, dt, 1.0, T1, T2)
    t = S.sample_times(n, dt)
    assert abs(w.max() - 1.0) < 1e-6
    ip = int(np.argmax(w))
    t10 = np.interp(0.1, w[:ip], t[:ip])
    t90 = np.interp(0.9, w[:ip], t[:ip])
    t50 = np.interp(0.5, w[ip:][::-1], t[ip:][::-1])
    T1m = 1.25 * (t90 - t10)
    T2m = t50 - (t10 - 0.1 * T1m)
    assert abs(T1m / T1 - 1) < 1e-3 and abs(T2m / T2 - 1) < 1e-3


def test_gaussian_sampling_times():
    dt = 1e-9
    g = S.gaussian(100, dt, 40 * dt, 12 * dt)
    assert g.argmax() in (39, 40)
    assert g[39] == pytest.approx(math.exp(-((39.5 - 40) / 12) ** 2))


def test_config1_probes_seeded_and_distinct():
    a, b = S.config1(), S.config1()
    assert [p[3:6] for p in a.probes] == [p[3:6] for p in b.probes]
    locs = {p[3:6] for p in a.probes}
    assert len(locs) == 8 and (24, 24, 24) not in locs


def test_config3_grids_fit_and_are_uneven():
    grids = S.config3(n_grids=32, n_steps=10)
    sizes = {(g.nx, g.ny, g.nz) for g in grids}
    assert len(sizes) > 20
    for g in grids:
        assert 32 <= g.ny <= 96 and 32 <= g.nz <= 96 and g.nx <= 96 or g.nx > 96
        ks, ke = g.meta["ks"], g.meta["ke"]
        assert g.npml < ke < ks < g.nz - g.npml


def test_config2_full_geometry():
    sc = S.config2(n_steps=4)
    assert (sc.nx, sc.ny, sc.nz) == (512, 512, 384)
    assert sc.meta["ks"] == 192 and sc.meta["kg"] == 252
    assert sc.wires[0][:5] == (2, 256, 256, 192, 60)
    names = [p[0] for p in sc.probes]
    assert "V_Ex(k=192)" in names and "V_Ex(k=252)" in names and "I_source" in names


def test_heidler_waveform_closed_forms():
    """Heidler current: zero before the delay, (I0 / eta) e^(-tau1 / tau2) / 2
    one tau1 after it, and at (1/2) tau1 the x^n factor 2^-n / (1 + 2^-n)."""
    import math
    import numpy as np
    from paper_2207_06908_amd import scenarios as S
    dt, tau1, tau2, n, t_d = 1e-9, 3.7e-7, 1.4e-5, 10.0, 1.85e-7
    w = S.heidler(2000, dt, 2.0, tau1, tau2, n, 1.5, t_d)
    t = (np.arange(2000) + 0.5) * dt
    assert np.all(w[t <= t_d] == 0.0)
    for frac in (0.5, 1.0):
        tq = t_d + frac * tau1
        idx = int(round(tq / dt - 0.5))
        x = (((idx + 0.5) * dt - t_d) / tau1) ** n
        want = 2.0 / 1.5 * x / (1 + x) * math.exp(-((idx + 0.5) * dt - t_d) / tau2)
        assert w[idx] == pytest.approx(want, rel=1e-12)
    assert np.argmax(w) > (t_d + tau1) / dt
