"""Host-side logic of the surrogate (no GPU): the network's input map, the
case quantisation and canonical grids, resampling, the double-exponential
source table and the error measures.  Each is checked against something
other than its own formula: exact inverses, closed forms, the IEC time
definitions measured on the produced waveform, or hand-computed values."""
import math

import numpy as np
import pytest

from paper_2207_06908_amd import scenarios as S
from paper_2207_06908_amd import surrogate as U


def _box_cases(n, seed):
    return S.draw_cases(n, seed=seed)


def test_training_box_maps_into_the_unit_box():
    X = U.features(_box_cases(4000, 11))
    assert X.shape == (4000, 5) and X.dtype == np.float32
    assert np.all(X >= -1.0 - 1e-6) and np.all(X <= 1.0 + 1e-6)
    # the box is filled, not squeezed: every input spans most of [-1, 1]
    assert np.all(X.min(axis=0) < -0.8) and np.all(X.max(axis=0) > 0.8)


def test_box_corners_reach_the_ends_of_the_conductance_inputs():
    R = U.RANGES
    lo = S.ElectrodeCase(R["log10_sigma"][0], R["eps_r"][0], 10.0, 0.75, R["T1"][1])
    hi = S.ElectrodeCase(R["log10_sigma"][1], R["eps_r"][1], 10.0, 0.75, R["T1"][0])
    rho_lo = S.ElectrodeCase(R["log10_sigma"][0], R["eps_r"][1], 10.0, 0.75, R["T1"][0])
    rho_hi = S.ElectrodeCase(R["log10_sigma"][1], R["eps_r"][0], 10.0, 0.75, R["T1"][1])
    X = U.features([lo, hi, rho_lo, rho_hi])
    assert X[0, 0] == pytest.approx(-1.0, abs=1e-6) and X[1, 0] == pytest.approx(1.0, abs=1e-6)
    assert X[2, 1] == pytest.approx(-1.0, abs=1e-6) and X[3, 1] == pytest.approx(1.0, abs=1e-6)


def test_input_map_is_invertible_for_sigma_and_eps_r():
    """(log10 g, sigma/g, T1) determine sigma and eps_r: sigma = rho g and
    eps_r = (1 - rho) g T1 / eps0."""
    cases = [U.quantize(c) for c in _box_cases(300, 12)]
    X = U.features(cases).astype(np.float64)
    (g0, g1), (r0, r1), _L, _d, (t0, t1) = U.FEATURE_BOX
    g = 10.0 ** (g0 + (X[:, 0] + 1.0) / 2.0 * (g1 - g0))
    rho = r0 + (X[:, 1] + 1.0) / 2.0 * (r1 - r0)
    T1 = t0 + (X[:, 4] + 1.0) / 2.0 * (t1 - t0)
    sigma = rho * g
    eps_r = (1.0 - rho) * g * T1 / U.EPS0
    want_s = np.array([10.0 ** c.log10_sigma for c in cases])
    want_e = np.array([c.eps_r for c in cases])
    np.testing.assert_allclose(sigma, want_s, rtol=2e-4)
    # eps_r is the small remainder when conduction dominates: compare on the
    # displacement conductance instead
    np.testing.assert_allclose(eps_r * U.EPS0 / T1, want_e * U.EPS0 / T1, rtol=2e-4, atol=2e-4 * g.max())


def test_quantize_and_canonical_grid():
    c = S.ElectrodeCase(-2.0, 10.0, 12.37, 0.62, 1e-6)
    q = U.quantize(c)
    assert q.length == pytest.approx(12.25) and q.depth == pytest.approx(0.5)
    assert U.canonical_dims(q) == (49 + 24, 48, 48)
    short = U.quantize(S.ElectrodeCase(-2.0, 10.0, 5.0, 1.0, 1e-6))
    assert U.canonical_dims(short) == (48, 48, 48)


def test_resample_is_exact_on_linear_ramps():
    n = 2000
    s = np.arange(1, n + 1, dtype=np.float64)
    ramp = np.stack([3.0 * s + 1.0, -0.5 * s])
    out = U.resample(ramp, 256)
    t = np.arange(1, 257) * (n / 256)
    np.testing.assert_allclose(out[0], 3.0 * t + 1.0, rtol=0, atol=1e-9)
    np.testing.assert_allclose(out[1], -0.5 * t, rtol=0, atol=1e-9)
    assert out[0, -1] == ramp[0, -1]  # the last output time is the last sample


@pytest.mark.parametrize("t1", [0.42e-6, 0.9e-6, 1.57e-6])
def test_source_table_reproduces_the_front_and_tail_times(t1):
    """The interpolated (alpha, beta) give a waveform whose IEC front time and
    time to half value, measured on it, are the requested T1 and T2."""
    a, b, k = U.source_table().params(t1)
    T1, T2 = S.dexp_times(a, b)
    assert T1 == pytest.approx(t1, rel=1e-6)
    assert T2 == pytest.approx(U.T2, rel=1e-6)
    tp = math.log(b / a) / (b - a)
    assert k * (math.exp(-a * tp) - math.exp(-b * tp)) == pytest.approx(1.0, rel=1e-12)


def test_source_table_rejects_t1_outside_its_nodes():
    with pytest.raises(ValueError):
        U.source_table().params(2.0e-6)


def test_error_measures_on_hand_values():
    ref = np.array([[0.0, 2.0, 1.0], [1.0, -1.0, 4.0]])
    pred = np.array([[0.0, 2.1, 1.0], [1.0, -1.0, 3.0]])
    np.testing.assert_allclose(U.peak_error(pred, ref), [0.05, 0.25])
    np.testing.assert_allclose(U.l2_error(pred, ref), [0.1 / math.sqrt(5.0), 1.0 / math.sqrt(18.0)])


def test_resistance_scale_is_inverse_in_the_conductance():
    """At fixed geometry the scale is proportional to 1/g: doubling sigma
    with the displacement term removed halves it; and it falls with length."""
    base = S.ElectrodeCase(-2.0, 1e-9, 10.0, 0.75, 1e-6)
    dbl = S.ElectrodeCase(-2.0 + math.log10(2.0), 1e-9, 10.0, 0.75, 1e-6)
    r = U.resistance_scale([base, dbl])
    assert r[0] / r[1] == pytest.approx(2.0, rel=1e-6)
    lengths = [5.0, 8.0, 12.0, 18.0]
    rs = U.resistance_scale([S.ElectrodeCase(-2.0, 10.0, L, 0.75, 1e-6) for L in lengths])
    assert np.all(np.diff(rs) < 0) and np.all(rs > 0)
