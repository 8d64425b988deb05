"""Post-processing of recorded series (Sec. III and IV quantities) against
signals whose answers are known in closed form."""
import math

import numpy as np
import pytest

from paper_1710_02065_amd import acoustics as A


def tone(n, period, amp=1.0, phase=0.3, offset=0.0):
    t = np.arange(n)
    return offset + amp * np.sin(2 * math.pi * t / period + phase)


def test_crossing_period_and_strouhal():
    x = tone(20000, 473.21, amp=0.5, offset=0.2)
    assert A.crossing_period(x) == pytest.approx(473.21, rel=1e-6)
    # St = f D / U with f = 1 / (period * dt)
    D, U, dt = 100.0, 0.11547, 2.0
    st = A.strouhal(x, D, U, dt=dt)
    assert st == pytest.approx(D / (473.21 * dt * U), rel=1e-6)
    assert A.crossing_period(np.ones(100)) is None


def test_peak_frequency():
    x = tone(8192, 61.7) + 0.1 * tone(8192, 9.3)
    assert A.peak_frequency(x) == pytest.approx(1 / 61.7, rel=2e-3)


def test_amplitude_and_coefficients():
    x = tone(10000, 100.0, amp=0.55, offset=1.3)
    assert A.amplitude(x) == pytest.approx(0.55, rel=1e-3)  # sampled crest
    F = np.array([[2.0, -1.0, 0.0]])
    cd, cl = A.force_coefficients(F, rho0=1.0, U=0.1, D=100.0)
    assert cd[0] == pytest.approx(2.0 / (0.5 * 0.01 * 100))
    assert cl[0] == pytest.approx(-1.0 / (0.5 * 0.01 * 100))


def test_psd_parseval_and_oaspl():
    amp, pref = 3e-3, 1e-5
    x = tone(16384, 37.3, amp=amp, offset=1.0 / 3.0)
    f, P = A.psd(x)
    assert P.sum() * (f[1] - f[0]) == pytest.approx(amp ** 2 / 2, rel=2e-3)
    assert A.oaspl(x, pref) == pytest.approx(10 * math.log10(amp ** 2 / 2 / pref ** 2), abs=0.01)
    rng = np.random.default_rng(0)
    w = rng.normal(0.0, 0.2, 1 << 16)
    f, P = A.psd(w, dt=0.5)
    assert P.sum() * (f[1] - f[0]) == pytest.approx(0.04, rel=0.02)
    # white noise: flat one-sided density 2 sigma^2 dt on average
    assert np.mean(P[10:-10]) == pytest.approx(2 * 0.04 * 0.5, rel=0.03)


def test_third_octave_bands_and_levels():
    fc, lo, hi = A.third_octave_bands(1e-3, 0.2)
    np.testing.assert_allclose(fc[1:] / fc[:-1], 2 ** (1 / 3))
    np.testing.assert_allclose(lo[1:], hi[:-1])
    assert np.all((fc >= 1e-3) & (fc <= 0.2))
    # a tone at a band centre puts its whole energy in that band
    k = 8
    amp, pref = 1e-3, 1e-6
    x = tone(1 << 15, 1.0 / fc[k], amp=amp)
    L = A.band_levels(x, 1.0, fc, lo, hi, pref)
    assert int(np.argmax(L)) == k
    assert L[k] == pytest.approx(A.oaspl(x, pref), abs=0.05)
    e = (10 ** (L[np.isfinite(L)] / 10)).sum()
    assert 10 * math.log10(e) == pytest.approx(A.oaspl(x, pref), abs=0.05)


def test_spreading_laws():
    assert A.extrapolate_level(100.0, 11.0, 22.0) == pytest.approx(100 - 20 * math.log10(2))
    assert A.extrapolate_level(100.0, 1.0, 10.0, "cylindrical") == pytest.approx(90.0)
    r = np.linspace(150, 450, 9)
    assert A.decay_exponent(r, -3.0 * r ** -0.5) == pytest.approx(-0.5, abs=1e-12)


def test_rms_from_running_sums():
    rng = np.random.default_rng(3)
    x = 1e-3 * rng.normal(size=(500, 7)) + 2e-4
    s1, s2 = x.sum(axis=0), (x * x).sum(axis=0)
    np.testing.assert_allclose(A.rms_from_sums(s1, s2, 500), x.std(axis=0), rtol=1e-9)


def test_directivity_peak_and_ring():
    ang = np.arange(0.0, 181.0, 2.0)
    rms = np.exp(-((ang - 78.2) / 30.0) ** 2)
    assert A.directivity_peak(rms, ang) == pytest.approx(78.2, abs=0.1)
    cells = A.ring_cells(64, 32, 20, 16, 10, [0.0, 90.0, 180.0])
    assert cells.tolist() == [16 * 64 + 30, 26 * 64 + 20, 16 * 64 + 10]


def test_tone_amplitude_rejects_drift_and_other_tones():
    n = 20000
    t = np.arange(n)
    x = (0.7 * np.sin(2 * math.pi * t / 431.0 + 1.1) + 2e-5 * t
         + 0.3 * np.sin(2 * math.pi * t / 97.0))
    assert A.tone_amplitude(x, 1 / 431.0) == pytest.approx(0.7, rel=2e-3)
