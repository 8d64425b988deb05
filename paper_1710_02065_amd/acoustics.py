"""Aeroacoustic post-processing of the time series the library records
(forces from lbm_force, probe densities from lbm_probe, running field sums
from lbm_accumulate).  Host-side analysis of small arrays: nothing here
touches the lattice.

Sec. III (cylinder): lift and drag coefficients, the shedding Strouhal
number St = f D / U, the fluctuating pressure (the pressure minus its
temporal mean) and its rms directivity, and the decay of wave peaks with
distance.  Sec. IV (jet): narrow-band and one-third-octave spectra of probe
pressure, overall sound pressure level, and extrapolation of levels from
the probe radius to a far-field radius assuming spherical spreading.

Lattice units throughout: p = cs^2 rho with cs^2 = 1/3, one time step = 1.
"""
import math

import numpy as np

CS2 = 1.0 / 3.0


def force_coefficients(F, rho0, U, D, span=1.0):
    """(C_D, C_L) from forces F [..., 3] on a body of diameter D and the given
    span (1 in 2D): C = F / (rho0 U^2 D span / 2) for the x and y
    components."""
    F = np.asarray(F, dtype=np.float64)
    q = 0.5 * rho0 * U * U * D * span
    return F[..., 0] / q, F[..., 1] / q


def crossing_period(x, dt=1.0):
    """Mean period of a periodic signal from its upward crossings of its own
    mean, located by linear interpolation between samples (robust for a
    single dominant tone with slowly varying amplitude).  None if fewer than
    two crossings."""
    x = np.asarray(x, dtype=np.float64)
    y = x - x.mean()
    k = np.nonzero((y[:-1] < 0.0) & (y[1:] >= 0.0))[0]
    if len(k) < 2:
        return None
    t = (k + y[k] / (y[k] - y[k + 1])) * dt
    return float((t[-1] - t[0]) / (len(t) - 1))


def peak_frequency(x, dt=1.0):
    """Frequency of the largest peak of the Hann-windowed one-sided spectrum
    of x (mean removed), refined by a parabola through the log magnitudes of
    the peak bin and its neighbours."""
    x = np.asarray(x, dtype=np.float64)
    n = len(x)
    X = np.abs(np.fft.rfft((x - x.mean()) * np.hanning(n)))
    k = int(np.argmax(X[1:]) + 1)
    if 1 <= k < len(X) - 1 and X[k - 1] > 0 and X[k + 1] > 0:
        a, b, c = np.log(X[k - 1]), np.log(X[k]), np.log(X[k + 1])
        den = a - 2 * b + c
        k = k + (0.5 * (a - c) / den if den != 0 else 0.0)
    return float(k / (n * dt))


def strouhal(x, D, U, dt=1.0):
    """St = f D / U of the dominant oscillation of x (from crossing_period;
    None if the signal does not oscillate)."""
    T = crossing_period(x, dt)
    return None if T is None else D / (T * U)


def amplitude(x):
    """Half the peak-to-peak range of x."""
    x = np.asarray(x, dtype=np.float64)
    return 0.5 * float(x.max() - x.min())


def tone_amplitude(x, f, dt=1.0):
    """Amplitude of the component of x at frequency f: least-squares fit of
    c0 + a cos(2 pi f t) + b sin(2 pi f t), returns sqrt(a^2 + b^2).  It
    separates a shedding tone from slow drifts and other frequencies."""
    x = np.asarray(x, dtype=np.float64)
    t = np.arange(len(x)) * dt
    w = 2.0 * math.pi * f
    M = np.stack([np.ones_like(t), np.cos(w * t), np.sin(w * t)], axis=1)
    c = np.linalg.lstsq(M, x, rcond=None)[0]
    return float(math.hypot(c[1], c[2]))


def fluctuation(p, axis=0):
    """Fluctuating pressure: p minus its temporal mean along `axis`."""
    p = np.asarray(p, dtype=np.float64)
    return p - p.mean(axis=axis, keepdims=True)


def rms_from_sums(s1, s2, n):
    """rms of the fluctuation about the temporal mean, from the running sums
    s1 = sum(x) and s2 = sum(x^2) of n samples (as lbm_accumulate keeps for
    x = rho - rho0): sqrt(max(s2/n - (s1/n)^2, 0))."""
    m = np.asarray(s1, dtype=np.float64) / n
    v = np.asarray(s2, dtype=np.float64) / n - m * m
    return np.sqrt(np.maximum(v, 0.0))


def psd(p, dt=1.0):
    """One-sided power spectral density of the fluctuation of p (periodogram
    with a Hann window, scaled so that sum(psd) * df equals the mean square
    of the windowed-and-rescaled signal); returns (frequencies, psd)."""
    p = fluctuation(p)
    n = len(p)
    w = np.hanning(n)
    X = np.fft.rfft(p * w)
    scale = 1.0 / (dt ** -1 * (w * w).sum())
    P = (np.abs(X) ** 2) * scale
    P[1:] *= 2.0
    if n % 2 == 0:
        P[-1] /= 2.0
    return np.fft.rfftfreq(n, dt), P


def third_octave_bands(f_lo, f_hi, f_ref=1.0):
    """Centre, lower and upper edges of the base-2 one-third-octave bands
    f_c = f_ref 2^(k/3) whose centres lie in [f_lo, f_hi]."""
    k0 = math.ceil(3 * math.log2(f_lo / f_ref) - 1e-9)
    k1 = math.floor(3 * math.log2(f_hi / f_ref) + 1e-9)
    fc = f_ref * 2.0 ** (np.arange(k0, k1 + 1) / 3.0)
    return fc, fc * 2 ** (-1 / 6), fc * 2 ** (1 / 6)


def band_levels(p, dt, fc, lo, hi, p_ref):
    """Sound pressure level in dB re p_ref of each band [lo, hi), from the
    PSD of p integrated over the band."""
    f, P = psd(p, dt)
    df = f[1] - f[0]
    out = []
    for a, b in zip(lo, hi):
        m = (f >= a) & (f < b)
        e = P[m].sum() * df
        out.append(10.0 * math.log10(e / p_ref ** 2) if e > 0 else -np.inf)
    return np.array(out)


def oaspl(p, p_ref):
    """Overall sound pressure level in dB re p_ref: 10 log10(<p'^2> / p_ref^2)
    with p' the fluctuation about the temporal mean."""
    ms = float(np.mean(fluctuation(p) ** 2))
    return 10.0 * math.log10(ms / p_ref ** 2)


def extrapolate_level(L, r_from, r_to, spreading="spherical"):
    """Level at r_to from the level L at r_from: amplitude ~ 1/r in 3D
    (spherical, -20 log10 of the radius ratio) and ~ r^-1/2 in 2D
    (cylindrical, -10 log10)."""
    k = 20.0 if spreading == "spherical" else 10.0
    return np.asarray(L, dtype=np.float64) - k * np.log10(r_to / r_from)


def decay_exponent(r, a):
    """Least-squares slope of log|a| against log r: -1/2 for waves spreading
    from a line source in 2D, -1 in 3D."""
    r = np.asarray(r, dtype=np.float64)
    a = np.abs(np.asarray(a, dtype=np.float64))
    return float(np.polyfit(np.log(r), np.log(a), 1)[0])


def directivity_peak(rms, angles_deg):
    """Angle (degrees) of the largest rms value on a ring of probes, refined
    by a parabola through the largest sample and its neighbours."""
    rms = np.asarray(rms, dtype=np.float64)
    ang = np.asarray(angles_deg, dtype=np.float64)
    k = int(np.argmax(rms))
    if 0 < k < len(rms) - 1:
        a, b, c = rms[k - 1], rms[k], rms[k + 1]
        den = a - 2 * b + c
        if den != 0:
            return float(ang[k] + 0.5 * (a - c) / den * (ang[k + 1] - ang[k]))
    return float(ang[k])


def ring_cells(nx, ny, cx, cy, r, angles_deg):
    """Cell indices (row-major, x fastest) nearest to the points at radius r
    and the given angles from the +x axis around (cx, cy)."""
    out = []
    for a in angles_deg:
        t = math.radians(a)
        x = int(round(cx + r * math.cos(t)))
        y = int(round(cy + r * math.sin(t)))
        out.append(min(max(y, 0), ny - 1) * nx + min(max(x, 0), nx - 1))
    return np.array(out, dtype=np.int64)
