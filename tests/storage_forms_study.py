"""Sixteen-bit storage forms emulated on the FP64 oracle.

Each form keeps the state as f_i = w_i rho0 + R(f_i - w_i rho0) after every
step, R rounding the shifted value (the rest-weight shift of the
FP16-shifted storage) to the form's grid with round-to-nearest-even:

* F16S: IEEE binary16 (5 exponent bits, 10 mantissa bits);
* F16C: a custom 16-bit float with 4 exponent bits and 11 mantissa bits
  (bias 15: normal magnitudes 2^-14 .. 2 - 2^-11, subnormal step 2^-25),
  the format Lehmann et al. (2022) pair with the shift: one more mantissa
  bit than binary16 for a range that still holds every shifted value;
* F32S: binary32, for scale.

Workload: the D3Q19 Taylor-Green vortex with an acoustic pulse, tau 0.52
(U = 0.1 cs, pulse 1e-3 rho0), scaled from 256^3 to n^3 (pulse sigma
scaled with n); the error is the relative L2 norm of p' = cs^2 (rho - rho0)
against the unrounded FP64 run at each horizon.

Run as `python -m tests.storage_forms_study [n] [horizons...]`.
"""
import math
import sys

import numpy as np

import oracle as O
from paper_1710_02065_amd import workloads as W


def round_float(x, mant_bits, emin, emax):
    """Round x to a binary float grid with `mant_bits` stored mantissa bits,
    normal exponents emin .. emax and subnormals below 2^emin, nearest even;
    magnitudes beyond the largest normal saturate to it."""
    a = np.abs(x)
    _, e = np.frexp(a)                       # a = m 2^e, m in [0.5, 1)
    E = np.maximum(e - 1, emin)              # exponent of the leading bit
    ulp = np.ldexp(1.0, E - mant_bits)
    q = np.round(a / ulp) * ulp              # numpy rounds halves to even
    top = (2.0 - 2.0 ** -mant_bits) * 2.0 ** emax
    return np.sign(x) * np.minimum(q, top)


FORMS = {
    "f16s": lambda h: h.astype(np.float16).astype(np.float64),
    "f16c": lambda h: round_float(h, 11, -14, 0),
    "f32s": lambda h: h.astype(np.float32).astype(np.float64),
}


def workload(n):
    U = 0.1 / math.sqrt(3)
    return W.taylor_green_3d(n, U, pulse_amp=1e-3, pulse_sigma=8.0 * n / 256.0)


def run(n=40, horizons=(100, 300, 500), forms=("f16s", "f16c")):
    rho, u = workload(n)
    _, w, _ = O.lattice(19)
    shift = w[:, None] * 1.0
    ref = O.Grid(19, n, n, n, tau=0.52).init(rho, u)
    grids = {k: O.Grid(19, n, n, n, tau=0.52).init(rho, u) for k in forms}
    for k, g in grids.items():
        g.f = shift + FORMS[k](g.f - shift)
    out = {}
    done = 0
    for T in horizons:
        while done < T:
            ref.step(1)
            for k, g in grids.items():
                g.step(1)
                g.f = shift + FORMS[k](g.f - shift)
            done += 1
        p_ref = (ref.moments()[0] - 1.0) / 3.0
        out[T] = {k: float(np.linalg.norm((g.moments()[0] - 1.0) / 3.0 - p_ref)
                           / np.linalg.norm(p_ref)) for k, g in grids.items()}
    return out


if __name__ == "__main__":
    n = int(sys.argv[1]) if len(sys.argv) > 1 else 40
    hs = tuple(int(v) for v in sys.argv[2:]) or (500, 5000)
    res = run(n, hs, ("f16s", "f16c", "f32s"))
    print("D3Q19 %d^3, relative L2 error of p' against FP64" % n)
    for T, row in res.items():
        print("%6d " % T + "  ".join("%s %.3e" % kv for kv in row.items()), flush=True)
