"""Stability of the collision operators (Sec. II.A: the regularized
operator is claimed more stable than LBM-BGK and LBM-MRT): for each
operator, the smallest relaxation time tau (largest Reynolds number) at
which a D2Q9 doubly periodic thick shear layer stays finite, found by
bisection in log(tau - 1/2).

    python -m paper_1710_02065_amd.stability_study [--n 128 --ma 0.2 ...]

prints one JSON line.  Every step runs in the HIP library.
"""
import argparse
import json
import math
import sys

import numpy as np

from . import lbm
from . import workloads as W

CS = math.sqrt(1.0 / 3.0)
OPERATORS = {"regularized_third": 0, "regularized_full": lbm.LBM_FULL_ORDER,
             "bgk": lbm.LBM_BGK, "mrt": lbm.LBM_MRT}


def stays_finite(flags, n, U, tau, steps, storage):
    """True if the shear layer runs `steps` steps with finite, positive
    density and |u| < 1 everywhere."""
    import torch
    rho, u = W.double_shear_layer(n, U)
    sim = lbm.Simulation(lattice=9, shape=(n, n, 1), tau=tau, storage=storage, flags=flags)
    sim.init(rho, u)
    sim.step(steps)
    try:
        r, uu = sim.moments()
        ok = bool(torch.isfinite(r).all()) and float(r.min()) > 0 and \
            float(uu.abs().max()) < 1.0
        sim.sync()
    except lbm.LbmError:
        ok = False
    sim.close()
    return ok


def min_stable_tau(flags, n, U, steps, storage, lo=1e-5, hi=0.3, iters=14):
    """Bisection on x = log(tau - 1/2) between lo and hi (hi must be
    stable); returns the smallest tau found stable."""
    if not stays_finite(flags, n, U, 0.5 + hi, steps, storage):
        return None
    if stays_finite(flags, n, U, 0.5 + lo, steps, storage):
        return 0.5 + lo
    a, b = math.log(lo), math.log(hi)  # a unstable, b stable
    for _ in range(iters):
        m = 0.5 * (a + b)
        if stays_finite(flags, n, U, 0.5 + math.exp(m), steps, storage):
            b = m
        else:
            a = m
    return 0.5 + math.exp(b)


def run(n=128, ma=0.2, periods=4.0, storage="f64", operators=None, log=None):
    U = ma * CS
    steps = int(periods * n / U)
    res = dict(workload="D2Q9 %dx%d doubly periodic thick shear layer (width 80, delta "
                        "0.05), Ma %.2f, %d steps (%g advection periods), %s storage"
                        % (n, n, ma, steps, periods, storage),
               steps=steps, operators={})
    for name in operators or OPERATORS:
        t = min_stable_tau(OPERATORS[name], n, U, steps, storage)
        if log:
            log("%s: min stable tau %s" % (name, t))
        res["operators"][name] = None if t is None else dict(
            min_stable_tau=round(t, 7), max_stable_re=round(U * n / ((t - 0.5) / 3.0), 1))
    return res


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--n", type=int, default=128)
    ap.add_argument("--ma", type=float, default=0.2)
    ap.add_argument("--periods", type=float, default=4.0)
    ap.add_argument("--storage", default="f64")
    args = ap.parse_args(argv)
    print(json.dumps(run(args.n, args.ma, args.periods, args.storage,
                         log=lambda m: print(m, file=sys.stderr, flush=True))), flush=True)


if __name__ == "__main__":
    main()
