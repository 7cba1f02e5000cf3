"""Write acoustic_iso.json: the equal-accuracy element sizes of the paper's
acoustic experiment (Sec. V-C) from the FP64 oracle's rod runs.

For each polynomial degree p = 4, 7, 15 (NGLL 5, 8, 16): the waveform error
at a station 12 km (8 s of travel) from a 20 Hz Ricker plane source, in a
homogeneous medium (1000 kg/m^3, 1500 m/s), dt = 1e-4 s, against the
closed-form solution, on a grid of element sizes; then the largest element
size whose relative L2 error stays at or below 1 % (error ratio 1e-4), by
bisection between the last passing and the first failing grid size.  Also
the time-step check on a resolved mesh (degree 8, h = 24 m).  Calls only
``oracle/``; run from the repository root:
    python tests/golden/make_acoustic_iso.py
"""
import json
import os
import sys

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__)))))
from oracle import acoustic as A  # noqa: E402

BOUND = 1e-4  # error ratio of a 1 % relative L2 error
GRID = {5: [10.0, 12.5, 15.0, 17.5, 20.0, 22.5, 25.0],
        8: [30.0, 35.0, 40.0, 45.0, 50.0, 55.0, 60.0],
        16: [90.0, 100.0, 110.0, 120.0, 130.0, 140.0, 150.0]}


def h_max(n, errs, tol=0.05):
    hs = sorted(errs)
    last_pass = None
    for h in hs:
        if errs[h] <= BOUND:
            last_pass = h
        elif last_pass is not None:
            lo, hi = last_pass, h
            while hi - lo > tol:
                mid = 0.5 * (lo + hi)
                e = A.rod_error(n, mid)
                print(f"  n={n} h={mid:.3f} ratio={e:.4e}", flush=True)
                lo, hi = (mid, hi) if e <= BOUND else (lo, mid)
            return lo
    return last_pass


def main():
    out = {"medium": {"rho": A.RHO, "vp": A.VP}, "f0": A.F0, "dt": A.DT, "x_rec": A.VP * A.T_PROP,
           "error": "sum (w - w_th)^2 / sum w_th^2 over the recording", "bound_ratio": BOUND,
           "time_step_check": {}, "orders": {}}
    for dt in (1e-4, 2e-4):
        e = A.rod_error(9, 24.0, dt=dt)
        out["time_step_check"][f"{dt:g}"] = e
        print(f"time step {dt:g}: ratio {e:.4e}", flush=True)
    for n, grid in GRID.items():
        errs = {}
        for h in grid:
            errs[h] = A.rod_error(n, h)
            print(f"n={n} h={h} ratio={errs[h]:.4e}", flush=True)
        hm = h_max(n, errs)
        out["orders"][str(n)] = {"p": n - 1, "errors": {f"{h:g}": e for h, e in errs.items()}, "h_max": hm,
                                 "error_at_h_max": A.rod_error(n, hm)}
        print(f"n={n}: h_max = {hm:.3f} m", flush=True)
    with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "acoustic_iso.json"), "w") as f:
        json.dump(out, f, indent=1)


if __name__ == "__main__":
    main()
