"""Write iso_accuracy.json: equal-accuracy resolutions of the GLL spectral
element discretisation.

For each NGLL 2..16 and each target relative phase-velocity error eps, the
number of GLL points per wavelength at which a plane wave along a lattice
axis reaches eps (and stays below it at finer resolution), from the
oracle's Bloch analysis (oracle/dispersion.py, iso_accuracy_ppw).  These are
the equal-error (h, p) configurations of the paper's dispersion-based
iso-accuracy study (Sec. IV-B, Sec. V-C), here for the elastic operator and
a prescribed error instead of a measured waveform misfit.  Run from the
repository root:  python tests/golden/make_iso_accuracy.py
"""
import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

EPS = (1e-3, 1e-4, 1e-5)
NGLL = tuple(range(2, 17))


def table():
    from oracle import dispersion as Dp
    return {"what": "GLL points per wavelength at which the relative phase-velocity error of a plane wave "
                    "along a lattice axis equals eps (1-D Bloch analysis of the oracle)",
            "eps": list(EPS), "ngll": list(NGLL),
            "ppw": [[round(Dp.iso_accuracy_ppw(n, e), 6) for n in NGLL] for e in EPS]}


if __name__ == "__main__":
    out = os.path.join(os.path.dirname(os.path.abspath(__file__)), "iso_accuracy.json")
    with open(out, "w") as fh:
        json.dump(table(), fh, indent=1)
        fh.write("\n")
    print(out)
