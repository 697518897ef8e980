"""Writes equal_dispersion_accuracy.json from the oracle only (python tests/golden/make_equal_dispersion_accuracy.py).

Sec. 3 compares OVFEM with the lumped trilinear element ("VFEM") at equal accuracy: the
trilinear mesh must be finer.  Without the paper's reference solutions, accuracy is
measured here by numerical dispersion: the RMS relative phase-velocity error of the
semi-discrete plane waves (oracle Bloch analysis), over 128 directions of a hemisphere
(Fibonacci points) and the three branches (two S at the given points per S wavelength,
P at twice that), Vp = 2 Vs.  For each OVFEM resolution the trilinear resolution with
the same error is found by bisection; a mesh finer by 1/r costs r^3 elements and r
times the steps (dt proportional to h), r^4 in all.
"""
import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import dispersion as dsp  # noqa: E402
from oracle import element as el  # noqa: E402

LAM, MU, RHO = 2.0, 1.0, 1.0
VS, VP = np.sqrt(MU / RHO), np.sqrt((LAM + 2 * MU) / RHO)


def directions(n=128):
    i = np.arange(n) + 0.5
    phi = np.arccos(1 - i / n)
    th = np.pi * (1 + 5 ** 0.5) * i
    return np.stack([np.cos(th) * np.sin(phi), np.sin(th) * np.sin(phi), np.cos(phi)], 1)


def rms_phase_error(K, ppw_s, dirs):
    e = []
    for d in dirs:
        cs = dsp.phase_velocities(K, RHO, 1.0, d, 2 * np.pi / ppw_s)
        cp = dsp.phase_velocities(K, RHO, 1.0, d, 2 * np.pi / (2 * ppw_s))
        e += [cs[0] / VS - 1, cs[1] / VS - 1, cp[2] / VP - 1]
    return float(np.sqrt(np.mean(np.square(e))))


def equal_accuracy(ppw_ovfem, dirs, iters=40):
    Kl, Km = el.ovfem_reference()
    Kov = LAM * Kl + MU * Km
    Ktr = el.trilinear_stiffness(LAM, MU, 1.0)
    e0 = rms_phase_error(Kov, ppw_ovfem, dirs)
    lo, hi = float(ppw_ovfem), 20.0 * ppw_ovfem
    for _ in range(iters):
        mid = np.sqrt(lo * hi)
        if rms_phase_error(Ktr, mid, dirs) > e0:
            lo = mid
        else:
            hi = mid
    r = hi / ppw_ovfem
    return {"ppw_ovfem": ppw_ovfem, "rms_phase_error": e0, "ppw_trilinear": hi, "h_ratio": 1.0 / r, "cost_factor": r ** 4}


def main():
    dirs = directions()
    rows = [equal_accuracy(p, dirs) for p in (5, 10, 20)]
    out = {"source": "tests/golden/make_equal_dispersion_accuracy.py (oracle Bloch analysis)",
           "measure": "RMS relative phase-velocity error, 128 hemisphere directions x (S1, S2, P), Vp = 2 Vs",
           "rows": rows}
    with open(os.path.join(HERE, "equal_dispersion_accuracy.json"), "w") as f:
        json.dump(out, f, indent=1)
    print(json.dumps(out, indent=1))


if __name__ == "__main__":
    main()
