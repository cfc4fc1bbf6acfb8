"""Writes c1_green_mp50.npz: G(0) and G(10) of the L=3, U=-4, beta=2 kagome
workload (mu = -t, the Dirac energy), seed-3 fields, computed by the oracle's
50-digit brute force (plain product of multiprecision matrix exponentials and
a plain inverse).  Calls only ``oracle/`` and ``seeded_inputs``."""
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import seeded_inputs as si  # noqa: E402
from oracle import brute, dqmc  # noqa: E402


def main():
    w = si.C1
    m = dqmc.Model.from_workload(w, mu=-1.0)
    f = si.ising_fields(w.L, m.L_tau, w.seed)
    e = brute.mp_propagator(m, dps=50)
    out = {"fields": f}
    for l in (0, 10):
        out[f"G{l}"] = brute.mp_green(m, f, l, dps=50, e=e)
    np.savez(os.path.join(HERE, "c1_green_mp50.npz"), **out)


if __name__ == "__main__":
    main()
