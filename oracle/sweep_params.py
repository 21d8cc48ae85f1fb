"""TEST INFRASTRUCTURE: choose (alpha, lambda, tau) once, with the FP64 oracle only.

The paper treats the regularisation weights as known a priori and tau as fixed
ahead of the iterations, and gives no values.  This sweep runs oracle
IRN-PICCS (3 reweightings x 5 LSQR iterations) on the 64^3 / 48-view synthetic
case against its ground truth and prints the grid ranked by relative error.
The winner is stored in paper_2509_08574_amd/synth.py (SOLVE_PARAMS) and used
unchanged by both the oracle checks and the GPU runs.

Usage: python oracle/sweep_params.py
"""
import itertools
import os
import sys

import numpy as np

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))

from oracle import oracle as orc  # noqa: E402
from paper_2509_08574_amd import synth  # noqa: E402


def main():
    g = orc.Geometry.from_dict(synth.geometry("c1"))
    prior, cur = synth.c1_case()
    b = synth.noisy_line_integrals(orc.forward(g, cur), 1e5, seed=101)
    print(f"prior error {np.linalg.norm(prior - cur) / np.linalg.norm(cur):.4f}")
    res = []
    for a, lam, tau in itertools.product([0.1, 0.3, 1.0, 3.0], [0.3, 1.0, 3.0, 10.0],
                                         [0.03, 0.1, 0.3]):
        r = orc.irn_piccs(g, b, prior, prior, a, lam, tau, 3, 5)
        e = float(np.linalg.norm(r.x - cur) / np.linalg.norm(cur))
        res.append((e, a, lam, tau))
        print(f"alpha={a} lambda={lam} tau={tau}: {e:.4f}", flush=True)
    res.sort()
    print("best (error, alpha, lambda, tau):", res[:3])


if __name__ == "__main__":
    main()
