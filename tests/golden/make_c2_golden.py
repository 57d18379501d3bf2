"""Write the oracle's expected values for the 512 x 256, 64-shot, 3000-step workload.

Calls only the FP64 oracle and the seeded input generators.  Output
(tests/golden/c2_golden.npz):
  H_y0     apply_H of the first trial function, float64 [256][512]
  F_shots  shot indices whose traces are stored
  F_y0     apply_F of the first trial at those shots, every 2nd time step, float32
Run:  python tests/golden/make_c2_golden.py [workers]   (about 10 min on 8 cores)
"""
import os
import sys
from multiprocessing import Pool

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import fixtures as F  # noqa: E402
from oracle import Problem  # noqa: E402

F_SHOTS = (5, 40)


def _shot(s):
    w = F.c2()
    c = F.medium(w)
    y = F.trials(w, c)[0]
    P = Problem(w, c)
    g, _ = P.background(s)
    d = P.born(s, y, g)
    img = P.adjoint(s, d, g)
    return s, img, (d[::2].astype(np.float32) if s in F_SHOTS else None)


def main():
    workers = int(sys.argv[1]) if len(sys.argv) > 1 else 6
    os.environ["OMP_NUM_THREADS"] = "1"
    w = F.c2()
    with Pool(workers) as pool:
        parts = dict((s, (img, d)) for s, img, d in pool.imap_unordered(_shot, range(w.ns)))
    H = None
    for s in range(w.ns):                      # shots stacked in increasing order
        H = parts[s][0] if H is None else H + parts[s][0]
    out = os.path.join(os.path.dirname(os.path.abspath(__file__)), "c2_golden.npz")
    np.savez(out, H_y0=H, F_shots=np.array(F_SHOTS), F_y0=np.stack([parts[s][1] for s in F_SHOTS]))
    print("wrote", out, float(np.linalg.norm(H)))


if __name__ == "__main__":
    main()
