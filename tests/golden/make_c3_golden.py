"""Write the oracle's expected values for eight shots of the 1024 x 512, 4000-step workload.

Calls only the FP64 oracle and the seeded input generators.  The shots are
every 16th of the workload's 128 (sources at x = 4, 132, ..., 900); the trial
is the workload's own (512 wavepackets, seed 7) and the data for F* are seeded
band-limited traces (seed 19, Ricker spectrum of the workload's 12 Hz).
Output (tests/golden/c3_golden.npz), stored as float32 (rounding 6e-8
relative, far below every bound the tests apply):
  shots    the shot indices used
  H_y      sum over those shots of F_s* F_s y, [512][1024]
  Fadj_d   sum over those shots of F_s* d_s, [512][1024]
  F_rec    receiver indices whose traces are stored (every 16th)
  F_y      F_s y at those receivers, every time step, [8][4000][32]
Run:  python tests/golden/make_c3_golden.py [workers]   (about 8 min per shot on
one core; each worker holds one shot's 16.8 GB g history, so two workers fit in
64 GB)
"""
import os
import sys
from multiprocessing import Pool

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import fixtures as F  # noqa: E402
from oracle import Problem  # noqa: E402

SHOTS = tuple(range(0, 128, 16))
REC = tuple(range(0, 512, 16))
DATA_SEED = 19


def workload():
    w = F.c3()
    return w.with_(src=w.src[list(SHOTS)])


def data(w):
    return F.bandlimited_data((w.ns, w.nt, w.nr), DATA_SEED, w.dt, w.f_peak)


def _shot(j):
    w = workload()
    c = F.medium(w)
    y = F.trials(w, c)[0]
    d = data(w)[j]
    P = Problem(w, c)
    g, _ = P.background(j)
    dy = P.born(j, y, g)
    both = P.adjoint(j, np.stack([dy, d.astype(np.float64)]), g)
    print(f"shot {SHOTS[j]} done", flush=True)
    return j, both[0], both[1], dy[:, list(REC)].astype(np.float32)


def main():
    workers = int(sys.argv[1]) if len(sys.argv) > 1 else 2
    os.environ["OMP_NUM_THREADS"] = "1"
    with Pool(workers) as pool:
        parts = dict((j, rest) for j, *rest in pool.imap_unordered(_shot, range(len(SHOTS))))
    H = Fa = None
    for j in range(len(SHOTS)):                 # shots stacked in increasing order
        H = parts[j][0] if H is None else H + parts[j][0]
        Fa = parts[j][1] if Fa is None else Fa + parts[j][1]
    out = os.path.join(os.path.dirname(os.path.abspath(__file__)), "c3_golden.npz")
    np.savez(out, shots=np.array(SHOTS), H_y=H.astype(np.float32), Fadj_d=Fa.astype(np.float32),
             F_rec=np.array(REC), F_y=np.stack([parts[j][2] for j in range(len(SHOTS))]))
    print("wrote", out, float(np.linalg.norm(H)), float(np.linalg.norm(Fa)))


if __name__ == "__main__":
    main()
