"""Write c3_long.json: the FP64 oracle's electronic temperatures of sampled
atoms of the 4,000,000-atom jittered FCC system (100^3 cells, cut-off 1.2a,
capped heat capacity) after 1,000, 2,500, 5,000 and 10,000 forward-Euler
sub-steps of Eq. 2 (Section 2.1), with the system's energy and ledgers at
the same points (Eq. 6).

Inputs come from the seeded workload generator and every number written
comes from the oracle; nothing here touches the GPU library.  Runs for about
35 minutes on 8 cores:  python tests/golden/make_c3_long.py
"""
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle             # noqa: E402
import workloads as W     # noqa: E402

CHECKPOINTS = (1000, 2500, 5000, 10000)


def sample_atoms(sy, seed=7):
    """Atoms at the hotspot centre, on the 15 A and 30 A shells around it
    (where the field moves most) and spread at random over the box."""
    c = sy.box_len / 2.0
    r = np.sqrt(((sy.pos - c[:, None]) ** 2).sum(0))
    rng = np.random.default_rng(seed)
    pick = [np.argsort(r)[:64]]
    for shell in (15.0, 30.0, 45.0):
        pick.append(np.argsort(np.abs(r - shell))[:64])
    pick.append(rng.choice(sy.n, 256, replace=False))
    return np.unique(np.concatenate(pick))


def main():
    w = W.c3()
    sy = w.systems[0]
    t0 = time.time()
    row, col = oracle.neighbors(sy.pos, sy.box_lo, sy.box_len, sy.periodic, w.r_cut)
    Tl, gated = oracle.lattice_temperature(row, col, sy.vel, sy.mass, sy.params["ke_eps"])
    idx = sample_atoms(sy)
    T = np.array(sy.T_e0, dtype=np.float64)
    led = np.zeros(3)
    step = 0
    out = dict(workload="c3: FCC 100^3 cells (4,000,000 atoms), jittered 0.05 A, r_c 1.2a",
               generator="tests/golden/make_c3_long.py (FP64 oracle only)",
               atoms=idx.tolist(), checkpoints=[])
    for c in CHECKPOINTS:
        T, led, bad = oracle.run(row, col, T, Tl, sy.params, c - step, step0=step, gated=gated,
                                 ledger=led)
        step = c
        E, S = oracle.energies(T, sy.params)
        out["checkpoints"].append(dict(step=c, T=[float(v) for v in T[idx]], E_e=E, sum_T=S,
                                       E_e_to_l=float(led[0]), T_ledger=float(led[2]),
                                       T_max=float(T.max()), T_min=float(T.min()),
                                       out_of_range=int(bad)))
        print(f"step {c}: {time.time() - t0:.0f} s, T_max {T.max():.3f}", flush=True)
    with open(os.path.join(HERE, "c3_long.json"), "w") as fh:
        json.dump(out, fh, indent=0)


if __name__ == "__main__":
    main()
