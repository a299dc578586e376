"""Writes c1_best_distribution.json: the FP64 oracle's best-pose energies and
RMSDs (to the input pose) for the 600-atom-pocket / 24-atom-ligand docking
workload, 64 trajectories x 100 MC steps x 10 Adam steps, seeds 0..3.

Calls only oracle/ and the seeded input generator.  The paper's sampler
(Methods, "Conformation sampling"; Fig. 2) with the readings in oracle/.

    python tests/golden/make_c1_best_distribution.py
"""
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import synth  # noqa: E402
from oracle import topology, score as SC, sampler as SM, fk as FK, best as BEST, params as P  # noqa: E402

SEEDS = (0, 1, 2, 3)


def main():
    pk, L, wl = synth.workload("C1")
    topo = topology.from_ligands(L, 0)
    w = np.asarray(P.TRIDS_WEIGHTS, np.float32).astype(np.float64)
    sc = SC.Scorer(pk[0], weights=w)
    out = dict(workload="C1", n_traj=wl["T"], n_steps=wl["S"], n_local=10, seeds=list(SEEDS),
               E_best=[], rmsd=[])
    t0 = time.time()
    for s in SEEDS:
        prm = SM.SamplerParams(n_traj=wl["T"], n_steps=wl["S"], n_local=10, seed=s)
        st = SM.sample(sc, topo, 0, prm)
        x = FK.fk(topo, st.q_best)
        out["E_best"].append([float(v) for v in st.E_best])
        out["rmsd"].append([float(v) for v in BEST.rmsd(x, topo.x0[None])])
        print("seed", s, "median E_best", np.median(st.E_best), "%.1fs" % (time.time() - t0), flush=True)
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "c1_best_distribution.json")
    with open(path, "w") as f:
        json.dump(out, f)
    print("wrote", path)


if __name__ == "__main__":
    main()
