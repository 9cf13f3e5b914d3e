"""Write tests/golden/adjoint_config5.json: the charging gradient of the
adjoint workload (1e5 particles, Re_tau = 180, 64^3 mesh, 500 steps) from the
oracle alone, for the seeds the GPU test runs.

For each seed: J = (mean particle charge, wall charge per unit time) after 500
steps, dJ/d(k_c, dU, e) by the oracle's forward-mode tangent along the
recorded run, and by central differences (h = 1e-6 relative) of the oracle
replaying the recorded events (cells, impacts, wraps).  The workload is the
adjoint configuration with a wall-normal velocity jitter of 3 and charges
drawn from U[-0.02, 0.02], so that impacts occur within 500 steps (particles
that start at the local mean flow, which is parallel to the walls, do not
reach a wall in that time).

Run from the repository root:  python tests/golden/make_adjoint_config5.py
(about 20 minutes per seed on one core; the seeds run in parallel).
"""
import json
import os
import sys
from concurrent.futures import ProcessPoolExecutor

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

SEEDS = (0, 1, 2, 3, 4)
N_STEPS = 500
OVERRIDES = dict(v_jitter=3.0, precharge=0.02)
OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "adjoint_config5.json")


def one(seed):
    import numpy as np

    import oracle as O
    from oracle import tangent as T
    from paper_2602_10761_amd import workload as W

    ens = W.make_workload(5, seed=seed, **OVERRIDES)[0]
    g = O.Geo.from_mesh(ens.mesh)
    J, dJ, recs = T.gradient_tangent(g, ens.U, O.state_of(ens), ens.params, N_STEPS)
    impacts = [int(sum(int((r["wall"] == w).sum()) for r in recs)) for w in (0, 1)]
    fd = T.gradient_fd(g, ens.U, O.state_of(ens), ens.params, recs, h=1e-6)
    return seed, {"J": [float(v) for v in J], "dJ_tangent": np.asarray(dJ).tolist(),
                  "dJ_fd": np.asarray(fd).tolist(), "impacts": impacts}


def main():
    with ProcessPoolExecutor(max_workers=len(SEEDS)) as ex:
        res = dict(ex.map(one, SEEDS))
    doc = {"workload": "adjoint configuration (1e5 particles, Re_tau = 180, 64^3, dt+ = 0.1), "
                       "wall-normal velocity jitter 3, charges U[-0.02, 0.02]",
           "overrides": OVERRIDES, "steps": N_STEPS, "h": 1e-6,
           "seeds": {str(s): res[s] for s in SEEDS}}
    with open(OUT, "w") as f:
        json.dump(doc, f, indent=1)
    print("wrote", OUT)


if __name__ == "__main__":
    main()
