"""Shared helpers of the test suite (comparison metrics, oracle runs)."""
import numpy as np

import oracle as O
from paper_2602_10761_amd import workload as W

KEYS = ("x", "y", "z", "vx", "vy", "vz", "q", "d")


def oracle_run(ens, n_steps, stats=True, record=None):
    g = O.Geo.from_mesh(ens.mesh)
    s = O.state_of(ens)
    st = O.Stats(g.ny) if stats else None
    for _ in range(n_steps):
        s = O.step(g, ens.U, s, ens.params, st, record=record)
    return s, st


def state_errors(a, b, mesh):
    """Normwise relative errors: positions by the domain length, velocity by
    max|v|, charge by max(max|q|, 1e-30)."""
    L = {"x": mesh.lx, "y": mesh.ly, "z": mesh.lz}
    vmax = max(np.abs(b[k]).max() for k in ("vx", "vy", "vz")) if len(b["x"]) else 1.0
    qmax = max(np.abs(b["q"]).max() if len(b["q"]) else 0.0, 1e-30)
    err = {}
    for k in ("x", "y", "z"):
        dd = np.abs(a[k] - b[k])
        if k in ("x", "z"):  # a wrap across the periodic seam is the same point
            dd = np.minimum(dd, L[k] - dd)
        err[k] = dd.max(initial=0.0) / L[k]
    for k in ("vx", "vy", "vz"):
        err[k] = np.abs(a[k] - b[k]).max(initial=0.0) / max(vmax, 1e-300)
    err["q"] = np.abs(a["q"] - b["q"]).max(initial=0.0) / qmax
    err["d"] = np.abs(a["d"] - b["d"]).max(initial=0.0)
    return err


def small(nx=32, ny=32, nz=32, n=3000, **kw):
    spec = W.CONFIGS[1].replace(nx=nx, ny=ny, nz=nz, n_particles=n, **kw)
    return W.make_ensemble(spec, 1, kw.pop("seed", 0) if "seed" in kw else 0)
