"""Tile-shape autotuner for the Poisson kernels, per mesh-size class.

For every distinct mesh (nx, ny, nz) among a set of ensembles, times the
z-transform kernels for each column width and the tridiagonal kernel for each
mode-tile size on a one-ensemble handle of that mesh (the Poisson kernels do
not depend on the particle count), keeps the fastest, caches the choice in a
JSON file keyed by GPU architecture and mesh, and registers it with the
library (tf_set_tuning_class) so that later handles use it.
"""
from __future__ import annotations

import json
import os
from typing import Dict, Iterable, Optional, Tuple

from . import runtime as R
from . import workload as W

CACHE = os.environ.get("TRIBO_TUNE_CACHE", os.path.join(os.path.dirname(os.path.abspath(__file__)),
                                                        "tune_cache.json"))
FZ_COLS = (4, 8, 12, 16)
# bumped whenever the tiled kernels change shape semantics (older entries are ignored)
KERNEL_REV = 6


def _arch() -> str:
    import torch
    return torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]


def _key(arch: str, mesh: Tuple[int, int, int]) -> str:
    return f"{arch}/r{KERNEL_REV}/{mesh[0]}x{mesh[1]}x{mesh[2]}"


def tri_candidates(ny: int):
    """Modes per tridiagonal tile (256 threads split among them) whose lanes cover
    ny with at most 16 rows each."""
    return [m for m in (4, 8, 16, 32) if -(-ny // (256 // m)) <= 16]


def _time_phases(mesh, fz: int, tm: int, steps: int) -> Dict[str, float]:
    nx, ny, nz = mesh
    spec = W.EnsembleSpec(nx=nx, ny=ny, nz=nz, n_particles=2048, n_modes=8)
    ens = W.make_ensemble(spec)
    R.set_tuning(0, fz, tm)
    try:
        sim = R.TriboSim([ens])
    finally:
        R.set_tuning(0, 0, 0)
    sim.step(2)
    sim.profile_begin(steps)
    sim.step(steps)
    ph, n = sim.profile_end()
    sim.close()
    return {k: 1e3 * v / n for k, v in ph.items()}


def tune_mesh(mesh: Tuple[int, int, int], steps: int = 8) -> Dict[str, int]:
    """Fastest (fz_cols, tri_modes) for one mesh, measured on the current GPU."""
    best_fz, t_fz = 2, float("inf")
    for fz in FZ_COLS:
        try:
            t = _time_phases(mesh, fz, 0, steps)
        except R.TriboError:
            continue
        tt = t["fftz_fwd"] + t["fftz_inv"]
        if tt < t_fz:
            best_fz, t_fz = fz, tt
    best_tm, t_tm = 0, float("inf")
    for tm in tri_candidates(mesh[1]):
        try:
            t = _time_phases(mesh, best_fz, tm, steps)
        except R.TriboError:
            continue
        if t["tridiag"] < t_tm:
            best_tm, t_tm = tm, t["tridiag"]
    return {"fz_cols": best_fz, "tri_modes": best_tm, "fftz_us": t_fz, "tridiag_us": t_tm}


def load_cache(path: str = CACHE) -> dict:
    if os.path.exists(path):
        with open(path) as f:
            return json.load(f)
    return {}


def ensure_tuned(meshes: Iterable[Tuple[int, int, int]], path: Optional[str] = CACHE, retune: bool = False,
                 steps: int = 8) -> dict:
    """Tune the meshes missing from the cache, register all of them, return the entries."""
    arch = _arch()
    cache = load_cache(path) if path else {}
    out = {}
    changed = False
    for mesh in sorted(set(tuple(m) for m in meshes)):
        k = _key(arch, mesh)
        if retune or k not in cache:
            cache[k] = tune_mesh(mesh, steps)
            changed = True
        ent = cache[k]
        R.set_tuning_class(*mesh, fz_cols=int(ent["fz_cols"]), tri_modes=int(ent["tri_modes"]))
        out[k] = ent
    if changed and path:
        tmp = path + ".tmp"
        with open(tmp, "w") as f:
            json.dump(cache, f, indent=1, sort_keys=True)
        os.replace(tmp, path)
    return out


def meshes_of(ensembles) -> list:
    return [(E.mesh.nx, E.mesh.ny, E.mesh.nz) for E in ensembles]
