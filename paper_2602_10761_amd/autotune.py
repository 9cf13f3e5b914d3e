"""Tile-shape autotuner, per mesh-size class and per workload.

For every distinct mesh (nx, ny, nz) among a set of ensembles it times, on a
one-ensemble handle of that mesh (the Poisson kernels do not depend on the
particle count): the z-transform kernels for each column width, the
tridiagonal kernel for each mode-tile size, and the inverse transforms in each
layout that fits the mesh (one, two or four blocks per y plane, or the z and x
kernels); it keeps the fastest.  The fused sort's member capacity depends on
the particles per row pair, so it is tuned on the workload's own ensemble (the
largest of its class) over a few candidate capacities.  Choices are cached in
a JSON file keyed by GPU architecture, mesh (and particle count for the sort)
and registered with the library (tf_set_tuning_class) for later handles.
"""
from __future__ import annotations

import json
import os
from typing import Dict, Iterable, Optional, Sequence, Tuple

from . import runtime as R
from . import workload as W

CACHE = os.environ.get("TRIBO_TUNE_CACHE", os.path.join(os.path.dirname(os.path.abspath(__file__)),
                                                        "tune_cache.json"))
FZ_COLS = (4, 8, 12, 16)
# bumped whenever the tiled kernels change shape semantics (older entries are ignored)
KERNEL_REV = 7
SORT_REV = 3  # the fused sort's list paths (member capacities tuned against them)
LDS_BYTES = 163840


def _arch() -> str:
    import torch
    return torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]


def _key(arch: str, mesh: Tuple[int, int, int]) -> str:
    return f"{arch}/r{KERNEL_REV}/{mesh[0]}x{mesh[1]}x{mesh[2]}"


def _sort_key(arch: str, mesh: Tuple[int, int, int], n: int) -> str:
    return f"{arch}/r{KERNEL_REV}/sort{SORT_REV}/{mesh[0]}x{mesh[1]}x{mesh[2]}/{n}"


def tri_candidates(ny: int):
    """Modes per tridiagonal tile (256 threads split among them) whose lanes cover
    ny with at most 16 rows each."""
    return [m for m in (4, 8, 16, 32) if -(-ny // (256 // m)) <= 16]


def inverse_layouts(nx: int, nz: int):
    """Layouts of the inverse transforms the library accepts for a mesh
    (tf_tuning.inv_plane): 1 one block per y plane, 2 two blocks (z-row
    parity), 4 four blocks (z-row residue mod 4), 3 z then x kernels."""
    nh = nx // 2 + 1
    out = []
    if nz * nh <= 10240 and 16 * (nx + nz + nz * nh) <= LDS_BYTES:
        out.append(1)
    if nz % 4 == 0 and (nz // 2) * nh <= 4736 and (nz // 4) * nx <= 4096:
        out.append(2)
    if nz % 8 == 0 and (nz // 4) * nh <= 4736 and (nz // 8) * nx <= 4736:
        out.append(4)
    out.append(3)
    return out


def _time_phases(ens, steps: int, sort_cap: int = 0, fz: int = 0, tm: int = 0, inv: int = 0,
                 push_order: int = 0) -> Dict[str, float]:
    R.set_tuning(sort_cap, fz, tm, inv, push_order)
    try:
        sim = R.TriboSim([ens])
    finally:
        R.set_tuning()
    sim.step(2)
    sim.profile_begin(steps)
    sim.step(steps)
    ph, n = sim.profile_end()
    sim.close()
    return {k: 1e3 * v / n for k, v in ph.items()}


def tune_mesh(mesh: Tuple[int, int, int], steps: int = 8) -> Dict[str, float]:
    """Fastest (fz_cols, tri_modes, inv_plane) for one mesh, measured on the current GPU."""
    nx, ny, nz = mesh
    ens = W.make_ensemble(W.EnsembleSpec(nx=nx, ny=ny, nz=nz, n_particles=2048, n_modes=8))
    best_fz, t_fz = 2, float("inf")
    for fz in FZ_COLS:
        try:
            t = _time_phases(ens, steps, fz=fz, inv=3)
        except R.TriboError:
            continue
        tt = t["fftz_fwd"] + t["fftz_inv"]
        if tt < t_fz:
            best_fz, t_fz = fz, tt
    best_tm, t_tm = 0, float("inf")
    for tm in tri_candidates(ny):
        try:
            t = _time_phases(ens, steps, fz=best_fz, tm=tm)
        except R.TriboError:
            continue
        if t["tridiag"] < t_tm:
            best_tm, t_tm = tm, t["tridiag"]
    best_inv, t_inv = 0, float("inf")
    for inv in inverse_layouts(nx, nz):
        try:
            t = _time_phases(ens, steps, fz=best_fz, tm=best_tm, inv=inv)
        except R.TriboError:
            continue
        tt = t["fftz_inv"] + t["ifftx"]
        if tt < t_inv:
            best_inv, t_inv = inv, tt
    return {"fz_cols": best_fz, "tri_modes": best_tm, "inv_plane": best_inv, "fftz_us": t_fz,
            "tridiag_us": t_tm, "inverse_us": t_inv}


def sort_cap_candidates(ens) -> Sequence[int]:
    """Member capacities around the mean row-pair population: multiples of 64
    from the mean to 2.5 times it, plus the largest capacity of each LDS
    occupancy level of the fused sort's blocks in that range."""
    m = ens.mesh
    pairs = m.ny * m.nz // 2
    mean = max(1, -(-ens.n // max(pairs, 1)))
    lo, hi = max(64, (mean // 64) * 64), max(128, -(-int(2.5 * mean) // 64) * 64)
    cands = set(range(lo, hi + 1, 64))
    nx = m.nx

    def lds(cap):
        lists = max(12 * cap, 16 * nx)
        lists = (lists + 15) // 16 * 16
        return 16 * nx + 4 * (lists + 24 * nx + 48)

    for blocks in range(1, 9):
        room = LDS_BYTES // blocks
        c = hi
        while c >= lo and lds(c) > room:
            c -= 8
        if c >= lo:
            cands.add(c)
    return sorted(cands)


def tune_sort_cap(ens, steps: int = 10) -> Dict[str, float]:
    """Fastest member capacity of the fused sort for this ensemble."""
    best, t_best = 0, float("inf")
    for cap in [0] + list(sort_cap_candidates(ens)):
        try:
            t = _time_phases(ens, steps, sort_cap=cap)["deposit_fftx"]
        except R.TriboError:
            continue
        if t < t_best:
            best, t_best = cap, t
    return {"sort_cap": best, "deposit_us": t_best}


def tune_push_order(ens, steps: int = 10) -> Dict[str, float]:
    """Faster block order of the push for this ensemble: consecutive slot
    ranges per XCD (1) or the hardware's round robin (2)."""
    best, t_best = 1, float("inf")
    for order in (1, 2):
        t = _time_phases(ens, steps, push_order=order)["push"]
        if t < t_best:
            best, t_best = order, t
    return {"push_order": best, "push_us": t_best}


def load_cache(path: str = CACHE) -> dict:
    if os.path.exists(path):
        with open(path) as f:
            return json.load(f)
    return {}


def _save(cache: dict, path: Optional[str]):
    if path:
        tmp = path + ".tmp"
        with open(tmp, "w") as f:
            json.dump(cache, f, indent=1, sort_keys=True)
        os.replace(tmp, path)


def ensure_tuned(meshes: Iterable[Tuple[int, int, int]], path: Optional[str] = CACHE, retune: bool = False,
                 steps: int = 8, sort_caps: Optional[Dict[Tuple[int, int, int], int]] = None,
                 push_orders: Optional[Dict[Tuple[int, int, int], int]] = None) -> dict:
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
        cap = (sort_caps or {}).get(mesh, 0)
        order = (push_orders or {}).get(mesh, 0)
        R.set_tuning_class(*mesh, fz_cols=int(ent["fz_cols"]), tri_modes=int(ent["tri_modes"]),
                           inv_plane=int(ent.get("inv_plane", 0)), sort_cap=int(cap), push_order=int(order))
        out[k] = dict(ent, sort_cap=cap, push_order=order)
    if changed:
        _save(cache, path)
    return out


def ensure_tuned_workload(ensembles, path: Optional[str] = CACHE, retune: bool = False) -> dict:
    """Tile shapes of every mesh class of a workload, the fused sort's member
    capacity and the push's block order tuned on the largest ensemble of each
    class."""
    arch = _arch()
    ensure_tuned(meshes_of(ensembles), path, retune)
    cache = load_cache(path) if path else {}
    caps, orders, changed = {}, {}, False
    for mesh in sorted(set(meshes_of(ensembles))):
        big = max((E for E in ensembles if (E.mesh.nx, E.mesh.ny, E.mesh.nz) == mesh), key=lambda E: E.n)
        k = _sort_key(arch, mesh, big.n)
        if retune or k not in cache:
            cache[k] = tune_sort_cap(big)
            changed = True
        if "push_order" not in cache[k]:
            cache[k].update(tune_push_order(big))
            changed = True
        caps[mesh] = int(cache[k]["sort_cap"])
        orders[mesh] = int(cache[k]["push_order"])
    if changed:
        _save(cache, path)
    return ensure_tuned(meshes_of(ensembles), path, False, sort_caps=caps, push_orders=orders)


def meshes_of(ensembles) -> list:
    return [(E.mesh.nx, E.mesh.ny, E.mesh.nz) for E in ensembles]
