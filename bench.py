"""Throughput of the particle step on one MI355X.

python bench.py [--steps K] [--warmup W] [--config C] [--no-cpu]

One step = the whole per-step particle phase (sort, deposit, Poisson solve,
push with wall charging) over one ensemble with inputs resident in HBM.
Prints one JSON line.  The metric is particle-steps per second with the
Poisson solve every step.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "particle-steps/s (fwd+Poisson) & adjoint/fwd time, batched vs plain, % HBM"
HBM_PEAK_GBS = 8000.0

WORKLOAD_NAME = {
    1: "Re_tau=180 channel 32^3 (tanh y, 2.0), 1e4 particles d+=0.5, rho_p/rho=1000, dt+=0.1",
    2: "Re_tau=180 channel 128^3 (tanh y, 2.0), 1e6 particles d+ in {0.25,0.5,1}, rho_p/rho=1000, dt+=0.1",
    3: "Re_tau=550 channel 192x160x192 (tanh y, 2.0), 4e6 particles d+ in {0.5,1,2}, dt+=0.05",
}


def algorithmic_bytes(phase, n_p, nx, ny, nz):
    """Bytes the method must move per launch of each kernel group (FP64)."""
    n_c = nx * ny * nz
    n_nodes = nx * (ny + 1) * nz
    nh = nx // 2 + 1
    spec = 16 * ny * nz * nh
    return {
        # state read (x, y, z, v, q, d) + write (x, y, z, v, q); carrier nodes; phi stencil
        "push": 120 * n_p + min(24 * n_nodes, 192 * n_p) + min(8 * n_c, 56 * n_p),
        # charges in, spectrum out
        "deposit_fftx": 8 * n_p + spec,
        "fftz_fwd": 2 * spec,
        "tridiag": 2 * spec,
        "fftz_inv": 2 * spec,
        # spectrum in, phi out
        "ifftx": spec + 8 * n_c,
        # keys in, permutation out
        "sort": 8 * n_p,
    }[phase]


def cpu_baseline(ens, n_steps):
    import numpy as np  # noqa: F401
    import oracle as O

    g = O.Geo.from_mesh(ens.mesh)
    s = O.state_of(ens)
    st = O.Stats(g.ny)
    t0 = time.perf_counter()
    for _ in range(n_steps):
        s = O.step(g, ens.U, s, ens.params, st)
    dt = time.perf_counter() - t0
    return ens.n * n_steps / dt, dt


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--config", type=int, default=2, choices=(1, 2, 3))
    ap.add_argument("--cpu-steps", type=int, default=4)
    ap.add_argument("--no-cpu", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              "(independent ensembles shard across GPUs without communication).", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_2602_10761_amd import workload as W
    from paper_2602_10761_amd.runtime import TriboSim

    ens = W.make_workload(args.config)[0]
    m = ens.mesh
    print(f"# workload config {args.config}: {ens.n} particles, mesh {m.nx}x{m.ny}x{m.nz}", file=sys.stderr,
          flush=True)
    sim = TriboSim([ens], device="cuda:0")
    sim.step(args.warmup)
    sim.synchronize()
    torch.cuda.synchronize()

    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    sim.profile_begin(args.steps)
    ev0.record(sim.stream)
    sim.step(args.steps)
    ev1.record(sim.stream)
    sim.synchronize()
    torch.cuda.synchronize()
    total_ms = ev0.elapsed_time(ev1)
    phase_ms, nprof = sim.profile_end()
    st = sim.stats(0)
    sim.close()

    ms_step = total_ms / args.steps
    value = ens.n * args.steps / (total_ms * 1e-3)
    per_launch = {k: v / nprof for k, v in phase_ms.items()}
    dom = max(per_launch, key=per_launch.get)
    ab = algorithmic_bytes(dom, ens.n, m.nx, m.ny, m.nz)
    achieved = ab / (per_launch[dom] * 1e-3) / 1e9
    step_bytes = sum(algorithmic_bytes(k, ens.n, m.nx, m.ny, m.nz) for k in per_launch)
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "particle-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": WORKLOAD_NAME[args.config], "n_particles": ens.n,
                   "mesh": [m.nx, m.ny, m.nz], "poisson_every": 1},
        "roofline": {"bound": "hbm", "kernel": dom, "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": None},
        "phase_us": {k: 1e3 * v for k, v in per_launch.items()},
        "step_algorithmic_GBs": step_bytes / (ms_step * 1e-3) / 1e9,
        "impacts": [int(v) for v in st["impacts"]],
        "flags": int(st["flags"]),
    }
    if not args.no_cpu:
        v, secs = cpu_baseline(ens, args.cpu_steps)
        out["cpu_baseline"] = {"value": v, "unit": "particle-steps/s", "cores": 1, "kind": "oracle",
                               "sample": f"first {args.cpu_steps} steps of the same workload "
                                         f"({secs:.1f} s, numpy single thread)"}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
