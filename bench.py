"""Throughput of the particle step on one MI355X.

python bench.py [--steps K] [--warmup W] [--config C] [--no-cpu] [--no-batched] [--no-adjoint]

One step = the whole per-step particle phase (sort, deposit, Poisson solve,
push with wall charging) with inputs resident in HBM.  Prints one JSON line:
the headline is particle-steps/s on the 4e6-particle 192x160x192 Re_tau = 550
channel with the Poisson solve every step (the largest single-GPU workload);
it also carries the 1e6-particle 128^3 workload, the batched-vs-plain time on
64 independent ensembles, the adjoint/forward time ratio, the roofline of the
dominant kernel (its launch duration from HIP events around every 10th launch
in the timed region, --event-every, against the method's own bytes; the
measured HBM bytes come from the committed rocprofv3 summary of the workload)
and the CPU oracle baseline.
"""
import argparse
import hashlib
import re
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
KERNEL_SOURCES = ["paper_2602_10761_amd/csrc/kernels.hip", "paper_2602_10761_amd/csrc/particle.h",
                  "paper_2602_10761_amd/csrc/tribo_dev.h"]


def plane_fused(nx, nz):
    """Whether the library runs both inverse transforms of a y plane without a
    pass through memory in between (the plane's half spectrum and twiddles within
    160 KiB, at most 10240 points: one block per plane, or two by z-row parity;
    else four blocks by z-row residue mod 4, each with a quarter plane of at
    most 4736 points)."""
    nh = nx // 2 + 1
    pts = nz * nh
    whole = pts <= 10240 and 16 * (nx + nz + pts) <= 163840
    quarter = nz % 8 == 0 and (nz // 4) * nh <= 4736 and (nz // 8) * nx <= 4736
    return whole or quarter


def algorithmic_step_bytes(n_p, nx, ny, nz):
    """Bytes the method itself must move per step (FP64): particle state read
    (x, v, q, d: 64 B) and written (x, v, q: 56 B); the carrier at most once per
    cell or 8 nodes per particle; the charge deposit write; the Poisson solve's
    density read and potential write; the potential stencil read for E.  Sort
    keys, particle ids and FFT intermediates are design overhead, not counted."""
    n_c = nx * ny * nz
    return (120 * n_p + min(24 * n_c, 192 * n_p) + min(8 * n_c, 8 * n_p) + 8 * n_c + 8 * n_c +
            min(8 * n_c, 56 * n_p))


def algorithmic_push_bytes(n_p, nx, ny, nz):
    """The push's share of the step's algorithmic bytes: particle state in and
    out, carrier gathers, potential stencil."""
    n_c = nx * ny * nz
    return 120 * n_p + min(24 * n_c, 192 * n_p) + min(8 * n_c, 56 * n_p)


def design_bytes(phase, n_p, nx, ny, nz):
    """Bytes each kernel group of this design moves per launch at the least
    (FP64 state, int32 keys): the algorithmic bytes plus the design's own
    traffic (sort bookkeeping, ids, spectra, Thomas factors)."""
    n_c = nx * ny * nz
    n_nodes = nx * (ny + 1) * nz
    nh = nx // 2 + 1
    spec = 16 * ny * nz * nh
    return {
        # particle state in (position, charge, velocity, diameter: 64 B) and out
        # (64 B); slot bookkeeping in (perm, cell, id: 12 B) and out (id, cell:
        # 8 B); carrier velocity at the nodes, phi stencil and cell starts,
        # each at most once per cell or per particle
        "push": 148 * n_p + min(24 * n_nodes, 192 * n_p) + min(8 * n_c, 56 * n_p) + min(4 * n_c, 8 * n_p),
        # incremental sort + deposit + x transform: keys and ids of the
        # members (8 B), their charge gathered (8 B), perm and cell written in
        # slot order (8 B); cell starts; the half spectrum
        "deposit_fftx": 24 * n_p + 4 * n_c + spec,
        "fftz_fwd": 2 * spec,
        # spectrum in and out, Thomas factors (16 B per mode and row, modes
        # mz <= nz / 2: mz and nz - mz share them)
        "tridiag": 2 * spec + 16 * ny * (nz // 2 + 1) * nh,
        # inverse transforms: fused per y plane (spectrum in, phi out) when the
        # plane fits one block's LDS, else z (spectrum in and out) then x
        "fftz_inv": spec + 8 * n_c if plane_fused(nx, nz) else 2 * spec,
        "ifftx": 0 if plane_fused(nx, nz) else spec + 8 * n_c,
        # row-pair counts in, row-pair starts out
        "sort": 4 * ny * nz,
    }[phase]


def traffic_file(config):
    return os.path.join(ROOT, "profiles", f"hbm_traffic_config{config}.txt")


def source_hash():
    """Hash of the kernel sources' code (comments and blank lines left out, so
    that a comment edit keeps a measurement valid)."""
    h = hashlib.sha256()
    for p in KERNEL_SOURCES:
        with open(os.path.join(ROOT, p), encoding="utf-8") as f:
            text = f.read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        text = re.sub(r"//[^\n]*", "", text)
        code = "\n".join(line.rstrip() for line in text.splitlines() if line.strip())
        h.update(code.encode())
    return h.hexdigest()[:16]


def measured_traffic(kernel, config):
    """HBM bytes per launch of `kernel` from the committed PMC summary of this
    workload, if it was taken on the current kernel sources (else None)."""
    path = traffic_file(config)
    if not os.path.exists(path):
        return None
    kv = {}
    for line in open(path):
        if ":" in line and not line.startswith("#"):
            k, v = line.split(":", 1)
            kv[k.strip()] = v.split("#", 1)[0].strip()
    if kv.get("source_hash") != source_hash():
        return None
    v = kv.get(f"{kernel}_bytes")
    return float(v) if v else None


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform
    return platform.processor() or "unknown"


def cpu_baseline(ens, n_steps):
    """The oracle as it stands (numpy, FP64; its FFT and scatter-adds run on one
    thread) over the first n_steps steps of the workload."""
    import oracle as O

    g = O.Geo.from_mesh(ens.mesh)
    s = O.state_of(ens)
    st = O.Stats(g.ny)
    t0 = time.perf_counter()
    for _ in range(n_steps):
        s = O.step(g, ens.U, s, ens.params, st)
    dt = time.perf_counter() - t0
    return ens.n * n_steps / dt, dt


def timed_steps(torch, sim, k):
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    sim.synchronize()
    ev0.record(sim.stream)
    sim.step(k)
    ev1.record(sim.stream)
    sim.synchronize()
    return ev0.elapsed_time(ev1)


def batched_vs_plain(torch, W, R, autotune, steps, log):
    ens = W.make_workload(4)
    n_tot = sum(E.n for E in ens)
    autotune.ensure_tuned_workload(ens)
    log(f"batched: {len(ens)} ensembles, {n_tot} particles")
    sim = R.TriboSim(ens, graphs=True)
    sim.step(3)
    ms_b = timed_steps(torch, sim, steps) / steps
    sim.close()
    del sim
    ms_p = 0.0
    for E in ens:
        s1 = R.TriboSim([E], graphs=True)
        s1.step(3)
        ms_p += timed_steps(torch, s1, steps) / steps
        s1.close()
    return {"workload": "64 ensembles: N_p log-uniform in [1e4, 1e6], Re_tau in {180, 300, 395, 550} "
                        "with meshes 64^3..160^3, d+ uniform in [0.25, 2]",
            "n_particles": n_tot, "ms_per_step_batched": ms_b, "ms_per_step_plain_sum": ms_p,
            "speedup_batched_vs_plain": ms_p / ms_b,
            "particle_steps_per_s_batched": n_tot / (ms_b * 1e-3)}


def source_cost(torch, W, R, steps, log):
    """Extra time of the 2-way coupling source (per-particle drag force written
    by the push, per-cell sums) on the headline workload, graph replays on and
    off the source."""
    ens = W.make_workload(2)[0]
    m = ens.mesh
    ms = {}
    for on in (False, True):
        sim = R.TriboSim([ens], graphs=True, source=on)
        sim.step(3)
        ms[on] = timed_steps(torch, sim, steps) / steps
        sim.close()
        del sim
    n_c = m.nx * m.ny * m.nz
    extra_bytes = 24 * ens.n + (4 * n_c + 24 * ens.n + 24 * n_c)  # push write; cell sums (starts, forces, source)
    d_us = (ms[True] - ms[False]) * 1e3
    log(f"2-way source: {ms[False] * 1e3:.1f} -> {ms[True] * 1e3:.1f} us/step")
    return {"workload": WORKLOAD_NAME[2], "us_per_step_without": ms[False] * 1e3, "us_per_step_with": ms[True] * 1e3,
            "extra_us_per_step": d_us, "extra_algorithmic_bytes": extra_bytes,
            "extra_GBs": extra_bytes / (d_us * 1e-6) / 1e9 if d_us > 0 else None}


def four_way_cost(torch, W, R, steps, log):
    """Time of the headline step with 4-way coupling (same-cell particle-particle
    collisions, k_pp = 1) against the plain step, graph replays, and the pairs
    that collided; and with the stochastic scaling model of wall charging."""
    ms, pairs = {}, 0
    ssm = (-2e-3, -1.5e-3, 4e-4, 0.6, 20.0, 0.5, 1.0)
    for on in (False, True, "ssm"):
        kw = dict(charging=1, ssm=ssm, seed=1) if on == "ssm" else dict(pp=int(on), k_pp=1.0)
        ens = W.make_workload(2, **kw)[0]
        sim = R.TriboSim([ens], graphs=True)
        sim.step(3)
        ms[on] = timed_steps(torch, sim, steps) / steps
        if on is True:
            pairs = int(sim.stats(0)["pp_pairs"])
        sim.close()
        del sim
    log(f"4-way coupling: {ms[False] * 1e3:.1f} -> {ms[True] * 1e3:.1f} us/step, {pairs} pairs; "
        f"SSM wall charging {ms['ssm'] * 1e3:.1f} us/step")
    return {"workload": WORKLOAD_NAME[2] + ", k_pp=1", "us_per_step_without": ms[False] * 1e3,
            "us_per_step_with": ms[True] * 1e3, "colliding_pairs": pairs, "steps": steps + 3,
            "us_per_step_ssm_wall_charging": ms["ssm"] * 1e3}


def carrier_stream_cost(torch, W, R, steps, log):
    """Step time of the headline workload when the carrier field changes every
    step (two fields alternating through tf_set_carrier, graph replays)."""
    import numpy as np
    ens = W.make_workload(2)[0]
    sim = R.TriboSim([ens], graphs=True)
    U2 = torch.as_tensor(np.ascontiguousarray(ens.U * 0.9), dtype=torch.float64).to(sim.dev)
    fields = [sim.U[0], U2]
    sim.step(3)
    sim.synchronize()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    ev0.record(sim.stream)
    for n in range(steps):
        sim.set_carrier(0, fields[n % 2])
        sim.step(1)
    ev1.record(sim.stream)
    sim.synchronize()
    ms = ev0.elapsed_time(ev1) / steps
    sim.close()
    log(f"carrier changed every step: {ms * 1e3:.1f} us/step")
    return {"workload": WORKLOAD_NAME[2] + ", two carrier fields alternating", "us_per_step": ms * 1e3}


def adjoint_ratio(torch, W, R, autotune, seg, log):
    ens = W.make_workload(5, v_jitter=3.0, precharge=0.02)[0]
    autotune.ensure_tuned(autotune.meshes_of([ens]))
    sim = R.TriboSim([ens], traj_steps=seg)
    sim.step(3)
    ms_fwd = timed_steps(torch, sim, seg)
    init = sim.state(0)
    sim.set_state(0, init)
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    lam = [{k: torch.zeros(ens.n, dtype=torch.float64, device=sim.dev) for k in R.KEYS}]
    lam[0]["q"].fill_(1.0 / ens.n)
    import numpy as np
    sim.synchronize()
    t0 = time.perf_counter()
    ev0.record(sim.stream)
    dth = torch.zeros((1, 3), dtype=torch.float64, device=sim.dev)
    sim.step(seg, record=True)
    sim.adjoint(lam, np.zeros((1, 2)), dtheta=dth)   # asynchronous on the library's stream
    ev1.record(sim.stream)
    sim.synchronize()
    ms_bwd = ev0.elapsed_time(ev1)
    wall_bwd = (time.perf_counter() - t0) * 1e3
    sim.close()
    log(f"adjoint: fwd {ms_fwd:.2f} ms, record+reverse {ms_bwd:.2f} ms per {seg} steps")
    return {"workload": "Re_tau=180 channel 64^3, 1e5 particles d+=0.5, segments of %d steps" % seg,
            "ms_forward_segment": ms_fwd, "ms_record_plus_adjoint_segment": ms_bwd,
            "adjoint_over_forward": ms_bwd / ms_fwd, "wall_ms_record_plus_adjoint": wall_bwd}


def plain_run(torch, W, R, autotune, config, args, log, **overrides):
    """One ensemble of a plain workload: warm-up, an untimed phase pass (an
    event at every phase boundary), then the timed region with HIP events only
    around the dominant kernel on every args.event_every-th step (on the
    library's stream).  Returns the measurement and the workload."""
    ens = W.make_workload(config, **overrides)[0]
    m = ens.mesh
    log(f"workload config {config}: {ens.n} particles, mesh {m.nx}x{m.ny}x{m.nz}")
    tuned = autotune.ensure_tuned_workload([ens])
    log(f"tiles: {tuned}")
    sim = R.TriboSim([ens], device="cuda:0", graphs=args.graphs)
    sim.step(args.warmup)
    sim.profile_begin(args.phase_steps)
    sim.step(args.phase_steps)
    phase_ms, nprof = sim.profile_end()
    per_phase = {k: v / nprof for k, v in phase_ms.items()}
    dom = max(per_phase, key=per_phase.get)
    sim.synchronize()
    torch.cuda.synchronize()

    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    if not args.graphs:
        sim.profile_begin((args.steps + args.event_every - 1) // args.event_every, phases=[dom],
                          every=args.event_every)
    ev0.record(sim.stream)
    sim.step(args.steps)
    ev1.record(sim.stream)
    sim.synchronize()
    torch.cuda.synchronize()
    total_ms = ev0.elapsed_time(ev1)
    dom_ms = None
    if not args.graphs:
        ph_t, n_t = sim.profile_end()
        dom_ms = ph_t[dom] / n_t
    st = sim.stats(0)
    sim.close()
    del sim
    ms_step = total_ms / args.steps
    log(f"config {config}: timed {args.steps} steps: {ms_step * 1e3:.1f} us/step")

    dms = dom_ms if dom_ms is not None else per_phase[dom]
    if dom == "push":
        ab = algorithmic_push_bytes(ens.n, m.nx, m.ny, m.nz)
    else:   # no kernel but the push carries a share of the method's own bytes
        ab = design_bytes(dom, ens.n, m.nx, m.ny, m.nz)
    achieved = ab / (dms * 1e-3) / 1e9
    tr = measured_traffic(dom, config)
    B = algorithmic_step_bytes(ens.n, m.nx, m.ny, m.nz)
    # the step's HBM bytes as counted (FETCH_SIZE + WRITE_SIZE of every kernel
    # with design traffic, from the committed summary of this workload)
    kern = [k for k in per_phase if design_bytes(k, ens.n, m.nx, m.ny, m.nz) > 0]
    mt = {k: measured_traffic(k, config) for k in kern}
    mb = None if overrides or any(v is None for v in mt.values()) else sum(mt.values())
    res = {
        "value": ens.n * args.steps / (total_ms * 1e-3),
        "ms_per_step": ms_step,
        "config": {"workload": WORKLOAD_NAME[config] + (f", {overrides}" if overrides else ""),
                   "n_particles": ens.n, "mesh": [m.nx, m.ny, m.nz],
                   "poisson_every": 1},
        "roofline": {"bound": "hbm", "kernel": dom, "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS,
                     "traffic": None if tr is None else tr / (dms * 1e-3) / 1e9,
                     "algorithmic_bytes_per_launch": ab,
                     "design_bytes_per_launch": design_bytes(dom, ens.n, m.nx, m.ny, m.nz),
                     "measured_bytes_per_launch": tr, "avg_launch_us": 1e3 * dms,
                     "launch_timing": (f"timed region, every {args.event_every}th launch"
                                       if dom_ms is not None else "phase pass")},
        "step": {"algorithmic_bytes": B, "algorithmic_GBs": B / (ms_step * 1e-3) / 1e9,
                 "algorithmic_frac": B / (ms_step * 1e-3) / 1e9 / HBM_PEAK_GBS,
                 "design_bytes": sum(design_bytes(k, ens.n, m.nx, m.ny, m.nz) for k in per_phase),
                 "measured_bytes": mb,
                 "measured_GBs": None if mb is None else mb / (ms_step * 1e-3) / 1e9,
                 "measured_frac": None if mb is None else mb / (ms_step * 1e-3) / 1e9 / HBM_PEAK_GBS},
        "phase_us": {k: 1e3 * v for k, v in per_phase.items()},
        "impacts": [int(v) for v in st["impacts"]],
        "flags": int(st["flags"]),
    }
    return res, ens


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--config", type=int, default=3, choices=(1, 2, 3),
                    help="headline workload (3: the largest single-GPU one)")
    ap.add_argument("--cpu-steps", type=int, default=0,
                    help="oracle steps of the CPU baseline (0: 5 for the 4e6-particle workload, else 8)")
    ap.add_argument("--phase-steps", type=int, default=10, help="untimed steps of the per-phase breakdown")
    ap.add_argument("--batched-steps", type=int, default=20)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--no-adjoint", action="store_true")
    ap.add_argument("--no-source", action="store_true", help="skip the 2-way coupling source timing")
    ap.add_argument("--no-fourway", action="store_true", help="skip the 4-way coupling timing")
    ap.add_argument("--no-second", action="store_true",
                    help="skip the 1e6-particle 128^3 workload measured beside the headline")
    ap.add_argument("--no-charged", action="store_true",
                    help="skip the headline workload with wall impacts and charged particles")
    ap.add_argument("--graphs", action="store_true", help="time graph replays instead of eager phase-timed steps")
    ap.add_argument("--event-every", type=int, default=10,
                    help="timed region: HIP events around the dominant kernel on every n-th step")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="first copy 256 MiB device-to-device (reference kernel for HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              "(independent ensembles shard across GPUs without communication).", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_2602_10761_amd import autotune
    from paper_2602_10761_amd import runtime as R
    from paper_2602_10761_amd import workload as W

    def log(msg):
        print("# " + msg, file=sys.stderr, flush=True)

    if args.calibrate_copy:
        a = torch.ones(32 * 1024 * 1024, dtype=torch.float64, device="cuda:0")
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b
    head, ens = plain_run(torch, W, R, autotune, args.config, args, log)
    out = {
        "metric": METRIC,
        "value": head["value"],
        "unit": "particle-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": head["config"],
        "roofline": head["roofline"],
        "step": head["step"],
        "phase_us": head["phase_us"],
        "impacts": head["impacts"],
        "flags": head["flags"],
    }
    if not args.no_second and args.config != 2:
        second, _ = plain_run(torch, W, R, autotune, 2, args, log)
        out["config2"] = second
    if not args.no_charged:
        # the headline workload starts uncharged and reaches no wall within the
        # timed steps; the same with wall impacts and charging at work
        ch, _ = plain_run(torch, W, R, autotune, args.config, args, log, v_jitter=3.0, precharge=0.05)
        out["charged"] = {k: ch[k] for k in ("value", "ms_per_step", "config", "phase_us", "impacts", "flags")}
    if not args.no_batched:
        out["batched"] = batched_vs_plain(torch, W, R, autotune, args.batched_steps, log)
    if not args.no_adjoint:
        out["adjoint"] = adjoint_ratio(torch, W, R, autotune, 50, log)
    if not args.no_source:
        out["two_way_source"] = source_cost(torch, W, R, 50, log)
    if not args.no_fourway:
        out["four_way"] = four_way_cost(torch, W, R, 50, log)
        out["carrier_every_step"] = carrier_stream_cost(torch, W, R, 50, log)
    if not args.no_cpu:
        n_cpu = args.cpu_steps or (5 if ens.n >= 2_000_000 else 8)
        v, secs = cpu_baseline(ens, n_cpu)
        out["cpu_baseline"] = {"value": v, "unit": "particle-steps/s", "cores": 1, "kind": "oracle",
                               "sample": f"first {n_cpu} steps of the same workload ({secs:.1f} s)",
                               "cpu_model": cpu_model(), "host_threads": len(os.sched_getaffinity(0))}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
