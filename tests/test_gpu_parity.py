"""GPU parity of the HIP particle step against the CPU oracle (through the C ABI).

Bars: deposit, impact counts and all integer statistics bit-exact; particle
state within 1e-12 normwise relative, after one step from the same input
state and after several (rounding differences grow through the charge
updates of wall impacts, collisions and the Coulomb sums; every case here
measured below 1e-13, e.g. 7e-14 after 40 steps with 110 impacts); potential
within 1e-12 relative to its maximum.
"""
import sys

import numpy as np
import pytest

import oracle as O
from helpers import KEYS, oracle_run, state_errors
from paper_2602_10761_amd import workload as W
from paper_2602_10761_amd.autotune import inverse_layouts

pytestmark = pytest.mark.gpu

TOL = 1e-12


def sim_of(ens_list, **kw):
    from paper_2602_10761_amd.runtime import TriboSim
    return TriboSim(ens_list if isinstance(ens_list, list) else [ens_list], **kw)


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def ens_small(nx=32, ny=32, nz=32, n=4000, seed=0, **kw):
    spec = W.CONFIGS[1].replace(nx=nx, ny=ny, nz=nz, n_particles=n, **kw)
    return W.make_ensemble(spec, 1, seed)


def assert_stats_equal(gs, os_):
    assert gs["steps"] == os_.steps
    assert gs["flags"] == os_.flags
    np.testing.assert_array_equal(gs["impacts"], os_.impacts)
    np.testing.assert_array_equal(gs["wallq"], os_.wallq)
    np.testing.assert_array_equal(gs["unhist"], os_.unhist)
    np.testing.assert_array_equal(gs["crel_y"], os_.crel_y)
    np.testing.assert_array_equal(gs["qcum_y"], os_.qcum_y)
    np.testing.assert_array_equal(gs["qnow_y"], os_.qnow_y)


# ---------------------------------------------------------------------------
# Poisson stage in isolation
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("shape,stretch", [((8, 6, 12), 1.5), ((24, 20, 40), 2.0), ((32, 32, 32), 2.0),
                                           ((64, 64, 64), 2.0), ((96, 64, 96), 2.0), ((128, 128, 128), 2.0),
                                           ((160, 160, 160), 2.0), ((192, 160, 192), 2.0), ((256, 8, 256), 1.0),
                                           ((4, 2, 4), 0.0)])
def test_poisson_parity(shape, stretch):
    nx, ny, nz = shape
    say("poisson", shape)
    ens = W.make_ensemble(W.CONFIGS[1].replace(nx=nx, ny=ny, nz=nz, n_particles=10, stretch=stretch, n_modes=4))
    g = O.Geo.from_mesh(ens.mesh)
    rng = np.random.default_rng(nx * 7 + ny)
    Q = np.zeros(g.ncell, dtype=np.int64)
    idx = rng.integers(0, g.ncell, max(4, g.ncell // 50))
    Q[idx] = rng.integers(-(1 << 50), 1 << 50, idx.size)
    sim = sim_of(ens)
    phi = sim.poisson(0, Q).cpu().numpy().reshape(ny, nz, nx)
    ref = O.poisson(g, Q)
    err = np.abs(phi - ref).max() / np.abs(ref).max()
    say("  rel err", err)
    assert err < TOL
    sim.close()


@pytest.mark.parametrize("shape", [(8, 6, 12), (24, 20, 40), (32, 32, 32), (128, 128, 128), (4, 2, 4),
                                   (192, 160, 192), (160, 24, 200), (64, 10, 48)])
def test_poisson_inverse_layouts(shape):
    """Every layout of the inverse transforms that fits the mesh (one block per
    y plane, two or four blocks per plane by z-row residue, z then x kernels)
    against the oracle."""
    from paper_2602_10761_amd import runtime as R
    nx, ny, nz = shape
    ens = W.make_ensemble(W.CONFIGS[1].replace(nx=nx, ny=ny, nz=nz, n_particles=10, stretch=2.0, n_modes=4))
    g = O.Geo.from_mesh(ens.mesh)
    rng = np.random.default_rng(nz * 3 + ny)
    Q = rng.integers(-(1 << 50), 1 << 50, g.ncell).astype(np.int64)
    ref = O.poisson(g, Q)
    phis = {}
    try:
        for mode in inverse_layouts(nx, nz):  # every layout the library accepts for the mesh
            say("poisson layout", shape, mode)
            R.set_tuning(inv_plane=mode)
            sim = sim_of(ens)
            phis[mode] = sim.poisson(0, Q).cpu().numpy().reshape(ny, nz, nx)
            sim.close()
    finally:
        R.set_tuning()
    for mode, phi in phis.items():
        err = np.abs(phi - ref).max() / np.abs(ref).max()
        say("  layout", mode, "rel err", err)
        assert err < TOL


def test_inverse_layout_refused():
    """Two blocks per plane need nz % 4 == 0, four need nz % 8 == 0."""
    from paper_2602_10761_amd import runtime as R
    ens = W.make_ensemble(W.CONFIGS[1].replace(nx=16, ny=8, nz=10, n_particles=10))
    ens4 = W.make_ensemble(W.CONFIGS[1].replace(nx=16, ny=8, nz=12, n_particles=10))
    try:
        R.set_tuning(inv_plane=2)
        with pytest.raises(R.TriboError, match="nz % 4"):
            sim_of(ens)
        R.set_tuning(inv_plane=4)
        with pytest.raises(R.TriboError, match="nz % 8"):
            sim_of(ens4)
    finally:
        R.set_tuning()


# ---------------------------------------------------------------------------
# one step from the same initial state
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("case", ["plain", "charged", "dense", "gravity"])
def test_one_step_parity(case):
    say("one step", case)
    kw = dict(plain=dict(v_jitter=3.0, density_ratio=50.0),
              charged=dict(v_jitter=3.0, precharge=0.5, density_ratio=50.0, c_el=30.0),
              dense=dict(nx=8, ny=8, nz=8, n=20000, precharge=0.3, c_el=5.0, v_jitter=2.0),
              gravity=dict(g=(0.0, -0.02, 0.01), precharge=0.1, v_jitter=1.0))[case]
    ens = ens_small(**kw)
    sim = sim_of(ens, keep_deposit=True, source=True)
    sim.step(1)
    gpu = sim.state_np(0)
    gst = sim.stats(0)
    Qg = sim.field(0, 1).cpu().numpy()
    phig = sim.field(0, 0).cpu().numpy()
    fsg = sim.field(0, 2).cpu().numpy().reshape(3, -1)
    g = O.Geo.from_mesh(ens.mesh)
    st = O.Stats(g.ny)
    want = {}
    ref = O.step(g, ens.U, O.state_of(ens), ens.params, st, want=want)
    np.testing.assert_array_equal(Qg, want["Q"])
    perr = np.abs(phig - want["phi"].ravel()).max() / max(np.abs(want["phi"]).max(), 1e-300)
    err = state_errors(gpu, ref, ens.mesh)
    say("  phi err", perr, " state err", {k: float(f"{v:.2e}") for k, v in err.items()})
    assert perr < TOL
    assert max(err.values()) < TOL
    assert_stats_equal(gst, st)
    # 2-way coupling source: same cells, same summation order (ascending id)
    fserr = np.abs(fsg - want["fs"]).max() / np.abs(want["fs"]).max()
    say("  source err", fserr)
    assert np.all((fsg == 0.0) == (want["fs"] == 0.0))
    assert fserr < TOL
    sim.close()


def test_multi_step_parity():
    say("multi step")
    # shallow channel (h = 20) so that many particles reach the walls within the window
    ens = ens_small(n=6000, v_jitter=4.0, precharge=0.2, density_ratio=30.0, re_tau=20.0, c_el=5.0)
    ens.params["k_c"] = 0.02
    n = 40
    sim = sim_of(ens)
    sim.step(n)
    gpu = sim.state_np(0)
    gst = sim.stats(0)
    ref, st = oracle_run(ens, n)
    err = state_errors(gpu, ref, ens.mesh)
    say("  impacts", st.impacts, " state err", {k: float(f"{v:.2e}") for k, v in err.items()})
    assert st.impacts.sum() > 50
    assert_stats_equal(gst, st)
    assert max(err.values()) < TOL
    sim.close()


def test_long_run_profiles():
    """1000 steps with wall impacts and charging: the accumulated concentration
    and charge profiles over the y rows, the impact counts and the wall charge
    agree with the oracle's within 1 % (normwise)."""
    say("long run profiles")
    ens = ens_small(nx=16, ny=24, nz=16, n=3000, v_jitter=3.0, precharge=0.2, re_tau=40.0, c_el=5.0,
                    density_ratio=30.0)
    ens.params["k_c"] = 0.02
    n = 1000
    sim = sim_of(ens)
    sim.step(n)
    gst = sim.stats(0)
    sim.close()
    _, st = oracle_run(ens, n)
    assert gst["steps"] == st.steps == n
    assert st.impacts.sum() > 200
    for k, ref in (("crel_y", st.crel_y), ("qcum_y", st.qcum_y), ("impacts", st.impacts), ("wallq", st.wallq)):
        g = np.asarray(gst[k], dtype=np.float64)
        o = np.asarray(ref, dtype=np.float64)
        err = np.abs(g - o).max() / np.abs(o).max()
        say(f"  {k}: normwise rel diff {err:.2e}")
        assert err < 0.01, k


@pytest.mark.parametrize("ny", [128, 300])
def test_many_row_pairs_multi_step(ny):
    """Incremental sorts on meshes with many row pairs (16384 and 38400: the
    pair scan over more than one block's chunk) against the oracle over
    several steps."""
    say("many row pairs", ny)
    ens = ens_small(nx=4, ny=ny, nz=256, n=20000, v_jitter=3.0, precharge=0.2, re_tau=40.0, c_el=5.0)
    n = 4
    sim = sim_of(ens)
    sim.step(n)
    gpu = sim.state_np(0)
    gst = sim.stats(0)
    sim.close()
    ref, st = oracle_run(ens, n)
    err = state_errors(gpu, ref, ens.mesh)
    say("  impacts", st.impacts, " state err", {k: float(f"{v:.2e}") for k, v in err.items()})
    assert_stats_equal(gst, st)
    assert max(err.values()) < TOL


def test_sort_capacity_paths():
    """The fused sort's paths (member list in LDS; one list round per row when
    the pair exceeds the list but each of its rows fits; a second candidate
    pass through global memory otherwise): bitwise the same results for every
    capacity, and the oracle's."""
    from paper_2602_10761_amd import runtime as R
    say("sort capacity paths")
    ens = ens_small(nx=16, ny=24, nz=16, n=12000, v_jitter=3.0, precharge=0.2, re_tau=40.0, c_el=5.0)
    n = 5
    runs = {}
    try:
        for cap in (-1, 8, 64, 0):
            R.set_tuning(sort_cap=cap)
            sim = sim_of(ens)
            sim.step(n)
            runs[cap] = (sim.state_np(0), sim.stats(0))
            sim.close()
    finally:
        R.set_tuning()
    ref, st = oracle_run(ens, n)
    err = state_errors(runs[0][0], ref, ens.mesh)
    say("  state err", {k: float(f"{v:.2e}") for k, v in err.items()})
    assert max(err.values()) < TOL
    assert_stats_equal(runs[0][1], st)
    for cap in (-1, 8, 64):
        for k in KEYS:
            np.testing.assert_array_equal(runs[cap][0][k], runs[0][0][k])


def test_push_orders_bitwise():
    """The push's two block orders over the XCDs (consecutive slot ranges per
    XCD, the hardware's round robin) give bitwise the same steps."""
    from paper_2602_10761_amd import runtime as R
    say("push orders")
    ens = ens_small(nx=32, ny=40, nz=32, n=30000, v_jitter=3.0, precharge=0.2, re_tau=40.0, c_el=5.0)
    runs = {}
    try:
        for order in (1, 2):
            R.set_tuning(push_order=order)
            sim = sim_of(ens)
            sim.step(6)
            runs[order] = (sim.state_np(0), sim.stats(0))
            sim.close()
    finally:
        R.set_tuning()
    for k in KEYS:
        np.testing.assert_array_equal(runs[1][0][k], runs[2][0][k])
    for k in ("impacts", "wallq", "crel_y", "qcum_y", "qnow_y", "unhist"):
        np.testing.assert_array_equal(runs[1][1][k], runs[2][1][k])
    assert runs[1][1]["impacts"].sum() > 0


@pytest.mark.parametrize("graphs", [False, True])
def test_carrier_replacement(graphs):
    """tf_set_carrier: steps after a new carrier field follow the oracle with
    that field (also when the steps replay captured graphs)."""
    say("carrier replacement", graphs)
    ens = ens_small(n=3000, v_jitter=2.0, precharge=0.2, c_el=5.0)
    sim = sim_of(ens, graphs=graphs)
    sim.step(2)
    mid = sim.state_np(0)
    rng = np.random.default_rng(7)
    U2 = ens.U * 0.5 + 0.1 * rng.standard_normal(ens.U.shape)
    sim.set_carrier(0, U2)
    sim.step(2)
    gpu = sim.state_np(0)
    sim.close()
    g = O.Geo.from_mesh(ens.mesh)
    s = {k: np.array(mid[k], dtype=np.float64) for k in KEYS}
    for _ in range(2):
        s = O.step(g, U2, s, ens.params, None)
    err = state_errors(gpu, s, ens.mesh)
    say("  state err", {k: float(f"{v:.2e}") for k, v in err.items()})
    assert max(err.values()) < TOL


def test_far_movers_multi_step():
    """Fast particles that cross two or more cell rows in y or z per step (the
    sort's far list), over several steps, against the oracle."""
    say("far movers")
    ens = ens_small(nx=16, ny=16, nz=16, n=3000, re_tau=20.0, v_jitter=60.0, density_ratio=1000.0)
    n = 6
    g = O.Geo.from_mesh(ens.mesh)
    s = O.state_of(ens)
    st = O.Stats(g.ny)
    far = 0
    for _ in range(n):
        _, j0, k0 = O.locate(g, s["x"], s["y"], s["z"])
        s = O.step(g, ens.U, s, ens.params, st)
        _, j1, k1 = O.locate(g, s["x"], s["y"], s["z"])
        dk = np.abs(k1 - k0)
        far += int(np.sum((np.abs(j1 - j0) > 1) | ((dk > 1) & (dk < g.nz - 1))))
    sim = sim_of(ens)
    sim.step(n)
    gpu = sim.state_np(0)
    gst = sim.stats(0)
    sim.close()
    err = state_errors(gpu, s, ens.mesh)
    say("  far moves", far, " state err", {k: float(f"{v:.2e}") for k, v in err.items()})
    assert far > 500
    # counts exact; the fixed-point charge sums take the charges of states that
    # already differ by rounding after 1000+ impacts, so a charge sitting on a
    # rounding boundary may land one unit apart
    assert gst["steps"] == st.steps and gst["flags"] == st.flags
    np.testing.assert_array_equal(gst["impacts"], st.impacts)
    np.testing.assert_array_equal(gst["crel_y"], st.crel_y)
    for k, ref in (("wallq", st.wallq), ("qcum_y", st.qcum_y), ("qnow_y", st.qnow_y)):
        d = np.abs(np.asarray(gst[k], dtype=np.float64) - np.asarray(ref, dtype=np.float64))
        assert d.max() <= 4 * n, (k, d.max())
    assert max(err.values()) < TOL


@pytest.mark.parametrize("cfg", [2, 3])
def test_full_size_one_step(cfg):
    """The benchmark workloads at full size: one step, every particle compared."""
    say("full size config", cfg)
    ens = W.make_workload(cfg, precharge=0.05)[0]
    sim = sim_of(ens)
    sim.step(1)
    gpu = sim.state_np(0)
    gst = sim.stats(0)
    phig = sim.field(0, 0).cpu().numpy()
    sim.close()
    g = O.Geo.from_mesh(ens.mesh)
    st = O.Stats(g.ny)
    want = {}
    ref = O.step(g, ens.U, O.state_of(ens), ens.params, st, want=want)
    perr = np.abs(phig - want["phi"].ravel()).max() / np.abs(want["phi"]).max()
    err = state_errors(gpu, ref, ens.mesh)
    say("  phi err", perr, " state err", {k: float(f"{v:.2e}") for k, v in err.items()})
    assert perr < TOL
    assert max(err.values()) < TOL
    assert_stats_equal(gst, st)


@pytest.mark.parametrize("cfg", [2, 3])
def test_full_size_incremental_steps(cfg):
    """The benchmark workloads at full size in the launch configuration the
    benchmark times (tiles, inverse layout and sort capacity from the
    committed tuning cache): three steps, so that the last two run the
    incremental sort; a wall-normal velocity jitter brings several hundred
    wall impacts (charging: charges that change between deposits);
    every particle, the potential and the statistics compared with the
    oracle."""
    from paper_2602_10761_amd import autotune
    from paper_2602_10761_amd import runtime as R
    say("full size incremental config", cfg)
    ens = W.make_workload(cfg, precharge=0.05, v_jitter=3.0)[0]
    m = ens.mesh
    autotune.ensure_tuned_workload([ens])
    n = 3
    try:
        sim = sim_of(ens)
        sim.step(n)
        gpu = sim.state_np(0)
        gst = sim.stats(0)
        phig = sim.field(0, 0).cpu().numpy()
        sim.close()
    finally:
        R.set_tuning_class(m.nx, m.ny, m.nz)  # back to the built-in choice
    g = O.Geo.from_mesh(m)
    st = O.Stats(g.ny)
    ref = O.state_of(ens)
    want = {}
    for k in range(n):
        ref = O.step(g, ens.U, ref, ens.params, st, want=want if k == n - 1 else None)
    perr = np.abs(phig - want["phi"].ravel()).max() / np.abs(want["phi"]).max()
    err = state_errors(gpu, ref, m)
    say("  impacts", st.impacts, " phi err", perr, " state err", {k: float(f"{v:.2e}") for k, v in err.items()})
    assert gst["steps"] == n and st.impacts.sum() > 500
    assert perr < TOL
    assert max(err.values()) < TOL
    assert_stats_equal(gst, st)


# ---------------------------------------------------------------------------
# determinism, graphs, batching, checkpoint/resume, edge cases
# ---------------------------------------------------------------------------
def test_run_twice_bitwise():
    ens = ens_small(n=5000, v_jitter=3.0, precharge=0.3, c_el=20.0)
    outs = []
    for _ in range(2):
        sim = sim_of(ens)
        sim.step(15)
        outs.append((sim.state_np(0), sim.stats(0)))
        sim.close()
    for k in KEYS:
        np.testing.assert_array_equal(outs[0][0][k], outs[1][0][k])
    for k in ("impacts", "wallq", "crel_y", "qcum_y", "qnow_y", "unhist"):
        np.testing.assert_array_equal(outs[0][1][k], outs[1][1][k])


def test_graphs_equal_eager():
    ens = ens_small(n=3000, v_jitter=3.0, precharge=0.3)
    res = []
    for graphs in (False, True):
        sim = sim_of(ens, graphs=graphs)
        sim.step(7)
        sim.step(4)
        res.append((sim.state_np(0), sim.stats(0)))
        sim.close()
    for k in KEYS:
        np.testing.assert_array_equal(res[0][0][k], res[1][0][k])
    np.testing.assert_array_equal(res[0][1]["crel_y"], res[1][1]["crel_y"])
    assert res[1][1]["steps"] == 11


def test_batched_equals_plain():
    specs = [W.CONFIGS[1].replace(nx=16, ny=24, nz=32, n_particles=2500, v_jitter=3.0, precharge=0.2),
             W.CONFIGS[1].replace(re_tau=300.0, nx=48, ny=40, nz=20, n_particles=7000, v_jitter=2.0, d_choices=(1.0,)),
             W.CONFIGS[1].replace(nx=8, ny=8, nz=8, n_particles=0),
             W.CONFIGS[1].replace(re_tau=550.0, nx=40, ny=16, nz=12, n_particles=1, v_jitter=1.0),
             # plane too large for the fused inverse transforms (nz (nx/2 + 1) > 10240)
             W.CONFIGS[1].replace(nx=256, ny=6, nz=96, n_particles=3000, v_jitter=2.0),
             # 4-way coupling on for this one only (the others run the collision-enabled push)
             W.CONFIGS[1].replace(re_tau=2.0, nx=4, ny=4, nz=4, n_particles=600, precharge=0.3, v_jitter=1.0,
                                  d_choices=(0.5, 1.0), density_ratio=50.0, pp=1, k_pp=2.0),
             W.CONFIGS[1].replace(re_tau=100.0, nx=64, ny=10, nz=48, n_particles=4000, v_jitter=2.0, precharge=0.1)]
    ens = [W.make_ensemble(s, 4, 0, sub=m) for m, s in enumerate(specs)]
    from paper_2602_10761_amd import runtime as R
    # the first one transformed per whole plane, the fifth by the z and x
    # kernels, the last per quarter plane, the others per half plane
    R.set_tuning_class(16, 24, 32, inv_plane=1)
    R.set_tuning_class(256, 6, 96, inv_plane=3)
    R.set_tuning_class(64, 10, 48, inv_plane=4)
    try:
        sim = sim_of(ens, graphs=True, source=True)
        sim.step(9)
        batched = [(sim.state_np(e), sim.stats(e), sim.field(e, 2).cpu().numpy()) for e in range(len(ens))]
        sim.close()
        plain = []
        for E in ens:
            s1 = sim_of(E, source=True)
            s1.step(9)
            plain.append((s1.state_np(0), s1.stats(0), s1.field(0, 2).cpu().numpy()))
            s1.close()
    finally:
        R.set_tuning_class(16, 24, 32)
        R.set_tuning_class(256, 6, 96)
        R.set_tuning_class(64, 10, 48)
    for e, E in enumerate(ens):
        st, ss, fs = plain[e]
        np.testing.assert_array_equal(batched[e][2], fs)
        for k in KEYS:
            np.testing.assert_array_equal(batched[e][0][k], st[k])
        for k in ("impacts", "wallq", "crel_y", "qcum_y", "qnow_y", "unhist"):
            np.testing.assert_array_equal(batched[e][1][k], ss[k])


def test_resume_equals_continuous():
    ens = ens_small(n=4000, v_jitter=3.0, precharge=0.3, c_el=10.0)
    a = sim_of(ens)
    a.step(12)
    ref = a.state_np(0)
    a.close()
    b = sim_of(ens)
    b.step(5)
    mid = b.state(0)
    b.close()
    c = sim_of(ens)
    c.set_state(0, mid)
    c.step(7)
    out = c.state_np(0)
    c.close()
    for k in KEYS:
        np.testing.assert_array_equal(out[k], ref[k])


def test_conservation_and_flags():
    ens = ens_small(n=5000, v_jitter=4.0, precharge=0.2, density_ratio=30.0, re_tau=20.0, c_el=5.0)
    ens.params["k_c"] = 0.05
    sim = sim_of(ens)
    q0 = ens.q.sum()
    sim.step(60)
    s = sim.state_np(0)
    st = sim.stats(0)
    sim.close()
    assert st["impacts"].sum() > 50
    assert st["flags"] == 0
    wall = st["wallq"].sum() * 2.0 ** -40
    assert abs(s["q"].sum() - q0 + wall) < 1e-9
    r = 0.5 * s["d"]
    assert np.all((s["y"] >= r) & (s["y"] <= ens.mesh.ly - r))


# ---------------------------------------------------------------------------
# 4-way coupling: particle-particle collisions and charge exchange
# ---------------------------------------------------------------------------
def pp_ensemble(n=800, seed=0, **kw):
    spec = W.CONFIGS[1].replace(re_tau=2.0, nx=4, ny=4, nz=4, n_particles=n, precharge=0.3, v_jitter=1.0,
                                d_choices=(0.5, 1.0), density_ratio=50.0, pp=1, k_pp=2.0, **kw)
    return W.make_ensemble(spec, 1, seed)


@pytest.mark.parametrize("steps", [1, 6])
def test_pp_collisions_parity(steps):
    say("pp collisions", steps)
    ens = pp_ensemble(k_c=0.01)
    sim = sim_of(ens)
    sim.step(steps)
    gpu = sim.state_np(0)
    gst = sim.stats(0)
    sim.close()
    ref, st = oracle_run(ens, steps)
    err = state_errors(gpu, ref, ens.mesh)
    say("  pairs", gst["pp_pairs"], st.pp_pairs, " state err", {k: float(f"{v:.2e}") for k, v in err.items()})
    assert st.pp_pairs > 10 * steps
    assert gst["pp_pairs"] == st.pp_pairs
    assert max(err.values()) < TOL
    np.testing.assert_array_equal(gst["impacts"], st.impacts)
    np.testing.assert_array_equal(gst["crel_y"], st.crel_y)
    assert abs(gpu["q"].sum() - ref["q"].sum()) < 1e-12


def test_full_size_next_rows():
    """The 1e6-particle 128^3 workload with the next rows on together: 4-way
    coupling, the stochastic wall-charging model and the 2-way coupling
    source, two steps against the oracle (state, collision pairs, impacts and
    histograms exact, wall charge to the rounding of its sums, source)."""
    say("full size next rows")
    ens = W.make_workload(2, precharge=0.05, v_jitter=3.0, pp=1, k_pp=1.0, charging=1, ssm=SSM_PARAMS)[0]
    n = 2
    sim = sim_of(ens, source=True)
    sim.step(n)
    gpu = sim.state_np(0)
    gst = sim.stats(0)
    fsg = sim.field(0, 2).cpu().numpy().reshape(3, -1)
    sim.close()
    g = O.Geo.from_mesh(ens.mesh)
    st = O.Stats(g.ny)
    ref = O.state_of(ens)
    want = {}
    for k in range(n):
        ref = O.step(g, ens.U, ref, ens.params, st, want=want if k == n - 1 else None)
    err = state_errors(gpu, ref, ens.mesh)
    fserr = np.abs(fsg - want["fs"]).max() / np.abs(want["fs"]).max()
    say("  pairs", gst["pp_pairs"], st.pp_pairs, " impacts", st.impacts, " source err", fserr,
        " state err", {k: float(f"{v:.2e}") for k, v in err.items()})
    assert st.pp_pairs > 100 and st.impacts.sum() > 100
    assert gst["pp_pairs"] == st.pp_pairs
    np.testing.assert_array_equal(gst["impacts"], st.impacts)
    np.testing.assert_array_equal(gst["unhist"], st.unhist)
    np.testing.assert_array_equal(gst["crel_y"], st.crel_y)
    assert np.all(np.abs(gst["wallq"] - st.wallq) <= st.impacts)
    assert max(err.values()) < TOL
    assert np.all((fsg == 0.0) == (want["fs"] == 0.0)) and fserr < TOL


def test_pp_record_refused():
    from paper_2602_10761_amd.runtime import TriboError
    sim = sim_of(pp_ensemble(n=100), traj_steps=2)
    with pytest.raises(TriboError):
        sim.step(1, record=True)
    sim.step(1)
    assert sim.stats(0)["steps"] == 1
    sim.close()


# ---------------------------------------------------------------------------
# stochastic scaling model of wall charging
# ---------------------------------------------------------------------------
SSM_PARAMS = (-2e-3, -1.5e-3, 4e-4, 0.6, 20.0, 0.5, 1.0)  # dq0min, mu0, sigma0, gamma0, csat, d0, un0


def ssm_ensemble(**kw):
    spec = W.CONFIGS[1].replace(re_tau=20.0, nx=16, ny=16, nz=16, n_particles=4000, v_jitter=4.0, precharge=0.0,
                                density_ratio=30.0, charging=1, ssm=SSM_PARAMS, seed=77, **kw)
    return W.make_ensemble(spec, 1, 0)


def test_ssm_parity():
    say("ssm")
    ens = ssm_ensemble()
    n = 30
    sim = sim_of(ens)
    sim.step(n)
    gpu = sim.state_np(0)
    gst = sim.stats(0)
    sim.close()
    ref, st = oracle_run(ens, n)
    err = state_errors(gpu, ref, ens.mesh)
    say("  impacts", st.impacts, " state err", {k: float(f"{v:.2e}") for k, v in err.items()})
    assert st.impacts.sum() > 40
    np.testing.assert_array_equal(gst["impacts"], st.impacts)
    np.testing.assert_array_equal(gst["unhist"], st.unhist)
    assert max(err.values()) < TOL
    # wall charge: sums of rne(-dq 2^40) (an impact may round the other way)
    assert np.all(np.abs(gst["wallq"] - st.wallq) <= st.impacts)
    assert np.std(gpu["q"][gpu["q"] != 0]) > 0  # random, not one value


def test_ssm_deterministic_limit_equals_condenser():
    # sigma0 = gamma0 = 0, mu0 = dq0min, csat and dq0min matched to k_c, delta_u
    kc, e, dU, d, un0 = 0.02, 0.9, 1.0, 0.5, 0.7
    dq0 = -kc * (1 + e) ** 0.4 * dU * un0 ** 0.8
    base = dict(re_tau=20.0, nx=16, ny=16, nz=16, n_particles=3000, v_jitter=4.0, density_ratio=30.0, k_c=kc, e=e)
    a = W.make_ensemble(W.CONFIGS[1].replace(**base), 1, 0)
    b = W.make_ensemble(W.CONFIGS[1].replace(charging=1, ssm=(dq0, dq0, 0.0, 0.0, 4.0 * dU / d ** 2, d, un0),
                                             **base), 1, 0)
    res = []
    for E in (a, b):
        sim = sim_of(E)
        sim.step(40)
        res.append((sim.state_np(0), sim.stats(0)))
        sim.close()
    assert res[0][1]["impacts"].sum() > 40
    np.testing.assert_array_equal(res[0][1]["impacts"], res[1][1]["impacts"])
    np.testing.assert_allclose(res[1][0]["q"], res[0][0]["q"], rtol=1e-12, atol=1e-15)


def test_carrier_every_step_with_graphs():
    """A carrier field that changes every step (alternating two fields), graph
    replays, against the oracle."""
    ens = ens_small(n=2000, v_jitter=2.0)
    rng = np.random.default_rng(3)
    U2 = ens.U * 0.8 + 0.2 * rng.standard_normal(ens.U.shape)
    sim = sim_of(ens, graphs=True)
    g = O.Geo.from_mesh(ens.mesh)
    s = O.state_of(ens)
    for n in range(6):
        U = ens.U if n % 2 == 0 else U2
        sim.set_carrier(0, U)
        sim.step(1)
        s = O.step(g, U, s, ens.params, None)
    gpu = sim.state_np(0)
    sim.close()
    err = state_errors(gpu, s, ens.mesh)
    say("  carrier every step, state err", {k: float(f"{v:.2e}") for k, v in err.items()})
    assert max(err.values()) < TOL
