"""The benchmark workloads at their stated shapes, against the oracle and
against each other (through the C ABI).

* the 64-ensemble batched workload (N_p log-uniform in [1e4, 1e6], Re_tau in
  {180, 300, 395, 550} with 64^3..160^3 meshes, one d_p+ per ensemble): every
  ensemble of the batched handle bitwise equal to its own plain run, and one
  ensemble per mesh class from the batched handle against the oracle (1e-12
  after one step with exact deposit statistics and impacts, and after ten);
* the 1e6-particle 128^3 and 4e6-particle 192x160x192 workloads over their
  2000 steps: invariants
  (flags, charge balance between particles and walls, containment, row
  counts) and bitwise repeatability;
* the 1e4-particle 32^3 workload at its own parameters over its 1000 steps:
  concentration and charge profiles within 1 % of the oracle's (measured:
  identical), and the same with wall-normal velocity jitter and charged
  particles, so that impacts and wall charging take part.
"""
import sys

import numpy as np
import pytest

import oracle as O
from helpers import KEYS, oracle_run, state_errors
from paper_2602_10761_amd import workload as W

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def stats_equal(gs, st):
    assert gs["steps"] == st.steps and gs["flags"] == st.flags
    for k, ref in (("impacts", st.impacts), ("wallq", st.wallq), ("unhist", st.unhist), ("crel_y", st.crel_y),
                   ("qcum_y", st.qcum_y), ("qnow_y", st.qnow_y)):
        np.testing.assert_array_equal(gs[k], ref, err_msg=k)


@pytest.fixture(scope="module")
def batch4():
    return W.make_workload(4)


def test_config4_batched_equals_plain(batch4):
    from paper_2602_10761_amd.runtime import TriboSim
    ens = batch4
    say("config 4:", len(ens), "ensembles,", sum(E.n for E in ens), "particles")
    n = 3
    sim = TriboSim(ens, graphs=True)
    sim.step(n)
    batched = [(sim.state_np(e), sim.stats(e)) for e in range(len(ens))]
    sim.close()
    del sim
    for e, E in enumerate(ens):
        s1 = TriboSim([E])
        s1.step(n)
        st, ss = s1.state_np(0), s1.stats(0)
        s1.close()
        for k in KEYS:
            np.testing.assert_array_equal(batched[e][0][k], st[k], err_msg=f"ensemble {e} {k}")
        for k in ("impacts", "wallq", "crel_y", "qcum_y", "qnow_y", "unhist"):
            np.testing.assert_array_equal(batched[e][1][k], ss[k], err_msg=f"ensemble {e} {k}")


def test_config4_mesh_classes_vs_oracle(batch4):
    from paper_2602_10761_amd.runtime import TriboSim
    ens = batch4
    # the smallest ensemble of each mesh class (keeps the oracle quick)
    pick = {}
    for e, E in enumerate(ens):
        m = E.mesh.nx
        if m not in pick or E.n < ens[pick[m]].n:
            pick[m] = e
    assert sorted(pick) == [64, 96, 128, 160]
    sim = TriboSim(ens, graphs=True)
    sim.step(1)
    one = {e: (sim.state_np(e), sim.stats(e)) for e in pick.values()}
    sim.step(9)
    ten = {e: (sim.state_np(e), sim.stats(e)) for e in pick.values()}
    sim.close()
    for m, e in sorted(pick.items()):
        E = ens[e]
        g = O.Geo.from_mesh(E.mesh)
        s = O.state_of(E)
        st = O.Stats(g.ny)
        for n in range(10):
            s = O.step(g, E.U, s, E.params, st)
            if n == 0:
                err = state_errors(one[e][0], s, E.mesh)
                say(f"  {m}^3 ensemble {e} ({E.n} particles): 1 step err {max(err.values()):.2e}")
                assert max(err.values()) < 1e-12
                stats_equal(one[e][1], st)
        err = state_errors(ten[e][0], s, E.mesh)
        say(f"  {m}^3 ensemble {e}: 10 steps err {max(err.values()):.2e}")
        assert max(err.values()) < 1e-12
        np.testing.assert_array_equal(ten[e][1]["impacts"], st.impacts)
        np.testing.assert_array_equal(ten[e][1]["crel_y"], st.crel_y)


@pytest.mark.parametrize("variant", ["own", "jitter"])
def test_config1_long_run(variant):
    from paper_2602_10761_amd.runtime import TriboSim
    kw = {} if variant == "own" else dict(v_jitter=3.0, precharge=0.01)
    ens = W.make_workload(1, **kw)[0]
    if variant == "jitter":
        ens.params["k_c"] = 0.02
    n = 1000
    sim = TriboSim([ens], graphs=True)
    sim.step(n)
    gs = sim.stats(0)
    sim.close()
    _, st = oracle_run(ens, n)
    say(f"config 1 ({variant}): impacts gpu {gs['impacts']} oracle {st.impacts}")
    assert gs["steps"] == st.steps == n
    if variant == "jitter":
        assert st.impacts.sum() > 100
    for k, ref in (("crel_y", st.crel_y), ("qcum_y", st.qcum_y), ("impacts", st.impacts), ("wallq", st.wallq)):
        g = np.asarray(gs[k], dtype=np.float64)
        o = np.asarray(ref, dtype=np.float64)
        err = np.abs(g - o).max() / max(np.abs(o).max(), 1e-300) if np.abs(o).max() > 0 else np.abs(g).max()
        say(f"  {k}: normwise rel diff {err:.2e}")
        assert err < 0.01, k


@pytest.mark.parametrize("cfg", [2, 3])
def test_full_length_invariants(cfg):
    """The 1e6-particle 128^3 and 4e6-particle 192x160x192 workloads over
    their stated 2000 steps in the
    launch configuration the benchmark times (tuned tiles, sort capacity and
    push order), charged and with wall-normal velocity jitter so that
    particles keep hitting the walls: no fault flag; the charge the particles
    lose is the charge the walls gain (to the fixed-point rounding of the wall
    sums, half a unit of 2^-40 per impact); every particle inside the
    channel; every step counts every particle once in the row histogram; a
    second run is bitwise the same.  The oracle's cost at this size rules out
    a particle-by-particle comparison over 2000 steps; the full-size one- and
    three-step comparisons cover that."""
    from paper_2602_10761_amd import autotune
    from paper_2602_10761_amd.runtime import TriboSim
    ens = W.make_workload(cfg, precharge=0.05, v_jitter=3.0)[0]
    autotune.ensure_tuned_workload([ens])
    n = 2000
    runs = []
    for rep in range(2):
        sim = TriboSim([ens])
        sim.step(n)
        runs.append((sim.state_np(0), sim.stats(0)))
        sim.close()
        say(f"config {cfg}, {n} steps, run {rep}: impacts {runs[-1][1]['impacts']}")
    s, st = runs[0]
    assert st["steps"] == n and st["flags"] == 0
    impacts = int(st["impacts"].sum())
    assert impacts > 0.01 * ens.n
    wall = st["wallq"].sum() * 2.0 ** -40
    q0, q1 = ens.q.sum(), s["q"].sum()
    tol = impacts * 2.0 ** -41 + 1e-12 * (np.abs(s["q"]).sum() + abs(wall))
    say(f"  charge: particles {q0:.6e} -> {q1:.6e}, walls {wall:.6e}, imbalance {q1 - q0 + wall:.2e} (bound {tol:.2e})")
    assert abs(q1 - q0 + wall) < tol
    r = 0.5 * s["d"]
    m = ens.mesh
    assert np.all((s["y"] >= r) & (s["y"] <= m.ly - r))
    assert np.all((s["x"] >= 0) & (s["x"] < m.lx) & (s["z"] >= 0) & (s["z"] < m.lz))
    assert int(st["crel_y"].sum()) == n * ens.n
    for k in KEYS:
        np.testing.assert_array_equal(runs[1][0][k], s[k], err_msg=k)
    for k in ("impacts", "wallq", "unhist", "crel_y", "qcum_y", "qnow_y"):
        np.testing.assert_array_equal(runs[1][1][k], st[k], err_msg=k)
