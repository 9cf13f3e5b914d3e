"""Sticky fault flags of the HIP step against the oracle (through the C ABI).

Each case plants its fault in the input data (a non-finite velocity, a charge
beyond the fixed-point range, a penetration deeper than the channel); every
kernel runs to completion.  After one step both sides must raise the same flag
and agree on every unaffected particle to the per-step bar.
"""
import sys

import numpy as np
import pytest

import oracle as O
from helpers import KEYS, state_errors
from paper_2602_10761_amd import workload as W

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def run_both(ens, s0, prm_over=None):
    from paper_2602_10761_amd.runtime import TriboSim
    for k in KEYS:
        setattr(ens, k, np.array(s0[k]))
    if prm_over:
        ens.params.update(prm_over)
    sim = TriboSim([ens])
    sim.step(1)
    gpu = sim.state_np(0)
    gst = sim.stats(0)
    sim.close()
    g = O.Geo.from_mesh(ens.mesh)
    st = O.Stats(g.ny)
    with np.errstate(invalid="ignore", over="ignore"):
        ref = O.step(g, ens.U, O.state_of(ens), ens.params, st)
    return gpu, gst, ref, st


def base(**kw):
    spec = W.CONFIGS[1].replace(nx=16, ny=16, nz=16, n_particles=2000, v_jitter=1.0, precharge=0.1, **kw)
    return W.make_ensemble(spec, 1, 0)


def compare(ens, gpu, gst, ref, st, flag, skip):
    say("  flags gpu", gst["flags"], "oracle", st.flags)
    assert st.flags == flag
    assert gst["flags"] == flag
    np.testing.assert_array_equal(gst["impacts"], st.impacts)
    np.testing.assert_array_equal(gst["crel_y"], st.crel_y)
    np.testing.assert_array_equal(gst["qnow_y"], st.qnow_y)
    keep = np.ones(ens.n, dtype=bool)
    keep[skip] = False
    err = state_errors({k: gpu[k][keep] for k in KEYS}, {k: ref[k][keep] for k in KEYS}, ens.mesh)
    say("  state err", {k: float(f"{v:.2e}") for k, v in err.items()})
    assert max(err.values()) < 1e-12


def test_flag_nonfinite():
    say("flag nonfinite")
    ens = base()
    s = O.state_of(ens)
    s["vz"][17] = np.nan
    gpu, gst, ref, st = run_both(ens, s)
    compare(ens, gpu, gst, ref, st, O.F_NONFINITE, [17])
    assert np.isnan(gpu["x"][17]) and np.isnan(gpu["vz"][17])


def test_flag_deposit_overflow():
    say("flag deposit overflow")
    ens = base(c_el=0.0)
    s = O.state_of(ens)
    s["q"][5] = 2.0 ** 14
    s["q"][9] = -3.0e4
    gpu, gst, ref, st = run_both(ens, s)
    compare(ens, gpu, gst, ref, st, O.F_OVERFLOW, [])


def test_flag_wall_charge_overflow():
    say("flag wall overflow")
    ens = base(c_el=0.0)
    s = O.state_of(ens)
    p = 11
    s["y"][p] = 0.5 * s["d"][p] + 1e-3
    s["vy"][p] = -40.0
    s["q"][p] = -1.0e4
    gpu, gst, ref, st = run_both(ens, s, dict(k_c=1.0e3))
    assert st.impacts.sum() >= 1
    compare(ens, gpu, gst, ref, st, O.F_OVERFLOW, [])


def test_flag_outside():
    say("flag outside")
    ens = base()
    s = O.state_of(ens)
    s["vy"][21] = -1.0e5
    gpu, gst, ref, st = run_both(ens, s)
    compare(ens, gpu, gst, ref, st, O.F_OUTSIDE, [])
