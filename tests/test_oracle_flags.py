"""Sticky fault flags of the oracle step (CPU only).

The paper defines no fault handling; the step's own contract is: a particle
whose new position, velocity or charge is not finite raises F_NONFINITE; a
fixed-point conversion whose rounded value reaches 2^62 in magnitude (or is
not finite) contributes 0 and raises F_OVERFLOW; a particle still outside
[d/2, ly - d/2] after its rebound raises F_OUTSIDE.  The step always runs to
completion.  The HIP step follows the same contract (tests/test_gpu_flags.py).
"""
import numpy as np
import pytest

import oracle as O
from paper_2602_10761_amd import workload as W


def ens_small(**kw):
    spec = W.CONFIGS[1].replace(nx=16, ny=16, nz=16, n_particles=500, v_jitter=1.0, precharge=0.1, **kw)
    return W.make_ensemble(spec, 1, 0)


def one_step(ens, s):
    g = O.Geo.from_mesh(ens.mesh)
    st = O.Stats(g.ny)
    want = {}
    with np.errstate(invalid="ignore", over="ignore"):
        out = O.step(g, ens.U, s, ens.params, st, want=want)
    return out, st, want


def test_clean_step_raises_nothing():
    ens = ens_small()
    _, st, _ = one_step(ens, O.state_of(ens))
    assert st.flags == 0


def test_nonfinite_velocity():
    ens = ens_small()
    s = O.state_of(ens)
    s["vz"][17] = np.nan
    out, st, _ = one_step(ens, s)
    assert st.flags == O.F_NONFINITE
    assert np.isnan(out["x"][17]) and np.isnan(out["vz"][17])
    others = np.arange(ens.n) != 17
    assert all(np.all(np.isfinite(out[k][others])) for k in O.KEYS)


def test_nonfinite_position_is_reported_once_in_y():
    ens = ens_small()
    s = O.state_of(ens)
    s["vy"][3] = np.inf
    out, st, _ = one_step(ens, s)
    assert st.flags & O.F_NONFINITE


def test_deposit_overflow_contributes_nothing():
    ens = ens_small(c_el=0.0)
    s = O.state_of(ens)
    big = 2.0 ** 14          # q 2^48 = 2^62: the first magnitude out of range
    s["q"][5] = big
    s["q"][9] = -3.0e4
    out, st, want = one_step(ens, s)
    assert st.flags == O.F_OVERFLOW
    keep = np.ones(ens.n, dtype=bool)
    keep[[5, 9]] = False
    # the cell sums hold every other particle's rne(q 2^48) exactly, nothing of the two
    Q = np.zeros_like(want["Q"])
    np.add.at(Q, want["cid"][keep], np.rint(s["q"][keep] * 2.0 ** 48).astype(np.int64))
    np.testing.assert_array_equal(want["Q"], Q)
    assert int(st.qnow_y.sum()) == int(Q.sum())
    # just inside the range: no flag
    s2 = O.state_of(ens)
    s2["q"][5] = np.nextafter(big, 0.0)
    _, st2, _ = one_step(ens, s2)
    assert st2.flags == 0


def test_wall_charge_overflow():
    ens = ens_small(c_el=0.0)
    g = O.Geo.from_mesh(ens.mesh)
    s = O.state_of(ens)
    p = 11
    s["y"][p] = 0.5 * s["d"][p] + 1e-3
    s["vy"][p] = -40.0
    s["q"][p] = -1.0e4        # inside the deposit range (below 2^14) ...
    prm = dict(ens.params, k_c=1.0e3)   # ... but |dq| = f |dU + q| beyond 2^22: -dq 2^40 out of range
    st = O.Stats(g.ny)
    with np.errstate(invalid="ignore", over="ignore"):
        out = O.step(g, ens.U, s, prm, st)
    assert st.impacts.sum() >= 1
    assert st.flags == O.F_OVERFLOW
    assert np.isfinite(out["q"][p])


def test_penetration_beyond_the_channel():
    ens = ens_small()
    s = O.state_of(ens)
    p = 21
    s["vy"][p] = -1.0e5       # one step carries it far below the lower wall
    out, st, _ = one_step(ens, s)
    assert st.impacts[0] >= 1
    assert st.flags == O.F_OUTSIDE
    assert out["y"][p] > ens.mesh.ly - 0.5 * s["d"][p]
