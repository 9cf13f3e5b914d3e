"""Pins of the oracle's forward-mode derivative (CPU only).

dJ/dtheta for theta = (k_c, dU, e), with the discrete events held fixed, is
checked against (1) the derivative of the closed-form repeated-impact charge
and (2) central differences of the oracle replaying the same events.
"""
import math

import numpy as np
import pytest

import oracle as O
from oracle import tangent as T
from paper_2602_10761_amd import workload as W

BASE = dict(dt=0.01, density_ratio=1e300, k_c=0.02, delta_u=1.0, e=0.9, c_el=0.0, g=(0.0, 0.0, 0.0),
            un_bin=0.05)


def closed_form_grad(n, V, kc, dU, e, q0=0.0):
    """d q_n / d(k_c, dU, e) for q_n = -dU + (dU + q0) prod_m (1 - f_m), f_m = k_c (1+e)^0.4 (V e^m)^0.8."""
    f = np.array([kc * (1 + e) ** 0.4 * (V * e ** m) ** 0.8 for m in range(n)])
    P = np.prod(1 - f)
    dkc = (dU + q0) * P * np.sum(-(f / kc) / (1 - f))
    ddU = -1.0 + P
    dfe = f * (0.4 / (1 + e) + 0.8 * np.arange(n) / e)
    de = (dU + q0) * P * np.sum(-dfe / (1 - f))
    return np.array([dkc, ddU, de])


def test_tangent_matches_closed_form_repeated_impacts():
    g = O.Geo(2, 2, 2, 10.0, 10.0, np.array([0.0, 1.0, 2.0]))
    U = np.zeros((3, 3, 2, 2))
    n = 3
    s = {k: np.zeros(n) for k in O.KEYS}
    s["d"][:] = 0.2
    V = np.array([1.0, 2.5, 0.7])
    s["vy"][:] = -V
    s["y"][:] = [0.5, 1.0, 1.5]
    s["x"][:] = [1.0, 3.0, 6.0]
    s["z"][:] = [1.0, 6.0, 3.0]
    steps = 900
    J, dJ, recs = T.gradient_tangent(g, U, s, BASE, steps)
    hits = sum((r["wall"] >= 0).astype(int) for r in recs)
    assert hits.min() >= 2
    want = np.mean([closed_form_grad(hits[p], V[p], BASE["k_c"], BASE["delta_u"], BASE["e"]) for p in range(n)], 0)
    np.testing.assert_allclose(dJ[0], want, rtol=1e-10, atol=1e-14)
    # wall flux: every impact moves charge from particle to wall, so J2 = -N dJ1/T
    np.testing.assert_allclose(dJ[1], -n * dJ[0] / (steps * BASE["dt"]), rtol=1e-10, atol=1e-14)


@pytest.mark.parametrize("seed,charged", [(0, False), (1, True)])
def test_tangent_matches_central_differences(seed, charged):
    spec = W.CONFIGS[1].replace(nx=8, ny=12, nz=8, n_particles=600, v_jitter=4.0, re_tau=10.0,
                                density_ratio=200.0, precharge=0.3 if charged else 0.0, c_el=40.0 if charged else 0.0)
    ens = W.make_ensemble(spec, 1, seed)
    g = O.Geo.from_mesh(ens.mesh)
    prm = dict(ens.params, k_c=0.05)
    s0 = O.state_of(ens)
    J, dJ, recs = T.gradient_tangent(g, ens.U, s0, prm, 40)
    assert sum(int((r["wall"] >= 0).sum()) for r in recs) > 50
    fd = T.gradient_fd(g, ens.U, s0, prm, recs, h=1e-6)
    scale = np.abs(dJ).max(axis=1, keepdims=True)
    assert np.all(np.abs(dJ - fd) <= 1e-6 * scale + 1e-12), (dJ, fd)
    # the replayed objective equals the free run (events identical at theta)
    np.testing.assert_allclose(T.objectives_replay(g, ens.U, s0, prm, recs), J, rtol=1e-14)
