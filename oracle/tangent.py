"""Forward-mode (tangent-linear) derivative of the particle step -- TEST INFRASTRUCTURE.

Derivatives of J1 = <q> (mean particle charge, normalised by q_sat as in
Sec. 4.1) and J2 = wall charge flux (charge received by the walls per unit
time) with respect to theta = (k_c, dU, e), the condenser-model charge
transfer coefficient, contact potential difference and restitution
coefficient (Sec. 2.2-2.3.1), with the discrete events of a recorded forward
run held fixed: the cell of every particle, the wall impacts and the periodic
wraps.  The fixed-point deposit is differentiated as the identity.

Each quantity of ``tribo_oracle.step`` is differentiated in the order the
step computes it; three tangent directions (one per component of theta) are
carried together on a leading axis.
"""
from __future__ import annotations

import math
from typing import Dict, List, Tuple

import numpy as np

from .tribo_oracle import (FIX_DEP, INV4PI, KEYS, TWO_THIRDS, Geo, cell_index, efield, interp,
                           poisson_density, same_cell_segments, step)


def interp_grad(g: Geo, U, x, y, z, i, j, k):
    """Jacobian of the trilinear carrier velocity w.r.t. position: [comp][dir]."""
    tx = (x - i * g.dx) / g.dx
    ty = (y - g.yf[j]) / g.dy[j]
    tz = (z - k * g.dz) / g.dz
    i1 = (i + 1) % g.nx
    k1 = (k + 1) % g.nz
    j1 = j + 1
    out = []
    for c in range(3):
        Uc = U[c]
        a000, a100 = Uc[j, k, i], Uc[j, k, i1]
        a001, a101 = Uc[j, k1, i], Uc[j, k1, i1]
        a010, a110 = Uc[j1, k, i], Uc[j1, k, i1]
        a011, a111 = Uc[j1, k1, i], Uc[j1, k1, i1]
        c00 = a000 * (1 - tx) + a100 * tx
        c01 = a001 * (1 - tx) + a101 * tx
        c10 = a010 * (1 - tx) + a110 * tx
        c11 = a011 * (1 - tx) + a111 * tx
        c0 = c00 * (1 - tz) + c01 * tz
        c1 = c10 * (1 - tz) + c11 * tz
        dtx = ((a100 - a000) * (1 - tz) + (a101 - a001) * tz) * (1 - ty) + \
              ((a110 - a010) * (1 - tz) + (a111 - a011) * tz) * ty
        dtz = (c01 - c00) * (1 - ty) + (c11 - c10) * ty
        dty = c1 - c0
        out.append((dtx / g.dx, dty / g.dy[j], dtz / g.dz))
    return out


def coulomb_tangent(x, y, z, q, dx_, dy_, dz_, dq, cid):
    """d/d(state) of S_i = sum_{j in cell, j != i} q_j r_ij / |r_ij|^3, 3 directions."""
    n = x.shape[0]
    nd = dq.shape[0]
    out = np.zeros((nd, 3, n))
    if n == 0:
        return out
    order, start, end = same_cell_segments(cid)
    pos = np.arange(n)
    kmax = int((end - start).max())
    for m in range(kmax):
        t = start + m
        ok = (t < end) & (t != pos)
        tt = np.where(ok, t, pos)
        a = order            # particle ids at sorted positions
        b = order[tt]
        r = np.stack([x[a] - x[b], y[a] - y[b], z[a] - z[b]])
        r2 = (r * r).sum(0)
        ok &= r2 > 0.0
        r2s = np.where(ok, r2, 1.0)
        inv3 = 1.0 / (r2s * np.sqrt(r2s))
        inv5 = inv3 / r2s
        for dd in range(nd):
            dr = np.stack([dx_[dd, a] - dx_[dd, b], dy_[dd, a] - dy_[dd, b], dz_[dd, a] - dz_[dd, b]])
            rdr = (r * dr).sum(0)
            # d(q_b r/|r|^3) = dq_b r/|r|^3 + q_b (dr/|r|^3 - 3 r (r.dr)/|r|^5)
            term = dq[dd, b] * r * inv3 + q[b] * (dr * inv3 - 3.0 * r * rdr * inv5)
            out[dd, :, a] += np.where(ok, term, 0.0).T
    return out


def step_tangent(g: Geo, U, s: Dict[str, np.ndarray], ds: Dict[str, np.ndarray], prm: dict,
                 dtheta: np.ndarray, rec: dict):
    """One step of the state and its tangents (ds[key] has shape [nd, n]).

    dtheta[nd, 3]: tangent of (k_c, dU, e) per direction.  Returns (s1, ds1,
    dW[nd, 2]) where dW is the tangent of the charge received by each wall.
    """
    x, y, z, vx, vy, vz, q, d = (s[k] for k in KEYS)
    nd = dtheta.shape[0]
    dt = prm["dt"]
    rr = prm["density_ratio"]
    kc, dU, e = prm["k_c"], prm["delta_u"], prm["e"]
    cel = prm["c_el"]
    i, j, k = rec["i"], rec["j"], rec["k"]
    cid = cell_index(g, i, j, k)
    dkc, ddU, de = dtheta[:, 0:1], dtheta[:, 1:2], dtheta[:, 2:3]

    # forward quantities, exactly as in step()
    s1 = step(g, U, s, prm, replay=rec, want=(want := {}))
    Ex, Ey, Ez = want["E"]
    Ep = np.stack([Ex.ravel()[cid], Ey.ravel()[cid], Ez.ravel()[cid]])
    u = np.stack(want["u"])
    S = np.stack(want["coul"])

    # tangent of the mesh field: deposit (identity), Poisson, E = -grad(phi)
    dEp = np.zeros((nd, 3, x.shape[0]))
    for dd in range(nd):
        dQ = np.zeros(g.ncell)
        np.add.at(dQ, cid, ds["q"][dd])
        dphi = poisson_density(g, dQ.reshape(g.ny, g.nz, g.nx) / g.vol[:, None, None])
        dE = efield(g, dphi)
        dEp[dd] = np.stack([dE[c].ravel()[cid] for c in range(3)])

    G = interp_grad(g, U, x, y, z, i, j, k)
    dX = np.stack([ds["x"], ds["y"], ds["z"]], axis=1)             # [nd, 3, n]
    du = np.stack([sum(G[c][a] * dX[:, a] for a in range(3)) for c in range(3)], axis=1)
    dS = coulomb_tangent(x, y, z, q, ds["x"], ds["y"], ds["z"], ds["q"], cid)

    ke = (cel * q) / ((d * d) * d)
    dke = cel * ds["q"] / ((d * d) * d)
    a = ke * (Ep + S * INV4PI)                                      # without gravity (constant)
    da = dke[:, None, :] * (Ep + S * INV4PI)[None] + ke[None, None, :] * (dEp + dS * INV4PI)

    v = np.stack([vx, vy, vz])
    dv = np.stack([ds["vx"], ds["vy"], ds["vz"]], axis=1)
    rel_v = v - u
    rel = np.sqrt((rel_v * rel_v).sum(0))
    re = rel * d
    phid = np.where(re <= 1000.0, 1.0 + np.power(re, TWO_THIRDS) / 6.0, 0.424 * re / 24.0)
    dphid_dre = np.where(re <= 1000.0, (TWO_THIRDS / 6.0) * np.power(np.where(re > 0, re, 1.0), -1.0 / 3.0),
                         0.424 / 24.0)
    dphid_dre = np.where(re > 0, dphid_dre, 0.0)
    taup = ((rr * d) * d) / 18.0
    sdr = phid / taup
    den = 1.0 + dt * sdr
    drel = dv - du
    unit = np.where(rel > 0, rel_v / np.where(rel > 0, rel, 1.0), 0.0)
    dre = d * (unit[None] * drel).sum(1)                            # [nd, n]
    dsdr = dphid_dre * dre / taup
    gp = np.array([(1.0 - 1.0 / rr) * gc for gc in prm.get("g", (0.0, 0.0, 0.0))])[:, None]
    v1 = (v + dt * (u * sdr + gp + a)) / den
    dv1 = (dv + dt * (du * sdr + u[None] * dsdr[:, None, :] + da)) / den - v1[None] * (dt * dsdr / den)[:, None, :]
    dx1 = dX + dt * dv1
    y1 = y + dt * v1[1]

    # wall impact (events replayed)
    wall = rec["wall"]
    r = 0.5 * d
    top = g.ly - r
    lo, hi = wall == 0, wall == 1
    hit = lo | hi
    rho = np.where(lo, r, top)
    sgn = np.where(lo, -1.0, 1.0)
    un = np.where(hit, sgn * v1[1], 0.0)
    dun = np.where(hit, sgn * dv1[:, 1], 0.0)
    P = math.pow(1.0 + e, 0.4)
    un08 = np.power(np.where(hit, un, 1.0), 0.8)
    f = np.where(hit, kc * P * un08, 0.0)
    unsafe = np.where(hit & (un > 0), un, 1.0)
    df = np.where(hit, P * un08 * dkc + f * (0.4 * de / (1.0 + e) + 0.8 * dun / unsafe), 0.0)
    gq = dU + q
    dgq = ddU + ds["q"]
    dq1 = np.where(hit, ds["q"] - df * gq - f * dgq, ds["q"])
    dW = np.zeros((nd, 2))
    for w, m in ((0, lo), (1, hi)):
        dW[:, w] = (df * gq + f * dgq)[:, m].sum(1)
    dy1 = np.where(hit, de * (rho - y1) - e * dx1[:, 1], dx1[:, 1])
    dvy1 = np.where(hit, -de * v1[1] - e * dv1[:, 1], dv1[:, 1])

    ds1 = dict(x=dx1[:, 0], y=dy1, z=dx1[:, 2], vx=dv1[:, 0], vy=dvy1, vz=dv1[:, 2], q=dq1,
               d=np.zeros_like(ds["q"]))
    return s1, ds1, dW


def objectives(s_final: Dict[str, np.ndarray], wall_total: float, n_steps: int, dt: float):
    """J1 = mean particle charge, J2 = wall charge received per unit time."""
    return np.array([s_final["q"].mean(), wall_total / (n_steps * dt)])


def gradient_tangent(g: Geo, U, s0: Dict[str, np.ndarray], prm: dict, n_steps: int):
    """J and dJ/dtheta ([2, 3]) by forward-mode differentiation along a recorded run."""
    from .tribo_oracle import Stats
    n = s0["x"].shape[0]
    records: List[dict] = []
    st = Stats(g.ny)
    s = {k: v.copy() for k, v in s0.items()}
    nd = 3
    ds = {k: np.zeros((nd, n)) for k in KEYS}
    dth = np.eye(3)
    dW = np.zeros((nd, 2))
    for _ in range(n_steps):
        rec = []
        step(g, U, s, prm, st, record=rec)
        records.append(rec[0])
        s, ds, dWs = step_tangent(g, U, s, ds, prm, dth, rec[0])
        dW += dWs
    J = objectives(s, st.wallq_f.sum(), n_steps, prm["dt"])
    T = n_steps * prm["dt"]
    dJ = np.stack([ds["q"].mean(1), dW.sum(1) / T])                # [2, 3]
    return J, dJ, records


def objectives_replay(g: Geo, U, s0, prm, records):
    """J of a run that replays recorded events (for central differences)."""
    from .tribo_oracle import Stats
    st = Stats(g.ny)
    s = {k: v.copy() for k, v in s0.items()}
    for rec in records:
        s = step(g, U, s, prm, st, replay=rec)
    return objectives(s, st.wallq_f.sum(), len(records), prm["dt"])


def gradient_fd(g: Geo, U, s0, prm, records, h: float = 1e-6):
    """Central differences of J over theta with the recorded events replayed."""
    names = ("k_c", "delta_u", "e")
    out = np.zeros((2, 3))
    for a, nm in enumerate(names):
        hp = h * max(1.0, abs(prm[nm]))
        pp = dict(prm, **{nm: prm[nm] + hp})
        pm = dict(prm, **{nm: prm[nm] - hp})
        out[:, a] = (objectives_replay(g, U, s0, pp, records) - objectives_replay(g, U, s0, pm, records)) / (2 * hp)
    return out
