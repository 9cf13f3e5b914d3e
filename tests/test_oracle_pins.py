"""Pins of the CPU oracle against things other than itself (CPU only).

Each test checks the oracle against a value the paper prints, a closed form,
an exact discrete identity, or a brute-force computation written differently,
so that a dropped term, wrong sign, wrong index or transposed operand in the
oracle fails at least one of them.
"""
import csv
import math
import os

import numpy as np
import pytest

import oracle as O
from paper_2602_10761_amd import workload as W

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def small_geo(nx=4, ny=5, nz=6, h=3.0, stretch=1.5):
    return O.Geo(nx, ny, nz, 4.0 * math.pi * h, 4.0 * math.pi * h / 3.0, W.y_faces(ny, h, stretch))


def zero_state(n):
    return {k: np.zeros(n) for k in O.KEYS}


BASE = dict(dt=0.1, density_ratio=1000.0, k_c=1e-3, delta_u=1.0, e=0.9, c_el=0.0,
            g=(0.0, 0.0, 0.0), un_bin=0.05)


# --------------------------------------------------------------------------
# Table 2 (Sec. 3.1): unit conversions used to build the workloads
# --------------------------------------------------------------------------
def test_table2_units():
    rows = [r for r in csv.reader(open(os.path.join(GOLDEN, "table2_particles.csv"))) if r and not r[0].startswith("#")]
    assert len(rows) == 15
    for kind, re, dum, dp, uc, st, om in rows:
        d = float(dum) * 1e-6
        assert abs(W.d_plus(d, float(re)) - float(dp)) <= 0.0051
        assert abs(W.stokes_number(d, float(uc)) - float(st)) <= 0.0051 * max(1.0, float(st))
        assert abs(W.volume_fraction_1e6(d) - float(om)) <= 0.0051
    # particle count of the paper's domain: C = 1e8 m^-3 times 12 x 2 x 4 delta^3
    assert round(1e8 * 96 * W.DELTA ** 3) == 76800


def test_derived_couplings():
    # readings: C_el from Table 1 and q_sat; k_c brackets the workload's 1e-3
    assert abs(W.electric_coupling(180.0) - 1.1316) < 1e-3
    assert abs(W.electric_coupling(550.0) / W.electric_coupling(180.0) - (550 / 180) ** 2) < 1e-12
    assert W.lumped_transfer_coefficient(180.0) < 1e-3 < W.lumped_transfer_coefficient(550.0)


# --------------------------------------------------------------------------
# Drag + gravity + integrator: Stokes settling with Schiller-Naumann
# --------------------------------------------------------------------------
def terminal_velocity(d, rr, gacc):
    """Solve v*phi_D(v d) = tau_p (1 - 1/rr) g by Newton (independent of the stepper)."""
    taup = rr * d * d / 18.0
    rhs = taup * (1.0 - 1.0 / rr) * gacc
    v = rhs
    for _ in range(100):
        re = v * d
        f = v * (1.0 + re ** (2.0 / 3.0) / 6.0) - rhs
        fp = 1.0 + re ** (2.0 / 3.0) / 6.0 + v * (2.0 / 3.0) * re ** (-1.0 / 3.0) * d / 6.0
        v -= f / fp
    return v


@pytest.mark.parametrize("rr,gacc,d", [(2.0, 320.0, 1.0), (1000.0, 0.5, 0.5), (5.0, 2000.0, 0.3)])
def test_stokes_settling(rr, gacc, d):
    g = small_geo()
    U = np.zeros((3, g.ny + 1, g.nz, g.nx))
    s = zero_state(3)
    s["d"][:] = d
    s["x"][:] = [1.0, 5.0, 9.0]
    s["y"][:] = g.ly / 2
    s["z"][:] = [0.5, 1.5, 2.5]
    prm = dict(BASE, density_ratio=rr, g=(gacc, 0.0, 0.0), dt=0.02 * rr * d * d / 18.0)
    vt = terminal_velocity(d, rr, gacc)
    assert vt * d > 1.0  # Schiller-Naumann correction matters
    for _ in range(3000):
        s = O.step(g, U, s, prm)
    np.testing.assert_allclose(s["vx"], vt, rtol=1e-12)
    assert np.all(s["vy"] == 0.0) and np.all(s["vz"] == 0.0)


def test_newton_regime_settling():
    # Re_p > 1000: C_D = 0.424, so phi_D = 0.424 Re_p / 24 and the terminal
    # velocity of the semi-implicit step, v phi_D(v d) / tau_p = (1 - 1/rr) g,
    # has the closed form v_t = sqrt(24 tau_p (1 - 1/rr) g / (0.424 d))
    g = small_geo()
    U = np.zeros((3, g.ny + 1, g.nz, g.nx))
    rr, d, gacc = 2.0, 1.0, 1.0e6
    taup = rr * d * d / 18.0
    vt = math.sqrt(24.0 * taup * (1.0 - 1.0 / rr) * gacc / (0.424 * d))
    assert vt * d > 1500.0
    s = zero_state(2)
    s["d"][:] = d
    s["x"][:] = [1.0, 5.0]
    s["y"][:] = g.ly / 2
    s["z"][:] = [0.5, 1.5]
    prm = dict(BASE, density_ratio=rr, g=(gacc, 0.0, 0.0), dt=0.02 * taup)
    for _ in range(2000):
        s = O.step(g, U, s, prm)
    np.testing.assert_allclose(s["vx"], vt, rtol=1e-12)
    assert np.all(s["vy"] == 0.0) and np.all(s["vz"] == 0.0)


def test_drag_relaxes_toward_carrier():
    # uniform carrier flow, particle at rest: velocity approaches u monotonically
    g = small_geo()
    U = np.zeros((3, g.ny + 1, g.nz, g.nx))
    U[2] = 1.5
    s = zero_state(1)
    s["d"][:] = 0.5
    s["y"][:] = g.ly / 2
    prm = dict(BASE, density_ratio=100.0)
    prev = 0.0
    for _ in range(200):
        s = O.step(g, U, s, prm)
        assert prev < s["vz"][0] < 1.5
        prev = s["vz"][0]
    assert 1.5 - prev < 1e-3


# --------------------------------------------------------------------------
# Condenser charging under repeated wall impacts: exact relaxation
# --------------------------------------------------------------------------
def closed_form_charge(n, V, kc, dU, e, q0=0.0):
    """q after n impacts with impact speeds V e^m: dU + q_n = (dU + q0) prod (1 - f_m)."""
    p = 1.0
    for m in range(n):
        p *= 1.0 - kc * (1.0 + e) ** 0.4 * (V * e ** m) ** 0.8
    return -dU + (dU + q0) * p


@pytest.mark.parametrize("e,kc,dU,q0", [(1.0, 0.02, 1.0, 0.0), (0.9, 1e-3, 1.0, 0.0),
                                        (0.7, 0.05, -0.5, 0.3), (0.95, 0.01, 2.0, -0.1)])
def test_repeated_impacts_closed_form(e, kc, dU, q0):
    g = O.Geo(2, 2, 2, 10.0, 10.0, np.array([0.0, 1.0, 2.0]))
    U = np.zeros((3, 3, 2, 2))
    n = 4
    s = zero_state(n)
    s["d"][:] = 0.2
    V = np.array([1.0, 2.5, 0.7, 3.3])
    s["vy"][:] = -V
    s["y"][:] = [0.5, 1.0, 1.5, 0.35]
    s["x"][:] = [1.0, 3.0, 6.0, 8.0]
    s["z"][:] = [1.0, 6.0, 3.0, 8.0]
    s["q"][:] = q0
    prm = dict(BASE, density_ratio=1e300, k_c=kc, delta_u=dU, e=e, dt=0.01)
    st = O.Stats(g.ny)
    hits = np.zeros(n, dtype=int)
    q_start = s["q"].sum()
    for _ in range(1500):
        rec = []
        s = O.step(g, U, s, prm, st, record=rec)
        hits += rec[0]["wall"] >= 0
        for p in range(n):
            np.testing.assert_allclose(s["q"][p], closed_form_charge(hits[p], V[p], kc, dU, e, q0),
                                       rtol=1e-12, atol=1e-15)
        assert np.all(s["y"] >= 0.1) and np.all(s["y"] <= 1.9)
    assert hits.min() >= 2 and hits.max() >= 5
    assert st.impacts.sum() == hits.sum()
    assert st.unhist.sum() == hits.sum()
    # wall charge balances particle charge (Sec. 2.3.1: the wall receives -dq)
    assert abs((s["q"].sum() - q_start) + st.wallq_f.sum()) < 1e-13
    # speed decays by e per impact
    np.testing.assert_allclose(np.abs(s["vy"]), V * e ** hits, rtol=1e-13)


def test_hand_built_impact():
    g = O.Geo(2, 2, 2, 10.0, 10.0, np.array([0.0, 1.0, 2.0]))
    U = np.zeros((3, 3, 2, 2))
    s = zero_state(2)
    s["d"][:] = 0.2
    s["y"][:] = [0.2, 1.75]
    s["vy"][:] = [-1.5, 1.0]
    s["x"][:] = [1.0, 7.0]
    prm = dict(BASE, density_ratio=1e300, e=0.8, k_c=0.1, delta_u=1.0, dt=0.1)
    rec = []
    s1 = O.step(g, U, s, prm, record=rec)
    # lower: y1 = 0.2 - 0.15 = 0.05 < r = 0.1 -> y = 0.1 + 0.8*0.05; upper: 1.85 > 1.9? no
    assert rec[0]["wall"].tolist() == [0, -1]
    assert abs(s1["y"][0] - (0.1 + 0.8 * 0.05)) < 1e-15
    assert abs(s1["vy"][0] - 1.2) < 1e-15
    assert abs(s1["q"][0] - (-0.1 * 1.8 ** 0.4 * 1.5 ** 0.8)) < 1e-15
    rec = []
    s2 = O.step(g, U, s1, prm, record=rec)
    assert rec[0]["wall"].tolist() == [-1, 1]       # 1.85 + 0.1 = 1.95 > 1.9
    assert abs(s2["y"][1] - (1.9 - 0.8 * 0.05)) < 1e-14


# --------------------------------------------------------------------------
# Poisson: dense brute force, exact discrete identities, sign
# --------------------------------------------------------------------------
def dense_operator(g):
    """Assemble -lap_h as a dense matrix from face fluxes, cell by cell."""
    n = g.ncell
    A = np.zeros((n, n))
    idx = lambda i, j, k: (j * g.nz + k) * g.nx + i
    for j in range(g.ny):
        for k in range(g.nz):
            for i in range(g.nx):
                r = idx(i, j, k)
                V = g.dx * g.dy[j] * g.dz
                # x faces (area dy dz, distance dx), periodic
                for di in (-1, 1):
                    c = idx((i + di) % g.nx, j, k)
                    w = g.dy[j] * g.dz / g.dx
                    A[r, r] += w / V
                    A[r, c] -= w / V
                for dk in (-1, 1):
                    c = idx(i, j, (k + dk) % g.nz)
                    w = g.dy[j] * g.dx / g.dz
                    A[r, r] += w / V
                    A[r, c] -= w / V
                for dj in (-1, 1):
                    jj = j + dj
                    w_area = g.dx * g.dz
                    if 0 <= jj < g.ny:
                        dist = abs(g.yc[jj] - g.yc[j])
                        A[r, r] += w_area / dist / V
                        A[r, idx(i, jj, k)] -= w_area / dist / V
                    else:  # grounded wall face at half a cell
                        dist = 0.5 * g.dy[j]
                        A[r, r] += w_area / dist / V
    return A


@pytest.mark.parametrize("shape", [(4, 5, 6), (6, 3, 4), (5, 8, 3)])
def test_poisson_dense(shape):
    nx, ny, nz = shape
    g = small_geo(nx, ny, nz, h=2.0, stretch=2.0)
    rng = np.random.default_rng(1)
    rho = rng.standard_normal((ny, nz, nx))
    phi = O.poisson_density(g, rho)
    ref = np.linalg.solve(dense_operator(g), rho.ravel()).reshape(phi.shape)
    np.testing.assert_allclose(phi, ref, rtol=0, atol=1e-12 * np.abs(ref).max())


def test_poisson_sheet_exact():
    # x-z uniform charge in one y-cell: the discrete solution is the 1-D Green's
    # function G(y, y0) = y_<(Ly - y_>)/Ly sampled at cell centres, exactly.
    g = small_geo(8, 16, 8, h=5.0, stretch=2.0)
    for j0 in (0, 3, 9, 15):
        rho = np.zeros((g.ny, g.nz, g.nx))
        sigma = 0.7
        rho[j0] = sigma / g.dy[j0]
        phi = O.poisson_density(g, rho)
        y0 = g.yc[j0]
        G = np.where(g.yc <= y0, g.yc * (g.ly - y0), y0 * (g.ly - g.yc)) / g.ly
        np.testing.assert_allclose(phi[:, 0, 0], sigma * G, rtol=1e-12)
        assert np.ptp(phi, axis=(1, 2)).max() < 1e-12 * np.abs(phi).max()


def wall_charges(g, phi):
    """Charge drawn onto each grounded wall: flux phi_wallcell/(dy/2) times face area."""
    a = g.dx * g.dz
    lo = (phi[0] / (0.5 * g.dy[0])).sum() * a
    hi = (phi[-1] / (0.5 * g.dy[-1])).sum() * a
    return lo, hi


def test_gauss_law_and_point_charge():
    g = small_geo(8, 12, 6, h=4.0, stretch=2.0)
    rng = np.random.default_rng(2)
    # random charges: total wall flux equals the enclosed charge (discrete Gauss law)
    Qf = rng.standard_normal(g.ncell)
    phi = O.poisson_density(g, Qf.reshape(g.ny, g.nz, g.nx) / g.vol[:, None, None])
    lo, hi = wall_charges(g, phi)
    assert abs(lo + hi - Qf.sum()) < 1e-11 * np.abs(Qf).sum()
    # single point charge in cell j0: the lower wall carries Q(Ly - y0)/Ly exactly
    for j0 in (0, 4, 11):
        Q = np.zeros(g.ncell, dtype=np.int64)
        Q[O.cell_index(g, 3, j0, 2)] = 1 << O.FIX_DEP
        phi = O.poisson(g, Q)
        lo, hi = wall_charges(g, phi)
        y0 = g.yc[j0]
        assert abs(lo - (g.ly - y0) / g.ly) < 1e-12
        assert abs(hi - y0 / g.ly) < 1e-12
        assert phi.min() > 0.0  # positive charge, grounded walls: phi > 0 inside


def test_efield_identities():
    g = small_geo(16, 10, 12, h=3.0, stretch=2.0)
    X = (np.arange(g.nx) * g.dx)[None, None, :]
    Z = (np.arange(g.nz) * g.dz)[None, :, None]
    kx = 2 * math.pi * 3 / g.lx
    kz = 2 * math.pi * 2 / g.lz
    phi = np.cos(kx * X) * np.cos(kz * Z) * np.ones((g.ny, 1, 1))
    Ex, Ey, Ez = O.efield(g, phi)
    np.testing.assert_allclose(Ex, np.sin(kx * X) * math.sin(kx * g.dx) / g.dx * np.cos(kz * Z) * np.ones((g.ny, 1, 1)), atol=1e-13)
    np.testing.assert_allclose(Ez, np.cos(kx * X) * np.sin(kz * Z) * math.sin(kz * g.dz) / g.dz * np.ones((g.ny, 1, 1)), atol=1e-13)
    # y: exact for a linear potential in the interior cells
    phi = (2.0 + 0.3 * g.yc)[:, None, None] * np.ones((1, g.nz, g.nx))
    Ex, Ey, Ez = O.efield(g, phi)
    np.testing.assert_allclose(Ey[1:-1], -0.3, rtol=1e-12)
    # image charge: a charge in the wall cell is pulled toward that wall
    for j0, sign in ((0, -1.0), (g.ny - 1, 1.0)):
        Q = np.zeros(g.ncell, dtype=np.int64)
        c = O.cell_index(g, 5, j0, 7)
        Q[c] = 3 << 40
        Ex, Ey, Ez = O.efield(g, O.poisson(g, Q))
        assert sign * Ey.ravel()[c] > 0.0
        assert abs(Ex.ravel()[c]) < 1e-12 * abs(Ey.ravel()[c]) and abs(Ez.ravel()[c]) < 1e-12 * abs(Ey.ravel()[c])


# --------------------------------------------------------------------------
# Interpolation, location, deposit, Coulomb: brute force on tiny inputs
# --------------------------------------------------------------------------
def test_interp_exact_for_linear_fields():
    g = small_geo(6, 7, 5, h=2.0, stretch=2.0)
    X = (np.arange(g.nx) * g.dx)[None, None, :]
    Y = g.yf[:, None, None]
    Z = (np.arange(g.nz) * g.dz)[None, :, None]
    a, b = np.array([0.3, -1.2, 2.0]), np.array([[0.5, -0.25, 1.5], [1.0, 0.2, -0.7], [-2.0, 0.1, 0.4]])
    U = np.stack([a[c] + b[c, 0] * X + b[c, 1] * Y + b[c, 2] * Z for c in range(3)])
    rng = np.random.default_rng(3)
    n = 500
    x = rng.uniform(0, (g.nx - 1) * g.dx, n)   # avoid the periodic seam (field not periodic)
    z = rng.uniform(0, (g.nz - 1) * g.dz, n)
    y = rng.uniform(0, g.ly, n)
    i, j, k = O.locate(g, x, y, z)
    u = O.interp(g, U, x, y, z, i, j, k)
    for c in range(3):
        np.testing.assert_allclose(u[c], a[c] + b[c, 0] * x + b[c, 1] * y + b[c, 2] * z, rtol=1e-12, atol=1e-12)


def test_locate_brute_force():
    g = small_geo(6, 9, 5, h=2.0, stretch=2.0)
    rng = np.random.default_rng(4)
    n = 2000
    x, y, z = rng.uniform(0, g.lx, n), rng.uniform(0, g.ly, n), rng.uniform(0, g.lz, n)
    y[:9] = g.yf[:9]            # exactly on faces: belongs to the cell above
    i, j, k = O.locate(g, x, y, z)
    for p in range(n):
        jj = max(jj for jj in range(g.ny) if g.yf[jj] <= y[p])
        assert j[p] == jj
        assert i[p] * g.dx <= x[p] < (i[p] + 1) * g.dx + 1e-12
        assert k[p] * g.dz <= z[p] < (k[p] + 1) * g.dz + 1e-12


def test_deposit_exact():
    g = small_geo(3, 4, 2)
    rng = np.random.default_rng(5)
    n = 300
    q = rng.uniform(-1, 1, n)
    cid = rng.integers(0, g.ncell, n)
    Q = O.deposit(g, q, cid)
    for c in range(g.ncell):
        assert Q[c] == sum(int(round(v * 2 ** 48)) for v in q[cid == c])
    assert Q.sum() == O.fixed(q, 48).sum()


def test_coulomb_brute_force():
    rng = np.random.default_rng(6)
    n = 40
    x, y, z = rng.uniform(0, 2, n), rng.uniform(0, 2, n), rng.uniform(0, 2, n)
    q = rng.uniform(-1, 1, n)
    cid = (x > 1).astype(int) + 2 * (y > 1) + 4 * (z > 1)
    S = O.coulomb_sums(x, y, z, q, cid)
    for a in range(n):
        acc = np.zeros(3)
        for b in range(n):
            if b != a and cid[a] == cid[b]:
                r = np.array([x[a] - x[b], y[a] - y[b], z[a] - z[b]])
                acc += q[b] * r / np.linalg.norm(r) ** 3
        np.testing.assert_allclose([S[0][a], S[1][a], S[2][a]], acc, rtol=1e-13, atol=1e-13)


def test_coulomb_pair_repels_like_charges():
    # two like charges alone in one cell, no flow, no mesh field contribution
    # beyond the symmetric part: the pair pushes apart along the separation
    g = O.Geo(2, 2, 2, 40.0, 40.0, np.array([0.0, 10.0, 20.0]))
    U = np.zeros((3, 3, 2, 2))
    s = zero_state(2)
    s["d"][:] = 0.5
    s["x"][:] = [5.0, 5.2]
    s["y"][:] = [15.0, 15.0]
    s["z"][:] = [5.0, 5.0]
    s["q"][:] = 0.5
    prm = dict(BASE, density_ratio=1e300, c_el=1e300)
    want = {}
    O.step(g, U, s, prm, want=want)
    sx = want["coul"][0]
    assert sx[0] < 0 < sx[1]
    np.testing.assert_allclose(abs(sx[0]), 0.5 / 0.2 ** 2, rtol=1e-12)


# --------------------------------------------------------------------------
# Electric acceleration (Sec. 2.2, hybrid scheme): the velocity a charged
# particle gains in one step from rest in still fluid, u = g = 0.  With
# Re_p = 0 the drag factor is 1 and the semi-implicit update gives
# v1 = dt a / (1 + dt / tau_p), tau_p = rho_r d^2 / 18, so the specific
# electric force a is read back from v1 and compared with Coulomb's and
# Gauss' laws evaluated here by hand.  In normalised units (eps = 1) the
# specific force of a field E on a particle of charge q and diameter d is
# c_el q E / d^3 (the particle mass grows as d^3).
# --------------------------------------------------------------------------
def _accel_from_v1(v1, d, dt, rr):
    return v1 * (1.0 + dt * 18.0 / (rr * d * d)) / dt


@pytest.mark.parametrize("q1,q2", [(0.3, 0.5), (0.4, -0.7), (-0.2, -0.6)])
def test_coulomb_pair_acceleration(q1, q2):
    # a y-centred cell of a wall-symmetric mesh (ny odd, faces mirror about
    # the centre plane): the charge of the cell is mirror-symmetric about its
    # centre in x, y and z, so the Gauss (mesh) field at the cell vanishes and
    # only the pair's Coulomb force remains
    g = small_geo(5, 7, 3, h=4.0, stretch=2.0)
    jc = g.ny // 2
    assert abs(g.yc[jc] - 0.5 * g.ly) < 1e-12 * g.ly
    xc, zc = (2 + 0.5) * g.dx, (1 + 0.5) * g.dz
    s = zero_state(2)
    s["x"][:] = [xc - 0.11 * g.dx, xc + 0.23 * g.dx]
    s["y"][:] = [g.yc[jc] + 0.17 * g.dy[jc], g.yc[jc] - 0.05 * g.dy[jc]]
    s["z"][:] = [zc + 0.2 * g.dz, zc - 0.09 * g.dz]
    s["q"][:] = [q1, q2]
    s["d"][:] = [1.0, 0.5]
    U = np.zeros((3, g.ny + 1, g.nz, g.nx))
    prm = dict(BASE, dt=0.05, density_ratio=800.0, c_el=2.5)
    want = {}
    out = O.step(g, U, s, prm, want=want)
    assert len(set(want["cid"].tolist())) == 1
    # Coulomb's law between the two, eps = 1: force on particle a from b is
    # q_a q_b / (4 pi r^2) along the unit vector from b to a (repulsive for
    # like charges)
    pos = np.stack([s["x"], s["y"], s["z"]], axis=1)
    for a, b in ((0, 1), (1, 0)):
        sep = pos[a] - pos[b]
        r = math.sqrt(float(sep @ sep))
        force = s["q"][a] * s["q"][b] / (4.0 * math.pi * r * r) * (sep / r)
        expect = prm["c_el"] * force / s["d"][a] ** 3
        got = np.array([_accel_from_v1(out[k][a], s["d"][a], prm["dt"], prm["density_ratio"])
                        for k in ("vx", "vy", "vz")])
        np.testing.assert_allclose(got, expect, rtol=1e-11, atol=1e-13 * np.abs(expect).max())
        # direction: away from the partner for like charges, toward it otherwise
        assert np.sign(got @ sep) == np.sign(s["q"][a] * s["q"][b])


@pytest.mark.parametrize("j0,q", [(0, 0.6), (0, -0.3), (4, 0.45), (4, -0.8)])
def test_lone_charge_pulled_to_grounded_wall(j0, q):
    # one charged particle in a wall cell, nothing else: its only force is the
    # Gauss part, E of its own cell from the potential of a charge q/V in that
    # cell between grounded walls.  The potential comes from the dense
    # face-by-face operator (not the oracle's transform solver); the cell
    # gradient takes face values interpolated linearly between cell centres
    # and phi = 0 on the wall faces.
    g = small_geo(4, 5, 6, h=2.0, stretch=2.0)
    i0, k0 = 1, 4
    s = zero_state(1)
    s["x"][:] = (i0 + 0.37) * g.dx
    s["z"][:] = (k0 + 0.61) * g.dz
    s["y"][:] = g.yf[j0] + 0.55 * g.dy[j0]
    s["q"][:] = q
    s["d"][:] = 0.02
    U = np.zeros((3, g.ny + 1, g.nz, g.nx))
    prm = dict(BASE, dt=1e-3, density_ratio=500.0, c_el=0.7)
    out = O.step(g, U, s, prm)
    rho = np.zeros((g.ny, g.nz, g.nx))
    qfix = float(np.rint(q * 2.0 ** 48)) * 2.0 ** -48      # the deposit's fixed-point charge
    rho[j0, k0, i0] = qfix / g.vol[j0]
    phi = np.linalg.solve(dense_operator(g), rho.ravel()).reshape(rho.shape)
    col = phi[:, k0, i0]
    def face(f):  # potential on y face f
        if f == 0 or f == g.ny:
            return 0.0
        w = (g.yf[f] - g.yc[f - 1]) / (g.yc[f] - g.yc[f - 1])
        return col[f - 1] + w * (col[f] - col[f - 1])
    Ey = -(face(j0 + 1) - face(j0)) / g.dy[j0]
    ay = prm["c_el"] * q * Ey / s["d"][0] ** 3
    got = [_accel_from_v1(out[k][0], s["d"][0], prm["dt"], prm["density_ratio"]) for k in ("vx", "vy", "vz")]
    np.testing.assert_allclose(got[1], ay, rtol=1e-10)
    # attraction by the image charge: toward the nearer wall whatever the sign
    toward = -1.0 if j0 == 0 else 1.0
    assert toward * got[1] > 0.0
    # the cell's charge is mirror-symmetric in x and z: no periodic-direction force
    assert abs(got[0]) < 1e-10 * abs(got[1]) and abs(got[2]) < 1e-10 * abs(got[1])


# --------------------------------------------------------------------------
# Whole-step invariants on a synthetic channel
# --------------------------------------------------------------------------
def test_profile_statistics_by_hand():
    # Sec. 4.1 profiles over the wall-normal grid rows: particles at rest in
    # still fluid without forces keep their rows and charges, so after n
    # steps the time-summed count and charge (2^-32 units) of a row are n
    # times its population and charge, and the latest charge (2^-48 units)
    # is the row's charge once; dyadic charges make every sum exact
    g = small_geo(ny=6)
    U = np.zeros((3, g.ny + 1, g.nz, g.nx))
    rows = [0, 2, 2, 3, 3, 3, 5]
    qs = [0.5, -0.25, 0.125, 1.0, -0.75, 0.0625, -1.5]
    s = zero_state(len(rows))
    s["d"][:] = 0.2
    for p, (j, q) in enumerate(zip(rows, qs)):
        s["x"][p] = (p + 0.5) * g.lx / (len(rows) + 1)
        s["y"][p] = 0.5 * (g.yf[j] + g.yf[j + 1])
        s["z"][p] = 0.3 * g.lz
        s["q"][p] = q
    n = 7
    st = O.Stats(g.ny)
    for _ in range(n):
        s = O.step(g, U, s, dict(BASE, k_c=0.0), st)
    want_c = [0] * g.ny
    want_q32 = [0] * g.ny
    want_q48 = [0] * g.ny
    for j, q in zip(rows, qs):
        want_c[j] += n
        want_q32[j] += n * int(q * 2 ** 32)
        want_q48[j] += int(q * 2 ** 48)
    assert st.crel_y.tolist() == want_c
    assert st.qcum_y.tolist() == want_q32
    assert st.qnow_y.tolist() == want_q48
    assert st.steps == n and st.flags == 0


def test_channel_invariants():
    ens = W.make_ensemble(W.CONFIGS[1].replace(n_particles=3000, precharge=0.01, v_jitter=3.0,
                                               density_ratio=100.0))
    g = O.Geo.from_mesh(ens.mesh)
    s = O.state_of(ens)
    prm = dict(ens.params, k_c=0.05)
    st = O.Stats(g.ny)
    q0 = s["q"].sum()
    for _ in range(60):
        s = O.step(g, ens.U, s, prm, st)
    assert st.impacts.sum() > 0
    assert st.flags == 0
    assert abs(s["q"].sum() - q0 + st.wallq_f.sum()) < 1e-12
    assert st.crel_y.sum() == 60 * 3000
    r = 0.5 * s["d"]
    assert np.all((s["y"] >= r) & (s["y"] <= g.ly - r))
    assert np.all((s["x"] >= 0) & (s["x"] <= g.lx) & (s["z"] >= 0) & (s["z"] <= g.lz))


# --------------------------------------------------------------------------
# 2-way coupling source (Sec. 2.1): momentum balance with the particles
# --------------------------------------------------------------------------
def test_two_way_source_balances_particle_momentum():
    # without gravity and electric forces the particles' momentum change over
    # a step is their drag impulse, which the fluid receives with the opposite
    # sign in the particles' cells of x^n: per cell, F_s V = -sum m_p dv / dt
    ens = W.make_ensemble(W.CONFIGS[1].replace(n_particles=2000, v_jitter=3.0, density_ratio=100.0,
                                               nx=8, ny=10, nz=6))
    g = O.Geo.from_mesh(ens.mesh)
    s = O.state_of(ens)
    prm = dict(ens.params, c_el=0.0, g=(0.0, 0.0, 0.0))
    want = {}
    s1 = O.step(g, ens.U, s, prm, want=want)
    dt, rr = prm["dt"], prm["density_ratio"]
    mp = rr * math.pi / 6.0 * s["d"] ** 3
    i, j, k = O.locate(g, s["x"], s["y"], s["z"])
    cell = (j * g.nz + k) * g.nx + i
    # wall impacts flip v_y after the drag: use the velocity before the rebound
    hit = want["wall"] >= 0
    vy1 = np.where(hit, -s1["vy"] / prm["e"], s1["vy"])
    for c, (a, b) in enumerate((("vx", s1["vx"]), ("vy", vy1), ("vz", s1["vz"]))):
        ref = np.zeros(g.ncell)
        np.add.at(ref, cell, -mp * (b - s[a]) / dt)
        vol = np.repeat(g.vol, g.nz * g.nx)
        got = want["fs"][c] * vol
        scale = np.abs(ref).max()
        assert scale > 0
        np.testing.assert_allclose(got, ref, rtol=0, atol=1e-10 * scale)
    # cells without particles receive nothing
    empty = np.setdiff1d(np.arange(g.ncell), cell)
    assert np.all(want["fs"][:, empty] == 0.0)


def test_two_way_source_single_particle_stokes():
    # one particle at rest in a uniform stream, Re_p -> 0 (phi_D -> 1): the
    # fluid loses 3 pi d u / (1 + dt / tau_p) per unit time (Stokes drag with
    # the implicit update) in the particle's cell only
    g = small_geo()
    U = np.zeros((3, g.ny + 1, g.nz, g.nx))
    u0 = 1e-7
    U[0] = u0
    s = zero_state(1)
    d = 0.5
    s["d"][:] = d
    s["x"][:], s["y"][:], s["z"][:] = 1.3, g.ly / 2, 2.1
    prm = dict(BASE, density_ratio=50.0)
    want = {}
    O.step(g, U, s, prm, want=want)
    taup = 50.0 * d * d / 18.0
    i, j, k = O.locate(g, s["x"], s["y"], s["z"])
    c = int(((j * g.nz + k) * g.nx + i)[0])
    expect = -(3.0 * math.pi * d * u0) / (1.0 + prm["dt"] / taup) / g.vol[j[0]]
    assert want["fs"][0, c] == pytest.approx(expect, rel=1e-4)  # phi_D - 1 ~ Re_p^(2/3) / 6 ~ 1e-6
    fs = want["fs"].copy()
    fs[0, c] = 0.0
    assert np.all(fs == 0.0)


# --------------------------------------------------------------------------
# 4-way coupling (Sec. 2.2, 2.3.1): particle-particle collisions
# --------------------------------------------------------------------------
def _pair(p1, p2, v1, v2, q=(0.0, 0.0), d=(1.0, 1.0)):
    arr = lambda a, b: np.array([a, b], dtype=np.float64)
    cid = np.array([0, 0])
    return (cid, arr(p1[0], p2[0]), arr(p1[1], p2[1]), arr(p1[2], p2[2]), arr(v1[0], v2[0]), arr(v1[1], v2[1]),
            arr(v1[2], v2[2]), arr(*q), arr(*d))


def test_pp_head_on_equal_spheres_swap_velocities():
    args = _pair((0.0, 0.0, 0.0), (0.9, 0.0, 0.0), (1.0, 0.2, 0.0), (-0.5, 0.2, 0.1), q=(0.3, -0.1))
    dvx, dvy, dvz, dq, npairs = O.collide_pp(*args, k_pp=0.5)
    assert npairs == 1
    np.testing.assert_allclose(args[4] + dvx, [-0.5, 1.0], rtol=0, atol=1e-15)  # normal components swap
    assert np.all(dvy == 0.0) and np.all(dvz == 0.0)                            # tangential unchanged
    # equal capacities: the charges relax toward their mean by 1 - exp(-x)
    x = 0.5 * 1.0 ** 4 * 2.0 ** -0.6 * 2.0 ** -0.8 * math.sqrt(1.5 ** 2 + 0.0 + 0.1 ** 2) ** 0.6
    expect = 0.5 * (-0.1 - 0.3) * (1.0 - math.exp(-x))
    np.testing.assert_allclose(dq, [expect, -expect], rtol=1e-14)


@pytest.mark.parametrize("seed", [0, 1, 2, 3])
def test_pp_conserves_momentum_energy_charge(seed):
    rng = np.random.default_rng(seed)
    d = rng.uniform(0.3, 2.0, 2)
    u = rng.normal(size=3)
    u /= np.linalg.norm(u)
    r = 0.5 * (d[0] + d[1]) * rng.uniform(0.3, 0.99)
    v1, v2 = rng.normal(size=3), rng.normal(size=3)
    if np.dot(v1 - v2, u) >= 0:  # make the pair approach along u (s1 - s2 = r u)
        v1, v2 = v2, v1
    args = _pair(tuple(r * u), (0.0, 0.0, 0.0), tuple(v1), tuple(v2), q=tuple(rng.normal(size=2)), d=tuple(d))
    dvx, dvy, dvz, dq, npairs = O.collide_pp(*args, k_pp=rng.uniform(0.1, 3.0))
    assert npairs == 1
    m = d ** 3
    vb = np.stack([args[4], args[5], args[6]])
    va = vb + np.stack([dvx, dvy, dvz])
    np.testing.assert_allclose(va @ m, vb @ m, atol=1e-14 * np.abs(vb).max() * m.sum())
    ke = lambda v: float(np.sum(m * np.sum(v * v, axis=0)))
    assert ke(va) == pytest.approx(ke(vb), rel=1e-13)
    # the pair separates afterwards, and charge is conserved
    assert np.dot(va[:, 0] - va[:, 1], u) > 0
    assert abs(dq.sum()) <= 1e-16 * max(1.0, np.abs(args[7]).max())
    # larger capacity (diameter) ends with the larger share: q/d moves toward equality
    qa = args[7] + dq
    gap0, gap1 = args[7][0] / d[0] - args[7][1] / d[1], qa[0] / d[0] - qa[1] / d[1]
    assert abs(gap1) < abs(gap0) and gap1 * gap0 >= 0


def test_pp_no_collision_when_apart_or_receding():
    apart = _pair((0.0, 0.0, 0.0), (1.01, 0.0, 0.0), (1.0, 0, 0), (-1.0, 0, 0))
    recede = _pair((0.0, 0.0, 0.0), (0.5, 0.0, 0.0), (-1.0, 0, 0), (1.0, 0, 0))
    for a in (apart, recede):
        dvx, dvy, dvz, dq, npairs = O.collide_pp(*a, k_pp=1.0)
        assert npairs == 0 and not np.any(dvx) and not np.any(dq)
    other_cell = list(_pair((0.0, 0.0, 0.0), (0.5, 0.0, 0.0), (1.0, 0, 0), (-1.0, 0, 0)))
    other_cell[0] = np.array([0, 1])
    assert O.collide_pp(*other_cell, k_pp=1.0)[4] == 0


def test_pp_repeated_exchange_closed_form():
    # equal diameters: each collision multiplies the charge difference by exp(-x_m)
    q = np.array([0.7, -0.2])
    prod = 1.0
    for m, speed in enumerate((0.5, 1.3, 2.0, 0.1)):
        args = list(_pair((0.0, 0.0, 0.0), (0.8, 0.0, 0.0), (speed, 0, 0), (0.0, 0, 0), q=tuple(q)))
        *_, dq, npairs = O.collide_pp(*args, k_pp=0.8)
        assert npairs == 1
        q = q + dq
        prod *= math.exp(-0.8 * 2.0 ** -0.6 * 2.0 ** -0.8 * speed ** 0.6)
    assert q[0] - q[1] == pytest.approx(0.9 * prod, rel=1e-13)
    assert q.sum() == pytest.approx(0.5, abs=1e-15)


def test_pp_pairs_brute_force_count():
    # the grouped pair search finds exactly the overlapping, approaching
    # same-cell pairs of an all-pairs scan
    rng = np.random.default_rng(5)
    n = 300
    cid = rng.integers(0, 20, n)
    x, y, z = rng.uniform(0, 3, (3, n))
    v = rng.normal(size=(3, n))
    q = rng.normal(size=n)
    d = rng.uniform(0.2, 1.2, n)
    *_, npairs = O.collide_pp(cid, x, y, z, v[0], v[1], v[2], q, d, k_pp=1.0)
    brute = 0
    for i in range(n):
        for j in range(n):
            if i < j and cid[i] == cid[j]:
                r = np.array([x[i] - x[j], y[i] - y[j], z[i] - z[j]])
                if 0 < r @ r < (0.5 * (d[i] + d[j])) ** 2 and (v[:, i] - v[:, j]) @ r < 0:
                    brute += 1
    assert npairs == brute > 10


def test_pp_in_step_conserves_charge():
    # a tiny dense channel where particles collide every step: particle-particle
    # exchange moves charge between particles only
    ens = W.make_ensemble(W.CONFIGS[1].replace(re_tau=2.0, nx=4, ny=4, nz=4, n_particles=800, precharge=0.3,
                                               v_jitter=1.0, d_choices=(0.5, 1.0), density_ratio=50.0))
    g = O.Geo.from_mesh(ens.mesh)
    s = O.state_of(ens)
    prm = dict(ens.params, pp=1, k_pp=2.0, k_c=0.0)
    st = O.Stats(g.ny)
    q0 = s["q"].sum()
    for _ in range(5):
        s = O.step(g, ens.U, s, prm, st)
    assert st.pp_pairs > 20
    assert s["q"].sum() == pytest.approx(q0, abs=1e-12)


def test_pp_exponent_is_the_hertz_condenser_chain():
    # Delta t_12 / T_12 from the paper's chain (Hertz contact radius alpha_12,
    # contact area A_12, contact time, relaxation time T_12 with capacities
    # 4 pi eps d / 2) for arbitrary material constants: one coefficient k_pp
    # fitted at one (d_i, d_j, |u_12|) reproduces every other case
    rho_p, k_e, mu_p, e_p, phi_p, eps = 1.3e3, 0.9, 0.3, 2.1e4, 7.0, 0.8

    def chain(di, dj, u):
        a = (di * dj / 2.0) * ((5.0 / 8.0) * math.pi * rho_p * (1 + k_e) * u * u * math.sqrt(di + dj)
                               / (di ** 3 + dj ** 3) * (1 - mu_p) / e_p) ** 0.4
        area = math.pi * di * dj * a / (2.0 * (di + dj))
        dt12 = 2.94 * a / u
        ci, cj = 4 * math.pi * eps * di / 2, 4 * math.pi * eps * dj / 2
        t12 = ci * cj / (ci + cj) * (di + dj) / (2 * area) * phi_p
        return dt12 / t12

    k_pp = chain(0.5, 1.0, 1.0) / O.pp_transfer_exponent(0.5, 1.0, 1.0, 1.0)
    for di, dj, u in ((0.25, 0.25, 0.3), (2.0, 0.5, 4.0), (1.0, 1.0, 0.01), (0.7, 1.9, 12.0)):
        assert O.pp_transfer_exponent(di, dj, u, k_pp) == pytest.approx(chain(di, dj, u), rel=1e-12)


# --------------------------------------------------------------------------
# Stochastic scaling model (Sec. 2.3.2) and its random numbers
# --------------------------------------------------------------------------
def test_philox_known_answers():
    for line in open(os.path.join(GOLDEN, "philox4x32_10_kat.txt")):
        if line.startswith("#") or not line.strip():
            continue
        ctr, key, out = (list(map(lambda h: int(h, 16), part.split())) for part in line.split("|"))
        got = O.philox4x32(*ctr, *key)
        assert [int(v) for v in got] == out


def _moments(x):
    m = x.mean()
    s = x.std()
    return m, s, np.mean(((x - m) / s) ** 3)


def test_impact_normals_are_standard():
    ids = np.arange(200_000)
    n0, n1 = O.impact_normals(ids, 7, 12345)
    for v in (n0, n1):
        m, s, g = _moments(v)
        assert abs(m) < 0.01 and abs(s - 1) < 0.01 and abs(g) < 0.03
    assert abs(np.corrcoef(n0, n1)[0, 1]) < 0.01
    # counter-based: the same (id, step, seed) gives the same numbers, another step others
    a, _ = O.impact_normals(ids[:10], 7, 12345)
    b, _ = O.impact_normals(ids[:10], 8, 12345)
    np.testing.assert_array_equal(a, n0[:10])
    assert not np.any(a == b)


@pytest.mark.parametrize("mu,sigma,gamma", [(0.0, 1.0, 0.0), (2.0, 0.5, 0.8), (-1.0, 3.0, -0.5)])
def test_skew_normal_moments(mu, sigma, gamma):
    n0, n1 = O.impact_normals(np.arange(400_000), 3, 99)
    x = O.skew_normal(mu, sigma, gamma, n0, n1)
    m, s, g = _moments(x)
    assert m == pytest.approx(mu, abs=0.01 * sigma)
    assert s == pytest.approx(sigma, rel=0.01)
    assert g == pytest.approx(gamma, abs=0.03)


SSM = dict(charging=1, ssm_dq0min=-2e-3, ssm_mu0=-1.5e-3, ssm_sigma0=4e-4, ssm_gamma0=0.6, ssm_csat=20.0,
           ssm_d0=0.5, ssm_un0=1.0, seed=2024)


def test_ssm_reproduces_reference_impact():
    # d = d_0, u_n = u_n0, q = 0: the impact charge has the reference
    # experiment's mean, standard deviation and skewness
    n = 400_000
    prm = dict(SSM)
    dq = O.ssm_wall_charge(np.zeros(n), np.full(n, 0.5), np.full(n, 1.0), np.arange(n), 5, prm)
    m, s, g = _moments(dq)
    assert m == pytest.approx(prm["ssm_mu0"], rel=0.01)
    assert s == pytest.approx(prm["ssm_sigma0"], rel=0.01)
    assert g == pytest.approx(prm["ssm_gamma0"], abs=0.03)


def test_ssm_deterministic_limit_is_the_condenser_model():
    # sigma_0 = gamma_0 = 0, mu_0 = dq0min: the SSM impact charge
    # dq0min (u_n/u_n0)^(4/5) (1 + q/dU) equals the condenser model's
    # -k_c (1 + e)^(2/5) u_n^(4/5) (dU + q) for monodisperse particles with
    # d_0 = d, dq0min = -k_c (1 + e)^(2/5) dU u_n0^(4/5), c_sat = 4 dU / d^2
    # (while 0 <= 1 + q/dU <= 1)
    ens = W.make_ensemble(W.CONFIGS[1].replace(re_tau=20.0, n_particles=3000, v_jitter=4.0, precharge=0.0,
                                               density_ratio=30.0, nx=16, ny=16, nz=16))
    g = O.Geo.from_mesh(ens.mesh)
    base = dict(ens.params, k_c=0.02)
    kc, e, dU, d = base["k_c"], base["e"], base["delta_u"], 0.5
    un0 = 0.7
    ssm = dict(base, charging=1, ssm_sigma0=0.0, ssm_gamma0=0.0, ssm_d0=d, ssm_un0=un0,
               ssm_dq0min=-kc * (1 + e) ** 0.4 * dU * un0 ** 0.8, ssm_csat=4.0 * dU / d ** 2, seed=1)
    ssm["ssm_mu0"] = ssm["ssm_dq0min"]
    sa, sb = O.state_of(ens), O.state_of(ens)
    sta, stb = O.Stats(g.ny), O.Stats(g.ny)
    for _ in range(40):
        sa = O.step(g, ens.U, sa, base, sta)
        sb = O.step(g, ens.U, sb, ssm, stb)
    assert sta.impacts.sum() > 40
    np.testing.assert_array_equal(sta.impacts, stb.impacts)
    np.testing.assert_allclose(sb["q"], sa["q"], rtol=1e-12, atol=1e-15)
    assert np.all(sa["q"] <= 0) and np.all(sa["q"] >= -dU)
    # the SSM path was taken: another reference impact speed changes the charges
    sc, stc = O.state_of(ens), O.Stats(g.ny)
    for _ in range(40):
        sc = O.step(g, ens.U, sc, dict(ssm, ssm_un0=2.0 * un0), stc)
    assert np.abs(sc["q"] - sa["q"]).max() > 1e-6
