"""Plain, slow, obviously-correct FP64 reference of one Lagrangian particle step.

TEST INFRASTRUCTURE ONLY (see the package header): the HIP library never
imports this module, and this module imports nothing from the HIP side.

What it computes, following Sec. 2.2-2.3 of Wilms & Grosshans (triboFoam),
in wall units (nu = u_tau = 1, h = Re_tau), charge in units of q_sat:

  * particle equation of motion, Eq. (2.5): du_p/dt = f_ad + f_g + f_el
    (particle-particle collisions are not part of this step),
  * drag, Eq. (2.6)-(2.7) (Schiller-Naumann), read as
    f_ad = -(u_p - u) C_D Re_p / (24 tau_p),  tau_p = rho_r d^2 / 18,
  * gravity/buoyancy f_g = (1 - rho/rho_p) g (Sec. 2.2),
  * hybrid electrostatics (Sec. 2.2): Coulomb's law, Eq. (2.8), between
    particles sharing a grid cell, plus Gauss' law through the Poisson
    equation lap(phi) = -rho_el/eps with the cell charge equal to the sum of
    the charges in it, E = -grad(phi), f = q E / m_p, Eq. (2.9),
  * grounded conducting walls (phi = 0) and periodic x, z (Sec. 3.1, 4.2),
  * hard-sphere wall rebound, wall-normal velocity flipped (Sec. 2.2), scaled
    by the restitution coefficient e,
  * condenser-model particle-wall charge transfer (Sec. 2.3.1, Eq. (2.13)-
    (2.19)) in the lumped normalised form dq = -f (dU + q),
    f = k_c (1 + e)^(2/5) u_n^(4/5),
  * grid-cell histograms of concentration and charge (Sec. 4.1).

Discretisation (second order finite volumes, Sec. 3.1): NGP charge
deposit onto cells, 5-point (per direction 3-point) FV Laplacian on the
tanh-stretched wall-normal grid with Dirichlet walls, Gauss-linear cell
gradient, trilinear carrier-velocity interpolation, semi-implicit Euler.
The Poisson equation is solved exactly (up to rounding) by a Fourier
transform in the periodic directions followed by one tridiagonal (Thomas)
solve per Fourier mode in y; numpy's FFT is the library primitive.

Events (cell of each particle, wall impacts, periodic wraps) can be recorded
and replayed, so that derivatives with respect to the charging parameters
can be taken with the discrete events held fixed.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import Dict, Optional

import numpy as np

FIX_DEP = 48      # deposit:           Q_c = sum rne(q * 2^48)
FIX_WALL = 40     # wall charge:       sum rne(-dq * 2^40)
FIX_QCUM = 32     # time-summed charge profile: sum rne(q * 2^32)
N_UNBIN = 64      # bins of the wall-normal impact-velocity histogram
INV4PI = 1.0 / (4.0 * math.pi)
TWO_THIRDS = 2.0 / 3.0

# error flags
F_NONFINITE = 1
F_OVERFLOW = 2
F_OUTSIDE = 4


def fixed(v: np.ndarray, shift: int) -> np.ndarray:
    """Round-to-nearest-even of v * 2^shift into int64."""
    return np.rint(np.asarray(v, dtype=np.float64) * (2.0 ** shift)).astype(np.int64)


FIX_LIMIT = 2.0 ** 62   # fixed-point values must stay below this magnitude


def fixed_checked(v: np.ndarray, shift: int):
    """rne(v * 2^shift) into int64 where its magnitude stays below 2^62.

    An entry at or beyond 2^62, or not finite, contributes 0 (so that sums of
    many entries cannot wrap) and the conversion reports an overflow, which
    the step turns into the sticky F_OVERFLOW flag.  Returns (values, overflowed).
    """
    s = np.rint(np.asarray(v, dtype=np.float64) * (2.0 ** shift))
    ok = np.abs(s) < FIX_LIMIT
    return np.where(ok, s, 0.0).astype(np.int64), bool(not ok.all())


# ----------------------------------------------------------------------------
# Mesh geometry (Sec. 3.1: periodic x, z; walls at y = 0 and y = 2h)
# ----------------------------------------------------------------------------
@dataclass
class Geo:
    nx: int
    ny: int
    nz: int
    lx: float
    lz: float
    yf: np.ndarray

    def __post_init__(self):
        self.yf = np.asarray(self.yf, dtype=np.float64)
        self.ly = float(self.yf[-1])
        self.dx = self.lx / self.nx
        self.dz = self.lz / self.nz
        self.dy = self.yf[1:] - self.yf[:-1]
        self.yc = 0.5 * (self.yf[:-1] + self.yf[1:])
        self.vol = (self.dx * self.dy) * self.dz          # per y-cell [ny]
        self.ncell = self.nx * self.ny * self.nz

    @staticmethod
    def from_mesh(m) -> "Geo":
        return Geo(m.nx, m.ny, m.nz, m.lx, m.lz, m.yf)


def locate(g: Geo, x, y, z):
    """Cell (i, j, k) holding each position: floor in x, z; face search in y."""
    i = np.clip(np.floor(x / g.dx).astype(np.int64), 0, g.nx - 1)
    k = np.clip(np.floor(z / g.dz).astype(np.int64), 0, g.nz - 1)
    j = np.clip(np.searchsorted(g.yf, y, side="right") - 1, 0, g.ny - 1)
    return i, j, k


def cell_index(g: Geo, i, j, k):
    """Linear cell index, x fastest, then z, then y: c = (j*nz + k)*nx + i."""
    return (j * g.nz + k) * g.nx + i


# ----------------------------------------------------------------------------
# Deposit: integral of rho_el over a cell = sum of the charges in it (Sec. 2.2)
# ----------------------------------------------------------------------------
def deposit(g: Geo, q, cid) -> np.ndarray:
    Q = np.zeros(g.ncell, dtype=np.int64)
    np.add.at(Q, cid, fixed_checked(q, FIX_DEP)[0])
    return Q


# ----------------------------------------------------------------------------
# Poisson equation lap(phi) = -rho (eps = 1 in these units), grounded walls
# ----------------------------------------------------------------------------
def y_coefficients(g: Geo):
    """Off-diagonal FV couplings of the wall-normal operator, per y-cell.

    am[j] = 1/(dy_j * (yc_j - yc_{j-1})), ap[j] = 1/(dy_j * (yc_{j+1} - yc_j));
    at the walls the neighbour distance is the distance to the wall face
    (half a cell) and the wall value is phi = 0.
    """
    hm = np.empty(g.ny)
    hp = np.empty(g.ny)
    hm[1:] = g.yc[1:] - g.yc[:-1]
    hm[0] = g.yc[0] - g.yf[0]
    hp[:-1] = g.yc[1:] - g.yc[:-1]
    hp[-1] = g.yf[-1] - g.yc[-1]
    am = 1.0 / (g.dy * hm)
    ap = 1.0 / (g.dy * hp)
    return am, ap


def modified_wavenumbers(g: Geo):
    """Eigenvalues of the periodic 3-point second difference: (2 - 2cos(k dx))/dx^2."""
    mx = np.arange(g.nx // 2 + 1)
    mz = np.arange(g.nz)
    kx2 = (2.0 - 2.0 * np.cos(2.0 * math.pi * mx / g.nx)) / (g.dx * g.dx)
    kz2 = (2.0 - 2.0 * np.cos(2.0 * math.pi * mz / g.nz)) / (g.dz * g.dz)
    return kx2, kz2


def thomas(lower, diag, upper, rhs):
    """Tridiagonal solve along axis 0 (textbook Thomas algorithm, no pivoting)."""
    n = rhs.shape[0]
    cp = np.empty(diag.shape, dtype=np.float64)
    dp = np.empty(rhs.shape, dtype=rhs.dtype)
    cp[0] = upper[0] / diag[0]
    dp[0] = rhs[0] / diag[0]
    for j in range(1, n):
        piv = diag[j] - lower[j] * cp[j - 1]
        cp[j] = upper[j] / piv
        dp[j] = (rhs[j] - lower[j] * dp[j - 1]) / piv
    out = np.empty_like(dp)
    out[n - 1] = dp[n - 1]
    for j in range(n - 2, -1, -1):
        out[j] = dp[j] - cp[j] * out[j + 1]
    return out


def poisson_density(g: Geo, rho: np.ndarray) -> np.ndarray:
    """phi[ny, nz, nx] solving the FV form of lap(phi) = -rho, phi = 0 on walls."""
    R = np.fft.rfft(rho, axis=2)
    R = np.fft.fft(R, axis=1)                      # [ny, nz, nx/2+1]
    kx2, kz2 = modified_wavenumbers(g)
    K2 = kz2[:, None] + kx2[None, :]
    am, ap = y_coefficients(g)
    shape = (g.ny,) + K2.shape
    lower = np.broadcast_to(-am[:, None, None], shape)
    upper = np.broadcast_to(-ap[:, None, None], shape)
    diag = (am + ap)[:, None, None] + K2[None, :, :]
    P = thomas(lower, diag, upper, R)
    P = np.fft.ifft(P, axis=1)
    return np.fft.irfft(P, n=g.nx, axis=2)


def poisson(g: Geo, Q: np.ndarray) -> np.ndarray:
    """Field of the fixed-point cell charges Q (scale 2^48): rho = Q 2^-48 / V."""
    rho = (Q.reshape(g.ny, g.nz, g.nx).astype(np.float64) * (2.0 ** -FIX_DEP)) / g.vol[:, None, None]
    return poisson_density(g, rho)


def efield(g: Geo, phi: np.ndarray):
    """E = -grad(phi) at cell centres, Gauss-linear FV gradient.

    x, z (uniform, periodic): face value = mean of the two cells, giving
    -(phi_{i+1} - phi_{i-1})/(2 dx).  y: linear interpolation to the face
    between the two cell centres, phi = 0 on the wall faces.
    """
    Ex = -(np.roll(phi, -1, axis=2) - np.roll(phi, 1, axis=2)) / (2.0 * g.dx)
    Ez = -(np.roll(phi, -1, axis=1) - np.roll(phi, 1, axis=1)) / (2.0 * g.dz)
    ny = g.ny
    pf = np.zeros((ny + 1,) + phi.shape[1:])
    beta = g.dy[:-1] / (g.dy[:-1] + g.dy[1:])       # face j (1..ny-1)
    pf[1:ny] = phi[:-1] + beta[:, None, None] * (phi[1:] - phi[:-1])
    Ey = -(pf[1:] - pf[:-1]) / g.dy[:, None, None]
    return Ex, Ey, Ez


# ----------------------------------------------------------------------------
# Carrier-flow interpolation (trilinear, linear in physical y)
# ----------------------------------------------------------------------------
def interp(g: Geo, U: np.ndarray, x, y, z, i, j, k):
    tx = (x - i * g.dx) / g.dx
    ty = (y - g.yf[j]) / g.dy[j]
    tz = (z - k * g.dz) / g.dz
    i1 = (i + 1) % g.nx
    k1 = (k + 1) % g.nz
    j1 = j + 1
    out = []
    for c in range(3):
        Uc = U[c]
        c00 = Uc[j, k, i] * (1.0 - tx) + Uc[j, k, i1] * tx
        c01 = Uc[j, k1, i] * (1.0 - tx) + Uc[j, k1, i1] * tx
        c10 = Uc[j1, k, i] * (1.0 - tx) + Uc[j1, k, i1] * tx
        c11 = Uc[j1, k1, i] * (1.0 - tx) + Uc[j1, k1, i1] * tx
        c0 = c00 * (1.0 - tz) + c01 * tz
        c1 = c10 * (1.0 - tz) + c11 * tz
        out.append(c0 * (1.0 - ty) + c1 * ty)
    return out


# ----------------------------------------------------------------------------
# Near field: Coulomb's law between particles of the same cell (Eq. (2.8))
# ----------------------------------------------------------------------------
def same_cell_segments(cid):
    """Order by (cell, id) and the [start, end) of each particle's cell run."""
    n = cid.shape[0]
    order = np.lexsort((np.arange(n), cid))
    cs = cid[order]
    pos = np.arange(n)
    first = np.ones(n, dtype=bool)
    first[1:] = cs[1:] != cs[:-1]
    start = np.maximum.accumulate(np.where(first, pos, 0))
    last = np.ones(n, dtype=bool)
    last[:-1] = cs[1:] != cs[:-1]
    end = np.minimum.accumulate(np.where(last, pos + 1, n + 1)[::-1])[::-1]
    return order, start, end


def coulomb_sums(x, y, z, q, cid):
    """S_i = sum_{j in cell(i), j != i} q_j (x_i - x_j)/|x_i - x_j|^3, partners in ascending id.

    Coincident pairs (zero separation) have no defined direction and add nothing.
    """
    n = x.shape[0]
    if n == 0:
        return np.zeros(0), np.zeros(0), np.zeros(0)
    order, start, end = same_cell_segments(cid)
    xs, ys, zs, qs = x[order], y[order], z[order], q[order]
    pos = np.arange(n)
    sx = np.zeros(n)
    sy = np.zeros(n)
    sz = np.zeros(n)
    kmax = int((end - start).max())
    for m in range(kmax):
        t = start + m
        ok = (t < end) & (t != pos)
        tt = np.where(ok, t, pos)
        rx = xs - xs[tt]
        ry = ys - ys[tt]
        rz = zs - zs[tt]
        r2 = (rx * rx + ry * ry) + rz * rz
        ok &= r2 > 0.0
        r2s = np.where(ok, r2, 1.0)
        w = qs[tt] / (r2s * np.sqrt(r2s))
        sx = np.where(ok, sx + w * rx, sx)
        sy = np.where(ok, sy + w * ry, sy)
        sz = np.where(ok, sz + w * rz, sz)
    out = [np.empty(n), np.empty(n), np.empty(n)]
    for o, s in zip(out, (sx, sy, sz)):
        o[order] = s
    return out


# ----------------------------------------------------------------------------
# Statistics (Sec. 4.1: histogram bins = grid cells; charge; wall impacts)
# ----------------------------------------------------------------------------
@dataclass
class Stats:
    ny: int
    steps: int = 0
    crel_y: np.ndarray = None     # time-summed particle count per y-cell
    qcum_y: np.ndarray = None     # time-summed sum rne(q 2^32) per y-cell
    qnow_y: np.ndarray = None     # sum rne(q 2^48) per y-cell at the latest deposit
    impacts: np.ndarray = None    # [2] lower, upper
    wallq: np.ndarray = None      # [2] sum rne(-dq 2^40)
    wallq_f: np.ndarray = None    # [2] float sum of -dq (conservation checks)
    unhist: np.ndarray = None     # [N_UNBIN]
    flags: int = 0
    pp_pairs: int = 0             # colliding particle pairs (4-way coupling)

    def __post_init__(self):
        z = lambda n: np.zeros(n, dtype=np.int64)
        self.crel_y = z(self.ny) if self.crel_y is None else self.crel_y
        self.qcum_y = z(self.ny) if self.qcum_y is None else self.qcum_y
        self.qnow_y = z(self.ny) if self.qnow_y is None else self.qnow_y
        self.impacts = z(2) if self.impacts is None else self.impacts
        self.wallq = z(2) if self.wallq is None else self.wallq
        self.wallq_f = np.zeros(2) if self.wallq_f is None else self.wallq_f
        self.unhist = z(N_UNBIN) if self.unhist is None else self.unhist


def _sum_by(index, values, n):
    out = np.zeros(n, dtype=np.int64)
    np.add.at(out, index, values)
    return out


# ----------------------------------------------------------------------------
# Stochastic scaling model (SSM) of particle-wall charging (Sec. 2.3.2)
# ----------------------------------------------------------------------------
SSM_KEY1 = 0x53534D31  # second key word of the impact random numbers


def philox4x32(c0, c1, c2, c3, k0, k1, rounds: int = 10):
    """Philox4x32-10 counter-based generator (Salmon, Moraes, Dror & Shaw,
    SC'11): ten rounds of two 32x32->64 multiplications (multipliers
    0xD2511F53, 0xCD9E8D57) with the key bumped by (0x9E3779B9, 0xBB67AE85)
    between rounds.  Arguments: integer arrays (or ints) < 2^32; returns the
    four output words."""
    m = np.uint64(0xFFFFFFFF)
    x = [np.asarray(v, dtype=np.uint64) & m for v in (c0, c1, c2, c3)]
    k0, k1 = np.asarray(k0, dtype=np.uint64) & m, np.asarray(k1, dtype=np.uint64) & m
    for r in range(rounds):
        if r:
            k0 = (k0 + np.uint64(0x9E3779B9)) & m
            k1 = (k1 + np.uint64(0xBB67AE85)) & m
        p0 = np.uint64(0xD2511F53) * x[0]
        p1 = np.uint64(0xCD9E8D57) * x[2]
        x = [(p1 >> np.uint64(32)) ^ x[1] ^ k0, p1 & m, (p0 >> np.uint64(32)) ^ x[3] ^ k1, p0 & m]
    return x


def impact_normals(ids, step: int, seed: int):
    """Two standard normal numbers per impact: Philox4x32-10 at counter
    (particle id, step number, 0, 0) and key (seed, SSM_KEY1); uniforms
    u = (w + 1/2) 2^-32 of the first two words; Box-Muller."""
    w = philox4x32(ids, step, 0, 0, seed, SSM_KEY1)
    u0 = (w[0].astype(np.float64) + 0.5) * 2.0 ** -32
    u1 = (w[1].astype(np.float64) + 0.5) * 2.0 ** -32
    r = np.sqrt(-2.0 * np.log(u0))
    t = 2.0 * math.pi * u1
    return r * np.cos(t), r * np.sin(t)


def skew_normal(mu, sigma, gamma, n0, n1):
    """A skew-normal sample with mean mu, standard deviation sigma and
    skewness gamma (|gamma| limited to 0.99), by the moment relations of the
    skew-normal family: delta from gamma, omega = sigma / sqrt(1 - 2 delta^2/pi),
    xi = mu - omega delta sqrt(2/pi), Z = delta |n0| + sqrt(1 - delta^2) n1."""
    g = np.clip(gamma, -0.99, 0.99)
    r = np.cbrt(2.0 * np.abs(g) / (4.0 - math.pi))
    delta = np.sign(g) * (r / np.sqrt(1.0 + r * r)) * math.sqrt(math.pi / 2.0)
    b = math.sqrt(2.0 / math.pi)
    omega = sigma / np.sqrt(1.0 - (b * delta) ** 2)
    xi = mu - omega * b * delta
    return xi + omega * (delta * np.abs(n0) + np.sqrt(1.0 - delta * delta) * n1)


def ssm_wall_charge(q, d, un, ids, step: int, prm: dict):
    """Charge received by each impacting particle under the SSM.

    Readings: the wall's active sites give the particle their mean,
    mu_w = dq0min N_w/N_w0 (a grounded conducting wall regenerates at once);
    the particle's sites give Delta q_1 ~ G(mu_i, sigma_i, gamma_i) to the
    wall, so dq = mu_w - Delta q_1 (mean mu_0 in the reference impact);
    A/A_0 = (d/d_0)^2 (u_n/u_n0)^(4/5) from the Hertz contact area with the
    material constants cancelling; chi_w/chi_0 = 1 - sgn(dq0min) 4q/(c_sat d^2),
    chi_i/chi_0 = 1 + sgn(dq0min - mu_0) 4q/(c_sat d^2), both clipped to [0, 1];
    the site density c/c_0 = 1 (no depletion: its history term is not fully
    specified); N/N_0 = 0 leaves no particle contribution."""
    dq0, mu0 = prm["ssm_dq0min"], prm["ssm_mu0"]
    s0, g0, csat = prm["ssm_sigma0"], prm["ssm_gamma0"], prm["ssm_csat"]
    area = (d / prm["ssm_d0"]) ** 2 * (un / prm["ssm_un0"]) ** 0.8
    load = 4.0 * q / (csat * (d * d))
    chi_w = np.clip(1.0 - np.sign(dq0) * load, 0.0, 1.0)
    chi_i = np.clip(1.0 + np.sign(dq0 - mu0) * load, 0.0, 1.0)
    nw = area * chi_w
    ni = area * chi_i
    mu_w = dq0 * nw
    n0, n1 = impact_normals(ids, step, prm["seed"])
    safe = np.where(ni > 0.0, ni, 1.0)
    dq1 = skew_normal((dq0 - mu0) * ni, s0 * np.sqrt(ni), -g0 / safe, n0, n1)
    return mu_w - np.where(ni > 0.0, dq1, 0.0)


# ----------------------------------------------------------------------------
# 4-way coupling: particle-particle collisions and charge exchange
# ----------------------------------------------------------------------------
def pp_transfer_exponent(di, dj, speed, k_pp):
    """Delta t_12 / T_12 of the particle-particle condenser model (Sec. 2.3.1)
    with the Hertzian contact area and duration substituted: the material
    constants (rho_p, k_e, mu_p, E_p, phi_p, eps) collapse into one
    coefficient k_pp, leaving
    k_pp (d_i d_j)^2 (d_i + d_j)^(-3/5) (d_i^3 + d_j^3)^(-4/5) |u_12|^(3/5)."""
    return k_pp * ((di * dj) ** 2 * (di + dj) ** -0.6 * (di ** 3 + dj ** 3) ** -0.8) * speed ** 0.6


def collide_pp(cid, x, y, z, vx, vy, vz, q, d, k_pp):
    """Binary hard-sphere collisions between particles sharing a grid cell,
    resolved simultaneously on the state at the start of the step (Sec. 2.2):
    a pair collides when it overlaps, |s_i - s_j| < (d_i + d_j)/2, and
    approaches, (u_i - u_j).(s_i - s_j) < 0.  Fully elastic, masses ~ d^3:
    u_i += -2 m_j / (m_i + m_j) ((u_i - u_j).n) n, n = (s_i - s_j)/|s_i - s_j|.
    Charge exchange (condenser model, Sec. 2.3.1), capacities ~ d:
    dq_i = -dq_j = (d_i q_j - d_j q_i)/(d_i + d_j) (1 - exp(-Delta t_12/T_12)).
    Every particle's increments are summed over its partners in ascending id.
    Returns (dvx, dvy, dvz, dq, number of colliding pairs)."""
    n = x.shape[0]
    dv = np.zeros((3, n))
    dq = np.zeros(n)
    pairs = 0
    order = np.lexsort((np.arange(n), cid))
    cs = cid[order]
    bounds = np.flatnonzero(np.diff(cs)) + 1
    for grp in np.split(order, bounds):
        m = len(grp)
        for a in range(m):
            for b in range(a + 1, m):
                i, j = grp[a], grp[b]
                rx, ry, rz = x[i] - x[j], y[i] - y[j], z[i] - z[j]
                r2 = (rx * rx + ry * ry) + rz * rz
                rc = 0.5 * (d[i] + d[j])
                if not (0.0 < r2 < rc * rc):
                    continue
                wx, wy, wz = vx[i] - vx[j], vy[i] - vy[j], vz[i] - vz[j]
                if (wx * rx + wy * ry) + wz * rz >= 0.0:
                    continue
                pairs += 1
                ri = 1.0 / math.sqrt(r2)
                nx_, ny_, nz_ = rx * ri, ry * ri, rz * ri
                un = (wx * nx_ + wy * ny_) + wz * nz_
                mi, mj = (d[i] * d[i]) * d[i], (d[j] * d[j]) * d[j]
                ci, cj = 2.0 * mj / (mi + mj) * un, 2.0 * mi / (mi + mj) * un
                dv[:, i] -= (ci * nx_, ci * ny_, ci * nz_)
                dv[:, j] += (cj * nx_, cj * ny_, cj * nz_)
                speed = math.sqrt((wx * wx + wy * wy) + wz * wz)
                fr = 1.0 - math.exp(-pp_transfer_exponent(d[i], d[j], speed, k_pp))
                t = (d[i] * q[j] - d[j] * q[i]) / (d[i] + d[j]) * fr
                dq[i] += t
                dq[j] -= t
    return dv[0], dv[1], dv[2], dq, pairs


# ----------------------------------------------------------------------------
# 2-way coupling: momentum source of the carrier
# ----------------------------------------------------------------------------
def two_way_source(g: Geo, cid: np.ndarray, d: np.ndarray, sdr: np.ndarray, u, v1, rr: float) -> np.ndarray:
    """Source term F_s of the carrier momentum equation (Sec. 2.1): the
    aerodynamic forces on the particles of a grid cell, summed and fed back to
    the fluid with the opposite sign, per unit fluid mass (fluid density 1 in
    these units), i.e. divided by the cell volume.

    Reading: the force on a particle over the step is the drag of the
    semi-implicit update, f_ad = m_p (phi_D / tau_p) (u - v^{n+1}), with
    m_p = rho_r pi d^3 / 6, so that the particles' drag impulse and the
    fluid's source balance exactly; the cell is the one of x^n (where the
    particle's charge is deposited).  Returns [3][ncell] (cell index
    (j nz + k) nx + i), summed over particles in ascending id.
    """
    mp = (rr * (math.pi / 6.0)) * ((d * d) * d)
    jrow = np.repeat(np.arange(g.ny), g.nz * g.nx)  # y row of every cell
    out = np.zeros((3, g.ncell))
    for c in range(3):
        f = (mp * sdr) * (u[c] - v1[c])
        np.add.at(out[c], cid, f)
        out[c] = -out[c] / g.vol[jrow]
    return out


# ----------------------------------------------------------------------------
# One step
# ----------------------------------------------------------------------------
KEYS = ("x", "y", "z", "vx", "vy", "vz", "q", "d")


def step(g: Geo, U: np.ndarray, s: Dict[str, np.ndarray], prm: dict, stats: Optional[Stats] = None,
         replay: Optional[dict] = None, record: Optional[list] = None, want: Optional[dict] = None):
    """Advance the particle state s (arrays indexed by particle id) by one step.

    Order within the step (the paper gives none): cells of x^n -> deposit
    q^n -> Poisson -> E -> per particle (carrier u, E, same-cell Coulomb at
    x^n, q^n) -> v^{n+1}, x^{n+1} -> wall impact (reflect, charge) -> wrap.
    With prm["pp"] (4-way coupling), same-cell particle-particle collisions
    (collide_pp, coefficient prm["k_pp"]) first change v^n and q^n; the drag
    update and the wall charging start from the changed values, the electric
    forces use the deposited q^n.
    """
    x, y, z, vx, vy, vz, q, d = (s[k] for k in KEYS)
    n = x.shape[0]
    dt = prm["dt"]
    rr = prm["density_ratio"]
    kc, dU, e = prm["k_c"], prm["delta_u"], prm["e"]
    cel = prm["c_el"]
    gvec = prm.get("g", (0.0, 0.0, 0.0))
    un_bin = prm.get("un_bin", 0.05)

    if replay is not None:
        i, j, k = replay["i"], replay["j"], replay["k"]
    else:
        i, j, k = locate(g, x, y, z)
    cid = cell_index(g, i, j, k)

    # deposit q^n and its statistics (a charge beyond the fixed-point range
    # deposits nothing and raises the overflow flag)
    fq, ovf_dep = fixed_checked(q, FIX_DEP)
    Q = np.zeros(g.ncell, dtype=np.int64)
    np.add.at(Q, cid, fq)
    if stats is not None:
        q32, ovf_cum = fixed_checked(q, FIX_QCUM)
        stats.crel_y += np.bincount(j, minlength=g.ny).astype(np.int64)
        stats.qcum_y += _sum_by(j, q32, g.ny)
        stats.qnow_y = _sum_by(j, fq, g.ny)
        if ovf_dep or ovf_cum:
            stats.flags |= F_OVERFLOW

    # 4-way coupling: collisions act on the velocities and charges at the start
    # of the step; the step's electric forces use the deposited charges q^n
    npp = 0
    qc = q
    if prm.get("pp", 0):
        dvxc, dvyc, dvzc, dqc, npp = collide_pp(cid, x, y, z, vx, vy, vz, q, d, prm["k_pp"])
        vx, vy, vz = vx + dvxc, vy + dvyc, vz + dvzc
        qc = q + dqc

    phi = poisson(g, Q)
    Ex, Ey, Ez = efield(g, phi)
    Epx, Epy, Epz = Ex.ravel()[cid], Ey.ravel()[cid], Ez.ravel()[cid]

    ux, uy, uz = interp(g, U, x, y, z, i, j, k)
    sx, sy, sz = coulomb_sums(x, y, z, q, cid)

    # forces and semi-implicit Euler
    gp = [(1.0 - 1.0 / rr) * gc for gc in gvec]
    ke = (cel * q) / ((d * d) * d)
    ax = gp[0] + ke * (Epx + sx * INV4PI)
    ay = gp[1] + ke * (Epy + sy * INV4PI)
    az = gp[2] + ke * (Epz + sz * INV4PI)

    dux, duy, duz = vx - ux, vy - uy, vz - uz
    rel = np.sqrt((dux * dux + duy * duy) + duz * duz)
    re = rel * d
    phid = np.where(re <= 1000.0, 1.0 + np.power(re, TWO_THIRDS) / 6.0, 0.424 * re / 24.0)
    taup = ((rr * d) * d) / 18.0
    sdr = phid / taup
    den = 1.0 + dt * sdr
    v1x = (vx + dt * (ux * sdr + ax)) / den
    v1y = (vy + dt * (uy * sdr + ay)) / den
    v1z = (vz + dt * (uz * sdr + az)) / den
    x1 = x + dt * v1x
    y1 = y + dt * v1y
    z1 = z + dt * v1z

    # wall impact: hard-sphere rebound and condenser charge transfer
    r = 0.5 * d
    top = g.ly - r
    if replay is not None:
        wall = replay["wall"]
    else:
        wall = np.where(y1 < r, 0, np.where(y1 > top, 1, -1))
    lo = wall == 0
    hi = wall == 1
    hit = lo | hi
    un = np.where(lo, -v1y, np.where(hi, v1y, 0.0))
    yr = np.where(lo, r + e * (r - y1), np.where(hi, top - e * (y1 - top), y1))
    vyr = np.where(hit, -e * v1y, v1y)
    if prm.get("charging", 0) == 1:
        # stochastic scaling model: random numbers per (particle id, step number)
        if stats is None:
            raise ValueError("the SSM draws its random numbers by step number: pass stats")
        dq = np.zeros(n)
        h = np.flatnonzero(hit)
        if h.size:
            dq[h] = ssm_wall_charge(qc[h], d[h], un[h], h, stats.steps + 1, prm)
    else:
        fchg = (kc * math.pow(1.0 + e, 0.4)) * np.power(np.where(hit, un, 0.0), 0.8)
        dq = np.where(hit, -fchg * (dU + qc), 0.0)
    q1 = np.where(hit, qc + dq, qc)

    # periodic wrap
    if replay is not None:
        wx, wz = replay["wx"], replay["wz"]
    else:
        wx = np.where(x1 >= g.lx, -1, np.where(x1 < 0.0, 1, 0))
        wz = np.where(z1 >= g.lz, -1, np.where(z1 < 0.0, 1, 0))
    x1 = np.where(wx == -1, x1 - g.lx, np.where(wx == 1, x1 + g.lx, x1))
    z1 = np.where(wz == -1, z1 - g.lz, np.where(wz == 1, z1 + g.lz, z1))

    if stats is not None:
        stats.steps += 1
        stats.pp_pairs += npp
        for w in (0, 1):
            m = wall == w
            stats.impacts[w] += int(m.sum())
            wq, ovf_w = fixed_checked(-dq[m], FIX_WALL)
            stats.wallq[w] += int(wq.sum())
            if ovf_w:
                stats.flags |= F_OVERFLOW
            stats.wallq_f[w] += float((-dq[m]).sum())
        b = np.minimum((un[hit] / un_bin).astype(np.int64), N_UNBIN - 1)
        stats.unhist += np.bincount(b, minlength=N_UNBIN).astype(np.int64)
        if replay is None:
            if np.any((yr < r) | (yr > top)):
                stats.flags |= F_OUTSIDE
        if not all(np.all(np.isfinite(a)) for a in (x1, yr, z1, v1x, vyr, v1z, q1)):
            stats.flags |= F_NONFINITE

    if record is not None:
        record.append(dict(i=i, j=j, k=k, wall=wall, wx=wx, wz=wz))
    if want is not None:
        want.update(Q=Q, phi=phi, E=(Ex, Ey, Ez), u=(ux, uy, uz), coul=(sx, sy, sz), cid=cid,
                    wall=wall, un=un, dq=dq,
                    fs=two_way_source(g, cid, d, sdr, (ux, uy, uz), (v1x, v1y, v1z), rr))
    return dict(x=x1, y=yr, z=z1, vx=v1x, vy=vyr, vz=v1z, q=q1, d=d)


def run(g: Geo, U, s, prm, n_steps: int, stats: Optional[Stats] = None, record=None, replay=None):
    for n in range(n_steps):
        s = step(g, U, s, prm, stats, replay=None if replay is None else replay[n], record=record)
    return s


def state_of(ens) -> Dict[str, np.ndarray]:
    return {k: np.array(getattr(ens, k), dtype=np.float64, copy=True) for k in KEYS}
