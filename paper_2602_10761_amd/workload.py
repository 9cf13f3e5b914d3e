"""Seeded synthetic channel workloads for the triboelectric particle step.

This module is the only code shared by the oracle side and the HIP side: it
produces *inputs* (mesh faces, a frozen carrier velocity field on the mesh
nodes, initial particle state, physical parameters) and holds none of the
particle-step arithmetic (no interpolation, forcing, charging, deposit or
Poisson solve).

Units are wall units throughout: nu = u_tau = 1, lengths in nu/u_tau, the
half channel height h equals Re_tau.  Charge is in units of the saturation
charge q_sat (the paper normalises particle charge by q_sat, Sec. 4.1).

Recipe (stands in for the paper's DNS/LES channel flows, Sec. 3.1-3.2, which
are not reproducible here):
  * domain 4*pi*h x 2h x (4/3)*pi*h, periodic in x and z (Sec. 3.1),
  * faces uniform in x and z, tanh-stretched in y,
  * carrier field = Reichardt mean profile + divergence-free Fourier modes
    (curl of a wall-damped vector potential), rescaled to unit rms,
  * particles uniform in the volume available to their centre, charge 0,
    velocity equal to the local mean flow.
Random draws come from counter-based SplitMix64 streams.
"""
from __future__ import annotations

import dataclasses
import math
from dataclasses import dataclass, field
from typing import List, Optional, Sequence, Tuple

import numpy as np

# ----------------------------------------------------------------------------
# Counter-based SplitMix64 (Steele, Lea & Flood 2014 finaliser)
# ----------------------------------------------------------------------------
_GAMMA = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)
_MASK = (1 << 64) - 1


def _mix64(z: np.ndarray) -> np.ndarray:
    z = np.asarray(z, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
    return z ^ (z >> np.uint64(31))


def _mix_int(v: int) -> int:
    return int(_mix64(np.array([v & _MASK], dtype=np.uint64))[0])


class Stream:
    """One counter-based SplitMix64 stream: value n = mix(seed + n*gamma)."""

    def __init__(self, seed: int):
        self.seed = np.uint64(seed & _MASK)
        self.ctr = 0

    def u64(self, n: int) -> np.ndarray:
        idx = np.arange(self.ctr + 1, self.ctr + n + 1, dtype=np.uint64)
        self.ctr += n
        with np.errstate(over="ignore"):
            return _mix64(self.seed + idx * _GAMMA)

    def uniform(self, n: int) -> np.ndarray:
        """Doubles in [0, 1): (u64 >> 11) * 2^-53."""
        return (self.u64(n) >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)


# stream tags
S_MODES, S_POS, S_DIAM, S_ENS, S_CHARGE = 0, 1, 2, 3, 4
MASTER_SEED = 260210761


def stream(config_index: int, seed: int, tag: int, sub: int = 0) -> Stream:
    master = _mix_int(MASTER_SEED + (config_index << 32) + seed)
    return Stream(_mix_int(master + (tag << 16) + (sub << 24) + 1))


# ----------------------------------------------------------------------------
# Physical constants (Table 1) and derived normalised couplings
# ----------------------------------------------------------------------------
MATERIAL = dict(
    mu_p=0.4, E_p=1e8, resistivity_p=1e13, k_e=0.95, mu_w=0.28, E_w=1e11,
    eps_w=5.0, h_sep=1e-9, eps=8.854e-12, nu=1.46e-5, rho=1.2, rho_p=1150.0,
)
DELTA = 0.02        # channel half height [m], Sec. 3.1
Q_SAT = 1.26e-13    # saturation charge [C], Sec. 3.1 (exponent sign garbled in print)


def u_tau(re_tau: float) -> float:
    """Friction velocity [m/s] from Re_tau = u_tau*delta/nu (Sec. 3.1)."""
    return re_tau * MATERIAL["nu"] / DELTA


def d_plus(d_m: float, re_tau: float) -> float:
    """Particle diameter in wall units (Table 2 column d_p^+)."""
    return d_m * u_tau(re_tau) / MATERIAL["nu"]


def stokes_number(d_m: float, u_c: float) -> float:
    """St = (1/18)(rho_p/rho)(d^2/nu)(u_c/delta), Sec. 3.1."""
    m = MATERIAL
    return (1.0 / 18.0) * (m["rho_p"] / m["rho"]) * (d_m ** 2 / m["nu"]) * (u_c / DELTA)


def volume_fraction_1e6(d_m: float, number_density: float = 1e8) -> float:
    """omega = C*pi*d^3/6, reported in units of 1e-6 (Table 2 last column)."""
    return number_density * math.pi * d_m ** 3 / 6.0 * 1e6


def electric_coupling(re_tau: float) -> float:
    """Normalised Gauss/Coulomb coupling C_el = 6 q_sat^2 u_tau^2/(pi eps rho_p nu^4).

    Specific electric force q E/m_p (Sec. 2.2) with m_p = pi rho_p d^3/6, the
    potential scaled by q_sat/(eps*l) and lengths by l = nu/u_tau, becomes
    C_el * q+ E+ / d+^3 in wall units.
    """
    m = MATERIAL
    ut = u_tau(re_tau)
    return 6.0 * Q_SAT ** 2 * ut ** 2 / (math.pi * m["eps"] * m["rho_p"] * m["nu"] ** 4)


def lumped_transfer_coefficient(re_tau: float) -> float:
    """k_c = (1/4)(K rho_p u_tau^2)^(2/5), K = (5 pi/8)[(1-mu_p^2)/E_p + (1-mu_w^2)/E_w].

    Contact-area fraction of the Hertz particle-wall contact (Sec. 2.3.1) per
    unit of (1+e)^(2/5) u_n+^(4/5); the workloads use the rounded value 1e-3.
    """
    m = MATERIAL
    K = 5.0 * math.pi / 8.0 * ((1 - m["mu_p"] ** 2) / m["E_p"] + (1 - m["mu_w"] ** 2) / m["E_w"])
    return 0.25 * (K * m["rho_p"] * u_tau(re_tau) ** 2) ** 0.4


# ----------------------------------------------------------------------------
# Mesh, carrier field, particles
# ----------------------------------------------------------------------------
def y_faces(ny: int, re_tau: float, stretch: float) -> np.ndarray:
    """Wall-normal faces y_j = h(1 - tanh(g(1-2j/ny))/tanh g), j = 0..ny."""
    h = float(re_tau)
    j = np.arange(ny + 1, dtype=np.float64)
    if stretch == 0.0:
        yf = 2.0 * h * j / ny
    else:
        yf = h * (1.0 - np.tanh(stretch * (1.0 - 2.0 * j / ny)) / math.tanh(stretch))
    yf[0] = 0.0
    yf[-1] = 2.0 * h
    return yf


def reichardt(yplus: np.ndarray) -> np.ndarray:
    """Reichardt's law of the wall U+(y+), kappa = 0.41."""
    k = 0.41
    return np.log1p(k * yplus) / k + 7.8 * (1.0 - np.exp(-yplus / 11.0) - (yplus / 11.0) * np.exp(-yplus / 3.0))


def mean_flow(y: np.ndarray, re_tau: float) -> np.ndarray:
    h = float(re_tau)
    return reichardt(np.minimum(y, 2.0 * h - y))


@dataclass
class Mesh:
    nx: int
    ny: int
    nz: int
    lx: float
    lz: float
    yf: np.ndarray  # ny+1 faces

    @property
    def ly(self) -> float:
        return float(self.yf[-1])

    @property
    def ncell(self) -> int:
        return self.nx * self.ny * self.nz


def carrier_field(mesh: Mesh, re_tau: float, n_modes: int, st: Stream, rms: float = 1.0) -> np.ndarray:
    """Frozen node field U[3, ny+1, nz, nx] at (x_i, y_j, z_k) = (i dx, yf[j], k dz).

    u' = curl(A), A = D(yh) sum_m a_m cos(k_m.x + th_m), D = (yh(2-yh))^2,
    yh = y/h: divergence free; u' vanishes on the walls, its wall-normal
    component quadratically.  The x-z dependence is summed spectrally (one 2-D FFT per
    y node), which evaluates the same finite mode sum at the grid points.
    """
    nx, ny, nz = mesh.nx, mesh.ny, mesh.nz
    h = float(re_tau)
    lx, ly, lz = mesh.lx, mesh.ly, mesh.lz
    u = st.uniform(7 * n_modes).reshape(n_modes, 7)
    nxm = np.maximum(1, nx // 4)
    nzm = nz // 4
    n_x = 1 + np.floor(u[:, 0] * nxm).astype(np.int64)
    n_x = np.minimum(n_x, nxm)
    n_z = -nzm + np.floor(u[:, 1] * (2 * nzm + 1)).astype(np.int64)
    n_z = np.minimum(n_z, nzm)
    kx = 2.0 * math.pi * n_x / lx
    kz = 2.0 * math.pi * n_z / lz
    ky = u[:, 2] * 8.0 * math.pi / ly
    cth = 2.0 * u[:, 3] - 1.0
    sth = np.sqrt(np.maximum(0.0, 1.0 - cth * cth))
    ph = 2.0 * math.pi * u[:, 4]
    kmag = np.sqrt(kx * kx + ky * ky + kz * kz)
    amp = kmag ** (-5.0 / 6.0)
    ax = amp * sth * np.cos(ph)
    ay = amp * sth * np.sin(ph)
    az = amp * cth
    theta = 2.0 * math.pi * u[:, 5]

    y = mesh.yf
    yh = y / h
    D = (yh * (2.0 - yh)) ** 2
    Dp = 2.0 * yh * (2.0 - yh) * (2.0 - 2.0 * yh) / h
    # spectral coefficients B[c, j, kz_idx, kx_idx]; x-z grid value = Re(sum B e^{i(kx x + kz z)})
    B = np.zeros((3, ny + 1, nz, nx), dtype=np.complex128)
    ph_y = np.exp(1j * (theta[None, :] + ky[None, :] * y[:, None]))          # [ny+1, M]
    Dj = D[:, None]
    Dpj = Dp[:, None]
    dyf = Dpj + 1j * ky[None, :] * Dj      # coefficient of e^{i psi} in d/dy f
    dxf = 1j * kx[None, :] * Dj
    dzf = 1j * kz[None, :] * Dj
    cx = (dyf * az[None, :] - dzf * ay[None, :]) * ph_y
    cy = (dzf * ax[None, :] - dxf * az[None, :]) * ph_y
    cz = (dxf * ay[None, :] - dyf * ax[None, :]) * ph_y
    kzi = np.mod(n_z, nz)
    kxi = np.mod(n_x, nx)
    for c, coef in enumerate((cx, cy, cz)):
        for m in range(n_modes):
            B[c, :, kzi[m], kxi[m]] += coef[:, m]
    # Re(sum_k B_k e^{i k.x}) on the grid = Re(ifft2(B) * nx * nz)
    up = np.real(np.fft.ifft2(B, axes=(2, 3))) * (nx * nz)
    # volume-weighted rms over the nodes (dual-cell widths in y)
    w = np.empty(ny + 1)
    w[1:-1] = 0.5 * (y[2:] - y[:-2])
    w[0] = 0.5 * (y[1] - y[0])
    w[-1] = 0.5 * (y[-1] - y[-2])
    ms = np.einsum("j,cjki->", w, up * up) / (w.sum() * nx * nz * 3.0)
    if ms > 0:
        up *= rms / math.sqrt(ms)
    U = up
    U[0] += mean_flow(y, re_tau)[:, None, None]
    U[:, 0] = 0.0
    U[:, -1] = 0.0
    return np.ascontiguousarray(U)


@dataclass
class EnsembleSpec:
    re_tau: float = 180.0
    nx: int = 32
    ny: int = 32
    nz: int = 32
    stretch: float = 2.0
    n_modes: int = 64
    n_particles: int = 10_000
    d_choices: Tuple[float, ...] = (0.5,)
    dt: float = 0.1
    density_ratio: float = 1000.0
    k_c: float = 1e-3
    delta_u: float = 1.0
    e: float = 0.9
    c_el: Optional[float] = None      # None: derive from re_tau
    g: Tuple[float, float, float] = (0.0, 0.0, 0.0)
    un_bin: float = 0.05
    pp: int = 0                      # 4-way coupling (particle-particle collisions) on
    k_pp: float = 0.0                # particle-particle charge-exchange coefficient
    charging: int = 0                # wall charging: 0 condenser, 1 stochastic scaling model
    ssm: Tuple[float, ...] = ()      # SSM (dq0min, mu0, sigma0, gamma0, csat, d0, un0)
    seed: int = 0                    # SSM random numbers
    steps: int = 1000
    precharge: float = 0.0           # q0 ~ U[-precharge, precharge]
    v_jitter: float = 0.0            # v0 += v_jitter * U[-1, 1]^3 (tests that need early impacts)

    def replace(self, **kw) -> "EnsembleSpec":
        return dataclasses.replace(self, **kw)


@dataclass
class Ensemble:
    spec: EnsembleSpec
    mesh: Mesh
    U: np.ndarray                      # [3, ny+1, nz, nx]
    x: np.ndarray
    y: np.ndarray
    z: np.ndarray
    vx: np.ndarray
    vy: np.ndarray
    vz: np.ndarray
    q: np.ndarray
    d: np.ndarray
    params: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return int(self.x.shape[0])

    def state(self) -> dict:
        return dict(x=self.x.copy(), y=self.y.copy(), z=self.z.copy(), vx=self.vx.copy(),
                    vy=self.vy.copy(), vz=self.vz.copy(), q=self.q.copy(), d=self.d.copy())


def make_ensemble(spec: EnsembleSpec, config_index: int = 0, seed: int = 0, sub: int = 0) -> Ensemble:
    h = float(spec.re_tau)
    mesh = Mesh(spec.nx, spec.ny, spec.nz, 4.0 * math.pi * h,
                4.0 * math.pi * h / 3.0, y_faces(spec.ny, spec.re_tau, spec.stretch))
    U = carrier_field(mesh, spec.re_tau, spec.n_modes, stream(config_index, seed, S_MODES, sub))
    n = spec.n_particles
    sd = stream(config_index, seed, S_DIAM, sub).uniform(n)
    choices = np.asarray(spec.d_choices, dtype=np.float64)
    d = choices[np.minimum((sd * len(choices)).astype(np.int64), len(choices) - 1)]
    sp = stream(config_index, seed, S_POS, sub).uniform(3 * n).reshape(3, n)
    r = 0.5 * d
    x = mesh.lx * sp[0]
    y = r + (mesh.ly - 2.0 * r) * sp[1]
    z = mesh.lz * sp[2]
    vx = mean_flow(y, spec.re_tau)
    vy = np.zeros(n)
    vz = np.zeros(n)
    if spec.v_jitter > 0:
        jt = stream(config_index, seed, S_CHARGE, sub + 1000).uniform(3 * n).reshape(3, n)
        vx = vx + spec.v_jitter * (2.0 * jt[0] - 1.0)
        vy = vy + spec.v_jitter * (2.0 * jt[1] - 1.0)
        vz = vz + spec.v_jitter * (2.0 * jt[2] - 1.0)
    if spec.precharge > 0:
        q = spec.precharge * (2.0 * stream(config_index, seed, S_CHARGE, sub).uniform(n) - 1.0)
    else:
        q = np.zeros(n)
    c_el = spec.c_el if spec.c_el is not None else electric_coupling(spec.re_tau)
    params = dict(dt=spec.dt, density_ratio=spec.density_ratio, k_c=spec.k_c,
                  delta_u=spec.delta_u, e=spec.e, c_el=c_el, g=tuple(spec.g), un_bin=spec.un_bin,
                  pp=spec.pp, k_pp=spec.k_pp, charging=spec.charging, seed=spec.seed)
    if spec.ssm:
        params.update(zip(("ssm_dq0min", "ssm_mu0", "ssm_sigma0", "ssm_gamma0", "ssm_csat", "ssm_d0", "ssm_un0"),
                          spec.ssm))
    return Ensemble(spec, mesh, U, x, y, z, vx, vy, vz, q, d, params)


# ----------------------------------------------------------------------------
# The five workloads (configurations of the benchmark)
# ----------------------------------------------------------------------------
CONFIGS = {
    1: EnsembleSpec(re_tau=180.0, nx=32, ny=32, nz=32, n_modes=64, n_particles=10_000,
                    d_choices=(0.5,), dt=0.1, steps=1000),
    2: EnsembleSpec(re_tau=180.0, nx=128, ny=128, nz=128, n_modes=256, n_particles=1_000_000,
                    d_choices=(0.25, 0.5, 1.0), dt=0.1, steps=2000),
    3: EnsembleSpec(re_tau=550.0, nx=192, ny=160, nz=192, n_modes=512, n_particles=4_000_000,
                    d_choices=(0.5, 1.0, 2.0), dt=0.05, steps=2000),
    5: EnsembleSpec(re_tau=180.0, nx=64, ny=64, nz=64, n_modes=128, n_particles=100_000,
                    d_choices=(0.5,), dt=0.1, steps=500),
}
BATCH_RE = (180.0, 300.0, 395.0, 550.0)
BATCH_MESH = {180.0: 64, 300.0: 96, 395.0: 128, 550.0: 160}


def batched_specs(n_ens: int = 64, seed: int = 0, np_lo: float = 1e4, np_hi: float = 1e6,
                  mesh_scale: float = 1.0) -> List[EnsembleSpec]:
    """Independent ensembles of the Re_tau x d_p sweep (Sec. 4.4, Table 2).

    N_p log-uniform in [np_lo, np_hi], Re_tau drawn from {180, 300, 395, 550}
    with meshes 64^3..160^3, d_p+ uniform in [0.25, 2] per ensemble.
    """
    u = stream(4, seed, S_ENS).uniform(3 * n_ens).reshape(n_ens, 3)
    out = []
    for m in range(n_ens):
        npart = int(round(np_lo * (np_hi / np_lo) ** u[m, 0]))
        re = BATCH_RE[min(int(u[m, 1] * 4), 3)]
        nm = max(8, int(round(BATCH_MESH[re] * mesh_scale / 8)) * 8)
        d = 0.25 + 1.75 * u[m, 2]
        out.append(EnsembleSpec(re_tau=re, nx=nm, ny=nm, nz=nm, n_modes=128, n_particles=npart,
                                d_choices=(d,), dt=0.1, steps=1000))
    return out


def make_workload(config_index: int, seed: int = 0, **overrides) -> List[Ensemble]:
    if config_index == 4:
        specs = batched_specs(seed=seed)
        return [make_ensemble(s.replace(**overrides), 4, seed, sub=m) for m, s in enumerate(specs)]
    return [make_ensemble(CONFIGS[config_index].replace(**overrides), config_index, seed)]
