// Per-particle forward evaluation of the step, shared by the push and its
// reverse-mode derivative (internal).  Everything up to the wall impact:
// carrier velocity, cell-centred E, same-cell Coulomb sum, forces and the
// semi-implicit Euler update.
#pragma once
#include "tribo_dev.h"

namespace tf {

__device__ __forceinline__ int clamp_floor(double v, int n) {
  const double f = floor(v);
  return (f >= 0.0) ? (f < (double)(n - 1) ? (int)f : n - 1) : 0;
}

// largest j in [0, ny-1] with yf[j] <= y (0 if none), searched from a guess
__device__ __forceinline__ int y_cell_from(const double* __restrict__ yf, int ny, double y, int j) {
  while (j > 0 && y < yf[j]) --j;
  while (j < ny - 1 && y >= yf[j + 1]) ++j;
  return j;
}

// two doubles with 8-byte alignment (one dwordx4 load)
typedef double d2u __attribute__((ext_vector_type(2), aligned(8)));

struct Fwd {
  int i, j, k, i1, k1, n00, n01, n10, n11, plane;
  double x, y, z, vx, vy, vz, q, d;
  double tx, ty, tz;
  double yf0, yf1;  // faces of the particle's cell row (yf[j], yf[j + 1])
  double u[3], Ep[3], S[3];
  double ke, a[3], du[3], re, phid, sdr, iden, v1[3];
  double x1, y1, z1;  // after the update, before rebound and wrap
  double qc;          // charge after particle-particle exchange (= q without 4-way coupling)
};

// Position, charge, velocity and diameter of slot s are gathered through
// C.perm from `in` (nearly coalesced: particles move little between sorts).
// SORTED (the push: the lanes of a wave hold consecutive slots): the cell
// mates' positions and charges come from their lanes; otherwise (the reverse
// step) they are gathered through C.perm as well.
// One binary collision of the particle (position difference r = s_self -
// s_mate, |r|^2 = r2, diameter d, velocity v, charge q) with the mate at old
// slot pj: hit when they overlap and approach; then the velocity and charge
// increments of the particle (fully elastic, masses ~ d^3; condenser exchange
// with the Hertz exponent).
struct PPHit {
  double dvx, dvy, dvz, dq;
  int hit;
};
__device__ __forceinline__ PPHit pp_pair(int pj, const PState& in, double kpp, double rx, double ry, double rz,
                                      double r2, double d, double vx, double vy, double vz, double q, double oq) {
  PPHit h{0.0, 0.0, 0.0, 0.0, 0};
  const double od = in.d[pj];
  const double rc = 0.5 * (d + od);
  if (!(r2 > 0.0 && r2 < rc * rc)) return h;
  const double wx = vx - in.vx[pj], wy = vy - in.vy[pj], wz = vz - in.vz[pj];
  if ((wx * rx + wy * ry) + wz * rz >= 0.0) return h;
  h.hit = 1;
  const double ri = 1.0 / sqrt(r2);
  const double nx_ = rx * ri, ny_ = ry * ri, nz_ = rz * ri;
  const double un = (wx * nx_ + wy * ny_) + wz * nz_;
  const double mi = (d * d) * d, mj = (od * od) * od;
  const double ci = 2.0 * mj / (mi + mj) * un;
  h.dvx = -(ci * nx_);
  h.dvy = -(ci * ny_);
  h.dvz = -(ci * nz_);
  const double speed = sqrt((wx * wx + wy * wy) + wz * wz);
  const double xe =
      kpp * (pow(d * od, 2.0) * pow(d + od, -0.6) * pow(pow(d, 3.0) + pow(od, 3.0), -0.8)) * pow(speed, 0.6);
  h.dq = (d * oq - od * q) / (d + od) * (1.0 - exp(-xe));
  return h;
}

// Slots [ra, rb) of cell c, from the sorted keys of the wave's lanes (which
// hold consecutive slots s, so a cell's slots are a run of equal keys).  A run
// that reaches the first or last lane may continue in the neighbouring wave:
// then ra or rb is -1 and the caller reads the cell start.  Every lane of the
// wave must take part.
__device__ __forceinline__ void cell_run(int s, int c, int* ra, int* rb) {
  const int lane = (int)(threadIdx.x & 63u);
  const int kp = __shfl_up(c, 1, 64);
  const unsigned long long heads = __ballot(lane == 0 || kp != c);
  const unsigned long long upto = (2ull << lane) - 1ull;  // lanes 0..lane (all for lane 63)
  const int hl = 63 - __clzll(heads & upto);              // lane 0 is always a head
  const unsigned long long after = heads & ~upto;
  const int el = after ? __ffsll((long long)after) - 1 : 64;
  const int s0 = s - lane;
  *ra = hl == 0 ? -1 : s0 + hl;
  *rb = el == 64 ? -1 : s0 + el;
}

// PP: compiled with the 4-way coupling (particle-particle collisions)
// [ra, rb): the slots of cell c (its particles, s among them)
// pmw (SORTED): lanes 0..31 hold the old slots of the 32 slots before the
// wave (nearest first), lanes 32..63 those of the 32 slots after it
template <bool SORTED, bool PP = false>
__device__ __forceinline__ void eval_particle(const Ctx& C, const Ens& E, const PState& in, int s, int p, int c,
                                              int ra, int rb, Fwd& F, int pmw = 0) {
  const int nx = E.nx, ny = E.ny, nz = E.nz;
  const int cl = c - (int)E.c_off;
  int jk, i, j, k;
  divmod(cl, nx, E.inv_nx, &jk, &i);
  divmod(jk, nz, E.inv_nz, &j, &k);
  const double* __restrict__ yf = C.yf + E.y_off;
  const double* __restrict__ idy = C.idy + E.y_off;

  const double x = in.x[p], y = in.y[p], z = in.z[p], q = in.q[p];
  const double vx = in.vx[p], vy = in.vy[p], vz = in.vz[p];
  const double d = in.d[p];

  // carrier velocity: trilinear in the cell, linear in physical y
  const int i1 = (i + 1 == nx) ? 0 : i + 1;
  const int k1 = (k + 1 == nz) ? 0 : k + 1;
  const double tx = (x - (double)i * E.dx) * E.inv_dx;
  const double ty = (y - yf[j]) * idy[j];
  const double tz = (z - (double)k * E.dz) * E.inv_dz;
  const int nxz = nz * nx;
  const int plane = (ny + 1) * nxz;
  const int n00 = (j * nz + k) * nx, n01 = (j * nz + k1) * nx;
  const int n10 = n00 + nxz, n11 = n01 + nxz;
  // nodes i and i + 1 of the four node rows of the cell, each pair one
  // 16-byte load from the padded copy (its ghost nodes make the periodic row
  // end an ordinary load): twelve loads with no branch between them, all in
  // flight together
  double uc[3];
  {
    const int nxp = E.nxp, rowp = nz * nxp, planep = (ny + 1) * rowp;
    const int p00 = (j * nz + k) * nxp + i, p01 = (j * nz + k1) * nxp + i;
    const double* __restrict__ ub = C.upad + E.up_off;
    d2u u[3][4];
#pragma unroll
    for (int cc = 0; cc < 3; ++cc) {
      const double* __restrict__ b = ub + cc * planep;
      u[cc][0] = *reinterpret_cast<const d2u*>(b + p00);
      u[cc][1] = *reinterpret_cast<const d2u*>(b + p01);
      u[cc][2] = *reinterpret_cast<const d2u*>(b + p00 + rowp);
      u[cc][3] = *reinterpret_cast<const d2u*>(b + p01 + rowp);
    }
#pragma unroll
    for (int cc = 0; cc < 3; ++cc) {
      const double c00 = u[cc][0].x * (1.0 - tx) + u[cc][0].y * tx;
      const double c01 = u[cc][1].x * (1.0 - tx) + u[cc][1].y * tx;
      const double c10 = u[cc][2].x * (1.0 - tx) + u[cc][2].y * tx;
      const double c11 = u[cc][3].x * (1.0 - tx) + u[cc][3].y * tx;
      const double c0 = c00 * (1.0 - tz) + c01 * tz;
      const double c1 = c10 * (1.0 - tz) + c11 * tz;
      uc[cc] = c0 * (1.0 - ty) + c1 * ty;
    }
  }

  // Gauss part: cell-centred E = -grad(phi), Gauss-linear, phi = 0 on the walls
  const double* __restrict__ ph = C.phi + E.c_off;
  const int im = (i == 0) ? nx - 1 : i - 1;
  const int km = (k == 0) ? nz - 1 : k - 1;
  const double pc = ph[cl];
  const double Ex = -(ph[n00 + i1] - ph[n00 + im]) * E.inv_2dx;
  const double Ez = -(ph[n01 + i] - ph[(j * nz + km) * nx + i]) * E.inv_2dz;
  // wall-normal neighbours from clamped rows (no branch around the loads);
  // the wall faces take phi = 0
  const bool has_top = j < ny - 1, has_bot = j > 0;
  const double pn = ph[n00 + (has_top ? nxz : 0) + i];
  const double pm = ph[n00 - (has_bot ? nxz : 0) + i];
  const double ftop = has_top ? pc + C.beta[E.y_off + j + 1] * (pn - pc) : 0.0;
  const double fbot = has_bot ? pm + C.beta[E.y_off + j] * (pc - pm) : 0.0;
  const double Ey = -(ftop - fbot) * idy[j];

  // near field: Coulomb's law with the other particles of the cell, ascending id
  double sx = 0.0, sy = 0.0, sz = 0.0;
  auto coulomb = [&](double ox, double oy, double oz, double oq) {
    const double rx = x - ox, ry = y - oy, rz = z - oz;
    const double r2 = (rx * rx + ry * ry) + rz * rz;
    if (r2 > 0.0) {
      const double ri = rsqrt(r2);
      const double w = oq * (ri * ri * ri);
      sx += w * rx;
      sy += w * ry;
      sz += w * rz;
    }
  };
  {
    const int a = ra, b = rb;
    if constexpr (SORTED) {
      // The lanes of a wave hold consecutive slots and a cell's particles
      // are consecutive slots, so most cell mates sit in this wave: their
      // position and charge come from their lanes (cross-lane reads), the
      // others (cells across the wave's ends) from memory.  Mates in
      // ascending id, as in the plain loop; the loop runs while some lane of
      // the wave has a mate left.
      const int lane = (int)(threadIdx.x & 63u);
      const int s0 = s - lane;
      const int n = b - a;
      for (int kk = 0; __any(kk < n); ++kk) {
        const int t = a + kk;
        const int src = t - s0;
        const bool inw = src >= 0 && src < 64;
        double ox = __shfl(x, src & 63, 64), oy = __shfl(y, src & 63, 64);
        double oz = __shfl(z, src & 63, 64), oq = __shfl(q, src & 63, 64);
        // a mate within 32 slots of the wave's ends: its old slot from pmw
        // (read at the kernel's start), so only its state is loaded here
        const int hb = s0 - 1 - t, ta = t - s0 - 64;
        const int pmv = __shfl(pmw, hb >= 0 ? (hb & 31) : 32 + (ta & 31), 64);
        if (kk < n && t != s) {
          if (!inw) {
            const int pt = (hb >= 0 && hb < 32) || (ta >= 0 && ta < 32) ? pmv : C.perm[t];
            ox = in.x[pt];
            oy = in.y[pt];
            oz = in.z[pt];
            oq = in.q[pt];
          }
          coulomb(ox, oy, oz, oq);
        }
      }
    } else {
      for (int t = a; t < b; ++t) {
        if (t == s) continue;
        const int pj = C.perm[t];
        coulomb(in.x[pj], in.y[pj], in.z[pj], in.q[pj]);
      }
    }
  }
  // 4-way coupling: the collision increments of this slot (k_collide)
  double cvx = 0.0, cvy = 0.0, cvz = 0.0, cq = 0.0;
  if constexpr (PP) {
    if (E.pp && C.chit[s]) {  // increments stored only for the slots with a collision
      const long long n = C.n_tot;
      cvx = C.cinc[s];
      cvy = C.cinc[n + s];
      cvz = C.cinc[2 * n + s];
      cq = C.cinc[3 * n + s];
    }
  }
  const bool pp = PP && E.pp;
  const double vxs = pp ? vx + cvx : vx, vys = pp ? vy + cvy : vy, vzs = pp ? vz + cvz : vz;
  // forces and semi-implicit Euler
  const double d2 = d * d;
  const double ke = (E.cel * q) / (d2 * d);
  const double ax = E.gp0 + ke * (Ex + sx * kInv4Pi);
  const double ay = E.gp1 + ke * (Ey + sy * kInv4Pi);
  const double az = E.gp2 + ke * (Ez + sz * kInv4Pi);
  const double dux = vxs - uc[0], duy = vys - uc[1], duz = vzs - uc[2];
  const double re = sqrt((dux * dux + duy * duy) + duz * duz) * d;
  const double phid = (re <= 1000.0) ? 1.0 + cbrt(re * re) * (1.0 / 6.0) : 0.424 * re * (1.0 / 24.0);
  const double sdr = phid * (E.c18 / d2);  // phi_D / tau_p
  const double iden = 1.0 / (1.0 + E.dt * sdr);
  const double v1x = (vxs + E.dt * (uc[0] * sdr + ax)) * iden;
  const double v1y = (vys + E.dt * (uc[1] * sdr + ay)) * iden;
  const double v1z = (vzs + E.dt * (uc[2] * sdr + az)) * iden;
  const double x1 = x + E.dt * v1x;
  const double y1 = y + E.dt * v1y;
  const double z1 = z + E.dt * v1z;
  F.i = i; F.j = j; F.k = k; F.i1 = i1; F.k1 = k1;
  F.n00 = n00; F.n01 = n01; F.n10 = n10; F.n11 = n11; F.plane = plane;
  F.x = x; F.y = y; F.z = z; F.vx = vx; F.vy = vy; F.vz = vz; F.q = q; F.d = d;
  F.tx = tx; F.ty = ty; F.tz = tz;
  F.yf0 = yf[j]; F.yf1 = yf[j + 1];
  F.u[0] = uc[0]; F.u[1] = uc[1]; F.u[2] = uc[2];
  F.Ep[0] = Ex; F.Ep[1] = Ey; F.Ep[2] = Ez;
  F.S[0] = sx; F.S[1] = sy; F.S[2] = sz;
  F.ke = ke; F.a[0] = ax; F.a[1] = ay; F.a[2] = az;
  F.du[0] = dux; F.du[1] = duy; F.du[2] = duz;
  F.re = re; F.phid = phid; F.sdr = sdr; F.iden = iden;
  F.v1[0] = v1x; F.v1[1] = v1y; F.v1[2] = v1z;
  F.x1 = x1; F.y1 = y1; F.z1 = z1;
  F.qc = pp ? q + cq : q;
}

}  // namespace tf
