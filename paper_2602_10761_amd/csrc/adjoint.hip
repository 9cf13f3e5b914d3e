// Reverse-mode derivative of recorded particle steps, events held fixed.
//
// For a step s_{n+1} = F(s_n, theta) the kernels map lambda_{n+1} (cotangent
// of the state leaving the step, slot order) to lambda_n (cotangent of the
// state entering it, previous slot order) and accumulate
// (dF/dtheta)^T lambda_{n+1} for theta = (k_c, dU, e):
//   adj_a      per slot: recompute the particle's forward quantities and run the
//              reverse of wrap, rebound/charging, position and velocity
//              update, drag, trilinear interpolation and the force terms
//   adj_ecell  per cell: sum of the particles' field cotangents (slot order)
//   adj_div    per cell: -G^T lambda_E (transpose of the Gauss-linear gradient)
//   Poisson    the discrete operator times cell volume is symmetric, so the
//              adjoint solve is the forward solve applied to -G^T lambda_E
//   adj_b      per slot: cell-charge cotangent (deposit transposed = gather)
//              and the same-cell Coulomb pair terms; scatter to the old slot
//   reduce     per ensemble, fixed order: d/dtheta
#include "adjoint.h"
#include "particle.h"

namespace tf {

AdjWork carve_adjoint(Carver& cv, long long n, long long c, long long, int n_ens, long long np_max, bool enabled) {
  AdjWork W{};
  W.enabled = enabled;
  if (!enabled) return W;
  auto lam = [&]() {
    AdjLam L;
    L.x = cv.take<double>(n);
    L.y = cv.take<double>(n);
    L.z = cv.take<double>(n);
    L.vx = cv.take<double>(n);
    L.vy = cv.take<double>(n);
    L.vz = cv.take<double>(n);
    L.q = cv.take<double>(n);
    return L;
  };
  W.lamA = lam();
  W.lamB = lam();
  W.lamP = lam();
  W.lamE = cv.take<double>(3 * n);
  W.lamS = cv.take<double>(3 * n);
  W.dth = cv.take<double>(3 * n);
  W.lamEc = cv.take<double>(3 * c);
  W.radj = cv.take<double>(c);
  W.lamQ = cv.take<double>(c);
  W.nch = (int)((np_max + kAdjChunk - 1) / kAdjChunk);
  W.part = cv.take<double>(3 * (size_t)n_ens * (size_t)(W.nch > 0 ? W.nch : 1));
  W.wwall = cv.take<double>(2 * n_ens);
  return W;
}

__device__ __forceinline__ void ens_of_cell(const Ctx& C, const Ens& Eone, int one, int c, int* e, Ens* E) {
  if (one) {
    *e = 0;
    *E = Eone;
  } else {
    *e = find_off(C.c_off, C.n_ens + 1, c);
    *E = C.ens[*e];
  }
}

__global__ __launch_bounds__(kBlock) void k_adj_a(Ctx C, Ens Eone, int one, PState in, AdjLam lam1, AdjWork W,
                                                  const signed char* __restrict__ wallrec) {
  const int s = blockIdx.x * kBlock + threadIdx.x;
  const bool act = s < C.n_tot;
  const int c = act ? C.skey[s] : 0x7fffffff;
  // as in the push: the old slots of the 32 slots on either side of the wave
  // and the lane's cell run from the wave's keys (every lane takes part)
  int pm = 0;
  {
    const int lane = (int)(threadIdx.x & 63u);
    const int s0 = s - lane;
    const int t = lane < 32 ? s0 - 1 - lane : s0 + 64 + (lane - 32);
    if (t >= 0 && t < C.n_tot) pm = C.perm[t];
  }
  int ra, rb;
  cell_run(s, c, &ra, &rb);
  if (!act) return;
  const long long n = C.n_tot;
  const int p = C.perm[s];
  if (ra < 0) ra = C.start[c];
  if (rb < 0) rb = C.start[c + 1];
  int e;
  Ens E;
  ens_of_cell(C, Eone, one, c, &e, &E);
  Fwd F;
  eval_particle<true>(C, E, in, s, p, c, ra, rb, F, pm);

  const double lx = lam1.x[s], ly = lam1.y[s], lz = lam1.z[s];
  const double lvx = lam1.vx[s], lvy = lam1.vy[s], lq = lam1.q[s], lvz = lam1.vz[s];
  double dkc = 0.0, ddu = 0.0, de = 0.0;
  double lyh = ly, lvyh = lvy, lqd = lq;
  const int wall = wallrec[s];
  if (wall >= 0) {
    // y1 = (1+e) rho - e yhat, vy1 = -e vyhat, u_n = sg vyhat,
    // f = k_c (1+e)^(2/5) u_n^(4/5), q1 = q - f (dU + q), W += f (dU + q)
    const double r = 0.5 * F.d;
    const double rho = (wall == 0) ? r : E.ly - r;
    const double sg = (wall == 0) ? -1.0 : 1.0;
    const double un = sg * F.v1[1];
    const double un08 = (un > 0.0) ? pow(un, 0.8) : 0.0;
    const double f = E.fe * un08;
    const double g = E.dU + F.q;
    const double lW = W.wwall[2 * e + wall];
    const double lf = g * (lW - lq);
    const double lg = f * (lW - lq);
    lqd = lq + lg;
    ddu += lg;
    dkc += lf * E.pe * un08;
    de += lf * f * 0.4 / (1.0 + E.e);
    const double lun = (un > 0.0) ? lf * 0.8 * f / un : 0.0;
    lyh = -E.e * ly;
    de += ly * (rho - F.y1);
    lvyh = -E.e * lvy + sg * lun;
    de += -F.v1[1] * lvy;
  }
  // x1 = x + dt v1 (wrap is a constant shift)
  const double dt = E.dt;
  const double lv1x = lvx + dt * lx, lv1y = lvyh + dt * lyh, lv1z = lvz + dt * lz;
  double lpx = lx, lpy = lyh, lpz = lz;
  // v1 = (v + dt (u sdr + a)) iden
  const double id = F.iden, sd = F.sdr;
  double lvdx = lv1x * id, lvdy = lv1y * id, lvdz = lv1z * id;
  double lux = lv1x * dt * sd * id, luy = lv1y * dt * sd * id, luz = lv1z * dt * sd * id;
  const double lax = lv1x * dt * id, lay = lv1y * dt * id, laz = lv1z * dt * id;
  const double ls = dt * id * (lv1x * (F.u[0] - F.v1[0]) + lv1y * (F.u[1] - F.v1[1]) + lv1z * (F.u[2] - F.v1[2]));
  // sdr = phi_D c18 / d^2, phi_D = 1 + re^(2/3)/6 (re <= 1000), re = |v - u| d
  const double d2 = F.d * F.d;
  const double lphid = ls * (E.c18 / d2);
  double lre = 0.0;
  if (F.re > 0.0) lre = (F.re <= 1000.0) ? lphid * (1.0 / 9.0) * cbrt(F.re * F.re) / F.re : lphid * (0.424 / 24.0);
  const double rel = F.re / F.d;
  if (rel > 0.0) {
    const double kk = lre * F.d / rel;
    lvdx += kk * F.du[0];
    lvdy += kk * F.du[1];
    lvdz += kk * F.du[2];
    lux -= kk * F.du[0];
    luy -= kk * F.du[1];
    luz -= kk * F.du[2];
  }
  // trilinear carrier velocity: lambda_x += (du/dx)^T lambda_u
  {
    const double lu[3] = {lux, luy, luz};
    const double tx = F.tx, ty = F.ty, tz = F.tz;
    const double idyj = C.idy[E.y_off + F.j];
#pragma unroll
    for (int cc = 0; cc < 3; ++cc) {
      const double* __restrict__ b = C.uptr[E.ei] + cc * F.plane;
      const double a000 = b[F.n00 + F.i], a100 = b[F.n00 + F.i1];
      const double a001 = b[F.n01 + F.i], a101 = b[F.n01 + F.i1];
      const double a010 = b[F.n10 + F.i], a110 = b[F.n10 + F.i1];
      const double a011 = b[F.n11 + F.i], a111 = b[F.n11 + F.i1];
      const double c00 = a000 * (1.0 - tx) + a100 * tx, c01 = a001 * (1.0 - tx) + a101 * tx;
      const double c10 = a010 * (1.0 - tx) + a110 * tx, c11 = a011 * (1.0 - tx) + a111 * tx;
      const double c0 = c00 * (1.0 - tz) + c01 * tz, c1 = c10 * (1.0 - tz) + c11 * tz;
      const double dtx = ((a100 - a000) * (1.0 - tz) + (a101 - a001) * tz) * (1.0 - ty) +
                         ((a110 - a010) * (1.0 - tz) + (a111 - a011) * tz) * ty;
      const double dtz = (c01 - c00) * (1.0 - ty) + (c11 - c10) * ty;
      const double dty = c1 - c0;
      lpx += lu[cc] * dtx * E.inv_dx;
      lpy += lu[cc] * dty * idyj;
      lpz += lu[cc] * dtz * E.inv_dz;
    }
  }
  // a = g' + ke (E + S/(4 pi)), ke = c_el q / d^3
  const double lke = lax * (F.Ep[0] + F.S[0] * kInv4Pi) + lay * (F.Ep[1] + F.S[1] * kInv4Pi) +
                     laz * (F.Ep[2] + F.S[2] * kInv4Pi);
  lqd += lke * E.cel / (d2 * F.d);
  W.lamE[s] = F.ke * lax;
  W.lamE[n + s] = F.ke * lay;
  W.lamE[2 * n + s] = F.ke * laz;
  W.lamS[s] = F.ke * lax * kInv4Pi;
  W.lamS[n + s] = F.ke * lay * kInv4Pi;
  W.lamS[2 * n + s] = F.ke * laz * kInv4Pi;
  W.lamP.x[s] = lpx;
  W.lamP.y[s] = lpy;
  W.lamP.z[s] = lpz;
  W.lamP.vx[s] = lvdx;
  W.lamP.vy[s] = lvdy;
  W.lamP.vz[s] = lvdz;
  W.lamP.q[s] = lqd;
  // summed per slot over the segment's steps (a slot stays inside its
  // ensemble's range, so the per-ensemble totals are unchanged)
  W.dth[s] += dkc;
  W.dth[n + s] += ddu;
  W.dth[2 * n + s] += de;
}

// field cotangent per cell: sum over the cell's run of slots, in slot order
__global__ __launch_bounds__(kBlock) void k_adj_ecell(Ctx C, AdjWork W) {
  const int cg = blockIdx.x * kBlock + threadIdx.x;
  if (cg >= C.c_tot) return;
  const long long n = C.n_tot, nc = C.c_tot;
  const int a = C.start[cg], b = C.start[cg + 1];
  double ex = 0.0, ey = 0.0, ez = 0.0;
  for (int s = a; s < b; ++s) {
    ex += W.lamE[s];
    ey += W.lamE[n + s];
    ez += W.lamE[2 * n + s];
  }
  W.lamEc[cg] = ex;
  W.lamEc[nc + cg] = ey;
  W.lamEc[2 * nc + cg] = ez;
}

// -G^T lambda_E, with (G phi) the Gauss-linear cell gradient of the forward step
__global__ __launch_bounds__(kBlock) void k_adj_div(Ctx C, Ens Eone, int one, AdjWork W) {
  const int cg = blockIdx.x * kBlock + threadIdx.x;
  if (cg >= C.c_tot) return;
  int e;
  Ens E;
  ens_of_cell(C, Eone, one, cg, &e, &E);
  const long long nc = C.c_tot;
  const int nx = E.nx, ny = E.ny, nz = E.nz;
  const int cl = cg - (int)E.c_off;
  int jk, i, j, k;
  divmod(cl, nx, E.inv_nx, &jk, &i);
  divmod(jk, nz, E.inv_nz, &j, &k);
  const double* lx = W.lamEc + E.c_off;
  const double* ly = W.lamEc + nc + E.c_off;
  const double* lz = W.lamEc + 2 * nc + E.c_off;
  const int ip = (i + 1 == nx) ? 0 : i + 1, im = (i == 0) ? nx - 1 : i - 1;
  const int kp = (k + 1 == nz) ? 0 : k + 1, km = (k == 0) ? nz - 1 : k - 1;
  const int row = (j * nz + k) * nx;
  const double gx = (lx[row + im] - lx[row + ip]) * E.inv_2dx;
  const double gz = (lz[(j * nz + km) * nx + i] - lz[(j * nz + kp) * nx + i]) * E.inv_2dz;
  const double* beta = C.beta + E.y_off;
  const double* idy = C.idy + E.y_off;
  const int nxz = nx * nz;
  double gy = 0.0;
  double diag = 0.0;
  if (j <= ny - 2) diag += 1.0 - beta[j + 1];
  if (j >= 1) diag -= beta[j];
  gy += ly[cl] * diag * idy[j];
  if (j >= 1) gy += ly[cl - nxz] * beta[j] * idy[j - 1];
  if (j <= ny - 2) gy -= ly[cl + nxz] * (1.0 - beta[j + 1]) * idy[j + 1];
  W.radj[cg] = -(gx + gy + gz);
}

__global__ __launch_bounds__(kBlock) void k_adj_b(Ctx C, Ens Eone, int one, PState in, AdjWork W, AdjLam lam0) {
  const int s = blockIdx.x * kBlock + threadIdx.x;
  const bool act = s < C.n_tot;
  (void)Eone;
  (void)one;
  const long long n = C.n_tot;
  const int c = act ? C.skey[s] : 0x7fffffff;
  // as in the push: the cell mates' positions, charges and lambda_S from
  // their lanes, those of cells across the wave's ends from memory (their
  // old slots read here for the 32 slots on either side), ascending id
  const int lane = (int)(threadIdx.x & 63u);
  const int s0 = s - lane;
  int pm = 0;
  {
    const int t = lane < 32 ? s0 - 1 - lane : s0 + 64 + (lane - 32);
    if (t >= 0 && t < C.n_tot) pm = C.perm[t];
  }
  int a, b;
  cell_run(s, c, &a, &b);
  if (!act) return;
  const int p = C.perm[s];
  if (a < 0) a = C.start[c];
  if (b < 0) b = C.start[c + 1];
  double lpx = W.lamP.x[s], lpy = W.lamP.y[s], lpz = W.lamP.z[s];
  double lq = W.lamP.q[s] + W.lamQ[c];
  const double x = in.x[p], y = in.y[p], z = in.z[p], q = in.q[p];
  const double lsx = W.lamS[s], lsy = W.lamS[n + s], lsz = W.lamS[2 * n + s];
  const int nm = b - a;
  for (int kk = 0; __any(kk < nm); ++kk) {
    const int t = a + kk, src = t - s0;
    double ox = __shfl(x, src & 63, 64), oy = __shfl(y, src & 63, 64);
    double oz = __shfl(z, src & 63, 64), qt = __shfl(q, src & 63, 64);
    double ltx = __shfl(lsx, src & 63, 64), lty = __shfl(lsy, src & 63, 64), ltz = __shfl(lsz, src & 63, 64);
    const int hb = s0 - 1 - t, ta = t - s0 - 64;
    const int pmv = __shfl(pm, hb >= 0 ? (hb & 31) : 32 + (ta & 31), 64);
    if (!(kk < nm) || t == s) continue;
    if (!(src >= 0 && src < 64)) {
      const int pt = (hb >= 0 && hb < 32) || (ta >= 0 && ta < 32) ? pmv : C.perm[t];
      ox = in.x[pt];
      oy = in.y[pt];
      oz = in.z[pt];
      qt = in.q[pt];
      ltx = W.lamS[t];
      lty = W.lamS[n + t];
      ltz = W.lamS[2 * n + t];
    }
    const double rx = x - ox, ry = y - oy, rz = z - oz;
    const double r2 = (rx * rx + ry * ry) + rz * rz;
    if (r2 > 0.0) {
      const double ri = rsqrt(r2);
      const double inv3 = ri * ri * ri;
      const double inv5 = inv3 * ri * ri;
      // S_t contains q_s (x_t - x_s)/|r|^3
      lq -= (ltx * rx + lty * ry + ltz * rz) * inv3;
      // d S_s / d x_s and d S_t / d x_s: J(r) (q_t lambda_S_s - q_s lambda_S_t)
      const double wx = qt * lsx - q * ltx, wy = qt * lsy - q * lty, wz = qt * lsz - q * ltz;
      const double rw = rx * wx + ry * wy + rz * wz;
      lpx += wx * inv3 - 3.0 * rx * rw * inv5;
      lpy += wy * inv3 - 3.0 * ry * rw * inv5;
      lpz += wz * inv3 - 3.0 * rz * rw * inv5;
    }
  }
  lam0.x[p] = lpx;
  lam0.y[p] = lpy;
  lam0.z[p] = lpz;
  lam0.vx[p] = W.lamP.vx[s];
  lam0.vy[p] = W.lamP.vy[s];
  lam0.vz[p] = W.lamP.vz[s];
  lam0.q[p] = lq;
}

// d/dtheta of each ensemble, summed in a fixed order (deterministic) in two
// stages: block (c, e) sums chunk c (kAdjChunk slots) of ensemble e, then one
// wavefront per ensemble sums its chunks
__global__ __launch_bounds__(kBlock) void k_adj_part(const double* __restrict__ dth, long long n,
                                                     const long long* __restrict__ p_off, int nch,
                                                     double* __restrict__ part) {
  __shared__ double red[3][kBlock];
  const int c = blockIdx.x, e = blockIdx.y;
  const long long n0 = p_off[e] + (long long)c * kAdjChunk;
  const long long n1 = min(p_off[e + 1], n0 + kAdjChunk);
  double a0 = 0.0, a1 = 0.0, a2 = 0.0;
  for (long long s = n0 + threadIdx.x; s < n1; s += kBlock) {
    a0 += dth[s];
    a1 += dth[n + s];
    a2 += dth[2 * n + s];
  }
  red[0][threadIdx.x] = a0;
  red[1][threadIdx.x] = a1;
  red[2][threadIdx.x] = a2;
  __syncthreads();
  for (int o = kBlock / 2; o > 0; o >>= 1) {
    if (threadIdx.x < o) {
      red[0][threadIdx.x] += red[0][threadIdx.x + o];
      red[1][threadIdx.x] += red[1][threadIdx.x + o];
      red[2][threadIdx.x] += red[2][threadIdx.x + o];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    double* o = part + 3 * ((long long)e * nch + c);
    o[0] = red[0][0];
    o[1] = red[1][0];
    o[2] = red[2][0];
  }
}

__global__ __launch_bounds__(64) void k_adj_sum(const double* __restrict__ part, int nch, double* __restrict__ dacc) {
  const int e = blockIdx.x, lane = threadIdx.x;
  double a[3] = {0.0, 0.0, 0.0};
  for (int c = lane; c < nch; c += 64)
#pragma unroll
    for (int k = 0; k < 3; ++k) a[k] += part[3 * ((long long)e * nch + c) + k];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    for (int o = 32; o > 0; o >>= 1) a[k] += __shfl_xor(a[k], o, 64);
    if (lane == 0) dacc[3 * e + k] += a[k];
  }
}

struct UserLam {
  double *x, *y, *z, *vx, *vy, *vz, *q;
};

// lambda of the final recorded state from id order into slot order
__global__ __launch_bounds__(kBlock) void k_lam_in(AdjLam lam, UserLam u, const int* __restrict__ id, long long p0,
                                                   int np) {
  const int t = blockIdx.x * kBlock + threadIdx.x;
  if (t >= np) return;
  const long long s = p0 + t;
  const int k = id[s];
  lam.x[s] = u.x[k];
  lam.y[s] = u.y[k];
  lam.z[s] = u.z[k];
  lam.vx[s] = u.vx[k];
  lam.vy[s] = u.vy[k];
  lam.vz[s] = u.vz[k];
  lam.q[s] = u.q[k];
}

// lambda of the first recorded state from slot order back to id order
__global__ __launch_bounds__(kBlock) void k_lam_out(AdjLam lam, UserLam u, const int* __restrict__ id, long long p0,
                                                    int np) {
  const int t = blockIdx.x * kBlock + threadIdx.x;
  if (t >= np) return;
  const long long s = p0 + t;
  const int k = id[s];
  u.x[k] = lam.x[s];
  u.y[k] = lam.y[s];
  u.z[k] = lam.z[s];
  u.vx[k] = lam.vx[s];
  u.vy[k] = lam.vy[s];
  u.vz[k] = lam.vz[s];
  u.q[k] = lam.q[s];
}

hipError_t run_adjoint(const Ctx& C0, const LaunchGeo& G, const AdjWork& W, int n_ens, const Ens* eh,
                       const long long* p_off, const long long* c_off, const TrajStep* steps, int T,
                       const double* const* lambda, const double* w_wall, double* dtheta, hipStream_t st) {
  (void)c_off;
  hipError_t err;
  if (!W.enabled) return hipErrorNotSupported;
  const long long n = C0.n_tot, nc = C0.c_tot;
  const int one = (n_ens == 1) ? 1 : 0;
  const Ens Eone = eh[0];
  if ((err = hipMemcpyAsync(W.wwall, w_wall, sizeof(double) * 2 * n_ens, hipMemcpyDeviceToDevice, st)) != hipSuccess)
    return err;
  if (n > 0 && (err = hipMemsetAsync(W.dth, 0, sizeof(double) * 3 * n, st)) != hipSuccess) return err;
  AdjLam cur = W.lamA, nxt = W.lamB;
  for (int e = 0; e < n_ens; ++e) {
    const int np = (int)(p_off[e + 1] - p_off[e]);
    if (np == 0) continue;
    const double* const* L = lambda + 8 * e;
    UserLam u{(double*)L[0], (double*)L[1], (double*)L[2], (double*)L[3], (double*)L[4], (double*)L[5], (double*)L[6]};
    k_lam_in<<<(np + kBlock - 1) / kBlock, kBlock, 0, st>>>(cur, u, steps[T].st.id, p_off[e], np);
  }
  const int nb = (int)((n + kBlock - 1) / kBlock);
  const int nbc = (int)((nc + kBlock - 1) / kBlock);
  for (int t = T - 1; t >= 0; --t) {
    Ctx C = C0;
    C.perm = steps[t].perm;
    C.skey = steps[t].skey;
    C.start = steps[t].start;
    C.phi = steps[t].phi;
    if (nb > 0) k_adj_a<<<nb, kBlock, 0, st>>>(C, Eone, one, steps[t].st, cur, W, steps[t].wall);
    k_adj_ecell<<<nbc, kBlock, 0, st>>>(C, W);
    k_adj_div<<<nbc, kBlock, 0, st>>>(C, Eone, one, W);
    if ((err = launch_poisson(C, G, 0, n_ens, nullptr, nullptr, nullptr, 0, W.lamQ, 0, 0, st, nullptr, W.radj)) !=
        hipSuccess)
      return err;
    if (nb > 0) k_adj_b<<<nb, kBlock, 0, st>>>(C, Eone, one, steps[t].st, W, nxt);
    AdjLam tmp = cur;
    cur = nxt;
    nxt = tmp;
  }
  // d/dtheta of the segment: the per-slot sums over its steps, per ensemble
  // (added to the caller's device dtheta)
  if (W.nch > 0) {
    k_adj_part<<<dim3(W.nch, n_ens), kBlock, 0, st>>>(W.dth, n, C0.p_off, W.nch, W.part);
    k_adj_sum<<<n_ens, 64, 0, st>>>(W.part, W.nch, dtheta);
  }
  for (int e = 0; e < n_ens; ++e) {
    const int np = (int)(p_off[e + 1] - p_off[e]);
    if (np == 0) continue;
    const double* const* L = lambda + 8 * e;
    UserLam u{(double*)L[0], (double*)L[1], (double*)L[2], (double*)L[3], (double*)L[4], (double*)L[5], (double*)L[6]};
    k_lam_out<<<(np + kBlock - 1) / kBlock, kBlock, 0, st>>>(cur, u, steps[0].st.id, p_off[e], np);
  }
  return hipGetLastError();
}

}  // namespace tf
