// C ABI of libtribo.so: configuration checks, workspace layout, host tables,
// step orchestration (eager or replayed from captured HIP graphs).
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <tuple>
#include <string>
#include <vector>

#include "../../include/tribo.h"
#include "adjoint.h"
#include "launch.h"
#include "tribo_dev.h"

using namespace tf;

namespace {

thread_local std::string g_err;
thread_local const char* g_err_lit = nullptr;  // set by fail_lit (no allocation), cleared by fail
tf_tuning g_tune = {0, 0, 0, 0, 0};
std::map<std::tuple<int, int, int>, tf_tuning> g_class_tune;  // per (nx, ny, nz)

int fail(int code, const std::string& msg) {
  g_err = msg;
  g_err_lit = nullptr;
  return code;
}

// the same with a string literal, for entry points that must not allocate
int fail_lit(int code, const char* msg) {
  g_err_lit = msg;
  return code;
}

#define HIPCHK(expr)                                                                         \
  do {                                                                                       \
    hipError_t e_ = (expr);                                                                  \
    if (e_ != hipSuccess) return fail(TF_EHIP, std::string(#expr) + ": " + hipGetErrorString(e_)); \
  } while (0)

bool radix_plan(int n, FftPlan* P) {
  P->n = n;
  P->npass = 0;
  P->rcode = 0;
  int m = n;
  auto push = [&](int r) {
    if (P->npass >= kMaxPass) return false;
    P->rcode |= (unsigned)r << (3 * P->npass++);
    m /= r;
    return true;
  };
  while (m % 4 == 0) if (!push(4)) return false;
  while (m % 2 == 0) if (!push(2)) return false;
  while (m % 3 == 0) if (!push(3)) return false;
  while (m % 5 == 0) if (!push(5)) return false;
  if (m != 1) return false;
  // in-place plan (fused inverse transforms): largest radices first
  P->np_ip = 0;
  P->rc_ip = 0;
  m = n;
  for (int r : {16, 8, 4, 2, 3, 5})
    while (m % r == 0) {
      if (P->np_ip >= 8) return false;
      P->rc_ip |= (unsigned)(r - 1) << (4 * P->np_ip++);
      m /= r;
    }
  return m == 1;
}

struct Sizes {
  long long n_tot = 0, c_tot = 0, s_tot = 0, rows = 0, np_max = 0;
  int y_tot = 0, kx_tot = 0, kz_tot = 0, tw_tot = 0, st_tot = 0;
  int nx_max = 0, nz_max = 0, ny_max = 0, wz = 8, tri_rows = 1;
  int sort_cap = 0;             // member capacity of the fused sort for this handle
  int push_order = 0;           // the push's block order over the XCDs (tf_tuning.push_order)
  long long tf_tot = 0;         // tridiagonal factors (double2 per mode and y row)
  std::vector<int> tf_src;      // ensemble whose factor table an ensemble uses (the first of its mesh)
  long long up_tot = 0;         // padded carrier copies (doubles)
  std::vector<int> e_wz, e_tm;  // per-ensemble tile shapes
  std::vector<int> fp_blk, fz_blk, tri_blk, pl_blk, ph_blk, pq_blk;
  std::vector<int> fps_blk, fzs_blk;  // the same as fp_blk / fz_blk for the ensembles with split inverse transforms
  int plane_max = 0, half_lds = 0, quarter_lds = 0;
  bool plane_any = false, half_any = false, quarter_any = false, split_any = false;
  bool pp_any = false;  // some ensemble has 4-way coupling on
  std::vector<int> e_plane;
  std::map<int, int> tw_off;
};

int check_config(const tf_ensemble* ens, int n_ens, Sizes* S) {
  if (!ens || n_ens < 1 || n_ens > 4096) return fail(TF_EINVAL, "n_ens must be in [1, 4096]");
  S->tf_src.clear();
  S->fp_blk.assign(n_ens + 1, 0);
  S->fz_blk.assign(n_ens + 1, 0);
  S->pl_blk.assign(n_ens + 1, 0);
  S->ph_blk.assign(n_ens + 1, 0);
  S->pq_blk.assign(n_ens + 1, 0);
  S->fps_blk.assign(n_ens + 1, 0);
  S->fzs_blk.assign(n_ens + 1, 0);
  S->tri_blk.assign(n_ens + 1, 0);
  for (int e = 0; e < n_ens; ++e) {
    const tf_ensemble& E = ens[e];
    FftPlan P;
    auto okn = [&](int n) { return n >= 4 && n <= 256 && n % 2 == 0 && radix_plan(n, &P); };
    char buf[160];
    snprintf(buf, sizeof buf, "ensemble %d: ", e);
    std::string pre(buf);
    if (!okn(E.nx) || !okn(E.nz)) return fail(TF_EINVAL, pre + "nx, nz must be even 2^a 3^b 5^c in [4, 256]");
    if (E.ny < 2 || E.ny > 1024) return fail(TF_EINVAL, pre + "ny must be in [2, 1024]");
    if (E.n_particles < 0 || E.n_particles > (1 << 30)) return fail(TF_EINVAL, pre + "n_particles out of range");
    if (!(E.lx > 0) || !(E.lz > 0) || !(E.dt > 0) || !(E.density_ratio > 0) || !(E.un_bin > 0))
      return fail(TF_EINVAL, pre + "lx, lz, dt, density_ratio, un_bin must be positive");
    if (!(E.e > 0 && E.e <= 1)) return fail(TF_EINVAL, pre + "restitution e must be in (0, 1]");
    if (!std::isfinite(E.k_c) || !std::isfinite(E.delta_u) || !std::isfinite(E.c_el))
      return fail(TF_EINVAL, pre + "k_c, delta_u, c_el must be finite");
    if ((E.pp != 0 && E.pp != 1) || !(E.k_pp >= 0) || !std::isfinite(E.k_pp))
      return fail(TF_EINVAL, pre + "pp must be 0 or 1 and k_pp finite and >= 0");
    if (E.pp) S->pp_any = true;
    if (E.charging != 0 && E.charging != 1) return fail(TF_EINVAL, pre + "charging must be 0 or 1");
    if (E.charging == 1 &&
        !(std::isfinite(E.ssm_dq0min) && std::isfinite(E.ssm_mu0) && std::isfinite(E.ssm_gamma0) &&
          E.ssm_sigma0 >= 0 && std::isfinite(E.ssm_sigma0) && E.ssm_csat != 0 && std::isfinite(E.ssm_csat) &&
          E.ssm_d0 > 0 && std::isfinite(E.ssm_d0) && E.ssm_un0 > 0 && std::isfinite(E.ssm_un0)))
      return fail(TF_EINVAL, pre + "SSM parameters: finite, sigma0 >= 0, csat != 0, d0 > 0, un0 > 0");
    if (!E.y_faces) return fail(TF_EINVAL, pre + "y_faces is NULL");
    if (!E.u_nodes) return fail(TF_EINVAL, pre + "u_nodes is NULL");
    if (E.y_faces[0] != 0.0) return fail(TF_EINVAL, pre + "y_faces[0] must be 0");
    for (int j = 0; j < E.ny; ++j)
      if (!(E.y_faces[j + 1] > E.y_faces[j])) return fail(TF_EINVAL, pre + "y_faces must increase strictly");
    long long ncell = (long long)E.nx * E.ny * E.nz;
    int nh = E.nx / 2 + 1, nhp = (nh + 7) & ~7;
    S->n_tot += E.n_particles;
    S->np_max = std::max<long long>(S->np_max, E.n_particles);
    S->c_tot += ncell;
    S->s_tot += (long long)E.ny * E.nz * nhp;
    // ensembles on the same mesh (sizes, lengths, y faces) share one factor table
    int src = e;
    for (int o = 0; o < e && src == e; ++o) {
      const tf_ensemble& F = ens[o];
      if (F.nx == E.nx && F.ny == E.ny && F.nz == E.nz && F.lx == E.lx && F.lz == E.lz &&
          std::memcmp(F.y_faces, E.y_faces, sizeof(double) * (E.ny + 1)) == 0)
        src = S->tf_src[o];
    }
    S->tf_src.push_back(src);
    // the factors depend on kz^2, the same for modes mz and nz - mz: rows mz <= nz / 2
    if (src == e) S->tf_tot += (long long)E.ny * (E.nz / 2 + 1) * nh;
    S->up_tot += 3LL * (E.ny + 1) * E.nz * (E.nx + 2);
    S->rows += (long long)E.ny * E.nz;
    S->y_tot += E.ny + 1;
    S->kx_tot += nh;
    S->kz_tot += E.nz;
    S->st_tot += stats_len(E.ny);
    S->nx_max = std::max(S->nx_max, E.nx);
    S->nz_max = std::max(S->nz_max, E.nz);
    S->ny_max = std::max(S->ny_max, E.ny);
    for (int n : {E.nx, E.nz})
      if (!S->tw_off.count(n)) {
        S->tw_off[n] = S->tw_tot;
        S->tw_tot += n;
      }
  }
  if (S->n_tot >= (1LL << 31) || S->c_tot >= (1LL << 31) - 2) return fail(TF_ESIZE, "too many particles or cells");
  // tridiagonal: tm modes per block, G = kBlock / tm lanes per mode, rows per
  // lane R = ceil(ny / G) <= 16 (one launch uses the largest R)
  S->e_wz.assign(n_ens, 2);
  S->e_tm.assign(n_ens, 1);
  S->e_plane.assign(n_ens, 0);
  std::vector<int> want_plane(n_ens, 0);
  S->wz = 1;
  S->tri_rows = 1;
  // the fused sort holds one member capacity per handle: the global choice,
  // else the one set for the mesh class when every ensemble has that mesh
  // (a batch of several classes takes the built-in rule over the whole batch)
  S->sort_cap = g_tune.sort_cap;
  S->push_order = g_tune.push_order;
  bool one_class = true;
  for (int e = 1; e < n_ens; ++e)
    one_class = one_class && ens[e].nx == ens[0].nx && ens[e].ny == ens[0].ny && ens[e].nz == ens[0].nz;
  for (int e = 0; e < n_ens; ++e) {
    const tf_ensemble& E = ens[e];
    tf_tuning t = g_tune;
    auto it = g_class_tune.find(std::make_tuple(E.nx, E.ny, E.nz));
    if (it != g_class_tune.end()) {
      if (it->second.fz_cols > 0) t.fz_cols = it->second.fz_cols;
      if (it->second.tri_modes > 0) t.tri_modes = it->second.tri_modes;
      if (it->second.inv_plane > 0) t.inv_plane = it->second.inv_plane;
      if (g_tune.sort_cap == 0 && one_class && it->second.sort_cap > 0) S->sort_cap = it->second.sort_cap;
      if (g_tune.push_order == 0 && one_class && it->second.push_order > 0) S->push_order = it->second.push_order;
    }
    want_plane[e] = t.inv_plane;
    const int wz = t.fz_cols > 0 ? t.fz_cols : 2;
    // default: the fewest lanes (at least 8) that keep R <= 8
    int lanes = 8;
    while (lanes < 64 && lanes * 8 < E.ny) lanes *= 2;
    const int tm = t.tri_modes > 0 ? t.tri_modes : kBlock / lanes;
    if (tm != 4 && tm != 8 && tm != 16 && tm != 32) return fail(TF_EINVAL, "tri_modes must be 4, 8, 16 or 32");
    const int rows = (E.ny + kBlock / tm - 1) / (kBlock / tm);
    if (rows > 16) return fail(TF_ESIZE, "tri_modes too large for ny (more than 16 rows per lane)");
    if (wz * E.nz > kZPts) return fail(TF_ESIZE, "fz_cols times nz exceeds the z-transform tile (2048 points)");
    S->e_wz[e] = wz;
    S->e_tm[e] = tm;
    S->wz = std::max(S->wz, wz);
    S->tri_rows = std::max(S->tri_rows, rows);
  }
  // push block order: a handle of several mesh classes (small ensembles
  // side by side) takes the round robin
  if (S->push_order == 0 && !one_class) S->push_order = 2;
  const size_t lds_fx = (size_t)9 * S->nx_max * 16;  // twiddles + 4 waves x 2 line buffers
  const size_t lds_fz = (size_t)(S->wz * S->nz_max + S->nz_max) * 16;
  const size_t lds_tri = ((size_t)kBlock * (S->tri_rows | 1) + kBlock) * 16;
  if (lds_fx > 65536 || lds_fz > (size_t)kLdsMax || lds_tri > (size_t)kLdsMax)
    return fail(TF_ESIZE, "tile shapes exceed the LDS of a block");
  for (int e = 0; e < n_ens; ++e) {
    const tf_ensemble& E = ens[e];
    int rows = E.ny * E.nz, nh = E.nx / 2 + 1;
    S->fp_blk[e + 1] = S->fp_blk[e] + (rows / 2 + 3) / 4;  // row pairs, 4 per block
    S->fz_blk[e + 1] = S->fz_blk[e] + E.ny * ((nh + S->e_wz[e] - 1) / S->e_wz[e]);
    S->tri_blk[e + 1] = S->tri_blk[e] + (((nh + 7) & ~7) * E.nz + S->e_tm[e] - 1) / S->e_tm[e];
  }
  // inverse transforms: per y plane in one block when the plane's half
  // spectrum and twiddles fit its LDS, in two blocks (z-row parity) when half
  // of it does.  By default the two-block form when an ensemble's 2 ny blocks
  // do not outnumber the CUs (it then keeps twice as many CUs busy at the cost
  // of a second read of each plane), else one block, else the z and x kernels.
  int cus = 256, dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) !=
                                              hipSuccess || cus < 1) {
    (void)hipGetLastError();
    cus = 256;
  }
  for (int e = 0; e < n_ens; ++e) {
    const tf_ensemble& E = ens[e];
    const int nh = E.nx / 2 + 1, pts = E.nz * nh, hpts = (E.nz / 2) * nh;
    const bool whole_ok = pts <= kPlanePts && (size_t)(S->nx_max + S->nz_max + pts) * 16 <= (size_t)kLdsMax;
    const size_t hlds = (size_t)(E.nx + E.nz / 2 + hpts) * 16;
    FftPlan P;
    const bool half_ok = E.nz % 4 == 0 && hpts <= kHalfPts && (E.nz / 4) * E.nx <= kHalfXPts &&
                         hlds <= (size_t)kLdsMax && radix_plan(E.nz / 2, &P);
    const int qpts = (E.nz / 4) * nh;
    const size_t qlds = (size_t)(E.nx + E.nz / 4 + qpts) * 16;
    const bool quarter_ok = E.nz % 8 == 0 && qpts <= kHalfPts && (E.nz / 8) * E.nx <= kQuarterXPts &&
                            qlds <= (size_t)kLdsMax && radix_plan(E.nz / 4, &P);
    int m;
    switch (want_plane[e]) {
      case 1: m = 1; if (!whole_ok) return fail(TF_ESIZE, "inv_plane 1: the plane exceeds a block's LDS"); break;
      case 2: m = 2; if (!half_ok) return fail(TF_ESIZE, "inv_plane 2: needs nz % 4 == 0 and half a plane within a block"); break;
      case 3: m = 0; break;
      case 4: m = 4; if (!quarter_ok) return fail(TF_ESIZE, "inv_plane 4: needs nz % 8 == 0 and a quarter plane within a block"); break;
      default: m = (half_ok && 2 * E.ny <= cus) ? 2 : whole_ok ? 1 : quarter_ok ? 4 : 0; break;
    }
    S->e_plane[e] = m;
    S->pl_blk[e + 1] = S->pl_blk[e] + (m == 1 ? E.ny : 0);
    S->ph_blk[e + 1] = S->ph_blk[e] + (m == 2 ? 2 * E.ny : 0);
    S->pq_blk[e + 1] = S->pq_blk[e] + (m == 4 ? 4 * E.ny : 0);
    S->fps_blk[e + 1] = S->fps_blk[e] + (m == 0 ? S->fp_blk[e + 1] - S->fp_blk[e] : 0);
    S->fzs_blk[e + 1] = S->fzs_blk[e] + (m == 0 ? S->fz_blk[e + 1] - S->fz_blk[e] : 0);
    if (m == 1) {
      S->plane_any = true;
      S->plane_max = std::max(S->plane_max, pts);
    } else if (m == 2) {
      S->half_any = true;
    } else if (m == 4) {
      S->quarter_any = true;
    } else {
      S->split_any = true;
    }
  }
  // one LDS size for the half-plane launch: the largest pieces over its ensembles
  int hx = 0, hz = 0, hp = 0;
  for (int e = 0; e < n_ens; ++e)
    if (S->e_plane[e] == 2) {
      hx = std::max(hx, ens[e].nx);
      hz = std::max(hz, ens[e].nz / 2);
      hp = std::max(hp, (ens[e].nz / 2) * (ens[e].nx / 2 + 1));
    }
  S->half_lds = (hx + hz + hp) * 16;
  if ((size_t)S->half_lds > (size_t)kLdsMax) return fail(TF_ESIZE, "half-plane tiles exceed the LDS of a block");
  int qx = 0, qz = 0, qp = 0;
  for (int e = 0; e < n_ens; ++e)
    if (S->e_plane[e] == 4) {
      qx = std::max(qx, ens[e].nx);
      qz = std::max(qz, ens[e].nz / 4);
      qp = std::max(qp, (ens[e].nz / 4) * (ens[e].nx / 2 + 1));
    }
  S->quarter_lds = (qx + qz + qp) * 16;
  if ((size_t)S->quarter_lds > (size_t)kLdsMax)
    return fail(TF_ESIZE, "quarter-plane tiles exceed the LDS of a block");
  return TF_OK;
}

// Spectrum scratch of tf_poisson_noalloc: a file-scope device array, one
// copy per GPU, held until the process ends.  Host code never passes the
// array's name to a kernel (on the host it is only a stand-in for the symbol):
// its device address comes from hipGetSymbolAddress, taken once per device
// with that device current, and kept in g_scratch.
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch[kMaxDevices] = {};

}  // namespace

static __device__ __align__(256) double2 scratch[TF_NOALLOC_MAX_SPECTRUM_BYTES / sizeof(double2)];

namespace {

// device address of `scratch` on the current device (looked up once per device)
int scratch_address(void** out) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess) return fail(TF_EHIP, "hipGetDevice failed");
  if (dev < 0 || dev >= kMaxDevices) return fail(TF_EINVAL, "device index beyond the scratch table");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return fail(TF_EHIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    g_scratch[dev] = p;
  }
  *out = g_scratch[dev];
  return TF_OK;
}

}  // namespace

struct TrajBuf {
  PState st;
  int* perm;
  int* skey;
  int* start;
  double* phi;
  signed char* wall;
};

struct tf_handle {
  int n_ens = 0;
  uint32_t flags = 0;
  hipStream_t stream = nullptr;
  Sizes S;
  std::vector<Ens> eh;              // host copies of the ensemble descriptors
  std::vector<long long> p_off, c_off;
  Ctx C{};
  LaunchGeo G{};
  Ens* d_ens = nullptr;
  PState A{}, B{}, cur{};
  bool cur_is_A = true;
  bool need_full = true;            // next sort from scratch (stored order is not a push's)
  int* d_fx = nullptr;
  int* d_fz = nullptr;
  int* d_tri = nullptr;
  int* d_pl = nullptr;
  int* d_ph = nullptr;
  int* d_pq = nullptr;
  int* d_fps = nullptr;
  int* d_fzs = nullptr;
  // recorded trajectory
  int traj_cap = 0, traj_len = 0;
  std::vector<TrajBuf> traj;        // traj_cap + 1 states (perm/phi used for the first traj_cap)
  AdjWork adj{};
  // graphs: one step A->B and one B->A
  hipGraphExec_t g_ab = nullptr, g_ba = nullptr;
  // this device's copy of the static spectrum scratch (tf_poisson_noalloc)
  double2* scratch = nullptr;
  // phase timing: TF_NPHASE + 1 events per profiled step
  int prof_cap = 0, prof_n = 0;
  int prof_every = 1, prof_seen = 0;  // events on every prof_every-th step
  uint32_t prof_mask = 0;           // phases bracketed by events
  std::vector<hipEvent_t> prof_ev;
};

namespace {

PState carve_state(Carver& cv, long long n) {
  PState s;
  double** f[8] = {&s.x, &s.y, &s.z, &s.vx, &s.vy, &s.vz, &s.q, &s.d};
  for (auto* p : f) *p = cv.take<double>(n);
  s.id = cv.take<int>(n);
  s.key = cv.take<int>(n);
  return s;
}

// Lay out every device array; with h == nullptr only the size is computed.
size_t layout(const Sizes& S, int n_ens, int traj_steps, uint32_t flags, void* base, tf_handle* h) {
  Carver cv(base);
  Ctx C{};
  C.ens = cv.take<Ens>(n_ens);
  C.p_off = cv.take<long long>(n_ens + 1);
  C.c_off = cv.take<long long>(n_ens + 1);
  int* fx = cv.take<int>(n_ens + 1);
  int* fz = cv.take<int>(n_ens + 1);
  int* tri = cv.take<int>(n_ens + 1);
  int* pl = cv.take<int>(n_ens + 1);
  int* ph = cv.take<int>(n_ens + 1);
  int* pq = cv.take<int>(n_ens + 1);
  int* fps = cv.take<int>(n_ens + 1);
  int* fzs = cv.take<int>(n_ens + 1);
  C.yf = cv.take<double>(S.y_tot);
  C.dy = cv.take<double>(S.y_tot);
  C.idy = cv.take<double>(S.y_tot);
  C.vol = cv.take<double>(S.y_tot);
  C.am = cv.take<double>(S.y_tot);
  C.ap = cv.take<double>(S.y_tot);
  C.beta = cv.take<double>(S.y_tot);
  C.kx2 = cv.take<double>(S.kx_tot);
  C.kz2 = cv.take<double>(S.kz_tot);
  C.tw = cv.take<double2>(S.tw_tot);
  C.tfac = cv.take<double2>(S.tf_tot);
  C.stats = cv.take<long long>(S.st_tot);
  C.rowq = cv.take<long long>(S.rows);
  C.rowacc = cv.take<longlong2>(S.rows);
  C.r_off = cv.take<long long>(n_ens + 1);
  C.n_rows = S.rows;
  C.pair_cnt = cv.take<int>(S.rows / 2);
  C.ps = cv.take<int>(S.rows / 2 + 1);
  C.rs_old = cv.take<int>(S.rows + 1);
  C.rs_new = cv.take<int>(S.rows + 1);
  C.mv = cv.take<int>((size_t)(S.rows / 2) * kMoverCap);
  C.mv_n = cv.take<int>(S.rows / 2);
  C.far = cv.take<int>(S.n_tot);
  C.far_n = cv.take<int>(2);
  C.uptr = cv.take<const double*>(n_ens);
  C.upad = cv.take<double>(S.up_tot);
  PState A = carve_state(cv, S.n_tot);
  PState B = carve_state(cv, S.n_tot);
  C.count = cv.take<int>(S.c_tot);
  C.start = cv.take<int>(S.c_tot + 1);
  C.tmp = cv.take<int4>(S.n_tot);
  C.perm = cv.take<int>(S.n_tot);
  C.skey = cv.take<int>(S.n_tot);
  C.sq = cv.take<double>(S.n_tot);
  const long long nbs = (S.c_tot + 4 * kBlock - 1) / (4 * kBlock);
  C.scan_part = cv.take<int>(nbs + 1);
  C.spec = cv.take<double2>(S.s_tot);
  C.phi = cv.take<double>(S.c_tot);
  C.qdep = (flags & TF_INIT_KEEP_DEPOSIT) ? cv.take<long long>(S.c_tot) : nullptr;
  C.fslot = (flags & TF_INIT_SOURCE) ? cv.take<double>(3 * S.n_tot) : nullptr;
  C.fsrc = (flags & TF_INIT_SOURCE) ? cv.take<double>(3 * S.c_tot) : nullptr;
  C.cinc = S.pp_any ? cv.take<double>(4 * S.n_tot) : nullptr;
  C.chit = S.pp_any ? cv.take<unsigned char>(S.n_tot) : nullptr;
  std::vector<TrajBuf> traj;
  if (traj_steps > 0) {
    for (int t = 0; t <= traj_steps; ++t) {
      TrajBuf tb;
      tb.st = carve_state(cv, S.n_tot);
      const bool last = (t == traj_steps);
      tb.perm = last ? nullptr : cv.take<int>(S.n_tot);
      tb.skey = last ? nullptr : cv.take<int>(S.n_tot);
      tb.start = last ? nullptr : cv.take<int>(S.c_tot + 1);
      tb.phi = last ? nullptr : cv.take<double>(S.c_tot);
      tb.wall = last ? nullptr : cv.take<signed char>(S.n_tot);
      traj.push_back(tb);
    }
  }
  AdjWork adj = carve_adjoint(cv, S.n_tot, S.c_tot, S.s_tot, n_ens, S.np_max, traj_steps > 0);
  if (h) {
    C.n_ens = n_ens;
    C.n_tot = S.n_tot;
    C.c_tot = S.c_tot;
    h->C = C;
    h->A = A;
    h->B = B;
    h->d_fx = fx;
    h->d_fz = fz;
    h->d_tri = tri;
    h->d_pl = pl;
    h->d_ph = ph;
    h->d_pq = pq;
    h->d_fps = fps;
    h->d_fzs = fzs;
    h->d_ens = (Ens*)C.ens;
    h->traj = traj;
    h->traj_cap = traj_steps;
    h->adj = adj;
  }
  return cv.off + 256;
}

void destroy_graphs(tf_handle* h) {
  if (h->g_ab) hipGraphExecDestroy(h->g_ab);
  if (h->g_ba) hipGraphExecDestroy(h->g_ba);
  h->g_ab = h->g_ba = nullptr;
}

hipError_t enqueue_step(tf_handle* h, const PState& in, const PState& out, const TrajBuf* rec, bool full = false) {
  hipError_t e;
  // phase-boundary events of a profiled step: boundary b opens phase b and
  // closes phase b - 1; only the boundaries of the bracketed phases are recorded
  hipEvent_t ev[TF_NPHASE + 1] = {};
  bool prof = false;
  if (h->prof_n < h->prof_cap && (h->prof_seen++ % h->prof_every) == 0) {
    hipEvent_t* all = &h->prof_ev[(size_t)h->prof_n++ * (TF_NPHASE + 1)];
    for (int b = 0; b <= TF_NPHASE; ++b) {
      const bool opens = b < TF_NPHASE && ((h->prof_mask >> b) & 1u);
      const bool closes = b > 0 && ((h->prof_mask >> (b - 1)) & 1u);
      if (opens || closes) ev[b] = all[b];
    }
    prof = true;
  }
  if (ev[0] && (e = hipEventRecord(ev[0], h->stream)) != hipSuccess) return e;
  // full: counting sort, then deposit + x transform from the sorted runs;
  // incremental: row scan, then the fused sort + deposit + x transform
  if ((e = launch_sort(h->C, h->G, in, full, h->stream)) != hipSuccess) return e;
  if (ev[1] && (e = hipEventRecord(ev[1], h->stream)) != hipSuccess) return e;
  if (!full && (e = launch_sort_dep(h->C, h->G, in, h->stream)) != hipSuccess) return e;
  if ((e = launch_poisson(h->C, h->G, 0, h->n_ens, in.q, in.key, nullptr, 0, h->C.phi, 0, 1, h->stream,
                          prof ? ev + 2 : nullptr, nullptr, !full, h->C.far_n)) != hipSuccess)
    return e;
  if (rec && (e = launch_record(rec->skey, h->C.skey, h->C.n_tot, rec->start, h->C.start, rec->phi, h->C.phi,
                                h->C.c_tot, h->stream)) != hipSuccess)
    return e;
  if (h->C.cinc && (e = launch_collide(h->C, h->G.eh[0], in, h->stream)) != hipSuccess) return e;
  if ((e = launch_push(h->C, h->G, in, out, rec ? rec->perm : nullptr, rec ? rec->wall : nullptr, h->stream)) !=
      hipSuccess)
    return e;
  if (h->C.fsrc && (e = launch_source(h->C, h->stream)) != hipSuccess) return e;
  if (ev[TF_NPHASE] && (e = hipEventRecord(ev[TF_NPHASE], h->stream)) != hipSuccess) return e;
  return hipSuccess;
}

int capture(tf_handle* h, const PState& in, const PState& out, hipGraphExec_t* exec) {
  hipGraph_t g = nullptr;
  HIPCHK(hipStreamBeginCapture(h->stream, hipStreamCaptureModeThreadLocal));
  hipError_t e = enqueue_step(h, in, out, nullptr);
  hipError_t e2 = hipStreamEndCapture(h->stream, &g);
  if (e != hipSuccess) return fail(TF_EHIP, std::string("graph capture: ") + hipGetErrorString(e));
  if (e2 != hipSuccess) return fail(TF_EHIP, std::string("graph capture end: ") + hipGetErrorString(e2));
  HIPCHK(hipGraphInstantiate(exec, g, nullptr, nullptr, 0));
  HIPCHK(hipGraphDestroy(g));
  return TF_OK;
}

PState& other(tf_handle* h) { return h->cur_is_A ? h->B : h->A; }

}  // namespace

extern "C" {

const char* tf_error_string(int code) {
  switch (code) {
    case TF_OK: return "ok";
    case TF_EINVAL: return "invalid argument";
    case TF_ESIZE: return "size limit or workspace too small";
    case TF_EHIP: return "HIP runtime error";
    case TF_ESTATE: return "invalid call for the handle state";
    case TF_EOVERFLOW: return "fixed-point overflow";
    default: return "unknown error";
  }
}

const char* tf_last_error(void) { return g_err_lit ? g_err_lit : g_err.c_str(); }

int tf_set_tuning(const tf_tuning* t) {
  if (!t) {
    g_tune = tf_tuning{0, 0, 0, 0, 0};
    return TF_OK;
  }
  if (t->sort_cap < -1 || t->sort_cap > 4096 || t->fz_cols < 0 || t->fz_cols > 64 || t->tri_modes < 0 ||
      t->tri_modes > 32 || t->inv_plane < 0 || t->inv_plane > 4 || t->push_order < 0 || t->push_order > 2)
    return fail(TF_EINVAL, "tuning value out of range");
  g_tune = *t;
  return TF_OK;
}

int tf_set_tuning_class(int32_t nx, int32_t ny, int32_t nz, const tf_tuning* t) {
  if (nx < 1 || ny < 1 || nz < 1) return fail(TF_EINVAL, "mesh sizes must be positive");
  const auto key = std::make_tuple(nx, ny, nz);
  if (!t) {
    g_class_tune.erase(key);
    return TF_OK;
  }
  if (t->sort_cap < 0 || t->sort_cap > 4096 || t->fz_cols < 0 || t->fz_cols > 64 || t->tri_modes < 0 ||
      t->tri_modes > 32 || t->inv_plane < 0 || t->inv_plane > 4 || t->push_order < 0 || t->push_order > 2)
    return fail(TF_EINVAL, "tuning value out of range");
  g_class_tune[key] = *t;
  return TF_OK;
}

size_t tf_workspace_size(const tf_ensemble* ens, int32_t n_ens, int32_t traj_steps) {
  Sizes S;
  if (check_config(ens, n_ens, &S) != TF_OK || traj_steps < 0) return 0;
  return layout(S, n_ens, traj_steps, TF_INIT_KEEP_DEPOSIT | TF_INIT_SOURCE, nullptr, nullptr);
}

int tf_init(const tf_ensemble* ens, int32_t n_ens, const tf_particles* init, void* workspace,
            size_t workspace_bytes, int32_t traj_steps, void* stream, uint32_t flags, tf_handle** out) {
  if (!out) return fail(TF_EINVAL, "out is NULL");
  *out = nullptr;
  Sizes S;
  int rc = check_config(ens, n_ens, &S);
  if (rc != TF_OK) return rc;
  if (traj_steps < 0 || traj_steps > 100000) return fail(TF_EINVAL, "traj_steps out of range");
  if (!init) return fail(TF_EINVAL, "init is NULL");
  if (!workspace) return fail(TF_EINVAL, "workspace is NULL");
  if ((uintptr_t)workspace % 256) return fail(TF_EINVAL, "workspace must be 256-byte aligned");
  const size_t need = layout(S, n_ens, traj_steps, flags, nullptr, nullptr);
  if (workspace_bytes < need) return fail(TF_ESIZE, "workspace too small");
  for (int e = 0; e < n_ens; ++e) {
    const tf_particles& P = init[e];
    if (ens[e].n_particles > 0 && (!P.x || !P.y || !P.z || !P.vx || !P.vy || !P.vz || !P.q || !P.d))
      return fail(TF_EINVAL, "initial particle pointer is NULL");
  }

  // the static scratch of tf_poisson_noalloc on this device (set up once per device)
  void* scr = nullptr;
  rc = scratch_address(&scr);
  if (rc != TF_OK) return rc;

  tf_handle* h = new tf_handle();
  h->scratch = (double2*)scr;
  h->n_ens = n_ens;
  h->flags = flags;
  h->stream = (hipStream_t)stream;
  h->S = S;
  layout(S, n_ens, traj_steps, flags, workspace, h);

  // host tables (same floating-point operations as the textbook definitions)
  std::vector<double> yf(S.y_tot, 0.0), dy(S.y_tot, 0.0), idy(S.y_tot, 0.0), vol(S.y_tot, 0.0), am(S.y_tot, 0.0),
      ap(S.y_tot, 0.0), beta(S.y_tot, 0.0), kx2(S.kx_tot), kz2(S.kz_tot);
  std::vector<double2> tw(S.tw_tot);
  for (auto& kv : S.tw_off) {
    const int n = kv.first;
    for (int k = 0; k < n; ++k) {
      const double a = 2.0 * M_PI * k / n;
      tw[kv.second + k] = make_double2(std::cos(a), -std::sin(a));
    }
  }
  h->eh.resize(n_ens);
  h->p_off.assign(n_ens + 1, 0);
  h->c_off.assign(n_ens + 1, 0);
  int y_off = 0, kx_off = 0, kz_off = 0, st_off = 0;
  long long s_off = 0, row_off = 0, tf_off = 0, up_off = 0;
  // Thomas factors of the y-systems, per Fourier mode (fixed by the mesh):
  // tfac[tf_off + mode * ny + j] = (1 / pivot_j, c'_j)
  std::vector<double2> tfac(S.tf_tot);
  std::vector<long long> r_offs(n_ens + 1, 0);
  for (int e = 0; e < n_ens; ++e) {
    const tf_ensemble& T = ens[e];
    Ens& E = h->eh[e];
    E.nx = T.nx;
    E.ny = T.ny;
    E.nz = T.nz;
    E.nh = T.nx / 2 + 1;
    E.nhp = (E.nh + 7) & ~7;  // rows of whole 128-byte lines
    E.np = T.n_particles;
    E.p_off = h->p_off[e];
    E.c_off = h->c_off[e];
    E.s_off = s_off;
    // (a mesh seen before shares that ensemble's factor table)
    E.tf_off = S.tf_src[e] == e ? tf_off : h->eh[S.tf_src[e]].tf_off;
    E.row_off = row_off;
    E.y_off = y_off;
    E.ei = e;
    E.kx_off = kx_off;
    E.kz_off = kz_off;
    E.st_off = st_off;
    E.wz = S.e_wz[e];
    E.tm = S.e_tm[e];
    E.plane = S.e_plane[e];
    E.lx = T.lx;
    E.lz = T.lz;
    E.ly = T.y_faces[T.ny];
    E.dx = T.lx / T.nx;
    E.dz = T.lz / T.nz;
    E.dt = T.dt;
    E.rr = T.density_ratio;
    E.kc = T.k_c;
    E.dU = T.delta_u;
    E.e = T.e;
    E.cel = T.c_el;
    E.gp0 = (1.0 - 1.0 / T.density_ratio) * T.g[0];
    E.gp1 = (1.0 - 1.0 / T.density_ratio) * T.g[1];
    E.gp2 = (1.0 - 1.0 / T.density_ratio) * T.g[2];
    E.un_bin = T.un_bin;
    E.inv_dx = 1.0 / E.dx;
    E.inv_dz = 1.0 / E.dz;
    E.inv_2dx = 1.0 / (2.0 * E.dx);
    E.inv_2dz = 1.0 / (2.0 * E.dz);
    E.inv_nx = 1.0 / T.nx;
    E.inv_nz = 1.0 / T.nz;
    E.pp = T.pp;
    E.kpp = T.k_pp;
    E.charging = T.charging;
    E.seed = T.seed;
    E.sdq0 = T.ssm_dq0min;
    E.smu0 = T.ssm_mu0;
    E.ssig0 = T.ssm_sigma0;
    E.sgam0 = T.ssm_gamma0;
    E.scsat = T.ssm_csat;
    E.sd0 = T.ssm_d0;
    E.sun0 = T.ssm_un0;
    E.c18 = 18.0 / T.density_ratio;
    E.fe = T.k_c * std::pow(1.0 + T.e, 0.4);
    E.pe = std::pow(1.0 + T.e, 0.4);
    E.U = T.u_nodes;
    E.nxp = T.nx + 2;
    E.up_off = up_off;
    up_off += 3LL * (T.ny + 1) * T.nz * E.nxp;
    radix_plan(T.nx, &E.fx);
    E.fx.tw_off = S.tw_off.at(T.nx);
    radix_plan(T.nz, &E.fz);
    E.fz.tw_off = S.tw_off.at(T.nz);
    E.fzh = FftPlan{};
    if (E.plane == 2 || E.plane == 4)
      radix_plan(T.nz / E.plane, &E.fzh);  // twiddles: every plane-th one of length nz
    const int ny = T.ny;
    double* Y = &yf[y_off];
    for (int j = 0; j <= ny; ++j) Y[j] = T.y_faces[j];
    std::vector<double> yc(ny), hm(ny), hp(ny);
    for (int j = 0; j < ny; ++j) {
      dy[y_off + j] = Y[j + 1] - Y[j];
      idy[y_off + j] = 1.0 / dy[y_off + j];
      yc[j] = 0.5 * (Y[j] + Y[j + 1]);
      vol[y_off + j] = (E.dx * dy[y_off + j]) * E.dz;
    }
    for (int j = 0; j < ny; ++j) {
      hm[j] = (j > 0) ? yc[j] - yc[j - 1] : yc[0] - Y[0];
      hp[j] = (j < ny - 1) ? yc[j + 1] - yc[j] : Y[ny] - yc[ny - 1];
      am[y_off + j] = 1.0 / (dy[y_off + j] * hm[j]);
      ap[y_off + j] = 1.0 / (dy[y_off + j] * hp[j]);
    }
    for (int f = 1; f < ny; ++f) beta[y_off + f] = dy[y_off + f - 1] / (dy[y_off + f - 1] + dy[y_off + f]);
    for (int m = 0; m < E.nh; ++m)
      kx2[kx_off + m] = (2.0 - 2.0 * std::cos(2.0 * M_PI * m / T.nx)) / (E.dx * E.dx);
    for (int m = 0; m < T.nz; ++m)
      kz2[kz_off + m] = (2.0 - 2.0 * std::cos(2.0 * M_PI * m / T.nz)) / (E.dz * E.dz);
    h->p_off[e + 1] = h->p_off[e] + T.n_particles;
    h->c_off[e + 1] = h->c_off[e] + (long long)T.nx * T.ny * T.nz;
    s_off += (long long)ny * T.nz * E.nhp;
    if (S.tf_src[e] == e) {
      // modes mz and nz - mz share kz^2 and so their factors: rows mz <= nz / 2
      const int nm = E.nh * (T.nz / 2 + 1);
      const double* AM = &am[y_off];
      const double* AP = &ap[y_off];
      for (int mz = 0; mz <= T.nz / 2; ++mz)
        for (int m = 0; m < E.nh; ++m) {
          const int mode = mz * E.nh + m;
          const double K2 = kz2[kz_off + mz] + kx2[kx_off + m];
          double cprev = 0.0;
          for (int j = 0; j < ny; ++j) {
            // -am_j phi_{j-1} + (am_j + ap_j + K2) phi_j - ap_j phi_{j+1} = rho_j
            const double piv = ((AM[j] + AP[j]) + K2) + (j > 0 ? AM[j] * cprev : 0.0);
            const double cp = (-AP[j]) / piv;
            tfac[tf_off + (size_t)mode * ny + j] = make_double2(1.0 / piv, cp);
            cprev = cp;
          }
        }
      tf_off += (long long)ny * nm;
    }
    row_off += (long long)ny * T.nz;
    r_offs[e + 1] = row_off;
    y_off += ny + 1;
    kx_off += E.nh;
    kz_off += T.nz;
    st_off += stats_len(ny);
  }

  auto up = [&](const void* dst, const void* src, size_t bytes) {
    return hipMemcpyAsync((void*)dst, src, bytes, hipMemcpyHostToDevice, h->stream);
  };
  hipError_t he = hipSuccess;
#define UP(dst, vec) \
  if (he == hipSuccess && !vec.empty()) he = up(dst, vec.data(), vec.size() * sizeof(vec[0]));
  UP(h->C.ens, h->eh);
  UP(h->C.p_off, h->p_off);
  UP(h->C.c_off, h->c_off);
  UP(h->C.r_off, r_offs);
  UP(h->d_fx, S.fp_blk);
  UP(h->d_fz, S.fz_blk);
  UP(h->d_tri, S.tri_blk);
  UP(h->d_pl, S.pl_blk);
  UP(h->d_ph, S.ph_blk);
  UP(h->d_pq, S.pq_blk);
  UP(h->d_fps, S.fps_blk);
  UP(h->d_fzs, S.fzs_blk);
  UP(h->C.yf, yf);
  UP(h->C.dy, dy);
  UP(h->C.idy, idy);
  UP(h->C.vol, vol);
  UP(h->C.am, am);
  UP(h->C.ap, ap);
  UP(h->C.beta, beta);
  UP(h->C.kx2, kx2);
  UP(h->C.kz2, kz2);
  UP(h->C.tw, tw);
  std::vector<const double*> uptr(n_ens);
  for (int e = 0; e < n_ens; ++e) uptr[e] = ens[e].u_nodes;
  UP(h->C.uptr, uptr);
  UP(h->C.tfac, tfac);
#undef UP
  for (int e = 0; e < n_ens && he == hipSuccess; ++e)
    he = launch_pad_carrier(h->C.upad + h->eh[e].up_off, ens[e].u_nodes, ens[e].nx, ens[e].ny, ens[e].nz,
                            h->stream);
  if (he == hipSuccess) he = hipMemsetAsync(h->C.stats, 0, sizeof(long long) * S.st_tot, h->stream);
  if (he == hipSuccess) he = hipMemsetAsync(h->C.rowq, 0, sizeof(long long) * S.rows, h->stream);
  if (he == hipSuccess) he = hipMemsetAsync(h->C.rowacc, 0, sizeof(longlong2) * S.rows, h->stream);
  if (he == hipSuccess && S.c_tot) he = hipMemsetAsync(h->C.count, 0, sizeof(int) * S.c_tot, h->stream);
  if (he == hipSuccess) he = hipMemsetAsync(h->C.pair_cnt, 0, sizeof(int) * (S.rows / 2), h->stream);
  if (he == hipSuccess) he = hipMemsetAsync(h->C.mv_n, 0, sizeof(int) * (S.rows / 2), h->stream);
  if (he == hipSuccess) he = hipMemsetAsync(h->C.rs_old, 0, sizeof(int) * (S.rows + 1), h->stream);
  if (he == hipSuccess) he = hipMemsetAsync(h->C.rs_new, 0, sizeof(int) * (S.rows + 1), h->stream);
  if (he == hipSuccess) he = hipMemsetAsync(h->C.far_n, 0, sizeof(int) * 2, h->stream);
  if (he == hipSuccess && S.c_tot) he = hipMemsetAsync(h->C.phi, 0, sizeof(double) * S.c_tot, h->stream);
  if (he == hipSuccess && h->C.fsrc && S.c_tot)
    he = hipMemsetAsync(h->C.fsrc, 0, sizeof(double) * 3 * S.c_tot, h->stream);
  for (int e = 0; e < n_ens && he == hipSuccess; ++e) {
    if (ens[e].n_particles == 0) continue;
    const tf_particles& P = init[e];
    const double* in8[8] = {P.x, P.y, P.z, P.vx, P.vy, P.vz, P.q, P.d};
    he = launch_put_state(h->A, in8, h->p_off[e], ens[e].n_particles, h->stream);
  }
  if (he == hipSuccess) he = launch_bin(h->C, h->A, 0, S.n_tot, h->stream);
  if (he == hipSuccess) he = hipStreamSynchronize(h->stream);
  if (he != hipSuccess) {
    delete h;
    return fail(TF_EHIP, std::string("tf_init: ") + hipGetErrorString(he));
  }
  h->G.nx_max = S.nx_max;
  h->G.nz_max = S.nz_max;
  h->G.wz = S.wz;
  h->G.ny_max = S.ny_max;
  h->G.tri_rows = S.tri_rows;
  h->G.sort_cap = S.sort_cap;
  h->G.push_order = S.push_order;
  h->G.fp_blk = h->S.fp_blk.data();
  h->G.fz_blk = h->S.fz_blk.data();
  h->G.tri_blk = h->S.tri_blk.data();
  h->G.d_fp_blk = h->d_fx;
  h->G.d_fz_blk = h->d_fz;
  h->G.d_tri_blk = h->d_tri;
  h->G.pl_blk = h->S.pl_blk.data();
  h->G.d_pl_blk = h->d_pl;
  h->G.ph_blk = h->S.ph_blk.data();
  h->G.d_ph_blk = h->d_ph;
  h->G.pq_blk = h->S.pq_blk.data();
  h->G.d_pq_blk = h->d_pq;
  h->G.fps_blk = h->S.fps_blk.data();
  h->G.d_fps_blk = h->d_fps;
  h->G.fzs_blk = h->S.fzs_blk.data();
  h->G.d_fzs_blk = h->d_fzs;
  h->G.plane_any = S.plane_any ? 1 : 0;
  h->G.half_any = S.half_any ? 1 : 0;
  h->G.half_lds = S.half_lds;
  h->G.quarter_any = S.quarter_any ? 1 : 0;
  h->G.quarter_lds = S.quarter_lds;
  h->G.pp_any = S.pp_any ? 1 : 0;
  h->G.split_any = S.split_any ? 1 : 0;
  h->G.plane_max = S.plane_max;
  h->G.eh = h->eh.data();
  h->cur = h->A;
  h->cur_is_A = true;
  *out = h;
  return TF_OK;
}

int tf_step(tf_handle* h, int32_t n_steps, uint32_t flags) {
  if (!h) return fail(TF_EINVAL, "handle is NULL");
  if (n_steps < 0) return fail(TF_EINVAL, "n_steps < 0");
  if (h->C.n_tot == 0) {
    // no particles: the field of zero charge and the step counters
    for (int s = 0; s < n_steps; ++s) HIPCHK(enqueue_step(h, h->cur, other(h), nullptr, false));
    return TF_OK;
  }
  const bool rec = (flags & TF_STEP_RECORD) != 0;
  if (rec)
    for (int e = 0; e < h->n_ens; ++e)
      if (h->eh[e].pp || h->eh[e].charging)
        return fail(TF_ESTATE, "recording (adjoint) is not available with collisions or the SSM");
  if (rec) {
    if (h->traj_cap == 0) return fail(TF_ESTATE, "no trajectory capacity (traj_steps = 0 at tf_init)");
    if (h->traj_len + n_steps > h->traj_cap) return fail(TF_ESIZE, "recorded trajectory would exceed traj_steps");
    for (int s = 0; s < n_steps; ++s) {
      TrajBuf& tb = h->traj[h->traj_len];
      if (h->traj_len == 0) {
        // the current state becomes the first recorded state
        const size_t n = h->C.n_tot;
        const PState& c = h->cur;
        const PState& t = tb.st;
        double* src[8] = {c.x, c.y, c.z, c.vx, c.vy, c.vz, c.q, c.d};
        double* dst[8] = {t.x, t.y, t.z, t.vx, t.vy, t.vz, t.q, t.d};
        for (int f = 0; f < 8; ++f)
          HIPCHK(hipMemcpyAsync(dst[f], src[f], n * sizeof(double), hipMemcpyDeviceToDevice, h->stream));
        HIPCHK(hipMemcpyAsync(t.id, c.id, n * sizeof(int), hipMemcpyDeviceToDevice, h->stream));
        HIPCHK(hipMemcpyAsync(t.key, c.key, n * sizeof(int), hipMemcpyDeviceToDevice, h->stream));
        h->cur = t;
      }
      const PState in = h->cur;
      const PState out = h->traj[h->traj_len + 1].st;
      HIPCHK(enqueue_step(h, in, out, &tb, h->need_full));
      h->need_full = false;
      h->cur = out;
      h->traj_len++;
    }
    return TF_OK;
  }
  // leave the trajectory store: continue in the ping-pong buffers
  const bool in_traj = !(h->cur.x == h->A.x || h->cur.x == h->B.x);
  int s = 0;
  if (in_traj && n_steps > 0) {
    HIPCHK(enqueue_step(h, h->cur, h->A, nullptr, h->need_full));
    h->need_full = false;
    h->cur = h->A;
    h->cur_is_A = true;
    s = 1;
  }
  const bool graphs = (h->flags & TF_INIT_GRAPHS) != 0 && h->prof_cap == 0;
  if (graphs && s < n_steps) {
    if (!h->g_ab) {
      int rc = capture(h, h->A, h->B, &h->g_ab);
      if (rc != TF_OK) return rc;
      rc = capture(h, h->B, h->A, &h->g_ba);
      if (rc != TF_OK) return rc;
    }
  }
  for (; s < n_steps; ++s) {
    if (graphs && !h->need_full) {
      HIPCHK(hipGraphLaunch(h->cur_is_A ? h->g_ab : h->g_ba, h->stream));
    } else {
      // the graphs hold the incremental sort: a step after a state upload runs eagerly
      HIPCHK(enqueue_step(h, h->cur, other(h), nullptr, h->need_full));
      h->need_full = false;
    }
    h->cur = other(h);
    h->cur_is_A = !h->cur_is_A;
  }
  return TF_OK;
}

int tf_stats(tf_handle* h, int32_t e, tf_stats_out* out) {
  if (!h || !out) return fail(TF_EINVAL, "NULL argument");
  if (e < 0 || e >= h->n_ens) return fail(TF_EINVAL, "ensemble index out of range");
  const Ens& E = h->eh[e];
  std::vector<long long> st(stats_len(E.ny)), rq((size_t)E.ny * E.nz);
  std::vector<longlong2> ra((size_t)E.ny * E.nz);
  HIPCHK(hipStreamSynchronize(h->stream));
  HIPCHK(hipMemcpy(st.data(), h->C.stats + E.st_off, st.size() * sizeof(long long), hipMemcpyDeviceToHost));
  HIPCHK(hipMemcpy(rq.data(), h->C.rowq + E.row_off, rq.size() * sizeof(long long), hipMemcpyDeviceToHost));
  HIPCHK(hipMemcpy(ra.data(), h->C.rowacc + E.row_off, ra.size() * sizeof(longlong2), hipMemcpyDeviceToHost));
  out->steps = st[ST_STEPS];
  out->flags = (int32_t)st[ST_FLAGS];
  out->ny = E.ny;
  for (int w = 0; w < 2; ++w) {
    out->impacts[w] = st[ST_IMP + w];
    out->wall_q[w] = st[ST_WQ + w];
  }
  for (int b = 0; b < kNbin; ++b) out->un_hist[b] = st[ST_HIST + b];
  out->pp_pairs = st[ST_PP];
  __int128 tot = 0;
  for (int j = 0; j < E.ny; ++j) {
    long long qj = 0, cj = 0, q32 = 0;
    for (int k = 0; k < E.nz; ++k) {
      const size_t r = (size_t)j * E.nz + k;
      qj += rq[r];
      cj += ra[r].x;
      q32 += ra[r].y;
    }
    tot += qj;
    if (out->crel_y) out->crel_y[j] = cj;
    if (out->qcum_y) out->qcum_y[j] = q32;
    if (out->qnow_y) out->qnow_y[j] = qj;
  }
  out->q_sum = (double)(long double)tot * (1.0 / 281474976710656.0);
  return TF_OK;
}

int tf_get_state(tf_handle* h, int32_t e, const tf_particles* out) {
  if (!h || !out) return fail(TF_EINVAL, "NULL argument");
  if (e < 0 || e >= h->n_ens) return fail(TF_EINVAL, "ensemble index out of range");
  const int n = h->eh[e].np;
  if (n == 0) return TF_OK;
  double* o8[8] = {out->x, out->y, out->z, out->vx, out->vy, out->vz, out->q, out->d};
  for (auto* p : o8)
    if (!p) return fail(TF_EINVAL, "output pointer is NULL");
  HIPCHK(launch_get_state(h->cur, o8, h->p_off[e], n, h->stream));
  return TF_OK;
}

int tf_set_state(tf_handle* h, int32_t e, const tf_particles* in) {
  if (!h || !in) return fail(TF_EINVAL, "NULL argument");
  if (e < 0 || e >= h->n_ens) return fail(TF_EINVAL, "ensemble index out of range");
  const int n = h->eh[e].np;
  h->traj_len = 0;
  // the current buffer may be a recorded one: continue in A (all ensembles)
  if (!(h->cur.x == h->A.x || h->cur.x == h->B.x)) {
    const size_t nt = h->C.n_tot;
    const PState& c = h->cur;
    const PState& t = h->A;
    double* src[8] = {c.x, c.y, c.z, c.vx, c.vy, c.vz, c.q, c.d};
    double* dst[8] = {t.x, t.y, t.z, t.vx, t.vy, t.vz, t.q, t.d};
    for (int f = 0; f < 8 && nt; ++f)
      HIPCHK(hipMemcpyAsync(dst[f], src[f], nt * sizeof(double), hipMemcpyDeviceToDevice, h->stream));
    if (nt) {
      HIPCHK(hipMemcpyAsync(t.id, c.id, nt * sizeof(int), hipMemcpyDeviceToDevice, h->stream));
      HIPCHK(hipMemcpyAsync(t.key, c.key, nt * sizeof(int), hipMemcpyDeviceToDevice, h->stream));
    }
    h->cur = h->A;
    h->cur_is_A = true;
  }
  if (n == 0) return TF_OK;
  const double* in8[8] = {in->x, in->y, in->z, in->vx, in->vy, in->vz, in->q, in->d};
  for (auto* p : in8)
    if (!p) return fail(TF_EINVAL, "input pointer is NULL");
  const long long ncell = (long long)h->eh[e].nx * h->eh[e].ny * h->eh[e].nz;
  HIPCHK(hipMemsetAsync(h->C.count + h->c_off[e], 0, sizeof(int) * ncell, h->stream));
  HIPCHK(launch_put_state(h->cur, in8, h->p_off[e], n, h->stream));
  HIPCHK(launch_bin(h->C, h->cur, h->p_off[e], h->p_off[e] + n, h->stream));
  h->need_full = true;
  return TF_OK;
}

int tf_set_carrier(tf_handle* h, int32_t e, const double* u_nodes) {
  if (!h || !u_nodes) return fail(TF_EINVAL, "NULL argument");
  if (e < 0 || e >= h->n_ens) return fail(TF_EINVAL, "ensemble index out of range");
  if (h->traj_len > 0) return fail(TF_ESTATE, "a recorded trajectory is pending (tf_adjoint_step first)");
  h->eh[e].U = u_nodes;
  // the step reads the padded copy, refreshed in stream order; the reverse
  // step reads the field through the device pointer table, replaced by one
  // tiny kernel.  No synchronisation; captured graphs stay valid.
  const Ens& E = h->eh[e];
  HIPCHK(launch_pad_carrier(h->C.upad + E.up_off, u_nodes, E.nx, E.ny, E.nz, h->stream));
  HIPCHK(launch_set_ptr(h->C.uptr + e, u_nodes, h->stream));
  return TF_OK;
}

int tf_set_params(tf_handle* h, const double* theta) {
  if (!h || !theta) return fail(TF_EINVAL, "NULL argument");
  // the reverse step reads the charging parameters of the descriptor: they
  // must stay those of the recorded steps
  if (h->traj_len > 0) return fail(TF_ESTATE, "a recorded trajectory is pending (tf_adjoint_step first)");
  for (int e = 0; e < h->n_ens; ++e) {
    const double kc = theta[3 * e], du = theta[3 * e + 1], ee = theta[3 * e + 2];
    if (!std::isfinite(kc) || !std::isfinite(du) || !(ee > 0 && ee <= 1))
      return fail(TF_EINVAL, "theta must be finite with 0 < e <= 1");
  }
  for (int e = 0; e < h->n_ens; ++e) {
    h->eh[e].kc = theta[3 * e];
    h->eh[e].dU = theta[3 * e + 1];
    h->eh[e].e = theta[3 * e + 2];
    h->eh[e].fe = h->eh[e].kc * std::pow(1.0 + h->eh[e].e, 0.4);
    h->eh[e].pe = std::pow(1.0 + h->eh[e].e, 0.4);
  }
  HIPCHK(hipMemcpyAsync((void*)h->C.ens, h->eh.data(), sizeof(Ens) * h->n_ens, hipMemcpyHostToDevice, h->stream));
  HIPCHK(hipStreamSynchronize(h->stream));
  destroy_graphs(h);  // captured launches carry the old descriptor by value
  return TF_OK;
}

int tf_poisson(tf_handle* h, int32_t e, const int64_t* q_fixed, double* phi) {
  if (!h || !q_fixed || !phi) return fail(TF_EINVAL, "NULL argument");
  if (e < 0 || e >= h->n_ens) return fail(TF_EINVAL, "ensemble index out of range");
  HIPCHK(launch_poisson(h->C, h->G, e, e + 1, nullptr, nullptr, (const long long*)q_fixed, h->c_off[e], phi, h->c_off[e], 0,
                        h->stream));
  return TF_OK;
}

int tf_poisson_noalloc(tf_handle* h, int32_t e, const int64_t* q_fixed, double* phi) {
  // no allocation on any path: errors carry string literals
  if (!h || !q_fixed || !phi) return fail_lit(TF_EINVAL, "NULL argument");
  if (e < 0 || e >= h->n_ens) return fail_lit(TF_EINVAL, "ensemble index out of range");
  const Ens& E = h->eh[e];
  const size_t need = (size_t)E.ny * E.nz * E.nhp * sizeof(double2);
  if (need > (size_t)TF_NOALLOC_MAX_SPECTRUM_BYTES)
    return fail_lit(TF_ESIZE, "the ensemble's spectrum exceeds TF_NOALLOC_MAX_SPECTRUM_BYTES");
  if (!h->scratch) return fail_lit(TF_ESTATE, "no static scratch on this handle's device");
  const hipError_t he = launch_poisson(h->C, h->G, e, e + 1, nullptr, nullptr, (const long long*)q_fixed,
                                       h->c_off[e], phi, h->c_off[e], 0, h->stream, nullptr, nullptr, false,
                                       nullptr, h->scratch);
  if (he != hipSuccess) return fail_lit(TF_EHIP, "kernel launch failed");
  return TF_OK;
}

int tf_field(tf_handle* h, int32_t e, int32_t which, void* out) {
  if (!h || !out) return fail(TF_EINVAL, "NULL argument");
  if (e < 0 || e >= h->n_ens) return fail(TF_EINVAL, "ensemble index out of range");
  const long long ncell = (long long)h->eh[e].nx * h->eh[e].ny * h->eh[e].nz;
  if (which == TF_FIELD_PHI) {
    HIPCHK(hipMemcpyAsync(out, h->C.phi + h->c_off[e], ncell * sizeof(double), hipMemcpyDeviceToDevice, h->stream));
  } else if (which == TF_FIELD_DEPOSIT) {
    if (!h->C.qdep) return fail(TF_ESTATE, "deposit not kept (TF_INIT_KEEP_DEPOSIT)");
    HIPCHK(hipMemcpyAsync(out, h->C.qdep + h->c_off[e], ncell * sizeof(long long), hipMemcpyDeviceToDevice,
                          h->stream));
  } else if (which == TF_FIELD_SOURCE) {
    if (!h->C.fsrc) return fail(TF_ESTATE, "source not computed (TF_INIT_SOURCE)");
    for (int c = 0; c < 3; ++c)
      HIPCHK(hipMemcpyAsync((double*)out + c * ncell, h->C.fsrc + c * h->C.c_tot + h->c_off[e],
                            ncell * sizeof(double), hipMemcpyDeviceToDevice, h->stream));
  } else {
    return fail(TF_EINVAL, "unknown field");
  }
  return TF_OK;
}

int tf_adjoint_step(tf_handle* h, const tf_particles* lambda, const double* w_wall, double* dtheta) {
  if (!h || !lambda || !w_wall || !dtheta) return fail(TF_EINVAL, "NULL argument");
  if (h->traj_len == 0) return fail(TF_ESTATE, "no recorded steps (tf_step with TF_STEP_RECORD)");
  std::vector<const double*> lam(8 * (size_t)h->n_ens);
  for (int e = 0; e < h->n_ens; ++e) {
    const tf_particles& L = lambda[e];
    const double* l8[8] = {L.x, L.y, L.z, L.vx, L.vy, L.vz, L.q, L.d};
    for (int f = 0; f < 7; ++f)
      if (h->eh[e].np > 0 && !l8[f]) return fail(TF_EINVAL, "lambda pointer is NULL");
    for (int f = 0; f < 8; ++f) lam[8 * e + f] = l8[f];
  }
  std::vector<TrajStep> steps(h->traj_len + 1);
  for (int t = 0; t <= h->traj_len; ++t) {
    steps[t].st = h->traj[t].st;
    steps[t].perm = h->traj[t].perm;
    steps[t].skey = h->traj[t].skey;
    steps[t].start = h->traj[t].start;
    steps[t].phi = h->traj[t].phi;
    steps[t].wall = h->traj[t].wall;
  }
  hipError_t he = run_adjoint(h->C, h->G, h->adj, h->n_ens, h->eh.data(), h->p_off.data(), h->c_off.data(),
                              steps.data(), h->traj_len, lam.data(), w_wall, dtheta, h->stream);
  if (he != hipSuccess) return fail(TF_EHIP, std::string("adjoint: ") + hipGetErrorString(he));
  h->traj_len = 0;
  return TF_OK;
}

int tf_profile_begin(tf_handle* h, int32_t max_steps, uint32_t phase_mask) {
  return tf_profile_begin_every(h, max_steps, phase_mask, 1);
}

int tf_profile_begin_every(tf_handle* h, int32_t max_steps, uint32_t phase_mask, int32_t every) {
  if (!h) return fail(TF_EINVAL, "handle is NULL");
  if (max_steps < 1 || max_steps > 100000) return fail(TF_EINVAL, "max_steps out of range");
  if (every < 1 || every > 100000) return fail(TF_EINVAL, "every out of range");
  if (h->prof_cap) return fail(TF_ESTATE, "profiling already active");
  const uint32_t all = (1u << TF_NPHASE) - 1u;
  if (phase_mask & ~all) return fail(TF_EINVAL, "phase_mask has bits beyond the phases");
  h->prof_mask = phase_mask ? phase_mask : all;
  h->prof_ev.assign((size_t)max_steps * (TF_NPHASE + 1), nullptr);
  for (auto& e : h->prof_ev) HIPCHK(hipEventCreate(&e));
  h->prof_cap = max_steps;
  h->prof_n = 0;
  h->prof_every = every;
  h->prof_seen = 0;
  return TF_OK;
}

int tf_profile_end(tf_handle* h, double* phase_ms, int32_t* n_steps) {
  if (!h || !phase_ms || !n_steps) return fail(TF_EINVAL, "NULL argument");
  if (!h->prof_cap) return fail(TF_ESTATE, "profiling not active");
  HIPCHK(hipStreamSynchronize(h->stream));
  for (int p = 0; p < TF_NPHASE; ++p) phase_ms[p] = 0.0;
  for (int s = 0; s < h->prof_n; ++s) {
    hipEvent_t* ev = &h->prof_ev[(size_t)s * (TF_NPHASE + 1)];
    for (int p = 0; p < TF_NPHASE; ++p) {
      if (!((h->prof_mask >> p) & 1u)) continue;
      float ms = 0.f;
      HIPCHK(hipEventElapsedTime(&ms, ev[p], ev[p + 1]));
      phase_ms[p] += ms;
    }
  }
  *n_steps = h->prof_n;
  for (auto& e : h->prof_ev) hipEventDestroy(e);
  h->prof_ev.clear();
  h->prof_cap = h->prof_n = 0;
  return TF_OK;
}

void tf_destroy(tf_handle* h) {
  if (!h) return;
  destroy_graphs(h);
  for (auto& e : h->prof_ev) hipEventDestroy(e);
  delete h;
}

}  // extern "C"
