// Internal device-side definitions shared by the kernels and the C-ABI layer
// of libtribo.so.  Not a public header.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace tf {

constexpr int kMaxPass = 10;
constexpr int kNbin = 64;
constexpr int kBlock = 256;
constexpr int kMoverCap = 32;  // mover list entries per row pair
constexpr int kFixDep = 48;
constexpr int kFixWall = 40;
constexpr int kFixQcum = 32;
constexpr double kInv4Pi = 1.0 / (4.0 * 3.14159265358979323846);
constexpr double kPi = 3.14159265358979323846;

// Complex FFT of length n, Stockham autosort; the radix of pass p is
// (rcode >> 3p) & 7, passes in order.
struct FftPlan {
  int n, npass, tw_off;
  unsigned rcode;   // radices 2..5, three bits a pass
  int np_ip;
  unsigned rc_ip;   // in-place passes: radix - 1 (radices 2, 3, 4, 5, 8, 16), four bits a pass
};

// One ensemble as seen by the kernels.
struct Ens {
  int nx, ny, nz, nh, nhp, np;
  long long p_off;   // first particle slot of this ensemble
  long long c_off;   // first cell (global cell index = c_off + (j*nz + k)*nx + i)
  long long s_off;   // first spectrum entry ([ny][nz][nhp] complex)
  long long row_off; // first (j, k) row
  long long tf_off;  // first tridiagonal factor ([(nz / 2 + 1) nh][ny], mode-major, mz <= nz / 2)
  int y_off;         // first entry in the per-y tables (ny+1 reserved)
  int ei;            // index of the ensemble (its carrier pointer: Ctx::uptr[ei])
  int kx_off, kz_off;
  int st_off;        // first int64 of the statistics block
  int wz, tm;        // tile shapes: z-transform columns, tridiagonal modes per block
  int plane;         // inverse transforms: 1 one block per y plane, 2 or 4 blocks per plane
                     // (z-row residue mod 2 or 4), 0 z then x kernels
  double lx, ly, lz, dx, dz;
  double dt, rr, kc, dU, e, cel, gp0, gp1, gp2, un_bin;
  // derived on the host
  double inv_dx, inv_dz, inv_2dx, inv_2dz;  // 1/dx, 1/dz, 1/(2dx), 1/(2dz)
  double inv_nx, inv_nz;                    // 1/nx, 1/nz (index decomposition)
  double c18;                               // 18 / rr  (1/tau_p = c18 / d^2)
  double fe;                                // k_c (1 + e)^(2/5)
  double kpp;                               // particle-particle charge-exchange coefficient
  int pp;                                   // 4-way coupling on
  int charging;                             // 0 condenser, 1 stochastic scaling model
  unsigned seed;                            // SSM random numbers
  double sdq0, smu0, ssig0, sgam0, scsat, sd0, sun0;  // SSM reference impact
  double pe;                                // (1 + e)^(2/5)
  const double* U;   // carrier velocity nodes [3][ny+1][nz][nx] at tf_init (kernels read Ctx::uptr)
  long long up_off;  // first entry of the ensemble's padded carrier copy in Ctx::upad
  int nxp;           // padded node-row length nx + 2 (nodes 0..nx-1, then nodes 0 and 1 again)
  FftPlan fx, fz;
  FftPlan fzh;       // length nz/plane (plane split over 2 or 4 blocks)
};

// statistics block (int64) of one ensemble; the per-height sums live per (j,k)
// row in Ctx::rowacc (each row owned by one deposit block: no atomics) and are
// summed over k when read
// ST_DMAX: bit pattern of an upper bound of the ensemble's diameters (set by
// the binning of uploaded particles; positive doubles order like their bits)
enum {
  ST_STEPS = 0, ST_FLAGS = 1, ST_IMP = 2, ST_WQ = 4, ST_HIST = 6, ST_PP = 6 + kNbin, ST_DMAX = 7 + kNbin,
  ST_END = 8 + kNbin
};
inline int stats_len(int) { return ST_END; }

enum { FLAG_NONFINITE = 1, FLAG_OVERFLOW = 2, FLAG_OUTSIDE = 4 };

// LDS per block available on gfx950
constexpr int kLdsMax = 163840;
// fused inverse transforms of a y plane: threads per block, largest nz (nx/2 + 1)
constexpr int kPlaneThreads = 768;
constexpr int kPlanePts = 10240;
// inverse transforms of a y plane split over two blocks: threads per block,
// largest (nz/2) (nx/2 + 1) (z transforms) and (nz/4) nx (x transforms)
constexpr int kHalfThreads = 1024;
constexpr int kHalfPts = 4736;
constexpr int kHalfXPts = 4096;
// split over four blocks (z-row residue mod 4): the same z-transform limit,
// and (nz/8) nx points of the x transforms
constexpr int kQuarterXPts = 4736;
// threads per quarter-plane block: two blocks (and their 78 KB of LDS for the
// 192 x 192 plane) share a CU at up to 128 VGPRs
constexpr int kQuarterThreads = 512;
// z transforms: largest tile of wz columns times nz points
constexpr int kZPts = 2048;

// Particle buffer (structure of arrays).  key = global cell of the position.
struct PState {
  double *x, *y, *z, *vx, *vy, *vz, *q, *d;
  int *id, *key;
};

// Everything the kernels share (device pointers into the workspace).
struct Ctx {
  const Ens* ens;
  const long long* p_off;    // [n_ens+1] particle slot offsets
  const long long* c_off;    // [n_ens+1] cell offsets
  int n_ens;
  int pad0;
  long long n_tot, c_tot;
  int* count;                // [c_tot]   particles per cell (built by atomics, consumed by the placement)
  int* start;                // [c_tot+1] exclusive prefix of count
  int4* tmp;                 // [n_tot]   (id, old slot, cell, 0), unordered within a cell
  int* perm;                 // [n_tot]   new slot -> old slot, ordered by (cell, id)
  int* skey;                 // [n_tot]   cell of each new slot
  double* sq;                // [n_tot]   charge of each new slot (after a full sort, for its deposit)
  // incremental sort: the state is stored in the previous sort's order, so a
  // row pair's new members are the ones of its own slot range that stayed
  // plus the particles that moved in (mover list, far list)
  const long long* r_off;    // [n_ens+1] (j, k) row offsets
  long long n_rows;
  int* pair_cnt;             // [n_rows/2]   members of each row pair (rows 2p, 2p+1) after this step's sort
  int* ps;                   // [n_rows/2+1] slot range of each row pair after this step's sort
  int* rs_old;               // [n_rows+1]   slot range of each row in the stored order
  int* rs_new;               // [n_rows+1]   slot range of each row after this step's sort
  int* mv;                   // [n_rows/2][kMoverCap] slots of the particles that moved into each row pair
  int* mv_n;                 // [n_rows/2] entries (the push appends; the sort reads and resets)
  int* far;                  // [n_tot]    movers beyond a full mover list
  int* far_n;                // [2]        [0]: entries (the push appends; reset before the next push)
  const double** uptr;       // [n_ens]    carrier field of each ensemble (replaced by tf_set_carrier in stream order)
  // the carrier of every ensemble copied with periodic ghost nodes, [3][ny+1][nz][nx+2]:
  // the x-neighbour pair (i, i+1) of a node row is always one 16-byte load
  double* upad;
  int* scan_part;            // scan block partials
  double2* spec;             // spectra
  double* phi;               // [c_tot]   potential of the latest step
  long long* stats;          // statistics blocks
  long long* rowq;           // [sum ny*nz] sum rne(q 2^48) per (j,k) row, latest deposit
  longlong2* rowacc;         // [sum ny*nz] (particle count, sum rne(q 2^32)) per row, summed over steps
  long long* qdep;           // optional [c_tot] per-cell deposit of the latest step
  double* fslot;             // optional [3][n_tot] drag force on the particle of each slot (2-way source)
  double* fsrc;              // optional [3][c_tot] 2-way coupling source of the latest step
  double* cinc;              // optional [4][n_tot] collision increments (vx, vy, vz, q) of each slot
  unsigned char* chit;       // optional [n_tot] the slot collided this step (cinc valid only there)
  const double *yf, *dy, *idy, *vol, *am, *ap, *beta, *kx2, *kz2;
  const double2* tw;         // twiddles exp(-2 pi i k/n)
  const double2* tfac;       // Thomas factors per mesh: [modes mz <= nz / 2][ny] (1 / pivot, c')
};

__device__ __forceinline__ int find_off(const long long* off, int n, long long v) {
  int lo = 0, hi = n - 1;
  while (lo < hi) {
    int mid = (lo + hi + 1) >> 1;
    if (off[mid] <= v) lo = mid; else hi = mid - 1;
  }
  return lo;
}

__device__ __forceinline__ int find_off_i(const int* off, int n, int v) {
  int lo = 0, hi = n - 1;
  while (lo < hi) {
    int mid = (lo + hi + 1) >> 1;
    if (off[mid] <= v) lo = mid; else hi = mid - 1;
  }
  return lo;
}

// Blocks are dealt round-robin to the 8 XCDs; remap so that each XCD gets a
// contiguous range of logical blocks (neighbouring particles share L2 lines).
__device__ __forceinline__ long long xcd_block(long long b, long long nb) {
  const long long nx = 8;
  long long q = nb / nx, r = nb % nx;
  long long x = b % nx, w = b / nx;
  return x * q + (x < r ? x : r) + w;
}

// floor(t / d) for 0 <= t, d < 2^16 by multiply-high with m = ceil(2^32 / d):
// t*m/2^32 exceeds t/d by less than t*d/2^32 / d < 1/d, the gap to the next
// integer.  2^32/d has a fractional part >= 1/d >= 2^-16 unless d | 2^32, so
// ceil of its correctly rounded double is exact.
__device__ __forceinline__ unsigned magic32(int d) {
  return d > 1 ? (unsigned)ceil(4294967296.0 / (double)d) : 0u;
}
__device__ __forceinline__ int fdiv32(int t, unsigned m, int d) {
  return d > 1 ? (int)__umulhi((unsigned)t, m) : t;
}

// quotient and remainder of a >= 0 (< 2^31) by d, with inv_d = 1/d
__device__ __forceinline__ void divmod(int a, int d, double inv_d, int* q, int* r) {
  int qq = (int)((double)a * inv_d);
  int rr = a - qq * d;
  if (rr < 0) {
    qq -= 1;
    rr += d;
  } else if (rr >= d) {
    qq += 1;
    rr -= d;
  }
  *q = qq;
  *r = rr;
}

// rne(v 2^shift) as int64.  A value whose rounded magnitude reaches 2^62, or
// that is not finite, contributes 0 (sums of many entries cannot wrap) and sets
// *ovf, which the callers raise as the sticky overflow flag.
__device__ __forceinline__ long long fixed_round(double v, int shift, bool* ovf) {
  double s = rint(v * (double)(1ULL << shift));
  if (!(fabs(s) < 0x1p62)) { *ovf = true; return 0; }
  return (long long)s;
}

}  // namespace tf
