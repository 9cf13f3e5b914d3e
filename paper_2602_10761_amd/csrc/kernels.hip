// Forward-step kernels of libtribo.so (gfx950, FP64, wave64).
//
// Per step (launch order):
//   scan_small            row-pair prefix of the member counts the last push made
//   row_sort_dep          per row pair: members from its own slot range and its
//                         mover list, ranked by (cell, id) -> perm, slot-ordered
//                         copies of charge and position; exact int64 cell charge,
//                         rho = Q 2^-48 / V, forward FFT along x of the two rows
//   z<fwd>                forward FFT along z
//   tri                   one tridiagonal y-solve per Fourier mode
//   plane_part / plane_inv  inverse FFTs along z and x per y plane (two or four
//                         blocks, or one), or z<inv> then pair_ifftx: phi on the cells
//   [collide]             4-way coupling: per-slot collision increments
//   push                  per particle: forces, integration, wall impact and
//                         charging, wrap, next cell key, row-pair counts, movers
//   [source]              2-way coupling source per cell
// After an upload of particles the sort is a full counting sort instead
// (count, scan_*, place, rank) followed by pair_fftx.
//
// Particle state is stored in the slot order of the previous step's sort; the
// push gathers velocity, diameter and id through perm (nearly coalesced) and
// writes in the new order.  The carrier is read from a copy with periodic
// ghost nodes (pad_carrier, at init and on every carrier replacement).  Device-scope atomics are kept out of contended
// addresses: they are resolved beyond the per-XCD L2 and serialize there.
#include <type_traits>

#include "tribo_dev.h"
#include "particle.h"

namespace tf {

// ---------------------------------------------------------------------------
// block-level scans (256 threads = 4 waves, or 1024 threads = 16 waves)
// ---------------------------------------------------------------------------
template <int NW>
__device__ __forceinline__ int block_excl_scan(int v, int* total) {
  __shared__ int wsum[NW];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  int incl = v;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    int t = __shfl_up(incl, o, 64);
    if (lane >= o) incl += t;
  }
  if (lane == 63) wsum[w] = incl;
  __syncthreads();
  int off = 0, tot = 0;
#pragma unroll
  for (int i = 0; i < NW; ++i) {
    int x = wsum[i];
    off += (i < w) ? x : 0;
    tot += x;
  }
  __syncthreads();
  *total = tot;
  return off + incl - v;
}

constexpr int kScanPer = 16;                   // counts per thread
constexpr int kScanChunk = kScanPer * kBlock;  // counts per block
constexpr int kScanFold = 4096;                // up to this many blocks, scan_down sums its own prefix

// n counts from cnt[base, base + kScanPer) (zero past n)
__device__ __forceinline__ void scan_load(const int* __restrict__ cnt, long long base, long long n, int* v) {
  if (base + kScanPer <= n) {
    const int4* c4 = reinterpret_cast<const int4*>(cnt + base);
#pragma unroll
    for (int r = 0; r < kScanPer / 4; ++r) {
      const int4 t = c4[r];
      v[4 * r] = t.x;
      v[4 * r + 1] = t.y;
      v[4 * r + 2] = t.z;
      v[4 * r + 3] = t.w;
    }
  } else {
#pragma unroll
    for (int r = 0; r < kScanPer; ++r) v[r] = (base + r < n) ? cnt[base + r] : 0;
  }
}

// exclusive prefix (starting at ex) of v[] into out[base, base + kScanPer)
// (nothing past n); 16-byte stores when the chunk is whole
__device__ __forceinline__ void scan_store(int* __restrict__ out, long long base, long long n, const int* v, int ex) {
  if (base + kScanPer <= n) {
    int4* o4 = reinterpret_cast<int4*>(out + base);
#pragma unroll
    for (int r = 0; r < kScanPer / 4; ++r) {
      int4 t;
      t.x = ex;
      ex += v[4 * r];
      t.y = ex;
      ex += v[4 * r + 1];
      t.z = ex;
      ex += v[4 * r + 2];
      t.w = ex;
      ex += v[4 * r + 3];
      o4[r] = t;
    }
  } else {
#pragma unroll
    for (int r = 0; r < kScanPer; ++r) {
      if (base + r < n) out[base + r] = ex;
      ex += v[r];
    }
  }
}

// per-block totals of the counts
__global__ __launch_bounds__(kBlock) void k_scan_reduce(const int* __restrict__ cnt, long long n,
                                                        int* __restrict__ part) {
  const long long base = (long long)blockIdx.x * kScanChunk + (long long)kScanPer * threadIdx.x;
  int v[kScanPer];
  scan_load(cnt, base, n, v);
  int s = 0;
#pragma unroll
  for (int r = 0; r < kScanPer; ++r) s += v[r];
  int tot;
  block_excl_scan<kBlock / 64>(s, &tot);
  if (threadIdx.x == 0) part[blockIdx.x] = tot;
}

// single block of 1024 threads: exclusive scan of the block totals (only when
// there are more than kScanFold blocks)
__global__ __launch_bounds__(1024) void k_scan_part(int* __restrict__ part, int nb) {
  int carry = 0;
  for (int base = 0; base < nb; base += 1024) {
    int i = base + threadIdx.x;
    int v = (i < nb) ? part[i] : 0;
    int tot;
    int ex = block_excl_scan<16>(v, &tot);
    if (i < nb) part[i] = carry + ex;
    carry += tot;
  }
}

// the whole exclusive prefix of n <= kSmallScan counts in one block of 1024
// threads, kScanPer consecutive counts per thread
constexpr int kSmallScan = kScanPer * 1024;

__global__ __launch_bounds__(1024) void k_scan_small(const int* __restrict__ cnt, int n, int* __restrict__ out) {
  const long long base = (long long)kScanPer * threadIdx.x;
  int v[kScanPer];
  scan_load(cnt, base, n, v);
  int s = 0;
#pragma unroll
  for (int r = 0; r < kScanPer; ++r) s += v[r];
  int tot;
  int ex = block_excl_scan<16>(s, &tot);
  scan_store(out, base, n, v, ex);
  if (threadIdx.x == 0) out[n] = tot;
}

// writes start[0..n]; the block prefix is the sum of the preceding block totals
// (fold) or the scanned total.  The placement then counts each cell back down
// to zero.
__global__ __launch_bounds__(kBlock) void k_scan_down(const int* __restrict__ cnt, long long n,
                                                      const int* __restrict__ part, int fold,
                                                      int* __restrict__ start) {
  int pre;
  if (fold) {
    int acc = 0;
    for (int i = threadIdx.x; i < (int)blockIdx.x; i += kBlock) acc += part[i];
    block_excl_scan<kBlock / 64>(acc, &pre);
  } else {
    pre = part[blockIdx.x];
  }
  const long long base = (long long)blockIdx.x * kScanChunk + (long long)kScanPer * threadIdx.x;
  int v[kScanPer];
  scan_load(cnt, base, n, v);
  int s = 0;
#pragma unroll
  for (int r = 0; r < kScanPer; ++r) s += v[r];
  int tot;
  const int ex = block_excl_scan<kBlock / 64>(s, &tot) + pre;
  scan_store(start, base, n, v, ex);
  if (blockIdx.x == gridDim.x - 1 && threadIdx.x == kBlock - 1) start[n] = pre + tot;
}

// ---------------------------------------------------------------------------
// counting sort by (cell, id); kIlp particles per thread keep several
// independent memory chains in flight
// ---------------------------------------------------------------------------
constexpr int kIlp = 4;

// place each particle in its cell's run (unordered within the run) as
// (id, old slot, cell)
__global__ __launch_bounds__(kBlock) void k_place(Ctx C, const int* __restrict__ key, const int* __restrict__ id) {
  const long long p0 = (long long)blockIdx.x * (kBlock * kIlp) + threadIdx.x;
  int c[kIlp], pid[kIlp];
#pragma unroll
  for (int r = 0; r < kIlp; ++r) {
    const long long p = p0 + r * kBlock;
    const bool ok = p < C.n_tot;
    c[r] = ok ? key[p] : -1;
    pid[r] = ok ? id[p] : 0;
  }
  int slot[kIlp], lo[kIlp], hi[kIlp];
#pragma unroll
  for (int r = 0; r < kIlp; ++r) {
    if (c[r] >= 0) {
      lo[r] = C.start[c[r]];
      hi[r] = C.start[c[r] + 1];
      // counting down the cell's arrivals leaves count[] zero for the next step
      slot[r] = lo[r] + atomicSub(&C.count[c[r]], 1) - 1;
    }
  }
#pragma unroll
  for (int r = 0; r < kIlp; ++r) {
    // a slot outside the run means counts inconsistent with keys: never by construction
    if (c[r] >= 0 && slot[r] >= lo[r] && slot[r] < hi[r])
      C.tmp[slot[r]] = make_int4(pid[r], (int)(p0 + r * kBlock), c[r], 0);
  }
}

// order each run by id: the slot of a particle is its run start plus the
// number of run members with a smaller id.  Writes perm, skey and the
// slot-ordered copy of the charge (read by the deposit that follows).
__global__ __launch_bounds__(kBlock) void k_rank(Ctx C, PState in) {
  const long long s0 = (long long)blockIdx.x * (kBlock * kIlp) + threadIdx.x;
  int4 rec[kIlp];
#pragma unroll
  for (int r = 0; r < kIlp; ++r) {
    const long long s = s0 + r * kBlock;
    rec[r] = (s < C.n_tot) ? C.tmp[s] : make_int4(0, -1, 0, 0);
  }
  bool ok[kIlp];
  int a[kIlp], b[kIlp];
  double q[kIlp];
#pragma unroll
  for (int r = 0; r < kIlp; ++r) {
    const int p = rec[r].y, c = rec[r].z;
    ok[r] = p >= 0 && p < C.n_tot && c >= 0 && c < C.c_tot;
    if (ok[r]) {
      a[r] = C.start[c];
      b[r] = C.start[c + 1];
      q[r] = in.q[p];
    }
  }
#pragma unroll
  for (int r = 0; r < kIlp; ++r) {
    if (!ok[r]) continue;
    int rk = 0;
    if (b[r] - a[r] > 1)
      for (int t = a[r]; t < b[r]; ++t) rk += (C.tmp[t].x < rec[r].x) ? 1 : 0;
    const int o = a[r] + rk;
    C.perm[o] = rec[r].y;
    C.skey[o] = rec[r].z;
    C.sq[o] = q[r];
  }
}

// full sort (after init or a state upload): cell counts by atomics
__global__ __launch_bounds__(kBlock) void k_count(Ctx C, const int* __restrict__ key) {
  const long long p = (long long)blockIdx.x * kBlock + threadIdx.x;
  if (p < C.n_tot) atomicAdd(&C.count[key[p]], 1);
}

// row slot ranges from the cell starts of a full sort; the pair counts restart
// from zero for this step's push
__global__ __launch_bounds__(kBlock) void k_rows_from_start(Ctx C) {
  const long long r = (long long)blockIdx.x * kBlock + threadIdx.x;
  if (r > C.n_rows) return;
  if (r == C.n_rows) {
    C.rs_new[r] = (int)C.n_tot;
    return;
  }
  const int e = find_off(C.r_off, C.n_ens + 1, r);
  const Ens& E = C.ens[e];
  C.rs_new[r] = C.start[E.c_off + (r - C.r_off[e]) * E.nx];
  if ((r & 1) == 0) {
    C.pair_cnt[r >> 1] = 0;
    C.mv_n[r >> 1] = 0;
  }
}

// ---------------------------------------------------------------------------
// FFT in LDS: Stockham autosort, mixed radix 2/3/4/5, runtime plan
// ---------------------------------------------------------------------------
// orders the LDS accesses of one wave (phases that use only that wave's LDS
// region need no block barrier)
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
}

__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ double2 cadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ double2 csub(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }
// multiply by -i (forward) or +i (inverse)
template <bool INV>
__device__ __forceinline__ double2 mul_mi(double2 a) {
  return INV ? make_double2(-a.y, a.x) : make_double2(a.y, -a.x);
}

template <int R, bool INV>
__device__ __forceinline__ void butterfly(double2* v) {
  if constexpr (R == 2) {
    double2 a = v[0], b = v[1];
    v[0] = cadd(a, b);
    v[1] = csub(a, b);
  } else if constexpr (R == 4) {
    double2 a = cadd(v[0], v[2]), b = csub(v[0], v[2]);
    double2 c = cadd(v[1], v[3]), d = mul_mi<INV>(csub(v[1], v[3]));
    v[0] = cadd(a, c);
    v[2] = csub(a, c);
    v[1] = cadd(b, d);
    v[3] = csub(b, d);
  } else if constexpr (R == 3) {
    const double s3 = 0.86602540378443864676;  // sin(2 pi/3)
    double2 t = cadd(v[1], v[2]);
    double2 u = mul_mi<INV>(csub(v[1], v[2]));
    double2 m = make_double2(v[0].x - 0.5 * t.x, v[0].y - 0.5 * t.y);
    v[0] = cadd(v[0], t);
    v[1] = make_double2(m.x + s3 * u.x, m.y + s3 * u.y);
    v[2] = make_double2(m.x - s3 * u.x, m.y - s3 * u.y);
  } else if constexpr (R == 5) {
    const double c1 = 0.30901699437494742410, c2 = -0.80901699437494742410;
    const double s1 = 0.95105651629515357212, s2 = 0.58778525229247312917;
    double2 a1 = cadd(v[1], v[4]), b1 = csub(v[1], v[4]);
    double2 a2 = cadd(v[2], v[3]), b2 = csub(v[2], v[3]);
    double2 m1 = make_double2(v[0].x + c1 * a1.x + c2 * a2.x, v[0].y + c1 * a1.y + c2 * a2.y);
    double2 m2 = make_double2(v[0].x + c2 * a1.x + c1 * a2.x, v[0].y + c2 * a1.y + c1 * a2.y);
    double2 n1 = mul_mi<INV>(make_double2(s1 * b1.x + s2 * b2.x, s1 * b1.y + s2 * b2.y));
    double2 n2 = mul_mi<INV>(make_double2(s2 * b1.x - s1 * b2.x, s2 * b1.y - s1 * b2.y));
    v[0] = cadd(v[0], cadd(a1, a2));
    v[1] = cadd(m1, n1);
    v[4] = csub(m1, n1);
    v[2] = cadd(m2, n2);
    v[3] = csub(m2, n2);
  }
}

// radix 8 and 16 butterflies in place (index n = n1 + 4 n2 in): a layer of
// radix 2/4 butterflies over n2, the internal twiddles W_R^(n1 k2), a layer
// of radix-4 butterflies over n1; output k = (R / 4) k1 + k2 is left at
// position k1 + 4 k2 (out_pos)
template <bool INV>
__device__ __forceinline__ double2 mul_w(double2 a, double c, double s) {  // a * exp(-/+ i theta), (c, s) = (cos, sin)
  return INV ? make_double2(a.x * c - a.y * s, a.x * s + a.y * c) : make_double2(a.x * c + a.y * s, a.y * c - a.x * s);
}
template <bool INV>
__device__ __forceinline__ void bf4(double2& v0, double2& v1, double2& v2, double2& v3) {
  const double2 a = cadd(v0, v2), b = csub(v0, v2);
  const double2 c = cadd(v1, v3), d = mul_mi<INV>(csub(v1, v3));
  v0 = cadd(a, c);
  v2 = csub(a, c);
  v1 = cadd(b, d);
  v3 = csub(b, d);
}
template <int R>
__host__ __device__ constexpr int out_pos(int r) {
  return R == 16 ? (r >> 2) + 4 * (r & 3) : R == 8 ? (r >> 1) + 4 * (r & 1) : r;
}
template <bool INV>
__device__ __forceinline__ void butterfly8(double2* v) {
  const double h = 0.70710678118654752440;  // cos(pi/4)
#pragma unroll
  for (int n1 = 0; n1 < 4; ++n1) {
    const double2 a = v[n1], b = v[n1 + 4];
    v[n1] = cadd(a, b);
    v[n1 + 4] = csub(a, b);
  }
  v[5] = mul_w<INV>(v[5], h, h);
  v[6] = mul_mi<INV>(v[6]);
  v[7] = mul_w<INV>(v[7], -h, h);
  bf4<INV>(v[0], v[1], v[2], v[3]);
  bf4<INV>(v[4], v[5], v[6], v[7]);
}
template <bool INV>
__device__ __forceinline__ void butterfly16(double2* v) {
  // cos and sin of 2 pi m / 16
  constexpr double c1 = 0.92387953251128675613, c2 = 0.70710678118654752440, c3 = 0.38268343236508977173;
#pragma unroll
  for (int n1 = 0; n1 < 4; ++n1) bf4<INV>(v[n1], v[n1 + 4], v[n1 + 8], v[n1 + 12]);
  // position n1 + 4 k2 now holds the k2 output of column n1: twiddle W16^(n1 k2)
  v[5] = mul_w<INV>(v[5], c1, c3);     // m = 1
  v[9] = mul_w<INV>(v[9], c2, c2);     // m = 2
  v[13] = mul_w<INV>(v[13], c3, c1);   // m = 3
  v[6] = mul_w<INV>(v[6], c2, c2);     // m = 2
  v[10] = mul_mi<INV>(v[10]);          // m = 4
  v[14] = mul_w<INV>(v[14], -c2, c2);  // m = 6
  v[7] = mul_w<INV>(v[7], c3, c1);     // m = 3
  v[11] = mul_w<INV>(v[11], -c2, c2);  // m = 6
  v[15] = mul_w<INV>(v[15], -c1, -c3); // m = 9
#pragma unroll
  for (int k2 = 0; k2 < 4; ++k2) bf4<INV>(v[4 * k2], v[4 * k2 + 1], v[4 * k2 + 2], v[4 * k2 + 3]);
}
template <int R, bool INV>
__device__ __forceinline__ void butterfly_any(double2* v) {
  if constexpr (R == 8) butterfly8<INV>(v);
  else if constexpr (R == 16) butterfly16<INV>(v);
  else butterfly<R, INV>(v);
}

template <int R, bool INV>
__device__ __forceinline__ void fft_pass(const double2* __restrict__ a, double2* __restrict__ b, int rows,
                                         int n, int pitch, int Ns, const double2* __restrict__ tw, int tid,
                                         int nthr) {
  const int nb = n / R;
  const int stride = n / (Ns * R);
  const int total = rows * nb;
  const unsigned mnb = rows > 1 ? magic32(nb) : 0u;
  const bool ns2 = (Ns & (Ns - 1)) == 0;
  const unsigned mns = ns2 ? 0u : magic32(Ns);
  for (int t = tid; t < total; t += nthr) {
    const int row = rows > 1 ? fdiv32(t, mnb, nb) : 0;
    const int jj = t - row * nb;
    const double2* s = a + row * pitch;
    double2* d = b + row * pitch;
    const int k = ns2 ? (jj & (Ns - 1)) : jj - fdiv32(jj, mns, Ns) * Ns;
    double2 v[R];
#pragma unroll
    for (int r = 0; r < R; ++r) v[r] = s[jj + r * nb];
#pragma unroll
    for (int r = 1; r < R; ++r) {
      double2 w = tw[r * k * stride];
      if (INV) w.y = -w.y;
      v[r] = cmul(v[r], w);
    }
    butterfly<R, INV>(v);
    const int base = (jj - k) * R + k;
#pragma unroll
    for (int r = 0; r < R; ++r) d[base + r * Ns] = v[r];
  }
}

// Transforms `rows` lines of length P.n (row pitch `pitch`) held in a, with
// scratch b, by the 64 lanes tid of one wave on its own buffers (a
// wavefront-level fence between passes); returns the buffer holding the
// result.  The caller orders the buffers' and twiddles' writes before the call.
template <bool INV>
__device__ double2* lds_fft(double2* a, double2* b, int rows, int pitch, const FftPlan& P, const double2* tw,
                            int tid, int nthr) {
  const int n = P.n;
  int Ns = 1;
  for (int ps = 0; ps < P.npass; ++ps) {
    const int R = (int)((P.rcode >> (3 * ps)) & 7u);
    switch (R) {
      case 2: fft_pass<2, INV>(a, b, rows, n, pitch, Ns, tw, tid, nthr); break;
      case 3: fft_pass<3, INV>(a, b, rows, n, pitch, Ns, tw, tid, nthr); break;
      case 4: fft_pass<4, INV>(a, b, rows, n, pitch, Ns, tw, tid, nthr); break;
      default: fft_pass<5, INV>(a, b, rows, n, pitch, Ns, tw, tid, nthr); break;
    }
    wave_sync();
    double2* t = a;
    a = b;
    b = t;
    Ns *= R;
  }
  return a;
}

// ---------------------------------------------------------------------------
// strided copy global -> LDS with U loads per thread in flight before the
// first store (a plain strided loop waits for every load in turn); loads past
// the end re-read the last element instead of branching around the load
// ---------------------------------------------------------------------------
template <int U, class Ld, class St>
__device__ __forceinline__ void staged_copy(int total, int tid, int nthr, Ld ld, St st) {
  for (int t0 = tid; t0 < total; t0 += nthr * U) {
    decltype(ld(0)) r[U];
#pragma unroll
    for (int u = 0; u < U; ++u) r[u] = ld(min(t0 + u * nthr, total - 1));
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int t = t0 + u * nthr;
      if (t < total) st(t, r[u]);
    }
  }
}

// ---------------------------------------------------------------------------
// wave-wide integer sum
// ---------------------------------------------------------------------------
__device__ __forceinline__ long long wave_sum(long long v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// ---------------------------------------------------------------------------
// x transforms on row pairs: one wave per pair of rows (j, k), (j, k+1) with k
// even (nz is even), kPairsPerBlock pairs per block.  The two real rows are
// the real and imaginary parts of one complex transform; their half spectra
// follow from the conjugate-symmetric and antisymmetric parts of the result.
// ---------------------------------------------------------------------------
constexpr int kPairsPerBlock = kBlock / 64;

// block -> ensemble and local block (block tables per ensemble)
__device__ __forceinline__ void block_ens(const Ctx& C, const Ens& Eone, int one, const int* __restrict__ blk_off,
                                          int blk0, Ens& E, int& lb) {
  if (one) {
    E = Eone;
    lb = blockIdx.x;
  } else {
    const int gb = blk0 + blockIdx.x;
    const int e = find_off_i(blk_off, C.n_ens + 1, gb);
    E = C.ens[e];
    lb = gb - blk_off[e];
  }
}

// transform buf0 = rho_A + i rho_B forward and store the half spectra of rows
// jkA and jkA + 1
__device__ __forceinline__ void pair_forward_store(const Ctx& C, const Ens& E, int jkA, double2* buf0, double2* buf1,
                                                   const double2* tw, int lane, bool ok) {
  const int nx = E.nx;
  double2* res = lds_fft<false>(buf0, buf1, 1, nx, E.fx, tw, lane, 64);
  if (!ok) return;
  double2* outA = C.spec + E.s_off + (long long)jkA * E.nhp;
  double2* outB = outA + E.nhp;
  for (int m = lane; m < E.nh; m += 64) {
    const double2 zm = res[m];
    const double2 zn = res[m == 0 ? 0 : nx - m];
    outA[m] = make_double2(0.5 * (zm.x + zn.x), 0.5 * (zm.y - zn.y));
    outB[m] = make_double2(0.5 * (zm.y + zn.y), -0.5 * (zm.x - zn.x));
  }
}

// deposit (or given density) + forward FFT along x.  Sources of the cell
// charge, per call: the sorted particle runs [start[c], start[c+1]) (exact
// int64 fixed-point sums, order-free), a per-cell fixed-point array q_in, or
// a density r_in (per unit volume after division by V).
__global__ __launch_bounds__(kBlock) void k_pair_fftx(Ctx C, Ens Eone, int one, const int* __restrict__ blk_off,
                                                      int blk0, int nmax, const long long* __restrict__ q_in,
                                                      long long q_shift, const double* __restrict__ r_in,
                                                      int do_stats) {
  extern __shared__ double2 lds[];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  double2* tw = lds;
  double2* buf0 = lds + nmax + (size_t)w * 2 * nmax;
  double2* buf1 = buf0 + nmax;
  Ens E;
  int lb;
  block_ens(C, Eone, one, blk_off, blk0, E, lb);
  const int nx = E.nx, nz = E.nz, n2 = 2 * E.nx;
  const int lp = lb * kPairsPerBlock + w;
  const bool ok = lp < ((E.ny * nz) >> 1);
  const int jkA = ok ? 2 * lp : 0;
  const int j = jkA / nz;
  const long long c0 = E.c_off + (long long)jkA * nx;
  const double rsc = (1.0 / 281474976710656.0) / C.vol[E.y_off + j];  // 2^-48 / V
  for (int t = threadIdx.x; t < nx; t += kBlock) tw[t] = C.tw[E.fx.tw_off + t];
  bool ovf = false;
  long long rq48[2] = {0, 0}, rq32[2] = {0, 0};
  int cnt[2] = {0, 0};
  const bool parts = !q_in && !r_in;
  long long* bins = reinterpret_cast<long long*>(buf1);  // 2 nx int64 in the scratch buffer
  int s0 = 0, s1 = 0;
  if (ok && parts) {
    for (int i = lane; i < n2; i += 64) bins[i] = 0;
    s0 = min(max(C.start[c0], 0), (int)C.n_tot);
    const int sm = C.start[c0 + nx];
    s1 = min(max(C.start[c0 + n2], s0), (int)C.n_tot);
    cnt[0] = sm - s0;
    cnt[1] = s1 - sm;
  }
  __syncthreads();
  if (ok) {
    if (r_in) {
      const double iv = 1.0 / C.vol[E.y_off + j];
      for (int i = lane; i < nx; i += 64) buf0[i] = make_double2(r_in[c0 + i] * iv, r_in[c0 + nx + i] * iv);
    } else if (q_in) {
      for (int i = lane; i < nx; i += 64) {
        const long long QA = q_in[c0 + i - q_shift], QB = q_in[c0 + nx + i - q_shift];
        rq48[0] += QA;
        rq48[1] += QB;
        buf0[i] = make_double2((double)QA * rsc, (double)QB * rsc);
      }
    } else {
      // particle-parallel over the pair's sorted slots: coalesced charge/key
      // loads, per-cell integer sums in LDS
      for (int s = s0 + lane; s < s1; s += 64) {
        const double qv = C.sq[s];
        const unsigned i = (unsigned)(C.skey[s] - (int)c0);
        const long long Q = fixed_round(qv, kFixDep, &ovf);
        const long long Q32 = fixed_round(qv, kFixQcum, &ovf);
        if (i < (unsigned)nx) rq32[0] += Q32; else rq32[1] += Q32;
        if (i < (unsigned)n2) atomicAdd(reinterpret_cast<unsigned long long*>(&bins[i]), (unsigned long long)Q);
      }
    }
  }
  __syncthreads();
  if (ok && parts) {
    for (int i = lane; i < nx; i += 64) {
      const long long QA = bins[i], QB = bins[nx + i];
      if (C.qdep) {
        C.qdep[c0 + i] = QA;
        C.qdep[c0 + nx + i] = QB;
      }
      rq48[0] += QA;
      rq48[1] += QB;
      buf0[i] = make_double2((double)QA * rsc, (double)QB * rsc);
    }
  }
  if (ok && do_stats) {
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const long long a48 = wave_sum(rq48[h]), a32 = wave_sum(rq32[h]);
      if (lane == 0) {
        const long long r = E.row_off + jkA + h;
        longlong2 acc = C.rowacc[r];
        acc.x += cnt[h];
        acc.y += a32;
        C.rowacc[r] = acc;
        C.rowq[r] = a48;
      }
    }
  }
  if (ovf) atomicOr((unsigned long long*)&C.stats[E.st_off + ST_FLAGS], (unsigned long long)FLAG_OVERFLOW);
  __syncthreads();
  pair_forward_store(C, E, jkA, buf0, buf1, tw, lane, ok);
}

// ---------------------------------------------------------------------------
// incremental sort fused with the deposit and the x transform, one wave per
// row pair (j, k), (j, k+1) of the new order (2 nx consecutive cells).  The
// state is stored in the previous sort's order, so the pair's members are
// the slots of the pair's own range in that order that stayed, plus the
// pair's mover list and the far list, both written by the push.  The push
// counted the members of every row pair (pair_cnt); their scan is ps.  The
// members are listed in LDS (at most cap of them), bucketed by cell, ranked
// by id and placed; a pair with more members is listed one row at a time
// when each row fits, else it takes a second candidate pass through global
// memory (C.tmp).  All paths give the same slots.
// ---------------------------------------------------------------------------
constexpr int kCand = 8;  // candidates per lane per batch (key loads in flight together)

// LDS of one wave: member list {id, old slot} (8 B), member index by cell
// position (u16), member cell (u16) -- later the first FFT buffer -- then the
// int64 cell charges (later the second FFT buffer), one int per cell (its
// count, then its start, then after bucketing its end), 16 free bytes and
// the pair's two row accumulators
__host__ __device__ inline size_t sortdep_lists_bytes(int nx_max, int cap) {
  const size_t lists = (size_t)cap * 12, buf = (size_t)nx_max * 16;
  return ((lists > buf ? lists : buf) + 15) & ~(size_t)15;
}
__host__ __device__ inline size_t sortdep_wave_bytes(int nx_max, int cap) {
  return sortdep_lists_bytes(nx_max, cap) + (size_t)nx_max * 24 + 48;
}

__global__ __launch_bounds__(kBlock) void k_row_sort_dep(Ctx C, Ens Eone, int one, PState in,
                                                         const int* __restrict__ blk_off, int nmax, int cap) {
  extern __shared__ __align__(16) unsigned char lds_b[];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  double2* tw = reinterpret_cast<double2*>(lds_b);
  unsigned char* base = lds_b + (size_t)nmax * 16 + (size_t)w * sortdep_wave_bytes(nmax, cap);
  const size_t ub = sortdep_lists_bytes(nmax, cap);
  int2* A = reinterpret_cast<int2*>(base);
  unsigned short* Bm = reinterpret_cast<unsigned short*>(base + (size_t)cap * 8);
  unsigned short* Ai = Bm + cap;
  double2* buf0 = reinterpret_cast<double2*>(base);
  long long* Q = reinterpret_cast<long long*>(base + ub);  // 2 nx int64, read into buf0 before buf1 is used
  double2* buf1 = reinterpret_cast<double2*>(Q);
  int* pre = reinterpret_cast<int*>(Q + 2 * nmax);  // per cell: count -> start -> end
  // (16 bytes free, then the row accumulators, 16-byte aligned: nmax is even)
  longlong2* racc = reinterpret_cast<longlong2*>(pre + 2 * nmax + 4);

  Ens E;
  int lb;
  block_ens(C, Eone, one, blk_off, 0, E, lb);
  const int nx = E.nx, ny = E.ny, nz = E.nz, n2 = 2 * E.nx;
  const int lp = lb * kPairsPerBlock + w;
  const bool ok = lp < ((ny * nz) >> 1);
  const int jkA = ok ? 2 * lp : 0;
  const int j = jkA / nz, k = jkA - j * nz;
  const long long rA = E.row_off + jkA;
  const long long c0 = E.c_off + (long long)jkA * nx, c1 = c0 + n2;
  // candidates t: [0, T) own range from slot a0, [T, TB) mover list mvp,
  // [TB, TT) far list
  int a0 = 0, r0 = 0, rm = 0, r1 = 0, T = 0, TB = 0, TT = 0;
  const int* mvp = C.mv + (rA >> 1) * (long long)kMoverCap;
  double vol = 1.0;  // cell volume of the pair's row (loaded with the set-up loads)
  if (ok) {
    vol = C.vol[E.y_off + j];
    // (slot bounds clamped to [0, n_tot]: memory-safe even for inconsistent ranges)
    a0 = min(max(C.rs_old[rA], 0), (int)C.n_tot);
    T = min(max(C.rs_old[rA + 2], a0), (int)C.n_tot) - a0;
    TB = T + min(max(C.mv_n[rA >> 1], 0), kMoverCap);
    // the pair's slot range (clamped: writes stay inside the arrays whatever the counts)
    r0 = min(max(C.ps[rA >> 1], 0), (int)C.n_tot);
    r1 = min(max(C.ps[(rA >> 1) + 1], r0), (int)C.n_tot);
    TT = TB + min(C.far_n[0], (int)C.n_tot);
    for (int i = lane; i < n2; i += 64) {
      pre[i] = 0;
      Q[i] = 0;
    }
    if (lane == 0) {
      // consumed by the pair scan and here: restart the counts for this step's push
      C.pair_cnt[rA >> 1] = 0;
      C.mv_n[rA >> 1] = 0;
      // the pair's row accumulators (only this wavefront updates them), read
      // with the other set-up loads instead of on the way to the transform
      racc[0] = C.rowacc[rA];
      racc[1] = C.rowacc[rA + 1];
    }
  }
  const int M = r1 - r0;
  const bool fast = M <= cap;  // wave-uniform: the whole pair fits the list
  const unsigned long long below = (1ull << lane) - 1ull;
  // twiddles of the x transform (nx <= kBlock), shared by the block's waves:
  // the kernel's only block barrier, taken while the waves are still
  // together (one before the transform made every wave wait for the block's
  // most populous row pair)
  if ((int)threadIdx.x < nx) tw[threadIdx.x] = C.tw[E.fx.tw_off + threadIdx.x];
  __syncthreads();
  // candidate pass over the pair's own range, its mover list and the far
  // list: with count (a compile-time tag), the cell counts; members of the cells [lo, hi) listed
  // in LDS (positions by ballot: no same-address LDS atomics), at most cap;
  // returns how many were listed (wave-uniform; the loop is wave-uniform).
  // Loads are unconditional from a clamped slot (no branches around them)
  const int last = (int)C.n_tot - 1;
  auto cand_pass = [&](auto count_tag, int lo, int hi) -> int {
    constexpr bool count = decltype(count_tag)::value;
    int nl = 0;
    for (int tb = 0; tb < TT; tb += 64 * kCand) {
      const int t0 = tb + lane;
      int sl[kCand], c[kCand], idv[kCand];
#pragma unroll
      for (int u = 0; u < kCand; ++u) {
        const int t = t0 + 64 * u;
        sl[u] = t < T ? a0 + t : -1;
      }
      if (tb + 64 * kCand > T && TT > T) {  // the batch reaches the mover or far list
#pragma unroll
        for (int u = 0; u < kCand; ++u) {
          const int t = t0 + 64 * u;
          if (t >= T && t < TB) sl[u] = mvp[t - T];
          else if (t >= TB && t < TT) sl[u] = C.far[t - TB];
        }
      }
#pragma unroll
      for (int u = 0; u < kCand; ++u) {
        const int kv = in.key[min(max(sl[u], 0), last)];
        c[u] = sl[u] >= 0 ? kv : -1;
      }
#pragma unroll
      for (int u = 0; u < kCand; ++u) idv[u] = in.id[min(max(sl[u], 0), last)];
#pragma unroll
      for (int u = 0; u < kCand; ++u) {
        const bool hit = c[u] >= c0 && c[u] < c1;
        const int i = c[u] - (int)c0;
        if (count && hit) atomicAdd(&pre[i], 1);
        const bool li = hit && i >= lo && i < hi;
        const unsigned long long mask = __ballot(li);
        if (li) {
          const int m = nl + __popcll(mask & below);
          if (m < cap) {
            A[m] = make_int2(idv[u], sl[u]);
            Ai[m] = (unsigned short)i;
          }
        }
        nl += __popcll(mask);
      }
    }
    return nl;
  };
  // pass 1: the counts, and the members listed: all of them when the pair
  // fits the list, else those of its first row (the pair may fit in two
  // rounds, one row each)
  const int nl1 = cand_pass(std::true_type{}, 0, fast ? n2 : nx);
  wave_sync();
  if (ok) {
    // exclusive scan of the pair's cell counts, in place: lane owns cells
    // [lane*mm, lane*mm + mm)
    const int mm = (n2 + 63) >> 6;
    int v = 0;
    for (int u = 0; u < mm; ++u) {
      const int i = lane * mm + u;
      if (i < n2) v += pre[i];
    }
    int incl = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      const int t = __shfl_up(incl, o, 64);
      if (lane >= o) incl += t;
    }
    int ex = incl - v;
    for (int u = 0; u < mm; ++u) {
      const int i = lane * mm + u;
      if (i < n2) {
        const int ci = pre[i];
        pre[i] = ex;
        C.start[c0 + i] = r0 + min(ex, M);
        ex += ci;
      }
    }
    if (rA + 2 == C.n_rows && lane == 0) C.start[c1] = r1;
  }
  wave_sync();
  if (ok) {
    // row slot ranges of the new order (the stored order of the next step)
    rm = r0 + min(pre[nx], M);
    if (lane == 0) {
      C.rs_new[rA] = r0;
      C.rs_new[rA + 1] = rm;
      if (rA + 2 == C.n_rows) C.rs_new[rA + 2] = r1;
    }
  }
  const int MA = rm - r0;  // members of the first row
  const bool rows2 = !fast && MA <= cap && M - MA <= cap;  // wave-uniform
  bool ovf = false;
  long long rq32[2] = {0, 0};
  // a member (old slot p, charge q, cell i, rank rk by id among its cell's
  // members, which start at position a): its slot and its deposit
  auto place = [&](double q, int p, int i, int a, int rk) {
    const int o = r0 + a + rk;
    C.perm[o] = p;
    C.skey[o] = (int)c0 + i;
    const long long Qd = fixed_round(q, kFixDep, &ovf);
    const long long Q32 = fixed_round(q, kFixQcum, &ovf);
    if (i < nx) rq32[0] += Q32; else rq32[1] += Q32;
    atomicAdd(reinterpret_cast<unsigned long long*>(&Q[i]), (unsigned long long)Qd);
  };
  if (fast || rows2) {
    // members listed in LDS, one round per listed range of positions
    // [base, lim) (the pair, or its first row and then its second): bucketed
    // by cell (pre[] becomes the cell ends, so cell i spans [pre[i - 1],
    // pre[i]), from 0 for i = 0), ranked by id, placed
    int nm = min(nl1, cap);
    for (int rd = 0; rd < (rows2 ? 2 : 1); ++rd) {  // wave-uniform
      if (rd == 1) {
        // the second row: its members listed by a candidate pass of their own
        nm = min(cand_pass(std::false_type{}, nx, n2), cap);
        wave_sync();
      }
      const int base = rd ? MA : 0, lim = fast ? M : (rd ? M : MA);
      for (int m = lane; m < nm; m += 64) {
        const int pos = atomicAdd(&pre[Ai[m]], 1);
        if (pos >= base && pos < lim) Bm[pos - base] = (unsigned short)m;
      }
      wave_sync();
      for (int t = base + lane; t < lim; t += 64) {
        const int m = Bm[t - base];
        if (m >= nm) continue;  // members inconsistent with the row counts: never by construction
        const int2 e = A[m];
        const int id = e.x, p = e.y, i = Ai[m];
        if (p < 0 || p >= C.n_tot || i < 0 || i >= n2) continue;
        const int b = min(pre[i], lim), a = i ? min(max(pre[i - 1], base), b) : base;
        const double q = in.q[p];  // in flight during the ranking
        int rk = 0;
        for (int u = a; u < b; ++u) {
          const int mu = Bm[u - base];
          rk += (mu < nm && A[mu].x < id) ? 1 : 0;
        }
        place(q, p, i, a, rk);
      }
      wave_sync();
    }
  } else {
    // more members than the LDS lists hold: a second candidate pass through C.tmp
    for (int t0 = lane; t0 < TT; t0 += 64 * kCand) {
      int sl[kCand], c[kCand], idv[kCand];
#pragma unroll
      for (int u = 0; u < kCand; ++u) {
        const int t = t0 + 64 * u;
        sl[u] = t < T ? a0 + t : t < TB ? mvp[t - T] : t < TT ? C.far[t - TB] : -1;
      }
#pragma unroll
      for (int u = 0; u < kCand; ++u) c[u] = sl[u] >= 0 ? in.key[sl[u]] : -1;
#pragma unroll
      for (int u = 0; u < kCand; ++u) idv[u] = (c[u] >= c0 && c[u] < c1) ? in.id[sl[u]] : 0;
#pragma unroll
      for (int u = 0; u < kCand; ++u) {
        if (c[u] >= c0 && c[u] < c1) {
          const int slot = r0 + atomicAdd(&pre[c[u] - (int)c0], 1);
          if (slot < r1) C.tmp[slot] = make_int4(idv[u], sl[u], c[u], 0);
        }
      }
    }
    wave_sync();
    for (int t = lane; t < M; t += 64) {
      const int4 rec = C.tmp[r0 + t];
      const int id = rec.x, p = rec.y, i = rec.z - (int)c0;
      if (p < 0 || p >= C.n_tot || i < 0 || i >= n2) continue;
      const int b = min(pre[i], M), a = i ? min(max(pre[i - 1], 0), b) : 0;
      const double q = in.q[p];
      int rk = 0;
      for (int u = a; u < b; u += 4) {
        int idu[4];
#pragma unroll
        for (int vv = 0; vv < 4; ++vv) idu[vv] = (u + vv < b) ? C.tmp[r0 + u + vv].x : 0x7fffffff;
#pragma unroll
        for (int vv = 0; vv < 4; ++vv) rk += (idu[vv] < id) ? 1 : 0;
      }
      place(q, p, i, a, rk);
    }
  }
  wave_sync();  // member lists read: the FFT buffers may overwrite them
  const double rsc = (1.0 / 281474976710656.0) / vol;  // 2^-48 / V
  long long rq48[2] = {0, 0};
  if (ok) {
    for (int i = lane; i < nx; i += 64) {
      const long long QA = Q[i], QB = Q[nx + i];
      if (C.qdep) {
        C.qdep[c0 + i] = QA;
        C.qdep[c0 + nx + i] = QB;
      }
      rq48[0] += QA;
      rq48[1] += QB;
      buf0[i] = make_double2((double)QA * rsc, (double)QB * rsc);
    }
    const int cntr[2] = {rm - r0, r1 - rm};
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const long long a48 = wave_sum(rq48[h]), a32 = wave_sum(rq32[h]);
      if (lane == 0) {
        longlong2 acc = racc[h];
        acc.x += cntr[h];
        acc.y += a32;
        C.rowacc[rA + h] = acc;
        C.rowq[rA + h] = a48;
      }
    }
  }
  if (ovf) atomicOr((unsigned long long*)&C.stats[E.st_off + ST_FLAGS], (unsigned long long)FLAG_OVERFLOW);
  wave_sync();
  pair_forward_store(C, E, jkA, buf0, buf1, tw, lane, ok);
}

// ---------------------------------------------------------------------------
// tridiagonal solve in y for a tile of Fourier modes (mz, mx):
//   -am_j phi_{j-1} + (am_j + ap_j + k^2) phi_j - ap_j phi_{j+1} = rho_j
// (FV Laplacian times -1, phi = 0 on both walls).  With the Thomas factors
// (1 / pivot_j, c'_j) of every mode precomputed from the mesh, both sweeps are
// first-order linear recurrences,
//   d_j = A_j d_{j-1} + B_j  (A_j = am_j / pivot_j, B_j = rho_j / pivot_j),
//   x_j = -c'_j x_{j+1} + d_j,
// solved as parallel prefix compositions of affine maps: G lanes per mode,
// R consecutive rows per lane (G R >= ny), a wavefront scan of the per-lane
// maps (Hillis-Steele with shuffles) between two local passes.  The tile
// (kBlock / G modes) is staged in LDS, [mode][lane][row] with an odd row
// stride, from coalesced loads.
// ---------------------------------------------------------------------------
template <int R>
__global__ __launch_bounds__(kBlock) void k_tri(Ctx C, Ens Eone, int one, const int* __restrict__ blk_off,
                                                int blk0) {
  extern __shared__ double2 col[];  // [tm][G][RS] + one pad entry per mode
  Ens E;
  int lb;
  block_ens(C, Eone, one, blk_off, blk0, E, lb);
  const int nh = E.nh, nz = E.nz, ny = E.ny, nhp = E.nhp;
  const int tm = E.tm, G = kBlock / tm;  // slots per block, lanes per slot
  constexpr int RS = R | 1;               // odd row stride: lanes of a quarter-wave hit distinct banks
  const int MS = G * RS + 1;              // mode stride: staging threads hit distinct banks
  // the tile is tm consecutive slots of the padded [nz][nhp] plane (aligned
  // segments of every y plane); padding slots pass through unchanged
  const int pitch = nz * nhp;
  const int slot0 = lb * tm;
  const int w = min(tm, pitch - slot0);
  double2* sp = C.spec + E.s_off + slot0;
  const unsigned mw = magic32(w);
  // rows per lane of this ensemble (Re <= R): the scan order, and so the
  // rounding, depends on the ensemble's own mesh only; slots r >= Re are
  // identity maps (exact: x * 1 + 0)
  const int Re = (ny + G - 1) / G;
  const unsigned mre = magic32(Re);
  auto lidx = [&](int c, int j) {
    const int g = fdiv32(j, mre, Re);
    return c * MS + g * RS + (j - g * Re);
  };
  // this lane's slot and rows; its factors are loaded with the tile
  const int c = threadIdx.x / G, g = threadIdx.x - c * G;
  const int mz = (slot0 + c) / nhp, m = slot0 + c - mz * nhp;
  const bool act = c < w && m < nh;
  const int j0 = g * Re;
  double A[R], Cc[R], ip[R];
  {
    // (1/pivot, c'); modes mz and nz - mz share their factors (the same kz^2)
    const int mzs = mz <= (nz >> 1) ? mz : nz - mz;
    const double2* __restrict__ tf = C.tfac + E.tf_off + (long long)(act ? mzs * nh + m : 0) * ny;
    const double* __restrict__ am = C.am + E.y_off;
#pragma unroll
    for (int r = 0; r < R; ++r) {
      // rows past the upper wall solve to zero
      const int j = j0 + r;
      const bool slot = r < Re, in = act && slot && j < ny;
      const double2 f = tf[in ? j : 0];
      const double a = am[in ? j : 0];
      ip[r] = in ? f.x : 0.0;
      A[r] = !slot ? 1.0 : (in && j > 0) ? a * f.x : 0.0;
      Cc[r] = !slot ? 1.0 : (in && j < ny - 1) ? -f.y : 0.0;
    }
  }
  staged_copy<8>(
      ny * w, threadIdx.x, kBlock,
      [&](int t) {
        const int j = fdiv32(t, mw, w), c = t - j * w;
        return sp[(long long)j * pitch + c];
      },
      [&](int t, double2 v) {
        const int j = fdiv32(t, mw, w), c = t - j * w;
        col[lidx(c, j)] = v;
      });
  __syncthreads();
  if (act) {
    double2* v = col + c * MS + g * RS;
    double2 B[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const double2 rv = (r < Re && j0 + r < ny) ? v[r] : make_double2(0.0, 0.0);
      B[r] = make_double2(rv.x * ip[r], rv.y * ip[r]);
    }
    // forward: d_j = A_j d_{j-1} + B_j; per-lane map, then an inclusive scan
    double al = 1.0;
    double2 bl = make_double2(0.0, 0.0);
#pragma unroll
    for (int r = 0; r < R; ++r) {
      al = A[r] * al;
      bl = make_double2(A[r] * bl.x + B[r].x, A[r] * bl.y + B[r].y);
    }
    for (int o = 1; o < G; o <<= 1) {
      const double ao = __shfl_up(al, o, G);
      const double bx = __shfl_up(bl.x, o, G), by = __shfl_up(bl.y, o, G);
      if (g >= o) {
        bl = make_double2(al * bx + bl.x, al * by + bl.y);
        al = al * ao;
      }
    }
    double dx = __shfl_up(bl.x, 1, G), dy = __shfl_up(bl.y, 1, G);
    if (g == 0) dx = dy = 0.0;
#pragma unroll
    for (int r = 0; r < R; ++r) {
      dx = A[r] * dx + B[r].x;
      dy = A[r] * dy + B[r].y;
      B[r] = r < Re ? make_double2(dx, dy) : make_double2(0.0, 0.0);
    }
    // backward: x_j = -c'_j x_{j+1} + d_j, suffix scan from the upper wall
    al = 1.0;
    bl = make_double2(0.0, 0.0);
#pragma unroll
    for (int r = R - 1; r >= 0; --r) {
      al = Cc[r] * al;
      bl = make_double2(Cc[r] * bl.x + B[r].x, Cc[r] * bl.y + B[r].y);
    }
    for (int o = 1; o < G; o <<= 1) {
      const double ao = __shfl_down(al, o, G);
      const double bx = __shfl_down(bl.x, o, G), by = __shfl_down(bl.y, o, G);
      if (g + o < G) {
        bl = make_double2(al * bx + bl.x, al * by + bl.y);
        al = al * ao;
      }
    }
    double xx = __shfl_down(bl.x, 1, G), xy = __shfl_down(bl.y, 1, G);
    if (g == G - 1) xx = xy = 0.0;
#pragma unroll
    for (int r = R - 1; r >= 0; --r) {
      xx = Cc[r] * xx + B[r].x;
      xy = Cc[r] * xy + B[r].y;
      if (r < Re && j0 + r < ny) v[r] = make_double2(xx, xy);
    }
  }
  __syncthreads();
  for (int t0 = threadIdx.x; t0 < ny * w; t0 += 4 * kBlock) {
    double2 r[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int t = min(t0 + u * kBlock, ny * w - 1);
      const int j = fdiv32(t, mw, w), cc = t - j * w;
      r[u] = col[lidx(cc, j)];
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int t = t0 + u * kBlock;
      if (t < ny * w) {
        const int j = fdiv32(t, mw, w), cc = t - j * w;
        sp[(long long)j * pitch + cc] = r[u];
      }
    }
  }
}

// ---------------------------------------------------------------------------
// inverse FFT along x on row pairs: Z = X_A + i X_B over the full line (each
// half spectrum extended by conjugate symmetry, the imaginary parts of its
// mean and Nyquist terms dropped), one inverse complex transform, phi_A and
// phi_B are the real and imaginary parts
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void k_pair_ifftx(Ctx C, Ens Eone, int one, const int* __restrict__ blk_off,
                                                       int blk0, int nmax, double* __restrict__ phi_out,
                                                       long long phi_shift, int* __restrict__ far_reset,
                                                       int bump) {
  // the sort of this step has read the far list: empty it for this step's push;
  // bump: count the step (the push then reads the step number)
  if (far_reset && blockIdx.x == 0) {
    if (threadIdx.x == 0) *far_reset = 0;
    if (bump)
      for (int e = threadIdx.x; e < C.n_ens; e += blockDim.x) C.stats[C.ens[e].st_off + ST_STEPS] += 1;
  }
  extern __shared__ double2 lds[];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  double2* tw = lds;
  double2* buf0 = lds + nmax + (size_t)w * 2 * nmax;
  double2* buf1 = buf0 + nmax;
  Ens E;
  int lb;
  block_ens(C, Eone, one, blk_off, blk0, E, lb);
  if (E.plane) return;  // fused inverse transforms of the plane
  const int nx = E.nx, nz = E.nz, half = E.nx >> 1;
  const int lp = lb * kPairsPerBlock + w;
  const bool ok = lp < ((E.ny * nz) >> 1);
  const int jkA = ok ? 2 * lp : 0;
  // twiddles (nx <= kBlock): the load is in flight with the spectrum loads
  const double2 twv = C.tw[E.fx.tw_off + min((int)threadIdx.x, nx - 1)];
  if (ok) {
    const double2* sa = C.spec + E.s_off + (long long)jkA * E.nhp;
    const double2* sb = sa + E.nhp;
    struct AB {
      double2 a, b;
    };
    staged_copy<4>(
        nx, lane, 64,
        [&](int t) {
          const int m = t <= half ? t : nx - t;
          return AB{sa[m], sb[m]};
        },
        [&](int t, AB v) {
          double2 z;
          if (t == 0 || t == half) z = make_double2(v.a.x, v.b.x);
          else if (t < half) z = make_double2(v.a.x - v.b.y, v.a.y + v.b.x);
          else z = make_double2(v.a.x + v.b.y, v.b.x - v.a.y);
          buf0[t] = z;
        });
  }
  if ((int)threadIdx.x < nx) tw[threadIdx.x] = twv;
  __syncthreads();
  double2* res = lds_fft<true>(buf0, buf1, 1, nx, E.fx, tw, lane, 64);
  if (!ok) return;
  const double sc = 1.0 / (double)nx;
  double* outA = phi_out + (E.c_off - phi_shift) + (long long)jkA * nx;
  double* outB = outA + nx;
  for (int t = lane; t < nx; t += 64) {
    const double2 v = res[t];
    outA[t] = v.x * sc;
    outB[t] = v.y * sc;
  }
}

// ---------------------------------------------------------------------------
// inverse z and x transforms of one y plane in a single block, when the
// plane's half spectrum fits the LDS (nz (nx/2 + 1) <= kPlanePts): one read
// of the spectrum and one write of phi, no intermediate pass through memory.
// The transforms run in place: every Stockham pass loads its butterflies'
// inputs into registers, synchronises the block, then writes the outputs.
// ---------------------------------------------------------------------------
// element i of line l at a[l * ls + i * es]
struct LineLd {
  const double2* a;
  int ls, es;
  __device__ double2 operator()(int l, int i) const { return a[l * ls + i * es]; }
};

template <int R, bool INV, int NT, int MAXPTS, class Ld>
__device__ __forceinline__ void ip_pass(double2* a, int lines, unsigned mlines, int ls, int es, int n, int Ns,
                                        const double2* __restrict__ tw, int tid, Ld ld) {
  constexpr int UM = (MAXPTS / R + NT - 1) / NT;
  const int nb = n / R, stride = n / (Ns * R), total = lines * nb;
  const int sin_ = nb * es, sout = Ns * es;  // element steps of a butterfly's inputs and outputs
  double2 v[UM][R];
#pragma unroll
  for (int u = 0; u < UM; ++u) {
    const int t = tid + u * NT;
    if (t < total) {
      const int jj = fdiv32(t, mlines, lines), line = t - jj * lines;
      if constexpr (std::is_same<Ld, LineLd>::value) {
        const double2* s = a + line * ls + jj * es;
#pragma unroll
        for (int r = 0; r < R; ++r) v[u][r] = s[r * sin_];
      } else {
#pragma unroll
        for (int r = 0; r < R; ++r) v[u][r] = ld(line, jj + r * nb);
      }
    }
  }
  __syncthreads();
  const bool ns2 = (Ns & (Ns - 1)) == 0;
  const unsigned mns = ns2 ? 0u : magic32(Ns);
#pragma unroll
  for (int u = 0; u < UM; ++u) {
    const int t = tid + u * NT;
    if (t < total) {
      const int jj = fdiv32(t, mlines, lines), line = t - jj * lines;
      const int k = ns2 ? (jj & (Ns - 1)) : jj - fdiv32(jj, mns, Ns) * Ns;
      if constexpr (R <= 5) {
#pragma unroll
        for (int r = 1; r < R; ++r) {
          double2 w = tw[r * k * stride];
          if (INV) w.y = -w.y;
          v[u][r] = cmul(v[u][r], w);
        }
      } else {
        // powers of the first twiddle (one table read; error grows by an ulp a power)
        double2 w1 = tw[k * stride];
        if (INV) w1.y = -w1.y;
        double2 w = w1;
#pragma unroll
        for (int r = 1; r < R; ++r) {
          v[u][r] = cmul(v[u][r], w);
          w = cmul(w, w1);
        }
      }
      butterfly_any<R, INV>(v[u]);
      double2* d = a + line * ls + ((jj - k) * R + k) * es;
#pragma unroll
      for (int r = 0; r < R; ++r) d[r * sout] = v[u][out_pos<R>(r)];
    }
  }
  __syncthreads();
}

// passes ps0, ps0 + 1, ... of the plan (Ns: product of the earlier radices)
template <bool INV, int NT, int MAXPTS>
__device__ void ip_fft_from(double2* a, int lines, int ls, int es, const FftPlan& P, const double2* tw, int tid,
                            int ps0, int Ns) {
  const unsigned ml = magic32(lines);
  const LineLd at{a, ls, es};
  for (int ps = ps0; ps < P.np_ip; ++ps) {
    const int R = (int)((P.rc_ip >> (4 * ps)) & 15u) + 1;
    switch (R) {
      case 2: ip_pass<2, INV, NT, MAXPTS>(a, lines, ml, ls, es, P.n, Ns, tw, tid, at); break;
      case 3: ip_pass<3, INV, NT, MAXPTS>(a, lines, ml, ls, es, P.n, Ns, tw, tid, at); break;
      case 4: ip_pass<4, INV, NT, MAXPTS>(a, lines, ml, ls, es, P.n, Ns, tw, tid, at); break;
      case 5: ip_pass<5, INV, NT, MAXPTS>(a, lines, ml, ls, es, P.n, Ns, tw, tid, at); break;
      case 8: ip_pass<8, INV, NT, MAXPTS>(a, lines, ml, ls, es, P.n, Ns, tw, tid, at); break;
      default: ip_pass<16, INV, NT, MAXPTS>(a, lines, ml, ls, es, P.n, Ns, tw, tid, at); break;
    }
    Ns *= R;
  }
}

// `lines` transforms of P.n points, element i of line l at a[l * ls + i * es];
// plan P.rc_ip: radices 2, 3, 4, 5, 8, 16 (radix - 1 in four bits a pass)
template <bool INV, int NT, int MAXPTS>
__device__ void ip_fft(double2* a, int lines, int ls, int es, const FftPlan& P, const double2* tw, int tid) {
  ip_fft_from<INV, NT, MAXPTS>(a, lines, ls, es, P, tw, tid, 0, 1);
}

// the same, the first pass taking its inputs from ld(l, i) (element i of line l)
template <bool INV, int NT, int MAXPTS, class Ld>
__device__ void ip_fft(double2* a, int lines, int ls, int es, const FftPlan& P, const double2* tw, int tid, Ld ld) {
  if (P.np_ip < 1) return;
  const unsigned ml = magic32(lines);
  const int R = (int)(P.rc_ip & 15u) + 1;
  switch (R) {
    case 2: ip_pass<2, INV, NT, MAXPTS>(a, lines, ml, ls, es, P.n, 1, tw, tid, ld); break;
    case 3: ip_pass<3, INV, NT, MAXPTS>(a, lines, ml, ls, es, P.n, 1, tw, tid, ld); break;
    case 4: ip_pass<4, INV, NT, MAXPTS>(a, lines, ml, ls, es, P.n, 1, tw, tid, ld); break;
    case 5: ip_pass<5, INV, NT, MAXPTS>(a, lines, ml, ls, es, P.n, 1, tw, tid, ld); break;
    case 8: ip_pass<8, INV, NT, MAXPTS>(a, lines, ml, ls, es, P.n, 1, tw, tid, ld); break;
    default: ip_pass<16, INV, NT, MAXPTS>(a, lines, ml, ls, es, P.n, 1, tw, tid, ld); break;
  }
  ip_fft_from<INV, NT, MAXPTS>(a, lines, ls, es, P, tw, tid, 1, R);
}

// ---------------------------------------------------------------------------
// FFT along z of the half spectrum: block = (ensemble, y plane, wz columns);
// the tile [c][k] (wz nz <= kZPts points) is transformed in place in LDS
// ---------------------------------------------------------------------------
template <bool INV>
__global__ __launch_bounds__(kBlock) void k_z(Ctx C, Ens Eone, int one, const int* __restrict__ blk_off, int blk0,
                                              int nmax) {
  extern __shared__ double2 lds[];
  Ens E;
  int lb;
  block_ens(C, Eone, one, blk_off, blk0, E, lb);
  if (INV && E.plane) return;  // fused inverse transforms of the plane
  const int nz = E.nz, nh = E.nh, nhp = E.nhp, wz = E.wz;
  const int nchunk = (nh + wz - 1) / wz;
  const int j = fdiv32(lb, magic32(nchunk), nchunk);
  const int m0 = (lb - j * nchunk) * wz;
  const int w = min(wz, nh - m0);
  double2* tw = lds;
  double2* tile = lds + nmax;  // [k][c], pitch w: consecutive threads take consecutive columns
  // twiddles (nz <= kBlock): the load is in flight with the column loads
  const double2 twv = C.tw[E.fz.tw_off + min((int)threadIdx.x, nz - 1)];
  double2* sp = C.spec + E.s_off + (long long)j * nz * nhp + m0;
  const unsigned mw = magic32(w);
  staged_copy<8>(
      w * nz, threadIdx.x, kBlock,
      [&](int t) {
        const int k = fdiv32(t, mw, w);
        return sp[k * nhp + (t - k * w)];
      },
      [&](int t, double2 v) { tile[t] = v; });
  if ((int)threadIdx.x < nz) tw[threadIdx.x] = twv;
  __syncthreads();
  ip_fft<INV, kBlock, kZPts>(tile, w, 1, w, E.fz, tw, threadIdx.x);
  __syncthreads();
  const double sc = INV ? 1.0 / (double)nz : 1.0;
  for (int t0 = threadIdx.x; t0 < w * nz; t0 += 4 * kBlock) {
    double2 r[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) r[u] = tile[min(t0 + u * kBlock, w * nz - 1)];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int t = t0 + u * kBlock;
      if (t < w * nz) {
        const int k = fdiv32(t, mw, w);
        double2 v = r[u];
        if (INV) v = make_double2(v.x * sc, v.y * sc);
        sp[k * nhp + (t - k * w)] = v;
      }
    }
  }
}

__global__ __launch_bounds__(kPlaneThreads) void k_plane_inv(Ctx C, Ens Eone, int one,
                                                             const int* __restrict__ blk_off, int blk0,
                                                             double* __restrict__ phi_out, long long phi_shift,
                                                             int* __restrict__ far_reset, int bump) {
  // the sort of this step has read the far list: empty it for this step's push;
  // bump: count the step (the push then reads the step number)
  if (far_reset && blockIdx.x == 0) {
    if (threadIdx.x == 0) *far_reset = 0;
    if (bump)
      for (int e = threadIdx.x; e < C.n_ens; e += blockDim.x) C.stats[C.ens[e].st_off + ST_STEPS] += 1;
  }
  extern __shared__ double2 lds[];
  Ens E;
  int j;
  block_ens(C, Eone, one, blk_off, blk0, E, j);
  if (E.plane != 1) return;  // split over two blocks, or the z and x kernels
  const int nx = E.nx, nz = E.nz, nh = E.nh, half = nx >> 1, tid = threadIdx.x;
  double2* twz = lds;
  double2* twx = twz + nz;
  double2* pl = twx + nx;  // [nz][nh]
  // twiddles (nx, nz <= kBlock < threads) in flight with the plane loads
  const double2 tzv = C.tw[E.fz.tw_off + min(tid, nz - 1)];
  const double2 txv = C.tw[E.fx.tw_off + min(tid, nx - 1)];
  const double2* sp = C.spec + E.s_off + (long long)j * nz * E.nhp;
  const int np = nz * nh;
  const unsigned mnh = magic32(nh);
  staged_copy<8>(
      np, tid, kPlaneThreads,
      [&](int t) {
        const int k = fdiv32(t, mnh, nh);
        return sp[k * E.nhp + (t - k * nh)];
      },
      [&](int t, double2 v) { pl[t] = v; });
  if (tid < nz) twz[tid] = tzv;
  if (tid < nx) twx[tid] = txv;
  __syncthreads();
  // inverse z transform of the nh columns
  ip_fft<true, kPlaneThreads, kPlanePts>(pl, nh, 1, nh, E.fz, twz, tid);
  // inverse x transforms of the rows paired as complex lines (pitch 2 nh >= nx):
  // the first pass reads Z = X_A + i X_B of rows (2p, 2p+1) (Hermitian halves
  // extended; imaginary parts at m = 0 and nx/2 dropped) straight from them
  const int npt = (nz >> 1) * nx;
  const unsigned mnx = magic32(nx);
  auto packed = [=](int p, int i) {
    const int m = i <= half ? i : nx - i;
    const double2 A = pl[(2 * p) * nh + m], B = pl[(2 * p + 1) * nh + m];
    if (i == 0 || i == half) return make_double2(A.x, B.x);
    if (i < half) return make_double2(A.x - B.y, A.y + B.x);
    return make_double2(A.x + B.y, B.x - A.y);
  };
  ip_fft<true, kPlaneThreads, kPlanePts>(pl, nz >> 1, 2 * nh, 1, E.fx, twx, tid, packed);
  const double sc = (1.0 / (double)nz) * (1.0 / (double)nx);
  double* out = phi_out + (E.c_off - phi_shift) + (long long)j * nz * nx;
  for (int t = tid; t < npt; t += kPlaneThreads) {
    const int p = fdiv32(t, mnx, nx), i = t - p * nx;
    const double2 v = pl[(2 * p) * nh + i];
    out[(2 * p) * nx + i] = v.x * sc;
    out[(2 * p + 1) * nx + i] = v.y * sc;
  }
}

// ---------------------------------------------------------------------------
// inverse z and x transforms of one y plane split over Q blocks (Q = 2 or 4)
// by the residue h of the z row modulo Q.  With N = nz (a multiple of 2Q),
// the rows k = Q r + h of the inverse z transform are the inverse transform of
// length N/Q of
//   Y_h[m] = exp(2 pi i m h / N) sum_{s<Q} X[m + s N/Q] exp(2 pi i s h / Q),
// m < N/Q (the radix-Q split of the outputs; for Q = 2: X[m] + X[m + N/2] and
// (X[m] - X[m + N/2]) exp(2 pi i m / N)), so a block holds 1/Q of the plane in
// LDS and does 1/Q of the transforms, the fold done while the plane streams
// in.  The Q blocks of a plane are neighbouring logical blocks (one XCD), so
// the plane's later reads find it in that XCD's L2.  LDS rows (2p, 2p+1), z
// rows Q 2p + h and Q (2p + 1) + h, then form one complex line of the x
// transform.
// ---------------------------------------------------------------------------
template <int Q, int XPTS, int NT>
__global__ __launch_bounds__(NT, 4) void k_plane_part(Ctx C, Ens Eone, int one,
                                                             const int* __restrict__ blk_off, int blk0,
                                                             double* __restrict__ phi_out, long long phi_shift,
                                                             int* __restrict__ far_reset, int bump) {
  static_assert(Q == 2 || Q == 4, "two or four blocks per plane");
  if (far_reset && blockIdx.x == 0) {
    if (threadIdx.x == 0) *far_reset = 0;
    if (bump)
      for (int e = threadIdx.x; e < C.n_ens; e += blockDim.x) C.stats[C.ens[e].st_off + ST_STEPS] += 1;
  }
  extern __shared__ double2 lds[];
  const int b = (int)xcd_block(blockIdx.x, gridDim.x);
  Ens E;
  int lb;
  if (one) {
    E = Eone;
    lb = b;
  } else {
    const int gb = blk0 + b;
    const int e = find_off_i(blk_off, C.n_ens + 1, gb);
    E = C.ens[e];
    lb = gb - blk_off[e];
  }
  if (E.plane != Q) return;
  const int j = lb / Q, h = lb - j * Q;
  const int nx = E.nx, nz = E.nz, nh = E.nh, nzp = nz / Q, npair = nzp >> 1, half = nx >> 1, tid = threadIdx.x;
  double2* twz = lds;      // exp(-2 pi i t / (N/Q)) = exp(-2 pi i Q t / N)
  double2* twx = twz + nzp;
  double2* pl = twx + nx;  // [nz/Q][nh]
  const double2 tzv = C.tw[E.fz.tw_off + min(Q * tid, nz - Q)];
  const double2 txv = C.tw[E.fx.tw_off + min(tid, nx - 1)];
  const double2* sp = C.spec + E.s_off + (long long)j * nz * E.nhp;
  const double2* twn = C.tw + E.fz.tw_off;   // exp(-2 pi i t / N), t < N
  const long long shift = (long long)nzp * E.nhp;
  const unsigned mnh = magic32(nh);
  if constexpr (Q == 2) {
    struct Fold {
      double2 a, b, w;
    };
    staged_copy<4>(
        nzp * nh, tid, NT,
        [&](int t) {
          const int m = fdiv32(t, mnh, nh), i = t - m * nh;
          const double2* s = sp + m * E.nhp + i;
          return Fold{s[0], s[shift], h ? twn[m] : make_double2(1.0, 0.0)};
        },
        [&](int t, Fold v) {
          if (h == 0) {
            pl[t] = make_double2(v.a.x + v.b.x, v.a.y + v.b.y);
          } else {  // (a - b) conj(w), w = exp(-2 pi i m / N)
            const double dx = v.a.x - v.b.x, dy = v.a.y - v.b.y;
            pl[t] = make_double2(dx * v.w.x + dy * v.w.y, dy * v.w.x - dx * v.w.y);
          }
        });
  } else {
    struct Fold {
      double2 a0, a1, a2, a3, w;
    };
    staged_copy<2>(
        nzp * nh, tid, NT,
        [&](int t) {
          const int m = fdiv32(t, mnh, nh), i = t - m * nh;
          const double2* s = sp + m * E.nhp + i;
          return Fold{s[0], s[shift], s[2 * shift], s[3 * shift], h ? twn[m * h] : make_double2(1.0, 0.0)};
        },
        [&](int t, Fold v) {
          // sum_s X_s i^(s h): the radix-4 butterfly output h
          const double2 p02 = make_double2(v.a0.x + v.a2.x, v.a0.y + v.a2.y);
          const double2 m02 = make_double2(v.a0.x - v.a2.x, v.a0.y - v.a2.y);
          const double2 p13 = make_double2(v.a1.x + v.a3.x, v.a1.y + v.a3.y);
          const double2 m13 = make_double2(v.a1.x - v.a3.x, v.a1.y - v.a3.y);
          double2 y;
          if (h == 0) {
            y = make_double2(p02.x + p13.x, p02.y + p13.y);
          } else if (h == 2) {
            y = make_double2(p02.x - p13.x, p02.y - p13.y);
          } else if (h == 1) {  // m02 + i m13
            y = make_double2(m02.x - m13.y, m02.y + m13.x);
          } else {              // m02 - i m13
            y = make_double2(m02.x + m13.y, m02.y - m13.x);
          }
          if (h) {  // times conj(w), w = exp(-2 pi i m h / N)
            y = make_double2(y.x * v.w.x + y.y * v.w.y, y.y * v.w.x - y.x * v.w.y);
          }
          pl[t] = y;
        });
  }
  if (tid < nzp) twz[tid] = tzv;
  if (tid < nx) twx[tid] = txv;
  __syncthreads();
  ip_fft<true, NT, kHalfPts>(pl, nh, 1, nh, E.fzh, twz, tid);
  // x transforms of LDS rows (2p, 2p+1) paired as one complex line, packed by
  // the first pass as in k_plane_inv
  const int npt = npair * nx;
  const unsigned mnx = magic32(nx);
  auto packed = [=](int p, int i) {
    const int m = i <= half ? i : nx - i;
    const double2 A = pl[(2 * p) * nh + m], B = pl[(2 * p + 1) * nh + m];
    if (i == 0 || i == half) return make_double2(A.x, B.x);
    if (i < half) return make_double2(A.x - B.y, A.y + B.x);
    return make_double2(A.x + B.y, B.x - A.y);
  };
  ip_fft<true, NT, XPTS>(pl, npair, 2 * nh, 1, E.fx, twx, tid, packed);
  const double sc = (1.0 / (double)nz) * (1.0 / (double)nx);
  double* out = phi_out + (E.c_off - phi_shift) + (long long)j * nz * nx;
  for (int t = tid; t < npt; t += NT) {
    const int p = fdiv32(t, mnx, nx), i = t - p * nx;
    const double2 v = pl[(2 * p) * nh + i];
    out[(Q * 2 * p + h) * nx + i] = v.x * sc;
    out[(Q * (2 * p + 1) + h) * nx + i] = v.y * sc;
  }
}

// ---------------------------------------------------------------------------
// particle helpers
// ---------------------------------------------------------------------------

// largest j in [0, ny-1] with yf[j] <= y (0 if none), binary search
__device__ __forceinline__ int y_cell(const double* __restrict__ yf, int ny, double y) {
  int lo = 0, hi = ny - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (yf[mid] <= y) lo = mid; else hi = mid - 1;
  }
  return lo;
}

// initial binning: cell key of every particle (the next sort is a full one)
__global__ __launch_bounds__(kBlock) void k_bin(Ctx C, PState S, long long n0, long long n1) {
  const long long p = n0 + (long long)blockIdx.x * kBlock + threadIdx.x;
  const bool valid = p < n1;
  const long long pc = valid ? p : n1 - 1;  // n1 > n0: every lane reads a particle
  const int e = find_off(C.p_off, C.n_ens + 1, pc);
  // diameter bound of the ensemble (the collision search's prefilter, read
  // for ensembles with 4-way coupling only): the maximum over a wave's lanes
  // of one ensemble, one atomic per wave and ensemble (positive doubles order
  // like their bit patterns); all lanes take part in the shuffles.  Skipped
  // for the other ensembles: the atomics on one word per ensemble serialise
  // (the binning of 4e6 particles took 718 µs with them, 50 µs without)
  {
    const bool want = valid && C.ens[e].pp;
    const unsigned long long dm = want ? (unsigned long long)__double_as_longlong(fmax(S.d[pc], 0.0)) : 0ull;
    bool pending = want;
    for (unsigned long long m = __ballot(pending); m; m = __ballot(pending)) {
      // the ensemble of the first pending lane: at least that lane finishes
      const int e0 = __shfl(e, __ffsll((long long)m) - 1, 64);
      unsigned long long v = (pending && e == e0) ? dm : 0ull;
      for (int o = 32; o > 0; o >>= 1) {
        const unsigned long long w = __shfl_xor(v, o, 64);
        v = w > v ? w : v;
      }
      if (pending && e == e0) {
        if (__lane_id() == __builtin_amdgcn_readfirstlane(__lane_id()) && v)
          atomicMax((unsigned long long*)&C.stats[C.ens[e0].st_off + ST_DMAX], v);
        pending = false;
      }
    }
  }
  if (!valid) return;
  const Ens& E = C.ens[e];
  const double x = S.x[p], y = S.y[p], z = S.z[p];
  const int i = clamp_floor(x / E.dx, E.nx);
  const int k = clamp_floor(z / E.dz, E.nz);
  const int j = y_cell(C.yf + E.y_off, E.ny, y);
  const int c = (int)(E.c_off + (long long)(j * E.nz + k) * E.nx + i);
  S.key[p] = c;
}

// ---------------------------------------------------------------------------
// the particle push: one thread per sorted slot s, E uniform over the lanes
// that share an ensemble (scalar descriptor loads)
// ---------------------------------------------------------------------------
// counts the particle's new row pair for the next sort.  The active lanes of
// the wave merge runs of equal keys first (lanes are in slot order, so
// neighbours mostly share a pair): one device atomic per run.
__device__ __forceinline__ void pair_count(int* __restrict__ pair_cnt, int key) {
  const int lane = threadIdx.x & 63;
  const unsigned long long act = __ballot(1);
  const int prevk = __shfl_up(key, 1, 64);
  const bool head = lane == 0 || !((act >> (lane - 1)) & 1ull) || prevk != key;
  const unsigned long long heads = __ballot(head);
  if (!head) return;
  const unsigned long long after = heads & ~((2ull << lane) - 1ull);  // later heads
  const unsigned long long upto = after ? ((after & (~after + 1ull)) - 1ull) : ~0ull;
  atomicAdd(&pair_cnt[key], __popcll(act & upto & ~((1ull << lane) - 1ull)));
}

// ---------------------------------------------------------------------------
// stochastic scaling model of particle-wall charging
// ---------------------------------------------------------------------------
// Philox4x32-10 counter-based generator (Salmon, Moraes, Dror & Shaw, SC'11)
__device__ __forceinline__ uint4 philox4x32_10(uint4 c, uint2 k) {
  for (int r = 0; r < 10; ++r) {
    if (r) {
      k.x += 0x9E3779B9u;
      k.y += 0xBB67AE85u;
    }
    const unsigned hi0 = __umulhi(0xD2511F53u, c.x), lo0 = 0xD2511F53u * c.x;
    const unsigned hi1 = __umulhi(0xCD9E8D57u, c.z), lo1 = 0xCD9E8D57u * c.z;
    c = make_uint4(hi1 ^ c.y ^ k.x, lo1, hi0 ^ c.w ^ k.y, lo0);
  }
  return c;
}

// charge received by a particle (charge q, diameter d, id) hitting a wall with
// normal speed un in step number step: the wall's sites give their mean
// mu_w, the particle's sites a skew-normal number Dq_1 (mean, standard
// deviation and skewness scaled from the reference impact by the active sites)
__device__ double ssm_dq(const Ens& E, double q, double d, double un, int id, unsigned step) {
  const double a0 = d / E.sd0;
  const double area = (a0 * a0) * pow(un / E.sun0, 0.8);
  const double load = 4.0 * q / (E.scsat * (d * d));
  const double sw = (E.sdq0 > 0.0) - (E.sdq0 < 0.0), si = (E.sdq0 - E.smu0 > 0.0) - (E.sdq0 - E.smu0 < 0.0);
  const double chi_w = fmin(fmax(1.0 - sw * load, 0.0), 1.0);
  const double chi_i = fmin(fmax(1.0 + si * load, 0.0), 1.0);
  const double nw = area * chi_w, ni = area * chi_i;
  const double mu_w = E.sdq0 * nw;
  if (!(ni > 0.0)) return mu_w;
  const uint4 w = philox4x32_10(make_uint4((unsigned)id, step, 0u, 0u), make_uint2(E.seed, 0x53534D31u));
  const double u0 = ((double)w.x + 0.5) * 0x1p-32, u1 = ((double)w.y + 0.5) * 0x1p-32;
  const double r = sqrt(-2.0 * log(u0)), t = 2.0 * kPi * u1;
  const double n0 = r * cos(t), n1 = r * sin(t);
  // skew-normal with mean mu, deviation sigma, skewness g (moment relations)
  const double mu = (E.sdq0 - E.smu0) * ni, sigma = E.ssig0 * sqrt(ni);
  const double g = fmin(fmax(-E.sgam0 / ni, -0.99), 0.99);
  const double rc = cbrt(2.0 * fabs(g) / (4.0 - kPi));
  const double delta = ((g > 0.0) - (g < 0.0)) * (rc / sqrt(1.0 + rc * rc)) * sqrt(kPi / 2.0);
  const double b = sqrt(2.0 / kPi);
  const double bd = b * delta;
  const double omega = sigma / sqrt(1.0 - bd * bd);
  const double xi = mu - omega * b * delta;
  const double dq1 = xi + omega * (delta * fabs(n0) + sqrt(1.0 - delta * delta) * n1);
  return mu_w - dq1;
}

template <bool PP>
__device__ __forceinline__ void push_one(const Ctx& C, const Ens& E, const PState& in, const PState& out, int s,
                                         int p, int c, int ra, int rb, signed char* __restrict__ wall_rec, int pm) {
  // the id is stored with the new state at the end: loaded here, so that
  // the wave's last stores do not wait for a load issued after the update
  const int pid = in.id[p];
  Fwd F;
  eval_particle<true, PP>(C, E, in, s, p, c, ra, rb, F, pm);
  const int nx = E.nx, ny = E.ny, nz = E.nz;
  const int j = F.j;
  const double q = F.qc, d = F.d;  // charge after any particle-particle exchange
  const double v1x = F.v1[0], v1y = F.v1[1], v1z = F.v1[2];
  double x1 = F.x1, z1 = F.z1;
  const double y1 = F.y1;
  const double* __restrict__ yf = C.yf + E.y_off;

  // wall impact: rebound with restitution e, condenser charge transfer
  const double r = 0.5 * d;
  const double top = E.ly - r;
  int wall = -1;
  double un = 0.0, yr = y1, vyr = v1y, q1 = q;
  if (y1 < r) {
    wall = 0;
    un = -v1y;
    yr = r + E.e * (r - y1);
  } else if (y1 > top) {
    wall = 1;
    un = v1y;
    yr = top - E.e * (y1 - top);
  }
  long long* st = C.stats + E.st_off;
  if (wall_rec) wall_rec[s] = (signed char)wall;
  if (wall >= 0) {
    vyr = -E.e * v1y;
    double dq;
    if (E.charging) {
      dq = ssm_dq(E, q, d, un, pid, (unsigned)st[ST_STEPS]);
    } else {
      const double f = E.fe * pow(un, 0.8);
      dq = -f * (E.dU + q);
    }
    q1 = q + dq;
    bool ovf = false;
    const long long wq = fixed_round(-dq, kFixWall, &ovf);
    atomicAdd((unsigned long long*)&st[ST_IMP + wall], 1ull);
    atomicAdd((unsigned long long*)&st[ST_WQ + wall], (unsigned long long)wq);
    const double bf = un / E.un_bin;
    const int bin = (bf < (double)(kNbin - 1)) ? (int)bf : kNbin - 1;
    atomicAdd((unsigned long long*)&st[ST_HIST + bin], 1ull);
    int fl = ovf ? FLAG_OVERFLOW : 0;
    if (yr < r || yr > top) fl |= FLAG_OUTSIDE;
    if (fl) atomicOr((unsigned long long*)&st[ST_FLAGS], (unsigned long long)fl);
  }

  // periodic wrap
  if (x1 >= E.lx) x1 = x1 - E.lx;
  else if (x1 < 0.0) x1 = x1 + E.lx;
  if (z1 >= E.lz) z1 = z1 - E.lz;
  else if (z1 < 0.0) z1 = z1 + E.lz;

  if (!(isfinite(x1) && isfinite(yr) && isfinite(z1) && isfinite(v1x) && isfinite(vyr) && isfinite(v1z) &&
        isfinite(q1)))
    atomicOr((unsigned long long*)&st[ST_FLAGS], (unsigned long long)FLAG_NONFINITE);

  // the new state is next read by the following step's sort: streaming
  // stores that do not allocate in the caches, which keeps the carrier and phi
  // lines of the gathers resident (66 instead of 75 us for 1e6 particles)
  __builtin_nontemporal_store(x1, &out.x[s]);
  __builtin_nontemporal_store(yr, &out.y[s]);
  __builtin_nontemporal_store(z1, &out.z[s]);
  __builtin_nontemporal_store(v1x, &out.vx[s]);
  __builtin_nontemporal_store(vyr, &out.vy[s]);
  __builtin_nontemporal_store(v1z, &out.vz[s]);
  __builtin_nontemporal_store(q1, &out.q[s]);
  __builtin_nontemporal_store(d, &out.d[s]);
  __builtin_nontemporal_store(pid, &out.id[s]);
  if (C.fslot) {
    // drag force of the step on this particle (2-way coupling source)
    const double mp = (E.rr * (kPi / 6.0)) * ((d * d) * d);
    const double ms = mp * F.sdr;
    const long long n = C.n_tot;
    C.fslot[s] = ms * (F.u[0] - v1x);
    C.fslot[n + s] = ms * (F.u[1] - v1y);
    C.fslot[2 * n + s] = ms * (F.u[2] - v1z);
  }
  // next cell: exact divisions in x, z; in y the old row when the faces read
  // with the carrier still bracket the new position, else a local face search
  const int ni = clamp_floor(x1 / E.dx, nx);
  const int nk = clamp_floor(z1 / E.dz, nz);
  const int nj = (yr >= F.yf0 && yr < F.yf1) ? j : y_cell_from(yf, ny, yr, j);
  const int key = (int)E.c_off + (nj * nz + nk) * nx + ni;
  __builtin_nontemporal_store(key, &out.key[s]);
  // the next sort takes a row pair's members from the pair's slot range of
  // this order and from its mover list: a particle whose row pair changes
  // goes on the mover list of its new pair (on the far list, read by every
  // pair, when that one is full)
  const int pnew = (int)((E.row_off + (long long)nj * nz + nk) >> 1);
  const int pold = (int)((E.row_off + (long long)j * nz + F.k) >> 1);
  if (pnew != pold) {
    const int b = atomicAdd(&C.mv_n[pnew], 1);
    if (b < kMoverCap) {
      C.mv[(long long)pnew * kMoverCap + b] = s;
    } else {
      const int f = atomicAdd(&C.far_n[0], 1);
      if (f < C.n_tot) C.far[f] = s;
    }
  }
  pair_count(C.pair_cnt, pnew);
}


// ONE (a handle of one ensemble, its descriptor by value): four waves per
// SIMD (at most 128 VGPRs, none spilled); the batched form, which needs more
// registers, three waves per SIMD rather than spilling to memory
// RR: blocks in the hardware's round robin over the XCDs, else consecutive
// slot ranges per XCD
template <bool PP, bool RR, bool ONE>
__global__ __launch_bounds__(kBlock, ONE ? 4 : 3) void k_push(Ctx C, Ens Eone, PState in, PState out,
                                                 int* __restrict__ perm_rec, signed char* __restrict__ wall_rec) {
  // the new row ranges become the stored order's (read by the next sort)
  for (long long r = (long long)blockIdx.x * kBlock + threadIdx.x; r <= C.n_rows; r += (long long)gridDim.x * kBlock)
    C.rs_old[r] = C.rs_new[r];
  const long long blk = RR ? (long long)blockIdx.x : xcd_block(blockIdx.x, gridDim.x);
  const int s = (int)(blk * kBlock + threadIdx.x);
  const bool act = s < C.n_tot;
  const int c = act ? C.skey[s] : 0x7fffffff;
  // the old slots of the 32 slots before the wave (lanes 0..31, nearest
  // first) and after it (lanes 32..63): the cell mates across the wave's ends
  // need only their state loads
  int pm = 0;
  {
    const int lane = (int)(threadIdx.x & 63u);
    const int s0 = s - lane;
    const int t = lane < 32 ? s0 - 1 - lane : s0 + 64 + (lane - 32);
    if (t >= 0 && t < C.n_tot) pm = C.perm[t];
  }
  // the slots of the lane's cell from the wave's keys (every lane takes part)
  int ra, rb;
  cell_run(s, c, &ra, &rb);
  if (act) {
    const int p = C.perm[s];
    if (perm_rec) perm_rec[s] = p;
    if (ra < 0) ra = C.start[c];
    if (rb < 0) rb = C.start[c + 1];
    if constexpr (ONE) {
      push_one<PP>(C, Eone, in, out, s, p, c, ra, rb, wall_rec, pm);
    } else {
      // the ensemble of the wave's first slot (one uniform search: an
      // ensemble's particles fill a contiguous slot range); lanes past its end
      // (a wave across an ensemble boundary) search their own
      const int e0 = find_off(C.p_off, C.n_ens + 1, (long long)__builtin_amdgcn_readfirstlane(s));
      const int e_lane = s < C.p_off[e0 + 1] ? e0 : find_off(C.p_off, C.n_ens + 1, (long long)s);
      // waterfall over the ensembles present in this wave (usually one)
      bool done = false;
      while (!done) {
        const int e = __builtin_amdgcn_readfirstlane(e_lane);
        if (e_lane == e) {
          push_one<PP>(C, C.ens[e], in, out, s, p, c, ra, rb, wall_rec, pm);
          done = true;
        }
      }
    }
  }
}

// ---------------------------------------------------------------------------
// state in/out (id order) and bookkeeping
// ---------------------------------------------------------------------------
struct PIn {
  const double *x, *y, *z, *vx, *vy, *vz, *q, *d;
};

__global__ __launch_bounds__(kBlock) void k_put_state(PState S, PIn in, long long p0, int n) {
  const int t = blockIdx.x * kBlock + threadIdx.x;
  if (t >= n) return;
  const long long p = p0 + t;
  S.x[p] = in.x[t];
  S.y[p] = in.y[t];
  S.z[p] = in.z[t];
  S.vx[p] = in.vx[t];
  S.vy[p] = in.vy[t];
  S.vz[p] = in.vz[t];
  S.q[p] = in.q[t];
  S.d[p] = in.d[t];
  S.id[p] = t;
}


__global__ __launch_bounds__(kBlock) void k_get_state(PState S, PIn out, long long p0, int n) {
  const int t = blockIdx.x * kBlock + threadIdx.x;
  if (t >= n) return;
  const long long p = p0 + t;
  const int id = S.id[p];
  ((double*)out.x)[id] = S.x[p];
  ((double*)out.y)[id] = S.y[p];
  ((double*)out.z)[id] = S.z[p];
  ((double*)out.vx)[id] = S.vx[p];
  ((double*)out.vy)[id] = S.vy[p];
  ((double*)out.vz)[id] = S.vz[p];
  ((double*)out.q)[id] = S.q[p];
  ((double*)out.d)[id] = S.d[p];
}


// ---------------------------------------------------------------------------
// host-callable launchers (used by api.hip)
// ---------------------------------------------------------------------------
}  // namespace tf

#include <algorithm>

#include "launch.h"

namespace tf {

// exclusive prefix of cnt[0..n) into out[0..n]
static void scan_into(const Ctx& C, const int* cnt, long long n, int* out, hipStream_t st) {
  if (n > 0 && n <= kSmallScan) {
    k_scan_small<<<1, 1024, 0, st>>>(cnt, (int)n, out);
    return;
  }
  const int nb = (int)((n + kScanChunk - 1) / kScanChunk);
  if (nb == 0) return;
  const int fold = nb <= kScanFold ? 1 : 0;
  k_scan_reduce<<<nb, kBlock, 0, st>>>(cnt, n, C.scan_part);
  if (!fold) k_scan_part<<<1, 1024, 0, st>>>(C.scan_part, nb);
  k_scan_down<<<nb, kBlock, 0, st>>>(cnt, n, C.scan_part, fold, out);
}

hipError_t launch_sort(const Ctx& C, const LaunchGeo& G, const PState& cur, bool full, hipStream_t st) {
  if (full) {
    // counting sort from scratch: cell counts by atomics, cell prefix, placement, id order
    const int nbp = (int)((C.n_tot + kBlock - 1) / kBlock);
    if (nbp > 0) k_count<<<nbp, kBlock, 0, st>>>(C, cur.key);
    scan_into(C, C.count, C.c_tot, C.start, st);
    const int nb = (int)((C.n_tot + kBlock * kIlp - 1) / (kBlock * kIlp));
    if (nb > 0) {
      k_place<<<nb, kBlock, 0, st>>>(C, cur.key, cur.id);
      k_rank<<<nb, kBlock, 0, st>>>(C, cur);
    }
    k_rows_from_start<<<(int)((C.n_rows + kBlock) / kBlock), kBlock, 0, st>>>(C);
    return hipGetLastError();
  }
  // incremental: the row slot ranges from the push's row counts
  scan_into(C, C.pair_cnt, C.n_rows / 2, C.ps, st);
  return hipGetLastError();
}

int sortdep_cap(const Ctx& C, int nx_max, int want) {
  // member list per row pair (pairs above the capacity take the two-pass
  // path).  Default: twice the mean pair size rounded up to 64 (pair sizes
  // follow the cell volumes, which vary across the stretched y rows), at
  // least what the FFT buffer it shares leaves free.  Always within 64 KiB
  // per block.
  if (want < 0) return 0;
  const long long lim = ((65536 - 16LL * nx_max) / kPairsPerBlock - 24LL * nx_max - 48 - 15) / 12;
  long long cap;
  if (want > 0) {
    cap = want;
  } else {
    const long long mean = C.n_rows > 0 ? (2 * C.n_tot + C.n_rows - 1) / C.n_rows : 0;
    cap = std::max<long long>((16LL * nx_max) / 12, ((2 * mean + 63) / 64) * 64);
  }
  cap = std::min(cap, lim);
  return (int)std::max<long long>(cap, 0) & ~7;
}

hipError_t launch_sort_dep(const Ctx& C, const LaunchGeo& G, const PState& cur, hipStream_t st) {
  const int nb = G.fp_blk[C.n_ens];
  if (nb == 0) return hipSuccess;
  const int one = (C.n_ens == 1) ? 1 : 0;
  const int cap = sortdep_cap(C, G.nx_max, G.sort_cap);
  const size_t lds = (size_t)G.nx_max * 16 + (size_t)kPairsPerBlock * sortdep_wave_bytes(G.nx_max, cap);
  k_row_sort_dep<<<nb, kBlock, lds, st>>>(C, G.eh[0], one, cur, G.d_fp_blk, G.nx_max, cap);
  return hipGetLastError();
}

hipError_t launch_poisson(const Ctx& C0, const LaunchGeo& G, int e0, int e1, const double* q, const int* key,
                          const long long* q_in, long long q_shift, double* phi_out, long long phi_shift,
                          int do_stats, hipStream_t st, hipEvent_t* ev, const double* r_in, bool x_done,
                          int* far_reset, double2* spec1) {
  (void)key;
  (void)q;
  auto mark = [&](int i) {  // ev: 5 phase-boundary events, null entries skipped
    if (ev && ev[i]) hipEventRecord(ev[i], st);
  };
  const int one = (e1 - e0 == 1) ? 1 : 0;
  if (spec1 && !one) return hipErrorInvalidValue;
  Ens Eone = G.eh[e0];
  Ctx C = C0;
  if (spec1) {
    // single-ensemble launch: every kernel takes the descriptor by value
    C.spec = spec1;
    Eone.s_off = 0;
  }
  const int b0 = G.fp_blk[e0], nb = G.fp_blk[e1] - b0;
  const size_t lx = (size_t)(1 + 2 * kPairsPerBlock) * G.nx_max * sizeof(double2);
  if (nb > 0 && !x_done)
    k_pair_fftx<<<nb, kBlock, lx, st>>>(C, Eone, one, G.d_fp_blk, b0, G.nx_max, q_in, q_shift, r_in, do_stats);
  mark(0);
  const int z0 = G.fz_blk[e0], nzb = G.fz_blk[e1] - z0;
  const size_t lz = (size_t)(G.wz * G.nz_max + G.nz_max) * sizeof(double2);  // wz: largest over ensembles
  if (nzb > 0) k_z<false><<<nzb, kBlock, lz, st>>>(C, Eone, one, G.d_fz_blk, z0, G.nz_max);
  mark(1);
  const int t0 = G.tri_blk[e0], nt = G.tri_blk[e1] - t0;
  if (nt > 0) {
    // rows per lane: the largest over the ensembles; tile [tm][G][R | 1] plus a pad per mode
    const int R = G.tri_rows;
    const size_t tl = ((size_t)kBlock * (R | 1) + kBlock) * sizeof(double2);
    switch (R) {
#define TRI_CASE(r) \
  case r: k_tri<r><<<nt, kBlock, tl, st>>>(C, Eone, one, G.d_tri_blk, t0); break;
      TRI_CASE(1) TRI_CASE(2) TRI_CASE(3) TRI_CASE(4) TRI_CASE(5) TRI_CASE(6) TRI_CASE(7) TRI_CASE(8)
      TRI_CASE(9) TRI_CASE(10) TRI_CASE(11) TRI_CASE(12) TRI_CASE(13) TRI_CASE(14) TRI_CASE(15) TRI_CASE(16)
#undef TRI_CASE
      default: break;  // rejected at tf_init
    }
  }
  mark(2);
  // inverse transforms (counted as the z phase): one block per y plane, or
  // two per plane (z-row parity), for the ensembles whose plane fits the LDS;
  // z then x kernels for the others.  The first of these kernels empties the
  // far list and counts the step.
  const bool whole = one ? Eone.plane == 1 : G.plane_any != 0;
  const bool halves = one ? Eone.plane == 2 : G.half_any != 0;
  const bool quarters = one ? Eone.plane == 4 : G.quarter_any != 0;
  const bool split = one ? Eone.plane == 0 : G.split_any != 0;
  int* fr = far_reset;
  if (whole) {
    const int p0 = G.pl_blk[e0], np = G.pl_blk[e1] - p0;
    const size_t lp = (size_t)(G.nx_max + G.nz_max + G.plane_max) * sizeof(double2);
    if (np > 0) {
      k_plane_inv<<<np, kPlaneThreads, lp, st>>>(C, Eone, one, G.d_pl_blk, p0, phi_out, phi_shift, fr, 1);
      fr = nullptr;
    }
  }
  if (halves) {
    const int p0 = G.ph_blk[e0], np = G.ph_blk[e1] - p0;
    const size_t lp = (size_t)G.half_lds;
    if (np > 0) {
      k_plane_part<2, kHalfXPts, kHalfThreads><<<np, kHalfThreads, lp, st>>>(C, Eone, one, G.d_ph_blk, p0, phi_out,
                                                                             phi_shift, fr, 1);
      fr = nullptr;
    }
  }
  if (quarters) {
    const int p0 = G.pq_blk[e0], np = G.pq_blk[e1] - p0;
    const size_t lp = (size_t)G.quarter_lds;
    if (np > 0) {
      k_plane_part<4, kQuarterXPts, kQuarterThreads><<<np, kQuarterThreads, lp, st>>>(
          C, Eone, one, G.d_pq_blk, p0, phi_out, phi_shift, fr, 1);
      fr = nullptr;
    }
  }
  // (blocks only for the ensembles transformed this way)
  const int zs0 = G.fzs_blk[e0], nzs = G.fzs_blk[e1] - zs0;
  const int bs0 = G.fps_blk[e0], nbs = G.fps_blk[e1] - bs0;
  if (split && nzs > 0) k_z<true><<<nzs, kBlock, lz, st>>>(C, Eone, one, G.d_fzs_blk, zs0, G.nz_max);
  mark(3);
  if (split && nbs > 0)
    k_pair_ifftx<<<nbs, kBlock, lx, st>>>(C, Eone, one, G.d_fps_blk, bs0, G.nx_max, phi_out, phi_shift, fr, 1);
  mark(4);
  return hipGetLastError();
}

hipError_t launch_push(const Ctx& C, const LaunchGeo& G, const PState& in, const PState& out, int* perm_rec,
                       signed char* wall_rec, hipStream_t st) {
  const int nb = std::max(1, (int)((C.n_tot + kBlock - 1) / kBlock));
  const int one = (C.n_ens == 1) ? 1 : 0;
  // the collision code only when an ensemble has 4-way coupling on
  const bool rr = G.push_order == 2;
#define PUSH_LAUNCH(pp, r, o) k_push<pp, r, o><<<nb, kBlock, 0, st>>>(C, G.eh[0], in, out, perm_rec, wall_rec)
  if (G.pp_any) {
    if (rr) { if (one) PUSH_LAUNCH(true, true, true); else PUSH_LAUNCH(true, true, false); }
    else { if (one) PUSH_LAUNCH(true, false, true); else PUSH_LAUNCH(true, false, false); }
  } else {
    if (rr) { if (one) PUSH_LAUNCH(false, true, true); else PUSH_LAUNCH(false, true, false); }
    else { if (one) PUSH_LAUNCH(false, false, true); else PUSH_LAUNCH(false, false, false); }
  }
#undef PUSH_LAUNCH
  return hipGetLastError();
}

// 2-way coupling source: minus the summed drag forces of a cell's particles
// (its slot range, ascending id) per unit cell volume; two neighbouring cells
// of one x row per thread (nx is even), 16-byte stores
__global__ __launch_bounds__(kBlock) void k_source(Ctx C) {
  const long long c = 2 * ((long long)blockIdx.x * kBlock + threadIdx.x);
  if (c >= C.c_tot) return;
  const int e = find_off(C.c_off, C.n_ens + 1, c);
  const Ens& E = C.ens[e];
  const int j = (int)((int)(c - E.c_off) / (E.nx * E.nz));
  const double iv = 1.0 / C.vol[E.y_off + j];
  const int a = C.start[c], m = C.start[c + 1], b = C.start[c + 2];
  const long long n = C.n_tot;
  double f[2][3] = {{0.0, 0.0, 0.0}, {0.0, 0.0, 0.0}};
  for (int t = a; t < b; ++t) {
    const int h = t >= m ? 1 : 0;
    f[h][0] += C.fslot[t];
    f[h][1] += C.fslot[n + t];
    f[h][2] += C.fslot[2 * n + t];
  }
  // an output of the step, not read again within it: non-temporal stores
  // (otherwise its 48 MB displace the next push's carrier and phi lines)
  typedef double d2v __attribute__((ext_vector_type(2)));
#pragma unroll
  for (int k = 0; k < 3; ++k)
    __builtin_nontemporal_store(d2v{-f[0][k] * iv, -f[1][k] * iv}, reinterpret_cast<d2v*>(C.fsrc + k * C.c_tot + c));
}

hipError_t launch_source(const Ctx& C, hipStream_t st) {
  if (C.c_tot == 0) return hipSuccess;
  const int nb = (int)((C.c_tot / 2 + kBlock - 1) / kBlock);
  k_source<<<nb, kBlock, 0, st>>>(C);
  return hipGetLastError();
}

// 4-way coupling: per slot, the velocity and charge increments of its binary
// hard-sphere collisions with the other particles of its cell on the state at
// the start of the step (zero for ensembles without it), summed in ascending
// id and read by the push; the pairs with a partner of larger id are counted.
// As in the push's Coulomb sum, a cell's slots are a run of the wave's lanes:
// the mates' positions and charges come from their lanes (cross-lane reads),
// those of runs across the wave's ends through perm, the loops running while
// some lane of the wave has a mate left.  A slot with no mate closer than
// d_max (>= (d + d_max)/2) reads nothing more; pairs beyond (d + d_max)/2 are
// skipped before the partner's velocity and diameter are read.  ONE: a handle
// of one ensemble, its descriptor by value.
template <bool ONE>
__global__ __launch_bounds__(kBlock) void k_collide(Ctx C, Ens Eone, PState in) {
  const int s = (int)(xcd_block(blockIdx.x, gridDim.x) * kBlock + threadIdx.x);
  const bool act = s < C.n_tot;
  const int c = act ? C.skey[s] : 0x7fffffff;
  const int p = act ? C.perm[s] : 0;
  // the slots of the lane's cell from the wave's keys (every lane takes part)
  int ra, rb;
  cell_run(s, c, &ra, &rb);
  int e = 0;
  bool want = false;
  double x = 0.0, y = 0.0, z = 0.0, q = 0.0, dmax = 0.0;
  if (act) {
    if constexpr (ONE) {
      want = Eone.pp != 0;
      if (want) dmax = __longlong_as_double(C.stats[Eone.st_off + ST_DMAX]);
    } else {
      // the ensemble of the wave's first slot (uniform search), else the lane's own
      const int e0 = find_off(C.p_off, C.n_ens + 1, (long long)__builtin_amdgcn_readfirstlane(s));
      e = s < C.p_off[e0 + 1] ? e0 : find_off(C.p_off, C.n_ens + 1, (long long)s);
      want = C.ens[e].pp != 0;
      if (want) dmax = __longlong_as_double(C.stats[C.ens[e].st_off + ST_DMAX]);
    }
    if (ra < 0) ra = C.start[c];
    if (rb < 0) rb = C.start[c + 1];
    x = in.x[p];
    y = in.y[p];
    z = in.z[p];
    q = in.q[p];
  }
  const int lane = (int)(threadIdx.x & 63u);
  const int s0 = s - lane;
  const int n = want ? rb - ra : 0;
  // is any mate closer than d_max (>= (d + d_max)/2)?
  bool near = false;
  for (int kk = 0; __any(kk < n); ++kk) {
    const int t = ra + kk, src = t - s0;
    double ox = __shfl(x, src & 63, 64), oy = __shfl(y, src & 63, 64), oz = __shfl(z, src & 63, 64);
    if (kk < n && t != s) {
      if (!(src >= 0 && src < 64)) {
        const int pt = C.perm[t];
        ox = in.x[pt];
        oy = in.y[pt];
        oz = in.z[pt];
      }
      const double rx = x - ox, ry = y - oy, rz = z - oz;
      const double r2 = (rx * rx + ry * ry) + rz * rz;
      near |= r2 < dmax * dmax;
    }
  }
  double inc[4] = {0.0, 0.0, 0.0, 0.0};
  int hit = 0, npp = 0;
  if (__any(near)) {
    const int m = near ? n : 0;
    double vx = 0.0, vy = 0.0, vz = 0.0, d = 0.0, rcut2 = 0.0, kpp = 0.0;
    if (near) {
      vx = in.vx[p];
      vy = in.vy[p];
      vz = in.vz[p];
      d = in.d[p];
      const double rc = 0.5 * (d + dmax);
      rcut2 = rc * rc;
      kpp = ONE ? Eone.kpp : C.ens[e].kpp;
    }
    for (int kk = 0; __any(kk < m); ++kk) {
      const int t = ra + kk, src = t - s0;
      double ox = __shfl(x, src & 63, 64), oy = __shfl(y, src & 63, 64), oz = __shfl(z, src & 63, 64);
      double oq = __shfl(q, src & 63, 64);
      const int pv = __shfl(p, src & 63, 64);
      if (kk < m && t != s) {
        int pt = pv;
        if (!(src >= 0 && src < 64)) {
          pt = C.perm[t];
          ox = in.x[pt];
          oy = in.y[pt];
          oz = in.z[pt];
          oq = in.q[pt];
        }
        const double rx = x - ox, ry = y - oy, rz = z - oz;
        const double r2 = (rx * rx + ry * ry) + rz * rz;
        if (r2 < rcut2) {
          const PPHit h = pp_pair(pt, in, kpp, rx, ry, rz, r2, d, vx, vy, vz, q, oq);
          if (h.hit) {
            hit = 1;
            if (t > s) ++npp;
            inc[0] += h.dvx;
            inc[1] += h.dvy;
            inc[2] += h.dvz;
            inc[3] += h.dq;
          }
        }
      }
    }
  }
  if (npp)
    atomicAdd((unsigned long long*)&C.stats[(ONE ? Eone.st_off : C.ens[e].st_off) + ST_PP], (unsigned long long)npp);
  if (!act) return;
  // the increments only where a collision happened (the push reads the flag)
  C.chit[s] = (unsigned char)hit;
  if (hit) {
    const long long nt = C.n_tot;
    C.cinc[s] = inc[0];
    C.cinc[nt + s] = inc[1];
    C.cinc[2 * nt + s] = inc[2];
    C.cinc[3 * nt + s] = inc[3];
  }
}

hipError_t launch_collide(const Ctx& C, const Ens& Eone, const PState& in, hipStream_t st) {
  if (C.n_tot == 0) return hipSuccess;
  const int nb = (int)((C.n_tot + kBlock - 1) / kBlock);
  if (C.n_ens == 1)
    k_collide<true><<<nb, kBlock, 0, st>>>(C, Eone, in);
  else
    k_collide<false><<<nb, kBlock, 0, st>>>(C, Eone, in);
  return hipGetLastError();
}

// the recorded step's sorted keys, cell starts and potential in one launch
// (grid-stride over the longest of the three)
__global__ __launch_bounds__(kBlock) void k_record(int* __restrict__ skey_d, const int* __restrict__ skey,
                                                   long long n, int* __restrict__ start_d,
                                                   const int* __restrict__ start, double* __restrict__ phi_d,
                                                   const double* __restrict__ phi, long long nc) {
  const long long m = n > nc + 1 ? n : nc + 1;
  for (long long t = (long long)blockIdx.x * kBlock + threadIdx.x; t < m; t += (long long)gridDim.x * kBlock) {
    if (t < n) skey_d[t] = skey[t];
    if (t <= nc) start_d[t] = start[t];
    if (t < nc) phi_d[t] = phi[t];
  }
}

hipError_t launch_record(int* skey_d, const int* skey, long long n, int* start_d, const int* start, double* phi_d,
                         const double* phi, long long nc, hipStream_t st) {
  const long long m = n > nc + 1 ? n : nc + 1;
  const int nb = (int)std::min<long long>((m + kBlock - 1) / kBlock, 4096);
  k_record<<<nb, kBlock, 0, st>>>(skey_d, skey, n, start_d, start, phi_d, phi, nc);
  return hipGetLastError();
}

__global__ void k_set_ptr(const double** slot, const double* value) { *slot = value; }

// carrier copy with periodic ghost nodes: rows of nx nodes -> rows of nxp =
// nx + 2 (nodes 0..nx-1, then nodes 0 and 1)
__global__ __launch_bounds__(kBlock) void k_pad_carrier(double* __restrict__ dst, const double* __restrict__ src,
                                                        int nx, int nxp, long long rows) {
  const long long total = rows * nxp;
  for (long long t = (long long)blockIdx.x * kBlock + threadIdx.x; t < total; t += (long long)gridDim.x * kBlock) {
    const long long r = t / nxp;
    const int i = (int)(t - r * nxp);
    dst[t] = src[r * nx + (i < nx ? i : i - nx)];
  }
}

hipError_t launch_set_ptr(const double** slot, const double* value, hipStream_t st) {
  k_set_ptr<<<1, 1, 0, st>>>(slot, value);
  return hipGetLastError();
}

hipError_t launch_pad_carrier(double* dst, const double* src, int nx, int ny, int nz, hipStream_t st) {
  const long long rows = 3LL * (ny + 1) * nz;
  const long long total = rows * (nx + 2);
  const int nb = (int)std::min<long long>((total + kBlock - 1) / kBlock, 8192);
  k_pad_carrier<<<nb, kBlock, 0, st>>>(dst, src, nx, nx + 2, rows);
  return hipGetLastError();
}

hipError_t launch_bin(const Ctx& C, const PState& S, long long n0, long long n1, hipStream_t st) {
  if (n1 <= n0) return hipSuccess;
  const int nb = (int)((n1 - n0 + kBlock - 1) / kBlock);
  k_bin<<<nb, kBlock, 0, st>>>(C, S, n0, n1);
  return hipGetLastError();
}

hipError_t launch_put_state(const PState& S, const double* const* in8, long long p0, int n, hipStream_t st) {
  PIn in{in8[0], in8[1], in8[2], in8[3], in8[4], in8[5], in8[6], in8[7]};
  k_put_state<<<(n + kBlock - 1) / kBlock, kBlock, 0, st>>>(S, in, p0, n);
  return hipGetLastError();
}

hipError_t launch_get_state(const PState& S, double* const* out8, long long p0, int n, hipStream_t st) {
  PIn out{out8[0], out8[1], out8[2], out8[3], out8[4], out8[5], out8[6], out8[7]};
  k_get_state<<<(n + kBlock - 1) / kBlock, kBlock, 0, st>>>(S, out, p0, n);
  return hipGetLastError();
}

}  // namespace tf
