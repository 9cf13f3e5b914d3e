// Host-side launch geometry and kernel launchers (internal).
#pragma once
#include "tribo_dev.h"

namespace tf {

// bump allocator over the caller's workspace (base == nullptr: size only)
struct Carver {
  char* base;
  size_t off = 0;
  explicit Carver(void* b) : base((char*)b) {}
  template <class T>
  T* take(size_t n) {
    off = (off + 255) & ~size_t(255);
    T* p = base ? (T*)(base + off) : nullptr;
    off += n * sizeof(T);
    return p;
  }
};

// Block tables of the cell-structured kernels: blocks of ensemble e are
// [xx_blk[e], xx_blk[e+1]) (host copies) / d_xx_blk (device copies).
struct LaunchGeo {
  int nx_max, nz_max;
  int wz;          // spectral columns per block in the z transforms
  int ny_max;
  int tri_rows;    // rows per lane of the tridiagonal scans (largest over the ensembles)
  int sort_cap;    // members per row pair in LDS for the fused sort (0 auto, -1 none)
  int push_order;  // the push's blocks: 0, 1 consecutive slot ranges per XCD, 2 the hardware's round robin
  int pp_any;      // some ensemble has 4-way coupling on
  int plane_any, half_any, split_any;  // some ensembles with inverse transforms per plane /
                                       // per half plane / by the z and x kernels
  int quarter_any;                     // ... per quarter plane
  int plane_max;   // largest nz (nx/2 + 1) over the ensembles transformed per plane
  int half_lds;    // LDS bytes of the half-plane kernel
  int quarter_lds; // LDS bytes of the quarter-plane kernel
  const int* fp_blk;  // x transforms and the fused sort: kPairsPerBlock row pairs per block
  const int* fz_blk;
  const int* tri_blk;
  const int* d_fp_blk;
  const int* d_fz_blk;
  const int* d_tri_blk;
  const int* pl_blk;  // inverse transforms per plane: one block per y plane
  const int* d_pl_blk;
  const int* ph_blk;  // per half plane: two blocks per y plane
  const int* d_ph_blk;
  const int* pq_blk;  // per quarter plane: four blocks per y plane
  const int* d_pq_blk;
  const int* fps_blk;  // fp_blk / fz_blk restricted to the ensembles whose inverse
  const int* d_fps_blk;  // transforms run as the z then x kernels
  const int* fzs_blk;
  const int* d_fzs_blk;
  const Ens* eh;   // host copies of the ensemble descriptors
};

// full: counting sort from scratch (after init or a state upload); otherwise
// the row scan of the incremental sort, valid when `cur` was written by the
// last push (the sort itself then runs fused with the deposit: launch_sort_dep)
hipError_t launch_sort(const Ctx& C, const LaunchGeo& G, const PState& cur, bool full, hipStream_t st);
hipError_t launch_sort_dep(const Ctx& C, const LaunchGeo& G, const PState& cur, hipStream_t st);
// x_done: the deposit and x transform already ran (launch_sort_dep).
// spec1: a single-ensemble launch (e1 == e0 + 1) keeps that ensemble's
// spectrum at spec1 instead of its place in C.spec.
hipError_t launch_poisson(const Ctx& C, const LaunchGeo& G, int e0, int e1, const double* q, const int* key,
                          const long long* q_in, long long q_shift, double* phi_out, long long phi_shift,
                          int do_stats, hipStream_t st, hipEvent_t* ev = nullptr, const double* r_in = nullptr,
                          bool x_done = false, int* far_reset = nullptr, double2* spec1 = nullptr);
hipError_t launch_push(const Ctx& C, const LaunchGeo& G, const PState& in, const PState& out, int* perm_rec,
                       signed char* wall_rec, hipStream_t st);
// 4-way coupling: per-slot collision increments (before the push)
hipError_t launch_collide(const Ctx& C, const Ens& Eone, const PState& in, hipStream_t st);
// copies of a recorded step's sorted keys [n], cell starts [nc + 1] and phi [nc]
hipError_t launch_record(int* skey_d, const int* skey, long long n, int* start_d, const int* start, double* phi_d,
                         const double* phi, long long nc, hipStream_t st);
// *slot = value, in stream order (a kernel: usable between captured graphs)
hipError_t launch_set_ptr(const double** slot, const double* value, hipStream_t st);
// copy of a carrier field [3][ny+1][nz][nx] with two periodic ghost nodes per
// node row ([3][ny+1][nz][nx+2]), in stream order
hipError_t launch_pad_carrier(double* dst, const double* src, int nx, int ny, int nz, hipStream_t st);
// 2-way coupling source per cell from the push's per-slot drag forces
hipError_t launch_source(const Ctx& C, hipStream_t st);
hipError_t launch_bin(const Ctx& C, const PState& S, long long n0, long long n1, hipStream_t st);
hipError_t launch_put_state(const PState& S, const double* const* in8, long long p0, int n, hipStream_t st);
hipError_t launch_get_state(const PState& S, double* const* out8, long long p0, int n, hipStream_t st);

}  // namespace tf
