// Aggregation multigrid preconditioner for the pressure Poisson system.
//
// The pressure matrix of a long channel with the only Dirichlet rows at the
// outlet has eigenvalues down to ~h^2 / L^2 of its diagonal scale, and
// Jacobi-preconditioned Krylov methods stall or diverge on it at a few
// hundred thousand nodes.  This preconditioner adds the missing coarse-scale
// correction:
//   * aggregates are the occupied cells of a grid of size 2^(l+1) h (2 x 2
//     cells of the level below), so every level keeps the geometry of the
//     node set; rows without off-diagonal entries (phi = 0 outlet rows) stay
//     out of the coarse spaces;
//   * coarse matrices are Galerkin products R A R^T with R the aggregate
//     indicator, summed per coarse row from sorted member lists (fixed order,
//     so the build is deterministic);
//   * the coarsest matrix (bordered when the system is singular) is inverted
//     once by Gauss-Jordan with partial pivoting and applied as a dense product;
//   * one V-cycle with damped Jacobi sweeps before and after the coarse
//     correction (two on every level by default; optionally
//     none before it on the finest level); every stencil pass gathers a single
//     vector; zero start, residual, restriction and prolongation are fused into
//     the neighbouring launches where that pays, and the levels below the finest
//     replay as one captured graph.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <vector>

#include "tile.h"
#include "vip_internal.h"

namespace vip {

namespace {

constexpr double kOmega = 0.7;       // Jacobi damping
constexpr int64_t kCoarseRows = 768;  // stop coarsening at or below this size
constexpr int kMaxCoarseWidth = 128;

__device__ __forceinline__ int64_t slot(const int64_t* ptr, int64_t r, int k) {
  return ptr[r / kSlice] + static_cast<int64_t>(k) * kSlice + (r % kSlice);
}

// keep[i] = 1 if row i has a nonzero off-diagonal entry
__global__ void k_keep(int64_t n, const int64_t* ptr, const int32_t* cols, const int32_t* rowlen,
                       const double* val, int32_t* keep) {
  const int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
  if (i >= n) return;
  int k = 0;
  for (int t = 0; t < rowlen[i]; ++t) {
    const int64_t s = slot(ptr, i, t);
    if (cols[s] != static_cast<int32_t>(i) && val[s] != 0.0) k = 1;
  }
  keep[i] = k;
}

// damped inverse diagonal (identity rows: plain inverse, so one sweep solves them)
__global__ void k_wdinv(int64_t n, const int64_t* ptr, const int32_t* cols, const int32_t* rowlen,
                        const double* val, const int32_t* keep, double omega, double* w64, float* w32) {
  const int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
  if (i >= n) return;
  double d = 0.0;
  for (int t = 0; t < rowlen[i]; ++t) {
    const int64_t s = slot(ptr, i, t);
    if (cols[s] == static_cast<int32_t>(i)) d += val[s];
  }
  const double w = d != 0.0 ? (keep[i] ? omega : 1.0) / d : 0.0;
  w64[i] = w;
  w32[i] = static_cast<float>(w);
}

// level-0 aggregation keys: cell of size 2h
__global__ void k_key0(int64_t n, const double* x, const double* y, double x0, double y0, double cell,
                       int32_t* kx, int32_t* ky) {
  const int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
  if (i >= n) return;
  kx[i] = static_cast<int32_t>(floor((x[i] - x0) / cell));
  ky[i] = static_cast<int32_t>(floor((y[i] - y0) / cell));
}

__global__ void k_mark(int64_t n, const int32_t* keep, const int32_t* kx, const int32_t* ky, int64_t gx,
                       int64_t* occ) {
  const int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
  if (i >= n || !keep[i]) return;
  occ[static_cast<int64_t>(ky[i]) * gx + kx[i]] = 1;
}

__global__ void k_assign(int64_t n, const int32_t* keep, const int32_t* kx, const int32_t* ky, int64_t gx,
                         const int64_t* idx, int32_t* agg, int32_t* ckx, int32_t* cky,
                         unsigned long long* count) {
  const int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
  if (i >= n) return;
  if (!keep[i]) {
    agg[i] = -1;
    return;
  }
  const int64_t a = idx[static_cast<int64_t>(ky[i]) * gx + kx[i]];
  agg[i] = static_cast<int32_t>(a);
  // key of the coarse row for the next aggregation (parent cell); same value from every member
  ckx[a] = kx[i] >> 1;
  cky[a] = ky[i] >> 1;
  atomicAdd(&count[a], 1ull);
}

__global__ void k_members(int64_t n, const int32_t* agg, const int64_t* mstart, unsigned long long* cursor,
                          int32_t* members) {
  const int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
  if (i >= n || agg[i] < 0) return;
  const unsigned long long k = atomicAdd(&cursor[agg[i]], 1ull);
  members[mstart[agg[i]] + static_cast<int64_t>(k)] = static_cast<int32_t>(i);
}

// sort each member list by row index (fixed summation order)
__global__ void k_sort_members(int64_t nc, const int64_t* mstart, int32_t* members) {
  const int64_t a = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
  if (a >= nc) return;
  for (int64_t p = mstart[a] + 1; p < mstart[a + 1]; ++p) {
    const int32_t v = members[p];
    int64_t q = p;
    while (q > mstart[a] && members[q - 1] > v) {
      members[q] = members[q - 1];
      --q;
    }
    members[q] = v;
  }
}

// Galerkin row I of R A R^T: count (fill == 0) or write (fill == 1) its sorted entries.
__global__ void k_galerkin(int64_t nc, const int64_t* mstart, const int32_t* members, const int64_t* ptr,
                           const int32_t* cols, const int32_t* rowlen, const double* val, const int32_t* agg,
                           int fill, int32_t* crowlen, const int64_t* cptr, int32_t* ccols, double* cval,
                           unsigned long long* overflow) {
  const int64_t I = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
  if (I >= nc) return;
  int32_t J[kMaxCoarseWidth];
  double V[kMaxCoarseWidth];
  int cnt = 0;
  bool over = false;
  for (int64_t m = mstart[I]; m < mstart[I + 1]; ++m) {
    const int64_t i = members[m];
    for (int t = 0; t < rowlen[i]; ++t) {
      const int64_t s = slot(ptr, i, t);
      const int32_t a = agg[cols[s]];
      if (a < 0) continue;
      int q = 0;
      while (q < cnt && J[q] != a) ++q;
      if (q == cnt) {
        if (cnt == kMaxCoarseWidth) {
          over = true;
          continue;
        }
        J[cnt] = a;
        V[cnt] = 0.0;
        ++cnt;
      }
      V[q] += val[s];
    }
  }
  if (over) atomicMin(overflow, static_cast<unsigned long long>(I));
  if (!fill) {
    crowlen[I] = cnt;
    return;
  }
  // insertion sort by column
  for (int p = 1; p < cnt; ++p) {
    const int32_t jv = J[p];
    const double vv = V[p];
    int q = p;
    while (q > 0 && J[q - 1] > jv) {
      J[q] = J[q - 1];
      V[q] = V[q - 1];
      --q;
    }
    J[q] = jv;
    V[q] = vv;
  }
  for (int p = 0; p < cnt; ++p) {
    const int64_t s = slot(cptr, I, p);
    ccols[s] = J[p];
    cval[s] = V[p];
  }
}

// ---- coarsest level: dense Gauss-Jordan inverse -------------------------------------------------

__global__ void k_dense_fill(int64_t m, int border, const int64_t* ptr, const int32_t* cols,
                             const int32_t* rowlen, const double* val, double* D, double* Inv) {
  const int64_t m1 = m + border;
  const int64_t e = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
  if (e >= m1 * m1) return;
  const int64_t i = e / m1, j = e % m1;
  Inv[e] = i == j ? 1.0 : 0.0;
  double v = 0.0;
  if (i < m && j < m) {
    for (int t = 0; t < rowlen[i]; ++t) {
      const int64_t s = slot(ptr, i, t);
      if (cols[s] == static_cast<int32_t>(j)) v += val[s];
    }
  } else if (i != j) {
    v = 1.0;   // border row and column
  }
  D[e] = v;
}

// pivot search and row swap for column k (one block)
__global__ void k_gj_pivot(int64_t m1, int64_t k, double* D, double* Inv, double* col, int* bad) {
  __shared__ double best[256];
  __shared__ int64_t arg[256];
  double b = -1.0;
  int64_t a = k;
  for (int64_t i = k + threadIdx.x; i < m1; i += blockDim.x) {
    const double v = fabs(D[i * m1 + k]);
    if (v > b) {
      b = v;
      a = i;
    }
  }
  best[threadIdx.x] = b;
  arg[threadIdx.x] = a;
  __syncthreads();
  for (int off = blockDim.x / 2; off > 0; off >>= 1) {
    if (static_cast<int>(threadIdx.x) < off) {
      const double o = best[threadIdx.x + off];
      const int64_t oa = arg[threadIdx.x + off];
      if (o > best[threadIdx.x] || (o == best[threadIdx.x] && oa < arg[threadIdx.x])) {
        best[threadIdx.x] = o;
        arg[threadIdx.x] = oa;
      }
    }
    __syncthreads();
  }
  const int64_t p = arg[0];
  if (threadIdx.x == 0 && !(best[0] > 0.0)) *bad = 1;
  if (p != k) {
    for (int64_t j = threadIdx.x; j < m1; j += blockDim.x) {
      double t = D[k * m1 + j];
      D[k * m1 + j] = D[p * m1 + j];
      D[p * m1 + j] = t;
      t = Inv[k * m1 + j];
      Inv[k * m1 + j] = Inv[p * m1 + j];
      Inv[p * m1 + j] = t;
    }
  }
  __syncthreads();
  for (int64_t i = threadIdx.x; i < m1; i += blockDim.x) col[i] = D[i * m1 + k];
}

// eliminate column k from every row but k, then (separately) scale row k
__global__ void k_gj_elim(int64_t m1, int64_t k, double* D, double* Inv, const double* col) {
  const int64_t e = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
  if (e >= m1 * m1) return;
  const int64_t i = e / m1, j = e % m1;
  if (i == k) return;
  const double f = col[i] / col[k];
  if (f == 0.0) return;
  D[e] -= f * D[k * m1 + j];
  Inv[e] -= f * Inv[k * m1 + j];
}

__global__ void k_gj_scale(int64_t m1, int64_t k, double* D, double* Inv, const double* col) {
  const int64_t j = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
  if (j >= m1) return;
  const double p = col[k];
  D[k * m1 + j] /= p;
  Inv[k * m1 + j] /= p;
}

__global__ void k_to32(int64_t m, const double* a, float* b) {
  const int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
  if (i < m) b[i] = static_cast<float>(a[i]);
}

// ---- V-cycle kernels ----------------------------------------------------------------------------

template <typename T>
struct LevelView {
  int64_t n;
  const int64_t* ptr;
  const int32_t* cols;
  const int16_t* dcols;   // row-relative columns (Ell::dcols), or null
  const uint8_t* dfit;    // per slice: 1 where dcols holds the slice's columns
  const T* val;
  const T* wdinv;
  const float* rsum;   // FP32 levels: row sums for the difference form
  // lattice-interior rows of level 0 (stencil.hip): pixel of a canonical row, else -1
  const int32_t* cpix;
  const int32_t* sbase;   // slice descriptors of those rows, or null
  const int32_t* node_of;
  int K;
  int disk;
  int box;                // taps are the 3 x 3 box (first coarse level)
  int32_t W;
  int32_t off[kMaxTaps];
  T w[kMaxTaps];
  T wdinv_c;
  float crsum;
  TileView tv;            // level 0: tile partition of the canonical rows (tile.h), if any
  int wd_uniform;         // 1: every tile row's damped inverse diagonal is wdinv_c
};

// a * b + c with one rounding, written out so that every path that must give the same bits
// (canonical and general rows, tile and row sweeps) rounds alike whatever the compiler fuses
template <typename T>
__device__ __forceinline__ T fmadd(T a, T b, T c) {
  if constexpr (sizeof(T) == 4) return fmaf(a, b, c);
  else return fma(a, b, c);
}

// Canonical row of a level: weights of the reference row, columns from the lattice map,
// slots to the accumulators in the general path's order (same bits).
template <typename T, class Tap>
__device__ __forceinline__ T disk_taps(const LevelView<T>& L, Tap&& tap) {
  const T yi = (sizeof(T) == 4) ? tap(2, 0) : T(0);
  T a0 = T(0), a1 = T(0);
#pragma unroll
  for (int k = 0; k < kDiskTaps; ++k) {
    const T d = tap(disk_row(k), disk_dx(k)) - yi;
    if (k & 1) a1 = fmadd(L.w[k], d, a1);
    else a0 = fmadd(L.w[k], d, a0);
  }
  if constexpr (sizeof(T) == 4) return fmadd(static_cast<T>(L.crsum), yi, a0 + a1);
  else return a0 + a1;
}

template <typename T, class Y>
__device__ __forceinline__ T disk_row_sum(const LevelView<T>& L, int64_t i, const int32_t (&b)[5], Y y) {
  (void)i;
  return disk_taps(L, [&](int r, int dx) __attribute__((always_inline)) { return y(b[r] + dx); });
}

// The 3 x 3 box row (first coarse level) with tap (r, dx) the value dx columns off in stencil
// row r (1..3, the row's own is 2): with 9 slots the general path sends slot k to accumulator
// k % 2 whatever the slice width.  Shared by the lattice-map and the LDS tile paths.
template <typename T, class Tap>
__device__ __forceinline__ T box_taps(const LevelView<T>& L, Tap&& tap) {
  const T yi = (sizeof(T) == 4) ? tap(2, 0) : T(0);
  T a0 = T(0), a1 = T(0);
#pragma unroll
  for (int k = 0; k < 9; ++k) {
    const T d = tap(k / 3 + 1, k % 3 - 1) - yi;
    if (k & 1) a1 = fmadd(L.w[k], d, a1);
    else a0 = fmadd(L.w[k], d, a0);
  }
  if constexpr (sizeof(T) == 4) return fmadd(static_cast<T>(L.crsum), yi, a0 + a1);
  else return a0 + a1;
}

// Stencil row of a tile row from the LDS copy: the disk (finest level) or the box (first
// coarse level).
template <typename T, class Tap>
__device__ __forceinline__ T lds_taps(const LevelView<T>& L, Tap&& tap) {
  if (L.box) return box_taps(L, tap);
  return disk_taps(L, tap);
}

// Canonical row of a level: weights of the reference row, columns from the lattice map,
// slots to the accumulators in the general path's order (same bits).
template <typename T, class Y>
__device__ __forceinline__ T canon_row(const LevelView<T>& L, int32_t p, int64_t i, int w, Y y) {
  if (L.disk) {
    int32_t b[5];
    disk_bases(L.node_of, p, L.W, i, b);
    return disk_row_sum(L, i, b, y);
  }
  if (L.box) {
    // 3 x 3 box: row bases from two lattice-map reads
    const int32_t b[3] = {L.node_of[p - L.W], static_cast<int32_t>(i), L.node_of[p + L.W]};
    return box_taps(L, [&](int r, int dx) __attribute__((always_inline)) { return y(b[r - 1] + dx); });
  }
  const T yi = (sizeof(T) == 4) ? y(static_cast<int32_t>(i)) : T(0);
  T a0 = T(0), a1 = T(0);
  const int full = w & ~3;
  const int32_t* nb = L.node_of + p;
  int k = 0;
  for (; k + 4 <= L.K && k + 4 <= full; k += 4) {
    const T y0 = y(nb[L.off[k]]), y1 = y(nb[L.off[k + 1]]), y2 = y(nb[L.off[k + 2]]), y3 = y(nb[L.off[k + 3]]);
    a0 = fmadd(L.w[k], y0 - yi, a0);
    a1 = fmadd(L.w[k + 1], y1 - yi, a1);
    a0 = fmadd(L.w[k + 2], y2 - yi, a0);
    a1 = fmadd(L.w[k + 3], y3 - yi, a1);
  }
  for (; k < L.K; ++k) {
    const T d = y(nb[L.off[k]]) - yi;
    if (k < full && (k & 1)) a1 = fmadd(L.w[k], d, a1);
    else a0 = fmadd(L.w[k], d, a0);
  }
  if constexpr (sizeof(T) == 4) return fmadd(static_cast<T>(L.crsum), yi, a0 + a1);
  else return a0 + a1;
}

template <typename T>
__device__ __forceinline__ T level_wdinv(const LevelView<T>& L, int64_t i) {
  if (L.sbase) {
    const int32_t sl = __builtin_amdgcn_readfirstlane(static_cast<int32_t>(i >> 6));
    if ((i >> 6) == sl && L.sbase[4 * static_cast<int64_t>(sl)] >= 0) return L.wdinv_c;
  }
  return (L.cpix && L.cpix[i] >= 0) ? L.wdinv_c : L.wdinv[i];
}

// cpix_out[i] = cpix_in[i] where the damped inverse diagonal also equals the reference bits
template <typename T>
__global__ void k_canon_wd(int64_t n, const int32_t* cin, const T* wd, T ref, int32_t* cout, int* dropped) {
  const int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
  if (i >= n) return;
  int32_t p = cin[i];
  if (p >= 0) {
    bool same;
    if constexpr (sizeof(T) == 4) same = __float_as_uint(wd[i]) == __float_as_uint(ref);
    else same = __double_as_longlong(wd[i]) == __double_as_longlong(ref);
    if (!same) {
      p = -1;
      *dropped = 1;   // every writer stores the same value
    }
  }
  cout[i] = p;
}

// (A y)_i with y_j given by a functor; FP32 levels use the difference form
// rsum_i y_i + sum a_ij (y_j - y_i) (rows sum to ~0, see row_dot in the solver).
template <typename T, class Y>
__device__ __forceinline__ T level_row(const LevelView<T>& L, int64_t i, Y y) {
  const int64_t sl = i / kSlice;
  const int64_t base = L.ptr[sl] + (i % kSlice);
  const int w = static_cast<int>((L.ptr[sl + 1] - L.ptr[sl]) / kSlice);
  if (L.sbase) {
    int32_t b[5];
    if (slice_disk_bases(L.sbase, i, b)) return disk_row_sum(L, i, b, y);
  }
  if (L.cpix) {
    const int32_t p = L.cpix[i];
    if (p >= 0) return canon_row(L, p, i, w, y);
  }
  const T yi = (sizeof(T) == 4) ? y(static_cast<int32_t>(i)) : T(0);
  // the slot loop once per column stream, so that each instance issues loads of one kind only
  auto sum = [&](auto col) __attribute__((always_inline)) -> T {
    T a0 = T(0), a1 = T(0);
    int k = 0;
    for (; k + 4 <= w; k += 4) {
      const int64_t q = base + static_cast<int64_t>(k) * kSlice;
      const int32_t c0 = col(q), c1 = col(q + kSlice), c2 = col(q + 2 * kSlice), c3 = col(q + 3 * kSlice);
      const T v0 = L.val[q], v1 = L.val[q + kSlice], v2 = L.val[q + 2 * kSlice], v3 = L.val[q + 3 * kSlice];
      const T y0 = y(c0), y1 = y(c1), y2 = y(c2), y3 = y(c3);
      a0 = fmadd(v0, y0 - yi, a0);
      a1 = fmadd(v1, y1 - yi, a1);
      a0 = fmadd(v2, y2 - yi, a0);
      a1 = fmadd(v3, y3 - yi, a1);
    }
    for (; k < w; ++k) {
      const int64_t q = base + static_cast<int64_t>(k) * kSlice;
      a0 = fmadd(L.val[q], y(col(q)) - yi, a0);
    }
    if constexpr (sizeof(T) == 4) return fmadd(static_cast<T>(L.rsum[i]), yi, a0 + a1);
    else return a0 + a1;
  };
  if (L.dcols && L.dfit[sl]) {
    const int32_t ii = static_cast<int32_t>(i);
    return sum([&](int64_t q) __attribute__((always_inline)) { return ii + static_cast<int32_t>(L.dcols[q]); });
  }
  return sum([&](int64_t q) __attribute__((always_inline)) { return L.cols[q]; });
}

// W b at row j, as a rounded product: without contraction, so that no fused multiply-add
// folds it into the arithmetic of a sweep that recomputes it
template <typename T>
__device__ __forceinline__ T zero_start_value(const T* wdinv, const T* b, int64_t j) {
#pragma clang fp contract(off)
  return wdinv[j] * b[j];
}

// x = W b   (damped Jacobi sweep from a zero start)
template <typename T>
__global__ void k_jacobi0(LevelView<T> L, const T* b, T* x, const int* on) {
  if (!*on) return;
  const int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
  if (i < L.n) x[i] = zero_start_value(L.wdinv, b, i);
}

// The FP32 tile kernels of a level (residual, sweeps of kind 0 and 1) are asked for 8 waves
// per SIMD: under the bound they fit in 57-59 vector registers, and the scalar registers are
// kept to that count (the excess scalars live in vector-register lanes, no scratch).  The
// FP64 and kind-2 instances would spill to scratch under it.
// r = b - A x
template <typename T>
__global__ void __launch_bounds__(kBlock, (sizeof(T) == 4 ? 8 : 1)) k_level_residual(LevelView<T> L, const T* b, const T* x, T* r, const int* on) {
  __shared__ T lds[1][kTileLdsH][kTileLdsW];
  __shared__ TileMeta meta;
  if (!*on) return;
  if (L.tv.tiles) {
    const T* xs[1] = {x};
    tile_walk(
        L.tv,
        [&](int64_t tk) __attribute__((always_inline)) {
          tile_stage<T, 1>(L.tv, tk, xs, lds, meta, true);
          const int wave = static_cast<int>(threadIdx.x >> 6), lane = static_cast<int>(threadIdx.x & 63);
#pragma unroll 1
          for (int k = 0; k < kTileRowsPerWave; ++k) {
            const int64_t row = tile_row_id(L.tv, meta, k);
            if (row < 0) continue;
            const int ly = wave + k * (kBlock / 64);
            const T bi = b[row];
            r[row] = bi - lds_taps(L, [&](int rr, int dx) __attribute__((always_inline)) { return lds[0][ly + rr][lane + 2 + dx]; });
          }
        },
        [&](int64_t i) __attribute__((always_inline)) { r[i] = b[i] - level_row(L, i, [&](int32_t j) __attribute__((always_inline)) { return x[j]; }); });
    return;
  }
  const int64_t lb = xcd_block(blockIdx.x, gridDim.x);
  const int64_t i = lb * blockDim.x + threadIdx.x;
  if (i >= L.n) return;
  r[i] = b[i] - level_row(L, i, [&](int32_t j) __attribute__((always_inline)) { return x[j]; });
}

// bc[I] = sum of r over the members of aggregate I
template <typename T>
__global__ void k_restrict(int64_t nc, const int64_t* mstart, const int32_t* members, const T* r, T* bc,
                           const int* on) {
  if (!*on) return;
  const int64_t I = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
  if (I >= nc) return;
  T s = T(0);
  for (int64_t m = mstart[I]; m < mstart[I + 1]; ++m) s += r[members[m]];
  bc[I] = s;
}

// bc[I] = sum over the members i of aggregate I of (b - A x)_i: the residual and the restriction
// in one launch, for coarse levels where launches cost more than the work.  Each member's
// residual is the expression k_level_residual stores, summed in k_restrict's order.  Four
// lanes per aggregate compute its first four members' residuals side by side (the first lane
// takes any further members itself); grid: 4 nc threads.
template <typename T>
__global__ void k_restrict_residual(LevelView<T> L, int64_t nc, const int64_t* mstart, const int32_t* members,
                                    const T* b, const T* x, T* bc, const int* on) {
  if (!*on) return;
  const int64_t t = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
  const int64_t I = t >> 2;
  const int k = static_cast<int>(t & 3);
  const bool valid = I < nc;
  const int64_t m0 = valid ? mstart[I] : 0, m1 = valid ? mstart[I + 1] : 0;
  auto res = [&](int64_t m) __attribute__((always_inline)) {
    const int32_t i = members[m];
    return b[i] - level_row(L, i, [&](int32_t j) __attribute__((always_inline)) { return x[j]; });
  };
  const T r = (m0 + k < m1) ? res(m0 + k) : T(0);
  // the group's four lanes are consecutive lanes of one wavefront (4 divides 64)
  const T r1 = __shfl(r, 1, 4), r2 = __shfl(r, 2, 4), r3 = __shfl(r, 3, 4);
  if (!valid || k != 0) return;
  const int64_t cnt = m1 - m0;
  T s = T(0);
  if (cnt > 0) s += r;
  if (cnt > 1) s += r1;
  if (cnt > 2) s += r2;
  if (cnt > 3) s += r3;
  for (int64_t m = m0 + 4; m < m1; ++m) s += res(m);
  bc[I] = s;
}

// (x + gamma P xc)_j, the corrected iterate at row j (x may be absent: zero pre-smoothing)
template <typename T>
__device__ __forceinline__ T prolong_value(const T* x, const int32_t* agg, const T* xc, T gamma, int64_t j) {
  const int32_t a = agg[j];
  const T base = x ? x[j] : T(0);
  return a >= 0 ? fmadd(gamma, xc[a], base) : base;
}

// y = x + gamma P xc   (coarse correction)
template <typename T>
__global__ void k_prolong(int64_t n, const int32_t* agg, const T* xc, T gamma, const T* x, T* y,
                          const int* on) {
  if (!*on) return;
  const int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
  if (i >= n) return;
  y[i] = prolong_value(x, agg, xc, gamma, i);
}

// The iterate a smoothing sweep starts from: y in memory (kind 0), the zero-start sweep's W b
// (kind 1, the output of k_jacobi0) or the coarse-corrected iterate x + gamma P xc (kind 2, the
// output of k_prolong), recomputed wherever it is needed with the same arithmetic as the launch
// it replaces, so the fused sweep gives the same bits as the two launches.
template <typename T>
struct SweepIn {
  const T* y;              // kind 0
  const T* b;              // kind 1
  const T* x;              // kind 2: pre-smoothed iterate, coarse correction, aggregate map
  const T* xc;
  const int32_t* agg;
  T gamma;
};

template <typename T, int KIND>
__device__ __forceinline__ T sweep_in(const LevelView<T>& L, const SweepIn<T>& in, int64_t j) {
  if constexpr (KIND == 0) return in.y[j];
  else if constexpr (KIND == 1) return zero_start_value(L.wdinv, in.b, j);
  else return prolong_value(in.x, in.agg, in.xc, in.gamma, j);
}

// out = y + W (b - A y)   (damped Jacobi sweep from the iterate of kind KIND)
template <typename T, int KIND>
__global__ void __launch_bounds__(kBlock, (sizeof(T) == 4 && KIND != 2 ? 8 : 1)) k_sweep(LevelView<T> L, const T* b, SweepIn<T> in, T* out,
                                                  const int* on) {
  __shared__ T lds[1][kTileLdsH][kTileLdsW];
  __shared__ TileMeta meta;
  if (!*on) return;
  auto yf = [&](int64_t j) __attribute__((always_inline)) { return sweep_in<T, KIND>(L, in, j); };
  if (L.tv.tiles) {
    // tile rows: the damped inverse diagonal is the reference one when every canonical row's
    // equals it (checked at setup), else read from memory; the same bits either way.  The
    // zero-start sweep (kind 1) always reads it: the choice cost it registers and time
    // (41.1 -> 43.5 us on the finest level), where the kind-0 sweep gained (31.8 -> 29.9 us)
    tile_walk(
        L.tv,
        [&](int64_t tk) __attribute__((always_inline)) {
          tile_stage_fn<T, 1>(
              L.tv, tk, [&](int, int32_t node) __attribute__((always_inline)) { return yf(node); }, lds, meta,
              true);
          const int wave = static_cast<int>(threadIdx.x >> 6), lane = static_cast<int>(threadIdx.x & 63);
#pragma unroll 1
          for (int k = 0; k < kTileRowsPerWave; ++k) {
            const int64_t row = tile_row_id(L.tv, meta, k);
            if (row < 0) continue;
            const int ly = wave + k * (kBlock / 64);
            const T bi = b[row], wd = (KIND != 1 && L.wd_uniform) ? L.wdinv_c : L.wdinv[row];
            const T ay = lds_taps(L, [&](int rr, int dx) __attribute__((always_inline)) { return lds[0][ly + rr][lane + 2 + dx]; });
            out[row] = fmadd(wd, bi - ay, lds[0][ly + 2][lane + 2]);
          }
        },
        [&](int64_t i) __attribute__((always_inline)) {
          const T ay = level_row(L, i, [&](int32_t j) __attribute__((always_inline)) { return yf(j); });
          out[i] = fmadd(level_wdinv(L, i), b[i] - ay, yf(i));
        });
    return;
  }
  const int64_t lb = xcd_block(blockIdx.x, gridDim.x);
  const int64_t i = lb * blockDim.x + threadIdx.x;
  if (i >= L.n) return;
  const T ay = level_row(L, i, [&](int32_t j) __attribute__((always_inline)) { return yf(j); });
  out[i] = fmadd(level_wdinv(L, i), b[i] - ay, yf(i));
}

// x[0..rows) = Inv[0..rows, 0..cols) b on the coarsest level (one wavefront per row);
// rows = cols = m applies the block that leaves out the border, rows = cols = m1
// the whole bordered inverse.
template <typename T>
__global__ void k_dense_apply(int64_t rows, int64_t cols, int64_t ld, const T* Inv, const T* b, T* x,
                              const int* on) {
  if (!*on) return;
  const int64_t row = (blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x) / 64;
  const int lane = threadIdx.x & 63;
  if (row >= rows) return;
  double acc = 0.0;
  for (int64_t j = lane; j < cols; j += 64) acc += static_cast<double>(Inv[row * ld + j]) * static_cast<double>(b[j]);
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
  if (lane == 0) x[row] = static_cast<T>(acc);
}

}  // namespace

namespace {

// lattice image of the next level's rows: the row of each occupied aggregation cell
__global__ void k_cell_map(int64_t ncell, const int64_t* occ, const int64_t* idx, int32_t* cell_node,
                           int32_t* cell_pix) {
  const int64_t q = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
  if (q >= ncell) return;
  if (occ[q]) {
    cell_node[q] = static_cast<int32_t>(idx[q]);
    cell_pix[idx[q]] = static_cast<int32_t>(q);
  } else {
    cell_node[q] = -1;
  }
}

}  // namespace

void amg_free(Ctx* c) {
  Amg& g = c->amg;
  for (int k = 0; k < 2; ++k) {
    if (g.coarse_exec[k]) (void)hipGraphExecDestroy(g.coarse_exec[k]);
    g.coarse_exec[k] = nullptr;
    g.coarse_out[k] = nullptr;
  }
  if (g.cap_stream) (void)hipStreamDestroy(g.cap_stream);
  g.cap_stream = nullptr;
  for (size_t l = 0; l < g.lv.size(); ++l) {
    AmgLevel& L = g.lv[l];
    if (l > 0) ell_free(L.A);
    dfree(L.wdinv);
    dfree(L.wdinv32);
    dfree(L.agg);
    dfree(L.keep);
    dfree(L.kx);
    dfree(L.ky);
    dfree(L.mstart);
    dfree(L.members);
    dfree(L.cpix64);
    dfree(L.cpix32);
    dfree(L.sbase64);
    dfree(L.sbase32);
    dfree(L.cell_node);
    dfree(L.cell_pix);
    tile_part_free(L.tpart32);
    tile_part_free(L.tpart64);
    L.tiles_filtered = false;
    tile_map_free(L.tmap);
    for (int k = 0; k < 3; ++k) {
      dfree(L.w64[k]);
      dfree(L.w32[k]);
    }
  }
  g.lv.clear();
  dfree(g.cinv);
  dfree(g.cinv32);
  g.ready = false;
}

int amg_setup(Ctx* c) {
  amg_free(c);
  Amg& g = c->amg;
  hipStream_t st = c->stream;
  unsigned long long* flag = nullptr;
  VIP_TRY(dalloc(c, &flag, 1));
  int rc = VIP_OK;
  // level 0 is the pressure matrix itself
  g.lv.emplace_back();
  {
    AmgLevel& L0 = g.lv[0];
    L0.n = c->n;
    L0.A = c->sys;   // shallow view, not owned
    L0.vs = 0;
    VIP_TRY(dalloc(c, &L0.kx, c->n));
    VIP_TRY(dalloc(c, &L0.ky, c->n));
    k_key0<<<grid_for(c->n), kBlock, 0, st>>>(c->n, c->x, c->y, c->xmin, c->ymin, 2.0 * c->h,
                                               L0.kx, L0.ky);
  }
  for (int level = 0; level < 24; ++level) {
    AmgLevel& L = g.lv[level];
    const Ell& A = L.A;
    const double* aval = A.val[L.vs];
    VIP_TRY(dalloc(c, &L.keep, L.n));
    VIP_TRY(dalloc(c, &L.wdinv, L.n));
    VIP_TRY(dalloc(c, &L.wdinv32, L.n));
    k_keep<<<grid_for(L.n), kBlock, 0, st>>>(L.n, A.ptr, A.cols, A.rowlen, aval, L.keep);
    k_wdinv<<<grid_for(L.n), kBlock, 0, st>>>(L.n, A.ptr, A.cols, A.rowlen, aval, L.keep, kOmega,
                                               L.wdinv, L.wdinv32);
    if (level == 1 && !c->no_canon && L.cell_node) {
      // canonical rows of the first coarse level on the lattice of aggregation cells
      const LatRef lat{L.W, L.H, L.cell_pix, L.cell_node, L.n, nullptr};
      VIP_TRY(canon_mark_on(c, L.A, 0, lat));
      VIP_TRY(canon_mark_on(c, L.A, 4, lat));
    }
    if (level <= 1 && !c->no_canon && A.canon.K > 0 && A.canon.ref_row >= 0) {
      // canonical rows of the sweeps: canonical matrix row and the reference damped diagonal
      const Canon& cn = A.canon;
      if (level == 0) {
        L.node_of = c->lat.node_of;
        L.W = c->lat.W;
      } else {
        L.node_of = L.cell_node;
      }
      const int64_t r64 = cn.vref[0] >= 0 ? cn.vref[0] : cn.ref_row;
      const int64_t r32 = cn.vref[4] >= 0 ? cn.vref[4] : cn.ref_row;
      VIP_HIP_TRY(c, hipMemcpyAsync(&L.wdinv_c, L.wdinv + r64, sizeof(double), hipMemcpyDeviceToHost, st));
      VIP_HIP_TRY(c, hipMemcpyAsync(&L.wdinv32_c, L.wdinv32 + r32, sizeof(float), hipMemcpyDeviceToHost, st));
      VIP_HIP_TRY(c, hipStreamSynchronize(st));
      int* dropped = nullptr;
      VIP_TRY(dalloc(c, &dropped, 2));
      VIP_HIP_TRY(c, hipMemsetAsync(dropped, 0, 2 * sizeof(int), st));
      if (cn.count[0] > 0 && cn.cpix[0]) {
        VIP_TRY(dalloc(c, &L.cpix64, L.n));
        k_canon_wd<double><<<grid_for(L.n), kBlock, 0, st>>>(L.n, cn.cpix[0], L.wdinv, L.wdinv_c, L.cpix64,
                                                              dropped);
        if (cn.disk && level == 0) VIP_TRY(slice_bases(c, L.cpix64, L.n, &L.sbase64));
      }
      if (cn.count[4] > 0 && cn.cpix[4]) {
        VIP_TRY(dalloc(c, &L.cpix32, L.n));
        k_canon_wd<float><<<grid_for(L.n), kBlock, 0, st>>>(L.n, cn.cpix[4], L.wdinv32, L.wdinv32_c, L.cpix32,
                                                             dropped + 1);
        if (cn.disk && level == 0) VIP_TRY(slice_bases(c, L.cpix32, L.n, &L.sbase32));
      }
      VIP_HIP_TRY(c, hipGetLastError());
      int hd[2] = {1, 1};
      const hipError_t e1 = hipMemcpyAsync(hd, dropped, sizeof(hd), hipMemcpyDeviceToHost, st);
      const hipError_t e2 = hipStreamSynchronize(st);
      dfree(dropped);
      if (e1 != hipSuccess || e2 != hipSuccess) return set_error(c, VIP_E_HIP, "checking the damped diagonals");
      L.wd_uniform64 = cn.count[0] > 0 && cn.cpix[0] && hd[0] == 0;
      L.wd_uniform32 = cn.count[4] > 0 && cn.cpix[4] && hd[1] == 0;
      if (level == 1 && cn.box && L.cell_node) {
        // tiles of the box rows on the cell lattice, from the filtered canonical sets: the tile
        // sweeps then take the reference damped diagonal for every tile row
        VIP_TRY(tile_part_build(c, L.W, L.H, L.cell_node, L.n, L.tmap, L.cpix32, nullptr, L.tpart32));
        VIP_TRY(tile_part_build(c, L.W, L.H, L.cell_node, L.n, L.tmap, L.cpix64, nullptr, L.tpart64));
        L.tiles_filtered = true;
        if (c->debug)
          std::fprintf(stderr, "[vip] level 1 tiles: %lld (FP32 rows), %lld (FP64 rows); irregular %lld, %lld of %lld\n",
                       static_cast<long long>(L.tpart32.ntiles), static_cast<long long>(L.tpart64.ntiles),
                       static_cast<long long>(L.tpart32.nirr), static_cast<long long>(L.tpart64.nirr),
                       static_cast<long long>(L.n));
      }
    }
    for (int k = 0; k < 3; ++k) {
      VIP_TRY(dalloc(c, &L.w64[k], L.n + 1));
      VIP_TRY(dalloc(c, &L.w32[k], L.n + 1));
    }
    if (L.n <= kCoarseRows) break;
    // grid of aggregation keys
    std::vector<int32_t> hx(L.n), hy(L.n);
    VIP_HIP_TRY(c, hipMemcpyAsync(hx.data(), L.kx, sizeof(int32_t) * L.n, hipMemcpyDeviceToHost, st));
    VIP_HIP_TRY(c, hipMemcpyAsync(hy.data(), L.ky, sizeof(int32_t) * L.n, hipMemcpyDeviceToHost, st));
    VIP_HIP_TRY(c, hipStreamSynchronize(st));
    int32_t mx = 0, my = 0, lx = 0, ly = 0;
    for (int64_t i = 0; i < L.n; ++i) {
      mx = std::max(mx, hx[i]);
      my = std::max(my, hy[i]);
      lx = std::min(lx, hx[i]);
      ly = std::min(ly, hy[i]);
    }
    if (lx < 0 || ly < 0) {
      rc = set_error(c, VIP_E_INVALID, "multigrid aggregation keys below the grid origin");
      break;
    }
    const int64_t gx = static_cast<int64_t>(mx) + 1, gy = static_cast<int64_t>(my) + 1;
    int64_t *occ = nullptr, *idx = nullptr;
    VIP_TRY(dalloc(c, &occ, gx * gy));
    VIP_TRY(dalloc(c, &idx, gx * gy + 1));
    VIP_HIP_TRY(c, hipMemsetAsync(occ, 0, sizeof(int64_t) * gx * gy, st));
    k_mark<<<grid_for(L.n), kBlock, 0, st>>>(L.n, L.keep, L.kx, L.ky, gx, occ);
    int64_t nc = 0;
    rc = scan_i64(c, occ, idx, gx * gy, &nc);
    if (rc != VIP_OK) break;
    if (nc == 0 || nc * 10 > L.n * 9) {   // no useful coarsening left
      dfree(occ);
      dfree(idx);
      break;
    }
    VIP_TRY(dalloc(c, &L.agg, L.n));
    AmgLevel C;
    C.n = nc;
    VIP_TRY(dalloc(c, &C.kx, nc));
    VIP_TRY(dalloc(c, &C.ky, nc));
    unsigned long long* cnt = nullptr;
    VIP_TRY(dalloc(c, &cnt, nc + 1));
    VIP_HIP_TRY(c, hipMemsetAsync(cnt, 0, sizeof(unsigned long long) * (nc + 1), st));
    k_assign<<<grid_for(L.n), kBlock, 0, st>>>(L.n, L.keep, L.kx, L.ky, gx, idx, L.agg, C.kx, C.ky, cnt);
    if (level == 0 && gx * gy <= 4 * nc + 4096 && gx <= 65536 && gy <= 65536) {
      C.W = static_cast<int32_t>(gx);
      C.H = static_cast<int32_t>(gy);
      VIP_TRY(dalloc(c, &C.cell_node, gx * gy));
      VIP_TRY(dalloc(c, &C.cell_pix, nc));
      k_cell_map<<<grid_for(gx * gy), kBlock, 0, st>>>(gx * gy, occ, idx, C.cell_node, C.cell_pix);
    }
    dfree(occ);
    dfree(idx);
    VIP_TRY(dalloc(c, &L.mstart, nc + 1));
    int64_t nm = 0;
    rc = scan_i64(c, reinterpret_cast<const int64_t*>(cnt), L.mstart, nc, &nm);
    if (rc != VIP_OK) break;
    VIP_HIP_TRY(c, hipMemcpyAsync(L.mstart + nc, &nm, sizeof(int64_t), hipMemcpyHostToDevice, st));
    VIP_TRY(dalloc(c, &L.members, nm));
    VIP_HIP_TRY(c, hipMemsetAsync(cnt, 0, sizeof(unsigned long long) * (nc + 1), st));
    k_members<<<grid_for(L.n), kBlock, 0, st>>>(L.n, L.agg, L.mstart, cnt, L.members);
    k_sort_members<<<grid_for(nc), kBlock, 0, st>>>(nc, L.mstart, L.members);
    dfree(cnt);
    // Galerkin coarse matrix
    C.A.nrows = nc;
    VIP_TRY(dalloc(c, &C.A.rowlen, nc));
    unsigned long long init = ~0ull;
    VIP_HIP_TRY(c, hipMemcpyAsync(flag, &init, sizeof(init), hipMemcpyHostToDevice, st));
    k_galerkin<<<grid_for(nc), kBlock, 0, st>>>(nc, L.mstart, L.members, A.ptr, A.cols, A.rowlen, aval,
                                                 L.agg, 0, C.A.rowlen, nullptr, nullptr, nullptr, flag);
    rc = ell_layout(c, C.A);
    if (rc != VIP_OK) break;
    VIP_TRY(dalloc(c, &C.A.val[0], C.A.nnz_slots));
    VIP_HIP_TRY(c, hipMemsetAsync(C.A.val[0], 0, sizeof(double) * std::max<int64_t>(C.A.nnz_slots, 1), st));
    k_galerkin<<<grid_for(nc), kBlock, 0, st>>>(nc, L.mstart, L.members, A.ptr, A.cols, A.rowlen, aval,
                                                 L.agg, 1, C.A.rowlen, C.A.ptr, C.A.cols, C.A.val[0], flag);
    VIP_TRY(dalloc(c, &C.A.val32, C.A.nnz_slots));
    k_to32<<<grid_for(C.A.nnz_slots), kBlock, 0, st>>>(C.A.nnz_slots, C.A.val[0], C.A.val32);
    VIP_TRY(ell_deltas(c, C.A));
    VIP_TRY(dalloc(c, &C.A.rsum32, nc));
    launch_rowsum32(st, nc, C.A.ptr, C.A.rowlen, C.A.val[0], C.A.rsum32);
    unsigned long long bad = 0;
    VIP_HIP_TRY(c, hipMemcpyAsync(&bad, flag, sizeof(bad), hipMemcpyDeviceToHost, st));
    VIP_HIP_TRY(c, hipStreamSynchronize(st));
    if (bad != ~0ull) {
      rc = set_error(c, VIP_E_INVALID, "multigrid coarse row wider than 128 entries");
      g.lv.push_back(C);
      break;
    }
    C.vs = 0;
    g.lv.push_back(C);
  }
  if (rc == VIP_OK) {
    // dense inverse of the coarsest level (bordered if the system is singular)
    AmgLevel& Lc = g.lv.back();
    const int64_t m = Lc.n;
    const int border = c->singular ? 1 : 0;
    const int64_t m1 = m + border;
    g.m = m;
    g.m1 = m1;
    if (m1 > 8192) {
      dfree(flag);
      return set_error(c, VIP_E_INVALID, "multigrid coarsening stalled at " + std::to_string(m) +
                                             " rows (dense coarsest solve limited to 8192)");
    }
    double *D = nullptr, *col = nullptr;
    int* badp = nullptr;
    VIP_TRY(dalloc(c, &D, m1 * m1));
    VIP_TRY(dalloc(c, &g.cinv, m1 * m1));
    VIP_TRY(dalloc(c, &g.cinv32, m1 * m1));
    VIP_TRY(dalloc(c, &col, m1));
    VIP_TRY(dalloc(c, &badp, 1));
    VIP_HIP_TRY(c, hipMemsetAsync(badp, 0, sizeof(int), st));
    const int64_t ge = (m1 * m1 + kBlock - 1) / kBlock;
    k_dense_fill<<<ge, kBlock, 0, st>>>(m, border, Lc.A.ptr, Lc.A.cols, Lc.A.rowlen, Lc.A.val[Lc.vs], D,
                                         g.cinv);
    for (int64_t k = 0; k < m1; ++k) {
      k_gj_pivot<<<1, 256, 0, st>>>(m1, k, D, g.cinv, col, badp);
      k_gj_elim<<<ge, kBlock, 0, st>>>(m1, k, D, g.cinv, col);
      k_gj_scale<<<(m1 + kBlock - 1) / kBlock, kBlock, 0, st>>>(m1, k, D, g.cinv, col);
    }
    k_to32<<<ge, kBlock, 0, st>>>(m1 * m1, g.cinv, g.cinv32);
    int bad = 0;
    VIP_HIP_TRY(c, hipMemcpyAsync(&bad, badp, sizeof(int), hipMemcpyDeviceToHost, st));
    VIP_HIP_TRY(c, hipStreamSynchronize(st));
    dfree(D);
    dfree(col);
    dfree(badp);
    if (bad) rc = set_error(c, VIP_E_SINGULAR, "coarsest multigrid matrix is singular");
  }
  dfree(flag);
  VIP_HIP_TRY(c, hipGetLastError());
  if (rc == VIP_OK) g.ready = true;
  return rc;
}

template <typename T>
static LevelView<T> view(const Ctx* c, int level) {
  const AmgLevel& L = c->amg.lv[level];
  LevelView<T> v;
  v.n = L.n;
  v.ptr = L.A.ptr;
  v.cols = L.A.cols;
  v.dcols = L.A.dcols;
  v.dfit = L.A.dfit;
  v.rsum = L.A.rsum32;
  v.cpix = nullptr;
  v.sbase = nullptr;
  v.node_of = L.node_of;
  v.K = L.A.canon.K;
  v.disk = L.A.canon.disk;
  v.box = L.A.canon.box;
  v.W = L.W;
  v.crsum = L.A.canon.rsum32[0];
  if constexpr (sizeof(T) == 4) {
    v.val = L.A.val32;
    v.wdinv = L.wdinv32;
    v.cpix = L.cpix32;
    v.sbase = L.A.canon.disk ? L.sbase32 : nullptr;
    v.wdinv_c = L.wdinv32_c;
    v.wd_uniform = L.wd_uniform32 ? 1 : 0;
    for (int k = 0; k < v.K; ++k) v.w[k] = L.A.canon.w32[0][k];
  } else {
    v.val = L.A.val[L.vs];
    v.wdinv = L.wdinv;
    v.cpix = L.cpix64;
    v.sbase = L.A.canon.disk ? L.sbase64 : nullptr;
    v.wdinv_c = L.wdinv_c;
    v.wd_uniform = L.wd_uniform64 ? 1 : 0;
    for (int k = 0; k < v.K; ++k) v.w[k] = L.A.canon.w[L.vs][k];
  }
  for (int k = 0; k < v.K; ++k) v.off[k] = L.A.canon.off[k];
  // level 0 with canonical rows on: the system layout's tile partition of the same value set;
  // level 1: its own partition on the cell lattice
  if (level == 0 && !c->no_canon && v.disk) {
    const int key = sizeof(T) == 4 ? 1 : (L.vs == 0 ? 0 : -1);
    if (key >= 0) v.tv = tile_view(c, c->sys.canon.tpart[key]);
  }
  if (level == 1 && !c->no_canon && v.box && v.cpix) {
    v.tv = tile_view_of(sizeof(T) == 4 ? L.tpart32 : L.tpart64, L.tmap, L.cell_node, L.W, L.H);
    // tiles built from the filtered sets hold only rows whose damped diagonal is the reference
    v.wd_uniform = L.tiles_filtered ? 1 : v.wd_uniform;
  }
  return v;
}

// Coarse levels below this many rows take the fused launches of the V-cycle (zero start with
// the first sweep, residual with the restriction, prolongation with the first post-sweep):
// there each launch costs a few microseconds however little it does.
constexpr int64_t kFuseRows = int64_t(1) << 20;

static bool fused_level(int l, int64_t n) { return l > 0 && n <= kFuseRows; }

// Blocks of a level-0 row launch: the tile partition's split, else one row per thread.
template <typename T>
static int64_t level_grid(const LevelView<T>& v) {
  return v.tv.tiles ? static_cast<int64_t>(v.tv.tile_blocks) + v.tv.irr_blocks : grid_for(v.n);
}

template <typename T>
__global__ void k_pass_one(const T* src, T* dst) {
  if (threadIdx.x == 0) dst[0] = src[0];
}

template <typename T>
static T* level_buf(Ctx* c, int l, int k) {
  if constexpr (sizeof(T) == 4) return c->amg.lv[l].w32[k];
  else return c->amg.lv[l].w64[k];
}

// Pre-smoothing and restriction on levels [l0, l1): rhs is level l0's right-hand side (level
// l > 0 holds its own in buffer 0 and ping-pongs the iterate between buffers 1 and 2); cur[l]
// becomes the pre-smoothed iterate (null when level 0 skips the pre-smoothing).  Returns the
// right-hand side of level l1.
template <typename T>
static int descend(Ctx* c, hipStream_t st, int l0, int l1, const T* rhs, bool pre_fine, std::vector<T*>& cur,
                   const T** rhs_out) {
  Amg& g = c->amg;
  const int* on = &c->sc->active[0];   // skip the cycle once the solve has stopped on the device
  auto w = [&](int l, int k) { return level_buf<T>(c, l, k); };
  for (int l = l0; l < l1; ++l) {
    const AmgLevel& L = g.lv[l];
    const bool pre = l > 0 || pre_fine;
    const int nu = l == 0 ? c->amg_nu : c->amg_nu_coarse;
    const bool fuse = fused_level(l, L.n);
    const T* res = rhs;
    if (pre) {
      T* a1 = w(l, 1);
      T* a2 = w(l, 2);
      const LevelView<T> lv = view<T>(c, l);
      // the fused zero-start sweep stages W b once per tile entry; on large levels without
      // tiles the row-by-row path would recompute it for every stencil entry, so there W b is
      // stored (small levels fuse anyway: the launch costs more than the recomputation)
      if (nu == 1 || (!lv.tv.tiles && !fuse)) {
        k_jacobi0<T><<<grid_for(L.n), kBlock, 0, st>>>(lv, rhs, a1, on);
        for (int k = 1; k < nu; ++k) {
          k_sweep<T, 0><<<level_grid(lv), kBlock, 0, st>>>(lv, rhs, SweepIn<T>{a1, nullptr},
                                                            a2, on);
          std::swap(a1, a2);
        }
      } else {
        // zero start and the first sweep in one launch
        k_sweep<T, 1><<<level_grid(lv), kBlock, 0, st>>>(lv, rhs, SweepIn<T>{nullptr, rhs},
                                                          a1, on);
        for (int k = 2; k < nu; ++k) {
          k_sweep<T, 0><<<level_grid(lv), kBlock, 0, st>>>(lv, rhs, SweepIn<T>{a1, nullptr},
                                                            a2, on);
          std::swap(a1, a2);
        }
      }
      cur[l] = a1;
      if (fuse) {
        k_restrict_residual<T><<<grid_for(4 * g.lv[l + 1].n), kBlock, 0, st>>>(
            lv, g.lv[l + 1].n, L.mstart, L.members, rhs, a1, w(l + 1, 0), on);
        rhs = w(l + 1, 0);
        continue;
      }
      k_level_residual<T><<<level_grid(lv), kBlock, 0, st>>>(lv, rhs, a1, a2, on);
      res = a2;
    }
    k_restrict<T><<<grid_for(g.lv[l + 1].n), kBlock, 0, st>>>(g.lv[l + 1].n, L.mstart, L.members, res,
                                                               w(l + 1, 0), on);
    rhs = w(l + 1, 0);
  }
  *rhs_out = rhs;
  VIP_HIP_TRY(c, hipGetLastError());
  return VIP_OK;
}

// Coarse correction and post-smoothing on levels l1-1 down to l0, from the coarse iterate xc
// of level l1.  Level 0's right-hand side is b and its last sweep writes x; *xc_out is the
// corrected iterate of level l0.
template <typename T>
static int ascend(Ctx* c, hipStream_t st, int l0, int l1, const T* b, const T* xc, T* x,
                  const std::vector<T*>& cur, const T** xc_out) {
  Amg& g = c->amg;
  const int* on = &c->sc->active[0];
  auto w = [&](int l, int k) { return level_buf<T>(c, l, k); };
  const T gamma = static_cast<T>(c->amg_gamma);
  for (int l = l1 - 1; l >= l0; --l) {
    const AmgLevel& L = g.lv[l];
    const int nu = l == 0 ? c->amg_nu : c->amg_nu_coarse;
    const T* bl = (l == 0) ? b : w(l, 0);
    // y = pre-smoothed iterate + gamma P xc into the buffer that is not cur[l]
    T* y = (cur[l] == w(l, 2)) ? w(l, 1) : w(l, 2);
    T* obuf = (y == w(l, 1)) ? w(l, 2) : w(l, 1);
    const LevelView<T> lv = view<T>(c, l);
    if (fused_level(l, L.n)) {
      // small level: the first sweep starts from x + gamma P xc computed where it is read
      // (saves a launch; on the finest level, tiled, the fused sweep was measured at 77.6 us
      // against 29.4 + 41.5 us for the two launches); sweep k writes bufs[k % 2]
      T* bufs[2] = {y, obuf};
      const T* src = nullptr;
      for (int k = 0; k < nu; ++k) {
        T* dst = bufs[k & 1];
        if (k == 0)
          k_sweep<T, 2><<<level_grid(lv), kBlock, 0, st>>>(
              lv, bl, SweepIn<T>{nullptr, nullptr, cur[l], xc, L.agg, gamma}, dst, on);
        else
          k_sweep<T, 0><<<level_grid(lv), kBlock, 0, st>>>(lv, bl, SweepIn<T>{src, nullptr}, dst, on);
        src = dst;
      }
      xc = src;
      continue;
    }
    // prolongation, then the sweeps (on the large levels a fused prolongation sweep was
    // measured no faster: its staging gathers the coarse correction through the aggregate map)
    k_prolong<T><<<grid_for(L.n), kBlock, 0, st>>>(L.n, L.agg, xc, gamma, cur[l], y, on);
    T* other = obuf;
    for (int k = 0; k < nu; ++k) {
      T* o = (l == 0 && k == nu - 1) ? x : other;
      KTimer kt(c, c->ktime[kTimeSweep0], l == 0 && sizeof(T) == 4, c->vcycle);
      k_sweep<T, 0><<<level_grid(lv), kBlock, 0, st>>>(lv, bl, SweepIn<T>{y, nullptr}, o, on);
      other = y;
      y = o;
    }
    xc = y;
  }
  *xc_out = xc;
  VIP_HIP_TRY(c, hipGetLastError());
  return VIP_OK;
}

// The cycle below the finest level: from level 1's right-hand side (its buffer 0) down to the
// coarsest solve and back; the corrected iterate of level 1 ends in one of its own buffers,
// the same one every cycle.
template <typename T>
static int coarse_cycle(Ctx* c, hipStream_t st, const T** xc_out) {
  Amg& g = c->amg;
  const int nl = static_cast<int>(g.lv.size());
  std::vector<T*> cur(nl, nullptr);
  const T* rhs = nullptr;
  VIP_TRY(descend<T>(c, st, 1, nl - 1, level_buf<T>(c, 1, 0), true, cur, &rhs));
  const T* inv;
  if constexpr (sizeof(T) == 4) inv = g.cinv32;
  else inv = g.cinv;
  T* coarse_out = level_buf<T>(c, nl - 1, 1);
  k_dense_apply<T><<<(g.m * 64 + kBlock - 1) / kBlock, kBlock, 0, st>>>(
      g.m, g.m, g.m1, inv, rhs, coarse_out, &c->sc->active[0]);
  VIP_HIP_TRY(c, hipGetLastError());
  return ascend<T>(c, st, 1, nl - 1, nullptr, coarse_out, nullptr, cur, xc_out);
}

// The coarse cycle as a graph launch: its ~4 launches per level are mostly a few microseconds
// each, and launched one by one after a host round trip the device idles between them.  The
// graph is captured once, on a private stream of its own (so that the caller's stream may be
// the null stream, which cannot be captured), and launched on the caller's stream.  It holds
// only kernel nodes; the kernels read the solve's active flag, so a stopped solve skips the
// work of a launch as it does without the graph.
template <typename T>
static int coarse_cycle_graph(Ctx* c, const T** xc_out) {
  Amg& g = c->amg;
  const int key = sizeof(T) == 4 ? 1 : 0;
  if (!g.coarse_exec[key]) {
    if (!g.cap_stream) VIP_HIP_TRY(c, hipStreamCreateWithFlags(&g.cap_stream, hipStreamNonBlocking));
    hipStream_t st = g.cap_stream;
    VIP_HIP_TRY(c, hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
    const T* out = nullptr;
    const int rc = coarse_cycle<T>(c, st, &out);
    hipGraph_t graph = nullptr;
    const hipError_t e = hipStreamEndCapture(st, &graph);
    if (rc != VIP_OK) {
      if (graph) (void)hipGraphDestroy(graph);
      return rc;
    }
    if (e != hipSuccess || !graph) return set_error(c, VIP_E_HIP, "capturing the coarse V-cycle");
    hipGraphExec_t exec = nullptr;
    const hipError_t e2 = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e2 != hipSuccess || !exec) return set_error(c, VIP_E_HIP, "instantiating the coarse V-cycle");
    g.coarse_exec[key] = exec;
    g.coarse_out[key] = const_cast<T*>(out);
  }
  VIP_HIP_TRY(c, hipGraphLaunch(g.coarse_exec[key], c->stream));
  *xc_out = static_cast<const T*>(g.coarse_out[key]);
  return VIP_OK;
}

// x = M^-1 b for the first n entries (one V-cycle); the border entry is passed through.
// With pre_fine == false the finest level skips its pre-smoothing sweep (a
// non-symmetric V(0,1) cycle there, for BiCGStab only).
template <typename T>
int amg_apply(Ctx* c, const T* b, T* x, bool border, bool pre_fine) {
  Amg& g = c->amg;
  hipStream_t st = c->stream;
  const int* on = &c->sc->active[0];   // skip the cycle once the solve has stopped on the device
  const int nl = static_cast<int>(g.lv.size());
  if (nl == 1) {
    // the whole system is the coarsest level: apply its inverse, bordered if singular
    const T* inv;
    if constexpr (sizeof(T) == 4) inv = g.cinv32;
    else inv = g.cinv;
    const int64_t r = border ? g.m1 : g.m;
    k_dense_apply<T><<<(r * 64 + kBlock - 1) / kBlock, kBlock, 0, st>>>(r, r, g.m1, inv, b, x, on);
    return VIP_OK;
  }
  std::vector<T*> cur(nl, nullptr);
  const T* rhs1 = nullptr;
  VIP_TRY(descend<T>(c, st, 0, 1, b, pre_fine, cur, &rhs1));
  const T* xc = nullptr;
  if (!c->no_graph) VIP_TRY(coarse_cycle_graph<T>(c, &xc));
  else VIP_TRY(coarse_cycle<T>(c, st, &xc));
  const T* x0 = nullptr;
  VIP_TRY(ascend<T>(c, st, 0, 1, b, xc, x, cur, &x0));
  ++c->vcycle;
  if (border) {
    // the border entry passes through (one thread; a runtime copy would take a blit launch)
    k_pass_one<T><<<1, 64, 0, st>>>(b + c->n, x + c->n);
    VIP_HIP_TRY(c, hipGetLastError());
  }
  return VIP_OK;
}

template int amg_apply<float>(Ctx*, const float*, float*, bool, bool);
template int amg_apply<double>(Ctx*, const double*, double*, bool, bool);

}  // namespace vip
