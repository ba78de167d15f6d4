// Krylov solvers of the pressure Poisson system (eq. 13) and of the two
// Crank-Nicolson predictor systems (eq. 12), on the sliced-ELL system layout.
//
// * SpMV kernels are one thread per row over 64-row column-major slices, with
//   the dot products the method needs next fused in.  Each block of a bounded
//   grid takes a contiguous chunk of rows (consecutive chunks on one XCD),
//   writes its partial sums, and a one-block kernel adds them in block order
//   and updates the step lengths (fixed summation order, so repeated runs are
//   bitwise identical; no atomics).  Step lengths (alpha, omega, beta) stay in
//   device memory; the host only reads the residual every few iterations.
// * BiCGStab (van der Vorst) with a Jacobi preconditioner for general systems,
//   Jacobi-preconditioned CG for symmetric ones.  Up to two systems with shared
//   columns (the u and v predictor matrices) run in lockstep.
// * Singular pressure systems are solved in bordered form
//   [A 1; 1^T 0][phi; lambda] = [b; 0]: the extra row and column are applied
//   inside the SpMV (lambda added to every row, sum(phi) as the last row).
// * Mixed precision: FP32 values and vectors in the inner solve, FP64 residual
//   and accumulation in an iterative-refinement outer loop.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <string>
#include <vector>

#include "tile.h"
#include "vip_internal.h"

namespace vip {

namespace {

constexpr int kWaves = kBlock / 64;
// Blocks of a reducing kernel (each takes a contiguous chunk of rows): VIP_MAX_GRID, default 2048
// (measured on the step at h = D/128 against 512, 1024, 4096, 8192 and 16384: enough blocks in
// flight to hide the loads, few enough partials for one-block finish kernels).
inline int64_t max_grid() {
  static const int64_t g = [] {
    const char* e = std::getenv("VIP_MAX_GRID");
    int64_t v = e ? std::atoll(e) : 2048;
    v = std::min<int64_t>(std::max<int64_t>(v, 64), int64_t{1} << 20);
    return (v + kNumXcd - 1) / kNumXcd * kNumXcd;
  }();
  return g;
}

// Grid of a reducing kernel over m items: bounded, a multiple of the XCD count.
inline int64_t red_grid(int64_t m) { return std::min<int64_t>(grid_for(m), max_grid()); }

// Contiguous chunk of items [begin, end) handled by this block; consecutive
// logical blocks (same XCD) get consecutive chunks.
struct Span {
  int64_t begin, end;
};

__device__ __forceinline__ Span block_span(int64_t m) {
  const int64_t lb = xcd_block(blockIdx.x, gridDim.x);
  const int64_t per = ((m + gridDim.x - 1) / gridDim.x + kSlice - 1) / kSlice * kSlice;
  const int64_t b = lb * per;
  return {b, b + per < m ? b + per : m};
}

// Block sums of NV values, written to partials[blockIdx.x * stride + a] (plain stores; stride NV
// unless several launches interleave their sums); a finishing kernel adds them up in block order.
template <int NV>
__device__ __forceinline__ void block_sum_store(double (&v)[NV], double* partials, int stride = NV) {
  __shared__ double red[NV][kWaves];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int a = 0; a < NV; ++a) {
    double t = v[a];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) t += __shfl_xor(t, off, 64);
    if (lane == 0) red[a][wave] = t;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
#pragma unroll
    for (int a = 0; a < NV; ++a) {
      double t = 0.0;
#pragma unroll
      for (int w = 0; w < kWaves; ++w) t += red[a][w];
      partials[static_cast<int64_t>(blockIdx.x) * stride + a] = t;
    }
  }
}

// Totals of the block sums of `nb` blocks, in a fixed order (one block of kBlock threads);
// the result is valid in every thread.
template <int NV>
__device__ __forceinline__ void grid_sum(const double* partials, int64_t nb, double (&tot)[NV]) {
  __shared__ double red[NV][kWaves];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  // each thread adds blocks threadIdx.x + 256 k in increasing k; eight blocks' values are
  // loaded before they are added, so the loads are in flight together
  double t[NV];
#pragma unroll
  for (int a = 0; a < NV; ++a) t[a] = 0.0;
  constexpr int kAhead = 8;
  int64_t b = threadIdx.x;
  for (; b + (kAhead - 1) * static_cast<int64_t>(blockDim.x) < nb; b += kAhead * static_cast<int64_t>(blockDim.x)) {
    double v[kAhead][NV];
#pragma unroll
    for (int u = 0; u < kAhead; ++u)
#pragma unroll
      for (int a = 0; a < NV; ++a) v[u][a] = partials[(b + u * static_cast<int64_t>(blockDim.x)) * NV + a];
#pragma unroll
    for (int u = 0; u < kAhead; ++u)
#pragma unroll
      for (int a = 0; a < NV; ++a) t[a] += v[u][a];
  }
  for (; b < nb; b += blockDim.x)
#pragma unroll
    for (int a = 0; a < NV; ++a) t[a] += partials[b * NV + a];
#pragma unroll
  for (int a = 0; a < NV; ++a) {
    double ta = t[a];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) ta += __shfl_xor(ta, off, 64);
    if (lane == 0) red[a][wave] = ta;
  }
  __syncthreads();
#pragma unroll
  for (int a = 0; a < NV; ++a) {
    double t = 0.0;
#pragma unroll
    for (int w = 0; w < kWaves; ++w) t += red[a][w];
    tot[a] = t;
  }
}

__device__ __forceinline__ double safe_div(double a, double b, int* flag) {
  if (b == 0.0 || !isfinite(a) || !isfinite(b)) {
    *flag = 1;
    return 0.0;
  }
  return a / b;
}

template <typename VT>
struct Mat {
  int64_t n;               // rows without the border
  int border;              // 1: bordered singular form
  const int64_t* ptr;
  const int32_t* cols;
  const VT* val[2];        // value sets of system 0 and 1
  const float* rsum[2];    // FP32 values only: row sums of systems 0 and 1 for the difference form
  // lattice-interior rows (stencil.hip): pixel of a canonical row, else -1; null = none
  const int32_t* cpix[2];
  const int32_t* sbase[2]; // slice descriptors of the canonical rows, or null
  const int32_t* node_of;
  int K;
  int disk;                // taps are the 21-point disk (unrolled path)
  int32_t W;               // lattice image width
  int32_t off[kMaxTaps];
  VT w[2][kMaxTaps];
  float crsum[2];
  TileView tv;             // tile partition of the systems' canonical rows (tile.h), if any
  int tile_general;        // 1: tile rows also take the row-by-row path (canonical rows off)
  const int16_t* dcols;    // row-relative columns (Ell::dcols), or null: read cols
  const uint8_t* dfit;     // per slice: 1 where dcols holds the slice's columns
};


// Total of an FP32 difference-form row, sum_j a_ij (x_j - x_i) + (sum_j a_ij) x_i: the two
// accumulators added in FP32, then the row-sum term by one explicit FP64 fused multiply-add (its
// product is exact).  Written out so that no variant of a row product leaves the contraction to
// the compiler, which fuses a product-then-add or not depending on the code around it.
__device__ __forceinline__ double diff_total(float a0, float a1, float rsum, float xi) {
  return fma(static_cast<double>(rsum), static_cast<double>(xi), static_cast<double>(a0 + a1));
}

// Every system a kernel will touch has its values (and, in FP32, its row sums).
template <typename VT>
int check_mat(Ctx* c, const Mat<VT>& A, int ns) {
  for (int s = 0; s < ns; ++s) {
    if (!A.val[s] || !A.ptr || !A.cols) return set_error(c, VIP_E_INVALID, "matrix of a system is missing");
    if (sizeof(VT) == 4 && !A.rsum[s]) return set_error(c, VIP_E_INVALID, "FP32 row sums of a system are missing");
  }
  return VIP_OK;
}

// Attach the canonical rows of value sets vs0 (system 0) and vs1 (system 1, -1 = none);
// sets 4..6 are the FP32 pressure and predictor sets.
template <typename VT>
void attach_canon(const Ctx* c, Mat<VT>& A, int vs0, int vs1) {
  const Canon& cn = c->sys.canon;
  A.cpix[0] = A.cpix[1] = nullptr;
  A.sbase[0] = A.sbase[1] = nullptr;
  // the tile partition fixes the order rows are visited in, so it is kept with canonical rows
  // off (every row then takes the row-by-row path) and reductions give the same bits
  const int key = (vs0 == 0 && vs1 < 0) ? 0 : (vs0 == 4 && vs1 < 0) ? 1 : (vs0 == 1 && vs1 == 2) ? 2
                : (vs0 == 5 && vs1 == 6) ? 3 : -1;
  A.tv = key >= 0 ? tile_view(c, cn.tpart[key]) : TileView();
  A.tile_general = c->no_canon ? 1 : 0;
  A.dcols = c->sys.dcols;
  A.dfit = c->sys.dfit;
  if (c->no_canon || cn.K == 0) return;
  const int vs[2] = {vs0, vs1};
  for (int s = 0; s < 2; ++s) {
    if (vs[s] < 0 || cn.count[vs[s]] == 0 || !cn.cpix[vs[s]]) continue;
    A.cpix[s] = cn.cpix[vs[s]];
    A.sbase[s] = cn.disk ? cn.sbase[vs[s]] : nullptr;
    for (int k = 0; k < cn.K; ++k)
      A.w[s][k] = (vs[s] >= 4) ? static_cast<VT>(cn.w32[vs[s] - 4][k]) : static_cast<VT>(cn.w[vs[s]][k]);
    A.crsum[s] = vs[s] >= 4 ? cn.rsum32[vs[s] - 4] : 0.0f;
  }
  A.node_of = c->lat.node_of;
  A.K = cn.K;
  A.disk = cn.disk;
  A.W = c->lat.W;
  for (int k = 0; k < cn.K; ++k) A.off[k] = cn.off[k];
}

// Blocks of a reducing SpMV launch: the tile partition's split, else the row grid.
template <typename VT>
int64_t spmv_grid(const Mat<VT>& A) {
  return A.tv.tiles ? static_cast<int64_t>(A.tv.tile_blocks) + A.tv.irr_blocks : red_grid(A.n);
}

template <typename T>
struct Vec {
  int64_t stride;          // distance between the vectors of system 0 and 1
  T* x;
  T* r;
  T* rhat;
  T* p;
  T* ph;
  T* v;
  T* s;
  T* sh;
  T* t;
  const T* dinv[2];
};

// Canonical row: the weights come from the reference row and the columns from the lattice
// map.  Slots go to the two accumulators in the general path's order (pairs of the unrolled
// groups alternate, the tail goes to the first), so the bits are the same.  Every product is
// added by an explicit fused multiply-add, here, in the general row and in the reductions of
// the kernels' two variants: left to the compiler, fusing depends on where the product lands
// in the code and then differs between the variants in the last bit.
// 21-point disk with the five row bases given: slots 0, 2, ..., 20 to the first accumulator,
// the odd ones to the second (a slice of such rows is at least 21 wide, so only slot 20 can
// fall in the tail of the general path)
template <typename VT, typename Tap>
__device__ __forceinline__ double disk_sum(const Mat<VT>& A, int sys, Tap&& tap) {
  if constexpr (sizeof(VT) == 4) {
    const float xi = static_cast<float>(tap(2, 0));
    float a0 = 0.0f, a1 = 0.0f;
#pragma unroll
    for (int k = 0; k < kDiskTaps; ++k) {
      const float d = static_cast<float>(tap(disk_row(k), disk_dx(k))) - xi;
      if (k & 1) a1 = fmaf(A.w[sys][k], d, a1);
      else a0 = fmaf(A.w[sys][k], d, a0);
    }
    return diff_total(a0, a1, A.crsum[sys], xi);
  } else {
    double a0 = 0.0, a1 = 0.0;
#pragma unroll
    for (int k = 0; k < kDiskTaps; ++k) {
      const double d = static_cast<double>(tap(disk_row(k), disk_dx(k)));
      if (k & 1) a1 = fma(A.w[sys][k], d, a1);
      else a0 = fma(A.w[sys][k], d, a0);
    }
    return a0 + a1;
  }
}

template <typename VT, typename X>
__device__ __forceinline__ double disk_dot(const Mat<VT>& A, int sys, int64_t i, const int32_t (&b)[5],
                                           const X& x) {
  (void)i;
  return disk_sum(A, sys, [&](int r, int dx) __attribute__((always_inline)) { return x[b[r] + dx]; });
}

// the same row from a tile's LDS copy (tile.h): tap (r, dx) of local row ly, lane lx
template <typename VT, typename T>
__device__ __forceinline__ double disk_lds(const Mat<VT>& A, int sys, const T (&t)[kTileLdsH][kTileLdsW], int ly,
                                           int lx) {
  return disk_sum(A, sys, [&](int r, int dx) __attribute__((always_inline)) { return t[ly + r][lx + 2 + dx]; });
}

template <typename VT, typename X>
__device__ __forceinline__ double canon_dot(const Mat<VT>& A, int sys, int32_t p, int64_t i, int w,
                                            const X& x) {
  if (A.disk) {
    int32_t b[5];
    disk_bases(A.node_of, p, A.W, i, b);
    return disk_dot(A, sys, i, b, x);
  }
  const int full = w & ~3;
  const int32_t* nb = A.node_of + p;
  if constexpr (sizeof(VT) == 4) {
    const float xi = static_cast<float>(x[i]);
    float a0 = 0.0f, a1 = 0.0f;
    int k = 0;
    for (; k + 4 <= A.K && k + 4 <= full; k += 4) {
      const int32_t c0 = nb[A.off[k]], c1 = nb[A.off[k + 1]], c2 = nb[A.off[k + 2]], c3 = nb[A.off[k + 3]];
      const float x0 = static_cast<float>(x[c0]), x1 = static_cast<float>(x[c1]),
                  x2 = static_cast<float>(x[c2]), x3 = static_cast<float>(x[c3]);
      a0 = fmaf(A.w[sys][k], x0 - xi, a0);
      a1 = fmaf(A.w[sys][k + 1], x1 - xi, a1);
      a0 = fmaf(A.w[sys][k + 2], x2 - xi, a0);
      a1 = fmaf(A.w[sys][k + 3], x3 - xi, a1);
    }
    for (; k < A.K; ++k) {
      const float d = static_cast<float>(x[nb[A.off[k]]]) - xi;
      if (k < full && (k & 1)) a1 = fmaf(A.w[sys][k], d, a1);
      else a0 = fmaf(A.w[sys][k], d, a0);
    }
    return diff_total(a0, a1, A.crsum[sys], xi);
  } else {
    double a0 = 0.0, a1 = 0.0;
    int k = 0;
    for (; k + 4 <= A.K && k + 4 <= full; k += 4) {
      const int32_t c0 = nb[A.off[k]], c1 = nb[A.off[k + 1]], c2 = nb[A.off[k + 2]], c3 = nb[A.off[k + 3]];
      const double x0 = static_cast<double>(x[c0]), x1 = static_cast<double>(x[c1]),
                   x2 = static_cast<double>(x[c2]), x3 = static_cast<double>(x[c3]);
      a0 = fma(A.w[sys][k], x0, a0);
      a1 = fma(A.w[sys][k + 1], x1, a1);
      a0 = fma(A.w[sys][k + 2], x2, a0);
      a1 = fma(A.w[sys][k + 3], x3, a1);
    }
    for (; k < A.K; ++k) {
      const double d = static_cast<double>(x[nb[A.off[k]]]);
      if (k < full && (k & 1)) a1 = fma(A.w[sys][k], d, a1);
      else a0 = fma(A.w[sys][k], d, a0);
    }
    return a0 + a1;
  }
}

// Row i of y = A x for system `sys`; x is the system's vector (a pointer, or any accessor whose
// x[j] gives entry j).  The slot loop is
// unrolled by four so the column loads of several slots are in flight before
// their gathers.
// (without the slice descriptors: canonical rows by pixel, else the sliced ELL)
template <typename VT, typename X>
__device__ __forceinline__ double row_dot_rows(const Mat<VT>& A, int sys, int64_t i, const X& x) {
  const int64_t sl = i / kSlice;
  const int64_t base = A.ptr[sl] + (i % kSlice);
  const int w = static_cast<int>((A.ptr[sl + 1] - A.ptr[sl]) / kSlice);
  if (A.cpix[sys]) {
    const int32_t p = A.cpix[sys][i];
    if (p >= 0) return canon_dot(A, sys, p, i, w, x);
  }
  const VT* vals = A.val[sys];
  // the slot loop once per column stream, so that each instance issues loads of one kind only
  auto sum = [&](auto col) __attribute__((always_inline)) -> double {
    if constexpr (sizeof(VT) == 4) {
      // difference form: rows of the pressure matrix sum to ~0, so on smooth x the
      // plain sum cancels most of its digits in FP32; x_j - x_i of nearby values is
      // exact and keeps them
      const float xi = static_cast<float>(x[i]);
      float a0 = 0.0f, a1 = 0.0f;
      int k = 0;
      for (; k + 4 <= w; k += 4) {
        const int64_t q = base + static_cast<int64_t>(k) * kSlice;
        const int32_t c0 = col(q), c1 = col(q + kSlice), c2 = col(q + 2 * kSlice), c3 = col(q + 3 * kSlice);
        const float v0 = vals[q], v1 = vals[q + kSlice], v2 = vals[q + 2 * kSlice], v3 = vals[q + 3 * kSlice];
        const float x0 = static_cast<float>(x[c0]), x1 = static_cast<float>(x[c1]),
                    x2 = static_cast<float>(x[c2]), x3 = static_cast<float>(x[c3]);
        a0 = fmaf(v0, x0 - xi, a0);
        a1 = fmaf(v1, x1 - xi, a1);
        a0 = fmaf(v2, x2 - xi, a0);
        a1 = fmaf(v3, x3 - xi, a1);
      }
      for (; k < w; ++k) {
        const int64_t q = base + static_cast<int64_t>(k) * kSlice;
        a0 = fmaf(static_cast<float>(vals[q]), static_cast<float>(x[col(q)]) - xi, a0);
      }
      return diff_total(a0, a1, A.rsum[sys][i], xi);
    } else {
      double a0 = 0.0, a1 = 0.0;
      int k = 0;
      for (; k + 4 <= w; k += 4) {
        const int64_t q = base + static_cast<int64_t>(k) * kSlice;
        const int32_t c0 = col(q), c1 = col(q + kSlice), c2 = col(q + 2 * kSlice), c3 = col(q + 3 * kSlice);
        const double v0 = vals[q], v1 = vals[q + kSlice], v2 = vals[q + 2 * kSlice], v3 = vals[q + 3 * kSlice];
        const double x0 = static_cast<double>(x[c0]), x1 = static_cast<double>(x[c1]),
                     x2 = static_cast<double>(x[c2]), x3 = static_cast<double>(x[c3]);
        a0 = fma(v0, x0, a0);
        a1 = fma(v1, x1, a1);
        a0 = fma(v2, x2, a0);
        a1 = fma(v3, x3, a1);
      }
      for (; k < w; ++k) {
        const int64_t q = base + static_cast<int64_t>(k) * kSlice;
        a0 = fma(static_cast<double>(vals[q]), static_cast<double>(x[col(q)]), a0);
      }
      return a0 + a1;
    }
  };
  if (A.dcols && A.dfit[sl]) {
    const int32_t ii = static_cast<int32_t>(i);
    return sum([&](int64_t q) __attribute__((always_inline)) { return ii + static_cast<int32_t>(A.dcols[q]); });
  }
  return sum([&](int64_t q) __attribute__((always_inline)) { return A.cols[q]; });
}

template <typename VT, typename X>
__device__ __forceinline__ double row_dot(const Mat<VT>& A, int sys, int64_t i, const X& x) {
  if (A.sbase[sys]) {
    int32_t b[5];
    if (slice_disk_bases(A.sbase[sys], i, b)) return disk_dot(A, sys, i, b, x);
  }
  return row_dot_rows(A, sys, i, x);
}

// Row loop of the reducing SpMV kernels: the block's rows sp.begin + threadIdx.x + 256 k (the
// order of a plain strided loop, so per-thread sums keep their order), visited as one 64-row
// slice per wave and step.  A slice described for every system in use (Canon::sbase; the
// systems then share the five row bases) goes to fast(i, b); its gathers for all systems can be
// in flight together, and the descriptors of the wave's next slice are loaded one step ahead.
// Other slices go row by row to slow(i).
template <typename VT, int NS, typename Fast, typename Slow>
__device__ __forceinline__ void walk_rows(const Mat<VT>& A, const bool (&use)[NS], Fast&& fast, Slow&& slow) {
  const Span sp = block_span(A.n);
  const int wave = __builtin_amdgcn_readfirstlane(static_cast<int>(threadIdx.x >> 6));
  const int lane = static_cast<int>(threadIdx.x & 63);
  const int64_t first = sp.begin / kSlice + wave;
  const int64_t last = (sp.end + kSlice - 1) / kSlice;
  bool any = false, desc = true;
#pragma unroll
  for (int s = 0; s < NS; ++s) {
    any = any || use[s];
    if (use[s] && !A.sbase[s]) desc = false;
  }
  if (!any) return;
  int4 nd[NS];
  auto fetch = [&](int64_t sl) __attribute__((always_inline)) {
#pragma unroll
    for (int s = 0; s < NS; ++s)
      nd[s] = desc && use[s] && sl < last ? *reinterpret_cast<const int4*>(A.sbase[s] + 4 * sl)
                                          : make_int4(-1, -1, -1, -1);
  };
  fetch(first);
  for (int64_t sl = first; sl < last; sl += kWaves) {
    int4 d[NS];
#pragma unroll
    for (int s = 0; s < NS; ++s) d[s] = nd[s];
    fetch(sl + kWaves);
    const int64_t i = sl * kSlice + lane;
    bool ok = desc;
    int4 db = make_int4(-1, -1, -1, -1);
#pragma unroll
    for (int s = 0; s < NS; ++s)
      if (use[s]) {
        ok = ok && __builtin_amdgcn_readfirstlane(d[s].x) >= 0;
        db = d[s];
      }
    if (ok) {
      // a described slice holds 64 rows below n, all inside this span
      const int32_t b[5] = {__builtin_amdgcn_readfirstlane(db.x) + lane, __builtin_amdgcn_readfirstlane(db.y) + lane,
                            static_cast<int32_t>(i), __builtin_amdgcn_readfirstlane(db.z) + lane,
                            __builtin_amdgcn_readfirstlane(db.w) + lane};
      fast(i, b);
    } else if (i < sp.end) {
      slow(i);
    }
  }
}

// ---- residual: r = b - A x, rr = |r|^2, bb = |b|^2 ----------------------------------------------
template <typename VT, typename XT, typename RT, int NS, bool GEN>
__global__ void __launch_bounds__(kBlock) k_residual(Mat<VT> A, const XT* x, const double* b, RT* r, int64_t stride,
                           double* partials) {
  __shared__ XT lds[NS][kTileLdsH][kTileLdsW];
  __shared__ TileMeta meta;
  double acc[3 * NS];
#pragma unroll
  for (int a = 0; a < 3 * NS; ++a) acc[a] = 0.0;
  double xn[NS];   // border unknowns (uniform)
#pragma unroll
  for (int s = 0; s < NS; ++s) xn[s] = A.border ? static_cast<double>(x[s * stride + A.n]) : 0.0;
  auto emit = [&](int s, int64_t i, double ax, double bi, double xi) __attribute__((always_inline)) {
    if (A.border) ax += xn[s];
    const double ri = bi - ax;
    r[s * stride + i] = static_cast<RT>(ri);
    acc[3 * s + 0] = fma(ri, ri, acc[3 * s + 0]);
    acc[3 * s + 1] = fma(bi, bi, acc[3 * s + 1]);
    if (A.border) acc[3 * s + 2] += xi;
  };
  auto slow = [&](int64_t i) __attribute__((always_inline)) {
#pragma unroll
    for (int s = 0; s < NS; ++s)
      emit(s, i, row_dot_rows(A, s, i, x + s * stride), b[s * stride + i], static_cast<double>(x[s * stride + i]));
  };
  if (A.tv.tiles) {
    const XT* xs[NS];
#pragma unroll
    for (int s = 0; s < NS; ++s) xs[s] = x + s * stride;
    tile_walk(
        A.tv,
        [&](int64_t tk) __attribute__((always_inline)) {
            tile_stage<XT, NS>(A.tv, tk, xs, lds, meta, !GEN);
            if constexpr (GEN) {
#pragma unroll 1
              for (int k = 0; k < kTileRowsPerWave; ++k) {
                const int64_t row = tile_row_id(A.tv, meta, k);
                if (row >= 0) slow(row);
              }
              return;
            }
            const int wave = static_cast<int>(threadIdx.x >> 6), lane = static_cast<int>(threadIdx.x & 63);
#pragma unroll 1
            for (int k = 0; k < kTileRowsPerWave; ++k) {
              const int64_t row = tile_row_id(A.tv, meta, k);
              if (row < 0) continue;
              const int ly = wave + k * (kBlock / 64);
              double bi[NS];
#pragma unroll
              for (int s = 0; s < NS; ++s) bi[s] = b[s * stride + row];
              double y[NS];
#pragma unroll
              for (int s = 0; s < NS; ++s) y[s] = disk_lds(A, s, lds[s], ly, lane);
#pragma unroll
              for (int s = 0; s < NS; ++s) emit(s, row, y[s], bi[s], static_cast<double>(lds[s][ly + 2][lane + 2]));
            }
          },
        slow);
  } else {
    bool use[NS];
#pragma unroll
    for (int s = 0; s < NS; ++s) use[s] = true;
    walk_rows(
        A, use,
        [&](int64_t i, const int32_t (&bs)[5]) {
          double y[NS], bi[NS], xi[NS];
#pragma unroll
          for (int s = 0; s < NS; ++s) {
            bi[s] = b[s * stride + i];
            xi[s] = static_cast<double>(x[s * stride + i]);
          }
#pragma unroll
          for (int s = 0; s < NS; ++s) y[s] = disk_dot(A, s, i, bs, x + s * stride);
#pragma unroll
          for (int s = 0; s < NS; ++s) emit(s, i, y[s], bi[s], xi[s]);
        },
        slow);
  }
  block_sum_store<3 * NS>(acc, partials);
}

template <typename RT, int NS>
__global__ void k_fin_residual(const double* partials, int64_t nb, int64_t n, int border, const double* b,
                               RT* r, int64_t stride, KrylovScalars* sc) {
  double tot[3 * NS];
  grid_sum<3 * NS>(partials, nb, tot);
  if (threadIdx.x != 0) return;
#pragma unroll
  for (int s = 0; s < NS; ++s) {
    double rr = tot[3 * s], bb = tot[3 * s + 1];
    if (border) {
      const double bn = b[s * stride + n];
      const double rn = bn - tot[3 * s + 2];
      r[s * stride + n] = static_cast<RT>(rn);
      rr += rn * rn;
      bb += bn * bn;
    }
    sc->rr[s] = rr;
    sc->bb[s] = bb;
  }
}

// ---- BiCGStab -------------------------------------------------------------------------------------
template <typename T, int NS>
__global__ void k_bicg_init(Vec<T> V, int64_t nvec, KrylovScalars* sc, int zero_x) {
  const int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
  if (i < nvec) {
#pragma unroll
    for (int s = 0; s < NS; ++s) {
      const int64_t o = s * V.stride + i;
      V.rhat[o] = V.r[o];
      V.p[o] = T(0);
      V.v[o] = T(0);
      if (zero_x) V.x[o] = T(0);
    }
  }
  if (i == 0) {
#pragma unroll
    for (int s = 0; s < NS; ++s) {
      sc->rho[s] = sc->rr[s];   // rhat = r
      sc->alpha[s] = 1.0;
      sc->omega[s] = 1.0;
      sc->beta[s] = 0.0;
      sc->breakdown[s] = 0;
      sc->pending[s] = 0;
      sc->par[s] = 0;
    }
  }
}

// p = r + beta (p - omega v); ph = D^-1 p (Jacobi)
template <typename T, int NS>
__global__ void k_bicg_p(Vec<T> V, int64_t nvec, const KrylovScalars* sc, int jac) {
  const int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
  if (i >= nvec) return;
#pragma unroll
  for (int s = 0; s < NS; ++s) {
    if (!sc->active[s]) continue;
    const int64_t o = s * V.stride + i;
    const T beta = static_cast<T>(sc->beta[s]), omega = static_cast<T>(sc->omega[s]);
    const T p = V.r[o] + beta * (V.p[o] - omega * V.v[o]);
    V.p[o] = p;
    if (jac) V.ph[o] = V.dinv[s][i] * p;
  }
}

// Waves per SIMD asked of the single-system FP32 SpMV kernels: their 63-64 VGPRs allow 8, and
// the bound lets the compiler keep the scalar registers to that count (the excess scalars live
// in vector-register lanes, no scratch); the t kernel that also forms s fits 6 (79 VGPRs).
// Other instances would spill to scratch under such a bound.
template <typename T, int NS, bool FS = false>
constexpr int kWavesFor = (sizeof(T) == 4 && NS == 1) ? (FS ? 6 : 8) : 1;

// The two-system FP32 SpMV walks its tiles pipelined (tile_walk_pp): measured 105.3 -> 91.8 us
// per launch at h = 1/128.  The single-system one stays on one tile at a time: the held
// operands cost it 3 of its 8 waves per SIMD, and it ran 41.6 -> 47.8 us.
template <typename T, int NS>
constexpr bool kPipelinedV = sizeof(T) == 4 && NS == 2;

// v = A ph; partial sums of rhat . v (and of ph for the border row).  A launch may take system q0
// of a two-system solve alone (A, V viewed at that system): its block sums then land at
// partials[pstride b + 2 q0 + a], interleaved with the other system's launch as a two-system
// launch stores them.
template <typename VT, typename T, int NS, bool GEN>
__global__ void __launch_bounds__(kBlock, (kWavesFor<T, NS>)) k_bicg_v(Mat<VT> A, Vec<T> V, double* partials,
                                                                      const KrylovScalars* sc, int q0 = 0,
                                                                      int pstride = 2 * NS) {
  __shared__ T lds[NS][kTileLdsH][kTileLdsW];
  __shared__ TileMeta meta2[2];
  TileMeta& meta = meta2[0];
  double acc[2 * NS];
#pragma unroll
  for (int a = 0; a < 2 * NS; ++a) acc[a] = 0.0;
  bool use[NS], any = false;
  double phn[NS];   // border unknowns (uniform)
#pragma unroll
  for (int s = 0; s < NS; ++s) {
    use[s] = sc->active[q0 + s] != 0;
    any = any || use[s];
    phn[s] = A.border ? static_cast<double>(V.ph[s * V.stride + A.n]) : 0.0;
  }
  auto emit = [&](int s, int64_t i, double y, T rh, T pc) __attribute__((always_inline)) {
    if (A.border) y += phn[s];
    const T yt = static_cast<T>(y);
    V.v[s * V.stride + i] = yt;
    acc[2 * s] = fma(static_cast<double>(rh), static_cast<double>(yt), acc[2 * s]);
    if (A.border) acc[2 * s + 1] += static_cast<double>(pc);
  };
  auto slow = [&](int64_t i) __attribute__((always_inline)) {
#pragma unroll
    for (int s = 0; s < NS; ++s)
      if (use[s])
        emit(s, i, row_dot_rows(A, s, i, V.ph + s * V.stride), V.rhat[s * V.stride + i], V.ph[s * V.stride + i]);
  };
  if (A.tv.tiles) {
    const T* xs[NS];
#pragma unroll
    for (int s = 0; s < NS; ++s) xs[s] = V.ph + s * V.stride;
    if (any) {
      if constexpr (GEN) {
        tile_walk(
            A.tv,
            [&](int64_t tk) __attribute__((always_inline)) {
              tile_stage<T, NS>(A.tv, tk, xs, lds, meta, false);
#pragma unroll 1
              for (int k = 0; k < kTileRowsPerWave; ++k) {
                const int64_t row = tile_row_id(A.tv, meta, k);
                if (row >= 0) slow(row);
              }
            },
            slow);
      } else {
        const int wave = static_cast<int>(threadIdx.x >> 6), lane = static_cast<int>(threadIdx.x & 63);
        int64_t rows[kTileRowsPerWave];
        T rh[NS][kTileRowsPerWave];
        auto tile_rows = [&](const TileMeta& mm) __attribute__((always_inline)) {
#pragma unroll
          for (int k = 0; k < kTileRowsPerWave; ++k) {
            rows[k] = tile_row_id(A.tv, mm, k);
#pragma unroll
            for (int s = 0; s < NS; ++s) rh[s][k] = rows[k] >= 0 ? V.rhat[s * V.stride + rows[k]] : T(0);
          }
        };
        auto tile_rows_compute = [&]() __attribute__((always_inline)) {
#pragma unroll 1
          for (int k = 0; k < kTileRowsPerWave; ++k) {
            if (rows[k] < 0) continue;
            const int ly = wave + k * (kBlock / 64);
            double y[NS];
#pragma unroll
            for (int s = 0; s < NS; ++s) y[s] = disk_lds(A, s, lds[s], ly, lane);
#pragma unroll
            for (int s = 0; s < NS; ++s) if (use[s]) emit(s, rows[k], y[s], rh[s][k], lds[s][ly + 2][lane + 2]);
          }
        };
        if constexpr (kPipelinedV<T, NS>) {
          // pipelined: the next tile's ph in flight while this one is computed; the rows' rhat
          // loaded when the tile is staged (the FP64 instances keep one tile at a time: the
          // held operands would cost them an occupancy step)
          tile_walk_pp<T, NS, T>(
              A.tv, lds, meta2, [&](int s, int32_t node) __attribute__((always_inline)) { return xs[s][node]; },
              [&](int, T x) __attribute__((always_inline)) { return x; },
              [&](int64_t, const TileMeta& mm) __attribute__((always_inline)) { tile_rows(mm); },
              [&](int64_t, const TileMeta&) __attribute__((always_inline)) { tile_rows_compute(); }, slow);
        } else {
          tile_walk(
              A.tv,
              [&](int64_t tk) __attribute__((always_inline)) {
                tile_stage<T, NS>(A.tv, tk, xs, lds, meta, true);
#pragma unroll 1
                for (int k = 0; k < kTileRowsPerWave; ++k) {
                  const int64_t row = tile_row_id(A.tv, meta, k);
                  if (row < 0) continue;
                  const int ly = wave + k * (kBlock / 64);
                  T rh1[NS];
#pragma unroll
                  for (int s = 0; s < NS; ++s) rh1[s] = V.rhat[s * V.stride + row];
                  double y[NS];
#pragma unroll
                  for (int s = 0; s < NS; ++s) y[s] = disk_lds(A, s, lds[s], ly, lane);
#pragma unroll
                  for (int s = 0; s < NS; ++s) if (use[s]) emit(s, row, y[s], rh1[s], lds[s][ly + 2][lane + 2]);
                }
              },
              slow);
        }
      }
    }
  } else {
    walk_rows(
        A, use,
        [&](int64_t i, const int32_t (&b)[5]) {
          // every system's row is computed (in-bounds reads) so all loads issue together
          double y[NS];
          T rh[NS], pc[NS];
#pragma unroll
          for (int s = 0; s < NS; ++s) {
            rh[s] = V.rhat[s * V.stride + i];
            pc[s] = V.ph[s * V.stride + i];
          }
#pragma unroll
          for (int s = 0; s < NS; ++s) y[s] = disk_dot(A, s, i, b, V.ph + s * V.stride);
#pragma unroll
          for (int s = 0; s < NS; ++s)
            if (use[s]) emit(s, i, y[s], rh[s], pc[s]);
        },
        slow);
  }
  block_sum_store<2 * NS>(acc, partials + 2 * q0, pstride);
}

// alpha = rho / (rhat . v), with the border row v[n] = sum(ph)
template <typename T, int NS>
__global__ void k_fin_bicg_v(const double* partials, int64_t nb, int64_t n, int border, Vec<T> V,
                             KrylovScalars* sc) {
  double tot[2 * NS];
  grid_sum<2 * NS>(partials, nb, tot);
  if (threadIdx.x != 0) return;
#pragma unroll
  for (int s = 0; s < NS; ++s) {
    sc->pending[s] = 0;   // (the update pass before this SpMV applied it)
    if (!sc->active[s]) continue;
    double d = tot[2 * s];
    if (border) {
      const T yn = static_cast<T>(tot[2 * s + 1]);
      V.v[s * V.stride + n] = yn;
      d += static_cast<double>(V.rhat[s * V.stride + n]) * static_cast<double>(yn);
    }
    sc->dot_a[s] = d;
    sc->alpha[s] = safe_div(sc->rho[s], d, &sc->breakdown[s]);
    if (sc->breakdown[s]) sc->active[s] = 0;
  }
}

// s = r - alpha v, one rounding; the one expression for s wherever it is formed
template <typename T>
__device__ __forceinline__ T bicg_s_value(T r, T v, T alpha) {
  if constexpr (sizeof(T) == 4) return fmaf(-alpha, v, r);
  else return fma(-alpha, v, r);
}

// s of one system computed where it is read (x[j] of a row product)
template <typename T>
struct SValues {
  const T* r;
  const T* v;
  T alpha;
  __device__ __forceinline__ T operator[](int64_t j) const { return bicg_s_value(r[j], v[j], alpha); }
};

// s = r - alpha v; sh = D^-1 s (Jacobi)
template <typename T, int NS>
__global__ void k_bicg_s(Vec<T> V, int64_t nvec, const KrylovScalars* sc, int jac) {
  const int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
  if (i >= nvec) return;
#pragma unroll
  for (int s = 0; s < NS; ++s) {
    if (!sc->active[s]) continue;
    const int64_t o = s * V.stride + i;
    const T sv = bicg_s_value(V.r[o], V.v[o], static_cast<T>(sc->alpha[s]));
    V.s[o] = sv;
    if (jac) V.sh[o] = V.dinv[s][i] * sv;
  }
}

// t = A sh; partial sums of t . s, t . t (and of sh for the border row).  With FS (no
// preconditioner, sh = s) the kernel also forms s = r - alpha v itself: it stages s computed from
// r and v, the row-by-row path computes it where it reads it, and each row writes its own s.
template <typename VT, typename T, int NS, bool GEN, bool FS = false>
__global__ void __launch_bounds__(kBlock, (kWavesFor<T, NS, FS>)) k_bicg_t(Mat<VT> A, Vec<T> V, double* partials,
                                                                       const KrylovScalars* sc, int sys0) {
  __shared__ T lds[NS][kTileLdsH][kTileLdsW];
  __shared__ TileMeta meta;
  double acc[3 * NS];
#pragma unroll
  for (int a = 0; a < 3 * NS; ++a) acc[a] = 0.0;
  bool use[NS], any = false;
  double shn[NS];   // border unknowns (uniform)
#pragma unroll
  for (int s = 0; s < NS; ++s) {
    use[s] = sc->active[sys0 + s] != 0;
    any = any || use[s];
    shn[s] = A.border ? static_cast<double>(V.sh[s * V.stride + A.n]) : 0.0;
  }
  SValues<T> sa[NS];
#pragma unroll
  for (int s = 0; s < NS; ++s) sa[s] = SValues<T>{V.r + s * V.stride, V.v + s * V.stride, static_cast<T>(sc->alpha[sys0 + s])};
  auto emit = [&](int s, int64_t i, double y, T sv, T si) __attribute__((always_inline)) {
    if (A.border) y += shn[s];
    const T yt = static_cast<T>(y);
    V.t[s * V.stride + i] = yt;
    if constexpr (FS) V.s[s * V.stride + i] = sv;
    acc[3 * s] = fma(static_cast<double>(yt), static_cast<double>(sv), acc[3 * s]);
    acc[3 * s + 1] = fma(static_cast<double>(yt), static_cast<double>(yt), acc[3 * s + 1]);
    if (A.border) acc[3 * s + 2] += static_cast<double>(si);
  };
  auto slow = [&](int64_t i) __attribute__((always_inline)) {
#pragma unroll
    for (int s = 0; s < NS; ++s)
      if (use[s]) {
        if constexpr (FS) {
          const T si = sa[s][i];
          emit(s, i, row_dot_rows(A, s, i, sa[s]), si, si);
        } else {
          emit(s, i, row_dot_rows(A, s, i, V.sh + s * V.stride), V.s[s * V.stride + i], V.sh[s * V.stride + i]);
        }
      }
  };
  if (A.tv.tiles) {
    const T* xs[NS];
#pragma unroll
    for (int s = 0; s < NS; ++s) xs[s] = V.sh + s * V.stride;
    if (any)
      tile_walk(
          A.tv,
          [&](int64_t tk) __attribute__((always_inline)) {
            if constexpr (FS)
              tile_stage_fn<T, NS>(
                  A.tv, tk, [&](int s, int32_t node) __attribute__((always_inline)) { return sa[s][node]; }, lds,
                  meta, !GEN);
            else
              tile_stage<T, NS>(A.tv, tk, xs, lds, meta, !GEN);
            if constexpr (GEN) {
#pragma unroll 1
              for (int k = 0; k < kTileRowsPerWave; ++k) {
                const int64_t row = tile_row_id(A.tv, meta, k);
                if (row >= 0) slow(row);
              }
              return;
            }
            const int wave = static_cast<int>(threadIdx.x >> 6), lane = static_cast<int>(threadIdx.x & 63);
#pragma unroll 1
            for (int k = 0; k < kTileRowsPerWave; ++k) {
              const int64_t row = tile_row_id(A.tv, meta, k);
              if (row < 0) continue;
              const int ly = wave + k * (kBlock / 64);
              T sv[NS];
              if constexpr (!FS) {
#pragma unroll
                for (int s = 0; s < NS; ++s) sv[s] = V.s[s * V.stride + row];
              }
              double y[NS];
#pragma unroll
              for (int s = 0; s < NS; ++s) y[s] = disk_lds(A, s, lds[s], ly, lane);
              // (with FS the staged centre is this row's s)
#pragma unroll
              for (int s = 0; s < NS; ++s)
                if (use[s]) emit(s, row, y[s], FS ? lds[s][ly + 2][lane + 2] : sv[s], lds[s][ly + 2][lane + 2]);
            }
          },
          slow);
  } else {
    walk_rows(
        A, use,
        [&](int64_t i, const int32_t (&b)[5]) {
          double y[NS];
          T sv[NS], si[NS];
#pragma unroll
          for (int s = 0; s < NS; ++s) {
            if constexpr (FS) {
              sv[s] = si[s] = sa[s][i];
            } else {
              sv[s] = V.s[s * V.stride + i];
              si[s] = V.sh[s * V.stride + i];
            }
          }
#pragma unroll
          for (int s = 0; s < NS; ++s) {
            if constexpr (FS) y[s] = disk_dot(A, s, i, b, sa[s]);
            else y[s] = disk_dot(A, s, i, b, V.sh + s * V.stride);
          }
#pragma unroll
          for (int s = 0; s < NS; ++s)
            if (use[s]) emit(s, i, y[s], sv[s], si[s]);
        },
        slow);
  }
  block_sum_store<3 * NS>(acc, partials);
}

// omega = (t . s) / (t . t), with the border row t[n] = sum(sh)
template <typename T, int NS>
__global__ void k_fin_bicg_t(const double* partials, int64_t nb, int64_t n, int border, Vec<T> V,
                             KrylovScalars* sc, int sys0) {
  double tot[3 * NS];
  grid_sum<3 * NS>(partials, nb, tot);
  if (threadIdx.x != 0) return;
#pragma unroll
  for (int s = 0; s < NS; ++s) {
    const int q = sys0 + s;
    if (!sc->active[q]) continue;
    double ts = tot[3 * s], tt = tot[3 * s + 1];
    if (border) {
      const T yn = static_cast<T>(tot[3 * s + 2]);
      V.t[s * V.stride + n] = yn;
      ts += static_cast<double>(yn) * static_cast<double>(V.s[s * V.stride + n]);
      tt += static_cast<double>(yn) * static_cast<double>(yn);
    }
    sc->dot_b[q] = ts;
    sc->dot_c[q] = tt;
    // tt == 0 means s == 0: the half step already solved the system
    sc->omega[q] = tt > 0.0 ? ts / tt : 0.0;
  }
}

// x += alpha ph + omega sh; r = s - omega t; partial sums of rhat . r and r . r
template <typename T, int NS>
__global__ void k_bicg_x(Vec<T> V, int64_t nvec, double* partials, const KrylovScalars* sc) {
  double acc[2 * NS];
#pragma unroll
  for (int a = 0; a < 2 * NS; ++a) acc[a] = 0.0;
  const Span sp = block_span(nvec);
  for (int64_t i = sp.begin + threadIdx.x; i < sp.end; i += blockDim.x) {
#pragma unroll
    for (int s = 0; s < NS; ++s) {
      if (!sc->active[s]) continue;
      const int64_t o = s * V.stride + i;
      const T alpha = static_cast<T>(sc->alpha[s]), omega = static_cast<T>(sc->omega[s]);
      V.x[o] = V.x[o] + alpha * V.ph[o] + omega * V.sh[o];
      const T r = V.s[o] - omega * V.t[o];
      V.r[o] = r;
      acc[2 * s] += static_cast<double>(V.rhat[o]) * static_cast<double>(r);
      acc[2 * s + 1] += static_cast<double>(r) * static_cast<double>(r);
    }
  }
  block_sum_store<2 * NS>(acc, partials);
}

// rho' = rhat . r; stop at convergence or breakdown; beta = (rho'/rho)(alpha/omega)
template <int NS>
__global__ void k_fin_bicg_x(const double* partials, int64_t nb, KrylovScalars* sc) {
  double tot[2 * NS];
  grid_sum<2 * NS>(partials, nb, tot);
  if (threadIdx.x != 0) return;
#pragma unroll
  for (int s = 0; s < NS; ++s) {
    if (!sc->active[s]) continue;
    const double rho_new = tot[2 * s];
    const double rr = tot[2 * s + 1];
    sc->rr[s] = rr;
    sc->iters[s] += 1;
    if (!(rr > sc->stop2[s])) {       // converged (or not a number): stop before the next update
      sc->active[s] = 0;
      if (!isfinite(rr)) sc->breakdown[s] = 1;
      continue;
    }
    const double ratio = safe_div(rho_new, sc->rho[s], &sc->breakdown[s]);
    const double om = sc->omega[s];
    const double beta = (om != 0.0 && isfinite(ratio)) ? ratio * (sc->alpha[s] / om) : 0.0;
    if (om == 0.0 || !isfinite(beta) || fabs(beta) > 1e30) sc->breakdown[s] = 1;
    sc->beta[s] = isfinite(beta) ? beta : 0.0;
    sc->rho[s] = rho_new;
    if (sc->breakdown[s]) sc->active[s] = 0;
  }
}

// ---- BiCGStab with the x, r and p updates in one pass ---------------------------------------------
// For the unpreconditioned FP32 solves on tiles (the predictor: Jacobi folded into its matrices).
// Iteration k is three launches:
//   (E) both systems, in place: the update of iteration k-1, x += alpha p + omega s and
//       r = s - omega t (s = r - alpha v), then p = r + beta (p - omega v);
//   (V) v = A p with the partial sums of rhat . v (the two-system SpMV);
//   (T) per system, t = A s with s = r - alpha v formed where it is read, with the partial sums
//       of t . s, t . t, s . s, rhat . s and rhat . t.
// From (T)'s sums: omega = (t . s)/(t . t); |s - omega t|^2 = s . s - omega (t . s); and
// rhat . r_new = rhat . s - omega (rhat . t).  So beta is known before r_new is formed, and the
// update of x and r shares its pass with the update of p: per iteration and system 12 vectors
// move in the vector passes where the separate p and x passes move 15 (11 + 4), and s is never
// stored; two launches fewer.

// (E): the pending update (x, r) and, while the system iterates, p.
template <typename T, int NS>
__global__ void k_bicg_e(Vec<T> V, int64_t nvec, const KrylovScalars* sc) {
  static_assert(sizeof(T) == 4, "FP32 vectors");
  const int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
  if (i >= nvec) return;
#pragma unroll
  for (int q = 0; q < NS; ++q) {
    const bool pend = sc->pending[q] != 0, act = sc->active[q] != 0;
    if (!pend && !act) continue;
    const int64_t o = q * V.stride + i;
    T r = V.r[o];
    const T p = V.p[o], v = V.v[o];
    const T om = static_cast<T>(sc->omega[q]);
    if (pend) {
      const T al = static_cast<T>(sc->alpha[q]);
      const T sv = bicg_s_value(r, v, al);
      V.x[o] = fmaf(om, sv, fmaf(al, p, V.x[o]));
      r = fmaf(-om, V.t[o], sv);
      V.r[o] = r;
    }
    if (act) V.p[o] = fmaf(static_cast<T>(sc->beta[q]), fmaf(-om, v, p), r);
  }
}

// (T) for one system q: t = A s, s = r - alpha v formed where it is read; partial sums of t . s,
// t . t, s . s, rhat . s and rhat . t, at partials[10 b + 5 q + a] (the two systems' launches
// interleave their sums so that one finishing pass adds both).  The rows' rhat are loaded before
// their products.  The tiles are walked pipelined (96 VGPRs, 5 waves per SIMD): 66.6 -> 57.2 us
// per launch at h = 1/128 against one tile at a time (79 VGPRs, 6 waves).
template <typename VT, bool GEN>
__global__ void __launch_bounds__(kBlock, GEN ? 1 : 5) k_bicg_ts(Mat<VT> A, Vec<float> V, double* partials,
                                                                 const KrylovScalars* sc, int q) {
  __shared__ float lds[1][kTileLdsH][kTileLdsW];
  __shared__ TileMeta meta2[2];
  TileMeta& meta = meta2[0];
  double acc[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
  const bool act = sc->active[q] != 0;
  const SValues<float> sa{V.r, V.v, static_cast<float>(sc->alpha[q])};
  auto emit = [&](int64_t i, double y, float sv, float rh) __attribute__((always_inline)) {
    const float yt = static_cast<float>(y);
    V.t[i] = yt;
    const double td = static_cast<double>(yt), sd = static_cast<double>(sv), rd = static_cast<double>(rh);
    acc[0] = fma(td, sd, acc[0]);
    acc[1] = fma(td, td, acc[1]);
    acc[2] = fma(sd, sd, acc[2]);
    acc[3] = fma(rd, sd, acc[3]);
    acc[4] = fma(rd, td, acc[4]);
  };
  auto slow = [&](int64_t i) __attribute__((always_inline)) {
    const float rh = V.rhat[i];
    emit(i, row_dot_rows(A, 0, i, sa), sa[i], rh);
  };
  if (act) {
    if constexpr (GEN) {
      tile_walk(
          A.tv,
          [&](int64_t tk) __attribute__((always_inline)) {
            tile_stage_fn<float, 1>(
                A.tv, tk, [&](int, int32_t node) __attribute__((always_inline)) { return sa[node]; }, lds, meta, false);
#pragma unroll 1
            for (int k = 0; k < kTileRowsPerWave; ++k) {
              const int64_t row = tile_row_id(A.tv, meta, k);
              if (row >= 0) slow(row);
            }
          },
          slow);
    } else {
      // pipelined: r and v of the next tile in flight while this one is computed; s is formed
      // from them when the tile is staged (the bits of sa[node])
      const int wave = static_cast<int>(threadIdx.x >> 6), lane = static_cast<int>(threadIdx.x & 63);
      int64_t rows[kTileRowsPerWave];
      float rh[kTileRowsPerWave];
      tile_walk_pp<float, 1, float2>(
          A.tv, lds, meta2,
          [&](int, int32_t node) __attribute__((always_inline)) { return make_float2(V.r[node], V.v[node]); },
          [&](int, float2 rv) __attribute__((always_inline)) { return bicg_s_value(rv.x, rv.y, sa.alpha); },
          [&](int64_t, const TileMeta& mm) __attribute__((always_inline)) {
#pragma unroll
            for (int k = 0; k < kTileRowsPerWave; ++k) {
              rows[k] = tile_row_id(A.tv, mm, k);
              rh[k] = rows[k] >= 0 ? V.rhat[rows[k]] : 0.0f;
            }
          },
          [&](int64_t, const TileMeta&) __attribute__((always_inline)) {
#pragma unroll 1
            for (int k = 0; k < kTileRowsPerWave; ++k) {
              if (rows[k] < 0) continue;
              const int ly = wave + k * (kBlock / 64);
              emit(rows[k], disk_lds(A, 0, lds[0], ly, lane), lds[0][ly + 2][lane + 2], rh[k]);
            }
          },
          slow);
    }
  }
  block_sum_store<5>(acc, partials + 5 * q, 10);
}

// After (T) of both systems: omega, the new |r|^2 and rhat . r from the sums; the iteration's
// update becomes pending (the next (E) applies it); stop at convergence or breakdown, else
// beta = (rho'/rho)(alpha/omega).
__global__ void k_fin_bicg_ts(const double* partials, int64_t nb, KrylovScalars* sc) {
  double all[10];
  grid_sum<10>(partials, nb, all);
  if (threadIdx.x != 0) return;
  for (int q = 0; q < 2; ++q) {
    const double* tot = all + 5 * q;
    if (sc->active[q]) {
      const double ts = tot[0], tt = tot[1], ss = tot[2], rs = tot[3], rt = tot[4];
      sc->dot_b[q] = ts;
      sc->dot_c[q] = tt;
      sc->dot_d[q] = ss;
      sc->dot_e[q] = rt;
      // tt == 0 means s == 0: the half step already solved the system
      const double om = tt > 0.0 ? ts / tt : 0.0;
      sc->omega[q] = om;
      sc->pending[q] = 1;
      sc->iters[q] += 1;
      double rr = ss - om * ts;   // |s - omega t|^2 (a NaN stays a NaN)
      if (rr < 0.0) rr = 0.0;
      sc->rr[q] = rr;
      if (!(rr > sc->stop2[q])) {   // converged (or not a number): the pending update finishes it
        sc->active[q] = 0;
        if (!isfinite(rr)) sc->breakdown[q] = 1;
      } else {
        const double rho_new = rs - om * rt;
        const double ratio = safe_div(rho_new, sc->rho[q], &sc->breakdown[q]);
        const double beta = (om != 0.0 && isfinite(ratio)) ? ratio * (sc->alpha[q] / om) : 0.0;
        if (om == 0.0 || !isfinite(beta) || fabs(beta) > 1e30) sc->breakdown[q] = 1;
        sc->beta[q] = isfinite(beta) ? beta : 0.0;
        sc->rho[q] = rho_new;
        if (sc->breakdown[q]) sc->active[q] = 0;
      }
    }
  }
}

// ---- CG -----------------------------------------------------------------------------------------------
// p = z with z = D^-1 r (Jacobi) or given in V.s; partial sums of r . z
template <typename T, int NS>
__global__ void k_cg_init(Vec<T> V, int64_t nvec, double* partials, int jac) {
  double acc[NS];
#pragma unroll
  for (int a = 0; a < NS; ++a) acc[a] = 0.0;
  const Span sp = block_span(nvec);
  for (int64_t i = sp.begin + threadIdx.x; i < sp.end; i += blockDim.x) {
#pragma unroll
    for (int s = 0; s < NS; ++s) {
      const int64_t o = s * V.stride + i;
      const T z = jac ? V.dinv[s][i] * V.r[o] : V.s[o];
      V.p[o] = z;
      acc[s] += static_cast<double>(V.r[o]) * static_cast<double>(z);
    }
  }
  block_sum_store<NS>(acc, partials);
}

template <int NS>
__global__ void k_fin_cg_init(const double* partials, int64_t nb, KrylovScalars* sc) {
  double tot[NS];
  grid_sum<NS>(partials, nb, tot);
  if (threadIdx.x != 0) return;
#pragma unroll
  for (int s = 0; s < NS; ++s) {
    sc->rho[s] = tot[s];
    sc->breakdown[s] = 0;
  }
}

// v = A p; partial sums of p . v
template <typename VT, typename T, int NS, bool GEN>
__global__ void __launch_bounds__(kBlock) k_cg_q(Mat<VT> A, Vec<T> V, double* partials, const KrylovScalars* sc) {
  __shared__ T lds[NS][kTileLdsH][kTileLdsW];
  __shared__ TileMeta meta;
  double acc[NS];
#pragma unroll
  for (int a = 0; a < NS; ++a) acc[a] = 0.0;
  bool use[NS], any = false;
#pragma unroll
  for (int s = 0; s < NS; ++s) {
    use[s] = sc->active[s] != 0;
    any = any || use[s];
  }
  auto emit = [&](int s, int64_t i, double y, T pc) __attribute__((always_inline)) {
    const T yt = static_cast<T>(y);
    V.v[s * V.stride + i] = yt;
    acc[s] = fma(static_cast<double>(pc), static_cast<double>(yt), acc[s]);
  };
  auto slow = [&](int64_t i) __attribute__((always_inline)) {
#pragma unroll
    for (int s = 0; s < NS; ++s)
      if (use[s]) emit(s, i, row_dot_rows(A, s, i, V.p + s * V.stride), V.p[s * V.stride + i]);
  };
  if (A.tv.tiles) {
    const T* xs[NS];
#pragma unroll
    for (int s = 0; s < NS; ++s) xs[s] = V.p + s * V.stride;
    if (any)
      tile_walk(
          A.tv,
          [&](int64_t tk) __attribute__((always_inline)) {
            tile_stage<T, NS>(A.tv, tk, xs, lds, meta, !GEN);
            if constexpr (GEN) {
#pragma unroll 1
              for (int k = 0; k < kTileRowsPerWave; ++k) {
                const int64_t row = tile_row_id(A.tv, meta, k);
                if (row >= 0) slow(row);
              }
              return;
            }
            const int wave = static_cast<int>(threadIdx.x >> 6), lane = static_cast<int>(threadIdx.x & 63);
#pragma unroll 1
            for (int k = 0; k < kTileRowsPerWave; ++k) {
              const int64_t row = tile_row_id(A.tv, meta, k);
              if (row < 0) continue;
              const int ly = wave + k * (kBlock / 64);
              double y[NS];
#pragma unroll
              for (int s = 0; s < NS; ++s) y[s] = disk_lds(A, s, lds[s], ly, lane);
#pragma unroll
              for (int s = 0; s < NS; ++s) if (use[s]) emit(s, row, y[s], lds[s][ly + 2][lane + 2]);
            }
          },
          slow);
  } else {
    walk_rows(
        A, use,
        [&](int64_t i, const int32_t (&b)[5]) {
          double y[NS];
          T pc[NS];
#pragma unroll
          for (int s = 0; s < NS; ++s) pc[s] = V.p[s * V.stride + i];
#pragma unroll
          for (int s = 0; s < NS; ++s) y[s] = disk_dot(A, s, i, b, V.p + s * V.stride);
#pragma unroll
          for (int s = 0; s < NS; ++s)
            if (use[s]) emit(s, i, y[s], pc[s]);
        },
        slow);
  }
  block_sum_store<NS>(acc, partials);
}

// alpha = rho / (p . v)
template <int NS>
__global__ void k_fin_cg_q(const double* partials, int64_t nb, KrylovScalars* sc) {
  double tot[NS];
  grid_sum<NS>(partials, nb, tot);
  if (threadIdx.x != 0) return;
#pragma unroll
  for (int s = 0; s < NS; ++s) {
    if (!sc->active[s]) continue;
    sc->dot_a[s] = tot[s];
    sc->alpha[s] = safe_div(sc->rho[s], tot[s], &sc->breakdown[s]);
    if (sc->breakdown[s]) sc->active[s] = 0;
  }
}

// x += alpha p; r -= alpha v; partial sums of r . D^-1 r (Jacobi) and r . r
template <typename T, int NS>
__global__ void k_cg_x(Vec<T> V, int64_t nvec, double* partials, const KrylovScalars* sc, int jac) {
  double acc[2 * NS];
#pragma unroll
  for (int a = 0; a < 2 * NS; ++a) acc[a] = 0.0;
  const Span sp = block_span(nvec);
  for (int64_t i = sp.begin + threadIdx.x; i < sp.end; i += blockDim.x) {
#pragma unroll
    for (int s = 0; s < NS; ++s) {
      if (!sc->active[s]) continue;
      const int64_t o = s * V.stride + i;
      const T alpha = static_cast<T>(sc->alpha[s]);
      V.x[o] = V.x[o] + alpha * V.p[o];
      const T r = V.r[o] - alpha * V.v[o];
      V.r[o] = r;
      if (jac) acc[2 * s] += static_cast<double>(r) * static_cast<double>(V.dinv[s][i] * r);
      acc[2 * s + 1] += static_cast<double>(r) * static_cast<double>(r);
    }
  }
  block_sum_store<2 * NS>(acc, partials);
}

// stop at convergence; with Jacobi also beta = rho'/rho
template <int NS>
__global__ void k_fin_cg_x(const double* partials, int64_t nb, KrylovScalars* sc, int jac) {
  double tot[2 * NS];
  grid_sum<2 * NS>(partials, nb, tot);
  if (threadIdx.x != 0) return;
#pragma unroll
  for (int s = 0; s < NS; ++s) {
    if (!sc->active[s]) continue;
    const double rr = tot[2 * s + 1];
    sc->rr[s] = rr;
    sc->iters[s] += 1;
    if (!(rr > sc->stop2[s])) {
      sc->active[s] = 0;
      if (!isfinite(rr)) sc->breakdown[s] = 1;
      continue;
    }
    if (jac) {
      sc->beta[s] = safe_div(tot[2 * s], sc->rho[s], &sc->breakdown[s]);
      sc->rho[s] = tot[2 * s];
      if (sc->breakdown[s]) sc->active[s] = 0;
    }
  }
}

// partial sums of r . z with z = M^-1 r in V.s
template <typename T, int NS>
__global__ void k_cg_rz(Vec<T> V, int64_t nvec, double* partials, const KrylovScalars* sc) {
  double acc[NS];
#pragma unroll
  for (int a = 0; a < NS; ++a) acc[a] = 0.0;
  const Span sp = block_span(nvec);
  for (int64_t i = sp.begin + threadIdx.x; i < sp.end; i += blockDim.x) {
#pragma unroll
    for (int s = 0; s < NS; ++s) {
      if (!sc->active[s]) continue;
      const int64_t o = s * V.stride + i;
      acc[s] += static_cast<double>(V.r[o]) * static_cast<double>(V.s[o]);
    }
  }
  block_sum_store<NS>(acc, partials);
}

// beta = rho'/rho
template <int NS>
__global__ void k_fin_cg_rz(const double* partials, int64_t nb, KrylovScalars* sc) {
  double tot[NS];
  grid_sum<NS>(partials, nb, tot);
  if (threadIdx.x != 0) return;
#pragma unroll
  for (int s = 0; s < NS; ++s) {
    if (!sc->active[s]) continue;
    sc->beta[s] = safe_div(tot[s], sc->rho[s], &sc->breakdown[s]);
    sc->rho[s] = tot[s];
    if (sc->breakdown[s]) sc->active[s] = 0;
  }
}

// p = z + beta p with z = D^-1 r (Jacobi) or z in V.s
template <typename T, int NS>
__global__ void k_cg_p(Vec<T> V, int64_t nvec, const KrylovScalars* sc, int jac) {
  const int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
  if (i >= nvec) return;
#pragma unroll
  for (int s = 0; s < NS; ++s) {
    if (!sc->active[s]) continue;
    const int64_t o = s * V.stride + i;
    const T z = jac ? V.dinv[s][i] * V.r[o] : V.s[o];
    V.p[o] = z + static_cast<T>(sc->beta[s]) * V.p[o];
  }
}

// ---- small vector kernels ------------------------------------------------------------------------
template <typename A, typename B>
__global__ void k_copy(int64_t m, const A* a, B* b) {
  const int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
  if (i < m) b[i] = static_cast<B>(a[i]);
}

template <typename T>
__global__ void k_fill(int64_t m, T* a, T v) {
  const int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
  if (i < m) a[i] = v;
}

__global__ void k_add_f32(int64_t m, double* x, const float* d) {
  const int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
  if (i < m) x[i] += static_cast<double>(d[i]);
}

// x += D^-1 y for two systems of `stride` entries (rows below n; D^-1 of system s in dinv_s)
__global__ void k_add_scaled(int64_t m, int64_t stride, int64_t n, double* x, const float* y, const double* dinv0,
                             const double* dinv1) {
  const int64_t o = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
  if (o >= m) return;
  const int64_t i = o % stride;
  if (i < n) x[o] += (o < stride ? dinv0 : dinv1)[i] * static_cast<double>(y[o]);
}

// x = 2 a - b (linear extrapolation from the last two values)
__global__ void k_extrapolate(int64_t n, const double* a, const double* b, double* x) {
  const int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
  if (i < n) x[i] = 2.0 * a[i] - b[i];
}

// x = 3 (a - b) + c (quadratic extrapolation from the last three values a, b, c, newest first)
__global__ void k_extrapolate3(int64_t n, const double* a, const double* b, const double* c, double* x) {
  const int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
  if (i < n) x[i] = 3.0 * (a[i] - b[i]) + c[i];
}

// partial sums of a[0..m)
__global__ void k_sum(int64_t m, const double* a, double* partials) {
  double acc[1] = {0.0};
  const Span sp = block_span(m);
  for (int64_t i = sp.begin + threadIdx.x; i < sp.end; i += blockDim.x) acc[0] += a[i];
  block_sum_store<1>(acc, partials);
}

__global__ void k_fin_mean(const double* partials, int64_t nb, int64_t m, KrylovScalars* sc) {
  double tot[1];
  grid_sum<1>(partials, nb, tot);
  if (threadIdx.x == 0) sc->mean = tot[0] / static_cast<double>(m);
}

__global__ void k_sub_mean(int64_t m, const double* a, double* out, const KrylovScalars* sc) {
  const int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
  if (i < m) out[i] = a[i] - sc->mean;
}

// ---- host side -----------------------------------------------------------------------------------

struct Timer {
  Ctx* c;
  bool on;
  std::pair<hipEvent_t, hipEvent_t> ev{};
  Timer(Ctx* cc, bool enable) : c(cc), on(enable && cc->timing.enabled) {
    if (!on) return;
    if (c->timing.pool.empty()) {
      hipEvent_t a, b;
      if (hipEventCreateWithFlags(&a, hipEventDisableSystemFence) != hipSuccess || hipEventCreateWithFlags(&b, hipEventDisableSystemFence) != hipSuccess) {
        on = false;
        return;
      }
      ev = {a, b};
    } else {
      ev = c->timing.pool.back();
      c->timing.pool.pop_back();
    }
    (void)hipEventRecord(ev.first, c->stream);
  }
  ~Timer() {
    if (!on) return;
    (void)hipEventRecord(ev.second, c->stream);
    c->timing.pending.push_back(ev);
  }
};

// Add the durations of timed launches [first, first + keep) of the pending list and
// recycle every pending event pair.
void harvest_timing(Ctx* c, size_t first = 0, size_t keep = SIZE_MAX) {
  for (size_t k = 0; k < c->timing.pending.size(); ++k) {
    auto& e = c->timing.pending[k];
    if (k >= first && k - first < keep) {
      float ms = 0.0f;
      if (hipEventElapsedTime(&ms, e.first, e.second) == hipSuccess) {
        c->timing.total_ms += ms;
        c->timing.count += 1;
      }
    }
    c->timing.pool.push_back(e);
  }
  c->timing.pending.clear();
}

int sync_scalars(Ctx* c) {
  VIP_HIP_TRY(c, hipMemcpyAsync(c->sc_host, c->sc, sizeof(KrylovScalars), hipMemcpyDeviceToHost,
                                c->stream));
  VIP_HIP_TRY(c, hipStreamSynchronize(c->stream));
  return VIP_OK;
}

int ensure_ws(Ctx* c, int64_t len64, int64_t len32) {
  if (c->ws_len < len64 || c->ws32_len < len32) VIP_HIP_TRY(c, hipStreamSynchronize(c->stream));
  if (c->ws_len < len64) {
    dfree(c->ws);
    VIP_TRY(dalloc(c, &c->ws, len64));
    c->ws_len = len64;
  }
  if (c->ws32_len < len32) {
    dfree(c->ws32);
    VIP_TRY(dalloc(c, &c->ws32, len32));
    c->ws32_len = len32;
  }
  return VIP_OK;
}

enum Method { kBiCGStab = 0, kCG = 1 };

// Tell the kernels which systems iterate and where each one stops.
// (One small kernel with the values as arguments: copies from host memory would each take a
// runtime transfer.)
__global__ void k_set_active(KrylovScalars* sc, int a0, int a1, double s0, double s1) {
  if (threadIdx.x == 0) {
    sc->iters[0] = 0;
    sc->iters[1] = 0;
    sc->active[0] = a0;
    sc->active[1] = a1;
    sc->stop2[0] = s0;
    sc->stop2[1] = s1;
  }
}

int set_active(Ctx* c, const int* act, const double* stop2) {
  k_set_active<<<1, 64, 0, c->stream>>>(c->sc, act[0], act[1], stop2[0], stop2[1]);
  VIP_HIP_TRY(c, hipGetLastError());
  return VIP_OK;
}

// Iterate until |r| <= tol |b| (recurrence residual) for every system, or maxit.
// On entry V.r holds the initial residual and sc->rr/bb its norms.  A system
// stops on the device as soon as it converges or breaks down; *bad reports a
// non-finite residual (the caller then discards the iterate).
//
// Iterations run in batches between host checks; every launch after the device has stopped
// returns at once but still costs a launch, so with a `hint` (the iterations the previous
// solve of the same kind took) the first check comes one iteration before that count and
// later ones every two iterations; *hint is updated on return.
// System q of a two-system matrix and of its vectors, as a one-system view (the kernels then
// read system 0's fields); the scalars stay shared and are indexed from q by the kernel.
template <typename VT>
Mat<VT> mat_sys(const Mat<VT>& A, int q) {
  Mat<VT> B = A;
  B.val[0] = A.val[q];
  B.rsum[0] = A.rsum[q];
  B.cpix[0] = A.cpix[q];
  B.sbase[0] = A.sbase[q];
  for (int k = 0; k < kMaxTaps; ++k) B.w[0][k] = A.w[q][k];
  B.crsum[0] = A.crsum[q];
  return B;
}

template <typename T>
Vec<T> vec_sys(const Vec<T>& V, int q) {
  const int64_t o = q * V.stride;
  auto at = [o](T* p) { return p ? p + o : p; };
  Vec<T> W = V;
  W.x = at(V.x);
  W.r = at(V.r);
  W.rhat = at(V.rhat);
  W.p = at(V.p);
  W.ph = at(V.ph);
  W.v = at(V.v);
  W.s = at(V.s);
  W.sh = at(V.sh);
  W.t = at(V.t);
  W.dinv[0] = V.dinv[q];
  return W;
}

template <typename VT, typename T, int NS>
int iterate(Ctx* c, Method m, const Mat<VT>& A, Vec<T>& V, double tol, int maxit, int* iters,
            bool time_spmv, const double* bnorm2, bool amg = false, bool* bad = nullptr,
            int* hint = nullptr, bool zero_x = false) {
  VIP_TRY(check_mat(c, A, NS));
  const int64_t nvec = A.n + A.border;
  const int64_t g_vec = grid_for(nvec);
  const int64_t r_rows = spmv_grid(A), r_vec = red_grid(nvec);
  // Jacobi vectors ph = D^-1 p, sh = D^-1 s unless multigrid makes them or there is no D^-1
  // (then ph and sh are p and s)
  const int jac = amg || !V.dinv[0] ? 0 : 1;
  // the unpreconditioned two-system FP32 solve on tiles (the predictor) folds its vector passes
  // into the two products
  constexpr bool kFuseAll = NS == 2 && sizeof(T) == 4 && sizeof(VT) == 4;
  const bool fused = kFuseAll && m == kBiCGStab && !amg && !jac && A.tv.tiles && V.sh == V.s && V.ph == V.p &&
                     !A.border && !c->no_fuse;
  VIP_TRY(ensure_partials(c, std::max(r_rows, r_vec), (fused ? 5 : 3) * NS));
  if (c->debug)
    std::fprintf(stderr, "[vip] iterate n %lld border %d tol %.3e rr0 %.3e bb %.3e\n",
                 static_cast<long long>(A.n), A.border, tol, c->sc_host->rr[0], bnorm2[0]);
  int act[2] = {1, NS > 1 ? 1 : 0};
  double stop2[2] = {0.0, 0.0};
  for (int s = 0; s < NS; ++s) {
    stop2[s] = tol * tol * bnorm2[s];
    if (c->sc_host->rr[s] <= stop2[s]) act[s] = 0;
  }
  if (bad) *bad = false;
  harvest_timing(c, 0, 0);   // nothing pending belongs to this call
  for (int k = 0; k < kTimePredRhs; ++k) harvest_kind(c->ktime[k], 0, 0);
  c->vcycle = 0;
  const bool tpred = NS == 2;   // the predictor's two-system solve
  VIP_TRY(set_active(c, act, stop2));
  double* part = c->partials;
  KrylovScalars* sc = c->sc;
  hipStream_t st = c->stream;
  // zero_x: the iterate starts from 0 (set here, with the other start vectors)
  if (m == kBiCGStab) {
    k_bicg_init<T, NS><<<g_vec, kBlock, 0, st>>>(V, nvec, sc, zero_x ? 1 : 0);
  } else {
    if (zero_x)
      for (int s = 0; s < NS; ++s) k_fill<T><<<g_vec, kBlock, 0, st>>>(nvec, V.x + s * V.stride, T(0));
    if constexpr (NS == 1) {
      if (amg) VIP_TRY(amg_apply<T>(c, V.r, V.s, false, true));
    }
    k_cg_init<T, NS><<<r_vec, kBlock, 0, st>>>(V, nvec, part, amg ? 0 : 1);
    k_fin_cg_init<NS><<<1, kBlock, 0, st>>>(part, r_vec, sc);
  }
  int it = 0;
  const int every = std::max(1, c->opt.check_every);
  int next = (hint && *hint > 0) ? std::max(1, std::min(every, *hint - 1)) : every;
  while ((act[0] || act[1]) && it < maxit) {
    const int batch = std::min(next, maxit - it);
    if (hint) next = std::min(every, 2);
    for (int b = 0; b < batch; ++b) {
      if (fused) {
        if constexpr (kFuseAll) {
          {
            KTimer kt(c, c->ktime[kTimePredX], tpred);
            k_bicg_e<T, NS><<<g_vec, kBlock, 0, st>>>(V, nvec, sc);
          }
          {
            // one launch per system: the single-system SpMV runs 8 waves per SIMD where the
            // two-system one runs 4 (the block sums interleave, so the bits are the same)
            Timer tm(c, time_spmv);
            KTimer kt(c, c->ktime[kTimePredV], tpred);
            for (int q = 0; q < NS; ++q) {
              if (A.tile_general)
                k_bicg_v<VT, T, 1, true><<<r_rows, kBlock, 0, st>>>(mat_sys(A, q), vec_sys(V, q), part, sc, q, 2 * NS);
              else
                k_bicg_v<VT, T, 1, false><<<r_rows, kBlock, 0, st>>>(mat_sys(A, q), vec_sys(V, q), part, sc, q, 2 * NS);
            }
          }
          k_fin_bicg_v<T, NS><<<1, kBlock, 0, st>>>(part, r_rows, A.n, A.border, V, sc);
          for (int q = 0; q < NS; ++q) {
            const Mat<VT> Aq = mat_sys(A, q);
            KTimer kt(c, c->ktime[kTimePredT], tpred);
            if (A.tile_general) k_bicg_ts<VT, true><<<r_rows, kBlock, 0, st>>>(Aq, vec_sys(V, q), part, sc, q);
            else k_bicg_ts<VT, false><<<r_rows, kBlock, 0, st>>>(Aq, vec_sys(V, q), part, sc, q);
          }
          k_fin_bicg_ts<<<1, kBlock, 0, st>>>(part, r_rows, sc);
        }
      } else if (m == kBiCGStab) {
        k_bicg_p<T, NS><<<g_vec, kBlock, 0, st>>>(V, nvec, sc, jac);
        if constexpr (NS == 1) {
          if (amg) VIP_TRY(amg_apply<T>(c, V.p, V.ph, A.border != 0, c->amg_pre_fine != 0));
        }
        {
          Timer tm(c, time_spmv);
          KTimer kt(c, c->ktime[kTimePredV], tpred);
          if (A.tile_general) k_bicg_v<VT, T, NS, true><<<r_rows, kBlock, 0, st>>>(A, V, part, sc);
          else k_bicg_v<VT, T, NS, false><<<r_rows, kBlock, 0, st>>>(A, V, part, sc);
        }
        k_fin_bicg_v<T, NS><<<1, kBlock, 0, st>>>(part, r_rows, A.n, A.border, V, sc);
        // the unpreconditioned two-system FP32 solve (the predictor) forms s inside the t kernel
        constexpr bool kFuseS = NS == 2 && sizeof(T) == 4 && sizeof(VT) == 4;
        const bool fuse_s = kFuseS && !amg && !jac && A.tv.tiles && V.sh == V.s;
        if (!fuse_s) k_bicg_s<T, NS><<<g_vec, kBlock, 0, st>>>(V, nvec, sc, jac);
        if constexpr (NS == 1) {
          if (amg) VIP_TRY(amg_apply<T>(c, V.s, V.sh, A.border != 0, c->amg_pre_fine != 0));
        }
        if constexpr (kFuseS) {
          if (fuse_s) {
            // one launch per system: the one-system kernel runs 6 waves per SIMD, the two-system
            // one 4 (126 VGPRs); each system's sums land in a partial block of their own and
            // are reduced in the same order as in the two-system launch
            for (int q = 0; q < NS; ++q) {
              const Mat<VT> Aq = mat_sys(A, q);
              const Vec<T> Vq = vec_sys(V, q);
              double* pq = part + q * 3 * r_rows;
              KTimer kt(c, c->ktime[kTimePredT], tpred);
              if (A.tile_general) k_bicg_t<VT, T, 1, true, true><<<r_rows, kBlock, 0, st>>>(Aq, Vq, pq, sc, q);
              else k_bicg_t<VT, T, 1, false, true><<<r_rows, kBlock, 0, st>>>(Aq, Vq, pq, sc, q);
            }
            for (int q = 0; q < NS; ++q)
              k_fin_bicg_t<T, 1><<<1, kBlock, 0, st>>>(part + q * 3 * r_rows, r_rows, A.n, A.border,
                                                       vec_sys(V, q), sc, q);
          }
        }
        if (!fuse_s) {
          if (A.tile_general) k_bicg_t<VT, T, NS, true><<<r_rows, kBlock, 0, st>>>(A, V, part, sc, 0);
          else k_bicg_t<VT, T, NS, false><<<r_rows, kBlock, 0, st>>>(A, V, part, sc, 0);
          k_fin_bicg_t<T, NS><<<1, kBlock, 0, st>>>(part, r_rows, A.n, A.border, V, sc, 0);
        }
        {
          KTimer kt(c, c->ktime[kTimePredX], tpred);
          k_bicg_x<T, NS><<<r_vec, kBlock, 0, st>>>(V, nvec, part, sc);
        }
        k_fin_bicg_x<NS><<<1, kBlock, 0, st>>>(part, r_vec, sc);
      } else {
        {
          Timer tm(c, time_spmv);
          if (A.tile_general) k_cg_q<VT, T, NS, true><<<r_rows, kBlock, 0, st>>>(A, V, part, sc);
          else k_cg_q<VT, T, NS, false><<<r_rows, kBlock, 0, st>>>(A, V, part, sc);
        }
        k_fin_cg_q<NS><<<1, kBlock, 0, st>>>(part, r_rows, sc);
        k_cg_x<T, NS><<<r_vec, kBlock, 0, st>>>(V, nvec, part, sc, amg ? 0 : 1);
        k_fin_cg_x<NS><<<1, kBlock, 0, st>>>(part, r_vec, sc, amg ? 0 : 1);
        if constexpr (NS == 1) {
          if (amg) {
            VIP_TRY(amg_apply<T>(c, V.r, V.s, false, true));
            k_cg_rz<T, NS><<<r_vec, kBlock, 0, st>>>(V, nvec, part, sc);
            k_fin_cg_rz<NS><<<1, kBlock, 0, st>>>(part, r_vec, sc);
          }
        }
        k_cg_p<T, NS><<<g_vec, kBlock, 0, st>>>(V, nvec, sc, amg ? 0 : 1);
      }
    }
    it += batch;
    VIP_HIP_TRY(c, hipGetLastError());
    VIP_TRY(sync_scalars(c));
    for (int s = 0; s < NS; ++s) {
      if (!act[s]) continue;
      if (!std::isfinite(c->sc_host->rr[s]) && bad) *bad = true;
      act[s] = c->sc_host->active[s];
    }
    if (c->debug) {
      const KrylovScalars& h = *c->sc_host;
      std::fprintf(stderr, "[vip] %s%s batch to %d: it %d rr %.3e stop2 %.3e rho %.3e alpha %.3e omega %.3e "
                   "beta %.3e brk %d act %d\n", m == kCG ? "cg" : "bicgstab", amg ? "+amg" : "", it,
                   h.iters[0], h.rr[0], h.stop2[0], h.rho[0], h.alpha[0], h.omega[0], h.beta[0],
                   h.breakdown[0], h.active[0]);
    }
  }
  if constexpr (kFuseAll) {
    if (fused) {
      // the update the last iteration left pending (a system that iterates no more forms no p)
      k_bicg_e<T, NS><<<g_vec, kBlock, 0, st>>>(V, nvec, sc);
      VIP_HIP_TRY(c, hipGetLastError());
    }
  }
  *iters = 0;
  for (int s = 0; s < NS; ++s) *iters = std::max(*iters, c->sc_host->iters[s]);
  if (hint) *hint = *iters;
  // one timed SpMV per iteration: launches after the device stopped the solve exit at once
  // and are not counted
  harvest_timing(c, 0, static_cast<size_t>(*iters));
  const size_t its = static_cast<size_t>(*iters);
  harvest_kind(c->ktime[kTimePredV], 0, its);
  harvest_kind(c->ktime[kTimePredT], 0, its * NS);   // the t launches that ran are one per system
  harvest_kind(c->ktime[kTimePredX], 0, its);
  // V-cycles of the iterations the device performed: two per BiCGStab iteration, one per CG
  // iteration plus the one before the first
  harvest_kind(c->ktime[kTimeSweep0], 0, SIZE_MAX,
               static_cast<int>(m == kBiCGStab ? 2 * its : its + 1));
  harvest_kind(c->ktime[kTimePredRhs], 0, SIZE_MAX);   // launched before this solve, complete now
  return VIP_OK;
}

template <typename VT, typename XT, typename RT, int NS>
int residual(Ctx* c, const Mat<VT>& A, const XT* x, const double* b, RT* r, int64_t stride) {
  VIP_TRY(check_mat(c, A, NS));
  const int64_t g = spmv_grid(A);
  VIP_TRY(ensure_partials(c, g, 3 * NS));
  if (A.tile_general) k_residual<VT, XT, RT, NS, true><<<g, kBlock, 0, c->stream>>>(A, x, b, r, stride, c->partials);
  else k_residual<VT, XT, RT, NS, false><<<g, kBlock, 0, c->stream>>>(A, x, b, r, stride, c->partials);
  k_fin_residual<RT, NS><<<1, kBlock, 0, c->stream>>>(c->partials, g, A.n, A.border, b, r, stride, c->sc);
  VIP_HIP_TRY(c, hipGetLastError());
  return sync_scalars(c);
}

template <typename T>
Vec<T> make_vec(T* base, int64_t stride, int ns, T* x) {
  // 8 work vectors per system after x: r rhat p ph v s sh t
  Vec<T> V{};
  V.stride = stride;
  const int64_t blk = stride * ns;
  V.x = x;
  V.r = base + 0 * blk;
  V.rhat = base + 1 * blk;
  V.p = base + 2 * blk;
  V.ph = base + 3 * blk;
  V.v = base + 4 * blk;
  V.s = base + 5 * blk;
  V.sh = base + 6 * blk;
  V.t = base + 7 * blk;
  return V;
}

// a residual in an error message: 3 significant digits, exponent form
std::string sci(double v) {
  char buf[32];
  std::snprintf(buf, sizeof buf, "%.3e", v);
  return buf;
}

Method choose_method(Ctx* c) {
  if (c->opt.krylov == VIP_K_PCG) return kCG;
  if (c->opt.krylov == VIP_K_BICGSTAB) return kBiCGStab;
  return c->symmetric ? kCG : kBiCGStab;
}

}  // namespace

KTimer::KTimer(Ctx* cc, Timing& t, bool enable, int tg) : c(cc), T(&t), on(enable && t.enabled), tag(tg) {
  if (!on) return;
  if (T->pool.empty()) {
    hipEvent_t a, b;
    if (hipEventCreateWithFlags(&a, hipEventDisableSystemFence) != hipSuccess || hipEventCreateWithFlags(&b, hipEventDisableSystemFence) != hipSuccess) {
      on = false;
      return;
    }
    ev = {a, b};
  } else {
    ev = T->pool.back();
    T->pool.pop_back();
  }
  (void)hipEventRecord(ev.first, c->stream);
}

KTimer::~KTimer() {
  if (!on) return;
  (void)hipEventRecord(ev.second, c->stream);
  T->pending.push_back(ev);
  T->tags.push_back(tag);
}

void harvest_kind(Timing& T, size_t first, size_t keep, int tag_limit) {
  for (size_t k = 0; k < T.pending.size(); ++k) {
    auto& e = T.pending[k];
    const bool tag_ok = tag_limit < 0 || (k < T.tags.size() && T.tags[k] < tag_limit);
    if (k >= first && k - first < keep && tag_ok) {
      float ms = 0.0f;
      if (hipEventElapsedTime(&ms, e.first, e.second) == hipSuccess) {
        T.total_ms += ms;
        T.count += 1;
      }
    }
    T.pool.push_back(e);
  }
  T.pending.clear();
  T.tags.clear();
}

int ensure_partials(Ctx* c, int64_t blocks, int per) {
  const int64_t need = blocks * per + 64;
  if (c->partials_len < need) {
    VIP_HIP_TRY(c, hipStreamSynchronize(c->stream));
    dfree(c->partials);
    VIP_TRY(dalloc(c, &c->partials, need));
    c->partials_len = need;
  }
  return VIP_OK;
}

// Pressure Poisson solve (eq. 13) on the context's system layout.
int poisson_solve(Ctx* c, const double* rhs, double* phi, double tol, bool use_x0, vip_step_stats* st) {
  const int64_t n = c->n;
  const Method m = choose_method(c);
  // CG on a singular symmetric matrix works on the range: project b, drop the border
  const bool border = c->singular && m == kBiCGStab;
  const bool project = c->singular && m == kCG;
  const int64_t stride = n + 1;
  const int64_t nvec = n + (border ? 1 : 0);
  const bool mixed = c->opt.precision == VIP_P_MIXED;
  const bool use_amg = c->opt.preconditioner == VIP_PC_AMG;
  if (use_amg && !c->amg.ready) VIP_TRY(amg_setup(c));
  VIP_TRY(ensure_ws(c, 11 * stride, mixed ? 10 * stride : 1));
  // a system that is neither bordered nor projected is solved in the caller's buffers (b is
  // only read, x = phi) when they do not overlap; else b and x are copies with the border entry
  const bool direct = !border && !project && (rhs + n <= phi || phi + n <= rhs);
  double* bw = c->ws + 8 * stride;      // right-hand side with border entry 0
  const double* b = direct ? rhs : bw;
  double* x = direct ? phi : c->ws + 10 * stride;   // FP64 solution (bordered)
  hipStream_t s = c->stream;
  const int64_t gv = grid_for(stride);
  VIP_TRY(ensure_partials(c, gv, 3));
  if (!direct) {
    k_copy<double, double><<<grid_for(n), kBlock, 0, s>>>(n, rhs, bw);
    k_fill<double><<<1, 64, 0, s>>>(1, bw + n, 0.0);
  }
  double lambda_proj = 0.0;
  if (project) {
    k_sum<<<red_grid(n), kBlock, 0, s>>>(n, b, c->partials);
    k_fin_mean<<<1, kBlock, 0, s>>>(c->partials, red_grid(n), n, c->sc);
    k_sub_mean<<<grid_for(n), kBlock, 0, s>>>(n, bw, bw, c->sc);
    VIP_TRY(sync_scalars(c));
    lambda_proj = c->sc_host->mean;
  }
  if (direct) {
    if (!use_x0) k_fill<double><<<grid_for(n), kBlock, 0, s>>>(n, x, 0.0);
  } else if (use_x0) {
    k_copy<double, double><<<grid_for(n), kBlock, 0, s>>>(n, phi, x);
    k_fill<double><<<1, 64, 0, s>>>(1, x + n, 0.0);
  } else {
    k_fill<double><<<gv, kBlock, 0, s>>>(stride, x, 0.0);
  }
  Mat<double> A64{n, border ? 1 : 0, c->sys.ptr, c->sys.cols, {c->sys.val[0], nullptr}, {nullptr, nullptr}};
  attach_canon(c, A64, 0, -1);
  int total_it = 0, outer = 0;
  int lpc_used = 0;
  double lpc_gain = 1.0;
  double relres = 0.0;
  const int maxit = c->opt.max_iters;
  bool converged = false;
  // FP64 refinement passes from the current FP64 iterate x
  auto fp64_passes = [&]() -> int {
    Vec<double> V = make_vec<double>(c->ws, stride, 1, x);
    V.dinv[0] = c->dinv[0];
    for (int k = 1; k <= 20; ++k, ++outer) {
      VIP_TRY((residual<double, double, double, 1>(c, A64, x, b, V.r, stride)));
      const double bb = c->sc_host->bb[0];
      if (bb == 0.0) {
        relres = 0.0;
        converged = true;
        break;
      }
      relres = std::sqrt(c->sc_host->rr[0] / bb);
      if (relres <= tol) {
        converged = true;
        break;
      }
      if (total_it >= maxit) break;
      int it = 0;
      bool bad = false;
      VIP_TRY((iterate<double, double, 1>(c, m, A64, V, tol, maxit - total_it, &it, true, &bb, use_amg,
                                          &bad, &c->hint_p64[std::min(k - 1, 3)])));
      total_it += it;
      if (bad) return set_error(c, VIP_E_NONFINITE, "non-finite Krylov residual");
    }
    return VIP_OK;
  };
  bool fallback = false;
  if (!mixed) {
    outer = 1;
    VIP_TRY(fp64_passes());
  } else {
    Mat<float> A32{n, border ? 1 : 0, c->sys.ptr, c->sys.cols, {c->sys.val32, nullptr}, {c->sys.rsum32, nullptr}};
    attach_canon(c, A32, 4, -1);
    float* d32 = c->ws32 + 8 * stride;
    float* r32base = c->ws32;
    Vec<float> V = make_vec<float>(r32base, stride, 1, d32);
    V.dinv[0] = c->dinv32;
    // an FP32 correction gets at most kInnerCap iterations; one that breaks down, or a pass that
    // does not halve the FP64 residual, hands the solve to FP64 iterations from the FP64 iterate
    // (the FP32 multigrid-preconditioned iteration stagnates on large singular bordered systems)
    constexpr int kInnerCap = 150;
    const double inner = std::max(c->opt.inner_tol, 1e-7);
    double prev = 0.0;
    const bool lpc = !border && !project && learn_precond_active(c);
    for (outer = 1; outer <= 200; ++outer) {
      // FP64 residual of the current FP64 iterate, cast into the inner right-hand side
      VIP_TRY((residual<double, double, float, 1>(c, A64, x, b, V.r, stride)));
      const double bb = c->sc_host->bb[0];
      if (bb == 0.0) {
        relres = 0.0;
        converged = true;
        break;
      }
      relres = std::sqrt(c->sc_host->rr[0] / bb);
      if (relres <= tol) {
        converged = true;
        break;
      }
      if (total_it >= maxit) break;
      if (outer > 1 && relres > 0.5 * prev) {
        fallback = true;
        break;
      }
      prev = relres;
      const double rr_outer = c->sc_host->rr[0];
      // inner: A32 d = r, from d = 0; its residual starts as r itself
      int it = 0;
      bool bad = false;
      const double target = std::max(inner, 0.5 * tol / relres);
      VIP_TRY((iterate<float, float, 1>(c, m, A32, V, target, std::min(kInnerCap, maxit - total_it), &it, true,
                                        &rr_outer, use_amg, &bad, &c->hint_p32[std::min(outer - 1, 3)], true)));
      total_it += it;
      if (bad) {
        fallback = true;   // x is unchanged: the broken correction is not added
        break;
      }
      if (lpc) {
        // the pass residual in V.r was overwritten by the inner solve: recompute it (FP32 copy
        // of the FP64 residual of x) for the network's input
        VIP_TRY((residual<double, double, float, 1>(c, A64, x, b, V.r, stride)));
        VIP_TRY(learn_precond_pass(c, V.r, b, d32, x, &lpc_used, &lpc_gain));
      } else {
        k_add_f32<<<gv, kBlock, 0, s>>>(nvec, x, d32);
      }
    }
    if (fallback) VIP_TRY(fp64_passes());
  }
  if (project) {
    // phi with zero mean
    k_sum<<<red_grid(n), kBlock, 0, s>>>(n, x, c->partials);
    k_fin_mean<<<1, kBlock, 0, s>>>(c->partials, red_grid(n), n, c->sc);
    k_sub_mean<<<grid_for(n), kBlock, 0, s>>>(n, x, phi, c->sc);
  } else if (!direct) {
    k_copy<double, double><<<grid_for(n), kBlock, 0, s>>>(n, x, phi);
  }
  double lam = lambda_proj;
  if (border) {
    // the border unknown is a statistic: read it back (the only wait after the last check)
    double h = 0.0;
    VIP_HIP_TRY(c, hipMemcpyAsync(&h, x + n, sizeof(double), hipMemcpyDeviceToHost, s));
    VIP_HIP_TRY(c, hipStreamSynchronize(s));
    lam = h;
  }
  VIP_HIP_TRY(c, hipGetLastError());
  if (st) {
    st->poisson_iters = total_it;
    st->poisson_outer = outer;
    st->poisson_residual = relres;
    st->krylov_used = m == kCG ? VIP_K_PCG : VIP_K_BICGSTAB;
    st->border_lambda = lam;
    st->poisson_fp64_fallback = fallback ? 1 : 0;
    st->learned_pc_passes = lpc_used;
    st->learned_pc_ratio = lpc_gain;
  }
  if (!std::isfinite(relres)) return set_error(c, VIP_E_NONFINITE, "non-finite Poisson residual");
  if (!converged)
    return set_error(c, VIP_E_NOT_CONVERGED, "Poisson solve stopped at relative residual " +
                                                 sci(relres));
  return VIP_OK;
}

// The two predictor systems H_u u* = r_u, H_v v* = r_v in lockstep: FP64 BiCGStab, or with
// VIP_P_MIXED FP32 BiCGStab corrections inside FP64 iterative refinement (FP64 residual and
// iterate, to the same FP64 tolerance).
int predictor_rhs_buffer(Ctx* c, double** b) {
  const int64_t stride = c->n + 1;
  const bool mixed = c->opt.precision == VIP_P_MIXED && c->sys.val32h[0] && c->sys.val32h[1];
  VIP_TRY(ensure_ws(c, 2 * 8 * stride + 2 * stride, mixed ? 2 * 8 * stride + 2 * stride : 1));
  *b = c->ws + 16 * stride;   // [2][stride]
  return VIP_OK;
}

int helmholtz_solve(Ctx* c, const double* ru, const double* rv, double** us_out, double** vs_out,
                    vip_step_stats* st) {
  const int64_t n = c->n;
  const int64_t stride = n + 1;
  const bool mixed = c->opt.precision == VIP_P_MIXED && c->sys.val32h[0] && c->sys.val32h[1];
  double* b = nullptr;
  VIP_TRY(predictor_rhs_buffer(c, &b));
  hipStream_t s = c->stream;
  if (ru != b) k_copy<double, double><<<grid_for(n), kBlock, 0, s>>>(n, ru, b);
  if (rv != b + stride) k_copy<double, double><<<grid_for(n), kBlock, 0, s>>>(n, rv, b + stride);
  // start vector: the quadratic extrapolation 3 u*(n-1) - 3 u*(n-2) + u*(n-3) of the last three
  // predictor solutions (error O(dt^3)), the linear one 2 u*(n-1) - u*(n-2) when two are held,
  // the last solution when one is held, else the right-hand side (the operators are close to
  // the identity); the history counts again only once this solve has succeeded.  The solutions
  // live in a ring of three slots: the solve runs in the slot after the newest (that of
  // u*(n-3), extrapolated in place), which then becomes the newest, so no solution is copied.
  const int held = c->nstar;
  c->nstar = 0;
  if (!c->star_ring) VIP_TRY(dalloc(c, &c->star_ring, 3 * 2 * stride));
  auto slot = [&](int k) { return c->star_ring + static_cast<int64_t>(((k % 3) + 3) % 3) * 2 * stride; };
  const int h = c->star_head;
  double* last = slot(h);
  double* before = slot(h - 1);
  double* x = slot(h + 1);   // [2][stride]; u*(n-3) when three are held
  if (held >= 3) {
    k_extrapolate3<<<grid_for(n), kBlock, 0, s>>>(n, last, before, x, x);
    k_extrapolate3<<<grid_for(n), kBlock, 0, s>>>(n, last + stride, before + stride, x + stride, x + stride);
  } else if (held == 2) {
    k_extrapolate<<<grid_for(n), kBlock, 0, s>>>(n, last, before, x);
    k_extrapolate<<<grid_for(n), kBlock, 0, s>>>(n, last + stride, before + stride, x + stride);
  } else if (held == 1) {
    k_copy<double, double><<<grid_for(n), kBlock, 0, s>>>(n, last, x);
    k_copy<double, double><<<grid_for(n), kBlock, 0, s>>>(n, last + stride, x + stride);
  } else {
    k_copy<double, double><<<grid_for(n), kBlock, 0, s>>>(n, b, x);
    k_copy<double, double><<<grid_for(n), kBlock, 0, s>>>(n, b + stride, x + stride);
  }
  c->star_head = (h + 1) % 3;
  *us_out = x;
  *vs_out = x + stride;
  Mat<double> H{n, 0, c->sys.ptr, c->sys.cols, {c->sys.val[1], c->sys.val[2]}, {nullptr, nullptr}};
  attach_canon(c, H, 1, 2);
  Vec<double> V = make_vec<double>(c->ws, stride, 2, x);
  V.dinv[0] = c->dinv[1];
  V.dinv[1] = c->dinv[2];
  Mat<float> H32{n, 0, c->sys.ptr, c->sys.cols, {c->sys.val32h[0], c->sys.val32h[1]},
                 {c->sys.rsum32h[0], c->sys.rsum32h[1]}};
  Vec<float> V32{};
  float* d32 = nullptr;
  if (mixed) {
    attach_canon(c, H32, 5, 6);
    d32 = c->ws32 + 16 * stride;         // [2][stride] FP32 correction
    V32 = make_vec<float>(c->ws32, stride, 2, d32);
    // the Jacobi preconditioner is folded into H32 = H D^-1: plain BiCGStab for y with
    // H32 y = r (the same residual r - H d for d = D^-1 y), no preconditioned vectors
    V32.dinv[0] = V32.dinv[1] = nullptr;
    V32.ph = V32.p;
    V32.sh = V32.s;
  }
  const double tol = c->opt.helmholtz_tol;
  const double inner = std::max(c->opt.inner_tol, 1e-7);
  int total = 0;
  double worst = 0.0;
  bool converged = false;
  for (int outer = 0; outer < (mixed ? 40 : 10); ++outer) {
    if (mixed) {
      VIP_TRY((residual<double, double, float, 2>(c, H, x, b, V32.r, stride)));
    } else {
      VIP_TRY((residual<double, double, double, 2>(c, H, x, b, V.r, stride)));
    }
    double bb[2] = {c->sc_host->bb[0], c->sc_host->bb[1]};
    double rr[2] = {c->sc_host->rr[0], c->sc_host->rr[1]};
    worst = 0.0;
    for (int k = 0; k < 2; ++k) worst = std::max(worst, bb[k] > 0.0 ? std::sqrt(rr[k] / bb[k]) : 0.0);
    if (worst <= tol) {
      converged = true;
      break;
    }
    if (total >= c->opt.max_iters) break;
    int it = 0;
    bool bad = false;
    if (mixed) {
      // FP32 correction d from 0 for the FP64 residual r, to `target` relative to |r|
      const double target = std::max(inner, 0.5 * tol / worst);
      VIP_TRY((iterate<float, float, 2>(c, kBiCGStab, H32, V32, target, c->opt.max_iters - total, &it, false,
                                        rr, false, &bad, &c->hint_h32[std::min(outer, 3)], true)));
      total += it;
      if (bad) return set_error(c, VIP_E_NONFINITE, "FP32 predictor correction produced a non-finite residual");
      k_add_scaled<<<grid_for(2 * stride), kBlock, 0, s>>>(2 * stride, stride, n, x, d32, c->dinv[1], c->dinv[2]);
    } else {
      // a system whose b is zero is solved by x = 0 exactly: give it a unit norm
      for (int k = 0; k < 2; ++k) if (bb[k] == 0.0) bb[k] = 1.0;
      VIP_TRY((iterate<double, double, 2>(c, kBiCGStab, H, V, tol, c->opt.max_iters - total, &it, false, bb,
                                          false, &bad, outer == 0 ? &c->hint_h : nullptr)));
      total += it;
      if (bad) return set_error(c, VIP_E_NONFINITE, "non-finite predictor residual");
    }
  }
  VIP_HIP_TRY(c, hipGetLastError());
  if (converged && std::isfinite(worst)) c->nstar = std::min(held + 1, 3);
  if (st) {
    st->helmholtz_iters = total;
    st->helmholtz_residual = worst;
  }
  if (!std::isfinite(worst)) return set_error(c, VIP_E_NONFINITE, "non-finite predictor residual");
  if (!converged)
    return set_error(c, VIP_E_NOT_CONVERGED, "predictor solve stopped at relative residual " +
                                                 sci(worst));
  return VIP_OK;
}

// y = A x for a generic FP64 operator (value set vs), one thread per row.
__global__ void k_apply(int64_t nrows, const int64_t* ptr, const int32_t* cols, const double* val,
                        const double* x, double* y) {
  const int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
  if (i >= nrows) return;
  const int64_t sl = i / kSlice;
  const int64_t base = ptr[sl] + (i % kSlice);
  const int64_t w = (ptr[sl + 1] - ptr[sl]) / kSlice;
  double acc = 0.0;
  for (int64_t k = 0; k < w; ++k) acc += val[base + k * kSlice] * x[cols[base + k * kSlice]];
  y[i] = acc;
}

// The input of a pressure product: x, or (DIFF) the difference x - x2 formed where it is read,
// with the bits of the separate difference pass (k_sub).
template <bool DIFF>
struct SysInput {
  const double* x;
  const double* x2;
  __device__ __forceinline__ double operator[](int64_t j) const {
    if constexpr (DIFF) return x[j] - x2[j];
    else return x[j];
  }
};

// Per row i of a pressure product y_i = (P x')_i: stores y, the residual b - y, the input x' (DIFF:
// the difference) and a copy of x, whichever are set.
__device__ __forceinline__ void sys_emit(const SysApply& P, int64_t i, double yi, double xi) {
  if (P.y) P.y[i] = yi;
  if (P.r) P.r[i] = P.b[i] - yi;
  if (P.xd) P.xd[i] = xi;
  if (P.cp) P.cp[i] = P.x[i];
}

// y = P x' for the FP64 pressure matrix (canonical rows included), one thread per row.
template <bool DIFF>
__global__ void k_sys_apply(Mat<double> A, SysApply P) {
  const int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
  if (i >= A.n) return;
  const SysInput<DIFF> x{P.x, P.x2};
  sys_emit(P, i, row_dot(A, 0, i, x), x[i]);
}

// The same over the tile partition: canonical rows from LDS tiles, the others row by row (the
// same bits as k_sys_apply).
template <bool GEN, bool DIFF>
__global__ void __launch_bounds__(kBlock) k_sys_apply_tiles(Mat<double> A, SysApply P) {
  __shared__ double lds[1][kTileLdsH][kTileLdsW];
  __shared__ TileMeta meta;
  const SysInput<DIFF> x{P.x, P.x2};
  tile_walk(
      A.tv,
      [&](int64_t tk) __attribute__((always_inline)) {
        tile_stage_fn<double, 1>(
            A.tv, tk, [&](int, int32_t node) __attribute__((always_inline)) { return x[node]; }, lds, meta, !GEN);
        const int wave = static_cast<int>(threadIdx.x >> 6), lane = static_cast<int>(threadIdx.x & 63);
#pragma unroll 1
        for (int k = 0; k < kTileRowsPerWave; ++k) {
          const int64_t row = tile_row_id(A.tv, meta, k);
          if (row < 0) continue;
          const int ly = wave + k * (kBlock / 64);
          if constexpr (GEN) sys_emit(P, row, row_dot_rows(A, 0, row, x), x[row]);
          else sys_emit(P, row, disk_lds(A, 0, lds[0], ly, lane), lds[0][ly + 2][lane + 2]);
        }
      },
      [&](int64_t i) __attribute__((always_inline)) { sys_emit(P, i, row_dot_rows(A, 0, i, x), x[i]); });
}

int pressure_apply(Ctx* c, const SysApply& P) {
  Mat<double> A{c->n, 0, c->sys.ptr, c->sys.cols, {c->sys.val[0], nullptr}, {nullptr, nullptr}};
  attach_canon(c, A, 0, -1);
  VIP_TRY(check_mat(c, A, 1));
  const bool diff = P.x2 != nullptr;
  if (A.tv.tiles) {
    const int64_t g = spmv_grid(A);
    if (A.tile_general && diff) k_sys_apply_tiles<true, true><<<g, kBlock, 0, c->stream>>>(A, P);
    else if (A.tile_general) k_sys_apply_tiles<true, false><<<g, kBlock, 0, c->stream>>>(A, P);
    else if (diff) k_sys_apply_tiles<false, true><<<g, kBlock, 0, c->stream>>>(A, P);
    else k_sys_apply_tiles<false, false><<<g, kBlock, 0, c->stream>>>(A, P);
    VIP_HIP_TRY(c, hipGetLastError());
    return VIP_OK;
  }
  if (diff) k_sys_apply<true><<<grid_for(c->n), kBlock, 0, c->stream>>>(A, P);
  else k_sys_apply<false><<<grid_for(c->n), kBlock, 0, c->stream>>>(A, P);
  VIP_HIP_TRY(c, hipGetLastError());
  return VIP_OK;
}

int pressure_apply(Ctx* c, const double* x, double* y) {
  SysApply P{};
  P.x = x;
  P.y = y;
  return pressure_apply(c, P);
}

int ell_apply(Ctx* c, const Ell& e, int vs, const double* x, double* y) {
  if (e.nrows == 0) return VIP_OK;
  k_apply<<<grid_for(e.nrows), kBlock, 0, c->stream>>>(e.nrows, e.ptr, e.cols, e.val[vs], x, y);
  VIP_HIP_TRY(c, hipGetLastError());
  return VIP_OK;
}

}  // namespace vip
