// Krylov solvers of the pressure Poisson system (eq. 13) and of the two
// Crank-Nicolson predictor systems (eq. 12), on the sliced-ELL system layout.
//
// * SpMV kernels are one thread per row over 64-row column-major slices, with
//   the dot products the method needs next fused in, reduced per block and
//   finished by the last block to arrive (fixed summation order, so repeated
//   runs are bitwise identical).  Step lengths (alpha, omega, beta) stay in
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
#include <vector>

#include "vip_internal.h"

namespace vip {

namespace {

constexpr int kWaves = kBlock / 64;

// Sum NV values over the block and publish the block sums; returns true in the
// last block to finish, whose threads then hold the grand totals in v[].
template <int NV>
__device__ __forceinline__ bool reduce_last(double (&v)[NV], double* partials, unsigned int* counter) {
  __shared__ double red[NV][kWaves];
  __shared__ int last;
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
      __hip_atomic_store(&partials[static_cast<int64_t>(blockIdx.x) * NV + a], t, __ATOMIC_RELAXED,
                         __HIP_MEMORY_SCOPE_AGENT);
    }
    const unsigned int prev =
        __hip_atomic_fetch_add(counter, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
    last = (prev == gridDim.x - 1) ? 1 : 0;
  }
  __syncthreads();
  if (!last) return false;
  __threadfence();
  const int64_t nb = gridDim.x;
#pragma unroll
  for (int a = 0; a < NV; ++a) {
    double t = 0.0;
    for (int64_t b = threadIdx.x; b < nb; b += blockDim.x)
      t += __hip_atomic_load(&partials[b * NV + a], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) t += __shfl_xor(t, off, 64);
    if (lane == 0) red[a][wave] = t;
  }
  __syncthreads();
#pragma unroll
  for (int a = 0; a < NV; ++a) {
    double t = 0.0;
#pragma unroll
    for (int w = 0; w < kWaves; ++w) t += red[a][w];
    v[a] = t;
  }
  if (threadIdx.x == 0) __hip_atomic_store(counter, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  return true;
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
};

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

// Row i of y = A x for system `sys`; x is the system's vector.
template <typename VT, typename T>
__device__ __forceinline__ double row_dot(const Mat<VT>& A, int sys, int64_t i, const T* x) {
  const int64_t sl = i / kSlice;
  const int64_t base = A.ptr[sl] + (i % kSlice);
  const int64_t w = (A.ptr[sl + 1] - A.ptr[sl]) / kSlice;
  const VT* vals = A.val[sys];
  double acc = 0.0;
  if constexpr (sizeof(VT) == 4) {
    float a32 = 0.0f;
    for (int64_t k = 0; k < w; ++k) {
      const int64_t q = base + k * kSlice;
      a32 += static_cast<float>(vals[q]) * static_cast<float>(x[A.cols[q]]);
    }
    acc = a32;
  } else {
    for (int64_t k = 0; k < w; ++k) {
      const int64_t q = base + k * kSlice;
      acc += static_cast<double>(vals[q]) * static_cast<double>(x[A.cols[q]]);
    }
  }
  return acc;
}

// ---- residual: r = b - A x (FP64 values), rr = |r|^2, bb = |b|^2 ---------------------------
template <typename VT, typename XT, typename RT, int NS>
__global__ void k_residual(Mat<VT> A, const XT* x, const double* b, RT* r, int64_t stride,
                           double* partials, unsigned int* counter, KrylovScalars* sc) {
  const int64_t lb = xcd_block(blockIdx.x, gridDim.x);
  const int64_t i = lb * blockDim.x + threadIdx.x;
  double acc[3 * NS];
#pragma unroll
  for (int a = 0; a < 3 * NS; ++a) acc[a] = 0.0;
  if (i < A.n) {
#pragma unroll
    for (int s = 0; s < NS; ++s) {
      const XT* xs = x + s * stride;
      double ax = row_dot(A, s, i, xs);
      if (A.border) ax += static_cast<double>(xs[A.n]);
      const double bi = b[s * stride + i];
      const double ri = bi - ax;
      r[s * stride + i] = static_cast<RT>(ri);
      acc[3 * s + 0] = ri * ri;
      acc[3 * s + 1] = bi * bi;
      acc[3 * s + 2] = A.border ? static_cast<double>(xs[i]) : 0.0;
    }
  }
  if (reduce_last<3 * NS>(acc, partials, counter) && threadIdx.x == 0) {
#pragma unroll
    for (int s = 0; s < NS; ++s) {
      double rr = acc[3 * s], bb = acc[3 * s + 1];
      if (A.border) {
        const double bn = b[s * stride + A.n];
        const double rn = bn - acc[3 * s + 2];
        r[s * stride + A.n] = static_cast<RT>(rn);
        rr += rn * rn;
        bb += bn * bn;
      }
      sc->rr[s] = rr;
      sc->bb[s] = bb;
    }
  }
}

// ---- BiCGStab -------------------------------------------------------------------------------
template <typename T, int NS>
__global__ void k_bicg_init(Vec<T> V, int64_t nvec, KrylovScalars* sc) {
  const int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
  if (i < nvec) {
#pragma unroll
    for (int s = 0; s < NS; ++s) {
      const int64_t o = s * V.stride + i;
      V.rhat[o] = V.r[o];
      V.p[o] = T(0);
      V.v[o] = T(0);
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
    }
  }
}

// p = r + beta (p - omega v); ph = D^-1 p
template <typename T, int NS>
__global__ void k_bicg_p(Vec<T> V, int64_t nvec, const KrylovScalars* sc, const int* active) {
  const int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
  if (i >= nvec) return;
#pragma unroll
  for (int s = 0; s < NS; ++s) {
    if (!active[s]) continue;
    const int64_t o = s * V.stride + i;
    const T beta = static_cast<T>(sc->beta[s]), omega = static_cast<T>(sc->omega[s]);
    const T p = V.r[o] + beta * (V.p[o] - omega * V.v[o]);
    V.p[o] = p;
    V.ph[o] = V.dinv[s][i] * p;
  }
}

// v = A ph; alpha = rho / (rhat . v)
template <typename VT, typename T, int NS>
__global__ void k_bicg_v(Mat<VT> A, Vec<T> V, double* partials, unsigned int* counter,
                         KrylovScalars* sc, const int* active) {
  const int64_t lb = xcd_block(blockIdx.x, gridDim.x);
  const int64_t i = lb * blockDim.x + threadIdx.x;
  double acc[2 * NS];
#pragma unroll
  for (int a = 0; a < 2 * NS; ++a) acc[a] = 0.0;
  if (i < A.n) {
#pragma unroll
    for (int s = 0; s < NS; ++s) {
      if (!active[s]) continue;
      const T* ph = V.ph + s * V.stride;
      double y = row_dot(A, s, i, ph);
      if (A.border) y += static_cast<double>(ph[A.n]);
      const T yt = static_cast<T>(y);
      V.v[s * V.stride + i] = yt;
      acc[2 * s] = static_cast<double>(V.rhat[s * V.stride + i]) * static_cast<double>(yt);
      acc[2 * s + 1] = A.border ? static_cast<double>(ph[i]) : 0.0;
    }
  }
  if (reduce_last<2 * NS>(acc, partials, counter) && threadIdx.x == 0) {
#pragma unroll
    for (int s = 0; s < NS; ++s) {
      if (!active[s]) continue;
      double d = acc[2 * s];
      if (A.border) {
        const T yn = static_cast<T>(acc[2 * s + 1]);
        V.v[s * V.stride + A.n] = yn;
        d += static_cast<double>(V.rhat[s * V.stride + A.n]) * static_cast<double>(yn);
      }
      sc->dot_a[s] = d;
      sc->alpha[s] = safe_div(sc->rho[s], d, &sc->breakdown[s]);
    }
  }
}

// s = r - alpha v; sh = D^-1 s
template <typename T, int NS>
__global__ void k_bicg_s(Vec<T> V, int64_t nvec, const KrylovScalars* sc, const int* active) {
  const int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
  if (i >= nvec) return;
#pragma unroll
  for (int s = 0; s < NS; ++s) {
    if (!active[s]) continue;
    const int64_t o = s * V.stride + i;
    const T sv = V.r[o] - static_cast<T>(sc->alpha[s]) * V.v[o];
    V.s[o] = sv;
    V.sh[o] = V.dinv[s][i] * sv;
  }
}

// t = A sh; omega = (t . s) / (t . t)
template <typename VT, typename T, int NS>
__global__ void k_bicg_t(Mat<VT> A, Vec<T> V, double* partials, unsigned int* counter,
                         KrylovScalars* sc, const int* active) {
  const int64_t lb = xcd_block(blockIdx.x, gridDim.x);
  const int64_t i = lb * blockDim.x + threadIdx.x;
  double acc[3 * NS];
#pragma unroll
  for (int a = 0; a < 3 * NS; ++a) acc[a] = 0.0;
  if (i < A.n) {
#pragma unroll
    for (int s = 0; s < NS; ++s) {
      if (!active[s]) continue;
      const T* sh = V.sh + s * V.stride;
      double y = row_dot(A, s, i, sh);
      if (A.border) y += static_cast<double>(sh[A.n]);
      const T yt = static_cast<T>(y);
      V.t[s * V.stride + i] = yt;
      const double sv = static_cast<double>(V.s[s * V.stride + i]);
      acc[3 * s] = static_cast<double>(yt) * sv;
      acc[3 * s + 1] = static_cast<double>(yt) * static_cast<double>(yt);
      acc[3 * s + 2] = A.border ? static_cast<double>(sh[i]) : 0.0;
    }
  }
  if (reduce_last<3 * NS>(acc, partials, counter) && threadIdx.x == 0) {
#pragma unroll
    for (int s = 0; s < NS; ++s) {
      if (!active[s]) continue;
      double ts = acc[3 * s], tt = acc[3 * s + 1];
      if (A.border) {
        const T yn = static_cast<T>(acc[3 * s + 2]);
        V.t[s * V.stride + A.n] = yn;
        ts += static_cast<double>(yn) * static_cast<double>(V.s[s * V.stride + A.n]);
        tt += static_cast<double>(yn) * static_cast<double>(yn);
      }
      sc->dot_b[s] = ts;
      sc->dot_c[s] = tt;
      // tt == 0 means s == 0: the half step already solved the system
      sc->omega[s] = tt > 0.0 ? ts / tt : 0.0;
    }
  }
}

// x += alpha ph + omega sh; r = s - omega t; rho' = rhat . r; beta = (rho'/rho)(alpha/omega)
template <typename T, int NS>
__global__ void k_bicg_x(Vec<T> V, int64_t nvec, double* partials, unsigned int* counter,
                         KrylovScalars* sc, const int* active) {
  const int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
  double acc[2 * NS];
#pragma unroll
  for (int a = 0; a < 2 * NS; ++a) acc[a] = 0.0;
  if (i < nvec) {
#pragma unroll
    for (int s = 0; s < NS; ++s) {
      if (!active[s]) continue;
      const int64_t o = s * V.stride + i;
      const T alpha = static_cast<T>(sc->alpha[s]), omega = static_cast<T>(sc->omega[s]);
      V.x[o] = V.x[o] + alpha * V.ph[o] + omega * V.sh[o];
      const T r = V.s[o] - omega * V.t[o];
      V.r[o] = r;
      acc[2 * s] = static_cast<double>(V.rhat[o]) * static_cast<double>(r);
      acc[2 * s + 1] = static_cast<double>(r) * static_cast<double>(r);
    }
  }
  if (reduce_last<2 * NS>(acc, partials, counter) && threadIdx.x == 0) {
#pragma unroll
    for (int s = 0; s < NS; ++s) {
      if (!active[s]) continue;
      const double rho_new = acc[2 * s];
      sc->rr[s] = acc[2 * s + 1];
      const double ratio = safe_div(rho_new, sc->rho[s], &sc->breakdown[s]);
      const double om = sc->omega[s];
      sc->beta[s] = (om != 0.0 && isfinite(ratio)) ? ratio * (sc->alpha[s] / om) : 0.0;
      if (om == 0.0 && acc[2 * s + 1] > 0.0) sc->breakdown[s] = 1;
      sc->rho[s] = rho_new;
    }
  }
}

// ---- CG ---------------------------------------------------------------------------------------
// z = D^-1 r; p = z; rho = r . z
template <typename T, int NS>
__global__ void k_cg_init(Vec<T> V, int64_t nvec, double* partials, unsigned int* counter,
                          KrylovScalars* sc) {
  const int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
  double acc[NS];
#pragma unroll
  for (int a = 0; a < NS; ++a) acc[a] = 0.0;
  if (i < nvec) {
#pragma unroll
    for (int s = 0; s < NS; ++s) {
      const int64_t o = s * V.stride + i;
      const T z = V.dinv[s][i] * V.r[o];
      V.p[o] = z;
      acc[s] = static_cast<double>(V.r[o]) * static_cast<double>(z);
    }
  }
  if (reduce_last<NS>(acc, partials, counter) && threadIdx.x == 0) {
#pragma unroll
    for (int s = 0; s < NS; ++s) {
      sc->rho[s] = acc[s];
      sc->breakdown[s] = 0;
    }
  }
}

// v = A p; alpha = rho / (p . v)
template <typename VT, typename T, int NS>
__global__ void k_cg_q(Mat<VT> A, Vec<T> V, double* partials, unsigned int* counter,
                       KrylovScalars* sc, const int* active) {
  const int64_t lb = xcd_block(blockIdx.x, gridDim.x);
  const int64_t i = lb * blockDim.x + threadIdx.x;
  double acc[NS];
#pragma unroll
  for (int a = 0; a < NS; ++a) acc[a] = 0.0;
  if (i < A.n) {
#pragma unroll
    for (int s = 0; s < NS; ++s) {
      if (!active[s]) continue;
      const T* p = V.p + s * V.stride;
      const T y = static_cast<T>(row_dot(A, s, i, p));
      V.v[s * V.stride + i] = y;
      acc[s] = static_cast<double>(p[i]) * static_cast<double>(y);
    }
  }
  if (reduce_last<NS>(acc, partials, counter) && threadIdx.x == 0) {
#pragma unroll
    for (int s = 0; s < NS; ++s) {
      if (!active[s]) continue;
      sc->dot_a[s] = acc[s];
      sc->alpha[s] = safe_div(sc->rho[s], acc[s], &sc->breakdown[s]);
    }
  }
}

// x += alpha p; r -= alpha v; rho' = r . D^-1 r; beta = rho'/rho
template <typename T, int NS>
__global__ void k_cg_x(Vec<T> V, int64_t nvec, double* partials, unsigned int* counter,
                       KrylovScalars* sc, const int* active) {
  const int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
  double acc[2 * NS];
#pragma unroll
  for (int a = 0; a < 2 * NS; ++a) acc[a] = 0.0;
  if (i < nvec) {
#pragma unroll
    for (int s = 0; s < NS; ++s) {
      if (!active[s]) continue;
      const int64_t o = s * V.stride + i;
      const T alpha = static_cast<T>(sc->alpha[s]);
      V.x[o] = V.x[o] + alpha * V.p[o];
      const T r = V.r[o] - alpha * V.v[o];
      V.r[o] = r;
      acc[2 * s] = static_cast<double>(r) * static_cast<double>(V.dinv[s][i] * r);
      acc[2 * s + 1] = static_cast<double>(r) * static_cast<double>(r);
    }
  }
  if (reduce_last<2 * NS>(acc, partials, counter) && threadIdx.x == 0) {
#pragma unroll
    for (int s = 0; s < NS; ++s) {
      if (!active[s]) continue;
      sc->rr[s] = acc[2 * s + 1];
      sc->beta[s] = safe_div(acc[2 * s], sc->rho[s], &sc->breakdown[s]);
      sc->rho[s] = acc[2 * s];
    }
  }
}

// p = D^-1 r + beta p
template <typename T, int NS>
__global__ void k_cg_p(Vec<T> V, int64_t nvec, const KrylovScalars* sc, const int* active) {
  const int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
  if (i >= nvec) return;
#pragma unroll
  for (int s = 0; s < NS; ++s) {
    if (!active[s]) continue;
    const int64_t o = s * V.stride + i;
    V.p[o] = V.dinv[s][i] * V.r[o] + static_cast<T>(sc->beta[s]) * V.p[o];
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

// sum of a[0..m) -> sc->mean = sum / m
__global__ void k_mean(int64_t m, const double* a, double* partials, unsigned int* counter,
                       KrylovScalars* sc) {
  const int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
  double acc[1] = {i < m ? a[i] : 0.0};
  if (reduce_last<1>(acc, partials, counter) && threadIdx.x == 0) sc->mean = acc[0] / static_cast<double>(m);
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
      if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess) {
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

void harvest_timing(Ctx* c) {
  for (auto& e : c->timing.pending) {
    float ms = 0.0f;
    if (hipEventElapsedTime(&ms, e.first, e.second) == hipSuccess) {
      c->timing.total_ms += ms;
      c->timing.count += 1;
    }
    c->timing.pool.push_back(e);
  }
  c->timing.pending.clear();
}

int sync_scalars(Ctx* c) {
  VIP_HIP_TRY(c, hipMemcpyAsync(c->sc_host, c->sc, sizeof(KrylovScalars), hipMemcpyDeviceToHost,
                                c->stream));
  VIP_HIP_TRY(c, hipStreamSynchronize(c->stream));
  harvest_timing(c);
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

// Device flags telling the kernels which systems are still iterating.
int* active_flags(Ctx* c) {
  return reinterpret_cast<int*>(c->partials + c->partials_len);   // tail of the partials buffer
}

int set_active(Ctx* c, const int* act) {
  VIP_HIP_TRY(c, hipMemcpyAsync(active_flags(c), act, 2 * sizeof(int), hipMemcpyHostToDevice,
                                c->stream));
  return VIP_OK;
}

// Iterate until |r| <= tol |b| (recurrence residual) for every system, or maxit.
// On entry V.r holds the initial residual and sc->rr/bb its norms.
template <typename VT, typename T, int NS>
int iterate(Ctx* c, Method m, const Mat<VT>& A, Vec<T>& V, double tol, int maxit, int* iters,
            bool time_spmv, const double* bnorm2) {
  const int64_t nvec = A.n + A.border;
  const int64_t g_rows = grid_for(A.n), g_vec = grid_for(nvec);
  VIP_TRY(ensure_partials(c, std::max(g_rows, g_vec), 3 * NS));
  int act[2] = {1, NS > 1 ? 1 : 0};
  for (int s = 0; s < NS; ++s)
    if (c->sc_host->rr[s] <= tol * tol * bnorm2[s]) act[s] = 0;
  VIP_TRY(set_active(c, act));
  const int* dact = active_flags(c);
  double* part = c->partials;
  unsigned int* cnt = c->counter;
  KrylovScalars* sc = c->sc;
  hipStream_t st = c->stream;
  if (m == kBiCGStab) {
    k_bicg_init<T, NS><<<g_vec, kBlock, 0, st>>>(V, nvec, sc);
  } else {
    k_cg_init<T, NS><<<g_vec, kBlock, 0, st>>>(V, nvec, part, cnt, sc);
  }
  int it = 0;
  const int every = std::max(1, c->opt.check_every);
  while ((act[0] || act[1]) && it < maxit) {
    const int batch = std::min(every, maxit - it);
    for (int b = 0; b < batch; ++b) {
      if (m == kBiCGStab) {
        k_bicg_p<T, NS><<<g_vec, kBlock, 0, st>>>(V, nvec, sc, dact);
        {
          Timer tm(c, time_spmv);
          k_bicg_v<VT, T, NS><<<g_rows, kBlock, 0, st>>>(A, V, part, cnt, sc, dact);
        }
        k_bicg_s<T, NS><<<g_vec, kBlock, 0, st>>>(V, nvec, sc, dact);
        k_bicg_t<VT, T, NS><<<g_rows, kBlock, 0, st>>>(A, V, part, cnt, sc, dact);
        k_bicg_x<T, NS><<<g_vec, kBlock, 0, st>>>(V, nvec, part, cnt, sc, dact);
      } else {
        {
          Timer tm(c, time_spmv);
          k_cg_q<VT, T, NS><<<g_rows, kBlock, 0, st>>>(A, V, part, cnt, sc, dact);
        }
        k_cg_x<T, NS><<<g_vec, kBlock, 0, st>>>(V, nvec, part, cnt, sc, dact);
        k_cg_p<T, NS><<<g_vec, kBlock, 0, st>>>(V, nvec, sc, dact);
      }
    }
    it += batch;
    VIP_HIP_TRY(c, hipGetLastError());
    VIP_TRY(sync_scalars(c));
    bool changed = false;
    for (int s = 0; s < NS; ++s) {
      if (!act[s]) continue;
      const double rr = c->sc_host->rr[s];
      if (!std::isfinite(rr)) return set_error(c, VIP_E_NONFINITE, "non-finite Krylov residual");
      if (rr <= tol * tol * bnorm2[s] || c->sc_host->breakdown[s]) {
        act[s] = 0;
        changed = true;
      }
    }
    if (changed) VIP_TRY(set_active(c, act));
  }
  *iters = it;
  return VIP_OK;
}

template <typename VT, typename XT, typename RT, int NS>
int residual(Ctx* c, const Mat<VT>& A, const XT* x, const double* b, RT* r, int64_t stride) {
  const int64_t g = grid_for(A.n);
  VIP_TRY(ensure_partials(c, g, 3 * NS));
  k_residual<VT, XT, RT, NS><<<g, kBlock, 0, c->stream>>>(A, x, b, r, stride, c->partials, c->counter,
                                                          c->sc);
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

Method choose_method(Ctx* c) {
  if (c->opt.krylov == VIP_K_PCG) return kCG;
  if (c->opt.krylov == VIP_K_BICGSTAB) return kBiCGStab;
  return c->symmetric ? kCG : kBiCGStab;
}

}  // namespace

int ensure_partials(Ctx* c, int64_t blocks, int per) {
  const int64_t need = blocks * per + 64;
  if (c->partials_len < need) {
    VIP_HIP_TRY(c, hipStreamSynchronize(c->stream));
    dfree(c->partials);
    // tail: 2 ints of active flags (fits in one extra double slot)
    VIP_TRY(dalloc(c, &c->partials, need + 1));
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
  VIP_TRY(ensure_ws(c, 11 * stride, mixed ? 10 * stride : 1));
  double* b = c->ws + 8 * stride;       // right-hand side with border entry 0
  double* x = c->ws + 10 * stride;      // FP64 solution (bordered)
  hipStream_t s = c->stream;
  const int64_t gv = grid_for(stride);
  VIP_TRY(ensure_partials(c, gv, 3));
  k_copy<double, double><<<grid_for(n), kBlock, 0, s>>>(n, rhs, b);
  k_fill<double><<<1, 64, 0, s>>>(1, b + n, 0.0);
  double lambda_proj = 0.0;
  if (project) {
    k_mean<<<grid_for(n), kBlock, 0, s>>>(n, b, c->partials, c->counter, c->sc);
    k_sub_mean<<<grid_for(n), kBlock, 0, s>>>(n, b, b, c->sc);
    VIP_TRY(sync_scalars(c));
    lambda_proj = c->sc_host->mean;
  }
  if (use_x0) {
    k_copy<double, double><<<grid_for(n), kBlock, 0, s>>>(n, phi, x);
    k_fill<double><<<1, 64, 0, s>>>(1, x + n, 0.0);
  } else {
    k_fill<double><<<gv, kBlock, 0, s>>>(stride, x, 0.0);
  }
  Mat<double> A64{n, border ? 1 : 0, c->sys.ptr, c->sys.cols, {c->sys.val[0], nullptr}};
  int total_it = 0, outer = 0;
  double relres = 0.0;
  const int maxit = c->opt.max_iters;
  bool converged = false;
  if (!mixed) {
    Vec<double> V = make_vec<double>(c->ws, stride, 1, x);
    V.dinv[0] = c->dinv[0];
    for (outer = 1; outer <= 20; ++outer) {
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
      VIP_TRY((iterate<double, double, 1>(c, m, A64, V, tol, maxit - total_it, &it, true, &bb)));
      total_it += it;
    }
  } else {
    const double inner = std::max(c->opt.inner_tol, 1e-7);
    Mat<float> A32{n, border ? 1 : 0, c->sys.ptr, c->sys.cols, {c->sys.val32, nullptr}};
    float* d32 = c->ws32 + 8 * stride;
    float* r32base = c->ws32;
    Vec<float> V = make_vec<float>(r32base, stride, 1, d32);
    V.dinv[0] = c->dinv32;
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
      const double rr_outer = c->sc_host->rr[0];
      k_fill<float><<<gv, kBlock, 0, s>>>(stride, d32, 0.0f);
      // inner: A32 d = r, from d = 0; its residual starts as r itself
      int it = 0;
      const double target = std::max(inner, 0.5 * tol / relres);
      VIP_TRY((iterate<float, float, 1>(c, m, A32, V, target, maxit - total_it, &it, true, &rr_outer)));
      total_it += it;
      k_add_f32<<<gv, kBlock, 0, s>>>(nvec, x, d32);
    }
  }
  if (project) {
    // phi with zero mean
    k_mean<<<grid_for(n), kBlock, 0, s>>>(n, x, c->partials, c->counter, c->sc);
    k_sub_mean<<<grid_for(n), kBlock, 0, s>>>(n, x, phi, c->sc);
  } else {
    k_copy<double, double><<<grid_for(n), kBlock, 0, s>>>(n, x, phi);
  }
  double lam = lambda_proj;
  if (border) {
    double h = 0.0;
    VIP_HIP_TRY(c, hipMemcpyAsync(&h, x + n, sizeof(double), hipMemcpyDeviceToHost, s));
    VIP_HIP_TRY(c, hipStreamSynchronize(s));
    lam = h;
  } else {
    VIP_HIP_TRY(c, hipStreamSynchronize(s));
  }
  if (st) {
    st->poisson_iters = total_it;
    st->poisson_outer = outer;
    st->poisson_residual = relres;
    st->krylov_used = m == kCG ? VIP_K_PCG : VIP_K_BICGSTAB;
    st->border_lambda = lam;
  }
  if (!std::isfinite(relres)) return set_error(c, VIP_E_NONFINITE, "non-finite Poisson residual");
  if (!converged)
    return set_error(c, VIP_E_NOT_CONVERGED, "Poisson solve stopped at relative residual " +
                                                 std::to_string(relres));
  return VIP_OK;
}

// The two predictor systems H_u u* = r_u, H_v v* = r_v in lockstep (FP64).
int helmholtz_solve(Ctx* c, const double* ru, const double* rv, double* us, double* vs,
                    vip_step_stats* st) {
  const int64_t n = c->n;
  const int64_t stride = n + 1;
  VIP_TRY(ensure_ws(c, 2 * 8 * stride + 2 * stride + 2 * stride, 1));
  double* b = c->ws + 16 * stride;      // [2][stride]
  double* x = c->ws + 18 * stride;      // [2][stride]
  hipStream_t s = c->stream;
  k_copy<double, double><<<grid_for(n), kBlock, 0, s>>>(n, ru, b);
  k_copy<double, double><<<grid_for(n), kBlock, 0, s>>>(n, rv, b + stride);
  // start from the right-hand side (the operators are close to the identity)
  k_copy<double, double><<<grid_for(n), kBlock, 0, s>>>(n, ru, x);
  k_copy<double, double><<<grid_for(n), kBlock, 0, s>>>(n, rv, x + stride);
  Mat<double> H{n, 0, c->sys.ptr, c->sys.cols, {c->sys.val[1], c->sys.val[2]}};
  Vec<double> V = make_vec<double>(c->ws, stride, 2, x);
  V.dinv[0] = c->dinv[1];
  V.dinv[1] = c->dinv[2];
  const double tol = c->opt.helmholtz_tol;
  int total = 0;
  double worst = 0.0;
  bool converged = false;
  for (int outer = 0; outer < 10; ++outer) {
    VIP_TRY((residual<double, double, double, 2>(c, H, x, b, V.r, stride)));
    double bb[2] = {c->sc_host->bb[0], c->sc_host->bb[1]};
    worst = 0.0;
    for (int k = 0; k < 2; ++k)
      worst = std::max(worst, bb[k] > 0.0 ? std::sqrt(c->sc_host->rr[k] / bb[k]) : 0.0);
    if (worst <= tol) {
      converged = true;
      break;
    }
    if (total >= c->opt.max_iters) break;
    // a system whose b is zero is solved by x = 0 exactly: give it a unit norm
    for (int k = 0; k < 2; ++k) if (bb[k] == 0.0) bb[k] = 1.0;
    int it = 0;
    VIP_TRY((iterate<double, double, 2>(c, kBiCGStab, H, V, tol, c->opt.max_iters - total, &it, false, bb)));
    total += it;
  }
  k_copy<double, double><<<grid_for(n), kBlock, 0, s>>>(n, x, us);
  k_copy<double, double><<<grid_for(n), kBlock, 0, s>>>(n, x + stride, vs);
  VIP_HIP_TRY(c, hipGetLastError());
  if (st) {
    st->helmholtz_iters = total;
    st->helmholtz_residual = worst;
  }
  if (!std::isfinite(worst)) return set_error(c, VIP_E_NONFINITE, "non-finite predictor residual");
  if (!converged)
    return set_error(c, VIP_E_NOT_CONVERGED, "predictor solve stopped at relative residual " +
                                                 std::to_string(worst));
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

int ell_apply(Ctx* c, const Ell& e, int vs, const double* x, double* y) {
  if (e.nrows == 0) return VIP_OK;
  k_apply<<<grid_for(e.nrows), kBlock, 0, c->stream>>>(e.nrows, e.ptr, e.cols, e.val[vs], x, y);
  VIP_HIP_TRY(c, hipGetLastError());
  return VIP_OK;
}

}  // namespace vip
