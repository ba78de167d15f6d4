// Per-step kernels of the fractional step (eqs. 12-15) built on the VIP
// operators: convection flux with Adams-Bashforth blending and the
// Crank-Nicolson right-hand side (one fused pass), the VIP divergence, and the
// projection with the pressure update (one fused pass).
#include <hip/hip_runtime.h>

#include <cmath>

#include "vip_internal.h"

namespace vip {

namespace {

struct Op {
  const int64_t* ptr;
  const int32_t* cols;
  const double* val;
};

// (A f)_i and (A g)_i sharing the column reads.
__device__ __forceinline__ void row2(const Op& A, int64_t i, const double* f, const double* g,
                                     double* af, double* ag) {
  const int64_t sl = i / kSlice;
  const int64_t base = A.ptr[sl] + (i % kSlice);
  const int64_t w = (A.ptr[sl + 1] - A.ptr[sl]) / kSlice;
  double a = 0.0, b = 0.0;
  for (int64_t k = 0; k < w; ++k) {
    const int64_t q = base + k * kSlice;
    const int32_t j = A.cols[q];
    const double v = A.val[q];
    a += v * f[j];
    b += v * g[j];
  }
  *af = a;
  *ag = b;
}

__device__ __forceinline__ double row1(const Op& A, int64_t i, const double* f) {
  const int64_t sl = i / kSlice;
  const int64_t base = A.ptr[sl] + (i % kSlice);
  const int64_t w = (A.ptr[sl + 1] - A.ptr[sl]) / kSlice;
  double a = 0.0;
  for (int64_t k = 0; k < w; ++k) {
    const int64_t q = base + k * kSlice;
    a += A.val[q] * f[A.cols[q]];
  }
  return a;
}

struct Vips {
  Op op[4];
  const double* d_ew;
  const double* d_ns;
};

// Convection flux of Section 4.1 item 1 at interior node i.
__device__ __forceinline__ void flux(const Vips& V, int64_t i, const double* u, const double* v,
                                     double* nx, double* ny) {
  double ue, ve, uw, vw, un, vn, us, vs;
  row2(V.op[0], i, u, v, &ue, &ve);
  row2(V.op[1], i, u, v, &uw, &vw);
  row2(V.op[2], i, u, v, &un, &vn);
  row2(V.op[3], i, u, v, &us, &vs);
  const double dew = V.d_ew[i], dns = V.d_ns[i];
  *nx = (ue * ue - uw * uw) / dew + (un * vn - us * vs) / dns;
  *ny = (ue * ve - uw * vw) / dew + (vn * vn - vs * vs) / dns;
}

struct Bnd {
  const int32_t* bpos;
  const int32_t* kind;
  const double* nx;
  const double* ny;
  const double* val;   // [nb][2]
  double two_d;        // 2 * vip_offset * h (scale of the Neumann rows)
};

// Right-hand sides of the two predictor systems (eq. 12 multiplied by dt).
__global__ void k_predictor_rhs(int64_t n, Op m00, Op lap, Vips V, Bnd B, const double* u,
                                const double* v, const double* p, double* nprev, int first,
                                double dt, double re, int exact_id, double* ru, double* rv) {
  const int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
  if (i >= n) return;
  const int32_t k = B.bpos[i];
  if (k >= 0) {
    nprev[i] = 0.0;
    nprev[n + i] = 0.0;
    const int32_t kind = B.kind[k];
    const bool normal_is_y = fabs(B.ny[k]) >= fabs(B.nx[k]);
    const bool u_held = kind == VIP_BC_DIRICHLET || (kind == VIP_BC_SLIP && !normal_is_y);
    const bool v_held = kind == VIP_BC_DIRICHLET || (kind == VIP_BC_SLIP && normal_is_y);
    const double out = kind == VIP_BC_OUTLET ? B.two_d * re * p[i] : 0.0;
    ru[i] = u_held ? B.val[2 * k] : out * B.nx[k];
    rv[i] = v_held ? B.val[2 * k + 1] : out * B.ny[k];
    return;
  }
  double nx, ny;
  flux(V, i, u, v, &nx, &ny);
  const double px = first ? nx : nprev[i];
  const double py = first ? ny : nprev[n + i];
  nprev[i] = nx;
  nprev[n + i] = ny;
  const double cx = 1.5 * nx - 0.5 * px;
  const double cy = 1.5 * ny - 0.5 * py;
  const double c = dt / (2.0 * re);
  // (I + c Delta) u with I = D^[0,0] (or the identity), sharing the column reads
  const int64_t sl = i / kSlice;
  const int64_t base = m00.ptr[sl] + (i % kSlice);
  const int64_t w = (m00.ptr[sl + 1] - m00.ptr[sl]) / kSlice;
  double au = 0.0, av = 0.0;
  for (int64_t t = 0; t < w; ++t) {
    const int64_t q = base + t * kSlice;
    const int32_t j = m00.cols[q];
    const double id = exact_id ? (j == static_cast<int32_t>(i) ? 1.0 : 0.0) : m00.val[q];
    const double r = id + c * lap.val[q];
    au += r * u[j];
    av += r * v[j];
  }
  ru[i] = au - dt * cx;
  rv[i] = av - dt * cy;
}

// b = div(u*) / dt at interior nodes, 0 on boundary rows (eq. 13).
__global__ void k_divergence(int64_t n, Vips V, const int32_t* bpos, const double* u, const double* v,
                             double scale, double* b) {
  const int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
  if (i >= n) return;
  if (bpos[i] >= 0) {
    b[i] = 0.0;
    return;
  }
  const double ue = row1(V.op[0], i, u), uw = row1(V.op[1], i, u);
  const double vn = row1(V.op[2], i, v), vs = row1(V.op[3], i, v);
  b[i] = ((ue - uw) / V.d_ew[i] + (vn - vs) / V.d_ns[i]) * scale;
}

// u = u* - dt grad phi at interior nodes (u = u* on boundary nodes), eq. 14;
// p = phi - (dt / 2 Re) Delta phi, eq. 15.
__global__ void k_project(int64_t n, Vips V, Op lap, const int32_t* bpos, const double* us,
                          const double* vs, const double* phi, double dt, double c, double* u,
                          double* v, double* p) {
  const int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
  if (i >= n) return;
  if (bpos[i] >= 0) {
    u[i] = us[i];
    v[i] = vs[i];
  } else {
    const double pe = row1(V.op[0], i, phi), pw = row1(V.op[1], i, phi);
    const double pn = row1(V.op[2], i, phi), ps = row1(V.op[3], i, phi);
    u[i] = us[i] - dt * ((pe - pw) / V.d_ew[i]);
    v[i] = vs[i] - dt * ((pn - ps) / V.d_ns[i]);
  }
  p[i] = phi[i] - c * row1(lap, i, phi);
}

__global__ void k_flux_only(int64_t n, Vips V, const int32_t* bpos, const double* u, const double* v,
                            double* nx, double* ny) {
  const int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
  if (i >= n) return;
  if (bpos[i] >= 0) {
    nx[i] = 0.0;
    ny[i] = 0.0;
    return;
  }
  flux(V, i, u, v, &nx[i], &ny[i]);
}

__global__ void k_gradient(int64_t n, Vips V, const int32_t* bpos, const double* f, double* gx,
                           double* gy) {
  const int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
  if (i >= n) return;
  if (bpos[i] >= 0) {
    gx[i] = 0.0;
    gy[i] = 0.0;
    return;
  }
  gx[i] = (row1(V.op[0], i, f) - row1(V.op[1], i, f)) / V.d_ew[i];
  gy[i] = (row1(V.op[2], i, f) - row1(V.op[3], i, f)) / V.d_ns[i];
}

Vips vips_of(Ctx* c) {
  Vips V;
  for (int k = 0; k < 4; ++k) V.op[k] = Op{c->vipop[k].ptr, c->vipop[k].cols, c->vipop[k].val[0]};
  V.d_ew = c->d_ew;
  V.d_ns = c->d_ns;
  return V;
}

}  // namespace

int assemble_helmholtz(Ctx* c, double dt, double re);

int step(Ctx* c, double* u, double* v, double* p, double dt, double re, vip_step_stats* st) {
  const int64_t n = c->n;
  if (!c->assembled || dt != c->cur_dt || re != c->cur_re) {
    VIP_TRY(assemble_helmholtz(c, dt, re));
    c->have_prev_n = false;   // AB2 restarts after a change of dt or Re
    c->learn.have_eprev = false;
  }
  if (!c->stepbuf) VIP_TRY(dalloc(c, &c->stepbuf, 5 * n));
  double* ru = c->stepbuf;
  double* rv = ru + n;
  double* us = rv + n;
  double* vs = us + n;
  double* b = vs + n;
  hipStream_t s = c->stream;
  const Vips V = vips_of(c);
  const Op m00{c->node.ptr, c->node.cols, c->node.val[0]};
  const Op lap{c->node.ptr, c->node.cols, c->node.val[1]};
  const Bnd B{c->bpos, c->bkind, c->bnx, c->bny, c->bval, 2.0 * c->opt.vip_offset * c->h};
  k_predictor_rhs<<<grid_for(n), kBlock, 0, s>>>(n, m00, lap, V, B, u, v, p, c->nprev,
                                                  c->have_prev_n ? 0 : 1, dt, re,
                                                  c->opt.identity == VIP_I_EXACT ? 1 : 0, ru, rv);
  VIP_HIP_TRY(c, hipGetLastError());
  int rc_h = helmholtz_solve(c, ru, rv, us, vs, st);
  if (rc_h != VIP_OK && rc_h != VIP_E_NOT_CONVERGED) return rc_h;
  k_divergence<<<grid_for(n), kBlock, 0, s>>>(n, V, c->bpos, us, vs, 1.0 / dt, b);
  VIP_HIP_TRY(c, hipGetLastError());
  const int ws = c->opt.warmstart;
  const bool warm = ws != VIP_WS_ZERO && c->have_prev_phi;
  const bool predict = (ws == VIP_WS_LEARNED || ws == VIP_WS_EXTRAP) && c->have_prev_phi;
  const bool capture = c->have_prev_phi && static_cast<int>(c->learn.snaps.size()) < c->learn.capacity;
  const bool track = predict || capture;
  if (st) {
    st->warm_start = warm ? VIP_WS_PREV : VIP_WS_ZERO;
    st->warm_ratio = 0.0;
    st->warm_alpha = 0.0;
    st->warm_beta = 0.0;
  }
  if (track) VIP_TRY(learn_prepare(c, b, c->phi, ws == VIP_WS_LEARNED || capture));
  if (predict) VIP_TRY(learn_warm_start(c, ws, b, c->phi, st));
  int rc_p = poisson_solve(c, b, c->phi, c->opt.poisson_tol, warm, st);
  if (rc_p != VIP_OK && rc_p != VIP_E_NOT_CONVERGED) return rc_p;
  if (track) {
    VIP_TRY(learn_finish(c, b, c->phi, capture));
  } else {
    c->learn.have_eprev = false;   // the chain of increments is not followed
  }
  k_project<<<grid_for(n), kBlock, 0, s>>>(n, V, lap, c->bpos, us, vs, c->phi, dt, dt / (2.0 * re), u,
                                            v, p);
  VIP_HIP_TRY(c, hipGetLastError());
  VIP_HIP_TRY(c, hipStreamSynchronize(s));
  c->have_prev_n = true;
  c->have_prev_phi = true;
  if (rc_h != VIP_OK) return rc_h;
  return rc_p;
}

int convection(Ctx* c, const double* u, const double* v, double* nx, double* ny) {
  k_flux_only<<<grid_for(c->n), kBlock, 0, c->stream>>>(c->n, vips_of(c), c->bpos, u, v, nx, ny);
  VIP_HIP_TRY(c, hipGetLastError());
  VIP_HIP_TRY(c, hipStreamSynchronize(c->stream));
  return VIP_OK;
}

int divergence(Ctx* c, const double* u, const double* v, double* d) {
  k_divergence<<<grid_for(c->n), kBlock, 0, c->stream>>>(c->n, vips_of(c), c->bpos, u, v, 1.0, d);
  VIP_HIP_TRY(c, hipGetLastError());
  VIP_HIP_TRY(c, hipStreamSynchronize(c->stream));
  return VIP_OK;
}

int gradient(Ctx* c, const double* f, double* gx, double* gy) {
  k_gradient<<<grid_for(c->n), kBlock, 0, c->stream>>>(c->n, vips_of(c), c->bpos, f, gx, gy);
  VIP_HIP_TRY(c, hipGetLastError());
  VIP_HIP_TRY(c, hipStreamSynchronize(c->stream));
  return VIP_OK;
}

}  // namespace vip
