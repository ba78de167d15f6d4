// Per-step kernels of the fractional step (eqs. 12-15) built on the VIP
// operators: convection flux with Adams-Bashforth blending and the
// Crank-Nicolson right-hand side (one fused pass), the VIP divergence, and the
// projection with the pressure update (one fused pass).
#include <hip/hip_runtime.h>

#include <cmath>

#include "tile.h"
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
    a = fma(v, f[j], a);
    b = fma(v, g[j], b);
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
    a = fma(A.val[q], f[A.cols[q]], a);
  }
  return a;
}

struct Vips {
  Op op[4];
  const double* d_ew;
  const double* d_ns;
};

// Canonical nodes (all six per-step rows lattice-interior): the reference weights and the
// lattice map replace the column and value streams.  Sums run in slot order with explicit fused
// multiply-adds, as in row1/row2, so both paths give the same bits.
struct VC {
  const int32_t* cpix;              // nullptr: every node takes the sliced-ELL path
  const int32_t* node_of;
  int W;
  int8_t dx0[kVcOps][kVcRows];
  int8_t len[kVcOps][kVcRows];
  uint8_t used[kVcRows];
  double w[kVcOps + 1][kMaxTaps];
};

// Row products of node i from the sliced ELL.
struct EllRows {
  const Vips& V;
  const Op& lap;
  int64_t i;
  __device__ __forceinline__ double vip(int o, const double* f) const { return row1(V.op[o], i, f); }
  __device__ __forceinline__ void vip2(int o, const double* f, const double* g, double* a, double* b) const {
    row2(V.op[o], i, f, g, a, b);
  }
  __device__ __forceinline__ double laplacian(const double* f) const { return row1(lap, i, f); }
  // (D^[0,0] + c Delta) applied to u and v (D^[0,0] replaced by I when exact_id)
  __device__ __forceinline__ void helm2(const Op& m00, const int32_t* rowlen, int exact_id, double c,
                                        const double* u, const double* v, double* au, double* av) const {
    const int64_t sl = i / kSlice;
    const int64_t base = m00.ptr[sl] + (i % kSlice);
    const int w = rowlen[i];   // padding slots hold column 0 and must not meet the identity test
    double a = 0.0, b = 0.0;
    for (int t = 0; t < w; ++t) {
      const int64_t q = base + static_cast<int64_t>(t) * kSlice;
      const int32_t j = m00.cols[q];
      const double id = exact_id ? (j == static_cast<int32_t>(i) ? 1.0 : 0.0) : m00.val[q];
      const double r = fma(c, lap.val[q], id);
      a = fma(r, u[j], a);
      b = fma(r, v[j], b);
    }
    *au = a;
    *av = b;
  }
};

// Row products of a canonical node: taps rb[d] + dx0 .. + len - 1 per stencil row d.
struct CanonRows {
  const VC& C;
  int32_t rb[kVcRows];
  __device__ __forceinline__ CanonRows(const VC& c, int32_t p, int64_t i) : C(c) {
#pragma unroll
    for (int d = 0; d < kVcRows; ++d)
      rb[d] = d == 3 ? static_cast<int32_t>(i) : (C.used[d] ? C.node_of[p + (d - 3) * C.W] : 0);
  }
  __device__ __forceinline__ double vip(int o, const double* f) const {
    double a = 0.0;
    int k = 0;
#pragma unroll
    for (int d = 0; d < kVcRows; ++d) {
      const int L = C.len[o][d];
      const double* fr = f + rb[d] + C.dx0[o][d];
      for (int t = 0; t < L; ++t) a = fma(C.w[o][k + t], fr[t], a);
      k += L;
    }
    return a;
  }
  __device__ __forceinline__ void vip2(int o, const double* f, const double* g, double* pa, double* pb) const {
    double a = 0.0, b = 0.0;
    int k = 0;
#pragma unroll
    for (int d = 0; d < kVcRows; ++d) {
      const int L = C.len[o][d];
      const int32_t j0 = rb[d] + C.dx0[o][d];
      for (int t = 0; t < L; ++t) {
        const double w = C.w[o][k + t];
        a = fma(w, f[j0 + t], a);
        b = fma(w, g[j0 + t], b);
      }
      k += L;
    }
    *pa = a;
    *pb = b;
  }
  __device__ __forceinline__ double laplacian(const double* f) const {
    double a = 0.0;
    int k = 0;
#pragma unroll
    for (int d = 0; d < kVcRows; ++d) {
      const int L = C.len[4][d];
      const double* fr = f + rb[d] + C.dx0[4][d];
      for (int t = 0; t < L; ++t) a = fma(C.w[kVcOps][k + t], fr[t], a);
      k += L;
    }
    return a;
  }
  __device__ __forceinline__ void helm2(const Op&, const int32_t*, int exact_id, double c, const double* u,
                                        const double* v, double* au, double* av) const {
    double a = 0.0, b = 0.0;
    int k = 0;
#pragma unroll
    for (int d = 0; d < kVcRows; ++d) {
      const int L = C.len[4][d];
      const int dx0 = C.dx0[4][d];
      const int32_t j0 = rb[d] + dx0;
      for (int t = 0; t < L; ++t) {
        const double id = exact_id ? (d == 3 && dx0 + t == 0 ? 1.0 : 0.0) : C.w[4][k + t];
        const double r = fma(c, C.w[kVcOps][k + t], id);
        a = fma(r, u[j0 + t], a);
        b = fma(r, v[j0 + t], b);
      }
      k += L;
    }
    *au = a;
    *av = b;
  }
};

// Convection flux of Section 4.1 item 1 at interior node i.
template <class R>
__device__ __forceinline__ void flux(const R& rows, const Vips& V, int64_t i, const double* u, const double* v,
                                     double* nx, double* ny) {
  double ue, ve, uw, vw, un, vn, us, vs;
  rows.vip2(0, u, v, &ue, &ve);
  rows.vip2(1, u, v, &uw, &vw);
  rows.vip2(2, u, v, &un, &vn);
  rows.vip2(3, u, v, &us, &vs);
  const double dew = V.d_ew[i], dns = V.d_ns[i];
  // products by explicit fused multiply-adds, so that every variant of the kernels gives the same bits
  *nx = fma(ue, ue, -(uw * uw)) / dew + fma(un, vn, -(us * vs)) / dns;
  *ny = fma(ue, ve, -(uw * vw)) / dew + fma(vn, vn, -(vs * vs)) / dns;
}

struct Bnd {
  const int32_t* bpos;
  const int32_t* kind;
  const double* nx;
  const double* ny;
  const double* val;   // [nb][2]
  double two_d;        // 2 * vip_offset * h (scale of the Neumann rows)
  const double* two_db;  // per boundary entry 2 vip_offset h_b on adaptive node sets, else null
};

template <class R>
__device__ __forceinline__ void predictor_interior(const R& rows, int64_t n, int64_t i, const Op& m00,
                                                   const int32_t* rowlen, const Vips& V, const double* u,
                                                   const double* v, double* nprev, int first, double dt,
                                                   double re, int exact_id, double* ru, double* rv) {
  double nx, ny;
  flux(rows, V, i, u, v, &nx, &ny);
  const double px = first ? nx : nprev[i];
  const double py = first ? ny : nprev[n + i];
  nprev[i] = nx;
  nprev[n + i] = ny;
  const double cx = fma(1.5, nx, -(0.5 * px));
  const double cy = fma(1.5, ny, -(0.5 * py));
  double au, av;
  rows.helm2(m00, rowlen, exact_id, dt / (2.0 * re), u, v, &au, &av);
  ru[i] = fma(-dt, cx, au);
  rv[i] = fma(-dt, cy, av);
}

// Right-hand sides of the two predictor systems (eq. 12 multiplied by dt) at node i.
__device__ __forceinline__ void predictor_node(int64_t n, int64_t i, const Op& m00, const Op& lap,
                                               const int32_t* rowlen, const Vips& V, const VC& C, const Bnd& B,
                                               const double* u, const double* v, const double* p, double* nprev,
                                               int first, double dt, double re, int exact_id, double* ru,
                                               double* rv) {
  const int32_t k = B.bpos[i];
  if (k >= 0) {
    nprev[i] = 0.0;
    nprev[n + i] = 0.0;
    const int32_t kind = B.kind[k];
    const bool normal_is_y = fabs(B.ny[k]) >= fabs(B.nx[k]);
    const bool u_held = kind == VIP_BC_DIRICHLET || (kind == VIP_BC_SLIP && !normal_is_y);
    const bool v_held = kind == VIP_BC_DIRICHLET || (kind == VIP_BC_SLIP && normal_is_y);
    const double out = kind == VIP_BC_OUTLET ? (B.two_db ? B.two_db[k] : B.two_d) * re * p[i] : 0.0;
    ru[i] = u_held ? B.val[2 * k] : out * B.nx[k];
    rv[i] = v_held ? B.val[2 * k + 1] : out * B.ny[k];
    return;
  }
  const int32_t cp = C.cpix ? C.cpix[i] : -1;
  if (cp >= 0)
    predictor_interior(CanonRows(C, cp, i), n, i, m00, rowlen, V, u, v, nprev, first, dt, re, exact_id, ru, rv);
  else
    predictor_interior(EllRows{V, lap, i}, n, i, m00, rowlen, V, u, v, nprev, first, dt, re, exact_id, ru, rv);
}

__global__ void k_predictor_rhs(int64_t n, Op m00, Op lap, const int32_t* rowlen, Vips V, VC C, Bnd B,
                                const double* u, const double* v, const double* p, double* nprev, int first,
                                double dt, double re, int exact_id, double* ru, double* rv) {
  const int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
  if (i >= n) return;
  predictor_node(n, i, m00, lap, rowlen, V, C, B, u, v, p, nprev, first, dt, re, exact_id, ru, rv);
}

template <class R>
__device__ __forceinline__ double divergence_at(const R& rows, const Vips& V, int64_t i, const double* u,
                                                const double* v) {
  const double ue = rows.vip(0, u), uw = rows.vip(1, u);
  const double vn = rows.vip(2, v), vs = rows.vip(3, v);
  return (ue - uw) / V.d_ew[i] + (vn - vs) / V.d_ns[i];
}

// b = div(u*) / dt at interior nodes, 0 on boundary rows (eq. 13), at node i.
__device__ __forceinline__ void divergence_node(int64_t i, const Vips& V, const VC& C, const int32_t* bpos,
                                                const double* u, const double* v, double scale, double* b) {
  if (bpos[i] >= 0) {
    b[i] = 0.0;
    return;
  }
  const Op lap{nullptr, nullptr, nullptr};
  const int32_t cp = C.cpix ? C.cpix[i] : -1;
  const double d = cp >= 0 ? divergence_at(CanonRows(C, cp, i), V, i, u, v)
                           : divergence_at(EllRows{V, lap, i}, V, i, u, v);
  b[i] = d * scale;
}

__global__ void k_divergence(int64_t n, Vips V, VC C, const int32_t* bpos, const double* u, const double* v,
                             double scale, double* b) {
  const int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
  if (i >= n) return;
  divergence_node(i, V, C, bpos, u, v, scale, b);
}

template <class R>
__device__ __forceinline__ void project_at(const R& rows, const Vips& V, int64_t i, bool interior,
                                           const double* us, const double* vs, const double* phi, double dt,
                                           double c, double* u, double* v, double* p) {
  if (interior) {
    const double pe = rows.vip(0, phi), pw = rows.vip(1, phi);
    const double pn = rows.vip(2, phi), ps = rows.vip(3, phi);
    u[i] = fma(-dt, (pe - pw) / V.d_ew[i], us[i]);
    v[i] = fma(-dt, (pn - ps) / V.d_ns[i], vs[i]);
  } else {
    u[i] = us[i];
    v[i] = vs[i];
  }
  p[i] = fma(-c, rows.laplacian(phi), phi[i]);
}

// u = u* - dt grad phi at interior nodes (u = u* on boundary nodes), eq. 14;
// p = phi - (dt / 2 Re) Delta phi, eq. 15.
__device__ __forceinline__ void project_node(int64_t i, const Vips& V, const VC& C, const Op& lap,
                                             const int32_t* bpos, const double* us, const double* vs,
                                             const double* phi, double dt, double c, double* u, double* v,
                                             double* p) {
  const bool interior = bpos[i] < 0;
  const int32_t cp = interior && C.cpix ? C.cpix[i] : -1;
  if (cp >= 0)
    project_at(CanonRows(C, cp, i), V, i, true, us, vs, phi, dt, c, u, v, p);
  else
    project_at(EllRows{V, lap, i}, V, i, interior, us, vs, phi, dt, c, u, v, p);
}

__global__ void k_project(int64_t n, Vips V, VC C, Op lap, const int32_t* bpos, const double* us,
                          const double* vs, const double* phi, double dt, double c, double* u,
                          double* v, double* p) {
  const int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
  if (i >= n) return;
  project_node(i, V, C, lap, bpos, us, vs, phi, dt, c, u, v, p);
}

// ---- the same kernels over LDS tiles --------------------------------------------------------------
// Canonical interior nodes on the lattice are taken tile by tile: a block stages the FP64 fields
// the products read over a 64 x 16 pixel tile and a 3-pixel halo (every tap of the reference rows
// lies within 3 pixels; 70 x 22 values per field), and a wavefront computes 4 tile rows, lane =
// column, reading its taps from LDS in the slot order of the per-node path, so the two give the
// same bits.  Boundary nodes, other nodes, and nodes off the lattice are taken one per thread by
// the first blocks of the same launch (tile_walk).
// Halo of the staged frame: 3 pixels for general runs (every tap within 3 pixels), 2 for the
// lattice runs (every tap within 2); SH x SH frames of kTileX + 2 SH by kTileY + 2 SH pixels.
template <int SH>
struct StFrame {
  static constexpr int W = kTileX + 2 * SH;
  static constexpr int H = kTileY + 2 * SH;
};

// Stage NF fields over listed tile k of the partition (0 where a pixel holds no node).  Starts
// and ends with a block barrier.
template <int NF, int SH>
__device__ __forceinline__ void step_stage(const TileView& tv, int64_t k, const double* const (&src)[NF],
                                           double (&t)[NF][StFrame<SH>::H][StFrame<SH>::W], TileMeta& m) {
  constexpr int kStW = StFrame<SH>::W, kStH = StFrame<SH>::H;
  const int tid = static_cast<int>(threadIdx.x);
  __syncthreads();
  if (tid < kTileRecWords) m.w[tid] = tv.rec[k * kTileRecWords + tid];
  __syncthreads();
  const int wave = tid >> 6, lane = tid & 63;
  const int tx = m.tx(), ty = m.ty();
  // the record's row starts cover the 2-pixel halo frame: rows and columns from SH - 2 on here
  constexpr int o = SH - 2;
  auto node_at = [&](int r, int cc) __attribute__((always_inline)) -> int32_t {
    if (r >= o && r < o + kTileLdsH && cc >= o && cc < o + kTileLdsW) {
      const int32_t rs = m.rs(r - o);
      if (rs >= 0) return rs + cc - o;
    }
    const int gx = tx * kTileX + cc - SH, gy = ty * kTileY + r - SH;
    if (gx >= 0 && gx < tv.W && gy >= 0 && gy < tv.H) return tv.node_of[static_cast<int64_t>(gy) * tv.W + gx];
    return -1;
  };
  constexpr int kWaves = kBlock / 64, kRows = (kStH + kWaves - 1) / kWaves, kEdge = kStW - 64;
  static_assert(kEdge > 0 && kEdge * kStH <= kBlock, "step tile staging shape");
  int32_t node[kRows + 1];
#pragma unroll
  for (int j = 0; j < kRows; ++j) {
    const int r = wave + j * kWaves;
    node[j] = r < kStH ? node_at(r, lane) : -1;
  }
  const bool edge = tid < kEdge * kStH;
  node[kRows] = edge ? node_at(tid / kEdge, 64 + tid % kEdge) : -1;
  double val[NF][kRows + 1];
#pragma unroll
  for (int j = 0; j <= kRows; ++j)
#pragma unroll
    for (int f = 0; f < NF; ++f) val[f][j] = node[j] >= 0 ? src[f][node[j]] : 0.0;
#pragma unroll
  for (int j = 0; j < kRows; ++j) {
    const int r = wave + j * kWaves;
    if (r < kStH)
#pragma unroll
      for (int f = 0; f < NF; ++f) t[f][r][lane] = val[f][j];
  }
  if (edge)
#pragma unroll
    for (int f = 0; f < NF; ++f) t[f][tid / kEdge][64 + tid % kEdge] = val[f][kRows];
  __syncthreads();
}

// The canonical runs (dx0, len per stencil row dy = -3..3) of the five operators on a uniform
// lattice with the default options (MLS support of at least 12 neighbours, VIP offset h/2):
// the same on every such node set, whatever its spacing.  Kernels instantiated for it (FIX)
// unroll every tap loop with constant LDS offsets, so the compiler reads each staged value
// once per node for all five operators (21 pixels per field instead of 85 taps); the others
// take the runs from the kernel arguments.  Same taps in the same order: the same bits.
constexpr int8_t kLatDx0[kVcOps][kVcRows] = {{0, 0, -1, -1, -1, 0, 0},
                                             {0, -1, -2, -2, -2, -1, 0},
                                             {0, 0, -1, -2, -2, -1, 0},
                                             {0, -1, -2, -2, -1, 0, 0},
                                             {0, -1, -2, -2, -2, -1, 0}};
constexpr int8_t kLatLen[kVcOps][kVcRows] = {{0, 2, 4, 4, 4, 2, 0},
                                             {0, 2, 4, 4, 4, 2, 0},
                                             {0, 0, 3, 5, 5, 3, 0},
                                             {0, 3, 5, 5, 3, 0, 0},
                                             {0, 3, 5, 5, 5, 3, 0}};

bool vc_is_lattice_shape(const VC& C) {
  for (int o = 0; o < kVcOps; ++o)
    for (int d = 0; d < kVcRows; ++d)
      if (C.len[o][d] != kLatLen[o][d] || (C.len[o][d] > 0 && C.dx0[o][d] != kLatDx0[o][d])) return false;
  return true;
}

// Row products of a canonical node from the staged fields (local row ly, column lx); a field is
// named by the pointer it was staged from.  FIX: the runs are the lattice shape above.
template <int NF, bool FIX = false>
struct LdsRows {
  static constexpr int kSH = FIX ? 2 : 3;   // staged halo; stencil row d (dy = d - 3) at ly + kSH - 3 + d
  static constexpr int kRow = kSH - 3;
  const VC& C;
  const double (&t)[NF][StFrame<kSH>::H][StFrame<kSH>::W];
  const double* const (&src)[NF];
  int ly, lx;
  __device__ __forceinline__ int len(int o, int d) const { return FIX ? kLatLen[o][d] : C.len[o][d]; }
  __device__ __forceinline__ int dx0(int o, int d) const { return FIX ? kLatDx0[o][d] : C.dx0[o][d]; }
  __device__ __forceinline__ int field(const double* f) const { return (NF > 1 && f == src[1]) ? 1 : 0; }
  __device__ __forceinline__ double run(int a, int o, int wo) const {
    double acc = 0.0;
    int k = 0;
#pragma unroll
    for (int d = 0; d < kVcRows; ++d) {
      const int L = len(o, d);
      const double* tr = &t[a][ly + kRow + d][lx + kSH + dx0(o, d)];
      for (int q = 0; q < L; ++q) acc = fma(C.w[wo][k + q], tr[q], acc);
      k += L;
    }
    return acc;
  }
  __device__ __forceinline__ double vip(int o, const double* f) const { return run(field(f), o, o); }
  __device__ __forceinline__ void vip2(int o, const double* f, const double* g, double* pa, double* pb) const {
    const int a0 = field(f), a1 = field(g);
    double a = 0.0, b = 0.0;
    int k = 0;
#pragma unroll
    for (int d = 0; d < kVcRows; ++d) {
      const int L = len(o, d);
      const int c0 = lx + kSH + dx0(o, d);
      for (int q = 0; q < L; ++q) {
        const double w = C.w[o][k + q];
        a = fma(w, t[a0][ly + kRow + d][c0 + q], a);
        b = fma(w, t[a1][ly + kRow + d][c0 + q], b);
      }
      k += L;
    }
    *pa = a;
    *pb = b;
  }
  __device__ __forceinline__ double laplacian(const double* f) const { return run(field(f), 4, kVcOps); }
  __device__ __forceinline__ void helm2(const Op&, const int32_t*, int exact_id, double c, const double* u,
                                        const double* v, double* au, double* av) const {
    const int a0 = field(u), a1 = field(v);
    double a = 0.0, b = 0.0;
    int k = 0;
#pragma unroll
    for (int d = 0; d < kVcRows; ++d) {
      const int L = len(4, d);
      const int dx0 = this->dx0(4, d);
      const int c0 = lx + kSH + dx0;
      for (int q = 0; q < L; ++q) {
        const double id = exact_id ? (d == 3 && dx0 + q == 0 ? 1.0 : 0.0) : C.w[4][k + q];
        const double r = fma(c, C.w[kVcOps][k + q], id);
        a = fma(r, t[a0][ly + kRow + d][c0 + q], a);
        b = fma(r, t[a1][ly + kRow + d][c0 + q], b);
      }
      k += L;
    }
    *au = a;
    *av = b;
  }
};

// The tile rows of the wave: f(node, ly, lane) for each.
template <typename F>
__device__ __forceinline__ void step_rows(const TileView& tv, const TileMeta& m, F&& f) {
  const int wave = static_cast<int>(threadIdx.x >> 6), lane = static_cast<int>(threadIdx.x & 63);
#pragma unroll 1
  for (int k = 0; k < kTileRowsPerWave; ++k) {
    const int64_t row = tile_row_id(tv, m, k);
    if (row >= 0) f(row, wave + k * (kBlock / 64), lane);
  }
}

template <bool FIX>
__global__ void __launch_bounds__(kBlock) k_predictor_rhs_tiles(TileView tv, int64_t n, Op m00, Op lap,
                                                                const int32_t* rowlen, Vips V, VC C, Bnd B,
                                                                const double* u, const double* v,
                                                                const double* p, double* nprev, int first,
                                                                double dt, double re, int exact_id, double* ru,
                                                                double* rv) {
  constexpr int SH = LdsRows<2, FIX>::kSH;
  __shared__ double t[2][StFrame<SH>::H][StFrame<SH>::W];
  __shared__ TileMeta m;
  const double* const src[2] = {u, v};
  tile_walk(
      tv,
      [&](int64_t tk) __attribute__((always_inline)) {
        step_stage<2, SH>(tv, tk, src, t, m);
        step_rows(tv, m, [&](int64_t i, int ly, int lx) __attribute__((always_inline)) {
          predictor_interior(LdsRows<2, FIX>{C, t, src, ly, lx}, n, i, m00, rowlen, V, u, v, nprev, first, dt, re,
                             exact_id, ru, rv);
        });
      },
      [&](int64_t i) __attribute__((always_inline)) {
        predictor_node(n, i, m00, lap, rowlen, V, C, B, u, v, p, nprev, first, dt, re, exact_id, ru, rv);
      });
}

template <bool FIX>
__global__ void __launch_bounds__(kBlock) k_divergence_tiles(TileView tv, Vips V, VC C, const int32_t* bpos,
                                                             const double* u, const double* v, double scale,
                                                             double* b) {
  constexpr int SH = LdsRows<2, FIX>::kSH;
  __shared__ double t[2][StFrame<SH>::H][StFrame<SH>::W];
  __shared__ TileMeta m;
  const double* const src[2] = {u, v};
  tile_walk(
      tv,
      [&](int64_t tk) __attribute__((always_inline)) {
        step_stage<2, SH>(tv, tk, src, t, m);
        step_rows(tv, m, [&](int64_t i, int ly, int lx) __attribute__((always_inline)) {
          b[i] = divergence_at(LdsRows<2, FIX>{C, t, src, ly, lx}, V, i, u, v) * scale;
        });
      },
      [&](int64_t i) __attribute__((always_inline)) { divergence_node(i, V, C, bpos, u, v, scale, b); });
}

template <bool FIX>
__global__ void __launch_bounds__(kBlock) k_project_tiles(TileView tv, Vips V, VC C, Op lap, const int32_t* bpos,
                                                          const double* us, const double* vs, const double* phi,
                                                          double dt, double c, double* u, double* v, double* p) {
  constexpr int SH = LdsRows<1, FIX>::kSH;
  __shared__ double t[1][StFrame<SH>::H][StFrame<SH>::W];
  __shared__ TileMeta m;
  const double* const src[1] = {phi};
  tile_walk(
      tv,
      [&](int64_t tk) __attribute__((always_inline)) {
        step_stage<1, SH>(tv, tk, src, t, m);
        step_rows(tv, m, [&](int64_t i, int ly, int lx) __attribute__((always_inline)) {
          project_at(LdsRows<1, FIX>{C, t, src, ly, lx}, V, i, true, us, vs, phi, dt, c, u, v, p);
        });
      },
      [&](int64_t i) __attribute__((always_inline)) { project_node(i, V, C, lap, bpos, us, vs, phi, dt, c, u, v, p); });
}

__global__ void k_flux_only(int64_t n, Vips V, VC C, const int32_t* bpos, const double* u, const double* v,
                            double* nx, double* ny) {
  const int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
  if (i >= n) return;
  if (bpos[i] >= 0) {
    nx[i] = 0.0;
    ny[i] = 0.0;
    return;
  }
  const Op lap{nullptr, nullptr, nullptr};
  const int32_t cp = C.cpix ? C.cpix[i] : -1;
  if (cp >= 0)
    flux(CanonRows(C, cp, i), V, i, u, v, &nx[i], &ny[i]);
  else
    flux(EllRows{V, lap, i}, V, i, u, v, &nx[i], &ny[i]);
}

template <class R>
__device__ __forceinline__ void gradient_at(const R& rows, const Vips& V, int64_t i, const double* f, double* gx,
                                            double* gy) {
  gx[i] = (rows.vip(0, f) - rows.vip(1, f)) / V.d_ew[i];
  gy[i] = (rows.vip(2, f) - rows.vip(3, f)) / V.d_ns[i];
}

__global__ void k_gradient(int64_t n, Vips V, VC C, const int32_t* bpos, const double* f, double* gx,
                           double* gy) {
  const int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
  if (i >= n) return;
  if (bpos[i] >= 0) {
    gx[i] = 0.0;
    gy[i] = 0.0;
    return;
  }
  const Op lap{nullptr, nullptr, nullptr};
  const int32_t cp = C.cpix ? C.cpix[i] : -1;
  if (cp >= 0)
    gradient_at(CanonRows(C, cp, i), V, i, f, gx, gy);
  else
    gradient_at(EllRows{V, lap, i}, V, i, f, gx, gy);
}

VC vc_of(const Ctx* c) {
  VC C{};
  const VipCanon& S = c->vcanon;
  C.cpix = c->no_canon || S.count == 0 ? nullptr : S.cpix;
  C.node_of = c->lat.node_of;
  C.W = c->lat.W;
  for (int o = 0; o < kVcOps; ++o)
    for (int d = 0; d < kVcRows; ++d) {
      C.dx0[o][d] = S.dx0[o][d];
      C.len[o][d] = S.len[o][d];
    }
  for (int d = 0; d < kVcRows; ++d) C.used[d] = S.used[d];
  for (int o = 0; o <= kVcOps; ++o)
    for (int k = 0; k < kMaxTaps; ++k) C.w[o][k] = S.w[o][k];
  return C;
}

// The step kernels' tile partition, or an empty view (then they run one node per thread).
TileView step_tiles(const Ctx* c) {
  if (c->no_canon || !vc_of(c).cpix || !c->vcanon.tpart.tiles) return TileView();
  return tile_view_of(c->vcanon.tpart, c->tmap, c->lat.node_of, c->lat.W, c->lat.H);
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
    c->nstar = 0;
    c->learn.have_eprev = false;
    c->learn.have_eprev2 = false;
  }
  if (!c->stepbuf) VIP_TRY(dalloc(c, &c->stepbuf, n));
  double* b = c->stepbuf;          // the Poisson right-hand side
  // the predictor right-hand sides, written where the predictor solve reads them
  double* ru = nullptr;
  VIP_TRY(predictor_rhs_buffer(c, &ru));
  double* rv = ru + (n + 1);
  double* us = nullptr;            // the predictor solutions (set by the solve)
  double* vs = nullptr;
  hipStream_t s = c->stream;
  const Vips V = vips_of(c);
  const Op m00{c->node.ptr, c->node.cols, c->node.val[0]};
  const Op lap{c->node.ptr, c->node.cols, c->node.val[1]};
  const Bnd B{c->bpos, c->bkind, c->bnx, c->bny, c->bval, 2.0 * c->opt.vip_offset * c->h, c->two_db};
  const VC C = vc_of(c);
  const TileView T = step_tiles(c);
  const bool fix = vc_is_lattice_shape(C);   // the tiled kernels' unrolled instance applies
  const int64_t tgrid = static_cast<int64_t>(T.tile_blocks) + T.irr_blocks;
  {
    KTimer kt(c, c->ktime[kTimePredRhs], true);
    const int first = c->have_prev_n ? 0 : 1, exact = c->opt.identity == VIP_I_EXACT ? 1 : 0;
    if (T.tiles && fix)
      k_predictor_rhs_tiles<true><<<tgrid, kBlock, 0, s>>>(T, n, m00, lap, c->node.rowlen, V, C, B, u, v, p,
                                                            c->nprev, first, dt, re, exact, ru, rv);
    else if (T.tiles)
      k_predictor_rhs_tiles<false><<<tgrid, kBlock, 0, s>>>(T, n, m00, lap, c->node.rowlen, V, C, B, u, v, p,
                                                             c->nprev, first, dt, re, exact, ru, rv);
    else
      k_predictor_rhs<<<grid_for(n), kBlock, 0, s>>>(n, m00, lap, c->node.rowlen, V, C, B, u, v, p, c->nprev,
                                                      c->have_prev_n ? 0 : 1, dt, re,
                                                      c->opt.identity == VIP_I_EXACT ? 1 : 0, ru, rv);
  }
  VIP_HIP_TRY(c, hipGetLastError());
  int rc_h = helmholtz_solve(c, ru, rv, &us, &vs, st);
  if (rc_h != VIP_OK && rc_h != VIP_E_NOT_CONVERGED) return rc_h;
  if (T.tiles && fix) k_divergence_tiles<true><<<tgrid, kBlock, 0, s>>>(T, V, C, c->bpos, us, vs, 1.0 / dt, b);
  else if (T.tiles) k_divergence_tiles<false><<<tgrid, kBlock, 0, s>>>(T, V, C, c->bpos, us, vs, 1.0 / dt, b);
  else k_divergence<<<grid_for(n), kBlock, 0, s>>>(n, V, C, c->bpos, us, vs, 1.0 / dt, b);
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
    st->warm_gamma = 0.0;
  }
  if (track) VIP_TRY(learn_prepare(c, b, c->phi, ws == VIP_WS_LEARNED || capture));
  if (predict) VIP_TRY(learn_warm_start(c, ws, b, c->phi, st));
  int rc_p = poisson_solve(c, b, c->phi, c->opt.poisson_tol, warm, st);
  if (rc_p != VIP_OK && rc_p != VIP_E_NOT_CONVERGED) return rc_p;
  if (predict) VIP_TRY(learn_warm_stats(c, st));
  if (track) {
    VIP_TRY(learn_finish(c, b, c->phi, capture));
  } else {
    c->learn.have_eprev = false;   // the chain of increments is not followed
    c->learn.have_eprev2 = false;
  }
  if (T.tiles && fix)
    k_project_tiles<true><<<tgrid, kBlock, 0, s>>>(T, V, C, lap, c->bpos, us, vs, c->phi, dt, dt / (2.0 * re), u,
                                                   v, p);
  else if (T.tiles)
    k_project_tiles<false><<<tgrid, kBlock, 0, s>>>(T, V, C, lap, c->bpos, us, vs, c->phi, dt, dt / (2.0 * re), u,
                                                    v, p);
  else
    k_project<<<grid_for(n), kBlock, 0, s>>>(n, V, C, lap, c->bpos, us, vs, c->phi, dt, dt / (2.0 * re), u,
                                              v, p);
  VIP_HIP_TRY(c, hipGetLastError());
  // no wait here: the statistics are final (the solves' last convergence checks are behind
  // us) and the projection completes in stream order, overlapping the caller's next host work
  c->have_prev_n = true;
  c->have_prev_phi = true;
  if (rc_h != VIP_OK) return rc_h;
  return rc_p;
}

int convection(Ctx* c, const double* u, const double* v, double* nx, double* ny) {
  k_flux_only<<<grid_for(c->n), kBlock, 0, c->stream>>>(c->n, vips_of(c), vc_of(c), c->bpos, u, v, nx, ny);
  VIP_HIP_TRY(c, hipGetLastError());
  VIP_HIP_TRY(c, hipStreamSynchronize(c->stream));
  return VIP_OK;
}

int divergence(Ctx* c, const double* u, const double* v, double* d) {
  const TileView T = step_tiles(c);
  const VC C = vc_of(c);
  const int64_t tgrid = static_cast<int64_t>(T.tile_blocks) + T.irr_blocks;
  if (T.tiles && vc_is_lattice_shape(C))
    k_divergence_tiles<true><<<tgrid, kBlock, 0, c->stream>>>(T, vips_of(c), C, c->bpos, u, v, 1.0, d);
  else if (T.tiles)
    k_divergence_tiles<false><<<tgrid, kBlock, 0, c->stream>>>(T, vips_of(c), C, c->bpos, u, v, 1.0, d);
  else
    k_divergence<<<grid_for(c->n), kBlock, 0, c->stream>>>(c->n, vips_of(c), vc_of(c), c->bpos, u, v, 1.0, d);
  VIP_HIP_TRY(c, hipGetLastError());
  VIP_HIP_TRY(c, hipStreamSynchronize(c->stream));
  return VIP_OK;
}

int gradient(Ctx* c, const double* f, double* gx, double* gy) {
  k_gradient<<<grid_for(c->n), kBlock, 0, c->stream>>>(c->n, vips_of(c), vc_of(c), c->bpos, f, gx, gy);
  VIP_HIP_TRY(c, hipGetLastError());
  VIP_HIP_TRY(c, hipStreamSynchronize(c->stream));
  return VIP_OK;
}

}  // namespace vip
