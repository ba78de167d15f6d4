// Stencil build: neighbour search, virtual interpolation points, batched MLS
// shape functions and operator assembly (Sections 3 and 4 of the paper).
//
// Evaluation points come in families, each filling one sliced-ELL operator:
//   node      x_i                               -> D^[0,0] and D^[2,0] + D^[0,2]
//   vip[k]    x_i +- o e_x, x_i +- o e_y        -> Psi^[0,0] at e, w, n, s (interior rows)
//   normal[m] x_b - (m+1) d n_b, per boundary   -> Psi^[0,0] (Neumann rows)
// One thread evaluates one point: a wavefront carries a batch of 64 points of
// one family, each lane accumulating its own 6x6 moment matrix in registers.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <limits>
#include <vector>

#include "vip_internal.h"

namespace vip {

// ---- small device helpers --------------------------------------------------------

// Minimum-image displacement along one axis (L = 0: not periodic).
__device__ __forceinline__ double min_image(double d, double L) {
#pragma clang fp contract(off)
  return L > 0.0 ? d - L * rint(d / L) : d;
}

struct Grid {
  double x0, y0;        // origin of cell (0, 0)
  double cw, ch;        // cell width and height
  int64_t ncx, ncy;
  double Lx, Ly;        // periodic lengths or 0
  const int64_t* start;  // [ncx*ncy + 1]
  const int32_t* items;  // [n]
};

__device__ __forceinline__ int64_t cell_coord(double v, double o, double w, int64_t nc,
                                              double L) {
  if (L > 0.0) {
    double m = v - L * floor(v / L);
    int64_t c = static_cast<int64_t>(floor(m / w));
    return c < 0 ? 0 : (c >= nc ? nc - 1 : c);
  }
  int64_t c = static_cast<int64_t>(floor((v - o) / w));
  return c < 0 ? 0 : (c >= nc ? nc - 1 : c);
}

// Visit every node j with |x_j - q|^2 < R^2 (minimum image), in cell order.
template <class F>
__device__ void for_each_neighbour(const Grid& g, const double* x, const double* y, double qx,
                                   double qy, double R, F&& f) {
#pragma clang fp contract(off)
  int64_t lo[2], hi[2];
  const double q[2] = {qx, qy};
  const double o[2] = {g.x0, g.y0};
  const double w[2] = {g.cw, g.ch};
  const int64_t nc[2] = {g.ncx, g.ncy};
  const double L[2] = {g.Lx, g.Ly};
  bool all[2];
  for (int a = 0; a < 2; ++a) {
    if (L[a] > 0.0) {
      lo[a] = static_cast<int64_t>(floor((q[a] - R) / w[a]));
      hi[a] = static_cast<int64_t>(floor((q[a] + R) / w[a]));
      all[a] = (hi[a] - lo[a] + 1) >= nc[a];
      if (all[a]) { lo[a] = 0; hi[a] = nc[a] - 1; }
    } else {
      lo[a] = static_cast<int64_t>(floor((q[a] - R - o[a]) / w[a]));
      hi[a] = static_cast<int64_t>(floor((q[a] + R - o[a]) / w[a]));
      lo[a] = lo[a] < 0 ? 0 : lo[a];
      hi[a] = hi[a] >= nc[a] ? nc[a] - 1 : hi[a];
      all[a] = false;
    }
  }
  const double R2 = R * R;
  for (int64_t cy = lo[1]; cy <= hi[1]; ++cy) {
    int64_t wy = cy;
    if (L[1] > 0.0) wy = ((cy % nc[1]) + nc[1]) % nc[1];
    for (int64_t cx = lo[0]; cx <= hi[0]; ++cx) {
      int64_t wx = cx;
      if (L[0] > 0.0) wx = ((cx % nc[0]) + nc[0]) % nc[0];
      const int64_t cell = wy * g.ncx + wx;
      for (int64_t t = g.start[cell]; t < g.start[cell + 1]; ++t) {
        const int32_t j = g.items[t];
        const double dx = min_image(x[j] - qx, g.Lx);
        const double dy = min_image(y[j] - qy, g.Ly);
        const double d2 = dx * dx + dy * dy;
        if (d2 < R2) f(j, dx, dy);
      }
    }
  }
}

// ---- cell list -------------------------------------------------------------------------

__global__ void k_cell_count(const double* x, const double* y, int64_t n, Grid g,
                             int64_t* cell_of, int64_t* count) {
  int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
  if (i >= n) return;
  const int64_t cx = cell_coord(x[i], g.x0, g.cw, g.ncx, g.Lx);
  const int64_t cy = cell_coord(y[i], g.y0, g.ch, g.ncy, g.Ly);
  const int64_t c = cy * g.ncx + cx;
  cell_of[i] = c;
  atomicAdd(reinterpret_cast<unsigned long long*>(&count[c]), 1ull);
}

__global__ void k_cell_fill(int64_t n, const int64_t* cell_of, const int64_t* start,
                            int64_t* cursor, int32_t* items) {
  int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
  if (i >= n) return;
  const int64_t c = cell_of[i];
  const unsigned long long k = atomicAdd(reinterpret_cast<unsigned long long*>(&cursor[c]), 1ull);
  items[start[c] + static_cast<int64_t>(k)] = static_cast<int32_t>(i);
}

// ---- scan (exclusive prefix sum of int64) -----------------------------------------------

constexpr int kScanBlock = 1024;

__global__ void k_scan_block_sums(const int64_t* in, int64_t n, int64_t per_block, int64_t* sums) {
  __shared__ int64_t s[kScanBlock];
  const int64_t b0 = blockIdx.x * per_block;
  int64_t acc = 0;
  for (int64_t i = b0 + threadIdx.x; i < b0 + per_block && i < n; i += blockDim.x) acc += in[i];
  s[threadIdx.x] = acc;
  __syncthreads();
  for (int off = blockDim.x / 2; off > 0; off >>= 1) {
    if (static_cast<int>(threadIdx.x) < off) s[threadIdx.x] += s[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) sums[blockIdx.x] = s[0];
}

// Single-block exclusive scan of `m` values (m small), also writes the total.
__global__ void k_scan_small(int64_t* v, int64_t m, int64_t* total) {
  __shared__ int64_t s[kScanBlock];
  __shared__ int64_t carry;
  if (threadIdx.x == 0) carry = 0;
  __syncthreads();
  for (int64_t base = 0; base < m; base += blockDim.x) {
    const int64_t i = base + threadIdx.x;
    const int64_t val = i < m ? v[i] : 0;
    s[threadIdx.x] = val;
    __syncthreads();
    for (int off = 1; off < static_cast<int>(blockDim.x); off <<= 1) {
      int64_t t = static_cast<int>(threadIdx.x) >= off ? s[threadIdx.x - off] : 0;
      __syncthreads();
      s[threadIdx.x] += t;
      __syncthreads();
    }
    if (i < m) v[i] = carry + s[threadIdx.x] - val;
    __syncthreads();
    if (threadIdx.x == blockDim.x - 1) carry += s[threadIdx.x];
    __syncthreads();
  }
  if (threadIdx.x == 0) *total = carry;
}

// Sequential scan inside each chunk (one thread per chunk) starting from the chunk offset.
__global__ void k_scan_apply(const int64_t* in, int64_t* out, int64_t n, int64_t per_block,
                             const int64_t* offsets) {
  __shared__ int64_t s[kScanBlock];
  const int64_t b0 = blockIdx.x * per_block;
  const int64_t chunk = (per_block + blockDim.x - 1) / blockDim.x;
  const int64_t c0 = b0 + threadIdx.x * chunk;
  int64_t acc = 0;
  for (int64_t i = c0; i < c0 + chunk && i < b0 + per_block && i < n; ++i) acc += in[i];
  s[threadIdx.x] = acc;
  __syncthreads();
  // exclusive scan of the per-thread chunk sums
  for (int off = 1; off < static_cast<int>(blockDim.x); off <<= 1) {
    int64_t t = static_cast<int>(threadIdx.x) >= off ? s[threadIdx.x - off] : 0;
    __syncthreads();
    s[threadIdx.x] += t;
    __syncthreads();
  }
  int64_t run = offsets[blockIdx.x] + s[threadIdx.x] - acc;
  for (int64_t i = c0; i < c0 + chunk && i < b0 + per_block && i < n; ++i) {
    const int64_t v = in[i];
    out[i] = run;
    run += v;
  }
}

int scan_i64(Ctx* c, const int64_t* in, int64_t* out, int64_t n, int64_t* total_host) {
  if (n <= 0) {
    *total_host = 0;
    return VIP_OK;
  }
  const int64_t per_block = 16 * kScanBlock;
  const int64_t nblocks = (n + per_block - 1) / per_block;
  int64_t* sums = nullptr;
  VIP_TRY(dalloc(c, &sums, nblocks + 1));
  k_scan_block_sums<<<nblocks, kScanBlock, 0, c->stream>>>(in, n, per_block, sums);
  k_scan_small<<<1, kScanBlock, 0, c->stream>>>(sums, nblocks, sums + nblocks);
  k_scan_apply<<<nblocks, kScanBlock, 0, c->stream>>>(in, out, n, per_block, sums);
  hipError_t e = hipMemcpyAsync(total_host, sums + nblocks, sizeof(int64_t), hipMemcpyDeviceToHost,
                                c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  dfree(sums);
  if (e != hipSuccess) return set_error(c, VIP_E_HIP, std::string("scan: ") + hipGetErrorString(e));
  return VIP_OK;
}

// ---- evaluation points ------------------------------------------------------------------

// VIPs of interior nodes, moved onto the tangent line of the nearest boundary
// node when they fall outside it (the paper leaves near-boundary VIPs open).
__global__ void k_vip_points(Grid g, const double* x, const double* y, int64_t n,
                             const int32_t* bpos, const double* bnx, const double* bny,
                             double off0, double rho00, const double* scale, double* px, double* py,
                             double* dew, double* dns) {
#pragma clang fp contract(off)
  int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
  if (i >= n) return;
  // offset and support radius of this node (scaled by its local spacing on adaptive sets)
  const double off = scale ? off0 * scale[i] : off0;
  const double rho0 = scale ? rho00 * scale[i] : rho00;
  const double dirx[4] = {1.0, -1.0, 0.0, 0.0};
  const double diry[4] = {0.0, 0.0, 1.0, -1.0};
  const double xi = x[i], yi = y[i];
  double vx[4], vy[4];
  for (int k = 0; k < 4; ++k) {
    vx[k] = xi + off * dirx[k];
    vy[k] = yi + off * diry[k];
  }
  if (bpos[i] >= 0) {
    for (int k = 0; k < 4; ++k) {
      px[k * n + i] = 0.0;
      py[k * n + i] = 0.0;
    }
    dew[i] = 1.0;
    dns[i] = 1.0;
    return;
  }
  double best_d2[4];
  int32_t best_k[4];
  int32_t best_j[4];
  for (int k = 0; k < 4; ++k) {
    best_d2[k] = INFINITY;
    best_k[k] = -1;
    best_j[k] = -1;
  }
  // boundary nodes within rho0 of x_i (plain differences: boundaries are never periodic)
  for_each_neighbour(g, x, y, xi, yi, rho0, [&](int32_t j, double, double) {
    const int32_t bk = bpos[j];
    if (bk < 0) return;
    const double ex = x[j] - xi, ey = y[j] - yi;
    if (!(ex * ex + ey * ey < rho0 * rho0)) return;
    for (int k = 0; k < 4; ++k) {
      const double dx = x[j] - vx[k], dy = y[j] - vy[k];
      const double d2 = dx * dx + dy * dy;
      if (d2 < best_d2[k] || (d2 == best_d2[k] && bk < best_k[k])) {
        best_d2[k] = d2;
        best_k[k] = bk;
        best_j[k] = j;
      }
    }
  });
  for (int k = 0; k < 4; ++k) {
    if (best_k[k] >= 0) {
      const int32_t b = best_k[k], j = best_j[k];
      const double nx = bnx[b], ny = bny[b];
      const double side = nx * (vx[k] - x[j]) + ny * (vy[k] - y[j]);
      if (side > 0.0) {
        const double ndir = nx * dirx[k] + ny * diry[k];
        double t = (nx * (x[j] - xi) + ny * (y[j] - yi)) / ndir;
        t = t < 0.0 ? 0.0 : (t > off ? off : t);
        vx[k] = xi + t * dirx[k];
        vy[k] = yi + t * diry[k];
      }
    }
    px[k * n + i] = vx[k];
    py[k * n + i] = vy[k];
  }
  const double ax = vx[0] - vx[1], ay = vy[0] - vy[1];
  const double bx = vx[2] - vx[3], by = vy[2] - vy[3];
  dew[i] = sqrt(ax * ax + ay * ay);
  dns[i] = sqrt(bx * bx + by * by);
}

__global__ void k_normal_points(const double* x, const double* y, const int64_t* bidx,
                                const double* bnx, const double* bny, int64_t nb, double d0,
                                const double* bscale, double* px1, double* py1, double* px2, double* py2) {
#pragma clang fp contract(off)
  int64_t k = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
  if (k >= nb) return;
  const int64_t b = bidx[k];
  const double d = bscale ? d0 * bscale[k] : d0;
  px1[k] = x[b] - 1.0 * d * bnx[k];
  py1[k] = y[b] - 1.0 * d * bny[k];
  px2[k] = x[b] - 2.0 * d * bnx[k];
  py2[k] = y[b] - 2.0 * d * bny[k];
}

// ---- neighbour counts with support growth ---------------------------------------------

struct Family {
  int64_t nrows;
  const double* px;     // point coordinates per row
  const double* py;
  const int32_t* bpos;  // non-null: rows with bpos >= 0 are inactive (VIP families)
  const double* scale;  // non-null: the row's support radius is rho0 * scale[row] (local spacing
                        // of the node the point belongs to over the reference spacing)
};

__global__ void k_count(Grid g, const double* x, const double* y, Family f, double rho0,
                        int min_nb, int32_t* rowlen, double* rho_out,
                        unsigned long long* fail_row) {
  int64_t r = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
  if (r >= f.nrows) return;
  if (f.bpos && f.bpos[r] >= 0) {
    rowlen[r] = 0;
    rho_out[r] = 0.0;
    return;
  }
  const double qx = f.px[r], qy = f.py[r];
  double R = f.scale ? rho0 * f.scale[r] : rho0;
  int cnt = 0;
  for (int grow = 0; grow <= 2; ++grow) {
    cnt = 0;
    for_each_neighbour(g, x, y, qx, qy, R, [&](int32_t, double, double) { ++cnt; });
    if (cnt >= min_nb) break;
    if (grow < 2) R *= 1.25;
  }
  if (cnt < min_nb || cnt > kMaxWidth) {
    atomicMin(fail_row, static_cast<unsigned long long>(r));
    cnt = 0;
  }
  rowlen[r] = cnt;
  rho_out[r] = R;
}

// Neighbour lists in ascending node order, written to the ELL columns.
__global__ void k_fill(Grid g, const double* x, const double* y, Family f, const double* rho,
                       const int32_t* rowlen, const int64_t* ptr, int32_t* cols) {
  int64_t r = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
  if (r >= f.nrows) return;
  const int32_t K = rowlen[r];
  if (K == 0) return;
  int32_t list[kMaxWidth];
  int cnt = 0;
  for_each_neighbour(g, x, y, f.px[r], f.py[r], rho[r], [&](int32_t j, double, double) {
    if (cnt >= kMaxWidth) return;
    int p = cnt++;
    while (p > 0 && list[p - 1] > j) {
      list[p] = list[p - 1];
      --p;
    }
    list[p] = j;
  });
  const int64_t s = r / kSlice, l = r % kSlice;
  const int64_t base = ptr[s] + l;
  for (int k = 0; k < K && k < cnt; ++k) cols[base + static_cast<int64_t>(k) * kSlice] = list[k];
}

// ---- slice layout -------------------------------------------------------------------------

__global__ void k_slice_width(const int32_t* rowlen, int64_t nrows, int64_t nslices, int32_t* width,
                              int64_t* slots) {
  int64_t s = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
  if (s >= nslices) return;
  int32_t w = 0;
  for (int64_t r = s * kSlice; r < (s + 1) * kSlice && r < nrows; ++r) w = max(w, rowlen[r]);
  width[s] = w;
  slots[s] = static_cast<int64_t>(w) * kSlice;
}

// Padding slots get column 0: those of short rows and every slot of the lanes past the last
// row in a ragged last slice (launched over all nslices * kSlice lanes), so that no stored
// column is ever uninitialised.
__global__ void k_fill_padding(const int64_t* ptr, const int32_t* width, const int32_t* rowlen,
                               int64_t nrows, int64_t nlanes, int32_t* cols) {
  int64_t r = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
  if (r >= nlanes) return;
  const int64_t s = r / kSlice, l = r % kSlice;
  const int32_t first = r < nrows ? rowlen[r] : 0;
  for (int32_t k = first; k < width[s]; ++k) cols[ptr[s] + static_cast<int64_t>(k) * kSlice + l] = 0;
}

int ell_layout(Ctx* c, Ell& e) {
  e.nslices = (e.nrows + kSlice - 1) / kSlice;
  VIP_TRY(dalloc(c, &e.width, e.nslices));
  VIP_TRY(dalloc(c, &e.ptr, e.nslices + 1));
  int64_t* slots = nullptr;
  VIP_TRY(dalloc(c, &slots, e.nslices + 1));
  if (e.nslices > 0) {
    k_slice_width<<<grid_for(e.nslices), kBlock, 0, c->stream>>>(e.rowlen, e.nrows, e.nslices,
                                                                  e.width, slots);
  }
  int64_t total = 0;
  int rc = scan_i64(c, slots, e.ptr, e.nslices, &total);
  dfree(slots);
  VIP_TRY(rc);
  VIP_HIP_TRY(c, hipMemcpyAsync(e.ptr + e.nslices, &total, sizeof(int64_t), hipMemcpyHostToDevice,
                                c->stream));
  e.nnz_slots = total;
  VIP_TRY(dalloc(c, &e.cols, total));
  if (e.nrows > 0)
    k_fill_padding<<<grid_for(e.nslices * kSlice), kBlock, 0, c->stream>>>(e.ptr, e.width, e.rowlen, e.nrows,
                                                                            e.nslices * kSlice, e.cols);
  // largest width and stored entries
  std::vector<int32_t> w(static_cast<size_t>(e.nslices)), rl(static_cast<size_t>(e.nrows));
  if (e.nslices > 0)
    VIP_HIP_TRY(c, hipMemcpyAsync(w.data(), e.width, sizeof(int32_t) * e.nslices,
                                  hipMemcpyDeviceToHost, c->stream));
  if (e.nrows > 0)
    VIP_HIP_TRY(c, hipMemcpyAsync(rl.data(), e.rowlen, sizeof(int32_t) * e.nrows,
                                  hipMemcpyDeviceToHost, c->stream));
  VIP_HIP_TRY(c, hipStreamSynchronize(c->stream));
  e.max_width = 0;
  for (int32_t v : w) e.max_width = std::max<int64_t>(e.max_width, v);
  e.nnz = 0;
  for (int32_t v : rl) e.nnz += v;
  return VIP_OK;
}

// ---- row-relative int16 columns ------------------------------------------------------------------

// One wavefront per slice: dcols of every slot of the slice (col - row for stored entries, 0 in
// padding), and dfit[slice] = 1 when every stored column lies within +-32767 of its row
__global__ void k_deltas(const int64_t* ptr, const int32_t* width, const int32_t* rowlen, const int32_t* cols,
                         int64_t nrows, int64_t nslices, int16_t* dcols, uint8_t* dfit) {
  const int64_t s = (blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x) / kSlice;
  const int l = static_cast<int>(threadIdx.x % kSlice);
  if (s >= nslices) return;
  const int64_t r = s * kSlice + l;
  const int32_t len = r < nrows ? rowlen[r] : 0;
  bool fit = true;
  for (int32_t k = 0; k < width[s]; ++k) {
    const int64_t q = ptr[s] + static_cast<int64_t>(k) * kSlice + l;
    int64_t d = 0;
    if (k < len) {
      d = static_cast<int64_t>(cols[q]) - r;
      if (d < -32767 || d > 32767) {
        fit = false;
        d = 0;
      }
    }
    dcols[q] = static_cast<int16_t>(d);
  }
  const bool all = __all(fit);
  if (l == 0) dfit[s] = all ? 1 : 0;
}

// out[0] = slices with dfit = 1, out[1] = stored entries of their rows (one block, fixed order)
__global__ void k_count_fit(int64_t nslices, int64_t nrows, const uint8_t* dfit, const int32_t* rowlen,
                            int64_t* out) {
  __shared__ int64_t sh[2][256];
  int64_t a = 0, b = 0;
  for (int64_t s = threadIdx.x; s < nslices; s += blockDim.x) {
    if (!dfit[s]) continue;
    a += 1;
    for (int64_t r = s * kSlice; r < (s + 1) * kSlice && r < nrows; ++r) b += rowlen[r];
  }
  sh[0][threadIdx.x] = a;
  sh[1][threadIdx.x] = b;
  __syncthreads();
  for (int off = blockDim.x / 2; off > 0; off >>= 1) {
    if (static_cast<int>(threadIdx.x) < off) {
      sh[0][threadIdx.x] += sh[0][threadIdx.x + off];
      sh[1][threadIdx.x] += sh[1][threadIdx.x + off];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    out[0] = sh[0][0];
    out[1] = sh[1][0];
  }
}

int ell_deltas(Ctx* c, Ell& e) {
  dfree(e.dcols);
  dfree(e.dfit);
  e.dfit_slices = 0;
  if (c->no_delta || e.nrows == 0 || e.nnz_slots == 0) return VIP_OK;
  int64_t* cnt = nullptr;
  VIP_TRY(dalloc(c, &cnt, 2));
  VIP_TRY(dalloc(c, &e.dcols, e.nnz_slots));
  VIP_TRY(dalloc(c, &e.dfit, e.nslices));
  hipStream_t st = c->stream;
  int64_t hc[2] = {0, 0};
  k_deltas<<<(e.nslices * kSlice + kBlock - 1) / kBlock, kBlock, 0, st>>>(e.ptr, e.width, e.rowlen, e.cols, e.nrows,
                                                                            e.nslices, e.dcols, e.dfit);
  k_count_fit<<<1, 256, 0, st>>>(e.nslices, e.nrows, e.dfit, e.rowlen, cnt);
  hipError_t err = hipGetLastError();
  if (err == hipSuccess) err = hipMemcpyAsync(hc, cnt, sizeof(hc), hipMemcpyDeviceToHost, st);
  if (err == hipSuccess) err = hipStreamSynchronize(st);
  dfree(cnt);
  if (err != hipSuccess) {
    dfree(e.dcols);
    dfree(e.dfit);
    return set_error(c, VIP_E_HIP, std::string("row-relative columns: ") + hipGetErrorString(err));
  }
  e.dfit_slices = hc[0];
  e.dfit_nnz = hc[1];
  if (hc[0] == 0) {   // no slice fits: keep the int32 stream only
    dfree(e.dcols);
    dfree(e.dfit);
  }
  return VIP_OK;
}

// ---- MLS shape functions ---------------------------------------------------------------------

__device__ __forceinline__ double weight_fn(double r, int kind) {
#pragma clang fp contract(off)
  if (kind == VIP_W_PAPER) {
    if (!(r < 1.0)) return 0.0;
    const double e = (1.0 - r) * (1.0 - r);
    const double t = 1.0 - pow(r, e);
    return (t * t) * (t * t);
  }
  if (r <= 0.5) return 2.0 / 3.0 - 4.0 * (r * r) + 4.0 * (r * r * r);
  if (r < 1.0) {
    const double s = 1.0 - r;
    return (4.0 / 3.0) * (s * s * s);
  }
  return 0.0;
}

// Packed lower triangle index of (a, b), a >= b.
__host__ __device__ constexpr int tri(int a, int b) { return a * (a + 1) / 2 + b; }

// mode 0: Psi^[0,0] into val0.  mode 1: also the Laplacian (2/rho^2)(c_3 + c_5) into val1.
__global__ void k_mls(const double* x, const double* y, Family f, const double* rho,
                      const int32_t* rowlen, const int64_t* ptr, const int32_t* cols, double Lx,
                      double Ly, int wkind, int mode, double* val0, double* val1,
                      unsigned long long* fail_row) {
#pragma clang fp contract(off)
  int64_t r = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
  if (r >= f.nrows) return;
  const int32_t K = rowlen[r];
  if (K == 0) return;
  const double qx = f.px[r], qy = f.py[r], R = rho[r];
  const int64_t s = r / kSlice, l = r % kSlice;
  const int64_t base = ptr[s] + l;
  double m[21];
#pragma unroll
  for (int a = 0; a < 21; ++a) m[a] = 0.0;
  for (int k = 0; k < K; ++k) {
    const int32_t j = cols[base + static_cast<int64_t>(k) * kSlice];
    const double xi = min_image(x[j] - qx, Lx) / R;
    const double eta = min_image(y[j] - qy, Ly) / R;
    const double w = weight_fn(sqrt(xi * xi + eta * eta), wkind);
    const double p[6] = {1.0, xi, eta, xi * xi, xi * eta, eta * eta};
#pragma unroll
    for (int a = 0; a < 6; ++a)
#pragma unroll
      for (int b = 0; b <= a; ++b) m[tri(a, b)] += w * p[a] * p[b];
  }
  // Cholesky M = L L^T in place
  double dmax = 0.0;
#pragma unroll
  for (int a = 0; a < 6; ++a) dmax = fmax(dmax, m[tri(a, a)]);
  bool ok = dmax > 0.0;
#pragma unroll
  for (int a = 0; a < 6; ++a) {
    double d = m[tri(a, a)];
#pragma unroll
    for (int k = 0; k < a; ++k) d -= m[tri(a, k)] * m[tri(a, k)];
    if (!(d > 1e-13 * dmax)) {
      ok = false;
      d = 1.0;
    }
    const double dd = sqrt(d);
    m[tri(a, a)] = dd;
#pragma unroll
    for (int b = a + 1; b < 6; ++b) {
      double v = m[tri(b, a)];
#pragma unroll
      for (int k = 0; k < a; ++k) v -= m[tri(b, k)] * m[tri(a, k)];
      m[tri(b, a)] = v / dd;
    }
  }
  if (!ok) {
    atomicMin(fail_row, static_cast<unsigned long long>(r));
    return;
  }
  // z0 = M^-1 e0 ; zl = M^-1 (2/R^2)(e3 + e5)
  double z0[6], zl[6];
  {
    double t0[6], tl[6];
    const double c2 = 2.0 / (R * R);
#pragma unroll
    for (int a = 0; a < 6; ++a) {
      double v0 = (a == 0) ? 1.0 : 0.0;
      double vl = (a == 3 || a == 5) ? c2 : 0.0;
#pragma unroll
      for (int k = 0; k < a; ++k) {
        v0 -= m[tri(a, k)] * t0[k];
        vl -= m[tri(a, k)] * tl[k];
      }
      t0[a] = v0 / m[tri(a, a)];
      tl[a] = vl / m[tri(a, a)];
    }
#pragma unroll
    for (int a = 5; a >= 0; --a) {
      double v0 = t0[a], vl = tl[a];
#pragma unroll
      for (int k = a + 1; k < 6; ++k) {
        v0 -= m[tri(k, a)] * z0[k];
        vl -= m[tri(k, a)] * zl[k];
      }
      z0[a] = v0 / m[tri(a, a)];
      zl[a] = vl / m[tri(a, a)];
    }
  }
  for (int k = 0; k < K; ++k) {
    const int64_t slot = base + static_cast<int64_t>(k) * kSlice;
    const int32_t j = cols[slot];
    const double xi = min_image(x[j] - qx, Lx) / R;
    const double eta = min_image(y[j] - qy, Ly) / R;
    const double w = weight_fn(sqrt(xi * xi + eta * eta), wkind);
    const double p[6] = {1.0, xi, eta, xi * xi, xi * eta, eta * eta};
    double a0 = 0.0, al = 0.0;
#pragma unroll
    for (int a = 0; a < 6; ++a) {
      a0 += z0[a] * p[a];
      al += zl[a] * p[a];
    }
    val0[slot] = w * a0;
    if (mode == 1) val1[slot] = w * al;
  }
}

// ---- system rows (pressure and predictor matrices) --------------------------------------------

struct RowView {
  const int64_t* ptr;
  const int32_t* cols;
  const double* val;
  const int32_t* rowlen;
};

__device__ __forceinline__ int64_t slot_of(const int64_t* ptr, int64_t r, int k) {
  return ptr[r / kSlice] + static_cast<int64_t>(k) * kSlice + (r % kSlice);
}

// Row lengths of the system layout: node stencil at interior rows; at boundary
// rows the sorted union of {b}, the stencil of x_b - d n and that of x_b - 2 d n.
__global__ void k_sys_rowlen(int64_t n, const int32_t* bpos, RowView node, RowView n1, RowView n2,
                             int32_t* rowlen) {
  int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
  if (i >= n) return;
  const int32_t k = bpos[i];
  if (k < 0) {
    rowlen[i] = node.rowlen[i];
    return;
  }
  const int la = n1.rowlen[k], lb = n2.rowlen[k];
  int ia = 0, ib = 0, cnt = 0;
  bool self_done = false;
  const int32_t self = static_cast<int32_t>(i);
  while (ia < la || ib < lb || !self_done) {
    int32_t ca = ia < la ? n1.cols[slot_of(n1.ptr, k, ia)] : INT32_MAX;
    int32_t cb = ib < lb ? n2.cols[slot_of(n2.ptr, k, ib)] : INT32_MAX;
    int32_t cs = self_done ? INT32_MAX : self;
    int32_t cmin = min(ca, min(cb, cs));
    if (ca == cmin) ++ia;
    if (cb == cmin) ++ib;
    if (cs == cmin) self_done = true;
    ++cnt;
  }
  rowlen[i] = cnt;
}

// Fill the system layout: columns, Poisson values, and the boundary rows of the
// predictor matrices (their interior rows depend on dt and Re, see k_assemble_helm).
__global__ void k_sys_fill(int64_t n, const int32_t* bpos, const int32_t* bkind, const double* bnx,
                           const double* bny, RowView node, const double* node_lap, RowView n1,
                           RowView n2, const int64_t* sptr, int32_t* scols, double* P, double* Hu,
                           double* Hv) {
  int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
  if (i >= n) return;
  const int32_t k = bpos[i];
  if (k < 0) {
    const int32_t K = node.rowlen[i];
    for (int t = 0; t < K; ++t) {
      const int64_t a = slot_of(node.ptr, i, t), d = slot_of(sptr, i, t);
      scols[d] = node.cols[a];
      P[d] = node_lap[a];
    }
    return;
  }
  const int32_t kind = bkind[k];
  const bool normal_is_y = fabs(bny[k]) >= fabs(bnx[k]);
  const bool u_held = kind == VIP_BC_DIRICHLET || (kind == VIP_BC_SLIP && !normal_is_y);
  const bool v_held = kind == VIP_BC_DIRICHLET || (kind == VIP_BC_SLIP && normal_is_y);
  const bool p_ident = kind == VIP_BC_OUTLET;
  const int la = n1.rowlen[k], lb = n2.rowlen[k];
  int ia = 0, ib = 0, t = 0;
  bool self_done = false;
  const int32_t self = static_cast<int32_t>(i);
  while (ia < la || ib < lb || !self_done) {
    int32_t ca = ia < la ? n1.cols[slot_of(n1.ptr, k, ia)] : INT32_MAX;
    int32_t cb = ib < lb ? n2.cols[slot_of(n2.ptr, k, ib)] : INT32_MAX;
    int32_t cs = self_done ? INT32_MAX : self;
    int32_t cmin = min(ca, min(cb, cs));
    double neu = 0.0;
    if (cs == cmin) {
      neu += 3.0;
      self_done = true;
    }
    if (ca == cmin) neu -= 4.0 * n1.val[slot_of(n1.ptr, k, ia++)];
    if (cb == cmin) neu += n2.val[slot_of(n2.ptr, k, ib++)];
    const double ident = (cmin == self) ? 1.0 : 0.0;
    const int64_t d = slot_of(sptr, i, t++);
    scols[d] = cmin;
    P[d] = p_ident ? ident : neu;
    Hu[d] = u_held ? ident : neu;
    Hv[d] = v_held ? ident : neu;
  }
}

// Interior rows of the predictor matrices: D^[0,0] - c Delta (or I - c Delta).
__global__ void k_assemble_helm(int64_t n, const int32_t* bpos, RowView node, const double* node_m00,
                                const double* node_lap, const int64_t* sptr, double c, int exact_id,
                                double* Hu, double* Hv) {
  int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
  if (i >= n) return;
  if (bpos[i] >= 0) return;
  const int32_t K = node.rowlen[i];
  for (int t = 0; t < K; ++t) {
    const int64_t a = slot_of(node.ptr, i, t), d = slot_of(sptr, i, t);
    const double id = exact_id ? (node.cols[a] == static_cast<int32_t>(i) ? 1.0 : 0.0) : node_m00[a];
    const double h = id - c * node_lap[a];
    Hu[d] = h;
    Hv[d] = h;
  }
}

__global__ void k_diag_inv(int64_t n, const int64_t* sptr, const int32_t* scols, const int32_t* rowlen,
                           const double* A, double* dinv) {
  int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
  if (i >= n) return;
  double d = 0.0;
  for (int t = 0; t < rowlen[i]; ++t) {
    const int64_t s = slot_of(sptr, i, t);
    if (scols[s] == static_cast<int32_t>(i)) d += A[s];
  }
  dinv[i] = d != 0.0 ? 1.0 / d : 1.0;
}

// Row sums of a sliced-ELL matrix (FP64 sum, stored as FP32).
__global__ void k_rowsum32(int64_t n, const int64_t* ptr, const int32_t* rowlen, const double* val,
                           float* out) {
  int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
  if (i >= n) return;
  double s = 0.0;
  for (int t = 0; t < rowlen[i]; ++t)
    s += val[ptr[i / kSlice] + static_cast<int64_t>(t) * kSlice + (i % kSlice)];
  out[i] = static_cast<float>(s);
}

// FP32 copy of a value set with every column scaled by dinv (out = val * dinv[col]), one lane
// per slice row (nslices * kSlice lanes); padding slots and lanes past the last row hold 0 and
// their columns are not read
__global__ void k_colscale_f32(int64_t nrows, int64_t nlanes, const int64_t* ptr, const int32_t* width,
                               const int32_t* rowlen, const int32_t* cols, const double* val,
                               const double* dinv, float* out) {
  const int64_t r = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
  if (r >= nlanes) return;
  const int64_t s = r / kSlice, l = r % kSlice;
  const int32_t len = r < nrows ? rowlen[r] : 0;
  for (int32_t k = 0; k < width[s]; ++k) {
    const int64_t q = ptr[s] + static_cast<int64_t>(k) * kSlice + l;
    out[q] = k < len ? static_cast<float>(val[q] * dinv[cols[q]]) : 0.0f;
  }
}

// row sums of the column-scaled values (FP64 sum, stored as FP32)
__global__ void k_rowsum32_colscaled(int64_t n, const int64_t* ptr, const int32_t* rowlen, const int32_t* cols,
                                     const double* val, const double* dinv, float* out) {
  const int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
  if (i >= n) return;
  double s = 0.0;
  for (int t = 0; t < rowlen[i]; ++t) {
    const int64_t q = ptr[i / kSlice] + static_cast<int64_t>(t) * kSlice + (i % kSlice);
    s += val[q] * dinv[cols[q]];
  }
  out[i] = static_cast<float>(s);
}

void launch_rowsum32(hipStream_t st, int64_t n, const int64_t* ptr, const int32_t* rowlen,
                     const double* val, float* out) {
  if (n > 0) k_rowsum32<<<grid_for(n), kBlock, 0, st>>>(n, ptr, rowlen, val, out);
}

__global__ void k_to_f32(int64_t m, const double* a, float* b) {
  int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
  if (i < m) b[i] = static_cast<float>(a[i]);
}

__global__ void k_bpos(int64_t n, int32_t* bpos) {
  int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
  if (i < n) bpos[i] = -1;
}

__global__ void k_bpos_scatter(int64_t nb, const int64_t* bidx, int32_t* bpos) {
  int64_t k = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
  if (k < nb) bpos[bidx[k]] = static_cast<int32_t>(k);
}

// Largest |a_ij - a_ji| and |a_ij| over the pressure matrix (one thread per row).
__global__ void k_asym(int64_t n, const int64_t* sptr, const int32_t* scols, const int32_t* rowlen,
                       const double* A, unsigned long long* out) {
  int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
  if (i >= n) return;
  double dmax = 0.0, amax = 0.0;
  for (int t = 0; t < rowlen[i]; ++t) {
    const int64_t s = slot_of(sptr, i, t);
    const int32_t j = scols[s];
    const double a = A[s];
    amax = fmax(amax, fabs(a));
    double b = 0.0;
    for (int u = 0; u < rowlen[j]; ++u) {
      const int64_t q = slot_of(sptr, j, u);
      if (scols[q] == static_cast<int32_t>(i)) b += A[q];
    }
    dmax = fmax(dmax, fabs(a - b));
  }
  // non-negative doubles order like their bit patterns
  atomicMax(&out[0], static_cast<unsigned long long>(__double_as_longlong(dmax)));
  atomicMax(&out[1], static_cast<unsigned long long>(__double_as_longlong(amax)));
}

// ---- host orchestration --------------------------------------------------------------------------

namespace {

int build_family(Ctx* c, const Grid& g, const Family& f, Ell& e, int mode, const char* name,
                 unsigned long long* fail) {
  e.nrows = f.nrows;
  VIP_TRY(dalloc(c, &e.rowlen, e.nrows));
  double* rho = nullptr;
  VIP_TRY(dalloc(c, &rho, e.nrows));
  unsigned long long init = ~0ull;
  VIP_HIP_TRY(c, hipMemcpyAsync(fail, &init, sizeof(init), hipMemcpyHostToDevice, c->stream));
  if (e.nrows > 0)
    k_count<<<grid_for(e.nrows), kBlock, 0, c->stream>>>(g, c->x, c->y, f, c->rho0,
                                                          c->opt.min_neighbours, e.rowlen, rho, fail);
  unsigned long long bad = 0;
  VIP_HIP_TRY(c, hipMemcpyAsync(&bad, fail, sizeof(bad), hipMemcpyDeviceToHost, c->stream));
  VIP_HIP_TRY(c, hipStreamSynchronize(c->stream));
  if (bad != ~0ull) {
    dfree(rho);
    return set_error(c, VIP_E_SINGULAR,
                     std::string(name) + " evaluation point " + std::to_string(bad) +
                         ": fewer than min_neighbours (or more than 128) nodes inside the grown support");
  }
  VIP_TRY(ell_layout(c, e));
  if (e.nrows > 0)
    k_fill<<<grid_for(e.nrows), kBlock, 0, c->stream>>>(g, c->x, c->y, f, rho, e.rowlen, e.ptr,
                                                         e.cols);
  const int nv = mode == 1 ? 2 : 1;
  for (int v = 0; v < nv; ++v) {
    VIP_TRY(dalloc(c, &e.val[v], e.nnz_slots));
    VIP_HIP_TRY(c, hipMemsetAsync(e.val[v], 0, sizeof(double) * std::max<int64_t>(e.nnz_slots, 1),
                                  c->stream));
  }
  VIP_HIP_TRY(c, hipMemcpyAsync(fail, &init, sizeof(init), hipMemcpyHostToDevice, c->stream));
  if (e.nrows > 0)
    k_mls<<<grid_for(e.nrows), kBlock, 0, c->stream>>>(c->x, c->y, f, rho, e.rowlen, e.ptr, e.cols,
                                                        c->opt.period[0], c->opt.period[1],
                                                        c->opt.weight, mode, e.val[0], e.val[1], fail);
  VIP_HIP_TRY(c, hipMemcpyAsync(&bad, fail, sizeof(bad), hipMemcpyDeviceToHost, c->stream));
  VIP_HIP_TRY(c, hipStreamSynchronize(c->stream));
  if (mode == 1) {
    c->rho_node = rho;
  } else {
    dfree(rho);
  }
  if (bad != ~0ull)
    return set_error(c, VIP_E_SINGULAR, std::string(name) + " evaluation point " +
                                            std::to_string(bad) + ": moment matrix not positive definite");
  return VIP_OK;
}

}  // namespace

int build_stencils(Ctx* c, const double* xy, int64_t n, const int64_t* bidx, const double* bnrm,
                   const int32_t* bkind, const double* bval, int64_t nb, int basis_order, double rho,
                   double h, const vip_options* opt, const double* h_node) {
  vip_options o;
  vip_default_options(&o);
  if (opt) o = *opt;
  if (n <= 0 || n > INT32_MAX - 1) return set_error(c, VIP_E_INVALID, "n_nodes must be in [1, 2^31-2]");
  if (nb < 0 || nb > n) return set_error(c, VIP_E_INVALID, "n_bnd must be in [0, n_nodes]");
  if (basis_order != 2) return set_error(c, VIP_E_INVALID, "basis_order must be 2 (quadratic basis)");
  if (!(rho > 0.0) || !std::isfinite(rho)) return set_error(c, VIP_E_INVALID, "support_radius must be > 0");
  if (!(h > 0.0) || !std::isfinite(h)) return set_error(c, VIP_E_INVALID, "h must be > 0");
  if (!xy) return set_error(c, VIP_E_INVALID, "nodes_xy is NULL");
  if (nb > 0 && (!bidx || !bnrm || !bkind || !bval))
    return set_error(c, VIP_E_INVALID, "boundary arrays are NULL");
  if (o.weight != VIP_W_CUBIC_SPLINE && o.weight != VIP_W_PAPER)
    return set_error(c, VIP_E_INVALID, "unknown weight");
  if (o.min_neighbours < 6 || o.min_neighbours > kMaxWidth)
    return set_error(c, VIP_E_INVALID, "min_neighbours must be in [6, 128]");
  if (!(o.vip_offset > 0.0) || !(o.vip_offset < 2.0))
    return set_error(c, VIP_E_INVALID, "vip_offset must be in (0, 2)");
  const bool px = o.period[0] > 0.0, py = o.period[1] > 0.0;
  if (px != py) return set_error(c, VIP_E_INVALID, "periodicity must be set on both axes or neither");
  const double rmax = rho * 1.25 * 1.25;
  if (px && (o.period[0] <= 2.0 * rmax || o.period[1] <= 2.0 * rmax))
    return set_error(c, VIP_E_INVALID, "periodic box shorter than twice the largest support");
  if (px && nb > 0) return set_error(c, VIP_E_INVALID, "a periodic box has no boundary nodes");

  // local spacing of adaptive node sets, as a scale over h
  std::vector<double> hscale, hbscale;
  double smax = 1.0;
  if (h_node) {
    hscale.resize(static_cast<size_t>(n));
    for (int64_t i = 0; i < n; ++i) {
      if (!(h_node[i] > 0.0) || !std::isfinite(h_node[i]))
        return set_error(c, VIP_E_INVALID, "h_node must be finite and > 0 (node " + std::to_string(i) + ")");
      hscale[i] = h_node[i] / h;
      smax = std::max(smax, hscale[i]);
    }
  }
  if (px && h_node && (o.period[0] <= 2.0 * rmax * smax || o.period[1] <= 2.0 * rmax * smax))
    return set_error(c, VIP_E_INVALID, "periodic box shorter than twice the largest support");

  // split coordinates, validate, bounding box
  std::vector<double> hx(static_cast<size_t>(n)), hy(static_cast<size_t>(n));
  double xmin = INFINITY, xmax = -INFINITY, ymin = INFINITY, ymax = -INFINITY;
  for (int64_t i = 0; i < n; ++i) {
    const double a = xy[2 * i], b = xy[2 * i + 1];
    if (!std::isfinite(a) || !std::isfinite(b))
      return set_error(c, VIP_E_INVALID, "non-finite coordinate at node " + std::to_string(i));
    hx[i] = a;
    hy[i] = b;
    xmin = std::min(xmin, a);
    xmax = std::max(xmax, a);
    ymin = std::min(ymin, b);
    ymax = std::max(ymax, b);
  }
  std::vector<double> hbnx(static_cast<size_t>(nb)), hbny(static_cast<size_t>(nb));
  std::vector<char> seen(static_cast<size_t>(n), 0);
  for (int64_t k = 0; k < nb; ++k) {
    const int64_t b = bidx[k];
    if (b < 0 || b >= n) return set_error(c, VIP_E_INVALID, "bnd_idx out of range at entry " + std::to_string(k));
    if (seen[b]) return set_error(c, VIP_E_INVALID, "node listed twice in bnd_idx: " + std::to_string(b));
    seen[b] = 1;
    if (bkind[k] < VIP_BC_DIRICHLET || bkind[k] > VIP_BC_OUTLET)
      return set_error(c, VIP_E_INVALID, "unknown bnd_kind at entry " + std::to_string(k));
    hbnx[k] = bnrm[2 * k];
    hbny[k] = bnrm[2 * k + 1];
    const double nn = hbnx[k] * hbnx[k] + hbny[k] * hbny[k];
    if (!(std::fabs(nn - 1.0) < 1e-6))
      return set_error(c, VIP_E_INVALID, "bnd_normal not of unit length at entry " + std::to_string(k));
    if (!std::isfinite(bval[2 * k]) || !std::isfinite(bval[2 * k + 1]))
      return set_error(c, VIP_E_INVALID, "non-finite bnd_value at entry " + std::to_string(k));
  }

  ctx_free_build(c);
  c->opt = o;
  c->n = n;
  c->nb = nb;
  c->h = h;
  c->rho0 = rho;
  c->xmin = xmin;
  c->ymin = ymin;
  c->xmax = xmax;
  c->ymax = ymax;
  c->periodic = px;
  bool has_outlet = false;
  c->h_bkind.assign(bkind, bkind + nb);
  c->h_bpos.assign(n, -1);
  for (int64_t k = 0; k < nb; ++k) c->h_bpos[bidx[k]] = static_cast<int32_t>(k);
  for (int64_t k = 0; k < nb; ++k) has_outlet |= bkind[k] == VIP_BC_OUTLET;
  c->singular = px || !has_outlet;

  hipStream_t st = c->stream;
  VIP_TRY(dalloc(c, &c->x, n));
  VIP_TRY(dalloc(c, &c->y, n));
  if (h_node) {
    // per-node and per-boundary-entry spacing scales, and the Neumann-row scale 2 d_b
    hbscale.resize(static_cast<size_t>(nb));
    std::vector<double> h2d(static_cast<size_t>(nb));
    for (int64_t k = 0; k < nb; ++k) {
      hbscale[k] = hscale[bidx[k]];
      h2d[k] = 2.0 * o.vip_offset * h * hbscale[k];
    }
    VIP_TRY(dalloc(c, &c->hscale, n));
    VIP_TRY(dalloc(c, &c->bscale, nb));
    VIP_TRY(dalloc(c, &c->two_db, nb));
    VIP_HIP_TRY(c, hipMemcpyAsync(c->hscale, hscale.data(), sizeof(double) * n, hipMemcpyHostToDevice, st));
    if (nb > 0) {
      VIP_HIP_TRY(c, hipMemcpyAsync(c->bscale, hbscale.data(), sizeof(double) * nb, hipMemcpyHostToDevice, st));
      VIP_HIP_TRY(c, hipMemcpyAsync(c->two_db, h2d.data(), sizeof(double) * nb, hipMemcpyHostToDevice, st));
    }
    VIP_HIP_TRY(c, hipStreamSynchronize(st));   // the host vectors go out of scope
  }
  VIP_TRY(dalloc(c, &c->bpos, n));
  VIP_TRY(dalloc(c, &c->bidx, nb));
  VIP_TRY(dalloc(c, &c->bnx, nb));
  VIP_TRY(dalloc(c, &c->bny, nb));
  VIP_TRY(dalloc(c, &c->bkind, nb));
  VIP_TRY(dalloc(c, &c->bval, 2 * nb));
  VIP_HIP_TRY(c, hipMemcpyAsync(c->x, hx.data(), sizeof(double) * n, hipMemcpyHostToDevice, st));
  VIP_HIP_TRY(c, hipMemcpyAsync(c->y, hy.data(), sizeof(double) * n, hipMemcpyHostToDevice, st));
  if (nb > 0) {
    VIP_HIP_TRY(c, hipMemcpyAsync(c->bidx, bidx, sizeof(int64_t) * nb, hipMemcpyHostToDevice, st));
    VIP_HIP_TRY(c, hipMemcpyAsync(c->bnx, hbnx.data(), sizeof(double) * nb, hipMemcpyHostToDevice, st));
    VIP_HIP_TRY(c, hipMemcpyAsync(c->bny, hbny.data(), sizeof(double) * nb, hipMemcpyHostToDevice, st));
    VIP_HIP_TRY(c, hipMemcpyAsync(c->bkind, bkind, sizeof(int32_t) * nb, hipMemcpyHostToDevice, st));
    VIP_HIP_TRY(c, hipMemcpyAsync(c->bval, bval, sizeof(double) * 2 * nb, hipMemcpyHostToDevice, st));
  }
  k_bpos<<<grid_for(n), kBlock, 0, st>>>(n, c->bpos);
  if (nb > 0) k_bpos_scatter<<<grid_for(nb), kBlock, 0, st>>>(nb, c->bidx, c->bpos);

  // cell list with cells no smaller than rho
  Grid g{};
  g.Lx = o.period[0];
  g.Ly = o.period[1];
  if (px) {
    g.x0 = 0.0;
    g.y0 = 0.0;
    g.ncx = std::max<int64_t>(1, static_cast<int64_t>(std::floor(o.period[0] / rho)));
    g.ncy = std::max<int64_t>(1, static_cast<int64_t>(std::floor(o.period[1] / rho)));
    g.cw = o.period[0] / g.ncx;
    g.ch = o.period[1] / g.ncy;
  } else {
    g.x0 = xmin;
    g.y0 = ymin;
    g.cw = rho;
    g.ch = rho;
    g.ncx = static_cast<int64_t>(std::floor((xmax - xmin) / rho)) + 1;
    g.ncy = static_cast<int64_t>(std::floor((ymax - ymin) / rho)) + 1;
  }
  const int64_t ncell = g.ncx * g.ncy;
  if (ncell > 4 * n + 1024)
    return set_error(c, VIP_E_INVALID, "support radius too small for the node extent (cell grid too large)");
  int64_t *cell_of = nullptr, *count = nullptr, *start = nullptr, *cursor = nullptr;
  int32_t* items = nullptr;
  VIP_TRY(dalloc(c, &cell_of, n));
  VIP_TRY(dalloc(c, &count, ncell + 1));
  VIP_TRY(dalloc(c, &start, ncell + 1));
  VIP_TRY(dalloc(c, &cursor, ncell + 1));
  VIP_TRY(dalloc(c, &items, n));
  VIP_HIP_TRY(c, hipMemsetAsync(count, 0, sizeof(int64_t) * (ncell + 1), st));
  VIP_HIP_TRY(c, hipMemsetAsync(cursor, 0, sizeof(int64_t) * (ncell + 1), st));
  k_cell_count<<<grid_for(n), kBlock, 0, st>>>(c->x, c->y, n, g, cell_of, count);
  int64_t total = 0;
  VIP_TRY(scan_i64(c, count, start, ncell, &total));
  VIP_HIP_TRY(c, hipMemcpyAsync(start + ncell, &total, sizeof(int64_t), hipMemcpyHostToDevice, st));
  k_cell_fill<<<grid_for(n), kBlock, 0, st>>>(n, cell_of, start, cursor, items);
  g.start = start;
  g.items = items;

  // evaluation points
  const double off = o.vip_offset * h;
  VIP_TRY(dalloc(c, &c->vip_px, 4 * n));
  VIP_TRY(dalloc(c, &c->vip_py, 4 * n));
  VIP_TRY(dalloc(c, &c->d_ew, n));
  VIP_TRY(dalloc(c, &c->d_ns, n));
  k_vip_points<<<grid_for(n), kBlock, 0, st>>>(g, c->x, c->y, n, c->bpos, c->bnx, c->bny, off, rho,
                                                c->hscale, c->vip_px, c->vip_py, c->d_ew, c->d_ns);
  double *np1x = nullptr, *np1y = nullptr, *np2x = nullptr, *np2y = nullptr;
  VIP_TRY(dalloc(c, &np1x, nb));
  VIP_TRY(dalloc(c, &np1y, nb));
  VIP_TRY(dalloc(c, &np2x, nb));
  VIP_TRY(dalloc(c, &np2y, nb));
  if (nb > 0)
    k_normal_points<<<grid_for(nb), kBlock, 0, st>>>(c->x, c->y, c->bidx, c->bnx, c->bny, nb, off,
                                                      c->bscale, np1x, np1y, np2x, np2y);

  unsigned long long* fail = nullptr;
  VIP_TRY(dalloc(c, &fail, 2));
  int rc = VIP_OK;
  {
    Family f{n, c->x, c->y, nullptr, c->hscale};
    rc = build_family(c, g, f, c->node, 1, "node", fail);
  }
  const char* vname[4] = {"east VIP", "west VIP", "north VIP", "south VIP"};
  for (int k = 0; k < 4 && rc == VIP_OK; ++k) {
    Family f{n, c->vip_px + k * n, c->vip_py + k * n, c->bpos, c->hscale};
    rc = build_family(c, g, f, c->vipop[k], 0, vname[k], fail);
  }
  if (rc == VIP_OK) {
    Family f{nb, np1x, np1y, nullptr, c->bscale};
    rc = build_family(c, g, f, c->normal[0], 0, "inner normal point (d)", fail);
  }
  if (rc == VIP_OK) {
    Family f{nb, np2x, np2y, nullptr, c->bscale};
    rc = build_family(c, g, f, c->normal[1], 0, "inner normal point (2d)", fail);
  }
  dfree(cell_of);
  dfree(count);
  dfree(start);
  dfree(cursor);
  dfree(items);
  dfree(np1x);
  dfree(np1y);
  dfree(np2x);
  dfree(np2y);
  if (rc != VIP_OK) {
    dfree(fail);
    return rc;
  }

  // system layout: pressure and predictor matrices
  Ell& s = c->sys;
  s.nrows = n;
  VIP_TRY(dalloc(c, &s.rowlen, n));
  RowView nodev{c->node.ptr, c->node.cols, c->node.val[0], c->node.rowlen};
  RowView n1{c->normal[0].ptr, c->normal[0].cols, c->normal[0].val[0], c->normal[0].rowlen};
  RowView n2{c->normal[1].ptr, c->normal[1].cols, c->normal[1].val[0], c->normal[1].rowlen};
  k_sys_rowlen<<<grid_for(n), kBlock, 0, st>>>(n, c->bpos, nodev, n1, n2, s.rowlen);
  VIP_TRY(ell_layout(c, s));
  for (int v = 0; v < 3; ++v) {
    VIP_TRY(dalloc(c, &s.val[v], s.nnz_slots));
    VIP_HIP_TRY(c, hipMemsetAsync(s.val[v], 0, sizeof(double) * std::max<int64_t>(s.nnz_slots, 1), st));
  }
  VIP_TRY(dalloc(c, &s.val32, s.nnz_slots));
  k_sys_fill<<<grid_for(n), kBlock, 0, st>>>(n, c->bpos, c->bkind, c->bnx, c->bny, nodev,
                                              c->node.val[1], n1, n2, s.ptr, s.cols, s.val[0],
                                              s.val[1], s.val[2]);
  k_to_f32<<<grid_for(s.nnz_slots), kBlock, 0, st>>>(s.nnz_slots, s.val[0], s.val32);
  VIP_TRY(dalloc(c, &s.rsum32, n));
  launch_rowsum32(st, n, s.ptr, s.rowlen, s.val[0], s.rsum32);
  VIP_TRY(ell_deltas(c, s));
  for (int v = 0; v < 3; ++v) VIP_TRY(dalloc(c, &c->dinv[v], n + 1));
  VIP_TRY(dalloc(c, &c->dinv32, n + 1));
  k_diag_inv<<<grid_for(n), kBlock, 0, st>>>(n, s.ptr, s.cols, s.rowlen, s.val[0], c->dinv[0]);
  {
    // the border row (singular systems) keeps a unit preconditioner entry
    const double one = 1.0;
    VIP_HIP_TRY(c, hipMemcpyAsync(c->dinv[0] + n, &one, sizeof(double), hipMemcpyHostToDevice, st));
  }
  k_to_f32<<<grid_for(n + 1), kBlock, 0, st>>>(n + 1, c->dinv[0], c->dinv32);

  // symmetry of the pressure matrix (selects PCG under VIP_K_AUTO)
  unsigned long long zero2[2] = {0ull, 0ull};
  VIP_HIP_TRY(c, hipMemcpyAsync(fail, zero2, sizeof(zero2), hipMemcpyHostToDevice, st));
  k_asym<<<grid_for(n), kBlock, 0, st>>>(n, s.ptr, s.cols, s.rowlen, s.val[0], fail);
  unsigned long long asym[2];
  VIP_HIP_TRY(c, hipMemcpyAsync(asym, fail, sizeof(asym), hipMemcpyDeviceToHost, st));
  VIP_HIP_TRY(c, hipStreamSynchronize(st));
  double dmax, amax;
  std::memcpy(&dmax, &asym[0], sizeof(double));
  std::memcpy(&amax, &asym[1], sizeof(double));
  c->symmetric = dmax <= 1e-12 * amax;
  dfree(fail);

  // step state
  VIP_TRY(dalloc(c, &c->nprev, 2 * n));
  VIP_TRY(dalloc(c, &c->phi, n + 1));
  VIP_HIP_TRY(c, hipMemsetAsync(c->phi, 0, sizeof(double) * (n + 1), st));
  c->assembled = false;
  c->have_prev_n = false;
  c->nstar = 0;
  c->have_prev_phi = false;
  c->cur_dt = 0.0;
  c->cur_re = 0.0;
  VIP_HIP_TRY(c, hipStreamSynchronize(st));
  VIP_HIP_TRY(c, hipGetLastError());
  // lattice-interior rows of the pressure matrix (FP64 and FP32 value sets)
  VIP_TRY(canon_mark(c, s, 0));
  VIP_TRY(canon_mark(c, s, 4));
  VIP_TRY(tile_part(c, 0));
  VIP_TRY(tile_part(c, 1));
  // lattice-interior rows of the per-step VIP and node products
  VIP_TRY(vip_canon_setup(c));
  c->built = true;
  return VIP_OK;
}

int assemble_helmholtz(Ctx* c, double dt, double re) {
  const double cc = dt / (2.0 * re);
  RowView nodev{c->node.ptr, c->node.cols, c->node.val[0], c->node.rowlen};
  k_assemble_helm<<<grid_for(c->n), kBlock, 0, c->stream>>>(
      c->n, c->bpos, nodev, c->node.val[0], c->node.val[1], c->sys.ptr, cc,
      c->opt.identity == VIP_I_EXACT ? 1 : 0, c->sys.val[1], c->sys.val[2]);
  k_diag_inv<<<grid_for(c->n), kBlock, 0, c->stream>>>(c->n, c->sys.ptr, c->sys.cols, c->sys.rowlen,
                                                        c->sys.val[1], c->dinv[1]);
  k_diag_inv<<<grid_for(c->n), kBlock, 0, c->stream>>>(c->n, c->sys.ptr, c->sys.cols, c->sys.rowlen,
                                                        c->sys.val[2], c->dinv[2]);
  // FP32 copies for the mixed-precision predictor solve, with the Jacobi preconditioner folded
  // in: H D^-1 (every column scaled by the inverse diagonal) and its row sums
  Ell& s = c->sys;
  for (int k = 0; k < 2; ++k) {
    if (!s.val32h[k]) VIP_TRY(dalloc(c, &s.val32h[k], s.nnz_slots));
    if (!s.rsum32h[k]) VIP_TRY(dalloc(c, &s.rsum32h[k], c->n));
    k_colscale_f32<<<grid_for(s.nslices * kSlice), kBlock, 0, c->stream>>>(
        c->n, s.nslices * kSlice, s.ptr, s.width, s.rowlen, s.cols, s.val[1 + k], c->dinv[1 + k], s.val32h[k]);
    k_rowsum32_colscaled<<<grid_for(c->n), kBlock, 0, c->stream>>>(c->n, s.ptr, s.rowlen, s.cols, s.val[1 + k],
                                                                    c->dinv[1 + k], s.rsum32h[k]);
  }
  VIP_HIP_TRY(c, hipGetLastError());
  VIP_TRY(canon_mark(c, c->sys, 1));
  VIP_TRY(canon_mark(c, c->sys, 2));
  VIP_TRY(canon_mark(c, c->sys, 5));
  VIP_TRY(canon_mark(c, c->sys, 6));
  VIP_TRY(tile_part(c, 2));
  VIP_TRY(tile_part(c, 3));
  c->cur_dt = dt;
  c->cur_re = re;
  c->assembled = true;
  return VIP_OK;
}

}  // namespace vip
