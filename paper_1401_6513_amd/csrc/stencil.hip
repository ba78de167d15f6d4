// Lattice map of the node set and the canonical rows of the system operators.
//
// A canonical row also needs the nodes of each lattice row of its stencil numbered
// consecutively (true for row-by-row lattice orderings), so that a tap's node is the node
// straight above or below plus its offset along the row.
//
// On a lattice-based node set every interior node far from the boundary sees the same
// neighbourhood, so its MLS weights (Section 3) and every operator built from them (eq.
// vip:1, eq. 12, eq. 13) repeat from row to row.  When the lattice coordinates are exact in
// binary (h a power of two) the repeats are exact to the bit.  A row whose stored entries sit
// at the reference row's lattice offsets and equal its values bit for bit is "canonical":
// products over it need neither the column nor the value streams of the sliced ELL.  Rows
// near the boundary, off-lattice nodes and rows of node sets whose coordinates do not repeat
// exactly stay on the general path.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cmath>
#include <cstring>
#include <map>
#include <vector>

#include "vip_internal.h"

namespace vip {

namespace {

__global__ void k_fill_i32(int64_t n, int32_t v, int32_t* a) {
  const int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
  if (i < n) a[i] = v;
}

// the lowest node index on a lattice position claims its pixel
__global__ void k_pixel_claim(int64_t n, const double* x, const double* y, double x0, double y0, double h,
                              int W, int H, int32_t* node_of) {
  const int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
  if (i >= n) return;
  const double fx = (x[i] - x0) / h, fy = (y[i] - y0) / h;
  const double rx = rint(fx), ry = rint(fy);
  if (fabs(fx - rx) < 1e-6 && fabs(fy - ry) < 1e-6 && rx >= 0 && ry >= 0 && rx < W && ry < H)
    atomicMin(&node_of[static_cast<int64_t>(ry) * W + static_cast<int64_t>(rx)], static_cast<int32_t>(i));
}

__global__ void k_pixel_finish(int64_t npix, int32_t* node_of, int32_t* pix) {
  const int64_t q = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
  if (q >= npix) return;
  const int32_t node = node_of[q];
  if (node == INT32_MAX) {
    node_of[q] = -1;
  } else {
    pix[node] = static_cast<int32_t>(q);
  }
}

// Row data of sampled rows for choosing the reference row: length, boundary flag, pixel,
// pixels of the stored columns and the bits of their values.
__global__ void k_gather_rows(int m, const int64_t* rows, const int64_t* ptr, const int32_t* rowlen,
                              const int32_t* cols, const int32_t* bpos, const int32_t* pix, const double* v64,
                              const float* v32, const float* rsum32, int32_t* o_len, int32_t* o_bpos,
                              int32_t* o_pix, int32_t* o_cpix, uint64_t* o_bits, uint32_t* o_rsum) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= m) return;
  const int64_t i = rows[s];
  const int len = rowlen[i];
  o_len[s] = len;
  o_bpos[s] = bpos ? bpos[i] : -1;
  o_pix[s] = pix[i];
  o_rsum[s] = rsum32 ? __float_as_uint(rsum32[i]) : 0u;
  const int64_t base = ptr[i / kSlice] + (i % kSlice);
  for (int k = 0; k < len && k < kMaxTaps; ++k) {
    const int64_t q = base + static_cast<int64_t>(k) * kSlice;
    o_cpix[s * kMaxTaps + k] = pix[cols[q]];
    o_bits[s * kMaxTaps + k] = v64 ? static_cast<uint64_t>(__double_as_longlong(v64[q]))
                                   : static_cast<uint64_t>(__float_as_uint(v32[q]));
  }
}

struct MarkArgs {
  int K, W, H;
  int32_t dx[kMaxTaps], dy[kMaxTaps];
  uint64_t bits[kMaxTaps];
  uint32_t rsum_bits;
};

// cpix[i] = pixel of row i if it is canonical for the given value set, else -1
__global__ void k_canon_mark(int64_t n, MarkArgs a, const int32_t* bpos, const int32_t* pix,
                             const int32_t* node_of, const int64_t* ptr, const int32_t* rowlen,
                             const int32_t* cols, const double* v64, const float* v32, const float* rsum32,
                             int32_t* cpix) {
  const int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
  if (i >= n) return;
  int32_t out = -1;
  const int32_t p = pix[i];
  if ((!bpos || bpos[i] < 0) && p >= 0 && rowlen[i] == a.K) {
    const int ix = p % a.W, iy = p / a.W;
    const int64_t base = ptr[i / kSlice] + (i % kSlice);
    bool ok = true;
    for (int k = 0; k < a.K; ++k) {
      const int jx = ix + a.dx[k], jy = iy + a.dy[k];
      if (jx < 0 || jx >= a.W || jy < 0 || jy >= a.H) {
        ok = false;
        break;
      }
      const int64_t q = base + static_cast<int64_t>(k) * kSlice;
      // the tap's node, and the nodes of its lattice row numbered consecutively from the node
      // straight above or below the row's node
      const int32_t rowbase = node_of[static_cast<int64_t>(jy) * a.W + ix];
      if (node_of[static_cast<int64_t>(jy) * a.W + jx] != cols[q] || rowbase < 0 || cols[q] != rowbase + a.dx[k])
        ok = false;
      const uint64_t bits = v64 ? static_cast<uint64_t>(__double_as_longlong(v64[q]))
                                : static_cast<uint64_t>(__float_as_uint(v32[q]));
      if (bits != a.bits[k]) ok = false;
    }
    if (ok && !v64 && __float_as_uint(rsum32[i]) != a.rsum_bits) ok = false;
    if (ok) out = p;
  }
  cpix[i] = out;
}

// per-block counts of entries >= 0
__global__ void k_count_nonneg(int64_t n, const int32_t* a, int64_t* part) {
  __shared__ int64_t s[256];
  int64_t c = 0;
  for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x)
    c += a[i] >= 0 ? 1 : 0;
  s[threadIdx.x] = c;
  __syncthreads();
  for (int off = blockDim.x / 2; off > 0; off >>= 1) {
    if (static_cast<int>(threadIdx.x) < off) s[threadIdx.x] += s[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = s[0];
}

// slice s: rows 64 s .. 64 s + 63 all canonical on consecutive pixels of one lattice row
__global__ void k_slice_bases(int64_t nslices, int64_t n, const int32_t* cpix, const int32_t* node_of, int W,
                              int32_t* out) {
  const int64_t s = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
  if (s >= nslices) return;
  const int64_t i0 = s * kSlice;
  bool ok = i0 + kSlice <= n;
  const int32_t p0 = ok ? cpix[i0] : -1;
  ok = ok && p0 >= 0 && (p0 % W) + kSlice <= W;
  for (int l = 1; l < kSlice && ok; ++l)
    if (cpix[i0 + l] != p0 + l) ok = false;
  int4 d = make_int4(-1, -1, -1, -1);
  if (ok) d = make_int4(node_of[p0 - 2 * W], node_of[p0 - W], node_of[p0 + W], node_of[p0 + 2 * W]);
  if (d.x < 0 || d.y < 0 || d.z < 0 || d.w < 0) d = make_int4(-1, -1, -1, -1);
  reinterpret_cast<int4*>(out)[s] = d;
}

// per-block counts of a[stride * i] >= 0, i < n
__global__ void k_count_nonneg_stride(int64_t n, const int32_t* a, int stride, int64_t* part) {
  __shared__ int64_t s[256];
  int64_t c = 0;
  for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x)
    c += a[stride * i] >= 0 ? 1 : 0;
  s[threadIdx.x] = c;
  __syncthreads();
  for (int off = blockDim.x / 2; off > 0; off >>= 1) {
    if (static_cast<int>(threadIdx.x) < off) s[threadIdx.x] += s[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = s[0];
}

// out[i] = a0[i] if rows i of all six operators are canonical (they then share the pixel)
__global__ void k_vc_combine(int64_t n, const int32_t* a0, const int32_t* a1, const int32_t* a2,
                             const int32_t* a3, const int32_t* a4, const int32_t* a5, int32_t* out) {
  const int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
  if (i >= n) return;
  const int32_t p = a0[i];
  const bool ok = p >= 0 && a1[i] == p && a2[i] == p && a3[i] == p && a4[i] == p && a5[i] == p;
  out[i] = ok ? p : -1;
}

// Runs of one reference row: stencil rows in increasing dy, consecutive dx within a row.
bool vc_runs(const Canon& cn, int8_t (&dx0)[kVcRows], int8_t (&len)[kVcRows]) {
  for (int d = 0; d < kVcRows; ++d) dx0[d] = len[d] = 0;
  int last = -1;
  for (int k = 0; k < cn.K; ++k) {
    const int d = cn.dy[k] + 3;
    if (d < 0 || d >= kVcRows || d < last || cn.dx[k] < -64 || cn.dx[k] > 63) return false;
    if (d != last) {
      if (len[d] != 0) return false;
      dx0[d] = static_cast<int8_t>(cn.dx[k]);
    } else if (cn.dx[k] != dx0[d] + len[d]) {
      return false;
    }
    len[d] = static_cast<int8_t>(len[d] + 1);
    last = d;
  }
  return cn.K > 0;
}

// rowstart[(yy, tx)]: the node at pixel (64 tx - 2, yy - 2) when the 68 pixels of the tile's LDS
// row hold consecutive nodes, else -1
__global__ void k_tile_rowstart(int64_t m, int ntx, int W, int H, const int32_t* node_of, int32_t* out) {
  const int64_t q = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
  if (q >= m) return;
  const int yy = static_cast<int>(q / ntx), tx = static_cast<int>(q % ntx);
  const int gy = yy - 2, gx0 = tx * kTileX - 2;
  int32_t r = -1;
  if (gy >= 0 && gy < H && gx0 >= 0 && gx0 + kTileX + 4 <= W) {
    const int32_t* row = node_of + static_cast<int64_t>(gy) * W + gx0;
    const int32_t s0 = row[0];
    bool ok = s0 >= 0;
    for (int k = 1; k < kTileX + 4 && ok; ++k) ok = row[k] == s0 + k;
    if (ok) r = s0;
  }
  out[q] = r;
}

// bits[(y, tx)]: pixels of the word whose node is canonical in c0 (and c1)
__global__ void k_tile_bits(int64_t m, int ntx, int W, int H, const int32_t* node_of, const int32_t* c0,
                            const int32_t* c1, uint64_t* bits) {
  const int64_t q = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
  if (q >= m) return;
  const int gy = static_cast<int>(q / ntx), tx = static_cast<int>(q % ntx);
  uint64_t w = 0;
  if (gy < H) {
    for (int lx = 0; lx < kTileX; ++lx) {
      const int gx = tx * kTileX + lx;
      if (gx >= W) break;
      const int32_t node = node_of[static_cast<int64_t>(gy) * W + gx];
      if (node >= 0 && c0[node] >= 0 && (!c1 || c1[node] >= 0)) w |= 1ull << lx;
    }
  }
  bits[q] = w;
}

// Records of the listed tiles (word d of record k): 0 tx, 1 ty, 2..21 the row starts of halo
// rows 0..19, 22..31 zero, 32..63 the 16 row masks as (low, high) word pairs.
__global__ void k_tile_rec(int64_t ntiles, const int32_t* tiles, int ntx, const int32_t* rowstart,
                           const uint64_t* bits, uint32_t* rec) {
  const int64_t q = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
  if (q >= ntiles * kTileRecWords) return;
  const int64_t k = q / kTileRecWords;
  const int d = static_cast<int>(q % kTileRecWords);
  const int t = tiles[k], tx = t % ntx, ty = t / ntx;
  uint32_t v = 0;
  if (d == 0) {
    v = static_cast<uint32_t>(tx);
  } else if (d == 1) {
    v = static_cast<uint32_t>(ty);
  } else if (d < 2 + kTileY + 4) {
    v = static_cast<uint32_t>(rowstart[static_cast<int64_t>(ty * kTileY + d - 2) * ntx + tx]);
  } else if (d >= 32) {
    const uint64_t w = bits[static_cast<int64_t>(ty * kTileY + (d - 32) / 2) * ntx + tx];
    v = (d & 1) ? static_cast<uint32_t>(w >> 32) : static_cast<uint32_t>(w);
  }
  rec[q] = v;
}

// flag[t] = 1 if tile t holds a tile row
__global__ void k_tile_flag(int64_t ntiles, int ntx, const uint64_t* bits, int64_t* flag) {
  const int64_t t = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
  if (t >= ntiles) return;
  const int tx = static_cast<int>(t % ntx), ty = static_cast<int>(t / ntx);
  uint64_t any = 0;
  for (int ly = 0; ly < kTileY; ++ly) any |= bits[static_cast<int64_t>(ty * kTileY + ly) * ntx + tx];
  flag[t] = any ? 1 : 0;
}

// flag[i] = 1 if row i is not a tile row
__global__ void k_irr_flag(int64_t n, const int32_t* c0, const int32_t* c1, int64_t* flag) {
  const int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
  if (i >= n) return;
  flag[i] = (c0[i] >= 0 && (!c1 || c1[i] >= 0)) ? 0 : 1;
}

// out[pos[i]] = i where flag[i] (pos: exclusive scan of flag)
__global__ void k_compact(int64_t n, const int64_t* flag, const int64_t* pos, int32_t* out) {
  const int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
  if (i < n && flag[i]) out[pos[i]] = static_cast<int32_t>(i);
}

struct RowSample {
  int len = 0, bpos = 0, pix = -1;
  std::vector<int32_t> cpix;
  std::vector<uint64_t> bits;
  uint32_t rsum = 0;
};

// Sampled rows' data (value set vs) copied to the host.
int gather(Ctx* c, const Ell& e, int vs, const LatRef& L, const std::vector<int64_t>& rows,
           std::vector<RowSample>* out) {
  const int m = static_cast<int>(rows.size());
  int64_t* d_rows = nullptr;
  int32_t *d_len = nullptr, *d_bpos = nullptr, *d_pix = nullptr, *d_cpix = nullptr;
  uint64_t* d_bits = nullptr;
  uint32_t* d_rsum = nullptr;
  int rc = VIP_OK;
  std::vector<int32_t> len(m), bp(m), px(m), cp(static_cast<size_t>(m) * kMaxTaps, -1);
  std::vector<uint64_t> bits(static_cast<size_t>(m) * kMaxTaps, 0);
  std::vector<uint32_t> rs(m);
  do {
    if ((rc = dalloc(c, &d_rows, m)) || (rc = dalloc(c, &d_len, m)) || (rc = dalloc(c, &d_bpos, m)) ||
        (rc = dalloc(c, &d_pix, m)) || (rc = dalloc(c, &d_cpix, static_cast<int64_t>(m) * kMaxTaps)) ||
        (rc = dalloc(c, &d_bits, static_cast<int64_t>(m) * kMaxTaps)) || (rc = dalloc(c, &d_rsum, m)))
      break;
    hipStream_t st = c->stream;
    if (hipMemcpyAsync(d_rows, rows.data(), sizeof(int64_t) * m, hipMemcpyHostToDevice, st) != hipSuccess) {
      rc = set_error(c, VIP_E_HIP, "copy of sampled rows");
      break;
    }
    const float* v32 = vs == 4 ? e.val32 : vs > 4 ? e.val32h[vs - 5] : nullptr;
    const float* r32 = vs == 4 ? e.rsum32 : vs > 4 ? e.rsum32h[vs - 5] : nullptr;
    k_gather_rows<<<(m + 63) / 64, 64, 0, st>>>(m, d_rows, e.ptr, e.rowlen, e.cols, L.bpos, L.pix,
                                                vs < 4 ? e.val[vs] : nullptr, v32, r32, d_len, d_bpos, d_pix,
                                                d_cpix, d_bits, d_rsum);
    if (hipGetLastError() != hipSuccess ||
        hipMemcpyAsync(len.data(), d_len, sizeof(int32_t) * m, hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipMemcpyAsync(bp.data(), d_bpos, sizeof(int32_t) * m, hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipMemcpyAsync(px.data(), d_pix, sizeof(int32_t) * m, hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipMemcpyAsync(cp.data(), d_cpix, sizeof(int32_t) * m * kMaxTaps, hipMemcpyDeviceToHost, st) !=
            hipSuccess ||
        hipMemcpyAsync(bits.data(), d_bits, sizeof(uint64_t) * m * kMaxTaps, hipMemcpyDeviceToHost, st) !=
            hipSuccess ||
        hipMemcpyAsync(rs.data(), d_rsum, sizeof(uint32_t) * m, hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess) {
      rc = set_error(c, VIP_E_HIP, "gathering sampled rows");
      break;
    }
  } while (false);
  dfree(d_rows);
  dfree(d_len);
  dfree(d_bpos);
  dfree(d_pix);
  dfree(d_cpix);
  dfree(d_bits);
  dfree(d_rsum);
  if (rc != VIP_OK) return rc;
  out->assign(m, RowSample());
  for (int s = 0; s < m; ++s) {
    RowSample& r = (*out)[s];
    r.len = len[s];
    r.bpos = bp[s];
    r.pix = px[s];
    r.rsum = rs[s];
    const int k = std::min(r.len, kMaxTaps);
    r.cpix.assign(cp.begin() + static_cast<size_t>(s) * kMaxTaps, cp.begin() + static_cast<size_t>(s) * kMaxTaps + k);
    r.bits.assign(bits.begin() + static_cast<size_t>(s) * kMaxTaps,
                  bits.begin() + static_cast<size_t>(s) * kMaxTaps + k);
  }
  return VIP_OK;
}

}  // namespace

void lattice_free(Lattice& lat) {
  dfree(lat.pix);
  dfree(lat.node_of);
  lat.tried = lat.ok = false;
  lat.W = lat.H = 0;
}

void canon_free(Canon& cn) {
  for (auto& tp : cn.tpart) tile_part_free(tp);
  for (auto& p : cn.cpix) dfree(p);
  for (auto& p : cn.sbase) dfree(p);
  cn.K = 0;
  cn.ref_row = -1;
  for (auto& k : cn.count) k = 0;
  for (auto& r : cn.vref) r = -1;
}

int lattice_map(Ctx* c, bool* ok) {
  Lattice& L = c->lat;
  if (!L.tried) {
    L.tried = true;
    L.ok = false;
    const double h = c->h;
    const double wx = std::floor((c->xmax - c->xmin) / h + 0.5) + 1.0;
    const double wy = std::floor((c->ymax - c->ymin) / h + 0.5) + 1.0;
    if (wx * wy <= 4.0 * static_cast<double>(c->n) + 4096.0 && wx <= 65536.0 && wy <= 65536.0 && wx >= 1 &&
        wy >= 1) {
      L.W = static_cast<int>(wx);
      L.H = static_cast<int>(wy);
      const int64_t npix = static_cast<int64_t>(L.W) * L.H;
      VIP_TRY(dalloc(c, &L.pix, c->n));
      VIP_TRY(dalloc(c, &L.node_of, npix));
      hipStream_t st = c->stream;
      k_fill_i32<<<grid_for(c->n), kBlock, 0, st>>>(c->n, -1, L.pix);
      k_fill_i32<<<grid_for(npix), kBlock, 0, st>>>(npix, INT32_MAX, L.node_of);
      k_pixel_claim<<<grid_for(c->n), kBlock, 0, st>>>(c->n, c->x, c->y, c->xmin, c->ymin, h, L.W, L.H,
                                                       L.node_of);
      k_pixel_finish<<<grid_for(npix), kBlock, 0, st>>>(npix, L.node_of, L.pix);
      VIP_HIP_TRY(c, hipGetLastError());
      VIP_HIP_TRY(c, hipStreamSynchronize(st));
      L.ok = true;
    }
  }
  if (ok) *ok = L.ok;
  return VIP_OK;
}

int slice_bases(Ctx* c, const int32_t* cpix, int64_t n, int32_t** out, int64_t* described) {
  const int64_t ns = (n + kSlice - 1) / kSlice;
  if (!*out) VIP_TRY(dalloc(c, out, 4 * ns));
  k_slice_bases<<<grid_for(ns), kBlock, 0, c->stream>>>(ns, n, cpix, c->lat.node_of, c->lat.W, *out);
  VIP_HIP_TRY(c, hipGetLastError());
  if (described) {
    // described slices: first entries >= 0, counted in fixed block order
    int64_t* part = nullptr;
    VIP_TRY(dalloc(c, &part, 256));
    k_count_nonneg_stride<<<256, 256, 0, c->stream>>>(ns, *out, 4, part);
    std::vector<int64_t> hp(256);
    hipError_t e1 = hipMemcpyAsync(hp.data(), part, sizeof(int64_t) * 256, hipMemcpyDeviceToHost, c->stream);
    hipError_t e2 = hipStreamSynchronize(c->stream);
    dfree(part);
    if (e1 != hipSuccess || e2 != hipSuccess) return set_error(c, VIP_E_HIP, "counting described slices");
    int64_t cnt = 0;
    for (int64_t v : hp) cnt += v;
    *described = cnt * kSlice;
  }
  return VIP_OK;
}

int canon_mark(Ctx* c, Ell& e, int vs) {
  bool ok = false;
  VIP_TRY(lattice_map(c, &ok));
  if (!ok || e.nrows != c->n) return VIP_OK;
  const Lattice& L = c->lat;
  return canon_mark_on(c, e, vs, LatRef{L.W, L.H, L.pix, L.node_of, c->n, c->bpos});
}

int canon_mark_on(Ctx* c, Ell& e, int vs, const LatRef& L) {
  Canon& cn = e.canon;
  const float* v32 = vs == 4 ? e.val32 : vs > 4 && vs <= 6 ? e.val32h[vs - 5] : nullptr;
  const float* r32 = vs == 4 ? e.rsum32 : vs > 4 && vs <= 6 ? e.rsum32h[vs - 5] : nullptr;
  if (vs < 0 || vs > 6 || (vs < 4 && !e.val[vs]) || (vs >= 4 && (!v32 || !r32))) return VIP_OK;
  if (e.nrows != L.n || L.n == 0) return VIP_OK;
  if (cn.ref_row == -2) return VIP_OK;   // no repeated interior pattern
  // reference of this value set: the most common (offsets, values) pattern among evenly spaced
  // interior rows. Once a first set has fixed the offsets, later sets keep them and choose among
  // rows with those offsets: a row typical of one set need not be typical of another (columns
  // scaled by their own rows' diagonals differ next to the boundary).
  int64_t ref_row = -1;
  {
    const int m = static_cast<int>(std::min<int64_t>(1024, L.n));
    std::vector<int64_t> rows(m);
    for (int s = 0; s < m; ++s) rows[s] = static_cast<int64_t>((s + 0.5) * static_cast<double>(L.n) / m);
    std::vector<RowSample> smp;
    VIP_TRY(gather(c, e, vs, L, rows, &smp));
    std::map<std::vector<uint64_t>, std::pair<int, int64_t>> freq;
    for (int s = 0; s < m; ++s) {
      const RowSample& r = smp[s];
      if (r.bpos >= 0 || r.pix < 0 || r.len < 1 || r.len > kMaxTaps) continue;
      if (cn.K != 0 && r.len != cn.K) continue;
      std::vector<uint64_t> key;
      bool good = true;
      for (int k = 0; k < r.len; ++k) {
        if (r.cpix[k] < 0) {
          good = false;
          break;
        }
        const int64_t dx = static_cast<int64_t>(r.cpix[k] % L.W) - r.pix % L.W;
        const int64_t dy = static_cast<int64_t>(r.cpix[k] / L.W) - r.pix / L.W;
        if (cn.K != 0 && (dx != cn.dx[k] || dy != cn.dy[k])) {
          good = false;
          break;
        }
        key.push_back(static_cast<uint64_t>((dy + 1024) * 4096 + (dx + 1024)));
        key.push_back(r.bits[k]);
      }
      if (!good) continue;
      auto& f = freq[key];
      if (f.first == 0) f.second = rows[s];
      f.first += 1;
    }
    int best = 0;
    for (const auto& kv : freq)
      if (kv.second.first > best) {
        best = kv.second.first;
        ref_row = kv.second.second;
      }
    if (best < 2) {
      if (cn.ref_row == -1) cn.ref_row = -2;
      return VIP_OK;
    }
    if (cn.ref_row == -1) cn.ref_row = ref_row;
  }
  // the reference row's offsets and the bits of value set vs
  std::vector<RowSample> ref;
  VIP_TRY(gather(c, e, vs, L, std::vector<int64_t>{ref_row}, &ref));
  const RowSample& r = ref[0];
  if (r.len < 1 || r.len > kMaxTaps || r.pix < 0) return VIP_OK;
  MarkArgs a{};
  a.K = r.len;
  a.W = L.W;
  a.H = L.H;
  for (int k = 0; k < r.len; ++k) {
    if (r.cpix[k] < 0) return VIP_OK;
    a.dx[k] = r.cpix[k] % L.W - r.pix % L.W;
    a.dy[k] = r.cpix[k] / L.W - r.pix / L.W;
    a.bits[k] = r.bits[k];
  }
  a.rsum_bits = r.rsum;
  if (cn.K != 0 && cn.K != a.K) return set_error(c, VIP_E_INVALID, "canonical rows changed shape");
  cn.K = a.K;
  for (int k = 0; k < a.K; ++k) {
    cn.dx[k] = a.dx[k];
    cn.dy[k] = a.dy[k];
    cn.off[k] = a.dy[k] * L.W + a.dx[k];
    if (vs < 4) {
      double d;
      std::memcpy(&d, &a.bits[k], sizeof(d));
      cn.w[vs][k] = d;
    } else {
      const uint32_t b = static_cast<uint32_t>(a.bits[k]);
      float f;
      std::memcpy(&f, &b, sizeof(f));
      cn.w32[vs - 4][k] = f;
    }
  }
  if (vs >= 4) std::memcpy(&cn.rsum32[vs - 4], &a.rsum_bits, sizeof(float));
  cn.disk = a.K == kDiskTaps ? 1 : 0;
  for (int k = 0; k < a.K && cn.disk; ++k)
    if (a.dy[k] != disk_row(k) - 2 || a.dx[k] != disk_dx(k)) cn.disk = 0;
  cn.box = a.K == 9 ? 1 : 0;
  for (int k = 0; k < a.K && cn.box; ++k)
    if (a.dy[k] != k / 3 - 1 || a.dx[k] != k % 3 - 1) cn.box = 0;
  cn.vref[vs] = ref_row;
  if (!cn.cpix[vs]) VIP_TRY(dalloc(c, &cn.cpix[vs], L.n));
  hipStream_t st = c->stream;
  k_canon_mark<<<grid_for(L.n), kBlock, 0, st>>>(L.n, a, L.bpos, L.pix, L.node_of, e.ptr, e.rowlen, e.cols,
                                                  vs < 4 ? e.val[vs] : nullptr, v32, r32, cn.cpix[vs]);
  // number of canonical rows (kernels skip the canonical path when it is zero)
  int64_t* part = nullptr;
  VIP_TRY(dalloc(c, &part, 256));
  k_count_nonneg<<<256, 256, 0, st>>>(L.n, cn.cpix[vs], part);
  std::vector<int64_t> hp(256);
  hipError_t e1 = hipMemcpyAsync(hp.data(), part, sizeof(int64_t) * 256, hipMemcpyDeviceToHost, st);
  hipError_t e2 = hipStreamSynchronize(st);
  dfree(part);
  if (e1 != hipSuccess || e2 != hipSuccess) return set_error(c, VIP_E_HIP, "counting canonical rows");
  int64_t cnt = 0;
  for (int64_t v : hp) cnt += v;
  cn.count[vs] = cnt;
  cn.described[vs] = 0;
  if (cn.disk && cnt > 0 && L.node_of == c->lat.node_of)
    VIP_TRY(slice_bases(c, cn.cpix[vs], L.n, &cn.sbase[vs], &cn.described[vs]));
  if (c->debug)
    std::fprintf(stderr, "[vip] canonical rows, value set %d: %lld of %lld (%d taps, reference row %lld)\n", vs,
                 static_cast<long long>(cnt), static_cast<long long>(L.n), cn.K,
                 static_cast<long long>(ref_row));
  return VIP_OK;
}

void tile_part_free(TilePart& tp) {
  dfree(tp.bits);
  dfree(tp.tiles);
  dfree(tp.irr);
  dfree(tp.rec);
  tp = TilePart();
}

void tile_map_free(TileMap& tm) {
  dfree(tm.rowstart);
  tm = TileMap();
}

namespace {

// indices i < m with flag[i] != 0, ascending, into a new device array
int compact(Ctx* c, const int64_t* flag, int64_t m, int32_t** out, int64_t* count) {
  int64_t* pos = nullptr;
  VIP_TRY(dalloc(c, &pos, m));
  int64_t total = 0;
  int rc = scan_i64(c, flag, pos, m, &total);
  if (rc == VIP_OK) rc = dalloc(c, out, total);
  if (rc == VIP_OK && total > 0) {
    k_compact<<<grid_for(m), kBlock, 0, c->stream>>>(m, flag, pos, *out);
    if (hipGetLastError() != hipSuccess || hipStreamSynchronize(c->stream) != hipSuccess)
      rc = set_error(c, VIP_E_HIP, "compacting a tile list");
  }
  dfree(pos);
  *count = total;
  return rc;
}

}  // namespace

int tile_part_build(Ctx* c, int W, int H, const int32_t* node_of, int64_t n, TileMap& tm, const int32_t* c0,
                    const int32_t* c1, TilePart& tp) {
  tile_part_free(tp);
  if (!c0 || !node_of || n == 0 || W <= 0 || H <= 0) return VIP_OK;
  hipStream_t st = c->stream;
  if (!tm.rowstart) {
    tm.ntx = (W + kTileX - 1) / kTileX;
    tm.nty = (H + kTileY - 1) / kTileY;
    const int64_t m = static_cast<int64_t>(tm.nty * kTileY + 4) * tm.ntx;
    VIP_TRY(dalloc(c, &tm.rowstart, m));
    k_tile_rowstart<<<grid_for(m), kBlock, 0, st>>>(m, tm.ntx, W, H, node_of, tm.rowstart);
    VIP_HIP_TRY(c, hipGetLastError());
  }
  const int64_t nw = static_cast<int64_t>(tm.nty * kTileY) * tm.ntx;
  VIP_TRY(dalloc(c, &tp.bits, nw));
  k_tile_bits<<<grid_for(nw), kBlock, 0, st>>>(nw, tm.ntx, W, H, node_of, c0, c1, tp.bits);
  VIP_HIP_TRY(c, hipGetLastError());
  const int64_t nt = static_cast<int64_t>(tm.nty) * tm.ntx;
  int64_t* flag = nullptr;
  VIP_TRY(dalloc(c, &flag, std::max(nt, n)));
  int rc = VIP_OK;
  do {
    k_tile_flag<<<grid_for(nt), kBlock, 0, st>>>(nt, tm.ntx, tp.bits, flag);
    if ((rc = compact(c, flag, nt, &tp.tiles, &tp.ntiles)) != VIP_OK) break;
    if ((rc = dalloc(c, &tp.rec, tp.ntiles * kTileRecWords)) != VIP_OK) break;
    if (tp.ntiles > 0)
      k_tile_rec<<<grid_for(tp.ntiles * kTileRecWords), kBlock, 0, st>>>(tp.ntiles, tp.tiles, tm.ntx, tm.rowstart,
                                                                          tp.bits, tp.rec);
    k_irr_flag<<<grid_for(n), kBlock, 0, st>>>(n, c0, c1, flag);
    if ((rc = compact(c, flag, n, &tp.irr, &tp.nirr)) != VIP_OK) break;
  } while (false);
  dfree(flag);
  if (rc != VIP_OK) {
    tile_part_free(tp);
    return rc;
  }
  // launch split (both multiples of the XCD count): one tile per block up to 6144 tile blocks
  // (24 per CU), one irregular row per thread up to 1024 blocks.  Measured on the 9821 tiles at
  // h = D/128 with the tile kernels at 8 waves per SIMD: the pressure SpMV took 43.5 us at 5120
  // or 6144 blocks against 46.0 at 4096, 44.5 at 7168, 46.0 at 8192 and 46.8 at one tile per
  // block (at 5 waves per SIMD, 4096 had been best)
  tp.tile_blocks = static_cast<int>(std::min<int64_t>((tp.ntiles + kNumXcd - 1) / kNumXcd * kNumXcd, 6144));
  tp.irr_blocks = static_cast<int>(
      std::min<int64_t>(((tp.nirr + kBlock - 1) / kBlock + kNumXcd - 1) / kNumXcd * kNumXcd, 1024));
  return VIP_OK;
}

int tile_part(Ctx* c, int key) {
  Canon& cn = c->sys.canon;
  if (key < 0 || key > 3) return set_error(c, VIP_E_INVALID, "tile partition key");
  TilePart& tp = cn.tpart[key];
  tile_part_free(tp);
  static const int sets[4][2] = {{0, -1}, {4, -1}, {1, 2}, {5, 6}};
  const int v0 = sets[key][0], v1 = sets[key][1];
  if (!cn.disk || cn.ref_row < 0 || !cn.cpix[v0] || cn.count[v0] == 0 || (v1 >= 0 && (!cn.cpix[v1] || cn.count[v1] == 0)))
    return VIP_OK;
  const Lattice& L = c->lat;
  if (!L.ok) return VIP_OK;
  VIP_TRY(tile_part_build(c, L.W, L.H, L.node_of, c->n, c->tmap, cn.cpix[v0], v1 >= 0 ? cn.cpix[v1] : nullptr,
                          tp));
  if (c->debug)
    std::fprintf(stderr, "[vip] tile partition %d: %lld tiles, %lld irregular rows of %lld\n", key,
                 static_cast<long long>(tp.ntiles), static_cast<long long>(tp.nirr), static_cast<long long>(c->n));
  return VIP_OK;
}

void vip_canon_free(Ctx* c) {
  dfree(c->vcanon.cpix);
  tile_part_free(c->vcanon.tpart);
  c->vcanon = VipCanon();
}

// Canonical nodes that are not boundary nodes (the rows the step kernels take from LDS tiles).
__global__ void k_interior_canon(int64_t n, const int32_t* cpix, const int32_t* bpos, int32_t* out) {
  const int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
  if (i < n) out[i] = bpos[i] < 0 ? cpix[i] : -1;
}

int vip_canon_setup(Ctx* c) {
  vip_canon_free(c);
  VipCanon& V = c->vcanon;
  if (c->no_canon || c->n == 0) return VIP_OK;
  Ell* ops[kVcOps] = {&c->vipop[0], &c->vipop[1], &c->vipop[2], &c->vipop[3], &c->node};
  for (int o = 0; o < kVcOps; ++o) VIP_TRY(canon_mark(c, *ops[o], 0));
  VIP_TRY(canon_mark(c, c->node, 1));
  bool ok = true;
  for (int o = 0; o < kVcOps && ok; ++o) {
    const Canon& cn = ops[o]->canon;
    ok = cn.ref_row >= 0 && cn.cpix[0] && cn.count[0] > 0 && vc_runs(cn, V.dx0[o], V.len[o]);
    if (ok)
      for (int k = 0; k < cn.K; ++k) V.w[o][k] = cn.w[0][k];
  }
  ok = ok && c->node.canon.cpix[1] && c->node.canon.count[1] > 0;
  if (ok) {
    for (int k = 0; k < c->node.canon.K; ++k) V.w[kVcOps][k] = c->node.canon.w[1][k];
    for (int d = 0; d < kVcRows; ++d) {
      V.used[d] = 0;
      for (int o = 0; o < kVcOps; ++o) V.used[d] |= V.len[o][d] > 0 ? 1 : 0;
    }
    VIP_TRY(dalloc(c, &V.cpix, c->n));
    k_vc_combine<<<grid_for(c->n), kBlock, 0, c->stream>>>(
        c->n, ops[0]->canon.cpix[0], ops[1]->canon.cpix[0], ops[2]->canon.cpix[0], ops[3]->canon.cpix[0],
        c->node.canon.cpix[0], c->node.canon.cpix[1], V.cpix);
    VIP_HIP_TRY(c, hipGetLastError());
    int64_t* part = nullptr;
    VIP_TRY(dalloc(c, &part, 256));
    k_count_nonneg<<<256, 256, 0, c->stream>>>(c->n, V.cpix, part);
    std::vector<int64_t> hp(256);
    hipError_t e1 = hipMemcpyAsync(hp.data(), part, sizeof(int64_t) * 256, hipMemcpyDeviceToHost, c->stream);
    hipError_t e2 = hipStreamSynchronize(c->stream);
    dfree(part);
    if (e1 != hipSuccess || e2 != hipSuccess) return set_error(c, VIP_E_HIP, "counting canonical VIP rows");
    V.count = 0;
    for (int64_t v : hp) V.count += v;
  }
  // the per-operator marks are folded into V.cpix
  for (int o = 0; o < kVcOps; ++o) canon_free(ops[o]->canon);
  if (V.count == 0) vip_canon_free(c);
  // tiles for the step kernels: every tap of the reference rows within 3 pixels of the node
  bool fits = V.count > 0 && c->lat.ok;
  for (int o = 0; o < kVcOps && fits; ++o)
    for (int d = 0; d < kVcRows; ++d)
      if (V.len[o][d] > 0 && (V.dx0[o][d] < -3 || V.dx0[o][d] + V.len[o][d] - 1 > 3)) fits = false;
  if (fits) {
    int32_t* inner = nullptr;
    VIP_TRY(dalloc(c, &inner, c->n));
    k_interior_canon<<<grid_for(c->n), kBlock, 0, c->stream>>>(c->n, V.cpix, c->bpos, inner);
    const int rc = tile_part_build(c, c->lat.W, c->lat.H, c->lat.node_of, c->n, c->tmap, inner, nullptr, V.tpart);
    dfree(inner);
    VIP_TRY(rc);
    if (c->debug)
      std::fprintf(stderr, "[vip] step tiles: %lld tiles, %lld irregular nodes\n",
                   static_cast<long long>(V.tpart.ntiles), static_cast<long long>(V.tpart.nirr));
  }
  if (c->debug) {
    std::fprintf(stderr, "[vip] canonical VIP/node rows: %lld of %lld\n", static_cast<long long>(c->vcanon.count),
                 static_cast<long long>(c->n));
    for (int o = 0; o < kVcOps && c->vcanon.count > 0; ++o) {
      std::fprintf(stderr, "[vip] canonical runs of operator %d (dx0,len per dy = -3..3):", o);
      for (int d = 0; d < kVcRows; ++d) std::fprintf(stderr, " (%d,%d)", V.dx0[o][d], V.len[o][d]);
      std::fprintf(stderr, "\n");
    }
  }
  return VIP_OK;
}

}  // namespace vip
