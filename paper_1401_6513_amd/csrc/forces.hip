// Force on a body from the fluid, by traction on its surface nodes (the drag and lift
// coefficients of the cylinder cases, Section 5.4), and the dominant frequency of a sampled
// signal (the Strouhal number from the lift history).
//
// Traction.  Section 5.4 defines the traction as t = -p n + (1/Re) du/dn, n the outward normal
// of the flow domain (at a surface node it points into the body); the force of the fluid on
// the body is F = -sum over the surface of t dS.  (On a no-slip wall of an incompressible flow
// this is sigma n of the Newtonian stress: the extra term n (n . du/dn) vanishes there.)  The
// normal derivative is the one the boundary rows of eqs. 12-13 use: values interpolated by
// Psi^[0,0] at x_b - d n and x_b - 2 d n, du/dn = (3 u_b - 4 u(x_b - d n) + u(x_b - 2 d n)) / (2d),
// d = vip_offset h (exact for quadratics).  dS is the trapezoid weight of the closed chain of
// surface nodes: half the chords to the previous and the next node.
#include <hip/hip_runtime.h>

#include <cmath>
#include <mutex>
#include <vector>

#include "vip_internal.h"

namespace vip {
namespace {

struct NormalRows {
  const int64_t* ptr;
  const int32_t* rowlen;
  const int32_t* cols;
  const double* val;
};

__device__ __forceinline__ double row_dot(const NormalRows& e, int64_t r, const double* f) {
  const int64_t base = e.ptr[r / kSlice] + (r % kSlice);
  const int len = e.rowlen[r];
  double s = 0.0;
  for (int k = 0; k < len; ++k) {
    const int64_t q = base + static_cast<int64_t>(k) * kSlice;
    s = fma(e.val[q], f[e.cols[q]], s);
  }
  return s;
}

// traction times the trapezoid weight at each surface node: buf[2k], buf[2k + 1]
__global__ void k_traction(int64_t ns, const int64_t* surf, const int32_t* bpos, const double* bnx,
                           const double* bny, const double* x, const double* y, NormalRows n1, NormalRows n2,
                           const double* u, const double* v, const double* p, double inv_re, double inv_2d0,
                           const double* bscale, double* buf) {
  const int64_t k = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
  if (k >= ns) return;
  const int64_t i = surf[k];
  const int64_t ip = surf[(k + ns - 1) % ns], in = surf[(k + 1) % ns];
  const int32_t b = bpos[i];
  const double inv_2d = bscale ? inv_2d0 / bscale[b] : inv_2d0;   // local spacing on adaptive sets
  const double w = 0.5 * (hypot(x[in] - x[i], y[in] - y[i]) + hypot(x[i] - x[ip], y[i] - y[ip]));
  const double nx = bnx[b], ny = bny[b];
  const double dudn = (3.0 * u[i] - 4.0 * row_dot(n1, b, u) + row_dot(n2, b, u)) * inv_2d;
  const double dvdn = (3.0 * v[i] - 4.0 * row_dot(n1, b, v) + row_dot(n2, b, v)) * inv_2d;
  buf[2 * k] = w * (p[i] * nx - inv_re * dudn);
  buf[2 * k + 1] = w * (p[i] * ny - inv_re * dvdn);
}

// out[0..1] = sums of the pairs in buf, in a fixed order (one block)
__global__ void k_sum_pairs(int64_t ns, const double* buf, double* out) {
  __shared__ double sx[256], sy[256];
  double ax = 0.0, ay = 0.0;
  for (int64_t k = threadIdx.x; k < ns; k += blockDim.x) {
    ax += buf[2 * k];
    ay += buf[2 * k + 1];
  }
  sx[threadIdx.x] = ax;
  sy[threadIdx.x] = ay;
  __syncthreads();
  for (int off = blockDim.x / 2; off > 0; off >>= 1) {
    if (static_cast<int>(threadIdx.x) < off) {
      sx[threadIdx.x] += sx[threadIdx.x + off];
      sy[threadIdx.x] += sy[threadIdx.x + off];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    out[0] = sx[0];
    out[1] = sy[0];
  }
}

NormalRows rows_of(const Ell& e) { return NormalRows{e.ptr, e.rowlen, e.cols, e.val[0]}; }

}  // namespace

int forces_check(Ctx* c, const int64_t* surf, int64_t ns, double re) {
  if (!surf) return set_error(c, VIP_E_INVALID, "surface node list is NULL");
  if (ns < 3) return set_error(c, VIP_E_INVALID, "a closed surface chain needs at least 3 nodes");
  if (!(re > 0.0) || !std::isfinite(re)) return set_error(c, VIP_E_INVALID, "Re must be positive");
  for (int64_t k = 0; k < ns; ++k) {
    const int64_t i = surf[k];
    if (i < 0 || i >= c->n) return set_error(c, VIP_E_INVALID, "surface node index out of range");
    if (c->h_bpos[i] < 0)
      return set_error(c, VIP_E_INVALID, "surface node " + std::to_string(i) + " is not a boundary node");
  }
  return VIP_OK;
}

int forces(Ctx* c, const double* u, const double* v, const double* p, double re, const int64_t* surf,
           int64_t ns, double* out, int64_t* surf_dev, double* buf) {
  hipStream_t st = c->stream;
  VIP_HIP_TRY(c, hipMemcpyAsync(surf_dev, surf, sizeof(int64_t) * ns, hipMemcpyHostToDevice, st));
  const double d = c->opt.vip_offset * c->h;
  const int64_t blocks = (ns + kBlock - 1) / kBlock;
  k_traction<<<blocks, kBlock, 0, st>>>(ns, surf_dev, c->bpos, c->bnx, c->bny, c->x, c->y, rows_of(c->normal[0]),
                                        rows_of(c->normal[1]), u, v, p, 1.0 / re, 1.0 / (2.0 * d), c->bscale,
                                        buf);
  k_sum_pairs<<<1, 256, 0, st>>>(ns, buf, buf + 2 * ns);
  VIP_HIP_TRY(c, hipGetLastError());
  VIP_HIP_TRY(c, hipMemcpyAsync(out, buf + 2 * ns, 2 * sizeof(double), hipMemcpyDeviceToHost, st));
  VIP_HIP_TRY(c, hipStreamSynchronize(st));
  return VIP_OK;
}

void forces_free(Ctx* c) {
  dfree(c->fsurf);
  dfree(c->fbuf);
  c->fcap = 0;
}

// Work memory of vip_forces_noalloc: a file-scope device array, one copy per GPU, held until
// the process ends.  Host code never uses its name as an address: forces_scratch_init looks
// up each device's copy once (with that device current) and every later use goes through the
// pointer kept for that device.
constexpr int64_t kScratchBytes = int64_t{1} << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch[kMaxDevices] = {};
}  // namespace

// byte offset of the traction pairs behind a surface list of ns entries (256-byte aligned)
static int64_t scratch_buf_offset(int64_t ns) { return ((8 * ns + 255) / 256) * 256; }

int64_t forces_noalloc_max_surface() {
  // largest ns with offset(ns) + 8 (2 ns + 2) <= kScratchBytes
  int64_t lo = 0, hi = kScratchBytes / 8;
  while (lo < hi) {
    const int64_t mid = (lo + hi + 1) / 2;
    if (scratch_buf_offset(mid) + 8 * (2 * mid + 2) <= kScratchBytes)
      lo = mid;
    else
      hi = mid - 1;
  }
  return lo;
}

int forces_scratch_init(Ctx* c) {
  if (c->device < 0 || c->device >= kMaxDevices)
    return set_error(c, VIP_E_INVALID, "device index beyond the scratch table");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch[c->device]) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr)
      return set_error(c, VIP_E_HIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    g_scratch[c->device] = ptr;
  }
  c->scratch = g_scratch[c->device];
  return VIP_OK;
}

}  // namespace vip

using vip::Ctx;

extern "C" {

int vip_forces(void* p, const double* u, const double* v, const double* pr, double re, const int64_t* surf,
               int64_t n_surf, double* force) {
  Ctx* c = static_cast<Ctx*>(p);
  if (!c) return VIP_E_INVALID;
  if (!c->built) return vip::set_error(c, VIP_E_NOT_BUILT, "vip_build_stencils has not succeeded");
  if (!u || !v || !pr || !force) return vip::set_error(c, VIP_E_INVALID, "NULL vector or output");
  VIP_TRY(vip::forces_check(c, surf, n_surf, re));
  VIP_HIP_TRY(c, hipSetDevice(c->device));
  if (c->fcap < n_surf) {
    VIP_HIP_TRY(c, hipStreamSynchronize(c->stream));
    vip::forces_free(c);
    VIP_TRY(vip::dalloc(c, &c->fsurf, n_surf));
    VIP_TRY(vip::dalloc(c, &c->fbuf, 2 * n_surf + 2));
    c->fcap = n_surf;
  }
  return vip::forces(c, u, v, pr, re, surf, n_surf, force, c->fsurf, c->fbuf);
}

int vip_forces_noalloc(void* p, const double* u, const double* v, const double* pr, double re,
                       const int64_t* surf, int64_t n_surf, double* force) {
  Ctx* c = static_cast<Ctx*>(p);
  if (!c) return VIP_E_INVALID;
  if (!c->built) return vip::set_error(c, VIP_E_NOT_BUILT, "vip_build_stencils has not succeeded");
  if (!c->scratch) return vip::set_error(c, VIP_E_HIP, "no scratch memory on this device");
  if (!u || !v || !pr || !force) return vip::set_error(c, VIP_E_INVALID, "NULL vector or output");
  const int64_t cap = vip::forces_noalloc_max_surface();
  if (n_surf > cap)
    return vip::set_error(c, VIP_E_INVALID, "n_surf = " + std::to_string(n_surf) +
                                                " exceeds the fixed scratch of vip_forces_noalloc (at most " +
                                                std::to_string(cap) + " surface nodes)");
  VIP_TRY(vip::forces_check(c, surf, n_surf, re));
  VIP_HIP_TRY(c, hipSetDevice(c->device));
  unsigned char* base = static_cast<unsigned char*>(c->scratch);
  return vip::forces(c, u, v, pr, re, surf, n_surf, force, reinterpret_cast<int64_t*>(base),
                     reinterpret_cast<double*>(base + vip::scratch_buf_offset(n_surf)));
}

// Dominant frequency of a real signal: the maximum of the Hann-windowed periodogram (mean
// removed), first on the DFT bins k / (n dt), k = 1 .. n/2, then refined on the continuous
// spectrum between the neighbouring bins by golden-section search.
int vip_spectral_peak(const double* s, int64_t n, double dt, double* freq, double* amp) {
  if (!s || !freq || n < 8 || !(dt > 0.0)) return VIP_E_INVALID;
  double mean = 0.0;
  for (int64_t k = 0; k < n; ++k) {
    if (!std::isfinite(s[k])) return VIP_E_INVALID;
    mean += s[k];
  }
  mean /= static_cast<double>(n);
  const double pi = 3.14159265358979323846;
  std::vector<double> w(n);
  double wsum = 0.0;
  for (int64_t k = 0; k < n; ++k) {
    w[k] = (s[k] - mean) * 0.5 * (1.0 - std::cos(2.0 * pi * static_cast<double>(k) / static_cast<double>(n - 1)));
    wsum += 0.5 * (1.0 - std::cos(2.0 * pi * static_cast<double>(k) / static_cast<double>(n - 1)));
  }
  // |sum_k w_k exp(-2 pi i f k dt)|^2, evaluated by the angle-addition recurrence
  auto power = [&](double f) {
    const double th = 2.0 * pi * f * dt;
    const double c1 = std::cos(th), s1 = std::sin(th);
    double cr = 1.0, ci = 0.0, re = 0.0, im = 0.0;
    for (int64_t k = 0; k < n; ++k) {
      re += w[k] * cr;
      im -= w[k] * ci;
      const double t = cr * c1 - ci * s1;
      ci = cr * s1 + ci * c1;
      cr = t;
    }
    return re * re + im * im;
  };
  const double df = 1.0 / (static_cast<double>(n) * dt);
  int64_t best = 1;
  double pbest = -1.0;
  for (int64_t k = 1; k <= n / 2; ++k) {
    const double pk = power(k * df);
    if (pk > pbest) {
      pbest = pk;
      best = k;
    }
  }
  double a = (best - 1) * df, b = (best + 1) * df;
  const double g = 0.5 * (std::sqrt(5.0) - 1.0);
  double x1 = b - g * (b - a), x2 = a + g * (b - a);
  double p1 = power(x1), p2 = power(x2);
  for (int it = 0; it < 60; ++it) {
    if (p1 > p2) {
      b = x2;
      x2 = x1;
      p2 = p1;
      x1 = b - g * (b - a);
      p1 = power(x1);
    } else {
      a = x1;
      x1 = x2;
      p1 = p2;
      x2 = a + g * (b - a);
      p2 = power(x2);
    }
  }
  const double f = 0.5 * (a + b);
  *freq = f;
  // amplitude of a sinusoid with that periodogram peak: 2 |X(f)| / sum(window)
  if (amp) *amp = 2.0 * std::sqrt(power(f)) / wsum;
  return VIP_OK;
}

}  // extern "C"
