// C ABI entry points (include/vip.h): argument checks, context lifetime and
// dispatch to the build, step and solver code.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdlib>
#include <cstring>
#include <new>
#include <vector>

#include "vip_internal.h"

namespace vip {

int set_error(Ctx* c, int code, const std::string& msg) {
  if (c) {
    c->err.code = code;
    c->err.msg = msg;
  }
  return code;
}

void ell_free(Ell& e) {
  canon_free(e.canon);
  dfree(e.ptr);
  dfree(e.width);
  dfree(e.rowlen);
  dfree(e.cols);
  dfree(e.dcols);
  dfree(e.dfit);
  for (auto& v : e.val) dfree(v);
  dfree(e.val32);
  dfree(e.rsum32);
  for (auto& v : e.val32h) dfree(v);
  for (auto& v : e.rsum32h) dfree(v);
  e = Ell{};
}

void ctx_free_build(Ctx* c) {
  c->built = false;
  amg_free(c);
  dfree(c->x);
  dfree(c->y);
  dfree(c->bpos);
  dfree(c->bidx);
  dfree(c->bnx);
  dfree(c->bny);
  dfree(c->bkind);
  dfree(c->bval);
  dfree(c->hscale);
  dfree(c->bscale);
  dfree(c->two_db);
  dfree(c->vip_px);
  dfree(c->vip_py);
  dfree(c->d_ew);
  dfree(c->d_ns);
  dfree(c->rho_node);
  ell_free(c->node);
  for (auto& e : c->vipop) ell_free(e);
  for (auto& e : c->normal) ell_free(e);
  ell_free(c->sys);
  for (auto& d : c->dinv) dfree(d);
  dfree(c->dinv32);
  dfree(c->nprev);
  dfree(c->stepbuf);
  dfree(c->star_ring);
  c->nstar = 0;
  dfree(c->phi);
  dfree(c->ws);
  c->ws_len = 0;
  dfree(c->ws32);
  c->ws32_len = 0;
  c->assembled = false;
  c->have_prev_n = false;
  c->nstar = 0;
  c->have_prev_phi = false;
  learn_free_nodeset(c);
  vip_canon_free(c);
  tile_map_free(c->tmap);
  lattice_free(c->lat);
  for (auto& h : c->hint_p64) h = 0;
  for (auto& h : c->hint_p32) h = 0;
  for (auto& h : c->hint_h32) h = 0;
  c->hint_h = 0;
}

namespace {

Ctx* as_ctx(void* p) { return static_cast<Ctx*>(p); }

int need_built(Ctx* c) {
  if (!c) return VIP_E_INVALID;
  if (!c->built) return set_error(c, VIP_E_NOT_BUILT, "vip_build_stencils has not succeeded");
  return VIP_OK;
}

int bind_device(Ctx* c) {
  VIP_HIP_TRY(c, hipSetDevice(c->device));
  return VIP_OK;
}

const Ell* op_of(Ctx* c, int which, int* vs, bool* f32) {
  *f32 = false;
  *vs = 0;
  switch (which) {
    case VIP_OP_IDENTITY: return &c->node;
    case VIP_OP_LAPLACIAN: *vs = 1; return &c->node;
    case VIP_OP_VIP_E: return &c->vipop[0];
    case VIP_OP_VIP_W: return &c->vipop[1];
    case VIP_OP_VIP_N: return &c->vipop[2];
    case VIP_OP_VIP_S: return &c->vipop[3];
    case VIP_OP_NORMAL1: return &c->normal[0];
    case VIP_OP_NORMAL2: return &c->normal[1];
    case VIP_OP_POISSON: return &c->sys;
    case VIP_OP_HELM_U: *vs = 1; return &c->sys;
    case VIP_OP_HELM_V: *vs = 2; return &c->sys;
    case VIP_OP_POISSON32: *f32 = true; return &c->sys;
    default: return nullptr;
  }
}

}  // namespace
}  // namespace vip

using vip::Ctx;

extern "C" {

void vip_default_options(vip_options* o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->weight = VIP_W_CUBIC_SPLINE;
  o->identity = VIP_I_MLS;
  o->precision = VIP_P_FP64;
  o->krylov = VIP_K_AUTO;
  o->warmstart = VIP_WS_ZERO;
  o->min_neighbours = 12;
  o->vip_offset = 0.5;
  o->period[0] = 0.0;
  o->period[1] = 0.0;
  o->poisson_tol = 1e-8;
  o->helmholtz_tol = 1e-12;
  o->inner_tol = 1e-5;
  o->max_iters = 200000;
  o->check_every = 16;
  o->preconditioner = VIP_PC_AMG;
}

int vip_create(void** out, int device, void* stream) {
  if (!out) return VIP_E_INVALID;
  *out = nullptr;
  Ctx* c = new (std::nothrow) Ctx();
  if (!c) return VIP_E_INVALID;
  c->device = device;
  c->stream = static_cast<hipStream_t>(stream);
  const char* dbg = std::getenv("VIP_DEBUG");
  c->debug = (dbg && dbg[0] == '1') ? 1 : 0;
  const char* nc = std::getenv("VIP_NO_CANON");
  c->no_canon = (nc && nc[0] == '1') ? 1 : 0;
  const char* cl = std::getenv("VIP_CNN_LAYERED");
  c->cnn_layered = (cl && cl[0] == '1') ? 1 : 0;
  const char* nd = std::getenv("VIP_NO_DELTA");
  c->no_delta = (nd && nd[0] == '1') ? 1 : 0;
  const char* nf = std::getenv("VIP_NO_FUSE");
  c->no_fuse = (nf && nf[0] == '1') ? 1 : 0;
  const char* ng = std::getenv("VIP_NO_GRAPH");
  c->no_graph = (ng && ng[0] == '1') ? 1 : 0;
  const char* pre = std::getenv("VIP_AMG_PRE_FINE");
  c->amg_pre_fine = (pre && pre[0] == '0') ? 0 : 1;
  if (const char* g = std::getenv("VIP_AMG_GAMMA")) c->amg_gamma = std::min(2.0, std::max(0.5, std::atof(g)));
  if (const char* v = std::getenv("VIP_AMG_NU")) c->amg_nu = std::min(8, std::max(1, std::atoi(v)));
  if (const char* v = std::getenv("VIP_AMG_NU_COARSE")) c->amg_nu_coarse = std::min(4, std::max(1, std::atoi(v)));
  vip_default_options(&c->opt);
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) {
    delete c;
    return VIP_E_HIP;
  }
  if (hipSetDevice(device) != hipSuccess || hipMalloc(&c->sc, sizeof(vip::KrylovScalars)) != hipSuccess ||
      hipHostMalloc(&c->sc_host, sizeof(vip::KrylovScalars), hipHostMallocDefault) != hipSuccess ||
      hipMemset(c->sc, 0, sizeof(vip::KrylovScalars)) != hipSuccess ||
      vip::forces_scratch_init(c) != VIP_OK) {
    if (c->sc) (void)hipFree(c->sc);
    if (c->sc_host) (void)hipHostFree(c->sc_host);
    delete c;
    return VIP_E_HIP;
  }
  *out = c;
  return VIP_OK;
}

int vip_destroy(void* p) {
  Ctx* c = vip::as_ctx(p);
  if (!c) return VIP_E_INVALID;
  (void)hipSetDevice(c->device);
  (void)hipStreamSynchronize(c->stream);
  vip::ctx_free_build(c);
  vip::learn_free(c);
  vip::forces_free(c);
  vip::dfree(c->partials);
  vip::dfree(c->sc);
  if (c->sc_host) (void)hipHostFree(c->sc_host);
  for (auto& e : c->timing.pool) {
    (void)hipEventDestroy(e.first);
    (void)hipEventDestroy(e.second);
  }
  for (auto& e : c->timing.pending) {
    (void)hipEventDestroy(e.first);
    (void)hipEventDestroy(e.second);
  }
  for (auto* T : {&c->conv_timing, &c->ktime[0], &c->ktime[1], &c->ktime[2], &c->ktime[3], &c->ktime[4]}) {
    for (auto& e : T->pool) {
      (void)hipEventDestroy(e.first);
      (void)hipEventDestroy(e.second);
    }
    for (auto& e : T->pending) {
      (void)hipEventDestroy(e.first);
      (void)hipEventDestroy(e.second);
    }
  }
  delete c;
  return VIP_OK;
}

const char* vip_last_error(const void* p) {
  const Ctx* c = static_cast<const Ctx*>(p);
  if (!c) return "null context";
  return c->err.msg.c_str();
}

int vip_build_stencils(void* p, const double* nodes_xy, int64_t n_nodes, const int64_t* bnd_idx,
                       const double* bnd_normal, const int32_t* bnd_kind, const double* bnd_value,
                       int64_t n_bnd, int basis_order, double support_radius, double h,
                       const vip_options* opt) {
  Ctx* c = vip::as_ctx(p);
  if (!c) return VIP_E_INVALID;
  VIP_TRY(vip::bind_device(c));
  int rc = vip::build_stencils(c, nodes_xy, n_nodes, bnd_idx, bnd_normal, bnd_kind, bnd_value, n_bnd,
                               basis_order, support_radius, h, opt);
  if (rc != VIP_OK) c->built = false;
  return rc;
}

int vip_build_stencils_adaptive(void* p, const double* nodes_xy, int64_t n_nodes, const int64_t* bnd_idx,
                                const double* bnd_normal, const int32_t* bnd_kind, const double* bnd_value,
                                int64_t n_bnd, int basis_order, double support_radius, double h,
                                const double* h_node, const vip_options* opt) {
  Ctx* c = vip::as_ctx(p);
  if (!c) return VIP_E_INVALID;
  if (!h_node) return vip::set_error(c, VIP_E_INVALID, "h_node is NULL");
  VIP_TRY(vip::bind_device(c));
  int rc = vip::build_stencils(c, nodes_xy, n_nodes, bnd_idx, bnd_normal, bnd_kind, bnd_value, n_bnd,
                               basis_order, support_radius, h, opt, h_node);
  if (rc != VIP_OK) c->built = false;
  return rc;
}

int vip_column_bytes(void* p, int64_t* sys_entries, int64_t* sys_entries_int16, int* amg_levels,
                     int* amg_levels_delta) {
  Ctx* c = vip::as_ctx(p);
  VIP_TRY(vip::need_built(c));
  if (sys_entries) *sys_entries = c->sys.nnz;
  if (sys_entries_int16) *sys_entries_int16 = c->sys.dcols ? c->sys.dfit_nnz : 0;
  int nl = 0, nd = 0;
  for (size_t l = 1; l < c->amg.lv.size(); ++l) {
    if (c->amg.lv[l].A.nrows == 0) continue;
    ++nl;
    nd += c->amg.lv[l].A.dcols ? 1 : 0;
  }
  if (amg_levels) *amg_levels = nl;
  if (amg_levels_delta) *amg_levels_delta = nd;
  return VIP_OK;
}

int vip_set_options(void* p, const vip_options* opt) {
  Ctx* c = vip::as_ctx(p);
  VIP_TRY(vip::need_built(c));
  if (!opt) return vip::set_error(c, VIP_E_INVALID, "options pointer is NULL");
  if (opt->precision != VIP_P_FP64 && opt->precision != VIP_P_MIXED)
    return vip::set_error(c, VIP_E_INVALID, "unknown precision");
  if (opt->krylov < VIP_K_AUTO || opt->krylov > VIP_K_BICGSTAB)
    return vip::set_error(c, VIP_E_INVALID, "unknown krylov method");
  if (opt->identity != VIP_I_MLS && opt->identity != VIP_I_EXACT)
    return vip::set_error(c, VIP_E_INVALID, "unknown identity");
  if (opt->warmstart < VIP_WS_ZERO || opt->warmstart > VIP_WS_EXTRAP)
    return vip::set_error(c, VIP_E_INVALID, "unknown warm start");
  if (opt->preconditioner != VIP_PC_JACOBI && opt->preconditioner != VIP_PC_AMG)
    return vip::set_error(c, VIP_E_INVALID, "unknown preconditioner");
  if (!(opt->poisson_tol > 0.0) || !(opt->helmholtz_tol > 0.0) || !(opt->inner_tol > 0.0) ||
      opt->max_iters <= 0 || opt->check_every <= 0)
    return vip::set_error(c, VIP_E_INVALID, "tolerances and limits must be positive");
  const bool id_changed = opt->identity != c->opt.identity;
  vip_options keep = c->opt;
  c->opt = *opt;
  // stencil-defining fields stay as built
  c->opt.weight = keep.weight;
  c->opt.vip_offset = keep.vip_offset;
  c->opt.period[0] = keep.period[0];
  c->opt.period[1] = keep.period[1];
  c->opt.min_neighbours = keep.min_neighbours;
  if (id_changed) c->assembled = false;
  return VIP_OK;
}

int vip_step(void* p, double* u, double* v, double* pr, double dt, double Re, vip_step_stats* st) {
  Ctx* c = vip::as_ctx(p);
  VIP_TRY(vip::need_built(c));
  if (!u || !v || !pr) return vip::set_error(c, VIP_E_INVALID, "state pointer is NULL");
  if (!(dt > 0.0) || !(Re > 0.0) || !std::isfinite(dt) || !std::isfinite(Re))
    return vip::set_error(c, VIP_E_INVALID, "dt and Re must be positive and finite");
  VIP_TRY(vip::bind_device(c));
  if (st) std::memset(st, 0, sizeof(*st));
  return vip::step(c, u, v, pr, dt, Re, st);
}

int vip_reset_history(void* p) {
  Ctx* c = vip::as_ctx(p);
  VIP_TRY(vip::need_built(c));
  c->have_prev_n = false;
  c->nstar = 0;
  c->have_prev_phi = false;
  c->learn.have_eprev = false;
  c->learn.have_eprev2 = false;
  return VIP_OK;
}

int vip_poisson_solve(void* p, const double* rhs, double* phi, double tol, int use_x0,
                      vip_step_stats* st) {
  Ctx* c = vip::as_ctx(p);
  VIP_TRY(vip::need_built(c));
  if (!rhs || !phi) return vip::set_error(c, VIP_E_INVALID, "NULL vector");
  if (!(tol > 0.0)) return vip::set_error(c, VIP_E_INVALID, "tol must be > 0");
  VIP_TRY(vip::bind_device(c));
  if (st) std::memset(st, 0, sizeof(*st));
  int rc = vip::poisson_solve(c, rhs, phi, tol, use_x0 != 0, st);
  VIP_HIP_TRY(c, hipStreamSynchronize(c->stream));
  return rc;
}

int vip_operator_shape(void* p, int which, int64_t* n_rows, int64_t* max_width, int64_t* nnz) {
  Ctx* c = vip::as_ctx(p);
  VIP_TRY(vip::need_built(c));
  int vs;
  bool f32;
  const vip::Ell* e = vip::op_of(c, which, &vs, &f32);
  if (!e) return vip::set_error(c, VIP_E_INVALID, "unknown operator");
  if (n_rows) *n_rows = e->nrows;
  if (max_width) *max_width = e->max_width;
  if (nnz) *nnz = e->nnz;
  return VIP_OK;
}

int vip_get_operator(void* p, int which, int32_t* cols, double* vals) {
  Ctx* c = vip::as_ctx(p);
  VIP_TRY(vip::need_built(c));
  int vs;
  bool f32;
  const vip::Ell* e = vip::op_of(c, which, &vs, &f32);
  if (!e) return vip::set_error(c, VIP_E_INVALID, "unknown operator");
  if ((which == VIP_OP_HELM_U || which == VIP_OP_HELM_V) && !c->assembled)
    return vip::set_error(c, VIP_E_NOT_BUILT, "Helmholtz operators not assembled (call vip_assemble)");
  if (!cols || !vals) return vip::set_error(c, VIP_E_INVALID, "NULL output");
  VIP_TRY(vip::bind_device(c));
  const int64_t nr = e->nrows, W = e->max_width, ns = e->nslices, nz = e->nnz_slots;
  std::vector<int64_t> ptr(ns + 1);
  std::vector<int32_t> rowlen(nr), col(nz);
  std::vector<double> val(nz);
  std::vector<float> val32;
  hipStream_t s = c->stream;
  VIP_HIP_TRY(c, hipMemcpyAsync(ptr.data(), e->ptr, sizeof(int64_t) * (ns + 1), hipMemcpyDeviceToHost, s));
  if (nr > 0)
    VIP_HIP_TRY(c, hipMemcpyAsync(rowlen.data(), e->rowlen, sizeof(int32_t) * nr, hipMemcpyDeviceToHost, s));
  if (nz > 0) {
    VIP_HIP_TRY(c, hipMemcpyAsync(col.data(), e->cols, sizeof(int32_t) * nz, hipMemcpyDeviceToHost, s));
    if (f32) {
      val32.resize(nz);
      VIP_HIP_TRY(c, hipMemcpyAsync(val32.data(), e->val32, sizeof(float) * nz, hipMemcpyDeviceToHost, s));
    } else {
      VIP_HIP_TRY(c, hipMemcpyAsync(val.data(), e->val[vs], sizeof(double) * nz, hipMemcpyDeviceToHost, s));
    }
  }
  VIP_HIP_TRY(c, hipStreamSynchronize(s));
  for (int64_t r = 0; r < nr; ++r) {
    const int64_t sl = r / vip::kSlice, l = r % vip::kSlice;
    for (int64_t k = 0; k < W; ++k) {
      int32_t cc = -1;
      double vv = 0.0;
      if (k < rowlen[r]) {
        const int64_t q = ptr[sl] + k * vip::kSlice + l;
        cc = col[q];
        vv = f32 ? static_cast<double>(val32[q]) : val[q];
      }
      cols[r * W + k] = cc;
      vals[r * W + k] = vv;
    }
  }
  return VIP_OK;
}

int vip_apply(void* p, int which, const double* x, double* y) {
  Ctx* c = vip::as_ctx(p);
  VIP_TRY(vip::need_built(c));
  int vs;
  bool f32;
  const vip::Ell* e = vip::op_of(c, which, &vs, &f32);
  if (!e || f32 || which == VIP_OP_NORMAL1 || which == VIP_OP_NORMAL2)
    return vip::set_error(c, VIP_E_INVALID, "operator cannot be applied (needs N rows, FP64)");
  if ((which == VIP_OP_HELM_U || which == VIP_OP_HELM_V) && !c->assembled)
    return vip::set_error(c, VIP_E_NOT_BUILT, "Helmholtz operators not assembled (call vip_assemble)");
  if (!x || !y) return vip::set_error(c, VIP_E_INVALID, "NULL vector");
  VIP_TRY(vip::bind_device(c));
  VIP_TRY(vip::ell_apply(c, *e, vs, x, y));
  VIP_HIP_TRY(c, hipStreamSynchronize(c->stream));
  return VIP_OK;
}

int vip_assemble(void* p, double dt, double Re) {
  Ctx* c = vip::as_ctx(p);
  VIP_TRY(vip::need_built(c));
  if (!(dt > 0.0) || !(Re > 0.0)) return vip::set_error(c, VIP_E_INVALID, "dt and Re must be positive");
  VIP_TRY(vip::bind_device(c));
  VIP_TRY(vip::assemble_helmholtz(c, dt, Re));
  c->have_prev_n = false;
  c->nstar = 0;
  VIP_HIP_TRY(c, hipStreamSynchronize(c->stream));
  return VIP_OK;
}

int vip_get_geometry(void* p, double* vip_xy, double* d_ew, double* d_ns, double* rho_node) {
  Ctx* c = vip::as_ctx(p);
  VIP_TRY(vip::need_built(c));
  VIP_TRY(vip::bind_device(c));
  const int64_t n = c->n;
  hipStream_t s = c->stream;
  if (vip_xy) {
    std::vector<double> px(4 * n), py(4 * n);
    VIP_HIP_TRY(c, hipMemcpyAsync(px.data(), c->vip_px, sizeof(double) * 4 * n, hipMemcpyDeviceToHost, s));
    VIP_HIP_TRY(c, hipMemcpyAsync(py.data(), c->vip_py, sizeof(double) * 4 * n, hipMemcpyDeviceToHost, s));
    VIP_HIP_TRY(c, hipStreamSynchronize(s));
    for (int64_t i = 0; i < n; ++i)
      for (int k = 0; k < 4; ++k) {
        vip_xy[(i * 4 + k) * 2 + 0] = px[k * n + i];
        vip_xy[(i * 4 + k) * 2 + 1] = py[k * n + i];
      }
  }
  if (d_ew) VIP_HIP_TRY(c, hipMemcpyAsync(d_ew, c->d_ew, sizeof(double) * n, hipMemcpyDeviceToHost, s));
  if (d_ns) VIP_HIP_TRY(c, hipMemcpyAsync(d_ns, c->d_ns, sizeof(double) * n, hipMemcpyDeviceToHost, s));
  if (rho_node)
    VIP_HIP_TRY(c, hipMemcpyAsync(rho_node, c->rho_node, sizeof(double) * n, hipMemcpyDeviceToHost, s));
  VIP_HIP_TRY(c, hipStreamSynchronize(s));
  return VIP_OK;
}

int vip_convection(void* p, const double* u, const double* v, double* nx, double* ny) {
  Ctx* c = vip::as_ctx(p);
  VIP_TRY(vip::need_built(c));
  if (!u || !v || !nx || !ny) return vip::set_error(c, VIP_E_INVALID, "NULL vector");
  VIP_TRY(vip::bind_device(c));
  return vip::convection(c, u, v, nx, ny);
}

int vip_divergence(void* p, const double* u, const double* v, double* d) {
  Ctx* c = vip::as_ctx(p);
  VIP_TRY(vip::need_built(c));
  if (!u || !v || !d) return vip::set_error(c, VIP_E_INVALID, "NULL vector");
  VIP_TRY(vip::bind_device(c));
  return vip::divergence(c, u, v, d);
}

int vip_gradient(void* p, const double* f, double* gx, double* gy) {
  Ctx* c = vip::as_ctx(p);
  VIP_TRY(vip::need_built(c));
  if (!f || !gx || !gy) return vip::set_error(c, VIP_E_INVALID, "NULL vector");
  VIP_TRY(vip::bind_device(c));
  return vip::gradient(c, f, gx, gy);
}

int vip_kernel_timing(void* p, int which, int enable, int reset, double* avg_ms, int64_t* count) {
  Ctx* c = vip::as_ctx(p);
  if (!c) return VIP_E_INVALID;
  if (which < 0 || which >= 2 + vip::kTimedKinds) return vip::set_error(c, VIP_E_INVALID, "unknown timed kernel");
  vip::Timing& T = which == 0 ? c->timing : which == 1 ? c->conv_timing : c->ktime[which - 2];
  if (reset) {
    T.total_ms = 0.0;
    T.count = 0;
  }
  T.enabled = enable != 0;
  if (avg_ms) *avg_ms = T.count > 0 ? T.total_ms / T.count : 0.0;
  if (count) *count = T.count;
  return VIP_OK;
}

int vip_canonical_rows(void* p, int64_t* counts, int64_t* described, int* taps) {
  Ctx* c = vip::as_ctx(p);
  VIP_TRY(vip::need_built(c));
  const vip::Canon& cn = c->sys.canon;
  if (counts)
    for (int k = 0; k < 7; ++k) counts[k] = c->no_canon ? 0 : k == 3 ? c->vcanon.count : cn.count[k];
  if (described)
    for (int k = 0; k < 7; ++k) described[k] = c->no_canon ? 0 : cn.described[k];
  if (taps) *taps = cn.K;
  return VIP_OK;
}

int vip_learn_n_params(void) { return vip::learn_n_params(); }

int vip_learn_init(void* p, uint64_t seed) {
  Ctx* c = vip::as_ctx(p);
  if (!c) return VIP_E_INVALID;
  VIP_TRY(vip::bind_device(c));
  return vip::learn_init(c, seed);
}

int vip_learn_set_params(void* p, const double* theta, int64_t n) {
  Ctx* c = vip::as_ctx(p);
  if (!c) return VIP_E_INVALID;
  if (!theta || n != vip::learn_n_params())
    return vip::set_error(c, VIP_E_INVALID, "parameter vector must hold vip_learn_n_params() values");
  VIP_TRY(vip::bind_device(c));
  return vip::learn_set_params(c, theta);
}

int vip_learn_get_params(void* p, double* theta, int64_t n) {
  Ctx* c = vip::as_ctx(p);
  if (!c) return VIP_E_INVALID;
  if (!theta || n != vip::learn_n_params())
    return vip::set_error(c, VIP_E_INVALID, "parameter vector must hold vip_learn_n_params() values");
  VIP_TRY(vip::bind_device(c));
  return vip::learn_get_params(c, theta);
}

int vip_learn_eval(void* p, const double* x, const double* target, const double* mask, int batch, int height,
                   int width, double* y, double* loss, double* grad, double lr) {
  Ctx* c = vip::as_ctx(p);
  if (!c) return VIP_E_INVALID;
  VIP_TRY(vip::bind_device(c));
  return vip::learn_eval(c, x, target, mask, batch, height, width, y, loss, grad, lr);
}

int vip_learn_infer(void* p, const double* x, int batch, int height, int width, double* y) {
  Ctx* c = vip::as_ctx(p);
  if (!c) return VIP_E_INVALID;
  VIP_TRY(vip::bind_device(c));
  return vip::learn_infer(c, x, batch, height, width, y);
}

int vip_learn_capture(void* p, int max_snapshots) {
  Ctx* c = vip::as_ctx(p);
  if (!c) return VIP_E_INVALID;
  if (max_snapshots < 0) return vip::set_error(c, VIP_E_INVALID, "max_snapshots must be >= 0");
  c->learn.capacity = max_snapshots;
  return VIP_OK;
}

int vip_learn_snapshot_count(void* p, int* count) {
  Ctx* c = vip::as_ctx(p);
  if (!c || !count) return VIP_E_INVALID;
  *count = static_cast<int>(c->learn.snaps.size());
  return VIP_OK;
}

int vip_learn_clear(void* p) {
  Ctx* c = vip::as_ctx(p);
  if (!c) return VIP_E_INVALID;
  VIP_TRY(vip::bind_device(c));
  VIP_HIP_TRY(c, hipStreamSynchronize(c->stream));
  vip::learn_clear(c);
  return VIP_OK;
}

int vip_learn_train(void* p, int iters, int batch, int crop, double lr, uint64_t seed, double* last_loss) {
  Ctx* c = vip::as_ctx(p);
  if (!c) return VIP_E_INVALID;
  VIP_TRY(vip::bind_device(c));
  return vip::learn_train(c, iters, batch, crop, lr, seed, last_loss);
}

}  // extern "C"
