"""Thin Python binding of the C ABI in include/vip.h (argument marshalling only).

Every computation runs in the HIP library libvip.so built in this package
directory; importing this module without the library raises.  Device arrays
are torch tensors (float64, contiguous, on the context's device), passed by
data pointer; host arrays are NumPy arrays.  PyTorch supplies only device
memory and the stream.
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libvip.so")

VIP_OK = 0
ERRORS = {-1: "VIP_E_INVALID", -2: "VIP_E_SINGULAR", -3: "VIP_E_NOT_CONVERGED", -4: "VIP_E_HIP",
          -5: "VIP_E_NOT_BUILT", -6: "VIP_E_NONFINITE"}
VIP_E_NOT_CONVERGED = -3

BC_DIRICHLET, BC_SLIP, BC_OUTLET = 0, 1, 2
W_CUBIC_SPLINE, W_PAPER = 0, 1
I_MLS, I_EXACT = 0, 1
P_FP64, P_MIXED = 0, 1
K_AUTO, K_PCG, K_BICGSTAB = 0, 1, 2
WS_ZERO, WS_PREV, WS_LEARNED, WS_EXTRAP = 0, 1, 2, 3
PC_JACOBI, PC_AMG = 0, 1
OP = dict(identity=0, laplacian=1, vip_e=2, vip_w=3, vip_n=4, vip_s=5, normal1=6, normal2=7,
          poisson=8, helm_u=9, helm_v=10, poisson32=11)


class VipOptions(ctypes.Structure):
    _fields_ = [("weight", ctypes.c_int), ("identity", ctypes.c_int), ("precision", ctypes.c_int),
                ("krylov", ctypes.c_int), ("warmstart", ctypes.c_int),
                ("min_neighbours", ctypes.c_int), ("vip_offset", ctypes.c_double),
                ("period", ctypes.c_double * 2), ("poisson_tol", ctypes.c_double),
                ("helmholtz_tol", ctypes.c_double), ("inner_tol", ctypes.c_double),
                ("max_iters", ctypes.c_int), ("check_every", ctypes.c_int),
                ("preconditioner", ctypes.c_int), ("learned_precond", ctypes.c_int)]


class VipStepStats(ctypes.Structure):
    _fields_ = [("poisson_iters", ctypes.c_int), ("poisson_outer", ctypes.c_int),
                ("helmholtz_iters", ctypes.c_int), ("krylov_used", ctypes.c_int),
                ("poisson_residual", ctypes.c_double), ("helmholtz_residual", ctypes.c_double),
                ("border_lambda", ctypes.c_double), ("warm_start", ctypes.c_int),
                ("warm_ratio", ctypes.c_double), ("warm_alpha", ctypes.c_double),
                ("warm_beta", ctypes.c_double), ("poisson_fp64_fallback", ctypes.c_int),
                ("learned_pc_passes", ctypes.c_int), ("learned_pc_ratio", ctypes.c_double),
                ("warm_gamma", ctypes.c_double)]

    def as_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_}


class VipError(RuntimeError):
    def __init__(self, code, func, msg):
        super().__init__("%s returned %s: %s" % (func, ERRORS.get(code, code), msg))
        self.code = code


_lib = None

_P = ctypes.c_void_p
_I64 = ctypes.c_int64
_D = ctypes.c_double
_INT = ctypes.c_int

SIGNATURES = {
    "vip_default_options": (None, [ctypes.POINTER(VipOptions)]),
    "vip_create": (_INT, [ctypes.POINTER(ctypes.c_void_p), _INT, _P]),
    "vip_destroy": (_INT, [_P]),
    "vip_last_error": (ctypes.c_char_p, [_P]),
    "vip_build_stencils": (_INT, [_P, _P, _I64, _P, _P, _P, _P, _I64, _INT, _D, _D,
                                  ctypes.POINTER(VipOptions)]),
    "vip_build_stencils_adaptive": (_INT, [_P, _P, _I64, _P, _P, _P, _P, _I64, _INT, _D, _D, _P,
                                           ctypes.POINTER(VipOptions)]),
    "vip_set_options": (_INT, [_P, ctypes.POINTER(VipOptions)]),
    "vip_step": (_INT, [_P, _P, _P, _P, _D, _D, ctypes.POINTER(VipStepStats)]),
    "vip_reset_history": (_INT, [_P]),
    "vip_poisson_solve": (_INT, [_P, _P, _P, _D, _INT, ctypes.POINTER(VipStepStats)]),
    "vip_operator_shape": (_INT, [_P, _INT, ctypes.POINTER(_I64), ctypes.POINTER(_I64),
                                  ctypes.POINTER(_I64)]),
    "vip_get_operator": (_INT, [_P, _INT, _P, _P]),
    "vip_apply": (_INT, [_P, _INT, _P, _P]),
    "vip_assemble": (_INT, [_P, _D, _D]),
    "vip_get_geometry": (_INT, [_P, _P, _P, _P, _P]),
    "vip_convection": (_INT, [_P, _P, _P, _P, _P]),
    "vip_divergence": (_INT, [_P, _P, _P, _P]),
    "vip_gradient": (_INT, [_P, _P, _P, _P]),
    "vip_kernel_timing": (_INT, [_P, _INT, _INT, _INT, ctypes.POINTER(_D), ctypes.POINTER(_I64)]),
    "vip_canonical_rows": (_INT, [_P, _P, _P, ctypes.POINTER(_INT)]),
    "vip_column_bytes": (_INT, [_P, ctypes.POINTER(_I64), ctypes.POINTER(_I64), ctypes.POINTER(_INT),
                                ctypes.POINTER(_INT)]),
    "vip_forces": (_INT, [_P, _P, _P, _P, _D, _P, _I64, _P]),
    "vip_forces_noalloc": (_INT, [_P, _P, _P, _P, _D, _P, _I64, _P]),
    "vip_spectral_peak": (_INT, [_P, _I64, _D, ctypes.POINTER(_D), ctypes.POINTER(_D)]),
    "vip_learn_n_params": (_INT, []),
    "vip_learn_init": (_INT, [_P, ctypes.c_uint64]),
    "vip_learn_set_params": (_INT, [_P, _P, _I64]),
    "vip_learn_get_params": (_INT, [_P, _P, _I64]),
    "vip_learn_eval": (_INT, [_P, _P, _P, _P, _INT, _INT, _INT, _P, ctypes.POINTER(_D), _P, _D]),
    "vip_learn_infer": (_INT, [_P, _P, _INT, _INT, _INT, _P]),
    "vip_learn_capture": (_INT, [_P, _INT]),
    "vip_learn_snapshot_count": (_INT, [_P, ctypes.POINTER(_INT)]),
    "vip_learn_clear": (_INT, [_P]),
    "vip_learn_train": (_INT, [_P, _INT, _INT, _INT, _D, ctypes.c_uint64, ctypes.POINTER(_D)]),
}


def load():
    """Load libvip.so (built in-tree); raises if it is missing."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError("libvip.so is not built (run __graft_entry__.build() or "
                           "python paper_1401_6513_amd/build.py); there is no fallback path")
    lib = ctypes.CDLL(LIB_PATH)
    for name, (res, args) in SIGNATURES.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


def default_options(**kw):
    o = VipOptions()
    load().vip_default_options(ctypes.byref(o))
    for k, v in kw.items():
        if k == "period":
            o.period[0], o.period[1] = float(v[0]), float(v[1])
        else:
            setattr(o, k, v)
    return o


def _host(a, dtype):
    return np.ascontiguousarray(np.asarray(a, dtype=dtype))


def _dev(t, n, device):
    """Data pointer of a device vector after checking what the library will assume of it:
    a contiguous float64 tensor on the context's device holding exactly `n` entries.  The
    library checks pointers only for NULL, so a shorter tensor, or one on another device,
    would be read and written out of bounds."""
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda or t.dtype != torch.float64 \
            or not t.is_contiguous():
        raise TypeError("expected a contiguous float64 CUDA tensor")
    if t.device.index != device:
        raise ValueError("tensor is on cuda:%s, the context on cuda:%d" % (t.device.index, device))
    if t.numel() != n:
        raise ValueError("tensor has %d entries, the node set %d" % (t.numel(), n))
    return ctypes.c_void_p(t.data_ptr())


def spectral_peak(signal, dt):
    """(frequency, amplitude) of the periodogram peak of a sampled signal (vip_spectral_peak)."""
    s = _host(signal, np.float64).reshape(-1)
    f, a = _D(), _D()
    rc = load().vip_spectral_peak(s.ctypes.data, len(s), float(dt), ctypes.byref(f), ctypes.byref(a))
    if rc != VIP_OK:
        raise VipError(rc, "vip_spectral_peak", "invalid signal or spacing")
    return f.value, a.value


class Context:
    """One library context bound to a device and a stream."""

    def __init__(self, device=0, stream=None):
        lib = load()
        if stream is None:
            import torch
            stream = torch.cuda.current_stream(device).cuda_stream
        h = ctypes.c_void_p()
        rc = lib.vip_create(ctypes.byref(h), int(device), ctypes.c_void_p(stream))
        if rc != VIP_OK:
            raise VipError(rc, "vip_create", "could not create a context on device %d" % device)
        self._h = h
        self.lib = lib
        self.device = int(device)
        self.n = 0

    def _d(self, t):
        """Device pointer of a node vector of this context (see _dev)."""
        if self.n <= 0:
            raise VipError(-5, "binding", "no node set built on this context")
        return _dev(t, self.n, self.device)

    def close(self):
        if self._h:
            self.lib.vip_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, rc, func, allow=()):
        if rc != VIP_OK and rc not in allow:
            raise VipError(rc, func, self.lib.vip_last_error(self._h).decode())
        return rc

    # ---- C ABI calls ---------------------------------------------------------------
    def vip_build_stencils(self, xy, bnd_idx, bnd_normal, bnd_kind, bnd_value, support_radius, h,
                           basis_order=2, options=None, h_node=None):
        """vip_build_stencils, or vip_build_stencils_adaptive when h_node is given."""
        xy = _host(xy, np.float64).reshape(-1, 2)
        bi = _host(bnd_idx, np.int64).reshape(-1)
        nb = len(bi)
        bn = _host(bnd_normal, np.float64).reshape(nb, 2)
        bk = _host(bnd_kind, np.int32).reshape(nb)
        bv = _host(bnd_value, np.float64).reshape(nb, 2)
        opt = options if options is not None else default_options()
        self.n = 0
        if h_node is None:
            rc = self.lib.vip_build_stencils(self._h, xy.ctypes.data, len(xy), bi.ctypes.data,
                                             bn.ctypes.data, bk.ctypes.data, bv.ctypes.data, nb,
                                             int(basis_order), float(support_radius), float(h),
                                             ctypes.byref(opt))
            self._check(rc, "vip_build_stencils")
        else:
            hn = _host(h_node, np.float64).reshape(-1)
            if len(hn) != len(xy):
                raise ValueError("h_node needs one spacing per node")
            rc = self.lib.vip_build_stencils_adaptive(self._h, xy.ctypes.data, len(xy), bi.ctypes.data,
                                                      bn.ctypes.data, bk.ctypes.data, bv.ctypes.data,
                                                      nb, int(basis_order), float(support_radius),
                                                      float(h), hn.ctypes.data, ctypes.byref(opt))
            self._check(rc, "vip_build_stencils_adaptive")
        self.n = len(xy)

    def vip_set_options(self, options):
        self._check(self.lib.vip_set_options(self._h, ctypes.byref(options)), "vip_set_options")

    def vip_step(self, u, v, p, dt, Re, allow_not_converged=False):
        st = VipStepStats()
        rc = self.lib.vip_step(self._h, self._d(u), self._d(v), self._d(p), float(dt), float(Re),
                               ctypes.byref(st))
        self._check(rc, "vip_step", (VIP_E_NOT_CONVERGED,) if allow_not_converged else ())
        return st.as_dict()

    def vip_reset_history(self):
        self._check(self.lib.vip_reset_history(self._h), "vip_reset_history")

    def vip_poisson_solve(self, rhs, phi, tol, use_x0=False):
        st = VipStepStats()
        rc = self.lib.vip_poisson_solve(self._h, self._d(rhs), self._d(phi), float(tol), int(use_x0),
                                        ctypes.byref(st))
        self._check(rc, "vip_poisson_solve")
        return st.as_dict()

    def vip_get_operator(self, which):
        """(cols [rows, width] int32 with -1 padding, vals [rows, width] float64)."""
        w = OP[which] if isinstance(which, str) else int(which)
        nr, mw, _ = self.vip_operator_shape(w)
        nr, mw = _I64(nr), _I64(mw)
        cols = np.empty((nr.value, max(mw.value, 1)), np.int32)
        vals = np.empty((nr.value, max(mw.value, 1)), np.float64)
        if mw.value == 0:
            cols[:] = -1
            vals[:] = 0.0
            return cols, vals
        self._check(self.lib.vip_get_operator(self._h, w, cols.ctypes.data, vals.ctypes.data),
                    "vip_get_operator")
        return cols, vals

    def vip_operator_shape(self, which):
        """(rows, largest row length, stored entries) of an operator."""
        w = OP[which] if isinstance(which, str) else int(which)
        nr, mw, nz = _I64(), _I64(), _I64()
        self._check(self.lib.vip_operator_shape(self._h, w, ctypes.byref(nr), ctypes.byref(mw),
                                                ctypes.byref(nz)), "vip_operator_shape")
        return nr.value, mw.value, nz.value

    def vip_apply(self, which, x, y):
        w = OP[which] if isinstance(which, str) else int(which)
        self._check(self.lib.vip_apply(self._h, w, self._d(x), self._d(y)), "vip_apply")

    def vip_assemble(self, dt, Re):
        self._check(self.lib.vip_assemble(self._h, float(dt), float(Re)), "vip_assemble")

    def vip_get_geometry(self):
        n = self.n
        vxy = np.empty((n, 4, 2))
        dew = np.empty(n)
        dns = np.empty(n)
        rho = np.empty(n)
        self._check(self.lib.vip_get_geometry(self._h, vxy.ctypes.data, dew.ctypes.data,
                                              dns.ctypes.data, rho.ctypes.data), "vip_get_geometry")
        return vxy, dew, dns, rho

    def vip_convection(self, u, v, nx, ny):
        self._check(self.lib.vip_convection(self._h, self._d(u), self._d(v), self._d(nx), self._d(ny)),
                    "vip_convection")

    def vip_divergence(self, u, v, d):
        self._check(self.lib.vip_divergence(self._h, self._d(u), self._d(v), self._d(d)), "vip_divergence")

    def vip_gradient(self, f, gx, gy):
        self._check(self.lib.vip_gradient(self._h, self._d(f), self._d(gx), self._d(gy)), "vip_gradient")

    def vip_kernel_timing(self, enable=True, reset=False, which=0):
        """(average ms, launches) of kernel `which` (0 pressure SpMV, 1 CNN MFMA layer)."""
        avg = _D()
        cnt = _I64()
        self._check(self.lib.vip_kernel_timing(self._h, int(which), int(enable), int(reset),
                                               ctypes.byref(avg), ctypes.byref(cnt)),
                    "vip_kernel_timing")
        return avg.value, cnt.value

    def vip_canonical_rows(self, described=False):
        """(counts per value set [P64, Hu, Hv, step VIP/node rows, P32, Hu32, Hv32], taps of the
        reference row),
        with the rows of described slices per set as a third item if `described`."""
        counts = np.zeros(7, np.int64)
        desc = np.zeros(7, np.int64)
        taps = _INT()
        self._check(self.lib.vip_canonical_rows(self._h, counts.ctypes.data, desc.ctypes.data,
                                                ctypes.byref(taps)), "vip_canonical_rows")
        if described:
            return counts, taps.value, desc
        return counts, taps.value

    def vip_column_bytes(self):
        """(stored entries of the system matrices, those held as int16 row-relative columns,
        coarse multigrid levels, coarse levels with int16 slices)."""
        a, b = _I64(), _I64()
        d, e = _INT(), _INT()
        self._check(self.lib.vip_column_bytes(self._h, ctypes.byref(a), ctypes.byref(b), ctypes.byref(d),
                                              ctypes.byref(e)), "vip_column_bytes")
        return a.value, b.value, d.value, e.value

    # ---- body forces -------------------------------------------------------------------
    def vip_forces(self, u, v, p, Re, surf_idx):
        """(F_x, F_y) on the body whose surface nodes, in order around it, are surf_idx."""
        s = _host(surf_idx, np.int64).reshape(-1)
        f = np.empty(2)
        self._check(self.lib.vip_forces(self._h, self._d(u), self._d(v), self._d(p), float(Re),
                                        s.ctypes.data, len(s), f.ctypes.data), "vip_forces")
        return f

    def vip_forces_noalloc(self, u, v, p, Re, surf_idx):
        """vip_forces with the library's fixed device scratch (allocates nothing)."""
        s = _host(surf_idx, np.int64).reshape(-1)
        f = np.empty(2)
        self._check(self.lib.vip_forces_noalloc(self._h, self._d(u), self._d(v), self._d(p),
                                                float(Re), s.ctypes.data, len(s), f.ctypes.data),
                    "vip_forces_noalloc")
        return f

    # ---- learned start vector ---------------------------------------------------------
    def vip_learn_n_params(self):
        return int(self.lib.vip_learn_n_params())

    def vip_learn_init(self, seed):
        self._check(self.lib.vip_learn_init(self._h, ctypes.c_uint64(int(seed))), "vip_learn_init")

    def vip_learn_set_params(self, theta):
        th = _host(theta, np.float64).reshape(-1)
        self._check(self.lib.vip_learn_set_params(self._h, th.ctypes.data, len(th)),
                    "vip_learn_set_params")

    def vip_learn_get_params(self):
        th = np.empty(self.vip_learn_n_params())
        self._check(self.lib.vip_learn_get_params(self._h, th.ctypes.data, len(th)),
                    "vip_learn_get_params")
        return th

    def vip_learn_eval(self, x, target=None, mask=None, lr=0.0, want_grad=True):
        """x [B,H,W,3] host images -> (y [B,H,W], loss or None, grad or None)."""
        x = _host(x, np.float64)
        B, H, W, C = x.shape
        if C != 3:
            raise ValueError("input images need 3 channels")
        y = np.empty((B, H, W))
        have_t = target is not None
        t = _host(target, np.float64).reshape(B, H, W) if have_t else None
        m = _host(mask, np.float64).reshape(B, H, W) if have_t else None
        loss = _D()
        g = np.empty(self.vip_learn_n_params()) if (have_t and want_grad) else None
        rc = self.lib.vip_learn_eval(self._h, x.ctypes.data, t.ctypes.data if have_t else None,
                                     m.ctypes.data if have_t else None, B, H, W, y.ctypes.data,
                                     ctypes.byref(loss) if have_t else None,
                                     g.ctypes.data if g is not None else None, float(lr))
        self._check(rc, "vip_learn_eval")
        return y, (loss.value if have_t else None), g

    def vip_learn_infer(self, x):
        """x [B,H,W,3] host images -> y [B,H,W] by the fused inference launch of vip_step."""
        x = _host(x, np.float64)
        B, H, W, C = x.shape
        if C != 3:
            raise ValueError("input images need 3 channels")
        y = np.empty((B, H, W))
        self._check(self.lib.vip_learn_infer(self._h, x.ctypes.data, B, H, W, y.ctypes.data),
                    "vip_learn_infer")
        return y

    def vip_learn_capture(self, max_snapshots):
        self._check(self.lib.vip_learn_capture(self._h, int(max_snapshots)), "vip_learn_capture")

    def vip_learn_snapshot_count(self):
        k = _INT()
        self._check(self.lib.vip_learn_snapshot_count(self._h, ctypes.byref(k)),
                    "vip_learn_snapshot_count")
        return k.value

    def vip_learn_clear(self):
        self._check(self.lib.vip_learn_clear(self._h), "vip_learn_clear")

    def vip_learn_train(self, iters, batch, crop, lr, seed):
        loss = _D()
        self._check(self.lib.vip_learn_train(self._h, int(iters), int(batch), int(crop), float(lr),
                                             ctypes.c_uint64(int(seed)), ctypes.byref(loss)),
                    "vip_learn_train")
        return loss.value

    # ---- convenience ---------------------------------------------------------------
    def build_from_spec(self, spec, **opts):
        """Build from a nodesets.NodeSetSpec (options by keyword)."""
        opt = default_options(period=spec.period, **opts)
        self.vip_build_stencils(spec.xy, spec.bnd_idx, spec.bnd_normal, spec.bnd_kind,
                                spec.bnd_value, spec.rho, spec.h, options=opt,
                                h_node=getattr(spec, "h_node", None))
        self.options = opt
        return opt
