"""vip_forces_noalloc (fixed device scratch, no allocation) against vip_forces, through the
C ABI: two calls in a row, the second on a smaller surface, each compared with the allocating
entry point; sizes beyond the fixed scratch are rejected with the limit in the message."""
import ctypes

import numpy as np
import pytest

from paper_1401_6513_amd import nodesets as ns

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _vip():
    from paper_1401_6513_amd import vip
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return vip


def _dev(a):
    return torch.tensor(np.asarray(a, dtype=np.float64), device="cuda")


def _abi_forces(lib, ctx, name, u, v, p, re, surf):
    s = np.ascontiguousarray(surf, dtype=np.int64)
    out = np.full(2, np.nan)
    rc = getattr(lib, name)(ctx._h, ctypes.c_void_p(u.data_ptr()), ctypes.c_void_p(v.data_ptr()),
                            ctypes.c_void_p(p.data_ptr()), ctypes.c_double(re),
                            ctypes.c_void_p(s.ctypes.data), ctypes.c_int64(len(s)),
                            ctypes.c_void_p(out.ctypes.data))
    return rc, out


def test_noalloc_forces_match_the_allocating_entry_point():
    vip = _vip()
    lib = vip.load()
    specs = [ns.cylinder_channel(1.0 / 16, box=(-2.0, 4.0, -2.0, 2.0), n_surface=96),
             ns.cylinder_channel(0.125, box=(-2.0, 3.0, -2.0, 2.0), shape=(0.05, 12), n_surface=24)]
    ctxs, states, refs = [], [], []
    try:
        for k, spec in enumerate(specs):
            ctx = vip.Context(0)
            ctxs.append(ctx)
            ctx.build_from_spec(spec)
            st = [_dev(ns.random_field(spec.n, seed=50 + 3 * k + j)) for j in range(3)]
            states.append(st)
            rc, f = _abi_forces(lib, ctx, "vip_forces", *st, 80.0, spec.surface)
            assert rc == 0
            refs.append(f)
        # two no-allocation calls in a row, the second on the smaller surface
        for ctx, spec, st, ref in zip(ctxs, specs, states, refs):
            rc, f = _abi_forces(lib, ctx, "vip_forces_noalloc", *st, 80.0, spec.surface)
            assert rc == 0
            print("surface %d: alloc %r noalloc %r" % (len(spec.surface), ref, f))
            # same kernels, same order of summation: the same bits
            assert np.array_equal(ref, f)
    finally:
        for ctx in ctxs:
            ctx.close()


def test_noalloc_rejects_sizes_beyond_its_scratch():
    vip = _vip()
    lib = vip.load()
    spec = ns.cylinder_channel(0.125, box=(-2.0, 3.0, -2.0, 2.0), n_surface=24)
    ctx = vip.Context(0)
    try:
        ctx.build_from_spec(spec)
        u = _dev(np.zeros(spec.n))
        big = np.resize(spec.surface, 43681)
        rc, _ = _abi_forces(lib, ctx, "vip_forces_noalloc", u, u, u, 80.0, big)
        assert rc == -1
        msg = lib.vip_last_error(ctx._h).decode()
        assert "43680" in msg, msg
        # the limit itself is accepted (a repeated chain is still a valid list of boundary nodes)
        rc, f = _abi_forces(lib, ctx, "vip_forces_noalloc", u, u, u, 80.0, np.resize(spec.surface, 43680))
        assert rc == 0 and np.all(np.isfinite(f))
    finally:
        ctx.close()
