"""CPU checks of the C ABI boundary: the library builds for gfx950, exports every
entry point include/vip.h declares, its structs have the layout the binding
assumes, and the binding refuses to run without the library (no fallback)."""
import ctypes
import os
import re
import subprocess
import tempfile

import pytest

from paper_1401_6513_amd import vip

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "vip.h")


def _ensure_built():
    if not os.path.exists(vip.LIB_PATH):
        from paper_1401_6513_amd import build
        build.build()


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(vip_[a-z_0-9]+)\s*\(", text)))


def test_every_declared_symbol_is_exported():
    _ensure_built()
    names = _declared()
    assert len(names) >= 15
    lib = ctypes.CDLL(vip.LIB_PATH)
    for name in names:
        assert hasattr(lib, name), name
    assert set(names) == set(vip.SIGNATURES), set(names) ^ set(vip.SIGNATURES)


def test_struct_layout_matches_header():
    src = r"""
#include <stddef.h>
#include <stdio.h>
#include "vip.h"
#define F(T, m) printf(#T "." #m " %zu\n", offsetof(T, m));
int main(void) {
  printf("vip_options %zu\nvip_step_stats %zu\n", sizeof(vip_options), sizeof(vip_step_stats));
  F(vip_options, weight) F(vip_options, identity) F(vip_options, precision) F(vip_options, krylov)
  F(vip_options, warmstart) F(vip_options, min_neighbours) F(vip_options, vip_offset)
  F(vip_options, period) F(vip_options, poisson_tol) F(vip_options, helmholtz_tol)
  F(vip_options, inner_tol) F(vip_options, max_iters) F(vip_options, check_every)
  F(vip_options, preconditioner) F(vip_options, learned_precond)
  F(vip_step_stats, poisson_iters) F(vip_step_stats, poisson_outer) F(vip_step_stats, helmholtz_iters)
  F(vip_step_stats, krylov_used) F(vip_step_stats, poisson_residual)
  F(vip_step_stats, helmholtz_residual) F(vip_step_stats, border_lambda)
  F(vip_step_stats, warm_start) F(vip_step_stats, warm_ratio) F(vip_step_stats, warm_alpha) F(vip_step_stats, warm_beta)
  F(vip_step_stats, poisson_fp64_fallback) F(vip_step_stats, learned_pc_passes)
  F(vip_step_stats, learned_pc_ratio) F(vip_step_stats, warm_gamma)
  return 0;
}
"""
    with tempfile.TemporaryDirectory() as d:
        c = os.path.join(d, "t.c")
        exe = os.path.join(d, "t")
        open(c, "w").write(src)
        subprocess.run(["gcc", "-I", os.path.dirname(HEADER), c, "-o", exe], check=True)
        out = subprocess.run([exe], check=True, capture_output=True, text=True).stdout.split("\n")
    got = dict(line.rsplit(" ", 1) for line in out if line)
    assert int(got["vip_options"]) == ctypes.sizeof(vip.VipOptions)
    assert int(got["vip_step_stats"]) == ctypes.sizeof(vip.VipStepStats)
    for T, name in ((vip.VipOptions, "vip_options"), (vip.VipStepStats, "vip_step_stats")):
        for field, _ in T._fields_:
            assert int(got["%s.%s" % (name, field)]) == getattr(T, field).offset, field


def test_binding_refuses_to_run_without_library(monkeypatch):
    monkeypatch.setattr(vip, "LIB_PATH", os.path.join(ROOT, "does_not_exist", "libvip.so"))
    monkeypatch.setattr(vip, "_lib", None)
    with pytest.raises(RuntimeError, match="not built"):
        vip.load()


def test_default_options_through_the_abi():
    _ensure_built()
    o = vip.default_options()
    assert (o.weight, o.identity, o.precision, o.krylov, o.warmstart) == (0, 0, 0, 0, 0)
    assert o.min_neighbours == 12 and o.vip_offset == 0.5
    assert o.poisson_tol == 1e-8 and o.helmholtz_tol == 1e-12 and o.inner_tol == 1e-5


def test_product_code_never_imports_the_oracle():
    pkg = os.path.join(ROOT, "paper_1401_6513_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".h", ".cpp")):
                text = open(os.path.join(dirpath, f)).read()
                assert not re.search(r"^\s*(import|from)\s+oracle\b", text, re.M), f
                assert "oracle/" not in text, f


def test_network_size_matches_the_oracle_layout():
    """The flat parameter vector of the learned start vector has the oracle's layout size
    (a call that touches no device)."""
    _ensure_built()
    from oracle import cnn
    assert vip.load().vip_learn_n_params() == cnn.n_params() == 19681
