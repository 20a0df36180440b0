"""C ABI checks that need no GPU: every declared symbol is exported, struct
layouts agree between include/bsi.h and the Python binding, and calls without
a device or handle fail cleanly."""
import ctypes as C
import os
import re
import subprocess
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "bsi.h")


@pytest.fixture(scope="module")
def native():
    from paper_2604_22048_amd import _native
    if not os.path.exists(_native.LIB_PATH):
        from paper_2604_22048_amd import build
        build.build()
    return _native


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(bsi_[a-z_]+)\s*\(", src)))


def test_every_declared_symbol_is_exported(native):
    names = declared_functions()
    assert len(names) >= 10
    lib = native.load()
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(native.SIGNATURES), set(names) ^ set(native.SIGNATURES)


def test_struct_layouts_match_header(native):
    prog = r"""
#include <stdio.h>
#include <stddef.h>
#include "bsi.h"
#define F(T, m) printf(#T "." #m " %zu\n", offsetof(T, m));
int main(void) {
  printf("bsi_batch %zu\n", sizeof(bsi_batch));
  printf("bsi_interim %zu\n", sizeof(bsi_interim));
  printf("bsi_hmc_cfg %zu\n", sizeof(bsi_hmc_cfg));
  printf("bsi_true_prior %zu\n", sizeof(bsi_true_prior));
  printf("bsi_shear_hmc_cfg %zu\n", sizeof(bsi_shear_hmc_cfg));
  printf("bsi_slots_cfg %zu\n", sizeof(bsi_slots_cfg));
  printf("bsi_request %zu\n", sizeof(bsi_request));
  printf("bsi_slots_info %zu\n", sizeof(bsi_slots_info));
  printf("bsi_reserve_cfg %zu\n", sizeof(bsi_reserve_cfg));
  F(bsi_batch, psf_fwhm) F(bsi_batch, pixel_scale) F(bsi_batch, profile) F(bsi_batch, spergel_nu)
  F(bsi_hmc_cfg, step_size) F(bsi_hmc_cfg, form) F(bsi_hmc_cfg, seed) F(bsi_hmc_cfg, uid_base)
  F(bsi_hmc_cfg, trace) F(bsi_hmc_cfg, waves_per_chain) F(bsi_hmc_cfg, sampler) F(bsi_hmc_cfg, max_tree_depth)
  F(bsi_true_prior, mu_ln_f) F(bsi_true_prior, sigma_ln_f)
  F(bsi_shear_hmc_cfg, jitter) F(bsi_shear_hmc_cfg, inv_mass) F(bsi_shear_hmc_cfg, seed)
  F(bsi_shear_hmc_cfg, use_graph) F(bsi_shear_hmc_cfg, trace)
  F(bsi_slots_cfg, hbm_budget) F(bsi_slots_cfg, hmc) F(bsi_slots_cfg, interim)
  F(bsi_slots_cfg, pixel_scale) F(bsi_slots_cfg, profile) F(bsi_slots_cfg, spergel_nu) F(bsi_slots_cfg, pace)
  F(bsi_slots_cfg, ess_target) F(bsi_slots_cfg, ess_every)
  F(bsi_request, stamp) F(bsi_request, psf_fwhm) F(bsi_request, ref_y) F(bsi_request, init)
  F(bsi_slots_info, budget) F(bsi_slots_info, arena_largest_free)
  F(bsi_reserve_cfg, max_n) F(bsi_reserve_cfg, max_shear_gal) F(bsi_reserve_cfg, max_points)
  F(bsi_reserve_cfg, max_boot)
  return 0;
}
"""
    with tempfile.TemporaryDirectory() as d:
        c = os.path.join(d, "layout.c")
        exe = os.path.join(d, "layout")
        open(c, "w").write(prog)
        subprocess.check_call(["gcc", "-I", os.path.dirname(HEADER), c, "-o", exe])
        out = dict(line.rsplit(" ", 1) for line in subprocess.check_output([exe], text=True).splitlines())
    assert int(out["bsi_reserve_cfg"]) == C.sizeof(native.ReserveCfg)
    for m in ("max_n", "max_shear_gal", "max_points", "max_boot"):
        assert int(out[f"bsi_reserve_cfg.{m}"]) == getattr(native.ReserveCfg, m).offset, m
    assert int(out["bsi_batch"]) == C.sizeof(native.Batch)
    assert int(out["bsi_interim"]) == C.sizeof(native.Interim)
    assert int(out["bsi_hmc_cfg"]) == C.sizeof(native.HmcCfg)
    assert int(out["bsi_true_prior"]) == C.sizeof(native.TruePrior)
    assert int(out["bsi_shear_hmc_cfg"]) == C.sizeof(native.ShearHmcCfg)
    assert int(out["bsi_slots_cfg"]) == C.sizeof(native.SlotsCfg)
    assert int(out["bsi_request"]) == C.sizeof(native.Request)
    assert int(out["bsi_slots_info"]) == C.sizeof(native.SlotsInfo)
    for key, val in out.items():
        if "." in key:
            t, m = key.split(".")
            cls = {"bsi_batch": native.Batch, "bsi_hmc_cfg": native.HmcCfg,
                   "bsi_true_prior": native.TruePrior, "bsi_shear_hmc_cfg": native.ShearHmcCfg,
                   "bsi_slots_cfg": native.SlotsCfg, "bsi_request": native.Request,
                   "bsi_slots_info": native.SlotsInfo, "bsi_reserve_cfg": native.ReserveCfg}[t]
            assert getattr(cls, m).offset == int(val), key


def test_no_device_and_null_handle_paths(native):
    lib = native.load()
    n = C.c_int32(-1)
    assert lib.bsi_device_count(C.byref(n)) == 0 and n.value >= 0
    assert lib.bsi_version() == 4
    assert lib.bsi_create(None, 0, None) == -1
    if n.value == 0:
        h = C.c_void_p()
        assert lib.bsi_create(C.byref(h), 0, None) == -5
        assert b"device" in lib.bsi_last_error(None)
        assert lib.bsi_create(C.byref(h), 0, b"/nonexistent/cache") == -5   # device checked first
    b = native.Batch()
    assert lib.bsi_render_stamps(None, C.byref(b), None, None, None) == -1
    assert lib.bsi_loglik_grad(None, C.byref(b), None, None, None, None, None, 0, None) == -1
    assert lib.bsi_ess(None, 1, 1, 10, 1, None, None, None, None, None) == -1
    r = native.ReserveCfg(max_stamps=10, max_n=53, max_chains=4)
    assert lib.bsi_reserve(None, C.byref(r)) == -1
    assert lib.bsi_shear_hmc(None, 1, 1, None, None, None, None, None, None, None, None, None,
                             None, None) == -1
    assert lib.bsi_slots_create(None, None, None, None) == -1
    assert lib.bsi_set_plan(None, 53, 6) == -1
    assert lib.bsi_autotune(None, 0, None, 4, None, None) == -1
    assert lib.bsi_slots_advance(None, 1) == -1
    assert lib.bsi_slots_get_info(None, None) == -1
    assert lib.bsi_slots_poll(None, None) == -1
    lib.bsi_slots_destroy(None)
    lib.bsi_destroy(None)
    assert lib.bsi_device_count(None) == -1


def test_binding_fails_loudly_without_library(tmp_path, monkeypatch):
    from paper_2604_22048_amd import _native
    monkeypatch.setattr(_native, "LIB_PATH", str(tmp_path / "missing.so"))
    monkeypatch.setattr(_native, "_lib", None)
    with pytest.raises(RuntimeError, match="no CPU fallback"):
        _native.load()
