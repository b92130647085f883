"""The C-ABI library loads, exports every declared symbol, and the ctypes
structures match the C header's layout (CPU only, no compute calls)."""
import ctypes
import os
import re
import subprocess

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "spmv.h")


def _declared():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(spmv_[a-z_0-9]+)\s*\(", txt)))


def test_library_exports_every_declared_symbol():
    from paper_1210_2536_amd import capi
    L = capi.lib()
    names = _declared()
    assert len(names) >= 20
    for n in names:
        assert hasattr(L, n), n
    assert sorted(capi.exported_symbols()) == names


def test_status_strings_without_gpu():
    from paper_1210_2536_amd import capi
    L = capi.lib()
    assert L.spmv_status_string(capi.SPMV_EINVAL) == b"SPMV_EINVAL"
    assert L.spmv_kernel_name(capi.K_DIA) == b"dia"
    assert L.spmv_mlp_param_count(7) == 64 * 12 + 64 + 64 * 64 + 64 + 7 * 64 + 7
    # argument checks that return before touching a device
    assert L.spmv_plan_create(None, None, None, None) == capi.SPMV_EINVAL
    out = ctypes.c_void_p()
    assert L.spmv_plan_create(None, None, None, ctypes.byref(out)) == capi.SPMV_EINVAL
    assert b"NULL" in L.spmv_last_error()
    csr = capi.spmv_csr(-1, 4, 0, None, None, None, 0)
    assert L.spmv_plan_create(ctypes.byref(csr), None, None, ctypes.byref(out)) == capi.SPMV_EINVAL
    csr = capi.spmv_csr(4, 4, 1 << 31, 1, 1, 1, 1)
    assert L.spmv_plan_create(ctypes.byref(csr), None, None, ctypes.byref(out)) == capi.SPMV_EUNSUPPORTED
    csr = capi.spmv_csr(4, 4, 3, 1, 1, 1, 7)
    assert L.spmv_plan_create(ctypes.byref(csr), None, None, ctypes.byref(out)) == capi.SPMV_EINVAL
    assert L.spmv_plan_destroy(None) == capi.SPMV_OK
    assert L.spmv_selector_set_domain(None, None, None) == capi.SPMV_EINVAL
    assert L.spmv_plan_segment(None, 0, None, None) == capi.SPMV_EINVAL
    assert L.spmv_selector_set_stage(None, None, None, None, None, None, None, 0) == capi.SPMV_EINVAL
    o = capi.spmv_plan_opts()
    assert L.spmv_plan_opts_default(ctypes.byref(o)) == capi.SPMV_OK
    assert o.measure_topk == 3 and o.timing_reps == 5 and abs(o.confidence_tau - 0.1) < 1e-7
    assert o.staged == 1 and abs(o.stage_conf - 0.98) < 1e-7
    assert not o.allocator.alloc and not o.allocator.free
    # an allocator needs both callbacks (checked before any device work)
    o.allocator.alloc = capi.ALLOC_FN(lambda nbytes, ctx: None)
    csr = capi.spmv_csr(4, 4, 3, 1, 1, 1, 1)
    assert L.spmv_plan_create(ctypes.byref(csr), ctypes.byref(o), None,
                              ctypes.byref(out)) == capi.SPMV_EINVAL
    assert b"allocator" in L.spmv_last_error()


PROBE = r"""
#include <stdio.h>
#include <stddef.h>
#include "spmv.h"
#define S(t) printf(#t " %zu\n", sizeof(t));
#define O(t, f) printf(#t "." #f " %zu\n", offsetof(t, f));
int main(void) {
  S(spmv_csr) S(spmv_params) S(spmv_plan_opts) S(spmv_features) S(spmv_plan_info)
  O(spmv_plan_opts, mem_cap_bytes) O(spmv_plan_opts, model) O(spmv_plan_opts, params)
  O(spmv_plan_info, measured_ms) O(spmv_plan_info, features) O(spmv_plan_info, params)
  O(spmv_plan_info, m_pad) O(spmv_plan_info, t_plan_ms) O(spmv_features, aver_rd)
  O(spmv_plan_info, mlp_input) O(spmv_plan_info, rules_kernel) O(spmv_plan_info, out_of_domain) O(spmv_plan_info, t_tune_ms) O(spmv_plan_info, bcsr_blocks) O(spmv_plan_info, n_segments) O(spmv_plan_opts, segments)
  O(spmv_plan_opts, staged) O(spmv_plan_opts, stage_conf) O(spmv_plan_info, feature_stage) O(spmv_plan_info, stage_confidence) O(spmv_plan_info, tune_rejected) O(spmv_plan_info, long_lanes) O(spmv_plan_info, long_rows) O(spmv_params, long_lds) O(spmv_plan_opts, allocator) S(spmv_allocator)
  O(spmv_features, dia_feasible)
  O(spmv_params, panel_direct_max) O(spmv_params, tile_row_min) O(spmv_plan_opts, time_baseline) O(spmv_plan_opts, log)
  O(spmv_plan_info, t_run_ms) O(spmv_plan_info, break_even_calls)
  return 0;
}
"""


def test_ctypes_layout_matches_header(tmp_path):
    from paper_1210_2536_amd import capi
    src = tmp_path / "probe.c"
    src.write_text(PROBE)
    exe = tmp_path / "probe"
    subprocess.run(["gcc", "-std=c11", "-I", os.path.dirname(HEADER), str(src), "-o", str(exe)],
                   check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout
    for line in out.strip().splitlines():
        key, val = line.split()
        val = int(val)
        if "." in key:
            t, f = key.split(".")
            assert getattr(getattr(capi, t), f).offset == val, key
        else:
            assert ctypes.sizeof(getattr(capi, key)) == val, key
