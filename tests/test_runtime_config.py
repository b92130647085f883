"""Runtime configuration on the host: environment overrides of the C library
(spmv_plan_opts_apply_env), the Python layer's weights and autotune-cache
variables, and the Equation 2 arithmetic the benchmark reports (CPU only)."""
import ctypes
import math

import pytest

from oracle import amortize
from paper_1210_2536_amd import capi as C
from paper_1210_2536_amd import workloads


def _opts():
    o = C.spmv_plan_opts()
    assert C.lib().spmv_plan_opts_default(ctypes.byref(o)) == C.SPMV_OK
    return o


@pytest.fixture
def clean_env(monkeypatch):
    for k in ("SPMV_SELECTOR", "SPMV_TAU", "SPMV_LOG", "SPMV_WEIGHTS", "SPMV_AUTOTUNE_CACHE"):
        monkeypatch.delenv(k, raising=False)
    return monkeypatch


def test_env_unset_changes_nothing(clean_env):
    a, b = _opts(), _opts()
    assert C.lib().spmv_plan_opts_apply_env(ctypes.byref(b)) == C.SPMV_OK
    assert bytes(a) == bytes(b)
    assert C.lib().spmv_plan_opts_apply_env(None) == C.SPMV_EINVAL


@pytest.mark.parametrize("value,selector,forced", [
    ("rules", C.SELECT_RULES, -1), ("exhaustive", C.SELECT_EXHAUSTIVE, -1),
    ("csr_adaptive", C.SELECT_FORCED, C.K_CSR_ADAPTIVE), ("dia", C.SELECT_FORCED, C.K_DIA),
    ("bcsr", C.SELECT_FORCED, C.K_BCSR)])
def test_env_selector(clean_env, value, selector, forced):
    clean_env.setenv("SPMV_SELECTOR", value)
    o = _opts()
    C.lib().spmv_plan_opts_apply_env(ctypes.byref(o))
    assert o.selector == selector and o.force_kernel == forced


def test_env_selector_mlp_needs_a_model_and_junk_is_ignored(clean_env, capfd):
    clean_env.setenv("SPMV_SELECTOR", "mlp")
    o = _opts()
    C.lib().spmv_plan_opts_apply_env(ctypes.byref(o))
    assert o.selector == -1                     # no model: left alone
    o.model = ctypes.c_void_p(1)                # any non-NULL handle (never dereferenced)
    C.lib().spmv_plan_opts_apply_env(ctypes.byref(o))
    assert o.selector == C.SELECT_MLP
    clean_env.setenv("SPMV_SELECTOR", "fastest")
    o = _opts()
    C.lib().spmv_plan_opts_apply_env(ctypes.byref(o))
    assert o.selector == -1
    assert "SPMV_SELECTOR=fastest ignored" in capfd.readouterr().err


def test_env_tau_and_log(clean_env, capfd):
    clean_env.setenv("SPMV_TAU", "0.25")
    clean_env.setenv("SPMV_LOG", "1")
    o = _opts()
    C.lib().spmv_plan_opts_apply_env(ctypes.byref(o))
    assert abs(o.confidence_tau - 0.25) < 1e-7 and o.log == 1
    for bad in ("-1", "abc", "0.1x", "inf"):
        clean_env.setenv("SPMV_TAU", bad)
        o = _opts()
        C.lib().spmv_plan_opts_apply_env(ctypes.byref(o))
        assert abs(o.confidence_tau - 0.1) < 1e-7, bad
    clean_env.setenv("SPMV_LOG", "yes")
    o = _opts()
    C.lib().spmv_plan_opts_apply_env(ctypes.byref(o))
    assert o.log == 0
    assert "SPMV_LOG=yes ignored" in capfd.readouterr().err


def test_python_weights_and_cache_variables(clean_env, tmp_path):
    from paper_1210_2536_amd import spmv
    assert spmv.weights_path() == spmv.DEFAULT_WEIGHTS
    clean_env.setenv("SPMV_WEIGHTS", str(tmp_path / "w.json"))
    assert spmv.weights_path() == str(tmp_path / "w.json")
    assert spmv.default_selector() is None       # absent file: no model
    with pytest.raises(ValueError):
        spmv.TuneCache()
    clean_env.setenv("SPMV_AUTOTUNE_CACHE", str(tmp_path / "tune.json"))
    tc = spmv.TuneCache()
    assert tc.path == str(tmp_path / "tune.json") and tc.entries == {}


@pytest.mark.parametrize("plan,plain,tuned", [(19.0, 1.0, 1 / 3), (217.0, 3.0, 0.075),
                                              (5.0, 2.0, 2.5), (0.4, 0.01, 0.002)])
def test_break_even_matches_equation_2(plan, plain, tuned):
    """bench.py's break-even count equals the oracle's Equation 2 reading with
    the plan cost in plain-CSR units and the speedup plain/tuned."""
    got = workloads.break_even_calls(plan, plain, tuned)
    ref = amortize.break_even_calls(plan / plain, plain / tuned)
    assert (math.isinf(got) and math.isinf(ref)) or math.isclose(got, ref, rel_tol=1e-12)
    if plan == 19.0:
        assert math.floor(got) + 1 == 29        # the paper's worked number
