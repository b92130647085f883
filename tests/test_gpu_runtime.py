"""Runtime reporting on the GPU: Equation 2 timings in the plan report, the
one-line plan log (opts.log and SPMV_LOG), an environment-forced kernel, and
the read-dominant bandwidth probe's arithmetic."""
import math

import numpy as np
import pytest

from paper_1210_2536_amd import synth as S

from gpu_util import assert_parity, dev, note, vec

pytestmark = pytest.mark.gpu


def test_time_baseline_reports_equation_2():
    from paper_1210_2536_amd.spmv import Plan
    A = S.stencil_7pt(64)
    rp, col, val = dev(A, np.float64)
    note("[runtime] time_baseline on lap7_64^3")
    p = Plan(rp, col, val, n=A.n, selector="rules", time_baseline=True)
    I = p.info()
    assert I["t_run_ms"] > 0 and I["t_plain_ms"] > 0
    if I["t_plain_ms"] > I["t_run_ms"]:
        want = I["t_plan_ms"] / (I["t_plain_ms"] - I["t_run_ms"])
        assert math.isclose(I["break_even_calls"], want, rel_tol=1e-12)
    else:
        assert math.isinf(I["break_even_calls"])
    q = Plan(rp, col, val, n=A.n, selector="rules")
    assert q.info()["t_run_ms"] == -1 and q.info()["break_even_calls"] == -1
    x = S.uniform_vector(A.n, 3)
    assert_parity(p.run(vec(x, np.float64)).cpu().numpy(), A, x, np.float64)


def test_plan_log_line_and_env(capfd, monkeypatch):
    from paper_1210_2536_amd.spmv import Plan
    A = S.stencil_5pt(64)
    rp, col, val = dev(A, np.float32)
    note("[runtime] plan log")
    capfd.readouterr()
    Plan(rp, col, val, n=A.n, selector="ell", log=True, time_baseline=True)
    err = capfd.readouterr().err
    assert "[spmv] plan m=4096 n=4096 nnz=20224 f32 kernel=ell selector=forced" in err
    assert "break_even=" in err
    monkeypatch.setenv("SPMV_LOG", "1")
    monkeypatch.setenv("SPMV_SELECTOR", "coo")
    p = Plan(rp, col, val, n=A.n, selector="rules")
    err = capfd.readouterr().err
    assert p.info()["kernel_name"] == "coo" and "kernel=coo selector=forced" in err
    x = S.uniform_vector(A.n, 4)
    assert_parity(p.run(vec(x, np.float32)).cpu().numpy(), A, x, np.float32)


def test_stream_read_probe_sums_every_word():
    import torch
    from paper_1210_2536_amd import capi as C
    from paper_1210_2536_amd.spmv import stream_read
    g = torch.Generator().manual_seed(5)
    for n16 in (1, 1000, 3 * 524288 + 17):       # 16-byte pieces, below and above the grid
        note(f"[runtime] stream_read {n16} pieces")
        src = torch.randint(0, 2 ** 31, (n16 * 4,), generator=g, dtype=torch.int64)
        h = src.numpy().astype(np.uint32).reshape(-1, 4)
        d = torch.from_numpy(h.view(np.int32).reshape(-1)).cuda()
        out = stream_read(d).cpu().numpy().view(np.uint32).reshape(-1, 4)
        assert out.shape[0] * 16 == C.lib().spmv_stream_read_out_bytes()
        want = h.astype(np.uint64).sum(axis=0) % (1 << 32)
        got = out.astype(np.uint64).sum(axis=0) % (1 << 32)
        assert np.array_equal(got, want)
