"""GPU: the library's kernel trace records every kernel it launches, or with
a name filter only the kernels of that name, with their durations."""
import numpy as np
import pytest

from paper_2311_15439_amd import inputs, spx

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _adjoint_calls(reps):
    res = spx.spx_level_resolutions(16, 1.5, 8)
    enc = spx.Encoding(2, res, 16)
    N = 5000
    pts = torch.from_numpy(inputs.uniform_points(N, 2, 3)).cuda()
    d_out = torch.ones((N, enc.n_levels * enc.n_feat), dtype=torch.float32, device="cuda")
    grad = torch.zeros((enc.n_levels, 1 << 16, enc.n_feat), dtype=torch.float32, device="cuda")
    ws = torch.empty(spx.spx_encode_bwd_workspace(enc, N), dtype=torch.uint8, device="cuda")

    def run():
        for _ in range(reps):
            spx.spx_encode_bwd(enc, pts, d_out, grad, ws)
    return run


def test_trace_all_kernels():
    run = _adjoint_calls(2)
    run()
    tr = spx.Trace(capacity=64)
    with tr:
        run()
    res = tr.results()
    names = [n for n, _, _ in res]
    assert names.count("bin_accum") == 2 and "bin_scatter" in names and "bin_count" in names
    assert all(ms > 0 and nb > 0 for _, nb, ms in res)


def test_trace_one_kernel():
    run = _adjoint_calls(3)
    run()
    tr = spx.Trace(capacity=64, only="bin_accum")
    with tr:
        run()
    res = tr.results()
    assert [n for n, _, _ in res] == ["bin_accum"] * 3
    assert all(ms > 0 and nb > 0 for _, nb, ms in res)
    # a filter that matches nothing records nothing, and the trace still works after it
    tr2 = spx.Trace(capacity=8, only="no_such_kernel")
    with tr2:
        run()
    assert tr2.results() == []
