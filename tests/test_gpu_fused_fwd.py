"""GPU: the fused encoding + network training forward equals the separate
kernels bit for bit (features and outputs), through the C ABI."""
import numpy as np
import pytest

from paper_2311_15439_amd import inputs, spx

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("n,cell,d_out", [(2, spx.SPX_SIMPLEX, 3), (3, spx.SPX_SIMPLEX, 4), (2, spx.SPX_GRID, 1),
                                          (3, spx.SPX_GRID, 16)])
def test_fused_forward_equals_separate(n, cell, d_out):
    res = spx.spx_level_resolutions(16, 1.5, 16)
    enc = spx.Encoding(n, res, 18, 2, table_dtype=spx.SPX_F16, cell=cell)
    mlp = spx.make_mlp(32, 64, d_out)
    tab = torch.from_numpy(inputs.tables(16, 1 << 18, 2, 0.5, 60 + n, True)).cuda()
    W = [torch.from_numpy(w).cuda() for w in inputs.mlp_weights(32, 64, d_out, 61)]
    for N in [1, 15, 16, 17, 1000, 65539, 1 << 20]:
        pts = torch.from_numpy(np.concatenate([inputs.uniform_points(N - 1, n, 62 + N),
                                               np.full((1, n), 1.0, np.float32)])).cuda()
        f_sep = torch.empty((N, 32), dtype=torch.float16, device="cuda")
        y_sep = torch.empty((N, d_out), dtype=torch.float32, device="cuda")
        spx.spx_encode_fwd(enc, pts, tab, f_sep)
        spx.spx_mlp_fwd(mlp, f_sep, *W, y_sep)
        f_fus = torch.full((N, 32), 7.0, dtype=torch.float16, device="cuda")
        y_fus = torch.full((N, d_out), 7.0, dtype=torch.float32, device="cuda")
        spx.spx_encode_mlp_fwd(enc, mlp, pts, tab, *W, y_fus, feats=f_fus)
        y_only = torch.full((N, d_out), 7.0, dtype=torch.float32, device="cuda")
        spx.spx_encode_mlp_fwd(enc, mlp, pts, tab, *W, y_only)
        torch.cuda.synchronize()
        assert torch.equal(f_fus, f_sep), N
        assert torch.equal(y_fus, y_sep), N
        assert torch.equal(y_only, y_sep), N


def test_fused_forward_rejects_other_shapes():
    enc = spx.Encoding(2, [16] * 8, 14, 2, table_dtype=spx.SPX_F16)
    mlp = spx.make_mlp(16, 64, 3)
    tab = torch.zeros(enc.table_shape, dtype=torch.float16, device="cuda")
    W = [torch.zeros(s, dtype=torch.float16, device="cuda") for s in [(64, 16), (64, 64), (3, 64)]]
    with pytest.raises(spx.SpxError):
        spx.spx_encode_mlp_fwd(enc, mlp, torch.zeros((4, 2), device="cuda"), tab, *W,
                               torch.zeros((4, 3), device="cuda"))
