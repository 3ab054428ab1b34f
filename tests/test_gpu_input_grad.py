"""GPU: gradient of the encoding with respect to the input points, against
the oracle, through the C ABI.

Bound from the binary32 steps: per level a row difference (one rounding
against |t_{k+1}| + |t_k|), the product with the output gradient and the
sum over F features, the skew chain (a sum over n axes, two products and a
sum), and the sum over L levels; the grid adds up to 2n roundings for its
weight products and V terms per axis.  So
    |gpu - oracle| <= 2 (F + 2n + V + L + 8) u * mag
where mag is the oracle's same sum over absolute values.
"""
import numpy as np
import pytest

import oracle
from paper_2311_15439_amd import inputs, spx

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
U = 2.0 ** -24

CASES = [
    # n, res, log2_T, F, tables f16, d_out f16, cell
    (1, [9, 100], 10, 2, False, False, spx.SPX_SIMPLEX),
    (2, [16, 24, 36, 54], 14, 2, True, False, spx.SPX_SIMPLEX),
    (2, [16, 24, 36, 54], 14, 2, True, False, spx.SPX_GRID),
    (3, [16, 64, 512, 2048], 19, 2, True, True, spx.SPX_SIMPLEX),
    (3, [16, 64, 512, 2048], 19, 2, True, True, spx.SPX_GRID),
    (4, [10, 80], 16, 4, False, False, spx.SPX_SIMPLEX),
    (5, [16, 90], 16, 8, False, True, spx.SPX_SIMPLEX),
    (6, [7, 40], 20, 1, True, False, spx.SPX_SIMPLEX),
    (6, [7, 40], 20, 2, True, False, spx.SPX_GRID),
]


@pytest.mark.parametrize("case", CASES, ids=lambda c: f"n{c[0]}F{c[3]}{'h' if c[4] else 'f'}{'h' if c[5] else 'f'}c{c[6]}")
def test_input_grad_parity(case):
    n, res, log2_T, F, tf16, gf16, cell = case
    g = spx.Encoding(n, res, log2_T, n_feat=F, table_dtype=spx.SPX_F16 if tf16 else spx.SPX_F32, cell=cell)
    o = oracle.Encoding(n, res, log2_T, n_feat=F, table_dtype=oracle.F16 if tf16 else oracle.F32, cell=cell)
    rng = np.random.default_rng(3)
    pts = np.concatenate([inputs.uniform_points(4000, n, 80 + n), -0.3 + 1.6 * inputs.uniform_points(50, n, 81),
                          np.full((1, n), 0.5, np.float32), np.zeros((1, n), np.float32)])
    tab = inputs.tables(len(res), 1 << log2_T, F, 1.0, 82 + n, tf16)
    d = inputs.gradients(len(pts), len(res) * F, 83 + n)
    if gf16:
        d = d.astype(np.float16)
    out = torch.empty((len(pts), n), dtype=torch.float32, device="cuda")
    spx.spx_encode_input_grad(g, torch.from_numpy(pts).cuda(), torch.from_numpy(tab).cuda(),
                              torch.from_numpy(d).cuda(), out)
    torch.cuda.synchronize()
    got = out.cpu().numpy().astype(np.float64)
    ref, mag = oracle.encode_input_grad(o, pts, tab, d.astype(np.float64), with_mag=True)
    V = (1 << n) if cell == spx.SPX_GRID else n + 1
    tol = 2 * (F + 2 * n + V + len(res) + 8) * U * mag + 1e-30
    err = np.abs(got - ref)
    worst = np.unravel_index(np.argmax(err / tol), err.shape)
    assert (err <= tol).all(), f"worst err/tol {np.max(err / tol):.3f} at {worst}: {got[worst]} vs {ref[worst]}"


def test_input_grad_full_image_workload_sampled():
    """The image workload's shape (2^20 points, 16 levels, 2^22-entry
    binary16 tables), compared with the oracle on a sample of points."""
    w = inputs.IMAGE_2D
    res = oracle.level_resolutions(w.n_min, w.growth, w.n_levels)
    g = spx.Encoding(2, list(res), w.log2_T, 2, table_dtype=spx.SPX_F16)
    o = oracle.Encoding(2, list(res), w.log2_T, 2, table_dtype=oracle.F16)
    pts = inputs.pixel_points(w.n_points, w.seed_points)
    tab = inputs.tables(w.n_levels, 1 << w.log2_T, 2, 0.5, w.seed_tables, True)
    d = inputs.gradients(len(pts), 32, 84)
    out = torch.empty((len(pts), 2), dtype=torch.float32, device="cuda")
    spx.spx_encode_input_grad(g, torch.from_numpy(pts).cuda(), torch.from_numpy(tab).cuda(),
                              torch.from_numpy(d).cuda(), out)
    torch.cuda.synchronize()
    idx = np.random.default_rng(85).choice(len(pts), 4000, replace=False)
    ref, mag = oracle.encode_input_grad(o, pts[idx], tab, d[idx].astype(np.float64), with_mag=True)
    got = out.cpu().numpy()[idx].astype(np.float64)
    tol = 2 * (2 + 4 + 3 + 16 + 8) * U * mag + 1e-30
    assert (np.abs(got - ref) <= tol).all()
