"""GPU: the gather twin (the forward's measurement reference) gathers the
rows it documents -- the cell corner of the oracle's lookup, then one step
along each axis in index order (all 2^n corners for the grid) -- and sums
them without weights."""
import numpy as np
import pytest

import oracle
from paper_2311_15439_amd import inputs, spx

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _expected(oe, pts, tab16, cell):
    dbg = oracle.encode_debug(oe, pts)
    corner = dbg["verts"][:, :, 0, :].astype(np.int64)  # [N, L, n]
    n, L = oe.n_dims, oe.n_levels
    P = np.array(oracle.hash_primes()[:n], dtype=np.uint64)
    mask = np.uint64((1 << oe.log2_T) - 1)
    if cell == spx.SPX_SIMPLEX:
        steps = [np.array([1 if i < k else 0 for i in range(n)]) for k in range(n + 1)]
    else:
        steps = [np.array([(c >> i) & 1 for i in range(n)]) for c in range(1 << n)]
    acc = np.zeros((len(pts), L, 2), np.float32)
    lv = np.arange(L)[None, :]
    for s in steps:
        v = (corner + s).astype(np.uint64) & np.uint64(0xFFFFFFFF)
        h = np.zeros(v.shape[:2], np.uint64)
        for i in range(n):
            h ^= (v[..., i] * P[i]) & np.uint64(0xFFFFFFFF)
        rows = tab16[lv, (h & mask).astype(np.int64)].astype(np.float32)
        acc = acc + rows  # binary32, vertex order
    return acc.reshape(len(pts), L * 2).astype(np.float16)


@pytest.mark.parametrize("n", [2, 3, 4])
@pytest.mark.parametrize("cell", [spx.SPX_SIMPLEX, spx.SPX_GRID])
def test_twin_rows(n, cell):
    res = spx.spx_level_resolutions(16, 1.5, 6)
    enc = spx.Encoding(n, res, 16, 2, table_dtype=spx.SPX_F16, cell=cell)
    oe = oracle.Encoding(n, list(res), 16, 2, table_dtype=oracle.F16, cell=cell)
    N = 3000
    pts = inputs.uniform_points(N, n, 40 + n)
    tab = inputs.tables(6, 1 << 16, 2, 1.0, 41, True)
    out = torch.empty((N, 12), dtype=torch.float16, device="cuda")
    spx.spx_encode_gather_twin(enc, torch.from_numpy(pts).cuda(), torch.from_numpy(tab).cuda(), out)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(out.cpu().numpy(), _expected(oe, pts, tab, cell))


def test_twin_rejects_other_layouts():
    enc = spx.Encoding(2, [16, 24], 14, 4, table_dtype=spx.SPX_F16)
    tab = torch.zeros(enc.table_shape, dtype=torch.float16, device="cuda")
    out = torch.empty((8, 8), dtype=torch.float16, device="cuda")
    with pytest.raises(RuntimeError):
        spx.spx_encode_gather_twin(enc, torch.zeros((8, 2), device="cuda"), tab, out)
