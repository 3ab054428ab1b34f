"""GPU: the level-major forward (levels in groups that fit one XCD's L2,
the grid ordered group by group; used from n = 3 and 2^18 points when the
levels' tables together exceed the L2 and each group fits) gives the same
bits as the all-levels forward, which runs below 2^18 points, and matches
the oracle on sampled points.  Through the C ABI."""
import numpy as np
import pytest

import oracle
from paper_2311_15439_amd import inputs, spx
from test_gpu_encode import _check_fwd

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
DEV = "cuda"
SMALL = (1 << 18) - 1   # the all-levels kernel
LARGE = (1 << 18) + 4097  # level-major, with a partial last block per group

CASES = [
    # name, n, res, log2_T, F, binary16 tables, cell, layout
    ("volume", 3, spx.spx_level_resolutions(16, inputs.VOLUME_3D.growth, 16), 19, 2, True, spx.SPX_SIMPLEX,
     spx.SPX_LAYOUT_HASHED),
    ("volume-grid", 3, spx.spx_level_resolutions(16, inputs.VOLUME_3D.growth, 16), 19, 2, True, spx.SPX_GRID,
     spx.SPX_LAYOUT_HASHED),
    ("sweep4", 4, spx.spx_level_resolutions(16, 1.5, 8), 20, 2, True, spx.SPX_SIMPLEX, spx.SPX_LAYOUT_HASHED),
    ("n5-f32-F4", 5, spx.spx_level_resolutions(8, 1.6, 6), 17, 4, False, spx.SPX_SIMPLEX, spx.SPX_LAYOUT_HASHED),
    ("volume-sized", 3, spx.spx_level_resolutions(16, inputs.VOLUME_3D.growth, 16), 19, 2, True, spx.SPX_SIMPLEX,
     spx.SPX_LAYOUT_SIZED),
]


def _level_major(enc, N, l2=4 << 20):
    """The library's rule: from 3 dimensions and 2^18 points, when every
    level's reachable rows (a dense level's table; a hashed level's 128-byte
    line per box vertex, at most its table) fit one XCD's L2 and all levels
    together do not."""
    lay = spx.spx_table_layout(enc)
    row = enc.n_feat * (2 if enc.table_dtype == spx.SPX_F16 else 4)
    reach = [r * row if d else min(float(e) ** enc.n_dims * 128, r * row)
             for r, e, d in zip(lay["rows"], lay["box_extent"], lay["dense"])]
    return enc.n_dims >= 3 and N >= 1 << 18 and max(reach) <= l2 < sum(reach)


def _run(enc, pts, tab, out_f16):
    out = torch.full((len(pts), enc.n_levels * enc.n_feat), 7.0, device=DEV,
                     dtype=torch.float16 if out_f16 else torch.float32)
    spx.spx_encode_fwd(enc, pts, tab, out)
    torch.cuda.synchronize()
    return out


@pytest.mark.parametrize("out_f16", [True, False])
@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_level_major_same_bits_and_oracle(case, out_f16):
    name, n, res, log2_T, F, f16, cell, layout = case
    enc = spx.Encoding(n, res, log2_T, F, table_dtype=spx.SPX_F16 if f16 else spx.SPX_F32, cell=cell, layout=layout)
    assert _level_major(enc, LARGE) and not _level_major(enc, SMALL)
    if n == 3:  # samples along rays, as in the volume workload
        host_pts = np.concatenate([inputs.ray_points(LARGE // 256, 256, 90), inputs.uniform_points(LARGE % 256, 3, 91)])
    else:
        host_pts = inputs.uniform_points(LARGE, n, 90 + n)
    host_tab = inputs.dense_values(enc.table_shape, 92 + n)
    host_tab = host_tab.astype(np.float16) if f16 else host_tab.astype(np.float32)
    pts = torch.from_numpy(host_pts).to(DEV)
    tab = torch.from_numpy(host_tab).to(DEV)
    big = _run(enc, pts, tab, out_f16)
    small = _run(enc, pts[:SMALL].contiguous(), tab, out_f16)
    assert torch.equal(big[:SMALL], small)
    sel = np.sort(np.concatenate([np.random.default_rng(93).choice(LARGE, 1500, replace=False),
                                  np.arange(LARGE - 300, LARGE)]))
    o = oracle.Encoding(n, list(res), log2_T, n_feat=F, table_dtype=oracle.F16 if f16 else oracle.F32, cell=cell,
                        layout=oracle.SIZED if layout == spx.SPX_LAYOUT_SIZED else oracle.HASHED)
    got = big.cpu().numpy().astype(np.float64)[sel]
    _check_fwd(got, oracle.encode_fwd(o, host_pts[sel], host_tab), oracle.encode_fwd_absmag(o, host_pts[sel], host_tab),
               out_f16)
