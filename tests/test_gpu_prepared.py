"""GPU parity of the adjoint split in two: spx_encode_bwd_prepare (the part
that depends only on the points) on a second stream, joined by an event,
then spx_encode_bwd_prepared / spx_encode_bwd_adam_prepared.  Against the
CPU oracle with the adjoint's per-slot bound (m + n + 2) * 2^-24 * sum |w d|,
on inputs that take each shape of the count pass and scatter: many buckets
per level, few buckets with coherent ray samples, densely stored levels,
and two level groups (only the first is prepared)."""
import numpy as np
import pytest

import oracle
from paper_2311_15439_amd import inputs, spx
from test_gpu_encode import adam_problem

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

DEV = "cuda"

CASES = [
    # (name, n, res, log2_T, cell, layout, points)
    ("many-buckets", 2, [16, 64, 256, 1024, 4096], 18, spx.SPX_SIMPLEX, spx.SPX_LAYOUT_HASHED, "uniform"),
    ("rays-few-buckets", 3, [4, 16, 60, 200, 700], 14, spx.SPX_SIMPLEX, spx.SPX_LAYOUT_HASHED, "rays"),
    ("rays-grid", 3, [4, 16, 60, 200, 700], 14, spx.SPX_GRID, spx.SPX_LAYOUT_HASHED, "rays"),
    ("dense-levels", 2, [70, 90, 300], 16, spx.SPX_SIMPLEX, spx.SPX_LAYOUT_SIZED, "uniform"),
    # 2^18 points x 64 corners: two level groups
    ("two-groups", 6, [3, 5, 9, 12] * 4, 14, spx.SPX_GRID, spx.SPX_LAYOUT_HASHED, "large"),
]


def _pair(n, res, log2_T, cell, layout):
    g = spx.Encoding(n, list(res), log2_T, n_feat=2, table_dtype=spx.SPX_F32, cell=cell, layout=layout)
    o = oracle.Encoding(n, list(res), log2_T, n_feat=2, table_dtype=oracle.F32, cell=cell,
                        layout=oracle.SIZED if layout == spx.SPX_LAYOUT_SIZED else oracle.HASHED)
    return g, o


def _points(kind, n):
    if kind == "rays":
        return inputs.ray_points(64, 256, 80 + n)
    if kind == "large":
        return inputs.uniform_points((1 << 18) + 3, n, 81)
    return np.concatenate([inputs.uniform_points(20001, n, 82), -0.5 + 2.0 * inputs.uniform_points(97, n, 83)])


def _prepare_on_side_stream(enc, p, ws):
    """The counting pass on a second stream, beside whatever the caller's
    stream runs, with an event that the caller's stream then waits on."""
    main = torch.cuda.current_stream()
    side = torch.cuda.Stream()
    start, done = torch.cuda.Event(), torch.cuda.Event()
    start.record(main)
    side.wait_event(start)
    spx.spx_encode_bwd_prepare(enc, p, ws, stream=side)
    done.record(side)
    main.wait_event(done)


@pytest.mark.parametrize("case", CASES, ids=lambda c: c[0])
def test_prepared_adjoint_matches_the_oracle(case):
    _, n, res, log2_T, cell, layout, kind = case
    g, o = _pair(n, res, log2_T, cell, layout)
    pts = _points(kind, n)
    d = inputs.gradients(len(pts), len(res) * 2, 84 + n)
    p, dd = torch.from_numpy(pts).to(DEV), torch.from_numpy(d).to(DEV)
    ws = torch.empty(spx.spx_encode_bwd_workspace(g, len(pts)), dtype=torch.uint8, device=DEV)
    ref, mag, cnt = oracle.encode_bwd(o, pts, d.astype(np.float64), with_stats=True)
    tol = (cnt + n + 2) * 2.0 ** -24 * mag + 1e-30
    # a forward on the caller's stream while the counting runs beside it
    tab = torch.zeros(g.table_shape, dtype=torch.float32, device=DEV)
    feats = torch.empty((len(pts), len(res) * 2), dtype=torch.float32, device=DEV)
    for rep in range(2):  # the workspace is reused: the second call prepares over the first's contents
        grad = torch.zeros(g.table_shape, dtype=torch.float32, device=DEV)
        _prepare_on_side_stream(g, p, ws)
        spx.spx_encode_fwd(g, p, tab, feats)
        spx.spx_encode_bwd_prepared(g, p, dd, grad, ws)
        torch.cuda.synchronize()
        got = grad.cpu().numpy().astype(np.float64)
        err = np.abs(got - ref)
        assert (err <= tol).all(), f"rep {rep}: worst {err.max()} ; {int((err > tol).sum())} slots out of tolerance"
        assert np.all(got[cnt == 0] == 0)


def test_prepared_adjoint_with_adam_matches_the_oracle():
    n, res, log2_T = 3, [4, 16, 64, 200], 13
    g, o = _pair(n, res, log2_T, spx.SPX_SIMPLEX, spx.SPX_LAYOUT_HASHED)
    pts = inputs.ray_points(96, 256, 85)
    d = inputs.gradients(len(pts), len(res) * 2, 86) * 1e-3
    shape = g.table_shape
    rng = np.random.default_rng(87)
    p0 = (rng.normal(size=shape) * 1e-2).astype(np.float32)
    m0 = (rng.normal(size=shape) * 1e-3).astype(np.float32)
    v0 = (rng.random(shape) * 1e-5 + 1e-7).astype(np.float32)
    f32 = lambda x: float(np.float32(x))
    lr, b1, b2, eps, step = f32(1e-2), f32(0.9), f32(0.99), f32(1e-15), 3
    tp, tm, tv = (torch.from_numpy(a.copy()).to(DEV) for a in (p0, m0, v0))
    th = torch.empty(shape, dtype=torch.float16, device=DEV)
    p = torch.from_numpy(pts).to(DEV)
    ws = torch.empty(spx.spx_encode_bwd_workspace(g, len(pts)), dtype=torch.uint8, device=DEV)
    _prepare_on_side_stream(g, p, ws)
    spx.spx_encode_bwd_adam_prepared(g, p, torch.from_numpy(d).to(DEV), tp, tm, tv, th, lr=lr, beta1=b1, beta2=b2,
                                     eps=eps, step=step, workspace=ws)
    torch.cuda.synchronize()
    gref, gmag, cnt = oracle.encode_bwd(o, pts, d.astype(np.float64), with_stats=True)
    tolg = (cnt + n + 2) * 2.0 ** -24 * gmag + 1e-30
    prob = adam_problem(p0, m0, v0, gref, tolg, tp, tm, tv, lr, b1, b2, eps, step)
    assert prob is None, prob
    np.testing.assert_array_equal(th.cpu().numpy().view(np.uint16).ravel(),
                                  oracle.cast_f32_f16(tp.cpu().numpy().ravel()))


def test_prepare_rejects_bad_arguments():
    g, _ = _pair(2, [16, 64], 14, spx.SPX_SIMPLEX, spx.SPX_LAYOUT_HASHED)
    p = torch.from_numpy(inputs.uniform_points(1000, 2, 88)).to(DEV)
    small = torch.empty(16, dtype=torch.uint8, device=DEV)
    with pytest.raises(spx.SpxError):
        spx.spx_encode_bwd_prepare(g, p, small)
    # N = 0: nothing to count
    spx.spx_encode_bwd_prepare(g, p[:0], small)
