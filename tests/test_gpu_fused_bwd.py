"""GPU: the network backward fused into the encoding's adjoint
(spx_encode_mlp_bwd_adam), through the C ABI.

  * Against the oracle (small batches, every table entry): the weight
    gradients within the network backward's bounds (tests/tolerances.py);
    the tables' Adam state within the oracle's Adam step applied to the
    oracle's table gradient, where each slot's gradient may differ by the
    adjoint's summation bound plus the network's input-gradient bound
    carried through the adjoint (the weights are non-negative, so the
    adjoint of the per-entry bound bounds the carried error).
  * Against the unfused path (spx_mlp_bwd, then spx_encode_bwd_adam) at
    batches that give each workgroup several rounds, in both scatter shapes:
    weight gradients bit for bit, the tables within the freedom of the
    summation order (the records are the same, their order is not).
Points whose network pre-activations lie within 1e-3 of the ReLU kink are
left out of the oracle cases (binary32 and binary64 sums may take different
branches there)."""
import numpy as np
import pytest

import oracle
from paper_2311_15439_amd import inputs, spx
from test_gpu_encode import adam_problem
from tolerances import BWD_BOUND, TINY, mlp_bwd_problem

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
DEV = "cuda"
U = 2.0 ** -24
KW = dict(lr=1e-2, beta1=0.9, beta2=0.99, eps=1e-15)


def _f32(x):
    return float(np.float32(x))


def _res(n_min, growth):
    return spx.spx_level_resolutions(n_min, growth, 16)


# name, n, res, log2_T, cell, layout, N, point kind, d_out
ORACLE_CASES = [
    ("n2-simplex", 2, _res(16, 1.5), 14, spx.SPX_SIMPLEX, spx.SPX_LAYOUT_HASHED, 6000, "uniform", 3),
    ("n3-rays-few", 3, _res(16, 1.3), 15, spx.SPX_SIMPLEX, spx.SPX_LAYOUT_HASHED, 6144, "rays", 4),
    ("n3-grid", 3, _res(8, 1.25), 15, spx.SPX_GRID, spx.SPX_LAYOUT_HASHED, 5000, "uniform", 4),
    ("n2-sized", 2, _res(16, 1.4), 15, spx.SPX_SIMPLEX, spx.SPX_LAYOUT_SIZED, 6000, "uniform", 3),
    ("n2-grid", 2, _res(16, 1.45), 14, spx.SPX_GRID, spx.SPX_LAYOUT_HASHED, 4097, "uniform", 3),
    ("n1", 1, _res(16, 1.6), 12, spx.SPX_SIMPLEX, spx.SPX_LAYOUT_HASHED, 3000, "uniform", 1),
    ("n2-no-private", 2, _res(600, 1.2), 14, spx.SPX_SIMPLEX, spx.SPX_LAYOUT_HASHED, 5000, "uniform", 3),
]


def _points(kind, N, n, seed):
    if kind == "rays":
        return inputs.ray_points(N // 256, 256, seed)
    return inputs.uniform_points(N, n, seed)


def _encodings(n, res, log2_T, cell, layout):
    g = spx.Encoding(n, list(res), log2_T, 2, table_dtype=spx.SPX_F16, cell=cell, layout=layout)
    o = oracle.Encoding(n, list(res), log2_T, n_feat=2, table_dtype=oracle.F16, cell=cell,
                        layout=oracle.SIZED if layout == spx.SPX_LAYOUT_SIZED else oracle.HASHED)
    return g, o


def _state(shape, seed):
    rng = np.random.default_rng(seed)
    return ((rng.normal(size=shape) * 1e-2).astype(np.float32), (rng.normal(size=shape) * 1e-3).astype(np.float32),
            (rng.random(shape) * 1e-5 + 1e-7).astype(np.float32))


def _t(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def _fused(enc, mlp, pts, x, W, dy, state, step):
    """spx_encode_mlp_bwd_adam: returns (dW list, p, m, v, p16) on the device."""
    tp, tm, tv = (_t(a.copy()) for a in state)
    th = torch.empty(enc.table_shape, dtype=torch.float16, device=DEV)
    dW = [torch.full(w.shape, float("nan"), dtype=torch.float32, device=DEV) for w in W]
    ws = torch.empty(max(spx.spx_encode_mlp_bwd_workspace(enc, mlp, len(pts)), 256), dtype=torch.uint8, device=DEV)
    spx.spx_encode_mlp_bwd_adam(enc, mlp, _t(pts), _t(x), *[_t(w) for w in W], _t(dy), *dW, tp, tm, tv, th,
                                step=step, workspace=ws, **KW)
    torch.cuda.synchronize()
    return dW, tp, tm, tv, th


def _unfused(enc, mlp, pts, x, W, dy, state, step):
    """spx_mlp_bwd then spx_encode_bwd_adam; also returns the input gradient."""
    N = len(pts)
    tp, tm, tv = (_t(a.copy()) for a in state)
    th = torch.empty(enc.table_shape, dtype=torch.float16, device=DEV)
    dW = [torch.full(w.shape, float("nan"), dtype=torch.float32, device=DEV) for w in W]
    dx = torch.empty((N, 32), dtype=torch.float32, device=DEV)
    mws = torch.empty(spx.spx_mlp_bwd_workspace(mlp, N), dtype=torch.uint8, device=DEV)
    spx.spx_mlp_bwd(mlp, _t(x), *[_t(w) for w in W], _t(dy), dx, *dW, mws)
    bws = torch.empty(spx.spx_encode_bwd_workspace(enc, N), dtype=torch.uint8, device=DEV)
    tpts = _t(pts)
    spx.spx_encode_bwd_adam(enc, tpts, dx, tp, tm, tv, th, step=step, workspace=bws, **KW)
    torch.cuda.synchronize()
    return dW, tp, tm, tv, th, dx, tpts, bws


@pytest.mark.parametrize("case", ORACLE_CASES, ids=[c[0] for c in ORACLE_CASES])
def test_fused_bwd_matches_oracle(case):
    name, n, res, log2_T, cell, layout, N, kind, d_out = case
    enc, o = _encodings(n, res, log2_T, cell, layout)
    mlp = spx.make_mlp(32, 64, d_out)
    W = inputs.mlp_weights(32, 64, d_out, 70 + n)
    pts = _points(kind, N, n, 71 + n)
    x = inputs.features_f16(len(pts), 32, 72 + n)
    dy = inputs.gradients(len(pts), d_out, 73 + n, scale=1e-2)
    keep = oracle.mlp_bwd(x, *W, dy)["margin"] >= 1e-3
    assert keep.mean() > 0.5
    pts, x, dy = pts[keep], x[keep], dy[keep]
    state = _state(enc.table_shape, 74 + n)
    step = 3
    dW, tp, tm, tv, th = _fused(enc, mlp, pts, x, W, dy, state, step)

    ref = oracle.mlp_bwd(x, *W, dy, with_mag=True)
    got = dict(dW1=dW[0].cpu().numpy(), dW2=dW[1].cpu().numpy(), dW3=dW[2].cpu().numpy())
    p = mlp_bwd_problem(got, ref, keys=("dW1", "dW2", "dW3"))
    assert p is None, p
    gref, gmag, cnt = oracle.encode_bwd(o, pts, ref["d_x"], with_stats=True)
    carried = oracle.encode_bwd(o, pts, BWD_BOUND * ref["mag_d_x"] + TINY)  # sum of w * (input-gradient bound)
    assert (carried >= 0).all()
    tolg = (cnt + n + 2) * U * gmag + carried + 1e-30
    lr, b1, b2, eps = (_f32(KW[k]) for k in ("lr", "beta1", "beta2", "eps"))
    p = adam_problem(*state, gref, tolg, tp, tm, tv, lr, b1, b2, eps, step)
    assert p is None, f"{name}: {p}"
    np.testing.assert_array_equal(th.cpu().numpy().view(np.uint16).ravel(),
                                  oracle.cast_f32_f16(tp.cpu().numpy().ravel()))


# name, n, res, log2_T, cell, layout, N, point kind, d_out: several rounds
# per workgroup (the staged scatter's rounds are 2048 points for 2-D
# simplex cells and 1024 for few buckets in 3-D)
LARGE_CASES = [
    ("image-many", 2, _res(16, 1.38), 19, spx.SPX_SIMPLEX, spx.SPX_LAYOUT_HASHED, (1 << 21) + 333, "uniform", 3),
    ("volume-few", 3, _res(16, 1.32), 19, spx.SPX_SIMPLEX, spx.SPX_LAYOUT_HASHED, 1200 * 1024, "rays", 4),
    ("volume-many", 3, _res(16, 1.32), 21, spx.SPX_SIMPLEX, spx.SPX_LAYOUT_HASHED, 600 * 1024, "rays", 4),
    ("volume-grid-sized", 3, _res(16, 1.32), 19, spx.SPX_GRID, spx.SPX_LAYOUT_SIZED, 700 * 1024, "rays", 4),
]


@pytest.mark.parametrize("case", LARGE_CASES, ids=[c[0] for c in LARGE_CASES])
def test_fused_bwd_matches_unfused(case):
    """Same records as the unfused path (the input gradient has the same
    bits), summed in another order: per entry the two gradients differ by
    at most twice the summation bound (counts from the oracle, which depend
    only on the points; magnitudes sum |w d_x| from the device's own
    adjoint of |d_x|, a consistency bound between two device paths)."""
    name, n, res, log2_T, cell, layout, N, kind, d_out = case
    enc, o = _encodings(n, res, log2_T, cell, layout)
    mlp = spx.make_mlp(32, 64, d_out)
    W = inputs.mlp_weights(32, 64, d_out, 80 + n)
    pts = _points(kind, N, n, 81 + n)
    x = inputs.features_f16(len(pts), 32, 82 + n)
    dy = inputs.gradients(len(pts), d_out, 83 + n, scale=1e-2)
    state = _state(enc.table_shape, 84 + n)
    step = 2
    fdW, fp, fm, fv, fh = _fused(enc, mlp, pts, x, W, dy, state, step)
    udW, up, um, uv, uh, dx, tpts, bws = _unfused(enc, mlp, pts, x, W, dy, state, step)
    for a, b in zip(fdW, udW):
        assert torch.equal(a, b)
    gmag = torch.zeros(enc.table_shape, dtype=torch.float32, device=DEV)
    spx.spx_encode_bwd(enc, tpts, dx.abs(), gmag, bws)
    torch.cuda.synchronize()
    _, _, cnt = oracle.encode_bwd(o, pts, np.zeros((len(pts), 32)), with_stats=True)
    S = (2 * (cnt + n + 2) * U * gmag.cpu().numpy().astype(np.float64)).ravel()
    b1, b2 = _f32(KW["beta1"]), _f32(KW["beta2"])
    m0, v0 = (a.ravel().astype(np.float64) for a in state[1:])
    gm_f, gm_u = (t.cpu().numpy().ravel().astype(np.float64) for t in (fm, um))
    gv_f, gv_u = (t.cpu().numpy().ravel().astype(np.float64) for t in (fv, uv))
    G = np.abs(gm_u - b1 * m0) / (1 - b1) + S  # |gradient| bound recovered from m
    tol_m = (1 - b1) * S + 6 * U * (b1 * np.abs(m0) + (1 - b1) * G)
    tol_v = (1 - b2) * (2 * G + S) * S + 8 * U * (b2 * v0 + (1 - b2) * G ** 2)
    for nm, a, b, tol in [("m", gm_f, gm_u, tol_m), ("v", gv_f, gv_u, tol_v)]:
        err = np.abs(a - b)
        assert (err <= tol + 1e-30).all(), f"{name} {nm}: worst err/tol {np.max(err / (tol + 1e-30)):.3f}"
    # the step itself is the same code on the same m and v: p follows them
    np.testing.assert_allclose(fp.cpu().numpy(), up.cpu().numpy(), rtol=0, atol=1e-6)
    np.testing.assert_array_equal(fh.cpu().numpy().view(np.uint16).ravel(),
                                  oracle.cast_f32_f16(fp.cpu().numpy().ravel()))


def test_fused_bwd_without_points():
    """No points: weight gradients are zero and every table entry takes its
    Adam step with a zero gradient, as spx_encode_bwd_adam without points."""
    enc, _ = _encodings(3, _res(16, 1.3), 15, spx.SPX_SIMPLEX, spx.SPX_LAYOUT_HASHED)
    mlp = spx.make_mlp(32, 64, 4)
    W = inputs.mlp_weights(32, 64, 4, 90)
    state = _state(enc.table_shape, 91)
    e2 = np.zeros((0, 3), np.float32)
    dW, tp, tm, tv, th = _fused(enc, mlp, e2, np.zeros((0, 32), np.float16), W, np.zeros((0, 4), np.float32),
                                state, 4)
    for d in dW:
        assert torch.count_nonzero(d).item() == 0
    b = [_t(a.copy()) for a in state]
    hb = torch.empty(enc.table_shape, dtype=torch.float16, device=DEV)
    spx.spx_adam_step(b[0], torch.zeros(enc.table_shape, device=DEV), b[1], b[2], hb, zero_grad=False, step=4, **KW)
    torch.cuda.synchronize()
    for x, y in zip([tp, tm, tv, th], b + [hb]):
        assert torch.equal(x, y)
