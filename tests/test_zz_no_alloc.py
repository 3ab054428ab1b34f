"""The allocation-free MLP backward (spx_mlp_bwd_noalloc, static device
scratch) against spx_mlp_bwd with a caller workspace, through the C ABI:
same kernels, same number of workgroups and the same fixed reduction order,
so the results must be bit-identical.  Two calls in a row, the second with
fewer points (its scratch still holds the first call's partials), then the
first size again."""
import numpy as np
import pytest

from paper_2311_15439_amd import inputs, spx

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
DEV = "cuda"


def _t(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def _run(fn, m, x, W, dy, with_dx=True):
    N = x.shape[0]
    dx = torch.full((N, m.d_in), float("nan"), dtype=torch.float32, device=DEV) if with_dx else None
    dW = [torch.full(w.shape, float("nan"), dtype=torch.float32, device=DEV) for w in W]
    if fn == "workspace":
        ws = torch.empty(spx.spx_mlp_bwd_workspace(m, N), dtype=torch.uint8, device=DEV)
        spx.spx_mlp_bwd(m, x, *W, dy, dx, *dW, ws)
    else:
        spx.spx_mlp_bwd_noalloc(m, x, *W, dy, dx, *dW)
    torch.cuda.synchronize()
    out = [d.cpu().numpy() for d in dW]
    if with_dx:
        out.append(dx.cpu().numpy())
    return out


def test_noalloc_matches_workspace_backward():
    d_out = 3
    m = spx.make_mlp(32, 64, d_out)
    W = [_t(w) for w in inputs.mlp_weights(32, 64, d_out, 71)]
    # 2^18 points use the full 512 workgroups; 1000 points use 16
    for N, seed in ((1 << 18, 72), (1000, 73), (1 << 18, 74)):
        print(f"noalloc case N={N} seed={seed}", flush=True)
        x = _t(inputs.features_f16(N, 32, seed))
        dy = _t(inputs.gradients(N, d_out, seed + 100))
        ref = _run("workspace", m, x, W, dy)
        got = _run("noalloc", m, x, W, dy)
        for a, b in zip(got, ref):
            assert np.isfinite(a).all()
            np.testing.assert_array_equal(a, b)


def test_noalloc_without_dx_and_empty_batch():
    m = spx.make_mlp(32, 64, 4)
    W = [_t(w) for w in inputs.mlp_weights(32, 64, 4, 75)]
    x = _t(inputs.features_f16(5000, 32, 76))
    dy = _t(inputs.gradients(5000, 4, 77))
    a = _run("noalloc", m, x, W, dy, with_dx=False)
    b = _run("workspace", m, x, W, dy, with_dx=False)
    for u, v in zip(a, b):
        np.testing.assert_array_equal(u, v)
    z = _run("noalloc", m, x[:0], W, dy[:0], with_dx=False)
    for u in z:
        assert np.all(u == 0)


def test_noalloc_rejects_bad_arguments():
    m = spx.make_mlp(32, 64, 3)
    W = [_t(w) for w in inputs.mlp_weights(32, 64, 3, 78)]
    x = _t(inputs.features_f16(64, 32, 79))
    dy = _t(inputs.gradients(64, 3, 80))
    dW = [torch.empty(w.shape, dtype=torch.float32, device=DEV) for w in W]
    bad = spx.make_mlp(48, 64, 3)
    with pytest.raises(spx.SpxError) as e:
        spx.spx_mlp_bwd_noalloc(bad, torch.empty((64, 48), dtype=torch.float16, device=DEV), *W, dy, None, *dW)
    assert e.value.status == spx.SPX_EUNSUPPORTED
    with pytest.raises(spx.SpxError) as e:
        xs = x.view(-1)[1:1 + 63 * 32].view(63, 32)  # starts 2 bytes in: not 16-byte aligned
        spx.spx_mlp_bwd_noalloc(m, xs, *W, dy[1:], None, *dW)
    assert e.value.status == spx.SPX_EALIGN
