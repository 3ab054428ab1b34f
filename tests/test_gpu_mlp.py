"""GPU parity of the matrix-core MLP against the CPU oracle, through the C
ABI.  The bounds (tests/tolerances.py) follow from the arithmetic: the
kernel accumulates in binary32 where the oracle uses binary64, so a value
rounded to binary16 (forward) or bfloat16 (backward) may land one unit in
the last place away; every entry is held to that worst case times the
oracle's ReLU-masked magnitude, and all but 0.1 % of the entries to 2^-14
of it.  The backward is also compared with the network's exact derivative
(no bfloat16 rounding), and its error is reported."""
import json
import os

import numpy as np
import pytest

import oracle
from paper_2311_15439_amd import inputs, spx
from tolerances import mlp_bwd_problem, mlp_bwd_vs_exact, mlp_fwd_problem

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
DEV = "cuda"


def _report(name, rec):
    """Append a record to the file named by SPX_TEST_REPORT, if set."""
    path = os.environ.get("SPX_TEST_REPORT")
    if path:
        with open(path, "a") as fh:
            fh.write(json.dumps({"test": name, **rec}) + "\n")


def _t(a, dtype=None):
    t = torch.from_numpy(np.ascontiguousarray(a)).to(DEV)
    return t if dtype is None else t.to(dtype)


def _gpu_fwd(x, W1, W2, W3):
    m = spx.make_mlp(x.shape[1], W1.shape[0], W3.shape[0])
    y = torch.empty((len(x), W3.shape[0]), dtype=torch.float32, device=DEV)
    spx.spx_mlp_fwd(m, _t(x), _t(W1), _t(W2), _t(W3), y)
    torch.cuda.synchronize()
    return y.cpu().numpy().astype(np.float64)


def _gpu_bwd(x, W1, W2, W3, dy, with_dx=True):
    m = spx.make_mlp(x.shape[1], W1.shape[0], W3.shape[0])
    N = len(x)
    ws = torch.empty(spx.spx_mlp_bwd_workspace(m, N), dtype=torch.uint8, device=DEV)
    dx = torch.empty((N, x.shape[1]), dtype=torch.float32, device=DEV) if with_dx else None
    dW = [torch.full(w.shape, float("nan"), dtype=torch.float32, device=DEV) for w in (W1, W2, W3)]
    spx.spx_mlp_bwd(m, _t(x), _t(W1), _t(W2), _t(W3), _t(dy), dx, *dW, ws)
    torch.cuda.synchronize()
    out = dict(dW1=dW[0].cpu().numpy(), dW2=dW[1].cpu().numpy(), dW3=dW[2].cpu().numpy())
    if with_dx:
        out["d_x"] = dx.cpu().numpy()
    return out


def _safe_points(x, W1, W2, W3, dy, margin=1e-3):
    """Keep the points whose pre-activations are all at least `margin` away
    from the ReLU kink (where binary32 and binary64 sums could take
    different branches)."""
    mg = oracle.mlp_bwd(x, W1, W2, W3, dy)["margin"]
    keep = mg >= margin
    assert keep.mean() > 0.5
    return x[keep], dy[keep]


@pytest.mark.parametrize("d_out,N", [(3, 5000), (4, 4099), (16, 1000), (1, 17)])
def test_mlp_fwd_parity(d_out, N):
    W1, W2, W3 = inputs.mlp_weights(32, 64, d_out, 10 + d_out)
    x = inputs.features_f16(N, 32, 20 + d_out)
    got = _gpu_fwd(x, W1, W2, W3)
    ref, mag = oracle.mlp_fwd(x, W1, W2, W3, with_absmag=True)
    p = mlp_fwd_problem(got, ref, mag)
    assert p is None, p
    np.testing.assert_array_equal(got, _gpu_fwd(x, W1, W2, W3))  # deterministic


@pytest.mark.parametrize("d_out,N", [(3, 6000), (4, 777), (16, 2000), (2, 1)])
def test_mlp_bwd_parity(d_out, N):
    W1, W2, W3 = inputs.mlp_weights(32, 64, d_out, 30 + d_out)
    x = inputs.features_f16(N + N // 4 + 8, 32, 40 + d_out)
    dy = inputs.gradients(len(x), d_out, 50 + d_out)
    x, dy = _safe_points(x, W1, W2, W3, dy)
    got = _gpu_bwd(x, W1, W2, W3, dy)
    ref = oracle.mlp_bwd(x, W1, W2, W3, dy, with_mag=True)
    p = mlp_bwd_problem(got, ref)
    assert p is None, p
    again = _gpu_bwd(x, W1, W2, W3, dy)
    for key in ("dW1", "dW2", "dW3", "d_x"):
        np.testing.assert_array_equal(got[key], again[key])  # fixed reduction order
    # against the network's exact derivative (no bfloat16 rounding)
    exact = oracle.mlp_bwd(x, W1, W2, W3, dy, mode=oracle.MLP_EXACT, with_mag=True)
    rep = mlp_bwd_vs_exact(got, exact)
    _report(f"mlp_bwd_vs_exact d_out={d_out} N={len(x)}", rep)
    for k, r in rep.items():
        assert r["ok"], (k, r)


def test_mlp_bwd_without_dx_and_empty_batch():
    W1, W2, W3 = inputs.mlp_weights(32, 64, 3, 1)
    x = inputs.features_f16(300, 32, 2)
    dy = inputs.gradients(300, 3, 3)
    a = _gpu_bwd(x, W1, W2, W3, dy, with_dx=False)
    b = _gpu_bwd(x, W1, W2, W3, dy, with_dx=True)
    for key in ("dW1", "dW2", "dW3"):
        np.testing.assert_array_equal(a[key], b[key])
    z = _gpu_bwd(x[:0], W1, W2, W3, dy[:0], with_dx=False)
    for key in ("dW1", "dW2", "dW3"):
        assert np.all(z[key] == 0)


def test_mlp_full_size_sampled():
    """2^20 points as in the image workload's training step; outputs of a
    sample of points are compared one by one, and the weight gradient is
    checked on a batch whose output gradient is non-zero only on the sample."""
    N = 1 << 20
    W1, W2, W3 = inputs.mlp_weights(32, 64, 3, 60)
    x = inputs.features_f16(N, 32, 61, scale=0.5)
    got = _gpu_fwd(x, W1, W2, W3)
    sel = np.random.default_rng(2).choice(N, 4096, replace=False)
    ref, mag = oracle.mlp_fwd(x[sel], W1, W2, W3, with_absmag=True)
    p = mlp_fwd_problem(got[sel], ref, mag)
    assert p is None, p
    dy = np.zeros((N, 3), np.float32)
    keep = oracle.mlp_bwd(x[sel], W1, W2, W3, np.ones((len(sel), 3), np.float32))["margin"] >= 1e-3
    sel = sel[keep]
    dy[sel] = inputs.gradients(len(sel), 3, 62)
    g = _gpu_bwd(x, W1, W2, W3, dy)
    r = oracle.mlp_bwd(x[sel], W1, W2, W3, dy[sel], with_mag=True)
    p = mlp_bwd_problem(dict(g, d_x=g["d_x"][sel]), r)
    assert p is None, p
    others = np.ones(N, bool)
    others[sel] = False
    assert np.all(g["d_x"][others] == 0)
    exact = oracle.mlp_bwd(x[sel], W1, W2, W3, dy[sel], mode=oracle.MLP_EXACT, with_mag=True)
    rep = mlp_bwd_vs_exact(dict(g, d_x=g["d_x"][sel]), exact)
    _report("mlp_bwd_vs_exact full size (2^20 points, 4096 with gradient)", rep)
    for k, v in rep.items():
        assert v["ok"], (k, v)
