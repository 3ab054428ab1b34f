"""CPU: the network parity bounds of tests/tolerances.py bite.  Oracle
outputs of a wrong network -- one hidden unit dropped, one weight matrix
transposed -- must fail them, while a binary32-accumulating evaluation with
the kernel's rounding points (binary16 activations, bfloat16 backward
operands) must pass."""
import numpy as np
import pytest

import oracle
from paper_2311_15439_amd import inputs
from tolerances import mlp_bwd_problem, mlp_fwd_problem


def _bf16(a):
    b = np.ascontiguousarray(a, np.float32).view(np.uint32).astype(np.uint64)
    return (((b + 0x7FFF + ((b >> 16) & 1)) >> 16) << 16).astype(np.uint32).view(np.float32)


def _f32_fwd(x, W1, W2, W3):
    f = lambda a: a.astype(np.float32)
    h1 = np.maximum(f(x) @ f(W1).T, 0).astype(np.float16).astype(np.float32)
    h2 = np.maximum(h1 @ f(W2).T, 0).astype(np.float16).astype(np.float32)
    return h2 @ f(W3).T


def _f32_bwd(x, W1, W2, W3, dy):
    f = lambda a: a.astype(np.float32)
    h1 = np.maximum(f(x) @ f(W1).T, 0).astype(np.float16).astype(np.float32)
    h2 = np.maximum(h1 @ f(W2).T, 0).astype(np.float16).astype(np.float32)
    g = _bf16(dy)
    dh2 = _bf16(np.where(h2 > 0, g @ _bf16(f(W3)), 0))
    dh1 = _bf16(np.where(h1 > 0, dh2 @ _bf16(f(W2)), 0))
    return dict(dW3=g.T @ _bf16(h2), dW2=dh2.T @ _bf16(h1), dW1=dh1.T @ _bf16(f(x)), d_x=dh1 @ _bf16(f(W1)))


def _wrong_networks(W1, W2, W3):
    """(name, W1, W2, W3) of networks that differ from the right one by one
    plausible mistake."""
    out = []
    for j in (0, 17, 40, 63):
        a = W1.copy()
        a[j] = 0
        out.append((f"layer-1 unit {j} dropped", a, W2, W3))
        b = W2.copy()
        b[j] = 0
        out.append((f"layer-2 unit {j} dropped", W1, b, W3))
    out.append(("W2 transposed", W1, np.ascontiguousarray(W2.T), W3))
    return out


@pytest.mark.parametrize("d_out", [3, 4, 16])
def test_forward_bound_rejects_wrong_networks(d_out):
    W1, W2, W3 = inputs.mlp_weights(32, 64, d_out, 10 + d_out)
    x = inputs.features_f16(3000, 32, 20 + d_out)
    ref, mag = oracle.mlp_fwd(x, W1, W2, W3, with_absmag=True)
    assert mlp_fwd_problem(_f32_fwd(x, W1, W2, W3), ref, mag) is None
    for name, a, b, c in _wrong_networks(W1, W2, W3):
        assert mlp_fwd_problem(oracle.mlp_fwd(x, a, b, c), ref, mag) is not None, name


@pytest.mark.parametrize("d_out", [3, 4, 16])
def test_backward_bound_rejects_wrong_networks(d_out):
    W1, W2, W3 = inputs.mlp_weights(32, 64, d_out, 30 + d_out)
    x = inputs.features_f16(3000, 32, 40 + d_out)
    dy = inputs.gradients(3000, d_out, 50 + d_out)
    keep = oracle.mlp_bwd(x, W1, W2, W3, dy)["margin"] >= 1e-3
    x, dy = x[keep], dy[keep]
    ref = oracle.mlp_bwd(x, W1, W2, W3, dy, with_mag=True)
    assert mlp_bwd_problem(_f32_bwd(x, W1, W2, W3, dy), ref) is None
    for name, a, b, c in _wrong_networks(W1, W2, W3):
        assert mlp_bwd_problem(oracle.mlp_bwd(x, a, b, c, dy), ref) is not None, name
    # the bfloat16 rounding itself is an error the bound must see: the exact
    # derivative differs from the kernel's arithmetic by far more than a flip
    exact = oracle.mlp_bwd(x, W1, W2, W3, dy, mode=oracle.MLP_EXACT)
    assert mlp_bwd_problem(exact, ref) is not None
