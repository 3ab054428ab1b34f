"""GPU parity of the elementwise kernels (binary16 copy, fused Adam) with
the oracle, through the C ABI."""
import numpy as np
import pytest

import oracle
from paper_2311_15439_amd import spx

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
DEV = "cuda"


@pytest.mark.parametrize("n", [1, 1000, (1 << 20) + 3])
def test_cast_bit_exact(n):
    rng = np.random.default_rng(n)
    v = (rng.normal(size=n) * 10.0 ** rng.uniform(-8, 5.5, n)).astype(np.float32)
    src = torch.from_numpy(v).to(DEV)
    dst = torch.empty(n, dtype=torch.float16, device=DEV)
    spx.spx_cast_f32_f16(src, dst)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(dst.cpu().numpy().view(np.uint16), oracle.cast_f32_f16(v))


def test_adam_matches_oracle():
    n = 100003
    rng = np.random.default_rng(1)
    p = rng.normal(size=n).astype(np.float32) * 1e-3
    m = np.zeros(n, np.float32)
    v = np.zeros(n, np.float32)
    tp, tm, tv = (torch.from_numpy(a.copy()).to(DEV) for a in (p, m, v))
    th = torch.empty(n, dtype=torch.float16, device=DEV)
    for step in range(1, 5):
        g = (rng.normal(size=n) * 1e-2).astype(np.float32)
        tg = torch.from_numpy(g).to(DEV)
        spx.spx_adam_step(tp, tg, tm, tv, th, lr=1e-2, beta1=0.9, beta2=0.99, eps=1e-15, step=step, zero_grad=True)
        p, m, v, h = oracle.adam_step(p, g, m, v, 1e-2, 0.9, 0.99, 1e-15, step)
        torch.cuda.synchronize()
        assert torch.count_nonzero(tg).item() == 0  # gradient cleared for the next accumulation
        gp = tp.cpu().numpy()
        np.testing.assert_allclose(gp, p, rtol=1e-5, atol=1e-7)
        np.testing.assert_allclose(tm.cpu().numpy(), m, rtol=1e-5, atol=1e-12)
        np.testing.assert_allclose(tv.cpu().numpy(), v, rtol=1e-5, atol=1e-16)
        # the binary16 image is the round-to-nearest-even copy of the GPU's own parameters
        np.testing.assert_array_equal(th.cpu().numpy().view(np.uint16), oracle.cast_f32_f16(gp))
        p = gp  # continue from the GPU state so rounding differences do not compound


def test_mse_grad_matches_oracle():
    rng = np.random.default_rng(3)
    y = rng.normal(size=(12345, 3)).astype(np.float32)
    t = rng.random((12345, 3)).astype(np.float32)
    ty, tt = torch.from_numpy(y).to(DEV), torch.from_numpy(t).to(DEV)
    d = torch.empty_like(ty)
    scale = 2.0 / y.size
    spx.spx_mse_grad(ty, tt, d, scale)
    torch.cuda.synchronize()
    ref = oracle.mse_grad(y, t, np.float32(scale))
    np.testing.assert_allclose(d.cpu().numpy(), ref, rtol=2 * 2.0 ** -24, atol=0)
