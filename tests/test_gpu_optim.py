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
    """Each step is compared from the same starting state (the GPU's), with
    the binary32 hyper-parameters the kernel receives.  Bounds count the
    binary32 roundings of each update: m and v take three, the parameter
    update about eight relative to its size."""
    n = 100003
    rng = np.random.default_rng(1)
    f32 = lambda v: float(np.float32(v))
    lr, b1, b2, eps = f32(1e-2), f32(0.9), f32(0.99), f32(1e-15)
    u = 2.0 ** -24
    p = (rng.normal(size=n) * 1e-3).astype(np.float32)
    tp = torch.from_numpy(p.copy()).to(DEV)
    tm = torch.zeros(n, device=DEV)
    tv = torch.zeros(n, device=DEV)
    th = torch.empty(n, dtype=torch.float16, device=DEV)
    for step in range(1, 6):
        p0, m0, v0 = tp.cpu().numpy(), tm.cpu().numpy(), tv.cpu().numpy()
        g = (rng.normal(size=n) * 1e-2).astype(np.float32)
        tg = torch.from_numpy(g).to(DEV)
        spx.spx_adam_step(tp, tg, tm, tv, th, lr=lr, beta1=b1, beta2=b2, eps=eps, step=step, zero_grad=True)
        p, m, v, _ = oracle.adam_step(p0, g, m0, v0, lr, b1, b2, eps, step)
        torch.cuda.synchronize()
        assert torch.count_nonzero(tg).item() == 0  # gradient cleared for the next accumulation
        gp, gm, gv = tp.cpu().numpy(), tm.cpu().numpy(), tv.cpu().numpy()
        g64 = g.astype(np.float64)
        tol_m = 3 * u * (b1 * np.abs(m0) + (1 - b1) * np.abs(g64)) + 1e-45
        tol_v = 4 * u * (b2 * v0 + (1 - b2) * g64 ** 2) + 1e-45
        upd = np.abs(p0.astype(np.float64) - p)
        # one ulp (both sides round p to binary32), the update's own roundings,
        # and the error of m carried through lr * m_hat / sqrt(v_hat)
        vhat = v.astype(np.float64) / (1 - b2 ** step)
        carried = lr * tol_m / (1 - b1 ** step) / (np.sqrt(vhat) + eps)
        tol_p = 2 * u * np.abs(p) + 10 * u * upd + carried + 1e-45
        for name, got, ref, tol in [("m", gm, m, tol_m), ("v", gv, v, tol_v), ("p", gp, p, tol_p)]:
            err = np.abs(got.astype(np.float64) - ref)
            assert (err <= tol).all(), f"step {step} {name}: worst err/tol {np.max(err / tol):.3f}"
        # the binary16 image is the round-to-nearest-even copy of the GPU's own parameters
        np.testing.assert_array_equal(th.cpu().numpy().view(np.uint16), oracle.cast_f32_f16(gp))


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
