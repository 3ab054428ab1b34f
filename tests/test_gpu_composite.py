"""GPU: volume rendering of ray samples (Eq. 5 quadrature) and its adjoint
against the oracle, through the C ABI.

Tolerance, from the binary32 arithmetic: the optical depth before a sample
is a scan of up to S terms (a 6-level wave scan per row plus a running sum
over m = ceil(S / 64) rows), so its relative error is at most (6 + m) u;
exp turns that into a relative error of (6 + m) u P in T, where P is the
ray's total optical depth; softplus, expm1, sigmoid and the products add a
few u each, and the per-lane and wave sums (m + 6) u.  Every term of the
output is non-negative, so per channel
    |gpu - oracle| <= 4 u ((6 + m) P + m + 20) * rgba
(a margin of 4 over the first-order sum).  The adjoint is bounded the same
way against the oracle's magnitude of each derivative expression.
"""
import numpy as np
import pytest

import oracle
from paper_2311_15439_amd import spx

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
U = 2.0 ** -24


def _rays(R, S, seed, special=False):
    rng = np.random.default_rng(seed)
    raw = (rng.normal(size=(R, S, 4)) * 2.0).astype(np.float32)
    raw[..., 0] += np.float32(rng.uniform(-3, 1))
    delta = rng.uniform(0.2, 2.0, (R, S)).astype(np.float32) / S
    if special and R >= 4:
        raw[0, 0, 0] = 60.0            # opaque first sample
        delta[0, 0] = 1.0
        raw[1, :, 0] = -40.0           # empty ray
        raw[2, :, 0] = 12.0            # dense medium
        raw[3] = raw[3, :1]            # constant medium
        delta[3] = delta[3, 0]
    return raw, delta


def _optical_depth(raw, delta):
    return (np.logaddexp(0.0, raw[..., 0].astype(np.float64)) * delta).sum(1)


def _gpu(raw, delta, d_rgba=None):
    tr, td = torch.from_numpy(raw).cuda(), torch.from_numpy(delta).cuda()
    rgba = torch.empty((raw.shape[0], 4), dtype=torch.float32, device="cuda")
    spx.spx_composite_fwd(tr, td, rgba)
    d_raw = None
    if d_rgba is not None:
        d_raw = torch.empty_like(tr)
        spx.spx_composite_bwd(tr, td, torch.from_numpy(d_rgba.astype(np.float32)).cuda(), d_raw)
        d_raw = d_raw.cpu().numpy().astype(np.float64)
    torch.cuda.synchronize()
    return rgba.cpu().numpy().astype(np.float64), d_raw


@pytest.mark.parametrize("R,S", [(1, 1), (37, 7), (64, 64), (33, 65), (300, 256), (20, 1000), (9, 1024),
                                 (1 << 13, 256)])
def test_composite_parity(R, S):
    raw, delta = _rays(R, S, 1000 + S, special=True)
    g = np.random.default_rng(S).normal(size=(R, 4))
    got, d_got = _gpu(raw, delta, g)
    ref = oracle.composite_fwd(raw, delta)
    d_ref, mag = oracle.composite_bwd(raw, delta, g.astype(np.float32).astype(np.float64), with_mag=True)
    m = (S + 63) // 64
    P = _optical_depth(raw, delta)
    scale = (6 + m) * P + m + 20
    tol = 4 * U * scale[:, None] * ref + 1e-30
    err = np.abs(got - ref)
    assert (err <= tol).all(), f"forward: worst err/tol {np.max(err / tol):.3f}"
    tol_b = 4 * U * (scale + 10)[:, None, None] * mag + 1e-30
    err_b = np.abs(d_got - d_ref)
    worst = np.unravel_index(np.argmax(err_b / tol_b), err_b.shape)
    assert (err_b <= tol_b).all(), (f"adjoint: worst err/tol {np.max(err_b / tol_b):.3f} at {worst}: "
                                    f"gpu {d_got[worst]:.9e} oracle {d_ref[worst]:.9e} mag {mag[worst]:.3e}")


def test_composite_edge_arguments():
    raw = torch.zeros((0, 8, 4), device="cuda")
    spx.spx_composite_fwd(raw, torch.zeros((0, 8), device="cuda"), torch.zeros((0, 4), device="cuda"))
    big = torch.zeros((1, 1025, 4), device="cuda")
    with pytest.raises(spx.SpxError):
        spx.spx_composite_fwd(big, torch.zeros((1, 1025), device="cuda"), torch.zeros((1, 4), device="cuda"))
