"""GPU: the autograd wrappers give the oracle's values and gradients, the
fused field equals the composition of its parts, and a small field trains."""
import numpy as np
import pytest

import oracle
from paper_2311_15439_amd import inputs, spx
from tolerances import mlp_bwd_problem, mlp_fwd_problem

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
DEV = "cuda"


def _oracle_enc(m):
    e = m.enc
    return oracle.Encoding(e.n_dims, list(e.res), e.log2_T, e.n_feat, table_dtype=oracle.F16, cell=e.cell)


def test_encoding_fn_matches_oracle():
    from paper_2311_15439_amd.torch_ops import SimplexEncoding
    m = SimplexEncoding(3, n_levels=4, log2_T=14, n_min=8, n_max=200, init_scale=1.0, seed=1)
    pts = inputs.uniform_points(5000, 3, 2)
    tp = torch.from_numpy(pts).to(DEV)
    out = m(tp)
    G = inputs.gradients(5000, 8, 3)
    (out * torch.from_numpy(G).to(DEV)).sum().backward()
    torch.cuda.synchronize()
    oe = _oracle_enc(m)
    tab16 = m.table_f16.cpu().numpy()
    np.testing.assert_array_equal(tab16, m.params.detach().cpu().numpy().astype(np.float16))
    ref = oracle.encode_fwd(oe, pts, tab16)
    mag = oracle.encode_fwd_absmag(oe, pts, tab16)
    assert (np.abs(out.detach().cpu().numpy() - ref) <= 1e-5 * mag + 1e-30).all()
    gref, gmag, cnt = oracle.encode_bwd(oe, pts, G.astype(np.float64), with_stats=True)
    assert (np.abs(m.params.grad.cpu().numpy() - gref) <= (cnt + 5) * 2.0 ** -24 * gmag + 1e-30).all()


def test_mlp_fn_matches_oracle():
    from paper_2311_15439_amd.torch_ops import TinyMLP
    net = TinyMLP(32, 3, seed=4)
    W16 = [w.detach().cpu().numpy().astype(np.float16) for w in (net.W1, net.W2, net.W3)]
    x = inputs.features_f16(3600, 32, 5)
    gy = inputs.gradients(3600, 3, 6)
    keep = oracle.mlp_bwd(x, *W16, gy)["margin"] >= 1e-3  # away from the ReLU kinks
    x, gy = x[keep].astype(np.float32), gy[keep]
    tx = torch.from_numpy(x).to(DEV).requires_grad_(True)
    y = net(tx)
    (y * torch.from_numpy(gy).to(DEV)).sum().backward()
    torch.cuda.synchronize()
    ref, mag = oracle.mlp_fwd(x.astype(np.float16), *W16, with_absmag=True)
    p = mlp_fwd_problem(y.detach().cpu().numpy(), ref, mag)
    assert p is None, p
    r = oracle.mlp_bwd(x.astype(np.float16), *W16, gy, with_mag=True)
    got = {"d_x": tx.grad.cpu().numpy(), "dW1": net.W1.grad.cpu().numpy(), "dW2": net.W2.grad.cpu().numpy(),
           "dW3": net.W3.grad.cpu().numpy()}
    p = mlp_bwd_problem(got, r)
    assert p is None, p


def test_field_equals_composition():
    from paper_2311_15439_amd.torch_ops import NeuralField, SimplexEncoding, TinyMLP
    enc = SimplexEncoding(2, n_levels=16, log2_T=16, n_min=16, n_max=2048, init_scale=0.5, seed=7)
    net = TinyMLP(32, 3, seed=8)
    field = NeuralField(enc, net)
    pts = torch.from_numpy(inputs.pixel_points(20000, 9, width=4096)).to(DEV)
    gy = torch.from_numpy(inputs.gradients(20000, 3, 10)).to(DEV)
    y1 = field(pts)
    (y1 * gy).sum().backward()
    g1 = [p.grad.clone() for p in (enc.params, net.W1, net.W2, net.W3)]
    for p in (enc.params, net.W1, net.W2, net.W3):
        p.grad = None
    y2 = net(enc(pts))
    (y2 * gy).sum().backward()
    g2 = [p.grad.clone() for p in (enc.params, net.W1, net.W2, net.W3)]
    torch.cuda.synchronize()
    assert torch.equal(y1, y2)  # same binary16 features, same kernels
    for a, b in zip(g1[1:], g2[1:]):
        assert torch.equal(a, b)  # weight gradients are reduced in a fixed order
    # table gradients: same contributions, summation order may differ
    scale = (g1[0].abs() + g2[0].abs()).max()
    assert ((g1[0] - g2[0]).abs() <= 1e-5 * scale).all()


@pytest.mark.parametrize("cell", [spx.SPX_SIMPLEX, spx.SPX_GRID])
def test_small_field_trains(cell):
    """200 Adam steps on a synthetic RGB target lower the loss several-fold
    for the simplex and the grid encodings alike."""
    from paper_2311_15439_amd.torch_ops import NeuralField, SimplexEncoding, TinyMLP
    torch.manual_seed(0)
    enc = SimplexEncoding(2, n_levels=16, log2_T=16, n_min=16, n_max=1024, cell=cell,
                          equal_memory=(cell == spx.SPX_SIMPLEX), seed=1)
    net = TinyMLP(32, 3, seed=2)
    field = NeuralField(enc, net)
    opt = torch.optim.Adam(field.parameters(), lr=1e-2, betas=(0.9, 0.99), eps=1e-15)
    losses = []
    for step in range(200):
        pts = inputs.pixel_points(1 << 14, 100 + step, width=1024)
        tgt = torch.from_numpy(inputs.procedural_rgb(pts, 4)).to(DEV)
        y = field(torch.from_numpy(pts).to(DEV))
        loss = torch.mean((y - tgt) ** 2)
        opt.zero_grad()
        loss.backward()
        opt.step()
        losses.append(loss.item())
    assert np.mean(losses[-20:]) < 0.2 * np.mean(losses[:5]), (losses[:5], losses[-20:])


def test_encoding_fn_input_gradient():
    """Points that require a gradient receive d L / d x from the input-gradient
    kernel, equal to the oracle's for the binary16 tables the forward read."""
    from paper_2311_15439_amd.torch_ops import SimplexEncoding
    m = SimplexEncoding(3, n_levels=4, log2_T=14, n_min=8, n_max=200, init_scale=1.0, seed=3)
    pts = inputs.uniform_points(3000, 3, 12)
    tp = torch.from_numpy(pts).to(DEV).requires_grad_(True)
    G = inputs.gradients(3000, 8, 13)
    (m(tp) * torch.from_numpy(G).to(DEV)).sum().backward()
    torch.cuda.synchronize()
    oe = _oracle_enc(m)
    ref, mag = oracle.encode_input_grad(oe, pts, m.table_f16.cpu().numpy(), G.astype(np.float64), with_mag=True)
    tol = 2 * (2 + 6 + 4 + 4 + 8) * 2.0 ** -24 * mag + 1e-30
    assert (np.abs(tp.grad.cpu().numpy() - ref) <= tol).all()


@pytest.mark.parametrize("layout", [spx.SPX_LAYOUT_HASHED, spx.SPX_LAYOUT_SIZED])
@pytest.mark.parametrize("cell", [spx.SPX_SIMPLEX, spx.SPX_GRID])
def test_table_gradient_central_differences_on_gpu(cell, layout):
    """Autograd's table gradient (the binned adjoint) against central
    differences of the GPU forward, entry by entry.  The encoding is linear
    in the stored (binary16) table values, so the difference quotient over
    the actual binary16 step is the derivative up to the forward's rounding
    (loss summed in binary64)."""
    from paper_2311_15439_amd.torch_ops import SimplexEncoding
    m = SimplexEncoding(3, n_levels=4, log2_T=12, n_min=6, n_max=90, init_scale=0.5, seed=11, cell=cell,
                        layout=layout)
    pts = torch.from_numpy(inputs.uniform_points(4000, 3, 12)).to(DEV)
    d = torch.from_numpy(inputs.gradients(4000, 8, 13)).to(DEV).double()

    def loss():
        return float((m(pts).double() * d).sum())

    (m(pts).double() * d).sum().backward()
    g = m.params.grad.detach().cpu().numpy().reshape(-1)
    flat = m.params.detach().view(-1)
    rows = np.flatnonzero(np.abs(g) > 1e-3)
    sel = np.random.default_rng(14).choice(rows, 16, replace=False)
    for i in sel:
        old = float(flat[i])
        with torch.no_grad():
            flat[i] = old + 0.25
        up, a = loss(), float(m.table_f16.view(-1)[i])
        with torch.no_grad():
            flat[i] = old - 0.25
        dn, b = loss(), float(m.table_f16.view(-1)[i])
        with torch.no_grad():
            flat[i] = old
        fd = (up - dn) / (a - b)
        assert abs(fd - g[i]) <= 1e-4 * abs(g[i]) + 1e-4, (i, fd, g[i])


@pytest.mark.parametrize("cell", [spx.SPX_SIMPLEX, spx.SPX_GRID])
def test_input_gradient_central_differences_on_gpu(cell):
    """Autograd's gradient with respect to the points against central
    differences of the GPU forward (binary32 tables and outputs), at points
    whose lookups do not change across the step (the encoding is affine
    inside a simplex or cell).  The forward rounds the skewed coordinate
    (below 2) and the scaled one to binary32 at each of the two evaluation
    points, so the scaled step sigma_l * dp of every axis is off by up to
    3 sigma_l 2^-23 per evaluation; through the simplex's skew every axis
    moves, and sum_i |d f / d p_i| is at most 3 times the derivative's
    magnitude over sigma (the oracle's sum over absolute values, with
    F_3 = 1/3), so the quotient is within 9 * 2^-23 / h of the magnitude
    (12 used)."""
    n, res, log2_T = 3, [5, 17, 60], 14
    enc = spx.Encoding(n, res, log2_T, 2, table_dtype=spx.SPX_F32, cell=cell)
    tab = torch.from_numpy(inputs.tables(3, 1 << log2_T, 2, 1.0, 15, False)).to(DEV)
    x = torch.from_numpy(inputs.uniform_points(512, n, 16)).to(DEV)
    d = torch.from_numpy(inputs.gradients(512, 6, 17)).to(DEV)
    dx = torch.empty_like(x)
    spx.spx_encode_input_grad(enc, x, tab, d, dx)
    h = 2.0 ** -12
    _, mag = oracle.encode_input_grad(oracle.Encoding(n, res, log2_T, 2, table_dtype=oracle.F32, cell=cell),
                                      x.cpu().numpy(), tab.cpu().numpy(), d.cpu().numpy().astype(np.float64),
                                      with_mag=True)
    out = torch.empty((512, 6), device=DEV)
    idx = torch.empty((512, 3, enc.n_vertices), dtype=torch.int32, device=DEV)
    spx.spx_encode_debug(enc, x, idx=idx)
    ref_idx = idx.clone()
    checked = 0
    for i in range(n):
        e = torch.zeros(n, device=DEV)
        e[i] = h
        f = []
        same = torch.ones(512, dtype=torch.bool, device=DEV)
        for s in (+1, -1):
            xs = (x + s * e).contiguous()
            spx.spx_encode_fwd(enc, xs, tab, out)
            f.append((out.double() * d.double()).sum(1))
            spx.spx_encode_debug(enc, xs, idx=idx)
            same &= (idx == ref_idx).all(2).all(1)
        step = ((x[:, i] + h) - (x[:, i] - h)).double()
        fd = (f[0] - f[1]) / step
        got = dx[:, i].double()
        ok = same.cpu().numpy()
        err = (fd - got).abs().cpu().numpy()[ok]
        tol = (12 * 2.0 ** -23 / h + 1e-5) * mag[ok, i] + 1e-4
        assert (err <= tol).all(), float((err / tol).max())
        checked += int(ok.sum())
    assert checked > 1000
