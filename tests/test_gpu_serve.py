"""GPU: the fused multi-field query equals the separate encoding and network
kernels bit for bit, whatever the batch, and the server returns the same
result for a request alone and in a mix."""
import numpy as np
import pytest

import oracle
from paper_2311_15439_amd import inputs, spx
from tolerances import mlp_fwd_problem

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
DEV = "cuda"

SPECS = [(3, spx.SPX_SIMPLEX, 4), (2, spx.SPX_SIMPLEX, 3), (3, spx.SPX_GRID, 4), (2, spx.SPX_GRID, 16)]


def _make_fields():
    out = []
    for i, (n, cell, d_out) in enumerate(SPECS):
        res = spx.spx_level_resolutions(16, 1.38, 16)
        enc = spx.Encoding(n, res, 14, 2, table_dtype=spx.SPX_F16, cell=cell)
        tab = torch.from_numpy(inputs.tables(16, 1 << 14, 2, 0.5, 30 + i, True)).to(DEV)
        W = [torch.from_numpy(w).to(DEV) for w in inputs.mlp_weights(32, 64, d_out, 40 + i)]
        out.append(dict(enc=enc, tab=tab, W=W, d_out=d_out, desc=spx.spx_field_init(enc, tab, *W, d_out)))
    return out


def _separate(fd, pts):
    N = pts.shape[0]
    feats = torch.empty((N, 32), dtype=torch.float16, device=DEV)
    spx.spx_encode_fwd(fd["enc"], pts, fd["tab"], feats)
    y = torch.empty((N, fd["d_out"]), dtype=torch.float32, device=DEV)
    spx.spx_mlp_fwd(spx.make_mlp(32, 64, fd["d_out"]), feats, *fd["W"], y)
    return y


def test_field_query_equals_separate_kernels():
    fields = _make_fields()
    fdev = torch.frombuffer(bytearray(spx.as_bytes([f["desc"] for f in fields])), dtype=torch.uint8).to(DEV)
    rng = np.random.default_rng(1)
    sizes = [1, 15, 16, 17, 1000, 4097, 3, 65536, 700, 33]
    segs, bufs, first = [], [], 0
    for k, m in enumerate(sizes):
        f = int(rng.integers(0, len(fields))) if k != 6 else 99  # one segment names no field
        n = fields[f]["enc"].n_dims if f < len(fields) else 3
        pts = torch.from_numpy(inputs.uniform_points(m, n, 100 + k)).to(DEV)
        d_out = fields[f]["d_out"] if f < len(fields) else 4
        out = torch.full((m, d_out), float("nan"), device=DEV)
        s = spx.spx_segment()
        s.pts, s.out, s.count, s.first_tile, s.field = pts.data_ptr(), out.data_ptr(), m, first, f
        first += (m + 15) // 16
        segs.append(s)
        bufs.append((f, pts, out))
    sdev = torch.frombuffer(bytearray(spx.as_bytes(segs)), dtype=torch.uint8).to(DEV)
    spx.spx_field_query_batched(fdev, len(fields), sdev, len(segs), first)
    torch.cuda.synchronize()
    for f, pts, out in bufs:
        if f >= len(fields):
            assert torch.isnan(out).all()  # skipped, untouched
            continue
        ref = _separate(fields[f], pts)
        assert torch.equal(out, ref)
    # and the separate kernels match the oracle for one field
    f, pts, out = bufs[4]
    fd = fields[f]
    oe = oracle.Encoding(fd["enc"].n_dims, list(fd["enc"].res), 14, 2, table_dtype=oracle.F16, cell=fd["enc"].cell)
    gfeats = torch.empty((len(pts), 32), dtype=torch.float16, device=DEV)
    spx.spx_encode_fwd(fd["enc"], pts, fd["tab"], gfeats)
    gfeats = gfeats.cpu().numpy()
    p_np, tab_np = pts.cpu().numpy(), fd["tab"].cpu().numpy()
    fo, fm = oracle.encode_fwd(oe, p_np, tab_np), oracle.encode_fwd_absmag(oe, p_np, tab_np)
    assert (np.abs(gfeats.astype(np.float64) - fo) <= 1e-5 * fm + 2.0 ** -11 * np.abs(fo) + 2.0 ** -25).all()
    # the network on the features the kernel encoded (binary16, as it feeds them to the matrix cores)
    yo, ym = oracle.mlp_fwd(gfeats, *[w.cpu().numpy() for w in fd["W"]], with_absmag=True)
    p = mlp_fwd_problem(out.cpu().numpy(), yo, ym)
    assert p is None, p


def test_server_alone_equals_mixed_on_gpu():
    from paper_2311_15439_amd.serve import GpuBackend, Server
    fields = _make_fields()
    be = GpuBackend([f["desc"] for f in fields])
    srv = Server(be, [f["enc"].n_dims for f in fields], [f["d_out"] for f in fields], arena_bytes=64 << 20,
                 chunk_points=1 << 14, batch_points=1 << 16).start()
    try:
        pts = inputs.uniform_points(50000, 3, 7)
        alone = srv.submit(0, pts).wait(60)
        rs = [srv.submit(i % 4, inputs.uniform_points(1000 + 997 * i, SPECS[i % 4][0], i)) for i in range(20)]
        mixed = srv.submit(0, pts)
        rs += [srv.submit(i % 4, inputs.uniform_points(5000, SPECS[i % 4][0], 50 + i)) for i in range(10)]
        np.testing.assert_array_equal(mixed.wait(60), alone)
        ref = _separate(fields[0], torch.from_numpy(pts).to(DEV)).cpu().numpy()
        np.testing.assert_array_equal(alone, ref)
        for r in rs:
            r.wait(60)
        assert srv.batches >= 2
    finally:
        srv.stop()
    assert srv.arena.free_bytes == srv.arena.capacity
