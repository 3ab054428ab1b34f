"""C ABI checks that need no GPU: the library loads, exports every symbol
the header declares, its host helpers agree bit for bit with the oracle's
independently derived constants, and malformed calls are rejected on the
host before anything is launched."""
import ctypes as C
import subprocess

import numpy as np
import pytest

import oracle
from paper_2311_15439_amd import inputs, spx


def test_exports_every_header_symbol():
    names = spx.header_symbols()
    assert len(names) >= 14
    out = subprocess.run(["nm", "-D", "--defined-only", spx.LIB_PATH], capture_output=True, text=True, check=True).stdout
    exported = {ln.split()[-1] for ln in out.splitlines() if " T " in ln}
    missing = [n for n in names if n not in exported]
    assert not missing, missing
    for n in names:
        assert hasattr(spx.lib(), n)
    assert set(names) == set(spx._SIGNATURES)


def test_abi_version_and_status_strings():
    assert spx.spx_abi_version() == 2
    for s in range(5):
        assert spx.spx_status_str(s).startswith("SPX_")


def test_hash_primes_match_oracle():
    assert spx.spx_hash_primes() == [int(p) for p in oracle.hash_primes()]


@pytest.mark.parametrize("w", [inputs.PLAIN_2D, inputs.IMAGE_2D, inputs.VOLUME_3D] +
                         [inputs.sweep_workload(n) for n in range(2, 7)])
def test_level_resolutions_match_oracle(w):
    ours = spx.spx_level_resolutions(w.n_min, w.growth, w.n_levels)
    assert ours == list(oracle.level_resolutions(w.n_min, w.growth, w.n_levels))


@pytest.mark.parametrize("n", range(1, 7))
@pytest.mark.parametrize("cell", [spx.SPX_SIMPLEX, spx.SPX_GRID])
@pytest.mark.parametrize("em", [False, True])
def test_level_scales_match_oracle(n, cell, em):
    res = [1, 2, 3, 16, 24, 36, 54, 100, 1000, 2048, 32768, 1 << 20]
    enc = spx.Encoding(n, res, 14, cell=cell, equal_memory=em)
    ours = np.array(spx.spx_level_scales(enc), np.float32)
    theirs = oracle.level_scales(n, res, cell=cell, equal_memory=em and cell == spx.SPX_SIMPLEX)
    np.testing.assert_array_equal(ours, theirs)


@pytest.mark.parametrize("n,res,log2_T,cell", [
    (2, [16, 24, 36, 54], 14, spx.SPX_SIMPLEX), (3, [4, 9, 20, 45, 90], 16, spx.SPX_SIMPLEX),
    (2, [5, 12, 130, 700], 14, spx.SPX_GRID), (4, [3, 6, 11, 19], 12, spx.SPX_SIMPLEX),
    (3, [6, 30, 150], 18, spx.SPX_GRID), (6, [16, 28, 50, 90], 20, spx.SPX_SIMPLEX),
    (1, [7, 70, 7000], 10, spx.SPX_SIMPLEX)])
@pytest.mark.parametrize("layout", [spx.SPX_LAYOUT_HASHED, spx.SPX_LAYOUT_SIZED])
def test_table_layout_matches_oracle(n, res, log2_T, cell, layout):
    """Rows, box extents and dense flags per level, computed by the library
    and by the oracle from the same reading of Sec. 5.2, agree exactly."""
    g = spx.spx_table_layout(spx.Encoding(n, res, log2_T, cell=cell, layout=layout))
    o = oracle.table_layout(oracle.Encoding(n, res, log2_T, cell=cell, layout=layout))
    assert g["rows"] == list(o["rows"]) and g["box_extent"] == list(o["extent"]) and g["dense"] == list(o["dense"])
    assert g["offsets"] == list(o["offsets"]) and g["total_rows"] == o["offsets"][-1]


@pytest.mark.parametrize("w", [inputs.IMAGE_2D, inputs.VOLUME_3D] + [inputs.sweep_workload(n) for n in range(2, 7)])
def test_sized_layout_of_the_workloads(w):
    res = spx.spx_level_resolutions(w.n_min, w.growth, w.n_levels)
    for cell in (spx.SPX_SIMPLEX, spx.SPX_GRID):
        g = spx.spx_table_layout(spx.Encoding(w.n_dims, res, w.log2_T, cell=cell, layout=spx.SPX_LAYOUT_SIZED))
        o = oracle.table_layout(oracle.Encoding(w.n_dims, res, w.log2_T, cell=cell, layout=oracle.SIZED))
        assert g["rows"] == list(o["rows"]) and g["dense"] == list(o["dense"])
        assert g["total_rows"] <= w.n_levels << w.log2_T


def test_layout_argument_checks():
    L = spx.lib()
    e = spx.Encoding(2, [16], 14)
    e._c.layout = 7
    assert L.spx_table_layout(e.ref(), None, None, None, None) == spx.SPX_EINVAL
    enc = spx.Encoding(2, [16] * 16, 14, layout=spx.SPX_LAYOUT_SIZED)
    f = spx.spx_field()
    fake = C.c_void_p(0x10000)
    assert L.spx_field_init(enc.ref(), fake, fake, fake, fake, 3, C.byref(f)) == spx.SPX_EUNSUPPORTED


def _status(fn, *args):
    return fn(*args)


def test_encode_argument_checks_on_host():
    L = spx.lib()
    good = spx.Encoding(3, [16, 32], 19)
    fake = C.c_void_p(0x10000)  # never dereferenced: every call below fails its checks first
    s = C.c_void_p(0)

    def fwd(enc, N=10, pts=fake, tab=fake, out=fake, odt=spx.SPX_F32):
        return L.spx_encode_fwd(enc.ref() if enc is not None else None, N, pts, tab, out, odt, s)

    assert fwd(None) == spx.SPX_EINVAL
    for bad in [dict(n_dims=0), dict(n_dims=7), dict(log2_T=0), dict(log2_T=27), dict(n_feat=3),
                dict(table_dtype=5), dict(cell=2)]:
        kw = dict(n_dims=3, res=[16, 32], log2_T=19)
        kw.update(bad)
        assert fwd(spx.Encoding(**kw)) == spx.SPX_EINVAL, bad
    assert fwd(spx.Encoding(3, [16, 0], 19)) == spx.SPX_EINVAL
    assert fwd(spx.Encoding(3, [], 19)) == spx.SPX_EINVAL
    assert fwd(spx.Encoding(3, list(range(1, 34)), 19)) == spx.SPX_EINVAL
    assert fwd(good, N=-1) == spx.SPX_EINVAL
    assert fwd(good, pts=None) == spx.SPX_EINVAL
    assert fwd(good, odt=7) == spx.SPX_EINVAL
    assert fwd(good, out=None) == spx.SPX_EINVAL
    assert fwd(good, pts=C.c_void_p(0x10002)) == spx.SPX_EALIGN
    assert fwd(good, tab=C.c_void_p(0x10002)) == spx.SPX_EALIGN       # f16 F=2 rows are 4 bytes
    assert fwd(good, out=C.c_void_p(0x10004)) == spx.SPX_EALIGN       # f32 F=2 rows are 8 bytes
    assert "aligned" in spx.spx_last_error()
    # N = 0 is a no-op that touches nothing
    assert fwd(good, N=0, pts=None, tab=None, out=None) == spx.SPX_OK
    assert L.spx_encode_bwd(good.ref(), 0, None, None, spx.SPX_F32, None, None, 0, s) == spx.SPX_OK
    assert L.spx_encode_bwd(good.ref(), 5, fake, fake, spx.SPX_F32, C.c_void_p(0x10001), None, 0, s) == spx.SPX_EALIGN
    need = spx.spx_encode_bwd_workspace(good, 5)
    assert need > 0
    assert L.spx_encode_bwd(good.ref(), 5, fake, fake, spx.SPX_F32, fake, fake, need - 1, s) == spx.SPX_EINVAL
    assert L.spx_encode_bwd(good.ref(), 5, fake, fake, spx.SPX_F32, fake, C.c_void_p(0x10010), need, s) \
        == spx.SPX_EALIGN
    assert L.spx_encode_debug(good.ref(), 5, fake, None, None, s) == spx.SPX_OK  # nothing requested
    # the adjoint split in two: the counting pass and the adjoints after it need the workspace
    ws = C.c_void_p(0x100000)
    assert L.spx_encode_bwd_prepare(good.ref(), 0, None, None, 0, s) == spx.SPX_OK
    assert L.spx_encode_bwd_prepare(good.ref(), -1, fake, ws, need, s) == spx.SPX_EINVAL
    assert L.spx_encode_bwd_prepare(good.ref(), 5, None, ws, need, s) == spx.SPX_EINVAL
    assert L.spx_encode_bwd_prepare(good.ref(), 5, fake, None, need, s) == spx.SPX_EINVAL
    assert L.spx_encode_bwd_prepare(good.ref(), 5, fake, ws, need - 1, s) == spx.SPX_EINVAL
    assert L.spx_encode_bwd_prepare(good.ref(), 5, fake, C.c_void_p(0x100010), need, s) == spx.SPX_EALIGN
    assert L.spx_encode_bwd_prepared(good.ref(), 5, fake, fake, spx.SPX_F32, fake, None, 0, s) == spx.SPX_EINVAL
    assert L.spx_encode_bwd_prepared(good.ref(), 5, fake, fake, spx.SPX_F32, fake, ws, need - 1, s) == spx.SPX_EINVAL
    adam = (C.c_float(1e-2), C.c_float(0.9), C.c_float(0.99), C.c_float(1e-15))
    assert L.spx_encode_bwd_adam_prepared(good.ref(), 5, fake, fake, spx.SPX_F32, ws, ws, ws, None, *adam, 1,
                                          None, 0, s) == spx.SPX_EINVAL
    assert L.spx_encode_bwd_adam_prepared(good.ref(), 5, fake, fake, spx.SPX_F32, ws, ws, ws, None, *adam, 0,
                                          ws, need, s) == spx.SPX_EINVAL  # step < 1


def test_other_argument_checks_on_host():
    L = spx.lib()
    fake = C.c_void_p(0x10000)
    s = C.c_void_p(0)
    assert L.spx_cast_f32_f16(-1, fake, fake, s) == spx.SPX_EINVAL
    assert L.spx_cast_f32_f16(0, None, None, s) == spx.SPX_OK
    assert L.spx_adam_step(4, fake, fake, fake, fake, None, 1e-2, 0.9, 0.99, 1e-15, 0, 0, s) == spx.SPX_EINVAL
    assert L.spx_adam_step(4, fake, fake, fake, fake, None, 1e-2, 1.0, 0.99, 1e-15, 1, 0, s) == spx.SPX_EINVAL
    m = spx.make_mlp(32, 64, 3)
    bad = spx.make_mlp(48, 64, 3)
    size = C.c_size_t(0)
    assert L.spx_mlp_bwd_workspace(C.byref(m), 1 << 20, C.byref(size)) == spx.SPX_OK and size.value > 0
    assert L.spx_mlp_fwd(C.byref(bad), 10, fake, fake, fake, fake, fake, s) == spx.SPX_EUNSUPPORTED
    assert L.spx_mlp_fwd(C.byref(spx.make_mlp(32, 64, 17)), 10, fake, fake, fake, fake, fake, s) == spx.SPX_EINVAL
    assert L.spx_mlp_fwd(C.byref(m), 10, C.c_void_p(0x10008), fake, fake, fake, fake, s) == spx.SPX_EALIGN
    assert L.spx_mlp_bwd(C.byref(m), 10, fake, fake, fake, fake, fake, None, fake, fake, fake, fake, 16, s) \
        == spx.SPX_EINVAL  # workspace too small


def test_binned_workspace_sizes():
    """The binned adjoint's workspace: records for every contribution plus
    counters; bigger for more points and more vertices."""
    e2 = spx.Encoding(2, [16] * 16, 22)
    a = spx.spx_encode_bwd_workspace(e2, 1 << 20)
    assert a >= (1 << 20) * 16 * 3 * 12  # one 12-byte record (F = 2) per (point, level, vertex)
    assert spx.spx_encode_bwd_workspace(e2, 1 << 10) < a
    g3 = spx.Encoding(3, [16] * 16, 19, cell=spx.SPX_GRID)
    s3 = spx.Encoding(3, [16] * 16, 19)
    assert spx.spx_encode_bwd_workspace(g3, 1 << 16) > spx.spx_encode_bwd_workspace(s3, 1 << 16)
    # the largest table still bins (one level per group)
    assert spx.spx_encode_bwd_workspace(spx.Encoding(6, [16] * 32, 26, n_feat=8), 1 << 16) > 0


def test_fused_network_backward_coverage_on_host():
    """spx_encode_mlp_bwd_workspace / _adam decide on the host, before any
    launch, which configurations the fused network backward covers."""
    L = spx.lib()
    fake = C.c_void_p(0x10000)
    s = C.c_void_p(0)
    mlp = spx.make_mlp(32, 64, 3)
    res16 = spx.spx_level_resolutions(16, 1.38, 16)
    image = spx.Encoding(2, res16, 19, 2, table_dtype=spx.SPX_F16)
    volume = spx.Encoding(3, spx.spx_level_resolutions(16, 1.32, 16), 19, 2, table_dtype=spx.SPX_F16)
    for enc, N in [(image, 1 << 20), (volume, 1 << 21), (image, 0), (image, 1)]:
        # the unfused workspaces plus N rows of the privatised levels' units
        need = spx.spx_encode_mlp_bwd_workspace(enc, mlp, N)
        assert need >= spx.spx_encode_bwd_workspace(enc, N) + spx.spx_mlp_bwd_workspace(mlp, N)
    out = C.c_size_t(0)

    def ws(enc, m=mlp, N=1000):
        return L.spx_encode_mlp_bwd_workspace(enc.ref(), C.byref(m), N, C.byref(out))

    assert ws(spx.Encoding(4, res16, 14, 2)) == spx.SPX_EUNSUPPORTED                    # n > 3
    assert ws(spx.Encoding(2, res16[:8], 14, 4)) == spx.SPX_EUNSUPPORTED                # n_feat 4
    assert ws(spx.Encoding(2, res16[:12], 14, 2)) == spx.SPX_EINVAL                     # d_in != L * F
    assert ws(image, spx.make_mlp(32, 32, 3)) == spx.SPX_EUNSUPPORTED                   # hidden 32
    # more buckets than one level group holds (2^26 rows per level, 16 levels)
    assert ws(spx.Encoding(2, res16, 26, 2)) == spx.SPX_EUNSUPPORTED
    assert "level group" in spx.spx_last_error()
    need = spx.spx_encode_mlp_bwd_workspace(image, mlp, 1000)

    def fused(enc=image, N=1000, nbytes=need, wsp=fake, step=1, param=fake):
        return L.spx_encode_mlp_bwd_adam(enc.ref(), C.byref(mlp), N, fake, fake, fake, fake, fake, fake, fake, fake,
                                         fake, param, fake, fake, None, 1e-2, 0.9, 0.99, 1e-15, step, wsp, nbytes, s)

    assert fused(nbytes=need - 1) == spx.SPX_EINVAL
    assert fused(wsp=C.c_void_p(0x10010)) == spx.SPX_EALIGN
    assert fused(step=0) == spx.SPX_EINVAL
    assert fused(param=C.c_void_p(0x10004)) == spx.SPX_EALIGN
    assert fused(enc=spx.Encoding(4, res16, 14, 2)) == spx.SPX_EUNSUPPORTED
