"""Scheduler of the query server on the CPU (no GPU): results, chunking of
large requests, memory admission and back-pressure, mixing of fields in a
batch, and failure handling forced from the host."""
import time

import numpy as np
import pytest

import oracle
from paper_2311_15439_amd import inputs
from paper_2311_15439_amd.serve import Arena, RequestError, Server
from serve_cpu_backend import CpuBackend


def _fields(k=3):
    out = []
    for i in range(k):
        n = 3 if i % 2 == 0 else 2
        res = list(oracle.level_resolutions(16, 1.38, 16))
        enc = oracle.Encoding(n, res, 12, 2, table_dtype=oracle.F16)
        tables = inputs.tables(16, 1 << 12, 2, 0.5, 10 + i, True).view(np.uint16)
        W1, W2, W3 = inputs.mlp_weights(32, 64, 4, 20 + i)
        out.append(dict(enc=enc, tables=tables, W1=W1, W2=W2, W3=W3, d_out=4))
    return out


def _reference(fd, pts):
    feats = oracle.encode_fwd(fd["enc"], pts, fd["tables"]).astype(np.float16)
    return oracle.mlp_fwd(feats, fd["W1"], fd["W2"], fd["W3"]).astype(np.float32)


def _server(fields, **kw):
    be = CpuBackend(fields, latency=kw.pop("latency", 0.0), fail_launches=kw.pop("fail", ()))
    srv = Server(be, [f["enc"].n_dims for f in fields], [f["d_out"] for f in fields], **kw).start()
    return srv, be


def test_arena_first_fit_and_coalescing():
    a = Arena(4096)
    x = a.alloc(1000)
    y = a.alloc(1000)
    z = a.alloc(1000)
    assert (x, y, z) == (0, 1024, 2048)
    assert a.alloc(2000) is None
    a.release(y, 1000)
    assert a.alloc(1024) == 1024
    a.release(x, 1000)
    a.release(1024, 1024)
    a.release(z, 1000)
    assert a.free == [(0, 4096)]


def test_results_match_oracle_with_chunking_and_mixing():
    fields = _fields()
    srv, be = _server(fields, arena_bytes=1 << 22, chunk_points=500, batch_points=2000)
    try:
        reqs = []
        rng = np.random.default_rng(0)
        for i in range(12):
            f = int(rng.integers(0, len(fields)))
            m = int(rng.integers(1, 1700))
            pts = inputs.uniform_points(m, fields[f]["enc"].n_dims, 100 + i)
            reqs.append((f, pts, srv.submit(f, pts)))
        empty = srv.submit(0, np.zeros((0, 3), np.float32))
        for f, pts, r in reqs:
            np.testing.assert_array_equal(r.wait(30), _reference(fields[f], pts))
            assert r.latency is not None and r.latency >= 0
        assert empty.wait(1).shape == (0, 4)
        assert any(len({f for f, _ in b}) > 1 for b in be.batches)  # fields mixed in a batch
        assert max(sum(m for _, m in b) for b in be.batches) <= 2000
    finally:
        srv.stop()
    assert srv.arena.free == [(0, 1 << 22)]


def test_memory_admission_and_back_pressure():
    """An arena that holds only two chunks at a time still serves a burst of
    requests; the scheduler never over-commits it."""
    fields = _fields(1)
    chunk = 256
    per_chunk = ((chunk * 3 * 4 + 255) // 256) * 256 + chunk * 4 * 4
    srv, be = _server(fields, arena_bytes=2 * ((per_chunk + 255) // 256 * 256), chunk_points=chunk,
                      batch_points=4096, latency=0.002)
    try:
        reqs = []
        for i in range(10):
            pts = inputs.uniform_points(700, 3, i)
            reqs.append((pts, srv.submit(0, pts)))
        for pts, r in reqs:
            np.testing.assert_array_equal(r.wait(30), _reference(fields[0], pts))
        assert max(sum(m for _, m in b) for b in be.batches) <= 2 * chunk
    finally:
        srv.stop()
    assert srv.arena.free_bytes == srv.arena.capacity


def test_failures_are_contained():
    """An unknown field fails only its request; an injected launch failure
    fails the requests of that batch; a request that cannot get memory
    before its deadline times out; everything else completes and the arena
    is fully released."""
    fields = _fields(2)
    srv, be = _server(fields, arena_bytes=1 << 20, chunk_points=300, batch_points=300, fail=(1,))
    try:
        bad = srv.submit(7, np.zeros((5, 3), np.float32))
        with pytest.raises(RequestError, match="unknown field"):
            bad.wait(1)
        reqs = [srv.submit(0, inputs.uniform_points(300, 3, i)) for i in range(4)]
        outcomes = []
        for r in reqs:
            try:
                r.wait(30)
                outcomes.append("ok")
            except RequestError as e:
                assert "injected failure" in str(e)
                outcomes.append("failed")
        assert outcomes.count("failed") == 1 and outcomes.count("ok") == 3
        with pytest.raises(ValueError):
            srv.submit(0, np.zeros((5, 2), np.float32))  # wrong dimension for the field
    finally:
        srv.stop()
    assert srv.arena.free_bytes == srv.arena.capacity
    # a request larger than memory allows can only time out while it waits
    srv2, _ = _server(fields, arena_bytes=4096, chunk_points=1 << 20)
    try:
        r = srv2.submit(0, inputs.uniform_points(5000, 3, 1), timeout=0.05)
        with pytest.raises(RequestError, match="arena|timed out"):
            r.wait(5)
    finally:
        srv2.stop()


def test_result_alone_equals_result_in_mix():
    fields = _fields(3)
    pts = inputs.uniform_points(999, 3, 42)
    srv, _ = _server(fields, arena_bytes=1 << 22, chunk_points=256, batch_points=3000)
    try:
        alone = srv.submit(0, pts).wait(30)
        noise = [srv.submit(i % 3, inputs.uniform_points(300 + 7 * i, fields[i % 3]["enc"].n_dims, i)) for i in range(6)]
        mixed = srv.submit(0, pts)
        more = [srv.submit(i % 3, inputs.uniform_points(200, fields[i % 3]["enc"].n_dims, 50 + i)) for i in range(4)]
        np.testing.assert_array_equal(mixed.wait(30), alone)
        for r in noise + more:
            r.wait(30)
    finally:
        srv.stop()
