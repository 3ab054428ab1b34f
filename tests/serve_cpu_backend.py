"""A CPU stand-in for the GPU serving backend, for scheduler tests: device
memory is a numpy byte array, a batch is computed with the oracle (encoding
to binary16 features, then the network), and completion times, launch
failures and peak arena use are controlled or recorded by the test."""
import time

import numpy as np

import oracle


class CpuBackend:
    def __init__(self, fields, latency=0.0, fail_launches=()):
        self.fields = fields            # list of dict(enc, tables, W1, W2, W3, d_out)
        self.latency = latency
        self.fail_launches = set(fail_launches)
        self.launches = 0
        self.batches = []               # list of [(field, count)] per launch

    def alloc_arena(self, nbytes):
        self.mem = np.zeros(nbytes, np.uint8)
        self.used = np.zeros(nbytes, bool)
        self.peak = 0

    def upload(self, off, pts):
        b = pts.view(np.uint8).reshape(-1)
        self.mem[off:off + b.size] = b
        return ("t", time.perf_counter())

    def launch(self, items):
        k = self.launches
        self.launches += 1
        if k in self.fail_launches:
            raise RuntimeError(f"injected failure of launch {k}")
        self.batches.append([(f, m) for f, _, _, m in items])
        for f, in_off, out_off, m in items:
            fd = self.fields[f]
            n = fd["enc"].n_dims
            pts = self.mem[in_off:in_off + m * n * 4].view(np.float32).reshape(m, n)
            feats = oracle.encode_fwd(fd["enc"], pts, fd["tables"]).astype(np.float16)
            y = oracle.mlp_fwd(feats, fd["W1"], fd["W2"], fd["W3"]).astype(np.float32)
            self.mem[out_off:out_off + y.nbytes] = y.view(np.uint8).reshape(-1)
        return ("t", time.perf_counter() + self.latency)

    def download(self, off, shape, after):
        return ("d", after[1], off, shape)

    def done(self, h):
        return time.perf_counter() >= h[1]

    def result(self, h):
        _, _, off, shape = h
        n = int(np.prod(shape)) * 4
        return self.mem[off:off + n].view(np.float32).reshape(shape).copy()
