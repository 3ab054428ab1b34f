#!/usr/bin/env python3
"""Benchmark: one training step of the multiresolution simplex hash encoding
on the image-fitting workload (n=2, L=16, T=2^22, F=2 binary16 tables,
resolutions 16..32768, 2^20 random pixel positions of a 16384^2 image per
step, MLP 32->64->64->3).

A step is the whole hot path on one batch already resident in GPU memory:
  encode forward -> MLP forward -> L2 loss gradient -> MLP backward ->
  encode adjoint -> Adam on the tables (binary32 master + binary16 copy,
  gradient cleared) -> Adam on the MLP weights.
The same step with the 2^n-corner grid baseline, the encoding kernels alone
(simplex and grid, with their fraction of the measured random-gather
ceiling), the volume workload, serving, and the CPU oracle on a bounded
sample are reported beside it.  The full record goes to a JSON file
(--detail-out); stdout ends with a few '#' summary lines and one compact
JSON line (under 4 KB) carrying the headline figures.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W]
"""
from __future__ import annotations

import argparse
import gc
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X published HBM3E bandwidth
LINE_BYTES = 128  # cache line of gfx950's vector L1 and L2
# one 64-byte HBM access per random gather: the theoretical random-gather rate
HBM_RANDOM_GATHERS_PER_S = HBM_PEAK_GBS * 1e9 / 64.0
DETAIL_DEFAULT = os.path.join("results", "bench_detail.json")  # the full record beside the one-line summary


def expected_unique(M, k):
    """Expected number of distinct items among k uniform draws from M."""
    M = float(M)
    return -M * np.expm1(k * np.log1p(-1.0 / M)) if M > 1 else 1.0


def wave_unique_lines(idx, log2_T, row_bytes, wave=64):
    """Mean number of distinct cache lines one wave (`wave` consecutive
    points) touches at each level, over all its vertices: idx [N, L, V]
    slots in launch order.  Lines shared by lanes or by the vertices of one
    lane count once (an optimistic count for the kernel)."""
    N, L, V = idx.shape
    W = N // wave
    a = idx[:W * wave].astype(np.int64).reshape(W, wave, L, V).transpose(0, 2, 1, 3).reshape(W, L, wave * V)
    lines = np.sort((a * row_bytes) // LINE_BYTES, axis=2)
    uniq = 1 + np.count_nonzero(np.diff(lines, axis=2), axis=2)
    return uniq.mean(axis=0)


def level_footprints(sigma, reach, n, log2_T, row_bytes, simplex):
    """Bytes of whole cache lines each level can touch: the lattice box the
    unit cube reaches (extent floor(sigma * reach) + 2 per axis), its
    vertices hashed uniformly over the level's T rows."""
    T = 1 << log2_T
    M_tot = max(1.0, T * row_bytes / LINE_BYTES)
    out = []
    for s in sigma:
        box = (np.floor(float(s) * reach) + 2.0) ** n
        out.append(LINE_BYTES * expected_unique(M_tot, min(box, float(T))))
    return out


def line_rate(probe, nbytes):
    """Measured random-gather rate at a buffer of nbytes, in distinct line
    requests per second: the probe's gathers/s (log-linear interpolation
    between its power-of-two sizes, clamped to its range) times the
    fraction of a wave's 64 gathers that fall on distinct lines."""
    sizes = np.array(sorted(probe), dtype=np.float64)
    rates = np.array([probe[int(k)] for k in sizes])
    x = np.clip(np.log2(max(nbytes, 1.0)), np.log2(sizes[0]), np.log2(sizes[-1]))
    g = float(np.interp(x, np.log2(sizes), rates))
    M = 2.0 ** x / LINE_BYTES
    return g * expected_unique(M, 64) / 64.0


def gather_ceiling_ms(N, unique_per_wave, footprints, probe, wave=64):
    """Time the memory system needs for one pass of the encoding's gathers
    at the measured random-gather rates: per level, the waves' distinct
    line requests at that level's footprint."""
    waves = N / wave
    return 1e3 * sum(waves * u / line_rate(probe, f) for u, f in zip(unique_per_wave, footprints))


COPY_ELEMS = 1 << 26  # calibration copy: 256 MiB read, 128 MiB written
# per workload: the traffic file of its dominant kernel ({} -> image2d / volume3d)
TRAFFIC_FILE = os.path.join("profiles", "bin_accum_adam_{}_traffic.json")


def _traffic_path(workload):
    tag = "volume3d" if workload.startswith("volume") else "image2d"
    return os.path.join(ROOT, TRAFFIC_FILE.format(tag))
# kernels whose counters the traffic file holds, and the sources that define them
TRAFFIC_KERNELS = {"bin_accum_adam": ("bin_accum_kernel", "true")}
TRAFFIC_SOURCES = ["paper_2311_15439_amd/csrc/binned_accum.hpp", "paper_2311_15439_amd/csrc/spx_internal.h",
                   "paper_2311_15439_amd/csrc/encode_kernels.hpp", "paper_2311_15439_amd/csrc/lookup.hpp",
                   "paper_2311_15439_amd/csrc/wave_runs.hpp"]


def _sources_digest():
    import hashlib
    h = hashlib.sha256()
    for f in TRAFFIC_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


# Read bytes per dispatch from the L2's read requests to memory, by request
# size.  (rocprofv3's derived FETCH_SIZE takes the 128-byte requests from
# TCC_BUBBLE, which reads 0 on gfx950, and so counts each 128-byte line fill
# as 64 bytes: half of a streaming kernel's reads.)
READ_COUNTERS = {"TCC_EA0_RDREQ_128B_sum": 128.0, "TCC_EA0_RDREQ_64B_sum": 64.0, "TCC_EA0_RDREQ_32B_sum": 32.0}


def _counter_rows(path):
    """{(dispatch id, kernel name): {counter: value}} of a rocprofv3 --pmc CSV."""
    import csv
    out = {}
    with open(path, newline="") as fh:
        for r in csv.DictReader(fh):
            out.setdefault((int(r["Dispatch_Id"]), r["Kernel_Name"]), {})[r["Counter_Name"]] = float(r["Counter_Value"])
    return out


def write_traffic(read_csv, write_csv, workload):
    """HBM bytes per launch of the dominant kernel from two counter runs of
    `--pmc-pass` on `workload`: bytes read from the read requests by size
    (READ_COUNTERS), bytes written from WRITE_SIZE (KiB).  The calibration
    copy of known size (the last cast kernel dispatch) is reported beside
    them as a check of both."""
    res = {"sources_sha256": _sources_digest(), "workload": workload, "copy_elems": COPY_ELEMS, "kernels": {}}
    reads = sorted(_counter_rows(read_csv).items())
    writes = sorted(_counter_rows(write_csv).items())

    def read_bytes(c):
        return sum(c.get(k, 0.0) * b for k, b in READ_COUNTERS.items())

    copy_r = [read_bytes(c) for (_, k), c in reads if "cast_kernel" in k][-1]
    copy_w = [c["WRITE_SIZE"] * 1024.0 for (_, k), c in writes if "cast_kernel" in k][-1]
    res["copy_check"] = {"read_bytes": copy_r, "read_expected": COPY_ELEMS * 4.0,
                         "written_bytes": copy_w, "written_expected": COPY_ELEMS * 2.0}
    for name, (sym, tmpl) in TRAFFIC_KERNELS.items():
        def mine(k):
            return sym in k and tmpl in k.split(sym, 1)[1]
        r = [read_bytes(c) for (_, k), c in reads if mine(k)][-1]
        w = [c["WRITE_SIZE"] * 1024.0 for (_, k), c in writes if mine(k)][-1]
        res["kernels"][name] = {"read_bytes": r, "written_bytes": w, "bytes": r + w}
    with open(_traffic_path(workload), "w") as fh:
        json.dump(res, fh, indent=1)
    print(json.dumps(res))


def measured_traffic(kernel, workload):
    """HBM bytes per launch measured by the counter runs, or None if there is
    no measurement for this kernel on this workload or its sources changed
    since it was taken."""
    try:
        with open(_traffic_path(workload)) as fh:
            t = json.load(fh)
    except OSError:
        return None
    if (t.get("sources_sha256") != _sources_digest() or t.get("workload") != workload
            or kernel not in t.get("kernels", {})):
        return None
    return t["kernels"][kernel]["bytes"]


def _workload(name):
    from paper_2311_15439_amd import inputs
    return {"image-2d": inputs.IMAGE_2D, "volume-3d": inputs.VOLUME_3D}[name]


def _points(w, batch):
    from paper_2311_15439_amd import inputs
    if w.name.startswith("image"):
        return inputs.pixel_points(w.n_points, w.seed_points + 1000 * batch)
    if w.name.startswith("field"):
        return inputs.uniform_points(w.n_points, w.n_dims, w.seed_points + 1000 * batch)
    return inputs.ray_points(w.n_points // 256, 256, w.seed_points + 1000 * batch)


def _targets(w, pts, batch):
    from paper_2311_15439_amd import inputs
    if w.name.startswith("image"):
        return inputs.procedural_rgb(pts, 4)
    if w.name.startswith("field"):
        return inputs.procedural_nd(pts, 60 + w.n_dims)
    return inputs.procedural_density(pts, 7)


def _colour_target(w):
    """Targets that are colours in [0, 1] (PSNR against peak 1, outputs
    clamped), as opposed to the volume's density and colour."""
    return w.name.startswith("image") or w.name.startswith("field")


_SIDE_STREAM = None


def side_stream():
    """The one second stream (default priority) every step and timing here
    uses beside the caller's stream.  Streams share the device's few hardware
    queues round-robin, so a stream created later may land on the same queue
    as the caller's stream and run serialised behind it; reusing the first
    one keeps the two apart for the whole run."""
    global _SIDE_STREAM
    if _SIDE_STREAM is None:
        import torch
        _SIDE_STREAM = torch.cuda.Stream()
    return _SIDE_STREAM


class TrainStep:
    """All device buffers of one training step; launches only library kernels."""

    def __init__(self, w, cell, batches, host_tables, weights, d_out, fused=True, equal_memory=False, layout=0,
                 fused_bwd=False):
        import torch
        from paper_2311_15439_amd import spx
        self.torch, self.spx = torch, spx
        dev = "cuda"
        self.w = w
        self.res = spx.spx_level_resolutions(w.n_min, w.growth, w.n_levels)
        self.enc = spx.Encoding(w.n_dims, self.res, w.log2_T, w.n_feat, table_dtype=spx.SPX_F16, cell=cell,
                                equal_memory=equal_memory, layout=layout)
        if tuple(host_tables.shape) != self.enc.table_shape:
            # another table layout: the same initial distribution over its rows
            host_tables = np.random.default_rng(w.seed_tables).uniform(
                -w.table_init, w.table_init, self.enc.table_shape).astype(np.float32)
        self.N = w.n_points
        self.batches = [(torch.from_numpy(p).to(dev), torch.from_numpy(t).to(dev)) for p, t in batches]
        self.master = torch.from_numpy(host_tables.astype(np.float32)).to(dev)
        self.tab16 = torch.from_numpy(host_tables.astype(np.float16)).to(dev)
        self.grad = torch.zeros_like(self.master)
        self.m = torch.zeros_like(self.master)
        self.v = torch.zeros_like(self.master)
        D = w.n_levels * w.n_feat
        self.d_out = d_out
        self.mlp = spx.make_mlp(D, 64, d_out)
        W1, W2, W3 = weights
        sizes = [W1.size, W2.size, W3.size]
        flat = np.concatenate([W1.ravel(), W2.ravel(), W3.ravel()])
        self.W16 = torch.from_numpy(flat.astype(np.float16)).to(dev)
        self.Wm = torch.from_numpy(flat.astype(np.float32)).to(dev)
        self.dW = torch.zeros_like(self.Wm)
        self.Wmm = torch.zeros_like(self.Wm)
        self.Wvv = torch.zeros_like(self.Wm)
        o = np.cumsum([0] + sizes)
        shapes = [W1.shape, W2.shape, W3.shape]
        self.Wv = [self.W16[o[i]:o[i + 1]].view(*shapes[i]) for i in range(3)]
        self.dWv = [self.dW[o[i]:o[i + 1]].view(*shapes[i]) for i in range(3)]
        self.feats = torch.empty((self.N, D), dtype=torch.float16, device=dev)
        self.y = torch.empty((self.N, d_out), dtype=torch.float32, device=dev)
        self.dy = torch.empty_like(self.y)
        self.dfeats = torch.empty((self.N, D), dtype=torch.float32, device=dev)
        self.ws = torch.empty(spx.spx_mlp_bwd_workspace(self.mlp, self.N), dtype=torch.uint8, device=dev)
        self.bws = torch.empty(spx.spx_encode_bwd_workspace(self.enc, self.N), dtype=torch.uint8, device=dev)
        self.t = 0
        self.lr = 1e-2
        self.fused = fused
        # the fused encoding + network forward covers 2-/3-D fields of 16 levels x 2 features, hashed tables
        self.fused_fwd = w.n_dims in (2, 3) and D == 32 and w.n_feat == 2 and layout == spx.SPX_LAYOUT_HASHED
        # the network backward inside the adjoint's scatter (with the tables' Adam step)
        self.fused_bwd = fused_bwd and fused
        # the adjoint's counting pass (it needs only the points) on a second
        # stream beside the forward and the network, joined by an event
        # before the adjoint (spx_encode_bwd_prepare, then the *_prepared call)
        self.prepare = fused and not self.fused_bwd
        if self.prepare:
            self.side = side_stream()
            self.ev_fork, self.ev_join = torch.cuda.Event(), torch.cuda.Event()
            # the network's Adam step also runs there, beside the adjoint
            self.ev_mlp, self.ev_adam = torch.cuda.Event(), torch.cuda.Event()
        if self.fused_bwd:
            self.nws = torch.empty(spx.spx_encode_mlp_bwd_workspace(self.enc, self.mlp, self.N), dtype=torch.uint8,
                                   device=dev)

    @property
    def names(self):
        return [n for n, _ in self._calls(0)]

    def _calls(self, b):
        """The step's library calls in order, as (name, thunk)."""
        spx = self.spx
        pts, tgt = self.batches[b % len(self.batches)]
        calls = []
        if self.prepare:
            def fork():
                import torch
                # the side stream starts after everything issued so far (the
                # previous step's adjoint still reads the workspace)
                self.ev_fork.record(torch.cuda.current_stream())
                self.side.wait_event(self.ev_fork)
                spx.spx_encode_bwd_prepare(self.enc, pts, self.bws, stream=self.side)
                self.ev_join.record(self.side)
            calls.append(("encode_bwd_prepare", fork))
        if self.fused_fwd:
            calls.append(("encode_mlp_fwd", lambda: spx.spx_encode_mlp_fwd(self.enc, self.mlp, pts, self.tab16, *self.Wv,
                                                                           self.y, feats=self.feats)))
        else:
            calls.append(("encode_fwd", lambda: spx.spx_encode_fwd(self.enc, pts, self.tab16, self.feats)))
            calls.append(("mlp_fwd", lambda: spx.spx_mlp_fwd(self.mlp, self.feats, *self.Wv, self.y)))
        calls += self._loss_calls(b, tgt)
        if self.fused_bwd:
            calls.append(("encode_mlp_bwd_adam", lambda: spx.spx_encode_mlp_bwd_adam(
                self.enc, self.mlp, pts, self.feats, *self.Wv, self.dy, *self.dWv, self.master, self.m, self.v,
                self.tab16, lr=self.lr, beta1=0.9, beta2=0.99, eps=1e-15, step=self.t, workspace=self.nws)))
        else:
            calls.append(("mlp_bwd", lambda: spx.spx_mlp_bwd(self.mlp, self.feats, *self.Wv, self.dy, self.dfeats,
                                                             *self.dWv, self.ws)))
        if self.fused_bwd:
            pass
        elif self.fused:
            # adjoint and Adam on the tables in one pass (no gradient table),
            # after the counting pass on the side stream
            def bwd_adam():
                import torch
                torch.cuda.current_stream().wait_event(self.ev_join)
                spx.spx_encode_bwd_adam_prepared(
                    self.enc, pts, self.dfeats, self.master, self.m, self.v, self.tab16, lr=self.lr, beta1=0.9,
                    beta2=0.99, eps=1e-15, step=self.t, workspace=self.bws)
            calls.append(("encode_bwd_adam", bwd_adam))
        else:
            calls.append(("encode_bwd", lambda: spx.spx_encode_bwd(self.enc, pts, self.dfeats, self.grad, self.bws)))
            calls.append(("adam_tables", lambda: spx.spx_adam_step(
                self.master, self.grad, self.m, self.v, self.tab16, lr=self.lr, beta1=0.9, beta2=0.99, eps=1e-15,
                step=self.t, zero_grad=True)))
        def adam_mlp(stream=None):
            spx.spx_adam_step(self.Wm, self.dW, self.Wmm, self.Wvv, self.W16, lr=self.lr, beta1=0.9, beta2=0.99,
                              eps=1e-15, step=self.t, zero_grad=False, stream=stream)
        if self.prepare:
            # the network's Adam step on the side stream as soon as its
            # gradient is reduced, beside the adjoint; the caller's stream
            # waits for it at the end of the step (the next forward reads
            # the weights)
            def adam_side():
                import torch
                self.ev_mlp.record(torch.cuda.current_stream())
                self.side.wait_event(self.ev_mlp)
                adam_mlp(self.side)
                self.ev_adam.record(self.side)
            k = next(i for i, (nm, _) in enumerate(calls) if nm == "mlp_bwd") + 1
            calls.insert(k, ("adam_mlp", adam_side))
            calls.append(("join", lambda: self.torch.cuda.current_stream().wait_event(self.ev_adam)))
        else:
            calls.append(("adam_mlp", adam_mlp))
        return calls

    def _loss_calls(self, b, tgt):
        spx = self.spx
        return [("mse_grad", lambda: spx.spx_mse_grad(self.y, tgt, self.dy, 2.0 / (self.N * self.d_out)))]

    def step(self, b, ev=None):
        self.t += 1
        calls = self._calls(b)
        for i, (_, fn) in enumerate(calls):
            if ev is not None:
                ev[i].record()
            fn()
        if ev is not None:
            ev[len(calls)].record()

    def algorithmic_bytes(self):
        """Bytes each kernel must move per launch (what the method reads and
        writes, once each)."""
        w, N = self.w, self.N
        n, L, F = w.n_dims, w.n_levels, w.n_feat
        V = (1 << n) if self.enc.cell == self.spx.SPX_GRID else n + 1
        P = L * (1 << w.log2_T) * F
        nw = self.Wm.numel()
        D = L * F
        return {
            "encode_bwd_prepare": 0,  # its kernels run on the side stream and are listed by name
            "encode_fwd": N * (4 * n + L * V * F * 2 + D * 2),
            "encode_mlp_fwd": N * (4 * n + L * V * F * 2 + D * 2 + 4 * self.d_out),
            "mlp_fwd": N * (2 * D + 4 * self.d_out),
            "mse_grad": N * self.d_out * 12,
            "mlp_bwd": N * (2 * D + 4 * self.d_out + 4 * D),
            # adjoint: points and output gradient in, one binary32 read-modify-write of
            # every touched slot per contribution (the scatter the method defines)
            "encode_bwd": N * (4 * n + 4 * D + L * V * F * 8),
            # fused: the adjoint's inputs plus the dense Adam update's 26 bytes per
            # parameter (read param, m, v; write param, m, v, binary16 copy)
            "encode_bwd_adam": N * (4 * n + 4 * D + L * V * F * 8) + P * 26,
            # network backward inside the adjoint: features and network output
            # gradient in (no input gradient stored), the scatter and the Adam update
            "encode_mlp_bwd_adam": N * (4 * n + 2 * D + 4 * self.d_out + L * V * F * 8) + P * 26,
            "adam_tables": P * 34 if not self.fused else 0,
            "adam_mlp": nw * 34,
            "join": 0,
        }


class RenderStep(TrainStep):
    """Volume-rendering training step: the rays' samples are encoded, the
    network gives (density, colour) per sample, the samples are composited
    along each ray (Eq. 5 quadrature) and the loss is on the rays' colours
    and opacities; its gradient flows back through the compositing, the
    network and the encoding."""

    def __init__(self, w, cell, batches, host_tables, weights, n_samples, equal_memory=False):
        # batches: (points [R*S, 3], delta [R*S], target rgba [R, 4])
        import torch
        super().__init__(w, cell, [(p, t) for p, _, t in batches], host_tables, weights, 4,
                         equal_memory=equal_memory)
        self.S = n_samples
        self.R = self.N // n_samples
        self.deltas = [torch.from_numpy(d.reshape(self.R, self.S)).to("cuda") for _, d, _ in batches]
        self.rgba = torch.empty((self.R, 4), dtype=torch.float32, device="cuda")
        self.drgba = torch.empty_like(self.rgba)

    def _loss_calls(self, b, tgt):
        spx = self.spx
        delta = self.deltas[b % len(self.deltas)]
        raw = self.y.view(self.R, self.S, 4)
        return [("composite_fwd", lambda: spx.spx_composite_fwd(raw, delta, self.rgba)),
                ("mse_grad", lambda: spx.spx_mse_grad(self.rgba, tgt, self.drgba, 2.0 / (self.R * 4))),
                ("composite_bwd", lambda: spx.spx_composite_bwd(raw, delta, self.drgba, self.dy.view(self.R, self.S, 4)))]


def _render_batch(w, b, n_samples):
    """Ray samples, their segment lengths, and the target colour and opacity
    of each ray: the procedural density field rendered along the same rays
    (its density and colour mapped through the inverse activations and
    composited by the library, once, at set-up)."""
    import torch
    from paper_2311_15439_amd import inputs, spx
    R = w.n_points // n_samples
    p = inputs.ray_points(R, n_samples, w.seed_points + 1000 * b)
    pr = p.reshape(R, n_samples, 3).astype(np.float64)
    seg = np.linalg.norm(np.diff(pr, axis=1), axis=2)
    delta = np.concatenate([seg, seg[:, -1:]], axis=1).astype(np.float32)
    field = inputs.procedural_density(p, 7).reshape(R, n_samples, 4).astype(np.float64)
    raw = np.empty_like(field)
    raw[..., 0] = np.log(np.expm1(np.maximum(field[..., 0], 1e-6)))       # softplus^-1
    c = np.clip(field[..., 1:], 1e-4, 1 - 1e-4)
    raw[..., 1:] = np.log(c / (1.0 - c))                                   # sigmoid^-1
    traw = torch.from_numpy(raw.astype(np.float32)).cuda()
    rgba = torch.empty((R, 4), dtype=torch.float32, device="cuda")
    spx.spx_composite_fwd(traw, torch.from_numpy(delta).cuda(), rgba)
    return p, delta.reshape(-1), rgba.cpu().numpy()


def render_bench(steps=10, warmup=3, train_steps=1000):
    """The volume workload as a rendering task (NeRF-style): training step
    simplex vs grid, and held-out PSNR of the rendered rays after
    train_steps steps (step size decaying 1e-2 -> 1e-3)."""
    import torch
    from paper_2311_15439_amd import inputs, spx
    w = inputs.VOLUME_3D
    S = 256
    print("# rendering: generating rays and targets", file=sys.stderr, flush=True)
    host_tables = inputs.tables(w.n_levels, 1 << w.log2_T, w.n_feat, w.table_init, w.seed_tables, False)
    weights = inputs.mlp_weights(w.n_levels * w.n_feat, 64, 4, 9)
    batches = [_render_batch(w, b, S) for b in range(3)]
    held = batches.pop()
    out = {"workload": f"{w.name}, {w.n_points // S} rays x {S} samples per step, MLP 32-64-64-4, "
                       "loss on composited ray colour and opacity"}
    for cell, name in ((spx.SPX_SIMPLEX, "simplex"), (spx.SPX_GRID, "grid")):
        print(f"# rendering: {name} step", file=sys.stderr, flush=True)
        rs = RenderStep(w, cell, batches, host_tables, weights, S)
        ms, per, _, kern = time_steps(rs, steps, warmup)
        for i in range(train_steps):
            rs.lr = 1e-2 * 0.1 ** (i / train_steps)
            rs.step(i)
        hp = torch.from_numpy(held[0]).cuda()
        spx.spx_encode_fwd(rs.enc, hp, rs.tab16, rs.feats)
        spx.spx_mlp_fwd(rs.mlp, rs.feats, *rs.Wv, rs.y)
        spx.spx_composite_fwd(rs.y.view(rs.R, S, 4), torch.from_numpy(held[1].reshape(rs.R, S)).cuda(), rs.rgba)
        mse = torch.mean((rs.rgba - torch.from_numpy(held[2]).cuda()) ** 2).item()
        out[name] = {"ms_per_step": ms, "samples_per_s": rs.N / (ms * 1e-3), "rays_per_s": rs.R / (ms * 1e-3),
                     "kernels_ms": {k: round(v["avg_ms"] * v["launches_per_step"], 5) for k, v in kern.items()},
                     "heldout_psnr_db": 10.0 * np.log10(1.0 / mse), "train_steps": train_steps}
        del rs
        torch.cuda.empty_cache()
    out["simplex_speedup"] = out["grid"]["ms_per_step"] / out["simplex"]["ms_per_step"]
    return out


def time_steps(ts, steps, warmup):
    """Whole-step time and the dominant kernel's duration over exactly
    `steps` timed steps, plus every call's and kernel's duration from an
    instrumented pass of as many steps before them.

    The instrumented pass (events between the calls, and the library's
    trace around every kernel) finds the dominant kernel and gives the
    per-kernel table; its events add gaps between the kernels, so the timed
    steps carry events only at their ends and around the dominant kernel."""
    import torch
    from paper_2311_15439_amd import spx
    for i in range(warmup):
        ts.step(i)
    torch.cuda.synchronize()
    K = len(ts.names)
    evs = [[torch.cuda.Event(enable_timing=True) for _ in range(K + 1)] for _ in range(steps)]
    trace = spx.Trace(capacity=32 * steps)
    with trace:
        for i in range(steps):
            ts.step(warmup + i, evs[i])
    torch.cuda.synchronize()
    per = {n: float(np.mean([evs[i][k].elapsed_time(evs[i][k + 1]) for i in range(steps)]))
           for k, n in enumerate(ts.names)}
    kern = {}
    for name, nbytes, ms in trace.results():
        k = kern.setdefault(name, [0.0, 0.0, 0])
        k[0] += ms
        k[1] += nbytes
        k[2] += 1
    kernels = {n: {"avg_ms": v[0] / v[2], "bytes_per_launch": v[1] / v[2], "launches_per_step": v[2] / steps}
               for n, v in kern.items()}
    dom = max(kernels, key=lambda n: kernels[n]["avg_ms"] * kernels[n]["launches_per_step"])
    dtrace = spx.Trace(capacity=4 * steps, only=dom)
    start, end = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    start.record()
    with dtrace:
        for i in range(steps):
            ts.step(warmup + steps + i)
    end.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    total_ms = start.elapsed_time(end)
    d = [(nb, ms) for _, nb, ms in dtrace.results()]
    kernels[dom]["timed_avg_ms"] = float(np.mean([ms for _, ms in d]))
    kernels[dom]["timed_bytes_per_launch"] = float(np.mean([nb for nb, _ in d]))
    kernels[dom]["dominant"] = True
    return total_ms / steps, per, wall, kernels


def time_encode_only(ts, reps=20):
    """Encoding kernels alone (forward; adjoint) on the step's first batch."""
    import torch
    spx = ts.spx
    pts, _ = ts.batches[0]
    for _ in range(3):
        spx.spx_encode_fwd(ts.enc, pts, ts.tab16, ts.feats)
        spx.spx_encode_bwd(ts.enc, pts, ts.dfeats, ts.grad, ts.bws)
    torch.cuda.synchronize()
    e = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
    e[0].record()
    for _ in range(reps):
        spx.spx_encode_fwd(ts.enc, pts, ts.tab16, ts.feats)
    e[1].record()
    for _ in range(reps):
        spx.spx_encode_bwd(ts.enc, pts, ts.dfeats, ts.grad, ts.bws)
    e[2].record()
    torch.cuda.synchronize()
    ts.grad.zero_()
    f = e[0].elapsed_time(e[1]) / reps
    b = e[1].elapsed_time(e[2]) / reps
    return {"fwd_ms": f, "bwd_ms": b, "fwd_points_per_s": ts.N / (f * 1e-3),
            "fwd_bwd_points_per_s": ts.N / ((f + b) * 1e-3)}


def probe_gather_rates(log2_min=12, log2_max=28, threads=1 << 20, per_thread=64, reps=5):
    """Uniformly random 4-byte gathers (spx_gather_probe) from buffers of
    2^log2_min .. 2^log2_max bytes: {bytes: gathers/s}, the best of `reps`
    timed launches after two untimed ones."""
    import torch
    from paper_2311_15439_amd import spx
    buf = torch.zeros(1 << (log2_max - 2), dtype=torch.int32, device="cuda")
    out = torch.empty(threads, dtype=torch.int32, device="cuda")
    rates = {}
    for e in range(log2_min, log2_max + 1):
        view = buf[: 1 << (e - 2)]
        for _ in range(2):
            spx.spx_gather_probe(view, threads, per_thread, e, out)
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(2 * reps)]
        for r in range(reps):
            ev[2 * r].record()
            spx.spx_gather_probe(view, threads, per_thread, 1000 * r + e, out)
            ev[2 * r + 1].record()
        torch.cuda.synchronize()
        ms = min(ev[2 * r].elapsed_time(ev[2 * r + 1]) for r in range(reps))
        rates[1 << e] = threads * per_thread / (ms * 1e-3)
    del buf, out
    return rates


def encode_gather_ceiling(enc, pts, res_sigma, probe, sample=1 << 16):
    """The forward's gather ceiling on these points: distinct lines per
    wave and level from the lookup's slots on the first `sample` points (in
    launch order), each level's footprint, and the time the measured
    random-gather rates need for all N points."""
    import torch
    from paper_2311_15439_amd import spx
    N = pts.shape[0]
    S = min(sample, N) // 64 * 64
    V = enc.n_vertices
    idx = torch.empty((S, enc.n_levels, V), dtype=torch.int32, device="cuda")
    spx.spx_encode_debug(enc, pts[:S].contiguous(), idx=idx)
    slots = idx.cpu().numpy().view(np.uint32)
    row = enc.n_feat * (2 if enc.table_dtype == spx.SPX_F16 else 4)
    uniq = wave_unique_lines(slots, enc.log2_T, row)
    simplex = enc.cell == spx.SPX_SIMPLEX
    reach = float(np.sqrt(enc.n_dims + 1.0)) if simplex else 1.0
    foot = level_footprints(res_sigma, reach, enc.n_dims, enc.log2_T, row, simplex)
    return {"ceiling_ms": gather_ceiling_ms(N, uniq, foot, probe),
            "lines_per_point": float(np.sum(uniq) / 64.0),
            "footprint_MiB": [round(f / 2 ** 20, 3) for f in foot]}


def _quantiles(ms):
    q = np.percentile(np.asarray(ms), [10, 50, 90])
    return {"p10_ms": float(q[0]), "median_ms": float(q[1]), "p90_ms": float(q[2])}


def time_encode_sweep(reps=30, warm=5, probe=None):
    """Encoding alone, simplex vs the 2^n grid on identical points and tables:
    the image workload, the volume workload (n=3, L=16, T=2^19, 2^21 ray
    samples) and the dimension sweep (n=2..6, L=8, T=2^20, 2^20 uniform
    points).  Forward, and forward + binned adjoint with the gradient
    clearing: in order (`fwd_bwd`, each part timed on its own too; the
    figure the rates and fractions use), and with the adjoint's counting
    pass, which needs only the points, on a second stream beside the forward
    (`fwd_bwd_pipelined`); median and p10/p90 over per-repetition events.  Gather
    fractions are the measured random-gather ceiling's time
    (encode_gather_ceiling) over the kernel's time; forward + adjoint touch
    every row twice."""
    import torch
    from paper_2311_15439_amd import inputs, spx
    dev = "cuda"
    out = {}
    wls = [inputs.PLAIN_2D, inputs.IMAGE_2D, inputs.VOLUME_3D] + [inputs.sweep_workload(n) for n in range(2, 7)]
    for w in wls:
        print(f"# encode sweep: {w.name}", file=sys.stderr, flush=True)
        if w.name.startswith("volume"):
            p = inputs.ray_points(w.n_points // 256, 256, w.seed_points)
        elif w.name.startswith("image"):
            p = inputs.pixel_points(w.n_points, w.seed_points)
        else:
            p = inputs.uniform_points(w.n_points, w.n_dims, w.seed_points)
        N = p.shape[0]
        pts = torch.from_numpy(p).to(dev)
        # binary16 tables and features, except the plain configuration's binary32 ones
        f16 = w.table_f16
        tab = torch.from_numpy(inputs.tables(w.n_levels, 1 << w.log2_T, w.n_feat, w.table_init, w.seed_tables,
                                             f16)).to(dev)
        D = w.n_levels * w.n_feat
        dout = torch.from_numpy(inputs.gradients(N, D, w.seed_points + 50)).to(dev)
        feats = torch.empty((N, D), dtype=torch.float16 if f16 else torch.float32, device=dev)
        grad = torch.zeros(tab.shape, dtype=torch.float32, device=dev)
        res = spx.spx_level_resolutions(w.n_min, w.growth, w.n_levels)
        row = {"points": N}
        for cell, cname in ((spx.SPX_SIMPLEX, "simplex"), (spx.SPX_GRID, "grid")):
            enc = spx.Encoding(w.n_dims, res, w.log2_T, w.n_feat, table_dtype=spx.SPX_F16 if f16 else spx.SPX_F32,
                               cell=cell)
            ws = torch.empty(spx.spx_encode_bwd_workspace(enc, N), dtype=torch.uint8, device=dev)

            def twin():
                if f16:  # the twin covers binary16 tables
                    spx.spx_encode_gather_twin(enc, pts, tab, feats)

            for _ in range(warm):
                twin()
                spx.spx_encode_fwd(enc, pts, tab, feats)
                grad.zero_()
                spx.spx_encode_bwd(enc, pts, dout, grad, ws)
            ev = [[torch.cuda.Event(enable_timing=True) for _ in range(5)] for _ in range(reps)]
            torch.cuda.synchronize()
            for r in range(reps):
                ev[r][0].record()
                twin()
                ev[r][1].record()
                spx.spx_encode_fwd(enc, pts, tab, feats)
                ev[r][2].record()
                grad.zero_()
                ev[r][3].record()
                spx.spx_encode_bwd(enc, pts, dout, grad, ws)
                ev[r][4].record()
            torch.cuda.synchronize()
            # forward + adjoint with the adjoint's counting pass (points only) on
            # a second stream beside the forward, joined before the adjoint
            side = side_stream()
            pev = [[torch.cuda.Event(enable_timing=True) for _ in range(2)] for _ in range(reps)]
            fork = [torch.cuda.Event() for _ in range(reps)]
            join = [torch.cuda.Event() for _ in range(reps)]
            main = torch.cuda.current_stream()
            for r in range(warm + reps):
                rr = r - warm
                if rr >= 0:
                    pev[rr][0].record()
                fork[rr % reps].record(main)
                side.wait_event(fork[rr % reps])
                spx.spx_encode_bwd_prepare(enc, pts, ws, stream=side)
                join[rr % reps].record(side)
                spx.spx_encode_fwd(enc, pts, tab, feats)
                grad.zero_()
                main.wait_event(join[rr % reps])
                spx.spx_encode_bwd_prepared(enc, pts, dout, grad, ws)
                if rr >= 0:
                    pev[rr][1].record()
            torch.cuda.synchronize()
            pipelined = _quantiles([e[0].elapsed_time(e[1]) for e in pev])
            # gradient with respect to the points (same rows as the forward)
            dpts = torch.empty((N, w.n_dims), dtype=torch.float32, device=dev)
            ig_ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
            spx.spx_encode_input_grad(enc, pts, tab, dout, dpts)
            ig_ev[0].record()
            for _ in range(10):
                spx.spx_encode_input_grad(enc, pts, tab, dout, dpts)
            ig_ev[1].record()
            torch.cuda.synchronize()
            input_grad_ms = ig_ev[0].elapsed_time(ig_ev[1]) / 10
            del dpts
            # one traced adjoint: where its time goes, kernel by kernel
            grad.zero_()
            trace = spx.Trace(capacity=64)
            with trace:
                spx.spx_encode_bwd(enc, pts, dout, grad, ws)
            bwd_kernels = {}
            for kname, nbytes, kms in trace.results():
                k = bwd_kernels.setdefault(kname, {"ms": 0.0, "GB_s": 0.0, "bytes": 0.0})
                k["ms"] += kms
                k["bytes"] += nbytes
            for k in bwd_kernels.values():
                k["GB_s"] = k["bytes"] / (k["ms"] * 1e-3) / 1e9 if k["ms"] > 0 else None
            ceil = encode_gather_ceiling(enc, pts, spx.spx_level_scales(enc), probe) if probe else None
            tw = [e[0].elapsed_time(e[1]) for e in ev]
            f = [e[1].elapsed_time(e[2]) for e in ev]
            z = [e[2].elapsed_time(e[3]) for e in ev]
            b = [e[3].elapsed_time(e[4]) for e in ev]
            t = [e[1].elapsed_time(e[4]) for e in ev]
            fq, tq, wq = _quantiles(f), _quantiles(t), _quantiles(tw)
            V = enc.n_vertices
            gathers = N * w.n_levels * V
            row[cname] = {"fwd": fq, "zero_grad": _quantiles(z), "bwd": _quantiles(b), "fwd_bwd": tq,
                          "fwd_bwd_pipelined": pipelined,
                          "gather_twin": wq if f16 else None, "bwd_kernels": bwd_kernels,
                          "input_grad_ms": input_grad_ms,
                          "fwd_points_per_s": N / (fq["median_ms"] * 1e-3),
                          "fwd_bwd_points_per_s": N / (tq["median_ms"] * 1e-3),
                          "fwd_gathers_per_s": gathers / (fq["median_ms"] * 1e-3),
                          "twin_gathers_per_s": gathers / (wq["median_ms"] * 1e-3) if f16 else None}
            if ceil:
                row[cname]["gather_ceiling"] = ceil
                row[cname]["fwd_gather_frac"] = ceil["ceiling_ms"] / fq["median_ms"]
                row[cname]["fwd_bwd_gather_frac"] = 2.0 * ceil["ceiling_ms"] / tq["median_ms"]
            del ws
        row["simplex_speedup_fwd"] = row["grid"]["fwd"]["median_ms"] / row["simplex"]["fwd"]["median_ms"]
        row["simplex_speedup_fwd_bwd"] = row["grid"]["fwd_bwd"]["median_ms"] / row["simplex"]["fwd_bwd"]["median_ms"]
        out[w.name] = row
        del pts, tab, dout, feats, grad
        torch.cuda.empty_cache()
    return out


EQUAL_ACCURACY_VARIANTS = (("simplex_equal_memory", 0, True, 0), ("simplex", 0, False, 0), ("grid", 1, False, 0))


def equal_accuracy(w, host_tables, weights, d_out, steps=2000, n_train=6, variants=EQUAL_ACCURACY_VARIANTS):
    """Accuracy at equal memory: train the field with each variant (name,
    cell, equal-memory level scaling, table layout) for the same number of
    steps on the same batches, then compare the PSNR on a held-out batch
    (colour targets: clamped to [0, 1], peak 1; volume: density and colour,
    peak = the largest held-out target value).  Adam's step size decays
    from 1e-2 to 1e-3 over the run, so the end point is not dominated by
    step noise.  Also reported per variant: the mean training step time over
    the run and the table's rows and bytes (binary16 copy; the binary32
    master and Adam's two moments are 6 times that)."""
    import torch
    from paper_2311_15439_amd import spx
    batches = []
    for b in range(n_train + 1):
        p = _points(w, 100 + b)
        batches.append((p, _targets(w, p, 100 + b)))
    held_p, held_t = batches.pop()
    out = {"steps": steps, "train_batches": n_train, "points_per_step": w.n_points}
    for name, cell, em, layout in variants:
        print(f"# accuracy {w.name}: training {name} for {steps} steps", file=sys.stderr, flush=True)
        ts = TrainStep(w, cell, batches, host_tables, weights, d_out, equal_memory=em, layout=layout)
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
        ev[0].record()
        for i in range(steps):
            ts.lr = 1e-2 * 0.1 ** (i / steps)  # exponential decay to 1e-3: a settled end point
            ts.step(i)
        ev[1].record()
        hp = torch.from_numpy(held_p).to("cuda")
        ht = torch.from_numpy(held_t).to("cuda")
        spx.spx_encode_fwd(ts.enc, hp, ts.tab16, ts.feats)
        spx.spx_mlp_fwd(ts.mlp, ts.feats, *ts.Wv, ts.y)
        if _colour_target(w):
            mse, peak = torch.mean((ts.y.clamp(0, 1) - ht) ** 2).item(), 1.0
        else:
            mse, peak = torch.mean((ts.y - ht) ** 2).item(), float(held_t.max())
        rows = int(np.prod(ts.enc.table_shape)) // w.n_feat
        out[name] = {"psnr_db": 10.0 * np.log10(peak * peak / mse), "mse": mse,
                     "ms_per_step": ev[0].elapsed_time(ev[1]) / steps, "table_rows": rows,
                     "table_f16_MiB": rows * w.n_feat * 2 / 2 ** 20}
        del ts
        torch.cuda.empty_cache()
    names = [v[0] for v in variants]
    if "grid" in names:
        for nm in names:
            if nm != "grid":
                out[f"{nm}_minus_grid_db"] = out[nm]["psnr_db"] - out["grid"]["psnr_db"]
                out[f"{nm}_speedup"] = out["grid"]["ms_per_step"] / out[nm]["ms_per_step"]
    return out


def nd_accuracy(dims=(3, 4, 5, 6), steps=1000):
    """Beyond three dimensions: an n-dimensional colour field (inputs.
    nd_workload: 16 levels 16..512, T = 2^20, 2^18 points per step, MLP
    32-64-64-3) trained with the simplex (plain and equal-memory) and the
    2^n grid; held-out PSNR and training step time for each."""
    from paper_2311_15439_amd import inputs
    out = {}
    for n in dims:
        w = inputs.nd_workload(n)
        host_tables = inputs.tables(w.n_levels, 1 << w.log2_T, w.n_feat, w.table_init, w.seed_tables, False)
        weights = inputs.mlp_weights(w.n_levels * w.n_feat, 64, 3, 9)
        out[w.name] = equal_accuracy(w, host_tables, weights, 3, steps=steps, n_train=4)
    return out


def layout_accuracy(steps=2000):
    """Sec. 5.2's table sizing: the image and volume workloads trained with
    every level hashed into T rows (the paper's configurations) and with the
    sized layout (dense coarse levels, hashed levels sized by the simplex's
    used share), beside the grid with hashed tables on the same batches;
    held-out PSNR, table memory and step time."""
    from paper_2311_15439_amd import inputs, spx
    out = {}
    for w, d_out in ((inputs.IMAGE_2D, 3), (inputs.VOLUME_3D, 4)):
        host_tables = inputs.tables(w.n_levels, 1 << w.log2_T, w.n_feat, w.table_init, w.seed_tables, False)
        weights = inputs.mlp_weights(w.n_levels * w.n_feat, 64, d_out, 9)
        out[w.name] = equal_accuracy(w, host_tables, weights, d_out, steps=steps, n_train=4,
                                     variants=(("hashed", spx.SPX_SIMPLEX, False, spx.SPX_LAYOUT_HASHED),
                                               ("sized", spx.SPX_SIMPLEX, False, spx.SPX_LAYOUT_SIZED),
                                               ("grid", spx.SPX_GRID, False, spx.SPX_LAYOUT_HASHED)))
        r = out[w.name]
        r["sized_memory_fraction"] = r["sized"]["table_rows"] / r["hashed"]["table_rows"]
        r["sized_minus_hashed_db"] = r["sized"]["psnr_db"] - r["hashed"]["psnr_db"]
        r["sized_minus_grid_db"] = r["sized"]["psnr_db"] - r["grid"]["psnr_db"]
        r["sized_speedup_vs_grid"] = r["grid"]["ms_per_step"] / r["sized"]["ms_per_step"]
    return out


def volume_bench(with_accuracy=True, steps=10, warmup=3):
    """The volume workload's training step (2^13 rays x 256 samples, n=3,
    L=16, T=2^19, MLP 32-64-64-4 regressing density and colour), simplex
    vs the 8-corner grid on the same batches, and their accuracy at equal
    memory."""
    import torch
    from paper_2311_15439_amd import inputs, spx
    w = inputs.VOLUME_3D
    print(f"# volume: generating inputs", file=sys.stderr, flush=True)
    host_tables = inputs.tables(w.n_levels, 1 << w.log2_T, w.n_feat, w.table_init, w.seed_tables, False)
    weights = inputs.mlp_weights(w.n_levels * w.n_feat, 64, 4, 9)
    batches = []
    for b in range(2):
        p = _points(w, b)
        batches.append((p, _targets(w, p, b)))
    out = {"workload": w.name + f", {w.n_points} points/step, MLP 32-64-64-4"}
    for cell, name, fb in ((spx.SPX_SIMPLEX, "simplex", False), (spx.SPX_GRID, "grid", False),
                           (spx.SPX_SIMPLEX, "simplex_fused_network_backward", True)):
        print(f"# volume: timing {name} step", file=sys.stderr, flush=True)
        ts = TrainStep(w, cell, batches, host_tables, weights, 4, fused_bwd=fb)
        ms, per, _, kern = time_steps(ts, steps, warmup)
        out[name] = {"ms_per_step": ms, "points_per_s": ts.N / (ms * 1e-3),
                     "kernels_ms": {k: round(v["avg_ms"] * v["launches_per_step"], 5) for k, v in kern.items()}}
        del ts
        torch.cuda.empty_cache()
    out["simplex_speedup"] = out["grid"]["ms_per_step"] / out["simplex"]["ms_per_step"]
    if with_accuracy:
        out["equal_accuracy"] = equal_accuracy(w, host_tables, weights, 4, n_train=4)
    return out


def time_stream_reference(ts, reps=10):
    """Plain streaming kernels over the whole table, for the practical HBM
    ceiling: the unfused Adam (36 bytes per parameter) and the binary16 copy
    (6 bytes per parameter)."""
    import torch
    spx = ts.spx
    P = ts.master.numel()
    kw = dict(lr=1e-2, beta1=0.9, beta2=0.99, eps=1e-15, step=1, zero_grad=True)
    for _ in range(2):
        spx.spx_adam_step(ts.master, ts.grad, ts.m, ts.v, ts.tab16, **kw)
        spx.spx_cast_f32_f16(ts.master.view(-1), ts.tab16.view(-1))
    e = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
    e[0].record()
    for _ in range(reps):
        spx.spx_adam_step(ts.master, ts.grad, ts.m, ts.v, ts.tab16, **kw)
    e[1].record()
    for _ in range(reps):
        spx.spx_cast_f32_f16(ts.master.view(-1), ts.tab16.view(-1))
    e[2].record()
    torch.cuda.synchronize()
    a = e[0].elapsed_time(e[1]) / reps
    c = e[1].elapsed_time(e[2]) / reps
    return {"adam_ms": a, "adam_GB_s": P * 36 / (a * 1e-3) / 1e9, "cast_ms": c, "cast_GB_s": P * 6 / (c * 1e-3) / 1e9}


def time_fused_query(ts, reps=20):
    """The serving kernel (encoding and network forward fused, features kept
    in registers) on the step's first batch, against the separate encode
    forward and network forward kernels."""
    import torch
    spx = ts.spx
    pts, _ = ts.batches[0]
    field = spx.spx_field_init(ts.enc, ts.tab16, *ts.Wv, ts.d_out)
    fdev = torch.frombuffer(bytearray(spx.as_bytes([field])), dtype=torch.uint8).cuda()
    seg = spx.spx_segment()
    seg.pts, seg.out, seg.count, seg.first_tile, seg.field = pts.data_ptr(), ts.y.data_ptr(), ts.N, 0, 0
    sdev = torch.frombuffer(bytearray(spx.as_bytes([seg])), dtype=torch.uint8).cuda()
    tiles = (ts.N + 15) // 16
    for _ in range(3):
        spx.spx_field_query_batched(fdev, 1, sdev, 1, tiles)
    e = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
    e[0].record()
    for _ in range(reps):
        spx.spx_field_query_batched(fdev, 1, sdev, 1, tiles)
    e[1].record()
    for _ in range(reps):
        spx.spx_encode_fwd(ts.enc, pts, ts.tab16, ts.feats)
        spx.spx_mlp_fwd(ts.mlp, ts.feats, *ts.Wv, ts.y)
    e[2].record()
    torch.cuda.synchronize()
    return {"fused_ms": e[0].elapsed_time(e[1]) / reps, "separate_ms": e[1].elapsed_time(e[2]) / reps}


def cpu_encode_rates(S=1 << 16):
    """The oracle's encoding on the host cores, simplex and grid (points/s;
    beside the GPU tables, as the paper reports CPU timings per dimension):
    the plain 2-D configuration's forward in full (all threads, then one),
    and forward plus adjoint on S points of the volume workload and of the
    dimension sweep n=2..6 (the forward on all threads, the adjoint, a
    binary64 sum in point order, on one)."""
    import oracle
    from paper_2311_15439_amd import inputs
    threads = oracle.max_threads()
    out = {"threads_all": threads, "sample_points": S}
    p = inputs.PLAIN_2D
    pts = inputs.uniform_points(p.n_points, p.n_dims, p.seed_points)
    tab = inputs.tables(p.n_levels, 1 << p.log2_T, p.n_feat, p.table_init, p.seed_tables, p.table_f16)
    res = oracle.level_resolutions(p.n_min, p.growth, p.n_levels)
    try:
        for nt in (threads, 1):
            oracle.set_threads(nt)
            oracle.encode_fwd(oracle.Encoding(p.n_dims, list(res), p.log2_T, p.n_feat), pts[:1024], tab)  # warm-up
            for cell, cname in ((oracle.SIMPLEX, "simplex"), (oracle.GRID, "grid")):
                e = oracle.Encoding(p.n_dims, list(res), p.log2_T, p.n_feat, table_dtype=oracle.F32, cell=cell)
                t0 = time.perf_counter()
                oracle.encode_fwd(e, pts, tab)
                out.setdefault(p.name, {})[f"{cname}_fwd_points_per_s_{nt}t"] = p.n_points / (time.perf_counter() - t0)
    finally:
        oracle.set_threads(threads)
    for w in [inputs.VOLUME_3D] + [inputs.sweep_workload(n) for n in range(2, 7)]:
        if w.name.startswith("volume"):
            pts = inputs.ray_points(S // 256, 256, w.seed_points)
        else:
            pts = inputs.uniform_points(S, w.n_dims, w.seed_points)
        tab = inputs.tables(w.n_levels, 1 << w.log2_T, w.n_feat, w.table_init, w.seed_tables, True)
        res = oracle.level_resolutions(w.n_min, w.growth, w.n_levels)
        dout = inputs.gradients(S, w.n_levels * w.n_feat, w.seed_points + 50).astype(np.float64)
        row = out.setdefault(w.name, {})
        for cell, cname in ((oracle.SIMPLEX, "simplex"), (oracle.GRID, "grid")):
            e = oracle.Encoding(w.n_dims, list(res), w.log2_T, w.n_feat, table_dtype=oracle.F16, cell=cell)
            t0 = time.perf_counter()
            oracle.encode_fwd(e, pts, tab)
            t1 = time.perf_counter()
            oracle.encode_bwd(e, pts, dout)
            t2 = time.perf_counter()
            row[f"{cname}_fwd_points_per_s"] = S / (t1 - t0)
            row[f"{cname}_fwd_bwd_points_per_s"] = S / (t2 - t0)
    return out


def cpu_identity():
    """The host's CPU model (first /proc/cpuinfo entry) and usable cores."""
    model = None
    try:
        with open("/proc/cpuinfo") as fh:
            for ln in fh:
                if ln.startswith("model name"):
                    model = ln.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        cores = len(os.sched_getaffinity(0))
    except AttributeError:
        cores = os.cpu_count()
    return model, cores


def use_timing_oracle():
    """Build the oracle for this host (-O3 -march=native) in a temporary
    directory and load it; the parity build is used if that fails.
    Returns the build's description."""
    import tempfile

    import oracle
    try:
        path = oracle.build_timing(os.path.join(tempfile.mkdtemp(prefix="spx_oracle_"), "liboracle_native.so"))
        oracle.use_library(path)
        return "gcc -O3 -march=native -ffp-contract=off -fopenmp"
    except Exception as e:  # noqa: BLE001  (the parity build still times the oracle)
        print(f"# timing build of the oracle failed ({e}); timing the parity build", file=sys.stderr, flush=True)
        return "gcc -O2 -ffp-contract=off -fopenmp (parity build)"


def cpu_baseline(w, host_tables, weights, batch, S=1 << 16):
    """The oracle (as it stands) on a bounded sample of the same step: the
    per-point work on S points, Adam on 1/16 of the tables; scaled to one
    step of N points."""
    import oracle
    from paper_2311_15439_amd import spx as _spx  # noqa: F401  (only for the schedule helper below)
    res = oracle.level_resolutions(w.n_min, w.growth, w.n_levels)
    oe = oracle.Encoding(w.n_dims, list(res), w.log2_T, w.n_feat, table_dtype=oracle.F16)
    pts, tgt = batch[0][:S], batch[1][:S]
    tab16 = host_tables.astype(np.float16)
    W1, W2, W3 = weights
    t0 = time.perf_counter()
    feats = oracle.encode_fwd(oe, pts, tab16)
    f16 = feats.astype(np.float16)
    y = oracle.mlp_fwd(f16, W1, W2, W3)
    dy = oracle.mse_grad(y.astype(np.float32), tgt, 2.0 / y.size).astype(np.float32)
    g = oracle.mlp_bwd(f16, W1, W2, W3, dy)
    oracle.encode_bwd(oe, pts, g["d_x"])
    t_pts = time.perf_counter() - t0
    P = host_tables.size // 16
    flat = host_tables.reshape(-1)[:P].astype(np.float32)
    t0 = time.perf_counter()
    oracle.adam_step(flat, flat * 0.01, np.zeros(P, np.float32), np.zeros(P, np.float32), 1e-2, 0.9, 0.99, 1e-15, 1)
    t_adam = (time.perf_counter() - t0) * 16
    t_step = t_pts * (w.n_points / S) + t_adam
    threads = oracle.max_threads()
    model, ncpu = cpu_identity()
    return {"value": w.n_points / t_step, "unit": "points/s", "cores": threads, "kind": "oracle",
            "sample": f"oracle training step on {S} of the {w.n_points} points ({t_pts:.2f} s) plus Adam on 1/16 "
                      f"of the tables ({t_adam / 16:.2f} s), scaled to one {w.n_points}-point step; "
                      f"encode fwd and MLP fwd on {threads} OpenMP threads, the rest on one",
            "cpu_model": model, "host_cores": ncpu}


def serving_bench(n_fields=8, n_requests=2000, warm=200, loads=(0.5, 0.8), train_steps=2000):
    """Serving: resident 3-D fields (n=3, L=16, T=2^19, F=2 binary16, MLP
    32-64-64-4), each trained for train_steps Adam steps on its own
    synthetic density (2^16 points per step); requests
    of log-uniform size 2^8..2^20 points on a uniformly chosen field.  First
    the saturation rate (requests submitted back to back), then Poisson
    arrivals at fractions of it; latency is submit -> results in host
    memory."""
    import threading

    import torch
    from paper_2311_15439_amd import inputs, spx
    from paper_2311_15439_amd.serve import GpuBackend, Server
    from paper_2311_15439_amd.torch_ops import NeuralField, SimplexEncoding, TinyMLP

    w = inputs.VOLUME_3D
    descs, keep = [], []
    train_pts = inputs.uniform_points(1 << 16, 3, 99)
    tp = torch.from_numpy(train_pts).cuda()
    for f in range(n_fields):
        print(f"# serving: training field {f} ({train_steps} steps)", file=sys.stderr, flush=True)
        enc = SimplexEncoding(3, w.n_levels, w.log2_T, 2, n_min=w.n_min, growth=w.growth, seed=20 + f)
        net = TinyMLP(32, 4, seed=40 + f)
        field = NeuralField(enc, net)
        tgt = torch.from_numpy(inputs.procedural_density(train_pts, 20 + f)).cuda()
        opt = torch.optim.Adam(field.parameters(), lr=1e-2, betas=(0.9, 0.99), eps=1e-15)
        for _ in range(train_steps):
            loss = torch.mean((field(tp) - tgt) ** 2)
            opt.zero_grad()
            loss.backward()
            opt.step()
        enc.sync()
        net.sync()
        descs.append(spx.spx_field_init(enc.enc, enc.table_f16, *net._W16, 4))
        keep.append((enc, net))
    torch.cuda.synchronize()
    pool = inputs.uniform_points(1 << 22, 3, 123)
    rng = np.random.default_rng(30)

    def make(k):
        sizes = np.floor(2.0 ** rng.uniform(8, 20, k)).astype(int)
        fields = rng.integers(0, n_fields, k)
        starts = rng.integers(0, len(pool) - (1 << 20), k)
        return [(int(f), pool[s:s + m]) for f, s, m in zip(fields, starts, sizes)]

    be = GpuBackend(descs)
    srv = Server(be, [3] * n_fields, [4] * n_fields, arena_bytes=1 << 30, chunk_points=1 << 18,
                 batch_points=1 << 21).start()
    try:
        for f, p in make(warm):
            srv.submit(f, p)
        reqs = make(n_requests)
        t0 = time.perf_counter()
        rs = [srv.submit(f, p) for f, p in reqs]
        for r in rs:
            r.wait(120)
        sat_s = time.perf_counter() - t0
        pts_total = sum(len(p) for _, p in reqs)
        sat = pts_total / sat_s
        mean_m = pts_total / len(reqs)
        out = {"fields": n_fields, "requests_per_load": n_requests, "mean_request_points": mean_m,
               "saturation_points_per_s": sat, "saturation_requests_per_s": len(reqs) / sat_s, "loads": []}
        for load in loads:
            lam = load * sat / mean_m
            reqs = make(n_requests)
            gaps = rng.exponential(1.0 / lam, len(reqs))
            submitted = []

            def client():
                t = time.perf_counter()
                for (f, p), g in zip(reqs, gaps):
                    t += g
                    d = t - time.perf_counter()
                    if d > 0:
                        time.sleep(d)
                    submitted.append(srv.submit(f, p))

            th = threading.Thread(target=client)
            t0 = time.perf_counter()
            th.start()
            th.join()
            for r in submitted:
                r.wait(120)
            span = time.perf_counter() - t0
            lat = np.array([r.latency for r in submitted]) * 1e3
            out["loads"].append({"load": load, "offered_requests_per_s": lam,
                                 "p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
                                 "points_per_s": sum(len(p) for _, p in reqs) / span})
        out["batches"] = srv.batches
    finally:
        srv.stop()
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="image-2d", choices=["image-2d", "volume-3d"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-grid", action="store_true")
    ap.add_argument("--no-serving", action="store_true")
    ap.add_argument("--no-sweep", action="store_true", help="skip the volume / dimension-sweep encoding timings")
    ap.add_argument("--no-accuracy", action="store_true", help="skip the equal-memory accuracy comparison")
    ap.add_argument("--no-volume", action="store_true",
                    help="skip the volume workload's training step (simplex vs grid) and its accuracy comparison")
    ap.add_argument("--no-render", action="store_true",
                    help="skip the volume-rendering training step (compositing along rays), simplex vs grid")
    ap.add_argument("--no-nd", action="store_true",
                    help="skip the n-dimensional accuracy and step-time comparison (n = 3..6), simplex vs grid")
    ap.add_argument("--no-layout", action="store_true",
                    help="skip the table-layout comparison (hashed vs sized tables: accuracy, memory)")
    ap.add_argument("--detail-out", default=DETAIL_DEFAULT,
                    help="file for the full JSON record (the last stdout line is a compact summary)")
    ap.add_argument("--pmc-pass", action="store_true",
                    help="run two training steps and a binary32->binary16 copy of 2^26 elements, then exit "
                         "(the program profiled by the rocprofv3 --pmc traffic runs)")
    ap.add_argument("--write-traffic", nargs=2, metavar=("READ_CSV", "WRITE_CSV"),
                    help="turn the counter CSVs of the two --pmc runs (of --pmc-pass on --workload) into "
                         + TRAFFIC_FILE.format("<workload>") + " and exit")
    args = ap.parse_args()
    if args.write_traffic:
        write_traffic(*args.write_traffic, _workload(args.workload).name)
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU; --gpus {args.gpus} is not supported "
              "(sharding the tables by level over several GPUs is not implemented)", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2311_15439_amd import inputs, spx
    spx.lib()
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)

    w = _workload(args.workload)
    d_out = 3 if w.name.startswith("image") else 4
    print(f"# setup {w.name}: generating inputs", file=sys.stderr, flush=True)
    host_tables = inputs.tables(w.n_levels, 1 << w.log2_T, w.n_feat, w.table_init, w.seed_tables, False)
    weights = inputs.mlp_weights(w.n_levels * w.n_feat, 64, d_out, 9)
    batches = []
    for b in range(2):
        p = _points(w, b)
        batches.append((p, _targets(w, p, b)))

    ts = TrainStep(w, spx.SPX_SIMPLEX, batches, host_tables, weights, d_out)
    res = ts.res
    if args.pmc_pass:
        for b in range(2):
            ts.step(b)
        torch.cuda.synchronize()
        src = torch.ones(COPY_ELEMS, dtype=torch.float32, device="cuda")
        dst = torch.empty(COPY_ELEMS, dtype=torch.float16, device="cuda")
        spx.spx_cast_f32_f16(src, dst)
        torch.cuda.synchronize()
        print("# pmc pass done", file=sys.stderr, flush=True)
        return
    print("# timing simplex step", file=sys.stderr, flush=True)
    ms, per, wall, kern = time_steps(ts, args.steps, args.warmup)
    enc_s = time_encode_only(ts)
    stream = time_stream_reference(ts)
    fused_query = time_fused_query(ts)
    bytes_ = ts.algorithmic_bytes()
    per = {k: v for k, v in per.items() if bytes_.get(k, 0) > 0}
    # dominant single kernel of the step (total time per step), timed inside the timed steps
    dom = next(n for n, v in kern.items() if v.get("dominant"))
    achieved = kern[dom]["timed_bytes_per_launch"] / (kern[dom]["timed_avg_ms"] * 1e-3) / 1e9
    calls = {k: {"avg_ms": round(v, 5), "algorithmic_GB_s": round(bytes_[k] / (v * 1e-3) / 1e9, 1)}
             for k, v in per.items()}
    kernels = {n: {"avg_ms": round(v["avg_ms"], 5), "launches_per_step": v["launches_per_step"],
                   "algorithmic_GB_s": round(v["bytes_per_launch"] / (v["avg_ms"] * 1e-3) / 1e9, 1)}
               for n, v in sorted(kern.items(), key=lambda kv: -kv[1]["avg_ms"] * kv[1]["launches_per_step"])}

    # the network backward inside the adjoint's scatter (spx_encode_mlp_bwd_adam), same batches
    del ts
    torch.cuda.empty_cache()
    print("# timing the step with the network backward fused into the adjoint", file=sys.stderr, flush=True)
    tf = TrainStep(w, spx.SPX_SIMPLEX, batches, host_tables, weights, d_out, fused_bwd=True)
    fms, fper, _, fkern = time_steps(tf, max(5, args.steps // 2), 2)
    fused_bwd = {"ms_per_step": fms, "step_points_per_s": tf.N / (fms * 1e-3), "vs_separate": ms / fms,
                 "calls_ms": {k: round(v, 5) for k, v in fper.items()},
                 "kernels_ms": {k: round(v["avg_ms"] * v["launches_per_step"], 5) for k, v in fkern.items()}}
    del tf
    torch.cuda.empty_cache()

    grid = None
    if not args.no_grid:
        torch.cuda.empty_cache()
        tg = TrainStep(w, spx.SPX_GRID, batches, host_tables, weights, d_out)
        print("# timing grid step", file=sys.stderr, flush=True)
        gms, gper, _, gkern = time_steps(tg, max(5, args.steps // 2), 2)
        genc = time_encode_only(tg)
        gb = tg.algorithmic_bytes()
        grid = {"step_points_per_s": tg.N / (gms * 1e-3), "ms_per_step": gms,
                "kernels_ms": {k: round(v, 5) for k, v in gper.items() if gb.get(k, 0) > 0}, "encode_only": genc}
        del tg
        torch.cuda.empty_cache()

    accuracy = None
    if not args.no_accuracy:
        accuracy = {w.name: equal_accuracy(w, host_tables, weights, d_out)}

    volume = None
    if not args.no_volume and w.name.startswith("image"):
        volume = volume_bench(with_accuracy=not args.no_accuracy)

    render = None
    if not args.no_render and w.name.startswith("image"):
        render = render_bench()

    nd, layout = None, None
    if not args.no_nd:
        nd = nd_accuracy()
    if not args.no_layout:
        layout = layout_accuracy()

    sweep, probe = None, None
    if not args.no_sweep:
        print("# random-gather probe", file=sys.stderr, flush=True)
        probe = probe_gather_rates()
        sweep = time_encode_sweep(probe=probe)

    serving = None
    if not args.no_serving:
        print("# serving: training resident fields, then saturation and Poisson loads", file=sys.stderr, flush=True)
        # the serving scheduler is host-bound: start it without the earlier sections' garbage and
        # cached allocations
        gc.collect()
        torch.cuda.empty_cache()
        serving = serving_bench()

    cpu, cpu_rates = None, None
    if not args.no_cpu_baseline:
        print("# timing the CPU oracle sample", file=sys.stderr, flush=True)
        build = use_timing_oracle()
        cpu = cpu_baseline(w, host_tables, weights, batches[0])
        cpu["build"] = build
        cpu_rates = cpu_encode_rates()

    value = w.n_points / (ms * 1e-3)
    detail = {
        "value_is": ("points/s of the whole simplex training step (encode fwd, MLP fwd, loss gradient, MLP bwd, "
                     "encode adjoint fused with Adam on the tables, Adam on the MLP) on the image workload"),
        "ms_per_step": ms,
        "config": {"workload": w.name, "points_per_step": w.n_points, "levels": res,
                   "mlp": f"{w.n_levels * w.n_feat}-64-64-{d_out}"},
        "roofline": {"bound": "hbm", "kernel": dom, "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": measured_traffic(dom, w.name),
                     "avg_ms": kern[dom]["timed_avg_ms"], "bytes_per_launch": kern[dom]["timed_bytes_per_launch"]},
        "cpu_baseline": cpu,
        "cpu_encode_rates": cpu_rates,
        "kernels": kernels,
        "calls": calls,
        "encode_only": {"simplex": enc_s, "grid": grid["encode_only"] if grid else None},
        "grid_baseline_step": ({"points_per_s": grid["step_points_per_s"], "ms_per_step": grid["ms_per_step"],
                                "kernels_ms": grid["kernels_ms"]} if grid else None),
        "stream_reference": stream,
        "fused_query": fused_query,
        "fused_network_backward": fused_bwd,
        "gather_probe_gathers_per_s": probe,
        "encode_sweep": sweep,
        "equal_accuracy": accuracy,
        "nd_accuracy": nd,
        "layout_accuracy": layout,
        "volume_step": volume,
        "render_step": render,
        "serving": serving,
        "wall_s_timed": wall,
    }
    if args.detail_out:
        d = os.path.dirname(args.detail_out)
        if d:
            os.makedirs(d, exist_ok=True)
        with open(args.detail_out, "w") as fh:
            json.dump(detail, fh, indent=1)
    for ln in summary_lines(detail):
        print(ln)
    line = headline(detail, value, args.steps, args.warmup, args.detail_out)
    print(json.dumps(line, separators=(",", ":")), flush=True)


def _r(x, nd=4):
    """Round to nd significant digits (None stays None)."""
    if x is None:
        return None
    return float(f"{x:.{nd}g}")


def summary_lines(d):
    """Short human-readable lines (prefixed '#') printed before the JSON
    line: one per section of the detail record."""
    out = []
    sw = d.get("encode_sweep") or {}
    for name, row in sw.items():
        s, g = row["simplex"], row["grid"]
        out.append(f"# encode {name}: fwd {s['fwd']['median_ms']:.3f}/{g['fwd']['median_ms']:.3f} ms, "
                   f"fwd+bwd {s['fwd_bwd']['median_ms']:.3f}/{g['fwd_bwd']['median_ms']:.3f} ms (simplex/grid); "
                   f"gather frac simplex fwd {_r(s.get('fwd_gather_frac'), 3)} fwd+bwd "
                   f"{_r(s.get('fwd_bwd_gather_frac'), 3)}")
    acc = dict(d.get("equal_accuracy") or {})
    if d.get("volume_step") and d["volume_step"].get("equal_accuracy"):
        acc["volume"] = d["volume_step"]["equal_accuracy"]
    for name, a in acc.items():
        out.append(f"# accuracy {name}: PSNR simplex {a['simplex']['psnr_db']:.2f}, equal-memory "
                   f"{a['simplex_equal_memory']['psnr_db']:.2f}, grid {a['grid']['psnr_db']:.2f} dB")
    for name, a in (d.get("nd_accuracy") or {}).items():
        out.append(f"# accuracy {name}: PSNR simplex {a['simplex']['psnr_db']:.2f}, equal-memory "
                   f"{a['simplex_equal_memory']['psnr_db']:.2f}, grid {a['grid']['psnr_db']:.2f} dB; step "
                   f"{a['simplex']['ms_per_step']:.3f} / {a['grid']['ms_per_step']:.3f} ms (simplex / grid)")
    for name, a in (d.get("layout_accuracy") or {}).items():
        out.append(f"# table layout {name}: sized tables {a['sized_memory_fraction']:.3f} of the hashed rows, PSNR "
                   f"{a['sized']['psnr_db']:.2f} vs {a['hashed']['psnr_db']:.2f} dB (grid {a['grid']['psnr_db']:.2f}); "
                   f"step {a['sized']['ms_per_step']:.3f} / {a['hashed']['ms_per_step']:.3f} / "
                   f"{a['grid']['ms_per_step']:.3f} ms (sized / hashed / grid)")
    fb = d.get("fused_network_backward")
    if fb:
        out.append(f"# network backward fused into the adjoint: {fb['ms_per_step']:.3f} ms per step, "
                   f"{fb['vs_separate']:.3f}x the separate kernels' {d['ms_per_step']:.3f} ms")
    sv = d.get("serving")
    if sv:
        loads = ", ".join(f"{l['load']:.0%}: p50 {l['p50_ms']:.2f} p99 {l['p99_ms']:.2f} ms" for l in sv["loads"])
        out.append(f"# serving: saturation {sv['saturation_points_per_s'] / 1e6:.0f} M points/s; {loads}")
    return out


# what one timed step of each workload is, for the headline line
STEP_WORKLOADS = {
    "image-2d n=2 L=16 T=2^22 F=2 f16":
        ("image-2d training step: n=2, L=16, T=2^22, F=2 f16 tables, N_l 16..32768, "
         "2^20 random pixels of a 16384^2 image per step, MLP 32-64-64-3, Adam"),
    "volume-3d n=3 L=16 T=2^19 F=2 f16":
        ("volume-3d training step: n=3, L=16, T=2^19, F=2 f16 tables, N_l 16..2048, "
         "2^13 rays x 256 samples per step, MLP 32-64-64-4, Adam"),
}


def headline(d, value, steps, warmup, detail_path):
    """The one JSON line the run ends with (compact; the full record is in
    the detail file)."""
    rf = d["roofline"]
    cpu = d.get("cpu_baseline")
    line = {
        "metric": "encoded points/s fwd & fwd+bwd, simplex vs 2^n-grid same GPU; serving p50/p99 ms",
        "value": _r(value, 6),
        "unit": "points/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": warmup,
        "ms_per_step": _r(d["ms_per_step"], 6),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f16 tables+features, f32 accumulate; MLP f16 MFMA fwd, bf16 MFMA operands bwd",
        "data": "synthetic",
        "config": {"workload": STEP_WORKLOADS.get(d["config"]["workload"], d["config"]["workload"]),
                   "parallelism": "single GPU"},
        "roofline": {"bound": rf["bound"], "kernel": rf["kernel"], "achieved": _r(rf["achieved"]),
                     "peak": rf["peak"], "unit": rf["unit"], "frac": _r(rf["frac"]),
                     "traffic": _r(rf["traffic"]), "avg_ms": _r(rf["avg_ms"]),
                     "bytes_per_launch": _r(rf["bytes_per_launch"])},
        "cpu_baseline": None if cpu is None else {
            "value": _r(cpu["value"]), "unit": cpu["unit"], "cores": cpu["cores"], "kind": cpu["kind"],
            "sample": "oracle step on 2^16 of 2^20 points + Adam on 1/16 of the tables, scaled",
            "cpu_model": cpu.get("cpu_model"), "build": cpu.get("build")},
    }
    g = d.get("grid_baseline_step")
    if g:
        line["grid_step"] = {"points_per_s": _r(g["points_per_s"]), "ms_per_step": _r(g["ms_per_step"]),
                             "simplex_speedup": _r(g["ms_per_step"] / d["ms_per_step"], 3)}
    sw = d.get("encode_sweep")
    if sw:
        enc = {"cols": ["fwd_pts_s", "fwd_bwd_pts_s", "grid_fwd_pts_s", "grid_fwd_bwd_pts_s",
                        "gather_frac_fwd", "gather_frac_fwd_bwd"]}
        for name, row in sw.items():
            s, gr = row["simplex"], row["grid"]
            enc[name.split(" L=")[0]] = [_r(s["fwd_points_per_s"], 3), _r(s["fwd_bwd_points_per_s"], 3),
                                        _r(gr["fwd_points_per_s"], 3), _r(gr["fwd_bwd_points_per_s"], 3),
                                        _r(s.get("fwd_gather_frac"), 3), _r(s.get("fwd_bwd_gather_frac"), 3)]
        line["encode"] = enc
    acc = {}
    for name, a in (d.get("equal_accuracy") or {}).items():
        acc[name.split(" ")[0]] = [_r(a["simplex_minus_grid_db"], 3), _r(a["simplex_equal_memory_minus_grid_db"], 3)]
    vol = d.get("volume_step")
    if vol:
        line["volume_step"] = {"points_per_s": _r(vol["simplex"]["points_per_s"]),
                               "simplex_speedup": _r(vol["simplex_speedup"], 3)}
        if vol.get("equal_accuracy"):
            a = vol["equal_accuracy"]
            acc["volume-3d"] = [_r(a["simplex_minus_grid_db"], 3), _r(a["simplex_equal_memory_minus_grid_db"], 3)]
    if acc:
        acc["cols"] = ["simplex_minus_grid_db", "equal_memory_minus_grid_db"]
        line["accuracy"] = acc
    nd = d.get("nd_accuracy")
    if nd:
        line["nd_accuracy"] = {"cols": ["simplex_minus_grid_db", "equal_memory_minus_grid_db", "simplex_step_speedup"]}
        for name, a in nd.items():
            line["nd_accuracy"][name.split(" L=")[0]] = [_r(a["simplex_minus_grid_db"], 3),
                                                         _r(a["simplex_equal_memory_minus_grid_db"], 3),
                                                         _r(a["simplex_speedup"], 3)]
    lay = d.get("layout_accuracy")
    if lay:
        line["table_layout"] = {"cols": ["sized_memory_fraction", "sized_minus_hashed_db", "sized_minus_grid_db",
                                         "sized_speedup_vs_grid"]}
        for name, a in lay.items():
            line["table_layout"][name.split(" ")[0]] = [_r(a["sized_memory_fraction"], 3),
                                                        _r(a["sized_minus_hashed_db"], 3),
                                                        _r(a.get("sized_minus_grid_db"), 3),
                                                        _r(a.get("sized_speedup_vs_grid"), 3)]
    fb = d.get("fused_network_backward")
    if fb:
        line["fused_network_backward"] = {"ms_per_step": _r(fb["ms_per_step"]), "vs_separate": _r(fb["vs_separate"], 3)}
    sv = d.get("serving")
    if sv:
        line["serving"] = {"saturation_points_per_s": _r(sv["saturation_points_per_s"]),
                           "loads": [[l["load"], _r(l["p50_ms"], 3), _r(l["p99_ms"], 3), _r(l["points_per_s"], 3)]
                                     for l in sv["loads"]],
                           "cols": ["load", "p50_ms", "p99_ms", "points_per_s"]}
    line["detail"] = detail_path
    return line


if __name__ == "__main__":
    main()
