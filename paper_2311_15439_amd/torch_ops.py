"""torch.autograd wrappers over the C ABI (argument marshalling only).

* ``SimplexEncodingFn``: points -> encoded features (binary32 out), with the
  binary32 master tables as the differentiable input; the forward gathers
  from their binary16 copy, the backward runs the binned adjoint (and, when
  the points require a gradient, the input-gradient kernel).
* ``MLPFn``: features (binary32) -> network output; weights as binary32
  masters, binary16 copies for the matrix cores.
* ``FieldFn``: encoding and network together, keeping the binary16 features
  internal and handing the network's binary32 feature gradient straight to
  the adjoint (what a training step wants).

The modules keep the binary16 copies in sync with their masters by watching
the masters' version counters (optimizers update parameters in place).
"""
from __future__ import annotations

import math
from typing import Optional

import numpy as np
import torch

from . import spx


class _Workspace:
    """Grow-only device scratch buffer (the library never allocates)."""

    def __init__(self):
        self.buf: Optional[torch.Tensor] = None

    def get(self, nbytes: int, device) -> torch.Tensor:
        if self.buf is None or self.buf.numel() < nbytes or self.buf.device != torch.device(device):
            self.buf = torch.empty(max(nbytes, 256), dtype=torch.uint8, device=device)
        return self.buf[:max(nbytes, 256)]


def _f16_copy(master: torch.Tensor, copy: torch.Tensor) -> None:
    spx.spx_cast_f32_f16(master.detach().reshape(-1), copy.reshape(-1))


class SimplexEncodingFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, pts, params, enc, table_f16, ws):
        N = pts.shape[0]
        out = torch.empty((N, enc.n_levels * enc.n_feat), dtype=torch.float32, device=pts.device)
        spx.spx_encode_fwd(enc, pts, table_f16, out)
        ctx.save_for_backward(pts, table_f16)
        ctx.enc, ctx.ws = enc, ws
        return out

    @staticmethod
    def backward(ctx, grad_out):
        pts, table_f16 = ctx.saved_tensors
        enc = ctx.enc
        g = grad_out.contiguous().float()
        grad = torch.zeros(enc.table_shape, dtype=torch.float32, device=pts.device)
        if pts.shape[0] > 0:
            w = ctx.ws.get(spx.spx_encode_bwd_workspace(enc, pts.shape[0]), pts.device)
            spx.spx_encode_bwd(enc, pts, g, grad, w)
        d_pts = None
        if ctx.needs_input_grad[0]:
            d_pts = torch.empty_like(pts)
            if pts.shape[0] > 0:
                spx.spx_encode_input_grad(enc, pts, table_f16, g, d_pts)
        return d_pts, grad, None, None, None


class MLPFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, x, W1, W2, W3, mlp, W16, ws):
        N = x.shape[0]
        x16 = torch.empty(x.shape, dtype=torch.float16, device=x.device)
        spx.spx_cast_f32_f16(x.contiguous().reshape(-1), x16.reshape(-1))
        y = torch.empty((N, mlp.d_out), dtype=torch.float32, device=x.device)
        spx.spx_mlp_fwd(mlp, x16, *W16, y)
        ctx.save_for_backward(x16)
        ctx.mlp, ctx.W16, ctx.ws = mlp, W16, ws
        return y

    @staticmethod
    def backward(ctx, gy):
        (x16,) = ctx.saved_tensors
        mlp, W16 = ctx.mlp, ctx.W16
        N = x16.shape[0]
        dx = torch.empty(x16.shape, dtype=torch.float32, device=x16.device)
        dW = [torch.empty(w.shape, dtype=torch.float32, device=x16.device) for w in W16]
        w = ctx.ws.get(spx.spx_mlp_bwd_workspace(mlp, N), x16.device)
        spx.spx_mlp_bwd(mlp, x16, *W16, gy.contiguous().float(), dx, *dW, w)
        return dx, dW[0], dW[1], dW[2], None, None, None


class FieldFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, pts, params, W1, W2, W3, enc, table_f16, mlp, W16, ws_enc, ws_mlp):
        N = pts.shape[0]
        feats = torch.empty((N, enc.n_levels * enc.n_feat), dtype=torch.float16, device=pts.device)
        y = torch.empty((N, mlp.d_out), dtype=torch.float32, device=pts.device)
        if (enc.n_dims in (2, 3) and enc.n_levels == 16 and enc.n_feat == 2 and mlp.d_in == 32
                and enc.layout == spx.SPX_LAYOUT_HASHED):
            # one kernel: features go from the gathers to the matrix cores in registers
            spx.spx_encode_mlp_fwd(enc, mlp, pts, table_f16, *W16, y, feats=feats)
        else:
            spx.spx_encode_fwd(enc, pts, table_f16, feats)
            spx.spx_mlp_fwd(mlp, feats, *W16, y)
        ctx.save_for_backward(pts, feats, table_f16)
        ctx.enc, ctx.mlp, ctx.W16, ctx.ws_enc, ctx.ws_mlp = enc, mlp, W16, ws_enc, ws_mlp
        return y

    @staticmethod
    def backward(ctx, gy):
        pts, feats, table_f16 = ctx.saved_tensors
        enc, mlp, W16 = ctx.enc, ctx.mlp, ctx.W16
        N = pts.shape[0]
        dfeats = torch.empty(feats.shape, dtype=torch.float32, device=pts.device)
        dW = [torch.empty(w.shape, dtype=torch.float32, device=pts.device) for w in W16]
        spx.spx_mlp_bwd(mlp, feats, *W16, gy.contiguous().float(), dfeats, *dW,
                        ctx.ws_mlp.get(spx.spx_mlp_bwd_workspace(mlp, N), pts.device))
        grad = torch.zeros(enc.table_shape, dtype=torch.float32, device=pts.device)
        if N > 0:
            spx.spx_encode_bwd(enc, pts, dfeats, grad,
                               ctx.ws_enc.get(spx.spx_encode_bwd_workspace(enc, N), pts.device))
        d_pts = None
        if ctx.needs_input_grad[0]:
            d_pts = torch.empty_like(pts)
            if N > 0:
                spx.spx_encode_input_grad(enc, pts, table_f16, dfeats, d_pts)
        return d_pts, grad, dW[0], dW[1], dW[2], None, None, None, None, None, None


class SimplexEncoding(torch.nn.Module):
    """Multiresolution simplex (or grid) hash encoding with binary32 master
    tables ``params`` (shape ``enc.table_shape``: [L, T, F] for the hashed
    layout) and a binary16 copy used by the forward."""

    def __init__(self, n_dims: int, n_levels: int = 16, log2_T: int = 19, n_feat: int = 2,
                 n_min: float = 16, n_max: Optional[float] = None, growth: Optional[float] = None,
                 cell: int = spx.SPX_SIMPLEX, equal_memory: bool = False, init_scale: float = 1e-4,
                 seed: int = 0, device="cuda", layout: int = spx.SPX_LAYOUT_HASHED):
        super().__init__()
        if growth is None:
            growth = 1.5 if n_max is None else (n_max / n_min) ** (1.0 / max(n_levels - 1, 1))
        res = spx.spx_level_resolutions(n_min, growth, n_levels)
        self.enc = spx.Encoding(n_dims, res, log2_T, n_feat, table_dtype=spx.SPX_F16, cell=cell,
                                equal_memory=equal_memory, layout=layout)
        init = np.random.default_rng(seed).uniform(-init_scale, init_scale, self.enc.table_shape)
        self.params = torch.nn.Parameter(torch.from_numpy(init.astype(np.float32)).to(device))
        self.register_buffer("table_f16", torch.empty(self.enc.table_shape, dtype=torch.float16, device=device))
        self._synced = None
        self._ws = _Workspace()

    @property
    def out_dim(self) -> int:
        return self.enc.n_levels * self.enc.n_feat

    def sync(self) -> None:
        key = (self.params._version, self.params.data_ptr())
        if key != self._synced:
            _f16_copy(self.params, self.table_f16)
            self._synced = key

    def forward(self, pts: torch.Tensor) -> torch.Tensor:
        self.sync()
        return SimplexEncodingFn.apply(pts.contiguous(), self.params, self.enc, self.table_f16, self._ws)


class TinyMLP(torch.nn.Module):
    """d_in -> 64 -> 64 -> d_out, ReLU hidden, linear output; binary32 masters."""

    def __init__(self, d_in: int = 32, d_out: int = 3, hidden: int = 64, seed: int = 0, device="cuda"):
        super().__init__()
        self.mlp = spx.make_mlp(d_in, hidden, d_out)
        rng = np.random.default_rng(seed)

        def init(o, i):
            b = math.sqrt(6.0 / i)
            return torch.nn.Parameter(torch.from_numpy(rng.uniform(-b, b, (o, i)).astype(np.float32)).to(device))

        self.W1, self.W2, self.W3 = init(hidden, d_in), init(hidden, hidden), init(d_out, hidden)
        self._W16 = [torch.empty(w.shape, dtype=torch.float16, device=device) for w in (self.W1, self.W2, self.W3)]
        self._synced = None
        self._ws = _Workspace()

    def sync(self) -> None:
        key = tuple((w._version, w.data_ptr()) for w in (self.W1, self.W2, self.W3))
        if key != self._synced:
            for w, c in zip((self.W1, self.W2, self.W3), self._W16):
                _f16_copy(w, c)
            self._synced = key

    def forward(self, x: torch.Tensor) -> torch.Tensor:
        self.sync()
        return MLPFn.apply(x, self.W1, self.W2, self.W3, self.mlp, self._W16, self._ws)


class NeuralField(torch.nn.Module):
    """Encoding followed by the tiny network, run as one autograd node."""

    def __init__(self, encoding: SimplexEncoding, net: TinyMLP):
        super().__init__()
        self.encoding, self.net = encoding, net

    def forward(self, pts: torch.Tensor) -> torch.Tensor:
        self.encoding.sync()
        self.net.sync()
        e, n = self.encoding, self.net
        return FieldFn.apply(pts.contiguous(), e.params, n.W1, n.W2, n.W3, e.enc, e.table_f16, n.mlp, n._W16,
                             e._ws, n._ws)
