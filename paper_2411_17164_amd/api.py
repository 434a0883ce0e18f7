"""Python face of the xmgn library: thin wrappers with the names of the C ABI.

Device arrays are torch CUDA (HIP) tensors, host arrays numpy arrays; every
call passes pointers and sizes to libxmgn.so and runs on the tensor's current
stream.  Nothing here computes.
"""
from __future__ import annotations

import ctypes as C
from dataclasses import dataclass

import numpy as np
import torch

from ._lib import Desc, XmgnError, check, lib

ACTIVATIONS = {"relu": 0, "silu": 1}
PRECISIONS = {"fp32": 0, "bf16": 1}
AGGREGATES = {"message": 0, "edge": 1}


@dataclass(frozen=True)
class Model:
    """Model description (see xmgn_model_desc in include/xmgn.h)."""
    hidden: int
    n_layers: int
    node_in: int = 6
    edge_in: int = 4
    out_dim: int = 4
    activation: str = "relu"
    precision: str = "fp32"
    aggregate: str = "message"
    ln_eps: float = 1e-5

    def desc(self) -> Desc:
        return Desc(self.hidden, self.n_layers, self.node_in, self.edge_in, self.out_dim,
                    ACTIVATIONS[self.activation], PRECISIONS[self.precision],
                    AGGREGATES[self.aggregate], self.ln_eps)

    def param_count(self) -> int:
        n = C.c_int64()
        check(lib.xmgn_param_count(C.byref(self.desc()), C.byref(n)))
        return n.value

    def param_offset(self, block: int, layer: int, tensor: int) -> int:
        n = C.c_int64()
        check(lib.xmgn_param_offset(C.byref(self.desc()), block, layer, tensor, C.byref(n)))
        return n.value

    def param_tensors(self):
        """[(block, layer, tensor, kind, shape, offset)] in blob order, with
        offsets from the library (kinds: weight, bias, gamma, beta)."""
        H, out = self.hidden, []
        mlp = {0: [self.node_in, H, H, H], 1: [self.edge_in, H, H, H], 2: [3 * H, H, H],
               3: [2 * H, H, H], 4: [H, H, H, self.out_dim]}
        order = [(0, 0), (1, 0)] + [(b, l) for l in range(self.n_layers) for b in (2, 3)] + [(4, 0)]
        for b, l in order:
            dims = mlp[b]
            ents = []
            for i in range(len(dims) - 1):
                ents += [("weight", (dims[i + 1], dims[i])), ("bias", (dims[i + 1],))]
            if b != 4:
                ents += [("gamma", (H,)), ("beta", (H,))]
            for t, (kind, shape) in enumerate(ents):
                out.append((b, l, t, kind, shape, self.param_offset(b, l, t)))
        return out


def _i32(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.int32)


def _ptr32(a: np.ndarray):
    return a.ctypes.data_as(C.POINTER(C.c_int32))


def _dev(t: torch.Tensor, dtype=torch.float32) -> int:
    if not t.is_cuda or t.dtype != dtype or not t.is_contiguous():
        raise ValueError("expected a contiguous device tensor of dtype %s" % dtype)
    return t.data_ptr()


def _stream(stream=None) -> int:
    s = stream if stream is not None else torch.cuda.current_stream()
    return s.cuda_stream


class Graph:
    """Receiver-sorted CSR graph (library handle)."""

    def __init__(self, handle):
        self._h = handle

    @classmethod
    def from_csr(cls, row_ptr, col) -> "Graph":
        rp, cl = _i32(row_ptr), _i32(col)
        h = C.c_void_p()
        check(lib.xmgn_graph_from_csr(len(rp) - 1, _ptr32(rp), _ptr32(cl) if len(cl) else None, C.byref(h)))
        return cls(h)

    def info(self):
        n, e = C.c_int32(), C.c_int64()
        check(lib.xmgn_graph_info(self._h, C.byref(n), C.byref(e)))
        return n.value, e.value

    def export(self):
        n, e = self.info()
        rp = np.zeros(n + 1, np.int32)
        cl = np.zeros(max(e, 1), np.int32)
        check(lib.xmgn_graph_export(self._h, _ptr32(rp), _ptr32(cl)))
        return rp, cl[:e]

    def __del__(self, _destroy=lib.xmgn_graph_destroy):
        if getattr(self, "_h", None):
            _destroy(self._h)
            self._h = None


class Partset:
    """Partitions with halos (library handle)."""

    def __init__(self, handle):
        self._h = handle

    @classmethod
    def halo(cls, graph: Graph, pos: np.ndarray, sizes, halo_hops: int) -> "Partset":
        p = np.ascontiguousarray(pos, dtype=np.float32)
        sz = None if sizes is None else _i32(sizes)
        n_parts = 1 if sizes is None else len(sz)
        h = C.c_void_p()
        check(lib.xmgn_partition_halo(graph._h, p.ctypes.data_as(C.POINTER(C.c_float)), n_parts,
                                      None if sz is None else _ptr32(sz), halo_hops, C.byref(h)))
        return cls(h)

    @classmethod
    def explicit(cls, graph: Graph, inner_lists, halo_hops: int) -> "Partset":
        counts = _i32([len(x) for x in inner_lists])
        flat = _i32(np.concatenate([np.asarray(x) for x in inner_lists]))
        h = C.c_void_p()
        check(lib.xmgn_partition_explicit(graph._h, len(counts), _ptr32(counts), _ptr32(flat), halo_hops,
                                          C.byref(h)))
        return cls(h)

    def count(self):
        n, g = C.c_int32(), C.c_int32()
        check(lib.xmgn_partset_count(self._h, C.byref(n), C.byref(g)))
        return n.value, g.value

    def info(self, part: int):
        ni, nh, ne = C.c_int32(), C.c_int32(), C.c_int64()
        check(lib.xmgn_partset_info(self._h, part, C.byref(ni), C.byref(nh), C.byref(ne)))
        return ni.value, nh.value, ne.value

    def export(self, part: int):
        ni, nh, ne = self.info(part)
        nl = ni + nh
        gid = np.zeros(nl, np.int32)
        hop = np.zeros(nl, np.int32)
        rp = np.zeros(nl + 1, np.int32)
        cl = np.zeros(max(ne, 1), np.int32)
        check(lib.xmgn_partset_export(self._h, part, _ptr32(gid), _ptr32(hop), _ptr32(rp), _ptr32(cl)))
        return dict(gid=gid, hop=hop, row_ptr=rp, col=cl[:ne], n_inner=ni)

    def __del__(self, _destroy=lib.xmgn_partset_destroy):
        if getattr(self, "_h", None):
            _destroy(self._h)
            self._h = None


class Context:
    """Device context: workspace, tape and cached batch plans."""

    def __init__(self, device: int = 0):
        h = C.c_void_p()
        check(lib.xmgn_ctx_create(device, C.byref(h)))
        self._h = h
        self.device = device

    def set_tiles(self, edge_rows: int = 0, node_rows: int = 0, grid: int = 0, edge_waves: int = 0):
        check(lib.xmgn_ctx_set_tiles(self._h, edge_rows, node_rows, grid, edge_waves))

    def set_bwd_tiles(self, edge_rows: int = 0, edge_waves: int = 0):
        """Rows per edge tile and waves per workgroup of the edge adjoint
        (0 = the forward's)."""
        check(lib.xmgn_ctx_set_bwd_tiles(self._h, edge_rows, edge_waves))

    def get_bwd_tiles(self) -> tuple[int, int]:
        """(edge rows, edge waves) of the edge adjoint; 0 = the forward's."""
        r, w = C.c_int32(), C.c_int32()
        check(lib.xmgn_ctx_get_bwd_tiles(self._h, C.byref(r), C.byref(w)))
        return r.value, w.value

    def set_timing(self, enable: bool):
        check(lib.xmgn_ctx_set_timing(self._h, 1 if enable else 0))

    def timings(self) -> dict:
        """{kernel class: (total_ms, launches)} since set_timing(True)."""
        n = C.c_int32()
        check(lib.xmgn_ctx_timing_count(self._h, C.byref(n)))
        out = {}
        for i in range(n.value):
            buf = C.create_string_buffer(64)
            ms, cnt = C.c_double(), C.c_int64()
            check(lib.xmgn_ctx_timing_read(self._h, i, buf, 64, C.byref(ms), C.byref(cnt)))
            out[buf.value.decode()] = (ms.value, cnt.value)
        return out

    def tape_serial(self) -> int:
        """Serial of the tape the next backward would consume (0 = none)."""
        n = C.c_int64()
        check(lib.xmgn_ctx_tape_serial(self._h, C.byref(n)))
        return n.value

    def memory(self) -> int:
        """Device bytes held by the context."""
        b = C.c_int64()
        check(lib.xmgn_ctx_memory(self._h, C.byref(b)))
        return b.value

    def host_memory(self) -> int:
        """Page-locked host bytes held by the context (the offloaded tape)."""
        b = C.c_int64()
        check(lib.xmgn_ctx_host_memory(self._h, C.byref(b)))
        return b.value

    def set_tape(self, keep_hidden: bool):
        """Tape policy: keep the edge MLPs' hidden activations (BF16 forms) or
        recompute them from the checkpoints (synchronises the device)."""
        check(lib.xmgn_ctx_set_tape(self._h, 1 if keep_hidden else 0))

    def get_tape(self) -> bool:
        v = C.c_int32()
        check(lib.xmgn_ctx_get_tape(self._h, C.byref(v)))
        return bool(v.value)

    def set_edge_split(self, split: bool):
        """Edge forward form: the first layer re-associated over its input
        blocks (node projections of W1, Eq. 1) instead of the gathered 3H
        product; used where no adjoint recomputes that product."""
        check(lib.xmgn_ctx_set_edge_split(self._h, 1 if split else 0))

    def get_edge_split(self) -> bool:
        v = C.c_int32()
        check(lib.xmgn_ctx_get_edge_split(self._h, C.byref(v)))
        return bool(v.value)

    def set_offload(self, enable: bool):
        """Keep the training tape's checkpoints in host memory (synchronises the device)."""
        check(lib.xmgn_ctx_set_offload(self._h, 1 if enable else 0))

    def build_knn(self, pos: torch.Tensor, level_end, k_intra: int, k_cross: int = 0, stream=None) -> Graph:
        le = _i32(level_end)
        h = C.c_void_p()
        check(lib.xmgn_build_knn(self._h, _dev(pos), pos.shape[0], _ptr32(le), len(le), k_intra, k_cross,
                                 C.byref(h), _stream(stream)))
        return Graph(h)

    def forward(self, model: Model, params: torch.Tensor, ps: Partset, part_ids, node_in: torch.Tensor,
                pos: torch.Tensor, edge_norm, out: torch.Tensor, keep_tape: bool = True, stream=None):
        ids = _i32(part_ids)
        en = np.ascontiguousarray(edge_norm, dtype=np.float32).reshape(-1)
        # the backward re-reads node_in and pos: keep them alive until then
        self._fwd_refs = (params, node_in)
        check(lib.xmgn_forward(self._h, C.byref(model.desc()), _dev(params), ps._h, _ptr32(ids), len(ids),
                               _dev(node_in), _dev(pos), en.ctypes.data_as(C.POINTER(C.c_float)), _dev(out),
                               1 if keep_tape else 0, _stream(stream)))

    def autotune(self, model: Model, params: torch.Tensor, ps: Partset, part_ids, node_in: torch.Tensor,
                 pos: torch.Tensor, edge_norm, out: torch.Tensor, d_out: torch.Tensor, d_params: torch.Tensor,
                 cache_path: str | None = None, stream=None):
        """Pick the fastest tile configuration for this batch (see
        xmgn_autotune); returns (edge_rows, node_rows, grid, edge_waves, step_ms)."""
        ids = _i32(part_ids)
        en = np.ascontiguousarray(edge_norm, dtype=np.float32).reshape(-1)
        self._fwd_refs = (params, node_in)
        er, nr, g, wv, ms = C.c_int32(), C.c_int32(), C.c_int32(), C.c_int32(), C.c_float()
        check(lib.xmgn_autotune(self._h, C.byref(model.desc()), _dev(params), ps._h, _ptr32(ids), len(ids),
                                _dev(node_in), _dev(pos), en.ctypes.data_as(C.POINTER(C.c_float)), _dev(out),
                                _dev(d_out), _dev(d_params), cache_path.encode() if cache_path else None,
                                C.byref(er), C.byref(nr), C.byref(g), C.byref(wv), C.byref(ms), _stream(stream)))
        return er.value, nr.value, g.value, wv.value, ms.value

    def mse_grad(self, out: torch.Tensor, target: torch.Tensor, n_total: int, d_out: torch.Tensor,
                 loss: torch.Tensor, stream=None):
        check(lib.xmgn_mse_grad(self._h, _dev(out), _dev(target), n_total, _dev(d_out), _dev(loss),
                                _stream(stream)))

    def backward(self, model: Model, params: torch.Tensor, d_out: torch.Tensor, d_params: torch.Tensor,
                 stream=None):
        check(lib.xmgn_backward(self._h, C.byref(model.desc()), _dev(params), _dev(d_out), _dev(d_params),
                                _stream(stream)))

    def __del__(self, _destroy=lib.xmgn_ctx_destroy):
        if getattr(self, "_h", None):
            _destroy(self._h)
            self._h = None


def grad_accumulate(acc: torch.Tensor, g: torch.Tensor, stream=None):
    if acc.numel() != g.numel():
        raise ValueError("size mismatch")
    check(lib.xmgn_grad_accumulate(_dev(acc), _dev(g), acc.numel(), _stream(stream)))


def cosine_lr(t: int, total: int, lr_max: float, lr_min: float) -> float:
    return float(lib.xmgn_cosine_lr(t, total, lr_max, lr_min))


class Adam:
    """Optimizer state (m, v, step) for xmgn_adam_step on one parameter blob."""

    def __init__(self, ctx: Context, params: torch.Tensor, betas=(0.9, 0.999), eps: float = 1e-8,
                 clip_norm: float = 32.0):
        self.ctx, self.params = ctx, params
        self.m = torch.zeros_like(params)
        self.v = torch.zeros_like(params)
        self.norm = torch.zeros(1, device=params.device)
        self.betas, self.eps, self.clip_norm = betas, eps, clip_norm
        self.t = 0

    def step(self, grad: torch.Tensor, lr: float, stream=None):
        if grad.numel() != self.params.numel():
            raise ValueError("size mismatch")
        check(lib.xmgn_adam_step(self.ctx._h, _dev(self.params), _dev(grad), _dev(self.m), _dev(self.v),
                                 self.params.numel(), self.t + 1, lr, self.betas[0], self.betas[1], self.eps,
                                 self.clip_norm, _dev(self.norm), _stream(stream)))
        self.t += 1


def adam_step_noalloc(params: torch.Tensor, grad: torch.Tensor, m: torch.Tensor, v: torch.Tensor, step: int,
                      lr: float, betas=(0.9, 0.999), eps: float = 1e-8, clip_norm: float = 32.0,
                      grad_norm: torch.Tensor | None = None, stream=None):
    """One Adam step through xmgn_adam_step_noalloc (no context, allocates
    nothing; see include/xmgn.h) on the tensors' device."""
    n = params.numel()
    if not (grad.numel() == m.numel() == v.numel() == n):
        raise ValueError("size mismatch")
    check(lib.xmgn_adam_step_noalloc(params.device.index or 0, _dev(params), _dev(grad), _dev(m), _dev(v), n, step,
                                     lr, betas[0], betas[1], eps, clip_norm,
                                     None if grad_norm is None else _dev(grad_norm), _stream(stream)))


class ProcessorFn(torch.autograd.Function):
    """out = X-MeshGraphNet(params) on a batch of partitions; backward returns
    d_params through the hand-written adjoint (xmgn_backward), which
    recomputes every layer from the context's checkpoints.

    A context holds the tape of its last forward only.  The backward of an
    application whose tape a later forward on the same context replaced
    raises XmgnError (code XMGN_ERR_STATE) instead of returning the gradient
    of another batch; give each application that must stay differentiable a
    context of its own, or run its backward before the next forward."""

    @staticmethod
    def forward(fctx, params, node_in, pos, ctx: Context, model: Model, ps: Partset, part_ids, edge_norm):
        out = torch.zeros(node_in.shape[0], model.out_dim, device=params.device, dtype=torch.float32)
        ctx.forward(model, params, ps, part_ids, node_in, pos, edge_norm, out, keep_tape=True)
        fctx.xm = (ctx, model, ctx.tape_serial())
        fctx.save_for_backward(params)
        return out

    @staticmethod
    def backward(fctx, d_out):
        ctx, model, serial = fctx.xm
        if ctx.tape_serial() != serial:
            raise XmgnError(-6, "the context's tape belongs to a later forward: this application's "
                                "checkpoints are gone (run its backward before the next forward on "
                                "the context, or give it a context of its own)")
        (params,) = fctx.saved_tensors
        d_params = torch.empty_like(params)
        ctx.backward(model, params, d_out.contiguous(), d_params)
        return d_params, None, None, None, None, None, None, None


__all__ = ["Model", "Graph", "Partset", "Context", "ProcessorFn", "grad_accumulate", "XmgnError"]
