"""MI355X blockBP surface-code decoder (arXiv 2402.04834): Python front end of libbbp.so.

The functions below marshal arguments into the C ABI of include/bbp.h; PyTorch provides device memory
and streams. Nothing here computes any step of the decoder, and there is no CPU fallback: on a machine
without the built library or without a GPU the calls fail.
"""
from __future__ import annotations

import ctypes as C

import numpy as np

from . import _lib
from ._lib import BbpError, bbp_group, bbp_opts, bbp_plan_info, bbp_timing, bbp_tuning, default_opts

__all__ = ["default_opts", "plan_query", "build_network", "workspace_size", "decode_device", "decode_groups",
           "decode_device_noalloc", "noalloc_max_batch",
           "autotune", "set_tuning", "blockbp_decode", "reference_update_host", "BbpError", "bbp_opts",
           "bbp_timing", "bbp_tuning"]


def plan_query(d: int, opts: bbp_opts) -> bbp_plan_info:
    info = bbp_plan_info()
    _lib.check(_lib.lib().bbp_plan_query(d, C.byref(opts), C.byref(info)))
    return info


class Network:
    """Host-side network of one syndrome (owns a bbp_net)."""

    def __init__(self, d: int, p: float, syndrome):
        s = np.ascontiguousarray(np.asarray(syndrome, dtype=np.uint8))
        h = C.c_void_p()
        _lib.check(_lib.lib().bbp_build_network(d, p, s.ctypes.data, s.size, C.byref(h)))
        self.handle = h
        self.d = d

    def labels(self) -> np.ndarray:
        L = 2 * self.d - 1
        out = np.zeros((4, L, L), dtype=np.uint8)
        _lib.check(_lib.lib().bbp_net_labels(self.handle, out.ctypes.data))
        return out

    def dims(self):
        d, n, m = C.c_int32(), C.c_int32(), C.c_int32()
        _lib.check(_lib.lib().bbp_net_dims(self.handle, C.byref(d), C.byref(n), C.byref(m)))
        return d.value, n.value, m.value

    def __del__(self):
        if getattr(self, "handle", None):
            _lib.lib().bbp_free_network(self.handle)
            self.handle = None


def build_network(d: int, p: float, syndrome) -> Network:
    return Network(d, p, syndrome)


def workspace_size(d: int, batch: int, opts: bbp_opts) -> int:
    n = C.c_size_t()
    _lib.check(_lib.lib().bbp_workspace_size(d, batch, C.byref(opts), C.byref(n)))
    return n.value


def _outputs(batch, n, dev):
    import torch
    return dict(
        loglik=torch.empty((batch, 4), dtype=torch.float64, device=dev),
        delta=torch.empty((batch, 4), dtype=torch.float64, device=dev),
        iters=torch.empty((batch, 4), dtype=torch.int32, device=dev),
        coset=torch.empty((batch,), dtype=torch.uint8, device=dev),
        correction=torch.empty((batch, n), dtype=torch.uint8, device=dev),
    )


def decode_device(d: int, p: float, syndromes, opts: bbp_opts, *, workspace=None, messages: bool = False,
                  timing: bool = False, stream=None, out=None):
    """Decode a batch of syndromes held in a torch uint8 CUDA tensor [batch, m].
    Returns a dict of torch tensors on the same device (loglik, delta, iters, coset, correction and
    optionally messages) plus a bbp_timing when requested. Work is enqueued on torch's current stream
    (or `stream`). `out` (a dict returned by an earlier call of the same shape) receives the results in
    place, which keeps the arguments of a graph-mode decode identical between calls."""
    import torch

    assert syndromes.is_cuda and syndromes.dtype == torch.uint8 and syndromes.dim() == 2
    syndromes = syndromes.contiguous()
    batch = syndromes.shape[0]
    dev = syndromes.device
    n = d * d + (d - 1) * (d - 1)
    ws_bytes = workspace_size(d, batch, opts)
    if workspace is None or workspace.numel() < ws_bytes:
        workspace = torch.empty(max(ws_bytes, 1), dtype=torch.uint8, device=dev)
    if out is None:
        out = _outputs(batch, n, dev)
    else:
        assert out["loglik"].shape == (batch, 4) and out["correction"].shape == (batch, n)
        out = {k: v for k, v in out.items() if k in ("loglik", "delta", "iters", "coset", "correction")}
    msg_ptr = None
    if messages:
        info = plan_query(d, opts)
        out["messages"] = torch.empty((batch, 4, max(info.num_messages, 1), info.message_stride),
                                      dtype=torch.float32, device=dev)
        msg_ptr = out["messages"].data_ptr()
    st = (stream if stream is not None else torch.cuda.current_stream(dev)).cuda_stream
    tm = bbp_timing() if timing else None
    _lib.check(_lib.lib().bbp_decode_device(
        d, p, syndromes.data_ptr(), batch, C.byref(opts), workspace.data_ptr(), workspace.numel(),
        out["loglik"].data_ptr(), out["delta"].data_ptr(), out["iters"].data_ptr(), out["coset"].data_ptr(),
        out["correction"].data_ptr(), msg_ptr, st, C.byref(tm) if tm is not None else None))
    if tm is not None:
        out["timing"] = tm
    out["workspace"] = workspace
    return out


def noalloc_max_batch(d: int, opts: bbp_opts) -> int:
    """Largest batch that bbp_decode_device_noalloc accepts for distance d under opts."""
    n = C.c_int64(0)
    _lib.check(_lib.lib().bbp_noalloc_max_batch(d, C.byref(opts), C.byref(n)))
    return n.value


def decode_device_noalloc(d: int, p: float, syndromes, opts: bbp_opts, *, stream=None, out=None):
    """The allocation-free decode (bbp_decode_device_noalloc) of a torch uint8 CUDA tensor [batch, m]: the
    library's static device array holds its workspace; `out` (a dict of output tensors as returned by
    decode_device) receives the results, else they are allocated here, before the call."""
    import torch

    assert syndromes.is_cuda and syndromes.dtype == torch.uint8 and syndromes.dim() == 2
    syndromes = syndromes.contiguous()
    batch = syndromes.shape[0]
    dev = syndromes.device
    n = d * d + (d - 1) * (d - 1)
    if out is None:
        out = _outputs(batch, n, dev)
    st = (stream if stream is not None else torch.cuda.current_stream(dev)).cuda_stream
    _lib.check(_lib.lib().bbp_decode_device_noalloc(
        d, p, syndromes.data_ptr(), batch, C.byref(opts), out["loglik"].data_ptr(), out["delta"].data_ptr(),
        out["iters"].data_ptr(), out["coset"].data_ptr(), out["correction"].data_ptr(), st))
    return out


def bmps_workspace_size(d: int, batch: int, chi: int = 16) -> int:
    n = C.c_size_t(0)
    _lib.check(_lib.lib().bbp_bmps_workspace_size(d, batch, chi, C.byref(n)))
    return n.value


def bmps_decode(d: int, p, syndromes, chi: int = 16, *, workspace=None, correction: bool = True,
                timing: bool = False, stream=None):
    """Boundary-MPS decoder (the single-block limit of blockBP) on a torch uint8 CUDA tensor [batch, m] of
    syndromes: p is a float (depolarizing rate), a float64 CUDA tensor [batch] of per-syndrome rates or a
    4-sequence of Pauli probabilities (I, X, Z, Y). Returns a dict of torch tensors (loglik [batch, 4],
    coset [batch], correction [batch, n] unless correction=False), the workspace, and with timing=True the
    contraction kernel's duration in ms ('kernel_ms', measured with HIP events on the stream)."""
    import torch

    assert syndromes.is_cuda and syndromes.dtype == torch.uint8 and syndromes.dim() == 2
    syndromes = syndromes.contiguous()
    batch = syndromes.shape[0]
    dev = syndromes.device
    n = d * d + (d - 1) * (d - 1)
    ws_bytes = bmps_workspace_size(d, batch, chi)
    if workspace is None or workspace.numel() < ws_bytes:
        workspace = torch.empty(max(ws_bytes, 1), dtype=torch.uint8, device=dev)
    pval, p_ptr, noise, keep = 0.0, None, None, None
    if isinstance(p, torch.Tensor):
        keep = p.to(device=dev, dtype=torch.float64).contiguous()
        p_ptr = keep.data_ptr()
    elif isinstance(p, (tuple, list)):
        noise = (C.c_double * 4)(*[float(v) for v in p])
    else:
        pval = float(p)
    out = dict(loglik=torch.empty((batch, 4), dtype=torch.float64, device=dev),
               coset=torch.empty(batch, dtype=torch.uint8, device=dev))
    if correction:
        out["correction"] = torch.empty((batch, n), dtype=torch.uint8, device=dev)
    st = (stream if stream is not None else torch.cuda.current_stream(dev)).cuda_stream
    ms = C.c_float(0.0)
    _lib.check(_lib.lib().bbp_bmps_decode_device(
        d, pval, p_ptr, noise, syndromes.data_ptr(), batch, chi, workspace.data_ptr(), workspace.numel(),
        out["loglik"].data_ptr(), out["coset"].data_ptr(),
        out["correction"].data_ptr() if correction else None, st, C.byref(ms) if timing else None))
    if timing:
        out["kernel_ms"] = ms.value
    out["workspace"] = workspace
    return out


def decode_groups(groups, opts: bbp_opts, *, workspace=None, timing: bool = False, stream=None, outs=None,
                  messages: bool = False):
    """Decode a mixed batch: `groups` is a list of (d, p, syndromes[, chi[, init]]) with syndromes a torch
    uint8 CUDA tensor [batch, 2d(d-1)], p a float (depolarizing rate), a float64 CUDA tensor [batch] of
    per-syndrome depolarizing rates or a 4-sequence of Pauli probabilities (I, X, Z, Y) for biased noise,
    chi the group's bond dimension (0 or absent: opts.chi) and init optional start messages (float32
    CUDA tensor [batch, 4, M, S] with S the plan's message_stride, e.g. from warm.predict; None: the uniform
    start). Returns (list of
    per-group output dicts as in decode_device, workspace, bbp_timing or None). `outs` (from an earlier
    call with the same groups) receives the results in place, keeping graph-mode arguments identical.
    messages=True adds each group's final messages [batch, 4, M, S] as 'messages'."""
    import torch

    gs = (bbp_group * len(groups))()
    outs_in = outs
    outs, keep = [], []
    dev = None
    for k, grp in enumerate(groups):
        d, p, syn = grp[:3]
        chi = grp[3] if len(grp) > 3 else 0
        init = grp[4] if len(grp) > 4 else None
        assert syn.is_cuda and syn.dtype == torch.uint8 and syn.dim() == 2
        syn = syn.contiguous()
        keep.append(syn)
        dev = syn.device
        b = syn.shape[0]
        p_ptr, p_val, noise = None, p, (0.0, 0.0, 0.0, 0.0)
        if isinstance(p, (tuple, list, np.ndarray)):      # biased noise: probabilities of I, X, Z, Y
            assert len(p) == 4
            noise, p_val = tuple(float(v) for v in p), 0.0
        elif torch.is_tensor(p):
            assert p.is_cuda and p.dtype == torch.float64 and p.shape == (b,)
            p = p.contiguous()
            keep.append(p)
            p_ptr, p_val = p.data_ptr(), 0.0
        o = outs_in[k] if outs_in is not None else _outputs(b, d * d + (d - 1) * (d - 1), dev)
        outs.append(o)
        init_ptr = None
        if init is not None:
            assert init.is_cuda and init.dtype == torch.float32 and init.shape[0] == b and init.shape[1] == 4
            init = init.contiguous()
            keep.append(init)
            init_ptr = init.data_ptr()
        msg_ptr = None
        if messages:
            if "messages" not in o:
                info = plan_query(d, _with_chi(opts, chi))
                o["messages"] = torch.empty((b, 4, max(info.num_messages, 1), info.message_stride),
                                            dtype=torch.float32, device=dev)
            msg_ptr = o["messages"].data_ptr()
        gs[k] = bbp_group(d, chi, p_val, p_ptr, syn.data_ptr(), b, o["loglik"].data_ptr(), o["delta"].data_ptr(),
                          o["iters"].data_ptr(), o["coset"].data_ptr(), o["correction"].data_ptr(), init_ptr,
                          msg_ptr, (C.c_double * 4)(*noise))
    n = C.c_size_t()
    _lib.check(_lib.lib().bbp_workspace_size_groups(gs, len(groups), C.byref(opts), C.byref(n)))
    if workspace is None or workspace.numel() < n.value:
        workspace = torch.empty(max(n.value, 1), dtype=torch.uint8, device=dev)
    st = (stream if stream is not None else torch.cuda.current_stream(dev)).cuda_stream
    tm = bbp_timing() if timing else None
    _lib.check(_lib.lib().bbp_decode_groups(gs, len(groups), C.byref(opts), workspace.data_ptr(),
                                            workspace.numel(), st, C.byref(tm) if tm is not None else None))
    return outs, workspace, tm


def _with_chi(opts: bbp_opts, chi: int) -> bbp_opts:
    o = bbp_opts.from_buffer_copy(opts)
    if chi:
        o.chi = chi
    return o


def autotune(d: int, p: float, syndromes, opts: bbp_opts, *, workspace=None, stream=None) -> bbp_tuning:
    """Time the launch variants of the block sweeps on this batch and keep the fastest for (d, opts)."""
    import torch

    syndromes = syndromes.contiguous()
    ws_bytes = workspace_size(d, syndromes.shape[0], opts)
    if workspace is None or workspace.numel() < ws_bytes:
        workspace = torch.empty(max(ws_bytes, 1), dtype=torch.uint8, device=syndromes.device)
    st = (stream if stream is not None else torch.cuda.current_stream(syndromes.device)).cuda_stream
    best = bbp_tuning()
    _lib.check(_lib.lib().bbp_autotune(d, p, syndromes.data_ptr(), syndromes.shape[0], C.byref(opts),
                                       workspace.data_ptr(), workspace.numel(), st, C.byref(best)))
    return best


def set_tuning(d: int, opts: bbp_opts, order: int, streams: int) -> None:
    t = bbp_tuning(order, streams, 0.0)
    _lib.check(_lib.lib().bbp_set_tuning(d, C.byref(opts), C.byref(t)))


def blockbp_decode(nets, opts: bbp_opts):
    """Host convenience: decode a list of Network objects (up to 8 distinct (d, p), any order); returns
    numpy outputs in input order, correction rows of the largest qubit count."""
    batch = len(nets)
    n = max(x.dims()[1] for x in nets)
    arr = (C.c_void_p * batch)(*[x.handle.value for x in nets])
    ll = np.zeros((batch, 4)); dl = np.zeros((batch, 4)); it = np.zeros((batch, 4), dtype=np.int32)
    cs = np.zeros(batch, dtype=np.uint8); corr = np.zeros((batch, n), dtype=np.uint8)
    _lib.check(_lib.lib().bbp_blockbp_decode(arr, batch, C.byref(opts), ll.ctypes.data, dl.ctypes.data,
                                             it.ctypes.data, cs.ctypes.data, corr.ctypes.data))
    return dict(loglik=ll, delta=dl, iters=it, coset=cs, correction=corr)


def reference_update_host(d: int, p: float, opts: bbp_opts, labels, msg_id: int, msgs):
    """Validation hook of the C ABI (host float64 evaluation of one block sweep with the kernel's index
    arithmetic). Returns (state vector of 2^kp entries, log-scale)."""
    labels = np.ascontiguousarray(np.asarray(labels, dtype=np.uint8))
    msgs = np.ascontiguousarray(np.asarray(msgs, dtype=np.float64))
    out = np.zeros(64)
    ls = C.c_double()
    _lib.check(_lib.lib().bbp_reference_update_host(d, p, C.byref(opts), labels.ctypes.data, msg_id,
                                                    msgs.ctypes.data, out.ctypes.data, C.byref(ls)))
    return out, ls.value
