"""Learned warm start of blockBP: binding of the network entry points of libbbp.so (argument marshalling;
the forward, backward and optimiser steps all run in the library's kernels), the training loop that fits
the network to converged cold-start messages, and the warm-started decode with its cold fallback.

BP of blockBP starts from uniform messages (Alg. 1, remark 2); the paper lists machine learning among the
ways to improve BP (Sec. V). The network and its loss are described in include/bbp.h.
"""
from __future__ import annotations

import ctypes as C
import os
import time

import numpy as np

from . import _lib
from ._lib import bbp_opts

HERE = os.path.dirname(os.path.abspath(__file__))
WEIGHTS_PATH = os.path.join(HERE, "weights", "warmstart_d13-21.npy")
CHANNELS = (11, 64, 128, 96)


def param_count() -> int:
    n = C.c_int64()
    _lib.check_warm(_lib.lib().bbp_warm_param_count(C.byref(n)))
    return n.value


def _sizes():
    c0, c1, c2, c3 = CHANNELS
    out = [(9 * c0, c1), (c1,), (9 * c1, c2), (c2,), (9 * c2, c3), (c3,)]
    for _ in range(4):
        out += [(2 * c3, 2), (2,), (4 * c3, 4), (4,)]
    return out


def init_params(seed: int = 0) -> np.ndarray:
    """He-normal convolution weights, zero biases, small head weights (start messages near uniform)."""
    g = np.random.Generator(np.random.PCG64(np.random.SeedSequence(seed)))
    parts = []
    for k, s in enumerate(_sizes()):
        if len(s) == 1:
            parts.append(np.zeros(s))
        elif k < 6:
            parts.append(g.standard_normal(s) * np.sqrt(2.0 / s[0]))
        else:
            parts.append(g.standard_normal(s) * (0.1 / np.sqrt(s[0])))
    theta = np.concatenate([x.ravel() for x in parts]).astype(np.float32)
    assert theta.size == param_count()
    return theta


def load(path: str = WEIGHTS_PATH) -> np.ndarray:
    theta = np.load(path, allow_pickle=False)
    assert theta.dtype == np.float32 and theta.shape == (param_count(),), "weights of another network"
    return theta


def save(theta, path: str = WEIGHTS_PATH) -> None:
    os.makedirs(os.path.dirname(path), exist_ok=True)
    np.save(path, np.asarray(theta, dtype=np.float32), allow_pickle=False)


def _stream(stream, dev):
    import torch
    return (stream if stream is not None else torch.cuda.current_stream(dev)).cuda_stream


def _p_args(p, b):
    import torch
    if torch.is_tensor(p):
        assert p.is_cuda and p.dtype == torch.float64 and p.shape == (b,)
        return 0.0, p.contiguous()
    return float(p), None


def workspace_size(d: int, batch: int, opts: bbp_opts, train: bool) -> int:
    n = C.c_size_t()
    _lib.check_warm(_lib.lib().bbp_warm_workspace_size(d, batch, C.byref(opts), int(train), C.byref(n)))
    return n.value


def predict(d: int, p, syndromes, opts: bbp_opts, params, *, precision: int = 1, workspace=None, stream=None):
    """Start messages [batch, 4, M, 64] (float32, unit norm) for syndromes [batch, m] (uint8 CUDA).
    precision 1: BF16 weights and activations, FP32 accumulation (inference); 0: FP32 throughout."""
    import torch
    syndromes = syndromes.contiguous()
    b, dev = syndromes.shape[0], syndromes.device
    M = max(_plan_messages(d, opts), 1)
    out = torch.empty((b, 4, M, 64), dtype=torch.float32, device=dev)
    ws_bytes = workspace_size(d, b, opts, False)
    if workspace is None or workspace.numel() < ws_bytes:
        workspace = torch.empty(ws_bytes, dtype=torch.uint8, device=dev)
    pv, pt = _p_args(p, b)
    _lib.check_warm(_lib.lib().bbp_warm_predict(
        d, pv, pt.data_ptr() if pt is not None else None, syndromes.data_ptr(), b, C.byref(opts),
        params.data_ptr(), precision, out.data_ptr(), workspace.data_ptr(), workspace.numel(), _stream(stream, dev)))
    return out


def _plan_messages(d, opts):
    from . import plan_query
    return plan_query(d, opts).num_messages


def loss_grad(d: int, p, syndromes, opts: bbp_opts, params, targets, use, *, workspace=None, stream=None):
    """(loss [1] float32, gradient [P] float32) of the mean over the messages of the used coset jobs of
    KL(q || softmax(s)), q the target message normalised to sum 1 and s the network's scores (the loss of
    bbp_warm_loss_grad); targets [batch, 4, M, 64] float32, use [batch * 4] uint8 (CUDA tensors)."""
    import torch
    syndromes = syndromes.contiguous()
    b, dev = syndromes.shape[0], syndromes.device
    M = _plan_messages(d, opts)
    assert targets.shape == (b, 4, max(M, 1), 64) and targets.dtype == torch.float32
    assert use.shape == (4 * b,) and use.dtype == torch.uint8
    n_used = int(use.sum().item())
    loss = torch.zeros(1, dtype=torch.float32, device=dev)
    grad = torch.empty_like(params)
    if n_used == 0 or M == 0:
        grad.zero_()
        return loss, grad
    ws_bytes = workspace_size(d, b, opts, True)
    if workspace is None or workspace.numel() < ws_bytes:
        workspace = torch.empty(ws_bytes, dtype=torch.uint8, device=dev)
    pv, pt = _p_args(p, b)
    targets, use = targets.contiguous(), use.contiguous()
    _lib.check_warm(_lib.lib().bbp_warm_loss_grad(
        d, pv, pt.data_ptr() if pt is not None else None, syndromes.data_ptr(), b, C.byref(opts),
        params.data_ptr(), targets.data_ptr(), use.data_ptr(), n_used * M, grad.data_ptr(), loss.data_ptr(),
        workspace.data_ptr(), workspace.numel(), _stream(stream, dev)))
    return loss, grad


def adam(params, grad, m, v, step: int, lr: float, *, stream=None) -> None:
    _lib.check_warm(_lib.lib().bbp_warm_adam(params.data_ptr(), grad.data_ptr(), m.data_ptr(), v.data_ptr(), step,
                                             lr, _stream(stream, params.device)))


def trained_range(path: str = WEIGHTS_PATH):
    """(smallest, largest) distance the weights at `path` were trained on, from their metadata file."""
    import json
    meta = json.load(open(os.path.splitext(path)[0] + ".json"))
    return min(meta["distances"]), max(meta["distances"])


def decode(d: int, p, syndromes, opts: bbp_opts, params, *, precision: int = 1, trained=None, workspace=None,
           stream=None, out=None):
    """Warm-started decode with cold fallback (bbp_warm_decode). `trained` = (smallest, largest) distance the
    parameters were trained on (default: the committed weights' range; None-equivalent (0, 0) disables the
    check): outside it the whole batch is decoded from the uniform start. Returns the output dict of
    decode_device plus 'fallback' (number of syndromes decoded from the uniform start)."""
    import torch
    from . import _outputs
    syndromes = syndromes.contiguous()
    b, dev = syndromes.shape[0], syndromes.device
    n = C.c_size_t()
    _lib.check_warm(_lib.lib().bbp_warm_decode_workspace_size(d, b, C.byref(opts), C.byref(n)))
    if workspace is None or workspace.numel() < n.value:
        workspace = torch.empty(n.value, dtype=torch.uint8, device=dev)
    if out is None:
        out = _outputs(b, d * d + (d - 1) * (d - 1), dev)
    pv, pt = _p_args(p, b)
    fb = C.c_int64()
    lo, hi = trained_range() if trained is None else trained
    _lib.check_warm(_lib.lib().bbp_warm_decode(
        d, pv, pt.data_ptr() if pt is not None else None, syndromes.data_ptr(), b, C.byref(opts),
        params.data_ptr(), precision, lo, hi, workspace.data_ptr(), workspace.numel(), out["loglik"].data_ptr(),
        out["delta"].data_ptr(),
        out["iters"].data_ptr(), out["coset"].data_ptr(), out["correction"].data_ptr(), C.byref(fb),
        _stream(stream, dev)))
    res = dict(out)
    res["fallback"] = fb.value
    res["workspace"] = workspace
    return res


# ------------------------------------------------------------------------------------------- training
TRAIN_DISTANCES = (13, 15, 17, 19, 21)
TRAIN_P = (0.05, 0.15)


def make_training_set(count: int, opts: bbp_opts, dev, log=print):
    """Training pool: `count` syndromes with d uniform over 13..21 (odd) and p uniform over [0.05, 0.15],
    each decoded cold on the GPU; targets are the final messages, used where the coset converged (final
    distance below delta0). Returns {d: dict(syn, p, targets, use)} of CUDA tensors."""
    import torch
    from . import decode_groups, workload
    items = workload.mixed_batch(count, distances=TRAIN_DISTANCES, p_range=TRAIN_P, workload="warm")
    pool = {}
    for d in TRAIN_DISTANCES:
        sel = [(p, s) for (dd, p, _, s) in items if dd == d]
        if not sel:
            continue
        syn = torch.from_numpy(np.stack([s for _, s in sel])).to(dev)
        pt = torch.tensor([p for p, _ in sel], dtype=torch.float64, device=dev)
        t0 = time.time()
        msgs, use = [], []
        for b0 in range(0, syn.shape[0], 4096):
            outs, _, _ = decode_groups([(d, pt[b0:b0 + 4096], syn[b0:b0 + 4096])], opts, messages=True)
            msgs.append(outs[0]["messages"])
            use.append((outs[0]["delta"] < opts.delta0).reshape(-1).to(torch.uint8))
        torch.cuda.synchronize()
        pool[d] = dict(syn=syn, p=pt, targets=torch.cat(msgs), use=torch.cat(use))
        log(f"[warm train] pool d={d}: {syn.shape[0]} syndromes, converged cosets "
            f"{int(pool[d]['use'].sum())}/{4 * syn.shape[0]}, {time.time() - t0:.1f} s")
    return pool


def train(pool, opts: bbp_opts, *, steps: int = 2000, batch: int = 16, lr: float = 1e-3, seed: int = 0,
          theta0=None, log=print, every: int = 100):
    """Adam on the loss of bbp_warm_loss_grad over minibatches drawn from the pool (one distance per step,
    cycling through the pool's distances; learning rate decayed from lr to lr / 10 along a cosine). Returns
    (parameters as a float32 CUDA tensor, loss history)."""
    import torch
    dev = next(iter(pool.values()))["syn"].device
    theta = torch.from_numpy(init_params(seed) if theta0 is None else np.asarray(theta0, np.float32)).to(dev)
    m, v = torch.zeros_like(theta), torch.zeros_like(theta)
    g = np.random.Generator(np.random.PCG64(np.random.SeedSequence(seed + 1)))
    ds = sorted(pool)
    ws = {}
    hist = []
    t0 = time.time()
    for step in range(1, steps + 1):
        # cosine decay from lr to lr / 10
        lr_t = lr * (0.1 + 0.45 * (1.0 + np.cos(np.pi * (step - 1) / max(steps - 1, 1))))
        d = ds[(step - 1) % len(ds)]
        P = pool[d]
        idx = torch.from_numpy(g.choice(P["syn"].shape[0], size=batch, replace=False)).to(dev)
        use = P["use"].view(-1, 4)[idx].reshape(-1).contiguous()
        if d not in ws:
            ws[d] = torch.empty(workspace_size(d, batch, opts, True), dtype=torch.uint8, device=dev)
        loss, grad = loss_grad(d, P["p"][idx].contiguous(), P["syn"][idx].contiguous(), opts, theta,
                               P["targets"][idx].contiguous(), use, workspace=ws[d])
        adam(theta, grad, m, v, step, lr_t)
        hist.append(loss)
        if step % every == 0 or step == steps:
            recent = torch.stack(hist[-every:]).mean().item()
            log(f"[warm train] step {step}/{steps} d={d} loss {recent:.5f} ({time.time() - t0:.1f} s)")
    torch.cuda.synchronize()
    return theta, torch.stack(hist).cpu().numpy().ravel()
