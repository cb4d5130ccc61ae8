"""GPU tests of the learned warm start: the network's forward (start messages) and its loss gradient
through the C ABI against the FP64 oracle (oracle/warmnet.py, full channel sizes), the decoder started
from given messages, the warm decode's cold fallback, training, and the gain of the committed weights.

Tolerances (FP32 products and sums in the GPU network): a forward value is a chain of three convolution
sums of at most 9 * 128 = 1152 terms and a head sum of 384 terms, so its relative rounding error is below
about (1152 + 576 + 72 + 384) * 2^-24 ~ 1.3e-4 of the sums of absolute values; messages are compared at
2e-4 absolute (entries of unit vectors). Gradients add a sum over all rows of the batch (<= 8 * 13^2 =
1352 terms), so their bound grows to about (2184 + 1352) * 2^-24 ~ 2e-4 relative: each parameter block is
compared at 2e-4 of its largest oracle entry (measured errors are about 1e-6 of it).
"""
import os
import sys

import numpy as np
import pytest

from oracle import blockbp, warmnet
from paper_2402_04834_amd import workload

pytestmark = pytest.mark.gpu

KEYS = ("loglik", "delta", "iters", "coset", "correction")


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def dev():
    import torch
    import paper_2402_04834_amd as bbp
    bbp._lib.lib()
    return torch.device("cuda:0")


def _theta(seed, head_scale=1.0):
    """Random parameters with head weights large enough that messages are far from uniform."""
    from paper_2402_04834_amd import warm
    th = warm.init_params(seed).astype(np.float64)
    parts = warmnet.unpack(th)
    rng = np.random.default_rng(seed + 7)
    for n, v in parts.items():
        if n.startswith("head"):
            parts[n] = rng.normal(size=v.shape) * head_scale / np.sqrt(v.shape[0] if v.ndim > 1 else 4)
        elif n.endswith(".b"):
            parts[n] = rng.normal(size=v.shape) * 0.1
    return warmnet.pack(parts).astype(np.float32)


def _oracle_jobs(d, syn, ps):
    """Input grids of every coset job, [batch * 4] in job order (4 * syndrome + coset)."""
    out = []
    for s, p in zip(syn, ps):
        for k in range(4):
            out.append(warmnet.features(d, s, p, k))
    return out


CASES = [(5, 3), (7, 4), (9, 6)]


@pytest.mark.parametrize("d,k", CASES)
def test_forward_messages_against_oracle(dev, d, k):
    import torch
    import paper_2402_04834_amd as bbp
    from paper_2402_04834_amd import warm
    b = 3
    _, syn = workload.make_batch(d, 0.1, b, workload="warm", p_index=200 + d)
    ps = np.array([0.06, 0.1, 0.14])
    th = _theta(d)
    opts = bbp.default_opts(block=k, chi=32)
    _say(f"[warm fwd] d={d} k={k} batch {b}")
    got = warm.predict(d, torch.from_numpy(ps).to(dev), torch.from_numpy(syn).to(dev), opts,
                       torch.from_numpy(th).to(dev), precision=0).cpu().numpy()
    torch.cuda.synchronize()
    plan = blockbp.Plan(d, k, k)
    for j, X0 in enumerate(_oracle_jobs(d, syn, ps)):
        ref = warmnet.predict(th.astype(np.float64), X0, d, plan)
        np.testing.assert_allclose(got[j // 4, j % 4, :plan.M], ref, atol=2e-4, err_msg=f"job {j}")
    # messages are far from uniform (the comparison is not trivial)
    assert np.abs(got[..., :8] - got[..., :1]).max() > 0.05


# d=25: the largest grid (L=49) of the haloed-tile convolutions, whose halo then fills its LDS rows exactly;
# d=27 (L=53): the gather kernels that serve larger grids
@pytest.mark.parametrize("d,k", [(5, 3), (9, 6), (25, 6), (27, 6)])
def test_bf16_forward_against_oracle(dev, d, k):
    """Inference precision: BF16 convolution weights, input channels and hidden activations, FP32 sums, the last
    convolution composed with the head (its per-site projections). The oracle runs the same arithmetic in FP64
    and rounds to BF16 at the same storage points (warmnet.predict_stored(store=round_bf16)), from the FP32
    parameters as the GPU does. What remains is FP32 against FP64 summation (<= K 2^-24 of the
    absolute sums, K <= 1152: about 1e-4 relative), which can also move a stored value across a BF16
    rounding midpoint -- one BF16 step, 2^-7 relative, at the rare positions where that happens. Both shift
    the scores s(b) by O(1e-3) nats, against score ranges of several nats here. Compared: log m(b) where the
    oracle's entry exceeds 1e-4, up to the common normalisation constant; tolerance 0.02 nats."""
    import torch
    import paper_2402_04834_amd as bbp
    from paper_2402_04834_amd import warm
    b = 2
    _, syn = workload.make_batch(d, 0.1, b, workload="warm", p_index=250 + d)
    ps = np.array([0.07, 0.13])
    th = _theta(d + 1)
    opts = bbp.default_opts(block=k, chi=32)
    _say(f"[warm bf16 fwd] d={d} k={k}")
    got = warm.predict(d, torch.from_numpy(ps).to(dev), torch.from_numpy(syn).to(dev), opts,
                       torch.from_numpy(th).to(dev), precision=1).cpu().numpy()
    torch.cuda.synchronize()
    plan = blockbp.Plan(d, k, k)
    worst, span = 0.0, 0.0
    for j, X0 in enumerate(_oracle_jobs(d, syn, ps)):
        ref = warmnet.predict_stored(th.astype(np.float64), X0, d, plan, warmnet.round_bf16)
        g = got[j // 4, j % 4, :plan.M]
        for e in range(plan.M):
            K = len(warmnet.legs(d, plan, e))
            r, q = ref[e, :2 ** K], g[e, :2 ** K]
            sel = r > 1e-4
            diff = np.log(np.maximum(q[sel], 1e-30)) - np.log(r[sel])
            worst = max(worst, float(diff.max() - diff.min()))
            span = max(span, float(np.log(r[sel]).max() - np.log(r[sel]).min()))
            assert diff.max() - diff.min() <= 0.02, (j, e, diff)
    _say(f"   largest log-message spread: {worst:.2e} nats (score differences up to {span:.1f} nats)")
    assert span > 1.0      # the comparison is not trivial


def test_bf16_forward_several_chunks(dev):
    """The inference forward runs in chunks of 512 syndromes (2048 coset jobs, one workspace slot set): a batch
    of 600 at d=9 takes two, the second ragged. Its messages equal those of the same syndromes forwarded in
    separate calls (512, then 88) bitwise -- a site's sums do not depend on where its tile starts -- and the
    first and last syndromes of both chunks match the oracle as in test_bf16_forward_against_oracle."""
    import torch
    import paper_2402_04834_amd as bbp
    from paper_2402_04834_amd import warm
    d, k, b = 9, 6, 600
    _, syn = workload.make_batch(d, 0.1, b, workload="warm", p_index=290)
    ps = np.random.default_rng(290).uniform(0.05, 0.15, size=b)
    th = _theta(29)
    opts = bbp.default_opts(block=k, chi=32)
    tp, ts, tt = torch.from_numpy(ps).to(dev), torch.from_numpy(syn).to(dev), torch.from_numpy(th).to(dev)
    _say(f"[warm bf16 chunks] d={d} batch {b}")
    whole = warm.predict(d, tp, ts, opts, tt, precision=1).cpu().numpy()
    parts = [warm.predict(d, tp[a:z], ts[a:z], opts, tt, precision=1).cpu().numpy() for a, z in ((0, 512), (512, b))]
    torch.cuda.synchronize()
    np.testing.assert_array_equal(whole, np.concatenate(parts))
    plan = blockbp.Plan(d, k, k)
    for i in (0, 511, 512, b - 1):
        for c in range(4):
            ref = warmnet.predict_stored(th.astype(np.float64), warmnet.features(d, syn[i], ps[i], c), d, plan,
                                         warmnet.round_bf16)
            for e in range(plan.M):
                K = len(warmnet.legs(d, plan, e))
                r, q = ref[e, :2 ** K], whole[i, c, e, :2 ** K]
                sel = r > 1e-4
                diff = np.log(np.maximum(q[sel], 1e-30)) - np.log(r[sel])
                assert diff.max() - diff.min() <= 0.02, (i, c, e, diff)


@pytest.mark.parametrize("d,k", [(5, 3), (7, 4)])
def test_loss_gradient_against_oracle(dev, d, k):
    import torch
    import paper_2402_04834_amd as bbp
    from paper_2402_04834_amd import warm
    b = 2
    _, syn = workload.make_batch(d, 0.1, b, workload="warm", p_index=300 + d)
    ps = np.array([0.08, 0.12])
    th = _theta(100 + d, head_scale=0.5)
    plan = blockbp.Plan(d, k, k)
    rng = np.random.default_rng(d)
    targets = np.zeros((b, 4, plan.M, 64), dtype=np.float32)
    for e, (src, dst, _) in enumerate(plan.edges):
        K = plan.msg_len(src, dst)
        t = rng.random((b, 4, 2 ** K)) + 0.05
        targets[:, :, e, :2 ** K] = t / np.linalg.norm(t, axis=-1, keepdims=True)
    use = np.array([1, 0, 1, 1, 1, 1, 0, 1], dtype=np.uint8)
    opts = bbp.default_opts(block=k, chi=32)
    _say(f"[warm grad] d={d} k={k} batch {b}, {int(use.sum())} used jobs")
    loss, grad = warm.loss_grad(d, torch.from_numpy(ps).to(dev), torch.from_numpy(syn).to(dev), opts,
                                torch.from_numpy(th).to(dev), torch.from_numpy(targets).to(dev),
                                torch.from_numpy(use).to(dev))
    torch.cuda.synchronize()
    loss, grad = float(loss.cpu()[0]), grad.cpu().numpy().astype(np.float64)
    _say(f"   loss {loss:.6f}")
    jobs = _oracle_jobs(d, syn, ps)
    ref_l, ref_g = 0.0, np.zeros(th.size)
    used = [j for j in range(4 * b) if use[j]]
    for j in used:
        l, g = warmnet.loss_and_grad(th.astype(np.float64), jobs[j], d, plan,
                                     targets[j // 4, j % 4].astype(np.float64), list(range(plan.M)))
        ref_l += l / len(used)
        ref_g += g / len(used)
    assert abs(loss - ref_l) <= 1e-5 + 1e-4 * abs(ref_l), (loss, ref_l)
    gp, rp = warmnet.unpack(grad), warmnet.unpack(ref_g)
    for n in rp:
        scale = np.abs(rp[n]).max()
        assert scale > 0, n
        err = np.abs(gp[n] - rp[n]).max()
        _say(f"   {n}: max|ref| {scale:.3e} max err {err:.3e}")
        assert err <= 2e-4 * scale, n


def _np(out):
    return {k: out[k].cpu().numpy() for k in KEYS}


def test_decode_from_converged_messages_exits_early(dev):
    """Started from the converged messages of a cold decode, BP is already at its fixed point: the first
    iteration's distance is below delta0 and the Bethe estimates equal the cold ones."""
    import torch
    import paper_2402_04834_amd as bbp
    d, p = 11, 0.1
    _, syn = workload.make_batch(d, p, 24, workload="warm", p_index=411)
    s = torch.from_numpy(syn).to(dev)
    opts = bbp.default_opts(block=6, chi=32, max_iter=40)
    _say("[warm init] cold decode with messages, then restart from them")
    cold, _, _ = bbp.decode_groups([(d, p, s)], opts, messages=True)
    hot, _, _ = bbp.decode_groups([(d, p, s, 0, cold[0]["messages"])], opts)
    torch.cuda.synchronize()
    c, h = _np(cold[0]), _np(hot[0])
    conv = np.all(c["delta"] < opts.delta0, axis=1)
    assert conv.sum() >= 16
    assert np.all(h["iters"][conv] == 1)
    np.testing.assert_allclose(h["loglik"][conv], c["loglik"][conv], atol=1e-3)
    assert np.all(h["coset"][conv] == c["coset"][conv])
    assert h["iters"].mean() < c["iters"].mean()


def test_uniform_given_messages_equal_default_start(dev):
    import torch
    import paper_2402_04834_amd as bbp
    d, p = 9, 0.1
    _, syn = workload.make_batch(d, p, 8, workload="warm", p_index=412)
    s = torch.from_numpy(syn).to(dev)
    opts = bbp.default_opts(block=6, chi=32, max_iter=20)
    M = bbp.plan_query(d, opts).num_messages
    plan = blockbp.Plan(d, 6, 6)
    init = torch.zeros((8, 4, M, 64), dtype=torch.float32, device=dev)
    for e, (src, dst, _) in enumerate(plan.edges):
        K = plan.msg_len(src, dst)
        init[:, :, e, :2 ** K] = 3.0      # any positive scale: the decoder normalises
    a, _, _ = bbp.decode_groups([(d, p, s)], opts)
    g, _, _ = bbp.decode_groups([(d, p, s, 0, init)], opts)
    torch.cuda.synchronize()
    A, G = _np(a[0]), _np(g[0])
    np.testing.assert_allclose(G["loglik"], A["loglik"], atol=1e-4)
    np.testing.assert_array_equal(G["coset"], A["coset"])


def test_warm_decode_fallback(dev):
    """bbp_warm_decode = predict + decode from the predicted messages, and every syndrome with a coset whose
    final distance is not below delta1, or whose decided coset took more iterations than another of its
    cosets, decoded again cold: its results are the cold decode's and its iteration counts the sum of both
    runs; the others keep the warm results. (No trained-range check: these parameters are a test network.)"""
    import torch
    import paper_2402_04834_amd as bbp
    from paper_2402_04834_amd import warm
    d, p, b = 9, 0.1, 16
    _, syn = workload.make_batch(d, p, b, workload="warm", p_index=413)
    s = torch.from_numpy(syn).to(dev)
    th = torch.from_numpy(_theta(5, head_scale=0.3)).to(dev)
    total_fb = 0
    for max_iter in (20, 3):
        opts = bbp.default_opts(block=6, chi=32, max_iter=max_iter)
        _say(f"[warm fallback] max_iter {max_iter}")
        cold = _np(bbp.decode_device(d, p, s, opts))
        init = warm.predict(d, p, s, opts, th)
        wo, _, _ = bbp.decode_groups([(d, p, s, 0, init)], opts)
        res = warm.decode(d, p, s, opts, th, trained=(0, 0))
        torch.cuda.synchronize()
        only, got = _np(wo[0]), _np(res)
        slower = only["iters"][np.arange(b), only["coset"]] > only["iters"].min(axis=1)
        fb = np.any(~(only["delta"] < opts.delta1), axis=1) | slower
        assert res["fallback"] == fb.sum()
        total_fb += int(fb.sum())
        for k in ("loglik", "delta", "coset", "correction"):
            np.testing.assert_array_equal(got[k][fb], cold[k][fb], err_msg=k)
            np.testing.assert_array_equal(got[k][~fb], only[k][~fb], err_msg=k)
        np.testing.assert_array_equal(got["iters"][fb], only["iters"][fb] + cold["iters"][fb])
        np.testing.assert_array_equal(got["iters"][~fb], only["iters"][~fb])
    assert total_fb > 0     # the fallback path ran


def test_warm_decode_outside_trained_range_is_cold(dev):
    """For a distance outside the parameters' trained range the warm decode is the cold decode, bitwise, and
    reports every syndrome as decoded from the uniform start; a range with one bound 0 is refused."""
    import torch
    import paper_2402_04834_amd as bbp
    from paper_2402_04834_amd import warm
    d, p, b = 9, 0.1, 12
    _, syn = workload.make_batch(d, p, b, workload="warm", p_index=415)
    s = torch.from_numpy(syn).to(dev)
    th = torch.from_numpy(_theta(5, head_scale=0.3)).to(dev)
    opts = bbp.default_opts(block=6, chi=32, max_iter=20)
    _say("[warm range] d=9 against a network trained on 13..21")
    cold = _np(bbp.decode_device(d, p, s, opts))
    res = warm.decode(d, p, s, opts, th, trained=(13, 21))
    torch.cuda.synchronize()
    assert res["fallback"] == b
    got = _np(res)
    for k in ("loglik", "delta", "iters", "coset", "correction"):
        np.testing.assert_array_equal(got[k], cold[k], err_msg=k)
    with pytest.raises(bbp.BbpError):
        warm.decode(d, p, s, opts, th, trained=(0, 21))


def test_warm_in_distribution_agreement_d17(dev):
    """Decision agreement of the warm decode (committed weights, trained on d 13..21) with the cold decode at
    d=17, p=0.10, 4096 syndromes, <= 60 iterations (the benchmark's warm workload at a trained distance):
    at least 99.9 % of the syndromes (measured without any fallback: 99.95 %)."""
    import torch
    import paper_2402_04834_amd as bbp
    from paper_2402_04834_amd import warm
    d, p, b = 17, 0.10, 4096
    _, syn = workload.make_batch(d, p, b, workload="warm", p_index=10)
    s = torch.from_numpy(syn).to(dev)
    th = torch.from_numpy(warm.load()).to(dev)
    opts = bbp.default_opts(block=6, chi=32, max_iter=60)
    _say("[warm d=17] 4096 syndromes, committed weights")
    cold = _np(bbp.decode_device(d, p, s, opts))
    res = warm.decode(d, p, s, opts, th)
    torch.cuda.synchronize()
    hot = _np(res)
    agree = (hot["coset"] == cold["coset"]).mean()
    _say(f"   agreement {agree:.5f}, fallback {res['fallback']}")
    assert agree >= 0.999
    np.testing.assert_array_equal(workload.syndrome_of(d, hot["correction"]), syn)


def test_training_reduces_loss(dev):
    import torch
    import paper_2402_04834_amd as bbp
    from paper_2402_04834_amd import warm
    opts = bbp.default_opts(block=6, chi=32, max_iter=30)
    d = 9
    _, syn = workload.make_batch(d, 0.1, 64, workload="warm", p_index=414)
    s = torch.from_numpy(syn).to(dev)
    pt = torch.full((64,), 0.1, dtype=torch.float64, device=dev)
    outs, _, _ = bbp.decode_groups([(d, pt, s)], opts, messages=True)
    pool = {d: dict(syn=s, p=pt, targets=outs[0]["messages"],
                    use=(outs[0]["delta"] < opts.delta0).reshape(-1).to(torch.uint8))}
    _say("[warm train] 150 Adam steps on 64 syndromes at d=9")
    _, hist = warm.train(pool, opts, steps=150, batch=8, lr=2e-3, seed=3, log=_say, every=50)
    first, last = hist[:10].mean(), hist[-10:].mean()
    assert np.all(np.isfinite(hist))
    assert last < 0.8 * first, (first, last)


def test_committed_weights_against_cold_start(dev):
    """The committed network (trained on d 13..21) against the uniform start on held-out syndromes at d=13,
    p=0.10: the warm decode agrees with the cold decisions on nearly every syndrome and its iteration
    count stays close to the cold one. (Measured: the network does not reduce the iterations; the numbers
    of the d=25 comparison are in the benchmark's warm workload.)"""
    import torch
    import paper_2402_04834_amd as bbp
    from paper_2402_04834_amd import warm
    d, p, b = 13, 0.10, 512
    _, syn = workload.make_batch(d, p, b, workload="warm", p_index=1013)
    s = torch.from_numpy(syn).to(dev)
    th = torch.from_numpy(warm.load()).to(dev)
    opts = bbp.default_opts(block=6, chi=32, max_iter=40)
    cold = _np(bbp.decode_device(d, p, s, opts))
    res = warm.decode(d, p, s, opts, th)
    torch.cuda.synchronize()
    hot = _np(res)
    agree = (hot["coset"] == cold["coset"]).mean()
    ci, wi = cold["iters"].mean(), hot["iters"].mean()
    _say(f"[warm weights] d={d}: agreement {agree:.4f}, iterations cold {ci:.2f} warm {wi:.2f}, "
         f"fallback {res['fallback']}")
    assert np.all(np.isfinite(hot["loglik"]))
    assert agree >= 0.99
    assert wi <= 1.1 * ci
