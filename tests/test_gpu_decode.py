"""GPU parity: the HIP decoder (through the C ABI) against the FP64 oracle on the same seeded syndromes.

Tolerances (FP32 block contractions, FP64 sums): every coset log-likelihood within
|ln Z_gpu - ln Z_oracle| <= 2e-4 + 2e-6 |ln Z_oracle| in fixed-iteration mode, every dense message within
2e-5 (entries of unit vectors), decisions equal wherever the oracle's best coset leads the runner-up by
more than 1e-3 nats (the FP32 error budget), and identical iteration counts in early-exit mode away from
the delta0 threshold.
"""
import math
import sys

import numpy as np
import pytest

from oracle import blockbp, lattice, mps, network
from paper_2402_04834_amd import workload

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def dev():
    import torch
    import paper_2402_04834_amd as bbp
    bbp._lib.lib()
    return torch.device("cuda:0")


def _gpu_decode(dev, d, p, syn, messages=True, **kw):
    import torch
    import paper_2402_04834_amd as bbp
    opts = bbp.default_opts(**kw)
    st = torch.from_numpy(np.ascontiguousarray(syn)).to(dev)
    out = bbp.decode_device(d, p, st, opts, messages=messages)
    torch.cuda.synchronize()
    return {k: (v.cpu().numpy() if hasattr(v, "cpu") else v) for k, v in out.items() if k != "workspace"}


def _ll_tol(ref):
    return 2e-4 + 2e-6 * np.abs(ref)


def _check_messages(gpu_msgs, res, plan):
    msgs = res["messages"]
    S = gpu_msgs.shape[0]
    for e, (src, dst, _) in enumerate(plan.edges):
        K = plan.msg_len(src, dst)
        ref = mps.to_dense(msgs[(src, dst)]).reshape(S, 4, 2 ** K)
        got = gpu_msgs[:, :, e, : 2 ** K]
        np.testing.assert_allclose(got, ref, atol=2e-5, err_msg=f"message {e} {src}->{dst}")
        assert np.all(gpu_msgs[:, :, e, 2 ** K:] == 0)


def _decisions_agree(gpu_coset, ref_ll, ref_coset, ref_delta, delta1):
    """Decisions must agree where the oracle's choice is not within the FP32 error of a tie."""
    ok = gpu_coset == ref_coset
    for i in np.nonzero(~ok)[0]:
        trusted = ref_delta[i] < delta1
        cand = np.where(trusted, ref_ll[i], -np.inf) if trusted.any() else -ref_delta[i]
        srt = np.sort(cand)[::-1]
        assert srt[0] - srt[1] < 1e-3, (i, ref_ll[i], ref_delta[i], gpu_coset[i], ref_coset[i])


@pytest.mark.parametrize("d,p,k,chi,iters,eta,count", [
    (5, 0.10, 3, 4, 10, 0.1, 24),       # the small configuration: d=5, 3x3 blocks, chi 4, 10 iterations
    (7, 0.12, 4, 16, 6, 0.5, 12),       # ragged 4x4 blocks ([4, 4, 4, 1]), damping 0.5
    (7, 0.08, 6, 32, 5, 0.1, 8),        # 6x6 blocks with a 1-wide remainder
    (9, 0.10, 6, 32, 4, 0.1, 4),        # 6x6 blocks with a 5-wide remainder, both caps of dimension 8
    (11, 0.09, 6, 32, 3, 0.1, 2),       # 4x4 grid of blocks [6, 6, 6, 3]: every cap pattern of the d=17 workload
    (5, 0.10, 1, 2, 6, 0.1, 8),         # 1x1 blocks: plain BP between single tensors (the paper's naive limit)
    (7, 0.10, 2, 4, 5, 0.1, 6),         # 2x2 blocks ([2, 2, 2, 2, 2, 2, 1])
    (9, 0.10, 5, 32, 4, 0.1, 4),        # 5x5 blocks ([5, 5, 5, 2])
])
def test_fixed_iterations_parity(dev, d, p, k, chi, iters, eta, count):
    _say(f"[parity] d={d} p={p} k={k} chi={chi} iters={iters} eta={eta} count={count}")
    _, syn = workload.make_batch(d, p, count, workload="test", p_index=d)
    ref = blockbp.decode(d, p, syn, block=(k, k), chi=chi, max_iter=iters, eta=eta, fixed_iters=True,
                         return_messages=True)
    got = _gpu_decode(dev, d, p, syn, block=k, chi=chi, max_iter=iters, damping=eta, fixed_iters=1)
    assert np.all(got["iters"] == iters)
    np.testing.assert_allclose(got["loglik"], ref["loglik"], rtol=0, atol=_ll_tol(ref["loglik"]).max())
    np.testing.assert_allclose(got["delta"], ref["delta"], rtol=2e-2, atol=2e-6)
    _check_messages(got["messages"], ref, ref["plan"])
    _decisions_agree(got["coset"], ref["loglik"], ref["coset"], ref["delta"], 1e-2)
    # the correction carries the syndrome and lies in the decided coset
    np.testing.assert_array_equal(workload.syndrome_of(d, got["correction"]), syn)


def test_early_exit_parity(dev):
    d, p, k, chi = 5, 0.08, 3, 4
    _say(f"[early-exit] d={d} p={p}")
    _, syn = workload.make_batch(d, p, 32, workload="test", p_index=77)
    ref = blockbp.decode(d, p, syn, block=(k, k), chi=chi, max_iter=20)
    got = _gpu_decode(dev, d, p, syn, block=k, chi=chi, max_iter=20)
    # iteration counts agree except where the oracle's distance sits within FP32 noise of delta0
    near = np.abs(np.log(np.maximum(ref["delta"], 1e-30) / 1e-4)) < 0.05
    assert np.all((got["iters"] == ref["iters"]) | near)
    same = got["iters"] == ref["iters"]
    np.testing.assert_allclose(got["loglik"][same], ref["loglik"][same], atol=_ll_tol(ref["loglik"]).max())
    _decisions_agree(got["coset"], ref["loglik"], ref["coset"], ref["delta"], 1e-2)


def test_uniform_noise_closed_form_on_gpu(dev):
    # eps = 3/4: ln Z = (m - 2n) ln 2 for every coset; converged after one iteration
    d = 9
    _say("[closed form] d=9 eps=3/4")
    rng = np.random.default_rng(5)
    syn = rng.integers(0, 2, size=(6, 2 * d * (d - 1)), dtype=np.uint8)
    got = _gpu_decode(dev, d, 0.75, syn, block=4, chi=16, max_iter=5)
    m, n = 2 * d * (d - 1), d * d + (d - 1) ** 2
    np.testing.assert_allclose(got["loglik"], (m - 2 * n) * math.log(2.0), atol=1e-4)
    assert np.all(got["iters"] == 1)


def test_single_block_equals_exact_contraction(dev):
    # one block covering the whole d=3 lattice: no messages; the closing sweep is the exact contraction
    d, p = 3, 0.1
    _say("[single block] d=3")
    _, syn = workload.make_batch(d, p, 16, workload="test", p_index=3)
    got = _gpu_decode(dev, d, p, syn, block=5, chi=4, max_iter=2)
    ex = network.exact_coset_loglik(d, syn, p)
    np.testing.assert_allclose(got["loglik"], ex, atol=2e-5)
    np.testing.assert_array_equal(got["coset"], np.argmax(ex, axis=1))


def test_tree_partition_equals_exact_contraction(dev):
    # one block row: BP on a path is exact; with no damping it converges to the exact coset probabilities
    d, p = 3, 0.12
    _say("[tree] d=3 blocks 5x2")
    _, syn = workload.make_batch(d, p, 8, workload="test", p_index=4)
    got = _gpu_decode(dev, d, p, syn, block=(5, 2), chi=8, max_iter=8, damping=0.0, fixed_iters=1)
    ex = network.exact_coset_loglik(d, syn, p)
    np.testing.assert_allclose(got["loglik"], ex, atol=5e-5)


def test_batch_of_one_and_ragged_batches_are_independent(dev):
    # results do not depend on the batch composition: decoding a syndrome alone or inside a batch gives
    # bitwise identical outputs
    d, p = 7, 0.1
    _say("[batch independence] d=7")
    _, syn = workload.make_batch(d, p, 9, workload="test", p_index=9)
    full = _gpu_decode(dev, d, p, syn, block=6, chi=32, max_iter=4)
    for i in (0, 4, 8):
        one = _gpu_decode(dev, d, p, syn[i:i + 1], block=6, chi=32, max_iter=4)
        np.testing.assert_array_equal(one["loglik"][0], full["loglik"][i])
        np.testing.assert_array_equal(one["coset"][0], full["coset"][i])


def test_full_size_d17_against_oracle_fixture(dev):
    """The benchmark workload in the benchmark's launch configuration (d=17, p=0.10, 4096 syndromes, 6x6
    blocks, chi=32, <= 20 iterations with early exit), checked on the syndromes of the committed oracle
    fixture (tests/golden/d17_p010_k6_chi32.json, written by make_oracle_fixtures.py from oracle/ only)."""
    import json
    import os
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "d17_p010_k6_chi32.json")
    g = json.load(open(path))
    meta = g["meta"]
    assert (meta["d"], meta["block"], meta["chi"], meta["max_iter"]) == (17, 6, 32, 20)
    _say(f"[full size] d=17 batch=4096, {len(g['records'])} oracle records")
    _, syn = workload.make_batch(17, meta["p"], 4096, workload=meta["workload"], p_index=meta["p_index"])
    got = _gpu_decode(dev, 17, meta["p"], syn, messages=False, block=6, chi=32, max_iter=20,
                      damping=meta["eta"], delta0=meta["delta0"], delta1=meta["delta1"])
    idx = np.array([r["index"] for r in g["records"]])
    ref_ll = np.array([r["loglik"] for r in g["records"]])
    ref_dl = np.array([r["delta"] for r in g["records"]])
    ref_it = np.array([r["iters"] for r in g["records"]])
    ref_cs = np.array([r["coset"] for r in g["records"]])
    it, ll = got["iters"][idx], got["loglik"][idx]
    near = np.abs(np.log(np.maximum(ref_dl, 1e-30) / meta["delta0"])) < 0.05
    assert np.all((it == ref_it) | near)
    same = (it == ref_it) & np.isfinite(ref_ll)
    assert same.sum() >= 0.95 * same.size
    np.testing.assert_array_less(np.abs(ll[same] - ref_ll[same]), _ll_tol(ref_ll[same]))
    _decisions_agree(got["coset"][idx], ref_ll, ref_cs, ref_dl, meta["delta1"])
    # every syndrome of the batch is decided, with a finite estimate for its decided coset
    assert np.all(got["coset"] < 4)
    assert np.all(np.isfinite(got["loglik"][np.arange(4096), got["coset"]]))


def test_d5_configuration_against_oracle(dev):
    """The small configuration whole: d=5, p=0.10, 200 seeded syndromes, 3x3 blocks, chi=4, 10 iterations;
    every coset estimate, message and decision against the oracle."""
    d, p = 5, 0.10
    _, syn = workload.make_batch(d, p, 200, workload="d5")
    _say("[d=5] 200 syndromes, fixed 10 iterations")
    ref = blockbp.decode(d, p, syn, block=(3, 3), chi=4, max_iter=10, fixed_iters=True, return_messages=True)
    got = _gpu_decode(dev, d, p, syn, block=3, chi=4, max_iter=10, fixed_iters=1)
    np.testing.assert_allclose(got["loglik"], ref["loglik"], rtol=0, atol=_ll_tol(ref["loglik"]).max())
    _check_messages(got["messages"], ref, ref["plan"])
    _decisions_agree(got["coset"], ref["loglik"], ref["coset"], ref["delta"], 1e-2)
    _say(f"   decisions equal: {(got['coset'] == ref['coset']).sum()} / 200")


@pytest.mark.parametrize("tag", ["p005", "p010", "p015"])
def test_d11_configuration_against_oracle_fixture(dev, tag):
    """Plain FP32 blockBP at d=11 (p 0.05, 0.10, 0.15; 1024 syndromes each, 4x4 blocks, chi=16, 20
    iterations, damping 0.5): the whole batch is decoded and every syndrome is checked against the committed
    oracle fixture (tests/golden/d11_<p>_k4_chi16_eta05.json, all 1024 syndromes, from oracle/ only)."""
    import json
    import os
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", f"d11_{tag}_k4_chi16_eta05.json")
    g = json.load(open(path))
    meta = g["meta"]
    assert (meta["d"], meta["block"], meta["chi"], meta["max_iter"], meta["eta"]) == (11, 4, 16, 20, 0.5)
    assert sorted(r["index"] for r in g["records"]) == list(range(1024))
    _say(f"[d=11] p={meta['p']} batch=1024, {len(g['records'])} oracle records")
    _, syn = workload.make_batch(11, meta["p"], 1024, workload=meta["workload"], p_index=meta["p_index"])
    got = _gpu_decode(dev, 11, meta["p"], syn, messages=False, block=4, chi=16, max_iter=20,
                      damping=meta["eta"], delta0=meta["delta0"], delta1=meta["delta1"])
    idx = np.array([r["index"] for r in g["records"]])
    ref_ll = np.array([r["loglik"] for r in g["records"]])
    ref_dl = np.array([r["delta"] for r in g["records"]])
    ref_it = np.array([r["iters"] for r in g["records"]])
    ref_cs = np.array([r["coset"] for r in g["records"]])
    it, ll = got["iters"][idx], got["loglik"][idx]
    near = np.abs(np.log(np.maximum(ref_dl, 1e-30) / meta["delta0"])) < 0.05
    assert np.all((it == ref_it) | near)
    same = (it == ref_it) & np.isfinite(ref_ll)
    np.testing.assert_array_less(np.abs(ll[same] - ref_ll[same]), _ll_tol(ref_ll[same]))
    _decisions_agree(got["coset"][idx], ref_ll, ref_cs, ref_dl, meta["delta1"])
    assert np.all(got["coset"] < 4)
    np.testing.assert_array_equal(workload.syndrome_of(11, got["correction"]), syn)


@pytest.mark.parametrize("d,p,k,chi,iters,count", [(5, 0.10, 3, 4, 10, 16), (7, 0.08, 6, 32, 5, 6), (9, 0.10, 6, 32, 4, 4)])
def test_bf16_input_precision_against_oracle(dev, d, p, k, chi, iters, count):
    """Precision mode 1 (BF16 operands at the middle-site contractions on the matrix cores, FP32 elsewhere) in
    fixed-iteration mode. Bound: no more than the n qubit factors and message entries of a coset's estimate
    can enter through operands rounded to 8 significant bits (relative error <= 2^-8), two per product, so
    |d ln Z| <= n 2^-7 (+0.05 for the messages' own rounding); coset differences are held to the same bound
    and decisions must agree wherever the oracle's margin exceeds it. (d=5 with 3x3 blocks has no
    middle-site contraction on the matrix cores: there mode 1 is FP32.)"""
    _say(f"[bf16 inputs] d={d} k={k} chi={chi} iters={iters} count={count}")
    _, syn = workload.make_batch(d, p, count, workload="test", p_index=40 + d)
    ref = blockbp.decode(d, p, syn, block=(k, k), chi=chi, max_iter=iters, fixed_iters=True)
    got = _gpu_decode(dev, d, p, syn, messages=False, block=k, chi=chi, max_iter=iters, fixed_iters=1, precision=1)
    n = d * d + (d - 1) ** 2
    tol = n * 2.0 ** -7 + 0.05
    err = np.abs(got["loglik"] - ref["loglik"])
    assert err.max() <= tol, (err.max(), tol)
    diff_err = np.abs((got["loglik"] - got["loglik"][:, :1]) - (ref["loglik"] - ref["loglik"][:, :1]))
    assert diff_err.max() <= tol, (diff_err.max(), tol)
    srt = np.sort(ref["loglik"], axis=1)
    clear = (srt[:, -1] - srt[:, -2]) > 0.2 * tol
    np.testing.assert_array_equal(got["coset"][clear], ref["coset"][clear])


def test_bf16_d17_full_fixture(dev):
    """Precision mode 1 at the benchmark's size (d=17, p=0.10, 4096 syndromes, 6x6 blocks, chi 32, <= 20
    iterations with early exit) against the FP64 oracle fixture. In this mode BF16 enters only at the
    contractions with the side messages' middle sites (one per cap per sweep): each operand there is rounded
    to 8 significant bits (relative error <= 2^-8), so a product is within 2^-7 and, all terms being
    non-negative, so is each contraction; a sweep with two caps is within 2^-6, entry by entry. At a BP fixed
    point the Bethe estimate is stationary in the messages, so where both runs end at the same fixed point a
    coset's estimate moves by at most the closing sweeps' and overlaps' own errors: |d ln Z| <= (blocks +
    edges) 2^-6 (1.5 nats at d=17). That holds for every coset converged on both sides within 6 nats of its
    syndrome's best coset (the ones a decision can turn on). A coset still drifting slowly when its distance
    first falls below delta0 may stop at another point of its drift (seen far below the best coset); such
    cosets further down must stay more than twice the bound below the GPU's best, so that no decision can
    turn on them. Decisions must be equal wherever the oracle's margin exceeds twice the bound; the counts
    and error quantiles are printed."""
    import json
    import os
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "d17_p010_k6_chi32.json")
    g = json.load(open(path))
    meta = g["meta"]
    _say(f"[bf16 full size] d=17 batch=4096 precision 1, {len(g['records'])} oracle records")
    _, syn = workload.make_batch(17, meta["p"], 4096, workload=meta["workload"], p_index=meta["p_index"])
    got = _gpu_decode(dev, 17, meta["p"], syn, messages=False, block=6, chi=32, max_iter=20,
                      damping=meta["eta"], delta0=meta["delta0"], delta1=meta["delta1"], precision=1)
    idx = np.array([r["index"] for r in g["records"]])
    ref_ll = np.array([r["loglik"] for r in g["records"]])
    ref_dl = np.array([r["delta"] for r in g["records"]])
    ref_cs = np.array([r["coset"] for r in g["records"]])
    ll, dl, cs = got["loglik"][idx], got["delta"][idx], got["coset"][idx]
    bound = (36 + 60) * 2.0 ** -6
    conv = (ref_dl < meta["delta0"]) & (dl < meta["delta0"]) & np.isfinite(ref_ll)
    best = np.max(np.where(np.isfinite(ref_ll), ref_ll, -np.inf), axis=1)
    best_gpu = np.max(np.where(np.isfinite(ll), ll, -np.inf), axis=1)
    near = conv & (best[:, None] - ref_ll < 6.0)
    far = conv & ~near
    err = np.abs(ll - ref_ll)
    _say(f"   converged cosets {conv.sum()} ({near.sum()} within 6 nats of the best): |dlnZ| max "
         f"{err[near].max():.3e} p99 {np.percentile(err[near], 99):.3e} median {np.median(err[near]):.3e}; "
         f"further below: max {err[far].max():.3e}, {(err[far] > bound).sum()} beyond the bound")
    assert err[near].max() <= bound
    assert np.all((best_gpu[:, None] - ll)[far] > 2 * bound)
    srt = np.sort(np.where(np.isfinite(ref_ll), ref_ll, -np.inf), axis=1)
    clear = (srt[:, -1] - srt[:, -2]) > 2 * bound
    _say(f"   decisions equal {(cs == ref_cs).sum()} / {len(idx)} (clear margins: {clear.sum()})")
    np.testing.assert_array_equal(cs[clear], ref_cs[clear])
    assert np.all(got["coset"] < 4)
    np.testing.assert_array_equal(workload.syndrome_of(17, got["correction"]), syn)


@pytest.mark.parametrize("d,k,iters", [(5, 3, 8), (7, 4, 5), (9, 6, 4)])
def test_biased_noise_parity(dev, d, k, iters):
    """Z-biased Pauli noise (bias 10, p=0.12) given as four probabilities: the qubit entries take
    pi[code] for the flipped label; against the oracle with the same pi (same tolerances as above)."""
    import torch
    import paper_2402_04834_amd as bbp
    probs = workload.biased_probs(0.12, 10.0)                       # I, X, Z, Y
    pi = np.array([[probs[0], probs[2]], [probs[1], probs[3]]])      # oracle layout [x][z]
    _, syn = workload.make_batch_pauli(d, probs, 6, p_index=d)
    _say(f"[biased] d={d} k={k} iters={iters}")
    ref = blockbp.decode(d, 0.12, syn, block=(k, k), chi=32, max_iter=iters, fixed_iters=True, noise=pi,
                         return_messages=True)
    opts = bbp.default_opts(block=k, chi=32, max_iter=iters, fixed_iters=1)
    outs, _, _ = bbp.decode_groups([(d, probs, torch.from_numpy(syn).to(dev))], opts, messages=True)
    torch.cuda.synchronize()
    got = {key: v.cpu().numpy() for key, v in outs[0].items()}
    np.testing.assert_allclose(got["loglik"], ref["loglik"], rtol=0, atol=_ll_tol(ref["loglik"]).max())
    _check_messages(got["messages"], ref, ref["plan"])
    _decisions_agree(got["coset"], ref["loglik"], ref["coset"], ref["delta"], 1e-2)
    np.testing.assert_array_equal(workload.syndrome_of(d, got["correction"]), syn)
    # depolarizing noise given as four probabilities matches the depolarizing path to FP32 rounding
    p = 0.1
    dep = bbp.decode_device(d, p, torch.from_numpy(syn).to(dev), opts)
    four, _, _ = bbp.decode_groups([(d, (1 - p, p / 3, p / 3, p / 3), torch.from_numpy(syn).to(dev))], opts)
    torch.cuda.synchronize()
    np.testing.assert_allclose(four[0]["loglik"].cpu().numpy(), dep["loglik"].cpu().numpy(), rtol=0, atol=1e-4)


def test_residual_gate_limits(dev):
    """Residual-gated schedule at its limits, through the C ABI: a gate of 1e-300 skips only updates whose
    message and inputs did not change at all in FP32, which reproduce their message up to rounding; a gate
    above the largest possible term (8) lets only the first iteration update, so the messages after three
    iterations are those after one, Delta is 0 and early exit happens after the second iteration."""
    d, p, k, chi = 7, 0.10, 4, 16
    _say(f"[gate limits] d={d} k={k} chi={chi}")
    _, syn = workload.make_batch(d, p, 8, workload="test", p_index=41)
    base = _gpu_decode(dev, d, p, syn, block=k, chi=chi, max_iter=6, fixed_iters=1)
    tiny = _gpu_decode(dev, d, p, syn, block=k, chi=chi, max_iter=6, fixed_iters=1, gate=1e-300)
    np.testing.assert_allclose(tiny["messages"], base["messages"], rtol=0, atol=1e-6)
    np.testing.assert_allclose(tiny["loglik"], base["loglik"], rtol=0, atol=1e-5)
    np.testing.assert_array_equal(tiny["coset"], base["coset"])
    one = _gpu_decode(dev, d, p, syn, block=k, chi=chi, max_iter=1, fixed_iters=1)
    big = _gpu_decode(dev, d, p, syn, block=k, chi=chi, max_iter=3, fixed_iters=1, gate=10.0)
    np.testing.assert_array_equal(big["messages"], one["messages"])
    assert np.all(big["delta"] == 0.0) and np.all(one["delta"] > 1e-3)
    ex = _gpu_decode(dev, d, p, syn, block=k, chi=chi, max_iter=20, gate=10.0)
    assert np.all(ex["iters"] == 2)


def test_residual_gate_against_oracle(dev):
    """Gate 1e-6 in early-exit mode against the oracle's gated schedule. FP32 and FP64 distance terms may fall
    on different sides of the gate, and a skip decision taken differently moves a message by about the
    square root of the gate, so estimates must agree to 2e-3 nats, iteration counts to 3, decisions exactly
    away from ties."""
    d, p, k, chi = 7, 0.10, 4, 16
    _say(f"[gate parity] d={d} k={k} chi={chi} gate=1e-6")
    _, syn = workload.make_batch(d, p, 6, workload="test")
    ref = blockbp.decode(d, p, syn, block=(k, k), chi=chi, max_iter=40, gate=1e-6)
    got = _gpu_decode(dev, d, p, syn, block=k, chi=chi, max_iter=40, gate=1e-6)
    err = np.abs(got["loglik"] - ref["loglik"])
    _say(f"   max |d lnZ| {err.max():.2e}, iterations gpu {got['iters'].mean():.2f} oracle {ref['iters'].mean():.2f}")
    assert err.max() < 2e-3
    assert np.all(np.abs(got["iters"] - ref["iters"]) <= 3)
    _decisions_agree(got["coset"], ref["loglik"], ref["coset"], ref["delta"], 1e-2)
