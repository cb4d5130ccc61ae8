"""GPU parity of the truncating block sweeps (Sec. III.D with a binding chi) against the FP64 oracle.

Sweeps whose boundary MPS can exceed chi -- 6x6 blocks below chi 16, and every sweep of a plan with 7x7 or
8x8 blocks -- run the device's QR + truncated-SVD compression (FP64 arithmetic, FP32 message storage). The
oracle runs the literal boundary-MPS sweep (numpy QR and SVD). Tolerances: every dense message entry within
2e-6, every coset log-likelihood within 2e-5 + 2e-7 |ln Z| (FP32 rounding of the stored messages between
updates, amplified by the truncation), decisions equal wherever the oracle's best coset leads by more than
1e-4 nats, and equal iteration counts in early-exit mode away from the delta0 threshold.
"""
import sys

import numpy as np
import pytest

from oracle import blockbp, mps
from paper_2402_04834_amd import workload

pytestmark = pytest.mark.gpu

MSG_TOL = 2e-6


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def dev():
    import torch
    import paper_2402_04834_amd as bbp
    bbp._lib.lib()
    return torch.device("cuda:0")


def _ll_tol(ref):
    return 2e-5 + 2e-7 * np.nanmax(np.abs(ref))


def _decode(dev, d, p, syn, messages=True, **kw):
    import torch
    import paper_2402_04834_amd as bbp
    opts = bbp.default_opts(**kw)
    st = torch.from_numpy(np.ascontiguousarray(syn)).to(dev)
    out = bbp.decode_device(d, p, st, opts, messages=messages)
    torch.cuda.synchronize()
    return {k: (v.cpu().numpy() if hasattr(v, "cpu") else v) for k, v in out.items() if k != "workspace"}


def _check_messages(gpu_msgs, res, plan, tol=MSG_TOL):
    S = gpu_msgs.shape[0]
    for e, (src, dst, _) in enumerate(plan.edges):
        K = plan.msg_len(src, dst)
        ref = mps.to_dense(res["messages"][(src, dst)]).reshape(S, 4, 2 ** K)
        np.testing.assert_allclose(gpu_msgs[:, :, e, : 2 ** K], ref, rtol=0, atol=tol, err_msg=f"message {e}")
        assert np.all(gpu_msgs[:, :, e, 2 ** K:] == 0)


def _check_loglik(got, ref):
    np.testing.assert_array_equal(np.isnan(got), np.isnan(ref))
    ok = ~np.isnan(ref)
    np.testing.assert_allclose(got[ok], ref[ok], rtol=0, atol=_ll_tol(ref))


def _decisions_agree(gpu_coset, ref_ll, ref_coset, ref_delta, delta1, margin=1e-4):
    for i in np.nonzero(gpu_coset != ref_coset)[0]:
        trusted = ref_delta[i] < delta1
        cand = np.where(trusted, ref_ll[i], -np.inf) if trusted.any() else -ref_delta[i]
        srt = np.sort(np.nan_to_num(cand, nan=-np.inf))[::-1]
        assert srt[0] - srt[1] < margin, (i, ref_ll[i], gpu_coset[i], ref_coset[i])


@pytest.mark.parametrize("d,p,k,chi,iters,eta,count", [
    (5, 0.10, 3, 2, 4, 0.1, 8),     # 3x3 blocks at chi 2 (the smallest binding chi with exact messages)
    (7, 0.10, 6, 8, 4, 0.1, 6),     # one interior 6x6 block, chi 8 (boundary rank 16)
    (7, 0.12, 6, 12, 3, 0.5, 6),    # chi 12, damping 0.5
    (9, 0.10, 6, 8, 3, 0.1, 4),     # 6x6 blocks with a 5-wide remainder: truncating and exact sweeps mixed
    (9, 0.10, 7, 16, 3, 0.1, 4),    # 7x7 blocks (message stride 128), every sweep truncating
    (9, 0.08, 8, 16, 3, 0.1, 4),    # 8x8 blocks (message stride 256), caps of bond 16
    (9, 0.10, 7, 8, 3, 0.1, 3),     # 7x7 blocks at chi 8: the narrow form at its limit (chain bonds 8)
    (11, 0.10, 4, 4, 3, 0.1, 3),    # 4x4 blocks at chi 4, ragged [4, 4, 4, 4, 4, 1]
])
def test_truncating_fixed_iterations_parity(dev, d, p, k, chi, iters, eta, count):
    import paper_2402_04834_amd as bbp
    _say(f"[trunc] d={d} p={p} k={k} chi={chi} iters={iters} eta={eta} count={count}")
    info = bbp.plan_query(d, bbp.default_opts(block=k, chi=chi))
    assert info.gpu_supported == 1 and info.truncating_sweeps > 0 and info.exact_sweeps == 0
    _, syn = workload.make_batch(d, p, count, workload="test", p_index=d + k + chi)
    ref = blockbp.decode(d, p, syn, block=(k, k), chi=chi, max_iter=iters, eta=eta, fixed_iters=True,
                         return_messages=True)
    got = _decode(dev, d, p, syn, block=k, chi=chi, max_iter=iters, damping=eta, fixed_iters=1)
    assert got["messages"].shape[-1] == info.message_stride
    assert np.all(got["iters"] == iters)
    _check_messages(got["messages"], ref, ref["plan"])
    _check_loglik(got["loglik"], ref["loglik"])
    _decisions_agree(got["coset"], ref["loglik"], ref["coset"], ref["delta"], 1e-2)
    np.testing.assert_array_equal(workload.syndrome_of(d, got["correction"]), syn)


@pytest.mark.parametrize("d,k,chi,count", [(11, 6, 8, 4), (13, 8, 16, 2)])
def test_truncating_early_exit_decode_against_oracle(dev, d, k, chi, count):
    # the whole decoder (early exit, Bethe estimate, decision) with truncating sweeps
    p = 0.10
    _say(f"[trunc-decode] d={d} k={k} chi={chi} count={count}")
    _, syn = workload.make_batch(d, p, count, workload="test", p_index=3 * d + k)
    ref = blockbp.decode(d, p, syn, block=(k, k), chi=chi, max_iter=20)
    got = _decode(dev, d, p, syn, messages=False, block=k, chi=chi, max_iter=20)
    # iteration counts agree except where Delta lands within rounding of delta0 at the exit iteration
    same = got["iters"] == ref["iters"]
    assert same.mean() >= 0.9, (got["iters"], ref["iters"])
    both = same & ~np.isnan(ref["loglik"])
    np.testing.assert_allclose(got["loglik"][both], ref["loglik"][both], rtol=0, atol=2e-4)
    _decisions_agree(got["coset"], ref["loglik"], ref["coset"], ref["delta"], 1e-2, margin=1e-3)


def test_truncating_and_exact_groups_in_one_call(dev):
    # one decode_groups call mixing truncating groups (6x6 blocks at chi 8 and 12) with an exact one (chi 32),
    # chi per group: every group equals its own single-group decode bit for bit
    import torch
    import paper_2402_04834_amd as bbp
    opts = bbp.default_opts(block=6, chi=32, max_iter=4, fixed_iters=1)
    items = []
    for d, n, chi in [(9, 3, 8), (7, 2, 32), (11, 1, 12)]:
        _, syn = workload.make_batch(d, 0.1, n, workload="test", p_index=d)
        items.append((d, 0.1, torch.from_numpy(syn).to(dev), chi))
        info = bbp.plan_query(d, bbp.default_opts(block=6, chi=chi))
        assert (info.truncating_sweeps > 0) == (chi < 16) and info.num_messages > 0
    _say("[trunc-groups] d=9 (chi 8), d=7 (exact, chi 32), d=11 (chi 12), 6x6 blocks")
    outs, _, _ = bbp.decode_groups(items, opts, messages=True)
    torch.cuda.synchronize()
    for (d, p, syn, chi), o in zip(items, outs):
        one = bbp.decode_device(d, p, syn, bbp.default_opts(block=6, chi=chi, max_iter=4, fixed_iters=1),
                                messages=True)
        torch.cuda.synchronize()
        for key in ("loglik", "messages", "coset"):
            a, b = o[key].cpu().numpy(), one[key].cpu().numpy()
            np.testing.assert_array_equal(np.nan_to_num(a, nan=7.0), np.nan_to_num(b, nan=7.0), err_msg=f"d={d} {key}")


def test_truncating_start_messages_and_ragged_batches(dev):
    # start messages at the 256-float stride: n iterations, then one more from the returned messages, equal
    # n + 1 iterations in one call; syndromes decode independently of the batch they come in
    import torch
    import paper_2402_04834_amd as bbp
    d, k, chi = 9, 8, 16
    _, syn = workload.make_batch(d, 0.1, 3, workload="test", p_index=5)
    st = torch.from_numpy(syn).to(dev)
    opts = lambda n: bbp.default_opts(block=k, chi=chi, max_iter=n, fixed_iters=1)
    _say("[trunc-init] 3 + 1 iterations against 4")
    three = bbp.decode_device(d, 0.1, st, opts(3), messages=True)
    four = bbp.decode_device(d, 0.1, st, opts(4), messages=True)
    torch.cuda.synchronize()
    outs, _, _ = bbp.decode_groups([(d, 0.1, st, chi, three["messages"])], opts(1), messages=True)
    torch.cuda.synchronize()
    m4, m31 = four["messages"].cpu().numpy(), outs[0]["messages"].cpu().numpy()
    assert np.abs(m4 - m31).max() < 1e-5
    np.testing.assert_allclose(outs[0]["loglik"].cpu().numpy(), four["loglik"].cpu().numpy(), rtol=0, atol=1e-4)
    for lo, hi in [(0, 1), (1, 3)]:
        part = bbp.decode_device(d, 0.1, st[lo:hi].contiguous(), opts(4), messages=True)
        torch.cuda.synchronize()
        np.testing.assert_array_equal(part["messages"].cpu().numpy(), m4[lo:hi])
        np.testing.assert_array_equal(part["loglik"].cpu().numpy(), four["loglik"].cpu().numpy()[lo:hi])


def test_truncating_launch_in_several_chunks(dev):
    # a round with more truncating items than one launch has workspace slots for (32768) runs in chunks:
    # every syndrome decodes bit for bit as it does alone. 19 truncating sweeps over three lists put at least
    # 7 in one, so 1200 syndromes (4800 jobs) make at least 33600 items.
    import torch
    import paper_2402_04834_amd as bbp
    d, k, chi, n = 9, 6, 8, 1200
    opts = bbp.default_opts(block=k, chi=chi, max_iter=2, fixed_iters=1)
    assert bbp.plan_query(d, opts).truncating_sweeps == 19
    _, syn = workload.make_batch(d, 0.1, n, workload="test", p_index=17)
    st = torch.from_numpy(syn).to(dev)
    _say(f"[trunc-chunks] d={d} k={k} chi={chi} batch={n}")
    big = bbp.decode_device(d, 0.1, st, opts, messages=True)
    torch.cuda.synchronize()
    bm, bl = big["messages"].cpu().numpy(), big["loglik"].cpu().numpy()
    for i in (0, 611, n - 1):
        one = bbp.decode_device(d, 0.1, st[i:i + 1].contiguous(), opts, messages=True)
        torch.cuda.synchronize()
        np.testing.assert_array_equal(one["messages"].cpu().numpy()[0], bm[i], err_msg=f"syndrome {i}")
        np.testing.assert_array_equal(one["loglik"].cpu().numpy()[0], bl[i], err_msg=f"syndrome {i}")


@pytest.mark.parametrize("fixture,k,chi,batch", [("d17_p010_k6_chi8_first64.json", 6, 8, 256),
                                                 ("d17_p010_k8_chi16_first32.json", 8, 16, 256)])
def test_full_size_d17_truncating_against_oracle_fixture(dev, fixture, k, chi, batch):
    # the truncating workload of the benchmark (the first 256 syndromes of the d=17, p=0.10 batch, <= 20
    # iterations with early exit) in one decode, checked on the syndromes of a committed oracle fixture
    # (tests/golden, written by make_oracle_fixtures.py from oracle/ only): iteration counts equal away from
    # delta0, ln Z of the cosets with equal counts within the early-exit tolerance, decisions equal beyond
    # a 1e-3-nat margin (measured at 6x6, chi 8: all 256 iteration counts equal, |dlnZ| <= 2.6e-6)
    import json
    import os
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", fixture)
    g = json.load(open(path))
    meta = g["meta"]
    assert (meta["d"], meta["block"], meta["chi"], meta["max_iter"]) == (17, k, chi, 20)
    _say(f"[trunc full size] d=17 {k}x{k} chi {chi} batch={batch}, {len(g['records'])} oracle records")
    _, syn = workload.make_batch(17, meta["p"], batch, workload=meta["workload"], p_index=meta["p_index"])
    got = _decode(dev, 17, meta["p"], syn, messages=False, block=k, chi=chi, max_iter=20, damping=meta["eta"],
                  delta0=meta["delta0"], delta1=meta["delta1"])
    idx = np.array([r["index"] for r in g["records"]])
    ref_ll = np.array([r["loglik"] for r in g["records"]])
    ref_dl = np.array([r["delta"] for r in g["records"]])
    ref_it = np.array([r["iters"] for r in g["records"]])
    ref_cs = np.array([r["coset"] for r in g["records"]])
    it, ll = got["iters"][idx], got["loglik"][idx]
    same = it == ref_it
    near = np.abs(np.log(np.maximum(ref_dl, 1e-30) / meta["delta0"])) < 0.1
    assert np.all(same | near), (it[~(same | near)], ref_it[~(same | near)])
    ok = same & np.isfinite(ref_ll)
    err = np.abs(ll[ok] - ref_ll[ok])
    _say(f"   same iteration counts {same.mean():.3f}; |dlnZ| max {err.max():.2e} median {np.median(err):.2e}")
    np.testing.assert_array_less(err, 2e-5 + 2e-7 * np.abs(ref_ll[ok]))
    _decisions_agree(got["coset"][idx], ref_ll, ref_cs, ref_dl, meta["delta1"], margin=1e-3)
    assert np.all(got["coset"] < 4)
