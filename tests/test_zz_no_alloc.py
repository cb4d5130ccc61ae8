"""GPU test of the allocation-free decode (bbp_decode_device_noalloc): its workspace and plan tables live in
the library's static device array; its results must equal those of bbp_decode_device (the same kernels on
the same inputs: bitwise), on two calls in a row where the second has a smaller input (another distance,
fewer syndromes) and so reuses the array the first call left behind."""
import sys

import numpy as np
import pytest

from paper_2402_04834_amd import workload

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _np(out):
    return {k: out[k].cpu().numpy() for k in ("loglik", "delta", "iters", "coset", "correction")}


def test_noalloc_equals_workspace_decode_two_calls():
    import torch
    import paper_2402_04834_amd as bbp
    dev = torch.device("cuda:0")
    cases = [(9, 0.10, 64, 6, 32, 20), (7, 0.08, 12, 4, 16, 12)]   # second call: smaller input
    for d, p, batch, k, chi, iters in cases:
        opts = bbp.default_opts(block=k, chi=chi, max_iter=iters)
        assert batch <= bbp.noalloc_max_batch(d, opts)
        _, syn = workload.make_batch(d, p, batch, workload="test", p_index=70 + d)
        s = torch.from_numpy(syn).to(dev)
        _say(f"[noalloc] d={d} batch={batch} blocks {k} chi {chi} iters {iters}")
        got = bbp.decode_device_noalloc(d, p, s, opts)
        torch.cuda.synchronize()
        got = _np(got)
        ref = _np(bbp.decode_device(d, p, s, opts))
        torch.cuda.synchronize()
        for key in ref:
            np.testing.assert_array_equal(got[key], ref[key], err_msg=f"{key} d={d}")
        assert np.all(got["coset"] < 4)
        np.testing.assert_array_equal(workload.syndrome_of(d, got["correction"]), syn)


def test_noalloc_truncating_plan_equals_workspace_decode():
    # a plan with truncating sweeps (6x6 blocks at chi 8): their per-sweep workspace slots also sit in the
    # static array
    import torch
    import paper_2402_04834_amd as bbp
    dev = torch.device("cuda:0")
    d, p, batch = 7, 0.10, 3
    opts = bbp.default_opts(block=6, chi=8, max_iter=4, fixed_iters=1)
    assert bbp.plan_query(d, opts).truncating_sweeps > 0
    assert batch <= bbp.noalloc_max_batch(d, opts)
    _, syn = workload.make_batch(d, p, batch, workload="test", p_index=91)
    s = torch.from_numpy(syn).to(dev)
    _say(f"[noalloc] d={d} batch={batch} blocks 6 chi 8 (truncating sweeps)")
    got = _np(bbp.decode_device_noalloc(d, p, s, opts))
    torch.cuda.synchronize()
    ref = _np(bbp.decode_device(d, p, s, opts))
    torch.cuda.synchronize()
    for key in ref:
        np.testing.assert_array_equal(got[key], ref[key], err_msg=key)
    np.testing.assert_array_equal(workload.syndrome_of(d, got["correction"]), syn)


def test_noalloc_limit_is_refused():
    import torch
    import paper_2402_04834_amd as bbp
    dev = torch.device("cuda:0")
    d = 17
    opts = bbp.default_opts(block=6, chi=32, max_iter=20)
    cap = bbp.noalloc_max_batch(d, opts)
    assert 100 < cap < 4096
    # sizes are checked before anything is enqueued: a batch one beyond the limit is refused
    s = torch.zeros((cap + 1, 2 * d * (d - 1)), dtype=torch.uint8, device=dev)
    with pytest.raises(bbp.BbpError) as e:
        bbp.decode_device_noalloc(d, 0.1, s, opts)
    assert e.value.code == -1 and "limit" in str(e.value)
    _say(f"[noalloc] d=17 limit {cap} syndromes")
