"""GPU tests of batching: mixed-distance groups in one call, HIP-graph capture and replay, and the launch
variants the autotuner chooses among. Every variant must give results identical to a plain decode of each
group alone, and a mixed call is also checked against the FP64 oracle."""
import sys

import numpy as np
import pytest

from oracle import blockbp
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


def _np(out):
    return {k: out[k].cpu().numpy() for k in KEYS}


def _alone(dev, d, p, syn, opts):
    import torch
    import paper_2402_04834_amd as bbp
    out = bbp.decode_device(d, p, torch.from_numpy(syn).to(dev), opts)
    torch.cuda.synchronize()
    return _np(out)


def _same(a, b, what):
    for k in KEYS:
        np.testing.assert_array_equal(a[k], b[k], err_msg=f"{what}: {k}")


MIX = [(5, 0.10, 7), (7, 0.08, 5), (9, 0.12, 3), (11, 0.10, 2), (17, 0.10, 3)]


def _mix_inputs():
    return [(d, p, workload.make_batch(d, p, b, workload="mixed", p_index=d)[1]) for d, p, b in MIX]


def test_mixed_groups_equal_separate_decodes(dev):
    import torch
    import paper_2402_04834_amd as bbp
    opts = bbp.default_opts(block=6, chi=32, max_iter=12)
    inputs = _mix_inputs()
    _say("[mixed] groups", [(d, p, s.shape[0]) for d, p, s in inputs])
    outs, _, _ = bbp.decode_groups([(d, p, torch.from_numpy(s).to(dev)) for d, p, s in inputs], opts)
    torch.cuda.synchronize()
    for (d, p, s), o in zip(inputs, outs):
        _same(_np(o), _alone(dev, d, p, s, opts), f"d={d}")


def test_mixed_groups_against_oracle(dev):
    import torch
    import paper_2402_04834_amd as bbp
    opts = bbp.default_opts(block=6, chi=32, max_iter=4, fixed_iters=1)
    inputs = [(5, 0.10, workload.make_batch(5, 0.10, 4, workload="mixed", p_index=50)[1]),
              (7, 0.09, workload.make_batch(7, 0.09, 3, workload="mixed", p_index=70)[1])]
    _say("[mixed oracle] d=5 x4, d=7 x3, fixed 4 iterations")
    outs, _, _ = bbp.decode_groups([(d, p, torch.from_numpy(s).to(dev)) for d, p, s in inputs], opts)
    torch.cuda.synchronize()
    for (d, p, s), o in zip(inputs, outs):
        ref = blockbp.decode(d, p, s, block=(6, 6), chi=32, max_iter=4, fixed_iters=True)
        got = o["loglik"].cpu().numpy()
        np.testing.assert_allclose(got, ref["loglik"], atol=2e-4 + 2e-6 * np.abs(ref["loglik"]).max())
        np.testing.assert_array_equal(o["coset"].cpu().numpy(), ref["coset"])


def test_graph_replays_match_eager(dev):
    import torch
    import paper_2402_04834_amd as bbp
    d, p = 9, 0.10
    _, syn = workload.make_batch(d, p, 16, workload="mixed", p_index=90)
    eager_opts = bbp.default_opts(block=6, chi=32, max_iter=10)
    ref = _alone(dev, d, p, syn, eager_opts)
    graph_opts = bbp.default_opts(block=6, chi=32, max_iter=10, graph=1)
    st = torch.cuda.Stream(dev)
    syn_dev = torch.from_numpy(syn).to(dev)
    ws = torch.empty(bbp.workspace_size(d, 16, graph_opts), dtype=torch.uint8, device=dev)
    other = torch.from_numpy(workload.make_batch(d, p, 8, workload="mixed", p_index=91)[1]).to(dev)
    out = None
    for rep in range(4):
        _say(f"[graph] {'capture' if rep == 0 else 'replay'} {rep}")
        with torch.cuda.stream(st):
            out = bbp.decode_device(d, p, syn_dev, graph_opts, workspace=ws, stream=st, out=out)
        st.synchronize()
        _same(_np(out), ref, f"replay {rep}")
        # eager work of the program between replays, on the default stream
        bbp.decode_device(d, p, other, eager_opts)
        torch.cuda.synchronize()


def test_launch_variants_give_identical_results(dev):
    import torch
    import paper_2402_04834_amd as bbp
    d, p = 11, 0.10
    _, syn = workload.make_batch(d, p, 12, workload="mixed", p_index=110)
    opts = bbp.default_opts(block=6, chi=32, max_iter=15)
    bbp.set_tuning(d, opts, 0, 1)
    ref = _alone(dev, d, p, syn, opts)
    for order in (0, 1):
        for streams in (1, 2, 4):
            _say(f"[variant] order={order} streams={streams}")
            bbp.set_tuning(d, opts, order, streams)
            _same(_alone(dev, d, p, syn, opts), ref, f"order {order} streams {streams}")
    best = bbp.autotune(d, p, torch.from_numpy(syn).to(dev), opts)
    torch.cuda.synchronize()
    assert best.order in (0, 1) and best.streams in (1, 2, 4) and best.ms > 0
    _same(_alone(dev, d, p, syn, opts), ref, "autotuned")
    bbp.set_tuning(d, opts, 0, 1)


def test_host_api_mixed_networks_in_input_order(dev):
    import paper_2402_04834_amd as bbp
    opts = bbp.default_opts(block=6, chi=32, max_iter=8)
    items = []
    for d, p in ((5, 0.1), (7, 0.1), (5, 0.1), (9, 0.08), (7, 0.1)):
        _, s = workload.make_batch(d, p, 1, workload="mixed", p_index=100 + d, start=len(items))
        items.append((d, p, s[0]))
    _say("[host mixed] 5 networks of d 5, 7, 9")
    nets = [bbp.build_network(d, p, s) for d, p, s in items]
    got = bbp.blockbp_decode(nets, opts)
    nmax = got["correction"].shape[1]
    assert nmax == 9 * 9 + 8 * 8
    for i, (d, p, s) in enumerate(items):
        ref = _alone(dev, d, p, s[None, :], opts)
        n = d * d + (d - 1) * (d - 1)
        np.testing.assert_array_equal(got["loglik"][i], ref["loglik"][0])
        np.testing.assert_array_equal(got["iters"][i], ref["iters"][0])
        assert got["coset"][i] == ref["coset"][0]
        np.testing.assert_array_equal(got["correction"][i, :n], ref["correction"][0])
        assert np.all(got["correction"][i, n:] == 0)
