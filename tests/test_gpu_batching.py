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


@pytest.mark.parametrize("precision", [0, 1])
def test_mixed_groups_equal_separate_decodes(dev, precision):
    # FP32, and precision mode 1 (BF16 matrix-core contractions): batching never changes a result
    import torch
    import paper_2402_04834_amd as bbp
    opts = bbp.default_opts(block=6, chi=32, max_iter=12, precision=precision)
    inputs = _mix_inputs()
    _say("[mixed] groups", [(d, p, s.shape[0]) for d, p, s in inputs], "precision", precision)
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


def test_graph_capture_of_multi_stream_rounds(dev):
    """A decode whose rounds spread over 4 streams (fork / join events) captures into one graph; its replays
    equal the eager decode bitwise."""
    import torch
    import paper_2402_04834_amd as bbp
    d, p = 9, 0.10
    _, syn = workload.make_batch(d, p, 16, workload="mixed", p_index=95)
    eager_opts = bbp.default_opts(block=6, chi=32, max_iter=10)
    bbp.set_tuning(d, eager_opts, 1, 4)
    ref = _alone(dev, d, p, syn, eager_opts)
    graph_opts = bbp.default_opts(block=6, chi=32, max_iter=10, graph=1)
    st = torch.cuda.Stream(dev)
    syn_dev = torch.from_numpy(syn).to(dev)
    ws = torch.empty(bbp.workspace_size(d, 16, graph_opts), dtype=torch.uint8, device=dev)
    out = None
    for rep in range(3):
        _say(f"[graph 4 streams] {'capture' if rep == 0 else 'replay'} {rep}")
        with torch.cuda.stream(st):
            out = bbp.decode_device(d, p, syn_dev, graph_opts, workspace=ws, stream=st, out=out)
        st.synchronize()
        _same(_np(out), ref, f"replay {rep}")
    bbp.set_tuning(d, eager_opts, 0, 1)


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


def _mixed_workload(count):
    """The mixed-distance workload: per syndrome d uniform over {9, 13, 17, 21} and p uniform over
    [0.05, 0.15]; chi 16 for d <= 13 and 32 above. Returns {d: (indices, p array, syndromes)}."""
    items = workload.mixed_batch(count)
    groups = {}
    for i, (d, p, _, s) in enumerate(items):
        groups.setdefault(d, ([], [], []))
        groups[d][0].append(i)
        groups[d][1].append(p)
        groups[d][2].append(s)
    return {d: (np.array(ix), np.array(ps), np.stack(ss)) for d, (ix, ps, ss) in sorted(groups.items())}


def test_mixed_distance_workload_one_graph(dev):
    import torch
    import paper_2402_04834_amd as bbp
    mix = _mixed_workload(8192)
    _say("[mixed workload] 8192 syndromes:", {d: len(v[0]) for d, v in mix.items()})
    opts = bbp.default_opts(block=6, chi=32, max_iter=20, graph=1)
    chi_of = {9: 16, 13: 16, 17: 32, 21: 32}
    groups = [(d, torch.from_numpy(ps).to(dev), torch.from_numpy(ss).to(dev), chi_of[d])
              for d, (ix, ps, ss) in mix.items()]
    st = torch.cuda.Stream(dev)
    with torch.cuda.stream(st):
        outs, ws, _ = bbp.decode_groups(groups, opts, stream=st)
    st.synchronize()
    # each group decoded alone (eager) gives identical results
    eager = bbp.default_opts(block=6, chi=32, max_iter=20)
    for (d, p_t, s_t, chi), o in zip(groups, outs):
        _say(f"[mixed workload] d={d} alone")
        alone, _, _ = bbp.decode_groups([(d, p_t, s_t, chi)], eager)
        torch.cuda.synchronize()
        _same(_np(o), _np(alone[0]), f"d={d}")
        assert np.all(o["coset"].cpu().numpy() < 4)
    # oracle parity on the committed fixture: the first 64 syndromes of every distance, each at its own p
    # (tests/golden/mixed_8192_first64_per_d.json, written by make_oracle_fixtures.py from oracle/ only)
    import json
    import os
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "mixed_8192_first64_per_d.json")
    fx = json.load(open(path))
    assert fx["meta"]["count"] == 8192 and fx["meta"]["max_iter"] == 20
    per_d = {}
    for r in fx["records"]:
        d = r["d"]
        ix, ps, _ = mix[d]
        j = int(np.nonzero(ix == r["index"])[0][0])
        assert abs(ps[j] - r["p"]) < 1e-15 and r["chi"] == chi_of[d]
        per_d.setdefault(d, []).append((j, r))
    for d, recs in sorted(per_d.items()):
        o = _np(outs[list(mix).index(d)])
        j = np.array([jj for jj, _ in recs])
        ref_ll = np.array([r["loglik"] for _, r in recs])
        ref_dl = np.array([r["delta"] for _, r in recs])
        ref_it = np.array([r["iters"] for _, r in recs])
        ref_cs = np.array([r["coset"] for _, r in recs])
        it, ll = o["iters"][j], o["loglik"][j]
        near = np.abs(np.log(np.maximum(ref_dl, 1e-30) / 1e-4)) < 0.05
        assert np.all((it == ref_it) | near), f"d={d}"
        same = (it == ref_it) & np.isfinite(ref_ll)
        np.testing.assert_array_less(np.abs(ll[same] - ref_ll[same]), 2e-4 + 2e-6 * np.abs(ref_ll[same]))
        bad = o["coset"][j] != ref_cs
        for i in np.nonzero(bad)[0]:   # only ties within the FP32 error may differ
            trusted = ref_dl[i] < 1e-2
            cand = np.where(trusted, ref_ll[i], -np.inf) if trusted.any() else -ref_dl[i]
            srt = np.sort(cand)[::-1]
            assert srt[0] - srt[1] < 1e-3, (d, i, ref_ll[i], ref_dl[i])
        _say(f"[mixed workload] d={d}: {len(recs)} oracle records, decisions equal {int((~bad).sum())}, "
             f"max |dlnZ| {np.abs(ll[same] - ref_ll[same]).max():.2e}")

def test_concurrent_multistream_decodes_match_serial(dev):
    """Two host threads decoding at once with the four-stream launch variant (which shares the device's
    auxiliary streams and events), eagerly and through captured graphs, each on its own stream: every result
    is bitwise the serial decode's."""
    import threading
    import torch
    import paper_2402_04834_amd as bbp
    d, p = 9, 0.10
    opts = bbp.default_opts(block=6, chi=32, max_iter=20)
    gopts = bbp.default_opts(block=6, chi=32, max_iter=20, graph=1)
    bbp.set_tuning(d, opts, 1, 4)
    try:
        syn = [torch.from_numpy(workload.make_batch(d, p, 48, workload="mixed", p_index=120 + k)[1]).to(dev)
               for k in range(2)]
        ref = [_np(bbp.decode_device(d, p, s, opts)) for s in syn]
        torch.cuda.synchronize()
        errors, results = [], [[], []]

        def worker(k):
            try:
                st = torch.cuda.Stream(dev)
                ws = torch.empty(bbp.workspace_size(d, 48, opts), dtype=torch.uint8, device=dev)
                out = None
                for rep in range(6):
                    o = gopts if rep % 2 else opts
                    out = bbp.decode_device(d, p, syn[k], o, workspace=ws, stream=st, out=out)
                    st.synchronize()
                    results[k].append(_np(out))
            except Exception as e:   # reported by the main thread
                errors.append(e)

        _say("[concurrent] two threads, 4-stream variant, eager and graph")
        th = [threading.Thread(target=worker, args=(k,)) for k in range(2)]
        for t in th:
            t.start()
        for t in th:
            t.join()
        assert not errors, errors
        for k in range(2):
            assert len(results[k]) == 6
            for r in results[k]:
                _same(r, ref[k], f"thread {k}")
    finally:
        bbp.set_tuning(d, opts, 0, 1)
