"""GPU parity of the boundary-MPS decoder (the single-block limit of blockBP) against the FP64 oracle.

The kernel (FP64 matrix work) is compared with the oracle's bMPS at the same chi and, where chi covers the
largest Schmidt rank, with the exact contraction; decisions must agree wherever the oracle's best coset
leads the runner-up by more than the allowance, and the correction must be the labels of the decided coset.
"""
import sys

import numpy as np
import pytest

from oracle import bmps, lattice, network
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


def _gpu(dev, d, p, syn, chi, **kw):
    import torch
    import paper_2402_04834_amd as bbp
    st = torch.from_numpy(np.ascontiguousarray(syn)).to(dev)
    if hasattr(p, "shape"):
        p = torch.from_numpy(np.asarray(p, dtype=np.float64)).to(dev)
    out = bbp.bmps_decode(d, p, st, chi, **kw)
    torch.cuda.synchronize()
    return {k: (v.cpu().numpy() if hasattr(v, "cpu") else v) for k, v in out.items() if k != "workspace"}


def _report(tag, got, ref):
    err = np.abs(got - ref)
    _say(f"   {tag}: max |d lnZ| {err.max():.3e}, median {np.median(err):.3e}, max |lnZ| {np.abs(ref).max():.1f}")
    if ref.ndim == 2:
        gap = ref.max(axis=1, keepdims=True) - ref
        for i in np.argsort(err.ravel())[::-1][:4]:
            _say(f"      err {err.ravel()[i]:.2e} at gap {gap.ravel()[i]:.1f} nats (coset {i % 4})")
    return err


def _check_fp64(got_ll, ref_ll):
    """Two FP64 evaluations of one bMPS contraction agree on a coset's value Z_k only to a relative accuracy
    eps with respect to the dominant scale of the contraction (the likeliest configurations, about Z of the
    best coset): rounding in different orders, and -- where chi truncates -- different but equally valid
    choices at near-ties of the singular values at a cut. The error in ln Z_k is then about eps * exp(gap)
    for a coset gap nats below the best. With eps = 1e-9 (measured up to 3e-11 at d = 13), cosets within 12
    nats of the best must agree to 1e-8 + 1e-9 exp(gap) nats; a coset further below, which no decision can
    pick, must stay more than 8 nats below the GPU's best."""
    gap = ref_ll.max(axis=1, keepdims=True) - ref_ll
    got_gap = got_ll.max(axis=1, keepdims=True) - got_ll
    err = np.abs(got_ll - ref_ll)
    near = gap <= 12.0
    bad = near & (err > 1e-8 + 1e-9 * np.exp(np.minimum(gap, 12.0)))
    assert not bad.any(), f"errors {err[bad]} at gaps {gap[bad]}"
    far_bad = ~near & ~(got_gap > 8.0)
    assert not far_bad.any(), f"far cosets {got_ll[far_bad]} not far below the best"


def _check_decisions(got, ref_ll, margin):
    srt = np.sort(ref_ll, axis=-1)
    clear = srt[:, -1] - srt[:, -2] > margin
    np.testing.assert_array_equal(got["coset"][clear], bmps.decide(ref_ll)[clear])
    np.testing.assert_array_equal(got["coset"], bmps.decide(got["loglik"]))


def _check_correction(d, syn, got):
    x, z = lattice.coset_labels(d, syn)
    n = workload.num_qubits(d)
    for i in range(syn.shape[0]):
        k = int(got["coset"][i])
        codes = lattice.codes_from_pauli_grid(d, x[i, k], z[i, k])
        np.testing.assert_array_equal(got["correction"][i, :n], codes)


@pytest.mark.parametrize("d,chi,p", [(3, 4, 0.10), (5, 16, 0.05), (5, 16, 0.15)])
def test_exact_regime_against_exact_contraction(dev, d, chi, p):
    _say(f"[bmps exact] d={d} chi={chi} p={p}")
    _, syn = workload.make_batch(d, p, 24, workload="test")
    got = _gpu(dev, d, p, syn, chi)
    ref = network.exact_coset_loglik(d, syn, p)
    _report("gpu vs exact", got["loglik"], ref)
    _check_fp64(got["loglik"], ref)
    _check_decisions(got, ref, 1e-6)
    _check_correction(d, syn, got)


@pytest.mark.parametrize("d,chi,p", [(7, 16, 0.10), (9, 16, 0.10), (7, 8, 0.10), (9, 4, 0.12), (11, 16, 0.08),
                                     (13, 16, 0.10), (13, 12, 0.14)])
def test_truncated_against_oracle(dev, d, chi, p):
    _say(f"[bmps truncated] d={d} chi={chi} p={p}")
    _, syn = workload.make_batch(d, p, 8, workload="test")
    got = _gpu(dev, d, p, syn, chi)
    ref = bmps.bmps_coset_loglik(d, syn, network.depolarizing(p), chi)
    _report("gpu vs oracle bMPS", got["loglik"], ref)
    _check_fp64(got["loglik"], ref)
    _check_decisions(got, ref, 1e-5)
    _check_correction(d, syn, got)


def test_biased_and_per_syndrome_noise(dev):
    d, chi = 5, 16
    probs = workload.biased_probs(0.12, 4.0)
    _, syn = workload.make_batch_pauli(d, probs, 12)
    _say(f"[bmps biased] d={d} chi={chi}")
    got = _gpu(dev, d, probs, syn, chi)
    pI, pX, pZ, pY = probs
    x, z = lattice.coset_labels(d, syn)
    ref = network.exact_log_contraction(d, x, z, np.array([[pI, pZ], [pX, pY]]))
    _report("biased gpu vs exact", got["loglik"], ref)
    _check_fp64(got["loglik"], ref)
    ps = np.linspace(0.04, 0.16, 12)
    _, syn2 = workload.make_batch(d, 0.1, 12, workload="test", p_index=3)
    got2 = _gpu(dev, d, ps, syn2, chi)
    ref2 = np.stack([network.exact_coset_loglik(d, syn2[i:i + 1], ps[i])[0] for i in range(12)])
    _report("per-syndrome p gpu vs exact", got2["loglik"], ref2)
    _check_fp64(got2["loglik"], ref2)


def test_edge_cases(dev):
    import torch
    import paper_2402_04834_amd as bbp
    d = 5
    _, syn = workload.make_batch(d, 0.1, 4, workload="test")
    # chi = 1: every bond truncated to one value; the oracle at chi = 1 is the reference
    got = _gpu(dev, d, 0.1, syn, 1)
    ref = bmps.bmps_coset_loglik(d, syn, network.depolarizing(0.1), 1)
    _report("chi=1", got["loglik"], ref)
    _check_fp64(got["loglik"], ref)
    # d = 2 (smallest lattice), zero syndromes
    _, syn2 = workload.make_batch(2, 0.1, 4, workload="test")
    got2 = _gpu(dev, 2, 0.1, syn2, 16)
    np.testing.assert_allclose(got2["loglik"], network.exact_coset_loglik(2, syn2, 0.1), atol=1e-8)
    zero = np.zeros((3, workload.num_checks(d)), dtype=np.uint8)
    got3 = _gpu(dev, d, 0.1, zero, 16)
    assert np.all(got3["coset"] == 0)
    # empty batch, invalid chi, short workspace
    empty = torch.zeros((0, workload.num_checks(d)), dtype=torch.uint8, device=dev)
    out = bbp.bmps_decode(d, 0.1, empty, 16)
    assert out["loglik"].shape == (0, 4)
    with pytest.raises(bbp.BbpError):
        bbp.bmps_decode(d, 0.1, torch.from_numpy(syn).to(dev), 17)
    # through the C ABI: a workspace below bbp_bmps_workspace_size is refused before any launch
    sd = torch.from_numpy(syn).to(dev)
    small = torch.empty(16, dtype=torch.uint8, device=dev)
    ll = torch.empty((4, 4), dtype=torch.float64, device=dev)
    cs = torch.empty(4, dtype=torch.uint8, device=dev)
    rc = bbp._lib.lib().bbp_bmps_decode_device(d, 0.1, None, None, sd.data_ptr(), 4, 16, small.data_ptr(), 16,
                                                ll.data_ptr(), cs.data_ptr(), None, None, None)
    assert rc == -1 and b"workspace" in bbp._lib.lib().bbp_last_error()



def test_full_size_sampled(dev):
    """The bench configuration: d=17, p=0.10, chi 16, 4096 syndromes in one launch; eight syndromes spread
    over the batch are recomputed by the oracle."""
    d, p, chi, count = 17, 0.10, 16, 4096
    _say(f"[bmps full] d={d} chi={chi} batch {count}")
    _, syn = workload.make_batch(d, p, count, workload="d17")
    got = _gpu(dev, d, p, syn, chi, timing=True)
    _say(f"   contraction kernel {got['kernel_ms']:.1f} ms")
    idx = np.array([0, 1, 511, 1024, 2047, 3000, 4094, 4095])
    ref = bmps.bmps_coset_loglik(d, syn[idx], network.depolarizing(p), chi)
    sub = {k: got[k][idx] for k in ("loglik", "coset", "correction")}
    _report("sampled gpu vs oracle bMPS", sub["loglik"], ref)
    _check_fp64(sub["loglik"], ref)
    _check_decisions(sub, ref, 1e-5)
    _check_correction(d, syn[idx], sub)
    # a coset estimate may end non-positive (NaN) only far below a finite best one
    ll = got["loglik"]
    best = np.nanmax(ll, axis=1)
    _say(f"   NaN estimates: {int(np.isnan(ll).sum())} of {ll.size}")
    assert np.all(np.isfinite(best))
    assert np.all(np.isnan(ll).sum(axis=1) < 4)


def test_biased_truncated_against_oracle(dev):
    """Biased noise where chi truncates (d=9, chi 8) against the oracle's bMPS with the same Pauli table."""
    d, chi = 9, 8
    probs = workload.biased_probs(0.10, 10.0)
    _, syn = workload.make_batch_pauli(d, probs, 6, p_index=9)
    _say(f"[bmps biased truncated] d={d} chi={chi}")
    got = _gpu(dev, d, probs, syn, chi)
    pI, pX, pZ, pY = probs
    ref = bmps.bmps_coset_loglik(d, syn, np.array([[pI, pZ], [pX, pY]]), chi)
    _report("biased gpu vs oracle bMPS", got["loglik"], ref)
    _check_fp64(got["loglik"], ref)
    _check_decisions(got, ref, 1e-5)
    _check_correction(d, syn, got)


def test_graph_capture_and_replay(dev):
    """The decode launches three kernels and allocates nothing inside the call (the caller owns workspace
    and outputs), so it can be captured into a HIP graph: every replay, with eager work between them, must
    reproduce the eager results bitwise."""
    import torch
    import paper_2402_04834_amd as bbp
    d, chi = 7, 16
    _, syn = workload.make_batch(d, 0.1, 16, workload="test", p_index=5)
    s = torch.from_numpy(syn).to(dev)
    eager = bbp.bmps_decode(d, 0.1, s, chi)
    ws = eager["workspace"]
    torch.cuda.synchronize()
    st = torch.cuda.Stream()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.stream(st):
        bbp.bmps_decode(d, 0.1, s, chi, workspace=ws, stream=st)    # warm-up on the capture stream
        st.synchronize()
        with torch.cuda.graph(g, stream=st):
            cap = bbp.bmps_decode(d, 0.1, s, chi, workspace=ws, stream=st)
    for rep in range(3):
        cap["loglik"].zero_()
        cap["coset"].zero_()
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        for k in ("loglik", "coset", "correction"):
            assert torch.equal(cap[k], eager[k]), (rep, k)
        other = bbp.bmps_decode(5, 0.1, torch.from_numpy(workload.make_batch(5, 0.1, 4)[1]).to(dev), 8)
        torch.cuda.synchronize()
        del other
