"""Pins for the boundary-MPS oracle (the single-block limit of blockBP, Sec. III.A and III.D of the paper).

Where chi is at least the largest Schmidt rank across a row cut, 2^floor(L/2), the compression keeps every
singular value and bMPS is an exact contraction: it must equal the exact column-transfer contraction of
`oracle.network` (itself pinned to brute force over all Pauli errors), for depolarizing and biased noise,
and its decisions must be the exact DQMLD decisions. Below that rank the result is an approximation whose
error shrinks as chi grows.
"""
import numpy as np
import pytest

from oracle import bmps, lattice, network
from paper_2402_04834_amd import workload


def _biased_table(p, eta):
    pI, pX, pZ, pY = workload.biased_probs(p, eta)
    return np.array([[pI, pZ], [pX, pY]])     # pi[x][z]


@pytest.mark.parametrize("d,chi", [(2, 2), (3, 4), (5, 16)])
@pytest.mark.parametrize("p", [0.03, 0.10, 0.18])
def test_exact_when_chi_covers_the_schmidt_rank(d, chi, p):
    _, syn = workload.make_batch(d, p, 12, workload="test")
    ll, tw = bmps.bmps_coset_loglik(d, syn, network.depolarizing(p), chi, with_truncation=True)
    ex = network.exact_coset_loglik(d, syn, p)
    np.testing.assert_allclose(ll, ex, rtol=0, atol=1e-9)
    assert np.all(tw < 1e-20)
    top2 = np.sort(ex, axis=-1)[:, -2:]
    clear = top2[:, 1] - top2[:, 0] > 1e-6           # exact ties (small d) may go either way
    np.testing.assert_array_equal(bmps.decide(ll)[clear], bmps.decide(ex)[clear])


def test_exact_for_biased_noise():
    d, p = 5, 0.12
    probs = workload.biased_probs(p, 4.0)
    _, syn = workload.make_batch_pauli(d, probs, 8)
    pi = _biased_table(p, 4.0)
    x, z = lattice.coset_labels(d, syn)
    np.testing.assert_allclose(bmps.bmps_log_contraction(d, x, z, pi, 16),
                               network.exact_log_contraction(d, x, z, pi), rtol=0, atol=1e-9)


def test_schmidt_rank_bound_is_tight():
    """One below the largest Schmidt rank the compression must discard weight on some syndrome, so the
    exactness above is not an accident of small ranks."""
    d, p = 5, 0.10
    _, syn = workload.make_batch(d, p, 12, workload="test")
    _, tw = bmps.bmps_coset_loglik(d, syn, network.depolarizing(p), 8, with_truncation=True)
    assert tw.max() > 1e-12


def test_truncation_error_shrinks_with_chi():
    d, p = 7, 0.10
    _, syn = workload.make_batch(d, p, 4, workload="test")
    pi = network.depolarizing(p)
    ex = network.exact_coset_loglik(d, syn, p)
    err = [np.abs(bmps.bmps_coset_loglik(d, syn, pi, chi) - ex).max() for chi in (2, 4, 16)]
    assert err[0] > err[1] > err[2]
    assert err[2] < 1e-2


def test_decide_nan_and_ties():
    ll = np.array([[np.nan, -3.0, -3.0, -5.0], [-1.0, -1.0, np.nan, -2.0], [np.nan] * 4])
    np.testing.assert_array_equal(bmps.decide(ll), [1, 0, 0])
