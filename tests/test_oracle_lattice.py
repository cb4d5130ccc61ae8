"""Pins for the oracle's surface-code geometry (Sec. II.B of the paper)."""
import numpy as np
import pytest

from oracle import lattice
from paper_2402_04834_amd import workload


def _pauli_of_check(d, r, c):
    L = lattice.side(d)
    x = np.zeros((L, L), dtype=np.uint8)
    z = np.zeros((L, L), dtype=np.uint8)
    for rr, cc in lattice.neighbours(d, r, c):
        if r % 2 == 0:
            z[rr, cc] = 1      # A_u = product of Z on the edges at a site
        else:
            x[rr, cc] = 1      # B_p = product of X around a plaquette
    return x, z


@pytest.mark.parametrize("d", [2, 3, 5, 7])
def test_counts(d):
    # n = d^2 + (d-1)^2 qubits, m = 2d(d-1) checks, one logical qubit (Sec. II.B)
    assert len(lattice.qubits(d)) == d * d + (d - 1) ** 2
    assert len(lattice.checks(d)) == 2 * d * (d - 1)
    assert len(lattice.qubits(d)) - len(lattice.checks(d)) == 1
    h = [q for q in lattice.qubits(d) if q[0] % 2 == 0]
    assert len(h) == d * d


@pytest.mark.parametrize("d", [3, 4, 5])
def test_checks_and_logicals_commute(d):
    ch = [_pauli_of_check(d, r, c) for r, c in lattice.checks(d)]
    for a in ch:
        for b in ch:
            assert lattice.commutes(a[0], a[1], b[0], b[1]) == 1
    xm, zm = lattice.logical_masks(d)
    zero = np.zeros_like(xm)
    for cx, cz in ch:
        assert lattice.commutes(xm, zero, cx, cz) == 1
        assert lattice.commutes(zero, zm, cx, cz) == 1
    assert lattice.commutes(xm, zero, zero, zm) == 0   # logical X and Z anticommute


@pytest.mark.parametrize("d", [3, 5, 7])
def test_pauli_for_syndrome_reproduces_syndrome(d):
    rng = np.random.default_rng(d)
    s = rng.integers(0, 2, size=(50, 2 * d * (d - 1)), dtype=np.uint8)
    fx, fz = lattice.pauli_for_syndrome(d, s)
    codes = lattice.codes_from_pauli_grid(d, fx, fz)
    # syndrome measured by the workload generator's own check supports
    np.testing.assert_array_equal(workload.syndrome_of(d, codes), s)
    np.testing.assert_array_equal(lattice.syndrome_of_grid(d, fx, fz), s)


def test_coset_labels_differ_by_logicals():
    d = 5
    s = np.zeros((1, 2 * d * (d - 1)), dtype=np.uint8)
    s[0, [1, 7, 30]] = 1
    x, z = lattice.coset_labels(d, s)
    xm, zm = lattice.logical_masks(d)
    np.testing.assert_array_equal(x[0, 1] ^ x[0, 0], xm)
    np.testing.assert_array_equal(z[0, 3] ^ z[0, 0], zm)
    np.testing.assert_array_equal(x[0, 2] ^ x[0, 0], xm)
    np.testing.assert_array_equal(z[0, 2] ^ z[0, 0], zm)
    for k in range(4):   # every coset representative carries the same syndrome
        np.testing.assert_array_equal(lattice.syndrome_of_grid(d, x[:, k], z[:, k]), s)


def test_pauli_sampler_frequencies():
    """The biased sampler draws I, X, Z, Y with the given probabilities (4 sigma of the binomial)."""
    probs = workload.biased_probs(0.1, 10.0)
    assert abs(sum(probs) - 1.0) < 1e-12 and abs(probs[2] / (probs[1] + probs[3]) - 10.0) < 1e-9
    e, s = workload.make_batch_pauli(9, probs, 400, p_index=3)
    n = e.size
    for code, pr in enumerate(probs):
        f = np.mean(e == code)
        assert abs(f - pr) <= 4 * np.sqrt(pr * (1 - pr) / n) + 1e-12, (code, f, pr)
    np.testing.assert_array_equal(s, workload.syndrome_of(9, e))
