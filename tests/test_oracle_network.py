"""Pins for the coset tensor networks and their exact contraction (Sec. II.A, III.A of the paper).

The defining identity is Tr T_s(L) = pi(f_s L G) = sum_{g in G} pi(f_s L g). At d = 3 it is checked against a
brute-force enumeration of all 4^13 Pauli errors that uses only the check supports of the workload
generator (not the tensor network): every error is binned by its syndrome and by its logical class
relative to f_s.
"""
import numpy as np
import pytest

from oracle import lattice, network
from paper_2402_04834_amd import workload


def _bruteforce_coset_probs(d, eps, pi=None):
    """P[s_key, coset] = sum of pi(E) over all errors E with syndrome s in coset f_s L G; pi[x][z] the
    single-qubit Pauli probabilities (default: depolarizing with eps)."""
    n = workload.num_qubits(d)
    m = workload.num_checks(d)
    nz = m // 2                                   # Z-checks come first in the syndrome
    vals = np.arange(1 << n, dtype=np.int64)
    bits = ((vals[:, None] >> np.arange(n)) & 1).astype(np.uint8)     # [2^n, n], qubit i = bit i
    # Z-check syndrome of an X-type error, X-check syndrome of a Z-type error
    sx = workload.syndrome_of(d, bits)[:, :nz]
    sz = workload.syndrome_of(d, 2 * bits)[:, nz:]
    kx = (sx.astype(np.int64) << np.arange(nz)).sum(1)
    kz = (sz.astype(np.int64) << np.arange(nz)).sum(1)
    # class bits relative to f_s: component along logical X is detected by logical Z (column 0) and
    # vice versa; f_s's x part depends only on the Z-check bits, its z part only on the X-check bits
    xm, zm = lattice.logical_masks(d)
    q = lattice.qubits(d)
    xbar = np.array([xm[r, c] for r, c in q], dtype=np.int64)
    zbar = np.array([zm[r, c] for r, c in q], dtype=np.int64)
    full_x = np.concatenate([sx, np.zeros_like(sx)], axis=1)
    full_z = np.concatenate([np.zeros_like(sz), sz], axis=1)
    fx, _ = lattice.pauli_for_syndrome(d, full_x)
    _, fz = lattice.pauli_for_syndrome(d, full_z)
    fxc = lattice.codes_from_pauli_grid(d, fx, np.zeros_like(fx)).astype(np.int64)
    fzc = (lattice.codes_from_pauli_grid(d, np.zeros_like(fz), fz) >> 1).astype(np.int64)
    ax = ((bits.astype(np.int64) ^ fxc) @ zbar) & 1
    az = ((bits.astype(np.int64) ^ fzc) @ xbar) & 1
    pc = np.array([bin(v).count("1") for v in range(1 << n)])
    if pi is None:
        pi = [[1 - eps, eps / 3], [eps / 3, eps / 3]]
    lp = np.log(np.asarray(pi, dtype=np.float64))            # [x][z]
    P = np.zeros((1 << nz, 2, 1 << nz, 2))
    zkey = kz * 2 + az
    for xv in range(1 << n):
        # per-qubit counts of Y (x and z), X (x only), Z (z only) and I for every z pattern
        ny = pc[xv & vals]
        nx = pc[xv] - ny
        nzz = pc[vals] - ny
        ni = n - nx - ny - nzz
        w = np.exp(ni * lp[0, 0] + nx * lp[1, 0] + nzz * lp[0, 1] + ny * lp[1, 1])
        acc = np.bincount(zkey, weights=w, minlength=(1 << nz) * 2).reshape(1 << nz, 2)
        P[kx[xv], ax[xv]] += acc
    # full syndrome key: bit i of the key = syndrome bit i (Z-checks low, X-checks high)
    out = np.zeros((1 << m, 4))
    idx = np.arange(1 << nz)
    key = idx[:, None] + (idx[None, :] << nz)                       # [kx, kz]
    cls = {(0, 0): 0, (1, 0): 1, (1, 1): 2, (0, 1): 3}
    for (a, b), k in cls.items():
        out[key.ravel(), k] = P[:, a, :, b].ravel()
    return out


@pytest.fixture(scope="module")
def bruteforce_d3():
    return _bruteforce_coset_probs(3, 0.1)


def _all_syndromes(m):
    keys = np.arange(1 << m)
    return ((keys[:, None] >> np.arange(m)) & 1).astype(np.uint8)


def test_exact_contraction_equals_bruteforce_d3(bruteforce_d3):
    d, m = 3, 12
    s = _all_syndromes(m)
    got = np.exp(network.exact_coset_loglik(d, s, 0.1))
    np.testing.assert_allclose(got, bruteforce_d3, rtol=1e-10, atol=1e-18)


def test_coset_sum_is_syndrome_probability_d3(bruteforce_d3):
    # sum over the 4 cosets = P(s), and sum over all syndromes = 1
    d, m = 3, 12
    s = _all_syndromes(m)
    got = np.exp(network.exact_coset_loglik(d, s, 0.1)).sum(1)
    np.testing.assert_allclose(got, bruteforce_d3.sum(1), rtol=1e-10)
    assert abs(got.sum() - 1.0) < 1e-12


def test_exact_contraction_equals_bruteforce_biased_d3():
    """Biased Pauli noise (each of I, X, Z, Y its own probability): the qubit tensors take pi[x][z]."""
    d, m = 3, 12
    pi = np.array([[0.85, 0.09], [0.04, 0.02]])          # [x][z]: I, Z / X, Y
    ref = _bruteforce_coset_probs(d, None, pi)
    s = _all_syndromes(m)
    x, z = lattice.coset_labels(d, s)
    got = np.exp(network.exact_log_contraction(d, x, z, pi))
    np.testing.assert_allclose(got, ref, rtol=1e-10, atol=1e-18)
    assert abs(ref.sum() - 1.0) < 1e-12


@pytest.mark.parametrize("d", [3, 5, 7])
def test_uniform_noise_closed_form(d):
    # eps = 3/4 makes every Pauli equally likely (1/4 per qubit): pi(coset) = 2^m * 4^-n for every syndrome
    rng = np.random.default_rng(1)
    m, n = 2 * d * (d - 1), d * d + (d - 1) ** 2
    s = rng.integers(0, 2, size=(3, m), dtype=np.uint8)
    got = network.exact_coset_loglik(d, s, 0.75)
    np.testing.assert_allclose(got, (m - 2 * n) * np.log(2.0), rtol=0, atol=1e-10)


@pytest.mark.parametrize("d", [3, 5])
def test_transpose_symmetry(d):
    # depolarizing noise is X/Z symmetric: transposing the lattice swaps the check types, so the network of
    # labels (x, z) and the one of (z^T, x^T) contract to the same value
    rng = np.random.default_rng(2)
    L = 2 * d - 1
    x = rng.integers(0, 2, size=(4, L, L), dtype=np.uint8)
    z = rng.integers(0, 2, size=(4, L, L), dtype=np.uint8)
    pi = network.depolarizing(0.13)
    a = network.exact_log_contraction(d, x, z, pi)
    b = network.exact_log_contraction(d, np.swapaxes(z, -1, -2), np.swapaxes(x, -1, -2), pi)
    np.testing.assert_allclose(a, b, rtol=1e-12)


def test_stabilizer_multiplication_leaves_coset_unchanged():
    # multiplying the label by a check generator stays in the same coset of G
    d = 5
    rng = np.random.default_rng(3)
    s = rng.integers(0, 2, size=(2, 2 * d * (d - 1)), dtype=np.uint8)
    x, z = lattice.coset_labels(d, s)
    pi = network.depolarizing(0.1)
    base = network.exact_log_contraction(d, x, z, pi)
    x2, z2 = x.copy(), z.copy()
    for (r, c) in [lattice.checks(d)[3], lattice.checks(d)[-2]]:
        for rr, cc in lattice.neighbours(d, r, c):
            if r % 2 == 0:
                z2[..., rr, cc] ^= 1
            else:
                x2[..., rr, cc] ^= 1
    np.testing.assert_allclose(network.exact_log_contraction(d, x2, z2, pi), base, rtol=1e-12)


# Coset probabilities at d = 3, eps = 0.1 (order I, X, Y, Z) for four syndromes, from an enumeration of all
# 4^13 errors written independently of oracle/ (key = sum_i s_i 2^i, Z-checks first).
# They fix the conventions of the syndrome order, the chains of f_s and the logical representatives
# together: a transposed check order or a logical on the wrong boundary moves these values between columns.
T1_D3_EPS010 = {
    0: (2.542961146460e-01, 4.503023314070e-05, 4.059547115007e-07, 4.503023314070e-05),
    1: (9.794635497390e-03, 3.918170363417e-04, 1.885841496142e-06, 1.676060097254e-05),
    2608: (6.515426510093e-05, 3.537310818141e-04, 2.227326173760e-06, 2.303217803742e-06),
    4095: (3.655236905926e-07, 1.207486874366e-07, 1.494542070982e-06, 1.207486874366e-07),
}


@pytest.mark.parametrize("key", sorted(T1_D3_EPS010))
def test_literal_coset_probabilities_d3(key, bruteforce_d3):
    want = np.array(T1_D3_EPS010[key])
    s = ((key >> np.arange(12)) & 1).astype(np.uint8)[None]
    np.testing.assert_allclose(bruteforce_d3[key], want, rtol=1e-11)
    np.testing.assert_allclose(np.exp(network.exact_coset_loglik(3, s, 0.1))[0], want, rtol=1e-11)
