"""Pins for the oracle's MPS machinery against dense linear algebra written out independently here."""
import numpy as np
import pytest

from oracle import mps


def _rand_mps(rng, phys, bonds, batch=()):
    return [rng.standard_normal(batch + (bonds[i], p, bonds[i + 1])) for i, p in enumerate(phys)]


def _best_rank(mat, k):
    u, s, vh = np.linalg.svd(mat, full_matrices=False)
    k = min(k, s.size)
    return (u[:, :k] * s[:k]) @ vh[:k]


def test_dense_roundtrip():
    rng = np.random.default_rng(0)
    dims = [2, 3, 2, 2, 4]
    v = rng.standard_normal((3, int(np.prod(dims))))
    np.testing.assert_allclose(mps.to_dense(mps.from_dense(v, dims)), v, atol=1e-12)


def test_left_canonical_isometries_and_state():
    rng = np.random.default_rng(1)
    a = _rand_mps(rng, [2, 2, 3, 2, 2], [1, 3, 5, 4, 2, 1])
    dense = mps.to_dense(a)
    c = mps.left_canonicalize(a)
    np.testing.assert_allclose(mps.to_dense(c), dense, atol=1e-12)
    for A in c[:-1]:
        Dl, p, Dr = A.shape
        mat = A.reshape(Dl * p, Dr)
        np.testing.assert_allclose(mat.T @ mat, np.eye(Dr), atol=1e-12)


def test_compress_exact_when_chi_large():
    rng = np.random.default_rng(2)
    a = _rand_mps(rng, [2] * 6, [1, 4, 8, 8, 8, 4, 1])
    dense = mps.to_dense(a)
    c, ln = mps.compress(a, 64)
    np.testing.assert_allclose(mps.to_dense(c) * np.exp(ln), dense, rtol=1e-10, atol=1e-12)
    assert abs(np.linalg.norm(mps.to_dense(c)) - 1.0) < 1e-12


@pytest.mark.parametrize("chi", [2, 3, 5])
def test_compress_is_sequential_best_rank_truncation(chi):
    # the QR sweep + truncated-SVD sweep equals, cut by cut from the right end, the best rank-chi
    # approximation of the dense state reshaped across that cut
    rng = np.random.default_rng(3 + chi)
    phys = [2, 3, 2, 2, 3, 2]
    a = _rand_mps(rng, phys, [1, 2, 6, 8, 8, 3, 1])
    v = mps.to_dense(a)
    for cut in range(len(phys) - 1, 0, -1):
        left = int(np.prod(phys[:cut]))
        v = _best_rank(v.reshape(left, -1), chi).ravel()
    c, ln = mps.compress(a, chi)
    np.testing.assert_allclose(mps.to_dense(c) * np.exp(ln), v, rtol=1e-9, atol=1e-10)


def test_overlap_and_direct_sum():
    rng = np.random.default_rng(4)
    a = _rand_mps(rng, [2, 2, 2, 2], [1, 2, 3, 2, 1], (5,))
    b = _rand_mps(rng, [2, 2, 2, 2], [1, 2, 4, 2, 1], (5,))
    da, db = mps.to_dense(a), mps.to_dense(b)
    np.testing.assert_allclose(mps.overlap(a, b), (da * db).sum(-1), rtol=1e-12)
    ca, cb = rng.standard_normal(5), rng.standard_normal(5)
    s = mps.direct_sum(a, b, ca, cb)
    np.testing.assert_allclose(mps.to_dense(s), ca[:, None] * da + cb[:, None] * db, atol=1e-12)


def test_canonical_message_static_bonds():
    rng = np.random.default_rng(5)
    K, chi = 6, 32
    v = rng.standard_normal(2 ** K)
    raw = mps.from_dense(v, [2] * K)
    m, ln = mps.canonical_message(raw, chi)
    assert [A.shape[0] for A in m] + [1] == [1, 2, 4, 8, 4, 2, 1]
    np.testing.assert_allclose(mps.to_dense(m), v / np.linalg.norm(v), atol=1e-12)
    np.testing.assert_allclose(ln, np.log(np.linalg.norm(v)), rtol=1e-12)
    for A in m[:-1]:
        Dl, p, Dr = A.shape
        mat = A.reshape(Dl * p, Dr)
        np.testing.assert_allclose(mat.T @ mat, np.eye(Dr), atol=1e-12)
    # a product (rank-one) message keeps the static bonds too, with square orthogonal sites up to the middle
    u = mps.uniform([2] * K, chi)
    assert [A.shape[0] for A in u] + [1] == [1, 2, 4, 8, 4, 2, 1]
    np.testing.assert_allclose(mps.to_dense(u), np.full(2 ** K, 2.0 ** (-K / 2)), atol=1e-12)
    for A in u[:3]:
        Dl, p, Dr = A.shape
        assert Dl * p == Dr
        mat = A.reshape(Dl * p, Dr)
        np.testing.assert_allclose(mat @ mat.T, np.eye(Dr), atol=1e-12)
