"""Pins of the warm-start oracle (oracle/warmnet.py): finite-difference gradients on tiny networks,
the adjointness of im2col / col2im, a 3x3 convolution against its definition, the head's closed form
without pairwise terms, loss invariances and the input channels."""
import numpy as np
import pytest

from oracle import blockbp, warmnet
from paper_2402_04834_amd import workload

TINY = (3, 4, 2)


def _job(d, p=0.1, k=3, seed=0):
    _, syn = workload.make_batch(d, p, 1, workload="warm", p_index=seed)
    lab = warmnet.job_labels(d, syn[0])
    X0 = warmnet.features(d, syn[0], p, seed % 4)
    return X0, blockbp.Plan(d, k, k), syn[0], lab


def test_input_channels():
    d = 5
    L = 2 * d - 1
    _, syn = workload.make_batch(d, 0.1, 1, workload="warm", p_index=0)
    lab = warmnet.job_labels(d, syn[0])
    for coset in range(4):
        X0 = warmnet.features(d, syn[0], 0.1, coset)
        kinds = X0[..., 3] + X0[..., 4] + X0[..., 5]
        assert np.all(kinds == 1.0)
        assert X0[..., 2].sum() == syn[0].sum()
        for r in range(L):
            for c in range(L):
                if (r + c) % 2 == 0:
                    assert X0[r, c, 0] + 2 * X0[r, c, 1] == lab[coset, r, c]
        assert np.all(X0[..., 7] == 1.0) and np.allclose(X0[..., 6], 0.1)
        assert np.all(X0[..., 8] == (coset in (1, 2))) and np.all(X0[..., 9] == (coset in (2, 3)))


@pytest.mark.parametrize("d", [3, 5, 7])
def test_generator_bits_clear_the_horizontal_edges(d):
    """Multiplying the coset label by the plaquettes (x part) and vertices (z part) whose G bit is 1 leaves
    no x on the horizontal edges but the last row, and no z on the horizontal edges but the last column
    (a plaquette flips x on its 4 edges, a vertex flips z on its 4 edges)."""
    L = 2 * d - 1
    _, syn = workload.make_batch(d, 0.15, 4, workload="warm", p_index=77)
    for s in syn:
        lab = warmnet.job_labels(d, s)
        for coset in range(4):
            X0 = warmnet.features(d, s, 0.15, coset)
            x = (lab[coset] & 1).copy()
            z = ((lab[coset] >> 1) & 1).copy()
            for r in range(L):
                for c in range(L):
                    if (r + c) % 2 == 0 or X0[r, c, 10] == 0:
                        continue
                    tgt = x if r % 2 == 1 else z
                    for rr, cc in ((r - 1, c), (r + 1, c), (r, c - 1), (r, c + 1)):
                        if 0 <= rr < L and 0 <= cc < L:
                            tgt[rr, cc] ^= 1
            for r in range(0, L, 2):
                for c in range(0, L, 2):
                    if r != L - 1:
                        assert x[r, c] == 0, (r, c)
                    if c != L - 1:
                        assert z[r, c] == 0, (r, c)


def test_im2col_col2im_adjoint():
    rng = np.random.default_rng(1)
    X = rng.normal(size=(7, 7, 3))
    G = rng.normal(size=(49, 27))
    assert np.isclose((warmnet.im2col(X) * G).sum(), (X * warmnet.col2im(G, 7, 3)).sum())


def test_conv_matches_definition():
    rng = np.random.default_rng(2)
    L, ci, co = 5, 2, 3
    X = rng.normal(size=(L, L, ci))
    W = rng.normal(size=(9 * ci, co))
    b = rng.normal(size=co)
    Y = warmnet.conv(X, W, b)
    for r in range(L):
        for c in range(L):
            for o in range(co):
                acc = b[o]
                for dy in range(3):
                    for dx in range(3):
                        rr, cc = r + dy - 1, c + dx - 1
                        if 0 <= rr < L and 0 <= cc < L:
                            for i in range(ci):
                                acc += X[rr, cc, i] * W[(dy * 3 + dx) * ci + i, o]
                assert np.isclose(Y[r, c, o], acc)


def test_head_without_pairwise_terms_is_a_product():
    # with Wp = bp = 0 the message is the normalised Kronecker product of the legs' exp(u_i)
    rng = np.random.default_rng(3)
    d, plan = 5, blockbp.Plan(5, 3, 3)
    theta = rng.normal(size=warmnet.count(TINY)) * 0.3
    prm = warmnet.unpack(theta, TINY)
    for k in range(4):
        prm[f"head{k}.Wp"][:] = 0.0
        prm[f"head{k}.bp"][:] = 0.0
    X0, _, _, _ = _job(d)
    F, _ = warmnet.trunk(prm, X0)
    e = 0
    lg = warmnet.legs(d, plan, e)
    direction = warmnet.direction_of(plan, e)
    m = warmnet.head_message(prm, F, lg, direction)
    v = np.ones(1)
    for a, b in lg:
        u = np.concatenate([F[a], F[b]]) @ prm[f"head{direction}.Wu"] + prm[f"head{direction}.bu"]
        v = np.kron(v, np.exp(u))
    np.testing.assert_allclose(m, v / np.linalg.norm(v), rtol=1e-12)


def test_legs_cross_the_boundary():
    d = 7
    plan = blockbp.Plan(d, 4, 4)
    for e in range(plan.M):
        (I, J), (I2, J2), _ = plan.edges[e]
        lg = warmnet.legs(d, plan, e)
        assert len(lg) == plan.msg_len((I, J), (I2, J2))
        for a, b in lg:
            assert abs(a[0] - b[0]) + abs(a[1] - b[1]) == 1          # adjacent sites
            inside = lambda s, B: plan.rows[B[0]][0] <= s[0] < sum(plan.rows[B[0]]) and \
                plan.cols[B[1]][0] <= s[1] < sum(plan.cols[B[1]])
            assert inside(a, (I, J)) and inside(b, (I2, J2))


def test_loss_is_zero_on_its_own_prediction_and_scale_invariant():
    rng = np.random.default_rng(4)
    d = 5
    X0, plan, _, _ = _job(d)
    theta = rng.normal(size=warmnet.count(TINY)) * 0.3
    pred = warmnet.predict(theta, X0, d, plan, TINY)
    ids = list(range(plan.M))
    l0, g0 = warmnet.loss_and_grad(theta, X0, d, plan, pred, ids, TINY)
    l1, _ = warmnet.loss_and_grad(theta, X0, d, plan, 3.0 * pred, ids, TINY)
    assert abs(l0) < 1e-12 and abs(l1) < 1e-12
    assert np.abs(g0).max() < 1e-12
    # any other target gives a positive loss (KL divergence of distinct distributions)
    other = pred.copy()
    other[0, :2] = other[0, 1::-1]
    assert warmnet.loss_and_grad(theta, X0, d, plan, other, ids, TINY)[0] > 0


@pytest.mark.parametrize("d,k", [(3, 2), (5, 3)])
def test_gradient_matches_finite_differences(d, k):
    rng = np.random.default_rng(5 + d)
    X0, _, _, _ = _job(d, k=k, seed=d)
    plan = blockbp.Plan(d, k, k)
    theta = rng.normal(size=warmnet.count(TINY)) * 0.4
    # targets: unit vectors with positive entries, zero beyond 2^K
    T = np.zeros((plan.M, 64))
    for e in range(plan.M):
        K = len(warmnet.legs(d, plan, e))
        t = rng.uniform(0.1, 1.0, size=2 ** K)
        T[e, :2 ** K] = t / np.linalg.norm(t)
    ids = list(range(plan.M))
    _, g = warmnet.loss_and_grad(theta, X0, d, plan, T, ids, TINY)
    h = 1e-6
    for j in range(theta.size):
        tp, tm = theta.copy(), theta.copy()
        tp[j] += h
        tm[j] -= h
        fd = (warmnet.loss_and_grad(tp, X0, d, plan, T, ids, TINY)[0] -
              warmnet.loss_and_grad(tm, X0, d, plan, T, ids, TINY)[0]) / (2 * h)
        assert abs(fd - g[j]) <= 1e-6 + 1e-5 * abs(fd), (j, fd, g[j])


def test_bf16_rounding():
    """round_bf16 keeps 8 significant bits with ties to even, and is the identity on BF16 values."""
    x = np.array([1.0, 1.0 + 2 ** -8, 1.0 + 2 ** -7, 1.0 + 3 * 2 ** -8, -2.5, 0.0, 3.0e-30, 65536.0 * 1.00390625])
    r = warmnet.round_bf16(x)
    np.testing.assert_array_equal(r, [1.0, 1.0, 1.0 + 2 ** -7, 1.0 + 2 ** -6, -2.5, 0.0, r[6], 65536.0])
    assert abs(r[6] - 3.0e-30) <= 2 ** -8 * 3.0e-30
    np.testing.assert_array_equal(warmnet.round_bf16(r), r)
    rng = np.random.default_rng(9)
    y = rng.normal(size=1000) * 10.0
    # 8 significant bits: relative error <= 2^-8; float64 values pass through float32 first (the values the
    # GPU rounds are float32), which adds 2^-24
    assert np.all(np.abs(warmnet.round_bf16(y) - y) <= (2 ** -8 + 2 ** -24) * np.abs(y))


def test_trunk_store_identity_is_exact():
    rng = np.random.default_rng(10)
    X0, _, _, _ = _job(5)
    theta = rng.normal(size=warmnet.count(TINY)) * 0.3
    prm = warmnet.unpack(theta, TINY)
    a, _ = warmnet.trunk(prm, X0)
    b, _ = warmnet.trunk(prm, X0, store=lambda t: t)
    np.testing.assert_array_equal(a, b)


@pytest.mark.parametrize("d,k", [(5, 3), (7, 4)])
def test_composed_last_layer_equals_the_network(d, k):
    """predict_stored with exact storage (the last convolution composed with the head's weights, the head
    then summing per-site projections) gives the network's own messages: the composition only regroups the
    head's linear maps."""
    rng = np.random.default_rng(11 + d)
    X0, _, _, _ = _job(d, k=k, seed=d)
    plan = blockbp.Plan(d, k, k)
    theta = rng.normal(size=warmnet.count(TINY)) * 0.3
    a = warmnet.predict(theta, X0, d, plan, TINY)
    b = warmnet.predict_stored(theta, X0, d, plan, lambda t: t, TINY)
    np.testing.assert_allclose(b, a, rtol=1e-10, atol=1e-13)
    # and rounding the stored values changes them (the pin is not vacuous)
    c = warmnet.predict_stored(theta, X0, d, plan, warmnet.round_bf16, TINY)
    assert np.abs(c - a).max() > 1e-6
