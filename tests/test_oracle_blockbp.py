"""Pins for the oracle's blockBP: closed forms, trees, the single-block limit, dense contraction of a block,
Lemma 3.1 against the direct Bethe free energy, exact symmetries, and the decision rule."""
import numpy as np
import pytest

from oracle import blockbp, lattice, mps, network
from paper_2402_04834_amd import workload

from dense_sweep import dense_update


def _coset_tensors(d, syndromes, eps):
    x, z = lattice.coset_labels(d, syndromes)
    L = 2 * d - 1
    S = syndromes.shape[0]
    return network.coset_tensors(d, x.reshape(S * 4, L, L), z.reshape(S * 4, L, L), network.depolarizing(eps))


@pytest.mark.parametrize("d,block,chi", [(3, (2, 2), 4), (3, (3, 2), 2), (5, (3, 3), 4), (5, (4, 4), 16)])
def test_uniform_noise_closed_form(d, block, chi):
    # eps = 3/4: constant qubit tensors, the uniform messages are a BP fixed point and the Bethe estimate
    # is exact: ln Z = (m - 2n) ln 2 for every syndrome and coset; BP stops after one iteration
    _, s = workload.make_batch(d, 0.1, 3)
    r = blockbp.decode(d, 0.75, s, block=block, chi=chi, max_iter=5)
    m, n = 2 * d * (d - 1), d * d + (d - 1) ** 2
    np.testing.assert_allclose(r["loglik"], (m - 2 * n) * np.log(2.0), atol=1e-10)
    assert (r["iters"] == 1).all()
    assert (r["delta"] < 1e-6).all()


@pytest.mark.parametrize("d,block,chi", [(3, (5, 1), 8), (3, (1, 5), 8), (3, (5, 2), 8), (5, (9, 2), 16),
                                         (5, (3, 9), 16)])
def test_tree_partition_is_exact(d, block, chi):
    # one block row (or column) makes the block graph a path; BP is exact on trees (Sec. III.B-C) and the
    # Bethe estimate of Lemma 3.1 equals the contraction when chi never truncates
    _, s = workload.make_batch(d, 0.12, 3)
    ex = network.exact_coset_loglik(d, s, 0.12)
    r = blockbp.decode(d, 0.12, s, block=block, chi=chi, max_iter=8, eta=0.0, fixed_iters=True)
    np.testing.assert_allclose(r["loglik"], ex, atol=1e-9)


@pytest.mark.parametrize("d,chi", [(3, 4), (5, 16)])
def test_single_block_is_bmps_and_exact(d, chi):
    # one block covering the lattice: blockBP is the boundary-MPS contraction (Sec. III.D), exact once chi
    # reaches the natural bond dimension
    L = 2 * d - 1
    _, s = workload.make_batch(d, 0.1, 3)
    ex = network.exact_coset_loglik(d, s, 0.1)
    r = blockbp.decode(d, 0.1, s, block=(L, L), chi=chi, max_iter=1)
    np.testing.assert_allclose(r["loglik"], ex, atol=1e-9)
    r2 = blockbp.decode(d, 0.1, s, block=(L, L), chi=2, max_iter=1)
    if d == 5:   # a binding chi changes the estimate
        assert np.nanmax(np.abs(r2["loglik"] - ex)) > 1e-6


def _block_einsum(tensors, plan, I, J, frame, dense_in):
    """Dense contraction of block (I, J) with dense incoming messages (dict side -> vector or None),
    leaving the legs on side `frame` open (the BP update rule, Sec. III.C)."""
    r0, kr = plan.rows[I]
    c0, kc = plan.cols[J]
    letters = iter("ABCDEFGHIJKLMNOPQRSTUVWXYZabcdefghijklmnopqrstuvwxyz")
    hb = {}   # horizontal bond between (r, c) and (r, c+1): key (r, c)
    vb = {}   # vertical bond between (r, c) and (r+1, c): key (r, c)
    for r in range(r0 - 1, r0 + kr):
        for c in range(c0 - 1, c0 + kc):
            hb[(r, c)] = next(letters)
            vb[(r, c)] = next(letters)
    ops, subs = [], []
    for r in range(r0, r0 + kr):
        for c in range(c0, c0 + kc):
            t = tensors[r][c][0]
            ops.append(t)
            subs.append(vb[(r - 1, c)] + hb[(r, c - 1)] + vb[(r, c)] + hb[(r, c)])
    sides = {"W": [hb[(r, c0 - 1)] for r in range(r0, r0 + kr)],
             "E": [hb[(r, c0 + kc - 1)] for r in range(r0, r0 + kr)],
             "N": [vb[(r0 - 1, c)] for c in range(c0, c0 + kc)],
             "S": [vb[(r0 + kr - 1, c)] for c in range(c0, c0 + kc)]}
    for side, legs in sides.items():
        if side == frame:
            continue
        v = dense_in.get(side)
        if v is None:
            continue
        ops.append(np.asarray(v).reshape((2,) * len(legs)))
        subs.append("".join(legs))
    out = "".join(sides[frame])
    res = np.einsum(",".join(subs) + "->" + out, *ops, optimize=True)
    return res.reshape(-1)


def _random_messages(plan, I, J, rng, chi):
    me = (I, J)
    dense, msgs = {}, {}
    for side, (dI, dJ) in blockbp.DIRS.items():
        nb = (I + dI, J + dJ)
        if not plan.has(nb):
            dense[side] = None
            continue
        K = plan.msg_len(nb, me)
        v = rng.uniform(0.05, 1.0, size=2 ** K)
        v /= np.linalg.norm(v)
        dense[side] = v
        msgs[(nb, me)], _ = mps.canonical_message(mps.from_dense(v[None], [2] * K), chi)
    return dense, msgs


def _vec(v, n):
    """Dense vector padded to n entries (legs of dimension 1 at the lattice edge give fewer entries)."""
    out = np.zeros(n)
    out[: v.size] = v
    return out


@pytest.mark.parametrize("frame", ["E", "W", "S", "N"])
@pytest.mark.parametrize("d,block,IJ", [(5, (3, 3), (1, 1)), (5, (3, 3), (2, 0)), (5, (4, 3), (2, 1))])
def test_block_update_equals_dense_contraction(frame, d, block, IJ):
    # with chi above every natural bond the boundary-MPS sweep is exact: the outgoing message equals the
    # dense contraction of the block with its other incoming messages, up to the split-off scale
    rng = np.random.default_rng(hash((frame, d, block, IJ)) % 2 ** 32)
    _, s = workload.make_batch(d, 0.1, 1)
    tensors = _coset_tensors(d, s, 0.1)
    tensors = [[t[:1] for t in row] for row in tensors]
    plan = blockbp.Plan(d, *block)
    I, J = IJ
    dI, dJ = blockbp.DIRS[frame]
    if not plan.has((I + dI, J + dJ)):
        pytest.skip("no receiver on that side")
    dense_in, msgs = _random_messages(plan, I, J, rng, 64)
    ref = _block_einsum(tensors, plan, I, J, frame, dense_in)
    out, ls = blockbp.block_sweep(plan, tensors, msgs, I, J, frame, 64, (1,))
    got = mps.to_dense(out)[0] * np.exp(ls[0])
    np.testing.assert_allclose(got, ref, rtol=1e-10, atol=1e-14 * np.abs(ref).max())


def _interior_6x6(chi, frame, seed):
    d = 7
    rng = np.random.default_rng(seed)
    _, s = workload.make_batch(d, 0.1, 1)
    tensors = _coset_tensors(d, s, 0.1)
    tensors = [[t[:1] for t in row] for row in tensors]
    plan = blockbp.Plan(d, 6, 6)
    I, J = 1, 1
    dense_in, msgs = _random_messages(plan, I, J, rng, chi)
    out, ls = blockbp.block_sweep(plan, tensors, msgs, I, J, frame, chi, (1,))
    got = mps.to_dense(out)[0] * np.exp(ls[0])
    r0, kr = plan.rows[I]
    c0, kc = plan.cols[J]
    blk = [[tensors[r][c][0] for c in range(c0, c0 + kc)] for r in range(r0, r0 + kr)]
    opposite = {"E": "W", "W": "E", "S": "N", "N": "S"}[frame]
    caps = {"E": ("N", "S"), "W": ("N", "S"), "S": ("W", "E"), "N": ("W", "E")}[frame]
    args = (blk, frame, dense_in[opposite], dense_in[caps[0]], dense_in[caps[1]])
    return got, args, (tensors, plan, dense_in)


@pytest.mark.parametrize("frame", ["E", "W", "S", "N"])
@pytest.mark.parametrize("chi", [16, 32])
def test_sixbysix_block_never_truncates_at_chi_16(frame, chi):
    # the Schmidt rank of the boundary state of a 6x6 block never exceeds 16 (the COPY checks tie many
    # bond values together), so the chi-truncated sweep equals the exact block contraction
    seed = 11 + ord(frame)
    got, args, _ = _interior_6x6(chi, frame, seed)
    ref, _, _ = _interior_6x6(4096, frame, seed)      # chi above every dimension: no truncation possible
    np.testing.assert_allclose(got, ref, rtol=1e-9, atol=1e-12 * np.abs(ref).max())
    dense, ld = dense_update(*args, 4096)
    np.testing.assert_allclose(got, dense * np.exp(ld), rtol=1e-9, atol=1e-12 * np.abs(ref).max())


@pytest.mark.parametrize("frame", ["E", "W", "S", "N"])
@pytest.mark.parametrize("chi", [8, 12])
def test_truncating_sweep_is_sequential_best_rank_truncation_of_the_dense_state(frame, chi):
    # below rank 16 the truncation acts; the MPS sweep must then equal the dense state truncated cut by
    # cut from the bottom to its best rank-chi approximation, with every cap indexed by the message legs it
    # has not absorbed yet (the gauge-free form of a cap whose remaining part is an isometry)
    seed = 3 + chi + ord(frame)
    got, args, _ = _interior_6x6(chi, frame, seed)
    dense, ld = dense_update(*args, chi, caps="remaining")
    scale = np.abs(got).max()
    np.testing.assert_allclose(got, dense * np.exp(ld), rtol=1e-7, atol=1e-9 * scale)
    exact, _, _ = _interior_6x6(4096, frame, seed)
    assert np.abs(exact - got).max() > 1e-6 * scale          # the truncation really acted


def _uniform_caps(plan, I, J, chi, kind, rng):
    """The uniform start message of every neighbour of block (I, J) in one of three exact left-canonical
    forms: as the oracle builds it (zero-padded product), from the dense vector by successive QR, and the
    first with a random orthogonal gauge on every bond."""
    me = (I, J)
    msgs = {}
    for side, (dI, dJ) in blockbp.DIRS.items():
        nb = (I + dI, J + dJ)
        if not plan.has(nb):
            continue
        K = plan.msg_len(nb, me)
        if kind == "dense":
            v = np.full((1, 2 ** K), 2.0 ** (-K / 2))
            msgs[(nb, me)], _ = mps.canonical_message(mps.from_dense(v, [2] * K), chi)
            continue
        m = [x.copy() for x in mps.uniform([2] * K, chi, (1,))]
        if kind == "gauge":
            for j in range(K - 1):
                G, _ = np.linalg.qr(rng.normal(size=(m[j].shape[-1],) * 2))
                m[j] = np.einsum("...apb,bc->...apc", m[j], G)
                m[j + 1] = np.einsum("cb,...bpe->...cpe", G.T, m[j + 1])
        msgs[(nb, me)] = m
    return msgs


@pytest.mark.parametrize("frame", ["E", "W", "S", "N"])
def test_truncating_sweep_does_not_depend_on_the_canonical_form_of_its_caps(frame):
    # the uniform start is rank 1 at every bond, so its left-canonical sites hold weightless completion
    # directions that differ between exact constructions; the truncated sweep must not see them (chi = 4:
    # with product caps the boundary rank stays within 8)
    d, chi = 7, 4
    _, s = workload.make_batch(d, 0.1, 1)
    tensors = [[t[:1] for t in row] for row in _coset_tensors(d, s, 0.1)]
    plan = blockbp.Plan(d, 6, 6)
    rng = np.random.default_rng(ord(frame))
    outs = []
    for kind in ("pad", "dense", "gauge"):
        out, ls = blockbp.block_sweep(plan, tensors, _uniform_caps(plan, 1, 1, chi, kind, rng), 1, 1, frame, chi, (1,))
        outs.append(mps.to_dense(out)[0] * np.exp(ls[0]))
    scale = np.abs(outs[0]).max()
    for o in outs[1:]:
        np.testing.assert_allclose(o, outs[0], rtol=0, atol=1e-11 * scale)
    exact, _ = blockbp.block_sweep(plan, tensors, _uniform_caps(plan, 1, 1, 4096, "pad", rng), 1, 1, frame, 4096, (1,))
    assert np.abs(mps.to_dense(exact)[0] * np.exp(_[0]) - outs[0]).max() > 1e-6 * scale   # truncation acted


def test_lemma_matches_direct_bethe_free_energy():
    # Lemma 3.1 vs the Bethe free energy written from vertex and edge marginals (eq. Bethe-orig, App. A),
    # for plain BP (one tensor per block) at a converged fixed point
    d, eps = 3, 0.1
    _, s = workload.make_batch(d, eps, 2)
    r = blockbp.decode(d, eps, s, block=(1, 1), chi=2, max_iter=400, eta=0.3, delta0=1e-15,
                       return_messages=True)
    x, z = lattice.coset_labels(d, s)
    L = 2 * d - 1
    tensors = network.coset_tensors(d, x.reshape(-1, L, L), z.reshape(-1, L, L), network.depolarizing(eps))
    msgs = r["messages"]
    conv = r["delta"].ravel() < 1e-12
    assert conv.sum() >= 4
    F = np.zeros(x.shape[0] * 4)
    vec = lambda a, b: msgs[(a, b)][0][:, 0, :, 0]           # [B, 2]
    for rr in range(L):
        for cc in range(L):
            T = tensors[rr][cc]
            P = T.copy()
            for axis, nb in enumerate([(rr - 1, cc), (rr, cc - 1), (rr + 1, cc), (rr, cc + 1)]):
                if 0 <= nb[0] < L and 0 <= nb[1] < L:
                    shape = [P.shape[0], 1, 1, 1, 1]
                    shape[1 + axis] = 2
                    P = P * vec(nb, (rr, cc)).reshape(shape)
            P = P / P.sum(axis=(1, 2, 3, 4), keepdims=True)
            safe = np.where(P > 0, P / np.where(T > 0, T, 1.0), 1.0)
            F += np.sum(np.where(P > 0, P * np.log(safe), 0.0), axis=(1, 2, 3, 4))
    for rr in range(L):
        for cc in range(L):
            for nb in [(rr + 1, cc), (rr, cc + 1)]:
                if nb[0] < L and nb[1] < L:
                    Pe = vec((rr, cc), nb) * vec(nb, (rr, cc))
                    Pe = Pe / Pe.sum(axis=1, keepdims=True)
                    F -= np.sum(np.where(Pe > 0, Pe * np.log(np.where(Pe > 0, Pe, 1.0)), 0.0), axis=1)
    np.testing.assert_allclose(r["loglik"].ravel()[conv], -F[conv], atol=1e-9)


def test_invariance_under_stabilizer_and_logical_relabelling():
    # f_s -> f_s g (g a stabilizer) permutes bond values by X on the bonds of one check: an orthogonal map,
    # so blockBP (with binding truncation) is unchanged; f_s -> f_s X permutes the cosets (I<->X, Y<->Z)
    d, chi, eps = 5, 8, 0.1
    _, s = workload.make_batch(d, eps, 2)
    L = 2 * d - 1
    x, z = lattice.coset_labels(d, s)
    x = x.reshape(-1, L, L)
    z = z.reshape(-1, L, L)
    pi = network.depolarizing(eps)
    plan = blockbp.Plan(d, 4, 4)

    def run(xx, zz):
        t = network.coset_tensors(d, xx, zz, pi)
        msgs, _, _ = blockbp.run_bp(plan, t, chi, 3, 1e-4, 0.1, True)
        return blockbp.bethe(plan, t, msgs, chi)[0]

    base = run(x, z)
    x2, z2 = x.copy(), z.copy()
    for (r, c) in [lattice.checks(d)[5], lattice.checks(d)[-7]]:
        for rr, cc in lattice.neighbours(d, r, c):
            if r % 2 == 0:
                z2[:, rr, cc] ^= 1
            else:
                x2[:, rr, cc] ^= 1
    np.testing.assert_allclose(run(x2, z2), base, rtol=1e-10)
    xm, _ = lattice.logical_masks(d)
    perm = run(x ^ xm, z).reshape(-1, 4)
    np.testing.assert_allclose(perm, base.reshape(-1, 4)[:, [1, 0, 3, 2]], rtol=1e-10)


def test_decision_rule():
    ll = np.array([[-5.0, -3.0, -9.0, -4.0],
                   [-5.0, -3.0, -9.0, -4.0],
                   [-5.0, -3.0, -9.0, -4.0],
                   [-5.0, -5.0, -9.0, -5.0],
                   [np.nan, -3.0, -9.0, -4.0]])
    dl = np.array([[1e-5, 1e-5, 1e-5, 1e-5],       # all trusted: argmax
                   [1e-5, 2e-2, 1e-5, 1e-5],       # X untrusted: best trusted is Z
                   [5e-2, 3e-2, 4e-2, 2e-1],       # none trusted: smallest Delta (X)
                   [1e-5, 1e-5, 1e-5, 1e-5],       # tie: lowest index
                   [1e-5, 1e-5, 1e-5, 1e-5]])      # nan never wins
    np.testing.assert_array_equal(blockbp.decide(ll, dl, 1e-2), [1, 3, 1, 0, 1])
    np.testing.assert_array_equal(blockbp.decide(ll, dl, 1e-2, rule=1), [1, 1, 1, 0, 1])


def test_decode_outputs_consistent():
    d = 5
    e, s = workload.make_batch(d, 0.1, 6)
    r = blockbp.decode(d, 0.1, s, block=(3, 3), chi=4, max_iter=10)
    # the correction carries the syndrome and lies in the decided coset f_s L*
    np.testing.assert_array_equal(workload.syndrome_of(d, r["correction"]), s)
    fx, fz = lattice.pauli_for_syndrome(d, s)
    cx, cz = lattice.pauli_grid_from_codes(d, r["correction"])
    xm, zm = lattice.logical_masks(d)
    for i, k in enumerate(r["coset"]):
        bx, bz = lattice.COSET_BITS[k]
        np.testing.assert_array_equal(cx[i] ^ fx[i], xm * bx)
        np.testing.assert_array_equal(cz[i] ^ fz[i], zm * bz)
    assert r["loglik"].shape == (6, 4) and r["iters"].max() <= 10


def test_blockbp_approaches_exact_as_blocks_grow():
    # d = 5: the estimate error shrinks from 3x3 blocks to a single block (which is exact at chi = 16)
    d = 5
    _, s = workload.make_batch(d, 0.1, 6)
    ex = network.exact_coset_loglik(d, s, 0.1)
    errs = []
    for k in (3, 5, 9):
        r = blockbp.decode(d, 0.1, s, block=(k, k), chi=16, max_iter=20, eta=0.1)
        errs.append(np.abs(r["loglik"] - ex).mean())
    assert errs[2] < 1e-9
    assert errs[1] < errs[0]


def _gated_run(gate, max_iter, fixed=True, d=5, block=3, chi=8, eps=0.1):
    _, s = workload.make_batch(d, eps, 2)
    L = 2 * d - 1
    x, z = lattice.coset_labels(d, s)
    t = network.coset_tensors(d, x.reshape(-1, L, L), z.reshape(-1, L, L), network.depolarizing(eps))
    plan = blockbp.Plan(d, block, block)
    return plan, blockbp.run_bp(plan, t, chi, max_iter, 1e-4, 0.1, fixed, gate)


def test_residual_gate_limits():
    """Residual-gated schedule: a gate below every distance term skips nothing (the run equals the paper's
    schedule); a gate above the largest possible term (8 for unit vectors) lets only the first iteration
    update, so later iterations leave every message unchanged and measure Delta = 0."""
    plan, (m0, d0, i0) = _gated_run(0.0, 4)
    _, (m1, d1, i1) = _gated_run(1e-300, 4)
    for key in m0:
        for a, b in zip(m0[key], m1[key]):
            np.testing.assert_array_equal(a, b)
    np.testing.assert_array_equal(d0, d1)
    _, (ma, da, _) = _gated_run(10.0, 1)
    _, (mb, db, ib) = _gated_run(10.0, 3)
    for key in ma:
        for a, b in zip(ma[key], mb[key]):
            np.testing.assert_allclose(a, b, rtol=0, atol=1e-14)
    assert np.all(db < 1e-6) and np.all(da > 1e-3) and np.all(ib == 3)


def test_residual_gate_keeps_decisions():
    """With a gate of 1e-6 (per-message distance term) the decoder skips the updates of messages that have
    settled together with their inputs: it needs fewer iterations, and its estimates stay within 0.05 nats of
    the paper's schedule with the same decisions (d=7, 4x4 blocks, chi 16)."""
    _, s = workload.make_batch(7, 0.1, 6, workload="test")
    a = blockbp.decode(7, 0.1, s, block=(4, 4), chi=16, max_iter=40)
    b = blockbp.decode(7, 0.1, s, block=(4, 4), chi=16, max_iter=40, gate=1e-6)
    np.testing.assert_array_equal(a["coset"], b["coset"])
    assert np.nanmax(np.abs(a["loglik"] - b["loglik"])) < 0.05
    assert b["iters"].mean() < a["iters"].mean()


def _dense_bp_by_hand(plan, tensors, eta, iters):
    """Two-colour BP written out with dense messages and the dense block contraction above, independent of
    run_bp: every message starts uniform (remark 2); in a round each block of that colour sends to every
    neighbour the contraction of itself with the messages on its other sides, scaled to unit norm
    (remark 3), then mixed as (1 - eta) * new + eta * old and scaled to unit norm again (remark 7); the
    distance of an iteration is (1/M) * sqrt(sum over all M messages of 2 - 2 <new, old>^2) (remark 4).
    Returns (messages, distances)."""
    msgs = {}
    for (src, dst, _) in plan.edges:
        K = plan.msg_len(src, dst)
        msgs[(src, dst)] = np.full(2 ** K, 2.0 ** (-K / 2))
    dists = []
    for _ in range(iters):
        before = dict(msgs)
        for colour in (0, 1):
            fresh = {}
            for (src, dst, dname) in plan.edges:
                if (src[0] + src[1]) % 2 != colour:
                    continue
                dense_in = {}
                for side, (dI, dJ) in blockbp.DIRS.items():
                    nb = (src[0] + dI, src[1] + dJ)
                    dense_in[side] = msgs[(nb, src)] if (side != dname and plan.has(nb)) else None
                new = _block_einsum(tensors, plan, src[0], src[1], dname, dense_in)
                new = new / np.linalg.norm(new)
                mixed = (1.0 - eta) * new + eta * msgs[(src, dst)]
                fresh[(src, dst)] = mixed / np.linalg.norm(mixed)
            msgs.update(fresh)
        acc = sum(2.0 - 2.0 * float(msgs[k] @ before[k]) ** 2 for k in msgs)
        dists.append(np.sqrt(acc) / plan.M)
    return msgs, dists


@pytest.mark.parametrize("iters", [1, 2])
@pytest.mark.parametrize("d,block", [(3, (3, 3)), (5, (4, 2))])
def test_damping_and_distance_by_hand(d, block, iters):
    # remark 7 weights the OLD message by eta, and remark 4 takes the prefactor 1/M outside the square root:
    # with eta = 0.3 (not 1/2, so that eta and 1 - eta differ) and M > 1 swapping either reading changes
    # both the messages and Delta well beyond rounding
    eta = 0.3
    _, s = workload.make_batch(d, 0.1, 1)
    tensors = _coset_tensors(d, s, 0.1)
    plan = blockbp.Plan(d, *block)
    assert plan.M > 4
    for job in (0, 2):
        tj = [[t[job:job + 1] for t in row] for row in tensors]
        want, dists = _dense_bp_by_hand(plan, tj, eta, iters)
        msgs, delta, it = blockbp.run_bp(plan, tj, chi=64, max_iter=iters, delta0=1e-4, eta=eta, fixed_iters=True)
        assert it[0] == iters
        for key, v in want.items():
            got = mps.to_dense(msgs[key])[0].reshape(-1)
            np.testing.assert_allclose(got, v, atol=1e-12)
        np.testing.assert_allclose(delta[0], dists[-1], rtol=1e-10)
        # the readings the pin excludes are far away
        assert abs(dists[-1] * np.sqrt(plan.M) - delta[0]) > 0.1 * delta[0]
