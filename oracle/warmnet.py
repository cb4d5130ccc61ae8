"""FP64 oracle of the learned warm start (test infrastructure only: tests/, the smoke check and the
benchmark's CPU baseline import it; the decoder never does).

The network predicts, from the syndrome, the initial messages of blockBP (the uniform start of Alg. 1,
remark 2, is what it replaces; the paper names machine learning as a way to improve BP in Sec. V). Plain
NumPy, generic channel counts so that tests can use tiny networks; every step is written out directly (no
blocking or fusion).

Input, per coset job, a (2d-1) x (2d-1) grid with 11 channels per site:
  0 x bit and 1 z bit of the coset label f_s L at qubit sites (0 at checks),
  2 syndrome bit at check sites (0 at qubits),
  3 qubit, 4 Z-check (even row, odd column), 5 X-check (odd row, even column) indicators,
  6 the noise rate p, 7 constant 1 (marks the inside of the grid against the zero padding),
  8, 9 the coset's x and z bits (1 for X and Y, 1 for Y and Z),
  10 at check sites the generator bit G: for a plaquette (X-check) at (r, c) the parity of the x bits of
     f_s L on the horizontal edges above it in column c, for a vertex (Z-check) at (r, c) the parity of
     the z bits of f_s L on the horizontal edges left of it in row r (the generators that clear f_s L from
     the horizontal edges except the last row / column).
No absolute position enters, so the network applies unchanged to distances it was not trained on.
Three 3x3 convolutions with zero padding, ReLU after the first two, give features F [L, L, C3].

Message head, per directed message u -> v with K legs (the crossing bonds of the boundary, position 0 at
the top / left): leg i joins site a_i in u to site b_i in v. With f_i = [F[a_i], F[b_i]] and the
direction's weights,
  unary     u_i = Wu^T f_i + bu                      (2 values: leg value 0 / 1)
  pairwise  P_i = Wp^T [f_i, f_{i+1}] + bp          (4 values, index 2 b_i + b_{i+1})
  s(b) = sum_i u_i[b_i] + sum_i P_i[b_i, b_{i+1}],  m(b) = exp(s(b)) / ||exp(s)||_2
over the 2^K leg configurations b (dense index with leg 0 most significant, as the messages of the
decoder). Loss of a message against its converged target t (non-negative): KL(q || p) with q = t / sum(t)
and p = softmax(s) (invariant to the scale of t; zero when t is proportional to the prediction); the
training loss is the mean over messages.

Parameter vector (FP32 on the GPU, float64 here), in this order:
  conv1 W [9*C0][C1] (row (dy*3 + dx)*C0 + ci), b [C1]; conv2 W [9*C1][C2], b [C2]; conv3 W [9*C2][C3], b [C3];
  for each direction E, W, S, N: Wu [2*C3][2], bu [2], Wp [4*C3][4], bp [4].
"""
from __future__ import annotations

import numpy as np

C0 = 11
CHANNELS = (64, 128, 96)   # C1, C2, C3 of the network the GPU trains


def sizes(ch=CHANNELS):
    c1, c2, c3 = ch
    return [("conv1.W", (9 * C0, c1)), ("conv1.b", (c1,)), ("conv2.W", (9 * c1, c2)), ("conv2.b", (c2,)),
            ("conv3.W", (9 * c2, c3)), ("conv3.b", (c3,))] + [
        (f"head{k}.{n}", s) for k in range(4)
        for n, s in (("Wu", (2 * c3, 2)), ("bu", (2,)), ("Wp", (4 * c3, 4)), ("bp", (4,)))]


def count(ch=CHANNELS):
    return int(sum(np.prod(s) for _, s in sizes(ch)))


def unpack(theta, ch=CHANNELS):
    out, o = {}, 0
    for n, s in sizes(ch):
        k = int(np.prod(s))
        out[n] = np.asarray(theta[o:o + k], dtype=np.float64).reshape(s)
        o += k
    assert o == len(theta)
    return out


def pack(parts, ch=CHANNELS):
    return np.concatenate([np.asarray(parts[n], dtype=np.float64).ravel() for n, _ in sizes(ch)])


def features(d, syndrome, p, coset):
    """Input grid [L, L, 11] of coset job `coset` (0..3 = I, X, Y, Z) of a syndrome [m] (0/1)."""
    from . import lattice
    L = 2 * d - 1
    nz = d * (d - 1)
    xs, zs = lattice.coset_labels(d, np.asarray(syndrome))
    lx, lz = np.asarray(xs[coset], dtype=np.int64), np.asarray(zs[coset], dtype=np.int64)
    bx, bz = lattice.COSET_BITS[coset]
    X = np.zeros((L, L, C0))
    for r in range(L):
        for c in range(L):
            if (r + c) % 2 == 0:
                X[r, c, 0] = lx[r, c]
                X[r, c, 1] = lz[r, c]
                X[r, c, 3] = 1.0
            elif r % 2 == 0:          # Z-check (vertex)
                X[r, c, 2] = syndrome[(r // 2) * (d - 1) + (c - 1) // 2]
                X[r, c, 4] = 1.0
                X[r, c, 10] = sum(lz[r, cc] for cc in range(0, c, 2)) % 2
            else:                     # X-check (plaquette)
                X[r, c, 2] = syndrome[nz + ((r - 1) // 2) * d + c // 2]
                X[r, c, 5] = 1.0
                X[r, c, 10] = sum(lx[rr, c] for rr in range(0, r, 2)) % 2
            X[r, c, 6] = p
            X[r, c, 7] = 1.0
            X[r, c, 8] = bx
            X[r, c, 9] = bz
    return X


def job_labels(d, syndrome):
    """Coset label grids [4, L, L] (bit 0 x, bit 1 z of f_s L for L = I, X, Y, Z) of one syndrome."""
    from . import lattice
    xs, zs = lattice.coset_labels(d, np.asarray(syndrome))
    return (np.asarray(xs, dtype=np.int64) | (np.asarray(zs, dtype=np.int64) << 1))


def im2col(X):
    """[L, L, C] -> [L*L, 9*C], column (dy*3 + dx)*C + c holds X[r + dy - 1, c + dx - 1] (0 outside)."""
    L, _, C = X.shape
    P = np.zeros((L + 2, L + 2, C))
    P[1:-1, 1:-1] = X
    cols = np.zeros((L, L, 9, C))
    for dy in range(3):
        for dx in range(3):
            cols[:, :, dy * 3 + dx] = P[dy:dy + L, dx:dx + L]
    return cols.reshape(L * L, 9 * C)


def col2im(G, L, C):
    """Adjoint of im2col: [L*L, 9*C] -> [L, L, C]."""
    G = G.reshape(L, L, 9, C)
    P = np.zeros((L + 2, L + 2, C))
    for dy in range(3):
        for dx in range(3):
            P[dy:dy + L, dx:dx + L] += G[:, :, dy * 3 + dx]
    return P[1:-1, 1:-1]


def conv(X, W, b):
    L = X.shape[0]
    return (im2col(X) @ W + b).reshape(L, L, -1)


def trunk(prm, X0, store=None):
    """Forward of the three convolutions; returns the features and the intermediates for backward.
    store: optional rounding applied where the inference variant stores values in a narrower format (the
    input channels and the two hidden activations); None = exact."""
    keep = (lambda a: a) if store is None else store
    X0 = keep(X0)
    Z1 = conv(X0, prm["conv1.W"], prm["conv1.b"])
    A1 = keep(np.maximum(Z1, 0.0))
    Z2 = conv(A1, prm["conv2.W"], prm["conv2.b"])
    A2 = keep(np.maximum(Z2, 0.0))
    F = conv(A2, prm["conv3.W"], prm["conv3.b"])
    return F, (X0, Z1, A1, Z2, A2)


def round_bf16(x):
    """Round to BF16 (8 significant bits, nearest even) through the float32 bit pattern; the BF16
    inference variant stores its input channels, hidden activations and convolution weights this way."""
    f = np.asarray(x, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    u = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


DIRECTIONS = {"E": 0, "W": 1, "S": 2, "N": 3}


def direction_of(plan, e):
    return DIRECTIONS[plan.edges[e][2]]


def legs(d, plan, e):
    """Sites (a_i, b_i) of the legs of directed message e: a in the sending block, b across the boundary."""
    (I, J), _, name = plan.edges[e]
    r0, kr = plan.rows[I]
    c0, kc = plan.cols[J]
    if name == "E":
        return [((r0 + i, c0 + kc - 1), (r0 + i, c0 + kc)) for i in range(kr)]
    if name == "W":
        return [((r0 + i, c0), (r0 + i, c0 - 1)) for i in range(kr)]
    if name == "S":
        return [((r0 + kr - 1, c0 + i), (r0 + kr, c0 + i)) for i in range(kc)]
    return [((r0, c0 + i), (r0 - 1, c0 + i)) for i in range(kc)]   # N


def head_message(prm, F, lg, direction):
    """Dense unit message (2^K entries, leg 0 most significant) of one directed message."""
    s, _ = _head_scores(prm, F, lg, direction)
    m = np.exp(s - s.max())
    return m / np.linalg.norm(m)


def _head_scores(prm, F, lg, direction):
    K = len(lg)
    Wu, bu = prm[f"head{direction}.Wu"], prm[f"head{direction}.bu"]
    Wp, bp = prm[f"head{direction}.Wp"], prm[f"head{direction}.bp"]
    f = [np.concatenate([F[a], F[b]]) for a, b in lg]
    u = [f[i] @ Wu + bu for i in range(K)]
    P = [np.concatenate([f[i], f[i + 1]]) @ Wp + bp for i in range(K - 1)]
    s = np.zeros(2 ** K)
    for idx in range(2 ** K):
        bits = [(idx >> (K - 1 - i)) & 1 for i in range(K)]
        s[idx] = sum(u[i][bits[i]] for i in range(K)) + sum(P[i][2 * bits[i] + bits[i + 1]] for i in range(K - 1))
    return s, (f, u, P)


def loss_and_grad(theta, X0, d, plan, targets, msg_ids, ch=CHANNELS):
    """Mean over msg_ids of KL(q_e || softmax(s_e)), q_e = t_e / sum(t_e), for one coset job, and its
    gradient with respect to theta. targets: [M, 64] non-negative messages (entries beyond 2^K ignored)."""
    prm = unpack(theta, ch)
    F, (X0_, Z1, A1, Z2, A2) = trunk(prm, X0)
    L = F.shape[0]
    grads = {n: np.zeros(s) for n, s in sizes(ch)}
    dF = np.zeros_like(F)
    total = 0.0
    for e in msg_ids:
        direction = direction_of(plan, e)
        lg = legs(d, plan, e)
        K = len(lg)
        s, (f, u, P) = _head_scores(prm, F, lg, direction)
        logp = s - s.max() - np.log(np.exp(s - s.max()).sum())
        q = np.maximum(targets[e, :2 ** K], 0.0)
        q = q / q.sum()
        nzq = q > 0
        total += float((q[nzq] * (np.log(q[nzq]) - logp[nzq])).sum())
        # d KL / d s = softmax(s) - q
        g_s = np.exp(logp) - q
        gu = [np.zeros(2) for _ in range(K)]
        gP = [np.zeros(4) for _ in range(K - 1)]
        for idx in range(2 ** K):
            bits = [(idx >> (K - 1 - i)) & 1 for i in range(K)]
            for i in range(K):
                gu[i][bits[i]] += g_s[idx]
            for i in range(K - 1):
                gP[i][2 * bits[i] + bits[i + 1]] += g_s[idx]
        Wu, Wp = prm[f"head{direction}.Wu"], prm[f"head{direction}.Wp"]
        gf = [np.zeros_like(f[0]) for _ in range(K)]
        for i in range(K):
            grads[f"head{direction}.Wu"] += np.outer(f[i], gu[i])
            grads[f"head{direction}.bu"] += gu[i]
            gf[i] += Wu @ gu[i]
        for i in range(K - 1):
            g = np.concatenate([f[i], f[i + 1]])
            grads[f"head{direction}.Wp"] += np.outer(g, gP[i])
            grads[f"head{direction}.bp"] += gP[i]
            gg = Wp @ gP[i]
            gf[i] += gg[:len(f[i])]
            gf[i + 1] += gg[len(f[i]):]
        C3 = F.shape[2]
        for i, (a, b) in enumerate(lg):
            dF[a] += gf[i][:C3]
            dF[b] += gf[i][C3:]
    n = max(len(msg_ids), 1)
    for k in grads:
        grads[k] /= n
    dF /= n
    # backward through the convolutions
    def conv_back(Xin, W, dY):
        cols = im2col(Xin)
        dYm = dY.reshape(L * L, -1)
        return cols.T @ dYm, dYm.sum(axis=0), col2im(dYm @ W.T, L, Xin.shape[2])
    gW3, gb3, dA2 = conv_back(A2, prm["conv3.W"], dF)
    dZ2 = dA2 * (Z2 > 0)
    gW2, gb2, dA1 = conv_back(A1, prm["conv2.W"], dZ2)
    dZ1 = dA1 * (Z1 > 0)
    gW1, gb1, _ = conv_back(X0_, prm["conv1.W"], dZ1)
    grads.update({"conv1.W": gW1, "conv1.b": gb1, "conv2.W": gW2, "conv2.b": gb2, "conv3.W": gW3, "conv3.b": gb3})
    return total / n, pack(grads, ch)


def predict_stored(theta, X0, d, plan, store, ch=CHANNELS):
    """Dense initial messages [M, 64] of one coset job in the arithmetic of the inference variant: the input
    channels, both hidden activations and the first two convolutions' weights go through `store` (the
    narrower storage format); the last convolution is composed with the head, i.e. for each direction the
    features are projected on the six 96-row blocks of the head's weights that a site contributes as a_i,
    b_i, a_{i+1} or b_{i+1} of a message (Wu's two halves, Wp's four quarters), the composed weights W3 Hc also
    going through `store`; every sum is exact. With store = identity this equals predict()."""
    prm = unpack(theta, ch)
    X0 = store(X0)
    A1 = store(np.maximum(conv(X0, store(prm["conv1.W"]), prm["conv1.b"]), 0.0))
    A2 = store(np.maximum(conv(A1, store(prm["conv2.W"]), prm["conv2.b"]), 0.0))
    C3 = ch[2]
    proj = {}
    for name, k in DIRECTIONS.items():
        Wu, Wp = prm[f"head{k}.Wu"], prm[f"head{k}.Wp"]
        Hc = np.concatenate([Wu[:C3], Wu[C3:], Wp[:C3], Wp[C3:2 * C3], Wp[2 * C3:3 * C3], Wp[3 * C3:]], axis=1)
        proj[k] = conv(A2, store(prm["conv3.W"] @ Hc), prm["conv3.b"] @ Hc)      # [L, L, 20]
    out = np.zeros((plan.M, 64))
    for e in range(plan.M):
        lg = legs(d, plan, e)
        k = direction_of(plan, e)
        P, K = proj[k], len(lg)
        bu, bp = prm[f"head{k}.bu"], prm[f"head{k}.bp"]
        u = [P[a][0:2] + P[b][2:4] + bu for a, b in lg]
        pair = [P[lg[i][0]][4:8] + P[lg[i][1]][8:12] + P[lg[i + 1][0]][12:16] + P[lg[i + 1][1]][16:20] + bp
                for i in range(K - 1)]
        sc = np.zeros(2 ** K)
        for idx in range(2 ** K):
            bits = [(idx >> (K - 1 - i)) & 1 for i in range(K)]
            sc[idx] = sum(u[i][bits[i]] for i in range(K)) + sum(pair[i][2 * bits[i] + bits[i + 1]]
                                                                 for i in range(K - 1))
        m = np.exp(sc - sc.max())
        out[e, :2 ** K] = m / np.linalg.norm(m)
    return out


def predict(theta, X0, d, plan, ch=CHANNELS, store=None):
    """Dense initial messages [M, 64] of one coset job (store: see trunk)."""
    prm = unpack(theta, ch)
    F, _ = trunk(prm, X0, store)
    out = np.zeros((plan.M, 64))
    for e in range(plan.M):
        lg = legs(d, plan, e)
        out[e, :2 ** len(lg)] = head_message(prm, F, lg, direction_of(plan, e))
    return out
