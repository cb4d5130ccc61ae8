"""A second, dense formulation of one blockBP message update, written independently of the oracle's MPS
code (test helper; not collected by pytest).

The boundary state of the in-block sweep is held as one dense array psi[top cap][h_0 .. h_{k-1}][bottom cap]
instead of an MPS. The side messages enter through their own legs: a K-site message m(v_0..v_{K-1}) is
read as the product-of-identities MPS whose bond j carries the legs v_0..v_{j-1} for j <= K//2 and the legs
v_j..v_{K-1} above that, with the whole vector sitting on site K//2. For j <= K/2 this bond basis is related
to the left-canonical one by an orthogonal map, so truncations that act while both caps sit at such bonds
give the same state as the canonical MPS algorithm. Truncation is applied cut by cut from the bottom end
as best rank-chi approximations of the dense state (what the MPS compression computes).
"""
import numpy as np

PERM = {"E": (0, 1, 2, 3), "W": (0, 3, 2, 1), "S": (1, 0, 3, 2), "N": (1, 2, 3, 0)}


def frame_tensor(block, frame, t, i):
    """block[r][c] has legs (up, left, down, right); returns the (up, in, down, out) tensor, zero-padded to
    dimension 2 on every leg."""
    kr, kc = len(block), len(block[0])
    if frame == "E":
        T = block[i][t]
    elif frame == "W":
        T = block[i][kc - 1 - t]
    elif frame == "S":
        T = block[t][i]
    else:
        T = block[kr - 1 - t][i]
    T = np.transpose(T, PERM[frame])
    out = np.zeros((2, 2, 2, 2))
    out[:T.shape[0], :T.shape[1], :T.shape[2], :T.shape[3]] = T
    return out


def canonical_sites(msg, K):
    """Left-canonical MPS of a dense K-site message with bonds min(2^j, 2^(K-j)) (successive QR)."""
    sites = []
    rest = np.asarray(msg, dtype=np.float64).reshape(1, -1)
    for j in range(K - 1):
        b = rest.shape[0]
        q, r = np.linalg.qr(rest.reshape(2 * b, -1))
        sites.append(q.reshape(b, 2, q.shape[1]))
        rest = r
    sites.append(rest.reshape(rest.shape[0], 2, 1))
    return sites


def cap_operator(msg, K, js, forward, canonical=False):
    """Operator [old cap, emitted leg, new cap] for absorbing site js of a K-site side message."""
    if msg is None:
        op = np.zeros((1, 2, 1))
        op[0, 0, 0] = 1.0
        return op
    if canonical:
        A = canonical_sites(msg, K)[js]
        return A if forward else np.transpose(A, (2, 1, 0))
    D = K // 2
    m = np.asarray(msg, dtype=np.float64).reshape(2 ** D, 2, 2 ** (K - D - 1))
    if forward:
        if js < D:       # (v_0..v_{js-1}) -> (v_0..v_js)
            op = np.zeros((2 ** js, 2, 2 ** (js + 1)))
            for a in range(2 ** js):
                for v in range(2):
                    op[a, v, 2 * a + v] = 1
        elif js == D:    # (v_0..v_{D-1}) -> (v_{D+1}..v_{K-1}), weighted by the message
            op = m
        else:            # (v_js..) -> (v_{js+1}..)
            r = 2 ** (K - js - 1)
            op = np.zeros((2 * r, 2, r))
            for v in range(2):
                for b in range(r):
                    op[v * r + b, v, b] = 1
    else:
        if js > D:       # (v_{js+1}..) -> (v_js..)
            r = 2 ** (K - js - 1)
            op = np.zeros((r, 2, 2 * r))
            for v in range(2):
                for b in range(r):
                    op[b, v, v * r + b] = 1
        elif js == D:    # (v_{D+1}..) -> (v_0..v_{D-1}), weighted by the message
            op = np.transpose(m, (2, 1, 0))
        else:            # (v_0..v_js) -> (v_0..v_{js-1})
            op = np.zeros((2 ** (js + 1), 2, 2 ** js))
            for a in range(2 ** js):
                for v in range(2):
                    op[2 * a + v, v, a] = 1
    return op


def dense_update(block, frame, init, top, bottom, chi, canonical=False):
    """One BP message update of a block (its tensors block[r][c], legs (up, left, down, right)) toward side
    `frame`, with incoming dense messages (None where the neighbour is absent). With canonical=True the side
    messages enter through their left-canonical MPS sites (valid for any chi); otherwise through the
    open-leg reading above (valid while no truncation acts with a cap past the middle bond).
    Returns (outgoing dense message, natural log of the split-off scale)."""
    kr, kc = len(block), len(block[0])
    kt, kp = (kc, kr) if frame in "EW" else (kr, kc)
    forward = frame in "ES"
    hl = [chr(ord("a") + j) for j in range(kp)]
    psi = np.zeros((1,) + (2,) * kp + (1,))
    if init is None:
        psi[(0,) * (kp + 2)] = 1.0
    else:
        psi[0, ..., 0] = np.asarray(init, dtype=np.float64).reshape((2,) * kp)
    logscale = 0.0
    for t in range(kt):
        js = t if forward else kt - 1 - t
        psi = np.einsum("n...,nvq->qv...", psi, cap_operator(top, kt, js, forward, canonical))   # [n', v, h.., s]
        for i in range(kp):
            F = frame_tensor(block, frame, t, i)
            src = "nv" + "".join(hl) + "s"
            dst = "nw" + "".join("o" if j == i else hl[j] for j in range(kp)) + "s"
            psi = np.einsum(f"{src},v{hl[i]}wo->{dst}", psi, F)
        psi = np.moveaxis(psi, 1, -2)                                               # [n', h', v, s]
        psi = np.einsum("...vs,svq->...q", psi, cap_operator(bottom, kt, js, forward, canonical))
        shape = psi.shape
        for cut in range(kp + 1, 0, -1):
            mat = psi.reshape(int(np.prod(shape[:cut])), -1)
            u, s, vh = np.linalg.svd(mat, full_matrices=False)
            k = min(chi, s.size)
            psi = ((u[:, :k] * s[:k]) @ vh[:k]).reshape(shape)
        nrm = np.linalg.norm(psi)
        psi = psi / nrm
        logscale += np.log(nrm)
    return psi.reshape(-1), logscale
