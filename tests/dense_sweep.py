"""A second, dense formulation of one blockBP message update, written independently of the oracle's MPS
code (test helper; not collected by pytest).

The boundary state of the in-block sweep is held as one dense array psi[top cap][h_0 .. h_{k-1}][bottom cap]
instead of an MPS. Two readings of the side messages' legs are offered:
  * caps="open": a K-site message m(v_0..v_{K-1}) is read as the product-of-identities MPS whose bond j
    carries the legs v_0..v_{j-1} for j <= K//2 and the legs v_j..v_{K-1} above that, with the whole vector
    sitting on site K//2 (small caps; exact contractions only, i.e. while chi truncates nothing);
  * caps="remaining": the cap index is the tuple of the message legs not yet absorbed, and the whole
    message is applied when its first leg is absorbed. The part of the cap still to be absorbed is then
    the identity -- an isometry -- so this is the gauge-free form of a cap whose remaining sites are
    canonical, and the truncations below act in the metric of the rest of the cap.
Truncation is applied cut by cut from the bottom end as best rank-chi approximations of the dense state
(what the MPS compression computes).
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


def remaining_cap_operator(msg, K, js, forward):
    """caps="remaining": [old cap, emitted leg, new cap] with the cap index the legs still to be absorbed
    (first leg most significant); the message itself is applied at the first absorbed site."""
    m = np.asarray(msg, dtype=np.float64)
    if forward:
        if js == 0:                                   # () -> (v_1..v_{K-1})
            return m.reshape(1, 2, 2 ** (K - 1))
        r = 2 ** (K - js - 1)                         # (v_js..) -> (v_{js+1}..)
        op = np.zeros((2 * r, 2, r))
        for v in range(2):
            for b in range(r):
                op[v * r + b, v, b] = 1
        return op
    if js == K - 1:                                   # () -> (v_0..v_{K-2})
        return np.transpose(m.reshape(2 ** (K - 1), 2, 1), (2, 1, 0))
    r = 2 ** js                                       # (v_0..v_js) -> (v_0..v_{js-1})
    op = np.zeros((2 * r, 2, r))
    for a in range(r):
        for v in range(2):
            op[2 * a + v, v, a] = 1
    return op


def cap_operator(msg, K, js, forward, caps="open"):
    """Operator [old cap, emitted leg, new cap] for absorbing site js of a K-site side message."""
    if msg is None:
        op = np.zeros((1, 2, 1))
        op[0, 0, 0] = 1.0
        return op
    if caps == "remaining":
        return remaining_cap_operator(msg, K, js, forward)
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


def dense_update(block, frame, init, top, bottom, chi, caps="open"):
    """One BP message update of a block (its tensors block[r][c], legs (up, left, down, right)) toward side
    `frame`, with incoming dense messages (None where the neighbour is absent), the side messages read as
    `caps` says (module docstring). Returns (outgoing dense message, natural log of the split-off scale)."""
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
        psi = np.einsum("n...,nvq->qv...", psi, cap_operator(top, kt, js, forward, caps))   # [n', v, h.., s]
        for i in range(kp):
            F = frame_tensor(block, frame, t, i)
            src = "nv" + "".join(hl) + "s"
            dst = "nw" + "".join("o" if j == i else hl[j] for j in range(kp)) + "s"
            psi = np.einsum(f"{src},v{hl[i]}wo->{dst}", psi, F)
        psi = np.moveaxis(psi, 1, -2)                                               # [n', h', v, s]
        psi = np.einsum("...vs,svq->...q", psi, cap_operator(bottom, kt, js, forward, caps))
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
