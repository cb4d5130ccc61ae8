"""Coset tensor networks T_s(L) and their exact contraction (oracle; test infrastructure only).

Paper, Sec. III.A and Fig. 1: for a syndrome s and a logical L the decoder builds a square tensor network
of (2d-1) x (2d-1) tensors with bond dimension 2 whose contraction equals the coset probability
pi(f_s L G) = sum_{g in G} pi(f_s L g) (eq. for pi of a coset, Sec. II.A). The construction itself is
deferred by the paper to Bravyi-Suchara-Vargo; the reading used here:
  * every check is a COPY tensor: its bond variable says whether the generator is included in g, and all
    of its legs carry that variable (1 when all legs agree, else 0);
  * every qubit tensor is the noise probability of the label f_s L on that qubit, flipped by the checks
    around it: a horizontal edge (even row) has plaquettes (X-checks) above/below and sites (Z-checks)
    left/right, so T(u, l, d, r) = pi(x ^ u ^ d, z ^ l ^ r); a vertical edge (odd row) has the roles
    swapped, T(u, l, d, r) = pi(x ^ l ^ r, z ^ u ^ d);
  * legs are ordered (up, left, down, right); a leg leaving the grid has dimension 1.
Summing over all 2^m check variables enumerates the stabilizer group exactly once, so Tr T_s(L) is the
coset probability.

Noise: a 2x2 table pi[x][z] of single-qubit Pauli probabilities; the paper's depolarizing channel
(Sec. IV) is pi[0][0] = 1 - eps and eps/3 for X, Y, Z.
"""
from __future__ import annotations

import numpy as np

from . import lattice


def depolarizing(eps: float) -> np.ndarray:
    return np.array([[1.0 - eps, eps / 3.0], [eps / 3.0, eps / 3.0]], dtype=np.float64)


def leg_dims(d: int, r: int, c: int):
    L = lattice.side(d)
    return (2 if r > 0 else 1, 2 if c > 0 else 1, 2 if r < L - 1 else 1, 2 if c < L - 1 else 1)


def site_tensor(d: int, r: int, c: int, x: np.ndarray, z: np.ndarray, pi: np.ndarray) -> np.ndarray:
    """Tensor at grid site (r, c) with legs (up, left, down, right), batched over the label arrays
    x, z [...] (ignored at check sites). Returns [..., du, dl, dd, dr]."""
    du, dl, dd, dr = leg_dims(d, r, c)
    x = np.asarray(x)
    batch = x.shape
    u = np.arange(du)[:, None, None, None]
    l = np.arange(dl)[None, :, None, None]
    dn = np.arange(dd)[None, None, :, None]
    rt = np.arange(dr)[None, None, None, :]
    if not lattice.is_qubit(r, c):
        t = np.ones((du, dl, dd, dr))
        # COPY: every present leg equal (absent legs are fixed at 0 and take no part)
        vals = [v for v, dim in ((u, du), (l, dl), (dn, dd), (rt, dr)) if dim == 2]
        for a in vals[1:]:
            t = t * (a == vals[0])
        return np.broadcast_to(t, batch + t.shape).copy()
    if r % 2 == 0:   # horizontal edge: up/down are X-checks (flip x), left/right are Z-checks (flip z)
        px = (u ^ dn)
        pz = (l ^ rt)
    else:            # vertical edge: left/right are X-checks, up/down are Z-checks
        px = (l ^ rt)
        pz = (u ^ dn)
    px = np.broadcast_to(px, (du, dl, dd, dr))
    pz = np.broadcast_to(pz, (du, dl, dd, dr))
    xe = np.asarray(x, dtype=np.int64)[..., None, None, None, None] ^ px
    ze = np.asarray(z, dtype=np.int64)[..., None, None, None, None] ^ pz
    return pi[xe, ze]


def coset_tensors(d: int, x: np.ndarray, z: np.ndarray, pi: np.ndarray):
    """All site tensors of T_s(L) for label grids x, z [..., L, L]: a list of lists [r][c]."""
    L = lattice.side(d)
    return [[site_tensor(d, r, c, x[..., r, c], z[..., r, c], pi) for c in range(L)] for r in range(L)]


def exact_log_contraction(d: int, x: np.ndarray, z: np.ndarray, pi: np.ndarray) -> np.ndarray:
    """ln Tr T_s(L) for label grids [..., L, L], exactly, by sweeping a dense column-transfer vector over the
    L horizontal bonds from the left edge to the right edge (state size 2^L; practical for d <= 9).
    A running log-scale keeps the vector in range."""
    x = np.asarray(x)
    batch = x.shape[:-2]
    L = lattice.side(d)
    B = int(np.prod(batch)) if batch else 1
    xb = x.reshape(B, L, L)
    zb = np.asarray(z).reshape(B, L, L)
    state = np.ones((B, 1))
    hdims = [1] * L
    logs = np.zeros(B)
    for c in range(L):
        pre = 1
        phi = state.reshape(B, 1, 1, -1)
        newdims = []
        for r in range(L):
            T = site_tensor(d, r, c, xb[:, r, c], zb[:, r, c], pi)       # (B, du, dl, dd, dr)
            h = hdims[r]
            post = phi.shape[3] // h
            phi5 = phi.reshape(B, pre, T.shape[1], h, post)
            out = np.einsum("bpvhq,bvhds->bpsdq", phi5, T)
            pre *= T.shape[4]
            newdims.append(T.shape[4])
            phi = out.reshape(B, pre, T.shape[3], post)
        state = phi.reshape(B, -1)
        hdims = newdims
        scale = np.abs(state).max(axis=1)
        state = state / scale[:, None]
        logs += np.log(scale)
    return (logs + np.log(state[:, 0])).reshape(batch)


def exact_coset_loglik(d: int, syndrome: np.ndarray, eps: float) -> np.ndarray:
    """ln pi(f_s L G) for L in (I, X, Y, Z): [..., 4]."""
    x, z = lattice.coset_labels(d, syndrome)
    return exact_log_contraction(d, x, z, depolarizing(eps))
