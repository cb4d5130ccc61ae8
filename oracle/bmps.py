"""Boundary-MPS (bMPS) contraction of the coset tensor networks: the single-block limit of blockBP
(oracle; test infrastructure only).

Sec. III.A of the paper recalls the bMPS decoder of Bravyi, Suchara and Vargo: the 2D network is contracted
column by column from left to right; the contraction up to column c is approximated by an MPS over the L
rows whose physical legs are the right legs of column c; column c+1, viewed as an MPO with vertical bonds of
dimension 2, is applied to it (doubling its bonds), and the product is compressed back to bond dimension chi.
Sec. III.D notes that blockBP with a single block covering the whole network is this algorithm, and Sec. IV
uses it with chi = 16 as the accuracy reference. The decoder takes the coset with the largest estimate (the
DQMLD rule of Sec. II.A).

The paper leaves the compression to standard MPS methods. The reading used here, applied after every column
but the last, is `mps.compress`: a QR sweep from the top row to the bottom row (left-canonical form), then a
sweep from the bottom row to the top that keeps the chi largest singular values of every bond (all of them
where there are no more than chi), and the norm split off into a running log-scale. The last column has no
right legs: its MPO is applied and the resulting chain of matrices is multiplied out, so that the estimate
keeps its sign. ln Z = log-scale + ln(value); a value that is not positive gives NaN.

Parity: pinned to the exact contraction (`network.exact_log_contraction`) wherever chi is at least the
largest Schmidt rank 2^floor(L/2), so that no truncation happens; below that the result is an approximation
whose truncated weight is reported beside it.
"""
from __future__ import annotations

import numpy as np

from . import lattice, mps, network


def apply_column(A, T):
    """Apply the MPO of one column to an MPS: A_r [B, Dl, S, Dr] (S = the previous column's right legs),
    T_r [B, du, S, dd, dt] (legs up, left, down, right). The row-r result has left bond (a, u), physical leg
    t and right bond (b, dn), each pair flattened with the MPO index fastest."""
    out = []
    for Ar, Tr in zip(A, T):
        Bn = np.einsum("basc,busdt->bautcd", Ar, Tr)
        b, Dl, du, dt, Dr, dd = Bn.shape
        out.append(Bn.reshape(b, Dl * du, dt, Dr * dd))
    return out


def _discarded_weight(A_before, chi):
    """Relative weight that compressing a left-canonical MPS to chi discards, summed over its bonds.
    Evaluated on a separate copy (the compression itself is mps.compress)."""
    A = mps.left_canonicalize(A_before)
    w = np.zeros(A[0].shape[0])
    for i in range(len(A) - 1, 0, -1):
        X = A[i]
        b, Dl, p, Dr = X.shape
        u, s, vh = np.linalg.svd(X.reshape(b, Dl, p * Dr), full_matrices=False)
        tot = (s ** 2).sum(axis=1)
        k = min(chi, s.shape[1])
        w += np.where(tot > 0, (s[:, k:] ** 2).sum(axis=1) / np.where(tot > 0, tot, 1.0), 0.0)
        A[i] = vh[:, :k, :].reshape(b, k, p, Dr)
        A[i - 1] = np.einsum("bapk,bkj->bapj", A[i - 1], u[:, :, :k] * s[:, None, :k])
    return w


def bmps_log_contraction(d: int, x, z, pi, chi: int, with_truncation: bool = False):
    """ln Tr T_s(L) by boundary-MPS contraction with bond dimension chi, for label grids x, z [..., L, L] and
    the 2x2 single-qubit table pi[x][z]. With with_truncation, also returns the summed relative weight that
    the compressions discarded (0 when the result is exact)."""
    x = np.asarray(x)
    batch = x.shape[:-2]
    L = lattice.side(d)
    B = int(np.prod(batch)) if batch else 1
    xb = x.reshape(B, L, L)
    zb = np.asarray(z).reshape(B, L, L)
    A = [np.ones((B, 1, 1, 1)) for _ in range(L)]
    logs = np.zeros(B)
    trunc = np.zeros(B)
    for c in range(L):
        T = [network.site_tensor(d, r, c, xb[:, r, c], zb[:, r, c], pi) for r in range(L)]
        A = apply_column(A, T)
        if c == L - 1:
            break
        if with_truncation:
            trunc += _discarded_weight(A, chi)
        A, lg = mps.compress(A, chi)
        logs += lg
    v = np.ones((B, 1))
    for r in range(L):
        v = np.einsum("ba,bac->bc", v, A[r][:, :, 0, :])
        s = np.abs(v).max(axis=1)
        v = v / np.where(s > 0, s, 1.0)[:, None]
        logs += np.log(s)
    val = v[:, 0]
    with np.errstate(invalid="ignore", divide="ignore"):
        ll = np.where(val > 0, logs + np.log(np.where(val > 0, val, 1.0)), np.nan)
    ll = ll.reshape(batch)
    return (ll, trunc.reshape(batch)) if with_truncation else ll


def bmps_coset_loglik(d: int, syndrome, pi, chi: int, with_truncation: bool = False):
    """bMPS estimates of ln pi(f_s L G) for L in (I, X, Y, Z): [..., 4] (and the discarded weight)."""
    x, z = lattice.coset_labels(d, syndrome)
    return bmps_log_contraction(d, x, z, pi, chi, with_truncation)


def decide(loglik):
    """DQMLD decision over the four estimates: the largest, NaN counting as -inf, ties to the lowest index."""
    ll = np.where(np.isnan(loglik), -np.inf, loglik)
    return np.argmax(ll, axis=-1)
