"""Matrix-product-state tools for the oracle (test infrastructure only).

An MPS is a list of site tensors of shape [..., D_left, p, D_right] (end bonds of dimension 1) with an
arbitrary leading batch. These are the textbook operations the boundary-MPS method relies on
(Sec. III.A of the paper; the compression "truncates the bond dimension back to chi using well-established
MPS methods"):
  * left_canonicalize: QR sweep from the first site to the last; right_canonicalize the mirror image;
  * compress: left-canonicalize, then sweep back from the last site keeping, at every bond, the
    min(chi, available) largest singular values (a full SVD where truncation can act, an LQ step where the
    bond cannot exceed chi); the norm is split off as a log-scale;
  * overlap, direct_sum, to_dense, and padding to the static bond dimensions used for messages.
"""
from __future__ import annotations

import numpy as np


def to_dense(sites):
    """Contract an MPS into its dense vector [..., p0 * p1 * ...] (first physical leg most significant)."""
    acc = sites[0]
    acc = acc.reshape(acc.shape[:-3] + (acc.shape[-2], acc.shape[-1]))      # [..., P, D]
    for s in sites[1:]:
        acc = np.einsum("...PD,...Dpe->...Ppe", acc, s)
        acc = acc.reshape(acc.shape[:-3] + (acc.shape[-3] * acc.shape[-2], acc.shape[-1]))
    return acc[..., 0]


def from_dense(vec, dims):
    """Exact MPS of a dense vector [..., prod(dims)] with natural bonds (successive QR, no truncation)."""
    vec = np.asarray(vec, dtype=np.float64)
    batch = vec.shape[:-1]
    sites = []
    rest = vec.reshape(batch + (1, -1))
    for i, p in enumerate(dims[:-1]):
        Dl = rest.shape[-2]
        mat = rest.reshape(batch + (Dl * p, -1))
        q, r = np.linalg.qr(mat)
        sites.append(q.reshape(batch + (Dl, p, q.shape[-1])))
        rest = r
    sites.append(rest.reshape(batch + (rest.shape[-2], dims[-1], 1)))
    return sites


def left_canonicalize(sites):
    """QR sweep first -> last; every site but the last becomes an isometry (left-canonical)."""
    sites = list(sites)
    for i in range(len(sites) - 1):
        A = sites[i]
        b = A.shape[:-3]
        Dl, p, Dr = A.shape[-3:]
        q, r = np.linalg.qr(A.reshape(b + (Dl * p, Dr)))
        sites[i] = q.reshape(b + (Dl, p, q.shape[-1]))
        sites[i + 1] = np.einsum("...kd,...dpe->...kpe", r, sites[i + 1])
    return sites


def right_canonicalize(sites):
    """LQ sweep last -> first; every site but the first becomes a co-isometry (right-canonical) and the
    first carries the whole weight."""
    sites = list(sites)
    for i in range(len(sites) - 1, 0, -1):
        A = sites[i]
        b = A.shape[:-3]
        Dl, p, Dr = A.shape[-3:]
        q, r = np.linalg.qr(np.swapaxes(A.reshape(b + (Dl, p * Dr)), -1, -2))   # A = r^T q^T
        sites[i] = np.swapaxes(q, -1, -2).reshape(b + (q.shape[-1], p, Dr))
        sites[i - 1] = np.einsum("...apk,...jk->...apj", sites[i - 1], r)
    return sites


def compress(sites, chi: int):
    """Boundary-MPS compression to bond dimension chi: left-canonical QR sweep, then a sweep from the last
    site to the first that keeps min(chi, available) singular values at every bond.
    Returns (sites, log_norm): the returned MPS has unit norm and is right-canonical from site 1 on."""
    sites = left_canonicalize(sites)
    for i in range(len(sites) - 1, 0, -1):
        A = sites[i]
        b = A.shape[:-3]
        Dl, p, Dr = A.shape[-3:]
        mat = A.reshape(b + (Dl, p * Dr))
        if min(Dl, p * Dr) > chi:
            u, s, vh = np.linalg.svd(mat, full_matrices=False)
            u, s, vh = u[..., :, :chi], s[..., :chi], vh[..., :chi, :]
            sites[i] = vh.reshape(b + (chi, p, Dr))
            sites[i - 1] = np.einsum("...apk,...kj->...apj", sites[i - 1], u * s[..., None, :])
        else:
            q, r = np.linalg.qr(np.swapaxes(mat, -1, -2))          # mat = r^T q^T
            K = q.shape[-1]
            sites[i] = np.swapaxes(q, -1, -2).reshape(b + (K, p, Dr))
            sites[i - 1] = np.einsum("...apk,...jk->...apj", sites[i - 1], r)
    nrm = np.sqrt(np.sum(sites[0] ** 2, axis=(-3, -2, -1)))
    sites[0] = sites[0] / nrm[..., None, None, None]
    return sites, np.log(nrm)


def overlap(a, b):
    """<a, b> for real MPSs with equal physical dimensions."""
    E = np.ones(a[0].shape[:-3] + (1, 1))
    for x, y in zip(a, b):
        E = np.einsum("...ab,...apc,...bpd->...cd", E, x, y)
    return E[..., 0, 0]


def norm(a):
    return np.sqrt(overlap(a, a))


def direct_sum(a, b, ca, cb):
    """MPS of ca*a + cb*b (bond dimensions add)."""
    n = len(a)
    out = []
    for i, (x, y) in enumerate(zip(a, b)):
        bt = np.broadcast_shapes(x.shape[:-3], y.shape[:-3])
        x = np.broadcast_to(x, bt + x.shape[-3:])
        y = np.broadcast_to(y, bt + y.shape[-3:])
        if i == 0:
            x = x * np.asarray(ca)[..., None, None, None]
            y = y * np.asarray(cb)[..., None, None, None]
        if n == 1:
            out.append(x + y)
        elif i == 0:
            out.append(np.concatenate([x, y], axis=-1))
        elif i == n - 1:
            out.append(np.concatenate([x, y], axis=-3))
        else:
            Dla, p, Dra = x.shape[-3:]
            Dlb, _, Drb = y.shape[-3:]
            z = np.zeros(bt + (Dla + Dlb, p, Dra + Drb))
            z[..., :Dla, :, :Dra] = x
            z[..., Dla:, :, Dra:] = y
            out.append(z)
    return out


def natural_bonds(phys, chi: int):
    """Static bond dimensions of a message MPS: min(chi, product of legs on the left, on the right)."""
    n = len(phys)
    out = []
    for j in range(n + 1):
        left = int(np.prod(phys[:j])) if j else 1
        right = int(np.prod(phys[j:])) if j < n else 1
        out.append(min(chi, left, right))
    return out


def pad_bonds(sites, bonds):
    """Zero-pad (or keep) every bond to the given dimensions; bonds larger than requested are an error."""
    out = []
    for i, A in enumerate(sites):
        Dl, p, Dr = A.shape[-3:]
        tl, tr = bonds[i], bonds[i + 1]
        if Dl > tl or Dr > tr:
            raise ValueError("pad_bonds: bond larger than target")
        z = np.zeros(A.shape[:-3] + (tl, p, tr))
        z[..., :Dl, :, :Dr] = A
        out.append(z)
    return out


def uniform(phys, chi: int, batch=()):
    """The uniform product message (every site (1, 1)/sqrt(2) for p = 2), held at the static bond
    dimensions and left-canonical."""
    sites = [np.broadcast_to(np.full((1, p, 1), 1.0 / np.sqrt(p)), batch + (1, p, 1)).copy() for p in phys]
    return left_canonicalize(pad_bonds(sites, natural_bonds(phys, chi)))


def canonical_message(sites, chi: int):
    """Remark 3 of Alg. 1: make a message left-canonical with unit L2 norm. The message is first compressed
    to chi, then held at the static bond dimensions min(chi, 2^j, 2^(K-j)) (zero-padded where its
    Schmidt rank is lower) so that its canonical bond spaces do not depend on the rank.
    Returns (sites, log_norm)."""
    phys = [A.shape[-2] for A in sites]
    sites, lognorm = compress(sites, chi)
    sites = left_canonicalize(pad_bonds(sites, natural_bonds(phys, chi)))
    nrm = np.sqrt(np.sum(sites[-1] ** 2, axis=(-3, -2, -1)))
    sites[-1] = sites[-1] / nrm[..., None, None, None]
    return sites, lognorm + np.log(nrm)
