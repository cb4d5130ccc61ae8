"""Surface-code geometry for the oracle (test infrastructure only).

Paper, Sec. II.B and Fig. 1: a d x d open lattice with d^2 horizontal and (d-1)^2 vertical edges, qubits on
edges (n = d^2 + (d-1)^2), site checks A_u = prod Z on the edges at site u and plaquette checks
B_p = prod X around plaquette p, d(d-1) of each (m = 2d(d-1), one logical qubit). The logical X is X on a
row of horizontal edges and the logical Z is Z on a column of horizontal edges.

Readings where the paper is silent (all drawn on the (2d-1) x (2d-1) grid of the tensor network):
  * horizontal edges at (even r, even c); vertical edges at (odd r, odd c); sites (A_u) at (even r, odd c);
    plaquettes (B_p) at (odd r, even c). Each check touches its in-grid 4-neighbours.
  * syndrome order: Z-checks row-major, then X-checks row-major; qubits row-major.
  * f_s: for every flipped Z-check at (r, c) apply X to the horizontal edges (r, 0), (r, 2), ..., (r, c-1);
    for every flipped X-check at (r, c) apply Z to (0, c), (2, c), ..., (r-1, c).
  * logical representatives: X on row 0 of horizontal edges, Z on column 0 of horizontal edges,
    Y = XZ; coset order (I, X, Y, Z).
Pauli bits are (x, z): I = (0,0), X = (1,0), Z = (0,1), Y = (1,1).
"""
from __future__ import annotations

import numpy as np

COSETS = ("I", "X", "Y", "Z")
# (x-flip of the row-0 logical, z-flip of the column-0 logical) for each coset in COSETS order
COSET_BITS = ((0, 0), (1, 0), (1, 1), (0, 1))


def side(d: int) -> int:
    return 2 * d - 1


def is_qubit(r: int, c: int) -> bool:
    return (r + c) % 2 == 0


def z_checks(d: int):
    L = side(d)
    return [(r, c) for r in range(0, L, 2) for c in range(1, L, 2)]


def x_checks(d: int):
    L = side(d)
    return [(r, c) for r in range(1, L, 2) for c in range(0, L, 2)]


def checks(d: int):
    """All checks in syndrome order (Z-checks then X-checks, each row-major)."""
    return z_checks(d) + x_checks(d)


def qubits(d: int):
    L = side(d)
    return [(r, c) for r in range(L) for c in range(L) if is_qubit(r, c)]


def neighbours(d: int, r: int, c: int):
    L = side(d)
    return [(rr, cc) for rr, cc in ((r - 1, c), (r, c - 1), (r + 1, c), (r, c + 1))
            if 0 <= rr < L and 0 <= cc < L]


def pauli_grid_from_codes(d: int, codes: np.ndarray):
    """Per-qubit codes [..., n] (x + 2z) -> (x, z) bit grids [..., L, L] (zero at check sites)."""
    codes = np.asarray(codes)
    L = side(d)
    x = np.zeros(codes.shape[:-1] + (L, L), dtype=np.uint8)
    z = np.zeros_like(x)
    for i, (r, c) in enumerate(qubits(d)):
        x[..., r, c] = codes[..., i] & 1
        z[..., r, c] = (codes[..., i] >> 1) & 1
    return x, z


def codes_from_pauli_grid(d: int, x: np.ndarray, z: np.ndarray) -> np.ndarray:
    """(x, z) grids [..., L, L] -> per-qubit codes [..., n]."""
    q = qubits(d)
    rr = np.array([r for r, _ in q])
    cc = np.array([c for _, c in q])
    return (x[..., rr, cc] + 2 * z[..., rr, cc]).astype(np.uint8)


def syndrome_of_grid(d: int, x: np.ndarray, z: np.ndarray) -> np.ndarray:
    """Syndrome [..., m] of a Pauli given as bit grids: a Z-check (A_u) anticommutes with the X parts on its
    edges, an X-check (B_p) with the Z parts (Sec. II.A-B)."""
    out = []
    for (r, c) in checks(d):
        src = x if r % 2 == 0 else z
        acc = np.zeros(src.shape[:-2], dtype=np.uint8)
        for (rr, cc) in neighbours(d, r, c):
            acc ^= src[..., rr, cc]
        out.append(acc)
    return np.stack(out, axis=-1)


def pauli_for_syndrome(d: int, syndrome: np.ndarray):
    """f_s of Alg. 1: a Pauli (bit grids [..., L, L]) whose syndrome is `syndrome` [..., m]."""
    syndrome = np.asarray(syndrome, dtype=np.uint8)
    L = side(d)
    x = np.zeros(syndrome.shape[:-1] + (L, L), dtype=np.uint8)
    z = np.zeros_like(x)
    for i, (r, c) in enumerate(checks(d)):
        s = syndrome[..., i]
        if r % 2 == 0:      # Z-check at (r, c): X chain along row r from the left boundary
            for cc in range(0, c, 2):
                x[..., r, cc] ^= s
        else:               # X-check at (r, c): Z chain along column c from the top boundary
            for rr in range(0, r, 2):
                z[..., rr, c] ^= s
    return x, z


def logical_masks(d: int):
    """(x-mask of logical X, z-mask of logical Z) as [L, L] bit grids."""
    L = side(d)
    xm = np.zeros((L, L), dtype=np.uint8)
    zm = np.zeros((L, L), dtype=np.uint8)
    xm[0, 0::2] = 1
    zm[0::2, 0] = 1
    return xm, zm


def coset_labels(d: int, syndrome: np.ndarray):
    """Labels f_s * L for L in (I, X, Y, Z): bit grids [..., 4, L, L] (Alg. 1, coset loop)."""
    fx, fz = pauli_for_syndrome(d, syndrome)
    xm, zm = logical_masks(d)
    xs, zs = [], []
    for bx, bz in COSET_BITS:
        xs.append(fx ^ (xm * bx))
        zs.append(fz ^ (zm * bz))
    return np.stack(xs, axis=-3), np.stack(zs, axis=-3)


def commutes(x1, z1, x2, z2) -> np.ndarray:
    """1 where two Paulis (bit grids) commute (even symplectic product), else 0."""
    s = (x1 & z2) ^ (z1 & x2)
    return 1 - (np.bitwise_xor.reduce(s.reshape(s.shape[:-2] + (-1,)), axis=-1) & 1)
