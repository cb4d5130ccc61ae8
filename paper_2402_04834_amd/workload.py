"""Seeded synthetic workloads: i.i.d. depolarizing errors on the planar surface code and their syndromes.

This module is the only code shared by the GPU path's tests and the FP64 oracle's tests. It holds the
experiment's noise model and syndrome measurement (Sec. IV of the paper: code capacity, perfect syndrome
measurement, single-qubit depolarizing noise where X, Y and Z each occur with probability p/3), and none
of the decoder's arithmetic.

Conventions (shared as a data contract with the C-ABI library and the oracle):
  * grid of L = 2d-1 rows and columns, site (r, c);
  * qubits at r+c even (horizontal edges at even r, vertical edges at odd r), numbered row-major;
  * Z-checks A_u (products of Z on the edges around a site) at (even r, odd c);
    X-checks B_p (products of X around a plaquette) at (odd r, even c);
  * syndrome bit order: all Z-checks row-major, then all X-checks row-major (m = 2d(d-1) bits);
  * a Pauli on one qubit is coded x + 2z: 0 = I, 1 = X, 2 = Z, 3 = Y.
"""
from __future__ import annotations

import numpy as np

SEED_ENTROPY = 240204834

# workload identifiers used in the seed's spawn key
WORKLOAD_IDS = {"d5": 1, "d11": 2, "d17": 3, "mixed": 4, "warm": 5, "biased": 6, "test": 9}


def grid_size(d: int) -> int:
    return 2 * d - 1


def qubit_coords(d: int) -> np.ndarray:
    L = grid_size(d)
    return np.array([(r, c) for r in range(L) for c in range(L) if (r + c) % 2 == 0], dtype=np.int64)


def check_coords(d: int) -> np.ndarray:
    L = grid_size(d)
    zc = [(r, c) for r in range(0, L, 2) for c in range(1, L, 2)]
    xc = [(r, c) for r in range(1, L, 2) for c in range(0, L, 2)]
    return np.array(zc + xc, dtype=np.int64)


def num_qubits(d: int) -> int:
    return d * d + (d - 1) * (d - 1)


def num_checks(d: int) -> int:
    return 2 * d * (d - 1)


def _check_supports(d: int):
    """For every check (syndrome order): indices of its neighbouring qubits and whether it reads x or z."""
    L = grid_size(d)
    qidx = -np.ones((L, L), dtype=np.int64)
    for i, (r, c) in enumerate(qubit_coords(d)):
        qidx[r, c] = i
    sup, reads_x = [], []
    for r, c in check_coords(d):
        nb = [qidx[rr, cc] for rr, cc in ((r - 1, c), (r, c - 1), (r + 1, c), (r, c + 1))
              if 0 <= rr < L and 0 <= cc < L]
        sup.append(nb)
        reads_x.append(r % 2 == 0)   # Z-checks (even row) detect X components
    return sup, reads_x


_SUPPORT_TABLES = {}


def _support_table(d: int):
    """[m, 4] indices into the concatenation (x bits, z bits, one zero) of each check's neighbours."""
    if d not in _SUPPORT_TABLES:
        n = num_qubits(d)
        sup, reads_x = _check_supports(d)
        t = np.full((len(sup), 4), 2 * n, dtype=np.int64)
        for i, (nb, rx) in enumerate(zip(sup, reads_x)):
            t[i, :len(nb)] = np.asarray(nb, dtype=np.int64) + (0 if rx else n)
        _SUPPORT_TABLES[d] = t
    return _SUPPORT_TABLES[d]


def syndrome_of(d: int, errors: np.ndarray) -> np.ndarray:
    """Syndrome bits [..., m] of Pauli errors [..., n] coded x + 2z: a Z-check is the parity of the x
    components on its neighbouring qubits, an X-check that of the z components."""
    errors = np.asarray(errors, dtype=np.uint8)
    x = errors & 1
    z = (errors >> 1) & 1
    bits = np.concatenate([x, z, np.zeros(errors.shape[:-1] + (1,), dtype=np.uint8)], axis=-1)
    return np.bitwise_xor.reduce(bits[..., _support_table(d)], axis=-1).astype(np.uint8)


def _rng(*key: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence(SEED_ENTROPY, spawn_key=tuple(key))))


def sample_errors(d: int, p: float, count: int, workload: str = "test", p_index: int = 0,
                  start: int = 0) -> np.ndarray:
    """Depolarizing errors [count, n] (codes x + 2z); error i uses its own counter-keyed stream, so any
    slice [start, start+count) of a workload is reproducible on its own."""
    wid = WORKLOAD_IDS[workload]
    n = num_qubits(d)
    out = np.empty((count, n), dtype=np.uint8)
    paulis = np.array([1, 3, 2], dtype=np.uint8)  # X, Y, Z each with probability p/3
    for i in range(count):
        u = _rng(wid, d, p_index, start + i).random(n)
        which = np.minimum((u * (3.0 / p)).astype(np.int64), 2)
        out[i] = np.where(u < p, paulis[which], 0)
    return out


def biased_probs(p: float, eta: float):
    """Pauli probabilities (I, X, Z, Y) -- index = code x + 2z -- of Z-biased noise with total rate p and
    bias eta = p_Z / (p_X + p_Y), p_X = p_Y."""
    pz = p * eta / (1.0 + eta)
    px = py = p / (2.0 * (1.0 + eta))
    return (1.0 - p, px, pz, py)


def sample_errors_pauli(d: int, probs, count: int, workload: str = "biased", p_index: int = 0,
                        start: int = 0) -> np.ndarray:
    """Errors [count, n] (codes x + 2z) of i.i.d. single-qubit Pauli noise with probabilities probs of
    (I, X, Z, Y); error i uses its own counter-keyed stream like sample_errors."""
    wid = WORKLOAD_IDS[workload]
    n = num_qubits(d)
    _, px, pz, py = (float(v) for v in probs)
    out = np.empty((count, n), dtype=np.uint8)
    for i in range(count):
        u = _rng(wid, d, p_index, start + i).random(n)
        out[i] = np.where(u < px, 1, np.where(u < px + py, 3, np.where(u < px + py + pz, 2, 0)))
    return out


def make_batch_pauli(d: int, probs, count: int, workload: str = "biased", p_index: int = 0, start: int = 0):
    """(errors [count, n], syndromes [count, m]) of i.i.d. Pauli noise with probabilities (I, X, Z, Y)."""
    e = sample_errors_pauli(d, probs, count, workload, p_index, start)
    return e, syndrome_of(d, e)


def make_batch(d: int, p: float, count: int, workload: str = "test", p_index: int = 0, start: int = 0):
    """(errors [count, n], syndromes [count, m]) for one distance and noise level."""
    e = sample_errors(d, p, count, workload, p_index, start)
    return e, syndrome_of(d, e)


def mixed_batch(count: int, distances=(9, 13, 17, 21), p_range=(0.05, 0.15), workload: str = "mixed"):
    """Mixed-distance workload: per syndrome, d uniform over `distances`, p uniform over `p_range`.
    Returns a list of (d, p, errors [n], syndrome [m])."""
    wid = WORKLOAD_IDS[workload]
    out = []
    for i in range(count):
        g = _rng(wid, 0, 0, i)
        d = int(distances[g.integers(len(distances))])
        p = float(g.uniform(*p_range))
        e = sample_errors(d, p, 1, workload, 1, i)[0]
        out.append((d, p, e, syndrome_of(d, e)))
    return out
