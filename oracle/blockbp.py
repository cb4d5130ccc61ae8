"""blockBP decoder, FP64 reference (oracle; test infrastructure only).

Follows Alg. 1 of the paper (Sec. III.E) and its remarks:
  * partition the coset network into rectangular blocks; blocks at the edges are smaller when the block
    size does not divide 2d-1 (remark 1) -- here the last block row / column holds the remainder;
  * messages between neighbouring blocks are MPSs with one site per crossing bond, ordered top->bottom
    across vertical cuts and left->right across horizontal cuts, with bond dimension at most chi
    (Sec. III.D); they start as the uniform distribution (remark 2);
  * a block's outgoing message is the BP update rule (eq. for m_{v->u}, Sec. III.C) evaluated by the
    boundary-MPS method with bond chi inside the block (Sec. III.D, Fig. 3): the sweep starts from the
    message entering on the side opposite the receiver, absorbs the block column by column, and the
    messages on the two remaining sides enter as end caps of the boundary MPS, one site per column, in the
    canonical form whose not-yet-absorbed part is an isometry (right-canonical when walked from the first
    site, left-canonical from the last: this implementation's reading, see block_sweep); after every column
    the boundary MPS is compressed to chi (QR sweep, then truncated-SVD sweep);
  * outgoing messages are made left-canonical with unit norm (remark 3), damped
    m <- (1-eta) m_new + eta m_old and renormalised (remark 7);
  * schedule: blocks are coloured as a chessboard, colour (I+J) even sends first, then the other colour
    using the fresh messages (remark 8); one iteration = both rounds;
  * convergence distance Delta = (1/M) * sqrt(sum_i || |m_i^t><m_i^t| - |m_i^{t-1}><m_i^{t-1}| ||_F^2)
    over all M directed messages, with || |a><a| - |b><b| ||_F^2 = 2 - 2<a,b>^2 for unit vectors;
    the loop exits when Delta < delta0 (remark 4), unless a fixed iteration count is requested;
  * Bethe estimate (Lemma 3.1): ln Z = sum_v ln W_v - sum_e ln o_e, where W_v contracts block v with its
    four incoming unit messages (the same chi-truncated sweep, closed against the last message) and
    o_e = <m_{u->v}, m_{v->u}>; rescaling each message by 1/sqrt(o_e) gives the normalisation the lemma
    asks for;
  * decision (Alg. 1 tail, remark 6): among cosets with Delta < delta1 take the largest ln Z; if none,
    the smallest Delta; ties go to the lowest index in (I, X, Y, Z). rule=1 is the plain argmax of ln Z.
A non-positive W_v or o_e marks the coset untrusted (Delta = +inf, ln Z = nan).
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from . import lattice, mps, network

DIRS = {"E": (0, 1), "W": (0, -1), "S": (1, 0), "N": (-1, 0)}
# frame leg permutation: (up, in, down, out) expressed in the tensor's (up, left, down, right) axes
FRAME_PERM = {"E": (0, 1, 2, 3), "W": (0, 3, 2, 1), "S": (1, 0, 3, 2), "N": (1, 2, 3, 0)}


def splits(L: int, k: int):
    """Block extents along one axis: [k, ..., k, L mod k] (remark 1)."""
    out, s = [], 0
    while s < L:
        out.append((s, min(k, L - s)))
        s += k
    return out


@dataclass
class Plan:
    d: int
    kr: int
    kc: int

    def __post_init__(self):
        L = lattice.side(self.d)
        self.rows = splits(L, self.kr)
        self.cols = splits(L, self.kc)
        self.nI, self.nJ = len(self.rows), len(self.cols)
        self.blocks = [(I, J) for I in range(self.nI) for J in range(self.nJ)]
        self.edges = []          # directed (src, dst, direction from src)
        for (I, J) in self.blocks:
            for dname, (dI, dJ) in DIRS.items():
                nb = (I + dI, J + dJ)
                if 0 <= nb[0] < self.nI and 0 <= nb[1] < self.nJ:
                    self.edges.append(((I, J), nb, dname))
        self.M = len(self.edges)

    def has(self, b):
        return 0 <= b[0] < self.nI and 0 <= b[1] < self.nJ

    def msg_len(self, src, dst):
        """Number of sites of the message between two adjacent blocks."""
        if src[0] == dst[0]:
            return self.rows[src[0]][1]
        return self.cols[src[1]][1]


def _frame(plan: Plan, tensors, I: int, J: int, frame: str):
    """Frame view of block (I, J) for a sweep toward side `frame`: returns (kt, kp, F) where F(t, i) is the
    tensor at sweep step t and position i with legs (up, in, down, out), plus the neighbours
    (init, top cap, bottom cap, receiver) and whether the caps are consumed first-site-first."""
    r0, kr = plan.rows[I]
    c0, kc = plan.cols[J]
    perm = FRAME_PERM[frame]

    def T(r, c):
        t = tensors[r][c]
        nb = t.ndim - 4
        return np.transpose(t, tuple(range(nb)) + tuple(nb + a for a in perm))

    if frame == "E":
        F = lambda t, i: T(r0 + i, c0 + t)
        return kc, kr, F, (I, J - 1), (I - 1, J), (I + 1, J), (I, J + 1), True
    if frame == "W":
        F = lambda t, i: T(r0 + i, c0 + kc - 1 - t)
        return kc, kr, F, (I, J + 1), (I - 1, J), (I + 1, J), (I, J - 1), False
    if frame == "S":
        F = lambda t, i: T(r0 + t, c0 + i)
        return kr, kc, F, (I - 1, J), (I, J - 1), (I, J + 1), (I + 1, J), True
    if frame == "N":
        F = lambda t, i: T(r0 + kr - 1 - t, c0 + i)
        return kr, kc, F, (I + 1, J), (I, J - 1), (I, J + 1), (I - 1, J), False
    raise ValueError(frame)


def block_sweep(plan: Plan, tensors, msgs, I: int, J: int, frame: str, chi: int, batch):
    """Boundary-MPS contraction of block (I, J) with its incoming messages except the one from the
    receiver on side `frame` (eq. of the BP update, evaluated as in Sec. III.D).
    Returns (k-site MPS over the receiver-side legs, log-scale split off during the sweep)."""
    kt, kp, F, init_nb, top_nb, bot_nb, _, forward = _frame(plan, tensors, I, J, frame)
    me = (I, J)
    one = np.ones(batch + (1, 1, 1))

    if plan.has(init_nb):
        h = list(msgs[(init_nb, me)])
    else:
        h = [one] * kp
    state = [one] + h + [one]
    logscale = np.zeros(batch)

    # The side messages enter with the part still to be absorbed an isometry: a sweep that walks a message
    # from its first site takes the right-canonical form (weight on site 0), one that walks it from its last
    # site the stored left-canonical form (weight on the last site). The truncations then see the boundary
    # state in the metric of the rest of the cap, and the result depends on the message only, not on the
    # choice of its canonical form (a left-canonical form walked from its first site would put weightless
    # completion directions -- e.g. those of the rank-1 uniform start -- into every truncation).
    right = {}

    def cap_site(nb, t):
        if not plan.has(nb):
            return one
        m = msgs[(nb, me)]
        if forward:
            if nb not in right:
                right[nb] = mps.right_canonicalize(m)
            return right[nb][t]
        return np.swapaxes(m[kt - 1 - t], -1, -3)   # consumed last-site-first: (b_{j+1}, 2, b_j)

    for t in range(kt):
        A = cap_site(top_nb, t)
        Bc = cap_site(bot_nb, t)
        new = []
        C = state[0]
        c = np.einsum("...aPd,...PvQ->...aQdv", C, A)
        new.append(c.reshape(batch + (1, c.shape[-3], c.shape[-2] * c.shape[-1])))
        for i in range(kp):
            H = state[1 + i]
            Ft = F(t, i)
            o = np.einsum("...aib,...uido->...auobd", H, Ft)
            s = o.shape
            new.append(o.reshape(batch + (s[-5] * s[-4], s[-3], s[-2] * s[-1])))
        C = state[-1]
        c = np.einsum("...dPa,...PvQ->...dvQa", C, Bc)
        new.append(c.reshape(batch + (c.shape[-4] * c.shape[-3], c.shape[-2], 1)))
        state, ls = mps.compress(new, chi)
        logscale = logscale + ls

    top = state[0].reshape(batch + (1, state[0].shape[-1]))
    bot = state[-1].reshape(batch + (state[-1].shape[-3], 1))
    out = state[1:-1]
    out[0] = np.einsum("...ad,...dpe->...ape", top, out[0])
    out[-1] = np.einsum("...apd,...de->...ape", out[-1], bot)
    return out, logscale


def _take(sites, idx):
    return [s[idx] for s in sites]


def run_bp(plan: Plan, tensors, chi: int, max_iter: int, delta0: float, eta: float, fixed_iters: bool,
           gate: float = 0.0):
    """BP loop of Alg. 1 for a batch of coset networks (tensors[r][c] of shape [B, ...]).
    Returns (messages dict, Delta [B], iterations [B]).

    gate > 0 selects the residual-gated schedule, a scheduling variant (Sec. IV names smarter BP scheduling
    as a way to improve the hardest regimes and leaves it open; the rule itself is this implementation's
    reading): in a colour round the update of message u->v is skipped for a coset when the message itself and
    every message entering block u other than v->u changed, in their most recent updates, by a distance term
    2 - 2<m, m_old>^2 below gate; a skipped message keeps its value and its term becomes 0. Messages that were
    never updated count as changed. (With damping, a message whose inputs have settled still moves towards
    their image, so its own change is part of the test.)"""
    B = tensors[0][0].shape[0]
    msgs = {}
    for (src, dst, _) in plan.edges:
        K = plan.msg_len(src, dst)
        msgs[(src, dst)] = mps.uniform([2] * K, chi, (B,))
    delta = np.full(B, np.inf)
    iters = np.zeros(B, dtype=np.int64)
    terms = {(src, dst): np.full(B, np.inf) for (src, dst, _) in plan.edges}
    inputs = {(src, dst): [(w, s2) for (w, s2, _) in plan.edges if s2 == src and w != dst]
              for (src, dst, _) in plan.edges}
    active = np.arange(B)
    L = len(tensors)
    for _ in range(max_iter):
        if active.size == 0:
            break
        nb = (active.size,)
        sub_t = [[tensors[r][c][active] for c in range(L)] for r in range(L)]
        sub_m = {e: _take(v, active) for e, v in msgs.items()}
        prev = dict(sub_m)
        for colour in (0, 1):
            fresh = {}
            for (src, dst, dname) in plan.edges:
                if (src[0] + src[1]) % 2 != colour:
                    continue
                raw, _ = block_sweep(plan, sub_t, sub_m, src[0], src[1], dname, chi, nb)
                m_new, _ = mps.canonical_message(raw, chi)
                if eta > 0.0:
                    mix = mps.direct_sum(m_new, sub_m[(src, dst)], np.full(nb, 1.0 - eta), np.full(nb, eta))
                    m_new, _ = mps.canonical_message(mix, chi)
                if gate > 0.0:
                    changed = ~(terms[(src, dst)][active] < gate)
                    for key_in in inputs[(src, dst)]:
                        changed |= ~(terms[key_in][active] < gate)
                    old = sub_m[(src, dst)]
                    m_new = [np.where(changed[:, None, None, None], a_new, a_old)
                             for a_new, a_old in zip(m_new, old)]
                fresh[(src, dst)] = m_new
            sub_m.update(fresh)
            if gate > 0.0:
                for key, v in fresh.items():
                    ov = mps.overlap(v, prev[key])
                    t = terms[key]
                    t[active] = 2.0 - 2.0 * ov * ov
        acc = np.zeros(nb)
        for e in plan.edges:
            key = (e[0], e[1])
            ov = mps.overlap(sub_m[key], prev[key])
            acc += 2.0 - 2.0 * ov * ov
        dlt = np.sqrt(np.maximum(acc, 0.0)) / max(plan.M, 1)
        for key, v in sub_m.items():
            for s_full, s_sub in zip(msgs[key], v):
                s_full[active] = s_sub
        delta[active] = dlt
        iters[active] += 1
        if not fixed_iters:
            active = active[dlt >= delta0]
    return msgs, delta, iters


def bethe(plan: Plan, tensors, msgs, chi: int):
    """Lemma 3.1: ln Z = sum_v ln W_v - sum_e ln <m_{u->v}, m_{v->u}>. Returns (ln Z [B], bad [B])."""
    B = tensors[0][0].shape[0]
    batch = (B,)
    lnz = np.zeros(B)
    bad = np.zeros(B, dtype=bool)
    for (I, J) in plan.blocks:
        st, ls = block_sweep(plan, tensors, msgs, I, J, "E", chi, batch)
        east = (I, J + 1)
        if plan.has(east):
            w = mps.overlap(st, msgs[(east, (I, J))])
        else:
            w = mps.to_dense(st)[..., 0]
        bad |= ~(w > 0)
        lnz += ls + np.log(np.abs(w))
    for (src, dst, _) in plan.edges:
        if src < dst:
            o = mps.overlap(msgs[(src, dst)], msgs[(dst, src)])
            bad |= ~(o > 0)
            lnz -= np.log(np.abs(o))
    return lnz, bad


def decide(loglik: np.ndarray, delta: np.ndarray, delta1: float, rule: int = 0) -> np.ndarray:
    """Coset decision over [S, 4] arrays (Alg. 1 tail; remark 6)."""
    ll = np.where(np.isnan(loglik), -np.inf, loglik)
    if rule == 1:
        return np.argmax(ll, axis=-1)
    trusted = delta < delta1
    best_trusted = np.argmax(np.where(trusted, ll, -np.inf), axis=-1)
    return np.where(trusted.any(axis=-1), best_trusted, np.argmin(delta, axis=-1))


def decode(d: int, eps: float, syndromes: np.ndarray, block=(6, 6), chi: int = 16, max_iter: int = 20,
           delta0: float = 1e-4, delta1: float = 1e-2, eta: float = 0.1, fixed_iters: bool = False,
           rule: int = 0, noise=None, return_messages: bool = False, gate: float = 0.0):
    """Decode syndromes [S, m]. Returns a dict with loglik [S, 4] (ln of the Bethe estimate of each coset
    probability, order I, X, Y, Z), delta [S, 4], iters [S, 4], coset [S], correction [S, n] (codes
    x + 2z of f_s L*), and optionally the final messages."""
    syndromes = np.atleast_2d(np.asarray(syndromes, dtype=np.uint8))
    S = syndromes.shape[0]
    pi = network.depolarizing(eps) if noise is None else np.asarray(noise, dtype=np.float64)
    x, z = lattice.coset_labels(d, syndromes)                       # [S, 4, L, L]
    L = lattice.side(d)
    xb = x.reshape(S * 4, L, L)
    zb = z.reshape(S * 4, L, L)
    plan = Plan(d, block[0], block[1])
    tensors = network.coset_tensors(d, xb, zb, pi)
    msgs, delta, iters = run_bp(plan, tensors, chi, max_iter, delta0, eta, fixed_iters, gate)
    lnz, bad = bethe(plan, tensors, msgs, chi)
    lnz = np.where(bad, np.nan, lnz)
    delta = np.where(bad, np.inf, delta)
    loglik = lnz.reshape(S, 4)
    delta = delta.reshape(S, 4)
    coset = decide(loglik, delta, delta1, rule)
    fx, fz = lattice.pauli_for_syndrome(d, syndromes)
    xm, zm = lattice.logical_masks(d)
    bits = np.array(lattice.COSET_BITS)[coset]                      # [S, 2]
    cx = fx ^ (xm[None] * bits[:, 0, None, None]).astype(np.uint8)
    cz = fz ^ (zm[None] * bits[:, 1, None, None]).astype(np.uint8)
    out = dict(loglik=loglik, delta=delta, iters=iters.reshape(S, 4), coset=coset,
               correction=lattice.codes_from_pauli_grid(d, cx, cz), plan=plan)
    if return_messages:
        out["messages"] = msgs
    return out
