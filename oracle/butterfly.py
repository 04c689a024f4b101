"""Plain tensor butterfly: construction (Algorithm 1), contraction
(Algorithm 2) and the conjugate-transposed contraction.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

Everything is FP64 and unpadded: every skeleton keeps its true rank, every
intermediate tensor is a dense numpy array whose mode-k length is the sum of
the ranks of the nodes it concatenates, and every block-diagonal factor is
formed explicitly with ``scipy.linalg.block_diag`` before a mode product.

Trees and levels (section 3.2)
------------------------------
Every mode of both grids has a binary tree of L levels with leaves of C_b
indices, n = C_b 2^L; node b at level l covers [b n/2^l, (b+1) n/2^l).  The
paper takes L even and meets in the middle at L^c = L/2.  For odd L this
oracle puts the target middle level at Lt = ceil(L/2) and the source middle
level at Ls = L - Lt (identical to the paper when L is even):

* source side, levels l = 0..Lt: for every source middle multi-set s (level
  Ls), every target multi-set tau at level l, every mode k and every node nu
  at depth Lt - l below s_k (absolute level L - l), an ID of the mode-(d+k)
  unfolding of K(tau, s_{k<-nu}) sampled at proxies, with columns nu's
  indices (l = 0, giving V) or the two children's skeletons from level l-1
  with the parent p_tau (l > 0, giving W);  equations for the source-side
  tensor CLR and transfer matrices in section 3.2;
* target side, levels l = 0..Ls, symmetric: for every target middle
  multi-set t (level Lt), every source multi-set nu at level l, every mode k
  and every node tau at depth Ls - l below t_k, an ID of the mode-k unfolding
  of K(t_{k<-tau}, nu) giving U (l = 0) or P (l > 0);
* cores: K at the skeletons of the top source IDs (tau = t) and the top
  target IDs (nu = s) for every middle pair (t, s).

ID orientation: every interpolation matrix X is r x c with
A ~= A(:, J) X for the sampled unfolding A (columns = the mode's indices).
A source-side X acts on input fibres as X f; a target-side X acts on output
fibres as X^T g (plain transpose).  The conjugate appears only in the adjoint.

Proxy rule (the paper only asks for O(r) "judiciously selected" indices per
mode): for a node covering [lo, lo + len) and a count p, the proxies are
lo + floor((2q + 1) len / (2p)), q = 0..p-1, or the whole node if len <= p
(p <= 0 means the whole node).  The mode paired with the skeletonised one
(tau_k on the source side, nu_k on the target side) gets p = p_pair * c for
an ID with c columns (twice oversampled by default: with as many samples as
columns, equispaced samples of an oscillatory block alias and the sampled
block looks rank deficient), every other mode a fixed ``p_other``.

Multi-set flattening: a multi-set (b_1..b_d) at level l has flat index
sum_k b_k 2^(l (d-1-k)).  Source items are keyed (s_flat, tau_flat), target
items (t_flat, nu_flat), cores (t_flat, s_flat).
"""
from __future__ import annotations

import itertools
import math
from dataclasses import dataclass, field

import numpy as np
from scipy.linalg import block_diag

from .idqr import column_id
from .kernels import Operator
from .tucker import mode_product


# ----------------------------------------------------------------------------
# bookkeeping
# ----------------------------------------------------------------------------

def unflatten(flat: int, level: int, d: int) -> tuple:
    mask = (1 << level) - 1
    return tuple((flat >> (level * (d - 1 - k))) & mask for k in range(d))


def flatten(b, level: int) -> int:
    out = 0
    for bk in b:
        out = (out << level) | int(bk)
    return out


def node_range(level: int, b: int, n: int) -> tuple:
    size = n >> level
    return b * size, size


def proxies(lo: int, length: int, p: int) -> np.ndarray:
    if p <= 0 or length <= p:
        return np.arange(lo, lo + length, dtype=np.int64)
    q = np.arange(p, dtype=np.int64)
    return lo + ((2 * q + 1) * length) // (2 * p)


def default_proxy_counts(d: int, leaf: int) -> tuple:
    """(p_pair, p_other) used when none are given: the paired mode takes
    p_pair samples per ID column, every other mode p_other samples (an ID's
    unfolding has 2d - 1 sampled modes, so p_other shrinks with d: 4 leaf
    for d = 2, 4 for d = 3, 2 from d = 4 on)."""
    return 2, (4 * leaf if d == 2 else (4 if d == 3 else 2))


DEFAULT_ID_TOL_SCALE = 0.3


def _pair_count(p_pair: int, ncols: int) -> int:
    return 0 if p_pair <= 0 else p_pair * ncols


@dataclass
class Skeleton:
    """One ID: skeleton indices (global, in pivot order) and X (r x c)."""
    skel: np.ndarray
    X: np.ndarray

    @property
    def rank(self) -> int:
        return int(self.skel.shape[0])


@dataclass
class Plan:
    op: Operator
    tol: float
    eps_id: float
    leaf: int
    L: int
    Lt: int
    Ls: int
    p_pair: int
    p_other: int
    # src[l][(s_flat, tau_flat)][k][nu] ; tgt[l][(t_flat, nu_flat)][k][tau]
    src: list = field(default_factory=list)
    tgt: list = field(default_factory=list)
    cores: dict = field(default_factory=dict)   # (t_flat, s_flat) -> (RT, RS)

    @property
    def d(self) -> int:
        return self.op.d

    @property
    def n(self) -> int:
        return self.op.n

    def ranks(self):
        """All ID ranks, source and target."""
        out = []
        for side in (self.src, self.tgt):
            for lev in side:
                for per_k in lev.values():
                    for ids in per_k:
                        out.extend(sk.rank for sk in ids)
        return np.array(out)

    def core_shape(self, t_flat: int, s_flat: int) -> tuple:
        rt = [self.tgt[self.Ls][(t_flat, s_flat)][k][0].rank for k in range(self.d)]
        rs = [self.src[self.Lt][(s_flat, t_flat)][k][0].rank for k in range(self.d)]
        return rt, rs


# ----------------------------------------------------------------------------
# construction (Algorithm 1)
# ----------------------------------------------------------------------------

def _product_rows(lists):
    """Cartesian product of per-mode index lists, shape (R, len(lists))."""
    grids = np.meshgrid(*lists, indexing="ij")
    return np.stack([g.reshape(-1) for g in grids], axis=-1)


def _sample(op: Operator, tgt_rows, src_rows, k_src=None, k_tgt=None,
            cols=None):
    """Sampled unfolding A[row, c]: the column index replaces mode k of the
    source (``k_src``) or of the target (``k_tgt``)."""
    R, C = tgt_rows.shape[0], len(cols)
    ti = np.broadcast_to(tgt_rows[:, None, :], (R, C, op.d)).copy()
    sj = np.broadcast_to(src_rows[:, None, :], (R, C, op.d)).copy()
    if k_src is not None:
        sj[:, :, k_src] = cols[None, :]
    else:
        ti[:, :, k_tgt] = cols[None, :]
    return op.entries(ti, sj)


def source_unfolding(plan: Plan, s, l: int, tau, k: int, cols) -> np.ndarray:
    """Proxy-sampled mode-k unfolding of a source-side ID (section 3.2,
    Algorithm 1 step 1): rows are the proxy targets of tau (level l) in every
    mode, times the proxy sources of the middle multi-set s in every mode
    but k; columns are the candidate mode-k source indices ``cols``.  The
    paired mode k of tau gets p_pair samples per column."""
    op, n, d = plan.op, plan.n, plan.d
    tlists = []
    for i in range(d):
        lo, ln = node_range(l, tau[i], n)
        p = _pair_count(plan.p_pair, len(cols)) if i == k else plan.p_other
        tlists.append(proxies(lo, ln, p))
    slists = []
    for i in range(d):
        if i == k:
            slists.append(np.zeros(1, dtype=np.int64))
        else:
            lo, ln = node_range(plan.Ls, s[i], n)
            slists.append(proxies(lo, ln, plan.p_other))
    rows = _product_rows(tlists + slists)
    return _sample(op, rows[:, :d], rows[:, d:], k_src=k, cols=np.asarray(cols))


def target_unfolding(plan: Plan, t, l: int, nu, k: int, cols) -> np.ndarray:
    """The target-side mirror of ``source_unfolding``: rows are the proxy
    targets of the middle multi-set t in every mode but k, times the proxy
    sources of nu (level l) in every mode; columns are mode-k target
    indices."""
    op, n, d = plan.op, plan.n, plan.d
    tlists = []
    for i in range(d):
        if i == k:
            tlists.append(np.zeros(1, dtype=np.int64))
        else:
            lo, ln = node_range(plan.Lt, t[i], n)
            tlists.append(proxies(lo, ln, plan.p_other))
    slists = []
    for i in range(d):
        lo, ln = node_range(l, nu[i], n)
        p = _pair_count(plan.p_pair, len(cols)) if i == k else plan.p_other
        slists.append(proxies(lo, ln, p))
    rows = _product_rows(tlists + slists)
    return _sample(op, rows[:, :d], rows[:, d:], k_tgt=k, cols=np.asarray(cols))


def construct(op: Operator, tol: float, leaf: int = 8, p_pair: int | None = None,
              p_other: int | None = None, id_tol_scale: float | None = None,
              lt: int | None = None) -> Plan:
    """Algorithm 1.  ``tol`` is the requested relative accuracy of the
    butterfly; every ID runs at eps = id_tol_scale * tol, by default 0.3 tol.
    (The paper runs its IDs at the tolerance itself and reports end-to-end
    errors of 1-2 times it; one middle-level Tucker-ID alone can reach
    sqrt(2d) eps by section 3.1, and the nesting over levels adds to that.)
    ``lt`` overrides the target middle level (default ceil(L/2))."""
    n, d = op.n, op.d
    L = int(round(math.log2(n / leaf)))
    if leaf * (1 << L) != n or L < 0:
        raise ValueError("n must be leaf * 2^L")
    dp, do = default_proxy_counts(d, leaf)
    p_pair = dp if p_pair is None else p_pair
    p_other = do if p_other is None else p_other
    Lt = L - L // 2 if lt is None else lt
    if not 0 <= Lt <= L:
        raise ValueError("target middle level out of range")
    Ls = L - Lt
    if id_tol_scale is None:
        id_tol_scale = DEFAULT_ID_TOL_SCALE
    eps = tol * id_tol_scale
    plan = Plan(op, tol, eps, leaf, L, Lt, Ls, p_pair, p_other)

    # (1) source side: V at l = 0, W at l = 1..Lt
    for l in range(Lt + 1):
        depth = Lt - l
        lev = {}
        for s_flat in range(1 << (d * Ls)):
            s = unflatten(s_flat, Ls, d)
            for tau_flat in range(1 << (d * l)):
                tau = unflatten(tau_flat, l, d)
                per_k = []
                for k in range(d):
                    ids = []
                    for nu in range(1 << depth):
                        if l == 0:
                            nu_abs = s[k] * (1 << depth) + nu
                            cols = np.arange(nu_abs * leaf, (nu_abs + 1) * leaf)
                        else:
                            ptau = flatten([b >> 1 for b in tau], l - 1)
                            par = plan.src[l - 1][(s_flat, ptau)][k]
                            cols = np.concatenate([par[2 * nu].skel, par[2 * nu + 1].skel])
                        A = source_unfolding(plan, s, l, tau, k, cols)
                        cid = column_id(A, eps)
                        ids.append(Skeleton(cols[cid.skel], cid.X))
                    per_k.append(ids)
                lev[(s_flat, tau_flat)] = per_k
        plan.src.append(lev)

    # (2) target side: U at l = 0, P at l = 1..Ls
    for l in range(Ls + 1):
        depth = Ls - l
        lev = {}
        for t_flat in range(1 << (d * Lt)):
            t = unflatten(t_flat, Lt, d)
            for nu_flat in range(1 << (d * l)):
                nu = unflatten(nu_flat, l, d)
                per_k = []
                for k in range(d):
                    ids = []
                    for tau in range(1 << depth):
                        if l == 0:
                            tau_abs = t[k] * (1 << depth) + tau
                            cols = np.arange(tau_abs * leaf, (tau_abs + 1) * leaf)
                        else:
                            pnu = flatten([b >> 1 for b in nu], l - 1)
                            par = plan.tgt[l - 1][(t_flat, pnu)][k]
                            cols = np.concatenate([par[2 * tau].skel, par[2 * tau + 1].skel])
                        A = target_unfolding(plan, t, l, nu, k, cols)
                        cid = column_id(A, eps)
                        ids.append(Skeleton(cols[cid.skel], cid.X))
                    per_k.append(ids)
                lev[(t_flat, nu_flat)] = per_k
        plan.tgt.append(lev)

    # (3) cores K(tbar, sbar) for every middle pair
    for t_flat in range(1 << (d * Lt)):
        for s_flat in range(1 << (d * Ls)):
            plan.cores[(t_flat, s_flat)] = core_entries(plan, t_flat, s_flat)
    return plan


def core_entries(plan: Plan, t_flat: int, s_flat: int) -> np.ndarray:
    """K(tbar, sbar) as an R_T x R_S matrix, rows and columns row-major over
    the modes (mode d fastest), each mode in skeleton (pivot) order."""
    d = plan.d
    tb = [plan.tgt[plan.Ls][(t_flat, s_flat)][k][0].skel for k in range(d)]
    sb = [plan.src[plan.Lt][(s_flat, t_flat)][k][0].skel for k in range(d)]
    ti = _product_rows(tb)
    sj = _product_rows(sb)
    return plan.op.entries(ti[:, None, :], sj[None, :, :])


# ----------------------------------------------------------------------------
# contraction (Algorithm 2) and its conjugate transpose
# ----------------------------------------------------------------------------

def _block(x: np.ndarray, lo, size) -> np.ndarray:
    """x[:, lo_0:lo_0+size_0, ...] for an (nv, n, ..., n) array."""
    sl = (slice(None),) + tuple(slice(a, a + b) for a, b in zip(lo, size))
    return x[sl]


def _src_block_index(plan: Plan, s):
    size = plan.n >> plan.Ls
    return [b * size for b in s], [size] * plan.d


def _tgt_block_index(plan: Plan, t):
    size = plan.n >> plan.Lt
    return [b * size for b in t], [size] * plan.d


def apply(plan: Plan, f: np.ndarray) -> np.ndarray:
    """u = K_BF f for f of shape (nv, n, ..., n) (or (n, ..., n))."""
    d, n, Lt, Ls = plan.d, plan.n, plan.Lt, plan.Ls
    f = np.asarray(f, dtype=np.complex128)
    if f.shape == (n,) * d:
        f = f[None]
    nv = f.shape[0]

    # step (1): V at l = 0, then W at l = 1..Lt; F[(s_flat, tau_flat)]
    F = {}
    for s_flat in range(1 << (d * Ls)):
        s = unflatten(s_flat, Ls, d)
        lo, size = _src_block_index(plan, s)
        T = np.moveaxis(_block(f, lo, size), 0, -1)
        ids = plan.src[0][(s_flat, 0)]
        for k in range(d):
            T = mode_product(T, block_diag(*[sk.X for sk in ids[k]]), k)
        F[(s_flat, 0)] = T
    for l in range(1, Lt + 1):
        Fn = {}
        for s_flat in range(1 << (d * Ls)):
            for tau_flat in range(1 << (d * l)):
                tau = unflatten(tau_flat, l, d)
                ptau = flatten([b >> 1 for b in tau], l - 1)
                T = F[(s_flat, ptau)]
                ids = plan.src[l][(s_flat, tau_flat)]
                for k in range(d):
                    T = mode_product(T, block_diag(*[sk.X for sk in ids[k]]), k)
                Fn[(s_flat, tau_flat)] = T
        F = Fn

    # step (2): G_{t,s} = K(tbar, sbar) x F_{t,s}
    G = {}
    for t_flat in range(1 << (d * Lt)):
        for s_flat in range(1 << (d * Ls)):
            Ft = F[(s_flat, t_flat)]
            rt, rs = plan.core_shape(t_flat, s_flat)
            g = plan.cores[(t_flat, s_flat)] @ Ft.reshape(-1, nv)
            G[(t_flat, s_flat)] = g.reshape(tuple(rt) + (nv,))

    # step (3): P^T at l = Ls..1 with accumulation into the parent, U^T at 0
    for l in range(Ls, 0, -1):
        Gp = {}
        for t_flat in range(1 << (d * Lt)):
            for nu_flat in range(1 << (d * l)):
                nu = unflatten(nu_flat, l, d)
                pnu = flatten([b >> 1 for b in nu], l - 1)
                T = G[(t_flat, nu_flat)]
                ids = plan.tgt[l][(t_flat, nu_flat)]
                for k in range(d):
                    T = mode_product(T, block_diag(*[sk.X.T for sk in ids[k]]), k)
                key = (t_flat, pnu)
                Gp[key] = T if key not in Gp else Gp[key] + T
        G = Gp
    u = np.zeros((nv,) + (n,) * d, dtype=np.complex128)
    for t_flat in range(1 << (d * Lt)):
        t = unflatten(t_flat, Lt, d)
        T = G[(t_flat, 0)]
        ids = plan.tgt[0][(t_flat, 0)]
        for k in range(d):
            T = mode_product(T, block_diag(*[sk.X.T for sk in ids[k]]), k)
        lo, size = _tgt_block_index(plan, t)
        sl = (slice(None),) + tuple(slice(a, a + b) for a, b in zip(lo, size))
        u[sl] = np.moveaxis(T, -1, 0)
    return u


def apply_adjoint(plan: Plan, g: np.ndarray) -> np.ndarray:
    """v = K_BF^H g: every factor conjugate-transposed, in reverse order."""
    d, n, Lt, Ls = plan.d, plan.n, plan.Lt, plan.Ls
    g = np.asarray(g, dtype=np.complex128)
    if g.shape == (n,) * d:
        g = g[None]
    nv = g.shape[0]

    # target leaves: conj(U) maps each leaf's C_b values to its skeleton
    G = {}
    for t_flat in range(1 << (d * Lt)):
        t = unflatten(t_flat, Lt, d)
        lo, size = _tgt_block_index(plan, t)
        T = np.moveaxis(_block(g, lo, size), 0, -1)
        ids = plan.tgt[0][(t_flat, 0)]
        for k in range(d):
            T = mode_product(T, block_diag(*[np.conj(sk.X) for sk in ids[k]]), k)
        G[(t_flat, 0)] = T
    # target transfers, l = 1..Ls: every child nu reads its parent, conj(P)
    for l in range(1, Ls + 1):
        Gn = {}
        for t_flat in range(1 << (d * Lt)):
            for nu_flat in range(1 << (d * l)):
                nu = unflatten(nu_flat, l, d)
                pnu = flatten([b >> 1 for b in nu], l - 1)
                T = G[(t_flat, pnu)]
                ids = plan.tgt[l][(t_flat, nu_flat)]
                for k in range(d):
                    T = mode_product(T, block_diag(*[np.conj(sk.X) for sk in ids[k]]), k)
                Gn[(t_flat, nu_flat)] = T
        G = Gn
    # cores: F_{t,s} = K(tbar, sbar)^H G_{t,s}
    F = {}
    for t_flat in range(1 << (d * Lt)):
        for s_flat in range(1 << (d * Ls)):
            rt, rs = plan.core_shape(t_flat, s_flat)
            Gt = G[(t_flat, s_flat)]
            x = np.conj(plan.cores[(t_flat, s_flat)]).T @ Gt.reshape(-1, nv)
            F[(s_flat, t_flat)] = x.reshape(tuple(rs) + (nv,))
    # source transfers, l = Lt..1: W^H, summed over the 2^d children tau
    for l in range(Lt, 0, -1):
        Fp = {}
        for s_flat in range(1 << (d * Ls)):
            for tau_flat in range(1 << (d * l)):
                tau = unflatten(tau_flat, l, d)
                ptau = flatten([b >> 1 for b in tau], l - 1)
                T = F[(s_flat, tau_flat)]
                ids = plan.src[l][(s_flat, tau_flat)]
                for k in range(d):
                    T = mode_product(T, block_diag(*[np.conj(sk.X).T for sk in ids[k]]), k)
                key = (s_flat, ptau)
                Fp[key] = T if key not in Fp else Fp[key] + T
        F = Fp
    # source leaves: V^H
    v = np.zeros((nv,) + (n,) * d, dtype=np.complex128)
    for s_flat in range(1 << (d * Ls)):
        s = unflatten(s_flat, Ls, d)
        T = F[(s_flat, 0)]
        ids = plan.src[0][(s_flat, 0)]
        for k in range(d):
            T = mode_product(T, block_diag(*[np.conj(sk.X).T for sk in ids[k]]), k)
        lo, size = _src_block_index(plan, s)
        sl = (slice(None),) + tuple(slice(a, a + b) for a, b in zip(lo, size))
        v[sl] = np.moveaxis(T, -1, 0)
    return v


# ----------------------------------------------------------------------------
# accounting
# ----------------------------------------------------------------------------

def plan_stats(plan: Plan) -> dict:
    """Ranks, entry counts and exact complex multiply-add counts per RHS."""
    d = plan.d
    ranks = plan.ranks()
    factor_entries = 0
    for side in (plan.src, plan.tgt):
        for lev in side:
            for per_k in lev.values():
                for ids in per_k:
                    factor_entries += sum(sk.X.size for sk in ids)
    core_entries = sum(c.size for c in plan.cores.values())
    return {
        "L": plan.L, "Lt": plan.Lt, "Ls": plan.Ls,
        "r_min": int(ranks.min()), "r_max": int(ranks.max()),
        "n_ids": int(ranks.size),
        "factor_entries": int(factor_entries),
        "core_entries": int(core_entries),
        "pairs": len(plan.cores),
        "d": d,
    }


def all_multi_indices(level: int, d: int):
    return itertools.product(range(1 << level), repeat=d)
