"""Recursive strong skeletonization with dense bookkeeping (oracle; test infrastructure).

The whole scaled matrix A~ is kept as a dense array; every Schur-complement update is
applied to it in place, so that any entry can be inspected at any time. This is the
plainest possible form of the method of Sections 4.1-4.4 and 5.1-5.2:

  for each level l = L, L-1, ..., 2 (finest first, Section 4.2):
    for each level-l box B holding active DOFs, in the schedule below:
      classify every other active DOF by the box that owns it (near N, far F = Q u P);
      ID of the stacked matrix [A_QB ; A_BQ^T ; proxy outgoing ; proxy incoming]
        (Section 5.1.3, simultaneous skeletonization) -> S, R, T;
      elimination E, F with T, then L, U with the pivot block X_RR (Section 4.1,
        eq. strong-skel-elim); the Schur complement is subtracted from A_{(S u N)(S u N)};
      the redundant DOFs R become inactive.
  the remaining active DOFs B_t form the top block, factored by dense LU (Section 4.2).

Readings where the paper is silent (each is also listed in the design notes):
  * Owners. At level l every active DOF is owned either by its level-l ancestor box or,
    when its leaf is coarser than l, by that leaf (coarse leaves keep their points
    active until their own level).
  * Near/far split (Section 4.4, radius 5R/2 around B). With g the L-infinity gap
    between B (side R) and the owner box, in units of R: N if g = 0 (touching),
    Q if 0 < g < 2 (the owner meets the open cube of side 5R centred on B), P if
    g >= 2. Every P point is then at distance >= 2.5R from the centre of B, on or
    outside the proxy sphere. The cube is the sphere's bounding cube: it puts every box
    that meets the sphere into Q.
  * Boxes without far-field DOFs (Q and P empty) are not skeletonized at that level.
  * Order within a level: by colour (ix mod 2) + 2 (iy mod 2) + 4 (iz mod 2), then by
    Morton key. Same-colour boxes never touch, but two of them can lie in each other's Q
    region (one box side apart).
  * schedule="sequential" (the paper's box-by-box loop): each box classifies the DOFs that
    are active when its turn comes, so the redundant DOFs of a same-colour box eliminated
    earlier in the phase are gone from its Q rows.
    schedule="phase_start" (the colour phase as one concurrent step): every box of a colour
    phase classifies the DOFs that were active when the phase began, so its Q rows also
    hold the redundant DOFs R1 of an earlier same-colour box B1. Those rows are, to the ID
    tolerance, combinations of B1's skeleton rows (B1's own ID compressed A[B1, B2] with B2
    in B1's Q region: A[R1, B2] ~ T1^T A[S1, B2]), so the ID of the larger matrix is equally
    valid, and nothing else differs: a box's elimination reads only blocks between its own
    and its near DOFs, which no other box of its colour writes (same-colour boxes do not
    touch), and the Schur updates of same-colour boxes to shared near-near blocks add.
  * Proxy surface (Section 5.1, 5.2): sphere of radius rho = 2.5R about the centre of B,
    n_gamma Fibonacci points, n_gamma = max(64, 2 (p+1)^2) with
    p = ceil(log(1/eps) / log(rho/r_B)) + ceil(k 2 r_B), r_B = (sqrt 3 / 2) R. Proxy rows
    carry the L2 weight s = sqrt(4 pi rho^2 / n_gamma).
  * Outgoing proxy rows s K(y_l, x_j) sqrt(w_j) (source normal n_j); incoming proxy rows
    s G(x_j, y_l) sqrt(w_j) (single layer only, Section 5.1.2). Transposes are plain,
    not conjugate (Section 4.1, eq. proxy-split-1).
  * DOF order inside a box: tree order (the octree's point order); near DOFs listed
    owner by owner in tree order.
  * Quadrature corrections (Section 5.3, optional): target-dependent weights w_ij =
    w_j (1 + a_ij) for listed pairs make those entries differ from kernel values. An owner
    that would lie in B's P region but is linked to B's active DOFs by a listed pair (either
    direction) joins Q: its rows enter the ID explicitly instead of through the proxy
    surface, which represents kernel values only (spill-over). Such owners are never
    Schur-updated together with B (updates pair only owners next to a common box), so their
    blocks are still the corrected kernel values.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np
import scipy.linalg as sla

from . import dense, kernel
from .idqr import cpqr, interp_decomp
from .tree import Tree, morton

PROXY_RADIUS = 2.5


def fibonacci_dirs(n):
    """Unit vectors z_i = 1 - (2i+1)/n, phi_i = i pi (3 - sqrt 5)."""
    i = np.arange(n, dtype=np.float64)
    z = 1.0 - (2.0 * i + 1.0) / n
    phi = i * (math.pi * (3.0 - math.sqrt(5.0)))
    r = np.sqrt(np.maximum(0.0, 1.0 - z * z))
    return np.stack([r * np.cos(phi), r * np.sin(phi), z])


def proxy_count(side, k, eps):
    """n_gamma for a box of side R (reading of Section 5.2's multipole estimate)."""
    ratio = PROXY_RADIUS / (math.sqrt(3.0) / 2.0)
    p = math.ceil(math.log(1.0 / eps) / math.log(ratio)) + math.ceil(k * math.sqrt(3.0) * side)
    return max(64, 2 * (p + 1) ** 2)


def proxy_block(x, nrm, w, k, eta, eps, ctr, side, idx):
    """Proxy rows for the DOFs idx of a box with centre ctr and side `side` (Sections 5.1.1-
    5.1.3): on n_gamma Fibonacci points y_l of the sphere of radius 2.5 side about ctr,
    outgoing rows s K(y_l, x_j) sqrt(w_j) (source normal n_j) and incoming rows
    s G(x_j, y_l) sqrt(w_j), s = sqrt(4 pi rho^2 / n_gamma). Returns (pout, pin, n_gamma)."""
    rho = PROXY_RADIUS * side
    ng = proxy_count(side, k, eps)
    y = np.asarray(ctr, dtype=np.float64)[:, None] + rho * fibonacci_dirs(ng)
    sg = math.sqrt(4.0 * math.pi * rho * rho / ng)
    xb, nb, swb = x[:, idx], nrm[:, idx], np.sqrt(w[idx])
    pout = sg * kernel.cfie(y, xb, nb, k, eta) * swb[None, :]
    pin = sg * kernel.green(y, xb, k) * swb[None, :]
    return pout, pin, ng


def colour(c):
    return int(c[0] & 1) + 2 * int(c[1] & 1) + 4 * int(c[2] & 1)


@dataclass
class BoxFactor:
    """Factors of one eliminated box. Column (outgoing) sets R, S, N with T, and row
    (incoming) sets Rr, Sr, Nr with Tr; with shared skeletons the row sets are the column
    sets and Tr is T."""
    level: int
    box: int
    coord: tuple
    R: np.ndarray      # redundant column DOFs (global indices), in ID pivot order
    S: np.ndarray      # skeleton column DOFs, in ID pivot order
    N: np.ndarray      # near column DOFs
    T: np.ndarray      # s x r interpolation matrix of the columns: A_{F R} ~ A_{F S} T
    XRR: np.ndarray    # pivot block X_{Rr R}
    lu: tuple          # LU of XRR (scipy lu_factor)
    Lp: np.ndarray     # X_{(Sr u Nr) R} X_RR^{-1}
    Up: np.ndarray     # X_RR^{-1} X_{Rr (S u N)}
    m: int
    nq: int
    ngamma: int
    margins: dict = None  # decision margins of the box's CPQR (idqr.cpqr)
    Q: np.ndarray = None  # DOFs of the Q region (rows of the ID matrix's first two blocks)
    M: np.ndarray = None  # the ID matrix itself (kept only with keep_id=True)
    cols: np.ndarray = None  # the box's active DOFs: the ID matrix's columns, in order
    Rr: np.ndarray = None  # row sets and row interpolation matrix: A_{Rr F} ~ Tr^T A_{Sr F}
    Sr: np.ndarray = None
    Nr: np.ndarray = None
    Tr: np.ndarray = None
    margins_r: dict = None

    def __post_init__(self):
        if self.Rr is None:
            self.Rr, self.Sr, self.Nr, self.Tr = self.R, self.S, self.N, self.T

    @property
    def SN(self):
        return np.concatenate([self.S, self.N])

    @property
    def SNr(self):
        return np.concatenate([self.Sr, self.Nr])


def _id_at_rank(M, eps, s):
    """Greedy CPQR ID of M's columns at rank s (at least its own eps-rank): positions of the
    skeleton and redundant columns, T = R11^{-1} R12, and the decision margins."""
    piv, R, s0, mg = cpqr(M, eps, margins=True)
    if s0 < s:
        piv, R, s0 = cpqr(M, 0.0, max_rank=s)
    S, Rd = piv[:s].copy(), piv[s:].copy()
    T = sla.solve_triangular(R[:s, :s], R[:s, s:M.shape[1]], lower=False) if s else \
        np.zeros((0, M.shape[1]), dtype=np.complex128)
    return S, Rd, T, mg


class RSSFactor:
    """Dense-bookkeeping RS-S factorization of A~ (see module docstring)."""

    def __init__(self, x, nrm, w, k, eta, eps, leaf_size=64, check_invariant=False,
                 brute_force_check=False, use_proxy=True, schedule="sequential", keep_id=False,
                 separate=False, corr=None, spill=True):
        if schedule not in ("sequential", "phase_start"):
            raise ValueError(schedule)
        self.schedule = schedule
        self.separate = bool(separate)
        self.x = np.asarray(x, dtype=np.float64)
        self.nrm = np.asarray(nrm, dtype=np.float64)
        self.w = np.asarray(w, dtype=np.float64)
        self.k, self.eta, self.eps = float(k), float(eta), float(eps)
        self.n = self.x.shape[1]
        self.tree = Tree(self.x, leaf_size)
        A = dense.system_matrix(self.x, self.nrm, self.w, k, eta, corr=corr)
        # Section 5.3: DOFs linked by a quadrature correction (either direction); an owner box
        # linked to B that would lie in B's P region joins Q instead (spill-over)
        self.partners = None
        if corr is not None:
            row_ptr, ccol, _ = corr
            links = [set() for _ in range(self.n)]
            for i in range(self.n):
                for e in range(int(row_ptr[i]), int(row_ptr[i + 1])):
                    j = int(ccol[e])
                    if j != i:
                        links[i].add(j)
                        links[j].add(i)
            self.partners = [np.array(sorted(v), dtype=np.int64) for v in links]
        self.spill = bool(spill)
        self.spill_count = 0
        self.A0 = A.copy() if (check_invariant or brute_force_check) else None
        self.factors: list[BoxFactor] = []
        self.level_stats = []
        self.bf_errors = []
        self.invariant_checked = 0
        # active rows and columns (equal as long as skeletons are shared)
        act_r = np.ones(self.n, dtype=bool)
        act_c = np.ones(self.n, dtype=bool)
        t = self.tree
        rank = t.rank
        for lev in range(t.nlevels - 1, 1, -1):
            anc = self._owner_map(lev)
            owner = anc[t.point_leaf]
            processed = sorted(
                {int(owner[i]) for i in np.nonzero(act_r)[0] if t.level[owner[i]] == lev},
                key=lambda b: (colour(t.coord[b]), int(morton(*t.coord[b]))))
            nproc = 0
            phase_colour, frozen = None, None
            for B in processed:
                if colour(t.coord[B]) != phase_colour:
                    phase_colour, frozen = colour(t.coord[B]), (act_r.copy(), act_c.copy())
                ar, ac = frozen if schedule == "phase_start" else (act_r, act_c)
                rows, cols = np.nonzero(ar)[0], np.nonzero(ac)[0]
                own_r, own_c = owner[rows], owner[cols]
                ob = np.unique(own_r)  # owners holding active DOFs (the same for columns)
                gaps = self._gaps(lev, t.coord[B], ob)
                near_owners = [int(o) for o, g in zip(ob, gaps) if g == 0 and o != B]
                q_owners = [int(o) for o, g in zip(ob, gaps) if g == 1]
                p_owners = [int(o) for o, g in zip(ob, gaps) if g >= 2]
                if self.partners is not None and self.spill and p_owners:
                    mine = np.nonzero((owner == B) & (ar | ac))[0]
                    linked = np.unique(np.concatenate([self.partners[d] for d in mine])) if mine.size else mine
                    linked = linked[ar[linked] | ac[linked]]
                    lo = set(int(o) for o in owner[linked])
                    spill_owners = [o for o in p_owners if o in lo]
                    if spill_owners:
                        self.spill_count += len(spill_owners)
                        q_owners += spill_owners
                        p_owners = [o for o in p_owners if o not in lo]
                p_any = bool(p_owners)
                key = lambda o: rank[t.pts[o]].min() if t.pts[o].size else 0  # noqa: E731
                near_owners.sort(key=key)
                q_owners.sort(key=key)

                def gather(idx, own, owners):
                    return (np.concatenate([self._sorted(idx[own == o], rank) for o in owners])
                            if owners else np.zeros(0, np.int64))
                idxB_r, idxB_c = self._sorted(rows[own_r == B], rank), self._sorted(cols[own_c == B], rank)
                idxN_r, idxN_c = gather(rows, own_r, near_owners), gather(cols, own_c, near_owners)
                idxQ_r, idxQ_c = gather(rows, own_r, q_owners), gather(cols, own_c, q_owners)
                idxP_r, idxP_c = rows[np.isin(own_r, p_owners)], cols[np.isin(own_c, p_owners)]
                if idxQ_r.size == 0 and not p_any:
                    continue
                if check_invariant and idxP_r.size:
                    ok = (np.array_equal(A[np.ix_(idxP_r, idxB_c)], self.A0[np.ix_(idxP_r, idxB_c)])
                          and np.array_equal(A[np.ix_(idxB_r, idxP_c)], self.A0[np.ix_(idxB_r, idxP_c)]))
                    if not ok:
                        raise AssertionError(f"far-field block of box {B} was modified")
                    if self.partners is not None and self.spill:
                        mineB = np.concatenate([idxB_r, idxB_c])
                        far = set(np.concatenate([idxP_r, idxP_c]).tolist())
                        if any(int(p_) in far for d in mineB for p_ in self.partners[d]):
                            raise AssertionError(f"a quadrature correction links box {B} to its P region")
                    self.invariant_checked += 1
                # outgoing blocks (columns of B) and incoming blocks (rows of B, transposed)
                out_blk, in_blk = [], []
                if idxQ_r.size:
                    out_blk.append(A[np.ix_(idxQ_r, idxB_c)])
                    in_blk.append(A[np.ix_(idxB_r, idxQ_c)].T)
                ng = 0
                if p_any and use_proxy:
                    pout, _, ng = self.proxy_rows(B, idxB_c)
                    _, pin, _ = self.proxy_rows(B, idxB_r)
                    out_blk.append(pout)
                    in_blk.append(pin)
                elif p_any:
                    out_blk.append(A[np.ix_(idxP_r, idxB_c)])
                    in_blk.append(A[np.ix_(idxB_r, idxP_c)].T)
                if not self.separate:
                    # one ID of the stacked matrix [A_QB ; A_BQ^T ; proxy out ; proxy in]
                    # (the incoming block's columns are B's rows: the same DOFs here)
                    M = np.vstack(out_blk[:1] + in_blk[:1] + out_blk[1:] + in_blk[1:])
                    Spos, Rpos, T, margins = interp_decomp(M, self.eps, margins=True)
                    Spos_r, Rpos_r, Tr, margins_r = Spos, Rpos, T, margins
                else:
                    # separate IDs of the outgoing and incoming blocks, at a common rank (the
                    # larger of the two eps-ranks) so that the pivot block is square
                    Mo, Mi = np.vstack(out_blk), np.vstack(in_blk)
                    s_o = cpqr(Mo, self.eps)[2]
                    s_i = cpqr(Mi, self.eps)[2]
                    srank = max(s_o, s_i)
                    Spos, Rpos, T, margins = _id_at_rank(Mo, self.eps, srank)
                    Spos_r, Rpos_r, Tr, margins_r = _id_at_rank(Mi, self.eps, srank)
                    M = Mo
                if brute_force_check and idxP_r.size:
                    F_r, F_c = np.concatenate([idxQ_r, idxP_r]), np.concatenate([idxQ_c, idxP_c])
                    fo = A[np.ix_(F_r, idxB_c)]
                    fi = A[np.ix_(idxB_r, F_c)].T
                    errs = []
                    for full, S_, R_, T_ in ((fo, Spos, Rpos, T), (fi, Spos_r, Rpos_r, Tr)):
                        e = np.linalg.norm(full[:, R_] - full[:, S_] @ T_, 2) if R_.size else 0.0
                        errs.append(e / np.linalg.norm(full, 2))
                    self.bf_errors.append((B, max(errs), Spos.size, idxB_c.size))
                nproc += 1
                if Rpos.size == 0:
                    continue
                f = self._eliminate(A, lev, B, idxB_r[Rpos_r], idxB_r[Spos_r], idxN_r, Tr,
                                    idxB_c[Rpos], idxB_c[Spos], idxN_c, T, ng)
                f.nq = int(idxQ_r.size)
                f.margins, f.margins_r = margins, margins_r
                f.Q = idxQ_c
                f.cols = idxB_c
                if keep_id:
                    f.M = M
                self.factors.append(f)
                act_r[f.Rr] = False
                act_c[f.R] = False
            self.level_stats.append((lev, nproc, int(act_r.sum())))
        self.top_r = self._sorted(np.nonzero(act_r)[0], rank)
        self.top = self._sorted(np.nonzero(act_c)[0], rank)
        self.Att = A[np.ix_(self.top_r, self.top)].copy()
        self.top_lu = sla.lu_factor(self.Att, check_finite=False)
        self.A = A

    # -- helpers ----------------------------------------------------------------------
    @staticmethod
    def _sorted(idx, rank):
        return idx[np.argsort(rank[idx], kind="stable")]

    def _owner_map(self, lev):
        """For every box id: the level-`lev` ancestor of a box at level >= lev; itself
        otherwise (used on leaves only)."""
        t = self.tree
        nb = len(t.level)
        anc = np.arange(nb)
        for b in range(nb):
            a = b
            while t.level[a] > lev:
                a = t.parent[a]
            anc[b] = a
        return anc

    def _gaps(self, lev, c, owners):
        t = self.tree
        lv = t.level[owners]
        sh = (lev - lv)
        lo = t.coord[owners] << sh[:, None]
        hi = (t.coord[owners] + 1) << sh[:, None]
        c = np.asarray(c)
        g = np.maximum(lo - (c + 1), c - hi).max(axis=1)
        return np.maximum(g, 0)

    def proxy_rows(self, B, idxB):
        """Outgoing and incoming proxy blocks of box B (Section 5.1.1-5.1.3)."""
        t = self.tree
        return proxy_block(self.x, self.nrm, self.w, self.k, self.eta, self.eps, t.box_centre(B),
                           t.box_side(B), idxB)

    def _eliminate(self, A, lev, B, Rr, Sr, Nr, Tr, R, S, N, T, ng):
        """Section 4.1: row transform E with Tr on rows (Rr, Sr), column transform F with T on
        columns (R, S), then L, U with the pivot block X_{Rr R}; the Schur complement is
        subtracted from A_{(Sr u Nr)(S u N)} in place. With shared skeletons the row and
        column sets coincide."""
        Ttr = Tr.T
        A_RR, A_RS = A[np.ix_(Rr, R)], A[np.ix_(Rr, S)]
        A_SR, A_SS = A[np.ix_(Sr, R)], A[np.ix_(Sr, S)]
        A_RN, A_SN = A[np.ix_(Rr, N)], A[np.ix_(Sr, N)]
        A_NR, A_NS = A[np.ix_(Nr, R)], A[np.ix_(Nr, S)]
        XRR = A_RR - Ttr @ A_SR - A_RS @ T + Ttr @ A_SS @ T
        XRS = A_RS - Ttr @ A_SS
        XSR = A_SR - A_SS @ T
        XRN = A_RN - Ttr @ A_SN
        XNR = A_NR - A_NS @ T
        XR_SN = np.hstack([XRS, XRN])
        XSN_R = np.vstack([XSR, XNR])
        lu = sla.lu_factor(XRR, check_finite=False)
        if np.any(np.diag(lu[0]) == 0):
            raise np.linalg.LinAlgError(f"singular pivot block at box {B}")
        Up = sla.lu_solve(lu, XR_SN, check_finite=False)
        Lp = sla.lu_solve(lu, XSN_R.T, trans=1, check_finite=False).T
        SNr, SN = np.concatenate([Sr, Nr]), np.concatenate([S, N])
        A[np.ix_(SNr, SN)] -= XSN_R @ Up
        return BoxFactor(lev, B, tuple(int(v) for v in self.tree.coord[B]), R, S, N, T, XRR, lu,
                         Lp, Up, R.size + S.size, 0, ng, Rr=Rr, Sr=Sr, Nr=Nr, Tr=Tr)

    # -- application of the factors (Section 4.2) ----------------------------------------
    def solve(self, b):
        """x = A_f^{-1} b: V_1^{-1} ... V_M^{-1} in box order (E then L, on the row sets),
        D^{-1} (rows Rr to columns R, and the top block), then W_M^{-1} ... W_1^{-1} in reverse
        order (U then F, on the column sets)."""
        y = np.array(b, dtype=np.complex128, copy=True)
        for f in self.factors:
            y[f.Rr] -= f.Tr.T @ y[f.Sr]
            y[f.SNr] -= f.Lp @ y[f.Rr]
        x = np.zeros_like(y)
        for f in self.factors:
            x[f.R] = sla.lu_solve(f.lu, y[f.Rr], check_finite=False)
        x[self.top] = sla.lu_solve(self.top_lu, y[self.top_r], check_finite=False)
        for f in reversed(self.factors):
            x[f.R] -= f.Up @ x[f.SN]
            x[f.S] -= f.T @ x[f.R]
        return x

    def solve_adjoint(self, b):
        """x = A_f^{-H} b = V_1^{-H} ... V_M^{-H} D^{-H} W_M^{-H} ... W_1^{-H} b."""
        y = np.array(b, dtype=np.complex128, copy=True)
        for f in self.factors:
            y[f.R] -= f.T.conj().T @ y[f.S]
            y[f.SN] -= f.Up.conj().T @ y[f.R]
        x = np.zeros_like(y)
        for f in self.factors:
            x[f.Rr] = sla.lu_solve(f.lu, y[f.R], trans=2, check_finite=False)
        x[self.top_r] = sla.lu_solve(self.top_lu, y[self.top], trans=2, check_finite=False)
        for f in reversed(self.factors):
            x[f.Rr] -= f.Lp.conj().T @ x[f.SNr]
            x[f.Sr] -= f.Tr.conj() @ x[f.Rr]
        return x

    def apply(self, v):
        """A_f v = V_1 ... V_M D W_M ... W_1 v (the factored approximation of A~)."""
        x = np.array(v, dtype=np.complex128, copy=True)
        for f in self.factors:
            x[f.S] += f.T @ x[f.R]
            x[f.R] += f.Up @ x[f.SN]
        y = np.zeros_like(x)
        for f in self.factors:
            y[f.Rr] = f.XRR @ x[f.R]
        y[self.top_r] = self.Att @ x[self.top]
        for f in reversed(self.factors):
            y[f.SNr] += f.Lp @ y[f.Rr]
            y[f.Rr] += f.Tr.T @ y[f.Sr]
        return y

    @property
    def n0(self):
        return int(self.top.size)

    def factor_entries(self):
        """Stored complex entries (T, X_RR, L and U panels, top block)."""
        tot = self.top.size ** 2
        for f in self.factors:
            tot += f.T.size + f.XRR.size + f.Lp.size + f.Up.size + (f.Tr.size if f.Tr is not f.T else 0)
        return tot
