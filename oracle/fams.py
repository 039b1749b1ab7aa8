"""Oracle: F-AMS basis functions, coarse system, ILU(0) and the iteration.

Test infrastructure only (see the package docstring).  FP64 throughout,
single-threaded apart from what numpy/scipy do inside library primitives
(sparse products, dense solves, LU factorisation).

The prolongation follows App. A of the paper.  Writing its four block
formulas (Decoupled, Frac, Rock and Coupled-AMS) in one rule:

* every cell gets a rank rho(i): its wirebasket class tau (I=0 < F=1 < E=2 <
  V=3), lifted by 4 for the medium whose basis functions are computed first
  and then act as Dirichlet data for the other (fractures in Frac-AMS,
  App. A.2; the matrix in Rock-AMS, App. A.3);
* in a non-vertex row i a coupling A_ij is
    - "cut" when it crosses media in Decoupled-AMS (App. A.1: A^mf = A^fm = 0),
      or when it crosses media between same-class blocks that were not
      merged in Coupled-AMS (merge-size limit, Sec. 3.1);
    - "lumped" (removed and added to the diagonal -- the over/underlined
      diagonal blocks of App. A) when cut or when
      rho(j) < rho(i) (the localisation assumption, Sec. 3.1);
    - a right-hand-side term -A_ij P_j when rho(j) > rho(i) (the higher-rank
      sub-blocks of P act as boundary conditions, App. A.1);
    - kept when rho(j) = rho(i) and not cut;
* the local blocks are the connected components of the kept couplings (the
  dual edges, faces and interiors, merged across media in Coupled-AMS); they
  are solved from the highest rank down: P_K = A'_KK^{-1} B_K;
* vertex rows are the Kronecker delta of Eq. (kronecker-basis);
* wells (the last n_wells unknowns, Sec. 3: one fine-scale unknown and one
  coarse node per well, mapped by the identity) are vertices of a third
  medium ranked above every cell (rho = 8): a perforated cell's coupling to
  its well is never cut or lumped but taken as Dirichlet data, which is the
  beta (Phi - Phi^w) term of the skeleton equation (Sec. 3.1) with
  P^ww = I and P^wm = P^wf = 0 (Eq. prolongation_single).

Readings where the paper is silent (listed in the design notes):
  * Coupled-AMS merging (Sec. 3.1: neighbouring dual blocks of one type join
    across media, with an optional cap on merged size): first the within-medium
    blocks; then cross-media couplings between cells of the same class are
    visited in CSR order (i < j) and the two blocks are united unless the
    union would exceed ``merge_cap`` cells -- a rejected coupling is cut;
  * truncation (Sec. 4.3): in a non-vertex row, entries with |P_ij| < alpha
    are dropped and the survivors rescaled so the row keeps the sum it had
    before truncation (its partition-of-unity value); if nothing survives the
    largest entry (lowest column on ties) is kept; rows that lose nothing are
    left untouched;
  * restriction in the iteration: R = P^T (MSFE, the paper's choice for all of
    its experiments, Sec. 3) by default; MSFV (row i of R has a 1 on every
    cell of primal block i, Sec. 3.2) and MSMIX (Sec. 3 and 3.2: FV for the
    fractures, FE for the rock -- read as: the MSFV row for a coarse node whose
    vertex is a fracture cell, the MSFE row for a matrix one) on request; the
    coarse operator is then R A P with the same R;
  * the extra smoothing stage on the per-medium systems (Sec. 3.2 names it
    and leaves it to future work), on request: after the ILU(0) stage, one
    ILU(0) application of diag(A^mm, A^ff) to the updated residual;
  * GMRES: right preconditioned, restarted, modified Gram-Schmidt, the
    F-AMS two-stage step as preconditioner (Sec. 4.6), stopping on the true
    relative residual ||q - A p|| / ||q|| (p0 = 0).
"""
from __future__ import annotations

import ctypes

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp
from scipy.sparse.csgraph import connected_components

from . import _cbuild

DECOUPLED, FRAC, ROCK, COUPLED = 0, 1, 2, 3
VARIANTS = {"decoupled": DECOUPLED, "frac": FRAC, "rock": ROCK, "coupled": COUPLED}
KEPT, LUMPED, RHS = 1, 2, 3
OK, NOT_CONVERGED, DIVERGED = 0, 1, 2
RESTRICT_FE, RESTRICT_FV, RESTRICT_MIX = 0, 1, 2


def media(n, n_matrix, n_wells=0):
    """Medium of every unknown: 0 matrix, 1 fracture, 2 well (the last
    n_wells unknowns are well pressures)."""
    med = (np.arange(n) >= n_matrix).astype(np.int64)
    if n_wells:
        med[n - n_wells:] = 2
    return med


def ranks(wb_type, n_matrix, variant, n_wells=0):
    """rho(i) of every cell (see the module docstring).  A well is a coarse
    node of its own (Sec. 3: one coarse node per well, identity restriction)
    above every cell of both media, so the cells it perforates take it as
    Dirichlet data in every strategy (the well term of the skeleton equation
    of Sec. 3.1)."""
    tau = np.asarray(wb_type, dtype=np.int64)
    med = media(len(tau), n_matrix, n_wells)
    frac = med == 1
    if variant == FRAC:
        rho = tau + 4 * frac
    elif variant == ROCK:
        rho = tau + 4 * (med == 0)
    else:
        rho = tau.copy()
    rho[med == 2] = 8
    return rho


def _union_find_merge(rows, cols, base, sizes, cap):
    """Coupled-AMS merge: visit (i, j) in the given order; unite the blocks of i
    and j unless the union would exceed cap cells."""
    parent = np.arange(len(sizes))
    size = sizes.astype(np.int64).copy()

    def find(a):
        while parent[a] != a:
            parent[a] = parent[parent[a]]
            a = parent[a]
        return a

    for i, j in zip(rows, cols):
        a, b = find(base[i]), find(base[j])
        if a == b:
            continue
        if size[a] + size[b] <= cap:
            lo, hi = (a, b) if a < b else (b, a)
            parent[hi] = lo
            size[lo] += size[hi]
    return np.array([find(x) for x in range(len(sizes))])


def classify(A: sp.csr_matrix, wb_type, n_matrix, variant, merge_cap=4096, n_wells=0):
    """Class of every stored entry of A (0 for diagonals and vertex rows) and the
    local block (component) of every non-vertex cell (-1 for vertices)."""
    n = A.shape[0]
    rho = ranks(wb_type, n_matrix, variant, n_wells)
    tau = np.asarray(wb_type, dtype=np.int64)
    is_v = tau == 3
    med = media(n, n_matrix, n_wells)
    r = np.repeat(np.arange(n), np.diff(A.indptr))
    c = A.indices.astype(np.int64)
    off = (r != c) & ~is_v[r]
    cut = np.zeros(len(c), dtype=bool)
    if variant == DECOUPLED:   # matrix-fracture couplings only; wells are never cut
        cut = (med[r] != med[c]) & (med[r] < 2) & (med[c] < 2)
    elif variant == COUPLED:
        # within-medium blocks first
        same = off & ~is_v[c] & (tau[r] == tau[c]) & (med[r] == med[c])
        g = sp.csr_matrix((np.ones(same.sum()), (r[same], c[same])), shape=(n, n))
        nb, base = connected_components(g, directed=False)
        sizes = np.bincount(base, minlength=nb)
        cross = off & ~is_v[c] & (tau[r] == tau[c]) & (med[r] != med[c]) & (r < c)
        root = _union_find_merge(r[cross], c[cross], base, sizes, merge_cap)
        group = root[base]
        cut = (med[r] != med[c]) & (tau[r] == tau[c]) & (group[r] != group[c])
    cls = np.zeros(len(c), dtype=np.int8)
    lumped = off & (cut | (rho[c] < rho[r]))
    rhs = off & ~cut & (rho[c] > rho[r])
    kept = off & ~cut & (rho[c] == rho[r])
    cls[lumped] = LUMPED
    cls[rhs] = RHS
    cls[kept] = KEPT
    g = sp.csr_matrix((np.ones(kept.sum()), (r[kept], c[kept])), shape=(n, n))
    _, lab = connected_components(g, directed=False)
    comp = np.where(is_v, -1, lab)
    return cls, comp, rho


def _masked(A, mask):
    B = A.copy()
    B.data = np.where(mask, A.data, 0.0)
    B.eliminate_zeros()
    return B


def prolongation(A, wb_type, vertex, n_matrix, variant, alpha=0.0, merge_cap=4096,
                 return_blocks=False, n_wells=0):
    """The F-AMS prolongation P (N x n_c, CSR) for one coupling strategy."""
    A = sp.csr_matrix(A)
    A.sort_indices()
    n = A.shape[0]
    nc = len(vertex)
    if n_wells and np.any(np.asarray(wb_type)[n - n_wells:] != 3):
        raise ValueError("every well is a coarse node (class 3)")
    cls, comp, rho = classify(A, wb_type, n_matrix, variant, merge_cap, n_wells)
    is_v = np.asarray(wb_type) == 3
    coarse_of = np.full(n, -1, dtype=np.int64)
    coarse_of[np.asarray(vertex)] = np.arange(nc)
    if np.any(coarse_of[is_v] < 0) or np.any(np.asarray(wb_type)[np.asarray(vertex)] != 3):
        raise ValueError("vertex list and V cells disagree")
    A_keep = _masked(A, cls == KEPT)
    A_lump = _masked(A, cls == LUMPED)
    A_rhs = _masked(A, cls == RHS)
    dprime = A.diagonal() + np.asarray(A_lump.sum(axis=1)).ravel()

    row_cols = [None] * n
    row_vals = [None] * n
    for i in np.nonzero(is_v)[0]:
        row_cols[i] = np.array([coarse_of[i]])
        row_vals[i] = np.array([1.0])

    def current_P():
        lens = np.array([0 if rc is None else len(rc) for rc in row_cols])
        ptr = np.concatenate([[0], np.cumsum(lens)])
        cc = [rc for rc in row_cols if rc is not None]
        vv = [rv for rv in row_vals if rv is not None]
        cols = np.concatenate(cc) if cc else np.zeros(0, np.int64)
        vals = np.concatenate(vv) if vv else np.zeros(0)
        return sp.csr_matrix((vals, cols, ptr), shape=(n, nc))

    blocks = []
    for level in sorted(set(rho[~is_v].tolist()), reverse=True):
        cells = np.nonzero((rho == level) & ~is_v)[0]
        Pk = current_P()
        B = -(A_rhs[cells] @ Pk)
        B = sp.csr_matrix(B)
        pos = {int(c): k for k, c in enumerate(cells)}
        for K in np.unique(comp[cells]):
            idx = cells[comp[cells] == K]
            rows = [pos[int(i)] for i in idx]
            BK = B[rows]
            cols = np.unique(BK.indices)
            if len(cols) == 0:
                raise ValueError(f"local block with cells {idx[:5]}... has no higher-rank "
                                 "neighbour (singular local problem)")
            M = A_keep[idx][:, idx].toarray() + np.diag(dprime[idx])
            X = np.linalg.solve(M, BK[:, cols].toarray())
            for a, i in enumerate(idx):
                row_cols[i] = cols.astype(np.int64)
                row_vals[i] = X[a]
            blocks.append((level, idx))
    P = current_P()
    P.sort_indices()
    if alpha > 0:
        P = truncate(P, alpha, is_v)
    if return_blocks:
        return P, dict(cls=cls, comp=comp, rho=rho, blocks=blocks, dprime=dprime)
    return P


def truncate(P, alpha, is_vertex_row):
    """Drop |P_ij| < alpha in non-vertex rows; rescale to the row's prior sum."""
    P = sp.csr_matrix(P)
    ptr, cols, vals = P.indptr, P.indices, P.data
    nc_, nv_, np_ = [], [], [0]
    for i in range(P.shape[0]):
        c, v = cols[ptr[i]:ptr[i + 1]], vals[ptr[i]:ptr[i + 1]]
        if not is_vertex_row[i] and len(v):
            keep = np.abs(v) >= alpha
            if not keep.any():
                keep = np.zeros(len(v), dtype=bool)
                keep[int(np.argmax(np.abs(v)))] = True
            if not keep.all():
                s0 = float(np.sum(v))
                s1 = float(np.sum(v[keep]))
                c, v = c[keep], v[keep]
                if s1 != 0.0:
                    v = v * (s0 / s1)
        nc_.append(c)
        nv_.append(v)
        np_.append(np_[-1] + len(c))
    return sp.csr_matrix((np.concatenate(nv_), np.concatenate(nc_), np.array(np_)),
                         shape=P.shape)


def restriction(P, primal, vertex, n_matrix, kind=RESTRICT_FE):
    """The restriction operator R (Sec. 3.2): MSFE R = P^T; MSFV R[i, j] = 1
    when cell j lies in primal block i; MSMIX the MSFV row for a coarse node
    whose vertex is a fracture cell and the MSFE row otherwise."""
    RT = sp.csr_matrix(P.T)
    if kind == RESTRICT_FE:
        return RT
    primal = np.asarray(primal, dtype=np.int64)
    nc, n = RT.shape
    RFV = sp.csr_matrix((np.ones(n), (primal, np.arange(n))), shape=(nc, n))
    if kind == RESTRICT_FV:
        return RFV
    frac = np.asarray(vertex, dtype=np.int64) >= n_matrix
    pick = sp.diags(frac.astype(np.float64))
    return sp.csr_matrix(pick @ RFV + (sp.identity(nc) - pick) @ RT)


def media_blocks(A, n_matrix, n_wells=0):
    """diag(A^mm, A^ff) of Eq. (dis-mf): A without the couplings A^mf, A^fm
    between matrix cells (rows [0, n_matrix)) and fracture cells (and, with
    wells, without the couplings between wells and cells)."""
    A = sp.coo_matrix(A)
    med = media(A.shape[0], n_matrix, n_wells)
    keep = med[A.row] == med[A.col]
    return sp.csr_matrix((A.data[keep], (A.row[keep], A.col[keep])), shape=A.shape)


def coarse_operator(A, P, R=None):
    """A_c = R A P as a dense matrix (R = P^T unless given)."""
    if R is None:
        R = P.T
    return np.asarray((R @ (A @ P)).todense())


class ILU0:
    """ILU(0) of A in its given row order (plain C, see ilu0.c)."""

    def __init__(self, A):
        A = sp.csr_matrix(A)
        A.sort_indices()
        self.n = A.shape[0]
        self.rp = np.ascontiguousarray(A.indptr, dtype=np.int64)
        self.ci = np.ascontiguousarray(A.indices, dtype=np.int32)
        self.val = np.ascontiguousarray(A.data, dtype=np.float64).copy()
        self.diag = np.zeros(self.n, dtype=np.int64)
        rc = _cbuild.lib().oracle_ilu0_factor(self.n, self.rp.ctypes.data, self.ci.ctypes.data,
                                             self.val.ctypes.data, self.diag.ctypes.data)
        if rc != 0:
            raise ZeroDivisionError(f"ILU(0): non-positive pivot in row {-rc - 1}")

    def solve(self, b):
        b = np.ascontiguousarray(b, dtype=np.float64)
        x = np.empty_like(b)
        _cbuild.lib().oracle_ilu0_solve(self.n, self.rp.ctypes.data, self.ci.ctypes.data,
                                        self.val.ctypes.data, self.diag.ctypes.data,
                                        b.ctypes.data, x.ctypes.data)
        return x

    def factors(self):
        """(L unit lower, U upper) as CSR matrices."""
        M = sp.csr_matrix((self.val, self.ci, self.rp), shape=(self.n, self.n))
        L = sp.tril(M, -1).tocsr() + sp.identity(self.n, format="csr")
        U = sp.triu(M).tocsr()
        return L, U


class FAMS:
    """Setup (basis functions, coarse LU, ILU(0)) and the iteration."""

    def __init__(self, A, wb_type, vertex, n_matrix, variant=DECOUPLED, alpha=0.0,
                 merge_cap=4096, smoothing=True, primal=None, restriction_kind=RESTRICT_FE,
                 media_smoothing=False, n_wells=0):
        self.A = sp.csr_matrix(A)
        self.A.sort_indices()
        self.n_matrix = n_matrix
        self.n_wells = n_wells
        self.variant = variant
        if restriction_kind != RESTRICT_FE and primal is None:
            raise ValueError("the MSFV and MSMIX restrictions need the primal blocks")
        self._grid = (wb_type, vertex, primal)
        self._opts = (alpha, merge_cap, restriction_kind, smoothing, media_smoothing)
        self._basis()
        self._operators()

    def _basis(self):
        """P (and R) from the current A; remembers the values they follow."""
        wb_type, vertex, primal = self._grid
        alpha, merge_cap, kind = self._opts[:3]
        self.P = prolongation(self.A, wb_type, vertex, self.n_matrix, self.variant, alpha,
                              merge_cap, n_wells=self.n_wells)
        self.R = restriction(self.P, primal, vertex, self.n_matrix, kind)
        self.A_basis = self.A.copy()

    def _operators(self):
        """A_c = R A P, its LU and the smoothers, from the current A."""
        smoothing, media_smoothing = self._opts[3:]
        self.Ac = coarse_operator(self.A, self.P, self.R)
        self.lu = sla.lu_factor(self.Ac)
        self.ilu = ILU0(self.A) if smoothing else None
        # the extra smoothing stage on the per-medium systems (Sec. 3.2)
        self.ilu_media = (ILU0(media_blocks(self.A, self.n_matrix, self.n_wells))
                          if smoothing and media_smoothing else None)

    def update_values(self, A_new, threshold=0.0):
        """New values of A on the same pattern (Table 1, steps 2 and 4).  The
        basis functions follow only when the largest relative change of an
        entry since they were computed exceeds `threshold` (Sec. 3.1; an
        entry that was zero counts its absolute change); A_c, its LU and the
        smoothers always follow.  Returns True when P was recomputed."""
        A_new = sp.csr_matrix(A_new)
        A_new.sort_indices()
        if not (np.array_equal(A_new.indptr, self.A_basis.indptr)
                and np.array_equal(A_new.indices, self.A_basis.indices)):
            raise ValueError("update_values: the pattern of A changed")
        old, new = self.A_basis.data, A_new.data
        d = np.abs(new - old)
        rel = np.where(old != 0.0, d / np.where(old != 0.0, np.abs(old), 1.0), d)
        change = rel.max() if rel.size else 0.0
        recompute = not (change <= threshold)
        self.A = A_new
        if recompute:
            self._basis()
        self._operators()
        return recompute

    # Table 1, steps 5-7, applied to a residual r: returns dp_{1/2} + dp_{2/2}
    def stage(self, r):
        xc = sla.lu_solve(self.lu, self.R @ r)
        d1 = self.P @ xc
        if self.ilu is None:
            return d1
        r_half = r - self.A @ d1
        d2 = self.ilu.solve(r_half)
        if self.ilu_media is None:
            return d1 + d2
        return d1 + d2 + self.ilu_media.solve(r_half - self.A @ d2)

    def richardson(self, q, rtol=1e-6, max_iter=500, history=False):
        q = np.asarray(q, dtype=np.float64)
        p = np.zeros_like(q)
        r = q.copy()
        r0 = np.linalg.norm(r)
        hist = [r0]
        status, it = NOT_CONVERGED, 0
        if r0 == 0.0:
            status = OK
        while status != OK and it < max_iter:
            p = p + self.stage(r)
            r = q - self.A @ p
            it += 1
            nr = np.linalg.norm(r)
            hist.append(nr)
            if not np.isfinite(nr) or nr > 1e8 * r0:
                status = DIVERGED
                break
            if nr <= rtol * r0:
                status = OK
        info = dict(status=status, iterations=it, rel_residual=hist[-1] / r0 if r0 else 0.0)
        if history:
            info["history"] = np.array(hist)
        return p, info

    def gmres(self, q, rtol=1e-6, restart=30, max_iter=3000, history=False):
        """Right-preconditioned restarted GMRES (modified Gram-Schmidt)."""
        A = self.A
        q = np.asarray(q, dtype=np.float64)
        x = np.zeros_like(q)
        r0 = np.linalg.norm(q)
        tol = rtol * r0
        hist = [r0]
        it = 0
        status = NOT_CONVERGED
        while True:
            r = q - A @ x
            beta = np.linalg.norm(r)
            if beta <= tol:
                status = OK
                break
            if not np.isfinite(beta) or beta > 1e8 * r0:
                status = DIVERGED
                break
            if it >= max_iter:
                break
            m = restart
            V = np.zeros((m + 1, len(q)))
            Z = np.zeros((m, len(q)))
            H = np.zeros((m + 1, m))
            cs, sn = np.zeros(m), np.zeros(m)
            g = np.zeros(m + 1)
            g[0] = beta
            V[0] = r / beta
            k = 0
            for j in range(m):
                Z[j] = self.stage(V[j])
                w = A @ Z[j]
                for i in range(j + 1):
                    H[i, j] = np.dot(w, V[i])
                    w = w - H[i, j] * V[i]
                H[j + 1, j] = np.linalg.norm(w)
                for i in range(j):
                    t = cs[i] * H[i, j] + sn[i] * H[i + 1, j]
                    H[i + 1, j] = -sn[i] * H[i, j] + cs[i] * H[i + 1, j]
                    H[i, j] = t
                den = np.hypot(H[j, j], H[j + 1, j])
                cs[j], sn[j] = (1.0, 0.0) if den == 0 else (H[j, j] / den, H[j + 1, j] / den)
                H[j, j] = cs[j] * H[j, j] + sn[j] * H[j + 1, j]
                H[j + 1, j] = 0.0
                g[j + 1] = -sn[j] * g[j]
                g[j] = cs[j] * g[j]
                it += 1
                k = j + 1
                hist.append(abs(g[j + 1]))
                if abs(g[j + 1]) <= tol or it >= max_iter:
                    break
                hn = np.linalg.norm(w)
                if hn == 0.0:
                    break
                V[j + 1] = w / hn
            y = sla.solve_triangular(H[:k, :k], g[:k])
            x = x + Z[:k].T @ y
        nr = np.linalg.norm(q - A @ x)
        info = dict(status=status, iterations=it, rel_residual=nr / r0 if r0 else 0.0)
        if history:
            info["history"] = np.array(hist)
        return x, info
