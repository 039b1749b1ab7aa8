"""Oracle: finite-volume stage and conservative fine-scale flux reconstruction.

Test infrastructure only (see the package docstring).

The paper states (Sec. 1, Sec. 3, Sec. 3.2, Sec. 4.6) that after any stage
that uses the finite-volume restriction R^FV -- the 0/1 matrix whose row K
marks the fine cells of primal block K -- the fine-scale fluxes can be made
mass conservative, but gives no algorithm.  The reconstruction here
is the standard multiscale finite-volume one the paper cites:

1. FV stage: A_FV = R^FV A P;  x = A_FV^{-1} R^FV (q - A p) (LU with partial
   pivoting plus two steps of iterative refinement against the block
   defects R^FV (q - A p'), the residual written with the fluxes);
   p' = p + P x, so that R^FV (q - A p') = 0: every primal block conserves mass.
2. In each primal block K, a Neumann problem with the fluxes across the
   block boundary taken from p':
       sum_{j in K} T_ij (p''_i - p''_j) + s_i p''_i
           = q_i - sum_{j not in K} T_ij (p'_i - p'_j),   i in K,
   where T_ij = -A_ij and s_i = sum_j A_ij (the Dirichlet boundary term).
   If no cell of K has s_i > 0 the problem is singular but compatible, and
   p'' is pinned to p' at K's coarse node.  A row sum counts as zero when it
   is rounding, |s_i| <= 1e-10 sum_{j != i} |A_ij| (measured against the
   row's own couplings: a weakly coupled boundary cell next to
   high-transmissibility fractures still has a real s_i > 0, and pinning its
   block would leave s_i (p''_i - p'_i) unbalanced at the coarse node).
3. Fluxes F_ij = T_ij (p''_i - p''_j) inside a block and T_ij (p'_i - p'_j)
   across blocks; exchange E_i = s_i p''_i - q_i (boundary flux and sources).
   Each cell then balances: sum_j F_ij + E_i = 0.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp

SINGULAR_ROWSUM = 1e-10   # |s_i| <= this * sum_{j != i} |A_ij| counts as zero


def fv_restriction(primal, n_coarse):
    n = len(primal)
    return sp.csr_matrix((np.ones(n), (np.asarray(primal), np.arange(n))), shape=(n_coarse, n))


def dirichlet_rows(A):
    """Rows with a real (not rounding) row sum s_i: |s_i| > SINGULAR_ROWSUM
    sum_{j != i} |A_ij|."""
    A = sp.csr_matrix(A)
    s = np.asarray(A.sum(axis=1)).ravel()
    offsum = np.asarray(abs(A).sum(axis=1)).ravel() - np.abs(A.diagonal())
    return s > SINGULAR_ROWSUM * offsum


def flux_residual(A, q, p):
    """q - A p written with the fluxes: q_i - s_i p_i + sum_{j != i} A_ij (p_i -
    p_j) (s_i = sum_j A_ij).  Equal to q - A p; rounded relative to the fluxes
    rather than to the products A_ij p_j, which at a high conductivity
    contrast are many orders larger."""
    A = sp.csr_matrix(A)
    n = A.shape[0]
    r = np.repeat(np.arange(n), np.diff(A.indptr))
    c = A.indices
    off = r != c
    s = np.asarray(A.sum(axis=1)).ravel()
    terms = np.where(off, A.data * (p[r] - p[c]), 0.0)
    return q - s * p + np.bincount(r, weights=terms, minlength=n)


def fv_stage(A, P, primal, q, p, refine=2):
    """p' = p + P x with R^FV A p' = R^FV q: x from the LU of A_FV = R^FV A P,
    then `refine` steps of iterative refinement against the block defects
    R^FV (q - A p') (flux form)."""
    A = sp.csr_matrix(A)
    nc = P.shape[1]
    Rfv = fv_restriction(primal, nc)
    Afv = np.asarray((Rfv @ (A @ P)).todense())
    lu = sla.lu_factor(Afv)
    x = sla.lu_solve(lu, Rfv @ flux_residual(A, q, p))
    for _ in range(refine):
        x = x + sla.lu_solve(lu, Rfv @ flux_residual(A, q, p + P @ x))
    return p + P @ x


def reconstruct_flux(A, P, primal, vertex, q, p):
    """Returns (flux in A's CSR slots, diagonal slot = E_i; p'; p''; imbalance)."""
    A = sp.csr_matrix(A)
    A.sort_indices()
    n = A.shape[0]
    primal = np.asarray(primal)
    p1 = fv_stage(A, P, primal, q, p)
    s = np.asarray(A.sum(axis=1)).ravel()
    diag = A.diagonal()
    has_s = dirichlet_rows(A)
    rp, ci, va = A.indptr, A.indices, A.data
    p2 = np.empty(n)
    order = np.argsort(primal, kind="stable")
    bounds = np.searchsorted(primal[order], np.arange(P.shape[1] + 1))
    for K in range(P.shape[1]):
        cells = order[bounds[K]:bounds[K + 1]]
        if len(cells) == 0:
            continue
        loc = {int(c): a for a, c in enumerate(cells)}
        m = len(cells)
        M = np.zeros((m, m))
        b = np.zeros(m)
        for a, i in enumerate(cells):
            b[a] = q[i]
            M[a, a] = diag[i]
            for pp in range(rp[i], rp[i + 1]):
                j = ci[pp]
                if j == i:
                    continue
                if int(j) in loc:
                    M[a, loc[int(j)]] = va[pp]
                else:
                    M[a, a] += va[pp]
                    b[a] += va[pp] * (p1[i] - p1[j])
        if not has_s[cells].any():
            v = loc[int(vertex[K])]
            keep = np.array([a for a in range(m) if a != v], dtype=np.int64)
            sol = np.empty(m)
            sol[v] = p1[vertex[K]]
            if len(keep):
                sol[keep] = np.linalg.solve(M[np.ix_(keep, keep)],
                                            b[keep] - M[keep, v] * sol[v])
        else:
            sol = np.linalg.solve(M, b)
        p2[cells] = sol
    flux = np.empty_like(va)
    r = np.repeat(np.arange(n), np.diff(rp))
    same = primal[r] == primal[ci]
    pv = np.where(same, p2[r] - p2[ci], p1[r] - p1[ci])
    flux[:] = -va * pv
    isdiag = r == ci
    flux[isdiag] = s * p2 - q
    bal = np.bincount(r, weights=flux, minlength=n)
    scale = np.bincount(r, weights=np.abs(flux), minlength=n)
    imbalance = float(np.max(np.abs(bal)) / np.max(scale))
    return flux, p1, p2, imbalance
