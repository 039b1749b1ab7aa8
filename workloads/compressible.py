"""A slightly compressible single-phase model on an EDFM system, for the
Newton loop of Table 1 (steps 1-2: the system's entries are updated every
outer iteration; Eq. dis-mf notes A is non-symmetric with compressibility).

Problem data only: the residual and its Jacobian on the pattern of the
incompressible operator A of a FracturedSystem.  With T_ij = -A_ij (j != i)
and t_i = sum_j A_ij (the Dirichlet boundary transmissibility of row i):

    R_i(p) = a_i (rho(p_i) - rho(p_old_i))
             + sum_{j != i} T_ij rho_ij (p_i - p_j) + rho(p_i) (t_i p_i - q_i),

rho(p) = exp(c p), rho_ij = rho at the upstream cell (the one with the larger
pressure, i on ties), a_i = gamma A_ii (accumulation).  With c = 0 and
gamma = 0 this is A p - q.  Upwinding makes the Jacobian non-symmetric; its
off-diagonals stay non-positive.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla


def _parts(sysm):
    A = sysm.csr()
    A.sort_indices()
    n = A.shape[0]
    r = np.repeat(np.arange(n), np.diff(A.indptr))
    c = A.indices.astype(np.int64)
    off = r != c
    t = np.asarray(A.sum(axis=1)).ravel()
    return A, r, c, off, t


def residual_jacobian(sysm, p, p_old, c=0.2, gamma=0.1, q=None):
    """(R(p), J(p)) with J in CSR on A's pattern (same indptr/indices)."""
    A, r, col, off, t = _parts(sysm)
    q = sysm.q if q is None else q
    rho = np.exp(c * p)
    drho = c * rho
    a = gamma * A.diagonal()
    T = -A.data
    up_i = p[r] >= p[col]                      # upstream is the row's own cell
    rho_ij = np.where(up_i, rho[r], rho[col])
    dp = p[r] - p[col]
    flux = np.where(off, T * rho_ij * dp, 0.0)
    R = a * (rho - np.exp(c * p_old)) + np.bincount(r, weights=flux, minlength=len(p)) \
        + rho * (t * p - q)
    # d flux_ij / d p_j (off-diagonal slots) and d flux_ij / d p_i (summed on the diagonal)
    d_j = T * (-rho_ij + dp * np.where(up_i, 0.0, drho[col]))
    d_i = T * (rho_ij + dp * np.where(up_i, drho[r], 0.0))
    vals = np.where(off, d_j, 0.0)
    diag = a * drho + np.bincount(r, weights=np.where(off, d_i, 0.0), minlength=len(p)) \
        + drho * (t * p - q) + rho * t
    vals = np.where(off, vals, diag[r])
    J = sp.csr_matrix((vals, A.indices.copy(), A.indptr.copy()), shape=A.shape)
    return R, J


def newton_direct(sysm, p0, p_old, c=0.2, gamma=0.1, rtol=1e-10, max_it=20):
    """Newton's method with sparse direct linear solves (the reference
    iterates); returns (p, residual norms)."""
    p = p0.copy()
    hist = []
    for _ in range(max_it):
        R, J = residual_jacobian(sysm, p, p_old, c, gamma)
        hist.append(float(np.linalg.norm(R)))
        if hist[-1] <= rtol * hist[0]:
            break
        p = p + spla.spsolve(J.tocsc(), -R)
    return p, hist
