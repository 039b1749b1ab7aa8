"""Pins of the oracle's MSFV and MSMIX restrictions (Sec. 3.2)."""
import numpy as np
import pytest
import scipy.sparse.linalg as spl

from oracle import fams, grids
from tests._cases import small_case


def _setup(name, kind, variant=fams.DECOUPLED):
    s, spec = small_case(name)
    wb, primal, vertex, _ = grids.full_grid(s, spec["coarse"], spec["d_min"], spec["r_z"])
    F = fams.FAMS(s.csr(), wb, vertex, s.n_matrix, variant, primal=primal,
                  restriction_kind=kind)
    return s, F, np.asarray(primal), np.asarray(vertex)


def _block_sums(primal, nc, v):
    return np.bincount(primal, weights=v, minlength=nc)


def _after_coarse(F, r):
    """r - A P A_c^{-1} R r: the residual after the multiscale stage alone."""
    import scipy.linalg as sla
    xc = sla.lu_solve(F.lu, F.R @ r)
    return r - F.A @ (F.P @ xc)


@pytest.mark.parametrize("name", ["2d", "3d"])
def test_msfv_conserves_on_primal_blocks(name):
    """Sec. 3.2: after a coarse stage with R^FV the residual sums to zero over
    every primal block (coarse-scale mass conservation); with R^FE it does
    not in general, so the check tells the two apart."""
    r = np.random.default_rng(3).standard_normal(small_case(name)[0].n)
    s, F, primal, vertex = _setup(name, fams.RESTRICT_FV)
    nc = len(vertex)
    sums = _block_sums(primal, nc, _after_coarse(F, r))
    assert np.abs(sums).max() <= 1e-11 * np.abs(r).sum()
    _, Fe, _, _ = _setup(name, fams.RESTRICT_FE)
    sums_fe = _block_sums(primal, nc, _after_coarse(Fe, r))
    assert np.abs(sums_fe).max() > 1e-6 * np.abs(r).sum()


@pytest.mark.parametrize("name", ["2d", "3d"])
def test_msmix_rows(name):
    """MSMIX: the coarse nodes on fractures conserve over their primal
    blocks, the matrix ones are Galerkin (P_i^T r' = 0), and R has exactly
    those rows (an indicator of the block, or the column of P)."""
    r = np.random.default_rng(4).standard_normal(small_case(name)[0].n)
    s, F, primal, vertex = _setup(name, fams.RESTRICT_MIX)
    nc = len(vertex)
    frac = vertex >= s.n_matrix
    assert frac.any() and (~frac).any()
    rp = _after_coarse(F, r)
    scale = np.abs(r).sum()
    sums = _block_sums(primal, nc, rp)
    assert np.abs(sums[frac]).max() <= 1e-11 * scale
    gal = F.P.T @ rp
    assert np.abs(gal[~frac]).max() <= 1e-11 * scale
    R = F.R.toarray()
    ind = (primal[None, :] == np.arange(nc)[:, None]).astype(float)
    assert np.array_equal(R[frac], ind[frac])
    assert np.array_equal(R[~frac], F.P.T.toarray()[~frac])


@pytest.mark.parametrize("kind", [fams.RESTRICT_FV, fams.RESTRICT_MIX])
@pytest.mark.parametrize("name", ["2d", "3d"])
def test_restricted_gmres_reaches_direct_solution(name, kind):
    """With either restriction the preconditioned GMRES still converges to
    A^{-1} q (the coarse stage changes the preconditioner, not the answer)."""
    s, F, _, _ = _setup(name, kind)
    p, info = F.gmres(s.q, rtol=1e-10)
    assert info["status"] == fams.OK
    pd = spl.spsolve(s.csr().tocsc(), s.q)
    assert np.linalg.norm(p - pd) <= 1e-7 * np.linalg.norm(pd)
