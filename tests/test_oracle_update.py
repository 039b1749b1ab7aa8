"""Pins of the oracle's value update and basis re-setup policy (Table 1,
steps 2 and 4; Sec. 3.1)."""
import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spl

from oracle import fams, grids
from tests._cases import small_case


def _setup(name, variant=fams.DECOUPLED):
    s, spec = small_case(name)
    wb, primal, vertex, _ = grids.full_grid(s, spec["coarse"], spec["d_min"], spec["r_z"])
    return s, fams.FAMS(s.csr(), wb, vertex, s.n_matrix, variant)


def scaled(A, n, amp, seed=0):
    """D A D with d_i = 1 + amp sin(i + seed): symmetric, same pattern."""
    d = 1.0 + amp * np.sin(np.arange(n) + seed)
    D = sp.diags(d)
    return sp.csr_matrix(D @ A @ D)


@pytest.mark.parametrize("variant", [fams.DECOUPLED, fams.COUPLED])
@pytest.mark.parametrize("name", ["2d", "3d"])
def test_basis_is_scale_invariant(name, variant):
    """Every local problem of c A has the solution of A's (the right-hand side
    scales with the operator), so a recomputed basis for c A is the old one
    and A_c scales by c."""
    s, F = _setup(name, variant)
    P0, Ac0 = F.P.toarray(), F.Ac.copy()
    assert F.update_values(3.7 * s.csr(), threshold=-1.0)
    assert np.abs(F.P.toarray() - P0).max() <= 1e-13
    assert np.abs(F.Ac - 3.7 * Ac0).max() <= 1e-12 * np.abs(3.7 * Ac0).max()


@pytest.mark.parametrize("name", ["2d", "3d"])
def test_threshold_decides_the_basis(name):
    """A change of at most ~10% per entry: a threshold of 0.5 keeps P (the
    very same operator), 0.01 recomputes it (and then P differs)."""
    s, F = _setup(name)
    A2 = scaled(s.csr(), s.n, 0.05)
    P0 = F.P
    assert not F.update_values(A2, threshold=0.5)
    assert F.P is P0
    assert F.update_values(A2, threshold=0.01)
    assert np.abs(F.P.toarray() - P0.toarray()).max() > 1e-6


@pytest.mark.parametrize("name", ["2d", "3d"])
def test_kept_basis_still_converges(name):
    """With the basis of the old A and everything else following a new A (30%
    entry changes), GMRES still reaches A_new^{-1} q."""
    s, F = _setup(name)
    A2 = scaled(s.csr(), s.n, 0.3, seed=1)
    assert not F.update_values(A2, threshold=1e9)
    p, info = F.gmres(s.q, rtol=1e-10)
    assert info["status"] == fams.OK
    pd = spl.spsolve(A2.tocsc(), s.q)
    assert np.linalg.norm(p - pd) <= 1e-7 * np.linalg.norm(pd)
