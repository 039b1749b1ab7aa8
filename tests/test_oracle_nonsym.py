"""A non-symmetric A (a linearised compressible system, Eq. dis-mf: "A can be
non-symmetric, due to the compressibility effects"; Table 1 steps 1-2 update
it every outer iteration).  The oracle's prolongation is written for any A:
these pins check it on non-symmetric matrices against App. A's block
formulas, the partition of unity (a non-symmetric A with zero row sums), the
iteration's convergence to a direct solve, and a Newton loop with the value
update (Sec. 3.1's adaptive basis) against Newton with direct solves.  The
compressible residual's Jacobian is itself checked by finite differences."""
import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from oracle import fams, grids
from tests._cases import small_case
from tests.test_oracle_basis import appendix_a
from workloads.compressible import newton_direct, residual_jacobian

VARIANTS = [fams.DECOUPLED, fams.FRAC, fams.ROCK, fams.COUPLED]


def _grid(s, spec):
    return grids.full_grid(s, spec["coarse"], spec["d_min"], spec["r_z"])


def jacobian_case(name="3d", **kw):
    s, spec = small_case(name, **kw)
    p_old = spla.spsolve(s.csr().tocsc(), s.q)
    p = p_old + 0.05 * np.random.default_rng(1).standard_normal(s.n)
    R, J = residual_jacobian(s, p, p_old - 0.1)
    return s, spec, R, J


def test_jacobian_finite_differences():
    """Every column of J matches central differences of R (the model's own
    derivative, so that the non-symmetry is the model's, not a slip)."""
    s, _ = small_case("2d")
    p_old = spla.spsolve(s.csr().tocsc(), s.q)
    p = p_old + 0.05 * np.random.default_rng(2).standard_normal(s.n)
    _, J = residual_jacobian(s, p, p_old)
    Jd = J.toarray()
    h = 1e-6
    for k in np.random.default_rng(3).choice(s.n, 12, replace=False):
        e = np.zeros(s.n)
        e[k] = h
        fd = (residual_jacobian(s, p + e, p_old)[0] - residual_jacobian(s, p - e, p_old)[0]) / (2 * h)
        assert np.abs(fd - Jd[:, k]).max() <= 1e-6 * np.abs(Jd).max()
    assert np.abs(Jd - Jd.T).max() > 1e-3 * np.abs(Jd).max()      # really non-symmetric
    off = ~np.eye(s.n, dtype=bool)
    assert Jd[off].max() <= 0.0


@pytest.mark.parametrize("variant", VARIANTS)
@pytest.mark.parametrize("name,kw", [("2d", {}), ("3d", dict(nx=12, ny=12, nz=8, n_frac=4))])
def test_matches_appendix_a_nonsymmetric(name, variant, kw):
    """App. A's block formulas hold for any A; the rank rule reproduces them
    on the non-symmetric Jacobian."""
    s, spec, _, J = jacobian_case(name, **kw)
    wb, _, vertex, _ = _grid(s, spec)
    P = fams.prolongation(J, wb, vertex, s.n_matrix, variant, merge_cap=10**9).toarray()
    P_ref = appendix_a(J.toarray(), wb, s.n_matrix, vertex, variant)
    assert np.abs(P - P_ref).max() < 1e-11


@pytest.mark.parametrize("variant", VARIANTS)
def test_partition_of_unity_nonsymmetric(variant):
    """A non-symmetric A with zero row sums (a Neumann A plus a zero-row-sum
    upwind-like perturbation) gives P 1 = 1."""
    s, spec = small_case("3d", neumann=True)
    A = s.csr().tocoo()
    rng = np.random.default_rng(4)
    off = A.row != A.col
    eps = np.where(off, -rng.uniform(0.0, 0.5, A.nnz) * np.abs(A.data), 0.0)
    C = sp.csr_matrix((eps, (A.row, A.col)), shape=A.shape)
    C = C - sp.diags(np.asarray(C.sum(axis=1)).ravel())
    An = sp.csr_matrix(s.csr() + C)
    assert np.abs(np.asarray(An.sum(axis=1)).ravel()).max() < 1e-9
    assert abs(An - An.T).max() > 0
    wb, _, vertex, _ = _grid(s, spec)
    P = fams.prolongation(An, wb, vertex, s.n_matrix, variant).toarray()
    assert np.abs(P.sum(axis=1) - 1.0).max() < 1e-12


@pytest.mark.parametrize("variant", VARIANTS)
def test_gmres_nonsymmetric(variant):
    s, spec, R, J = jacobian_case()
    wb, _, vertex, _ = _grid(s, spec)
    F = fams.FAMS(J, wb, vertex, s.n_matrix, variant, 1e-2)
    x, info = F.gmres(-R, rtol=1e-11)
    ref = spla.spsolve(J.tocsc(), -R)
    assert info["status"] == fams.OK
    assert np.linalg.norm(x - ref) <= 1e-8 * np.linalg.norm(ref)


@pytest.mark.parametrize("threshold", [0.0, 0.05, np.inf])
def test_newton_with_value_update(threshold):
    """Table 1 as a Newton loop: every iteration updates A (the Jacobian) and
    q (-R); the basis is recomputed only when an entry changed by more than
    `threshold` (0: always; inf: never, the first basis is kept).  The
    iterates equal Newton with direct solves (1e-8) in as many iterations."""
    s, spec = small_case("3d")
    wb, _, vertex, _ = _grid(s, spec)
    p_old = spla.spsolve(s.csr().tocsc(), s.q)
    p_ref, hist = newton_direct(s, p_old, p_old - 0.1)
    p = p_old.copy()
    F = None
    norms = []
    for _ in range(20):
        R, J = residual_jacobian(s, p, p_old - 0.1)
        norms.append(float(np.linalg.norm(R)))
        if norms[-1] <= 1e-10 * norms[0]:
            break
        if F is None:
            F = fams.FAMS(J, wb, vertex, s.n_matrix, fams.COUPLED, 1e-2)
        else:
            F.update_values(J, threshold)
        d, info = F.gmres(-R, rtol=1e-12)
        assert info["status"] == fams.OK
        p = p + d
    assert len(norms) == len(hist)
    assert np.linalg.norm(p - p_ref) <= 1e-8 * np.linalg.norm(p_ref)
