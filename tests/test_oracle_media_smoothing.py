"""Pins of the oracle's per-medium smoothing stage (Sec. 3.2)."""
import numpy as np
import pytest
import scipy.sparse.linalg as spl

from oracle import fams, grids
from tests._cases import small_case


def _setup(name, media, variant=fams.DECOUPLED):
    s, spec = small_case(name)
    wb, primal, vertex, _ = grids.full_grid(s, spec["coarse"], spec["d_min"], spec["r_z"])
    F = fams.FAMS(s.csr(), wb, vertex, s.n_matrix, variant, media_smoothing=media)
    return s, F


@pytest.mark.parametrize("name", ["2d", "3d"])
def test_media_factors_are_the_per_medium_ilu0(name):
    """ILU(0) of diag(A^mm, A^ff) has no entry between the media, and its
    two diagonal blocks are the ILU(0) factors of A^mm and of A^ff computed
    on their own (the stage works on the two media separately)."""
    s, _ = small_case(name)
    A, nm = s.csr(), s.n_matrix
    assert 0 < nm < s.n
    B = fams.media_blocks(A, nm)
    assert abs(B[:nm, nm:]).sum() == 0 and abs(B[nm:, :nm]).sum() == 0
    assert (abs(A[:nm, nm:]) > 0).sum() > 0  # the media are coupled in A
    L, U = fams.ILU0(B).factors()
    assert abs(L[nm:, :nm]).sum() == 0 and abs(U[:nm, nm:]).sum() == 0
    for sl in (slice(0, nm), slice(nm, s.n)):
        Ls, Us = fams.ILU0(A[sl, sl]).factors()
        assert abs(L[sl, sl] - Ls).max() <= 1e-14 * abs(Ls).max()
        assert abs(U[sl, sl] - Us).max() <= 1e-14 * abs(Us).max()


@pytest.mark.parametrize("variant", [fams.DECOUPLED, fams.COUPLED])
@pytest.mark.parametrize("name", ["2d", "3d"])
def test_media_smoothing_converges_to_direct_solution(name, variant):
    """With the extra stage the preconditioner changes (the stage is not a
    no-op on coupled media) but GMRES and Richardson still reach A^{-1} q."""
    s, F = _setup(name, True, variant)
    _, F0 = _setup(name, False, variant)
    r = np.random.default_rng(5).standard_normal(s.n)
    assert np.linalg.norm(F.stage(r) - F0.stage(r)) > 1e-6 * np.linalg.norm(F0.stage(r))
    pd = spl.spsolve(s.csr().tocsc(), s.q)
    p, info = F.gmres(s.q, rtol=1e-10)
    assert info["status"] == fams.OK
    assert np.linalg.norm(p - pd) <= 1e-7 * np.linalg.norm(pd)
    p, info = F.richardson(s.q, rtol=1e-10, max_iter=400)
    assert info["status"] == fams.OK
    assert np.linalg.norm(p - pd) <= 1e-7 * np.linalg.norm(pd)
