"""Sanity of the seeded synthetic inputs (the EDFM fine-scale systems)."""
import numpy as np
import pytest

from workloads import make_config, make_small


@pytest.mark.parametrize("kind", ["2d", "3d"])
def test_small_system_is_symmetric_m_matrix(kind):
    s = make_small(kind)
    A = s.csr()
    assert abs(A - A.T).max() == 0
    off = A - np.diag(A.diagonal()) if False else A.copy()
    off.setdiag(0)
    off.eliminate_zeros()
    assert off.data.max() < 0                       # TPFA/CI couplings are negative
    rs = np.asarray(A.sum(axis=1)).ravel()
    assert rs.min() > -1e-9 * A.diagonal().max()    # weakly diagonally dominant
    assert np.all(np.diff(s.col[s.row_ptr[0]:s.row_ptr[1]]) > 0)
    assert s.q.sum() > 0                            # Dirichlet p=1 face feeds q


def test_seeded_and_deterministic():
    a, b = make_small("3d", seed=3), make_small("3d", seed=3)
    assert a.sha256() == b.sha256()
    assert make_small("3d", seed=4).sha256() != a.sha256()


def test_config1_shape():
    s = make_config(1)
    assert s.n_matrix == 100 * 100
    assert 500 < s.n_frac < 1500        # ~20 segments of 0.2-0.5 domain lengths
    assert s.t_ratio > 1.0
