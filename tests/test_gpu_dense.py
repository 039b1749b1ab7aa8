"""Dense kernels of the coarse system (FP64 MFMA product, Gauss-Jordan and
LU inverses, the one-workgroup LU solve) against numpy on seeded matrices."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)


@pytest.mark.parametrize("n", [1, 37, 64, 130, 600, 2000, 2049])
def test_mfma_product(n):
    from paper_1705_05784_amd import fams
    _say(f"[dense] product n={n}")
    a = np.random.default_rng(n).standard_normal((n, n))
    c = fams.dense_op(0, a).cpu().numpy()
    ref = a @ a
    assert np.abs(c - ref).max() <= 1e-12 * max(1.0, np.abs(ref).max())


@pytest.mark.parametrize("n", [1, 37, 100, 256, 257, 700, 1855, 4100])
def test_spd_gauss_jordan(n):
    from paper_1705_05784_amd import fams
    _say(f"[dense] gauss-jordan n={n}")
    m = np.random.default_rng(n + 1).standard_normal((n, n))
    a = m @ m.T / n + np.eye(n)
    x = fams.dense_op(1, a).cpu().numpy()
    assert np.abs(x @ a - np.eye(n)).max() <= 1e-10


def test_gauss_jordan_rejects_indefinite():
    from paper_1705_05784_amd import fams
    a = np.diag([1.0, -1.0, 2.0])
    with pytest.raises(fams.FamsError):
        fams.dense_op(1, a)


@pytest.mark.parametrize("n", [1, 37, 600, 1500, 2100])
def test_lu_inverse(n):
    from paper_1705_05784_amd import fams
    _say(f"[dense] lu inverse n={n}")
    a = np.random.default_rng(n + 2).standard_normal((n, n)) + 0.5 * np.eye(n)
    x = fams.dense_op(2, a).cpu().numpy()
    ref = np.linalg.inv(a)
    assert np.abs(x - ref).max() <= 1e-9 * np.abs(ref).max()


@pytest.mark.parametrize("n", [1, 37, 65, 300, 700])
def test_lu_solve(n):
    from paper_1705_05784_amd import fams
    _say(f"[dense] lu solve n={n}")
    a = np.random.default_rng(n + 3).standard_normal((n, n)) + 0.5 * np.eye(n)
    x = fams.dense_op(3, a).cpu().numpy()
    ref = np.linalg.inv(a)
    assert np.abs(x - ref).max() <= 1e-9 * np.abs(ref).max()


@pytest.mark.parametrize("n", [1, 17, 37, 600, 1500, 2100])
def test_lu_factors_match_getrf(n):
    """The pivoted LU makes the pivot choices of LAPACK getrf (first maximal
    |a| in the column): the packed factors equal scipy's to rounding, which a
    single different pivot would break at O(1).  n = 2100 starts with the
    32-column panels and then takes the 16-column register panels."""
    import scipy.linalg as sla
    from paper_1705_05784_amd import fams
    _say(f"[dense] lu factors n={n}")
    a = np.random.default_rng(n + 5).standard_normal((n, n))
    lu = fams.dense_op(4, a).cpu().numpy()
    ref, _ = sla.lu_factor(a)
    assert np.abs(lu - ref).max() <= 1e-9 * max(1.0, np.abs(ref).max())
