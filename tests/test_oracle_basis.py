"""Pins of the oracle's prolongation (Sec. 3.1, App. A) and truncation (Sec. 4.3)."""
import numpy as np
import pytest

from oracle import fams, grids
from tests._cases import hat_1d, homogeneous, small_case

VARIANTS = [fams.DECOUPLED, fams.FRAC, fams.ROCK, fams.COUPLED]


def _grid(s, spec):
    return grids.full_grid(s, spec["coarse"], spec["d_min"], spec["r_z"])


def test_hats_1d():
    """Homogeneous 1D: the basis functions are linear hats between coarse
    nodes and constant beyond the outermost ones (Neumann ends)."""
    s = homogeneous(21, 1, 1)
    wb, _, vertex = grids.structured_grid(21, 1, 1, 5, 1, 1)
    P = fams.prolongation(s.csr(), wb, vertex, s.n_matrix, fams.DECOUPLED).toarray()
    assert np.abs(P - hat_1d(21, 5)).max() < 1e-13


def test_hats_2d():
    """Homogeneous 2D 5-point: bilinear tensor-product hats."""
    nx, ny, c = 17, 13, 4
    s = homogeneous(nx, ny, 1)
    wb, _, vertex = grids.structured_grid(nx, ny, 1, c, c, 1)
    P = fams.prolongation(s.csr(), wb, vertex, s.n_matrix, fams.DECOUPLED).toarray()
    Hx, Hy = hat_1d(nx, c), hat_1d(ny, c)
    expect = np.einsum("yb,xa->yxba", Hy, Hx).reshape(nx * ny, -1)
    assert np.abs(P - expect).max() < 1e-12


def test_hats_3d():
    """Homogeneous 3D 7-point: trilinear tensor-product hats."""
    nx, ny, nz, c = 11, 9, 10, 3
    s = homogeneous(nx, ny, nz)
    wb, _, vertex = grids.structured_grid(nx, ny, nz, c, c, c)
    P = fams.prolongation(s.csr(), wb, vertex, s.n_matrix, fams.DECOUPLED).toarray()
    Hx, Hy, Hz = hat_1d(nx, c), hat_1d(ny, c), hat_1d(nz, c)
    expect = np.einsum("zc,yb,xa->zyxcba", Hz, Hy, Hx).reshape(nx * ny * nz, -1)
    assert np.abs(P - expect).max() < 1e-12


def test_fracture_chain_hats():
    """A straight fracture with equal segments: Decoupled-AMS fracture basis
    functions are linear hats along the chain between fracture nodes."""
    from workloads import Plate
    nx, ny = 20, 11
    h = 1.0 / nx
    pl = Plate(2 * h, 5.5 * h, 18 * h, 5.5 * h, 0, 1)
    s = homogeneous(nx, ny, 1, plates=[pl])
    assert s.n_frac == 16
    wb, primal, vertex, ncm = grids.full_grid(s, (5, 5, 1), d_min=4, r_z=1)
    fv = vertex[ncm:] - s.n_matrix
    assert list(fv) == [0, 4, 8, 12]
    P = fams.prolongation(s.csr(), wb, vertex, s.n_matrix, fams.DECOUPLED).toarray()
    Pff = P[s.n_matrix:, ncm:]
    H = np.zeros((16, 4))
    for x in range(16):
        if x >= 12:
            H[x, 3] = 1.0
        else:
            k = x // 4
            H[x, k] = (4 * (k + 1) - x) / 4
            if k + 1 < 4:
                H[x, k + 1] = (x - 4 * k) / 4
    assert np.abs(Pff - H).max() < 1e-12


@pytest.mark.parametrize("alpha", [0.0, 1e-2])
@pytest.mark.parametrize("variant", VARIANTS)
@pytest.mark.parametrize("name", ["2d", "3d"])
def test_partition_of_unity(name, variant, alpha):
    """All four strategies give a partition of unity (Sec. 3.1) when A has
    zero row sums; truncation keeps it (Sec. 4.3)."""
    s, spec = small_case(name, neumann=True)
    wb, _, vertex, _ = _grid(s, spec)
    P = fams.prolongation(s.csr(), wb, vertex, s.n_matrix, variant, alpha)
    assert np.abs(np.asarray(P.sum(axis=1)).ravel() - 1).max() < 1e-12
    if alpha:
        nonv = wb != 3
        assert np.all(np.abs(P[nonv].data) >= alpha)


@pytest.mark.parametrize("variant", VARIANTS)
@pytest.mark.parametrize("name", ["2d", "3d"])
def test_support_and_bounds(name, variant):
    """Support per strategy (Sec. 3, the four coupling definitions) and the
    discrete maximum principle 0 <= P <= 1."""
    s, spec = small_case(name)
    wb, _, vertex, ncm = _grid(s, spec)
    nm = s.n_matrix
    P = fams.prolongation(s.csr(), wb, vertex, nm, variant).toarray()
    assert P.min() >= 0.0 and P.max() <= 1.0 + 1e-12
    mf = np.abs(P[:nm, ncm:]).max()
    fm = np.abs(P[nm:, :ncm]).max()
    expect_mf = variant in (fams.FRAC, fams.COUPLED)
    expect_fm = variant in (fams.ROCK, fams.COUPLED)
    assert (mf > 0) == expect_mf
    assert (fm > 0) == expect_fm
    # vertex rows are Kronecker deltas
    assert np.array_equal(P[vertex], np.eye(len(vertex)))


# ---- App. A, evaluated literally as dense block formulas --------------------

def appendix_a(A, wb, nm, vertex, variant):
    n = A.shape[0]
    nc = len(vertex)
    cells = np.arange(n)
    m, f = cells[:nm], cells[nm:]
    sel = lambda S, t: S[wb[S] == t]  # noqa: E731
    Im, Fm, Em, Vm = (sel(m, t) for t in (0, 1, 2, 3))
    Ff, Ef, Vf = (sel(f, t) for t in (1, 2, 3))
    coarse = np.full(n, -1)
    coarse[vertex] = np.arange(nc)
    Cm = np.arange(nc)[np.asarray(vertex) < nm]
    Cf = np.arange(nc)[np.asarray(vertex) >= nm]
    B = lambda R, C: A[np.ix_(R, C)]  # noqa: E731

    def lumped(R, drop):
        return B(R, R) + np.diag(B(R, drop).sum(axis=1))

    def solve(M, rhs):
        return -np.linalg.solve(M, rhs) if len(M) else np.zeros((0, rhs.shape[1]))

    P = np.zeros((n, nc))
    P[vertex, np.arange(nc)] = 1.0
    cat = np.concatenate
    E, F, I, V = cat([Em, Ef]), cat([Fm, Ff]), Im, cat([Vm, Vf])
    if variant == fams.COUPLED:
        P[E] = solve(lumped(E, cat([F, I])), B(E, V) @ P[V])
        P[F] = solve(lumped(F, I), B(F, E) @ P[E] + B(F, V) @ P[V])
        P[I] = solve(B(I, I), B(I, F) @ P[F] + B(I, E) @ P[E] + B(I, V) @ P[V])
        return P
    ix = np.ix_
    if variant in (fams.DECOUPLED, fams.FRAC):      # fracture part, no-flow to matrix
        P[ix(Ef, Cf)] = solve(lumped(Ef, cat([Ff, m])), B(Ef, Vf) @ P[ix(Vf, Cf)])
        P[ix(Ff, Cf)] = solve(lumped(Ff, m), B(Ff, Ef) @ P[ix(Ef, Cf)])
    if variant in (fams.DECOUPLED, fams.ROCK):      # matrix part, no-flow to fractures
        P[ix(Em, Cm)] = solve(lumped(Em, cat([Fm, Im, f])), B(Em, Vm) @ P[ix(Vm, Cm)])
        P[ix(Fm, Cm)] = solve(lumped(Fm, cat([Im, f])), B(Fm, Em) @ P[ix(Em, Cm)])
        P[ix(Im, Cm)] = solve(lumped(Im, f), B(Im, Fm) @ P[ix(Fm, Cm)])
    if variant == fams.FRAC:                        # Eq. (FracAMS-prlg), matrix rows
        Ebar, Fbar, Aii = lumped(Em, cat([Fm, Im])), lumped(Fm, Im), B(Im, Im)
        P[ix(Em, Cm)] = solve(Ebar, B(Em, Vm) @ P[ix(Vm, Cm)])
        P[ix(Em, Cf)] = solve(Ebar, B(Em, f) @ P[ix(f, Cf)])
        P[ix(Fm, Cm)] = solve(Fbar, B(Fm, Em) @ P[ix(Em, Cm)])
        P[ix(Fm, Cf)] = solve(Fbar, B(Fm, Em) @ P[ix(Em, Cf)] + B(Fm, f) @ P[ix(f, Cf)])
        P[ix(Im, Cm)] = solve(Aii, B(Im, Fm) @ P[ix(Fm, Cm)])
        P[ix(Im, Cf)] = solve(Aii, B(Im, Fm) @ P[ix(Fm, Cf)] + B(Im, f) @ P[ix(f, Cf)])
    if variant == fams.ROCK:                        # Eq. (RockAMS-prlg), fracture rows
        Ebar, Aff = lumped(Ef, Ff), B(Ff, Ff)
        P[ix(Ef, Cm)] = solve(Ebar, B(Ef, m) @ P[ix(m, Cm)])
        P[ix(Ef, Cf)] = solve(Ebar, B(Ef, Vf) @ P[ix(Vf, Cf)])
        P[ix(Ff, Cm)] = solve(Aff, B(Ff, Ef) @ P[ix(Ef, Cm)] + B(Ff, m) @ P[ix(m, Cm)])
        P[ix(Ff, Cf)] = solve(Aff, B(Ff, Ef) @ P[ix(Ef, Cf)])
    return P


def _tpfa_zero_blocks(A, wb, nm):
    """The blocks App. A states are zero for TPFA on structured grids."""
    n = A.shape[0]
    med = np.arange(n) >= nm
    r, c = np.nonzero(A)
    same_m = ~med[r] & ~med[c]
    same_f = med[r] & med[c]
    bad = same_m & (np.abs(wb[r].astype(int) - wb[c]) > 1)
    bad |= same_f & (((wb[r] == 1) & (wb[c] == 3)) | ((wb[r] == 3) & (wb[c] == 1)))
    return not bad.any()


@pytest.mark.parametrize("variant", VARIANTS)
@pytest.mark.parametrize("name,kw", [("2d", {}), ("3d", dict(nx=12, ny=12, nz=8, n_frac=4))])
def test_matches_appendix_a(name, variant, kw):
    """The generic rank/lumping rule reproduces the block formulas of App. A."""
    s, spec = small_case(name, **kw)
    wb, _, vertex, _ = _grid(s, spec)
    A = s.csr()
    Ad = A.toarray()
    assert _tpfa_zero_blocks(Ad, wb, s.n_matrix)
    P = fams.prolongation(A, wb, vertex, s.n_matrix, variant, merge_cap=10**9).toarray()
    P_ref = appendix_a(Ad, wb, s.n_matrix, vertex, variant)
    assert np.abs(P - P_ref).max() < 1e-11


def test_truncation_rule():
    """Sec. 4.3: drop below alpha, rescale survivors to the row's prior sum."""
    import scipy.sparse as sp
    P = sp.csr_matrix(np.array([[0.5, 0.005, 0.495, 0.0],
                                [0.001, 0.002, 0.003, 0.004],
                                [0.3, 0.3, 0.4, 0.0],
                                [1.0, 0.0, 0.0, 0.0]]))
    T = fams.truncate(P, 1e-2, np.array([False, False, False, True])).toarray()
    assert np.allclose(T[0], [0.5 / 0.995, 0, 0.495 / 0.995, 0], atol=1e-15)
    assert np.allclose(T[1], [0, 0, 0, 0.01], atol=1e-15)      # only the largest survives
    assert np.array_equal(T[2], [0.3, 0.3, 0.4, 0.0])           # untouched row
    assert np.array_equal(T[3], [1.0, 0, 0, 0])


# ---- Coupled-AMS merge under a size cap (Sec. 3.1) ---------------------------

def _cut_lumped(Ad, pairs):
    """A with the couplings in `pairs` taken out and added to the diagonal."""
    B = Ad.copy()
    for i, j in pairs:
        B[i, i] += B[i, j]
        B[i, j] = 0.0
    return B


@pytest.mark.parametrize("cap", [12, 20])
def test_coupled_merge_cap(cap):
    """With a merge cap that binds: every block that spans both media holds
    at most `cap` cells; a cross-media coupling between equal classes is cut
    only when the two blocks it joins could not have been united under the
    cap (their sizes add up to more than cap: blocks only grow, so this holds
    at the end if it held when the coupling was refused); P still gives a
    partition of unity on a Neumann A; and P equals App. A.4's Coupled-AMS
    block formulas evaluated densely on A with the cut couplings lumped into
    the diagonal."""
    s, spec = small_case("3d", neumann=True)
    wb, _, vertex, _ = _grid(s, spec)
    A = s.csr()
    nm = s.n_matrix
    _, free = fams.prolongation(A, wb, vertex, nm, fams.COUPLED, merge_cap=10**9,
                                return_blocks=True)
    med = np.arange(s.n) >= nm
    sizes_free = np.bincount(free["comp"][free["comp"] >= 0])
    assert sizes_free.max() > cap          # the cap binds on this case
    P, info = fams.prolongation(A, wb, vertex, nm, fams.COUPLED, merge_cap=cap,
                                return_blocks=True)
    comp = info["comp"]
    sizes = np.bincount(comp[comp >= 0])
    for K in np.unique(comp[comp >= 0]):
        cells = np.nonzero(comp == K)[0]
        if med[cells].any() and (~med[cells]).any():
            assert len(cells) <= cap
    r = np.repeat(np.arange(s.n), np.diff(A.indptr))
    c = A.indices
    cross = (med[r] != med[c]) & (wb[r] == wb[c]) & (wb[r] != 3) & (r != c)
    cut = cross & (comp[r] != comp[c])
    assert cut.any()
    for i, j in zip(r[cut], c[cut]):
        assert sizes[comp[i]] + sizes[comp[j]] > cap
    assert np.abs(np.asarray(P.sum(axis=1)).ravel() - 1).max() < 1e-12
    Acut = _cut_lumped(A.toarray(), zip(r[cut], c[cut]))
    P_ref = appendix_a(Acut, wb, nm, vertex, fams.COUPLED)
    assert np.abs(P.toarray() - P_ref).max() < 1e-11
