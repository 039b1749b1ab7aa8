"""Wells as coarse nodes (Sec. 2: the Peaceman term beta (p^w - p) in every
perforated cell; Sec. 3: one fine-scale unknown and one coarse node per
well, mapped by the identity; Sec. 3.1: the beta (Phi - Phi^w) term of the
skeleton equation).  The oracle's prolongation with wells against App. A's
block formulas with the well columns added, its partition of unity, the
well rows (P^ww = I, P^wm = P^wf = 0, Eq. prolongation_single), where a
well's function can be non-zero under each coupling strategy (Sec. 3.1:
inside the fractures for a matrix-only well under Rock- and Coupled-AMS
only), and the iteration's convergence to a direct solve."""
import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from oracle import fams, grids
from tests._cases import small_case, wells_case
from workloads import Well, add_wells

VARIANTS = [fams.DECOUPLED, fams.FRAC, fams.ROCK, fams.COUPLED]


def well_case(name="3d", neumann=False, **kw):
    sw, spec = wells_case(name, neumann=neumann, **kw)
    wb, pr, vx, _ = grids.full_grid(sw, spec["coarse"], spec["d_min"], spec["r_z"])
    return sw, spec, wb, pr, vx


def _P(sw, wb, vx, variant, alpha=0.0, merge_cap=10**9):
    return fams.prolongation(sw.csr(), wb, vx, sw.n_matrix, variant, alpha, merge_cap,
                             n_wells=sw.n_wells).toarray()


def test_add_wells_peaceman():
    """The well rows and columns are Peaceman's: WI = 2 pi k h_z / ln(r_e / r_w)
    with r_e = 0.2 h; a cell row's sum is unchanged and a well row's sum is 0."""
    s, _ = small_case("3d")
    ix, iy = 2, 3
    sw = add_wells(s, [Well(ix, iy, 1, 4, rate=2.0)], r_w=0.05)
    A0, A = s.csr(), sw.csr()
    n0 = s.n
    w = n0
    cells = [ix + s.nx * (iy + s.ny * z) for z in range(1, 4)]
    k = np.exp(s.lnk)
    for z, m in zip(range(1, 4), cells):
        wi = 2 * np.pi * k[z, iy, ix] * s.h / np.log(0.2 / 0.05)
        assert np.isclose(A[m, w], -wi, rtol=1e-14)
        assert np.isclose(A[w, m], -wi, rtol=1e-14)
        assert np.isclose(A[m, m], A0[m, m] + wi, rtol=1e-14)
    rs = np.asarray(A.sum(axis=1)).ravel()
    assert np.allclose(rs[:n0], np.asarray(A0.sum(axis=1)).ravel(), rtol=0, atol=1e-9)
    assert abs(rs[w]) < 1e-9 * A[w, w]
    assert sw.q[w] == 2.0 and sw.n_wells == 1 and sw.n_frac == s.n_frac
    assert (A - A.T).count_nonzero() == 0


@pytest.mark.parametrize("variant", VARIANTS)
def test_well_rows(variant):
    """P^ww = I and P^wm = P^wf = 0 (Eq. prolongation_single)."""
    sw, _, wb, _, vx = well_case()
    P = _P(sw, wb, vx, variant)
    nw = sw.n_wells
    rows = np.arange(sw.n - nw, sw.n)
    cols = np.searchsorted(vx, rows)
    assert np.array_equal(vx[cols], rows)
    expect = np.zeros((nw, P.shape[1]))
    expect[np.arange(nw), cols] = 1.0
    assert np.array_equal(P[rows], expect)


@pytest.mark.parametrize("alpha", [0.0, 1e-2])
@pytest.mark.parametrize("variant", VARIANTS)
@pytest.mark.parametrize("name", ["2d", "3d"])
def test_partition_of_unity_with_wells(name, variant, alpha):
    """With a Neumann A (zero row sums; the well terms keep them zero) every
    row of P sums to one, the well columns included."""
    sw, _, wb, _, vx = well_case(name, neumann=True)
    assert np.abs(np.asarray(sw.csr().sum(axis=1)).ravel()).max() < 1e-9
    P = _P(sw, wb, vx, variant, alpha)
    assert np.abs(P.sum(axis=1) - 1.0).max() < 1e-12


def appendix_a_wells(A, wb, nm, nw, vertex, variant):
    """App. A's block formulas with wells: the wells W are Dirichlet data of
    every block (the beta term of the skeleton equation) and their columns
    join the column set of each medium; nothing is ever lumped into them."""
    n = A.shape[0]
    nc = len(vertex)
    cells = np.arange(n)
    m, f, W = cells[:nm], cells[nm:n - nw], cells[n - nw:]
    sel = lambda S, t: S[wb[S] == t]  # noqa: E731
    Im, Fm, Em, Vm = (sel(m, t) for t in (0, 1, 2, 3))
    Ff, Ef, Vf = (sel(f, t) for t in (1, 2, 3))
    vtx = np.asarray(vertex)
    Cm = np.arange(nc)[vtx < nm]
    Cf = np.arange(nc)[(vtx >= nm) & (vtx < n - nw)]
    Cw = np.arange(nc)[vtx >= n - nw]
    B = lambda R, C: A[np.ix_(R, C)]  # noqa: E731
    cat = np.concatenate

    def lumped(R, drop):
        return B(R, R) + np.diag(B(R, drop).sum(axis=1))

    def solve(M, rhs):
        return -np.linalg.solve(M, rhs) if len(M) else np.zeros((0, rhs.shape[1]))

    P = np.zeros((n, nc))
    P[vertex, np.arange(nc)] = 1.0
    # each medium's Dirichlet set and column set, with the wells added
    Vm_, Vf_, Cm_, Cf_ = cat([Vm, W]), cat([Vf, W]), cat([Cm, Cw]), cat([Cf, Cw])
    E, F, I, V = cat([Em, Ef]), cat([Fm, Ff]), Im, cat([Vm, Vf, W])
    if variant == fams.COUPLED:
        P[E] = solve(lumped(E, cat([F, I])), B(E, V) @ P[V])
        P[F] = solve(lumped(F, I), B(F, E) @ P[E] + B(F, V) @ P[V])
        P[I] = solve(B(I, I), B(I, F) @ P[F] + B(I, E) @ P[E] + B(I, V) @ P[V])
        return P
    ix = np.ix_
    if variant in (fams.DECOUPLED, fams.FRAC):      # fracture part, no-flow to matrix
        P[ix(Ef, Cf_)] = solve(lumped(Ef, cat([Ff, m])), B(Ef, Vf_) @ P[ix(Vf_, Cf_)])
        P[ix(Ff, Cf_)] = solve(lumped(Ff, m), B(Ff, Ef) @ P[ix(Ef, Cf_)] + B(Ff, W) @ P[ix(W, Cf_)])
    if variant in (fams.DECOUPLED, fams.ROCK):      # matrix part, no-flow to fractures
        P[ix(Em, Cm_)] = solve(lumped(Em, cat([Fm, Im, f])), B(Em, Vm_) @ P[ix(Vm_, Cm_)])
        P[ix(Fm, Cm_)] = solve(lumped(Fm, cat([Im, f])),
                               B(Fm, Em) @ P[ix(Em, Cm_)] + B(Fm, W) @ P[ix(W, Cm_)])
        P[ix(Im, Cm_)] = solve(lumped(Im, f), B(Im, Fm) @ P[ix(Fm, Cm_)] + B(Im, W) @ P[ix(W, Cm_)])
    if variant == fams.FRAC:                        # matrix rows, fractures (and wells) as data
        f_ = cat([f, W])
        Ebar, Fbar, Aii = lumped(Em, cat([Fm, Im])), lumped(Fm, Im), B(Im, Im)
        P[ix(Em, Cm)] = solve(Ebar, B(Em, Vm) @ P[ix(Vm, Cm)])
        P[ix(Em, Cf_)] = solve(Ebar, B(Em, f_) @ P[ix(f_, Cf_)])
        P[ix(Fm, Cm)] = solve(Fbar, B(Fm, Em) @ P[ix(Em, Cm)])
        P[ix(Fm, Cf_)] = solve(Fbar, B(Fm, Em) @ P[ix(Em, Cf_)] + B(Fm, f_) @ P[ix(f_, Cf_)])
        P[ix(Im, Cm)] = solve(Aii, B(Im, Fm) @ P[ix(Fm, Cm)])
        P[ix(Im, Cf_)] = solve(Aii, B(Im, Fm) @ P[ix(Fm, Cf_)] + B(Im, f_) @ P[ix(f_, Cf_)])
    if variant == fams.ROCK:                        # fracture rows, matrix (and wells) as data
        m_ = cat([m, W])
        Ebar, Aff = lumped(Ef, Ff), B(Ff, Ff)
        P[ix(Ef, Cm_)] = solve(Ebar, B(Ef, m_) @ P[ix(m_, Cm_)])
        P[ix(Ef, Cf)] = solve(Ebar, B(Ef, Vf) @ P[ix(Vf, Cf)])
        P[ix(Ff, Cm_)] = solve(Aff, B(Ff, Ef) @ P[ix(Ef, Cm_)] + B(Ff, m_) @ P[ix(m_, Cm_)])
        P[ix(Ff, Cf)] = solve(Aff, B(Ff, Ef) @ P[ix(Ef, Cf)])
    return P


@pytest.mark.parametrize("variant", VARIANTS)
@pytest.mark.parametrize("name,kw", [("2d", {}), ("3d", dict(nx=12, ny=12, nz=8, n_frac=4))])
def test_matches_appendix_a_with_wells(name, variant, kw):
    """The rank rule with wells ranked above both media reproduces App. A's
    block formulas extended by the wells' Dirichlet data and columns."""
    sw, _, wb, _, vx = well_case(name, **kw)
    P = _P(sw, wb, vx, variant)
    P_ref = appendix_a_wells(sw.csr().toarray(), wb, sw.n_matrix, sw.n_wells, vx, variant)
    assert np.abs(P - P_ref).max() < 1e-11


@pytest.mark.parametrize("variant", VARIANTS)
def test_well_function_support(variant):
    """Sec. 3.1: a matrix-only well's function is non-zero inside the
    fractures under Rock-AMS (fracture blocks take matrix values as data)
    and zero there under Decoupled- and Frac-AMS; a well that perforates
    fracture cells reaches them under every strategy; both are non-zero on
    their perforated cells."""
    sw, _, wb, _, vx = well_case()
    P = _P(sw, wb, vx, variant)
    nm, n, nw = sw.n_matrix, sw.n, sw.n_wells
    A = sw.csr()
    c1, c2 = np.searchsorted(vx, [n - nw, n - nw + 1])
    frac_rows = np.arange(nm, n - nw)
    perf1 = A[:, n - nw].nonzero()[0]
    perf1 = perf1[perf1 < n - nw]
    perf2 = A[:, n - nw + 1].nonzero()[0]
    perf2 = perf2[perf2 < n - nw]
    assert np.all(perf1 < nm) and np.any(perf2 >= nm)
    assert np.all(P[perf1[wb[perf1] != 3], c1] > 0)
    assert np.all(P[perf2[wb[perf2] != 3], c2] > 0)
    in_frac = np.abs(P[frac_rows, c1]).max()
    if variant in (fams.DECOUPLED, fams.FRAC):
        assert in_frac == 0.0
    elif variant == fams.ROCK:
        assert in_frac > 0.0
    assert np.abs(P[frac_rows, c2]).max() > 0.0


@pytest.mark.parametrize("variant", VARIANTS)
def test_wells_converge(variant):
    """GMRES with the F-AMS stage (wells as coarse nodes) reaches the direct
    solution of the system with rate-controlled wells."""
    sw, _, wb, _, vx = well_case()
    A = sw.csr()
    p_ref = spla.spsolve(A.tocsc(), sw.q)
    F = fams.FAMS(A, wb, vx, sw.n_matrix, variant, 1e-2, n_wells=sw.n_wells)
    p, info = F.gmres(sw.q, rtol=1e-11)
    assert info["status"] == fams.OK
    assert np.linalg.norm(p - p_ref) <= 1e-8 * np.linalg.norm(p_ref)


def test_restriction_and_media_with_wells():
    """MSMIX takes the finite-volume row for a well (its primal block is the
    well alone, so the row is the unit vector of the well), and the
    per-medium system keeps only the wells' diagonal."""
    sw, _, wb, pr, vx = well_case()
    n, nw = sw.n, sw.n_wells
    P = fams.prolongation(sw.csr(), wb, vx, sw.n_matrix, fams.COUPLED, n_wells=nw)
    R = fams.restriction(P, pr, vx, sw.n_matrix, fams.RESTRICT_MIX).toarray()
    for w in range(n - nw, n):
        c = int(np.searchsorted(vx, w))
        e = np.zeros(n)
        e[w] = 1.0
        assert np.array_equal(R[c], e)
    M = fams.media_blocks(sw.csr(), sw.n_matrix, nw)
    Mw = sp.csr_matrix(M)[n - nw:]
    assert Mw.nnz == nw and np.array_equal(Mw.indices, np.arange(n - nw, n))
    A = sw.csr()
    assert np.array_equal(M[n - nw:, n - nw:].toarray(), A[n - nw:, n - nw:].toarray())
