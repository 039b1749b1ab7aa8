"""GPU parity: the HIP path through the C ABI against the FP64 oracle.

Every step is compared on the same seeded inputs: P (pattern bit-exact,
values to 1e-10), A_c (relative Frobenius 1e-12), the ILU(0) factors (1e-12),
one application of Table 1 steps 5-7 (1e-10), and converged solutions of the
Richardson loop and GMRES (1e-8 relative to the oracle and to a direct solve).
"""
import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spl

from oracle import fams as ofams
from oracle import grids
from tests._cases import small_case

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

VARIANTS = [0, 1, 2, 3]
_cache = {}


def say(msg):
    print(msg, flush=True)


def case(name, variant, alpha=0.0, precision=0, seed=0, **kw):
    key = (name, variant, alpha, precision, seed, tuple(sorted(kw.items())))
    if key in _cache:
        return _cache[key]
    from paper_1705_05784_amd import fams
    say(f"[case] {key}")
    s, spec = small_case(name, seed=seed, **kw)
    og = grids.full_grid(s, spec["coarse"], spec["d_min"], spec["r_z"])
    gg = fams.full_grid(s, spec["coarse"], spec["d_min"], spec["r_z"])
    for a, b in zip(og, gg):
        assert np.array_equal(np.asarray(a), np.asarray(b))
    wb, pr, vx, _ = gg
    gpu = fams.Solver(s.row_ptr, s.col, s.val, s.n_matrix, wb, pr, vx, variant=variant,
                      precision=precision, alpha=alpha)
    ora = ofams.FAMS(s.csr(), og[0], og[2], s.n_matrix, variant, alpha)
    _cache[key] = (s, gpu, ora)
    return _cache[key]


@pytest.mark.parametrize("alpha", [0.0, 1e-2])
@pytest.mark.parametrize("variant", VARIANTS)
@pytest.mark.parametrize("name", ["2d", "3d", "cfg2s"])
def test_prolongation(name, variant, alpha):
    s, gpu, ora = case(name, variant, alpha)
    rp, ci, va = gpu.prolongation()
    P = ora.P
    assert np.array_equal(rp, P.indptr)
    assert np.array_equal(ci, P.indices)
    assert np.abs(va - P.data).max() <= 1e-10


@pytest.mark.parametrize("variant", VARIANTS)
@pytest.mark.parametrize("name", ["2d", "3d", "cfg2s"])
def test_coarse_matrix(name, variant):
    s, gpu, ora = case(name, variant)
    Ac = gpu.coarse_matrix()
    assert np.linalg.norm(Ac - ora.Ac) <= 1e-12 * np.linalg.norm(ora.Ac)


@pytest.mark.parametrize("name", ["2d", "3d"])
def test_ilu_factors(name):
    s, gpu, ora = case(name, 0)
    lu = gpu.ilu()
    assert np.abs(lu - ora.ilu.val).max() <= 1e-12 * np.abs(ora.ilu.val).max()


@pytest.mark.parametrize("variant", VARIANTS)
@pytest.mark.parametrize("name", ["2d", "3d"])
def test_stage(name, variant):
    s, gpu, ora = case(name, variant)
    r = np.random.default_rng(7).standard_normal(s.n)
    z = gpu.apply_stage(torch.from_numpy(r)).cpu().numpy()
    zr = ora.stage(r)
    assert np.abs(z - zr).max() <= 1e-10 * np.abs(zr).max()


@pytest.mark.parametrize("outer", ["richardson", "gmres"])
@pytest.mark.parametrize("variant", VARIANTS)
@pytest.mark.parametrize("name", ["2d", "3d", "cfg2s"])
def test_solve(name, variant, outer):
    s, gpu, ora = case(name, variant)
    p, info = gpu.solve(torch.from_numpy(s.q), outer=outer, rtol=1e-10, max_iter=400)
    p = p.cpu().numpy()
    if outer == "gmres":
        pr, oi = ora.gmres(s.q, rtol=1e-10)
    else:
        pr, oi = ora.richardson(s.q, rtol=1e-10, max_iter=400)
    assert info[0]["status"] == 0
    assert abs(info[0]["iterations"] - oi["iterations"]) <= 1
    assert np.linalg.norm(p - pr) <= 1e-8 * np.linalg.norm(pr)
    # as close to the direct solution as the oracle's own iterate is
    pd = spl.spsolve(s.csr().tocsc(), s.q)
    e_gpu = np.linalg.norm(p - pd) / np.linalg.norm(pd)
    e_ora = np.linalg.norm(pr - pd) / np.linalg.norm(pd)
    assert e_gpu <= max(2.0 * e_ora, 1e-9)


@pytest.mark.parametrize("variant", VARIANTS)
def test_mixed_precision_reaches_fp64_accuracy(variant):
    s, gpu, ora = case("3d", variant, 1e-2, precision=1)
    p, info = gpu.solve(torch.from_numpy(s.q), outer="gmres", rtol=1e-10, max_iter=400)
    assert info[0]["status"] == 0
    pd = spl.spsolve(s.csr().tocsc(), s.q)
    assert np.linalg.norm(p.cpu().numpy() - pd) <= 1e-8 * np.linalg.norm(pd)


def test_deterministic():
    from paper_1705_05784_amd import fams
    s, spec = small_case("3d", seed=1)
    wb, pr, vx, _ = fams.full_grid(s, spec["coarse"], spec["d_min"], spec["r_z"])
    outs = []
    for _ in range(2):
        g = fams.Solver(s.row_ptr, s.col, s.val, s.n_matrix, wb, pr, vx, variant=3, alpha=1e-2)
        p, _ = g.solve(torch.from_numpy(s.q), rtol=1e-8)
        outs.append((g.prolongation()[2], g.coarse_matrix(), p.cpu().numpy()))
        g.close()
    for a, b in zip(*outs):
        assert np.array_equal(a, b)


@pytest.mark.parametrize("variant", VARIANTS)
@pytest.mark.parametrize("name", ["2d", "3d"])
def test_flux_reconstruction(name, variant):
    """GPU flux vs the oracle's reconstruction from the same pressure: the FV
    pressure p' and the fluxes agree, and every cell balances to 1e-10."""
    from oracle import flux as oflux
    s, gpu, ora = case(name, variant)
    p, _ = gpu.solve(torch.from_numpy(s.q), rtol=1e-6)
    fl, pfv, imb = gpu.reconstruct_flux(torch.from_numpy(s.q), p)
    spec_grid = grids.full_grid(s, *[small_case(name)[1][k] for k in ("coarse", "d_min", "r_z")])
    fr, p1, p2, imr = oflux.reconstruct_flux(ora.A, ora.P, spec_grid[1], spec_grid[2], s.q,
                                             p.cpu().numpy())
    assert imb <= 1e-10
    assert np.abs(pfv.cpu().numpy() - p1).max() <= 1e-9 * np.abs(p1).max()
    assert np.abs(fl.cpu().numpy() - fr).max() <= 1e-8 * np.abs(fr).max()


@pytest.mark.parametrize("variant", VARIANTS)
@pytest.mark.parametrize("name,lds_limit", [("3d", 24576), ("3d", 49152), ("cfg2s", 65536)])
def test_global_band_modes(name, lds_limit, variant, monkeypatch):
    """A lowered LDS budget moves the local blocks (basis and Neumann solves)
    to the blocked global-memory factorisations; P, the FV pressure and the
    fluxes still match the oracle."""
    from paper_1705_05784_amd import fams
    from oracle import flux as oflux
    s, gpu0, ora = case(name, variant)
    spec = small_case(name)[1]
    wb, pr, vx, _ = grids.full_grid(s, spec["coarse"], spec["d_min"], spec["r_z"])
    monkeypatch.setenv("FAMS_LDS_LIMIT", str(lds_limit))
    say(f"[case] {name} variant {variant} lds_limit {lds_limit}")
    gpu = fams.Solver(s.row_ptr, s.col, s.val, s.n_matrix, wb, pr, vx, variant=variant)
    rp, ci, va = gpu.prolongation()
    assert np.array_equal(rp, ora.P.indptr)
    assert np.array_equal(ci, ora.P.indices)
    assert np.abs(va - ora.P.data).max() <= 1e-10
    p, _ = gpu.solve(torch.from_numpy(s.q), rtol=1e-6)
    fl, pfv, imb = gpu.reconstruct_flux(torch.from_numpy(s.q), p)
    og = grids.full_grid(s, spec["coarse"], spec["d_min"], spec["r_z"])
    fr, p1, p2, imr = oflux.reconstruct_flux(ora.A, ora.P, og[1], og[2], s.q, p.cpu().numpy())
    assert imb <= 1e-10
    assert np.abs(pfv.cpu().numpy() - p1).max() <= 1e-9 * np.abs(p1).max()
    assert np.abs(fl.cpu().numpy() - fr).max() <= 1e-8 * np.abs(fr).max()


@pytest.mark.parametrize("range_rows", [0, 64, 1000, 16384])
@pytest.mark.parametrize("name", ["3d", "cfg2s"])
def test_sweep_schedules(name, range_rows, monkeypatch):
    """ILU(0) applied by level chunks (0) or by row ranges of several sizes
    (small ranges make most dependencies cross ranges): the two-stage
    step matches the oracle, and every schedule gives the same bits."""
    from paper_1705_05784_amd import fams
    s, gpu0, ora = case(name, 0)
    spec = small_case(name)[1]
    wb, pr, vx, _ = grids.full_grid(s, spec["coarse"], spec["d_min"], spec["r_z"])
    monkeypatch.setenv("FAMS_ILU_RANGE", str(range_rows))
    say(f"[case] {name} ilu range rows {range_rows}")
    gpu = fams.Solver(s.row_ptr, s.col, s.val, s.n_matrix, wb, pr, vx, variant=0)
    r = np.random.default_rng(7).standard_normal(s.n)
    z = gpu.apply_stage(torch.from_numpy(r)).cpu().numpy()
    zr = ora.stage(r)
    assert np.abs(z - zr).max() <= 1e-10 * np.abs(zr).max()
    z0 = gpu0.apply_stage(torch.from_numpy(r)).cpu().numpy()
    assert np.array_equal(z, z0)
    gm = fams.Solver(s.row_ptr, s.col, s.val, s.n_matrix, wb, pr, vx, variant=0,
                     precision=fams.MIXED)
    p, info = gm.solve(torch.from_numpy(s.q), rtol=1e-10)
    assert info[0]["status"] == 0


@pytest.mark.parametrize("stage", [0, 5])
@pytest.mark.parametrize("range_rows", [64, 8192])
@pytest.mark.parametrize("name", ["3d", "cfg2s"])
def test_ilu_factor_forms(name, range_rows, stage, monkeypatch):
    """The one-launch ILU(0) factorisation with every row taken entry by
    entry (stage 0), or only the rows past 5 entries (stage 5, both forms in
    one launch), on small and large ranges, gives the same bits as the
    per-level IKJ launches and matches the oracle."""
    from paper_1705_05784_amd import fams
    s, _, ora = case(name, 0)
    spec = small_case(name)[1]
    wb, pr, vx, _ = grids.full_grid(s, spec["coarse"], spec["d_min"], spec["r_z"])
    monkeypatch.setenv("FAMS_ILU_RANGE", "0")
    ref = fams.Solver(s.row_ptr, s.col, s.val, s.n_matrix, wb, pr, vx, variant=0).ilu()
    monkeypatch.setenv("FAMS_ILU_RANGE", str(range_rows))
    monkeypatch.setenv("FAMS_ILU_STAGE", str(stage))
    say(f"[case] {name} ilu range rows {range_rows} stage width {stage}")
    lu = fams.Solver(s.row_ptr, s.col, s.val, s.n_matrix, wb, pr, vx, variant=0).ilu()
    assert np.array_equal(lu, ref)
    assert np.abs(lu - ora.ilu.val).max() <= 1e-12 * np.abs(ora.ilu.val).max()


@pytest.mark.parametrize("precision", [0, 1])
@pytest.mark.parametrize("kind", [1, 2])
@pytest.mark.parametrize("variant", [0, 3])
@pytest.mark.parametrize("name", ["2d", "3d"])
def test_restriction_forms(name, variant, kind, precision):
    """MSFV (kind 1) and MSMIX (kind 2) restrictions (Sec. 3.2): R, A_c = R A P
    and its pivoted-LU inverse built on the GPU give the oracle's two-stage
    step (FP64 form, 1e-10), and GMRES reaches the oracle's solution (1e-8;
    the precision form to the same tolerance after convergence)."""
    from paper_1705_05784_amd import fams
    s, spec = small_case(name)
    wb, primal, vertex, _ = grids.full_grid(s, spec["coarse"], spec["d_min"], spec["r_z"])
    say(f"[case] {name} variant {variant} restriction {kind} precision {precision}")
    gpu = fams.Solver(s.row_ptr, s.col, s.val, s.n_matrix, wb, primal, vertex, variant=variant,
                      precision=precision, restriction=kind)
    ora = ofams.FAMS(s.csr(), wb, vertex, s.n_matrix, variant, primal=primal,
                     restriction_kind=kind)
    if precision == 0:
        r = np.random.default_rng(11).standard_normal(s.n)
        z = gpu.apply_stage(torch.from_numpy(r)).cpu().numpy()
        zr = ora.stage(r)
        assert np.abs(z - zr).max() <= 1e-10 * np.abs(zr).max()
    p, info = gpu.solve(torch.from_numpy(s.q), outer="gmres", rtol=1e-10, max_iter=400)
    p = p.cpu().numpy()
    pr, oi = ora.gmres(s.q, rtol=1e-10)
    assert info[0]["status"] == 0
    if precision == 0:
        assert abs(info[0]["iterations"] - oi["iterations"]) <= 1
    assert np.linalg.norm(p - pr) <= 1e-8 * np.linalg.norm(pr)
    gpu.close()


@pytest.mark.parametrize("iters", [1, 3])
@pytest.mark.parametrize("name", ["2d", "3d"])
def test_approximate_mode(name, iters):
    """A few F-AMS iterations with the MSFV restriction, then the flux
    reconstruction (Sec. 4.6: an approximate, conservative solution): the
    unconverged iterate still yields a flux field whose every cell balances
    (1e-10), equal to the oracle's reconstruction from the same pressure."""
    from oracle import flux as oflux
    from paper_1705_05784_amd import fams
    s, spec = small_case(name)
    wb, primal, vertex, _ = grids.full_grid(s, spec["coarse"], spec["d_min"], spec["r_z"])
    say(f"[case] {name} MSFV, {iters} iterations, then flux")
    gpu = fams.Solver(s.row_ptr, s.col, s.val, s.n_matrix, wb, primal, vertex,
                      restriction=fams.RESTRICT_FV)
    ora = ofams.FAMS(s.csr(), wb, vertex, s.n_matrix, 0, primal=primal,
                     restriction_kind=ofams.RESTRICT_FV)
    p, info = gpu.solve(torch.from_numpy(s.q), outer="richardson", rtol=1e-14, max_iter=iters)
    assert info[0]["status"] == 1 and info[0]["iterations"] == iters  # not converged
    fl, pfv, imb = gpu.reconstruct_flux(torch.from_numpy(s.q), p)
    fr, p1, _, _ = oflux.reconstruct_flux(ora.A, ora.P, primal, vertex, s.q, p.cpu().numpy())
    assert imb <= 1e-10
    assert np.abs(pfv.cpu().numpy() - p1).max() <= 1e-9 * np.abs(p1).max()
    assert np.abs(fl.cpu().numpy() - fr).max() <= 1e-8 * np.abs(fr).max()
    pr, _ = ora.richardson(s.q, rtol=1e-14, max_iter=iters)
    assert np.linalg.norm(p.cpu().numpy() - pr) <= 1e-9 * np.linalg.norm(pr)
    gpu.close()


@pytest.mark.parametrize("precision", [0, 1])
@pytest.mark.parametrize("variant", [0, 3])
@pytest.mark.parametrize("name", ["2d", "3d", "cfg2s"])
def test_media_smoothing(name, variant, precision):
    """Smoother 2: ILU(0), then one ILU(0) application of diag(A^mm, A^ff)
    to the updated residual (Sec. 3.2).  The two-stage step matches the
    oracle's (FP64 form, 1e-10) and GMRES reaches the oracle's solution
    (1e-8) in both forms, with iteration counts within 1 in FP64."""
    from paper_1705_05784_amd import fams
    s, spec = small_case(name)
    wb, primal, vertex, _ = grids.full_grid(s, spec["coarse"], spec["d_min"], spec["r_z"])
    say(f"[case] {name} variant {variant} media smoothing precision {precision}")
    gpu = fams.Solver(s.row_ptr, s.col, s.val, s.n_matrix, wb, primal, vertex, variant=variant,
                      precision=precision, smoother=2)
    ora = ofams.FAMS(s.csr(), wb, vertex, s.n_matrix, variant, media_smoothing=True)
    if precision == 0:
        r = np.random.default_rng(13).standard_normal(s.n)
        z = gpu.apply_stage(torch.from_numpy(r)).cpu().numpy()
        zr = ora.stage(r)
        assert np.abs(z - zr).max() <= 1e-10 * np.abs(zr).max()
    p, info = gpu.solve(torch.from_numpy(s.q), outer="gmres", rtol=1e-10, max_iter=400)
    p = p.cpu().numpy()
    pr, oi = ora.gmres(s.q, rtol=1e-10)
    assert info[0]["status"] == 0
    if precision == 0:
        assert abs(info[0]["iterations"] - oi["iterations"]) <= 1
    assert np.linalg.norm(p - pr) <= 1e-8 * np.linalg.norm(pr)
    gpu.close()


def _scaled_values(s, amp, seed=0):
    """A's values with every transmissibility scaled by 1 + amp sin(i + j +
    seed) (symmetric) and the diagonal moved so that every row sum is kept:
    still a TPFA M-matrix with the same boundary terms (a permeability
    change), in A's CSR slots."""
    rows = np.repeat(np.arange(s.n), np.diff(s.row_ptr))
    off = rows != s.col
    v = s.val.copy()
    v[off] *= 1.0 + amp * np.sin(rows[off] + s.col[off] + seed)
    moved = np.bincount(rows[off], weights=(v - s.val)[off], minlength=s.n)
    v[~off] -= moved[rows[~off]]
    return v


@pytest.mark.parametrize("precision", [0, 1])
@pytest.mark.parametrize("variant", [0, 3])
@pytest.mark.parametrize("name", ["2d", "3d"])
def test_update_recompute_matches_fresh_setup(name, variant, precision):
    """fams_update_values with a recomputed basis leaves the handle exactly
    as a fresh setup on the new values: P, A_c, the ILU(0) factors, one stage
    and the reconstructed fluxes agree bit for bit (no stale state)."""
    from paper_1705_05784_amd import fams
    s, spec = small_case(name)
    wb, primal, vertex, _ = grids.full_grid(s, spec["coarse"], spec["d_min"], spec["r_z"])
    say(f"[case] {name} variant {variant} update (recompute) precision {precision}")
    v2 = _scaled_values(s, 0.2)
    g = fams.Solver(s.row_ptr, s.col, s.val, s.n_matrix, wb, primal, vertex, variant=variant,
                    precision=precision)
    r = np.random.default_rng(17).standard_normal(s.n)
    g.apply_stage(torch.from_numpy(r))
    g.reconstruct_flux(torch.from_numpy(s.q), torch.zeros(s.n, dtype=torch.float64))
    assert g.update_values(v2, threshold=0.01)
    f = fams.Solver(s.row_ptr, s.col, v2, s.n_matrix, wb, primal, vertex, variant=variant,
                    precision=precision)
    for a, b in zip(g.prolongation(), f.prolongation()):
        assert np.array_equal(a, b)
    assert np.array_equal(g.coarse_matrix(), f.coarse_matrix())
    assert np.array_equal(g.ilu(), f.ilu())
    za = g.apply_stage(torch.from_numpy(r)).cpu().numpy()
    zb = f.apply_stage(torch.from_numpy(r)).cpu().numpy()
    assert np.array_equal(za, zb)
    p = torch.from_numpy(np.random.default_rng(19).standard_normal(s.n))
    fa = g.reconstruct_flux(torch.from_numpy(s.q), p)
    fb = f.reconstruct_flux(torch.from_numpy(s.q), p)
    assert np.array_equal(fa[0].cpu().numpy(), fb[0].cpu().numpy())
    g.close()
    f.close()


@pytest.mark.parametrize("variant", [0, 3])
@pytest.mark.parametrize("name", ["2d", "3d", "cfg2s"])
def test_update_kept_basis(name, variant):
    """Below the threshold the basis stays: the GPU keeps P and rebuilds A_c,
    its inverse and ILU(0) from the new A, like the oracle's update (one stage
    1e-10, GMRES 1e-8 and within one iteration)."""
    from paper_1705_05784_amd import fams
    s, spec = small_case(name)
    wb, primal, vertex, _ = grids.full_grid(s, spec["coarse"], spec["d_min"], spec["r_z"])
    say(f"[case] {name} variant {variant} update (basis kept)")
    v2 = _scaled_values(s, 0.3, seed=1)
    g = fams.Solver(s.row_ptr, s.col, s.val, s.n_matrix, wb, primal, vertex, variant=variant)
    ora = ofams.FAMS(s.csr(), wb, vertex, s.n_matrix, variant)
    P0 = g.prolongation()
    assert not g.update_values(v2, threshold=1e9)
    A2 = sp.csr_matrix((v2, s.col, s.row_ptr), shape=(s.n, s.n))
    assert not ora.update_values(A2, threshold=1e9)
    for a, b in zip(g.prolongation(), P0):
        assert np.array_equal(a, b)
    r = np.random.default_rng(23).standard_normal(s.n)
    z = g.apply_stage(torch.from_numpy(r)).cpu().numpy()
    zr = ora.stage(r)
    assert np.abs(z - zr).max() <= 1e-10 * np.abs(zr).max()
    p, info = g.solve(torch.from_numpy(s.q), outer="gmres", rtol=1e-10, max_iter=400)
    pr, oi = ora.gmres(s.q, rtol=1e-10)
    assert info[0]["status"] == 0
    assert abs(info[0]["iterations"] - oi["iterations"]) <= 1
    assert np.linalg.norm(p.cpu().numpy() - pr) <= 1e-8 * np.linalg.norm(pr)
    g.close()


def test_flux_weakly_coupled_boundary():
    """Low-permeability Dirichlet cells beside fractures 1e7 times more
    conductive: their blocks have real (tiny) row sums and are not pinned,
    on the GPU as in the oracle (whose reading is pinned in
    test_oracle_solve.py): the balance stays at FP64's floor for the case
    and the FV pressure matches the oracle's."""
    from oracle import flux as oflux
    from paper_1705_05784_amd import fams
    from tests.test_oracle_solve import _weak_boundary_case
    s, spec = _weak_boundary_case()
    wb, pr, vx, _ = grids.full_grid(s, spec["coarse"], spec["d_min"], spec["r_z"])
    say("[case] weak boundary, contrast 1e7")
    gpu = fams.Solver(s.row_ptr, s.col, s.val, s.n_matrix, wb, pr, vx, variant=3, alpha=1e-2)
    ora = ofams.FAMS(s.csr(), wb, vx, s.n_matrix, 3, 1e-2)
    p, _ = gpu.solve(torch.from_numpy(s.q), rtol=1e-4)
    fl, pfv, imb = gpu.reconstruct_flux(torch.from_numpy(s.q), p)
    _, p1, _, imr = oflux.reconstruct_flux(ora.A, ora.P, pr, vx, s.q, p.cpu().numpy())
    assert imb <= 1e-8 and imr <= 1e-8
    assert np.abs(pfv.cpu().numpy() - p1).max() <= 1e-9 * np.abs(p1).max()
    gpu.close()
