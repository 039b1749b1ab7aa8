"""Wells as coarse nodes on the GPU against the oracle (the oracle's well
handling is pinned in test_oracle_wells.py): the grid helpers, P (pattern
bit-exact, values to 1e-10), A_c (1e-12), one stage (1e-10), the converged
pressure (1e-8, iterations within one in FP64), the flux reconstruction, the
per-medium smoothing stage and the MSMIX restriction with wells, and a
lock-step solve of several right-hand sides."""
import numpy as np
import pytest

from oracle import fams as ofams
from oracle import grids
from tests._cases import wells_case

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

VARIANTS = [0, 1, 2, 3]
_cache = {}


def say(msg):
    print(msg, flush=True)


def system(name):
    if name not in _cache:
        from paper_1705_05784_amd import fams
        sw, spec = wells_case(name)
        args = (spec["coarse"], spec["d_min"], spec["r_z"])
        og = grids.full_grid(sw, *args)
        gg = fams.full_grid(sw, *args)
        for a, b in zip(og, gg):
            assert np.array_equal(np.asarray(a), np.asarray(b))
        _cache[name] = (sw, og)
    return _cache[name]


def pair(name, variant, alpha=0.0, precision=0, **kw):
    from paper_1705_05784_amd import fams
    sw, og = system(name)
    wb, pr, vx, _ = og
    say(f"[wells] {name} variant={variant} alpha={alpha} precision={precision} {kw}")
    gkw = {k: v for k, v in kw.items() if k in ("smoother", "restriction")}
    okw = {}
    if kw.get("smoother") == 2:
        okw["media_smoothing"] = True
    if kw.get("restriction"):
        okw["restriction_kind"] = kw["restriction"]
        okw["primal"] = pr
    gpu = fams.Solver(sw.row_ptr, sw.col, sw.val, sw.n_matrix, wb, pr, vx, variant=variant,
                      precision=precision, alpha=alpha, n_wells=sw.n_wells, **gkw)
    ora = ofams.FAMS(sw.csr(), wb, vx, sw.n_matrix, variant, alpha, n_wells=sw.n_wells, **okw)
    return sw, gpu, ora


@pytest.mark.parametrize("alpha", [0.0, 1e-2])
@pytest.mark.parametrize("variant", VARIANTS)
@pytest.mark.parametrize("name", ["2d", "3d", "cfg2s"])
def test_wells_prolongation_and_coarse(name, variant, alpha):
    sw, gpu, ora = pair(name, variant, alpha)
    rp, ci, va = gpu.prolongation()
    assert np.array_equal(rp, ora.P.indptr)
    assert np.array_equal(ci, ora.P.indices)
    assert np.abs(va - ora.P.data).max() <= 1e-10
    Ac = gpu.coarse_matrix()
    assert np.linalg.norm(Ac - ora.Ac) <= 1e-12 * np.linalg.norm(ora.Ac)
    r = np.random.default_rng(variant).standard_normal(sw.n)
    z = gpu.apply_stage(torch.from_numpy(r)).cpu().numpy()
    zr = ora.stage(r)
    assert np.abs(z - zr).max() <= 1e-10 * np.abs(zr).max()
    gpu.close()


@pytest.mark.parametrize("precision", [0, 1])
@pytest.mark.parametrize("variant", VARIANTS)
@pytest.mark.parametrize("name", ["3d", "cfg2s"])
def test_wells_solve(name, variant, precision):
    sw, gpu, ora = pair(name, variant, 1e-2, precision)
    p, info = gpu.solve(torch.from_numpy(sw.q), rtol=1e-10, max_iter=400)
    pr, oi = ora.gmres(sw.q, rtol=1e-10)
    assert info[0]["status"] == 0 and oi["status"] == 0
    if precision == 0:
        assert abs(info[0]["iterations"] - oi["iterations"]) <= 1
    assert np.linalg.norm(p.cpu().numpy() - pr) <= 1e-8 * np.linalg.norm(pr)
    gpu.close()


@pytest.mark.parametrize("variant", VARIANTS)
def test_wells_flux(variant):
    """The conservative flux with wells (each well a primal block of its
    own): the FV pressure and fluxes equal the oracle's from the same
    pressure, and every cell and well balances to 1e-10."""
    from oracle import flux as oflux
    sw, gpu, ora = pair("3d", variant)
    _, og = system("3d")
    p, _ = gpu.solve(torch.from_numpy(sw.q), rtol=1e-6)
    fl, pfv, imb = gpu.reconstruct_flux(torch.from_numpy(sw.q), p)
    fr, p1, _, imr = oflux.reconstruct_flux(ora.A, ora.P, og[1], og[2], sw.q, p.cpu().numpy())
    assert imb <= 1e-10 and imr <= 1e-10
    assert np.abs(pfv.cpu().numpy() - p1).max() <= 1e-9 * np.abs(p1).max()
    assert np.abs(fl.cpu().numpy() - fr).max() <= 1e-8 * np.abs(fr).max()
    gpu.close()


@pytest.mark.parametrize("precision", [0, 1])
@pytest.mark.parametrize("form", ["media", "mix"])
def test_wells_stage_forms(form, precision):
    """The per-medium smoothing stage (wells keep only their diagonal) and the
    MSMIX restriction (a well's row is its unit vector) with wells: one stage
    against the oracle (FP64 form), and the converged pressure."""
    kw = dict(smoother=2) if form == "media" else dict(restriction=ofams.RESTRICT_MIX)
    sw, gpu, ora = pair("3d", 3, 1e-2, precision, **kw)
    if precision == 0:
        r = np.random.default_rng(7).standard_normal(sw.n)
        z = gpu.apply_stage(torch.from_numpy(r)).cpu().numpy()
        zr = ora.stage(r)
        assert np.abs(z - zr).max() <= 1e-10 * np.abs(zr).max()
    p, info = gpu.solve(torch.from_numpy(sw.q), rtol=1e-10, max_iter=400)
    pr, oi = ora.gmres(sw.q, rtol=1e-10)
    assert info[0]["status"] == 0
    assert np.linalg.norm(p.cpu().numpy() - pr) <= 1e-8 * np.linalg.norm(pr)
    gpu.close()


def test_wells_lockstep():
    """Several right-hand sides with wells (different well rates) in one
    lock-step group equal their own single solves."""
    sw, gpu, _ = pair("cfg2s", 3, 1e-2)
    rng = np.random.default_rng(3)
    Q = np.stack([sw.q.copy() for _ in range(4)])
    Q[:, sw.n - sw.n_wells:] = rng.uniform(-2.0, 2.0, size=(4, sw.n_wells))
    P, info = gpu.solve(torch.from_numpy(Q), rtol=1e-10, max_iter=300)
    P = P.cpu().numpy()
    for r in range(4):
        p1, i1 = gpu.solve(torch.from_numpy(Q[r]), rtol=1e-10, max_iter=300)
        assert info[r]["status"] == 0 and abs(info[r]["iterations"] - i1[0]["iterations"]) <= 1
        p1 = p1.cpu().numpy()
        assert np.linalg.norm(P[r] - p1) <= 1e-9 * np.linalg.norm(p1)
    gpu.close()
