"""Non-symmetric A on the GPU (the compressible Jacobian of
workloads.compressible; banded LU local solves without pivoting and the
pivoted-LU coarse inverse) against the oracle (pinned on non-symmetric
matrices in test_oracle_nonsym.py): P (pattern bit-exact, values 1e-10), A_c
(1e-12), one stage (1e-10), the converged correction (1e-8), both precision
forms; lock-step right-hand sides; a Newton loop with the value update
against Newton with direct solves; and the flux reconstruction refused."""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

from oracle import fams as ofams
from oracle import grids
from tests._cases import small_case
from workloads.compressible import newton_direct, residual_jacobian

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

VARIANTS = [0, 1, 2, 3]


def say(msg):
    print(msg, flush=True)


_cache = {}


def jac(name):
    if name not in _cache:
        s, spec = small_case(name)
        p_old = spla.spsolve(s.csr().tocsc(), s.q)
        p = p_old + 0.05 * np.random.default_rng(1).standard_normal(s.n)
        R, J = residual_jacobian(s, p, p_old - 0.1)
        g = grids.full_grid(s, spec["coarse"], spec["d_min"], spec["r_z"])
        _cache[name] = (s, spec, R, J, g)
    return _cache[name]


def solver(s, J, g, variant, precision=0, alpha=1e-2):
    from paper_1705_05784_amd import fams
    wb, pr, vx, _ = g
    return fams.Solver(J.indptr, J.indices, J.data, s.n_matrix, wb, pr, vx, variant=variant,
                       precision=precision, alpha=alpha, nonsymmetric=True)


@pytest.mark.parametrize("precision", [0, 1])
@pytest.mark.parametrize("variant", VARIANTS)
@pytest.mark.parametrize("name", ["2d", "3d", "cfg2s"])
def test_nonsymmetric_parity(name, variant, precision):
    s, spec, R, J, g = jac(name)
    say(f"[nonsym] {name} variant={variant} precision={precision}")
    gpu = solver(s, J, g, variant, precision)
    ora = ofams.FAMS(J, g[0], g[2], s.n_matrix, variant, 1e-2)
    if precision == 0:   # the precision form's FP32 basis may truncate differently
        rp, ci, va = gpu.prolongation()
        assert np.array_equal(rp, ora.P.indptr)
        assert np.array_equal(ci, ora.P.indices)
        assert np.abs(va - ora.P.data).max() <= 1e-10
        Ac = gpu.coarse_matrix()
        assert np.linalg.norm(Ac - ora.Ac) <= 1e-12 * np.linalg.norm(ora.Ac)
        r = np.random.default_rng(variant).standard_normal(s.n)
        z = gpu.apply_stage(torch.from_numpy(r)).cpu().numpy()
        zr = ora.stage(r)
        assert np.abs(z - zr).max() <= 1e-10 * np.abs(zr).max()
    d, info = gpu.solve(torch.from_numpy(-R), rtol=1e-10, max_iter=400)
    dr, oi = ora.gmres(-R, rtol=1e-10)
    assert info[0]["status"] == 0 and oi["status"] == 0
    if precision == 0:
        assert abs(info[0]["iterations"] - oi["iterations"]) <= 1
    assert np.linalg.norm(d.cpu().numpy() - dr) <= 1e-8 * np.linalg.norm(dr)
    gpu.close()


def test_nonsymmetric_lockstep():
    s, spec, R, J, g = jac("cfg2s")
    gpu = solver(s, J, g, 3)
    Q = np.stack([-R * (1.0 + 0.1 * k) + 0.01 * np.random.default_rng(k).standard_normal(s.n)
                  for k in range(4)])
    P, info = gpu.solve(torch.from_numpy(Q), rtol=1e-10, max_iter=300)
    P = P.cpu().numpy()
    for r in range(4):
        p1, i1 = gpu.solve(torch.from_numpy(Q[r]), rtol=1e-10, max_iter=300)
        assert info[r]["status"] == 0 and abs(info[r]["iterations"] - i1[0]["iterations"]) <= 1
        p1 = p1.cpu().numpy()
        assert np.linalg.norm(P[r] - p1) <= 1e-9 * np.linalg.norm(p1)
    gpu.close()


@pytest.mark.parametrize("precision", [0, 1])
@pytest.mark.parametrize("threshold", [0.0, 0.05, -1.0])
def test_newton_loop(threshold, precision):
    """Table 1 as a Newton loop on the GPU: each outer iteration hands the new
    Jacobian to fams_update_values (basis recomputed above `threshold`;
    negative: always) and solves for the correction; the iterates reach the
    direct-solve Newton solution (1e-8) in as many iterations."""
    from paper_1705_05784_amd import fams
    s, spec = small_case("cfg2s")
    wb, pr, vx, _ = grids.full_grid(s, spec["coarse"], spec["d_min"], spec["r_z"])
    p_old = spla.spsolve(s.csr().tocsc(), s.q)
    p_ref, hist = newton_direct(s, p_old, p_old - 0.1)
    say(f"[newton] threshold={threshold} precision={precision} reference its={len(hist)}")
    p = p_old.copy()
    S = None
    norms, recomputed = [], []
    for _ in range(20):
        R, J = residual_jacobian(s, p, p_old - 0.1)
        norms.append(float(np.linalg.norm(R)))
        if norms[-1] <= 1e-10 * norms[0]:
            break
        if S is None:
            S = fams.Solver(J.indptr, J.indices, J.data, s.n_matrix, wb, pr, vx, variant=3,
                            precision=precision, alpha=1e-2, nonsymmetric=True)
        else:
            recomputed.append(S.update_values(J.data, threshold))
        d, info = S.solve(torch.from_numpy(-R), rtol=1e-12, max_iter=400)
        assert info[0]["status"] == 0
        p = p + d.cpu().numpy()
    S.close()
    assert len(norms) == len(hist)
    assert np.linalg.norm(p - p_ref) <= 1e-8 * np.linalg.norm(p_ref)
    if threshold < 0:
        assert all(recomputed)


def test_flux_refused():
    from paper_1705_05784_amd import fams
    s, spec, R, J, g = jac("3d")
    gpu = solver(s, J, g, 0)
    d, _ = gpu.solve(torch.from_numpy(-R), rtol=1e-8)
    with pytest.raises(fams.FamsError):
        gpu.reconstruct_flux(torch.from_numpy(-R), d)
    gpu.close()
