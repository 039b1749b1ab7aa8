"""Several right-hand sides on one setup, solved in lock-step (fams_solve with
nrhs > 1), against solves of one right-hand side at a time and against the
FP64 oracle.  Each column keeps its own outer iteration, so its iteration
count equals that of its own solve and its solution agrees with it to
rounding; the converged pressure matches the oracle's GMRES to 1e-8."""
import numpy as np
import pytest

from oracle import fams as ofams
from oracle import grids
from tests._cases import small_case

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def say(msg):
    print(msg, flush=True)


def rhs_set(s, k, seed=0):
    from workloads.serving import well_rhs
    rng = np.random.default_rng(seed)
    return np.stack([well_rhs(s, int(rng.integers(2, 9)), rng) for _ in range(k)])


def solver(name, variant, precision=0, alpha=1e-2, **kw):
    from paper_1705_05784_amd import fams
    s, spec = small_case(name)
    wb, pr, vx, _ = fams.full_grid(s, spec["coarse"], spec["d_min"], spec["r_z"])
    return s, spec, fams.Solver(s.row_ptr, s.col, s.val, s.n_matrix, wb, pr, vx, variant=variant,
                                precision=precision, alpha=alpha, **kw)


@pytest.mark.parametrize("outer", ["gmres", "richardson"])
@pytest.mark.parametrize("precision", [0, 1])
@pytest.mark.parametrize("variant", [0, 3])
@pytest.mark.parametrize("nrhs", [2, 3, 8, 17])
def test_lockstep_equals_single(nrhs, variant, precision, outer):
    """Columns of a lock-step solve equal their own single solves: the same
    iteration counts, pressures within 1e-10 relative (reduction order is the
    only difference), status OK everywhere."""
    say(f"[lockstep] nrhs={nrhs} variant={variant} precision={precision} outer={outer}")
    s, _, g = solver("3d", variant, precision)
    Q = rhs_set(s, nrhs, seed=nrhs)
    it_max = 400 if outer == "richardson" else 300
    P, info = g.solve(torch.from_numpy(Q), outer=outer, rtol=1e-10, max_iter=it_max)
    P = P.cpu().numpy()
    for r in range(nrhs):
        p1, i1 = g.solve(torch.from_numpy(Q[r]), outer=outer, rtol=1e-10, max_iter=it_max)
        p1 = p1.cpu().numpy()
        assert info[r]["status"] == 0 and i1[0]["status"] == 0
        assert abs(info[r]["iterations"] - i1[0]["iterations"]) <= 1, (r, info[r], i1[0])
        assert np.linalg.norm(P[r] - p1) <= 1e-9 * np.linalg.norm(p1), r
    g.close()


@pytest.mark.parametrize("variant", [0, 1, 2, 3])
def test_lockstep_matches_oracle(variant):
    """Eight right-hand sides in one lock-step group against the oracle's
    GMRES(30) on each: pressures within 1e-8, iterations within one."""
    say(f"[lockstep-oracle] variant={variant}")
    s, spec, g = solver("3d", variant, 0, alpha=0.0)
    og = grids.full_grid(s, spec["coarse"], spec["d_min"], spec["r_z"])
    ora = ofams.FAMS(s.csr(), og[0], og[2], s.n_matrix, variant, 0.0)
    Q = rhs_set(s, 8, seed=100 + variant)
    P, info = g.solve(torch.from_numpy(Q), outer="gmres", rtol=1e-10, max_iter=300)
    P = P.cpu().numpy()
    for r in range(8):
        pr, oi = ora.gmres(Q[r], rtol=1e-10)
        assert info[r]["status"] == 0
        assert abs(info[r]["iterations"] - oi["iterations"]) <= 1
        assert np.linalg.norm(P[r] - pr) <= 1e-8 * np.linalg.norm(pr)
    g.close()


def test_lockstep_initial_guess_and_uneven_convergence():
    """Initial guesses per column (the stopping test is relative to each
    column's own initial residual), a zero column that takes no iteration and
    stays zero, and columns that stop at different iterations: every column
    equals its own single solve from the same initial guess."""
    s, _, g = solver("3d", 3, 0)
    Q = rhs_set(s, 4, seed=7)
    Q[1] = 0.0
    Q[2] *= 1e-3
    p0, _ = g.solve(torch.from_numpy(Q[0]), rtol=1e-4, max_iter=300)
    P0 = np.zeros_like(Q)
    P0[0] = 0.5 * p0.cpu().numpy()
    P0[2] = 1e-4 * np.random.default_rng(3).standard_normal(s.n)
    P, info = g.solve(torch.from_numpy(Q), p=torch.from_numpy(P0.copy()), rtol=1e-10,
                      max_iter=300, use_initial_guess=True)
    P = P.cpu().numpy()
    assert info[1]["iterations"] == 0 and info[1]["status"] == 0
    assert not P[1].any()
    for r in (0, 2, 3):
        p1, i1 = g.solve(torch.from_numpy(Q[r]), p=torch.from_numpy(P0[r].copy()), rtol=1e-10,
                         max_iter=300, use_initial_guess=True)
        p1 = p1.cpu().numpy()
        assert info[r]["status"] == 0 and i1[0]["status"] == 0
        assert abs(info[r]["iterations"] - i1[0]["iterations"]) <= 1
        assert np.linalg.norm(P[r] - p1) <= 1e-9 * np.linalg.norm(p1)
    g.close()


@pytest.mark.parametrize("precision", [0, 1])
def test_lockstep_media_smoothing_and_fv_restriction(precision):
    """The per-medium smoothing stage and the MSFV restriction in lock-step
    give the single-column results."""
    s, _, g = solver("3d", 3, precision, smoother=2, restriction="fv")
    Q = rhs_set(s, 5, seed=11)
    P, info = g.solve(torch.from_numpy(Q), rtol=1e-10, max_iter=300)
    P = P.cpu().numpy()
    for r in range(5):
        p1, i1 = g.solve(torch.from_numpy(Q[r]), rtol=1e-10, max_iter=300)
        assert info[r]["status"] == 0
        assert abs(info[r]["iterations"] - i1[0]["iterations"]) <= 1
        assert np.linalg.norm(P[r] - p1.cpu().numpy()) <= 1e-9 * np.linalg.norm(p1.cpu().numpy())
    g.close()


@pytest.mark.parametrize("restart", [5, 40])
def test_lockstep_restart_lengths(restart):
    """Restart lengths on both sides of the fused Gram-Schmidt passes' basis
    limit (32 vectors; longer bases take the general kernels): the columns
    still equal their own single solves."""
    say(f"[lockstep] restart={restart}")
    s, _, g = solver("cfg2s", 3, 0)   # about 37 iterations at 1e-12: bases past 32 vectors
    Q = rhs_set(s, 4, seed=restart)
    P, info = g.solve(torch.from_numpy(Q), restart=restart, rtol=1e-12, max_iter=300)
    P = P.cpu().numpy()
    assert max(i["iterations"] for i in info) > 33
    for r in range(4):
        p1, i1 = g.solve(torch.from_numpy(Q[r]), restart=restart, rtol=1e-12, max_iter=300)
        p1 = p1.cpu().numpy()
        assert info[r]["status"] == 0 and i1[0]["status"] == 0
        assert abs(info[r]["iterations"] - i1[0]["iterations"]) <= 1, (r, info[r], i1[0])
        assert np.linalg.norm(P[r] - p1) <= 1e-9 * np.linalg.norm(p1), r
    g.close()


@pytest.mark.parametrize("outer", ["gmres", "richardson"])
def test_lockstep_group_of_32(outer):
    """33 right-hand sides: one group of 32 (32 rows per sweep chunk) and one
    padded group; every column equals its own single solve."""
    say(f"[lockstep] nrhs=33 outer={outer}")
    s, _, g = solver("3d", 3, 1)
    Q = rhs_set(s, 33, seed=33)
    it_max = 400 if outer == "richardson" else 300
    P, info = g.solve(torch.from_numpy(Q), outer=outer, rtol=1e-10, max_iter=it_max)
    P = P.cpu().numpy()
    for r in range(33):
        p1, i1 = g.solve(torch.from_numpy(Q[r]), outer=outer, rtol=1e-10, max_iter=it_max)
        p1 = p1.cpu().numpy()
        assert info[r]["status"] == 0 and i1[0]["status"] == 0
        assert abs(info[r]["iterations"] - i1[0]["iterations"]) <= 1, (r, info[r], i1[0])
        assert np.linalg.norm(P[r] - p1) <= 1e-9 * np.linalg.norm(p1), r
    g.close()


@pytest.mark.parametrize("precision", [0, 1])
def test_lockstep_tiled_row_order(precision):
    """An 80x70x12 grid: the lock-step products with A visit the matrix rows
    in slabs of 51 grid lines marched along z (the second slab 19 lines
    wide); every column still equals its own single solve."""
    from paper_1705_05784_amd import fams
    say(f"[lockstep] tiled 80x70x12 precision={precision}")
    s, spec = small_case("cfg2s", dims=(80, 70, 12), n_frac=20)
    wb, pr, vx, _ = fams.full_grid(s, spec["coarse"], spec["d_min"], spec["r_z"])
    g = fams.Solver(s.row_ptr, s.col, s.val, s.n_matrix, wb, pr, vx, variant=fams.COUPLED,
                    precision=precision, alpha=1e-2)
    assert g.setup_info()["tiled_rows"] == 0
    Q = rhs_set(s, 5, seed=5)
    P, info = g.solve(torch.from_numpy(Q), rtol=1e-10, max_iter=300)
    assert g.setup_info()["tiled_rows"] == s.n_matrix == 80 * 70 * 12
    P = P.cpu().numpy()
    for r in range(5):
        p1, i1 = g.solve(torch.from_numpy(Q[r]), rtol=1e-10, max_iter=300)
        p1 = p1.cpu().numpy()
        assert info[r]["status"] == 0 and i1[0]["status"] == 0
        assert abs(info[r]["iterations"] - i1[0]["iterations"]) <= 1, (r, info[r], i1[0])
        assert np.linalg.norm(P[r] - p1) <= 1e-9 * np.linalg.norm(p1), r
    g.close()
