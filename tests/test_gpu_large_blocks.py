"""Fracture networks dense enough that dual blocks percolate through plate
intersections into components above the LDS ordering limit (global-memory
breadth-first ordering, wide-panel elimination): every coupling strategy
still solves the system (against a sparse direct solve) and conserves mass."""
import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla
import torch

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dense_network():
    from workloads.serving import make_system
    s = make_system(40, 300, 1e4, 3)
    A = sp.csr_matrix((s.val, s.col, s.row_ptr), shape=(s.n, s.n)).tocsc()
    return s, spla.splu(A).solve(s.q)


@pytest.mark.parametrize("variant", [0, 1, 2, 3])
def test_percolating_blocks(dense_network, variant):
    from paper_1705_05784_amd import fams
    s, p_ref = dense_network
    wb, pr, vx, _ = fams.full_grid(s, (10, 10, 10), 8, 8)
    print(f"[large] variant {variant} n={s.n}", flush=True)
    S = fams.Solver(s.row_ptr, s.col, s.val, s.n_matrix, wb, pr, vx, variant=variant,
                    precision=fams.MIXED, alpha=1e-2)
    info = S.setup_info()
    q = torch.from_numpy(s.q)
    p, st = S.solve(q, rtol=1e-10, max_iter=2000)
    _, _, imb = S.reconstruct_flux(q, p)
    err = np.linalg.norm(p.cpu().numpy() - p_ref) / np.linalg.norm(p_ref)
    print(f"  max block {info['max_block']} iterations {st[0]['iterations']} err {err:.2e} "
          f"balance {imb:.2e}", flush=True)
    assert info["max_block"] > 6144
    assert st[0]["status"] == 0
    assert err <= 1e-6
    assert imb <= 1e-10
