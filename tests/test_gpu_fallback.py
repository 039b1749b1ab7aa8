"""The precision form's FP64 re-solve of local blocks (a block whose FP32
factorisation meets a non-positive pivot is solved again in FP64).  Real
breakdowns are rare on these inputs, so FAMS_FORCE_FP64_BLOCKS=k sends every
block whose id is a multiple of k down that path: the fallback count is
reported, the re-solved rows equal the FP64 basis rounded to FP32, the
whole P still matches the oracle, and the solve reaches the oracle's
pressure."""
import os

import numpy as np
import pytest
import scipy.sparse as sp

from oracle import fams as ofams
from oracle import grids
from tests._cases import small_case

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _P(g, n, nc):
    rp, ci, va = g.prolongation()
    return sp.csr_matrix((va, ci, rp), shape=(n, nc)).toarray()


@pytest.mark.parametrize("variant", [0, 3])
def test_forced_fp64_resolve(variant):
    from paper_1705_05784_amd import fams
    print(f"[fallback] variant={variant}", flush=True)
    s, spec = small_case("3d")
    wb, pr, vx, _ = fams.full_grid(s, spec["coarse"], spec["d_min"], spec["r_z"])
    nc = len(vx)
    mk = lambda prec: fams.Solver(s.row_ptr, s.col, s.val, s.n_matrix, wb, pr, vx,  # noqa: E731
                                  variant=variant, precision=prec, alpha=0.0)
    g64 = mk(fams.FP64)
    g32 = mk(fams.MIXED)
    os.environ["FAMS_FORCE_FP64_BLOCKS"] = "3"
    try:
        gf = mk(fams.MIXED)
    finally:
        del os.environ["FAMS_FORCE_FP64_BLOCKS"]
    assert g32.setup_info()["fp32_fallback_blocks"] == 0
    assert gf.setup_info()["fp32_fallback_blocks"] > 0
    P64, P32, Pf = _P(g64, s.n, nc), _P(g32, s.n, nc), _P(gf, s.n, nc)
    og = grids.full_grid(s, spec["coarse"], spec["d_min"], spec["r_z"])
    ora = ofams.FAMS(s.csr(), og[0], og[2], s.n_matrix, variant, 0.0)
    assert np.abs(Pf - ora.P.toarray()).max() <= 1e-5
    # rows equal to the FP64 basis rounded to FP32
    r64 = P64.astype(np.float32).astype(np.float64)
    exact = lambda P: int(np.sum(np.all(np.abs(P - r64) <= 1e-7 * np.abs(r64) + 1e-30, axis=1)))  # noqa: E731
    assert exact(Pf) > exact(P32)
    p, info = gf.solve(torch.from_numpy(s.q), rtol=1e-10, max_iter=400)
    p_ora, _ = ora.gmres(s.q, rtol=1e-10)
    assert info[0]["status"] == 0
    assert np.linalg.norm(p.cpu().numpy() - p_ora) <= 1e-8 * np.linalg.norm(p_ora)
    for g in (g64, g32, gf):
        g.close()
