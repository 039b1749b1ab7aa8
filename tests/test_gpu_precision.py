"""Precision form across fracture/matrix contrasts (the 2M-cell workload's
shapes at reduced size): mixed FP32/FP64 and plain FP64, iterated to 1e-10,
both against a sparse direct solve of the same system, and the per-cell mass
balance of the reconstructed flux.  Iterations stop at 1e-10 or after 1500."""
import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla
import torch

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("contrast", [1e2, 1e4, 1e6, 1e8])
def test_contrast_sweep(contrast):
    from paper_1705_05784_amd import fams
    from workloads import make_config
    s = make_config(3, instance=7, dims=(60, 60, 30), n_frac=40, contrast=contrast)
    print(f"[precision] contrast {contrast:g} n={s.n}", flush=True)
    A = sp.csr_matrix((s.val, s.col, s.row_ptr), shape=(s.n, s.n)).tocsc()
    p_ref = spla.splu(A).solve(s.q)
    wb, pr, vx, _ = fams.full_grid(s, (10, 10, 10), 10, 10)
    out = {}
    for prec in (fams.MIXED, fams.FP64):
        S = fams.Solver(s.row_ptr, s.col, s.val, s.n_matrix, wb, pr, vx, variant=fams.COUPLED,
                        precision=prec, alpha=1e-2)
        q = torch.from_numpy(s.q)
        p, info = S.solve(q, rtol=1e-10, max_iter=1500)
        _, _, imb = S.reconstruct_flux(q, p)
        err = np.linalg.norm(p.cpu().numpy() - p_ref) / np.linalg.norm(p_ref)
        out[prec] = (info[0], err, imb)
        S.close()
        print(f"  {'mixed' if prec else 'fp64 '}: status {info[0]['status']} "
              f"iterations {info[0]['iterations']} rel.res {info[0]['rel_residual']:.2e} "
              f"err vs direct {err:.2e} balance {imb:.2e}", flush=True)
    for prec, (info, err, imb) in out.items():
        # at the highest contrast FP64 itself stagnates just above 1e-10 (both
        # forms alike); the stagnation level is recorded and bounded
        assert info["status"] == 0 or (contrast >= 1e8 and info["rel_residual"] <= 1e-9)
        assert err <= 1e-6
        # fluxes are differences of FP64 pressures: at contrast 1e8 fracture
        # pressure differences are ~1e-8 of the pressure level, which puts the
        # balance floor of FP64 near 2e-10 there
        assert imb <= (1e-10 if contrast < 1e8 else 1e-9)
