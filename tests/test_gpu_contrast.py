"""The 200x200x50 workload with 400 plates at full size, at the two ends of
the fracture/matrix contrast sweep (1e2 and 1e8): Coupled-AMS, alpha 1e-2,
precision form and plain FP64, each iterated to a relative residual of
1e-10.  Both forms converge; each pressure matches the oracle's (FP64 GMRES
of the same system, a data file written by `python -m oracle.make_pref`) to
1e-6; the two forms agree to 1e-8; the reconstructed fluxes balance every
cell to 1e-9."""
import os

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.parametrize("contrast", [1e2, 1e8])
def test_contrast_ends_full_size(contrast):
    from paper_1705_05784_amd import fams
    from workloads import make_config
    from workloads.edfm import system_key
    print(f"[contrast] building the 200x200x50 workload at contrast {contrast:g}", flush=True)
    s = make_config(3, contrast=contrast)
    key = system_key(s.row_ptr, s.col, s.val, s.q)
    pref_path = os.path.join(ROOT, "oracle", "_pref", key + ".npy")
    if not os.path.exists(pref_path):
        pytest.skip("the oracle's stored pressure for this system is absent "
                    "(python -m oracle.make_pref --config 3 --contrast C writes it)")
    pref = np.load(pref_path)
    wb, pr, vx, _ = fams.full_grid(s, (10, 10, 10), 10, 10)
    dev = torch.device("cuda", 0)
    args = [torch.from_numpy(a).to(dev) for a in (s.row_ptr, s.col, s.val, wb, pr, vx)]
    q = torch.from_numpy(s.q).to(dev)
    ps = {}
    for name, prec in (("mixed", fams.MIXED), ("fp64", fams.FP64)):
        g = fams.Solver(*args[:3], s.n_matrix, *args[3:], variant=fams.COUPLED, precision=prec,
                        alpha=1e-2)
        p, info = g.solve(q, rtol=1e-10, max_iter=3000)
        _, _, imb = g.reconstruct_flux(q, p)
        g.close()
        ps[name] = p.cpu().numpy()
        err = np.linalg.norm(ps[name] - pref) / np.linalg.norm(pref)
        print(f"[contrast] {name}: {info[0]['iterations']} iterations, residual "
              f"{info[0]['rel_residual']:.2e}, error vs oracle {err:.2e}, balance {imb:.2e}",
              flush=True)
        assert info[0]["status"] == fams.OK, info
        assert info[0]["rel_residual"] <= 1e-10
        assert err <= 1e-6, (name, err)
        assert imb <= 1e-9, (name, imb)
    d = np.linalg.norm(ps["mixed"] - ps["fp64"]) / np.linalg.norm(ps["fp64"])
    assert d <= 1e-8, d
