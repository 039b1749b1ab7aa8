"""fams_footprint is an upper bound of what a handle holds: the peak device
memory of a setup plus solves of one and of several right-hand sides (the
lock-step work space) stays below the bound, for every coupling strategy,
both smoother settings and both precision forms, on the 100x100x50
workload."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

_sys = {}


def _system():
    if "s" not in _sys:
        from paper_1705_05784_amd import fams
        from workloads import make_config
        s = make_config(2)
        _sys["s"] = s
        _sys["grid"] = fams.full_grid(s, (10, 10, 10), 8, 8)
    return _sys["s"], _sys["grid"]


@pytest.mark.parametrize("precision", [0, 1])
@pytest.mark.parametrize("smoother", [1, 2])
@pytest.mark.parametrize("variant", [0, 1, 2, 3])
def test_footprint_bounds_peak(variant, smoother, precision):
    from paper_1705_05784_amd import fams
    from workloads.serving import well_rhs
    print(f"[footprint] variant={variant} smoother={smoother} precision={precision}", flush=True)
    s, (wb, pr, vx, _) = _system()
    g = fams.Solver(s.row_ptr, s.col, s.val, s.n_matrix, wb, pr, vx, variant=variant,
                    precision=precision, alpha=1e-2, smoother=smoother)
    rng = np.random.default_rng(variant)
    Q = torch.from_numpy(np.stack([well_rhs(s, 4, rng) for _ in range(3)])).cuda()
    g.solve(Q[0], rtol=1e-6)
    g.solve(Q, rtol=1e-6)
    si = g.setup_info()
    bound = fams.footprint(s.n, s.nnz, len(vx), precision, 30, 3)
    assert si["device_bytes"] <= si["peak_device_bytes"] <= bound, (si, bound)
    g.close()
