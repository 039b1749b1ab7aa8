"""The allocation hook of fams_setup (fams_allocator_t) with torch's caching
allocator behind it: every buffer of the handle comes from the hook (torch
counts them while the handle lives and gets them all back when it is
destroyed), the results match those of the default allocator, and a second
handle of the same shape reuses the cached memory instead of reserving more.
100x100x50 workload, FP64 and mixed precision, single and lock-step solves."""
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


def _run(allocator, precision, Q):
    from paper_1705_05784_amd import fams
    s, (wb, pr, vx, _) = _system()
    g = fams.Solver(s.row_ptr, s.col, s.val, s.n_matrix, wb, pr, vx, variant=fams.COUPLED,
                    precision=precision, alpha=1e-2, allocator=allocator)
    p1, i1 = g.solve(Q[0], rtol=1e-8)
    P, infos = g.solve(Q, rtol=1e-8)
    torch.cuda.synchronize()
    return g, p1, P, [i1[0]] + list(infos)


@pytest.mark.parametrize("precision", [0, 1])
def test_torch_allocator_matches_default_and_reuses_memory(precision):
    from paper_1705_05784_amd import fams
    from workloads.serving import well_rhs
    print(f"[allocator] precision={precision}", flush=True)
    s, _ = _system()
    rng = np.random.default_rng(11 + precision)
    Q = torch.from_numpy(np.stack([well_rhs(s, 4, rng) for _ in range(5)])).cuda()
    g, p1_ref, P_ref, inf_ref = _run(None, precision, Q)
    g.close()
    torch.cuda.synchronize()
    base = torch.cuda.memory_allocated()
    reserved = []
    for rep in range(2):
        g, p1, P, inf = _run("torch", precision, Q)
        si = g.setup_info()
        held = torch.cuda.memory_allocated() - base
        # the handle's buffers (and the two solution tensors) are torch's now
        assert held >= si["device_bytes"], (held, si["device_bytes"])
        assert all(i["status"] == fams.OK for i in inf), inf
        assert [i["iterations"] for i in inf] == [i["iterations"] for i in inf_ref]
        tol = 1e-12 * float(torch.linalg.norm(P_ref))
        assert float(torch.linalg.norm(P - P_ref)) <= tol
        assert float(torch.linalg.norm(p1 - p1_ref)) <= 1e-12 * float(torch.linalg.norm(p1_ref))
        g.close()
        del p1, P
        torch.cuda.synchronize()
        assert torch.cuda.memory_allocated() == base   # everything went back to the cache
        reserved.append(torch.cuda.memory_reserved())
    assert reserved[1] == reserved[0], reserved      # the second handle took cached blocks


def test_allocator_name_is_checked():
    from paper_1705_05784_amd import fams
    s, (wb, pr, vx, _) = _system()
    with pytest.raises(ValueError):
        fams.Solver(s.row_ptr, s.col, s.val, s.n_matrix, wb, pr, vx, allocator="malloc")


def test_hook_refusal_narrows_the_group():
    """A hook that refuses every allocation above 3 GB: the 16-wide lock-step
    work space of the 100x100x50 system (about 5.6 GB) is asked for and
    refused, the solve falls back to groups of 8, and every column still
    equals its own single solve."""
    from paper_1705_05784_amd import fams
    from workloads.serving import well_rhs
    print("[allocator] refusing hook", flush=True)
    s, (wb, pr, vx, _) = _system()
    cap = 3 << 30
    refused = []

    def alloc(ctx, nbytes, stream):
        if nbytes > cap:
            refused.append(int(nbytes))
            return None
        return torch.cuda.caching_allocator_alloc(int(nbytes), torch.cuda.current_device(),
                                                  int(stream or 0))

    def free(ctx, ptr, stream):
        torch.cuda.caching_allocator_delete(int(ptr))

    hook = fams.AllocatorHook(None, fams._ALLOC_FN(alloc), fams._FREE_FN(free))
    g = fams.Solver(s.row_ptr, s.col, s.val, s.n_matrix, wb, pr, vx, variant=fams.COUPLED,
                    precision=fams.MIXED, alpha=1e-2, allocator=hook)
    rng = np.random.default_rng(3)
    Q = torch.from_numpy(np.stack([well_rhs(s, 4, rng) for _ in range(12)])).cuda()
    P, infos = g.solve(Q, rtol=1e-10)
    assert refused and min(refused) > cap, refused   # the 16-wide work space was refused
    assert g.setup_info()["device_bytes"] < 2 * cap
    for r in range(12):
        p1, i1 = g.solve(Q[r], rtol=1e-10)
        assert infos[r]["status"] == 0 and i1[0]["status"] == 0
        assert abs(infos[r]["iterations"] - i1[0]["iterations"]) <= 1, (r, infos[r], i1[0])
        err = float(torch.linalg.norm(P[r] - p1) / torch.linalg.norm(p1))
        assert err <= 1e-9, (r, err)
    g.close()
