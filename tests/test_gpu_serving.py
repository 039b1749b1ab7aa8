"""Serving form on the GPU: each request's result is the same alone and in
the mix, and matches a direct solve of its own system."""
import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)


def test_alone_vs_mix():
    from paper_1705_05784_amd import fams
    from paper_1705_05784_amd.serving import ProcessRunner, Server, prepare, request_footprint, summarize
    from workloads.serving import make_stream

    reqs = prepare(make_stream(8, rate=0.0, pool=3, seed=5, side=(20, 32), n_frac=(5, 20),
                               nrhs=(1, 3)))
    fp = lambda r: request_footprint(r, fams.MIXED)  # noqa: E731
    kw = dict(alpha=1e-2, rtol=1e-10, flux=True, keep_pressures=True)
    _say("[serving] alone (1 slot process)")
    with ProcessRunner(1, fams.MIXED, **kw) as run1:
        alone = Server(run1, slots=1, footprint=fp).run(reqs, realtime=False)
    _say("[serving] mix (2 slot processes, the serving default)")
    with ProcessRunner(2, fams.MIXED, **kw) as run2:
        srv = Server(run2, slots=2, footprint=fp)
        mix = srv.run(reqs, realtime=False)
    assert srv.peak_inflight >= 2
    worst = 0.0
    for r, a, m in zip(reqs, alone, mix):
        assert a.status == 0 and m.status == 0, (a.error, m.error)
        assert a.iterations == m.iterations
        d = np.abs(a.pressures - m.pressures).max() / np.abs(a.pressures).max()
        worst = max(worst, d)
        assert max(m.imbalance) <= 1e-10
    assert worst <= 1e-12, worst
    # every request against a direct solve of its own system (p = A^-1 q)
    for r, m in zip(reqs, mix):
        s = r.system
        A = sp.csr_matrix((s.val, s.col, s.row_ptr), shape=(s.n, s.n)).tocsc()
        lu = spla.splu(A)
        for k in range(r.rhs.shape[0]):
            pd = lu.solve(r.rhs[k])
            e = np.linalg.norm(m.pressures[k] - pd) / np.linalg.norm(pd)
            assert e <= 1e-6, (r.rid, k, e)
    _say(f"[serving] {summarize(mix)}")
