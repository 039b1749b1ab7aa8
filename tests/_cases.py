"""Small seeded cases shared by the tests (inputs only)."""
import numpy as np

from workloads import Plate, Well, add_wells, build_system, make_small


def homogeneous(nx, ny, nz, neumann=True, plates=()):
    lnk = np.zeros((nz, ny, nx))
    return build_system(nx, ny, nz, lnk, list(plates), 100.0, neumann=neumann)


def hat_1d(n, c):
    """Closed-form 1D interpolants on n cells with coarse nodes from
    oracle-independent arithmetic: nodes at block centres, linear between
    consecutive nodes, constant beyond the outermost ones."""
    starts = np.arange(0, n, c)
    nodes = starts + (np.minimum(starts + c, n) - starts) // 2
    H = np.zeros((n, len(nodes)))
    for x in range(n):
        if x <= nodes[0]:
            H[x, 0] = 1.0
        elif x >= nodes[-1]:
            H[x, -1] = 1.0
        else:
            k = np.searchsorted(nodes, x, side="right") - 1
            a, b = nodes[k], nodes[k + 1]
            H[x, k] = (b - x) / (b - a)
            H[x, k + 1] = (x - a) / (b - a)
    return H


SMALL = {
    "2d": dict(kind="2d", coarse=(4, 4, 1), d_min=4, r_z=1),
    "3d": dict(kind="3d", coarse=(4, 4, 4), d_min=4, r_z=4),
    # the full-size workload's shapes, shrunk: coarsening 10^3, d_min = r_z = 8
    "cfg2s": dict(kind="cfg2s", coarse=(10, 10, 10), d_min=8, r_z=8),
}


def small_case(name, seed=0, neumann=False, **kw):
    spec = SMALL[name]
    if spec["kind"] == "cfg2s":
        from workloads import make_config
        s = make_config(2, instance=100 + seed, dims=kw.get("dims", (42, 36, 22)),
                        n_frac=kw.get("n_frac", 12), neumann=neumann)
        return s, spec
    s = make_small(spec["kind"], seed=seed, neumann=neumann, **kw)
    return s, spec


def wells_case(name="3d", neumann=False, **kw):
    """A small case with two wells: one through the matrix column of the first
    fracture cell's host, perforating matrix cells only (so its cells are
    connected to that fracture), and one through another fracture's host
    column perforating the fracture cells there too."""
    s, spec = small_case(name, neumann=neumann, **kw)
    nx, ny, nz = s.nx, s.ny, s.nz

    def col_of(m):
        return m % nx, (m // nx) % ny, m // (nx * ny)

    ix, iy, iz = col_of(int(s.host[0]))
    w1 = Well(ix, iy, max(0, iz - 1), min(nz, iz + 2), rate=1.0, fractures=False)
    far = [c for c in range(len(s.host)) if col_of(int(s.host[c]))[:2] != (ix, iy)
           and abs(col_of(int(s.host[c]))[0] - ix) + abs(col_of(int(s.host[c]))[1] - iy) > 3]
    jx, jy, _ = col_of(int(s.host[far[len(far) // 2]]))
    w2 = Well(jx, jy, 0, nz, rate=-1.0, fractures=True)
    return add_wells(s, [w1, w2]), spec
