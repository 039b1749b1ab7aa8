"""Pins of the oracle's coarse-grid helpers (Sec. 3, Fig. 2; Table 2; Sec. 4.3)."""
import os

import numpy as np
import pytest
import scipy.sparse as sp
from scipy.sparse.csgraph import shortest_path

from oracle import grids
from tests._cases import small_case

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def path_graph(n):
    ptr = [0]
    adj = []
    for i in range(n):
        nb = [j for j in (i - 1, i + 1) if 0 <= j < n]
        adj.extend(nb)
        ptr.append(len(adj))
    return np.array(ptr), np.array(adj)


def test_axis_nodes_closed_form():
    assert list(grids.axis_nodes(100, 10)) == list(range(5, 100, 10))
    # partial last block 250..255 has its node at its own centre
    assert grids.axis_nodes(256, 10)[-1] == 253
    assert list(grids.axis_nodes(7, 1)) == list(range(7))


def test_structured_small_by_hand():
    # 6 x 4 grid, coarsening 3 x 2: x-nodes {1, 4}, y-nodes {1, 3}
    wb, primal, vertex = grids.structured_grid(6, 4, 1, 3, 2, 1)
    expect = np.array([[1, 2, 1, 1, 2, 1],
                       [2, 3, 2, 2, 3, 2],
                       [1, 2, 1, 1, 2, 1],
                       [2, 3, 2, 2, 3, 2]])
    assert np.array_equal(wb.reshape(4, 6), expect)
    assert list(vertex) == [7, 10, 19, 22]
    y, x = np.mgrid[0:4, 0:6]
    assert np.array_equal(primal.reshape(4, 6), x // 3 + 2 * (y // 2))


def test_structured_counts_3d():
    wb, primal, vertex = grids.structured_grid(100, 100, 50, 10, 10, 10)
    assert len(vertex) == 10 * 10 * 5
    assert (wb == 3).sum() == 500
    # every primal block holds exactly its own coarse node
    assert np.array_equal(primal[vertex], np.arange(500))
    # interiors: 9 x 9 x 9 per block away from the far boundary
    assert (wb == 0).sum() == 10 * 10 * 5 * 9 * 9 * 9


@pytest.mark.parametrize("d", [2, 3, 5, 8])
@pytest.mark.parametrize("n", [1, 7, 23, 40])
def test_table2_path_graph(n, d):
    """Path graph, start = cell 0: a vertex every d cells; every cell belongs to
    the nearest vertex, ties to the earlier one (Table 2 steps 12-14)."""
    ptr, adj = path_graph(n)
    verts, primal, level = grids.table2_coarsening(n, ptr, adj, d)
    expect = list(range(0, n, d))
    assert list(verts) == expect
    for x in range(n):
        dists = [abs(x - v) for v in expect]
        best = min(dists)
        assert level[x] == best
        assert primal[x] == dists.index(best)


def test_table2_infinite_dmin_single_node():
    """d_min = infinity gives one coarse node per network (Sec. 4.1, Fig. 8a)."""
    ptr, adj = path_graph(30)
    verts, primal, level = grids.table2_coarsening(30, ptr, adj, 0)
    assert list(verts) == [0]
    assert np.all(primal == 0)
    assert list(level) == list(range(30))


def test_table2_golden_tree():
    """Hand-worked Table 2 run on a small branched network (golden fixture)."""
    with open(os.path.join(GOLDEN, "table2_tree.txt")) as f:
        lines = [ln.split("#")[0].strip() for ln in f]
    lines = [ln for ln in lines if ln]
    n = int(lines[0])
    edges = [tuple(map(int, ln.split())) for ln in lines[1:] if ln[0].isdigit() and len(ln.split()) == 2]
    kv = {ln.split("=")[0].strip(): ln.split("=")[1].strip() for ln in lines if "=" in ln}
    g = sp.coo_matrix((np.ones(len(edges)), tuple(np.array(edges).T)), shape=(n, n))
    g = (g + g.T).tocsr()
    g.sort_indices()
    verts, primal, level = grids.table2_coarsening(n, g.indptr, g.indices, int(kv["d_min"]))
    assert list(verts) == [int(v) for v in kv["vertices"].split()]
    assert list(primal) == [int(v) for v in kv["primal"].split()]
    assert list(level) == [int(v) for v in kv["level"].split()]


@pytest.mark.parametrize("seed", range(6))
@pytest.mark.parametrize("d", [2, 3, 6])
def test_table2_distance_guarantee(seed, d):
    """Sec. 4.1: a distance of at least d_min cells between each pair of coarse
    nodes; and every cell ends closer than d_min to its vertex."""
    rng = np.random.default_rng(seed)
    n = 60
    # random tree plus a few extra edges
    e = [(i, int(rng.integers(0, i))) for i in range(1, n)]
    e += [tuple(sorted(map(int, rng.integers(0, n, 2)))) for _ in range(6)]
    e = [(a, b) for a, b in e if a != b]
    g = sp.coo_matrix((np.ones(len(e)), tuple(np.array(e).T)), shape=(n, n))
    g = ((g + g.T) > 0).astype(float).tocsr()
    g.sort_indices()
    verts, primal, level = grids.table2_coarsening(n, g.indptr, g.indices, d)
    D = shortest_path(g, unweighted=True)
    for a in range(len(verts)):
        for b in range(a + 1, len(verts)):
            assert D[verts[a], verts[b]] >= d
    assert level.max() <= d - 1
    # level is the true graph distance to the nearest vertex
    assert np.array_equal(level, D[verts].min(axis=0).astype(int))


@pytest.mark.parametrize("name", ["2d", "3d"])
def test_fracture_grid_valid(name):
    s, spec = small_case(name)
    wb, primal, vertex, ncm = grids.full_grid(s, spec["coarse"], spec["d_min"], spec["r_z"])
    nm = s.n_matrix
    wbf = wb[nm:]
    assert wbf.min() >= 1                      # fractures have no interiors (App. A)
    if name == "2d":
        assert set(np.unique(wbf)) <= {2, 3}   # 1D networks: V and E only
    # one coarse node per primal block, inside it
    assert np.array_equal(primal[vertex], np.arange(len(vertex)))
    assert np.all(wb[vertex] == 3)
    assert (wb == 3).sum() == len(vertex)
    # fracture primal blocks are connected through fracture connections
    A = s.csr()
    Aff = A[nm:, nm:]
    for K in range(ncm, len(vertex)):
        cells = np.nonzero(primal[nm:] == K)[0]
        sub = Aff[cells][:, cells]
        from scipy.sparse.csgraph import connected_components
        assert connected_components(sub, directed=False)[0] == 1


def _extrusion_case():
    """Two intersecting plates of the golden fixture fracture_extrusion.txt."""
    cells = [(c, z, 0) for z in range(0, 6) for c in range(0, 6)]
    cells += [(c, z, 1) for z in range(3, 6) for c in range(6, 8)]
    index = {(c, z): 1 + k for k, (c, z, _) in enumerate(cells)}
    links = set()
    for (c, z, pl) in cells:
        for (c2, z2) in ((c + 1, z), (c, z + 1)):
            same_plate = (c2 <= 5) == (c <= 5)
            if (c2, z2) in index and same_plate:
                links.add((index[(c, z)], index[(c2, z2)]))
    for z in (3, 4, 5):   # the intersection of column 1 with column 7
        links.add((index[(1, z)], index[(7, z)]))
    n = 1 + len(cells)
    rows = [[i] for i in range(n)]
    for a, b in links:
        rows[a].append(b)
        rows[b].append(a)
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    col = []
    for i in range(n):
        col.extend(sorted(rows[i]))
        row_ptr[i + 1] = len(col)
    col_adj_lists = {0: [1], 1: [0, 2, 7], 2: [1, 3], 3: [2, 4], 4: [3, 5], 5: [4], 6: [7],
                     7: [1, 6]}
    col_ptr = np.cumsum([0] + [len(col_adj_lists[c]) for c in range(8)]).astype(np.int64)
    col_adj = np.array(sum((col_adj_lists[c] for c in range(8)), []), dtype=np.int32)
    return dict(n_matrix=1, row_ptr=row_ptr, col=np.array(col, dtype=np.int32),
                cell_col=np.array([c for c, _, _ in cells], dtype=np.int32),
                cell_z=np.array([z for _, z, _ in cells], dtype=np.int32),
                col_plate=np.array([0] * 6 + [1] * 2, dtype=np.int32), col_ptr=col_ptr,
                col_adj=col_adj, plate_zlo=np.array([0, 3], dtype=np.int32),
                plate_zhi=np.array([6, 6], dtype=np.int32))


def _golden_kv(name):
    with open(os.path.join(GOLDEN, name)) as f:
        lines = [ln.split("#")[0].strip() for ln in f]
    return {ln.split("=")[0].strip(): [int(v) for v in ln.split("=")[1].split()]
            for ln in lines if "=" in ln}


def test_fracture_extrusion_golden():
    """Hand-worked 3D fracture grid (Sec. 4.1 Table 2 on the projection,
    Sec. 4.3 extrusion): coarse-layer rule and its middle-layer fallback,
    V/E/F classes, the promotion of an E block without a V neighbour, and a
    nearest-vertex partition with ties to the lower coarse id."""
    g = _golden_kv("fracture_extrusion.txt")
    c = _extrusion_case()
    verts, _, _ = grids.table2_coarsening(8, c["col_ptr"], c["col_adj"], 4)
    assert sorted(verts.tolist()) == g["vertex_columns"]
    wb, primal, vertex = grids.fracture_grid(
        c["n_matrix"], c["row_ptr"], c["col"], c["cell_col"], c["cell_z"], c["col_plate"],
        c["col_ptr"], c["col_adj"], c["plate_zlo"], c["plate_zhi"], d_min=4, r_z=4,
        n_coarse_matrix=1)
    assert wb.tolist() == g["wb_type"]
    assert primal.tolist() == g["primal"]
    assert vertex.tolist() == g["vertex"]


def test_fracture_extrusion_golden_library_helper():
    """The library's host helper gives the same hand-worked grid."""
    from paper_1705_05784_amd import fams as gfams
    if not os.path.exists(gfams.LIB_PATH):
        pytest.skip("libfams.so not built")
    import ctypes as C
    g = _golden_kv("fracture_extrusion.txt")
    c = _extrusion_case()
    nf = len(c["cell_col"])
    wb = np.empty(nf, dtype=np.int8)
    pr = np.empty(nf, dtype=np.int32)
    vx = np.empty(nf, dtype=np.int64)
    ncf = C.c_int64()
    st = gfams.lib().fams_grid_fracture(
        c["n_matrix"], c["n_matrix"] + nf, c["row_ptr"].ctypes.data, c["col"].ctypes.data,
        c["cell_col"].ctypes.data, c["cell_z"].ctypes.data, 8, c["col_plate"].ctypes.data,
        c["col_ptr"].ctypes.data, c["col_adj"].ctypes.data, 2, c["plate_zlo"].ctypes.data,
        c["plate_zhi"].ctypes.data, 4, 4, 1, wb.ctypes.data, pr.ctypes.data, vx.ctypes.data,
        C.byref(ncf))
    assert st == 0
    assert wb.tolist() == g["wb_type"]
    assert pr.tolist() == g["primal"]
    assert vx[:ncf.value].tolist() == g["vertex"]
