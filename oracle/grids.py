"""Oracle: coarse grids for the matrix and the fracture networks.

Test infrastructure only (see the package docstring).

Cell classes follow the wirebasket hierarchy of Sec. 3.1 / App. A:
0 = interior (I), 1 = face (F), 2 = edge (E), 3 = vertex (V).

Readings where the paper is silent (they are listed in the design notes):
  * the coarse node of a structured primal block is its centre cell, per axis
    start + floor(len/2), the last partial block included (Fig. 2 shows only
    pictures);
  * a matrix cell's class is the number of its coordinates lying on a
    coarse-node plane (3 = V, 2 = E, 1 = F, 0 = I); a 2D grid is a 3D grid with
    nz = cz = 1, so it has V, E and F ("faces" = the 2D dual blocks) only;
  * fracture coarsening runs Table 2 on the x-y projection of each network
    (Sec. 4.3) with the start cell = the lowest-index column of the network,
    a FIFO Q_vertex and neighbours visited in ascending order; coarse layers
    are the global layers k with k mod r_z = floor(r_z/2), or the middle layer
    of a plate that contains none; a fracture cell is V when its column is a
    vertex column and its layer a coarse layer, E when exactly one holds,
    F otherwise;
  * an E component of fracture cells with no V neighbour, or an F component
    with no E/V neighbour, gets its lowest-index cell promoted to V (such a
    block would otherwise have a singular local problem);
  * fracture primal blocks: every fracture cell belongs to the nearest V cell
    by graph distance on the fracture-fracture connections, ties to the
    lower coarse index (for a 1D network this is Table 2's own primal
    assignment up to tie-breaking);
  * coarse ids: matrix blocks first (x fastest), then fracture V cells in
    ascending fine index, then one per well (class V, a primal block of its
    own) in well order.
"""
from __future__ import annotations

from collections import deque

import numpy as np

WB_I, WB_F, WB_E, WB_V = 0, 1, 2, 3


def axis_nodes(n: int, c: int) -> np.ndarray:
    """Coarse-node positions along one axis of n cells with coarsening c."""
    starts = np.arange(0, n, c)
    ends = np.minimum(starts + c, n)
    return starts + (ends - starts) // 2


def structured_grid(nx, ny, nz, cx, cy, cz):
    """Wirebasket classes, primal ids and coarse nodes of a structured grid.

    Returns (wb_type int8 [nx*ny*nz], primal int32 [...], vertex int64 [ncm]).
    """
    on = []
    blk = []
    nb = []
    for n, c in ((nx, cx), (ny, cy), (nz, cz)):
        f = np.zeros(n, dtype=bool)
        f[axis_nodes(n, c)] = True
        on.append(f)
        blk.append(np.arange(n) // c)
        nb.append(-(-n // c))
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    cnt = on[0][x].astype(int) + on[1][y] + on[2][z]
    wb = cnt.astype(np.int8).ravel()
    primal = (blk[0][x] + nb[0] * (blk[1][y] + nb[1] * blk[2][z])).astype(np.int32).ravel()
    nxn, nyn, nzn = axis_nodes(nx, cx), axis_nodes(ny, cy), axis_nodes(nz, cz)
    Z, Y, X = np.meshgrid(nzn, nyn, nxn, indexing="ij")
    vertex = (X + nx * (Y + ny * Z)).astype(np.int64).ravel()
    return wb, primal, vertex


def table2_coarsening(n_cells, adj_ptr, adj, d_min):
    """Distance-based coarsening of a graph, following Table 2 of the paper.

    ``d_min <= 0`` means d_min = infinity.  Networks (connected components)
    are processed in ascending order of their lowest cell, which is also the
    start cell.  Returns (vertices in creation order, primal block index per
    cell, level per cell).
    """
    inf = np.iinfo(np.int64).max
    dmax = inf if d_min <= 0 else int(d_min)
    level = np.full(n_cells, inf, dtype=np.int64)
    primal = np.full(n_cells, -1, dtype=np.int64)
    seen = np.zeros(n_cells, dtype=bool)
    vertices = []
    for start in range(n_cells):
        if seen[start]:
            continue
        # mark the network of `start` as seen
        stack = [start]
        seen[start] = True
        while stack:
            c = stack.pop()
            for nb in adj[adj_ptr[c]:adj_ptr[c + 1]]:
                if not seen[nb]:
                    seen[nb] = True
                    stack.append(nb)
        q_vertex = deque([start])
        in_qv = {start}
        while q_vertex:
            v = q_vertex.popleft()
            in_qv.discard(v)
            pid = len(vertices)
            vertices.append(v)
            primal[v] = pid
            level[v] = 0
            q1 = [v]
            dist = 1
            while dist <= dmax and q1:
                q2 = []
                for c in q1:
                    for nb in adj[adj_ptr[c]:adj_ptr[c + 1]]:
                        if level[nb] > dist:
                            if nb in in_qv:
                                q_vertex.remove(nb)
                                in_qv.discard(nb)
                            level[nb] = dist
                            primal[nb] = pid
                            q2.append(nb)
                q1 = q2
                dist += 1
            if dist > dmax:          # the loop ran up to and including d_min
                for c in q1:
                    q_vertex.append(c)
                    in_qv.add(c)
    return np.asarray(vertices, dtype=np.int64), primal, level


def _coarse_layers(zlo, zhi, r_z):
    ks = [k for k in range(zlo, zhi) if k % r_z == r_z // 2]
    if not ks:
        ks = [zlo + (zhi - zlo - 1) // 2]
    return set(ks)


def _components(cells_mask, ptr, adj):
    """Connected components among cells where mask holds; list of sorted lists."""
    n = len(cells_mask)
    comp = np.full(n, -1, dtype=np.int64)
    out = []
    for s in range(n):
        if not cells_mask[s] or comp[s] >= 0:
            continue
        comp[s] = len(out)
        members = [s]
        stack = [s]
        while stack:
            c = stack.pop()
            for nb in adj[ptr[c]:ptr[c + 1]]:
                if cells_mask[nb] and comp[nb] < 0:
                    comp[nb] = comp[s]
                    members.append(nb)
                    stack.append(nb)
        out.append(sorted(members))
    return out


def fracture_grid(n_matrix, row_ptr, col, cell_col, cell_z, col_plate, col_ptr, col_adj,
                  plate_zlo, plate_zhi, d_min, r_z, n_coarse_matrix):
    """Fracture wirebasket classes, primal ids and coarse nodes.

    Returns (wb_type int8 [n_f], primal int32 [n_f] (global coarse ids),
    vertex int64 [n_cf] (global fine indices)).
    """
    nf = len(cell_col)
    if nf == 0:
        return (np.zeros(0, np.int8), np.zeros(0, np.int32), np.zeros(0, np.int64))
    ncols = len(col_plate)
    verts, _, _ = table2_coarsening(ncols, col_ptr, col_adj, d_min)
    vcol = np.zeros(ncols, dtype=bool)
    vcol[verts] = True
    layers = [_coarse_layers(int(plate_zlo[p]), int(plate_zhi[p]), r_z)
              for p in range(len(plate_zlo))]
    wb = np.empty(nf, dtype=np.int8)
    for c in range(nf):
        a = bool(vcol[cell_col[c]])
        b = int(cell_z[c]) in layers[col_plate[cell_col[c]]]
        wb[c] = WB_V if (a and b) else (WB_E if (a or b) else WB_F)

    # fracture-fracture adjacency (local indices) from the fine system
    fptr = np.zeros(nf + 1, dtype=np.int64)
    fadj = []
    for c in range(nf):
        i = n_matrix + c
        row = col[row_ptr[i]:row_ptr[i + 1]]
        nbrs = [int(j) - n_matrix for j in row if n_matrix <= j < n_matrix + nf and j != i]
        fadj.extend(nbrs)
        fptr[c + 1] = len(fadj)
    fadj = np.asarray(fadj, dtype=np.int64)

    def touches(cells, classes):
        for c in cells:
            for nb in fadj[fptr[c]:fptr[c + 1]]:
                if wb[nb] in classes:
                    return True
        return False

    for comp in _components(wb == WB_E, fptr, fadj):
        if not touches(comp, (WB_V,)):
            wb[comp[0]] = WB_V
    for comp in _components(wb == WB_F, fptr, fadj):
        if not touches(comp, (WB_E, WB_V)):
            wb[comp[0]] = WB_V

    vloc = np.nonzero(wb == WB_V)[0]
    coarse = np.full(nf, -1, dtype=np.int64)
    coarse[vloc] = n_coarse_matrix + np.arange(len(vloc))
    # nearest-vertex partition, ties to the lower coarse id
    dist = np.full(nf, -1, dtype=np.int64)
    owner = np.full(nf, -1, dtype=np.int64)
    dist[vloc] = 0
    owner[vloc] = coarse[vloc]
    frontier = list(vloc)
    d = 0
    while frontier:
        nxt = []
        for c in frontier:
            for nb in fadj[fptr[c]:fptr[c + 1]]:
                if dist[nb] < 0:
                    dist[nb] = d + 1
                    owner[nb] = owner[c]
                    nxt.append(nb)
                elif dist[nb] == d + 1 and owner[c] < owner[nb]:
                    owner[nb] = owner[c]
        frontier = nxt
        d += 1
    if np.any(owner < 0):
        raise ValueError("fracture cell not connected to any coarse node")
    return wb, owner.astype(np.int32), (vloc + n_matrix).astype(np.int64)


def full_grid(sysm, coarse, d_min, r_z):
    """Matrix + fracture (+ well) grid for a workloads.FracturedSystem: each
    well is a coarse node of its own (class V, its own primal block; Sec. 3,
    one coarse node per well with the identity restriction)."""
    cx, cy, cz = coarse
    nw = getattr(sysm, "n_wells", 0)
    wbm, pm, vm = structured_grid(sysm.nx, sysm.ny, sysm.nz, cx, cy, cz)
    wbf, pf, vf = fracture_grid(sysm.n_matrix, sysm.row_ptr, sysm.col, sysm.cell_col,
                                sysm.cell_z, sysm.col_plate, sysm.col_ptr, sysm.col_adj,
                                sysm.plate_zlo, sysm.plate_zhi, d_min, r_z, len(vm))
    nc0 = len(vm) + len(vf)
    wbw = np.full(nw, WB_V, dtype=np.int8)
    pw = np.arange(nc0, nc0 + nw, dtype=np.int32)
    vw = np.arange(sysm.n - nw, sysm.n, dtype=np.int64)
    return (np.concatenate([wbm, wbf, wbw]), np.concatenate([pm, pf, pw]),
            np.concatenate([vm, vf, vw]), len(vm))
