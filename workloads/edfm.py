"""Seeded synthetic EDFM fine-scale systems (problem inputs, not the solver).

This module builds the fine-scale linear system ``A p = q`` of the paper's
Section 2 (matrix/fracture mass balance, Darcy flux with TPFA, matrix-fracture
exchange through a connectivity index CI = A/<d>) on synthetic inputs with the
shapes of the paper's workloads.  It contains none of the multiscale method:
no wirebasket classification, no basis functions, no coarse operators.  Both
the oracle and the GPU library receive the arrays built here as plain data.

Conventions (fixed here and stated in the design notes):
  * cubic cells of size h = 1/nx; the domain is [0,1] x [0, ny*h] x [0, nz*h];
  * matrix cells in natural order (x fastest, then y, then z);
  * fracture cells after all matrix cells, plate by plate, and inside a plate
    trace position fastest, then z layer;
  * TPFA transmissibility between matrix cells: h^(d-2) * harmonic mean of k;
  * Dirichlet p=1 on the x=0 face and p=0 on the x=L face through a half-cell
    transmissibility 2*k*h^(d-2); no other boundary flux (keeps A SPD);
  * fracture aperture a = h, fracture permeability k_f = contrast * k_g with
    k_g the geometric mean of the matrix permeability;
  * along-trace fracture transmissibility k_f*a*w/d (w = 1 in 2D, h in 3D;
    d = distance between segment centroids), vertical k_f*a*l_seg/h;
  * matrix-fracture transmissibility k_m * CI, CI = l_seg*w/<d>, with <d> the
    mean distance from the host cell to the fracture line (8x8 midpoint rule);
  * two intersecting fractures connect the two segments that contain the
    intersection point, per shared layer, with T1*T2/(T1+T2),
    T_k = k_f*a*w/d_k and d_k the centroid-to-intersection distance.
"""
from __future__ import annotations

import dataclasses
import hashlib

import numpy as np
import scipy.sparse as sp
from scipy import ndimage


@dataclasses.dataclass
class Plate:
    """One straight fracture trace (2D segment or 3D vertical plate)."""
    x0: float
    y0: float
    x1: float
    y1: float
    zlo: int            # first layer (inclusive)
    zhi: int            # last layer (exclusive)


@dataclasses.dataclass
class FracturedSystem:
    """A fine-scale EDFM system and the geometry the coarse-grid helpers need."""
    nx: int
    ny: int
    nz: int
    h: float
    n_matrix: int
    n: int
    row_ptr: np.ndarray          # int64 [n+1]
    col: np.ndarray              # int32 [nnz], sorted per row, diagonal present
    val: np.ndarray              # float64 [nnz]
    q: np.ndarray                # float64 [n]  (boundary term + sources)
    lnk: np.ndarray              # matrix ln k, shape (nz, ny, nx)
    # fracture geometry for the coarse-grid helpers (host data only)
    cell_col: np.ndarray         # int32 [n_f]: fracture column (plate, trace pos)
    cell_z: np.ndarray           # int32 [n_f]: z layer of each fracture cell
    col_plate: np.ndarray        # int32 [n_cols]
    col_ptr: np.ndarray          # int64 [n_cols+1]: projected column graph (CSR)
    col_adj: np.ndarray          # int32: neighbours, ascending per column
    plate_zlo: np.ndarray        # int32 [n_plates]
    plate_zhi: np.ndarray        # int32 [n_plates]
    host: np.ndarray             # int64 [n_f]: host matrix cell of each fracture cell
    t_ratio: float               # mean fracture T / mean matrix T (paper Eq. tratio)
    meta: dict
    n_wells: int = 0             # the last n_wells unknowns are well pressures

    @property
    def n_frac(self) -> int:
        return self.n - self.n_matrix - self.n_wells

    @property
    def nnz(self) -> int:
        return int(self.row_ptr[-1])

    def csr(self) -> sp.csr_matrix:
        return sp.csr_matrix((self.val, self.col, self.row_ptr), shape=(self.n, self.n))

    def sha256(self) -> str:
        m = hashlib.sha256()
        for a in (self.row_ptr, self.col, self.val, self.q):
            m.update(np.ascontiguousarray(a).tobytes())
        return m.hexdigest()


def system_key(row_ptr, col, val, q) -> str:
    """SHA-256 (24 hex digits) of a system and one right-hand side: the key
    under which a reference pressure computed for exactly this input is kept."""
    m = hashlib.sha256()
    for a in (row_ptr, col, val, q):
        m.update(np.ascontiguousarray(a).tobytes())
    return m.hexdigest()[:24]


def lnk_field(shape, std, corr, rng):
    """Gaussian random field: iid N(0,1), Gaussian filter, standardised, scaled."""
    z = rng.standard_normal(shape)
    if np.any(np.asarray(corr) > 0):
        z = ndimage.gaussian_filter(z, sigma=corr, mode="reflect")
    s = z.std()
    z = (z - z.mean()) / (s if s > 0 else 1.0)
    return std * z


def _clip_segment(x0, y0, x1, y1, lx, ly):
    """Liang-Barsky clip of a segment to [0,lx]x[0,ly]; None if outside."""
    dx, dy = x1 - x0, y1 - y0
    t0, t1 = 0.0, 1.0
    for p, qv in ((-dx, x0), (dx, lx - x0), (-dy, y0), (dy, ly - y0)):
        if p == 0.0:
            if qv < 0:
                return None
            continue
        t = qv / p
        if p < 0:
            t0 = max(t0, t)
        else:
            t1 = min(t1, t)
    if t0 >= t1:
        return None
    return (x0 + t0 * dx, y0 + t0 * dy, x0 + t1 * dx, y0 + t1 * dy)


def _trace_pieces(pl: Plate, h, nx, ny):
    """Split a trace at matrix-cell boundaries: (t0, t1, host ix, iy) per piece."""
    dx, dy = pl.x1 - pl.x0, pl.y1 - pl.y0
    ts = [0.0, 1.0]
    if abs(dx) > 0:
        for i in range(nx + 1):
            t = (i * h - pl.x0) / dx
            if 0.0 < t < 1.0:
                ts.append(t)
    if abs(dy) > 0:
        for j in range(ny + 1):
            t = (j * h - pl.y0) / dy
            if 0.0 < t < 1.0:
                ts.append(t)
    ts = np.unique(np.array(ts))
    length = np.hypot(dx, dy)
    out = []
    for a, b in zip(ts[:-1], ts[1:]):
        if (b - a) * length <= 1e-9 * h:
            continue
        tm = 0.5 * (a + b)
        xm, ym = pl.x0 + tm * dx, pl.y0 + tm * dy
        ix = min(max(int(np.floor(xm / h)), 0), nx - 1)
        iy = min(max(int(np.floor(ym / h)), 0), ny - 1)
        out.append((a, b, ix, iy))
    return out


def _mean_distance_to_line(ix, iy, h, pl: Plate, npts=8):
    """<d>: mean distance from the host cell square to the fracture's line."""
    dx, dy = pl.x1 - pl.x0, pl.y1 - pl.y0
    L = np.hypot(dx, dy)
    nxn, nyn = -dy / L, dx / L
    s = (np.arange(npts) + 0.5) / npts
    X = (ix + s)[None, :] * h
    Y = (iy + s)[:, None] * h
    d = np.abs((X - pl.x0) * nxn + (Y - pl.y0) * nyn)
    return float(d.mean())


def _locate(pieces, t):
    for p, (t0, t1, _, _) in enumerate(pieces):
        if t0 <= t <= t1:
            return p
    return None


def _cat(parts, dtype):
    return (np.concatenate(parts).astype(dtype) if parts else np.zeros(0, dtype=dtype))


def build_system(nx, ny, nz, lnk, plates, contrast, sources=None,
                 rhs_dirichlet=True, neumann=False, meta=None) -> FracturedSystem:
    """Assemble the EDFM system for a matrix ln k field and a list of plates.

    ``neumann=True`` drops the Dirichlet faces (A then has zero row sums; used
    by tests of partition of unity).  ``sources`` is an optional list of
    (matrix cell, rate) pairs added to q.
    """
    dim = 2 if nz == 1 else 3
    h = 1.0 / nx
    hd = h ** (dim - 2)
    k = np.exp(lnk).reshape(nz, ny, nx)
    kg = float(np.exp(lnk.mean()))
    kf = contrast * kg
    aperture = h
    w = h if dim == 3 else 1.0
    nm = nx * ny * nz

    rows, cols, tvals = [], [], []
    mm_T = []

    idx = np.arange(nm).reshape(nz, ny, nx)
    for axis in (2, 1, 0):
        if k.shape[axis] < 2:
            continue
        sl_a = [slice(None)] * 3
        sl_b = [slice(None)] * 3
        sl_a[axis] = slice(0, -1)
        sl_b[axis] = slice(1, None)
        ka, kb = k[tuple(sl_a)], k[tuple(sl_b)]
        t = hd * 2.0 * ka * kb / (ka + kb)
        rows.append(idx[tuple(sl_a)].ravel())
        cols.append(idx[tuple(sl_b)].ravel())
        tvals.append(t.ravel())
        mm_T.append(t.ravel())
    rows = [np.atleast_1d(np.asarray(r)) for r in rows]
    cols = [np.atleast_1d(np.asarray(c)) for c in cols]
    tvals = [np.atleast_1d(np.asarray(t, dtype=np.float64)) for t in tvals]

    diag_extra = np.zeros(nm)
    q = np.zeros(nm)
    if not neumann:
        tb_left = 2.0 * k[:, :, 0] * hd
        tb_right = 2.0 * k[:, :, -1] * hd
        diag_extra[idx[:, :, 0].ravel()] += tb_left.ravel()
        diag_extra[idx[:, :, -1].ravel()] += tb_right.ravel()
        if rhs_dirichlet:
            q[idx[:, :, 0].ravel()] += tb_left.ravel() * 1.0

    # ---- fractures -------------------------------------------------------
    frac_rows, frac_cols, frac_t = [], [], []
    ff_T = []
    cell_col, cell_z, host = [], [], []
    col_plate = []
    col_edges = []
    plate_pieces = []
    plate_offsets = []
    col_offsets = []
    kflat = k.reshape(-1)
    nf = 0
    ncol = 0
    for pi, pl in enumerate(plates):
        pieces = _trace_pieces(pl, h, nx, ny)
        plate_pieces.append(pieces)
        plate_offsets.append(nm + nf)
        col_offsets.append(ncol)
        npc = len(pieces)
        H = pl.zhi - pl.zlo
        if npc == 0 or H <= 0:
            continue
        length = np.hypot(pl.x1 - pl.x0, pl.y1 - pl.y0)
        t0 = np.array([a for (a, _, _, _) in pieces])
        t1 = np.array([b for (_, b, _, _) in pieces])
        ixs = np.array([c for (_, _, c, _) in pieces], dtype=np.int64)
        iys = np.array([c for (_, _, _, c) in pieces], dtype=np.int64)
        lseg = (t1 - t0) * length
        cen = 0.5 * (t0 + t1)
        davg = np.array([_mean_distance_to_line(ix, iy, h, pl) for ix, iy in zip(ixs, iys)])
        davg = np.maximum(davg, 1e-6 * h)
        ci = lseg * w / davg
        kz = np.arange(H, dtype=np.int64)
        pp = np.arange(npc, dtype=np.int64)
        gi = nm + nf + kz[:, None] * npc + pp[None, :]            # [H, npc]
        mz = pl.zlo + kz
        m = ixs[None, :] + nx * (iys[None, :] + ny * mz[:, None])  # [H, npc]
        cell_col.append(np.broadcast_to(ncol + pp, (H, npc)).ravel())
        cell_z.append(np.broadcast_to(mz[:, None], (H, npc)).ravel())
        host.append(m.ravel())
        frac_rows.append(m.ravel())
        frac_cols.append(gi.ravel())
        frac_t.append((kflat[m] * ci[None, :]).ravel())
        if npc > 1:
            d = np.abs(cen[1:] - cen[:-1]) * length
            t = np.broadcast_to(kf * aperture * w / d, (H, npc - 1)).ravel()
            frac_rows.append(gi[:, :-1].ravel())
            frac_cols.append(gi[:, 1:].ravel())
            frac_t.append(t)
            ff_T.append(t)
        if H > 1:
            t = np.broadcast_to(kf * aperture * lseg / h, (H - 1, npc)).ravel()
            frac_rows.append(gi[:-1, :].ravel())
            frac_cols.append(gi[1:, :].ravel())
            frac_t.append(t)
            ff_T.append(t)
        col_plate.append(np.full(npc, pi, dtype=np.int64))
        if npc > 1:
            col_edges.append(np.stack([ncol + pp[:-1], ncol + pp[1:]], axis=1))
        nf += npc * H
        ncol += npc

    # intersections: all plate pairs at once, then per intersecting pair
    npl = len(plates)
    if npl > 1:
        P0 = np.array([[p.x0, p.y0] for p in plates])
        P1 = np.array([[p.x1, p.y1] for p in plates])
        R = P1 - P0
        den = R[:, None, 0] * R[None, :, 1] - R[:, None, 1] * R[None, :, 0]
        W = P0[None, :, :] - P0[:, None, :]
        with np.errstate(divide="ignore", invalid="ignore"):
            ta = (W[..., 0] * R[None, :, 1] - W[..., 1] * R[None, :, 0]) / den
            tb = (W[..., 0] * R[:, None, 1] - W[..., 1] * R[:, None, 0]) / den
        ok = (np.abs(den) > 1e-14) & (ta >= 0) & (ta <= 1) & (tb >= 0) & (tb <= 1)
        ok &= np.triu(np.ones((npl, npl), dtype=bool), 1)
        for a, b in zip(*np.nonzero(ok)):
            pa, pb = plates[a], plates[b]
            if not plate_pieces[a] or not plate_pieces[b]:
                continue
            zlo, zhi = max(pa.zlo, pb.zlo), min(pa.zhi, pb.zhi)
            if zlo >= zhi:
                continue
            qa = _locate(plate_pieces[a], ta[a, b])
            qb = _locate(plate_pieces[b], tb[a, b])
            if qa is None or qb is None:
                continue
            La = np.hypot(*R[a])
            Lb = np.hypot(*R[b])
            ca = 0.5 * (plate_pieces[a][qa][0] + plate_pieces[a][qa][1])
            cb = 0.5 * (plate_pieces[b][qb][0] + plate_pieces[b][qb][1])
            da = max(abs(ta[a, b] - ca) * La, 1e-3 * h)
            db = max(abs(tb[a, b] - cb) * Lb, 1e-3 * h)
            t1_ = kf * aperture * w / da
            t2_ = kf * aperture * w / db
            t = t1_ * t2_ / (t1_ + t2_)
            npa, npb = len(plate_pieces[a]), len(plate_pieces[b])
            mzs = np.arange(zlo, zhi, dtype=np.int64)
            frac_rows.append(plate_offsets[a] + (mzs - pa.zlo) * npa + qa)
            frac_cols.append(plate_offsets[b] + (mzs - pb.zlo) * npb + qb)
            frac_t.append(np.full(len(mzs), t))
            ff_T.append(np.full(len(mzs), t))
            col_edges.append(np.array([[col_offsets[a] + qa, col_offsets[b] + qb]]))

    n = nm + nf
    r_all = np.concatenate(rows + frac_rows).astype(np.int64)
    c_all = np.concatenate(cols + frac_cols).astype(np.int64)
    t_all = np.concatenate(tvals + frac_t).astype(np.float64)
    off = sp.coo_matrix((-t_all, (r_all, c_all)), shape=(n, n)).tocsr()
    off = off + off.T
    off.sum_duplicates()
    diag = -np.asarray(off.sum(axis=1)).ravel()
    diag[:nm] += diag_extra
    A = (off + sp.diags(diag)).tocsr()
    A.sort_indices()
    A.sum_duplicates()

    qf = np.zeros(n)
    qf[:nm] = q
    if sources:
        for m, rate in sources:
            qf[m] += rate

    # projected column graph (CSR, ascending neighbours, no duplicates)
    if ncol:
        e = (np.concatenate(col_edges).astype(np.int64).reshape(-1, 2)
             if col_edges else np.zeros((0, 2), dtype=np.int64))
        g = sp.coo_matrix((np.ones(len(e)), (e[:, 0], e[:, 1])), shape=(ncol, ncol))
        g = (g + g.T).tocsr()
        g.sum_duplicates()
        g.sort_indices()
        col_ptr = g.indptr.astype(np.int64)
        col_adj = g.indices.astype(np.int32)
    else:
        col_ptr = np.zeros(1, dtype=np.int64)
        col_adj = np.zeros(0, dtype=np.int32)

    mmT = np.concatenate(mm_T) if mm_T else np.zeros(1)
    t_ratio = float(np.mean(np.concatenate(ff_T)) / np.mean(mmT)) if ff_T else 0.0
    return FracturedSystem(
        nx=nx, ny=ny, nz=nz, h=h, n_matrix=nm, n=n,
        row_ptr=A.indptr.astype(np.int64), col=A.indices.astype(np.int32),
        val=A.data.astype(np.float64), q=qf, lnk=np.asarray(lnk).reshape(nz, ny, nx),
        cell_col=_cat(cell_col, np.int32),
        cell_z=_cat(cell_z, np.int32),
        col_plate=_cat(col_plate, np.int32),
        col_ptr=col_ptr, col_adj=col_adj,
        plate_zlo=np.asarray([p.zlo for p in plates], dtype=np.int32),
        plate_zhi=np.asarray([p.zhi for p in plates], dtype=np.int32),
        host=_cat(host, np.int64),
        t_ratio=t_ratio, meta=dict(meta or {}))


def random_plates_2d(rng, n_frac, len_lo, len_hi, lx=1.0, ly=1.0, h=0.01):
    """2D segments: centre ~ U(domain), length ~ U(lo,hi)*lx, angle ~ U[0,pi)."""
    plates = []
    for _ in range(n_frac):
        cx, cy = rng.uniform(0, lx), rng.uniform(0, ly)
        L = rng.uniform(len_lo, len_hi) * lx
        th = rng.uniform(0, np.pi)
        dx, dy = 0.5 * L * np.cos(th), 0.5 * L * np.sin(th)
        c = _clip_segment(cx - dx, cy - dy, cx + dx, cy + dy, lx, ly)
        if c is None or np.hypot(c[2] - c[0], c[3] - c[1]) < h:
            continue
        plates.append(Plate(c[0], c[1], c[2], c[3], 0, 1))
    return plates


def random_plates_3d(rng, n_frac, nx, ny, nz, len_cells, h_cells):
    """3D vertical plates: trace centre ~ U(x-y), angle ~ U[0,pi),
    length ~ U{len_cells} cells, height ~ U{h_cells} layers, z0 so it fits."""
    h = 1.0 / nx
    lx, ly = nx * h, ny * h
    plates = []
    for _ in range(n_frac):
        cx, cy = rng.uniform(0, lx), rng.uniform(0, ly)
        L = rng.integers(len_cells[0], len_cells[1] + 1) * h
        th = rng.uniform(0, np.pi)
        H = int(min(rng.integers(h_cells[0], h_cells[1] + 1), nz))
        z0 = int(rng.integers(0, nz - H + 1))
        dx, dy = 0.5 * L * np.cos(th), 0.5 * L * np.sin(th)
        c = _clip_segment(cx - dx, cy - dy, cx + dx, cy + dy, lx, ly)
        if c is None or np.hypot(c[2] - c[0], c[3] - c[1]) < h:
            continue
        plates.append(Plate(c[0], c[1], c[2], c[3], z0, z0 + H))
    return plates


@dataclasses.dataclass
class Well:
    """A rate-controlled vertical well through matrix column (ix, iy), layers
    [zlo, zhi); with ``fractures`` it also perforates the fracture cells
    hosted in those matrix cells."""
    ix: int
    iy: int
    zlo: int
    zhi: int
    rate: float
    fractures: bool = False


def add_wells(sysm: FracturedSystem, wells, kf=None, r_w=0.05) -> FracturedSystem:
    """The system with rate-controlled wells as extra unknowns (the last rows).

    Each perforated cell i couples to its well w through Peaceman's well
    index WI_i = 2 pi k_i h_z / ln(r_e / r_w) with r_e = 0.2 h (square cells,
    isotropic k), r_w in units of h and h_z = h in 3D (per unit thickness in
    2D): the cell's row gains WI_i on the diagonal and -WI_i towards the well,
    and the well's row reads sum_i WI_i (p_w - p_i) = rate (the well's total
    rate).  Fracture perforations take k = kf (default: the contrast in the
    system's meta times the geometric mean of the matrix k, else 1e3 times).
    Row sums of the cell rows are unchanged, so a Neumann system stays one.
    """
    n0, nw = sysm.n, len(wells)
    h = sysm.h
    hz = h if sysm.nz > 1 else 1.0
    k = np.exp(sysm.lnk)
    if kf is None:
        kf = float(sysm.meta.get("contrast", 1e3)) * float(np.exp(sysm.lnk.mean()))
    geo = 2.0 * np.pi * hz / np.log(0.2 / r_w)
    rows, cols, wi = [], [], []
    for w, wl in enumerate(wells):
        for z in range(wl.zlo, wl.zhi):
            m = wl.ix + sysm.nx * (wl.iy + sysm.ny * z)
            rows.append(m)
            cols.append(w)
            wi.append(geo * k[z, wl.iy, wl.ix])
            if wl.fractures:
                for c in np.nonzero(sysm.host == m)[0]:
                    rows.append(sysm.n_matrix + int(c))
                    cols.append(w)
                    wi.append(geo * kf)
    rows, cols, wi = np.asarray(rows), np.asarray(cols), np.asarray(wi)
    A = sysm.csr()
    B = sp.csr_matrix((-wi, (rows, cols)), shape=(n0, nw))
    Ad = A + sp.diags(np.bincount(rows, weights=wi, minlength=n0))
    D = sp.diags(np.bincount(cols, weights=wi, minlength=nw))
    Aw = sp.bmat([[Ad, B], [B.T, D]], format="csr")
    Aw.sort_indices()
    Aw.sum_duplicates()
    q = np.concatenate([sysm.q, [float(wl.rate) for wl in wells]])
    return dataclasses.replace(
        sysm, n=n0 + nw, row_ptr=Aw.indptr.astype(np.int64), col=Aw.indices.astype(np.int32),
        val=Aw.data.astype(np.float64), q=q, n_wells=sysm.n_wells + nw,
        meta=dict(sysm.meta, wells=[dataclasses.asdict(wl) for wl in wells]))
