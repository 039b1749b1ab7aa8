"""The five benchmark workloads and small variants of them, all seeded.

Seeds: numpy PCG64 from SeedSequence([1705, 5784, config_id, instance]).
Each config reproduces the shapes of one of the paper's test families:
2D 100x100 with 20 segments; 3D blocks with vertical rectangular plates.
"""
from __future__ import annotations

import numpy as np

from .edfm import build_system, lnk_field, random_plates_2d, random_plates_3d

# name -> parameters; coarsening (cx, cy, cz), fracture d_min and r_z
CONFIGS = {
    1: dict(dims=(100, 100, 1), std=2.0, corr=(10, 10), n_frac=20, len2d=(0.2, 0.5),
            contrast=1e4, coarse=(10, 10, 1), d_min=10, r_z=1),
    2: dict(dims=(100, 100, 50), std=3.0, corr=(4, 8, 8), n_frac=100, len3d=(20, 60),
            h3d=(10, 40), contrast=1e4, coarse=(10, 10, 10), d_min=8, r_z=8),
    3: dict(dims=(200, 200, 50), std=3.0, corr=(4, 8, 8), n_frac=400, len3d=(20, 60),
            h3d=(5, 25), contrast=1e4, coarse=(10, 10, 10), d_min=10, r_z=10),
    5: dict(dims=(256, 256, 128), std=4.0, corr=(4, 8, 8), n_frac=2000, len3d=(20, 60),
            h3d=(5, 15), contrast=1e6, coarse=(10, 10, 10), d_min=10, r_z=10),
}


def _rng(config_id, instance):
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence([1705, 5784, config_id, instance])))


def make_config(config_id: int, instance: int = 0, contrast=None, dims=None, n_frac=None,
                neumann=False):
    """Generate config ``config_id``; ``dims``/``n_frac`` shrink it for tests."""
    c = dict(CONFIGS[config_id])
    if dims is not None:
        c["dims"] = dims
    if n_frac is not None:
        c["n_frac"] = n_frac
    if contrast is not None:
        c["contrast"] = contrast
    nx, ny, nz = c["dims"]
    rng = _rng(config_id, instance)
    if nz == 1:
        lnk = lnk_field((1, ny, nx), c["std"], (0, c["corr"][1], c["corr"][0]), rng)
        plates = random_plates_2d(rng, c["n_frac"], *c["len2d"], lx=1.0, ly=ny / nx, h=1.0 / nx)
    else:
        lnk = lnk_field((nz, ny, nx), c["std"], c["corr"], rng)
        plates = random_plates_3d(rng, c["n_frac"], nx, ny, nz, c["len3d"], c["h3d"])
    sysm = build_system(nx, ny, nz, lnk, plates, c["contrast"], neumann=neumann,
                        meta=dict(config=config_id, instance=instance, **c))
    return sysm


def make_small(kind: str, seed: int = 0, **kw):
    """Small systems for parity tests (a few hundred to a few thousand cells)."""
    rng = _rng(900, seed)
    if kind == "2d":
        nx, ny = kw.get("nx", 24), kw.get("ny", 20)
        lnk = lnk_field((1, ny, nx), kw.get("std", 1.5), (0, 3, 3), rng)
        plates = random_plates_2d(rng, kw.get("n_frac", 4), 0.2, 0.5, lx=1.0, ly=ny / nx, h=1.0 / nx)
        return build_system(nx, ny, 1, lnk, plates, kw.get("contrast", 1e3),
                            neumann=kw.get("neumann", False), meta=dict(kind=kind, seed=seed))
    if kind == "3d":
        nx, ny, nz = kw.get("nx", 16), kw.get("ny", 14), kw.get("nz", 12)
        lnk = lnk_field((nz, ny, nx), kw.get("std", 1.5), (2, 3, 3), rng)
        if "lnk_hook" in kw:    # tests: edit the field (same geometry and seeds)
            lnk = kw["lnk_hook"](lnk)
        plates = random_plates_3d(rng, kw.get("n_frac", 5), nx, ny, nz,
                                  kw.get("len3d", (6, 12)), kw.get("h3d", (4, 9)))
        return build_system(nx, ny, nz, lnk, plates, kw.get("contrast", 1e3),
                            neumann=kw.get("neumann", False), meta=dict(kind=kind, seed=seed))
    raise ValueError(kind)


def config_rhs(sysm, config_id: int, nrhs: int, instance: int = 0) -> np.ndarray:
    """Right-hand sides of a config that reuses one setup (config 5: 64 of
    them): the Dirichlet boundary term plus 2-8 point rates in matrix cells
    summing to zero, as in the serving requests.  Row k is right-hand side k."""
    from .serving import well_rhs
    rng = _rng(config_id, 10**6 + instance)
    return np.stack([well_rhs(sysm, int(rng.integers(2, 9)), rng) for _ in range(nrhs)])
