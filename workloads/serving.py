"""Request streams for the serving form (seeded, synthetic).

A stream of solve requests on 3D EDFM systems whose grids are cubes with a
side drawn uniformly from [side_lo, side_hi] (32..128 at full size), 10-300
vertical plates, fracture/matrix contrast log-uniform in [1e3, 1e6] and a
basis variant drawn uniformly.  Each request reuses its setup for 1-16
right-hand sides: the Dirichlet boundary term plus 2-8 point sources/sinks
in matrix cells whose rates sum to zero.  Arrivals form a Poisson process.

Building a system in numpy takes seconds at these sizes, so a stream draws
its systems from a pool of `pool` distinct systems (each request still runs
its own setup on the device); the pool spans the side range evenly.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from .edfm import build_system, lnk_field, random_plates_3d

# grid shapes of the serving requests; coarsening 10^3, fracture d_min = r_z = 8
SERVING = dict(side=(32, 128), n_frac=(10, 300), contrast=(1e3, 1e6), nrhs=(1, 16),
               n_wells=(2, 8), std=3.0, corr=(4, 8, 8), coarse=(10, 10, 10), d_min=8, r_z=8)


def _rng(*key):
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence([1705, 5784, 4, *key])))


@dataclass
class ServingRequest:
    rid: int
    system: object               # workloads.FracturedSystem
    variant: int                 # 0 Decoupled, 1 Frac, 2 Rock, 3 Coupled
    rhs: np.ndarray              # float64 [nrhs, n]
    arrival: float               # seconds after the stream starts
    meta: dict = field(default_factory=dict)


def make_system(side: int, n_frac: int, contrast: float, seed: int):
    """One cubic serving system of side `side` (plates scaled to the grid)."""
    rng = _rng(0, seed)
    lnk = lnk_field((side, side, side), SERVING["std"], SERVING["corr"], rng)
    lo = max(4, side // 5)
    plates = random_plates_3d(rng, n_frac, side, side, side, (lo, max(lo, 3 * side // 5)),
                              (max(2, side // 10), max(2, 2 * side // 5)))
    return build_system(side, side, side, lnk, plates, contrast,
                        meta=dict(side=side, n_frac=n_frac, contrast=contrast, seed=seed))


def well_rhs(sysm, n_wells: int, rng) -> np.ndarray:
    """Boundary term plus n_wells point rates in matrix cells summing to zero."""
    q = sysm.q.copy()
    cells = rng.choice(sysm.n_matrix, size=n_wells, replace=False)
    scale = float(np.abs(sysm.q).max()) or 1.0
    rates = rng.uniform(0.5, 2.0, n_wells) * scale * np.where(np.arange(n_wells) % 2 == 0, 1.0, -1.0)
    rates[-1] -= rates.sum()
    np.add.at(q, cells, rates)
    return q


def make_stream(n_requests: int, rate: float, pool: int = 8, seed: int = 0,
                side=None, n_frac=None, nrhs=None, variants=(0, 1, 2, 3)) -> list[ServingRequest]:
    """A Poisson stream of `n_requests` requests at `rate` requests/s."""
    side = side or SERVING["side"]
    n_frac = n_frac or SERVING["n_frac"]
    nrhs = nrhs or SERVING["nrhs"]
    rng = _rng(1, seed)
    sides = np.linspace(side[0], side[1], pool).round().astype(int)
    systems = []
    for k, s in enumerate(sides):
        nf = int(rng.integers(n_frac[0], n_frac[1] + 1))
        c = float(np.exp(rng.uniform(np.log(SERVING["contrast"][0]), np.log(SERVING["contrast"][1]))))
        systems.append(make_system(int(s), nf, c, seed * 1000 + k))
    t = 0.0
    reqs = []
    for rid in range(n_requests):
        t += float(rng.exponential(1.0 / rate)) if rate > 0 else 0.0
        sysm = systems[int(rng.integers(pool))]
        k = int(rng.integers(nrhs[0], nrhs[1] + 1))
        w = SERVING["n_wells"]
        rhs = np.stack([well_rhs(sysm, int(rng.integers(w[0], w[1] + 1)), rng) for _ in range(k)])
        reqs.append(ServingRequest(rid, sysm, int(variants[int(rng.integers(len(variants)))]), rhs,
                                   t, meta=dict(side=sysm.nx, n=sysm.n, nrhs=k)))
    return reqs
