"""FP64 CPU oracle of the F-AMS pressure solve -- TEST INFRASTRUCTURE ONLY.

This package is a plain, slow, obviously-correct restatement of what the paper
(Tene, Al Kobaisi, Hajibeygi, "Algebraic multiscale method for flow in
heterogeneous porous media with embedded discrete fractures (F-AMS)") says the
method computes.  It exists to check the GPU library; only the tests, the
smoke check and the CPU-baseline leg of the benchmark may import it.  The GPU
library never calls it, and it shares no code with the library.

Modules:
  grids    -- coarse grids: structured wirebasket classes (Sec. 3, Fig. 2) and
              the distance-based fracture coarsening (Table 2, Sec. 4.1, and
              its extrusion along z, Sec. 4.3).
  fams     -- basis functions per coupling strategy (Sec. 3.1, App. A),
              truncation (Sec. 4.3), coarse operator R A P with R = P^T
              (Sec. 3.2, App. A), ILU(0) (Sec. 3.2), the two-stage iteration
              (Table 1) as a Richardson loop or inside right-preconditioned
              GMRES (Sec. 4.6).
  flux     -- finite-volume stage and conservative flux reconstruction
              (Sec. 3.2; the paper states it exists after any R^FV stage but
              gives no algorithm -- the standard MSFV reconstruction is used).
  ilu0.c   -- the ILU(0) factorisation and triangular solves in plain C.

Parity pins for every function live in tests/test_oracle_*.py.
"""
