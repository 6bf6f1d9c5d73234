"""FP64 CPU oracle for the Onsager-Machlup path gradient -- TEST INFRASTRUCTURE ONLY.

Only the test suite, the package smoke check and the CPU-baseline leg of the benchmark
may import, call, link or execute anything in this folder.  The HIP library never
routes through it and shares no code with it.

Contents
    potential.py  U, F = -grad U and the Hessian-vector product H v of the short-range
                  potential (shifted-force Lennard-Jones + reaction field, harmonic
                  bonds, 1-2/1-3 exclusions), by brute force over all minimum-image pairs.
    ewald.py      The Ewald sum of periodic Coulomb interactions (real, reciprocal, self,
                  excluded-pair and background terms), the definition PME approximates.
    pme.py        Smooth particle-mesh Ewald: spline weights, charge grid, influence
                  function, energy, forces and the exact Hessian-vector product.
                  potential.Model uses it (with the Ewald real-space pair term) for
                  systems with elec = "pme".
    path.py       The effective potential of eq. (3), its exact gradient, the
                  finite-difference Hessian term of eq. (5), and a literal evaluation of
                  the effective forces of eqs. (5)-(7).
    celllist.c    The same U / F / H v in plain C with a cell list for neighbour search
                  (OpenMP over atoms), for large systems and the timed CPU baseline.
    cl.py         ctypes wrapper of celllist.c.

Pins (tests/test_oracle_*.py) tie every function to something other than itself:
textbook closed forms for the pair terms, central finite differences, translation
invariance, Hessian symmetry, automatic differentiation of the energy, brute force vs
cell list, and path identities (a drift-only Euler path has zero spring energy; a
recorded-noise path has residuals equal to the noise).  See each function's docstring
for the passage it follows.
"""
