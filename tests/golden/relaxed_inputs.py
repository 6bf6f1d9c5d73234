"""Writes the stored inputs of the large workloads with the FP64 CPU oracle's forces.

    python tests/golden/relaxed_inputs.py [cfg1] [cfg3] [cfg4]

cfg3, cfg4  relaxed_cfgN.npz: the generated structure after steepest descent
            (workloads.steepest_descent: energy-checked steps of at most 2e-3 nm, until
            max |F| <= 5e3 kJ/mol/nm or 500 force evaluations) on the energy and forces of
            oracle.cl.CellModel for the system with its charges switched off (Lennard-Jones
            and bonds: the packing).  Random placement at liquid density leaves
            overlapping atoms (the mixed types reach sigma = 0.38 nm at 100-120
            atoms/nm^3); relaxing them first gives the bulk, not a few overlaps, the weight
            in every force and gradient norm.  Charges stay off because the water
            hydrogens carry no Lennard-Jones term: with charges on, the energy has no lower
            bound (a hydrogen can fall onto a negative site) and a descent follows it.
cfg1        path_cfg1.npz: 32 beads of the Euler-Maruyama discretisation of eq. (1),
            R^{n+1} = R^n + c F(R^n) + sigma zeta^n with c = dt/(m nu), sigma = 0.005 nm
            and the seeded noise of workloads.path_noise (workloads.drifted_path), forces
            from oracle.potential.Model.

Every file records the digest of the generated system it started from, so a changed
generator is detected when the inputs are loaded (workloads.load_stored).
"""
from __future__ import annotations

import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import workloads as W  # noqa: E402
from oracle import cl  # noqa: E402
from oracle import path as OP  # noqa: E402
from oracle.potential import Model  # noqa: E402


def log(*a):
    print(*a, flush=True)


def relaxed(name):
    s = W.CONFIGS[name]["make"]()
    m0 = cl.CellModel(dict(s, charge=np.zeros(s["Q"])))
    t0 = time.perf_counter()
    x, it, fm = W.steepest_descent(s, lambda X: m0.eval(X)[:2], log=log)
    fn = np.linalg.norm(cl.CellModel(s).forces(x), axis=1)
    f0 = np.linalg.norm(cl.CellModel(s).forces(s["x"]), axis=1)
    log(f"{name}: {it} iterations, packing max|F| {fm:.3e}; full potential: max|F| "
        f"{fn.max():.3e} (before {f0.max():.3e}), median {np.median(fn):.3e} "
        f"(before {np.median(f0):.3e}), {time.perf_counter() - t0:.0f} s")
    out = os.path.join(W.STORE_DIR, W.STORED[name])
    np.savez_compressed(out, x=x, digest=np.array(W.system_digest(s)), iterations=it,
                        packing_max_force=fm, max_force=float(fn.max()),
                        median_force=float(np.median(fn)))
    log(f"wrote {out}")


def cfg1_path():
    s = W.cfg1()
    c = W.CONFIGS["cfg1"]
    m = Model(s)
    coef, _ = OP.coefficients(m)
    R, _, _ = W.drifted_path(s, c["N"], c["path_seed"], lambda X: coef[:, None] * m.forces(X),
                             c["sigma"])
    out = os.path.join(W.STORE_DIR, W.STORED["cfg1"])
    np.savez_compressed(out, R=R, digest=np.array(W.system_digest(s)))
    log(f"cfg1: Euler-Maruyama path {R.shape}; wrote {out}")


if __name__ == "__main__":
    names = sys.argv[1:] or ["cfg1", "cfg3", "cfg4"]
    for n in names:
        if n == "cfg1":
            cfg1_path()
        else:
            relaxed(n)
