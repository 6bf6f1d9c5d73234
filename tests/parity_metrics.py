"""Error measures of the parity tests (GPU result a against FP64 oracle b, per atom rows).

A relative L2 norm over a whole bead is dominated by the atoms with the largest values;
the per-atom measures below make sure the bulk of the atoms is pinned too:
    bulk   relative L2 over the atoms whose oracle value is at or below the 90th
           percentile of |b_i| (the largest tenth left out);
    worst  max_i |a_i - b_i| / (|b_i| + median_i |b_i|): every atom's error against its
           own size, floored by the typical size (so atoms whose value nearly vanishes
           are not compared with zero).
"""
import numpy as np


def rel(a, b):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def per_atom(a, b):
    a = np.asarray(a, np.float64).reshape(-1, 3)
    b = np.asarray(b, np.float64).reshape(-1, 3)
    nb = np.linalg.norm(b, axis=1)
    nd = np.linalg.norm(a - b, axis=1)
    keep = nb <= np.percentile(nb, 90.0)
    bulk = float(np.linalg.norm(nd[keep]) / max(np.linalg.norm(nb[keep]), 1e-300))
    worst = float(np.max(nd / (nb + np.median(nb) + 1e-300)))
    return bulk, worst


def check(a, b, tol, what=""):
    """relL2 <= tol, bulk relL2 <= tol and worst <= 10 tol; returns a one-line summary."""
    e = rel(a, b)
    bulk, worst = per_atom(a, b)
    msg = f"{what} relL2 {e:.2e}, bulk {bulk:.2e}, worst atom {worst:.2e}"
    assert e < tol and bulk < tol and worst < 10.0 * tol, msg
    return msg
