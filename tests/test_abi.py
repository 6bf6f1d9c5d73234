"""C-ABI contract tests that need no GPU: the library loads, exports every function
include/mop.h declares, and rejects bad system descriptions on the host."""
import ctypes as C
import os
import re

import numpy as np
import pytest

import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mop.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[A-Za-z_][\w\s\*]*?\b([a-z_][a-z0-9_]*)\s*\(", text, flags=re.M)
    return sorted(set(n for n in names if n not in ("if", "while", "for", "sizeof")))


@pytest.fixture(scope="module")
def mop():
    import paper_2501_11962_amd as m
    if not os.path.exists(m.LIB_PATH):
        from paper_2501_11962_amd import build
        build.build()
    return m


def test_header_declares_the_four_path_calls():
    names = declared_functions()
    for n in ("veff_energy", "veff_grad", "bead_forces", "bead_hvp"):
        assert n in names


def test_library_exports_every_declared_symbol(mop):
    L = mop.lib()
    names = declared_functions()
    assert len(names) >= 20
    for n in names:
        assert hasattr(L, n), n
    assert set(names) == set(mop.EXPORTS)


def test_binding_constants_match_the_header(mop):
    """Every MOP_* constant the Python binding defines has the header's value, and the
    binding's phase names follow the header's phase indices."""
    h = open(os.path.join(ROOT, "include", "mop.h")).read()
    d = {m.group(1): int(m.group(2)) for m in re.finditer(r"#define (MOP_\w+)\s+\(?(-?\d+)\)?", h)}
    names = [k for k in dir(mop) if k.startswith("MOP_")]
    assert names
    for k in names:
        assert d[k] == getattr(mop, k), k
    assert len(mop.PHASES) == d["MOP_NPHASES"]
    for i, ph in enumerate(mop.PHASES):
        assert d["MOP_PHASE_" + ph.upper()] == i


def test_strerror(mop):
    L = mop.lib()
    for code in (0, -1, -2, -3, -4, -5, -6, -7):
        assert L.mop_strerror(code)
    assert L.mop_strerror(-2).decode().startswith("cutoff")


def test_system_check_accepts_workloads(mop):
    for s in (W.cfg1(), W.cfg2(), W.cfg3(), W.tiny(), W.water_box(1002, 3)):
        assert mop.system_check(s) == 0
        assert mop.system_check(s, use_molecules=True) == 0


def test_system_check_rejections(mop):
    s = W.tiny()
    bad = dict(s, rc=0.81)                      # >= box/2
    assert mop.system_check(bad) == -2
    bad = dict(s, rc=0.0)
    assert mop.system_check(bad) == -2
    t = s["type"].copy()
    t[3] = 7
    assert mop.system_check(dict(s, type=t)) == -3
    m = s["mass"].copy()
    m[0] = 0.0
    assert mop.system_check(dict(s, mass=m)) == -1
    # a ring of three bonded atoms is not a linear chain
    ring = dict(s, bonds=np.array([[0, 1], [1, 2], [2, 0]]), bond_r0=np.full(3, 0.3),
                bond_k=np.full(3, 1e3))
    assert mop.system_check(ring) == -6
    # explicit molecule keys make any topology acceptable
    assert mop.system_check(ring, use_molecules=True) == 0
    b = s["bonds"].copy()
    b[0, 1] = s["Q"] + 5
    assert mop.system_check(dict(s, bonds=b)) == -1
    sig = np.full(17, 0.3)
    assert mop.system_check(dict(s, sigma=sig, epsilon=sig)) == -3
    # exclusion keys are numbered compactly, so sparse molecule ids are fine; a chain
    # position that would push the keys past 2^27 is refused
    sparse = dict(s, mol=np.asarray(s["mol"], np.int64) * 40000000 + 7)
    assert mop.system_check(sparse, use_molecules=True) == 0
    far = np.asarray(s["molpos"]).copy()
    far[0] = 1 << 27
    assert mop.system_check(dict(s, molpos=far), use_molecules=True) == -6


def test_ctx_create_reports_missing_device(mop):
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    h = C.c_void_p()
    assert mop.lib().mop_ctx_create(0, None, C.byref(h)) == -4


def test_calls_reject_null_handles(mop):
    L = mop.lib()
    assert L.bead_forces(None, None, 1, None, None, None) == -1
    assert L.veff_grad(None, None, 1, None, None, 0, 0.0, None) == -1
    assert L.veff_energy(None, None, 1, None, None, None, None) == -1
    assert L.bead_hvp(None, None, None, 1, None, None) == -1
    assert L.mop_batch_create(0, None, None, C.byref(C.c_void_p())) == -1


def test_system_check_pme(mop):
    s = W.tiny()
    assert mop.system_check(W.with_pme(s)) == 0
    assert mop.system_check(W.with_pme(s, order=8)) == 0
    assert mop.system_check(dict(W.with_pme(s), pme_grid=None)) == 0        # automatic grid
    assert mop.system_check(W.with_pme(s, order=5)) == -1                   # odd order
    assert mop.system_check(W.with_pme(s, grid=[14, 14, 3])) == -1          # below the order
    assert mop.system_check(W.with_pme(s, grid=[1024, 1024, 256])) == -1    # too many points
    assert mop.system_check(W.with_pme(s, rtol=1.0)) == -1
    with pytest.raises(ValueError):
        mop.system_check(dict(s, elec="coulomb"))


def test_ewald_erfc_constants_match_their_fit():
    """The Ewald pair kernels' erfc polynomial is the one erfc_fit.py produces, and its
    FP32 evaluation stays within 4e-7 relative error of erfc on 0 <= x <= 6."""
    from scipy.special import erfc
    from paper_2501_11962_amd import erfc_fit as EF
    src = open(os.path.join(ROOT, "paper_2501_11962_amd", "csrc", "kernels_pair.hip")).read()
    body = src[src.index("float erfc_ex2("):]
    body = body[:body.index("return")]
    consts = [float(v) for v in re.findall(r"(-?\d\.\d+e[-+]\d+)f", body)]
    x, _, coef = EF.fit()
    assert len(consts) == EF.DEG + 1
    assert np.allclose(consts[::-1], coef, rtol=1e-8, atol=0)
    p = EF.eval_f32(np.array(consts[::-1]), x).astype(np.float64)
    e = np.abs(np.exp(-x * x) * p - erfc(x)) / erfc(x)
    assert e.max() < 4e-7


def test_loaded_library_is_the_selected_build(mop):
    """The process maps the library file the binding selected (the in-tree build, or the
    host-sanitized one when MOP_LIBRARY names it)."""
    mop.lib()
    maps = open("/proc/self/maps").read()
    assert os.path.realpath(mop.LIB_PATH) in maps


def test_system_check_of_every_workload_size(mop):
    """Host validation and exclusion-key numbering at the benchmark sizes (150,000 atoms
    with 50-atom chains and waters; PME variants)."""
    s4 = W.cfg4()
    assert mop.system_check(s4) == 0
    assert mop.system_check(s4, use_molecules=True) == 0
    assert mop.system_check(W.with_pme(s4)) == 0
    for s_, _, _ in W.cfg5()[:4]:
        assert mop.system_check(s_) == 0
