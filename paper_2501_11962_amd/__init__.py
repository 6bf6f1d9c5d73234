"""Python binding of libmop.so: the Onsager-Machlup path gradient on MI355X (gfx950).

Names follow the C ABI of include/mop.h.  This module only marshals arguments: every
step of the computation runs in the HIP kernels of libmop.so, and PyTorch supplies
device memory and the current stream.  There is no CPU fallback: importing works
without a GPU, but any call fails loudly when the library or the device is missing.

    ctx = Context()                       # device of torch.cuda.current_device()
    sys_ = System(ctx, system_dict)       # system description (see workloads)
    plan = Plan(sys_, max_beads=16)
    G, veff = veff_grad(plan, R)          # R: (N, Q, 3) float64 CUDA tensor
    v = VeffFn.apply(R, plan)             # autograd: backward is veff_grad
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# MOP_LIBRARY selects another build of the same library (the host-sanitized one of
# build.py --sanitize, loaded by the sanitizer test with its runtime preloaded)
LIB_PATH = os.environ.get("MOP_LIBRARY") or os.path.join(_HERE, "libmop.so")

MOP_OK = 0
MOP_DEV_NONFINITE = 1
MOP_DEV_CAPACITY = 2
MOP_DEV_OVERLAP = 4
MOP_STATIC_WORKSPACE_BYTES = 67108864
MOP_PLAN_NEWTON3 = 1
MOP_PLAN_ONE_STREAM = 2
MOP_PLAN_PERSISTENT = 4
MOP_ELEC_RF, MOP_ELEC_PME = 0, 1

_lib = None


class MopError(RuntimeError):
    def __init__(self, code, what=""):
        self.code = code
        msg = lib().mop_strerror(code).decode() if _lib is not None else str(code)
        super().__init__(f"{what}: {msg} (code {code})" if what else f"{msg} (code {code})")


class _Desc(C.Structure):
    _fields_ = [
        ("Q", C.c_int32), ("box", C.c_double * 3),
        ("mass", C.c_void_p), ("charge", C.c_void_p), ("type", C.c_void_p),
        ("ntypes", C.c_int32), ("sigma", C.c_void_p), ("epsilon", C.c_void_p),
        ("nbonds", C.c_int32), ("bond_ij", C.c_void_p), ("bond_r0", C.c_void_p),
        ("bond_k", C.c_void_p), ("excl_mol", C.c_void_p), ("excl_pos", C.c_void_p),
        ("r_cut", C.c_double), ("eps_rf", C.c_double), ("eps_r", C.c_double),
        ("dt", C.c_double), ("nu", C.c_double),
        ("elec", C.c_int32), ("pme_order", C.c_int32), ("ewald_rtol", C.c_double),
        ("pme_grid", C.c_int32 * 3),
    ]


class _PmdParams(C.Structure):
    _fields_ = [("tau", C.c_double), ("gamma", C.c_double), ("kT", C.c_double),
                ("seed", C.c_uint64)]


class _BiasDesc(C.Structure):
    _fields_ = [("nA", C.c_int32), ("nB", C.c_int32), ("groupA", C.c_void_p),
                ("groupB", C.c_void_p), ("sigma", C.c_double), ("height", C.c_double),
                ("bias_factor", C.c_double), ("kT", C.c_double), ("stride", C.c_int32),
                ("max_gaussians", C.c_int32)]


class _Opts(C.Structure):
    _fields_ = [("col_width", C.c_double), ("zbin", C.c_double), ("waves", C.c_int32),
                ("flags", C.c_int32), ("list_cap", C.c_int32)]


EXPORTS = [
    "mop_system_check", "mop_ctx_create", "mop_ctx_set_stream", "mop_ctx_destroy",
    "mop_system_create", "mop_system_destroy", "mop_plan_create", "mop_plan_destroy",
    "mop_workspace_size", "bead_forces", "bead_hvp", "veff_energy", "veff_grad",
    "mop_batch_create", "mop_batch_destroy", "mop_batch_workspace_size",
    "mop_batch_veff_grad", "mop_status", "mop_status_clear", "mop_strerror", "mop_plan_info",
    "veff_grad_timed", "pmd_step", "mop_bias_create", "mop_bias_destroy", "mop_bias_reset",
    "mop_bias_apply", "mop_bias_history", "mop_system_pme_info", "bead_forces_static",
]
PHASES = ["bin", "force", "pme_force", "resid", "hvp", "pme_hvp", "fd", "assemble"]


def lib():
    """Load libmop.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2501_11962_amd.build`")
    L = C.CDLL(LIB_PATH)
    vp, i32, pp = C.c_void_p, C.c_int32, C.POINTER(C.c_void_p)
    sig = {
        "mop_system_check": ([C.POINTER(_Desc)], C.c_int),
        "mop_ctx_create": ([C.c_int, vp, pp], C.c_int),
        "mop_ctx_set_stream": ([vp, vp], C.c_int),
        "mop_ctx_destroy": ([vp], None),
        "mop_system_create": ([vp, C.POINTER(_Desc), pp], C.c_int),
        "mop_system_destroy": ([vp], None),
        "mop_plan_create": ([vp, i32, C.POINTER(_Opts), pp], C.c_int),
        "mop_plan_destroy": ([vp], None),
        "mop_workspace_size": ([vp, C.POINTER(C.c_size_t)], C.c_int),
        "bead_forces": ([vp, vp, i32, vp, vp, vp], C.c_int),
        "bead_hvp": ([vp, vp, vp, i32, vp, vp], C.c_int),
        "veff_energy": ([vp, vp, i32, vp, vp, vp, vp], C.c_int),
        "veff_grad": ([vp, vp, i32, vp, vp, i32, C.c_double, vp], C.c_int),
        "mop_batch_create": ([i32, vp, vp, pp], C.c_int),
        "mop_batch_destroy": ([vp], None),
        "mop_batch_workspace_size": ([vp, C.POINTER(C.c_size_t)], C.c_int),
        "mop_batch_veff_grad": ([vp, vp, vp, vp, i32, C.c_double, vp], C.c_int),
        "mop_status": ([vp, vp, C.POINTER(C.c_int32)], C.c_int),
        "mop_status_clear": ([vp, vp], C.c_int),
        "mop_strerror": ([C.c_int], C.c_char_p),
        "mop_plan_info": ([vp, C.POINTER(i32), C.POINTER(i32), C.POINTER(i32), C.POINTER(i32)], C.c_int),
        "veff_grad_timed": ([vp, vp, i32, vp, vp, i32, C.c_double, vp, C.POINTER(C.c_float)], C.c_int),
        "pmd_step": ([vp, vp, vp, vp, vp, i32, C.POINTER(_PmdParams), C.c_uint64, i32, vp, vp],
                     C.c_int),
        "mop_bias_create": ([vp, C.POINTER(_BiasDesc), pp], C.c_int),
        "mop_bias_destroy": ([vp], None),
        "mop_bias_reset": ([vp], C.c_int),
        "mop_bias_apply": ([vp, vp, i32, vp, vp, i32, vp], C.c_int),
        "mop_bias_history": ([vp, C.POINTER(i32), vp, vp, i32], C.c_int),
        "mop_system_pme_info": ([vp, C.POINTER(i32), C.POINTER(C.c_double)], C.c_int),
        "bead_forces_static": ([vp, vp, i32, vp, vp, vp], C.c_int),
    }
    for name, (args, res) in sig.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = res
    _lib = L
    return L


def _check(code, what):
    if code != MOP_OK:
        raise MopError(code, what)


def _torch():
    import torch
    return torch


def _stream_ptr():
    torch = _torch()
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t):
    return C.c_void_p(0 if t is None else t.data_ptr())


def _dev_tensor(t, dtype, shape=None):
    torch = _torch()
    if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == dtype and t.is_contiguous()):
        raise TypeError(f"expected a contiguous CUDA tensor of {dtype}")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"expected shape {tuple(shape)}, got {tuple(t.shape)}")
    return t


def _beads(plan, R):
    """R must be (B, Q, 3) float64 on the device, Q the plan's atom count: the library
    takes only the bead count and reads B * Q * 3 values."""
    torch = _torch()
    _dev_tensor(R, torch.float64)
    if R.dim() != 3 or R.shape[0] < 1 or R.shape[1] != plan.Q or R.shape[2] != 3:
        raise ValueError(f"expected shape (beads, {plan.Q}, 3), got {tuple(R.shape)}")
    return R


class _HostArrays:
    """Keeps the host arrays of a descriptor alive."""

    def __init__(self, system, use_molecules=False):
        s = system
        self.mass = np.ascontiguousarray(s["mass"], np.float64)
        self.charge = np.ascontiguousarray(s["charge"], np.float64)
        self.type = np.ascontiguousarray(s["type"], np.int32)
        self.sigma = np.ascontiguousarray(s["sigma"], np.float64)
        self.epsilon = np.ascontiguousarray(s["epsilon"], np.float64)
        self.bonds = np.ascontiguousarray(np.asarray(s["bonds"]).reshape(-1, 2), np.int32)
        self.r0 = np.ascontiguousarray(s["bond_r0"], np.float64)
        self.kb = np.ascontiguousarray(s["bond_k"], np.float64)
        self.mol = np.ascontiguousarray(s["mol"], np.int32) if use_molecules else None
        self.pos = np.ascontiguousarray(s["molpos"], np.int32) if use_molecules else None
        d = _Desc()
        d.Q = int(s["Q"])
        d.box[:] = [float(v) for v in s["box"]]
        d.mass, d.charge, d.type = self.mass.ctypes.data, self.charge.ctypes.data, self.type.ctypes.data
        d.ntypes = int(self.sigma.shape[0])
        d.sigma, d.epsilon = self.sigma.ctypes.data, self.epsilon.ctypes.data
        d.nbonds = int(self.bonds.shape[0])
        d.bond_ij = self.bonds.ctypes.data if d.nbonds else None
        d.bond_r0 = self.r0.ctypes.data if d.nbonds else None
        d.bond_k = self.kb.ctypes.data if d.nbonds else None
        d.excl_mol = self.mol.ctypes.data if use_molecules else None
        d.excl_pos = self.pos.ctypes.data if use_molecules else None
        d.r_cut, d.eps_rf = float(s["rc"]), float(s["eps_rf"])
        d.eps_r, d.dt, d.nu = float(s.get("eps_r", 1.0)), float(s["dt"]), float(s["nu"])
        elec = s.get("elec", "rf")
        if elec not in ("rf", "pme"):
            raise ValueError("elec must be 'rf' or 'pme'")
        d.elec = MOP_ELEC_PME if elec == "pme" else MOP_ELEC_RF
        if elec == "pme":
            d.pme_order = int(s.get("pme_order", 0))
            d.ewald_rtol = float(s.get("ewald_rtol", 0.0))
            g = s.get("pme_grid")
            d.pme_grid[:] = [0, 0, 0] if g is None else [int(k) for k in g]
        self.desc = d


def system_check(system, use_molecules=False):
    """Host-only validation of a system description (return code)."""
    h = _HostArrays(system, use_molecules)
    return lib().mop_system_check(C.byref(h.desc))


class Context:
    def __init__(self, device=None, stream=None):
        torch = _torch()
        if not torch.cuda.is_available():
            raise RuntimeError("no GPU available: the HIP library has no CPU path")
        self.device = torch.cuda.current_device() if device is None else int(device)
        h = C.c_void_p()
        st = C.c_void_p(stream) if stream is not None else _stream_ptr()
        _check(lib().mop_ctx_create(self.device, st, C.byref(h)), "mop_ctx_create")
        self.h = h

    def set_stream(self, stream_ptr=None):
        st = C.c_void_p(stream_ptr) if stream_ptr is not None else _stream_ptr()
        _check(lib().mop_ctx_set_stream(self.h, st), "mop_ctx_set_stream")

    def __del__(self):
        if getattr(self, "h", None) and _lib is not None:
            _lib.mop_ctx_destroy(self.h)
            self.h = None


class System:
    def __init__(self, ctx, system, use_molecules=False):
        self.ctx = ctx
        self.Q = int(system["Q"])
        self._host = _HostArrays(system, use_molecules)
        h = C.c_void_p()
        _check(lib().mop_system_create(ctx.h, C.byref(self._host.desc), C.byref(h)),
               "mop_system_create")
        self.h = h

    def pme_info(self):
        """(grid (3,), beta) of a PME system."""
        g = (C.c_int32 * 3)()
        b = C.c_double()
        _check(lib().mop_system_pme_info(self.h, g, C.byref(b)), "mop_system_pme_info")
        return [int(v) for v in g], float(b.value)

    def __del__(self):
        if getattr(self, "h", None) and _lib is not None:
            _lib.mop_system_destroy(self.h)
            self.h = None


class Plan:
    """Plan for up to max_beads beads; owns a device workspace (torch uint8)."""

    def __init__(self, system, max_beads, col_width=0.0, zbin=0.0, waves=0, newton3=False,
                 list_cap=0, one_stream=False, persistent=False):
        torch = _torch()
        self.system = system
        self.Q = system.Q
        self.max_beads = int(max_beads)
        flags = ((MOP_PLAN_NEWTON3 if newton3 else 0) | (MOP_PLAN_ONE_STREAM if one_stream else 0)
                 | (MOP_PLAN_PERSISTENT if persistent else 0))
        o = _Opts(col_width, zbin, waves, flags, int(list_cap))
        h = C.c_void_p()
        _check(lib().mop_plan_create(system.h, self.max_beads, C.byref(o), C.byref(h)),
               "mop_plan_create")
        self.h = h
        n = C.c_size_t()
        _check(lib().mop_workspace_size(h, C.byref(n)), "mop_workspace_size")
        self.ws_bytes = int(n.value)
        self.ws = torch.zeros(self.ws_bytes, dtype=torch.uint8, device=f"cuda:{system.ctx.device}")

    def info(self):
        v = [C.c_int32() for _ in range(4)]
        _check(lib().mop_plan_info(self.h, *[C.byref(x) for x in v]), "mop_plan_info")
        return dict(ncx=v[0].value, ncy=v[1].value, nzb=v[2].value, slots=v[3].value)

    def status(self):
        s = C.c_int32()
        _check(lib().mop_status(self.h, _ptr(self.ws), C.byref(s)), "mop_status")
        return int(s.value)

    def clear_status(self):
        _check(lib().mop_status_clear(self.h, _ptr(self.ws)), "mop_status_clear")

    def __del__(self):
        if getattr(self, "h", None) and _lib is not None:
            _lib.mop_plan_destroy(self.h)
            self.h = None


def bead_forces(plan, R, F=None, U=None, want_energy=True):
    """F = -grad U per configuration: R (B, Q, 3) float64 -> F (B, Q, 3) float32, U (B,)."""
    torch = _torch()
    _beads(plan, R)
    B = R.shape[0]
    if F is None:
        F = torch.empty((B, plan.Q, 3), dtype=torch.float32, device=R.device)
    _dev_tensor(F, torch.float32, (B, plan.Q, 3))
    if U is None and want_energy:
        U = torch.empty(B, dtype=torch.float64, device=R.device)
    if U is not None:
        _dev_tensor(U, torch.float64, (B,))
    _check(lib().bead_forces(plan.h, _ptr(R), B, _ptr(F), _ptr(U), _ptr(plan.ws)), "bead_forces")
    return F, U


def bead_forces_static(plan, R, F=None, U=None, want_energy=True, status=None):
    """bead_forces in the library's static workspace (no plan workspace, no allocation in
    the library): outputs as bead_forces; status, if given, is a (1,) int32 CUDA tensor that
    receives the call's device status word."""
    torch = _torch()
    _beads(plan, R)
    B = R.shape[0]
    if F is None:
        F = torch.empty((B, plan.Q, 3), dtype=torch.float32, device=R.device)
    _dev_tensor(F, torch.float32, (B, plan.Q, 3))
    if U is None and want_energy:
        U = torch.empty(B, dtype=torch.float64, device=R.device)
    if U is not None:
        _dev_tensor(U, torch.float64, (B,))
    if status is not None:
        _dev_tensor(status, torch.int32, (1,))
    _check(lib().bead_forces_static(plan.h, _ptr(R), B, _ptr(F), _ptr(U), _ptr(status)),
           "bead_forces_static")
    return F, U


def bead_hvp(plan, R, V, HV=None):
    """H(R^b) V^b: R, V (B, Q, 3) float64 -> (B, Q, 3) float32."""
    torch = _torch()
    _beads(plan, R)
    _dev_tensor(V, torch.float64, R.shape)
    B = R.shape[0]
    if HV is None:
        HV = torch.empty((B, plan.Q, 3), dtype=torch.float32, device=R.device)
    _dev_tensor(HV, torch.float32, (B, plan.Q, 3))
    _check(lib().bead_hvp(plan.h, _ptr(R), _ptr(V), B, _ptr(HV), _ptr(plan.ws)), "bead_hvp")
    return HV


def veff_energy(plan, R):
    """(V_eff, U(R^1), spring energy) as a (3,) float64 CUDA tensor."""
    torch = _torch()
    _beads(plan, R)
    out = torch.empty(3, dtype=torch.float64, device=R.device)
    p = out.data_ptr()
    _check(lib().veff_energy(plan.h, _ptr(R), R.shape[0], C.c_void_p(p), C.c_void_p(p + 8),
                             C.c_void_p(p + 16), _ptr(plan.ws)), "veff_energy")
    return out


def veff_grad(plan, R, mode=0, fd_h=1e-4, G=None, veff=None):
    """(G, V_eff): G (N, Q, 3) float64 = grad V_eff; mode 0 exact HVP, 1 finite differences
    (displaced configurations re-binned), 2 finite differences on the binning of R."""
    torch = _torch()
    _beads(plan, R)
    if G is None:
        G = torch.empty_like(R)
    if veff is None:
        veff = torch.empty(1, dtype=torch.float64, device=R.device)
    _dev_tensor(G, torch.float64, R.shape)
    _dev_tensor(veff, torch.float64, (1,))
    _check(lib().veff_grad(plan.h, _ptr(R), R.shape[0], _ptr(G), _ptr(veff), int(mode),
                           float(fd_h), _ptr(plan.ws)), "veff_grad")
    return G, veff


class Bias:
    """Metadynamics bias on the end-to-end variable of eq. (8) for paths of `plan`."""

    def __init__(self, plan, groupA, groupB, sigma, height, bias_factor=0.0, kT=0.0,
                 stride=1, max_gaussians=4096):
        self.plan = plan
        a = np.ascontiguousarray(groupA, np.int32)
        b = np.ascontiguousarray(groupB, np.int32)
        d = _BiasDesc(len(a), len(b), a.ctypes.data, b.ctypes.data, float(sigma),
                      float(height), float(bias_factor), float(kT), int(stride),
                      int(max_gaussians))
        h = C.c_void_p()
        _check(lib().mop_bias_create(plan.h, C.byref(d), C.byref(h)), "mop_bias_create")
        self.h = h
        self.capacity = int(max_gaussians)

    def apply(self, R, G=None, deposit=False):
        """Adds grad V_bias to G (if given); returns a CUDA tensor {V_bias, S}."""
        torch = _torch()
        _beads(self.plan, R)
        if G is not None:
            _dev_tensor(G, torch.float64, R.shape)
        out = torch.empty(2, dtype=torch.float64, device=R.device)
        _check(lib().mop_bias_apply(self.h, _ptr(R), R.shape[0], _ptr(G) if G is not None else None,
                                    _ptr(out), int(bool(deposit)), _ptr(self.plan.ws)),
               "mop_bias_apply")
        return out

    def reset(self):
        _check(lib().mop_bias_reset(self.h), "mop_bias_reset")

    def history(self):
        """(centres, heights) of the deposited Gaussians (numpy)."""
        n = C.c_int32()
        c = np.zeros(self.capacity)
        w = np.zeros(self.capacity)
        _check(lib().mop_bias_history(self.h, C.byref(n), c.ctypes.data, w.ctypes.data,
                                      self.capacity), "mop_bias_history")
        m = min(int(n.value), self.capacity)
        return c[:m].copy(), w[:m].copy()

    def __del__(self):
        if getattr(self, "h", None) and _lib is not None:
            _lib.mop_bias_destroy(self.h)
            self.h = None


def pmd_step(plan, R, V, G, tau, nsteps=1, gamma=0.0, kT=0.0, seed=0, step0=0,
             energies=None, bias=None):
    """nsteps B A O A B steps of the path (R, V) in place; G must hold the gradient of the
    total potential at R on entry and holds that of the final R on exit.  Returns energies
    (nsteps, 4) float64 {V_eff, kinetic, V_bias, S} after each step (a CUDA tensor)."""
    torch = _torch()
    _beads(plan, R)
    for t in (V, G):
        _dev_tensor(t, torch.float64, R.shape)
    if energies is None:
        energies = torch.empty((int(nsteps), 4), dtype=torch.float64, device=R.device)
    _dev_tensor(energies, torch.float64, (int(nsteps), 4))
    prm = _PmdParams(float(tau), float(gamma), float(kT), int(seed) & (2 ** 64 - 1))
    _check(lib().pmd_step(plan.h, bias.h if bias is not None else None, _ptr(R), _ptr(V),
                          _ptr(G), R.shape[0], C.byref(prm), int(step0), int(nsteps),
                          _ptr(energies), _ptr(plan.ws)), "pmd_step")
    return energies


def veff_grad_timed(plan, R, mode=0, fd_h=1e-4, G=None, veff=None):
    """veff_grad with HIP events between phases; returns (G, veff, {phase: ms})."""
    torch = _torch()
    _beads(plan, R)
    if G is None:
        G = torch.empty_like(R)
    if veff is None:
        veff = torch.empty(1, dtype=torch.float64, device=R.device)
    _dev_tensor(G, torch.float64, R.shape)
    _dev_tensor(veff, torch.float64, (1,))
    ms = (C.c_float * len(PHASES))()
    _check(lib().veff_grad_timed(plan.h, _ptr(R), R.shape[0], _ptr(G), _ptr(veff), int(mode),
                                 float(fd_h), _ptr(plan.ws), ms), "veff_grad_timed")
    return G, veff, dict(zip(PHASES, [float(x) for x in ms]))


class Batch:
    """P independent paths of their own plans, evaluated in one launch per phase.
    R is one flat float64 CUDA tensor holding the paths back to back."""

    def __init__(self, plans, N):
        torch = _torch()
        self.plans = list(plans)
        self.N = [int(n) for n in N]
        self.P = len(self.plans)
        arr = (C.c_void_p * self.P)(*[p.h.value for p in self.plans])
        narr = (C.c_int32 * self.P)(*self.N)
        h = C.c_void_p()
        _check(lib().mop_batch_create(self.P, arr, narr, C.byref(h)), "mop_batch_create")
        self.h = h
        n = C.c_size_t()
        _check(lib().mop_batch_workspace_size(h, C.byref(n)), "mop_batch_workspace_size")
        dev = self.plans[0].ws.device
        self.ws = torch.zeros(int(n.value), dtype=torch.uint8, device=dev)
        self.sizes = [n_ * p.Q * 3 for n_, p in zip(self.N, self.plans)]
        self.offsets = np.concatenate([[0], np.cumsum(self.sizes)]).astype(np.int64)

    def pack(self, paths):
        torch = _torch()
        return torch.cat([p.reshape(-1) for p in paths]).contiguous()

    def unpack(self, flat):
        return [flat[self.offsets[k]:self.offsets[k + 1]].view(self.N[k], self.plans[k].Q, 3)
                for k in range(self.P)]

    def veff_grad(self, Rflat, mode=0, fd_h=1e-4, G=None, veff=None):
        torch = _torch()
        _dev_tensor(Rflat, torch.float64, (int(self.offsets[-1]),))
        if G is None:
            G = torch.empty_like(Rflat)
        if veff is None:
            veff = torch.empty(self.P, dtype=torch.float64, device=Rflat.device)
        _dev_tensor(G, torch.float64, Rflat.shape)
        _dev_tensor(veff, torch.float64, (self.P,))
        _check(lib().mop_batch_veff_grad(self.h, _ptr(Rflat), _ptr(G), _ptr(veff), int(mode),
                                         float(fd_h), _ptr(self.ws)), "mop_batch_veff_grad")
        return G, veff

    def status(self):
        s = C.c_int32()
        _check(lib().mop_status(self.plans[0].h, _ptr(self.ws), C.byref(s)), "mop_status")
        return int(s.value)

    def __del__(self):
        if getattr(self, "h", None) and _lib is not None:
            _lib.mop_batch_destroy(self.h)
            self.h = None


def _autograd_function():
    torch = _torch()

    class VeffFn(torch.autograd.Function):
        """V_eff(R) with backward = veff_grad (exact Hessian-vector products).
        forward runs veff_grad once and keeps G for the backward pass."""

        @staticmethod
        def forward(ctx, R, plan, mode=0, fd_h=1e-4):
            G, v = veff_grad(plan, R.detach().contiguous(), mode, fd_h)
            ctx.save_for_backward(G)
            return v[0].clone()

        @staticmethod
        def backward(ctx, g):
            (G,) = ctx.saved_tensors
            return g * G, None, None, None

    return VeffFn


class _Lazy:
    def __init__(self):
        self._fn = None

    def __getattr__(self, name):
        if self._fn is None:
            self._fn = _autograd_function()
        return getattr(self._fn, name)


VeffFn = _Lazy()
