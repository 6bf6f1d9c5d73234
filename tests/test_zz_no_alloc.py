"""bead_forces_static (the entry point that allocates nothing: its workspace is a static
device array of the library) against bead_forces on the same plans, through the C ABI:
two calls in a row, the second on a smaller system with fewer beads, so that what the
first call left in the shared array cannot leak into the second."""
import ctypes as C

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu


def _call_static(mop, plan, Rt):
    import torch
    B, Q = Rt.shape[0], plan.Q
    F = torch.full((B, Q, 3), float("nan"), dtype=torch.float32, device=Rt.device)
    U = torch.full((B,), float("nan"), dtype=torch.float64, device=Rt.device)
    st = torch.full((1,), -1, dtype=torch.int32, device=Rt.device)
    rc = mop.lib().bead_forces_static(plan.h, C.c_void_p(Rt.data_ptr()), B, C.c_void_p(F.data_ptr()),
                                      C.c_void_p(U.data_ptr()), C.c_void_p(st.data_ptr()))
    assert rc == 0, mop.lib().mop_strerror(rc)
    torch.cuda.synchronize()
    return F.cpu().numpy(), U.cpu().numpy(), int(st.cpu()[0])


def test_static_workspace_matches_bead_forces():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2501_11962_amd as mop
    ctx = mop.Context()
    cases = [(W.water_box(3000, seed=201, rc=1.0), 4, 11), (W.cfg1(), 2, 12)]
    for s, B, seed in cases:
        print(f"[static] Q={s['Q']} B={B}", flush=True)
        R, _, _ = W.random_walk_path(s, B, seed, 0.005)
        plan = mop.Plan(mop.System(ctx, s), B)
        Rt = torch.from_numpy(R).cuda()
        Fs, Us, st = _call_static(mop, plan, Rt)
        Fr, Ur = (x.cpu().numpy() for x in mop.bead_forces(plan, Rt))
        assert plan.status() == 0 and st == 0
        # the same kernels on the same binning: equal bits
        assert np.array_equal(Fs, Fr), float(np.abs(Fs - Fr).max())
        assert np.array_equal(Us, Ur)
    # sizes beyond the static workspace are refused before anything is enqueued
    big = mop.Plan(mop.System(ctx, W.cfg2()), 64)
    assert big.ws_bytes > mop.MOP_STATIC_WORKSPACE_BYTES
    Rb = torch.zeros((2, 3000, 3), dtype=torch.float64, device="cuda")
    rc = mop.lib().bead_forces_static(big.h, C.c_void_p(Rb.data_ptr()), 2, C.c_void_p(Rb.data_ptr()),
                                      None, None)
    assert rc == -7
