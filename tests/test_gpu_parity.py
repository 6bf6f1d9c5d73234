"""GPU parity: the HIP library (through its C ABI) against the FP64 CPU oracle.

Tolerances, relative L2 per bead: forces 1e-5, Hessian-vector products 1e-4, gradient
1e-5; V_eff 1e-6 relative (FP32 pair forces enter V_eff through c*F); the FP64-only
stages (bonds, residuals, sums) 1e-10 when no FP32 pair term contributes.
"""
import math

import numpy as np
import pytest

import workloads as W
from parity_metrics import check
from oracle import path as OP
from oracle.potential import Model

pytestmark = pytest.mark.gpu

TOL_F, TOL_HV, TOL_G, TOL_V = 1e-5, 1e-4, 1e-5, 1e-6


@pytest.fixture(scope="module")
def mop():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2501_11962_amd as m
    m.lib()
    return m


@pytest.fixture(scope="module")
def ctx(mop):
    return mop.Context()


def rel(a, b):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def cuda(x):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x, np.float64)).cuda()


def oracle_model(s, cl_oracle):
    return cl_oracle.CellModel(s) if s["Q"] > 3000 else Model(s)


SMALL = {
    "tiny": lambda: W.tiny(),
    "cfg1": W.cfg1,
    "water300": lambda: W.water_box(300, seed=5, rc=0.6),
    "cfg2": W.cfg2,
    "water1002_cw03": lambda: W.water_box(1002, seed=9, rc=1.0),
}


def say(*a):
    print(*a, flush=True)


@pytest.mark.parametrize("name", list(SMALL))
def test_bead_forces_and_energy(name, mop, ctx, cl_oracle):
    s = SMALL[name]()
    R, _, _ = W.random_walk_path(s, 3, 11, 0.01)
    say(f"[bead_forces] {name} Q={s['Q']} B=3")
    sysm = mop.System(ctx, s)
    plan = mop.Plan(sysm, 3)
    F, U = mop.bead_forces(plan, cuda(R))
    F, U = F.cpu().numpy(), U.cpu().numpy()
    assert plan.status() == 0
    m = oracle_model(s, cl_oracle)
    for b in range(3):
        Fo = m.forces(R[b])
        e = rel(F[b], Fo)
        eu = abs(U[b] - m.energy(R[b])) / max(abs(m.energy(R[b])), 1.0)
        say(f"   bead {b}: force relL2 {e:.2e}  energy rel {eu:.2e}")
        assert e < TOL_F
        assert eu < TOL_F


@pytest.mark.parametrize("name", list(SMALL))
def test_bead_hvp(name, mop, ctx, cl_oracle):
    s = SMALL[name]()
    R, _, _ = W.random_walk_path(s, 2, 12, 0.01)
    V = np.random.default_rng(3).standard_normal(R.shape) * 1e-3
    say(f"[bead_hvp] {name}")
    plan = mop.Plan(mop.System(ctx, s), 2)
    HV = mop.bead_hvp(plan, cuda(R), cuda(V)).cpu().numpy()
    m = oracle_model(s, cl_oracle)
    for b in range(2):
        e = rel(HV[b], m.hvp(R[b], V[b]))
        say(f"   bead {b}: hvp relL2 {e:.2e}")
        assert e < TOL_HV


@pytest.mark.parametrize("name,N", [("tiny", 5), ("cfg1", 32), ("water300", 6), ("cfg2", 8)])
def test_veff_energy_and_grad(name, N, mop, ctx, cl_oracle):
    s = SMALL[name]()
    sigma = 0.005 if name == "cfg1" else None
    R, _, _ = W.random_walk_path(s, N, 21, sigma)
    say(f"[veff] {name} N={N}")
    plan = mop.Plan(mop.System(ctx, s), N)
    Rt = cuda(R)
    ve = mop.veff_energy(plan, Rt).cpu().numpy()
    G, v = mop.veff_grad(plan, Rt)
    G, v = G.cpu().numpy(), float(v.cpu().numpy()[0])
    assert np.isfinite(G).all()
    assert plan.status() == 0
    m = oracle_model(s, cl_oracle)
    Go, vo = OP.veff_grad(m, R)
    vo2, u1o, eso = OP.veff(m, R)
    say(f"   V_eff gpu {v:.10e} oracle {vo:.10e} rel {abs(v - vo) / abs(vo):.2e}")
    assert abs(v - vo) < TOL_V * abs(vo)
    assert abs(ve[0] - vo) < TOL_V * abs(vo)
    assert abs(ve[1] - u1o) < TOL_F * max(abs(u1o), 1.0)
    assert abs(ve[2] - eso) < TOL_V * abs(eso)
    errs = [rel(G[n], Go[n]) for n in range(N)]
    say(f"   G relL2 per bead: max {max(errs):.2e} mean {np.mean(errs):.2e}")
    assert max(errs) < TOL_G


def test_fp64_stages_without_pair_terms(mop, ctx):
    """Charges and LJ switched off: only FP64 bonds, residuals and sums remain."""
    s = W.water_box(300, seed=5, rc=0.6)
    s = dict(s, charge=np.zeros(s["Q"]), epsilon=np.zeros(2))
    N = 6
    R, _, _ = W.random_walk_path(s, N, 4)
    plan = mop.Plan(mop.System(ctx, s), N)
    G, v = mop.veff_grad(plan, cuda(R))
    m = Model(s)
    Go, vo = OP.veff_grad(m, R)
    assert abs(float(v.cpu()[0]) - vo) < 1e-10 * abs(vo)
    assert rel(G.cpu().numpy(), Go) < 1e-10


def test_single_bead_and_single_atom(mop, ctx):
    s = W.cfg1()
    R = s["x"][None]
    plan = mop.Plan(mop.System(ctx, s), 4)
    G, v = mop.veff_grad(plan, cuda(R))
    m = Model(s)
    assert rel(G.cpu().numpy()[0], -m.forces(R[0])) < TOL_F
    assert abs(float(v.cpu()[0]) - m.energy(R[0])) < TOL_F * abs(m.energy(R[0]))
    # one atom: no pairs at all
    one = dict(Q=1, box=np.array([2.0, 2.0, 2.0]), x=np.array([[0.3, 0.4, 0.5]]),
               mass=np.array([16.0]), charge=np.array([0.5]), type=np.array([0]),
               sigma=np.array([0.3]), epsilon=np.array([0.5]), bonds=np.zeros((0, 2)),
               bond_r0=np.zeros(0), bond_k=np.zeros(0), mol=np.array([0]),
               molpos=np.array([0]), rc=0.9, eps_rf=78.0, eps_r=1.0, dt=0.001, nu=250.0, kT=2.5)
    R1, _, _ = W.random_walk_path(one, 3, 1, 0.01)
    p1 = mop.Plan(mop.System(ctx, one), 3)
    G1, v1 = mop.veff_grad(p1, cuda(R1))
    Go, vo = OP.veff_grad(Model(one), R1)
    assert rel(G1.cpu().numpy(), Go) < 1e-12
    assert abs(float(v1.cpu()[0]) - vo) < 1e-12 * abs(vo)


@pytest.mark.parametrize("pme", [False, True])
def test_plan_capacity_above_the_path_length(pme, mop, ctx):
    """A plan made for more beads than the path gives the same gradient as one made for
    exactly its beads (bit for bit with reaction field; PME transforms run over the plan's
    whole bead capacity, so there the batch size may change rounding); a path longer than
    the plan is refused with MOP_ESIZE (-7)."""
    s = W.water_box(1002, seed=9, rc=1.0)
    if pme:
        s = W.with_pme(s)
    R, _, _ = W.random_walk_path(s, 5, 43)
    sysm = mop.System(ctx, s)
    G5, v5 = (x.cpu().numpy() for x in mop.veff_grad(mop.Plan(sysm, 5), cuda(R)))
    big = mop.Plan(sysm, 9)
    G9, v9 = (x.cpu().numpy() for x in mop.veff_grad(big, cuda(R)))
    assert big.status() == 0
    if pme:
        assert rel(G9, G5) < 1e-12 and abs(v9[0] - v5[0]) < 1e-12 * abs(v5[0])
    else:
        assert np.array_equal(G9, G5) and np.array_equal(v9, v5)
    R12, _, _ = W.random_walk_path(s, 12, 44)
    with pytest.raises(mop.MopError) as e:
        mop.veff_grad(big, cuda(R12))
    assert e.value.code == -7


def test_binding_checks_shapes_before_any_launch(mop, ctx):
    """The C calls take only a bead count and read B * Q * 3 values, so the binding refuses
    tensors whose shape does not match the plan before anything reaches the device."""
    import torch
    s = W.cfg1()
    R, _, _ = W.random_walk_path(s, 3, 2, 0.005)
    plan = mop.Plan(mop.System(ctx, s), 3)
    Rt = cuda(R)
    bad = [cuda(R[:, :-1]), cuda(R[..., :2]), cuda(R[0]), cuda(R.reshape(3, -1))]
    for B in bad:
        for call in (lambda x: mop.veff_grad(plan, x), lambda x: mop.veff_energy(plan, x),
                     lambda x: mop.bead_forces(plan, x), lambda x: mop.bead_hvp(plan, x, x)):
            with pytest.raises(ValueError):
                call(B)
    with pytest.raises(ValueError):
        mop.veff_grad(plan, Rt, G=torch.empty((2, s["Q"], 3), dtype=torch.float64, device="cuda"))
    with pytest.raises(TypeError):
        mop.bead_forces(plan, Rt, F=torch.empty((3, s["Q"], 3), dtype=torch.float64, device="cuda"))
    bt = mop.Batch([plan], [3])
    with pytest.raises(ValueError):
        bt.veff_grad(Rt.reshape(-1)[:-3].contiguous())
    G, v = mop.veff_grad(plan, Rt)          # the right shapes still work
    assert plan.status() == 0 and torch.isfinite(G).all()


def test_unwrapped_coordinates(mop, ctx):
    s = W.cfg2()
    R, _, _ = W.random_walk_path(s, 4, 5)
    Rw = R + np.array([3.0, -2.0, 7.0]) * s["box"]
    Rw[2] = np.mod(Rw[2], s["box"])
    plan = mop.Plan(mop.System(ctx, s), 4)
    G1, v1 = mop.veff_grad(plan, cuda(R))
    G2, v2 = mop.veff_grad(plan, cuda(Rw))
    m = Model(s)
    Go, vo = OP.veff_grad(m, R)
    assert rel(G2.cpu().numpy(), Go) < TOL_G
    assert abs(float(v2.cpu()[0]) - vo) < TOL_V * abs(vo)


@pytest.mark.parametrize("cw,zb,waves", [(0.35, 0.05, 1), (0.8, 0.3, 2), (0.5, 0.1, 8)])
def test_plan_options_give_the_same_result(cw, zb, waves, mop, ctx):
    s = W.water_box(3 * 900, seed=2, rc=0.9)
    R, _, _ = W.random_walk_path(s, 3, 6)
    plan = mop.Plan(mop.System(ctx, s), 3, col_width=cw, zbin=zb, waves=waves)
    say(f"[options] cw={cw} zbin={zb} waves={waves} info={plan.info()}")
    G, v = mop.veff_grad(plan, cuda(R))
    Go, vo = OP.veff_grad(Model(s), R)
    assert rel(G.cpu().numpy(), Go) < TOL_G


def test_fd_mode_matches_oracle_fd(mop, ctx):
    s = W.cfg1()
    N, h = 5, 1e-3
    R, _, _ = W.random_walk_path(s, N, 8, 0.005)
    plan = mop.Plan(mop.System(ctx, s), N)
    Gfd, _ = mop.veff_grad(plan, cuda(R), mode=1, fd_h=h)
    m = Model(s)
    Gofd = OP.veff_grad_fd(m, R, h)
    Go, _ = OP.veff_grad(m, R)
    e_fd = rel(Gfd.cpu().numpy(), Gofd)
    say(f"[fd] gpu-FD vs oracle-FD relL2 {e_fd:.2e}; oracle FD vs exact {rel(Gofd, Go):.2e}")
    assert e_fd < 1e-4


@pytest.mark.parametrize("name,N", [("cfg1", 5), ("water300", 5)])
def test_shared_bin_fd_matches_oracle_fd(name, N, mop, ctx):
    """veff_grad mode 2 (finite differences on the binning of R) against the oracle's FD
    gradient and against mode 1 (re-binned), at fd_h = the neighbour search margin."""
    s = SMALL[name]()
    h = 1e-4
    R, _, _ = W.random_walk_path(s, N, 8, 0.005 if name == "cfg1" else None)
    plan = mop.Plan(mop.System(ctx, s), N)
    G2, v2 = mop.veff_grad(plan, cuda(R), mode=2, fd_h=h)
    G1, v1 = mop.veff_grad(plan, cuda(R), mode=1, fd_h=h)
    assert plan.status() == 0
    Gofd = OP.veff_grad_fd(Model(s), R, h)
    e2, e12 = rel(G2.cpu().numpy(), Gofd), rel(G2.cpu().numpy(), G1.cpu().numpy())
    say(f"[fd shared-bin] {name}: vs oracle FD relL2 {e2:.2e}; vs re-binned FD {e12:.2e}")
    assert e2 < 1e-4 and e12 < 1e-4
    assert float(v1[0]) == float(v2[0])


def test_batch_matches_single_paths(mop, ctx):
    specs = [(1002, 7, 31), (1503, 12, 32), (2001, 5, 33)]
    plans, paths, refs = [], [], []
    for Q, N, seed in specs:
        s = W.water_box(Q, seed, rc=1.0 if Q > 1500 else 0.9)
        R, _, _ = W.random_walk_path(s, N, seed + 100)
        pl = mop.Plan(mop.System(ctx, s), N)
        plans.append(pl)
        paths.append(cuda(R))
        refs.append(OP.veff_grad(Model(s), R))
    bt = mop.Batch(plans, [sp[1] for sp in specs])
    Gflat, v = bt.veff_grad(bt.pack(paths))
    assert bt.status() == 0
    for k, (G, (Go, vo)) in enumerate(zip(bt.unpack(Gflat), refs)):
        e = rel(G.cpu().numpy(), Go)
        say(f"[batch] path {k} G relL2 {e:.2e} V_eff rel {abs(float(v[k]) - vo) / abs(vo):.2e}")
        assert e < TOL_G
        assert abs(float(v[k]) - vo) < TOL_V * abs(vo)


def test_nonfinite_input_sets_status(mop, ctx):
    s = W.cfg1()
    R, _, _ = W.random_walk_path(s, 3, 1, 0.005)
    R[1, 5, 0] = np.nan
    plan = mop.Plan(mop.System(ctx, s), 3)
    plan.clear_status()
    mop.veff_grad(plan, cuda(R))
    assert plan.status() & mop.MOP_DEV_NONFINITE
    plan.clear_status()
    R2, _, _ = W.random_walk_path(s, 3, 1, 0.005)
    mop.veff_grad(plan, cuda(R2))
    assert plan.status() == 0


def test_overlap_sets_status(mop, ctx):
    """Two atoms of different molecules 0.005 nm apart set MOP_DEV_OVERLAP in every force
    pass (bead_forces, veff_grad) and the call still completes; the same plan on the
    unperturbed path then reports nothing."""
    s = W.cfg1()
    x = s["x"].copy()
    x[1] = x[0] + np.array([0.005, 0.0, 0.0])
    s2 = dict(s, x=x)
    R, _, _ = W.random_walk_path(s2, 3, 1, 0.0)
    plan = mop.Plan(mop.System(ctx, s2), 3)
    plan.clear_status()
    F, _ = mop.bead_forces(plan, cuda(R))
    st = plan.status()
    say(f"[overlap] bead_forces status {st}, forces finite: {bool(np.isfinite(F.cpu().numpy()).all())}")
    assert st & mop.MOP_DEV_OVERLAP
    plan.clear_status()
    mop.veff_grad(plan, cuda(R))
    assert plan.status() & mop.MOP_DEV_OVERLAP
    plan.clear_status()
    R0, _, _ = W.random_walk_path(s, 3, 1, 0.0)
    mop.veff_grad(plan, cuda(R0))
    mop.bead_forces(plan, cuda(R0))
    assert plan.status() == 0


def test_autograd_function(mop, ctx):
    import torch
    s = W.cfg1()
    R, _, _ = W.random_walk_path(s, 4, 2, 0.005)
    plan = mop.Plan(mop.System(ctx, s), 4)
    Rt = cuda(R).requires_grad_(True)
    v = mop.VeffFn.apply(Rt, plan)
    (2.5 * v).backward()
    G, v2 = mop.veff_grad(plan, cuda(R))
    # binning orders atoms deterministically, so the autograd call and the direct call
    # run the same kernels on the same slot order: equal bits (times the exact 2.5)
    assert torch.equal(Rt.grad, 2.5 * G)
    assert float(v.detach()) == float(v2[0])


def test_gpu_invariants(mop, ctx):
    """Properties that hold at any size, on GPU outputs alone."""
    s, R = W.make_config("cfg3", 2)
    plan = mop.Plan(mop.System(ctx, s), 2)
    F, _ = mop.bead_forces(plan, cuda(R))
    F = F.cpu().numpy().astype(np.float64)
    for b in range(2):
        assert np.linalg.norm(F[b].sum(0)) < 1e-4 * np.linalg.norm(F[b]) / math.sqrt(s["Q"]) * 100
    rng = np.random.default_rng(1)
    U_, V_ = rng.standard_normal(R.shape) * 1e-3, rng.standard_normal(R.shape) * 1e-3
    HU = mop.bead_hvp(plan, cuda(R), cuda(U_)).cpu().numpy().astype(np.float64)
    HV = mop.bead_hvp(plan, cuda(R), cuda(V_)).cpu().numpy().astype(np.float64)
    for b in range(2):
        a, c = np.sum(U_[b] * HV[b]), np.sum(V_[b] * HU[b])
        assert abs(a - c) < 1e-5 * np.linalg.norm(HU[b]) * np.linalg.norm(V_[b])


@pytest.mark.parametrize("cfg,N", [("cfg3", 3)])
def test_cfg3_parity(cfg, N, mop, ctx, cl_oracle):
    s, R = W.make_config(cfg, N)
    say(f"[{cfg}] Q={s['Q']} N={N}")
    plan = mop.Plan(mop.System(ctx, s), N)
    G, v = mop.veff_grad(plan, cuda(R))
    m = cl_oracle.CellModel(s)
    Go, vo = OP.veff_grad(m, R)
    G = G.cpu().numpy()
    for n in range(N):
        say("   " + check(G[n], Go[n], TOL_G, f"G bead {n + 1}"))
    say(f"   V_eff rel {abs(float(v[0]) - vo) / abs(vo):.2e}")
    assert abs(float(v[0]) - vo) < TOL_V * abs(vo)


@pytest.mark.parametrize("cfg", ["cfg2", "cfg3"])
def test_full_size_config_sampled(cfg, mop, ctx, cl_oracle):
    """The water box (3,000 atoms x 64 beads) and the mixed-chain box (23,000 x 128) at
    their full sizes, in the launch configuration bench.py times.  G^n depends only on
    beads n-1, n and n+1, so beads 1, N and three interior beads are checked through the
    2- and 3-bead sub-paths around them; V_eff is checked whole."""
    s, R = W.make_config(cfg)
    N = R.shape[0]
    plan = mop.Plan(mop.System(ctx, s), N)
    G, v = mop.veff_grad(plan, cuda(R))
    assert plan.status() == 0
    G = G.cpu().numpy()
    m = cl_oracle.CellModel(s)
    say(f"[{cfg}] Q={s['Q']} N={N}")
    say("   " + check(G[0], OP.veff_grad(m, np.ascontiguousarray(R[0:2]))[0][0], TOL_G, "G bead 1"))
    say("   " + check(G[N - 1], OP.veff_grad(m, np.ascontiguousarray(R[N - 2:N]))[0][1], TOL_G,
                      f"G bead {N}"))
    for n in np.random.default_rng(6).choice(np.arange(1, N - 1), 3, replace=False):
        say("   " + check(G[n], OP.veff_grad(m, np.ascontiguousarray(R[n - 1:n + 2]))[0][1], TOL_G,
                          f"G bead {n + 1}"))
    vo = OP.veff(m, R)[0]
    say(f"   V_eff rel {abs(float(v[0]) - vo) / abs(vo):.2e}")
    assert abs(float(v[0]) - vo) < TOL_V * abs(vo)


@pytest.mark.parametrize("name,N", [("cfg1", 4), ("cfg2", 4)])
def test_newton3_mode(name, N, mop, ctx):
    """Newton's-third-law variant (atomics) gives the same gradient."""
    s = SMALL[name]()
    R, _, _ = W.random_walk_path(s, N, 17, 0.005 if name == "cfg1" else None)
    plan = mop.Plan(mop.System(ctx, s), N, newton3=True)
    G, v = mop.veff_grad(plan, cuda(R))
    Go, vo = OP.veff_grad(Model(s), R)
    G = G.cpu().numpy()
    errs = [rel(G[n], Go[n]) for n in range(N)]
    say(f"[newton3] {name} G relL2 max {max(errs):.2e}")
    assert max(errs) < TOL_G
    assert abs(float(v[0]) - vo) < TOL_V * abs(vo)
    # run to run: summation order differs, well below the tolerance
    G2, _ = mop.veff_grad(plan, cuda(R))
    assert rel(G2.cpu().numpy(), G) < 1e-6


@pytest.mark.parametrize("persistent", [False, True])
def test_graph_replay_matches_eager(persistent, mop, ctx):
    """The whole veff_grad call captured once and replayed; each replay checked against
    an eager call, with eager work and synchronisation between replays.  Persistent plans
    put the reset of their work queues into the graph as kernels."""
    import torch
    s = W.cfg2()
    N = 6
    R, _, _ = W.random_walk_path(s, N, 23)
    plan = mop.Plan(mop.System(ctx, s), N, persistent=persistent)
    Rt = cuda(R)
    G = torch.empty_like(Rt)
    v = torch.empty(1, dtype=torch.float64, device=Rt.device)
    mop.veff_grad(plan, Rt, 0, 0.0, G, v)  # warm-up outside capture
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    cs = torch.cuda.Stream()
    cs.wait_stream(torch.cuda.current_stream())
    with torch.cuda.graph(g, stream=cs):
        ctx.set_stream()
        mop.veff_grad(plan, Rt, 0, 0.0, G, v)
    ctx.set_stream()
    torch.cuda.synchronize()
    Go, vo = OP.veff_grad(Model(s), R)
    Ge, ve = mop.veff_grad(plan, Rt)  # eager reference for bit-level comparison
    Ge, ve = Ge.cpu().numpy(), float(ve[0])
    for k in range(4):
        # eager work on the same workspace between replays (different input)
        Rk = Rt + 1e-3 * (k + 1)
        mop.veff_grad(plan, Rk)
        torch.cuda.synchronize()
        G.zero_()
        g.replay()
        torch.cuda.synchronize()
        e = rel(G.cpu().numpy(), Go)
        say(f"[graph] replay {k}: G relL2 {e:.2e}, V_eff rel {abs(float(v[0]) - vo) / abs(vo):.2e}")
        assert e < TOL_G
        assert abs(float(v[0]) - vo) < TOL_V * abs(vo)
        # binning orders atoms deterministically: replays equal the eager call exactly
        assert np.array_equal(G.cpu().numpy(), Ge) and float(v[0]) == ve
    assert plan.status() == 0


def test_repeated_calls_bit_identical(mop, ctx):
    """Every call orders the atoms of a bin by index, so the pair sums, and the gradient,
    do not depend on scheduling: repeated calls give identical bits (also for
    bead_forces and bead_hvp)."""
    s = W.water_box(1002, seed=9, rc=1.0)
    N = 4
    R, _, _ = W.random_walk_path(s, N, 29)
    plan = mop.Plan(mop.System(ctx, s), N)
    Rt = cuda(R)
    G0, v0 = (x.cpu().numpy() for x in mop.veff_grad(plan, Rt))
    F0 = mop.bead_forces(plan, Rt)[0].cpu().numpy()
    Vt = cuda(np.random.default_rng(3).normal(0.0, 1e-3, R.shape))
    H0 = mop.bead_hvp(plan, Rt, Vt).cpu().numpy()
    for _ in range(3):
        G1, v1 = (x.cpu().numpy() for x in mop.veff_grad(plan, Rt))
        assert np.array_equal(G0, G1) and np.array_equal(v0, v1)
        assert np.array_equal(F0, mop.bead_forces(plan, Rt)[0].cpu().numpy())
        assert np.array_equal(H0, mop.bead_hvp(plan, Rt, Vt).cpu().numpy())


@pytest.mark.parametrize("name,N", [("cfg2", 5), ("water300", 5)])
def test_analytic_beats_fd_accuracy(name, N, mop, ctx, cl_oracle):
    """Equal-accuracy comparison: the exact HVP path against the FD-HVP path of eq. (5)
    over a sweep of displacement lengths h; both measured against the FP64 exact G."""
    s = SMALL[name]()
    R, _, _ = W.random_walk_path(s, N, 41)
    plan = mop.Plan(mop.System(ctx, s), N)
    Go, _ = OP.veff_grad(oracle_model(s, cl_oracle), R)
    Rt = cuda(R)
    Ga, _ = mop.veff_grad(plan, Rt)
    ea = rel(Ga.cpu().numpy(), Go)
    efd = {}
    for h in (1e-5, 3e-5, 1e-4, 3e-4, 1e-3):
        Gf, _ = mop.veff_grad(plan, Rt, mode=1, fd_h=h)
        efd[h] = rel(Gf.cpu().numpy(), Go)
    say(f"[accuracy] {name}: analytic relL2 {ea:.2e}; FD " +
        ", ".join(f"h={h:g}: {e:.2e}" for h, e in efd.items()))
    assert ea < TOL_G
    assert ea < min(efd.values())


def test_cfg4_full_size_sampled(mop, ctx, cl_oracle):
    """The benchmark workload (150,000 atoms x 16 beads) in the launch configuration
    bench.py times: V_eff and the gradient of beads 1, 2 and 16 against the FP64 cell-list
    oracle; forces of bead 1 through bead_forces."""
    from oracle import path as OPth
    s, R = W.make_config("cfg4")
    N, Q = R.shape[0], s["Q"]
    plan = mop.Plan(mop.System(ctx, s), N)
    Rt = cuda(R)
    G, v = mop.veff_grad(plan, Rt)
    G = G.cpu().numpy()
    v = float(v[0])
    assert plan.status() == 0
    m = cl_oracle.CellModel(s)
    c, K = OPth.coefficients(m)
    F = {n: m.forces(R[n]) for n in range(N - 1)}
    d = {n: OPth.min_image(R[n + 1] - R[n], m.box) - c[:, None] * F[n] for n in range(N - 1)}
    vo = m.energy(R[0]) + sum(float(np.sum(0.5 * K[:, None] * d[n] ** 2)) for n in range(N - 1))
    Go0 = -F[0] - K[:, None] * d[0] + 0.5 * m.hvp(R[0], d[0])
    Go1 = K[:, None] * d[0] - K[:, None] * d[1] + 0.5 * m.hvp(R[1], d[1])
    GoN = K[:, None] * d[N - 2]
    for n, Gon in ((0, Go0), (1, Go1), (N - 1, GoN)):
        say("[cfg4] " + check(G[n], Gon, TOL_G, f"G bead {n + 1}"))
    say(f"[cfg4] V_eff rel {abs(v - vo) / abs(vo):.2e}")
    assert abs(v - vo) < TOL_V * abs(vo)
    Fg, _ = mop.bead_forces(plan, Rt[:1].contiguous(), want_energy=False)
    say("[cfg4] " + check(Fg.cpu().numpy()[0], F[0], TOL_F, "bead_forces"))
    HV = mop.bead_hvp(plan, Rt[:1].contiguous(), cuda(d[0][None])).cpu().numpy()[0]
    say("[cfg4] " + check(HV, m.hvp(R[0], d[0]), TOL_HV, "bead_hvp (v = d^1)"))


def test_cfg5_full_batch_sampled(mop, ctx, cl_oracle):
    """The uneven batch at its benchmark size (24 water paths, Q 1.4e3..1.7e4, N 33..122,
    1.2e7 atom*beads) in one call.  G^n depends only on beads n-1, n and n+1, so the
    gradient of bead 1, of one interior bead and of bead N of every path equals that of
    the 2- or 3-bead sub-path around it, which the FP64 cell-list oracle evaluates; V_eff
    is checked whole on the paths of least work."""
    from oracle import path as OPth
    batch = W.batch_paths()
    specs = [(s_, R.shape[0], seed) for s_, R, seed in batch]
    rng = np.random.default_rng(5)
    plans, paths, Rs = [], [], []
    for s_, R, _ in batch:
        N = R.shape[0]
        Rs.append(R)
        plans.append(mop.Plan(mop.System(ctx, s_), N))
        paths.append(cuda(R))
    bt = mop.Batch(plans, [n for _, n, _ in specs])
    Gflat, v = bt.veff_grad(bt.pack(paths))
    assert bt.status() == 0
    Gs = [g.cpu().numpy() for g in bt.unpack(Gflat)]
    v = v.cpu().numpy()
    worst = 0.0
    for k, ((s_, N, _), R) in enumerate(zip(specs, Rs)):
        m = cl_oracle.CellModel(s_)
        n = int(rng.integers(1, N - 1))                      # interior bead (0-based)
        G1, _ = OPth.veff_grad(m, np.ascontiguousarray(R[0:2]))
        Gn, _ = OPth.veff_grad(m, np.ascontiguousarray(R[n - 1:n + 2]))
        GN, _ = OPth.veff_grad(m, np.ascontiguousarray(R[N - 2:N]))
        e = max(rel(Gs[k][0], G1[0]), rel(Gs[k][n], Gn[1]), rel(Gs[k][N - 1], GN[1]))
        worst = max(worst, e)
        assert e < TOL_G, (k, n, e)
    order = np.argsort([s_["Q"] * N for s_, N, _ in specs])[:6]
    for k in order:
        s_, N, _ = specs[k]
        vo = OPth.veff(cl_oracle.CellModel(s_), Rs[k])[0]
        assert abs(float(v[k]) - vo) < TOL_V * abs(vo), (k, float(v[k]), vo)
    say(f"[cfg5] {len(specs)} paths: worst G relL2 (beads 1, interior, N) {worst:.2e}")


@pytest.mark.parametrize("name", ["water1002_cw03", "cfg2"])
def test_neighbour_list_replay_is_exact(name, mop, ctx):
    """The Hessian pass replaying the force pass's neighbour lists gives bit-identical
    gradients to searching again (lists off), also when most clusters overflow a small
    list and fall back to the search."""
    s = SMALL[name]()
    N = 5
    R, _, _ = W.random_walk_path(s, N, 19)
    Rt = cuda(R)
    sysm = mop.System(ctx, s)
    out = {}
    for cap in (0, -1, 64):
        plan = mop.Plan(sysm, N, list_cap=cap)
        G, v = mop.veff_grad(plan, Rt)
        assert plan.status() == 0
        out[cap] = (G.cpu().numpy(), float(v[0]))
    say(f"[lists] {name}: max |dG| auto vs off {np.max(np.abs(out[0][0] - out[-1][0])):.1e}, "
        f"cap 64 vs off {np.max(np.abs(out[64][0] - out[-1][0])):.1e}")
    assert np.array_equal(out[0][0], out[-1][0])
    assert np.array_equal(out[64][0], out[-1][0])
    assert out[0][1] == out[-1][1] == out[64][1]


@pytest.mark.parametrize("name,waves,N", [("water1002_cw03", 4, 5), ("cfg2", 1, 5), ("cfg2", 8, 5),
                                          ("water30000", 4, 6)])
def test_persistent_plan_is_bit_identical(name, waves, N, mop, ctx):
    """MOP_PLAN_PERSISTENT launches the pair kernels as resident grids that take clusters
    from per-XCD work queues: every output (both gradient modes, finite differences on
    shared bins, bead forces, Hessian-vector products, batches) equals the flat launch's
    bit for bit, also on a second call (the queues start from zero every launch).  The
    30,000-atom path is large enough (over 16,384 clusters per pass) for the force pass to
    run as two launches, bead 1 with energies and the others without."""
    s = W.water_box(30000, seed=3, rc=1.0) if name == "water30000" else SMALL[name]()
    R, _, _ = W.random_walk_path(s, N, 29)
    Rt = cuda(R)
    Vt = cuda(np.random.default_rng(6).normal(0.0, 1e-3, R.shape))
    sysm = mop.System(ctx, s)
    out = []
    for persistent in (False, True):
        plan = mop.Plan(sysm, N, waves=waves, persistent=persistent)
        res = []
        for _ in range(2):
            G, v = mop.veff_grad(plan, Rt)
            G2, v2 = mop.veff_grad(plan, Rt, mode=2, fd_h=1e-4)
            F, U = mop.bead_forces(plan, Rt)
            H = mop.bead_hvp(plan, Rt, Vt)
            res.append([x.cpu().numpy() for x in (G, v, G2, v2, F, U, H)])
        assert plan.status() == 0
        for a, b in zip(*res):
            assert np.array_equal(a, b)
        # U(R^1) of veff_energy (the force pass of a path: bead 1 in the energy launch) and
        # of bead_forces (every bead with energies): same pair sums, bonds summed apart
        e = mop.veff_energy(plan, Rt).cpu().numpy()
        U0 = res[0][5][0]
        assert abs(e[1] - U0) <= 1e-12 * abs(U0), (e[1], U0)
        assert abs(e[0] - (e[1] + e[2])) <= 1e-12 * abs(e[0])
        assert float(res[0][1][0]) == e[0]
        bt = mop.Batch([plan, plan], [N, N - 2])
        Gb, vb = bt.veff_grad(bt.pack([Rt, Rt[:N - 2].contiguous()]))
        assert bt.status() == 0
        res[0] += [Gb.cpu().numpy(), vb.cpu().numpy()]
        out.append(res[0])
    for k, (a, b) in enumerate(zip(*out)):
        assert np.array_equal(a, b), k
    say(f"[persistent] {name} waves={waves}: {len(out[0])} outputs bit-identical")


def test_waves_per_workgroup_are_bit_identical(mop, ctx):
    """Each i-cluster's sums do not depend on how many waves share a workgroup: plans with
    1, 2, 4 and 8 waves per workgroup give bit-identical gradients and V_eff."""
    s = W.cfg2()
    N = 4
    R, _, _ = W.random_walk_path(s, N, 41)
    Rt = cuda(R)
    sysm = mop.System(ctx, s)
    out = []
    for waves in (1, 2, 4, 8):
        plan = mop.Plan(sysm, N, waves=waves)
        G, v = mop.veff_grad(plan, Rt)
        assert plan.status() == 0
        out.append((G.cpu().numpy(), float(v[0])))
    for G, v in out[1:]:
        assert np.array_equal(G, out[0][0]) and v == out[0][1]


def test_batch_with_degenerate_paths_matches_single_calls(mop, ctx):
    """A batch holding a 1-bead path (V_eff = U(R^1), G = -F^1), a 2-bead path and a
    30,000-atom path of 6 beads (enough clusters for the force pass to run as two
    launches, bead 1 of every path with energies, then the rest) gives every path the
    gradient and V_eff of its own single-path call, bit for bit."""
    systems = [W.water_box(30000, seed=3, rc=1.0), W.cfg2(), W.water_box(1002, seed=9, rc=1.0)]
    Ns = [6, 1, 2]
    plans, paths, single = [], [], []
    for k, (s_, N) in enumerate(zip(systems, Ns)):
        R, _, _ = W.random_walk_path(s_, N, 60 + k)
        pl = mop.Plan(mop.System(ctx, s_), N)
        Rt = cuda(R)
        G, v = mop.veff_grad(pl, Rt)
        assert pl.status() == 0
        single.append((G.cpu().numpy(), float(v[0])))
        plans.append(pl)
        paths.append(Rt)
    # the 1-bead path: V_eff is U(R^1) and G is -F^1
    F1, U1 = mop.bead_forces(plans[1], paths[1])
    assert abs(single[1][1] - float(U1[0])) <= 1e-12 * abs(float(U1[0]))
    assert rel(single[1][0][0], -F1.cpu().numpy()[0].astype(np.float64)) < 1e-6
    bt = mop.Batch(plans, Ns)
    Gflat, v = bt.veff_grad(bt.pack(paths))
    assert bt.status() == 0
    for k, G in enumerate(bt.unpack(Gflat)):
        assert np.array_equal(G.cpu().numpy(), single[k][0]), k
        assert float(v[k]) == single[k][1], k


@pytest.mark.parametrize("mode", [1, 2])
def test_graph_replay_of_fd_modes_matches_eager(mode, mop, ctx):
    """The finite-difference modes (re-binned and shared-bin) run without host
    synchronisation too: a captured call replays bit-identically to the eager call, with
    eager work on the same workspace between replays."""
    import torch
    s = W.cfg2()
    N = 5
    R, _, _ = W.random_walk_path(s, N, 43)
    plan = mop.Plan(mop.System(ctx, s), N)
    Rt = cuda(R)
    G = torch.empty_like(Rt)
    v = torch.empty(1, dtype=torch.float64, device=Rt.device)
    mop.veff_grad(plan, Rt, mode, 1e-4, G, v)
    torch.cuda.synchronize()
    Ge, ve = G.cpu().numpy().copy(), float(v[0])
    g = torch.cuda.CUDAGraph()
    cs = torch.cuda.Stream()
    cs.wait_stream(torch.cuda.current_stream())
    with torch.cuda.graph(g, stream=cs):
        ctx.set_stream()
        mop.veff_grad(plan, Rt, mode, 1e-4, G, v)
    ctx.set_stream()
    torch.cuda.synchronize()
    for k in range(3):
        mop.veff_grad(plan, Rt + 1e-3 * (k + 1), mode, 1e-4)
        torch.cuda.synchronize()
        G.zero_()
        g.replay()
        torch.cuda.synchronize()
        assert np.array_equal(G.cpu().numpy(), Ge) and float(v[0]) == ve, k
    assert plan.status() == 0


def test_graph_replay_of_bead_calls_matches_eager(mop, ctx):
    """bead_forces (with energies) and bead_hvp captured in one graph: every replay equals
    the eager calls bit for bit."""
    import torch
    s = W.cfg2()
    B = 3
    R, _, _ = W.random_walk_path(s, B, 47)
    plan = mop.Plan(mop.System(ctx, s), B)
    Rt = cuda(R)
    Vt = cuda(np.random.default_rng(8).normal(0.0, 1e-3, R.shape))
    F = torch.empty((B, s["Q"], 3), dtype=torch.float32, device=Rt.device)
    U = torch.empty(B, dtype=torch.float64, device=Rt.device)
    H = torch.empty((B, s["Q"], 3), dtype=torch.float32, device=Rt.device)
    mop.bead_forces(plan, Rt, F, U)
    mop.bead_hvp(plan, Rt, Vt, H)
    torch.cuda.synchronize()
    Fe, Ue, He = F.cpu().numpy().copy(), U.cpu().numpy().copy(), H.cpu().numpy().copy()
    g = torch.cuda.CUDAGraph()
    cs = torch.cuda.Stream()
    cs.wait_stream(torch.cuda.current_stream())
    with torch.cuda.graph(g, stream=cs):
        ctx.set_stream()
        mop.bead_forces(plan, Rt, F, U)
        mop.bead_hvp(plan, Rt, Vt, H)
    ctx.set_stream()
    torch.cuda.synchronize()
    for k in range(3):
        mop.bead_forces(plan, Rt + 1e-3 * (k + 1))
        torch.cuda.synchronize()
        F.zero_()
        H.zero_()
        g.replay()
        torch.cuda.synchronize()
        assert np.array_equal(F.cpu().numpy(), Fe) and np.array_equal(U.cpu().numpy(), Ue), k
        assert np.array_equal(H.cpu().numpy(), He), k
    assert plan.status() == 0
