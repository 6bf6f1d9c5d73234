"""Benchmark: veff_grad throughput (atom*beads/s) on one MI355X.

One step = one veff_grad call over one path (binning, pair forces of beads 1..N-1,
FP64 residuals and spring energy, pair Hessian-vector products, FP64 gradient assembly
and V_eff reduction), inputs already resident in HBM.  Default workload: the
membrane-shaped system, 150,000 atoms x 16 beads, cutoff 1.2 nm.

Prints ONE JSON line with the throughput, the roofline of the dominant kernel (the pair
Hessian-vector kernel, FP32 ALU-bound), the finite-difference comparison path, and the
FP64 CPU oracle timed on a bounded sample of the same workload.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--config cfg4]
                    [--no-cpu-baseline] [--no-fd] [--no-graph]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "veff_grad atom·beads/s, analytic HVP vs finite-diff HVP, 1 MI355X"
PEAK_FP32_TFLOPS = 157.3      # MI355X FP32 vector (published)
PEAK_HBM_GBS = 8000.0
# Algorithmic FLOPs per unique within-cutoff pair (FMA = 2, rsqrt = 1, others 1),
# counted term by term from the pair formulas, each pair once (Newton's third law: the
# partner's update is counted as well):
#   force  d 3, r^2 5, rsqrt 1, r^-2 r^-3 r^-6 r^-8 4, q_i q_j 1, C1 2, G6 2, g 6,
#          g d 3, two 3-vector updates 6                                        = 33
#   HVP    d 3, r^2 5, rsqrt 1, powers 4, q_i q_j 1, C1 2, G6 2, g 6, h6 2, r^-5 1,
#          h 7, dv 3, d.dv 5, h d.dv 1, g dv + (h d.dv) d 9, two updates 6      = 58
FLOP_FORCE_PAIR = 33
FLOP_HVP_PAIR = 58
# Ewald real space: the reaction-field terms of g (and h) replaced by erfc/exp terms
# (erfc as exp(-x^2) times a degree-8 polynomial in 1/(1 + x/2); exp and reciprocal 1 each):
# g 11 -> 38 flops, h 11 -> 16 flops.
FLOP_FORCE_PAIR_EWALD = 61
FLOP_HVP_PAIR_EWALD = 92
FD_SWEEP = (1e-5, 3e-5, 1e-4, 3e-4, 1e-3)   # FD displacement lengths h (nm)
PAIR_SRC = os.path.join(ROOT, "paper_2501_11962_amd", "csrc", "kernels_pair.hip")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def settle(fn, calls, seconds=0.3):
    """Untimed warm-up: at least `calls` calls of fn and at least `seconds` of wall time
    with the GPU busy.  After a pause (a capture, host work) the GPU clock takes tens of
    calls to climb back: in a kernel trace the first replays after a capture ran up to 15%
    slower than the settled ones."""
    import torch
    t0 = time.perf_counter()
    k = 0
    while k < calls or time.perf_counter() - t0 < seconds:
        fn()
        k += 1
        if k % 4 == 0:
            torch.cuda.synchronize()
    torch.cuda.synchronize()
    return k


def unique_pairs(system, X):
    """Unique non-excluded atom pairs closer than the cutoff (minimum image), counted
    with a periodic k-d tree; bonded 1-2/1-3 pairs are always within the cutoff here and
    are subtracted."""
    from scipy.spatial import cKDTree
    box = np.asarray(system["box"], np.float64)
    Y = X - box * np.floor(X / box)
    Y = np.minimum(Y, np.nextafter(box, 0))
    t = cKDTree(Y, boxsize=box)
    n = int(t.count_neighbors(t, system["rc"]))
    Q = system["Q"]
    within = (n - Q) // 2
    # excluded pairs: bond-graph distance 1 or 2
    nb = [[] for _ in range(Q)]
    for i, j in np.asarray(system["bonds"]).reshape(-1, 2):
        nb[i].append(int(j))
        nb[j].append(int(i))
    ex = set()
    for i in range(Q):
        for j in nb[i]:
            ex.add((min(i, j), max(i, j)))
            for k in nb[j]:
                if k != i:
                    ex.add((min(i, k), max(i, k)))
    return within - len(ex)


def profile_summary(name):
    """The machine-readable lines (`- key: value`) of a committed counter summary under
    profiles/, if it was taken on the current pair-kernel source; else None."""
    p = os.path.join(ROOT, "profiles", name)
    if not os.path.exists(p):
        return None
    kv = {}
    for line in open(p):
        if ":" in line and line.strip().startswith("- "):
            k, v = line.strip()[2:].split(":", 1)
            kv[k.strip()] = v.strip().strip("`")
    h = hashlib.sha256(open(PAIR_SRC, "rb").read()).hexdigest()
    return kv if kv.get("kernel_source_sha256") == h else None


def traffic_from_profiles(workload):
    """HBM bytes per launch of the force and Hessian pair kernels measured by rocprofv3
    counters (FETCH_SIZE and WRITE_SIZE, each scaled by what the counter reads for a plain
    copy of known size), from the committed summary, if it was taken on the current kernel
    source; else None for each."""
    kv = profile_summary(f"traffic_pair_{workload}.md") or {}
    out = {}
    for k in ("force", "hvp"):
        try:
            out[k] = int(float(kv[f"{k}_bytes_per_launch"]))
        except (KeyError, ValueError):
            out[k] = None
    return out


def cpu_description():
    """Model name, family / model / stepping numbers and core count of the host CPU."""
    info = {}
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if ":" in line:
                    k, v = line.split(":", 1)
                    info.setdefault(k.strip(), v.strip())
    except OSError:
        pass
    name = info.get("model name", "unknown")
    ids = ", ".join(f"{k} {info[k]}" for k in ("cpu family", "model", "stepping") if k in info)
    return f"{name} ({ids})" if ids else name


def executed_from_profiles(workload):
    """Executed FP32 FLOPs per launch of the Hessian and force pair kernels, counted by
    rocprofv3 (SQ_INSTS_VALU_FLOPS_FP32 counts each wave instruction once, so it is
    multiplied by the 64 lanes; masked lanes are included), and their VALU instructions
    per compute-unit cycle, from the committed summary if it matches the kernel source."""
    kv = profile_summary(f"valu_pair_{workload}.md")
    try:
        return None if kv is None else {k: float(v) for k, v in kv.items()
                                        if k.endswith(("_per_launch", "_per_cu_cycle"))}
    except ValueError:
        return None


def cpu_baseline(system, R, beads):
    """FP64 cell-list oracle (all host threads) on the first `beads` beads of the path."""
    from oracle import cl
    from oracle import path as OP
    m = cl.CellModel(system)
    sub = np.ascontiguousarray(R[:beads])
    t0 = time.perf_counter()
    Gsub, _ = OP.veff_grad(m, sub)
    dt = time.perf_counter() - t0
    # one thread on a two-bead sample (one force and one Hessian-vector pass)
    m1 = cl.CellModel(system, nthreads=1)
    t1 = time.perf_counter()
    OP.veff_grad(m1, np.ascontiguousarray(R[:2]))
    dt1 = time.perf_counter() - t1
    model = cpu_description()
    # beads 1 .. beads-1 of the sub-path carry the same gradient as in the whole path
    return dict(value=system["Q"] * beads / dt, unit="atom·beads/s", cores=cl.max_threads(),
                kind="oracle", cpu_model=model, host_cpus=os.cpu_count(),
                one_thread=dict(value=system["Q"] * 2 / dt1,
                                sample=f"veff_grad of the first 2 beads, {dt1:.1f} s wall"),
                sample=f"veff_grad of the first {beads} beads of the same path "
                       f"({beads - 1} force + {beads - 1} Hessian-vector passes over "
                       f"{system['Q']} atoms), {dt:.1f} s wall"), Gsub[:beads - 1]


def bench_batch(args, mop, ctx, log):
    """The uneven batch: 24 independent water paths (Q log-uniform in [1e3, 2e4], N
    uniform in [16, 128], tethered Brownian beads) in one launch per phase, captured once
    in a graph.  Aggregate
    atom*beads/s, and each path's gradient of beads 1-2 against the FP64 oracle (C cell
    list) on the first three beads."""
    import torch
    import workloads as W
    batch = W.batch_paths()
    specs = [(s_, R.shape[0], seed) for s_, R, seed in batch]
    plans, paths, Rs, popts = [], [], [], []
    tuned = not args.no_autotune
    if tuned:
        from paper_2501_11962_amd import autotune as A
        # a batch takes its launch shape (waves, persistent) from its first plan
        space = {k: v for k, v in A.SPACE.items() if k not in ("waves", "persistent")}
    for s_, R, seed in batch:
        N = R.shape[0]
        Rs.append(R)
        Rp = torch.from_numpy(R).cuda()
        o = A.autotune(ctx, s_, Rp, space=space, cache=args.tune_cache) if tuned else {}
        popts.append(o)
        plans.append(mop.Plan(mop.System(ctx, s_), N, **o))
        paths.append(Rp)
    bt = mop.Batch(plans, [n for _, n, _ in specs])
    Rf = bt.pack(paths)
    G = torch.empty_like(Rf)
    v = torch.empty(bt.P, dtype=torch.float64, device=Rf.device)
    for _ in range(args.warmup):
        bt.veff_grad(Rf, G=G, veff=v)
    torch.cuda.synchronize()
    if bt.status():
        raise SystemExit(f"batch device status {bt.status()}")
    settle(lambda: bt.veff_grad(Rf, G=G, veff=v), 1)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(args.steps):
        bt.veff_grad(Rf, G=G, veff=v)
    e1.record()
    torch.cuda.synchronize()
    ms_eager = e0.elapsed_time(e1) / args.steps
    ms_graph = None
    if not args.no_graph:
        g = torch.cuda.CUDAGraph()
        cs = torch.cuda.Stream()
        cs.wait_stream(torch.cuda.current_stream())
        Gref = G.clone()
        with torch.cuda.graph(g, stream=cs):
            ctx.set_stream()
            bt.veff_grad(Rf, G=G, veff=v)
        ctx.set_stream()
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        if torch.equal(G, Gref):
            settle(g.replay, args.warmup)
            e0.record()
            for _ in range(args.steps):
                g.replay()
            e1.record()
            torch.cuda.synchronize()
            ms_graph = e0.elapsed_time(e1) / args.steps
        else:
            log("[bench] batch graph replay differs from the eager call; graph timing skipped")
    ms = ms_graph if ms_graph is not None else ms_eager   # graph replay, as for the headline
    ms_default = None
    if tuned:
        # the same batch with default plans, for the autotuner's gain
        dplans = [mop.Plan(mop.System(ctx, s_), n) for s_, n, _ in specs]
        dbt = mop.Batch(dplans, [n for _, n, _ in specs])
        for _ in range(args.warmup):
            dbt.veff_grad(Rf, G=G, veff=v)
        torch.cuda.synchronize()
        e0.record()
        for _ in range(args.steps):
            dbt.veff_grad(Rf, G=G, veff=v)
        e1.record()
        torch.cuda.synchronize()
        ms_default = e0.elapsed_time(e1) / args.steps
        del dbt, dplans
        bt.veff_grad(Rf, G=G, veff=v)   # G of the tuned batch again, for the error check
        torch.cuda.synchronize()
    work = sum(s_["Q"] * n for s_, n, _ in specs)
    out = dict(workload=f"cfg5: {bt.P} water paths, Q {min(s_['Q'] for s_, _, _ in specs)}.."
                        f"{max(s_['Q'] for s_, _, _ in specs)}, N {min(n for _, n, _ in specs)}.."
                        f"{max(n for _, n, _ in specs)}, rc 1.0 nm",
               value=work / (ms * 1e-3), unit="atom·beads/s", ms_per_call=ms,
               ms_eager=ms_eager, ms_graph=ms_graph,
               graph=ms_graph is not None, atom_beads=work,
               plan_options=popts if tuned else "default",
               ms_eager_default_plans=ms_default)
    log(f"[bench] batch: {ms:.3f} ms/call, {out['value']:.3e} atom*beads/s")
    if not args.no_cpu_baseline:
        from oracle import cl
        from oracle import path as OP
        errs = []
        Gs = bt.unpack(G)
        for k, ((s_, N, _), R) in enumerate(zip(specs, Rs)):
            Go, _ = OP.veff_grad(cl.CellModel(s_), np.ascontiguousarray(R[:3]))
            Gg = Gs[k][:2].cpu().numpy()
            errs.append(float(np.linalg.norm(Gg - Go[:2]) / np.linalg.norm(Go[:2])))
        out["path_relL2_beads_1_2"] = dict(max=max(errs), median=float(np.median(errs)))
        log(f"[bench] batch per-path relL2 (beads 1-2): max {max(errs):.2e}")
    return out


def bench_pmd(args, mop, ctx, plan, system, Rt, ms_grad, log):
    """Path dynamics on the same workload: Langevin B A O A B steps (gamma = 250 / ps,
    300 K, time step 0.5 fs) with the metadynamics bias on the end-to-end variable of
    eq. (8), from the relaxed starting structure.  Groups: one bonded 50-atom chain
    (ligand-sized) and the atoms within 1.2 nm of its first atom (pocket-sized).  Reports
    ms per step, what the integrator and the bias add to one veff_grad call, and whether
    the energies stayed finite."""
    import torch
    X = np.asarray(system["x"])
    L = np.asarray(system["box"])
    bonds = np.asarray(system["bonds"]).reshape(-1, 2)
    a0 = int(bonds[0, 0])
    mol = np.asarray(system["mol"])
    d = X - X[a0]
    d -= L * np.rint(d / L)
    r2 = (d * d).sum(1)
    A = np.nonzero((mol == mol[a0]) & (r2 < 0.8 ** 2))[0]      # compact: < half the box
    B = np.setdiff1d(np.nonzero(r2 < 1.2 ** 2)[0], A)
    kT = 0.0083144626 * 300.0
    bias = mop.Bias(plan, A, B, 0.02, 1.0, 10.0, kT, stride=5, max_gaussians=1 << 16)
    R = Rt.clone()
    V = torch.zeros_like(R)
    G, _ = mop.veff_grad(plan, R)
    bias.apply(R, G)
    steps = max(args.steps // 2, 5)
    tau = 5e-4
    mop.pmd_step(plan, R, V, G, tau, 2, 250.0, kT, seed=7, step0=0, bias=bias)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    E = mop.pmd_step(plan, R, V, G, tau, steps, 250.0, kT, seed=7, step0=2, bias=bias)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    st = plan.status()
    Q, N = system["Q"], Rt.shape[0]
    out = dict(workload=f"Langevin path dynamics with the end-to-end bias: groups of {len(A)} "
                        f"and {len(B)} atoms, deposit every 5 steps, tau {tau * 1e3:g} fs",
               ms_per_step=ms, value=Q * N / (ms * 1e-3), unit="atom·beads/s",
               overhead_vs_veff_grad_ms=ms - ms_grad, steps=steps,
               gaussians=len(bias.history()[0]), device_status=st,
               energies_finite=bool(torch.isfinite(E).all()))
    log(f"[bench] pmd: {ms:.3f} ms/step (veff_grad {ms_grad:.3f}), status {st}")
    plan.clear_status()
    if not args.no_cpu_baseline:
        # CPU baseline: one biased Langevin step of the FP64 oracle (cell list, all host
        # threads) on the first two beads of the path
        from oracle import cl
        from oracle import mop_bias as MB
        from oracle import path as OP
        from oracle import pmd
        m = cl.CellModel(system)
        R2 = np.ascontiguousarray(Rt[:2].cpu().numpy())
        ob = MB.Bias(A, B, system["mass"], system["box"], 0.02, 1.0, 10.0, kT, stride=5)
        G2, _ = OP.veff_grad(m, R2)
        G2 = G2 + ob.apply(R2, 0)[2]
        t0 = time.perf_counter()
        pmd.baoab_step(m, R2, np.zeros_like(R2), G2, system["mass"], tau, 250.0, kT, 7, 1, ob)
        dt = time.perf_counter() - t0
        Qs = system["Q"]
        out["cpu_baseline"] = dict(value=Qs * 2 / dt, unit="atom·beads/s", cores=cl.max_threads(),
                                   kind="oracle",
                                   sample=f"one biased Langevin step of a 2-bead path "
                                          f"({Qs} atoms), {dt:.1f} s wall")
        log(f"[bench] pmd CPU oracle: {Qs * 2 / dt:.3e} atom*beads/s")
    return out


def bench_pme(args, mop, ctx, system, R, ms_rf, npairs, log):
    """The same path with particle-mesh Ewald electrostatics, the paper's own setting
    (Appendix A.1): Ewald real-space pair kernels at the same cut-off, B-spline order 4
    on a grid of at most 0.12 nm per point, rocFFT (FP64 force passes, FP32 Hessian pass).  Reports ms per veff_grad
    (eager and graph), the phase split and the cost relative to reaction field."""
    import torch
    import workloads as W
    s = W.with_pme(system)
    N, Q = R.shape[0], s["Q"]
    sysm = mop.System(ctx, s)
    grid, beta = sysm.pme_info()
    plan = mop.Plan(sysm, N, one_stream=args.pme_one_stream)
    Rt = torch.from_numpy(R).cuda()
    G = torch.empty_like(Rt)
    v = torch.empty(1, dtype=torch.float64, device=Rt.device)
    for _ in range(2):
        mop.veff_grad(plan, Rt, 0, 0.0, G, v)
    torch.cuda.synchronize()
    st = plan.status()
    settle(lambda: mop.veff_grad(plan, Rt, 0, 0.0, G, v), 1)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(args.steps):
        mop.veff_grad(plan, Rt, 0, 0.0, G, v)
    e1.record()
    torch.cuda.synchronize()
    ms_eager = e0.elapsed_time(e1) / args.steps
    ms_graph = None
    if not args.no_graph:
        g = torch.cuda.CUDAGraph()
        cs = torch.cuda.Stream()
        cs.wait_stream(torch.cuda.current_stream())
        with torch.cuda.graph(g, stream=cs):
            ctx.set_stream()
            mop.veff_grad(plan, Rt, 0, 0.0, G, v)
        ctx.set_stream()
        torch.cuda.synchronize()
        settle(g.replay, args.warmup)
        e0.record()
        for _ in range(args.steps):
            g.replay()
        e1.record()
        torch.cuda.synchronize()
        ms_graph = e0.elapsed_time(e1) / args.steps
    ms = min(ms_eager, ms_graph) if ms_graph is not None else ms_eager
    n = max(args.steps // 2, 3)

    def phase_means(pl):
        acc = None
        for _ in range(n):
            _, _, ph = mop.veff_grad_timed(pl, Rt, 0, 0.0, G, v)
            acc = ph if acc is None else {k: acc[k] + ph[k] for k in acc}
        return {k: acc[k] / n for k in acc}

    # phases of the timed call (mesh work beside the pair kernels: pme_force / pme_hvp
    # are the waits at the joins), then of the same call on one stream, where each kernel
    # runs alone and the mesh passes are phases of their own
    phases = phase_means(plan)
    if args.pme_one_stream:
        phases_1s = phases
    else:
        plan1 = mop.Plan(sysm, N, one_stream=True)
        phases_1s = phase_means(plan1)
        del plan1
    pair_beads = N - 1
    t_hvp, t_force = phases_1s["hvp"] * 1e-3, phases_1s["force"] * 1e-3
    ach = FLOP_HVP_PAIR_EWALD * npairs * pair_beads / t_hvp / 1e12
    roof = dict(bound="alu", kernel="k_pair<1,4,0,1,0> (Ewald pair Hessian-vector product)",
                achieved=round(ach, 3), peak=PEAK_FP32_TFLOPS, unit="TFLOP/s",
                frac=round(ach / PEAK_FP32_TFLOPS, 4), launch_ms=round(phases_1s["hvp"], 4),
                launch_ms_beside_mesh=round(phases["hvp"], 4),
                force_kernel=dict(achieved=round(FLOP_FORCE_PAIR_EWALD * npairs * pair_beads
                                                 / t_force / 1e12, 3),
                                  launch_ms=round(phases_1s["force"], 4),
                                  launch_ms_beside_mesh=round(phases["force"], 4)),
                mesh_ms=dict(force=round(phases_1s["pme_force"], 4),
                             hvp=round(phases_1s["pme_hvp"], 4)),
                mesh_wait_at_join_ms=dict(force=round(phases["pme_force"], 4),
                                          hvp=round(phases["pme_hvp"], 4)))
    ex = executed_from_profiles(args.config)
    if ex and "ewald_hvp_executed_flops_per_launch" in ex:
        # counted FP32 work of the Ewald kernels over their one-stream launch times
        e_h = ex["ewald_hvp_executed_flops_per_launch"] / t_hvp / 1e12
        roof["executed"] = dict(tflops=round(e_h, 3), frac=round(e_h / PEAK_FP32_TFLOPS, 4),
                                valu_per_cu_cycle=ex.get("ewald_hvp_valu_per_cu_cycle"),
                                source=f"profiles/valu_pair_{args.config}.md")
        roof["force_kernel"]["executed_tflops"] = round(
            ex["ewald_force_executed_flops_per_launch"] / t_force / 1e12, 3)
    out = dict(workload=f"{system['name']} with particle-mesh Ewald: grid {grid[0]}x{grid[1]}x"
                        f"{grid[2]}, order {s['pme_order']}, beta {beta:.4f} / nm, "
                        f"real-space cut-off {s['rc']} nm",
               ms_per_step=ms, ms_eager=ms_eager, ms_graph=ms_graph,
               value=Q * N / (ms * 1e-3), unit="atom·beads/s",
               cost_vs_reaction_field=ms / ms_rf, phases_ms=phases,
               phases_ms_one_stream=phases_1s, roofline=roof,
               device_status=st,
               veff_finite=bool(torch.isfinite(v).all()))
    log(f"[bench] PME: {ms:.3f} ms/step (eager {ms_eager:.3f}, graph {ms_graph}), "
        f"phases {json.dumps({k: round(x, 3) for k, x in phases.items()})}, one stream "
        f"{json.dumps({k: round(x, 3) for k, x in phases_1s.items()})}, status {st}")
    if not args.no_cpu_baseline:
        # CPU baseline: the FP64 oracle (Ewald real space in the C cell list on all host
        # threads, the mesh in numpy) on the first two beads, and the error of bead 1
        from oracle import cl
        from oracle import path as OP
        mop.veff_grad(plan, Rt, 0, 0.0, G, v)
        G1 = G[0].cpu().numpy()
        m = cl.CellModel(s)
        t0 = time.perf_counter()
        Gsub, _ = OP.veff_grad(m, np.ascontiguousarray(R[:2]))
        dt = time.perf_counter() - t0
        out["cpu_baseline"] = dict(
            value=Q * 2 / dt, unit="atom·beads/s", cores=cl.max_threads(), kind="oracle",
            sample=f"veff_grad of the first 2 beads (1 force + 1 Hessian-vector pass over {Q} "
                   f"atoms, real space in C, mesh in numpy), {dt:.1f} s wall")
        out["accuracy_relL2_bead1"] = float(np.linalg.norm(G1 - Gsub[0]) / np.linalg.norm(Gsub[0]))
        log(f"[bench] PME CPU oracle: {Q * 2 / dt:.3e} atom*beads/s; bead-1 G error "
            f"{out['accuracy_relL2_bead1']:.2e}")
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--config", default="cfg4")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-beads", type=int, default=12)
    ap.add_argument("--no-fd", action="store_true")
    ap.add_argument("--fd-h", type=float, default=1e-4)
    ap.add_argument("--no-graph", action="store_true")
    ap.add_argument("--no-batch", action="store_true")
    ap.add_argument("--no-pmd", action="store_true")
    ap.add_argument("--no-pme", action="store_true")
    ap.add_argument("--no-autotune", action="store_true",
                    help="default plan options instead of the autotuner's choice")
    ap.add_argument("--tune-cache", default=os.path.join("/tmp", f"mop_autotune_{os.getuid()}.json"),
                    help="autotuner cache file (JSON)")
    ap.add_argument("--pme-one-stream", action="store_true",
                    help="PME leg: mesh work on the caller's stream (times each kernel alone)")
    ap.add_argument("--calib-copy-mib", type=int, default=0,
                    help="run one plain device copy of this many MiB first (a known-size "
                         "kernel that scales HBM byte counters read by a profiler)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (--gpus {args.gpus} requested): the library "
              f"has no multi-GPU path; run with --gpus 1.", flush=True)
        sys.exit(2)

    import torch
    import workloads as W
    import paper_2501_11962_amd as mop

    t0 = time.perf_counter()
    system, R = W.make_config(args.config)
    N, Q = R.shape[0], system["Q"]
    log(f"[bench] workload {args.config}: Q={Q} N={N} rc={system['rc']} ({time.perf_counter() - t0:.1f} s)")
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    Rt = torch.from_numpy(R).to(dev)
    ctx = mop.Context()
    tune = None
    opts = {}
    if not args.no_autotune:
        # plan geometry and launch shape chosen on this path (outside the timed region)
        from paper_2501_11962_amd import autotune as A
        opts, tinfo = A.autotune(ctx, system, Rt, with_info=True, cache=args.tune_cache,
                                 log=log)
        tune = dict(default_ms=tinfo["default_ms"], tuned_ms=tinfo["ms"],
                    settings_timed=len(tinfo["tried"]), cached=tinfo["cached"])
        log(f"[bench] autotuned plan options {opts} ({tinfo['ms']:.3f} ms against "
            f"{tinfo['default_ms']} ms for the default plan)")
    plan = mop.Plan(mop.System(ctx, system), N, **opts)
    G = torch.empty_like(Rt)
    v = torch.empty(1, dtype=torch.float64, device=dev)
    if args.calib_copy_mib > 0:
        n = args.calib_copy_mib << 18
        a = torch.ones(n, dtype=torch.float32, device=dev)
        b = torch.empty_like(a)
        torch.neg(a, out=b)             # reads and writes 4 n bytes each
        torch.cuda.synchronize()
        log(f"[bench] calibration copy: {4 * n} bytes read, {4 * n} bytes written")
        del a, b

    def step():
        mop.veff_grad(plan, Rt, 0, 0.0, G, v)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    st = plan.status()
    if st:
        raise SystemExit(f"device status {st} after warm-up")
    log(f"[bench] warm-up done, V_eff = {float(v[0]):.6e}")

    def timed(fn, steps):
        """Mean over `steps` back-to-back calls (events bracketing the window, the host
        synchronised on both sides) and the median of the per-call times (an event between
        consecutive calls)."""
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
        torch.cuda.synchronize()
        ev[0].record()
        for k in range(steps):
            fn()
            ev[k + 1].record()
        torch.cuda.synchronize()
        per = [ev[k].elapsed_time(ev[k + 1]) for k in range(steps)]
        return ev[0].elapsed_time(ev[steps]) / steps, float(np.median(per))

    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    # eager timing
    settle(step, 0)
    ms_eager, med_eager = timed(step, args.steps)
    log(f"[bench] eager: {ms_eager:.3f} ms/step (median {med_eager:.3f})")

    # the whole call captured once in a graph and replayed
    ms_graph = med_graph = None
    if not args.no_graph:
        try:
            g = torch.cuda.CUDAGraph()
            cs = torch.cuda.Stream()
            cs.wait_stream(torch.cuda.current_stream())
            with torch.cuda.graph(g, stream=cs):
                ctx.set_stream()
                step()
            ctx.set_stream()
            torch.cuda.synchronize()
            Gref = G.clone()
            g.replay()
            torch.cuda.synchronize()
            # atoms are binned in a fixed order, so a replay reproduces the eager bits
            if not torch.equal(G, Gref):
                err = float((G - Gref).norm() / Gref.norm())
                raise RuntimeError(f"graph replay differs from eager (rel L2 {err:.2e})")
            settle(g.replay, max(3, args.warmup))
            ms_graph, med_graph = timed(g.replay, args.steps)
            log(f"[bench] graph: {ms_graph:.3f} ms/step (median {med_graph:.3f})")
        except Exception as ex:  # graph capture is optional; eager timing stands
            log(f"[bench] graph capture skipped: {ex}")
            ctx.set_stream()
    # the headline is the graph replay (the whole call captured once, the way a serving
    # loop issues it); eager launches are reported beside it
    ms = ms_graph if ms_graph is not None else ms_eager

    # per-phase times (HIP events between phases, same stream)
    acc = None
    for _ in range(args.steps):
        _, _, ph = mop.veff_grad_timed(plan, Rt, 0, 0.0, G, v)
        acc = ph if acc is None else {k: acc[k] + ph[k] for k in acc}
    phases = {k: acc[k] / args.steps for k in acc}
    log(f"[bench] phases (ms): {json.dumps({k: round(x, 4) for k, x in phases.items()})}")

    Ga_head = G[:max(args.cpu_beads - 1, 1)].cpu().numpy()

    # finite-difference comparison path (eq. 5 as printed: 3 force passes per bead)
    fd = None
    Gfd_head = {}
    if not args.no_fd:
        for _ in range(2):
            mop.veff_grad(plan, Rt, 1, args.fd_h, G, v)
        torch.cuda.synchronize()
        e0.record()
        for _ in range(args.steps):
            mop.veff_grad(plan, Rt, 1, args.fd_h, G, v)
        e1.record()
        torch.cuda.synchronize()
        ms_fd = e0.elapsed_time(e1) / args.steps
        fd = dict(value=Q * N / (ms_fd * 1e-3), ms_per_step=ms_fd, fd_h_nm=args.fd_h,
                  speedup_analytic_over_fd=ms_fd / ms, binning="each displaced configuration re-binned")
        log(f"[bench] FD path: {ms_fd:.3f} ms/step")
        # shared-bin variant: the displaced configurations keep R's binning
        for _ in range(2):
            mop.veff_grad(plan, Rt, 2, args.fd_h, G, v)
        torch.cuda.synchronize()
        e0.record()
        for _ in range(args.steps):
            mop.veff_grad(plan, Rt, 2, args.fd_h, G, v)
        e1.record()
        torch.cuda.synchronize()
        ms_fd2 = e0.elapsed_time(e1) / args.steps
        Gfd2_head = G[:Ga_head.shape[0]].cpu().numpy()
        fd["shared_bin"] = dict(value=Q * N / (ms_fd2 * 1e-3), ms_per_step=ms_fd2,
                                speedup_analytic_over_fd=ms_fd2 / ms)
        log(f"[bench] FD path, shared binning: {ms_fd2:.3f} ms/step")
        for h in FD_SWEEP:
            mop.veff_grad(plan, Rt, 1, h, G, v)
            Gfd_head[h] = G[:Ga_head.shape[0]].cpu().numpy()

    # roofline of the pair kernels; the headline fields are those of the one with the
    # longer launch (the dominant kernel of the step)
    npairs = unique_pairs(system, R[0])
    pair_beads = N - 1
    traffic = traffic_from_profiles(args.config)
    ex = executed_from_profiles(args.config) or {}
    kern = {}
    for k, name, fpp in (("force", "force pass: k_pair<0,4,0,0,1> (bead 1, with energies) + "
                                   "k_pair<0,4,0,0,0> (beads 2..N-1); pair forces + "
                                   "neighbour-list records", FLOP_FORCE_PAIR),
                         ("hvp", "k_pair<1,4,0,0,0> (pair Hessian-vector product, list replay)",
                          FLOP_HVP_PAIR)):
        t = phases[k] * 1e-3
        flops = fpp * npairs * pair_beads
        ach = flops / t / 1e12
        kk = dict(kernel=name, achieved=round(ach, 3), frac=round(ach / PEAK_FP32_TFLOPS, 4),
                  launch_ms=round(phases[k], 4), flop_per_pair=fpp,
                  algorithmic_flops_per_launch=flops, traffic=traffic[k])
        if traffic[k] is not None:
            gbs = traffic[k] / t / 1e9
            kk.update(hbm_gbs=round(gbs, 1), hbm_frac=round(gbs / PEAK_HBM_GBS, 4))
        if f"{k}_executed_flops_per_launch" in ex:
            # executed work (both sides of each pair, combinations beyond the cutoff, search
            # and bookkeeping instructions) per launch, over this run's launch time
            e_t = ex[f"{k}_executed_flops_per_launch"] / t / 1e12
            kk["executed"] = dict(tflops=round(e_t, 3), frac=round(e_t / PEAK_FP32_TFLOPS, 4),
                                  valu_per_cu_cycle=ex.get(f"{k}_valu_per_cu_cycle"),
                                  source=f"profiles/valu_pair_{args.config}.md")
        kern[k] = kk
    dom = max(kern, key=lambda k: kern[k]["launch_ms"])
    roof = dict(bound="alu", peak=PEAK_FP32_TFLOPS, unit="TFLOP/s", **kern[dom],
                dominant=dom, pairs_per_bead=npairs, pair_beads_per_launch=pair_beads,
                hbm_peak_gbs=PEAK_HBM_GBS, kernels=kern,
                whole_step_tflops=round((FLOP_FORCE_PAIR + FLOP_HVP_PAIR) * npairs * pair_beads
                                        / (ms * 1e-3) / 1e12, 3),
                launch_timing="HIP events on the library stream around each pair pass "
                              "(veff_grad_timed), mean over the timed calls; the force pass is "
                              "two launches, the Hessian pass one")

    out = dict(metric=METRIC, value=Q * N / (ms * 1e-3), unit="atom·beads/s", n_gpus=1,
               steps=args.steps, warmup=args.warmup, ms_per_step=ms, higher_is_better=True,
               scaling="weak", vs_baseline=None, dtype="f32",
               data="synthetic",
               config=dict(workload=f"{args.config}: {system['name']} Q={Q} atoms x N={N} beads, "
                                    f"rc={system['rc']} nm, analytic HVP",
                           Q=Q, N=N, rc=system["rc"], box=[float(b) for b in system["box"]],
                           graph=ms_graph is not None,
                           ms_eager=ms_eager, ms_graph=ms_graph,
                           median_ms_eager=med_eager, median_ms_graph=med_graph,
                           plan_options=opts or "default", autotune=tune,
                           precision="FP32 pair terms from 32-bit fixed-point coordinates; "
                                     "FP64 bonds, residuals, reductions, gradient"),
               roofline=roof, fd=fd, phases_ms=phases)
    if not args.no_cpu_baseline:
        log(f"[bench] CPU oracle on {args.cpu_beads} beads ...")
        out["cpu_baseline"], Go_head = cpu_baseline(system, R, args.cpu_beads)
        log(f"[bench] CPU oracle: {out['cpu_baseline']['value']:.3e} atom*beads/s")

        def rel(a, b):
            return float(np.linalg.norm(a - b) / np.linalg.norm(b))
        acc = dict(reference=f"FP64 oracle gradient of beads 1..{Go_head.shape[0]}",
                   analytic=rel(Ga_head, Go_head))
        if Gfd_head:
            acc["fd_by_h_nm"] = {f"{h:g}": rel(g, Go_head) for h, g in Gfd_head.items()}
            acc["fd_best"] = min(acc["fd_by_h_nm"].values())
            acc["fd_shared_bin_at_fd_h"] = rel(Gfd2_head, Go_head)
        out["accuracy_relL2"] = acc
        log(f"[bench] accuracy: {json.dumps(acc)}")
    if not args.no_pmd:
        out["pmd"] = bench_pmd(args, mop, ctx, plan, system, Rt, ms_eager, log)
    if not args.no_batch:
        out["batch"] = bench_batch(args, mop, ctx, log)
    if not args.no_pme:
        out["pme"] = bench_pme(args, mop, ctx, system, R, ms, npairs, log)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
