"""GPU parity of the metadynamics-of-paths bias (mop_bias_*) and of biased path dynamics
against the oracle (oracle/mop_bias.py, oracle/pmd.py).

The bias itself is FP64 on both sides (tolerance 1e-12 on S, V_bias and the Gaussian
history for identical inputs); in integrated runs the FP32 pair terms of V_eff's gradient
make positions differ by ~1e-7 relative, so S and the deposited centres then agree to
~1e-8 absolute.
"""
import numpy as np
import pytest

import workloads as W
from oracle import mop_bias as MB
from oracle import path as OP
from oracle import pmd
from oracle.potential import Model

pytestmark = pytest.mark.gpu


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


def cuda(x):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x, np.float64)).cuda()


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / max(np.linalg.norm(b), 1e-300))


def say(*a):
    print(*a, flush=True)


def groups(s, a0=0, b0=100, na=6, nb=8):
    """The na atoms nearest atom a0 and the nb atoms nearest atom b0 (disjoint)."""
    X, L = s["x"], s["box"]

    def near(i, n, skip=()):
        d = X - X[i]
        d -= L * np.rint(d / L)
        order = np.argsort((d * d).sum(1))
        return np.array([j for j in order if j not in skip][:n], np.int32)
    A = near(a0, na)
    return A, near(b0, nb, set(A.tolist()))


def test_bias_apply_deposit_and_history(mop, ctx):
    s = W.cfg1()
    N = 6
    A, B = groups(s)
    plan = mop.Plan(mop.System(ctx, s), N)
    sig, w0, gam, kT = 0.02, 1.5, 5.0, 2.494
    bias = mop.Bias(plan, A, B, sig, w0, gam, kT, stride=1, max_gaussians=64)
    ob = MB.Bias(A, B, s["mass"], s["box"], sig, w0, gam, kT, stride=1)
    paths = [W.random_walk_path(s, N, 40 + k, 0.01)[0] for k in range(5)]
    for k, R in enumerate(paths):
        out = bias.apply(cuda(R), deposit=True).cpu().numpy()
        S, V, _ = ob.apply(R, step=0)
        say(f"[bias] deposit {k}: S {out[1]:.6f} (oracle {S:.6f}), V {out[0]:.6e} ({V:.6e})")
        assert out[1] == pytest.approx(S, rel=1e-12, abs=1e-14)
        assert out[0] == pytest.approx(V, rel=1e-12, abs=1e-14)
    c, w = bias.history()
    assert np.allclose(c, ob.centers, rtol=1e-12, atol=1e-14)
    assert np.allclose(w, ob.heights, rtol=1e-12)
    # gradient of V_eff + V_bias on a new path
    R = W.random_walk_path(s, N, 77, 0.01)[0]
    Rt = cuda(R)
    G, _ = mop.veff_grad(plan, Rt)
    out = bias.apply(Rt, G).cpu().numpy()
    S, V, Gb = MB.bias_gradient(R, A, B, s["mass"], s["box"], ob.centers, ob.heights, sig)
    assert abs(V) > 0.0
    Go, _ = OP.veff_grad(Model(s), R)
    e = rel(G.cpu().numpy(), Go + Gb)
    say(f"[bias] total gradient relL2 {e:.2e}; bias part max {np.max(np.abs(Gb)):.3e}")
    assert e < 1e-5
    # the bias part alone, FP64 on both sides
    Gz = cuda(np.zeros_like(R))
    bias.apply(Rt, Gz)
    assert np.max(np.abs(Gz.cpu().numpy() - Gb)) < 1e-11 * max(np.max(np.abs(Gb)), 1e-30)
    assert plan.status() == 0


def test_biased_pmd_matches_oracle(mop, ctx):
    s = W.cfg1()
    N, steps, tau = 8, 6, 1e-3
    A, B = groups(s)
    R0, _, _ = W.random_walk_path(s, N, 31, 0.005)
    V0 = np.random.default_rng(9).normal(0.0, 0.3, R0.shape)
    sig, w0, gam, kT = 0.01, 3.0, 4.0, 2.494
    plan = mop.Plan(mop.System(ctx, s), N)
    bias = mop.Bias(plan, A, B, sig, w0, gam, kT, stride=2)
    R, V = cuda(R0), cuda(V0)
    G, _ = mop.veff_grad(plan, R)
    bias.apply(R, G)
    E = mop.pmd_step(plan, R, V, G, tau, steps, 250.0, kT, seed=3, step0=0, bias=bias)
    assert plan.status() == 0
    ob = MB.Bias(A, B, s["mass"], s["box"], sig, w0, gam, kT, stride=2)
    Ro, Vo, Go, Eo = pmd.run(Model(s), R0, V0, s["mass"], tau, steps, 250.0, kT, 3, 0, ob)
    Eg = E.cpu().numpy()
    eR = rel(R.cpu().numpy() - R0, Ro - R0)
    say(f"[bias pmd] displacement relL2 {eR:.2e}; S {Eg[:, 3]} vs {Eo[:, 3]}")
    assert eR < 1e-6 and rel(V.cpu().numpy(), Vo) < 1e-5
    assert np.allclose(Eg[:, 3], Eo[:, 3], rtol=0, atol=1e-8)
    assert np.allclose(Eg[:, 2], Eo[:, 2], rtol=1e-6, atol=1e-9)
    assert np.allclose(Eg[:, :2], Eo[:, :2], rtol=1e-6)
    c, w = bias.history()
    assert len(c) == 3                       # steps 0, 2, 4
    assert np.allclose(c, ob.centers, rtol=0, atol=1e-8)
    assert np.allclose(w, ob.heights, rtol=1e-6)


def test_bias_capacity_reset_and_bad_args(mop, ctx):
    s = W.cfg1()
    A, B = groups(s)
    plan = mop.Plan(mop.System(ctx, s), 3)
    bias = mop.Bias(plan, A, B, 0.02, 1.0, max_gaussians=2)
    R = cuda(W.random_walk_path(s, 3, 5, 0.01)[0])
    plan.clear_status()
    for _ in range(3):
        bias.apply(R, deposit=True)
    assert len(bias.history()[0]) == 2
    assert plan.status() & 2                 # MOP_DEV_CAPACITY
    plan.clear_status()
    bias.reset()
    assert len(bias.history()[0]) == 0
    out = bias.apply(R).cpu().numpy()
    assert out[0] == 0.0
    for kw in (dict(groupA=A, groupB=np.concatenate([B, A[:1]])),       # overlapping
               dict(groupA=A, groupB=[s["Q"]]),                          # out of range
               dict(groupA=A, groupB=B, sigma=0.0),
               dict(groupA=A, groupB=B, bias_factor=0.5),
               dict(groupA=A, groupB=B, bias_factor=4.0, kT=0.0),
               dict(groupA=A, groupB=B, stride=0)):
        args = dict(sigma=0.02, height=1.0)
        args.update(kw)
        with pytest.raises(mop.MopError):
            mop.Bias(plan, **args)
    with pytest.raises(mop.MopError):       # a bias of another plan
        other = mop.Plan(mop.System(ctx, s), 3)
        mop.pmd_step(other, R, R.clone() * 0, R.clone() * 0, 1e-3, bias=bias)
