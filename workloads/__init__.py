"""Seeded synthetic systems and paths for the Onsager-Machlup path-gradient workloads.

This module only *places* atoms and draws random numbers.  It contains none of the
method's arithmetic (no potential, no force, no Hessian, no residual): both the
FP64 CPU oracle and the HIP library consume what it produces, and neither is
imported here.

Units: nm, ps, amu, kJ/mol, e.

A system is a plain ``dict``:

    Q            number of atoms
    box          (3,) orthorhombic box lengths
    x            (Q, 3) float64 reference coordinates in [0, box)
    mass         (Q,) float64
    charge       (Q,) float64
    type         (Q,) int32 LJ type index
    sigma, epsilon (ntypes,) float64 per-type LJ parameters (mixed by Lorentz-Berthelot)
    bonds        (nb, 2) int32 harmonic bonds (i, j)
    bond_r0, bond_k (nb,) float64
    mol, molpos  (Q,) int32: molecule id and position along a linear chain; every
                 molecule is a linear chain (a water is H-O-H), which is what the
                 1-2/1-3 exclusion rule needs
    rc, eps_rf, eps_r, dt, nu, kT
    name         workload label

A path is an (N, Q, 3) float64 array of bead coordinates.  The method draws no random
numbers itself; the Gaussian increments used to build a path are returned so tests
can check closed forms that involve them.

Five workloads follow the paper's setting (overdamped Langevin trajectories of
molecular systems, section 1.1 and Appendix A.2) at the sizes the benchmark uses:

    cfg1  256-atom FCC Lennard-Jones + reaction-field crystal, 32 beads
    cfg2  1,000 flexible 3-site waters, 64 beads
    cfg3  23,000 atoms, 4 LJ types, 35 % in 50-atom chains, 128 beads
    cfg4  150,000 atoms, membrane-shaped: water + dense chain slab + core, 16 beads
    cfg5  24 water boxes of uneven size and length (batched)
"""
from __future__ import annotations

import hashlib
import math
import os

import numpy as np

KB = 0.0083144626  # kJ mol^-1 K^-1

# Water model used by cfg2/cfg4/cfg5 (3-site, flexible O-H bonds, LJ on O only).
WATER_Q_O, WATER_Q_H = -0.82, 0.41
WATER_R0, WATER_KB = 0.1, 345000.0
WATER_ANGLE = math.radians(104.52)
M_O, M_H, M_DEFAULT = 15.999, 1.008, 16.0
SIG_O, EPS_O = 0.315, 0.65

# Mixed-type recipe (cfg3, cfg4 slab): four (sigma, epsilon) types.
MIX_SIGMA = np.array([0.25, 0.29333333333333333, 0.33666666666666667, 0.38])
MIX_EPS = np.array([0.2, 0.43333333333333335, 0.66666666666666667, 0.9])
CHAIN_LEN = 50
CHAIN_KB = 2.5e5

# Time step and friction for cfg2-cfg5 (Appendix A.2: 1 fs, 0.25 fs^-1).
DT_PMD, NU_PMD = 0.001, 250.0


def _system(name, box, x, mass, charge, typ, sigma, eps, bonds, r0, kb, mol, molpos,
            rc, dt, nu, T=300.0, eps_rf=78.0, eps_r=1.0):
    Q = x.shape[0]
    box = np.asarray(box, dtype=np.float64)
    x = np.mod(np.asarray(x, dtype=np.float64), box)
    return dict(
        name=name, Q=int(Q), box=box, x=x,
        mass=np.asarray(mass, np.float64), charge=np.asarray(charge, np.float64),
        type=np.asarray(typ, np.int32),
        sigma=np.asarray(sigma, np.float64), epsilon=np.asarray(eps, np.float64),
        bonds=np.asarray(bonds, np.int32).reshape(-1, 2),
        bond_r0=np.asarray(r0, np.float64), bond_k=np.asarray(kb, np.float64),
        mol=np.asarray(mol, np.int32), molpos=np.asarray(molpos, np.int32),
        rc=float(rc), eps_rf=float(eps_rf), eps_r=float(eps_r),
        dt=float(dt), nu=float(nu), kT=KB * T,
    )


def _random_rotations(rng, n):
    """n uniformly random rotation matrices (QR of Gaussian matrices, sign-fixed)."""
    a = rng.standard_normal((n, 3, 3))
    q, r = np.linalg.qr(a)
    d = np.sign(np.diagonal(r, axis1=1, axis2=2))
    q = q * d[:, None, :]
    det = np.linalg.det(q)
    q[:, :, 0] *= det[:, None]
    return q


def _water_molecules(rng, o_pos, first_mol=0):
    """Atoms of waters whose oxygens sit at o_pos; order per molecule is H1, O, H2."""
    n = o_pos.shape[0]
    half = 0.5 * WATER_ANGLE
    h_local = np.array([[math.sin(half), math.cos(half), 0.0],
                        [-math.sin(half), math.cos(half), 0.0]]) * WATER_R0
    rot = _random_rotations(rng, n)
    h = np.einsum("nij,kj->nki", rot, h_local) + o_pos[:, None, :]
    x = np.empty((n, 3, 3))
    x[:, 0], x[:, 1], x[:, 2] = h[:, 0], o_pos, h[:, 1]
    x = x.reshape(-1, 3)
    mass = np.tile([M_H, M_O, M_H], n)
    charge = np.tile([WATER_Q_H, WATER_Q_O, WATER_Q_H], n)
    typ = np.tile([1, 0, 1], n)  # 0 = O (LJ), 1 = H (no LJ)
    base = 3 * np.arange(n)
    bonds = np.stack([np.stack([base, base + 1], 1), np.stack([base + 1, base + 2], 1)], 1).reshape(-1, 2)
    mol = np.repeat(np.arange(n) + first_mol, 3)
    molpos = np.tile([0, 1, 2], n)
    return x, mass, charge, typ, bonds, mol, molpos


def _wrap(x, box):
    y = x - box * np.floor(x / box)
    return np.minimum(y, np.nextafter(box, 0.0))


def _declash_waters(rng, x, mol, box, first, nwat, dmin=0.16, iters=40):
    """Re-draw the orientation of waters (atoms [first, first + 3 nwat), order H, O, H)
    that have an atom closer than dmin to an atom of another molecule.  Pure geometry
    on the periodic box; oxygen positions are kept."""
    from scipy.spatial import cKDTree
    half = 0.5 * WATER_ANGLE
    h_local = np.array([[math.sin(half), math.cos(half), 0.0],
                        [-math.sin(half), math.cos(half), 0.0]]) * WATER_R0
    for _ in range(iters):
        pairs = cKDTree(_wrap(x, box), boxsize=box).query_pairs(dmin, output_type="ndarray")
        if len(pairs):
            pairs = pairs[mol[pairs[:, 0]] != mol[pairs[:, 1]]]
        atoms = np.unique(pairs.ravel()) if len(pairs) else np.zeros(0, np.int64)
        atoms = atoms[(atoms >= first) & (atoms < first + 3 * nwat)]
        w = np.unique((atoms - first) // 3)
        if len(w) == 0:
            break
        o = x[first + 3 * w + 1]
        h = np.einsum("nij,kj->nki", _random_rotations(rng, len(w)), h_local) + o[:, None, :]
        x[first + 3 * w] = h[:, 0]
        x[first + 3 * w + 2] = h[:, 1]
    return x


def _lattice_sites(counts, spacing, origin=(0.0, 0.0, 0.0)):
    nx, ny, nz = counts
    g = np.stack(np.meshgrid(np.arange(nx), np.arange(ny), np.arange(nz), indexing="ij"), -1).reshape(-1, 3)
    return (g + 0.5) * np.asarray(spacing) + np.asarray(origin)


def water_box(Q, seed, rc=1.0, name=None, dt=DT_PMD, nu=NU_PMD, density=100.0, jitter=0.02):
    """Q/3 flexible waters at `density` atoms/nm^3 in a cubic box; oxygens on a jittered
    simple-cubic lattice (random subset of sites when Q/3 is not a cube)."""
    assert Q % 3 == 0 and Q >= 3
    rng = np.random.default_rng(seed)
    nmol = Q // 3
    L = (Q / density) ** (1.0 / 3.0)
    m = int(math.ceil(nmol ** (1.0 / 3.0) - 1e-9))
    sites = _lattice_sites((m, m, m), L / m)
    if sites.shape[0] > nmol:
        sites = sites[np.sort(rng.choice(sites.shape[0], nmol, replace=False))]
    o = sites + rng.normal(0.0, jitter, sites.shape)
    x, mass, charge, typ, bonds, mol, molpos = _water_molecules(rng, o)
    box = np.array([L, L, L])
    x = _declash_waters(rng, x, mol, box, 0, nmol)
    nb = bonds.shape[0]
    return _system(name or f"water{Q}", [L, L, L], x, mass, charge, typ,
                   [SIG_O, 0.0], [EPS_O, 0.0], bonds, np.full(nb, WATER_R0),
                   np.full(nb, WATER_KB), mol, molpos, rc, dt, nu)


def cfg1(seed=101):
    """256-atom jittered FCC crystal, LJ (0.315 nm, 0.65 kJ/mol) + reaction field,
    alternating +/-0.4 e charges, cutoff 0.9 nm, dt 2 fs, nu 5/ps, m 16 amu."""
    rng = np.random.default_rng(seed)
    L = 1.97
    a = L / 4
    basis = np.array([[0, 0, 0], [0.5, 0.5, 0], [0.5, 0, 0.5], [0, 0.5, 0.5]])
    cells = _lattice_sites((4, 4, 4), a) - 0.5 * a
    x = (cells[:, None, :] + basis[None] * a).reshape(-1, 3) + 0.25 * a
    x = x + rng.normal(0.0, 0.02, x.shape)
    Q = x.shape[0]
    charge = np.where(np.arange(Q) % 2 == 0, 0.4, -0.4)
    return _system("cfg1", [L, L, L], x, np.full(Q, M_DEFAULT), charge, np.zeros(Q),
                   [SIG_O], [EPS_O], np.zeros((0, 2)), [], [], np.arange(Q),
                   np.zeros(Q), rc=0.9, dt=0.002, nu=5.0)


def cfg2(seed=201):
    """1,000 flexible waters (3,000 atoms), 100 atoms/nm^3, cutoff 1.0 nm."""
    return water_box(3000, seed, rc=1.0, name="cfg2")


def _serpentine(counts):
    """Lattice sites ordered so that consecutive sites are nearest neighbours: rows
    along x alternate direction globally, rows along y alternate per layer."""
    nx, ny, nz = counts
    order = []
    row = 0
    for k in range(nz):
        ys = range(ny) if k % 2 == 0 else range(ny - 1, -1, -1)
        for j in ys:
            xs = range(nx) if row % 2 == 0 else range(nx - 1, -1, -1)
            order.extend((i, j, k) for i in xs)
            row += 1
    return np.array(order, dtype=np.int64)


def _chains_on_serpentine(counts, nchains, chain_len):
    """Start index (in serpentine order) of each chain, spread so chains never share a
    site and every bond joins lattice neighbours."""
    total = counts[0] * counts[1] * counts[2]
    assert nchains * chain_len <= total
    return (np.arange(nchains) * total) // nchains


def _mixed_chain_atoms(rng, n):
    typ = rng.integers(0, 4, n)
    q = rng.normal(0.0, 0.3, n)
    return typ, q


def cfg3(seed=301):
    """23,000 atoms in a 6.1 nm box: four LJ types, N(0, 0.3 e) charges neutralised,
    35 % of the atoms in 50-atom chains (self-avoiding lattice walks), cutoff 1.0 nm."""
    rng = np.random.default_rng(seed)
    Q, L = 23000, 6.1
    nch = int(round(0.35 * Q / CHAIN_LEN))  # 161 chains
    m = int(math.ceil(Q ** (1.0 / 3.0)))    # 29^3 = 24,389 sites
    a = L / m
    sites = _lattice_sites((m, m, m), a).reshape(m, m, m, 3)
    # chains: serpentine walk through the lattice, one chain per slab of the order
    order = _serpentine((m, m, m))
    used = np.zeros(m ** 3, bool)
    flat = lambda ijk: (ijk[:, 0] * m + ijk[:, 1]) * m + ijk[:, 2]
    total = m ** 3
    starts = (np.arange(nch) * (total - CHAIN_LEN)) // max(nch - 1, 1)
    chain_sites = []
    for s in starts:
        idx = flat(order[s:s + CHAIN_LEN])
        if used[idx].any():
            continue
        used[idx] = True
        chain_sites.append(idx)
    chain_sites = np.stack(chain_sites)[:nch]
    nch = chain_sites.shape[0]
    free = np.flatnonzero(~used)
    nfree = Q - nch * CHAIN_LEN
    free = np.sort(rng.choice(free, nfree, replace=False))
    site_xyz = sites.reshape(-1, 3)
    x = np.concatenate([site_xyz[chain_sites.reshape(-1)], site_xyz[free]])
    nchain_atoms = nch * CHAIN_LEN
    jit = np.where(np.arange(Q)[:, None] < nchain_atoms, 0.005, 0.02)
    x = x + rng.normal(0.0, 1.0, x.shape) * jit
    typ, q = _mixed_chain_atoms(rng, Q)
    q = q - q.mean()
    base = np.arange(nch)[:, None] * CHAIN_LEN
    bi = (base + np.arange(CHAIN_LEN - 1)).reshape(-1)
    bonds = np.stack([bi, bi + 1], 1)
    mol = np.concatenate([np.repeat(np.arange(nch), CHAIN_LEN), nch + np.arange(nfree)])
    molpos = np.concatenate([np.tile(np.arange(CHAIN_LEN), nch), np.zeros(nfree, int)])
    return _system("cfg3", [L, L, L], x, np.full(Q, M_DEFAULT), q, typ, MIX_SIGMA, MIX_EPS,
                   bonds, np.full(len(bonds), a), np.full(len(bonds), CHAIN_KB), mol, molpos,
                   rc=1.0, dt=DT_PMD, nu=NU_PMD)


def cfg4(seed=401):
    """150,000 atoms in a 10 x 10 x 15 nm box shaped like a solvated membrane: water at
    92.6 atoms/nm^3 outside a 4 nm slab (|z - 7.5| < 2 nm) that is 30 % denser and made
    of 963 bonded 50-atom chains on a 0.2 nm lattice; the 100 chains closest to the
    slab centre form the 5,000-atom core (own types).  Cutoff 1.2 nm."""
    rng = np.random.default_rng(seed)
    Lx, Ly, Lz = 10.0, 10.0, 15.0
    # --- slab: 50 x 50 x 20 lattice, spacing 0.2 nm, z in [5.5, 9.5)
    cnt = (50, 50, 20)
    a = 0.2
    order = _serpentine(cnt)
    nch = 963
    starts = _chains_on_serpentine(cnt, nch, CHAIN_LEN)
    ijk = order[(starts[:, None] + np.arange(CHAIN_LEN)).reshape(-1)]
    slab_x = (ijk + 0.5) * a + np.array([0.0, 0.0, 5.5])
    slab_x = slab_x + rng.normal(0.0, 0.005, slab_x.shape)
    nslab = slab_x.shape[0]
    centre = slab_x.reshape(nch, CHAIN_LEN, 3).mean(1)
    rxy = np.hypot(centre[:, 0] - 5.0, centre[:, 1] - 5.0) + 0.3 * np.abs(centre[:, 2] - 7.5)
    core = np.zeros(nch, bool)
    core[np.argsort(rxy)[:100]] = True
    styp, sq = _mixed_chain_atoms(rng, nslab)
    styp = styp + 2                       # lipid types 2..5
    core_atoms = np.repeat(core, CHAIN_LEN)
    styp = np.where(core_atoms, rng.integers(0, 4, nslab) + 6, styp)  # core types 6..9
    sq = sq - sq.mean()
    # --- solvent: 33,950 waters on a 31 x 31 x 36 lattice over the 11 nm of solvent
    nwat = (150000 - nslab) // 3
    wcnt = (31, 31, 36)
    wsp = np.array([Lx / 31, Ly / 31, 11.0 / 36])
    wsites = _lattice_sites(wcnt, wsp)
    wsites = wsites[np.sort(rng.choice(wsites.shape[0], nwat, replace=False))]
    wsites[:, 2] = np.where(wsites[:, 2] < 5.5, wsites[:, 2], wsites[:, 2] + 4.0)
    o = wsites + rng.normal(0.0, 0.02, wsites.shape)
    wx, wm, wq, wt, wb, wmol, wpos = _water_molecules(rng, o)
    # --- assemble: slab chains first, then waters
    x = np.concatenate([slab_x, wx])
    Q = x.shape[0]
    assert Q == 150000, Q
    mol_all = np.concatenate([np.repeat(np.arange(nch), CHAIN_LEN), wmol + nch])
    x = _declash_waters(rng, x, mol_all, np.array([Lx, Ly, Lz]), nslab, nwat)
    base = np.arange(nch)[:, None] * CHAIN_LEN
    bi = (base + np.arange(CHAIN_LEN - 1)).reshape(-1)
    sbonds = np.stack([bi, bi + 1], 1)
    bonds = np.concatenate([sbonds, wb + nslab])
    r0 = np.concatenate([np.full(len(sbonds), a), np.full(len(wb), WATER_R0)])
    kb = np.concatenate([np.full(len(sbonds), CHAIN_KB), np.full(len(wb), WATER_KB)])
    mol = np.concatenate([np.repeat(np.arange(nch), CHAIN_LEN), wmol + nch])
    molpos = np.concatenate([np.tile(np.arange(CHAIN_LEN), nch), wpos])
    typ = np.concatenate([styp, wt])
    mass = np.concatenate([np.full(nslab, M_DEFAULT), wm])
    charge = np.concatenate([sq, wq])
    sigma = np.concatenate([[SIG_O, 0.0], MIX_SIGMA, MIX_SIGMA])
    eps = np.concatenate([[EPS_O, 0.0], MIX_EPS, MIX_EPS])
    return _system("cfg4", [Lx, Ly, Lz], x, mass, charge, typ, sigma, eps, bonds, r0, kb,
                   mol, molpos, rc=1.2, dt=DT_PMD, nu=NU_PMD)


def cfg5(seed=500, npaths=24):
    """24 independent water boxes: Q log-uniform in [1e3, 2e4] (rounded to whole
    waters), N uniform in [16, 128], 100 atoms/nm^3, cutoff 1.0 nm.  Returns a list of
    (system, N, path_seed)."""
    rng = np.random.default_rng(seed)
    out = []
    for p in range(npaths):
        q = math.exp(rng.uniform(math.log(1000.0), math.log(20000.0)))
        Q = max(3 * int(round(q / 3.0)), 1002)
        N = int(rng.integers(16, 129))
        out.append((water_box(Q, seed + 1 + p, rc=1.0, name=f"cfg5_{p}"), N, seed + 1 + p))
    return out


def tiny(Q=24, L=1.6, seed=7, rc=0.7, charges=True, bonds=True, ntypes=2, dt=DT_PMD,
         nu=NU_PMD, jitter=0.03):
    """Small mixed system for tests: jittered cubic lattice, some 3-atom chains."""
    rng = np.random.default_rng(seed)
    m = int(math.ceil(Q ** (1.0 / 3.0)))
    sites = _lattice_sites((m, m, m), L / m)[:Q]
    x = sites + rng.normal(0.0, jitter, sites.shape)
    typ = rng.integers(0, ntypes, Q)
    sig = np.linspace(0.26, 0.34, ntypes)
    eps = np.linspace(0.3, 0.8, ntypes)
    q = rng.normal(0.0, 0.4, Q) if charges else np.zeros(Q)
    q = q - q.mean()
    mol = np.arange(Q)
    molpos = np.zeros(Q, int)
    bl = []
    if bonds:
        # chains of 3 consecutive lattice sites along x where available
        for s in range(0, Q - 2, 6):
            i, j, k = s, s + 1, s + 2
            if k < Q and (sites[k, 2] > sites[i, 2]):
                bl += [(i, j), (j, k)]
                mol[[i, j, k]] = mol[i]
                molpos[[i, j, k]] = [0, 1, 2]
    bl = np.array(bl, dtype=np.int32).reshape(-1, 2)
    r0 = np.full(len(bl), L / m)
    kb = np.full(len(bl), 5.0e4)
    mass = rng.uniform(8.0, 20.0, Q)
    return _system("tiny", [L, L, L], x, mass, q, typ, sig, eps, bl, r0, kb, mol, molpos,
                   rc=rc, dt=dt, nu=nu)


def _smooth_at_least(n):
    """Smallest integer >= n whose only prime factors are 2, 3, 5 and 7."""
    k = max(int(n), 1)
    while True:
        m = k
        for f in (2, 3, 5, 7):
            while m % f == 0:
                m //= f
        if m == 1:
            return k
        k += 1


def with_pme(system, spacing=0.12, order=4, rtol=1e-5, grid=None):
    """Copy of a system switched to particle-mesh Ewald electrostatics (the paper's
    standard-MD setting, Appendix A.1): real-space cut-off = the system's r_c, splitting
    parameter from erfc(beta r_c) = rtol, B-spline order `order`, and a grid of at most
    `spacing` nm per point (2,3,5,7-smooth sizes) unless `grid` is given."""
    s = dict(system)
    if grid is None:
        grid = [max(_smooth_at_least(math.ceil(L / spacing)), 2 * order) for L in s["box"]]
    s.update(elec="pme", pme_order=int(order), ewald_rtol=float(rtol),
             pme_grid=np.asarray(grid, np.int32), name=s["name"] + "+pme")
    return s


def noise_sigma(system, sigma=None):
    """Per-atom Gaussian step size of a Brownian path: sqrt(2 kT dt / (m nu)) unless a
    fixed value is given (cfg1 uses 0.005 nm)."""
    if sigma is not None:
        return np.full(system["Q"], float(sigma))
    return np.sqrt(2.0 * system["kT"] * system["dt"] / (system["mass"] * system["nu"]))


def path_noise(system, N, seed):
    """The (N-1, Q, 3) standard-normal increments zeta^n used to build a path."""
    rng = np.random.default_rng(seed)
    return rng.standard_normal((max(N - 1, 0), system["Q"], 3))


def random_walk_path(system, N, seed, sigma=None, x0=None):
    """Path R^1 = x0, R^{n+1} = R^n + s_i zeta^n (Brownian increments, no drift term).
    Returns (R, zeta, s)."""
    s = noise_sigma(system, sigma)
    zeta = path_noise(system, N, seed)
    R = np.empty((N, system["Q"], 3))
    R[0] = system["x"] if x0 is None else x0
    for n in range(N - 1):
        R[n + 1] = R[n] + s[:, None] * zeta[n]
    return R, zeta, s


TETHER = 0.1   # mean-reversion per bead of tethered_path


def tethered_path(system, N, seed, sigma=None, kappa=TETHER, x0=None):
    """Path R^1 = x0, R^{n+1} = R^n + kappa (R^1 - R^n) + s_i zeta^n: Brownian increments
    with a harmonic tether to the first bead (an Euler-Maruyama walk of overdamped motion
    in a harmonic well), so beads stay within about s_i / sqrt(2 kappa) of R^1 instead of
    drifting apart as sqrt(n) s_i; a free walk of 100 beads brings atoms of different
    molecules closer than 0.01 nm.  Returns (R, zeta, s)."""
    s = noise_sigma(system, sigma)
    zeta = path_noise(system, N, seed)
    R = np.empty((N, system["Q"], 3))
    R[0] = system["x"] if x0 is None else x0
    for n in range(N - 1):
        R[n + 1] = R[n] + kappa * (R[0] - R[n]) + s[:, None] * zeta[n]
    return R, zeta, s


def drifted_path(system, N, seed, drift, sigma=None):
    """Path R^{n+1} = R^n + drift(R^n) + s_i zeta^n with a caller-supplied drift
    callable (tests pass c*F from the oracle: an Euler-Maruyama trajectory).
    Returns (R, zeta, s)."""
    s = noise_sigma(system, sigma)
    zeta = path_noise(system, N, seed)
    R = np.empty((N, system["Q"], 3))
    R[0] = system["x"]
    for n in range(N - 1):
        R[n + 1] = R[n] + drift(R[n]) + s[:, None] * zeta[n]
    return R, zeta, s


def steepest_descent(system, energy_forces, max_step=2e-3, fmax=5e3, iters=500, log=None):
    """Steepest descent of the atoms of `system` under a caller-supplied callable
    x -> (U(x), F(x)) (energy and (Q, 3) forces): the atom with the largest force moves by
    the step h along its force and every other atom proportionally less
    (x' = x + h F / max_i |F_i|); a step that lowers U is kept and h grows by 1.2 (at most
    `max_step` nm), one that does not is undone and h shrinks by 0.2.  Stops when
    max_i |F_i| <= fmax or after `iters` force evaluations.  Removes the overlaps that
    random placement at liquid density leaves before a path is built (the paper's paths
    start from equilibrated structures, Appendix A.2).
    Returns (x wrapped into the box, evaluations done, final max |F|)."""
    box = np.asarray(system["box"], np.float64)
    x = np.array(system["x"], np.float64)
    U, F = energy_forces(x)
    fm = float(np.linalg.norm(F, axis=1).max())
    h = max_step
    it = 0
    for it in range(1, iters + 1):
        if fm <= fmax:
            break
        xn = x + (h / fm) * F
        Un, Fn = energy_forces(xn)
        if Un < U:
            x, U, F = xn, Un, Fn
            fm = float(np.linalg.norm(F, axis=1).max())
            h = min(1.2 * h, max_step)
        else:
            h *= 0.2
        if log is not None and it % 25 == 0:
            log(f"  sd {it}: U {U:.6e}, max|F| {fm:.3e}, step {h:.2e} nm")
    return _wrap(x, box), it, fm


CONFIGS = {
    "cfg1": dict(make=cfg1, N=32, path_seed=102, sigma=0.005),
    "cfg2": dict(make=cfg2, N=64, path_seed=202, sigma=None),
    "cfg3": dict(make=cfg3, N=128, path_seed=302, sigma=None),
    "cfg4": dict(make=cfg4, N=16, path_seed=402, sigma=None),
}

# Stored inputs (tests/golden/relaxed_inputs.py writes them with the FP64 oracle's
# forces): relaxed starting structures of cfg3 and cfg4, and cfg1's Euler-Maruyama path.
STORED = {
    "cfg1": "path_cfg1.npz",
    "cfg3": "relaxed_cfg3.npz",
    "cfg4": "relaxed_cfg4.npz",
}
STORE_DIR = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                         "tests", "golden")


def system_digest(system):
    """Hash of a generated system's coordinates and parameters: a stored input made from
    another version of the generator is refused."""
    h = hashlib.sha256()
    for k in ("x", "mass", "charge", "type", "sigma", "epsilon", "bonds"):
        h.update(np.ascontiguousarray(system[k]).tobytes())
    return h.hexdigest()[:16]


def load_stored(name, system):
    """The stored arrays of workload `name` (see STORED), checked against the system."""
    path = os.path.join(STORE_DIR, STORED[name])
    if not os.path.exists(path):
        raise FileNotFoundError(f"{path} is missing: run `python tests/golden/relaxed_inputs.py {name}`")
    with np.load(path, allow_pickle=False) as z:
        d = {k: z[k] for k in z.files}
    if str(d["digest"]) != system_digest(system):
        raise RuntimeError(f"{path} was made from another version of the {name} generator: "
                           f"run `python tests/golden/relaxed_inputs.py {name}`")
    return d


def make_config(name, N=None, relaxed=True):
    """(system, R) for one of cfg1-cfg4 with its path.
    cfg1: Euler-Maruyama path R^{n+1} = R^n + c F(R^n) + 0.005 nm noise (stored).
    cfg3, cfg4: tethered Brownian beads (tethered_path) from the relaxed structure
    (stored), which also replaces the system's reference coordinates.  cfg2: tethered
    Brownian beads from the generated structure (its waters are placed without
    contacts).  relaxed=False gives the unrelaxed inputs with free random-walk beads."""
    c = CONFIGS[name]
    sys_ = c["make"]()
    N = N or c["N"]
    if relaxed and name == "cfg1":
        R = load_stored(name, sys_)["R"]
        if N > R.shape[0]:
            raise ValueError(f"the stored cfg1 path has {R.shape[0]} beads")
        return sys_, np.ascontiguousarray(R[:N])
    if relaxed and name in STORED:
        sys_ = dict(sys_, x=load_stored(name, sys_)["x"])
    if not relaxed:
        R, _, _ = random_walk_path(sys_, N, c["path_seed"], c["sigma"])
    else:
        R, _, _ = tethered_path(sys_, N, c["path_seed"], c["sigma"])
    return sys_, R


def batch_paths(specs=None):
    """The uneven batch (cfg5): [(system, R, seed)] with tethered Brownian beads."""
    out = []
    for s_, N, seed in (specs or cfg5()):
        R, _, _ = tethered_path(s_, N, seed)
        out.append((s_, R, seed))
    return out
