"""Pins of the oracle's noise, BAOAB integrator and parareal drivers.

Noise: Philox4x64-10 raw words against NumPy's independent implementation.
Integrator: reduces to velocity Verlet at gamma = 0 (time reversibility, second-order
energy error), exact Ornstein-Uhlenbeck stationary variance m kB T at V = 0.
Parareal: the exactness properties stated in the paper's "Parareal method" section
(iterate k reproduces the sequential fine trajectory on slabs 0..k; convergence in at
most N iterations), the adaptive variant reducing to the classical one, and the
paper's cost formula recomputed from the iteration log."""
import numpy as np
import pytest

from oracle import oracle as O
from oracle import parareal as PR
from paper_2212_10508_amd import workloads as W


def test_philox_matches_numpy():
    rng = np.random.default_rng(0)
    for _ in range(20):
        key = rng.integers(0, 2**63, size=2, dtype=np.uint64)
        ctr = rng.integers(1, 2**63, size=4, dtype=np.uint64)
        mine = O.philox4x64_10(ctr, key)
        c0 = ctr.copy()
        c0[0] -= np.uint64(1)     # NumPy increments the counter before each block
        ref = np.random.Philox(key=key, counter=c0).random_raw(4)
        assert np.array_equal(mine, ref)


def test_gaussian_moments():
    g = np.array([O.gauss3(1234, 3, s, a) for s in range(200) for a in range(200)])
    n = g.size
    assert abs(g.mean()) < 4 / np.sqrt(n)
    assert abs(g.var() - 1) < 4 * np.sqrt(2 / n)
    assert abs(np.mean(g ** 4) - 3) < 0.1
    # components independent
    assert abs(np.corrcoef(g[:, 0], g[:, 1])[0, 1]) < 4 / np.sqrt(len(g))


def _fs_nve(x, p, box, dt, nsteps):
    return O.langevin(x, p, box, potential=O.POT_FS, nsteps=nsteps, dt=dt, gamma=0.0,
                      mass=W.MASS_W, T=0.0, seed=1, noise_id=0, step0=0, fs=W.FS_W,
                      want_traj=True)


def test_baoab_gamma0_is_reversible_verlet():
    x, box = W.bcc_sia(4, jitter=0.05, seed=1)
    p = W.maxwell_momenta(x.shape[1], 600.0, seed=1)
    r1 = _fs_nve(x, p, box, 1e-3, 40)
    r2 = _fs_nve(r1["x"], -r1["p"], box, 1e-3, 40)
    assert np.abs(r2["x"] - x).max() < 1e-10
    assert np.abs(-r2["p"] - p).max() < 1e-10 * np.abs(p).max()


def test_baoab_gamma0_energy_error_second_order():
    x, box = W.bcc_sia(4, jitter=0.05, seed=2)
    p = W.maxwell_momenta(x.shape[1], 800.0, seed=2)

    def max_err(dt, n):
        r = _fs_nve(x, p, box, dt, n)
        H = []
        for s in range(0, n + 1, max(1, n // 20)):
            e = O.fs_compute(r["traj_x"][s], box, W.FS_W)["E"]
            ke = 0.5 * np.sum(r["traj_p"][s] ** 2) / W.MASS_W * W.MVV2E
            H.append(e + ke)
        return np.max(np.abs(np.array(H) - H[0]))

    e1 = max_err(4e-3, 50)
    e2 = max_err(2e-3, 100)
    assert 3.0 < e1 / e2 < 5.0


def test_baoab_free_particle_stationary_variance():
    """V = 0: the O step is the exact Ornstein-Uhlenbeck flow, so Var(p) = m kB T."""
    N, T = 4000, 1000.0
    x = np.zeros((3, N))
    p = np.zeros((3, N))
    r = O.langevin(x, p, np.array([1e4] * 3), potential=O.POT_NONE, nsteps=3000, dt=1e-3,
                   gamma=5.0, mass=W.MASS_W, T=T, seed=7, noise_id=2, step0=0)
    v = r["p"] / W.MASS_W
    var = v.var()
    ref = W.KB * T / W.MASS_W / W.MVV2E
    assert abs(np.sqrt(ref) - 2.1267) < 1e-3
    assert abs(var - ref) < 4 * ref * np.sqrt(2 / v.size)


def test_same_state_same_noise():
    """Propagating the same state twice (any potential) consumes the same Gaussians."""
    x, box = W.bcc_sia(4, jitter=0.05, seed=3)
    p = W.maxwell_momenta(x.shape[1], 1000.0, seed=3)
    kw = dict(nsteps=5, dt=1e-3, gamma=1.0, mass=W.MASS_W, T=1000.0, seed=11, noise_id=4,
              step0=17, fs=W.FS_W)
    a = O.langevin(x, p, box, potential=O.POT_NONE, **kw)
    b = O.langevin(x, p, box, potential=O.POT_NONE, **kw)
    assert np.array_equal(a["x"], b["x"]) and np.array_equal(a["p"], b["p"])
    # V = 0 with gamma: after one step p = c1 (p + 0) + sigma G exactly
    one = O.langevin(x, p, box, potential=O.POT_NONE, **dict(kw, nsteps=1))
    c1 = np.exp(-1.0 * 1e-3)
    sig = np.sqrt((1 - c1 ** 2) * W.MASS_W * W.KB * 1000.0 / W.MVV2E)
    G = np.array([O.gauss3(11, 4, 17, i) for i in range(x.shape[1])]).T
    assert np.abs(one["p"] - (c1 * p + sig * G)).max() < 1e-12 * np.abs(p).max()


# ---------------------------------------------------------------------------
# Parareal
# ---------------------------------------------------------------------------
def _props(J=2, L=4, seed=5):
    x, box = W.bcc_sia(4, jitter=0.05, seed=seed)
    p = W.maxwell_momenta(x.shape[1], 1000.0, seed=seed)
    snap = dict(J=J, beta=W.snap_beta(J, seed=seed, scale=2e-2), rcut=W.SNAP_RCUT,
                rfac0=W.SNAP_RFAC0, rmin0=0.0)
    prop = PR.Propagators(box=box, L=L, dt=1e-3, gamma=1.0, mass=W.MASS_W, T=1000.0,
                          seed=99, noise_id=1, snap=snap, fs=W.FS_W)
    return prop, x, p


def test_parareal_exact_after_k_iterations():
    N = 4
    prop, x, p = _props()
    ref = PR.sequential_fine(prop, x, p, N)
    _, k, iters = PR.parareal_classic(prop, x, p, N, delta_conv=0.0, max_iter=N)
    scale = np.abs(ref[-1][0]).max()
    for kk in range(1, N + 1):
        for n in range(kk + 1):
            assert np.abs(iters[kk][n][0] - ref[n][0]).max() < 1e-12 * scale
    # iterate 1 differs from the reference somewhere beyond slab 1 (SNAP matters)
    assert np.abs(iters[1][N][0] - ref[N][0]).max() > 1e-9


def test_parareal_converges_within_n_iterations():
    N = 3
    prop, x, p = _props()
    traj, k, _ = PR.parareal_classic(prop, x, p, N, delta_conv=1e-14)
    assert k <= N + 1
    ref = PR.sequential_fine(prop, x, p, N)
    assert max(np.abs(traj[n][0] - ref[n][0]).max() for n in range(N + 1)) < 1e-11


def test_parareal_coarse_equal_fine_converges_in_one():
    N = 3
    prop, x, p = _props()
    prop.C = prop.F
    traj, k, _ = PR.parareal_classic(prop, x, p, N, delta_conv=1e-12)
    # the coarse initialisation is already the fine trajectory: one iteration sees no change
    assert k == 1
    ref = PR.sequential_fine(prop, x, p, N)
    assert max(np.abs(traj[n][0] - ref[n][0]).max() for n in range(N + 1)) < 1e-12


def test_adaptive_without_explosion_equals_classic():
    N = 4
    prop, x, p = _props()
    t1, k1, _ = PR.parareal_classic(prop, x, p, N, delta_conv=1e-10)
    log = []
    # a threshold no relative error reaches (the algorithm needs it finite)
    t2, nad, kc = PR.parareal_adaptive(prop, x, p, N, delta_conv=1e-10, delta_expl=1e100,
                                       log=log)
    assert nad == 1 and kc == [k1]
    for n in range(N + 1):
        assert np.array_equal(t1[n][0], t2[n][0])
    Cf, Cc = 7.0, 1.0
    assert PR.adaptive_cost(log, N, Cf, Cc) == N * Cc + k1 * ((Cf + Cc) + N * Cc)


def test_adaptive_shortening_still_reaches_reference():
    N = 5
    prop, x, p = _props(seed=6)
    log = []
    traj, nad, kc = PR.parareal_adaptive(prop, x, p, N, delta_conv=1e-12, delta_expl=1e-7,
                                         log=log)
    assert nad > 1                      # the tiny threshold forced shortened slabs
    assert any(it["n_fi_after"] < it["n_fi"] for it in log)
    ref = PR.sequential_fine(prop, x, p, N)
    assert max(np.abs(traj[n][0] - ref[n][0]).max() for n in range(N + 1)) < 1e-11
    # cost bookkeeping matches the paper's formula evaluated by hand from the log
    Cf, Cc = 100.0, 1.0
    cost = 0.0
    for it in log:
        first = all(o["n_in"] != it["n_in"] for o in log[:log.index(it)])
        if first:
            cost += (N - it["n_in"]) * Cc
        cost += Cf + Cc + (it["n_fi"] - it["n_in"]) * Cc
    assert PR.adaptive_cost(log, N, Cf, Cc) == pytest.approx(cost)


def test_strategy_one_snap_coarse_is_exact_after_k_iterations():
    """Strategy I: the coarse propagator is Finnis-Sinclair + a smaller SNAP model.  The
    parareal property (slabs 0..k exact after k iterations) holds for any coarse
    propagator, and the coarse trajectory differs from both the FS-only one and the fine
    one (the coarse SNAP term is really in C)."""
    N = 3
    prop, x, p = _props()
    coarse = dict(J=2, beta=W.snap_beta(2, seed=9, scale=2e-2), rcut=W.SNAP_RCUT, rfac0=W.SNAP_RFAC0,
                  rmin0=0.0)
    prop1 = PR.Propagators(box=prop.box, L=prop.L, coarse_snap=coarse, scheme=prop.scheme, **prop.kw)
    ref = PR.sequential_fine(prop1, x, p, N)
    _, _, iters = PR.parareal_classic(prop1, x, p, N, delta_conv=0.0, max_iter=N)
    scale = np.abs(ref[-1][0]).max()
    for k in range(1, N + 1):
        for n in range(k + 1):
            assert np.abs(iters[k][n][0] - ref[n][0]).max() < 1e-12 * scale
    c1, c2, f = prop1.C((x, p), 0)[0], prop.C((x, p), 0)[0], prop1.F((x, p), 0)[0]
    assert np.abs(c1 - c2).max() > 1e-9 and np.abs(c1 - f).max() > 1e-9
