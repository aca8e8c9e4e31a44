"""Pins of the oracle's relative error between two parareal iterates.

Section "Parareal method" defines E(q^{k-1}, q^k, N) with sums over n = 1..N of the
Euclidean norm of the position vector (`def:rel-Err`); Section "Adaptive parareal method"
extends it to a window [N_in, N_fi].  The oracle's reading sums over n_in+1 .. n, which at
n_in = 0 is `def:rel-Err` itself.  The values below come from closed forms, not from the
oracle's own loop: force-free, friction-free, zero-temperature trajectories are straight
lines, so every norm in the sums is linear in the slab index and the sums are
arithmetic series.  A squared norm, a per-atom or max norm, the n_in term in either
sum or an off-by-one upper limit all change the value by far more than the tolerance.
"""
import numpy as np
import pytest

from oracle import oracle as O
from oracle import parareal as PR

L, DT, MASS = 5, 2e-3, 183.84
BOX = np.array([1e4, 1e4, 1e4])
# two atoms: positions and momenta as [3, 2] arrays built from 6-vectors
W6 = np.array([1.0, 2.0, 2.0, 2.0, 4.0, 4.0])      # |W6| = sqrt(45); per-atom norms 3 and 6
D6 = np.array([2.0, -1.0, 2.0, 0.0, 3.0, -4.0])    # |D6| = sqrt(34); per-atom norms 3 and 5


def _as_state(v6):
    return v6.reshape(2, 3).T.copy()


def _ballistic(q0, p0, nslabs):
    """Slab-boundary states of a free particle pair (no force, gamma = 0, T = 0), from the
    oracle's BAOAB propagator, L steps per slab."""
    traj = [(q0.copy(), p0.copy())]
    for n in range(nslabs):
        r = O.langevin(traj[-1][0], traj[-1][1], BOX, potential=O.POT_NONE, nsteps=L, dt=DT, gamma=0.0,
                       mass=MASS, T=0.0, seed=0, noise_id=0, step0=n * L)
        traj.append((r["x"], r["p"]))
    return traj


A0, B0, C0 = 3.0, 250.0, 40.0     # q_0 = A0 W6, p_0 = B0 m W6 / |...|, dp = C0 m D6
NS = 9


@pytest.fixture(scope="module")
def pair():
    q0 = _as_state(A0 * W6)
    prev = _ballistic(q0, _as_state(B0 * MASS * W6), NS)
    cur = _ballistic(q0, _as_state((B0 * W6 + C0 * D6) * MASS), NS)
    return prev, cur


def _closed_form(n_in, n_to):
    """sum_{n=n_in+1}^{n_to} n L dt C0 |D6|  over  sum_{n=n_in+1}^{n_to} (A0 + n L dt B0) |W6|."""
    tau = L * DT
    s1 = (n_to * (n_to + 1) - n_in * (n_in + 1)) / 2.0   # sum of n
    cnt = n_to - n_in
    num = tau * C0 * np.sqrt(34.0) * s1
    den = np.sqrt(45.0) * (A0 * cnt + tau * B0 * s1)
    return num / den


def test_ballistic_trajectories_are_straight(pair):
    prev, cur = pair
    tau = L * DT
    for n in range(NS + 1):
        assert np.allclose(prev[n][0], _as_state((A0 + n * tau * B0) * W6), rtol=0, atol=1e-12)
        assert np.allclose(cur[n][0] - prev[n][0], _as_state(n * tau * C0 * D6), rtol=0, atol=1e-12)


@pytest.mark.parametrize("n_in,n_to", [(0, 1), (0, 4), (0, NS), (2, 3), (2, 7), (5, NS)])
def test_rel_error_closed_form(pair, n_in, n_to):
    prev, cur = pair
    assert PR.rel_error(prev, cur, n_in, n_to) == pytest.approx(_closed_form(n_in, n_to), rel=1e-12)


def test_rel_error_rejects_plausible_misreadings(pair):
    """The closed form separates the reading from its near misses by > 1 %."""
    prev, cur = pair
    tau = L * DT
    n_in, n_to = 2, 7
    ref = _closed_form(n_in, n_to)
    ns = np.arange(n_in + 1, n_to + 1)
    # denominator (and numerator) including the n_in term, as the windowed sums printed
    # from N_in would have it
    ns0 = np.arange(n_in, n_to + 1)
    with_nin = (tau * C0 * np.sqrt(34.0) * ns0.sum()) / (np.sqrt(45.0) * (A0 + tau * B0 * ns0).sum())
    squared = (((tau * C0 * ns) ** 2) * 34.0).sum() / (((A0 + tau * B0 * ns) ** 2) * 45.0).sum()
    per_atom = (tau * C0 * 8.0 * ns).sum() / ((A0 + tau * B0 * ns) * 9.0).sum()
    max_norm = (tau * C0 * 4.0 * ns).sum() / ((A0 + tau * B0 * ns) * 4.0).sum()
    one_more = _closed_form(n_in, n_to + 1)
    for wrong in (with_nin, squared, per_atom, max_norm, one_more):
        assert abs(wrong - ref) > 1e-2 * ref
    assert PR.rel_error(prev, cur, n_in, n_to) == pytest.approx(ref, rel=1e-12)


def test_rel_error_at_zero_is_classical_definition(pair):
    """n_in = 0: the slab-0 state (equal in both iterates, nonzero) is in neither sum."""
    prev, cur = pair
    # |q_0| = A0 |W6| > 0 would add A0 sqrt(45) to the denominator if it were summed
    assert np.linalg.norm(prev[0][0]) == pytest.approx(A0 * np.sqrt(45.0))
    tau = L * DT
    num = sum(n * tau * C0 * np.sqrt(34.0) for n in range(1, NS + 1))
    den = sum((A0 + n * tau * B0) * np.sqrt(45.0) for n in range(1, NS + 1))
    assert PR.rel_error(prev, cur, 0, NS) == pytest.approx(num / den, rel=1e-12)


def test_rel_error_vanishes_after_n_plus_one_iterations():
    """Parareal reproduces the sequential fine trajectory after N iterations, so the
    error between iterates N and N + 1 is zero (up to rounding, C(x) + F(x) - C(x) is not
    bitwise F(x)) while the earlier ones are not."""
    from oracle import parareal as P
    import paper_2212_10508_amd.workloads as W
    N = 3
    x, box = W.bcc_sia(4, jitter=0.05, seed=5)
    p = W.maxwell_momenta(x.shape[1], 1000.0, seed=5)
    snap = dict(J=2, beta=W.snap_beta(2, seed=5, scale=2e-2), rcut=W.SNAP_RCUT, rfac0=W.SNAP_RFAC0, rmin0=0.0)
    prop = P.Propagators(box=box, L=4, dt=1e-3, gamma=1.0, mass=W.MASS_W, T=1000.0, seed=99, noise_id=1,
                         snap=snap, fs=W.FS_W)
    _, _, iters = P.parareal_classic(prop, x, p, N, delta_conv=0.0, max_iter=N + 1)
    errs = [P.rel_error(iters[k - 1], iters[k], 0, N) for k in range(1, N + 2)]
    assert all(e > 1e-10 for e in errs[:N - 1])
    assert errs[N] < 1e-14
