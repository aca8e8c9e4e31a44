"""Parareal drivers of the oracle, sequential and literal.

TEST INFRASTRUCTURE ONLY (tests, smoke check and CPU-baseline leg of the benchmark).

Follows the paper's "Parareal method" and "Adaptive parareal method" sections:
classical parareal (coarse initialisation, then corrections with the jumps
F(prev_n) - C(prev_n) and a sequential coarse sweep; Algorithm "Parareal algorithm")
and its adaptive variant (slab shortening when the relative error exceeds the
explosion threshold; Algorithm "Adaptive parareal algorithm").

Propagators: F and C both take L Langevin steps of length dt from (q, p) on slab n,
with the same noise (global steps n*L .. n*L+L-1 of one noise stream), F on the
fine potential (Finnis-Sinclair + SNAP), C on the coarse one (Finnis-Sinclair, the
paper's strategy II with an EAM coarse potential, or Finnis-Sinclair + a second,
smaller SNAP model, its strategy I); the steps are BAOAB, or one application of L
iterates of the paper's BBK scheme.

Readings where the paper leaves room:
* Relative error E(prev, cur, n_in, n) = sum_{m=n_in+1}^{n} |cur_m - prev_m| /
  sum_{m=n_in+1}^{n} |prev_m|, |.| the Euclidean norm of the 3m position vector.  The
  windowed form printed in "Adaptive parareal method" starts both sums at N_in, while
  the classical definition (`def:rel-Err`) starts at n = 1; the paper calls the first a
  natural extension of the second, and the two agree only if the sums start after the
  window's first index.  That reading is taken here.  It is a choice that changes the
  value: leaving |prev_{n_in}| out of the denominator makes E about (m + 1)/m times the
  printed windowed form after m slabs (twice on the first slab), so windows shorten
  slightly earlier.  Pinned by closed forms of straight-line trajectories
  (tests/test_oracle_rel_error.py).
* A shortened window keeps at least one slab: n_fi := max(n, n_in + 1).
* The tentative window of a new time-slab is [n_in, min(N, n_in + max_window)]
  (max_window = N gives the paper's algorithm).
"""
import numpy as np

from . import oracle as O


class Propagators:
    """F and C of one trajectory (one noise stream) for the oracle."""

    def __init__(self, *, box, L, dt, gamma, mass, T, seed, noise_id, snap, fs, maxn=64, scheme="baoab",
                 cT=(1.0, 1.0), coarse_snap=None, coarse_fs=None):
        self.kw = dict(dt=dt, gamma=gamma, mass=mass, T=T, seed=seed, noise_id=noise_id,
                       snap=snap, fs=fs, maxn=maxn)
        self.box = box
        self.L = L
        self.scheme = scheme  # "baoab", or "bbk": the paper's scheme, one application per slab
        self.cT = cT
        self.coarse_snap = coarse_snap  # None: C on Finnis-Sinclair alone
        self.coarse_fs = coarse_fs      # None: C uses the fine potential's Finnis-Sinclair part
        self.n_fine = 0
        self.n_coarse = 0

    def _run(self, state, n, potential, snap=None, fs=None):
        q, p = state
        kw = dict(self.kw)
        if snap is not None:
            kw["snap"] = snap
        if fs is not None:
            kw["fs"] = fs
        if self.scheme == "bbk":
            r = O.bbk(q, p, self.box, potential=potential, nsteps=self.L, step0=n * self.L, cT=self.cT, **kw)
        else:
            r = O.langevin(q, p, self.box, potential=potential, nsteps=self.L, step0=n * self.L, **kw)
        return (r["x"], r["p"])

    def F(self, state, n):
        self.n_fine += 1
        return self._run(state, n, O.POT_FS_SNAP)

    def C(self, state, n):
        self.n_coarse += 1
        if self.coarse_snap is not None:
            return self._run(state, n, O.POT_FS_SNAP, self.coarse_snap, self.coarse_fs)
        return self._run(state, n, O.POT_FS, None, self.coarse_fs)


def rel_error(prev, cur, n_in, n_to):
    num = sum(np.linalg.norm(cur[m][0] - prev[m][0]) for m in range(n_in + 1, n_to + 1))
    den = sum(np.linalg.norm(prev[m][0]) for m in range(n_in + 1, n_to + 1))
    return num / den


def sequential_fine(prop, q0, p0, N):
    """Reference trajectory q_{n+1} = F(q_n)."""
    traj = [(q0.copy(), p0.copy())]
    for n in range(N):
        traj.append(prop.F(traj[-1], n))
    return traj


def parareal_classic(prop, q0, p0, N, delta_conv, max_iter=None):
    """Classical parareal.  Returns (trajectory, k_conv, list of iterates)."""
    cur = [(q0.copy(), p0.copy())]
    for n in range(N):
        cur.append(prop.C(cur[n], n))
    k, delta = 0, 2.0 * delta_conv
    iterates = [list(cur)]
    while delta >= delta_conv:
        if max_iter is not None and k >= max_iter:
            break
        k += 1
        prev = list(cur)
        jumps = []
        for n in range(N):
            fq, fp = prop.F(prev[n], n)
            cq, cp = prop.C(prev[n], n)
            jumps.append((fq - cq, fp - cp))
        for n in range(N):
            cq, cp = prop.C(cur[n], n)
            cur[n + 1] = (cq + jumps[n][0], cp + jumps[n][1])
        delta = rel_error(prev, cur, 0, N)
        iterates.append(list(cur))
    return cur, k, iterates


def parareal_adaptive(prop, q0, p0, N, delta_conv, delta_expl, max_window=None, log=None):
    """Adaptive parareal.  Returns (trajectory, N_ad, [k_conv^i]); ``log`` (a list)
    receives one dict per iteration: n_in, n_fi (window used), n_fi_after, delta.
    delta_expl must be finite (the algorithm starts from delta = (delta_conv + delta_expl)/2)."""
    max_window = N if max_window is None else max_window
    n_in, n_fi = 0, 0
    delta = 0.5 * (delta_conv + delta_expl)
    cur = [None] * (N + 1)
    cur[0] = (q0.copy(), p0.copy())
    kconv = []
    while n_fi < N:
        if delta < delta_expl:
            n_in = n_fi
            n_fi = min(N, n_in + max_window)
            for n in range(n_in, n_fi):
                cur[n + 1] = prop.C(cur[n], n)
            kconv.append(0)
        delta = 0.5 * (delta_conv + delta_expl)
        while delta_conv <= delta <= delta_expl:
            prev = list(cur)
            jumps = {}
            for n in range(n_in, n_fi):
                fq, fp = prop.F(prev[n], n)
                cq, cp = prop.C(prev[n], n)
                jumps[n] = (fq - cq, fp - cp)
            kconv[-1] += 1
            window = n_fi
            for n in range(n_in, window):
                cq, cp = prop.C(cur[n], n)
                cur[n + 1] = (cq + jumps[n][0], cp + jumps[n][1])
                delta = rel_error(prev, cur, n_in, n + 1)
                if delta > delta_expl:
                    n_fi = max(n, n_in + 1)
                    break
            if log is not None:
                log.append(dict(n_in=n_in, n_fi=window, n_fi_after=n_fi, delta=delta))
    return cur, len(kconv), kconv


def adaptive_cost(log, N, Cf, Cc):
    """Cost of the adaptive algorithm from its iteration log (paper's cost formula):
    per time-slab i, (N - n_in^i) Cc for the coarse initialisation, then per
    iteration (Cf + Cc) + (n_fi^{i,j} - n_in^i) Cc."""
    cost, seen = 0.0, set()
    for it in log:
        if it["n_in"] not in seen:
            # coarse initialisation over the tentative window (N - n_in for max_window = N)
            seen.add(it["n_in"])
            cost += (it["n_fi"] - it["n_in"]) * Cc
        cost += (Cf + Cc) + (it["n_fi"] - it["n_in"]) * Cc
    return cost
