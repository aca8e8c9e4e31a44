"""Equilibration and interstitial analysis around the propagation (section "Numerical
results" of the paper: insert the self-interstitial, minimise the energy, thermalise with
the fine potential, then follow the defect between its metastable states and record how
many time steps it stays in each).

The arithmetic runs in the library (snapmd_relax, langevin_steps, snapmd_ws_sites); this
module only chains the calls and reduces integer site histories on the host.
"""
import math

import numpy as np
import torch

from . import snapmd as S


def equilibrate(ctx, x, p, box, fs, J=None, beta=None, potential=None, relax_iter=5000, ftol=1e-4,
                thermal_steps=10000, dt=1e-3, gamma=1.0, mass=183.84, T=1000.0, seed=0, noise_id=0,
                scheme="bbk"):
    """Minimise the energy of one system (x, p device tensors [3, N], in place), then
    thermalise it with `thermal_steps` steps of the paper's scheme (one application, as the
    paper's sequential 10,000 steps).  Returns (max |F| after the minimisation, steps)."""
    N = x.shape[1]
    pot = potential if potential is not None else (S.POT_FS_SNAP if J else S.POT_FS)
    fmax, its = ctx.relax(pot, x, [0, N], box, fs, J=J, beta=beta, max_iter=relax_iter, ftol=ftol)
    if thermal_steps > 0:
        ctx.langevin_steps(pot, x, p, [0, N], box, thermal_steps, dt=dt, gamma=gamma, mass=mass, T=T, seed=seed,
                           step0=0, noise_id=noise_id, fs=fs, J=J, beta=beta, scheme=scheme)
    return fmax, its


def interstitial_site(occ):
    """Index of the site holding the most atoms (two for a dumbbell); -1 if every site
    holds at most one atom.  occ: int tensor or array of site occupancies."""
    o = occ.cpu().numpy() if isinstance(occ, torch.Tensor) else np.asarray(occ)
    k = int(np.argmax(o))
    return k if o[k] >= 2 else -1


def residence_times(sites):
    """Lengths of the runs of equal consecutive entries of `sites` (the defect site after
    each time step): the time steps spent in each well before a hop, in order.  The last
    run is still open at the end of the record; it is returned as the last entry."""
    runs = []
    prev, n = None, 0
    for s in sites:
        if prev is None or s == prev:
            n += 1
        else:
            runs.append(n)
            n = 1
        prev = s
    if prev is not None:
        runs.append(n)
    return runs


def mean_with_ci(times, z=1.96):
    """Mean of completed residence times and its normal-approximation confidence
    interval mean +- z s / sqrt(n) (z = 1.96: 95 %)."""
    t = np.asarray(times, np.float64)
    n = t.size
    if n == 0:
        return float("nan"), (float("nan"), float("nan"))
    m = float(t.mean())
    if n == 1:
        return m, (float("nan"), float("nan"))
    h = z * float(t.std(ddof=1)) / math.sqrt(n)
    return m, (m - h, m + h)


def slab_defect_history(ctx, q, p, box, L, *, n_slabs, a, J, beta, fs, dt=1e-3, gamma=1.0, mass=183.84, T=1000.0,
                        seed=0, noise_id=0):
    """Per-step interstitial sites of a trajectory given by its slab-boundary states
    q, p (device [n_slabs + 1, 3, N]): the fine propagator is run from every slab start
    at once (one batch of n_slabs systems, slab n at global steps n L ...), one step at a
    time, and the doubly occupied Wigner-Seitz site of every slab is read after each step.
    Returns the site after each of the n_slabs * L steps, in time order."""
    N = q.shape[2]
    X = q[:n_slabs].permute(1, 0, 2).reshape(3, n_slabs * N).contiguous()
    P = p[:n_slabs].permute(1, 0, 2).reshape(3, n_slabs * N).contiguous()
    off = np.arange(n_slabs + 1, dtype=np.int32) * N
    boxes = np.tile(np.asarray(box, np.float64), (n_slabs, 1))
    n_sites = 2 * int(round(box[0] / a)) * int(round(box[1] / a)) * int(round(box[2] / a))
    hist = np.zeros((n_slabs, L), np.int64)
    for l in range(L):
        ctx.langevin_steps(S.POT_FS_SNAP, X, P, off, boxes, 1, dt=dt, gamma=gamma, mass=mass, T=T, seed=seed,
                           step0=np.arange(n_slabs) * L + l, noise_id=noise_id, fs=fs, J=J, beta=beta)
        _, occ = ctx.ws_sites(X, off, boxes, a)
        o = occ.view(n_slabs, n_sites)
        k = torch.argmax(o, dim=1)
        dbl = torch.gather(o, 1, k[:, None])[:, 0] >= 2
        hist[:, l] = torch.where(dbl, k, torch.full_like(k, -1)).cpu().numpy()
    return hist.reshape(-1).tolist()


def sequential_defect_history(ctx, x, p, box, n_steps, *, a, J, beta, fs, dt=1e-3, gamma=1.0, mass=183.84,
                              T=1000.0, seed=0, noise_id=0):
    """Per-step interstitial sites of the sequential fine trajectory from (x, p) (copied)."""
    N = x.shape[1]
    xr, pr = x.clone(), p.clone()
    hist = []
    for step in range(n_steps):
        ctx.langevin_steps(S.POT_FS_SNAP, xr, pr, [0, N], box, 1, dt=dt, gamma=gamma, mass=mass, T=T, seed=seed,
                           step0=step, noise_id=noise_id, fs=fs, J=J, beta=beta)
        hist.append(interstitial_site(ctx.ws_sites(xr, [0, N], box, a)[1]))
    return hist


def batch_defect_history(ctx, X, P, off, boxes, n_steps, *, a, J, beta, fs, step0, noise_id, dt=1e-3, gamma=1.0,
                         mass=183.84, T=1000.0, seed=0):
    """Per-step interstitial sites of every system of a batch (X, P device [3, n_atoms],
    propagated in place one step at a time; systems of equal size and box): an array
    [n_sys, n_steps] of local site indices (-1: no doubly occupied site)."""
    n_sys = len(off) - 1
    boxes = np.asarray(boxes, np.float64).reshape(n_sys, 3)
    n_sites = 2 * int(round(boxes[0][0] / a)) * int(round(boxes[0][1] / a)) * int(round(boxes[0][2] / a))
    hist = np.zeros((n_sys, n_steps), np.int64)
    step0 = np.asarray(step0, np.int64)
    for l in range(n_steps):
        ctx.langevin_steps(S.POT_FS_SNAP, X, P, off, boxes, 1, dt=dt, gamma=gamma, mass=mass, T=T, seed=seed,
                           step0=step0 + l, noise_id=noise_id, fs=fs, J=J, beta=beta)
        _, occ = ctx.ws_sites(X, off, boxes, a)
        o = occ.view(n_sys, n_sites)
        k = torch.argmax(o, dim=1)
        dbl = torch.gather(o, 1, k[:, None])[:, 0] >= 2
        hist[:, l] = torch.where(dbl, k, torch.full_like(k, -1)).cpu().numpy()
    return hist


def residence_study(ctx, x0, box, *, R, N, L, J, beta, fs, T, delta_conv, delta_expl=0.3, thermal_steps=2000,
                    relax_iter=5000, dt=1e-3, gamma=1.0, mass=183.84, seed=0, a=3.1652, same_noise=False,
                    keep_histories=False):
    """The statistical test of the paper's "Statistical analyses" at the size of x0: one
    minimised configuration, R replicas thermalised with their own noise (the paper's
    scheme), then for every replica a sequential fine trajectory of N L steps and, with
    other noise streams, an adaptive parareal trajectory (threshold delta_conv) of the same
    length; the interstitial's residence times of all replicas are pooled per method and
    summarised by their mean and 95 % confidence interval.  The parareal trajectory between
    slab boundaries is the fine propagation from its converged slab states.  same_noise:
    the parareal trajectories use the sequential ones' noise streams (then a tight
    delta_conv reproduces them step by step, the paper's trajectorial test)."""
    from . import parareal as PR
    n = x0.shape[1]
    x = x0.clone()
    fmax, _ = ctx.relax(S.POT_FS_SNAP, x, [0, n], box, fs, J=J, beta=beta, max_iter=relax_iter, ftol=1e-4)
    X = x.repeat(1, R).contiguous()
    Pm = torch.zeros_like(X)  # at rest: the thermalisation heats the replicas
    off = np.arange(R + 1, dtype=np.int32) * n
    boxes = np.tile(np.asarray(box, np.float64), (R, 1))
    kw = dict(dt=dt, gamma=gamma, mass=mass, T=T, seed=seed, fs=fs, J=J, beta=beta)
    ctx.langevin_steps(S.POT_FS_SNAP, X, Pm, off, boxes, thermal_steps, step0=0, noise_id=np.arange(R) + 1000,
                       scheme="bbk", cT=(3.0, 1.0), **kw)
    X0, P0 = X.clone(), Pm.clone()
    # sequential fine trajectories (noise streams 0 .. R-1)
    hs = batch_defect_history(ctx, X, Pm, off, boxes, N * L, a=a, step0=np.zeros(R, np.int64),
                              noise_id=np.arange(R), **kw)
    # adaptive parareal trajectories (noise streams R .. 2R-1, or 0 .. R-1 with same_noise)
    # from the same thermalised states
    pnid = np.arange(R) + (0 if same_noise else R)
    q, p, n_ad, kconv = PR.adaptive_parareal_batch(ctx, X0, P0, off, boxes, N, L, delta_conv, delta_expl,
                                                   noise_id=pnid, **{**kw, "T": [T] * R})
    Xs = q[:N].permute(1, 0, 2).reshape(3, N * R * n)  # [slab][system] order
    Ps = p[:N].permute(1, 0, 2).reshape(3, N * R * n)
    offs = np.arange(N * R + 1, dtype=np.int32) * n
    step0 = np.repeat(np.arange(N) * L, R)
    nid = np.tile(pnid, N)
    hp = batch_defect_history(ctx, Xs.contiguous(), Ps.contiguous(), offs, np.tile(boxes, (N, 1)), L, a=a,
                              step0=step0, noise_id=nid, **kw)
    hp = hp.reshape(N, R, L).transpose(1, 0, 2).reshape(R, N * L)   # per replica, in time order
    out = {"relaxed_fmax": fmax, "iterations": [int(sum(k)) for k in kconv], "windows": n_ad}
    for name, h in (("sequential", hs), ("parareal", hp)):
        runs = [residence_times(list(h[r])) for r in range(R)]
        done = [t for rr in runs for t in rr[:-1]]       # completed residence times
        m, ci = mean_with_ci(done)
        out[name] = {"hops": len(done), "mean_steps": m, "ci95": ci}
    if keep_histories:
        out["histories"] = {"sequential": hs, "parareal": hp}
    lo = max(out["sequential"]["ci95"][0], out["parareal"]["ci95"][0])
    hi = min(out["sequential"]["ci95"][1], out["parareal"]["ci95"][1])
    out["ci_overlap"] = bool(lo <= hi)
    return out
