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
