"""Host driver of adaptive parareal over the library's parareal_iterate.

Follows the paper's "Adaptive parareal method" (its Algorithm "Adaptive parareal
algorithm"): a time window [n_in, n_fi] is initialised by a coarse sweep, then
corrected iterations (all fine and coarse slab propagations batched in one launch
sequence, followed by the sequential corrected coarse sweep) run until the relative
error falls below delta_conv; when it exceeds delta_expl the window is shortened.
The branch logic below is host code; every propagation runs in the HIP library.

Readings (shared with the oracle's driver): the relative error sums run over slabs
n_in+1 .. n (the n_in term is equal in both iterates); a shortened window keeps at
least one slab; the tentative window is [n_in, min(N, n_in + max_window)].
delta_expl must be finite (the algorithm starts from delta = (delta_conv+delta_expl)/2).
"""
import torch

from . import snapmd as S


def adaptive_parareal(ctx, q0, p0, box, N, L, delta_conv, delta_expl, *, dt, gamma, mass, T, seed, noise_id,
                      fs, J, beta, max_window=None, log=None, **snap_kw):
    """Run adaptive parareal for one trajectory of n atoms (q0, p0: device [3, n]).

    Returns (q, p, n_ad, kconv) with q, p device tensors [N+1, 3, n] holding the
    converged states at every slab boundary."""
    if not (delta_expl < float("inf")):
        raise ValueError("delta_expl must be finite (use a large value for the classical algorithm)")
    max_window = N if max_window is None else int(max_window)
    n = q0.shape[1]
    dev = q0.device
    q_cur = torch.zeros((N + 1, 3, n), dtype=torch.float64, device=dev)
    p_cur = torch.zeros_like(q_cur)
    q_prev = torch.zeros_like(q_cur)
    p_prev = torch.zeros_like(q_cur)
    q_cur[0].copy_(q0)
    p_cur[0].copy_(p0)
    kw = dict(dt=dt, gamma=gamma, mass=mass, T=T, seed=seed, noise_id=noise_id, fs=fs, J=J, beta=beta, **snap_kw)
    n_in, n_fi = 0, 0
    delta = 0.5 * (delta_conv + delta_expl)
    kconv = []
    while n_fi < N:
        if delta < delta_expl:
            n_in = n_fi
            n_fi = min(N, n_in + max_window)
            ctx.parareal_iterate(None, None, q_cur, p_cur, box, L, n_in, n_fi, delta_expl, **kw)
            kconv.append(0)
        delta = 0.5 * (delta_conv + delta_expl)
        while delta_conv <= delta <= delta_expl:
            window = n_fi
            delta, n_fi = ctx.parareal_iterate(q_prev, p_prev, q_cur, p_cur, box, L, n_in, n_fi, delta_expl, **kw)
            kconv[-1] += 1
            if log is not None:
                log.append(dict(n_in=n_in, n_fi=window, n_fi_after=n_fi, delta=delta))
    return q_cur, p_cur, len(kconv), kconv


def adaptive_parareal_batch(ctx, q0, p0, offset, box, N, L, delta_conv, delta_expl, *, dt, gamma, mass, T, seed,
                            noise_id, fs, J, beta, max_window=None, logs=None, **snap_kw):
    """Adaptive parareal for every system of a ragged batch at once, each system running
    the paper's algorithm on windows of its own.  q0, p0: device [3, offset[-1]]; box:
    [n_sys, 3]; T, noise_id: one per system.  Every round issues at most two calls of
    parareal_iterate over the whole batch: the initialisation of the systems that start a
    new window, then one corrected iteration of every system that is iterating (systems
    with nothing to do get an empty window).

    Returns (q, p, n_ad, kconv): q, p device [N+1, 3, n_atoms]; n_ad[r] and kconv[r] as
    the single-system driver returns them; logs (a list of R lists) receives each system's
    iterations like its log."""
    if not (delta_expl < float("inf")):
        raise ValueError("delta_expl must be finite (use a large value for the classical algorithm)")
    R = len(offset) - 1
    max_window = N if max_window is None else int(max_window)
    n = q0.shape[1]
    q_cur = torch.zeros((N + 1, 3, n), dtype=torch.float64, device=q0.device)
    p_cur = torch.zeros_like(q_cur)
    q_prev = torch.zeros_like(q_cur)
    p_prev = torch.zeros_like(q_cur)
    q_cur[0].copy_(q0)
    p_cur[0].copy_(p0)
    kw = dict(dt=dt, gamma=gamma, mass=mass, T=T, seed=seed, noise_id=noise_id, fs=fs, J=J, beta=beta, **snap_kw)
    mid = 0.5 * (delta_conv + delta_expl)
    NEW, ITER, DONE = 0, 1, 2
    phase = [NEW] * R
    n_in, n_fi = [0] * R, [0] * R
    kconv = [[] for _ in range(R)]
    while any(ph != DONE for ph in phase):
        starting = [r for r in range(R) if phase[r] == NEW]
        if starting:
            a, b = [0] * R, [0] * R
            for r in starting:
                n_in[r] = n_fi[r]
                n_fi[r] = min(N, n_in[r] + max_window)
                a[r], b[r] = n_in[r], n_fi[r]
                kconv[r].append(0)
                phase[r] = ITER
            ctx.parareal_iterate_batch(None, None, q_cur, p_cur, offset, box, L, a, b, delta_expl, **kw)
        it = [r for r in range(R) if phase[r] == ITER]
        a = [n_in[r] if phase[r] == ITER else 0 for r in range(R)]
        b = [n_fi[r] if phase[r] == ITER else 0 for r in range(R)]
        delta, nfi = ctx.parareal_iterate_batch(q_prev, p_prev, q_cur, p_cur, offset, box, L, a, b, delta_expl, **kw)
        for r in it:
            window = n_fi[r]
            n_fi[r] = int(nfi[r])
            kconv[r][-1] += 1
            d = float(delta[r])
            if logs is not None:
                logs[r].append(dict(n_in=n_in[r], n_fi=window, n_fi_after=n_fi[r], delta=d))
            if delta_conv <= d <= delta_expl:
                continue                      # next iteration on the same window
            if n_fi[r] >= N:
                phase[r] = DONE
            elif d < delta_expl:
                phase[r] = NEW                # converged on its window: the next one starts
            # else: shortened window, iterate on it (delta restarts from the midpoint)
    return q_cur, p_cur, [len(k) for k in kconv], kconv


def adaptive_cost(log, N, Cf, Cc):
    """The paper's cost of the adaptive algorithm from an iteration log: per time
    window, the coarse initialisation over its tentative span, then per iteration
    (Cf + Cc) + (n_fi - n_in) Cc."""
    cost, seen = 0.0, set()
    for it in log:
        if it["n_in"] not in seen:
            seen.add(it["n_in"])
            cost += (it["n_fi"] - it["n_in"]) * Cc
        cost += (Cf + Cc) + (it["n_fi"] - it["n_in"]) * Cc
    return cost


def sequential_fine(ctx, q0, p0, box, N, L, *, dt, gamma, mass, T, seed, noise_id, fs, J, beta, **snap_kw):
    """Reference trajectory q_{n+1} = F(q_n) on the device ([N+1, 3, n])."""
    n = q0.shape[1]
    q = torch.zeros((N + 1, 3, n), dtype=torch.float64, device=q0.device)
    p = torch.zeros_like(q)
    q[0].copy_(q0)
    p[0].copy_(p0)
    x, v = q0.clone(), p0.clone()
    for s in range(N):
        ctx.langevin_steps(S.POT_FS_SNAP, x, v, [0, n], box, L, dt=dt, gamma=gamma, mass=mass, T=T, seed=seed,
                           step0=s * L, noise_id=noise_id, fs=fs, J=J, beta=beta, **snap_kw)
        q[s + 1].copy_(x)
        p[s + 1].copy_(v)
    return q, p
