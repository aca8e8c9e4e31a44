"""Autotuner of the slab chunks of parareal_iterate.

The pipelined parareal iteration propagates the S slabs of a window in chunks of
consecutive slabs; the sequential coarse sweep over chunk c overlaps the SNAP
propagation of chunk c + 1, so only the sweep of the last chunk is exposed.  Small
chunks expose less sweep but fill the device worse (the SNAP adjoint runs one
64-atom workgroup per compute unit, so a chunk costs about as much as the whole
adjoint rounds it occupies).  The best split depends on the atom count, the number
of compute units and the relative speed of the sweep, so it is measured: every
candidate plan is timed on the caller's own iteration and the fastest is kept.
"""
import time


def candidate_plans(S, N, n_cus, builtin=None, max_chunks=4, limit=24):
    """Chunk plans to time for a window of S slabs of N atoms: chunks of whole adjoint
    rounds (R slabs fill one round of 64-atom workgroups on the compute units left
    to the SNAP pass), or one or two slabs short of them, in non-increasing order, and
    a last chunk of at most R slabs."""
    R = max(1, ((n_cus - 16) * 64) // max(N, 1))
    sizes = sorted({v for k in (1, 2, 3) for v in (k * R - 2, k * R - 1, k * R) if 1 <= v < S}, reverse=True)
    plans = []

    def rec(prefix, left):
        if len(plans) >= 4 * limit:
            return
        if 1 <= left <= R and prefix:
            plans.append(prefix + [left])
        if len(prefix) + 1 >= max_chunks:
            return
        for v in sizes:
            if v < left and (not prefix or v <= prefix[-1]):
                rec(prefix + [v], left - v)

    rec([], S)
    # prefer few chunks and a small last chunk; keep the built-in plan
    plans.sort(key=lambda p: (len(p), p[-1]))
    out = []
    if builtin:
        out.append(list(builtin))
    for p in plans:
        if p not in out:
            out.append(p)
        if len(out) >= limit:
            break
    # when the sweep is as slow as the SNAP propagation, chunks of one round each start it
    # early and leave a short last sweep; pipelined iterations (the last sweep overlaps the
    # next iteration) favour chunks of two rounds, a little short of them where the
    # workgroups beside the propagation take more compute units
    for c in (R - 1, R, 2 * R - 3, 2 * R - 2, 2 * R - 1):
        if 1 <= c < S:
            p = [c] * (S // c) + ([S % c] if S % c else [])
            if p not in out:
                out.append(p)
    return out


def tune_chunk_plan(ctx, run_iteration, S, N, n_cus, passes=2, limit=16, log=None):
    """Time run_iteration() (one parareal iteration over a window of S slabs, synchronised
    by the caller) under each candidate plan, refine the best by moving one slab between
    neighbouring chunks, and keep it only if it beats the built-in plan when the two are
    timed alternately.  Every plan runs once untimed first (its launch sequences are
    captured then), and candidates are timed in interleaved passes, so a slow drift of
    the device's speed does not favour the plans timed last.  Sets the chosen plan on ctx
    and returns (plan, {tuple(plan): seconds})."""
    builtin = list(ctx.chunk_plan(S, N))
    times = {}

    def once(plan):
        ctx.set_chunk_plan(list(plan))
        t0 = time.perf_counter()
        run_iteration()
        return time.perf_counter() - t0

    def record(plan, t):
        key = tuple(plan)
        times[key] = min(times.get(key, float("inf")), t)

    cands = [tuple(p) for p in candidate_plans(S, N, n_cus, builtin=builtin, limit=limit)]
    for p in cands:
        once(p)
    for _ in range(passes):
        for p in cands:
            record(p, once(p))
    best = min(times, key=times.get)
    improved = True
    while improved:
        improved = False
        for c in range(len(best) - 1):
            for d in (1, -1):
                p = list(best)
                p[c] += d
                p[c + 1] -= d
                if min(p) < 1 or tuple(p) in times:
                    continue
                once(p)
                for _ in range(passes):
                    record(p, once(p))
                if times[tuple(p)] < times[best]:
                    best, improved = tuple(p), True
    # final check against the built-in plan, timed alternately
    tb = tn = float("inf")
    for _ in range(passes + 1):
        tb = min(tb, once(best))
        tn = min(tn, once(builtin))
    times[best] = min(times[best], tb)
    times[tuple(builtin)] = min(times[tuple(builtin)], tn)
    chosen = list(best) if tb < tn else builtin
    if log:
        for p in sorted(times, key=times.get):
            log("chunk plan %s: %.2f ms" % (list(p), times[p] * 1e3))
    ctx.set_chunk_plan(chosen)
    return chosen, times


def tune_sweep_width(ctx, run_iteration, N, widths=None, passes=2, log=None):
    """Time run_iteration() with the on-device coarse sweep spread over each of the given
    numbers of workgroups (by default 1 and the widths of at most 128, 96, 64, 48 and 32
    atoms per workgroup; those the system of N atoms cannot use are skipped), in
    interleaved passes after one untimed run each, and keep the fastest (1: the
    one-workgroup sweep, where the system fits in one compute unit).  Wider sweeps do
    less work per workgroup between exchanges but exchange among more workgroups and take
    more compute units from the SNAP propagation beside them.  Sets the width on ctx and
    returns (K, {K: seconds})."""
    ctx.set_sweep_workgroups(0)
    builtin = ctx.sweep_workgroups(N)
    if builtin <= 1:
        return builtin, {}
    if widths is None:
        widths = [1] + sorted({-(-N // a) for a in (128, 96, 64, 48, 32)})
    cands = []
    for K in [builtin] + list(widths):
        ctx.set_sweep_workgroups(K)
        if ctx.sweep_workgroups(N) == K and K not in cands:
            cands.append(K)
    times = {}

    def once(K):
        ctx.set_sweep_workgroups(K)
        t0 = time.perf_counter()
        run_iteration()
        return time.perf_counter() - t0

    for K in cands:
        once(K)
    for _ in range(passes):
        for K in cands:
            times[K] = min(times.get(K, float("inf")), once(K))
    best = min(times, key=times.get)
    if log:
        for K in sorted(times, key=times.get):
            log("sweep workgroups %d: %.2f ms" % (K, times[K] * 1e3))
    ctx.set_sweep_workgroups(best)
    return best, times


# ---------------------------------------------------------------------------
# Kernel shapes of the SNAP passes
# ---------------------------------------------------------------------------
def shape_candidates():
    """Every compiled kernel shape (density_acc, dedr_stage_atoms, adjoint_waves,
    density_parts), the built-in one first."""
    from itertools import product
    from .snapmd import SHAPE_CHOICES, DEFAULT_SHAPE
    out = [tuple(DEFAULT_SHAPE)]
    for s in product(SHAPE_CHOICES["density_acc"], SHAPE_CHOICES["dedr_stage_atoms"], SHAPE_CHOICES["adjoint_waves"],
                     SHAPE_CHOICES["density_parts"]):
        if s not in out:
            out.append(s)
    return out


def shape_cache_path():
    import os
    return os.environ.get("SNAPMD_TUNE_CACHE",
                          os.path.join(os.path.expanduser("~"), ".cache", "snapmd", "kernel_shapes.json"))


def shape_cache_key(arch, J, atoms_per_launch):
    """(architecture, twojmax, size class): the size class is the power of two nearest to
    the atoms one launch of the SNAP passes covers."""
    import math
    return "%s:J%d:2^%d" % (arch, J, int(round(math.log2(max(atoms_per_launch, 1)))))


def load_shape(key, path=None):
    import json
    try:
        with open(path or shape_cache_path()) as fh:
            ent = json.load(fh).get(key)
        return tuple(ent["shape"]) if ent else None
    except (OSError, ValueError, KeyError):
        return None


def save_shape(key, shape, record, path=None):
    import json
    import os
    path = path or shape_cache_path()
    try:
        with open(path) as fh:
            data = json.load(fh)
    except (OSError, ValueError):
        data = {}
    data[key] = dict(record, shape=list(shape))
    os.makedirs(os.path.dirname(path), exist_ok=True)
    tmp = path + ".tmp%d" % os.getpid()
    with open(tmp, "w") as fh:
        json.dump(data, fh, indent=1, sort_keys=True)
    os.replace(tmp, path)


def tune_kernel_shapes(ctx, J, run, force_error, tol=1e-10, passes=2, log=None):
    """Choose the kernel shape of the SNAP passes at twojmax J.  Every candidate is first
    checked: force_error() (forces of a sampled system under the current shape against the
    oracle, norm-wise relative) must be <= tol, or the candidate is dropped.  The passing
    candidates then run once untimed (their launch sequences are captured) and are timed
    with run() (synchronised by the caller) in `passes` interleaved passes; the fastest
    total wins if it beats the built-in shape by more than 1 %, else the built-in one stays.  Returns (shape, table) with table[i] = dict(shape, force_error, ms or
    None) for every candidate; the context is left on the chosen shape."""
    table = []
    for s in shape_candidates():
        ctx.set_kernel_shape(J, s)
        err = float(force_error())
        table.append(dict(shape=list(s), force_error=err, ms=None, passed=err <= tol))
        if log:
            log("shape %s: force error %.2e%s" % (s, err, "" if err <= tol else " -- dropped"))
    ok = [t for t in table if t["passed"]]
    if not ok:
        ctx.set_kernel_shape(J, None)
        raise RuntimeError("no kernel shape passes the force check")
    for t in ok:
        ctx.set_kernel_shape(J, t["shape"])
        run()
    for t in ok:
        t["ms"] = 0.0
    for _ in range(passes):
        for t in ok:
            ctx.set_kernel_shape(J, t["shape"])
            t0 = time.perf_counter()
            run()
            t["ms"] += (time.perf_counter() - t0) * 1e3 / passes
    best = min(ok, key=lambda t: t["ms"])
    # the built-in shape stays unless a candidate beats it by more than the run-to-run
    # noise (1 %)
    builtin = [t for t in ok if tuple(t["shape"]) == tuple(shape_candidates()[0])]
    if builtin and best["ms"] > 0.99 * builtin[0]["ms"]:
        best = builtin[0]
    if log:
        for t in ok:
            log("shape %s: %.2f ms" % (tuple(t["shape"]), t["ms"]))
    ctx.set_kernel_shape(J, best["shape"])
    return tuple(best["shape"]), table
