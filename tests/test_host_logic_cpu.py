"""Host-side logic that needs no GPU: the chunk tuner's candidate plans and its
selection, and the one-GPU guard of bench.py."""
import os
import subprocess
import sys

import pytest

from paper_2212_10508_amd import tune

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.parametrize("S,N,cus", [(64, 1025, 256), (32, 16001, 256), (7, 1025, 256), (1, 129, 256),
                                     (100, 2000, 80)])
def test_candidate_plans_cover_the_window(S, N, cus):
    builtin = [S]
    plans = tune.candidate_plans(S, N, cus, builtin=builtin, limit=24)
    assert plans[0] == builtin
    assert len(plans) == len({tuple(p) for p in plans})  # no duplicates
    for p in plans:
        assert sum(p) == S and min(p) >= 1, p


def test_candidate_plans_include_one_round_chunks():
    # 64 slabs of 1025 atoms on 256 CUs: rounds of (256 - 16) * 64 atoms hold R = 14 slabs
    plans = tune.candidate_plans(64, 1025, 256, builtin=[29, 22, 13])
    assert [14, 14, 14, 14, 8] in plans and [13, 13, 13, 13, 12] in plans
    # and chunks of about two rounds (pipelined iterations)
    assert [26, 26, 12] in plans and [27, 27, 10] in plans
    # the whole-round plans are non-increasing with a last chunk of at most one round
    for p in plans[1:]:
        if len(p) <= 4:
            assert all(a >= b for a, b in zip(p, p[1:])) and p[-1] <= 14, p


class _FakeCtx:
    """Stands in for a snapmd context: a plan's 'iteration time' is a fixed function of
    the plan, so the tuner's choice can be checked without a device."""

    def __init__(self, builtin, cost):
        self.plan, self.builtin, self.cost, self.k = None, builtin, cost, 0

    def chunk_plan(self, S, N):
        return list(self.plan) if self.plan else list(self.builtin)

    def set_chunk_plan(self, p):
        self.plan = list(p) if p else None

    def set_sweep_workgroups(self, K):
        self.k = K

    def sweep_workgroups(self, N):
        # the library's rule: 1, or 8 to 64 workgroups of at most 128 atoms; otherwise the
        # built-in width (the fewest from 8 up with at most 64 atoms each)
        if self.k == 1 or (8 <= self.k <= 64 and -(-N // self.k) <= 128):
            return self.k
        return max(8, -(-N // 64))


def test_tuner_keeps_the_fastest_plan(monkeypatch):
    target = (15, 13, 14, 15, 7)
    cost = lambda p: 0.170 + 0.001 * sum(abs(a - b) for a, b in zip(p + (0,) * 5, target)) + 0.01 * abs(len(p) - 5)
    ctx = _FakeCtx([29, 22, 13], cost)
    clock = {"t": 0.0}
    monkeypatch.setattr(tune.time, "perf_counter", lambda: clock["t"])

    def run():
        clock["t"] += cost(tuple(ctx.chunk_plan(64, 1025)))

    plan, times = tune.tune_chunk_plan(ctx, run, 64, 1025, 256, passes=1)
    # the refinement walks from the nearest candidate to the cheapest plan
    assert tuple(plan) == target and ctx.plan == list(target)
    assert times[target] == min(times.values())


def test_sweep_width_tuner_picks_the_fastest(monkeypatch):
    ctx = _FakeCtx([29, 22, 13], None)
    clock = {"t": 0.0}
    monkeypatch.setattr(tune.time, "perf_counter", lambda: clock["t"])
    # default candidates at 1025 atoms: 1, the built-in 17 and the widths of at most 128,
    # 96, 64, 48 and 32 atoms per workgroup (9, 11, 17, 22, 33)
    for width_cost, best in (({1: 0.30, 9: 0.195, 11: 0.194, 17: 0.19, 22: 0.192, 33: 0.2}, 17),
                             ({1: 0.30, 9: 0.195, 11: 0.194, 17: 0.19, 22: 0.188, 33: 0.2}, 22)):
        ctx.k = 0

        def run():
            clock["t"] += width_cost[ctx.k if ctx.k else 17]

        K, times = tune.tune_sweep_width(ctx, run, 1025)
        assert K == best and ctx.k == best and set(times) == {1, 9, 11, 17, 22, 33}


def test_bench_refuses_more_than_one_gpu():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2 and "single GPU" in r.stderr


def test_parareal_windows_are_checked_before_any_call():
    """Windows must lie inside the state arrays (slots 0 .. n_slots - 1): the binding
    refuses any other before the library is called (an out-of-range window would make the
    library copy and write past the arrays)."""
    from paper_2212_10508_amd.snapmd import check_windows
    check_windows([0], [4], 5, 1)
    check_windows([0, 2], [4, 2], 5, 2)          # an empty window leaves a system of a batch out
    for n_in, n_fi, slots, R in (([0], [5], 5, 1), ([-1], [2], 5, 1), ([3], [2], 5, 1), ([2], [2], 5, 1),
                                 ([0, 1], [4, 6], 6, 2), ([0], [4], 5, 2)):
        with pytest.raises(ValueError):
            check_windows(n_in, n_fi, slots, R)


def test_kernel_shape_cache_round_trip(tmp_path):
    """Tuned kernel shapes are cached as JSON keyed by (architecture, twojmax, size class);
    another key misses, and the candidates list every compiled variant once, the built-in
    shape first."""
    path = str(tmp_path / "shapes.json")
    k = tune.shape_cache_key("gfx950", 8, 15 * 1025)
    assert k == "gfx950:J8:2^14"
    assert tune.load_shape(k, path) is None
    tune.save_shape(k, (28, 3, 12, 2), {"ms": 170.0}, path)
    tune.save_shape(tune.shape_cache_key("gfx950", 6, 129), (21, 0, 8, 1), {"ms": 1.0}, path)
    assert tune.load_shape(k, path) == (28, 3, 12, 2)
    assert tune.load_shape("gfx942:J8:2^14", path) is None
    c = tune.shape_candidates()
    assert c[0] == (45, 0, 12, 0) and len(c) == len(set(c)) == 54


def test_shape_tuner_keeps_builtin_within_noise(monkeypatch):
    """The kernel-shape tuner keeps the built-in shape unless a candidate beats it by more
    than 1 %; a candidate failing the force check is never chosen."""
    clock = {"t": 0.0}
    monkeypatch.setattr(tune.time, "perf_counter", lambda: clock["t"])
    builtin = tune.shape_candidates()[0]

    class Ctx:
        shape = None

        def set_kernel_shape(self, J, s):
            self.shape = tuple(s) if s is not None else None

        def kernel_shape(self, J):
            return self.shape

    for gain, want_builtin in ((0.005, True), (0.02, False)):
        ctx = Ctx()
        fast = tune.shape_candidates()[5]
        bad = tune.shape_candidates()[6]

        def run():
            clock["t"] += 0.100 * (1.0 - (gain if ctx.shape == fast else 0.0) - (0.5 if ctx.shape == bad else 0.0))

        shape, table = tune.tune_kernel_shapes(ctx, 8, run, lambda: 1.0 if ctx.shape == bad else 0.0, passes=1)
        assert shape == (builtin if want_builtin else fast) and ctx.shape == shape
        assert [t["passed"] for t in table if tuple(t["shape"]) == bad] == [False]


def _bench_module():
    import importlib.util
    spec = importlib.util.spec_from_file_location("bench_mod", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_bench_density_segment_count_follows_the_kernel_rule():
    """Waves per tile of the density pass as the kernel's segment rule gives them (column
    chains cut at the register budget; the last column rides on the previous column's
    last segment where it fits with its chain copy): the counts the automatic density
    split is decided by."""
    B = _bench_module()
    want = {(2, 45): 1, (4, 21): 3, (6, 45): 3, (8, 45): 4, (8, 28): 8, (8, 21): 11, (10, 45): 9, (14, 45): 18}
    for (J, acc), n in want.items():
        assert B.dens_segments(J, acc) == n, (J, acc)


def test_bench_traffic_resolves_the_automatic_split_per_chunk():
    """With density split 0 each chunk's launches take the measured bytes of the split they
    run: 26-slab chunks of 1025 atoms (1,668 density waves) unsplit, the 12-slab chunk
    (772) split, on 1,024 SIMDs."""
    B = _bench_module()
    per1, per2 = 5000.0, 7000.0
    # the per-shape figures (measured, keyed by the source hash) replaced by two constants
    B.traffic_per_unit = lambda kernel, shape: ({1: per1, 2: per2}.get(tuple(shape)[3]), "atom")
    chunks = [26 * 1025, 26 * 1025, 12 * 1025]
    got, _ = B.traffic_per_launch("adjoint", (45, 0, 12, 0), chunks, 26.0, 1024, 8)
    assert got == pytest.approx((2 * 26 * 1025 * per1 + 12 * 1025 * per2) / 3)
    got1, _ = B.traffic_per_launch("adjoint", (45, 0, 12, 1), chunks, 26.0, 1024, 8)
    assert got1 == pytest.approx(64 * 1025 * per1 / 3)
