"""Captured-graph replay of the Langevin launch sequence against one-by-one launches.

The same kernels run either way, so replays must reproduce the eager trajectory bit
for bit.  Each graph is replayed several times with eager work and synchronisations
between the replays, and every replay is checked."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_2212_10508_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def S():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2212_10508_amd import snapmd
    return snapmd


def dev(a):
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")


def _batch(n_sys=3, seed=11):
    xs, ps = [], []
    for s in range(n_sys):
        x, box = W.bcc_sia(4, jitter=0.05, seed=seed + s)
        xs.append(x)
        ps.append(W.maxwell_momenta(x.shape[1], 1000.0, seed=seed + s))
    n = xs[0].shape[1]
    X = np.concatenate(xs, axis=1)
    P = np.concatenate(ps, axis=1)
    off = np.arange(n_sys + 1, dtype=np.int32) * n
    return X, P, off, np.tile(box, (n_sys, 1))


@pytest.mark.parametrize("pot", ["fs", "fs_snap"])
def test_graph_replays_match_eager(S, pot):
    J = 6
    X, P, off, boxes = _batch()
    beta = W.snap_beta(J, seed=2, scale=2e-2)
    potential = S.POT_FS_SNAP if pot == "fs_snap" else S.POT_FS
    kw = dict(dt=1e-3, gamma=1.0, mass=W.MASS_W, T=1000.0, seed=5, noise_id=0, fs=W.FS_W, J=J, beta=beta)
    ctx = S.Context(0)
    L = 7
    ctx.use_graphs(False)
    ref = []
    xe, pe = torch.tensor(X, device="cuda"), torch.tensor(P, device="cuda")
    for r in range(3):
        ctx.langevin_steps(potential, xe, pe, off, boxes, L, step0=[r * L] * 3, **kw)
        torch.cuda.synchronize()
        ref.append((xe.clone(), pe.clone()))
    ctx.use_graphs(True)
    xg, pg = torch.tensor(X, device="cuda"), torch.tensor(P, device="cuda")
    for r in range(3):
        ctx.langevin_steps(potential, xg, pg, off, boxes, L, step0=[r * L] * 3, **kw)
        torch.cuda.synchronize()
        # eager work on the same context between replays
        f = ctx.eam_forces(xg.clone(), off, boxes, W.FS_W)
        torch.cuda.synchronize()
        assert torch.isfinite(f).all()
        assert torch.equal(xg, ref[r][0]) and torch.equal(pg, ref[r][1]), r


def test_graph_parareal_iterations_match_eager(S):
    J = 2
    x, box = W.bcc_sia(4, jitter=0.05, seed=4)
    p = W.maxwell_momenta(x.shape[1], 1000.0, seed=4)
    beta = W.snap_beta(J, seed=4, scale=2e-2)
    kw = dict(dt=1e-3, gamma=1.0, mass=W.MASS_W, T=1000.0, seed=9, noise_id=0, fs=W.FS_W, J=J, beta=beta)
    kwc = {k: v for k, v in kw.items() if k not in ("J", "beta")}
    N, L, n = 4, 5, x.shape[1]
    out = {}
    for graphs in (False, True):
        ctx = S.Context(0)
        ctx.use_graphs(graphs)
        q = torch.zeros((N + 1, 3, n), dtype=torch.float64, device="cuda")
        pp, qp, ppv = torch.zeros_like(q), torch.zeros_like(q), torch.zeros_like(q)
        q[0] = torch.tensor(x, device="cuda")
        pp[0] = torch.tensor(p, device="cuda")
        ctx.parareal_iterate(None, None, q, pp, box, L, 0, N, 1e100, **kwc)
        hist = []
        for k in range(3):
            d, _ = ctx.parareal_iterate(qp, ppv, q, pp, box, L, 0, N, 1e100, **kw)
            torch.cuda.synchronize()
            hist.append((d, q.clone(), pp.clone()))
        out[graphs] = hist
    for (d0, q0, p0), (d1, q1, p1) in zip(out[False], out[True]):
        assert d0 == d1
        assert torch.equal(q0, q1) and torch.equal(p0, p1)


@pytest.mark.parametrize("pot,scheme", [("fs", "baoab"), ("fs", "bbk"), ("fs_snap", "baoab")])
def test_long_call_replays_segments(S, pot, scheme):
    """A call of more than 1000 steps is replayed in captured segments of 250 steps (head
    with the initial force, middle segments with the step offsets advanced on the device,
    a tail holding the last step).  The same kernels run with the same arguments, so the
    result equals the call launched kernel by kernel bit for bit, for BAOAB and for the
    BBK scheme (whose first and last iterates differ from the others).  BAOAB also splits
    exactly: 1200 steps in one call equal two captured calls of 600."""
    x, box = W.bcc_sia(4, jitter=0.05, seed=41)
    n = x.shape[1]
    p = W.maxwell_momenta(n, 1000.0, seed=41)
    J = 2
    kw = dict(dt=1e-3, gamma=1.0, mass=W.MASS_W, T=1000.0, seed=3, noise_id=0, fs=W.FS_W, scheme=scheme,
              J=J, beta=W.snap_beta(J, seed=4, scale=2e-2))
    potential = S.POT_FS_SNAP if pot == "fs_snap" else S.POT_FS
    nsteps = 1200 if pot == "fs" else 1030   # 1030: head, three middle segments, a 30-step tail
    eager = S.Context(0)
    eager.use_graphs(False)
    xe, pe = dev(x), dev(p)
    eager.langevin_steps(potential, xe, pe, [0, n], box, nsteps, step0=7, **kw)
    ctx = S.Context(0)
    for rep in range(2):      # the second call replays the cached segments
        xa, pa = dev(x), dev(p)
        ctx.langevin_steps(potential, xa, pa, [0, n], box, nsteps, step0=7, **kw)
        torch.cuda.synchronize()
        assert torch.equal(xa, xe) and torch.equal(pa, pe), rep
        f = ctx.eam_forces(xa.clone(), [0, n], box, W.FS_W)   # eager work between replays
        torch.cuda.synchronize()
        assert torch.isfinite(f).all()
    if scheme == "baoab" and pot == "fs":
        xb, pb = dev(x), dev(p)
        ctx.langevin_steps(potential, xb, pb, [0, n], box, 600, step0=7, **kw)
        ctx.langevin_steps(potential, xb, pb, [0, n], box, 600, step0=607, **kw)
        torch.cuda.synchronize()
        assert torch.max(torch.abs(xa - xb)).item() < 1e-9
        assert torch.max(torch.abs(pa - pb)).item() < 1e-9 * torch.max(torch.abs(pb)).item()


def test_graph_key_tells_apart_batches_with_other_largest_system(S):
    """Two batches with the same atom count, system count and cell count but a different
    largest system: the neighbour build of the second sizes its local memory for its own
    largest system, so its launch sequence is captured anew (not replayed from the first)
    and equals the kernel-by-kernel run."""
    x8, box8 = W.bcc_sia(8, jitter=0.05, seed=13)
    J = 2
    kw = dict(dt=1e-3, gamma=1.0, mass=W.MASS_W, T=1000.0, seed=5, noise_id=0, fs=W.FS_W, J=J,
              beta=W.snap_beta(J, seed=2, scale=2e-2))
    boxes = np.tile(box8, (3, 1))
    splits = ([1025, 525, 525], [725, 725, 625])   # 2075 atoms, 3 systems, 3 cell grids each
    ctx = S.Context(0)
    ref = S.Context(0)
    ref.use_graphs(False)
    xg = torch.zeros((3, 2075), dtype=torch.float64, device="cuda")
    pg = torch.zeros_like(xg)
    for sizes in splits:
        X = np.concatenate([x8[:, :m] for m in sizes], axis=1)
        P = np.concatenate([W.maxwell_momenta(m, 1000.0, seed=m) for m in sizes], axis=1)
        off = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int32)
        xg.copy_(dev(X))
        pg.copy_(dev(P))
        ctx.langevin_steps(S.POT_FS_SNAP, xg, pg, off, boxes, 5, step0=0, **kw)
        xr, pr = dev(X), dev(P)
        ref.langevin_steps(S.POT_FS_SNAP, xr, pr, off, boxes, 5, step0=0, **kw)
        torch.cuda.synchronize()
        assert torch.equal(xg, xr) and torch.equal(pg, pr), sizes


def test_graph_key_holds_every_kernel_shape_field(S):
    """Every field of the kernel shape is part of the captured sequence's key: after a
    capture with one slot split of the density pass, the other split captures anew (its
    trajectory equals the kernel-by-kernel run with that split, and differs in the last
    bits from the first split's)."""
    J = 8
    X, P, off, boxes = _batch(n_sys=2)
    kw = dict(dt=1e-3, gamma=1.0, mass=W.MASS_W, T=1000.0, seed=5, noise_id=0, fs=W.FS_W, J=J,
              beta=W.snap_beta(J, seed=2, scale=2e-2))
    ctx = S.Context(0)
    ref = S.Context(0)
    ref.use_graphs(False)
    out = {}
    for parts in (1, 2):
        ctx.set_kernel_shape(J, (45, 0, 12, parts))
        ref.set_kernel_shape(J, (45, 0, 12, parts))
        xg, pg = dev(X), dev(P)
        ctx.langevin_steps(S.POT_FS_SNAP, xg, pg, off, boxes, 10, step0=0, **kw)
        xr, pr = dev(X), dev(P)
        ref.langevin_steps(S.POT_FS_SNAP, xr, pr, off, boxes, 10, step0=0, **kw)
        torch.cuda.synchronize()
        assert torch.equal(xg, xr) and torch.equal(pg, pr), parts
        out[parts] = xg
    assert not torch.equal(out[1], out[2])
    assert torch.max(torch.abs(out[1] - out[2])).item() < 1e-9


def test_window_noise_distinguishes_seeds_equal_as_doubles(S):
    """The Gaussians of a window are cached per (window, seed, stream); two 64-bit seeds
    that round to the same double (2^60 and 2^60 + 1) must not share them."""
    x, box = W.bcc_sia(4, jitter=0.05, seed=4)
    p = W.maxwell_momenta(x.shape[1], 1000.0, seed=4)
    n, N, L = x.shape[1], 3, 5
    assert float(2 ** 60) == float(2 ** 60 + 1)
    kwc = dict(dt=1e-3, gamma=1.0, mass=W.MASS_W, T=1000.0, noise_id=0, fs=W.FS_W)

    def init(ctx, seed):
        q = torch.zeros((N + 1, 3, n), dtype=torch.float64, device="cuda")
        pp = torch.zeros_like(q)
        q[0] = dev(x)
        pp[0] = dev(p)
        ctx.parareal_iterate(None, None, q, pp, box, L, 0, N, 1e100, seed=seed, **kwc)
        torch.cuda.synchronize()
        return q, pp

    ctx = S.Context(0)
    qa, _ = init(ctx, 2 ** 60)
    qb, pb = init(ctx, 2 ** 60 + 1)
    qc, pc = init(S.Context(0), 2 ** 60 + 1)
    assert torch.equal(qb, qc) and torch.equal(pb, pc)
    assert not torch.equal(qa[N], qb[N])


def test_profile_samples_every_kth_launch(S):
    """snapmd_profile(ctx, s) records every s-th launch of each timed kernel: 11 force
    evaluations (the initial one and 10 steps) give launches 0, 3, 6, 9 at s = 3."""
    J = 2
    X, P, off, boxes = _batch(n_sys=2)
    beta = W.snap_beta(J, seed=3, scale=2e-2)
    kw = dict(dt=1e-3, gamma=1.0, mass=W.MASS_W, T=1000.0, seed=5, noise_id=0, fs=W.FS_W, J=J, beta=beta)
    ctx = S.Context(0)
    for every, want in ((1, 11), (3, 4)):
        x, p = torch.tensor(X, device="cuda"), torch.tensor(P, device="cuda")
        ctx.profile(True, every=every)
        ctx.langevin_steps(S.POT_FS_SNAP, x, p, off, boxes, 10, step0=0, **kw)
        for kid in (S.Context.PROF_DEDR, S.Context.PROF_ADJOINT, S.Context.PROF_DENSITY, S.Context.PROF_NEIGH):
            ms, n = ctx.profile_read(kid)
            assert n == want and ms > 0.0, (every, kid, n, ms)
        ctx.profile(False)
    with pytest.raises(S.SnapmdError):
        ctx.profile(True, every=-1)
