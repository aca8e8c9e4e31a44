"""Parity of the HIP path (through the C ABI) against the CPU oracle, element by element.

Tolerances (FP64 on both sides, different summation order and FMA contraction):
  forces      max_i |F_i - F_i^oracle| / max_i |F_i^oracle| <= 1e-10
  energies    relative 1e-12 per atom (scale: max |E_i|)
  bispectrum  relative 1e-12 (scale: max |B_k| per component)
  trajectory  100 BAOAB steps under shared noise: max |dq| <= 1e-8 A and
              max |dp| <= 1e-8 max |p|
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import oracle as O
from paper_2212_10508_amd import workloads as W

pytestmark = pytest.mark.gpu

FTOL, ETOL, BTOL, QTOL = 1e-10, 1e-12, 1e-12, 1e-8


@pytest.fixture(scope="module")
def S():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2212_10508_amd import snapmd
    return snapmd


def dev(a):
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def frel(f, ref):
    return np.max(np.linalg.norm(f - ref, axis=0)) / np.max(np.linalg.norm(ref, axis=0))


@pytest.mark.parametrize("J", [2, 4, 6, 8])
def test_snap_forces_and_energy(S, J):
    x, box = W.bcc_sia(4, jitter=0.1, seed=20 + J)
    beta = W.snap_beta(J, seed=J)
    beta[0] = -0.25
    ref = O.snap_compute(x, box, J, beta)
    N = x.shape[1]
    e = torch.zeros(N, dtype=torch.float64, device="cuda")
    f = S.snap_forces(dev(x), [0, N], box, J, beta, e_atom=e)
    fg, eg = host(f), host(e)
    assert frel(fg, ref["f"]) < FTOL
    assert np.max(np.abs(eg - ref["e_atom"])) < ETOL * np.max(np.abs(ref["e_atom"]))
    assert np.abs(fg.sum(axis=1)).max() < 1e-11 * np.abs(fg).max() * np.sqrt(N)


@pytest.mark.parametrize("J", [6, 8])
def test_bispectrum(S, J):
    x, box = W.bcc_sia(4, jitter=0.1, seed=30 + J)
    beta = W.snap_beta(J, seed=J)
    ref = O.snap_compute(x, box, J, beta)["B"]            # [N, K]
    B = host(S.context().bispectrum(dev(x), [0, x.shape[1]], box, J, beta)).T
    assert np.max(np.abs(B - ref) / np.max(np.abs(ref), axis=0)) < BTOL


def test_eam_forces_and_energy(S):
    x, box = W.bcc_sia(6, jitter=0.1, seed=3)
    ref = O.fs_compute(x, box, W.FS_W)
    N = x.shape[1]
    e = torch.zeros(N, dtype=torch.float64, device="cuda")
    f = S.eam_forces(dev(x), [0, N], box, W.FS_W, e_atom=e)
    assert frel(host(f), ref["f"]) < FTOL
    assert np.max(np.abs(host(e) - ref["e_atom"])) < ETOL * np.max(np.abs(ref["e_atom"]))


def test_perfect_lattice_zero_force(S):
    x, box = W.bcc_sia(4, interstitial=False)
    J = 8
    beta = W.snap_beta(J, seed=5, scale=1e-2)
    f = host(S.snap_forces(dev(x), [0, x.shape[1]], box, J, beta))
    assert np.abs(f).max() < 1e-11
    e = torch.zeros(x.shape[1], dtype=torch.float64, device="cuda")
    S.eam_forces(dev(x), [0, x.shape[1]], box, W.FS_W, e_atom=e)
    assert abs(host(e).mean() - (-8.9000024)) < 5e-7


def test_ragged_batch_snap_and_accumulate(S):
    """Systems of 129, 433, 0 (empty) and 129 atoms in one launch, forces added onto FS."""
    J = 8
    beta = W.snap_beta(J, seed=1)
    parts = [W.bcc_sia(4, jitter=0.08, seed=1), W.bcc_sia(6, jitter=0.08, seed=2),
             (np.zeros((3, 0)), np.array([12.66, 12.66, 12.66])), W.bcc_sia(4, jitter=0.12, seed=3)]
    X, off, B = W.pack([p[0] for p in parts], [p[1] for p in parts])
    N = X.shape[1]
    xd = dev(X)
    f = S.eam_forces(xd, off, B, W.FS_W)
    S.snap_forces(xd, off, B, J, beta, f=f, accumulate=True)
    fg = host(f)
    for s, (x, box) in enumerate(parts):
        if x.shape[1] == 0:
            continue
        ref = O.snap_compute(x, box, J, beta)["f"] + O.fs_compute(x, box, W.FS_W)["f"]
        assert frel(fg[:, off[s]:off[s + 1]], ref) < FTOL


@pytest.mark.parametrize("J", [2, 8])
def test_propagation_forces_fold_fs_into_snap(S, J):
    """A propagation step evaluates FS + SNAP as one chain (the FS density term in the slot
    table, rho and F'(rho) in the density pass, the FS half of dE_i/dr in k_dedr).  Its
    force at the final positions (f_out) against the separate FS and SNAP kernels at the
    same positions, and against the oracle, on a ragged batch with an empty system and a
    1025-atom system (cell grid)."""
    beta = W.snap_beta(J, seed=4, scale=2e-2)
    parts = [W.bcc_sia(4, jitter=0.08, seed=5), (np.zeros((3, 0)), np.array([12.66, 12.66, 12.66])),
             W.bcc_sia(8, jitter=0.05, seed=6), W.bcc_sia(6, jitter=0.1, seed=7)]
    X, off, B = W.pack([p[0] for p in parts], [p[1] for p in parts])
    N = X.shape[1]
    P = np.concatenate([W.maxwell_momenta(x.shape[1], 1000.0, seed=8 + s) for s, (x, _) in enumerate(parts)],
                       axis=1)
    ctx = S.context()
    xd, pd = dev(X), dev(P)
    f = torch.zeros((3, N), dtype=torch.float64, device="cuda")
    ctx.langevin_steps(S.POT_FS_SNAP, xd, pd, off, B, 1, step0=0, dt=1e-3, gamma=1.0, mass=W.MASS_W, T=1000.0,
                       seed=3, noise_id=0, fs=W.FS_W, J=J, beta=beta, f_out=f)
    fg = host(f)
    ref = S.eam_forces(xd.clone(), off, B, W.FS_W)
    S.snap_forces(xd.clone(), off, B, J, beta, f=ref, accumulate=True)
    assert frel(fg, host(ref)) < FTOL
    xh = host(xd)
    for s, (x, box) in enumerate(parts):
        if x.shape[1] == 0:
            continue
        xs = xh[:, off[s]:off[s + 1]]
        fo = O.snap_compute(xs, box, J, beta)["f"] + O.fs_compute(xs, box, W.FS_W)["f"]
        assert frel(fg[:, off[s]:off[s + 1]], fo) < FTOL, s


def test_full_size_slab_batch_sampled(S):
    """64 slabs x 1025 atoms, twojmax 8 (the benchmark launch): systems sampled."""
    J = 8
    wl = W.slabs_1025(n_slabs=64, seed=1)
    X, off, B = W.pack(wl["xs"], [wl["box"]] * 64)
    f = host(S.snap_forces(dev(X), off, B, J, wl["beta"]))
    for s in (0, 37, 63):
        ref = O.snap_compute(wl["xs"][s], wl["box"], J, wl["beta"])["f"]
        assert frel(f[:, off[s]:off[s + 1]], ref) < FTOL


def test_determinism_bitwise(S):
    x, box = W.bcc_sia(6, jitter=0.1, seed=9)
    J = 8
    beta = W.snap_beta(J, seed=9)
    a = host(S.snap_forces(dev(x), [0, x.shape[1]], box, J, beta))
    b = host(S.snap_forces(dev(x), [0, x.shape[1]], box, J, beta))
    assert np.array_equal(a, b)


def _langevin_pair(S, potential, x, p, box, nsteps, J=None, beta=None, step0=0, noise_id=0, T=1000.0):
    kw = dict(dt=1e-3, gamma=1.0, mass=W.MASS_W, T=T, seed=4242, step0=step0, noise_id=noise_id)
    xd, pd = dev(x), dev(p)
    S.langevin_steps(potential, xd, pd, [0, x.shape[1]], box, nsteps, fs=W.FS_W, J=J, beta=beta, **kw)
    snap = dict(J=J, beta=beta, rcut=W.SNAP_RCUT, rfac0=W.SNAP_RFAC0, rmin0=0.0) if J else None
    ref = O.langevin(x, p, box, potential=potential, nsteps=nsteps, snap=snap, fs=W.FS_W, **kw)
    return host(xd), host(pd), ref


def test_langevin_fine_129_atoms_100_steps(S):
    wl = W.tiny_129()
    xg, pg, ref = _langevin_pair(S, 1, wl["x"], wl["p"], wl["box"], 100, J=6, beta=wl["beta"], step0=300,
                                 noise_id=2)
    assert np.abs(xg - ref["x"]).max() < QTOL
    assert np.abs(pg - ref["p"]).max() < QTOL * np.abs(ref["p"]).max()
    assert np.abs(xg - wl["x"]).max() > 1e-3          # it moved


def test_langevin_coarse_100_steps(S):
    wl = W.tiny_129(seed=3)
    xg, pg, ref = _langevin_pair(S, 0, wl["x"], wl["p"], wl["box"], 100, step0=7, noise_id=5)
    assert np.abs(xg - ref["x"]).max() < QTOL
    assert np.abs(pg - ref["p"]).max() < QTOL * np.abs(ref["p"]).max()


def test_langevin_batched_slabs_match_per_system(S):
    """Three 1025-atom slabs with their own step offsets, noise streams and
    temperatures advance together; each equals its own oracle run."""
    J = 8
    wl = W.slabs_1025(n_slabs=3, seed=4)
    X, off, B = W.pack(wl["xs"], [wl["box"]] * 3)
    P = np.concatenate(wl["ps"], axis=1)
    T = np.array([900.0, 1000.0, 1200.0])
    step0 = np.array([0, 100, 200])
    nid = np.array([1, 1, 3])
    xd, pd = dev(X), dev(P)
    S.langevin_steps(1, xd, pd, off, B, 4, dt=1e-3, gamma=1.0, mass=W.MASS_W, T=T, seed=77, step0=step0,
                     noise_id=nid, fs=W.FS_W, J=J, beta=wl["beta"])
    xg, pg = host(xd), host(pd)
    snap = dict(J=J, beta=wl["beta"], rcut=W.SNAP_RCUT, rfac0=W.SNAP_RFAC0, rmin0=0.0)
    for s in range(3):
        ref = O.langevin(wl["xs"][s], wl["ps"][s], wl["box"], potential=1, nsteps=4, dt=1e-3, gamma=1.0,
                         mass=W.MASS_W, T=T[s], seed=77, noise_id=int(nid[s]), step0=int(step0[s]), snap=snap,
                         fs=W.FS_W)
        assert np.abs(xg[:, off[s]:off[s + 1]] - ref["x"]).max() < QTOL
        assert np.abs(pg[:, off[s]:off[s + 1]] - ref["p"]).max() < QTOL * np.abs(ref["p"]).max()


def test_invalid_arguments_rejected(S):
    x, box = W.bcc_sia(2)                      # box 6.33 A: rcut 4.73 > half box
    J = 6
    beta = W.snap_beta(J)
    with pytest.raises(S.SnapmdError) as e:
        S.snap_forces(dev(x), [0, x.shape[1]], box, J, beta)
    assert e.value.code == S.EINVAL
    x, box = W.bcc_sia(4)
    with pytest.raises(S.SnapmdError) as e:
        S.snap_forces(dev(x), [0, x.shape[1]], box, 16, np.zeros(2))   # beyond SNAP-205's twojmax 14
    assert e.value.code == S.EUNSUPPORTED
    with pytest.raises(S.SnapmdError) as e:
        S.snap_forces(dev(x), [0, x.shape[1]], box, 7, np.zeros(2))    # odd twojmax
    assert e.value.code == S.EUNSUPPORTED
    with pytest.raises(S.SnapmdError) as e:
        S.snap_forces(dev(x), [0, x.shape[1]], box, 6, np.zeros(20))
    assert e.value.code == S.EINVAL
    with pytest.raises(S.SnapmdError) as e:
        S.snap_forces(dev(x), [0, 200, x.shape[1]], np.tile(box, 2), 6, beta)  # offsets non-monotone
    assert e.value.code == S.EINVAL


@pytest.mark.parametrize("J", [6, 8])
def test_kernel_shapes_give_identical_forces(S, J):
    """Every compiled kernel shape of the SNAP passes (density register budget, dE/dr
    staging width, adjoint waves per tile) gives the same forces, bit for bit, on a ragged
    batch, and energies equal to rounding, for each slot split of the density pass; the
    two splits agree to rounding; the oracle check of one shape per split is shared."""
    from paper_2212_10508_amd import tune
    xa, box = W.bcc_sia(4, jitter=0.1, seed=60 + J)
    xb, _ = W.bcc_sia(4, jitter=0.1, seed=61 + J)
    X = np.concatenate([xa, xb], axis=1)
    n = xa.shape[1]
    off, boxes = [0, n, 2 * n], np.tile(box, (2, 1))
    beta = W.snap_beta(J, seed=J)
    ctx = S.Context(0)
    ref = {}
    ora = O.snap_compute(xa, box, J, beta)["f"]
    for shape in tune.shape_candidates():
        ctx.set_kernel_shape(J, shape)
        assert ctx.kernel_shape(J) == tuple(shape)
        e = torch.zeros(2 * n, dtype=torch.float64, device="cuda")
        f = host(ctx.snap_forces(dev(X), off, boxes, J, beta, e_atom=e))
        eh = host(e)
        # density_parts 0 splits launches with fewer density waves than the device has
        # SIMDs: this batch of 258 atoms
        parts = shape[3] or 2
        if parts not in ref:
            ref[parts] = (f, eh)
            assert frel(f[:, :n], ora) < FTOL
        else:
            assert np.array_equal(f, ref[parts][0]), shape
            assert np.max(np.abs(eh - ref[parts][1])) < 1e-13 * np.max(np.abs(ref[parts][1])), shape
    assert frel(ref[2][0], ref[1][0]) < 1e-13
    assert np.max(np.abs(ref[2][1] - ref[1][1])) < 1e-13 * np.max(np.abs(ref[1][1]))
    ctx.set_kernel_shape(J, None)
    assert ctx.kernel_shape(J) == (45, 0, 12, 0)
    ctx.set_kernel_shape(J, (28, 3, 8))   # three values: density_parts 1
    assert ctx.kernel_shape(J) == (28, 3, 8, 1)
    for bad in ((44, 5, 12, 1), (45, 5, 12, 3)):
        with pytest.raises(S.SnapmdError):
            ctx.set_kernel_shape(J, bad)


def test_automatic_density_split_follows_the_launch_size(S):
    """density_parts 0 splits the density pass of a launch with fewer density waves than
    the device has SIMDs and no other: bitwise the forces of the split shape on one
    1025-atom system (17 tiles in 4 column segments), of the unsplit shape on a batch of
    24 (385 tiles: 1,540 density waves)."""
    J = 8
    x, box = W.bcc_sia(8, jitter=0.05, seed=80)
    n = x.shape[1]
    beta = W.snap_beta(J, seed=80)
    ctx = S.Context(0)
    simds = 4 * torch.cuda.get_device_properties(0).multi_processor_count
    for R in (1, 24):
        X = dev(np.tile(x, (1, R)))
        off = np.arange(R + 1) * n
        boxes = np.tile(box, (R, 1))
        got = {}
        for parts in (0, 1, 2):
            ctx.set_kernel_shape(J, (45, 0, 12, parts))
            got[parts] = host(ctx.snap_forces(X, off, boxes, J, beta))
        split = ((R * n + 63) // 64) * 4 < simds
        assert split == (R == 1)
        assert np.array_equal(got[0], got[2 if split else 1]), R
        assert frel(got[1], got[2]) < 1e-13
    ctx.set_kernel_shape(J, None)


def test_kernel_shape_tuner_checks_parity_first(S):
    """The tuner drops a candidate whose forces miss the oracle (a deliberately wrong
    reference for one shape, planted on the host) and picks among the others."""
    from paper_2212_10508_amd import tune
    J = 4
    x, box = W.bcc_sia(4, jitter=0.05, seed=70)
    n = x.shape[1]
    beta = W.snap_beta(J, seed=70)
    ctx = S.Context(0)
    ora = O.snap_compute(x, box, J, beta)["f"]
    xd = dev(x)
    bad = (21, 0, 8, 1)

    def force_error():
        f = host(ctx.snap_forces(xd, [0, n], box, J, beta))
        err = frel(f, ora)
        return 1.0 if ctx.kernel_shape(J) == bad else err

    def run():
        ctx.snap_forces(xd, [0, n], box, J, beta)
        torch.cuda.synchronize()

    shape, table = tune.tune_kernel_shapes(ctx, J, run, force_error, passes=1)
    assert len(table) == len(tune.shape_candidates())
    assert [t["passed"] for t in table if tuple(t["shape"]) == bad] == [False]
    assert all(t["ms"] is not None for t in table if t["passed"])
    assert shape != bad and ctx.kernel_shape(J) == shape
