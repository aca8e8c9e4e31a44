"""Interstitial analysis on the GPU (snapmd_ws_sites, snapmd_relax through the C ABI)
against the oracle's brute-force definitions, and the defect's site history of converged
parareal against the sequential fine trajectory."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import analysis as OA
from oracle import oracle as O
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


def test_ws_sites_match_oracle_ragged_unwrapped(S):
    parts = [W.bcc_sia(4, jitter=0.15, seed=21), W.bcc_sia(6, jitter=0.15, seed=22),
             W.bcc_sia(3, jitter=0.1, seed=23, interstitial=False)]
    xs = []
    for q, (x, box) in enumerate(parts):  # unwrapped: atoms moved by whole boxes
        shift = np.random.default_rng(q).integers(-3, 4, size=(3, x.shape[1]))
        xs.append(x + shift * box[:, None])
    X, off, B = W.pack(xs, [p[1] for p in parts])
    ctx = S.context()
    site, occ = ctx.ws_sites(dev(X), off, B, W.A_W)
    site, occ = site.cpu().numpy(), occ.cpu().numpy()
    first = 0
    for q, (x, box) in enumerate(parts):
        n = int(round(box[0] / W.A_W))
        ref, rocc = OA.ws_sites(xs[q], n, W.A_W)
        assert np.array_equal(site[off[q]:off[q + 1]] - first, ref)
        assert np.array_equal(occ[first:first + 2 * n ** 3], rocc)
        first += 2 * n ** 3
    from paper_2212_10508_amd import analysis as A
    assert A.interstitial_site(occ[:128]) == 0  # the dumbbell of the first system


def test_ws_sites_rejects_a_box_of_partial_cells(S):
    x, box = W.bcc_sia(4)
    with pytest.raises(S.SnapmdError):
        S.context().ws_sites(dev(x), [0, x.shape[1]], box * 1.01, W.A_W)


def test_relax_reaches_a_force_minimum(S):
    x, box = W.bcc_sia(4, jitter=0.05, seed=24)
    xd = dev(x)
    ctx = S.context()
    n = x.shape[1]
    e0 = torch.zeros(n, dtype=torch.float64, device="cuda")
    ctx.eam_forces(xd, [0, n], box, W.FS_W, e_atom=e0)
    fmax, its = ctx.relax(S.POT_FS, xd, [0, n], box, W.FS_W, max_iter=20000, ftol=1e-4)
    assert fmax < 1e-4 and its > 0
    ref = O.fs_compute(xd.cpu().numpy(), box, W.FS_W)
    assert np.abs(ref["f"]).max() < 1e-4 * 1.01
    assert ref["E"] < e0.sum().item() - 1e-3
    site, occ = ctx.ws_sites(xd, [0, n], box, W.A_W)
    assert np.count_nonzero(occ.cpu().numpy() == 2) == 1  # the dumbbell survives relaxation


def test_defect_history_of_converged_parareal_equals_sequential(S):
    """As the paper's trajectorial test: with a tight convergence threshold the parareal
    trajectory visits the same interstitial sites as the sequential one (here at every slab
    boundary), and the library's residence times equal the oracle's on a per-step record."""
    from paper_2212_10508_amd import analysis as A
    from paper_2212_10508_amd import parareal as PR
    x, box = W.bcc_sia(4, jitter=0.0, seed=25)
    n = x.shape[1]
    J = 4
    beta = W.snap_beta(J, seed=25, scale=2e-2)
    kw = dict(dt=1e-3, gamma=1.0, mass=W.MASS_W, T=2000.0, seed=31, noise_id=0, fs=W.FS_W, J=J, beta=beta)
    ctx = S.context()
    xd, pd = dev(x), dev(W.maxwell_momenta(n, 2000.0, seed=25))
    fmax, _ = A.equilibrate(ctx, xd, pd, box, W.FS_W, J=J, beta=beta, relax_iter=20000, thermal_steps=300,
                            T=2000.0, seed=77)
    assert fmax < 1e-4
    N, L = 6, 40
    qs, _ = PR.sequential_fine(ctx, xd.clone(), pd.clone(), box, N, L, **kw)
    q, _, nad, kc = PR.adaptive_parareal(ctx, xd.clone(), pd.clone(), box, N, L, 1e-10, 1e100, **kw)
    s_seq = [A.interstitial_site(ctx.ws_sites(qs[m].contiguous(), [0, n], box, W.A_W)[1]) for m in range(N + 1)]
    s_par = [A.interstitial_site(ctx.ws_sites(q[m].contiguous(), [0, n], box, W.A_W)[1]) for m in range(N + 1)]
    assert s_seq == s_par and all(s >= 0 for s in s_seq)
    # per-step record of the sequential trajectory
    xr, pr = xd.clone(), pd.clone()
    hist = []
    for step in range(200):
        ctx.langevin_steps(S.POT_FS_SNAP, xr, pr, [0, n], box, 1, step0=step, **kw)
        hist.append(A.interstitial_site(ctx.ws_sites(xr, [0, n], box, W.A_W)[1]))
    assert A.residence_times(hist) == OA.residence_times(hist)
    assert sum(A.residence_times(hist)) == 200


def test_residence_study_reproduces_sequential_histories(S):
    """The statistical study's machinery on two 129-atom replicas: with the sequential runs'
    noise streams and a tight threshold, the parareal trajectories rebuilt step by step from
    their converged slab states (the fine propagation of every slab at once) have the same
    interstitial site after every step as the sequential trajectories, hence the same
    residence times; every step of every replica is accounted for."""
    from paper_2212_10508_amd import analysis as A
    x, box = W.bcc_sia(4, jitter=0.0, seed=5)
    ctx = S.context()
    N, L, R = 4, 25, 2
    r = A.residence_study(ctx, dev(x), box, R=R, N=N, L=L, J=4, beta=W.snap_beta(4, seed=5, scale=2e-2),
                          fs=W.FS_W, T=2000.0, delta_conv=1e-10, thermal_steps=500, seed=3, mass=W.MASS_W,
                          same_noise=True, keep_histories=True)
    hs, hp = r["histories"]["sequential"], r["histories"]["parareal"]
    assert hs.shape == hp.shape == (R, N * L)
    assert np.array_equal(hs, hp)
    assert (hs >= 0).all()                  # the dumbbell is found after every step
    assert r["sequential"]["hops"] == r["parareal"]["hops"]
    for k in range(R):
        assert sum(A.residence_times(list(hs[k]))) == N * L
