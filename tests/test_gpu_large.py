"""Full-size workloads on the GPU: cell-list neighbour search (systems of several
thousand atoms), the 16001-atom slab size, the host-driven coarse sweep used for
systems too large for the LDS sweep, and the 256-replica mixed-size batch."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import oracle as O
from paper_2212_10508_amd import workloads as W

pytestmark = pytest.mark.gpu

FTOL = 1e-10


@pytest.fixture(scope="module")
def S():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2212_10508_amd import snapmd
    return snapmd


def dev(a):
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")


def frel(f, ref):
    return np.max(np.linalg.norm(f - ref, axis=0)) / np.max(np.linalg.norm(ref, axis=0))


@pytest.mark.parametrize("ncell", [15, 20])
def test_cell_list_forces_match_oracle(S, ncell):
    """6751 and 16001 atoms (the 16001-atom slab of the scale workload): cell-list
    neighbour search, FS + SNAP twojmax 8 forces against the oracle on every atom."""
    x, box = W.bcc_sia(ncell, jitter=0.05, seed=ncell)
    J = 8
    beta = W.snap_beta(J, seed=5)
    N = x.shape[1]
    xd = dev(x)
    f = S.eam_forces(xd, [0, N], box, W.FS_W)
    S.snap_forces(xd, [0, N], box, J, beta, f=f, accumulate=True)
    ref = O.snap_compute(x, box, J, beta)["f"] + O.fs_compute(x, box, W.FS_W)["f"]
    assert frel(f.cpu().numpy(), ref) < FTOL


def test_replica_batch_256_mixed_sizes_sampled(S):
    """256 replicas of 129/433/1025 atoms with their own temperatures advance together
    (two BAOAB steps); sampled replicas equal their own oracle runs."""
    J = 8
    wl = W.replicas_mixed(n_rep=256, seed=2)
    X, off, B = W.pack(wl["xs"], wl["boxes"])
    P = np.concatenate(wl["ps"], axis=1)
    nid = np.arange(256)
    xd, pd = dev(X), dev(P)
    S.langevin_steps(1, xd, pd, off, B, 2, dt=1e-3, gamma=1.0, mass=W.MASS_W, T=wl["T"], seed=8, step0=0,
                     noise_id=nid, fs=W.FS_W, J=J, beta=wl["beta"])
    xg, pg = xd.cpu().numpy(), pd.cpu().numpy()
    snap = dict(J=J, beta=wl["beta"], rcut=W.SNAP_RCUT, rfac0=W.SNAP_RFAC0, rmin0=0.0)
    for r in (0, 1, 2, 128, 255):
        ref = O.langevin(wl["xs"][r], wl["ps"][r], wl["boxes"][r], potential=1, nsteps=2, dt=1e-3, gamma=1.0,
                         mass=W.MASS_W, T=wl["T"][r], seed=8, noise_id=r, step0=0, snap=snap, fs=W.FS_W)
        assert np.abs(xg[:, off[r]:off[r + 1]] - ref["x"]).max() < 1e-8
        assert np.abs(pg[:, off[r]:off[r + 1]] - ref["p"]).max() < 1e-8 * np.abs(ref["p"]).max()


def test_host_driven_sweep_16001_atoms(S):
    """16001 atoms take the host-driven sweep: window initialisation equals slab-by-slab
    coarse propagation, and after k corrected iterations slabs 0..k equal the
    sequential fine trajectory."""
    from paper_2212_10508_amd import parareal as PR
    x, box = W.bcc_sia(20, jitter=0.05, seed=3)
    n = x.shape[1]
    p = W.maxwell_momenta(n, 1000.0, seed=3)
    J, N, L = 2, 3, 3
    beta = W.snap_beta(J, seed=3, scale=2e-2)
    kw = dict(dt=1e-3, gamma=1.0, mass=W.MASS_W, T=1000.0, seed=5, noise_id=2, fs=W.FS_W, J=J, beta=beta)
    ctx = S.context()
    q = torch.zeros((N + 1, 3, n), dtype=torch.float64, device="cuda")
    pp, qp, ppv = torch.zeros_like(q), torch.zeros_like(q), torch.zeros_like(q)
    q[0], pp[0] = dev(x), dev(p)
    ctx.parareal_iterate(None, None, q, pp, box, L, 0, N, 1e100, **kw)
    xc, pc = dev(x), dev(p)
    for s in range(N):
        ctx.langevin_steps(S.POT_FS, xc, pc, [0, n], box, L, step0=s * L, dt=1e-3, gamma=1.0, mass=W.MASS_W,
                           T=1000.0, seed=5, noise_id=2, fs=W.FS_W)
        assert torch.max(torch.abs(q[s + 1] - xc)).item() < 1e-9
    qs, _ = PR.sequential_fine(ctx, dev(x), dev(p), box, N, L, **kw)
    scale = torch.max(torch.abs(qs)).item()
    for k in range(1, N + 1):
        ctx.parareal_iterate(qp, ppv, q, pp, box, L, 0, N, 1e100, **kw)
        err = [torch.max(torch.abs(q[m] - qs[m])).item() for m in range(N + 1)]
        assert max(err[:k + 1]) < 1e-12 * scale, (k, err)
