"""twojmax 10, 12 and 14 (the paper's SNAP-92, SNAP-141 and SNAP-205 sizes, Table
"tabl:cost") through the C ABI against the CPU oracle: forces, per-atom energies and
bispectrum on a jittered 129-atom system and a ragged batch, and a short trajectory
under shared noise.  Tolerances as in test_gpu_parity.py."""
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


@pytest.mark.parametrize("J", [10, 12, 14])
def test_snap_forces_energy_bispectrum_large_twojmax(S, J):
    x, box = W.bcc_sia(4, jitter=0.1, seed=40 + J)
    beta = W.snap_beta(J, seed=J)
    beta[0] = -0.25
    print("twojmax %d: %d coefficients, oracle ..." % (J, len(beta) - 1), flush=True)
    ref = O.snap_compute(x, box, J, beta)
    N = x.shape[1]
    ctx = S.context()
    e = torch.zeros(N, dtype=torch.float64, device="cuda")
    f = ctx.snap_forces(dev(x), [0, N], box, J, beta, e_atom=e)
    fg, eg = host(f), host(e)
    assert frel(fg, ref["f"]) < FTOL
    assert np.max(np.abs(eg - ref["e_atom"])) < ETOL * np.max(np.abs(ref["e_atom"]))
    assert np.abs(fg.sum(axis=1)).max() < 1e-11 * np.abs(fg).max() * np.sqrt(N)
    B = host(ctx.bispectrum(dev(x), [0, N], box, J, beta)).T
    assert B.shape == ref["B"].shape
    assert np.max(np.abs(B - ref["B"]) / np.max(np.abs(ref["B"]), axis=0)) < BTOL


def test_ragged_batch_twojmax_10(S):
    """Systems of 129 atoms, none and 129 atoms again (another state) in one call."""
    J = 10
    beta = W.snap_beta(J, seed=5)
    xa, box = W.bcc_sia(4, jitter=0.1, seed=51)
    xb, _ = W.bcc_sia(4, jitter=0.15, seed=52)
    X = np.concatenate([xa, xb], axis=1)
    n = xa.shape[1]
    off = [0, n, n, 2 * n]
    boxes = np.tile(box, (3, 1))
    f = host(S.context().snap_forces(dev(X), off, boxes, J, beta))
    for k, x in enumerate((xa, xb)):
        ref = O.snap_compute(x, box, J, beta)["f"]
        assert frel(f[:, k * n:(k + 1) * n], ref) < FTOL


def test_langevin_twojmax_10_matches_oracle(S):
    """Ten BAOAB steps on FS + SNAP at twojmax 10, 129 atoms, shared noise."""
    J = 10
    x, box = W.bcc_sia(4, jitter=0.05, seed=53)
    p = W.maxwell_momenta(x.shape[1], 1000.0, seed=53)
    beta = W.snap_beta(J, seed=53, scale=1e-3)
    kw = dict(dt=1e-3, gamma=1.0, mass=W.MASS_W, T=1000.0, seed=7, noise_id=2, step0=30)
    n = x.shape[1]
    xd, pd = dev(x), dev(p)
    S.langevin_steps(S.POT_FS_SNAP, xd, pd, [0, n], box, 10, fs=W.FS_W, J=J, beta=beta, **kw)
    ref = O.langevin(x, p, box, potential=O.POT_FS_SNAP, nsteps=10, fs=W.FS_W,
                     snap=dict(J=J, beta=beta, rcut=W.SNAP_RCUT, rfac0=W.SNAP_RFAC0, rmin0=0.0), **kw)
    assert np.abs(host(xd) - ref["x"]).max() < QTOL
    assert np.abs(host(pd) - ref["p"]).max() < QTOL * np.abs(ref["p"]).max()


def test_twojmax_limits(S):
    """twojmax 16 is refused (SNAPMD_EUNSUPPORTED) and the coefficient gradient stays at
    twojmax <= 8; neither launches anything."""
    x, box = W.bcc_sia(4, seed=1)
    n = x.shape[1]
    with pytest.raises(S.SnapmdError) as e:
        S.context().snap_forces(dev(x), [0, n], box, 16, np.zeros(2))
    assert e.value.code == S.EUNSUPPORTED
    with pytest.raises(S.SnapmdError) as e:
        S.context().snap_beta_grad(dev(x), dev(np.zeros((3, n))), [0, n], box, 10, W.snap_beta(10, seed=1))
    assert e.value.code == S.EUNSUPPORTED
