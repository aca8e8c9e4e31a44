"""SNAP coefficient gradients on the GPU (snap_beta_grad through the C ABI and the
autograd Function) against the oracle and against central finite differences."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

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


def _configs(seed, sizes=(4, 6), sigma=0.1):
    parts = [W.bcc_sia(n, jitter=sigma, seed=seed + q) for q, n in enumerate(sizes)]
    X, off, B = W.pack([p[0] for p in parts], [p[1] for p in parts])
    return parts, X, off, B


@pytest.mark.parametrize("J", [6, 8])
def test_dE_dbeta_is_sum_of_bispectrum(S, J):
    parts, X, off, B = _configs(40 + J)
    beta = W.snap_beta(J, seed=J)
    w = np.zeros_like(X)
    dE, gF = S.context().snap_beta_grad(dev(X), dev(w), off, B, J, beta)
    dE = dE.cpu().numpy()
    ref = np.zeros(len(beta))
    ref[0] = X.shape[1]
    for x, box in parts:
        ref[1:] += O.snap_compute(x, box, J, beta)["B"].sum(axis=0)
    assert np.max(np.abs(dE - ref) / np.maximum(np.abs(ref), 1.0)) < 1e-12
    assert np.abs(gF.cpu().numpy()).max() == 0.0


def test_force_jacobian_contraction_matches_oracle(S):
    """sum_i w_i . dF_i/dbeta_k; the oracle's forces at beta = e_k are exactly dF/dbeta_k."""
    J = 6
    parts, X, off, B = _configs(50, sizes=(4,))
    x, box = parts[0]
    rng = np.random.default_rng(3)
    w = rng.normal(size=X.shape)
    beta = W.snap_beta(J, seed=3)
    _, gF = S.context().snap_beta_grad(dev(X), dev(w), off, B, J, beta)
    gF = gF.cpu().numpy()
    K = W.snap_ncoeff(J)
    ref = np.zeros(K + 1)
    for k in range(1, K + 1):
        e = np.zeros(K + 1)
        e[k] = 1.0
        ref[k] = np.sum(w * O.snap_compute(x, box, J, e)["f"])
    assert np.max(np.abs(gF - ref)) < 1e-10 * np.max(np.abs(ref))


def _loss(S, beta_t, x, off, B, J, fref):
    from paper_2212_10508_amd.autograd import snap_energy_forces
    E, F = snap_energy_forces(beta_t, x, off, B, J)
    return ((F - fref) ** 2).sum() / F.numel()


def test_force_matching_loss_gradient(S):
    """Loss (1/3N) sum |F(beta) - F_ref|^2 with F_ref from a teacher beta*: autograd gradient
    against central finite differences (the loss is quadratic in beta) and zero at beta*."""
    J = 8
    parts, X, off, B = _configs(60, sizes=(4, 6, 4))
    x = dev(X)
    teacher = W.snap_beta(J, seed=61)
    fref = S.snap_forces(x, off, B, J, teacher)
    beta0 = W.snap_beta(J, seed=62)
    beta_t = torch.tensor(beta0, dtype=torch.float64, requires_grad=True)
    L = _loss(S, beta_t, x, off, B, J, fref)
    L.backward()
    g = beta_t.grad.numpy()
    h = 1e-5
    for k in (1, 7, 30, 55):
        bp, bm = beta0.copy(), beta0.copy()
        bp[k] += h
        bm[k] -= h
        lp = _loss(S, torch.tensor(bp), x, off, B, J, fref).item()
        lm = _loss(S, torch.tensor(bm), x, off, B, J, fref).item()
        fd = (lp - lm) / (2 * h)
        assert abs(fd - g[k]) < 1e-6 * max(abs(fd), 1e-3) + 1e-12
    assert g[0] == 0.0
    bt = torch.tensor(teacher, dtype=torch.float64, requires_grad=True)
    Lt = _loss(S, bt, x, off, B, J, fref)
    Lt.backward()
    assert Lt.item() < 1e-24 and np.abs(bt.grad.numpy()).max() < 1e-12


def test_energy_gradient_through_autograd(S):
    J = 6
    parts, X, off, B = _configs(70, sizes=(4,))
    from paper_2212_10508_amd.autograd import snap_energy_forces
    beta_t = torch.tensor(W.snap_beta(J, seed=7), dtype=torch.float64, requires_grad=True)
    E, F = snap_energy_forces(beta_t, dev(X), off, B, J)
    E.backward()
    Bref = O.snap_compute(parts[0][0], parts[0][1], J, beta_t.detach().numpy())["B"].sum(axis=0)
    g = beta_t.grad.numpy()
    assert g[0] == X.shape[1]
    assert np.max(np.abs(g[1:] - Bref) / np.maximum(np.abs(Bref), 1.0)) < 1e-12
