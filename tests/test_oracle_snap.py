"""Pins of the oracle's SNAP and Finnis-Sinclair arithmetic against facts fixed
outside the oracle: exact CG values from sympy, group-theory identities of the
Wigner-D matrices, closed forms of bispectrum components, symmetry invariances,
Euler's theorem for the cubic energy, finite differences, and the published
Finnis-Sinclair cohesive energy of tungsten."""
import numpy as np
import pytest

from oracle import defn
from oracle import oracle as O
from paper_2212_10508_amd import workloads as W

RCUT, RFAC0 = W.SNAP_RCUT, W.SNAP_RFAC0


def rand_su2(rng):
    q = rng.normal(size=4)
    q /= np.linalg.norm(q)
    return complex(q[0], q[1]), complex(q[2], q[3])


def su2(a, b):
    return np.array([[a, b], [-np.conj(b), np.conj(a)]])


def cluster(rng, m, rmin=1.8, rmax=4.6, L=60.0):
    """A centre atom at the box centre plus m neighbours in a large periodic box."""
    c = np.full(3, L / 2)
    d = rng.normal(size=(m, 3))
    d *= (rng.uniform(rmin, rmax, m) / np.linalg.norm(d, axis=1))[:, None]
    pos = np.vstack([c, c + d])
    return np.ascontiguousarray(pos.T), np.array([L, L, L]), d


# ---------------------------------------------------------------------------
# Clebsch-Gordan
# ---------------------------------------------------------------------------
def test_cg_matches_sympy_exact():
    from sympy import Rational, N
    from sympy.physics.wigner import clebsch_gordan
    rng = np.random.default_rng(0)
    checked = 0
    for n1 in range(9):
        for n2 in range(n1 + 1):
            for n in range(n1 - n2, n1 + n2 + 1, 2):
                combos = [(k1, k2) for k1 in range(n1 + 1) for k2 in range(n2 + 1)
                          if 0 <= k1 + k2 - (n1 + n2 - n) // 2 <= n]
                if n1 > 5:
                    combos = [combos[i] for i in rng.choice(len(combos), min(4, len(combos)),
                                                            replace=False)]
                for k1, k2 in combos:
                    k = k1 + k2 - (n1 + n2 - n) // 2
                    ref = float(N(clebsch_gordan(Rational(n1, 2), Rational(n2, 2), Rational(n, 2),
                                                 Rational(2 * k1 - n1, 2), Rational(2 * k2 - n2, 2),
                                                 Rational(2 * k - n, 2)), 30))
                    assert abs(defn.cg(n1, k1, n2, k2, n, k) - ref) < 1e-15
                    assert abs(O.cg(n1, k1, n2, k2, n, k) - ref) < 1e-14
                    checked += 1
    assert checked > 500


def test_cg_orthogonality():
    for n1, n2 in [(3, 2), (4, 4), (8, 6)]:
        for n in range(abs(n1 - n2), n1 + n2 + 1, 2):
            for np_ in range(abs(n1 - n2), n1 + n2 + 1, 2):
                for k in range(n + 1):
                    kp = k + (np_ - n) // 2
                    if not 0 <= kp <= np_:
                        continue
                    s = 0.0
                    for k1 in range(n1 + 1):
                        k2 = k - k1 + (n1 + n2 - n) // 2
                        k2p = kp - k1 + (n1 + n2 - np_) // 2
                        if 0 <= k2 <= n2 and k2 == k2p:
                            s += O.cg(n1, k1, n2, k2, n, k) * O.cg(n1, k1, n2, k2, np_, kp)
                    assert abs(s - (1.0 if n == np_ else 0.0)) < 1e-13


# ---------------------------------------------------------------------------
# Wigner-D
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("n", [0, 1, 2, 5, 8])
def test_wigner_group_identities(n):
    rng = np.random.default_rng(n)
    a1, b1 = rand_su2(rng)
    a2, b2 = rand_su2(rng)
    g = su2(a1, b1) @ su2(a2, b2)
    for D in (defn.wigner_d, O.wigner):
        D1, D2, D12 = D(n, a1, b1), D(n, a2, b2), D(n, g[0, 0], g[0, 1])
        assert np.abs(D1 @ D2 - D12).max() < 1e-13                       # homomorphism
        assert np.abs(D1 @ D1.conj().T - np.eye(n + 1)).max() < 1e-13    # unitarity
        th = np.arccos(a1.real)                                           # character
        assert abs(np.trace(D1) - np.sin((n + 1) * th) / np.sin(th)) < 1e-12
        # mirror symmetry D[n-k, n-l] = (-1)^(k-l) conj(D[k, l])
        for k in range(n + 1):
            for l in range(n + 1):
                assert abs(D1[n - k, n - l] - (-1) ** (k - l) * np.conj(D1[k, l])) < 1e-13
    assert np.abs(O.wigner(n, a1, b1) - defn.wigner_d(n, a1, b1)).max() < 1e-14


@pytest.mark.parametrize("n1,n2", [(1, 1), (3, 2), (4, 4), (6, 3)])
def test_wigner_cg_series(n1, n2):
    """D^{n1} (x) D^{n2} = sum_n C_n D^n C_n^T: pins D and CG conventions together."""
    rng = np.random.default_rng(10 * n1 + n2)
    a, b = rand_su2(rng)
    lhs = np.kron(O.wigner(n1, a, b), O.wigner(n2, a, b))
    rhs = np.zeros_like(lhs)
    for n in range(abs(n1 - n2), n1 + n2 + 1, 2):
        Cm = np.zeros(((n1 + 1) * (n2 + 1), n + 1))
        for k1 in range(n1 + 1):
            for k2 in range(n2 + 1):
                k = k1 + k2 - (n1 + n2 - n) // 2
                if 0 <= k <= n:
                    Cm[k1 * (n2 + 1) + k2, k] = O.cg(n1, k1, n2, k2, n, k)
        rhs += Cm @ O.wigner(n, a, b) @ Cm.T
    assert np.abs(lhs - rhs).max() < 1e-13


# ---------------------------------------------------------------------------
# Bispectrum
# ---------------------------------------------------------------------------
def _chebyshev_u(n, x):
    if abs(abs(x) - 1.0) < 1e-14:
        return (n + 1) * np.sign(x) ** n
    t = np.arccos(np.clip(x, -1.0, 1.0))
    return np.sin((n + 1) * t) / np.sin(t)


def test_bispectrum_closed_form_n0n():
    """B_{n,0,n} = (sum_k w_k) sum_{k,l} w_k w_l U_n(cos alpha_kl) with U_n the Chebyshev
    polynomial of the second kind and alpha_kl the angle between the 4-D unit points
    (z0, x, y, z)/r0 (self = (1,0,0,0), weight 1): independent of D and CG phases."""
    rng = np.random.default_rng(3)
    J = 8
    x, box, d = cluster(rng, 9)
    res = O.snap_compute(x, box, J, np.zeros(W.snap_ncoeff(J) + 1))
    B0 = res["B"][0]
    tri = defn.canonical_triples(J)
    pts, w = [np.array([1.0, 0, 0, 0])], [1.0]
    for rv in d:
        r = np.linalg.norm(rv)
        th = RFAC0 * np.pi * r / RCUT
        z0 = r / np.tan(th)
        r0 = np.hypot(r, z0)
        pts.append(np.array([z0, *rv]) / r0)
        w.append(0.5 * (np.cos(np.pi * r / RCUT) + 1.0))
    for n in range(J + 1):
        ref = sum(w) * sum(w[k] * w[l] * _chebyshev_u(n, pts[k] @ pts[l])
                           for k in range(len(w)) for l in range(len(w)))
        assert abs(B0[tri.index((n, 0, n))] - ref) < 1e-11 * max(1.0, abs(ref))


def test_bispectrum_perfect_lattice_b000():
    """Perfect bcc: B_000 = (1 + sum_k f_c(r_k))^3 over 8 + 6 + 12 shell neighbours."""
    x, box = W.bcc_sia(4, interstitial=False)
    res = O.snap_compute(x, box, 6, np.zeros(W.snap_ncoeff(6) + 1))
    a = W.A_W
    fc = lambda r: 0.5 * (np.cos(np.pi * r / RCUT) + 1.0)
    u0 = 1 + 8 * fc(a * np.sqrt(3) / 2) + 6 * fc(a) + 12 * fc(a * np.sqrt(2))
    assert abs(u0 - 5.5756) < 1e-4
    assert np.abs(res["B"][:, 0] - u0 ** 3).max() < 1e-11


def test_bispectrum_rotation_inversion_invariance():
    rng = np.random.default_rng(4)
    J = 8
    x, box, d = cluster(rng, 10)
    B = O.snap_compute(x, box, J, np.zeros(W.snap_ncoeff(J) + 1))["B"][0]
    Q, _ = np.linalg.qr(rng.normal(size=(3, 3)))
    for R in (Q, -Q):                     # proper and improper
        d2 = d @ R.T
        c = x[:, :1]
        x2 = np.hstack([c, c + d2.T])
        B2 = O.snap_compute(x2, box, J, np.zeros(W.snap_ncoeff(J) + 1))["B"][0]
        assert np.abs(B2 - B).max() < 1e-12 * np.abs(B).max()
    # neighbour permutation and translation
    perm = rng.permutation(len(d))
    x3 = np.hstack([x[:, :1] + 1.234, x[:, :1] + 1.234 + d[perm].T])
    B3 = O.snap_compute(x3, box, J, np.zeros(W.snap_ncoeff(J) + 1))["B"][0]
    assert np.abs(B3 - B).max() < 1e-12 * np.abs(B).max()


def test_bispectrum_cg_symmetry_definition_tier():
    """(n1+1) X_{n1 n2 n} = (n+1) X_{n n2 n1} for X = sum conj(u^n) Z^n_{n1 n2}
    (symmetry of the coupling coefficients under exchange of j and j1)."""
    rng = np.random.default_rng(5)
    J = 4
    _, _, d = cluster(rng, 5)
    u = defn.density(d, J, RCUT)
    for (n1, n2, n) in [(2, 2, 4), (3, 1, 4), (4, 2, 2), (3, 3, 2), (4, 4, 0), (2, 2, 0)]:
        X = np.sum(np.conj(u[n]) * defn.z_block(u, n1, n2, n))
        Xs = np.sum(np.conj(u[n1]) * defn.z_block(u, n, n2, n1))
        assert abs((n1 + 1) * X - (n + 1) * Xs) < 1e-12 * abs(X)
        assert abs(X.imag) < 1e-12 * abs(X)


def test_o1_matches_definition_tier():
    rng = np.random.default_rng(6)
    J = 4
    x, box, d = cluster(rng, 6)
    beta = W.snap_beta(J, seed=6)
    u_ref = defn.density(d, J, RCUT)
    B_ref = defn.bispectrum(u_ref, J)
    Y_ref = defn.adjoint_brute(u_ref, J, beta)
    res = O.snap_compute(x, box, J, beta)
    assert np.abs(res["B"][0] - B_ref).max() < 1e-12 * np.abs(B_ref).max()
    u, y = O.snap_uy(x, box, J, beta)
    for n in range(J + 1):
        assert np.abs(u[n][0] - u_ref[n]).max() < 1e-13
        assert np.abs(y[n][0] - Y_ref[n]).max() < 1e-15 + 1e-12 * np.abs(Y_ref[n]).max()


def test_euler_identity_adjoint():
    """E is a cubic form in (u, conj u): E - beta0 = Re sum conj(Y) u / 3."""
    x, box = W.bcc_sia(4, jitter=0.1, seed=7)
    J = 6
    beta = W.snap_beta(J, seed=7)
    beta[0] = 0.37
    res = O.snap_compute(x, box, J, beta)
    u, y = O.snap_uy(x, box, J, beta)
    s = sum(np.sum(np.conj(y[n]) * u[n], axis=(1, 2)).real for n in range(J + 1))
    assert np.abs(res["e_atom"] - beta[0] - s / 3).max() < 1e-13


def test_forces_direct_vs_adjoint():
    x, box = W.bcc_sia(4, jitter=0.08, seed=8)
    x = x[:, :]
    J = 4
    beta = W.snap_beta(J, seed=8)
    fa = O.snap_compute(x, box, J, beta, route=0)["f"]
    fd = O.snap_compute(x, box, J, beta, route=1)["f"]
    assert np.abs(fa - fd).max() < 1e-12 * np.abs(fa).max()


@pytest.mark.parametrize("J", [2, 6])
def test_snap_forces_finite_difference_and_net_zero(J):
    x, box = W.bcc_sia(4, jitter=0.1, seed=9)
    beta = W.snap_beta(J, seed=9, scale=1e-2)
    res = O.snap_compute(x, box, J, beta)
    f = res["f"]
    fmax = np.abs(f).max()
    assert np.abs(f.sum(axis=1)).max() < 1e-12 * fmax * x.shape[1] ** 0.5
    rng = np.random.default_rng(9)
    h = 1e-5
    for _ in range(4):
        i, al = int(rng.integers(x.shape[1])), int(rng.integers(3))
        xp, xm = x.copy(), x.copy()
        xp[al, i] += h
        xm[al, i] -= h
        ep = O.snap_compute(xp, box, J, beta)["E"]
        em = O.snap_compute(xm, box, J, beta)["E"]
        assert abs(-(ep - em) / (2 * h) - f[al, i]) < 1e-7 * fmax


def test_snap_perfect_lattice_zero_force():
    x, box = W.bcc_sia(4, interstitial=False)
    J = 6
    beta = W.snap_beta(J, seed=10, scale=1e-2)
    f = O.snap_compute(x, box, J, beta)["f"]
    assert np.abs(f).max() < 1e-12


# ---------------------------------------------------------------------------
# Finnis-Sinclair
# ---------------------------------------------------------------------------
def test_fs_cohesive_energy_and_lattice_forces():
    """Perfect bcc W at a = 3.1652 A: E/atom = -8.9000024 eV (Finnis-Sinclair fit target)."""
    x, box = W.bcc_sia(4, interstitial=False)
    r = O.fs_compute(x, box, W.FS_W)
    assert abs(r["E"] / x.shape[1] - (-8.9000024)) < 5e-7
    assert np.abs(r["f"]).max() < 1e-12


def test_fs_forces_finite_difference_and_net_zero():
    x, box = W.bcc_sia(4, jitter=0.1, seed=11)
    r = O.fs_compute(x, box, W.FS_W)
    f = r["f"]
    assert np.abs(f.sum(axis=1)).max() < 1e-11
    rng = np.random.default_rng(11)
    h = 1e-5
    for _ in range(6):
        i, al = int(rng.integers(x.shape[1])), int(rng.integers(3))
        xp, xm = x.copy(), x.copy()
        xp[al, i] += h
        xm[al, i] -= h
        fd = -(O.fs_compute(xp, box, W.FS_W)["E"] - O.fs_compute(xm, box, W.FS_W)["E"]) / (2 * h)
        assert abs(fd - f[al, i]) < 1e-7 * np.abs(f).max()


def test_wigner_d_derivative_is_generator_action():
    """D is a representation of SU(2), so along a path g(t): dD/dt = dD(X) D with
    X = g' g^-1 in su(2), whose action on the rows of a column is three-term:
    dD[k] = X11 (2k - n) D[k] + X21 sqrt((k+1)(n-k)) D[k+1] + X12 sqrt(k(n-k+1)) D[k-1].
    Checked against central differences of the defined D along the SNAP map of a moving
    neighbour (the identity the force pass uses)."""
    rng = np.random.default_rng(3)
    for _ in range(3):
        r = rng.normal(size=3)
        r *= rng.uniform(2.0, 4.5) / np.linalg.norm(r)
        a, b = defn.su2_from_neighbor(r, RCUT, RFAC0, 0.0)
        for al in range(3):
            h = 1e-6
            e = np.zeros(3)
            e[al] = h
            ap, bp = defn.su2_from_neighbor(r + e, RCUT, RFAC0, 0.0)
            am, bm = defn.su2_from_neighbor(r - e, RCUT, RFAC0, 0.0)
            da, db = (ap - am) / (2 * h), (bp - bm) / (2 * h)
            X11 = da * np.conj(a) + db * np.conj(b)
            X12 = db * a - da * b
            X21 = -np.conj(X12)
            assert abs(X11.real) < 1e-9  # su(2): X11 is imaginary
            for n in (1, 4, 8):
                D = defn.wigner_d(n, a, b)
                fd = (defn.wigner_d(n, ap, bp) - defn.wigner_d(n, am, bm)) / (2 * h)
                G = np.zeros_like(D)
                for k in range(n + 1):
                    G[k] = X11 * (2 * k - n) * D[k]
                    if k < n:
                        G[k] += X21 * np.sqrt((k + 1) * (n - k)) * D[k + 1]
                    if k > 0:
                        G[k] += X12 * np.sqrt(k * (n - k + 1)) * D[k - 1]
                assert np.abs(G - fd).max() < 1e-8 * max(1.0, np.abs(fd).max())
