"""Seeded synthetic inputs shared by the library's tests, benchmark and oracle checks.

This module holds no arithmetic of the method itself (no forces, no integrator,
no parareal): it only builds initial conditions and parameters, so that the HIP
path and the CPU oracle can be fed the very same arrays.

Workload recipe (stands in for the paper's tungsten self-interstitial system of its
"MD settings" section; trained SNAP/EAM weights are not available, so a
Finnis-Sinclair tungsten potential plus a SNAP correction with seeded random
coefficients takes their place):

* body-centred cubic tungsten, lattice constant a = 3.1652 A, n^3 cubic cells
  (2 n^3 sites), periodic orthorhombic box of edge n a;
* one <111> dumbbell self-interstitial: lattice site 0 is replaced by two atoms at
  +/- u (1,1,1)/sqrt(3) with u = a sqrt(3)/6 (2 n^3 + 1 atoms: 129, 433, 1025, 16001);
* optional Gaussian jitter N(0, sigma^2) per coordinate from ``default_rng(seed)``;
  positions are wrapped into [0, L) once, at creation;
* momenta p = m v drawn from the Maxwell-Boltzmann law at temperature T;
* SNAP coefficients beta_0 = 0, beta_k ~ N(0, (1e-3)^2) from ``default_rng(seed)``.
"""
import numpy as np

A_W = 3.1652            # bcc tungsten lattice constant (A)
MASS_W = 183.84         # amu
KB = 8.617333262145179e-5        # eV/K
MVV2E = 1.0364269652680506e-4    # eV per amu*A^2/ps^2

# Finnis-Sinclair tungsten (Finnis & Sinclair 1984)
FS_W = dict(A=1.896373, d=4.400224, c=3.25, c0=47.1346499, c1=-33.7665655, c2=6.2541999)

# SNAP hyper-parameters (single element, unit neighbour weight, self term on)
SNAP_RCUT = 4.73
SNAP_RFAC0 = 0.99363
SNAP_RMIN0 = 0.0


def snap_ncoeff(J):
    """Number of bispectrum components for twojmax J (canonical index triples)."""
    K = 0
    for n1 in range(J + 1):
        for n2 in range(n1 + 1):
            for n in range(n1 - n2, min(J, n1 + n2) + 1, 2):
                if n >= n1:
                    K += 1
    return K


def bcc_sia(ncell, a=A_W, jitter=0.0, seed=0, interstitial=True):
    """Positions float64[3, N] and box float64[3] of a bcc supercell (+ dumbbell)."""
    base = np.array([[0.0, 0.0, 0.0], [0.5, 0.5, 0.5]])
    cells = np.array([[i, j, k] for i in range(ncell) for j in range(ncell) for k in range(ncell)],
                     dtype=np.float64)
    sites = (cells[:, None, :] + base[None, :, :]).reshape(-1, 3) * a
    if interstitial:
        u = a * np.sqrt(3.0) / 6.0
        e = np.ones(3) / np.sqrt(3.0)
        sites = np.concatenate([sites[1:], (sites[0] + u * e)[None], (sites[0] - u * e)[None]])
    L = ncell * a
    if jitter > 0:
        rng = np.random.default_rng(seed)
        sites = sites + rng.normal(0.0, jitter, size=sites.shape)
    sites = np.mod(sites, L)
    return np.ascontiguousarray(sites.T), np.array([L, L, L])


def snap_beta(J, seed=0, scale=1e-3):
    """beta[0] = 0 and beta[1..K] ~ N(0, scale^2) in canonical-triple order."""
    K = snap_ncoeff(J)
    return np.concatenate([[0.0], np.random.default_rng(seed).normal(0.0, scale, K)])


def maxwell_momenta(N, T, mass=MASS_W, seed=0):
    """p = m v with each component ~ N(0, m kB T) (expressed in amu*A/ps)."""
    sd = np.sqrt(mass * KB * T / MVV2E)
    return np.ascontiguousarray(np.random.default_rng(seed).normal(0.0, sd, size=(3, N)))


# ----------------------------------------------------------------------------
# Named workloads (sizes of the benchmark configurations)
# ----------------------------------------------------------------------------
def tiny_129(seed=0):
    """129 atoms (4x4x4 bcc + dumbbell), twojmax 6, 1000 K, dt 1 fs, gamma 1/ps."""
    x, box = bcc_sia(4, jitter=0.0, seed=seed)
    return dict(x=x, box=box, J=6, beta=snap_beta(6, seed), T=1000.0, dt=1e-3, gamma=1.0,
                mass=MASS_W, p=maxwell_momenta(x.shape[1], 1000.0, seed=seed), L=100)


def slabs_1025(n_slabs=64, seed=1, jitter=0.05, J=8):
    """1025 atoms (8x8x8 bcc + dumbbell), twojmax 8, one initial state per slab
    (each slab starts from its own jittered copy: stands in for the states q_n)."""
    xs, ps = [], []
    for s in range(n_slabs):
        x, box = bcc_sia(8, jitter=jitter, seed=seed * 100003 + s)
        xs.append(x)
        ps.append(maxwell_momenta(x.shape[1], 1000.0, seed=seed * 100003 + s))
    return dict(xs=xs, ps=ps, box=box, J=J, beta=snap_beta(J, seed), T=1000.0, dt=1e-3,
                gamma=1.0, mass=MASS_W, L=100)


def replicas_mixed(n_rep=256, seed=2, jitter=0.05, J=8):
    """Replica r has [129, 433, 1025][r mod 3] atoms; T_r ~ U(600, 1500) K."""
    sizes = [4, 6, 8]
    T = np.random.default_rng(seed).uniform(600.0, 1500.0, n_rep)
    xs, ps, boxes = [], [], []
    for r in range(n_rep):
        x, box = bcc_sia(sizes[r % 3], jitter=jitter, seed=seed * 100003 + r)
        xs.append(x)
        boxes.append(box)
        ps.append(maxwell_momenta(x.shape[1], T[r], seed=seed * 100003 + r))
    return dict(xs=xs, ps=ps, boxes=boxes, T=T, J=J, beta=snap_beta(J, seed), dt=1e-3,
                gamma=1.0, mass=MASS_W)


def pack(xs, boxes):
    """Concatenate per-system SoA arrays into one batch: (x[3, Ntot], offset, box[n_sys, 3])."""
    sizes = [x.shape[1] for x in xs]
    off = np.zeros(len(xs) + 1, np.int32)
    off[1:] = np.cumsum(sizes)
    X = np.ascontiguousarray(np.concatenate(xs, axis=1))
    B = np.ascontiguousarray(np.array(boxes, dtype=np.float64).reshape(len(xs), 3))
    return X, off, B
