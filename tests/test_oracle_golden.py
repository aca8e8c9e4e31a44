"""Pins of the oracle against numbers the paper prints (fixtures in tests/golden/, each
with its citation).

* The SNAP family SNAP-6 ... SNAP-205 (Section "MD settings", Table "tabl:cost") is named
  by its number of features; the oracle's enumeration of canonical bispectrum triples
  plus the constant term reproduces all seven names for twojmax 2 .. 14.  A wrong
  selection rule (j >= j1 dropped, parity ignored, j2 > j1 allowed) changes them.
* The uncorrected modified BBK scheme equilibrates at beta^-1 (1 - 1/(2L)): the paper
  prints 285 for L = 10, beta^-1 = 300 (Appendix "Stationary state of the kinetic
  temperature"); the oracle's scheme, at the appendix's time step 0.5 fs and
  gamma^-1 = 1 ps, must reach it up to its O(gamma dt) remainder."""
import os

import numpy as np

from oracle import defn
from oracle import oracle as O
from paper_2212_10508_amd import workloads as W

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _rows(name):
    out = []
    for line in open(os.path.join(GOLDEN, name)):
        line = line.split("#", 1)[0].split()
        if line:
            out.append([float(v) for v in line])
    return out


def test_snap_feature_counts_match_the_paper():
    rows = _rows("snap_feature_counts.txt")
    assert len(rows) == 7
    for J, feat in rows:
        J = int(J)
        assert len(defn.canonical_triples(J)) + 1 == int(feat), J
        if J <= 8:
            assert O.ncoeff(J) + 1 == int(feat), J


def _k_eq_uncorrected(L, dt, gamma):
    """Fixed point of Var p_L = a_L^2 Var p_0 + sum_j c_Lj^2 for the oracle's scheme with
    no forces, as a multiple of m kB T / mvv2e (the oracle's response to unit inputs)."""
    N = L + 2
    x = np.zeros((3, N))
    p = np.zeros((3, N))
    p[0, 0] = 1.0
    G = np.zeros((L + 1, 3, N))
    for j in range(L + 1):
        G[j, 0, j + 1] = 1.0
    T = 1000.0
    r = O.bbk(x, p, np.array([1e4] * 3), potential=O.POT_NONE, nsteps=L, dt=dt, gamma=gamma,
              mass=W.MASS_W, T=T, cT=(1.0, 1.0), G=G, want_traj=True)
    tp = r["traj_p"][:, 0, :]
    aL, cL = tp[L, 0], tp[L, 1:]
    kT = W.KB * T / W.MVV2E
    return np.sum(cL ** 2) / (1.0 - aL ** 2) / (W.MASS_W * kT)


def test_bbk_kinetic_temperature_printed_value():
    for L, tinv, k_printed, dt, gamma in _rows("bbk_kinetic_temperature.txt"):
        k = tinv * _k_eq_uncorrected(int(L), dt, gamma)
        assert abs(k - k_printed) < 0.5, (L, k, k_printed)
