"""Interstitial analysis of the oracle, written from the definitions (brute force).

TEST INFRASTRUCTURE ONLY (tests, smoke check and CPU-baseline leg of the benchmark).

* Wigner-Seitz site of an atom: the nearest site of the perfect bcc lattice (cube
  corners (i, j, k) a and centres (i + 1/2, j + 1/2, k + 1/2) a of an n x n x n periodic
  box), found by measuring the minimum-image distance to every site.  Site numbering:
  2 (i n^2 + j n + k) + b, b = 0 corner, 1 centre (the library's convention, fixed by its
  interface).  The site holding two atoms locates the interstitial (the paper follows the
  defect with a Voronoi analysis, section "Numerical results").
* Residence times: the number of consecutive time steps the defect stays on one site.
"""
import numpy as np


def ws_sites(x, n, a):
    """x [3, N] (unwrapped positions), n cells per edge: (site [N], occupancy [2 n^3])."""
    L = n * a
    idx = np.arange(n)
    ci, cj, ck = np.meshgrid(idx, idx, idx, indexing="ij")
    corners = np.stack([ci.ravel(), cj.ravel(), ck.ravel()], axis=1) * a
    sites = np.empty((2 * n ** 3, 3))
    sites[0::2] = corners
    sites[1::2] = corners + 0.5 * a
    N = x.shape[1]
    out = np.empty(N, np.int64)
    for i in range(N):
        d = sites - x[:, i][None, :]
        d -= L * np.round(d / L)
        out[i] = int(np.argmin(np.einsum("ij,ij->i", d, d)))
    occ = np.bincount(out, minlength=2 * n ** 3)
    return out, occ


def residence_times(sites):
    """Run lengths of the defect's site history, in order (the last run is open)."""
    out = []
    i = 0
    while i < len(sites):
        j = i
        while j + 1 < len(sites) and sites[j + 1] == sites[i]:
            j += 1
        out.append(j - i + 1)
        i = j + 1
    return out
