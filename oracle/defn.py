"""Definition tier of the oracle: SNAP written straight from its mathematical definition.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import this module;
only tests, the smoke check and the CPU-baseline leg of the benchmark use the oracle.

The paper (Section "MD settings") uses the spectral neighbour analysis potential
(SNAP) of Thompson et al. as its fine force field but prints none of its formulas;
this module restates the published SNAP definition with plain, slow NumPy and exact
rational arithmetic, for tiny inputs:

* Clebsch-Gordan coefficients from Racah's closed formula in exact integers.
* The (n+1)-dimensional irreducible representation of SU(2) (n = 2j) built as
  the action of g = [[a, b], [-conj(b), conj(a)]] on homogeneous polynomials of
  degree n in (u, v), in the orthonormal monomial basis
  e_k = u^k v^(n-k) / sqrt(k! (n-k)!), k = 0..n (m = k - n/2):
  the substitution (u, v) -> (a u - conj(b) v, b u + conj(a) v) sends e_l to
  sum_k D[k, l] e_k.  This is a homomorphism: D(g1 g2) = D(g1) D(g2).
* The SNAP map of a neighbour vector r = (x, y, z) to the 3-sphere:
  theta0 = rfac0 * pi * (r - rmin0) / (rcut - rmin0), z0 = r cot(theta0),
  r0 = r / sin(theta0), a = (z0 - i z) / r0, b = (y - i x) / r0,
  with switching function f_c(r) = (cos(pi (r - rmin0)/(rcut - rmin0)) + 1) / 2.
* Density coefficients u^n = I + sum_k f_c(r_ik) D^n(g(r_ik)).
* Z^n_{n1 n2}[k, l] = sum C^{n k}_{n1 k1, n2 k2} C^{n l}_{n1 l1, n2 l2} u^{n1}[k1, l1] u^{n2}[k2, l2],
  B_{n1 n2 n} = Re sum_{k, l} conj(u^n[k, l]) Z^n_{n1 n2}[k, l] over the canonical
  triples 0 <= n2 <= n1 <= n <= J, n1 - n2 <= n <= n1 + n2, n1 + n2 + n even,
  in lexicographic (n1, n2, n) order.
* E_i = beta_0 + sum_k beta_k B_k.

All indices are 2j-integers (n = 2j); rows k and columns l run over 0..n.
"""
from fractions import Fraction
from functools import lru_cache
from math import factorial, sqrt, pi, cos, sin

import numpy as np


# ----------------------------------------------------------------------------
# Index sets
# ----------------------------------------------------------------------------
def canonical_triples(J):
    """Canonical (n1, n2, n) triples in lexicographic order; their count is K."""
    out = []
    for n1 in range(J + 1):
        for n2 in range(n1 + 1):
            for n in range(n1 - n2, min(J, n1 + n2) + 1, 2):
                if n >= n1:
                    out.append((n1, n2, n))
    return out


# ----------------------------------------------------------------------------
# Clebsch-Gordan coefficients (Racah's formula), 2j-integer arguments
# ----------------------------------------------------------------------------
@lru_cache(maxsize=None)
def cg_exact_sq(n1, k1, n2, k2, n, k):
    """Return (sign, Fraction) with C = sign * sqrt(Fraction) for
    C^{j m}_{j1 m1, j2 m2}, j = n/2, m = k - n/2 (likewise for 1, 2)."""
    # m in 2j units: 2m = 2k - n
    tm1, tm2, tm = 2 * k1 - n1, 2 * k2 - n2, 2 * k - n
    if tm1 + tm2 != tm:
        return 0, Fraction(0)
    if n < abs(n1 - n2) or n > n1 + n2 or (n1 + n2 + n) % 2:
        return 0, Fraction(0)
    if not (0 <= k1 <= n1 and 0 <= k2 <= n2 and 0 <= k <= n):
        return 0, Fraction(0)
    h = lambda t: t // 2  # all combinations below are even
    a = h(n + n1 - n2)
    b = h(n - n1 + n2)
    c = h(n1 + n2 - n)
    d = h(n1 + n2 + n) + 1
    pref = Fraction((n + 1) * factorial(a) * factorial(b) * factorial(c), factorial(d))
    pref *= (factorial(h(n + tm)) * factorial(h(n - tm)) * factorial(h(n1 - tm1)) *
             factorial(h(n1 + tm1)) * factorial(h(n2 - tm2)) * factorial(h(n2 + tm2)))
    s = Fraction(0)
    for t in range(0, c + 1):
        args = (t, c - t, h(n1 - tm1) - t, h(n2 + tm2) - t,
                h(n - n2 + tm1) + t, h(n - n1 - tm2) + t)
        if min(args) < 0:
            continue
        den = 1
        for x in args:
            den *= factorial(x)
        s += Fraction((-1) ** t, den)
    if s == 0:
        return 0, Fraction(0)
    sign = 1 if s > 0 else -1
    return sign, pref * s * s


def cg(n1, k1, n2, k2, n, k):
    sign, sq = cg_exact_sq(n1, k1, n2, k2, n, k)
    if sign == 0:
        return 0.0
    return sign * sqrt(sq.numerator / sq.denominator)


# ----------------------------------------------------------------------------
# Wigner-D by the polynomial (symmetric power) construction
# ----------------------------------------------------------------------------
def _poly_mul(p, q):
    """Multiply polynomials in (u, v) stored as {power_of_u: coeff} (homogeneous)."""
    out = {}
    for i, x in p.items():
        for j, y in q.items():
            out[i + j] = out.get(i + j, 0) + x * y
    return out


def wigner_d(n, a, b):
    """(n+1)x(n+1) matrix D[k, l] of g = [[a, b], [-conj(b), conj(a)]]."""
    up = {1: a, 0: -np.conj(b)}       # u' = a u - conj(b) v   ({power of u: coeff})
    vp = {1: b, 0: np.conj(a)}        # v' = b u + conj(a) v
    D = np.zeros((n + 1, n + 1), dtype=complex)
    for l in range(n + 1):
        p = {0: 1.0 + 0j}
        for _ in range(l):
            p = _poly_mul(p, up)
        for _ in range(n - l):
            p = _poly_mul(p, vp)
        for k, coef in p.items():
            D[k, l] = coef * sqrt(factorial(k) * factorial(n - k) /
                                  (factorial(l) * factorial(n - l)))
    return D


def su2_from_neighbor(r_vec, rcut, rfac0, rmin0):
    """Cayley-Klein parameters (a, b) of a neighbour vector."""
    x, y, z = r_vec
    r = sqrt(x * x + y * y + z * z)
    theta0 = rfac0 * pi * (r - rmin0) / (rcut - rmin0)
    z0 = r * cos(theta0) / sin(theta0)
    r0 = sqrt(r * r + z0 * z0)
    return complex(z0, -z) / r0, complex(y, -x) / r0


def switch_fc(r, rcut, rmin0):
    if r >= rcut:
        return 0.0
    return 0.5 * (cos(pi * (r - rmin0) / (rcut - rmin0)) + 1.0)


# ----------------------------------------------------------------------------
# Density, Z, B, energy for one atom
# ----------------------------------------------------------------------------
def density(rij, J, rcut, rfac0=0.99363, rmin0=0.0):
    """u^n for n = 0..J for one centre atom with neighbour vectors rij (m x 3)."""
    u = [np.eye(n + 1, dtype=complex) for n in range(J + 1)]
    for rv in rij:
        r = float(np.linalg.norm(rv))
        if r >= rcut:
            continue
        fc = switch_fc(r, rcut, rmin0)
        a, b = su2_from_neighbor(rv, rcut, rfac0, rmin0)
        for n in range(J + 1):
            u[n] = u[n] + fc * wigner_d(n, a, b)
    return u


def z_block(u, n1, n2, n):
    """Full (n+1)x(n+1) Z^n_{n1 n2}."""
    Z = np.zeros((n + 1, n + 1), dtype=complex)
    off = (n1 + n2 - n) // 2
    for k in range(n + 1):
        for l in range(n + 1):
            s = 0j
            for k1 in range(n1 + 1):
                k2 = k - k1 + off
                if not 0 <= k2 <= n2:
                    continue
                ck = cg(n1, k1, n2, k2, n, k)
                for l1 in range(n1 + 1):
                    l2 = l - l1 + off
                    if not 0 <= l2 <= n2:
                        continue
                    s += ck * cg(n1, l1, n2, l2, n, l) * u[n1][k1, l1] * u[n2][k2, l2]
            Z[k, l] = s
    return Z


def bispectrum_complex(u, J):
    """sum conj(u^n) * Z^n_{n1 n2} for each canonical triple (imaginary part ~ 0)."""
    return np.array([np.sum(np.conj(u[n]) * z_block(u, n1, n2, n))
                     for (n1, n2, n) in canonical_triples(J)])


def bispectrum(u, J):
    return bispectrum_complex(u, J).real


def energy_atom(u, J, beta):
    """beta = [beta_0, beta_1 .. beta_K]."""
    return beta[0] + float(np.dot(beta[1:], bispectrum(u, J)))


def adjoint_brute(u, J, beta):
    """Y^n = 2 dE/d conj(u^n) (Wirtinger), from differentiating the cubic form
    E = beta_0 + sum_k beta_k Re X_k with X = sum conj(u^n) C C u^{n1} u^{n2}:
    dX/d conj(u^n) = Z^n_{n1 n2} and dX/du^{n1}, dX/du^{n2} by the product rule;
    Y = sum_k beta_k [dX_k/d conj(u) + conj(dX_k/du)]."""
    Y = [np.zeros((n + 1, n + 1), dtype=complex) for n in range(J + 1)]
    for bk, (n1, n2, n) in zip(beta[1:], canonical_triples(J)):
        off = (n1 + n2 - n) // 2
        Y[n] += bk * z_block(u, n1, n2, n)
        for k in range(n + 1):
            for l in range(n + 1):
                for k1 in range(n1 + 1):
                    k2 = k - k1 + off
                    if not 0 <= k2 <= n2:
                        continue
                    ck = cg(n1, k1, n2, k2, n, k)
                    for l1 in range(n1 + 1):
                        l2 = l - l1 + off
                        if not 0 <= l2 <= n2:
                            continue
                        c = ck * cg(n1, l1, n2, l2, n, l)
                        cu = np.conj(u[n][k, l])
                        # conj of dX/du^{n1}[k1,l1] = conj(c * conj(u^n) * u^{n2})
                        Y[n1][k1, l1] += bk * np.conj(c * cu * u[n2][k2, l2])
                        Y[n2][k2, l2] += bk * np.conj(c * cu * u[n1][k1, l1])
    return Y
