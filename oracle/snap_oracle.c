/*
 * Plain FP64 CPU oracle for the fine/coarse propagators of adaptive parareal
 * Langevin dynamics (SNAP + Finnis-Sinclair forces inside BAOAB steps).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the CPU-baseline
 * leg of the benchmark may load this library.  It shares no code, table or
 * constant generator with the HIP library: every formula below is written out
 * from its definition, slowly and in full (non-symmetric) storage.
 *
 * Built with -O2 -fno-fast-math -ffp-contract=off (no FMA contraction).
 *
 * Contents (all indices are 2j-integers n = 2j; rows k, columns l in 0..n):
 *   - Clebsch-Gordan coefficients by Racah's closed formula.
 *   - Wigner-D matrices of SU(2) by the explicit binomial expansion of the action
 *     of g = [[a, b], [-conj b, conj a]] on degree-n polynomials in (u, v):
 *       D[k][l] = sqrt(k!(n-k)!/(l!(n-l)!)) *
 *                 sum_{p+q=k} C(l,p) C(n-l,q) a^p (-conj b)^(l-p) b^q (conj a)^(n-l-q)
 *     and its derivative by the product rule.
 *   - SNAP (Thompson et al., the fine potential of the paper's "MD settings"):
 *     neighbour map to the 3-sphere, density u, Z, bispectrum B, energy, and forces
 *     by two routes: the direct product rule on B, and the adjoint (Wirtinger
 *     derivative Y = 2 dE/d conj(u) of the cubic form, brute force).
 *   - Finnis-Sinclair EAM (energy and forces).
 *   - Philox4x64-10 (Salmon et al., SC'11) and Box-Muller Gaussians.
 *   - BAOAB Langevin steps (discretisation of the Langevin equation of the
 *     paper's "Algorithm" section, with masses), one force evaluation per step.
 *   - The paper's own integrator: the modified BBK scheme (eq:scheme_debut,
 *     eq:scheme) with the temperature schedule of eq:scheme_corrected_debut,
 *     eq:scheme_corrected, one call = one application of L iterates.
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef double complex cplx;

#define ORA_PI 3.14159265358979323846
#define ORA_KB 8.617333262145179e-5      /* Boltzmann constant, eV/K */
#define ORA_MVV2E 1.0364269652680506e-4  /* eV per amu*A^2/ps^2 */

/* ------------------------------------------------------------------------- */
/* Clebsch-Gordan by Racah's formula                                           */
/* ------------------------------------------------------------------------- */
static double ofact(int n) {
    double r = 1.0;
    for (int i = 2; i <= n; i++) r *= (double)i;
    return r;
}

/* C^{j m}_{j1 m1, j2 m2} with j = n/2, m = k - n/2, etc. */
double ora_cg(int n1, int k1, int n2, int k2, int n, int k) {
    int tm1 = 2 * k1 - n1, tm2 = 2 * k2 - n2, tm = 2 * k - n;
    if (tm1 + tm2 != tm) return 0.0;
    if (n < abs(n1 - n2) || n > n1 + n2 || ((n1 + n2 + n) & 1)) return 0.0;
    if (k1 < 0 || k1 > n1 || k2 < 0 || k2 > n2 || k < 0 || k > n) return 0.0;
    int a = (n + n1 - n2) / 2, b = (n - n1 + n2) / 2, c = (n1 + n2 - n) / 2;
    int d = (n1 + n2 + n) / 2 + 1;
    double pref = (n + 1) * ofact(a) * ofact(b) * ofact(c) / ofact(d);
    pref *= ofact((n + tm) / 2) * ofact((n - tm) / 2) * ofact((n1 - tm1) / 2) *
            ofact((n1 + tm1) / 2) * ofact((n2 - tm2) / 2) * ofact((n2 + tm2) / 2);
    double s = 0.0;
    for (int t = 0; t <= c; t++) {
        int e[6] = {t, c - t, (n1 - tm1) / 2 - t, (n2 + tm2) / 2 - t,
                    (n - n2 + tm1) / 2 + t, (n - n1 - tm2) / 2 + t};
        int ok = 1;
        double den = 1.0;
        for (int q = 0; q < 6; q++) {
            if (e[q] < 0) { ok = 0; break; }
            den *= ofact(e[q]);
        }
        if (!ok) continue;
        s += ((t & 1) ? -1.0 : 1.0) / den;
    }
    return sqrt(pref) * s;
}

/* ------------------------------------------------------------------------- */
/* Wigner-D by explicit expansion                                              */
/* ------------------------------------------------------------------------- */
static double binom(int n, int k) { return ofact(n) / (ofact(k) * ofact(n - k)); }

static cplx ipow(cplx z, int e) {
    cplx r = 1.0;
    for (int i = 0; i < e; i++) r *= z;
    return r;
}

/* D is (n+1)x(n+1) row-major D[k*(n+1)+l]. */
static void wigner_full(int n, cplx a, cplx b, cplx *D) {
    cplx mb = -conj(b), ca = conj(a);
    for (int k = 0; k <= n; k++)
        for (int l = 0; l <= n; l++) {
            cplx s = 0.0;
            for (int p = 0; p <= l; p++) {
                int q = k - p;
                if (q < 0 || q > n - l) continue;
                s += binom(l, p) * binom(n - l, q) * ipow(a, p) * ipow(mb, l - p) *
                     ipow(b, q) * ipow(ca, n - l - q);
            }
            D[k * (n + 1) + l] = s * sqrt(ofact(k) * ofact(n - k) / (ofact(l) * ofact(n - l)));
        }
}

/* dD[alpha][k*(n+1)+l] = dD/dx_alpha given da/dx_alpha, db/dx_alpha. */
static void wigner_full_deriv(int n, cplx a, cplx b, const cplx da[3], const cplx db[3],
                              cplx *dD) {
    cplx mb = -conj(b), ca = conj(a);
    int sz = (n + 1) * (n + 1);
    for (int al = 0; al < 3; al++) {
        cplx dmb = -conj(db[al]), dca = conj(da[al]);
        for (int k = 0; k <= n; k++)
            for (int l = 0; l <= n; l++) {
                cplx s = 0.0;
                for (int p = 0; p <= l; p++) {
                    int q = k - p;
                    if (q < 0 || q > n - l) continue;
                    int e1 = p, e2 = l - p, e3 = q, e4 = n - l - q;
                    cplx f1 = ipow(a, e1), f2 = ipow(mb, e2), f3 = ipow(b, e3), f4 = ipow(ca, e4);
                    cplx d1 = e1 ? e1 * ipow(a, e1 - 1) * da[al] : 0.0;
                    cplx d2 = e2 ? e2 * ipow(mb, e2 - 1) * dmb : 0.0;
                    cplx d3 = e3 ? e3 * ipow(b, e3 - 1) * db[al] : 0.0;
                    cplx d4 = e4 ? e4 * ipow(ca, e4 - 1) * dca : 0.0;
                    cplx t = d1 * f2 * f3 * f4 + f1 * d2 * f3 * f4 + f1 * f2 * d3 * f4 +
                             f1 * f2 * f3 * d4;
                    s += binom(l, p) * binom(n - l, q) * t;
                }
                dD[al * sz + k * (n + 1) + l] =
                    s * sqrt(ofact(k) * ofact(n - k) / (ofact(l) * ofact(n - l)));
            }
    }
}

void ora_wigner(int n, double ar, double ai, double br, double bi, double *out /* 2*(n+1)^2 */) {
    int sz = (n + 1) * (n + 1);
    cplx *D = malloc(sizeof(cplx) * sz);
    wigner_full(n, ar + I * ai, br + I * bi, D);
    for (int i = 0; i < sz; i++) { out[2 * i] = creal(D[i]); out[2 * i + 1] = cimag(D[i]); }
    free(D);
}

/* ------------------------------------------------------------------------- */
/* SNAP                                                                        */
/* ------------------------------------------------------------------------- */
typedef struct {
    int J;
    double rcut, rfac0, rmin0;
} ora_snap;

/* Neighbour map to the 3-sphere and the switching function, with derivatives
 * with respect to the components of r = x_j - x_i. */
static void cayley_klein(const double rv[3], const ora_snap *s, cplx *a, cplx *b, cplx da[3],
                         cplx db[3], double *fc, double dfc[3]) {
    double x = rv[0], y = rv[1], z = rv[2];
    double r = sqrt(x * x + y * y + z * z);
    double c = s->rfac0 * ORA_PI / (s->rcut - s->rmin0);
    double th = c * (r - s->rmin0);
    double z0 = r * cos(th) / sin(th);
    double r0 = sqrt(r * r + z0 * z0);
    double dz0dr = cos(th) / sin(th) - r * c / (sin(th) * sin(th));
    double dr0dr = (r + z0 * dz0dr) / r0;
    *a = (z0 - I * z) / r0;
    *b = (y - I * x) / r0;
    for (int al = 0; al < 3; al++) {
        double drdx = rv[al] / r;
        cplx num_a = dz0dr * drdx - (al == 2 ? I : 0.0);
        da[al] = num_a / r0 - (z0 - I * z) * dr0dr * drdx / (r0 * r0);
        cplx num_b = (al == 1 ? 1.0 : 0.0) - (al == 0 ? I : 0.0);
        db[al] = num_b / r0 - (y - I * x) * dr0dr * drdx / (r0 * r0);
    }
    double w = ORA_PI / (s->rcut - s->rmin0);
    *fc = 0.5 * (cos(w * (r - s->rmin0)) + 1.0);
    double dfdr = -0.5 * w * sin(w * (r - s->rmin0));
    for (int al = 0; al < 3; al++) dfc[al] = dfdr * rv[al] / r;
}

static int n_ulevel_off(int n) { /* offset of level n in full storage */
    int o = 0;
    for (int m = 0; m < n; m++) o += (m + 1) * (m + 1);
    return o;
}

int ora_snap_ncoeff(int J) {
    int K = 0;
    for (int n1 = 0; n1 <= J; n1++)
        for (int n2 = 0; n2 <= n1; n2++)
            for (int n = n1 - n2; n <= (J < n1 + n2 ? J : n1 + n2); n += 2)
                if (n >= n1) K++;
    return K;
}

/* Minimum-image displacement x_j - x_i in an orthorhombic periodic box. */
static void min_image(const double *x, int N, int i, int j, const double box[3], double d[3]) {
    for (int al = 0; al < 3; al++) {
        double t = x[al * N + j] - x[al * N + i];
        t -= box[al] * nearbyint(t / box[al]);
        d[al] = t;
    }
}

/* Brute-force full neighbour list: every j != i with |d| < rcut. */
int ora_neighbors(int N, const double *x, const double box[3], double rcut, int maxn, int *count,
                  int *list) {
    int over = 0;
    for (int i = 0; i < N; i++) {
        int c = 0;
        for (int j = 0; j < N; j++) {
            if (j == i) continue;
            double d[3];
            min_image(x, N, i, j, box, d);
            double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
            if (r2 < rcut * rcut) {
                if (c < maxn) list[i * maxn + c] = j;
                c++;
            }
        }
        count[i] = c;
        if (c > maxn) over = 1;
    }
    return over ? -1 : 0;
}

/* Density u (full storage, all levels) of atom i. */
static void atom_density(const ora_snap *s, int N, const double *x, const double box[3], int i,
                         const int *count, const int *list, int maxn, cplx *u) {
    int J = s->J;
    int tot = n_ulevel_off(J + 1);
    memset(u, 0, sizeof(cplx) * tot);
    for (int n = 0; n <= J; n++)
        for (int k = 0; k <= n; k++) u[n_ulevel_off(n) + k * (n + 1) + k] = 1.0;
    cplx *D = malloc(sizeof(cplx) * (J + 1) * (J + 1));
    for (int t = 0; t < count[i]; t++) {
        int j = list[i * maxn + t];
        double d[3];
        min_image(x, N, i, j, box, d);
        double r = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
        if (r >= s->rcut) continue;
        cplx a, b, da[3], db[3];
        double fc, dfc[3];
        cayley_klein(d, s, &a, &b, da, db, &fc, dfc);
        for (int n = 0; n <= J; n++) {
            wigner_full(n, a, b, D);
            for (int q = 0; q < (n + 1) * (n + 1); q++) u[n_ulevel_off(n) + q] += fc * D[q];
        }
    }
    free(D);
}

/* Z^n_{n1 n2}(u1, u2) in full (n+1)^2 storage. */
static void zblock(const cplx *u, const cplx *v, int n1, int n2, int n, int J, cplx *Z) {
    (void)J;
    int off = (n1 + n2 - n) / 2;
    const cplx *U1 = u + n_ulevel_off(n1), *U2 = v + n_ulevel_off(n2);
    for (int k = 0; k <= n; k++)
        for (int l = 0; l <= n; l++) {
            cplx s = 0.0;
            for (int k1 = 0; k1 <= n1; k1++) {
                int k2 = k - k1 + off;
                if (k2 < 0 || k2 > n2) continue;
                double ck = ora_cg(n1, k1, n2, k2, n, k);
                for (int l1 = 0; l1 <= n1; l1++) {
                    int l2 = l - l1 + off;
                    if (l2 < 0 || l2 > n2) continue;
                    s += ck * ora_cg(n1, l1, n2, l2, n, l) * U1[k1 * (n1 + 1) + l1] *
                         U2[k2 * (n2 + 1) + l2];
                }
            }
            Z[k * (n + 1) + l] = s;
        }
}

/* Bispectrum of one atom from its density (real part of sum conj(u^n) Z). */
static void atom_bispectrum(int J, const cplx *u, double *B) {
    cplx *Z = malloc(sizeof(cplx) * (J + 1) * (J + 1));
    int t = 0;
    for (int n1 = 0; n1 <= J; n1++)
        for (int n2 = 0; n2 <= n1; n2++)
            for (int n = n1 - n2; n <= (J < n1 + n2 ? J : n1 + n2); n += 2) {
                if (n < n1) continue;
                zblock(u, u, n1, n2, n, J, Z);
                cplx s = 0.0;
                const cplx *Un = u + n_ulevel_off(n);
                for (int q = 0; q < (n + 1) * (n + 1); q++) s += conj(Un[q]) * Z[q];
                B[t++] = creal(s);
            }
    free(Z);
}

/* Adjoint Y = 2 dE/d conj(u) of E = beta0 + sum beta_t Re X_t, brute force. */
static void atom_adjoint(int J, const cplx *u, const double *beta, cplx *Y) {
    int tot = n_ulevel_off(J + 1);
    memset(Y, 0, sizeof(cplx) * tot);
    cplx *Z = malloc(sizeof(cplx) * (J + 1) * (J + 1));
    int t = 0;
    for (int n1 = 0; n1 <= J; n1++)
        for (int n2 = 0; n2 <= n1; n2++)
            for (int n = n1 - n2; n <= (J < n1 + n2 ? J : n1 + n2); n += 2) {
                if (n < n1) continue;
                double bk = beta[1 + t];
                t++;
                int off = (n1 + n2 - n) / 2;
                const cplx *Un = u + n_ulevel_off(n), *U1 = u + n_ulevel_off(n1),
                           *U2 = u + n_ulevel_off(n2);
                cplx *Yn = Y + n_ulevel_off(n), *Y1 = Y + n_ulevel_off(n1),
                     *Y2 = Y + n_ulevel_off(n2);
                zblock(u, u, n1, n2, n, J, Z);
                for (int q = 0; q < (n + 1) * (n + 1); q++) Yn[q] += bk * Z[q];
                for (int k = 0; k <= n; k++)
                    for (int l = 0; l <= n; l++)
                        for (int k1 = 0; k1 <= n1; k1++) {
                            int k2 = k - k1 + off;
                            if (k2 < 0 || k2 > n2) continue;
                            double ck = ora_cg(n1, k1, n2, k2, n, k);
                            for (int l1 = 0; l1 <= n1; l1++) {
                                int l2 = l - l1 + off;
                                if (l2 < 0 || l2 > n2) continue;
                                double c = ck * ora_cg(n1, l1, n2, l2, n, l);
                                cplx cu = conj(Un[k * (n + 1) + l]);
                                Y1[k1 * (n1 + 1) + l1] += bk * conj(c * cu * U2[k2 * (n2 + 1) + l2]);
                                Y2[k2 * (n2 + 1) + l2] += bk * conj(c * cu * U1[k1 * (n1 + 1) + l1]);
                            }
                        }
            }
    free(Z);
}

/* Per-pair derivative dE_i/dr_ij (3 components) by the adjoint route. */
static void pair_dedr_adjoint(const ora_snap *s, const double d[3], const cplx *Y, double g[3]) {
    int J = s->J;
    cplx a, b, da[3], db[3];
    double fc, dfc[3];
    cayley_klein(d, s, &a, &b, da, db, &fc, dfc);
    cplx *D = malloc(sizeof(cplx) * (J + 1) * (J + 1));
    cplx *dD = malloc(sizeof(cplx) * 3 * (J + 1) * (J + 1));
    g[0] = g[1] = g[2] = 0.0;
    for (int n = 0; n <= J; n++) {
        int sz = (n + 1) * (n + 1);
        wigner_full(n, a, b, D);
        wigner_full_deriv(n, a, b, da, db, dD);
        const cplx *Yn = Y + n_ulevel_off(n);
        for (int al = 0; al < 3; al++)
            for (int q = 0; q < sz; q++) {
                cplx du = dfc[al] * D[q] + fc * dD[al * sz + q];
                g[al] += creal(conj(Yn[q]) * du);
            }
    }
    free(D);
    free(dD);
}

/* Per-pair derivative dE_i/dr_ij by the direct product rule on every B_t. */
static void pair_dedr_direct(const ora_snap *s, const double d[3], const cplx *u,
                             const double *beta, double g[3]) {
    int J = s->J;
    int tot = n_ulevel_off(J + 1);
    cplx a, b, da[3], db[3];
    double fc, dfc[3];
    cayley_klein(d, s, &a, &b, da, db, &fc, dfc);
    cplx *du = calloc((size_t)3 * tot, sizeof(cplx)); /* du[al][full index] */
    cplx *D = malloc(sizeof(cplx) * (J + 1) * (J + 1));
    cplx *dD = malloc(sizeof(cplx) * 3 * (J + 1) * (J + 1));
    for (int n = 0; n <= J; n++) {
        int sz = (n + 1) * (n + 1);
        wigner_full(n, a, b, D);
        wigner_full_deriv(n, a, b, da, db, dD);
        for (int al = 0; al < 3; al++)
            for (int q = 0; q < sz; q++)
                du[al * tot + n_ulevel_off(n) + q] = dfc[al] * D[q] + fc * dD[al * sz + q];
    }
    cplx *Z = malloc(sizeof(cplx) * (J + 1) * (J + 1));
    cplx *Za = malloc(sizeof(cplx) * (J + 1) * (J + 1));
    cplx *Zb = malloc(sizeof(cplx) * (J + 1) * (J + 1));
    g[0] = g[1] = g[2] = 0.0;
    int t = 0;
    for (int n1 = 0; n1 <= J; n1++)
        for (int n2 = 0; n2 <= n1; n2++)
            for (int n = n1 - n2; n <= (J < n1 + n2 ? J : n1 + n2); n += 2) {
                if (n < n1) continue;
                double bk = beta[1 + t];
                t++;
                zblock(u, u, n1, n2, n, J, Z);
                const cplx *Un = u + n_ulevel_off(n);
                for (int al = 0; al < 3; al++) {
                    const cplx *dul = du + al * tot;
                    zblock(dul, u, n1, n2, n, J, Za); /* dZ from d u^{n1} */
                    zblock(u, dul, n1, n2, n, J, Zb); /* dZ from d u^{n2} */
                    const cplx *dUn = dul + n_ulevel_off(n);
                    cplx sdb = 0.0;
                    for (int q = 0; q < (n + 1) * (n + 1); q++)
                        sdb += conj(dUn[q]) * Z[q] + conj(Un[q]) * (Za[q] + Zb[q]);
                    g[al] += bk * creal(sdb);
                }
            }
    free(du); free(D); free(dD); free(Z); free(Za); free(Zb);
}

/* SNAP energy per atom, bispectrum and forces for one periodic system.
 * x, f: SoA [3][N].  route 0 = adjoint, 1 = direct.  B (nullable): [N][K].
 * Returns the total energy, or NAN if the neighbour list overflowed. */
double ora_snap_compute(int J, double rcut, double rfac0, double rmin0, const double *beta, int N,
                        const double *x, const double box[3], int route, double *f,
                        double *e_atom, double *B, double *dedr_out /* nullable [N][maxn][3] */,
                        int maxn, int *count_out, int *list_out) {
    ora_snap s = {J, rcut, rfac0, rmin0};
    int K = ora_snap_ncoeff(J);
    int tot = n_ulevel_off(J + 1);
    int *count = malloc(sizeof(int) * N), *list = malloc(sizeof(int) * (size_t)N * maxn);
    if (ora_neighbors(N, x, box, rcut, maxn, count, list) != 0) {
        free(count); free(list);
        return NAN;
    }
    double *g = calloc((size_t)N * maxn * 3, sizeof(double));
    double *ea = malloc(sizeof(double) * N);
    double *Bl = malloc(sizeof(double) * (size_t)N * K);
#pragma omp parallel for schedule(dynamic)
    for (int i = 0; i < N; i++) {
        cplx *u = malloc(sizeof(cplx) * tot);
        cplx *Y = malloc(sizeof(cplx) * tot);
        atom_density(&s, N, x, box, i, count, list, maxn, u);
        atom_bispectrum(J, u, Bl + (size_t)i * K);
        double e = beta[0];
        for (int t = 0; t < K; t++) e += beta[1 + t] * Bl[(size_t)i * K + t];
        ea[i] = e;
        if (route == 0) atom_adjoint(J, u, beta, Y);
        for (int t = 0; t < count[i]; t++) {
            int j = list[i * maxn + t];
            double d[3];
            min_image(x, N, i, j, box, d);
            double *gg = g + ((size_t)i * maxn + t) * 3;
            if (route == 0)
                pair_dedr_adjoint(&s, d, Y, gg);
            else
                pair_dedr_direct(&s, d, u, beta, gg);
        }
        free(u);
        free(Y);
    }
    /* F = -grad E: E_i depends on r_ij = x_j - x_i, so dE_i/dx_j = g_ij, dE_i/dx_i = -g_ij */
    for (int q = 0; q < 3 * N; q++) f[q] = 0.0;
    double etot = 0.0;
    for (int i = 0; i < N; i++) {
        etot += ea[i];
        for (int t = 0; t < count[i]; t++) {
            int j = list[i * maxn + t];
            const double *gg = g + ((size_t)i * maxn + t) * 3;
            for (int al = 0; al < 3; al++) {
                f[al * N + i] += gg[al];
                f[al * N + j] -= gg[al];
            }
        }
    }
    if (e_atom) memcpy(e_atom, ea, sizeof(double) * N);
    if (B) memcpy(B, Bl, sizeof(double) * (size_t)N * K);
    if (dedr_out) memcpy(dedr_out, g, sizeof(double) * (size_t)N * maxn * 3);
    if (count_out) memcpy(count_out, count, sizeof(int) * N);
    if (list_out) memcpy(list_out, list, sizeof(int) * (size_t)N * maxn);
    free(count); free(list); free(g); free(ea); free(Bl);
    return etot;
}

/* Density u and adjoint Y of every atom, full storage interleaved (re, im):
 * u_out, y_out: [N][2*tot] (y_out nullable). */
int ora_snap_uy(int J, double rcut, double rfac0, double rmin0, const double *beta, int N,
                const double *x, const double box[3], int maxn, double *u_out, double *y_out) {
    ora_snap s = {J, rcut, rfac0, rmin0};
    int tot = n_ulevel_off(J + 1);
    int *count = malloc(sizeof(int) * N), *list = malloc(sizeof(int) * (size_t)N * maxn);
    if (ora_neighbors(N, x, box, rcut, maxn, count, list) != 0) {
        free(count); free(list);
        return -1;
    }
#pragma omp parallel for schedule(dynamic)
    for (int i = 0; i < N; i++) {
        cplx *u = malloc(sizeof(cplx) * tot);
        cplx *Y = malloc(sizeof(cplx) * tot);
        atom_density(&s, N, x, box, i, count, list, maxn, u);
        for (int q = 0; q < tot; q++) {
            u_out[(size_t)i * 2 * tot + 2 * q] = creal(u[q]);
            u_out[(size_t)i * 2 * tot + 2 * q + 1] = cimag(u[q]);
        }
        if (y_out) {
            atom_adjoint(J, u, beta, Y);
            for (int q = 0; q < tot; q++) {
                y_out[(size_t)i * 2 * tot + 2 * q] = creal(Y[q]);
                y_out[(size_t)i * 2 * tot + 2 * q + 1] = cimag(Y[q]);
            }
        }
        free(u);
        free(Y);
    }
    free(count);
    free(list);
    return 0;
}

/* ------------------------------------------------------------------------- */
/* Finnis-Sinclair EAM                                                          */
/* E = sum_i [ -A sqrt(rho_i) + 1/2 sum_j V(r_ij) ],  rho_i = sum_j phi(r_ij)   */
/* phi(r) = (r-d)^2 (r<d),  V(r) = (r-c)^2 (c0 + c1 r + c2 r^2) (r<c)           */
/* ------------------------------------------------------------------------- */
double ora_fs_compute(double A, double dd, double cc, double c0, double c1, double c2, int N,
                      const double *x, const double box[3], double *f, double *e_atom) {
    double rc = dd > cc ? dd : cc;
    double *rho = calloc(N, sizeof(double));
    double *epair = calloc(N, sizeof(double));
    for (int i = 0; i < N; i++)
        for (int j = 0; j < N; j++) {
            if (j == i) continue;
            double d[3];
            min_image(x, N, i, j, box, d);
            double r = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
            if (r >= rc) continue;
            if (r < dd) rho[i] += (r - dd) * (r - dd);
            if (r < cc) epair[i] += 0.5 * (r - cc) * (r - cc) * (c0 + c1 * r + c2 * r * r);
        }
    double etot = 0.0;
    for (int i = 0; i < N; i++) {
        double e = -A * sqrt(rho[i]) + epair[i];
        if (e_atom) e_atom[i] = e;
        etot += e;
    }
    for (int q = 0; q < 3 * N; q++) f[q] = 0.0;
    for (int i = 0; i < N; i++)
        for (int j = 0; j < N; j++) {
            if (j == i) continue;
            double d[3];
            min_image(x, N, i, j, box, d);
            double r = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
            if (r >= rc) continue;
            /* dE/dr for the pair (i,j), counted from i's side for this ordered pair:
             * pair term 1/2 V'(r) from E_i (E_j's half comes with the (j,i) visit),
             * embedding F'(rho_i) phi'(r) from E_i. */
            double dEdr = 0.0;
            if (r < cc)
                dEdr += 0.5 * (2.0 * (r - cc) * (c0 + c1 * r + c2 * r * r) +
                               (r - cc) * (r - cc) * (c1 + 2.0 * c2 * r));
            if (r < dd && rho[i] > 0.0) dEdr += -A / (2.0 * sqrt(rho[i])) * 2.0 * (r - dd);
            /* E_i depends on x_j - x_i: force on i is +dEdr * d/r, on j is -dEdr * d/r */
            for (int al = 0; al < 3; al++) {
                f[al * N + i] += dEdr * d[al] / r;
                f[al * N + j] -= dEdr * d[al] / r;
            }
        }
    free(rho);
    free(epair);
    return etot;
}

/* ------------------------------------------------------------------------- */
/* Philox4x64-10 and Gaussians                                                 */
/* ------------------------------------------------------------------------- */
static void mulhilo64(uint64_t a, uint64_t b, uint64_t *hi, uint64_t *lo) {
    __uint128_t p = (__uint128_t)a * b;
    *hi = (uint64_t)(p >> 64);
    *lo = (uint64_t)p;
}

void ora_philox4x64_10(const uint64_t ctr_in[4], const uint64_t key_in[2], uint64_t out[4]) {
    const uint64_t M0 = 0xD2E7470EE14C6C93ULL, M1 = 0xCA5A826395121157ULL;
    const uint64_t W0 = 0x9E3779B97F4A7C15ULL, W1 = 0xBB67AE8584CAA73BULL;
    uint64_t c[4] = {ctr_in[0], ctr_in[1], ctr_in[2], ctr_in[3]};
    uint64_t k[2] = {key_in[0], key_in[1]};
    for (int r = 0; r < 10; r++) {
        if (r > 0) { k[0] += W0; k[1] += W1; }
        uint64_t hi0, lo0, hi1, lo1;
        mulhilo64(M0, c[0], &hi0, &lo0);
        mulhilo64(M1, c[2], &hi1, &lo1);
        uint64_t n0 = hi1 ^ c[1] ^ k[0], n1 = lo1, n2 = hi0 ^ c[3] ^ k[1], n3 = lo0;
        c[0] = n0; c[1] = n1; c[2] = n2; c[3] = n3;
    }
    memcpy(out, c, sizeof(c));
}

/* Three standard Gaussians for (seed, noise stream, global step, atom, tag); the tag is
 * the fourth counter word (0 for BAOAB, 1 and 2 for the BBK scheme). */
void ora_gauss3t(uint64_t seed, uint64_t noise_id, uint64_t step, uint64_t atom, uint64_t tag, double g[3]) {
    uint64_t ctr[4] = {noise_id, step, atom, tag}, key[2] = {seed, 0}, w[4];
    ora_philox4x64_10(ctr, key, w);
    const double two53 = 1.0 / 9007199254740992.0;
    double u1 = 1.0 - (double)(w[0] >> 11) * two53; /* (0, 1] */
    double u2 = (double)(w[1] >> 11) * two53;
    double u3 = 1.0 - (double)(w[2] >> 11) * two53;
    double u4 = (double)(w[3] >> 11) * two53;
    double r1 = sqrt(-2.0 * log(u1)), r2 = sqrt(-2.0 * log(u3));
    g[0] = r1 * cos(2.0 * ORA_PI * u2);
    g[1] = r1 * sin(2.0 * ORA_PI * u2);
    g[2] = r2 * cos(2.0 * ORA_PI * u4);
}

/* Three standard Gaussians for (seed, noise stream, global step, atom). */
void ora_gauss3(uint64_t seed, uint64_t noise_id, uint64_t step, uint64_t atom, double g[3]) {
    ora_gauss3t(seed, noise_id, step, atom, 0, g);
}

/* ------------------------------------------------------------------------- */
/* BAOAB Langevin steps                                                         */
/* ------------------------------------------------------------------------- */
typedef struct {
    int potential; /* 0 = FS (coarse), 1 = FS + SNAP (fine), 2 = none (V = 0) */
    int J;
    double rcut, rfac0, rmin0;
    const double *beta;
    double A, d, c, c0, c1, c2;
    int maxn;
} ora_pot;

static double total_forces(const ora_pot *P, int N, const double *x, const double box[3],
                           double *f, double *tmp) {
    double e = 0.0;
    for (int q = 0; q < 3 * N; q++) f[q] = 0.0;
    if (P->potential == 2) return 0.0;
    e += ora_fs_compute(P->A, P->d, P->c, P->c0, P->c1, P->c2, N, x, box, f, NULL);
    if (P->potential == 1) {
        e += ora_snap_compute(P->J, P->rcut, P->rfac0, P->rmin0, P->beta, N, x, box, 0, tmp, NULL,
                              NULL, NULL, P->maxn, NULL, NULL);
        for (int q = 0; q < 3 * N; q++) f[q] += tmp[q];
    }
    return e;
}

/* Advance one system by nsteps BAOAB steps of length dt (ps), in place.
 * x, p: SoA [3][N] (positions in A, momenta p = m v in amu*A/ps).
 * The force at the start is evaluated from x; f_out (nullable) gets the last force.
 * traj_x, traj_p (nullable): [nsteps+1][3][N] snapshots (index 0 = start). */
int ora_langevin(int potential, int J, double rcut, double rfac0, double rmin0,
                 const double *beta, double A, double dd, double cc, double c0, double c1,
                 double c2, int maxn, int N, const double box[3], double dt, double gamma,
                 double mass, double T, uint64_t seed, uint64_t noise_id, int64_t step0,
                 int nsteps, double *x, double *p, double *f_out, double *traj_x,
                 double *traj_p) {
    ora_pot P = {potential, J, rcut, rfac0, rmin0, beta, A, dd, cc, c0, c1, c2, maxn};
    double *f = malloc(sizeof(double) * 3 * N), *tmp = malloc(sizeof(double) * 3 * N);
    double c1f = exp(-gamma * dt);
    double sig = sqrt((1.0 - c1f * c1f) * mass * ORA_KB * T / ORA_MVV2E);
    total_forces(&P, N, x, box, f, tmp);
    if (traj_x) memcpy(traj_x, x, sizeof(double) * 3 * N);
    if (traj_p) memcpy(traj_p, p, sizeof(double) * 3 * N);
    for (int s = 0; s < nsteps; s++) {
        uint64_t gstep = (uint64_t)(step0 + s);
        for (int q = 0; q < 3 * N; q++) p[q] += 0.5 * dt * f[q] / ORA_MVV2E;
        for (int q = 0; q < 3 * N; q++) x[q] += 0.5 * dt * p[q] / mass;
        for (int i = 0; i < N; i++) {
            double g[3];
            ora_gauss3(seed, noise_id, gstep, (uint64_t)i, g);
            for (int al = 0; al < 3; al++) p[al * N + i] = c1f * p[al * N + i] + sig * g[al];
        }
        for (int q = 0; q < 3 * N; q++) x[q] += 0.5 * dt * p[q] / mass;
        double e = total_forces(&P, N, x, box, f, tmp);
        if (!isfinite(e)) {
            free(f); free(tmp);
            return -1; /* non-finite energy or neighbour-list overflow */
        }
        for (int q = 0; q < 3 * N; q++) p[q] += 0.5 * dt * f[q] / ORA_MVV2E;
        if (traj_x) memcpy(traj_x + (size_t)(s + 1) * 3 * N, x, sizeof(double) * 3 * N);
        if (traj_p) memcpy(traj_p + (size_t)(s + 1) * 3 * N, p, sizeof(double) * 3 * N);
    }
    if (f_out) memcpy(f_out, f, sizeof(double) * 3 * N);
    free(f);
    free(tmp);
    return 0;
}

/* ------------------------------------------------------------------------- */
/* Modified BBK scheme (the paper's integrator)                                 */
/* ------------------------------------------------------------------------- */
/* One application of L = nsteps iterates of the paper's scheme to one system, in place,
 * with masses and metal units (F in eV/A enters dp/dt as F / mvv2e; q' = p / m):
 *   iterate 0 (eq:scheme_corrected_debut) and l >= 1 (eq:scheme_corrected):
 *     p_{l+1/2} = p_l + (dt/2) F(q_l) - (dt/2) gamma p_{l-1/2} + s_l G_l,
 *                 with p_{-1/2} replaced by p_0 in iterate 0,
 *     q_{l+1}   = q_l + dt p_{l+1/2} / m,
 *     p_{l+1}   = p_{l+1/2} + (dt/2) F(q_{l+1}) - (dt/2) gamma p_{l+1/2} + s_{l+1} G_{l+1},
 *   s_l = (1/2) sqrt(2 gamma m kB T_l dt / mvv2e), T_l = C_l T with C_0 = cT0 and
 *   C_l = cT1 for l >= 1 (cT0 = cT1 = 1 is eq:scheme_debut / eq:scheme).
 * G: [nsteps+1][3][N] Gaussians G_0 .. G_L, or NULL: then G_l is drawn with counter
 * (noise_id, step0 + l, atom, 1) for l < L and G_L with (noise_id, step0 + L, atom, 2),
 * so that G_L of one call and G_0 of the call that starts at step0 + L differ.
 * traj_x, traj_p (nullable): [nsteps+1][3][N] (q_l, p_l); f_out: the last force. */
int ora_bbk(int potential, int J, double rcut, double rfac0, double rmin0, const double *beta,
            double A, double dd, double cc, double c0, double c1, double c2, int maxn, int N,
            const double box[3], double dt, double gamma, double mass, double T, double cT0,
            double cT1, uint64_t seed, uint64_t noise_id, int64_t step0, const double *G,
            int nsteps, double *x, double *p, double *f_out, double *traj_x, double *traj_p) {
    ora_pot P = {potential, J, rcut, rfac0, rmin0, beta, A, dd, cc, c0, c1, c2, maxn};
    const size_t n3 = (size_t)3 * N;
    double *f = malloc(sizeof(double) * n3), *tmp = malloc(sizeof(double) * n3);
    double *prev = malloc(sizeof(double) * n3), *half = malloc(sizeof(double) * n3);
    double *gl = malloc(sizeof(double) * n3);
    int rc = 0;
    total_forces(&P, N, x, box, f, tmp);
    memcpy(prev, p, sizeof(double) * n3); /* p_{-1/2} := p_0 */
    if (traj_x) memcpy(traj_x, x, sizeof(double) * n3);
    if (traj_p) memcpy(traj_p, p, sizeof(double) * n3);
    for (int l = 0; l <= nsteps && rc == 0; l++) {
        /* G_l and s_l */
        if (G) {
            memcpy(gl, G + (size_t)l * n3, sizeof(double) * n3);
        } else {
            for (int i = 0; i < N; i++) {
                double g[3];
                ora_gauss3t(seed, noise_id, (uint64_t)(step0 + l), (uint64_t)i, l < nsteps ? 1 : 2, g);
                for (int al = 0; al < 3; al++) gl[al * N + i] = g[al];
            }
        }
        const double Tl = (l == 0 ? cT0 : cT1) * T;
        const double sl = 0.5 * sqrt(2.0 * gamma * mass * ORA_KB * Tl * dt / ORA_MVV2E);
        if (l > 0) {
            /* last line of iterate l-1: p_l from p_{l-1/2} (in half) and F(q_l) (in f) */
            for (size_t q = 0; q < n3; q++)
                p[q] = half[q] + 0.5 * dt * f[q] / ORA_MVV2E - 0.5 * dt * gamma * half[q] + sl * gl[q];
            memcpy(prev, half, sizeof(double) * n3);
            if (traj_x) memcpy(traj_x + (size_t)l * n3, x, sizeof(double) * n3);
            if (traj_p) memcpy(traj_p + (size_t)l * n3, p, sizeof(double) * n3);
        }
        if (l == nsteps) break;
        /* first two lines of iterate l */
        for (size_t q = 0; q < n3; q++)
            half[q] = p[q] + 0.5 * dt * f[q] / ORA_MVV2E - 0.5 * dt * gamma * prev[q] + sl * gl[q];
        for (size_t q = 0; q < n3; q++) x[q] += dt * half[q] / mass;
        const double e = total_forces(&P, N, x, box, f, tmp);
        if (!isfinite(e)) rc = -1;
    }
    if (f_out && rc == 0) memcpy(f_out, f, sizeof(double) * n3);
    free(f);
    free(tmp);
    free(prev);
    free(half);
    free(gl);
    return rc;
}

/* Threads of the OpenMP loops over atoms (measurement support: the benchmark times the
 * oracle on one core and on all cores).  Returns the count in effect afterwards. */
#ifdef _OPENMP
#include <omp.h>
#endif
int ora_set_threads(int n) {
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
    return omp_get_max_threads();
#else
    (void)n;
    return 1;
#endif
}
