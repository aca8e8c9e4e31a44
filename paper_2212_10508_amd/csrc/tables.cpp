// Host-side index and coupling tables of the SNAP kernels.
//
// Clebsch-Gordan coefficients C^{j m}_{j1 m1, j2 m2} follow Racah's closed formula,
// evaluated with long-double factorials (exact integers up to 25!).  The SNAP
// bispectrum (Thompson et al.; the fine potential of the paper's "MD settings"
// section) is B_{j1 j2 j} = sum conj(u^j_{m m'}) Z^j_{j1 j2 m m'} with
//   Z^j_{j1 j2 m m'} = sum C^{j m}_{j1 m1, j2 m2} C^{j m'}_{j1 m1', j2 m2'} u^{j1}_{m1 m1'} u^{j2}_{m2 m2'}.
// The adjoint Y^j = 2 dE/d conj(u^j) of E = beta0 + sum_k beta_k B_k collects, for every
// coupling block (j1 >= j2, j), beta_k * mult * (2 j_max + 1)/(2 j + 1) Z^j_{j1 j2} where
// (j1, j2, j) sorted is the canonical triple k, j_max its largest entry and mult the
// number of its entries equal to j (the coupling-coefficient symmetry under exchange of
// j with j1 or j2 turns the derivatives along u^{j1}, u^{j2} into Z blocks).
#include <algorithm>
#include <cmath>
#include <map>
#include <mutex>
#include <tuple>

#include "snapmd_internal.h"

namespace snapmd {

static long double lfact(int n) {
    long double r = 1.0L;
    for (int i = 2; i <= n; ++i) r *= (long double)i;
    return r;
}

double cg_coeff(int n1, int k1, int n2, int k2, int n, int k) {
    const int tm1 = 2 * k1 - n1, tm2 = 2 * k2 - n2, tm = 2 * k - n;
    if (tm1 + tm2 != tm) return 0.0;
    if (n < std::abs(n1 - n2) || n > n1 + n2 || ((n1 + n2 + n) & 1)) return 0.0;
    if (k1 < 0 || k1 > n1 || k2 < 0 || k2 > n2 || k < 0 || k > n) return 0.0;
    const int a = (n + n1 - n2) / 2, b = (n - n1 + n2) / 2, c = (n1 + n2 - n) / 2;
    const int d = (n1 + n2 + n) / 2 + 1;
    long double pre = (long double)(n + 1) * lfact(a) * lfact(b) * lfact(c) / lfact(d);
    pre *= lfact((n + tm) / 2) * lfact((n - tm) / 2) * lfact((n1 + tm1) / 2) *
           lfact((n1 - tm1) / 2) * lfact((n2 + tm2) / 2) * lfact((n2 - tm2) / 2);
    long double s = 0.0L;
    for (int t = 0; t <= c; ++t) {
        const int e0 = t, e1 = c - t, e2 = (n1 - tm1) / 2 - t, e3 = (n2 + tm2) / 2 - t;
        const int e4 = (n - n2 + tm1) / 2 + t, e5 = (n - n1 - tm2) / 2 + t;
        if (e0 < 0 || e1 < 0 || e2 < 0 || e3 < 0 || e4 < 0 || e5 < 0) continue;
        const long double den = lfact(e0) * lfact(e1) * lfact(e2) * lfact(e3) * lfact(e4) * lfact(e5);
        s += ((t & 1) ? -1.0L : 1.0L) / den;
    }
    return (double)(sqrtl(pre) * s);
}

int snap_ncoeff(int J) {
    int K = 0;
    for (int n1 = 0; n1 <= J; ++n1)
        for (int n2 = 0; n2 <= n1; ++n2)
            for (int n = n1 - n2; n <= std::min(J, n1 + n2); n += 2)
                if (n >= n1) ++K;
    return K;
}

namespace {
// Location of full-storage element (n, k, l) in half storage.
struct Loc {
    int h;
    int conj;
    double sign;
};
Loc locate(int n, int k, int l) {
    if (2 * l <= n) return {half_idx(n, k, l), 0, 1.0};
    // D[k][l] = (-1)^(k-l) conj(D[n-k][n-l])
    return {half_idx(n, n - k, n - l), 1, ((k - l) & 1) ? -1.0 : 1.0};
}

void build(int J, SnapTables &T) {
    T.J = J;
    T.nh = n_half(J);
    T.nrm.assign(T.nh, 0.0);
    T.ymult.assign(T.nh, 0.0);
    T.elem_n.assign(T.nh, 0);
    T.elem_k.assign(T.nh, 0);
    T.elem_l.assign(T.nh, 0);
    for (int n = 0; n <= J; ++n)
        for (int l = 0; 2 * l <= n; ++l)
            for (int k = 0; k <= n; ++k) {
                const int e = half_idx(n, k, l);
                T.elem_n[e] = n;
                T.elem_k[e] = k;
                T.elem_l[e] = l;
                T.nrm[e] = (double)sqrtl(lfact(k) * lfact(n - k) / (lfact(l) * lfact(n - l)));
                double m = 2.0;
                if (2 * l == n) m = (2 * k < n) ? 2.0 : (2 * k == n ? 1.0 : 0.0);
                T.ymult[e] = m;
            }
    // canonical triples
    std::map<std::tuple<int, int, int>, int> canon;
    for (int n1 = 0; n1 <= J; ++n1)
        for (int n2 = 0; n2 <= n1; ++n2)
            for (int n = n1 - n2; n <= std::min(J, n1 + n2); n += 2)
                if (n >= n1) {
                    canon[{n1, n2, n}] = (int)T.tr_n1.size();
                    T.tr_n1.push_back(n1);
                    T.tr_n2.push_back(n2);
                    T.tr_n.push_back(n);
                }
    T.K = (int)T.tr_n1.size();
    // Z blocks with their adjoint weights
    for (int n1 = 0; n1 <= J; ++n1)
        for (int n2 = 0; n2 <= n1; ++n2)
            for (int n = n1 - n2; n <= std::min(J, n1 + n2); n += 2) {
                int s[3] = {n1, n2, n};
                std::sort(s, s + 3);  // s[0] <= s[1] <= s[2]
                const int q = s[0], p = s[1], r = s[2];
                const int mult = (p == n) + (q == n) + (r == n);
                T.zb_n1.push_back(n1);
                T.zb_n2.push_back(n2);
                T.zb_n.push_back(n);
                T.zb_canon.push_back(canon.at({p, q, r}));
                T.zb_wt.push_back(mult * double(r + 1) / double(n + 1));
            }
    // Y program (output elements in half order, skipping multiplicity-0 entries)
    T.ystart.assign(T.nh + 1, 0);
    for (int e = 0; e < T.nh; ++e) {
        T.ystart[e] = (int)T.yidx.size();
        if (T.ymult[e] == 0.0) continue;
        const int n = T.elem_n[e], k = T.elem_k[e], l = T.elem_l[e];
        for (int b = 0; b < (int)T.zb_n.size(); ++b) {
            if (T.zb_n[b] != n) continue;
            const int n1 = T.zb_n1[b], n2 = T.zb_n2[b], off = (n1 + n2 - n) / 2;
            for (int k1 = 0; k1 <= n1; ++k1) {
                const int k2 = k - k1 + off;
                if (k2 < 0 || k2 > n2) continue;
                const double c1 = cg_coeff(n1, k1, n2, k2, n, k);
                if (c1 == 0.0) continue;
                for (int l1 = 0; l1 <= n1; ++l1) {
                    const int l2 = l - l1 + off;
                    if (l2 < 0 || l2 > n2) continue;
                    const double c2 = cg_coeff(n1, l1, n2, l2, n, l);
                    if (c2 == 0.0) continue;
                    const Loc a = locate(n1, k1, l1), bb = locate(n2, k2, l2);
                    T.yidx.push_back((uint32_t)a.h | ((uint32_t)bb.h << 12) | ((uint32_t)a.conj << 24) |
                                     ((uint32_t)bb.conj << 25));
                    T.ycg.push_back(c1 * c2 * a.sign * bb.sign);
                    T.yblock.push_back(b);
                }
            }
        }
    }
    T.ystart[T.nh] = (int)T.yidx.size();
    // B program: canonical triple t, half elements e of level n
    T.bstart.assign(T.K + 1, 0);
    for (int t = 0; t < T.K; ++t) {
        T.bstart[t] = (int)T.bidx.size();
        const int n1 = T.tr_n1[t], n2 = T.tr_n2[t], n = T.tr_n[t], off = (n1 + n2 - n) / 2;
        for (int l = 0; 2 * l <= n; ++l)
            for (int k = 0; k <= n; ++k) {
                const int e = half_idx(n, k, l);
                if (T.ymult[e] == 0.0) continue;
                for (int k1 = 0; k1 <= n1; ++k1) {
                    const int k2 = k - k1 + off;
                    if (k2 < 0 || k2 > n2) continue;
                    const double c1 = cg_coeff(n1, k1, n2, k2, n, k);
                    if (c1 == 0.0) continue;
                    for (int l1 = 0; l1 <= n1; ++l1) {
                        const int l2 = l - l1 + off;
                        if (l2 < 0 || l2 > n2) continue;
                        const double c2 = cg_coeff(n1, l1, n2, l2, n, l);
                        if (c2 == 0.0) continue;
                        const Loc a = locate(n1, k1, l1), bb = locate(n2, k2, l2);
                        T.bidx.push_back((uint32_t)a.h | ((uint32_t)bb.h << 12) |
                                         ((uint32_t)a.conj << 24) | ((uint32_t)bb.conj << 25));
                        T.bel.push_back(e);
                        T.bcg.push_back(c1 * c2 * a.sign * bb.sign * T.ymult[e]);
                    }
                }
            }
    }
    T.bstart[T.K] = (int)T.bidx.size();
}
}  // namespace

const SnapTables &snap_tables(int J) {
    static std::mutex mu;
    static std::map<int, SnapTables> cache;
    std::lock_guard<std::mutex> g(mu);
    auto it = cache.find(J);
    if (it != cache.end()) return it->second;
    SnapTables &T = cache[J];
    build(J, T);
    return T;
}

}  // namespace snapmd
