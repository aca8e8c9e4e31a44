// Small device helpers shared by the snapmd HIP sources (internal).
#pragma once
#include <hip/hip_runtime.h>

namespace snapmd {

__device__ __forceinline__ double2 cadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ double2 csub(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }
// Products as explicit FMAs: left to contraction, which of the two products is fused
// follows the compiler's operand order, which changes with the surrounding code (so two
// kernel shapes of one pass would round differently).
__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
    return make_double2(fma(a.x, b.x, -a.y * b.y), fma(a.x, b.y, a.y * b.x));
}
// a*b + c*d
__device__ __forceinline__ double2 cmul2(double2 a, double2 b, double2 c, double2 d) {
    return make_double2(fma(a.x, b.x, fma(-a.y, b.y, fma(c.x, d.x, -c.y * d.y))),
                        fma(a.x, b.y, fma(a.y, b.x, fma(c.x, d.y, c.y * d.x))));
}
// a*b + c*d + e*f + g*h as one FMA chain per component (no separate products or adds)
__device__ __forceinline__ double2 cmul4(double2 a, double2 b, double2 c, double2 d, double2 e, double2 f,
                                         double2 g, double2 h) {
    return make_double2(
        fma(a.x, b.x, fma(-a.y, b.y, fma(c.x, d.x, fma(-c.y, d.y, fma(e.x, f.x, fma(-e.y, f.y, fma(g.x, h.x, -g.y * h.y))))))),
        fma(a.x, b.y, fma(a.y, b.x, fma(c.x, d.y, fma(c.y, d.x, fma(e.x, f.y, fma(e.y, f.x, fma(g.x, h.y, g.y * h.x))))))));
}
__device__ __forceinline__ double2 cconj(double2 a) { return make_double2(a.x, -a.y); }

// 1/sqrt(r2) for a normal r2 > 0: the hardware estimate (about 24 bits) refined by two
// Newton steps y <- y + y (1 - r2 y^2) / 2 (below one ulp); r = r2 * rsqrt_nr(r2).
__device__ __forceinline__ double rsqrt_nr(double r2) {
    double y = __builtin_amdgcn_rsq(r2);
    double e = fma(-r2 * y, y, 1.0);
    y = fma(0.5 * y, e, y);
    e = fma(-r2 * y, y, 1.0);
    return fma(0.5 * y, e, y);
}

__device__ __forceinline__ int sys_of(const int *__restrict__ off, int n_sys, int i) {
    int lo = 0, hi = n_sys - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (off[mid] <= i) lo = mid; else hi = mid - 1;
    }
    return lo;
}

}  // namespace snapmd
