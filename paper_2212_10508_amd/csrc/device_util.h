// Small device helpers shared by the snapmd HIP sources (internal).
#pragma once
#include <hip/hip_runtime.h>

namespace snapmd {

__device__ __forceinline__ double2 cadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
    return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
// a*b + c*d
__device__ __forceinline__ double2 cmul2(double2 a, double2 b, double2 c, double2 d) {
    return make_double2(fma(a.x, b.x, fma(-a.y, b.y, fma(c.x, d.x, -c.y * d.y))),
                        fma(a.x, b.y, fma(a.y, b.x, fma(c.x, d.y, c.y * d.x))));
}
__device__ __forceinline__ double2 cconj(double2 a) { return make_double2(a.x, -a.y); }

__device__ __forceinline__ int sys_of(const int *__restrict__ off, int n_sys, int i) {
    int lo = 0, hi = n_sys - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (off[mid] <= i) lo = mid; else hi = mid - 1;
    }
    return lo;
}

}  // namespace snapmd
