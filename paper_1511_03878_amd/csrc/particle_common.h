// Per-particle helpers shared by the 2-D and 3-D particle kernels: quadratic
// shape weights, the four-node Esirkepov window, fast reciprocals and a wave
// reduction.
#pragma once

#include <math.h>

#include "pic_dev.h"

namespace pic {

constexpr int kWave = 64;

// Quadratic B-spline weights of the nodes i0-1, i0, i0+1 for the offset
// dl = xi - i0 in [-1/2, 1/2).
template <typename A>
__device__ __forceinline__ void qweights(A dl, A &wm, A &w0, A &wp)
{
    A a = A(0.5) - dl, b = A(0.5) + dl;
    wm = A(0.5) * a * a;
    w0 = A(0.75) - dl * dl;
    wp = A(0.5) * b * b;
}

// Window of four nodes per axis that holds both the old and the new
// quadratic supports of a move shorter than one cell.  On return S0/DS are
// the old weights and the weight change at nodes m..m+3, computed in FP64 and
// rounded once to W.  The new offset is formed from the exact old offset and
// the displacement in FP64, so the weight change keeps full relative accuracy
// (to W's rounding) even for FP32 storage.
template <typename T, typename W>
__device__ __forceinline__ bool window4(T xl, double disp, int &m, W S0[4], W DS[4])
{
    int i0 = (int)floor(xl + T(0.5));
    double d0 = (double)(xl - (T)i0);  // exact
    double a = d0 + disp;
    int sg = (int)floor(a + 0.5);       // -1, 0 or +1
    double d1 = a - (double)sg;
    double o0m, o00, o0p, o1m, o10, o1p;
    qweights(d0, o0m, o00, o0p);
    qweights(d1, o1m, o10, o1p);
    int lo = sg < 0 ? sg : 0;
    m = i0 - 1 + lo;
    bool s0 = lo < 0;   // old support starts at window slot 1
    bool s1 = sg > 0;   // new support starts at window slot 1
    double A0[4] = {s0 ? 0.0 : o0m, s0 ? o0m : o00, s0 ? o00 : o0p, s0 ? o0p : 0.0};
    double A1[4] = {s1 ? 0.0 : o1m, s1 ? o1m : o10, s1 ? o10 : o1p, s1 ? o1p : 0.0};
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        S0[k] = (W)A0[k];
        DS[k] = (W)(A1[k] - A0[k]);
    }
    // window slot 3 carries weight only when the nearest node changed
    return sg != 0;
}

// Reciprocal and reciprocal square root: hardware approximations (about one
// ulp) for FP32, correctly rounded operations for FP64.
__device__ __forceinline__ float rcp_(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ double rcp_(double x) { return 1.0 / x; }
__device__ __forceinline__ float rsq_(float x) { return __builtin_amdgcn_rsqf(x); }
__device__ __forceinline__ double rsq_(double x) { return 1.0 / sqrt(x); }

template <typename T>
__device__ __forceinline__ T below(T v);
template <>
__device__ __forceinline__ float below<float>(float v) { return nextafterf(v, 0.0f); }
template <>
__device__ __forceinline__ double below<double>(double v) { return nextafter(v, 0.0); }

__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
    return v;
}

}  // namespace pic
