// Fixed-point current: the weight bound behind its scale, and the conversion
// of the deterministic accumulators into the step's current.
//
// The particle kernels accumulate each work item's current in a 64-bit
// fixed-point LDS tile whose scale follows from a bound on the particles'
// weights (fix_scale).  With deterministic deposition a simulation's tiles
// are added to 64-bit integer accumulators with integer atomics: integer
// sums do not depend on the order in which work items finish, so a run
// repeats bit for bit and a simulation computes the same bits alone and in a
// batch.  The conversion pass then writes J[step & 1] (cleared by the
// previous step's field update) in storage precision and clears the
// accumulators.
#include "runtime.h"

namespace pic {

namespace {

constexpr int kCB = 256;

// Weight bound of a freshly loaded simulation: max |w| over the live slots
// of every patch (one workgroup per patch, grid-stride).
template <typename T>
__global__ __launch_bounds__(kCB) void k_wmax(const SimDev<T> *__restrict__ sp)
{
    const SimDev<T> &S = *sp;
    double m = 0.0;
    for (int p = blockIdx.x; p < S.npatch; p += gridDim.x) {
        const int n = glb(S.count)[p];
        const gptr_t<const T> M = glb((const T *)S.mom) + 4 * glb(S.off)[p];
        for (int k = threadIdx.x; k < n; k += kCB) m = fmax(m, fabs((double)M[4 * k + 3]));
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) m = fmax(m, __shfl_xor(m, o, 64));
    if ((threadIdx.x & 63) == 0 && m > 0.0) raise_wmax(S, m);
}

// Accumulators -> J[step & 1] of every active simulation of the list; node
// g of the concatenated node ranges (prefix: exclusive, nlist + 1 entries).
template <typename T>
__global__ __launch_bounds__(kCB) void k_jfix(const SimDev<T> *__restrict__ sims, const int *__restrict__ list,
                                              const int64_t *__restrict__ prefix, int nlist)
{
    const int64_t total = prefix[nlist];
    for (int64_t g = blockIdx.x * (int64_t)kCB + threadIdx.x; g < total; g += (int64_t)gridDim.x * kCB) {
        int lo = 0, hi = nlist - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (prefix[mid] <= g) lo = mid;
            else hi = mid - 1;
        }
        const SimDev<T> &S = sims[list[lo]];
        const gptr_t<const SimState> st = glb((const SimState *)S.st);
        if (!st->active) continue;
        const int64_t k = g - prefix[lo];
        const double inv = 1.0 / fix_scale(S);
        const int par = (int)(st->step & 1);
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const gptr_t<int64_t> acc = glb(S.Jacc[c]) + k;
            const int64_t v = *acc;
            if (v != 0) {
                glb(S.J[par][c])[k] = (T)((double)v * inv);
                *acc = 0;
            }
        }
    }
}

}  // namespace

template <typename T>
void launch_wmax(const SimDev<T> *sim, int npatch, hipStream_t st)
{
    hipLaunchKernelGGL((k_wmax<T>), dim3(std::max(1, std::min(npatch, 4096))), dim3(kCB), 0, st, sim);
}

template <typename T>
void launch_jfix(const SimDev<T> *sims, const int *list, const int64_t *prefix, int nlist, int64_t total,
                 hipStream_t st)
{
    if (nlist <= 0 || total <= 0) return;
    const int64_t blocks = std::min<int64_t>((total + kCB - 1) / kCB, 8 * 2048);
    hipLaunchKernelGGL((k_jfix<T>), dim3((unsigned)blocks), dim3(kCB), 0, st, sims, list, prefix, nlist);
}

#define PIC_CURRENT_INST(T)                                                                         \
    template void launch_wmax<T>(const SimDev<T> *, int, hipStream_t);                             \
    template void launch_jfix<T>(const SimDev<T> *, const int *, const int64_t *, int, int64_t,    \
                                 hipStream_t);
PIC_CURRENT_INST(float)
PIC_CURRENT_INST(double)

}  // namespace pic
