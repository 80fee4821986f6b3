// Moving window along x (2-D, open x faces).
//
// The laser-wakefield runs follow the pulse over more than a millimetre of
// plasma (sections 2.1 and 2.3), which a box of fixed size covers only if it
// moves with the pulse.  With the patch structure (section 3.1) a jump of one
// patch column is a relabelling: patch (px, py) takes the particle segment of
// patch (px + 1, py) with its count and capacity, unchanged (positions are
// stored relative to the patch), the segment of the dropped column (0, py)
// becomes the new last column and receives the injected plasma, and the
// fields and currents move left by P[0] nodes with zeros entering at the
// right.  No particle is copied.
//
// The jump is due at the end of step n when floor(v (n + 1 - start) dt /
// (P[0] dx)), evaluated in FP64, exceeds the jumps done so far.  It runs
// between the re-binning and the step close (the close then advances the
// jump counter and the next particle id), so the next step's work queue is
// built on the new layout.

#include <hip/hip_runtime.h>

#include "kernels.h"
#include "pic_dev.h"

namespace pic {
namespace {

constexpr int kWB = 256;       // threads per workgroup
constexpr int kWRow = 16;      // patch columns held per thread while a row rotates (np[0] <= 4096)
constexpr int kWFields = 9;    // E, B of the next step and the last deposit
static_assert(kWRow * kWB == kWindowMaxPatchColumns, "row rotation covers the largest patch row");

__device__ __forceinline__ double column_density(const double *dens, int64_t ncols, int64_t col)
{
    return glb(dens)[col < ncols ? col : ncols - 1];
}

template <typename T>
__global__ __launch_bounds__(kWB) void k_window2d(const SimDev<T> *__restrict__ sp)
{
    const SimDev<T> &S = *sp;
    if (!S.win) return;
    const gptr_t<SimState> st = glb(S.st);
    // the same test in every workgroup: nothing it reads changes in this kernel
    if (!st->active || !st->rebinned || (st->flags & kFlagPending)) return;
    const int64_t step = st->step;
    const int64_t N = step + 1 - S.wstart;
    if (N <= 0) return;
    const int64_t due = (int64_t)floor(S.wvel * (double)N * S.wdt / ((double)S.P[0] * S.wdx));
    const int64_t done = st->wshift;
    if (due <= done) return;

    const int tid = threadIdx.x;
    const int sh = S.P[0], P1 = S.P[1];
    const int fn0 = S.fn[0], fn1 = S.fn[1];
    const int npx = S.np[0], npy = S.np[1];
    const int nfield = kWFields * fn1;
    const int ppc = S.wppc[0] * S.wppc[1];
    // global column of the first cell of the new last column
    const int64_t col0 = (done + 1) * sh + (int64_t)(npx - 1) * sh;

    for (int u = blockIdx.x; u < nfield + npy; u += gridDim.x) {
        if (u < nfield) {
            // one row of one array, shifted in place left to right in chunks:
            // a chunk reads only nodes beyond everything written before it
            const int c = u / fn1, j = u % fn1;
            T *const arr = c < 6 ? S.F[(step + 1) & 1][c] : S.J[step & 1][c - 6];
            const gptr_t<T> row = glb(arr) + (int64_t)j * fn0;
            constexpr int R = 4;
            for (int i0 = 0; i0 < fn0; i0 += R * kWB) {
                T v[R];
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    const int i = i0 + r * kWB + tid;
                    v[r] = (i + sh < fn0) ? row[i + sh] : T(0);
                }
                __syncthreads();
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    const int i = i0 + r * kWB + tid;
                    if (i < fn0) row[i] = v[r];
                }
                __syncthreads();
            }
            continue;
        }
        // one row of patches: rotate count, capacity and segment one column left
        const int py = u - nfield;
        const int p0 = npx * py;
        gptr_t<int32_t> cnt = glb(S.count) + p0;
        gptr_t<int32_t> cap = glb((int32_t *)S.cap) + p0;
        gptr_t<int64_t> off = glb((int64_t *)S.off) + p0;
        int32_t oc[kWRow], ocap[kWRow];
        int64_t oo[kWRow];
#pragma unroll
        for (int r = 0; r < kWRow; ++r) {
            const int px = tid + r * kWB;
            if (px < npx) { oc[r] = cnt[px]; ocap[r] = cap[px]; oo[r] = off[px]; }
        }
        const int32_t gone = cnt[0], cap0 = cap[0];
        const int64_t seg = off[0];
        // particles injected per patch (the density depends on the column only)
        int per_row = 0;
        for (int il = 0; il < sh; ++il)
            if (column_density(S.wdens, S.wncols, col0 + il) > 0.0) per_row += ppc;
        int ninj = per_row * P1;
        if (ninj > cap0) ninj = -1;  // cannot happen when capacities were set up for the window
        __syncthreads();
#pragma unroll
        for (int r = 0; r < kWRow; ++r) {
            const int px = tid + r * kWB;
            if (px < npx) {
                const int q = px == 0 ? npx - 1 : px - 1;
                cnt[q] = px == 0 ? max(ninj, 0) : oc[r];
                cap[q] = ocap[r];
                off[q] = oo[r];
                glb(S.moved)[p0 + q] = 1;
            }
        }
        if (tid == 0) {
            if (gone)
                __hip_atomic_fetch_add(&st->removed, (int64_t)gone, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if (ninj < 0)
                __hip_atomic_fetch_or(&st->flags, kFlagWin, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if (py == 0) {
                st->wadd = (int64_t)max(ninj, 0) * npy;
                st->wpend = 1u;
            }
        }
        if (ninj <= 0) continue;
        // the cold lattice of the new column, in (cell row, cell column, b, a) order
        const int64_t id0 = st->next_id + (int64_t)py * ninj;
        double wloc = 0.0;  // largest injected weight of this thread
        for (int t = tid; t < ninj; t += kWB) {
            const int jl = t / per_row, rem = t - jl * per_row;
            int k = rem / ppc;
            const int m = rem - k * ppc;
            // the k-th column of the patch that holds plasma
            int il = 0;
            for (int c = 0; c < sh; ++c)
                if (column_density(S.wdens, S.wncols, col0 + c) > 0.0 && k-- == 0) {
                    il = c;
                    break;
                }
            const int b = m / S.wppc[0], a = m - b * S.wppc[0];
            const double dens = column_density(S.wdens, S.wncols, col0 + il);
            const int64_t slot = seg + t;
            // (the window is 2-D: two position entries per slot)
            v2(S.pos)[slot] = Vec2<T>{(T)((double)il + ((double)a + 0.5) / S.wppc[0]),
                                   (T)((double)jl + ((double)b + 0.5) / S.wppc[1])};
            v4(S.mom)[slot] = Vec4<T>{T(0), T(0), T(0), (T)(dens / ppc)};
            wloc = fmax(wloc, fabs((double)(T)(dens / ppc)));
            glb(S.id)[slot] = id0 + t;
            glb(S.code)[slot] = (uint8_t)kStay2;
        }
        // the bound behind the fixed-point current scale covers the new weights
        if (wloc > 0.0) raise_wmax(S, wloc);
    }
}

}  // namespace

template <typename T>
void launch_window(const SimDev<T> *sim, int fn1, int npy, hipStream_t st)
{
    const int units = kWFields * fn1 + npy;
    hipLaunchKernelGGL((k_window2d<T>), dim3(std::min(units, 2048)), dim3(kWB), 0, st, sim);
}

template void launch_window<float>(const SimDev<float> *, int, int, hipStream_t);
template void launch_window<double>(const SimDev<double> *, int, int, hipStream_t);

}  // namespace pic
