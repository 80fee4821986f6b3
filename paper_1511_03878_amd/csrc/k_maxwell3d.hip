// Yee update of the 3-D patch-PIC step on a periodic box, as three passes
// over the nodes (one thread per node, neighbours through the caches):
//   1. B^{n+1/2} = B^n - dt/2 curl E^n          (read F[n & 1], write B of F[(n+1) & 1])
//      and the field energy of E^n, B^n per block of 256 nodes;
//   2. E^{n+1} = E^n + dt (curl B^{n+1/2} - J)   (write E of F[(n+1) & 1]; clear the
//      other J buffer, which the next step deposits into);
//   3. B^{n+1} = B^{n+1/2} - dt/2 curl E^{n+1}   (in place: a node's B reads only its
//      own B and neighbouring E).
// B updates take forward differences of E, E updates backward differences of B;
// staggering as in the particle kernel.  A "tile" here is a block of 256
// consecutive nodes (x fastest) of one simulation.  A simulation with the
// sixth-order solver takes the same passes with the three-pair staggered
// differences (weights 75/64, -25/384, 3/640) in place of the two-point ones.
#include "kernels.h"

namespace pic {

namespace {

constexpr int kMB = 256;

struct Node3 {
    int64_t k;                // flat index
    int64_t ip, jp, kp;       // flat index of the +1 neighbour along x, y, z
    int64_t im, jm, km;       // flat index of the -1 neighbour along x, y, z
};

__device__ __forceinline__ Node3 node3(int64_t k, int fn0, int fn1, int fn2)
{
    const int i = (int)(k % fn0), j = (int)((k / fn0) % fn1), l = (int)(k / ((int64_t)fn0 * fn1));
    const int64_t sx = 1, sy = fn0, sz = (int64_t)fn0 * fn1;
    Node3 r;
    r.k = k;
    r.ip = k + (i + 1 < fn0 ? sx : -(int64_t)(fn0 - 1) * sx);
    r.im = k + (i > 0 ? -sx : (int64_t)(fn0 - 1) * sx);
    r.jp = k + (j + 1 < fn1 ? sy : -(int64_t)(fn1 - 1) * sy);
    r.jm = k + (j > 0 ? -sy : (int64_t)(fn1 - 1) * sy);
    r.kp = k + (l + 1 < fn2 ? sz : -(int64_t)(fn2 - 1) * sz);
    r.km = k + (l > 0 ? -sz : (int64_t)(fn2 - 1) * sz);
    return r;
}

// Sixth-order staggered difference of f along the axis with node index i of
// n (stride between neighbours `stride`), periodic: forward (the half point
// after node k) or backward (the half point before it).
template <typename T>
__device__ __forceinline__ T d6(const gptr_t<const T> f, int64_t k, int64_t stride, int i, int n, bool fwd)
{
    auto at = [&](int o) {
        int ii = i + o;
        ii += ii < 0 ? n : 0;
        ii -= ii >= n ? n : 0;
        return f[k + (int64_t)(ii - i) * stride];
    };
    const T c1 = T(75.0 / 64.0), c2 = T(-25.0 / 384.0), c3 = T(3.0 / 640.0);
    return fwd ? c1 * (at(1) - at(0)) + c2 * (at(2) - at(-1)) + c3 * (at(3) - at(-2))
               : c1 * (at(0) - at(-1)) + c2 * (at(1) - at(-2)) + c3 * (at(2) - at(-3));
}

// pass 1 (PASS = 0) and pass 3 (PASS = 2): B -= h curl E
template <typename T, int PASS>
__global__ __launch_bounds__(kMB) void k_maxwell3d_b(const SimDev<T> *__restrict__ sims, int nsims,
                                                     const int *__restrict__ tile_prefix, int total)
{
    __shared__ double s_red[kMB / 64];
    for (int tile = blockIdx.x; tile < total; tile += gridDim.x) {
        const int s = find_sim(tile_prefix, nsims, tile);
        const SimDev<T> &S = sims[s];
        if (!glb(S.st)->active) continue;
        const int lt = tile - tile_prefix[s];
        const int fn0 = S.fn[0], fn1 = S.fn[1], fn2 = S.fn[2];
        const int64_t fsize = (int64_t)fn0 * fn1 * fn2;
        const int64_t stepn = glb(S.st)->step;
        T *const *Fc = S.F[stepn & 1];
        T *const *Fn = S.F[(stepn + 1) & 1];
        // E^n and B^n for the first half, E^{n+1} and B^{n+1/2} for the second
        T *const *Esrc = PASS == 0 ? Fc : Fn;
        T *const *Bsrc = PASS == 0 ? Fc : Fn;
        const T h = T(0.5) * S.dt;
        const T ix = T(1) / S.d[0], iy = T(1) / S.d[1], iz = T(1) / S.d[2];
        const int64_t k = (int64_t)lt * kMB + threadIdx.x;
        double esum = 0.0;
        if (k < fsize) {
            const Node3 nd = node3(k, fn0, fn1, fn2);
            const gptr_t<const T> Ex = glb((const T *)Esrc[0]), Ey = glb((const T *)Esrc[1]),
                                  Ez = glb((const T *)Esrc[2]);
            const T ex = Ex[k], ey = Ey[k], ez = Ez[k];
            const T bx = glb((const T *)Bsrc[3])[k], by = glb((const T *)Bsrc[4])[k],
                    bz = glb((const T *)Bsrc[5])[k];
            if (PASS == 0) {
                esum = (double)ex * ex + (double)ey * ey + (double)ez * ez + (double)bx * bx +
                       (double)by * by + (double)bz * bz;
            }
            if (S.morder == 6) {
                const int i = (int)(k % fn0), j = (int)((k / fn0) % fn1), l = (int)(k / ((int64_t)fn0 * fn1));
                const int64_t sy = fn0, sz = (int64_t)fn0 * fn1;
                auto dx = [&](gptr_t<const T> f) { return d6<T>(f, k, 1, i, fn0, true); };
                auto dy = [&](gptr_t<const T> f) { return d6<T>(f, k, sy, j, fn1, true); };
                auto dz = [&](gptr_t<const T> f) { return d6<T>(f, k, sz, l, fn2, true); };
                glb(Fn[3])[k] = bx - h * (dy(Ez) * iy - dz(Ey) * iz);
                glb(Fn[4])[k] = by - h * (dz(Ex) * iz - dx(Ez) * ix);
                glb(Fn[5])[k] = bz - h * (dx(Ey) * ix - dy(Ex) * iy);
            } else {
                glb(Fn[3])[k] = bx - h * ((Ez[nd.jp] - ez) * iy - (Ey[nd.kp] - ey) * iz);
                glb(Fn[4])[k] = by - h * ((Ex[nd.kp] - ex) * iz - (Ez[nd.ip] - ez) * ix);
                glb(Fn[5])[k] = bz - h * ((Ey[nd.ip] - ey) * ix - (Ex[nd.jp] - ex) * iy);
            }
        }
        if (PASS == 0) {
#pragma unroll
            for (int o = 32; o > 0; o >>= 1) esum += __shfl_xor(esum, o, 64);
            if ((threadIdx.x & 63) == 0) s_red[threadIdx.x >> 6] = esum;
            __syncthreads();
            if (threadIdx.x == 0) {
                double tot = 0.0;
                for (int w = 0; w < kMB / 64; ++w) tot += s_red[w];
                glb(S.upart)[lt] = 0.5 * S.vcell * tot;
            }
            __syncthreads();
        }
    }
}

// pass 2: E += dt (curl B - J); clear the next step's J
template <typename T>
__global__ __launch_bounds__(kMB) void k_maxwell3d_e(const SimDev<T> *__restrict__ sims, int nsims,
                                                     const int *__restrict__ tile_prefix, int total)
{
    for (int tile = blockIdx.x; tile < total; tile += gridDim.x) {
        const int s = find_sim(tile_prefix, nsims, tile);
        const SimDev<T> &S = sims[s];
        if (!glb(S.st)->active) continue;
        const int lt = tile - tile_prefix[s];
        const int fn0 = S.fn[0], fn1 = S.fn[1], fn2 = S.fn[2];
        const int64_t fsize = (int64_t)fn0 * fn1 * fn2;
        const int64_t stepn = glb(S.st)->step;
        T *const *Fc = S.F[stepn & 1];
        T *const *Fn = S.F[(stepn + 1) & 1];
        T *const *Jc = S.J[stepn & 1];
        T *const *Jn = S.J[(stepn + 1) & 1];
        const T dt = S.dt;
        const T ix = T(1) / S.d[0], iy = T(1) / S.d[1], iz = T(1) / S.d[2];
        const int64_t k = (int64_t)lt * kMB + threadIdx.x;
        if (k >= fsize) continue;
        const Node3 nd = node3(k, fn0, fn1, fn2);
        const gptr_t<const T> Bx = glb((const T *)Fn[3]), By = glb((const T *)Fn[4]),
                              Bz = glb((const T *)Fn[5]);
        const T bx = Bx[k], by = By[k], bz = Bz[k];
        if (S.morder == 6) {
            const int i = (int)(k % fn0), j = (int)((k / fn0) % fn1), l = (int)(k / ((int64_t)fn0 * fn1));
            const int64_t sy = fn0, sz = (int64_t)fn0 * fn1;
            auto dx = [&](gptr_t<const T> f) { return d6<T>(f, k, 1, i, fn0, false); };
            auto dy = [&](gptr_t<const T> f) { return d6<T>(f, k, sy, j, fn1, false); };
            auto dz = [&](gptr_t<const T> f) { return d6<T>(f, k, sz, l, fn2, false); };
            glb(Fn[0])[k] = glb((const T *)Fc[0])[k] + dt * (dy(Bz) * iy - dz(By) * iz - glb((const T *)Jc[0])[k]);
            glb(Fn[1])[k] = glb((const T *)Fc[1])[k] + dt * (dz(Bx) * iz - dx(Bz) * ix - glb((const T *)Jc[1])[k]);
            glb(Fn[2])[k] = glb((const T *)Fc[2])[k] + dt * (dx(By) * ix - dy(Bx) * iy - glb((const T *)Jc[2])[k]);
            glb(Jn[0])[k] = T(0);
            glb(Jn[1])[k] = T(0);
            glb(Jn[2])[k] = T(0);
            continue;
        }
        glb(Fn[0])[k] = glb((const T *)Fc[0])[k] +
                        dt * ((bz - Bz[nd.jm]) * iy - (by - By[nd.km]) * iz - glb((const T *)Jc[0])[k]);
        glb(Fn[1])[k] = glb((const T *)Fc[1])[k] +
                        dt * ((bx - Bx[nd.km]) * iz - (bz - Bz[nd.im]) * ix - glb((const T *)Jc[1])[k]);
        glb(Fn[2])[k] = glb((const T *)Fc[2])[k] +
                        dt * ((by - By[nd.im]) * ix - (bx - Bx[nd.jm]) * iy - glb((const T *)Jc[2])[k]);
        glb(Jn[0])[k] = T(0);
        glb(Jn[1])[k] = T(0);
        glb(Jn[2])[k] = T(0);
    }
}

}  // namespace

template <typename T>
void launch_maxwell3d(const SimDev<T> *sims, int nsims, const int *tile_prefix, int total_tiles,
                      int grid, hipStream_t st, Ev2 ev)
{
    hipExtLaunchKernelGGL((k_maxwell3d_b<T, 0>), dim3(grid), dim3(kMB), 0, st, ev.start, nullptr, 0,
                          sims, nsims, tile_prefix, total_tiles);
    hipLaunchKernelGGL((k_maxwell3d_e<T>), dim3(grid), dim3(kMB), 0, st, sims, nsims, tile_prefix,
                       total_tiles);
    hipExtLaunchKernelGGL((k_maxwell3d_b<T, 2>), dim3(grid), dim3(kMB), 0, st, nullptr, ev.stop, 0,
                          sims, nsims, tile_prefix, total_tiles);
}

template void launch_maxwell3d<float>(const SimDev<float> *, int, const int *, int, int, hipStream_t,
                                      Ev2);
template void launch_maxwell3d<double>(const SimDev<double> *, int, const int *, int, int,
                                       hipStream_t, Ev2);

}  // namespace pic
