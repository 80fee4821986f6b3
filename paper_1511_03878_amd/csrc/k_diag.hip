// Diagnostics of a simulation, off the timed path: the charge density of the
// particles on primal nodes (2-D and 3-D), and the node reductions behind the
// Gauss and continuity residuals.
//
// rho[node] = q sum_p w_p prod_a S2(xi_p,a - node_a) with the quadratic
// B-spline S2 (the charge assignment that goes with the quadratic gather);
// it is accumulated in FP64 with device-scope atomics into a caller-given
// array of fn[0] fn[1] fn[2] doubles that the caller has cleared.
//
// Residuals (evaluated in FP64 at primal nodes, with J on E's staggered
// positions so that div J and div E sit on primal nodes):
//   Gauss:       div E^k - (rho^k - rho^0)   (rho^0: the particles' charge at
//                load; the immobile ions carry -rho^0, so the total charge is
//                rho^k - rho^0 and E = 0 at t = 0 makes the residual 0 then);
//   continuity:  rho^k - rho^{k-1} + dt div J^{k-1/2}.
// Nodes within three cells of an open face are left out: a particle absorbed
// there takes its charge with it after depositing its whole move, which
// breaks both identities on the nodes its shape still covered.
#include "runtime.h"

namespace pic {

namespace {

__global__ void k_fill(double *__restrict__ p, int64_t n, double v)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

__device__ __forceinline__ void sweights(double d, double w[3])
{
    w[0] = 0.5 * (0.5 - d) * (0.5 - d);
    w[1] = 0.75 - d * d;
    w[2] = 0.5 * (0.5 + d) * (0.5 + d);
}

// One workgroup per patch; every particle adds its 3^ND node charges.
template <typename T, int ND>
__global__ void k_rho(const SimDev<T> *__restrict__ S, double *__restrict__ out)
{
    const int p = blockIdx.x;
    const int n = S->count[p];
    const int64_t base = S->off[p];
    const int o[3] = {(p % S->np[0]) * S->P[0], ((p / S->np[0]) % S->np[1]) * S->P[1],
                      (p / (S->np[0] * S->np[1])) * S->P[2]};
    constexpr int PW = ND == 3 ? 4 : 2;
    const gptr_t<const T> X = glb((const T *)S->pos) + PW * base;
    const gptr_t<const T> M = glb((const T *)S->mom) + 4 * base;
    const double q = (double)S->q;
    const int64_t fn0 = S->fn[0], fn1 = S->fn[1];
    for (int k = threadIdx.x; k < n; k += blockDim.x) {
        const double xs[3] = {(double)X[PW * k], (double)X[PW * k + 1], ND == 3 ? (double)X[PW * k + 2] : 0.0};
        const double qw = q * (double)M[4 * k + 3];
        int i0[3];
        double w[3][3];
        for (int a = 0; a < ND; ++a) {
            i0[a] = (int)floor(xs[a] + 0.5);
            sweights(xs[a] - i0[a], w[a]);
        }
        const int nc = ND == 3 ? 3 : 1;
        for (int c = 0; c < nc; ++c) {
            const int gk = ND == 3 ? axis_node(o[2] + i0[2] + c - 1, S->n[2], S->periodic[2], 0) : 0;
            const double wz = ND == 3 ? w[2][c] : 1.0;
            for (int b = 0; b < 3; ++b) {
                const int gj = axis_node(o[1] + i0[1] + b - 1, S->n[1], S->periodic[1], 0);
                for (int a = 0; a < 3; ++a) {
                    const int gi = axis_node(o[0] + i0[0] + a - 1, S->n[0], S->periodic[0], 0);
                    if (gi >= 0 && gj >= 0 && gk >= 0)
                        atomicAdd(&out[gi + fn0 * (gj + fn1 * gk)], qw * w[0][a] * w[1][b] * wz);
                }
            }
        }
    }
}

__device__ __forceinline__ double wave_max(double v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
    return v;
}

constexpr int kResBlock = 256;
constexpr int kResMaxBlocks = 2048;

// Per node: |Gauss residual|, |continuity residual|, |rho^k|, |rho^0|; the
// maxima of each workgroup go to partials[4 * block + m].
template <typename T, int ND>
__global__ __launch_bounds__(kResBlock) void k_residual_nodes(
    const SimDev<T> *__restrict__ S, int fpar, int jpar, const double *__restrict__ rho,
    const double *__restrict__ rho0, const double *__restrict__ rho_prev, double *__restrict__ partials)
{
    __shared__ double red[4][kResBlock / 64];
    const int n0 = S->n[0], n1 = S->n[1], n2 = S->n[2];
    const int fn0 = S->fn[0], fn1 = S->fn[1], fn2 = ND == 3 ? S->fn[2] : 1;
    const int64_t fsize = (int64_t)fn0 * fn1 * fn2;
    const bool openx = !S->periodic[0];
    const double idx = 1.0 / (double)S->d[0], idy = 1.0 / (double)S->d[1];
    const double idz = ND == 3 ? 1.0 / (double)S->d[2] : 0.0;
    const double dt = (double)S->dt;
    const gptr_t<const T> Ex = glb((const T *)S->F[fpar][0]), Ey = glb((const T *)S->F[fpar][1]);
    const gptr_t<const T> Ez = glb((const T *)S->F[fpar][2]);
    const gptr_t<const T> Jx = glb((const T *)S->J[jpar][0]), Jy = glb((const T *)S->J[jpar][1]);
    const gptr_t<const T> Jz = glb((const T *)S->J[jpar][2]);
    double m[4] = {0.0, 0.0, 0.0, 0.0};
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < fsize;
         t += (int64_t)gridDim.x * blockDim.x) {
        const int i = (int)(t % fn0), j = (int)((t / fn0) % fn1), k = (int)(t / ((int64_t)fn0 * fn1));
        // backward neighbours along each axis (periodic wrap; an open x axis
        // has no node below 0 and is skipped there)
        const int im = i == 0 ? (openx ? 0 : n0 - 1) : i - 1;
        const int jm = j == 0 ? n1 - 1 : j - 1;
        const int km = ND == 3 ? (k == 0 ? n2 - 1 : k - 1) : 0;
        const int64_t rowb = (int64_t)fn0 * (j + (int64_t)fn1 * k);
        const int64_t tx = im + rowb;
        const int64_t ty = i + (int64_t)fn0 * (jm + (int64_t)fn1 * k);
        const int64_t tz = i + (int64_t)fn0 * (j + (int64_t)fn1 * km);
        double divE = ((double)Ex[t] - (double)Ex[tx]) * idx + ((double)Ey[t] - (double)Ey[ty]) * idy;
        double divJ = ((double)Jx[t] - (double)Jx[tx]) * idx + ((double)Jy[t] - (double)Jy[ty]) * idy;
        if (ND == 3) {
            divE += ((double)Ez[t] - (double)Ez[tz]) * idz;
            divJ += ((double)Jz[t] - (double)Jz[tz]) * idz;
        }
        const double r = rho[t];
        const bool inner = !openx || (i >= 3 && i <= n0 - 3);
        if (inner && rho0) m[0] = fmax(m[0], fabs(divE - (r - rho0[t])));
        if (inner && rho_prev) m[1] = fmax(m[1], fabs(r - rho_prev[t] + dt * divJ));
        m[2] = fmax(m[2], fabs(r));
        if (rho0) m[3] = fmax(m[3], fabs(rho0[t]));
    }
    const int wv = threadIdx.x / 64, ln = threadIdx.x % 64;
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        const double v = wave_max(m[c]);
        if (ln == 0) red[c][wv] = v;
    }
    __syncthreads();
    if (threadIdx.x < 4) {
        double v = 0.0;
        for (int w = 0; w < kResBlock / 64; ++w) v = fmax(v, red[threadIdx.x][w]);
        partials[4 * blockIdx.x + threadIdx.x] = v;
    }
}

__global__ void k_residual_final(const double *__restrict__ partials, int nblocks, double *__restrict__ out)
{
    __shared__ double red[4][4];
    const int wv = threadIdx.x / 64, ln = threadIdx.x % 64;
    for (int c = 0; c < 4; ++c) {
        double v = 0.0;
        for (int b = threadIdx.x; b < nblocks; b += blockDim.x) v = fmax(v, partials[4 * b + c]);
        v = wave_max(v);
        if (ln == 0) red[c][wv] = v;
    }
    __syncthreads();
    if (threadIdx.x < 4) out[threadIdx.x] = fmax(fmax(red[threadIdx.x][0], red[threadIdx.x][1]),
                                                 fmax(red[threadIdx.x][2], red[threadIdx.x][3]));
}

__global__ void k_copy_int(const int *__restrict__ src, int *__restrict__ dst)
{
    if (threadIdx.x == 0) *dst = *src;
}

}  // namespace

void launch_copy_int(const int *src, int *dst, hipStream_t st)
{
    hipLaunchKernelGGL(k_copy_int, dim3(1), dim3(64), 0, st, src, dst);
}

void fill_doubles(double *p, int64_t n, double v, hipStream_t st)
{
    if (n <= 0) return;
    const int grid = (int)std::min<int64_t>((n + 255) / 256, 4096);
    hipLaunchKernelGGL(k_fill, dim3(grid), dim3(256), 0, st, p, n, v);
}

template <typename T>
void launch_rho(const SimDev<T> *sim, int npatch, int ndim, double *out, hipStream_t st)
{
    if (npatch <= 0) return;
    if (ndim == 3)
        hipLaunchKernelGGL((k_rho<T, 3>), dim3(npatch), dim3(256), 0, st, sim, out);
    else
        hipLaunchKernelGGL((k_rho<T, 2>), dim3(npatch), dim3(256), 0, st, sim, out);
}

template <typename T>
void launch_residuals(const SimDev<T> *sim, int ndim, int64_t fsize, int fpar, int jpar,
                      const double *rho, const double *rho0, const double *rho_prev,
                      double *partials, double *out, hipStream_t st)
{
    const int nb = (int)std::max<int64_t>(1, std::min<int64_t>((fsize + kResBlock - 1) / kResBlock,
                                                                kResMaxBlocks));
    if (ndim == 3)
        hipLaunchKernelGGL((k_residual_nodes<T, 3>), dim3(nb), dim3(kResBlock), 0, st, sim, fpar, jpar,
                           rho, rho0, rho_prev, partials);
    else
        hipLaunchKernelGGL((k_residual_nodes<T, 2>), dim3(nb), dim3(kResBlock), 0, st, sim, fpar, jpar,
                           rho, rho0, rho_prev, partials);
    hipLaunchKernelGGL(k_residual_final, dim3(1), dim3(256), 0, st, partials, nb, out);
}

int residual_partials() { return 4 * kResMaxBlocks; }

#define PIC_INST(T)                                                                                \
    template void launch_rho<T>(const SimDev<T> *, int, int, double *, hipStream_t);              \
    template void launch_residuals<T>(const SimDev<T> *, int, int64_t, int, int, const double *,  \
                                      const double *, const double *, double *, double *,         \
                                      hipStream_t);
PIC_INST(float)
PIC_INST(double)
#undef PIC_INST

}  // namespace pic
