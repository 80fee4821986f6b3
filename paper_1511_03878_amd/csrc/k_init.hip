// Particle loading on the device from a species description (pic_particles_init).
//
// Particles are made cell by cell in row-major cell order (x fastest), k = 0
// .. count - 1 inside a cell; that order is the id order.  Work is split
// into row segments: the cells of one grid row (fixed y, z) inside one patch
// column.  A first pass counts each segment's particles; the host turns the
// counts into the id of each segment's first particle (row-major prefix) and
// its first slot inside its patch (the patch's earlier rows); a second pass
// writes every particle straight into its patch slot, so the initial order
// inside a patch is id order.
//
// Random numbers: SplitMix64 (Steele, Lea and Flood, OOPSLA 2014) in counter
// form.  The generator's state grows by gamma = 0x9E3779B97F4A7C15 per output
// and each output is the state after two xor-shift-multiply rounds and an
// xor-shift, so output c of the generator seeded with s is a function of
// s + (c + 1) gamma alone.  Draw d of particle g in stream r uses counter
// r 2^44 + 8 g + d; a uniform double is the top 53 bits times 2^-53.  Stream
// 0 holds the position draws (one per axis), stream 1 the momentum draws
// (Box-Muller on draws 0, 1 and 2, 3).
#include <algorithm>

#include "kernels.h"
#include "particle_common.h"

namespace pic {

namespace {

__device__ __forceinline__ uint64_t sm64(uint64_t seed, uint64_t c)
{
    uint64_t z = seed + (c + 1ull) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

__device__ __forceinline__ double unit_draw(uint64_t seed, uint64_t stream, int64_t g, int d)
{
    return (double)(sm64(seed, (stream << 44) + ((uint64_t)g << 3) + (uint64_t)d) >> 11) * 0x1.0p-53;
}

// Plasma density at a point given in cell units (no fused multiply-adds, so
// the values equal a plain IEEE evaluation of the same expressions).
__device__ double density(const InitSpec &sp, const double x[3])
{
#pragma clang fp contract(off)
    if (sp.profile == kProfileRamp) {
        const double X0 = sp.p[0] / sp.d[0], X1 = sp.p[1] / sp.d[0];
        if (x[0] < X0) return 0.0;
        if (X1 <= X0 || x[0] >= X1) return sp.n0;
        return sp.n0 * ((x[0] - X0) / (X1 - X0));
    }
    if (sp.profile == kProfileCosSphere) {
        double r2 = 0.0;
        for (int a = 0; a < sp.nd; ++a) {
            const double e = x[a] * sp.d[a] - sp.p[1 + a];
            r2 = r2 + e * e;
        }
        if (r2 <= sp.p[4] * sp.p[4]) return sp.p[5] * sp.n0;
        const double c = cos(2.0 * M_PI * x[0] / (double)sp.n[0]);
        return sp.n0 * (1.0 + sp.p[0] * c);
    }
    return sp.n0;
}

__device__ int cell_particles(const InitSpec &sp, int i, int j, int k)
{
#pragma clang fp contract(off)
    if (sp.profile == kProfileRamp) return (double)i >= sp.p[0] / sp.d[0] ? sp.ppc : 0;
    const double xc[3] = {(double)i + 0.5, (double)j + 0.5, (double)k + 0.5};
    const double nn = density(sp, xc);
    if (sp.loading == kLoadCount) return (int)rint((double)sp.ppc * nn / sp.n0);
    return nn > 0.0 ? sp.ppc : 0;
}

// Segment s: grid row r = s / np0 (y + n1 z), patch column px = s % np0.
__global__ void k_init_count(InitSpec sp, int64_t nseg, int64_t *__restrict__ seg)
{
    for (int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; s < nseg;
         s += (int64_t)gridDim.x * blockDim.x) {
        const int px = (int)(s % sp.np[0]);
        const int64_t r = s / sp.np[0];
        const int j = (int)(r % sp.n[1]), k = (int)(r / sp.n[1]);
        int64_t c = 0;
        for (int i = px * sp.P[0]; i < (px + 1) * sp.P[0]; ++i) c += cell_particles(sp, i, j, k);
        seg[s] = c;
    }
}

template <typename T>
__global__ void k_init_fill(InitSpec sp, int64_t nseg, const int64_t *__restrict__ first,
                            const int32_t *__restrict__ slot0, const SimDev<T> *__restrict__ S)
{
#pragma clang fp contract(off)
    const T pmax[3] = {below((T)sp.P[0]), below((T)sp.P[1]), below((T)sp.P[2])};
    for (int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; s < nseg;
         s += (int64_t)gridDim.x * blockDim.x) {
        const int px = (int)(s % sp.np[0]);
        const int64_t r = s / sp.np[0];
        const int j = (int)(r % sp.n[1]), k = (int)(r / sp.n[1]);
        const int p = px + sp.np[0] * (j / sp.P[1] + sp.np[1] * (k / sp.P[2]));
        const int o[3] = {px * sp.P[0], (j / sp.P[1]) * sp.P[1], (k / sp.P[2]) * sp.P[2]};
        const int64_t base = S->off[p] + slot0[s];
        int64_t g = first[s], t = 0;
        for (int i = px * sp.P[0]; i < (px + 1) * sp.P[0]; ++i) {
            const int cnt = cell_particles(sp, i, j, k);
            const int cell[3] = {i, j, k};
            for (int q = 0; q < cnt; ++q, ++g, ++t) {
                double x[3] = {0.0, 0.0, 0.0};
                for (int a = 0; a < sp.nd; ++a) {
                    x[a] = (double)cell[a] + unit_draw(sp.seed, 0, g, a);
                    if (x[a] >= (double)(cell[a] + 1)) x[a] = nextafter((double)(cell[a] + 1), 0.0);
                }
                double w;
                if (sp.profile == kProfileRamp) {
                    w = density(sp, x) / sp.ppc;
                } else if (sp.loading == kLoadCount) {
                    w = sp.n0 / sp.ppc;
                } else {
                    const double xc[3] = {(double)i + 0.5, (double)j + 0.5, (double)k + 0.5};
                    w = density(sp, xc) / sp.ppc;
                }
                double u[3] = {0.0, 0.0, 0.0};
                if (sp.sigma > 0.0) {
                    const double ra = sqrt(-2.0 * log(1.0 - unit_draw(sp.seed, 1, g, 0)));
                    const double rb = sqrt(-2.0 * log(1.0 - unit_draw(sp.seed, 1, g, 2)));
                    const double fa = 2.0 * M_PI * unit_draw(sp.seed, 1, g, 1);
                    const double fb = 2.0 * M_PI * unit_draw(sp.seed, 1, g, 3);
                    u[0] = sp.sigma * ra * cos(fa);
                    u[1] = sp.sigma * ra * sin(fa);
                    u[2] = sp.sigma * rb * cos(fb);
                }
                const int64_t slot = base + t;
                for (int a = 0; a < sp.nd; ++a) {
                    T loc = (T)(x[a] - (double)o[a]);
                    if (loc > pmax[a]) loc = pmax[a];
                    if (loc < T(0)) loc = T(0);
                    S->pos[slot * S->pw + a] = loc;
                }
                v4(S->mom)[slot] = Vec4<T>{(T)u[0], (T)u[1], (T)u[2], (T)w};
                if (sp.nd == 3) S->pos[slot * 4 + 3] = id_pad<T>(g);
                else S->id[slot] = g;
                S->code[slot] = (uint8_t)(sp.nd == 3 ? kStay3 : kStay2);
            }
        }
    }
}

int grid_for(int64_t n)
{
    return (int)std::max<int64_t>(1, std::min<int64_t>((n + 255) / 256, 1 << 16));
}

}  // namespace

void launch_init_count(const InitSpec &sp, int64_t nseg, int64_t *seg, hipStream_t st)
{
    hipLaunchKernelGGL(k_init_count, dim3(grid_for(nseg)), dim3(256), 0, st, sp, nseg, seg);
}

template <typename T>
void launch_init_fill(const InitSpec &sp, int64_t nseg, const int64_t *first, const int32_t *slot0,
                      const SimDev<T> *sim, hipStream_t st)
{
    hipLaunchKernelGGL((k_init_fill<T>), dim3(grid_for(nseg)), dim3(256), 0, st, sp, nseg, first, slot0,
                       sim);
}

template void launch_init_fill<float>(const InitSpec &, int64_t, const int64_t *, const int32_t *,
                                      const SimDev<float> *, hipStream_t);
template void launch_init_fill<double>(const InitSpec &, int64_t, const int64_t *, const int32_t *,
                                       const SimDev<double> *, hipStream_t);

}  // namespace pic
