// Field update of the 3-D patch-PIC step on a periodic box.  The Yee solver
// runs as one fused kernel over blocks of nodes (k_maxwell3d_yee, below); the
// sixth-order solver as three passes over the nodes (one thread per node,
// neighbours through the caches):
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

// Tiles of workgroup b.  Workgroups are dispatched to the 8 XCDs in turn
// (workgroup b to XCD b % 8), each with its own L2; XCD x takes the
// contiguous band [x T / 8, (x + 1) T / 8) of the T tiles and its workgroups
// stride through it, so neighbouring blocks, which share halo nodes, are
// mostly read through the same L2.
struct TileWalk {
    int first, end, step;
};
__device__ __forceinline__ TileWalk tile_walk(int total)
{
    const int g = (int)gridDim.x, b = (int)blockIdx.x;
    if (g & 7) return {b, total, g};
    const int x = b & 7;
    return {(int)((int64_t)total * x / 8) + (b >> 3), (int)((int64_t)total * (x + 1) / 8), g >> 3};
}

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
        if (!glb(S.st)->active || S.morder != 6) continue;
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
        if (!glb(S.st)->active || S.morder != 6) continue;
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

// ---- fused Yee update of a block of nodes -------------------------------------
//
// Block [X, X + BX) x [Y, Y + BY) x [Z, Z + BZ) of the nodes.  E is staged on
// [X - 1, X + BX + 2) per axis and B on [X - 1, X + BX + 1) (periodic, so a
// block at the grid's end reads its halo from the start), then in LDS
//   B' = B - dt/2 curl E          on the whole B tile (in place),
//   E' = E + dt (curl B' - J)     on [X, X + BX + 1) per axis (in place; J
//                                  is loaded into registers with the tiles),
//   B'' = B' - dt/2 curl E'       on the block,
// and E', B'' of the block are written to the other field buffer and the
// block's nodes of the other J buffer cleared: the three passes' arithmetic
// in the same order, with HBM reads of E, B and J once per node plus the
// halo.  Both tiles start at X - 1, so a node has the same local coordinates
// in each.  Nodes of a block past the grid's end (n not a multiple of the
// block) are computed from wrapped data and not written.
constexpr int kYT = 256;                                          // threads
constexpr int kEX = kYee3X + 3, kEY = kYee3Y + 3, kEZ = kYee3Z + 3;  // E tile
constexpr int kBX = kYee3X + 2, kBY = kYee3Y + 2, kBZ = kYee3Z + 2;  // B tile
constexpr int kEN = kEX * kEY * kEZ, kBN = kBX * kBY * kBZ;
constexpr int kE2X = kYee3X + 1, kE2Y = kYee3Y + 1, kE2Z = kYee3Z + 1;  // E' nodes
constexpr int kE2N = kE2X * kE2Y * kE2Z;
constexpr int kON = kYee3X * kYee3Y * kYee3Z;  // the block's own nodes
constexpr int kRE = (kEN + kYT - 1) / kYT, kRB = (kBN + kYT - 1) / kYT, kRJ = (kE2N + kYT - 1) / kYT;
static_assert(kON % kYT == 0, "own nodes per thread");

template <typename T>
__global__ __launch_bounds__(kYT) void k_maxwell3d_yee(const SimDev<T> *__restrict__ sims, int nsims,
                                                       const int *__restrict__ tile_prefix, int total)
{
    __shared__ T sE[3][kEN];
    __shared__ T sB[3][kBN];
    __shared__ int s_wrap[kEX + kEY + kEZ];  // wrapped node index of each local index, per axis
    __shared__ double s_red[kYT / 64];
    const int tid = threadIdx.x;
    const TileWalk tw = tile_walk(total);
    for (int tile = tw.first; tile < tw.end; tile += tw.step) {
        const int s = find_sim(tile_prefix, nsims, tile);
        const SimDev<T> &S = sims[s];
        if (!glb(S.st)->active || S.morder == 6) continue;
        const int lt = tile - tile_prefix[s];
        const int fn0 = S.fn[0], fn1 = S.fn[1], fn2 = S.fn[2];
        const int nbx = (fn0 + kYee3X - 1) / kYee3X, nby = (fn1 + kYee3Y - 1) / kYee3Y;
        // global index of local index 0 on each axis
        const int x0 = (lt % nbx) * kYee3X - 1, y0 = ((lt / nbx) % nby) * kYee3Y - 1,
                  z0 = (lt / (nbx * nby)) * kYee3Z - 1;
        const int64_t stepn = glb(S.st)->step;
        T *const *Fc = S.F[stepn & 1];
        T *const *Fn = S.F[(stepn + 1) & 1];
        T *const *Jc = S.J[stepn & 1];
        T *const *Jn = S.J[(stepn + 1) & 1];
        const T dt = S.dt, h = T(0.5) * S.dt;
        const T ix = T(1) / S.d[0], iy = T(1) / S.d[1], iz = T(1) / S.d[2];
        for (int i = tid; i < kEX + kEY + kEZ; i += kYT) {
            int g, n;
            if (i < kEX) {
                g = x0 + i;
                n = fn0;
            } else if (i < kEX + kEY) {
                g = y0 + i - kEX;
                n = fn1;
            } else {
                g = z0 + i - kEX - kEY;
                n = fn2;
            }
            g %= n;
            s_wrap[i] = g < 0 ? g + n : g;
        }
        __syncthreads();
        const int *wx = s_wrap, *wy = s_wrap + kEX, *wz = s_wrap + kEX + kEY;
        auto gidx = [&](int lx, int ly, int lz) {
            return ((int64_t)wz[lz] * fn1 + wy[ly]) * fn0 + wx[lx];
        };
        // ---- stage E, B; J of the E' nodes into registers (every load from an
        // in-range index; duplicates write the same value) -------------------------
        {
            const gptr_t<const T> E0 = glb((const T *)Fc[0]), E1 = glb((const T *)Fc[1]),
                                  E2 = glb((const T *)Fc[2]);
#pragma unroll
            for (int r = 0; r < kRE; ++r) {
                const int i = min(tid + r * kYT, kEN - 1);
                const int64_t g = gidx(i % kEX, (i / kEX) % kEY, i / (kEX * kEY));
                sE[0][i] = E0[g];
                sE[1][i] = E1[g];
                sE[2][i] = E2[g];
            }
            const gptr_t<const T> B0 = glb((const T *)Fc[3]), B1 = glb((const T *)Fc[4]),
                                  B2 = glb((const T *)Fc[5]);
#pragma unroll
            for (int r = 0; r < kRB; ++r) {
                const int i = min(tid + r * kYT, kBN - 1);
                const int64_t g = gidx(i % kBX, (i / kBX) % kBY, i / (kBX * kBY));
                sB[0][i] = B0[g];
                sB[1][i] = B1[g];
                sB[2][i] = B2[g];
            }
        }
        T jr[3][kRJ];
        {
            const gptr_t<const T> J0 = glb((const T *)Jc[0]), J1 = glb((const T *)Jc[1]),
                                  J2 = glb((const T *)Jc[2]);
#pragma unroll
            for (int r = 0; r < kRJ; ++r) {
                const int j = min(tid + r * kYT, kE2N - 1);
                const int64_t g = gidx(j % kE2X + 1, (j / kE2X) % kE2Y + 1, j / (kE2X * kE2Y) + 1);
                jr[0][r] = J0[g];
                jr[1][r] = J1[g];
                jr[2][r] = J2[g];
            }
        }
        __syncthreads();

        // ---- B' on the B tile, and the energy of E^n, B^n over the block ----------
        double esum = 0.0;
#pragma unroll
        for (int r = 0; r < kRB; ++r) {
            const int i = tid + r * kYT;
            if (i < kBN) {
                const int lx = i % kBX, ly = (i / kBX) % kBY, lz = i / (kBX * kBY);
                const int e = (lz * kEY + ly) * kEX + lx;
                const T ex = sE[0][e], ey = sE[1][e], ez = sE[2][e];
                const T bx = sB[0][i], by = sB[1][i], bz = sB[2][i];
                const bool own = lx >= 1 && lx <= kYee3X && ly >= 1 && ly <= kYee3Y && lz >= 1 &&
                                 lz <= kYee3Z && x0 + lx < fn0 && y0 + ly < fn1 && z0 + lz < fn2;
                if (own)
                    esum += (double)ex * ex + (double)ey * ey + (double)ez * ez + (double)bx * bx +
                            (double)by * by + (double)bz * bz;
                sB[0][i] = bx - h * ((sE[2][e + kEX] - ez) * iy - (sE[1][e + kEX * kEY] - ey) * iz);
                sB[1][i] = by - h * ((sE[0][e + kEX * kEY] - ex) * iz - (sE[2][e + 1] - ez) * ix);
                sB[2][i] = bz - h * ((sE[1][e + 1] - ey) * ix - (sE[0][e + kEX] - ex) * iy);
            }
        }
        __syncthreads();

        // ---- E' on [X, X + BX + 1) per axis -----------------------------------------
#pragma unroll
        for (int r = 0; r < kRJ; ++r) {
            const int j = tid + r * kYT;
            if (j < kE2N) {
                const int lx = j % kE2X + 1, ly = (j / kE2X) % kE2Y + 1, lz = j / (kE2X * kE2Y) + 1;
                const int e = (lz * kEY + ly) * kEX + lx;
                const int b = (lz * kBY + ly) * kBX + lx;
                const T bx = sB[0][b], by = sB[1][b], bz = sB[2][b];
                sE[0][e] = sE[0][e] + dt * ((bz - sB[2][b - kBX]) * iy - (by - sB[1][b - kBX * kBY]) * iz - jr[0][r]);
                sE[1][e] = sE[1][e] + dt * ((bx - sB[0][b - kBX * kBY]) * iz - (bz - sB[2][b - 1]) * ix - jr[1][r]);
                sE[2][e] = sE[2][e] + dt * ((by - sB[1][b - 1]) * ix - (bx - sB[0][b - kBX]) * iy - jr[2][r]);
            }
        }
        __syncthreads();

        // ---- B'' on the block; write E', B'' and clear the other J ---------------
        {
            const gptr_t<T> E0 = glb(Fn[0]), E1 = glb(Fn[1]), E2 = glb(Fn[2]);
            const gptr_t<T> B0 = glb(Fn[3]), B1 = glb(Fn[4]), B2 = glb(Fn[5]);
            const gptr_t<T> J0 = glb(Jn[0]), J1 = glb(Jn[1]), J2 = glb(Jn[2]);
#pragma unroll
            for (int r = 0; r < kON / kYT; ++r) {
                const int o = tid + r * kYT;
                const int lx = o % kYee3X + 1, ly = (o / kYee3X) % kYee3Y + 1, lz = o / (kYee3X * kYee3Y) + 1;
                if (x0 + lx >= fn0 || y0 + ly >= fn1 || z0 + lz >= fn2) continue;
                const int e = (lz * kEY + ly) * kEX + lx;
                const int b = (lz * kBY + ly) * kBX + lx;
                const T ex = sE[0][e], ey = sE[1][e], ez = sE[2][e];
                const int64_t g = ((int64_t)(z0 + lz) * fn1 + (y0 + ly)) * fn0 + (x0 + lx);
                B0[g] = sB[0][b] - h * ((sE[2][e + kEX] - ez) * iy - (sE[1][e + kEX * kEY] - ey) * iz);
                B1[g] = sB[1][b] - h * ((sE[0][e + kEX * kEY] - ex) * iz - (sE[2][e + 1] - ez) * ix);
                B2[g] = sB[2][b] - h * ((sE[1][e + 1] - ey) * ix - (sE[0][e + kEX] - ex) * iy);
                E0[g] = ex;
                E1[g] = ey;
                E2[g] = ez;
                J0[g] = T(0);
                J1[g] = T(0);
                J2[g] = T(0);
            }
        }
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) esum += __shfl_xor(esum, o, 64);
        if ((tid & 63) == 0) s_red[tid >> 6] = esum;
        __syncthreads();
        if (tid == 0) {
            double tot = 0.0;
            for (int w = 0; w < kYT / 64; ++w) tot += s_red[w];
            glb(S.upart)[lt] = 0.5 * S.vcell * tot;
        }
        // (the next block's wrap table and tiles are written after the
        // barrier that follows it)
    }
}

}  // namespace

template <typename T>
void launch_maxwell3d(const SimDev<T> *sims, int nsims, const int *tile_prefix, int total_tiles,
                      int grid, bool yee, bool hi_order, hipStream_t st, Ev2 ev)
{
    if (yee)
        hipExtLaunchKernelGGL((k_maxwell3d_yee<T>), dim3(grid), dim3(kYT), 0, st, ev.start,
                              hi_order ? nullptr : ev.stop, 0, sims, nsims, tile_prefix, total_tiles);
    if (!hi_order) return;
    hipExtLaunchKernelGGL((k_maxwell3d_b<T, 0>), dim3(grid), dim3(kMB), 0, st, yee ? nullptr : ev.start,
                          nullptr, 0, sims, nsims, tile_prefix, total_tiles);
    hipLaunchKernelGGL((k_maxwell3d_e<T>), dim3(grid), dim3(kMB), 0, st, sims, nsims, tile_prefix,
                       total_tiles);
    hipExtLaunchKernelGGL((k_maxwell3d_b<T, 2>), dim3(grid), dim3(kMB), 0, st, nullptr, ev.stop, 0,
                          sims, nsims, tile_prefix, total_tiles);
}

template void launch_maxwell3d<float>(const SimDev<float> *, int, const int *, int, int, bool, bool,
                                      hipStream_t, Ev2);
template void launch_maxwell3d<double>(const SimDev<double> *, int, const int *, int, int, bool, bool,
                                       hipStream_t, Ev2);

}  // namespace pic
