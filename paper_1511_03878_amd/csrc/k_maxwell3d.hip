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

// ---- fused Yee update of a column of node planes ------------------------------
//
// Block [X, X + BX) x [Y, Y + BY) x [Z, Z + BZ) of the nodes, taken plane by
// plane along z.  Per plane, E is staged on [X - 1, X + BX + 2) x [Y - 1,
// Y + BY + 2) and B on [X - 1, X + BX + 1) x [Y - 1, Y + BY + 1) (periodic,
// so a block at the grid's end reads its halo from the start); three E
// planes (z, z + 1, z + 2) and two B planes (z, z + 1) rotate in LDS.  For
// output plane z:
//   B' = B - dt/2 curl E        on plane z + 1 (in place; needs E of z + 1, z + 2),
//   E' = E + dt (curl B' - J)   on plane z + 1 over [X, X + BX + 1) x [Y, Y + BY + 1)
//                                (in place; needs B' of z, z + 1; J loaded per node),
//   B'' = B' - dt/2 curl E'     on plane z over the block (needs E' of z, z + 1),
// and E', B'' of plane z are written to the other field buffer and its nodes
// of the other J buffer cleared: the three passes' arithmetic in the same
// order, reading E, B and J once per node plus an x-y halo (z needs none
// beyond the two planes before the first).  Both plane tiles start at X - 1,
// Y - 1, so a node has the same local coordinates in each.  Nodes past the
// grid's end (n not a multiple of the block) are computed from wrapped data
// and not written.
constexpr int kYT = 256;                              // threads
constexpr int kEX = kYee3X + 3, kEY = kYee3Y + 3;     // E plane tile
constexpr int kBX = kYee3X + 2, kBY = kYee3Y + 2;     // B plane tile
constexpr int kE2X = kYee3X + 1, kE2Y = kYee3Y + 1;   // E' nodes of a plane
constexpr int kEP = kEX * kEY, kBP = kBX * kBY, kE2P = kE2X * kE2Y, kOP = kYee3X * kYee3Y;
constexpr int kRE = (kEP + kYT - 1) / kYT, kRB = (kBP + kYT - 1) / kYT, kRJ = (kE2P + kYT - 1) / kYT;
static_assert(kOP % kYT == 0, "own nodes of a plane per thread");

template <typename T>
__global__ __launch_bounds__(kYT) void k_maxwell3d_yee(const SimDev<T> *__restrict__ sims, int nsims,
                                                       const int *__restrict__ tile_prefix, int total)
{
    __shared__ T sE[3][3][kEP];  // [plane slot][component][node]
    __shared__ T sB[2][3][kBP];
    __shared__ int s_wrap[kEX + kEY];  // wrapped node index of each local index, x then y
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
        // global index of local index 0 along x and y; the block's planes
        const int x0 = (lt % nbx) * kYee3X - 1, y0 = ((lt / nbx) % nby) * kYee3Y - 1;
        const int zs = (lt / (nbx * nby)) * kYee3Z, ze = min(zs + kYee3Z, fn2);
        const int64_t stepn = glb(S.st)->step;
        T *const *Fc = S.F[stepn & 1];
        T *const *Fn = S.F[(stepn + 1) & 1];
        T *const *Jc = S.J[stepn & 1];
        T *const *Jn = S.J[(stepn + 1) & 1];
        const T dt = S.dt, h = T(0.5) * S.dt;
        const T ix = T(1) / S.d[0], iy = T(1) / S.d[1], iz = T(1) / S.d[2];
        for (int i = tid; i < kEX + kEY; i += kYT) {
            const int n = i < kEX ? fn0 : fn1;
            int g = (i < kEX ? x0 + i : y0 + i - kEX) % n;
            s_wrap[i] = g < 0 ? g + n : g;
        }
        __syncthreads();
        const int *wx = s_wrap, *wy = s_wrap + kEX;
        auto zrow = [&](int z) {  // first node of wrapped plane z, in rows of fn0
            z %= fn2;
            return (int64_t)(z < 0 ? z + fn2 : z) * fn1;
        };
        // stage plane z of E (or B) into slot sl (every load from an in-range
        // index; duplicates write the same value)
        auto load_e = [&](int sl, int z) {
            const int64_t zr = zrow(z);
#pragma unroll
            for (int r = 0; r < kRE; ++r) {
                const int i = min(tid + r * kYT, kEP - 1);
                const int64_t g = (zr + wy[i / kEX]) * fn0 + wx[i % kEX];
#pragma unroll
                for (int c = 0; c < 3; ++c) sE[sl][c][i] = glb((const T *)Fc[c])[g];
            }
        };
        auto load_b = [&](int sl, int z) {
            const int64_t zr = zrow(z);
#pragma unroll
            for (int r = 0; r < kRB; ++r) {
                const int i = min(tid + r * kYT, kBP - 1);
                const int64_t g = (zr + wy[i / kBX]) * fn0 + wx[i % kBX];
#pragma unroll
                for (int c = 0; c < 3; ++c) sB[sl][c][i] = glb((const T *)Fc[3 + c])[g];
            }
        };
        // J of plane z at the E' nodes, into registers
        T jr[3][kRJ];
        auto load_j = [&](int z) {
            const int64_t zr = zrow(z);
#pragma unroll
            for (int r = 0; r < kRJ; ++r) {
                const int j = min(tid + r * kYT, kE2P - 1);
                const int64_t g = (zr + wy[j / kE2X + 1]) * fn0 + wx[j % kE2X + 1];
#pragma unroll
                for (int c = 0; c < 3; ++c) jr[c][r] = glb((const T *)Jc[c])[g];
            }
        };
        // B' of the plane in B slot bs from E slots ec (same plane) and en (the
        // next); with `own`, the energy of the plane's incoming E, B over the block
        double esum = 0.0;
        auto bprime = [&](int bs, int ec, int en, bool own_plane) {
#pragma unroll
            for (int r = 0; r < kRB; ++r) {
                const int i = tid + r * kYT;
                if (i < kBP) {
                    const int lx = i % kBX, ly = i / kBX;
                    const int e = ly * kEX + lx;
                    const T ex = sE[ec][0][e], ey = sE[ec][1][e], ez = sE[ec][2][e];
                    const T bx = sB[bs][0][i], by = sB[bs][1][i], bz = sB[bs][2][i];
                    if (own_plane && lx >= 1 && lx <= kYee3X && ly >= 1 && ly <= kYee3Y && x0 + lx < fn0 &&
                        y0 + ly < fn1)
                        esum += (double)ex * ex + (double)ey * ey + (double)ez * ez + (double)bx * bx +
                                (double)by * by + (double)bz * bz;
                    sB[bs][0][i] = bx - h * ((sE[ec][2][e + kEX] - ez) * iy - (sE[en][1][e] - ey) * iz);
                    sB[bs][1][i] = by - h * ((sE[en][0][e] - ex) * iz - (sE[ec][2][e + 1] - ez) * ix);
                    sB[bs][2][i] = bz - h * ((sE[ec][1][e + 1] - ey) * ix - (sE[ec][0][e + kEX] - ex) * iy);
                }
            }
        };
        // E' of the plane in E slot es from B' slots bc (same plane) and bp (the previous)
        auto eprime = [&](int es, int bc, int bp) {
#pragma unroll
            for (int r = 0; r < kRJ; ++r) {
                const int j = tid + r * kYT;
                if (j < kE2P) {
                    const int lx = j % kE2X + 1, ly = j / kE2X + 1;
                    const int e = ly * kEX + lx, b = ly * kBX + lx;
                    const T bx = sB[bc][0][b], by = sB[bc][1][b], bz = sB[bc][2][b];
                    sE[es][0][e] = sE[es][0][e] + dt * ((bz - sB[bc][2][b - kBX]) * iy - (by - sB[bp][1][b]) * iz - jr[0][r]);
                    sE[es][1][e] = sE[es][1][e] + dt * ((bx - sB[bp][0][b]) * iz - (bz - sB[bc][2][b - 1]) * ix - jr[1][r]);
                    sE[es][2][e] = sE[es][2][e] + dt * ((by - sB[bc][1][b - 1]) * ix - (bx - sB[bc][0][b - kBX]) * iy - jr[2][r]);
                }
            }
        };
        // B'' of plane z from B' (slot bc) and E' of planes z (ec), z + 1 (en);
        // write E', B'' and clear the other J
        auto write_plane = [&](int z, int ec, int en, int bc) {
            const gptr_t<T> E0 = glb(Fn[0]), E1 = glb(Fn[1]), E2 = glb(Fn[2]);
            const gptr_t<T> B0 = glb(Fn[3]), B1 = glb(Fn[4]), B2 = glb(Fn[5]);
            const gptr_t<T> J0 = glb(Jn[0]), J1 = glb(Jn[1]), J2 = glb(Jn[2]);
#pragma unroll
            for (int r = 0; r < kOP / kYT; ++r) {
                const int o = tid + r * kYT;
                const int lx = o % kYee3X + 1, ly = o / kYee3X + 1;
                if (x0 + lx >= fn0 || y0 + ly >= fn1) continue;
                const int e = ly * kEX + lx, b = ly * kBX + lx;
                const T ex = sE[ec][0][e], ey = sE[ec][1][e], ez = sE[ec][2][e];
                const int64_t g = ((int64_t)z * fn1 + (y0 + ly)) * fn0 + (x0 + lx);
                B0[g] = sB[bc][0][b] - h * ((sE[ec][2][e + kEX] - ez) * iy - (sE[en][1][e] - ey) * iz);
                B1[g] = sB[bc][1][b] - h * ((sE[en][0][e] - ex) * iz - (sE[ec][2][e + 1] - ez) * ix);
                B2[g] = sB[bc][2][b] - h * ((sE[ec][1][e + 1] - ey) * ix - (sE[ec][0][e + kEX] - ex) * iy);
                E0[g] = ex;
                E1[g] = ey;
                E2[g] = ez;
                J0[g] = T(0);
                J1[g] = T(0);
                J2[g] = T(0);
            }
        };

        // ---- first plane: E of zs - 1 .. zs + 1, B of zs - 1, zs, J of zs ---------
        load_e(0, zs - 1);
        load_e(1, zs);
        load_e(2, zs + 1);
        load_b(0, zs - 1);
        load_b(1, zs);
        load_j(zs);
        __syncthreads();
        bprime(0, 0, 1, false);  // B'(zs - 1)
        bprime(1, 1, 2, true);   // B'(zs), energy of plane zs
        __syncthreads();
        eprime(1, 1, 0);  // E'(zs)
        __syncthreads();
        // E slots: ec = E'(z), en = E(z + 1) raw, ef free; B slots: bc = B'(z), bf free
        int ec = 1, en = 2, ef = 0, bc = 1, bf = 0;
        for (int z = zs; z < ze; ++z) {
            load_e(ef, z + 2);
            load_b(bf, z + 1);
            load_j(z + 1);
            __syncthreads();
            bprime(bf, en, ef, z + 1 < ze);  // B'(z + 1)
            __syncthreads();
            eprime(en, bf, bc);  // E'(z + 1)
            __syncthreads();
            write_plane(z, ec, en, bc);
            __syncthreads();  // before the next planes are loaded into the freed slots
            const int t = ec;
            ec = en;
            en = ef;
            ef = t;
            const int u = bc;
            bc = bf;
            bf = u;
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
        // (the next block's wrap table and planes are written after the
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
