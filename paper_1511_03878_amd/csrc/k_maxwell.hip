// Fused Yee update of the 2-D patch-PIC step.
//
// One workgroup updates a TX x TY tile of nodes with all three sweeps held in
// LDS: B^{n+1/2} = B^n - dt/2 curl E^n, E^{n+1} = E^n + dt (curl B^{n+1/2} -
// J^{n+1/2}), B^{n+1} = B^{n+1/2} - dt/2 curl E^{n+1}.  B updates use forward
// differences of E and E updates backward differences of B, so a one-node
// halo on every side is enough for the three sweeps.  On an open x axis the
// E update at the faces needs By and Bz half a cell outside; they follow from
// the first-order characteristic (Silver-Mueller) condition at the face and
// time n + 1/2 combined with the 1-D Yee update (r = dt/dx, B_1 the first
// inside dual B, E^n the face E):
//   x = 0, incident Ey_i, Ez_i:  Bz = (4 Ey_i - 2 Ey^n - (1 - r) B_1) / (1 + r)
//                                By = (2 Ez^n - (1 - r) B_1 - 4 Ez_i) / (1 + r)
//   x = L, outflow:              Bz = (2 Ey^n - (1 - r) B_1) / (1 + r)
//                                By = (-2 Ez^n - (1 - r) B_1) / (1 + r)
// The kernel reads E^n, B^n from one field buffer and writes E^{n+1},
// B^{n+1} to the other (tiles read halos of their neighbours, which must not
// have been advanced yet).  It also accumulates the field energy of E^n, B^n
// over the tile's own nodes and clears the tile of the J buffer the next step
// deposits into.
#include "kernels.h"

namespace pic {

namespace {

// Field of a 2-D Gaussian beam at the x = 0 face at time t and transverse
// position y.  L = {a0, omega0, w0, tau, t0, x_focus, y_center, phase}.
// Paraxial beam in one transverse dimension: waist w0 at x_focus, Rayleigh
// length z_R = omega0 w0^2 / 2; at the face (distance s = -x_focus from the
// waist) the spot is w0 sqrt(1 + (s / z_R)^2), the wavefront curvature
// s / (s^2 + z_R^2), the Gouy shift atan(s / z_R) / 2, and the amplitude
// a0 omega0 sqrt(w0 / spot).  Envelope exp(-2 ln2 ((t - t0) / tau)^2), tau the
// intensity FWHM; carrier sin(omega0 (t - t0) - omega0 y'^2 curv / 2 +
// Gouy + phase), y' = y - y_center.  Evaluated in FP64.
__device__ double beam_field(const double L[8], double t, double y)
{
    const double om = L[1], w0 = L[2], s = -L[5];
    const double zr = 0.5 * om * w0 * w0;
    const double spot = w0 * sqrt(1.0 + (s / zr) * (s / zr));
    const double curv = s / (s * s + zr * zr);
    const double gouy = 0.5 * atan2(s, zr);
    const double yr = y - L[6], tr = (t - L[4]) / L[3];
    const double env = exp(-2.0 * M_LN2 * tr * tr);
    const double prof = exp(-(yr / spot) * (yr / spot));
    const double ph = om * (t - L[4]) - 0.5 * om * yr * yr * curv + gouy + L[7];
    return L[0] * om * sqrt(w0 / spot) * env * prof * sin(ph);
}

// Workgroups are dispatched to the 8 XCDs in turn (workgroup b to XCD b % 8),
// and each XCD has its own L2.  Renumbering the workgroups XCD-major gives
// every XCD a contiguous band of tiles, so the halo rows and columns a tile
// shares with its neighbours are mostly fetched into the same L2.
__device__ __forceinline__ int xcd_block()
{
    const int g = (int)gridDim.x, b = (int)blockIdx.x;
    return (g & 7) ? b : (b & 7) * (g >> 3) + (b >> 3);
}

template <typename T, int TX, int TY>
__global__ __launch_bounds__(256) void k_maxwell2d(const SimDev<T> *__restrict__ sims, int nsims,
                                                   const int *__restrict__ tile_prefix, int total)
{
    constexpr int W = TX + 3, H = TY + 3, NB = W * H;
    constexpr int NE = (TX + 1) * (TY + 1);  // nodes of sweep 2
    __shared__ T sE[3][NB], sB[3][NB];
    __shared__ double s_red[4];
    const int tid = threadIdx.x;

    for (int tile = xcd_block(); tile < total; tile += gridDim.x) {
        const int s = find_sim(tile_prefix, nsims, tile);
        const SimDev<T> &S = sims[s];
        if (!glb(S.st)->active || S.morder == 6) continue;
        const int lt = tile - tile_prefix[s];
        const int n0 = S.n[0], n1 = S.n[1], fn0 = S.fn[0], fn1 = S.fn[1];
        const int per0 = S.periodic[0], per1 = S.periodic[1];
        const int ntx = (fn0 + TX - 1) / TX;
        const int X0 = (lt % ntx) * TX, Y0 = (lt / ntx) * TY;
        const int64_t stepn = glb(S.st)->step;
        T *const *Jc = S.J[stepn & 1];
        T *const *Jn = S.J[(stepn + 1) & 1];
        T *const *Fc = S.F[stepn & 1];
        T *const *Fn = S.F[(stepn + 1) & 1];

        // ---- load nodes [X0-1, X0+TX+1] x [Y0-1, Y0+TY+1] -------------------
        // All loads of the tile are issued before the first LDS write, from an
        // index that is always in range (a node that does not exist reads node
        // 0 and the value is dropped afterwards), so no load sits behind a
        // branch and each thread keeps all its requests in flight.  J is read
        // straight into the registers of the thread that uses it in sweep 2.
        // staggering: Ex (d,p) Ey (p,d) Ez (p,p) Bx (p,d) By (d,p) Bz (d,d)
        struct Idx {
            int64_t dp, pd, pp, dd;
        };
        auto node_idx = [&](int a, int b) {
            const int gi = X0 - 1 + a, gj = Y0 - 1 + b;
            // nodes more than one past the last stored node feed no update
            // (tiles may be wider than the grid); they stay zero
            const bool need = gi <= fn0 + 1 && gj <= fn1 + 1;
            const int ip = need ? axis_node(gi, n0, per0, 0) : -1;
            const int id = need ? axis_node(gi, n0, per0, 1) : -1;
            const int jp = need ? axis_node(gj, n1, per1, 0) : -1;
            const int jd = need ? axis_node(gj, n1, per1, 1) : -1;
            Idx r;
            r.dp = (id >= 0 && jp >= 0) ? id + (int64_t)fn0 * jp : -1;
            r.pd = (ip >= 0 && jd >= 0) ? ip + (int64_t)fn0 * jd : -1;
            r.pp = (ip >= 0 && jp >= 0) ? ip + (int64_t)fn0 * jp : -1;
            r.dd = (id >= 0 && jd >= 0) ? id + (int64_t)fn0 * jd : -1;
            return r;
        };
        auto ld = [&](T *f, int64_t k) {
            const T x = glb(f)[k >= 0 ? k : 0];
            return k >= 0 ? x : T(0);
        };
        constexpr int NIT = (NB + 255) / 256;
        constexpr int NJT = (NE + 255) / 256;
        T v[NIT][6];
        T jv[NJT][3];
        double esum = 0.0;
#pragma unroll
        for (int r = 0; r < NIT; ++r) {
            const int t = min(tid + 256 * r, NB - 1);
            const Idx q = node_idx(t % W, t / W);
            v[r][0] = ld(Fc[0], q.dp);
            v[r][1] = ld(Fc[1], q.pd);
            v[r][2] = ld(Fc[2], q.pp);
            v[r][3] = ld(Fc[3], q.pd);
            v[r][4] = ld(Fc[4], q.dp);
            v[r][5] = ld(Fc[5], q.dd);
        }
#pragma unroll
        for (int r = 0; r < NJT; ++r) {
            const int t = min(tid + 256 * r, NE - 1);
            const Idx q = node_idx(1 + t % (TX + 1), 1 + t / (TX + 1));
            jv[r][0] = ld(Jc[0], q.dp);
            jv[r][1] = ld(Jc[1], q.pd);
            jv[r][2] = ld(Jc[2], q.pp);
        }
#pragma unroll
        for (int r = 0; r < NIT; ++r) {
            const int t = tid + 256 * r;
            if (t >= NB) break;
            const int a = t % W, b = t / W;
            const int gi = X0 - 1 + a, gj = Y0 - 1 + b;
            const bool own = a >= 1 && a <= TX && b >= 1 && b <= TY && gi < fn0 && gj < fn1;
            sE[0][t] = v[r][0]; sE[1][t] = v[r][1]; sE[2][t] = v[r][2];
            sB[0][t] = v[r][3]; sB[1][t] = v[r][4]; sB[2][t] = v[r][5];
            if (own) {
                // invalid (outside) nodes were loaded as zero, so they add nothing
#pragma unroll
                for (int c = 0; c < 6; ++c) esum += (double)v[r][c] * (double)v[r][c];
            }
        }
        __syncthreads();

        const T dt = S.dt, h = T(0.5) * S.dt;
        const T ix = T(1) / S.d[0], iy = T(1) / S.d[1];

        // ---- sweep 1: B^{n+1/2} on a in [0, TX+1], b in [0, TY+1] -----------
        for (int t = tid; t < (TX + 2) * (TY + 2); t += 256) {
            const int a = t % (TX + 2), b = t / (TX + 2);
            const int c = b * W + a;
            sB[0][c] -= h * (sE[2][c + W] - sE[2][c]) * iy;
            sB[1][c] += h * (sE[2][c + 1] - sE[2][c]) * ix;
            sB[2][c] -= h * ((sE[1][c + 1] - sE[1][c]) * ix - (sE[0][c + W] - sE[0][c]) * iy);
        }
        __syncthreads();

        // ---- Silver-Mueller ghosts on an open x axis -------------------------
        if (!per0) {
            const T r = dt * ix;
            const T ir = T(1) / (T(1) + r);
            if (X0 == 0) {
                const int64_t ls = stepn;
                for (int b = tid; b < H; b += 256) {
                    const int gj = wrap_idx(Y0 - 1 + b, n1);
                    T eyi = T(0), ezi = T(0);
                    if (ls < S.laser_steps) {
                        if (S.laser_ey) eyi = glb(S.laser_ey)[ls * n1 + gj];
                        if (S.laser_ez) ezi = glb(S.laser_ez)[ls * n1 + gj];
                    }
                    if (S.nlaser) {
                        const double t = ((double)ls + 0.5) * S.wdt;
                        double ey = 0.0, ez = 0.0;
                        for (int l = 0; l < S.nlaser; ++l) {
                            if (S.las_pol[l] == 1) ey += beam_field(S.las[l], t, ((double)gj + 0.5) * S.dd[1]);
                            else ez += beam_field(S.las[l], t, (double)gj * S.dd[1]);
                        }
                        eyi += (T)ey;
                        ezi += (T)ez;
                    }
                    const int c = b * W;  // a = 0 is x-node -1 (dual -1/2 for By, Bz)
                    sB[2][c] = (T(4) * eyi - T(2) * sE[1][c + 1] - (T(1) - r) * sB[2][c + 1]) * ir;
                    sB[1][c] = (T(2) * sE[2][c + 1] - (T(1) - r) * sB[1][c + 1] - T(4) * ezi) * ir;
                }
            }
            const int ag = n0 - X0 + 1;  // local column of dual x index n0 (x = L + 1/2)
            if (ag >= 1 && ag <= TX + 1) {
                for (int b = tid; b < H; b += 256) {
                    const int c = b * W + ag;
                    sB[2][c] = (T(2) * sE[1][c] - (T(1) - r) * sB[2][c - 1]) * ir;
                    sB[1][c] = (-T(2) * sE[2][c] - (T(1) - r) * sB[1][c - 1]) * ir;
                }
            }
            __syncthreads();
        }

        // ---- sweep 2: E^{n+1} on a in [1, TX+1], b in [1, TY+1] -------------
#pragma unroll
        for (int r = 0; r < NJT; ++r) {
            const int t = tid + 256 * r;
            if (t >= NE) break;
            const int a = 1 + t % (TX + 1), b = 1 + t / (TX + 1);
            const int c = b * W + a;
            sE[0][c] += dt * ((sB[2][c] - sB[2][c - W]) * iy - jv[r][0]);
            sE[1][c] += dt * (-(sB[2][c] - sB[2][c - 1]) * ix - jv[r][1]);
            sE[2][c] += dt * ((sB[1][c] - sB[1][c - 1]) * ix - (sB[0][c] - sB[0][c - W]) * iy - jv[r][2]);
        }
        __syncthreads();

        // ---- sweep 3: B^{n+1} on the tile's own nodes, then write back -------
        for (int t = tid; t < TX * TY; t += 256) {
            const int a = 1 + t % TX, b = 1 + t / TX;
            const int gi = X0 + a - 1, gj = Y0 + b - 1;
            if (gi >= fn0 || gj >= fn1) continue;
            const int c = b * W + a;
            const T bx = sB[0][c] - h * (sE[2][c + W] - sE[2][c]) * iy;
            const T by = sB[1][c] + h * (sE[2][c + 1] - sE[2][c]) * ix;
            const T bz = sB[2][c] - h * ((sE[1][c + 1] - sE[1][c]) * ix - (sE[0][c + W] - sE[0][c]) * iy);
            // own nodes are inside the periodic range; on an open axis the dual
            // components stop one node short
            const bool dx_ok = per0 || gi <= n0 - 1;
            const int64_t k = gi + (int64_t)fn0 * gj;
            glb(Fn[1])[k] = sE[1][c];
            glb(Fn[2])[k] = sE[2][c];
            glb(Fn[3])[k] = bx;
            glb(Jn[1])[k] = T(0);
            glb(Jn[2])[k] = T(0);
            if (dx_ok) {
                glb(Fn[0])[k] = sE[0][c];
                glb(Fn[4])[k] = by;
                glb(Fn[5])[k] = bz;
                glb(Jn[0])[k] = T(0);
            }
        }

        // ---- field energy of E^n, B^n ----------------------------------------
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) esum += __shfl_xor(esum, o, 64);
        if ((tid & 63) == 0) s_red[tid >> 6] = esum;
        __syncthreads();
        if (tid == 0)
            glb(S.upart)[lt] = 0.5 * S.vcell * (s_red[0] + s_red[1] + s_red[2] + s_red[3]);
        __syncthreads();
    }
}

// Sixth-order staggered field solver (2-D, periodic axes): the same three
// sweeps as three passes over the tiles of the Yee decomposition (so the
// per-tile energy partials line up), one node per thread iteration, the
// neighbours read from global memory (L2 hits).  The derivative at a half
// point comes from the three node pairs around it with the weights that cancel
// the h^2 and h^4 terms of the Taylor series: 75/64, -25/384, 3/640.
// PASS 0: B^{n+1/2} from E^n into the other buffer, energy of E^n, B^n;
// PASS 1: E^{n+1} from B^{n+1/2} and J, clears the other J buffer;
// PASS 2: B^{n+1} from E^{n+1}, in place (it reads E only).
template <typename T, int PASS>
__global__ __launch_bounds__(256) void k_maxwell2d_hi(const SimDev<T> *__restrict__ sims, int nsims,
                                                      const int *__restrict__ tile_prefix, int total,
                                                      int TX, int TY)
{
    __shared__ double s_red[4];
    const int tid = threadIdx.x;
    constexpr T c1 = T(75.0 / 64.0), c2 = T(-25.0 / 384.0), c3 = T(3.0 / 640.0);
    for (int tile = xcd_block(); tile < total; tile += gridDim.x) {
        const int s = find_sim(tile_prefix, nsims, tile);
        const SimDev<T> &S = sims[s];
        if (!glb(S.st)->active || S.morder != 6) continue;
        const int lt = tile - tile_prefix[s];
        const int n0 = S.n[0], n1 = S.n[1];
        const int ntx = (n0 + TX - 1) / TX;
        const int X0 = (lt % ntx) * TX, Y0 = (lt / ntx) * TY;
        const int64_t stepn = glb(S.st)->step;
        T *const *Fc = S.F[stepn & 1];
        T *const *Fn = S.F[(stepn + 1) & 1];
        const T dt = S.dt, h = T(0.5) * S.dt;
        const T ix = T(1) / S.d[0], iy = T(1) / S.d[1];
        double esum = 0.0;
        for (int t = tid; t < TX * TY; t += 256) {
            const int gi = X0 + t % TX, gj = Y0 + t / TX;
            if (gi >= n0 || gj >= n1) continue;
            const int64_t k = gi + (int64_t)n0 * gj;
            // value of array f at node (gi + di, gj + dj), periodic (|d| <= 3 <= n)
            auto node = [&](const T *f, int di, int dj) {
                int a = gi + di, b = gj + dj;
                a += a < 0 ? n0 : 0;
                a -= a >= n0 ? n0 : 0;
                b += b < 0 ? n1 : 0;
                b -= b >= n1 ? n1 : 0;
                return glb(f)[a + (int64_t)n0 * b];
            };
            // forward difference (half point after the node) and backward
            // (half point before it) along x (ax = 0) or y (ax = 1)
            auto dfw = [&](const T *f, int ax) {
                const int u = ax == 0, v = ax == 1;
                return c1 * (node(f, u, v) - node(f, 0, 0)) + c2 * (node(f, 2 * u, 2 * v) - node(f, -u, -v)) +
                       c3 * (node(f, 3 * u, 3 * v) - node(f, -2 * u, -2 * v));
            };
            auto dbw = [&](const T *f, int ax) {
                const int u = ax == 0, v = ax == 1;
                return c1 * (node(f, 0, 0) - node(f, -u, -v)) + c2 * (node(f, u, v) - node(f, -2 * u, -2 * v)) +
                       c3 * (node(f, 2 * u, 2 * v) - node(f, -3 * u, -3 * v));
            };
            if constexpr (PASS == 0 || PASS == 2) {
                T *const *E = PASS == 0 ? Fc : Fn;
                const T bx0 = glb(PASS == 0 ? Fc[3] : Fn[3])[k];
                const T by0 = glb(PASS == 0 ? Fc[4] : Fn[4])[k];
                const T bz0 = glb(PASS == 0 ? Fc[5] : Fn[5])[k];
                const T bx = bx0 - h * dfw(E[2], 1) * iy;
                const T by = by0 + h * dfw(E[2], 0) * ix;
                const T bz = bz0 - h * (dfw(E[1], 0) * ix - dfw(E[0], 1) * iy);
                if constexpr (PASS == 0) {
                    const T ex = glb(Fc[0])[k], ey = glb(Fc[1])[k], ez = glb(Fc[2])[k];
                    esum += (double)ex * ex + (double)ey * ey + (double)ez * ez + (double)bx0 * bx0 +
                            (double)by0 * by0 + (double)bz0 * bz0;
                }
                glb(Fn[3])[k] = bx;
                glb(Fn[4])[k] = by;
                glb(Fn[5])[k] = bz;
            } else {
                T *const *Jc = S.J[stepn & 1];
                T *const *Jn = S.J[(stepn + 1) & 1];
                const T ex = glb(Fc[0])[k] + dt * (dbw(Fn[5], 1) * iy - glb(Jc[0])[k]);
                const T ey = glb(Fc[1])[k] + dt * (-dbw(Fn[5], 0) * ix - glb(Jc[1])[k]);
                const T ez = glb(Fc[2])[k] + dt * (dbw(Fn[4], 0) * ix - dbw(Fn[3], 1) * iy - glb(Jc[2])[k]);
                glb(Fn[0])[k] = ex;
                glb(Fn[1])[k] = ey;
                glb(Fn[2])[k] = ez;
                glb(Jn[0])[k] = T(0);
                glb(Jn[1])[k] = T(0);
                glb(Jn[2])[k] = T(0);
            }
        }
        if constexpr (PASS == 0) {
#pragma unroll
            for (int o = 32; o > 0; o >>= 1) esum += __shfl_xor(esum, o, 64);
            if ((tid & 63) == 0) s_red[tid >> 6] = esum;
            __syncthreads();
            if (tid == 0)
                glb(S.upart)[lt] = 0.5 * S.vcell * (s_red[0] + s_red[1] + s_red[2] + s_red[3]);
            __syncthreads();
        }
    }
}

}  // namespace

// Tile shapes (TX x TY nodes per workgroup) the tuner can choose from.
// FP32 tiles hold 9 x (TX+3)(TY+3) floats of LDS, FP64 tiles doubles.
namespace {
constexpr int kTiles32[6][2] = {{64, 16}, {64, 8}, {128, 8}, {32, 16}, {32, 32}, {128, 4}};
constexpr int kTiles64[6][2] = {{64, 8}, {32, 16}, {32, 8}, {16, 16}, {64, 4}, {128, 4}};
}  // namespace

template <typename T>
void maxwell_tile(int preset, int &tx, int &ty)
{
    const int p = (preset >= 0 && preset < 6) ? preset : 0;
    tx = sizeof(T) == 4 ? kTiles32[p][0] : kTiles64[p][0];
    ty = sizeof(T) == 4 ? kTiles32[p][1] : kTiles64[p][1];
}

template <typename T>
void launch_maxwell(const SimDev<T> *sims, int nsims, const int *tile_prefix, int total_tiles,
                    int grid, int preset, bool yee, bool hi_order, hipStream_t st, Ev2 ev)
{
    hipEvent_t stop1 = hi_order ? nullptr : ev.stop;
#define PIC_MW(TX, TY)                                                                          \
    hipExtLaunchKernelGGL((k_maxwell2d<T, TX, TY>), dim3(grid), dim3(256), 0, st, ev.start,    \
                          stop1, 0, sims, nsims, tile_prefix, total_tiles)
    const int p = (preset >= 0 && preset < 6) ? preset : 0;
    if (!yee) {
        // every simulation of the batch uses the sixth-order solver
    } else if constexpr (sizeof(T) == 4) {
        switch (p) {
        case 1: PIC_MW(64, 8); break;
        case 2: PIC_MW(128, 8); break;
        case 3: PIC_MW(32, 16); break;
        case 4: PIC_MW(32, 32); break;
        case 5: PIC_MW(128, 4); break;
        default: PIC_MW(64, 16); break;
        }
    } else {
        switch (p) {
        case 1: PIC_MW(32, 16); break;
        case 2: PIC_MW(32, 8); break;
        case 3: PIC_MW(16, 16); break;
        case 4: PIC_MW(64, 4); break;
        case 5: PIC_MW(128, 4); break;
        default: PIC_MW(64, 8); break;
        }
    }
#undef PIC_MW
    if (hi_order) {
        // the sixth-order simulations of the batch (the Yee kernel skipped their tiles)
        int tx, ty;
        maxwell_tile<T>(preset, tx, ty);
        hipExtLaunchKernelGGL((k_maxwell2d_hi<T, 0>), dim3(grid), dim3(256), 0, st, yee ? nullptr : ev.start,
                              nullptr, 0, sims, nsims, tile_prefix, total_tiles, tx, ty);
        hipLaunchKernelGGL((k_maxwell2d_hi<T, 1>), dim3(grid), dim3(256), 0, st, sims, nsims, tile_prefix,
                           total_tiles, tx, ty);
        hipExtLaunchKernelGGL((k_maxwell2d_hi<T, 2>), dim3(grid), dim3(256), 0, st, nullptr, ev.stop, 0,
                              sims, nsims, tile_prefix, total_tiles, tx, ty);
    }
}

template void maxwell_tile<float>(int, int &, int &);
template void maxwell_tile<double>(int, int &, int &);
template void launch_maxwell<float>(const SimDev<float> *, int, const int *, int, int, int, bool, bool,
                                    hipStream_t, Ev2);
template void launch_maxwell<double>(const SimDev<double> *, int, const int *, int, int, int, bool, bool,
                                     hipStream_t, Ev2);

}  // namespace pic
