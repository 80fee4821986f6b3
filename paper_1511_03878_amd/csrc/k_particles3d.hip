// Fused particle kernel of the 3-D patch-PIC step (periodic boxes): per work
// item (a chunk of one patch) stage the patch's E and B into LDS, then per
// particle gather with quadratic shapes on 27 nodes, relativistic Boris push,
// move, classify the destination among the 26 neighbours, and deposit the
// charge-conserving (Esirkepov) current on a 4 x 4 x 4 node window into an
// FP64 LDS tile that is flushed to the global current once per item.
//
// Staggering (half a cell up): Ex, Ey, Ez along their own axis; Bx, By, Bz
// along the two other axes.  The LDS holds the field tile of (P+3)^3 nodes
// and the current tile of (P+5)^3 nodes, so the patch edge is limited (8
// cells per axis fits twice over in one CU's LDS for FP32).
#include <type_traits>

#include "kernels.h"
#include "particle_common.h"

namespace pic {

namespace {

// 27-node gather from an LDS tile: the window starts at tile entry (i0, j0,
// k0), which holds patch-local node (i0 - 1, j0 - 1, k0 - 1).
template <typename T>
__device__ __forceinline__ T gather27(const T *tile, int fw, int fwh, int i0, int j0, int k0,
                                      const T wx[3], const T wy[3], const T wz[3])
{
    const T *r = tile + k0 * fwh + j0 * fw + i0;
    T acc = T(0);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        T plane = T(0);
#pragma unroll
        for (int b = 0; b < 3; ++b) {
            const T *q = r + c * fwh + b * fw;
            plane += (q[0] * wx[0] + q[1] * wx[1] + q[2] * wx[2]) * wy[b];
        }
        acc += plane * wz[c];
    }
    return acc;
}

template <typename T, int BLOCK>
__global__ __launch_bounds__(BLOCK) void k_particles3d(const SimDev<T> *__restrict__ sims,
                                                       const Item *__restrict__ items,
                                                       const int *__restrict__ nitems,
                                                       int *__restrict__ head)
{
    using W = typename std::conditional<sizeof(T) == 4, float, double>::type;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    __shared__ int s_item[2];

    const int tid = threadIdx.x, ln = tid % kWave;
    const int total = *glb(nitems);
    // items claimed one ahead, kinetic energy kept per wave (as in 2-D)
    if (tid == 0) s_item[0] = atomicAdd(head, 1);
    __syncthreads();
    int idx = __builtin_amdgcn_readfirstlane(s_item[0]);
    int slot = 1;
    double kin = 0.0;
    int kin_sim = -1, kin_p = 0;
    auto flush_kin = [&]() {
        const double t = wave_sum(kin);
        if (kin_sim >= 0 && ln == 0) gadd(glb(sims[kin_sim].kpart) + kin_p, t * sims[kin_sim].vcell);
        kin = 0.0;
    };
    while (idx < total) {
        int next = 0;
        if (tid == 0) next = atomicAdd(head, 1);
        const Item it = items[idx];
        const int si = __builtin_amdgcn_readfirstlane(it.x & kItemSimMask);
        const int par = __builtin_amdgcn_readfirstlane(it.x >> 30);
        const SimDev<T> &S = sims[si];
        const int p = __builtin_amdgcn_readfirstlane(it.y);
        const int64_t base = __builtin_amdgcn_readfirstlane(it.z);
        const int cnt = __builtin_amdgcn_readfirstlane(it.w);
        const int P0 = S.P[0], P1 = S.P[1], P2 = S.P[2];
        const int pxi = p % S.np[0], pyi = (p / S.np[0]) % S.np[1], pzi = p / (S.np[0] * S.np[1]);
        const int ox = pxi * P0, oy = pyi * P1, oz = pzi * P2;
        const int fw = P0 + 3, fh = P1 + 3, fd = P2 + 3, fwh = fw * fh;
        const int jw = P0 + 5, jh = P1 + 5, jd = P2 + 5, jwh = jw * jh;
        const int fstride = fwh * fd, jstride = jwh * jd;
        double *Jt = reinterpret_cast<double *>(smem_raw);
        T *Ft = reinterpret_cast<T *>(Jt + 3 * jstride);
        const int n0 = S.n[0], n1 = S.n[1], n2 = S.n[2];
        const int fn0 = S.fn[0], fn1 = S.fn[1];
        if (si != kin_sim) {
            flush_kin();
            kin_sim = si;
        }
        kin_p = p;

        const gptr_t<T> X0 = glb(S.x[0]) + base, X1 = glb(S.x[1]) + base, X2 = glb(S.x[2]) + base;
        const gptr_t<T> U0 = glb(S.u[0]) + base, U1 = glb(S.u[1]) + base, U2 = glb(S.u[2]) + base;
        const gptr_t<const T> Wt = glb((const T *)S.w) + base;
        const gptr_t<uint8_t> Cd = glb(S.code) + base;

        // lane mapping, remainder units and prefetch as in 2-D: no lane
        // branches around a memory access, lanes past the end repeat the
        // item's last particle with zero weight
        constexpr int NW = BLOCK / kWave;
        const int S_ = S.lane_stride;
        const int wv = __builtin_amdgcn_readfirstlane(tid / kWave);
        const int npass = cnt / (kWave * S_), ufull = npass * S_;
        const int uend = ufull + (cnt - npass * kWave * S_ + kWave - 1) / kWave;
        auto unit_particle = [&](int u) {
            return u < ufull ? kWave * S_ * (u / S_) + ln * S_ + (u % S_)
                             : kWave * S_ * npass + kWave * (u - ufull) + ln;
        };
        T nx_, ny_, nz_, nux, nuy, nuz, nw_;
        auto load_unit = [&](int u) {
            const int kn = min(unit_particle(u), cnt - 1);
            nx_ = X0[kn]; ny_ = X1[kn]; nz_ = X2[kn];
            nux = U0[kn]; nuy = U1[kn]; nuz = U2[kn]; nw_ = Wt[kn];
        };
        load_unit(wv);

        // ---- stage E, B of nodes [o-1, o+P+1] on every axis (periodic) -----
        // (unconditional loads from an in-range node; only tile nodes are stored)
        T *const *Fc = S.F[par];
        for (int t0 = 0; t0 < fstride; t0 += 4 * BLOCK) {
            T v[4][6];
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int t = t0 + r * BLOCK + tid;
                const int tt = t < fstride ? t : 0;
                const int a = tt % fw, b = (tt / fw) % fh, c = tt / fwh;
                const int gi = axis_node(ox - 1 + a, n0, 1, 0);
                const int gj = axis_node(oy - 1 + b, n1, 1, 0);
                const int gk = axis_node(oz - 1 + c, n2, 1, 0);
                const int64_t k = gi + (int64_t)fn0 * (gj + (int64_t)fn1 * gk);
#pragma unroll
                for (int cc = 0; cc < 6; ++cc) v[r][cc] = glb(Fc[cc])[k];
            }
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int t = t0 + r * BLOCK + tid;
                if (t < fstride)
#pragma unroll
                    for (int cc = 0; cc < 6; ++cc) Ft[cc * fstride + t] = v[r][cc];
            }
        }
        for (int t = tid; t < 3 * jstride; t += BLOCK) Jt[t] = 0.0;
        __syncthreads();
        if (tid == 0) s_item[slot] = next;  // read after the item's last barrier

        const T dt = S.dt, q = S.q, m = S.m;
        const T eps = q * dt / (T(2) * m);
        const T rdx = dt / S.d[0], rdy = dt / S.d[1], rdz = dt / S.d[2];
        const double cx_ = -(double)q * (double)S.d[0] / (double)dt;
        const double cy_ = -(double)q * (double)S.d[1] / (double)dt;
        const double cz_ = -(double)q * (double)S.d[2] / (double)dt;
        const T Pmax0 = below((T)P0), Pmax1 = below((T)P1), Pmax2 = below((T)P2);
        uint32_t err = 0;
        bool left = false;

        for (int u = wv; u < uend; u += NW) {
            const int kr = unit_particle(u), k = min(kr, cnt - 1);
            const T xl = nx_, yl = ny_, zl = nz_;
            T ux = nux, uy = nuy, uz = nuz;
            const T wgt = kr < cnt ? nw_ : T(0);
            load_unit(u + NW);

            // ---- gather -------------------------------------------------
            int ip[3], id[3];
            T wp[3][3], wd[3][3];
            const T xs[3] = {xl, yl, zl};
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                ip[a] = (int)floor(xs[a] + T(0.5));
                id[a] = (int)floor(xs[a]);
                qweights(xs[a] - (T)ip[a], wp[a][0], wp[a][1], wp[a][2]);
                qweights(xs[a] - (T)id[a] - T(0.5), wd[a][0], wd[a][1], wd[a][2]);
            }
            const T Ex = gather27(Ft + 0 * fstride, fw, fwh, id[0], ip[1], ip[2], wd[0], wp[1], wp[2]);
            const T Ey = gather27(Ft + 1 * fstride, fw, fwh, ip[0], id[1], ip[2], wp[0], wd[1], wp[2]);
            const T Ez = gather27(Ft + 2 * fstride, fw, fwh, ip[0], ip[1], id[2], wp[0], wp[1], wd[2]);
            const T Bx = gather27(Ft + 3 * fstride, fw, fwh, ip[0], id[1], id[2], wp[0], wd[1], wd[2]);
            const T By = gather27(Ft + 4 * fstride, fw, fwh, id[0], ip[1], id[2], wd[0], wp[1], wd[2]);
            const T Bz = gather27(Ft + 5 * fstride, fw, fwh, id[0], id[1], ip[2], wd[0], wd[1], wp[2]);

            // ---- Boris --------------------------------------------------------
            const T usq0 = ux * ux + uy * uy + uz * uz;
            T umx = ux + eps * Ex, umy = uy + eps * Ey, umz = uz + eps * Ez;
            const T igm = rsq_(T(1) + umx * umx + umy * umy + umz * umz);
            const T tx = eps * igm * Bx, ty = eps * igm * By, tz = eps * igm * Bz;
            const T t2 = tx * tx + ty * ty + tz * tz;
            const T s2 = T(2) * rcp_(T(1) + t2);
            const T sx = s2 * tx, sy = s2 * ty, sz = s2 * tz;
            const T upx = umx + (umy * tz - umz * ty);
            const T upy = umy + (umz * tx - umx * tz);
            const T upz = umz + (umx * ty - umy * tx);
            umx += upy * sz - upz * sy;
            umy += upz * sx - upx * sz;
            umz += upx * sy - upy * sx;
            ux = umx + eps * Ex;
            uy = umy + eps * Ey;
            uz = umz + eps * Ez;
            const T usq1 = ux * ux + uy * uy + uz * uz;
            const T ig1 = rsq_(T(1) + usq1);
            if constexpr (sizeof(T) == 4) {
                const float a0 = 1.0f + usq0;
                const float g0p = a0 * rsq_(a0) + 1.0f, g1p = (1.0f + usq1) * ig1 + 1.0f;
                kin += (double)(wgt * m * 0.5f * (usq0 * rcp_(g0p) + usq1 * rcp_(g1p)));
            } else {
                const double g0p = sqrt(1.0 + (double)usq0) + 1.0;
                const double g1p = (double)(T(1) + usq1) * (double)ig1 + 1.0;
                kin += (double)wgt * (double)m * 0.5 *
                       ((double)usq0 * g1p + (double)usq1 * g0p) / (g0p * g1p);
            }

            // ---- move and classify --------------------------------------------
            const T dxl = rdx * ux * ig1, dyl = rdy * uy * ig1, dzl = rdz * uz * ig1;
            uint8_t code;
            T x1 = xl + dxl, y1 = yl + dyl, z1 = zl + dzl;
            if (!(fabs(dxl) < T(1) && fabs(dyl) < T(1) && fabs(dzl) < T(1))) {
                err |= (isfinite(ux) && isfinite(uy) && isfinite(uz)) ? kFlagCFL : kFlagNaN;
                code = kRemoved;
                x1 = xl;
                y1 = yl;
                z1 = zl;
            } else {
                if (dxl != T(0) || dyl != T(0) || dzl != T(0)) {
                    // ---- Esirkepov deposit on a 4x4x4 node window -------------
                    // W_a = DS_a (S0_b S0_c + DS_b S0_c / 2 + S0_b DS_c / 2 +
                    // DS_b DS_c / 3) = DS_a (A_b S0_c + B_b DS_c) with
                    // A = S0 + DS / 2, B = S0 / 2 + DS / 3; J_a is the running
                    // sum of -q w (d_a / dt) W_a along a.  Window slot 3 of an
                    // axis carries weight only when its nearest node changed;
                    // its (exactly zero) entries skip their atomics.
                    int mx, my, mz;
                    // weights and products in W (FP32 for FP32 storage: fewer live
                    // registers, so more waves fit); sums in the FP64 tile
                    W S0x[4], DSx[4], S0y[4], DSy[4], S0z[4], DSz[4];
                    const bool cx = window4(xl, (double)dxl, mx, S0x, DSx);
                    const bool cy = window4(yl, (double)dyl, my, S0y, DSy);
                    const bool cz = window4(zl, (double)dzl, mz, S0z, DSz);
                    const W qw = (W)wgt;
                    W Ax[4], Bx_[4], Ay[4], By_[4];
#pragma unroll
                    for (int k2 = 0; k2 < 4; ++k2) {
                        Ax[k2] = S0x[k2] + W(0.5) * DSx[k2];
                        Bx_[k2] = W(0.5) * S0x[k2] + DSx[k2] * W(1.0 / 3.0);
                        Ay[k2] = S0y[k2] + W(0.5) * DSy[k2];
                        By_[k2] = W(0.5) * S0y[k2] + DSy[k2] * W(1.0 / 3.0);
                    }
                    const W cq = (W)cx_ * qw, dq = (W)cy_ * qw, eq = (W)cz_ * qw;
                    W px[3], py[3], pz[3];
                    px[0] = cq * DSx[0];
                    py[0] = dq * DSy[0];
                    pz[0] = eq * DSz[0];
#pragma unroll
                    for (int k2 = 1; k2 < 3; ++k2) {
                        px[k2] = px[k2 - 1] + cq * DSx[k2];
                        py[k2] = py[k2 - 1] + dq * DSy[k2];
                        pz[k2] = pz[k2 - 1] + eq * DSz[k2];
                    }
                    double *Jxt = Jt, *Jyt = Jt + jstride, *Jzt = Jt + 2 * jstride;
                    const int r0 = (mz + 2) * jwh + (my + 2) * jw + (mx + 2);
                    const int ni = cx ? 3 : 2, nj = cy ? 3 : 2, nk = cz ? 3 : 2;
                    const int mi = cx ? 4 : 3, mj = cy ? 4 : 3, mk = cz ? 4 : 3;
                    // Jx: dual x (prefix index i), transverse (j, k)
#pragma unroll
                    for (int kk = 0; kk < 4; ++kk) {
                        if (kk >= mk) break;
#pragma unroll
                        for (int j = 0; j < 4; ++j) {
                            if (j >= mj) break;
                            const W tr = Ay[j] * S0z[kk] + By_[j] * DSz[kk];
#pragma unroll
                            for (int i = 0; i < 3; ++i) {
                                if (i >= ni) break;
                                atomicAdd(&Jxt[r0 + kk * jwh + j * jw + i], (double)(px[i] * tr));
                            }
                        }
                    }
                    // Jy: dual y (prefix index j), transverse (i, k)
#pragma unroll
                    for (int kk = 0; kk < 4; ++kk) {
                        if (kk >= mk) break;
#pragma unroll
                        for (int i = 0; i < 4; ++i) {
                            if (i >= mi) break;
                            const W tr = Ax[i] * S0z[kk] + Bx_[i] * DSz[kk];
#pragma unroll
                            for (int j = 0; j < 3; ++j) {
                                if (j >= nj) break;
                                atomicAdd(&Jyt[r0 + kk * jwh + j * jw + i], (double)(py[j] * tr));
                            }
                        }
                    }
                    // Jz: dual z (prefix index k), transverse (i, j)
#pragma unroll
                    for (int j = 0; j < 4; ++j) {
                        if (j >= mj) break;
#pragma unroll
                        for (int i = 0; i < 4; ++i) {
                            if (i >= mi) break;
                            const W tr = Ax[i] * S0y[j] + Bx_[i] * DSy[j];
#pragma unroll
                            for (int kk = 0; kk < 3; ++kk) {
                                if (kk >= nk) break;
                                atomicAdd(&Jzt[r0 + kk * jwh + j * jw + i], (double)(pz[kk] * tr));
                            }
                        }
                    }
                }
                const int sx_ = x1 < T(0) ? -1 : (x1 >= (T)P0 ? 1 : 0);
                const int sy_ = y1 < T(0) ? -1 : (y1 >= (T)P1 ? 1 : 0);
                const int sz_ = z1 < T(0) ? -1 : (z1 >= (T)P2 ? 1 : 0);
                x1 -= (T)(sx_ * P0);
                y1 -= (T)(sy_ * P1);
                z1 -= (T)(sz_ * P2);
                if (x1 > Pmax0) x1 = Pmax0;
                if (y1 > Pmax1) y1 = Pmax1;
                if (z1 > Pmax2) z1 = Pmax2;
                code = (uint8_t)((sx_ + 1) + 3 * (sy_ + 1) + 9 * (sz_ + 1));
            }
            X0[k] = x1;
            X1[k] = y1;
            X2[k] = z1;
            U0[k] = ux;
            U1[k] = uy;
            U2[k] = uz;
            Cd[k] = code;
            left |= code != kStay3;
        }
        if (__ballot(left) && ln == 0) *glb(S.moved + p) = 1;
        if (err)
            __hip_atomic_fetch_or(&glb(S.st)->flags, err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __syncthreads();

        // ---- flush the current tile (nodes [o-2, o+P+2] on every axis) ------
        {
            const gptr_t<T> Jgx = glb(S.J[par][0]), Jgy = glb(S.J[par][1]), Jgz = glb(S.J[par][2]);
            for (int t = tid; t < jstride; t += BLOCK) {
                const int a = t % jw, b = (t / jw) % jh, c = t / jwh;
                const int gi = axis_node(ox - 2 + a, n0, 1, 0);
                const int gj = axis_node(oy - 2 + b, n1, 1, 0);
                const int gk = axis_node(oz - 2 + c, n2, 1, 0);
                const int64_t k = gi + (int64_t)fn0 * (gj + (int64_t)fn1 * gk);
                const T vx = (T)Jt[t], vy = (T)Jt[jstride + t], vz = (T)Jt[2 * jstride + t];
                if (vx != T(0)) gadd(Jgx + k, vx);
                if (vy != T(0)) gadd(Jgy + k, vy);
                if (vz != T(0)) gadd(Jgz + k, vz);
            }
        }
        __syncthreads();
        idx = __builtin_amdgcn_readfirstlane(s_item[slot]);
        slot ^= 1;
    }
    flush_kin();
}

}  // namespace

size_t particles3d_lds_bytes(int precision, int P0, int P1, int P2)
{
    const size_t fs = (size_t)(P0 + 3) * (P1 + 3) * (P2 + 3);
    const size_t js = (size_t)(P0 + 5) * (P1 + 5) * (P2 + 5);
    return sizeof(double) * 3 * js + (size_t)(precision / 8) * 6 * fs;
}

template <typename T>
void launch_particles3d(const SimDev<T> *sims, const Item *items, const int *nitems, int *head,
                        int grid, int block, int maxP0, int maxP1, int maxP2, hipStream_t st,
                        Ev2 ev)
{
    const size_t lds = particles3d_lds_bytes(sizeof(T) * 8, maxP0, maxP1, maxP2);
    if (block == 1024)
        hipExtLaunchKernelGGL((k_particles3d<T, 1024>), dim3(grid), dim3(1024), lds, st, ev.start,
                              ev.stop, 0, sims, items, nitems, head);
    else if (block == 256)
        hipExtLaunchKernelGGL((k_particles3d<T, 256>), dim3(grid), dim3(256), lds, st, ev.start,
                              ev.stop, 0, sims, items, nitems, head);
    else
        hipExtLaunchKernelGGL((k_particles3d<T, 512>), dim3(grid), dim3(512), lds, st, ev.start,
                              ev.stop, 0, sims, items, nitems, head);
}

template <typename T>
int particles3d_occupancy(int block, int maxP0, int maxP1, int maxP2)
{
    const size_t lds = particles3d_lds_bytes(sizeof(T) * 8, maxP0, maxP1, maxP2);
    int nb = 0;
    hipError_t e;
    if (block == 1024)
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_particles3d<T, 1024>, 1024, lds);
    else if (block == 256)
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_particles3d<T, 256>, 256, lds);
    else
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_particles3d<T, 512>, 512, lds);
    return e == hipSuccess ? nb : 0;
}

template void launch_particles3d<float>(const SimDev<float> *, const Item *, const int *, int *, int,
                                        int, int, int, int, hipStream_t, Ev2);
template void launch_particles3d<double>(const SimDev<double> *, const Item *, const int *, int *,
                                         int, int, int, int, int, hipStream_t, Ev2);
template int particles3d_occupancy<float>(int, int, int, int);
template int particles3d_occupancy<double>(int, int, int, int);

}  // namespace pic
