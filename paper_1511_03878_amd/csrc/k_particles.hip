// Fused particle kernel of the 2-D patch-PIC step (one work item = a chunk of
// one patch): stage the patch's E and B into LDS, then per particle gather
// with quadratic shapes, relativistic Boris push, move, classify the
// destination patch, and deposit the charge-conserving (Esirkepov) current
// into a 64-bit fixed-point LDS tile (exact integer sums, independent of the
// order of the atomics) that is flushed to the global current once per item.
//
// The paper's patches (section 3.1) are small independent structures of
// fields and particles; here one workgroup owns one patch chunk at a time,
// and workgroups pull items from a queue ordered by particle count (the
// single-GPU form of exchanging patches to even out load).
#include <math.h>

#include <algorithm>

#include "kernels.h"
#include "particle_common.h"

namespace pic {

namespace {

template <typename T>
__device__ __forceinline__ T gather9(const T *tile, int fw, int i0, int j0, const T wx[3],
                                     const T wy[3])
{
    // tile entry of node (i, j) is (j + 1) * fw + (i + 1)
    const T *r = tile + j0 * fw + i0;
    T acc = T(0);
#pragma unroll
    for (int b = 0; b < 3; ++b) {
        T row = r[b * fw] * wx[0] + r[b * fw + 1] * wx[1] + r[b * fw + 2] * wx[2];
        acc += row * wy[b];
    }
    return acc;
}

// PC > 0: every simulation of the launch has PC x PC-cell patches, so tile
// strides are compile-time constants and LDS offsets fold into instructions.
// FP32 512-thread workgroups are held to 128 VGPRs (4 waves per SIMD): two of
// them then share a CU, which their two 62 KB LDS tiles allow.
template <typename T, int BLOCK, int PC>
__global__ __launch_bounds__(BLOCK, (BLOCK == 512 && sizeof(T) == 4) ? 4 : 1) void k_particles2d(const SimDev<T> *__restrict__ sims,
                                                       const Item *__restrict__ items,
                                                       const int *__restrict__ nitems,
                                                       int *__restrict__ head, int fstride_rt,
                                                       int jstride_rt, ItemStamp *__restrict__ stamps)
{
    const int fstride = PC ? (PC + 3) * (PC + 3) : fstride_rt;
    const int jstride = PC ? (PC + 5) * (PC + 5) : jstride_rt;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    // current tile first (FP64 accumulation for either storage precision:
    // LDS float atomics are much slower here than FP64 ones), then fields
    long long *Jt = reinterpret_cast<long long *>(smem_raw);
    T *Ft = reinterpret_cast<T *>(Jt + 3 * jstride);
    __shared__ int s_item[2];

    const int tid = threadIdx.x, ln = tid % kWave;
    const int total = *nitems;
    // Items are claimed one ahead: the next index is requested while the
    // current item runs and published through the other of two LDS slots.
    if (tid == 0) s_item[0] = atomicAdd(head, 1);
    __syncthreads();
    int idx = __builtin_amdgcn_readfirstlane(s_item[0]);
    int slot = 1;
    // Kinetic energy: a running sum per lane, reduced over the wave and
    // added to the simulation's per-patch partials when the wave moves on to
    // another simulation and at the end (partials of different waves land
    // on different patches, so they rarely collide).
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
        const long long t_item = (stamps && tid == 0) ? wall_clock64() : 0;
        const int si = __builtin_amdgcn_readfirstlane(it.x & kItemSimMask);
        const int par = __builtin_amdgcn_readfirstlane(it.x >> 30);  // field level of this step
        const SimDev<T> &S = sims[si];
        const int p = __builtin_amdgcn_readfirstlane(it.y);
        const int64_t base = __builtin_amdgcn_readfirstlane(it.z);
        const int cnt = __builtin_amdgcn_readfirstlane(it.w);
        const int P0 = PC ? PC : S.P[0], P1 = PC ? PC : S.P[1];
        const int pxi = p % S.np[0], pyi = p / S.np[0];
        const int ox = pxi * P0, oy = pyi * P1;
        const int fw = P0 + 3, fh = P1 + 3, jw = P0 + 5, jh = P1 + 5;
        const int n0 = S.n[0], n1 = S.n[1], fn0 = S.fn[0];
        const int per0 = S.periodic[0], per1 = S.periodic[1];

        T *const *Fc = S.F[par];
        // the item's particles through 32-bit offsets from per-item bases
        // (positions x, y and momenta with weight u_x, u_y, u_z, w: one access each)
        const gptr_t<Vec2<T>> Pp = v2(S.pos) + base;
        const gptr_t<Vec4<T>> Mp = v4(S.mom) + base;
        const gptr_t<uint8_t> Cd = glb(S.code) + base;
        const T dt = S.dt, q = S.q, m = S.m;
        const T eps = q * dt / (T(2) * m);
        const T rdx = dt / S.d[0], rdy = dt / S.d[1];
        const double cx_ = -(double)q * (double)S.d[0] / (double)dt;
        const double cy_ = -(double)q * (double)S.d[1] / (double)dt;
        const double fs = fix_scale(S), fsinv = 1.0 / fs;  // fixed-point scale of the current
        const T Pmax0 = below((T)P0), Pmax1 = below((T)P1);
        const bool edge_lo = !per0 && pxi == 0, edge_hi = !per0 && pxi == S.np[0] - 1;
        if (si != kin_sim) {
            flush_kin();
            kin_sim = si;
        }
        kin_p = p;
        uint32_t err = 0;
        bool left = false;  // a particle of this lane changed patch or was removed
        float kin32 = 0.0f;

        // Lane mapping.  The item's particles are cut into units of 64
        // lanes.  Full passes of 64 S particles (S = lane_stride) give S units,
        // unit u taking particles 64 S (u / S) + l S + (u % S) for lanes
        // l = 0..63: a larger S spreads the lanes of a wave over more cells
        // (fewer LDS atomics on one address) but makes every particle load and
        // store touch more cache lines; S = 2 is the measured balance.  The
        // rest after the last full pass is cut into units of 64 consecutive
        // particles, so every unit holds at least one particle, and the lanes
        // past the item's end repeat its last particle with zero weight: they
        // compute and store the same values in the same instruction, and no
        // lane branches around a memory access (the compiler would otherwise
        // wait for the stores of one unit before starting the next).  Waves
        // take units round-robin; the next unit's particle is loaded before
        // the current one is pushed, and the first unit's before the field
        // tile is staged (the two latencies overlap).
        constexpr int NW = BLOCK / kWave;
        const int S_ = S.lane_stride;
        const int wv = __builtin_amdgcn_readfirstlane(tid / kWave);
        const int npass = cnt / (kWave * S_), ufull = npass * S_;
        const int uend = ufull + (cnt - npass * kWave * S_ + kWave - 1) / kWave;
        auto unit_particle = [&](int u) {
            return u < ufull ? kWave * S_ * (u / S_) + ln * S_ + (u % S_)
                             : kWave * S_ * npass + kWave * (u - ufull) + ln;
        };
        // an item holds at least one particle, so index cnt - 1 is valid
        T nx_, ny_, nux, nuy, nuz, nw_;
        auto load_unit = [&](int u) {
            const uint32_t kn = min(unit_particle(u), cnt - 1);  // unsigned: base + 32-bit offset addressing
            const Vec2<T> pv = *at(Pp, kn);
            const Vec4<T> mv = *at(Mp, kn);
            nx_ = pv.x; ny_ = pv.y;
            nux = mv.x; nuy = mv.y; nuz = mv.z; nw_ = mv.w;
        };
        load_unit(wv);
        // ---- stage E, B of nodes [ox-1, ox+P0+1] x [oy-1, oy+P1+1] --------
        // four nodes per thread per round, all loads issued before the stores
        for (int t0 = 0; t0 < fw * fh; t0 += 4 * BLOCK) {
            // Every load is unconditional, from node 0 where the tile node is
            // outside the grid or past the tile, and zeroed afterwards: a
            // load under a condition becomes a branch, and the compiler then
            // waits for each load before issuing the next.
            T v[4][6];
            bool ok[4][6];
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int t = t0 + r * BLOCK + tid;
                const bool in = t < fw * fh;
                const int tt = in ? t : 0;
                const int gi = ox - 1 + tt % fw, gj = oy - 1 + tt / fw;
                const int ip = axis_node(gi, n0, per0, 0), id = axis_node(gi, n0, per0, 1);
                const int jp = axis_node(gj, n1, per1, 0), jd = axis_node(gj, n1, per1, 1);
                // staggering: Ex (d,p) Ey (p,d) Ez (p,p) Bx (p,d) By (d,p) Bz (d,d)
                const int ix[6] = {id, ip, ip, ip, id, id}, jy[6] = {jp, jd, jp, jd, jp, jd};
#pragma unroll
                for (int c = 0; c < 6; ++c) {
                    ok[r][c] = in && ix[c] >= 0 && jy[c] >= 0;
                    v[r][c] = glb(Fc[c])[ok[r][c] ? ix[c] + fn0 * jy[c] : 0];
                }
            }
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int t = t0 + r * BLOCK + tid;
                if (t < fw * fh)
#pragma unroll
                    for (int c = 0; c < 6; ++c) Ft[c * fstride + t] = ok[r][c] ? v[r][c] : T(0);
            }
        }
        for (int t = tid; t < 3 * jstride; t += BLOCK) Jt[t] = 0;
        __syncthreads();
        if (tid == 0) s_item[slot] = next;  // read after the item's last barrier

        for (int u = wv; u < uend; u += NW) {
            const int kr = unit_particle(u);
            const uint32_t k = min(kr, cnt - 1);
            const T xl = nx_, yl = ny_;
            T ux = nux, uy = nuy, uz = nuz;
            const T wgt = kr < cnt ? nw_ : T(0);
            const T wst = nw_;  // stored back as loaded (lanes past the end repeat the last particle)
            load_unit(u + NW);

            // ---- gather ---------------------------------------------------
            const int ipx = (int)floor(xl + T(0.5)), idx_ = (int)floor(xl);
            const int ipy = (int)floor(yl + T(0.5)), idy = (int)floor(yl);
            T wpx[3], wdx[3], wpy[3], wdy[3];
            qweights(xl - (T)ipx, wpx[0], wpx[1], wpx[2]);
            qweights(xl - (T)idx_ - T(0.5), wdx[0], wdx[1], wdx[2]);
            qweights(yl - (T)ipy, wpy[0], wpy[1], wpy[2]);
            qweights(yl - (T)idy - T(0.5), wdy[0], wdy[1], wdy[2]);
            // node i0-1 sits at tile column i0, so the window starts at i0
            const T Ex = gather9(Ft + 0 * fstride, fw, idx_, ipy, wdx, wpy);
            const T Ey = gather9(Ft + 1 * fstride, fw, ipx, idy, wpx, wdy);
            const T Ez = gather9(Ft + 2 * fstride, fw, ipx, ipy, wpx, wpy);
            const T Bx = gather9(Ft + 3 * fstride, fw, ipx, idy, wpx, wdy);
            const T By = gather9(Ft + 4 * fstride, fw, idx_, ipy, wdx, wpy);
            const T Bz = gather9(Ft + 5 * fstride, fw, idx_, idy, wdx, wdy);

            // ---- Boris ------------------------------------------------------
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
            // w m ((gamma0 - 1) + (gamma1 - 1)) / 2 with gamma - 1 = u^2 / (gamma + 1)
            // (no cancellation; FP32 storage keeps the diagnostic in FP32
            // arithmetic: a per-lane FP32 sum over the item, without the
            // factor m / 2, added to the FP64 running sum once per item)
            if constexpr (sizeof(T) == 4) {
                const float a0 = 1.0f + usq0;
                const float g0p = a0 * rsq_(a0) + 1.0f, g1p = (1.0f + usq1) * ig1 + 1.0f;
                kin32 += wgt * (usq0 * g1p + usq1 * g0p) * rcp_(g0p * g1p);
            } else {
                const double g0p = sqrt(1.0 + (double)usq0) + 1.0;
                const double g1p = (double)(T(1) + usq1) * (double)ig1 + 1.0;
                kin += (double)wgt * (double)m * 0.5 *
                       ((double)usq0 * g1p + (double)usq1 * g0p) / (g0p * g1p);
            }

            // ---- move and classify -------------------------------------------
            const T dxl = rdx * ux * ig1, dyl = rdy * uy * ig1;
            uint8_t code;
            T x1 = xl + dxl, y1 = yl + dyl;
            if (!(fabs(dxl) < T(1) && fabs(dyl) < T(1))) {
                err |= (isfinite(ux) && isfinite(uy) && isfinite(uz)) ? kFlagCFL : kFlagNaN;
                code = kRemoved;
                x1 = xl;
                y1 = yl;
            } else {
                // ---- Esirkepov deposit on a 4x4 node window ------------------
                // Only window slot 3 of an axis depends on whether the nearest
                // node changed; its entries are exactly zero otherwise and their
                // atomics are skipped (masked lanes cost the LDS nothing).
                int mx, my;
                double S0x[4], DSx[4], S0y[4], DSy[4];
                const bool cx = window4(xl, (double)dxl, mx, S0x, DSx);
                const bool cy = window4(yl, (double)dyl, my, S0y, DSy);
                const double qw = (double)wgt;
                // factors of the current carry the fixed-point scale fs
                const double az = (double)q * qw * (double)(uz * ig1) * fs;
                long long *Jxt = Jt, *Jyt = Jt + jstride, *Jzt = Jt + 2 * jstride;
                const int r0 = (my + 2) * jw + (mx + 2);
                // time-averaged transverse weights
                double wx[4], wy[4];
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    wx[k] = S0x[k] + 0.5 * DSx[k];
                    wy[k] = S0y[k] + 0.5 * DSy[k];
                }
                if (dxl != T(0) || dyl != T(0)) {
                    // Jx on dual x nodes: running sums of -q w (dx/dt) DSx, times wy
                    double px[3], py[3];
                    const double cq = cx_ * qw * fs, dq = cy_ * qw * fs;
                    px[0] = cq * DSx[0];
                    px[1] = px[0] + cq * DSx[1];
                    px[2] = px[1] + cq * DSx[2];
                    py[0] = dq * DSy[0];
                    py[1] = py[0] + dq * DSy[1];
                    py[2] = py[1] + dq * DSy[2];
#pragma unroll
                    for (int j = 0; j < 3; ++j) {
                        fix_add_prod(&Jxt[r0 + j * jw + 0], px[0], wy[j]);
                        fix_add_prod(&Jxt[r0 + j * jw + 1], px[1], wy[j]);
                        if (cx) fix_add_prod(&Jxt[r0 + j * jw + 2], px[2], wy[j]);
                    }
                    if (cy) {
                        fix_add_prod(&Jxt[r0 + 3 * jw + 0], px[0], wy[3]);
                        fix_add_prod(&Jxt[r0 + 3 * jw + 1], px[1], wy[3]);
                        if (cx) fix_add_prod(&Jxt[r0 + 3 * jw + 2], px[2], wy[3]);
                    }
                    // Jy on dual y nodes: running sums along y, times wx
#pragma unroll
                    for (int i = 0; i < 3; ++i) {
                        fix_add_prod(&Jyt[r0 + 0 * jw + i], py[0], wx[i]);
                        fix_add_prod(&Jyt[r0 + 1 * jw + i], py[1], wx[i]);
                        if (cy) fix_add_prod(&Jyt[r0 + 2 * jw + i], py[2], wx[i]);
                    }
                    if (cx) {
                        fix_add_prod(&Jyt[r0 + 0 * jw + 3], py[0], wx[3]);
                        fix_add_prod(&Jyt[r0 + 1 * jw + 3], py[1], wx[3]);
                        if (cy) fix_add_prod(&Jyt[r0 + 2 * jw + 3], py[2], wx[3]);
                    }
                }
                if (az != 0.0) {
                    // Jz = q w vz (S0x S0y + DSx S0y / 2 + S0x DSy / 2 + DSx DSy / 3)
                    //    = q w vz (wx S0y + bx DSy), bx = S0x / 2 + DSx / 3
                    double ax_[4], bx_[4];
#pragma unroll
                    for (int k = 0; k < 4; ++k) {
                        ax_[k] = az * wx[k];
                        bx_[k] = az * (0.5 * S0x[k] + DSx[k] * (1.0 / 3.0));
                    }
#pragma unroll
                    for (int j = 0; j < 3; ++j) {
#pragma unroll
                        for (int i = 0; i < 3; ++i)
                            fix_add_2prod(&Jzt[r0 + j * jw + i], ax_[i], S0y[j], bx_[i], DSy[j]);
                        if (cx) fix_add_2prod(&Jzt[r0 + j * jw + 3], ax_[3], S0y[j], bx_[3], DSy[j]);
                    }
                    if (cy) {
#pragma unroll
                        for (int i = 0; i < 3; ++i)
                            fix_add_2prod(&Jzt[r0 + 3 * jw + i], ax_[i], S0y[3], bx_[i], DSy[3]);
                        if (cx) fix_add_2prod(&Jzt[r0 + 3 * jw + 3], ax_[3], S0y[3], bx_[3], DSy[3]);
                    }
                }

                const int sx_ = x1 < T(0) ? -1 : (x1 >= (T)P0 ? 1 : 0);
                const int sy_ = y1 < T(0) ? -1 : (y1 >= (T)P1 ? 1 : 0);
                const bool gone = (sx_ < 0 && edge_lo) || (sx_ > 0 && edge_hi);
                x1 -= (T)(sx_ * P0);
                y1 -= (T)(sy_ * P1);
                if (x1 > Pmax0) x1 = Pmax0;
                if (y1 > Pmax1) y1 = Pmax1;
                code = gone ? kRemoved : (uint8_t)((sx_ + 1) + 3 * (sy_ + 1));
            }
            *at(Pp, k) = Vec2<T>{x1, y1};
            *at(Mp, k) = Vec4<T>{ux, uy, uz, wst};
            *at(Cd, k) = code;
            left |= code != kStay2;
        }
        kin += 0.5 * (double)m * (double)kin32;
        // the re-binning scans only patches that may have leavers
        if (__ballot(left) && ln == 0) *glb(S.moved + p) = 1;
        if (err) __hip_atomic_fetch_or(&glb(S.st)->flags, err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __syncthreads();

        // ---- flush the current tile -------------------------------------------
        {
            const gptr_t<T> Jgx = glb(S.J[par][0]), Jgy = glb(S.J[par][1]), Jgz = glb(S.J[par][2]);
            const bool det = S.det != 0;
            for (int t = tid; t < jw * jh; t += BLOCK) {
                const int gi = ox - 2 + t % jw, gj = oy - 2 + t / jw;
                const int ip = axis_node(gi, n0, per0, 0), id = axis_node(gi, n0, per0, 1);
                const int jp = axis_node(gj, n1, per1, 0), jd = axis_node(gj, n1, per1, 1);
                const long long vx = Jt[t], vy = Jt[jstride + t], vz = Jt[2 * jstride + t];
                const bool kx = vx != 0 && id >= 0 && jp >= 0, ky = vy != 0 && ip >= 0 && jd >= 0;
                const bool kz = vz != 0 && ip >= 0 && jp >= 0;
                // deterministic: integer adds to the fixed-point accumulators;
                // else the values in storage precision through float atomics
                if (det) {
                    if (kx) gadd(glb(S.Jacc[0]) + (id + fn0 * jp), (int64_t)vx);
                    if (ky) gadd(glb(S.Jacc[1]) + (ip + fn0 * jd), (int64_t)vy);
                    if (kz) gadd(glb(S.Jacc[2]) + (ip + fn0 * jp), (int64_t)vz);
                } else {
                    if (kx) gadd(Jgx + (id + fn0 * jp), (T)((double)vx * fsinv));
                    if (ky) gadd(Jgy + (ip + fn0 * jd), (T)((double)vy * fsinv));
                    if (kz) gadd(Jgz + (ip + fn0 * jp), (T)((double)vz * fsinv));
                }
            }
        }
        __syncthreads();
        if (stamps && tid == 0) record_item(stamps + idx, t_item, si, p, it.w);
        idx = __builtin_amdgcn_readfirstlane(s_item[slot]);
        slot ^= 1;
    }
    flush_kin();
}

template <typename T>
size_t lds_bytes(int maxP0, int maxP1, int &fstride, int &jstride)
{
    fstride = (maxP0 + 3) * (maxP1 + 3);
    jstride = (maxP0 + 5) * (maxP1 + 5);
    return sizeof(int64_t) * (size_t)(3 * jstride) + sizeof(T) * (size_t)(6 * fstride);
}

}  // namespace

template <typename T, int BLOCK>
static void launch_pc(int pc, const SimDev<T> *sims, const Item *items, const int *nitems, int *head,
                      int grid, size_t lds, int fs, int js, ItemStamp *stamps, hipStream_t st, Ev2 ev)
{
    if (pc == 32)
        hipExtLaunchKernelGGL((k_particles2d<T, BLOCK, 32>), dim3(grid), dim3(BLOCK), lds, st,
                              ev.start, ev.stop, 0, sims, items, nitems, head, fs, js, stamps);
    else if (pc == 16)
        hipExtLaunchKernelGGL((k_particles2d<T, BLOCK, 16>), dim3(grid), dim3(BLOCK), lds, st,
                              ev.start, ev.stop, 0, sims, items, nitems, head, fs, js, stamps);
    else
        hipExtLaunchKernelGGL((k_particles2d<T, BLOCK, 0>), dim3(grid), dim3(BLOCK), lds, st,
                              ev.start, ev.stop, 0, sims, items, nitems, head, fs, js, stamps);
}

template <typename T>
void launch_particles(const SimDev<T> *sims, const Item *items, const int *nitems, int *head,
                      int grid, int block, int maxP0, int maxP1, int pc, ItemStamp *stamps,
                      hipStream_t st, Ev2 ev)
{
    int fs, js;
    size_t lds = lds_bytes<T>(maxP0, maxP1, fs, js);
    if (block == 1024) launch_pc<T, 1024>(pc, sims, items, nitems, head, grid, lds, fs, js, stamps, st, ev);
    else if (block == 512) launch_pc<T, 512>(pc, sims, items, nitems, head, grid, lds, fs, js, stamps, st, ev);
    else launch_pc<T, 256>(pc, sims, items, nitems, head, grid, lds, fs, js, stamps, st, ev);
}

template <typename T>
int particles_occupancy(int block, int maxP0, int maxP1)
{
    int fs, js, nb = 0;
    size_t lds = lds_bytes<T>(maxP0, maxP1, fs, js);
    hipError_t e;
    const void *f;
    if (block == 1024) {
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_particles2d<T, 1024, 0>, 1024, lds);
        f = (const void *)k_particles2d<T, 1024, 0>;
    } else if (block == 512) {
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_particles2d<T, 512, 0>, 512, lds);
        f = (const void *)k_particles2d<T, 512, 0>;
    } else {
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_particles2d<T, 256, 0>, 256, lds);
        f = (const void *)k_particles2d<T, 256, 0>;
    }
    const int own = resident_workgroups(f, block, lds);
    return std::max(e == hipSuccess ? nb : 0, own);
}

template void launch_particles<float>(const SimDev<float> *, const Item *, const int *, int *, int,
                                      int, int, int, int, ItemStamp *, hipStream_t, Ev2);
template void launch_particles<double>(const SimDev<double> *, const Item *, const int *, int *,
                                       int, int, int, int, int, ItemStamp *, hipStream_t, Ev2);
template int particles_occupancy<float>(int, int, int);
template int particles_occupancy<double>(int, int, int);

}  // namespace pic
