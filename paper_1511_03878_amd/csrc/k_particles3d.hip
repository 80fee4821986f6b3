// Fused particle kernel of the 3-D patch-PIC step (periodic boxes): per work
// item (a chunk of one patch) stage the patch's E and B into LDS, then per
// particle gather with quadratic shapes on 27 nodes, relativistic Boris push,
// move, classify the destination among the 26 neighbours, and deposit the
// charge-conserving (Esirkepov) current into a 64-bit fixed-point LDS tile
// (exact integer sums, so the tile does not depend on the order of the
// atomics) that is flushed to the global current once per item.
//
// Deposit in two classes.  A particle whose nearest node changes on no axis
// has a fixed window (2 x 3 x 3 entries per current component, 54 LDS
// atomics); one whose nearest node changes on some axis (about one in six in
// a 10 keV plasma at the Courant limit) needs up to 4 x 4 x 3 per component
// (144).  A masked LDS atomic costs a wave as much as a full one, so mixing
// the two in one wave would issue the full window for nearly every wave.
// The second class is deferred instead: its momentum is stored, its old
// position left in memory, and its slot listed in LDS; the list is deposited
// 64 particles at a time, and what remains at the end of an item is pooled
// over the workgroup's waves.
//
// Staggering (half a cell up): Ex, Ey, Ez along their own axis; Bx, By, Bz
// along the two other axes.  Each component's tile holds just the nodes its
// stencil can reach from a particle of the patch: on an axis where the
// component sits on primal nodes the gather reads nodes -1 .. P+1 (P + 3),
// where it sits half a cell up -1 .. P (P + 2); the current J_a spans dual
// nodes -2 .. P+1 along a (P + 4) and primal nodes -2 .. P+2 across (P + 5).
// For 8^3-cell patches the two tiles take 76 KB (FP32 fields, 64-bit
// currents), so two workgroups share a CU.  Patch shapes 8 x 8 x 8 and
// 8 x 8 x 4 are compiled with constant tile pitches (LDS offsets become
// instruction immediates); other shapes take the general kernel.
#include <algorithm>
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

// Esirkepov deposit of one particle into the fixed-point current tiles (fs: scale):
// W_a = DS_a (S0_b S0_c + DS_b S0_c / 2 + S0_b DS_c / 2 + DS_b DS_c / 3)
//     = DS_a (A_b S0_c + B_b DS_c) with A = S0 + DS / 2, B = S0 / 2 + DS / 3,
// and J_a is the running sum of -q w (d_a / dt) W_a along a (cq, dq, eq hold
// -q w d_a / dt).  Window slot 3 of an axis carries weight only when the
// particle's nearest node on that axis changed (c_a).  FULL = false is the
// fixed window of a particle whose nearest node changed on no axis (2 x 3 x 3
// entries per component); FULL = true takes each lane's own extents.
template <bool FULL, typename W>
__device__ __forceinline__ void deposit_window(long long *Jxt, long long *Jyt, long long *Jzt, const int jpl[3],
                                               const int jrow[3], int mx, int my, int mz, bool cx, bool cy,
                                               bool cz, const W S0x[4], const W DSx[4], const W S0y[4],
                                               const W DSy[4], const W S0z[4], const W DSz[4], W cq, W dq,
                                               W eq, double fs)
{
    W Ax[4], Bx[4], Ay[4], By[4];
#pragma unroll
    for (int k2 = 0; k2 < 4; ++k2) {
        Ax[k2] = S0x[k2] + W(0.5) * DSx[k2];
        Bx[k2] = W(0.5) * S0x[k2] + DSx[k2] * W(1.0 / 3.0);
        Ay[k2] = S0y[k2] + W(0.5) * DSy[k2];
        By[k2] = W(0.5) * S0y[k2] + DSy[k2] * W(1.0 / 3.0);
    }
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
    // running sums carry the fixed-point scale (FP64: each atomic's integer
    // then comes from one fused multiply-add)
    double pxd[3], pyd[3], pzd[3];
#pragma unroll
    for (int k2 = 0; k2 < 3; ++k2) {
        pxd[k2] = (double)px[k2] * fs;
        pyd[k2] = (double)py[k2] * fs;
        pzd[k2] = (double)pz[k2] * fs;
    }
    const int rx = (mz + 2) * jpl[0] + (my + 2) * jrow[0] + (mx + 2);
    const int ry = (mz + 2) * jpl[1] + (my + 2) * jrow[1] + (mx + 2);
    const int rz = (mz + 2) * jpl[2] + (my + 2) * jrow[2] + (mx + 2);
    // prefix entries (the last one is the particle's net zero) and transverse extents
    const int ni = FULL && cx ? 3 : 2, nj = FULL && cy ? 3 : 2, nk = FULL && cz ? 3 : 2;
    const int mi = FULL && cx ? 4 : 3, mj = FULL && cy ? 4 : 3, mk = FULL && cz ? 4 : 3;
    // Jx: dual x (prefix index i), transverse (j, k)
#pragma unroll
    for (int kk = 0; kk < 4; ++kk) {
        if (kk >= mk) break;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            if (j >= mj) break;
            const W tr = Ay[j] * S0z[kk] + By[j] * DSz[kk];
#pragma unroll
            for (int i = 0; i < 3; ++i) {
                if (i >= ni) break;
                fix_add_prod(&Jxt[rx + kk * jpl[0] + j * jrow[0] + i], pxd[i], (double)tr);
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
            const W tr = Ax[i] * S0z[kk] + Bx[i] * DSz[kk];
#pragma unroll
            for (int j = 0; j < 3; ++j) {
                if (j >= nj) break;
                fix_add_prod(&Jyt[ry + kk * jpl[1] + j * jrow[1] + i], pyd[j], (double)tr);
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
            const W tr = Ax[i] * S0y[j] + Bx[i] * DSy[j];
#pragma unroll
            for (int kk = 0; kk < 3; ++kk) {
                if (kk >= nk) break;
                fix_add_prod(&Jzt[rz + kk * jpl[2] + j * jrow[2] + i], pzd[kk], (double)tr);
            }
        }
    }
}

// A wave deposits its deferred list once it would pass this many entries
// (at most 64, the list's size).
constexpr int kDeferBatch = 64;

// Per-component tile geometry: entries of component c along axis a.
__host__ __device__ constexpr int fext(int P, int c, int a)
{
    // E_c is half a cell up along c; B_c along the two other axes
    return P + 3 - (c < 3 ? (a == c ? 1 : 0) : (a == c - 3 ? 0 : 1));
}
__host__ __device__ constexpr int jext(int P, int c, int a) { return P + 5 - (a == c ? 1 : 0); }

// FP32 512-thread workgroups are held to 128 VGPRs (4 waves per SIMD), so
// two of them share a CU (their LDS tiles fit twice in 160 KB for 8^3
// patches); the FP64 kernel would spill at that bound.
template <typename T, int BLOCK, int PX, int PY, int PZ>
__global__ __launch_bounds__(BLOCK, (BLOCK == 512 && sizeof(T) == 4) ? 4 : 1) void k_particles3d(const SimDev<T> *__restrict__ sims,
                                                       const Item *__restrict__ items,
                                                       const int *__restrict__ nitems,
                                                       int *__restrict__ head,
                                                       ItemStamp *__restrict__ stamps)
{
    using W = typename std::conditional<sizeof(T) == 4, float, double>::type;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    __shared__ int s_item[2];
    __shared__ int s_q[BLOCK / kWave][kWave];  // per wave: slots of deferred particles
    __shared__ int s_qn[BLOCK / kWave];

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
        const long long t_item = (stamps && tid == 0) ? wall_clock64() : 0;
        const int si = __builtin_amdgcn_readfirstlane(it.x & kItemSimMask);
        const int par = __builtin_amdgcn_readfirstlane(it.x >> 30);
        const SimDev<T> &S = sims[si];
        const int p = __builtin_amdgcn_readfirstlane(it.y);
        const int64_t base = __builtin_amdgcn_readfirstlane(it.z);
        const int cnt = __builtin_amdgcn_readfirstlane(it.w);
        const int P0 = PX ? PX : S.P[0], P1 = PY ? PY : S.P[1], P2 = PZ ? PZ : S.P[2];
        const int pxi = p % S.np[0], pyi = (p / S.np[0]) % S.np[1], pzi = p / (S.np[0] * S.np[1]);
        const int ox = pxi * P0, oy = pyi * P1, oz = pzi * P2;
        // staging box (every component's tile fits in it) and current box
        const int fw = P0 + 3, fh = P1 + 3, fwh = fw * fh, fstride = fwh * (P2 + 3);
        const int jw = P0 + 5, jh = P1 + 5, jwh = jw * jh, jstride = jwh * (P2 + 5);
        // component tiles: row pitch, plane pitch and start of each
        int frow[6], fpl[6], fofs[6], jrow[3], jpl[3], jofs[3];
        {
            int o = 0;
#pragma unroll
            for (int c = 0; c < 6; ++c) {
                frow[c] = fext(P0, c, 0);
                fpl[c] = frow[c] * fext(P1, c, 1);
                fofs[c] = o;
                o += fpl[c] * fext(P2, c, 2);
            }
            o = 0;
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                jrow[c] = jext(P0, c, 0);
                jpl[c] = jrow[c] * jext(P1, c, 1);
                jofs[c] = o;
                o += jpl[c] * jext(P2, c, 2);
            }
        }
        const int jtot = jofs[2] + jpl[2] * jext(P2, 2, 2);
        long long *Jt = reinterpret_cast<long long *>(smem_raw);
        T *Ft = reinterpret_cast<T *>(Jt + jtot);
        const int n0 = S.n[0], n1 = S.n[1], n2 = S.n[2];
        const int fn0 = S.fn[0], fn1 = S.fn[1];
        if (si != kin_sim) {
            flush_kin();
            kin_sim = si;
        }
        kin_p = p;

        // (positions x, y, z with the id and momenta with weight u_x, u_y,
        // u_z, w: one access each; the id and the weight are stored back as
        // loaded)
        const gptr_t<Vec4<T>> Pp = v4(S.pos) + base;
        const gptr_t<Vec4<T>> Mp = v4(S.mom) + base;
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
        T nx_, ny_, nz_, nid, nux, nuy, nuz, nw_;
        auto load_unit = [&](int u) {
            const int kn = min(unit_particle(u), cnt - 1);
            const Vec4<T> pv = Pp[kn];
            const Vec4<T> mv = Mp[kn];
            nx_ = pv.x; ny_ = pv.y; nz_ = pv.z; nid = pv.w;
            nux = mv.x; nuy = mv.y; nuz = mv.z; nw_ = mv.w;
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
                if (t < fstride) {
                    const int a = t % fw, b = (t / fw) % fh, c = t / fwh;
#pragma unroll
                    for (int cc = 0; cc < 6; ++cc)
                        if (a < fext(P0, cc, 0) && b < fext(P1, cc, 1) && c < fext(P2, cc, 2))
                            Ft[fofs[cc] + c * fpl[cc] + b * frow[cc] + a] = v[r][cc];
                }
            }
        }
        for (int t = tid; t < jtot; t += BLOCK) Jt[t] = 0;
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
        long long *Jxt = Jt + jofs[0], *Jyt = Jt + jofs[1], *Jzt = Jt + jofs[2];
        const double fs = fix_scale(S), fsinv = 1.0 / fs;  // fixed-point scale of the current

        // new position inside the patch (wrapped by one patch edge, kept
        // below P in storage precision) and the destination code
        auto place = [&](T &x1, T &y1, T &z1) -> uint8_t {
            const int sx_ = x1 < T(0) ? -1 : (x1 >= (T)P0 ? 1 : 0);
            const int sy_ = y1 < T(0) ? -1 : (y1 >= (T)P1 ? 1 : 0);
            const int sz_ = z1 < T(0) ? -1 : (z1 >= (T)P2 ? 1 : 0);
            x1 -= (T)(sx_ * P0);
            y1 -= (T)(sy_ * P1);
            z1 -= (T)(sz_ * P2);
            if (x1 > Pmax0) x1 = Pmax0;
            if (y1 > Pmax1) y1 = Pmax1;
            if (z1 > Pmax2) z1 = Pmax2;
            return (uint8_t)((sx_ + 1) + 3 * (sy_ + 1) + 9 * (sz_ + 1));
        };
        // Deferred particles (nearest node changed on some axis): their
        // momentum is already stored and their old position is still in
        // memory; deposit on the full window, then store position and code.
        auto push_deferred = [&](bool valid, int kq) {
            const int k = valid ? kq : 0;
            const Vec4<T> pk = Pp[k];
            const Vec4<T> mk = Mp[k];
            const T xl = pk.x, yl = pk.y, zl = pk.z;
            const T ux = mk.x, uy = mk.y, uz = mk.z;
            const W qw = valid ? (W)mk.w : W(0);
            const T ig1 = rsq_(T(1) + (ux * ux + uy * uy + uz * uz));
            const T dxl = rdx * ux * ig1, dyl = rdy * uy * ig1, dzl = rdz * uz * ig1;
            int mx, my, mz;
            W S0x[4], DSx[4], S0y[4], DSy[4], S0z[4], DSz[4];
            const bool cx = window4(xl, (double)dxl, mx, S0x, DSx);
            const bool cy = window4(yl, (double)dyl, my, S0y, DSy);
            const bool cz = window4(zl, (double)dzl, mz, S0z, DSz);
            if (valid)
                deposit_window<true>(Jxt, Jyt, Jzt, jpl, jrow, mx, my, mz, cx, cy, cz, S0x, DSx, S0y, DSy,
                                     S0z, DSz, (W)cx_ * qw, (W)cy_ * qw, (W)cz_ * qw, fs);
            T x1 = xl + dxl, y1 = yl + dyl, z1 = zl + dzl;
            const uint8_t code = place(x1, y1, z1);
            if (valid) {
                Pp[k] = Vec4<T>{x1, y1, z1, pk.w};
                Cd[k] = code;
                left |= code != kStay3;
            }
        };
        int qn = 0;  // entries in this wave's deferred list (wave-uniform)

        for (int u = wv; u < uend; u += NW) {
            const int kr = unit_particle(u), k = min(kr, cnt - 1);
            const T xl = nx_, yl = ny_, zl = nz_;
            T ux = nux, uy = nuy, uz = nuz;
            const T wgt = kr < cnt ? nw_ : T(0);
            const T wst = nw_, ist = nid;  // stored back as loaded (lanes past the end repeat the last particle)
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
            const T Ex = gather27(Ft + fofs[0], frow[0], fpl[0], id[0], ip[1], ip[2], wd[0], wp[1], wp[2]);
            const T Ey = gather27(Ft + fofs[1], frow[1], fpl[1], ip[0], id[1], ip[2], wp[0], wd[1], wp[2]);
            const T Ez = gather27(Ft + fofs[2], frow[2], fpl[2], ip[0], ip[1], id[2], wp[0], wp[1], wd[2]);
            const T Bx = gather27(Ft + fofs[3], frow[3], fpl[3], ip[0], id[1], id[2], wp[0], wd[1], wd[2]);
            const T By = gather27(Ft + fofs[4], frow[4], fpl[4], id[0], ip[1], id[2], wd[0], wp[1], wd[2]);
            const T Bz = gather27(Ft + fofs[5], frow[5], fpl[5], id[0], id[1], ip[2], wd[0], wd[1], wp[2]);

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

            // ---- move, deposit, classify ---------------------------------------
            const T dxl = rdx * ux * ig1, dyl = rdy * uy * ig1, dzl = rdz * uz * ig1;
            uint8_t code;
            bool defer = false;
            T x1 = xl + dxl, y1 = yl + dyl, z1 = zl + dzl;
            if (!(fabs(dxl) < T(1) && fabs(dyl) < T(1) && fabs(dzl) < T(1))) {
                err |= (isfinite(ux) && isfinite(uy) && isfinite(uz)) ? kFlagCFL : kFlagNaN;
                code = kRemoved;
                x1 = xl;
                y1 = yl;
                z1 = zl;
            } else {
                if (dxl != T(0) || dyl != T(0) || dzl != T(0)) {
                    // weights and products in W (FP32 for FP32 storage: fewer live
                    // registers, so more waves fit); sums in the fixed-point tile
                    int mx, my, mz;
                    W S0x[4], DSx[4], S0y[4], DSy[4], S0z[4], DSz[4];
                    const bool cx = window4(xl, (double)dxl, mx, S0x, DSx);
                    const bool cy = window4(yl, (double)dyl, my, S0y, DSy);
                    const bool cz = window4(zl, (double)dzl, mz, S0z, DSz);
                    defer = cx || cy || cz;
                    if (!defer) {
                        const W qw = (W)wgt;
                        deposit_window<false>(Jxt, Jyt, Jzt, jpl, jrow, mx, my, mz, false, false, false, S0x,
                                              DSx, S0y, DSy, S0z, DSz, (W)cx_ * qw, (W)cy_ * qw, (W)cz_ * qw,
                                              fs);
                    }
                }
                code = place(x1, y1, z1);
            }
            // a deferred particle keeps its old position in memory until its
            // deposit (stores stay unconditional: the same value is rewritten)
            Pp[k] = Vec4<T>{defer ? xl : x1, defer ? yl : y1, defer ? zl : z1, ist};
            Mp[k] = Vec4<T>{ux, uy, uz, wst};
            Cd[k] = code;
            left |= !defer && code != kStay3;

            // ---- deferred list: batches of 64 on the full window ---------------
            // (lanes past the item's end repeat its last particle and are not
            // listed: the real lane lists it)
            const bool listed = defer && kr < cnt;
            const uint64_t dm = __ballot(listed);
            const int c = __popcll(dm);
            if (qn + c > kDeferBatch) {
                push_deferred(ln < qn, s_q[wv][ln]);
                qn = 0;
            }
            // rank among the listed lanes below this one
            const int rank = __builtin_amdgcn_mbcnt_hi((uint32_t)(dm >> 32),
                                                       __builtin_amdgcn_mbcnt_lo((uint32_t)dm, 0u));
            if (listed) s_q[wv][qn + rank] = k;
            qn += c;
        }

        // ---- what is left on the deferred lists of all waves, 64 per wave ---
        if (ln == 0) s_qn[wv] = qn;
        __syncthreads();
        {
            int pre[NW + 1];
            pre[0] = 0;
#pragma unroll
            for (int w = 0; w < NW; ++w) pre[w + 1] = pre[w] + __builtin_amdgcn_readfirstlane(s_qn[w]);
            const int L = pre[NW];
            for (int e0 = wv * kWave; e0 < L; e0 += BLOCK) {
                const int e = e0 + ln;
                // source wave and position of entry e (selects, no indexed registers)
                int src = 0, off = e;
#pragma unroll
                for (int w = 1; w < NW; ++w)
                    if (e >= pre[w]) {
                        src = w;
                        off = e - pre[w];
                    }
                const bool valid = e < L;
                const int k = s_q[src][valid ? off : 0];  // always an in-range entry
                push_deferred(valid, k);
            }
        }
        if (__ballot(left) && ln == 0) *glb(S.moved + p) = 1;
        if (err)
            __hip_atomic_fetch_or(&glb(S.st)->flags, err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __syncthreads();

        // ---- flush the current tile (nodes [o-2, o+P+2] on every axis) ------
        // deterministic: integer adds to the fixed-point accumulators; else
        // the tile's values in storage precision through float atomics
        {
            const gptr_t<T> Jgx = glb(S.J[par][0]), Jgy = glb(S.J[par][1]), Jgz = glb(S.J[par][2]);
            const bool det = S.det != 0;
            for (int t = tid; t < jstride; t += BLOCK) {
                const int a = t % jw, b = (t / jw) % jh, c = t / jwh;
                const int gi = axis_node(ox - 2 + a, n0, 1, 0);
                const int gj = axis_node(oy - 2 + b, n1, 1, 0);
                const int gk = axis_node(oz - 2 + c, n2, 1, 0);
                const int64_t k = gi + (int64_t)fn0 * (gj + (int64_t)fn1 * gk);
                // entries outside a component's tile hold no current
                const long long vx = a < jrow[0] ? Jt[jofs[0] + c * jpl[0] + b * jrow[0] + a] : 0;
                const long long vy = b < jext(P1, 1, 1) ? Jt[jofs[1] + c * jpl[1] + b * jrow[1] + a] : 0;
                const long long vz = c < jext(P2, 2, 2) ? Jt[jofs[2] + c * jpl[2] + b * jrow[2] + a] : 0;
                if (det) {
                    if (vx) gadd(glb(S.Jacc[0]) + k, (int64_t)vx);
                    if (vy) gadd(glb(S.Jacc[1]) + k, (int64_t)vy);
                    if (vz) gadd(glb(S.Jacc[2]) + k, (int64_t)vz);
                } else {
                    if (vx) gadd(Jgx + k, (T)((double)vx * fsinv));
                    if (vy) gadd(Jgy + k, (T)((double)vy * fsinv));
                    if (vz) gadd(Jgz + k, (T)((double)vz * fsinv));
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

}  // namespace

size_t particles3d_lds_bytes(int precision, int P0, int P1, int P2)
{
    size_t js = 0, fs = 0;
    for (int c = 0; c < 3; ++c) js += (size_t)jext(P0, c, 0) * jext(P1, c, 1) * jext(P2, c, 2);
    for (int c = 0; c < 6; ++c) fs += (size_t)fext(P0, c, 0) * fext(P1, c, 1) * fext(P2, c, 2);
    return sizeof(int64_t) * js + (size_t)(precision / 8) * fs;
}

namespace {

// The kernel for a launch: shape 1 = every patch 8 x 8 x 8, 2 = 8 x 8 x 4,
// 0 = general.
template <typename T, int BLOCK>
auto kernel_for(int shape) -> decltype(&k_particles3d<T, BLOCK, 0, 0, 0>)
{
    if (shape == 1) return &k_particles3d<T, BLOCK, 8, 8, 8>;
    if (shape == 2) return &k_particles3d<T, BLOCK, 8, 8, 4>;
    return &k_particles3d<T, BLOCK, 0, 0, 0>;
}

template <typename T>
auto kernel_for(int block, int shape) -> decltype(&k_particles3d<T, 512, 0, 0, 0>)
{
    if (block == 1024) return kernel_for<T, 1024>(shape);
    if (block == 256) return kernel_for<T, 256>(shape);
    return kernel_for<T, 512>(shape);
}

}  // namespace

int particles3d_shape(int P0, int P1, int P2)
{
    if (P0 == 8 && P1 == 8 && P2 == 8) return 1;
    if (P0 == 8 && P1 == 8 && P2 == 4) return 2;
    return 0;
}

template <typename T>
void launch_particles3d(const SimDev<T> *sims, const Item *items, const int *nitems, int *head,
                        int grid, int block, int maxP0, int maxP1, int maxP2, int shape,
                        ItemStamp *stamps, hipStream_t st, Ev2 ev)
{
    const size_t lds = particles3d_lds_bytes(sizeof(T) * 8, maxP0, maxP1, maxP2);
    const int b = block == 1024 || block == 256 ? block : 512;
    hipExtLaunchKernelGGL(kernel_for<T>(b, shape), dim3(grid), dim3(b), lds, st, ev.start, ev.stop, 0, sims,
                          items, nitems, head, stamps);
}

template <typename T>
int particles3d_occupancy(int block, int maxP0, int maxP1, int maxP2, int shape)
{
    const size_t lds = particles3d_lds_bytes(sizeof(T) * 8, maxP0, maxP1, maxP2);
    const int b = block == 1024 || block == 256 ? block : 512;
    int nb = 0;
    const hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, kernel_for<T>(b, shape), b, lds);
    const int own = resident_workgroups((const void *)kernel_for<T>(b, shape), b, lds);
    return std::max(e == hipSuccess ? nb : 0, own);
}

template void launch_particles3d<float>(const SimDev<float> *, const Item *, const int *, int *, int,
                                        int, int, int, int, int, ItemStamp *, hipStream_t, Ev2);
template void launch_particles3d<double>(const SimDev<double> *, const Item *, const int *, int *,
                                         int, int, int, int, int, int, ItemStamp *, hipStream_t, Ev2);
template int particles3d_occupancy<float>(int, int, int, int, int);
template int particles3d_occupancy<double>(int, int, int, int, int);

}  // namespace pic
