// Particle merging (dynamic load limiting, section 3.2), 2-D.
//
// Where a cell holds more than cmax particles, their momenta u = p / (m c)
// are grouped by weighted Lloyd iterations into k = cmax / 2 clusters
// (centroids start at the momenta of members floor(j n / k) in slot order;
// each round assigns every member to its nearest centroid, lowest index on
// ties, and moves every non-empty centroid to its cluster's weighted mean).
// A final cluster of three or more members becomes two particles of half its
// weight W each, at its weighted mean position, with momenta
// |u_t| (cos t e1 +- sin t e2): gamma_t = E / W, |u_t| = sqrt(gamma_t^2 - 1),
// e1 along the cluster momentum P (x if P = 0), cos t = |P| / (W |u_t|), e2 the
// axis least aligned with e1 made orthogonal to it.  Weight, momentum, kinetic
// energy and the first moment of the charge of every cell are kept; the pair
// takes the two smallest ids of its cluster.  A patch then holds its untouched
// particles in slot order followed by the pairs in (cell, cluster) order.
//
// One workgroup per patch.  The members of every crowded cell are copied,
// in slot order, into a contiguous run of the staging arrays (free outside
// the re-binning), with their slots listed in the vacated-slot list; the
// clustering of a cell runs on one thread in FP64 over that contiguous run in
// the same order of operations as a plain sequential loop (no contraction into
// fused multiply-adds); the untouched particles are then compacted in place
// (in slot order) and the pairs written after them.  The pass runs between the
// re-binning and the step close, before a window jump.

#include <hip/hip_runtime.h>

#include "kernels.h"
#include "pic_dev.h"

namespace pic {
namespace {

constexpr int kMB = 256;          // threads per workgroup
constexpr int kMaxCells = 4096;   // cells per patch (64 x 64)
constexpr int kKMax = 16;         // clusters per cell (cmax <= 32)
// The kernel is built for at most KMAX = 4, 8 or 16 clusters (the smallest
// that holds cmax / 2): a cell's centroids and sums live in registers, and
// fewer of them leave room for more waves per SIMD (cmax 8: 4 clusters).
constexpr uint8_t kKeep = 0xFF;   // a particle that stays as it is
constexpr int kAsgLDS = 32768;    // members whose clusters are also kept in LDS (per patch)

// Exclusive prefix sum of a[0..n) in place (n <= kMaxCells); returns the total.
__device__ int block_scan(int *a, int n, int *s_w)
{
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int per = (n + kMB - 1) / kMB;
    int loc = 0;
    for (int r = 0; r < per; ++r) {
        const int i = tid * per + r;
        if (i < n) loc += a[i];
    }
    int inc = loc;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const int v = __shfl_up(inc, o, 64);
        if (lane >= o) inc += v;
    }
    if (lane == 63) s_w[wave] = inc;
    __syncthreads();
    int before = inc - loc;
    for (int w = 0; w < wave; ++w) before += s_w[w];
    const int total = s_w[0] + s_w[1] + s_w[2] + s_w[3];
    for (int r = 0; r < per; ++r) {
        const int i = tid * per + r;
        if (i < n) {
            const int v = a[i];
            a[i] = before;
            before += v;
        }
    }
    __syncthreads();
    return total;
}

// Weighted Lloyd clustering of one cell's members: their data at staging
// slots lst .. lst + n (member order), their own slots in mem[0..n) (relative
// to the patch segment).  Each round assigns a member and adds it to its
// cluster's sums in one pass (the sums of a cluster still grow in member
// order), centroids and sums in registers (k <= KMAX); the final round's
// cluster of every member goes to code[] at its own slot.
template <typename T, int KMAX>
__device__ void cluster_cell(const SimDev<T> &S, int64_t base, int64_t lst, const int32_t *mem, int n,
                             int k, int iters, uint8_t *asg)
{
#pragma clang fp contract(off)
    // staged members: momentum and weight at sM[4 (lst + i) + c]
    const gptr_t<const T> Mm = glb((const T *)S.smom) + 4 * lst;
    auto U0 = [&](int64_t i) { return Mm[4 * i]; };
    auto U1 = [&](int64_t i) { return Mm[4 * i + 1]; };
    auto U2 = [&](int64_t i) { return Mm[4 * i + 2]; };
    auto Wt = [&](int64_t i) { return Mm[4 * i + 3]; };
    double cx[KMAX], cy[KMAX], cz[KMAX];
#pragma unroll
    for (int j = 0; j < KMAX; ++j) {
        cx[j] = cy[j] = cz[j] = 0.0;
        if (j < k) {
            const int64_t q = (int64_t)j * n / k;
            cx[j] = (double)U0(q);
            cy[j] = (double)U1(q);
            cz[j] = (double)U2(q);
        }
    }
    for (int it = 0; it < iters; ++it) {
        double sw[KMAX], sx[KMAX], sy[KMAX], sz[KMAX];
#pragma unroll
        for (int j = 0; j < KMAX; ++j) sw[j] = sx[j] = sy[j] = sz[j] = 0.0;
        for (int i = 0; i < n; ++i) {
            const double ux = U0(i), uy = U1(i), uz = U2(i);
            const double w = Wt(i);
            int best = 0;
            double bd = 0.0;
#pragma unroll
            for (int j = 0; j < KMAX; ++j) {
                if (j < k) {
                    const double dx = ux - cx[j], dy = uy - cy[j], dz = uz - cz[j];
                    const double d2 = dx * dx + dy * dy + dz * dz;
                    if (j == 0 || d2 < bd) {
                        bd = d2;
                        best = j;
                    }
                }
            }
#pragma unroll
            for (int j = 0; j < KMAX; ++j)
                if (j == best) {
                    sw[j] += w;
                    sx[j] += w * ux;
                    sy[j] += w * uy;
                    sz[j] += w * uz;
                }
            if (it == iters - 1) {
                glb(S.code)[base + mem[i]] = (uint8_t)best;
                if (asg) asg[i] = (uint8_t)best;
            }
        }
#pragma unroll
        for (int j = 0; j < KMAX; ++j)
            if (j < k && sw[j] > 0.0) {
                cx[j] = sx[j] / sw[j];
                cy[j] = sy[j] / sw[j];
                cz[j] = sz[j] / sw[j];
            }
    }
}

// Cluster of member i: from LDS when the patch's members fit there, else from
// code[] at the member's slot.
template <typename T>
__device__ __forceinline__ int member_cluster(const SimDev<T> &S, int64_t base, const int32_t *mem,
                                              const uint8_t *asg, int i)
{
    return asg ? asg[i] : glb(S.code)[base + mem[i]];
}

// The conserving pair of cluster j, members' data at staging slots
// lst .. lst + n; written to the particle arrays at slots dst, dst + 1.
template <typename T>
__device__ void write_pair(const SimDev<T> &S, int64_t base, int64_t lst, const int32_t *mem,
                           const uint8_t *asg, int n, int j, int64_t dst)
{
#pragma clang fp contract(off)
    double W = 0.0, E = 0.0, P0 = 0.0, P1 = 0.0, P2 = 0.0, X0 = 0.0, X1 = 0.0;
    int64_t id0 = INT64_MAX, id1 = INT64_MAX;
    for (int i = 0; i < n; ++i) {
        if (member_cluster(S, base, mem, asg, i) != j) continue;
        const int64_t q = lst + i;
        const Vec4<T> mq = v4(S.smom)[q];
        const double w = mq.w;
        const double ux = mq.x, uy = mq.y, uz = mq.z;
        const double g = sqrt(1.0 + ux * ux + uy * uy + uz * uz);
        W += w;
        E += w * g;
        P0 += w * ux;
        P1 += w * uy;
        P2 += w * uz;
        const Vec2<T> xq = v2(S.spos)[q];
        X0 += w * (double)xq.x;
        X1 += w * (double)xq.y;
        const int64_t id = glb(S.sid)[q];
        if (id < id0) {
            id1 = id0;
            id0 = id;
        } else if (id < id1) {
            id1 = id;
        }
    }
    const double gt = E / W;
    const double ut = gt > 1.0 ? sqrt(gt * gt - 1.0) : 0.0;
    const double pn = sqrt(P0 * P0 + P1 * P1 + P2 * P2);
    double e1[3] = {1.0, 0.0, 0.0};
    if (pn > 0.0) {
        e1[0] = P0 / pn;
        e1[1] = P1 / pn;
        e1[2] = P2 / pn;
    }
    int ax = 0;
    for (int a = 1; a < 3; ++a)
        if (fabs(e1[a]) < fabs(e1[ax])) ax = a;
    double e2[3] = {0.0, 0.0, 0.0};
    e2[ax] = 1.0;
    const double dp = e1[ax];
    for (int a = 0; a < 3; ++a) e2[a] -= dp * e1[a];
    const double en = sqrt(e2[0] * e2[0] + e2[1] * e2[1] + e2[2] * e2[2]);
    for (int a = 0; a < 3; ++a) e2[a] /= en;
    double ct = ut > 0.0 ? pn / (W * ut) : 0.0;
    if (ct > 1.0) ct = 1.0;
    const double st = sqrt(1.0 - ct * ct);
    // the pair's weight can exceed every earlier weight: raise the bound
    // behind the fixed-point current scale
    raise_wmax(S, (double)(T)(0.5 * W));
    for (int h = 0; h < 2; ++h) {
        const int64_t t = dst + h;
        const double sg = h == 0 ? 1.0 : -1.0;
        T ua[3];
        for (int a = 0; a < 3; ++a) ua[a] = (T)(ut * (ct * e1[a] + sg * st * e2[a]));
        v4(S.mom)[t] = Vec4<T>{ua[0], ua[1], ua[2], (T)(0.5 * W)};
        v2(S.pos)[t] = Vec2<T>{(T)(X0 / W), (T)(X1 / W)};
        glb(S.id)[t] = h == 0 ? id0 : id1;
    }
}

template <typename T, int KMAX>
__global__ __launch_bounds__(kMB) void k_merge2d(const SimDev<T> *__restrict__ sp, int cmax, int iters,
                                                 int forced)
{
    __shared__ int s_cnt[kMaxCells];   // particles per cell
    __shared__ int s_pos[kMaxCells];   // start of the cell's member run (its end while it is built)
    __shared__ int s_out[kMaxCells];   // first pair output of the cell
    __shared__ uint8_t s_asg[kAsgLDS]; // final cluster of every member, in run order
    __shared__ int s_w[4];
    __shared__ int s_run;
    const SimDev<T> &S = *sp;
    const gptr_t<SimState> st = glb(S.st);
    if (!forced) {
        if (S.mevery <= 0) return;
        if (!st->active || !st->rebinned || (st->flags & kFlagPending)) return;
        if ((st->step + 1) % S.mevery != 0) return;
        cmax = S.mcmax;
        iters = S.miters;
    }
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    const int P0 = S.P[0], P1 = S.P[1], ncell = P0 * P1;
    const int k = min(cmax / 2, KMAX);  // (the host picks KMAX >= cmax / 2)
    int64_t taken = 0;
    for (int p = blockIdx.x; p < S.npatch; p += gridDim.x) {
        const int n = glb(S.count)[p];
        if (n <= cmax) continue;
        const int64_t base = glb(S.off)[p];
        auto cell_of = [&](int i) {
            const Vec2<T> xi = v2(S.pos)[base + i];
            int cx = (int)floor(xi.x), cy = (int)floor(xi.y);
            cx = min(max(cx, 0), P0 - 1);
            cy = min(max(cy, 0), P1 - 1);
            return cx + P0 * cy;
        };
        // ---- cell counts; every particle starts as kept ----
        for (int c = tid; c < ncell; c += kMB) s_cnt[c] = 0;
        __syncthreads();
        for (int i = tid; i < n; i += kMB) {
            atomicAdd(&s_cnt[cell_of(i)], 1);
            glb(S.code)[base + i] = kKeep;
        }
        __syncthreads();
        // member runs of the cells above the threshold, one after another
        for (int c = tid; c < ncell; c += kMB) s_pos[c] = s_cnt[c] > cmax ? s_cnt[c] : 0;
        __syncthreads();
        const int heavy = block_scan(s_pos, ncell, s_w);
        if (heavy == 0) continue;
        const bool in_lds = heavy <= kAsgLDS;
        // ---- member runs in slot order, one wave of 64 consecutive slots at a
        // time: lanes of one cell find each other with ballots, and the waves of
        // a chunk take their places in wave order ----
        const gptr_t<int32_t> mem = glb(S.holes) + base;
        for (int i0 = 0; i0 < n; i0 += kMB) {
            const int i = i0 + tid;
            const int c = i < n ? cell_of(i) : -1;
            const bool hv = c >= 0 && s_cnt[c] > cmax;
            // lanes of this wave in the same crowded cell
            uint64_t match = 0, todo = __ballot(hv);
            while (todo) {
                const int lead = __ffsll((unsigned long long)todo) - 1;
                const int cl = __shfl(c, lead, 64);
                const uint64_t m = __ballot(hv && c == cl);
                if (hv && c == cl) match = m;
                todo &= ~m;
            }
            const int rank = __popcll(match & lt), same = __popcll(match);
            for (int w = 0; w < kMB / 64; ++w) {
                if (wave == w && hv) {
                    const int at_ = s_pos[c] + rank;
                    mem[at_] = i;
                    const int64_t src = base + i, dst = base + at_;
                    v2(S.spos)[dst] = v2(S.pos)[src];
                    v4(S.smom)[dst] = v4(S.mom)[src];
                    glb(S.sid)[dst] = glb(S.id)[src];
                }
                __syncthreads();
                if (wave == w && hv && rank == 0) s_pos[c] += same;
                __syncthreads();
            }
        }
        // ---- clustering, one thread per crowded cell; the threads take the
        // cells one at a time from a counter, so that a few very crowded cells
        // do not leave one thread with all the work ----
        for (int c = tid; c < ncell; c += kMB) {
            if (s_cnt[c] > cmax) s_pos[c] -= s_cnt[c];  // back to the run's start
            s_out[c] = 0;
        }
        if (tid == 0) s_run = 0;
        __syncthreads();
        for (;;) {
            const int c = atomicAdd(&s_run, 1);
            if (c >= ncell) break;
            const int nc = s_cnt[c];
            int outs = 0;
            if (nc > cmax) {
                const int32_t *m = (const int32_t *)&mem[s_pos[c]];
                uint8_t *asg = in_lds ? &s_asg[s_pos[c]] : nullptr;
                cluster_cell<T, KMAX>(S, base, base + s_pos[c], m, nc, k, iters, asg);
                int size[KMAX];
                for (int j = 0; j < k; ++j) size[j] = 0;
                for (int i = 0; i < nc; ++i) {
                    const int cj = member_cluster(S, base, m, asg, i);
                    if (cj < k) size[cj]++;
                }
                for (int j = 0; j < k; ++j) outs += size[j] >= 3 ? 2 : 0;
                // members of clusters of one or two stay as they are
                for (int i = 0; i < nc; ++i) {
                    const int cj = member_cluster(S, base, m, asg, i);
                    if (cj < k && size[cj] < 3) glb(S.code)[base + m[i]] = kKeep;
                }
                s_out[c] = outs;
            }
        }
        __syncthreads();
        const int nout = block_scan(s_out, ncell, s_w);
        // ---- kept particles, in slot order, compacted in place: a chunk reads
        // its particles before any of them is written, and writes only below
        // the next chunk's first slot ----
        if (tid == 0) s_run = 0;
        __syncthreads();
        for (int i0 = 0; i0 < n; i0 += kMB) {
            const int i = i0 + tid;
            const bool kp = i < n && glb(S.code)[base + i] == kKeep;
            const uint64_t b = __ballot(kp);
            if (lane == 0) s_w[wave] = __popcll(b);
            Vec2<T> vx{T(0), T(0)};
            Vec4<T> vm{T(0), T(0), T(0), T(0)};
            int64_t vid = 0;
            if (kp) {
                const int64_t src = base + i;
                vx = v2(S.pos)[src];
                vm = v4(S.mom)[src];
                vid = glb(S.id)[src];
            }
            __syncthreads();
            if (kp) {
                int r = s_run + __popcll(b & lt);
                for (int w = 0; w < wave; ++w) r += s_w[w];
                const int64_t dst = base + r;
                v2(S.pos)[dst] = vx;
                v4(S.mom)[dst] = vm;
                glb(S.id)[dst] = vid;
            }
            __syncthreads();
            if (tid == 0) s_run += s_w[0] + s_w[1] + s_w[2] + s_w[3];
            __syncthreads();
        }
        const int nkeep = s_run;
        // ---- the pairs after them, in (cell, cluster) order (the members'
        // clusters stay in code[] at their old slots until every pair is out) ----
        for (int c = tid; c < ncell; c += kMB) {
            const int nc = s_cnt[c];
            if (nc <= cmax) continue;
            const int32_t *m = (const int32_t *)&mem[s_pos[c]];
            const uint8_t *asg = in_lds ? &s_asg[s_pos[c]] : nullptr;
            // (without the LDS copy, members of clusters of one or two read as
            // kKeep and are not counted: those clusters make no pair either way)
            int size[KMAX];
            for (int j = 0; j < k; ++j) size[j] = 0;
            for (int i = 0; i < nc; ++i) {
                const int cj = member_cluster(S, base, m, asg, i);
                if (cj < k) size[cj]++;
            }
            int64_t dst = base + nkeep + s_out[c];
            for (int j = 0; j < k; ++j) {
                if (size[j] < 3) continue;
                write_pair(S, base, base + s_pos[c], m, asg, nc, j, dst);
                dst += 2;
            }
        }
        __syncthreads();
        const int nn = nkeep + nout;
        for (int i = tid; i < nn; i += kMB) glb(S.code)[base + i] = (uint8_t)kStay2;
        if (tid == 0) {
            glb(S.count)[p] = nn;
            taken += n - nn;
        }
        __syncthreads();
    }
    if (tid == 0 && taken)
        __hip_atomic_fetch_add(&st->merged, taken, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

}  // namespace

template <typename T>
void launch_merge(const SimDev<T> *sim, int npatch, int cmax, int iters, int forced, int cmax_bound,
                  hipStream_t st)
{
    const dim3 grid(std::min(npatch, 2048)), block(kMB);
    if (cmax_bound / 2 <= 4)
        hipLaunchKernelGGL((k_merge2d<T, 4>), grid, block, 0, st, sim, cmax, iters, forced);
    else if (cmax_bound / 2 <= 8)
        hipLaunchKernelGGL((k_merge2d<T, 8>), grid, block, 0, st, sim, cmax, iters, forced);
    else
        hipLaunchKernelGGL((k_merge2d<T, kKMax>), grid, block, 0, st, sim, cmax, iters, forced);
}

template void launch_merge<float>(const SimDev<float> *, int, int, int, int, int, hipStream_t);
template void launch_merge<double>(const SimDev<double> *, int, int, int, int, int, hipStream_t);

}  // namespace pic
