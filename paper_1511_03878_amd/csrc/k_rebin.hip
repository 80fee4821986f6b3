// Per-patch re-binning, work-queue build and small service kernels of the
// 2-D patch-PIC step.
//
// Re-binning keeps every patch's particles in slots 0..count-1 and moves only
// the particles that change patch, under a canonical rule that fixes every
// slot bit for bit: in patch P with n old slots, L leavers (sent elsewhere or
// removed) and A arrivals, the new count is n' = n - L + A; the leaver slots
// below n' (ascending) are filled first by the arrivals, ordered by (source
// patch id, source slot), then by the stayers found in [n', n) (ascending);
// what remains of the arrivals is appended from slot n on.  The paper's
// patches (section 3.1) move particles between patches every step; this rule
// is the deterministic in-patch order adopted for that exchange.
//
// Three passes:
//  count   (one workgroup per source patch): per destination key, stable
//          ranks of the leavers by wave ballots; leavers are copied to a
//          staging area grouped by destination; vacated slots are listed;
//  check   (one thread per patch): arrivals, new count, vacated slots below
//          it; a patch that would exceed its capacity raises the pending flag
//          and the scatter of that simulation is skipped (state stays valid:
//          the host grows capacities and re-runs the three passes);
//  scatter (one workgroup per destination patch): arrivals into holes / the
//          tail, tail stayers into the remaining holes, new count; the
//          workgroup of patch 0 closes the step (counter, energy history).
#include "kernels.h"
#include "rebin_common.h"

namespace pic {

namespace {

// threads of a scatter workgroup (one arrival per thread; measured faster
// than 256 beside the field update, in 2-D and 3-D)
constexpr int kRB = 128;

template <typename T, int ND, int NT>
__global__ __launch_bounds__(NT) void k_rebin_count(const SimDev<T> *__restrict__ sims, int nsims,
                                                    const int *__restrict__ patch_prefix, int total)
{
    __shared__ CountSmem<ND, NT / 64> sm;
    for (int gp = blockIdx.x; gp < total; gp += gridDim.x) {
        const int s = find_sim(patch_prefix, nsims, gp);
        const SimDev<T> &S = sims[s];
        const int p = gp - patch_prefix[s];
        // the state the patch's count needs, loaded together
        const uint32_t active = glb(S.st)->active;
        const int moved = *glb(S.moved + p);
        const int n = glb(S.count)[p];
        const int64_t base = glb(S.off)[p];
        const int key = threadIdx.x < ND ? nb_row<ND>(S.nbt, p)[threadIdx.x] : 0;
        if (!active) continue;
        if (!moved) {
            // no particle of the patch changed patch or was removed: no leavers
            if (threadIdx.x < ND) glb(S.kcnt)[p * ND + threadIdx.x] = 0;
            if (threadIdx.x <= ND) glb(S.kofs)[p * (ND + 1) + threadIdx.x] = 0;
            if (threadIdx.x == 0) glb(S.nleave)[p] = 0;
            continue;
        }
        count_patch<T, ND, NT / 64>(S, p, n, base, key, sm);
    }
}

template <typename T, int ND>
__global__ __launch_bounds__(256) void k_rebin_check(const SimDev<T> *__restrict__ sims, int nsims,
                                                     const int *__restrict__ patch_prefix, int total)
{
    const int gp = blockIdx.x * blockDim.x + threadIdx.x;
    if (gp >= total) return;
    const int s = find_sim(patch_prefix, nsims, gp);
    const SimDev<T> &S = sims[s];
    if (!glb(S.st)->active) return;
    const int q = gp - patch_prefix[s];
    const gptr_t<const int32_t> row = nb_row<ND>(S.nbt, q);
    const int ns = row[ND];
    int A = 0;
    for (int i = 0; i < ns; ++i) A += glb(S.kcnt)[row[ND + 1 + i] * ND + row[2 * ND + i]];
    const int n = glb(S.count)[q], L = glb(S.nleave)[q];
    const int np = n - L + A;
    // vacated slots below the new count (the list is ascending)
    const gptr_t<const int32_t> h = glb((const int32_t *)S.holes) + glb(S.off)[q];
    int lo = 0, hi = L;
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (h[mid] < np) lo = mid + 1; else hi = mid;
    }
    glb(S.newcount)[q] = np;
    glb(S.narrive)[q] = A;
    glb(S.nhole)[q] = lo;
    if (np > glb(S.cap)[q])
        __hip_atomic_fetch_or(&glb(S.st)->flags, kFlagPending, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

template <typename T, int ND, int NT>
__global__ __launch_bounds__(NT) void k_rebin_scatter(const SimDev<T> *__restrict__ sims, int nsims,
                                                       const int *__restrict__ patch_prefix,
                                                       int total)
{
    constexpr int NS = ND - 1;  // at most this many distinct source patches
    constexpr int kNW = NT / 64;
    static_assert(NT >= 64 + ND, "threads 64 .. 64 + ND hold the direction keys");
    __shared__ int s_scnt[NS];
    __shared__ int64_t s_sbase[NS];
    __shared__ int s_ns;
    __shared__ int s_key[ND];
    __shared__ int s_wc[kNW];
    __shared__ int s_run;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));

    for (int gp = blockIdx.x; gp < total; gp += gridDim.x) {
        const int s = find_sim(patch_prefix, nsims, gp);
        const SimDev<T> &S = sims[s];
        const int q = gp - patch_prefix[s];
        // everything that depends on q alone, loaded together: the state,
        // the patch's counts, and per thread one entry of its neighbour row
        // (threads below NS: a source and its key; threads 64 .. 64 + ND: a
        // direction's key)
        const uint32_t active = glb(S.st)->active, flags = glb(S.st)->flags;
        const int n = glb(S.count)[q], np = glb(S.newcount)[q], nH = glb(S.nhole)[q], A = glb(S.narrive)[q];
        const int L = glb(S.nleave)[q], nstaged = glb(S.kofs)[q * (ND + 1) + ND];
        const int64_t base = glb(S.off)[q];
        const gptr_t<const int32_t> row = nb_row<ND>(S.nbt, q);
        int r_ns = 0, r_a = 0, r_b = 0;
        if (tid < NS) {
            r_ns = row[ND];
            r_a = row[ND + 1 + tid];
            r_b = row[2 * ND + tid];
        } else if (tid >= 64 && tid < 64 + ND) {
            r_a = row[tid - 64];
        }
        if (!active || (flags & kFlagPending)) continue;
        if (A == 0 && np == n && L == 0) {
            // nothing arrives and nothing leaves
            if (tid == 0) {
                if (q == 0) glb(S.st)->rebinned = 1u;
                *glb(S.moved + q) = 0;
            }
            continue;
        }
        if (tid < NS) {
            // one thread per source: its count and staging base for this patch
            if (tid < r_ns) {
                const int sp = r_a, k = r_b;
                s_scnt[tid] = glb(S.kcnt)[sp * ND + k];
                s_sbase[tid] = glb(S.off)[sp] + glb(S.kofs)[sp * (ND + 1) + k];
            }
            if (tid == 0) {
                s_ns = r_ns;
                s_run = 0;
                if (q == 0) glb(S.st)->rebinned = 1u;
            }
        } else if (tid >= 64 && tid < 64 + ND) {
            s_key[tid - 64] = r_a;
        }
        __syncthreads();
        // arrivals (sources in ascending id, each in its slot order): holes
        // first, then appended from slot n; one thread per arrival, so the
        // copies of all sources are in flight together
        for (int a = tid; a < A; a += NT) {
            int i = 0, a0 = 0;
            while (i + 1 < s_ns && a >= a0 + s_scnt[i]) a0 += s_scnt[i++];
            const int target = a < nH ? glb(S.holes)[base + a] : n + (a - nH);
            copy_particle(S, s_sbase[i] + (a - a0), base + target, true, false);
        }
        // stayers in [n', n) fill the remaining holes
        if (np < n) {
            for (int c0 = np; c0 < n; c0 += NT) {
                const int k = c0 + tid;
                bool stay = false;
                if (k < n) {
                    const uint8_t c = glb(S.code)[base + k];
                    stay = c != kRemoved && s_key[c] < 0;
                }
                const uint64_t b = __ballot(stay);
                if (lane == 0) s_wc[wave] = __popcll(b);
                __syncthreads();
                if (stay) {
                    int r = s_run + __popcll(b & lt);
                    for (int w = 0; w < wave; ++w) r += s_wc[w];
                    copy_particle(S, base + k, base + glb(S.holes)[base + A + r], false, false);
                }
                __syncthreads();
                if (tid == 0) {
                    int add = 0;
                    for (int w = 0; w < kNW; ++w) add += s_wc[w];
                    s_run += add;
                }
                __syncthreads();
            }
        }
        if (tid == 0) {
            glb(S.count)[q] = np;
            *glb(S.moved + q) = 0;
            const int removed = L - nstaged;
            if (removed)
                __hip_atomic_fetch_add(&glb(S.st)->removed, (uint64_t)removed, __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_AGENT);
        }
        __syncthreads();
    }
}

// ---- step close and work queue --------------------------------------------------
//
// One workgroup.  Phase A closes the step of every simulation whose
// re-binning was applied (one wave per simulation: reduce the per-tile field
// energies and per-patch kinetic energies, write the history entry, advance
// the step counter and spend one step of its budget) and decides which
// simulations take part in the next step.  Phase B builds the work queue of
// that step: every patch is cut into chunks of at most `chunk` particles and
// the chunks are placed in order of decreasing size, so that persistent
// workgroups pulling from the queue start with the largest items (the
// single-GPU counterpart of evening out load by exchanging patches).
// Batches of more than kCntCache patches build the queue with two grid
// kernels instead (k_queue_hist, k_queue_place): one workgroup would walk
// their patch counts in many dependent rounds.

constexpr int kQB = 1024;   // threads of the single queue workgroup
constexpr int kQW = kQB / 64;
constexpr int kBuckets = 1024;
constexpr int kCntCache = 8192;
constexpr int kQS = 256;    // threads of a grid queue workgroup
static_assert(2 * kBuckets + kMaxBatch == kQueueScratch, "queue scratch layout");
static_assert(kBuckets % kQS == 0, "buckets per thread");

// bucket of a chunk of c particles (0: full chunks; larger chunks first)
__device__ __forceinline__ int chunk_bucket(int c, int chunk)
{
    return kBuckets - 1 - (int)(((int64_t)(c - 1) * kBuckets) / chunk);
}

// patch at queue position gp of simulation s (curve order when the
// simulation asks for it, else patch id order)
template <typename T>
__device__ __forceinline__ int queue_patch(const SimDev<T> *sims, const int *pp, int gp, int s)
{
    const int lp = gp - pp[s];
    const int32_t *po = sims[s].porder;
    return po ? (int)glb(po)[lp] : lp;
}

__device__ __forceinline__ int wave_incl_scan(int v, int lane)
{
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const int y = __shfl_up(v, o, 64);
        if (lane >= o) v += y;
    }
    return v;
}

template <typename T>
__global__ __launch_bounds__(kQB) void k_close_queue(const SimDev<T> *__restrict__ sims,
                                                     QueueArgs qa)
{
    __shared__ int s_hist[kBuckets];
    __shared__ uint8_t s_act[kMaxBatch];
    __shared__ uint8_t s_par[kMaxBatch];   // parity of the step the queue is for
    __shared__ int s_pushed[kMaxBatch];
    __shared__ int s_pp[kMaxBatch + 1];  // patch prefix of the batch
    __shared__ int s_cnt[kCntCache];     // particle counts at the first kCntCache queue positions
    __shared__ int s_off[kCntCache];     // and their first particle slots
    __shared__ int s_wsum[kQW];
    __shared__ double s_red[kQW][2];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    const int nsims = qa.nsims;

    // ---- phase A: close steps, decide participation -------------------------------
    // G waves work on one simulation (all 16 for a single simulation, one each
    // for batches of 16 or more); rounds cover the batch.
    int G = kQW;
    while (G > 1 && G * nsims > kQW) G >>= 1;
    const int per_round = kQW / G;
    const int sub = wave % G;
    for (int r0 = 0; r0 < nsims; r0 += per_round) {
        const int s = r0 + wave / G;
        bool closing = false;
        int64_t left = 0;
        uint32_t flags = 0;
        if (s < nsims) {
            const SimDev<T> &S = sims[s];
            const gptr_t<SimState> st = glb(S.st);
            flags = st->flags;
            left = st->steps_left;
            closing = st->active && st->rebinned && !(flags & kFlagPending);
            double u = 0.0, k = 0.0;
            if (closing) {
                const int nt = qa.tile_prefix[s + 1] - qa.tile_prefix[s];
                const gptr_t<const double> up = glb((const double *)S.upart);
                const gptr_t<double> kp = glb(S.kpart);
#pragma unroll 8
                for (int i = sub * 64 + lane; i < nt; i += G * 64) u += up[i];
#pragma unroll 8
                for (int i = sub * 64 + lane; i < S.npatch; i += G * 64) {
                    k += kp[i];
                    kp[i] = 0.0;
                }
#pragma unroll
                for (int o = 32; o > 0; o >>= 1) {
                    u += __shfl_xor(u, o, 64);
                    k += __shfl_xor(k, o, 64);
                }
            }
            if (lane == 0) { s_red[wave][0] = u; s_red[wave][1] = k; }
        }
        __syncthreads();
        if (s < nsims && sub == 0 && lane == 0) {
            const SimDev<T> &S = sims[s];
            const gptr_t<SimState> st = glb(S.st);
            if (closing) {
                double u = 0.0, k = 0.0;
                for (int w = wave; w < wave + G; ++w) { u += s_red[w][0]; k += s_red[w][1]; }
                if (left > 0) left -= 1;
                const int64_t n = st->step;
                gptr_t<double> h = glb(S.hist) + (n % kHistLen) * 4;
                h[0] = u;
                h[1] = k;
                h[2] = (double)st->pushed;
                h[3] = (double)st->removed;
                st->U = u;
                st->K = k;
                if (st->wpend) {
                    // the window jumped at the end of this step
                    st->next_id += st->wadd;
                    st->wshift += 1;
                    st->wadd = 0;
                    st->wpend = 0u;
                }
                st->step = n + 1;
                st->steps_left = left;
                st->rebinned = 0u;
            }
            const uint32_t act = left > 0 && !(flags & (kFlagPending | kFlagErrMask));
            st->active = act;
            s_act[s] = (uint8_t)act;
            s_par[s] = (uint8_t)(st->step & 1);
            s_pushed[s] = 0;
        }
        __syncthreads();
    }
    if (qa.total_patches > kCntCache) {
        // the grid kernels build the queue: clear their bucket counts and
        // cursors and the pushed counters they add to, and hand them each
        // simulation's participation and step parity
        const gptr_t<int> sc = glb(qa.scratch);
        for (int b = tid; b < 2 * kBuckets; b += kQB) sc[b] = 0;
        for (int s = tid; s < nsims; s += kQB) {
            sc[2 * kBuckets + s] = s_act[s] | (int)s_par[s] << 1;
            if (s_act[s]) glb(sims[s].st)->pushed = 0;
        }
        return;
    }
    for (int b = tid; b < kBuckets; b += kQB) s_hist[b] = 0;
    for (int i = tid; i <= nsims; i += kQB) s_pp[i] = qa.patch_prefix[i];
    __syncthreads();

    auto patch_at = [&](int gp, int s) { return queue_patch(sims, s_pp, gp, s); };
    // ---- particle counts of the first kCntCache patches, loaded together ----------
    const int total = s_pp[nsims];
    const int ncache = min(total, kCntCache);
    for (int g0 = 0; g0 < ncache; g0 += 8 * kQB) {
        int v[8], o[8];
#pragma unroll
        for (int r = 0; r < 8; ++r) {
            const int gp = g0 + r * kQB + tid;
            v[r] = 0;
            o[r] = 0;
            if (gp < ncache) {
                const int s = find_sim(s_pp, nsims, gp);
                if (s_act[s]) {
                    const int p = patch_at(gp, s);
                    v[r] = glb((const int32_t *)sims[s].count)[p];
                    o[r] = (int)glb((const int64_t *)sims[s].off)[p];
                }
            }
        }
#pragma unroll
        for (int r = 0; r < 8; ++r) {
            const int gp = g0 + r * kQB + tid;
            if (gp < ncache) {
                s_cnt[gp] = v[r];
                s_off[gp] = o[r];
            }
        }
    }
    __syncthreads();
    auto count_of = [&](int gp, int s) {
        if (gp < kCntCache) return s_cnt[gp];
        return s_act[s] ? glb((const int32_t *)sims[s].count)[patch_at(gp, s)] : 0;
    };

    // ---- phase B: chunk histogram (bucket 0 = largest chunks) ------------------------
    // A patch of n particles gives n / chunk full chunks (bucket 0) and one
    // partial chunk.  Full chunks of a wave are counted with one LDS atomic
    // (wave sum) and placed by a wave prefix sum; a partial chunk takes one
    // LDS atomic on its own bucket.  Items of one bucket land in arbitrary
    // order.
    const int chunk = qa.chunk;
    auto bucket = [&](int c) { return chunk_bucket(c, chunk); };
    for (int g0 = 0; g0 < total; g0 += kQB) {
        const int gp = g0 + tid;
        int s = 0, n = 0;
        if (gp < total) {
            s = find_sim(s_pp, nsims, gp);
            n = count_of(gp, s);
        }
        // pushed particles per simulation: one LDS atomic per simulation per wave
        uint64_t todo = __ballot(n > 0);
        while (todo) {
            const int sl = __shfl(s, __ffsll((unsigned long long)todo) - 1, 64);
            const uint64_t same = __ballot(n > 0 && s == sl);
            int v = (n > 0 && s == sl) ? n : 0;
#pragma unroll
            for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
            if (lane == 0) atomicAdd(&s_pushed[sl], v);
            todo &= ~same;
        }
        const int nfull = n / chunk, rem = n - nfull * chunk;
        const int fsum = __shfl(wave_incl_scan(nfull, lane), 63, 64);
        if (lane == 0 && fsum) atomicAdd(&s_hist[0], fsum);
        if (rem) atomicAdd(&s_hist[bucket(rem)], 1);
    }
    __syncthreads();
    for (int s = tid; s < nsims; s += kQB)
        if (s_act[s]) glb(sims[s].st)->pushed = s_pushed[s];
    // exclusive scan of the histogram (one bucket per thread)
    const int v = s_hist[tid];
    int incl = wave_incl_scan(v, lane);
    if (lane == 63) s_wsum[wave] = incl;
    __syncthreads();
    int woff = 0;
    for (int w = 0; w < wave; ++w) woff += s_wsum[w];
    int ntot = 0;
    for (int w = 0; w < kQW; ++w) ntot += s_wsum[w];
    __syncthreads();
    s_hist[tid] = woff + incl - v;
    __syncthreads();
    // ---- phase B: placement ------------------------------------------------------
    const gptr_t<int> items = glb(reinterpret_cast<int *>(qa.items));
    // item = {simulation | step parity << 30, patch, first slot, count}: the
    // particle kernel starts on it without reading the simulation's state
    auto put = [&](int pos, int s, int p, int64_t slot, int c) {
        if (pos >= qa.max_items) return;
        const gptr_t<int> it = items + 4 * (int64_t)pos;
        it[0] = s | ((int)s_par[s] << 30);
        it[1] = p;
        it[2] = (int)slot;
        it[3] = c;
    };
    for (int g0 = 0; g0 < total; g0 += kQB) {
        const int gp = g0 + tid;
        int s = 0, p = 0, n = 0;
        if (gp < total) {
            s = find_sim(s_pp, nsims, gp);
            p = patch_at(gp, s);
            n = count_of(gp, s);
        }
        const int nfull = n / chunk, rem = n - nfull * chunk;
        const int incl_f = wave_incl_scan(nfull, lane);
        const int fsum = __shfl(incl_f, 63, 64);
        int fbase = 0;
        if (lane == 0 && fsum) fbase = atomicAdd(&s_hist[0], fsum);
        fbase = __shfl(fbase, 0, 64) + incl_f - nfull;
        const int64_t o = n == 0 ? 0 : gp < kCntCache ? s_off[gp] : glb((const int64_t *)sims[s].off)[p];
        for (int k = 0; k < nfull; ++k) put(fbase + k, s, p, o + (int64_t)k * chunk, chunk);
        if (rem) put(atomicAdd(&s_hist[bucket(rem)], 1), s, p, o + (int64_t)nfull * chunk, rem);
    }
    if (tid == 0) {
        *glb(qa.nitems) = min(ntot, qa.max_items);
        *glb(qa.head) = 0;
    }
}

// ---- grid-wide queue build (batches of more than kCntCache patches) -------------
//
// k_queue_hist: each workgroup counts the chunks of its patches per bucket
// and the particles pushed per simulation in LDS, then adds its nonzero
// counts to the global ones (one atomic per bucket or simulation).
// k_queue_place: every workgroup scans the global bucket counts itself, then,
// round by round, ranks its chunks per bucket in LDS, takes one run of places
// per nonzero bucket from a global cursor and writes its items there.  Items
// of one bucket land in arbitrary order, as in the one-workgroup build.

template <typename T>
__global__ __launch_bounds__(kQS) void k_queue_hist(const SimDev<T> *__restrict__ sims, QueueArgs qa)
{
    __shared__ int s_hist[kBuckets];
    __shared__ int s_pp[kMaxBatch + 1];
    __shared__ uint8_t s_act[kMaxBatch];
    __shared__ unsigned long long s_pushed[kMaxBatch];
    const int tid = threadIdx.x, lane = tid & 63;
    const int nsims = qa.nsims, chunk = qa.chunk;
    const gptr_t<int> sc = glb(qa.scratch);
    for (int b = tid; b < kBuckets; b += kQS) s_hist[b] = 0;
    for (int i = tid; i <= nsims; i += kQS) s_pp[i] = qa.patch_prefix[i];
    for (int s = tid; s < nsims; s += kQS) {
        s_act[s] = (uint8_t)(sc[2 * kBuckets + s] & 1);
        s_pushed[s] = 0;
    }
    __syncthreads();
    const int total = s_pp[nsims];
    for (int g0 = blockIdx.x * kQS; g0 < total; g0 += gridDim.x * kQS) {
        const int gp = g0 + tid;
        int s = 0, n = 0;
        if (gp < total) {
            s = find_sim(s_pp, nsims, gp);
            if (s_act[s]) n = glb((const int32_t *)sims[s].count)[queue_patch(sims, s_pp, gp, s)];
        }
        uint64_t todo = __ballot(n > 0);
        while (todo) {
            const int sl = __shfl(s, __ffsll((unsigned long long)todo) - 1, 64);
            const uint64_t same = __ballot(n > 0 && s == sl);
            long long v = (n > 0 && s == sl) ? n : 0;
#pragma unroll
            for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
            if (lane == 0) atomicAdd(&s_pushed[sl], (unsigned long long)v);
            todo &= ~same;
        }
        const int nfull = n / chunk, rem = n - nfull * chunk;
        const int fsum = __shfl(wave_incl_scan(nfull, lane), 63, 64);
        if (lane == 0 && fsum) atomicAdd(&s_hist[0], fsum);
        if (rem) atomicAdd(&s_hist[chunk_bucket(rem, chunk)], 1);
    }
    __syncthreads();
    for (int b = tid; b < kBuckets; b += kQS)
        if (s_hist[b]) __hip_atomic_fetch_add(&sc[b], s_hist[b], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    for (int s = tid; s < nsims; s += kQS)
        if (s_pushed[s])
            __hip_atomic_fetch_add(&glb(sims[s].st)->pushed, (int64_t)s_pushed[s], __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_AGENT);
}

template <typename T>
__global__ __launch_bounds__(kQS) void k_queue_place(const SimDev<T> *__restrict__ sims, QueueArgs qa)
{
    constexpr int kPer = kBuckets / kQS;
    __shared__ int s_scan[kBuckets];  // first place of each bucket
    __shared__ int s_cnt[kBuckets];   // this round's chunks per bucket
    __shared__ int s_base[kBuckets];  // this round's first place in each bucket
    __shared__ int s_pp[kMaxBatch + 1];
    __shared__ uint8_t s_flag[kMaxBatch];
    __shared__ int s_wsum[kQS / 64];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int nsims = qa.nsims, chunk = qa.chunk;
    const gptr_t<int> sc = glb(qa.scratch);
    // exclusive scan of the bucket counts: kPer consecutive buckets per thread
    int v[kPer], sum = 0;
#pragma unroll
    for (int r = 0; r < kPer; ++r) {
        v[r] = sc[tid * kPer + r];
        sum += v[r];
    }
    for (int i = tid; i <= nsims; i += kQS) s_pp[i] = qa.patch_prefix[i];
    for (int s = tid; s < nsims; s += kQS) s_flag[s] = (uint8_t)sc[2 * kBuckets + s];
    const int incl = wave_incl_scan(sum, lane);
    if (lane == 63) s_wsum[wave] = incl;
    __syncthreads();
    int run = incl - sum, ntot = 0;
    for (int w = 0; w < kQS / 64; ++w) {
        if (w < wave) run += s_wsum[w];
        ntot += s_wsum[w];
    }
#pragma unroll
    for (int r = 0; r < kPer; ++r) {
        s_scan[tid * kPer + r] = run;
        s_cnt[tid * kPer + r] = 0;
        run += v[r];
    }
    __syncthreads();
    const gptr_t<int> items = glb(reinterpret_cast<int *>(qa.items));
    auto put = [&](int pos, int s, int p, int64_t slot, int c) {
        if (pos >= qa.max_items) return;
        const gptr_t<int> it = items + 4 * (int64_t)pos;
        it[0] = s | ((int)(s_flag[s] >> 1) << 30);
        it[1] = p;
        it[2] = (int)slot;
        it[3] = c;
    };
    const int total = s_pp[nsims];
    for (int g0 = blockIdx.x * kQS; g0 < total; g0 += gridDim.x * kQS) {
        const int gp = g0 + tid;
        int s = 0, p = 0, n = 0;
        int64_t o = 0;
        if (gp < total) {
            s = find_sim(s_pp, nsims, gp);
            if (s_flag[s] & 1) {
                p = queue_patch(sims, s_pp, gp, s);
                n = glb((const int32_t *)sims[s].count)[p];
                o = glb((const int64_t *)sims[s].off)[p];
            }
        }
        // ranks inside this round: full chunks by a wave scan, partial ones
        // by an LDS atomic on their bucket
        const int nfull = n / chunk, rem = n - nfull * chunk;
        const int incl_f = wave_incl_scan(nfull, lane);
        const int fsum = __shfl(incl_f, 63, 64);
        int fr = 0;
        if (lane == 0 && fsum) fr = atomicAdd(&s_cnt[0], fsum);
        fr = __shfl(fr, 0, 64) + incl_f - nfull;
        const int b = rem ? chunk_bucket(rem, chunk) : 0;
        const int rr = rem ? atomicAdd(&s_cnt[b], 1) : 0;
        __syncthreads();
        for (int k = tid; k < kBuckets; k += kQS) {
            const int c = s_cnt[k];
            s_base[k] = c ? __hip_atomic_fetch_add(&sc[kBuckets + k], c, __ATOMIC_RELAXED,
                                                   __HIP_MEMORY_SCOPE_AGENT)
                          : 0;
            s_cnt[k] = 0;
        }
        __syncthreads();
        const int fb = s_scan[0] + s_base[0] + fr;
        for (int k = 0; k < nfull; ++k) put(fb + k, s, p, o + (int64_t)k * chunk, chunk);
        if (rem) put(s_scan[b] + s_base[b] + rr, s, p, o + (int64_t)nfull * chunk, rem);
    }
    if (blockIdx.x == 0 && tid == 0) {
        *glb(qa.nitems) = min(ntot, qa.max_items);
        *glb(qa.head) = 0;
    }
}

// ---- capacity growth ------------------------------------------------------------

template <typename T>
__global__ void k_relayout(const SimDev<T> *__restrict__ src, const SimDev<T> *__restrict__ dst)
{
    const int p = blockIdx.x;
    const int n = src->count[p];
    const int64_t a = src->off[p], b = dst->off[p];
    for (int k = threadIdx.x; k < n; k += blockDim.x) {
        v4(dst->mom)[b + k] = v4(src->mom)[a + k];
        if (src->pw == 4) {
            v4(dst->pos)[b + k] = v4(src->pos)[a + k];  // (with the id)
        } else {
            v2(dst->pos)[b + k] = v2(src->pos)[a + k];
            dst->id[b + k] = src->id[a + k];
        }
        dst->code[b + k] = src->code[a + k];
    }
}

// ---- diagnostics ------------------------------------------------------------------

__global__ void k_scatter_codes(const uint8_t *__restrict__ packed,
                                const int64_t *__restrict__ packed_off,
                                const int64_t *__restrict__ off, const int32_t *__restrict__ count,
                                uint8_t *__restrict__ code)
{
    const int p = blockIdx.x;
    const int n = count[p];
    for (int k = threadIdx.x; k < n; k += blockDim.x) code[off[p] + k] = packed[packed_off[p] + k];
}

}  // namespace

template <typename T>
void launch_close_queue(const SimDev<T> *sims, const QueueArgs &q, hipStream_t st, Ev2 ev)
{
    if (q.total_patches <= kCntCache) {
        hipExtLaunchKernelGGL((k_close_queue<T>), dim3(1), dim3(kQB), 0, st, ev.start, ev.stop, 0, sims,
                              q);
        return;
    }
    const int grid = std::min((q.total_patches + kQS - 1) / kQS, 1024);
    hipExtLaunchKernelGGL((k_close_queue<T>), dim3(1), dim3(kQB), 0, st, ev.start, nullptr, 0, sims, q);
    hipLaunchKernelGGL((k_queue_hist<T>), dim3(grid), dim3(kQS), 0, st, sims, q);
    hipExtLaunchKernelGGL((k_queue_place<T>), dim3(grid), dim3(kQS), 0, st, nullptr, ev.stop, 0, sims, q);
}

template <typename T, int ND>
static void launch_rebin_nd(const SimDev<T> *sims, int nsims, const int *patch_prefix,
                            int total_patches, int grid, hipStream_t st, Ev2 ev)
{
    // one count workgroup per patch (the hardware balances uneven patches)
    constexpr int NT = ND == kNDir3 ? kRC3 : kRC;
    hipExtLaunchKernelGGL((k_rebin_count<T, ND, NT>), dim3(std::min(total_patches, 1 << 20)), dim3(NT),
                          0, st, ev.start, nullptr, 0, sims, nsims, patch_prefix, total_patches);
    hipLaunchKernelGGL((k_rebin_check<T, ND>), dim3((total_patches + 255) / 256), dim3(256), 0, st,
                       sims, nsims, patch_prefix, total_patches);
    hipExtLaunchKernelGGL((k_rebin_scatter<T, ND, kRB>), dim3(grid), dim3(kRB), 0, st, nullptr, ev.stop, 0,
                          sims, nsims, patch_prefix, total_patches);
}

template <typename T>
void launch_rebin(const SimDev<T> *sims, int nsims, const int *patch_prefix, int total_patches,
                  int grid, int ndim, hipStream_t st, Ev2 ev)
{
    if (ndim == 3)
        launch_rebin_nd<T, kNDir3>(sims, nsims, patch_prefix, total_patches, grid, st, ev);
    else
        launch_rebin_nd<T, kNDir2>(sims, nsims, patch_prefix, total_patches, grid, st, ev);
}

template <typename T>
void launch_relayout(const SimDev<T> *src, const SimDev<T> *dst, int npatch, hipStream_t st)
{
    hipLaunchKernelGGL((k_relayout<T>), dim3(npatch), dim3(256), 0, st, src, dst);
}

void launch_scatter_codes(const uint8_t *packed, const int64_t *packed_off, const int64_t *off,
                          const int32_t *count, uint8_t *code, int npatch, hipStream_t st)
{
    hipLaunchKernelGGL(k_scatter_codes, dim3(npatch), dim3(256), 0, st, packed, packed_off, off,
                       count, code);
}

#define PIC_INST(T)                                                                              \
    template void launch_close_queue<T>(const SimDev<T> *, const QueueArgs &, hipStream_t, Ev2); \
    template void launch_rebin<T>(const SimDev<T> *, int, const int *, int, int, int,            \
                                  hipStream_t, Ev2);                                             \
    template void launch_relayout<T>(const SimDev<T> *, const SimDev<T> *, int, hipStream_t);
PIC_INST(float)
PIC_INST(double)
#undef PIC_INST

}  // namespace pic
