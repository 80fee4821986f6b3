// Re-binning helpers: neighbour-table rows, particle copies and the
// per-patch leaver count of the re-binning kernels.
#pragma once

#include "pic_dev.h"

namespace pic {

// The neighbour table of a simulation (built once on the host from the patch
// grid) holds per patch: the canonical key of each of the ND directions (the
// smallest direction reaching the same neighbour; -1 when the neighbour is the
// patch itself, i.e. the particle stays; ND when it leaves an open face),
// then the number of distinct source patches, the sources in ascending id and
// the key under which each source stages the particles it sends here.  Key ND
// also stands for a removed particle.
template <int ND>
__device__ __forceinline__ gptr_t<const int32_t> nb_row(const int32_t *nbt, int p)
{
    return glb(nbt) + (int64_t)p * nb_stride(ND);
}

template <typename T>
__device__ __forceinline__ void copy_particle(const SimDev<T> &S, int64_t from, int64_t to,
                                              bool from_stage, bool to_stage)
{
    T *fP = from_stage ? S.spos : S.pos, *fM = from_stage ? S.smom : S.mom;
    T *tP = to_stage ? S.spos : S.pos, *tM = to_stage ? S.smom : S.mom;
    const int64_t *fi = from_stage ? S.sid : S.id;
    int64_t *ti = to_stage ? S.sid : S.id;
    v4(tM)[to] = v4(fM)[from];
    if (S.pw == 4) {
        v4(tP)[to] = v4(fP)[from];  // (with the id)
    } else {
        v2(tP)[to] = v2(fP)[from];
        glb(ti)[to] = glb(fi)[from];
    }
}

// Count pass.  Each wave of the workgroup owns a contiguous range of the
// patch's slots and loads the destination codes of up to kU x 64 of them at
// once (one batch; a patch of at most waves x kU x 64 particles is one batch).
// Leaver counts per key come from ballots, one per key present in a 64-slot
// chunk, and are kept lane-indexed in a register (lane k: key k, lane kKeys:
// all keys).  After one exchange of the per-wave counts through LDS every wave
// knows where its leavers go: the vacated slots are listed in slot order and
// the staged leavers are queued in a per-wave LDS ring, which is drained 64
// entries at a time (one lane per particle, so the particle loads of 64
// leavers are in flight together).
// threads of the count workgroup: 2-D, and 3-D one wave per patch (about a
// hundred leavers per 8^3 patch); measured beside the field update, smaller
// workgroups keep more patches in flight (2-D: 512 and 128 slower than 256)
constexpr int kRC = 256;
constexpr int kRC3 = 64;
constexpr int kU = 16;    // 64-slot chunks per batch of code loads (63 VGPRs: 8 waves per SIMD)
constexpr int kRing = 128;

template <typename T>
__device__ __forceinline__ void drain_ring(const SimDev<T> &S, int64_t base, const int2 *ring,
                                           int &head, int tail, int lane)
{
    // copy up to 64 queued leavers (ring positions head .. min(tail, head + 64))
    const int n = min(64, tail - head);
    if (lane < n) {
        const int2 e = ring[(head + lane) & (kRing - 1)];
        copy_particle(S, base + e.x, base + e.y, false, true);
    }
    head += n;
}

template <int ND, int NWV>
struct CountSmem {
    uint8_t kb[256];             // code -> key + 1 (0: the particle stays)
    int wc[NWV][ND + 3];         // per wave: leavers of each key, then of all keys
    int2 ring[NWV][kRing];       // per wave: (slot, staging slot) of queued leavers
};

// Leavers of patch p: per-key counts (kcnt, nleave), the vacated slots in
// ascending order (holes) and the staged copies of the leavers, grouped by
// destination key in slot order.  Called by every thread of a workgroup of
// NWV waves (contains barriers).  n and base are the patch's count and first
// slot, key (threads tid < ND) the canonical key of direction tid: the caller
// loads them together with its own checks, so that their latencies overlap,
// and the first codes are loaded before the key table is built.
template <typename T, int ND, int NWV>
__device__ __forceinline__ void count_patch(const SimDev<T> &S, int p, int n, int64_t base, int key,
                                            CountSmem<ND, NWV> &sm)
{
    constexpr int kKeys = ND + 1;  // ND direction keys + removed
    constexpr int kThreads = NWV * 64;
    // (NWV == 1: one wave per patch, synchronised by wave barriers only)
    const int tid = NWV == 1 ? (int)(threadIdx.x & 63) : (int)threadIdx.x;
    const int lane = threadIdx.x & 63, wave = NWV == 1 ? 0 : (int)(threadIdx.x >> 6);
    auto group_sync = [&]() {
        if constexpr (NWV == 1) __builtin_amdgcn_wave_barrier();
        else __syncthreads();
    };
    const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    const gptr_t<const uint8_t> code = glb((const uint8_t *)S.code) + base;
    const int per = ((n + kThreads - 1) / kThreads) * 64;
    const int lo = min(n, wave * per), hi = min(n, lo + per);
    const bool one = hi - lo <= 64 * kU;
    // codes of a batch, then keys + 1 of the batch, four 64-slot chunks per register
    uint8_t t[kU];
    uint32_t cw[kU / 4];
    auto fetch = [&](int q0) {
        const gptr_t<const uint8_t> cp = code + q0 + lane;
        const int left = hi - q0 - lane;  // chunk u holds a slot while 64 u < left
#pragma unroll
        for (int u = 0; u < kU; ++u) t[u] = 64 * u < left ? cp[64 * u] : uint8_t(ND / 2);
    };
    auto translate = [&]() {
#pragma unroll
        for (int u = 0; u < kU; u += 4)
            cw[u / 4] = (uint32_t)sm.kb[t[u]] | ((uint32_t)sm.kb[t[u + 1]] << 8) |
                        ((uint32_t)sm.kb[t[u + 2]] << 16) | ((uint32_t)sm.kb[t[u + 3]] << 24);
    };
    auto key1 = [&](int u) { return (int)((cw[u / 4] >> (8 * (u % 4))) & 0xffu); };
    fetch(lo);
    for (int e = tid; e < 256; e += kThreads) {
        int kb = 0;
        if (e < ND) kb = key + 1;  // e == tid here (ND < kThreads)
        else if (e == kRemoved) kb = ND + 1;
        sm.kb[e] = (uint8_t)kb;
    }
    group_sync();

    // ---- walk 1: leavers per key in [lo, hi) ------------------------------
    int cnt = 0;
    for (int q0 = lo; q0 < hi; q0 += 64 * kU) {
        if (q0 != lo) fetch(q0);
        translate();
#pragma unroll
        for (int u = 0; u < kU; ++u) {
            if (q0 + 64 * u >= hi) break;
            const int kc = key1(u);
            uint64_t m = __ballot(kc != 0);
            cnt += lane == kKeys ? __popcll(m) : 0;
            while (m) {
                const int kk = __builtin_amdgcn_readlane(kc, __ffsll((long long)m) - 1);
                const uint64_t b = __ballot(kc == kk);
                cnt += lane == kk - 1 ? __popcll(b) : 0;
                m &= ~b;
            }
        }
    }
    if (lane <= kKeys) sm.wc[wave][lane] = cnt;
    group_sync();

    // ---- starting points: lane k of wave w holds the staging slot of the
    // next key-k leaver of the wave (key offset + earlier waves), lane kKeys
    // the next hole index ---------------------------------------------------
    int run = 0;
    if (lane <= kKeys) {
        for (int w = 0; w < wave; ++w) run += sm.wc[w][lane];
        if (lane < kKeys)
            for (int kk = 0; kk < lane; ++kk)
                for (int w = 0; w < NWV; ++w) run += sm.wc[w][kk];
    }
    if (wave == 0 && lane <= kKeys) {
        int tot = 0;
        for (int w = 0; w < NWV; ++w) tot += sm.wc[w][lane];
        if (lane < ND) glb(S.kcnt)[p * ND + lane] = tot;
        if (lane < kKeys) glb(S.kofs)[p * kKeys + lane] = run;  // wave 0: the key's offset
        if (lane == kKeys) glb(S.nleave)[p] = tot;
    }

    // ---- walk 2: list holes, queue and copy staged leavers -----------------
    if (__builtin_amdgcn_readlane(cnt, kKeys) > 0) {
        int2 *ring = sm.ring[wave];
        int head = 0, tail = 0;
        for (int q0 = lo; q0 < hi; q0 += 64 * kU) {
            if (!one) {
                fetch(q0);
                translate();
            }
#pragma unroll
            for (int u = 0; u < kU; ++u) {
                if (q0 + 64 * u >= hi) break;
                const int kc = key1(u);
                const int k = q0 + 64 * u + lane;
                uint64_t m = __ballot(kc != 0);
                if (!m) continue;
                const int h0 = __builtin_amdgcn_readlane(run, kKeys);
                if (kc) glb(S.holes)[base + h0 + __popcll(m & lt)] = k;
                run += lane == kKeys ? __popcll(m) : 0;
                const uint64_t st = m & ~__ballot(kc == ND + 1);
                int dest = 0;
                while (m) {
                    const int kk = __builtin_amdgcn_readlane(kc, __ffsll((long long)m) - 1);
                    const uint64_t b = __ballot(kc == kk);
                    const int r0 = __builtin_amdgcn_readlane(run, kk - 1);
                    if (kc == kk) dest = r0 + __popcll(b & lt);
                    run += lane == kk - 1 ? __popcll(b) : 0;
                    m &= ~b;
                }
                if (st) {
                    if ((st >> lane) & 1)
                        ring[(tail + __popcll(st & lt)) & (kRing - 1)] = make_int2(k, dest);
                    tail += __popcll(st);
                    __builtin_amdgcn_wave_barrier();
                    if (tail - head >= 64) {
                        drain_ring(S, base, ring, head, tail, lane);
                        __builtin_amdgcn_wave_barrier();
                    }
                }
            }
        }
        while (head < tail) {
            drain_ring(S, base, ring, head, tail, lane);
            __builtin_amdgcn_wave_barrier();
        }
    }
    group_sync();
}

}  // namespace pic
