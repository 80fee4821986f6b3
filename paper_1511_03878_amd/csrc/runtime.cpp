// Host runtime of the patch-PIC library: simulation and batch objects, device
// memory through the allocator hook, step orchestration on a HIP stream, and
// capacity growth when a patch overflows.  Exposed through the C ABI in
// capi.cpp.
#include "runtime.h"

#include <chrono>
#include <cstdio>
#include <cstdlib>
#include <fstream>

#include <algorithm>
#include <memory>
#include <climits>
#include <limits>
#include <cmath>
#include <cstring>
#include <numeric>

namespace pic {

thread_local std::string g_last_error;

void set_error(const std::string &m) { g_last_error = m; }

// ---------------------------------------------------------------------------
// device memory

void *Allocator::get(size_t bytes)
{
    if (bytes == 0) bytes = 256;
    bytes = (bytes + 255) & ~size_t(255);
    void *p = nullptr;
    if (hook.alloc) {
        p = hook.alloc(bytes, hook.ctx);
    } else if (hipMalloc(&p, bytes) != hipSuccess) {
        (void)hipGetLastError();
        p = nullptr;
    }
    if (!p) throw Error(PIC_ENOMEM, "device allocation of " + std::to_string(bytes) + " bytes failed");
    live_bytes += bytes;
    sizes[p] = bytes;
    return p;
}

void Allocator::put(void *p)
{
    if (!p) return;
    auto it = sizes.find(p);
    if (it != sizes.end()) {
        live_bytes -= it->second;
        sizes.erase(it);
    }
    if (hook.free) hook.free(p, hook.ctx);
    else (void)hipFree(p);
}

void hipcheck(hipError_t e, const char *what)
{
    if (e != hipSuccess) {
        (void)hipGetLastError();
        throw Error(PIC_EHIP, std::string(what) + ": " + hipGetErrorString(e));
    }
}

static int cu_count()
{
    static int cached = 0;
    if (!cached) {
        int dev = 0, n = 0;
        hipcheck(hipGetDevice(&dev), "hipGetDevice");
        hipcheck(hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev),
                 "hipDeviceGetAttribute");
        cached = n > 0 ? n : 1;
    }
    return cached;
}

// ---------------------------------------------------------------------------
// descriptor validation (host only, before any device call)

int validate_desc(const PicSimDesc &d, std::string &why)
{
    if (d.ndim != 2 && d.ndim != 3) { why = "ndim must be 2 or 3"; return PIC_ENOTSUP; }
    if (d.precision != 32 && d.precision != 64) { why = "precision must be 32 or 64"; return PIC_EINVAL; }
    double inv2 = 0.0;
    for (int a = 0; a < d.ndim; ++a) {
        if (d.n[a] < 4 || d.patch[a] <= 0) { why = "at least 4 cells per axis and positive patch sizes"; return PIC_EINVAL; }
        if (d.patch[a] > kMaxPatch) { why = "patch size above 64 cells"; return PIC_EINVAL; }
        if (d.n[a] % d.patch[a]) { why = "patch size must divide the cell count"; return PIC_EINVAL; }
        if (!(d.d[a] > 0.0) || !std::isfinite(d.d[a])) { why = "cell sizes must be positive"; return PIC_EINVAL; }
        if (a > 0 && !d.periodic[a]) { why = "only the x axis may be open"; return PIC_EINVAL; }
        inv2 += 1.0 / (d.d[a] * d.d[a]);
    }
    if (d.ndim == 3) {
        for (int a = 0; a < 3; ++a)
            if (!d.periodic[a]) { why = "3-D boxes must be periodic on every axis"; return PIC_ENOTSUP; }
        // the particle kernel holds the patch's field and current tiles in LDS
        if (particles3d_lds_bytes(d.precision, d.patch[0], d.patch[1], d.patch[2]) > 150 * 1024) {
            why = "3-D patch too large for the LDS tiles (8 x 8 x 8 cells fit)";
            return PIC_ENOTSUP;
        }
    }
    const int64_t cells = (int64_t)d.n[0] * d.n[1] * (d.ndim == 3 ? d.n[2] : 1);
    if (cells > (int64_t)1 << 30) { why = "grid too large"; return PIC_EINVAL; }
    if (!(d.dt > 0.0) || d.dt >= 1.0 / std::sqrt(inv2)) { why = "dt must be positive and below the Yee limit"; return PIC_EINVAL; }
    if (!(d.m > 0.0) || !std::isfinite(d.q)) { why = "species mass must be positive"; return PIC_EINVAL; }
    if (d.capacity_factor != 0.0 && !(d.capacity_factor >= 1.0)) { why = "capacity_factor must be >= 1"; return PIC_EINVAL; }
    if (d.min_capacity < 0 || d.chunk < 0) { why = "negative min_capacity or chunk"; return PIC_EINVAL; }
    // the fixed-point current tile of one item sums at most chunk contributions below 2^48
    if (d.chunk > 16384) { why = "chunk must be at most 16384"; return PIC_EINVAL; }
    if (d.deterministic != 0 && d.deterministic != 1) { why = "deterministic must be 0 or 1"; return PIC_EINVAL; }
    if (d.field_tile < 0 || d.field_tile > 5) { why = "field_tile must be 0..5"; return PIC_EINVAL; }
    if (d.lane_stride < 0 || d.lane_stride > 64) { why = "lane_stride must be 0..64"; return PIC_EINVAL; }
    if (d.block != 0 && d.block != 256 && d.block != 512 && d.block != 1024) { why = "block must be 0, 256, 512 or 1024"; return PIC_EINVAL; }
    if (d.graph != 0 && d.graph != 1) { why = "graph must be 0 or 1"; return PIC_EINVAL; }
    if (d.patch_order != 0 && d.patch_order != 1) { why = "patch_order must be 0 or 1"; return PIC_EINVAL; }
    if (d.maxwell_order != 0 && d.maxwell_order != 2 && d.maxwell_order != 6) {
        why = "maxwell_order must be 0, 2 or 6";
        return PIC_EINVAL;
    }
    if (d.maxwell_order == 6) {
        for (int a = 0; a < d.ndim; ++a)
            if (!d.periodic[a]) { why = "the sixth-order field solver needs every axis periodic"; return PIC_EINVAL; }
        // its largest modified wave number per axis is (2 / d) (75/64 + 25/384 + 3/640)
        const double S6 = 75.0 / 64.0 + 25.0 / 384.0 + 3.0 / 640.0;
        if (d.dt >= 1.0 / (S6 * std::sqrt(inv2))) { why = "dt above the sixth-order solver's stability limit"; return PIC_EINVAL; }
    }
    return PIC_OK;
}

// Particles between adjacent lanes of the particle kernels (unless the
// descriptor sets it).  2-D: 2, coalesced particle access outweighs fewer
// same-address LDS atomics (stride 8 measured 1.5x slower on the laser box).
// 3-D: 4, where each particle issues up to 144 window atomics and spreading
// a wave over more cells pays (8^3-cell patches of the blob box, 512-thread
// workgroups, two per CU: 22.55 ms per launch against 22.85 ms at stride 2).
static int default_lane_stride(int nd) { return nd == 3 ? 4 : 2; }

// ---------------------------------------------------------------------------
// SimImpl

template <typename T>
SimImpl<T>::SimImpl(const PicSimDesc &d, const PicAllocator *a, hipStream_t s)
{
    desc = d;
    if (desc.capacity_factor == 0.0) desc.capacity_factor = 3.0;
    precision = d.precision;
    stream = s;
    if (a) alloc.hook = *a;
    nd = d.ndim;
    ndir = nd == 3 ? kNDir3 : kNDir2;
    for (int ax = 0; ax < 3; ++ax) {
        n[ax] = ax < nd ? d.n[ax] : 1;
        P[ax] = ax < nd ? d.patch[ax] : 1;
        periodic[ax] = ax < nd ? (d.periodic[ax] ? 1 : 0) : 1;
        np[ax] = n[ax] / P[ax];
        fn[ax] = (ax < nd && !periodic[ax]) ? n[ax] + 1 : n[ax];
    }
    npatch = np[0] * np[1] * np[2];
    fsize = (int64_t)fn[0] * fn[1] * fn[2];
    std::memset(&v, 0, sizeof(v));
    try {
        for (int b = 0; b < 2; ++b)
            for (int c = 0; c < 6; ++c) F[b][c] = (T *)alloc.get(sizeof(T) * fsize);
        for (int b = 0; b < 2; ++b)
            for (int c = 0; c < 3; ++c) J[b][c] = (T *)alloc.get(sizeof(T) * fsize);
        if (desc.deterministic)
            for (int c = 0; c < 3; ++c) Jacc[c] = (int64_t *)alloc.get(sizeof(int64_t) * fsize);
        st = (SimState *)alloc.get(sizeof(SimState));
        hist = (double *)alloc.get(sizeof(double) * kHistLen * 4);
        counts_d = (int32_t *)alloc.get(sizeof(int32_t) * npatch);
        newcount_d = (int32_t *)alloc.get(sizeof(int32_t) * npatch);
        kcnt_d = (int32_t *)alloc.get(sizeof(int32_t) * npatch * ndir);
        kofs_d = (int32_t *)alloc.get(sizeof(int32_t) * npatch * (ndir + 1));
        nleave_d = (int32_t *)alloc.get(sizeof(int32_t) * npatch);
        narrive_d = (int32_t *)alloc.get(sizeof(int32_t) * npatch);
        nhole_d = (int32_t *)alloc.get(sizeof(int32_t) * npatch);
        moved_d = (int32_t *)alloc.get(sizeof(int32_t) * npatch);
        // every patch is scanned by the first re-binning
        hipcheck(hipMemsetAsync(moved_d, 1, sizeof(int32_t) * npatch, stream), "memset moved");
        if (desc.patch_order == 1) {
            const int npc[3] = {np[0], np[1], nd == 3 ? np[2] : 1};
            std::vector<int32_t> ord;
            std::string why;
            const int rc = hilbert_patch_order(nd, npc, ord, why);
            if (rc != PIC_OK) throw Error(PIC_EINVAL, "patch_order 1: " + why);
            porder_d = (int32_t *)alloc.get(sizeof(int32_t) * npatch);
            hipcheck(hipMemcpyAsync(porder_d, ord.data(), sizeof(int32_t) * npatch, hipMemcpyHostToDevice, stream), "order");
            hipcheck(hipStreamSynchronize(stream), "sync");
        }
        prefix_d = (int *)alloc.get(sizeof(int) * 2);
        tprefix_d = (int *)alloc.get(sizeof(int) * 2);
        view_d = (SimDev<T> *)alloc.get(sizeof(SimDev<T>));
        // per-tile energy partials, sized for the smallest Yee tile preset (16 x 4)
        // in 2-D and for blocks of nodes in 3-D
        max_tiles = nd == 3 ? std::max(maxwell3d_tiles(fn, 2), maxwell3d_tiles(fn, 6))
                            : (int64_t)((fn[0] + 15) / 16) * ((fn[1] + 3) / 4);
        upart = (double *)alloc.get(sizeof(double) * max_tiles);
        kpart = (double *)alloc.get(sizeof(double) * npatch);
        hipcheck(hipMemsetAsync(upart, 0, sizeof(double) * max_tiles, stream), "memset upart");
        hipcheck(hipMemsetAsync(kpart, 0, sizeof(double) * npatch, stream), "memset kpart");
        for (int b = 0; b < 2; ++b)
            for (int c = 0; c < 6; ++c)
                hipcheck(hipMemsetAsync(F[b][c], 0, sizeof(T) * fsize, stream), "memset F");
        for (int b = 0; b < 2; ++b)
            for (int c = 0; c < 3; ++c)
                hipcheck(hipMemsetAsync(J[b][c], 0, sizeof(T) * fsize, stream), "memset J");
        for (int c = 0; c < 3; ++c)
            if (Jacc[c]) hipcheck(hipMemsetAsync(Jacc[c], 0, sizeof(int64_t) * fsize, stream), "memset Jacc");
        hipcheck(hipMemsetAsync(st, 0, sizeof(SimState), stream), "memset state");
        hipcheck(hipMemsetAsync(hist, 0, sizeof(double) * kHistLen * 4, stream), "memset hist");
        hipcheck(hipMemsetAsync(counts_d, 0, sizeof(int32_t) * npatch, stream), "memset counts");
        int pre[2] = {0, npatch};
        hipcheck(hipMemcpyAsync(prefix_d, pre, sizeof(pre), hipMemcpyHostToDevice, stream), "prefix");
        build_neighbour_table();
        // an empty particle layout so that every kernel sees valid pointers
        std::vector<int32_t> cnt0(npatch, 0);
        layout_particles(cnt0);
        hipcheck(hipStreamSynchronize(stream), "create sync");
    } catch (...) {
        release();
        throw;
    }
}

template <typename T>
SimImpl<T>::~SimImpl()
{
    if (stream) (void)hipStreamSynchronize(stream);
    if (batch) {
        try { batch->remove(this); } catch (...) {}
    }
    delete solo;
    solo = nullptr;
    release();
}

template <typename T>
void SimImpl<T>::step(int64_t nsteps)
{
    check_free();
    if (nsteps < 0) throw Error(PIC_EINVAL, "negative step count");
    if (nsteps == 0) return;
    SimState s = read_state();
    if (s.flags & kFlagWin) throw Error(PIC_EOVERFLOW, "a window jump found a patch too small");
    if (s.flags & kFlagErrMask) throw Error((s.flags & kFlagNaN) ? PIC_ENAN : PIC_ECFL, "simulation stopped by a particle error");
    if (!solo) {
        solo = new BatchImpl<T>(stream);
        solo->solo_mode = true;
        solo->nd = nd;
        solo->members.push_back(this);
        solo->dirty = true;
    }
    s.steps_left = nsteps;
    hipcheck(hipMemcpy(&st->steps_left, &s.steps_left, sizeof(int64_t), hipMemcpyHostToDevice), "budget");
    if (solo->dirty) solo->build_tables();
    else solo->refresh_member_views();
    if (solo->dirty) solo->build_tables();
    solo->run(0, true);
}

// Patch topology used by the re-binning (static for a grid): per patch the
// canonical key of each direction, and the distinct source patches in
// ascending id with the key each of them stages its particles under.
template <typename T>
void SimImpl<T>::build_neighbour_table()
{
    // direction d = (dx + 1) + 3 (dy + 1) [+ 9 (dz + 1)]
    const int stay = ndir / 2, stride = nb_stride(ndir);
    auto nbr = [&](int p, int d) {
        int q[3] = {p % np[0], (p / np[0]) % np[1], p / (np[0] * np[1])};
        const int dd[3] = {d % 3 - 1, (d / 3) % 3 - 1, d / 9 - 1};
        for (int a = 0; a < nd; ++a) {
            q[a] += dd[a];
            if (q[a] < 0 || q[a] >= np[a]) {
                if (!periodic[a]) return -1;
                q[a] = (q[a] + np[a]) % np[a];
            }
        }
        return q[0] + np[0] * (q[1] + np[1] * q[2]);
    };
    auto key_of = [&](int p, int target) {
        for (int d = 0; d < ndir; ++d)
            if (d != stay && nbr(p, d) == target) return d;
        return -1;
    };
    std::vector<int32_t> t((size_t)npatch * stride, -1);
    std::vector<int> nb(ndir);
    for (int p = 0; p < npatch; ++p) {
        int32_t *row = &t[(size_t)p * stride];
        for (int d = 0; d < ndir; ++d) nb[d] = nbr(p, d);
        for (int d = 0; d < ndir; ++d) {
            if (d == stay || nb[d] == p) row[d] = -1;
            else if (nb[d] < 0) row[d] = ndir;
            else row[d] = key_of(p, nb[d]);
        }
        std::vector<int> src;
        for (int d = 0; d < ndir; ++d)
            if (d != stay && nb[d] >= 0 && nb[d] != p &&
                std::find(src.begin(), src.end(), nb[d]) == src.end())
                src.push_back(nb[d]);
        std::sort(src.begin(), src.end());
        row[ndir] = (int32_t)src.size();
        for (size_t i = 0; i < src.size(); ++i) {
            row[ndir + 1 + i] = src[i];
            row[2 * ndir + i] = key_of(src[i], p);
        }
    }
    nbt_d = (int32_t *)alloc.get(sizeof(int32_t) * t.size());
    hipcheck(hipMemcpyAsync(nbt_d, t.data(), sizeof(int32_t) * t.size(), hipMemcpyHostToDevice, stream), "neighbour table");
    hipcheck(hipStreamSynchronize(stream), "sync");
}

template <typename T>
void SimImpl<T>::free_particles()
{
    for (void *p : part_bufs) alloc.put(p);
    part_bufs.clear();
}

template <typename T>
void SimImpl<T>::release()
{
    free_particles();
    for (int b = 0; b < 2; ++b)
        for (int c = 0; c < 6; ++c) alloc.put(F[b][c]);
    for (int b = 0; b < 2; ++b)
        for (int c = 0; c < 3; ++c) alloc.put(J[b][c]);
    for (int c = 0; c < 3; ++c) {
        alloc.put(Jacc[c]);
        Jacc[c] = nullptr;
    }
    alloc.put(st);
    alloc.put(hist);
    alloc.put(counts_d);
    alloc.put(wdens_d);
    wdens_d = nullptr;
    alloc.put(newcount_d);
    alloc.put(kcnt_d);
    alloc.put(kofs_d);
    alloc.put(nleave_d);
    alloc.put(narrive_d);
    alloc.put(nhole_d);
    alloc.put(moved_d);
    if (porder_d) alloc.put(porder_d);
    alloc.put(prefix_d);
    alloc.put(tprefix_d);
    alloc.put(nbt_d);
    alloc.put(upart);
    alloc.put(kpart);
    alloc.put(rho0_d);
    alloc.put(rhoprev_d);
    rho0_d = rhoprev_d = nullptr;
    alloc.put(view_d);
    alloc.put(laser_ey);
    alloc.put(laser_ez);
    for (auto &e : timing.events) {
        (void)hipEventDestroy(e.a);
        (void)hipEventDestroy(e.b);
    }
    for (auto &e : timing.pool) (void)hipEventDestroy(e);
    timing.events.clear();
    timing.pool.clear();
}

// Allocate a particle layout whose patch capacities hold `need` particles
// with slack, and point the view at it.  The previous buffers are kept in
// `old` (caller frees them) so their contents can be copied over.
template <typename T>
std::vector<void *> SimImpl<T>::layout_particles(const std::vector<int32_t> &need)
{
    sync_layout();
    std::vector<int32_t> cap(npatch);
    std::vector<int64_t> off(npatch + 1, 0);
    // floor of every patch: the given minimum, or else the mean occupancy
    int64_t floor_cap = desc.min_capacity;
    if (floor_cap == 0) {
        int64_t tot = 0;
        for (int p = 0; p < npatch; ++p) tot += need[p];
        floor_cap = std::max<int64_t>(64, (tot + npatch - 1) / std::max(npatch, 1));
    }
    for (int p = 0; p < npatch; ++p) {
        int64_t c = (int64_t)std::ceil(desc.capacity_factor * need[p]);
        c = std::max<int64_t>(c, floor_cap);
        c = std::max<int64_t>(c, need[p]);
        c = (c + 63) & ~int64_t(63);
        if (p < (int)cap_h.size()) c = std::max<int64_t>(c, cap_h[p]);  // never shrink
        c = std::max<int64_t>(c, cap_floor);
        if (c > INT32_MAX / 2) throw Error(PIC_EOVERFLOW, "patch capacity overflow");
        cap[p] = (int32_t)c;
        off[p + 1] = off[p] + c;
    }
    const int64_t total = off[npatch];
    // work items address particle slots with 32-bit offsets
    if (total > INT32_MAX) throw Error(PIC_EOVERFLOW, "more than 2^31 - 1 particle slots in one simulation");
    std::vector<void *> old;
    old.swap(part_bufs);
    try {
        auto get = [&](size_t bytes) {
            void *p = alloc.get(bytes);
            part_bufs.push_back(p);
            return p;
        };
        pwid = nd == 3 ? 4 : 2;
        pP = (T *)get(sizeof(T) * total * pwid);
        sP = (T *)get(sizeof(T) * total * pwid);
        pM = (T *)get(sizeof(T) * total * 4);
        sM = (T *)get(sizeof(T) * total * 4);
        // (in 3-D the id rides in the position vector)
        pid = nd == 2 ? (int64_t *)get(sizeof(int64_t) * total) : nullptr;
        sid = nd == 2 ? (int64_t *)get(sizeof(int64_t) * total) : nullptr;
        code = (uint8_t *)get(total);
        holes = (int32_t *)get(sizeof(int32_t) * total);
        cap_d = (int32_t *)get(sizeof(int32_t) * npatch);
        off_d = (int64_t *)get(sizeof(int64_t) * (npatch + 1));
        hipcheck(hipMemcpyAsync(cap_d, cap.data(), sizeof(int32_t) * npatch, hipMemcpyHostToDevice, stream), "cap");
        hipcheck(hipMemcpyAsync(off_d, off.data(), sizeof(int64_t) * (npatch + 1), hipMemcpyHostToDevice, stream), "off");
    } catch (...) {
        for (void *p : part_bufs) alloc.put(p);
        part_bufs.swap(old);
        throw;
    }
    cap_h = cap;
    off_h = off;
    total_cap = total;
    max_items_cache = -1;
    refresh_view();
    return old;
}

template <typename T>
void SimImpl<T>::refresh_view()
{
    SimDev<T> &V = v;
    for (int a = 0; a < 3; ++a) {
        V.n[a] = n[a];
        V.P[a] = P[a];
        V.np[a] = np[a];
        V.fn[a] = fn[a];
        V.periodic[a] = periodic[a];
        V.d[a] = (T)(a < nd ? desc.d[a] : 1.0);
    }
    V.npatch = npatch;
    V.ndim = nd;
    V.lane_stride = lane_stride;
    V.morder = desc.maxwell_order == 6 ? 6 : 2;
    V.win = win_on ? 1 : 0;
    V.wppc[0] = win_ppc[0];
    V.wppc[1] = win_ppc[1];
    V.wstart = win_start;
    V.wvel = win_v;
    V.wdt = desc.dt;
    V.wdx = desc.d[0];
    V.wdens = wdens_d;
    V.wncols = win_ncols;
    V.mevery = merge_every;
    V.mcmax = merge_cmax;
    V.miters = merge_iters;
    V.dt = (T)desc.dt;
    V.q = (T)desc.q;
    V.m = (T)desc.m;
    V.vcell = desc.d[0] * desc.d[1] * (nd == 3 ? desc.d[2] : 1.0);
    for (int b = 0; b < 2; ++b)
        for (int c = 0; c < 6; ++c) V.F[b][c] = F[b][c];
    for (int b = 0; b < 2; ++b)
        for (int c = 0; c < 3; ++c) V.J[b][c] = J[b][c];
    V.det = desc.deterministic ? 1 : 0;
    for (int c = 0; c < 3; ++c) V.Jacc[c] = Jacc[c];
    V.pos = pP; V.spos = sP; V.mom = pM; V.smom = sM; V.pw = pwid;
    V.id = pid; V.sid = sid; V.code = code; V.holes = holes;
    V.cap = cap_d; V.off = off_d; V.count = counts_d; V.newcount = newcount_d;
    V.kcnt = kcnt_d; V.kofs = kofs_d; V.nleave = nleave_d; V.narrive = narrive_d; V.nhole = nhole_d;
    V.moved = moved_d;
    V.porder = porder_d;
    V.laser_ey = laser_ey; V.laser_ez = laser_ez; V.laser_steps = laser_steps;
    V.nlaser = (int)lasers.size();
    for (int l = 0; l < V.nlaser; ++l) {
        const PicLaserDesc &L = lasers[l];
        const double vals[8] = {L.a0, L.omega0, L.w0, L.tau, L.t0, L.x_focus, L.y_center, L.phase};
        for (int c = 0; c < 8; ++c) V.las[l][c] = vals[c];
        V.las_pol[l] = L.polarisation;
    }
    for (int a = 0; a < 3; ++a) V.dd[a] = a < nd ? desc.d[a] : 1.0;
    V.st = st; V.hist = hist; V.upart = upart; V.kpart = kpart; V.nbt = nbt_d;
    hipcheck(hipMemcpyAsync(view_d, &v, sizeof(v), hipMemcpyHostToDevice, stream), "view upload");
    ++layout_version;
}

template <typename T>
void SimImpl<T>::set_particles(int64_t cnt, const double *const xs[3], const double *const us[3],
                               const double *w)
{
    check_free();
    for (int64_t k = 0; k < cnt; ++k)
        for (int a = 0; a < nd; ++a)
            if (!(xs[a][k] >= 0.0 && xs[a][k] < (double)n[a]))
                throw Error(PIC_EINVAL, "particle " + std::to_string(k) + " outside the domain");
    if (nd == 3 && sizeof(T) == 4 && cnt >= ((int64_t)1 << 32))
        throw Error(PIC_EINVAL, "a 3-D FP32 simulation holds fewer than 2^32 particles");
    // cell and patch of each particle, and counts
    auto cell_of = [&](int64_t k, int a) { return a < nd ? std::min((int)std::floor(xs[a][k]), n[a] - 1) : 0; };
    std::vector<int32_t> pp(cnt), counts(npatch, 0);
    for (int64_t k = 0; k < cnt; ++k) {
        pp[k] = cell_of(k, 0) / P[0] + np[0] * (cell_of(k, 1) / P[1] + np[1] * (cell_of(k, 2) / P[2]));
        counts[pp[k]]++;
    }
    lane_stride = desc.lane_stride ? desc.lane_stride : default_lane_stride(nd);
    hipcheck(hipStreamSynchronize(stream), "sync");
    std::vector<void *> old = layout_particles(counts);
    for (void *p : old) alloc.put(p);
    // canonical initial order: id order inside each patch
    std::vector<int64_t> pos(off_h.begin(), off_h.end() - 1);
    const int64_t tot = total_cap;
    std::vector<T> hP((size_t)tot * pwid, T(0)), hM((size_t)tot * 4, T(0));
    std::vector<int64_t> hid(tot, -1);
    const T pmax[3] = {std::nextafter((T)P[0], (T)0), std::nextafter((T)P[1], (T)0),
                       std::nextafter((T)P[2], (T)0)};
    for (int64_t k = 0; k < cnt; ++k) {
        const int p = pp[k];
        const int64_t t = pos[p]++;
        const int o[3] = {(p % np[0]) * P[0], ((p / np[0]) % np[1]) * P[1], (p / (np[0] * np[1])) * P[2]};
        for (int a = 0; a < nd; ++a) {
            T loc = (T)(xs[a][k] - (double)o[a]);
            if (loc > pmax[a]) loc = pmax[a];
            if (loc < T(0)) loc = T(0);
            hP[(size_t)t * pwid + a] = loc;
        }
        for (int a = 0; a < 3; ++a) hM[(size_t)t * 4 + a] = us[a] ? (T)us[a][k] : T(0);
        hM[(size_t)t * 4 + 3] = (T)w[k];
        if (nd == 3) hP[(size_t)t * 4 + 3] = id_pad<T>(k);
        else hid[t] = k;
    }
    hipcheck(hipMemcpyAsync(pP, hP.data(), sizeof(T) * hP.size(), hipMemcpyHostToDevice, stream), "x");
    hipcheck(hipMemcpyAsync(pM, hM.data(), sizeof(T) * hM.size(), hipMemcpyHostToDevice, stream), "u, w");
    if (pid) hipcheck(hipMemcpyAsync(pid, hid.data(), sizeof(int64_t) * tot, hipMemcpyHostToDevice, stream), "id");
    hipcheck(hipMemsetAsync(code, ndir / 2, tot, stream), "code");
    finish_load(counts, cnt);
}

// Common end of a particle load: counts, a fresh state block (step 0), the
// load-time charge density.
template <typename T>
void SimImpl<T>::finish_load(const std::vector<int32_t> &counts, int64_t total)
{
    hipcheck(hipMemcpyAsync(counts_d, counts.data(), sizeof(int32_t) * npatch, hipMemcpyHostToDevice, stream), "counts");
    hipcheck(hipMemsetAsync(moved_d, 1, sizeof(int32_t) * npatch, stream), "moved");
    SimState s0;
    std::memset(&s0, 0, sizeof(s0));
    s0.next_id = total;
    hipcheck(hipMemcpyAsync(st, &s0, sizeof(s0), hipMemcpyHostToDevice, stream), "state");
    // the weight bound behind the fixed-point scale of the current
    launch_wmax<T>(view_d, npatch, stream);
    hipcheck(hipGetLastError(), "weight bound launch");
    hipcheck(hipStreamSynchronize(stream), "sync");
    relayouts = 0;
    if (solo) solo->dirty = true;
    record_rho0();
}

// Species description (one species per simulation; the immobile neutralising
// ions are implicit: their charge is minus the species' charge at load).
template <typename T>
void SimImpl<T>::add_species(const PicSpeciesDesc &sp)
{
    check_free();
    if (has_species) throw Error(PIC_ENOTSUP, "one species per simulation");
    if (sp.q != desc.q || sp.m != desc.m) throw Error(PIC_EINVAL, "species charge and mass must equal the descriptor's");
    if (sp.profile < 0 || sp.profile > 2) throw Error(PIC_EINVAL, "unknown density profile");
    if (sp.loading < 0 || sp.loading > 1) throw Error(PIC_EINVAL, "unknown loading rule");
    if (sp.ppc < 1 || sp.ppc > 4096) throw Error(PIC_EINVAL, "ppc must be 1..4096");
    if (!(sp.n0 > 0.0) || !(sp.temperature >= 0.0) || !std::isfinite(sp.temperature))
        throw Error(PIC_EINVAL, "n0 must be positive and the temperature finite and non-negative");
    for (double v : sp.param)
        if (!std::isfinite(v)) throw Error(PIC_EINVAL, "profile parameters must be finite");
    if (sp.profile == PIC_PROFILE_COS_SPHERE && (sp.param[4] < 0.0 || sp.param[5] < 0.0 || std::fabs(sp.param[0]) > 1.0))
        throw Error(PIC_EINVAL, "cosine modulation above 1 or negative sphere radius / factor");
    species = sp;
    has_species = true;
}

// Generate the species' particles on the device (see k_init.hip).
template <typename T>
void SimImpl<T>::particles_init()
{
    check_free();
    if (!has_species) throw Error(PIC_ESTATE, "no species added");
    InitSpec sp;
    std::memset(&sp, 0, sizeof(sp));
    sp.profile = species.profile;
    sp.loading = species.loading;
    sp.ppc = species.ppc;
    sp.nd = nd;
    sp.n0 = species.n0;
    for (int i = 0; i < 6; ++i) sp.p[i] = species.param[i];
    sp.sigma = std::sqrt(species.temperature);
    sp.seed = species.seed;
    for (int a = 0; a < 3; ++a) {
        sp.n[a] = n[a];
        sp.P[a] = P[a];
        sp.np[a] = np[a];
        sp.d[a] = a < nd ? desc.d[a] : 1.0;
    }
    const int64_t nseg = (int64_t)n[1] * n[2] * np[0];
    hipcheck(hipStreamSynchronize(stream), "sync");
    int64_t *seg_d = (int64_t *)alloc.get(sizeof(int64_t) * nseg);
    std::vector<int64_t> seg(nseg);
    launch_init_count(sp, nseg, seg_d, stream);
    hipcheck(hipGetLastError(), "init count launch");
    hipcheck(hipMemcpyAsync(seg.data(), seg_d, sizeof(int64_t) * nseg, hipMemcpyDeviceToHost, stream), "segments");
    hipcheck(hipStreamSynchronize(stream), "sync");
    alloc.put(seg_d);
    // first id of every segment (row-major order) and its first slot in its
    // patch (segments of a patch come in the patch's own row-major order)
    std::vector<int64_t> first(nseg);
    std::vector<int32_t> slot0(nseg), counts(npatch, 0);
    std::vector<int64_t> pcount(npatch, 0);
    int64_t total = 0;
    for (int64_t s_ = 0; s_ < nseg; ++s_) {
        first[s_] = total;
        total += seg[s_];
        const int px = (int)(s_ % np[0]);
        const int64_t r = s_ / np[0];
        const int j = (int)(r % n[1]), k = (int)(r / n[1]);
        const int p = px + np[0] * (j / P[1] + np[1] * (k / P[2]));
        slot0[s_] = (int32_t)pcount[p];
        pcount[p] += seg[s_];
        if (pcount[p] > INT32_MAX / 4) throw Error(PIC_EOVERFLOW, "too many particles in one patch");
    }
    if (total >= ((int64_t)1 << 41)) throw Error(PIC_EINVAL, "too many particles");
    if (nd == 3 && sizeof(T) == 4 && total >= ((int64_t)1 << 32))
        throw Error(PIC_EINVAL, "a 3-D FP32 simulation holds fewer than 2^32 particles");
    for (int p = 0; p < npatch; ++p) counts[p] = (int32_t)pcount[p];
    lane_stride = desc.lane_stride ? desc.lane_stride : default_lane_stride(nd);
    std::vector<void *> old = layout_particles(counts);
    for (void *p : old) alloc.put(p);
    const int64_t tot = total_cap;
    hipcheck(hipMemsetAsync(pP, 0, sizeof(T) * tot * pwid, stream), "clear x");
    hipcheck(hipMemsetAsync(pM, 0, sizeof(T) * tot * 4, stream), "clear u, w");
    if (pid) hipcheck(hipMemsetAsync(pid, 0xff, sizeof(int64_t) * tot, stream), "clear id");
    hipcheck(hipMemsetAsync(code, ndir / 2, tot, stream), "code");
    int64_t *first_d = (int64_t *)alloc.get(sizeof(int64_t) * nseg);
    int32_t *slot_d = nullptr;
    try {
        slot_d = (int32_t *)alloc.get(sizeof(int32_t) * nseg);
    } catch (...) {
        alloc.put(first_d);
        throw;
    }
    hipcheck(hipMemcpyAsync(first_d, first.data(), sizeof(int64_t) * nseg, hipMemcpyHostToDevice, stream), "first ids");
    hipcheck(hipMemcpyAsync(slot_d, slot0.data(), sizeof(int32_t) * nseg, hipMemcpyHostToDevice, stream), "first slots");
    launch_init_fill<T>(sp, nseg, first_d, slot_d, view_d, stream);
    hipcheck(hipGetLastError(), "init fill launch");
    hipcheck(hipStreamSynchronize(stream), "sync");
    alloc.put(first_d);
    alloc.put(slot_d);
    finish_load(counts, total);
}

// Gaussian laser through the open x = 0 face (2-D), evaluated by the Yee
// kernel every step.
template <typename T>
void SimImpl<T>::add_laser(const PicLaserDesc &l)
{
    check_free();
    if (nd != 2) throw Error(PIC_ENOTSUP, "laser injection needs an open x face (2-D boxes)");
    if (periodic[0]) throw Error(PIC_EINVAL, "laser injection needs an open x axis");
    if (l.face != 0) throw Error(PIC_ENOTSUP, "only the x = 0 face takes a laser");
    if ((int)lasers.size() >= kMaxLasers) throw Error(PIC_ENOTSUP, "at most four lasers");
    if (l.polarisation != 1 && l.polarisation != 2) throw Error(PIC_EINVAL, "polarisation must be 1 (Ey) or 2 (Ez)");
    const double v[8] = {l.a0, l.omega0, l.w0, l.tau, l.t0, l.x_focus, l.y_center, l.phase};
    for (double x : v)
        if (!std::isfinite(x)) throw Error(PIC_EINVAL, "laser parameters must be finite");
    if (!(l.a0 >= 0.0 && l.omega0 > 0.0 && l.w0 > 0.0 && l.tau > 0.0))
        throw Error(PIC_EINVAL, "a0 >= 0, omega0 > 0, w0 > 0 and tau > 0 are required");
    hipcheck(hipStreamSynchronize(stream), "sync");
    lasers.push_back(l);
    refresh_view();
    hipcheck(hipStreamSynchronize(stream), "sync");
}

// Charge density of the particles as loaded: the reference of the Gauss
// residual (the immobile neutralising ions carry its negative).
template <typename T>
void SimImpl<T>::record_rho0()
{
    if (!rho0_d) rho0_d = (double *)alloc.get(sizeof(double) * fsize);
    fill_doubles(rho0_d, fsize, 0.0, stream);
    launch_rho<T>(view_d, npatch, nd, rho0_d, stream);
    hipcheck(hipGetLastError(), "rho launch");
    hipcheck(hipStreamSynchronize(stream), "sync");
    rho0_valid = true;
    alloc.put(rhoprev_d);
    rhoprev_d = nullptr;
    rhoprev_step = -1;
}

// Charge density without any allocation: the static per-device scratch
// holds the node sums (cleared by a kernel), then one copy to the host.
template <typename T>
void SimImpl<T>::rho_noalloc(double *h, size_t count)
{
    if ((int64_t)count != fsize) throw Error(PIC_EINVAL, "count must equal the number of field nodes");
    if (fsize > (int64_t)PIC_NOALLOC_MAX_NODES)
        throw Error(PIC_EINVAL, "grid has " + std::to_string(fsize) + " nodes, more than the " +
                                    std::to_string((int64_t)PIC_NOALLOC_MAX_NODES) +
                                    " the allocation-free scratch holds");
    double *scr = noalloc_scratch();
    fill_doubles(scr, fsize, 0.0, stream);
    launch_rho<T>(view_d, npatch, nd, scr, stream);
    hipcheck(hipGetLastError(), "rho launch");
    hipcheck(hipMemcpyAsync(h, scr, sizeof(double) * fsize, hipMemcpyDeviceToHost, stream), "rho");
    hipcheck(hipStreamSynchronize(stream), "sync");
}

// The paper's imbalance measure (section 3.1, Fig. 4: time of the busiest
// unit over the mean) from the item stamps of the last stamped particle
// launch: per compute unit, the summed time of this simulation's items.
template <typename T>
void SimImpl<T>::imbalance(PicImbalance *out)
{
    BatchImpl<T> *b = batch ? batch : solo;
    if (!b || !b->stamps_d || b->dirty) throw Error(PIC_ESTATE, "no particle launch has been stamped");
    int slot = -1;
    for (size_t i = 0; i < b->members.size(); ++i)
        if (b->members[i] == this) slot = (int)i;
    hipcheck(hipStreamSynchronize(stream), "sync");
    int n = 0;
    hipcheck(hipMemcpy(&n, b->stamp_n_d, sizeof(int), hipMemcpyDeviceToHost), "stamp count");
    n = std::max(0, std::min(n, b->table_cap_items));
    std::vector<ItemStamp> rec(n);
    if (n) hipcheck(hipMemcpy(rec.data(), b->stamps_d, sizeof(ItemStamp) * n, hipMemcpyDeviceToHost), "stamps");
    int dev = 0, khz = 0;
    hipcheck(hipGetDevice(&dev), "device");
    hipcheck(hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev), "clock rate");
    if (khz <= 0) throw Error(PIC_EHIP, "no device clock rate");
    const double us = 1000.0 / khz;
    std::map<int, double> busy;
    std::vector<double> pcost(npatch, 0.0);
    long long t_lo = LLONG_MAX, t_hi = LLONG_MIN;
    int items = 0;
    for (const ItemStamp &r : rec) {
        if (r.sim != slot || r.t1 < r.t0 || r.patch < 0 || r.patch >= npatch) continue;
        const double d = (double)(r.t1 - r.t0) * us;
        busy[r.hw] += d;
        pcost[r.patch] += d;
        t_lo = std::min(t_lo, r.t0);
        t_hi = std::max(t_hi, r.t1);
        ++items;
    }
    if (!items) throw Error(PIC_ESTATE, "the stamped launch ran no item of this simulation");
    const int ncu = cu_count();
    double tot = 0.0, mx = 0.0;
    for (auto &kv : busy) {
        tot += kv.second;
        mx = std::max(mx, kv.second);
    }
    // the same item times dealt to the CUs as fixed domains: equal runs of
    // patch ids, or curve segments cut by particle count (section 3.1)
    auto worst = [&](const std::vector<int64_t> &bounds, const std::vector<int32_t> &order) {
        double w = 0.0;
        for (int r = 0; r < ncu; ++r) {
            double c = 0.0;
            for (int64_t q = bounds[r]; q < bounds[r + 1]; ++q) c += pcost[order[q]];
            w = std::max(w, c);
        }
        return w;
    };
    std::vector<int32_t> ids(npatch);
    std::iota(ids.begin(), ids.end(), 0);
    std::vector<int64_t> eq(ncu + 1);
    for (int r = 0; r <= ncu; ++r) eq[r] = (int64_t)r * npatch / ncu;
    std::vector<int32_t> curve;
    std::string why;
    const int npc[3] = {np[0], np[1], nd == 3 ? np[2] : 1};
    if (hilbert_patch_order(nd, npc, curve, why) != PIC_OK) curve = ids;
    std::vector<int32_t> cnt = read_counts();
    std::vector<int64_t> cost(npatch), seg(ncu + 1);
    for (int q = 0; q < npatch; ++q) cost[q] = cnt[curve[q]];
    curve_segments(cost.data(), npatch, ncu, seg.data());
    const double mean = tot / ncu;
    const SimState s = read_state();
    out->step = s.step;
    out->items = items;
    out->units = (int32_t)busy.size();
    out->device_units = ncu;
    out->span_us = (double)(t_hi - t_lo) * us;
    out->busy_max_us = mx;
    out->busy_mean_us = mean;
    out->imbalance = mean > 0 ? mx / mean : 0.0;
    out->static_imbalance = mean > 0 ? worst(eq, ids) / mean : 0.0;
    out->segment_imbalance = mean > 0 ? worst(seg, curve) / mean : 0.0;
    out->patch_max_us = *std::max_element(pcost.begin(), pcost.end());
    out->patch_mean_us = tot / npatch;
}

// Gauss and continuity residuals of the current state (see k_diag.hip).
template <typename T>
void SimImpl<T>::residuals(PicResiduals *out)
{
    if (win_on) throw Error(PIC_ENOTSUP, "residuals are not defined for a moving window");
    const SimState s = read_state();
    if (s.flags & kFlagPending) throw Error(PIC_ESTATE, "a re-binning is pending");
    double *rho = (double *)alloc.get(sizeof(double) * fsize);
    double *part = nullptr;
    try {
        part = (double *)alloc.get(sizeof(double) * (residual_partials() + 4));
    } catch (...) {
        alloc.put(rho);
        throw;
    }
    fill_doubles(rho, fsize, 0.0, stream);
    launch_rho<T>(view_d, npatch, nd, rho, stream);
    const bool cont = rhoprev_d && rhoprev_step == s.step - 1;
    launch_residuals<T>(view_d, nd, fsize, (int)(s.step & 1), (int)((s.step + 1) & 1), rho,
                        rho0_valid ? rho0_d : nullptr, cont ? rhoprev_d : nullptr, part,
                        part + residual_partials(), stream);
    hipcheck(hipGetLastError(), "residual launch");
    double m[4];
    hipcheck(hipMemcpyAsync(m, part + residual_partials(), sizeof(m), hipMemcpyDeviceToHost, stream), "residuals");
    hipcheck(hipStreamSynchronize(stream), "sync");
    alloc.put(part);
    alloc.put(rhoprev_d);
    rhoprev_d = rho;
    rhoprev_step = s.step;
    const double nan = std::numeric_limits<double>::quiet_NaN();
    out->step = s.step;
    out->gauss = rho0_valid ? (m[3] > 0.0 ? m[0] / m[3] : m[0]) : nan;
    out->continuity = cont ? (m[2] > 0.0 ? m[1] / m[2] : m[1]) : nan;
    out->rho_max = m[2];
    out->rho0_max = rho0_valid ? m[3] : nan;
}

template <typename T>
void SimImpl<T>::set_laser(int64_t nsteps, const double *ey, const double *ez)
{
    check_free();
    if (nd != 2) throw Error(PIC_ENOTSUP, "laser injection needs an open x face (2-D boxes)");
    hipcheck(hipStreamSynchronize(stream), "sync");
    alloc.put(laser_ey);
    alloc.put(laser_ez);
    laser_ey = laser_ez = nullptr;
    laser_steps = nsteps;
    const size_t cnt = (size_t)nsteps * n[1];
    std::vector<T> tmp(cnt);
    if (ey) {
        for (size_t k = 0; k < cnt; ++k) tmp[k] = (T)ey[k];
        laser_ey = (T *)alloc.get(sizeof(T) * cnt);
        hipcheck(hipMemcpyAsync(laser_ey, tmp.data(), sizeof(T) * cnt, hipMemcpyHostToDevice, stream), "laser");
        hipcheck(hipStreamSynchronize(stream), "sync");
    }
    if (ez) {
        for (size_t k = 0; k < cnt; ++k) tmp[k] = (T)ez[k];
        laser_ez = (T *)alloc.get(sizeof(T) * cnt);
        hipcheck(hipMemcpyAsync(laser_ez, tmp.data(), sizeof(T) * cnt, hipMemcpyHostToDevice, stream), "laser");
        hipcheck(hipStreamSynchronize(stream), "sync");
    }
    refresh_view();
    hipcheck(hipStreamSynchronize(stream), "sync");
}

// Moving window (2-D, open x): jumps of one patch column; every patch must
// be able to hold the particles one jump injects into it.
template <typename T>
void SimImpl<T>::set_window(int64_t start, double vel, int ppcx, int ppcy, const double *dens,
                            int64_t ncols)
{
    check_free();
    if (nd != 2) throw Error(PIC_ENOTSUP, "the moving window is built for 2-D boxes");
    if (periodic[0]) throw Error(PIC_EINVAL, "the moving window needs an open x axis");
    if (!(vel > 0.0 && vel <= 1.0)) throw Error(PIC_EINVAL, "window speed must be in (0, 1]");
    if (start < 0) throw Error(PIC_EINVAL, "negative window start");
    if (ppcx < 1 || ppcy < 1 || (int64_t)ppcx * ppcy > 4096) throw Error(PIC_EINVAL, "particles per cell must be 1..4096");
    if (ncols < 1 || !dens) throw Error(PIC_EINVAL, "empty density table");
    for (int64_t c = 0; c < ncols; ++c)
        if (!(dens[c] >= 0.0) || !std::isfinite(dens[c])) throw Error(PIC_EINVAL, "density must be finite and non-negative");
    if (np[0] > kWindowMaxPatchColumns) throw Error(PIC_ENOTSUP, "more than 4096 patch columns");
    const int64_t need = (int64_t)P[0] * P[1] * ppcx * ppcy;
    if (need > INT32_MAX / 4) throw Error(PIC_EINVAL, "too many injected particles per patch");
    hipcheck(hipStreamSynchronize(stream), "sync");
    double *d = (double *)alloc.get(sizeof(double) * ncols);
    hipcheck(hipMemcpyAsync(d, dens, sizeof(double) * ncols, hipMemcpyHostToDevice, stream), "window");
    hipcheck(hipStreamSynchronize(stream), "sync");
    alloc.put(wdens_d);
    wdens_d = d;
    win_on = true;
    win_start = start;
    win_v = vel;
    win_ppc[0] = ppcx;
    win_ppc[1] = ppcy;
    win_ncols = ncols;
    cap_floor = (int32_t)need;
    sync_layout();
    bool small = false;
    for (int32_t c : cap_h) small = small || c < cap_floor;
    if (small) relayout(read_counts());
    refresh_view();
    hipcheck(hipStreamSynchronize(stream), "sync");
}

// Particle merging (2-D): after every `every`-th step (0: never), or now.
template <typename T>
void SimImpl<T>::set_merge(int every, int cmax, int iters)
{
    check_free();
    if (every < 0) throw Error(PIC_EINVAL, "negative merge interval");
    if (every > 0) {
        if (nd != 2) throw Error(PIC_ENOTSUP, "particle merging is built for 2-D boxes");
        if (cmax < 4 || cmax > 32) throw Error(PIC_EINVAL, "cell_max must be 4..32");
        if (iters < 1 || iters > 64) throw Error(PIC_EINVAL, "iterations must be 1..64");
    }
    hipcheck(hipStreamSynchronize(stream), "sync");
    merge_every = every;
    merge_cmax = cmax;
    merge_iters = iters;
    refresh_view();
    hipcheck(hipStreamSynchronize(stream), "sync");
    // the step pass launches the merge kernel built for this cmax (a captured
    // graph holds the launch of the earlier setting)
    if (solo) solo->dirty = true;
}

template <typename T>
int64_t SimImpl<T>::merge_now(int cmax, int iters)
{
    check_free();
    if (nd != 2) throw Error(PIC_ENOTSUP, "particle merging is built for 2-D boxes");
    if (cmax < 4 || cmax > 32) throw Error(PIC_EINVAL, "cell_max must be 4..32");
    if (iters < 1 || iters > 64) throw Error(PIC_EINVAL, "iterations must be 1..64");
    const SimState s0 = read_state();
    if (s0.flags & kFlagPending) throw Error(PIC_ESTATE, "a re-binning is pending");
    if (!cap_d) return 0;
    launch_merge<T>(view_d, npatch, cmax, iters, 1, cmax, stream);
    hipcheck(hipGetLastError(), "merge launch");
    const SimState s1 = read_state();
    return s1.merged - s0.merged;
}

// Re-read the capacities and segment offsets that window jumps rotate.
template <typename T>
void SimImpl<T>::sync_layout()
{
    if (!win_on || cap_h.empty() || !cap_d) return;
    hipcheck(hipStreamSynchronize(stream), "sync");
    hipcheck(hipMemcpyAsync(cap_h.data(), cap_d, sizeof(int32_t) * npatch, hipMemcpyDeviceToHost, stream), "cap");
    hipcheck(hipMemcpyAsync(off_h.data(), off_d, sizeof(int64_t) * (npatch + 1), hipMemcpyDeviceToHost, stream), "off");
    hipcheck(hipStreamSynchronize(stream), "sync");
}

template <typename T>
void SimImpl<T>::set_step(int64_t step)
{
    check_free();
    if (step < 0) throw Error(PIC_EINVAL, "negative step");
    SimState s = read_state();
    if (s.flags & kFlagPending) throw Error(PIC_ESTATE, "a re-binning is pending");
    // the current E, B move to the buffer of the new step's parity
    if ((s.step & 1) != (step & 1))
        for (int c = 0; c < 6; ++c)
            hipcheck(hipMemcpyAsync(F[step & 1][c], F[s.step & 1][c], sizeof(T) * fsize, hipMemcpyDeviceToDevice, stream), "fields");
    s.step = step;
    hipcheck(hipMemcpyAsync(&st->step, &s.step, sizeof(int64_t), hipMemcpyHostToDevice, stream), "step");
    hipcheck(hipStreamSynchronize(stream), "sync");
    rhoprev_step = -1;
}

template <typename T>
void SimImpl<T>::set_field(int comp, const double *h)
{
    check_free();
    if (comp < 0 || comp > 5) throw Error(PIC_EINVAL, "only E and B components can be set");
    std::vector<T> tmp(fsize);
    for (int64_t k = 0; k < fsize; ++k) tmp[k] = (T)h[k];
    const SimState s = read_state();
    hipcheck(hipMemcpyAsync(F[s.step & 1][comp], tmp.data(), sizeof(T) * fsize, hipMemcpyHostToDevice, stream), "field");
    hipcheck(hipStreamSynchronize(stream), "sync");
}

template <typename T>
void SimImpl<T>::get_field(int comp, double *h)
{
    if (comp < 0 || comp > 9) throw Error(PIC_EINVAL, "bad component");
    hipcheck(hipStreamSynchronize(stream), "sync");
    if (comp == PIC_RHO) {
        double *tmp = (double *)alloc.get(sizeof(double) * fsize);
        fill_doubles(tmp, fsize, 0.0, stream);
        launch_rho<T>(view_d, npatch, nd, tmp, stream);
        hipcheck(hipGetLastError(), "rho launch");
        hipcheck(hipMemcpyAsync(h, tmp, sizeof(double) * fsize, hipMemcpyDeviceToHost, stream), "rho");
        hipcheck(hipStreamSynchronize(stream), "sync");
        alloc.put(tmp);
        return;
    }
    SimState s;
    hipcheck(hipMemcpy(&s, st, sizeof(s), hipMemcpyDeviceToHost), "state");
    const T *src = comp < 6 ? F[s.step & 1][comp] : J[(s.step + 1) & 1][comp - 6];
    std::vector<T> tmp(fsize);
    hipcheck(hipMemcpyAsync(tmp.data(), src, sizeof(T) * fsize, hipMemcpyDeviceToHost, stream), "field");
    hipcheck(hipStreamSynchronize(stream), "sync");
    for (int64_t k = 0; k < fsize; ++k) h[k] = (double)tmp[k];
}

template <typename T>
SimState SimImpl<T>::read_state()
{
    SimState s;
    hipcheck(hipMemcpyAsync(&s, st, sizeof(s), hipMemcpyDeviceToHost, stream), "state");
    hipcheck(hipStreamSynchronize(stream), "sync");
    return s;
}

template <typename T>
std::vector<int32_t> SimImpl<T>::read_counts()
{
    std::vector<int32_t> c(npatch);
    hipcheck(hipMemcpyAsync(c.data(), counts_d, sizeof(int32_t) * npatch, hipMemcpyDeviceToHost, stream), "counts");
    hipcheck(hipStreamSynchronize(stream), "sync");
    return c;
}

template <typename T>
int64_t SimImpl<T>::num_particles()
{
    auto c = read_counts();
    return std::accumulate(c.begin(), c.end(), int64_t(0));
}

template <typename T>
void SimImpl<T>::get_particles(double *xo[3], double *uo[3], double *wo, int64_t *ido, size_t cnt)
{
    sync_layout();
    auto c = read_counts();
    const int64_t live = std::accumulate(c.begin(), c.end(), int64_t(0));
    if ((int64_t)cnt < live) throw Error(PIC_EINVAL, "output arrays too small");
    const int64_t tot = total_cap;
    std::vector<T> tmp;
    std::vector<int64_t> itmp;
    // component comp of an interleaved array of width wid (downloaded once)
    auto fetch = [&](const std::vector<T> &buf, int wid, int comp, double *dst, int axis) {
        int64_t o = 0;
        for (int p = 0; p < npatch; ++p) {
            const double org = axis == 0 ? (double)((p % np[0]) * P[0])
                             : axis == 1 ? (double)(((p / np[0]) % np[1]) * P[1])
                             : axis == 2 ? (double)((p / (np[0] * np[1])) * P[2]) : 0.0;
            for (int k = 0; k < c[p]; ++k) dst[o++] = org + (double)buf[(size_t)(off_h[p] + k) * wid + comp];
        }
    };
    auto download = [&](const T *src, int wid) {
        tmp.resize((size_t)tot * wid);
        hipcheck(hipMemcpyAsync(tmp.data(), src, sizeof(T) * tmp.size(), hipMemcpyDeviceToHost, stream), "particles");
        hipcheck(hipStreamSynchronize(stream), "sync");
    };
    if (xo[0] || xo[1] || (nd == 3 && xo[2])) {
        download(pP, pwid);
        for (int a = 0; a < nd; ++a) if (xo[a]) fetch(tmp, pwid, a, xo[a], a);
    }
    if (nd == 2 && xo[2]) std::fill(xo[2], xo[2] + live, 0.0);
    if (uo[0] || uo[1] || uo[2] || wo) {
        download(pM, 4);
        for (int a = 0; a < 3; ++a) if (uo[a]) fetch(tmp, 4, a, uo[a], 3);
        if (wo) fetch(tmp, 4, 3, wo, 3);
    }
    if (ido && nd == 3) {
        // (ids ride in the position vectors)
        download(pP, 4);
        int64_t o = 0;
        for (int p = 0; p < npatch; ++p)
            for (int k = 0; k < c[p]; ++k) ido[o++] = pad_id<T>(tmp[(size_t)(off_h[p] + k) * 4 + 3]);
    } else if (ido) {
        itmp.resize(tot);
        hipcheck(hipMemcpyAsync(itmp.data(), pid, sizeof(int64_t) * tot, hipMemcpyDeviceToHost, stream), "ids");
        hipcheck(hipStreamSynchronize(stream), "sync");
        int64_t o = 0;
        for (int p = 0; p < npatch; ++p)
            for (int k = 0; k < c[p]; ++k) ido[o++] = itmp[off_h[p] + k];
    }
}

template <typename T>
void SimImpl<T>::history(int64_t first, int64_t cnt, double *U, double *K, int64_t *pushed)
{
    SimState s = read_state();
    if (first < 0 || cnt < 0 || first + cnt > s.step || s.step - first > kHistLen)
        throw Error(PIC_EINVAL, "history range not available");
    std::vector<double> h(kHistLen * 4);
    hipcheck(hipMemcpyAsync(h.data(), hist, sizeof(double) * h.size(), hipMemcpyDeviceToHost, stream), "hist");
    hipcheck(hipStreamSynchronize(stream), "sync");
    for (int64_t k = 0; k < cnt; ++k) {
        const double *r = &h[((first + k) % kHistLen) * 4];
        if (U) U[k] = r[0];
        if (K) K[k] = r[1];
        if (pushed) pushed[k] = (int64_t)r[2];
    }
}

// ---------------------------------------------------------------------------
// checkpoint
//
// Blob layout (host byte order): a header, the patch counts, E and B of the
// current time level and the last deposit (3 + 3 + 3 arrays of fsize values
// of the simulation's precision), the particles in canonical (patch, slot)
// order (patch-local positions per axis, three momenta, weight, 64-bit id),
// and the energy-history ring.

namespace {
struct CkptHeader {
    char magic[8];
    int32_t version, ndim, precision, npatch;
    int32_t n[3], patch[3], periodic[3];
    int64_t live, step, removed, fsize;
    double U, K;
    int64_t wshift, next_id;  // moving window: jumps done, next injected id
};
constexpr char kCkptMagic[8] = {'P', 'I', 'C', 'S', 'T', 'A', 'T', 'E'};
}  // namespace

template <typename T>
size_t SimImpl<T>::state_bytes()
{
    const int64_t live = num_particles();
    return sizeof(CkptHeader) + sizeof(int32_t) * npatch + sizeof(T) * 9 * fsize +
           (size_t)live * (sizeof(T) * (nd + 4) + sizeof(int64_t)) + sizeof(double) * kHistLen * 4;
}

template <typename T>
void SimImpl<T>::state_save(void *blob)
{
    hipcheck(hipStreamSynchronize(stream), "sync");
    sync_layout();
    const SimState s = read_state();
    if (s.flags & kFlagPending) throw Error(PIC_ESTATE, "a re-binning is pending");
    const std::vector<int32_t> c = read_counts();
    const int64_t live = std::accumulate(c.begin(), c.end(), int64_t(0));
    CkptHeader h;
    std::memset(&h, 0, sizeof(h));
    std::memcpy(h.magic, kCkptMagic, 8);
    h.version = 2;
    h.ndim = nd;
    h.precision = precision;
    h.npatch = npatch;
    for (int a = 0; a < 3; ++a) { h.n[a] = n[a]; h.patch[a] = P[a]; h.periodic[a] = periodic[a]; }
    h.live = live;
    h.step = s.step;
    h.removed = s.removed;
    h.fsize = fsize;
    h.U = s.U;
    h.K = s.K;
    h.wshift = s.wshift;
    h.next_id = s.next_id;
    char *o = static_cast<char *>(blob);
    std::memcpy(o, &h, sizeof(h));
    o += sizeof(h);
    std::memcpy(o, c.data(), sizeof(int32_t) * npatch);
    o += sizeof(int32_t) * npatch;
    auto d2h = [&](const void *src, size_t bytes) {
        hipcheck(hipMemcpyAsync(o, src, bytes, hipMemcpyDeviceToHost, stream), "checkpoint");
        o += bytes;
    };
    for (int k = 0; k < 6; ++k) d2h(F[s.step & 1][k], sizeof(T) * fsize);
    for (int k = 0; k < 3; ++k) d2h(J[(s.step + 1) & 1][k], sizeof(T) * fsize);
    hipcheck(hipStreamSynchronize(stream), "sync");
    // particles: compact each array patch by patch
    const int64_t tot = total_cap;
    // (the checkpoint holds one array per component: x..., u_x, u_y, u_z, w)
    std::vector<T> tmp;
    auto download = [&](const T *src, int wid) {
        tmp.resize((size_t)tot * wid);
        hipcheck(hipMemcpyAsync(tmp.data(), src, sizeof(T) * tmp.size(), hipMemcpyDeviceToHost, stream), "checkpoint");
        hipcheck(hipStreamSynchronize(stream), "sync");
    };
    auto pack = [&](int wid, int comp) {
        for (int p = 0; p < npatch; ++p)
            for (int k = 0; k < c[p]; ++k) {
                std::memcpy(o, &tmp[(size_t)(off_h[p] + k) * wid + comp], sizeof(T));
                o += sizeof(T);
            }
    };
    download(pP, pwid);
    for (int a = 0; a < nd; ++a) pack(pwid, a);
    std::vector<int64_t> itmp(tot);
    if (nd == 3) {
        // (3-D ids ride in the position vectors)
        for (int64_t k = 0; k < tot; ++k) itmp[k] = pad_id<T>(tmp[(size_t)k * 4 + 3]);
    } else {
        hipcheck(hipMemcpyAsync(itmp.data(), pid, sizeof(int64_t) * tot, hipMemcpyDeviceToHost, stream), "checkpoint");
        hipcheck(hipStreamSynchronize(stream), "sync");
    }
    download(pM, 4);
    for (int a = 0; a < 4; ++a) pack(4, a);
    for (int p = 0; p < npatch; ++p) {
        std::memcpy(o, itmp.data() + off_h[p], sizeof(int64_t) * c[p]);
        o += sizeof(int64_t) * c[p];
    }
    d2h(hist, sizeof(double) * kHistLen * 4);
    hipcheck(hipStreamSynchronize(stream), "sync");
}

template <typename T>
void SimImpl<T>::state_load(const void *blob, size_t size)
{
    check_free();
    if (size < sizeof(CkptHeader)) throw Error(PIC_EINVAL, "checkpoint too small");
    CkptHeader h;
    std::memcpy(&h, blob, sizeof(h));
    if (std::memcmp(h.magic, kCkptMagic, 8) || h.version != 2) throw Error(PIC_EINVAL, "not a checkpoint");
    bool same = h.ndim == nd && h.precision == precision && h.npatch == npatch && h.fsize == fsize;
    for (int a = 0; a < 3; ++a)
        same = same && h.n[a] == n[a] && h.patch[a] == P[a] && h.periodic[a] == periodic[a];
    if (!same) throw Error(PIC_EINVAL, "checkpoint of a different grid, patch layout or precision");
    const char *i = static_cast<const char *>(blob) + sizeof(h);
    std::vector<int32_t> c(npatch);
    std::memcpy(c.data(), i, sizeof(int32_t) * npatch);
    i += sizeof(int32_t) * npatch;
    int64_t live = 0;
    for (int32_t v : c) {
        if (v < 0) throw Error(PIC_EINVAL, "corrupt checkpoint");
        live += v;
    }
    if (live != h.live) throw Error(PIC_EINVAL, "corrupt checkpoint");
    const size_t need = sizeof(CkptHeader) + sizeof(int32_t) * npatch + sizeof(T) * 9 * fsize +
                        (size_t)live * (sizeof(T) * (nd + 4) + sizeof(int64_t)) + sizeof(double) * kHistLen * 4;
    if (size < need) throw Error(PIC_EINVAL, "checkpoint truncated");
    hipcheck(hipStreamSynchronize(stream), "sync");
    // fields: the current level into F[step & 1], the last deposit into J[(step + 1) & 1]
    auto h2d = [&](void *dst, size_t bytes) {
        hipcheck(hipMemcpyAsync(dst, i, bytes, hipMemcpyHostToDevice, stream), "restore");
        i += bytes;
    };
    for (int k = 0; k < 6; ++k) h2d(F[h.step & 1][k], sizeof(T) * fsize);
    for (int k = 0; k < 3; ++k) h2d(J[(h.step + 1) & 1][k], sizeof(T) * fsize);
    for (int k = 0; k < 3; ++k) hipcheck(hipMemsetAsync(J[h.step & 1][k], 0, sizeof(T) * fsize, stream), "restore");
    hipcheck(hipStreamSynchronize(stream), "sync");
    // particles into a fresh layout
    std::vector<void *> old = layout_particles(c);
    for (void *p : old) alloc.put(p);
    const int64_t tot = total_cap;
    std::vector<T> tmp;
    auto unpack = [&](int wid, int comp) {
        for (int p = 0; p < npatch; ++p)
            for (int k = 0; k < c[p]; ++k) {
                std::memcpy(&tmp[(size_t)(off_h[p] + k) * wid + comp], i, sizeof(T));
                i += sizeof(T);
            }
    };
    auto upload = [&](T *dst) {
        hipcheck(hipMemcpyAsync(dst, tmp.data(), sizeof(T) * tmp.size(), hipMemcpyHostToDevice, stream), "restore");
        hipcheck(hipStreamSynchronize(stream), "sync");
    };
    // the ids follow the position and momentum arrays in the checkpoint
    std::vector<int64_t> itmp(tot, -1);
    {
        const char *ids = i + (size_t)live * sizeof(T) * (nd + 4);
        for (int p = 0; p < npatch; ++p) {
            std::memcpy(itmp.data() + off_h[p], ids, sizeof(int64_t) * c[p]);
            ids += sizeof(int64_t) * c[p];
        }
    }
    if (nd == 3 && sizeof(T) == 4)
        for (int p = 0; p < npatch; ++p)
            for (int k = 0; k < c[p]; ++k)
                if (itmp[off_h[p] + k] < 0 || itmp[off_h[p] + k] >= ((int64_t)1 << 32))
                    throw Error(PIC_EINVAL, "corrupt checkpoint");
    tmp.assign((size_t)tot * pwid, T(0));
    for (int a = 0; a < nd; ++a) unpack(pwid, a);
    if (nd == 3)
        for (int64_t k = 0; k < tot; ++k) tmp[(size_t)k * 4 + 3] = id_pad<T>(itmp[k]);
    upload(pP);
    tmp.assign((size_t)tot * 4, T(0));
    for (int a = 0; a < 4; ++a) unpack(4, a);
    upload(pM);
    i += (size_t)live * sizeof(int64_t);
    if (pid) hipcheck(hipMemcpyAsync(pid, itmp.data(), sizeof(int64_t) * tot, hipMemcpyHostToDevice, stream), "restore");
    hipcheck(hipMemsetAsync(code, ndir / 2, tot, stream), "restore");
    hipcheck(hipMemcpyAsync(counts_d, c.data(), sizeof(int32_t) * npatch, hipMemcpyHostToDevice, stream), "restore");
    h2d(hist, sizeof(double) * kHistLen * 4);
    SimState s0;
    std::memset(&s0, 0, sizeof(s0));
    s0.step = h.step;
    s0.removed = h.removed;
    s0.U = h.U;
    s0.K = h.K;
    s0.wshift = h.wshift;
    s0.next_id = h.next_id;
    hipcheck(hipMemcpyAsync(st, &s0, sizeof(s0), hipMemcpyHostToDevice, stream), "restore");
    launch_wmax<T>(view_d, npatch, stream);
    hipcheck(hipGetLastError(), "weight bound launch");
    hipcheck(hipMemsetAsync(kpart, 0, sizeof(double) * npatch, stream), "restore");
    hipcheck(hipStreamSynchronize(stream), "sync");
    if (solo) solo->dirty = true;
    // the charge at load is not part of a checkpoint
    rho0_valid = false;
    rhoprev_step = -1;
}

// ---------------------------------------------------------------------------
// launch-setting tuner

template <typename T>
void SimImpl<T>::autotune(int steps, const char *cache, PicTuneResult *out)
{
    check_free();
    if (steps <= 0) steps = 10;
    const int64_t live = num_particles();
    int bucket = 0;
    while (((int64_t)1 << bucket) < std::max<int64_t>(live, 1)) ++bucket;
    char key[160];
    std::snprintf(key, sizeof(key), "pic-tune nd=%d prec=%d n=%d,%d,%d patch=%d,%d,%d np2=%d", nd, precision,
                  n[0], n[1], n[2], P[0], P[1], P[2], bucket);
    struct Cfg {
        int block, field_tile, lane_stride, chunk;
    };
    auto apply = [&](const Cfg &c) {
        desc.block = c.block;
        desc.field_tile = c.field_tile;
        desc.chunk = c.chunk;
        lane_stride = c.lane_stride;
        refresh_view();
        if (solo) solo->dirty = true;
    };
    PicTuneResult res;
    std::memset(&res, 0, sizeof(res));
    // cache lookup: "<key> block field_tile lane_stride chunk"
    if (cache) {
        std::ifstream f(cache);
        std::string line;
        const std::string k(key);
        while (std::getline(f, line)) {
            if (line.compare(0, k.size(), k) != 0 || line.size() <= k.size() || line[k.size()] != ' ') continue;
            Cfg c;
            if (std::sscanf(line.c_str() + k.size(), "%d %d %d %d", &c.block, &c.field_tile, &c.lane_stride,
                            &c.chunk) == 4) {
                apply(c);
                res = {c.block, c.field_tile, c.lane_stride, c.chunk, 0.0, 0, 1};
                if (out) *out = res;
                return;
            }
        }
    }
    std::vector<char> blob(state_bytes());
    state_save(blob.data());
    const int ls0 = lane_stride;
    auto timed = [&](const Cfg &c) {
        apply(c);
        state_load(blob.data(), blob.size());
        hipcheck(hipStreamSynchronize(stream), "sync");
        const auto t0 = std::chrono::steady_clock::now();
        step(steps);
        hipcheck(hipStreamSynchronize(stream), "sync");
        const auto t1 = std::chrono::steady_clock::now();
        ++res.trials;
        return std::chrono::duration<double, std::milli>(t1 - t0).count() / steps;
    };
    Cfg best{desc.block, desc.field_tile, ls0, desc.chunk};
    double best_ms = timed(best);
    auto try_knob = [&](int Cfg::*field, std::initializer_list<int> values) {
        for (int v : values) {
            if (v == best.*field) continue;
            Cfg c = best;
            c.*field = v;
            const double ms = timed(c);
            if (ms < 0.99 * best_ms) {
                best = c;
                best_ms = ms;
            }
        }
    };
    try_knob(&Cfg::block, {256, 512, 1024});
    if (nd == 2) try_knob(&Cfg::field_tile, {1, 2, 3, 4, 5});
    try_knob(&Cfg::lane_stride, {std::max(1, ls0 / 2), std::min(64, ls0 * 2), 1});
    try_knob(&Cfg::chunk, {1024, 2048, 4096, 8192});
    apply(best);
    state_load(blob.data(), blob.size());
    res.block = best.block;
    res.field_tile = best.field_tile;
    res.lane_stride = best.lane_stride;
    res.chunk = best.chunk;
    res.ms_per_step = best_ms;
    for (int i = 0; i < 3; ++i) res.patch[i] = P[i];
    if (cache) {
        std::ofstream f(cache, std::ios::app);
        f << key << ' ' << best.block << ' ' << best.field_tile << ' ' << best.lane_stride << ' ' << best.chunk
          << '\n';
    }
    if (out) *out = res;
}

// Patch-size tuner: temporary simulations of the descriptor at every
// candidate patch edge, loaded from the species description on the device.
void autotune_patch(PicSimDesc &d, const PicSpeciesDesc &sp, const PicLaserDesc *l, const int32_t *cand,
                    int ncand, int warm, int steps, const PicAllocator *a, hipStream_t stream,
                    const char *cache, PicTuneResult *out)
{
    if (steps <= 0) steps = 20;
    if (warm < 0) throw Error(PIC_EINVAL, "negative warm-up");
    if (!cand || ncand <= 0) throw Error(PIC_EINVAL, "no candidates");
    const int nd = d.ndim;
    char key[200];
    std::snprintf(key, sizeof(key), "pic-patch nd=%d prec=%d n=%d,%d,%d profile=%d load=%d ppc=%d", nd,
                  d.precision, d.n[0], d.n[1], nd == 3 ? d.n[2] : 1, sp.profile, sp.loading, sp.ppc);
    PicTuneResult res;
    std::memset(&res, 0, sizeof(res));
    if (cache) {
        std::ifstream f(cache);
        std::string line;
        const std::string k(key);
        while (std::getline(f, line)) {
            if (line.compare(0, k.size(), k) != 0 || line.size() <= k.size() || line[k.size()] != ' ') continue;
            int p0, p1, p2, blk;
            if (std::sscanf(line.c_str() + k.size(), "%d %d %d %d", &p0, &p1, &p2, &blk) == 4) {
                PicSimDesc t = d;
                t.patch[0] = p0; t.patch[1] = p1; t.patch[2] = p2;
                t.block = blk;
                std::string why;
                if (validate_desc(t, why) != PIC_OK) break;  // stale entry: tune again
                d = t;
                res.from_cache = 1;
                res.block = blk;
                for (int i = 0; i < 3; ++i) res.patch[i] = d.patch[i];
                if (out) *out = res;
                return;
            }
        }
    }
    double best_ms = -1.0;
    PicSimDesc best = d;
    const int blocks[3] = {256, 512, 1024};
    for (int ci = 0; ci < ncand; ++ci) {
        for (int bi = 0; bi < 3; ++bi) {
            PicSimDesc t = d;
            for (int ax = 0; ax < 3; ++ax) t.patch[ax] = ax < nd ? cand[ci] : 1;
            t.block = blocks[bi];
            std::string why;
            if (validate_desc(t, why) != PIC_OK) break;
            std::unique_ptr<SimBase> sim;
            if (t.precision == 32) sim.reset(new SimImpl<float>(t, a, stream));
            else sim.reset(new SimImpl<double>(t, a, stream));
            sim->add_species(sp);
            sim->particles_init();
            if (l) sim->add_laser(*l);
            if (warm) sim->step(warm);
            hipcheck(hipStreamSynchronize(stream), "sync");
            const auto t0 = std::chrono::steady_clock::now();
            sim->step(steps);
            hipcheck(hipStreamSynchronize(stream), "sync");
            const double ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count() / steps;
            ++res.trials;
            if (best_ms < 0 || ms < best_ms) {
                best_ms = ms;
                best = t;
            }
        }
    }
    if (best_ms < 0) throw Error(PIC_EINVAL, "no candidate patch size fits the grid");
    d = best;
    res.block = d.block;
    res.ms_per_step = best_ms;
    for (int i = 0; i < 3; ++i) res.patch[i] = d.patch[i];
    if (cache) {
        std::ofstream f(cache, std::ios::app);
        f << key << ' ' << d.patch[0] << ' ' << d.patch[1] << ' ' << d.patch[2] << ' ' << d.block << '\n';
    }
    if (out) *out = res;
}

// Grow patch capacities (only ever grows) so that every patch holds both its
// current particles and the count the pending re-binning needs, and copy the
// particles into the new layout.
template <typename T>
void SimImpl<T>::grow_capacity()
{
    hipcheck(hipStreamSynchronize(stream), "sync");
    sync_layout();
    std::vector<int32_t> cur = read_counts(), nxt(npatch);
    hipcheck(hipMemcpyAsync(nxt.data(), newcount_d, sizeof(int32_t) * npatch, hipMemcpyDeviceToHost, stream), "newcount");
    hipcheck(hipStreamSynchronize(stream), "sync");
    // every patch is sized again by the descriptor's rule (capacity_factor
    // times the larger of its current and its new count, never shrinking)
    std::vector<int32_t> need(npatch);
    for (int p = 0; p < npatch; ++p) need[p] = std::max(cur[p], nxt[p]);
    relayout(need);
}

// New layout for the given per-patch needs; the live particles are copied.
template <typename T>
void SimImpl<T>::relayout(const std::vector<int32_t> &need)
{
    SimDev<T> oldv = v;
    SimDev<T> *oldv_d = (SimDev<T> *)alloc.get(sizeof(SimDev<T>));
    hipcheck(hipMemcpyAsync(oldv_d, &oldv, sizeof(oldv), hipMemcpyHostToDevice, stream), "old view");
    std::vector<void *> old;
    try {
        old = layout_particles(need);
    } catch (...) {
        alloc.put(oldv_d);
        throw;
    }
    launch_relayout<T>(oldv_d, view_d, npatch, stream);
    hipcheck(hipGetLastError(), "relayout launch");
    hipcheck(hipStreamSynchronize(stream), "relayout");
    for (void *p : old) alloc.put(p);
    alloc.put(oldv_d);
    ++relayouts;
}

// Re-run the re-binning of the step whose scatter was skipped by the
// capacity check, after growing capacities.  The step is then closed by the
// next close/queue pass of the batch that runs the simulation.
template <typename T>
void SimImpl<T>::recover_pending()
{
    for (int attempt = 0; attempt < 4; ++attempt) {
        grow_capacity();
        SimState s = read_state();
        s.flags &= ~kFlagPending;
        s.active = 1;
        hipcheck(hipMemcpyAsync(&st->flags, &s.flags, sizeof(uint32_t) * 2, hipMemcpyHostToDevice, stream), "flags");
        launch_rebin<T>(view_d, 1, prefix_d, npatch, std::min(npatch, 4 * cu_count()), nd, stream);
        hipcheck(hipGetLastError(), "rebin launch");
        s = read_state();
        if (!(s.flags & kFlagPending)) return;
    }
    throw Error(PIC_EOVERFLOW, "patch capacity could not be grown enough");
}

template <typename T>
void SimImpl<T>::rebin_codes(const uint8_t *codes_h, size_t cnt)
{
    check_free();
    auto c = read_counts();
    const int64_t live = std::accumulate(c.begin(), c.end(), int64_t(0));
    if ((int64_t)cnt != live) throw Error(PIC_EINVAL, "code count must equal the live particle count");
    for (size_t k = 0; k < cnt; ++k)
        if (codes_h[k] >= ndir && codes_h[k] != kRemoved) throw Error(PIC_EINVAL, "bad direction code");
    std::vector<int64_t> poff(npatch + 1, 0);
    for (int p = 0; p < npatch; ++p) poff[p + 1] = poff[p] + c[p];
    uint8_t *pk = (uint8_t *)alloc.get(std::max<size_t>(cnt, 1));
    int64_t *po = (int64_t *)alloc.get(sizeof(int64_t) * (npatch + 1));
    hipcheck(hipMemcpyAsync(pk, codes_h, cnt, hipMemcpyHostToDevice, stream), "codes");
    hipcheck(hipMemcpyAsync(po, poff.data(), sizeof(int64_t) * (npatch + 1), hipMemcpyHostToDevice, stream), "codes off");
    launch_scatter_codes(pk, po, off_d, counts_d, code, npatch, stream);
    hipcheck(hipGetLastError(), "codes launch");
    hipcheck(hipMemsetAsync(moved_d, 1, sizeof(int32_t) * npatch, stream), "moved");
    SimState s = read_state();
    s.active = 1;
    hipcheck(hipMemcpyAsync(&st->active, &s.active, sizeof(uint32_t), hipMemcpyHostToDevice, stream), "active");
    launch_rebin<T>(view_d, 1, prefix_d, npatch, std::min(npatch, 4 * cu_count()), nd, stream);
    hipcheck(hipGetLastError(), "rebin launch");
    s = read_state();
    alloc.put(pk);
    alloc.put(po);
    if (s.flags & kFlagPending) recover_pending();
    // only the re-binning was asked for: the step is not closed
    const uint32_t zero[1] = {0};
    hipcheck(hipMemcpyAsync(&st->active, zero, sizeof(uint32_t), hipMemcpyHostToDevice, stream), "active");
    hipcheck(hipMemcpyAsync(&st->rebinned, zero, sizeof(uint32_t), hipMemcpyHostToDevice, stream), "rebinned");
    hipcheck(hipStreamSynchronize(stream), "sync");
}

template <typename T>
int SimImpl<T>::max_items(int chunk)
{
    if (max_items_cache >= 0 && chunk == chunk_cache) return max_items_cache;
    int64_t m = 0;
    for (int p = 0; p < npatch; ++p) m += (cap_h[p] + chunk - 1) / chunk;
    max_items_cache = (int)std::min<int64_t>(m, INT32_MAX / 2);
    chunk_cache = chunk;
    return max_items_cache;
}

template <typename T>
void SimImpl<T>::check_free()
{
    if (batch) throw Error(PIC_ESTATE, "simulation is a member of a batch");
}

// ---------------------------------------------------------------------------
// timing

Ev2 Timing::pair(int k)
{
    Ev2 r;
    if (!enabled || (only >= 0 && k != only)) return r;
    Ev e;
    e.kind = k;
    auto take = [&](hipEvent_t &ev) {
        if (!pool.empty()) {
            ev = pool.back();
            pool.pop_back();
        } else {
            hipcheck(hipEventCreate(&ev), "event");
        }
    };
    take(e.a);
    take(e.b);
    events.push_back(e);
    r.start = e.a;
    r.stop = e.b;
    return r;
}

void Timing::collect()
{
    for (auto &e : events) {
        float ms = 0.f;
        hipcheck(hipEventSynchronize(e.b), "event sync");
        hipcheck(hipEventElapsedTime(&ms, e.a, e.b), "event time");
        total_ms[e.kind] += ms;
        launches[e.kind] += 1;
        pool.push_back(e.a);
        pool.push_back(e.b);
    }
    events.clear();
}

const char *const Timing::names[kKinds] = {"close_queue", "particles", "maxwell", "rebin"};

// ---------------------------------------------------------------------------
// BatchImpl

template <typename T>
BatchImpl<T>::BatchImpl(hipStream_t s) { stream = s; precision = sizeof(T) == 4 ? 32 : 64; }

template <typename T>
BatchImpl<T>::~BatchImpl()
{
    free_graph();
    if (capture_stream) (void)hipStreamDestroy(capture_stream);
    if (ev_fork) (void)hipEventDestroy(ev_fork);
    if (ev_join) (void)hipEventDestroy(ev_join);
    if (side_stream) (void)hipStreamDestroy(side_stream);
    if (!solo_mode)
        for (auto *m : members) m->batch = nullptr;
    free_tables();
}

// The second stream (default priority) and the two events that order it.
template <typename T>
bool BatchImpl<T>::ensure_side()
{
    if (side_stream) return true;
    if (side_failed) return false;
    if (hipStreamCreateWithFlags(&side_stream, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&ev_fork, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&ev_join, hipEventDisableTiming) != hipSuccess) {
        if (side_stream) (void)hipStreamDestroy(side_stream);
        if (ev_fork) (void)hipEventDestroy(ev_fork);
        if (ev_join) (void)hipEventDestroy(ev_join);
        side_stream = nullptr;
        ev_fork = ev_join = nullptr;
        side_failed = true;
        (void)hipGetLastError();
        return false;
    }
    return true;
}

template <typename T>
void BatchImpl<T>::free_graph()
{
    if (graph_exec) (void)hipGraphExecDestroy(graph_exec);
    graph_exec = nullptr;
}

// Capture kGraphSteps step passes into a graph on a private stream (a null
// stream cannot be captured); the graph is replayed on the batch's stream.
// Kernel arguments are the batch tables, so the graph lives until they are
// rebuilt.  On any capture failure graphs are switched off for the batch.
template <typename T>
bool BatchImpl<T>::capture_graph()
{
    if (graph_failed) return false;
    if (!capture_stream) {
        if (hipStreamCreateWithFlags(&capture_stream, hipStreamNonBlocking) != hipSuccess) {
            capture_stream = nullptr;
            graph_failed = true;
            return false;
        }
    }
    hipStream_t user = stream;
    stream = capture_stream;
    hipGraph_t g = nullptr;
    bool ok = hipStreamBeginCapture(capture_stream, hipStreamCaptureModeThreadLocal) == hipSuccess;
    if (ok) {
        try {
            for (int k = 0; k < kGraphSteps; ++k) launch_one_step();
        } catch (...) {
            ok = false;
        }
        ok = (hipStreamEndCapture(capture_stream, &g) == hipSuccess) && ok && g;
    }
    stream = user;
    if (ok) ok = hipGraphInstantiate(&graph_exec, g, nullptr, nullptr, 0) == hipSuccess;
    if (g) (void)hipGraphDestroy(g);
    (void)hipGetLastError();
    if (!ok) {
        graph_exec = nullptr;
        graph_failed = true;
    }
    return ok;
}

template <typename T>
void BatchImpl<T>::free_tables()
{
    free_graph();
    for (void *p : table_bufs) {
        if (p) (void)hipFree(p);
    }
    table_bufs.clear();
    sims_d = nullptr;
    patch_prefix_d = tile_prefix_d = nullptr;
    det_list_d = nullptr;
    det_prefix_d = nullptr;
    ndet = 0;
    det_nodes = 0;
    items_d = nullptr;
    stamps_d = nullptr;
    nitems_d = head_d = stamp_n_d = nullptr;
    qscratch_d = nullptr;
    table_cap_items = 0;
}

template <typename T>
void BatchImpl<T>::add(SimImpl<T> *s, int64_t nsteps)
{
    if (s->batch) throw Error(PIC_ESTATE, "simulation already in a batch");
    if (s->stream != stream) throw Error(PIC_EINVAL, "simulation and batch must share a stream");
    if (nd && s->nd != nd) throw Error(PIC_EINVAL, "simulation and batch differ in dimensions");
    SimState st = s->read_state();
    st.steps_left = nsteps;
    hipcheck(hipMemcpyAsync(&s->st->steps_left, &st.steps_left, sizeof(int64_t), hipMemcpyHostToDevice, stream), "budget");
    hipcheck(hipStreamSynchronize(stream), "sync");
    s->batch = this;
    members.push_back(s);
    nd = s->nd;
    dirty = true;
}

template <typename T>
void BatchImpl<T>::remove(SimImpl<T> *s)
{
    auto it = std::find(members.begin(), members.end(), s);
    if (it == members.end()) throw Error(PIC_EINVAL, "not a member");
    hipcheck(hipStreamSynchronize(stream), "sync");
    int64_t zero = 0;
    hipcheck(hipMemcpyAsync(&s->st->steps_left, &zero, sizeof(zero), hipMemcpyHostToDevice, stream), "budget");
    hipcheck(hipStreamSynchronize(stream), "sync");
    s->batch = nullptr;
    members.erase(it);
    dirty = true;
}

template <typename T>
void BatchImpl<T>::build_tables()
{
    hipcheck(hipStreamSynchronize(stream), "sync");
    const int ns = (int)members.size();
    std::vector<int> pp(ns + 1, 0), tp(ns + 1, 0);
    tile_preset = 0;
    for (auto *m : members) if (m->desc.field_tile) tile_preset = m->desc.field_tile;
    hi_order = yee_any = false;
    for (auto *m : members) {
        hi_order = hi_order || m->desc.maxwell_order == 6;
        yee_any = yee_any || m->desc.maxwell_order != 6;
    }
    int tx, ty;
    maxwell_tile<T>(tile_preset, tx, ty);
    maxP0 = maxP1 = maxP2 = 1;
    int64_t items = 0;
    int64_t particles = 0;
    if (ns > kMaxBatch) throw Error(PIC_EINVAL, "too many simulations in one batch");
    for (int i = 0; i < ns; ++i) {
        SimImpl<T> *m = members[i];
        pp[i + 1] = pp[i] + m->npatch;
        // Yee tiles: TX x TY node tiles in 2-D, blocks of nodes in 3-D
        const int ntiles = nd == 3 ? (int)maxwell3d_tiles(m->fn, m->desc.maxwell_order)
                                   : ((m->fn[0] + tx - 1) / tx) * ((m->fn[1] + ty - 1) / ty);
        tp[i + 1] = tp[i] + ntiles;
        const int own[2] = {0, ntiles};
        hipcheck(hipMemcpyAsync(m->tprefix_d, own, sizeof(own), hipMemcpyHostToDevice, stream), "tile count");
        maxP0 = std::max(maxP0, m->P[0]);
        maxP1 = std::max(maxP1, m->P[1]);
        maxP2 = std::max(maxP2, m->P[2]);
        particles += m->num_particles();
    }
    total_patches = pp[ns];
    total_tiles = tp[ns];
    // a common patch size selects a kernel compiled for it: square 16 or 32
    // in 2-D, 8 x 8 x 8 or 8 x 8 x 4 in 3-D
    patch_const = 0;
    if (nd == 2 && ns > 0 && (members[0]->P[0] == 16 || members[0]->P[0] == 32)) {
        patch_const = members[0]->P[0];
        for (auto *m : members)
            if (m->P[0] != patch_const || m->P[1] != patch_const) patch_const = 0;
    }
    if (nd == 3 && ns > 0) {
        patch_const = particles3d_shape(members[0]->P[0], members[0]->P[1], members[0]->P[2]);
        for (auto *m : members)
            if (particles3d_shape(m->P[0], m->P[1], m->P[2]) != patch_const ||
                m->P[0] != members[0]->P[0] || m->P[1] != members[0]->P[1] || m->P[2] != members[0]->P[2])
                patch_const = 0;
    }
    // chunk: enough items to fill every CU several times over, at most 4096
    // particles in 2-D (laser box: 4096 beat 8192 and 16384) and 16384 in 3-D
    // (blob box: one item per 8^3 patch saves the per-item staging, flush and
    // deferred-list batches; 22.0 ms per launch against 22.7 ms at 4096)
    chunk = 0;
    for (auto *m : members) chunk = std::max(chunk, (int)m->desc.chunk);
    if (chunk == 0) {
        const int64_t target = (int64_t)cu_count() * 8;
        int64_t c = particles / std::max<int64_t>(target, 1);
        c = std::max<int64_t>(c, 256);
        c = std::min<int64_t>(c, nd == 3 ? 16384 : 4096);
        chunk = (int)c;
    }
    for (auto *m : members) items += m->max_items(chunk);
    items = std::max<int64_t>(items, 1);
    use_graph = false;
    for (auto *m : members) use_graph = use_graph || m->desc.graph;
    block = (sizeof(T) == 8 && nd == 2) ? 1024 : 512;
    for (auto *m : members) if (m->desc.block) block = m->desc.block;
    const int occ = std::max(1, nd == 3 ? particles3d_occupancy<T>(block, maxP0, maxP1, maxP2, patch_const)
                                        : particles_occupancy<T>(block, maxP0, maxP1));
    grid_particles = cu_count() * occ;
    grid_maxwell = std::max(1, std::min(total_tiles, cu_count() * (nd == 3 ? 32 : 8)));
    grid_rebin = std::max(1, std::min(total_patches, cu_count() * 8));
    if (std::getenv("PIC_LOG"))
        std::fprintf(stderr,
                     "[pic] batch of %d: %d patches, %lld items of <= %d particles, particle kernel "
                     "block %d x grid %d (%d per CU), shape %d, Yee grid %d, re-binning grid %d\n",
                     ns, total_patches, (long long)items, chunk, block, grid_particles, occ, patch_const,
                     grid_maxwell, grid_rebin);

    // device tables (hipMalloc directly: small, batch-owned)
    free_tables();
    auto get = [&](size_t bytes) {
        void *p = nullptr;
        hipcheck(hipMalloc(&p, std::max<size_t>(bytes, 256)), "batch tables");
        table_bufs.push_back(p);
        return p;
    };
    sims_d = (SimDev<T> *)get(sizeof(SimDev<T>) * std::max(ns, 1));
    std::vector<int> dl;
    std::vector<int64_t> dp(1, 0);
    for (int i = 0; i < ns; ++i)
        if (members[i]->desc.deterministic) {
            dl.push_back(i);
            dp.push_back(dp.back() + members[i]->fsize);
        }
    ndet = (int)dl.size();
    det_nodes = dp.back();
    det_list_d = (int *)get(sizeof(int) * std::max(ndet, 1));
    det_prefix_d = (int64_t *)get(sizeof(int64_t) * (ndet + 1));
    if (ndet) {
        hipcheck(hipMemcpyAsync(det_list_d, dl.data(), sizeof(int) * ndet, hipMemcpyHostToDevice, stream), "det list");
        hipcheck(hipMemcpyAsync(det_prefix_d, dp.data(), sizeof(int64_t) * (ndet + 1), hipMemcpyHostToDevice, stream),
                 "det prefix");
    }
    patch_prefix_d = (int *)get(sizeof(int) * (ns + 1));
    tile_prefix_d = (int *)get(sizeof(int) * (ns + 1));
    items_d = (Item *)get(sizeof(Item) * items);
    stamps_d = (ItemStamp *)get(sizeof(ItemStamp) * items);
    nitems_d = (int *)get(sizeof(int) * 4);
    head_d = nitems_d + 1;
    stamp_n_d = nitems_d + 2;
    qscratch_d = (int *)get(sizeof(int) * kQueueScratch);
    table_cap_items = (int)items;
    std::vector<SimDev<T>> views(ns);
    for (int i = 0; i < ns; ++i) {
        views[i] = members[i]->v;
        seen_version.resize(ns);
        seen_version[i] = members[i]->layout_version;
    }
    if (ns) hipcheck(hipMemcpyAsync(sims_d, views.data(), sizeof(SimDev<T>) * ns, hipMemcpyHostToDevice, stream), "views");
    hipcheck(hipMemcpyAsync(patch_prefix_d, pp.data(), sizeof(int) * (ns + 1), hipMemcpyHostToDevice, stream), "prefix");
    hipcheck(hipMemcpyAsync(tile_prefix_d, tp.data(), sizeof(int) * (ns + 1), hipMemcpyHostToDevice, stream), "prefix");
    hipcheck(hipMemsetAsync(nitems_d, 0, sizeof(int) * 4, stream), "nitems");
    hipcheck(hipStreamSynchronize(stream), "sync");
    dirty = false;
}

template <typename T>
void BatchImpl<T>::refresh_member_views()
{
    bool changed = false;
    for (size_t i = 0; i < members.size(); ++i) {
        if (seen_version[i] != members[i]->layout_version) {
            hipcheck(hipMemcpyAsync(sims_d + i, &members[i]->v, sizeof(SimDev<T>), hipMemcpyHostToDevice, stream), "view");
            seen_version[i] = members[i]->layout_version;
            changed = true;
        }
    }
    if (changed) {
        // capacities grew: the item buffer may need to be larger
        int64_t items = 0;
        for (auto *m : members) items += m->max_items(chunk);
        if (items > table_cap_items) dirty = true;
    }
}

template <typename T>
QueueArgs BatchImpl<T>::queue_args() const
{
    QueueArgs qa;
    qa.nsims = (int)members.size();
    qa.patch_prefix = patch_prefix_d;
    qa.tile_prefix = tile_prefix_d;
    qa.items = items_d;
    qa.nitems = nitems_d;
    qa.head = head_d;
    qa.max_items = table_cap_items;
    qa.chunk = chunk;
    qa.total_patches = total_patches;
    qa.scratch = qscratch_d;
    return qa;
}

// Close whatever steps are complete and queue the next one.
template <typename T>
void BatchImpl<T>::launch_close_queue_pass()
{
    // merges, then window jumps, of the steps that close in this pass
    for (size_t i = 0; i < members.size(); ++i)
        if (members[i]->merge_every > 0 && members[i]->cap_d)
            launch_merge<T>(sims_d + i, members[i]->npatch, 0, 0, 0, members[i]->merge_cmax, stream);
    for (size_t i = 0; i < members.size(); ++i)
        if (members[i]->win_on && members[i]->cap_d)
            launch_window<T>(sims_d + i, members[i]->fn[1], members[i]->np[1], stream);
    launch_close_queue<T>(sims_d, queue_args(), stream, timing().pair(0));
    hipcheck(hipGetLastError(), "queue launch");
}

// One step pass: particles, Yee, re-binning, then close + next queue.
template <typename T>
void BatchImpl<T>::launch_one_step()
{
    const int ns = (int)members.size();
    Timing &tm = timing();
    ItemStamp *stamps = tm.stamp ? stamps_d : nullptr;
    if (stamps) launch_copy_int(nitems_d, stamp_n_d, stream);
    if (nd == 3)
        launch_particles3d<T>(sims_d, items_d, nitems_d, head_d, grid_particles, block, maxP0, maxP1,
                              maxP2, patch_const, stamps, stream, tm.pair(1));
    else
        launch_particles<T>(sims_d, items_d, nitems_d, head_d, grid_particles, block, maxP0, maxP1,
                            patch_const, stamps, stream, tm.pair(1));
    // deterministic members: fixed-point accumulators -> J[step & 1]
    if (ndet) launch_jfix<T>(sims_d, det_list_d, det_prefix_d, ndet, det_nodes, stream);
    // the field update (fields, currents, tile energies) and the re-binning
    // (particles, counts) touch disjoint data: run them side by side
    const bool fork = ensure_side();
    hipStream_t fs = stream;
    if (fork) {
        hipcheck(hipEventRecord(ev_fork, stream), "fork");
        hipcheck(hipStreamWaitEvent(side_stream, ev_fork, 0), "fork");
        fs = side_stream;
    }
    if (nd == 3)
        launch_maxwell3d<T>(sims_d, ns, tile_prefix_d, total_tiles, grid_maxwell, yee_any, hi_order, fs,
                            tm.pair(2));
    else
        launch_maxwell<T>(sims_d, ns, tile_prefix_d, total_tiles, grid_maxwell, tile_preset, yee_any, hi_order,
                          fs, tm.pair(2));
    if (fork) hipcheck(hipEventRecord(ev_join, side_stream), "join");
    launch_rebin<T>(sims_d, ns, patch_prefix_d, total_patches, grid_rebin, nd, stream, tm.pair(3));
    if (fork) hipcheck(hipStreamWaitEvent(stream, ev_join, 0), "join");
    launch_close_queue_pass();
}

template <typename T>
Timing &BatchImpl<T>::timing()
{
    // a batch of one reports into its simulation; larger batches into the first member
    return members.empty() ? own_timing : members[0]->timing;
}

// Run up to max_steps step passes; each member advances while it has budget.
// Returns the number of members that used up their budget in this call.
template <typename T>
int BatchImpl<T>::run(int64_t max_steps, bool until_done)
{
    if (members.empty()) return 0;
    if (dirty) build_tables();
    std::vector<int64_t> before(members.size());
    int64_t budget = 0;  // largest remaining step budget among the members
    for (size_t i = 0; i < members.size(); ++i) {
        SimState s = members[i]->read_state();
        before[i] = s.steps_left;
        if (!(s.flags & kFlagErrMask)) budget = std::max(budget, s.steps_left);
    }
    int64_t launched = 0;
    const int64_t K = kGraphSteps;
    int finished = 0;
    launch_close_queue_pass();  // queue of the first step
    for (;;) {
        // never launch more passes than the largest budget still needs
        int64_t todo = std::min<int64_t>(K, budget);
        if (!until_done) todo = std::min<int64_t>(todo, max_steps - launched);
        if (todo <= 0) break;
        bool replayed = false;
        if (todo == kGraphSteps && use_graph && !timing().enabled) {
            if (graph_exec || capture_graph()) {
                hipcheck(hipGraphLaunch(graph_exec, stream), "graph launch");
                replayed = true;
            }
        }
        if (!replayed)
            for (int64_t k = 0; k < todo; ++k) launch_one_step();
        launched += todo;
        // poll member states
        bool any_left = false;
        bool recovered = false;
        budget = 0;
        for (size_t i = 0; i < members.size(); ++i) {
            SimImpl<T> *m = members[i];
            SimState s = m->read_state();
            if (s.flags & kFlagPending) {
                m->recover_pending();
                recovered = true;
            }
            if (s.steps_left > 0 && !(s.flags & kFlagErrMask)) {
                any_left = true;
                budget = std::max(budget, s.steps_left);
            }
        }
        if (recovered) {
            refresh_member_views();
            if (dirty) build_tables();
            // close the recovered steps and queue the next step for everyone
            launch_close_queue_pass();
            budget = 0;
            any_left = false;
            for (auto *m : members) {
                SimState s = m->read_state();
                if (s.steps_left > 0 && !(s.flags & kFlagErrMask)) {
                    any_left = true;
                    budget = std::max(budget, s.steps_left);
                }
            }
        }
        if (!any_left) break;
        if (!until_done && launched >= max_steps) break;
    }
    for (size_t i = 0; i < members.size(); ++i) {
        SimState s = members[i]->read_state();
        if (before[i] > 0 && (s.steps_left == 0 || (s.flags & kFlagErrMask))) ++finished;
    }
    return finished;
}

template <typename T>
void BatchImpl<T>::finished(std::vector<SimBase *> &out)
{
    for (auto *m : members) {
        SimState s = m->read_state();
        if (s.steps_left == 0 || (s.flags & kFlagErrMask)) out.push_back(m);
    }
}

template struct SimImpl<float>;
template struct SimImpl<double>;
template struct BatchImpl<float>;
template struct BatchImpl<double>;

}  // namespace pic
