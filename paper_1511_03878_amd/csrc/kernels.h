// Launch wrappers of the 2-D patch-PIC kernels (defined in the .hip files).
#pragma once

#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include "pic_dev.h"

namespace pic {

// Optional start / stop events of a timed launch: recorded by the dispatch
// itself (hipExtLaunchKernel), so timing adds no packets between kernels.
struct Ev2 {
    hipEvent_t start = nullptr, stop = nullptr;
};

// Workgroups of `func` (block threads, dyn_lds bytes of dynamic LDS) that fit
// on one CU together, from the kernel's own register and LDS use: 512 VGPRs
// per SIMD lane (allocated in granules of 8), 8 wave slots per SIMD, and the
// device's LDS per CU (160 KB on gfx950).  The runtime's occupancy query
// caps LDS lower, so the larger of the two answers sizes persistent grids
// (a workgroup that cannot be resident at once just starts later).
inline int resident_workgroups(const void *func, int block, size_t dyn_lds)
{
    hipFuncAttributes a;
    if (hipFuncGetAttributes(&a, func) != hipSuccess) return 0;
    int dev = 0, lds_cu = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&lds_cu, hipDeviceAttributeMaxSharedMemoryPerMultiprocessor, dev) != hipSuccess)
        return 0;
    const int waves = (block + 63) / 64, per_simd = (waves + 3) / 4;
    const int regs = ((a.numRegs > 0 ? a.numRegs : 1) + 7) / 8 * 8;
    const int by_regs = (512 / regs) / per_simd;
    const size_t lds = dyn_lds + a.sharedSizeBytes;
    const int by_lds = lds ? (int)((size_t)lds_cu / lds) : 64;
    const int by_slots = 32 / waves;
    int n = by_regs < by_lds ? by_regs : by_lds;
    return n < by_slots ? n : by_slots;
}

// Work item of the particle kernel: {simulation slot | parity of the step
// << 30, patch, slot of the item's first particle in the simulation's
// particle arrays, count}.
using Item = int4;
constexpr int kItemSimMask = (1 << 30) - 1;

// Optional per-item record of a particle launch (diagnostics): start and end
// of the item on the device's constant-rate clock, the compute unit that ran
// it (__smid: XCD, shader engine and CU ids), its simulation slot, patch and
// particle count.  Written by thread 0 of the workgroup with vector stores.
struct ItemStamp {
    long long t0, t1;
    int hw, sim, patch, count;
};

__device__ __forceinline__ void record_item(ItemStamp *r, long long t0, int sim, int patch, int count)
{
    ItemStamp v;
    v.t0 = t0;
    v.t1 = wall_clock64();
    v.hw = (int)__smid();
    v.sim = sim;
    v.patch = patch;
    v.count = count;
    *r = v;
}

struct QueueArgs {
    int nsims;
    const int *patch_prefix;  // nsims + 1 entries (global patch numbering)
    const int *tile_prefix;   // nsims + 1 entries (Yee tiles of each simulation)
    Item *items;
    int *nitems;
    int *head;
    int max_items;
    int chunk;                // max particles per item
    int total_patches;        // patch_prefix[nsims]
    // scratch of the grid-wide queue build (kQueueScratch ints): bucket
    // counts, bucket cursors, then one participation word per simulation
    int *scratch;
};
// ints of QueueArgs::scratch (two sets of 1024 buckets and kMaxBatch words)
constexpr int kQueueScratch = 2 * 1024 + kMaxBatch;

// Close the steps whose re-binning was applied (energy reduction, history,
// step counter, budget) and build the work queue of the next step.
template <typename T>
void launch_close_queue(const SimDev<T> *sims, const QueueArgs &q, hipStream_t st, Ev2 ev = {});

// Persistent particle kernel: gather, Boris, move, classify, Esirkepov deposit.
// pc: common square patch size of every simulation in the launch (16 or 32)
// for the specialised kernel, 0 for the general one.
template <typename T>
void launch_particles(const SimDev<T> *sims, const Item *items, const int *nitems, int *head,
                      int grid, int block, int maxP0, int maxP1, int pc, ItemStamp *stamps,
                      hipStream_t st, Ev2 ev = {});
template <typename T>
int particles_occupancy(int block, int maxP0, int maxP1);

// 3-D particle kernel (periodic boxes): 27-node gather, Boris, move, 26-way
// classification, Esirkepov deposit on a 4x4x4 window.  LDS per workgroup:
// particles3d_lds_bytes(precision, largest patch edges).
// shape: particles3d_shape() of the common patch shape of every simulation
// in the launch (1: 8 x 8 x 8, 2: 8 x 8 x 4, compiled with constant tile
// pitches), 0 for the general kernel.
template <typename T>
void launch_particles3d(const SimDev<T> *sims, const Item *items, const int *nitems, int *head,
                        int grid, int block, int maxP0, int maxP1, int maxP2, int shape,
                        ItemStamp *stamps, hipStream_t st, Ev2 ev = {});
template <typename T>
int particles3d_occupancy(int block, int maxP0, int maxP1, int maxP2, int shape);
size_t particles3d_lds_bytes(int precision, int P0, int P1, int P2);
int particles3d_shape(int P0, int P1, int P2);

// 3-D field update on a periodic box, with the field energy of the incoming
// E, B per tile.  Yee: one fused kernel over blocks of kYee3X x kYee3Y x
// kYee3Z nodes, taken plane by plane along z; sixth order: three passes over
// runs of kMaxwell3dTile nodes.
// yee / hi_order: the batch holds simulations of that solver.
template <typename T>
void launch_maxwell3d(const SimDev<T> *sims, int nsims, const int *tile_prefix, int total_tiles,
                      int grid, bool yee, bool hi_order, hipStream_t st, Ev2 ev = {});
constexpr int kMaxwell3dTile = 256;
constexpr int kYee3X = 32, kYee3Y = 8, kYee3Z = 32;
// field-update tiles of a 3-D simulation with fn nodes per axis
inline int64_t maxwell3d_tiles(const int fn[3], int order)
{
    if (order == 6) return ((int64_t)fn[0] * fn[1] * fn[2] + kMaxwell3dTile - 1) / kMaxwell3dTile;
    return (int64_t)((fn[0] + kYee3X - 1) / kYee3X) * ((fn[1] + kYee3Y - 1) / kYee3Y) *
           ((fn[2] + kYee3Z - 1) / kYee3Z);
}

// Moving-window jump of one simulation (2-D): a no-op unless the step in
// flight ends with a jump.  fn1 = field rows, npy = patch rows.
template <typename T>
void launch_window(const SimDev<T> *sim, int fn1, int npy, hipStream_t st);
constexpr int kWindowMaxPatchColumns = 4096;

// Particle merging of one simulation (2-D).  forced = 0: a no-op unless the
// step in flight is a merge step (cmax, iters then come from the simulation);
// forced = 1: merge now with the given cmax (4..32) and iters.
template <typename T>
void launch_merge(const SimDev<T> *sim, int npatch, int cmax, int iters, int forced, int cmax_bound,
                  hipStream_t st);

// Fused Yee update (half B, E, half B) with face conditions; clears the
// other J buffer and accumulates the field energy of the incoming E, B.
// yee: the batch holds simulations with the Yee solver; hi_order: it holds
// simulations with the sixth-order solver, which take three further passes.
template <typename T>
void launch_maxwell(const SimDev<T> *sims, int nsims, const int *tile_prefix, int total_tiles,
                    int grid, int preset, bool yee, bool hi_order, hipStream_t st, Ev2 ev = {});
template <typename T>
void maxwell_tile(int preset, int &tx, int &ty);

// Re-binning: count and stage leavers; check capacity; scatter (ndim 2 or 3:
// 9 or 27 neighbour directions).
template <typename T>
void launch_rebin(const SimDev<T> *sims, int nsims, const int *patch_prefix, int total_patches,
                  int grid, int ndim, hipStream_t st, Ev2 ev = {});

// Copy particles into a new per-patch layout (capacity growth).
template <typename T>
void launch_relayout(const SimDev<T> *src, const SimDev<T> *dst, int npatch, hipStream_t st);

// Fixed-point current (k_current.hip).  launch_wmax raises the simulation's
// weight bound to the largest |w| of its particles (after a load).
// launch_jfix converts the deterministic accumulators of the listed
// simulations into J[step & 1] and clears them (prefix: exclusive prefix of
// their node counts, nlist + 1 entries; total = prefix[nlist]).
template <typename T>
void launch_wmax(const SimDev<T> *sim, int npatch, hipStream_t st);
template <typename T>
void launch_jfix(const SimDev<T> *sims, const int *list, const int64_t *prefix, int nlist, int64_t total,
                 hipStream_t st);

// Diagnostics (k_diag.hip).  fill_doubles clears with a kernel (safe under
// graph capture).  launch_rho adds the particles' charge density on primal
// nodes (2-D or 3-D) into `out` (fn[0] fn[1] fn[2] doubles, cleared by the
// caller).  launch_residuals reduces, over nodes, the Gauss residual
// div E - (rho - rho0), the continuity residual rho - rho_prev + dt div J, and
// the largest |rho| and |rho0|, into out[0..3] (rho0 / rho_prev may be null:
// that entry is then 0); `partials` holds residual_partials() doubles.
void fill_doubles(double *p, int64_t n, double v, hipStream_t st);
template <typename T>
void launch_rho(const SimDev<T> *sim, int npatch, int ndim, double *out, hipStream_t st);
template <typename T>
void launch_residuals(const SimDev<T> *sim, int ndim, int64_t fsize, int fpar, int jpar,
                      const double *rho, const double *rho0, const double *rho_prev,
                      double *partials, double *out, hipStream_t st);
int residual_partials();
// copy *src to *dst on the stream (one thread)
void launch_copy_int(const int *src, int *dst, hipStream_t st);

// Particle loading from a species description (k_init.hip): count the
// particles of every row segment (one grid row inside one patch column,
// nseg = rows x patch columns), then write them into their patch slots
// given each segment's first id and first slot inside its patch.
constexpr int kProfileUniform = 0, kProfileRamp = 1, kProfileCosSphere = 2;
constexpr int kLoadWeight = 0, kLoadCount = 1;
struct InitSpec {
    int profile, loading, ppc, nd;
    int n[3], P[3], np[3];
    double n0, p[6], sigma, d[3];
    uint64_t seed;
};
void launch_init_count(const InitSpec &sp, int64_t nseg, int64_t *seg, hipStream_t st);
template <typename T>
void launch_init_fill(const InitSpec &sp, int64_t nseg, const int64_t *first, const int32_t *slot0,
                      const SimDev<T> *sim, hipStream_t st);

// Set the destination codes of all live particles from a packed host-supplied
// array in (patch, slot) order.
void launch_scatter_codes(const uint8_t *packed, const int64_t *packed_off, const int64_t *off,
                          const int32_t *count, uint8_t *code, int npatch, hipStream_t st);

}  // namespace pic
