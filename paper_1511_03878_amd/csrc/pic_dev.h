// Device-side data layout and shared device helpers of the patch-PIC library.
//
// Layout in HBM (per simulation):
//  - fields: one array per component (two buffers of Ex Ey Ez Bx By Bz, and two
//    J buffers of three components), row-major with x fastest, fn[a] nodes per axis;
//  - particles: structure of arrays (local position per axis, u_x, u_y, u_z,
//    weight, 64-bit id, 1-byte destination code) grouped by patch: patch p owns
//    slots [off[p], off[p] + cap[p]) of every array and uses the first count[p];
//    positions are offsets from the patch origin in cell units;
//  - re-binning scratch with the same per-patch layout: a staging copy of the
//    particle arrays for leavers and a list of vacated slots;
//  - a small state block (step counter, remaining step budget, sticky flags,
//    energy accumulators) and an energy-history ring.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pic {

constexpr int kMaxPatch = 64;      // cells per patch per axis
constexpr int kHistLen = 4096;     // energy-history ring length
constexpr int kMaxBatch = 2048;    // simulations per batch
constexpr int kMaxLasers = 4;      // Gaussian lasers per simulation
constexpr int kNDir2 = 9;          // neighbour directions in 2-D (4 = stay)
constexpr int kStay2 = 4;
constexpr int kNDir3 = 27;         // neighbour directions in 3-D (13 = stay)
constexpr int kStay3 = 13;
// neighbour-table entries per patch: nd keys, the number of distinct source
// patches, up to nd - 1 sources and the key each of them stages under
constexpr int nb_stride(int nd) { return nd + 1 + 2 * (nd - 1); }
constexpr int kNbStride = nb_stride(kNDir2);
constexpr uint8_t kRemoved = 255;

// sticky state flags
constexpr uint32_t kFlagPending = 1u;  // a patch overflowed: re-binning of the last step not applied
constexpr uint32_t kFlagNaN = 2u;      // non-finite momentum
constexpr uint32_t kFlagCFL = 4u;      // a particle moved a cell or more
constexpr uint32_t kFlagWin = 8u;      // a window jump found a patch too small for its injected particles
constexpr uint32_t kFlagErrMask = kFlagNaN | kFlagCFL | kFlagWin;

struct SimState {
    int64_t step;        // completed steps
    int64_t steps_left;  // step budget; kernels skip the simulation at 0
    uint32_t flags;
    uint32_t active;     // set by the queue kernel for the step in flight
    int64_t removed;
    int64_t pushed;      // particles pushed in the step in flight
    double U, K;         // energies of the last completed step
    uint32_t rebinned;   // the step in flight has applied its re-binning
    uint32_t pad;
    // moving window
    int64_t next_id;     // id of the next injected particle
    int64_t wshift;      // window jumps done (each one patch column)
    int64_t wadd;        // particles injected by the jump of the step in flight
    uint32_t wpend;      // the step in flight jumped (applied when the step closes)
    uint32_t pad2;
    int64_t merged;      // particles taken out by merging so far
    uint64_t wmax_bits;  // bound on |weight| of every particle (FP64 bits; set at load, raised by
                         // merging and window injection)
};

template <typename T>
struct SimDev {
    int n[3], P[3], np[3], fn[3], periodic[3];
    int npatch;
    int ndim;
    int lane_stride;   // particles between consecutive lanes of a wave
    int morder;        // field solver order: 2 (Yee) or 6
    // moving window (2-D, open x): jumps of P[0] cells, cold lattice injection
    int win;           // 1: the window moves
    int wppc[2];       // injected particles per cell along x, y
    int64_t wstart;    // completed steps before the window starts
    double wvel, wdt, wdx;  // speed (units of c), time step and cell size along x, in FP64
    const double *wdens;    // density per global cell column (the last entry continues)
    int64_t wncols;
    // particle merging (2-D): after every mevery-th step (0: never)
    int mevery, mcmax, miters;
    T d[3];
    T dt;
    T q, m;
    double vcell;
    // fields: two buffers of E, B (the step's input is F[step & 1], the Yee
    // update writes F[(step + 1) & 1], so no tile reads a halo another tile
    // has already advanced) and two current buffers (deposit into J[step & 1])
    T *F[2][6];
    T *J[2][3];
    // deterministic deposition: the particle kernel adds its current tiles to
    // these fixed-point accumulators (integer sums do not depend on order);
    // a conversion pass turns them into J[step & 1] and clears them
    int det;
    int64_t *Jacc[3];
    // particles, slot k: position pos[pw k + a] (pw = 2 in 2-D: x, y; pw = 4
    // in 3-D: x, y, z and the id, see pad_id), momentum and weight
    // mom[4 k + c] (u_x, u_y, u_z, w), the id in 2-D id[k] (null in 3-D).
    // One particle is two or three short runs of memory, so the re-binning
    // moves it with two (3-D) or three (2-D) scattered accesses instead of
    // one per component.
    T *pos, *mom;
    int pw;
    int64_t *id;
    uint8_t *code;
    // staging copy for leavers (same layout)
    T *spos, *smom;
    int64_t *sid;
    int32_t *holes;
    const int32_t *cap;
    const int64_t *off;
    int32_t *count;
    int32_t *newcount;
    int32_t *kcnt;     // per patch: leavers per canonical direction key (kNDir2)
    int32_t *kofs;     // per patch: ND + 1 entries, the staging offset of each key's leavers, then
                       // the number of staged leavers (the removed ones follow them)
    int32_t *nleave;   // per patch: all leavers (incl. removed)
    int32_t *narrive;  // per patch: arrivals (set by the capacity check)
    int32_t *nhole;    // per patch: vacated slots below the new count
    int32_t *moved;    // per patch: nonzero when a particle may have left since the last re-binning
    const int32_t *porder;  // queue order of the patches (position -> patch id), or null: id order
    const T *laser_ey, *laser_ez;
    int64_t laser_steps;
    // Gaussian lasers through x = 0, evaluated in FP64 every step: a0, omega0,
    // w0, tau, t0, x_focus, y_center, phase; polarisation 1 (Ey) or 2 (Ez)
    int nlaser;
    int las_pol[kMaxLasers];
    double las[kMaxLasers][8];
    double dd[3];      // cell sizes in FP64
    SimState *st;
    double *hist;      // [kHistLen][4]: U, K, pushed, removed
    const int32_t *nbt; // neighbour table, kNbStride entries per patch
    double *upart;     // per Yee tile: field energy of the step in flight
    double *kpart;     // per patch: kinetic energy of the step in flight
};

// ---- small helpers ----------------------------------------------------------

__device__ __forceinline__ int wrap_idx(int i, int n)
{
    i %= n;
    return i < 0 ? i + n : i;
}

// Storage index of node i on an axis, or -1 outside an open axis.  stag = 1
// for dual (half-cell) positions, which exist only up to n-1 on an open axis.
// Callers pass indices within a few nodes of [0, n), so one conditional
// shift replaces the modulo on a periodic axis.
__device__ __forceinline__ int axis_node(int i, int n, int periodic, int stag)
{
    if (periodic) return i < 0 ? i + n : (i >= n ? i - n : i);
    if (i < 0 || i > n - stag) return -1;
    return i;
}

// Neighbour patch of patch p in direction dir (2-D, (dx+1) + 3 (dy+1)), with
// periodic wrap; -1 when it falls off an open axis.
template <typename T>
__device__ __forceinline__ int neighbour2(const SimDev<T> &S, int p, int dir)
{
    int px = p % S.np[0], py = p / S.np[0];
    int qx = px + (dir % 3) - 1, qy = py + (dir / 3) - 1;
    if (qx < 0 || qx >= S.np[0]) {
        if (!S.periodic[0]) return -1;
        qx = wrap_idx(qx, S.np[0]);
    }
    if (qy < 0 || qy >= S.np[1]) {
        if (!S.periodic[1]) return -1;
        qy = wrap_idx(qy, S.np[1]);
    }
    return qx + S.np[0] * qy;
}

// Global-memory view of a device pointer read from a descriptor.  The
// compiler cannot tell the address space of such a pointer and would emit
// flat instructions, which also occupy the LDS counter (so a wait for an LDS
// result waits for every flat load in flight) and need 64-bit lane addresses.
template <typename T>
using gptr_t = __attribute__((address_space(1))) T *;

template <typename T>
__device__ __forceinline__ gptr_t<T> glb(T *p)
{
    return (gptr_t<T>)p;
}

// Relaxed device-scope atomic add on global memory.
// Element i of a global array through a 32-bit byte offset from a uniform
// base: the load or store then takes the base from scalar registers and only
// the offset from a vector register (no 64-bit address arithmetic per lane).
// The caller keeps i * sizeof(T) below 2^32.
template <typename T>
__device__ __forceinline__ gptr_t<T> at(gptr_t<T> base, uint32_t i)
{
    typedef __attribute__((address_space(1))) char gchar;
    return (gptr_t<T>)((gchar *)base + i * (uint32_t)sizeof(T));
}

// A 3-D particle's id in the fourth entry of its position vector, as bits:
// all 64 in FP64 storage, the low 32 in FP32 storage (a 3-D FP32 simulation
// holds fewer than 2^32 particles: the library refuses more).
template <typename T>
__host__ __device__ __forceinline__ T id_pad(int64_t id)
{
    if constexpr (sizeof(T) == 8) return __builtin_bit_cast(T, id);
    else return __builtin_bit_cast(T, (uint32_t)id);
}
template <typename T>
__host__ __device__ __forceinline__ int64_t pad_id(T v)
{
    if constexpr (sizeof(T) == 8) return __builtin_bit_cast(int64_t, v);
    else return (int64_t)__builtin_bit_cast(uint32_t, v);
}

// Two and four consecutive particle components, loaded or stored as one
// access (vector types of the compiler: copies through address-space
// pointers need no constructors).
template <typename T>
using Vec2 = T __attribute__((ext_vector_type(2)));
template <typename T>
using Vec4 = T __attribute__((ext_vector_type(4)));

template <typename T>
__device__ __forceinline__ gptr_t<Vec2<T>> v2(T *p)
{
    return (gptr_t<Vec2<T>>)glb(p);
}
template <typename T>
__device__ __forceinline__ gptr_t<Vec4<T>> v4(T *p)
{
    return (gptr_t<Vec4<T>>)glb(p);
}

template <typename T>
__device__ __forceinline__ void gadd(gptr_t<T> p, T v)
{
    __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Locate the simulation of a global work index through an exclusive prefix
// table of per-simulation work counts (nsims + 1 entries).
__device__ __forceinline__ int find_sim(const int *prefix, int nsims, int g)
{
    int lo = 0, hi = nsims - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (prefix[mid] <= g) lo = mid; else hi = mid - 1;
    }
    return lo;
}


// ---- fixed-point current ---------------------------------------------------
// Current tiles accumulate integers: a contribution c enters as round(c 2^s)
// with 2^(48 - s) above |q| w_max, which bounds every contribution one
// particle makes to one node of one component: Esirkepov's running sum of
// the shape differences along a is the change of a discrete shape CDF whose
// slope is at most one, so it is at most the move d_a in cells, and
// (-q w Delta_a / dt) d_a = -q w v_a with |v_a| < 1; the time-averaged
// transverse weights lie in [0, 1]; the 2-D out-of-plane current is q w v_z
// times such weights.  One item's sum at a node stays below 2^62 for items
// of up to 2^14 particles; the deterministic accumulators hold the sum over
// every particle depositing at a node in one step, below 2^63 while those
// number at most 2^15.  One unit is at most 2^-47 |q| w_max.  The integer of
// a double below 2^51 in magnitude is read from the low mantissa bits of
// v + 1.5 * 2^52 (the addition rounds to nearest).
constexpr double kFixMagic = 6755399441055744.0;  // 1.5 * 2^52
constexpr long long kFixMagicBits = 0x4338000000000000LL;

template <typename T>
__device__ __forceinline__ double fix_scale(const SimDev<T> &S)
{
    const double wmax = __longlong_as_double((long long)glb(S.st)->wmax_bits);
    const double cb = fabs((double)S.q) * wmax;
    if (!(cb > 0.0) || !(cb < 1e300)) return 1.0;
    return ldexp(1.0, 48 - (ilogb(cb) + 1));
}

__device__ __forceinline__ long long to_fix(double c, double scale)
{
    return __double_as_longlong(fma(c, scale, kFixMagic)) - kFixMagicBits;
}

// LDS atomic add of a contribution to a fixed-point tile entry
__device__ __forceinline__ void fix_add(long long *p, double c, double scale)
{
    atomicAdd(reinterpret_cast<unsigned long long *>(p), (unsigned long long)to_fix(c, scale));
}

// The same for a contribution a b whose factors already carry the scale:
// one fused multiply-add rounds the exact product to an integer.
__device__ __forceinline__ void fix_add_prod(long long *p, double a, double b)
{
    const long long v = __double_as_longlong(fma(a, b, kFixMagic)) - kFixMagicBits;
    atomicAdd(reinterpret_cast<unsigned long long *>(p), (unsigned long long)v);
}

// ... and for a b + c d (two roundings to an integer: within one unit)
__device__ __forceinline__ void fix_add_2prod(long long *p, double a, double b, double c, double d)
{
    const long long v = __double_as_longlong(fma(a, b, fma(c, d, kFixMagic))) - kFixMagicBits;
    atomicAdd(reinterpret_cast<unsigned long long *>(p), (unsigned long long)v);
}

// Raise the simulation's weight bound to |w| (FP64 bits of non-negative
// numbers order like the numbers).
template <typename T>
__device__ __forceinline__ void raise_wmax(const SimDev<T> &S, double w)
{
    atomicMax(reinterpret_cast<unsigned long long *>(&S.st->wmax_bits),
              (unsigned long long)__double_as_longlong(fabs(w)));
}

}  // namespace pic
