/*
 * pic.h -- C ABI of the MI355X patch-PIC library (libpic.so).
 *
 * The library runs the data-parallel hot path of a patch-decomposed
 * electromagnetic particle-in-cell step on one gfx950 GPU: quadratic-shape
 * field gather, relativistic Boris push, charge-conserving (Esirkepov)
 * current deposition, Yee FDTD update with periodic or Silver-Mueller faces,
 * and the per-patch particle re-binning whose cost spread across patches is
 * the load imbalance studied in the paper (Beck, Frederiksen, Derouillat,
 * "Load management strategy for Particle-In-Cell simulations in high energy
 * particle acceleration", sections 3 and 3.1: patches of fields and
 * super-particles, dynamic exchange of patches to even out load).
 *
 * Conventions
 *  - Units: c = eps0 = e = m_e = 1; lengths in c/omega_r, time in
 *    1/omega_r (section 2.2 quotes its resolutions this way).
 *  - Grid: n[a] cells of size d[a] per axis, x fastest.  Field component
 *    arrays exchanged with the host are FP64, row-major with x fastest,
 *    fn[a] nodes per axis: fn = n on a periodic axis, n + 1 on an open axis
 *    (only x may be open).  Yee staggering (half a cell up): Ex (1/2,0,0),
 *    Ey (0,1/2,0), Ez (0,0,1/2), Bx (0,1/2,1/2), By (1/2,0,1/2),
 *    Bz (1/2,1/2,0); J shares E's positions.  In 2-D the z offsets vanish.
 *    On an open x axis the dual-x components use nodes 0..n-1 and entry n
 *    is unused (reads back as 0).
 *  - Time levels: after k completed steps the library holds x^k, u^{k-1/2},
 *    E^k and B^k (B at integer time), and J^{k-1/2} (the last deposit).
 *  - Particles are held in patches of patch[a] cells; a particle's patch is
 *    floor(x/d / patch) per axis, patch id row-major with x fastest.  Inside
 *    a patch particles occupy slots 0..count-1 in a canonical order: the
 *    initial order is id order; after every step the re-binning fills
 *    vacated slots below the new count with arrivals (ordered by source
 *    patch id, then source slot) and then with the stayers beyond the new
 *    count, and appends what remains.  Getters return particles in
 *    (patch, slot) order.
 *  - Status: every int-returning call returns PIC_OK (0) or a negative
 *    PIC_E* code; pic_last_error() gives a thread-local message.  Arguments
 *    are validated before any device work, so bad descriptors fail without
 *    touching the GPU.  No C++ exception crosses this interface.
 *  - Host pointers are borrowed for the duration of the call only.  Device
 *    memory is owned by the handle and obtained through the allocator hook
 *    given at creation (NULL: hipMalloc / hipFree).
 *  - All device work of a handle is ordered on the HIP stream given at
 *    creation (NULL: the default stream).  Handles are not thread-safe.
 */
#ifndef PIC_H
#define PIC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    PIC_OK = 0,
    PIC_EINVAL = -1,    /* invalid argument or descriptor */
    PIC_ENOMEM = -2,    /* allocation through the hook failed */
    PIC_EBUDGET = -3,   /* a memory budget would be exceeded */
    PIC_EHIP = -4,      /* a HIP runtime call failed */
    PIC_EOVERFLOW = -5, /* patch capacity could not be grown */
    PIC_ENAN = -6,      /* a particle produced a non-finite momentum */
    PIC_ECFL = -7,      /* a particle moved one cell or more in a step */
    PIC_ESTATE = -8,    /* call not valid in the handle's current state */
    PIC_ENOTSUP = -9    /* configuration not supported by this build */
};

/* Field component ids for pic_fields_set / pic_fields_get. */
enum {
    PIC_EX = 0, PIC_EY = 1, PIC_EZ = 2,
    PIC_BX = 3, PIC_BY = 4, PIC_BZ = 5,
    PIC_JX = 6, PIC_JY = 7, PIC_JZ = 8,
    PIC_RHO = 9 /* charge density q sum_p w_p prod_a S2(xi_p,a - node_a) of the particles on
                   primal nodes, FP64, 2-D and 3-D (get only) */
};

typedef struct PicSim PicSim;
typedef struct PicBatch PicBatch;

/* Device-memory hook: alloc returns device memory of at least `bytes`
 * (256-byte aligned) or NULL; free releases it.  Called only from the
 * creating thread.  Python routes these to torch's caching allocator. */
typedef struct {
    void *(*alloc)(size_t bytes, void *ctx);
    void (*free)(void *ptr, void *ctx);
    void *ctx;
} PicAllocator;

/* Simulation descriptor.  One electron-like species per simulation
 * (immobile neutralising ions enter only diagnostics). */
typedef struct {
    int32_t ndim;          /* 2 or 3 (3-D boxes are periodic on every axis) */
    int32_t precision;     /* 32 or 64: storage and arithmetic of fields and particles */
    int32_t n[3];          /* cells per axis, at least 4 (n[2] ignored in 2-D) */
    double d[3];           /* cell size per axis */
    double dt;             /* time step; must satisfy dt < (sum 1/d^2)^(-1/2) */
    int32_t patch[3];      /* cells per patch per axis; must divide n; at most 64 */
    int32_t periodic[3];   /* 1 periodic; 0 open: Silver-Mueller fields, absorbing
                              particles (x axis only) */
    double q, m;           /* species charge and mass */
    double capacity_factor;/* slots per patch = max(min_capacity, factor * count); 0 = 3 */
    int32_t min_capacity;  /* 0 = the mean patch occupancy (at least 64) */
    int32_t chunk;         /* max particles per work item, at most 16384; 0 = chosen from the load */
    int32_t block;         /* threads per particle workgroup: 256, 512 or 1024; 0 = 512 (FP32) / 1024 (FP64) */
    int32_t field_tile;    /* Yee tile shape preset 0..5 (0 = default for the precision) */
    int32_t lane_stride;   /* particles between adjacent lanes of the particle kernel, 1..64;
                              0 = 2 in 2-D, 4 in 3-D */
    int32_t graph;         /* 1: step in batches of 32 replayed from a captured HIP graph
                              (when kernel timing is off); 0: plain launches */
    int32_t patch_order;   /* order of equal-size work items: 0 = patch id; 1 = the Hilbert
                              curve of pic_patch_order (power-of-two patch grids only) */
    int32_t maxwell_order; /* field solver: 0 or 2 = Yee (second order, Sec. 2.1); 6 = staggered
                              differences of sixth order on the same grid (every axis periodic,
                              dt < (sum_m |c_m|)^(-1) (sum 1/d^2)^(-1/2) with
                              c = 75/64, -25/384, 3/640) */
    int32_t deterministic; /* 1: currents are summed in 64-bit fixed point across work items
                              (integer atomics), so a run repeats bit for bit and gives the same
                              bits alone and in a batch; needs 24 more bytes per field node and
                              holds while at most 32768 particles deposit at one node in a step.
                              0: work items add their current tiles
                              through float atomics (faster; summation order varies at the
                              rounding level).  The paper does not treat summation order. */
} PicSimDesc;

/* Diagnostics of a simulation (pic_diag_get synchronises the stream). */
typedef struct {
    int64_t step;          /* completed steps */
    int64_t particles;     /* live particles */
    int64_t removed;       /* particles absorbed at open faces so far */
    double field_energy;   /* U(E^{k-1}, B^{k-1}) of the last completed step */
    double kinetic_energy; /* K^{k-1} = sum w m (gamma^{k-3/2} + gamma^{k-1/2}) / 2 - 1) V_cell */
    int32_t occupancy_min, occupancy_max; /* particles per patch */
    double occupancy_mean;
    int32_t flags;         /* sticky device error bits (see pic_sync) */
    int32_t relayouts;     /* capacity re-layouts performed so far */
    int64_t window_cells;  /* cells the moving window has travelled (0 without one) */
    int64_t merged;        /* particles taken out by merging so far */
    int64_t device_bytes;  /* device memory the handle holds now (grows with patch capacity) */
} PicDiag;

/* Residuals of the discrete conservation laws (pic_residuals).  The paper
 * states none; they check the charge-conserving deposition and the Yee
 * update on the device's own state, in FP64, at primal nodes (div E and
 * div J are backward differences of the staggered E and J):
 *   gauss      = max |div E^k - (rho^k - rho^0)| / max |rho^0|, where rho^0 is
 *                the particles' charge density when they were loaded (the
 *                immobile neutralising ions carry -rho^0); NaN after a
 *                checkpoint load (the load-time charge is not saved);
 *   continuity = max |rho^k - rho^{k-1} + dt div J^{k-1/2}| / max |rho^k|,
 *                defined only when the previous pic_residuals call on this
 *                handle was made one step earlier (else NaN).
 * Each ratio falls back to the plain maximum when its denominator is 0.
 * Nodes within three cells of an open x face are left out (an absorbed
 * particle takes its charge with it after depositing its whole move).  Merging changes the node charge of the cells it touches,
 * so the Gauss residual is meaningful only before the first merge. */
typedef struct {
    int64_t step;          /* k: completed steps of the state examined */
    double gauss;
    double continuity;
    double rho_max;        /* max |rho^k| */
    double rho0_max;       /* max |rho^0| (NaN when unknown) */
} PicResiduals;

/* Per-kernel timing accumulated while timing is enabled (HIP events on the
 * handle's stream around every launch). */
typedef struct {
    int32_t nkernels;
    const char *name[8];
    double total_ms[8];
    int64_t launches[8];
} PicTiming;

/* ---- lifetime ---------------------------------------------------------- */

/* Create a simulation: allocate E, B (zero) and two J buffers on the device.
 * `d` is validated (ndim, precision, divisibility, CFL, open axes) before
 * any device call.  *out receives the handle. */
int pic_sim_create(const PicSimDesc *d, const PicAllocator *a, void *hip_stream, PicSim **out);
void pic_sim_destroy(PicSim *s);

/* ---- state in ------------------------------------------------------------ */

/* Load n particles given in id order (ids 0..n-1): positions in cell units
 * (x/d, global, each in [0, n_cells)), momenta u = p/(m c) at time -1/2,
 * weights (density contributed, in units of the reference density).  z and
 * uz may be NULL in 2-D (uz NULL = 0).  Replaces any previous particles and
 * resets the step counter to 0.  Values are rounded to the handle's
 * precision; positions are stored as offsets from their patch origin.  A 3-D
 * FP32 handle holds fewer than 2^32 particles (its ids are stored in 32 bits):
 * PIC_EINVAL for more, as for pic_particles_init. */
int pic_particles_set(PicSim *s, int64_t n, const double *x, const double *y, const double *z,
                      const double *ux, const double *uy, const double *uz, const double *w);

/* ---- species and lasers -------------------------------------------------- */

/* The paper sets up its runs by laser and plasma parameters (section 2.2: a
 * Gaussian pulse of given a0, waist and duration focused at the foot of a
 * density ramp; section 3: a plasma whose super-particle density follows the
 * density).  These calls load the species and drive the laser from such
 * descriptions, on the device.
 *
 * Density profiles (lengths in c/omega_r, densities in n_r):
 *   PIC_PROFILE_UNIFORM     n0 everywhere;
 *   PIC_PROFILE_RAMP        0 below x0 = param[0], rising linearly to n0 at
 *                           x1 = param[1], n0 beyond (cells whose lower x face
 *                           is at or beyond x0 hold plasma);
 *   PIC_PROFILE_COS_SPHERE  n0 (1 + param[0] cos(2 pi x / L_x)), and
 *                           param[5] n0 inside the sphere of centre
 *                           (param[1], param[2], param[3]) and radius param[4]
 *                           (evaluated at cell centres).
 * Loading rules: PIC_LOAD_WEIGHT puts ppc particles in every plasma cell with
 * weight n / ppc (n at the particle for the ramp, at the cell centre
 * otherwise); PIC_LOAD_COUNT puts round(ppc n / n0) particles in a cell with
 * weight n0 / ppc (super-particle count follows the density, as in the
 * paper's 3-D runs, section 3).
 * Particles are generated cell by cell in row-major order (x fastest), k =
 * 0 .. count - 1 in a cell; that order is the id order.  Random numbers come
 * from SplitMix64 (Steele, Lea and Flood, OOPSLA 2014) in counter form: draw
 * d of particle g in stream r is output r 2^44 + 8 g + d of the generator
 * seeded with `seed`, and a uniform double is its top 53 bits times 2^-53.
 * Stream 0: position on axis a = cell index + draw a (kept below the cell's
 * upper face).  Stream 1: momenta, every component Gaussian with
 * sigma = sqrt(temperature) by Box-Muller (radius from 1 - draw 0 and 1 -
 * draw 2, angles 2 pi draw 1 and 2 pi draw 3; u_x, u_y from the first pair,
 * u_z the cosine of the second); temperature 0 is a cold species. */
enum { PIC_PROFILE_UNIFORM = 0, PIC_PROFILE_RAMP = 1, PIC_PROFILE_COS_SPHERE = 2 };
enum { PIC_LOAD_WEIGHT = 0, PIC_LOAD_COUNT = 1 };
typedef struct {
    double q, m;           /* must equal the simulation descriptor's */
    int32_t profile;       /* PIC_PROFILE_* */
    int32_t loading;       /* PIC_LOAD_* */
    int32_t ppc;           /* 1..4096 */
    int32_t reserved;      /* 0 */
    double n0;             /* reference density (> 0) */
    double param[6];       /* profile parameters (see above) */
    double temperature;    /* kT / (m c^2) >= 0 */
    uint64_t seed;
} PicSpeciesDesc;

/* Describe the simulation's species (one per simulation; the immobile
 * neutralising ions are implicit and carry minus its charge at load).  *sid
 * (may be NULL) receives 0.  Host-only.  PIC_EINVAL for bad values,
 * PIC_ENOTSUP for a second species, PIC_ESTATE in a batch. */
int pic_species_add(PicSim *s, const PicSpeciesDesc *d, int32_t *sid);
/* Generate species sid's particles on the device as described above; replaces
 * any previous particles and resets the step counter to 0, like
 * pic_particles_set.  PIC_ESTATE without a species or in a batch; PIC_EINVAL
 * when the description gives 2^41 particles or more (2^32 for a 3-D FP32
 * handle). */
int pic_particles_init(PicSim *s, int32_t sid);

/* A Gaussian laser pulse driving the open x = 0 face of a 2-D box (the LWFA
 * driver of section 2.2), evaluated in FP64 by the field update every step
 * at time (n + 1/2) dt on the face's Ey (y = (j + 1/2) d_y) or Ez (y = j d_y)
 * positions: a 2-D paraxial Gaussian beam of waist w0 (1/e field radius) in
 * the plane x = x_focus, Rayleigh length omega0 w0^2 / 2; at the face, a
 * distance s = -x_focus from the waist, spot w = w0 sqrt(1 + (s / x_R)^2),
 * curvature s / (s^2 + x_R^2), Gouy shift atan(s / x_R) / 2, amplitude
 * a0 omega0 sqrt(w0 / w); field
 *   E = a0 omega0 sqrt(w0 / w) exp(-2 ln 2 (t - t0)^2 / tau^2) exp(-(y - yc)^2 / w^2)
 *       sin(omega0 (t - t0) - omega0 (y - yc)^2 curv / 2 + Gouy + phase),
 * tau the FWHM of the intensity.  Lasers add to each other and to a table
 * set with pic_laser_set.  Not part of a checkpoint (add them again after
 * pic_state_load).  PIC_ENOTSUP in 3-D, for another face or beyond four
 * lasers; PIC_EINVAL for a periodic x axis or bad values; PIC_ESTATE in a
 * batch. */
typedef struct {
    double a0;             /* peak field a0 omega0, in m_e c omega_r / e */
    double omega0;         /* carrier frequency (units of omega_r) */
    double w0;             /* waist */
    double tau;            /* FWHM duration of the intensity */
    double t0;             /* time of the envelope peak at the face */
    double x_focus;        /* position of the waist along x */
    double y_center;       /* beam axis */
    double phase;          /* carrier phase */
    int32_t polarisation;  /* 1: Ey (in the plane), 2: Ez */
    int32_t face;          /* 0: x = 0 (the only face supported) */
} PicLaserDesc;
int pic_laser_add(PicSim *s, const PicLaserDesc *d);

/* Incident field driving the open x = 0 face: row t (t = 0..nsteps-1) holds
 * the incident Ey (at y = (j + 1/2) d_y) and Ez (at y = j d_y) at time
 * (t + 1/2) dt, n[1] values per row.  ey or ez may be NULL (zero).  Steps
 * beyond the table see no incident field. */
int pic_laser_set(PicSim *s, int64_t nsteps, const double *ey, const double *ez);

/* Moving window along x (2-D boxes with open x faces).  The LWFA runs follow
 * the pulse over more than a millimetre of plasma (Sec. 2.1, 2.3); the box
 * follows it by jumps of one patch column (patch[0] cells, Sec. 3.1): after
 * step n completes, a jump is made when floor(velocity * (n + 1 - start_step)
 * * dt / (patch[0] * d[0])), evaluated in FP64, exceeds the jumps made so far.
 * A jump moves E, B and the last deposit left by patch[0] nodes (zeros enter
 * at the right), removes the particles of the first patch column (counted in
 * PicDiag.removed), gives every other patch the particles of its right
 * neighbour in the same slots, and fills the new last column with a cold
 * plasma: ppc_x * ppc_y particles per cell at offsets ((a + 1/2) / ppc_x,
 * (b + 1/2) / ppc_y), weight density / (ppc_x * ppc_y), zero momentum, ids
 * continuing from the largest handed out, in (patch row, cell row, cell
 * column, b, a) order.  density[c] (host, FP64, ncols >= 1 values, copied) is
 * the plasma density of global cell column c, counted from the box's initial
 * x = 0; columns beyond the table take density[ncols - 1].  velocity in (0, 1]
 * (units of c), start_step >= 0, ppc_x * ppc_y <= 4096, at most 4096 patch
 * columns.  Patch capacities are raised to hold one column's injection
 * (grows device memory).  The window's configuration is not part of a
 * checkpoint (its progress is); set it again after pic_state_load.  Errors:
 * PIC_ENOTSUP in 3-D or beyond 4096 patch columns, PIC_EINVAL for a periodic
 * x axis or bad arguments, PIC_ESTATE while the simulation is in a batch. */
int pic_window_set(PicSim *s, int64_t start_step, double velocity, int32_t ppc_x, int32_t ppc_y,
                   const double *density, int64_t ncols);

/* Particle merging, the dynamic load limiting of Sec. 3.2 (2-D): in every
 * cell holding more than cell_max particles (4..32), the momenta u = p/(mc),
 * taken in slot order, are grouped by weighted k-means into k = cell_max / 2
 * clusters (centroids start at the momenta of members floor(j n / k); each
 * of `iterations` rounds (1..64) assigns every member to its nearest centroid,
 * lowest index on ties, then moves every non-empty centroid to its cluster's
 * weighted mean).  A cluster of three or more becomes two particles of half
 * its weight W at its weighted mean position, with momenta
 * |u_t| (cos t e1 +- sin t e2), gamma_t = (sum w gamma) / W,
 * |u_t| = sqrt(gamma_t^2 - 1), e1 along the cluster momentum P (x if P = 0),
 * cos t = |P| / (W |u_t|), e2 the axis least aligned with e1 made orthogonal
 * to it; the pair takes the cluster's two smallest ids.  Each cell keeps its
 * weight (charge), momentum, kinetic energy and charge centre; afterwards no
 * cell holds more than cell_max particles.  A patch then holds its untouched
 * particles in slot order followed by the pairs in (cell, cluster) order.
 * The clustering runs in FP64 (FP32 particles are widened).
 * pic_merge_set: merge after every `every`-th step (0: never; the pass runs
 * after the re-binning, before a window jump).  pic_merge: one pass now;
 * *taken (may be NULL) receives the particles taken out.  Errors: PIC_ENOTSUP
 * in 3-D, PIC_EINVAL for out-of-range arguments, PIC_ESTATE in a batch or
 * while a re-binning is pending. */
int pic_merge_set(PicSim *s, int32_t every, int32_t cell_max, int32_t iterations);
int pic_merge(PicSim *s, int32_t cell_max, int32_t iterations, int64_t *taken);

/* Set the completed-step counter of a state loaded from elsewhere
 * (particles and fields at time step * dt): a laser's time and the field
 * buffer that pic_fields_set writes follow it, so call it before
 * pic_fields_set.  The energy history restarts at that step.  PIC_ESTATE in
 * a batch or while a capacity-overflow recovery is pending. */
int pic_step_set(PicSim *s, int64_t step);

/* Overwrite one field component (E or B) from a host FP64 array of
 * count = fn[0]*fn[1]*fn[2] values. */
int pic_fields_set(PicSim *s, int comp, const double *host, size_t count);

/* ---- stepping -------------------------------------------------------------- */

/* Enqueue nsteps full PIC steps on the handle's stream: work-queue build,
 * fused gather / Boris / move / Esirkepov deposit, Yee update with face
 * conditions, re-binning.  Returns after the steps are enqueued; it blocks
 * only to grow patch capacity when a patch overflows (checked every few
 * steps).  Device errors are sticky and reported by pic_sync. */
int pic_step(PicSim *s, int64_t nsteps);

/* Wait for the handle's stream; return PIC_ENAN / PIC_ECFL if a particle
 * error was raised since creation, else PIC_OK. */
int pic_sync(PicSim *s);

/* ---- state out ------------------------------------------------------------- */

int pic_fields_get(PicSim *s, int comp, double *host, size_t count);
int pic_num_particles(PicSim *s, int64_t *n);
/* Particles in canonical (patch, slot) order; each non-NULL array holds at
 * least `count` >= live particles entries.  Positions are global cell units. */
int pic_particles_get(PicSim *s, double *x, double *y, double *z, double *ux, double *uy,
                      double *uz, double *w, int64_t *id, size_t count);
int pic_patch_counts_get(PicSim *s, int32_t *counts, size_t count);
/* The particle permutation: ids[k] is the id of the particle in canonical
 * (patch, slot) position k (count >= live particles). */
int pic_perm_get(PicSim *s, int64_t *ids, size_t count);
int pic_diag_get(PicSim *s, PicDiag *out);
/* Device memory the handle holds now (host-only, no synchronisation): what
 * admission control charges a resident simulation; it grows when patch
 * capacities grow. */
int pic_device_bytes(PicSim *s, int64_t *bytes);
/* Gauss and continuity residuals of the current state (see PicResiduals);
 * synchronises the stream.  Each call records rho^k for the continuity
 * residual of a call one step later.  PIC_ENOTSUP with a moving window,
 * PIC_ESTATE while a capacity-overflow recovery is pending. */
int pic_residuals(PicSim *s, PicResiduals *out);
/* Energy history of completed steps first..first+n-1 (the last 4096 steps
 * are kept): U^k and K^k of step k and the particles it pushed. */
int pic_history_get(PicSim *s, int64_t first, int64_t n, double *U, double *K, int64_t *pushed);

/* ---- re-binning as a function (test hook) ---------------------------------- */

/* Launch-setting tuner.  Tries, by coordinate descent, the workgroup size of
 * the particle kernel, the Yee tile shape (2-D), the lane stride and the
 * chunk size; each candidate runs `steps` steps (0 = 10) from the same saved
 * state, and the simulation's state is restored afterwards (tuning does not
 * advance it).  The fastest settings are applied to the handle.  With a
 * non-NULL `cache` path the result is stored in that text file under a key
 * of dimensions, precision, grid, patch shape and particle count (to a
 * factor of two); a later call with the same key applies the stored
 * settings without running.  `out` (may be NULL) receives the settings in
 * effect.  Not for members of a batch (PIC_ESTATE). */
typedef struct {
    int32_t block, field_tile, lane_stride, chunk;
    double ms_per_step;    /* of the chosen settings (0 on a cache hit) */
    int32_t trials;        /* candidates timed */
    int32_t from_cache;    /* 1 when the settings came from the cache */
    int32_t patch[3];      /* patch shape (pic_autotune_patch; else the handle's) */
} PicTuneResult;
int pic_autotune(PicSim *s, int32_t steps, const char *cache, PicTuneResult *out);

/* Patch-size tuner.  The patch is the paper's unit of load balance (section
 * 3.1) and is fixed when a handle is created, so this tunes a descriptor:
 * for each candidate edge c (patches of c cells on every axis; candidates
 * that do not divide the grid or that the descriptor rules refuse are
 * skipped) it builds a temporary simulation of *d with that patch, loads
 * species sp on the device (and laser l, may be NULL), runs `warm` steps and
 * then times `steps` steps (0 = 20), and writes the fastest candidate's
 * shape into d->patch.  The fastest workgroup size of the particle kernel is
 * chosen along with it (written into d->block).  With a non-NULL `cache` path
 * the choice is stored under a key of dimensions, precision, grid, density
 * profile, loading and ppc, and a later call with the same key applies it
 * without running.  Device memory comes from `a` (NULL: hipMalloc / hipFree)
 * and work runs on hip_stream.  PIC_EINVAL when no candidate fits. */
int pic_autotune_patch(PicSimDesc *d, const PicSpeciesDesc *sp, const PicLaserDesc *l,
                       const int32_t *candidates, int32_t ncand, int32_t warm, int32_t steps,
                       const PicAllocator *a, void *hip_stream, const char *cache,
                       PicTuneResult *out);

/* Checkpoint / resume.  pic_state_save writes the whole simulation state
 * (E and B of the current time level, the last deposit J, the particles in
 * canonical (patch, slot) order with their ids, patch counts, step and
 * removed counters, energy history) into a host buffer: with blob == NULL it
 * only stores the bytes needed in *size; otherwise *size must be at least
 * that and receives the bytes written.  Fails with PIC_ESTATE while a
 * capacity-overflow recovery is pending.  pic_state_load restores such a
 * blob into a handle created with the same grid, patch layout and precision
 * (PIC_EINVAL otherwise; the handle is unchanged when the header is
 * rejected), after which stepping continues bit for bit as from the saved
 * handle.  Both synchronise the handle's stream; the blob is borrowed. */
int pic_state_save(PicSim *s, void *blob, size_t *size);
int pic_state_load(PicSim *s, const void *blob, size_t size);

/* Apply only the re-binning to the current particles, with the destination
 * of each particle given in (patch, slot) order as a direction code:
 * (dx+1) + 3 (dy+1) for a move to the neighbour patch (dx, dy) in
 * {-1,0,1}^2 (4 = stay), or 255 = removed.  Local positions are left as
 * they are.  The step counter is not advanced. */
int pic_rebin_codes(PicSim *s, const uint8_t *codes, size_t count);

/* ---- timing ------------------------------------------------------------------ */

/* Per-kernel timing from start/stop events recorded by the dispatches.
 * mode 0: off; 1: every kernel group (queue, particles, Yee, re-binning);
 * 2: the particle kernel only (one event pair per step, the least
 * perturbation); 3: as 2, and every work item of the particle launch also
 * records when it started and ended and on which compute unit it ran (for
 * pic_imbalance).  Enabling resets the totals; timing also turns graph
 * replay off while on. */
int pic_timing_enable(PicSim *s, int mode);
int pic_timing_get(PicSim *s, PicTiming *out); /* synchronises */

/* Load imbalance of the last particle launch made while timing mode 3 was on
 * (the paper's measure, section 3.1 and Fig. 4: the time of the busiest
 * processing unit over the mean).  The work of one step is this
 * simulation's work items; a compute unit's busy time is the summed
 * duration (start to end on the device clock) of the items it ran.  For
 * comparison the same item times are also dealt out as fixed domains, one
 * per compute unit: equal runs of patch ids (a static decomposition without
 * balancing) and contiguous segments of the Hilbert-curve patch order cut
 * by particle count (pic_curve_segments; patch id order on grids the curve
 * does not cover).  Synchronises.  PIC_ESTATE when no stamped launch ran
 * this simulation's items. */
typedef struct {
    int64_t step;             /* completed steps (the stamps describe the last stamped step) */
    int32_t items;            /* this simulation's work items in that launch */
    int32_t units;            /* compute units that ran at least one of them */
    int32_t device_units;     /* compute units of the device */
    double span_us;           /* first item start to last item end */
    double busy_max_us;       /* busiest compute unit */
    double busy_mean_us;      /* mean over every compute unit of the device */
    double imbalance;         /* busy_max / busy_mean with the work queue */
    double static_imbalance;  /* max / mean with equal runs of patch ids per unit */
    double segment_imbalance; /* max / mean with count-balanced curve segments per unit */
    double patch_max_us, patch_mean_us; /* summed item time per patch */
} PicImbalance;
int pic_imbalance(PicSim *s, PicImbalance *out);

/* ---- batches of simulations stepped together ------------------------------- */

/* A batch steps many simulations of the same ndim and precision together:
 * one work queue over all their patches (ordered by particle count), one
 * persistent particle launch, one Maxwell and one re-binning pass per step.
 * Member simulations keep their own state and results and can be read with
 * the pic_* getters between batch steps.  All members must share the
 * batch's stream. */
int pic_batch_create(int32_t ndim, int32_t precision, void *hip_stream, PicBatch **out);
void pic_batch_destroy(PicBatch *b);
/* Add a simulation that will be advanced by `nsteps` more steps. */
int pic_batch_add(PicBatch *b, PicSim *s, int64_t nsteps);
int pic_batch_remove(PicBatch *b, PicSim *s);
/* Advance every member by up to `max_steps` steps (members stop when their
 * own step budget is used up).  *done receives the number of members that
 * finished their budget during this call. */
int pic_batch_step(PicBatch *b, int64_t max_steps, int32_t *done);
/* Members whose step budget is used up (they stay members until removed). */
int pic_batch_finished(PicBatch *b, PicSim **out, int32_t cap, int32_t *n);
int pic_batch_size(PicBatch *b, int32_t *n);

/* ---- admission ---------------------------------------------------------------- */

/* Device bytes a simulation of descriptor `d` holding `nparticles` particles
 * (and a laser table of `laser_steps` rows) is expected to allocate under the
 * default capacity policy: fields, two current buffers, particle slots with
 * their staging copy, per-patch tables.  Host-only; used by admission
 * control against an HBM budget. */
int pic_estimate_bytes(const PicSimDesc *d, int64_t nparticles, int64_t laser_steps,
                       int64_t *bytes);

/* ---- patch order and segments (section 3.1, Fig. 2) ------------------------------ */

/* Patch ids (x + np[0] (y + np[1] z), row-major) in the order of the Hilbert
 * space-filling curve along which the paper arranges its patches (section
 * 3.1; Fig. 2: on a 32 x 32 grid the curve visits every patch once, from
 * patch (0, 0) to patch (31, 0)).  ndim 2 or 3; np[a] patches per axis, each a
 * power of two; in 3-D two axes equal and the third at least as long.  Longer
 * grids are cut into squares (cubes) of the shortest side along the longest
 * axis, traversed in turn; consecutive patches of the order are always face
 * neighbours.  `order` (caller-owned, n = product of np entries) receives the
 * ids.  Host-only.  PIC_EINVAL for bad arguments or n not matching np,
 * PIC_ENOTSUP for other grid shapes. */
int pic_patch_order(int32_t ndim, const int32_t np[3], int32_t *order, int64_t n);

/* Cut a sequence of n non-negative costs (patch loads in curve order) into k
 * contiguous segments, one per process in the paper's decomposition: segment
 * j is [bounds[j], bounds[j + 1]), where bounds[j] is the first position whose
 * preceding costs sum to at least j / k of the total, so every segment costs at
 * most total / k plus the largest single cost.  `bounds` (caller-owned) has
 * k + 1 entries.  Host-only.  PIC_EINVAL for a null pointer, n < 0, k < 1 or a
 * negative cost. */
int pic_curve_segments(const int64_t *cost, int64_t n, int32_t k, int64_t *bounds);

/* ---- allocation-free entry point ---------------------------------------------- */

/* Largest grid (fn[0] fn[1] fn[2] field nodes) pic_rho_get_noalloc accepts. */
#define PIC_NOALLOC_MAX_NODES 8388608

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation): the charge
 * density of pic_fields_get(s, PIC_RHO, host, count) without any device
 * allocation.  The node sums are kept in a static device array of
 * PIC_NOALLOC_MAX_NODES doubles (64 MiB) that the library holds on every GPU
 * it runs on until the process ends; it is cleared by a kernel on every call.
 * All calls on one GPU share that array, so calls that overlap on one GPU
 * (from several threads or streams) race.  count must equal the grid's node
 * count; grids with more than PIC_NOALLOC_MAX_NODES nodes fail with
 * PIC_EINVAL before any device work.  Synchronises the handle's stream. */
int pic_rho_get_noalloc(PicSim *s, double *host, size_t count);

/* ---- errors ------------------------------------------------------------------ */

const char *pic_strerror(int code);
const char *pic_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* PIC_H */
