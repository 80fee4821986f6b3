// Host runtime declarations of the patch-PIC library.
#pragma once

#include <hip/hip_runtime.h>

#include <map>
#include <stdexcept>
#include <string>
#include <vector>

#include "../../include/pic.h"
#include "kernels.h"
#include "pic_dev.h"

namespace pic {

struct Error : std::runtime_error {
    int code;
    Error(int c, const std::string &m) : std::runtime_error(m), code(c) {}
};

void set_error(const std::string &m);
// Device address, on the current device, of the static scratch of the
// allocation-free charge-density call (PIC_NOALLOC_MAX_NODES doubles).
constexpr int kMaxDevices = 64;
double *noalloc_scratch();
extern thread_local std::string g_last_error;
void hipcheck(hipError_t e, const char *what);
int validate_desc(const PicSimDesc &d, std::string &why);
// patch ids in Hilbert-curve order (order.cpp); PIC_ENOTSUP for unsupported grids
int hilbert_patch_order(int nd, const int np[3], std::vector<int32_t> &out, std::string &why);
void curve_segments(const int64_t *cost, int64_t n, int k, int64_t *bounds);
void autotune_patch(PicSimDesc &d, const PicSpeciesDesc &sp, const PicLaserDesc *l, const int32_t *cand,
                    int ncand, int warm, int steps, const PicAllocator *a, hipStream_t stream,
                    const char *cache, PicTuneResult *out);

struct Allocator {
    PicAllocator hook{nullptr, nullptr, nullptr};
    size_t live_bytes = 0;
    std::map<void *, size_t> sizes;
    void *get(size_t bytes);
    void put(void *p);
};

struct Timing {
    static constexpr int kKinds = 4;
    static const char *const names[kKinds];
    struct Ev {
        int kind;
        hipEvent_t a, b;
    };
    bool enabled = false;
    bool stamp = false;  // record per-item stamps in the particle launch
    int only = -1;  // time only this kind (-1: all)
    std::vector<Ev> events;
    std::vector<hipEvent_t> pool;
    double total_ms[kKinds] = {0, 0, 0, 0};
    int64_t launches[kKinds] = {0, 0, 0, 0};
    // events for one timed launch (or group of launches) of `kind`; both
    // null when timing is off
    Ev2 pair(int kind);
    void collect();
};

struct SimBase {
    virtual ~SimBase() {}
    PicSimDesc desc{};
    int precision = 64;
    hipStream_t stream = nullptr;
    Timing timing;
    int relayouts = 0;
    void *handle = nullptr;  // the C handle wrapping this object

    virtual void set_particles(int64_t n, const double *const xs[3], const double *const us[3],
                               const double *w) = 0;
    virtual void set_laser(int64_t nsteps, const double *ey, const double *ez) = 0;
    virtual void add_laser(const PicLaserDesc &l) = 0;
    virtual void add_species(const PicSpeciesDesc &sp) = 0;
    virtual void particles_init() = 0;
    virtual void set_window(int64_t start, double vel, int ppcx, int ppcy, const double *dens,
                            int64_t ncols) = 0;
    virtual void set_merge(int every, int cmax, int iters) = 0;
    virtual int64_t merge_now(int cmax, int iters) = 0;
    virtual void set_field(int comp, const double *h) = 0;
    virtual void set_step(int64_t step) = 0;
    virtual void get_field(int comp, double *h) = 0;
    virtual SimState read_state() = 0;
    virtual std::vector<int32_t> read_counts() = 0;
    virtual int64_t num_particles() = 0;
    virtual void get_particles(double *xo[3], double *uo[3], double *wo, int64_t *ido, size_t n) = 0;
    virtual void history(int64_t first, int64_t n, double *U, double *K, int64_t *pushed) = 0;
    virtual void rebin_codes(const uint8_t *codes, size_t n) = 0;
    virtual void residuals(PicResiduals *out) = 0;
    virtual void imbalance(PicImbalance *out) = 0;
    virtual void rho_noalloc(double *h, size_t count) = 0;
    virtual void step(int64_t nsteps) = 0;
    virtual bool in_batch() const = 0;
    virtual size_t device_bytes() const = 0;
    virtual void autotune(int steps, const char *cache, PicTuneResult *out) = 0;
    // checkpoint: bytes of the blob, write it, restore from it
    virtual size_t state_bytes() = 0;
    virtual void state_save(void *blob) = 0;
    virtual void state_load(const void *blob, size_t size) = 0;
};

template <typename T>
struct BatchImpl;

template <typename T>
struct SimImpl : SimBase {
    Allocator alloc;
    int nd = 2;     // dimensions
    int ndir = 9;   // neighbour directions (9 in 2-D, 27 in 3-D)
    int n[3], P[3], np[3], fn[3], periodic[3];
    int npatch = 0;
    int64_t fsize = 0;
    T *F[2][6] = {};
    T *J[2][3] = {};
    int64_t *Jacc[3] = {};  // fixed-point current accumulators (deterministic deposition only)
    SimState *st = nullptr;
    double *hist = nullptr;
    int32_t *counts_d = nullptr, *newcount_d = nullptr, *kcnt_d = nullptr, *kofs_d = nullptr, *nleave_d = nullptr;
    int32_t *narrive_d = nullptr, *nhole_d = nullptr, *moved_d = nullptr, *porder_d = nullptr;
    int *prefix_d = nullptr, *tprefix_d = nullptr;
    int32_t *nbt_d = nullptr;
    double *upart = nullptr, *kpart = nullptr;
    int64_t max_tiles = 0;
    // diagnostics: the particles' charge density at load (the immobile ions
    // carry its negative) and at the last residual call
    double *rho0_d = nullptr, *rhoprev_d = nullptr;
    bool rho0_valid = false;
    int64_t rhoprev_step = -1;
    T *laser_ey = nullptr, *laser_ez = nullptr;
    int64_t laser_steps = 0;
    std::vector<PicLaserDesc> lasers;
    bool has_species = false;
    PicSpeciesDesc species{};
    // particle layout
    std::vector<void *> part_bufs;
    // interleaved: positions pwid per slot, momenta and weight 4 per slot (see SimDev)
    T *pP = nullptr, *sP = nullptr, *pM = nullptr, *sM = nullptr;
    int pwid = 2;
    int64_t *pid = nullptr, *sid = nullptr;
    uint8_t *code = nullptr;
    int32_t *holes = nullptr, *cap_d = nullptr;
    int64_t *off_d = nullptr;
    std::vector<int32_t> cap_h;
    std::vector<int64_t> off_h;
    // moving window: jumps rotate count/cap/off on the device, so cap_h and
    // off_h are re-read (sync_layout) before the host uses them
    bool win_on = false;
    int64_t win_start = 0, win_ncols = 0;
    double win_v = 0.0;
    int win_ppc[2] = {1, 1};
    double *wdens_d = nullptr;
    int32_t cap_floor = 0;  // smallest patch capacity (the particles one jump injects)
    int merge_every = 0, merge_cmax = 16, merge_iters = 8;
    int64_t total_cap = 0;
    int max_items_cache = -1, chunk_cache = -1;
    int64_t layout_version = 0;
    int lane_stride = 1;
    SimDev<T> v;
    SimDev<T> *view_d = nullptr;
    BatchImpl<T> *batch = nullptr;  // user batch this simulation belongs to
    BatchImpl<T> *solo = nullptr;   // private batch used by step()

    SimImpl(const PicSimDesc &d, const PicAllocator *a, hipStream_t s);
    ~SimImpl() override;
    void release();
    void free_particles();
    std::vector<void *> layout_particles(const std::vector<int32_t> &need);
    void refresh_view();
    void grow_capacity();
    void relayout(const std::vector<int32_t> &need);
    void sync_layout();
    void recover_pending();
    void build_neighbour_table();
    int max_items(int chunk);
    void check_free();

    void set_particles(int64_t n, const double *const xs[3], const double *const us[3],
                       const double *w) override;
    void set_laser(int64_t nsteps, const double *ey, const double *ez) override;
    void add_laser(const PicLaserDesc &l) override;
    void add_species(const PicSpeciesDesc &sp) override;
    void particles_init() override;
    void finish_load(const std::vector<int32_t> &counts, int64_t total);
    void set_window(int64_t start, double vel, int ppcx, int ppcy, const double *dens,
                    int64_t ncols) override;
    void set_merge(int every, int cmax, int iters) override;
    int64_t merge_now(int cmax, int iters) override;
    void set_field(int comp, const double *h) override;
    void set_step(int64_t step) override;
    void get_field(int comp, double *h) override;
    SimState read_state() override;
    std::vector<int32_t> read_counts() override;
    int64_t num_particles() override;
    void get_particles(double *xo[3], double *uo[3], double *wo, int64_t *ido, size_t n) override;
    void history(int64_t first, int64_t n, double *U, double *K, int64_t *pushed) override;
    void rebin_codes(const uint8_t *codes, size_t n) override;
    void residuals(PicResiduals *out) override;
    void imbalance(PicImbalance *out) override;
    void rho_noalloc(double *h, size_t count) override;
    void record_rho0();
    void step(int64_t nsteps) override;
    bool in_batch() const override { return batch != nullptr; }
    size_t device_bytes() const override { return alloc.live_bytes; }
    void autotune(int steps, const char *cache, PicTuneResult *out) override;
    size_t state_bytes() override;
    void state_save(void *blob) override;
    void state_load(const void *blob, size_t size) override;
};

struct BatchBase {
    virtual ~BatchBase() {}
    int precision = 64;
    hipStream_t stream = nullptr;
};

template <typename T>
struct BatchImpl : BatchBase {
    std::vector<SimImpl<T> *> members;
    std::vector<int64_t> seen_version;
    bool dirty = true;
    bool solo_mode = false;
    std::vector<void *> table_bufs;
    SimDev<T> *sims_d = nullptr;
    int *patch_prefix_d = nullptr, *tile_prefix_d = nullptr;
    // members with deterministic deposition: their indices and the exclusive
    // prefix of their field-node counts (for the accumulator conversion)
    int ndet = 0;
    int64_t det_nodes = 0;
    int *det_list_d = nullptr;
    int64_t *det_prefix_d = nullptr;
    Item *items_d = nullptr;
    int *nitems_d = nullptr, *head_d = nullptr;
    int *qscratch_d = nullptr;  // grid-wide queue build: bucket counts and cursors, participation
    ItemStamp *stamps_d = nullptr;  // per-item records of the last stamped particle launch
    int *stamp_n_d = nullptr;       // its item count
    int table_cap_items = 0;
    int total_patches = 0, total_tiles = 0;
    int nd = 0;  // dimensions of the members (set by the first one)
    int maxP0 = 1, maxP1 = 1, maxP2 = 1;
    int chunk = 256, block = 256, tile_preset = 0, patch_const = 0;
    bool hi_order = false;  // some member uses the sixth-order field solver
    bool yee_any = true;    // some member uses the Yee solver
    int grid_particles = 1, grid_maxwell = 1, grid_rebin = 1;
    Timing own_timing;
    // step batches replayed from a captured graph
    static constexpr int kGraphSteps = 32;
    bool use_graph = false, graph_failed = false;
    hipGraphExec_t graph_exec = nullptr;
    hipStream_t capture_stream = nullptr;
    // the field update runs on a second stream beside the re-binning (they
    // share no data); forked after the particle kernel, joined before the close
    hipStream_t side_stream = nullptr;
    hipEvent_t ev_fork = nullptr, ev_join = nullptr;
    bool side_failed = false;
    bool ensure_side();
    void free_graph();
    bool capture_graph();

    explicit BatchImpl(hipStream_t s);
    ~BatchImpl() override;
    void free_tables();
    void add(SimImpl<T> *s, int64_t nsteps);
    void remove(SimImpl<T> *s);
    void build_tables();
    void refresh_member_views();
    QueueArgs queue_args() const;
    void launch_close_queue_pass();
    void launch_one_step();
    Timing &timing();
    int run(int64_t max_steps, bool until_done);
    void finished(std::vector<SimBase *> &out);
};

}  // namespace pic
