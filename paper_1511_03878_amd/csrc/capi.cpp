// C ABI of the patch-PIC library: argument validation, handle management and
// translation of runtime errors into status codes.  No exception crosses
// this boundary.
#include <algorithm>
#include <cstring>

#include "runtime.h"

using namespace pic;

struct PicSim {
    SimBase *impl;
};
struct PicBatch {
    BatchBase *impl;
    int32_t ndim, precision;
};

namespace {

template <typename F>
int guarded(F &&f)
{
    try {
        f();
        return PIC_OK;
    } catch (const Error &e) {
        set_error(e.what());
        return e.code;
    } catch (const std::bad_alloc &) {
        set_error("host allocation failed");
        return PIC_ENOMEM;
    } catch (const std::exception &e) {
        set_error(e.what());
        return PIC_EINVAL;
    } catch (...) {
        set_error("unknown error");
        return PIC_EINVAL;
    }
}

int bad(int code, const char *msg)
{
    set_error(msg);
    return code;
}

template <typename T>
SimImpl<T> *as(PicSim *s)
{
    return static_cast<SimImpl<T> *>(s->impl);
}

}  // namespace

extern "C" {

const char *pic_strerror(int code)
{
    switch (code) {
    case PIC_OK: return "ok";
    case PIC_EINVAL: return "invalid argument";
    case PIC_ENOMEM: return "out of device memory";
    case PIC_EBUDGET: return "memory budget exceeded";
    case PIC_EHIP: return "HIP runtime error";
    case PIC_EOVERFLOW: return "patch capacity overflow";
    case PIC_ENAN: return "non-finite particle momentum";
    case PIC_ECFL: return "particle moved a cell or more in one step";
    case PIC_ESTATE: return "call not valid in the current state";
    case PIC_ENOTSUP: return "not supported";
    default: return "unknown status";
    }
}

const char *pic_last_error(void) { return g_last_error.c_str(); }

int pic_sim_create(const PicSimDesc *d, const PicAllocator *a, void *hip_stream, PicSim **out)
{
    if (!d || !out) return bad(PIC_EINVAL, "null descriptor or output");
    *out = nullptr;
    std::string why;
    int rc = validate_desc(*d, why);
    if (rc != PIC_OK) return bad(rc, why.c_str());
    if (a && (!a->alloc || !a->free)) return bad(PIC_EINVAL, "allocator needs both alloc and free");
    return guarded([&] {
        PicSim *h = new PicSim;
        try {
            if (d->precision == 32)
                h->impl = new SimImpl<float>(*d, a, (hipStream_t)hip_stream);
            else
                h->impl = new SimImpl<double>(*d, a, (hipStream_t)hip_stream);
            h->impl->handle = h;
        } catch (...) {
            delete h;
            throw;
        }
        *out = h;
    });
}

void pic_sim_destroy(PicSim *s)
{
    if (!s) return;
    try {
        delete s->impl;
    } catch (...) {
    }
    delete s;
}

int pic_particles_set(PicSim *s, int64_t n, const double *x, const double *y, const double *z,
                      const double *ux, const double *uy, const double *uz, const double *w)
{
    if (!s) return bad(PIC_EINVAL, "null handle");
    if (n < 0) return bad(PIC_EINVAL, "negative particle count");
    if (n > 0 && (!x || !y || !ux || !uy || !w)) return bad(PIC_EINVAL, "null particle array");
    if (n > (int64_t)1 << 34) return bad(PIC_EINVAL, "too many particles");
    const bool three = s->impl->desc.ndim == 3;
    if (n > 0 && three && !z) return bad(PIC_EINVAL, "null z positions in a 3-D box");
    return guarded([&] {
        const double *xs[3] = {x, y, three ? z : nullptr};
        const double *us[3] = {ux, uy, uz};
        s->impl->set_particles(n, xs, us, w);
    });
}

int pic_species_add(PicSim *s, const PicSpeciesDesc *d, int32_t *sid)
{
    if (!s || !d) return bad(PIC_EINVAL, "null argument");
    return guarded([&] {
        s->impl->add_species(*d);
        if (sid) *sid = 0;
    });
}

int pic_particles_init(PicSim *s, int32_t sid)
{
    if (!s) return bad(PIC_EINVAL, "null handle");
    if (sid != 0) return bad(PIC_EINVAL, "unknown species id");
    return guarded([&] { s->impl->particles_init(); });
}

int pic_laser_add(PicSim *s, const PicLaserDesc *d)
{
    if (!s || !d) return bad(PIC_EINVAL, "null argument");
    return guarded([&] { s->impl->add_laser(*d); });
}

int pic_perm_get(PicSim *s, int64_t *ids, size_t count)
{
    if (!s || !ids) return bad(PIC_EINVAL, "null argument");
    return guarded([&] {
        double *xo[3] = {nullptr, nullptr, nullptr}, *uo[3] = {nullptr, nullptr, nullptr};
        s->impl->get_particles(xo, uo, nullptr, ids, count);
    });
}

int pic_step_set(PicSim *s, int64_t step)
{
    if (!s) return bad(PIC_EINVAL, "null handle");
    return guarded([&] { s->impl->set_step(step); });
}

int pic_window_set(PicSim *s, int64_t start_step, double velocity, int32_t ppc_x, int32_t ppc_y,
                   const double *density, int64_t ncols)
{
    if (!s || !density) return bad(PIC_EINVAL, "null argument");
    return guarded([&] { s->impl->set_window(start_step, velocity, ppc_x, ppc_y, density, ncols); });
}

int pic_merge_set(PicSim *s, int32_t every, int32_t cell_max, int32_t iterations)
{
    if (!s) return bad(PIC_EINVAL, "null handle");
    return guarded([&] { s->impl->set_merge(every, cell_max, iterations); });
}

int pic_merge(PicSim *s, int32_t cell_max, int32_t iterations, int64_t *taken)
{
    if (!s) return bad(PIC_EINVAL, "null handle");
    return guarded([&] {
        const int64_t t = s->impl->merge_now(cell_max, iterations);
        if (taken) *taken = t;
    });
}

int pic_laser_set(PicSim *s, int64_t nsteps, const double *ey, const double *ez)
{
    if (!s) return bad(PIC_EINVAL, "null handle");
    if (nsteps < 0) return bad(PIC_EINVAL, "negative table length");
    if (s->impl->desc.ndim != 2) return bad(PIC_ENOTSUP, "laser injection is 2-D only");
    if (s->impl->desc.periodic[0]) return bad(PIC_ESTATE, "the driven face needs an open x axis");
    return guarded([&] { s->impl->set_laser(nsteps, ey, ez); });
}

static size_t field_count(PicSim *s)
{
    const PicSimDesc &d = s->impl->desc;
    size_t fx = d.periodic[0] ? d.n[0] : d.n[0] + 1;
    size_t fy = d.periodic[1] ? d.n[1] : d.n[1] + 1;
    size_t fz = d.ndim == 3 ? (size_t)d.n[2] : 1;
    return fx * fy * fz;
}

int pic_fields_set(PicSim *s, int comp, const double *host, size_t count)
{
    if (!s || !host) return bad(PIC_EINVAL, "null argument");
    if (comp < PIC_EX || comp > PIC_BZ) return bad(PIC_EINVAL, "only E and B can be set");
    if (count != field_count(s)) return bad(PIC_EINVAL, "field size mismatch");
    return guarded([&] { s->impl->set_field(comp, host); });
}

int pic_fields_get(PicSim *s, int comp, double *host, size_t count)
{
    if (!s || !host) return bad(PIC_EINVAL, "null argument");
    if (comp < PIC_EX || comp > PIC_RHO) return bad(PIC_EINVAL, "bad component");
    if (count != field_count(s)) return bad(PIC_EINVAL, "field size mismatch");
    return guarded([&] { s->impl->get_field(comp, host); });
}

int pic_step(PicSim *s, int64_t nsteps)
{
    if (!s) return bad(PIC_EINVAL, "null handle");
    if (nsteps < 0) return bad(PIC_EINVAL, "negative step count");
    return guarded([&] { s->impl->step(nsteps); });
}

int pic_sync(PicSim *s)
{
    if (!s) return bad(PIC_EINVAL, "null handle");
    int rc = PIC_OK;
    int g = guarded([&] {
        SimState st = s->impl->read_state();
        if (st.flags & kFlagNaN) rc = PIC_ENAN;
        else if (st.flags & kFlagCFL) rc = PIC_ECFL;
        else if (st.flags & kFlagWin) rc = PIC_EOVERFLOW;
    });
    if (g != PIC_OK) return g;
    if (rc != PIC_OK) set_error("a particle error stopped the simulation");
    return rc;
}

int pic_num_particles(PicSim *s, int64_t *n)
{
    if (!s || !n) return bad(PIC_EINVAL, "null argument");
    return guarded([&] { *n = s->impl->num_particles(); });
}

int pic_particles_get(PicSim *s, double *x, double *y, double *z, double *ux, double *uy,
                      double *uz, double *w, int64_t *id, size_t count)
{
    if (!s) return bad(PIC_EINVAL, "null handle");
    return guarded([&] {
        double *xo[3] = {x, y, z};
        double *uo[3] = {ux, uy, uz};
        s->impl->get_particles(xo, uo, w, id, count);
    });
}

int pic_patch_counts_get(PicSim *s, int32_t *counts, size_t count)
{
    if (!s || !counts) return bad(PIC_EINVAL, "null argument");
    return guarded([&] {
        auto c = s->impl->read_counts();
        if (count != c.size()) throw Error(PIC_EINVAL, "count array size mismatch");
        std::memcpy(counts, c.data(), sizeof(int32_t) * c.size());
    });
}

int pic_residuals(PicSim *s, PicResiduals *out)
{
    if (!s || !out) return bad(PIC_EINVAL, "null argument");
    return guarded([&] { s->impl->residuals(out); });
}

int pic_rho_get_noalloc(PicSim *s, double *host, size_t count)
{
    if (!s || !host) return bad(PIC_EINVAL, "null argument");
    return guarded([&] { s->impl->rho_noalloc(host, count); });
}

int pic_device_bytes(PicSim *s, int64_t *bytes)
{
    if (!s || !bytes) return bad(PIC_EINVAL, "null argument");
    *bytes = (int64_t)s->impl->device_bytes();
    return PIC_OK;
}

int pic_imbalance(PicSim *s, PicImbalance *out)
{
    if (!s || !out) return bad(PIC_EINVAL, "null argument");
    return guarded([&] { s->impl->imbalance(out); });
}

int pic_diag_get(PicSim *s, PicDiag *out)
{
    if (!s || !out) return bad(PIC_EINVAL, "null argument");
    return guarded([&] {
        SimState st = s->impl->read_state();
        auto c = s->impl->read_counts();
        std::memset(out, 0, sizeof(*out));
        out->step = st.step;
        out->removed = st.removed;
        int64_t tot = 0;
        int32_t mn = c.empty() ? 0 : c[0], mx = mn;
        for (int32_t v : c) {
            tot += v;
            mn = std::min(mn, v);
            mx = std::max(mx, v);
        }
        out->particles = tot;
        out->occupancy_min = mn;
        out->occupancy_max = mx;
        out->occupancy_mean = c.empty() ? 0.0 : (double)tot / c.size();
        out->flags = (int32_t)st.flags;
        out->relayouts = s->impl->relayouts;
        out->window_cells = st.wshift * s->impl->desc.patch[0];
        out->merged = st.merged;
        out->device_bytes = (int64_t)s->impl->device_bytes();
        if (st.step > 0) {
            double U = 0, K = 0;
            int64_t pushed = 0;
            s->impl->history(st.step - 1, 1, &U, &K, &pushed);
            out->field_energy = U;
            out->kinetic_energy = K;
        }
    });
}

int pic_history_get(PicSim *s, int64_t first, int64_t n, double *U, double *K, int64_t *pushed)
{
    if (!s) return bad(PIC_EINVAL, "null handle");
    return guarded([&] { s->impl->history(first, n, U, K, pushed); });
}

int pic_autotune(PicSim *s, int32_t steps, const char *cache, PicTuneResult *out)
{
    if (!s) return bad(PIC_EINVAL, "null handle");
    if (steps < 0) return bad(PIC_EINVAL, "negative step count");
    return guarded([&] { s->impl->autotune(steps, cache, out); });
}

int pic_autotune_patch(PicSimDesc *d, const PicSpeciesDesc *sp, const PicLaserDesc *l,
                       const int32_t *candidates, int32_t ncand, int32_t warm, int32_t steps,
                       const PicAllocator *a, void *hip_stream, const char *cache,
                       PicTuneResult *out)
{
    if (!d || !sp || !candidates) return bad(PIC_EINVAL, "null argument");
    if (ncand <= 0 || warm < 0 || steps < 0) return bad(PIC_EINVAL, "bad candidate count or step counts");
    std::string why;
    int rc = validate_desc(*d, why);
    if (rc != PIC_OK) return bad(rc, why.c_str());
    if (a && (!a->alloc || !a->free)) return bad(PIC_EINVAL, "allocator needs both alloc and free");
    return guarded([&] {
        autotune_patch(*d, *sp, l, candidates, ncand, warm, steps, a, (hipStream_t)hip_stream, cache, out);
    });
}

int pic_state_save(PicSim *s, void *blob, size_t *size)
{
    if (!s || !size) return bad(PIC_EINVAL, "null argument");
    return guarded([&] {
        const size_t need = s->impl->state_bytes();
        if (!blob) {
            *size = need;
            return;
        }
        if (*size < need) throw Error(PIC_EINVAL, "checkpoint buffer too small");
        s->impl->state_save(blob);
        *size = need;
    });
}

int pic_state_load(PicSim *s, const void *blob, size_t size)
{
    if (!s || !blob) return bad(PIC_EINVAL, "null argument");
    return guarded([&] { s->impl->state_load(blob, size); });
}

int pic_rebin_codes(PicSim *s, const uint8_t *codes, size_t count)
{
    if (!s || (count && !codes)) return bad(PIC_EINVAL, "null argument");
    return guarded([&] { s->impl->rebin_codes(codes, count); });
}

int pic_timing_enable(PicSim *s, int on)
{
    if (!s) return bad(PIC_EINVAL, "null handle");
    if (on < 0 || on > 3) return bad(PIC_EINVAL, "timing mode must be 0, 1, 2 or 3");
    return guarded([&] {
        s->impl->timing.collect();
        s->impl->timing.enabled = on != 0;
        s->impl->timing.only = on >= 2 ? 1 : -1;
        s->impl->timing.stamp = on == 3;
        if (on) {
            for (int k = 0; k < Timing::kKinds; ++k) {
                s->impl->timing.total_ms[k] = 0;
                s->impl->timing.launches[k] = 0;
            }
        }
    });
}

int pic_timing_get(PicSim *s, PicTiming *out)
{
    if (!s || !out) return bad(PIC_EINVAL, "null argument");
    return guarded([&] {
        s->impl->timing.collect();
        std::memset(out, 0, sizeof(*out));
        out->nkernels = Timing::kKinds;
        for (int k = 0; k < Timing::kKinds; ++k) {
            out->name[k] = Timing::names[k];
            out->total_ms[k] = s->impl->timing.total_ms[k];
            out->launches[k] = s->impl->timing.launches[k];
        }
    });
}

int pic_patch_order(int32_t ndim, const int32_t np[3], int32_t *order, int64_t n)
{
    if (!np || !order || (ndim != 2 && ndim != 3)) return bad(PIC_EINVAL, "bad argument");
    int64_t total = 1;
    int p[3] = {1, 1, 1};
    for (int a = 0; a < ndim; ++a) {
        if (np[a] < 1 || np[a] > (1 << 20)) return bad(PIC_EINVAL, "patch counts must be in [1, 2^20]");
        p[a] = np[a];
        total *= np[a];
    }
    if (total != n) return bad(PIC_EINVAL, "n must equal the number of patches");
    return guarded([&] {
        std::vector<int32_t> out;
        std::string why;
        const int rc = hilbert_patch_order(ndim, p, out, why);
        if (rc != PIC_OK) throw Error(rc, why);
        std::memcpy(order, out.data(), sizeof(int32_t) * (size_t)n);
    });
}

int pic_curve_segments(const int64_t *cost, int64_t n, int32_t k, int64_t *bounds)
{
    if ((!cost && n > 0) || !bounds || n < 0 || k < 1) return bad(PIC_EINVAL, "bad argument");
    for (int64_t i = 0; i < n; ++i)
        if (cost[i] < 0) return bad(PIC_EINVAL, "negative cost");
    curve_segments(cost, n, k, bounds);
    return PIC_OK;
}

int pic_estimate_bytes(const PicSimDesc *d, int64_t nparticles, int64_t laser_steps,
                       int64_t *bytes)
{
    if (!d || !bytes || nparticles < 0 || laser_steps < 0) return bad(PIC_EINVAL, "bad argument");
    std::string why;
    int rc = validate_desc(*d, why);
    if (rc != PIC_OK) return bad(rc, why.c_str());
    const int64_t s = d->precision == 32 ? 4 : 8;
    const bool three = d->ndim == 3;
    const int64_t fx = d->periodic[0] ? d->n[0] : d->n[0] + 1;
    const int64_t fy = d->periodic[1] ? d->n[1] : d->n[1] + 1;
    const int64_t fz = three ? d->n[2] : 1;
    const int64_t fsize = fx * fy * fz;
    const int64_t npatch = (int64_t)(d->n[0] / d->patch[0]) * (d->n[1] / d->patch[1]) *
                           (three ? d->n[2] / d->patch[2] : 1);
    const int64_t ndir = three ? 27 : 9;
    const double factor = d->capacity_factor > 0.0 ? d->capacity_factor : 3.0;
    const int64_t mean = std::max<int64_t>(64, (nparticles + npatch - 1) / npatch);
    const int64_t floor_cap = d->min_capacity ? d->min_capacity : mean;
    // capacity policy: max(factor x count, floor) per patch, rounded up to 64
    int64_t slots = std::max<int64_t>((int64_t)(factor * nparticles), floor_cap * npatch) + 64 * npatch;
    // particles + staging (3-D: position with the id and momentum with the
    // weight, four entries each; 2-D: six entries and the id), code, hole list
    const int64_t per_slot = 2 * (three ? 8 * s : 6 * s + 8) + 1 + 4;
    const int fn3[3] = {(int)fx, (int)fy, (int)fz};
    const int64_t max_tiles = three ? std::max(maxwell3d_tiles(fn3, 2), maxwell3d_tiles(fn3, 6))
                                    : ((fx + 15) / 16) * ((fy + 3) / 4);
    int64_t b = 18 * fsize * s;                        // two E, B buffers, two J buffers
    b += slots * per_slot;
    // counts, keys, neighbour table, partials, offsets
    b += npatch * (4 * 7 + 4 * ndir + 4 * (ndir + 1) + 4 * (3 * ndir - 1) + 8 + 8 + 4);
    b += max_tiles * 8 + 8 * 4 * 4096 + 4096;          // tile partials, history, state
    b += 8 * fsize;                                    // charge density at load (diagnostics)
    if (d->deterministic) b += 3 * 8 * fsize;          // fixed-point current accumulators
    b += laser_steps * d->n[1] * s * 2;
    *bytes = b;
    return PIC_OK;
}

// ---- batches --------------------------------------------------------------------

int pic_batch_create(int32_t ndim, int32_t precision, void *hip_stream, PicBatch **out)
{
    if (!out) return bad(PIC_EINVAL, "null output");
    *out = nullptr;
    if (ndim != 2 && ndim != 3) return bad(PIC_ENOTSUP, "ndim must be 2 or 3");
    if (precision != 32 && precision != 64) return bad(PIC_EINVAL, "precision must be 32 or 64");
    return guarded([&] {
        PicBatch *b = new PicBatch;
        b->ndim = ndim;
        b->precision = precision;
        if (precision == 32) {
            auto *bi = new BatchImpl<float>((hipStream_t)hip_stream);
            bi->nd = ndim;
            b->impl = bi;
        } else {
            auto *bi = new BatchImpl<double>((hipStream_t)hip_stream);
            bi->nd = ndim;
            b->impl = bi;
        }
        b->impl->precision = precision;
        b->impl->stream = (hipStream_t)hip_stream;
        *out = b;
    });
}

void pic_batch_destroy(PicBatch *b)
{
    if (!b) return;
    try {
        delete b->impl;
    } catch (...) {
    }
    delete b;
}

int pic_batch_add(PicBatch *b, PicSim *s, int64_t nsteps)
{
    if (!b || !s) return bad(PIC_EINVAL, "null argument");
    if (nsteps < 0) return bad(PIC_EINVAL, "negative step budget");
    if (s->impl->precision != b->precision) return bad(PIC_EINVAL, "precision mismatch");
    return guarded([&] {
        if (b->precision == 32) static_cast<BatchImpl<float> *>(b->impl)->add(as<float>(s), nsteps);
        else static_cast<BatchImpl<double> *>(b->impl)->add(as<double>(s), nsteps);
    });
}

int pic_batch_remove(PicBatch *b, PicSim *s)
{
    if (!b || !s) return bad(PIC_EINVAL, "null argument");
    if (s->impl->precision != b->precision) return bad(PIC_EINVAL, "not a member");
    return guarded([&] {
        if (b->precision == 32) static_cast<BatchImpl<float> *>(b->impl)->remove(as<float>(s));
        else static_cast<BatchImpl<double> *>(b->impl)->remove(as<double>(s));
    });
}

int pic_batch_step(PicBatch *b, int64_t max_steps, int32_t *done)
{
    if (!b) return bad(PIC_EINVAL, "null batch");
    if (max_steps < 0) return bad(PIC_EINVAL, "negative step count");
    return guarded([&] {
        int d = 0;
        if (b->precision == 32) d = static_cast<BatchImpl<float> *>(b->impl)->run(max_steps, false);
        else d = static_cast<BatchImpl<double> *>(b->impl)->run(max_steps, false);
        if (done) *done = d;
    });
}

int pic_batch_finished(PicBatch *b, PicSim **out, int32_t cap, int32_t *n)
{
    if (!b || !n || (cap > 0 && !out)) return bad(PIC_EINVAL, "null argument");
    return guarded([&] {
        std::vector<SimBase *> fin;
        if (b->precision == 32) static_cast<BatchImpl<float> *>(b->impl)->finished(fin);
        else static_cast<BatchImpl<double> *>(b->impl)->finished(fin);
        int32_t k = 0;
        for (SimBase *m : fin) {
            if (k < cap) out[k] = static_cast<PicSim *>(m->handle);
            ++k;
        }
        *n = k;
    });
}

int pic_batch_size(PicBatch *b, int32_t *n)
{
    if (!b || !n) return bad(PIC_EINVAL, "null argument");
    if (b->precision == 32) *n = (int32_t)static_cast<BatchImpl<float> *>(b->impl)->members.size();
    else *n = (int32_t)static_cast<BatchImpl<double> *>(b->impl)->members.size();
    return PIC_OK;
}

}  // extern "C"
