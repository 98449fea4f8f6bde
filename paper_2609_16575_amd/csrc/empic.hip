// empic.hip -- host runtime of libempic: the C ABI declared in include/empic.h.
//
// Owns no device memory: fields, particle buffers and the workspace come from
// the caller; this file validates arguments, carves the workspace, orders the
// kernel launches of the PIC cycle on the caller's stream (Sec. 2.2 of
// KEMPIC-3D) and converts kernel fault words and HIP errors into status codes.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "internal.hpp"

using namespace empic;

// The workspace of empic_create_static: each GPU the library runs on holds
// its own copy until the process ends.  In host code the name is a host-side
// stand-in, never passed to a kernel or a copy: the device address comes from
// hipGetSymbolAddress, once per device, and is kept per device.
static __device__ __align__(256) unsigned char scratch[EMPIC_STATIC_SCRATCH_BYTES];

namespace {

constexpr size_t ALIGN = 256;
inline size_t up_align(size_t x) { return (x + ALIGN - 1) / ALIGN * ALIGN; }

struct Layout {
    size_t Bbar, fault, table, partials, result, rho_cur, rho_prev, tile_off, counts, scan, rank,
        fb_mask, fb_tiles, adj, jfix, filt, mur, total;
    size_t tile_off_stride;
    long long mur_stride;
};

// The tile shape of a grid: 16 x 2 x 8 when it is at most three cells thick
// along y (the two-dimensional runs), else 8 x 8 x 4.
void tile_shape_of(const empic_grid_desc *d, int t[3], int &slab) {
    slab = d->n[1] <= 3 ? 1 : 0;
    t[0] = slab ? TileSlab::TX : TileCube::TX;
    t[1] = slab ? TileSlab::TY : TileCube::TY;
    t[2] = slab ? TileSlab::TZ : TileCube::TZ;
}

void grid_info(const empic_grid_desc *d, GridP &g, TileInfo &ti) {
    int t[3];
    tile_shape_of(d, t, ti.slab);
    for (int a = 0; a < 3; ++a) {
        g.n[a] = d->n[a];
        g.bc[a] = d->bc[a];
        g.ext[a] = d->n[a] + (d->bc[a] != EMPIC_BC_PERIODIC ? 1 : 0);  // walled: n+1 planes
        g.d[a] = d->d[a];
        g.inv_d[a] = 1.0 / d->d[a];
        ti.nt[a] = (d->n[a] + t[a] - 1) / t[a];
        int lg = 0;
        while ((1 << lg) < t[a]) ++lg;
        ti.lg[a] = lg;
    }
    g.dt = d->dt;
    g.V = (long long)g.ext[0] * g.ext[1] * g.ext[2];
    ti.ntiles = ti.nt[0] * ti.nt[1] * ti.nt[2];
    ti.NK = (long long)ti.ntiles * TC;
}

Layout layout(const empic_grid_desc *d, int max_species, long long max_capacity) {
    GridP g;
    TileInfo ti;
    grid_info(d, g, ti);
    const size_t es = d->precision == EMPIC_FP64_PLAIN ? 8 : 4;
    Layout L;
    size_t o = 0;
    L.Bbar = o;
    o += up_align(3 * (size_t)g.V * es);
    L.fault = o;
    o += up_align(64);
    L.table = o;
    o += up_align(sizeof(DevSpecies) * 2 * EMPIC_MAX_SPECIES);  // own sets; state-to-state
    L.partials = o;
    o += up_align((size_t)NQ * PSTRIDE * 8);
    L.result = o;
    o += up_align(NQ * 8);
    L.rho_cur = o;
    o += up_align((size_t)g.V * 8);
    L.rho_prev = o;
    o += up_align((size_t)g.V * 8);
    L.tile_off = o;
    L.tile_off_stride = up_align(((size_t)ti.ntiles + 1) * 4 + 4);
    o += L.tile_off_stride * (size_t)max_species;
    L.counts = o;
    o += up_align(((size_t)ti.NK + 1) * 4);
    L.scan = o;
    o += up_align(((size_t)(ti.NK + 1023) / 1024 + 2) * 4);
    L.rank = o;
    o += up_align((size_t)max_capacity * 4);
    L.fb_mask = o;  // out-of-window marks (FP32 step, adjoint): one bit per slot and species
    o += up_align((size_t)max_species * (size_t)((max_capacity + 31) / 32) * 4);
    L.fb_tiles = o;  // tiles with marked particles in one step
    o += up_align((size_t)ti.ntiles * 4);
    L.adj = o;      // adjoint accumulators (FP32 path): gather lam_E, lam_Bbar, lam_B'
    o += d->precision == EMPIC_FP64_PLAIN ? 0 : up_align((size_t)9 * g.V * 4);
    L.jfix = o;     // FP32 path: the step's current as int64 sums (units 1/jscale)
    o += d->precision == EMPIC_FP64_PLAIN ? 0 : up_align((size_t)3 * g.V * 8);
    L.filt = o;     // current filter: the second buffer of its passes
    o += up_align((size_t)3 * g.V * es);
    long long ps = 0;
    for (int a = 0; a < 3; ++a) {
        const int b1 = a == 0 ? 1 : 0, b2 = a == 2 ? 1 : 2;
        const long long area = (long long)g.ext[b1] * g.ext[b2];
        if (area > ps) ps = area;
    }
    L.mur_stride = ps;
    L.mur = o;
    const bool absorbing = d->bc[0] == EMPIC_BC_ABSORBING || d->bc[1] == EMPIC_BC_ABSORBING ||
                           d->bc[2] == EMPIC_BC_ABSORBING;
    o += absorbing ? up_align((size_t)3 * 2 * 4 * ps * es) : 0;
    L.total = o;
    return L;
}

struct SpeciesState {
    empic_species_desc desc{};
    long long capacity = 0;
    empic_particle_buffers buf[2]{};
    bool has_alt = false;
    int cur = 0;
    int32_t *tile_off = nullptr;  // ntiles + 1
    int32_t *dcount = nullptr;    // device slot count
    long long host_count = 0;
    bool tiles_valid = false;     // particles grouped by the tile offsets of a previous sort
    double wmax = 0.0;            // largest |weight| (species w, or the loaded per-particle max)
    long long next_id = 0;        // id of the next injected particle
    bool inject = false;          // moving-window injection of this species
    int inj_per[3] = {1, 1, 1};
    double inj_w = 0.0;
};

struct TimedEvent {
    hipEvent_t a, b;
    int kind;  // 0 push, 1 field, 2 sort
};

}  // namespace

struct empic_sim {
    empic_grid_desc desc{};
    GridP g{};
    TileInfo ti{};
    Layout L{};
    hipStream_t stream = nullptr;
    char *ws = nullptr;
    void *Bbar[3]{};
    uint32_t *fault = nullptr;
    unsigned long long *fallback = nullptr;
    DevSpecies *table = nullptr;   // the species' own buffer sets
    DevSpecies *xtable = nullptr;  // (source, destination) state of empic_step_state
    double *partials = nullptr, *result = nullptr, *rho_cur = nullptr, *rho_prev = nullptr;
    int32_t *counts = nullptr, *scan_blocks = nullptr, *rank = nullptr;
    void *mur = nullptr;
    uint32_t *fb_mask = nullptr;
    long long mask_words = 0;
    int *fb_tiles = nullptr;
    unsigned *fb_count = nullptr;
    float *adj = nullptr;
    unsigned long long *jfix[3]{};  // FP32 path: the current as exact int64 sums
    void *E[3]{}, *B[3]{}, *J[3]{};
    bool bound = false;
    SpeciesState sp[EMPIC_MAX_SPECIES];
    int nsp = 0, max_species = 0;
    long long max_capacity = 0;
    double rho_bg = 0.0;
    empic_laser_desc laser{};
    empic_port_desc port{};
    int filter_passes = 0, filter_comp = 0;
    empic_window_desc window{};
    long long window_shifts = 0;
    void *filt = nullptr;
    long long nstep = 0, rho_prev_step = -1;
    bool need_sort = true;
    // adaptive sorting (sort_every = -1): every step's out-of-window pass
    // writes the cumulative out-of-window count into a ring of pinned host
    // slots; the step two steps later reads it (so the GPU keeps a step
    // queued)
    bool adaptive = false;
    unsigned long long *fb_host = nullptr;  // ADAPT_RING slots
    unsigned long long *fb_dev = nullptr;   // the same slots as the device addresses them
    hipEvent_t fb_ev[4] = {nullptr, nullptr, nullptr, nullptr};
    long long fb_tag[4] = {-1, -1, -1, -1};  // nstep after which each slot was copied
    long long fb_prev_tag = -1, last_sort_step = 0;
    unsigned long long fb_prev = 0;
    double jscale = 1099511627776.0;  // fixed-point scale of the fused kernel's current window
    bool poisoned = false;
    std::string err;
    int timing = 0;  // 0 off, 1 every timed kernel group, 2 the particle kernel only
    std::vector<TimedEvent> events;
    double t_ms[3] = {0, 0, 0};
    long long t_n[3] = {0, 0, 0};
    int static_dev = -1;  // >= 0: the handle of empic_create_static on that device
};

namespace {

empic_status fail(empic_sim *s, empic_status st, const std::string &msg) {
    if (s) s->err = msg;
    return st;
}

empic_status hip_fail(empic_sim *s, hipError_t e, const char *what) {
    if (s) {
        s->poisoned = true;
        s->err = std::string(what) + ": " + hipGetErrorString(e);
    }
    return EMPIC_E_HIP;
}

#define EMPIC_HIP(call)                                 \
    do {                                                \
        hipError_t e_ = (call);                         \
        if (e_ != hipSuccess) return hip_fail(s, e_, #call); \
    } while (0)

#define EMPIC_GUARD(s)                                                               \
    do {                                                                             \
        if (!(s)) return EMPIC_E_ARG;                                                \
        if ((s)->poisoned) return fail((s), EMPIC_E_HIP, "handle poisoned by an earlier HIP error"); \
        (s)->err.clear();                                                            \
    } while (0)

bool fp64(const empic_sim *s) { return s->desc.precision == EMPIC_FP64_PLAIN; }

SpeciesP species_params(const empic_sim *s, int i, int which) {
    const SpeciesState &S = s->sp[i];
    const empic_particle_buffers &b = S.buf[which];
    SpeciesP p;
    p.cell = (uint32_t *)b.cell;
    for (int a = 0; a < 3; ++a) {
        p.pos[a] = b.pos[a];
        p.u[a] = b.u[a];
    }
    p.id = b.id;
    p.w = S.desc.per_particle_w ? b.w : nullptr;
    p.tile_off = S.tile_off;
    p.count = S.dcount;
    p.capacity = S.capacity;
    p.q = S.desc.q;
    p.m = S.desc.m;
    p.w_species = S.desc.w;
    p.per_particle_w = S.desc.per_particle_w;
    return p;
}

void ev_begin(empic_sim *s, TimedEvent &t, int kind) {
    t.kind = kind;
    t.a = t.b = nullptr;
    if (!(s->timing == 1 || (s->timing == 2 && kind == 0))) return;  // mode 2: particle kernels only
    (void)hipEventCreate(&t.a);
    (void)hipEventCreate(&t.b);
    (void)hipEventRecord(t.a, s->stream);
}
void ev_end(empic_sim *s, TimedEvent &t) {
    if (!t.a) return;
    (void)hipEventRecord(t.b, s->stream);
    s->events.push_back(t);
}

template <typename T>
void field_ptrs(empic_sim *s, T *E[3], T *B[3], T *J[3], T *Bb[3]) {
    for (int a = 0; a < 3; ++a) {
        E[a] = (T *)s->E[a];
        B[a] = (T *)s->B[a];
        J[a] = (T *)s->J[a];
        Bb[a] = (T *)s->Bbar[a];
    }
}

void do_sort(empic_sim *s, int32_t *const *perm = nullptr) {
    TimedEvent t;
    ev_begin(s, t, 2);
    for (int i = 0; i < s->nsp; ++i) {
        SpeciesState &S = s->sp[i];
        const SpeciesP cur = species_params(s, i, S.cur);
        const SpeciesP alt = species_params(s, i, 1 - S.cur);
        launch_sort(s->g, s->ti, cur, alt, s->counts, s->scan_blocks, s->rank, S.tile_off,
                    s->fault, S.tiles_valid, perm ? perm[i] : nullptr, s->stream);
        S.cur = 1 - S.cur;
        S.tiles_valid = true;
    }
    ev_end(s, t);
    s->need_sort = false;
    s->last_sort_step = s->nstep;
}

// Adaptive sorting.  Particles that have drifted out of their tile's LDS
// windows since the last sort are pushed by the slower global-memory pass,
// and their number grows quickly once drift reaches the window margin.  The
// step reads the count of two steps earlier (waiting for that step only, so
// one step stays queued on the GPU); once out-of-window particles arrive
// faster than SORT_RATE of the particle slots per step after the last sort,
// or SORT_MAX steps have passed, it starts with a sort.
constexpr int ADAPT_RING = 4;
constexpr int ADAPT_LAG = 2;
constexpr double SORT_RATE = 2e-5;
constexpr int SORT_MAX = 64;

void release_adaptive(empic_sim *s) {
    for (int r = 0; r < ADAPT_RING; ++r)
        if (s->fb_ev[r]) {
            (void)hipEventSynchronize(s->fb_ev[r]);
            (void)hipEventDestroy(s->fb_ev[r]);
            s->fb_ev[r] = nullptr;
        }
    if (s->fb_host) (void)hipHostFree(s->fb_host);
    s->fb_host = nullptr;
}

void adaptive_poll(empic_sim *s) {
    if (s->nstep - s->last_sort_step >= SORT_MAX) s->need_sort = true;
    const long long want = s->nstep - ADAPT_LAG;
    if (want < 1) return;
    const int slot = (int)(want % ADAPT_RING);
    if (s->fb_tag[slot] != want) return;  // not recorded (first steps, other entry points)
    s->fb_tag[slot] = -1;
    if (hipEventSynchronize(s->fb_ev[slot]) != hipSuccess) return;  // reported by the step's check
    const unsigned long long c = ((volatile unsigned long long *)s->fb_host)[slot];
    if (s->fb_prev_tag == want - 1 && want - 1 >= s->last_sort_step && c >= s->fb_prev) {
        long long slots = 0;
        for (int i = 0; i < s->nsp; ++i) slots += s->sp[i].host_count;
        if ((double)(c - s->fb_prev) > SORT_RATE * (double)(slots > 0 ? slots : 1))
            s->need_sort = true;
    }
    s->fb_prev = c;
    s->fb_prev_tag = want;
}

// slot that the step about to run publishes into (the state after it)
unsigned long long *adaptive_slot(empic_sim *s) {
    return s->fb_dev + (s->nstep + 1) % ADAPT_RING;
}

// after the step: mark its slot with an event (the write itself is done by
// the step's out-of-window pass)
void adaptive_record(empic_sim *s) {
    const int slot = (int)(s->nstep % ADAPT_RING);
    if (hipEventRecord(s->fb_ev[slot], s->stream) != hipSuccess) return;  // reported by the step
    s->fb_tag[slot] = s->nstep;
}

// One PIC cycle.  FP32 path: particles are read from buffer set bit s of
// rd_mask and written to bit s of wr_mask of table `tbl` (the species' own
// sets by default).
template <typename T>
void one_step(empic_sim *s, const DevSpecies *tbl = nullptr, int rd_mask = -1, int wr_mask = -1,
              unsigned long long *publish = nullptr) {
    T *E[3], *B[3], *J[3], *Bb[3];
    field_ptrs<T>(s, E, B, J, Bb);
    const bool absorbing = s->g.bc[0] == EMPIC_BC_ABSORBING || s->g.bc[1] == EMPIC_BC_ABSORBING ||
                           s->g.bc[2] == EMPIC_BC_ABSORBING;
    const bool pec = s->g.bc[0] == EMPIC_BC_PEC || s->g.bc[1] == EMPIC_BC_PEC ||
                     s->g.bc[2] == EMPIC_BC_PEC;
    TimedEvent t;
    ev_begin(s, t, 1);
    // 1. Faraday + temporal centring of B; J (FP64) or its fixed-point sums
    // (FP32) zeroed for this step's deposit
    constexpr bool f32 = sizeof(T) == 4;
    launch_faraday<T>(s->g, E, B, Bb, f32 ? nullptr : J, f32 ? s->jfix : nullptr, true,
                      s->stream, f32 ? s->fb_count : nullptr);
    ev_end(s, t);
    // 2. gather, Boris, move, ZigZag for every species
    if constexpr (sizeof(T) == 4) {
        if (s->nsp > 0) {  // a handle without species has nothing to push
            unsigned mask = 0;
            for (int i = 0; i < s->nsp; ++i) mask |= (unsigned)s->sp[i].cur << i;
            if (!tbl) tbl = s->table;
            const unsigned rmask = rd_mask < 0 ? mask : (unsigned)rd_mask;
            const unsigned wmask = wr_mask < 0 ? mask : (unsigned)wr_mask;
            // the fused kernel is timed by events attached to its own dispatch
            TimedEvent tp{nullptr, nullptr, 0};
            if (s->timing) {
                (void)hipEventCreate(&tp.a);
                (void)hipEventCreate(&tp.b);
            }
            for (int pass = 0; pass < 2; ++pass)
                launch_push_fused(s->g, s->ti, (float *const *)E, (float *const *)Bb,
                                  s->jfix, tbl, s->nsp, rmask, wmask, s->fault,
                                  s->fallback, s->fb_mask, s->mask_words, s->fb_tiles,
                                  s->fb_count, s->jscale,
                                  pass == 1, s->stream, pass == 0 ? tp.a : nullptr,
                                  pass == 0 ? tp.b : nullptr, pass == 1 ? publish : nullptr);
            if (s->timing) s->events.push_back(tp);
        }
    } else {
        ev_begin(s, t, 0);
        for (int i = 0; i < s->nsp; ++i)
            launch_push_f64(s->g, (double *const *)E, (double *const *)Bb, (double *const *)J,
                            species_params(s, i, 0), s->sp[i].host_count, s->fault, s->stream);
        ev_end(s, t);
    }
    // 3. current filter, Ampere-Maxwell, external source, absorbing faces.
    // FP32 path: J = the fixed-point sums, converted once (by Ampere itself
    // when there is no filter)
    ev_begin(s, t, 1);
    const long long *const *jf = f32 ? (const long long *const *)s->jfix : nullptr;
    const double jinv = 1.0 / s->jscale;
    if (s->filter_passes || s->filter_comp) {
        if (f32) {
            launch_j_from_fixed(s->g, (float *const *)J, jf, jinv, s->stream);
            jf = nullptr;
        }
        T *tmp[3];
        for (int c = 0; c < 3; ++c) tmp[c] = (T *)s->filt + (size_t)c * s->g.V;
        launch_filter<T>(s->g, J, tmp, s->filter_passes, s->filter_comp, s->stream);
    }
    if (absorbing) launch_mur_save<T>(s->g, E, (T *)s->mur, s->L.mur_stride, s->stream);
    launch_ampere<T>(s->g, E, B, J, jf, jinv, s->stream);
    if (s->laser.enabled) launch_laser<T>(s->g, E, s->laser, (s->nstep + 0.5) * s->g.dt, s->stream);
    if (absorbing) launch_mur_apply<T>(s->g, E, (const T *)s->mur, s->L.mur_stride, s->stream);
    if (pec) launch_pec<T>(s->g, E, s->stream);
    if (s->port.enabled) launch_port<T>(s->g, E, s->port, (s->nstep + 1) * s->g.dt, s->stream);
    ev_end(s, t);
    s->nstep += 1;
}

// Moving window (FP32 path): at the start of a step, once the window has
// travelled (t - t_start) v >= (shifts + 1) cells d, fields and particles
// move `cells` cells back along the window axis, particles behind it are
// removed, cold plasma is injected into the new cells, and the next sort
// regroups everything.
// Returns false, changing nothing, when the injection would take a species'
// int32 particle ids past 2^31 - 1.
bool window_step(empic_sim *s) {
    const empic_window_desc &W = s->window;
    const int a = W.axis;
    const double t = s->nstep * s->g.dt;
    if ((t - W.t_start) * W.velocity < (double)(s->window_shifts + 1) * W.cells * s->g.d[a])
        return true;
    for (int i = 0; i < s->nsp; ++i) {
        const SpeciesState &S = s->sp[i];
        if (!S.inject) continue;
        long long m = (long long)S.inj_per[0] * S.inj_per[1] * S.inj_per[2] * W.cells;
        for (int b = 0; b < 3; ++b)
            if (b != a) m *= s->g.n[b];
        if (S.next_id + m > 2147483647LL) return false;
    }
    s->window_shifts += 1;
    float *E[3], *B[3], *tmp[3];
    for (int c = 0; c < 3; ++c) {
        E[c] = (float *)s->E[c];
        B[c] = (float *)s->B[c];
        tmp[c] = (float *)s->filt + (size_t)c * s->g.V;
    }
    launch_window_shift<float>(s->g, E, tmp, a, W.cells, false, s->stream);
    launch_window_shift<float>(s->g, B, tmp, a, W.cells, true, s->stream);
    int32_t *reserve = (int32_t *)((char *)s->fault + 32);
    for (int i = 0; i < s->nsp; ++i) {
        SpeciesState &S = s->sp[i];
        const SpeciesP cur = species_params(s, i, S.cur);
        launch_window_particles(cur, a, W.cells, s->stream);
        if (S.inject) {
            int lo[3] = {0, 0, 0}, nc[3] = {s->g.n[0], s->g.n[1], s->g.n[2]};
            lo[a] = s->g.n[a] - W.cells;
            nc[a] = W.cells;
            launch_inject(cur, lo, nc, S.inj_per, (float)S.inj_w, (int)S.next_id, reserve, s->fault,
                          s->stream);
            S.next_id += (long long)nc[0] * S.inj_per[0] * nc[1] * S.inj_per[1] * nc[2] * S.inj_per[2];
        }
        S.tiles_valid = false;
    }
    s->need_sort = true;
    s->rho_prev_step = -1;
    return true;
}

empic_status check_launch(empic_sim *s, const char *what) {
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(s, e, what);
    return EMPIC_OK;
}

empic_status read_fault(empic_sim *s, uint32_t *word) {
    EMPIC_HIP(hipMemcpyAsync(word, s->fault, 4, hipMemcpyDeviceToHost, s->stream));
    EMPIC_HIP(hipStreamSynchronize(s->stream));
    return EMPIC_OK;
}

empic_status fault_status(empic_sim *s, uint32_t w) {
    if (w & EMPIC_FAULT_NONFINITE)
        return fail(s, EMPIC_E_NONFINITE, "non-finite momentum after the push");
    if (w & (EMPIC_FAULT_FAST | EMPIC_FAULT_OFFSET | EMPIC_FAULT_CELL)) {
        char buf[160];
        snprintf(buf, sizeof buf, "corrupted particle state (fault word 0x%x)", w);
        return fail(s, EMPIC_E_STATE, buf);
    }
    if (w & EMPIC_FAULT_CAPACITY)
        return fail(s, EMPIC_E_CAPACITY, "moving-window injection skipped: species capacity");
    return EMPIC_OK;
}

bool aligned16(const void *p) { return ((uintptr_t)p & 15u) == 0; }

// Fixed-point scale of the fused kernel's LDS current window: a power of two
// S with S * B <= 2^48, B the largest current one particle can put on one
// edge in one step, |q| w_max max_a(d_a) / (dt dV) * 13/12 (|dxi| < 1; the
// segment weights are at most 1 + 1/12).  A register run of 4 particles then
// stays below 2^51 (exact conversion) and one edge of a tile window can take
// 2^15 contributions before the int64 sum could overflow.
void update_jscale(empic_sim *s) {
    const double dV = s->g.d[0] * s->g.d[1] * s->g.d[2];
    const double dmax = std::fmax(s->g.d[0], std::fmax(s->g.d[1], s->g.d[2]));
    double B = 0.0;
    for (int i = 0; i < s->nsp; ++i)
        B = std::fmax(B, std::fabs(s->sp[i].desc.q) * s->sp[i].wmax * dmax / (s->g.dt * dV) * 13.0 / 12.0);
    if (!(B > 0.0) || !std::isfinite(B)) {
        s->jscale = 1099511627776.0;
        return;
    }
    s->jscale = std::ldexp(1.0, (int)std::floor(std::log2(std::ldexp(1.0, 48) / B)));
}

// Checks of empic_create and empic_create_static on the grid and sizes; the
// workspace layout on success.
empic_status validate_create(const empic_grid_desc *g, int32_t max_species, int64_t max_capacity,
                             Layout &L) {
    if (max_species < 1 || max_species > EMPIC_MAX_SPECIES || max_capacity < 0) return EMPIC_E_ARG;
    if (g->precision != EMPIC_FP32_CELLREL && g->precision != EMPIC_FP64_PLAIN) return EMPIC_E_ARG;
    double inv2 = 0.0;
    long long V = 1;
    for (int a = 0; a < 3; ++a) {
        if (g->n[a] < 1 || !(g->d[a] > 0.0) || !std::isfinite(g->d[a])) return EMPIC_E_ARG;
        if (g->bc[a] != EMPIC_BC_PERIODIC && g->bc[a] != EMPIC_BC_ABSORBING &&
            g->bc[a] != EMPIC_BC_PEC)
            return EMPIC_E_ARG;
        if (g->bc[a] != EMPIC_BC_PERIODIC && g->n[a] < 2) return EMPIC_E_ARG;
        inv2 += 1.0 / (g->d[a] * g->d[a]);
        V *= g->n[a] + (g->bc[a] != EMPIC_BC_PERIODIC ? 1 : 0);
    }
    if (!(g->dt > 0.0) || !std::isfinite(g->dt)) return EMPIC_E_ARG;
    if (g->dt > (1.0 + 1e-12) / std::sqrt(inv2)) return EMPIC_E_CFL;  // 3D CFL, c = 1
    if (g->sort_every < -1) return EMPIC_E_ARG;
    if (V >= (1LL << 31)) return EMPIC_E_UNSUPPORTED;
    for (int a = 0; a < 3; ++a)  // launch grids put one axis in a grid dimension
        if (g->n[a] + 1 > 65535) return EMPIC_E_UNSUPPORTED;
    // the packed cell index of the FP32 particles (a handle without particles
    // has no such limit)
    if (g->precision == EMPIC_FP32_CELLREL && max_capacity > 0 &&
        (g->n[0] > 2047 || g->n[1] > 2047 || g->n[2] > 1023))
        return EMPIC_E_UNSUPPORTED;
    if (g->precision == EMPIC_FP64_PLAIN && (g->bc[0] || g->bc[1] || g->bc[2]))
        return EMPIC_E_UNSUPPORTED;
    if (max_capacity >= (1LL << 31)) return EMPIC_E_UNSUPPORTED;
    L = layout(g, max_species, max_capacity);
    return EMPIC_OK;
}

// Fill a fresh handle: carve the workspace ws (L.total bytes), zero what the
// kernels expect zero, set up the adaptive sort's host ring.  False on a HIP
// error (the caller releases the handle).
bool init_handle(empic_sim *s, const empic_grid_desc *g, const Layout &L, int32_t max_species,
                 int64_t max_capacity, void *hip_stream, char *ws) {
    s->desc = *g;
    grid_info(g, s->g, s->ti);
    s->L = L;
    s->stream = (hipStream_t)hip_stream;
    s->ws = ws;
    const size_t es = g->precision == EMPIC_FP64_PLAIN ? 8 : 4;
    for (int a = 0; a < 3; ++a) s->Bbar[a] = s->ws + L.Bbar + (size_t)a * s->g.V * es;
    s->fault = (uint32_t *)(s->ws + L.fault);
    s->fallback = (unsigned long long *)(s->ws + L.fault + 8);
    s->table = (DevSpecies *)(s->ws + L.table);
    s->filt = s->ws + L.filt;
    s->xtable = s->table + EMPIC_MAX_SPECIES;
    s->partials = (double *)(s->ws + L.partials);
    s->result = (double *)(s->ws + L.result);
    s->rho_cur = (double *)(s->ws + L.rho_cur);
    s->rho_prev = (double *)(s->ws + L.rho_prev);
    s->counts = (int32_t *)(s->ws + L.counts);
    s->scan_blocks = (int32_t *)(s->ws + L.scan);
    s->rank = (int32_t *)(s->ws + L.rank);
    s->mur = s->ws + L.mur;
    s->fb_mask = (uint32_t *)(s->ws + L.fb_mask);
    s->fb_tiles = (int *)(s->ws + L.fb_tiles);
    s->mask_words = (max_capacity + 31) / 32;
    s->adj = (float *)(s->ws + L.adj);
    if (g->precision == EMPIC_FP32_CELLREL)
        for (int a = 0; a < 3; ++a)
            s->jfix[a] = (unsigned long long *)(s->ws + L.jfix) + (size_t)a * s->g.V;
    s->fb_count = (unsigned *)(s->ws + L.fault + 16);
    s->max_species = max_species;
    s->max_capacity = max_capacity;
    for (int i = 0; i < max_species; ++i) {
        s->sp[i].tile_off = (int32_t *)(s->ws + L.tile_off + (size_t)i * L.tile_off_stride);
        s->sp[i].dcount = s->sp[i].tile_off + (s->ti.ntiles + 1);
    }
    // zero the fault word, counters, the out-of-window marks and the Bbar array
    // (fill kernels; no memset nodes)
    launch_fill_i32((int32_t *)(s->ws + L.fault), 16, 0, s->stream);
    launch_fill_i32((int32_t *)(s->ws + L.fb_mask),
                    (long long)max_species * ((max_capacity + 31) / 32), 0, s->stream);
    launch_fill_i32((int32_t *)(s->ws + L.Bbar), (long long)(3 * s->g.V * es / 4), 0, s->stream);
    bool ok = true;
    if (g->sort_every < 0 && g->precision == EMPIC_FP32_CELLREL) {
        s->adaptive = true;
        // coherent: the device's writes reach host memory without a flush
        ok = hipHostMalloc((void **)&s->fb_host, ADAPT_RING * sizeof(unsigned long long),
                           hipHostMallocMapped | hipHostMallocCoherent) == hipSuccess;
        ok = ok && hipHostGetDevicePointer((void **)&s->fb_dev, s->fb_host, 0) == hipSuccess;
        for (int r = 0; ok && r < ADAPT_RING; ++r) {
            ok = hipEventCreateWithFlags(&s->fb_ev[r], hipEventDisableTiming) == hipSuccess;
            if (ok) s->fb_host[r] = 0;
        }
    }
    if (!ok || hipGetLastError() != hipSuccess) {
        (void)hipGetLastError();
        return false;
    }
    return true;
}

// At most one live handle of empic_create_static per device, on the
// device's copy of `scratch`.
constexpr int STATIC_MAX_DEVICES = 64;
struct StaticSlot {
    char *scratch = nullptr;  // the device address of `scratch` on this device
    bool in_use = false;
    alignas(empic_sim) unsigned char mem[sizeof(empic_sim)];  // the handle itself
};
StaticSlot g_static[STATIC_MAX_DEVICES];
std::mutex g_static_mu;

}  // namespace

extern "C" {

size_t empic_workspace_bytes(const empic_grid_desc *g, int32_t max_species, int64_t max_capacity) {
    if (!g || max_species < 1 || max_species > EMPIC_MAX_SPECIES || max_capacity < 0) return 0;
    for (int a = 0; a < 3; ++a)
        if (g->n[a] < 1) return 0;
    return layout(g, max_species, max_capacity).total;
}

empic_status empic_create(const empic_grid_desc *g, int32_t max_species, int64_t max_capacity,
                          void *hip_stream, void *workspace, size_t workspace_bytes,
                          empic_sim **out) {
    if (!g || !out || !workspace) return EMPIC_E_ARG;
    *out = nullptr;
    Layout L;
    const empic_status st = validate_create(g, max_species, max_capacity, L);
    if (st != EMPIC_OK) return st;
    if (((uintptr_t)workspace & (ALIGN - 1)) != 0) return EMPIC_E_ARG;
    if (workspace_bytes < L.total) return EMPIC_E_ARG;
    empic_sim *s = new empic_sim();
    if (!init_handle(s, g, L, max_species, max_capacity, hip_stream, (char *)workspace)) {
        release_adaptive(s);
        delete s;
        return EMPIC_E_HIP;
    }
    *out = s;
    return EMPIC_OK;
}

empic_status empic_create_static(const empic_grid_desc *g, int32_t max_species,
                                 int64_t max_capacity, void *hip_stream, empic_sim **out) {
    if (!g || !out) return EMPIC_E_ARG;
    *out = nullptr;
    Layout L;
    const empic_status st = validate_create(g, max_species, max_capacity, L);
    if (st != EMPIC_OK) return st;
    if (L.total > (size_t)EMPIC_STATIC_SCRATCH_BYTES) return EMPIC_E_CAPACITY;
    // the adaptive sort policy needs pinned host memory; a fixed cadence does not
    if (g->sort_every < 0 && g->precision == EMPIC_FP32_CELLREL) return EMPIC_E_UNSUPPORTED;
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= STATIC_MAX_DEVICES) return EMPIC_E_HIP;
    if (hip_stream) {
        int sdev = -1;
        if (hipStreamGetDevice((hipStream_t)hip_stream, &sdev) != hipSuccess) return EMPIC_E_HIP;
        if (sdev != dev) return EMPIC_E_ARG;
    }
    std::lock_guard<std::mutex> lock(g_static_mu);
    StaticSlot &slot = g_static[dev];
    if (slot.in_use) return EMPIC_E_ARG;
    if (!slot.scratch) {
        // the device's own copy of the array, looked up once with the device current
        void *p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) {
            (void)hipGetLastError();
            return EMPIC_E_HIP;
        }
        slot.scratch = (char *)p;
    }
    empic_sim *s = new (slot.mem) empic_sim();  // placement: no allocation
    s->static_dev = dev;
    if (!init_handle(s, g, L, max_species, max_capacity, hip_stream, slot.scratch)) {
        s->~empic_sim();
        return EMPIC_E_HIP;
    }
    slot.in_use = true;
    *out = s;
    return EMPIC_OK;
}

empic_status empic_bind_fields(empic_sim *s, void *const E[3], void *const B[3], void *const J[3]) {
    EMPIC_GUARD(s);
    if (!E || !B || !J) return fail(s, EMPIC_E_ARG, "null field array list");
    for (int a = 0; a < 3; ++a)
        if (!E[a] || !B[a] || !J[a]) return fail(s, EMPIC_E_ARG, "null field array");
    for (int a = 0; a < 3; ++a) {
        s->E[a] = E[a];
        s->B[a] = B[a];
        s->J[a] = J[a];
    }
    s->bound = true;
    return EMPIC_OK;
}

empic_status empic_add_species(empic_sim *s, const empic_species_desc *desc, int64_t capacity,
                               const empic_particle_buffers *buf0,
                               const empic_particle_buffers *buf1, int32_t *species_id_out) {
    EMPIC_GUARD(s);
    if (!desc || !buf0) return fail(s, EMPIC_E_ARG, "null species descriptor or buffers");
    if (s->nsp >= s->max_species) return fail(s, EMPIC_E_ARG, "species limit of the handle reached");
    if (!(desc->m > 0.0) || !std::isfinite(desc->q) || !std::isfinite(desc->w))
        return fail(s, EMPIC_E_ARG, "species needs m > 0 and finite q, w");
    if (capacity < 0 || capacity > s->max_capacity)
        return fail(s, EMPIC_E_CAPACITY, "species capacity exceeds the handle's max_capacity");
    if (capacity % 8 != 0) return fail(s, EMPIC_E_ARG, "capacity must be a multiple of 8");
    const bool f32 = !fp64(s);
    const empic_particle_buffers *bufs[2] = {buf0, buf1};
    for (int k = 0; k < 2; ++k) {
        const empic_particle_buffers *b = bufs[k];
        if (!b) continue;
        bool ok = b->pos[0] && b->pos[1] && b->pos[2] && b->u[0] && b->u[1] && b->u[2] && b->id;
        if (f32) ok = ok && b->cell;
        if (desc->per_particle_w) ok = ok && b->w;
        if (!ok) return fail(s, EMPIC_E_ARG, "missing particle buffer");
        if (f32) {
            bool al = aligned16(b->cell);
            for (int a = 0; a < 3; ++a) al = al && aligned16(b->pos[a]) && aligned16(b->u[a]);
            if (desc->per_particle_w) al = al && aligned16(b->w);
            if (!al) return fail(s, EMPIC_E_ARG, "FP32 particle buffers must be 16-byte aligned");
        }
    }
    if (f32 && !buf1) return fail(s, EMPIC_E_ARG, "the FP32 path needs a second buffer set for sorting");
    SpeciesState &S = s->sp[s->nsp];
    S.desc = *desc;
    S.capacity = capacity;
    S.buf[0] = *buf0;
    S.has_alt = buf1 != nullptr;
    if (buf1) S.buf[1] = *buf1;
    S.cur = 0;
    S.host_count = 0;
    launch_fill_i32(S.tile_off, s->ti.ntiles + 2, 0, s->stream);  // offsets and count
    const int id = s->nsp;
    s->nsp += 1;
    S.wmax = desc->per_particle_w ? 0.0 : std::fabs(desc->w);
    DevSpecies D;
    D.p[0] = species_params(s, id, 0);
    D.p[1] = species_params(s, id, S.has_alt ? 1 : 0);
    fill_species_consts(D, s->g, desc->q, desc->m, desc->per_particle_w ? 1.0 : desc->w);
    launch_write_species(s->table + id, D, s->stream);
    if (species_id_out) *species_id_out = id;
    s->need_sort = true;
    return check_launch(s, "add_species");
}

empic_status empic_load_particles_f64(empic_sim *s, int32_t sp, int64_t count,
                                      const double *pos_xyz, const double *u_xyz, const double *w,
                                      const int32_t *ids) {
    EMPIC_GUARD(s);
    if (sp < 0 || sp >= s->nsp) return fail(s, EMPIC_E_ARG, "no such species");
    SpeciesState &S = s->sp[sp];
    if (count < 0 || count > S.capacity) return fail(s, EMPIC_E_CAPACITY, "count exceeds capacity");
    if (count > 0 && (!pos_xyz || !u_xyz)) return fail(s, EMPIC_E_ARG, "null position or momentum");
    if (S.desc.per_particle_w && count > 0 && !w)
        return fail(s, EMPIC_E_ARG, "species takes per-particle weights");
    S.cur = 0;
    const SpeciesP p = species_params(s, sp, 0);
    if (fp64(s)) {
        launch_load_f64(s->g, p, count, pos_xyz, u_xyz, w, ids, s->fault, s->stream);
        launch_fill_i32(S.dcount, 1, (int32_t)count, s->stream);
    } else {
        launch_load_f32(s->g, p, count, pos_xyz, u_xyz, w, ids, s->fault, s->stream);
    }
    S.host_count = count;
    S.next_id = count;
    S.tiles_valid = false;
    s->need_sort = true;
    s->rho_prev_step = -1;
    if (S.desc.per_particle_w && count > 0) {
        launch_absmax_f64(w, count, s->result, s->stream);
        double wm = 0.0;
        EMPIC_HIP(hipGetLastError());
        EMPIC_HIP(hipMemcpyAsync(&wm, s->result, 8, hipMemcpyDeviceToHost, s->stream));
        EMPIC_HIP(hipStreamSynchronize(s->stream));
        S.wmax = std::fmax(S.wmax, wm);
    }
    update_jscale(s);
    return check_launch(s, "load_particles");
}

empic_status empic_store_particles_f64(empic_sim *s, int32_t sp, double *pos_xyz, double *u_xyz,
                                       int32_t *ids, int64_t *count_out) {
    EMPIC_GUARD(s);
    if (sp < 0 || sp >= s->nsp || !pos_xyz || !u_xyz || !count_out)
        return fail(s, EMPIC_E_ARG, "bad store arguments");
    SpeciesState &S = s->sp[sp];
    const SpeciesP p = species_params(s, sp, S.cur);
    if (fp64(s)) {
        launch_store_f64(p, S.host_count, pos_xyz, u_xyz, ids, s->stream);
        EMPIC_HIP(hipGetLastError());
        EMPIC_HIP(hipStreamSynchronize(s->stream));
        *count_out = S.host_count;
    } else {
        launch_store_f32(s->g, p, pos_xyz, u_xyz, ids, s->stream);
        EMPIC_HIP(hipGetLastError());
        int32_t c = 0;
        EMPIC_HIP(hipMemcpyAsync(&c, S.dcount, 4, hipMemcpyDeviceToHost, s->stream));
        EMPIC_HIP(hipStreamSynchronize(s->stream));
        *count_out = c;
    }
    return EMPIC_OK;
}

empic_status empic_current_buffer(empic_sim *s, int32_t sp, int32_t *which) {
    EMPIC_GUARD(s);
    if (sp < 0 || sp >= s->nsp || !which) return fail(s, EMPIC_E_ARG, "bad arguments");
    *which = s->sp[sp].cur;
    return EMPIC_OK;
}

empic_status empic_set_background(empic_sim *s, double rho_bg) {
    EMPIC_GUARD(s);
    if (!std::isfinite(rho_bg)) return fail(s, EMPIC_E_ARG, "non-finite background");
    s->rho_bg = rho_bg;
    return EMPIC_OK;
}

empic_status empic_set_laser(empic_sim *s, const empic_laser_desc *laser) {
    EMPIC_GUARD(s);
    if (!laser) return fail(s, EMPIC_E_ARG, "null laser");
    if (laser->enabled) {
        if (laser->i_s < 0 || laser->i_s > s->g.n[0]) return fail(s, EMPIC_E_ARG, "laser plane outside the grid");
        if (!(laser->tau > 0.0) || !(laser->w0 > 0.0)) return fail(s, EMPIC_E_ARG, "laser needs tau, w0 > 0");
    }
    s->laser = *laser;
    return EMPIC_OK;
}

empic_status empic_set_port(empic_sim *s, const empic_port_desc *port) {
    EMPIC_GUARD(s);
    if (!port) return fail(s, EMPIC_E_ARG, "null port");
    if (port->enabled) {
        const int a = port->axis, c = port->comp, pa = port->prof_axis;
        if (a < 0 || a > 2 || c < 0 || c > 2 || pa < 0 || pa > 2 || c == a || pa == a)
            return fail(s, EMPIC_E_ARG, "port axis, component and profile axis must be transverse");
        if (port->plane < 0 || port->plane >= s->g.ext[a])
            return fail(s, EMPIC_E_ARG, "port plane outside the grid");
        if (!(port->tau > 0.0) || !std::isfinite(port->e0) || !std::isfinite(port->omega))
            return fail(s, EMPIC_E_ARG, "port needs tau > 0 and finite e0, omega");
    }
    s->port = *port;
    return EMPIC_OK;
}

empic_status empic_set_window(empic_sim *s, const empic_window_desc *w) {
    EMPIC_GUARD(s);
    if (!w) return fail(s, EMPIC_E_ARG, "null window");
    if (w->enabled) {
        if (fp64(s)) return fail(s, EMPIC_E_UNSUPPORTED, "the moving window is for the FP32 path");
        if (w->axis < 0 || w->axis > 2 || s->g.bc[w->axis] != EMPIC_BC_ABSORBING)
            return fail(s, EMPIC_E_ARG, "the window moves along an absorbing axis");
        if (w->cells < 1 || w->cells >= s->g.n[w->axis])
            return fail(s, EMPIC_E_ARG, "window shift must be 1 .. n-1 cells");
        if (!(w->velocity > 0.0) || !std::isfinite(w->velocity) || !std::isfinite(w->t_start))
            return fail(s, EMPIC_E_ARG, "window needs a finite velocity > 0 and start time");
    }
    s->window = *w;
    s->window_shifts = 0;
    return EMPIC_OK;
}

empic_status empic_set_injection(empic_sim *s, int32_t sp, const int32_t per_cell[3], double w) {
    EMPIC_GUARD(s);
    if (sp < 0 || sp >= s->nsp || !per_cell) return fail(s, EMPIC_E_ARG, "bad injection species");
    SpeciesState &S = s->sp[sp];
    if (per_cell[0] == 0 && per_cell[1] == 0 && per_cell[2] == 0) {
        S.inject = false;
        return EMPIC_OK;
    }
    for (int a = 0; a < 3; ++a)
        if (per_cell[a] < 1 || per_cell[a] > 64) return fail(s, EMPIC_E_ARG, "1..64 particles per axis");
    if (!(w > 0.0) || !std::isfinite(w)) return fail(s, EMPIC_E_ARG, "injection weight must be > 0");
    if (!S.desc.per_particle_w && std::fabs(w - S.desc.w) > 1e-12 * std::fabs(S.desc.w))
        return fail(s, EMPIC_E_ARG, "a species without per-particle weights injects its own weight");
    S.inject = true;
    for (int a = 0; a < 3; ++a) S.inj_per[a] = per_cell[a];
    S.inj_w = w;
    if (w > S.wmax) {
        S.wmax = w;
        update_jscale(s);
    }
    return EMPIC_OK;
}

empic_status empic_set_filter(empic_sim *s, int32_t passes, int32_t compensate) {
    EMPIC_GUARD(s);
    if (passes < 0 || passes > 16 || (compensate != 0 && compensate != 1))
        return fail(s, EMPIC_E_ARG, "filter: 0..16 binomial passes, compensate 0 or 1");
    s->filter_passes = passes;
    s->filter_comp = compensate;
    return EMPIC_OK;
}

empic_status empic_set_shape_order(empic_sim *s, int32_t order) {
    EMPIC_GUARD(s);
    if (order != 1 && order != 2) return fail(s, EMPIC_E_ARG, "shape order 1 or 2");
    if (order == 2) {
        if (fp64(s))
            return fail(s, EMPIC_E_UNSUPPORTED, "second-order shapes: FP32 path only");
        if (s->g.bc[0] || s->g.bc[1] || s->g.bc[2] || s->ti.slab)
            return fail(s, EMPIC_E_UNSUPPORTED,
                        "second-order shapes: periodic three-dimensional grids only");
    }
    s->g.shape_order = order;
    s->rho_prev_step = -1;  // the next continuity residual compares like with like
    return EMPIC_OK;
}

empic_status empic_sort(empic_sim *s) {
    EMPIC_GUARD(s);
    if (fp64(s)) return EMPIC_OK;  // the plain path keeps its order
    if (s->nsp == 0) return EMPIC_OK;
    do_sort(s);
    return check_launch(s, "sort");
}

empic_status empic_step(empic_sim *s, int32_t nsteps) {
    EMPIC_GUARD(s);
    if (!s->bound) return fail(s, EMPIC_E_ARG, "fields not bound");
    if (nsteps < 0) return fail(s, EMPIC_E_ARG, "negative step count");
    for (int k = 0; k < nsteps; ++k) {
        if (fp64(s)) {
            one_step<double>(s);
        } else {
            if (s->window.enabled && !window_step(s))
                return fail(s, EMPIC_E_CAPACITY,
                            "the injected plasma would take particle ids past 2^31 - 1");
            if (s->adaptive) adaptive_poll(s);
            const int S = s->desc.sort_every;
            if (s->nsp > 0 && (s->need_sort || (S > 0 && s->nstep % S == 0))) do_sort(s);
            const bool publish = s->adaptive && s->nsp > 0;
            one_step<float>(s, nullptr, -1, -1, publish ? adaptive_slot(s) : nullptr);
            if (publish) adaptive_record(s);
        }
    }
    return check_launch(s, "step");
}

empic_status empic_deposit_rho(empic_sim *s, int32_t sp, double *rho_out) {
    EMPIC_GUARD(s);
    if (!rho_out || sp < -1 || sp >= s->nsp) return fail(s, EMPIC_E_ARG, "bad rho arguments");
    launch_zero_f64(rho_out, s->g.V, s->stream);
    for (int i = 0; i < s->nsp; ++i) {
        if (sp >= 0 && i != sp) continue;
        const SpeciesP p = species_params(s, i, s->sp[i].cur);
        if (fp64(s)) {
            launch_rho_f64(s->g, p, s->sp[i].host_count, rho_out, s->stream);
        } else {
            // fixed-point scale of the tile windows: one contribution |q| w / dV <= 2^48
            const double dV = s->g.d[0] * s->g.d[1] * s->g.d[2];
            const double B = std::fabs(s->sp[i].desc.q) * s->sp[i].wmax / dV;
            const double e =
                B > 0.0 && std::isfinite(B) ? std::floor(std::log2(std::ldexp(1.0, 48) / B)) : 0.0;
            const double scale = std::ldexp(1.0, (int)std::fmax(-1000.0, std::fmin(1000.0, e)));
            launch_rho_f32(s->g, s->ti, s->sp[i].tiles_valid, scale, p, rho_out, s->stream);
        }
    }
    return check_launch(s, "deposit_rho");
}

empic_status empic_diagnostics(empic_sim *s, empic_diag *out) {
    EMPIC_GUARD(s);
    if (!out) return fail(s, EMPIC_E_ARG, "null diag");
    if (!s->bound) return fail(s, EMPIC_E_ARG, "fields not bound");
    std::memset(out, 0, sizeof(*out));
    launch_zero_f64(s->partials, (long long)NQ * PSTRIDE, s->stream);
    empic_status st = empic_deposit_rho(s, -1, s->rho_cur);
    if (st != EMPIC_OK) return st;
    const bool cont = s->rho_prev_step >= 0 && s->rho_prev_step == s->nstep - 1;
    if (fp64(s)) {
        double *E[3], *B[3], *J[3], *Bb[3];
        field_ptrs<double>(s, E, B, J, Bb);
        launch_gauss<double>(s->g, E, s->rho_cur, s->rho_bg, s->partials, s->stream);
        if (cont) launch_continuity<double>(s->g, J, s->rho_cur, s->rho_prev, s->partials, s->stream);
        launch_field_energy<double>(s->g, E, B, s->partials, s->stream);
        launch_faraday<double>(s->g, E, B, Bb, nullptr, nullptr, false, s->stream);
        for (int i = 0; i < s->nsp; ++i) {
            const SpeciesP p = species_params(s, i, 0);
            launch_kinetic_f64(p, s->sp[i].host_count, s->partials + (Q_KM + i) * PSTRIDE, s->stream);
            launch_dry_push_f64(s->g, E, Bb, p, s->sp[i].host_count,
                                s->partials + (Q_KP + i) * PSTRIDE, s->fault, s->stream);
        }
    } else {
        float *E[3], *B[3], *J[3], *Bb[3];
        field_ptrs<float>(s, E, B, J, Bb);
        launch_gauss<float>(s->g, E, s->rho_cur, s->rho_bg, s->partials, s->stream);
        if (cont) launch_continuity<float>(s->g, J, s->rho_cur, s->rho_prev, s->partials, s->stream);
        launch_field_energy<float>(s->g, E, B, s->partials, s->stream);
        launch_faraday<float>(s->g, E, B, Bb, nullptr, nullptr, false, s->stream);
        for (int i = 0; i < s->nsp; ++i) {
            const SpeciesP p = species_params(s, i, s->sp[i].cur);
            launch_kinetic_f32(p, s->partials + (Q_KM + i) * PSTRIDE, s->stream);
            launch_dry_push_f32(s->g, E, Bb, p, s->partials + (Q_KP + i) * PSTRIDE, s->fault,
                                s->stream);
        }
    }
    launch_final_reduce(s->partials, s->result, s->stream);
    st = check_launch(s, "diagnostics");
    if (st != EMPIC_OK) return st;
    double res[NQ];
    uint32_t fw[4] = {0, 0, 0, 0};
    EMPIC_HIP(hipMemcpyAsync(res, s->result, sizeof res, hipMemcpyDeviceToHost, s->stream));
    EMPIC_HIP(hipMemcpyAsync(fw, s->fault, 16, hipMemcpyDeviceToHost, s->stream));
    int32_t counts[EMPIC_MAX_SPECIES] = {0, 0, 0, 0};
    for (int i = 0; i < s->nsp; ++i)
        EMPIC_HIP(hipMemcpyAsync(&counts[i], s->sp[i].dcount, 4, hipMemcpyDeviceToHost, s->stream));
    EMPIC_HIP(hipStreamSynchronize(s->stream));
    std::swap(s->rho_cur, s->rho_prev);
    s->rho_prev_step = s->nstep;
    const double dV = s->g.d[0] * s->g.d[1] * s->g.d[2];
    out->step = s->nstep;
    out->t = s->nstep * s->g.dt;
    out->U_E = 0.5 * dV * res[Q_EE];
    out->U_B = 0.5 * dV * res[Q_BB];
    double ksum = 0.0;
    for (int i = 0; i < s->nsp; ++i) {
        out->K_minus[i] = res[Q_KM + i];
        out->K_plus[i] = res[Q_KP + i];
        out->K[i] = 0.5 * (out->K_minus[i] + out->K_plus[i]);
        ksum += out->K[i];
        out->n_particles[i] = fp64(s) ? s->sp[i].host_count : counts[i];
    }
    out->U_tot = out->U_E + out->U_B + ksum;
    long long nodes = s->g.V;
    out->gauss_max = res[Q_GMAX];
    out->gauss_l2 = std::sqrt(res[Q_G2] / (double)nodes);
    out->cont_valid = cont ? 1 : 0;
    out->cont_max = cont ? res[Q_CMAX] : 0.0;
    out->rho_max = cont ? res[Q_RMAX] : 0.0;
    out->fault_word = fw[0];
    out->fallback_particles = (int64_t)(((unsigned long long)fw[3] << 32) | fw[2]);
    return fault_status(s, fw[0]);
}

empic_status empic_particle_count(empic_sim *s, int32_t sp, int64_t *n) {
    EMPIC_GUARD(s);
    if (sp < 0 || sp >= s->nsp || !n) return fail(s, EMPIC_E_ARG, "bad arguments");
    if (fp64(s)) {
        *n = s->sp[sp].host_count;
        return EMPIC_OK;
    }
    int32_t c = 0;
    EMPIC_HIP(hipMemcpyAsync(&c, s->sp[sp].dcount, 4, hipMemcpyDeviceToHost, s->stream));
    EMPIC_HIP(hipStreamSynchronize(s->stream));
    *n = c;
    return EMPIC_OK;
}

empic_status empic_sync(empic_sim *s) {
    EMPIC_GUARD(s);
    EMPIC_HIP(hipGetLastError());
    uint32_t w = 0;
    const empic_status st = read_fault(s, &w);
    if (st != EMPIC_OK) return st;
    return fault_status(s, w);
}

empic_status empic_enable_timing(empic_sim *s, int32_t enable) {
    EMPIC_GUARD(s);
    if (enable < 0 || enable > 2) return fail(s, EMPIC_E_ARG, "timing mode is 0, 1 or 2");
    s->timing = enable;
    return EMPIC_OK;
}

empic_status empic_kernel_times(empic_sim *s, double *push_ms, int64_t *push_launches,
                                double *field_ms, int64_t *field_launches, double *sort_ms,
                                int64_t *sort_launches) {
    EMPIC_GUARD(s);
    EMPIC_HIP(hipStreamSynchronize(s->stream));
    for (TimedEvent &t : s->events) {
        float ms = 0.f;
        EMPIC_HIP(hipEventElapsedTime(&ms, t.a, t.b));
        s->t_ms[t.kind] += ms;
        s->t_n[t.kind] += 1;
        (void)hipEventDestroy(t.a);
        (void)hipEventDestroy(t.b);
    }
    s->events.clear();
    if (push_ms) *push_ms = s->t_ms[0];
    if (push_launches) *push_launches = s->t_n[0];
    if (field_ms) *field_ms = s->t_ms[1];
    if (field_launches) *field_launches = s->t_n[1];
    if (sort_ms) *sort_ms = s->t_ms[2];
    if (sort_launches) *sort_launches = s->t_n[2];
    for (int k = 0; k < 3; ++k) {
        s->t_ms[k] = 0;
        s->t_n[k] = 0;
    }
    return EMPIC_OK;
}

static empic_status copy_state(empic_sim *s, const empic_state *st, bool save) {
    const size_t fb = (size_t)s->g.V * 4;
    auto cp = [&](void *state_arr, void *live, size_t n) {
        return hipMemcpyAsync(save ? state_arr : live, save ? live : state_arr, n,
                              hipMemcpyDeviceToDevice, s->stream);
    };
    for (int a = 0; a < 3; ++a)
        if (!st->E[a] || !st->B[a]) return fail(s, EMPIC_E_ARG, "null state field");
    for (int i = 0; i < s->nsp; ++i) {
        const SpeciesState &S = s->sp[i];
        if (S.capacity == 0) continue;
        bool ok = st->cell[i] && st->id[i] && st->tiles[i];
        for (int a = 0; a < 3; ++a) ok = ok && st->pos[i][a] && st->u[i][a];
        if (S.desc.per_particle_w) ok = ok && st->w[i];
        if (!ok) return fail(s, EMPIC_E_ARG, "null state particle array");
    }
    for (int a = 0; a < 3; ++a) {
        EMPIC_HIP(cp(st->E[a], s->E[a], fb));
        EMPIC_HIP(cp(st->B[a], s->B[a], fb));
    }
    for (int i = 0; i < s->nsp; ++i) {
        const SpeciesState &S = s->sp[i];
        const empic_particle_buffers &b = S.buf[S.cur];
        const size_t pb = (size_t)S.capacity * 4;
        if (pb == 0) continue;
        EMPIC_HIP(cp(st->cell[i], b.cell, pb));
        EMPIC_HIP(cp(st->id[i], b.id, pb));
        for (int a = 0; a < 3; ++a) {
            EMPIC_HIP(cp(st->pos[i][a], b.pos[a], pb));
            EMPIC_HIP(cp(st->u[i][a], b.u[a], pb));
        }
        if (S.desc.per_particle_w) EMPIC_HIP(cp(st->w[i], b.w, pb));
        // tile offsets and the slot count after them
        EMPIC_HIP(cp(st->tiles[i], S.tile_off, ((size_t)s->ti.ntiles + 2) * 4));
    }
    return EMPIC_OK;
}

empic_status empic_state_tile_words(empic_sim *s, int64_t *words) {
    EMPIC_GUARD(s);
    if (!words) return fail(s, EMPIC_E_ARG, "null output");
    *words = (int64_t)s->ti.ntiles + 2;
    return EMPIC_OK;
}

empic_status empic_save_state(empic_sim *s, const empic_state *dst) {
    EMPIC_GUARD(s);
    if (!dst || !s->bound) return fail(s, EMPIC_E_ARG, "null state or fields not bound");
    if (fp64(s)) return fail(s, EMPIC_E_UNSUPPORTED, "states are for the FP32 path");
    if (s->nsp > 0 && s->need_sort)
        return fail(s, EMPIC_E_ARG, "sort the particles before saving a state");
    return copy_state(s, dst, true);
}

empic_status empic_load_state(empic_sim *s, const empic_state *src) {
    EMPIC_GUARD(s);
    if (!src || !s->bound) return fail(s, EMPIC_E_ARG, "null state or fields not bound");
    if (fp64(s)) return fail(s, EMPIC_E_UNSUPPORTED, "states are for the FP32 path");
    const empic_status st = copy_state(s, src, false);
    if (st != EMPIC_OK) return st;
    // a saved state is grouped by its own tile offsets
    for (int i = 0; i < s->nsp; ++i) s->sp[i].tiles_valid = true;
    s->need_sort = false;
    s->rho_prev_step = -1;
    return EMPIC_OK;
}

empic_status empic_sort_recorded(empic_sim *s, int32_t *const perm[EMPIC_MAX_SPECIES]) {
    EMPIC_GUARD(s);
    if (!perm) return fail(s, EMPIC_E_ARG, "null permutation arrays");
    if (fp64(s)) return fail(s, EMPIC_E_UNSUPPORTED, "the FP64 path does not sort");
    for (int i = 0; i < s->nsp; ++i)
        if (s->sp[i].capacity > 0 && !perm[i]) return fail(s, EMPIC_E_ARG, "null permutation array");
    if (s->nsp == 0) return EMPIC_OK;
    do_sort(s, perm);
    return check_launch(s, "sort_recorded");
}

empic_status empic_sort_vjp(empic_sim *s, int32_t *const perm[EMPIC_MAX_SPECIES],
                            const empic_adjoint *lam) {
    EMPIC_GUARD(s);
    if (!perm || !lam) return fail(s, EMPIC_E_ARG, "null permutation or adjoint");
    if (fp64(s)) return fail(s, EMPIC_E_UNSUPPORTED, "the FP64 path does not sort");
    for (int i = 0; i < s->nsp; ++i) {
        const SpeciesState &S = s->sp[i];
        if (S.capacity == 0) continue;
        float *lx[3], *lu[3], *scratch[6];
        bool ok = perm[i] != nullptr && S.has_alt;
        const empic_particle_buffers &alt = S.buf[1 - S.cur];
        for (int a = 0; a < 3; ++a) {
            lx[a] = (float *)lam->pos[i][a];
            lu[a] = (float *)lam->u[i][a];
            scratch[a] = (float *)alt.pos[a];
            scratch[3 + a] = (float *)alt.u[a];
            ok = ok && lx[a] && lu[a];
        }
        if (!ok) return fail(s, EMPIC_E_ARG, "null permutation or adjoint array");
        launch_sort_vjp(perm[i], S.capacity, lx, lu, scratch, s->stream);
    }
    return check_launch(s, "sort_vjp");
}

empic_status empic_step_vjp(empic_sim *s, const empic_state *st, const empic_adjoint *lam) {
    EMPIC_GUARD(s);
    if (!st || !lam || !s->bound) return fail(s, EMPIC_E_ARG, "null state or adjoint");
    if (fp64(s) || s->g.bc[0] || s->g.bc[1] || s->g.bc[2])
        return fail(s, EMPIC_E_UNSUPPORTED, "the adjoint needs the FP32 path on a periodic grid");
    if (s->g.shape_order != 1)
        return fail(s, EMPIC_E_UNSUPPORTED, "the adjoint is of the first-order (CIC) step");
    float *E[3], *B[3], *Bb[3], *lE[3], *lB[3], *lEg[3], *lBb[3], *tB[3];
    for (int a = 0; a < 3; ++a) {
        E[a] = (float *)st->E[a];
        B[a] = (float *)st->B[a];
        Bb[a] = (float *)s->Bbar[a];
        lE[a] = (float *)lam->E[a];
        lB[a] = (float *)lam->B[a];
        lEg[a] = s->adj + (size_t)a * s->g.V;
        lBb[a] = s->adj + (size_t)(3 + a) * s->g.V;
        tB[a] = s->adj + (size_t)(6 + a) * s->g.V;
        if (!E[a] || !B[a] || !lE[a] || !lB[a]) return fail(s, EMPIC_E_ARG, "null field array");
    }
    // centred B of the state
    launch_faraday<float>(s->g, E, B, Bb, nullptr, nullptr, false, s->stream);
    SpeciesP sp[EMPIC_MAX_SPECIES];
    const int32_t *tiles[EMPIC_MAX_SPECIES] = {};
    float *lx[EMPIC_MAX_SPECIES][3], *lu[EMPIC_MAX_SPECIES][3];
    for (int i = 0; i < s->nsp; ++i) {
        sp[i] = species_params(s, i, s->sp[i].cur);
        if (s->sp[i].capacity > 0) {
            if (!st->cell[i] || !st->tiles[i])
                return fail(s, EMPIC_E_ARG, "null state cell or tile array");
            if (s->sp[i].desc.per_particle_w && !st->w[i])
                return fail(s, EMPIC_E_ARG, "null state weight array");
            sp[i].cell = (uint32_t *)st->cell[i];
            sp[i].w = st->w[i];
            tiles[i] = st->tiles[i];
        }
        for (int a = 0; a < 3; ++a) {
            sp[i].pos[a] = st->pos[i][a];
            sp[i].u[a] = st->u[i][a];
            lx[i][a] = (float *)lam->pos[i][a];
            lu[i][a] = (float *)lam->u[i][a];
            if (s->sp[i].capacity > 0 && (!sp[i].pos[a] || !sp[i].u[a] || !lx[i][a] || !lu[i][a]))
                return fail(s, EMPIC_E_ARG, "null particle array in state or adjoint");
        }
    }
    // scratch free between steps and sorts: the step kernels' out-of-window
    // list, each species' second buffer set (its offsets and momenta) for the
    // per-particle gather adjoints, the sort-key counters for tile exponents
    float *l6[EMPIC_MAX_SPECIES][6] = {};
    for (int i = 0; i < s->nsp; ++i) {
        const SpeciesState &S = s->sp[i];
        if (S.capacity == 0) continue;
        if (!S.has_alt) return fail(s, EMPIC_E_ARG, "the adjoint needs the second buffer set");
        const empic_particle_buffers &alt = S.buf[1 - S.cur];
        for (int a = 0; a < 3; ++a) {
            l6[i][a] = (float *)alt.pos[a];
            l6[i][3 + a] = (float *)alt.u[a];
        }
    }
    // with a current filter F between deposit and Ampere the deposit's adjoint
    // is F^T lam_E' = F lam_E' (the stencils are symmetric); tB is free until
    // the transposed curls, so it serves as the filter's second buffer
    float *lJdep[3] = {lE[0], lE[1], lE[2]};
    if (s->filter_passes || s->filter_comp) {
        float *fl[3];
        for (int a = 0; a < 3; ++a) {
            fl[a] = (float *)s->filt + (size_t)a * s->g.V;
            EMPIC_HIP(hipMemcpyAsync(fl[a], lE[a], (size_t)s->g.V * 4, hipMemcpyDeviceToDevice,
                                     s->stream));
        }
        launch_filter<float>(s->g, fl, tB, s->filter_passes, s->filter_comp, s->stream);
        for (int a = 0; a < 3; ++a) lJdep[a] = fl[a];
    }
    launch_step_vjp(s->g, s->ti, E, Bb, lE, lJdep, lB, lEg, lBb, tB, sp, tiles, lx, lu, s->nsp,
                    s->fb_mask, s->fb_count, l6, s->counts, s->stream);
    return check_launch(s, "step_vjp");
}

empic_status empic_step_state(empic_sim *s, const empic_state *src, const empic_state *dst) {
    EMPIC_GUARD(s);
    if (!src || !dst || !s->bound) return fail(s, EMPIC_E_ARG, "null state or fields not bound");
    if (fp64(s)) return fail(s, EMPIC_E_UNSUPPORTED, "states are for the FP32 path");
    if (src == dst) return fail(s, EMPIC_E_ARG, "source and destination must differ");
    // a state carries no time: a step whose sources or window depend on it
    // cannot be taken from a state
    if (s->laser.enabled || s->port.enabled || s->window.enabled)
        return fail(s, EMPIC_E_UNSUPPORTED,
                    "step_state: a laser, port or moving window depends on the step's time");
    for (int a = 0; a < 3; ++a)
        if (!src->E[a] || !src->B[a] || !dst->E[a] || !dst->B[a])
            return fail(s, EMPIC_E_ARG, "null state field");
    for (int i = 0; i < s->nsp; ++i) {
        const SpeciesState &S = s->sp[i];
        if (S.capacity == 0) continue;
        const empic_state *st[2] = {src, dst};
        for (const empic_state *x : st) {
            bool ok = x->cell[i] && x->id[i] && x->tiles[i];
            for (int a = 0; a < 3; ++a) ok = ok && x->pos[i][a] && x->u[i][a];
            if (S.desc.per_particle_w) ok = ok && x->w[i];
            bool al = aligned16(x->cell[i]);
            for (int a = 0; a < 3; ++a) al = al && aligned16(x->pos[i][a]) && aligned16(x->u[i][a]);
            if (!ok) return fail(s, EMPIC_E_ARG, "null state particle array");
            if (!al) return fail(s, EMPIC_E_ARG, "state particle arrays must be 16-byte aligned");
        }
        if (dst->cell[i] == src->cell[i]) return fail(s, EMPIC_E_ARG, "source and destination overlap");
    }
    // fields of the source into the destination's arrays, which the step then
    // updates in place (the handle's own E and B are not touched)
    {
        const float *from[6];
        float *to[6];
        for (int a = 0; a < 3; ++a) {
            from[a] = (const float *)src->E[a];
            from[3 + a] = (const float *)src->B[a];
            to[a] = (float *)dst->E[a];
            to[3 + a] = (float *)dst->B[a];
        }
        launch_copy6(from, to, s->g.V, s->stream);
    }
    // species table: set 0 = source state, set 1 = destination state
    const size_t tw = ((size_t)s->ti.ntiles + 2) * 4;
    for (int i = 0; i < s->nsp; ++i) {
        const SpeciesState &S = s->sp[i];
        DevSpecies D;
        const empic_state *st[2] = {src, dst};
        for (int k = 0; k < 2; ++k) {
            SpeciesP p = species_params(s, i, S.cur);
            p.cell = (uint32_t *)st[k]->cell[i];
            for (int a = 0; a < 3; ++a) {
                p.pos[a] = st[k]->pos[i][a];
                p.u[a] = st[k]->u[i][a];
            }
            p.id = st[k]->id[i];
            p.w = S.desc.per_particle_w ? st[k]->w[i] : nullptr;
            p.tile_off = st[k]->tiles[i];
            p.count = st[k]->tiles[i] ? st[k]->tiles[i] + s->ti.ntiles + 1 : nullptr;
            D.p[k] = p;
        }
        fill_species_consts(D, s->g, S.desc.q, S.desc.m, S.desc.per_particle_w ? 1.0 : S.desc.w);
        launch_write_species(s->xtable + i, D, s->stream);
        if (S.capacity == 0) continue;
        const size_t pb = (size_t)S.capacity * 4;
        EMPIC_HIP(hipMemcpyAsync(dst->tiles[i], src->tiles[i], tw, hipMemcpyDeviceToDevice, s->stream));
        if (dst->id[i] != src->id[i])
            EMPIC_HIP(hipMemcpyAsync(dst->id[i], src->id[i], pb, hipMemcpyDeviceToDevice, s->stream));
        if (S.desc.per_particle_w && dst->w[i] != src->w[i])
            EMPIC_HIP(hipMemcpyAsync(dst->w[i], src->w[i], pb, hipMemcpyDeviceToDevice, s->stream));
    }
    // the handle's own clock (diagnostics, sort schedule) does not move
    const long long nstep = s->nstep;
    void *E0[3], *B0[3];
    for (int a = 0; a < 3; ++a) {
        E0[a] = s->E[a];
        B0[a] = s->B[a];
        s->E[a] = dst->E[a];
        s->B[a] = dst->B[a];
    }
    one_step<float>(s, s->xtable, 0, (int)((1u << s->nsp) - 1u));
    for (int a = 0; a < 3; ++a) {
        s->E[a] = E0[a];
        s->B[a] = B0[a];
    }
    s->nstep = nstep;
    s->rho_prev_step = -1;
    return check_launch(s, "step_state");
}

empic_status empic_dot_f64(empic_sim *s, const float *a, const float *b, int64_t n, double *out) {
    EMPIC_GUARD(s);
    if (!out || n < 0 || (n > 0 && (!a || !b))) return fail(s, EMPIC_E_ARG, "bad dot arguments");
    static_assert(RED_BLOCKS <= PSTRIDE, "dot partials fit one slot");
    double *partials = s->partials + (size_t)Q_DOT * PSTRIDE;
    launch_dot_f64(a, b, (long long)n, partials, s->result + Q_DOT, s->stream);
    const empic_status st = check_launch(s, "dot_f64");
    if (st != EMPIC_OK) return st;
    EMPIC_HIP(hipMemcpyAsync(out, s->result + Q_DOT, 8, hipMemcpyDeviceToHost, s->stream));
    EMPIC_HIP(hipStreamSynchronize(s->stream));
    return EMPIC_OK;
}

void empic_tile_shape(int32_t out[3]) {
    if (!out) return;
    out[0] = TileCube::TX;
    out[1] = TileCube::TY;
    out[2] = TileCube::TZ;
}

void empic_grid_tile_shape(const empic_grid_desc *g, int32_t out[3]) {
    if (!g || !out) return;
    int t[3], slab;
    tile_shape_of(g, t, slab);
    for (int a = 0; a < 3; ++a) out[a] = t[a];
}

const char *empic_last_error(const empic_sim *s) { return s ? s->err.c_str() : "null handle"; }

void empic_destroy(empic_sim *s) {
    if (!s) return;
    release_adaptive(s);
    for (TimedEvent &t : s->events) {
        (void)hipEventDestroy(t.a);
        (void)hipEventDestroy(t.b);
    }
    if (s->static_dev >= 0) {
        std::lock_guard<std::mutex> lock(g_static_mu);
        StaticSlot &slot = g_static[s->static_dev];
        s->~empic_sim();
        slot.in_use = false;
        return;
    }
    delete s;
}

}  // extern "C"
