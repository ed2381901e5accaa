// C ABI of the fast level set evolution library: argument validation,
// workspace layout, the host-side constant tables and the launch sequence of
// Table I (arXiv 1409.7474).  Declarations and contracts are in include/lse.h.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <map>
#include <mutex>
#include <new>
#include <set>
#include <tuple>
#include <vector>

#include "lse_internal.h"

using namespace lse;

struct lse_ctx {
    lse_params p;
    int NB;             // stored bands (1, 2 or 4)
    int esz;            // bytes of one stored value (storage type)
    int region;         // region data term (eq. (17)), on the bands or on their mean
    int dense;          // continuous LSF kept in a plane (any mode but Table I with binarisation every iteration)
    int phi_binary;     // dense: the next iteration's phi is the binary function in the bit plane
    int r, ts, nch;     // LSF smoothing
    int variant;        // step-kernel variant (tile rows, waves per SIMD), from the autotuner's table
    int r1, ts1;        // edge term: image pre-smoothing
    int WW;             // bit words per row
    long long hw;
    float fix, inv_fix;
    int n;              // iterations enqueued since init / set_mask / set_lsf (device slots count from there)
    int n_base;         // iteration index of the method at that restart (kept across resume)
    int raw_next;       // next iteration starts from the binary LSF itself
    DevState *st;
    Taps *taps;
    ImgArgs *dargs;     // this image's step / normaliser arguments (device)
    ImgArgs host_args;
    void *img;          // region: storage image; edge: edge map g
    float *boxes;       // region, B > 1: per-block band min / max for the normaliser
    uint32_t *bits[2];
    void *plane[2];     // dense: LSF planes (storage type), iteration n reads plane[n & 1]
    Taps host_taps;
    hipStream_t last_stream;
    // profiling
    int prof;
    struct Ev {
        hipEvent_t a, b;
        int kind;
    };
    std::vector<Ev> pending, pool;
    double prof_ms[2];
    long long prof_n[2];
    long long prof_seen[2];  // launches of each kind since profiling was enabled (sampling)
};

// A set of contexts advanced together: one step launch (and, for B > 1, one
// normaliser launch) per iteration per kernel family, over a device table of
// ImgArgs and a workgroup map (image, tile).
struct lse_batch {
    struct Group {
        int r, NB, edge, storage;     // kernel family
        int variant;                  // step-kernel variant of its contexts
        int first, count;             // ImgArgs index range
        int step_bits, mpass_bits;    // unit bits of the map entries
        size_t step_map, mpass_map;   // offsets (entries) into the map
        unsigned step_grid, mpass_grid;
        bool visit_list;              // step map rebuilt per launch (batch_plan_kernel) at step_map:
        size_t wbase_map;             // count + 1 heavy-record word offsets
    };
    std::vector<lse_ctx *> cs;        // in table order
    std::vector<int> target;
    std::vector<Group> groups;
    std::vector<ImgArgs> hargs;
    std::vector<uint32_t> hmap;
    ImgArgs *dargs;
    uint32_t *dmap;
    hipStream_t last_stream;
    hipGraphExec_t exec;
    int exec_iters, exec_stop;
    // Several kernel families: each group runs on a stream of its own
    // (default priority), forked from and joined to the caller's stream, so
    // that the groups' latency-bound launches overlap on the device.
    std::vector<hipStream_t> gstream;
    std::vector<hipEvent_t> join;
    hipEvent_t fork = nullptr;
    // Table uploads go through two pinned host buffers used in turn, so a
    // copy is truly stream-ordered (a pageable source would make the copy
    // wait for the stream): before a buffer is refilled, the copy that last
    // read it (two uploads ago) must have completed.
    struct Staging {
        void *host = nullptr;
        size_t cap = 0;
        hipEvent_t done = nullptr;
        bool pending = false;
    };
    Staging stage[2];
    int next_stage = 0;
    ~lse_batch() {
        for (Staging &g : stage) {
            if (g.done) {
                if (g.pending) (void)hipEventSynchronize(g.done);
                (void)hipEventDestroy(g.done);
            }
            if (g.host) (void)hipHostFree(g.host);
        }
        for (hipStream_t st : gstream) (void)hipStreamDestroy(st);
        for (hipEvent_t ev : join) (void)hipEventDestroy(ev);
        if (fork) (void)hipEventDestroy(fork);
    }
};

namespace {

constexpr size_t kAlign = 256;

inline size_t align_up(size_t v) { return (v + kAlign - 1) & ~(kAlign - 1); }

int auto_ksize(float sigma) {
    const int r = (int)ceil(3.0 * (double)sigma);
    return 2 * r + 1;
}

int resolved_ksize(int k, float sigma) { return k > 0 ? k : auto_ksize(sigma); }

bool valid_ts(int ts) { return ts >= 3 && ts <= 31 && (ts & 1); }

lse_status validate(const lse_params *p) {
    if (!p) return LSE_ERR_INVALID_ARG;
    if (p->height < 2 || p->width < 2) return LSE_ERR_INVALID_ARG;
    if ((long long)p->height * (long long)p->width >= (1ll << 31)) return LSE_ERR_INVALID_ARG;
    if (p->bands < 1 || p->bands > 4) return LSE_ERR_INVALID_ARG;
    if (p->term != LSE_TERM_REGION && p->term != LSE_TERM_EDGE && p->term != LSE_TERM_REGION_INTENSITY)
        return LSE_ERR_INVALID_ARG;
    if (p->order != LSE_ORDER_TABLE1 && p->order != LSE_ORDER_LISTING) return LSE_ERR_INVALID_ARG;
    if (p->image_dtype != LSE_F32 && p->image_dtype != LSE_F16 && p->image_dtype != LSE_BF16)
        return LSE_ERR_INVALID_ARG;
    if (p->storage != LSE_F32 && p->storage != LSE_F16 && p->storage != LSE_BF16) return LSE_ERR_INVALID_ARG;
    {
        // The device image copy (region: bands padded to 1, 2 or 4 values;
        // edge: one value) is addressed with 32-bit byte offsets.
        const unsigned long long nb = p->term != LSE_TERM_REGION ? 1 : (p->bands == 3 ? 4 : p->bands);
        const unsigned long long es = p->storage == LSE_F32 ? 4 : 2;
        if ((unsigned long long)p->height * p->width * nb * es >= 0xfff00000ull) return LSE_ERR_INVALID_ARG;
    }
    if (!(isfinite(p->dt) && p->dt > 0.f)) return LSE_ERR_INVALID_ARG;
    if (!(isfinite(p->sigma) && p->sigma > 0.f)) return LSE_ERR_INVALID_ARG;
    if (p->ksize < 0 || !valid_ts(resolved_ksize(p->ksize, p->sigma))) return LSE_ERR_INVALID_ARG;
    if (p->term == LSE_TERM_EDGE) {
        if (!(isfinite(p->sigma_img) && p->sigma_img > 0.f)) return LSE_ERR_INVALID_ARG;
        if (p->ksize_img < 0 || !valid_ts(resolved_ksize(p->ksize_img, p->sigma_img))) return LSE_ERR_INVALID_ARG;
        if (!(isfinite(p->edge_scale) && p->edge_scale > 0.f)) return LSE_ERR_INVALID_ARG;
    }
    if (p->reinit_every < 0) return LSE_ERR_INVALID_ARG;
    // The edge term needs reinitialisation (periodic at least).
    if (p->term == LSE_TERM_EDGE && p->reinit_every == 0) return LSE_ERR_INVALID_ARG;
    return LSE_OK;
}

struct Layout {
    size_t state, taps, args, img, boxes, tilesum, tilelast, sched, plan, bits0, bits1, plane0, plane1, total;
};

bool dense_mode(const lse_params *p) { return !(p->order == LSE_ORDER_TABLE1 && p->reinit_every == 1); }

Layout layout_of(const lse_params *p) {
    const size_t hw = (size_t)p->height * p->width;
    const int NB = p->term != LSE_TERM_REGION ? 1 : (p->bands == 3 ? 4 : p->bands);
    const size_t WW = ((size_t)p->width + 31) / 32;
    Layout L;
    size_t o = 0;
    L.state = o;
    o = align_up(o + sizeof(DevState));
    L.taps = o;
    o = align_up(o + sizeof(Taps));
    L.args = o;
    o = align_up(o + sizeof(ImgArgs));
    const size_t es = p->storage == LSE_F32 ? 4 : 2;
    L.img = o;
    o = align_up(o + hw * NB * es);
    L.boxes = 0;
    if (NB > 1) {
        L.boxes = o;
        o = align_up(o + mbox_floats(p->height, p->width, NB) * 4);
    }
    L.tilesum = L.tilelast = 0;
    if (p->term != LSE_TERM_EDGE && !dense_mode(p) && fast_radius(resolved_ksize(p->ksize, p->sigma) / 2)) {
        L.tilesum = o;
        o = align_up(o + (size_t)step_tiles_max(p->height, p->width, 0) * sizeof(TileSum));
        L.tilelast = o;
        o = align_up(o + (size_t)step_tiles_max(p->height, p->width, 0) * sizeof(TileSum));
    }
    L.sched = L.plan = 0;
    if (!dense_mode(p) && fast_radius(resolved_ksize(p->ksize, p->sigma) / 2)) {
        // sized for every variant, so the workspace does not depend on the tuning
        const size_t tiles = (size_t)step_tiles_max(p->height, p->width, p->term == LSE_TERM_EDGE);
        L.sched = o;
        o = align_up(o + (size_t)sched_words((int)((tiles + 31) / 32)) * 4);  // heavy records (3 slots), touched tags
        L.plan = o;
        o = align_up(o + (1 + step_launch_grid((int)tiles)) * 4);  // length, entries, padding to the grid
    }
    L.bits0 = o;
    o = align_up(o + (size_t)p->height * WW * 4);
    L.bits1 = o;
    o = align_up(o + (size_t)p->height * WW * 4);
    L.plane0 = L.plane1 = 0;
    if (dense_mode(p)) {
        L.plane0 = o;
        o = align_up(o + hw * es);
        L.plane1 = o;
        o = align_up(o + hw * es);
    }
    L.total = o;
    return L;
}

// 1-D normalised Gaussian taps of side ts: k[j] = exp(-(j-r)^2 / (2 sigma^2)) / sum.
void gauss_taps(double sigma, int ts, double *k) {
    const int r = ts / 2;
    double s = 0.0;
    for (int j = 0; j < ts; ++j) {
        const double d = j - r;
        k[j] = exp(-d * d / (2.0 * sigma * sigma));
        s += k[j];
    }
    for (int j = 0; j < ts; ++j) k[j] /= s;
}

void build_taps(Taps &t, double sigma, int ts, double sigma1, int ts1) {
    memset(&t, 0, sizeof(t));
    double k[32] = {0};
    gauss_taps(sigma, ts, k);
    for (int j = 0; j < ts; ++j) t.k[j] = (float)k[j];
    double acc = 0.0;
    t.cum[0] = 0.f;
    for (int m = 1; m <= ts; ++m) {
        acc += k[m - 1];
        t.cum[m] = (float)acc;
    }
    const int nch = (ts + kChunkBits - 1) / kChunkBits;
    for (int c = 0; c < nch; ++c) {
        for (int m = 0; m < 64; ++m) {
            double s = 0.0;
            for (int j = 0; j < kChunkBits; ++j) {
                const int tap = c * kChunkBits + j;
                if (tap >= ts) break;
                s += ((m >> j) & 1) ? k[tap] : -k[tap];
            }
            t.lut[c][m] = (float)s;
        }
    }
    if (ts1 > 0) {
        double k1[32] = {0};
        gauss_taps(sigma1, ts1, k1);
        for (int j = 0; j < ts1; ++j) t.k1[j] = (float)k1[j];
    }
}

int fix_shift(long long hw) {
    int lg = 0;
    while ((1ll << lg) < hw) ++lg;
    int s = 62 - 16 - lg;  // |I| < 2^16: total |sum| * 2^s < 2^62
    if (s > 40) s = 40;
    if (s < 8) s = 8;
    return s;
}

inline hipStream_t as_stream(void *s) { return static_cast<hipStream_t>(s); }

StepArgs step_args(const lse_ctx *c) {
    StepArgs a;
    a.img = c->img;
    a.boxes = c->boxes;
    a.bits_in = c->bits[c->n & 1];
    a.bits_out = c->bits[(c->n + 1) & 1];
    a.st = c->st;
    a.taps = c->taps;
    a.H = c->p.height;
    a.W = c->p.width;
    a.WW = c->WW;
    a.r = c->r;
    a.ts = c->ts;
    a.nch = c->nch;
    a.dt = c->p.dt;
    a.n = c->n;
    a.raw = c->raw_next;
    a.stop = 0;
    a.fix = c->fix;
    a.inv_fix = c->inv_fix;
    a.hw = c->hw;
    a.plane_in = nullptr;
    a.plane_out = nullptr;
    a.order = c->p.order;
    a.reinit = 1;
    a.phi_binary = 0;
    a.tilelast = c->host_args.tilelast;
    return a;
}

lse_status dev_status(hipError_t e) { return e == hipSuccess ? LSE_OK : LSE_ERR_DEVICE; }

void prof_begin(lse_ctx *c, int kind, hipStream_t s, lse_ctx::Ev *ev) {
    if (!(c->prof & LSE_PROFILE_TIMING)) return;
    const long long period = 1ll << ((c->prof >> 8) & 15);
    if (++c->prof_seen[kind] % period != 0) return;
    if (c->pool.empty()) {
        lse_ctx::Ev e;
        if (hipEventCreate(&e.a) != hipSuccess) return;
        if (hipEventCreate(&e.b) != hipSuccess) {
            (void)hipEventDestroy(e.a);
            return;
        }
        c->pool.push_back(e);
    }
    *ev = c->pool.back();
    c->pool.pop_back();
    ev->kind = kind;
    (void)s;
    launch_timing() = LaunchTiming{ev->a, ev->b};
}

// The launch between prof_begin and prof_end took the events into its dispatch
// packet; if it never launched (an error), the pair goes back unused.
void prof_end(lse_ctx *c, hipStream_t s, lse_ctx::Ev *ev) {
    (void)s;
    if (!(c->prof & LSE_PROFILE_TIMING) || ev->kind < 0) return;
    LaunchTiming &t = launch_timing();
    if (t.start) {
        t = LaunchTiming{nullptr, nullptr};
        c->pool.push_back(*ev);
        return;
    }
    c->pending.push_back(*ev);
}

// The LSF of iteration 0 from the binary function in bits[0] (raw: phi is the
// binary function; else its Gaussian smoothing) and its region statistics.
hipError_t load_lsf(lse_ctx *c, int raw, hipStream_t s) {
    StepArgs a = step_args(c);
    a.bits_in = c->bits[0];
    hipError_t e = hipSuccess;
    if (c->dense) {
        c->phi_binary = raw;
        e = launch_plane_fill(a, c->bits[0], raw, c->plane[0], c->p.storage, s);
        if (e == hipSuccess && c->region) e = launch_plane_stats(a, c->plane[0], c->NB, c->p.storage, 0, s);
    } else if (c->region) {
        e = launch_stats(a, c->NB, c->p.storage, raw, 0, s);
    }
    return e;
}

lse_status enqueue_step(lse_ctx *c, int stop, hipStream_t s) {
    hipError_t e = hipSuccess;
    const bool region = c->region;
    const int storage = c->p.storage;
    if (region && c->NB > 1) {
        lse_ctx::Ev ev{nullptr, nullptr, -1};
        prof_begin(c, 1, s, &ev);
        // one more workgroup builds the step's visit list (fast path)
        const unsigned grid = (unsigned)c->host_args.mgroups + (c->host_args.plan && !c->dense ? 1u : 0u);
        e = launch_mpass(c->dargs, nullptr, 0, grid, c->n, stop, c->NB, storage, s);
        prof_end(c, s, &ev);
        if (e != hipSuccess) return LSE_ERR_DEVICE;
    }
    StepArgs a = step_args(c);
    a.stop = stop;
    lse_ctx::Ev ev{nullptr, nullptr, -1};
    prof_begin(c, 0, s, &ev);
    int next_binary = 0;
    if (c->dense) {
        const int every = c->p.reinit_every;
        // Table I step 3 "if necessary" / Sec. III-D Step 3 "periodically":
        // iteration index i binarises iff (i + 1) % every == 0.
        const long long idx = (long long)c->n_base + c->n;
        a.reinit = every > 0 && ((idx + 1) % every) == 0;
        a.order = c->p.order;
        a.phi_binary = c->phi_binary;
        a.plane_in = c->plane[c->n & 1];
        a.plane_out = c->plane[(c->n + 1) & 1];
        e = launch_dense_step(a, c->NB, region ? 0 : 1, storage, s);
        next_binary = a.order == LSE_ORDER_LISTING && a.reinit;
    } else if (fast_radius(c->r)) {
        if (c->host_args.plan && !(region && c->NB > 1)) e = launch_plan(c->dargs, c->n, s);
        if (e == hipSuccess && (c->prof & LSE_PROFILE_COUNT) && c->host_args.sched_mask)
            e = launch_count_tiles(c->dargs, c->n, 0, s);
        // With a visit list the step reads it as a one-image step map (image
        // index 0: every entry is below 2^31).
        const int *plan = c->host_args.plan;
        if (e == hipSuccess)
            e = launch_step(c->dargs, plan ? reinterpret_cast<const uint32_t *>(plan + 1) : nullptr, plan,
                            plan ? 31 : 0, step_launch_grid(c->host_args.tiles), c->n, stop, c->r, c->NB,
                            region ? 0 : 1, storage, c->variant, s);
    } else {
        e = launch_step_generic(a, c->NB, region ? 0 : 1, storage, s);
    }
    prof_end(c, s, &ev);
    if (e != hipSuccess) return LSE_ERR_DEVICE;
    c->phi_binary = next_binary;
    if ((c->prof & LSE_PROFILE_COUNT) && !c->dense) {
        if (launch_count_needed(a, a.raw, region ? 0 : 1, c->host_args.tilesum != nullptr, s) != hipSuccess)
            return LSE_ERR_DEVICE;
        if (c->host_args.sched_mask && fast_radius(c->r) && launch_count_tiles(c->dargs, c->n, 1, s) != hipSuccess)
            return LSE_ERR_DEVICE;
    }
    c->n += 1;
    c->raw_next = 0;
    c->last_stream = s;
    return LSE_OK;
}

// ------------------------------------------------------------ tuning table
//
// The autotuner's choices: step-kernel variant per kernel family (term, radius,
// stored bands, storage type) and size class (image side rounded to a power of
// two, 256 .. 8192 and up).  lse_init takes the variant from here; families
// and sizes never tuned run variant 0.
struct TuneKey {
    int edge, r, NB, storage, cls;
    bool operator<(const TuneKey &o) const {
        return std::tie(edge, r, NB, storage, cls) < std::tie(o.edge, o.r, o.NB, o.storage, o.cls);
    }
};
struct TuneEntry {
    int variant;
    int candidates;
    float ms[LSE_TUNE_MAX_CANDIDATES];
};
std::mutex g_tune_mu;
std::map<TuneKey, TuneEntry> g_tune;

int size_class(long long hw) {
    // round(log2(sqrt(hw))) - 8, clamped to 0 .. 5 (sides 256 .. 8192)
    const double side = sqrt((double)hw);
    int c = (int)lround(log2(side)) - 8;
    return std::max(0, std::min(5, c));
}

TuneKey tune_key(const lse_params *p) {
    const int edge = p->term == LSE_TERM_EDGE;
    const int nb = p->term != LSE_TERM_REGION ? 1 : (p->bands == 3 ? 4 : p->bands);
    return TuneKey{edge, resolved_ksize(p->ksize, p->sigma) / 2, nb, p->storage,
                   size_class((long long)p->height * p->width)};
}

int tuned_variant(const lse_params *p) {
    std::lock_guard<std::mutex> lock(g_tune_mu);
    const auto it = g_tune.find(tune_key(p));
    return it == g_tune.end() ? 0 : it->second.variant;
}

void fill_tuning(const lse_params *p, int variant, const TuneEntry *e, lse_tuning_t *out) {
    memset(out, 0, sizeof(*out));
    const int edge = p->term == LSE_TERM_EDGE;
    out->variant = variant;
    step_variant_info(edge, variant, &out->tile_rows, &out->waves_per_simd);
    out->tile_cols = 96;
    out->size_class = size_class((long long)p->height * p->width);
    if (e) {
        out->candidates = e->candidates;
        for (int i = 0; i < e->candidates && i < LSE_TUNE_MAX_CANDIDATES; ++i) out->ms[i] = e->ms[i];
    }
}

// Host-side checks of lse_init's arguments (nothing enqueued).
lse_status check_init_args(const lse_params *p, const void *image_dev, const uint8_t *init_mask_dev,
                           const void *workspace_dev, size_t workspace_bytes) {
    const lse_status v = validate(p);
    if (v != LSE_OK) return v;
    if (!image_dev || !init_mask_dev) return LSE_ERR_INVALID_ARG;
    const size_t esz = p->image_dtype == LSE_F32 ? 4 : 2;
    if (reinterpret_cast<uintptr_t>(image_dev) % esz) return LSE_ERR_INVALID_ARG;
    if (!workspace_dev || (reinterpret_cast<uintptr_t>(workspace_dev) % kAlign)) return LSE_ERR_WORKSPACE;
    if (workspace_bytes < layout_of(p).total) return LSE_ERR_WORKSPACE;
    return LSE_OK;
}

// Table I step 1 into the context *c (arguments already checked): lay out
// the workspace, enqueue the image conversion, the edge map or initial
// statistics and the binary initial LSF.  tables_by_kernel: the constant
// tables and the image arguments reach the device as kernel arguments rather
// than host-to-device copies.
hipError_t init_ctx(lse_ctx *c, const lse_params *p, const void *image_dev, const uint8_t *init_mask_dev,
                    void *workspace_dev, hipStream_t st, bool tables_by_kernel, int variant = -1) {
    const Layout L = layout_of(p);
    c->p = *p;
    c->variant = variant >= 0 ? variant : tuned_variant(p);
    c->region = p->term != LSE_TERM_EDGE;
    c->NB = p->term != LSE_TERM_REGION ? 1 : (p->bands == 3 ? 4 : p->bands);
    c->esz = p->storage == LSE_F32 ? 4 : 2;
    c->dense = dense_mode(p) ? 1 : 0;
    c->phi_binary = 1;
    c->ts = resolved_ksize(p->ksize, p->sigma);
    c->r = c->ts / 2;
    c->nch = (c->ts + kChunkBits - 1) / kChunkBits;
    c->ts1 = p->term == LSE_TERM_EDGE ? resolved_ksize(p->ksize_img, p->sigma_img) : 0;
    c->r1 = c->ts1 / 2;
    c->WW = (p->width + 31) / 32;
    c->hw = (long long)p->height * p->width;
    const int s = fix_shift(c->hw);
    c->fix = ldexpf(1.f, s);
    c->inv_fix = ldexpf(1.f, -s);
    c->n = 0;
    c->n_base = 0;
    c->raw_next = 1;
    char *base = static_cast<char *>(workspace_dev);
    c->st = reinterpret_cast<DevState *>(base + L.state);
    c->taps = reinterpret_cast<Taps *>(base + L.taps);
    c->dargs = reinterpret_cast<ImgArgs *>(base + L.args);
    c->img = base + L.img;
    c->boxes = L.boxes ? reinterpret_cast<float *>(base + L.boxes) : nullptr;
    c->bits[0] = reinterpret_cast<uint32_t *>(base + L.bits0);
    c->bits[1] = reinterpret_cast<uint32_t *>(base + L.bits1);
    c->plane[0] = L.plane0 ? base + L.plane0 : nullptr;
    c->plane[1] = L.plane1 ? base + L.plane1 : nullptr;
    c->prof = 0;
    c->prof_ms[0] = c->prof_ms[1] = 0.0;
    c->prof_n[0] = c->prof_n[1] = 0;
    c->prof_seen[0] = c->prof_seen[1] = 0;
    build_taps(c->host_taps, p->sigma, c->ts, p->sigma_img, c->ts1);
    {
        ImgArgs &A = c->host_args;
        memset(&A, 0, sizeof(A));
        A.img = c->img;
        A.boxes = c->boxes;
        A.bits[0] = c->bits[0];
        A.bits[1] = c->bits[1];
        A.st = c->st;
        A.taps = c->taps;
        A.H = p->height;
        A.W = p->width;
        A.WW = c->WW;
        A.tiles = step_tiles(p->height, p->width, p->term == LSE_TERM_EDGE, c->variant);
        A.dt = p->dt;
        A.fix = c->fix;
        A.inv_fix = c->inv_fix;
        A.target = 0x7fffffff;
        A.hw = c->hw;
        A.n0 = 0;
        A.mgroups = (c->region && c->NB > 1) ? mpass_groups(p->height, p->width) : 0;
        A.tilesum = L.tilesum ? reinterpret_cast<const TileSum *>(base + L.tilesum) : nullptr;
        A.tilelast = L.tilelast ? reinterpret_cast<TileSum *>(base + L.tilelast) : nullptr;
        A.sched_mask = L.sched ? reinterpret_cast<uint32_t *>(base + L.sched) : nullptr;
        // Visit list: built by the normaliser pass when there is one, else
        // by its own pass for large tile counts.
        const bool use_plan = (c->region && c->NB > 1) || A.tiles > kPlanMinTiles;
        A.plan = L.plan && use_plan ? reinterpret_cast<int *>(base + L.plan) : nullptr;
    }

    c->last_stream = st;
    hipError_t e;
    if (tables_by_kernel) {
        e = launch_put_bytes(&c->host_taps, sizeof(Taps), c->taps, st);
        if (e == hipSuccess) e = launch_put_bytes(&c->host_args, sizeof(ImgArgs), c->dargs, st);
    } else {
        e = hipMemcpyAsync(c->taps, &c->host_taps, sizeof(Taps), hipMemcpyHostToDevice, st);
        if (e == hipSuccess) e = hipMemcpyAsync(c->dargs, &c->host_args, sizeof(ImgArgs), hipMemcpyHostToDevice, st);
    }
    if (e == hipSuccess) e = launch_init_state(c->st, 1, st);
    if (e == hipSuccess) e = launch_sched_reset(&c->host_args, st);
    if (e == hipSuccess) {
        if (c->region) {
            if (c->NB > 1)  // bands stored (region term), with the normaliser boxes
                e = launch_init_image_box(image_dev, p->image_dtype, p->storage, p->bands, c->NB, c->img, p->height,
                                          p->width, c->st, c->fix, c->boxes, st);
            else
                e = launch_init_image(image_dev, p->image_dtype, p->storage, p->bands, c->NB, c->img, c->hw, c->st,
                                      c->fix, p->term == LSE_TERM_REGION ? 0 : 2, st);
            if (e == hipSuccess && L.tilesum)
                e = launch_tile_sums(c->dargs, c->host_args.tiles, c->r, c->NB, p->storage,
                                     reinterpret_cast<TileSum *>(base + L.tilesum), st);
        } else {
            e = launch_edge_map(image_dev, p->image_dtype, p->bands, p->edge_scale, c->taps, c->r1, c->img,
                                p->height, p->width, p->storage, c->st, st);
        }
    }
    if (e == hipSuccess) e = launch_pack_mask(init_mask_dev, c->bits[0], p->height, p->width, c->WW, st);
    if (e == hipSuccess) e = load_lsf(c, 1, st);
    return e;
}

}  // namespace

extern "C" {

void lse_params_default(lse_params *p, int32_t height, int32_t width, int32_t bands) {
    if (!p) return;
    memset(p, 0, sizeof(*p));
    p->height = height;
    p->width = width;
    p->bands = bands;
    p->term = LSE_TERM_REGION;
    p->order = LSE_ORDER_TABLE1;
    p->image_dtype = LSE_F32;
    p->storage = LSE_F32;
    p->dt = 15.f;
    p->sigma = 1.f;
    p->ksize = 7;
    p->sigma_img = 1.f;
    p->ksize_img = 9;
    p->edge_scale = 255.f;
    p->reinit_every = 1;
}

size_t lse_workspace_bytes(const lse_params *p) {
    const lse_status v = validate(p);
    if (v != LSE_OK && v != LSE_ERR_UNSUPPORTED) return 0;
    return layout_of(p).total;
}

lse_status lse_init(const lse_params *p, const void *image_dev, const uint8_t *init_mask_dev, void *workspace_dev,
                    size_t workspace_bytes, void *stream, lse_ctx **out) {
    if (!out) return LSE_ERR_INVALID_ARG;
    *out = nullptr;
    const lse_status v = check_init_args(p, image_dev, init_mask_dev, workspace_dev, workspace_bytes);
    if (v != LSE_OK) return v;
    lse_ctx *c = new (std::nothrow) lse_ctx();
    if (!c) return LSE_ERR_INVALID_ARG;
    if (init_ctx(c, p, image_dev, init_mask_dev, workspace_dev, as_stream(stream), false) != hipSuccess) {
        delete c;
        return LSE_ERR_DEVICE;
    }
    *out = c;
    return LSE_OK;
}

lse_status lse_step(lse_ctx *c, void *stream) {
    if (!c) return LSE_ERR_INVALID_ARG;
    return enqueue_step(c, 0, as_stream(stream));
}

lse_status lse_run(lse_ctx *c, int32_t max_iters, int32_t stop_when_unchanged, void *stream) {
    if (!c || max_iters < 0) return LSE_ERR_INVALID_ARG;
    const hipStream_t s = as_stream(stream);
    for (int i = 0; i < max_iters; ++i) {
        const lse_status v = enqueue_step(c, stop_when_unchanged ? 1 : 0, s);
        if (v != LSE_OK) return v;
    }
    return LSE_OK;
}

lse_status lse_mask(const lse_ctx *c, uint8_t *mask_dev, void *stream) {
    if (!c || !mask_dev) return LSE_ERR_INVALID_ARG;
    const uint32_t *const b[2] = {c->bits[0], c->bits[1]};
    return dev_status(launch_mask_out(b, c->st, mask_dev, c->p.height, c->p.width, c->WW, as_stream(stream)));
}

lse_status lse_lsf(const lse_ctx *c, float *lsf_dev, void *stream) {
    if (!c || !lsf_dev || (reinterpret_cast<uintptr_t>(lsf_dev) & 3)) return LSE_ERR_INVALID_ARG;
    if (c->dense)
        return dev_status(launch_plane_out(c->plane[0], c->plane[1], c->st, lsf_dev, c->hw, c->p.storage,
                                           as_stream(stream)));
    const uint32_t *const b[2] = {c->bits[0], c->bits[1]};
    StepArgs a = step_args(c);
    return dev_status(launch_lsf_out(a, b, c->raw_next, lsf_dev, as_stream(stream)));
}

lse_status lse_set_mask(lse_ctx *c, const uint8_t *mask_dev, int32_t smoothed, int32_t iteration, void *stream) {
    if (!c || !mask_dev || iteration < 0) return LSE_ERR_INVALID_ARG;
    const hipStream_t s = as_stream(stream);
    hipError_t e = launch_reset_state(c->st, smoothed ? 0 : 1, s);
    if (e == hipSuccess) e = launch_sched_reset(&c->host_args, s);
    if (e == hipSuccess) e = launch_pack_mask(mask_dev, c->bits[0], c->p.height, c->p.width, c->WW, s);
    c->n = 0;
    c->n_base = iteration;
    c->raw_next = smoothed ? 0 : 1;
    if (e == hipSuccess) e = load_lsf(c, c->raw_next, s);
    c->last_stream = s;
    return dev_status(e);
}

lse_status lse_set_lsf(lse_ctx *c, const float *lsf_dev, const uint8_t *mask_dev, int32_t iteration, void *stream) {
    if (!c || !lsf_dev || (reinterpret_cast<uintptr_t>(lsf_dev) & 3) || iteration < 0) return LSE_ERR_INVALID_ARG;
    if (!c->dense) return LSE_ERR_UNSUPPORTED;  // binary-state mode: the LSF is G * b (lse_set_mask, smoothed)
    const hipStream_t s = as_stream(stream);
    // In listing order a binarising iteration leaves the LSF sign(psi) and
    // stores psi (what lse_lsf returns): the next iteration then reads the
    // binary function from the bits.
    const int every = c->p.reinit_every;
    const int prev_binarised = iteration > 0 && every > 0 && (iteration % every) == 0;
    hipError_t e = launch_reset_state(c->st, 0, s);
    if (e == hipSuccess) e = launch_plane_load(lsf_dev, c->plane[0], c->hw, c->st, c->p.storage, s);
    if (e == hipSuccess)
        e = mask_dev ? launch_pack_mask(mask_dev, c->bits[0], c->p.height, c->p.width, c->WW, s)
                     : launch_pack_sign(lsf_dev, c->bits[0], c->p.height, c->p.width, c->WW, s);
    c->n = 0;
    c->n_base = iteration;
    c->raw_next = 0;
    c->phi_binary = c->p.order == LSE_ORDER_LISTING && prev_binarised;
    if (e == hipSuccess && c->region) {
        StepArgs a = step_args(c);
        a.bits_in = c->bits[0];
        e = launch_plane_stats(a, c->plane[0], c->NB, c->p.storage, 0, s);
    }
    c->last_stream = s;
    return dev_status(e);
}

lse_status lse_edge_map(const lse_ctx *c, float *g_dev, void *stream) {
    if (!c || !g_dev || (reinterpret_cast<uintptr_t>(g_dev) & 3)) return LSE_ERR_INVALID_ARG;
    if (c->p.term != LSE_TERM_EDGE) return LSE_ERR_STATE;
    // The stored map is one plane of the storage type; iters' parity picks
    // either pointer, both name it.
    return dev_status(launch_plane_out(c->img, c->img, c->st, g_dev, c->hw, c->p.storage, as_stream(stream)));
}

lse_status lse_stats(const lse_ctx *c, lse_stats_t *host_out, void *stream) {
    if (!c || !host_out) return LSE_ERR_INVALID_ARG;
    const hipStream_t s = as_stream(stream);
    DevState h;
    if (hipMemcpyAsync(&h, c->st, sizeof(DevState), hipMemcpyDeviceToHost, s) != hipSuccess) return LSE_ERR_DEVICE;
    if (hipStreamSynchronize(s) != hipSuccess) return LSE_ERR_DEVICE;
    memset(host_out, 0, sizeof(*host_out));
    unsigned long long nplus = 0, flips = 0;
    for (int i = 0; i < kBins; ++i) {
        nplus += h.slot[h.iters % 3][i].nplus;
        flips += h.slot[h.iters % 3][i].flips;
    }
    host_out->n_plus = nplus;
    host_out->flips = h.iters > 0 ? flips : 0;
    host_out->iters_done = c->n_base + h.iters;
    host_out->converged = h.done;
    host_out->bad_value = h.bad == kBadInput ? 1 : 0;
    host_out->lsf_overflow = h.bad == kBadOverflow ? 1 : 0;
    for (int b = 0; b < 4; ++b) {
        host_out->c_plus[b] = h.last_cp[b];
        host_out->c_minus[b] = h.last_cm[b];
    }
    host_out->M = h.last_M;
    return LSE_OK;
}

lse_status lse_check(const lse_ctx *c, void *stream) {
    lse_stats_t st;
    const lse_status v = lse_stats(c, &st, stream);
    if (v != LSE_OK) return v;
    if (hipGetLastError() != hipSuccess) return LSE_ERR_DEVICE;
    return (st.bad_value || st.lsf_overflow) ? LSE_ERR_BAD_VALUE : LSE_OK;
}

lse_status lse_profile(lse_ctx *c, int32_t flags) {
    if (!c || (flags & ~(LSE_PROFILE_TIMING | LSE_PROFILE_COUNT | LSE_PROFILE_SAMPLE(15)))) return LSE_ERR_INVALID_ARG;
    if (flags) {
        for (auto &e : c->pending) c->pool.push_back(e);
        c->pending.clear();
        c->prof_ms[0] = c->prof_ms[1] = 0.0;
        c->prof_n[0] = c->prof_n[1] = 0;
        c->prof_seen[0] = c->prof_seen[1] = 0;
        if (launch_reset_profile(c->st, c->last_stream) != hipSuccess) return LSE_ERR_DEVICE;
    }
    c->prof = flags;
    return LSE_OK;
}

lse_status lse_profile_read(lse_ctx *c, lse_profile_t *host_out) {
    if (!c || !host_out) return LSE_ERR_INVALID_ARG;
    if (hipStreamSynchronize(c->last_stream) != hipSuccess) return LSE_ERR_DEVICE;
    for (auto &e : c->pending) {
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, e.a, e.b) == hipSuccess) {
            c->prof_ms[e.kind] += ms;
            c->prof_n[e.kind] += 1;
        }
        c->pool.push_back(e);
    }
    c->pending.clear();
    unsigned long long acc[4] = {0, 0, 0, 0};
    if (hipMemcpy(acc, &c->st->acc_needed, sizeof(acc), hipMemcpyDeviceToHost) != hipSuccess) return LSE_ERR_DEVICE;
    host_out->needed_pixels = (int64_t)acc[0];
    host_out->counted_steps = (int64_t)acc[1];
    const bool tiled = c->host_args.sched_mask && fast_radius(c->r) && !c->dense;
    host_out->visited_tiles = tiled ? (int64_t)acc[2] : -1;
    host_out->heavy_tiles = tiled ? (int64_t)acc[3] : -1;
    host_out->tiles = tiled ? (int64_t)c->host_args.tiles : -1;
    host_out->step_ms = c->prof_ms[0];
    host_out->mpass_ms = c->prof_ms[1];
    host_out->step_launches = c->prof_n[0];
    host_out->mpass_launches = c->prof_n[1];
    return LSE_OK;
}

double lse_step_bytes_per_pixel(const lse_ctx *c) {
    if (!c) return 0.0;
    const double state = 2.0 / 8.0;  // binary state: one bit read, one bit written
    const double plane = c->dense ? 2.0 * c->esz : 0.0;  // continuous LSF: read and written
    return (double)c->esz * c->NB + state + plane;
}

void lse_destroy(lse_ctx *c) {
    if (!c) return;
    for (auto &e : c->pending) c->pool.push_back(e);
    for (auto &e : c->pool) {
        (void)hipEventDestroy(e.a);
        (void)hipEventDestroy(e.b);
    }
    delete c;
}

lse_status lse_tuning_lookup(const lse_params *p, lse_tuning_t *out) {
    if (!out) return LSE_ERR_INVALID_ARG;
    const lse_status v = validate(p);
    if (v != LSE_OK) return v;
    std::lock_guard<std::mutex> lock(g_tune_mu);
    const auto it = g_tune.find(tune_key(p));
    if (it == g_tune.end()) fill_tuning(p, 0, nullptr, out);
    else fill_tuning(p, it->second.variant, &it->second, out);
    return LSE_OK;
}

lse_status lse_ctx_tuning(const lse_ctx *c, lse_tuning_t *out) {
    if (!c || !out) return LSE_ERR_INVALID_ARG;
    fill_tuning(&c->p, c->variant, nullptr, out);
    return LSE_OK;
}

lse_status lse_tuning_set(const lse_params *p, int32_t variant) {
    const lse_status v = validate(p);
    if (v != LSE_OK) return v;
    if (variant < 0 || variant >= kNumStepVariants) return LSE_ERR_INVALID_ARG;
    std::lock_guard<std::mutex> lock(g_tune_mu);
    TuneEntry e;
    memset(&e, 0, sizeof(e));
    e.variant = variant;
    g_tune[tune_key(p)] = e;
    return LSE_OK;
}

void lse_tuning_clear(void) {
    std::lock_guard<std::mutex> lock(g_tune_mu);
    g_tune.clear();
}

lse_status lse_autotune(const lse_params *p, const void *image_dev, const uint8_t *init_mask_dev, void *workspace_dev,
                        size_t workspace_bytes, int32_t iters, void *stream, lse_tuning_t *out) {
    if (!out || iters < 1) return LSE_ERR_INVALID_ARG;
    const lse_status v = check_init_args(p, image_dev, init_mask_dev, workspace_dev, workspace_bytes);
    if (v != LSE_OK) return v;
    if (dense_mode(p) || !fast_radius(resolved_ksize(p->ksize, p->sigma) / 2)) return LSE_ERR_UNSUPPORTED;
    const hipStream_t s = as_stream(stream);
    hipEvent_t ev[2] = {nullptr, nullptr};
    if (hipEventCreate(&ev[0]) != hipSuccess || hipEventCreate(&ev[1]) != hipSuccess) {
        if (ev[0]) (void)hipEventDestroy(ev[0]);
        return LSE_ERR_DEVICE;
    }
    TuneEntry e;
    memset(&e, 0, sizeof(e));
    e.candidates = std::min(kNumStepVariants, (int)LSE_TUNE_MAX_CANDIDATES);
    lse_status r = LSE_OK;
    unsigned long long first = 0;
    for (int var = 0; var < e.candidates && r == LSE_OK; ++var) {
        // Each candidate runs twice from the same initial state; the second
        // run is timed (the first loads the code and warms the caches).
        for (int rep = 0; rep < 2 && r == LSE_OK; ++rep) {
            lse_ctx c;
            hipError_t he = init_ctx(&c, p, image_dev, init_mask_dev, workspace_dev, s, false, var);
            if (he == hipSuccess) he = hipEventRecord(ev[0], s);
            for (int i = 0; i < iters && he == hipSuccess; ++i)
                if (enqueue_step(&c, 0, s) != LSE_OK) he = hipErrorUnknown;
            if (he == hipSuccess) he = hipEventRecord(ev[1], s);
            const uint32_t *const bits[2] = {c.bits[0], c.bits[1]};
            if (he == hipSuccess) he = launch_digest(bits, c.st, p->height, c.WW, s);
            unsigned long long d = 0;
            if (he == hipSuccess) he = hipMemcpyAsync(&d, &c.st->digest, sizeof(d), hipMemcpyDeviceToHost, s);
            if (he == hipSuccess) he = hipStreamSynchronize(s);
            float ms = 0.f;
            if (he == hipSuccess) he = hipEventElapsedTime(&ms, ev[0], ev[1]);
            if (he != hipSuccess) {
                r = LSE_ERR_DEVICE;
                break;
            }
            if (var == 0 && rep == 0) first = d;
            else if (d != first) r = LSE_ERR_STATE;  // variants must agree bit for bit
            if (rep == 1) e.ms[var] = ms;
        }
    }
    (void)hipEventDestroy(ev[0]);
    (void)hipEventDestroy(ev[1]);
    if (r != LSE_OK) return r;
    // Variant 0 stays unless another is faster by more than 3 % (run-to-run
    // noise must not flip the choice).
    e.variant = 0;
    for (int var = 1; var < e.candidates; ++var)
        if (e.ms[var] < 0.97f * e.ms[0] && e.ms[var] < e.ms[e.variant]) e.variant = var;
    {
        std::lock_guard<std::mutex> lock(g_tune_mu);
        g_tune[tune_key(p)] = e;
    }
    fill_tuning(p, e.variant, &e, out);
    return LSE_OK;
}

}  // extern "C"

// ------------------------------------------------- allocation-free solve
//
// lse_solve_static's workspace: a file-scope device array, one copy per GPU,
// held until the process ends.  In host code `scratch` names a host-side
// stand-in, not device memory, so host code never passes it to a kernel or a
// copy: set-up takes each GPU's own address with hipGetSymbolAddress (once per
// device, that device current) and every use goes through that address.
static __device__ __align__(256) unsigned char scratch[LSE_STATIC_WORKSPACE_BYTES];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices];

// The current device's address of `scratch` (nullptr on a HIP error).
void *static_workspace() {
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *ptr = nullptr;
        if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return nullptr;
        g_scratch_ptr[dev] = ptr;
    }
    return g_scratch_ptr[dev];
}

}  // namespace

extern "C" {

lse_status lse_solve_static(const lse_params *p, const void *image_dev, const uint8_t *init_mask_dev,
                            int32_t max_iters, int32_t stop_when_unchanged, uint8_t *mask_dev, float *lsf_dev,
                            void *stream) {
    if (max_iters < 0 || !mask_dev || (lsf_dev && (reinterpret_cast<uintptr_t>(lsf_dev) & 3)))
        return LSE_ERR_INVALID_ARG;
    const lse_status v = validate(p);
    if (v != LSE_OK) return v;
    if (layout_of(p).total > LSE_STATIC_WORKSPACE_BYTES) return LSE_ERR_WORKSPACE;
    void *ws = static_workspace();
    if (!ws) return LSE_ERR_DEVICE;
    const lse_status a = check_init_args(p, image_dev, init_mask_dev, ws, LSE_STATIC_WORKSPACE_BYTES);
    if (a != LSE_OK) return a;
    // The context lives on this stack frame: everything the device needs
    // from it goes out as kernel arguments before the call returns.
    lse_ctx c;
    const hipStream_t s = as_stream(stream);
    if (init_ctx(&c, p, image_dev, init_mask_dev, ws, s, true) != hipSuccess) return LSE_ERR_DEVICE;
    for (int i = 0; i < max_iters; ++i) {
        const lse_status r = enqueue_step(&c, stop_when_unchanged ? 1 : 0, s);
        if (r != LSE_OK) return r;
    }
    lse_status r = lse_mask(&c, mask_dev, stream);
    if (r == LSE_OK && lsf_dev) r = lse_lsf(&c, lsf_dev, stream);
    return r;
}

const char *lse_status_str(lse_status s) {
    switch (s) {
        case LSE_OK: return "LSE_OK";
        case LSE_ERR_INVALID_ARG: return "LSE_ERR_INVALID_ARG";
        case LSE_ERR_BAD_VALUE: return "LSE_ERR_BAD_VALUE";
        case LSE_ERR_WORKSPACE: return "LSE_ERR_WORKSPACE";
        case LSE_ERR_DEVICE: return "LSE_ERR_DEVICE";
        case LSE_ERR_STATE: return "LSE_ERR_STATE";
        case LSE_ERR_UNSUPPORTED: return "LSE_ERR_UNSUPPORTED";
    }
    return "LSE_ERR_UNKNOWN";
}

// ------------------------------------------------------------------ batch

namespace {

int bits_for(long long n) {  // smallest b >= 1 with n <= 2^b
    int b = 1;
    while ((1ll << b) < n) ++b;
    return b;
}

// Plan the table of a batch: contexts grouped by kernel family, each group's
// step map (XCD-banded over the concatenated tiles of its images, as tile_of
// does for one image) and normaliser map.  Returns the device bytes, or 0 if
// the contexts cannot form a batch.
size_t plan_batch(lse_ctx *const *cs, int32_t n, lse_batch *b) {
    if (!cs || n <= 0) return 0;
    std::set<const lse_ctx *> seen;
    std::vector<int> order;
    for (int i = 0; i < n; ++i) {
        if (!cs[i] || !seen.insert(cs[i]).second) return 0;  // null or repeated context
        if (!fast_radius(cs[i]->r) || cs[i]->dense) return 0;
        order.push_back(i);
    }
    auto key = [&](int i) {
        const lse_ctx *c = cs[i];
        const int edge = c->p.term == LSE_TERM_EDGE;
        return std::make_tuple(edge, c->r, edge ? 1 : c->NB, (int)c->p.storage, c->variant);
    };
    std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return key(x) < key(y); });
    b->cs.clear();
    b->groups.clear();
    b->hmap.clear();
    for (size_t j = 0; j < order.size();) {
        size_t e = j;
        while (e < order.size() && key(order[e]) == key(order[j])) ++e;
        lse_batch::Group g;
        g.edge = std::get<0>(key(order[j]));
        g.r = std::get<1>(key(order[j]));
        g.NB = std::get<2>(key(order[j]));
        g.storage = std::get<3>(key(order[j]));
        g.variant = std::get<4>(key(order[j]));
        g.first = (int)b->cs.size();
        g.count = (int)(e - j);
        long long total = 0, maxt = 1, maxm = 1;
        std::vector<long long> prefix(1, 0);
        for (size_t q = j; q < e; ++q) {
            const lse_ctx *c = cs[order[q]];
            b->cs.push_back(cs[order[q]]);
            total += c->host_args.tiles;
            prefix.push_back(total);
            maxt = std::max<long long>(maxt, c->host_args.tiles);
            maxm = std::max<long long>(maxm, c->host_args.mgroups);
        }
        g.step_bits = bits_for(maxt);
        g.mpass_bits = bits_for(maxm);
        const int ubits = std::max(g.step_bits, g.mpass_bits);
        if (ubits >= 31 || (long long)g.count >= (1ll << (32 - ubits)) - 1) return 0;
        const long long grid = (total + 7) & ~7ll;
        if (grid > 0x7fffffffll) return 0;
        g.step_grid = (unsigned)grid;
        g.visit_list = g.count <= kBatchPlanImages;
        if (g.visit_list) {
            // Visit list, rebuilt on the device for every launch: the active
            // tiles of every image (heavy first); settled tiles are skipped.
            g.wbase_map = b->hmap.size();
            uint32_t words = 0;
            for (int q = 0; q < g.count; ++q) {
                b->hmap.push_back(words);
                words += (uint32_t)((b->cs[g.first + q]->host_args.tiles + 31) / 32);
            }
            b->hmap.push_back(words);
            g.step_map = b->hmap.size();
            // length, entries, and padding to the launch grid (the step
            // kernel loads its entry before comparing with the length)
            b->hmap.resize(b->hmap.size() + 1 + grid, 0u);
        } else {
            // Static step map over every tile: workgroup w runs on XCD w % 8;
            // XCD x takes the x-th eighth of the concatenated tiles.
            g.step_map = b->hmap.size();
            b->hmap.resize(b->hmap.size() + grid, kNoTile);
            const long long per = grid / 8;
            for (long long w = 0; w < grid; ++w) {
                const long long x = w & 7, slot = w >> 3;
                const long long lo = total * x / 8, hi = total * (x + 1) / 8;
                const long long t = lo + slot;
                if (slot >= per || t >= hi) continue;
                const long long im = std::upper_bound(prefix.begin(), prefix.end(), t) - prefix.begin() - 1;
                b->hmap[g.step_map + w] = ((uint32_t)im << g.step_bits) | (uint32_t)(t - prefix[im]);
            }
        }
        // Normaliser map (B > 1 region images): image-major block groups.
        g.mpass_map = b->hmap.size();
        g.mpass_grid = 0;
        if (!g.edge && g.NB > 1) {
            for (int q = 0; q < g.count; ++q) {
                const int mg = b->cs[g.first + q]->host_args.mgroups;
                for (int u = 0; u < mg; ++u) b->hmap.push_back(((uint32_t)q << g.mpass_bits) | (uint32_t)u);
            }
            g.mpass_grid = (unsigned)(b->hmap.size() - g.mpass_map);
        }
        b->groups.push_back(g);
        j = e;
    }
    return align_up(b->cs.size() * sizeof(ImgArgs)) + align_up(b->hmap.size() * sizeof(uint32_t));
}

}  // namespace

size_t lse_batch_bytes(lse_ctx *const *cs, int32_t n) {
    lse_batch b;
    return plan_batch(cs, n, &b);
}

namespace {

// Check the arguments of a batch plan for cs / targets and plan it into *b;
// LSE_OK or the reason it cannot be planned.
lse_status plan_checked(lse_ctx *const *cs, int32_t n, const int32_t *targets, void *table_dev, size_t table_bytes,
                        lse_batch *b) {
    if (!cs || n <= 0) return LSE_ERR_INVALID_ARG;
    for (int i = 0; i < n; ++i)
        if (!cs[i]) return LSE_ERR_INVALID_ARG;
    if (targets)
        for (int i = 0; i < n; ++i)
            if (targets[i] < 0) return LSE_ERR_INVALID_ARG;
    const size_t need = plan_batch(cs, n, b);
    if (need == 0) {
        // Repeated or null contexts are invalid; a radius without a compiled
        // step variant is valid but not batched by this build.
        std::set<const lse_ctx *> seen;
        for (int i = 0; i < n; ++i)
            if (!seen.insert(cs[i]).second) return LSE_ERR_INVALID_ARG;
        return LSE_ERR_UNSUPPORTED;
    }
    if (!table_dev || (reinterpret_cast<uintptr_t>(table_dev) % kAlign)) return LSE_ERR_WORKSPACE;
    if (table_bytes < need) return LSE_ERR_WORKSPACE;
    b->dargs = static_cast<ImgArgs *>(table_dev);
    b->dmap = reinterpret_cast<uint32_t *>(static_cast<char *>(table_dev) + align_up(b->cs.size() * sizeof(ImgArgs)));
    b->hargs.resize(b->cs.size());
    b->target.resize(b->cs.size());
    for (size_t i = 0; i < b->cs.size(); ++i) {
        int t = 0x7fffffff;
        if (targets) {
            const lse_ctx *c = b->cs[i];
            for (int j = 0; j < n; ++j)
                if (cs[j] == c) t = targets[j];
        }
        b->hargs[i] = b->cs[i]->host_args;
        b->hargs[i].target = t;
        b->hargs[i].n0 = 0;
        b->target[i] = t;
    }
    return LSE_OK;
}

// Streams and events for the batch's kernel families (more than one family:
// each on a stream of its own, default priority); kept across updates.
hipError_t ensure_streams(lse_batch *b) {
    if (b->groups.size() <= 1) return hipSuccess;
    if (!b->fork && hipEventCreateWithFlags(&b->fork, hipEventDisableTiming) != hipSuccess) return hipErrorUnknown;
    while (b->gstream.size() < b->groups.size()) {
        hipStream_t st = nullptr;
        hipEvent_t ev = nullptr;
        if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) return hipErrorUnknown;
        if (hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess) {
            (void)hipStreamDestroy(st);
            return hipErrorUnknown;
        }
        b->gstream.push_back(st);
        b->join.push_back(ev);
    }
    return hipSuccess;
}

// Copy the planned table (argument records, then maps) to the device on s
// through the next pinned staging buffer.  Only the parts the device reads
// before writing are copied: a visit list is rebuilt by every launch.
hipError_t upload_table(lse_batch *b, hipStream_t s) {
    const size_t a_bytes = b->hargs.size() * sizeof(ImgArgs);
    const size_t m_bytes = b->hmap.size() * sizeof(uint32_t);
    const size_t total = a_bytes + m_bytes;
    lse_batch::Staging &g = b->stage[b->next_stage];
    b->next_stage ^= 1;
    if (g.pending) {
        if (hipEventSynchronize(g.done) != hipSuccess) return hipErrorUnknown;
        g.pending = false;
    }
    if (!g.done && hipEventCreateWithFlags(&g.done, hipEventDisableTiming) != hipSuccess) return hipErrorUnknown;
    if (g.cap < total) {
        if (g.host) (void)hipHostFree(g.host);
        g.host = nullptr;
        g.cap = 0;
        const size_t cap = std::max<size_t>(total + total / 2, 4096);
        if (hipHostMalloc(&g.host, cap, hipHostMallocDefault) != hipSuccess) {
            g.host = nullptr;
            return hipErrorUnknown;
        }
        g.cap = cap;
    }
    char *h = static_cast<char *>(g.host);
    memcpy(h, b->hargs.data(), a_bytes);
    memcpy(h + a_bytes, b->hmap.data(), m_bytes);
    hipError_t e = hipMemcpyAsync(b->dargs, h, a_bytes, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipMemcpyAsync(b->dmap, h + a_bytes, m_bytes, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipEventRecord(g.done, s);
    g.pending = e == hipSuccess;
    return e;
}

}  // namespace

lse_status lse_batch_create(lse_ctx *const *cs, int32_t n, const int32_t *targets, void *table_dev,
                            size_t table_bytes, void *stream, lse_batch **out) {
    if (!out) return LSE_ERR_INVALID_ARG;
    *out = nullptr;
    lse_batch *b = new (std::nothrow) lse_batch();
    if (!b) return LSE_ERR_INVALID_ARG;
    const lse_status v = plan_checked(cs, n, targets, table_dev, table_bytes, b);
    if (v != LSE_OK) {
        delete b;
        return v;
    }
    b->exec = nullptr;
    b->exec_iters = -1;
    b->exec_stop = -1;
    const hipStream_t s = as_stream(stream);
    b->last_stream = s;
    if (ensure_streams(b) != hipSuccess || upload_table(b, s) != hipSuccess) {
        delete b;
        return LSE_ERR_DEVICE;
    }
    *out = b;
    return LSE_OK;
}

lse_status lse_batch_update(lse_batch *b, lse_ctx *const *cs, int32_t n, const int32_t *targets, void *table_dev,
                            size_t table_bytes, void *stream) {
    if (!b) return LSE_ERR_INVALID_ARG;
    // A batch replayed from a graph is not re-planned: its captured launch
    // sequence names the old table, and capturing again after a re-plan has
    // failed on the host (a segmentation fault inside the capture, cause not
    // found), so that path is not taken.
    if (b->exec) return LSE_ERR_STATE;
    lse_batch next;
    const lse_status v = plan_checked(cs, n, targets, table_dev, table_bytes, &next);
    if (v != LSE_OK) return v;
    const hipStream_t s = as_stream(stream);
    b->cs.swap(next.cs);
    b->target.swap(next.target);
    b->groups.swap(next.groups);
    b->hargs.swap(next.hargs);
    b->hmap.swap(next.hmap);
    b->dargs = next.dargs;
    b->dmap = next.dmap;
    b->last_stream = s;
    if (ensure_streams(b) != hipSuccess || upload_table(b, s) != hipSuccess) return LSE_ERR_DEVICE;
    return LSE_OK;
}

namespace {

hipError_t enqueue_batch(lse_batch *b, int iters, int stop, hipStream_t s) {
    hipError_t e = launch_batch_prepare(b->dargs, (int)b->cs.size(), s);
    // Several groups: fork their streams from `s` after the prepare kernel
    // and join them back at the end (inside a graph capture, these event
    // records and waits make the group streams part of the captured graph).
    const size_t ng = b->groups.size();
    const bool multi = ng > 1;
    if (multi) {
        if (e == hipSuccess) e = hipEventRecord(b->fork, s);
        for (size_t gi = 0; gi < ng && e == hipSuccess; ++gi)
            e = hipStreamWaitEvent(b->gstream[gi], b->fork, 0);
    }
    for (int k = 0; k < iters && e == hipSuccess; ++k) {
        for (size_t gi = 0; gi < b->groups.size(); ++gi) {
            const auto &g = b->groups[gi];
            const hipStream_t gs = multi ? b->gstream[gi] : s;
            uint32_t *map = b->dmap + g.step_map;
            const int *nmap = nullptr;
            if (g.visit_list) {
                e = launch_batch_plan(b->dargs + g.first, b->dmap + g.wbase_map, g.count, g.step_bits, k, map, gs);
                nmap = reinterpret_cast<const int *>(map);
                map += 1;
            }
            if (e == hipSuccess && g.mpass_grid)
                e = launch_mpass(b->dargs + g.first, b->dmap + g.mpass_map, g.mpass_bits, g.mpass_grid, k, stop, g.NB,
                                 g.storage, gs);
            if (e == hipSuccess)
                e = launch_step(b->dargs + g.first, map, nmap, g.step_bits, g.step_grid, k, stop, g.r, g.NB, g.edge,
                                g.storage, g.variant, gs);
            if (e != hipSuccess) break;
        }
    }
    if (multi) {
        for (size_t gi = 0; gi < ng; ++gi) {
            // Join even after an error, so that no group stream is left
            // forked (or a capture left open on it).
            const hipError_t r = hipEventRecord(b->join[gi], b->gstream[gi]);
            const hipError_t w = r == hipSuccess ? hipStreamWaitEvent(s, b->join[gi], 0) : r;
            if (e == hipSuccess) e = w;
        }
    }
    return e;
}

}  // namespace

lse_status lse_batch_run(lse_batch *b, int32_t iters, int32_t stop_when_unchanged, int32_t flags, void *stream) {
    if (!b || iters < 0 || (flags & ~LSE_BATCH_GRAPH)) return LSE_ERR_INVALID_ARG;
    const hipStream_t s = as_stream(stream);
    const int stop = stop_when_unchanged ? 1 : 0;
    if (iters == 0) return LSE_OK;
    hipError_t e = hipSuccess;
    if (flags & LSE_BATCH_GRAPH) {
        if (!s) return LSE_ERR_INVALID_ARG;  // the default stream cannot be captured
        if (!b->exec || b->exec_iters != iters || b->exec_stop != stop) {
            if (b->exec) {
                if (hipStreamSynchronize(b->last_stream) != hipSuccess) return LSE_ERR_DEVICE;
                (void)hipGraphExecDestroy(b->exec);
                b->exec = nullptr;
            }
            hipGraph_t graph = nullptr;
            e = hipStreamBeginCapture(s, hipStreamCaptureModeRelaxed);
            if (e != hipSuccess) return LSE_ERR_DEVICE;
            const hipError_t le = enqueue_batch(b, iters, stop, s);
            e = hipStreamEndCapture(s, &graph);
            if (le != hipSuccess || e != hipSuccess || !graph) {
                if (graph) (void)hipGraphDestroy(graph);
                return LSE_ERR_DEVICE;
            }
            e = hipGraphInstantiate(&b->exec, graph, nullptr, nullptr, 0);
            (void)hipGraphDestroy(graph);
            if (e != hipSuccess) {
                b->exec = nullptr;
                return LSE_ERR_DEVICE;
            }
            b->exec_iters = iters;
            b->exec_stop = stop;
        }
        e = hipGraphLaunch(b->exec, s);
    } else {
        e = enqueue_batch(b, iters, stop, s);
    }
    if (e != hipSuccess) return LSE_ERR_DEVICE;
    for (size_t i = 0; i < b->cs.size(); ++i) {
        lse_ctx *c = b->cs[i];
        const long long left = (long long)b->target[i] - c->n;
        const int ran = (int)std::max(0ll, std::min((long long)iters, left));
        c->n += ran;
        if (ran > 0) c->raw_next = 0;
        c->last_stream = s;
    }
    b->last_stream = s;
    return LSE_OK;
}

void lse_batch_destroy(lse_batch *b) {
    if (!b) return;
    // The caller's stream joins the group streams: once it is idle, so are they.
    if (b->exec || !b->gstream.empty()) (void)hipStreamSynchronize(b->last_stream);
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    delete b;
}

int32_t lse_version(void) { return 106; }

}  // extern "C"
