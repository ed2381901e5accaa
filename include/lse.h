/*
 * lse.h -- C ABI of the MI355X (gfx950) fast level set evolution library.
 *
 * The library implements the two fast level set evolutions (LSE) of Li, Shi,
 * Wang and Miao, "Extracting Man-Made Objects From Remote Sensing Images via
 * Fast Level Set Evolutions" (arXiv 1409.7474):
 *   - region LSE, eq. (17): phi_t = R(I; c+, c-) |grad phi|,
 *       R = (c+ - c-)(2I - c+ - c-) / max |(c+ - c-)(2I - c+ - c-)|,
 *     c+ / c- the band means over {phi >= 0} / {phi < 0} (eq. (15));
 *   - edge LSE, eq. (14): phi_t = g(I) |grad phi|, g = 1 / (1 + |grad G*I|^2);
 * iterated as Table I: (1) binary initial LSF, eq. (13); (2) data term and
 * explicit Euler update, eq. (18); (3) reinitialisation to a binary function;
 * (4) Gaussian smoothing of the LSF in place of curvature regularisation;
 * (5) stop when the result stops changing; (6) return the binary result.
 *
 * Conventions used everywhere:
 *   - images are H x W x B, row-major, band fastest (pixel (y, x) band b at
 *     ((y * W) + x) * B + b); masks and LSF planes are H x W row-major;
 *   - ties phi == 0 (and u == 0) belong to the + side (+1, inside);
 *   - convolutions use zero padding and same-size output; gradients are
 *     central differences inside and one-sided at the image border;
 *   - all arithmetic on the GPU is FP32 (no FP64 anywhere on the device).
 *
 * Memory ownership: the caller allocates every device buffer (image, masks,
 * workspace, outputs).  The library never allocates device memory; it needs
 * one caller-provided workspace of lse_workspace_bytes() bytes that must stay
 * alive, and untouched, until lse_destroy().  All calls taking a `stream`
 * (a hipStream_t; NULL = the default stream) enqueue work on it and return
 * without synchronising, except lse_stats() and lse_profile_read(), which
 * synchronise that stream.  One context must not be used from two streams at
 * the same time; distinct contexts are independent.
 *
 * Errors: every call returns an lse_status and never throws or aborts.
 * Arguments are validated on the host before anything is enqueued.  A HIP
 * launch or runtime error is returned as LSE_ERR_DEVICE.
 */
#ifndef LSE_H
#define LSE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    LSE_OK = 0,
    LSE_ERR_INVALID_ARG = -1, /* bad parameter, size, pointer or alignment   */
    LSE_ERR_BAD_VALUE = -2,   /* non-finite or out-of-range value in the image */
    LSE_ERR_WORKSPACE = -3,   /* workspace missing, too small or misaligned  */
    LSE_ERR_DEVICE = -4,      /* HIP runtime / launch error                  */
    LSE_ERR_STATE = -5,       /* call not valid in the context's state       */
    LSE_ERR_UNSUPPORTED = -6  /* valid request this build does not implement */
} lse_status;

/* Data term: region, eq. (17), on the band vector; edge, eq. (14) (on the band
 * mean); region on the band-mean intensity only (B values averaged at init,
 * then the single-band region term). */
typedef enum { LSE_TERM_REGION = 0, LSE_TERM_EDGE = 1, LSE_TERM_REGION_INTENSITY = 2 } lse_term;

/* Element types of caller buffers and of the device-resident image copy. */
typedef enum { LSE_F32 = 0, LSE_F16 = 1, LSE_BF16 = 2 } lse_dtype;

/* Step order.  TABLE1: update -> binarise -> smooth (Table I steps 2-4).
 * LISTING: update -> smooth -> binarise (the appendix code): the LSF is the
 * sign of the smoothed update; lse_lsf then returns that pre-sign field. */
typedef enum { LSE_ORDER_TABLE1 = 0, LSE_ORDER_LISTING = 1 } lse_order;

typedef struct {
    int32_t height, width; /* H, W >= 2; H * W * (bands, 3 counted as 4) * 4 bytes
                              below 4 GiB - 1 MiB (edge term: H * W * 4)      */
    int32_t bands;         /* B in 1..4                                       */
    int32_t term;          /* lse_term                                        */
    int32_t order;         /* lse_order                                       */
    int32_t image_dtype;   /* lse_dtype of the caller's image buffer          */
    int32_t storage;       /* lse_dtype of the resident image (region) or edge
                              map (edge); values are rounded to it once at
                              init, all arithmetic stays FP32.  The LSF itself
                              is kept as its binary function (1 bit per pixel)
                              in every mode.                                  */
    float dt;              /* time step of eq. (18), finite, > 0 (paper: 15)  */
    float sigma;           /* LSF smoothing: sigma of (17) / sigma2 of (14)   */
    int32_t ksize;         /* its template side TS, odd 3..31; 0 = 2*ceil(3 sigma)+1 */
    float sigma_img;       /* edge term: image pre-smoothing sigma1 (listing: 1) */
    int32_t ksize_img;     /* edge term: its template side, odd 3..31 (listing: 9) */
    float edge_scale;      /* edge term: intensity scale applied to the band
                              mean before g(I) (255 = 8-bit numbers as in the
                              listing, for images given in [0, 1])            */
    int32_t reinit_every;  /* binarise in iteration n (0-based) iff
                              (n + 1) % reinit_every == 0; 1 = every iteration
                              (the fast binary-state path), 0 = never (region
                              terms only; the edge term needs reinitialisation).
                              Other than TABLE1 with 1, the LSF is kept as a
                              continuous plane of the storage type.            */
} lse_params;

/* Fill *p with the defaults (region term, Table I order, dt 15, sigma 1,
 * TS 7, sigma1 1, TS1 9, edge scale 255, FP32 image and storage) for an
 * H x W x B image.  With 16-bit storage the H x W x B limit on height applies
 * with 2 bytes per value instead of 4. */
void lse_params_default(lse_params *p, int32_t height, int32_t width, int32_t bands);

/* State after the last executed iteration (see lse_stats). */
typedef struct {
    uint64_t n_plus;     /* #{phi >= 0} of the current LSF                    */
    uint64_t flips;      /* pixels whose binary result changed in the last iteration */
    int32_t iters_done;  /* iteration index: iterations run since lse_init, or
                            since lse_set_mask / lse_set_lsf plus their
                            `iteration` argument                            */
    int32_t converged;   /* 1 once an iteration changed no pixel (Step 5)     */
    int32_t bad_value;   /* 1 if lse_init found a non-finite / out-of-range value */
    int32_t lsf_overflow;/* 1 if a continuous LSF (no binarisation in some
                            iterations) left the range of the storage type;
                            the iteration stopped there                       */
    float c_plus[4];     /* c+ used by the last iteration (region term)       */
    float c_minus[4];    /* c- used by the last iteration (region term)       */
    float M;             /* normaliser max|D| used by the last iteration      */
    float pad[3];
} lse_stats_t;

/* Totals accumulated while profiling is enabled (see lse_profile). */
typedef struct {
    double step_ms;      /* fused update/binarise/smooth/statistics kernel    */
    double mpass_ms;     /* normaliser pass of eq. (17) (B > 1)               */
    int64_t step_launches;
    int64_t mpass_launches;
    int64_t needed_pixels; /* LSE_PROFILE_COUNT: pixels whose image (region) or
                              edge-map (edge) value the counted steps read    */
    int64_t counted_steps;
    int64_t visited_tiles; /* LSE_PROFILE_COUNT, binary-state path: step tiles
                              the counted steps visited (the others were
                              settled, Table I step 3 leaving them unchanged);
                              -1 where the path has no tile schedule          */
    int64_t heavy_tiles;   /* of those, tiles whose bit window was not uniform */
    int64_t tiles;         /* step tiles of one iteration (-1 as above)       */
} lse_profile_t;

/* lse_profile flags.  LSE_PROFILE_SAMPLE(k), k = 0..15, or-ed with
 * LSE_PROFILE_TIMING, times one launch in 2^k of each kernel (launches
 * 2^k - 1, 2 * 2^k - 1, ...): the events of a timed launch cost the device a
 * few microseconds, so a sample keeps them out of the throughput. */
enum { LSE_PROFILE_TIMING = 1, LSE_PROFILE_COUNT = 2 };
#define LSE_PROFILE_SAMPLE(k) ((int32_t)(k) << 8)

typedef struct lse_ctx lse_ctx; /* opaque, host-side */

/* Bytes of device workspace lse_init needs for *p; 0 if *p is invalid.  The
 * workspace holds the whole state of the iteration of Table I: the resident
 * image (region term, eq. (17)) or edge map g (edge term, eq. (14)) in the
 * storage type, the LSF as its binary function of Table I step 3 (two bit
 * planes, b^(n-1) and b^n), the region statistics of eq. (15) and, in the
 * continuous-LSF modes, two LSF planes of the storage type. */
size_t lse_workspace_bytes(const lse_params *p);

/* Table I step 1.  Copies/converts the image (H x W x B, p->image_dtype) into
 * the workspace, builds the binary initial LSF of eq. (13) from init_mask
 * (H x W uint8, nonzero = inside the initial curve = +1), computes the edge
 * map g of eq. (14) (edge term) or the initial region statistics (region
 * term).  Image values must be finite with |value| < 65536; the check runs on
 * the device and is reported by lse_stats().bad_value / lse_check() (the
 * iteration then leaves the LSF unchanged).  image_dev and init_mask_dev are
 * read in stream order and may be reused once the stream has passed this
 * call.  workspace_dev must be 256-byte aligned.  On success *out receives a
 * new context. */
lse_status lse_init(const lse_params *p, const void *image_dev, const uint8_t *init_mask_dev,
                    void *workspace_dev, size_t workspace_bytes, void *stream, lse_ctx **out);

/* One iteration: Table I steps 2-4 (data term, Euler update eq. (18),
 * binarisation, Gaussian smoothing). */
lse_status lse_step(lse_ctx *c, void *stream);

/* Up to max_iters iterations (steps 2-5).  With stop_when_unchanged != 0 the
 * device stops after the first iteration that changes no pixel; the host does
 * not synchronise (iterations past that point become no-ops). */
lse_status lse_run(lse_ctx *c, int32_t max_iters, int32_t stop_when_unchanged, void *stream);

/* Step 6: the binary result (1 = inside, phi >= 0) as H x W uint8. */
lse_status lse_mask(const lse_ctx *c, uint8_t *mask_dev, void *stream);

/* The current LSF as H x W float32 (lsf_dev 4-byte aligned, caller-owned):
 * the result of Table I step 4, G_sigma * b, after at least one iteration, the
 * binary initial LSF of eq. (13) before the first.  Continuous-LSF modes: the
 * stored plane (G_sigma * u after an iteration without binarisation; in
 * listing order after a binarising iteration the smoothed update psi whose
 * sign is the LSF). */
lse_status lse_lsf(const lse_ctx *c, float *lsf_dev, void *stream);

/* Load a state whose LSF is a function of a binary mask (checkpoint / resume,
 * Table I steps 1 and 4): mask_dev (H x W uint8, nonzero = +1) becomes the
 * binary function; smoothed = 0 makes it the initial LSF of eq. (13),
 * smoothed = 1 makes the LSF its Gaussian smoothing (the state after an
 * iteration of Table I order with binarisation).  `iteration` (>= 0) is the
 * number of iterations the state has already run (lse_stats().iters_done of
 * the checkpoint): the next iteration has that index, so a periodic
 * reinitialisation schedule continues where it stopped, and iters_done counts
 * on from it.  Region statistics are recomputed; the converged flag is reset.
 * In the continuous-LSF modes use lse_set_lsf for a state between
 * binarisations. */
lse_status lse_set_mask(lse_ctx *c, const uint8_t *mask_dev, int32_t smoothed, int32_t iteration, void *stream);

/* Load a continuous LSF (checkpoint / resume of the continuous-LSF modes:
 * listing order or reinit_every != 1, where Table I step 3 does not run in
 * every iteration).  lsf_dev: H x W float32 as lse_lsf returned it (rounded
 * once to the storage type; a value that is not finite after the rounding is
 * reported by lse_check as LSE_ERR_BAD_VALUE).  mask_dev: H x W uint8, the
 * binary result of the last iteration as lse_mask returned it (flips of the
 * next iteration are counted against it), or NULL for the sign of lsf_dev
 * (>= 0 -> 1).  iteration: as for lse_set_mask; in listing order, when
 * iteration - 1 was a binarising iteration, lsf_dev is the pre-sign field psi
 * and the LSF is the binary function of mask_dev, as in the run that wrote
 * them.  A checkpoint (lse_lsf, lse_mask, lse_stats().iters_done) loaded here
 * continues bit for bit as the uninterrupted run.  Region statistics are
 * recomputed.  LSE_ERR_UNSUPPORTED in the Table I binary-state mode
 * (reinit_every = 1), whose LSF is always G_sigma * b: lse_set_mask with
 * smoothed = 1 is the exact resume there. */
lse_status lse_set_lsf(lse_ctx *c, const float *lsf_dev, const uint8_t *mask_dev, int32_t iteration, void *stream);

/* The edge term's g of eq. (14) as the iterations read it (rounded once to the
 * storage type), H x W float32, g_dev 4-byte aligned and caller-owned.
 * LSE_ERR_STATE for the region terms. */
lse_status lse_edge_map(const lse_ctx *c, float *g_dev, void *stream);

/* Copy the state summary to *host_out (Table I step 5: the flip count of the
 * last iteration and whether an iteration changed no pixel; the c+ / c- of
 * eq. (15) and the normaliser M of eq. (17) it used); synchronises `stream`.
 * iters_done is the iteration index: iterations run since lse_init, or since
 * a resume plus its `iteration` argument. */
lse_status lse_stats(const lse_ctx *c, lse_stats_t *host_out, void *stream);

/* Synchronise `stream`; LSE_ERR_BAD_VALUE if lse_init found a bad value or the
 * LSF overflowed, LSE_ERR_DEVICE on a pending device error, LSE_OK otherwise. */
lse_status lse_check(const lse_ctx *c, void *stream);

/* Profiling of this context; `flags` (0 = off) resets the totals.
 * LSE_PROFILE_TIMING: HIP events carried by the dispatch of every step and
 *   normaliser launch (or of one in 2^k with LSE_PROFILE_SAMPLE(k)): the
 *   kernel's own start and end.
 * LSE_PROFILE_COUNT: after every step, an extra kernel counts the pixels whose
 *   image value that step needed (the + side of the new LSF for the region
 *   sums, and pixels with |grad phi| != 0 for the update) -- the algorithmic
 *   bytes of the step.  It slows the run; do not time with it. */
lse_status lse_profile(lse_ctx *c, int32_t flags);

/* Totals since profiling was enabled; synchronises the stream last used. */
lse_status lse_profile_read(lse_ctx *c, lse_profile_t *host_out);

/* Algorithmic HBM bytes per pixel and iteration of the fused step kernel for
 * this context (image or edge map read once, binary state read and written
 * once); used for roofline figures.  0 if c is NULL. */
double lse_step_bytes_per_pixel(const lse_ctx *c);

/* Release the context (host memory only; the workspace stays the caller's). */
void lse_destroy(lse_ctx *c);

/* ------------------------------------------------------------------ batch
 *
 * Many contexts (uneven sizes, either term, any storage) advanced together:
 * each iteration of the batch is one launch of the step kernel (plus one of
 * the normaliser pass for B > 1 region images) per kernel family (term, B,
 * template side, storage), covering the tiles of all images of that family.
 * Every image keeps its own state and statistics, so its results are bit for
 * bit those of lse_run on it alone.  Contexts need a template side TS in
 * 7..15 (LSE_ERR_UNSUPPORTED otherwise).
 *
 * The batch table (argument copies and the workgroup -> (image, tile) maps)
 * lives in caller-provided device memory of lse_batch_bytes() bytes, 256-byte
 * aligned, that must stay alive and untouched until lse_batch_destroy().  The
 * contexts must outlive the batch; while a batch exists its contexts may still
 * be stepped alone (lse_step / lse_run) on the same stream.  lse_set_mask on a
 * member context is allowed; targets count iterations since the last
 * lse_init / lse_set_mask (not the iteration index a resume starts from). */
typedef struct lse_batch lse_batch; /* opaque, host-side */

/* lse_batch_run flags. */
enum { LSE_BATCH_GRAPH = 1 };

/* Device bytes of the batch table for these n contexts; 0 if they cannot form
 * a batch (null or repeated context, unsupported template side). */
size_t lse_batch_bytes(lse_ctx *const *cs, int32_t n);

/* Build a batch of n distinct contexts.  targets (n entries, or NULL for no
 * limit): context i stops iterating once it has run targets[i] iterations
 * since its lse_init / lse_set_mask.  The table is written on `stream`. */
lse_status lse_batch_create(lse_ctx *const *cs, int32_t n, const int32_t *targets, void *table_dev,
                            size_t table_bytes, void *stream, lse_batch **out);

/* Re-plan an existing batch for a new set of n distinct contexts (members
 * joining or leaving, as in continuous batching), keeping its family streams
 * and events: nothing is synchronised.  LSE_ERR_STATE for a batch that has
 * run with LSE_BATCH_GRAPH (its captured sequence names the old table; create
 * a new batch instead).  The new
 * table (table_dev, lse_batch_bytes(cs, n) bytes) is written on `stream`;
 * the previous table must stay alive and untouched until the last run
 * enqueued on it has completed (the caller tracks that, e.g. with an event).
 * targets as for lse_batch_create.  On an error the batch is unchanged. */
lse_status lse_batch_update(lse_batch *b, lse_ctx *const *cs, int32_t n, const int32_t *targets, void *table_dev,
                            size_t table_bytes, void *stream);

/* Up to `iters` iterations of every context of the batch (each stops at its
 * target, and with stop_when_unchanged at its Step-5 fixed point), enqueued
 * on `stream` without synchronising.  With more than one kernel family, each
 * family's launches go to a stream of the batch's own (created with it, at
 * the default priority), forked from `stream` and joined back to it, so the
 * families overlap on the device; work enqueued on `stream` afterwards
 * starts after all of them.  LSE_BATCH_GRAPH: the launch sequence is captured
 * once into a HIP graph (re-captured when iters or the stop flag change) and
 * launched as one graph; needs a non-default stream. */
lse_status lse_batch_run(lse_batch *b, int32_t iters, int32_t stop_when_unchanged, int32_t flags, void *stream);

/* Release the batch (synchronises the stream of its last run when it used a
 * graph or streams of its own).  The table memory and the contexts stay the
 * caller's. */
void lse_batch_destroy(lse_batch *b);

/* ---------------------------------------------------------------- autotuner
 *
 * The binary-state step kernel (Table I order, binarisation every iteration,
 * TS 7..15) comes in variants: the tile's owned rows (edge term: 64, 48 or 80;
 * region terms: 48) and the waves per SIMD it is compiled for (region terms:
 * 4, 3 or 5; edge: 4).  All variants compute the same results bit for bit.
 * A process-wide table holds the variant per kernel family (term, template
 * radius, stored bands, storage type) and size class (round(log2(side)) - 8
 * clamped to 0..5, side = sqrt(H * W)); lse_init, lse_solve_static and the
 * batch planner use it (variant 0 where the table has no entry).  Batches
 * group contexts by family and variant. */
#define LSE_TUNE_MAX_CANDIDATES 4
typedef struct {
    int32_t variant;        /* step-kernel variant, 0 .. 2                    */
    int32_t tile_rows;      /* owned rows of a step tile                       */
    int32_t tile_cols;      /* owned columns of a step tile (96)               */
    int32_t waves_per_simd; /* occupancy the variant is compiled for           */
    int32_t size_class;     /* size class of the image                         */
    int32_t candidates;     /* variants timed by lse_autotune (0: not timed)   */
    float ms[LSE_TUNE_MAX_CANDIDATES]; /* each candidate's run time, in variant order */
} lse_tuning_t;

/* Time every variant on this job: lse_init (on the caller's workspace, as
 * for lse_init) and `iters` iterations per candidate, twice, the second run
 * timed with events on `stream` (synchronises it).  Checks that the
 * candidates end in the same binary state (LSE_ERR_STATE otherwise, never
 * expected), enters the fastest in the table for this family and size class
 * (variant 0 unless another is more than 3 % faster), and reports it in *out.  The workspace holds the last candidate's state
 * afterwards (initialise again before use).  LSE_ERR_UNSUPPORTED for the
 * modes without variants (continuous LSF, TS outside 7..15). */
lse_status lse_autotune(const lse_params *p, const void *image_dev, const uint8_t *init_mask_dev, void *workspace_dev,
                        size_t workspace_bytes, int32_t iters, void *stream, lse_tuning_t *out);

/* The table's entry for p's family and size class (variant 0 and
 * candidates 0 when there is none). */
lse_status lse_tuning_lookup(const lse_params *p, lse_tuning_t *out);

/* The variant a context runs (fixed at its lse_init). */
lse_status lse_ctx_tuning(const lse_ctx *c, lse_tuning_t *out);

/* Enter `variant` for p's family and size class by hand (tests, or a table
 * kept from an earlier process). */
lse_status lse_tuning_set(const lse_params *p, int32_t variant);

/* Empty the table. */
void lse_tuning_clear(void);

/* ------------------------------------------------- allocation-free solve
 *
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): one whole
 * solve -- lse_init, lse_run(max_iters, stop_when_unchanged), lse_mask and,
 * if lsf_dev is not NULL, lse_lsf -- enqueued on `stream` with the workspace
 * taken from a library-owned device array of LSE_STATIC_WORKSPACE_BYTES per
 * GPU (allocated when the library is loaded, held until the process ends)
 * instead of a caller buffer.  The call allocates nothing (no hipMalloc,
 * hipFree, pinned staging or host-to-device copy: the constant tables travel
 * as kernel arguments) and returns without synchronising.  Results equal
 * those of the workspace entry points bit for bit.
 *
 * image_dev / init_mask_dev: as for lse_init; mask_dev: H x W uint8 out (1 =
 * inside); lsf_dev: H x W float32 out (4-byte aligned) or NULL.  The current
 * HIP device must be the one the stream and buffers belong to.
 * LSE_ERR_WORKSPACE when lse_workspace_bytes(p) exceeds
 * LSE_STATIC_WORKSPACE_BYTES (e.g. a 4-band FP32 region image above about
 * 4.1 Mpx, or an FP32 edge image above about 5.5 Mpx); other errors as
 * lse_init.
 *
 * Every call on one GPU uses that GPU's one array, which keeps the last
 * call's contents (each call rewrites every part of it it reads before
 * reading it).  Calls that overlap on one GPU -- on two streams, or from two
 * host threads without ordering -- race on it: serialise them. */
#define LSE_STATIC_WORKSPACE_BYTES ((size_t)64 << 20)
lse_status lse_solve_static(const lse_params *p, const void *image_dev, const uint8_t *init_mask_dev,
                            int32_t max_iters, int32_t stop_when_unchanged, uint8_t *mask_dev, float *lsf_dev,
                            void *stream);

/* Human-readable name of a status code. */
const char *lse_status_str(lse_status s);

/* ABI version (major * 100 + minor). */
int32_t lse_version(void);

#ifdef __cplusplus
}
#endif

#endif /* LSE_H */
