// Internal declarations shared by the HIP kernels and the C ABI layer.
#pragma once

#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/lse.h"

namespace lse {

// Kernel timing for lse_profile: when armed, the next launch of the step path
// passes the event pair into its own dispatch packet, so the events hold that
// kernel's start and end (no marker packets or queue gaps around it), and the
// pair is disarmed.  Unarmed launches are plain launches.
struct LaunchTiming {
    hipEvent_t start, stop;
};
LaunchTiming &launch_timing();  // the calling host thread's

template <typename F, typename... A>
hipError_t launch_timed(F kernel, dim3 grid, dim3 block, uint32_t smem, hipStream_t s, A... args) {
    LaunchTiming &t = launch_timing();
    if (t.start) {
        const LaunchTiming e = t;
        t = LaunchTiming{nullptr, nullptr};
        hipExtLaunchKernelGGL(kernel, grid, block, smem, s, e.start, e.stop, 0u, args...);
    } else {
        kernel<<<grid, block, smem, s>>>(args...);
    }
    return hipGetLastError();
}

constexpr int kMaxBands = 4;
constexpr int kMaxRadius = 15;   // template side TS <= 31
constexpr int kChunkBits = 6;    // binary-window lookup tables of 64 entries
constexpr int kMaxChunks = 6;    // ceil(31 / 6)
constexpr int kTileX = 64;       // owned columns of one step workgroup (2 bit words)
constexpr int kTileY = 32;       // owned rows of one step workgroup
constexpr int kThreads = 256;    // 4 wave64 per workgroup
constexpr int kRowWords = 5;     // bit words staged per row in LDS (4 used + 1 pad)
constexpr uint64_t kNoFlips = ~0ull;  // "no previous iteration" marker

constexpr int kBins = 64;             // accumulation lines (one per lane of a wave)
constexpr int kBadInput = 1;          // DevState::bad values
constexpr int kBadOverflow = 2;

// One accumulation line of the region statistics of one LSF: fixed-point band
// sums over {phi >= 0}, the count, the flip count of the iteration that
// produced the LSF, and the normaliser key used with it: (bits of max|D|) << 32
// | (0xffffffff - pixel index of the maximum), so that the maximum and its
// pixel (smallest index on ties) come out of one 64-bit atomic max.
// Workgroup w adds into line w % kBins, so atomics spread over kBins cache
// lines instead of serialising on one; readers sum the lines (integer sums,
// exact and order-independent).
struct alignas(128) Bin {
    long long sum[4];
    unsigned long long nplus;
    unsigned long long flips;
    unsigned long long mkey;
    unsigned long long pad[9];
};
static_assert(sizeof(Bin) == 128, "one bin per 128-byte line");

// Per-image statistics lines (band totals, min / max keys), filled by init.
struct alignas(128) ImgBin {
    long long total[4];
    unsigned int imin_key[4];
    unsigned int imax_key[4];
    unsigned long long pad[8];
};
static_assert(sizeof(ImgBin) == 128, "one bin per 128-byte line");

// Device-resident state, at the start of the workspace.
struct DevState {
    Bin slot[3][kBins];           // triple-buffered: read n%3, write (n+1)%3, clear (n+2)%3
    ImgBin img[kBins];
    int bad;                      // kBadInput: bad value found by init; kBadOverflow: LSF left the storage range
    int done;                     // sticky "stopped" flag (Step 5)
    int iters;                    // iterations executed since init / set_mask
    int raw;                      // iteration 0 starts from the binary function itself (no smoothing)
    float last_cp[4], last_cm[4];
    float last_M;
    int pad1[3];
    unsigned long long acc_needed;  // profiling: pixels whose image value the steps needed
    unsigned long long acc_steps;   // profiling: steps counted into acc_needed
    unsigned long long acc_visited; // profiling: step tiles the counted steps visited (fast path)
    unsigned long long acc_heavy;   // profiling: of those, tiles recorded as heavy (not quiet)
    unsigned long long digest;      // launch_digest: digest of the binary state
};

// Fixed-point region sums and count of one step tile: the all-inside case
// (the value the step kernel's own reduction would produce when every pixel
// is on the + side), or a tile's latest contribution to the totals.
struct alignas(64) TileSum {
    long long sum[4];
    long long cnt;
    long long pad[3];
};

// Constant tables, copied once into the workspace.
struct Taps {
    float k[32];                    // 1-D LSF smoothing taps, k[j] for offset j - r
    float cum[33];                  // cum[m] = k[0] + ... + k[m-1] (border correction)
    float lut[kMaxChunks][64];      // lut[c][m] = sum_j (bit j of m ? +1 : -1) k[6c + j]
    float k1[32];                   // edge term: image pre-smoothing taps
    float pad[31];
};

// Arguments of one host-launched kernel on one image (initial statistics,
// LSF export, profiling count, and the step for templates outside the
// compile-time radius range).
struct StepArgs {
    const void *img;          // storage image (NB interleaved bands) or edge map
    const float *boxes;       // region term, B > 1: per-block band min / max (normaliser pruning)
    const uint32_t *bits_in;  // binary state b^{n-1}
    uint32_t *bits_out;       // binary state b^n
    DevState *st;
    const Taps *taps;
    int H, W, WW;             // WW = 32-bit words per bit row
    int r, ts, nch;           // smoothing radius, side, lookup chunks
    float dt;
    int n;                    // iteration index since init / set_mask (slot parity)
    int raw;                  // 1: phi^n is the binary function itself (first iteration)
    int stop;                 // stop when an iteration changes nothing
    float fix;                // 2^s, fixed-point scale of the band sums
    float inv_fix;            // 2^-s
    long long hw;
    // Continuous-LSF modes (other step orders / reinitialisation schedules):
    const void *plane_in;     // phi^n (or the pre-sign field of a binarised phi^n), storage type
    void *plane_out;          // the field stored by this iteration
    int order;                // lse_order
    int reinit;               // this iteration binarises (Table I step 3)
    int phi_binary;           // phi^n is the binary function in bits_in (sign of the stored field)
    TileSum *tilelast;        // region, fast path: initial statistics record each step tile's sums here
};

// Device-resident arguments of one image for the step and normaliser
// kernels.  A single image keeps one in its workspace (n0 = 0: launch k is
// iteration k); a batch keeps an array of them plus a workgroup map, so that
// one launch advances every image of the batch by one iteration.
struct alignas(16) ImgArgs {
    const void *img;          // region: image (NB interleaved bands); edge: edge map g (storage type)
    const float *boxes;       // region, B > 1: per-block band min / max
    uint32_t *bits[2];        // iteration n reads bits[n & 1] and writes bits[(n + 1) & 1]
    DevState *st;
    const Taps *taps;
    int H, W, WW;
    int tiles;                // workgroup tiles of the step kernel
    float dt, fix, inv_fix;
    int target;               // iterations n >= target are not run
    long long hw;
    int n0;                   // iteration index of launch k = 0
    int mgroups;              // workgroups of the normaliser pass (B > 1)
    const TileSum *tilesum;   // region term: per-tile sums of the all-inside case
    TileSum *tilelast;        // region term: each tile's latest contribution to the totals
    uint32_t *sched_mask;     // fast path, 3 x ceil(tiles / 32) words: [n % 3] tiles that were heavy
                              // (not quiet) in iteration n - 1, all of them after a restart
    int *plan;                // fast path, single image, 1 + tiles: [0] tiles the next step visits,
                              // [1 ..] those tiles, heavy ones first (null: each workgroup finds its
                              // tile in sched_mask)
};

constexpr uint32_t kNoTile = 0xffffffffu;  // workgroup-map entry of a spare workgroup
// A single-image step without a normaliser pass finds its tiles in the heavy
// record itself up to this many tiles (two mask words per lane of one wave);
// larger images get a visit list from a separate pass.
constexpr int kPlanMinTiles = 4096;
// Schedule words for nw record words: three heavy-tile records, then (from a
// 16-byte aligned word) one touched-tag byte per tile.
__host__ __device__ constexpr int sched_tag_offset(int nw) { return (3 * nw + 3) & ~3; }
__host__ __device__ constexpr int sched_words(int nw) { return sched_tag_offset(nw) + 8 * nw; }

// Kernels whose code depends on the storage type T of the resident image
// (float, __half or __hip_bfloat16).  The member functions are defined in
// lse_store.h and instantiated once per type (lse_store_*.hip).
template <typename T>
struct Store {
    static hipError_t init_image(const void *src, int src_dtype, int B, int NB, void *dst, long long npx,
                                 DevState *st, float fix, int mode, hipStream_t s);
    static hipError_t edge_map(const void *src, int src_dtype, int B, float scale, const Taps *taps, int r1, void *g,
                               int H, int W, DevState *st, hipStream_t s);
    template <typename S>
    static hipError_t edge_map_t(const S *src, int B, float scale, const Taps *taps, int r1, T *g, int H, int W,
                                 DevState *st, hipStream_t s);
    static hipError_t init_image_box(const void *src, int src_dtype, int B, int NB, void *dst, int H, int W,
                                     DevState *st, float fix, float *boxes, hipStream_t s);
    template <typename S>
    static hipError_t init_image_box_t(const S *src, int B, int NB, T *dst, int H, int W, DevState *st, float fix,
                                       float *boxes, hipStream_t s);
    static hipError_t stats(const StepArgs &a, int NB, int raw, int slot, hipStream_t s);
    static hipError_t step(const ImgArgs *args, const uint32_t *map, const int *nmap, int unit_bits, unsigned grid,
                           int k, int stop, int r, int NB, int edge, int variant, hipStream_t s);
    static hipError_t step_generic(const StepArgs &a, int NB, int edge, hipStream_t s);
    static hipError_t mpass(const ImgArgs *args, const uint32_t *map, int unit_bits, unsigned grid, int k, int stop,
                            int NB, hipStream_t s);
    // Continuous-LSF modes: one iteration; the LSF plane from the binary
    // function (raw: +-1; else its Gaussian smoothing); the region statistics
    // of a plane; the plane as FP32.
    static hipError_t dense_step(const StepArgs &a, int NB, int edge, hipStream_t s);
    static hipError_t plane_fill(const StepArgs &a, const uint32_t *bits, int raw, void *plane, hipStream_t s);
    static hipError_t plane_stats(const StepArgs &a, const void *plane, int NB, int slot, hipStream_t s);
    static hipError_t plane_out(const void *p0, const void *p1, const DevState *st, float *out, long long n,
                                hipStream_t s);
    // A caller's FP32 LSF into a storage plane (resume of the continuous modes).
    static hipError_t plane_load(const float *src, void *dst, long long n, DevState *st, hipStream_t s);
    // Per-tile region sums of the all-inside case (args[0], radius r).
    static hipError_t tile_sums(const ImgArgs *args, int tiles, int r, int NB, TileSum *out, hipStream_t s);
};

// Kernel launchers (lse_kernels.hip).  All return hipSuccess or the launch
// error; `storage` is an lse_dtype.
size_t tile_smem_bytes(int r, int nch, int edge);
bool fast_radius(int r);                 // the step kernel has a compiled variant for radius r
// Step-kernel variants (tile rows, waves per SIMD; see StepVariant).
constexpr int kNumStepVariants = 3;
void step_variant_info(int edge, int variant, int *tile_rows, int *waves_per_simd);
int step_tiles(int H, int W, int edge, int variant);  // workgroup tiles of the step kernel for an H x W image
int step_tiles_max(int H, int W, int edge);           // the most over the variants (workspace sizing)
int mpass_groups(int H, int W);          // workgroups of the normaliser pass
// Copy `bytes` (a multiple of 4, at most kPutWords words) of host memory to
// dst on the stream, carried as a kernel argument (no host-to-device copy).
constexpr int kPutWords = 512;
static_assert(sizeof(Taps) <= 4 * kPutWords && sizeof(ImgArgs) <= 4 * kPutWords, "tables fit one kernel argument");
hipError_t launch_put_bytes(const void *host, size_t bytes, void *dst, hipStream_t s);
hipError_t launch_init_state(DevState *st, int raw, hipStream_t s);
hipError_t launch_reset_state(DevState *st, int raw, hipStream_t s);
// mode 0: bands; 2: band mean (intensity-only region term).
hipError_t launch_init_image(const void *src, int src_dtype, int storage, int B, int NB, void *dst, long long npx,
                             DevState *st, float fix, int mode, hipStream_t s);
hipError_t launch_pack_mask(const uint8_t *mask, uint32_t *bits, int H, int W, int WW, hipStream_t s);
// Bits of sign(lsf) (lsf >= 0 -> 1), H x W float32.
hipError_t launch_pack_sign(const float *lsf, uint32_t *bits, int H, int W, int WW, hipStream_t s);
hipError_t launch_plane_load(const float *src, void *dst, long long n, DevState *st, int storage, hipStream_t s);
hipError_t launch_stats(const StepArgs &a, int NB, int storage, int raw, int slot, hipStream_t s);
// Edge map g of eq. (14) from the caller's image (B bands of src_dtype), in
// one launch: gray = scale x band mean, smoothed by the k1 taps, central-
// difference gradient, g = 1 / (1 + |grad|^2) stored as `storage`.
hipError_t launch_edge_map(const void *src, int src_dtype, int B, float scale, const Taps *taps, int r1, void *g,
                           int H, int W, int storage, DevState *st, hipStream_t s);
size_t mbox_floats(int H, int W, int NB);
// Region image of NB = 2 or 4 stored bands (init_image mode 0) and its
// normaliser boxes (per 64 x 32 block, the band minima and maxima of the
// stored values) in one pass.
hipError_t launch_init_image_box(const void *src, int src_dtype, int storage, int B, int NB, void *dst, int H, int W,
                                 DevState *st, float fix, float *boxes, hipStream_t s);
// Step / normaliser launches over ImgArgs: map == nullptr runs image args[0]
// (grid = step_launch_grid / mpass_groups); else map[blockIdx.x] holds
// (image << unit_bits) | unit, or kNoTile.  A step map built on the device
// (batch visit list) has *nmap entries; workgroups past them have no work.
unsigned step_launch_grid(int tiles);
hipError_t launch_step(const ImgArgs *args, const uint32_t *map, const int *nmap, int unit_bits, unsigned grid, int k,
                       int stop, int r, int NB, int edge, int storage, int variant, hipStream_t s);
// Order-independent 64-bit digest of the current binary state (bits[iters &
// 1]) into st->digest (cleared first): a check that two runs agree.
hipError_t launch_digest(const uint32_t *const bits[2], DevState *st, int H, int WW, hipStream_t s);
// Batch visit list of one group for launch k: list[0] entries, then
// (image << unit_bits) | tile, heavy tiles first.  wbase: nimg + 1 prefix
// offsets of the images' heavy-record words.
constexpr int kBatchPlanImages = 4096;
hipError_t launch_batch_plan(const ImgArgs *args, const uint32_t *wbase, int nimg, int unit_bits, int k,
                             uint32_t *list, hipStream_t s);
hipError_t launch_step_generic(const StepArgs &a, int NB, int edge, int storage, hipStream_t s);
hipError_t launch_dense_step(const StepArgs &a, int NB, int edge, int storage, hipStream_t s);
hipError_t launch_plane_fill(const StepArgs &a, const uint32_t *bits, int raw, void *plane, int storage,
                             hipStream_t s);
hipError_t launch_plane_stats(const StepArgs &a, const void *plane, int NB, int storage, int slot, hipStream_t s);
hipError_t launch_plane_out(const void *p0, const void *p1, const DevState *st, float *out, long long n, int storage,
                            hipStream_t s);
hipError_t launch_mpass(const ImgArgs *args, const uint32_t *map, int unit_bits, unsigned grid, int k, int stop,
                        int NB, int storage, hipStream_t s);
hipError_t launch_batch_prepare(ImgArgs *args, int n, hipStream_t s);
hipError_t launch_sched_reset(const ImgArgs *host_args, hipStream_t s);
hipError_t launch_plan(const ImgArgs *dev_args, int k, hipStream_t s);
hipError_t launch_tile_sums(const ImgArgs *args, int tiles, int r, int NB, int storage, TileSum *out, hipStream_t s);
hipError_t launch_mask_out(const uint32_t *const bits[2], const DevState *st, uint8_t *mask, int H, int W,
                           int WW, hipStream_t s);
hipError_t launch_lsf_out(const StepArgs &a, const uint32_t *const bits[2], int raw, float *out,
                          hipStream_t s);
hipError_t launch_count_needed(const StepArgs &a, int raw, int edge, int fast_quiet, hipStream_t s);
hipError_t launch_reset_profile(DevState *st, hipStream_t s);
// Profiling: after launch k of a single image on the fast path, add the tiles
// that step visited and the tiles it recorded as heavy to the totals.
hipError_t launch_count_tiles(const ImgArgs *dev_args, int k, int heavy, hipStream_t s);

}  // namespace lse
