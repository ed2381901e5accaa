// Internal declarations shared by the HIP kernels and the C ABI layer.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/lse.h"

namespace lse {

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
    int bad;                      // nonzero: bad value found by init
    int done;                     // sticky "stopped" flag (Step 5)
    int iters;                    // iterations executed since init / set_mask
    int pad0;
    float last_cp[4], last_cm[4];
    float last_M;
    int pad1[3];
    unsigned long long acc_needed;  // profiling: pixels whose image value the steps needed
    unsigned long long acc_steps;   // profiling: steps counted into acc_needed
};

// Constant tables, copied once into the workspace.
struct Taps {
    float k[32];                    // 1-D LSF smoothing taps, k[j] for offset j - r
    float cum[33];                  // cum[m] = k[0] + ... + k[m-1] (border correction)
    float lut[kMaxChunks][64];      // lut[c][m] = sum_j (bit j of m ? +1 : -1) k[6c + j]
    float k1[32];                   // edge term: image pre-smoothing taps
    float pad[31];
};

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
};

// Kernel launchers (lse_kernels.hip).  All return hipSuccess or the launch error.
size_t tile_smem_bytes(int r, int nch, int edge);
hipError_t launch_init_state(DevState *st, hipStream_t s);
hipError_t launch_reset_state(DevState *st, hipStream_t s);
hipError_t launch_init_image(const void *src, int src_dtype, int B, int NB, float *dst, long long npx,
                             DevState *st, float fix, int want_gray, float gray_scale, hipStream_t s);
hipError_t launch_pack_mask(const uint8_t *mask, uint32_t *bits, int H, int W, int WW, hipStream_t s);
hipError_t launch_stats(const StepArgs &a, int NB, int raw, int slot, hipStream_t s);
hipError_t launch_edge_map(const float *gray, int H, int W, const Taps *taps, int r1, float *tmp, float *Is,
                           float *g, hipStream_t s);
hipError_t launch_mpass(const StepArgs &a, int NB, hipStream_t s);
size_t mbox_floats(int H, int W, int NB);
hipError_t launch_mbox(const float *img, int H, int W, int NB, float *boxes, hipStream_t s);
hipError_t launch_step(const StepArgs &a, int NB, int edge, hipStream_t s);
hipError_t launch_mask_out(const uint32_t *const bits[2], const DevState *st, uint8_t *mask, int H, int W,
                           int WW, hipStream_t s);
hipError_t launch_lsf_out(const StepArgs &a, const uint32_t *const bits[2], int raw, float *out,
                          hipStream_t s);
hipError_t launch_count_needed(const StepArgs &a, int raw, int edge, hipStream_t s);
hipError_t launch_reset_profile(DevState *st, hipStream_t s);

}  // namespace lse
