// HIP kernels of the fast level set evolution (arXiv 1409.7474) for gfx950:
// the kernels that do not depend on the storage type of the image, and the
// launchers that dispatch on it.
//
// State representation.  With reinitialisation every iteration (Table I
// step 3) the LSF after step 4 is phi^{n+1} = G * b^n, the Gaussian smoothing
// of a binary function.  The device therefore keeps only the binary function
// b (1 bit per pixel, 32-pixel words per row) and recomputes phi on the fly in
// FP32: a horizontal pass turns each 1 x TS window of bits into a weighted sum
// through 64-entry lookup tables (6 bits per lookup), a vertical pass applies
// the taps with FMAs.  Zero padding at the image border is exact: taps that
// fall outside are forced to +1 and their weight subtracted.
//
// One iteration of the region term is one fused kernel per 96 x 48 tile
// (lse_store.h; plus, for B > 1, a read-only pass for the normaliser of
// eq. (17)):
//   A. stage b^{n-1} on the tile plus a halo of 2r+1 in LDS;
//   B. phi^n = G * b^{n-1} on the tile plus a halo of r+1;
//   C. data term, |grad phi^n|, Euler update eq. (18) and sign -> b^n on the
//      tile plus a halo of r (wave64 ballots build the bit words);
//   D. sign(G * b^n) on the tile -> region sums for iteration n+1 (eq. (15)),
//      reduced per wave, per workgroup, then one 64-bit atomic per band.
// The halo of phase C is recomputed by neighbouring tiles with the same
// position-only arithmetic, so every tile sees identical bits.  The edge term
// (eq. (14)) needs no statistics: its tile halo is only r+1.  A batch launch
// covers the tiles of many images, each with its own state.
//
// Region sums: FP32 within a workgroup, converted per workgroup to 64-bit
// fixed point (scale 2^s) and added atomically, so totals do not depend on
// workgroup scheduling or on which other images share a launch.
#include <string.h>

#include <algorithm>

#include "lse_device.h"

namespace lse {

LaunchTiming &launch_timing() {
    static thread_local LaunchTiming t{nullptr, nullptr};
    return t;
}

// ------------------------------------------------------------- init kernels

// Zero the statistics lines (and, unless keep_image_stats, the image lines and
// the bad-value flag); mark slot 0 as having no previous iteration; raw: the
// LSF of iteration 0 is the binary function itself.
__global__ void init_state_kernel(DevState *st, int keep_image_stats, int raw) {
    unsigned long long *slots = reinterpret_cast<unsigned long long *>(&st->slot[0][0]);
    for (int i = threadIdx.x; i < (int)(sizeof(st->slot) / 8); i += blockDim.x) slots[i] = 0ull;
    if (!keep_image_stats) {
        unsigned long long *img = reinterpret_cast<unsigned long long *>(&st->img[0]);
        for (int i = threadIdx.x; i < (int)(sizeof(st->img) / 8); i += blockDim.x) img[i] = 0ull;
    }
    __syncthreads();
    if (!keep_image_stats && threadIdx.x < kBins)
        for (int b = 0; b < 4; ++b) st->img[threadIdx.x].imin_key[b] = 0xffffffffu;
    if (threadIdx.x == 0) {
        st->slot[0][0].flips = kNoFlips;
        st->done = 0;
        st->iters = 0;
        st->raw = raw;
        for (int b = 0; b < 4; ++b) st->last_cp[b] = st->last_cm[b] = 0.f;
        st->last_M = 0.f;
        if (!keep_image_stats) st->bad = 0;
    }
}

// Bit rows from a per-pixel predicate, one thread per 16-pixel segment (two
// per bit word).  The thread forms its segment's 16 bits (one 16-byte read
// when the segment is aligned and inside the row), and the even thread of a
// pair writes the word with its partner's bits above its own.  Bit i of word
// w is column 32 w + i; bits past the row end are zero.
template <typename SEG>
__device__ __forceinline__ void pack_segments(SEG seg, uint32_t *__restrict__ bits, int H, int W, int WW) {
    const long long g = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const int nseg = 2 * WW;
    const bool live = g < (long long)H * nseg;  // H * nseg is even: pairs are live together
    int y = 0, s = 0;
    uint32_t m = 0u;
    if (live) {
        y = (int)(g / nseg);
        s = (int)(g - (long long)y * nseg);
        m = seg((size_t)y * W, 16 * s, W);
    }
    const uint32_t hi = __shfl_xor(m, 1, 64);
    if (live && (s & 1) == 0) bits[(size_t)y * WW + (s >> 1)] = m | (hi << 16);
}

// uint8 mask (nonzero = inside) -> bit words.
__global__ void pack_mask_kernel(const uint8_t *__restrict__ mask, uint32_t *__restrict__ bits, int H, int W,
                                 int WW) {
    pack_segments(
        [&](size_t row, int x0, int w) {
            const uint8_t *p = mask + row + x0;
            uint32_t m = 0u;
            if (x0 + 16 <= w && ((uintptr_t)p & 15u) == 0) {
                const uint4 q = *reinterpret_cast<const uint4 *>(p);
                const uint32_t v[4] = {q.x, q.y, q.z, q.w};
#pragma unroll
                for (int j = 0; j < 4; ++j)
#pragma unroll
                    for (int b = 0; b < 4; ++b) m |= (((v[j] >> (8 * b)) & 0xFFu) != 0u ? 1u : 0u) << (4 * j + b);
            } else {
                for (int i = 0; i < 16 && x0 + i < w; ++i) m |= (p[i] != 0 ? 1u : 0u) << i;
            }
            return m;
        },
        bits, H, W, WW);
}

// sign(lsf) -> bit words (lsf >= 0 -> 1, the tie rule of eq. (15)).
__global__ void pack_sign_kernel(const float *__restrict__ lsf, uint32_t *__restrict__ bits, int H, int W, int WW) {
    pack_segments(
        [&](size_t row, int x0, int w) {
            const float *p = lsf + row + x0;
            uint32_t m = 0u;
            if (x0 + 16 <= w && ((uintptr_t)p & 15u) == 0) {
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    const float4 q = reinterpret_cast<const float4 *>(p)[j];
                    m |= (q.x >= 0.f ? 1u : 0u) << (4 * j) | (q.y >= 0.f ? 1u : 0u) << (4 * j + 1) |
                         (q.z >= 0.f ? 1u : 0u) << (4 * j + 2) | (q.w >= 0.f ? 1u : 0u) << (4 * j + 3);
                }
            } else {
                for (int i = 0; i < 16 && x0 + i < w; ++i) m |= (p[i] >= 0.f ? 1u : 0u) << i;
            }
            return m;
        },
        bits, H, W, WW);
}

// Per-block band min / max for the normaliser pruning (64 x 32 blocks).
size_t mbox_floats(int H, int W, int NB) {
    const size_t nbx = (W + kMBX - 1) / kMBX, nby = (H + kMBY - 1) / kMBY;
    return nbx * nby * 2 * NB;
}

// --------------------------------------------------------------- exports

// Bits -> uint8 mask (1 inside), one thread per 16-pixel segment (one
// 16-byte store when the segment is aligned and inside the row).
__global__ void mask_out_kernel(const uint32_t *__restrict__ b0, const uint32_t *__restrict__ b1,
                                const DevState *__restrict__ st, uint8_t *__restrict__ mask, int H, int W, int WW) {
    const long long g = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const int nseg = 2 * WW;
    if (g >= (long long)H * nseg) return;
    const int y = (int)(g / nseg), s = (int)(g - (long long)y * nseg);
    const int x0 = 16 * s;
    if (x0 >= W) return;
    const uint32_t *bits = (st->iters & 1) ? b1 : b0;
    const uint32_t m = bits[(size_t)y * WW + (s >> 1)] >> (16 * (s & 1));
    uint8_t *p = mask + (size_t)y * W + x0;
    if (x0 + 16 <= W && ((uintptr_t)p & 15u) == 0) {
        uint32_t v[4];
#pragma unroll
        for (int j = 0; j < 4; ++j)
            v[j] = ((m >> (4 * j)) & 1u) | ((m >> (4 * j + 1)) & 1u) << 8 | ((m >> (4 * j + 2)) & 1u) << 16 |
                   ((m >> (4 * j + 3)) & 1u) << 24;
        *reinterpret_cast<uint4 *>(p) = make_uint4(v[0], v[1], v[2], v[3]);
    } else {
        for (int i = 0; i < 16 && x0 + i < W; ++i) p[i] = (uint8_t)((m >> i) & 1u);
    }
}

// phi = G * b (or b itself when raw) on 64 x 32 tiles, with the same
// arithmetic as the step kernel.
__global__ __launch_bounds__(kThreads) void lsf_out_kernel(StepArgs A, const uint32_t *__restrict__ b0,
                                                           const uint32_t *__restrict__ b1, int raw,
                                                           float *__restrict__ out) {
    extern __shared__ float smem[];
    const TileSmem s = carve(smem, A.r, A.nch, 0);
    const int x0 = blockIdx.x * kTileX, y0 = blockIdx.y * kTileY;
    const uint32_t *bits = (A.st->iters & 1) ? b1 : b0;
    stage_tables(s, A.taps, A.ts, A.nch);
    stage_bits(s.bn, bits, y0 - A.r, kTileY + 2 * A.r, x0, A.H, A.WW);
    __syncthreads();
    if (!raw) {
        for (int i = threadIdx.x; i < (kTileY + 2 * A.r) * kTileX; i += kThreads) {
            const int uy = i / kTileX, ox = i - uy * kTileX;
            const int y = y0 - A.r + uy, x = x0 + ox;
            float h = 0.f;
            if (y >= 0 && y < A.H && x < A.W)
                h = hconv_bits(s.bn + uy * kRowWords, ox + 32, x, A.W, A.r, A.ts, A.nch, s.lut, s.cum);
            s.h[i] = h;
        }
        __syncthreads();
    }
    for (int k = 0; k < (kTileX * kTileY) / kThreads; ++k) {
        const int i = threadIdx.x + k * kThreads;
        const int oy = i / kTileX, ox = i - oy * kTileX;
        const int y = y0 + oy, x = x0 + ox;
        if (y < A.H && x < A.W) {
            float v;
            if (raw) {
                const uint32_t wd = s.bn[(oy + A.r) * kRowWords + ((ox + 32) >> 5)];
                v = ((wd >> ((ox + 32) & 31)) & 1u) ? 1.f : -1.f;
            } else {
                v = vconv(s.h + oy * kTileX + ox, kTileX, s.k, A.ts);
            }
            out[(size_t)y * A.W + x] = v;
        }
    }
}

// ---------------------------------------------------------- profiling count

// Pixels whose image (or edge-map) value one iteration needed, for roofline
// accounting: pixels on the + side of phi^{n+1} (read for the region sums) and
// pixels where |grad phi^n| != 0 (read for the data term of the update).
// Recomputes phi^n from b^{n-1} (bits_in) and phi^{n+1} from b^n (bits_out)
// with the step's own arithmetic, so the decisions match the step kernel's.
// Profiling only; not part of any timed path.
__global__ __launch_bounds__(kThreads) void count_needed_kernel(StepArgs A, int raw, int edge, int fast_quiet) {
    extern __shared__ float smem[];
    __shared__ int part[kThreads / 64];
    __shared__ int quiet1[4];
    if (A.st->done || A.st->bad) return;  // the step did not run
    const int r = A.r, ts = A.ts, nch = A.nch, H = A.H, W = A.W;
    const int x0 = blockIdx.x * kTileX, y0 = blockIdx.y * kTileY;
    // carve: tables, prev bits (TY + 2 + 2r rows), cur bits (TY + 2r rows), h, phi (TY + 2) x (TX + 2)
    float *lut = smem, *cum = lut + nch * 64, *k = cum + 36;
    uint32_t *bp = reinterpret_cast<uint32_t *>(k + 32);
    const int BPR = kTileY + 2 + 2 * r, BCR = kTileY + 2 * r;
    uint32_t *bc = bp + BPR * kRowWords;
    float *h = reinterpret_cast<float *>(bc + BCR * kRowWords);  // BPR x (TX + 2), reused for BCR x TX
    float *phi = h + BPR * (kTileX + 2);                            // (TY + 2) x (TX + 2)
    for (int i = threadIdx.x; i < nch * 64; i += kThreads) lut[i] = (&A.taps->lut[0][0])[i];
    for (int i = threadIdx.x; i <= ts; i += kThreads) cum[i] = A.taps->cum[i];
    for (int i = threadIdx.x; i < ts; i += kThreads) k[i] = A.taps->k[i];
    stage_bits(bp, A.bits_in, y0 - 1 - r, BPR, x0, H, A.WW);
    stage_bits(bc, A.bits_out, y0 - r, BCR, x0, H, A.WW);
    __syncthreads();
    const int PWc = kTileX + 2;
    // phi^n on rows y0-1 .. y0+TY, columns x0-1 .. x0+TX
    if (raw) {
        for (int i = threadIdx.x; i < (kTileY + 2) * PWc; i += kThreads) {
            const int q = i / PWc, p = i - q * PWc, y = y0 - 1 + q, x = x0 - 1 + p;
            float v = 0.f;
            if (y >= 0 && y < H && x >= 0 && x < W) {
                const uint32_t wd = bp[(q + r) * kRowWords + ((x - x0 + 32) >> 5)];
                v = ((wd >> ((x - x0 + 32) & 31)) & 1u) ? 1.f : -1.f;
            }
            phi[i] = v;
        }
    } else {
        for (int i = threadIdx.x; i < BPR * PWc; i += kThreads) {
            const int row = i / PWc, p = i - row * PWc, y = y0 - 1 - r + row, x = x0 - 1 + p;
            float v = 0.f;
            if (y >= 0 && y < H && x >= 0 && x < W)
                v = hconv_bits(bp + row * kRowWords, x - x0 + 32, x, W, r, ts, nch, lut, cum);
            h[i] = v;
        }
        __syncthreads();
        for (int i = threadIdx.x; i < (kTileY + 2) * PWc; i += kThreads) {
            const int q = i / PWc, p = i - q * PWc, y = y0 - 1 + q, x = x0 - 1 + p;
            phi[i] = (y >= 0 && y < H && x >= 0 && x < W) ? vconv(h + q * PWc + p, PWc, k, ts) : 0.f;
        }
    }
    __syncthreads();
    // h of b^n for the owned columns (region term)
    if (!edge) {
        for (int i = threadIdx.x; i < BCR * kTileX; i += kThreads) {
            const int row = i / kTileX, ox = i - row * kTileX, y = y0 - r + row, x = x0 + ox;
            float v = 0.f;
            if (y >= 0 && y < H && x < W) v = hconv_bits(bc + row * kRowWords, ox + 32, x, W, r, ts, nch, lut, cum);
            h[i] = v;
        }
        __syncthreads();
    }
    // The step kernel takes the region sums of a quiet all-inside tile (its
    // 96 x kFYRegion tiling, b^{n-1} uniform over the tile's whole bit
    // window, away from the image border) from the sums stored at init: such
    // pixels need no image read for the statistics.  This 64 x 32 tile meets
    // at most 2 x 2 of those tiles.
    const int fx0 = x0 / kFX, fy0 = y0 / kFYRegion;
    for (int q = 0; q < 4; ++q) {
        const int fx = fx0 + (q & 1), fy = fy0 + (q >> 1);
        const int X0 = fx * kFX, Y0 = fy * kFYRegion;
        const int BY0 = Y0 - 2 * r - 1, NR = kFYRegion + 4 * r + 2;
        int ones = 0;
        if (fast_quiet && !edge && X0 < W && Y0 < H && !(X0 - 2 * r - 2 < 0 || X0 + kFX + 2 * r + 2 > W) &&
            BY0 >= 0 && BY0 + NR <= H) {
            const int c0 = X0 - 1 - 2 * r, c1 = X0 + kFX + 1 + 2 * r;  // bit columns [c0, c1)
            const int w0 = c0 >> 5, w1 = (c1 - 1) >> 5, nw = w1 - w0 + 1;
            int all1 = 1;
            for (int i = threadIdx.x; i < NR * nw; i += kThreads) {
                const int row = i / nw, wi = w0 + i % nw;
                uint32_t m = ~0u;
                if (wi == w0) m &= ~0u << (c0 & 31);
                if (wi == w1) m &= ~0u >> (31 - ((c1 - 1) & 31));
                const uint32_t v = A.bits_in[(size_t)(BY0 + row) * A.WW + wi];
                all1 &= (v & m) == m;
            }
            ones = __syncthreads_and(all1);
        }
        if (threadIdx.x == 0) quiet1[q] = ones;
    }
    __syncthreads();
    int cnt = 0;
    for (int i = threadIdx.x; i < kTileY * kTileX; i += kThreads) {
        const int oy = i / kTileX, ox = i - oy * kTileX, y = y0 + oy, x = x0 + ox;
        if (y >= H || x >= W) continue;
        const float *c = phi + (oy + 1) * PWc + (ox + 1);
        float gx, gy;
        if (x == 0) gx = c[1] - c[0];
        else if (x == W - 1) gx = c[0] - c[-1];
        else gx = 0.5f * (c[1] - c[-1]);
        if (y == 0) gy = c[PWc] - c[0];
        else if (y == H - 1) gy = c[0] - c[-PWc];
        else gy = 0.5f * (c[PWc] - c[-PWc]);
        bool need = !(gx == 0.f && gy == 0.f);
        if (!edge && !quiet1[(x / kFX - fx0) + 2 * (y / kFYRegion - fy0)])
            need = need || vconv(h + oy * kTileX + ox, kTileX, k, ts) >= 0.f;
        cnt += need ? 1 : 0;
    }
    cnt = wave_sum_i(cnt);
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = cnt;
    __syncthreads();
    if (threadIdx.x == 0) {
        int tot = 0;
        for (int w = 0; w < kThreads / 64; ++w) tot += part[w];
        atomicAdd(&A.st->acc_needed, (unsigned long long)tot);
        if (blockIdx.x == 0 && blockIdx.y == 0) atomicAdd(&A.st->acc_steps, 1ull);
    }
}

__global__ void reset_profile_kernel(DevState *st) {
    if (threadIdx.x == 0) {
        st->acc_needed = 0;
        st->acc_steps = 0;
        st->acc_visited = 0;
        st->acc_heavy = 0;
    }
}


// Schedule masks: no tile recorded as heavy (the first iteration takes the
// tiles in order).
// Schedule record for a restart at iteration 0: every tile counts as heavy
// in slot 0 (so every tile is visited), the other slots clear.
// Restart: every tile heavy in the record that the next step reads (slot 0),
// the other heavy records empty, no tile tagged.
__global__ void sched_reset_kernel(uint32_t *mask, int nw, int ntiles) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= sched_words(nw)) return;
    uint32_t v = 0u;
    if (i < nw) {
        const int valid = ntiles - 32 * i;
        v = valid >= 32 ? ~0u : ((1u << valid) - 1u);
    }
    mask[i] = v;
}

hipError_t launch_sched_reset(const ImgArgs *a, hipStream_t s) {
    if (!a->sched_mask) return hipSuccess;
    const int nw = (a->tiles + 31) >> 5;
    hipLaunchKernelGGL(sched_reset_kernel, dim3((unsigned)((sched_words(nw) + 255) / 256)), dim3(256), 0, s, a->sched_mask,
                       nw, a->tiles);
    return hipGetLastError();
}

constexpr int kPlanThreads = 1024;

// Visit list of the single-image step (build_plan), for the terms without a
// normaliser pass to carry it.
__global__ __launch_bounds__(kPlanThreads) void plan_kernel(const ImgArgs *__restrict__ args, int k) {
    __shared__ int s_tot[2 * (kPlanThreads / 64)];
    build_plan<kPlanThreads>(args[0], args[0].n0 + k, s_tot);
}

// Batch visit list of one group: the words of every image's heavy record,
// concatenated (image i from wbase[i]), split over the threads; each word
// gives the image's heavy tiles and their other neighbours for that image's
// own iteration n0 + k (none once the image reached its target).  All heavy
// tiles of the group come first, then the others, as in build_plan.
__global__ __launch_bounds__(kPlanThreads) void batch_plan_kernel(const ImgArgs *__restrict__ args,
                                                                  const uint32_t *__restrict__ wbase, int nimg,
                                                                  int unit_bits, int k, uint32_t *__restrict__ list) {
    __shared__ uint32_t s_wb[kBatchPlanImages + 1];
    __shared__ int s_tot[2 * (kPlanThreads / 64)];
    const int tid = (int)threadIdx.x, lane = tid & 63, wave = tid >> 6;
    for (int i = tid; i <= nimg; i += kPlanThreads) s_wb[i] = wbase[i];
    __syncthreads();
    const int tw = (int)s_wb[nimg];
    const int per = (tw + kPlanThreads - 1) / kPlanThreads;
    const int g0 = tid * per;
    // Heavy and other active tiles of concatenated word g; img = its image.
    auto word_masks = [&](int g, uint32_t &h, uint32_t &a, int &img) {
        int lo = 0, hi = nimg - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if ((int)s_wb[mid] <= g) lo = mid; else hi = mid - 1;
        }
        img = lo;
        h = a = 0u;
        const ImgArgs &E = args[img];
        const int n = E.n0 + k;
        if (n >= E.target) return;
        const int nw = (E.tiles + 31) >> 5, w = g - (int)s_wb[img];
        const int valid = min(32, E.tiles - 32 * w);
        const uint32_t vm = valid >= 32 ? ~0u : ((1u << valid) - 1u);
        h = record_word(heavy_record(E.sched_mask, nw, n % 3), w) & vm;
        a = touched_word(E.sched_mask, nw, w, touch_tag(n - 1)) & vm & ~h;
    };
    int nh = 0, na = 0;
    for (int i = 0; i < per; ++i) {
        const int g = g0 + i;
        if (g < tw) {
            uint32_t h, a;
            int img;
            word_masks(g, h, a, img);
            nh += __popc(h);
            na += __popc(a);
        }
    }
    int ih = nh, ia = na;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const int vh = __shfl_up(ih, d, 64), va = __shfl_up(ia, d, 64);
        if (lane >= d) {
            ih += vh;
            ia += va;
        }
    }
    if (lane == 63) {
        s_tot[wave] = ih;
        s_tot[kPlanThreads / 64 + wave] = ia;
    }
    __syncthreads();
    int bh = 0, ba = 0, NH = 0, NA = 0;
    for (int v = 0; v < kPlanThreads / 64; ++v) {
        if (v < wave) {
            bh += s_tot[v];
            ba += s_tot[kPlanThreads / 64 + v];
        }
        NH += s_tot[v];
        NA += s_tot[kPlanThreads / 64 + v];
    }
    int oh = 1 + bh + ih - nh, oa = 1 + NH + ba + ia - na;
    for (int i = 0; i < per; ++i) {
        const int g = g0 + i;
        if (g < tw) {
            uint32_t h, a;
            int img;
            word_masks(g, h, a, img);
            const uint32_t base = ((uint32_t)img << unit_bits) | (uint32_t)(32 * (g - (int)s_wb[img]));
            for (; h; h &= h - 1u) list[oh++] = base + (uint32_t)(__ffs((int)h) - 1);
            for (; a; a &= a - 1u) list[oa++] = base + (uint32_t)(__ffs((int)a) - 1);
        }
    }
    if (tid == 0) list[0] = (uint32_t)(NH + NA);
}

hipError_t launch_batch_plan(const ImgArgs *args, const uint32_t *wbase, int nimg, int unit_bits, int k,
                             uint32_t *list, hipStream_t s) {
    if (nimg < 1 || nimg > kBatchPlanImages) return hipErrorInvalidValue;
    hipLaunchKernelGGL(batch_plan_kernel, dim3(1), dim3(kPlanThreads), 0, s, args, wbase, nimg, unit_bits, k, list);
    return hipGetLastError();
}

// Profiling, step n = n0 + k.  Before the step (heavy = 0): the tiles it
// visits, those that iteration n - 1 recorded as heavy (slot n % 3) or
// tagged as touched (the step overwrites tags).  After it (heavy = 1): the
// tiles it recorded as heavy (slot (n + 1) % 3, intact until step n + 1).
__global__ __launch_bounds__(kPlanThreads) void count_tiles_kernel(const ImgArgs *__restrict__ args, int k,
                                                                   int heavy) {
    const ImgArgs &E = args[0];
    const int n = E.n0 + k;
    const int ntiles = E.tiles, nw = (ntiles + 31) >> 5;
    unsigned long long c = 0;
    for (int w = threadIdx.x; w < nw; w += blockDim.x) {
        const int valid = min(32, ntiles - 32 * w);
        const uint32_t vm = valid >= 32 ? ~0u : ((1u << valid) - 1u);
        const uint32_t m = heavy ? record_word(heavy_record(E.sched_mask, nw, (n + 1) % 3), w)
                                 : record_word(heavy_record(E.sched_mask, nw, n % 3), w) |
                                       touched_word(E.sched_mask, nw, w, touch_tag(n - 1));
        c += __popc(m & vm);
    }
    if (c) atomicAdd(heavy ? &E.st->acc_heavy : &E.st->acc_visited, c);
}

hipError_t launch_count_tiles(const ImgArgs *dev_args, int k, int heavy, hipStream_t s) {
    hipLaunchKernelGGL(count_tiles_kernel, dim3(1), dim3(kPlanThreads), 0, s, dev_args, k, heavy);
    return hipGetLastError();
}

hipError_t launch_plan(const ImgArgs *dev_args, int k, hipStream_t s) {
    hipLaunchKernelGGL(plan_kernel, dim3(1), dim3(kPlanThreads), 0, s, dev_args, k);
    return hipGetLastError();
}

// Batch: freeze each image's iteration count as the index of launch k = 0.
__global__ void batch_prepare_kernel(ImgArgs *args, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) args[i].n0 = args[i].st->iters;
}

// Host bytes carried to the device as a kernel argument: the launch copies
// them when it is enqueued, so the source may change or vanish afterwards and
// no host-to-device copy (or pinned staging) is involved.
struct alignas(16) Words {
    uint32_t w[kPutWords];
};
__global__ void put_words_kernel(Words src, uint32_t *__restrict__ dst, int n) {
    for (int i = threadIdx.x; i < n; i += blockDim.x) dst[i] = src.w[i];
}

hipError_t launch_put_bytes(const void *host, size_t bytes, void *dst, hipStream_t s) {
    if (bytes % 4 || bytes > sizeof(Words) || (reinterpret_cast<uintptr_t>(dst) & 3)) return hipErrorInvalidValue;
    Words w;
    memset(&w, 0, sizeof(w));
    memcpy(w.w, host, bytes);
    hipLaunchKernelGGL(put_words_kernel, dim3(1), dim3(256), 0, s, w, static_cast<uint32_t *>(dst), (int)(bytes / 4));
    return hipGetLastError();
}

hipError_t launch_init_state(DevState *st, int raw, hipStream_t s) {
    hipLaunchKernelGGL(init_state_kernel, dim3(1), dim3(256), 0, s, st, 0, raw);
    return hipGetLastError();
}

hipError_t launch_reset_state(DevState *st, int raw, hipStream_t s) {
    hipLaunchKernelGGL(init_state_kernel, dim3(1), dim3(256), 0, s, st, 1, raw);
    return hipGetLastError();
}

hipError_t launch_init_image(const void *src, int src_dtype, int storage, int B, int NB, void *dst, long long npx,
                             DevState *st, float fix, int mode, hipStream_t s) {
    switch (storage) {
        case LSE_F32: return Store<float>::init_image(src, src_dtype, B, NB, dst, npx, st, fix, mode, s);
        case LSE_F16: return Store<__half>::init_image(src, src_dtype, B, NB, dst, npx, st, fix, mode, s);
        case LSE_BF16: return Store<__hip_bfloat16>::init_image(src, src_dtype, B, NB, dst, npx, st, fix, mode, s);
    }
    return hipErrorInvalidValue;
}

// Workgroups of the segment kernels: one thread per 16 pixels of a row (two per bit word).
static inline unsigned seg_blocks(int H, int WW) {
    const long long threads = (long long)H * 2 * WW;
    return (unsigned)((threads + 255) / 256);
}

hipError_t launch_pack_mask(const uint8_t *mask, uint32_t *bits, int H, int W, int WW, hipStream_t s) {
    hipLaunchKernelGGL(pack_mask_kernel, dim3(seg_blocks(H, WW)), dim3(256), 0, s, mask, bits, H, W, WW);
    return hipGetLastError();
}

hipError_t launch_pack_sign(const float *lsf, uint32_t *bits, int H, int W, int WW, hipStream_t s) {
    hipLaunchKernelGGL(pack_sign_kernel, dim3(seg_blocks(H, WW)), dim3(256), 0, s, lsf, bits, H, W, WW);
    return hipGetLastError();
}

hipError_t launch_plane_load(const float *src, void *dst, long long n, DevState *st, int storage, hipStream_t s) {
    switch (storage) {
        case LSE_F32: return Store<float>::plane_load(src, dst, n, st, s);
        case LSE_F16: return Store<__half>::plane_load(src, dst, n, st, s);
        case LSE_BF16: return Store<__hip_bfloat16>::plane_load(src, dst, n, st, s);
    }
    return hipErrorInvalidValue;
}

size_t tile_smem_bytes(int r, int nch, int edge) { return tile_smem_words(r, nch, edge) * 4; }

bool fast_radius(int r) { return r >= 3 && r <= 7; }

void step_variant_info(int edge, int variant, int *tile_rows, int *waves_per_simd) {
    static_assert(kNumStepVariants == kStepVariants, "host and device agree on the variants");
    int fy = 0, occ = 0;
    switch (variant) {
        case 0: fy = edge ? StepVariant<true, 0>::FY : StepVariant<false, 0>::FY;
                occ = edge ? StepVariant<true, 0>::OCC : StepVariant<false, 0>::OCC; break;
        case 1: fy = edge ? StepVariant<true, 1>::FY : StepVariant<false, 1>::FY;
                occ = edge ? StepVariant<true, 1>::OCC : StepVariant<false, 1>::OCC; break;
        case 2: fy = edge ? StepVariant<true, 2>::FY : StepVariant<false, 2>::FY;
                occ = edge ? StepVariant<true, 2>::OCC : StepVariant<false, 2>::OCC; break;
    }
    if (tile_rows) *tile_rows = fy;
    if (waves_per_simd) *waves_per_simd = occ;
}

int step_tiles(int H, int W, int edge, int variant) {
    int fy = 0;
    step_variant_info(edge, variant, &fy, nullptr);
    if (fy <= 0) return 0;
    return ((W + kFX - 1) / kFX) * ((H + fy - 1) / fy);
}

int step_tiles_max(int H, int W, int edge) {
    int t = 0;
    for (int v = 0; v < kNumStepVariants; ++v) t = std::max(t, step_tiles(H, W, edge, v));
    return t;
}

int mpass_groups(int H, int W) {
    const int nblk = ((W + kMBX - 1) / kMBX) * ((H + kMBY - 1) / kMBY);
    return (nblk + kMBlocksPerWG - 1) / kMBlocksPerWG;
}

// One workgroup per tile, rounded up to a multiple of 8 (one band of tiles
// per XCD, see tile_of).
unsigned step_launch_grid(int tiles) { return (unsigned)((tiles + 7) & ~7); }

hipError_t launch_stats(const StepArgs &a, int NB, int storage, int raw, int slot, hipStream_t s) {
    switch (storage) {
        case LSE_F32: return Store<float>::stats(a, NB, raw, slot, s);
        case LSE_F16: return Store<__half>::stats(a, NB, raw, slot, s);
        case LSE_BF16: return Store<__hip_bfloat16>::stats(a, NB, raw, slot, s);
    }
    return hipErrorInvalidValue;
}

hipError_t launch_edge_map(const void *src, int src_dtype, int B, float scale, const Taps *taps, int r1, void *g,
                           int H, int W, int storage, DevState *st, hipStream_t s) {
    switch (storage) {
        case LSE_F32: return Store<float>::edge_map(src, src_dtype, B, scale, taps, r1, g, H, W, st, s);
        case LSE_F16: return Store<__half>::edge_map(src, src_dtype, B, scale, taps, r1, g, H, W, st, s);
        case LSE_BF16: return Store<__hip_bfloat16>::edge_map(src, src_dtype, B, scale, taps, r1, g, H, W, st, s);
    }
    return hipErrorInvalidValue;
}

hipError_t launch_init_image_box(const void *src, int src_dtype, int storage, int B, int NB, void *dst, int H, int W,
                                 DevState *st, float fix, float *boxes, hipStream_t s) {
    switch (storage) {
        case LSE_F32: return Store<float>::init_image_box(src, src_dtype, B, NB, dst, H, W, st, fix, boxes, s);
        case LSE_F16: return Store<__half>::init_image_box(src, src_dtype, B, NB, dst, H, W, st, fix, boxes, s);
        case LSE_BF16:
            return Store<__hip_bfloat16>::init_image_box(src, src_dtype, B, NB, dst, H, W, st, fix, boxes, s);
    }
    return hipErrorInvalidValue;
}

hipError_t launch_step(const ImgArgs *args, const uint32_t *map, const int *nmap, int unit_bits, unsigned grid, int k,
                       int stop, int r, int NB, int edge, int storage, int variant, hipStream_t s) {
    if (grid == 0) return hipSuccess;
    switch (storage) {
        case LSE_F32: return Store<float>::step(args, map, nmap, unit_bits, grid, k, stop, r, NB, edge, variant, s);
        case LSE_F16: return Store<__half>::step(args, map, nmap, unit_bits, grid, k, stop, r, NB, edge, variant, s);
        case LSE_BF16:
            return Store<__hip_bfloat16>::step(args, map, nmap, unit_bits, grid, k, stop, r, NB, edge, variant, s);
    }
    return hipErrorInvalidValue;
}

__global__ void digest_clear_kernel(DevState *st) {
    if (threadIdx.x == 0) st->digest = 0ull;
}

// Sum over the words of the current bit plane of a per-word mix of value and
// index (modulo 2^64, so the order of the atomics does not matter).
__global__ void digest_kernel(const uint32_t *__restrict__ b0, const uint32_t *__restrict__ b1, DevState *st,
                              long long nwords) {
    const uint32_t *bits = (st->iters & 1) ? b1 : b0;
    unsigned long long acc = 0ull;
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < nwords;
         i += (long long)gridDim.x * blockDim.x) {
        unsigned long long v = ((unsigned long long)bits[i] + 0x9E3779B97F4A7C15ull) * 0xBF58476D1CE4E5B9ull;
        v ^= (unsigned long long)i * 0x94D049BB133111EBull;
        acc += v ^ (v >> 31);
    }
    if (acc) atomicAdd(&st->digest, acc);
}

hipError_t launch_digest(const uint32_t *const bits[2], DevState *st, int H, int WW, hipStream_t s) {
    const long long n = (long long)H * WW;
    hipLaunchKernelGGL(digest_clear_kernel, dim3(1), dim3(64), 0, s, st);
    hipLaunchKernelGGL(digest_kernel, dim3(stream_blocks(n, 8)), dim3(kThreads), 0, s, bits[0], bits[1], st, n);
    return hipGetLastError();
}

hipError_t launch_step_generic(const StepArgs &a, int NB, int edge, int storage, hipStream_t s) {
    switch (storage) {
        case LSE_F32: return Store<float>::step_generic(a, NB, edge, s);
        case LSE_F16: return Store<__half>::step_generic(a, NB, edge, s);
        case LSE_BF16: return Store<__hip_bfloat16>::step_generic(a, NB, edge, s);
    }
    return hipErrorInvalidValue;
}

hipError_t launch_mpass(const ImgArgs *args, const uint32_t *map, int unit_bits, unsigned grid, int k, int stop,
                        int NB, int storage, hipStream_t s) {
    if (grid == 0) return hipSuccess;
    switch (storage) {
        case LSE_F32: return Store<float>::mpass(args, map, unit_bits, grid, k, stop, NB, s);
        case LSE_F16: return Store<__half>::mpass(args, map, unit_bits, grid, k, stop, NB, s);
        case LSE_BF16: return Store<__hip_bfloat16>::mpass(args, map, unit_bits, grid, k, stop, NB, s);
    }
    return hipErrorInvalidValue;
}

hipError_t launch_dense_step(const StepArgs &a, int NB, int edge, int storage, hipStream_t s) {
    switch (storage) {
        case LSE_F32: return Store<float>::dense_step(a, NB, edge, s);
        case LSE_F16: return Store<__half>::dense_step(a, NB, edge, s);
        case LSE_BF16: return Store<__hip_bfloat16>::dense_step(a, NB, edge, s);
    }
    return hipErrorInvalidValue;
}

hipError_t launch_plane_fill(const StepArgs &a, const uint32_t *bits, int raw, void *plane, int storage,
                             hipStream_t s) {
    switch (storage) {
        case LSE_F32: return Store<float>::plane_fill(a, bits, raw, plane, s);
        case LSE_F16: return Store<__half>::plane_fill(a, bits, raw, plane, s);
        case LSE_BF16: return Store<__hip_bfloat16>::plane_fill(a, bits, raw, plane, s);
    }
    return hipErrorInvalidValue;
}

hipError_t launch_plane_stats(const StepArgs &a, const void *plane, int NB, int storage, int slot, hipStream_t s) {
    switch (storage) {
        case LSE_F32: return Store<float>::plane_stats(a, plane, NB, slot, s);
        case LSE_F16: return Store<__half>::plane_stats(a, plane, NB, slot, s);
        case LSE_BF16: return Store<__hip_bfloat16>::plane_stats(a, plane, NB, slot, s);
    }
    return hipErrorInvalidValue;
}

hipError_t launch_plane_out(const void *p0, const void *p1, const DevState *st, float *out, long long n, int storage,
                            hipStream_t s) {
    switch (storage) {
        case LSE_F32: return Store<float>::plane_out(p0, p1, st, out, n, s);
        case LSE_F16: return Store<__half>::plane_out(p0, p1, st, out, n, s);
        case LSE_BF16: return Store<__hip_bfloat16>::plane_out(p0, p1, st, out, n, s);
    }
    return hipErrorInvalidValue;
}

hipError_t launch_tile_sums(const ImgArgs *args, int tiles, int r, int NB, int storage, TileSum *out, hipStream_t s) {
    switch (storage) {
        case LSE_F32: return Store<float>::tile_sums(args, tiles, r, NB, out, s);
        case LSE_F16: return Store<__half>::tile_sums(args, tiles, r, NB, out, s);
        case LSE_BF16: return Store<__hip_bfloat16>::tile_sums(args, tiles, r, NB, out, s);
    }
    return hipErrorInvalidValue;
}

hipError_t launch_batch_prepare(ImgArgs *args, int n, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(batch_prepare_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, args, n);
    return hipGetLastError();
}

hipError_t launch_mask_out(const uint32_t *const bits[2], const DevState *st, uint8_t *mask, int H, int W, int WW,
                           hipStream_t s) {
    hipLaunchKernelGGL(mask_out_kernel, dim3(seg_blocks(H, WW)), dim3(256), 0, s, bits[0], bits[1], st, mask, H, W,
                       WW);
    return hipGetLastError();
}

hipError_t launch_count_needed(const StepArgs &a, int raw, int edge, int fast_quiet, hipStream_t s) {
    const int BPR = kTileY + 2 + 2 * a.r, BCR = kTileY + 2 * a.r;
    const size_t words = (size_t)a.nch * 64 + 36 + 32 + (size_t)(BPR + BCR) * kRowWords +
                         (size_t)BPR * (kTileX + 2) + (size_t)(kTileY + 2) * (kTileX + 2);
    const hipError_t e = ensure_lds(count_needed_kernel, words * 4);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(count_needed_kernel, tile_grid(a.H, a.W), dim3(kThreads), words * 4, s, a, raw, edge,
                       fast_quiet);
    return hipGetLastError();
}

hipError_t launch_reset_profile(DevState *st, hipStream_t s) {
    hipLaunchKernelGGL(reset_profile_kernel, dim3(1), dim3(64), 0, s, st);
    return hipGetLastError();
}

hipError_t launch_lsf_out(const StepArgs &a, const uint32_t *const bits[2], int raw, float *out, hipStream_t s) {
    const size_t sm = tile_smem_bytes(a.r, a.nch, 0);
    const hipError_t e = ensure_lds(lsf_out_kernel, sm);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(lsf_out_kernel, tile_grid(a.H, a.W), dim3(kThreads), sm, s, a, bits[0], bits[1], raw, out);
    return hipGetLastError();
}

}  // namespace lse
