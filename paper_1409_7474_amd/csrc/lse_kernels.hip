// HIP kernels of the fast level set evolution (arXiv 1409.7474) for gfx950.
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
// One iteration of the region term is one fused kernel per 64 x 32 tile
// (plus, for B > 1, a read-only pass for the normaliser of eq. (17)):
//   A. stage b^{n-1} on the tile plus a halo of 2r+1 in LDS;
//   B. phi^n = G * b^{n-1} on the tile plus a halo of r+1;
//   C. data term, |grad phi^n|, Euler update eq. (18) and sign -> b^n on the
//      tile plus a halo of r (wave64 ballots build the bit words);
//   D. sign(G * b^n) on the tile -> region sums for iteration n+1 (eq. (15)),
//      reduced per wave, per workgroup, then one 64-bit atomic per band.
// The halo of phase C is recomputed by neighbouring tiles with the same
// position-only arithmetic, so every tile sees identical bits.  The edge term
// (eq. (14)) needs no statistics: its tile halo is only r+1.
//
// Region sums: FP32 within a workgroup, converted per workgroup to 64-bit
// fixed point (scale 2^s) and added atomically, so totals do not depend on
// workgroup scheduling.
#include <hip/hip_bf16.h>
#include <hip/hip_fp16.h>

#include "lse_internal.h"

namespace lse {

// ------------------------------------------------------------------ helpers

__device__ __forceinline__ unsigned int float_key(float f) {
    unsigned int u = __float_as_uint(f);
    return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}

__device__ __forceinline__ float key_float(unsigned int k) {
    unsigned int u = (k & 0x80000000u) ? (k & 0x7fffffffu) : ~k;
    return __uint_as_float(u);
}

__device__ __forceinline__ float wave_sum_f(float v) {
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m, 64);
    return v;
}

__device__ __forceinline__ int wave_sum_i(int v) {
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m, 64);
    return v;
}

__device__ __forceinline__ float wave_max_f(float v) {
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) v = fmaxf(v, __shfl_xor(v, m, 64));
    return v;
}

__device__ __forceinline__ float wave_min_f(float v) {
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) v = fminf(v, __shfl_xor(v, m, 64));
    return v;
}

__device__ __forceinline__ long long wave_sum_ll(long long v) {
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m, 64);
    return v;
}

__device__ __forceinline__ unsigned int wave_max_u(unsigned int v) {
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) v = max(v, (unsigned int)__shfl_xor(v, m, 64));
    return v;
}

__device__ __forceinline__ unsigned long long wave_max_u64(unsigned long long v) {
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) {
        const unsigned long long o = (unsigned long long)__shfl_xor((long long)v, m, 64);
        v = o > v ? o : v;
    }
    return v;
}

__device__ __forceinline__ unsigned int wave_min_u(unsigned int v) {
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) v = min(v, (unsigned int)__shfl_xor(v, m, 64));
    return v;
}

__device__ __forceinline__ int block_linear_id() { return blockIdx.y * gridDim.x + blockIdx.x; }


// Totals of one statistics slot and of the image lines, reduced over the
// kBins accumulation lines: wave 0 takes the slot (line i in lane i), wave 1
// the image lines.  Called by every thread of the workgroup.
struct Totals {
    long long sum[4];
    unsigned long long nplus, flips, mkey;
    int done, bad;
    long long total[4];
    unsigned int imin_key[4], imax_key[4];
};

__device__ __forceinline__ void load_totals(const DevState *st, int sl, bool want_img, Totals *t) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (wave == 0) {
        const Bin &b = st->slot[sl][lane];
        long long v[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) v[k] = wave_sum_ll(b.sum[k]);
        const long long np = wave_sum_ll((long long)b.nplus);
        const long long fl = wave_sum_ll((long long)b.flips);
        const unsigned long long mk = wave_max_u64(b.mkey);
        if (lane == 0) {
#pragma unroll
            for (int k = 0; k < 4; ++k) t->sum[k] = v[k];
            t->nplus = (unsigned long long)np;
            t->flips = (unsigned long long)fl;
            t->mkey = mk;
        }
    } else if (wave == 2) {
        if (lane == 0) {
            t->done = st->done;
            t->bad = st->bad;
        }
    } else if (wave == 1 && want_img) {
        const ImgBin &b = st->img[lane];
        long long v[4];
        unsigned int lo[4], hi[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            v[k] = wave_sum_ll(b.total[k]);
            lo[k] = wave_min_u(b.imin_key[k]);
            hi[k] = wave_max_u(b.imax_key[k]);
        }
        if (lane == 0) {
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                t->total[k] = v[k];
                t->imin_key[k] = lo[k];
                t->imax_key[k] = hi[k];
            }
        }
    }
    __syncthreads();
}

template <int NB>
struct Px {
    float v[NB];
};

template <int NB>
__device__ __forceinline__ Px<NB> load_px(const float *__restrict__ img, long long pix) {
    Px<NB> p;
    if constexpr (NB == 4) {
        float4 f = *reinterpret_cast<const float4 *>(img + pix * 4);
        p.v[0] = f.x;
        p.v[1] = f.y;
        p.v[2] = f.z;
        p.v[3] = f.w;
    } else if constexpr (NB == 2) {
        float2 f = *reinterpret_cast<const float2 *>(img + pix * 2);
        p.v[0] = f.x;
        p.v[1] = f.y;
    } else {
        p.v[0] = img[pix];
    }
    return p;
}

// Raw buffer loads.  The descriptor bounds the image in bytes; an offset past
// it returns zeros without touching memory.  Lanes that do not need a value
// get kNoLoad, so every load instruction is issued by the whole wave (no
// branch around it) and the compiler can count outstanding loads statically,
// which keeps several loads in flight; no bytes are read for those lanes.
constexpr uint32_t kNoLoad = 0xfffffff0u;

__device__ __forceinline__ __amdgpu_buffer_rsrc_t image_rsrc(const void *base, uint32_t bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(base), (short)0, (int)bytes, 0x00020000);
}

template <int NB>
__device__ __forceinline__ Px<NB> buffer_px(__amdgpu_buffer_rsrc_t r, uint32_t byte_off) {
    Px<NB> p;
    if constexpr (NB == 4) {
        const auto v = __builtin_amdgcn_raw_buffer_load_b128(r, byte_off, 0, 0);
#pragma unroll
        for (int b = 0; b < 4; ++b) p.v[b] = __int_as_float(v[b]);
    } else if constexpr (NB == 2) {
        const auto v = __builtin_amdgcn_raw_buffer_load_b64(r, byte_off, 0, 0);
        p.v[0] = __int_as_float(v[0]);
        p.v[1] = __int_as_float(v[1]);
    } else {
        p.v[0] = __int_as_float(__builtin_amdgcn_raw_buffer_load_b32(r, byte_off, 0, 0));
    }
    return p;
}

// Band means of eq. (15) from the fixed-point sums of one slot.
template <int NB>
__device__ __forceinline__ void slot_means(const Totals &t, long long hw, float inv_fix, float (&cp)[NB],
                                           float (&cm)[NB]) {
    const unsigned long long np = t.nplus;
    const long long nm = hw - (long long)np;
    const float fnp = (float)np, fnm = (float)nm;
#pragma unroll
    for (int b = 0; b < NB; ++b) {
        const long long S = t.sum[b];
        const long long T = t.total[b];
        cp[b] = np > 0 ? ((float)S * inv_fix) / fnp : 0.f;
        cm[b] = nm > 0 ? ((float)(T - S) * inv_fix) / fnm : 0.f;
    }
}

// Numerator of eq. (17): D = sum_b (c+ - c-)(2 I_b - c+ - c-), with
// a_b = c+ - c- and m_b = c+ + c-.  The same expression is used by every
// kernel so that the normaliser pass and the update agree bit for bit.
template <int NB>
__device__ __forceinline__ float region_D(const Px<NB> &p, const float (&a)[NB], const float (&m)[NB]) {
    float d = 0.f;
#pragma unroll
    for (int b = 0; b < NB; ++b) d = fmaf(a[b], fmaf(2.f, p.v[b], -m[b]), d);
    return d;
}

// Horizontal Gaussian of a binary row at image column x (eq. (13) values
// +1 / -1, zero outside the image).  `row` holds kRowWords bit words whose bit
// 0 is image column x0 - 32; xb is the bit position of column x.
__device__ __forceinline__ float hconv_bits(const uint32_t *row, int xb, int x, int W, int r, int ts,
                                            int nch, const float *lut, const float *cum) {
    const int ws = xb - r;
    const int wi = ws >> 5;
    const uint32_t lo = row[wi], hi = row[wi + 1];
    const uint32_t full = (1u << ts) - 1u;
    uint32_t win = __builtin_amdgcn_alignbit(hi, lo, (uint32_t)(ws & 31)) & full;
    float corr = 0.f;
    const int left = r - x;             // taps left of column 0
    const int right = x + r - (W - 1);  // taps right of column W - 1
    if (left > 0) {
        win |= (1u << left) - 1u;
        corr = cum[left];
    }
    if (right > 0) {
        win |= full & ~((1u << (ts - right)) - 1u);
        corr += cum[right];
    }
    float h = lut[win & 63u];
    for (int c = 1; c < nch; ++c) h += lut[c * 64 + ((win >> (6 * c)) & 63u)];
    return h - corr;
}

// Vertical Gaussian: acc = sum_j k[j] col[j * stride], j = 0 .. ts-1, in order.
__device__ __forceinline__ float vconv(const float *col, int stride, const float *k, int ts) {
    float acc = 0.f;
    for (int j = 0; j < ts; ++j) acc = fmaf(k[j], col[j * stride], acc);
    return acc;
}

// LDS carve-up shared by the tile kernels.
struct TileSmem {
    float *lut, *cum, *k, *h, *phi, *red;
    uint32_t *bits, *bn;
};

__host__ __device__ inline int tile_ru(int edge, int r) { return edge ? 0 : r; }

__host__ __device__ inline size_t tile_smem_words(int r, int nch, int edge) {
    const int RU = tile_ru(edge, r);
    const int UH = kTileY + 2 * RU;
    const int PH = UH + 2, PW = kTileX + 2 * RU + 2;
    const int BH = PH + 2 * r;
    size_t hwords = (size_t)BH * PW;
    if ((size_t)UH * kTileX > hwords) hwords = (size_t)UH * kTileX;
    return (size_t)nch * 64 + 36 + 32 + (size_t)BH * kRowWords + (size_t)UH * kRowWords + hwords +
           (size_t)PH * PW + 4 * 8;
}

__device__ __forceinline__ TileSmem carve(float *smem, int r, int nch, int edge) {
    const int RU = tile_ru(edge, r);
    const int UH = kTileY + 2 * RU;
    const int PH = UH + 2, PW = kTileX + 2 * RU + 2;
    const int BH = PH + 2 * r;
    size_t hwords = (size_t)BH * PW;
    if ((size_t)UH * kTileX > hwords) hwords = (size_t)UH * kTileX;
    TileSmem t;
    float *p = smem;
    t.lut = p;
    p += nch * 64;
    t.cum = p;
    p += 36;
    t.k = p;
    p += 32;
    t.bits = reinterpret_cast<uint32_t *>(p);
    p += BH * kRowWords;
    t.bn = reinterpret_cast<uint32_t *>(p);
    p += UH * kRowWords;
    t.h = p;
    p += hwords;
    t.phi = p;
    p += PH * PW;
    t.red = p;
    return t;
}

__device__ __forceinline__ void stage_tables(const TileSmem &s, const Taps *__restrict__ taps, int ts, int nch) {
    for (int i = threadIdx.x; i < nch * 64; i += kThreads) s.lut[i] = (&taps->lut[0][0])[i];
    for (int i = threadIdx.x; i <= ts; i += kThreads) s.cum[i] = taps->cum[i];
    for (int i = threadIdx.x; i < ts; i += kThreads) s.k[i] = taps->k[i];
}

// Stage bit rows [row0, row0 + nrows) of the tile's 4-word window starting
// at global word (x0 / 32) - 1; out-of-image rows and words read as 0.
__device__ __forceinline__ void stage_bits(uint32_t *dst, const uint32_t *__restrict__ bits, int row0, int nrows,
                                           int x0, int H, int WW) {
    const int wb0 = (x0 >> 5) - 1;
    for (int i = threadIdx.x; i < nrows * kRowWords; i += kThreads) {
        const int row = i / kRowWords, wc = i - row * kRowWords;
        const int y = row0 + row, gw = wb0 + wc;
        uint32_t v = 0;
        if (wc < 4 && y >= 0 && y < H && gw >= 0 && gw < WW) v = bits[(size_t)y * WW + gw];
        dst[i] = v;
    }
}

// Phase D: sign of G * b on the owned tile (b given in s.bn for rows
// y0 - r .. y0 + kTileY + r), accumulated into per-thread sums.  When raw is
// set the LSF is b itself.  Shared by the step kernel and the statistics
// kernel so that both produce identical partial sums.
template <int NB>
__device__ __forceinline__ void stats_tile(const TileSmem &s, const float *__restrict__ img, int x0, int y0,
                                           int H, int W, int r, int ts, int nch, int raw, float (&acc)[NB],
                                           int &cnt) {
    const int UH = kTileY + 2 * r;
    if (!raw) {
        for (int i = threadIdx.x; i < UH * kTileX; i += kThreads) {
            const int uy = i / kTileX, ox = i - uy * kTileX;
            const int y = y0 - r + uy, x = x0 + ox;
            float h = 0.f;
            if (y >= 0 && y < H && x < W) h = hconv_bits(s.bn + uy * kRowWords, ox + 32, x, W, r, ts, nch, s.lut, s.cum);
            s.h[i] = h;
        }
        __syncthreads();
    }
#pragma unroll
    for (int b = 0; b < NB; ++b) acc[b] = 0.f;
    cnt = 0;
    for (int k = 0; k < (kTileX * kTileY) / kThreads; ++k) {
        const int i = threadIdx.x + k * kThreads;
        const int oy = i / kTileX, ox = i - oy * kTileX;
        const int y = y0 + oy, x = x0 + ox;
        if (y < H && x < W) {
            bool inside;
            if (raw) {
                const uint32_t w = s.bn[(oy + r) * kRowWords + ((ox + 32) >> 5)];
                inside = (w >> ((ox + 32) & 31)) & 1u;
            } else {
                inside = vconv(s.h + oy * kTileX + ox, kTileX, s.k, ts) >= 0.f;
            }
            if (inside) {
                const Px<NB> p = load_px<NB>(img, (long long)y * W + x);
#pragma unroll
                for (int b = 0; b < NB; ++b) acc[b] += p.v[b];
                ++cnt;
            }
        }
    }
}

// Workgroup reduction of (NB sums, count, flips) and one atomic per value.
template <int NB>
__device__ __forceinline__ void reduce_commit(const TileSmem &s, float (&acc)[NB], int cnt, int flips, Bin *out,
                                             float fix, bool with_sums) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (with_sums) {
#pragma unroll
        for (int b = 0; b < NB; ++b) acc[b] = wave_sum_f(acc[b]);
        cnt = wave_sum_i(cnt);
    }
    flips = wave_sum_i(flips);
    if (lane == 0) {
        float *rw = s.red + wave * 8;
#pragma unroll
        for (int b = 0; b < NB; ++b) rw[b] = acc[b];
        reinterpret_cast<int *>(rw)[6] = cnt;
        reinterpret_cast<int *>(rw)[7] = flips;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        float S[NB];
        int C = 0, F = 0;
#pragma unroll
        for (int b = 0; b < NB; ++b) S[b] = 0.f;
        for (int w = 0; w < kThreads / 64; ++w) {
            const float *rw = s.red + w * 8;
#pragma unroll
            for (int b = 0; b < NB; ++b) S[b] += rw[b];
            C += reinterpret_cast<const int *>(rw)[6];
            F += reinterpret_cast<const int *>(rw)[7];
        }
        if (with_sums) {
#pragma unroll
            for (int b = 0; b < NB; ++b)
                atomicAdd(reinterpret_cast<unsigned long long *>(&out->sum[b]),
                          (unsigned long long)__float2ll_rn(S[b] * fix));
            atomicAdd(&out->nplus, (unsigned long long)C);
        }
        if (F) atomicAdd(&out->flips, (unsigned long long)F);
    }
}

// ------------------------------------------------------------- init kernels

// Zero the statistics lines (and, unless keep_image_stats, the image lines and
// the bad-value flag); mark slot 0 as having no previous iteration.
__global__ void init_state_kernel(DevState *st, int keep_image_stats) {
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
        for (int b = 0; b < 4; ++b) st->last_cp[b] = st->last_cm[b] = 0.f;
        st->last_M = 0.f;
        if (!keep_image_stats) st->bad = 0;
    }
}

template <typename T>
__device__ __forceinline__ float to_f32(T v);
template <>
__device__ __forceinline__ float to_f32<float>(float v) { return v; }
template <>
__device__ __forceinline__ float to_f32<__half>(__half v) { return __half2float(v); }
template <>
__device__ __forceinline__ float to_f32<__hip_bfloat16>(__hip_bfloat16 v) { return __bfloat162float(v); }

// Convert the caller's image to the FP32 interleaved storage (NB >= B bands,
// extra bands zero), check values, and reduce per-band min / max and totals.
template <typename T>
__global__ __launch_bounds__(kThreads) void init_image_kernel(const T *__restrict__ src, int B, int NB,
                                                              float *__restrict__ dst, long long npx,
                                                              DevState *st, float fix, int want_gray,
                                                              float gray_scale) {
    float sum[4] = {0.f, 0.f, 0.f, 0.f};
    float mn[4] = {INFINITY, INFINITY, INFINITY, INFINITY};
    float mx[4] = {-INFINITY, -INFINITY, -INFINITY, -INFINITY};
    int bad = 0;
    for (long long i = (long long)blockIdx.x * kThreads + threadIdx.x; i < npx; i += (long long)gridDim.x * kThreads) {
        float v[4] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            if (b < B) {
                v[b] = to_f32<T>(src[i * B + b]);
                if (!(fabsf(v[b]) < 65536.f)) bad = 1;  // also catches NaN / Inf
            }
        }
        if (want_gray) {
            float s = 0.f;
#pragma unroll
            for (int b = 0; b < 4; ++b)
                if (b < B) s += v[b];
            dst[i] = gray_scale * (s / (float)B);
        } else {
#pragma unroll
            for (int b = 0; b < 4; ++b)
                if (b < NB) dst[i * NB + b] = v[b];
        }
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            if (b < B) {
                sum[b] += v[b];
                mn[b] = fminf(mn[b], v[b]);
                mx[b] = fmaxf(mx[b], v[b]);
            }
        }
    }
    __shared__ float red[kThreads / 64][4][3];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (bad) st->bad = 1;
#pragma unroll
    for (int b = 0; b < 4; ++b) {
        const float s = wave_sum_f(sum[b]);
        const float lo = wave_min_f(mn[b]);
        const float hi = wave_max_f(mx[b]);
        if (lane == 0) {
            red[wave][b][0] = s;
            red[wave][b][1] = lo;
            red[wave][b][2] = hi;
        }
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        ImgBin &bin = st->img[blockIdx.x % kBins];
        for (int b = 0; b < B; ++b) {
            float s = 0.f, lo = INFINITY, hi = -INFINITY;
            for (int w = 0; w < kThreads / 64; ++w) {
                s += red[w][b][0];
                lo = fminf(lo, red[w][b][1]);
                hi = fmaxf(hi, red[w][b][2]);
            }
            if (!want_gray)
                atomicAdd(reinterpret_cast<unsigned long long *>(&bin.total[b]),
                          (unsigned long long)__float2ll_rn(s * fix));
            atomicMin(&bin.imin_key[b], float_key(lo));
            atomicMax(&bin.imax_key[b], float_key(hi));
        }
    }
}

// uint8 mask (nonzero = inside) -> bit words, bit i of word w = column 32 w + i.
__global__ void pack_mask_kernel(const uint8_t *__restrict__ mask, uint32_t *__restrict__ bits, int H, int W,
                                 int WW) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (long long)H * WW) return;
    const int y = (int)(i / WW), w = (int)(i - (long long)y * WW);
    uint32_t v = 0;
    for (int b = 0; b < 32; ++b) {
        const int x = w * 32 + b;
        if (x < W && mask[(size_t)y * W + x]) v |= 1u << b;
    }
    bits[i] = v;
}

// Region statistics of the LSF given by `bits` (raw: phi = b; else phi = G * b).
template <int NB>
__global__ __launch_bounds__(kThreads) void stats_kernel(StepArgs A, int raw, int slot) {
    extern __shared__ float smem[];
    const TileSmem s = carve(smem, A.r, A.nch, 0);
    const int x0 = blockIdx.x * kTileX, y0 = blockIdx.y * kTileY;
    stage_tables(s, A.taps, A.ts, A.nch);
    stage_bits(s.bn, A.bits_in, y0 - A.r, kTileY + 2 * A.r, x0, A.H, A.WW);
    __syncthreads();
    float acc[NB];
    int cnt;
    stats_tile<NB>(s, static_cast<const float *>(A.img), x0, y0, A.H, A.W, A.r, A.ts, A.nch, raw, acc, cnt);
    reduce_commit<NB>(s, acc, cnt, 0, &A.st->slot[slot][block_linear_id() % kBins], A.fix, true);
}

// ------------------------------------------------------------ edge map init

// out(y, x) = sum_j k[j] in(y, x + j - r)   (zero outside)
__global__ void hconv_f32_kernel(const float *__restrict__ in, float *__restrict__ out, int H, int W,
                                 const Taps *__restrict__ taps, int r) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (long long)H * W) return;
    const int y = (int)(i / W), x = (int)(i - (long long)y * W);
    float acc = 0.f;
    for (int j = 0; j <= 2 * r; ++j) {
        const int xx = x + j - r;
        if (xx >= 0 && xx < W) acc = fmaf(taps->k1[j], in[(size_t)y * W + xx], acc);
    }
    out[i] = acc;
}

// out(y, x) = sum_j k[j] in(y + j - r, x)   (zero outside)
__global__ void vconv_f32_kernel(const float *__restrict__ in, float *__restrict__ out, int H, int W,
                                 const Taps *__restrict__ taps, int r) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (long long)H * W) return;
    const int y = (int)(i / W), x = (int)(i - (long long)y * W);
    float acc = 0.f;
    for (int j = 0; j <= 2 * r; ++j) {
        const int yy = y + j - r;
        if (yy >= 0 && yy < H) acc = fmaf(taps->k1[j], in[(size_t)yy * W + x], acc);
    }
    out[i] = acc;
}

// g = 1 / (1 + |grad Is|^2), eq. (14); central differences inside, one-sided
// at the border.
__global__ void edge_g_kernel(const float *__restrict__ Is, float *__restrict__ g, int H, int W) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (long long)H * W) return;
    const int y = (int)(i / W), x = (int)(i - (long long)y * W);
    const float *row = Is + (size_t)y * W;
    float gx, gy;
    if (x == 0)
        gx = row[1] - row[0];
    else if (x == W - 1)
        gx = row[W - 1] - row[W - 2];
    else
        gx = 0.5f * (row[x + 1] - row[x - 1]);
    if (y == 0)
        gy = Is[(size_t)W + x] - Is[x];
    else if (y == H - 1)
        gy = Is[(size_t)(H - 1) * W + x] - Is[(size_t)(H - 2) * W + x];
    else
        gy = 0.5f * (Is[(size_t)(y + 1) * W + x] - Is[(size_t)(y - 1) * W + x]);
    g[i] = 1.f / (1.f + (gx * gx + gy * gy));
}

// ------------------------------------------------------------ normaliser

// Normaliser M = max_x |D(x)| of eq. (17), for B > 1 (B = 1 uses the closed
// form from the image min / max, since D is then monotone in I).
//
// Exact, with pruning: the image is cut into 64 x 32 blocks whose per-band
// min / max are stored at init.  D is affine in the pixel value, so over a
// block |D| is bounded by its value at the box corners; a rounding margin
// makes the bound hold for the FP32 D of every pixel.  The previous
// iteration's maximising pixel, evaluated with the current means, gives a
// lower bound LB <= M; only blocks whose bound reaches LB can hold the
// maximum, and only those are read.  With no previous pixel (LB = 0) every
// block is read.  The result (value and pixel) equals a full scan bit for bit.
constexpr int kMBX = 64, kMBY = 32, kMBlocksPerWG = 8;

size_t mbox_floats(int H, int W, int NB) {
    const size_t nbx = (W + kMBX - 1) / kMBX, nby = (H + kMBY - 1) / kMBY;
    return nbx * nby * 2 * NB;
}

template <int NB>
__global__ __launch_bounds__(kThreads) void mbox_kernel(const float *__restrict__ img, int H, int W,
                                                         float *__restrict__ boxes) {
    __shared__ float red[kThreads / 64][2 * NB];
    const int nbx = (W + kMBX - 1) / kMBX;
    const int bx = blockIdx.x % nbx, by = blockIdx.x / nbx;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    float lo[NB], hi[NB];
#pragma unroll
    for (int b = 0; b < NB; ++b) {
        lo[b] = INFINITY;
        hi[b] = -INFINITY;
    }
    const int x = bx * kMBX + lane;
    for (int r = wave; r < kMBY; r += kThreads / 64) {
        const int y = by * kMBY + r;
        if (x < W && y < H) {
            const Px<NB> p = load_px<NB>(img, (long long)y * W + x);
#pragma unroll
            for (int b = 0; b < NB; ++b) {
                lo[b] = fminf(lo[b], p.v[b]);
                hi[b] = fmaxf(hi[b], p.v[b]);
            }
        }
    }
#pragma unroll
    for (int b = 0; b < NB; ++b) {
        lo[b] = wave_min_f(lo[b]);
        hi[b] = wave_max_f(hi[b]);
    }
    if (lane == 0) {
#pragma unroll
        for (int b = 0; b < NB; ++b) {
            red[wave][b] = lo[b];
            red[wave][NB + b] = hi[b];
        }
    }
    __syncthreads();
    if (threadIdx.x < 2 * NB) {
        const int k = threadIdx.x;
        float v = red[0][k];
        for (int w = 1; w < kThreads / 64; ++w) v = k < NB ? fminf(v, red[w][k]) : fmaxf(v, red[w][k]);
        boxes[(size_t)blockIdx.x * 2 * NB + k] = v;
    }
}

__device__ __forceinline__ unsigned long long mkey_of(float absd, unsigned int pix) {
    return ((unsigned long long)__float_as_uint(absd) << 32) | (unsigned long long)(0xffffffffu - pix);
}

template <int NB>
__global__ __launch_bounds__(kThreads) void mpass_kernel(StepArgs A) {
    DevState *st = A.st;
    const int sl = A.n % 3;
    __shared__ Totals tot;
    __shared__ unsigned long long prev_key, wkey[kThreads / 64];
    __shared__ int scan_list[kMBlocksPerWG];
    __shared__ int nscan;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (wave == 2) {  // previous iteration's maximum (slot n - 1 == (n + 2) % 3)
        const unsigned long long k = wave_max_u64(st->slot[(A.n + 2) % 3][lane].mkey);
        if (lane == 0) prev_key = k;
    }
    // This workgroup's block boxes (lane k < kMBlocksPerWG of wave 0) do not
    // depend on the statistics: load them before the statistics barrier.
    const int nbx = (A.W + kMBX - 1) / kMBX, nby = (A.H + kMBY - 1) / kMBY, nblk = nbx * nby;
    const int myblk = blockIdx.x * kMBlocksPerWG + lane;
    float blo[NB], bhi[NB];
    if (wave == 0 && lane < kMBlocksPerWG && myblk < nblk) {
        const float *bx = A.boxes + (size_t)myblk * 2 * NB;
#pragma unroll
        for (int b = 0; b < NB; ++b) {
            blo[b] = bx[b];
            bhi[b] = bx[NB + b];
        }
    }
    load_totals(st, sl, true, &tot);
    if (tot.done || tot.bad || (A.stop && tot.flips == 0)) return;
    float cp[NB], cm[NB], a[NB], m[NB];
    slot_means<NB>(tot, A.hw, A.inv_fix, cp, cm);
#pragma unroll
    for (int b = 0; b < NB; ++b) {
        a[b] = cp[b] - cm[b];
        m[b] = cp[b] + cm[b];
    }
    const float *img = static_cast<const float *>(A.img);
    const unsigned int ppix = 0xffffffffu - (unsigned int)(prev_key & 0xffffffffu);
    const float lb = (long long)ppix < A.hw ? fabsf(region_D<NB>(load_px<NB>(img, ppix), a, m)) : 0.f;

    if (wave == 0) {
        const int blk = myblk;
        bool need = false;
        if (lane < kMBlocksPerWG && blk < nblk) {
            float dmax = 0.f, dmin = 0.f, scale = 0.f;
#pragma unroll
            for (int b = 0; b < NB; ++b) {
                const float lo = blo[b], hi = bhi[b];
                const float tl = a[b] * (2.f * lo - m[b]), th = a[b] * (2.f * hi - m[b]);
                dmax += fmaxf(tl, th);
                dmin += fminf(tl, th);
                scale += fabsf(a[b]) * (2.f * fmaxf(fabsf(lo), fabsf(hi)) + fabsf(m[b]));
            }
            // |FP32 D - exact D| <= ~6 u scale at any pixel and for dmax/dmin;
            // 2^-18 scale is a wide margin over both.
            const float ub = fmaxf(fabsf(dmax), fabsf(dmin)) + scale * 3.814697265625e-06f;
            need = ub >= lb;
        }
        const unsigned long long bal = __ballot(need);
        if (lane == 0) nscan = __popcll(bal);
        if (need) scan_list[__popcll(bal & ((1ull << lane) - 1ull))] = blk;
    }
    __syncthreads();
    unsigned long long best = 0ull;
    for (int k = 0; k < nscan; ++k) {
        const int blk = scan_list[k];
        const int bx = blk % nbx, by = blk / nbx;
        const int x = bx * kMBX + lane;
        for (int r = wave; r < kMBY; r += kThreads / 64) {
            const int y = by * kMBY + r;
            if (x < A.W && y < A.H) {
                const unsigned int pix = (unsigned int)((long long)y * A.W + x);
                const float d = fabsf(region_D<NB>(load_px<NB>(img, pix), a, m));
                const unsigned long long key = mkey_of(d, pix);
                best = key > best ? key : best;
            }
        }
    }
    best = wave_max_u64(best);
    if (lane == 0) wkey[wave] = best;
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < kThreads / 64; ++w) best = wkey[w] > best ? wkey[w] : best;
        if (best) atomicMax(&st->slot[sl][blockIdx.x % kBins].mkey, best);
    }
}

// ------------------------------------------------------------------- step

template <int NB, bool EDGE>
__global__ __launch_bounds__(kThreads) void step_kernel(StepArgs A) {
    extern __shared__ float smem[];
    __shared__ Totals tot;
    DevState *st = A.st;
    const int sl = A.n % 3;
    const bool lead_block = blockIdx.x == 0 && blockIdx.y == 0;
    const bool lead = lead_block && threadIdx.x == 0;
    load_totals(st, sl, !EDGE, &tot);
    {
        int done = st->done | st->bad;
        if (!done && A.stop && tot.flips == 0) done = 1;
        if (done) {
            if (lead && !st->bad) st->done = 1;
            return;
        }
    }
    const int r = A.r, ts = A.ts, nch = A.nch, H = A.H, W = A.W;
    const int RU = tile_ru(EDGE, r);
    const int UH = kTileY + 2 * RU;
    const int PH = UH + 2, PW = kTileX + 2 * RU + 2;
    const int BH = PH + 2 * r;
    const int x0 = blockIdx.x * kTileX, y0 = blockIdx.y * kTileY;
    const int by0 = y0 - RU - 1 - r;      // image row of staged bit row 0
    const int px0 = x0 - RU - 1, py0 = y0 - RU - 1;  // image coords of phi(0, 0)
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const TileSmem s = carve(smem, r, nch, EDGE);

    // A: tables and b^{n-1}
    stage_tables(s, A.taps, ts, nch);
    stage_bits(s.bits, A.bits_in, by0, BH, x0, H, A.WW);
    __syncthreads();

    // Data-term coefficients (identical in every workgroup).
    float a[NB], m[NB], w = 0.f;
    float cp[NB], cm[NB], M = 0.f;
    if constexpr (!EDGE) {
        slot_means<NB>(tot, A.hw, A.inv_fix, cp, cm);
#pragma unroll
        for (int b = 0; b < NB; ++b) {
            a[b] = cp[b] - cm[b];
            m[b] = cp[b] + cm[b];
        }
        if constexpr (NB == 1) {
            Px<1> lo, hi;
            lo.v[0] = key_float(tot.imin_key[0]);
            hi.v[0] = key_float(tot.imax_key[0]);
            M = fmaxf(fabsf(region_D<1>(lo, a, m)), fabsf(region_D<1>(hi, a, m)));
        } else {
            M = __uint_as_float((unsigned int)(tot.mkey >> 32));
        }
        w = M > 0.f ? A.dt / M : 0.f;
    }

    // B: phi^n on the tile + (RU + 1) halo.
    if (A.raw) {
        for (int i = tid; i < PH * PW; i += kThreads) {
            const int q = i / PW, p = i - q * PW;
            const int y = py0 + q, x = px0 + p;
            float v = 0.f;
            if (y >= 0 && y < H && x >= 0 && x < W) {
                const int xb = x - x0 + 32;
                const uint32_t wd = s.bits[(q + r) * kRowWords + (xb >> 5)];
                v = ((wd >> (xb & 31)) & 1u) ? 1.f : -1.f;
            }
            s.phi[i] = v;
        }
    } else {
        for (int i = tid; i < BH * PW; i += kThreads) {
            const int row = i / PW, p = i - row * PW;
            const int y = by0 + row, x = px0 + p;
            float h = 0.f;
            if (y >= 0 && y < H && x >= 0 && x < W)
                h = hconv_bits(s.bits + row * kRowWords, x - x0 + 32, x, W, r, ts, nch, s.lut, s.cum);
            s.h[i] = h;
        }
        __syncthreads();
        for (int i = tid; i < PH * PW; i += kThreads) {
            const int q = i / PW, p = i - q * PW;
            const int y = py0 + q, x = px0 + p;
            float v = 0.f;
            if (y >= 0 && y < H && x >= 0 && x < W) v = vconv(s.h + q * PW + p, PW, s.k, ts);
            s.phi[i] = v;
        }
    }
    __syncthreads();

    // C: update eq. (18) and binarisation on the tile + RU halo.
    for (int t = wave; t < UH * 2; t += kThreads / 64) {
        const int uy = t >> 1, half = t & 1;
        const int xb = half * 64 + lane;
        const int x = x0 - 32 + xb, y = y0 - RU + uy;
        bool pred = false;
        if (xb >= 32 - RU && xb < 96 + RU && x >= 0 && x < W && y >= 0 && y < H) {
            const int q = uy + 1, p = x - px0;
            const float *c = s.phi + q * PW + p;
            float gx, gy;
            if (x == 0)
                gx = c[1] - c[0];
            else if (x == W - 1)
                gx = c[0] - c[-1];
            else
                gx = 0.5f * (c[1] - c[-1]);
            if (y == 0)
                gy = c[PW] - c[0];
            else if (y == H - 1)
                gy = c[0] - c[-PW];
            else
                gy = 0.5f * (c[PW] - c[-PW]);
            const float gm = sqrtf(gx * gx + gy * gy);
            const long long pix = (long long)y * W + x;
            float coef;
            if constexpr (EDGE) {
                coef = A.dt * static_cast<const float *>(A.img)[pix];
            } else {
                coef = w * region_D<NB>(load_px<NB>(static_cast<const float *>(A.img), pix), a, m);
            }
            pred = fmaf(coef, gm, c[0]) >= 0.f;
        }
        const unsigned long long bal = __ballot(pred);
        if (lane == 0) {
            s.bn[uy * kRowWords + 2 * half] = (uint32_t)bal;
            s.bn[uy * kRowWords + 2 * half + 1] = (uint32_t)(bal >> 32);
            if (half) s.bn[uy * kRowWords + 4] = 0u;
        }
    }
    __syncthreads();

    // Owned words of b^n to global memory, and flips against b^{n-1}.
    int flips = 0;
    if (tid < kTileY * 2) {
        const int row = tid >> 1, wsel = tid & 1;
        const int y = y0 + row, gw = (x0 >> 5) + wsel;
        if (y < H && gw < A.WW) {
            const int xs = gw * 32;
            const uint32_t valid = (W - xs >= 32) ? ~0u : ((1u << (W - xs)) - 1u);
            const uint32_t nw = s.bn[(row + RU) * kRowWords + 1 + wsel] & valid;
            const uint32_t ow = s.bits[(row + RU + 1 + r) * kRowWords + 1 + wsel] & valid;
            A.bits_out[(size_t)y * A.WW + gw] = nw;
            flips = __popc(nw ^ ow);
        }
    }

    Bin *out = &st->slot[(A.n + 1) % 3][block_linear_id() % kBins];
    float acc[NB];
#pragma unroll
    for (int b = 0; b < NB; ++b) acc[b] = 0.f;
    int cnt = 0;
    if constexpr (!EDGE) {
        // D: statistics of phi^{n+1} = G * b^n for the next iteration.
        stats_tile<NB>(s, static_cast<const float *>(A.img), x0, y0, H, W, r, ts, nch, 0, acc, cnt);
    }
    reduce_commit<NB>(s, acc, cnt, flips, out, A.fix, !EDGE);

    if (lead_block) {
        // Clear the slot of iteration n + 2 (nobody reads or writes it now).
        unsigned long long *z = reinterpret_cast<unsigned long long *>(&st->slot[(A.n + 2) % 3][0]);
        for (int i = threadIdx.x; i < (int)(kBins * sizeof(Bin) / 8); i += kThreads) z[i] = 0ull;
    }
    if (lead) {
        st->iters += 1;
        if constexpr (!EDGE) {
            for (int b = 0; b < NB; ++b) {
                st->last_cp[b] = cp[b];
                st->last_cm[b] = cm[b];
            }
            st->last_M = M;
        }
    }
}

// ------------------------------------------------------------- fast step
//
// Same arithmetic as step_kernel, organised for throughput when the template
// radius R is a compile-time constant: tiles of 96 owned columns x 64 owned
// rows, lanes mapped to columns, each wave taking a vertical segment of rows
// so that the vertical Gaussian runs over a register window (each horizontal
// sum computed once per segment).  The 6-bit lookup tables live in one VGPR
// per chunk and are read with ds_bpermute (a crossbar, no bank conflicts).

constexpr int kFX = 96;        // owned columns (3 bit words)
constexpr int kFY = 64;        // owned rows
constexpr int kFWords = 6;     // staged bit words per row: global words x0/32 - 1 .. x0/32 + 4

constexpr int kSB = 8;         // rows per block of the rolling vertical window
constexpr int kCG = 4;         // rows per group of data-term loads in the binarisation phase

template <int R, bool EDGE>
struct FastGeom {
    static constexpr int TS = 2 * R + 1;
    static constexpr int RU = EDGE ? 0 : R;      // halo of the binarised field
    static constexpr int UH = kFY + 2 * RU;      // rows where b^n is computed
    static constexpr int PH = UH + 2;            // rows of phi^n
    static constexpr int PW = kFX + 2 * RU + 2;  // columns of phi^n (<= 128)
    static constexpr int NBLK = (PH + 2 * kSB - 1) / (2 * kSB);  // window blocks per segment
    static constexpr int SEG = NBLK * kSB;       // phi rows per wave (2 segments x 2 chunks)
    static constexpr int PHP = 2 * SEG;          // phi rows allocated (>= PH)
    static constexpr int BH = PHP + 2 * R;       // staged rows of b^{n-1}
    static constexpr int SEGD = kFY / 2;         // statistics rows per wave
    static constexpr int NCH = (TS + 5) / 6;     // lookup chunks
    static constexpr int PS = PW;                // phi row stride (floats)
    static constexpr int smem_words = BH * kFWords + PHP * PS + UH * kFWords + BH * 2 + PHP * 2 + 16;
};

template <int NCH>
__device__ __forceinline__ void load_luts(const Taps *__restrict__ taps, int (&lut)[NCH]) {
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int c = 0; c < NCH; ++c) lut[c] = __float_as_int(taps->lut[c][lane]);
}

// Horizontal Gaussian of a binary row, as hconv_bits; must be called with all
// 64 lanes active (ds_bpermute).  `border` (uniform) enables the zero-padding
// correction, needed only by tiles that touch the left or right image edge.
template <int R, int NCH>
__device__ __forceinline__ float hconv_fast(const uint32_t *row, int xb, int x, int W, bool border,
                                            const int (&lut)[NCH], const float *__restrict__ cum) {
    constexpr int TS = 2 * R + 1;
    constexpr uint32_t FULL = (1u << TS) - 1u;
    const int ws = xb - R;
    const int wi = ws >> 5;
    uint32_t win = __builtin_amdgcn_alignbit(row[wi + 1], row[wi], (uint32_t)(ws & 31)) & FULL;
    float corr = 0.f;
    if (border) {
        const int left = min(R - x, TS);
        const int right = min(x + R - (W - 1), TS);
        if (left > 0) {
            win |= (1u << left) - 1u;
            corr = cum[left];
        }
        if (right > 0) {
            win |= FULL & ~((1u << (TS - right)) - 1u);
            corr += cum[right];
        }
    }
    float h = 0.f;
#pragma unroll
    for (int c = 0; c < NCH; ++c) {
        const int idx = (int)((win >> (6 * c)) & 63u);
        h += __int_as_float(__builtin_amdgcn_ds_bpermute(idx << 2, lut[c]));
    }
    return h - corr;
}

__device__ __forceinline__ uint32_t bits_extract(unsigned long long m, int off, int k) {
    const int d = 32 * k - off;  // right shift that brings word k of the row to bit 0
    if (d >= 64 || d <= -32) return 0u;
    return d >= 0 ? (uint32_t)(m >> d) : (uint32_t)(m << (-d));
}

// 0 if bits [lo, hi) of a staged row are all 0, 1 if all 1, 2 if mixed.
__device__ __forceinline__ int range_code(const uint32_t *row, int lo, int hi) {
    uint32_t any1 = 0u, any0 = 0u;
    const int j0 = lo >> 5, j1 = (hi - 1) >> 5;
    for (int j = j0; j <= j1; ++j) {
        uint32_t m = ~0u;
        if (j == j0) m &= ~0u << (lo & 31);
        if (j == j1) m &= ~0u >> (31 - ((hi - 1) & 31));
        any1 |= row[j] & m;
        any0 |= ~row[j] & m;
    }
    return (any1 && any0) ? 2 : (any1 ? 1 : 0);
}

// Wave-uniform test: do rows [row0, row0 + n) all carry code c (0 or 1)?
// Returns 1 (all ones), 0 (all zeros) or -1.  n <= 64.
__device__ __forceinline__ int block_code(const int *codes, int row0, int n, int chunk) {
    const int lane = (int)threadIdx.x & 63;
    const int c = lane < n ? codes[(row0 + lane) * 2 + chunk] : -1;
    const unsigned long long full = (n >= 64) ? ~0ull : ((1ull << n) - 1ull);
    if (__ballot(c == 1) == full) return 1;
    if (__ballot(c == 0) == full) return 0;
    return -1;
}

// Stage bit rows [row0, row0 + nrows) of global words x0/32 - 1 .. x0/32 + 4.
__device__ __forceinline__ void stage_bits_fast(uint32_t *dst, const uint32_t *__restrict__ bits, int row0,
                                                int nrows, int x0, int H, int WW) {
    const int wb0 = (x0 >> 5) - 1;
    for (int i = threadIdx.x; i < nrows * kFWords; i += kThreads) {
        const int row = i / kFWords, wc = i - row * kFWords;
        const int y = row0 + row, gw = wb0 + wc;
        uint32_t v = 0;
        if (wc < kFWords - 1 && y >= 0 && y < H && gw >= 0 && gw < WW) v = bits[(size_t)y * WW + gw];
        dst[i] = v;
    }
}

// Codes of the owned-column spans of the U rows (b^n): chunk 0 = owned
// columns 0..63, chunk 1 = 64..95, each with its R halo.
template <int R>
__device__ __forceinline__ void code_rows_owned(const uint32_t *bn, int nrows, int *codes) {
    for (int i = (int)threadIdx.x; i < nrows * 2; i += kThreads) {
        const int row = i >> 1, c = i & 1;
        codes[i] = c == 0 ? range_code(bn + row * kFWords, 32 - R, 96 + R)
                          : range_code(bn + row * kFWords, 96 - R, 128 + R);
    }
}

// Statistics of phi^{n+1} = G * b on the owned 96 x 64 tile (b in `bn`, rows
// y0 - R .. y0 + 64 + R, bit 0 of each row = column x0 - 32).  raw: phi = b.
// Every owned pixel of the image is read once (dense streaming); blocks of
// 8 rows whose whole bit window is uniform take the sign without the
// Gaussian sums (their value would be the same constant in every pixel).
template <int R, int NB>
__device__ __forceinline__ void stats_fast(const uint32_t *bn, const int *codes, const float *__restrict__ img,
                                           int x0, int y0, int H, int W, bool border, bool raw,
                                           const int (&lut)[FastGeom<R, false>::NCH], const float (&kk)[2 * R + 1],
                                           const float *__restrict__ cum, float (&acc)[NB], int &cnt) {
    using G = FastGeom<R, false>;
    static_assert(G::SEGD % kSB == 0, "statistics segment must be a whole number of blocks");
    const int tid = (int)threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int chunk = wave & 1, seg = wave >> 1;
    const int ox = chunk * 64 + lane;
    const int x = x0 + ox;
    const bool colok = ox < kFX && x < W;
#pragma unroll
    for (int b = 0; b < NB; ++b) acc[b] = 0.f;
    cnt = 0;
    const int urow0 = seg * G::SEGD;  // U row of output row 0 of this segment's window
    static_assert(G::SEGD <= 32, "inside flags of a segment fit one 32-bit mask");
    // Pass 1: which output rows of this lane's column are on the + side.
    uint32_t inmask = 0u;
    if (raw) {
        for (int j = 0; j < G::SEGD; ++j) {
            const uint32_t wd = bn[(urow0 + j + R) * kFWords + ((ox + 32) >> 5)];
            inmask |= ((wd >> ((ox + 32) & 31)) & 1u) << j;
        }
    } else {
        constexpr int NW = 2 * R + kSB;
        float win[NW];
        bool have_win = false;  // win[0 .. 2R) holds rows rb .. rb + 2R of the current block
#pragma unroll 1
        for (int blk = 0; blk < G::SEGD / kSB; ++blk) {
            const int rb = urow0 + blk * kSB;
            const int yb = y0 - R + rb;  // image row of U row rb
            int uni = -1;
            if (!border && yb >= 0 && yb + kSB + 2 * R <= H) uni = block_code(codes, rb, kSB + 2 * R, chunk);
            if (uni >= 0) {
                // Uniform block: every pixel has the sign of the constant.
                if (uni == 1) inmask |= ((1u << kSB) - 1u) << (blk * kSB);
                have_win = false;
                continue;
            }
            if (!have_win) {
#pragma unroll
                for (int t = 0; t < 2 * R; ++t) {
                    const int y = yb + t;
                    const float v = hconv_fast<R, G::NCH>(bn + (rb + t) * kFWords, ox + 32, x, W, border, lut, cum);
                    win[t] = (y >= 0 && y < H) ? v : 0.f;
                }
            }
#pragma unroll
            for (int t = 0; t < kSB; ++t) {
                const int urow = rb + 2 * R + t;
                const int y = y0 - R + urow;
                const float v = hconv_fast<R, G::NCH>(bn + urow * kFWords, ox + 32, x, W, border, lut, cum);
                win[2 * R + t] = (y >= 0 && y < H) ? v : 0.f;
            }
#pragma unroll
            for (int j = 0; j < kSB; ++j) {
                float ph = 0.f;
#pragma unroll
                for (int i = 0; i < 2 * R + 1; ++i) ph = fmaf(kk[i], win[j + i], ph);
                inmask |= (ph >= 0.f ? 1u : 0u) << (blk * kSB + j);
            }
#pragma unroll
            for (int t = 0; t < 2 * R; ++t) win[t] = win[t + kSB];
            have_win = true;
        }
    }
    // Pass 2: add the image values of the + side rows in row order.  Loads
    // of one group of rows are in flight while the previous group is added;
    // only + side pixels are read (the others get kNoLoad).
    if (!colok) inmask = 0u;
    const int nrows = min(G::SEGD, H - (y0 + urow0));
    if (nrows < G::SEGD) inmask &= nrows > 0 ? ((1u << nrows) - 1u) : 0u;
    const __amdgpu_buffer_rsrc_t rs = image_rsrc(img, (uint32_t)((unsigned long long)H * W * NB * 4));
    const uint32_t off0 = (uint32_t)(((y0 + urow0) * W + x) * NB * 4);
    const uint32_t rstride = (uint32_t)(W * NB * 4);
    constexpr int GR = 4;
    Px<NB> ba[GR], bb[GR];
    auto load_group = [&](Px<NB>(&buf)[GR], int g) {
#pragma unroll
        for (int i = 0; i < GR; ++i) {
            const int j = g * GR + i;
            buf[i] = buffer_px<NB>(rs, ((inmask >> j) & 1u) ? off0 + j * rstride : kNoLoad);
        }
    };
    auto add_group = [&](const Px<NB>(&buf)[GR], int g) {
#pragma unroll
        for (int i = 0; i < GR; ++i) {
            const bool in = (inmask >> (g * GR + i)) & 1u;
#pragma unroll
            for (int b = 0; b < NB; ++b) acc[b] += in ? buf[i].v[b] : 0.f;
            cnt += in ? 1 : 0;
        }
    };
    constexpr int NG = G::SEGD / GR;
    static_assert(NG % 2 == 0, "groups come in pairs");
    load_group(ba, 0);
#pragma unroll 1
    for (int g = 0; g < NG; g += 2) {
        load_group(bb, g + 1);
        add_group(ba, g);
        if (g + 2 < NG) load_group(ba, g + 2);
        add_group(bb, g + 1);
    }
}

// Tile of this workgroup.  Workgroup j runs on XCD j % 8 (the hardware
// dispatches workgroups round-robin over the 8 XCDs); each XCD takes a
// contiguous band of tile rows, so tiles that re-read each other's halo share
// that XCD's L2.  The grid is the tile count rounded up to a multiple of 8;
// returns -1 for the spare workgroups.
__device__ __forceinline__ int tile_of(int ntiles) {
    const int g = gridDim.x, j = blockIdx.x;
    if ((g & 7) != 0) return j < ntiles ? j : -1;
    const int xcd = j & 7, per = g >> 3;
    const int lo = (int)((long long)ntiles * xcd / 8), hi = (int)((long long)ntiles * (xcd + 1) / 8);
    const int t = lo + (j >> 3);
    return (t < hi && (j >> 3) < per) ? t : -1;
}

template <int R, int NB, bool EDGE>
__global__ __launch_bounds__(kThreads) void step_fast_kernel(StepArgs A) {
    using G = FastGeom<R, EDGE>;
    constexpr int TS = G::TS;
    extern __shared__ float smem[];
    __shared__ Totals tot;
    __shared__ float red[kThreads / 64 * 8];
    DevState *st = A.st;
    const int sl = A.n % 3;
    const bool lead_block = blockIdx.x == 0;
    const bool lead = lead_block && threadIdx.x == 0;
    const int H = A.H, W = A.W;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int ntx = (W + kFX - 1) / kFX, nty = (H + kFY - 1) / kFY;
    const int t = tile_of(ntx * nty);
    const int x0 = (t >= 0 ? t % ntx : 0) * kFX, y0 = (t >= 0 ? t / ntx : 0) * kFY;
    const int by0 = y0 - G::RU - 1 - R;  // image row of staged bit row 0
    const int px0 = x0 - G::RU - 1, py0 = y0 - G::RU - 1;
    const bool border = x0 - 2 * R - 2 < 0 || x0 + kFX + 2 * R + 2 > W;
    uint32_t *s_bits = reinterpret_cast<uint32_t *>(smem);
    float *s_phi = smem + G::BH * kFWords;
    uint32_t *s_bn = reinterpret_cast<uint32_t *>(s_phi + G::PHP * G::PS);
    int *s_codes = reinterpret_cast<int *>(s_bn + G::UH * kFWords);    // [max(BH, UH)][2]
    int *s_pcode = s_codes + G::BH * 2;                                  // [PHP][2]: phi row uniformity
    uint32_t *s_const = reinterpret_cast<uint32_t *>(s_pcode + G::PHP * 2);  // all-ones / all-zeros rows

    // A: b^{n-1} on the tile + 2R+1 halo.  Issued before the statistics
    // loads so that the two memory round trips overlap.
    if (t >= 0) stage_bits_fast(s_bits, A.bits_in, by0, G::BH, x0, H, A.WW);
    if (tid < 16) s_const[tid] = tid < 8 ? ~0u : 0u;
    // Tables do not depend on the statistics either: load them before the
    // statistics barrier (one memory round trip for the whole set-up).
    int lut[G::NCH];
    load_luts<G::NCH>(A.taps, lut);
    float kk[TS];
#pragma unroll
    for (int i = 0; i < TS; ++i) kk[i] = A.taps->k[i];
    const float *cum = A.taps->cum;
    load_totals(st, sl, !EDGE, &tot);
    {
        int done = tot.done | tot.bad;
        if (!done && A.stop && tot.flips == 0) done = 1;
        if (done) {
            if (lead && !tot.bad) st->done = 1;
            return;
        }
    }

    float a[NB], m[NB], w = 0.f;
    float cp[NB], cm[NB], M = 0.f;
    if constexpr (!EDGE) {
        slot_means<NB>(tot, A.hw, A.inv_fix, cp, cm);
#pragma unroll
        for (int b = 0; b < NB; ++b) {
            a[b] = cp[b] - cm[b];
            m[b] = cp[b] + cm[b];
        }
        if constexpr (NB == 1) {
            Px<1> lo, hi;
            lo.v[0] = key_float(tot.imin_key[0]);
            hi.v[0] = key_float(tot.imax_key[0]);
            M = fmaxf(fabsf(region_D<1>(lo, a, m)), fabsf(region_D<1>(hi, a, m)));
        } else {
            M = __uint_as_float((unsigned int)(tot.mkey >> 32));
        }
        w = M > 0.f ? A.dt / M : 0.f;
    }
    // LSF value of an all-ones / all-zeros window (same arithmetic as any pixel).
    float phi_one = 0.f, phi_zero = 0.f;
    {
        const float h1 = hconv_fast<R, G::NCH>(s_const, 64, 64, 1 << 30, false, lut, cum);
        const float h0 = hconv_fast<R, G::NCH>(s_const + 8, 64, 64, 1 << 30, false, lut, cum);
#pragma unroll
        for (int i = 0; i < TS; ++i) {
            phi_one = fmaf(kk[i], h1, phi_one);
            phi_zero = fmaf(kk[i], h0, phi_zero);
        }
    }
    const __amdgpu_buffer_rsrc_t img_rs =
        image_rsrc(A.img, (uint32_t)((unsigned long long)H * W * (EDGE ? 1 : NB) * 4));
    // U-row words of an all-ones binarised row (the two ballots' valid lanes).
    const unsigned long long ones1 = (32 + 2 * G::RU >= 64) ? ~0ull : ((1ull << (32 + 2 * G::RU)) - 1ull);

    if (t >= 0) {
        // Codes of the staged rows over each chunk's window span.
        for (int i = tid; i < G::BH * 2; i += kThreads) {
            const int row = i >> 1, c = i & 1;
            s_codes[i] = c == 0 ? range_code(s_bits + row * kFWords, 31 - G::RU - R, 95 - G::RU + R)
                                : range_code(s_bits + row * kFWords, 95 - G::RU - R, 129 + G::RU + R);
        }
        __syncthreads();

        // B: phi^n on P = tile + (RU + 1) halo; wave = (column chunk, row segment).
        {
            const int chunk = wave & 1, seg = wave >> 1;
            const int p = chunk * 64 + lane;
            const int x = px0 + p;
            const int xb = x - x0 + 32;
            const bool colok = p < G::PW && x >= 0 && x < W;
            if (A.raw) {
                for (int j = 0; j < G::SEG; ++j) {
                    const int q = seg * G::SEG + j, y = py0 + q;
                    float v = 0.f;
                    if (colok && y >= 0 && y < H) {
                        const uint32_t wd = s_bits[(q + R) * kFWords + (xb >> 5)];
                        v = ((wd >> (xb & 31)) & 1u) ? 1.f : -1.f;
                    }
                    if (p < G::PW) s_phi[q * G::PS + p] = v;
                    if (lane == 0) s_pcode[q * 2 + chunk] = 2;
                }
            } else {
                constexpr int NW = 2 * R + kSB;
                float win[NW];
                const int brow0 = seg * G::SEG;  // staged bit row of window entry 0
                bool have_win = false;
#pragma unroll 1
                for (int blk = 0; blk < G::NBLK; ++blk) {
                    const int rb = brow0 + blk * kSB;
                    int uni = -1;
                    if (!border && by0 + rb >= 0 && by0 + rb + kSB + 2 * R <= H)
                        uni = block_code(s_codes, rb, kSB + 2 * R, chunk);
                    if (uni >= 0) {
                        const float v = uni ? phi_one : phi_zero;
#pragma unroll
                        for (int j = 0; j < kSB; ++j) {
                            const int q = rb + j;
                            if (p < G::PW) s_phi[q * G::PS + p] = colok ? v : 0.f;
                        }
                        if (lane < kSB) s_pcode[(rb + lane) * 2 + chunk] = uni;
                        have_win = false;
                        continue;
                    }
                    if (!have_win) {
#pragma unroll
                        for (int t2 = 0; t2 < 2 * R; ++t2) {
                            const int y = by0 + rb + t2;
                            const float v =
                                hconv_fast<R, G::NCH>(s_bits + (rb + t2) * kFWords, xb, x, W, border, lut, cum);
                            win[t2] = (y >= 0 && y < H) ? v : 0.f;
                        }
                    }
#pragma unroll
                    for (int t2 = 0; t2 < kSB; ++t2) {
                        const int brow = rb + 2 * R + t2;
                        const int y = by0 + brow;
                        const float v = hconv_fast<R, G::NCH>(s_bits + brow * kFWords, xb, x, W, border, lut, cum);
                        win[2 * R + t2] = (y >= 0 && y < H) ? v : 0.f;
                    }
#pragma unroll
                    for (int j = 0; j < kSB; ++j) {
                        float ph = 0.f;
#pragma unroll
                        for (int i = 0; i < TS; ++i) ph = fmaf(kk[i], win[j + i], ph);
                        const int q = rb + j, y = py0 + q;  // phi row q <-> bit rows q .. q + 2R
                        if (p < G::PW) s_phi[q * G::PS + p] = (colok && y >= 0 && y < H) ? ph : 0.f;
                    }
                    if (lane < kSB) s_pcode[(rb + lane) * 2 + chunk] = 2;
#pragma unroll
                    for (int t2 = 0; t2 < 2 * R; ++t2) win[t2] = win[t2 + kSB];
                    have_win = true;
                }
            }
        }
        __syncthreads();

        // C: update eq. (18) and binarisation on U = tile + RU halo, in blocks
        // of 8 rows per wave task; blocks whose phi rows are one uniform
        // constant (interior tiles) have |grad phi| = 0: b = sign(phi).
        int flips = 0;
        constexpr int NBC = (G::UH + kSB - 1) / kSB;
#pragma unroll 1
        for (int bi = wave; bi < NBC; bi += kThreads / 64) {
            const int u0 = bi * kSB;
            const int nr = min(kSB, G::UH - u0);
            int rc = -1;
            if (!border) {
                const int ncode = (nr + 2) * 2;  // phi rows u0 .. u0 + nr + 1, both chunks
                const int c = lane < ncode ? s_pcode[u0 * 2 + lane] : -1;
                const unsigned long long full = (1ull << ncode) - 1ull;
                if (__ballot(c == 1) == full)
                    rc = 1;
                else if (__ballot(c == 0) == full)
                    rc = 0;
            }
            if (rc >= 0) {
                if (lane < nr * kFWords) {
                    const int r = lane / kFWords, k = lane - r * kFWords;
                    const int uy = u0 + r, y = y0 - G::RU + uy;
                    const uint32_t word = rc ? (bits_extract(~0ull, 32 - G::RU, k) |
                                                bits_extract(ones1, 96 - G::RU, k))
                                             : 0u;
                    s_bn[uy * kFWords + k] = word;
                    const int gw = (x0 >> 5) - 1 + k;
                    if (k >= 1 && k <= 3 && uy >= G::RU && uy < G::RU + kFY && y < H && gw < A.WW) {
                        const int xs = gw * 32;
                        const uint32_t valid = (W - xs >= 32) ? ~0u : ((1u << (W - xs)) - 1u);
                        const uint32_t nw = word & valid;
                        const uint32_t ow = s_bits[(uy + 1 + R) * kFWords + k] & valid;
                        A.bits_out[(size_t)y * A.WW + gw] = nw;
                        flips += __popc(nw ^ ow);
                    }
                }
                continue;
            }
            // Rows in groups of kCG: gradients first (LDS), then every data-term
            // load of the group, then the updates, so that one memory round
            // trip serves the whole group.
#pragma unroll 1
            for (int r0 = 0; r0 < nr; r0 += kCG) {
                float phv[kCG][2], gmv[kCG][2];
                bool need[kCG][2], pred[kCG][2];
                int pixv[kCG][2];
#pragma unroll
                for (int i = 0; i < kCG; ++i) {
                    const int uy = u0 + r0 + i;
                    const int y = y0 - G::RU + uy;
                    const bool rowok = r0 + i < nr && y >= 0 && y < H;
#pragma unroll
                    for (int c = 0; c < 2; ++c) {
                        const int xb = 32 - G::RU + c * 64 + lane;
                        const int x = x0 - 32 + xb;
                        need[i][c] = false;
                        pred[i][c] = false;
                        phv[i][c] = 0.f;
                        gmv[i][c] = 0.f;
                        pixv[i][c] = 0;
                        if (rowok && xb < 128 + G::RU && x >= 0 && x < W) {
                            const int p = c * 64 + lane + 1;
                            const float *cc = s_phi + (uy + 1) * G::PS + p;
                            float gx, gy;
                            if (x == 0)
                                gx = cc[1] - cc[0];
                            else if (x == W - 1)
                                gx = cc[0] - cc[-1];
                            else
                                gx = 0.5f * (cc[1] - cc[-1]);
                            if (y == 0)
                                gy = cc[G::PS] - cc[0];
                            else if (y == H - 1)
                                gy = cc[0] - cc[-G::PS];
                            else
                                gy = 0.5f * (cc[G::PS] - cc[-G::PS]);
                            phv[i][c] = cc[0];
                            pred[i][c] = cc[0] >= 0.f;  // |grad phi| = 0: u = phi exactly (eq. (18))
                            if (!(gx == 0.f && gy == 0.f)) {
                                need[i][c] = true;
                                gmv[i][c] = sqrtf(gx * gx + gy * gy);
                                pixv[i][c] = y * W + x;
                            }
                        }
                    }
                }
                float coef[kCG][2];
                {
                    constexpr int NV = EDGE ? 1 : NB;  // values per pixel: edge map or image bands
                    Px<NV> v[kCG][2];
#pragma unroll
                    for (int i = 0; i < kCG; ++i)
#pragma unroll
                        for (int c = 0; c < 2; ++c)
                            v[i][c] = buffer_px<NV>(img_rs, need[i][c] ? (uint32_t)pixv[i][c] * (NV * 4) : kNoLoad);
#pragma unroll
                    for (int i = 0; i < kCG; ++i)
#pragma unroll
                        for (int c = 0; c < 2; ++c) {
                            if constexpr (EDGE)
                                coef[i][c] = A.dt * v[i][c].v[0];
                            else
                                coef[i][c] = w * region_D<NB>(v[i][c], a, m);
                        }
                }
#pragma unroll
                for (int i = 0; i < kCG; ++i) {
                    if (r0 + i >= nr) break;
                    const int uy = u0 + r0 + i;
                    const int y = y0 - G::RU + uy;
                    const bool rowok = y >= 0 && y < H;
#pragma unroll
                    for (int c = 0; c < 2; ++c)
                        if (need[i][c]) pred[i][c] = fmaf(coef[i][c], gmv[i][c], phv[i][c]) >= 0.f;
                    const unsigned long long m0 = __ballot(pred[i][0]);
                    const unsigned long long m1 = __ballot(pred[i][1]);
                    if (lane < kFWords) {
                        const uint32_t word = bits_extract(m0, 32 - G::RU, lane) | bits_extract(m1, 96 - G::RU, lane);
                        s_bn[uy * kFWords + lane] = word;
                        const int gw = (x0 >> 5) - 1 + lane;
                        if (lane >= 1 && lane <= 3 && uy >= G::RU && uy < G::RU + kFY && rowok && gw < A.WW) {
                            const int xs = gw * 32;
                            const uint32_t valid = (W - xs >= 32) ? ~0u : ((1u << (W - xs)) - 1u);
                            const uint32_t nw = word & valid;
                            const uint32_t ow = s_bits[(uy + 1 + R) * kFWords + lane] & valid;
                            A.bits_out[(size_t)y * A.WW + gw] = nw;
                            flips += __popc(nw ^ ow);
                        }
                    }
                }
            }
        }
        __syncthreads();

        float acc[NB];
#pragma unroll
        for (int b = 0; b < NB; ++b) acc[b] = 0.f;
        int cnt = 0;
        if constexpr (!EDGE) {
            // D: statistics of phi^{n+1} = G * b^n for the next iteration.
            code_rows_owned<R>(s_bn, G::UH, s_codes);
            __syncthreads();
            stats_fast<R, NB>(s_bn, s_codes, static_cast<const float *>(A.img), x0, y0, H, W, border, false, lut,
                              kk, cum, acc, cnt);
        }
        TileSmem rs;
        rs.red = red;
        reduce_commit<NB>(rs, acc, cnt, flips, &st->slot[(A.n + 1) % 3][blockIdx.x % kBins], A.fix, !EDGE);
    }
    if (lead_block) {
        // Clear the slot of iteration n + 2 (nobody reads or writes it now).
        unsigned long long *z = reinterpret_cast<unsigned long long *>(&st->slot[(A.n + 2) % 3][0]);
        for (int i = threadIdx.x; i < (int)(kBins * sizeof(Bin) / 8); i += kThreads) z[i] = 0ull;
    }
    if (lead) {
        st->iters += 1;
        if constexpr (!EDGE) {
            for (int b = 0; b < NB; ++b) {
                st->last_cp[b] = cp[b];
                st->last_cm[b] = cm[b];
            }
            st->last_M = M;
        }
    }
}

// Region statistics on the fast tiling (used at init and by set_mask so that
// its partial sums equal the step kernel's bit for bit).
template <int R, int NB>
__global__ __launch_bounds__(kThreads) void stats_fast_kernel(StepArgs A, int raw, int slot) {
    extern __shared__ float smem[];
    __shared__ float red[kThreads / 64 * 8];
    using G = FastGeom<R, false>;
    uint32_t *s_bn = reinterpret_cast<uint32_t *>(smem);
    const int x0 = blockIdx.x * kFX, y0 = blockIdx.y * kFY;
    const bool border = x0 - 2 * R - 2 < 0 || x0 + kFX + 2 * R + 2 > A.W;
    int lut[G::NCH];
    load_luts<G::NCH>(A.taps, lut);
    float kk[2 * R + 1];
#pragma unroll
    for (int i = 0; i < 2 * R + 1; ++i) kk[i] = A.taps->k[i];
    int *s_codes = reinterpret_cast<int *>(s_bn + G::UH * kFWords);
    stage_bits_fast(s_bn, A.bits_in, y0 - R, G::UH, x0, A.H, A.WW);
    __syncthreads();
    code_rows_owned<R>(s_bn, G::UH, s_codes);
    __syncthreads();
    float acc[NB];
    int cnt;
    stats_fast<R, NB>(s_bn, s_codes, static_cast<const float *>(A.img), x0, y0, A.H, A.W, border, raw != 0, lut,
                      kk, A.taps->cum, acc, cnt);
    TileSmem rs;
    rs.red = red;
    reduce_commit<NB>(rs, acc, cnt, 0, &A.st->slot[slot][block_linear_id() % kBins], A.fix, true);
}

// --------------------------------------------------------------- exports

__global__ void mask_out_kernel(const uint32_t *__restrict__ b0, const uint32_t *__restrict__ b1,
                                const DevState *__restrict__ st, uint8_t *__restrict__ mask, int H, int W, int WW) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (long long)H * W) return;
    const int y = (int)(i / W), x = (int)(i - (long long)y * W);
    const uint32_t *bits = (st->iters & 1) ? b1 : b0;
    mask[i] = (bits[(size_t)y * WW + (x >> 5)] >> (x & 31)) & 1u;
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
__global__ __launch_bounds__(kThreads) void count_needed_kernel(StepArgs A, int raw, int edge) {
    extern __shared__ float smem[];
    __shared__ int part[kThreads / 64];
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
        if (!edge) need = need || vconv(h + oy * kTileX + ox, kTileX, k, ts) >= 0.f;
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
    }
}

// ---------------------------------------------------------------- launchers

// Workgroups may use more than 64 KB of LDS (gfx950 has 160 KB per CU) for
// large templates; raise the per-kernel limit when a launch needs it.
template <typename K>
static hipError_t ensure_lds(K kernel, size_t bytes) {
    if (bytes <= 65536) return hipSuccess;
    return hipFuncSetAttribute(reinterpret_cast<const void *>(kernel), hipFuncAttributeMaxDynamicSharedMemorySize,
                               (int)bytes);
}

static inline dim3 tile_grid(int H, int W) { return dim3((W + kTileX - 1) / kTileX, (H + kTileY - 1) / kTileY); }

static inline unsigned int stream_blocks(long long n, int per_thread = 1) {
    long long b = (n + (long long)kThreads * per_thread - 1) / ((long long)kThreads * per_thread);
    if (b < 1) b = 1;
    if (b > 8192) b = 8192;
    return (unsigned int)b;
}

hipError_t launch_init_state(DevState *st, hipStream_t s) {
    hipLaunchKernelGGL(init_state_kernel, dim3(1), dim3(256), 0, s, st, 0);
    return hipGetLastError();
}

hipError_t launch_reset_state(DevState *st, hipStream_t s) {
    hipLaunchKernelGGL(init_state_kernel, dim3(1), dim3(256), 0, s, st, 1);
    return hipGetLastError();
}

hipError_t launch_init_image(const void *src, int src_dtype, int B, int NB, float *dst, long long npx, DevState *st,
                             float fix, int want_gray, float gray_scale, hipStream_t s) {
    const dim3 grid(stream_blocks(npx, 4)), block(kThreads);
    switch (src_dtype) {
        case LSE_F32:
            hipLaunchKernelGGL(init_image_kernel<float>, grid, block, 0, s, static_cast<const float *>(src), B, NB,
                               dst, npx, st, fix, want_gray, gray_scale);
            break;
        case LSE_F16:
            hipLaunchKernelGGL(init_image_kernel<__half>, grid, block, 0, s, static_cast<const __half *>(src), B, NB,
                               dst, npx, st, fix, want_gray, gray_scale);
            break;
        case LSE_BF16:
            hipLaunchKernelGGL(init_image_kernel<__hip_bfloat16>, grid, block, 0, s,
                               static_cast<const __hip_bfloat16 *>(src), B, NB, dst, npx, st, fix, want_gray,
                               gray_scale);
            break;
        default:
            return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_pack_mask(const uint8_t *mask, uint32_t *bits, int H, int W, int WW, hipStream_t s) {
    const long long n = (long long)H * WW;
    hipLaunchKernelGGL(pack_mask_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, mask, bits, H, W, WW);
    return hipGetLastError();
}

size_t tile_smem_bytes(int r, int nch, int edge) { return tile_smem_words(r, nch, edge) * 4; }

hipError_t launch_stats_generic(const StepArgs &a, int NB, int raw, int slot, hipStream_t s) {
    const size_t sm = tile_smem_bytes(a.r, a.nch, 0);
    const dim3 grid = tile_grid(a.H, a.W);
    hipError_t e = hipSuccess;
    switch (NB) {
        case 1:
            if ((e = ensure_lds(stats_kernel<1>, sm)) != hipSuccess) return e;
            hipLaunchKernelGGL(stats_kernel<1>, grid, dim3(kThreads), sm, s, a, raw, slot);
            break;
        case 2:
            if ((e = ensure_lds(stats_kernel<2>, sm)) != hipSuccess) return e;
            hipLaunchKernelGGL(stats_kernel<2>, grid, dim3(kThreads), sm, s, a, raw, slot);
            break;
        case 4:
            if ((e = ensure_lds(stats_kernel<4>, sm)) != hipSuccess) return e;
            hipLaunchKernelGGL(stats_kernel<4>, grid, dim3(kThreads), sm, s, a, raw, slot);
            break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_edge_map(const float *gray, int H, int W, const Taps *taps, int r1, float *tmp, float *Is,
                           float *g, hipStream_t s) {
    const long long n = (long long)H * W;
    const dim3 grid((unsigned)((n + 255) / 256)), block(256);
    hipLaunchKernelGGL(hconv_f32_kernel, grid, block, 0, s, gray, tmp, H, W, taps, r1);
    hipLaunchKernelGGL(vconv_f32_kernel, grid, block, 0, s, tmp, Is, H, W, taps, r1);
    hipLaunchKernelGGL(edge_g_kernel, grid, block, 0, s, Is, g, H, W);
    return hipGetLastError();
}

hipError_t launch_mbox(const float *img, int H, int W, int NB, float *boxes, hipStream_t s) {
    const unsigned nblk = (unsigned)(((W + kMBX - 1) / kMBX) * ((H + kMBY - 1) / kMBY));
    switch (NB) {
        case 2: hipLaunchKernelGGL(mbox_kernel<2>, dim3(nblk), dim3(kThreads), 0, s, img, H, W, boxes); break;
        case 4: hipLaunchKernelGGL(mbox_kernel<4>, dim3(nblk), dim3(kThreads), 0, s, img, H, W, boxes); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_mpass(const StepArgs &a, int NB, hipStream_t s) {
    const long long nblk = (long long)((a.W + kMBX - 1) / kMBX) * ((a.H + kMBY - 1) / kMBY);
    const dim3 grid((unsigned)((nblk + kMBlocksPerWG - 1) / kMBlocksPerWG)), block(kThreads);
    switch (NB) {
        case 2: hipLaunchKernelGGL(mpass_kernel<2>, grid, block, 0, s, a); break;
        case 4: hipLaunchKernelGGL(mpass_kernel<4>, grid, block, 0, s, a); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <int R, int NB, bool EDGE>
static hipError_t launch_step_fast_t(const StepArgs &a, hipStream_t s) {
    const size_t sm = (size_t)FastGeom<R, EDGE>::smem_words * 4;
    const hipError_t e = ensure_lds(step_fast_kernel<R, NB, EDGE>, sm);
    if (e != hipSuccess) return e;
    // One workgroup per tile, rounded up to a multiple of 8 (one band of
    // tiles per XCD, see tile_of).
    const long long ntiles = (long long)((a.W + kFX - 1) / kFX) * ((a.H + kFY - 1) / kFY);
    const long long g = (ntiles + 7) & ~7ll;
    hipLaunchKernelGGL((step_fast_kernel<R, NB, EDGE>), dim3((unsigned)g), dim3(kThreads), sm, s, a);
    return hipGetLastError();
}

template <int R>
static hipError_t launch_step_fast_r(const StepArgs &a, int NB, int edge, hipStream_t s) {
    if (edge) return launch_step_fast_t<R, 1, true>(a, s);
    switch (NB) {
        case 1: return launch_step_fast_t<R, 1, false>(a, s);
        case 2: return launch_step_fast_t<R, 2, false>(a, s);
        case 4: return launch_step_fast_t<R, 4, false>(a, s);
    }
    return hipErrorInvalidValue;
}

template <int R, int NB>
static hipError_t launch_stats_fast_t(const StepArgs &a, int raw, int slot, hipStream_t s) {
    const size_t sm = (size_t)FastGeom<R, false>::UH * (kFWords + 2) * 4;
    const dim3 grid((a.W + kFX - 1) / kFX, (a.H + kFY - 1) / kFY);
    hipLaunchKernelGGL((stats_fast_kernel<R, NB>), grid, dim3(kThreads), sm, s, a, raw, slot);
    return hipGetLastError();
}

template <int R>
static hipError_t launch_stats_fast_r(const StepArgs &a, int NB, int raw, int slot, hipStream_t s) {
    switch (NB) {
        case 1: return launch_stats_fast_t<R, 1>(a, raw, slot, s);
        case 2: return launch_stats_fast_t<R, 2>(a, raw, slot, s);
        case 4: return launch_stats_fast_t<R, 4>(a, raw, slot, s);
    }
    return hipErrorInvalidValue;
}

static hipError_t launch_step_generic(const StepArgs &a, int NB, int edge, hipStream_t s) {
    const size_t sm = tile_smem_bytes(a.r, a.nch, edge);
    const dim3 grid = tile_grid(a.H, a.W), block(kThreads);
    hipError_t e = hipSuccess;
    if (edge) {
        if ((e = ensure_lds(step_kernel<1, true>, sm)) != hipSuccess) return e;
        hipLaunchKernelGGL((step_kernel<1, true>), grid, block, sm, s, a);
    } else {
        switch (NB) {
            case 1:
                if ((e = ensure_lds(step_kernel<1, false>, sm)) != hipSuccess) return e;
                hipLaunchKernelGGL((step_kernel<1, false>), grid, block, sm, s, a);
                break;
            case 2:
                if ((e = ensure_lds(step_kernel<2, false>, sm)) != hipSuccess) return e;
                hipLaunchKernelGGL((step_kernel<2, false>), grid, block, sm, s, a);
                break;
            case 4:
                if ((e = ensure_lds(step_kernel<4, false>, sm)) != hipSuccess) return e;
                hipLaunchKernelGGL((step_kernel<4, false>), grid, block, sm, s, a);
                break;
            default:
                return hipErrorInvalidValue;
        }
    }
    return hipGetLastError();
}

// The statistics kernel must use the same tiling as the step kernel that
// would have produced the statistics, so that resumed runs match bit for bit.
hipError_t launch_stats(const StepArgs &a, int NB, int raw, int slot, hipStream_t s) {
    switch (a.r) {
        case 3: return launch_stats_fast_r<3>(a, NB, raw, slot, s);
        case 4: return launch_stats_fast_r<4>(a, NB, raw, slot, s);
        case 5: return launch_stats_fast_r<5>(a, NB, raw, slot, s);
        case 6: return launch_stats_fast_r<6>(a, NB, raw, slot, s);
        case 7: return launch_stats_fast_r<7>(a, NB, raw, slot, s);
        default: break;
    }
    return launch_stats_generic(a, NB, raw, slot, s);
}

hipError_t launch_step(const StepArgs &a, int NB, int edge, hipStream_t s) {
    switch (a.r) {
        case 3: return launch_step_fast_r<3>(a, NB, edge, s);
        case 4: return launch_step_fast_r<4>(a, NB, edge, s);
        case 5: return launch_step_fast_r<5>(a, NB, edge, s);
        case 6: return launch_step_fast_r<6>(a, NB, edge, s);
        case 7: return launch_step_fast_r<7>(a, NB, edge, s);
        default: break;
    }
    return launch_step_generic(a, NB, edge, s);
}

hipError_t launch_mask_out(const uint32_t *const bits[2], const DevState *st, uint8_t *mask, int H, int W, int WW,
                           hipStream_t s) {
    const long long n = (long long)H * W;
    hipLaunchKernelGGL(mask_out_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, bits[0], bits[1], st,
                       mask, H, W, WW);
    return hipGetLastError();
}

hipError_t launch_count_needed(const StepArgs &a, int raw, int edge, hipStream_t s) {
    const int BPR = kTileY + 2 + 2 * a.r, BCR = kTileY + 2 * a.r;
    const size_t words = (size_t)a.nch * 64 + 36 + 32 + (size_t)(BPR + BCR) * kRowWords +
                         (size_t)BPR * (kTileX + 2) + (size_t)(kTileY + 2) * (kTileX + 2);
    const hipError_t e = ensure_lds(count_needed_kernel, words * 4);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(count_needed_kernel, tile_grid(a.H, a.W), dim3(kThreads), words * 4, s, a, raw, edge);
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
