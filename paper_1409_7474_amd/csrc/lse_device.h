// Device helpers shared by the HIP kernels of the fast level set evolution
// (arXiv 1409.7474): wave reductions, statistics totals, pixel loads of the
// three storage types, binary-window Gaussian sums and the tile geometry.
#pragma once

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

// Integer reductions over a whole wave without LDS traffic (the shuffles
// above are LDS permutes, which queue behind the phi pass's table lookups of
// other workgroups): a butterfly inside each row of 16 lanes by DPP moves
// (quad permutes for lane distances 1 and 2, row rotations by 4 and 8), after
// which every lane holds its row's result, then the four row results read
// into scalar registers.  Exact for any order; every lane of the wave must be
// active.  The result is the same in every lane.
template <int CTRL>
__device__ __forceinline__ uint32_t dpp_u32(uint32_t v) {
    return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, CTRL, 0xF, 0xF, false);
}
template <int CTRL>
__device__ __forceinline__ unsigned long long dpp_u64(unsigned long long v) {
    return ((unsigned long long)dpp_u32<CTRL>((uint32_t)(v >> 32)) << 32) | dpp_u32<CTRL>((uint32_t)v);
}
__device__ __forceinline__ unsigned long long lane_u64(unsigned long long v, int l) {
    return ((unsigned long long)(uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(v >> 32), l) << 32) |
           (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)v, l);
}
constexpr int kDppXor1 = 0xB1;   // quad_perm [1, 0, 3, 2]
constexpr int kDppXor2 = 0x4E;   // quad_perm [2, 3, 0, 1]
constexpr int kDppRor4 = 0x124;  // row_ror:4
constexpr int kDppRor8 = 0x128;  // row_ror:8

__device__ __forceinline__ long long wave_sum_ll_dpp(long long x) {
    unsigned long long v = (unsigned long long)x;
    v += dpp_u64<kDppXor1>(v);
    v += dpp_u64<kDppXor2>(v);
    v += dpp_u64<kDppRor4>(v);
    v += dpp_u64<kDppRor8>(v);
    return (long long)(lane_u64(v, 0) + lane_u64(v, 16) + lane_u64(v, 32) + lane_u64(v, 48));
}

__device__ __forceinline__ unsigned long long wave_max_u64_dpp(unsigned long long v) {
    auto mx = [](unsigned long long a, unsigned long long b) { return a > b ? a : b; };
    v = mx(v, dpp_u64<kDppXor1>(v));
    v = mx(v, dpp_u64<kDppXor2>(v));
    v = mx(v, dpp_u64<kDppRor4>(v));
    v = mx(v, dpp_u64<kDppRor8>(v));
    return mx(mx(lane_u64(v, 0), lane_u64(v, 16)), mx(lane_u64(v, 32), lane_u64(v, 48)));
}

__device__ __forceinline__ int wave_sum_i_dpp(int x) {
    uint32_t v = (uint32_t)x;
    v += dpp_u32<kDppXor1>(v);
    v += dpp_u32<kDppXor2>(v);
    v += dpp_u32<kDppRor4>(v);
    v += dpp_u32<kDppRor8>(v);
    return (int)((uint32_t)__builtin_amdgcn_readlane((int)v, 0) + (uint32_t)__builtin_amdgcn_readlane((int)v, 16) +
                 (uint32_t)__builtin_amdgcn_readlane((int)v, 32) + (uint32_t)__builtin_amdgcn_readlane((int)v, 48));
}

// FP32 sum in a fixed order: the row butterfly above (every lane of a row
// then holds its row's sum, lane 0 in the order ((l0 + l1) + (l2 + l3)) + ...),
// then the rows as (r0 + r1) + (r2 + r3) from lanes 0, 16, 32 and 48.
__device__ __forceinline__ float wave_sum_f_dpp(float x) {
    x += __uint_as_float(dpp_u32<kDppXor1>(__float_as_uint(x)));
    x += __uint_as_float(dpp_u32<kDppXor2>(__float_as_uint(x)));
    x += __uint_as_float(dpp_u32<kDppRor4>(__float_as_uint(x)));
    x += __uint_as_float(dpp_u32<kDppRor8>(__float_as_uint(x)));
    const float r0 = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x), 0));
    const float r1 = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x), 16));
    const float r2 = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x), 32));
    const float r3 = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x), 48));
    return (r0 + r1) + (r2 + r3);
}

template <bool MAX>
__device__ __forceinline__ unsigned int wave_ext_u_dpp(unsigned int v) {
    auto ex = [](unsigned int a, unsigned int b) { return MAX ? max(a, b) : min(a, b); };
    v = ex(v, dpp_u32<kDppXor1>(v));
    v = ex(v, dpp_u32<kDppXor2>(v));
    v = ex(v, dpp_u32<kDppRor4>(v));
    v = ex(v, dpp_u32<kDppRor8>(v));
    return ex(ex((unsigned int)__builtin_amdgcn_readlane((int)v, 0), (unsigned int)__builtin_amdgcn_readlane((int)v, 16)),
              ex((unsigned int)__builtin_amdgcn_readlane((int)v, 32), (unsigned int)__builtin_amdgcn_readlane((int)v, 48)));
}

__device__ __forceinline__ int block_linear_id() { return blockIdx.y * gridDim.x + blockIdx.x; }


// Totals of one statistics slot and of the image lines, reduced over the
// kBins accumulation lines: wave 0 takes the slot (line i in lane i), wave 1
// the image lines.  Called by every thread of the workgroup.
// Index of this thread's wave in the workgroup, as a wave-uniform (scalar)
// value: every lane of a wave64 has the same threadIdx.x >> 6, and saying so
// lets per-wave row and segment arithmetic run on the scalar unit.
__device__ __forceinline__ int wave_id() { return __builtin_amdgcn_readfirstlane((int)threadIdx.x >> 6); }

struct Totals {
    long long sum[4];
    unsigned long long nplus, flips, mkey;
    int done, bad, raw;
    long long total[4];
    unsigned int imin_key[4], imax_key[4];
};

// The statistics lines of one slot, in two halves so that a caller can put
// other loads in flight between them: totals_issue loads this wave's lines
// into registers (wave 0: the statistics bins, lane i = bin i; wave 1: the
// image bins; wave 2: the flags), totals_commit reduces them and writes
// `t` (the caller then synchronises the workgroup).
struct TotalsRegs {
    long long v[4], np, fl;
    unsigned long long mk;
    unsigned int lo[4], hi[4];
    int done, bad, raw;
};

__device__ __forceinline__ void totals_issue(const DevState *st, int sl, bool want_img, TotalsRegs &r,
                                             bool split = false, bool want_sums = true, bool want_keys = true) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (split) {
        // Four waves share the reductions: 0 the sums, 1 the band totals,
        // 2 count, flips, maximum key and flags, 3 the band minimum and
        // maximum keys (only the wanted ones are loaded).
        const Bin &b = st->slot[sl][lane];
        const ImgBin &ib = st->img[lane];
        if (wave == 0) {
            if (want_sums) {
#pragma unroll
                for (int k = 0; k < 4; ++k) r.v[k] = b.sum[k];
            }
        } else if (wave == 1) {
            if (want_img) {
#pragma unroll
                for (int k = 0; k < 4; ++k) r.v[k] = ib.total[k];
            }
        } else if (wave == 2) {
            r.fl = (long long)b.flips;
            if (want_sums) {
                r.np = (long long)b.nplus;
                r.mk = b.mkey;
            }
            if (lane == 0) {
                r.done = st->done;
                r.bad = st->bad;
                r.raw = st->raw;
            }
        } else if (want_img && want_keys) {
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                r.lo[k] = ib.imin_key[k];
                r.hi[k] = ib.imax_key[k];
            }
        }
        return;
    }
    if (wave == 0) {
        const Bin &b = st->slot[sl][lane];
#pragma unroll
        for (int k = 0; k < 4; ++k) r.v[k] = b.sum[k];
        r.np = (long long)b.nplus;
        r.fl = (long long)b.flips;
        r.mk = b.mkey;
    } else if (wave == 2) {
        if (lane == 0) {
            r.done = st->done;
            r.bad = st->bad;
            r.raw = st->raw;
        }
    } else if (wave == 1 && want_img) {
        const ImgBin &b = st->img[lane];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            r.v[k] = b.total[k];
            r.lo[k] = b.imin_key[k];
            r.hi[k] = b.imax_key[k];
        }
    }
}

// Reduce what totals_issue loaded and write `t` (the caller then synchronises
// the workgroup).  With `split` (four waves), the fields a caller did not
// want are written as zeros.
__device__ __forceinline__ void totals_commit(bool want_img, TotalsRegs &r, Totals *t, bool split = false,
                                              bool want_sums = true, bool want_keys = true) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (split) {
        if (wave == 0) {
#pragma unroll
            for (int k = 0; k < 4; ++k) r.v[k] = want_sums ? wave_sum_ll_dpp(r.v[k]) : 0;
            if (lane == 0) {
#pragma unroll
                for (int k = 0; k < 4; ++k) t->sum[k] = r.v[k];
            }
        } else if (wave == 1) {
#pragma unroll
            for (int k = 0; k < 4; ++k) r.v[k] = want_img ? wave_sum_ll_dpp(r.v[k]) : 0;
            if (lane == 0) {
#pragma unroll
                for (int k = 0; k < 4; ++k) t->total[k] = r.v[k];
            }
        } else if (wave == 2) {
            r.fl = wave_sum_ll_dpp(r.fl);
            r.np = want_sums ? wave_sum_ll_dpp(r.np) : 0;
            r.mk = want_sums ? wave_max_u64_dpp(r.mk) : 0ull;
            if (lane == 0) {
                t->nplus = (unsigned long long)r.np;
                t->flips = (unsigned long long)r.fl;
                t->mkey = r.mk;
                t->done = r.done;
                t->bad = r.bad;
                t->raw = r.raw;
            }
        } else {
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                r.lo[k] = want_img && want_keys ? wave_ext_u_dpp<false>(r.lo[k]) : 0u;
                r.hi[k] = want_img && want_keys ? wave_ext_u_dpp<true>(r.hi[k]) : 0u;
            }
            if (lane == 0) {
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    t->imin_key[k] = r.lo[k];
                    t->imax_key[k] = r.hi[k];
                }
            }
        }
        return;
    }
    if (wave == 0) {
#pragma unroll
        for (int k = 0; k < 4; ++k) r.v[k] = wave_sum_ll_dpp(r.v[k]);
        r.np = wave_sum_ll_dpp(r.np);
        r.fl = wave_sum_ll_dpp(r.fl);
        r.mk = wave_max_u64_dpp(r.mk);
        if (lane == 0) {
#pragma unroll
            for (int k = 0; k < 4; ++k) t->sum[k] = r.v[k];
            t->nplus = (unsigned long long)r.np;
            t->flips = (unsigned long long)r.fl;
            t->mkey = r.mk;
        }
    } else if (wave == 2) {
        if (lane == 0) {
            t->done = r.done;
            t->bad = r.bad;
            t->raw = r.raw;
        }
    } else if (wave == 1 && want_img) {
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            r.v[k] = wave_sum_ll_dpp(r.v[k]);
            r.lo[k] = wave_ext_u_dpp<false>(r.lo[k]);
            r.hi[k] = wave_ext_u_dpp<true>(r.hi[k]);
        }
        if (lane == 0) {
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                t->total[k] = r.v[k];
                t->imin_key[k] = r.lo[k];
                t->imax_key[k] = r.hi[k];
            }
        }
    }
}

__device__ __forceinline__ void load_totals(const DevState *st, int sl, bool want_img, Totals *t) {
    TotalsRegs r;
    totals_issue(st, sl, want_img, r);
    totals_commit(want_img, r, t);
    __syncthreads();
}

template <int NB>
struct Px {
    float v[NB];
};

// Element types of the resident image: FP32, or 16-bit FP16 / BF16 halves of
// a 32-bit word (low half = lower address).
template <typename ST>
__device__ __forceinline__ float half_lo(uint32_t w);
template <typename ST>
__device__ __forceinline__ float half_hi(uint32_t w);
template <>
__device__ __forceinline__ float half_lo<__half>(uint32_t w) {
    return (float)__builtin_bit_cast(_Float16, (unsigned short)(w & 0xffffu));
}
template <>
__device__ __forceinline__ float half_hi<__half>(uint32_t w) {
    return (float)__builtin_bit_cast(_Float16, (unsigned short)(w >> 16));
}
template <>
__device__ __forceinline__ float half_lo<__hip_bfloat16>(uint32_t w) { return __uint_as_float(w << 16); }
template <>
__device__ __forceinline__ float half_hi<__hip_bfloat16>(uint32_t w) { return __uint_as_float(w & 0xffff0000u); }

template <typename ST>
__device__ __forceinline__ float to_f32(ST v);
template <>
__device__ __forceinline__ float to_f32<float>(float v) { return v; }
template <>
__device__ __forceinline__ float to_f32<__half>(__half v) { return __half2float(v); }
template <>
__device__ __forceinline__ float to_f32<__hip_bfloat16>(__hip_bfloat16 v) { return __bfloat162float(v); }

// Round to the storage type (to nearest, ties to even).
template <typename ST>
__device__ __forceinline__ ST from_f32(float v);
template <>
__device__ __forceinline__ float from_f32<float>(float v) { return v; }
template <>
__device__ __forceinline__ __half from_f32<__half>(float v) { return __float2half_rn(v); }
template <>
__device__ __forceinline__ __hip_bfloat16 from_f32<__hip_bfloat16>(float v) { return __float2bfloat16(v); }

// Pixel `pix` of an image with NB interleaved bands of type ST.
template <typename ST, int NB>
__device__ __forceinline__ Px<NB> load_px(const ST *__restrict__ img, long long pix) {
    Px<NB> p;
    if constexpr (sizeof(ST) == 4) {
        const float *f = reinterpret_cast<const float *>(img) + pix * NB;
        if constexpr (NB == 4) {
            const float4 v = *reinterpret_cast<const float4 *>(f);
            p.v[0] = v.x;
            p.v[1] = v.y;
            p.v[2] = v.z;
            p.v[3] = v.w;
        } else if constexpr (NB == 2) {
            const float2 v = *reinterpret_cast<const float2 *>(f);
            p.v[0] = v.x;
            p.v[1] = v.y;
        } else {
            p.v[0] = f[0];
        }
    } else {
        const unsigned short *h = reinterpret_cast<const unsigned short *>(img) + pix * NB;
        if constexpr (NB == 4) {
            const uint2 v = *reinterpret_cast<const uint2 *>(h);
            p.v[0] = half_lo<ST>(v.x);
            p.v[1] = half_hi<ST>(v.x);
            p.v[2] = half_lo<ST>(v.y);
            p.v[3] = half_hi<ST>(v.y);
        } else if constexpr (NB == 2) {
            const uint32_t v = *reinterpret_cast<const uint32_t *>(h);
            p.v[0] = half_lo<ST>(v);
            p.v[1] = half_hi<ST>(v);
        } else {
            p.v[0] = half_lo<ST>((uint32_t)h[0]);
        }
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

// One pixel (NB values of type ST) at byte offset byte_off.
template <typename ST, int NB>
__device__ __forceinline__ Px<NB> buffer_px(__amdgpu_buffer_rsrc_t r, uint32_t byte_off) {
    Px<NB> p;
    if constexpr (sizeof(ST) == 4) {
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
    } else {
        if constexpr (NB == 4) {
            const auto v = __builtin_amdgcn_raw_buffer_load_b64(r, byte_off, 0, 0);
            p.v[0] = half_lo<ST>((uint32_t)v[0]);
            p.v[1] = half_hi<ST>((uint32_t)v[0]);
            p.v[2] = half_lo<ST>((uint32_t)v[1]);
            p.v[3] = half_hi<ST>((uint32_t)v[1]);
        } else if constexpr (NB == 2) {
            const uint32_t v = (uint32_t)__builtin_amdgcn_raw_buffer_load_b32(r, byte_off, 0, 0);
            p.v[0] = half_lo<ST>(v);
            p.v[1] = half_hi<ST>(v);
        } else {
            p.v[0] = half_lo<ST>((uint32_t)__builtin_amdgcn_raw_buffer_load_b16(r, byte_off, 0, 0));
        }
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
template <int NB, typename ST>
__device__ __forceinline__ void stats_tile(const TileSmem &s, const ST *__restrict__ img, int x0, int y0,
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
                const Px<NB> p = load_px<ST, NB>(img, (long long)y * W + x);
#pragma unroll
                for (int b = 0; b < NB; ++b) acc[b] += p.v[b];
                ++cnt;
            }
        }
    }
}

// Workgroup reduction of (NB sums, count, flips): the totals are valid in
// thread 0.  FP32 sums in a fixed order (wave_sum_f_dpp, then waves in
// order), so a tile's partial sums are a function of its data alone.
template <int NB>
__device__ __forceinline__ void block_reduce(const TileSmem &s, float (&acc)[NB], int cnt, int flips, bool with_sums,
                                             float (&S)[NB], int &C, int &F) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (with_sums) {
#pragma unroll
        for (int b = 0; b < NB; ++b) acc[b] = wave_sum_f_dpp(acc[b]);
        cnt = wave_sum_i_dpp(cnt);
    }
    flips = wave_sum_i_dpp(flips);
    if (lane == 0) {
        float *rw = s.red + wave * 8;
#pragma unroll
        for (int b = 0; b < NB; ++b) rw[b] = acc[b];
        reinterpret_cast<int *>(rw)[6] = cnt;
        reinterpret_cast<int *>(rw)[7] = flips;
    }
    __syncthreads();
    C = 0;
    F = 0;
#pragma unroll
    for (int b = 0; b < NB; ++b) S[b] = 0.f;
    if (threadIdx.x == 0) {
        for (int w = 0; w < kThreads / 64; ++w) {
            const float *rw = s.red + w * 8;
#pragma unroll
            for (int b = 0; b < NB; ++b) S[b] += rw[b];
            C += reinterpret_cast<const int *>(rw)[6];
            F += reinterpret_cast<const int *>(rw)[7];
        }
    }
}

// One thread: commit a tile's fixed-point region sums `cur` and count as the
// change from its previous record `prev` (null: nothing recorded, commit the
// values), and record them in `rec` (if not null).  Integer arithmetic
// modulo 2^64, so the totals stay exactly the sum of each tile's latest
// contribution and tiles that are not revisited keep theirs.
template <int NB>
__device__ __forceinline__ void commit_tile(const long long (&cur)[NB], long long cnt, const TileSum *prev,
                                            TileSum *rec, Bin *out) {
#pragma unroll
    for (int b = 0; b < NB; ++b) {
        const long long d = prev ? cur[b] - prev->sum[b] : cur[b];
        if (d) atomicAdd(reinterpret_cast<unsigned long long *>(&out->sum[b]), (unsigned long long)d);
    }
    const long long dc = prev ? cnt - prev->cnt : cnt;
    if (dc) atomicAdd(&out->nplus, (unsigned long long)dc);
    if (rec) {
#pragma unroll
        for (int b = 0; b < NB; ++b) rec->sum[b] = cur[b];
        rec->cnt = cnt;
    }
}

// Workgroup reduction of (NB sums, count, flips) and one atomic per value
// (sums: as the change from `prev` when given, recorded in `rec`).
template <int NB>
__device__ __forceinline__ void reduce_commit(const TileSmem &s, float (&acc)[NB], int cnt, int flips, Bin *out,
                                             float fix, bool with_sums, const TileSum *prev = nullptr,
                                             TileSum *rec = nullptr) {
    float S[NB];
    int C, F;
    block_reduce<NB>(s, acc, cnt, flips, with_sums, S, C, F);
    if (threadIdx.x == 0) {
        if (with_sums) {
            long long v[NB];
#pragma unroll
            for (int b = 0; b < NB; ++b) v[b] = __float2ll_rn(S[b] * fix);
            commit_tile<NB>(v, (long long)C, prev, rec, out);
        }
        if (F) atomicAdd(&out->flips, (unsigned long long)F);
    }
}


constexpr int kMBX = 64, kMBY = 32, kMBlocksPerWG = 64;  // one block per lane of wave 0

// One thread of a step's lead workgroup: the image values of the pixel that
// maximised |D| for this iteration (key `mkey`, from its statistics slot
// `sl`), kept in that slot's spare words for the next normaliser pass, whose
// lower bound they give without a dependent load.  The slot is cleared only
// by the step after that pass.
template <int NB, typename ST>
__device__ __forceinline__ void record_max_pixel(DevState *st, int sl, unsigned long long mkey, const void *img,
                                                 long long hw) {
    const unsigned int pix = 0xffffffffu - (unsigned int)(mkey & 0xffffffffu);
    if (mkey == 0ull || (long long)pix >= hw) return;
    const Px<NB> v = load_px<ST, NB>(static_cast<const ST *>(img), pix);
    Bin &b0 = st->slot[sl][0];
    float *pf = reinterpret_cast<float *>(&b0.pad[0]);
#pragma unroll
    for (int b = 0; b < NB; ++b) pf[b] = v.v[b];
    b0.pad[2] = (unsigned long long)pix + 1ull;
}

__device__ __forceinline__ unsigned long long mkey_of(float absd, unsigned int pix) {
    return ((unsigned long long)__float_as_uint(absd) << 32) | (unsigned long long)(0xffffffffu - pix);
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
constexpr int kFYRegion = 48;  // owned rows, region term (the front tiles are the critical path)
constexpr int kFYEdge = 64;    // owned rows, edge term
constexpr int kFWords = 6;     // staged bit words per row: global words x0/32 - 1 .. x0/32 + 4

constexpr int kSB = 8;         // rows per block of the rolling vertical window
constexpr int kCG = 4;         // rows per group of data-term loads in the binarisation phase

// Variants of the step kernel, picked per kernel family and image size by
// the autotuner (lse_autotune): the tile's owned rows and the waves per SIMD
// the kernel is compiled for (its register budget).  Every variant gives the
// same values bit for bit: the edge step's results are per pixel, and the
// region variants keep the 48-row tiling, which fixes the order of the FP32
// statistics sums within a tile.
constexpr int kStepVariants = 3;
template <bool EDGE, int V>
struct StepVariant {
    // edge: 64, 48 or 80 rows at 4 waves per SIMD; region: 48 rows at 4, 3 or 5.
    static constexpr int FY = EDGE ? (V == 0 ? kFYEdge : V == 1 ? 48 : 80) : kFYRegion;
    static constexpr int OCC = EDGE ? 4 : (V == 0 ? 4 : V == 1 ? 3 : 5);
};

template <int R, bool EDGE, int FYV = (EDGE ? kFYEdge : kFYRegion)>
struct FastGeom {
    static constexpr int TS = 2 * R + 1;
    static constexpr int RU = EDGE ? 0 : R;      // halo of the binarised field
    static constexpr int FY = FYV;               // owned rows
    static constexpr int UH = FY + 2 * RU;       // rows where b^n is computed
    static constexpr int PH = UH + 2;            // rows of phi^n
    static constexpr int PW = kFX + 2 * RU + 2;  // columns of phi^n (<= 128)
    // Rows per block of the phi pass's rolling window: kSB in the region
    // term (its PH = 2 (mod 16) wastes 2 rows); in the edge term the block
    // height that splits PH into two segments of at most 11-row blocks with
    // the fewest rows past PH (66 rows: 2 x 3 x 11, none).
    static constexpr int NBLK = EDGE ? (PH + 21) / 22 : (PH + 2 * kSB - 1) / (2 * kSB);  // window blocks per segment
    static constexpr int KB = EDGE ? (PH + 2 * NBLK - 1) / (2 * NBLK) : kSB;
    static constexpr int SEG = NBLK * KB;        // phi rows per wave (2 segments x 2 chunks)
    static constexpr int PHP = 2 * SEG;          // phi rows allocated (>= PH)
    static constexpr int BH = PHP + 2 * R;       // staged rows of b^{n-1}
    static constexpr int SEGD = FY / 2;          // statistics rows per wave
    static constexpr int NCH = (TS + 5) / 6;     // lookup chunks
    static constexpr int PS = PW;                // phi row stride (floats)
    // phi is stored for its PH rows only (the segment loop computes up to
    // PHP rows; the extra ones are not kept), which keeps the step kernel
    // within a quarter of the CU's LDS for the common radii.
    static constexpr int smem_words = BH * kFWords + PH * PS + UH * kFWords + BH * 2 + PHP * 2 + 16;
    // A quiet tile writes its owned words with one thread each.
    static_assert(FY * 3 <= kThreads, "owned bit words of a tile exceed the workgroup");
};

// Whether the staged bits lo .. hi of a fast tile (bit 0 = column x0 - 32)
// reach outside the image: only then do taps over them need the
// zero-padding correction, and only otherwise may a uniform window take the
// constant interior value.
__device__ __forceinline__ bool span_outside(int x0, int W, int lo, int hi) {
    return x0 - 32 + lo < 0 || x0 - 32 + hi > W - 1;
}

// The horizontal-sum tables in registers: chunk c in v[c] (lane m holds the
// sum for bit pattern m), and the last chunk's entries for patterns 0 and 1
// (scalar), which a one-bit last chunk selects between instead of a permute.
template <int NCH>
struct LutRegs {
    int v[NCH];
    float t0, t1;
};

template <int NCH>
__device__ __forceinline__ void load_luts(const Taps *__restrict__ taps, LutRegs<NCH> &lut) {
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int c = 0; c < NCH; ++c) lut.v[c] = __float_as_int(taps->lut[c][lane]);
    lut.t0 = taps->lut[NCH - 1][0];
    lut.t1 = taps->lut[NCH - 1][1];
}

// Zero padding of the horizontal taps at image column x (only where the
// taps reach outside the image, `border`): the window bits outside the image
// are set, as if they were inside, and their weight is subtracted.  It depends
// on the column alone, so a caller computes it once for its lane.
struct HPad {
    uint32_t orm;  // window bits forced to one
    float corr;    // weight of those bits
};

template <int R>
__device__ __forceinline__ HPad hpad_of(int x, int W, bool border, const float *__restrict__ cum) {
    constexpr int TS = 2 * R + 1;
    constexpr uint32_t FULL = (1u << TS) - 1u;
    HPad p{0u, 0.f};
    if (border) {
        const int left = min(R - x, TS);
        const int right = min(x + R - (W - 1), TS);
        if (left > 0) {
            p.orm |= (1u << left) - 1u;
            p.corr = cum[left];
        }
        if (right > 0) {
            p.orm |= FULL & ~((1u << (TS - right)) - 1u);
            p.corr += cum[right];
        }
    }
    return p;
}

// Horizontal Gaussian of a binary row, as hconv_bits; must be called with all
// 64 lanes active (ds_bpermute).  `pad` is the lane's zero-padding correction
// (hpad_of; all zero away from the left and right image edges).
template <int R, int NCH>
__device__ __forceinline__ float hconv_fast(const uint32_t *row, int xb, HPad pad, const LutRegs<NCH> &lut) {
    constexpr int TS = 2 * R + 1;
    constexpr uint32_t FULL = (1u << TS) - 1u;
    const int ws = xb - R;
    const int wi = ws >> 5;
    const uint32_t win =
        (__builtin_amdgcn_alignbit(row[wi + 1], row[wi], (uint32_t)(ws & 31)) & FULL) | pad.orm;
    float h = 0.f;
#pragma unroll
    for (int c = 0; c < NCH; ++c) {
        const int idx = (int)((win >> (6 * c)) & 63u);
        if (c == NCH - 1 && TS - 6 * c == 1)
            h += (idx & 1) ? lut.t1 : lut.t0;  // the same table entry, by a select
        else
            h += __int_as_float(__builtin_amdgcn_ds_bpermute(idx << 2, lut.v[c]));
    }
    return h - pad.corr;
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

// Stage NROWS rows of kFWords bit words (global words x0/32 - 1 .. x0/32 + 4;
// the last one is padding) starting at image row row0 into LDS; words
// outside the image are zero.  Buffer loads (zero outside their range) keep
// the loads branch-free: every load of a thread is in flight before its
// first LDS store.
template <int NROWS>
__device__ __forceinline__ void stage_bits_fast(uint32_t *dst, const uint32_t *__restrict__ bits, int row0, int x0,
                                                int H, int WW) {
    constexpr int N = NROWS * kFWords;
    constexpr int NIT = (N + kThreads - 1) / kThreads;
    const __amdgpu_buffer_rsrc_t rs = image_rsrc(bits, (uint32_t)((long long)H * WW * 4));
    const int wb0 = (x0 >> 5) - 1;
    uint32_t v[NIT];
#pragma unroll
    for (int k = 0; k < NIT; ++k) {
        const int i = (int)threadIdx.x + k * kThreads;
        const int row = i / kFWords, wc = i - row * kFWords;
        const int y = row0 + row, gw = wb0 + wc;
        const bool ok = i < N && wc < kFWords - 1 && y >= 0 && y < H && gw >= 0 && gw < WW;
        v[k] = (uint32_t)__builtin_amdgcn_raw_buffer_load_b32(rs, ok ? (uint32_t)(y * WW + gw) * 4u : kNoLoad, 0, 0);
    }
#pragma unroll
    for (int k = 0; k < NIT; ++k) {
        const int i = (int)threadIdx.x + k * kThreads;
        if (i < N) dst[i] = v[k];
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

// Statistics of phi^{n+1} = G * b on the owned 96 x FY tile (b in `bn`, rows
// y0 - R .. y0 + FY + R, bit 0 of each row = column x0 - 32).  raw: phi = b.
// Every owned pixel of the image is read once (dense streaming); blocks of
// 8 rows whose whole bit window is uniform take the sign without the
// Gaussian sums (their value would be the same constant in every pixel).
// GR: image rows per load group (two groups in flight); the sums do not
// depend on it (each lane adds its rows in order).
template <int R, int NB, typename ST, int GR = 4>
__device__ __forceinline__ void stats_fast(const uint32_t *bn, const int *codes, const ST *__restrict__ img,
                                           int x0, int y0, int H, int W, bool border, bool raw,
                                           const LutRegs<FastGeom<R, false>::NCH> &lut, const float (&kk)[2 * R + 1],
                                           const float *__restrict__ cum, float (&acc)[NB], int &cnt) {
    using G = FastGeom<R, false>;
    static_assert(G::SEGD % kSB == 0, "statistics segment must be a whole number of blocks");
    static_assert(kFX == 96 && kThreads == 256, "three waves cover the owned columns by row segments");
    const int tid = (int)threadIdx.x;
    const int lane = tid & 63, wave = wave_id();
#pragma unroll
    for (int b = 0; b < NB; ++b) acc[b] = 0.f;
    cnt = 0;
    // Waves 0 and 2: columns 0..63, rows of segment 0 / 1.  Wave 1: columns
    // 64..95, lanes 0..31 on segment 0 and lanes 32..63 on segment 1 (so no
    // lane idles).  Wave 3 has no statistics work.
    if (wave == 3) return;
    const int chunk = wave & 1;
    const int seg = chunk ? (lane >> 5) : (wave >> 1);
    const int ox = chunk ? 64 + (lane & 31) : lane;
    const int x = x0 + ox;
    const bool colok = x < W;
    // The window of this chunk's columns (bits of code_rows_owned) reaches
    // outside the image only next to the left or right edge.
    border = border && span_outside(x0, W, chunk == 0 ? 32 - R : 96 - R, chunk == 0 ? 96 + R : 128 + R);
    const int urow0 = seg * G::SEGD;  // U row of output row 0 of this lane's segment window
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
            // Uniform block: every pixel has the sign of the constant.  Only
            // the sign is needed, so this holds at the image edges too: bits
            // outside the image are zero, so an all-ones window lies inside
            // the image, and an all-zeros one gives minus a positive sum.
            // Wave 1 holds blocks of both segments: it skips only when both
            // are uniform (a computed uniform window gives the same sign).
            int uni;
            if (chunk) {
                const int u0 = block_code(codes, blk * kSB, kSB + 2 * R, 1);
                const int u1 = block_code(codes, G::SEGD + blk * kSB, kSB + 2 * R, 1);
                uni = (u0 >= 0 && u1 >= 0) ? (seg ? u1 : u0) : -1;
            } else {
                uni = block_code(codes, rb, kSB + 2 * R, 0);
            }
            if (uni >= 0) {
                if (uni == 1) inmask |= ((1u << kSB) - 1u) << (blk * kSB);
                have_win = false;
                continue;
            }
            // The padding is taken per row here: kept for the whole loop it
            // makes the R >= 6 step kernels spill.
            if (!have_win) {
#pragma unroll
                for (int t = 0; t < 2 * R; ++t) {
                    const int y = yb + t;
                    const float v =
                        hconv_fast<R, G::NCH>(bn + (rb + t) * kFWords, ox + 32, hpad_of<R>(x, W, border, cum), lut);
                    win[t] = (y >= 0 && y < H) ? v : 0.f;
                }
            }
#pragma unroll
            for (int t = 0; t < kSB; ++t) {
                const int urow = rb + 2 * R + t;
                const int y = y0 - R + urow;
                const float v =
                    hconv_fast<R, G::NCH>(bn + urow * kFWords, ox + 32, hpad_of<R>(x, W, border, cum), lut);
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
    constexpr int PB = NB * (int)sizeof(ST);  // bytes per pixel
    const __amdgpu_buffer_rsrc_t rs = image_rsrc(img, (uint32_t)((unsigned long long)H * W * PB));
    const uint32_t off0 = (uint32_t)(((y0 + urow0) * W + x) * PB);
    const uint32_t rstride = (uint32_t)(W * PB);
    static_assert(G::SEGD % (2 * GR) == 0, "load groups come in pairs");
    Px<NB> ba[GR], bb[GR];
    auto load_group = [&](Px<NB>(&buf)[GR], int g) {
#pragma unroll
        for (int i = 0; i < GR; ++i) {
            const int j = g * GR + i;
            buf[i] = buffer_px<ST, NB>(rs, ((inmask >> j) & 1u) ? off0 + j * rstride : kNoLoad);
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

// A record of heavy tiles: nw words, bit t % 32 of word t / 32 for tile t.
struct Record {
    const uint32_t *w;
    int nw;
};

// Word w of a record, or zero outside it.  The load address is clamped into
// the record, so every load stays in range whatever the compiler does with
// neighbouring loads (it may merge them), and the value is masked after.
__device__ __forceinline__ uint32_t record_word(Record rec, int w) {
    const int wc = min(max(w, 0), rec.nw - 1);
    const uint32_t v = rec.w[wc];
    return w == wc ? v : 0u;
}

// The schedule keeps three records of heavy tiles (iteration slots n % 3,
// nw words each), then, from word sched_tag_offset(nw) (16-byte aligned),
// one tag byte per tile (8 nw words): a tile is touched
// for step n + 1 when its byte holds touch_tag(n), written by a neighbour
// that flipped pixels inside its bit window in step n.  A byte left from an
// iteration 128 k earlier can match again; that only adds a visit.
__device__ __forceinline__ Record heavy_record(const uint32_t *sched, int nw, int slot) {
    return Record{sched + (size_t)slot * nw, nw};
}
__device__ __forceinline__ uint32_t touch_tag(int n) { return 0x80u | ((uint32_t)n & 0x7Fu); }

// Touched tiles of record word w (tiles 32 w .. 32 w + 31) for step n + 1
// (tag = touch_tag(n)); w is clamped into the record (callers mask the result).
__device__ __forceinline__ uint32_t touched_word(const uint32_t *sched, int nw, int w, uint32_t tag) {
    const uint4 *p = reinterpret_cast<const uint4 *>(sched + sched_tag_offset(nw)) + 2 * min(max(w, 0), nw - 1);
    const uint4 q0 = p[0], q1 = p[1];
    const uint32_t v[8] = {q0.x, q0.y, q0.z, q0.w, q1.x, q1.y, q1.z, q1.w};
    uint32_t m = 0u;
#pragma unroll
    for (int i = 0; i < 8; ++i)
#pragma unroll
        for (int b = 0; b < 4; ++b) m |= (((v[i] >> (8 * b)) & 0xFFu) == tag ? 1u : 0u) << (4 * i + b);
    return m;
}

// Neighbours whose bit windows reach the flipped bits f of owned word j
// (0..2, 32 columns each) of tile row ry, for a window halo of HWB pixels on
// every side: bit 0 left, 1 right, 2 up, 3 down, 4 up-left, 5 up-right,
// 6 down-left, 7 down-right.
template <int FY, int HWB>
__device__ __forceinline__ int flip_dirs(int ry, int j, uint32_t f) {
    static_assert(HWB < 32 && HWB <= FY, "window halo exceeds a bit word or a tile");
    // Branch-free: every term is 0 when f is.
    const bool any = f != 0u;
    const bool up = any && ry < HWB, dn = any && ry >= FY - HWB;
    const bool lf = j == 0 && (f & ((1u << HWB) - 1u)) != 0u;
    const bool rt = j == 2 && (f >> (32 - HWB)) != 0u;
    return (lf ? 1 : 0) | (rt ? 2 : 0) | (up ? 4 : 0) | (dn ? 8 : 0) | (lf && up ? 16 : 0) | (rt && up ? 32 : 0) |
           (lf && dn ? 64 : 0) | (rt && dn ? 128 : 0);
}

// Tag the neighbours of tile t (grid ntx x nty) named by dirs as touched
// (plain byte stores: no atomics, each byte is one tile's).
__device__ __forceinline__ void mark_touched(uint32_t *sched, int nw, int t, int ntx, int nty, int dirs, uint32_t tag) {
    uint8_t *tags = reinterpret_cast<uint8_t *>(sched + sched_tag_offset(nw));
    const int tx = t % ntx, ty = t / ntx;
#pragma unroll
    for (int d = 0; d < 8; ++d) {
        if (!((dirs >> d) & 1)) continue;
        const int x = tx + (d == 0 || d == 4 || d == 6 ? -1 : (d == 1 || d == 5 || d == 7 ? 1 : 0));
        const int y = ty + (d == 2 || d == 4 || d == 5 ? -1 : (d == 3 || d == 6 || d == 7 ? 1 : 0));
        if (x < 0 || x >= ntx || y < 0 || y >= nty) continue;
        tags[y * ntx + x] = (uint8_t)tag;
    }
}

// Tile of workgroup j of a single-image launch without a visit list,
// computed by one wave from the previous iteration's records (the order of
// build_plan: heavy tiles, then the other touched tiles).  Returns -1 for
// j >= the number of active tiles.  Every workgroup scans the whole records,
// so this serves small tile counts only (ntiles <= kPlanMinTiles: two
// record words per lane, kept in registers).
__device__ __forceinline__ int active_first_tile(const uint32_t *__restrict__ sched, int n, int ntiles, int j) {
    const int lane = (int)threadIdx.x & 63;
    if (j >= ntiles) return -1;
    constexpr int kPer = kPlanMinTiles / 32 / 64;  // words per lane (the caller keeps ntiles <= kPlanMinTiles)
    const int nw = (ntiles + 31) >> 5;
    const int w0 = lane * kPer;
    uint32_t hw[kPer], aw[kPer];                     // this lane's heavy and other active tiles
    const Record hr = heavy_record(sched, nw, n % 3);
    const uint32_t tag = touch_tag(n - 1);
    int nh = 0, na = 0;
#pragma unroll
    for (int i = 0; i < kPer; ++i) {
        const int w = w0 + i;
        const int valid = max(0, min(32, ntiles - 32 * w));  // 0 past the record
        const uint32_t vm = valid >= 32 ? ~0u : ((1u << valid) - 1u);
        hw[i] = record_word(hr, w) & vm;
        aw[i] = touched_word(sched, nw, w, tag) & vm & ~hw[i];
        nh += __popc(hw[i]);
        na += __popc(aw[i]);
    }
    int inch = nh, inca = na;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const int vh = __shfl_up(inch, d, 64), va = __shfl_up(inca, d, 64);
        if (lane >= d) {
            inch += vh;
            inca += va;
        }
    }
    const int NH = __shfl(inch, 63, 64), NA = __shfl(inca, 63, 64);
    if (j >= NH + NA) return -1;
    const bool first = j < NH;
    const int r = first ? j : j - NH;
    const int lo = first ? inch - nh : inca - na;
    const int hi = first ? inch : inca;
    const unsigned long long owner = __ballot(lo <= r && r < hi);
    const int src = __ffsll((long long)owner) - 1;
    int t = -1;
    if (lane == src) {
        int left = r - lo;
#pragma unroll
        for (int i = 0; i < kPer; ++i) {
            const uint32_t bits = first ? hw[i] : aw[i];
            const int c = __popc(bits);
            if (t < 0 && left < c) {
                uint32_t b = bits;
                for (int q = 0; q < left; ++q) b &= b - 1u;  // drop the lowest set bits
                t = 32 * (w0 + i) + (__ffs((int)b) - 1);
            } else if (t < 0) {
                left -= c;
            }
        }
    }
    return __shfl(t, src < 0 ? 0 : src, 64);
}

// Visit list of the single-image step of iteration n: the tiles that
// iteration n - 1 recorded as heavy (not quiet), in index order, then the
// other tiles it tagged as touched (a heavy neighbour flipped pixels in
// their bit window).  Every other tile is settled: it was quiet or settled
// in n - 1 and no pixel of its window changed, so its window is still
// uniform, both bit buffers already hold its value and its region sums are
// unchanged.  All NT threads of one workgroup call it; thread i takes a
// contiguous run of record words.  s_tot: 2 x NT / 64 ints of LDS.
template <int NT>
__device__ __forceinline__ void build_plan(const ImgArgs &E, int n, int *s_tot) {
    const int ntiles = E.tiles, nw = (ntiles + 31) >> 5;
    const Record hr = heavy_record(E.sched_mask, nw, n % 3);
    const uint32_t tag = touch_tag(n - 1);
    const int tid = (int)threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int per = (nw + NT - 1) / NT;
    const int w0 = tid * per;
    auto word_masks = [&](int w, uint32_t &h, uint32_t &a) {
        const int valid = min(32, ntiles - 32 * w);
        const uint32_t vm = valid >= 32 ? ~0u : ((1u << valid) - 1u);
        h = record_word(hr, w) & vm;
        a = touched_word(E.sched_mask, nw, w, tag) & vm & ~h;
    };
    // List positions of this thread's first heavy and first other tile: an
    // exclusive scan over the workgroup (within the wave, then over waves).
    auto offsets = [&](int nh, int na, int &oh, int &oa) {
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
            s_tot[NT / 64 + wave] = ia;
        }
        __syncthreads();
        int bh = 0, ba = 0, NH = 0, NA = 0;
        for (int v = 0; v < NT / 64; ++v) {
            if (v < wave) {
                bh += s_tot[v];
                ba += s_tot[NT / 64 + v];
            }
            NH += s_tot[v];
            NA += s_tot[NT / 64 + v];
        }
        oh = 1 + bh + ih - nh;
        oa = 1 + NH + ba + ia - na;
        if (tid == 0) E.plan[0] = NH + NA;
    };
    auto emit = [&](int w, uint32_t h, uint32_t a, int &oh, int &oa) {
        for (; h; h &= h - 1u) E.plan[oh++] = 32 * w + (__ffs((int)h) - 1);
        for (; a; a &= a - 1u) E.plan[oa++] = 32 * w + (__ffs((int)a) - 1);
    };
    constexpr int kKeep = 4;
    int nh = 0, na = 0, oh, oa;
    if (per <= kKeep) {
        // One pass of record loads; the word masks stay in registers.
        uint32_t hm[kKeep], am[kKeep];
#pragma unroll
        for (int i = 0; i < kKeep; ++i) {
            hm[i] = am[i] = 0u;
            if (i < per && w0 + i < nw) {
                word_masks(w0 + i, hm[i], am[i]);
                nh += __popc(hm[i]);
                na += __popc(am[i]);
            }
        }
        offsets(nh, na, oh, oa);
#pragma unroll
        for (int i = 0; i < kKeep; ++i) emit(w0 + i, hm[i], am[i], oh, oa);
    } else {
        // Many words per thread: count, then form the masks again to write.
        for (int i = 0; i < per; ++i) {
            const int w = w0 + i;
            if (w < nw) {
                uint32_t h, a;
                word_masks(w, h, a);
                nh += __popc(h);
                na += __popc(a);
            }
        }
        offsets(nh, na, oh, oa);
        for (int i = 0; i < per; ++i) {
            const int w = w0 + i;
            if (w < nw) {
                uint32_t h, a;
                word_masks(w, h, a);
                emit(w, h, a, oh, oa);
            }
        }
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
}  // namespace lse
