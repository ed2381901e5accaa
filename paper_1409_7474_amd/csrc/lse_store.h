// Kernels templated on the storage type of the resident image (FP32, FP16 or
// BF16) and their launchers.  Included once per storage type by
// lse_store_f32.hip, lse_store_f16.hip and lse_store_bf16.hip, each of which
// instantiates Store<T> for its type, so that every kernel is compiled in
// exactly one translation unit.
#pragma once

#include "lse_device.h"

namespace lse {

// Convert the caller's image (B bands of type T) to the resident copy of type
// ST and check its values.  mode 0: the bands (NB >= B slots, extra ones
// zero); mode 2: the band mean (intensity-only region term).  The per-band totals,
// minima and maxima of the stored (rounded) values are reduced into the image
// statistics lines, so that they describe exactly the image the iterations
// read.
template <typename T, typename ST>
__global__ __launch_bounds__(kThreads) void init_image_kernel(const T *__restrict__ src, int B, int NB,
                                                              ST *__restrict__ dst, long long npx,
                                                              DevState *st, float fix, int mode) {
    const int nsv = mode == 0 ? B : 1;  // statistics values per pixel
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
        if (mode != 0) {
            float g = 0.f;
#pragma unroll
            for (int b = 0; b < 4; ++b)
                if (b < B) g += v[b];
            g = g / (float)B;
            const ST q = from_f32<ST>(g);
            dst[i] = q;
            v[0] = to_f32<ST>(q);
        } else {
#pragma unroll
            for (int b = 0; b < 4; ++b) {
                if (b < NB) {
                    const ST q = from_f32<ST>(v[b]);
                    dst[i * NB + b] = q;
                    v[b] = to_f32<ST>(q);
                }
            }
        }
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            if (b < nsv) {
                if (!(fabsf(v[b]) < 65536.f)) bad = 1;  // overflow of the storage type
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
        for (int b = 0; b < nsv; ++b) {
            float s = 0.f, lo = INFINITY, hi = -INFINITY;
            for (int w = 0; w < kThreads / 64; ++w) {
                s += red[w][b][0];
                lo = fminf(lo, red[w][b][1]);
                hi = fmaxf(hi, red[w][b][2]);
            }
            atomicAdd(reinterpret_cast<unsigned long long *>(&bin.total[b]),
                      (unsigned long long)__float2ll_rn(s * fix));
            atomicMin(&bin.imin_key[b], float_key(lo));
            atomicMax(&bin.imax_key[b], float_key(hi));
        }
    }
}

// Region statistics of the LSF given by `bits` (raw: phi = b; else phi = G * b).
template <int NB, typename ST>
__global__ __launch_bounds__(kThreads) void stats_kernel(StepArgs A, int raw, int slot) {
    extern __shared__ float smem[];
    const TileSmem s = carve(smem, A.r, A.nch, 0);
    const int x0 = blockIdx.x * kTileX, y0 = blockIdx.y * kTileY;
    stage_tables(s, A.taps, A.ts, A.nch);
    stage_bits(s.bn, A.bits_in, y0 - A.r, kTileY + 2 * A.r, x0, A.H, A.WW);
    __syncthreads();
    float acc[NB];
    int cnt;
    stats_tile<NB, ST>(s, static_cast<const ST *>(A.img), x0, y0, A.H, A.W, A.r, A.ts, A.nch, raw, acc, cnt);
    reduce_commit<NB>(s, acc, cnt, 0, &A.st->slot[slot][block_linear_id() % kBins], A.fix, true);
}

// Edge map of eq. (14) in one pass over an EMX x EMY output tile: the gray
// value (band mean times the scale, as the listing's 8-bit intensity) on the
// tile plus a (r1 + 1) halo, the image pre-smoothing G_sigma1 * gray as a
// horizontal then a vertical FMA chain in tap order (taps outside the image
// contribute nothing: zero padding), the central-difference gradient of the
// smoothed image (one-sided on the image border), and g = 1 / (1 + |grad|^2)
// rounded once to the storage type.  Every value is computed with the same
// FP32 operations, in the same order, as separate whole-image passes would.
// Each wave takes whole rows (lane = column), so no index is divided.
constexpr int kEMX = 128, kEMY = 32;
constexpr int kMaxTaps1 = 31;  // 2 r1 + 1 <= 31

inline size_t edge_map_smem_bytes(int r1) {
    const size_t gw = kEMX + 2 + 2 * r1, gh = kEMY + 2 + 2 * r1;
    return (gh * gw + gh * (kEMX + 2)) * 4;
}

// The B band values of one pixel as FP32 (zeros past B); V4: four bands read
// with one vector load (the caller checked the alignment).
template <typename T, bool V4>
__device__ __forceinline__ void load_bands(const T *__restrict__ px, int B, float v[4]) {
    if constexpr (V4) {
        T q[4];
        if constexpr (sizeof(T) == 4) {
            const float4 f = *reinterpret_cast<const float4 *>(px);
            __builtin_memcpy(q, &f, sizeof(q));
        } else {
            const uint2 u = *reinterpret_cast<const uint2 *>(px);
            __builtin_memcpy(q, &u, sizeof(q));
        }
#pragma unroll
        for (int b = 0; b < 4; ++b) v[b] = to_f32<T>(q[b]);
    } else {
#pragma unroll
        for (int b = 0; b < 4; ++b) v[b] = b < B ? to_f32<T>(px[b]) : 0.f;
    }
}

template <typename T, typename ST, bool V4>
__global__ __launch_bounds__(kThreads) void edge_map_kernel(const T *__restrict__ src, int B, float scale,
                                                            const Taps *__restrict__ taps, int r1,
                                                            ST *__restrict__ g, int H, int W, DevState *st) {
    extern __shared__ float smem[];
    constexpr int NW = kThreads / 64;
    const int GW = kEMX + 2 + 2 * r1, GH = kEMY + 2 + 2 * r1, SW = kEMX + 2;
    // gray: GH x GW from image (y0 - 1 - r1, x0 - 1 - r1); later the smoothed
    // image, (kEMY + 2) x SW from (y0 - 1, x0 - 1).  Horizontal sums: GH x SW
    // from (y0 - 1 - r1, x0 - 1).
    float *sg = smem, *sh = smem + GH * GW;
    const int lane = threadIdx.x & 63, wave = wave_id();
    const int x0 = blockIdx.x * kEMX, y0 = blockIdx.y * kEMY;
    const int ts1 = 2 * r1 + 1;
    float k1[kMaxTaps1];
#pragma unroll
    for (int j = 0; j < kMaxTaps1; ++j) k1[j] = taps->k1[j];
    // FMA chain sum_j k1[j] p[j * stride] in tap order (unrolled: the taps
    // stay in scalar registers; the uniform test ends it after ts1 taps).
    auto chain = [&](const float *p, int stride) {
        float acc = 0.f;
#pragma unroll
        for (int j = 0; j < kMaxTaps1; ++j) {
            if (j >= ts1) break;
            acc = fmaf(k1[j], p[j * stride], acc);
        }
        return acc;
    };
    // Gray rows, four per wave at a time (twelve pixel loads in flight).
    constexpr int RB = 4;
    int bad = 0;
    for (int r0 = wave; r0 < GH; r0 += RB * NW) {
        float v[RB][3][4];
        bool ok[RB][3];
#pragma unroll
        for (int i = 0; i < RB; ++i) {
            const int r = r0 + i * NW, y = y0 - 1 - r1 + r;
            const bool rok = r < GH && y >= 0 && y < H;
#pragma unroll
            for (int q = 0; q < 3; ++q) {  // GW <= 160 < 3 x 64
                const int c = lane + 64 * q, x = x0 - 1 - r1 + c;
                ok[i][q] = rok && c < GW && x >= 0 && x < W;
                if (ok[i][q])
                    load_bands<T, V4>(src + ((size_t)y * W + x) * B, B, v[i][q]);
                else
                    v[i][q][0] = v[i][q][1] = v[i][q][2] = v[i][q][3] = 0.f;
            }
        }
#pragma unroll
        for (int i = 0; i < RB; ++i) {
            const int r = r0 + i * NW;
#pragma unroll
            for (int q = 0; q < 3; ++q) {
                const int c = lane + 64 * q;
                float sum = 0.f;
#pragma unroll
                for (int b = 0; b < 4; ++b) {
                    if (b < B) {
                        if (!(fabsf(v[i][q][b]) < 65536.f)) bad = 1;  // also catches NaN / Inf
                        sum += v[i][q][b];
                    }
                }
                if (r < GH && c < GW) sg[r * GW + c] = ok[i][q] ? scale * (sum / (float)B) : 0.f;
            }
        }
    }
    __syncthreads();
    for (int r = wave; r < GH; r += NW) {
#pragma unroll
        for (int q = 0; q < 3; ++q) {
            const int c = lane + 64 * q;
            if (c < SW) sh[r * SW + c] = chain(sg + r * GW + c, 1);
        }
    }
    __syncthreads();
    float *ss = sg;
    for (int r = wave; r < kEMY + 2; r += NW) {
#pragma unroll
        for (int q = 0; q < 3; ++q) {
            const int c = lane + 64 * q;
            if (c < SW) ss[r * SW + c] = chain(sh + r * SW + c, SW);
        }
    }
    __syncthreads();
    for (int ty = wave; ty < kEMY; ty += NW) {
        const int y = y0 + ty;
        if (y >= H) break;
#pragma unroll
        for (int q = 0; q < 2; ++q) {
            const int tx = lane + 64 * q, x = x0 + tx;
            if (x >= W) continue;
            const float *c0 = ss + (ty + 1) * SW + (tx + 1);
            float gx, gy;
            if (x == 0)
                gx = c0[1] - c0[0];
            else if (x == W - 1)
                gx = c0[0] - c0[-1];
            else
                gx = 0.5f * (c0[1] - c0[-1]);
            if (y == 0)
                gy = c0[SW] - c0[0];
            else if (y == H - 1)
                gy = c0[0] - c0[-SW];
            else
                gy = 0.5f * (c0[SW] - c0[-SW]);
            g[(size_t)y * W + x] = from_f32<ST>(1.f / (1.f + (gx * gx + gy * gy)));
        }
    }
    if (bad) st->bad = 1;
}

// Region image with several stored bands and its pruning boxes in one pass
// (init_image mode 0 together with the normaliser's block boxes): each workgroup converts
// kIBoxBlocks 64 x 32 blocks (a wave takes every fourth row, lane = column),
// stores each pixel's NB values with one vector store, and reduces both the
// block's band minima / maxima of the stored values (the normaliser boxes)
// and, as init_image does, the image statistics lines of the stored values.
constexpr int kIBoxBlocks = 4;

template <typename ST, int NB>
__device__ __forceinline__ void store_px(ST *__restrict__ dst, long long pix, const ST (&q)[NB]) {
    if constexpr (sizeof(ST) == 4) {
        float *f = reinterpret_cast<float *>(dst) + pix * NB;
        if constexpr (NB == 4)
            *reinterpret_cast<float4 *>(f) = make_float4(q[0], q[1], q[2], q[3]);
        else
            *reinterpret_cast<float2 *>(f) = make_float2(q[0], q[1]);
    } else {
        uint32_t u[NB];
#pragma unroll
        for (int b = 0; b < NB; ++b) u[b] = __builtin_bit_cast(unsigned short, q[b]);
        unsigned short *h = reinterpret_cast<unsigned short *>(dst) + pix * NB;
        if constexpr (NB == 4)
            *reinterpret_cast<uint2 *>(h) = make_uint2(u[0] | (u[1] << 16), u[2] | (u[3] << 16));
        else
            *reinterpret_cast<uint32_t *>(h) = u[0] | (u[1] << 16);
    }
}

template <typename T, typename ST, int NB, bool V4>
__global__ __launch_bounds__(kThreads) void init_image_box_kernel(const T *__restrict__ src, int B, ST *__restrict__ dst,
                                                                  int H, int W, DevState *st, float fix,
                                                                  float *__restrict__ boxes) {
    static_assert(NB == 2 || NB == 4, "boxes are kept for two or four stored bands");
    constexpr int NWV = kThreads / 64, RW = kMBY / NWV;
    __shared__ float sbox[NWV][2 * NB];
    __shared__ float red[NWV][4][3];
    const int lane = threadIdx.x & 63, wave = wave_id();
    const int nbx = (W + kMBX - 1) / kMBX, nblk = nbx * ((H + kMBY - 1) / kMBY);
    float sum[4] = {0.f, 0.f, 0.f, 0.f};
    float mn[4] = {INFINITY, INFINITY, INFINITY, INFINITY};
    float mx[4] = {-INFINITY, -INFINITY, -INFINITY, -INFINITY};
    int bad = 0;
    for (int qb = 0; qb < kIBoxBlocks; ++qb) {
        const int blk = blockIdx.x * kIBoxBlocks + qb;
        if (blk >= nblk) break;
        const int x = (blk % nbx) * kMBX + lane, y0 = (blk / nbx) * kMBY + wave;
        float v[RW][4];
        bool ok[RW];
#pragma unroll
        for (int i = 0; i < RW; ++i) {  // every row load of the wave in flight
            const int y = y0 + i * NWV;
            ok[i] = x < W && y < H;
            if (ok[i])
                load_bands<T, V4>(src + ((size_t)y * W + x) * B, B, v[i]);
            else
                v[i][0] = v[i][1] = v[i][2] = v[i][3] = 0.f;
        }
        float lo[NB], hi[NB];
#pragma unroll
        for (int b = 0; b < NB; ++b) {
            lo[b] = INFINITY;
            hi[b] = -INFINITY;
        }
#pragma unroll
        for (int i = 0; i < RW; ++i) {
            if (!ok[i]) continue;
            ST q[NB];
#pragma unroll
            for (int b = 0; b < NB; ++b) {
                if (b < B && !(fabsf(v[i][b]) < 65536.f)) bad = 1;  // also catches NaN / Inf
                q[b] = from_f32<ST>(b < B ? v[i][b] : 0.f);
                const float s = to_f32<ST>(q[b]);
                lo[b] = fminf(lo[b], s);
                hi[b] = fmaxf(hi[b], s);
                if (b < B) {
                    if (!(fabsf(s) < 65536.f)) bad = 1;  // overflow of the storage type
                    sum[b] += s;
                    mn[b] = fminf(mn[b], s);
                    mx[b] = fmaxf(mx[b], s);
                }
            }
            store_px<ST, NB>(dst, (long long)(y0 + i * NWV) * W + x, q);
        }
#pragma unroll
        for (int b = 0; b < NB; ++b) {
            lo[b] = wave_min_f(lo[b]);
            hi[b] = wave_max_f(hi[b]);
        }
        if (lane == 0) {
#pragma unroll
            for (int b = 0; b < NB; ++b) {
                sbox[wave][b] = lo[b];
                sbox[wave][NB + b] = hi[b];
            }
        }
        __syncthreads();
        if (threadIdx.x < 2 * NB) {
            const int k = threadIdx.x;
            float r = sbox[0][k];
            for (int w = 1; w < NWV; ++w) r = k < NB ? fminf(r, sbox[w][k]) : fmaxf(r, sbox[w][k]);
            boxes[(size_t)blk * 2 * NB + k] = r;
        }
        __syncthreads();  // sbox is reused by the next block
    }
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
            for (int w = 0; w < NWV; ++w) {
                s += red[w][b][0];
                lo = fminf(lo, red[w][b][1]);
                hi = fmaxf(hi, red[w][b][2]);
            }
            atomicAdd(reinterpret_cast<unsigned long long *>(&bin.total[b]),
                      (unsigned long long)__float2ll_rn(s * fix));
            atomicMin(&bin.imin_key[b], float_key(lo));
            atomicMax(&bin.imax_key[b], float_key(hi));
        }
    }
}

// ------------------------------------------------------------ normaliser

// Normaliser M = max_x |D(x)| of eq. (17), for B > 1 (B = 1 uses the closed
// form from the image min / max, since D is then monotone in I).
//
// Normaliser M of eq. (17), exact, with pruning: the image is cut into
// 64 x 32 blocks whose per-band min / max init_image_box_kernel stores at
// init.  D is affine in the pixel value, so over a
// block |D| is bounded by its value at the box corners; a rounding margin
// makes the bound hold for the FP32 D of every pixel.  The previous
// iteration's maximising pixel, evaluated with the current means, gives a
// lower bound LB <= M; only blocks whose bound reaches LB can hold the
// maximum, and only those are read.  With no previous pixel (LB = 0) every
// block is read.  The result (value and pixel) equals a full scan bit for bit.
// (mpass_kernel below.)

// Workgroup -> (image, unit) of a launch: single image (map == nullptr) or an
// entry of a batch map, image index in the high bits, unit (tile or block
// group) in the low `unit_bits` bits.  Returns false for a spare workgroup.
__device__ __forceinline__ bool batch_unit(const uint32_t *__restrict__ map, int unit_bits, int &img, int &unit) {
    if (!map) {
        img = 0;
        unit = (int)blockIdx.x;
        return true;
    }
    const uint32_t v = map[blockIdx.x];
    if (v == kNoTile) return false;
    img = (int)(v >> unit_bits);
    unit = (int)(v & ((1u << unit_bits) - 1u));
    return true;
}

template <int NB, typename ST>
__global__ __launch_bounds__(kThreads) void mpass_kernel(const ImgArgs *__restrict__ args,
                                                          const uint32_t *__restrict__ map, int unit_bits, int k,
                                                          int stop) {
    int ii, grp;
    if (!batch_unit(map, unit_bits, ii, grp)) return;
    const ImgArgs &A = args[ii];
    const int n = A.n0 + k;
    if (n >= A.target) return;
    if (!map && grp >= A.mgroups) {
        // One extra workgroup of a single-image launch builds the step's visit list.
        __shared__ int s_tot[2 * (kThreads / 64)];
        if (A.plan) build_plan<kThreads>(A, n, s_tot);
        return;
    }
    DevState *st = A.st;
    const int sl = n % 3;
    __shared__ Totals tot;
    __shared__ unsigned long long wkey[kThreads / 64];
    __shared__ int scan_list[kMBlocksPerWG];
    __shared__ int nscan;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    __shared__ float prev_px[NB];  // image values of the previous iteration's maximising pixel
    __shared__ int prev_ok;
    if (wave == 2 && lane == 0) {
        // Recorded by the step of iteration n - 1 in its statistics slot
        // ((n + 2) % 3, cleared only by the step of iteration n).
        const Bin &b0 = st->slot[(n + 2) % 3][0];
        const float *pf = reinterpret_cast<const float *>(&b0.pad[0]);
#pragma unroll
        for (int b = 0; b < NB; ++b) prev_px[b] = pf[b];
        prev_ok = b0.pad[2] != 0ull;
    }
    // This workgroup's block boxes (lane k < kMBlocksPerWG of wave 0) do not
    // depend on the statistics: load them before the statistics barrier.
    const int nbx = (A.W + kMBX - 1) / kMBX, nby = (A.H + kMBY - 1) / kMBY, nblk = nbx * nby;
    const int myblk = grp * kMBlocksPerWG + lane;
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
    if (tot.done || tot.bad || (stop && tot.flips == 0)) return;
    float cp[NB], cm[NB], a[NB], m[NB];
    slot_means<NB>(tot, A.hw, A.inv_fix, cp, cm);
#pragma unroll
    for (int b = 0; b < NB; ++b) {
        a[b] = cp[b] - cm[b];
        m[b] = cp[b] + cm[b];
    }
    const __amdgpu_buffer_rsrc_t img_rs = image_rsrc(A.img, (uint32_t)(A.hw * (long long)(NB * sizeof(ST))));
    float lb = 0.f;
    if (prev_ok) {
        Px<NB> pv;
#pragma unroll
        for (int b = 0; b < NB; ++b) pv.v[b] = prev_px[b];
        lb = fabsf(region_D<NB>(pv, a, m));
    }

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
    for (int q = 0; q < nscan; ++q) {
        const int blk = scan_list[q];
        const int bx = blk % nbx, by = blk / nbx;
        const int x = bx * kMBX + lane;
        // Every row load of this wave in flight at once (buffer loads: no
        // branches; outside the image they return zeros), then the keys.
        constexpr int RW = kMBY / (kThreads / 64);
        Px<NB> v[RW];
#pragma unroll
        for (int i = 0; i < RW; ++i) {
            const int y = by * kMBY + wave + i * (kThreads / 64);
            const bool ok = x < A.W && y < A.H;
            v[i] = buffer_px<ST, NB>(img_rs, ok ? (uint32_t)((long long)y * A.W + x) * (uint32_t)(NB * sizeof(ST))
                                                : kNoLoad);
        }
#pragma unroll
        for (int i = 0; i < RW; ++i) {
            const int y = by * kMBY + wave + i * (kThreads / 64);
            if (x < A.W && y < A.H) {
                const unsigned int pix = (unsigned int)((long long)y * A.W + x);
                const unsigned long long key = mkey_of(fabsf(region_D<NB>(v[i], a, m)), pix);
                best = key > best ? key : best;
            }
        }
    }
    best = wave_max_u64_dpp(best);
    if (lane == 0) wkey[wave] = best;
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < kThreads / 64; ++w) best = wkey[w] > best ? wkey[w] : best;
        if (best) atomicMax(&st->slot[sl][blockIdx.x % kBins].mkey, best);
    }
}

// ------------------------------------------------------------------- step

template <int NB, bool EDGE, typename ST>
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
                coef = A.dt * to_f32<ST>(static_cast<const ST *>(A.img)[pix]);
            } else {
                coef = w * region_D<NB>(load_px<ST, NB>(static_cast<const ST *>(A.img), pix), a, m);
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
        stats_tile<NB, ST>(s, static_cast<const ST *>(A.img), x0, y0, H, W, r, ts, nch, 0, acc, cnt);
    }
    reduce_commit<NB>(s, acc, cnt, flips, out, A.fix, !EDGE);

    if (lead_block) {
        // Clear the slot of iteration n + 2 (nobody reads or writes it now).
        unsigned long long *z = reinterpret_cast<unsigned long long *>(&st->slot[(A.n + 2) % 3][0]);
        for (int i = threadIdx.x; i < (int)(kBins * sizeof(Bin) / 8); i += kThreads) z[i] = 0ull;
    }
    if constexpr (!EDGE && NB > 1)
        if (lead) record_max_pixel<NB, ST>(st, sl, tot.mkey, A.img, A.hw);
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

// One iteration (Table I steps 2-4, plus the statistics of step 2.1 for the
// next iteration) on one 96 x FY tile of one image (FY = 48 rows for the
// region term, 64 for the edge term).  Launch k runs iteration
// n = n0 + k of every image it covers (one image when map is null; else the
// workgroup map names image and tile).
template <int R, int NB, bool EDGE, typename ST, int V>
// V: the variant's tile rows and waves per SIMD (StepVariant).  At 4 waves per
// SIMD the B = 4 region kernels of the larger radii are held to 128 VGPRs.
__global__ __launch_bounds__(kThreads, (StepVariant<EDGE, V>::OCC)) void step_fast_kernel(
    const ImgArgs *__restrict__ args, const uint32_t *__restrict__ map, const int *__restrict__ nmap, int unit_bits,
    int k, int stop) {
    using G = FastGeom<R, EDGE, StepVariant<EDGE, V>::FY>;
    constexpr int TS = G::TS;
    extern __shared__ float smem[];
    __shared__ Totals tot;
    __shared__ float red[kThreads / 64 * 8];
    __shared__ int s_tile;
    __shared__ int s_dirs;             // neighbours whose bit windows this step's flips reach (flip_dirs)
    __shared__ int s_uni[kThreads / 64];  // per wave: its codes of the quiet window all 1 (bit 0) / all 0 (bit 1)
    __shared__ TileSum s_prev, s_all;  // region: the tile's latest contribution; its all-inside sums
    int ii = 0, t = (int)blockIdx.x;
    if (map) {
        // Step map entry and (visit list) its length, loaded together: lists
        // are padded to the launch grid.  Workgroups past the length have no work.
        const uint32_t v = map[blockIdx.x];
        const int len = nmap ? *nmap : 0x7fffffff;
        if ((int)blockIdx.x >= len || v == kNoTile) return;
        ii = (int)(v >> unit_bits);
        t = (int)(v & ((1u << unit_bits) - 1u));
    }
    const ImgArgs &E = args[ii];
    // Single image without a visit list: the active tiles of small images,
    // heavy ones first, found by each workgroup in the records; settled
    // tiles have nothing to do.
    const bool dyn = map == nullptr && E.sched_mask != nullptr;
    if (!map && !dyn) t = tile_of(E.tiles);
    const int n = E.n0 + k;
    if (n >= E.target) return;
    if (dyn ? (int)blockIdx.x >= E.tiles : t < 0) return;
    const int nw = (E.tiles + 31) >> 5;                  // words of one schedule mask
    const int sbn = (n + 1) % 3, sbr = (n + 2) % 3;     // masks written / cleared by this iteration
    // Tables do not depend on the tile: their loads overlap the schedule's.
    LutRegs<G::NCH> lut;
    load_luts<G::NCH>(E.taps, lut);
    float kk[TS];
#pragma unroll
    for (int i = 0; i < TS; ++i) kk[i] = E.taps->k[i];
    const float *cum = E.taps->cum;
    if (dyn) {
        if ((threadIdx.x >> 6) == 0) {
            const int tt = active_first_tile(E.sched_mask, n, E.tiles, (int)blockIdx.x);
            if (threadIdx.x == 0) s_tile = tt;
        }
        __syncthreads();
        t = s_tile;
        if (t < 0) return;
    }
    StepArgs A;
    A.img = E.img;
    A.bits_in = E.bits[n & 1];
    A.bits_out = E.bits[(n + 1) & 1];
    A.st = E.st;
    A.taps = E.taps;
    A.H = E.H;
    A.W = E.W;
    A.WW = E.WW;
    A.dt = E.dt;
    A.n = n;
    A.stop = stop;
    A.fix = E.fix;
    A.inv_fix = E.inv_fix;
    A.hw = E.hw;
    DevState *st = A.st;
    const int sl = A.n % 3;
    const int H = A.H, W = A.W;
    const int tid = threadIdx.x, lane = tid & 63, wave = wave_id();
    const int ntx = (W + kFX - 1) / kFX;
    int x0 = 0, y0 = 0, by0 = 0, px0 = 0, py0 = 0;
    bool border = true;
    auto set_tile = [&](int tt) {
        x0 = (tt % ntx) * kFX;
        y0 = (tt / ntx) * G::FY;
        by0 = y0 - G::RU - 1 - R;  // image row of staged bit row 0
        px0 = x0 - G::RU - 1;
        py0 = y0 - G::RU - 1;
        border = x0 - 2 * R - 2 < 0 || x0 + kFX + 2 * R + 2 > W;
    };
    set_tile(t);
    uint32_t *s_bits = reinterpret_cast<uint32_t *>(smem);
    float *s_phi = smem + G::BH * kFWords;
    uint32_t *s_bn = reinterpret_cast<uint32_t *>(s_phi + G::PH * G::PS);
    int *s_codes = reinterpret_cast<int *>(s_bn + G::UH * kFWords);    // [max(BH, UH)][2]
    int *s_pcode = s_codes + G::BH * 2;                                  // [PHP][2]: phi row uniformity
    uint32_t *s_const = reinterpret_cast<uint32_t *>(s_pcode + G::PHP * 2);  // all-ones / all-zeros rows

    // A: b^{n-1} on the tile + 2R+1 halo, and (region) the tile's previous
    // record and all-inside sums, issued before the statistics loads so that
    // the memory round trips overlap.
    const bool track = !EDGE && E.tilelast != nullptr;
    // The totals this kernel reads: the edge term only the flips and flags;
    // the band minimum and maximum only for one band (the closed-form M).
    // Four waves share the reductions.
    static_assert(kThreads == 256, "the totals reductions are split over four waves");
    TotalsRegs tregs;
    totals_issue(st, sl, !EDGE, tregs, true, !EDGE, NB == 1);
    long long rec_w = 0, all_w = 0;
    if (!EDGE && tid < 8) {
        if (track) rec_w = reinterpret_cast<const long long *>(&E.tilelast[t])[tid];
        all_w = reinterpret_cast<const long long *>(&E.tilesum[t])[tid];
    }
    stage_bits_fast<G::BH>(s_bits, A.bits_in, by0, x0, H, A.WW);
    if (tid < 16) s_const[tid] = tid < 8 ? ~0u : 0u;
    if (tid == 0) s_dirs = 0;
    if (!EDGE && tid < 8) {
        reinterpret_cast<long long *>(&s_prev)[tid] = rec_w;
        reinterpret_cast<long long *>(&s_all)[tid] = all_w;
    }
    totals_commit(!EDGE, tregs, &tot, true, !EDGE, NB == 1);
    __syncthreads();
    // Tile 0 leads: every iteration visits it (it is always recorded heavy).
    const bool lead_block = t == 0;
    const bool lead = lead_block && threadIdx.x == 0;
    {
        int done = tot.done | tot.bad;
        if (!done && A.stop && tot.flips == 0) done = 1;
        if (done) {
            if (lead && !tot.bad) st->done = 1;
            return;
        }
    }
    const bool raw = tot.raw && n == 0;
    if constexpr (!EDGE) {
        // The totals of iteration n carry into n + 1; each visited tile adds
        // the change of its own sums.
        if (lead && track) {
            Bin *o = &st->slot[sbn][blockIdx.x % kBins];
#pragma unroll
            for (int b = 0; b < NB; ++b)
                if (tot.sum[b]) atomicAdd(reinterpret_cast<unsigned long long *>(&o->sum[b]),
                                          (unsigned long long)tot.sum[b]);
            if (tot.nplus) atomicAdd(&o->nplus, tot.nplus);
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
        const float h1 = hconv_fast<R, G::NCH>(s_const, 64, HPad{0u, 0.f}, lut);
        const float h0 = hconv_fast<R, G::NCH>(s_const + 8, 64, HPad{0u, 0.f}, lut);
#pragma unroll
        for (int i = 0; i < TS; ++i) {
            phi_one = fmaf(kk[i], h1, phi_one);
            phi_zero = fmaf(kk[i], h0, phi_zero);
        }
    }
    constexpr int NV = EDGE ? 1 : NB;               // values per pixel: edge map or image bands
    constexpr int PB = NV * (int)sizeof(ST);        // bytes per pixel
    const __amdgpu_buffer_rsrc_t img_rs = image_rsrc(A.img, (uint32_t)((unsigned long long)H * W * PB));
    // U-row words of an all-ones binarised row (the two ballots' valid lanes).
    const unsigned long long ones1 = (32 + 2 * G::RU >= 64) ? ~0ull : ((1ull << (32 + 2 * G::RU)) - 1ull);

    {
        // Codes of the staged rows over each chunk's window span: the bits
        // that phi^n of the chunk's columns reads, and (edge term) for chunk 0
        // also those of the first two phi columns of chunk 1, which the
        // gradient of its last pixels reads.
        // The same pass notes, per wave, whether its codes of the rows the
        // quiet test reads are all 1 or all 0, so that the test needs no
        // barrier of its own.
        int all1 = 1, all0 = 1;
        for (int i = tid; i < G::BH * 2; i += kThreads) {
            const int row = i >> 1, c = i & 1;
            const int code = c == 0 ? range_code(s_bits + row * kFWords, 31 - G::RU - R, (EDGE ? 97 : 95) - G::RU + R)
                                    : range_code(s_bits + row * kFWords, 95 - G::RU - R, 129 + G::RU + R);
            s_codes[i] = code;
            if (i < (G::PH + 2 * R) * 2) {
                all1 &= code == 1;
                all0 &= code == 0;
            }
        }
        {
            const unsigned long long n1 = __ballot(!all1), n0 = __ballot(!all0);
            if (lane == 0) s_uni[wave] = (n1 == 0ull ? 1 : 0) | (n0 == 0ull ? 2 : 0);
        }
        __syncthreads();

        // Quiet tile: inside the image with its whole halo, and b^{n-1}
        // uniform over every staged bit it reads.  Then phi^n is one constant
        // there, |grad phi^n| = 0 and u = phi^n exactly (eq. (18)), so b^n =
        // b^{n-1} on the tile plus its halo, and phi^{n+1} = G * b^n has that
        // sign on every owned pixel: the tile's region sums are all or
        // nothing.  The all-inside sums were computed at init by this
        // kernel's own reduction (tile_sums_kernel), so the totals are those
        // of the full computation bit for bit.
        // Tile 0 is never quiet (it is also a border tile): it carries the
        // bookkeeping of the iteration (totals carry-over, slot and record
        // clearing, iteration count), so it must be recorded heavy every
        // iteration, which makes the next iteration visit it.
        int quiet = -1;
        if (!border && t != 0 && by0 >= 0 && by0 + G::PH + 2 * R <= H) {
            int u = 3;
#pragma unroll
            for (int v = 0; v < kThreads / 64; ++v) u &= s_uni[v];
            quiet = (u & 1) ? 1 : ((u & 2) ? 0 : -1);
        }
        // Record heavy tiles: the next iteration visits them (and those of
        // their neighbours whose bit windows their flips reach: mark_touched).
        if (tid == 0 && quiet < 0 && E.sched_mask)
            atomicOr(&E.sched_mask[(size_t)sbn * nw + (t >> 5)], 1u << (t & 31));
        if (quiet >= 0) {
            if (tid < G::FY * 3) {
                const int row = tid / 3, k = tid - row * 3;
                A.bits_out[(size_t)(y0 + row) * A.WW + (x0 >> 5) + k] = quiet ? ~0u : 0u;
            }
            if constexpr (!EDGE) {
                // All or nothing: the all-inside sums, or zero.
                if (tid == 0) {
                    long long cur[NB];
#pragma unroll
                    for (int b = 0; b < NB; ++b) cur[b] = quiet ? s_all.sum[b] : 0;
                    commit_tile<NB>(cur, quiet ? s_all.cnt : 0, track ? &s_prev : nullptr,
                                    track ? &E.tilelast[t] : nullptr, &st->slot[sbn][blockIdx.x % kBins]);
                }
            }
        } else {
            // B: phi^n on P = tile + (RU + 1) halo; wave = (column chunk, row segment).
            {
                const int chunk = wave & 1, seg = wave >> 1;
                const int p = chunk * 64 + lane;
                const int x = px0 + p;
                const int xb = x - x0 + 32;
                const bool colok = p < G::PW && x >= 0 && x < W;
                // Only in border tiles, and there only in the chunk next to
                // the edge, do the taps reach outside the image.
                const bool cborder = border && span_outside(x0, W, chunk == 0 ? 31 - G::RU - R : 95 - G::RU - R,
                                                            chunk == 0 ? (EDGE ? 97 : 95) - G::RU + R : 129 + G::RU + R);
                if (raw) {
                    for (int j = 0; j < G::SEG; ++j) {
                        const int q = seg * G::SEG + j, y = py0 + q;
                        float v = 0.f;
                        if (colok && y >= 0 && y < H) {
                            const uint32_t wd = s_bits[(q + R) * kFWords + (xb >> 5)];
                            v = ((wd >> (xb & 31)) & 1u) ? 1.f : -1.f;
                        }
                        if (p < G::PW && q < G::PH) s_phi[q * G::PS + p] = v;
                        if (lane == 0) s_pcode[q * 2 + chunk] = 2;
                    }
                } else {
                    constexpr int KB = G::KB;
                    constexpr int NW = 2 * R + KB;
                    float win[NW];
                    const int brow0 = seg * G::SEG;  // staged bit row of window entry 0
                    const HPad pad = hpad_of<R>(x, W, cborder, cum);
                    bool have_win = false;
    #pragma unroll 1
                    for (int blk = 0; blk < G::NBLK; ++blk) {
                        const int rb = brow0 + blk * KB;
                        int uni = -1;
                        if (!cborder && by0 + rb >= 0 && by0 + rb + KB + 2 * R <= H)
                            uni = block_code(s_codes, rb, KB + 2 * R, chunk);
                        if (uni >= 0) {
                            const float v = uni ? phi_one : phi_zero;
    #pragma unroll
                            for (int j = 0; j < KB; ++j) {
                                const int q = rb + j;
                                if (p < G::PW && q < G::PH) s_phi[q * G::PS + p] = colok ? v : 0.f;
                            }
                            if (lane < KB) s_pcode[(rb + lane) * 2 + chunk] = uni;
                            have_win = false;
                            continue;
                        }
                        if (!have_win) {
    #pragma unroll
                            for (int t2 = 0; t2 < 2 * R; ++t2) {
                                const int y = by0 + rb + t2;
                                const float v =
                                    hconv_fast<R, G::NCH>(s_bits + (rb + t2) * kFWords, xb, pad, lut);
                                win[t2] = (y >= 0 && y < H) ? v : 0.f;
                            }
                        }
    #pragma unroll
                        for (int t2 = 0; t2 < KB; ++t2) {
                            const int brow = rb + 2 * R + t2;
                            const int y = by0 + brow;
                            const float v = hconv_fast<R, G::NCH>(s_bits + brow * kFWords, xb, pad, lut);
                            win[2 * R + t2] = (y >= 0 && y < H) ? v : 0.f;
                        }
    #pragma unroll
                        for (int j = 0; j < KB; ++j) {
                            float ph = 0.f;
    #pragma unroll
                            for (int i = 0; i < TS; ++i) ph = fmaf(kk[i], win[j + i], ph);
                            const int q = rb + j, y = py0 + q;  // phi row q <-> bit rows q .. q + 2R
                            if (p < G::PW && q < G::PH) s_phi[q * G::PS + p] = (colok && y >= 0 && y < H) ? ph : 0.f;
                        }
                        if (lane < KB) s_pcode[(rb + lane) * 2 + chunk] = 2;
    #pragma unroll
                        for (int t2 = 0; t2 < 2 * R; ++t2) win[t2] = win[t2 + KB];
                        have_win = true;
                    }
                }
            }
            __syncthreads();

            // C: update eq. (18) and binarisation on U = tile + RU halo, in blocks
            // of 8 rows per wave task; blocks whose phi rows are one uniform
            // constant (interior tiles) have |grad phi| = 0: b = sign(phi).
            int flips = 0;
            // Owned flips near the tile's sides, by the neighbours whose bit
            // windows (the staged rows and columns of the quiet test: RU + R + 1
            // pixels beyond the tile, one more on the right) they reach.
            int dirs = 0;
            constexpr int HWB = G::RU + R + 2;
            constexpr int NBC = (G::UH + kSB - 1) / kSB;
            // Word-forming lane of a row group: row wrow, word wk of the staged row.
            const int wrow = lane / kFWords, wk = lane - wrow * kFWords;
            // Per lane and chunk, fixed for the whole phase: the U column, its
            // image column, whether it lies in U and in the image, its phi
            // column, and the weights of the x difference (central inside,
            // one-sided on the image's first and last column):
            // gx = ar * phi(x+1) + al * phi(x-1) + ac * phi(x), each case
            // rounding exactly as 0.5 (phi(x+1) - phi(x-1)), phi(1) - phi(0)
            // or phi(W-1) - phi(W-2) does.
            // (The phi column of U column xb = 32 - RU + ucol is ucol + 1;
            // ac = -(ar + al).)
            // In the edge term U is the tile itself (RU = 0), so chunk 1 holds
            // only 32 columns: there each lane half takes its own row (lanes
            // 0-31 row 2j, lanes 32-63 row 2j + 1 of a packed slot).
            constexpr bool PK = G::RU == 0;
            const int hl = lane >> 5;
            const int ucol[2] = {lane, PK ? 64 + (lane & 31) : 64 + lane};
            const int cx0 = x0 - G::RU + lane;
            bool cok[2];
            float ar[2], al[2];
    #pragma unroll
            for (int c = 0; c < 2; ++c) {
                const int x = x0 - G::RU + ucol[c];
                cok[c] = ucol[c] < 96 + 2 * G::RU && x >= 0 && x < W;
                const bool first = x == 0, last = x == W - 1;
                ar[c] = first ? 1.f : (last ? 0.f : 0.5f);
                al[c] = first ? 0.f : (last ? -1.f : -0.5f);
            }
    #pragma unroll 1
            for (int bi = wave; bi < NBC; bi += kThreads / 64) {
                const int u0 = bi * kSB;
                const int nr = min(kSB, G::UH - u0);
                // Per chunk: whether phi rows u0 .. u0 + nr + 1 are one constant
                // over the chunk's phi columns (then |grad phi| = 0 there and
                // b = sign(phi), eq. (18)).  Both chunks alike, away from the
                // left and right image edges: the whole block at once.  The
                // edge term also takes one uniform chunk on its own (its codes
                // cover the gradient's extra columns); in the region kernel
                // that measured slower alone.
                int rc = -1, ucs[2];
                {
                    const int ncode = (nr + 2) * 2;  // entries (row, chunk)
                    const int c = lane < ncode ? s_pcode[u0 * 2 + lane] : -1;
                    const unsigned long long full = (1ull << ncode) - 1ull;
                    const unsigned long long ev = full & 0x5555555555555555ull, od = full & 0xAAAAAAAAAAAAAAAAull;
                    const unsigned long long b1 = __ballot(c == 1), b0 = __ballot(c == 0);
                    ucs[0] = (b1 & ev) == ev ? 1 : ((b0 & ev) == ev ? 0 : -1);
                    ucs[1] = (b1 & od) == od ? 1 : ((b0 & od) == od ? 0 : -1);
                    if (!border && ucs[0] >= 0 && ucs[0] == ucs[1]) rc = ucs[0];
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
                        if (k >= 1 && k <= 3 && uy >= G::RU && uy < G::RU + G::FY && y < H && gw < A.WW) {
                            const int xs = gw * 32;
                            const uint32_t valid = (W - xs >= 32) ? ~0u : ((1u << (W - xs)) - 1u);
                            const uint32_t nw = word & valid;
                            const uint32_t ow = s_bits[(uy + 1 + R) * kFWords + k] & valid;
                            A.bits_out[(size_t)y * A.WW + gw] = nw;
                            flips += __popc(nw ^ ow);
                            dirs |= flip_dirs<G::FY, HWB>(uy - G::RU, k - 1, nw ^ ow);
                        }
                    }
                    continue;
                }
                constexpr int CG = (NV >= 4 && (V != 0 || R > 6)) ? 2 : kCG;
                static_assert(CG * kFWords <= 64, "one lane per staged word of a row group");
                // Rows in groups of CG (kCG; 2 for four bands in the 3- and
                // 5-wave variants and at R = 7: measured faster at 3 waves,
                // and elsewhere the loaded values of 4 rows exceed the
                // register budget):
                // gradients first (LDS), then every data-term load of the
                // group, then the updates, so that one memory round trip
                // serves the whole group.
                // Slots of a row group: one wave-wide pass each, over (row,
                // chunk) pairs, or in the edge term CG rows of chunk 0 and
                // CG / 2 packed row pairs of chunk 1.
                static_assert(!PK || CG % 2 == 0, "packed slots take row pairs");
                constexpr int NS = PK ? CG + CG / 2 : 2 * CG;
    #pragma unroll 1
                for (int r0 = 0; r0 < nr; r0 += CG) {
                    // The rows' ballots go to the lanes that form their words
                    // (lane L: word L % kFWords of row L / kFWords), which
                    // then write the whole group's words at once.
                    unsigned long long w0 = 0ull, w1 = 0ull;
                    if constexpr (PK) {
                        float phv[NS], gmv[NS];
                        bool need[NS], pred[NS];
                        Px<NV> v[NS];
                        int pixv[NS];
    #pragma unroll
                        for (int s = 0; s < NS; ++s) {
                            const int c = s >= CG ? 1 : 0;
                            // Row of the slot: per lane in a packed slot.
                            const int i = s < CG ? s : 2 * (s - CG) + hl;
                            const int uy = u0 + r0 + i;
                            const int y = y0 - G::RU + uy;
                            const bool rowok = r0 + i < nr && y >= 0 && y < H;
                            // Rows past U read phi row UH instead (in the array; the
                            // results are masked).  The y difference like the x one.
                            const float *prow = s_phi + (min(uy, G::UH - 1) + 1) * G::PS;
                            const float dr = y == 0 ? 1.f : (y == H - 1 ? 0.f : 0.5f);
                            const float ur = y == 0 ? 0.f : (y == H - 1 ? -1.f : -0.5f);
                            const float cr0 = y == 0 ? -1.f : (y == H - 1 ? 1.f : 0.f);
                            const int rowpix = y * W;
                            const bool ok = rowok && cok[c];
                            if (ucs[c] >= 0) {  // constant phi over this chunk's gradients
                                phv[s] = 0.f;
                                pred[s] = ok && ucs[c] == 1;
                                need[s] = false;
                                gmv[s] = 0.f;
                            } else {
                                // All five values are read (branch-free: lanes
                                // outside U read phi inside the array) and the
                                // image-border cases are weights, so the reads of
                                // a group are in flight together.
                                const float *cc = prow + ucol[c] + 1;
                                const float c0 = cc[0], cl = cc[-1], cr = cc[1], cu = cc[-G::PS], cd = cc[G::PS];
                                const float gx = fmaf(ar[c], cr, fmaf(al[c], cl, -(ar[c] + al[c]) * c0));
                                const float gy = fmaf(dr, cd, fmaf(ur, cu, cr0 * c0));
                                const float g2 = gx * gx + gy * gy;
                                phv[s] = c0;
                                pred[s] = ok && c0 >= 0.f;  // |grad phi| = 0: u = phi exactly (eq. (18))
                                need[s] = ok && g2 != 0.f;
                                // The hardware square root (within 1 ulp, one
                                // instruction instead of the ~15 of a correctly
                                // rounded one): it moves u by at most
                                // dt |R| |grad phi| 2^-23 < 3e-6, inside the band
                                // where FP32 cannot decide the sign like FP64.
                                gmv[s] = __builtin_amdgcn_sqrtf(g2);
                            }
                            const int pix = rowpix + x0 + ucol[c];
                            pixv[s] = pix;
                        }
    #pragma unroll
                        for (int s = 0; s < NS; ++s)
                            v[s] = buffer_px<ST, NV>(img_rs, need[s] ? (uint32_t)pixv[s] * PB : kNoLoad);
                        float coef[NS];
    #pragma unroll
                        for (int s = 0; s < NS; ++s) coef[s] = A.dt * v[s].v[0];
                        // A packed slot's ballot holds row 2j's chunk-1 bits in
                        // its low half and row 2j + 1's in its high half.
    #pragma unroll
                        for (int s = 0; s < NS; ++s) {
                            if (need[s]) pred[s] = fmaf(coef[s], gmv[s], phv[s]) >= 0.f;
                            const unsigned long long m = __ballot(pred[s]);
                            if (s >= CG) {
                                if ((wrow >> 1) == s - CG) w1 = (wrow & 1) ? m >> 32 : m & 0xffffffffull;
                            } else if (wrow == s) {
                                w0 = m;
                            }
                        }
                    } else {
                        float phv[CG][2], gmv[CG][2];
                        bool need[CG][2], pred[CG][2];
                        // Data term of each pixel: the region term (B values per pixel) loads
                        // it as soon as the pixel's gradient is known (fewer live registers,
                        // earlier loads); the edge term loads the group afterwards (measured
                        // faster there).
                        Px<NV> v[CG][2];
                        int pixv[CG][2];
    #pragma unroll
                        for (int i = 0; i < CG; ++i) {
                            // Row quantities are the same in every lane (scalar).
                            const int uy = u0 + r0 + i;
                            const int y = y0 - G::RU + uy;
                            const bool rowok = r0 + i < nr && y >= 0 && y < H;
                            // Rows past U read phi row UH instead (in the array; the
                            // results are masked).  The y difference like the x one.
                            const float *prow = s_phi + (min(uy, G::UH - 1) + 1) * G::PS;
                            const float dr = y == 0 ? 1.f : (y == H - 1 ? 0.f : 0.5f);
                            const float ur = y == 0 ? 0.f : (y == H - 1 ? -1.f : -0.5f);
                            const float cr0 = y == 0 ? -1.f : (y == H - 1 ? 1.f : 0.f);
                            const int rowpix = y * W;
    #pragma unroll
                            for (int c = 0; c < 2; ++c) {
                                const bool ok = rowok && cok[c];
                                if (EDGE && ucs[c] >= 0) {  // constant phi over this chunk's gradients
                                    phv[i][c] = 0.f;
                                    pred[i][c] = ok && ucs[c] == 1;
                                    need[i][c] = false;
                                    gmv[i][c] = 0.f;
                                } else {
                                    // All five values are read (branch-free: lanes
                                    // outside U read phi inside the array) and the
                                    // image-border cases are weights, so the reads of
                                    // a group are in flight together.
                                    const float *cc = prow + 64 * c + lane + 1;
                                    const float c0 = cc[0], cl = cc[-1], cr = cc[1], cu = cc[-G::PS], cd = cc[G::PS];
                                    const float gx = fmaf(ar[c], cr, fmaf(al[c], cl, -(ar[c] + al[c]) * c0));
                                    const float gy = fmaf(dr, cd, fmaf(ur, cu, cr0 * c0));
                                    const float g2 = gx * gx + gy * gy;
                                    phv[i][c] = c0;
                                    pred[i][c] = ok && c0 >= 0.f;  // |grad phi| = 0: u = phi exactly (eq. (18))
                                    need[i][c] = ok && g2 != 0.f;
                                    // The hardware square root (within 1 ulp, one
                                    // instruction instead of the ~15 of a correctly
                                    // rounded one): it moves u by at most
                                    // dt |R| |grad phi| 2^-23 < 3e-6, inside the band
                                    // where FP32 cannot decide the sign like FP64.
                                    gmv[i][c] = __builtin_amdgcn_sqrtf(g2);
                                }
                                const int pix = rowpix + cx0 + 64 * c;
                                pixv[i][c] = pix;
                                if constexpr (!EDGE)
                                    v[i][c] = buffer_px<ST, NV>(img_rs, need[i][c] ? (uint32_t)pix * PB : kNoLoad);
                            }
                        }
                        if constexpr (EDGE) {
    #pragma unroll
                            for (int i = 0; i < CG; ++i)
    #pragma unroll
                                for (int c = 0; c < 2; ++c)
                                    v[i][c] = buffer_px<ST, NV>(img_rs, need[i][c] ? (uint32_t)pixv[i][c] * PB : kNoLoad);
                        }
                        float coef[CG][2];
                        {
    #pragma unroll
                            for (int i = 0; i < CG; ++i)
    #pragma unroll
                                for (int c = 0; c < 2; ++c) {
                                    if constexpr (EDGE)
                                        coef[i][c] = A.dt * v[i][c].v[0];
                                    else
                                        coef[i][c] = w * region_D<NB>(v[i][c], a, m);
                                }
                        }
    #pragma unroll
                        for (int i = 0; i < CG; ++i) {
    #pragma unroll
                            for (int c = 0; c < 2; ++c)
                                if (need[i][c]) pred[i][c] = fmaf(coef[i][c], gmv[i][c], phv[i][c]) >= 0.f;
                            const unsigned long long m0 = __ballot(pred[i][0]);
                            const unsigned long long m1 = __ballot(pred[i][1]);
                            if (wrow == i) {
                                w0 = m0;
                                w1 = m1;
                            }
                        }
                    }
                    if (wrow < CG && r0 + wrow < nr) {
                        const int uy = u0 + r0 + wrow;
                        const int y = y0 - G::RU + uy;
                        const uint32_t word = bits_extract(w0, 32 - G::RU, wk) | bits_extract(w1, 96 - G::RU, wk);
                        s_bn[uy * kFWords + wk] = word;
                        const int gw = (x0 >> 5) - 1 + wk;
                        if (wk >= 1 && wk <= 3 && uy >= G::RU && uy < G::RU + G::FY && y >= 0 && y < H && gw < A.WW) {
                            const int xs = gw * 32;
                            const uint32_t valid = (W - xs >= 32) ? ~0u : ((1u << (W - xs)) - 1u);
                            const uint32_t nw = word & valid;
                            const uint32_t ow = s_bits[(uy + 1 + R) * kFWords + wk] & valid;
                            A.bits_out[(size_t)y * A.WW + gw] = nw;
                            flips += __popc(nw ^ ow);
                            dirs |= flip_dirs<G::FY, HWB>(uy - G::RU, wk - 1, nw ^ ow);
                        }
                    }
                }
            }
            if (dirs) atomicOr(&s_dirs, dirs);
            __syncthreads();

            float acc[NB];
    #pragma unroll
            for (int b = 0; b < NB; ++b) acc[b] = 0.f;
            int cnt = 0;
            if constexpr (!EDGE) {
                // D: statistics of phi^{n+1} = G * b^n for the next iteration.
                code_rows_owned<R>(s_bn, G::UH, s_codes);
                __syncthreads();
                // Groups of 6 image rows (a 24-row segment in about two memory
                // round trips instead of three) where the register budget
                // allows it: at 5 waves per SIMD they spill.
                constexpr int GRD = (StepVariant<EDGE, V>::OCC <= 4 && G::SEGD % 12 == 0) ? 6 : 4;
                stats_fast<R, NB, ST, GRD>(s_bn, s_codes, static_cast<const ST *>(A.img), x0, y0, H, W, border, false,
                                      lut, kk, cum, acc, cnt);
            }
            TileSmem rs;
            rs.red = red;
            reduce_commit<NB>(rs, acc, cnt, flips, &st->slot[sbn][blockIdx.x % kBins], A.fix, !EDGE,
                              track ? &s_prev : nullptr, track ? &E.tilelast[t] : nullptr);
            // Touched neighbours: the next iteration visits them.
            if (tid == 0 && s_dirs && E.sched_mask)
                mark_touched(E.sched_mask, nw, t, ntx, E.tiles / ntx, s_dirs, touch_tag(n));
        }
    }
    if (lead_block) {
        // Clear the slot of iteration n + 2 and the schedule mask that
        // iteration n + 1 will fill (nobody reads or writes them now).
        unsigned long long *z = reinterpret_cast<unsigned long long *>(&st->slot[(A.n + 2) % 3][0]);
        for (int i = threadIdx.x; i < (int)(kBins * sizeof(Bin) / 8); i += kThreads) z[i] = 0ull;
        if (E.sched_mask)
            for (int i = threadIdx.x; i < nw; i += kThreads) E.sched_mask[(size_t)sbr * nw + i] = 0u;
    }
    if constexpr (!EDGE && NB > 1)
        if (lead) record_max_pixel<NB, ST>(st, sl, tot.mkey, A.img, A.hw);
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

// Region sums of each step tile in the all-inside case, through the step
// kernel's own statistics code and reduction (stats_fast with every pixel on
// the + side, block_reduce), converted to fixed point as the step would.
template <int R, int NB, typename ST>
__global__ __launch_bounds__(kThreads) void tile_sums_kernel(const ImgArgs *__restrict__ args,
                                                             TileSum *__restrict__ out) {
    extern __shared__ float smem[];
    __shared__ float red[kThreads / 64 * 8];
    using G = FastGeom<R, false>;
    const ImgArgs &E = args[0];
    const int t = blockIdx.x;
    const int ntx = (E.W + kFX - 1) / kFX;
    const int x0 = (t % ntx) * kFX, y0 = (t / ntx) * G::FY;
    const bool border = x0 - 2 * R - 2 < 0 || x0 + kFX + 2 * R + 2 > E.W;
    uint32_t *s_bn = reinterpret_cast<uint32_t *>(smem);
    for (int i = threadIdx.x; i < G::UH * kFWords; i += kThreads) s_bn[i] = ~0u;
    LutRegs<G::NCH> lut;
    load_luts<G::NCH>(E.taps, lut);
    float kk[2 * R + 1];
#pragma unroll
    for (int i = 0; i < 2 * R + 1; ++i) kk[i] = E.taps->k[i];
    __syncthreads();
    float acc[NB];
    int cnt;
    stats_fast<R, NB, ST>(s_bn, nullptr, static_cast<const ST *>(E.img), x0, y0, E.H, E.W, border, true, lut, kk,
                          E.taps->cum, acc, cnt);
    TileSmem rs;
    rs.red = red;
    float S[NB];
    int C, F;
    block_reduce<NB>(rs, acc, cnt, 0, true, S, C, F);
    if (threadIdx.x == 0) {
        TileSum v;
#pragma unroll
        for (int b = 0; b < 4; ++b) v.sum[b] = b < NB ? __float2ll_rn(S[b] * E.fix) : 0;
        v.cnt = C;
        v.pad[0] = v.pad[1] = v.pad[2] = 0;
        out[t] = v;
    }
}

// Region statistics on the fast tiling (used at init and by set_mask so that
// its partial sums equal the step kernel's bit for bit).
template <int R, int NB, typename ST>
__global__ __launch_bounds__(kThreads) void stats_fast_kernel(StepArgs A, int raw, int slot) {
    extern __shared__ float smem[];
    __shared__ float red[kThreads / 64 * 8];
    using G = FastGeom<R, false>;
    uint32_t *s_bn = reinterpret_cast<uint32_t *>(smem);
    const int x0 = blockIdx.x * kFX, y0 = blockIdx.y * G::FY;
    const bool border = x0 - 2 * R - 2 < 0 || x0 + kFX + 2 * R + 2 > A.W;
    LutRegs<G::NCH> lut;
    load_luts<G::NCH>(A.taps, lut);
    float kk[2 * R + 1];
#pragma unroll
    for (int i = 0; i < 2 * R + 1; ++i) kk[i] = A.taps->k[i];
    int *s_codes = reinterpret_cast<int *>(s_bn + G::UH * kFWords);
    stage_bits_fast<G::UH>(s_bn, A.bits_in, y0 - R, x0, A.H, A.WW);
    __syncthreads();
    code_rows_owned<R>(s_bn, G::UH, s_codes);
    __syncthreads();
    float acc[NB];
    int cnt;
    stats_fast<R, NB, ST>(s_bn, s_codes, static_cast<const ST *>(A.img), x0, y0, A.H, A.W, border, raw != 0,
                          lut, kk, A.taps->cum, acc, cnt);
    TileSmem rs;
    rs.red = red;
    reduce_commit<NB>(rs, acc, cnt, 0, &A.st->slot[slot][block_linear_id() % kBins], A.fix, true, nullptr,
                      A.tilelast ? &A.tilelast[blockIdx.y * gridDim.x + blockIdx.x] : nullptr);
}

// ------------------------------------------------------ continuous LSF
//
// Step orders and reinitialisation schedules other than "binarise every
// iteration, then smooth" keep a continuous LSF, stored as a plane of the
// storage type.  One iteration on a 64 x 32 tile:
//   1. phi^n on the tile plus an r+1 halo (from the plane, or +-1 from the bit
//      plane when phi^n is a binary function: the initial LSF of eq. (13), or
//      the sign of the field stored by a listing-order iteration);
//   2. u = phi^n + dt R |grad phi^n| (eq. (18)) on the tile plus an r halo,
//      binarised there when Table I step 3 applies in this iteration;
//   3. the separable Gaussian of that field (zero padding): psi on the tile;
//   4. the stored field is psi (the LSF, or in listing order with
//      binarisation the pre-sign field whose sign is the LSF);
//   5. the binary result b^n (sign of u after step 3, else sign of the new
//      LSF) as bit words, flips against b^{n-1}, and the region statistics of
//      the new LSF for the next iteration.
// The new LSF's sign is taken from the value as stored (after rounding to the
// storage type), so the statistics describe what the next iteration reads.

struct DenseSmem {
    float *P, *U, *Hh, *k, *red;
};

__host__ __device__ inline size_t dense_smem_words(int r) {
    const size_t PH = kTileY + 2 * r + 2, PW = kTileX + 2 * r + 2;
    const size_t UH = kTileY + 2 * r, UW = kTileX + 2 * r;
    return PH * PW + UH * UW + UH * kTileX + 32 + 32;
}

__device__ __forceinline__ DenseSmem dense_carve(float *smem, int r) {
    const int PH = kTileY + 2 * r + 2, PW = kTileX + 2 * r + 2;
    const int UH = kTileY + 2 * r, UW = kTileX + 2 * r;
    DenseSmem d;
    d.P = smem;
    d.U = d.P + PH * PW;
    d.Hh = d.U + UH * UW;
    d.k = d.Hh + UH * kTileX;
    d.red = d.k + 32;
    return d;
}

template <int NB, bool EDGE, typename ST>
__global__ __launch_bounds__(kThreads) void dense_step_kernel(StepArgs A) {
    extern __shared__ float smem[];
    __shared__ Totals tot;
    DevState *st = A.st;
    const int sl = A.n % 3;
    const bool lead_block = blockIdx.x == 0 && blockIdx.y == 0;
    const bool lead = lead_block && threadIdx.x == 0;
    load_totals(st, sl, !EDGE, &tot);
    {
        int done = tot.done | tot.bad;
        if (!done && A.stop && tot.flips == 0) done = 1;
        if (done) {
            if (lead && !tot.bad) st->done = 1;
            return;
        }
    }
    const int r = A.r, ts = A.ts, H = A.H, W = A.W;
    const int PH = kTileY + 2 * r + 2, PW = kTileX + 2 * r + 2;
    const int UH = kTileY + 2 * r, UW = kTileX + 2 * r;
    const int x0 = blockIdx.x * kTileX, y0 = blockIdx.y * kTileY;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const DenseSmem d = dense_carve(smem, r);
    const ST *plane_in = static_cast<const ST *>(A.plane_in);
    ST *plane_out = static_cast<ST *>(A.plane_out);
    const bool listing = A.order == LSE_ORDER_LISTING;
    const bool bin_u = !listing && A.reinit;   // Table I step 3 in this iteration

    // 1: phi^n on rows y0 - r - 1 .., columns x0 - r - 1 ..
    for (int i = tid; i < ts; i += kThreads) d.k[i] = A.taps->k[i];
    for (int i = tid; i < PH * PW; i += kThreads) {
        const int q = i / PW, p = i - q * PW;
        const int y = y0 - r - 1 + q, x = x0 - r - 1 + p;
        float v = 0.f;
        if (y >= 0 && y < H && x >= 0 && x < W) {
            if (A.phi_binary)
                v = ((A.bits_in[(size_t)y * A.WW + (x >> 5)] >> (x & 31)) & 1u) ? 1.f : -1.f;
            else
                v = to_f32<ST>(plane_in[(size_t)y * W + x]);
        }
        d.P[i] = v;
    }
    // Data-term coefficients.
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
    __syncthreads();

    // 2: u (or its sign) on the tile plus an r halo; zero outside the image.
    for (int i = tid; i < UH * UW; i += kThreads) {
        const int uy = i / UW, ux = i - uy * UW;
        const int y = y0 - r + uy, x = x0 - r + ux;
        float v = 0.f;
        if (y >= 0 && y < H && x >= 0 && x < W) {
            const float *c = d.P + (uy + 1) * PW + (ux + 1);
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
            float u = c[0];
            if (!(gx == 0.f && gy == 0.f)) {
                const long long pix = (long long)y * W + x;
                const float gm = sqrtf(gx * gx + gy * gy);
                float coef;
                if constexpr (EDGE)
                    coef = A.dt * to_f32<ST>(static_cast<const ST *>(A.img)[pix]);
                else
                    coef = w * region_D<NB>(load_px<ST, NB>(static_cast<const ST *>(A.img), pix), a, m);
                u = fmaf(coef, gm, u);
            }
            v = bin_u ? (u >= 0.f ? 1.f : -1.f) : u;
        }
        d.U[i] = v;
    }
    __syncthreads();

    // 3: horizontal then vertical Gaussian (taps in order, FMA).
    for (int i = tid; i < UH * kTileX; i += kThreads) {
        const int uy = i / kTileX, ox = i - uy * kTileX;
        const float *row = d.U + uy * UW + ox;
        float h = 0.f;
        for (int j = 0; j < ts; ++j) h = fmaf(d.k[j], row[j], h);
        d.Hh[i] = h;
    }
    __syncthreads();

    // 4-5: store, binary result, statistics of the new LSF.
    float acc[NB];
#pragma unroll
    for (int b = 0; b < NB; ++b) acc[b] = 0.f;
    int cnt = 0, flips = 0;
    bool overflow = false;
    for (int row = wave; row < kTileY; row += kThreads / 64) {
        const int y = y0 + row, x = x0 + lane;
        const bool ok = y < H && x < W;
        bool bit = false, inside = false;
        if (ok) {
            float psi = 0.f;
            const float *col = d.Hh + row * kTileX + lane;
            for (int i = 0; i < ts; ++i) psi = fmaf(d.k[i], col[i * kTileX], psi);
            const ST q = from_f32<ST>(psi);
            plane_out[(size_t)y * W + x] = q;
            const float stored = to_f32<ST>(q);
            overflow |= !isfinite(stored);
            // The next iteration's LSF: sign(psi) in listing order with
            // binarisation (read from the bit plane), else the stored value.
            inside = (listing && A.reinit) ? psi >= 0.f : stored >= 0.f;
            bit = bin_u ? d.U[(row + r) * UW + lane + r] > 0.f : inside;
            if constexpr (!EDGE) {
                if (inside) {
                    const Px<NB> p = load_px<ST, NB>(static_cast<const ST *>(A.img), (long long)y * W + x);
#pragma unroll
                    for (int b = 0; b < NB; ++b) acc[b] += p.v[b];
                    ++cnt;
                }
            }
        }
        const unsigned long long bal = __ballot(bit);
        if (lane < 2) {
            const int gw = (x0 >> 5) + lane;
            if (y < H && gw < A.WW) {
                const int xs = gw * 32;
                const uint32_t valid = (W - xs >= 32) ? ~0u : ((1u << (W - xs)) - 1u);
                const uint32_t nw = (uint32_t)(bal >> (32 * lane)) & valid;
                const uint32_t ow = A.bits_in[(size_t)y * A.WW + gw] & valid;
                A.bits_out[(size_t)y * A.WW + gw] = nw;
                flips += __popc(nw ^ ow);
            }
        }
    }
    // Without binarisation the LSF can grow until it leaves the range of the
    // storage type; such a state is flagged and stops the iteration.
    if (__any(overflow) && lane == 0) st->bad = kBadOverflow;
    TileSmem rs;
    rs.red = d.red;
    reduce_commit<NB>(rs, acc, cnt, flips, &st->slot[(A.n + 1) % 3][block_linear_id() % kBins], A.fix, !EDGE);
    if (lead_block) {
        unsigned long long *z = reinterpret_cast<unsigned long long *>(&st->slot[(A.n + 2) % 3][0]);
        for (int i = threadIdx.x; i < (int)(kBins * sizeof(Bin) / 8); i += kThreads) z[i] = 0ull;
    }
    if constexpr (!EDGE && NB > 1)
        if (lead) record_max_pixel<NB, ST>(st, sl, tot.mkey, A.img, A.hw);
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

// LSF plane from the binary function: +-1 (raw) or its Gaussian smoothing
// (the same tile arithmetic as the LSF export), rounded to the storage type.
template <typename ST>
__global__ __launch_bounds__(kThreads) void plane_fill_kernel(StepArgs A, const uint32_t *__restrict__ bits, int raw,
                                                              ST *__restrict__ plane) {
    extern __shared__ float smem[];
    const TileSmem s = carve(smem, A.r, A.nch, 0);
    const int x0 = blockIdx.x * kTileX, y0 = blockIdx.y * kTileY;
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
            plane[(size_t)y * A.W + x] = from_f32<ST>(v);
        }
    }
}

// Region statistics (eq. (15)) of the LSF stored in a plane.
template <int NB, typename ST>
__global__ __launch_bounds__(kThreads) void plane_stats_kernel(StepArgs A, const ST *__restrict__ plane, int slot) {
    __shared__ float red[kThreads / 64 * 8];
    const int x0 = blockIdx.x * kTileX, y0 = blockIdx.y * kTileY;
    float acc[NB];
#pragma unroll
    for (int b = 0; b < NB; ++b) acc[b] = 0.f;
    int cnt = 0;
    for (int k = 0; k < (kTileX * kTileY) / kThreads; ++k) {
        const int i = threadIdx.x + k * kThreads;
        const int oy = i / kTileX, ox = i - oy * kTileX;
        const int y = y0 + oy, x = x0 + ox;
        if (y < A.H && x < A.W && to_f32<ST>(plane[(size_t)y * A.W + x]) >= 0.f) {
            const Px<NB> p = load_px<ST, NB>(static_cast<const ST *>(A.img), (long long)y * A.W + x);
#pragma unroll
            for (int b = 0; b < NB; ++b) acc[b] += p.v[b];
            ++cnt;
        }
    }
    TileSmem rs;
    rs.red = red;
    reduce_commit<NB>(rs, acc, cnt, 0, &A.st->slot[slot][block_linear_id() % kBins], A.fix, true);
}

// The stored field as FP32: plane (iterations executed) & 1 holds it.
template <typename ST>
__global__ void plane_out_kernel(const ST *__restrict__ p0, const ST *__restrict__ p1, const DevState *st,
                                 float *__restrict__ out, long long n) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const ST *plane = (st->iters & 1) ? p1 : p0;
    if (i < n) out[i] = to_f32<ST>(plane[i]);
}

// ---------------------------------------------------------------- launchers

template <int R, int NB, bool EDGE, typename ST, int V>
static hipError_t launch_step_fast_v(const ImgArgs *args, const uint32_t *map, const int *nmap, int unit_bits,
                                     unsigned grid, int k, int stop, hipStream_t s) {
    const size_t sm = (size_t)FastGeom<R, EDGE, StepVariant<EDGE, V>::FY>::smem_words * 4;
    const hipError_t e = ensure_lds(step_fast_kernel<R, NB, EDGE, ST, V>, sm);
    if (e != hipSuccess) return e;
    return launch_timed(step_fast_kernel<R, NB, EDGE, ST, V>, dim3(grid), dim3(kThreads), (uint32_t)sm, s, args, map,
                        nmap, unit_bits, k, stop);
}

template <int R, int NB, bool EDGE, typename ST>
static hipError_t launch_step_fast_t(const ImgArgs *args, const uint32_t *map, const int *nmap, int unit_bits,
                                     unsigned grid, int k, int stop, int variant, hipStream_t s) {
    static_assert(kStepVariants == 3, "one case per variant");
    switch (variant) {
        case 0: return launch_step_fast_v<R, NB, EDGE, ST, 0>(args, map, nmap, unit_bits, grid, k, stop, s);
        case 1: return launch_step_fast_v<R, NB, EDGE, ST, 1>(args, map, nmap, unit_bits, grid, k, stop, s);
        case 2: return launch_step_fast_v<R, NB, EDGE, ST, 2>(args, map, nmap, unit_bits, grid, k, stop, s);
    }
    return hipErrorInvalidValue;
}

template <int R, typename ST>
static hipError_t launch_step_fast_r(const ImgArgs *args, const uint32_t *map, const int *nmap, int unit_bits,
                                     unsigned grid, int k, int stop, int NB, int edge, int variant, hipStream_t s) {
    if (edge) return launch_step_fast_t<R, 1, true, ST>(args, map, nmap, unit_bits, grid, k, stop, variant, s);
    switch (NB) {
        case 1: return launch_step_fast_t<R, 1, false, ST>(args, map, nmap, unit_bits, grid, k, stop, variant, s);
        case 2: return launch_step_fast_t<R, 2, false, ST>(args, map, nmap, unit_bits, grid, k, stop, variant, s);
        case 4: return launch_step_fast_t<R, 4, false, ST>(args, map, nmap, unit_bits, grid, k, stop, variant, s);
    }
    return hipErrorInvalidValue;
}

template <int R, int NB, typename ST>
static hipError_t launch_stats_fast_t(const StepArgs &a, int raw, int slot, hipStream_t s) {
    const size_t sm = (size_t)FastGeom<R, false>::UH * (kFWords + 2) * 4;
    const dim3 grid((a.W + kFX - 1) / kFX, (a.H + kFYRegion - 1) / kFYRegion);
    hipLaunchKernelGGL((stats_fast_kernel<R, NB, ST>), grid, dim3(kThreads), sm, s, a, raw, slot);
    return hipGetLastError();
}

template <int R, typename ST>
static hipError_t launch_stats_fast_r(const StepArgs &a, int NB, int raw, int slot, hipStream_t s) {
    switch (NB) {
        case 1: return launch_stats_fast_t<R, 1, ST>(a, raw, slot, s);
        case 2: return launch_stats_fast_t<R, 2, ST>(a, raw, slot, s);
        case 4: return launch_stats_fast_t<R, 4, ST>(a, raw, slot, s);
    }
    return hipErrorInvalidValue;
}

template <int NB, typename ST>
static hipError_t launch_stats_generic_t(const StepArgs &a, int raw, int slot, hipStream_t s) {
    const size_t sm = tile_smem_bytes(a.r, a.nch, 0);
    const hipError_t e = ensure_lds(stats_kernel<NB, ST>, sm);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((stats_kernel<NB, ST>), tile_grid(a.H, a.W), dim3(kThreads), sm, s, a, raw, slot);
    return hipGetLastError();
}

template <int NB, bool EDGE, typename ST>
static hipError_t launch_step_generic_t(const StepArgs &a, hipStream_t s) {
    const size_t sm = tile_smem_bytes(a.r, a.nch, EDGE ? 1 : 0);
    const hipError_t e = ensure_lds(step_kernel<NB, EDGE, ST>, sm);
    if (e != hipSuccess) return e;
    return launch_timed(step_kernel<NB, EDGE, ST>, tile_grid(a.H, a.W), dim3(kThreads), (uint32_t)sm, s, a);
}

template <typename ST>
hipError_t Store<ST>::init_image(const void *src, int src_dtype, int B, int NB, void *dst, long long npx,
                                 DevState *st, float fix, int mode, hipStream_t s) {
    const dim3 grid(stream_blocks(npx, 4)), block(kThreads);
    ST *d = static_cast<ST *>(dst);
    switch (src_dtype) {
        case LSE_F32:
            hipLaunchKernelGGL((init_image_kernel<float, ST>), grid, block, 0, s, static_cast<const float *>(src), B,
                               NB, d, npx, st, fix, mode);
            break;
        case LSE_F16:
            hipLaunchKernelGGL((init_image_kernel<__half, ST>), grid, block, 0, s, static_cast<const __half *>(src),
                               B, NB, d, npx, st, fix, mode);
            break;
        case LSE_BF16:
            hipLaunchKernelGGL((init_image_kernel<__hip_bfloat16, ST>), grid, block, 0, s,
                               static_cast<const __hip_bfloat16 *>(src), B, NB, d, npx, st, fix, mode);
            break;
        default:
            return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <typename ST>
template <typename T>
hipError_t Store<ST>::edge_map_t(const T *src, int B, float scale, const Taps *taps, int r1, ST *g, int H, int W,
                                 DevState *st, hipStream_t s) {
    const dim3 grid((W + kEMX - 1) / kEMX, (H + kEMY - 1) / kEMY);
    const size_t sm = edge_map_smem_bytes(r1);
    if (B == 4 && (reinterpret_cast<uintptr_t>(src) % (4 * sizeof(T))) == 0) {
        const hipError_t e = ensure_lds(edge_map_kernel<T, ST, true>, sm);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL((edge_map_kernel<T, ST, true>), grid, dim3(kThreads), sm, s, src, B, scale, taps, r1, g, H,
                           W, st);
    } else {
        const hipError_t e = ensure_lds(edge_map_kernel<T, ST, false>, sm);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL((edge_map_kernel<T, ST, false>), grid, dim3(kThreads), sm, s, src, B, scale, taps, r1, g,
                           H, W, st);
    }
    return hipGetLastError();
}

template <typename ST>
hipError_t Store<ST>::edge_map(const void *src, int src_dtype, int B, float scale, const Taps *taps, int r1, void *g,
                               int H, int W, DevState *st, hipStream_t s) {
    ST *out = static_cast<ST *>(g);
    switch (src_dtype) {
        case LSE_F32: return edge_map_t(static_cast<const float *>(src), B, scale, taps, r1, out, H, W, st, s);
        case LSE_F16: return edge_map_t(static_cast<const __half *>(src), B, scale, taps, r1, out, H, W, st, s);
        case LSE_BF16:
            return edge_map_t(static_cast<const __hip_bfloat16 *>(src), B, scale, taps, r1, out, H, W, st, s);
    }
    return hipErrorInvalidValue;
}

template <typename ST>
template <typename T>
hipError_t Store<ST>::init_image_box_t(const T *src, int B, int NB, ST *dst, int H, int W, DevState *st, float fix,
                                       float *boxes, hipStream_t s) {
    const int nblk = ((W + kMBX - 1) / kMBX) * ((H + kMBY - 1) / kMBY);
    const dim3 grid((unsigned)((nblk + kIBoxBlocks - 1) / kIBoxBlocks)), block(kThreads);
    const bool v4 = B == 4 && (reinterpret_cast<uintptr_t>(src) % (4 * sizeof(T))) == 0;
    if (NB == 4) {
        if (v4)
            hipLaunchKernelGGL((init_image_box_kernel<T, ST, 4, true>), grid, block, 0, s, src, B, dst, H, W, st, fix, boxes);
        else
            hipLaunchKernelGGL((init_image_box_kernel<T, ST, 4, false>), grid, block, 0, s, src, B, dst, H, W, st, fix,
                               boxes);
    } else if (NB == 2) {
        hipLaunchKernelGGL((init_image_box_kernel<T, ST, 2, false>), grid, block, 0, s, src, B, dst, H, W, st, fix, boxes);
    } else {
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <typename ST>
hipError_t Store<ST>::init_image_box(const void *src, int src_dtype, int B, int NB, void *dst, int H, int W,
                                     DevState *st, float fix, float *boxes, hipStream_t s) {
    ST *d = static_cast<ST *>(dst);
    switch (src_dtype) {
        case LSE_F32: return init_image_box_t(static_cast<const float *>(src), B, NB, d, H, W, st, fix, boxes, s);
        case LSE_F16: return init_image_box_t(static_cast<const __half *>(src), B, NB, d, H, W, st, fix, boxes, s);
        case LSE_BF16:
            return init_image_box_t(static_cast<const __hip_bfloat16 *>(src), B, NB, d, H, W, st, fix, boxes, s);
    }
    return hipErrorInvalidValue;
}

// The statistics kernel uses the same tiling as the step kernel that would
// have produced the statistics, so that resumed runs match bit for bit.
template <typename ST>
hipError_t Store<ST>::stats(const StepArgs &a, int NB, int raw, int slot, hipStream_t s) {
    switch (a.r) {
        case 3: return launch_stats_fast_r<3, ST>(a, NB, raw, slot, s);
        case 4: return launch_stats_fast_r<4, ST>(a, NB, raw, slot, s);
        case 5: return launch_stats_fast_r<5, ST>(a, NB, raw, slot, s);
        case 6: return launch_stats_fast_r<6, ST>(a, NB, raw, slot, s);
        case 7: return launch_stats_fast_r<7, ST>(a, NB, raw, slot, s);
        default: break;
    }
    switch (NB) {
        case 1: return launch_stats_generic_t<1, ST>(a, raw, slot, s);
        case 2: return launch_stats_generic_t<2, ST>(a, raw, slot, s);
        case 4: return launch_stats_generic_t<4, ST>(a, raw, slot, s);
    }
    return hipErrorInvalidValue;
}

template <typename ST>
hipError_t Store<ST>::step(const ImgArgs *args, const uint32_t *map, const int *nmap, int unit_bits, unsigned grid,
                           int k, int stop, int r, int NB, int edge, int variant, hipStream_t s) {
    switch (r) {
        case 3: return launch_step_fast_r<3, ST>(args, map, nmap, unit_bits, grid, k, stop, NB, edge, variant, s);
        case 4: return launch_step_fast_r<4, ST>(args, map, nmap, unit_bits, grid, k, stop, NB, edge, variant, s);
        case 5: return launch_step_fast_r<5, ST>(args, map, nmap, unit_bits, grid, k, stop, NB, edge, variant, s);
        case 6: return launch_step_fast_r<6, ST>(args, map, nmap, unit_bits, grid, k, stop, NB, edge, variant, s);
        case 7: return launch_step_fast_r<7, ST>(args, map, nmap, unit_bits, grid, k, stop, NB, edge, variant, s);
    }
    return hipErrorInvalidValue;
}

template <typename ST>
hipError_t Store<ST>::step_generic(const StepArgs &a, int NB, int edge, hipStream_t s) {
    if (edge) return launch_step_generic_t<1, true, ST>(a, s);
    switch (NB) {
        case 1: return launch_step_generic_t<1, false, ST>(a, s);
        case 2: return launch_step_generic_t<2, false, ST>(a, s);
        case 4: return launch_step_generic_t<4, false, ST>(a, s);
    }
    return hipErrorInvalidValue;
}

template <typename ST>
hipError_t Store<ST>::mpass(const ImgArgs *args, const uint32_t *map, int unit_bits, unsigned grid, int k, int stop,
                            int NB, hipStream_t s) {
    switch (NB) {
        case 2: return launch_timed(mpass_kernel<2, ST>, dim3(grid), dim3(kThreads), 0u, s, args, map, unit_bits, k, stop);
        case 4: return launch_timed(mpass_kernel<4, ST>, dim3(grid), dim3(kThreads), 0u, s, args, map, unit_bits, k, stop);
    }
    return hipErrorInvalidValue;
}

template <int NB, bool EDGE, typename ST>
static hipError_t launch_dense_t(const StepArgs &a, hipStream_t s) {
    const size_t sm = dense_smem_words(a.r) * 4;
    const hipError_t e = ensure_lds(dense_step_kernel<NB, EDGE, ST>, sm);
    if (e != hipSuccess) return e;
    return launch_timed(dense_step_kernel<NB, EDGE, ST>, tile_grid(a.H, a.W), dim3(kThreads), (uint32_t)sm, s, a);
}

template <typename ST>
hipError_t Store<ST>::dense_step(const StepArgs &a, int NB, int edge, hipStream_t s) {
    if (edge) return launch_dense_t<1, true, ST>(a, s);
    switch (NB) {
        case 1: return launch_dense_t<1, false, ST>(a, s);
        case 2: return launch_dense_t<2, false, ST>(a, s);
        case 4: return launch_dense_t<4, false, ST>(a, s);
    }
    return hipErrorInvalidValue;
}

template <typename ST>
hipError_t Store<ST>::plane_fill(const StepArgs &a, const uint32_t *bits, int raw, void *plane, hipStream_t s) {
    const size_t sm = tile_smem_bytes(a.r, a.nch, 0);
    const hipError_t e = ensure_lds(plane_fill_kernel<ST>, sm);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((plane_fill_kernel<ST>), tile_grid(a.H, a.W), dim3(kThreads), sm, s, a, bits, raw,
                       static_cast<ST *>(plane));
    return hipGetLastError();
}

template <typename ST>
hipError_t Store<ST>::plane_stats(const StepArgs &a, const void *plane, int NB, int slot, hipStream_t s) {
    const ST *p = static_cast<const ST *>(plane);
    switch (NB) {
        case 1: hipLaunchKernelGGL((plane_stats_kernel<1, ST>), tile_grid(a.H, a.W), dim3(kThreads), 0, s, a, p, slot); break;
        case 2: hipLaunchKernelGGL((plane_stats_kernel<2, ST>), tile_grid(a.H, a.W), dim3(kThreads), 0, s, a, p, slot); break;
        case 4: hipLaunchKernelGGL((plane_stats_kernel<4, ST>), tile_grid(a.H, a.W), dim3(kThreads), 0, s, a, p, slot); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <int R, int NB, typename ST>
static hipError_t launch_tile_sums_t(const ImgArgs *args, int tiles, TileSum *out, hipStream_t s) {
    const size_t sm = (size_t)FastGeom<R, false>::UH * kFWords * 4;
    hipLaunchKernelGGL((tile_sums_kernel<R, NB, ST>), dim3((unsigned)tiles), dim3(kThreads), sm, s, args, out);
    return hipGetLastError();
}

template <int R, typename ST>
static hipError_t launch_tile_sums_r(const ImgArgs *args, int tiles, int NB, TileSum *out, hipStream_t s) {
    switch (NB) {
        case 1: return launch_tile_sums_t<R, 1, ST>(args, tiles, out, s);
        case 2: return launch_tile_sums_t<R, 2, ST>(args, tiles, out, s);
        case 4: return launch_tile_sums_t<R, 4, ST>(args, tiles, out, s);
    }
    return hipErrorInvalidValue;
}

template <typename ST>
hipError_t Store<ST>::tile_sums(const ImgArgs *args, int tiles, int r, int NB, TileSum *out, hipStream_t s) {
    if (tiles <= 0) return hipSuccess;
    switch (r) {
        case 3: return launch_tile_sums_r<3, ST>(args, tiles, NB, out, s);
        case 4: return launch_tile_sums_r<4, ST>(args, tiles, NB, out, s);
        case 5: return launch_tile_sums_r<5, ST>(args, tiles, NB, out, s);
        case 6: return launch_tile_sums_r<6, ST>(args, tiles, NB, out, s);
        case 7: return launch_tile_sums_r<7, ST>(args, tiles, NB, out, s);
    }
    return hipErrorInvalidValue;
}

// A caller's FP32 LSF into a plane of the storage type (round to nearest); a
// value that is not finite after the rounding marks the state as overflowed.
template <typename ST>
__global__ void plane_load_kernel(const float *__restrict__ src, ST *__restrict__ dst, long long n, DevState *st) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    bool bad = false;
    if (i < n) {
        const ST q = from_f32<ST>(src[i]);
        dst[i] = q;
        bad = !isfinite(to_f32<ST>(q));
    }
    if (__any(bad) && (threadIdx.x & 63) == 0) st->bad = kBadOverflow;
}

template <typename ST>
hipError_t Store<ST>::plane_load(const float *src, void *dst, long long n, DevState *st, hipStream_t s) {
    hipLaunchKernelGGL((plane_load_kernel<ST>), dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, src,
                       static_cast<ST *>(dst), n, st);
    return hipGetLastError();
}

template <typename ST>
hipError_t Store<ST>::plane_out(const void *p0, const void *p1, const DevState *st, float *out, long long n,
                                hipStream_t s) {
    hipLaunchKernelGGL((plane_out_kernel<ST>), dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s,
                       static_cast<const ST *>(p0), static_cast<const ST *>(p1), st, out, n);
    return hipGetLastError();
}

}  // namespace lse
