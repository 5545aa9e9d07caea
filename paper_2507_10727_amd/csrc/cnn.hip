// Learned preconditioner kernels: BF16 MFMA 3x3 convolutions (forward, data
// gradient, weight gradient), pooling and upsampling with their adjoints,
// the preconditioner's input and output maps, the training loss and Adam.
//
// MFMA v_mfma_f32_16x16x32_bf16 (CDNA4) computes D = A B + C for a 16x32 A
// and a 32x16 B; lane l (of 64) holds A[l % 16][8 (l / 16) + j] and
// B[8 (l / 16) + j][l % 16], j = 0..7, and D[4 (l / 16) + i][l % 16],
// i = 0..3.
//
// Convolution as an implicit GEMM: A = weights (rows = output channels),
// B = the input patch (rows k = tap * cin_p + c, columns = pixels), so a lane
// ends with 4 consecutive output channels of one pixel: one 16-byte NHWC
// store.  The image is cut into column bands about 64 wide; a block takes
// 256 consecutive pixels of a band in row-major order (4 waves of 4 groups
// of 16), so grids of 2^k + 1 columns leave no block nearly empty.  The
// block's input patch (the band rows it touches plus a one-node halo, BF16,
// channel-contiguous with a 4-short pad per pixel so that the 16 lanes'
// 8-byte reads fall in distinct banks) is staged in LDS once and read by
// every k step.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "cnn.h"

namespace pic {

namespace {

typedef short v4s __attribute__((ext_vector_type(4)));
typedef short v8s __attribute__((ext_vector_type(8)));
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));
typedef float v4f __attribute__((ext_vector_type(4)));

constexpr int TR = 4;            // weight gradient: rows per pixel tile (one per wave)
constexpr int TX = 64;           // weight gradient: columns per pixel tile
constexpr int CONV_PIX = 256;    // forward / data gradient: pixels per block
constexpr int BAND_MAX = 72;     // widest column band
constexpr int PW = TX + 2;       // patch columns
constexpr int PH = TR + 2;       // patch rows
constexpr int EB = 256;          // threads of elementwise kernels
constexpr int CONV_LDS_MAX = 150 * 1024;   // dynamic LDS of a conv block of several channel tiles
constexpr int CONV_LDS_LIMIT = 160 * 1024; // a CU's LDS: the most any conv block may take
constexpr int STAGE = 8;                   // loads in flight per thread when staging tiles
constexpr int RB = 1024;                   // threads of the kernels ending in an FP64 block sum
inline int rblocks(int64_t n) { return (int)std::max<int64_t>(1, std::min<int64_t>((n + RB - 1) / RB, 256)); }

__device__ __forceinline__ uint32_t bf16_rne(float f)
{
    const uint32_t u = __float_as_uint(f);
    return (u + 0x7fffu + ((u >> 16) & 1u)) >> 16;
}
__device__ __forceinline__ uint2 pack4(float4 v)
{
    return make_uint2(bf16_rne(v.x) | (bf16_rne(v.y) << 16), bf16_rne(v.z) | (bf16_rne(v.w) << 16));
}

struct ConvArgs {
    const float *x;             // input NHWC [B][Hin][Win][cin_p]
    int32_t Hin, Win, up_in, cin_p;
    const short *w;             // BF16 rows [nt * 16][kpad]
    int32_t kpad;
    const float *bias;          // [cout_p] or null
    const float *skip;          // added before the ReLU, layout of y, or null
    const float *mask;          // y *= (mask > 0), layout of y, or null
    float *y;                   // output NHWC [B][H][W][cout_p]
    int32_t H, W, cout_p;
    int32_t relu, accumulate;
    int32_t nsplit;             // blocks per sample along the output tiles
    int32_t nband, bpb;         // column bands, blocks per band
};

__device__ __forceinline__ v4f mfma32(v8s a, v8s b, v4f c)
{
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(v8bf, a),
                                                   __builtin_bit_cast(v8bf, b), c, 0, 0, 0);
}

// input value quad (4 channels from c4) of output-grid pixel (ys, xs)
__device__ __forceinline__ float4 load_in(const float *x, int b, int ys, int xs, int H, int W,
                                          int Hin, int Win, int up_in, int cin_p, int c4)
{
    if (ys < 0 || ys >= H || xs < 0 || xs >= W) return make_float4(0.f, 0.f, 0.f, 0.f);
    int64_t pix;
    if (up_in) pix = ((int64_t)b * Hin + (ys >> 1)) * Win + (xs >> 1);
    else pix = ((int64_t)b * H + ys) * W + xs;
    return *(const float4 *)(x + pix * cin_p + c4);
}

// Row stride (shorts) of the weight rows staged in LDS: padded by 8 so that
// the 16 rows a wavefront reads at one column fall in different banks.
__host__ __device__ __forceinline__ int wrow_lds(int kpad) { return kpad + 8; }

// WG: the weights are read from global memory (L2) in the k loop, one step
// ahead, instead of staged in LDS; the block then holds only its patch in
// LDS, so more blocks fit a CU where the weights would have kept one out
template <int NT, bool WG>
__global__ void __launch_bounds__(256) k_conv3x3(ConvArgs a)
{
    extern __shared__ __align__(16) char lds[];
    // blockIdx.y = sample * nsplit + split: this block's 16-channel output
    // tiles are [split * NT, split * NT + NT); blockIdx.x = band * bpb + chunk
    const int b = blockIdx.y / a.nsplit, tile0 = (blockIdx.y - b * a.nsplit) * NT;
    const int band = blockIdx.x / a.bpb, chunk = blockIdx.x - band * a.bpb;
    const int c0 = (int)((int64_t)band * a.W / a.nband);
    const int bw = (int)((int64_t)(band + 1) * a.W / a.nband) - c0;
    const int npix = a.H * bw, i0 = chunk * CONV_PIX;
    if (i0 >= npix) return;                     // the whole block: a band's spare chunk
    const int i1 = min(npix, i0 + CONV_PIX);
    const int ra = i0 / bw, prows = (i1 - 1) / bw - ra + 3, pw = bw + 2;
    const int cst = a.cin_p + 4;
    short *patch = (short *)lds;                // [prows][pw][cst], image row ra - 1 first
    const int patch_bytes = (prows * pw * cst * 2 + 15) & ~15;
    int *off4 = (int *)(lds + patch_bytes);
    short *wl = (short *)(lds + patch_bytes + (((a.kpad >> 2) * 4 + 15) & ~15));
    const int wst = wrow_lds(a.kpad);
    // the block's weight rows, once, into LDS (16-byte pieces)
    // (every staging loop issues STAGE loads per thread before it stores any,
    // so a block waits for memory a few times, not once per piece)
    if constexpr (!WG) {
        const int pieces = a.kpad >> 3;            // 8 shorts per piece
        const int total = NT * 16 * pieces;
        const short *wsrc = a.w + (int64_t)tile0 * 16 * a.kpad;
        for (int t0 = threadIdx.x; t0 < total; t0 += 256 * STAGE) {
            uint4 v[STAGE];
#pragma unroll
            for (int u = 0; u < STAGE; ++u) {
                const int t = t0 + u * 256;
                v[u] = make_uint4(0u, 0u, 0u, 0u);   // defined on every path: kept in registers
                if (t < total) {
                    const int row = t / pieces, pc = t - row * pieces;
                    v[u] = *(const uint4 *)(wsrc + (int64_t)row * a.kpad + 8 * pc);
                }
            }
#pragma unroll
            for (int u = 0; u < STAGE; ++u) {
                const int t = t0 + u * 256;
                if (t < total) {
                    const int row = t / pieces, pc = t - row * pieces;
                    *(uint4 *)(wl + row * wst + 8 * pc) = v[u];
                }
            }
        }
    }
    const int quads = a.cin_p >> 2;
    {
        const int total = prows * pw * quads;
        for (int t0 = threadIdx.x; t0 < total; t0 += 256 * STAGE) {
            float4 v[STAGE];
#pragma unroll
            for (int u = 0; u < STAGE; ++u) {
                const int t = t0 + u * 256;
                v[u] = make_float4(0.f, 0.f, 0.f, 0.f);
                if (t < total) {
                    const int q = t % quads, pix = t / quads;
                    const int r = pix / pw, col = pix - r * pw;
                    v[u] = load_in(a.x, b, ra - 1 + r, c0 - 1 + col, a.H, a.W, a.Hin, a.Win,
                                   a.up_in, a.cin_p, 4 * q);
                }
            }
#pragma unroll
            for (int u = 0; u < STAGE; ++u) {
                const int t = t0 + u * 256;
                if (t < total) {
                    const int q = t % quads, pix = t / quads;
                    *(uint2 *)(patch + pix * cst + 4 * q) = pack4(v[u]);
                }
            }
        }
    }
    const int K = 9 * a.cin_p;
    for (int kk = threadIdx.x; kk < (a.kpad >> 2); kk += 256) {
        const int k = 4 * kk;
        int o = -1;
        if (k < K) {
            const int tap = k / a.cin_p, c = k - tap * a.cin_p;
            const int kh = tap / 3, kw = tap - 3 * kh;
            o = (kh * pw + kw) * cst + c;
        }
        off4[kk] = o;
    }
    __syncthreads();
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int m = lane & 15, g = lane >> 4;
    // this lane's pixel in each of the wave's four 16-pixel groups (the last
    // valid pixel stands in past the end, its result not stored)
    int prow[4], pcol[4], pofs[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        const int i = min(i0 + wave * 64 + t * 16 + m, i1 - 1);
        prow[t] = i / bw;
        pcol[t] = i - prow[t] * bw;
        pofs[t] = ((prow[t] - ra) * pw + pcol[t]) * cst;
    }
    v4f acc[4][NT];
#pragma unroll
    for (int t = 0; t < 4; ++t)
#pragma unroll
        for (int n = 0; n < NT; ++n) acc[t][n] = v4f{0.f, 0.f, 0.f, 0.f};
    const short *wbase = WG ? a.w + ((int64_t)tile0 * 16 + m) * a.kpad + 8 * g : wl + m * wst + 8 * g;
    const int wrow = WG ? a.kpad : wst;
    v8s wn[NT];
    if constexpr (WG) {
#pragma unroll
        for (int n = 0; n < NT; ++n) wn[n] = *(const v8s *)(wbase + n * 16 * wrow);
    }
    for (int kc = 0; kc < a.kpad; kc += 32) {
        v8s wa[NT];
        if constexpr (WG) {
#pragma unroll
            for (int n = 0; n < NT; ++n) {
                wa[n] = wn[n];
                if (kc + 32 < a.kpad) wn[n] = *(const v8s *)(wbase + n * 16 * wrow + kc + 32);
            }
        } else {
#pragma unroll
            for (int n = 0; n < NT; ++n) wa[n] = *(const v8s *)(wbase + n * 16 * wrow + kc);
        }
        const int o0 = off4[(kc >> 2) + 2 * g], o1 = off4[(kc >> 2) + 2 * g + 1];
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            v4s lo = {0, 0, 0, 0}, hi = {0, 0, 0, 0};
            if (o0 >= 0) lo = *(const v4s *)(patch + pofs[t] + o0);
            if (o1 >= 0) hi = *(const v4s *)(patch + pofs[t] + o1);
            const v8s pb = __builtin_shufflevector(lo, hi, 0, 1, 2, 3, 4, 5, 6, 7);
#pragma unroll
            for (int n = 0; n < NT; ++n) acc[t][n] = mfma32(wa[n], pb, acc[t][n]);
        }
    }
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        if (i0 + wave * 64 + t * 16 + m >= i1) continue;
        const int64_t pix = ((int64_t)b * a.H + prow[t]) * a.W + c0 + pcol[t];
#pragma unroll
        for (int n = 0; n < NT; ++n) {
            const int ch = (tile0 + n) * 16 + 4 * g;
            if (ch >= a.cout_p) continue;
            const int64_t o = pix * a.cout_p + ch;
            float4 v = make_float4(acc[t][n][0], acc[t][n][1], acc[t][n][2], acc[t][n][3]);
            if (a.bias) {
                const float4 bb = *(const float4 *)(a.bias + ch);
                v.x += bb.x; v.y += bb.y; v.z += bb.z; v.w += bb.w;
            }
            if (a.skip) {
                const float4 s = *(const float4 *)(a.skip + o);
                v.x += s.x; v.y += s.y; v.z += s.z; v.w += s.w;
            }
            if (a.relu) {
                v.x = fmaxf(v.x, 0.f); v.y = fmaxf(v.y, 0.f);
                v.z = fmaxf(v.z, 0.f); v.w = fmaxf(v.w, 0.f);
            }
            if (a.mask) {
                const float4 mk = *(const float4 *)(a.mask + o);
                v.x = mk.x > 0.f ? v.x : 0.f; v.y = mk.y > 0.f ? v.y : 0.f;
                v.z = mk.z > 0.f ? v.z : 0.f; v.w = mk.w > 0.f ? v.w : 0.f;
            }
            if (a.accumulate) {
                const float4 p = *(const float4 *)(a.y + o);
                v.x += p.x; v.y += p.y; v.z += p.z; v.w += p.w;
            }
            *(float4 *)(a.y + o) = v;
        }
    }
}

// Weight gradient: partial[split][n][k] = sum over the split's pixels of
// g[p][n] x[p + off(tap(k))][c(k)], and for k = 9 cin_p (bias column) sum of
// g[p][n].  GEMM with M = output channels, N = columns k, K = pixels.  Each
// wave owns PPW (n-tile, k-tile) pairs and keeps their accumulators over all
// tiles of its block's pixel range.
struct WgradArgs {
    const float *x;
    int32_t Hin, Win, up_in, cin_p;
    const float *g;             // NHWC [B][H][W][cout_p]
    int32_t cout_p, nt;
    int32_t H, W, B;
    int32_t kw;                 // row length of the result
    int32_t tiles_x, tiles_y;
    int32_t tiles_per_block;
    float *partial;             // [gridDim.y][nt * 16][kw]
};

constexpr int PPW = 4;

__global__ void __launch_bounds__(256) k_conv3x3_wgrad(WgradArgs a)
{
    extern __shared__ __align__(16) char lds[];
    short *gs = (short *)lds;                                   // [cout_p][TR * TX]
    short *xs = (short *)(lds + a.cout_p * TR * TX * 2);        // [cin_p][PH][PW]
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int m = lane & 15, g = lane >> 4;
    const int KT = a.kw >> 4, npairs = a.nt * KT;
    const int pair0 = (blockIdx.x * 4 + wave) * PPW;
    const int K = 9 * a.cin_p;
    v4f acc[PPW];
#pragma unroll
    for (int i = 0; i < PPW; ++i) acc[i] = v4f{0.f, 0.f, 0.f, 0.f};
    const int64_t ntiles = (int64_t)a.B * a.tiles_y * a.tiles_x;
    const int64_t t0 = (int64_t)blockIdx.y * a.tiles_per_block;
    const int64_t t1 = std::min<int64_t>(ntiles, t0 + a.tiles_per_block);
    const int gq = a.cout_p >> 2, xq = a.cin_p >> 2;
    for (int64_t tile = t0; tile < t1; ++tile) {
        const int tx = (int)(tile % a.tiles_x);
        const int64_t rest = tile / a.tiles_x;
        const int ty = (int)(rest % a.tiles_y), b = (int)(rest / a.tiles_y);
        const int x0 = tx * TX, y0 = ty * TR;
        __syncthreads();
        for (int t0 = threadIdx.x; t0 < TR * TX * gq; t0 += 256 * STAGE) {
            float4 v[STAGE];
#pragma unroll
            for (int u = 0; u < STAGE; ++u) {
                const int t = t0 + u * 256;
                v[u] = make_float4(0.f, 0.f, 0.f, 0.f);
                if (t < TR * TX * gq) {
                    const int q = t % gq, pix = t / gq;
                    const int r = pix / TX, col = pix - r * TX;
                    const int yy = y0 + r, xx = x0 + col;
                    if (yy < a.H && xx < a.W)
                        v[u] = *(const float4 *)(a.g + (((int64_t)b * a.H + yy) * a.W + xx) * a.cout_p + 4 * q);
                }
            }
#pragma unroll
            for (int u = 0; u < STAGE; ++u) {
                const int t = t0 + u * 256;
                if (t < TR * TX * gq) {
                    const int q = t % gq, pix = t / gq;
                    gs[(4 * q + 0) * TR * TX + pix] = (short)bf16_rne(v[u].x);
                    gs[(4 * q + 1) * TR * TX + pix] = (short)bf16_rne(v[u].y);
                    gs[(4 * q + 2) * TR * TX + pix] = (short)bf16_rne(v[u].z);
                    gs[(4 * q + 3) * TR * TX + pix] = (short)bf16_rne(v[u].w);
                }
            }
        }
        for (int t0 = threadIdx.x; t0 < PH * PW * xq; t0 += 256 * STAGE) {
            float4 v[STAGE];
#pragma unroll
            for (int u = 0; u < STAGE; ++u) {
                const int t = t0 + u * 256;
                v[u] = make_float4(0.f, 0.f, 0.f, 0.f);
                if (t < PH * PW * xq) {
                    const int q = t % xq, pix = t / xq;
                    const int r = pix / PW, col = pix - r * PW;
                    v[u] = load_in(a.x, b, y0 + r - 1, x0 + col - 1, a.H, a.W, a.Hin, a.Win,
                                   a.up_in, a.cin_p, 4 * q);
                }
            }
#pragma unroll
            for (int u = 0; u < STAGE; ++u) {
                const int t = t0 + u * 256;
                if (t < PH * PW * xq) {
                    const int q = t % xq, pix = t / xq;
                    const int r = pix / PW, col = pix - r * PW;
                    const int base = ((4 * q) * PH + r) * PW + col;
                    xs[base] = (short)bf16_rne(v[u].x);
                    xs[base + PH * PW] = (short)bf16_rne(v[u].y);
                    xs[base + 2 * PH * PW] = (short)bf16_rne(v[u].z);
                    xs[base + 3 * PH * PW] = (short)bf16_rne(v[u].w);
                }
            }
        }
        __syncthreads();
#pragma unroll
        for (int i = 0; i < PPW; ++i) {
            const int pr = pair0 + i;
            if (pr >= npairs) break;
            const int ntile = pr / KT, kt = pr - ntile * KT;
            const int n = ntile * 16 + m;           // A row of this lane
            const int k = kt * 16 + m;              // B column of this lane
            int xbase = -1;
            bool ones = false;
            if (k < K) {
                const int tap = k / a.cin_p, c = k - tap * a.cin_p;
                const int kh = tap / 3, kw = tap - 3 * kh;
                xbase = (c * PH + kh) * PW + kw;
            } else if (k == K) {
                ones = true;
            }
            const bool nok = n < a.cout_p;
            // K = the tile's pixels, 32 (half a row) per MFMA
            for (int ks = 0; ks < TR * TX / 32; ++ks) {
                v8s av = {0, 0, 0, 0, 0, 0, 0, 0};
                if (nok) av = *(const v8s *)(gs + n * TR * TX + ks * 32 + 8 * g);
                v8s bv = {0, 0, 0, 0, 0, 0, 0, 0};
                if (xbase >= 0) {
                    const int r = ks >> 1, col = (ks & 1) * 32 + 8 * g;
                    const short *px = xs + xbase + r * PW + col;
                    bv = v8s{px[0], px[1], px[2], px[3], px[4], px[5], px[6], px[7]};
                } else if (ones) {
                    const short one = (short)0x3f80;
                    bv = v8s{one, one, one, one, one, one, one, one};
                }
                acc[i] = mfma32(av, bv, acc[i]);
            }
        }
    }
    float *dst = a.partial + (int64_t)blockIdx.y * a.nt * 16 * a.kw;
#pragma unroll
    for (int i = 0; i < PPW; ++i) {
        const int pr = pair0 + i;
        if (pr >= npairs) break;
        const int ntile = pr / KT, kt = pr - ntile * KT;
#pragma unroll
        for (int j = 0; j < 4; ++j)
            dst[(int64_t)(ntile * 16 + 4 * g + j) * a.kw + kt * 16 + m] = acc[i][j];
    }
}

// out[t] += sum over the splits [64 blockIdx.y, 64 blockIdx.y + 64) of
// partial[split][t] (out zeroed before)
constexpr int RED_CHUNK = 64;
__global__ void k_wgrad_reduce(const float *partial, int splits, int64_t n, float *out)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n) return;
    const int k0 = blockIdx.y * RED_CHUNK, k1 = min(splits, k0 + RED_CHUNK);
    float s = 0.0f;
    for (int k = k0; k < k1; ++k) s += partial[(int64_t)k * n + t];
    unsafeAtomicAdd(out + t, s);
}

// ---- pooling and upsampling (NHWC float4 quads) ----------------------------
__global__ void k_pool2(const float *x, float *y, int B, int H, int W, int C_p)
{
    const int Hc = (H + 1) >> 1, Wc = (W + 1) >> 1, q4 = C_p >> 2;
    const int64_t total = (int64_t)B * Hc * Wc * q4;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total;
         t += (int64_t)gridDim.x * blockDim.x) {
        const int q = (int)(t % q4);
        int64_t r = t / q4;
        const int X = (int)(r % Wc);
        r /= Wc;
        const int Y = (int)(r % Hc);
        const int b = (int)(r / Hc);
        float4 s = make_float4(0.f, 0.f, 0.f, 0.f);
        int cnt = 0;
        for (int dy = 0; dy < 2; ++dy)
            for (int dx = 0; dx < 2; ++dx) {
                const int yy = 2 * Y + dy, xx = 2 * X + dx;
                if (yy >= H || xx >= W) continue;
                const float4 v = *(const float4 *)(x + (((int64_t)b * H + yy) * W + xx) * C_p + 4 * q);
                s.x += v.x; s.y += v.y; s.z += v.z; s.w += v.w;
                ++cnt;
            }
        const float inv = 1.0f / (float)cnt;
        *(float4 *)(y + t * 4) = make_float4(s.x * inv, s.y * inv, s.z * inv, s.w * inv);
    }
}

// dx = mask > 0 ? (accumulate ? dx : 0) + dy[coarse] / count : 0
__global__ void k_pool2_bwd(const float *dy, float *dx, const float *mask, int accumulate, int B,
                            int H, int W, int C_p)
{
    const int Hc = (H + 1) >> 1, Wc = (W + 1) >> 1, q4 = C_p >> 2;
    const int64_t total = (int64_t)B * H * W * q4;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total;
         t += (int64_t)gridDim.x * blockDim.x) {
        const int q = (int)(t % q4);
        int64_t r = t / q4;
        const int xx = (int)(r % W);
        r /= W;
        const int yy = (int)(r % H);
        const int b = (int)(r / H);
        const int Y = yy >> 1, X = xx >> 1;
        const float cnt = (float)(((2 * Y + 1 < H) ? 2 : 1) * ((2 * X + 1 < W) ? 2 : 1));
        const float4 g = *(const float4 *)(dy + (((int64_t)b * Hc + Y) * Wc + X) * C_p + 4 * q);
        const float inv = 1.0f / cnt;
        float4 v = make_float4(g.x * inv, g.y * inv, g.z * inv, g.w * inv);
        if (accumulate) {
            const float4 p = *(const float4 *)(dx + t * 4);
            v.x += p.x; v.y += p.y; v.z += p.z; v.w += p.w;
        }
        if (mask) {
            const float4 mk = *(const float4 *)(mask + t * 4);
            v.x = mk.x > 0.f ? v.x : 0.f; v.y = mk.y > 0.f ? v.y : 0.f;
            v.z = mk.z > 0.f ? v.z : 0.f; v.w = mk.w > 0.f ? v.w : 0.f;
        }
        *(float4 *)(dx + t * 4) = v;
    }
}

// adjoint of nearest upsampling to H x W, then dx *= (mask > 0)
__global__ void k_up2_bwd(const float *dy, float *dx, const float *mask, int B, int H, int W,
                          int C_p)
{
    const int Hc = (H + 1) >> 1, Wc = (W + 1) >> 1, q4 = C_p >> 2;
    const int64_t total = (int64_t)B * Hc * Wc * q4;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total;
         t += (int64_t)gridDim.x * blockDim.x) {
        const int q = (int)(t % q4);
        int64_t r = t / q4;
        const int X = (int)(r % Wc);
        r /= Wc;
        const int Y = (int)(r % Hc);
        const int b = (int)(r / Hc);
        float4 s = make_float4(0.f, 0.f, 0.f, 0.f);
        for (int a = 0; a < 2; ++a)
            for (int c = 0; c < 2; ++c) {
                const int yy = 2 * Y + a, xx = 2 * X + c;
                if (yy >= H || xx >= W) continue;
                const float4 v = *(const float4 *)(dy + (((int64_t)b * H + yy) * W + xx) * C_p + 4 * q);
                s.x += v.x; s.y += v.y; s.z += v.z; s.w += v.w;
            }
        if (mask) {
            const float4 mk = *(const float4 *)(mask + t * 4);
            s.x = mk.x > 0.f ? s.x : 0.f; s.y = mk.y > 0.f ? s.y : 0.f;
            s.z = mk.z > 0.f ? s.z : 0.f; s.w = mk.w > 0.f ? s.w : 0.f;
        }
        *(float4 *)(dx + t * 4) = s;
    }
}

// ---- block reduction helper -------------------------------------------------
// (blocks of up to 1024 threads; one FP64 atomic per block)
__device__ __forceinline__ void block_add(double v, double *dst)
{
    __shared__ double red[16];
    v = wave_sum(v);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        double s = 0.0;
        for (int w = 0; w < (int)(blockDim.x >> 6); ++w) s += red[w];
        if (s != 0.0) atomic_add_dev(dst, s);
    }
    __syncthreads();
}

// ---- preconditioner input / output --------------------------------------------
// ss[b] += sum over unknown nodes of (scale v)^2, sample b = blockIdx.y
template <typename T>
__global__ void __launch_bounds__(EB) k_pc_sumsq(const T *v, int64_t stride, double scale,
                                                  MGLevel L, double *ss)
{
    const int ld = L.nr + 1;
    const int64_t nn = (int64_t)ld * (L.nz + 1);
    const T *s = v + (int64_t)blockIdx.y * stride;
    double acc = 0.0;
    for (int64_t n = (int64_t)blockIdx.x * EB + threadIdx.x; n < nn; n += (int64_t)gridDim.x * EB) {
        int i, j;
        node_ij(n, ld, i, j);
        if (mg_unknown(L, i, j)) {
            const double t = scale * (double)s[n];
            acc += t * t;
        }
    }
    block_add(acc, ss + blockIdx.y);
}

// x[b][p] = (v / rho on unknowns, i / 256, 0, 0), rho = sqrt(ss[b] / n_unknown)
template <typename T>
__global__ void k_pc_input(const T *v, int64_t stride, double scale, const double *ss,
                           double inv_nunk, MGLevel L, float *x, int B)
{
    const int ld = L.nr + 1;
    const int64_t nn = (int64_t)ld * (L.nz + 1);
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < (int64_t)B * nn;
         t += (int64_t)gridDim.x * blockDim.x) {
        const int b = (int)((uint32_t)t / (uint32_t)nn);
        const int64_t n = t - (int64_t)b * nn;
        int i, j;
        node_ij(n, ld, i, j);
        const double rho = sqrt(ss[b] * inv_nunk);
        float r = 0.0f;
        if (rho > 0.0 && mg_unknown(L, i, j)) r = (float)(scale * (double)v[b * stride + n] / rho);
        *(float4 *)(x + t * 4) = make_float4(r, (float)i * (1.0f / 256.0f), 0.f, 0.f);
    }
}

__global__ void __launch_bounds__(RB) k_pc_identity(MGLevel L, const float *r, float *z, double *rz)
{
    const int ld = L.nr + 1;
    const int64_t nn = (int64_t)ld * (L.nz + 1);
    double acc = 0.0;
    for (int64_t n = (int64_t)blockIdx.x * RB + threadIdx.x; n < nn; n += (int64_t)gridDim.x * RB) {
        const float v = r[n];
        z[n] = v;
        acc += (double)v * (double)v;
    }
    block_add(acc, rz);
}

// ---- training -------------------------------------------------------------------
__device__ __forceinline__ double op_ae(const MGLevel &L, int i, int j)
{
    const double hz = (j == 0 || j == L.nz) ? 0.5 * (double)L.dz : (double)L.dz;
    return ((double)i + 0.5) * hz;
}
__device__ __forceinline__ double op_an(const MGLevel &L, int i)
{
    const double g = (i == 0) ? 0.125 : ((i == L.nr) ? 0.5 * (double)L.nr - 0.125 : (double)i);
    return g * (double)L.dr2dz;
}

// ---- red-black Gauss-Seidel around the network -------------------------------
// Half sweep of one colour ((i + j) & 1 == colour) of A x = b on the unknown
// nodes: x_p = (b_p + sum_nb c_nb x_nb) / sum_nb c_nb.  from_zero: the
// other colour and the Dirichlet nodes are set to 0 (x = 0 before the
// sweep).  With rz: rz += z.dot_r and, with zq, zq += z.dot_q over all nodes
// after the sweep.  Sample b = blockIdx.y at offset b * stride.
__global__ void __launch_bounds__(RB) k_rb_sweep(MGLevel L, const float *bv, float *xv,
                                                  int64_t stride, int colour, int from_zero,
                                                  const float *dot_r, const float *dot_q,
                                                  double *rz, double *zq)
{
    const int ld = L.nr + 1;
    const int64_t nn = (int64_t)ld * (L.nz + 1);
    const float *b = bv + (int64_t)blockIdx.y * stride;
    float *x = xv + (int64_t)blockIdx.y * stride;
    double arz = 0.0, azq = 0.0;
    for (int64_t n = (int64_t)blockIdx.x * RB + threadIdx.x; n < nn; n += (int64_t)gridDim.x * RB) {
        int i, j;
        node_ij(n, ld, i, j);
        const bool unk = mg_unknown(L, i, j);
        float v;
        if (unk && ((i + j) & 1) == colour) {
            float cw, ce, cs, cn;
            mg_coup(L, i, j, cw, ce, cs, cn);
            float off = 0.0f;
            if (!from_zero) {
                off = ce * x[n + 1] + cn * x[n + ld];
                if (i > 0) off += cw * x[n - 1];
                if (j > 0) off += cs * x[n - ld];
            }
            v = (b[n] + off) / (cw + ce + cs + cn);
            x[n] = v;
        } else if (from_zero) {
            v = 0.0f;
            x[n] = v;
        } else {
            v = x[n];
        }
        if (rz) {
            arz += (double)v * (double)dot_r[n];
            if (dot_q) azq += (double)v * (double)dot_q[n];
        }
    }
    if (rz) block_add(arz, rz);
    if (zq && dot_q) block_add(azq, zq);
}

// r = b - A x on unknown nodes (0 elsewhere); ss[sample] += r^2
__global__ void __launch_bounds__(RB) k_residual32(MGLevel L, const float *bv, const float *xv,
                                                    float *rv, int64_t stride, double *ss)
{
    const int ld = L.nr + 1;
    const int64_t nn = (int64_t)ld * (L.nz + 1);
    const float *b = bv + (int64_t)blockIdx.y * stride;
    const float *x = xv + (int64_t)blockIdx.y * stride;
    float *r = rv + (int64_t)blockIdx.y * stride;
    double acc = 0.0;
    for (int64_t n = (int64_t)blockIdx.x * RB + threadIdx.x; n < nn; n += (int64_t)gridDim.x * RB) {
        int i, j;
        node_ij(n, ld, i, j);
        float v = 0.0f;
        if (mg_unknown(L, i, j)) {
            float cw, ce, cs, cn;
            mg_coup(L, i, j, cw, ce, cs, cn);
            float ax = (cw + ce + cs + cn) * x[n] - ce * x[n + 1] - cn * x[n + ld];
            if (i > 0) ax -= cw * x[n - 1];
            if (j > 0) ax -= cs * x[n - ld];
            v = b[n] - ax;
            acc += (double)v * (double)v;
        }
        r[n] = v;
    }
    block_add(acc, ss + blockIdx.y);
}

// z = x1 + out_scale rho1 net on unknown nodes, 0 elsewhere
__global__ void k_pc_combine(const float *net, const double *ss, double inv_nunk, double out_scale,
                             MGLevel L, const float *x1, float *z)
{
    const int ld = L.nr + 1;
    const int64_t nn = (int64_t)ld * (L.nz + 1);
    const float sc = (float)(out_scale * sqrt(ss[0] * inv_nunk));
    for (int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; n < nn;
         n += (int64_t)gridDim.x * blockDim.x) {
        int i, j;
        node_ij(n, ld, i, j);
        z[n] = mg_unknown(L, i, j) ? x1[n] + sc * net[n * 4] : 0.0f;
    }
}

// bh = scale q / rho0 on unknown nodes (FP32), rho0 = sqrt(ss0 / n_unknown)
template <typename T>
__global__ void k_pc_scale_in(const T *q, int64_t stride, double scale, const double *ss0,
                              double inv_nunk, MGLevel L, float *bh, int B)
{
    const int ld = L.nr + 1;
    const int64_t nn = (int64_t)ld * (L.nz + 1);
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < (int64_t)B * nn;
         t += (int64_t)gridDim.x * blockDim.x) {
        const int b = (int)((uint32_t)t / (uint32_t)nn);
        const int64_t n = t - (int64_t)b * nn;
        int i, j;
        node_ij(n, ld, i, j);
        const double rho = ss0 ? sqrt(ss0[b] * inv_nunk) : 1.0;
        float v = 0.0f;
        if (rho > 0.0 && mg_unknown(L, i, j)) v = (float)(scale * (double)q[b * stride + n] / rho);
        bh[t] = v;
    }
}

__global__ void k_cast_out(const float *z, double *out, int64_t n)
{
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n;
         t += (int64_t)gridDim.x * blockDim.x)
        out[t] = (double)z[t];
}

// Training targets t = (phi / rho0 - x1) / rho1 (FP32) and den[b] = t.A t (FP64)
__global__ void __launch_bounds__(EB) k_pc_targets(const double *phi, int64_t stride,
                                                    const double *ss0, const double *ss1,
                                                    double inv_nunk, const float *x1v,
                                                    MGLevel L, float *tgt, double *den)
{
    const int ld = L.nr + 1;
    const int64_t nn = (int64_t)ld * (L.nz + 1);
    const int b = blockIdx.y;
    const double rho0 = sqrt(ss0[b] * inv_nunk), rho1 = sqrt(ss1[b] * inv_nunk);
    const double inv0 = rho0 > 0.0 ? 1.0 / rho0 : 0.0, inv1 = rho1 > 0.0 ? 1.0 / rho1 : 0.0;
    const double *p = phi + (int64_t)b * stride;
    const float *x1 = x1v + (int64_t)b * nn;
    auto tv = [&](int ii, int jj) {
        const int64_t q = (int64_t)jj * ld + ii;
        return mg_unknown(L, ii, jj) ? (double)(float)((p[q] * inv0 - (double)x1[q]) * inv1) : 0.0;
    };
    double acc = 0.0;
    for (int64_t n = (int64_t)blockIdx.x * EB + threadIdx.x; n < nn; n += (int64_t)gridDim.x * EB) {
        int i, j;
        node_ij(n, ld, i, j);
        float out = 0.0f;
        if (mg_unknown(L, i, j)) {
            const double c = tv(i, j);
            double a = op_ae(L, i, j) * (c - tv(i + 1, j)) + op_an(L, i) * (c - tv(i, j + 1));
            if (i > 0) a += op_ae(L, i - 1, j) * (c - tv(i - 1, j));
            if (j > 0) a += op_an(L, i) * (c - tv(i, j - 1));
            acc += c * a;
            out = (float)c;
        }
        tgt[(int64_t)b * nn + n] = out;
    }
    block_add(acc, den + b);
}

// e = out_scale net - tgt on unknowns; L += (1/2) e.Ae / (B den_b);
// gout = out_scale Ae / (B den_b) in channel 0 (FP32 stencil, FP64 sums)
__global__ void __launch_bounds__(EB) k_pc_loss(const float *net, const float *tgt,
                                                 const double *den, double out_scale, MGLevel L,
                                                 int B, float *gout, double *loss)
{
    const int ld = L.nr + 1;
    const int64_t nn = (int64_t)ld * (L.nz + 1);
    const int b = blockIdx.y;
    const float s = (float)out_scale;
    const float *nb = net + (int64_t)b * nn * 4;
    const float *tb = tgt + (int64_t)b * nn;
    const double w = 1.0 / ((double)B * den[b]);
    double acc = 0.0;
    for (int64_t n = (int64_t)blockIdx.x * EB + threadIdx.x; n < nn; n += (int64_t)gridDim.x * EB) {
        int i, j;
        node_ij(n, ld, i, j);
        float g = 0.0f;
        if (mg_unknown(L, i, j)) {
            auto e = [&](int ii, int jj) {
                const int64_t q = (int64_t)jj * ld + ii;
                return mg_unknown(L, ii, jj) ? s * nb[q * 4] - tb[q] : 0.0f;
            };
            float cw, ce, cs, cn;
            mg_coup(L, i, j, cw, ce, cs, cn);
            const float ec = e(i, j);
            float ae = ce * (ec - e(i + 1, j)) + cn * (ec - e(i, j + 1));
            if (i > 0) ae += cw * (ec - e(i - 1, j));
            if (j > 0) ae += cs * (ec - e(i, j - 1));
            acc += 0.5 * (double)ec * (double)ae * w;
            g = (float)((double)s * (double)ae * w);
        }
        *(float4 *)(gout + ((int64_t)b * nn + n) * 4) = make_float4(g, 0.f, 0.f, 0.f);
    }
    block_add(acc, loss);
}

// Adam (Kingma and Ba) with bias-corrected moments; a1 = 1 - beta1 and
// a2 = 1 - beta2 are passed rounded from their exact values (1 - 0.999f is
// 1.3e-5 off 0.001), c1 = 1 - beta1^t and c2 = 1 - beta2^t likewise.
__global__ void k_adam(float *w, const float *g, float *m, float *v, int64_t n, float lr, float b1,
                       float b2, float a1, float a2, float eps, float c1, float c2)
{
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n;
         t += (int64_t)gridDim.x * blockDim.x) {
        const float gt = g[t];
        const float mt = b1 * m[t] + a1 * gt;
        const float vt = b2 * v[t] + a2 * gt * gt;
        m[t] = mt;
        v[t] = vt;
        w[t] -= lr * (mt / c1) / (sqrtf(vt / c2) + eps);
    }
}

// BF16 forward / data-gradient rows and the FP32 bias of one layer
__global__ void k_pack(PcLayer l, const float *master, short *wf, short *wt, float *bias)
{
    const float *M = master + l.o_master;
    const int K = 9 * l.cin_p;
    const int nf = l.nt * 16 * l.kpad, nw = l.nt_t * 16 * l.kpad_t;
    for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < nf + nw + l.cout_p;
         t += gridDim.x * blockDim.x) {
        if (t < nf) {
            const int n = t / l.kpad, k = t - n * l.kpad;
            wf[l.o_wf + t] = (short)((k < K) ? bf16_rne(M[(int64_t)n * l.kw + k]) : 0u);
        } else if (t < nf + nw) {
            const int u = t - nf;
            const int c = u / l.kpad_t, k = u - c * l.kpad_t;
            uint32_t v = 0;
            if (k < 9 * l.cout_p && c < l.cin) {
                const int tap = k / l.cout_p, n = k - tap * l.cout_p;
                if (n < l.cout) v = bf16_rne(M[(int64_t)n * l.kw + (8 - tap) * l.cin_p + c]);
            }
            wt[l.o_wt + u] = (short)v;
        } else {
            const int n = t - nf - nw;
            bias[l.o_bias + n] = (n < l.cout) ? M[(int64_t)n * l.kw + K] : 0.0f;
        }
    }
}

inline int eblocks(int64_t n)
{
    return (int)std::max<int64_t>(1, std::min<int64_t>((n + EB - 1) / EB, 4096));
}
inline int64_t round_up(int64_t v, int64_t a) { return (v + a - 1) / a * a; }

// ---- launch helpers ------------------------------------------------------------
// Column bands of an H x W level for the forward / data-gradient kernel: the
// band count, blocks per band, and the most patch rows and columns a block
// stages (256 consecutive pixels of a band b wide span at most 2 + 255 / b
// rows; one halo row above and below, one halo column each side).
struct ConvGeom {
    int nband, bpb, prows, pw;
};
ConvGeom conv_geom(int H, int W)
{
    ConvGeom c;
    c.nband = std::max(1, (W + BAND_MAX - 1) / BAND_MAX);
    const int bwmax = (W + c.nband - 1) / c.nband, bwmin = W / c.nband;
    c.bpb = (int)(((int64_t)H * bwmax + CONV_PIX - 1) / CONV_PIX);
    c.prows = std::min(H, 2 + (CONV_PIX - 1) / bwmin) + 2;
    c.pw = bwmax + 2;
    return c;
}
int conv_lds(const ConvGeom &c, int cin_p, int kpad, int ntb)
{
    return ((c.prows * c.pw * (cin_p + 4) * 2 + 15) & ~15) + (((kpad / 4) * 4 + 15) & ~15) +
           ntb * 16 * wrow_lds(kpad) * 2;
}

void conv(const PcNet &n, int li, bool dgrad, const float *x, const float *skip, const float *mask,
          float *y, int relu, int accumulate, int B, hipStream_t s)
{
    const PcLayer &l = n.L[li];
    ConvArgs a;
    memset(&a, 0, sizeof(a));
    a.x = x;
    a.up_in = dgrad ? 0 : l.up_in;
    const int out_level = l.level;
    const int in_level = (l.up_in && !dgrad) ? l.level + 1 : l.level;
    a.Hin = n.H[in_level];
    a.Win = n.W[in_level];
    a.H = n.H[out_level];
    a.W = n.W[out_level];
    a.cin_p = dgrad ? l.cout_p : l.cin_p;
    a.cout_p = dgrad ? l.cin_p : l.cout_p;
    a.w = dgrad ? n.wt + l.o_wt : n.wf + l.o_wf;
    a.kpad = dgrad ? l.kpad_t : l.kpad;
    a.bias = dgrad ? nullptr : n.bias + l.o_bias;
    a.skip = skip;
    a.mask = mask;
    a.y = y;
    a.relu = relu;
    a.accumulate = accumulate;
    const int nt = dgrad ? l.nt_t : l.nt;
    const ConvGeom cg = conv_geom(a.H, a.W);
    a.nband = cg.nband;
    a.bpb = cg.bpb;
    // one block per tile of output channels when the grid alone is too
    // small to fill the chip or the block's weights would not fit in LDS
    const int64_t blocks = (int64_t)cg.nband * cg.bpb * B;
    int ntb = (nt > 1 && (blocks < 1024 || conv_lds(cg, a.cin_p, a.kpad, nt) > CONV_LDS_MAX)) ? 1 : nt;
    if (ntb != 3 && ntb != 5) ntb = 1;            // instantiated tile counts
    a.nsplit = nt / ntb;
    dim3 g(cg.nband * cg.bpb, B * a.nsplit);
    const int lds = conv_lds(cg, a.cin_p, a.kpad, ntb);
    // one channel tile of 16 or more input channels: read the weights from
    // L2 when leaving them out of LDS fits more blocks on a CU (the 2-channel
    // input layer, 64 k values, is faster with them in LDS)
    const int lds_wg = conv_lds(cg, a.cin_p, a.kpad, 0);
    if (ntb == 1 && a.cin_p >= 16 && CONV_LDS_LIMIT / lds_wg > CONV_LDS_LIMIT / lds) {
        hipLaunchKernelGGL((k_conv3x3<1, true>), g, dim3(256), lds_wg, s, a);
        return;
    }
    switch (ntb) {
        case 1: hipLaunchKernelGGL((k_conv3x3<1, false>), g, dim3(256), lds, s, a); break;
        case 3: hipLaunchKernelGGL((k_conv3x3<3, false>), g, dim3(256), lds, s, a); break;
        default: hipLaunchKernelGGL((k_conv3x3<5, false>), g, dim3(256), lds, s, a); break;
    }
}

// pair groups (blocks in x) and pixel-range splits (blocks in y, at most)
int wgrad_groups(const PcLayer &l)
{
    const int npairs = l.nt * (l.kw / 16);
    return (npairs + 4 * PPW - 1) / (4 * PPW);
}
int wgrad_splits(const PcLayer &l)
{
    return std::max(1, std::min(PC_WGRAD_SPLITS, (2048 + wgrad_groups(l) - 1) / wgrad_groups(l)));
}

// weight gradient of layer li from its forward input x and output gradient g
void wgrad(PcNet &n, int li, const float *x, const float *g, int B, hipStream_t s)
{
    const PcLayer &l = n.L[li];
    WgradArgs a;
    memset(&a, 0, sizeof(a));
    a.x = x;
    a.up_in = l.up_in;
    a.Hin = n.H[l.up_in ? l.level + 1 : l.level];
    a.Win = n.W[l.up_in ? l.level + 1 : l.level];
    a.cin_p = l.cin_p;
    a.g = g;
    a.cout_p = l.cout_p;
    a.nt = l.nt;
    a.H = n.H[l.level];
    a.W = n.W[l.level];
    a.B = B;
    a.kw = l.kw;
    a.tiles_x = (a.W + TX - 1) / TX;
    a.tiles_y = (a.H + TR - 1) / TR;
    const int64_t ntiles = (int64_t)B * a.tiles_x * a.tiles_y;
    const int gx = wgrad_groups(l);
    const int splits = (int)std::min<int64_t>(ntiles, wgrad_splits(l));
    a.tiles_per_block = (int)((ntiles + splits - 1) / splits);
    const int gy = (int)((ntiles + a.tiles_per_block - 1) / a.tiles_per_block);
    a.partial = n.partial;
    const int lds = l.cout_p * TR * TX * 2 + l.cin_p * PH * PW * 2;
    hipLaunchKernelGGL(k_conv3x3_wgrad, dim3(gx, gy), dim3(256), lds, s, a);
    const int64_t ne = (int64_t)l.nt * 16 * l.kw;
    launch_zero(n.grad + l.o_master, ne * 4, s);
    hipLaunchKernelGGL(k_wgrad_reduce, dim3((unsigned)((ne + EB - 1) / EB), (gy + RED_CHUNK - 1) / RED_CHUNK),
                       dim3(EB), 0, s, (const float *)n.partial, gy, ne, n.grad + l.o_master);
}

void pool(const PcNet &n, int level, const float *x, float *y, int C_p, int B, hipStream_t s)
{
    const int H = n.H[level], W = n.W[level];
    const int64_t tot = (int64_t)B * ((H + 1) / 2) * ((W + 1) / 2) * (C_p / 4);
    hipLaunchKernelGGL(k_pool2, dim3(eblocks(tot)), dim3(EB), 0, s, x, y, B, H, W, C_p);
}

void pool_bwd(const PcNet &n, int level, const float *dy, float *dx, const float *mask, int acc,
              int C_p, int B, hipStream_t s)
{
    const int H = n.H[level], W = n.W[level];
    const int64_t tot = (int64_t)B * H * W * (C_p / 4);
    hipLaunchKernelGGL(k_pool2_bwd, dim3(eblocks(tot)), dim3(EB), 0, s, dy, dx, mask, acc, B, H, W,
                       C_p);
}

void up_bwd(const PcNet &n, int level, const float *dy, float *dx, const float *mask, int C_p,
            int B, hipStream_t s)
{
    const int H = n.H[level], W = n.W[level];
    const int64_t tot = (int64_t)B * ((H + 1) / 2) * ((W + 1) / 2) * (C_p / 4);
    hipLaunchKernelGGL(k_up2_bwd, dim3(eblocks(tot)), dim3(EB), 0, s, dy, dx, mask, B, H, W, C_p);
}

void forward(PcNet &n, int B, hipStream_t s)
{
    conv(n, 0, false, n.x, nullptr, nullptr, n.c0a, 1, 0, B, s);
    conv(n, 1, false, n.c0a, nullptr, nullptr, n.e0, 1, 0, B, s);
    pool(n, 0, n.e0, n.p1, 16, B, s);
    conv(n, 2, false, n.p1, nullptr, nullptr, n.c1a, 1, 0, B, s);
    conv(n, 3, false, n.c1a, nullptr, nullptr, n.e1, 1, 0, B, s);
    pool(n, 1, n.e1, n.p2, 16, B, s);
    conv(n, 4, false, n.p2, nullptr, nullptr, n.c2a, 1, 0, B, s);
    conv(n, 5, false, n.c2a, nullptr, nullptr, n.e2, 1, 0, B, s);
    pool(n, 2, n.e2, n.p3, 48, B, s);
    conv(n, 6, false, n.p3, nullptr, nullptr, n.c3a, 1, 0, B, s);
    conv(n, 7, false, n.c3a, nullptr, nullptr, n.e3, 1, 0, B, s);
    conv(n, 8, false, n.e3, n.e2, nullptr, n.d2a, 1, 0, B, s);
    conv(n, 9, false, n.d2a, nullptr, nullptr, n.d2, 1, 0, B, s);
    conv(n, 10, false, n.d2, n.e1, nullptr, n.d1a, 1, 0, B, s);
    conv(n, 11, false, n.d1a, nullptr, nullptr, n.d1, 1, 0, B, s);
    conv(n, 12, false, n.d1, n.e0, nullptr, n.d0a, 1, 0, B, s);
    conv(n, 13, false, n.d0a, nullptr, nullptr, n.d0, 1, 0, B, s);
    conv(n, 14, false, n.d0, nullptr, nullptr, n.out, 0, 0, B, s);
}

// Backward from g_out.  Names: gA = gradient at a conv output's
// pre-activation, gS = at a skip-joined pre-activation (also the skip
// branch's gradient), gB = at an upsampled input, gC = encoder conv,
// gP = at a pooled input.  gA0 doubles as gB0 and gC0.
void backward(PcNet &n, int B, hipStream_t s)
{
    wgrad(n, 14, n.d0, n.g_out, B, s);
    conv(n, 14, true, n.g_out, nullptr, n.d0, n.gA0, 0, 0, B, s);
    wgrad(n, 13, n.d0a, n.gA0, B, s);
    conv(n, 13, true, n.gA0, nullptr, n.d0a, n.gS0, 0, 0, B, s);
    wgrad(n, 12, n.d1, n.gS0, B, s);
    conv(n, 12, true, n.gS0, nullptr, nullptr, n.gA0, 0, 0, B, s);           // gB0
    up_bwd(n, 0, n.gA0, n.gA1, n.d1, 16, B, s);
    wgrad(n, 11, n.d1a, n.gA1, B, s);
    conv(n, 11, true, n.gA1, nullptr, n.d1a, n.gS1, 0, 0, B, s);
    wgrad(n, 10, n.d2, n.gS1, B, s);
    conv(n, 10, true, n.gS1, nullptr, nullptr, n.gB1, 0, 0, B, s);
    up_bwd(n, 1, n.gB1, n.gA2, n.d2, 48, B, s);
    wgrad(n, 9, n.d2a, n.gA2, B, s);
    conv(n, 9, true, n.gA2, nullptr, n.d2a, n.gS2, 0, 0, B, s);
    wgrad(n, 8, n.e3, n.gS2, B, s);
    conv(n, 8, true, n.gS2, nullptr, nullptr, n.gB2, 0, 0, B, s);
    up_bwd(n, 2, n.gB2, n.gA3, n.e3, 80, B, s);
    wgrad(n, 7, n.c3a, n.gA3, B, s);
    conv(n, 7, true, n.gA3, nullptr, n.c3a, n.gC3, 0, 0, B, s);
    wgrad(n, 6, n.p3, n.gC3, B, s);
    conv(n, 6, true, n.gC3, nullptr, nullptr, n.gP3, 0, 0, B, s);
    pool_bwd(n, 2, n.gP3, n.gS2, n.e2, 1, 48, B, s);                        // gS2 += ..., masked
    wgrad(n, 5, n.c2a, n.gS2, B, s);
    conv(n, 5, true, n.gS2, nullptr, n.c2a, n.gA2, 0, 0, B, s);            // gC2
    wgrad(n, 4, n.p2, n.gA2, B, s);
    conv(n, 4, true, n.gA2, nullptr, nullptr, n.gP2, 0, 0, B, s);
    pool_bwd(n, 1, n.gP2, n.gS1, n.e1, 1, 16, B, s);
    wgrad(n, 3, n.c1a, n.gS1, B, s);
    conv(n, 3, true, n.gS1, nullptr, n.c1a, n.gA1, 0, 0, B, s);            // gC1
    wgrad(n, 2, n.p1, n.gA1, B, s);
    conv(n, 2, true, n.gA1, nullptr, nullptr, n.gP1, 0, 0, B, s);
    pool_bwd(n, 0, n.gP1, n.gS0, n.e0, 1, 16, B, s);
    wgrad(n, 1, n.c0a, n.gS0, B, s);
    conv(n, 1, true, n.gS0, nullptr, n.c0a, n.gA0, 0, 0, B, s);            // gC0
    wgrad(n, 0, n.x, n.gA0, B, s);
}

}  // namespace

// ---- layer table and workspace ---------------------------------------------------
void pc_describe(PcNet &n, int nr, int nz, int batch)
{
    static const int spec[PC_LAYERS][5] = {
        // cin, cout, level, up_in, relu
        {2, 16, 0, 0, 1},  {16, 16, 0, 0, 1}, {16, 16, 1, 0, 1}, {16, 16, 1, 0, 1},
        {16, 48, 2, 0, 1}, {48, 48, 2, 0, 1}, {48, 80, 3, 0, 1}, {80, 80, 3, 0, 1},
        {80, 48, 2, 1, 1}, {48, 48, 2, 0, 1}, {48, 16, 1, 1, 1}, {16, 16, 1, 0, 1},
        {16, 16, 0, 1, 1}, {16, 16, 0, 0, 1}, {16, 1, 0, 0, 0}};
    memset(&n, 0, sizeof(n));
    n.batch = batch;
    n.H[0] = nz + 1;
    n.W[0] = nr + 1;
    for (int l = 1; l < PC_LEVELS; ++l) {
        n.H[l] = (n.H[l - 1] + 1) / 2;
        n.W[l] = (n.W[l - 1] + 1) / 2;
    }
    int64_t om = 0, owf = 0, owt = 0, ob = 0, of = 0;
    for (int k = 0; k < PC_LAYERS; ++k) {
        PcLayer &l = n.L[k];
        l.cin = spec[k][0];
        l.cout = spec[k][1];
        l.level = spec[k][2];
        l.up_in = spec[k][3];
        l.relu = spec[k][4];
        l.cin_p = (int)round_up(l.cin, 4);
        l.cout_p = (int)round_up(l.cout, 4);
        l.nt = (l.cout + 15) / 16;
        l.nt_t = (l.cin + 15) / 16;
        l.kpad = (int)round_up(9 * l.cin_p, 32);   // whole 32-deep MFMA steps
        l.kpad_t = (int)round_up(9 * l.cout_p, 32);
        l.kw = (int)round_up(9 * l.cin_p + 1, 16);
        l.o_master = om;
        l.o_wf = owf;
        l.o_wt = owt;
        l.o_bias = ob;
        l.o_flat = of;
        om += (int64_t)l.nt * 16 * l.kw;
        owf += (int64_t)l.nt * 16 * l.kpad;
        owt += (int64_t)l.nt_t * 16 * l.kpad_t;
        ob += l.cout_p;
        of += (int64_t)l.cout * l.cin * 9 + l.cout;
    }
    n.n_master = om;
    n.n_flat = of;
    n.out_scale = 1.0;
}

namespace {
struct PcCarve {
    char *base;
    int64_t off = 0;
    template <typename P>
    P *take(int64_t count)
    {
        off = round_up(off, 256);
        P *p = base ? (P *)(base + off) : nullptr;
        off += count * (int64_t)sizeof(P);
        return p;
    }
};

int64_t pc_carve(PcNet &n, char *base)
{
    PcCarve c{base};
    const int64_t B = n.batch;
    int64_t P[PC_LEVELS];
    for (int l = 0; l < PC_LEVELS; ++l) P[l] = (int64_t)n.H[l] * n.W[l] * B;
    int64_t nbias = 0, nwf = 0, nwt = 0, npart = 0;
    for (int k = 0; k < PC_LAYERS; ++k) {
        const PcLayer &l = n.L[k];
        nbias += l.cout_p;
        nwf += (int64_t)l.nt * 16 * l.kpad;
        nwt += (int64_t)l.nt_t * 16 * l.kpad_t;
        npart = std::max<int64_t>(npart, (int64_t)wgrad_splits(l) * l.nt * 16 * l.kw);
    }
    n.master = c.take<float>(n.n_master);
    n.grad = c.take<float>(n.n_master);
    n.adam_m = c.take<float>(n.n_master);
    n.adam_v = c.take<float>(n.n_master);
    n.bias = c.take<float>(nbias);
    n.wf = c.take<short>(nwf);
    n.wt = c.take<short>(nwt);
    n.partial = c.take<float>(npart);
    n.x = c.take<float>(P[0] * 4);
    n.c0a = c.take<float>(P[0] * 16);
    n.e0 = c.take<float>(P[0] * 16);
    n.d0a = c.take<float>(P[0] * 16);
    n.d0 = c.take<float>(P[0] * 16);
    n.out = c.take<float>(P[0] * 4);
    n.p1 = c.take<float>(P[1] * 16);
    n.c1a = c.take<float>(P[1] * 16);
    n.e1 = c.take<float>(P[1] * 16);
    n.d1a = c.take<float>(P[1] * 16);
    n.d1 = c.take<float>(P[1] * 16);
    n.p2 = c.take<float>(P[2] * 16);
    n.c2a = c.take<float>(P[2] * 48);
    n.e2 = c.take<float>(P[2] * 48);
    n.d2a = c.take<float>(P[2] * 48);
    n.d2 = c.take<float>(P[2] * 48);
    n.p3 = c.take<float>(P[3] * 48);
    n.c3a = c.take<float>(P[3] * 80);
    n.e3 = c.take<float>(P[3] * 80);
    n.g_out = c.take<float>(P[0] * 4);
    n.gA0 = c.take<float>(P[0] * 16);
    n.gS0 = c.take<float>(P[0] * 16);
    n.gA1 = c.take<float>(P[1] * 16);
    n.gS1 = c.take<float>(P[1] * 16);
    n.gB1 = c.take<float>(P[1] * 48);
    n.gP1 = c.take<float>(P[1] * 16);
    n.gA2 = c.take<float>(P[2] * 48);
    n.gS2 = c.take<float>(P[2] * 48);
    n.gB2 = c.take<float>(P[2] * 80);
    n.gP2 = c.take<float>(P[2] * 16);
    n.gA3 = c.take<float>(P[3] * 80);
    n.gC3 = c.take<float>(P[3] * 80);
    n.gP3 = c.take<float>(P[3] * 48);
    n.tgt = c.take<float>(P[0]);
    n.vb = c.take<float>(P[0]);
    n.vx = c.take<float>(P[0]);
    n.vr = c.take<float>(P[0]);
    n.vz = c.take<float>(P[0]);
    n.scal = c.take<double>(4 * B);
    return c.off + 256;
}
}  // namespace

int64_t pc_bytes(const PcNet &n)
{
    PcNet t = n;
    return pc_carve(t, nullptr);
}

void pc_bind(PcNet &n, char *base) { pc_carve(n, base); }

bool pc_fits(const PcNet &n)
{
    for (int k = 0; k < PC_LAYERS; ++k) {
        const PcLayer &l = n.L[k];
        const ConvGeom cg = conv_geom(n.H[l.level], n.W[l.level]);
        if (conv_lds(cg, l.cin_p, l.kpad, 1) > CONV_LDS_LIMIT ||
            conv_lds(cg, l.cout_p, l.kpad_t, 1) > CONV_LDS_LIMIT)
            return false;
    }
    return true;
}

int pc_kernel_setup()
{
    const int lim = CONV_LDS_LIMIT;
    int e = 0;
    e |= (int)hipFuncSetAttribute((const void *)k_conv3x3<1, true>, hipFuncAttributeMaxDynamicSharedMemorySize, lim);
    e |= (int)hipFuncSetAttribute((const void *)k_conv3x3<1, false>, hipFuncAttributeMaxDynamicSharedMemorySize, lim);
    e |= (int)hipFuncSetAttribute((const void *)k_conv3x3<3, false>, hipFuncAttributeMaxDynamicSharedMemorySize, lim);
    e |= (int)hipFuncSetAttribute((const void *)k_conv3x3<5, false>, hipFuncAttributeMaxDynamicSharedMemorySize, lim);
    e |= (int)hipFuncSetAttribute((const void *)k_conv3x3_wgrad, hipFuncAttributeMaxDynamicSharedMemorySize, lim);
    return e;
}

// ---- parameters -----------------------------------------------------------------
void pc_pack(const PcNet &n, hipStream_t s)
{
    for (int k = 0; k < PC_LAYERS; ++k)
        hipLaunchKernelGGL(k_pack, dim3(64), dim3(EB), 0, s, n.L[k], (const float *)n.master, n.wf,
                           n.wt, n.bias);
}

void pc_upload(PcNet &n, const float *flat, hipStream_t s)
{
    std::vector<float> m((size_t)n.n_master, 0.0f);
    for (int k = 0; k < PC_LAYERS; ++k) {
        const PcLayer &l = n.L[k];
        const float *w = flat + l.o_flat;
        const float *b = w + (int64_t)l.cout * l.cin * 9;
        for (int o = 0; o < l.cout; ++o) {
            float *row = m.data() + l.o_master + (int64_t)o * l.kw;
            for (int c = 0; c < l.cin; ++c)
                for (int tap = 0; tap < 9; ++tap) row[tap * l.cin_p + c] = w[((int64_t)o * l.cin + c) * 9 + tap];
            row[9 * l.cin_p] = b[o];
        }
    }
    (void)hipMemcpyAsync(n.master, m.data(), m.size() * 4, hipMemcpyHostToDevice, s);
    launch_zero(n.adam_m, n.n_master * 4, s);
    launch_zero(n.adam_v, n.n_master * 4, s);
    launch_zero(n.grad, n.n_master * 4, s);
    (void)hipStreamSynchronize(s);
    n.adam_t = 0;
    pc_pack(n, s);
}

void pc_download_flat(const PcNet &n, const float *dev, float *flat, std::vector<float> &m)
{
    m.resize((size_t)n.n_master);
    (void)hipMemcpy(m.data(), dev, m.size() * 4, hipMemcpyDeviceToHost);
    for (int k = 0; k < PC_LAYERS; ++k) {
        const PcLayer &l = n.L[k];
        float *w = flat + l.o_flat;
        float *b = w + (int64_t)l.cout * l.cin * 9;
        for (int o = 0; o < l.cout; ++o) {
            const float *row = m.data() + l.o_master + (int64_t)o * l.kw;
            for (int c = 0; c < l.cin; ++c)
                for (int tap = 0; tap < 9; ++tap) w[((int64_t)o * l.cin + c) * 9 + tap] = row[tap * l.cin_p + c];
            b[o] = row[9 * l.cin_p];
        }
    }
}

// ---- application ------------------------------------------------------------------
namespace {
// z = post(x1 + correction(r - A x1), r), x1 = pre(r), all FP32 on level L
__global__ void k_copy32(const float *a, float *b, int64_t n)
{
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n;
         k += (int64_t)gridDim.x * blockDim.x)
        b[k] = a[k];
}

void copy32(const float *a, float *b, int64_t n, hipStream_t s)
{
    if (a == b) return;
    hipLaunchKernelGGL(k_copy32, dim3(eblocks(n)), dim3(EB), 0, s, a, b, n);
}

// x1 of one right-hand side r (float, level 0) into x: the Gauss-Seidel pair
// from zero, or a multigrid V-cycle through the hierarchy's level-0 buffers
void pre_step(const PcPre &pre, const MGLevel &L, const float *r, float *x, int64_t nn,
              hipStream_t s)
{
    const dim3 g(rblocks(nn), 1);
    const float *nf = nullptr;
    double *nd = nullptr;
    if (pre.H) {
        const MGLevel &F = pre.H->lv[0];
        copy32(r, F.b, nn, s);
        launch_mg_vcycle(*pre.H, nullptr, s, pre.two_level);
        copy32(F.xu, x, nn, s);
    } else {
        hipLaunchKernelGGL(k_rb_sweep, g, dim3(RB), 0, s, L, r, x, nn, 0, 1, nf, nf, nd, nd);
        hipLaunchKernelGGL(k_rb_sweep, g, dim3(RB), 0, s, L, r, x, nn, 1, 0, nf, nf, nd, nd);
    }
}

void sandwich(PcNet &n, const PcPre &pre, const MGLevel &L, double inv_nunk, const float *r,
              float *z, const float *q, double *rz, double *zq, double *ss, hipStream_t s)
{
    const int64_t nn = (int64_t)(L.nr + 1) * (L.nz + 1);
    const dim3 g(rblocks(nn), 1);
    const float *nf = nullptr;
    double *nd = nullptr;
    pre_step(pre, L, r, n.vx, nn, s);
    hipLaunchKernelGGL(k_residual32, g, dim3(RB), 0, s, L, r, (const float *)n.vx, n.vr, nn, ss);
    hipLaunchKernelGGL(k_pc_input<float>, dim3(eblocks(nn)), dim3(EB), 0, s, (const float *)n.vr,
                       nn, 1.0, (const double *)ss, inv_nunk, L, n.x, 1);
    forward(n, 1, s);
    hipLaunchKernelGGL(k_pc_combine, dim3(eblocks(nn)), dim3(EB), 0, s, (const float *)n.out,
                       (const double *)ss, inv_nunk, n.out_scale, L, (const float *)n.vx, z);
    hipLaunchKernelGGL(k_rb_sweep, g, dim3(RB), 0, s, L, r, z, nn, 1, 0, nf, nf, nd, nd);
    hipLaunchKernelGGL(k_rb_sweep, g, dim3(RB), 0, s, L, r, z, nn, 0, 0, r, q, rz, q ? zq : nd);
}
}  // namespace

void pc_apply32(PcNet &n, const PcPre &pre, const MGLevel &L, int64_t n_unknown, const float *r,
                float *z, const float *q, double *rz, double *zq, double *ss, hipStream_t s)
{
    const double inv = n_unknown > 0 ? 1.0 / (double)n_unknown : 0.0;
    sandwich(n, pre, L, inv, r, z, q, rz, zq, ss, s);
}

void pc_apply64(PcNet &n, const PcPre &pre, const MGLevel &L, int64_t n_unknown, const double *r,
                double *z, double *ss, hipStream_t s)
{
    const int64_t nn = (int64_t)(L.nr + 1) * (L.nz + 1);
    const double inv = n_unknown > 0 ? 1.0 / (double)n_unknown : 0.0;
    launch_zero(ss, 8, s);
    hipLaunchKernelGGL(k_pc_scale_in<double>, dim3(eblocks(nn)), dim3(EB), 0, s, r, nn, 1.0,
                       (const double *)nullptr, inv, L, n.vb, 1);
    sandwich(n, pre, L, inv, n.vb, n.vz, nullptr, nullptr, nullptr, ss, s);
    hipLaunchKernelGGL(k_cast_out, dim3(eblocks(nn)), dim3(EB), 0, s, (const float *)n.vz, z, nn);
}

void pc_identity32(const MGLevel &L, const float *r, float *z, double *rz, hipStream_t s)
{
    const int64_t nn = (int64_t)(L.nr + 1) * (L.nz + 1);
    hipLaunchKernelGGL(k_pc_identity, dim3(rblocks(nn)), dim3(RB), 0, s, L, r, z, rz);
}

// ---- training -------------------------------------------------------------------------
// scal: [0, B) sum b^2, [B, 2B) sum r1^2, [2B, 3B) den, [3B] loss
void pc_train_enqueue(PcNet &n, const PcPre &pre, const MGLevel &L, int64_t n_unknown,
                      const double *q, const double *phi, int B, float lr, double inv_2pi_eps0,
                      hipStream_t s)
{
    const int64_t nn = (int64_t)(L.nr + 1) * (L.nz + 1);
    const double inv = n_unknown > 0 ? 1.0 / (double)n_unknown : 0.0;
    double *ss0 = n.scal, *ss1 = n.scal + B, *den = n.scal + 2 * B, *loss = n.scal + 3 * B;
    launch_zero(n.scal, 4 * (int64_t)B * 8, s);
    const dim3 gb(rblocks(nn), B);
    const dim3 gbe(std::min(eblocks((nn + 1) / 2), 1024), B);
    const float *nf = nullptr;
    double *nd = nullptr;
    hipLaunchKernelGGL(k_pc_sumsq<double>, gbe, dim3(EB), 0, s, q, nn, inv_2pi_eps0, L, ss0);
    hipLaunchKernelGGL(k_pc_scale_in<double>, dim3(eblocks((int64_t)B * nn)), dim3(EB), 0, s, q, nn,
                       inv_2pi_eps0, (const double *)ss0, inv, L, n.vb, B);
    if (pre.H) {
        for (int b = 0; b < B; ++b)
            pre_step(pre, L, (const float *)n.vb + (int64_t)b * nn, n.vx + (int64_t)b * nn, nn, s);
    } else {
        hipLaunchKernelGGL(k_rb_sweep, gb, dim3(RB), 0, s, L, (const float *)n.vb, n.vx, nn, 0,
                           1, nf, nf, nd, nd);
        hipLaunchKernelGGL(k_rb_sweep, gb, dim3(RB), 0, s, L, (const float *)n.vb, n.vx, nn, 1,
                           0, nf, nf, nd, nd);
    }
    hipLaunchKernelGGL(k_residual32, gb, dim3(RB), 0, s, L, (const float *)n.vb,
                       (const float *)n.vx, n.vr, nn, ss1);
    hipLaunchKernelGGL(k_pc_input<float>, dim3(eblocks((int64_t)B * nn)), dim3(EB), 0, s,
                       (const float *)n.vr, nn, 1.0, (const double *)ss1, inv, L, n.x, B);
    hipLaunchKernelGGL(k_pc_targets, gbe, dim3(EB), 0, s, phi, nn, (const double *)ss0,
                       (const double *)ss1, inv, (const float *)n.vx, L, n.tgt, den);
    forward(n, B, s);
    hipLaunchKernelGGL(k_pc_loss, gbe, dim3(EB), 0, s, (const float *)n.out, (const float *)n.tgt,
                       (const double *)den, n.out_scale, L, B, n.g_out, loss);
    backward(n, B, s);
    if (lr > 0.0f) {
        n.adam_t++;
        // beta1 = 0.9, beta2 = 0.999; 1 - beta and the bias corrections
        // 1 - beta^t in FP64, then rounded (in FP32, 1 - 0.999f^t cancels)
        const double B1 = 0.9, B2 = 0.999;
        const float c1 = (float)(1.0 - std::pow(B1, (double)n.adam_t));
        const float c2 = (float)(1.0 - std::pow(B2, (double)n.adam_t));
        hipLaunchKernelGGL(k_adam, dim3(eblocks(n.n_master)), dim3(EB), 0, s, n.master,
                           (const float *)n.grad, n.adam_m, n.adam_v, n.n_master, lr, (float)B1,
                           (float)B2, (float)(1.0 - B1), (float)(1.0 - B2), 1e-8f, c1, c2);
        pc_pack(n, s);
    }
}

const double *pc_loss_ptr(const PcNet &n, int B) { return n.scal + 3 * B; }

}  // namespace pic
