// unet.hip -- the learned denoiser: a U-Net (the network family the paper
// trains, Sec. IV-A-3) with bfloat16 weights and activations on the matrix
// cores (v_mfma_f32_16x16x32_bf16, float accumulation) and float master
// weights updated by Adam.
//
// Layout: activations NHWC bfloat16 with channels padded to a multiple of
// 16; forward weights [Cout_p][K_p] with k = tap * Cin_p + ci (K_p = 9 * Cin_p
// rounded up to 32, zero padded); input-gradient weights are the same
// convolution with the kernel flipped and the channel roles swapped, so one
// implicit-GEMM kernel serves the forward pass and the input gradient.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>

#include <algorithm>
#include <string>
#include <vector>

#include "sc_internal.h"
#include "sc_unet.h"

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef float float2v __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));

__device__ __forceinline__ uint16_t to_bf16(float f) {
    // round to nearest even
    uint32_t u = __float_as_uint(f);
    if ((u & 0x7f800000u) == 0x7f800000u) return (uint16_t)(u >> 16);   // inf / nan
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float from_bf16(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

union Frag {
    bf16x8 v;
    uint4 u;
};

// ---------------------------------------------------------------- convolution
// One wave computes 16 consecutive output pixels x 64 output channels (four
// 16x16 tiles sharing the pixel operand).  Lane l feeds pixel l%16 and the
// k-group 8*(l/16)..+7 of the A operand, output channel l%16 of each B tile,
// and receives pixels 4*(l/16)+i of channel l%16.
template <int KS>
__global__ __launch_bounds__(256) void k_conv(const uint16_t* __restrict__ X, uint32_t P, uint32_t H, uint32_t W,
                                              uint32_t cin_p, const uint16_t* __restrict__ Wt, uint32_t kpad,
                                              const float* __restrict__ bias, uint32_t cout_p, uint32_t cout_real,
                                              uint16_t* __restrict__ Y, float* __restrict__ Yf, uint32_t y_stride,
                                              uint32_t y_off, int relu, const uint16_t* __restrict__ M) {
    const uint32_t lane = threadIdx.x & 63;
    const uint32_t wave = (blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const uint32_t n_groups = (cout_p / 16 + 3) / 4;
    const uint32_t tile = wave / n_groups;
    const uint32_t grp = wave % n_groups;
    const uint32_t n_tiles = (P + 15) / 16;
    if (tile >= n_tiles) return;
    const uint32_t nt_total = cout_p / 16;
    const uint32_t pl = lane & 15, g = lane >> 4;
    const uint32_t p = tile * 16 + pl;
    const bool pvalid = p < P;
    uint32_t x = 0, y = 0;
    if (KS == 3 && pvalid) {   // a 1x1 convolution needs no pixel coordinates
        const uint32_t rest = p / W;
        x = p - rest * W;
        y = rest % H;
    }
    const uint32_t K = KS * KS * cin_p;
    floatx4 acc[4];
    for (int j = 0; j < 4; ++j) acc[j] = floatx4{0.0f, 0.0f, 0.0f, 0.0f};
    // this lane's k-group (8 channels of one tap, as cin_p is a multiple of
    // 16) advances by 32 per step: tap and channel are carried along
    uint32_t tap = (8 * g) / cin_p, ci = (8 * g) % cin_p;
    const size_t pix0 = p;   // = (b H + y) W + x
    for (uint32_t k0 = 0; k0 < kpad; k0 += 32) {
        const uint32_t kk = k0 + 8 * g;
        Frag a;
        a.u = make_uint4(0u, 0u, 0u, 0u);
        if (pvalid && kk < K) {
            const int dy = KS == 3 ? (int)(tap >= 6 ? 2 : (tap >= 3 ? 1 : 0)) - 1 : 0;
            const int dx = KS == 3 ? (int)(tap - 3 * (uint32_t)(dy + 1)) - 1 : 0;
            const int yy = (int)y + dy, xx = (int)x + dx;
            if (yy >= 0 && yy < (int)H && xx >= 0 && xx < (int)W) {
                const size_t src = (size_t)((long long)pix0 + (long long)dy * W + dx) * cin_p + ci;
                a.u = *reinterpret_cast<const uint4*>(X + src);
            }
        }
        ci += 32;
        while (ci >= cin_p) {
            ci -= cin_p;
            ++tap;
        }
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const uint32_t nt = grp * 4 + j;
            if (nt < nt_total) {
                Frag bw;
                const uint32_t co = nt * 16 + pl;
                bw.u = *reinterpret_cast<const uint4*>(Wt + (size_t)co * kpad + kk);
                acc[j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a.v, bw.v, acc[j], 0, 0, 0);
            }
        }
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const uint32_t nt = grp * 4 + j;
        if (nt >= nt_total) continue;
        const uint32_t co = nt * 16 + pl;
        if (co >= cout_real) continue;
        const float bv = bias ? bias[co] : 0.0f;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const uint32_t po = tile * 16 + 4 * g + i;
            if (po >= P) continue;
            float v = acc[j][i] + bv;
            if (relu) v = fmaxf(v, 0.0f);
            const size_t o = (size_t)po * y_stride + y_off + co;
            if (Yf) {
                Yf[o] = v;
            } else {
                // M: the ReLU output this gradient flows back through (zero where it is not positive)
                Y[o] = M && !(from_bf16(M[o]) > 0.0f) ? (uint16_t)0 : to_bf16(v);
            }
        }
    }
}

// 3x3 convolution on the matrix cores.  A block owns 16 NT output channels
// (blockIdx.y selects the group) and walks pixel tiles of 4 RW x 16 with a
// stride of the grid; wave w computes tile rows RW w .. RW w + RW - 1.  The
// input channels are taken 32 at a time: the tile with its 1-pixel halo and
// the 16 NT x 9 x 32 weights of the chunk are staged in LDS, then every tap
// reads its operands there.  While a chunk is multiplied, the input pixels of
// the next (tile, chunk) are already being loaded into registers.  With one
// chunk (MODE 0: cin_p <= 32) the weights are staged once per block.  The
// operands are weights x pixels, so a lane receives 4 consecutive output
// channels of one pixel and writes them with one 8-byte store.  Channels past
// cin_p in the last chunk are zero in both tiles.  MODE 2: the input is the
// concatenation [nearest 2x upsampling of X (c_split channels at H/2 x W/2),
// X2 (cin_p - c_split channels)], read in place (decoder inference).  Every
// output sums chunk by chunk and tap by tap, so neither the tile shape nor the
// grid changes a result.  Element indices of one tensor fit in 32 bits (the
// host checks P * channels < 2^31); H and W are even.  M (input gradients
// only): the ReLU output of the layer below, laid out as Y; outputs where it
// is not positive are written as zero.
constexpr int kTC = 16, kHC = kTC + 2;
constexpr int kCC = 32;                 // input channels per chunk
constexpr int kWP = 9 * kCC + 8;        // LDS pitch of a weight row (bf16), padded against bank conflicts
constexpr int kConvTiles = 2;           // 16-channel output tiles per block
constexpr int kBigRW = 3;               // pixel rows per wave of the large tiles

template <int NT, int RW, int MODE>
__global__ __launch_bounds__(256) void k_conv3(const uint16_t* __restrict__ X, const uint16_t* __restrict__ X2,
                                               uint32_t c_split, uint32_t B, uint32_t H, uint32_t W, uint32_t cin_p,
                                               const uint16_t* __restrict__ Wt, uint32_t kpad,
                                               const float* __restrict__ bias, uint32_t cout_p,
                                               uint16_t* __restrict__ Y, uint32_t y_stride, int relu,
                                               const uint16_t* __restrict__ M) {
    constexpr int kTR = 4 * RW, kHR = kTR + 2;
    constexpr int kXS = kHR * kHC * 4;       // 16-byte pieces of a staged tile
    constexpr int kXI = (kXS + 255) / 256;   // ... per thread
    __shared__ uint4 xs4[kXS];
    __shared__ uint4 ws4[16 * NT * kWP / 8];
    const uint16_t* xs = reinterpret_cast<const uint16_t*>(xs4);
    const uint16_t* ws = reinterpret_cast<const uint16_t*>(ws4);
    const uint32_t tid = threadIdx.x, lane = tid & 63, wv = tid >> 6, pl = lane & 15, g = lane >> 4;
    const uint32_t piece = tid & 3;          // this thread's 8-channel piece in every staged pixel
    const uint32_t tiles_x = (W + kTC - 1) / kTC, tiles_y = (H + kTR - 1) / kTR;
    const uint32_t n_tiles = tiles_x * tiles_y * B;
    const uint32_t cg = blockIdx.y;
    const uint32_t nt_here = min((uint32_t)NT, cout_p / 16 - cg * NT);   // 16-channel tiles of this group
    const uint32_t n_chunks = (cin_p + kCC - 1) / kCC;
    const uint32_t Hh = H / 2, Wh = W / 2, c_rest = cin_p - c_split;
    // this thread's staged pixels: row and column in the haloed tile and the
    // element offset from the tile's corner pixel (y0 - 1, x0 - 1) (MODE 2:
    // from the upsampled corner and, for X2, from the corner)
    int32_t so[kXI], so2[kXI];
#pragma unroll
    for (int k = 0; k < kXI; ++k) {
        const uint32_t t = tid + 256 * k, pix = t >> 2;
        const bool in = t < kXS;
        const uint32_t sy = pix / kHC, sx = pix % kHC;
        if (MODE == 2) {
            const int fy = (int)((sy + 1) / 2) - 1, fx = (int)((sx + 1) / 2) - 1;
            so[k] = in ? (fy * (int)Wh + fx) * (int)c_split + (int)piece * 8 : 0;
            so2[k] = in ? ((int)sy * (int)W + (int)sx) * (int)c_rest + (int)piece * 8 : 0;
        } else {
            so[k] = in ? ((int)sy * (int)W + (int)sx) * (int)cin_p + (int)piece * 8 : 0;
            so2[k] = 0;
        }
    }
    auto corner = [&](uint32_t tile, uint32_t& b, uint32_t& y0, uint32_t& x0) {
        const uint32_t tx = tile % tiles_x, rest = tile / tiles_x;
        x0 = tx * kTC;
        y0 = (rest % tiles_y) * kTR;
        b = rest / tiles_y;
    };
    auto fetch = [&](uint32_t tile, uint32_t c0, uint4 (&v)[kXI]) {
        uint32_t b, y0, x0;
        corner(tile, b, y0, x0);
        const uint32_t cn = min((uint32_t)kCC, cin_p - c0);
        const bool pok = piece * 8 < cn;
        const int64_t corner_px = ((int64_t)(b * H + y0) - 1) * W + (int64_t)x0 - 1;
        const uint16_t* src;
        const uint16_t* src2 = nullptr;
        bool up = false;
        if (MODE == 2) {
            up = c0 + piece * 8 < c_split;
            src = X + ((int64_t)(b * Hh + y0 / 2) * Wh + x0 / 2) * c_split + c0;
            src2 = X2 + corner_px * c_rest + ((int64_t)c0 - (int64_t)c_split);
        } else {
            src = X + corner_px * cin_p + c0;
        }
        // tiles whose halo lies inside the image (most of them) need no
        // per-pixel bounds checks; the others recompute each pixel's place
        const bool inner = y0 >= 1 && y0 + kTR + 1 <= H && x0 >= 1 && x0 + kTC + 1 <= W;
#pragma unroll
        for (int k = 0; k < kXI; ++k) {
            v[k] = make_uint4(0u, 0u, 0u, 0u);
            const uint32_t t = tid + 256 * k;
            bool ok = pok && (k + 1 < kXI || t < (uint32_t)kXS);
            if (ok && !inner) {
                const uint32_t pix = t >> 2, sy = pix / kHC, sx = pix - sy * kHC;
                ok = y0 - 1u + sy < H && x0 - 1u + sx < W;   // -1 wraps to a large value
            }
            if (ok) {
                if (MODE == 2 && !up)
                    v[k] = *reinterpret_cast<const uint4*>(src2 + so2[k]);
                else
                    v[k] = *reinterpret_cast<const uint4*>(src + so[k]);
            }
        }
    };
    uint32_t tile = blockIdx.x, chunk = 0;
    if (tile >= n_tiles) return;   // the whole block
    uint4 pv[kXI];
    fetch(tile, 0, pv);
    floatx4 acc[RW][NT];
#pragma unroll
    for (int r = 0; r < RW; ++r)
#pragma unroll
        for (int j = 0; j < NT; ++j) acc[r][j] = floatx4{0.0f, 0.0f, 0.0f, 0.0f};
    bool w_staged = false;
    while (true) {
        const uint32_t c0 = chunk * kCC;
        __syncthreads();   // the previous item's operands are no longer read
#pragma unroll
        for (int k = 0; k < kXI; ++k)
            if (tid + 256 * k < (uint32_t)kXS) xs4[tid + 256 * k] = pv[k];
        if (MODE != 0 || !w_staged) {
            const uint32_t cn = min((uint32_t)kCC, cin_p - c0);
            const uint16_t* wsrc = Wt + (size_t)(cg * 16 * NT) * kpad + c0;
            for (uint32_t t = tid; t < 16 * nt_here * 9 * 4; t += 256) {
                const uint32_t rest = t >> 2;
                const uint32_t col = rest / 9, tap = rest - col * 9;
                uint4 v = make_uint4(0u, 0u, 0u, 0u);
                if (piece * 8 < cn) v = *reinterpret_cast<const uint4*>(wsrc + col * kpad + tap * cin_p + piece * 8);
                ws4[(col * kWP + tap * kCC) / 8 + piece] = v;
            }
            w_staged = true;
        }
        __syncthreads();
        uint32_t ntile = tile, nchunk = chunk + 1;
        if (nchunk == n_chunks) {
            nchunk = 0;
            ntile += gridDim.x;
        }
        const bool more = ntile < n_tiles;
        if (more) fetch(ntile, nchunk * kCC, pv);   // in flight while this item is multiplied
#pragma unroll
        for (int tap = 0; tap < 9; ++tap) {
            const int dy = tap / 3, dx = tap % 3;
            Frag px[RW];
#pragma unroll
            for (int r = 0; r < RW; ++r)
                px[r].u = *reinterpret_cast<const uint4*>(xs + (((RW * wv + r + dy) * kHC) + pl + dx) * kCC + 8 * g);
#pragma unroll
            for (int j = 0; j < NT; ++j) {
                if ((uint32_t)j < nt_here) {
                    Frag wt;
                    wt.u = *reinterpret_cast<const uint4*>(ws + (j * 16 + pl) * kWP + tap * kCC + 8 * g);
#pragma unroll
                    for (int r = 0; r < RW; ++r)
                        acc[r][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wt.v, px[r].v, acc[r][j], 0, 0, 0);
                }
            }
        }
        if (chunk + 1 == n_chunks) {   // the tile is complete: channels 4 g .. 4 g + 3 of pixel pl
            uint32_t b, y0, x0;
            corner(tile, b, y0, x0);
#pragma unroll
            for (int r = 0; r < RW; ++r) {
                const uint32_t yy = y0 + RW * wv + r;
                if (yy < H && x0 + pl < W) {
                    uint16_t* dst = Y + (size_t)((b * H + yy) * W + x0 + pl) * y_stride + cg * NT * 16 + 4 * g;
#pragma unroll
                    for (int j = 0; j < NT; ++j) {
                        if ((uint32_t)j >= nt_here) continue;
                        const float* bj = bias + (cg * NT + j) * 16 + 4 * g;
                        float2v lo, hi;
                        lo[0] = acc[r][j][0] + (bias ? bj[0] : 0.0f);
                        lo[1] = acc[r][j][1] + (bias ? bj[1] : 0.0f);
                        hi[0] = acc[r][j][2] + (bias ? bj[2] : 0.0f);
                        hi[1] = acc[r][j][3] + (bias ? bj[3] : 0.0f);
                        if (relu) {
                            lo[0] = fmaxf(lo[0], 0.0f);
                            lo[1] = fmaxf(lo[1], 0.0f);
                            hi[0] = fmaxf(hi[0], 0.0f);
                            hi[1] = fmaxf(hi[1], 0.0f);
                        }
                        const bf16x2 l2 = __builtin_convertvector(lo, bf16x2);   // round to nearest even
                        const bf16x2 h2 = __builtin_convertvector(hi, bf16x2);
                        uint2 o;
                        __builtin_memcpy(&o.x, &l2, 4);
                        __builtin_memcpy(&o.y, &h2, 4);
                        if (M) {   // input gradient through a ReLU: zero where its output is not positive
                            const uint2 mk = *reinterpret_cast<const uint2*>(M + (dst - Y) + 16 * j);
                            o.x &= (from_bf16((uint16_t)mk.x) > 0.0f ? 0xFFFFu : 0u) |
                                   (from_bf16((uint16_t)(mk.x >> 16)) > 0.0f ? 0xFFFF0000u : 0u);
                            o.y &= (from_bf16((uint16_t)mk.y) > 0.0f ? 0xFFFFu : 0u) |
                                   (from_bf16((uint16_t)(mk.y >> 16)) > 0.0f ? 0xFFFF0000u : 0u);
                        }
                        *reinterpret_cast<uint2*>(dst + 16 * j) = o;
                    }
                }
#pragma unroll
                for (int j = 0; j < NT; ++j) acc[r][j] = floatx4{0.0f, 0.0f, 0.0f, 0.0f};
            }
        }
        if (!more) break;
        tile = ntile;
        chunk = nchunk;
    }
}

// 1x1 convolution to float outputs (the network's last layer, 16 padded
// output channels): each wave keeps the weights of up to kOutChunks k-chunks
// of 32 as MFMA operands and walks 16-pixel tiles with a stride of the grid.
// The operands are weights x pixels, so lane (pixel l%16, group l/16)
// receives output channels 4 (l/16) .. 4 (l/16) + 3 of its pixel.  The sums
// run over the k-chunks in order, as in k_conv.
constexpr uint32_t kOutChunks = 4;
__global__ __launch_bounds__(256) void k_conv1_out(const uint16_t* __restrict__ X, uint32_t P, uint32_t cin_p,
                                                   const uint16_t* __restrict__ Wt, uint32_t kpad,
                                                   const float* __restrict__ bias, uint32_t cout_real,
                                                   float* __restrict__ Yf, uint32_t y_stride, int relu) {
    const uint32_t lane = threadIdx.x & 63, pl = lane & 15, g = lane >> 4;
    const uint32_t wave = (blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const uint32_t n_waves = (gridDim.x * blockDim.x) >> 6;
    const uint32_t nk = kpad / 32;
    Frag wt[kOutChunks];
#pragma unroll
    for (uint32_t c = 0; c < kOutChunks; ++c) {
        wt[c].u = make_uint4(0u, 0u, 0u, 0u);
        if (c < nk && 32 * c + 8 * g < cin_p)
            wt[c].u = *reinterpret_cast<const uint4*>(Wt + pl * kpad + 32 * c + 8 * g);
    }
    float bv[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const uint32_t co = 4 * g + i;
        bv[i] = (co < cout_real && bias) ? bias[co] : 0.0f;
    }
    const uint32_t n_tiles = (P + 15) / 16;
    for (uint32_t t = wave; t < n_tiles; t += n_waves) {
        const uint32_t p = t * 16 + pl;
        floatx4 acc = floatx4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
        for (uint32_t c = 0; c < kOutChunks; ++c) {
            if (c < nk) {
                Frag px;
                px.u = make_uint4(0u, 0u, 0u, 0u);
                const uint32_t k = 32 * c + 8 * g;
                if (p < P && k < cin_p) px.u = *reinterpret_cast<const uint4*>(X + (size_t)p * cin_p + k);
                acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wt[c].v, px.v, acc, 0, 0, 0);
            }
        }
        if (p < P) {
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const uint32_t co = 4 * g + i;
                if (co >= cout_real) continue;
                float v = acc[i] + bv[i];
                if (relu) v = fmaxf(v, 0.0f);
                Yf[(size_t)p * y_stride + co] = v;
            }
        }
    }
}

// Weight gradient through LDS: dW[co][k] = sum_p dZ[p][co] * X[shift_tap(p)][ci]
// (k = tap * cin_p + ci).  A block owns 16 CT output channels x 64 KW
// columns k (CT = channel tiles, KW = 4 / CT waves per tile, each wave one
// channel tile x 4 column tiles) and a range of pixels, taken 32 at a time:
// dZ (16 CT channels) and the shifted input (64 KW columns, 8 consecutive
// channels of one tap per 16-byte load) are loaded with 16-byte loads and
// stored transposed in LDS ([channel][pixel]), so every MFMA operand (8
// pixels of one channel) is one 16-byte LDS read.  Partial sums meet in
// dW with float atomics.  cin_p and cout_p are multiples of 16.  The blocks
// of the first column group also sum their staged dZ over the pixels: the
// bias gradient gb (if not null), one float atomic per channel and block.
constexpr int kWgPx = 32;             // pixels per step
constexpr int kWgPitch = kWgPx + 8;   // LDS row pitch (bf16)
template <int KS, int CT>
__global__ __launch_bounds__(256) void k_wgrad_lds(const uint16_t* __restrict__ dZ, uint32_t cout_p,
                                                   const uint16_t* __restrict__ X, uint32_t cin_p, uint32_t P,
                                                   uint32_t H, uint32_t W, uint32_t chunk, float* __restrict__ gw,
                                                   uint32_t kreal, uint32_t cout, uint32_t cin,
                                                   float* __restrict__ gb) {
    constexpr int KW = 4 / CT;          // waves along k per channel tile
    constexpr int NB = 64 * KW;         // columns k of the block
    constexpr int TPC = 256 / (16 * CT);   // threads per channel of the bias sum (4, 8, 16)
    constexpr int PPT = kWgPx / TPC;       // ... each over 8, 4 or 2 pixels of a step
    __shared__ __align__(16) uint16_t dzT[16 * CT][kWgPitch];
    __shared__ __align__(16) uint16_t xT[NB][kWgPitch];
    const uint32_t tid = threadIdx.x, lane = tid & 63, wv = tid >> 6, pl = lane & 15, g = lane >> 4;
    const uint32_t co_groups = (cout_p / 16 + CT - 1) / CT;
    const uint32_t k_groups = (kreal + NB - 1) / NB;
    uint32_t bid = blockIdx.x;
    const uint32_t cgp = bid % co_groups;
    bid /= co_groups;
    const uint32_t kgp = bid % k_groups;
    const uint32_t ch = bid / k_groups;
    const uint32_t co0 = cgp * 16 * CT, k0 = kgp * NB;
    const uint32_t p_begin = ch * chunk, p_end = min(P, p_begin + chunk);
    const uint32_t ctile = wv / KW, kq = wv % KW;   // this wave: channel tile, quarter of the columns
    const bool wave_on = co0 + 16 * ctile < cout_p;
    const bool bias_sum = gb != nullptr && kgp == 0;
    const uint32_t bc = tid / TPC, bq = tid % TPC;   // bias sum: channel co0 + bc, pixels PPT bq ..
    float bsum = 0.0f;
    floatx4 acc[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[j] = floatx4{0.0f, 0.0f, 0.0f, 0.0f};
    for (uint32_t p0 = p_begin; p0 < p_end; p0 += kWgPx) {
        __syncthreads();   // the previous step's tiles are no longer read
        // dZ: 16 CT channels x 32 pixels, 8 channels per piece
        for (uint32_t t = tid; t < 2 * CT * kWgPx; t += 256) {
            const uint32_t px = t % kWgPx, c8 = t / kWgPx;
            const uint32_t p = p0 + px, c = co0 + 8 * c8;
            union {
                uint4 u;
                uint16_t h[8];
            } v;
            v.u = make_uint4(0u, 0u, 0u, 0u);
            if (p < p_end && c < cout_p) v.u = *reinterpret_cast<const uint4*>(dZ + (size_t)p * cout_p + c);
#pragma unroll
            for (int e = 0; e < 8; ++e) dzT[8 * c8 + e][px] = v.h[e];
        }
        // shifted input: NB columns x 32 pixels, 8 columns (8 channels of one tap) per piece
        for (uint32_t t = tid; t < NB / 8 * kWgPx; t += 256) {
            const uint32_t px = t % kWgPx, k8 = t / kWgPx;
            const uint32_t p = p0 + px, k = k0 + 8 * k8;
            union {
                uint4 u;
                uint16_t h[8];
            } v;
            v.u = make_uint4(0u, 0u, 0u, 0u);
            if (p < p_end && k < kreal) {
                const uint32_t tap = k / cin_p, ci = k - tap * cin_p;
                int dy = 0, dx = 0;
                if (KS == 3) {
                    dy = (int)(tap / 3) - 1;
                    dx = (int)(tap % 3) - 1;
                }
                const uint32_t rest = p / W, x = p - rest * W, y = rest % H;
                const int yy = (int)y + dy, xx = (int)x + dx;
                if (yy >= 0 && yy < (int)H && xx >= 0 && xx < (int)W)
                    v.u = *reinterpret_cast<const uint4*>(X + (size_t)((int)p + dy * (int)W + dx) * cin_p + ci);
            }
#pragma unroll
            for (int e = 0; e < 8; ++e) xT[8 * k8 + e][px] = v.h[e];
        }
        __syncthreads();
        if (bias_sum) {   // pixels past p_end are zero in the tile
            // one 16-, 8- or 4-byte LDS read (rows are 80 bytes apart)
            uint16_t h[PPT];
            const uint16_t* src = &dzT[bc][PPT * bq];
            if constexpr (PPT == 8) *reinterpret_cast<uint4*>(h) = *reinterpret_cast<const uint4*>(src);
            else if constexpr (PPT == 4) *reinterpret_cast<uint2*>(h) = *reinterpret_cast<const uint2*>(src);
            else *reinterpret_cast<uint32_t*>(h) = *reinterpret_cast<const uint32_t*>(src);
#pragma unroll
            for (int e = 0; e < PPT; ++e) bsum += from_bf16(h[e]);
        }
        if (wave_on) {
            Frag a;
            a.u = *reinterpret_cast<const uint4*>(&dzT[16 * ctile + pl][8 * g]);
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                Frag b;
                b.u = *reinterpret_cast<const uint4*>(&xT[64 * kq + 16 * j + pl][8 * g]);
                // D[m = channel][n = column]: A = dZ^T (channels x pixels), B = X_shift (pixels x columns)
                acc[j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a.v, b.v, acc[j], 0, 0, 0);
            }
        }
    }
    if (bias_sum) {   // the TPC threads of a channel are adjacent lanes of one wave
#pragma unroll
        for (int off = TPC / 2; off > 0; off /= 2) bsum += __shfl_xor(bsum, off, 64);
        if (bq == 0 && co0 + bc < cout) atomicAdd(&gb[co0 + bc], bsum);
    }
    if (!wave_on) return;
    // lane holds D[channel 16 ctile + 4 g + i][column 64 kq + 16 j + pl]; the
    // real (unpadded) entries go to the parameter gradient [cout][tap][cin]
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const uint32_t k = k0 + 64 * kq + 16 * j + pl;
        if (k >= kreal) continue;
        const uint32_t tap = k / cin_p, ci = k - tap * cin_p;
        if (ci >= cin) continue;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const uint32_t c = co0 + 16 * ctile + 4 * g + i;
            if (c < cout) atomicAdd(&gw[((size_t)c * (KS * KS) + tap) * cin + ci], acc[j][i]);
        }
    }
}

// ---------------------------------------------------------------- elementwise
// 2x2 max pooling, 8 channels (16 bytes) per step; the arg-max (0..3, the
// first of equal maxima) is kept for the backward pass.  H and W are even and
// C a multiple of 8; element indices fit in 32 bits.
__global__ void k_maxpool(const uint16_t* __restrict__ X, uint32_t B, uint32_t H, uint32_t W, uint32_t C,
                          uint16_t* __restrict__ Y, uint8_t* __restrict__ idx) {
    const uint32_t h = H / 2, w = W / 2, c8n = C / 8;
    const uint32_t n = B * h * w * c8n;
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        const uint32_t pix = i / c8n, c = (i - pix * c8n) * 8;
        const uint32_t by = pix / w, x = pix - by * w;   // by = b h + y, so the input rows are 2 by and 2 by + 1
        union {
            uint4 u;
            uint16_t h[8];
        } q[4], out;
#pragma unroll
        for (uint32_t k = 0; k < 4; ++k)
            q[k].u = *reinterpret_cast<const uint4*>(X + (size_t)((2 * by + (k >> 1)) * W + 2 * x + (k & 1)) * C + c);
        uint32_t bi[2] = {0u, 0u};
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            float best = -INFINITY;
            uint32_t sel = 0;
            uint16_t bvv = 0;
#pragma unroll
            for (uint32_t k = 0; k < 4; ++k) {
                const float f = from_bf16(q[k].h[e]);
                if (f > best) {
                    best = f;
                    sel = k;
                    bvv = q[k].h[e];
                }
            }
            out.h[e] = bvv;
            bi[e >> 2] |= sel << (8 * (e & 3));
        }
        reinterpret_cast<uint4*>(Y)[i] = out.u;
        reinterpret_cast<uint2*>(idx)[i] = make_uint2(bi[0], bi[1]);
    }
}

// dX = scatter of dY to the arg-max position (+ add, the skip gradient),
// then zero where M (the ReLU output at dX's place, if not null) is not
// positive.  8 channels (16 bytes) per step; C is a multiple of 8.
__global__ void k_maxpool_bwd(const uint16_t* __restrict__ dY, const uint8_t* __restrict__ idx, uint32_t B,
                              uint32_t H, uint32_t W, uint32_t C, const uint16_t* __restrict__ add,
                              const uint16_t* __restrict__ M, uint16_t* __restrict__ dX) {
    const uint32_t c8n = C / 8;
    const size_t n = (size_t)B * H * W * c8n;
    const uint32_t w = W / 2, h = H / 2;
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
        const uint32_t c8 = i % c8n;
        size_t r = i / c8n;
        const uint32_t x = r % W;
        r /= W;
        const uint32_t y = r % H;
        const uint32_t b = r / H;
        const size_t o = (((size_t)b * h + y / 2) * w + x / 2) * C + 8 * c8;
        const uint8_t q = (uint8_t)(((y & 1) << 1) | (x & 1));
        union {
            uint4 u;
            uint16_t h[8];
        } g, a, m, out;
        union {
            uint2 u;
            uint8_t b[8];
        } ix;
        g.u = *reinterpret_cast<const uint4*>(dY + o);
        ix.u = *reinterpret_cast<const uint2*>(idx + o);
        a.u = add ? reinterpret_cast<const uint4*>(add)[i] : make_uint4(0u, 0u, 0u, 0u);
        m.u = M ? reinterpret_cast<const uint4*>(M)[i] : make_uint4(0u, 0u, 0u, 0u);
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            float v = ix.b[e] == q ? from_bf16(g.h[e]) : 0.0f;
            if (add) v += from_bf16(a.h[e]);
            out.h[e] = M && !(from_bf16(m.h[e]) > 0.0f) ? (uint16_t)0 : to_bf16(v);
        }
        reinterpret_cast<uint4*>(dX)[i] = out.u;
    }
}

// C[b,y,x,:] = [ D[b,y/2,x/2,:cu] | E[b,y,x,:ce] ]
// 8 channels (16 bytes) per step; cu and ce are multiples of 16
__global__ void k_upcat(const uint16_t* __restrict__ D, uint32_t cu, const uint16_t* __restrict__ E, uint32_t ce,
                        uint32_t B, uint32_t H, uint32_t W, uint16_t* __restrict__ Cc) {
    const uint32_t ct8 = (cu + ce) / 8;
    const size_t n = (size_t)B * H * W * ct8;
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
        const uint32_t c = (uint32_t)(i % ct8) * 8;
        const size_t pix = i / ct8;
        const uint32_t x = pix % W;
        const size_t r = pix / W;
        const uint32_t y = r % H;
        const uint32_t b = r / H;
        const uint16_t* src = c < cu ? D + (((size_t)b * (H / 2) + y / 2) * (W / 2) + x / 2) * cu + c
                                     : E + pix * ce + (c - cu);
        reinterpret_cast<uint4*>(Cc)[i] = *reinterpret_cast<const uint4*>(src);
    }
}

// dD = sum over each 2x2 block of the first cu channels, zero where M (the
// ReLU output that was upsampled, if not null) is not positive; dE = the
// rest.  8 channels (16 bytes) per step; cu and ce are multiples of 8.
__global__ void k_upcat_bwd(const uint16_t* __restrict__ dC, uint32_t cu, uint32_t ce, uint32_t B, uint32_t H,
                            uint32_t W, const uint16_t* __restrict__ M, uint16_t* __restrict__ dD,
                            uint16_t* __restrict__ dE) {
    const uint32_t ct = cu + ce, cu8 = cu / 8, ce8 = ce / 8;
    const uint32_t h = H / 2, w = W / 2;
    union V {
        uint4 u;
        uint16_t h[8];
    };
    const size_t nd = (size_t)B * h * w * cu8;
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < nd; i += (size_t)gridDim.x * blockDim.x) {
        const uint32_t c = (uint32_t)(i % cu8) * 8;
        size_t r = i / cu8;
        const uint32_t x = r % w;
        r /= w;
        const uint32_t y = r % h;
        const uint32_t b = r / h;
        float s[8] = {0, 0, 0, 0, 0, 0, 0, 0};
        for (uint32_t q = 0; q < 4; ++q) {
            const uint32_t yy = 2 * y + (q >> 1), xx = 2 * x + (q & 1);
            V v;
            v.u = *reinterpret_cast<const uint4*>(dC + (((size_t)b * H + yy) * W + xx) * ct + c);
#pragma unroll
            for (int e = 0; e < 8; ++e) s[e] += from_bf16(v.h[e]);
        }
        V m, out;
        m.u = M ? reinterpret_cast<const uint4*>(M)[i] : make_uint4(0u, 0u, 0u, 0u);
#pragma unroll
        for (int e = 0; e < 8; ++e) out.h[e] = M && !(from_bf16(m.h[e]) > 0.0f) ? (uint16_t)0 : to_bf16(s[e]);
        reinterpret_cast<uint4*>(dD)[i] = out.u;
    }
    const size_t ne = (size_t)B * H * W * ce8;
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < ne; i += (size_t)gridDim.x * blockDim.x)
        reinterpret_cast<uint4*>(dE)[i] = *reinterpret_cast<const uint4*>(dC + (i / ce8) * ct + cu + 8 * (i % ce8));
}

// network input: float [P][in_ch] -> bf16 [P][cin_p] (zero padded channels)
__global__ void k_pack_input(const float* __restrict__ f, uint32_t P, uint32_t in_ch, uint32_t cin_p,
                             uint16_t* __restrict__ X) {
    const size_t n = (size_t)P * cin_p;
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
        const uint32_t c = i % cin_p;
        X[i] = c < in_ch ? to_bf16(f[(i / cin_p) * in_ch + c]) : (uint16_t)0;
    }
}

// The network's 9 input features of pixel p of a render: log(1 + rgb)
// (negative radiance clamped to 0), grey albedo, world normal, normalised
// depth, transparent bit; absent buffers give 0.  The only definition of
// the feature map: inference (k_features) and training inputs
// (k_features_f32, sc_unet_features) both use it.
__device__ __forceinline__ void feature9(const float* __restrict__ rgb, const float* __restrict__ albedo,
                                         const float* __restrict__ normal, const float* __restrict__ depthn,
                                         const uint8_t* __restrict__ trans, uint32_t p, float* v) {
    for (int c = 0; c < 3; ++c) v[c] = log1pf(fmaxf(rgb[3 * (size_t)p + c], 0.0f));
    v[3] = albedo ? albedo[p] : 0.0f;
    for (int c = 0; c < 3; ++c) v[4 + c] = normal ? normal[3 * (size_t)p + c] : 0.0f;
    v[7] = depthn ? depthn[p] : 0.0f;
    v[8] = trans ? (float)trans[p] : 0.0f;
}

// features as float [h][w][9] (the training input of sc_unet_train_step)
__global__ void k_features_f32(const float* __restrict__ rgb, const float* __restrict__ albedo,
                               const float* __restrict__ normal, const float* __restrict__ depthn,
                               const uint8_t* __restrict__ trans, uint32_t n, float* __restrict__ F) {
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        float v[9];
        feature9(rgb, albedo, normal, depthn, trans, i, v);
#pragma unroll
        for (int c = 0; c < 9; ++c) F[9 * (size_t)i + c] = v[c];
    }
}

// features from the renderer's outputs into a zero-padded canvas of 16
// channels per pixel (two 16-byte stores)
__global__ void k_features(const float* __restrict__ rgb, const float* __restrict__ albedo,
                           const float* __restrict__ normal, const float* __restrict__ depthn,
                           const uint8_t* __restrict__ trans, uint32_t w, uint32_t h, uint32_t W, uint32_t H,
                           uint16_t* __restrict__ X) {
    const uint32_t n = W * H;
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        const uint32_t y = i / W, x = i - y * W;
        float v[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
        if (x < w && y < h) feature9(rgb, albedo, normal, depthn, trans, y * w + x, v);
        union {
            uint4 u[2];
            uint16_t h[16];
        } o;
#pragma unroll
        for (int c = 0; c < 16; ++c) o.h[c] = c < 9 ? to_bf16(v[c]) : (uint16_t)0;
        uint4* dst = reinterpret_cast<uint4*>(X + (size_t)i * 16);
        dst[0] = o.u[0];
        dst[1] = o.u[1];
    }
}

__global__ void k_expm1_crop(const float* __restrict__ pred, uint32_t W, uint32_t w, uint32_t h,
                             float* __restrict__ out) {
    const size_t n = (size_t)w * h;
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
        const uint32_t x = i % w, y = i / w;
        const size_t q = (size_t)y * W + x;
        for (int c = 0; c < 3; ++c) out[3 * i + c] = fmaxf(expm1f(pred[3 * q + c]), 0.0f);
    }
}

// L1 loss on log(1 + target): sum |pred - t| (atomic) and dY = sign / N as bf16
__global__ void k_l1_loss(const float* __restrict__ pred, const float* __restrict__ target, uint32_t P,
                          uint32_t cout_p, float inv_n, uint16_t* __restrict__ dY, float* __restrict__ loss_sum) {
    float s = 0.0f;
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < (size_t)P * cout_p;
         i += (size_t)gridDim.x * blockDim.x) {
        const uint32_t c = i % cout_p;
        const size_t p = i / cout_p;
        float g = 0.0f;
        if (c < 3) {
            const float d = pred[3 * p + c] - log1pf(fmaxf(target[3 * p + c], 0.0f));
            s += fabsf(d);
            g = d > 0.0f ? inv_n : (d < 0.0f ? -inv_n : 0.0f);
        }
        dY[i] = to_bf16(g);
    }
    // one atomic per block
    __shared__ float part[4];
    for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off);
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) atomicAdd(loss_sum, (part[0] + part[1]) + (part[2] + part[3]));
}

// bf16 [P][cp] -> float [P][c] (padding channels dropped)
__global__ void k_unpack_bf16(const uint16_t* __restrict__ X, uint32_t P, uint32_t cp, uint32_t c,
                              float* __restrict__ F) {
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < (size_t)P * c; i += (size_t)gridDim.x * blockDim.x)
        F[i] = __uint_as_float((uint32_t)X[(i / c) * cp + (i % c)] << 16);
}

// given dpred float [P][3] -> bf16 [P][cout_p]
__global__ void k_pack_dpred(const float* __restrict__ dp, uint32_t P, uint32_t cout_p, uint16_t* __restrict__ dY) {
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < (size_t)P * cout_p;
         i += (size_t)gridDim.x * blockDim.x) {
        const uint32_t c = i % cout_p;
        dY[i] = c < 3 ? to_bf16(dp[(i / cout_p) * 3 + c]) : (uint16_t)0;
    }
}

// float master weights of one layer (oracle packing [co][ky][kx][ci], then
// bias) -> forward and input-gradient bfloat16 matrices
__global__ void k_convert(const float* __restrict__ w, uint32_t cout, uint32_t cin, uint32_t ks, uint32_t cout_p,
                          uint32_t cin_p, uint32_t kpad, uint32_t kpad_t, uint16_t* __restrict__ Wf,
                          uint16_t* __restrict__ Wd) {
    const uint32_t taps = ks * ks;
    const size_t nf = (size_t)cout_p * kpad;
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < nf; i += (size_t)gridDim.x * blockDim.x) {
        const uint32_t co = i / kpad, k = i % kpad;
        const uint32_t tap = k / cin_p, ci = k % cin_p;
        float v = 0.0f;
        if (co < cout && tap < taps && ci < cin) v = w[((size_t)co * taps + tap) * cin + ci];
        Wf[i] = to_bf16(v);
    }
    const size_t nd = (size_t)cin_p * kpad_t;
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < nd; i += (size_t)gridDim.x * blockDim.x) {
        const uint32_t ci = i / kpad_t, k = i % kpad_t;
        const uint32_t tap = k / cout_p, co = k % cout_p;
        float v = 0.0f;
        if (ci < cin && tap < taps && co < cout) v = w[((size_t)co * taps + (taps - 1 - tap)) * cin + ci];
        Wd[i] = to_bf16(v);
    }
}

// where each layer's weights sit in the float vector and the bf16 matrices
struct LayerTab {
    static constexpr int kMax = 4 * 6 - 1;   // layers of a 6-level network
    uint32_t n;
    struct Entry {
        uint32_t w_off, nw, cin, taps, cin_p, cout_p, kpad, kpad_t, wf_off, wd_off;
    } e[kMax];
};

// One Adam step over the float parameters, which also refreshes the bf16
// forward and input-gradient matrices of every weight it updates (their
// padding stays zero from the full conversion) and clears the gradient for
// the next backward pass.
__global__ void k_adam(float* __restrict__ th, float* __restrict__ m, float* __restrict__ v,
                       float* __restrict__ g, size_t n, float lr, float b1, float b2, float eps, float c1, float c2,
                       LayerTab tab, uint16_t* __restrict__ Wf, uint16_t* __restrict__ Wd) {
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
        const float gi = g[i];
        const float mi = b1 * m[i] + (1.0f - b1) * gi;
        const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
        m[i] = mi;
        v[i] = vi;
        const float t = th[i] - lr * (mi / c1) / (sqrtf(vi / c2) + eps);
        th[i] = t;
        g[i] = 0.0f;
        uint32_t l = 0;
        while (l + 1 < tab.n && i >= tab.e[l + 1].w_off) ++l;
        const LayerTab::Entry& E = tab.e[l];
        uint32_t r = (uint32_t)i - E.w_off;
        if (r < E.nw) {   // a weight [co][tap][ci] (the layer's biases follow its weights)
            const uint32_t ci = r % E.cin;
            r /= E.cin;
            const uint32_t tap = r % E.taps, co = r / E.taps;
            const uint16_t b = to_bf16(t);
            Wf[E.wf_off + (size_t)co * E.kpad + tap * E.cin_p + ci] = b;
            Wd[E.wd_off + (size_t)ci * E.kpad_t + (E.taps - 1 - tap) * E.cout_p + co] = b;
        }
    }
}

__global__ void k_zero_f(float* p, size_t n) {
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) p[i] = 0.0f;
}

inline uint32_t blocks(size_t n, uint32_t bs = 256, uint32_t cap = 16384) {
    size_t g = (n + bs - 1) / bs;
    return (uint32_t)(g < 1 ? 1 : (g > cap ? cap : g));
}

}  // namespace

// =====================================================================
namespace scl {

namespace {

uint32_t round_up(uint32_t v, uint32_t m) { return (v + m - 1) / m * m; }

}  // namespace

sc_status unet_create(Ctx* c, const uint32_t* widths, uint32_t levels, Unet* u) {
    if (levels < 2 || levels > 6) return set_error(SC_EINVAL, "levels must be 2..6");
    attach(c, &u->ctx);
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, c->device) == hipSuccess && cus > 0)
        u->cus = (uint32_t)cus;
    u->widths.assign(widths, widths + levels);
    for (uint32_t i = 0; i < levels; ++i)
        if (widths[i] == 0 || widths[i] % 16 != 0 || widths[i] > 256)
            return set_error(SC_EINVAL, "widths must be multiples of 16 up to 256");
    // layer table in parameter order
    auto add = [&](uint32_t cout, uint32_t ks, uint32_t cin) {
        UnetLayer L;
        L.cout = cout; L.ks = ks; L.cin = cin;
        L.cout_p = round_up(cout, 16);
        L.cin_p = round_up(cin, 16);
        L.kpad = round_up(ks * ks * L.cin_p, 32);
        L.kpad_t = round_up(ks * ks * L.cout_p, 32);
        L.w_off = u->n_params;
        L.b_off = L.w_off + (size_t)cout * ks * ks * cin;
        u->n_params = L.b_off + cout;
        u->layers.push_back(L);
    };
    uint32_t cin = kUnetIn;
    for (uint32_t i = 0; i < levels; ++i) {
        add(widths[i], 3, cin);
        add(widths[i], 3, widths[i]);
        cin = widths[i];
    }
    for (int i = (int)levels - 2; i >= 0; --i) {
        add(widths[i], 3, cin + widths[i]);
        add(widths[i], 3, widths[i]);
        cin = widths[i];
    }
    add(kUnetOut, 1, cin);
    size_t wf = 0, wd = 0;
    for (auto& L : u->layers) {
        L.wf_off = wf;
        L.wd_off = wd;
        wf += (size_t)L.cout_p * L.kpad;
        wd += (size_t)L.cin_p * L.kpad_t;
    }
    SC_TRY(u->theta.alloc(4 * u->n_params));
    SC_TRY(u->m.alloc(4 * u->n_params));
    SC_TRY(u->v.alloc(4 * u->n_params));
    SC_TRY(u->grad.alloc(4 * u->n_params));
    SC_TRY(u->wf.alloc(2 * wf));
    SC_TRY(u->wd.alloc(2 * wd));
    SC_TRY(u->loss.alloc(16));
    hipLaunchKernelGGL(k_zero_f, dim3(blocks(u->n_params)), dim3(256), 0, c->stream, u->theta.as<float>(), u->n_params);
    hipLaunchKernelGGL(k_zero_f, dim3(blocks(u->n_params)), dim3(256), 0, c->stream, u->m.as<float>(), u->n_params);
    hipLaunchKernelGGL(k_zero_f, dim3(blocks(u->n_params)), dim3(256), 0, c->stream, u->v.as<float>(), u->n_params);
    SC_HIP(hipGetLastError());
    return unet_refresh(u);
}

sc_status unet_refresh(Unet* u) {
    hipStream_t st = u->ctx->stream;
    for (auto& L : u->layers) {
        hipLaunchKernelGGL(k_convert, dim3(blocks((size_t)L.cout_p * L.kpad)), dim3(256), 0, st,
                           u->theta.as<float>() + L.w_off, L.cout, L.cin, L.ks, L.cout_p, L.cin_p, L.kpad, L.kpad_t,
                           u->wf.as<uint16_t>() + L.wf_off, u->wd.as<uint16_t>() + L.wd_off);
    }
    SC_HIP(hipGetLastError());
    return SC_OK;
}

namespace {

// activation buffers for a batch shape
sc_status ensure_acts(Unet* u, uint32_t B, uint32_t H, uint32_t W) {
    if (u->B == B && u->H == H && u->W == W && u->acts.p) return SC_OK;
    const uint32_t L = (uint32_t)u->widths.size();
    // offsets (in bf16 elements) of every tensor
    size_t off = 0, largest = 0;
    auto take = [&](size_t n) {
        largest = std::max(largest, n);
        size_t o = off;
        off += (n + 127) / 128 * 128;
        return o;
    };
    u->t.clear();
    UnetTensors& T = u->t;
    const size_t P0 = (size_t)B * H * W;
    T.in = take(P0 * 16);
    for (uint32_t i = 0; i < L; ++i) {
        const size_t P = P0 >> (2 * i);
        const uint32_t w = u->widths[i];
        if (i > 0) {
            const uint32_t cprev = u->widths[i - 1];
            T.pool.push_back(take(P * cprev));
            T.pool_idx.push_back(take((P * cprev + 1) / 2));   // bytes stored in bf16 slots
        } else {
            T.pool.push_back(0);
            T.pool_idx.push_back(0);
        }
        T.enc_a.push_back(take(P * w));
        T.enc_b.push_back(take(P * w));
    }
    T.cat.assign(L, 0);
    T.dec_a.assign(L, 0);
    T.dec_b.assign(L, 0);
    for (int i = (int)L - 2; i >= 0; --i) {
        const size_t P = P0 >> (2 * i);
        const uint32_t cu = (i == (int)L - 2) ? u->widths[L - 1] : u->widths[i + 1];
        T.cat[i] = take(P * (cu + u->widths[i]));
        T.dec_a[i] = take(P * u->widths[i]);
        T.dec_b[i] = take(P * u->widths[i]);
    }
    // gradient scratch: two ping-pong buffers big enough for any tensor, plus skip grads
    size_t maxt = P0 * 16;
    for (uint32_t i = 0; i < L; ++i) {
        const size_t P = P0 >> (2 * i);
        maxt = std::max(maxt, P * (size_t)(2 * u->widths[std::min(i + 1, L - 1)] + u->widths[i]));
    }
    T.g0 = take(maxt);
    T.g2 = take(maxt);
    T.skip.assign(L, 0);
    for (uint32_t i = 0; i + 1 < L; ++i) T.skip[i] = take((P0 >> (2 * i)) * u->widths[i]);
    if (largest >= ((size_t)1 << 31))   // the kernels index the elements of one tensor in 32 bits
        return set_error(SC_EUNSUPPORTED, "U-Net tensor of 2^31 elements or more");
    SC_TRY(u->acts.alloc(2 * off));
    SC_TRY(u->pred.alloc(4 * P0 * 3));
    u->B = B;
    u->H = H;
    u->W = W;
    return SC_OK;
}

// blocks of a k_conv3 variant that one CU keeps resident (registers and LDS)
template <int RW, int MODE>
uint32_t conv3_per_cu() {
    static uint32_t n = 0;
    if (!n) {
        int v = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&v, k_conv3<kConvTiles, RW, MODE>, 256, 0) != hipSuccess ||
            v < 1)
            v = 1;
        n = (uint32_t)v;
    }
    return n;
}

void conv_launch(hipStream_t st, uint32_t cus, uint64_t big_tile, const UnetLayer& L, const uint16_t* X, uint32_t P,
                 uint32_t H, uint32_t W, const uint16_t* Wt, uint32_t cin_p, uint32_t kpad, const float* bias, uint32_t cout_p,
                 uint32_t cout_real, uint16_t* Y, float* Yf, uint32_t y_stride, int relu,
                 const uint16_t* X2 = nullptr, uint32_t c_split = 0, const uint16_t* M = nullptr) {
    const uint32_t n_tiles = (P + 15) / 16;
    const uint32_t groups = (cout_p / 16 + 3) / 4;
    const size_t waves = (size_t)n_tiles * groups;
    const uint32_t grid = (uint32_t)((waves + 3) / 4);
    if (L.ks == 3 && !Yf && cout_real == cout_p) {
        // 12-row tiles (3 rows per wave: each weight operand feeds 3 MFMAs;
        // 124 registers per lane and 35 KB of LDS, 4 blocks per CU; measured
        // at 1080p: 0.95 ms per call against 0.98 ms with 16-row tiles, whose
        // 160 registers leave 3 blocks per CU) where a layer has at least
        // big_tile of them, 8-row tiles otherwise;
        // the grid holds what the CUs keep resident, each block walking
        // several tiles
        const uint32_t B = P / (H * W);
        const uint32_t gy = (cout_p / 16 + kConvTiles - 1) / kConvTiles;
        const uint32_t tx = (W + kTC - 1) / kTC;
        const uint32_t tb = tx * ((H + 4 * kBigRW - 1) / (4 * kBigRW)) * B, t8 = tx * ((H + 7) / 8) * B;
        const bool big = (uint64_t)tb * gy >= big_tile;
        const int mode = X2 ? 2 : (cin_p <= (uint32_t)kCC ? 0 : 1);
        const uint32_t tiles = big ? tb : t8;
        const uint32_t per_cu = big ? (mode == 0   ? conv3_per_cu<kBigRW, 0>()
                                       : mode == 1 ? conv3_per_cu<kBigRW, 1>()
                                                   : conv3_per_cu<kBigRW, 2>())
                                    : (mode == 0 ? conv3_per_cu<2, 0>() : mode == 1 ? conv3_per_cu<2, 1>()
                                                                                 : conv3_per_cu<2, 2>());
        const uint32_t gx = std::max(1u, std::min(tiles, (cus * per_cu + gy - 1) / gy));
        const dim3 grid(gx, gy);
#define SC_CONV3(RW, MODE)                                                                                          \
    hipLaunchKernelGGL((k_conv3<kConvTiles, RW, MODE>), grid, dim3(256), 0, st, X, X2, c_split, B, H, W, cin_p, Wt, \
                       kpad, bias, cout_p, Y, y_stride, relu, M)
        if (big) {
            if (mode == 0) SC_CONV3(kBigRW, 0);
            else if (mode == 1) SC_CONV3(kBigRW, 1);
            else SC_CONV3(kBigRW, 2);
        } else {
            if (mode == 0) SC_CONV3(2, 0);
            else if (mode == 1) SC_CONV3(2, 1);
            else SC_CONV3(2, 2);
        }
#undef SC_CONV3
    } else if (L.ks == 3)   // float output or partial channel tiles: the plain implicit GEMM
        hipLaunchKernelGGL(k_conv<3>, dim3(grid), dim3(256), 0, st, X, P, H, W, cin_p, Wt, kpad, bias, cout_p,
                           cout_real, Y, Yf, y_stride, 0u, relu, M);
    else if (Yf && cout_p == 16 && kpad <= 32 * kOutChunks)   // the output layer
        hipLaunchKernelGGL(k_conv1_out, dim3(std::max(1u, std::min((n_tiles + 3) / 4, cus * 8))), dim3(256), 0, st, X,
                           P, cin_p, Wt, kpad, bias, cout_real, Yf, y_stride, relu);
    else
        hipLaunchKernelGGL(k_conv<1>, dim3(grid), dim3(256), 0, st, X, P, H, W, cin_p, Wt, kpad, bias, cout_p,
                           cout_real, Y, Yf, y_stride, 0u, relu, M);
}

}  // namespace

// Forward pass over the packed input in u->acts (T.in); prediction in u->pred.
sc_status unet_forward_packed(Unet* u, bool keep_cat) {
    hipStream_t st = u->ctx->stream;
    const uint64_t big = u->ctx->conv_big_tile;
    const uint32_t L = (uint32_t)u->widths.size();
    uint16_t* A = u->acts.as<uint16_t>();
    const float* th = u->theta.as<float>();
    const uint16_t* wf = u->wf.as<uint16_t>();
    UnetTensors& T = u->t;
    size_t li = 0;
    const uint16_t* h = A + T.in;
    uint32_t hc = 16;
    for (uint32_t i = 0; i < L; ++i) {
        const uint32_t H = u->H >> i, W = u->W >> i, P = u->B * H * W;
        if (i > 0) {
            hipLaunchKernelGGL(k_maxpool, dim3(blocks((size_t)P * hc)), dim3(256), 0, st, h, u->B, 2 * H, 2 * W, hc,
                               A + T.pool[i], reinterpret_cast<uint8_t*>(A + T.pool_idx[i]));
            h = A + T.pool[i];
        }
        for (int part = 0; part < 2; ++part) {
            const UnetLayer& Ly = u->layers[li++];
            uint16_t* out = A + (part == 0 ? T.enc_a[i] : T.enc_b[i]);
            conv_launch(st, u->cus, big, Ly, h, P, H, W, wf + Ly.wf_off, Ly.cin_p, Ly.kpad, th + Ly.b_off, Ly.cout_p,
                        Ly.cout, out, nullptr, Ly.cout, 1);
            h = out;
            hc = Ly.cout;
        }
    }
    for (int i = (int)L - 2; i >= 0; --i) {
        const uint32_t H = u->H >> i, W = u->W >> i, P = u->B * H * W;
        const uint16_t* skip = nullptr;   // read in place by the first convolution
        uint32_t split = 0;
        if (keep_cat) {   // the backward pass reads the concatenation
            hipLaunchKernelGGL(k_upcat, dim3(blocks((size_t)P * (hc + u->widths[i]) / 8)), dim3(256), 0, st, h, hc,
                               A + T.enc_b[i], u->widths[i], u->B, H, W, A + T.cat[i]);
            h = A + T.cat[i];
        } else {
            skip = A + T.enc_b[i];
            split = hc;
        }
        for (int part = 0; part < 2; ++part) {
            const UnetLayer& Ly = u->layers[li++];
            uint16_t* out = A + (part == 0 ? T.dec_a[i] : T.dec_b[i]);
            conv_launch(st, u->cus, big, Ly, h, P, H, W, wf + Ly.wf_off, Ly.cin_p, Ly.kpad, th + Ly.b_off, Ly.cout_p,
                        Ly.cout, out, nullptr, Ly.cout, 1, part == 0 ? skip : nullptr, part == 0 ? split : 0u);
            h = out;
            hc = Ly.cout;
        }
    }
    const UnetLayer& Lo = u->layers[li];
    const uint32_t P0 = u->B * u->H * u->W;
    conv_launch(st, u->cus, big, Lo, h, P0, u->H, u->W, wf + Lo.wf_off, Lo.cin_p, Lo.kpad, th + Lo.b_off, Lo.cout_p,
                Lo.cout, nullptr, u->pred.as<float>(), 3, 0);
    u->cat_valid = keep_cat;
    SC_HIP(hipGetLastError());
    return SC_OK;
}

namespace {

// gradient of one convolution: dZ (bf16, [P][cout_p] layout) given; adds
// the weight and bias gradient into u->grad and, if dX is not null, writes
// the input gradient, already passed back through the ReLU whose output is
// relu_out (same layout as dX) when that is not null
void conv_backward(Unet* u, const UnetLayer& Ly, const uint16_t* Xin, const uint16_t* dZ, uint32_t P, uint32_t H,
                   uint32_t W, uint16_t* dX, const uint16_t* relu_out) {
    hipStream_t st = u->ctx->stream;
    float* g = u->grad.as<float>();
    const uint32_t taps = Ly.ks * Ly.ks;
    const uint32_t kreal = taps * Ly.cin_p;
    // channel tiles per block (3 rounds up to 4: one wave idles), pixels per
    // block sized for about 2048 blocks, 256 to 8192 each (the partial sums
    // meet in float atomics)
    const uint32_t ctn = Ly.cout_p / 16;
    const uint32_t CT = ctn >= 3 ? 4u : ctn;
    const uint32_t nb = 64 * (4 / CT);
    const uint32_t tiles = (ctn + CT - 1) / CT * ((kreal + nb - 1) / nb);
    const uint32_t want_chunks = (2048 + tiles - 1) / tiles;
    const uint32_t chunk = std::min(8192u, std::max(256u, ((P + want_chunks - 1) / want_chunks + 31) / 32 * 32));
    const uint32_t grid = tiles * ((P + chunk - 1) / chunk);
#define SC_WGRAD(KS_, CT_)                                                                                          \
    hipLaunchKernelGGL((k_wgrad_lds<KS_, CT_>), dim3(grid), dim3(256), 0, st, dZ, Ly.cout_p, Xin, Ly.cin_p, P, H, W, \
                       chunk, g + Ly.w_off, kreal, Ly.cout, Ly.cin, g + Ly.b_off)
    if (Ly.ks == 3) {
        if (CT == 4) SC_WGRAD(3, 4);
        else if (CT == 2) SC_WGRAD(3, 2);
        else SC_WGRAD(3, 1);
    } else {
        if (CT == 4) SC_WGRAD(1, 4);
        else if (CT == 2) SC_WGRAD(1, 2);
        else SC_WGRAD(1, 1);
    }
#undef SC_WGRAD
    // the weight and bias gradients add into u->grad, cleared before the backward pass
    if (dX)
        conv_launch(st, u->cus, u->ctx->conv_big_tile, Ly, dZ, P, H, W, u->wd.as<uint16_t>() + Ly.wd_off, Ly.cout_p,
                    Ly.kpad_t, nullptr, Ly.cin_p, Ly.cin_p, dX, nullptr, Ly.cin_p, 0, nullptr, 0, relu_out);
}

}  // namespace

// Backward pass: dY (bf16 [P0][16], gradient of the prediction) in T.g0.
// A gradient that flows back into a ReLU output leaves the kernel that
// produces it (input-gradient convolution, split of the concatenation,
// scatter through the pooling) already zeroed where that output is not
// positive, so it is the next convolution's dZ as it stands.
sc_status unet_backward_packed(Unet* u) {
    hipStream_t st = u->ctx->stream;
    const uint32_t L = (uint32_t)u->widths.size();
    uint16_t* A = u->acts.as<uint16_t>();
    UnetTensors& T = u->t;
    uint16_t* gcur = A + T.g0;    // dZ of the layer at hand
    uint16_t* gn = A + T.g2;      // the gradient being produced
    const uint32_t P0 = u->B * u->H * u->W;
    // every layer's weight and bias gradients add into a cleared buffer (the
    // Adam step leaves it cleared)
    if (!u->grad_clear)
        hipLaunchKernelGGL(k_zero_f, dim3(blocks(u->n_params)), dim3(256), 0, st, u->grad.as<float>(), u->n_params);
    u->grad_clear = false;
    // output layer (no activation): dZ = dY; its input is the last ReLU output
    {
        const uint16_t* xin = A + T.dec_b[0];
        conv_backward(u, u->layers.back(), xin, gcur, P0, u->H, u->W, gn, xin);
        std::swap(gcur, gn);
    }
    // decoder levels, shallow to deep; their layers are stored from the
    // deepest level: index 2L + 2(L-2-i) + part
    for (uint32_t i = 0; i + 1 < L; ++i) {
        const uint32_t H = u->H >> i, W = u->W >> i, P = u->B * H * W;
        const size_t li = 2 * L + 2 * (L - 2 - i);
        conv_backward(u, u->layers[li + 1], A + T.dec_a[i], gcur, P, H, W, gn, A + T.dec_a[i]);
        std::swap(gcur, gn);
        conv_backward(u, u->layers[li], A + T.cat[i], gcur, P, H, W, gn, nullptr);   // input: the concatenation
        std::swap(gcur, gn);
        // split the concatenation's gradient: the upsampled part to the deeper
        // level's output (masked by it), the skip part kept for the encoder
        const uint32_t cu = (i == L - 2) ? u->widths[L - 1] : u->widths[i + 1];
        const uint16_t* deeper = A + (i == L - 2 ? T.enc_b[L - 1] : T.dec_b[i + 1]);
        hipLaunchKernelGGL(k_upcat_bwd, dim3(blocks((size_t)P * (cu + u->widths[i]) / 8)), dim3(256), 0, st, gcur,
                           cu, u->widths[i], u->B, H, W, deeper, gn, A + T.skip[i]);
        std::swap(gcur, gn);
    }
    // encoder levels, deep to shallow
    for (int i = (int)L - 1; i >= 0; --i) {
        const uint32_t H = u->H >> i, W = u->W >> i, P = u->B * H * W;
        conv_backward(u, u->layers[2 * i + 1], A + T.enc_a[i], gcur, P, H, W, gn, A + T.enc_a[i]);
        std::swap(gcur, gn);
        if (i == 0) {   // the network input needs no gradient
            conv_backward(u, u->layers[0], A + T.in, gcur, P, H, W, nullptr, nullptr);
            break;
        }
        conv_backward(u, u->layers[2 * i], A + T.pool[i], gcur, P, H, W, gn, nullptr);   // input: the pooling
        std::swap(gcur, gn);
        // through the pooling into level i-1, plus that level's skip
        // gradient, masked by that level's output
        const uint32_t c = u->widths[i - 1];
        const size_t n8 = (size_t)u->B * (2 * H) * (2 * W) * c / 8;
        hipLaunchKernelGGL(k_maxpool_bwd, dim3(blocks(n8)), dim3(256), 0, st, gcur,
                           reinterpret_cast<const uint8_t*>(A + T.pool_idx[i]), u->B, 2 * H, 2 * W, c,
                           A + T.skip[i - 1], A + T.enc_b[i - 1], gn);
        std::swap(gcur, gn);
    }
    SC_HIP(hipGetLastError());
    return SC_OK;
}

sc_status unet_prepare(Unet* u, uint32_t B, uint32_t H, uint32_t W) { return ensure_acts(u, B, H, W); }

sc_status unet_pack_input(Unet* u, const float* feat) {
    const uint32_t P = u->B * u->H * u->W;
    hipLaunchKernelGGL(k_pack_input, dim3(blocks((size_t)P * 16)), dim3(256), 0, u->ctx->stream, feat, P, kUnetIn, 16u,
                       u->acts.as<uint16_t>() + u->t.in);
    SC_HIP(hipGetLastError());
    return SC_OK;
}

sc_status unet_pack_dpred(Unet* u, const float* dpred) {
    const uint32_t P = u->B * u->H * u->W;
    hipLaunchKernelGGL(k_pack_dpred, dim3(blocks((size_t)P * 16)), dim3(256), 0, u->ctx->stream, dpred, P, 16u,
                       u->acts.as<uint16_t>() + u->t.g0);
    SC_HIP(hipGetLastError());
    return SC_OK;
}

sc_status unet_loss(Unet* u, const float* target, float* loss_dev) {
    const uint32_t P = u->B * u->H * u->W;
    hipStream_t st = u->ctx->stream;
    hipLaunchKernelGGL(k_zero_f, dim3(1), dim3(64), 0, st, loss_dev, (size_t)1);
    hipLaunchKernelGGL(k_l1_loss, dim3(std::min(1024u, blocks((size_t)P * 16))), dim3(256), 0, st,
                       u->pred.as<float>(), target, P, 16u,
                       1.0f / (float)((size_t)P * 3), u->acts.as<uint16_t>() + u->t.g0, loss_dev);
    SC_HIP(hipGetLastError());
    return SC_OK;
}

sc_status unet_adam(Unet* u, float lr) {
    u->step += 1;
    const float b1 = 0.9f, b2 = 0.999f;
    const float c1 = (float)(1.0 - pow(0.9, (double)u->step));
    const float c2 = (float)(1.0 - pow(0.999, (double)u->step));
    LayerTab tab{};
    tab.n = (uint32_t)u->layers.size();
    for (uint32_t l = 0; l < tab.n; ++l) {
        const UnetLayer& L = u->layers[l];
        tab.e[l] = LayerTab::Entry{(uint32_t)L.w_off, (uint32_t)(L.b_off - L.w_off), L.cin, L.ks * L.ks, L.cin_p,
                                   L.cout_p, L.kpad, L.kpad_t, (uint32_t)L.wf_off, (uint32_t)L.wd_off};
    }
    hipLaunchKernelGGL(k_adam, dim3(blocks(u->n_params)), dim3(256), 0, u->ctx->stream, u->theta.as<float>(),
                       u->m.as<float>(), u->v.as<float>(), u->grad.as<float>(), u->n_params, lr, b1, b2, 1e-8f, c1, c2,
                       tab, u->wf.as<uint16_t>(), u->wd.as<uint16_t>());
    SC_HIP(hipGetLastError());
    u->grad_clear = true;
    return SC_OK;
}

sc_status unet_features(Unet* u, const sc_aov& in, uint32_t w, uint32_t h) {
    hipLaunchKernelGGL(k_features, dim3(blocks((size_t)u->W * u->H)), dim3(256), 0, u->ctx->stream, in.rgb, in.albedo,
                       in.normal, in.depthn, in.trans, w, h, u->W, u->H, u->acts.as<uint16_t>() + u->t.in);
    SC_HIP(hipGetLastError());
    return SC_OK;
}

// One convolution layer alone (the per-layer check of the kernels): the
// input packed to bf16 as the network stores activations, the layer's own
// launch, its output converted back to float.
sc_status unet_layer_forward(Unet* u, uint32_t layer, const float* X, uint32_t n, uint32_t h, uint32_t w, int relu,
                             float* Y) {
    const UnetLayer& L = u->layers[layer];
    hipStream_t st = u->ctx->stream;
    const uint32_t P = n * h * w;
    DevBuf xb, yb;
    SC_TRY(xb.alloc(2 * (size_t)P * L.cin_p));
    hipLaunchKernelGGL(k_pack_input, dim3(blocks((size_t)P * L.cin_p)), dim3(256), 0, st, X, P, L.cin, L.cin_p,
                       xb.as<uint16_t>());
    const float* th = u->theta.as<float>();
    const uint16_t* wf = u->wf.as<uint16_t>();
    if (L.ks == 3) {
        SC_TRY(yb.alloc(2 * (size_t)P * L.cout_p));
        conv_launch(st, u->cus, u->ctx->conv_big_tile, L, xb.as<uint16_t>(), P, h, w, wf + L.wf_off, L.cin_p, L.kpad,
                    th + L.b_off, L.cout_p, L.cout, yb.as<uint16_t>(), nullptr, L.cout, relu);
        hipLaunchKernelGGL(k_unpack_bf16, dim3(blocks((size_t)P * L.cout)), dim3(256), 0, st, yb.as<uint16_t>(), P,
                           L.cout, L.cout, Y);
    } else {
        conv_launch(st, u->cus, u->ctx->conv_big_tile, L, xb.as<uint16_t>(), P, h, w, wf + L.wf_off, L.cin_p, L.kpad,
                    th + L.b_off, L.cout_p, L.cout, nullptr, Y, L.cout, relu);
    }
    SC_HIP(hipGetLastError());
    SC_HIP(hipStreamSynchronize(st));   // the temporaries are freed on return
    return SC_OK;
}

sc_status unet_layer_backward(Unet* u, uint32_t layer, const float* X, const float* dZ, uint32_t n, uint32_t h,
                              uint32_t w, float* dX, float* dW) {
    const UnetLayer& L = u->layers[layer];
    hipStream_t st = u->ctx->stream;
    const uint32_t P = n * h * w;
    DevBuf xb, dzb, dxb;
    SC_TRY(xb.alloc(2 * (size_t)P * L.cin_p));
    SC_TRY(dzb.alloc(2 * (size_t)P * L.cout_p));
    if (dX) SC_TRY(dxb.alloc(2 * (size_t)P * L.cin_p));
    hipLaunchKernelGGL(k_pack_input, dim3(blocks((size_t)P * L.cin_p)), dim3(256), 0, st, X, P, L.cin, L.cin_p,
                       xb.as<uint16_t>());
    hipLaunchKernelGGL(k_pack_input, dim3(blocks((size_t)P * L.cout_p)), dim3(256), 0, st, dZ, P, L.cout, L.cout_p,
                       dzb.as<uint16_t>());
    // the layer's gradient entries add up in u->grad: cleared first
    const size_t nw = (size_t)L.cout * L.ks * L.ks * L.cin;
    hipLaunchKernelGGL(k_zero_f, dim3(blocks(nw + L.cout)), dim3(256), 0, st, u->grad.as<float>() + L.w_off,
                       nw + L.cout);
    u->grad_clear = false;
    conv_backward(u, L, xb.as<uint16_t>(), dzb.as<uint16_t>(), P, h, w, dX ? dxb.as<uint16_t>() : nullptr, nullptr);
    if (dX)
        hipLaunchKernelGGL(k_unpack_bf16, dim3(blocks((size_t)P * L.cin)), dim3(256), 0, st, dxb.as<uint16_t>(), P,
                           L.cin_p, L.cin, dX);
    SC_HIP(hipMemcpyAsync(dW, u->grad.as<float>() + L.w_off, 4 * (nw + L.cout), hipMemcpyDeviceToDevice, st));
    SC_HIP(hipGetLastError());
    SC_HIP(hipStreamSynchronize(st));   // the temporaries are freed on return
    return SC_OK;
}

sc_status features_f32(Ctx* c, const sc_aov& in, uint32_t w, uint32_t h, float* out) {
    const size_t n = (size_t)w * h;
    hipLaunchKernelGGL(k_features_f32, dim3(blocks(n)), dim3(256), 0, c->stream, in.rgb, in.albedo, in.normal,
                       in.depthn, in.trans, (uint32_t)n, out);
    SC_HIP(hipGetLastError());
    return SC_OK;
}

sc_status unet_output_rgb(Unet* u, uint32_t w, uint32_t h, float* out) {
    hipLaunchKernelGGL(k_expm1_crop, dim3(blocks((size_t)w * h)), dim3(256), 0, u->ctx->stream, u->pred.as<float>(),
                       u->W, w, h, out);
    SC_HIP(hipGetLastError());
    return SC_OK;
}

}  // namespace scl

