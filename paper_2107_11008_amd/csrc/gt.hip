// gt.hip -- ground-truth passes over the renderer's buffers (the paper's
// Sec. III-D): local / non-local caustic mask from two renders, object
// outlines of a chosen thickness, occlusion boundaries.
#pragma clang fp contract(off)
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>

#include "sc_internal.h"

namespace {

// Rec. 709 luminance, evaluated left to right
__device__ __forceinline__ float luminance(const float* p) {
    return (0.2126f * p[0] + 0.7152f * p[1]) + 0.0722f * p[2];
}

__global__ void k_caustic_mask(const float* __restrict__ with_c, const float* __restrict__ without_c,
                               const uint8_t* __restrict__ trans, uint32_t n, float threshold,
                               uint8_t* __restrict__ mask) {
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        const float d = luminance(with_c + 3 * (size_t)i) - luminance(without_c + 3 * (size_t)i);
        mask[i] = d > threshold ? (trans && trans[i] ? 1 : 2) : 0;
    }
}

// running min / max of obj over a horizontal window of +-t (clipped)
__global__ void k_rows_minmax(const uint32_t* __restrict__ obj, uint32_t w, uint32_t h, uint32_t t,
                              uint32_t* __restrict__ mn, uint32_t* __restrict__ mx) {
    const uint32_t n = w * h;
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        const uint32_t x = i % w, y = i / w;
        const uint32_t x0 = x >= t ? x - t : 0, x1 = x + t < w ? x + t : w - 1;
        uint32_t a = 0xffffffffu, b = 0u;
        for (uint32_t xx = x0; xx <= x1; ++xx) {
            const uint32_t v = obj[(size_t)y * w + xx];
            a = v < a ? v : a;
            b = v > b ? v : b;
        }
        mn[i] = a;
        mx[i] = b;
    }
}

// outline: an object pixel whose (2t+1)^2 window holds another id
__global__ void k_cols_outline(const uint32_t* __restrict__ obj, const uint32_t* __restrict__ mn,
                               const uint32_t* __restrict__ mx, uint32_t w, uint32_t h, uint32_t t,
                               uint8_t* __restrict__ out) {
    const uint32_t n = w * h;
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        const uint32_t x = i % w, y = i / w;
        const uint32_t y0 = y >= t ? y - t : 0, y1 = y + t < h ? y + t : h - 1;
        uint32_t a = 0xffffffffu, b = 0u;
        for (uint32_t yy = y0; yy <= y1; ++yy) {
            const size_t q = (size_t)yy * w + x;
            a = mn[q] < a ? mn[q] : a;
            b = mx[q] > b ? mx[q] : b;
        }
        const uint32_t o = obj[i];
        out[i] = (o != 0u && (a != o || b != o)) ? 1 : 0;
    }
}

// The same outline in one launch for thickness t <= kTileHalo (a template
// parameter, so the window loops unroll): a block
// stages a kTileW x kTileH tile of ids with a t-pixel halo in LDS, takes the
// row min / max over +-t columns (clipped to the image), then the column
// min / max of those over +-t rows, and writes 4 output bytes per thread.
constexpr uint32_t kTileW = 64, kTileH = 16, kTileHalo = 8;
template <uint32_t t>
__global__ __launch_bounds__(256) void k_outline_tile(const uint32_t* __restrict__ obj, uint32_t w, uint32_t h,
                                                       uint8_t* __restrict__ out) {
    static_assert(t >= 1 && t <= kTileHalo, "halo");
    constexpr uint32_t lw = kTileW + 2 * t, lh = kTileH + 2 * t;   // the staged tile
    __shared__ uint32_t s_obj[lh][lw];
    __shared__ uint32_t s_mn[lh][kTileW], s_mx[lh][kTileW];
    const uint32_t x0 = blockIdx.x * kTileW, y0 = blockIdx.y * kTileH;
    for (uint32_t k = threadIdx.x; k < lw * lh; k += blockDim.x) {
        const uint32_t r = k / lw, c = k % lw;
        const long long gy = (long long)y0 - t + r, gx = (long long)x0 - t + c;
        s_obj[r][c] = (gy >= 0 && gy < h && gx >= 0 && gx < w) ? obj[(size_t)gy * w + gx] : 0u;
    }
    __syncthreads();
    // rows: staged row r, output column c (image column x0 + c)
    for (uint32_t k = threadIdx.x; k < lh * kTileW; k += blockDim.x) {
        const uint32_t r = k / kTileW, c = k % kTileW;
        uint32_t a = 0xffffffffu, b = 0u;
#pragma unroll
        for (uint32_t d = 0; d <= 2 * t; ++d) {
            const long long gx = (long long)x0 + c + d - t;
            if (gx < 0 || gx >= w) continue;
            const uint32_t v = s_obj[r][c + d];
            a = v < a ? v : a;
            b = v > b ? v : b;
        }
        s_mn[r][c] = a;
        s_mx[r][c] = b;
    }
    __syncthreads();
    // columns: 4 consecutive output pixels per thread
    const uint32_t c4 = (threadIdx.x % (kTileW / 4)) * 4, r = threadIdx.x / (kTileW / 4);
    const uint32_t y = y0 + r;
    if (r >= kTileH || y >= h) return;
    uint32_t res = 0;
    for (uint32_t e = 0; e < 4; ++e) {
        const uint32_t c = c4 + e, x = x0 + c;
        if (x >= w) break;
        uint32_t a = 0xffffffffu, b = 0u;
#pragma unroll
        for (uint32_t d = 0; d <= 2 * t; ++d) {
            const long long gy = (long long)y + d - t;
            if (gy < 0 || gy >= h) continue;
            a = s_mn[r + d][c] < a ? s_mn[r + d][c] : a;
            b = s_mx[r + d][c] > b ? s_mx[r + d][c] : b;
        }
        const uint32_t o = s_obj[r + t][c + t];
        res |= (uint32_t)((o != 0u && (a != o || b != o)) ? 1 : 0) << (8 * e);
    }
    const size_t i = (size_t)y * w + x0 + c4;
    if (x0 + c4 + 4 <= w && (reinterpret_cast<uintptr_t>(out + i) & 3u) == 0) {
        *reinterpret_cast<uint32_t*>(out + i) = res;
    } else {
        for (uint32_t e = 0; e < 4 && x0 + c4 + e < w; ++e) out[i + e] = (uint8_t)(res >> (8 * e));
    }
}

// occlusion boundary: the near side of a depth jump larger than rel * depth
__global__ void k_occlusion(const float* __restrict__ depth, uint32_t w, uint32_t h, float rel,
                            uint8_t* __restrict__ out) {
    const uint32_t n = w * h;
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        const int x = (int)(i % w), y = (int)(i / w);
        const float d = depth[i];
        uint8_t r = 0;
        if (d < INFINITY) {
            const float lim = rel * d;
            for (int dy = -1; dy <= 1; ++dy)
                for (int dx = -1; dx <= 1; ++dx) {
                    const int xx = x + dx, yy = y + dy;
                    if ((dx == 0 && dy == 0) || xx < 0 || yy < 0 || xx >= (int)w || yy >= (int)h) continue;
                    const float q = depth[(size_t)yy * w + xx];
                    if (q - d > lim) r = 1;
                }
        }
        out[i] = r;
    }
}

inline uint32_t blocks(size_t n) {
    size_t g = (n + 255) / 256;
    return (uint32_t)(g < 1 ? 1 : (g > 16384 ? 16384 : g));
}

}  // namespace

extern "C" {

sc_status sc_caustic_mask(sc_ctx* ctx, const float* rgb_with, const float* rgb_without, const uint8_t* trans,
                          uint32_t w, uint32_t h, float threshold, uint8_t* mask) {
    if (!ctx || !rgb_with || !rgb_without || !mask) return scl::set_error(SC_EINVAL, "NULL argument");
    if (w == 0 || h == 0) return SC_OK;
    const uint32_t n = w * h;
    hipLaunchKernelGGL(k_caustic_mask, dim3(blocks(n)), dim3(256), 0, ctx->c.stream, rgb_with, rgb_without, trans, n,
                       threshold, mask);
    SC_HIP(hipGetLastError());
    return SC_OK;
}

sc_status sc_outline(sc_ctx* ctx, const uint32_t* obj, uint32_t w, uint32_t h, uint32_t thickness, uint8_t* out) {
    if (!ctx || !obj || !out) return scl::set_error(SC_EINVAL, "NULL argument");
    if (thickness < 1 || thickness > 64) return scl::set_error(SC_EINVAL, "thickness must be 1..64");
    if (w == 0 || h == 0) return SC_OK;
    scl::Ctx& c = ctx->c;
    const size_t n = (size_t)w * h;
    if (thickness <= kTileHalo) {   // one launch through LDS tiles
        const dim3 grid((w + kTileW - 1) / kTileW, (h + kTileH - 1) / kTileH);
        switch (thickness) {
#define SC_OUTLINE(T) \
    case T: hipLaunchKernelGGL(k_outline_tile<T>, grid, dim3(256), 0, c.stream, obj, w, h, out); break;
            SC_OUTLINE(1) SC_OUTLINE(2) SC_OUTLINE(3) SC_OUTLINE(4)
            SC_OUTLINE(5) SC_OUTLINE(6) SC_OUTLINE(7) SC_OUTLINE(8)
#undef SC_OUTLINE
        }
        SC_HIP(hipGetLastError());
        return SC_OK;
    }
    SC_TRY(c.aos.ensure(std::max(c.aos.bytes, 2 * 4 * n + 512)));
    c.aos_n = 0;   // the SoA ray staging is reused as scratch here
    uint32_t* mn = c.aos.as<uint32_t>();
    uint32_t* mx = mn + ((n + 63) / 64) * 64;
    hipLaunchKernelGGL(k_rows_minmax, dim3(blocks(n)), dim3(256), 0, c.stream, obj, w, h, thickness, mn, mx);
    hipLaunchKernelGGL(k_cols_outline, dim3(blocks(n)), dim3(256), 0, c.stream, obj, mn, mx, w, h, thickness, out);
    SC_HIP(hipGetLastError());
    return SC_OK;
}

sc_status sc_occlusion_boundary(sc_ctx* ctx, const float* depth, uint32_t w, uint32_t h, float rel_jump,
                                uint8_t* out) {
    if (!ctx || !depth || !out) return scl::set_error(SC_EINVAL, "NULL argument");
    if (!(rel_jump >= 0.0f)) return scl::set_error(SC_EINVAL, "rel_jump must be >= 0");
    if (w == 0 || h == 0) return SC_OK;
    hipLaunchKernelGGL(k_occlusion, dim3(blocks((size_t)w * h)), dim3(256), 0, ctx->c.stream, depth, w, h, rel_jump, out);
    SC_HIP(hipGetLastError());
    return SC_OK;
}

}  // extern "C"
