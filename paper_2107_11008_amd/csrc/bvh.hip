// bvh.hip -- GPU construction of the wide BVH.
//
// 1. per-triangle bounds and centroids, centroid bounds of the scene;
// 2. 64-bit keys (36-bit Morton code of the centroid, 28-bit triangle index);
// 3. bitonic sort of the keys (LDS for short strides, global otherwise);
// 4. binary radix tree over the sorted keys (Karras, "Maximizing
//    parallelism in the construction of BVHs, octrees, and k-d trees",
//    HPG 2012), internal node i spanning a contiguous key range;
// 5. node boxes from a sparse table of range unions over the sorted
//    triangle boxes (every node spans a contiguous key range);
// 6. greedy collapse, one level of wide nodes per launch: a wide node opens
//    its largest-area non-leaf child until it holds 8 children; ranges of
//    at most leaf_max triangles become leaves;
// 7. triangles gathered in key order for the leaves.
#pragma clang fp contract(off)
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stdlib.h>

#include "sc_internal.h"

namespace {

__device__ __forceinline__ uint32_t ordered(float f) {
    const uint32_t b = __float_as_uint(f);
    return (b & 0x80000000u) ? ~b : (b | 0x80000000u);
}
__device__ __forceinline__ float unordered(uint32_t u) {
    return __uint_as_float((u & 0x80000000u) ? (u & 0x7fffffffu) : ~u);
}

__global__ void k_validate(const uint32_t* __restrict__ I, const uint32_t* __restrict__ tri_obj, uint32_t nt,
                           uint32_t nv, uint32_t n_mat, uint32_t* err) {
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < nt; i += gridDim.x * blockDim.x) {
        const uint32_t o = tri_obj[i];
        if (o == 0 || o >= n_mat) atomicOr(err, 1u);
        if (I[3 * (size_t)i] >= nv || I[3 * (size_t)i + 1] >= nv || I[3 * (size_t)i + 2] >= nv) atomicOr(err, 2u);
    }
}

// bounds [nt][6] (lo xyz, hi xyz) and centroid bounds (ordered uints).
// Vertex indices are clamped to the vertex array so that invalid input
// (reported by k_validate) reads nothing out of bounds.  One atomic per
// block for the centroid bounds.
__global__ __launch_bounds__(256) void k_tri_bounds(const float* __restrict__ V, const uint32_t* __restrict__ I,
                                                    uint32_t nt, uint32_t nv, float* __restrict__ bounds,
                                                    uint32_t* __restrict__ cb) {
    float clo[3] = {INFINITY, INFINITY, INFINITY}, chi[3] = {-INFINITY, -INFINITY, -INFINITY};
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < nt; i += gridDim.x * blockDim.x) {
        const uint32_t* idx = I + 3 * (size_t)i;
        const uint32_t i0 = min(idx[0], nv - 1), i1 = min(idx[1], nv - 1), i2 = min(idx[2], nv - 1);
        float lo[3], hi[3];
        bool finite = true;
        for (int k = 0; k < 3; ++k) {
            const float a = V[3 * (size_t)i0 + k], b = V[3 * (size_t)i1 + k], c = V[3 * (size_t)i2 + k];
            finite = finite && isfinite(a) && isfinite(b) && isfinite(c);
            lo[k] = fminf(a, fminf(b, c));
            hi[k] = fmaxf(a, fmaxf(b, c));
        }
        if (!finite) {
            // a triangle with a non-finite vertex can never be hit: empty box
            for (int k = 0; k < 3; ++k) { lo[k] = INFINITY; hi[k] = -INFINITY; }
        }
        for (int k = 0; k < 3; ++k) {
            bounds[6 * (size_t)i + k] = lo[k];
            bounds[6 * (size_t)i + 3 + k] = hi[k];
            if (finite) {
                const float c = 0.5f * lo[k] + 0.5f * hi[k];
                clo[k] = fminf(clo[k], c);
                chi[k] = fmaxf(chi[k], c);
            }
        }
    }
    __shared__ float red[4][6];
    for (int k = 0; k < 3; ++k) {
        for (int off = 32; off > 0; off >>= 1) {
            clo[k] = fminf(clo[k], __shfl_xor(clo[k], off));
            chi[k] = fmaxf(chi[k], __shfl_xor(chi[k], off));
        }
    }
    const uint32_t w = threadIdx.x >> 6;
    if (__lane_id() == 0)
        for (int k = 0; k < 3; ++k) { red[w][k] = clo[k]; red[w][3 + k] = chi[k]; }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (uint32_t v = 1; v < (blockDim.x >> 6); ++v)
            for (int k = 0; k < 3; ++k) {
                clo[k] = fminf(clo[k], red[v][k]);
                chi[k] = fmaxf(chi[k], red[v][3 + k]);
            }
        for (int k = 0; k < 3; ++k) {
            atomicMin(&cb[k], ordered(clo[k]));
            atomicMax(&cb[3 + k], ordered(chi[k]));
        }
    }
}

// Emissive triangles, compacted in index order: per segment of 256
// triangles a count, one scan over the segments, then each segment writes
// its emitters (index and the 9 vertex coordinates) at its offset.
__device__ __forceinline__ bool is_emitter(const uint32_t* __restrict__ tri_obj, const sc_material* __restrict__ mat,
                                           uint32_t n_mat, uint32_t i, uint32_t nt) {
    if (i >= nt) return false;
    const uint32_t o = tri_obj[i];
    return o >= 1 && o < n_mat && mat[o].type == SC_MAT_EMISSIVE;
}

__global__ __launch_bounds__(256) void k_emit_count(const uint32_t* __restrict__ tri_obj,
                                                    const sc_material* __restrict__ mat, uint32_t n_mat, uint32_t nt,
                                                    uint32_t* __restrict__ seg_cnt) {
    const uint32_t i = blockIdx.x * 256u + threadIdx.x;
    const int c = __syncthreads_count(is_emitter(tri_obj, mat, n_mat, i, nt));
    if (threadIdx.x == 0) seg_cnt[blockIdx.x] = (uint32_t)c;
}

// exclusive scan of nseg counts by one block of 1024 threads; total in *total
__global__ __launch_bounds__(1024) void k_emit_scan(const uint32_t* __restrict__ seg_cnt, uint32_t nseg,
                                                    uint32_t* __restrict__ seg_off, uint32_t* __restrict__ total) {
    __shared__ uint32_t part[1024];
    const uint32_t per = (nseg + 1023u) / 1024u;
    const uint32_t b0 = threadIdx.x * per, b1 = min(b0 + per, nseg);
    uint32_t sum = 0;
    for (uint32_t j = b0; j < b1; ++j) sum += seg_cnt[j];
    part[threadIdx.x] = sum;
    __syncthreads();
    for (uint32_t off = 1; off < 1024u; off <<= 1) {
        const uint32_t v = threadIdx.x >= off ? part[threadIdx.x - off] : 0u;
        __syncthreads();
        part[threadIdx.x] += v;
        __syncthreads();
    }
    uint32_t run = part[threadIdx.x] - sum;   // exclusive prefix of this thread's range
    for (uint32_t j = b0; j < b1; ++j) {
        seg_off[j] = run;
        run += seg_cnt[j];
    }
    if (threadIdx.x == 1023) *total = part[1023];
}

__global__ __launch_bounds__(256) void k_emit_gather(const uint32_t* __restrict__ tri_obj,
                                                     const sc_material* __restrict__ mat, uint32_t n_mat,
                                                     uint32_t nt, const uint32_t* __restrict__ I,
                                                     const float* __restrict__ V, uint32_t nv,
                                                     const uint32_t* __restrict__ seg_off,
                                                     uint32_t* __restrict__ out_prim, float* __restrict__ out_v) {
    __shared__ uint32_t wcnt[4];
    const uint32_t i = blockIdx.x * 256u + threadIdx.x;
    const bool e = is_emitter(tri_obj, mat, n_mat, i, nt);
    const unsigned long long m = __ballot(e);
    const uint32_t w = threadIdx.x >> 6;
    if (__lane_id() == 0) wcnt[w] = (uint32_t)__popcll(m);
    __syncthreads();
    uint32_t base = seg_off[blockIdx.x];
    for (uint32_t v = 0; v < w; ++v) base += wcnt[v];
    if (e) {
        const uint32_t k = base + __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
        out_prim[k] = i;
        for (int j = 0; j < 3; ++j) {
            const uint32_t vi = min(I[3 * (size_t)i + j], nv - 1);
            for (int c = 0; c < 3; ++c) out_v[9 * (size_t)k + 3 * j + c] = V[3 * (size_t)vi + c];
        }
    }
}

// Builder start state: error flags, node and emitter counts and the
// per-level work counts cleared, the root (radix-tree node 0, or the single
// leaf when n == 1) as the one work item of level 0, empty centroid bounds.
__global__ void k_build_init(uint32_t* meta, uint32_t n_meta, uint2* work0, uint32_t* cb) {
    for (uint32_t i = threadIdx.x; i < n_meta; i += blockDim.x) meta[i] = 0u;
    __syncthreads();
    if (threadIdx.x == 0) {
        meta[1] = 1u;          // nodes allocated: the root
        meta[8] = 1u;          // level 0 work: the root
        work0[0] = make_uint2(0u, 0u);
        for (int k = 0; k < 3; ++k) { cb[k] = 0xffffffffu; cb[3 + k] = 0u; }
    }
}

// bits 0..11 of x moved to bits 0, 3, 6, ..., 33
__device__ __forceinline__ unsigned long long spread12(uint32_t x) {
    unsigned long long r = 0;
    for (int b = 0; b < 12; ++b) r |= (unsigned long long)((x >> b) & 1u) << (3 * b);
    return r;
}

// key = 36-bit Morton code of the centroid (12 bits per axis over the
// centroid bounds) above the 28-bit triangle index (nt < 2^28)
constexpr int kKeyIndexBits = 28;
constexpr unsigned long long kKeyIndexMask = (1ull << kKeyIndexBits) - 1;

__global__ void k_morton(const float* __restrict__ bounds, uint32_t nt, uint32_t n_pad, const uint32_t* __restrict__ cb,
                         unsigned long long* __restrict__ keys) {
    float lo[3], inv[3];
    for (int k = 0; k < 3; ++k) {
        lo[k] = unordered(cb[k]);
        const float ext = unordered(cb[3 + k]) - lo[k];
        inv[k] = ext > 0.0f ? 4095.0f / ext : 0.0f;
    }
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n_pad; i += gridDim.x * blockDim.x) {
        if (i >= nt) {
            keys[i] = ~0ull;
            continue;
        }
        uint32_t q[3];
        for (int k = 0; k < 3; ++k) {
            const float l = bounds[6 * (size_t)i + k], h = bounds[6 * (size_t)i + 3 + k];
            float c = 0.5f * l + 0.5f * h;
            float f = isfinite(c) ? (c - lo[k]) * inv[k] : 0.0f;
            f = fminf(fmaxf(f, 0.0f), 4095.0f);
            q[k] = (uint32_t)f;
        }
        const unsigned long long m = (spread12(q[0]) << 2) | (spread12(q[1]) << 1) | spread12(q[2]);
        keys[i] = (m << kKeyIndexBits) | (unsigned long long)i;
    }
}

// Bitonic sort.  Element pairs (i, i ^ j) are ordered ascending when
// (i & k) == 0.  Strides below kLocal run in LDS.
constexpr int kLocal = 2048;  // elements per block in LDS (1024 threads x 2)

__global__ __launch_bounds__(1024) void k_bitonic_local(unsigned long long* keys, uint32_t k_begin, uint32_t k_end) {
    __shared__ unsigned long long s[kLocal];
    const uint32_t base = blockIdx.x * kLocal;
    s[threadIdx.x] = keys[base + threadIdx.x];
    s[threadIdx.x + 1024] = keys[base + threadIdx.x + 1024];
    __syncthreads();
    for (uint32_t k = k_begin; k <= k_end; k <<= 1) {
        const uint32_t jstart = (k <= (uint32_t)kLocal) ? (k >> 1) : (uint32_t)(kLocal >> 1);
        for (uint32_t j = jstart; j > 0; j >>= 1) {
            const uint32_t t = threadIdx.x;
            const uint32_t i = 2 * t - (t & (j - 1));   // lower index of the pair
            const uint32_t l = i + j;
            const bool up = ((base + i) & k) == 0;
            const unsigned long long a = s[i], b = s[l];
            if ((a > b) == up) { s[i] = b; s[l] = a; }
            __syncthreads();
        }
    }
    keys[base + threadIdx.x] = s[threadIdx.x];
    keys[base + threadIdx.x + 1024] = s[threadIdx.x + 1024];
}

__global__ void k_bitonic_global(unsigned long long* keys, uint32_t n, uint32_t k, uint32_t j) {
    for (uint32_t t = blockIdx.x * blockDim.x + threadIdx.x; t < n / 2; t += gridDim.x * blockDim.x) {
        const uint32_t i = 2 * t - (t & (j - 1));
        const uint32_t l = i + j;
        const bool up = (i & k) == 0;
        const unsigned long long a = keys[i], b = keys[l];
        if ((a > b) == up) { keys[i] = b; keys[l] = a; }
    }
}

__device__ __forceinline__ int delta(const unsigned long long* keys, uint32_t n, int i, int j) {
    if (j < 0 || j >= (int)n) return -1;
    return __clzll(keys[i] ^ keys[j]);
}

// Radix tree: internal nodes 0..n-2; child encoding: value < n-1 internal,
// value >= n-1 is leaf (value - (n-1)) = sorted position.
__global__ void k_radix_tree(const unsigned long long* __restrict__ keys, uint32_t n, int32_t* __restrict__ left,
                             int32_t* __restrict__ right, uint32_t* __restrict__ rlo, uint32_t* __restrict__ rhi) {
    for (uint32_t ii = blockIdx.x * blockDim.x + threadIdx.x; ii + 1 < n; ii += gridDim.x * blockDim.x) {
        const int i = (int)ii;
        const int d = (delta(keys, n, i, i + 1) - delta(keys, n, i, i - 1)) >= 0 ? 1 : -1;
        const int dmin = delta(keys, n, i, i - d);
        int lmax = 2;
        while (delta(keys, n, i, i + lmax * d) > dmin) lmax <<= 1;
        int l = 0;
        for (int t = lmax >> 1; t >= 1; t >>= 1)
            if (delta(keys, n, i, i + (l + t) * d) > dmin) l += t;
        const int j = i + l * d;
        const int dnode = delta(keys, n, i, j);
        int s = 0;
        int t = l;
        do {
            t = (t + 1) >> 1;
            if (delta(keys, n, i, i + (s + t) * d) > dnode) s += t;
        } while (t > 1);
        const int gamma = i + s * d + (d < 0 ? -1 : 0);
        const int lo = i < j ? i : j, hi = i < j ? j : i;
        const int lc = (lo == gamma) ? (int)(n - 1) + gamma : gamma;
        const int rc = (hi == gamma + 1) ? (int)(n - 1) + gamma + 1 : gamma + 1;
        left[i] = lc;
        right[i] = rc;
        rlo[i] = (uint32_t)lo;
        rhi[i] = (uint32_t)hi;
    }
}

// Range unions of the key-sorted triangle boxes: level 0 holds the box of
// the triangle at each sorted position, level L the union of positions
// [i, i + 2^L).  A radix-tree node spans a contiguous range [lo, hi], so its
// box is the union of two overlapping level-floor(log2(len)) windows.
__global__ void k_sparse_level0(const unsigned long long* __restrict__ keys, const float* __restrict__ tb, uint32_t n,
                                float* __restrict__ st) {
    for (uint32_t p = blockIdx.x * blockDim.x + threadIdx.x; p < n; p += gridDim.x * blockDim.x) {
        const uint32_t prim = (uint32_t)(keys[p] & kKeyIndexMask);
        for (int k = 0; k < 6; ++k) st[6 * (size_t)p + k] = tb[6 * (size_t)prim + k];
    }
}

__global__ void k_sparse_level(float* __restrict__ st, uint32_t n, uint32_t level) {
    const size_t src = (size_t)(level - 1) * n * 6, dst = (size_t)level * n * 6;
    const uint32_t half = 1u << (level - 1);
    const uint32_t cnt = n - (1u << level) + 1;
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < cnt; i += gridDim.x * blockDim.x) {
        const float* a = st + src + 6 * (size_t)i;
        const float* b = st + src + 6 * (size_t)(i + half);
        float* d = st + dst + 6 * (size_t)i;
        for (int k = 0; k < 3; ++k) {
            d[k] = fminf(a[k], b[k]);
            d[3 + k] = fmaxf(a[3 + k], b[3 + k]);
        }
    }
}

__device__ __forceinline__ void range_box(const float* __restrict__ st, uint32_t n, uint32_t lo, uint32_t cnt,
                                          float* box) {
    const uint32_t level = 31u - __clz(cnt);
    const float* a = st + ((size_t)level * n + lo) * 6;
    const float* b = st + ((size_t)level * n + (lo + cnt - (1u << level))) * 6;
    for (int k = 0; k < 3; ++k) {
        box[k] = fminf(a[k], b[k]);
        box[3 + k] = fmaxf(a[3 + k], b[3 + k]);
    }
}

__device__ __forceinline__ float half_area(const float* b) {
    // surface area / 2 of a box given as lo xyz, hi xyz (0 for an empty box)
    const float ex = b[3] - b[0], ey = b[4] - b[1], ez = b[5] - b[2];
    if (!(ex >= 0.0f) || !(ey >= 0.0f) || !(ez >= 0.0f)) return 0.0f;
    return ex * ey + ey * ez + ez * ex;
}

// One level of the collapse.  work[i] = (bvh2 node, wide node index).
__global__ void k_collapse(uint32_t n, const int32_t* __restrict__ left, const int32_t* __restrict__ right,
                           const uint32_t* __restrict__ rlo, const uint32_t* __restrict__ rhi,
                           const float* __restrict__ st, uint32_t leaf_max, uint32_t width,
                           const uint2* __restrict__ work, const uint32_t* __restrict__ n_work, uint2* next_work,
                           uint32_t* n_next, uint32_t* n_nodes, BNode* nodes) {
    const uint32_t nw = *n_work;
    for (uint32_t w = blockIdx.x * blockDim.x + threadIdx.x; w < nw; w += gridDim.x * blockDim.x) {
        const uint2 item = work[w];
        int32_t set[8];
        int cnt = 0;
        const int32_t root = (int32_t)item.x;
        auto range_of = [&](int32_t c, uint32_t& lo, uint32_t& cn) {
            if (c >= (int32_t)(n - 1)) { lo = (uint32_t)c - (n - 1); cn = 1; }
            else { lo = rlo[c]; cn = rhi[c] - rlo[c] + 1; }
        };
        if (root >= (int32_t)(n - 1)) {
            set[cnt++] = root;   // a single-triangle tree
        } else {
            set[cnt++] = left[root];
            set[cnt++] = right[root];
        }
        while (cnt < (int)width) {
            int best = -1;
            float ba = -1.0f;
            for (int c = 0; c < cnt; ++c) {
                uint32_t lo, cn;
                range_of(set[c], lo, cn);
                if (cn <= leaf_max) continue;
                float bx[6];
                range_box(st, n, lo, cn, bx);
                const float a = half_area(bx);
                if (a > ba) { ba = a; best = c; }
            }
            if (best < 0) break;
            const int32_t c = set[best];
            set[best] = left[c];
            set[cnt++] = right[c];
        }
        BNode node;
        for (int c = 0; c < 8; ++c) {
            if (c < cnt) {
                uint32_t lo, cn;
                range_of(set[c], lo, cn);
                float b[6];
                range_box(st, n, lo, cn, b);
                node.lox[c] = b[0]; node.loy[c] = b[1]; node.loz[c] = b[2];
                node.hix[c] = b[3]; node.hiy[c] = b[4]; node.hiz[c] = b[5];
                if (cn <= leaf_max) {
                    node.child[c] = SC_LEAF_BIT | ((cn - 1) << 28) | lo;
                } else {
                    const uint32_t idx = atomicAdd(n_nodes, 1u);
                    const uint32_t q = atomicAdd(n_next, 1u);
                    next_work[q] = make_uint2((uint32_t)set[c], idx);
                    node.child[c] = idx;
                }
            } else {
                node.lox[c] = INFINITY; node.loy[c] = INFINITY; node.loz[c] = INFINITY;
                node.hix[c] = -INFINITY; node.hiy[c] = -INFINITY; node.hiz[c] = -INFINITY;
                node.child[c] = SC_CHILD_EMPTY;
            }
            node.pad[c] = 0;
        }
        nodes[item.y] = node;
    }
}

__global__ void k_gather_tris(const unsigned long long* __restrict__ keys, uint32_t n, const float* __restrict__ V,
                              uint32_t nv, const uint32_t* __restrict__ I, float4* __restrict__ tris) {
    for (uint32_t p = blockIdx.x * blockDim.x + threadIdx.x; p < n; p += gridDim.x * blockDim.x) {
        const uint32_t prim = (uint32_t)(keys[p] & kKeyIndexMask);
        const uint32_t* idx = I + 3 * (size_t)prim;
        const float* a = V + 3 * (size_t)min(idx[0], nv - 1);
        const float* b = V + 3 * (size_t)min(idx[1], nv - 1);
        const float* c = V + 3 * (size_t)min(idx[2], nv - 1);
        tris[3 * (size_t)p + 0] = make_float4(a[0], a[1], a[2], __uint_as_float(prim));
        tris[3 * (size_t)p + 1] = make_float4(b[0], b[1], b[2], 0.0f);
        tris[3 * (size_t)p + 2] = make_float4(c[0], c[1], c[2], 0.0f);
    }
}

__global__ void k_init_u32(uint32_t* p, uint32_t n, uint32_t v) {
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) p[i] = v;
}
__global__ void k_init_i32(int32_t* p, uint32_t n, int32_t v) {
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) p[i] = v;
}

inline uint32_t grid_for(size_t n, uint32_t bs, uint32_t cap = 65536) {
    size_t g = (n + bs - 1) / bs;
    if (g < 1) g = 1;
    return (uint32_t)(g > cap ? cap : g);
}

}  // namespace

namespace scl {

static bool debug_sync() {
    static const bool on = getenv("SC_DEBUG_SYNC") != nullptr;
    return on;
}

#define SC_LAUNCH(...)                                                                   \
    do {                                                                                 \
        hipLaunchKernelGGL(__VA_ARGS__);                                                 \
        hipError_t _le = hipGetLastError();                                              \
        if (_le == hipSuccess && debug_sync()) _le = hipStreamSynchronize(st);           \
        if (_le != hipSuccess)                                                           \
            return set_error(SC_EDEVICE, std::string("launch failed: ") + hipGetErrorString(_le)); \
    } while (0)

constexpr uint32_t kMaxLevels = 64;   // wide levels (the radix tree is at most 62 deep)
constexpr uint32_t kMeta = 8 + kMaxLevels + 1;
constexpr uint32_t kLevelBatch = 12;  // collapse levels launched between host checks
constexpr uint32_t kEmitEager = 1024;  // emitter records read back with the level counts

sc_status build_wide_bvh(Ctx* ctx, Bvh* b, uint32_t width, uint32_t leaf_max, std::vector<uint32_t>& emit_prim,
                         std::vector<float>& emit_v) {
    hipStream_t st = ctx->stream;
    const sc_scene& sc = b->scene_in;
    const uint32_t n = sc.nt;
    uint32_t n_pad = 1;
    while (n_pad < n) n_pad <<= 1;
    if (n_pad < (uint32_t)kLocal) n_pad = kLocal;
    uint32_t levels = 1;
    while ((2u << (levels - 1)) <= n) ++levels;   // levels 0..floor(log2 n)
    const uint32_t nseg = (n + 255u) / 256u;
    const size_t ni = n > 1 ? n - 1 : 1;

    // temporaries, carved from one grow-only buffer of the context
    uint32_t *meta, *cb, *rlo, *rhi, *seg_cnt, *seg_off, *e_prim;
    float *bounds, *st_buf, *e_v;
    unsigned long long* keys;
    int32_t *left, *right;
    uint2 *work_a, *work_b;
    BNode* nodes_tmp;
    auto carve = [&](char* base) {
        Carver c{base};
        meta = c.take<uint32_t>(kMeta);
        cb = c.take<uint32_t>(6);
        bounds = c.take<float>(6 * (size_t)n);
        keys = c.take<unsigned long long>(n_pad);
        left = c.take<int32_t>(ni);
        right = c.take<int32_t>(ni);
        rlo = c.take<uint32_t>(ni);
        rhi = c.take<uint32_t>(ni);
        st_buf = c.take<float>(6 * (size_t)n * levels);
        work_a = c.take<uint2>(n);
        work_b = c.take<uint2>(n);
        nodes_tmp = c.take<BNode>(n);
        seg_cnt = c.take<uint32_t>(nseg);
        seg_off = c.take<uint32_t>(nseg);
        e_prim = c.take<uint32_t>(n);
        e_v = c.take<float>(9 * (size_t)n);
        return c.off;
    };
    SC_TRY(ctx->bvh_tmp.ensure(carve(nullptr) + 256));
    carve(static_cast<char*>(ctx->bvh_tmp.p));

    const uint32_t bs = 256;
    const sc_material* mat_d = b->mat.as<sc_material>();
    SC_LAUNCH(k_build_init, dim3(1), dim3(256), 0, st, meta, kMeta, work_a, cb);
    SC_LAUNCH(k_validate, dim3(grid_for(n, bs)), dim3(bs), 0, st, sc.I, sc.tri_obj, n, sc.nv, sc.n_mat, meta);
    SC_LAUNCH(k_tri_bounds, dim3(grid_for(n, bs, 512)), dim3(bs), 0, st, sc.V, sc.I, n, sc.nv, bounds, cb);
    SC_LAUNCH(k_emit_count, dim3(nseg), dim3(256), 0, st, sc.tri_obj, mat_d, sc.n_mat, n, seg_cnt);
    SC_LAUNCH(k_emit_scan, dim3(1), dim3(1024), 0, st, seg_cnt, nseg, seg_off, meta + 2);
    SC_LAUNCH(k_emit_gather, dim3(nseg), dim3(256), 0, st, sc.tri_obj, mat_d, sc.n_mat, n, sc.I, sc.V, sc.nv, seg_off,
              e_prim, e_v);
    SC_LAUNCH(k_morton, dim3(grid_for(n_pad, bs)), dim3(bs), 0, st, bounds, n, n_pad, cb, keys);
    // bitonic sort
    const uint32_t nblk = n_pad / kLocal;
    SC_LAUNCH(k_bitonic_local, dim3(nblk), dim3(1024), 0, st, keys, 2u, (uint32_t)kLocal);
    for (uint32_t k = 2 * kLocal; k <= n_pad; k <<= 1) {
        for (uint32_t j = k >> 1; j >= (uint32_t)kLocal; j >>= 1)
            SC_LAUNCH(k_bitonic_global, dim3(grid_for(n_pad / 2, bs)), dim3(bs), 0, st, keys, n_pad, k, j);
        SC_LAUNCH(k_bitonic_local, dim3(nblk), dim3(1024), 0, st, keys, k, k);
    }
    // radix tree
    if (n > 1) SC_LAUNCH(k_radix_tree, dim3(grid_for(n - 1, bs)), dim3(bs), 0, st, keys, n, left, right, rlo, rhi);
    // range-union table for node boxes
    SC_LAUNCH(k_sparse_level0, dim3(grid_for(n, bs)), dim3(bs), 0, st, keys, bounds, n, st_buf);
    for (uint32_t L = 1; L < levels; ++L)
        SC_LAUNCH(k_sparse_level, dim3(grid_for(n - (1u << L) + 1, bs)), dim3(bs), 0, st, st_buf, n, L);

    // collapse, one wide level per launch; level L reads its work count
    // from meta[8 + L] and appends the next level's items to meta[9 + L],
    // so the host checks for the end only every kLevelBatch levels
    uint32_t h[kMeta];
    uint32_t depth = 0;
    // the first emitter records come back with the counts (the rest, if
    // any, after them); records past n_emit are unused
    const uint32_t eager = n < kEmitEager ? n : kEmitEager;
    emit_prim.resize(eager);
    emit_v.resize(9 * (size_t)eager);
    std::vector<uint32_t>& eager_prim = emit_prim;
    std::vector<float>& eager_v = emit_v;
    for (uint32_t L0 = 0;; L0 += kLevelBatch) {
        if (L0 + kLevelBatch > kMaxLevels) return set_error(SC_EDEVICE, "BVH collapse did not terminate");
        for (uint32_t L = L0; L < L0 + kLevelBatch; ++L) {
            const uint2* wa = (L & 1u) ? work_b : work_a;
            uint2* wb = (L & 1u) ? work_a : work_b;
            SC_LAUNCH(k_collapse, dim3(grid_for(n, 128, 512)), dim3(128), 0, st, n, left, right, rlo, rhi, st_buf,
                      leaf_max, width, wa, meta + 8 + L, wb, meta + 9 + L, meta + 1, nodes_tmp);
        }
        SC_HIP(hipMemcpyAsync(h, meta, sizeof(h), hipMemcpyDeviceToHost, st));
        SC_HIP(hipMemcpyAsync(eager_prim.data(), e_prim, 4 * (size_t)eager, hipMemcpyDeviceToHost, st));
        SC_HIP(hipMemcpyAsync(eager_v.data(), e_v, 36 * (size_t)eager, hipMemcpyDeviceToHost, st));
        SC_HIP(hipStreamSynchronize(st));
        if (h[0] & 1u) return set_error(SC_EINVAL, "tri_obj holds an object id outside [1, n_mat)");
        if (h[0] & 2u) return set_error(SC_EINVAL, "I holds a vertex index >= nv");
        if (h[8 + L0 + kLevelBatch] == 0) break;
    }
    while (depth < kMaxLevels && h[8 + depth] > 0) ++depth;
    const uint32_t n_nodes = h[1];
    const uint32_t n_emit = h[2];

    SC_TRY(b->nodes.ensure(sizeof(BNode) * (size_t)n_nodes));
    SC_HIP(hipMemcpyAsync(b->nodes.p, nodes_tmp, sizeof(BNode) * (size_t)n_nodes, hipMemcpyDeviceToDevice, st));
    // padded: the traversal fetches 14 float4 from a leaf's first triangle
    SC_TRY(b->tris.ensure(sizeof(float4) * (3 * (size_t)n + 14)));
    SC_LAUNCH(k_gather_tris, dim3(grid_for(n, bs)), dim3(bs), 0, st, keys, n, sc.V, sc.nv, sc.I, b->tris.as<float4>());
    emit_prim.resize(n_emit);
    emit_v.resize(9 * (size_t)n_emit);
    if (n_emit > eager) {
        SC_HIP(hipMemcpyAsync(emit_prim.data() + eager, e_prim + eager, 4 * (size_t)(n_emit - eager),
                              hipMemcpyDeviceToHost, st));
        SC_HIP(hipMemcpyAsync(emit_v.data() + 9 * (size_t)eager, e_v + 9 * (size_t)eager,
                              36 * (size_t)(n_emit - eager), hipMemcpyDeviceToHost, st));
        SC_HIP(hipStreamSynchronize(st));
    }
    SC_HIP(hipGetLastError());
    b->n_nodes = n_nodes;
    b->depth = depth;
    b->width = width;
    b->leaf_max = leaf_max;
    b->max_stack = (width - 1) * depth + 1;
    return SC_OK;
}

}  // namespace scl
