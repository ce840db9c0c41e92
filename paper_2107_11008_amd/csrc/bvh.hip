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
// With the clustering builder (SC_OPT_BVH_BUILDER 1), steps 4 and 5 are
// replaced by PLOC over the sorted triangles, which gives every node its
// box and triangle count; the collapse then lays the triangles out depth
// first so that each leaf's triangles are adjacent.
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
        if (work0) work0[0] = make_uint2(0u, 0u);
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
        // area of each candidate that may be opened (-2: a leaf-sized range)
        float area[8];
        auto area_of = [&](int32_t c) -> float {
            uint32_t lo, cn;
            range_of(c, lo, cn);
            if (cn <= leaf_max) return -2.0f;
            float bx[6];
            range_box(st, n, lo, cn, bx);
            return half_area(bx);
        };
        if (root >= (int32_t)(n - 1)) {
            set[cnt] = root;   // a single-triangle tree
            area[cnt++] = -2.0f;
        } else {
            set[cnt] = left[root];
            area[cnt] = area_of(set[cnt]);
            ++cnt;
            set[cnt] = right[root];
            area[cnt] = area_of(set[cnt]);
            ++cnt;
        }
        while (cnt < (int)width) {   // open the largest candidate (the first of equal ones)
            int best = -1;
            float ba = -1.0f;
            for (int c = 0; c < cnt; ++c)
                if (area[c] > ba) { ba = area[c]; best = c; }
            if (best < 0) break;
            const int32_t c = set[best];
            set[best] = left[c];
            area[best] = area_of(set[best]);
            set[cnt] = right[c];
            area[cnt] = area_of(set[cnt]);
            ++cnt;
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

// ---------------------------------------------------------------- PLOC
// Parallel locally-ordered clustering (Meister and Bittner, "Parallel
// Locally-Ordered Clustering for Bounding Volume Hierarchy Construction",
// IEEE TVCG 2018).  The clusters start as the triangles in Morton order.
// Every iteration each cluster finds, among the kPlocRadius clusters on
// either side, the one whose union with it has the least surface area;
// mutual nearest neighbours merge into a new node, and the clusters left
// are compacted in order.  Equal areas are ordered by a hash of the pair
// (the same for both members), so the best pair of any neighbourhood is
// mutual and every iteration merges something, even when all boxes are
// equal.  Node ids are given from n-2 down, so the last node made (the
// root) is node 0.  A cluster is two float4: (lo xyz, subtree size) and
// (hi xyz, node: < n-1 internal, else leaf at sorted position - (n-1)).
constexpr uint32_t kPlocRadius = 16;
constexpr uint32_t kPlocChunk = 256;   // clusters per block step (= block size)

__device__ __forceinline__ uint32_t pair_hash(uint32_t a, uint32_t b) {
    uint32_t h = a * 0x9E3779B1u ^ (b + 0x7F4A7C15u + (a << 6) + (a >> 2));
    h ^= h >> 16;
    h *= 0x85EBCA6Bu;
    h ^= h >> 13;
    h *= 0xC2B2AE35u;
    h ^= h >> 16;
    return h;
}

// surface area / 2 of the union of two boxes as an order-preserving key
// (not-a-number and negative results sort last)
__device__ __forceinline__ uint32_t union_area_key(float4 al, float4 ah, float4 bl, float4 bh) {
    const float ex = fmaxf(ah.x, bh.x) - fminf(al.x, bl.x);
    const float ey = fmaxf(ah.y, bh.y) - fminf(al.y, bl.y);
    const float ez = fmaxf(ah.z, bh.z) - fminf(al.z, bl.z);
    const float a = ex * ey + ey * ez + ez * ex;
    return a >= 0.0f ? (__float_as_uint(a) & 0x7fffffffu) : 0x7f800001u;
}

// the neighbour of cluster i (of m) within kPlocRadius positions whose
// union with it has the least area; box(x) gives cluster x's two float4
template <typename BoxFn>
__device__ __forceinline__ int32_t ploc_nearest(uint32_t i, uint32_t m, BoxFn box) {
    constexpr uint32_t R = kPlocRadius;
    float4 al, ah;
    box(i, al, ah);
    const uint32_t jlo = i >= R ? i - R : 0u, jhi = min(m - 1u, i + R);
    unsigned long long best = ~0ull;
    int32_t bj = -1;
    for (uint32_t j = jlo; j <= jhi; ++j) {   // ascending: on equal keys the smaller j stays
        if (j == i) continue;
        float4 bl, bh;
        box(j, bl, bh);
        const unsigned long long key =
            ((unsigned long long)union_area_key(al, ah, bl, bh) << 32) | pair_hash(min(i, j), max(i, j));
        if (key < best) {
            best = key;
            bj = (int32_t)j;
        }
    }
    return bj;
}

constexpr uint32_t kPlocSmall = 4096;   // cluster counts finished by one block in LDS (k_ploc_finish)

// Nearest neighbours and merge flags of one chunk per block step.  The
// block also finds the neighbours of the kPlocRadius clusters on either
// side of its chunk (from a window of boxes 2 kPlocRadius wider), so it
// can tell mutual pairs without another launch.  Flags per cluster: bit 0
// = it survives (no mutual partner, or the smaller of a mutual pair), bit
// 1 = it makes a node with its partner; per chunk the counts of both.  At
// kPlocSmall clusters or fewer every cluster survives unchanged (the
// single-block kernel takes over).
__global__ __launch_bounds__(kPlocChunk) void k_ploc_nn_flags(const uint32_t* __restrict__ m_ptr,
                                                               const float4* __restrict__ cl,
                                                               const float4* __restrict__ ch,
                                                               int32_t* __restrict__ nn, uint8_t* __restrict__ fl,
                                                               uint2* __restrict__ chunk_cnt) {
    constexpr uint32_t R = kPlocRadius, WB = kPlocChunk + 4 * R, WN = kPlocChunk + 2 * R;
    __shared__ float4 sl[WB], sh[WB];
    __shared__ int32_t snn[WN];
    __shared__ uint32_t s_keep[kPlocChunk / 64], s_make[kPlocChunk / 64];
    const uint32_t m = *m_ptr;
    const bool merge = m > kPlocSmall;
    const uint32_t w = threadIdx.x >> 6;
    for (uint32_t c0 = blockIdx.x * kPlocChunk; c0 < m; c0 += gridDim.x * kPlocChunk) {
        __syncthreads();   // the previous step's windows are no longer read
        if (merge) {
            // boxes of clusters [c0 - 2R, c0 + chunk + 2R), the part inside [0, m)
            const long long b0 = (long long)c0 - 2 * (long long)R;
            for (uint32_t t = threadIdx.x; t < WB; t += blockDim.x) {
                const long long g = b0 + (long long)t;
                if (g >= 0 && g < (long long)m) {
                    sl[t] = cl[g];
                    sh[t] = ch[g];
                }
            }
            __syncthreads();
            // neighbours of clusters [c0 - R, c0 + chunk + R)
            for (uint32_t t = threadIdx.x; t < WN; t += blockDim.x) {
                const long long x = (long long)c0 - (long long)R + (long long)t;
                int32_t r = -1;
                if (x >= 0 && x < (long long)m)
                    r = ploc_nearest((uint32_t)x, m, [&](uint32_t y, float4& l, float4& h) {
                        const uint32_t k = (uint32_t)((long long)y - b0);   // |y - x| <= R: inside the window
                        l = sl[k];
                        h = sh[k];
                    });
                snn[t] = r;
            }
            __syncthreads();
        }
        const uint32_t i = c0 + threadIdx.x;
        uint32_t f = 0;
        if (i < m) {
            f = 1u;
            if (merge) {
                const int32_t j = snn[threadIdx.x + R];
                const long long kj = (long long)j - (long long)c0 + (long long)R;   // j within R of i
                const bool mutual = j >= 0 && snn[kj] == (int32_t)i;
                f = !mutual ? 1u : ((uint32_t)j > i ? 3u : 0u);
                nn[i] = j;
            }
            fl[i] = (uint8_t)f;
        }
        const unsigned long long mk = __ballot(f & 1u), mm = __ballot(f >> 1);
        if ((threadIdx.x & 63u) == 0) {
            s_keep[w] = (uint32_t)__popcll(mk);
            s_make[w] = (uint32_t)__popcll(mm);
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            uint32_t a = 0, b = 0;
            for (uint32_t k = 0; k < kPlocChunk / 64; ++k) {
                a += s_keep[k];
                b += s_make[k];
            }
            chunk_cnt[c0 / kPlocChunk] = make_uint2(a, b);
        }
    }
}

// inclusive scan of a pair of counts over a block of 1024 threads (16
// waves); returns the block's totals in tot
__device__ __forceinline__ uint2 block_scan_1024(uint2 c, uint2& tot) {
    __shared__ uint2 wsum[16];
    const uint32_t lane = threadIdx.x & 63u, w = threadIdx.x >> 6;
    uint2 v = c;
    for (uint32_t off = 1; off < 64; off <<= 1) {
        const uint32_t x = __shfl_up(v.x, off), y = __shfl_up(v.y, off);
        if (lane >= off) {
            v.x += x;
            v.y += y;
        }
    }
    if (lane == 63) wsum[w] = v;
    __syncthreads();
    if (w == 0) {
        uint2 s = lane < 16 ? wsum[lane] : make_uint2(0u, 0u);
        for (uint32_t off = 1; off < 16; off <<= 1) {
            const uint32_t x = __shfl_up(s.x, off), y = __shfl_up(s.y, off);
            if (lane >= off) {
                s.x += x;
                s.y += y;
            }
        }
        if (lane < 16) wsum[lane] = s;
    }
    __syncthreads();
    if (w > 0) {
        v.x += wsum[w - 1].x;
        v.y += wsum[w - 1].y;
    }
    tot = wsum[15];
    __syncthreads();   // wsum is reused by the next call
    return v;
}

// The last kPlocSmall clusters or fewer, clustered to one by a single
// block of 1024 threads with the clusters in LDS (iterations separated by
// barriers instead of launches); does nothing at more clusters or at one.
// Thread t takes a contiguous run of at most kPlocSmall / 1024 clusters,
// so a block-wide scan of the per-thread counts keeps the survivors in
// order; they are written back in place once every thread has read its
// inputs.
constexpr uint32_t kPlocPer = kPlocSmall / 1024;
__global__ __launch_bounds__(1024) void k_ploc_finish(uint32_t n, uint32_t* __restrict__ pm, uint32_t par,
                                                       const float4* __restrict__ al, const float4* __restrict__ ah,
                                                       const float4* __restrict__ bl, const float4* __restrict__ bh,
                                                       int32_t* __restrict__ left, int32_t* __restrict__ right,
                                                       float4* __restrict__ nlo, float4* __restrict__ nhi) {
    __shared__ float4 sl[kPlocSmall], sh[kPlocSmall];
    __shared__ int16_t snn[kPlocSmall];
    uint32_t m = pm[par];
    if (m > kPlocSmall || m <= 1) return;
    const float4* gl = par ? bl : al;
    const float4* gh = par ? bh : ah;
    const uint32_t t = threadIdx.x;
    for (uint32_t i = t; i < m; i += blockDim.x) {
        sl[i] = gl[i];
        sh[i] = gh[i];
    }
    uint32_t done = pm[2];
    __syncthreads();
    while (m > 1) {
        for (uint32_t i = t; i < m; i += blockDim.x)
            snn[i] = (int16_t)ploc_nearest(i, m, [&](uint32_t y, float4& l, float4& h) {
                l = sl[y];
                h = sh[y];
            });
        __syncthreads();
        const uint32_t per = (m + 1023u) / 1024u;   // <= kPlocPer
        const uint32_t i0 = min(m, t * per), i1 = min(m, i0 + per);
        uint2 c = make_uint2(0u, 0u);
        for (uint32_t i = i0; i < i1; ++i) {
            const int32_t j = snn[i];
            const bool mutual = j >= 0 && snn[j] == (int16_t)i;
            c.x += (!mutual || (uint32_t)j > i) ? 1u : 0u;
            c.y += (mutual && (uint32_t)j > i) ? 1u : 0u;
        }
        uint2 tot;
        const uint2 inc = block_scan_1024(c, tot);
        uint32_t pos = inc.x - c.x, made = inc.y - c.y;
        float4 ol[kPlocPer], oh[kPlocPer];
        bool ok[kPlocPer];
#pragma unroll
        for (uint32_t k = 0; k < kPlocPer; ++k) {
            const uint32_t i = i0 + k;
            ok[k] = false;
            if (i >= i1) continue;
            const int32_t j = snn[i];
            const bool mutual = j >= 0 && snn[j] == (int16_t)i;
            if (mutual && (uint32_t)j < i) continue;   // merged into its partner
            float4 a = sl[i], b = sh[i];
            if (mutual) {
                const float4 c2 = sl[j], d2 = sh[j];
                const uint32_t id = (n - 2u) - (done + made);
                ++made;
                left[id] = __float_as_int(b.w);
                right[id] = __float_as_int(d2.w);
                a = make_float4(fminf(a.x, c2.x), fminf(a.y, c2.y), fminf(a.z, c2.z),
                                __uint_as_float(__float_as_uint(a.w) + __float_as_uint(c2.w)));
                b = make_float4(fmaxf(b.x, d2.x), fmaxf(b.y, d2.y), fmaxf(b.z, d2.z), __int_as_float((int32_t)id));
                nlo[id] = a;
                nhi[id] = b;
            }
            ol[k] = a;
            oh[k] = b;
            ok[k] = true;
        }
        __syncthreads();   // every thread has read its inputs
#pragma unroll
        for (uint32_t k = 0; k < kPlocPer; ++k)
            if (ok[k]) {
                sl[pos] = ol[k];
                sh[pos] = oh[k];
                ++pos;
            }
        __syncthreads();
        m = tot.x;
        done += tot.y;
    }
    if (t == 0) {
        pm[par] = 1u;
        pm[2] = done;
    }
}

// Exclusive scan of the chunk counts (one block of 1024 threads); the next
// cluster count goes to pm[1 - par], this iteration's first node number to
// pm[3], and the running node count pm[2] grows by the nodes made.
__global__ __launch_bounds__(1024) void k_ploc_scan(uint32_t* __restrict__ pm, uint32_t par,
                                                     uint2* __restrict__ chunk_cnt) {
    __shared__ uint2 part[1024];
    const uint32_t m = pm[par];
    const uint32_t nc = (m + kPlocChunk - 1) / kPlocChunk;
    const uint32_t per = (nc + 1023u) / 1024u;
    const uint32_t b0 = threadIdx.x * per, b1 = min(nc, b0 + per);
    uint2 s = make_uint2(0u, 0u);
    for (uint32_t c = b0; c < b1; ++c) {
        const uint2 v = chunk_cnt[c];
        s.x += v.x;
        s.y += v.y;
    }
    part[threadIdx.x] = s;
    __syncthreads();
    for (uint32_t off = 1; off < 1024; off <<= 1) {   // inclusive scan over the threads
        uint2 v = make_uint2(0u, 0u);
        if (threadIdx.x >= off) v = part[threadIdx.x - off];
        __syncthreads();
        part[threadIdx.x].x += v.x;
        part[threadIdx.x].y += v.y;
        __syncthreads();
    }
    uint2 run = threadIdx.x ? part[threadIdx.x - 1] : make_uint2(0u, 0u);
    for (uint32_t c = b0; c < b1; ++c) {
        const uint2 v = chunk_cnt[c];
        chunk_cnt[c] = run;
        run.x += v.x;
        run.y += v.y;
    }
    if (threadIdx.x == 1023) {
        pm[1 - par] = part[1023].x;
        pm[3] = pm[2];
        pm[2] += part[1023].y;
    }
}

// Compaction: surviving clusters to their places in order; a cluster that
// makes a node writes the node (children, box, size) and stands for it.
__global__ __launch_bounds__(kPlocChunk) void k_ploc_merge(uint32_t n, const uint32_t* __restrict__ pm, uint32_t par,
                                                            const float4* __restrict__ cl, const float4* __restrict__ ch,
                                                            const int32_t* __restrict__ nn,
                                                            const uint8_t* __restrict__ fl,
                                                            const uint2* __restrict__ chunk_off,
                                                            float4* __restrict__ ol, float4* __restrict__ oh,
                                                            int32_t* __restrict__ left, int32_t* __restrict__ right,
                                                            float4* __restrict__ nlo, float4* __restrict__ nhi) {
    __shared__ uint32_t s_keep[kPlocChunk / 64], s_make[kPlocChunk / 64];
    const uint32_t m = pm[par];
    const uint32_t node_base = pm[3];
    const uint32_t w = threadIdx.x >> 6;
    for (uint32_t c0 = blockIdx.x * kPlocChunk; c0 < m; c0 += gridDim.x * kPlocChunk) {
        const uint32_t i = c0 + threadIdx.x;
        const uint32_t f = i < m ? fl[i] : 0u;
        const unsigned long long mk = __ballot(f & 1u), mm = __ballot(f >> 1);
        if ((threadIdx.x & 63u) == 0) {
            s_keep[w] = (uint32_t)__popcll(mk);
            s_make[w] = (uint32_t)__popcll(mm);
        }
        __syncthreads();
        uint32_t kb = 0, mb = 0;   // this wave's offsets in the chunk
        for (uint32_t k = 0; k < w; ++k) {
            kb += s_keep[k];
            mb += s_make[k];
        }
        __syncthreads();   // s_keep and s_make are rewritten by the next chunk
        if (!(f & 1u)) continue;
        const uint2 off = chunk_off[c0 / kPlocChunk];
        const uint32_t lane_keep = __builtin_amdgcn_mbcnt_hi((uint32_t)(mk >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)mk, 0u));
        const uint32_t p = off.x + kb + lane_keep;
        float4 a = cl[i], b = ch[i];
        if (f & 2u) {
            const uint32_t j = (uint32_t)nn[i];
            const float4 c = cl[j], d = ch[j];
            const uint32_t lane_make = __builtin_amdgcn_mbcnt_hi((uint32_t)(mm >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)mm, 0u));
            const uint32_t id = (n - 2u) - (node_base + off.y + mb + lane_make);
            left[id] = __float_as_int(b.w);
            right[id] = __float_as_int(d.w);
            a = make_float4(fminf(a.x, c.x), fminf(a.y, c.y), fminf(a.z, c.z),
                            __uint_as_float(__float_as_uint(a.w) + __float_as_uint(c.w)));
            b = make_float4(fmaxf(b.x, d.x), fmaxf(b.y, d.y), fmaxf(b.z, d.z), __int_as_float((int32_t)id));
            nlo[id] = a;
            nhi[id] = b;
        }
        ol[p] = a;
        oh[p] = b;
    }
}

// Leaf clusters: the key-sorted triangles' boxes, size 1.
__global__ void k_ploc_init(const unsigned long long* __restrict__ keys, const float* __restrict__ tb, uint32_t n,
                            float4* __restrict__ cl, float4* __restrict__ ch) {
    for (uint32_t p = blockIdx.x * blockDim.x + threadIdx.x; p < n; p += gridDim.x * blockDim.x) {
        const uint32_t prim = (uint32_t)(keys[p] & kKeyIndexMask);
        const float* b = tb + 6 * (size_t)prim;
        cl[p] = make_float4(b[0], b[1], b[2], __uint_as_float(1u));
        ch[p] = make_float4(b[3], b[4], b[5], __int_as_float((int32_t)(n - 1 + p)));
    }
}

// Clustering start state: n clusters, no nodes made; the root (node 0, or
// the single leaf when n == 1) as the one work item of the collapse.
__global__ void k_ploc_start(uint32_t* pm, uint32_t n, uint4* work0) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        pm[0] = n;
        pm[1] = 0u;
        pm[2] = 0u;
        pm[3] = 0u;
        work0[0] = make_uint4(0u, 0u, 0u, 0u);
    }
}

// One level of the collapse of a tree with explicit node boxes and subtree
// sizes (the clustering's): work[i] = (binary node, wide node, first leaf
// position, -).  Subtrees are laid out depth first, left before right, so
// a node of size s whose first leaf goes to position lo holds positions
// [lo, lo + s).  A child of at most leaf_max triangles becomes a leaf; its
// binary subtree's root is left in the node's pad word for k_leaf_keys.
__global__ void k_collapse_boxed(uint32_t n, const int32_t* __restrict__ left, const int32_t* __restrict__ right,
                                 const float4* __restrict__ nlo, const float4* __restrict__ nhi,
                                 const float* __restrict__ tb, const unsigned long long* __restrict__ keys,
                                 uint32_t leaf_max, uint32_t width, const uint4* __restrict__ work,
                                 const uint32_t* __restrict__ n_work, uint4* next_work, uint32_t* n_next,
                                 uint32_t* n_nodes, BNode* nodes) {
    const uint32_t nw = *n_work;
    const int32_t first_leaf = (int32_t)(n - 1);
    auto size_of = [&](int32_t c) -> uint32_t { return c >= first_leaf ? 1u : __float_as_uint(nlo[c].w); };
    auto box_of = [&](int32_t c, float* b) {
        if (c >= first_leaf) {
            const uint32_t prim = (uint32_t)(keys[c - first_leaf] & kKeyIndexMask);
            for (int k = 0; k < 6; ++k) b[k] = tb[6 * (size_t)prim + k];
        } else {
            const float4 l = nlo[c], h = nhi[c];
            b[0] = l.x; b[1] = l.y; b[2] = l.z;
            b[3] = h.x; b[4] = h.y; b[5] = h.z;
        }
    };
    for (uint32_t w = blockIdx.x * blockDim.x + threadIdx.x; w < nw; w += gridDim.x * blockDim.x) {
        const uint4 item = work[w];
        int32_t set[8];
        uint32_t slo[8];
        int cnt = 0;
        const int32_t root = (int32_t)item.x;
        // area of each candidate that may be opened (-2: leaf-sized)
        float area[8];
        auto area_of = [&](int32_t c) -> float {
            if (size_of(c) <= leaf_max) return -2.0f;
            float bx[6];
            box_of(c, bx);
            return half_area(bx);
        };
        if (root >= first_leaf) {
            set[0] = root;   // a single-triangle tree
            slo[0] = item.z;
            area[0] = -2.0f;
            cnt = 1;
        } else {
            set[0] = left[root];
            slo[0] = item.z;
            area[0] = area_of(set[0]);
            set[1] = right[root];
            slo[1] = item.z + size_of(set[0]);
            area[1] = area_of(set[1]);
            cnt = 2;
        }
        while (cnt < (int)width) {   // open the largest candidate (the first of equal ones)
            int best = -1;
            float ba = -1.0f;
            for (int c = 0; c < cnt; ++c)
                if (area[c] > ba) { ba = area[c]; best = c; }
            if (best < 0) break;
            const int32_t c = set[best];
            const uint32_t lo = slo[best];
            const uint32_t lsz = size_of(left[c]);
            set[best] = left[c];
            area[best] = area_of(set[best]);
            set[cnt] = right[c];
            slo[cnt] = lo + lsz;
            area[cnt] = area_of(set[cnt]);
            ++cnt;
        }
        BNode node;
        for (int c = 0; c < 8; ++c) {
            if (c < cnt) {
                const uint32_t sz = size_of(set[c]);
                float b[6];
                box_of(set[c], b);
                node.lox[c] = b[0]; node.loy[c] = b[1]; node.loz[c] = b[2];
                node.hix[c] = b[3]; node.hiy[c] = b[4]; node.hiz[c] = b[5];
                if (sz <= leaf_max) {
                    // the leaf's binary subtree, for k_leaf_keys (which clears the word)
                    node.child[c] = SC_LEAF_BIT | ((sz - 1) << 28) | slo[c];
                    node.pad[c] = (uint32_t)set[c];
                    continue;
                } else {
                    const uint32_t idx = atomicAdd(n_nodes, 1u);
                    const uint32_t q = atomicAdd(n_next, 1u);
                    next_work[q] = make_uint4((uint32_t)set[c], idx, slo[c], 0u);
                    node.child[c] = idx;
                }
                node.pad[c] = 0;
            } else {
                node.lox[c] = INFINITY; node.loy[c] = INFINITY; node.loz[c] = INFINITY;
                node.hix[c] = -INFINITY; node.hiy[c] = -INFINITY; node.hiz[c] = -INFINITY;
                node.child[c] = SC_CHILD_EMPTY;
                node.pad[c] = 0;
            }
        }
        nodes[item.y] = node;
    }
}

// The keys of every leaf's triangles at the leaf's positions, depth first
// through the leaf's binary subtree (root in the node's pad word, cleared
// here); one thread per child slot of the wide nodes.
__global__ void k_leaf_keys(uint32_t n, BNode* nodes, uint32_t n_nodes, const int32_t* __restrict__ left,
                            const int32_t* __restrict__ right, const unsigned long long* __restrict__ keys,
                            unsigned long long* __restrict__ keys_out) {
    const int32_t first_leaf = (int32_t)(n - 1);
    for (uint32_t s = blockIdx.x * blockDim.x + threadIdx.x; s < 8 * n_nodes; s += gridDim.x * blockDim.x) {
        BNode& nd = nodes[s / 8];
        const uint32_t c = s % 8;
        const uint32_t ch = nd.child[c];
        if (ch == SC_CHILD_EMPTY || !(ch & SC_LEAF_BIT)) continue;
        const uint32_t lo = ch & 0x0FFFFFFFu, end = lo + ((ch >> 28) & 7u) + 1u;
        // (the bounds on top and pos hold for any tree of end - lo leaves)
        int32_t stk[8];
        int top = 0;
        uint32_t pos = lo;
        stk[top++] = (int32_t)nd.pad[c];
        while (top > 0 && pos < end) {
            const int32_t x = stk[--top];
            if (x >= first_leaf) {
                if ((uint32_t)(x - first_leaf) < n) keys_out[pos] = keys[x - first_leaf];
                ++pos;
            } else if (x >= 0 && top + 2 <= 8) {
                stk[top++] = right[x];
                stk[top++] = left[x];
            }
        }
        nd.pad[c] = 0;
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
    // automatic choice: the clustering's fewer node fetches pay for its
    // longer build from about a million triangles (2M: build 2.4 -> 4.5 ms,
    // traversal -6.5 ms per 1080p 64-spp step; 198k: build 0.7 -> 2.1 ms,
    // traversal -0.1 ms)
    const uint32_t kPlocAutoMin = 1u << 20;
    const bool ploc = ctx->bvh_builder == 1 || (ctx->bvh_builder == 2 && n >= kPlocAutoMin);
    uint32_t n_pad = 1;
    while (n_pad < n) n_pad <<= 1;
    if (n_pad < (uint32_t)kLocal) n_pad = kLocal;
    uint32_t levels = 1;
    while ((2u << (levels - 1)) <= n) ++levels;   // levels 0..floor(log2 n)
    const uint32_t nseg = (n + 255u) / 256u;
    const size_t ni = n > 1 ? n - 1 : 1;

    // temporaries, carved from one grow-only buffer of the context
    uint32_t *meta, *cb, *rlo = nullptr, *rhi = nullptr, *seg_cnt, *seg_off, *e_prim;
    float *bounds, *st_buf = nullptr, *e_v;
    unsigned long long *keys, *keys_out = nullptr;
    int32_t *left, *right, *nn = nullptr;
    uint2 *work_a = nullptr, *work_b = nullptr, *chunk_cnt = nullptr;
    uint4 *work4_a = nullptr, *work4_b = nullptr;
    float4 *cla_l = nullptr, *cla_h = nullptr, *clb_l = nullptr, *clb_h = nullptr, *nlo = nullptr, *nhi = nullptr;
    uint32_t* pm = nullptr;
    uint8_t* fl = nullptr;
    BNode* nodes_tmp;
    const uint32_t n_chunks = (n + kPlocChunk - 1) / kPlocChunk;
    auto carve = [&](char* base) {
        Carver c{base};
        meta = c.take<uint32_t>(kMeta);
        cb = c.take<uint32_t>(6);
        bounds = c.take<float>(6 * (size_t)n);
        keys = c.take<unsigned long long>(n_pad);
        left = c.take<int32_t>(ni);
        right = c.take<int32_t>(ni);
        if (ploc) {   // clusters (two buffers), nearest neighbours, flags, node boxes, final key order
            pm = c.take<uint32_t>(4);
            cla_l = c.take<float4>(n);
            cla_h = c.take<float4>(n);
            clb_l = c.take<float4>(n);
            clb_h = c.take<float4>(n);
            nlo = c.take<float4>(ni);
            nhi = c.take<float4>(ni);
            nn = c.take<int32_t>(n);
            fl = c.take<uint8_t>(n);
            chunk_cnt = c.take<uint2>(n_chunks);
            keys_out = c.take<unsigned long long>(n);
            work4_a = c.take<uint4>(n);
            work4_b = c.take<uint4>(n);
        } else {      // radix tree key ranges and the range-union table
            rlo = c.take<uint32_t>(ni);
            rhi = c.take<uint32_t>(ni);
            st_buf = c.take<float>(6 * (size_t)n * levels);
            work_a = c.take<uint2>(n);
            work_b = c.take<uint2>(n);
        }
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
    SC_LAUNCH(k_build_init, dim3(1), dim3(256), 0, st, meta, kMeta, ploc ? nullptr : work_a, cb);
    if (ploc) SC_LAUNCH(k_ploc_start, dim3(1), dim3(64), 0, st, pm, n, work4_a);
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
    if (ploc) {
        // agglomerative clustering; the launches read the cluster count from
        // the device, the host reads it after each batch of iterations and
        // sizes the grids by the last count read, which only decreases
        SC_LAUNCH(k_ploc_init, dim3(grid_for(n, bs)), dim3(bs), 0, st, keys, bounds, n, cla_l, cla_h);
        uint32_t m_h = n, it = 0;
        while (m_h > 1) {
            const uint32_t g = grid_for((m_h + kPlocChunk - 1) / kPlocChunk, 1, 1024);
            // iterations expected down to kPlocSmall clusters (measured: about
            // 16 % of the clusters go per iteration on the test scenes), then
            // the single-block finish
            uint32_t batch = 0;
            for (double mm = m_h; mm > kPlocSmall && batch < 96; mm *= 0.84) ++batch;
            for (uint32_t k = 0; k < batch; ++k, ++it) {
                const uint32_t par = it & 1u;
                const float4* sl = par ? clb_l : cla_l;
                const float4* sh = par ? clb_h : cla_h;
                float4* dl = par ? cla_l : clb_l;
                float4* dh = par ? cla_h : clb_h;
                SC_LAUNCH(k_ploc_nn_flags, dim3(g), dim3(kPlocChunk), 0, st, pm + par, sl, sh, nn, fl, chunk_cnt);
                SC_LAUNCH(k_ploc_scan, dim3(1), dim3(1024), 0, st, pm, par, chunk_cnt);
                SC_LAUNCH(k_ploc_merge, dim3(g), dim3(kPlocChunk), 0, st, n, pm, par, sl, sh, nn, fl, chunk_cnt,
                          dl, dh, left, right, nlo, nhi);
            }
            SC_LAUNCH(k_ploc_finish, dim3(1), dim3(1024), 0, st, n, pm, it & 1u, cla_l, cla_h, clb_l, clb_h, left,
                      right, nlo, nhi);
            SC_HIP(hipMemcpyAsync(&m_h, pm + (it & 1u), 4, hipMemcpyDeviceToHost, st));
            SC_HIP(hipStreamSynchronize(st));
            // every iteration merges at least the best pair of the whole list
            if (it > n + 64) return set_error(SC_EDEVICE, "BVH clustering did not converge");
        }
    } else {
        // radix tree
        if (n > 1) SC_LAUNCH(k_radix_tree, dim3(grid_for(n - 1, bs)), dim3(bs), 0, st, keys, n, left, right, rlo, rhi);
        // range-union table for node boxes
        SC_LAUNCH(k_sparse_level0, dim3(grid_for(n, bs)), dim3(bs), 0, st, keys, bounds, n, st_buf);
        for (uint32_t L = 1; L < levels; ++L)
            SC_LAUNCH(k_sparse_level, dim3(grid_for(n - (1u << L) + 1, bs)), dim3(bs), 0, st, st_buf, n, L);
    }

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
            if (ploc) {
                const uint4* wa = (L & 1u) ? work4_b : work4_a;
                uint4* wb = (L & 1u) ? work4_a : work4_b;
                SC_LAUNCH(k_collapse_boxed, dim3(grid_for(n, 128, 512)), dim3(128), 0, st, n, left, right, nlo, nhi,
                          bounds, keys, leaf_max, width, wa, meta + 8 + L, wb, meta + 9 + L, meta + 1, nodes_tmp);
            } else {
                const uint2* wa = (L & 1u) ? work_b : work_a;
                uint2* wb = (L & 1u) ? work_a : work_b;
                SC_LAUNCH(k_collapse, dim3(grid_for(n, 128, 512)), dim3(128), 0, st, n, left, right, rlo, rhi, st_buf,
                          leaf_max, width, wa, meta + 8 + L, wb, meta + 9 + L, meta + 1, nodes_tmp);
            }
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

    if (ploc)
        SC_LAUNCH(k_leaf_keys, dim3(grid_for(8 * (size_t)n_nodes, bs)), dim3(bs), 0, st, n, nodes_tmp, n_nodes, left,
                  right, keys, keys_out);
    SC_TRY(b->nodes.ensure(sizeof(BNode) * (size_t)n_nodes));
    SC_HIP(hipMemcpyAsync(b->nodes.p, nodes_tmp, sizeof(BNode) * (size_t)n_nodes, hipMemcpyDeviceToDevice, st));
    // padded: the traversal fetches 14 float4 from a leaf's first triangle
    SC_TRY(b->tris.ensure(sizeof(float4) * (3 * (size_t)n + 14)));
    SC_LAUNCH(k_gather_tris, dim3(grid_for(n, bs)), dim3(bs), 0, st, ploc ? keys_out : keys, n, sc.V, sc.nv, sc.I,
              b->tris.as<float4>());
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
