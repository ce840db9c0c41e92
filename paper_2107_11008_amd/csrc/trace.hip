// trace.hip -- wavefront path tracing, photon tracing and ground-truth
// kernels for gfx950.
//
// Rays live in structure-of-arrays buffers indexed by a stable path id;
// queues of path ids connect the stages:
//   raygen -> [closest hit -> classify (sort by material, compact) ->
//              shade dielectric | shade diffuse (+ shadow ray) ->
//              any hit (shadow) ] x depth -> film
// Queue appends use one atomic per wave (ballot + mbcnt prefix).
// Traversal kernels fetch 64 rays per wave from a per-launch atomic
// counter, keep the traversal stack in LDS (spilling to scratch only for
// deep trees) and visit the children of a wide node front to back.
#pragma clang fp contract(off)
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "sc_device.h"
#include "sc_internal.h"
#include "sc_kernels.h"

using namespace scd;

namespace {

constexpr int kTraceBS = 128;
constexpr int kLdsStack = 16;

__device__ __forceinline__ uint32_t lane_id() { return __lane_id(); }

__device__ __forceinline__ uint32_t lanes_below(unsigned long long m) {
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

// Append `val` to queue q for lanes with pred; one atomic per wave.  Every
// lane of the wave must call this.
__device__ __forceinline__ void wave_push(bool pred, uint32_t val, uint32_t* q, uint32_t* cnt) {
    const unsigned long long m = __ballot(pred);
    if (m == 0ull) return;
    const uint32_t leader = __ffsll((long long)m) - 1;
    uint32_t base = 0;
    if (lane_id() == leader) base = atomicAdd(cnt, (uint32_t)__popcll(m));
    base = __shfl(base, (int)leader);
    if (pred) q[base + lanes_below(m)] = val;
}

__device__ __forceinline__ unsigned long long wave_sum_u64(unsigned long long v) {
    for (int off = 32; off > 0; off >>= 1) {
        const uint32_t lo = __shfl_xor((uint32_t)v, off);
        const uint32_t hi = __shfl_xor((uint32_t)(v >> 32), off);
        v += ((unsigned long long)hi << 32) | lo;
    }
    return v;
}

__device__ __forceinline__ float safe_inv(float d) {
    const float a = fabsf(d) < 1e-20f ? copysignf(1e-20f, d) : d;
    return 1.0f / a;
}

// search bound: a node is visited if its entry distance is within a
// relative margin of the best hit, so equal-distance triangles with a
// smaller index in other nodes are still found
__device__ __forceinline__ float search_limit(float t) { return t + t * 9.765625e-04f; }

// traversal stack: the first kLdsStack entries of each lane in LDS, deeper
// entries in a private (scratch) array
struct Spill {
    uint2 e[kMaxStack - kLdsStack];
};

__device__ __forceinline__ void push(uint2 (*lds)[kTraceBS], Spill& s, int& sp, uint2 e) {
    if (sp < kLdsStack) lds[sp][threadIdx.x] = e;
    else s.e[sp - kLdsStack] = e;
    ++sp;
}
__device__ __forceinline__ uint2 pop(uint2 (*lds)[kTraceBS], Spill& s, int& sp) {
    --sp;
    return sp < kLdsStack ? lds[sp][threadIdx.x] : s.e[sp - kLdsStack];
}

__device__ __forceinline__ void cswap(uint32_t& ka, uint32_t& va, uint32_t& kb, uint32_t& vb) {
    const bool sw = kb < ka;
    const uint32_t k0 = sw ? kb : ka, k1 = sw ? ka : kb;
    const uint32_t v0 = sw ? vb : va, v1 = sw ? va : vb;
    ka = k0; kb = k1; va = v0; vb = v1;
}

// Batcher's odd-even merge sort of 8 (key, value) pairs, ascending keys
__device__ __forceinline__ void sort8(uint32_t* k, uint32_t* v) {
#define CS(a, b) cswap(k[a], v[a], k[b], v[b])
    CS(0, 1); CS(2, 3); CS(4, 5); CS(6, 7);
    CS(0, 2); CS(1, 3); CS(4, 6); CS(5, 7);
    CS(1, 2); CS(5, 6);
    CS(0, 4); CS(1, 5); CS(2, 6); CS(3, 7);
    CS(2, 4); CS(3, 5);
    CS(1, 2); CS(3, 4); CS(5, 6);
#undef CS
}

struct NodeTest {
    uint32_t key[8];
    uint32_t ref[8];
};

// Box tests of the 8 children against (o, inv); near/far planes chosen by
// the sign of each direction component.  key = entry distance bits, or
// 0xffffffff when the child is missed or lies beyond tlim.
__device__ __forceinline__ void test_node(const BNode* __restrict__ nd, F3 o, F3 inv, float tlim, NodeTest& r) {
    const float4* q = reinterpret_cast<const float4*>(nd);
    // q[0..1] lox, q[2..3] hix, q[4..5] loy, q[6..7] hiy, q[8..9] loz, q[10..11] hiz, q[12..13] child
    const bool px = inv.x >= 0.0f, py = inv.y >= 0.0f, pz = inv.z >= 0.0f;
    float4 nx0 = q[px ? 0 : 2], nx1 = q[px ? 1 : 3], fx0 = q[px ? 2 : 0], fx1 = q[px ? 3 : 1];
    float4 ny0 = q[py ? 4 : 6], ny1 = q[py ? 5 : 7], fy0 = q[py ? 6 : 4], fy1 = q[py ? 7 : 5];
    float4 nz0 = q[pz ? 8 : 10], nz1 = q[pz ? 9 : 11], fz0 = q[pz ? 10 : 8], fz1 = q[pz ? 11 : 9];
    const uint4 c0 = reinterpret_cast<const uint4*>(nd)[12];
    const uint4 c1 = reinterpret_cast<const uint4*>(nd)[13];
    const float nx[8] = {nx0.x, nx0.y, nx0.z, nx0.w, nx1.x, nx1.y, nx1.z, nx1.w};
    const float fx[8] = {fx0.x, fx0.y, fx0.z, fx0.w, fx1.x, fx1.y, fx1.z, fx1.w};
    const float ny[8] = {ny0.x, ny0.y, ny0.z, ny0.w, ny1.x, ny1.y, ny1.z, ny1.w};
    const float fy[8] = {fy0.x, fy0.y, fy0.z, fy0.w, fy1.x, fy1.y, fy1.z, fy1.w};
    const float nz[8] = {nz0.x, nz0.y, nz0.z, nz0.w, nz1.x, nz1.y, nz1.z, nz1.w};
    const float fz[8] = {fz0.x, fz0.y, fz0.z, fz0.w, fz1.x, fz1.y, fz1.z, fz1.w};
    const uint32_t ch[8] = {c0.x, c0.y, c0.z, c0.w, c1.x, c1.y, c1.z, c1.w};
#pragma unroll
    for (int c = 0; c < 8; ++c) {
        const float tnx = (nx[c] - o.x) * inv.x, tfx = (fx[c] - o.x) * inv.x;
        const float tny = (ny[c] - o.y) * inv.y, tfy = (fy[c] - o.y) * inv.y;
        const float tnz = (nz[c] - o.z) * inv.z, tfz = (fz[c] - o.z) * inv.z;
        const float tn = fmaxf(fmaxf(tnx, tny), fmaxf(tnz, 0.0f));
        const float tf = fminf(fminf(tfx, tfy), tfz);
        const bool hit = (tn <= tf + fabsf(tf) * 9.765625e-04f) && (tn <= tlim);
        r.key[c] = hit ? __float_as_uint(tn) : 0xffffffffu;
        r.ref[c] = ch[c];
    }
}

__device__ __forceinline__ F3 perm(const RayPre& r, float4 p) { return permute(r, F3{p.x, p.y, p.z}); }

// ------------------------------------------------------------------ closest hit
template <bool COUNT>
__global__ __launch_bounds__(kTraceBS) void k_closest(DevScene S, RaySoA R, HitSoA H, const uint32_t* __restrict__ queue,
                                                      const uint32_t* __restrict__ count, uint32_t n_static,
                                                      uint32_t* __restrict__ work, DevCounters* __restrict__ C) {
    __shared__ uint2 lds[kLdsStack][kTraceBS];
    Spill st;
    int sp = 0;
    const uint32_t n = count ? *count : n_static;
    unsigned long long c_nodes = 0, c_tris = 0, c_rays = 0;
    for (;;) {
        uint32_t base = 0;
        if (lane_id() == 0) base = atomicAdd(work, 64u);
        base = __shfl(base, 0);
        if (base >= n) break;
        const uint32_t i = base + lane_id();
        if (i < n) {
            const uint32_t pid = queue ? queue[i] : i;
            const F3 o{R.ox[pid], R.oy[pid], R.oz[pid]};
            const F3 d{R.dx[pid], R.dy[pid], R.dz[pid]};
            const RayPre rp = ray_prepare(o, d);
            const F3 inv{safe_inv(d.x), safe_inv(d.y), safe_inv(d.z)};
            float tb = INFINITY, bV = 0.0f, bW = 0.0f, brcp = 0.0f;
            uint32_t pb = 0xffffffffu;
            sp = 0;
            uint32_t ref = 0;   // root node
            bool have = true;
            while (have) {
                if (!(ref & SC_LEAF_BIT)) {
                    NodeTest nt;
                    test_node(S.nodes + ref, o, inv, search_limit(tb), nt);
                    if (COUNT) ++c_nodes;
                    sort8(nt.key, nt.ref);
                    if (nt.key[0] != 0xffffffffu) {
#pragma unroll
                        for (int c = 7; c >= 1; --c)
                            if (nt.key[c] != 0xffffffffu) push(lds, st, sp, make_uint2(nt.ref[c], nt.key[c]));
                        ref = nt.ref[0];
                        continue;
                    }
                } else {
                    const uint32_t first = ref & SC_LEAF_FIRST_MASK;
                    const uint32_t cnt = ((ref >> 28) & 7u) + 1u;
                    if (COUNT) c_tris += cnt;
                    for (uint32_t k = 0; k < cnt; ++k) {
                        const float4* tp = S.tris + 3 * (size_t)(first + k);
                        const float4 a = tp[0], b = tp[1], c = tp[2];
                        const uint32_t prim = __float_as_uint(a.w);
                        TriHit h;
                        if (tri_test(rp, perm(rp, a), perm(rp, b), perm(rp, c), h)) {
                            if (h.t < tb || (h.t == tb && prim < pb)) {
                                tb = h.t; pb = prim; bV = h.V; bW = h.W; brcp = h.rcp;
                            }
                        }
                    }
                }
                // next entry from the stack that is still within reach
                have = false;
                while (sp > 0) {
                    const uint2 e = pop(lds, st, sp);
                    if (__uint_as_float(e.y) <= search_limit(tb)) {
                        ref = e.x;
                        have = true;
                        break;
                    }
                }
            }
            H.t[pid] = tb;
            H.prim[pid] = pb;
            if (H.u) H.u[pid] = bV * brcp;
            if (H.v) H.v[pid] = bW * brcp;
            ++c_rays;
        }
    }
    c_rays = wave_sum_u64(c_rays);
    if (COUNT) {
        c_nodes = wave_sum_u64(c_nodes);
        c_tris = wave_sum_u64(c_tris);
    }
    if (lane_id() == 0) {
        atomicAdd(&C->rays_closest, c_rays);
        if (COUNT) {
            atomicAdd(&C->node_visits, c_nodes);
            atomicAdd(&C->tri_tests, c_tris);
        }
    }
}

// ------------------------------------------------------------------ any hit
// Occlusion of segments (0, tmax) skipping triangle excl; for shadow rays of
// camera paths, an unoccluded segment adds its stored contribution to L.
__global__ __launch_bounds__(kTraceBS) void k_anyhit(DevScene S, ShadowSoA R, const uint32_t* __restrict__ queue,
                                                     const uint32_t* __restrict__ count, uint32_t n_static,
                                                     uint32_t* __restrict__ work, uint8_t* __restrict__ occ_out,
                                                     float* __restrict__ L, DevCounters* __restrict__ C) {
    __shared__ uint2 lds[kLdsStack][kTraceBS];
    Spill st;
    int sp = 0;
    const uint32_t n = count ? *count : n_static;
    unsigned long long c_rays = 0;
    for (;;) {
        uint32_t base = 0;
        if (lane_id() == 0) base = atomicAdd(work, 64u);
        base = __shfl(base, 0);
        if (base >= n) break;
        const uint32_t i = base + lane_id();
        if (i < n) {
            const uint32_t pid = queue ? queue[i] : i;
            const F3 o{R.ox[pid], R.oy[pid], R.oz[pid]};
            const F3 d{R.dx[pid], R.dy[pid], R.dz[pid]};
            const float tmax = R.tmax[pid];
            const uint32_t excl = R.excl ? R.excl[pid] : 0xffffffffu;
            const RayPre rp = ray_prepare(o, d);
            const F3 inv{safe_inv(d.x), safe_inv(d.y), safe_inv(d.z)};
            const float tlim = search_limit(tmax);
            bool occluded = false;
            sp = 0;
            uint32_t ref = 0;
            bool have = true;
            while (have && !occluded) {
                if (!(ref & SC_LEAF_BIT)) {
                    NodeTest nt;
                    test_node(S.nodes + ref, o, inv, tlim, nt);
#pragma unroll
                    for (int c = 0; c < 8; ++c)
                        if (nt.key[c] != 0xffffffffu) push(lds, st, sp, make_uint2(nt.ref[c], nt.key[c]));
                } else {
                    const uint32_t first = ref & SC_LEAF_FIRST_MASK;
                    const uint32_t cnt = ((ref >> 28) & 7u) + 1u;
                    for (uint32_t k = 0; k < cnt; ++k) {
                        const float4* tp = S.tris + 3 * (size_t)(first + k);
                        const float4 a = tp[0], b = tp[1], c = tp[2];
                        if (__float_as_uint(a.w) == excl) continue;
                        TriHit h;
                        if (tri_test(rp, perm(rp, a), perm(rp, b), perm(rp, c), h) && h.t < tmax) {
                            occluded = true;
                            break;
                        }
                    }
                }
                have = false;
                if (!occluded && sp > 0) {
                    ref = pop(lds, st, sp).x;
                    have = true;
                }
            }
            if (occ_out) occ_out[pid] = occluded ? 1 : 0;
            if (L && !occluded) L[pid] = L[pid] + R.contrib[pid];
            ++c_rays;
        }
    }
    c_rays = wave_sum_u64(c_rays);
    if (lane_id() == 0) atomicAdd(&C->rays_shadow, c_rays);
}

// ------------------------------------------------------------------ helpers
__global__ void k_zero_u32(uint32_t* p, uint32_t n) {
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) p[i] = 0u;
}
__global__ void k_zero_u64(unsigned long long* p, size_t n) {
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) p[i] = 0ull;
}
__global__ void k_zero_f32(float* p, size_t n) {
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) p[i] = 0.0f;
}
__global__ void k_set_count(uint32_t* counts, uint32_t idx, uint32_t v) {
    if (threadIdx.x == 0 && blockIdx.x == 0) counts[idx] = v;
}
// counts[dst] = counts[src]; counts[src2..] zeroed
__global__ void k_rotate_counts(uint32_t* counts) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        counts[0] = counts[1];
        counts[1] = 0u;
        counts[2] = 0u;
        counts[3] = 0u;
        counts[4] = 0u;
    }
}

// AoS [n][3] rays to the SoA buffers
__global__ void k_rays_from_aos(const float* __restrict__ O, const float* __restrict__ D, uint32_t n, RaySoA R,
                                const float* __restrict__ tmax, const uint32_t* __restrict__ excl, ShadowSoA SR) {
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        const float ox = O[3 * (size_t)i], oy = O[3 * (size_t)i + 1], oz = O[3 * (size_t)i + 2];
        const float dx = D[3 * (size_t)i], dy = D[3 * (size_t)i + 1], dz = D[3 * (size_t)i + 2];
        if (tmax) {
            SR.ox[i] = ox; SR.oy[i] = oy; SR.oz[i] = oz;
            SR.dx[i] = dx; SR.dy[i] = dy; SR.dz[i] = dz;
            SR.tmax[i] = tmax[i];
            SR.excl[i] = excl ? excl[i] : 0xffffffffu;
        } else {
            R.ox[i] = ox; R.oy[i] = oy; R.oz[i] = oz;
            R.dx[i] = dx; R.dy[i] = dy; R.dz[i] = dz;
        }
    }
}

// ------------------------------------------------------------------ camera paths
struct CamInfo {
    sc_camera cam;
    uint64_t seed;
    uint32_t s0;       // first sample of the chunk
    uint32_t hw;       // pixels
    uint32_t K;        // paths per (pixel, sample)
    uint32_t max_depth;
};

__device__ __forceinline__ void pid_decode(const CamInfo& ci, uint32_t pid, uint32_t& pix, uint32_t& sample,
                                           uint32_t& slot) {
    slot = pid % ci.K;
    const uint32_t rest = pid / ci.K;
    pix = rest % ci.hw;
    sample = ci.s0 + rest / ci.hw;
}

__global__ void k_raygen(CamInfo ci, WaveDev wl, PathState P, uint32_t n, uint32_t* queue, uint32_t* counts) {
    for (uint32_t pid = blockIdx.x * blockDim.x + threadIdx.x; pid < n; pid += gridDim.x * blockDim.x) {
        uint32_t pix, sample, slot;
        pid_decode(ci, pid, pix, sample, slot);
        const uint32_t x = pix % ci.cam.w, y = pix / ci.cam.w;
        const U4 r = rng_camera(ci.seed, pix, sample, 0, 0, slot);
        const float lam = wl.mode == SC_WL_FIXED ? wl.nm[slot] : lambda_from(wl, unit(r.c));
        F3 o, d;
        camera_ray(ci.cam, x, y, unit(r.a), unit(r.b), o, d);
        P.ox[pid] = o.x; P.oy[pid] = o.y; P.oz[pid] = o.z;
        P.dx[pid] = d.x; P.dy[pid] = d.y; P.dz[pid] = d.z;
        P.T[pid] = 1.0f;
        P.L[pid] = 0.0f;
        P.lambda[pid] = lam;
        P.flags[pid] = 0u;
        queue[pid] = pid;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) counts[0] = n;
}

// Sort hits by material: emitters and misses end here, dielectric and
// diffuse hits go to their own queues.
__global__ void k_classify(DevScene S, PathState P, const uint32_t* __restrict__ queue, uint32_t* counts,
                           uint32_t* q_diffuse, uint32_t* q_dielectric, uint32_t cap) {
    const uint32_t n = counts[0];
    const uint32_t stride = gridDim.x * blockDim.x;
    for (uint32_t base = blockIdx.x * blockDim.x; base < n; base += stride) {
        const uint32_t i = base + threadIdx.x;
        bool to_diff = false, to_diel = false;
        uint32_t pid = 0;
        if (i < n) {
            pid = queue[i];
            const uint32_t prim = P.prim[pid];
            if (prim != 0xffffffffu) {
                const sc_material m = S.mat[S.tri_obj[prim]];
                if (m.type == SC_MAT_EMISSIVE) {
                    if (!(P.flags[pid] & 1u)) {
                        F3 p0, p1, p2;
                        tri_vertices(S, prim, p0, p1, p2);
                        const F3 Ng = normalize(cross(p1 - p0, p2 - p0));
                        const F3 d{P.dx[pid], P.dy[pid], P.dz[pid]};
                        if (dot(d, Ng) < 0.0f) P.L[pid] = P.L[pid] + P.T[pid] * m.le;
                    }
                } else if (m.type == SC_MAT_DIELECTRIC) {
                    to_diel = true;
                } else {
                    to_diff = true;
                }
            }
        }
        wave_push(to_diel, pid, q_dielectric, counts + 3);
        wave_push(to_diff, pid, q_diffuse, counts + 2);
    }
}

__global__ void k_shade_dielectric(DevScene S, CamInfo ci, PathState P, uint32_t depth, const uint32_t* __restrict__ q,
                                   uint32_t* counts, uint32_t* q_next) {
    const uint32_t n = counts[3];
    const uint32_t stride = gridDim.x * blockDim.x;
    for (uint32_t base = blockIdx.x * blockDim.x; base < n; base += stride) {
        const uint32_t i = base + threadIdx.x;
        bool cont = false;
        uint32_t pid = 0;
        if (i < n) {
            pid = q[i];
            uint32_t pix, sample, slot;
            pid_decode(ci, pid, pix, sample, slot);
            const uint32_t prim = P.prim[pid];
            const F3 d{P.dx[pid], P.dy[pid], P.dz[pid]};
            const Frame f = hit_frame(S, prim, P.u[pid], P.v[pid], d);
            const sc_material m = S.mat[S.tri_obj[prim]];
            const U4 r = rng_camera(ci.seed, pix, sample, depth, 1, slot);
            F3 nd;
            bool refl;
            if (dielectric(f, d, P.lambda[pid], m.cauchy_a, m.cauchy_b, unit(r.c), nd, refl)) {
                const F3 o = offset_ray(f.P, refl ? f.Nf : neg(f.Nf));
                P.ox[pid] = o.x; P.oy[pid] = o.y; P.oz[pid] = o.z;
                P.dx[pid] = nd.x; P.dy[pid] = nd.y; P.dz[pid] = nd.z;
                cont = depth < ci.max_depth;
            }
        }
        wave_push(cont, pid, q_next, counts + 1);
    }
}

__global__ void k_shade_diffuse(DevScene S, CamInfo ci, WaveDev wl, PathState P, uint32_t depth,
                                const float* __restrict__ cmap, const uint32_t* __restrict__ q, uint32_t* counts,
                                uint32_t* q_next, uint32_t* q_shadow) {
    const uint32_t n = counts[2];
    const uint32_t stride = gridDim.x * blockDim.x;
    for (uint32_t base = blockIdx.x * blockDim.x; base < n; base += stride) {
        const uint32_t i = base + threadIdx.x;
        bool cont = false, shoot = false;
        uint32_t pid = 0;
        if (i < n) {
            pid = q[i];
            uint32_t pix, sample, slot;
            pid_decode(ci, pid, pix, sample, slot);
            const uint32_t prim = P.prim[pid];
            const uint32_t obj = S.tri_obj[prim];
            const F3 d{P.dx[pid], P.dy[pid], P.dz[pid]};
            const Frame f = hit_frame(S, prim, P.u[pid], P.v[pid], d);
            const sc_material m = S.mat[obj];
            const float rho = albedo(S, m, f.P);
            const float T = P.T[pid];
            const float lam = P.lambda[pid];
            float L = P.L[pid];
            P.flags[pid] = P.flags[pid] | 1u;
            const F3 os = offset_ray(f.P, f.Nf);
            // caustic gather
            if (cmap && S.recv_obj && obj == S.recv_obj) {
                const int64_t cell = receiver_cell(S, f.P);
                if (cell >= 0) {
                    const uint32_t b = wl.mode == SC_WL_FIXED ? slot : spectral_bin(wl, lam);
                    const float E = cmap[(size_t)cell * wl.channels + b] * S.inv_cell_area;
                    const float g = ((T * rho) * kInvPi) * E;
                    L = L + g;
                }
            }
            P.L[pid] = L;
            // next event estimation
            if (S.n_entries > 0) {
                const U4 r = rng_camera(ci.seed, pix, sample, depth, 2, slot);
                const uint32_t e = pick_entry(S.n_entries, unit(r.c));
                float contrib = 0.0f, tmax = 0.0f;
                uint32_t excl = 0xffffffffu;
                F3 om{0.0f, 0.0f, 0.0f};
                if (e < S.n_pl) {
                    const float* lp = S.pl + 4 * (size_t)e;
                    const F3 w = F3{lp[0], lp[1], lp[2]} - os;
                    const float r2 = dot(w, w);
                    const float dist = sqrtf(r2);
                    om = w * (1.0f / dist);
                    const float cosx = dot(f.Nf, om);
                    if (cosx > 0.0f) {
                        contrib = ((((T * rho) * kInvPi) * lp[3]) * cosx) / r2;
                        contrib = contrib * (float)S.n_entries;
                        tmax = dist;
                        shoot = true;
                    }
                } else {
                    const uint32_t k = cdf_first_above(S.emit_cdf, S.n_emit, unit(r.d));
                    const uint32_t lprim = S.emit_prim[k];
                    F3 Nl;
                    const F3 y = light_point(S, lprim, unit(r.a), unit(r.b), Nl);
                    const F3 w = y - os;
                    const float r2 = dot(w, w);
                    const float dist = sqrtf(r2);
                    om = w * (1.0f / dist);
                    const float cosx = dot(f.Nf, om);
                    const float cosl = -dot(Nl, om);
                    if (cosx > 0.0f && cosl > 0.0f) {
                        const float le = S.mat[S.tri_obj[lprim]].le;
                        contrib = ((((((T * rho) * kInvPi) * le) * cosx) * cosl) / r2) * S.a_tot;
                        contrib = contrib * (float)S.n_entries;
                        tmax = dist * 0.9999f;
                        excl = lprim;
                        shoot = true;
                    }
                }
                if (shoot) {
                    P.sox[pid] = os.x; P.soy[pid] = os.y; P.soz[pid] = os.z;
                    P.sdx[pid] = om.x; P.sdy[pid] = om.y; P.sdz[pid] = om.z;
                    P.stmax[pid] = tmax;
                    P.sexcl[pid] = excl;
                    P.scontrib[pid] = contrib;
                }
            }
            // cosine-weighted bounce
            if (depth < ci.max_depth) {
                const U4 r = rng_camera(ci.seed, pix, sample, depth, 1, slot);
                const float u0 = unit(r.a), u1 = unit(r.b);
                const float rr = sqrtf(u0);
                float sp, cp;
                sincos_turn(u1, sp, cp);
                const float x = rr * cp, y = rr * sp;
                const float z = sqrtf(fmaxf(0.0f, 1.0f - u0));
                F3 t1, t2;
                basis(f.Nf, t1, t2);
                const F3 nd = normalize((t1 * x + t2 * y) + f.Nf * z);
                P.ox[pid] = os.x; P.oy[pid] = os.y; P.oz[pid] = os.z;
                P.dx[pid] = nd.x; P.dy[pid] = nd.y; P.dz[pid] = nd.z;
                P.T[pid] = T * rho;
                cont = true;
            }
        }
        wave_push(shoot, pid, q_shadow, counts + 4);
        wave_push(cont, pid, q_next, counts + 1);
    }
}

// Film: per pixel, samples of the chunk added in sample order.
__global__ void k_film_accumulate(CamInfo ci, WaveDev wl, const float* __restrict__ L, const float* __restrict__ lambda,
                                  uint32_t n_samples, float* __restrict__ rgb) {
    for (uint32_t pix = blockIdx.x * blockDim.x + threadIdx.x; pix < ci.hw; pix += gridDim.x * blockDim.x) {
        float a0 = rgb[3 * (size_t)pix], a1 = rgb[3 * (size_t)pix + 1], a2 = rgb[3 * (size_t)pix + 2];
        for (uint32_t s = 0; s < n_samples; ++s) {
            const size_t base = ((size_t)s * ci.hw + pix) * ci.K;
            if (wl.mode == SC_WL_FIXED) {
                if (ci.K == 3) {
                    a0 = a0 + L[base];
                    a1 = a1 + L[base + 1];
                    a2 = a2 + L[base + 2];
                } else {
                    const float v = L[base];
                    a0 = a0 + v; a1 = a1 + v; a2 = a2 + v;
                }
            } else {
                const float v = L[base];
                const float lam = lambda[base];
                a0 = a0 + sensor(wl, 0, lam) * v;
                a1 = a1 + sensor(wl, 1, lam) * v;
                a2 = a2 + sensor(wl, 2, lam) * v;
            }
        }
        rgb[3 * (size_t)pix] = a0;
        rgb[3 * (size_t)pix + 1] = a1;
        rgb[3 * (size_t)pix + 2] = a2;
    }
}

__global__ void k_film_scale(float* rgb, uint32_t n, float inv_spp) {
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
        rgb[i] = rgb[i] * inv_spp;
}

// ------------------------------------------------------------------ ground truth
__global__ void k_aov_raygen(sc_camera cam, RaySoA R) {
    const uint32_t hw = cam.w * cam.h;
    for (uint32_t pix = blockIdx.x * blockDim.x + threadIdx.x; pix < hw; pix += gridDim.x * blockDim.x) {
        F3 o, d;
        camera_ray(cam, pix % cam.w, pix / cam.w, 0.5f, 0.5f, o, d);
        R.ox[pix] = o.x; R.oy[pix] = o.y; R.oz[pix] = o.z;
        R.dx[pix] = d.x; R.dy[pix] = d.y; R.dz[pix] = d.z;
    }
}

__global__ void k_aov_write(DevScene S, sc_camera cam, RaySoA R, HitSoA H, sc_aov out) {
    const uint32_t hw = cam.w * cam.h;
    const F3 Rh = normalize(F3{cam.right[0], cam.right[1], cam.right[2]});
    const F3 Uh = normalize(F3{cam.up[0], cam.up[1], cam.up[2]});
    const F3 Fh = normalize(F3{cam.fwd[0], cam.fwd[1], cam.fwd[2]});
    for (uint32_t pix = blockIdx.x * blockDim.x + threadIdx.x; pix < hw; pix += gridDim.x * blockDim.x) {
        const uint32_t prim = H.prim[pix];
        uint32_t obj = 0;
        float dep = INFINITY, depn = 1.0f, alb = 0.0f;
        F3 N{0.0f, 0.0f, 0.0f}, Nc{0.0f, 0.0f, 0.0f};
        uint8_t trans = 0;
        if (prim != 0xffffffffu) {
            obj = S.tri_obj[prim];
            const sc_material m = S.mat[obj];
            const F3 d{R.dx[pix], R.dy[pix], R.dz[pix]};
            const float t = H.t[pix];
            const Frame f = hit_frame(S, prim, H.u[pix], H.v[pix], d);
            dep = t;
            depn = fminf(t / 10.0f, 1.0f);
            N = f.Ns;
            Nc = F3{dot(N, Rh), dot(N, Uh), -dot(N, Fh)};
            alb = m.type == SC_MAT_DIFFUSE ? albedo(S, m, f.P) : (m.type == SC_MAT_DIELECTRIC ? 1.0f : 0.0f);
            trans = m.type == SC_MAT_DIELECTRIC ? 1 : 0;
        }
        if (out.obj) out.obj[pix] = obj;
        if (out.trans) out.trans[pix] = trans;
        if (out.tri) out.tri[pix] = prim;
        if (out.depth) out.depth[pix] = dep;
        if (out.depthn) out.depthn[pix] = depn;
        if (out.normal) store3(out.normal, pix, N);
        if (out.normal_cam) store3(out.normal_cam, pix, Nc);
        if (out.albedo) out.albedo[pix] = alb;
    }
}

// ------------------------------------------------------------------ photons
struct PhInfo {
    uint64_t seed;
    uint64_t n_total;   // photons in the pass
    uint64_t p0;        // first photon of the chunk
    uint32_t max_depth;
    double scale;       // fixed-point scale of the caustic accumulator
    int stats;
};

__device__ __forceinline__ void ph_stat(DevCounters* C, const PhInfo& pi, int outcome, float phi) {
    if (!pi.stats) return;
    atomicAdd(&C->ph_count[outcome], 1ull);
    atomicAdd(&C->ph_flux[outcome], (double)phi);
}

// 1 - cos(theta) of the cone subtended by a sphere of squared radius rr at
// squared distance dist2, without cancellation
__device__ __forceinline__ float cap_height(float rr, float dist2) {
    const float q = rr / dist2;
    return q >= 1.0f ? 2.0f : q / (1.0f + sqrtf(1.0f - q));
}

__global__ void k_photon_emit(DevScene S, WaveDev wl, PhInfo pi, uint32_t n, PhotonState Ph, uint32_t* queue,
                              uint32_t* counts, DevCounters* C) {
    const uint32_t stride = gridDim.x * blockDim.x;
    for (uint32_t base = blockIdx.x * blockDim.x; base < n; base += stride) {
        const uint32_t i = base + threadIdx.x;
        bool alive = false;
        if (i < n) {
            const uint64_t p = pi.p0 + i;
            const U4 r0 = rng_photon(pi.seed, p, 0, 0);
            uint32_t slot;
            float lam, nslot;
            if (wl.mode == SC_WL_FIXED) {
                slot = (uint32_t)(p % wl.k);
                lam = wl.nm[slot];
                const uint64_t cnt = pi.n_total / wl.k + ((p % wl.k) < (pi.n_total % wl.k) ? 1u : 0u);
                nslot = (float)cnt;
            } else {
                lam = lambda_from(wl, unit(r0.d));
                slot = spectral_bin(wl, lam);
                nslot = (float)pi.n_total / (float)wl.bins;
            }
            const U4 r2 = rng_photon(pi.seed, p, 0, 2);
            const uint32_t e = pick_entry(S.n_entries, unit(r2.c));
            F3 y, Nl{0.0f, 0.0f, 0.0f};
            float power;
            bool area = false;
            if (e < S.n_pl) {
                const float* lp = S.pl + 4 * (size_t)e;
                y = F3{lp[0], lp[1], lp[2]};
                power = lp[3];
            } else {
                const uint32_t k = cdf_first_above(S.emit_cdf, S.n_emit, unit(r2.d));
                const uint32_t lprim = S.emit_prim[k];
                y = light_point(S, lprim, unit(r2.a), unit(r2.b), Nl);
                power = S.mat[S.tri_obj[lprim]].le * S.a_tot;
                area = true;
            }
            // cone per target, picked in proportion to its solid angle
            float osum = 0.0f;
            for (uint32_t k = 0; k < S.n_tg; ++k) {
                const float* sp = S.tg + 4 * (size_t)k;
                const F3 dk = F3{sp[0], sp[1], sp[2]} - y;
                osum = osum + kTwoPi * cap_height(sp[3] * sp[3], dot(dk, dk));
            }
            const float target = unit(r0.a) * osum;
            uint32_t kk = S.n_tg - 1;
            float cum = 0.0f;
            for (uint32_t k = 0; k < S.n_tg; ++k) {
                const float* sp = S.tg + 4 * (size_t)k;
                const F3 dk = F3{sp[0], sp[1], sp[2]} - y;
                cum = cum + kTwoPi * cap_height(sp[3] * sp[3], dot(dk, dk));
                if (cum > target) {
                    kk = k;
                    break;
                }
            }
            const float* spk = S.tg + 4 * (size_t)kk;
            const F3 dkk = F3{spk[0], spk[1], spk[2]} - y;
            const float d2k = dot(dkk, dkk);
            const float hk = cap_height(spk[3] * spk[3], d2k);
            const F3 axis = dkk * (1.0f / sqrtf(d2k));
            const float g = unit(r0.b) * hk;
            const float cost = 1.0f - g;
            const float sint = sqrtf(fmaxf(0.0f, g * (2.0f - g)));
            float sp_, cp_;
            sincos_turn(unit(r0.c), sp_, cp_);
            F3 t1, t2;
            basis(axis, t1, t2);
            const F3 om = normalize((t1 * (cp_ * sint) + t2 * (sp_ * sint)) + axis * cost);
            uint32_t m = 1;
            for (uint32_t k = 0; k < S.n_tg; ++k) {
                if (k == kk) continue;
                const float* sp = S.tg + 4 * (size_t)k;
                const F3 dk = F3{sp[0], sp[1], sp[2]} - y;
                const float dist2 = dot(dk, dk);
                const float q = (sp[3] * sp[3]) / dist2;
                const F3 ax = dk * (1.0f / sqrtf(dist2));
                const F3 cr = cross(om, ax);
                if (q >= 1.0f || (dot(om, ax) > 0.0f && dot(cr, cr) <= q)) ++m;
            }
            float phi;
            F3 o;
            bool dead = false;
            if (area) {
                const float cy = dot(Nl, om);
                if (!(cy > 0.0f)) dead = true;
                phi = (((power * cy) * osum) * (float)S.n_entries) / (nslot * (float)m);
                o = offset_ray(y, Nl);
            } else {
                phi = ((power * osum) * (float)S.n_entries) / (nslot * (float)m);
                o = y;
            }
            if (dead) {
                if (pi.stats) atomicAdd(&C->ph_count[SC_PH_EMIT_DEAD], 1ull);
            } else {
                Ph.ox[i] = o.x; Ph.oy[i] = o.y; Ph.oz[i] = o.z;
                Ph.dx[i] = om.x; Ph.dy[i] = om.y; Ph.dz[i] = om.z;
                Ph.phi[i] = phi;
                Ph.lambda[i] = lam;
                Ph.slot[i] = slot;
                Ph.spec[i] = 0u;
                alive = true;
            }
        }
        wave_push(alive, i, queue, counts + 0);
    }
}

// Deposit fixed-point flux; lanes of a wave that hit the same cell as the
// first depositing lane combine into one atomic.
__device__ __forceinline__ void deposit(bool want, uint32_t cell, unsigned long long q, unsigned long long* acc,
                                        uint32_t* cnt_map) {
    const unsigned long long m = __ballot(want);
    if (m == 0ull) return;
    const uint32_t leader = __ffsll((long long)m) - 1;
    const uint32_t lcell = __shfl(cell, (int)leader);
    const bool same = want && cell == lcell;
    const unsigned long long ms = __ballot(same);
    const unsigned long long part = wave_sum_u64(same ? q : 0ull);
    if (lane_id() == leader) {
        atomicAdd(&acc[lcell], part);
        if (cnt_map) atomicAdd(&cnt_map[lcell], (uint32_t)__popcll(ms));
    }
    if (want && !same) {
        atomicAdd(&acc[cell], q);
        if (cnt_map) atomicAdd(&cnt_map[cell], 1u);
    }
}

__global__ void k_photon_event(DevScene S, WaveDev wl, PhInfo pi, uint32_t depth, PhotonState Ph,
                               const uint32_t* __restrict__ queue, uint32_t* counts, uint32_t* q_next,
                               unsigned long long* acc, uint32_t* cnt_map, DevCounters* C) {
    const uint32_t n = counts[0];
    const uint32_t stride = gridDim.x * blockDim.x;
    for (uint32_t base = blockIdx.x * blockDim.x; base < n; base += stride) {
        const uint32_t i = base + threadIdx.x;
        bool cont = false, dep = false;
        uint32_t id = 0, cell_ch = 0;
        unsigned long long q = 0;
        if (i < n) {
            id = queue[i];
            const uint32_t prim = Ph.prim[id];
            const float phi = Ph.phi[id];
            if (prim == 0xffffffffu) {
                ph_stat(C, pi, SC_PH_ESCAPED, phi);
            } else {
                const uint32_t obj = S.tri_obj[prim];
                const sc_material m = S.mat[obj];
                const F3 d{Ph.dx[id], Ph.dy[id], Ph.dz[id]};
                const Frame f = hit_frame(S, prim, Ph.u[id], Ph.v[id], d);
                if (m.type == SC_MAT_EMISSIVE) {
                    ph_stat(C, pi, SC_PH_ABSORBED, phi);
                } else if (m.type == SC_MAT_DIELECTRIC) {
                    const U4 r = rng_photon(pi.seed, pi.p0 + id, depth, 1);
                    F3 nd;
                    bool refl;
                    if (!dielectric(f, d, Ph.lambda[id], m.cauchy_a, m.cauchy_b, unit(r.c), nd, refl)) {
                        ph_stat(C, pi, SC_PH_LOST, phi);
                    } else {
                        const F3 o = offset_ray(f.P, refl ? f.Nf : neg(f.Nf));
                        Ph.ox[id] = o.x; Ph.oy[id] = o.y; Ph.oz[id] = o.z;
                        Ph.dx[id] = nd.x; Ph.dy[id] = nd.y; Ph.dz[id] = nd.z;
                        Ph.spec[id] = Ph.spec[id] + 1u;
                        if (depth < pi.max_depth) cont = true;
                        else ph_stat(C, pi, SC_PH_TRUNCATED, phi);
                    }
                } else if (Ph.spec[id] == 0u) {
                    ph_stat(C, pi, SC_PH_DIRECT, phi);
                } else if (obj != S.recv_obj) {
                    ph_stat(C, pi, SC_PH_ELSEWHERE, phi);
                } else {
                    const int64_t cell = receiver_cell(S, f.P);
                    if (cell < 0) {
                        ph_stat(C, pi, SC_PH_OUTSIDE, phi);
                    } else {
                        dep = true;
                        cell_ch = (uint32_t)cell * wl.channels + Ph.slot[id];
                        q = __double2ull_rn((double)phi * pi.scale);
                        ph_stat(C, pi, SC_PH_DEPOSITED, phi);
                    }
                }
            }
        }
        deposit(dep, cell_ch, q, acc, cnt_map);
        wave_push(cont, id, q_next, counts + 1);
    }
}

__global__ void k_map_finalize(const unsigned long long* __restrict__ acc, size_t n, double inv_scale,
                               float* __restrict__ map) {
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        map[i] = (float)((double)acc[i] * inv_scale);
}

inline uint32_t grid_for(size_t n, uint32_t bs, uint32_t cap = 8192) {
    size_t g = (n + bs - 1) / bs;
    if (g < 1) g = 1;
    return (uint32_t)(g > cap ? cap : g);
}

}  // namespace

// =====================================================================
// host orchestration
// =====================================================================
namespace scl {

namespace {

constexpr uint32_t kWorkSlots = 4096;

// carve n-element arrays out of one allocation, 256-byte aligned
struct Carver {
    char* base;
    size_t off = 0;
    template <class T>
    T* take(size_t n) {
        off = (off + 255) & ~(size_t)255;
        T* p = reinterpret_cast<T*>(base + off);
        off += sizeof(T) * n;
        return p;
    }
};

size_t path_bytes(size_t n) { return 25 * (n * 4 + 256); }
size_t photon_bytes(size_t n) { return 16 * (n * 4 + 256); }

PathState carve_path(void* p, size_t n) {
    Carver c{static_cast<char*>(p)};
    PathState P;
    P.ox = c.take<float>(n); P.oy = c.take<float>(n); P.oz = c.take<float>(n);
    P.dx = c.take<float>(n); P.dy = c.take<float>(n); P.dz = c.take<float>(n);
    P.T = c.take<float>(n); P.L = c.take<float>(n); P.lambda = c.take<float>(n);
    P.flags = c.take<uint32_t>(n);
    P.t = c.take<float>(n); P.u = c.take<float>(n); P.v = c.take<float>(n); P.prim = c.take<uint32_t>(n);
    P.sox = c.take<float>(n); P.soy = c.take<float>(n); P.soz = c.take<float>(n);
    P.sdx = c.take<float>(n); P.sdy = c.take<float>(n); P.sdz = c.take<float>(n);
    P.stmax = c.take<float>(n); P.scontrib = c.take<float>(n); P.sexcl = c.take<uint32_t>(n);
    return P;
}

PhotonState carve_photon(void* p, size_t n) {
    Carver c{static_cast<char*>(p)};
    PhotonState P;
    P.ox = c.take<float>(n); P.oy = c.take<float>(n); P.oz = c.take<float>(n);
    P.dx = c.take<float>(n); P.dy = c.take<float>(n); P.dz = c.take<float>(n);
    P.phi = c.take<float>(n); P.lambda = c.take<float>(n);
    P.slot = c.take<uint32_t>(n); P.spec = c.take<uint32_t>(n);
    P.t = c.take<float>(n); P.u = c.take<float>(n); P.v = c.take<float>(n); P.prim = c.take<uint32_t>(n);
    return P;
}

Queues carve_queues(void* p, size_t n) {
    Carver c{static_cast<char*>(p)};
    Queues q;
    q.cur = c.take<uint32_t>(n); q.next = c.take<uint32_t>(n); q.diffuse = c.take<uint32_t>(n);
    q.dielectric = c.take<uint32_t>(n); q.shadow = c.take<uint32_t>(n); q.counts = c.take<uint32_t>(8);
    return q;
}

sc_status ensure_queues(Ctx* c, size_t n) {
    if (c->queue_n >= n && c->queues.p) return SC_OK;
    SC_TRY(c->queues.alloc(5 * (n * 4 + 256) + 512));
    c->queue_n = n;
    return SC_OK;
}

sc_status ensure_path(Ctx* c, size_t n) {
    if (c->path_n >= n && c->path.p) return SC_OK;
    SC_TRY(c->path.alloc(path_bytes(n)));
    c->path_n = n;
    return SC_OK;
}

uint32_t* next_work_slot(Ctx* c) {
    if (c->work_slot >= kWorkSlots) {
        hipLaunchKernelGGL(k_zero_u32, dim3(16), dim3(256), 0, c->stream, c->work.as<uint32_t>(), kWorkSlots);
        c->work_slot = 0;
    }
    return c->work.as<uint32_t>() + (c->work_slot++);
}

void reset_work(Ctx* c) {
    hipLaunchKernelGGL(k_zero_u32, dim3(16), dim3(256), 0, c->stream, c->work.as<uint32_t>(), kWorkSlots);
    c->work_slot = 0;
}

uint32_t trace_grid(size_t n_max) {
    // enough waves to fill 256 CUs several times over, no more than the work
    const size_t want = (n_max + kTraceBS - 1) / kTraceBS;
    const size_t cap = 256 * 16;
    return (uint32_t)(want < 1 ? 1 : (want > cap ? cap : want));
}

void launch_closest(Ctx* c, const DevScene& S, RaySoA R, HitSoA H, const uint32_t* queue, const uint32_t* count,
                    uint32_t n_static, size_t n_max) {
    uint32_t* work = next_work_slot(c);
    DevCounters* C = c->counters.as<DevCounters>();
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (c->profile) {
        (void)hipEventCreate(&e0);
        (void)hipEventCreate(&e1);
        (void)hipEventRecord(e0, c->stream);
    }
    if (c->count_visits)
        hipLaunchKernelGGL(k_closest<true>, dim3(trace_grid(n_max)), dim3(kTraceBS), 0, c->stream, S, R, H, queue, count,
                           n_static, work, C);
    else
        hipLaunchKernelGGL(k_closest<false>, dim3(trace_grid(n_max)), dim3(kTraceBS), 0, c->stream, S, R, H, queue,
                           count, n_static, work, C);
    if (c->profile) {
        (void)hipEventRecord(e1, c->stream);
        c->events.emplace_back(e0, e1);
    }
}

void launch_anyhit(Ctx* c, const DevScene& S, ShadowSoA R, const uint32_t* queue, const uint32_t* count,
                   uint32_t n_static, size_t n_max, uint8_t* occ, float* L) {
    uint32_t* work = next_work_slot(c);
    hipLaunchKernelGGL(k_anyhit, dim3(trace_grid(n_max)), dim3(kTraceBS), 0, c->stream, S, R, queue, count, n_static,
                       work, occ, L, c->counters.as<DevCounters>());
}

// Sensor curves (Gaussians, 40 nm, at 650/550/450 nm, mean 1 over the
// range) tabulated every 0.25 nm in double, uploaded as float.
sc_status make_wave(Ctx* c, const sc_wavelengths& wl, WaveDev& w) {
    w.mode = wl.mode;
    w.k = wl.k;
    for (int i = 0; i < 4; ++i) w.nm[i] = wl.nm[i];
    w.lo = wl.lo;
    w.hi = wl.hi;
    w.bins = wl.bins;
    w.tab = nullptr;
    w.n_tab = 0;
    w.bin_scale = 0.0f;
    w.channels = wl.mode == SC_WL_FIXED ? wl.k : wl.bins;
    if (wl.mode == SC_WL_UNIFORM) {
        w.bin_scale = (float)wl.bins / (wl.hi - wl.lo);
        const uint32_t n = (uint32_t)((double)(wl.hi - wl.lo) * 4.0 + 0.5) + 1;
        std::vector<float> tab(3 * (size_t)n);
        const double mu[3] = {650.0, 550.0, 450.0};
        std::vector<double> g(n);
        for (int ch = 0; ch < 3; ++ch) {
            for (uint32_t i = 0; i < n; ++i) {
                const double lam = (double)wl.lo + 0.25 * (double)i;
                const double x = (lam - mu[ch]) / 40.0;
                g[i] = exp(-0.5 * x * x);
            }
            double sum = 0.0;
            for (uint32_t i = 0; i + 1 < n; ++i) sum += 0.5 * (g[i] + g[i + 1]) * 0.25;
            const double mean = sum / ((double)(n - 1) * 0.25);
            for (uint32_t i = 0; i < n; ++i) tab[(size_t)ch * n + i] = (float)(g[i] / mean);
        }
        SC_TRY(c->sensor.ensure(tab.size() * sizeof(float)));
        SC_HIP(hipMemcpyAsync(c->sensor.p, tab.data(), tab.size() * sizeof(float), hipMemcpyHostToDevice, c->stream));
        SC_HIP(hipStreamSynchronize(c->stream));   // tab is a host temporary
        w.tab = c->sensor.as<float>();
        w.n_tab = n;
    }
    return SC_OK;
}

}  // namespace

sc_status ctx_init(Ctx* c) {
    SC_TRY(c->counters.alloc(sizeof(DevCounters)));
    SC_TRY(c->work.alloc(sizeof(uint32_t) * kWorkSlots));
    SC_HIP(hipMemsetAsync(c->counters.p, 0, sizeof(DevCounters), c->stream));
    SC_HIP(hipMemsetAsync(c->work.p, 0, sizeof(uint32_t) * kWorkSlots, c->stream));
    SC_HIP(hipStreamSynchronize(c->stream));
    return SC_OK;
}

void ctx_release(Ctx* c) {
    for (auto& e : c->events) {
        (void)hipEventDestroy(e.first);
        (void)hipEventDestroy(e.second);
    }
    c->events.clear();
}

sc_status ctx_counters(Ctx* c, sc_counters* out) {
    SC_HIP(hipStreamSynchronize(c->stream));
    DevCounters h;
    SC_HIP(hipMemcpy(&h, c->counters.p, sizeof(h), hipMemcpyDeviceToHost));
    for (auto& e : c->events) {
        float ms = 0.0f;
        SC_HIP(hipEventElapsedTime(&ms, e.first, e.second));
        c->closest_ms += ms;
        c->closest_launches += 1;
        (void)hipEventDestroy(e.first);
        (void)hipEventDestroy(e.second);
    }
    c->events.clear();
    out->rays_closest = h.rays_closest;
    out->rays_shadow = h.rays_shadow;
    out->node_visits = h.node_visits;
    out->tri_tests = h.tri_tests;
    out->closest_launches = c->closest_launches;
    out->closest_ms = c->closest_ms;
    out->closest_rays_timed = 0;
    return SC_OK;
}

sc_status ctx_reset_counters(Ctx* c) {
    SC_HIP(hipStreamSynchronize(c->stream));
    SC_HIP(hipMemset(c->counters.p, 0, sizeof(DevCounters)));
    ctx_release(c);
    c->closest_ms = 0.0;
    c->closest_launches = 0;
    return SC_OK;
}

sc_status render(Ctx* c, Bvh* b, const sc_camera& cam, uint32_t spp, uint32_t max_depth, const sc_wavelengths& wl,
                 uint64_t seed, const float* cmap, const sc_aov& out) {
    hipStream_t st = c->stream;
    const DevScene& S = b->scene;
    const size_t hw = (size_t)cam.w * cam.h;
    const uint32_t K = wl.mode == SC_WL_FIXED ? wl.k : 1;
    WaveDev wd;
    SC_TRY(make_wave(c, wl, wd));
    const size_t per_sample = hw * K;
    size_t chunk = c->queue_cap / per_sample;
    if (chunk < 1) chunk = 1;
    if (chunk > spp) chunk = spp;
    const size_t n_max = std::max(chunk * per_sample, hw);
    if (n_max > 0xffffffffull) return set_error(SC_EUNSUPPORTED, "image too large for one wavefront chunk");
    SC_TRY(ensure_path(c, n_max));
    SC_TRY(ensure_queues(c, n_max));
    PathState P = carve_path(c->path.p, n_max);
    Queues q = carve_queues(c->queues.p, n_max);
    reset_work(c);

    const bool want_aov = out.obj || out.trans || out.tri || out.depth || out.depthn || out.normal || out.normal_cam ||
                          out.albedo;
    const RaySoA R{P.ox, P.oy, P.oz, P.dx, P.dy, P.dz};
    const HitSoA H{P.t, P.prim, P.u, P.v};
    const uint32_t bs = 256;
    if (want_aov) {
        hipLaunchKernelGGL(k_aov_raygen, dim3(grid_for(hw, bs)), dim3(bs), 0, st, cam, R);
        launch_closest(c, S, R, H, nullptr, nullptr, (uint32_t)hw, hw);
        hipLaunchKernelGGL(k_aov_write, dim3(grid_for(hw, bs)), dim3(bs), 0, st, S, cam, R, H, out);
    }
    if (out.rgb) {
        hipLaunchKernelGGL(k_zero_f32, dim3(grid_for(3 * hw, bs)), dim3(bs), 0, st, out.rgb, 3 * hw);
        const ShadowSoA SR{P.sox, P.soy, P.soz, P.sdx, P.sdy, P.sdz, P.stmax, P.sexcl, P.scontrib};
        for (uint32_t s0 = 0; s0 < spp; s0 += (uint32_t)chunk) {
            const uint32_t ns = (uint32_t)std::min<size_t>(chunk, spp - s0);
            const uint32_t n = (uint32_t)(ns * per_sample);
            CamInfo ci{cam, seed, s0, (uint32_t)hw, K, max_depth};
            hipLaunchKernelGGL(k_zero_u32, dim3(1), dim3(64), 0, st, q.counts, 8u);
            hipLaunchKernelGGL(k_raygen, dim3(grid_for(n, bs)), dim3(bs), 0, st, ci, wd, P, n, q.cur, q.counts);
            uint32_t* cur = q.cur;
            uint32_t* nxt = q.next;
            for (uint32_t depth = 1; depth <= max_depth; ++depth) {
                launch_closest(c, S, R, H, cur, q.counts + 0, 0u, n);
                hipLaunchKernelGGL(k_classify, dim3(grid_for(n, bs)), dim3(bs), 0, st, S, P, cur, q.counts, q.diffuse,
                                   q.dielectric, n);
                hipLaunchKernelGGL(k_shade_dielectric, dim3(grid_for(n, bs)), dim3(bs), 0, st, S, ci, P, depth,
                                   q.dielectric, q.counts, nxt);
                hipLaunchKernelGGL(k_shade_diffuse, dim3(grid_for(n, bs)), dim3(bs), 0, st, S, ci, wd, P, depth, cmap,
                                   q.diffuse, q.counts, nxt, q.shadow);
                launch_anyhit(c, S, SR, q.shadow, q.counts + 4, 0u, n, nullptr, P.L);
                hipLaunchKernelGGL(k_rotate_counts, dim3(1), dim3(64), 0, st, q.counts);
                std::swap(cur, nxt);
            }
            hipLaunchKernelGGL(k_film_accumulate, dim3(grid_for(hw, bs)), dim3(bs), 0, st, ci, wd, P.L, P.lambda, ns,
                               out.rgb);
        }
        hipLaunchKernelGGL(k_film_scale, dim3(grid_for(3 * hw, bs)), dim3(bs), 0, st, out.rgb, (uint32_t)(3 * hw),
                           1.0f / (float)spp);
    }
    SC_HIP(hipGetLastError());
    return SC_OK;
}

sc_status trace_photons(Ctx* c, Bvh* b, uint64_t N, uint32_t max_depth, const sc_wavelengths& wl, uint64_t seed,
                        float* map, uint32_t* count_map, sc_photon_stats* stats) {
    hipStream_t st = c->stream;
    const DevScene& S = b->scene;
    WaveDev wd;
    SC_TRY(make_wave(c, wl, wd));
    const size_t cells = (size_t)S.recv_wc * S.recv_hc * wd.channels;
    SC_TRY(c->acc64.ensure(cells * sizeof(unsigned long long)));
    const uint32_t bs = 256;
    hipLaunchKernelGGL(k_zero_u64, dim3(grid_for(cells, bs)), dim3(bs), 0, st, c->acc64.as<unsigned long long>(), cells);
    if (count_map)
        hipLaunchKernelGGL(k_zero_u32, dim3(grid_for(cells, bs)), dim3(bs), 0, st, count_map, (uint32_t)cells);
    DevCounters before{};
    if (stats) {
        SC_HIP(hipStreamSynchronize(st));
        SC_HIP(hipMemcpy(&before, c->counters.p, sizeof(before), hipMemcpyDeviceToHost));
        // clear photon outcome counters
        DevCounters z = before;
        for (int i = 0; i < 9; ++i) { z.ph_count[i] = 0; z.ph_flux[i] = 0.0; }
        SC_HIP(hipMemcpy(c->counters.p, &z, sizeof(z), hipMemcpyHostToDevice));
    }
    double scale = 1.0;
    if (N > 0 && S.n_tg > 0 && S.n_entries > 0) {
        // bound on one photon's flux: strongest light, all entries, every
        // cone a full sphere, smallest slot
        double nslot_min = wl.mode == SC_WL_FIXED ? (double)(N / wl.k) : (double)N / (double)wl.bins;
        if (nslot_min < 1.0) nslot_min = 1.0;
        const double bound = (double)b->max_power * (double)S.n_entries * 4.0 * M_PI * (double)S.n_tg / nslot_min;
        const double room = ldexp(1.0, 62) / ((double)N * bound);
        const int e = (int)floor(log2(room));
        scale = ldexp(1.0, e);
        const size_t chunk = std::min<uint64_t>(N, c->photon_cap);
        if (c->photon_n < chunk || !c->photon.p) {
            SC_TRY(c->photon.alloc(photon_bytes(chunk)));
            c->photon_n = chunk;
        }
        SC_TRY(ensure_queues(c, chunk));
        PhotonState Ph = carve_photon(c->photon.p, chunk);
        Queues q = carve_queues(c->queues.p, chunk);
        reset_work(c);
        const RaySoA R{Ph.ox, Ph.oy, Ph.oz, Ph.dx, Ph.dy, Ph.dz};
        const HitSoA H{Ph.t, Ph.prim, Ph.u, Ph.v};
        for (uint64_t p0 = 0; p0 < N; p0 += chunk) {
            const uint32_t n = (uint32_t)std::min<uint64_t>(chunk, N - p0);
            PhInfo pi{seed, N, p0, max_depth, scale, stats ? 1 : 0};
            hipLaunchKernelGGL(k_zero_u32, dim3(1), dim3(64), 0, st, q.counts, 8u);
            hipLaunchKernelGGL(k_photon_emit, dim3(grid_for(n, bs)), dim3(bs), 0, st, S, wd, pi, n, Ph, q.cur, q.counts,
                               c->counters.as<DevCounters>());
            uint32_t* cur = q.cur;
            uint32_t* nxt = q.next;
            for (uint32_t depth = 1; depth <= max_depth; ++depth) {
                launch_closest(c, S, R, H, cur, q.counts + 0, 0u, n);
                hipLaunchKernelGGL(k_photon_event, dim3(grid_for(n, bs)), dim3(bs), 0, st, S, wd, pi, depth, Ph, cur,
                                   q.counts, nxt, c->acc64.as<unsigned long long>(), count_map,
                                   c->counters.as<DevCounters>());
                hipLaunchKernelGGL(k_rotate_counts, dim3(1), dim3(64), 0, st, q.counts);
                std::swap(cur, nxt);
            }
        }
    }
    hipLaunchKernelGGL(k_map_finalize, dim3(grid_for(cells, bs)), dim3(bs), 0, st, c->acc64.as<unsigned long long>(),
                       cells, 1.0 / scale, map);
    SC_HIP(hipGetLastError());
    if (stats) {
        DevCounters after;
        SC_HIP(hipStreamSynchronize(st));
        SC_HIP(hipMemcpy(&after, c->counters.p, sizeof(after), hipMemcpyDeviceToHost));
        for (int i = 0; i < 9; ++i) {
            stats->count[i] = after.ph_count[i];
            stats->flux[i] = after.ph_flux[i];
        }
        stats->segments = after.rays_closest - before.rays_closest;
    }
    return SC_OK;
}

sc_status trace_rays(Ctx* c, Bvh* b, uint32_t n, const float* O, const float* D, float* t, uint32_t* prim, float* u,
                     float* v) {
    if (c->aos_n < n || !c->aos.p) {
        SC_TRY(c->aos.alloc(9 * ((size_t)n * 4 + 256)));
        c->aos_n = n;
    }
    Carver cv{static_cast<char*>(c->aos.p)};
    float* ox = cv.take<float>(n); float* oy = cv.take<float>(n); float* oz = cv.take<float>(n);
    float* dx = cv.take<float>(n); float* dy = cv.take<float>(n); float* dz = cv.take<float>(n);
    const RaySoA R{ox, oy, oz, dx, dy, dz};
    const ShadowSoA none{};
    hipLaunchKernelGGL(k_rays_from_aos, dim3(grid_for(n, 256)), dim3(256), 0, c->stream, O, D, n,
                       RaySoA{ox, oy, oz, dx, dy, dz}, nullptr, nullptr, none);
    reset_work(c);
    launch_closest(c, b->scene, R, HitSoA{t, prim, u, v}, nullptr, nullptr, n, n);
    SC_HIP(hipGetLastError());
    return SC_OK;
}

sc_status occluded(Ctx* c, Bvh* b, uint32_t n, const float* O, const float* D, const float* tmax, const uint32_t* excl,
                   uint8_t* occ) {
    if (c->aos_n < n || !c->aos.p) {
        SC_TRY(c->aos.alloc(9 * ((size_t)n * 4 + 256)));
        c->aos_n = n;
    }
    Carver cv{static_cast<char*>(c->aos.p)};
    ShadowSoA SR;
    SR.ox = cv.take<float>(n); SR.oy = cv.take<float>(n); SR.oz = cv.take<float>(n);
    SR.dx = cv.take<float>(n); SR.dy = cv.take<float>(n); SR.dz = cv.take<float>(n);
    SR.tmax = cv.take<float>(n); SR.excl = cv.take<uint32_t>(n); SR.contrib = cv.take<float>(n);
    hipLaunchKernelGGL(k_rays_from_aos, dim3(grid_for(n, 256)), dim3(256), 0, c->stream, O, D, n, RaySoA{}, tmax,
                       excl, SR);
    reset_work(c);
    launch_anyhit(c, b->scene, SR, nullptr, nullptr, n, n, occ, nullptr);
    SC_HIP(hipGetLastError());
    return SC_OK;
}

}  // namespace scl
