// trace.hip -- wavefront path tracing, photon tracing and ground-truth
// kernels for gfx950.
//
// Rays live in structure-of-arrays buffers indexed by a stable path id;
// queues of path ids connect the stages:
//   raygen -> [closest hit -> classify (sort by material, compact) ->
//              shade dielectric | shade diffuse (+ shadow ray) ->
//              any hit (shadow) ] x depth -> film
// Queue appends use one atomic per block and 8 items per thread (ballot +
// mbcnt prefix within a wave, offsets of the waves in LDS).
// Traversal kernels keep every lane busy: a wave takes batches of rays and
// refills the lanes whose ray is finished while the others go on; the
// traversal stack lives in LDS (spilling to scratch only for deep trees) and
// the children of a wide node are visited front to back.
#pragma clang fp contract(off)
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <mutex>
#include <string>

#include "sc_device.h"
#include "sc_internal.h"
#include "sc_kernels.h"
#include "sc_path.h"

using namespace scd;

namespace {

constexpr int kTraceBS = 128;
static_assert(kStackMax == kMaxStack, "stack bound shared with the host check");

__device__ __forceinline__ uint32_t lane_id() { return __lane_id(); }

__device__ __forceinline__ uint32_t lanes_below(unsigned long long m) {
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

// Queue appends of the streaming stages.  A block takes up to kPushItems
// items per thread between two appends (item k of thread t is item
// k * blockDim.x + t of the block's range); bit k of `keep` marks the items
// to append, val(k) gives the value, and the kept items go to the queue in
// item order with one atomic per block and queue.  Appends to one queue all
// hit one counter, and same-address atomics serialise in L2: at one atomic
// per 256 items they, not the bytes moved, bounded these stages.  Every
// thread of the block must call this (block size a multiple of 64, at most
// 1024).
constexpr uint32_t kPushItems = 8;

// Items per thread between two appends for a launch of n items: one sweep
// of the grid when it can (small launches keep one item per thread and
// every block busy), at most kPushItems.
__device__ __forceinline__ uint32_t push_items(uint32_t n) {
    const uint32_t threads = gridDim.x * blockDim.x;
    const uint32_t per = (n + threads - 1) / threads;
    return per < 1u ? 1u : (per > kPushItems ? kPushItems : per);
}

template <typename ValFn>
__device__ __forceinline__ void block_push(uint32_t keep, ValFn val, uint32_t* q, uint32_t* cnt) {
    __shared__ uint32_t s_off[kPushItems * 16];   // per (item, wave): count, then offset in the block's run
    __shared__ uint32_t s_base;
    const uint32_t w = threadIdx.x >> 6, nw = blockDim.x >> 6;
    unsigned long long m[kPushItems];
#pragma unroll
    for (uint32_t k = 0; k < kPushItems; ++k) m[k] = __ballot((keep >> k) & 1u);
    if (lane_id() == 0) {
#pragma unroll
        for (uint32_t k = 0; k < kPushItems; ++k) s_off[k * nw + w] = (uint32_t)__popcll(m[k]);
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t tot = 0;
        for (uint32_t j = 0; j < kPushItems * nw; ++j) {
            const uint32_t c = s_off[j];
            s_off[j] = tot;
            tot += c;
        }
        s_base = tot ? atomicAdd(cnt, tot) : 0u;
    }
    __syncthreads();
#pragma unroll
    for (uint32_t k = 0; k < kPushItems; ++k)
        if ((keep >> k) & 1u) q[s_base + s_off[k * nw + w] + lanes_below(m[k])] = val(k);
    __syncthreads();   // s_off and s_base are reused by the next call
}

__device__ __forceinline__ unsigned long long wave_sum_u64(unsigned long long v) {
    for (int off = 32; off > 0; off >>= 1) {
        const uint32_t lo = __shfl_xor((uint32_t)v, off);
        const uint32_t hi = __shfl_xor((uint32_t)(v >> 32), off);
        v += ((unsigned long long)hi << 32) | lo;
    }
    return v;
}

// ------------------------------------------------------------------ ray feed
constexpr uint32_t kRefill = 16;   // idle lanes that trigger a refill (traversal kernels)
constexpr uint32_t kRefillPath = 8;   // ... (path finishing kernels, whose paths take longer)
constexpr uint32_t kRefillCam = 4;    // ... (the stepped camera finishing: with its event turns,
                                      // large scene 47.6 -> 47.1 ms per launch against 8)
constexpr uint32_t kEventBatch = 32;   // pending photon events that are run together

// Persistent lanes: each wave owns a batch of rays [next, end) of the
// launch's list (the first batch by the wave's index in the grid, the rest
// from the launch's atomic counter, so small launches cost no atomics); a
// lane whose ray is finished takes the next ray of the batch once at least
// `refill` lanes of the wave are idle while the others go on, so a wave
// does not idle behind its slowest ray.  Batches are 64 to 256 rays, smaller for
// small launches so that the rays spread over the whole grid.  All members
// are wave-uniform.
struct RayFeed {
    uint32_t n, waves, batch, next, end, refill;
    uint32_t* counter;
    bool drained;

    __device__ __forceinline__ void init(uint32_t n_rays, uint32_t* work, uint32_t refill_lanes = kRefill) {
        n = n_rays;
        refill = refill_lanes;
        waves = gridDim.x * (blockDim.x >> 6);
        const uint32_t per_wave = n / (4u * waves);
        batch = per_wave >= 256u ? 256u : (per_wave >= 128u ? 128u : 64u);
        next = (blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6)) * batch;
        end = next < n ? min(next + batch, n) : next;
        drained = next >= n;
        counter = work;
    }

    // Called by every lane of the wave; returns the list index of the new
    // ray for an idle lane that receives one, else 0xffffffff.
    __device__ __forceinline__ uint32_t take(bool idle_lane) {
        const unsigned long long idle = __ballot(idle_lane);
        const uint32_t n_idle = (uint32_t)__popcll(idle);
        if (n_idle < refill) return 0xffffffffu;
        if (next >= end && !drained) {
            uint32_t base = 0;
            if (lane_id() == 0) base = atomicAdd(counter, batch);
            base = __shfl(base, 0) + waves * batch;
            next = base;
            end = base < n ? min(base + batch, n) : base;
            drained = base >= n;
        }
        const uint32_t i = next + lanes_below(idle);
        next = min(next + n_idle, end);
        return (idle_lane && i < end) ? i : 0xffffffffu;
    }
};

// ------------------------------------------------------------------ closest hit
template <bool COUNT>
__global__ __launch_bounds__(kTraceBS) void k_closest(DevScene S, RaySoA R, HitSoA H, const uint32_t* __restrict__ queue,
                                                      const uint32_t* __restrict__ count, uint32_t n_static,
                                                      uint32_t* __restrict__ work, DevCounters* __restrict__ C) {
    __shared__ uint2 lds[kLdsStack][kTraceBS];
    // the top of a large tree staged in LDS (measured on the 2M-triangle
    // scene: 2-3% less time per launch; the medium scene's 21k-node tree
    // keeps its top in cache and is 1% slower with it, so it is not staged)
    __shared__ float4 top[kTopNodes * 16];
    const bool use_top = S.n_nodes >= kTopMinNodes;
    if (use_top) {
        const float4* g = reinterpret_cast<const float4*>(S.nodes);
        for (uint32_t i = threadIdx.x; i < kTopNodes * 16; i += blockDim.x) top[i] = g[i];
        __syncthreads();
    }
    Spill st;
    const uint32_t n = count ? *count : n_static;
    RayFeed feed;
    feed.init(n, work);
    VisitCount vc;
    Trav t;
    uint32_t pid = 0;
    bool active = false;
    for (;;) {
        const uint32_t i = feed.take(!active);
        if (i != 0xffffffffu) {
            pid = queue ? queue[i] : i;
            trav_init(t, F3{R.ox[pid], R.oy[pid], R.oz[pid]}, F3{R.dx[pid], R.dy[pid], R.dz[pid]});
            active = true;
        }
        if (__ballot(active) == 0ull) break;
        if (active && trav_step<kTraceBS, COUNT>(S, t, lds, st, vc, use_top ? top : nullptr)) {
            const HitRec h = trav_result(t);
            H.t[pid] = h.t;
            H.prim[pid] = h.prim;
            if (H.u) H.u[pid] = h.u;
            if (H.v) H.v[pid] = h.v;
            active = false;
        }
    }
    // every ray of the list is traced exactly once
    if (blockIdx.x == 0 && threadIdx.x == 0 && n) {
        atomicAdd(&C->rays_closest, (unsigned long long)n);
        atomicAdd(&C->rays_staged, (unsigned long long)n);
    }
    if (COUNT) {
        const unsigned long long c_nodes = wave_sum_u64(vc.nodes), c_tris = wave_sum_u64(vc.tris);
        if (lane_id() == 0 && c_nodes) {
            atomicAdd(&C->node_visits, c_nodes);
            atomicAdd(&C->tri_tests, c_tris);
        }
    }
}

// ------------------------------------------------------------------ any hit
// Shadow / occlusion rays, with the persistent lanes of k_closest: a lane
// whose ray has ended takes the next one from the wave's batch, so a wave
// does not wait for its longest ray (shadow rays to the lights cross the
// whole scene when unoccluded and end at once when blocked).  For shadow
// rays of camera paths, an unoccluded segment adds its stored
// contribution to L.
template <bool COUNT>
__global__ __launch_bounds__(kTraceBS) void k_anyhit(DevScene S, ShadowSoA R, const uint32_t* __restrict__ queue,
                                                     const uint32_t* __restrict__ count, uint32_t n_static,
                                                     uint32_t* __restrict__ work, uint8_t* __restrict__ occ_out,
                                                     float* __restrict__ L, DevCounters* __restrict__ C) {
    __shared__ uint2 lds[kLdsStack][kTraceBS];
    __shared__ float4 top[kTopNodes * 16];   // as in k_closest
    const bool use_top = S.n_nodes >= kTopMinNodes;
    if (use_top) {
        const float4* g = reinterpret_cast<const float4*>(S.nodes);
        for (uint32_t i = threadIdx.x; i < kTopNodes * 16; i += blockDim.x) top[i] = g[i];
        __syncthreads();
    }
    Spill st;
    VisitCount vc;
    const uint32_t n = count ? *count : n_static;
    RayFeed feed;
    feed.init(n, work);
    Trav t;
    uint32_t pid = 0;
    bool active = false;
    for (;;) {
        const uint32_t i = feed.take(!active);
        if (i != 0xffffffffu) {
            pid = queue ? queue[i] : i;
            any_init(t, F3{R.ox[pid], R.oy[pid], R.oz[pid]}, F3{R.dx[pid], R.dy[pid], R.dz[pid]}, R.tmax[pid],
                     R.excl ? R.excl[pid] : 0xffffffffu);
            active = true;
        }
        if (__ballot(active) == 0ull) break;
        if (active && tstep<kTraceBS, COUNT, kAny>(S, t, lds, st, vc, use_top ? top : nullptr)) {
            if (occ_out) occ_out[pid] = t.hit ? 1 : 0;
            if (L && !t.hit) L[pid] = L[pid] + R.contrib[pid];
            active = false;
        }
    }
    if (blockIdx.x == 0 && threadIdx.x == 0 && n) {
        atomicAdd(&C->rays_shadow, (unsigned long long)n);
        atomicAdd(&C->any_rays, (unsigned long long)n);
    }
    if (COUNT) {
        const unsigned long long c_nodes = wave_sum_u64(vc.nodes), c_tris = wave_sum_u64(vc.tris);
        if (lane_id() == 0 && c_nodes) {
            atomicAdd(&C->any_nodes, c_nodes);
            atomicAdd(&C->any_tris, c_tris);
        }
    }
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

__device__ __forceinline__ CamPath load_path(const PathState& P, uint32_t pid) {
    CamPath c;
    c.o = F3{P.ox[pid], P.oy[pid], P.oz[pid]};
    c.d = F3{P.dx[pid], P.dy[pid], P.dz[pid]};
    c.T = P.T[pid];
    c.L = P.L[pid];
    c.lam = P.lambda[pid];
    c.flags = P.flags[pid];
    c.med = P.med[pid];
    return c;
}
__device__ __forceinline__ void store_ray(const PathState& P, uint32_t pid, const CamPath& c) {
    P.ox[pid] = c.o.x; P.oy[pid] = c.o.y; P.oz[pid] = c.o.z;
    P.dx[pid] = c.d.x; P.dy[pid] = c.d.y; P.dz[pid] = c.d.z;
}
__device__ __forceinline__ HitRec load_hit(const PathState& P, uint32_t pid) {
    return HitRec{P.t[pid], P.u[pid], P.v[pid], P.prim[pid]};
}

// `extra`: further entries another kernel appends to the same queue before
// the first closest-hit launch (the ground truth's pixel-centre rays).
__global__ void k_raygen(CamInfo ci, WaveDev wl, PathState P, uint32_t n, uint32_t* queue, uint32_t* counts,
                         uint32_t extra) {
    for (uint32_t pid = blockIdx.x * blockDim.x + threadIdx.x; pid < n; pid += gridDim.x * blockDim.x) {
        uint32_t pix, sample, slot;
        pid_decode(ci, pid, pix, sample, slot);
        const CamPath c = camera_start(ci.cam, wl, ci.seed, pix, sample, slot);
        store_ray(P, pid, c);
        P.T[pid] = c.T;
        P.L[pid] = c.L;
        P.lambda[pid] = c.lam;
        P.flags[pid] = c.flags;
        P.med[pid] = c.med;
        queue[pid] = pid;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) counts[QC_CUR] = n + extra;
}

// Sort hits by material: emitters and misses end here, dielectric and
// diffuse hits go to their own queues.  Queue entries from path_end on are
// not camera paths (the ground truth's rays traced in the same launch) and
// are left alone.
__global__ void k_classify(DevScene S, PathState P, const uint32_t* __restrict__ queue, uint32_t* counts,
                           uint32_t* q_diffuse, uint32_t* q_dielectric, uint32_t path_end) {
    const uint32_t n = counts[QC_CUR];
    const uint32_t per = push_items(n), span = blockDim.x * per;
    for (uint32_t base = blockIdx.x * span; base < n; base += gridDim.x * span) {
        uint32_t diff = 0, diel = 0;
        for (uint32_t k = 0; k < per; ++k) {
            const uint32_t i = base + k * blockDim.x + threadIdx.x;
            if (i >= n) break;
            const uint32_t pid = queue[i];
            if (pid >= path_end) continue;
            const uint32_t prim = P.prim[pid];
            if (prim == 0xffffffffu) continue;
            const uint32_t type = S.mat[S.tri_obj[prim]].type;
            if (type == SC_MAT_EMISSIVE) {
                CamPath c = load_path(P, pid);
                camera_emission(S, load_hit(P, pid), c);
                P.L[pid] = c.L;
            } else if (type == SC_MAT_DIELECTRIC) {
                diel |= 1u << k;
            } else {
                diff |= 1u << k;
            }
        }
        auto pid_of = [&](uint32_t k) { return queue[base + k * blockDim.x + threadIdx.x]; };
        block_push(diel, pid_of, q_dielectric, counts + QC_DIEL);
        block_push(diff, pid_of, q_diffuse, counts + QC_DIFF);
    }
}

__global__ void k_shade_dielectric(DevScene S, CamInfo ci, PathState P, uint32_t depth, const uint32_t* __restrict__ q,
                                   uint32_t* counts, uint32_t* q_next) {
    const uint32_t n = counts[QC_DIEL];
    const uint32_t per = push_items(n), span = blockDim.x * per;
    for (uint32_t base = blockIdx.x * span; base < n; base += gridDim.x * span) {
        uint32_t cont = 0;
        for (uint32_t k = 0; k < per; ++k) {
            const uint32_t i = base + k * blockDim.x + threadIdx.x;
            if (i >= n) break;
            const uint32_t pid = q[i];
            uint32_t pix, sample, slot;
            pid_decode(ci, pid, pix, sample, slot);
            CamPath c = load_path(P, pid);
            if (camera_dielectric(S, ci.seed, pix, sample, slot, depth, ci.max_depth, load_hit(P, pid), c)) {
                store_ray(P, pid, c);
                P.T[pid] = c.T;
                P.med[pid] = c.med;
                cont |= 1u << k;
            }
        }
        block_push(cont, [&](uint32_t k) { return q[base + k * blockDim.x + threadIdx.x]; }, q_next, counts + QC_NEXT);
    }
}

// PM: caustics gathered from a general photon map (pm), else from the
// receiver map cmap; the template lets the default path drop the gather.
template <bool PM>
__global__ void k_shade_diffuse(DevScene S, CamInfo ci, WaveDev wl, PathState P, uint32_t depth,
                                const float* __restrict__ cmap, PMapDev pm_arg, const uint32_t* __restrict__ q,
                                uint32_t* counts, uint32_t* q_next, uint32_t* q_shadow) {
    const PMapDev pm = PM ? pm_arg : PMapDev{};
    const uint32_t n = counts[QC_DIFF];
    const uint32_t per = push_items(n), span = blockDim.x * per;
    for (uint32_t base = blockIdx.x * span; base < n; base += gridDim.x * span) {
        uint32_t cont = 0, shoot = 0;
        for (uint32_t k = 0; k < per; ++k) {
            const uint32_t i = base + k * blockDim.x + threadIdx.x;
            if (i >= n) break;
            const uint32_t pid = q[i];
            uint32_t pix, sample, slot;
            pid_decode(ci, pid, pix, sample, slot);
            CamPath c = load_path(P, pid);
            ShadowReq sr;
            sr.shoot = false;
            const bool more = camera_diffuse(S, wl, cmap, pm, ci.seed, pix, sample, slot, depth, ci.max_depth,
                                             load_hit(P, pid), c, sr);
            P.L[pid] = c.L;
            P.flags[pid] = c.flags;
            if (sr.shoot) {
                P.sox[pid] = sr.o.x; P.soy[pid] = sr.o.y; P.soz[pid] = sr.o.z;
                P.sdx[pid] = sr.d.x; P.sdy[pid] = sr.d.y; P.sdz[pid] = sr.d.z;
                P.stmax[pid] = sr.tmax;
                P.sexcl[pid] = sr.excl;
                P.scontrib[pid] = sr.contrib;
                shoot |= 1u << k;
            }
            if (more) {
                store_ray(P, pid, c);
                P.T[pid] = c.T;
                cont |= 1u << k;
            }
        }
        auto pid_of = [&](uint32_t k) { return q[base + k * blockDim.x + threadIdx.x]; };
        block_push(shoot, pid_of, q_shadow, counts + QC_SHADOW);
        block_push(cont, pid_of, q_next, counts + QC_NEXT);
    }
}

// Film: per pixel, samples of the chunk added in sample order.
__global__ void k_film_accumulate(CamInfo ci, WaveDev wl, const float* __restrict__ L, const float* __restrict__ lambda,
                                  uint32_t n_samples, float* __restrict__ rgb) {
    for (uint32_t pix = blockIdx.x * blockDim.x + threadIdx.x; pix < ci.hw; pix += gridDim.x * blockDim.x) {
        float acc[3] = {rgb[3 * (size_t)pix], rgb[3 * (size_t)pix + 1], rgb[3 * (size_t)pix + 2]};
        for (uint32_t s = 0; s < n_samples; ++s) {
            const size_t base = ((size_t)s * ci.hw + pix) * ci.K;
            for (uint32_t slot = 0; slot < ci.K; ++slot) film_add(wl, ci.K, slot, L[base + slot], lambda[base + slot], acc);
        }
        rgb[3 * (size_t)pix] = acc[0];
        rgb[3 * (size_t)pix + 1] = acc[1];
        rgb[3 * (size_t)pix + 2] = acc[2];
    }
}

__global__ void k_film_scale(float* rgb, uint32_t n, float inv_spp) {
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
        rgb[i] = rgb[i] * inv_spp;
}

// ------------------------------------------------------------------ ground truth
// Pixel-centre rays of the ground truth; with `queue`, entry pix of it is
// set to id0 + pix (the rays then join a closest-hit launch's queue).
__global__ void k_aov_raygen(sc_camera cam, RaySoA R, uint32_t* queue, uint32_t id0) {
    const uint32_t hw = cam.w * cam.h;
    for (uint32_t pix = blockIdx.x * blockDim.x + threadIdx.x; pix < hw; pix += gridDim.x * blockDim.x) {
        F3 o, d;
        camera_ray(cam, pix % cam.w, pix / cam.w, 0.5f, 0.5f, o, d);
        R.ox[pix] = o.x; R.oy[pix] = o.y; R.oz[pix] = o.z;
        R.dx[pix] = d.x; R.dy[pix] = d.y; R.dz[pix] = d.z;
        if (queue) queue[pix] = id0 + pix;
    }
}

__global__ void k_aov_write(DevScene S, sc_camera cam, RaySoA R, HitSoA H, sc_aov out) {
    const uint32_t hw = cam.w * cam.h;
    for (uint32_t pix = blockIdx.x * blockDim.x + threadIdx.x; pix < hw; pix += gridDim.x * blockDim.x) {
        const F3 d{R.dx[pix], R.dy[pix], R.dz[pix]};
        aov_write(S, cam, pix, d, HitRec{H.t[pix], H.u[pix], H.v[pix], H.prim[pix]}, out);
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
    int general;        // deposits go to rec (general photon map) instead of the receiver map
    PmRecords rec;
    uint32_t* touched;  // receiver map: [0] count, then the cells the pass made non-zero
};

__device__ __forceinline__ void ph_stat(DevCounters* C, const PhInfo& pi, int outcome, float phi) {
    if (!pi.stats) return;
    atomicAdd(&C->ph_count[outcome], 1ull);
    atomicAdd(&C->ph_flux[outcome], (double)phi);
}

__global__ void k_photon_emit(DevScene S, WaveDev wl, PhInfo pi, uint32_t n, PhotonState Ph, uint32_t* queue,
                              uint32_t* counts, DevCounters* C) {
    const uint32_t per = push_items(n), span = blockDim.x * per;
    for (uint32_t base = blockIdx.x * span; base < n; base += gridDim.x * span) {
        uint32_t alive = 0;
        for (uint32_t k = 0; k < per; ++k) {
            const uint32_t i = base + k * blockDim.x + threadIdx.x;
            if (i >= n) break;
            PhotonPath ph;
            if (!photon_emit(S, wl, pi.seed, pi.n_total, pi.p0 + i, ph)) {
                if (pi.stats) atomicAdd(&C->ph_count[SC_PH_EMIT_DEAD], 1ull);
                continue;
            }
            Ph.ox[i] = ph.o.x; Ph.oy[i] = ph.o.y; Ph.oz[i] = ph.o.z;
            Ph.dx[i] = ph.d.x; Ph.dy[i] = ph.d.y; Ph.dz[i] = ph.d.z;
            Ph.phi[i] = ph.phi;
            Ph.lambda[i] = ph.lam;
            Ph.slot[i] = ph.slot;
            Ph.spec[i] = ph.spec;
            Ph.med[i] = ph.med;
            alive |= 1u << k;
        }
        block_push(alive, [&](uint32_t k) { return base + k * blockDim.x + threadIdx.x; }, queue, counts + QC_CUR);
    }
}

// Deposit fixed-point flux; lanes of a wave that hit the same cell as the
// first depositing lane combine into one atomic.
// Every lane of the wave calls it.  With `touched`, a cell that an add takes
// from zero is appended to it (one counter atomic per wave), so the map can
// be finalised and the accumulator cleared cell by cell.
__device__ __forceinline__ void deposit(bool want, uint32_t cell, unsigned long long q, unsigned long long* acc,
                                        uint32_t* cnt_map, uint32_t* touched) {
    const unsigned long long m = __ballot(want);
    if (m == 0ull) return;
    const uint32_t leader = __ffsll((long long)m) - 1;
    const uint32_t lcell = __shfl(cell, (int)leader);
    const bool same = want && cell == lcell;
    const unsigned long long ms = __ballot(same);
    const unsigned long long part = wave_sum_u64(same ? q : 0ull);
    bool first = false;
    uint32_t fcell = 0;
    if (lane_id() == leader) {
        if (touched) {
            const unsigned long long old = atomicAdd(&acc[lcell], part);
            first = old == 0ull && part != 0ull;
            fcell = lcell;
        } else {
            atomicAdd(&acc[lcell], part);
        }
        if (cnt_map) atomicAdd(&cnt_map[lcell], (uint32_t)__popcll(ms));
    }
    if (want && !same) {
        if (touched) {
            const unsigned long long old = atomicAdd(&acc[cell], q);
            first = old == 0ull && q != 0ull;
            fcell = cell;
        } else {
            atomicAdd(&acc[cell], q);
        }
        if (cnt_map) atomicAdd(&cnt_map[cell], 1u);
    }
    if (!touched) return;
    const unsigned long long fm = __ballot(first);
    if (fm != 0ull) {
        const uint32_t lo = __ffsll((long long)fm) - 1;
        uint32_t base = 0;
        if (lane_id() == lo) base = atomicAdd(touched, (uint32_t)__popcll(fm));
        base = __shfl(base, (int)lo);
        if (first) touched[1 + base + lanes_below(fm)] = fcell;
    }
}

__device__ __forceinline__ uint32_t wave_max_u32(uint32_t v) {
    for (int off = 32; off > 0; off >>= 1) v = max(v, (uint32_t)__shfl_xor((int)v, off));
    return v;
}

// Store one photon of a general photon map: one counter atomic per wave.
// Flux and coordinates are non-negative or compared by magnitude, so their
// maxima are tracked on the float bits.
__device__ __forceinline__ void pm_store(const PmRecords& R, uint32_t k, const Deposit& dp, uint32_t ch, float phi,
                                         uint64_t photon) {
    if (k >= R.cap) return;
    R.px[k] = dp.P.x; R.py[k] = dp.P.y; R.pz[k] = dp.P.z;
    R.nx[k] = dp.N.x; R.ny[k] = dp.N.y; R.nz[k] = dp.N.z;
    R.phi[k] = phi;
    R.ch[k] = ch;
    R.photon[k] = photon;
}

__device__ __forceinline__ uint32_t pm_extent_bits(const Deposit& dp) {
    return __float_as_uint(fmaxf(fabsf(dp.P.x), fmaxf(fabsf(dp.P.y), fabsf(dp.P.z))));
}

__device__ __forceinline__ void pm_append(bool want, const PmRecords& R, const Deposit& dp, uint32_t ch, float phi,
                                          uint64_t photon) {
    const unsigned long long m = __ballot(want);
    if (m == 0ull) return;
    const uint32_t leader = __ffsll((long long)m) - 1;
    const uint32_t mphi = wave_max_u32(want ? __float_as_uint(phi) : 0u);
    const uint32_t mext = wave_max_u32(want ? pm_extent_bits(dp) : 0u);
    uint32_t base = 0;
    if (lane_id() == leader) {
        base = atomicAdd(&R.stat[0], (uint32_t)__popcll(m));
        atomicMax(&R.stat[1], mphi);
        atomicMax(&R.stat[2], mext);
    }
    base = __shfl(base, (int)leader);
    if (want) pm_store(R, base + lanes_below(m), dp, ch, phi, photon);
}

__global__ void k_photon_event(DevScene S, WaveDev wl, PhInfo pi, uint32_t depth, PhotonState Ph,
                               const uint32_t* __restrict__ queue, uint32_t* counts, uint32_t* q_next,
                               unsigned long long* acc, uint32_t* cnt_map, DevCounters* C) {
    const uint32_t n = counts[QC_CUR];
    const uint32_t per = push_items(n), span = blockDim.x * per;
    for (uint32_t base = blockIdx.x * span; base < n; base += gridDim.x * span) {
        uint32_t cont = 0;
        for (uint32_t k = 0; k < per; ++k) {
            if (base + k * blockDim.x >= n) break;   // uniform over the block: the deposits below are wave-collective
            const uint32_t i = base + k * blockDim.x + threadIdx.x;
            bool dep = false;
            uint32_t id = 0, cell_ch = 0;
            unsigned long long fx = 0;
            float phi = 0.0f;
            Deposit dp;
            dp.cell_ch = -1;
            if (i < n) {
                id = queue[i];
                PhotonPath ph;
                ph.o = F3{Ph.ox[id], Ph.oy[id], Ph.oz[id]};
                ph.d = F3{Ph.dx[id], Ph.dy[id], Ph.dz[id]};
                ph.phi = Ph.phi[id];
                ph.lam = Ph.lambda[id];
                ph.slot = Ph.slot[id];
                ph.spec = Ph.spec[id];
                ph.med = Ph.med[id];
                int outcome = -1;
                const bool more = photon_event(S, wl, pi.seed, pi.p0 + id, depth, pi.max_depth, pi.general != 0,
                                               HitRec{Ph.t[id], Ph.u[id], Ph.v[id], Ph.prim[id]}, ph, outcome, dp);
                if (more) {
                    Ph.ox[id] = ph.o.x; Ph.oy[id] = ph.o.y; Ph.oz[id] = ph.o.z;
                    Ph.dx[id] = ph.d.x; Ph.dy[id] = ph.d.y; Ph.dz[id] = ph.d.z;
                    Ph.phi[id] = ph.phi;
                    Ph.spec[id] = ph.spec;
                    Ph.med[id] = ph.med;
                    cont |= 1u << k;
                } else {
                    ph_stat(C, pi, outcome, ph.phi);
                }
                if (dp.cell_ch >= 0) {
                    dep = true;
                    cell_ch = (uint32_t)dp.cell_ch;
                    fx = __double2ull_rn((double)ph.phi * pi.scale);
                    phi = ph.phi;
                }
            }
            if (pi.general) pm_append(dep, pi.rec, dp, cell_ch, phi, pi.p0 + id);
            else deposit(dep, cell_ch, fx, acc, cnt_map, pi.touched);
        }
        block_push(cont, [&](uint32_t k) { return queue[base + k * blockDim.x + threadIdx.x]; }, q_next,
                   counts + QC_NEXT);
    }
}

// ------------------------------------------------------------------ path finishing
// After the first bounces have run as one launch per stage, the paths still
// alive are few and a launch per further bounce would cost a whole traversal
// latency each.  These kernels give each remaining path (or photon) to one
// lane, which follows it one bounce per loop turn with the same per-path
// functions, so the outputs are the same bit for bit.  A lane whose path has
// ended takes the next one through the same feed as the traversal kernel
// (per-wave batches, refilled once enough lanes are idle), so a wave does not
// wait for its longest path with the other lanes idle.
__device__ __forceinline__ void count_rays(uint32_t n_cl, uint32_t n_sh, DevCounters* C) {
    const unsigned long long a = wave_sum_u64(n_cl), b = wave_sum_u64(n_sh);
    if (lane_id() == 0) {
        if (a) atomicAdd(&C->rays_closest, a);
        if (b) atomicAdd(&C->rays_shadow, b);
    }
}

// Camera paths: a lane advances its current ray (the next bounce's
// closest-hit ray or the last diffuse event's shadow ray, with the same
// traversal step) one step per loop turn, so no lane waits for the slowest
// traversal of its wave; the events run together once kEventBatch lanes have
// one pending or no lane is tracing.  The two costly kinds of event,
// dielectric and diffuse, take turns: a turn runs the kind with more lanes
// waiting (and every cheap one), the other kind waits for a later turn
// (both run once no lane is tracing).  Run together, each branch had held
// about 10 of the 64 lanes; large scene: 49.6 -> 47.5 ms per launch, the
// same image.  A shadow ray is traced before the
// path's next bounce, so radiance adds up in the same order as in
// camera_continue.  Register use is held to 128 (4 waves per SIMD, the 8
// blocks per CU of the persistent grid all resident): large scene, 42.5 ->
// 30.2 ms per step against one blocking traversal per bounce at 145
// registers (3 waves per SIMD).
// (PM is false here: paths gathering from a general photon map go to
// k_finish_camera_pm below.)
template <bool PM, bool COUNT>
__global__ __launch_bounds__(kTraceBS) __attribute__((amdgpu_waves_per_eu(4, 4))) void k_finish_camera(
    DevScene S, CamInfo ci, WaveDev wl, PathState P,
                                                            const float* __restrict__ cmap, PMapDev pm_arg,
                                                            const uint32_t* __restrict__ queue,
                                                            const uint32_t* __restrict__ count, uint32_t depth0,
                                                            uint32_t* __restrict__ work, DevCounters* __restrict__ C) {
    const PMapDev pm = PM ? pm_arg : PMapDev{};
    __shared__ uint2 lds[kLdsStack][kTraceBS];
    Spill st;
    VisitCount vc;
    const uint32_t n = *count;
    RayFeed feed;
    feed.init(n, work, kRefillCam);
    uint32_t n_cl = 0, n_sh = 0;
    CamPath c;
    Trav t;
    uint32_t pid = 0, pix = 0, sample = 0, slot = 0, depth = 0;
    float sh_contrib = 0.0f;
    bool after_shadow = false;   // the path goes on once its shadow ray is done
    // each lane: 0 idle, 1 tracing (its closest-hit ray or its shadow ray,
    // one step per loop turn), 2 traversal done and its event pending, then
    // at the next event turn 3 / 4 / 5 for a pending dielectric / diffuse /
    // other event (shadow result, miss, emission)
    uint32_t state = 0;
    for (;;) {
        const uint32_t i = feed.take(state == 0);
        if (i != 0xffffffffu) {
            pid = queue[i];
            pid_decode(ci, pid, pix, sample, slot);
            c = load_path(P, pid);
            depth = depth0;
            trav_init(t, c.o, c.d);
            state = 1;
        }
        if (__ballot(state != 0) == 0ull) break;
        if (state == 1 && tstep<kTraceBS, COUNT, kEither>(S, t, lds, st, vc)) state = 2;
        const unsigned long long pend = __ballot(state >= 2);
        const bool tracing = __ballot(state == 1) != 0ull;
        if (pend == 0ull || ((uint32_t)__popcll(pend) < kEventBatch && tracing)) continue;
        // new arrivals sorted by event kind: 3 dielectric, 4 diffuse, 5 the
        // rest (shadow result, miss, emission)
        if (state == 2) {
            uint32_t k = 5u;
            if (!t.any && t.pb != 0xffffffffu) {
                const uint32_t type = S.mat[S.tri_obj[t.pb]].type;
                k = type == SC_MAT_DIELECTRIC ? 3u : (type == SC_MAT_EMISSIVE ? 5u : 4u);
            }
            state = k;
        }
        const uint32_t n3 = (uint32_t)__popcll(__ballot(state == 3u)), n4 = (uint32_t)__popcll(__ballot(state == 4u));
        const uint32_t skip = tracing ? (n4 >= n3 ? 3u : 4u) : 0u;
        if (state < 3u || state == skip) continue;
        bool cont = false;
        if (t.any) {   // the shadow ray of the last diffuse event
            if (!t.hit) c.L = c.L + sh_contrib;
            cont = after_shadow;
        } else {       // one bounce, as in camera_continue
            const HitRec h = trav_result(t);
            ++n_cl;
            if (state == 3u) {
                cont = camera_dielectric(S, ci.seed, pix, sample, slot, depth, ci.max_depth, h, c);
            } else if (state == 4u) {
                ShadowReq sr;
                cont = camera_diffuse(S, wl, cmap, pm, ci.seed, pix, sample, slot, depth, ci.max_depth, h, c, sr);
                if (sr.shoot) {
                    ++n_sh;
                    sh_contrib = sr.contrib;
                    after_shadow = cont;
                    any_init(t, sr.o, sr.d, sr.tmax, sr.excl);
                    state = 1;
                    continue;
                }
            } else if (h.prim != 0xffffffffu) {
                camera_emission(S, h, c);
            }
        }
        if (cont) {
            ++depth;
            trav_init(t, c.o, c.d);
            state = 1;
        } else {
            P.L[pid] = c.L;
            state = 0;
        }
    }
    count_rays(n_cl, n_sh, C);
    const unsigned long long c_rays = wave_sum_u64(n_cl), c_sh = wave_sum_u64(n_sh);
    if (lane_id() == 0 && (c_rays || c_sh)) {
        atomicAdd(&C->cf_rays, c_rays);
        atomicAdd(&C->cf_shadow, c_sh);
    }
    if (blockIdx.x == 0 && threadIdx.x == 0 && n) atomicAdd(&C->cf_paths, (unsigned long long)n);
    if (COUNT) {
        const unsigned long long c_nodes = wave_sum_u64(vc.nodes), c_tris = wave_sum_u64(vc.tris);
        if (lane_id() == 0 && c_nodes) {
            atomicAdd(&C->cf_nodes, c_nodes);
            atomicAdd(&C->cf_tris, c_tris);
        }
    }
}

// General photon maps: the gather keeps 192 registers live, and held to
// 128 the stepped form above spilled and ran slower (clutter scene render
// 5.8 -> 7.0 ms), so these paths keep one blocking traversal per bounce.
template <bool COUNT>
__global__ __launch_bounds__(kTraceBS) void k_finish_camera_pm(DevScene S, CamInfo ci, WaveDev wl, PathState P,
                                                            const float* __restrict__ cmap, PMapDev pm_arg,
                                                            const uint32_t* __restrict__ queue,
                                                            const uint32_t* __restrict__ count, uint32_t depth0,
                                                            uint32_t* __restrict__ work, DevCounters* __restrict__ C) {
    const PMapDev pm = pm_arg;
    __shared__ uint2 lds[kLdsStack][kTraceBS];
    Spill st;
    VisitCount vc;
    const uint32_t n = *count;
    RayFeed feed;
    feed.init(n, work, kRefillPath);
    uint32_t n_cl = 0, n_sh = 0;
    CamPath c;
    uint32_t pid = 0, pix = 0, sample = 0, slot = 0, depth = 0;
    bool active = false;
    for (;;) {
        const uint32_t i = feed.take(!active);
        if (i != 0xffffffffu) {
            pid = queue[i];
            pid_decode(ci, pid, pix, sample, slot);
            c = load_path(P, pid);
            depth = depth0;
            active = true;
        }
        if (__ballot(active) == 0ull) break;
        if (!active) continue;
        // one bounce, as in camera_continue
        const HitRec h = trace_closest<kTraceBS, COUNT>(S, c.o, c.d, lds, st, vc);
        ++n_cl;
        bool cont = false;
        if (h.prim != 0xffffffffu) {
            const uint32_t type = S.mat[S.tri_obj[h.prim]].type;
            if (type == SC_MAT_EMISSIVE) {
                camera_emission(S, h, c);
            } else if (type == SC_MAT_DIELECTRIC) {
                cont = camera_dielectric(S, ci.seed, pix, sample, slot, depth, ci.max_depth, h, c);
            } else {
                ShadowReq sr;
                cont = camera_diffuse(S, wl, cmap, pm, ci.seed, pix, sample, slot, depth, ci.max_depth, h, c, sr);
                if (sr.shoot) {
                    ++n_sh;
                    if (!trace_any<kTraceBS, COUNT>(S, sr.o, sr.d, sr.tmax, sr.excl, lds, st, vc))
                        c.L = c.L + sr.contrib;
                }
            }
        }
        if (cont) {
            ++depth;
        } else {
            P.L[pid] = c.L;
            active = false;
        }
    }
    count_rays(n_cl, n_sh, C);
    const unsigned long long c_rays = wave_sum_u64(n_cl), c_sh = wave_sum_u64(n_sh);
    if (lane_id() == 0 && (c_rays || c_sh)) {
        atomicAdd(&C->cf_rays, c_rays);
        atomicAdd(&C->cf_shadow, c_sh);
    }
    if (blockIdx.x == 0 && threadIdx.x == 0 && n) atomicAdd(&C->cf_paths, (unsigned long long)n);
    if (COUNT) {
        const unsigned long long c_nodes = wave_sum_u64(vc.nodes), c_tris = wave_sum_u64(vc.tris);
        if (lane_id() == 0 && c_nodes) {
            atomicAdd(&C->cf_nodes, c_nodes);
            atomicAdd(&C->cf_tris, c_tris);
        }
    }
}

template <bool COUNT>
__global__ __launch_bounds__(kTraceBS) void k_finish_photons(DevScene S, WaveDev wl, PhInfo pi, uint32_t depth0,
                                                             PhotonState Ph, const uint32_t* __restrict__ queue,
                                                             const uint32_t* __restrict__ count,
                                                             uint32_t* __restrict__ work,
                                                             unsigned long long* __restrict__ acc,
                                                             uint32_t* __restrict__ cnt_map,
                                                             DevCounters* __restrict__ C) {
    __shared__ uint2 lds[kLdsStack][kTraceBS];
    // the top of a large tree staged in LDS, as in k_closest (2^24-photon
    // pass on the 2M-triangle scene: 25.2 -> 24.9 ms); idle lanes refilled
    // at 8 instead of 16 (21.8 -> 21.2 ms per launch; 4 lanes: the same)
    __shared__ float4 top[kTopNodes * 16];
    const bool use_top = S.n_nodes >= kTopMinNodes;
    if (use_top) {
        const float4* g = reinterpret_cast<const float4*>(S.nodes);
        for (uint32_t i = threadIdx.x; i < kTopNodes * 16; i += blockDim.x) top[i] = g[i];
        __syncthreads();
    }
    const float4* topp = use_top ? top : nullptr;
    Spill st;
    VisitCount vc;
    const uint32_t n = *count;
    RayFeed feed;
    feed.init(n, work, kRefillPath);
    uint32_t n_cl = 0;
    PhotonPath ph;
    Trav t;
    uint32_t id = 0, depth = 0;
    // each lane: 0 idle, 1 tracing its path's current segment, 2 hit found
    // and its photon event pending.  Traversal advances one step per loop
    // turn, so no lane waits for the slowest ray of its wave; the events
    // run together once kEventBatch lanes have one pending (or no lane is
    // tracing), so the event code is not entered for one lane at a time.
    uint32_t state = 0;
    // general photon maps: events wait for every lane (measured faster there)
    const uint32_t ev_batch = pi.general ? 65u : kEventBatch;
    for (;;) {
        const uint32_t i = feed.take(state == 0);
        if (i != 0xffffffffu) {
            id = queue[i];
            ph.o = F3{Ph.ox[id], Ph.oy[id], Ph.oz[id]};
            ph.d = F3{Ph.dx[id], Ph.dy[id], Ph.dz[id]};
            ph.phi = Ph.phi[id];
            ph.lam = Ph.lambda[id];
            ph.slot = Ph.slot[id];
            ph.spec = Ph.spec[id];
            ph.med = Ph.med[id];
            depth = depth0;
            trav_init(t, ph.o, ph.d);
            state = 1;
        }
        if (__ballot(state != 0) == 0ull) break;
        if (state == 1 && trav_step<kTraceBS, COUNT>(S, t, lds, st, vc, topp)) state = 2;
        const unsigned long long pend = __ballot(state == 2);
        if (pend == 0ull || ((uint32_t)__popcll(pend) < ev_batch && __ballot(state == 1) != 0ull)) continue;
        // the wave is converged here (the test above is the same for every
        // lane): the deposits below merge their atomics over the wave
        bool cont = false, dep = false;
        int outcome = -1;
        Deposit dp;
        dp.cell_ch = -1;
        if (state == 2) {   // one interaction, as in photon_continue
            const HitRec h = trav_result(t);
            ++n_cl;
            cont = photon_event(S, wl, pi.seed, pi.p0 + id, depth, pi.max_depth, pi.general != 0, h, ph, outcome,
                                dp);
            dep = dp.cell_ch >= 0;
        }
        if (pi.general)
            pm_append(dep, pi.rec, dp, (uint32_t)dp.cell_ch, ph.phi, pi.p0 + id);
        else
            deposit(dep, (uint32_t)dp.cell_ch, dep ? __double2ull_rn((double)ph.phi * pi.scale) : 0ull, acc, cnt_map,
                    pi.touched);
        if (state != 2) continue;
        if (cont) {
            ++depth;
            trav_init(t, ph.o, ph.d);
            state = 1;
        } else {
            if (outcome >= 0) ph_stat(C, pi, outcome, ph.phi);
            state = 0;
        }
    }
    count_rays(n_cl, 0u, C);
    const unsigned long long c_rays = wave_sum_u64(n_cl);
    if (lane_id() == 0 && c_rays) atomicAdd(&C->fin_rays, c_rays);
    if (blockIdx.x == 0 && threadIdx.x == 0 && n) atomicAdd(&C->fin_paths, (unsigned long long)n);
    if (COUNT) {
        const unsigned long long c_nodes = wave_sum_u64(vc.nodes), c_tris = wave_sum_u64(vc.tris);
        if (lane_id() == 0 && c_nodes) {
            atomicAdd(&C->fin_nodes, c_nodes);
            atomicAdd(&C->fin_tris, c_tris);
        }
    }
}

// the receiver map from the cells a pass touched (the rest of the map was
// filled with zeros); their accumulator entries are cleared for the next pass
__global__ void k_map_finalize(const uint32_t* __restrict__ touched, unsigned long long* __restrict__ acc,
                               double inv_scale, float* __restrict__ map) {
    const uint32_t n = touched[0];
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        const uint32_t c = touched[1 + i];
        map[c] = (float)((double)acc[c] * inv_scale);
        acc[c] = 0ull;
    }
}

// the whole receiver map (passes with many photons per cell)
__global__ void k_map_finalize_all(const unsigned long long* __restrict__ acc, size_t n, double inv_scale,
                                   float* __restrict__ map) {
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        map[i] = (float)((double)acc[i] * inv_scale);
}

__global__ void k_zero_f32x4(float4* p, size_t n4) {
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n4; i += (size_t)gridDim.x * blockDim.x)
        p[i] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
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

constexpr uint32_t kWorkSlots = 256;     // traversal launches between clears
constexpr uint32_t kWorkStride = 64;     // words per launch: one counter on its own line

// carve n-element arrays out of one allocation, 256-byte aligned
size_t path_bytes(size_t n) { return 27 * (n * 4 + 256); }
size_t photon_bytes(size_t n) { return 18 * (n * 4 + 256); }

PathState carve_path(void* p, size_t n) {
    Carver c{static_cast<char*>(p)};
    PathState P;
    P.ox = c.take<float>(n); P.oy = c.take<float>(n); P.oz = c.take<float>(n);
    P.dx = c.take<float>(n); P.dy = c.take<float>(n); P.dz = c.take<float>(n);
    P.T = c.take<float>(n); P.L = c.take<float>(n); P.lambda = c.take<float>(n);
    P.flags = c.take<uint32_t>(n); P.med = c.take<uint64_t>(n);
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
    P.slot = c.take<uint32_t>(n); P.spec = c.take<uint32_t>(n); P.med = c.take<uint64_t>(n);
    P.t = c.take<float>(n); P.u = c.take<float>(n); P.v = c.take<float>(n); P.prim = c.take<uint32_t>(n);
    return P;
}

Queues carve_queues(void* p, size_t n) {
    Carver c{static_cast<char*>(p)};
    Queues q;
    q.cur = c.take<uint32_t>(n); q.next = c.take<uint32_t>(n); q.diffuse = c.take<uint32_t>(n);
    q.dielectric = c.take<uint32_t>(n); q.shadow = c.take<uint32_t>(n); q.counts = nullptr;
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
        hipLaunchKernelGGL(k_zero_u32, dim3(64), dim3(256), 0, c->stream, c->work.as<uint32_t>(),
                           kWorkSlots * kWorkStride);
        c->work_slot = 0;
    }
    return c->work.as<uint32_t>() + (size_t)(c->work_slot++) * kWorkStride;
}

void reset_work(Ctx* c) {
    hipLaunchKernelGGL(k_zero_u32, dim3(64), dim3(256), 0, c->stream, c->work.as<uint32_t>(),
                       kWorkSlots * kWorkStride);
    c->work_slot = 0;
}

uint32_t trace_grid(const Ctx* c, size_t n_max) {
    // The persistent traversal kernels: 8 blocks of 128 threads per CU, no
    // more than the work.  Each wave's first batch of rays is fixed by its
    // place in the grid, so waves that only become resident once others
    // have exited start their batch late and lengthen the tail: a grid the
    // chip holds at once wins.  Measured on the medium scene, 4 / 6 / 8 / 10
    // / 16 blocks per CU: 13.2 / 11.6 / 11.3 / 12.0 / 12.3 ms per step.
    // (SC_OPT_TRACE_BLOCKS lowers it to leave room for another stream's work)
    const size_t want = (n_max + kTraceBS - 1) / kTraceBS;
    const size_t cap = (size_t)c->cus * c->trace_blocks;
    return (uint32_t)(want < 1 ? 1 : (want > cap ? cap : want));
}

// timing events are reused across launches (creating them costs host time
// inside the timed region)
hipEvent_t pooled_event(Ctx* c) {
    hipEvent_t e = nullptr;
    if (!c->event_pool.empty()) {
        e = c->event_pool.back();
        c->event_pool.pop_back();
    } else {
        (void)hipEventCreate(&e);
    }
    return e;
}

void launch_closest(Ctx* c, const DevScene& S, RaySoA R, HitSoA H, const uint32_t* queue, const uint32_t* count,
                    uint32_t n_static, size_t n_max) {
    uint32_t* work = next_work_slot(c);
    DevCounters* C = c->counters.as<DevCounters>();
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (c->profile) {
        e0 = pooled_event(c);
        e1 = pooled_event(c);
        (void)hipEventRecord(e0, c->stream);
    }
    if (c->count_visits)
        hipLaunchKernelGGL(k_closest<true>, dim3(trace_grid(c, n_max)), dim3(kTraceBS), 0, c->stream, S, R, H, queue,
                           count, n_static, work, C);
    else
        hipLaunchKernelGGL(k_closest<false>, dim3(trace_grid(c, n_max)), dim3(kTraceBS), 0, c->stream, S, R, H, queue,
                           count, n_static, work, C);
    if (c->profile) {
        (void)hipEventRecord(e1, c->stream);
        c->events.emplace_back(e0, e1);
    }
}

// HIP events around a launch when profiling is on; kind selects the list
// the pair is kept in until the counters are read
struct Timed {
    Ctx* c;
    std::vector<std::pair<hipEvent_t, hipEvent_t>>* list;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    Timed(Ctx* ctx, std::vector<std::pair<hipEvent_t, hipEvent_t>>& l) : c(ctx), list(&l) {
        if (c->profile) {
            e0 = pooled_event(c);
            e1 = pooled_event(c);
            (void)hipEventRecord(e0, c->stream);
        }
    }
    ~Timed() {
        if (c->profile) {
            (void)hipEventRecord(e1, c->stream);
            list->emplace_back(e0, e1);
        }
    }
};

void launch_anyhit(Ctx* c, const DevScene& S, ShadowSoA R, const uint32_t* queue, const uint32_t* count,
                   uint32_t n_static, size_t n_max, uint8_t* occ, float* L) {
    uint32_t* work = next_work_slot(c);
    Timed tm(c, c->any_events);
    if (c->count_visits)
        hipLaunchKernelGGL(k_anyhit<true>, dim3(trace_grid(c, n_max)), dim3(kTraceBS), 0, c->stream, S, R, queue, count,
                           n_static, work, occ, L, c->counters.as<DevCounters>());
    else
        hipLaunchKernelGGL(k_anyhit<false>, dim3(trace_grid(c, n_max)), dim3(kTraceBS), 0, c->stream, S, R, queue,
                           count, n_static, work, occ, L, c->counters.as<DevCounters>());
}

}  // namespace

// Sensor curves (Gaussians, 40 nm, at 650/550/450 nm, mean 1 over the
// range) tabulated every 0.25 nm in double, rounded to float.
uint32_t sensor_table(const sc_wavelengths& wl, std::vector<float>& tab) {
    const uint32_t n = (uint32_t)((double)(wl.hi - wl.lo) * 4.0 + 0.5) + 1;
    tab.assign(3 * (size_t)n, 0.0f);
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
    return n;
}

// device view of a wavelength setting; tab_dev receives the sensor table
// (uniform mode) when not NULL
WaveDev wave_view(const sc_wavelengths& wl, const float* tab_dev, uint32_t n_tab) {
    WaveDev w;
    w.mode = wl.mode;
    w.k = wl.k;
    for (int i = 0; i < 4; ++i) w.nm[i] = wl.nm[i];
    w.lo = wl.lo;
    w.hi = wl.hi;
    w.bins = wl.bins;
    w.tab = tab_dev;
    w.n_tab = n_tab;
    w.bin_scale = wl.mode == SC_WL_UNIFORM ? (float)wl.bins / (wl.hi - wl.lo) : 0.0f;
    w.channels = wl.mode == SC_WL_FIXED ? wl.k : wl.bins;
    return w;
}

double photon_scale(const Bvh* b, uint64_t N, const sc_wavelengths& wl) {
    const DevScene& S = b->scene;
    double nslot_min = wl.mode == SC_WL_FIXED ? (double)(N / wl.k) : (double)N / (double)wl.bins;
    if (nslot_min < 1.0) nslot_min = 1.0;
    const double bound = (double)b->max_power * (double)S.n_entries * 4.0 * M_PI * (double)S.n_tg / nslot_min;
    if (!(bound > 0.0) || N == 0) return 1.0;
    const double room = ldexp(1.0, 62) / ((double)N * bound);
    return ldexp(1.0, (int)floor(log2(room)));
}

namespace {

sc_status make_wave(Ctx* c, const sc_wavelengths& wl, WaveDev& w) {
    w = wave_view(wl, nullptr, 0);
    if (wl.mode == SC_WL_UNIFORM && c->sensor.p && c->sensor_lo == wl.lo && c->sensor_hi == wl.hi) {
        w.tab = c->sensor.as<float>();   // table of this range already on the device
        w.n_tab = c->sensor_n;
    } else if (wl.mode == SC_WL_UNIFORM) {
        std::vector<float> tab;
        const uint32_t n = sensor_table(wl, tab);
        SC_TRY(c->sensor.ensure(tab.size() * sizeof(float)));
        SC_HIP(hipMemcpyAsync(c->sensor.p, tab.data(), tab.size() * sizeof(float), hipMemcpyHostToDevice, c->stream));
        SC_HIP(hipStreamSynchronize(c->stream));   // tab is a host temporary
        w.tab = c->sensor.as<float>();
        w.n_tab = n;
        c->sensor_lo = wl.lo;
        c->sensor_hi = wl.hi;
        c->sensor_n = n;
    }
    return SC_OK;
}

}  // namespace

sc_status ctx_init(Ctx* c) {
    SC_TRY(c->counters.alloc(sizeof(DevCounters)));
    SC_TRY(c->work.alloc(sizeof(uint32_t) * kWorkSlots * kWorkStride));
    SC_HIP(hipMemsetAsync(c->counters.p, 0, sizeof(DevCounters), c->stream));
    SC_HIP(hipMemsetAsync(c->work.p, 0, sizeof(uint32_t) * kWorkSlots * kWorkStride, c->stream));
    SC_HIP(hipStreamSynchronize(c->stream));
    return SC_OK;
}

void ctx_release(Ctx* c) {
    for (auto& e : c->events) {
        (void)hipEventDestroy(e.first);
        (void)hipEventDestroy(e.second);
    }
    c->events.clear();
    for (auto& e : c->fin_events) {
        (void)hipEventDestroy(e.first);
        (void)hipEventDestroy(e.second);
    }
    c->fin_events.clear();
    for (auto* l : {&c->any_events, &c->cam_events}) {
        for (auto& e : *l) {
            (void)hipEventDestroy(e.first);
            (void)hipEventDestroy(e.second);
        }
        l->clear();
    }
    for (hipEvent_t e : c->event_pool) (void)hipEventDestroy(e);
    c->event_pool.clear();
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
        c->event_pool.push_back(e.first);
        c->event_pool.push_back(e.second);
    }
    c->events.clear();
    for (auto& e : c->fin_events) {
        float ms = 0.0f;
        SC_HIP(hipEventElapsedTime(&ms, e.first, e.second));
        c->finish_ms += ms;
        c->finish_launches += 1;
        c->event_pool.push_back(e.first);
        c->event_pool.push_back(e.second);
    }
    c->fin_events.clear();
    for (auto& e : c->any_events) {
        float ms = 0.0f;
        SC_HIP(hipEventElapsedTime(&ms, e.first, e.second));
        c->any_ms += ms;
        c->any_launches += 1;
        c->event_pool.push_back(e.first);
        c->event_pool.push_back(e.second);
    }
    c->any_events.clear();
    for (auto& e : c->cam_events) {
        float ms = 0.0f;
        SC_HIP(hipEventElapsedTime(&ms, e.first, e.second));
        c->cam_ms += ms;
        c->cam_launches += 1;
        c->event_pool.push_back(e.first);
        c->event_pool.push_back(e.second);
    }
    c->cam_events.clear();
    out->anyhit_launches = c->any_launches;
    out->anyhit_ms = c->any_ms;
    out->anyhit_rays = h.any_rays;
    out->anyhit_node_visits = h.any_nodes;
    out->anyhit_tri_tests = h.any_tris;
    out->cam_finish_launches = c->cam_launches;
    out->cam_finish_ms = c->cam_ms;
    out->cam_finish_paths = h.cf_paths;
    out->cam_finish_rays = h.cf_rays;
    out->cam_finish_shadow_rays = h.cf_shadow;
    out->cam_finish_node_visits = h.cf_nodes;
    out->cam_finish_tri_tests = h.cf_tris;
    out->finish_launches = c->finish_launches;
    out->finish_ms = c->finish_ms;
    out->finish_paths = h.fin_paths;
    out->finish_rays = h.fin_rays;
    out->finish_node_visits = h.fin_nodes;
    out->finish_tri_tests = h.fin_tris;
    out->rays_closest = h.rays_closest;
    out->rays_shadow = h.rays_shadow;
    out->node_visits = h.node_visits;
    out->tri_tests = h.tri_tests;
    out->closest_launches = c->closest_launches;
    out->closest_ms = c->closest_ms;
    out->closest_rays_timed = h.rays_staged;
    return SC_OK;
}

sc_status ctx_reset_counters(Ctx* c) {
    SC_HIP(hipStreamSynchronize(c->stream));
    SC_HIP(hipMemset(c->counters.p, 0, sizeof(DevCounters)));
    ctx_release(c);
    c->closest_ms = 0.0;
    c->closest_launches = 0;
    c->finish_ms = 0.0;
    c->finish_launches = 0;
    c->any_ms = 0.0;
    c->any_launches = 0;
    c->cam_ms = 0.0;
    c->cam_launches = 0;
    return SC_OK;
}

sc_status render(Ctx* c, Bvh* b, const sc_camera& cam, uint32_t spp, uint32_t max_depth, const sc_wavelengths& wl,
                 uint64_t seed, const float* cmap, const sc_aov& out, const PMapDev* pmap, hipEvent_t map_ready) {
    hipStream_t st = c->stream;
    PMapDev pm{};
    if (pmap) pm = *pmap;
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
    const bool want_aov = out.obj || out.trans || out.tri || out.depth || out.depthn || out.normal || out.normal_cam ||
                          out.albedo;
    // With an image too, the ground truth's pixel-centre rays are traced in
    // the first bounce's closest-hit launch (path slots n_max .. n_max + hw)
    // instead of a launch of their own, whose ramp and tail cost more than
    // its 1 ray per pixel.
    // bounces traced as one launch per stage (0: none, every path finished per lane)
    const uint32_t staged = std::min(c->staged_depth, max_depth);
    const bool merge_aov = want_aov && out.rgb && staged >= 1;
    const size_t n_cap = n_max + (merge_aov ? hw : 0);
    if (n_cap > 0xffffffffull) return set_error(SC_EUNSUPPORTED, "image too large for one wavefront chunk");
    SC_TRY(ensure_path(c, n_cap));
    SC_TRY(ensure_queues(c, n_cap));
    PathState P = carve_path(c->path.p, n_cap);
    Queues q = carve_queues(c->queues.p, n_cap);
    const uint32_t frame_words = (max_depth + 2) * QC_FRAME;
    SC_TRY(c->qcounts.ensure(4 * (size_t)frame_words));
    q.counts = c->qcounts.as<uint32_t>();
    reset_work(c);

    const RaySoA R{P.ox, P.oy, P.oz, P.dx, P.dy, P.dz};
    const HitSoA H{P.t, P.prim, P.u, P.v};
    const RaySoA Ra{P.ox + n_max, P.oy + n_max, P.oz + n_max, P.dx + n_max, P.dy + n_max, P.dz + n_max};
    const HitSoA Ha{P.t + n_max, P.prim + n_max, P.u + n_max, P.v + n_max};
    const uint32_t bs = 256;
    if (want_aov && !merge_aov) {
        hipLaunchKernelGGL(k_aov_raygen, dim3(grid_for(hw, bs)), dim3(bs), 0, st, cam, R, nullptr, 0u);
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
            hipLaunchKernelGGL(k_zero_u32, dim3(32), dim3(256), 0, st, q.counts, frame_words);
            const bool aov_here = merge_aov && s0 == 0;   // the ground truth joins the first bounce
            const uint32_t extra = aov_here ? (uint32_t)hw : 0u;
            hipLaunchKernelGGL(k_raygen, dim3(grid_for(n, bs)), dim3(bs), 0, st, ci, wd, P, n, q.cur, q.counts,
                               extra);
            if (aov_here)
                hipLaunchKernelGGL(k_aov_raygen, dim3(grid_for(hw, bs)), dim3(bs), 0, st, cam, Ra, q.cur + n,
                                   (uint32_t)n_max);
            uint32_t* cur = q.cur;
            uint32_t* nxt = q.next;
            for (uint32_t depth = 1; depth <= staged; ++depth) {
                uint32_t* fc = q.counts + (size_t)(depth - 1) * QC_FRAME;
                const uint32_t n_here = depth == 1 ? n + extra : n;
                launch_closest(c, S, R, H, cur, fc + QC_CUR, 0u, n_here);
                if (depth == 1 && aov_here)
                    hipLaunchKernelGGL(k_aov_write, dim3(grid_for(hw, bs)), dim3(bs), 0, st, S, cam, Ra, Ha, out);
                hipLaunchKernelGGL(k_classify, dim3(grid_for(n_here, bs)), dim3(bs), 0, st, S, P, cur, fc, q.diffuse,
                                   q.dielectric, (uint32_t)n_max);
                hipLaunchKernelGGL(k_shade_dielectric, dim3(grid_for(n, bs)), dim3(bs), 0, st, S, ci, P, depth,
                                   q.dielectric, fc, nxt);
                // the diffuse stage is the first reader of the caustic map;
                // everything before it may overlap the pass that writes it
                if (map_ready && s0 == 0 && depth == 1) SC_HIP(hipStreamWaitEvent(st, map_ready, 0));
                if (pm.on)
                    hipLaunchKernelGGL(k_shade_diffuse<true>, dim3(grid_for(n, bs)), dim3(bs), 0, st, S, ci, wd, P,
                                       depth, cmap, pm, q.diffuse, fc, nxt, q.shadow);
                else
                    hipLaunchKernelGGL(k_shade_diffuse<false>, dim3(grid_for(n, bs)), dim3(bs), 0, st, S, ci, wd, P,
                                       depth, cmap, pm, q.diffuse, fc, nxt, q.shadow);
                launch_anyhit(c, S, SR, q.shadow, fc + QC_SHADOW, 0u, n, nullptr, P.L);
                std::swap(cur, nxt);
            }
            if (staged < max_depth) {
                // with no staged bounce the finishing kernel is the map's first reader
                if (map_ready && s0 == 0 && staged == 0) SC_HIP(hipStreamWaitEvent(st, map_ready, 0));
                auto kfin = pm.on ? (c->count_visits ? k_finish_camera_pm<true> : k_finish_camera_pm<false>)
                                  : (c->count_visits ? k_finish_camera<false, true> : k_finish_camera<false, false>);
                uint32_t* work = next_work_slot(c);
                Timed tm(c, c->cam_events);
                hipLaunchKernelGGL(kfin, dim3(trace_grid(c, n)), dim3(kTraceBS), 0, st, S, ci, wd, P, cmap, pm, cur,
                                   q.counts + (size_t)staged * QC_FRAME + QC_CUR, staged + 1, work,
                                   c->counters.as<DevCounters>());
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
                        float* map, uint32_t* count_map, sc_photon_stats* stats, const PmRecords* rec) {
    hipStream_t st = c->stream;
    const DevScene& S = b->scene;
    WaveDev wd;
    SC_TRY(make_wave(c, wl, wd));
    // the general photon map keeps records instead of the receiver map
    const size_t cells = rec ? 0 : (size_t)S.recv_wc * S.recv_hc * wd.channels;
    const void* acc_before = c->acc64.p;
    SC_TRY(c->acc64.ensure(std::max<size_t>(cells, 1) * sizeof(unsigned long long)));
    if (c->acc64.p != acc_before) c->acc_clean = 0;   // fresh memory
    SC_TRY(c->touched.ensure((cells + 1) * sizeof(uint32_t)));
    const uint32_t bs = 256;
    // Passes with few photons per cell (a large map) keep the accumulator all
    // zero between passes: each clears the cells it touched, listed by the
    // deposits.  Passes with many photons per cell convert and clear the map
    // in full (streaming beats scattered access there).  Either way the map
    // is the same.  The accumulator is cleared in full after new memory, a
    // dense pass or a pass that did not finish.
    const bool sparse = cells > 8 * N;
    size_t clean_after = c->acc_clean;
    if (cells) {
        if (!sparse || c->acc_clean < cells) {
            hipLaunchKernelGGL(k_zero_u64, dim3(grid_for(cells, bs)), dim3(bs), 0, st,
                               c->acc64.as<unsigned long long>(), cells);
            clean_after = cells;
        }
        c->acc_clean = 0;
        if (sparse) {
            hipLaunchKernelGGL(k_zero_u32, dim3(1), dim3(64), 0, st, c->touched.as<uint32_t>(), 1u);
            // the float map is zero except at the cells the pass touches
            // (converted at the end); filled here, before the tracing, so the
            // fill does not queue behind another stream's persistent kernels
            // while they hold every compute unit (a 1080p frame's 268 MB fill
            // waited 3.4 ms behind its render's camera finishing)
            if (((uintptr_t)map & 15u) == 0)
                hipLaunchKernelGGL(k_zero_f32x4, dim3(grid_for(cells / 4, bs)), dim3(bs), 0, st,
                                   reinterpret_cast<float4*>(map), cells / 4);
            if (((uintptr_t)map & 15u) != 0 || cells % 4 != 0)
                hipLaunchKernelGGL(k_zero_f32, dim3(grid_for(cells, bs)), dim3(bs), 0, st, map, cells);
        }
    }
    if (count_map && cells)
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
        // fixed-point scale from a bound on one photon's flux (strongest
        // light, all entries, every cone a full sphere, smallest slot)
        scale = photon_scale(b, N, wl);
        const size_t chunk = std::min<uint64_t>(N, c->photon_cap);
        if (c->photon_n < chunk || !c->photon.p) {
            SC_TRY(c->photon.alloc(photon_bytes(chunk)));
            c->photon_n = chunk;
        }
        SC_TRY(ensure_queues(c, chunk));
        PhotonState Ph = carve_photon(c->photon.p, chunk);
        Queues q = carve_queues(c->queues.p, chunk);
        const uint32_t frame_words = (max_depth + 2) * QC_FRAME;
        SC_TRY(c->qcounts.ensure(4 * (size_t)frame_words));
        q.counts = c->qcounts.as<uint32_t>();
        reset_work(c);
        const RaySoA R{Ph.ox, Ph.oy, Ph.oz, Ph.dx, Ph.dy, Ph.dz};
        const HitSoA H{Ph.t, Ph.prim, Ph.u, Ph.v};
        for (uint64_t p0 = 0; p0 < N; p0 += chunk) {
            const uint32_t n = (uint32_t)std::min<uint64_t>(chunk, N - p0);
            PhInfo pi{seed, N, p0, max_depth, scale, stats ? 1 : 0, rec ? 1 : 0, rec ? *rec : PmRecords{},
                      cells && sparse ? c->touched.as<uint32_t>() : nullptr};
            hipLaunchKernelGGL(k_zero_u32, dim3(32), dim3(256), 0, st, q.counts, frame_words);
            hipLaunchKernelGGL(k_photon_emit, dim3(grid_for(n, bs)), dim3(bs), 0, st, S, wd, pi, n, Ph, q.cur, q.counts,
                               c->counters.as<DevCounters>());
            uint32_t* cur = q.cur;
            uint32_t* nxt = q.next;
            const uint32_t staged = std::min(c->photon_staged_depth, max_depth);   // 0: none
            for (uint32_t depth = 1; depth <= staged; ++depth) {
                uint32_t* fc = q.counts + (size_t)(depth - 1) * QC_FRAME;
                launch_closest(c, S, R, H, cur, fc + QC_CUR, 0u, n);
                hipLaunchKernelGGL(k_photon_event, dim3(grid_for(n, bs)), dim3(bs), 0, st, S, wd, pi, depth, Ph, cur,
                                   fc, nxt, c->acc64.as<unsigned long long>(), count_map,
                                   c->counters.as<DevCounters>());
                std::swap(cur, nxt);
            }
            if (staged < max_depth) {
                hipEvent_t e0 = nullptr, e1 = nullptr;
                if (c->profile) {
                    e0 = pooled_event(c);
                    e1 = pooled_event(c);
                    (void)hipEventRecord(e0, st);
                }
                uint32_t* fcount = q.counts + (size_t)staged * QC_FRAME + QC_CUR;
                if (c->count_visits)
                    hipLaunchKernelGGL(k_finish_photons<true>, dim3(trace_grid(c, n)), dim3(kTraceBS), 0, st, S, wd, pi,
                                       staged + 1, Ph, cur, fcount, next_work_slot(c),
                                       c->acc64.as<unsigned long long>(), count_map, c->counters.as<DevCounters>());
                else
                    hipLaunchKernelGGL(k_finish_photons<false>, dim3(trace_grid(c, n)), dim3(kTraceBS), 0, st, S, wd,
                                       pi, staged + 1, Ph, cur, fcount, next_work_slot(c),
                                       c->acc64.as<unsigned long long>(), count_map, c->counters.as<DevCounters>());
                if (c->profile) {
                    (void)hipEventRecord(e1, st);
                    c->fin_events.emplace_back(e0, e1);
                }
            }
        }
    }
    if (cells && !sparse) {
        hipLaunchKernelGGL(k_map_finalize_all, dim3(grid_for(cells, bs)), dim3(bs), 0, st,
                           c->acc64.as<unsigned long long>(), cells, 1.0 / scale, map);
        clean_after = 0;
    } else if (cells) {
        hipLaunchKernelGGL(k_map_finalize, dim3(grid_for(std::min<size_t>(cells, N), bs)), dim3(bs), 0, st,
                           c->touched.as<uint32_t>(), c->acc64.as<unsigned long long>(), 1.0 / scale, map);
    }
    SC_HIP(hipGetLastError());
    if (cells) c->acc_clean = clean_after;
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

// ------------------------------------------------------------------
// Closest hit without allocation.  The rays are staged into a fixed,
// file-scope device array (one copy per GPU, held until the process
// ends) instead of the context's grow-only buffer; the traversal kernel is
// k_closest, as in trace_rays.  Host code uses the array only through the
// address hipGetSymbolAddress returns on each device.
constexpr uint32_t kNoAllocMaxRays = 1u << 20;
constexpr size_t kNoAllocArray = (size_t)kNoAllocMaxRays * 4 + 256;   // one SoA array, 256-byte aligned
constexpr int kNoAllocMaxDevices = 64;
__device__ __align__(256) unsigned char scratch[6 * kNoAllocArray];
std::mutex g_scratch_mu;
void* g_scratch_ptr[kNoAllocMaxDevices] = {};

// With `device` current: look up this device's copy of the array (once).
sc_status scratch_init(int device) {
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (device < 0 || device >= kNoAllocMaxDevices) return set_error(SC_EUNSUPPORTED, "device index beyond 63");
    if (g_scratch_ptr[device]) return SC_OK;
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
        (void)hipGetLastError();
        return set_error(SC_EDEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    }
    g_scratch_ptr[device] = p;
    return SC_OK;
}

uint32_t trace_rays_noalloc_max() { return kNoAllocMaxRays; }

sc_status trace_rays_noalloc(Ctx* c, Bvh* b, uint32_t n, const float* O, const float* D, float* t, uint32_t* prim,
                             float* u, float* v) {
    if (n > kNoAllocMaxRays)
        return set_error(SC_EINVAL, "n = " + std::to_string(n) + " rays exceeds the allocation-free maximum of " +
                                        std::to_string(kNoAllocMaxRays));
    void* base = nullptr;
    {
        std::lock_guard<std::mutex> lock(g_scratch_mu);
        if (c->device >= 0 && c->device < kNoAllocMaxDevices) base = g_scratch_ptr[c->device];
    }
    if (!base) return set_error(SC_EDEVICE, "no scratch address for the context's device");
    Carver cv{static_cast<char*>(base)};
    float* ox = cv.take<float>(kNoAllocMaxRays); float* oy = cv.take<float>(kNoAllocMaxRays);
    float* oz = cv.take<float>(kNoAllocMaxRays); float* dx = cv.take<float>(kNoAllocMaxRays);
    float* dy = cv.take<float>(kNoAllocMaxRays); float* dz = cv.take<float>(kNoAllocMaxRays);
    const RaySoA R{ox, oy, oz, dx, dy, dz};
    const ShadowSoA none{};
    // every staged entry [0, n) is written before it is read; nothing in the
    // array has to start at zero
    hipLaunchKernelGGL(k_rays_from_aos, dim3(grid_for(n, 256)), dim3(256), 0, c->stream, O, D, n, R, nullptr, nullptr,
                       none);
    reset_work(c);
    uint32_t* work = next_work_slot(c);
    hipLaunchKernelGGL(k_closest<false>, dim3(trace_grid(c, n)), dim3(kTraceBS), 0, c->stream, b->scene, R,
                       HitSoA{t, prim, u, v}, nullptr, nullptr, n, work, c->counters.as<DevCounters>());
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
