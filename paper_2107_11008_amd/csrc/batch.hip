// batch.hip -- many scenes in one persistent launch.
//
// A batch of scenes of uneven size is rendered by two persistent kernels:
// waves pull work items -- 64*m photons or 64*m pixels of one scene -- from
// a global counter, and each lane follows its photon or its pixel's paths
// (all samples and wavelength slots, then the ground-truth ray) to the end
// with the same per-path device functions the wavefront kernels use, so the
// images, masks and caustic maps equal the one-scene-at-a-time results.
// The whole batch (clears, photons, map conversion, rendering) is captured
// once in a hipGraph and replayed.
#pragma clang fp contract(off)
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>
#include <string>
#include <vector>

#include "sc_batch.h"
#include "sc_kernels.h"
#include "sc_path.h"

using namespace scd;

namespace {

// scene containing work item `item` (items of scene s start at begin[s])
__device__ __forceinline__ uint32_t scene_of(const BatchScene* __restrict__ B, uint32_t n, uint32_t item, bool photons) {
    uint32_t lo = 0, hi = n - 1;
    while (lo < hi) {
        const uint32_t mid = (lo + hi + 1) >> 1;
        const uint32_t b = photons ? B[mid].ph_item_begin : B[mid].item_begin;
        if (b <= item) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// lanes of the wave below this one in mask m
__device__ __forceinline__ uint32_t below(unsigned long long m) {
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

constexpr uint32_t kBatchEvents = 32;   // pending photon events that are run together

// A wave takes one work item (per_item photons of one scene) at a time.
// Within it a lane whose photon has ended takes the item's next photon; the
// traversal of every lane advances one step per loop turn and the photon
// events run together once kBatchEvents lanes have one pending (or no lane
// is tracing), so no lane waits for the longest path of its wave.  Every
// photon's arithmetic is that of photon_continue; deposits are integer
// atomics, so the map does not depend on the schedule.
template <int BS>
__global__ __launch_bounds__(BS) __attribute__((amdgpu_waves_per_eu(4))) void k_batch_photons(
    const BatchScene* __restrict__ B, uint32_t n_scenes, uint32_t n_items, uint32_t per_item, uint32_t* work) {
    __shared__ uint2 lds[kLdsStack][BS];
    Spill st;
    VisitCount vc;
    const uint32_t lane = __lane_id();
    for (;;) {
        uint32_t item = 0;
        if (lane == 0) item = atomicAdd(work, 1u);
        item = __shfl(item, 0);
        if (item >= n_items) break;
        const uint32_t s = scene_of(B, n_scenes, item, true);
        const BatchScene& bs = B[s];
        const uint64_t first = (uint64_t)(item - bs.ph_item_begin) * per_item;
        const uint64_t left = first < bs.n_photons ? bs.n_photons - first : 0ull;
        const uint32_t count = left < per_item ? (uint32_t)left : per_item;
        uint32_t next = 0;   // the item's next photon (the same in every lane)
        uint32_t state = 0;  // 0 idle, 1 tracing, 2 hit found and its event pending
        uint32_t depth = 0;
        uint64_t p = 0;
        PhotonPath ph;
        Trav t;
        for (;;) {
            const unsigned long long idle = __ballot(state == 0);
            if (idle != 0ull && next < count) {
                const uint32_t k = next + below(idle);
                next = min(count, next + (uint32_t)__popcll(idle));
                if (state == 0 && k < count) {
                    p = first + k;
                    if (photon_emit(bs.S, bs.wl, bs.photon_seed, bs.n_photons, p, ph)) {
                        depth = 1;
                        trav_init(t, ph.o, ph.d);
                        state = 1;
                    }
                }
            }
            if (__ballot(state != 0) == 0ull) {
                if (next >= count) break;
                continue;
            }
            if (state == 1 && trav_step<BS, false>(bs.S, t, lds, st, vc)) state = 2;
            const unsigned long long pend = __ballot(state == 2);
            if (pend == 0ull || ((uint32_t)__popcll(pend) < kBatchEvents && __ballot(state == 1) != 0ull)) continue;
            if (state != 2) continue;
            // one interaction, as in photon_continue
            const HitRec h = trav_result(t);
            int outcome = -1;
            Deposit dp;
            const bool cont =
                photon_event(bs.S, bs.wl, bs.photon_seed, p, depth, bs.max_depth, false, h, ph, outcome, dp);
            if (dp.cell_ch >= 0) atomicAdd(&bs.acc[dp.cell_ch], __double2ull_rn((double)ph.phi * bs.scale));
            if (cont && depth < bs.max_depth) {
                ++depth;
                trav_init(t, ph.o, ph.d);
                state = 1;
            } else {
                state = 0;
            }
        }
    }
}

template <int BS>
__global__ __launch_bounds__(BS) void k_batch_render(const BatchScene* __restrict__ B, uint32_t n_scenes,
                                                     uint32_t n_items, uint32_t per_item, uint32_t* work) {
    __shared__ uint2 lds[kLdsStack][BS];
    Spill st;
    VisitCount vc;
    const uint32_t lane = __lane_id();
    for (;;) {
        uint32_t item = 0;
        if (lane == 0) item = atomicAdd(work, 1u);
        item = __shfl(item, 0);
        if (item >= n_items) break;
        const uint32_t s = scene_of(B, n_scenes, item, false);
        const BatchScene& bs = B[s];
        const uint32_t first = (item - bs.item_begin) * per_item;
        for (uint32_t j = lane; j < per_item; j += 64) {
            const uint32_t pix = first + j;
            if (pix >= bs.hw) break;
            if (bs.out.rgb) {
                float acc[3] = {0.0f, 0.0f, 0.0f};
                for (uint32_t sample = 0; sample < bs.spp; ++sample) {
                    for (uint32_t slot = 0; slot < bs.K; ++slot) {
                        CamPath P = camera_start(bs.cam, bs.wl, bs.seed, pix, sample, slot);
                        uint32_t n_cl = 0, n_sh = 0;
                        camera_continue<BS, false>(bs.S, bs.wl, bs.cmap, PMapDev{}, bs.seed, pix, sample, slot, 1,
                                                   bs.max_depth, P, lds, st, vc, n_cl, n_sh);
                        film_add(bs.wl, bs.K, slot, P.L, P.lam, acc);
                    }
                }
                const float inv_spp = 1.0f / (float)bs.spp;
                bs.out.rgb[3 * (size_t)pix] = acc[0] * inv_spp;
                bs.out.rgb[3 * (size_t)pix + 1] = acc[1] * inv_spp;
                bs.out.rgb[3 * (size_t)pix + 2] = acc[2] * inv_spp;
            }
            // ground truth of the pixel-centre ray
            F3 o, d;
            camera_ray(bs.cam, pix % bs.cam.w, pix / bs.cam.w, 0.5f, 0.5f, o, d);
            const HitRec h = trace_closest<BS, false>(bs.S, o, d, lds, st, vc);
            aov_write(bs.S, bs.cam, pix, d, h, bs.out);
        }
    }
}

__global__ void k_batch_zero(const BatchScene* __restrict__ B, uint32_t* work) {
    const BatchScene& bs = B[blockIdx.y];
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < bs.cells; i += (size_t)gridDim.x * blockDim.x)
        bs.acc[i] = 0ull;
    if (blockIdx.x == 0 && blockIdx.y == 0 && threadIdx.x < 2) work[threadIdx.x] = 0u;
}

__global__ void k_batch_finalize(const BatchScene* __restrict__ B) {
    const BatchScene& bs = B[blockIdx.y];
    if (!bs.n_photons) return;
    const double inv = 1.0 / bs.scale;
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < bs.cells; i += (size_t)gridDim.x * blockDim.x)
        bs.cmap[i] = (float)((double)bs.acc[i] * inv);
}

template <int BS>
void launch_all(hipStream_t st, const BatchScene* dB, uint32_t n, uint32_t ph_items, uint32_t px_items,
                uint32_t per_ph, uint32_t per_px, uint32_t* work, uint32_t grid, uint32_t zero_grid) {
    hipLaunchKernelGGL(k_batch_zero, dim3(zero_grid, n), dim3(256), 0, st, dB, work);
    if (ph_items)
        hipLaunchKernelGGL(k_batch_photons<BS>, dim3(grid), dim3(BS), 0, st, dB, n, ph_items, per_ph, work);
    hipLaunchKernelGGL(k_batch_finalize, dim3(zero_grid, n), dim3(256), 0, st, dB);
    hipLaunchKernelGGL(k_batch_render<BS>, dim3(grid), dim3(BS), 0, st, dB, n, px_items, per_px, work + 1);
}

}  // namespace

namespace scl {

sc_status batch_create(Ctx* c, uint32_t n, const sc_batch_item* items, const sc_tune& tune, Batch* bt) {
    scl::attach(c, &bt->ctx);
    bt->tune = tune;
    bt->n = n;
    std::vector<BatchScene> hs(n);
    uint32_t ph_items = 0, px_items = 0;
    const uint32_t per = tune.px_per_item;
    const uint32_t per_ph = tune.ph_per_item ? tune.ph_per_item : tune.px_per_item;
    size_t acc_total = 0, map_total = 0, tab_total = 0;
    std::vector<std::vector<float>> tabs(n);
    std::vector<uint32_t> ntab(n, 0);
    for (uint32_t i = 0; i < n; ++i) {
        const sc_batch_item& it = items[i];
        const Bvh* b = &it.bvh->b;
        const DevScene& S = b->scene;
        const uint32_t C = it.wl.mode == SC_WL_FIXED ? it.wl.k : it.wl.bins;
        const size_t cells = S.recv_obj ? (size_t)S.recv_wc * S.recv_hc * C : 0;
        if (it.n_photons && !S.recv_obj) return set_error(SC_EINVAL, "batch item " + std::to_string(i) + ": photons need a receiver");
        acc_total += it.n_photons ? cells : 0;
        map_total += (it.n_photons && !it.caustic_map) ? cells : 0;
        if (it.wl.mode == SC_WL_UNIFORM) {
            ntab[i] = sensor_table(it.wl, tabs[i]);
            tab_total += tabs[i].size();
        }
    }
    SC_TRY(bt->acc.alloc(8 * std::max<size_t>(acc_total, 1)));
    SC_TRY(bt->maps.alloc(4 * std::max<size_t>(map_total, 1)));
    SC_TRY(bt->tabs.alloc(4 * std::max<size_t>(tab_total, 1)));
    SC_TRY(bt->work.alloc(64));
    size_t acc_off = 0, map_off = 0, tab_off = 0;
    size_t max_cells = 1;
    for (uint32_t i = 0; i < n; ++i) {
        const sc_batch_item& it = items[i];
        const Bvh* b = &it.bvh->b;
        BatchScene& B = hs[i];
        B.S = b->scene;
        B.cam = it.cam;
        const float* tab_dev = nullptr;
        if (ntab[i]) {
            SC_HIP(hipMemcpy(bt->tabs.as<float>() + tab_off, tabs[i].data(), 4 * tabs[i].size(), hipMemcpyHostToDevice));
            tab_dev = bt->tabs.as<float>() + tab_off;
            tab_off += tabs[i].size();
        }
        B.wl = wave_view(it.wl, tab_dev, ntab[i]);
        B.seed = it.seed;
        B.photon_seed = it.photon_seed;
        B.n_photons = it.n_photons;
        B.spp = it.spp;
        B.max_depth = it.max_depth;
        B.K = it.wl.mode == SC_WL_FIXED ? it.wl.k : 1;
        B.hw = it.cam.w * it.cam.h;
        B.item_begin = px_items;
        px_items += (B.hw + per - 1) / per;
        B.ph_item_begin = ph_items;
        ph_items += (uint32_t)((it.n_photons + per_ph - 1) / per_ph);
        const size_t cells = B.S.recv_obj ? (size_t)B.S.recv_wc * B.S.recv_hc * B.wl.channels : 0;
        B.cells = it.n_photons ? cells : 0;
        B.acc = bt->acc.as<unsigned long long>() + acc_off;
        acc_off += B.cells;
        max_cells = std::max(max_cells, B.cells);
        if (it.n_photons) {
            B.cmap = it.caustic_map ? it.caustic_map : bt->maps.as<float>() + map_off;
            if (!it.caustic_map) map_off += cells;
        } else {
            B.cmap = const_cast<float*>(it.caustic_map);   // gather from a given map, or off
        }
        B.scale = it.n_photons ? photon_scale(b, it.n_photons, it.wl) : 1.0;
        B.out = it.out;
    }
    SC_TRY(bt->scenes.alloc(sizeof(BatchScene) * n));
    SC_HIP(hipMemcpy(bt->scenes.p, hs.data(), sizeof(BatchScene) * n, hipMemcpyHostToDevice));
    bt->ph_items = ph_items;
    bt->px_items = px_items;
    bt->zero_grid = (uint32_t)std::min<size_t>(1024, (max_cells + 255) / 256);
    int cus = 256;
    (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, c->device);
    bt->grid = (uint32_t)cus * tune.blocks_per_cu;
    if (tune.use_graph) {
        // capture on a private stream (the null stream cannot be captured);
        // the graph is launched on the context's stream
        hipStream_t cap = nullptr;
        SC_HIP(hipStreamCreateWithFlags(&cap, hipStreamNonBlocking));
        hipError_t e0 = hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal);
        if (e0 == hipSuccess) {
            bt->launch(cap);
            hipGraph_t g = nullptr;
            e0 = hipStreamEndCapture(cap, &g);
            bt->graph = g;
        }
        (void)hipStreamDestroy(cap);
        if (e0 != hipSuccess) return set_error(SC_EDEVICE, std::string("graph capture: ") + hipGetErrorString(e0));
        SC_HIP(hipGraphInstantiate(&bt->exec, bt->graph, nullptr, nullptr, 0));
    }
    return SC_OK;
}

void Batch::launch(hipStream_t st) {
    const BatchScene* dB = scenes.as<BatchScene>();
    uint32_t* w = work.as<uint32_t>();
    const uint32_t per_ph = tune.ph_per_item ? tune.ph_per_item : tune.px_per_item;
    switch (tune.block_size) {
        case 64: launch_all<64>(st, dB, n, ph_items, px_items, per_ph, tune.px_per_item, w, grid, zero_grid); break;
        case 128: launch_all<128>(st, dB, n, ph_items, px_items, per_ph, tune.px_per_item, w, grid, zero_grid); break;
        default: launch_all<256>(st, dB, n, ph_items, px_items, per_ph, tune.px_per_item, w, grid, zero_grid); break;
    }
}

sc_status batch_run(Batch* bt) {
    hipStream_t st = bt->ctx->stream;
    if (bt->exec) {
        SC_HIP(hipGraphLaunch(bt->exec, st));
    } else {
        bt->launch(st);
        SC_HIP(hipGetLastError());
    }
    return SC_OK;
}

Batch::~Batch() {
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
}

}  // namespace scl
