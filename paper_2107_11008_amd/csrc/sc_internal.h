// sc_internal.h -- host-side objects of the library (context, BVH handle,
// device buffers, error reporting).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <set>
#include <string>
#include <utility>
#include <vector>

#include "sc_types.h"

namespace scl {

sc_status set_error(sc_status code, const std::string& msg);

// RAII device allocation
struct DevBuf {
    void* p = nullptr;
    size_t bytes = 0;
    DevBuf() = default;
    DevBuf(const DevBuf&) = delete;
    DevBuf& operator=(const DevBuf&) = delete;
    ~DevBuf() { release(); }
    void release() {
        if (p) (void)hipFree(p);
        p = nullptr;
        bytes = 0;
    }
    sc_status alloc(size_t n) {
        release();
        if (n == 0) n = 16;
        if (hipMalloc(&p, n) != hipSuccess) {
            (void)hipGetLastError();
            p = nullptr;
            return set_error(SC_ENOMEM, "hipMalloc of " + std::to_string(n) + " bytes failed");
        }
        bytes = n;
        return SC_OK;
    }
    // grow-only
    sc_status ensure(size_t n) {
        if (n <= bytes && p) return SC_OK;
        return alloc(n);
    }
    template <class T>
    T* as() const {
        return static_cast<T*>(p);
    }
};

// Sub-allocation of one device buffer into 256-byte aligned arrays
// (base == nullptr only measures: off is then the bytes needed).
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

#define SC_TRY(expr)                      \
    do {                                  \
        sc_status _s = (expr);            \
        if (_s != SC_OK) return _s;       \
    } while (0)

#define SC_HIP(expr)                                                                               \
    do {                                                                                           \
        hipError_t _e = (expr);                                                                    \
        if (_e != hipSuccess)                                                                      \
            return ::scl::set_error(SC_EDEVICE, std::string(#expr) + ": " + hipGetErrorString(_e)); \
    } while (0)

struct Ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    bool count_visits = false;
    bool profile = false;
    // camera paths per wavefront chunk: all 64 samples of a 1080p frame
    // (132.7 M paths, ~17 GB of path state and queues) run as one chunk, so
    // the staged launches are large and the per-lane finishing tail is paid
    // once per frame (large scene: 2^23 / 2^24 / 2^25 / 2^26 / 2^27 paths
    // per chunk gave 257.6 / 218.5 / 205.5 / 196.8 / 190.6 ms per step)
    uint64_t queue_cap = 1ull << 27;
    uint32_t cus = 256;          // compute units of the device (sizes persistent grids)
    // camera bounces run as separate launches before the paths are finished
    // per lane (large scene, 1 / 2 / 3 / 4 staged bounces: 1080p 64-spp step
    // 148.1 / 151.1 / 153.6 ms at 2 / 3 / 4; plain 64-spp frame 118.6 /
    // 113.1 / 115.2 / 118.2 ms; medium step 10.8 / 11.0 / 11.3 ms at 2 / 3 / 4)
    uint32_t staged_depth = 2;
    uint32_t photon_staged_depth = 0;   // the same for photon paths (none: every photon finished per lane)
    uint64_t conv_big_tile = 2048;   // 16-row U-Net convolution tiles needed before they are used
    // photons per photon-pass chunk (2^24 photons of the large scene in one
    // chunk: 34.8 / 29.8 / 27.5 ms per pass at 2^22 / 2^23 / 2^24; ~1.5 GB)
    uint64_t photon_cap = 1ull << 24;
    uint32_t bvh_builder = 2;   // 0: radix tree over Morton codes, 1: locally-ordered clustering, 2: by size
    uint32_t trace_blocks = 8;  // blocks of 128 threads per CU in the persistent traversal grids
    DevBuf counters;   // DevCounters
    DevBuf work;       // per-launch work counters of the traversal kernels
    uint32_t work_slot = 0;
    DevBuf path;       // PathState arrays
    size_t path_n = 0;
    DevBuf queues;     // five queues
    size_t queue_n = 0;
    DevBuf qcounts;    // queue counter frames, one per bounce depth
    DevBuf photon;     // PhotonState arrays
    size_t photon_n = 0;
    DevBuf acc64;      // fixed-point caustic accumulator
    size_t acc_clean = 0;   // leading entries of acc64 known to be zero
    DevBuf touched;    // cells a photon pass made non-zero (count first)
    DevBuf sensor;     // sensor curve table of the range [sensor_lo, sensor_hi]
    float sensor_lo = -1.0f, sensor_hi = -1.0f;
    uint32_t sensor_n = 0;
    DevBuf aos;        // SoA copies for sc_trace_rays / sc_occluded
    DevBuf bvh_tmp;    // temporaries of the BVH builder (grow-only, reused)
    DevBuf pm_rec;     // records of a general photon map pass (grow-only)
    DevBuf pm_tmp;     // bucket ids, counts, cursors and scan sums of the photon map build
    size_t aos_n = 0;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> events;   // recorded, not yet read
    std::vector<hipEvent_t> event_pool;                       // read, free for reuse
    double closest_ms = 0.0;
    uint64_t closest_launches = 0;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> fin_events;   // photon finishing launches, not yet read
    double finish_ms = 0.0;
    uint64_t finish_launches = 0;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> any_events;   // any-hit launches, not yet read
    double any_ms = 0.0;
    uint64_t any_launches = 0;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> cam_events;   // camera path finishing launches, not yet read
    double cam_ms = 0.0;
    uint64_t cam_launches = 0;
    // the context pointers of the handles (BVH, photon map, U-Net, batch)
    // made on this context: cleared when it is destroyed, so a handle freed
    // after its context does not touch it
    std::set<Ctx**> handles;
};

// record that the handle whose context pointer is *slot belongs to c
inline void attach(Ctx* c, Ctx** slot) {
    if (*slot && *slot != c) (*slot)->handles.erase(slot);
    *slot = c;
    if (c) c->handles.insert(slot);
}
// the handle is being freed: its context forgets it
inline void detach(Ctx** slot) {
    if (*slot) (*slot)->handles.erase(slot);
    *slot = nullptr;
}

struct Bvh {
    Ctx* ctx = nullptr;
    sc_scene scene_in{};          // copy of the caller's description (pointers borrowed)
    DevScene scene{};             // device view
    DevBuf nodes, tris, mat, pl, tg, emit_prim, emit_cdf;
    uint32_t n_nodes = 0, depth = 0, width = 8, leaf_max = 4, max_stack = 0;
    // strongest light power (point intensity or emitted radiance x area)
    float max_power = 0.0f;
};

// A general photon map: stored photons counting-sorted into hash buckets.
struct Pmap {
    Ctx* ctx = nullptr;
    DevBuf mem;                              // sorted records and bucket starts
    PMapDev dev{};                           // device view
    const float* phi = nullptr;              // sorted fluxes (export)
    const uint32_t* ch = nullptr;            // sorted channels (export)
    const unsigned long long* photon = nullptr;   // sorted photon indices (export)
    uint64_t n = 0;
    float radius = 0.0f;
    uint32_t channels = 0, buckets = 0;
    double scale = 1.0;
    bool valid = false;                      // false after a failed rebuild
};

// Builds b->nodes and b->tris for b->scene_in (b->mat must already hold the
// materials on the device).  Also returns the emissive triangles in index
// order with their vertices (9 floats each).  Synchronises the stream.
sc_status build_wide_bvh(Ctx* ctx, Bvh* b, uint32_t width, uint32_t leaf_max, std::vector<uint32_t>& emit_prim,
                         std::vector<float>& emit_v);

}  // namespace scl

struct sc_ctx {
    scl::Ctx c;
};
struct sc_bvh {
    scl::Bvh b;
};
struct sc_pmap {
    scl::Pmap p;
};
