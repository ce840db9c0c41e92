// sc_kernels.h -- ray buffer views used by the traversal kernels and the
// entry points of the wavefront passes.
#pragma once
#include <stdint.h>

#include <vector>

#include "sc_internal.h"
#include "sc_types.h"

// maximum traversal stack entries per ray (LDS part plus scratch spill)
constexpr int kMaxStack = 160;

struct RaySoA {
    float *ox, *oy, *oz, *dx, *dy, *dz;
};
struct HitSoA {
    float* t;
    uint32_t* prim;
    float *u, *v;
};
struct ShadowSoA {
    float *ox, *oy, *oz, *dx, *dy, *dz;
    float* tmax;
    uint32_t* excl;
    float* contrib;
};

namespace scl {

// pmap: general photon map for the caustic gather, or null (receiver map cmap)
// map_ready: an event the stream waits for before the first kernel that
// reads cmap (the photon pass that writes it may run on another stream)
sc_status render(Ctx* c, Bvh* b, const sc_camera& cam, uint32_t spp, uint32_t max_depth, const sc_wavelengths& wl,
                 uint64_t seed, const float* cmap, const sc_aov& out, const PMapDev* pmap = nullptr,
                 hipEvent_t map_ready = nullptr);
// rec: records of a general photon map (deposits on every diffuse surface),
// or null (receiver map)
sc_status trace_photons(Ctx* c, Bvh* b, uint64_t n_photons, uint32_t max_depth, const sc_wavelengths& wl,
                        uint64_t seed, float* map, uint32_t* count_map, sc_photon_stats* stats,
                        const PmRecords* rec = nullptr);
// allocation-free closest hit: rays staged in a fixed per-device array
sc_status scratch_init(int device);
uint32_t trace_rays_noalloc_max();
sc_status trace_rays_noalloc(Ctx* c, Bvh* b, uint32_t n, const float* O, const float* D, float* t, uint32_t* prim,
                             float* u, float* v);
sc_status pmap_trace(Ctx* c, Bvh* b, uint64_t n_photons, uint32_t max_depth, const sc_wavelengths& wl, uint64_t seed,
                     float radius, Pmap* pm, sc_photon_stats* stats);
sc_status pmap_export(const Pmap* pm, float* pos, float* nrm, float* phi, uint32_t* channel, uint64_t* photon);
sc_status pmap_gather(Ctx* c, const Pmap* pm, uint32_t n, const float* P, const float* N, const uint32_t* ch, float* E);
sc_status trace_rays(Ctx* c, Bvh* b, uint32_t n, const float* O, const float* D, float* t, uint32_t* prim, float* u,
                     float* v);
sc_status occluded(Ctx* c, Bvh* b, uint32_t n, const float* O, const float* D, const float* tmax,
                   const uint32_t* excl, uint8_t* occ);
uint32_t sensor_table(const sc_wavelengths& wl, std::vector<float>& tab);
WaveDev wave_view(const sc_wavelengths& wl, const float* tab_dev, uint32_t n_tab);
double photon_scale(const Bvh* b, uint64_t n_photons, const sc_wavelengths& wl);
sc_status ctx_counters(Ctx* c, sc_counters* out);
sc_status ctx_reset_counters(Ctx* c);
sc_status ctx_init(Ctx* c);
void ctx_release(Ctx* c);

}  // namespace scl
