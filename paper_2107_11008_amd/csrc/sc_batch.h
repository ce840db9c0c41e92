// sc_batch.h -- host and device structures of the batched persistent launch.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "sc_internal.h"

// one scene of a batch, as the persistent kernels see it
struct BatchScene {
    DevScene S;
    sc_camera cam;
    WaveDev wl;
    uint64_t seed, photon_seed, n_photons;
    uint32_t spp, max_depth, K, hw;
    uint32_t item_begin, ph_item_begin;   // first pixel / photon work item
    unsigned long long* acc;              // fixed-point caustic accumulator
    size_t cells;
    float* cmap;                          // caustic map written by the photon pass and gathered
    double scale;
    sc_aov out;
};

namespace scl {

struct Batch {
    Ctx* ctx = nullptr;
    sc_tune tune{};
    uint32_t n = 0, ph_items = 0, px_items = 0, grid = 0, zero_grid = 1;
    DevBuf scenes, acc, maps, tabs, work;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    void launch(hipStream_t st);
    ~Batch();
};

sc_status batch_create(Ctx* c, uint32_t n, const sc_batch_item* items, const sc_tune& tune, Batch* bt);
sc_status batch_run(Batch* bt);

}  // namespace scl
