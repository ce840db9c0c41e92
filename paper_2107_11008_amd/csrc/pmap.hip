// pmap.hip -- the general photon map: caustic photons stored at their first
// diffuse hit on any object (Sec. III-D-6: caustic light on whatever
// surface lies behind the glass), kept in a hashed grid for a fixed-radius
// disc density estimate (Jensen, "Global Illumination using Photon Maps",
// EGWR 1996).
//
// Build: the photon pass appends records (position, normal on the
// photon's side, flux, channel, photon index); their count, largest flux
// and largest coordinate fix the fixed-point scale 2^S (the largest power
// of two with n * max(phi) * 2^S <= 2^62) and check the grid's range.
// Records are then counting-sorted into buckets of (cell, channel), cells
// 2.25 r wide: a bucket count, a three-phase exclusive scan and a scatter.
// The order inside a bucket is whatever the atomics give; the gather sums
// integers, so it does not matter.
#include <hip/hip_runtime.h>
#include <float.h>
#include <math.h>
#include <stdint.h>
#include <string.h>

#include <algorithm>
#include <numeric>
#include <vector>

#include "sc_device.h"
#include "sc_internal.h"
#include "sc_kernels.h"
#include "sc_path.h"

using namespace scd;

namespace {

constexpr uint32_t kScanBlock = 1024;   // counts per scan block (256 threads x 4)

__global__ void k_pm_zero(uint32_t* p, size_t n) {
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) p[i] = 0u;
}

__global__ void k_pm_bucket(PmRecords R, uint32_t n, float inv_h, uint32_t cbits, uint32_t mask,
                            uint32_t* __restrict__ bucket, uint32_t* __restrict__ counts) {
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        const uint32_t b = pm_bucket(pm_cell(R.px[i], inv_h), pm_cell(R.py[i], inv_h), pm_cell(R.pz[i], inv_h), R.ch[i],
                                     cbits, mask);
        bucket[i] = b;
        atomicAdd(&counts[b], 1u);
    }
}

// sum of each block of kScanBlock counts
__global__ __launch_bounds__(256) void k_scan_sums(const uint32_t* __restrict__ in, uint32_t n,
                                                   uint32_t* __restrict__ bsum) {
    __shared__ uint32_t red[256];
    const uint32_t base = blockIdx.x * kScanBlock + threadIdx.x * 4u;
    uint32_t s = 0;
    for (uint32_t j = 0; j < 4; ++j)
        if (base + j < n) s += in[base + j];
    red[threadIdx.x] = s;
    __syncthreads();
    for (uint32_t off = 128; off > 0; off >>= 1) {
        if (threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x == 0) bsum[blockIdx.x] = red[0];
}

// exclusive scan of nb block sums in place by one block of 1024 threads,
// each over a contiguous range; the grand total goes to *total
__global__ __launch_bounds__(1024) void k_scan_top(uint32_t* __restrict__ bsum, uint32_t nb,
                                                   uint32_t* __restrict__ total) {
    __shared__ uint32_t part[1024];
    const uint32_t per = (nb + 1023u) / 1024u;
    const uint32_t b0 = min(threadIdx.x * per, nb), b1 = min(b0 + per, nb);
    uint32_t sum = 0;
    for (uint32_t j = b0; j < b1; ++j) sum += bsum[j];
    part[threadIdx.x] = sum;
    __syncthreads();
    for (uint32_t off = 1; off < 1024u; off <<= 1) {
        const uint32_t v = threadIdx.x >= off ? part[threadIdx.x - off] : 0u;
        __syncthreads();
        part[threadIdx.x] += v;
        __syncthreads();
    }
    uint32_t run = part[threadIdx.x] - sum;
    for (uint32_t j = b0; j < b1; ++j) {
        const uint32_t v = bsum[j];
        bsum[j] = run;
        run += v;
    }
    if (threadIdx.x == 1023) *total = part[1023];
}

// exclusive scan inside each block of kScanBlock counts plus the block's offset
__global__ __launch_bounds__(256) void k_scan_apply(const uint32_t* __restrict__ in, uint32_t n,
                                                    const uint32_t* __restrict__ boff, uint32_t* __restrict__ out) {
    __shared__ uint32_t part[256];
    const uint32_t base = blockIdx.x * kScanBlock + threadIdx.x * 4u;
    uint32_t v[4], s = 0;
    for (uint32_t j = 0; j < 4; ++j) {
        v[j] = base + j < n ? in[base + j] : 0u;
        s += v[j];
    }
    part[threadIdx.x] = s;
    __syncthreads();
    for (uint32_t off = 1; off < 256u; off <<= 1) {
        const uint32_t t = threadIdx.x >= off ? part[threadIdx.x - off] : 0u;
        __syncthreads();
        part[threadIdx.x] += t;
        __syncthreads();
    }
    uint32_t run = boff[blockIdx.x] + part[threadIdx.x] - s;
    for (uint32_t j = 0; j < 4; ++j) {
        if (base + j < n) out[base + j] = run;
        run += v[j];
    }
}

struct PmSorted {
    float4* rec;   // [n][2] as in PMapDev
    float* phi;
    uint32_t* ch;  // channel (export)
    unsigned long long *q, *photon;
};

__global__ void k_pm_scatter(PmRecords R, uint32_t n, float inv_h, const uint32_t* __restrict__ bucket,
                             const uint32_t* __restrict__ start, uint32_t* __restrict__ cursor, double scale,
                             PmSorted O) {
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        const uint32_t b = bucket[i];
        const uint32_t k = start[b] + atomicAdd(&cursor[b], 1u);
        const uint64_t tag = pm_tag(pm_cell(R.px[i], inv_h), pm_cell(R.py[i], inv_h), pm_cell(R.pz[i], inv_h));
        O.rec[2 * (size_t)k] = make_float4(R.px[i], R.py[i], R.pz[i], __uint_as_float((uint32_t)tag));
        O.rec[2 * (size_t)k + 1] = make_float4(R.nx[i], R.ny[i], R.nz[i], __uint_as_float((uint32_t)(tag >> 32)));
        O.phi[k] = R.phi[i];
        O.ch[k] = R.ch[i];
        O.q[k] = __double2ull_rn((double)R.phi[i] * scale);
        O.photon[k] = R.photon[i];
    }
}

__global__ void k_pm_gather(PMapDev pm, uint32_t n, const float* __restrict__ P, const float* __restrict__ N,
                            const uint32_t* __restrict__ ch, float* __restrict__ E) {
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        const F3 p{P[3 * (size_t)i], P[3 * (size_t)i + 1], P[3 * (size_t)i + 2]};
        const F3 nn{N[3 * (size_t)i], N[3 * (size_t)i + 1], N[3 * (size_t)i + 2]};
        E[i] = pmap_gather(pm, p, nn, ch[i]);
    }
}

inline uint32_t grid_of(size_t n, uint32_t bs) {
    size_t g = (n + bs - 1) / bs;
    return (uint32_t)std::max<size_t>(1, std::min<size_t>(g, 8192));
}

size_t slot(size_t n, size_t elem) { return ((n * elem + 255) / 256) * 256; }

}  // namespace

namespace scl {

namespace {

PmRecords carve_records(void* p, size_t cap) {
    Carver c{static_cast<char*>(p)};
    PmRecords R;
    R.px = c.take<float>(cap); R.py = c.take<float>(cap); R.pz = c.take<float>(cap);
    R.nx = c.take<float>(cap); R.ny = c.take<float>(cap); R.nz = c.take<float>(cap);
    R.phi = c.take<float>(cap);
    R.ch = c.take<uint32_t>(cap);
    R.photon = c.take<unsigned long long>(cap);
    R.stat = c.take<uint32_t>(4);
    R.cap = (uint32_t)cap;
    return R;
}
size_t record_bytes(size_t cap) { return 8 * slot(cap, 4) + slot(cap, 8) + 256 + 9 * 256; }

PmSorted carve_sorted(void* p, size_t n, uint32_t buckets, uint32_t** start) {
    Carver c{static_cast<char*>(p)};
    PmSorted O;
    O.rec = c.take<float4>(2 * n);
    O.phi = c.take<float>(n);
    O.ch = c.take<uint32_t>(n);
    O.q = c.take<unsigned long long>(n);
    O.photon = c.take<unsigned long long>(n);
    *start = c.take<uint32_t>((size_t)buckets + 1);
    return O;
}
size_t sorted_bytes(size_t n, uint32_t buckets) {
    return slot(2 * n, 16) + 2 * slot(n, 4) + 2 * slot(n, 8) + slot((size_t)buckets + 1, 4) + 7 * 256;
}

}  // namespace

sc_status pmap_trace(Ctx* c, Bvh* b, uint64_t N, uint32_t max_depth, const sc_wavelengths& wl, uint64_t seed,
                     float radius, Pmap* pm, sc_photon_stats* stats) {
    if (!(radius > 0.0f && radius <= FLT_MAX)) return set_error(SC_EINVAL, "radius must be positive and finite");
    if (N > (1ull << 24)) return set_error(SC_EUNSUPPORTED, "the general photon map takes at most 2^24 photons");
    hipStream_t st = c->stream;
    const size_t cap = std::max<uint64_t>(N, 1);
    SC_TRY(c->pm_rec.ensure(record_bytes(cap)));
    const PmRecords R = carve_records(c->pm_rec.p, cap);
    SC_HIP(hipMemsetAsync(R.stat, 0, 4 * sizeof(uint32_t), st));
    SC_TRY(trace_photons(c, b, N, max_depth, wl, seed, nullptr, nullptr, stats, &R));
    uint32_t stat[3] = {0, 0, 0};
    SC_HIP(hipMemcpyAsync(stat, R.stat, sizeof(stat), hipMemcpyDeviceToHost, st));
    SC_HIP(hipStreamSynchronize(st));
    const uint32_t n = stat[0];
    if (n > cap) return set_error(SC_EDEVICE, "photon map record overflow");
    float phimax, ext;
    memcpy(&phimax, &stat[1], 4);
    memcpy(&ext, &stat[2], 4);
    double scale = 1.0;
    if (n > 0 && phimax > 0.0f) {
        int e;
        frexp(ldexp(1.0, 62) / ((double)n * (double)phimax), &e);
        scale = ldexp(1.0, e - 1);
    }
    const float inv_h = 1.0f / (2.25f * radius);
    if (!((double)ext * (double)inv_h + 1.1 * (double)radius * (double)inv_h + 0.5 < 65536.0))
        return set_error(SC_EUNSUPPORTED, "radius too small for the extent of the stored photons (2^16 cells)");
    const uint32_t channels = wl.mode == SC_WL_FIXED ? wl.k : wl.bins;
    uint32_t cbits = 0;
    while ((1u << cbits) < channels) ++cbits;
    uint32_t buckets = 1024;
    while ((buckets < 2ull * n || buckets < (2u << cbits)) && buckets < (1u << 26)) buckets <<= 1;

    pm->valid = false;
    SC_TRY(pm->mem.ensure(sorted_bytes(std::max<uint32_t>(n, 1), buckets)));   // grow-only: a rebuild reuses it
    uint32_t* start = nullptr;
    const PmSorted O = carve_sorted(pm->mem.p, std::max<uint32_t>(n, 1), buckets, &start);
    const uint32_t nb = (buckets + kScanBlock - 1) / kScanBlock;
    // scratch: bucket of each record, counts, cursors, block sums
    const size_t tmp = slot(cap, 4) + 2 * slot(buckets, 4) + slot(nb, 4);
    SC_TRY(c->pm_tmp.ensure(tmp));
    Carver cv{static_cast<char*>(c->pm_tmp.p)};
    uint32_t* bucket = cv.take<uint32_t>(cap);
    uint32_t* counts = cv.take<uint32_t>(buckets);
    uint32_t* cursor = cv.take<uint32_t>(buckets);
    uint32_t* bsum = cv.take<uint32_t>(nb);
    const uint32_t bs = 256;
    hipLaunchKernelGGL(k_pm_zero, dim3(grid_of(buckets, bs)), dim3(bs), 0, st, counts, (size_t)buckets);
    hipLaunchKernelGGL(k_pm_zero, dim3(grid_of(buckets, bs)), dim3(bs), 0, st, cursor, (size_t)buckets);
    if (n)
        hipLaunchKernelGGL(k_pm_bucket, dim3(grid_of(n, bs)), dim3(bs), 0, st, R, n, inv_h, cbits, buckets - 1, bucket,
                           counts);
    hipLaunchKernelGGL(k_scan_sums, dim3(nb), dim3(256), 0, st, counts, buckets, bsum);
    hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(1024), 0, st, bsum, nb, start + buckets);
    hipLaunchKernelGGL(k_scan_apply, dim3(nb), dim3(256), 0, st, counts, buckets, bsum, start);
    if (n)
        hipLaunchKernelGGL(k_pm_scatter, dim3(grid_of(n, bs)), dim3(bs), 0, st, R, n, inv_h, bucket, start, cursor,
                           scale, O);
    SC_HIP(hipGetLastError());
    SC_HIP(hipStreamSynchronize(st));

    attach(c, &pm->ctx);
    pm->n = n;
    pm->radius = radius;
    pm->channels = channels;
    pm->buckets = buckets;
    pm->scale = scale;
    pm->photon = O.photon;
    pm->phi = O.phi;
    pm->ch = O.ch;
    PMapDev& d = pm->dev;
    d.rec = O.rec;
    d.q = O.q;
    d.start = start;
    d.mask = buckets - 1;
    d.cbits = cbits;
    d.on = 1;
    d.r = radius;
    d.r2 = radius * radius;
    d.inv_h = inv_h;
    d.c = 1.0 / ((scale * 3.14159265358979323846) * ((double)radius * (double)radius));
    pm->valid = true;
    return SC_OK;
}

sc_status pmap_export(const Pmap* pm, float* pos, float* nrm, float* phi, uint32_t* channel, uint64_t* photon) {
    const size_t n = pm->n;
    if (n == 0) return SC_OK;
    std::vector<float4> rec(2 * n);
    std::vector<float> ph(n);
    std::vector<uint32_t> ch(n);
    std::vector<unsigned long long> id(n);
    SC_HIP(hipStreamSynchronize(pm->ctx->stream));
    SC_HIP(hipMemcpy(rec.data(), pm->dev.rec, 2 * n * sizeof(float4), hipMemcpyDeviceToHost));
    SC_HIP(hipMemcpy(ph.data(), pm->phi, n * sizeof(float), hipMemcpyDeviceToHost));
    SC_HIP(hipMemcpy(ch.data(), pm->ch, n * sizeof(uint32_t), hipMemcpyDeviceToHost));
    SC_HIP(hipMemcpy(id.data(), pm->photon, n * sizeof(unsigned long long), hipMemcpyDeviceToHost));
    std::vector<size_t> order(n);
    std::iota(order.begin(), order.end(), size_t{0});
    std::sort(order.begin(), order.end(), [&](size_t a, size_t b) { return id[a] < id[b]; });
    for (size_t j = 0; j < n; ++j) {
        const size_t k = order[j];
        const float4 a = rec[2 * k], b = rec[2 * k + 1];
        if (pos) { pos[3 * j] = a.x; pos[3 * j + 1] = a.y; pos[3 * j + 2] = a.z; }
        if (nrm) { nrm[3 * j] = b.x; nrm[3 * j + 1] = b.y; nrm[3 * j + 2] = b.z; }
        if (phi) phi[j] = ph[k];
        if (channel) channel[j] = ch[k];
        if (photon) photon[j] = id[k];
    }
    return SC_OK;
}

sc_status pmap_gather(Ctx* c, const Pmap* pm, uint32_t n, const float* P, const float* N, const uint32_t* ch,
                      float* E) {
    if (n == 0) return SC_OK;
    hipLaunchKernelGGL(k_pm_gather, dim3(grid_of(n, 256)), dim3(256), 0, c->stream, pm->dev, n, P, N, ch, E);
    SC_HIP(hipGetLastError());
    return SC_OK;
}

}  // namespace scl
