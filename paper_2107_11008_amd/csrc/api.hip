// api.hip -- the C ABI (include/sc.h): argument checks, handles, scene
// tables, and dispatch to the GPU passes.
#pragma clang fp contract(off)
#include <hip/hip_runtime.h>
#include <float.h>
#include <math.h>
#include <stdint.h>
#include <string.h>

#include <algorithm>
#include <new>
#include <string>
#include <vector>

#include "sc_internal.h"
#include "sc_kernels.h"
#include "sc_unet.h"
#include "sc_batch.h"

struct sc_unet {
    scl::Unet u;
};
struct sc_batch {
    scl::Batch bt;
};

namespace scl {

static thread_local std::string g_err;

sc_status set_error(sc_status code, const std::string& msg) {
    g_err = msg;
    return code;
}

}  // namespace scl

using scl::set_error;

namespace {

sc_status check_wavelengths(const sc_wavelengths* wl) {
    if (!wl) return set_error(SC_EINVAL, "wavelengths is NULL");
    if (wl->mode == SC_WL_FIXED) {
        if (!(wl->k == 1 || wl->k == 3)) return set_error(SC_EINVAL, "fixed wavelengths need k = 1 or 3");
        for (uint32_t i = 0; i < wl->k; ++i)
            if (!(wl->nm[i] > 0.0f) || !isfinite(wl->nm[i])) return set_error(SC_EINVAL, "wavelength must be > 0");
    } else if (wl->mode == SC_WL_UNIFORM) {
        if (wl->bins == 0 || wl->bins > 256) return set_error(SC_EINVAL, "uniform wavelengths need 1..256 bins");
        if (!(wl->hi > wl->lo) || !(wl->lo > 0.0f) || !isfinite(wl->hi))
            return set_error(SC_EINVAL, "uniform wavelengths need 0 < lo < hi");
    } else {
        return set_error(SC_EINVAL, "unknown wavelength mode");
    }
    return SC_OK;
}

sc_status upload(scl::DevBuf& buf, const void* host, size_t bytes, hipStream_t st) {
    SC_TRY(buf.ensure(bytes));
    if (bytes) SC_HIP(hipMemcpyAsync(buf.p, host, bytes, hipMemcpyHostToDevice, st));
    return SC_OK;
}

}  // namespace

extern "C" {

uint32_t sc_abi_version(void) { return SC_ABI_VERSION; }

const char* sc_last_error(void) { return scl::g_err.c_str(); }

sc_status sc_create(int device, void* hip_stream, sc_ctx** out) {
    if (!out) return set_error(SC_EINVAL, "out is NULL");
    *out = nullptr;
    int n = 0;
    if (hipGetDeviceCount(&n) != hipSuccess || n == 0) return set_error(SC_EDEVICE, "no HIP device");
    if (device < 0 || device >= n) return set_error(SC_EINVAL, "device index out of range");
    SC_HIP(hipSetDevice(device));
    sc_ctx* x = new (std::nothrow) sc_ctx();
    if (!x) return set_error(SC_ENOMEM, "host allocation failed");
    x->c.device = device;
    x->c.stream = static_cast<hipStream_t>(hip_stream);
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) == hipSuccess && cus > 0)
        x->c.cus = (uint32_t)cus;
    sc_status s = scl::ctx_init(&x->c);
    if (s == SC_OK) s = scl::scratch_init(device);   // the allocation-free entry point's array on this device
    if (s != SC_OK) {
        delete x;
        return s;
    }
    *out = x;
    return SC_OK;
}

sc_status sc_destroy(sc_ctx* ctx) {
    if (!ctx) return set_error(SC_EINVAL, "ctx is NULL");
    (void)hipStreamSynchronize(ctx->c.stream);
    scl::ctx_release(&ctx->c);
    for (scl::Ctx** slot : ctx->c.handles) *slot = nullptr;   // handles outlive their context safely
    ctx->c.handles.clear();
    delete ctx;
    return SC_OK;
}

sc_status sc_set_stream(sc_ctx* ctx, void* hip_stream) {
    if (!ctx) return set_error(SC_EINVAL, "ctx is NULL");
    SC_HIP(hipStreamSynchronize(ctx->c.stream));
    ctx->c.stream = static_cast<hipStream_t>(hip_stream);
    return SC_OK;
}

sc_status sc_set_option(sc_ctx* ctx, int32_t option, int64_t value) {
    if (!ctx) return set_error(SC_EINVAL, "ctx is NULL");
    switch (option) {
        case SC_OPT_COUNT_VISITS: ctx->c.count_visits = value != 0; return SC_OK;
        case SC_OPT_PROFILE: ctx->c.profile = value != 0; return SC_OK;
        case SC_OPT_QUEUE_CAP:
            if (value < 1024 || value > (int64_t)1 << 30) return set_error(SC_EINVAL, "queue cap out of range");
            ctx->c.queue_cap = (uint64_t)value;
            return SC_OK;
        case SC_OPT_STAGED_DEPTH:
            if (value < 0 || value > 1000000) return set_error(SC_EINVAL, "staged depth out of range");
            ctx->c.staged_depth = (uint32_t)value;
            return SC_OK;
        case SC_OPT_PHOTON_STAGED_DEPTH:
            if (value < 0 || value > 1000000) return set_error(SC_EINVAL, "staged depth out of range");
            ctx->c.photon_staged_depth = (uint32_t)value;
            return SC_OK;
        case SC_OPT_PHOTON_CAP:
            if (value < 1024 || value > (int64_t)1 << 28) return set_error(SC_EINVAL, "photon cap out of range");
            ctx->c.photon_cap = (uint64_t)value;
            return SC_OK;
        case SC_OPT_TRACE_BLOCKS:
            if (value < 1 || value > 16) return set_error(SC_EINVAL, "trace blocks per CU must be 1..16");
            ctx->c.trace_blocks = (uint32_t)value;
            return SC_OK;
        case SC_OPT_BVH_BUILDER:
            if (value < 0 || value > 2) return set_error(SC_EINVAL, "BVH builder must be 0, 1 or 2");
            ctx->c.bvh_builder = (uint32_t)value;
            return SC_OK;
        case SC_OPT_CONV_BIG_TILE:
            if (value < 0 || value > ((int64_t)1 << 32)) return set_error(SC_EINVAL, "tile threshold out of range");
            ctx->c.conv_big_tile = (uint64_t)value;
            return SC_OK;
        default: return set_error(SC_EINVAL, "unknown option");
    }
}

sc_status sc_sync(sc_ctx* ctx) {
    if (!ctx) return set_error(SC_EINVAL, "ctx is NULL");
    SC_HIP(hipStreamSynchronize(ctx->c.stream));
    SC_HIP(hipGetLastError());
    return SC_OK;
}

sc_status sc_get_counters(sc_ctx* ctx, sc_counters* out) {
    if (!ctx || !out) return set_error(SC_EINVAL, "ctx or out is NULL");
    return scl::ctx_counters(&ctx->c, out);
}

sc_status sc_reset_counters(sc_ctx* ctx) {
    if (!ctx) return set_error(SC_EINVAL, "ctx is NULL");
    return scl::ctx_reset_counters(&ctx->c);
}

namespace {

// a handle whose last rebuild failed holds no usable tree
sc_status check_built(const sc_bvh* bvh) {
    if (bvh->b.n_nodes == 0) return set_error(SC_EINVAL, "bvh holds no tree (its last rebuild failed)");
    return SC_OK;
}

sc_status check_scene(const sc_scene* sc) {
    if (!sc->V || !sc->I || !sc->tri_obj || !sc->mat) return set_error(SC_EINVAL, "scene arrays V, I, tri_obj, mat are required");
    if (sc->nt == 0 || sc->nv == 0) return set_error(SC_EINVAL, "scene has no triangles");
    if (sc->nt > (1u << 28) - 1) return set_error(SC_EUNSUPPORTED, "more than 2^28 - 1 triangles");
    if (sc->n_mat < 2) return set_error(SC_EINVAL, "n_mat must be >= 2 (row 0 is unused)");
    if (sc->n_mat > 65536u) return set_error(SC_EUNSUPPORTED, "more than 65536 materials (object ids are 16-bit in media sets)");
    for (uint32_t i = 1; i < sc->n_mat; ++i) {
        const sc_material& m = sc->mat[i];
        if (m.type > SC_MAT_EMISSIVE) return set_error(SC_EINVAL, "unknown material type");
        if (m.type == SC_MAT_DIELECTRIC) {
            for (int c = 0; c < 3; ++c)
                if (!(m.sigma[c] >= 0.0f && m.sigma[c] <= FLT_MAX))
                    return set_error(SC_EINVAL, "dielectric absorption must be finite and >= 0");
            if (!(m.roughness >= 0.0f && m.roughness <= 1.0f)) return set_error(SC_EINVAL, "roughness must be in [0, 1]");
        }
        if (m.type == SC_MAT_DIFFUSE && m.albedo_mode > SC_ALBEDO_TEXTURE_RGB) return set_error(SC_EINVAL, "unknown albedo mode");
        if (m.type == SC_MAT_DIFFUSE && m.albedo_mode == SC_ALBEDO_TEXTURE && !sc->tex)
            return set_error(SC_EINVAL, "texture albedo without a texture");
        if (m.type == SC_MAT_DIFFUSE && m.albedo_mode == SC_ALBEDO_TEXTURE_RGB && !sc->tex_rgb)
            return set_error(SC_EINVAL, "RGB texture albedo without an RGB texture");
    }
    if (sc->n_pl && !sc->point_lights) return set_error(SC_EINVAL, "point_lights is NULL");
    if (sc->n_tg && (!sc->targets_obj || !sc->targets_sphere)) return set_error(SC_EINVAL, "photon targets are NULL");
    if (sc->recv_obj) {
        if (sc->recv_obj >= sc->n_mat) return set_error(SC_EINVAL, "receiver object out of range");
        if (sc->recv_wc == 0 || sc->recv_hc == 0 || !(sc->recv_ext_u > 0.0f) || !(sc->recv_ext_v > 0.0f))
            return set_error(SC_EINVAL, "receiver needs cells and a positive extent");
    }
    if ((sc->tex || sc->tex_rgb) && (sc->tex_w == 0 || sc->tex_h == 0 || !(sc->tex_ext_u > 0.0f) || !(sc->tex_ext_v > 0.0f)))
        return set_error(SC_EINVAL, "texture needs a size and a positive extent");
    return SC_OK;
}

// (Re)builds b for scene sc: BVH, light and material tables, device view.
// Device buffers of b are reused when large enough.
sc_status build_into(scl::Ctx* c, scl::Bvh* b, const sc_scene* sc, uint32_t width, uint32_t leaf_max) {
    hipStream_t st = c->stream;
    scl::attach(c, &b->ctx);
    b->scene_in = *sc;
    b->scene = DevScene{};
    std::vector<float> tg(4 * (size_t)sc->n_tg);
    for (uint32_t i = 0; i < 4 * sc->n_tg; ++i) tg[i] = sc->targets_sphere[i];
    sc_status s = SC_OK;
    if ((s = upload(b->mat, sc->mat, sizeof(sc_material) * sc->n_mat, st)) == SC_OK &&
        (s = upload(b->pl, sc->point_lights, 16 * (size_t)sc->n_pl, st)) == SC_OK)
        s = upload(b->tg, tg.data(), 16 * (size_t)sc->n_tg, st);
    // emissive triangles in index order with their vertices, from the builder
    std::vector<uint32_t> emit_prim;
    std::vector<float> emit_v;
    if (s == SC_OK) s = scl::build_wide_bvh(c, b, width, leaf_max, emit_prim, emit_v);
    if (s == SC_OK && b->max_stack > (uint32_t)kMaxStack)
        s = set_error(SC_EUNSUPPORTED, "BVH depth " + std::to_string(b->depth) + " needs a traversal stack of " +
                                           std::to_string(b->max_stack) + " > " + std::to_string(kMaxStack));
    // emitter areas in double, cumulative distribution rounded to float
    std::vector<float> emit_cdf;
    double a_tot = 0.0;
    float max_power = 0.0f;
    if (s == SC_OK) {
        std::vector<double> area;
        area.reserve(emit_prim.size());
        for (size_t k = 0; k < emit_prim.size(); ++k) {
            const float* tv = emit_v.data() + 9 * k;
            double a[3], bb[3], cc[3];
            for (int j = 0; j < 3; ++j) {
                a[j] = tv[j];
                bb[j] = tv[3 + j];
                cc[j] = tv[6 + j];
            }
            const double e1[3] = {bb[0] - a[0], bb[1] - a[1], bb[2] - a[2]};
            const double e2[3] = {cc[0] - a[0], cc[1] - a[1], cc[2] - a[2]};
            const double cx = e1[1] * e2[2] - e1[2] * e2[1];
            const double cy = e1[2] * e2[0] - e1[0] * e2[2];
            const double cz = e1[0] * e2[1] - e1[1] * e2[0];
            area.push_back(0.5 * sqrt(cx * cx + cy * cy + cz * cz));
            a_tot += area.back();
        }
        double cum = 0.0;
        for (size_t j = 0; j < area.size(); ++j) {
            cum += area[j];
            emit_cdf.push_back((float)(cum / a_tot));
        }
        if (!emit_cdf.empty()) emit_cdf.back() = 1.0f;
    }
    if (s == SC_OK) {
        const float atf = (float)a_tot;
        for (uint32_t i = 0; i < sc->n_pl; ++i) max_power = std::max(max_power, sc->point_lights[4 * (size_t)i + 3]);
        if (!emit_prim.empty())
            for (uint32_t i = 1; i < sc->n_mat; ++i)
                if (sc->mat[i].type == SC_MAT_EMISSIVE) max_power = std::max(max_power, sc->mat[i].le * atf);
        b->max_power = max_power;
        if ((s = upload(b->emit_prim, emit_prim.data(), 4 * emit_prim.size(), st)) == SC_OK &&
            (s = upload(b->emit_cdf, emit_cdf.data(), 4 * emit_cdf.size(), st)) == SC_OK) {
            if (hipStreamSynchronize(st) != hipSuccess) s = set_error(SC_EDEVICE, "upload failed");
        }
    }
    if (s != SC_OK) return s;
    DevScene& D = b->scene;
    D.V = sc->V; D.I = sc->I; D.VN = sc->VN; D.tri_obj = sc->tri_obj; D.nt = sc->nt;
    D.mat = b->mat.as<sc_material>(); D.n_mat = sc->n_mat;
    D.pl = b->pl.as<float>(); D.n_pl = sc->n_pl;
    D.tg = b->tg.as<float>(); D.n_tg = sc->n_tg;
    D.tex = sc->tex; D.tex_rgb = sc->tex_rgb;
    D.tex_w = sc->tex_w; D.tex_h = sc->tex_h; D.tex_x0 = sc->tex_x0; D.tex_y0 = sc->tex_y0;
    const bool any_tex = sc->tex || sc->tex_rgb;
    D.tex_sx = any_tex ? (float)sc->tex_w / sc->tex_ext_u : 0.0f;
    D.tex_sy = any_tex ? (float)sc->tex_h / sc->tex_ext_v : 0.0f;
    D.recv_obj = sc->recv_obj; D.recv_wc = sc->recv_wc; D.recv_hc = sc->recv_hc;
    D.recv_x0 = sc->recv_x0; D.recv_y0 = sc->recv_y0;
    D.cell_sx = sc->recv_obj ? (float)sc->recv_wc / sc->recv_ext_u : 0.0f;
    D.cell_sy = sc->recv_obj ? (float)sc->recv_hc / sc->recv_ext_v : 0.0f;
    D.inv_cell_area = sc->recv_obj ? (float)(((double)sc->recv_wc * (double)sc->recv_hc) /
                                             ((double)sc->recv_ext_u * (double)sc->recv_ext_v))
                                   : 0.0f;
    D.emit_prim = b->emit_prim.as<uint32_t>(); D.emit_cdf = b->emit_cdf.as<float>();
    D.n_emit = (uint32_t)emit_prim.size(); D.a_tot = (float)a_tot;
    D.n_entries = sc->n_pl + (emit_prim.empty() ? 0u : 1u);
    D.nodes = b->nodes.as<BNode>(); D.tris = b->tris.as<float4>(); D.n_nodes = b->n_nodes;
    return SC_OK;
}

}  // namespace

sc_status sc_build_bvh(sc_ctx* ctx, const sc_scene* sc, const sc_bvh_opts* opts, sc_bvh** out) {
    if (!ctx || !sc || !out) return set_error(SC_EINVAL, "ctx, scene or out is NULL");
    *out = nullptr;
    SC_TRY(check_scene(sc));
    uint32_t width = opts && opts->width ? opts->width : 8u;
    uint32_t leaf_max = opts && opts->leaf_max ? opts->leaf_max : 4u;
    if (!(width == 4 || width == 8)) return set_error(SC_EINVAL, "width must be 4 or 8");
    if (leaf_max < 1 || leaf_max > 8) return set_error(SC_EINVAL, "leaf_max must be 1..8");
    sc_bvh* h = new (std::nothrow) sc_bvh();
    if (!h) return set_error(SC_ENOMEM, "host allocation failed");
    const sc_status s = build_into(&ctx->c, &h->b, sc, width, leaf_max);
    if (s != SC_OK) {
        delete h;
        return s;
    }
    *out = h;
    return SC_OK;
}

sc_status sc_bvh_rebuild(sc_ctx* ctx, sc_bvh* bvh, const sc_scene* sc) {
    if (!ctx || !bvh || !sc) return set_error(SC_EINVAL, "ctx, bvh or scene is NULL");
    if (bvh->b.ctx != &ctx->c) return set_error(SC_EINVAL, "bvh was built on another context");
    SC_TRY(check_scene(sc));
    const sc_status s = build_into(&ctx->c, &bvh->b, sc, bvh->b.width, bvh->b.leaf_max);
    if (s != SC_OK) bvh->b.n_nodes = 0;   // unusable until rebuilt
    return s;
}

sc_status sc_bvh_get_info(const sc_bvh* bvh, sc_bvh_info* out) {
    if (!bvh || !out) return set_error(SC_EINVAL, "bvh or out is NULL");
    const scl::Bvh& b = bvh->b;
    out->width = b.width;
    out->leaf_max = b.leaf_max;
    out->n_nodes = b.n_nodes;
    out->depth = b.depth;
    out->node_bytes = (uint64_t)b.n_nodes * sizeof(BNode);
    out->tri_bytes = (uint64_t)b.scene.nt * 48u;
    out->max_stack = b.max_stack;
    return SC_OK;
}

sc_status sc_bvh_export(const sc_bvh* bvh, void* nodes_host, void* tris_host) {
    if (!bvh) return set_error(SC_EINVAL, "bvh is NULL");
    const scl::Bvh& b = bvh->b;
    if (!b.ctx) return set_error(SC_EINVAL, "the bvh's context was destroyed");
    SC_HIP(hipStreamSynchronize(b.ctx->stream));
    if (nodes_host) SC_HIP(hipMemcpy(nodes_host, b.nodes.p, sizeof(BNode) * (size_t)b.n_nodes, hipMemcpyDeviceToHost));
    if (tris_host) SC_HIP(hipMemcpy(tris_host, b.tris.p, 48 * (size_t)b.scene.nt, hipMemcpyDeviceToHost));
    return SC_OK;
}

sc_status sc_bvh_free(sc_bvh* bvh) {
    if (!bvh) return set_error(SC_EINVAL, "bvh is NULL");
    if (bvh->b.ctx) (void)hipStreamSynchronize(bvh->b.ctx->stream);
    scl::detach(&bvh->b.ctx);
    delete bvh;
    return SC_OK;
}

sc_status sc_trace_rays(sc_ctx* ctx, const sc_bvh* bvh, uint32_t n, const float* O, const float* D, float* t,
                        uint32_t* prim, float* u, float* v) {
    if (!ctx || !bvh) return set_error(SC_EINVAL, "ctx or bvh is NULL");
    SC_TRY(check_built(bvh));
    if (n == 0) return SC_OK;
    if (!O || !D || !t || !prim) return set_error(SC_EINVAL, "O, D, t and prim are required");
    return scl::trace_rays(&ctx->c, const_cast<scl::Bvh*>(&bvh->b), n, O, D, t, prim, u, v);
}

sc_status sc_trace_rays_noalloc(sc_ctx* ctx, const sc_bvh* bvh, uint32_t n, const float* O, const float* D, float* t,
                                uint32_t* prim, float* u, float* v) {
    if (!ctx || !bvh) return set_error(SC_EINVAL, "ctx or bvh is NULL");
    SC_TRY(check_built(bvh));
    if (n == 0) return SC_OK;
    if (!O || !D || !t || !prim) return set_error(SC_EINVAL, "O, D, t and prim are required");
    return scl::trace_rays_noalloc(&ctx->c, const_cast<scl::Bvh*>(&bvh->b), n, O, D, t, prim, u, v);
}

uint32_t sc_trace_rays_noalloc_max(void) { return scl::trace_rays_noalloc_max(); }

sc_status sc_occluded(sc_ctx* ctx, const sc_bvh* bvh, uint32_t n, const float* O, const float* D, const float* tmax,
                      const uint32_t* excl, uint8_t* occ) {
    if (!ctx || !bvh) return set_error(SC_EINVAL, "ctx or bvh is NULL");
    SC_TRY(check_built(bvh));
    if (n == 0) return SC_OK;
    if (!O || !D || !tmax || !occ) return set_error(SC_EINVAL, "O, D, tmax and occluded are required");
    return scl::occluded(&ctx->c, const_cast<scl::Bvh*>(&bvh->b), n, O, D, tmax, excl, occ);
}

sc_status sc_trace_photons(sc_ctx* ctx, const sc_bvh* bvh, uint64_t n_photons, uint32_t max_depth,
                           const sc_wavelengths* wl, uint64_t seed, float* caustic_map, uint32_t* count_map,
                           sc_photon_stats* stats) {
    if (!ctx || !bvh || !caustic_map) return set_error(SC_EINVAL, "ctx, bvh or caustic_map is NULL");
    SC_TRY(check_built(bvh));
    SC_TRY(check_wavelengths(wl));
    if (max_depth == 0) return set_error(SC_EINVAL, "max_depth must be >= 1");
    if (!bvh->b.scene.recv_obj) return set_error(SC_EINVAL, "the scene has no caustic receiver");
    if (n_photons > (1ull << 40)) return set_error(SC_EINVAL, "n_photons too large");
    if (stats) memset(stats, 0, sizeof(*stats));
    return scl::trace_photons(&ctx->c, const_cast<scl::Bvh*>(&bvh->b), n_photons, max_depth, *wl, seed, caustic_map,
                              count_map, stats);
}

sc_status sc_pmap_trace(sc_ctx* ctx, const sc_bvh* bvh, uint64_t n_photons, uint32_t max_depth,
                        const sc_wavelengths* wl, uint64_t seed, float radius, sc_pmap** out, sc_photon_stats* stats) {
    if (!ctx || !bvh || !out) return set_error(SC_EINVAL, "ctx, bvh or out is NULL");
    *out = nullptr;
    SC_TRY(check_built(bvh));
    SC_TRY(check_wavelengths(wl));
    if (max_depth == 0) return set_error(SC_EINVAL, "max_depth must be >= 1");
    if (stats) memset(stats, 0, sizeof(*stats));
    sc_pmap* h = new (std::nothrow) sc_pmap();
    if (!h) return set_error(SC_ENOMEM, "host allocation failed");
    const sc_status s = scl::pmap_trace(&ctx->c, const_cast<scl::Bvh*>(&bvh->b), n_photons, max_depth, *wl, seed,
                                        radius, &h->p, stats);
    if (s != SC_OK) {
        delete h;
        return s;
    }
    *out = h;
    return SC_OK;
}

sc_status sc_pmap_retrace(sc_ctx* ctx, const sc_bvh* bvh, uint64_t n_photons, uint32_t max_depth,
                          const sc_wavelengths* wl, uint64_t seed, float radius, sc_pmap* pm, sc_photon_stats* stats) {
    if (!ctx || !bvh || !pm) return set_error(SC_EINVAL, "ctx, bvh or pmap is NULL");
    if (pm->p.ctx && pm->p.ctx != &ctx->c) return set_error(SC_EINVAL, "pmap belongs to another context");
    pm->p.valid = false;
    SC_TRY(check_built(bvh));
    SC_TRY(check_wavelengths(wl));
    if (max_depth == 0) return set_error(SC_EINVAL, "max_depth must be >= 1");
    if (stats) memset(stats, 0, sizeof(*stats));
    return scl::pmap_trace(&ctx->c, const_cast<scl::Bvh*>(&bvh->b), n_photons, max_depth, *wl, seed, radius, &pm->p,
                           stats);
}

sc_status sc_pmap_get_info(const sc_pmap* pm, sc_pmap_info* out) {
    if (!pm || !out) return set_error(SC_EINVAL, "pmap or out is NULL");
    if (!pm->p.valid) return set_error(SC_EINVAL, "pmap holds no map (a rebuild failed)");
    out->n_stored = pm->p.n;
    out->radius = pm->p.radius;
    out->channels = pm->p.channels;
    out->scale = pm->p.scale;
    out->buckets = pm->p.buckets;
    out->bytes = pm->p.mem.bytes;
    return SC_OK;
}

sc_status sc_pmap_export(const sc_pmap* pm, float* pos, float* nrm, float* phi, uint32_t* channel, uint64_t* photon) {
    if (!pm) return set_error(SC_EINVAL, "pmap is NULL");
    if (!pm->p.valid) return set_error(SC_EINVAL, "pmap holds no map (a rebuild failed)");
    return scl::pmap_export(&pm->p, pos, nrm, phi, channel, photon);
}

sc_status sc_pmap_gather(sc_ctx* ctx, const sc_pmap* pm, uint32_t n, const float* P, const float* N,
                         const uint32_t* ch, float* E) {
    if (!ctx || !pm) return set_error(SC_EINVAL, "ctx or pmap is NULL");
    if (n && (!P || !N || !ch || !E)) return set_error(SC_EINVAL, "gather arrays are NULL");
    if (pm->p.ctx != &ctx->c) return set_error(SC_EINVAL, "pmap belongs to another context");
    if (!pm->p.valid) return set_error(SC_EINVAL, "pmap holds no map (a rebuild failed)");
    return scl::pmap_gather(&ctx->c, &pm->p, n, P, N, ch, E);
}

sc_status sc_pmap_free(sc_pmap* pm) {
    if (pm) {
        if (pm->p.ctx) (void)hipStreamSynchronize(pm->p.ctx->stream);
        scl::detach(&pm->p.ctx);
        delete pm;
    }
    return SC_OK;
}

sc_status sc_render_pmap(sc_ctx* ctx, const sc_bvh* bvh, const sc_camera* cam, uint32_t spp, uint32_t max_depth,
                         const sc_wavelengths* wl, uint64_t seed, const sc_pmap* pm, const sc_aov* out) {
    if (!ctx || !bvh || !cam || !out || !pm) return set_error(SC_EINVAL, "ctx, bvh, camera, pmap or out is NULL");
    SC_TRY(check_built(bvh));
    SC_TRY(check_wavelengths(wl));
    if (spp == 0) return set_error(SC_EINVAL, "spp must be >= 1");
    if (max_depth == 0) return set_error(SC_EINVAL, "max_depth must be >= 1");
    if (cam->w == 0 || cam->h == 0) return set_error(SC_EINVAL, "camera has no pixels");
    if ((uint64_t)cam->w * cam->h > (1ull << 28)) return set_error(SC_EUNSUPPORTED, "image too large");
    if (pm->p.ctx != &ctx->c) return set_error(SC_EINVAL, "pmap belongs to another context");
    if (!pm->p.valid) return set_error(SC_EINVAL, "pmap holds no map (a rebuild failed)");
    const uint32_t ch = wl->mode == SC_WL_FIXED ? wl->k : wl->bins;
    if (ch != pm->p.channels) return set_error(SC_EINVAL, "the photon map has other channels than the wavelength setting");
    return scl::render(&ctx->c, const_cast<scl::Bvh*>(&bvh->b), *cam, spp, max_depth, *wl, seed, nullptr, *out,
                       &pm->p.dev);
}

sc_status sc_render(sc_ctx* ctx, const sc_bvh* bvh, const sc_camera* cam, uint32_t spp, uint32_t max_depth,
                    const sc_wavelengths* wl, uint64_t seed, const float* caustic_map, const sc_aov* out) {
    if (!ctx || !bvh || !cam || !out) return set_error(SC_EINVAL, "ctx, bvh, camera or out is NULL");
    SC_TRY(check_built(bvh));
    SC_TRY(check_wavelengths(wl));
    if (spp == 0) return set_error(SC_EINVAL, "spp must be >= 1");
    if (max_depth == 0) return set_error(SC_EINVAL, "max_depth must be >= 1");
    if (cam->w == 0 || cam->h == 0) return set_error(SC_EINVAL, "camera has no pixels");
    if ((uint64_t)cam->w * cam->h > (1ull << 28)) return set_error(SC_EUNSUPPORTED, "image too large");
    if (caustic_map && !bvh->b.scene.recv_obj) return set_error(SC_EINVAL, "caustic map given but no receiver");
    return scl::render(&ctx->c, const_cast<scl::Bvh*>(&bvh->b), *cam, spp, max_depth, *wl, seed, caustic_map, *out);
}

sc_status sc_render_overlap(sc_ctx* ctx, const sc_bvh* bvh, const sc_camera* cam, uint32_t spp, uint32_t max_depth,
                            const sc_wavelengths* wl, uint64_t seed, const float* caustic_map, void* map_ready,
                            const sc_aov* out) {
    if (!ctx || !bvh || !cam || !out) return set_error(SC_EINVAL, "ctx, bvh, camera or out is NULL");
    if (!caustic_map || !map_ready) return set_error(SC_EINVAL, "caustic_map or map_ready is NULL");
    SC_TRY(check_built(bvh));
    SC_TRY(check_wavelengths(wl));
    if (spp == 0) return set_error(SC_EINVAL, "spp must be >= 1");
    if (max_depth == 0) return set_error(SC_EINVAL, "max_depth must be >= 1");
    if (cam->w == 0 || cam->h == 0) return set_error(SC_EINVAL, "camera has no pixels");
    if ((uint64_t)cam->w * cam->h > (1ull << 28)) return set_error(SC_EUNSUPPORTED, "image too large");
    if (!bvh->b.scene.recv_obj) return set_error(SC_EINVAL, "caustic map given but no receiver");
    return scl::render(&ctx->c, const_cast<scl::Bvh*>(&bvh->b), *cam, spp, max_depth, *wl, seed, caustic_map, *out,
                       nullptr, static_cast<hipEvent_t>(map_ready));
}

static sc_status check_tune(const sc_tune& t) {
    if (!(t.block_size == 64 || t.block_size == 128 || t.block_size == 256))
        return set_error(SC_EINVAL, "block_size must be 64, 128 or 256");
    if (t.blocks_per_cu < 1 || t.blocks_per_cu > 32) return set_error(SC_EINVAL, "blocks_per_cu must be 1..32");
    if (t.px_per_item < 64 || t.px_per_item > 4096 || t.px_per_item % 64)
        return set_error(SC_EINVAL, "px_per_item must be a multiple of 64 up to 4096");
    if (t.ph_per_item > 65536 || t.ph_per_item % 64)
        return set_error(SC_EINVAL, "ph_per_item must be 0 or a multiple of 64 up to 65536");
    return SC_OK;
}

static sc_status check_batch_items(sc_ctx* ctx, uint32_t n, const sc_batch_item* items) {
    if (n == 0) return set_error(SC_EINVAL, "empty batch");
    for (uint32_t i = 0; i < n; ++i) {
        const sc_batch_item& it = items[i];
        const std::string where = "batch item " + std::to_string(i) + ": ";
        if (!it.bvh) return set_error(SC_EINVAL, where + "bvh is NULL");
        SC_TRY(check_built(it.bvh));
        SC_TRY(check_wavelengths(&it.wl));
        if (it.spp == 0 || it.max_depth == 0) return set_error(SC_EINVAL, where + "spp and max_depth must be >= 1");
        if (it.cam.w == 0 || it.cam.h == 0) return set_error(SC_EINVAL, where + "camera has no pixels");
        if ((uint64_t)it.cam.w * it.cam.h > (1ull << 28)) return set_error(SC_EUNSUPPORTED, where + "image too large");
        if ((it.n_photons || it.caustic_map) && !it.bvh->b.scene.recv_obj)
            return set_error(SC_EINVAL, where + "caustics need a receiver");
        if (it.bvh->b.ctx != &ctx->c) return set_error(SC_EINVAL, where + "bvh belongs to another context");
    }
    return SC_OK;
}

sc_status sc_batch_create(sc_ctx* ctx, uint32_t n, const sc_batch_item* items, const sc_tune* tune, sc_batch** out) {
    if (!ctx || !items || !out) return set_error(SC_EINVAL, "ctx, items or out is NULL");
    *out = nullptr;
    const sc_tune t = tune ? *tune : sc_tune{128, 8, 64, 1, 0, 8};
    SC_TRY(check_tune(t));
    SC_TRY(check_batch_items(ctx, n, items));
    sc_batch* b = new (std::nothrow) sc_batch();
    if (!b) return set_error(SC_ENOMEM, "host allocation failed");
    sc_status s = scl::batch_create(&ctx->c, n, items, t, &b->bt);
    if (s != SC_OK) {
        delete b;
        return s;
    }
    *out = b;
    return SC_OK;
}

sc_status sc_batch_run(sc_ctx* ctx, sc_batch* batch) {
    if (!ctx || !batch) return set_error(SC_EINVAL, "ctx or batch is NULL");
    if (batch->bt.ctx != &ctx->c) return set_error(SC_EINVAL, "batch belongs to another context");
    return scl::batch_run(&batch->bt);
}

sc_status sc_batch_free(sc_batch* batch) {
    if (!batch) return set_error(SC_EINVAL, "batch is NULL");
    if (batch->bt.ctx) (void)hipStreamSynchronize(batch->bt.ctx->stream);
    scl::detach(&batch->bt.ctx);
    delete batch;
    return SC_OK;
}

sc_status sc_render_batch(sc_ctx* ctx, uint32_t n, const sc_batch_item* items, const sc_tune* tune) {
    sc_batch* b = nullptr;
    SC_TRY(sc_batch_create(ctx, n, items, tune, &b));
    sc_status s = sc_batch_run(ctx, b);
    if (s == SC_OK && hipStreamSynchronize(ctx->c.stream) != hipSuccess) s = set_error(SC_EDEVICE, "batch failed");
    sc_batch_free(b);
    return s;
}

// The scene a built BVH was made from: the caller's device arrays as given
// at build time, the host tables read back from the handle's device copies.
static sc_status scene_of_bvh(const scl::Bvh& b, sc_scene& sc, std::vector<sc_material>& mat, std::vector<float>& pl,
                              std::vector<float>& tg, std::vector<uint32_t>& tg_obj) {
    sc = b.scene_in;
    mat.resize(sc.n_mat);
    pl.resize(4 * (size_t)sc.n_pl);
    tg.resize(4 * (size_t)sc.n_tg);
    tg_obj.assign(sc.n_tg, 1u);
    if (b.ctx) SC_HIP(hipStreamSynchronize(b.ctx->stream));
    SC_HIP(hipMemcpy(mat.data(), b.mat.p, sizeof(sc_material) * mat.size(), hipMemcpyDeviceToHost));
    if (sc.n_pl) SC_HIP(hipMemcpy(pl.data(), b.pl.p, 4 * pl.size(), hipMemcpyDeviceToHost));
    if (sc.n_tg) SC_HIP(hipMemcpy(tg.data(), b.tg.p, 4 * tg.size(), hipMemcpyDeviceToHost));
    sc.mat = mat.data();
    sc.point_lights = sc.n_pl ? pl.data() : nullptr;
    sc.targets_sphere = sc.n_tg ? tg.data() : nullptr;
    sc.targets_obj = sc.n_tg ? tg_obj.data() : nullptr;
    return SC_OK;
}

// mean ms of two runs of the batch with tuning t (after one untimed run)
static sc_status time_batch(sc_ctx* ctx, uint32_t n, const sc_batch_item* items, const sc_tune& t, float* ms) {
    sc_batch* b = nullptr;
    SC_TRY(sc_batch_create(ctx, n, items, &t, &b));
    hipEvent_t e0 = nullptr, e1 = nullptr;
    sc_status s = SC_OK;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) s = set_error(SC_EDEVICE, "event");
    if (s == SC_OK) s = sc_batch_run(ctx, b);
    if (s == SC_OK && hipEventRecord(e0, ctx->c.stream) != hipSuccess) s = set_error(SC_EDEVICE, "event record");
    for (int r = 0; r < 2 && s == SC_OK; ++r) s = sc_batch_run(ctx, b);
    if (s == SC_OK && hipEventRecord(e1, ctx->c.stream) != hipSuccess) s = set_error(SC_EDEVICE, "event record");
    if (s == SC_OK && hipEventSynchronize(e1) != hipSuccess) s = set_error(SC_EDEVICE, "batch run failed");
    if (s == SC_OK && hipEventElapsedTime(ms, e0, e1) != hipSuccess) s = set_error(SC_EDEVICE, "event time");
    if (s == SC_OK) *ms *= 0.5f;
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    sc_batch_free(b);
    return s;
}

sc_status sc_autotune(sc_ctx* ctx, uint32_t n, const sc_batch_item* items, sc_tune* out) {
    if (!ctx || !items || !out) return set_error(SC_EINVAL, "ctx, items or out is NULL");
    SC_TRY(check_batch_items(ctx, n, items));
    // reduced copies: 1 sample per pixel, 1/8 of the photons (at least 64)
    std::vector<sc_batch_item> red(items, items + n);
    for (auto& it : red) {
        it.spp = 1;
        if (it.n_photons) it.n_photons = std::max<uint64_t>(64, it.n_photons / 8);
    }
    sc_tune best{128, 8, 64, 1, 256, 8};
    float best_ms = 0.0f;
    auto trial = [&](const sc_tune& t, const std::vector<sc_batch_item>& its, float* ms) -> sc_status {
        const sc_status s = time_batch(ctx, n, its.data(), t, ms);
        if (s != SC_OK)
            return set_error(SC_EABORTED, std::string("autotune candidate {") + std::to_string(t.block_size) + ", " +
                                              std::to_string(t.blocks_per_cu) + ", " + std::to_string(t.px_per_item) +
                                              ", " + std::to_string(t.ph_per_item) + "} failed: " + sc_last_error());
        return SC_OK;
    };
    SC_TRY(trial(best, red, &best_ms));
    for (uint32_t bs : {64u, 128u, 256u})
        for (uint32_t bpc : {2u, 4u, 8u}) {
            sc_tune t = best;
            t.block_size = bs;
            t.blocks_per_cu = bpc;
            float ms = 0.0f;
            SC_TRY(trial(t, red, &ms));
            if (ms < best_ms) { best_ms = ms; best = t; }
        }
    for (uint32_t px : {64u, 128u, 256u, 512u}) {
        sc_tune t = best;
        t.px_per_item = px;
        float ms = 0.0f;
        SC_TRY(trial(t, red, &ms));
        if (ms < best_ms) { best_ms = ms; best = t; }
    }
    for (uint32_t ph : {64u, 256u, 1024u, 4096u}) {
        sc_tune t = best;
        t.ph_per_item = ph;
        float ms = 0.0f;
        SC_TRY(trial(t, red, &ms));
        if (ms < best_ms) { best_ms = ms; best = t; }
    }
    // BVH width: the items' trees against 4-wide trees of the same scenes
    const uint32_t own = items[0].bvh->b.width;
    const uint32_t other = own == 8 ? 4u : 8u;
    std::vector<sc_bvh*> alt(n, nullptr);
    sc_status s = SC_OK;
    for (uint32_t i = 0; i < n && s == SC_OK; ++i) {
        sc_scene sc;
        std::vector<sc_material> mat;
        std::vector<float> pl, tg;
        std::vector<uint32_t> tgo;
        s = scene_of_bvh(items[i].bvh->b, sc, mat, pl, tg, tgo);
        const sc_bvh_opts o{other, items[i].bvh->b.leaf_max};
        if (s == SC_OK) s = sc_build_bvh(ctx, &sc, &o, &alt[i]);
        red[i].bvh = alt[i];
    }
    float ms = 0.0f;
    if (s == SC_OK) s = trial(best, red, &ms);
    for (sc_bvh* b : alt)
        if (b) sc_bvh_free(b);
    if (s != SC_OK) return s == SC_EABORTED ? s : set_error(SC_EABORTED, std::string("autotune: ") + sc_last_error());
    best.bvh_width = ms < best_ms ? other : own;
    best.use_graph = 1;
    *out = best;
    return SC_OK;
}

sc_status sc_unet_create(sc_ctx* ctx, const uint32_t* widths, uint32_t levels, sc_unet** out) {
    if (!ctx || !widths || !out) return set_error(SC_EINVAL, "ctx, widths or out is NULL");
    *out = nullptr;
    sc_unet* n = new (std::nothrow) sc_unet();
    if (!n) return set_error(SC_ENOMEM, "host allocation failed");
    sc_status s = scl::unet_create(&ctx->c, widths, levels, &n->u);
    if (s == SC_OK && hipStreamSynchronize(ctx->c.stream) != hipSuccess) s = set_error(SC_EDEVICE, "init failed");
    if (s != SC_OK) {
        delete n;
        return s;
    }
    *out = n;
    return SC_OK;
}

sc_status sc_unet_free(sc_unet* net) {
    if (!net) return set_error(SC_EINVAL, "net is NULL");
    if (net->u.ctx) (void)hipStreamSynchronize(net->u.ctx->stream);
    scl::detach(&net->u.ctx);
    delete net;
    return SC_OK;
}

sc_status sc_unet_num_params(const sc_unet* net, uint64_t* n) {
    if (!net || !n) return set_error(SC_EINVAL, "net or n is NULL");
    *n = net->u.n_params;
    return SC_OK;
}

sc_status sc_unet_set_params(sc_unet* net, const float* host) {
    if (!net || !host) return set_error(SC_EINVAL, "net or params is NULL");
    scl::Unet& u = net->u;
    if (!u.ctx) return set_error(SC_EINVAL, "the network's context was destroyed");
    SC_HIP(hipStreamSynchronize(u.ctx->stream));
    SC_HIP(hipMemcpy(u.theta.p, host, 4 * u.n_params, hipMemcpyHostToDevice));
    SC_HIP(hipMemset(u.m.p, 0, 4 * u.n_params));
    SC_HIP(hipMemset(u.v.p, 0, 4 * u.n_params));
    u.step = 0;
    SC_TRY(scl::unet_refresh(&u));
    SC_HIP(hipStreamSynchronize(u.ctx->stream));
    return SC_OK;
}

sc_status sc_unet_get_params(sc_unet* net, float* host) {
    if (!net || !host) return set_error(SC_EINVAL, "net or params is NULL");
    if (!net->u.ctx) return set_error(SC_EINVAL, "the network's context was destroyed");
    SC_HIP(hipStreamSynchronize(net->u.ctx->stream));
    SC_HIP(hipMemcpy(host, net->u.theta.p, 4 * net->u.n_params, hipMemcpyDeviceToHost));
    return SC_OK;
}

static sc_status check_shape(const scl::Unet& u, uint32_t n, uint32_t w, uint32_t h) {
    const uint32_t m = 1u << (u.widths.size() - 1);
    if (n == 0 || w == 0 || h == 0) return set_error(SC_EINVAL, "empty batch");
    if (w % m || h % m) return set_error(SC_EINVAL, "w and h must be multiples of 2^(levels-1)");
    if ((uint64_t)n * w * h > (1ull << 28)) return set_error(SC_EUNSUPPORTED, "batch too large");
    return SC_OK;
}

sc_status sc_unet_forward(sc_ctx* ctx, sc_unet* net, const float* feat, uint32_t n, uint32_t w, uint32_t h,
                          float* pred) {
    if (!ctx || !net || !feat || !pred) return set_error(SC_EINVAL, "NULL argument");
    if (!net->u.ctx) return set_error(SC_EINVAL, "the network's context was destroyed");
    scl::Unet& u = net->u;
    SC_TRY(check_shape(u, n, w, h));
    SC_TRY(scl::unet_prepare(&u, n, h, w));
    SC_TRY(scl::unet_pack_input(&u, feat));
    SC_TRY(scl::unet_forward_packed(&u));
    SC_HIP(hipMemcpyAsync(pred, u.pred.p, 12 * (size_t)n * w * h, hipMemcpyDeviceToDevice, ctx->c.stream));
    return SC_OK;
}

sc_status sc_unet_backward(sc_ctx* ctx, sc_unet* net, const float* dpred, float* grad) {
    if (!ctx || !net || !dpred || !grad) return set_error(SC_EINVAL, "NULL argument");
    if (!net->u.ctx) return set_error(SC_EINVAL, "the network's context was destroyed");
    scl::Unet& u = net->u;
    if (!u.acts.p || !u.cat_valid) return set_error(SC_EINVAL, "sc_unet_backward needs a preceding sc_unet_forward");
    SC_TRY(scl::unet_pack_dpred(&u, dpred));
    SC_TRY(scl::unet_backward_packed(&u));
    SC_HIP(hipMemcpyAsync(grad, u.grad.p, 4 * u.n_params, hipMemcpyDeviceToDevice, ctx->c.stream));
    return SC_OK;
}

sc_status sc_unet_train_step(sc_ctx* ctx, sc_unet* net, const float* feat, const float* target, uint32_t n,
                             uint32_t w, uint32_t h, float lr, float* loss) {
    if (!ctx || !net || !feat || !target) return set_error(SC_EINVAL, "NULL argument");
    if (!net->u.ctx) return set_error(SC_EINVAL, "the network's context was destroyed");
    if (!(lr > 0.0f)) return set_error(SC_EINVAL, "lr must be > 0");
    scl::Unet& u = net->u;
    SC_TRY(check_shape(u, n, w, h));
    SC_TRY(scl::unet_prepare(&u, n, h, w));
    SC_TRY(scl::unet_pack_input(&u, feat));
    SC_TRY(scl::unet_forward_packed(&u));
    SC_TRY(scl::unet_loss(&u, target, u.loss.as<float>()));
    SC_TRY(scl::unet_backward_packed(&u));
    SC_TRY(scl::unet_adam(&u, lr));
    if (loss) {
        float s = 0.0f;
        SC_HIP(hipMemcpyAsync(&s, u.loss.p, 4, hipMemcpyDeviceToHost, ctx->c.stream));
        SC_HIP(hipStreamSynchronize(ctx->c.stream));
        *loss = s / (float)((double)n * w * h * 3);
    }
    return SC_OK;
}

static sc_status check_layer(sc_unet* net, uint32_t layer, uint32_t n, uint32_t h, uint32_t w) {
    if (!net->u.ctx) return set_error(SC_EINVAL, "the network's context was destroyed");
    if (layer >= net->u.layers.size()) return set_error(SC_EINVAL, "layer index out of range");
    if (n == 0 || w == 0 || h == 0) return set_error(SC_EINVAL, "empty batch");
    if ((uint64_t)n * w * h > (1ull << 26)) return set_error(SC_EUNSUPPORTED, "batch too large");
    return SC_OK;
}

sc_status sc_unet_layer_forward(sc_ctx* ctx, sc_unet* net, uint32_t layer, const float* X, uint32_t n, uint32_t h,
                                uint32_t w, int32_t relu, float* Y) {
    if (!ctx || !net || !X || !Y) return set_error(SC_EINVAL, "NULL argument");
    SC_TRY(check_layer(net, layer, n, h, w));
    return scl::unet_layer_forward(&net->u, layer, X, n, h, w, relu ? 1 : 0, Y);
}

sc_status sc_unet_layer_backward(sc_ctx* ctx, sc_unet* net, uint32_t layer, const float* X, const float* dZ,
                                 uint32_t n, uint32_t h, uint32_t w, float* dX, float* dW) {
    if (!ctx || !net || !X || !dZ || !dW) return set_error(SC_EINVAL, "NULL argument");
    SC_TRY(check_layer(net, layer, n, h, w));
    return scl::unet_layer_backward(&net->u, layer, X, dZ, n, h, w, dX, dW);
}

sc_status sc_unet_features(sc_ctx* ctx, const sc_aov* in, uint32_t w, uint32_t h, float* feat) {
    if (!ctx || !in || !in->rgb || !feat) return set_error(SC_EINVAL, "NULL argument");
    if (w == 0 || h == 0) return set_error(SC_EINVAL, "empty image");
    if ((uint64_t)w * h > (1ull << 28)) return set_error(SC_EUNSUPPORTED, "image too large");
    return scl::features_f32(&ctx->c, *in, w, h, feat);
}

sc_status sc_denoise(sc_ctx* ctx, sc_unet* net, const sc_aov* in, uint32_t w, uint32_t h, float* out_rgb) {
    if (!ctx || !net || !in || !in->rgb || !out_rgb) return set_error(SC_EINVAL, "NULL argument");
    if (!net->u.ctx) return set_error(SC_EINVAL, "the network's context was destroyed");
    if (w == 0 || h == 0) return set_error(SC_EINVAL, "empty image");
    scl::Unet& u = net->u;
    const uint32_t m = 1u << (u.widths.size() - 1);
    const uint32_t W = (w + m - 1) / m * m, H = (h + m - 1) / m * m;
    SC_TRY(check_shape(u, 1, W, H));
    SC_TRY(scl::unet_prepare(&u, 1, H, W));
    SC_TRY(scl::unet_features(&u, *in, w, h));
    SC_TRY(scl::unet_forward_packed(&u, false));
    SC_TRY(scl::unet_output_rgb(&u, w, h, out_rgb));
    return SC_OK;
}

}  // extern "C"
