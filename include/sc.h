/*
 * sc.h -- C ABI of the MI355X (gfx950) SuperCaustics rendering library.
 *
 * The library renders the outputs that the SuperCaustics paper defines for
 * scenes with transparent objects (arXiv 2107.11008):
 *   - a spectral image with refraction, dispersion, specular reflection and
 *     caustics (Abstract; Sec. I; caustic softness, Fig. 4);
 *   - depth, the distance from the camera to the surface seen in a pixel,
 *     raw and normalised over a 10 m range (Sec. III-D-1);
 *   - world- and camera-space surface normals (Sec. III-D-2);
 *   - the object mask: the object each pixel sees first, and whether it is
 *     transparent (Sec. III-D-3, pixel-perfect labels);
 *   - a caustic map on a receiver plane (the photon side of the caustic
 *     ground truth of Sec. III-D-6).
 * The paper obtains these from a game engine's hardware ray tracing; here
 * every step runs in hand-written HIP kernels: a BVH8 builder, a wavefront
 * path tracer (ray generation, closest- and any-hit traversal, material
 * sort and compaction, dielectric and diffuse shading), photon tracing with
 * fixed-point atomics into the caustic map, the ground-truth writer and the
 * film resolve.
 *
 * Conventions
 *   - Every call returns sc_status: 0 on success, a negative SC_E* code on
 *     failure; sc_last_error() returns a thread-local message for the last
 *     failure.  No C++ exception crosses this boundary.
 *   - Buffers named "device" are device pointers owned by the caller; they
 *     must stay valid until the stream has passed the call (and, for the
 *     scene arrays, for the lifetime of the sc_bvh built from them).
 *     Arrays named "host" are read during the call only.
 *   - Handles (sc_bvh, sc_pmap, sc_unet, sc_batch) may be freed before or
 *     after the context they were made on.  After that context is destroyed
 *     a BVH can still be rendered from by other contexts on its device;
 *     calls that need the handle's own context fail with EINVAL.
 *   - All kernels run on the context's stream.  Calls return after
 *     enqueueing, except sc_build_bvh (sizes its allocations), calls that
 *     fill host statistics, and sc_sync/sc_get_counters.  Argument errors
 *     are reported synchronously; device faults surface at sc_sync.
 *   - Units are metres, the world is right-handed with +z up.  Object id 0
 *     means "no hit"; every triangle belongs to an object id >= 1.
 *   - Floating point: IEEE binary32, no contraction, correctly rounded
 *     division and square root.  Given the same inputs and seeds the
 *     traced paths are bit-identical to the CPU oracle of the repository.
 */
#ifndef SC_H
#define SC_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SC_ABI_VERSION 6u

typedef int32_t sc_status;
#define SC_OK 0
#define SC_EINVAL (-1)        /* invalid argument (null, size, range) */
#define SC_ENOMEM (-2)        /* device allocation failed */
#define SC_EDEVICE (-3)       /* HIP runtime error */
#define SC_EUNSUPPORTED (-4)  /* valid but unsupported request */
#define SC_EABORTED (-5)      /* a multi-step operation stopped at a failed step; outputs unchanged */

typedef struct sc_ctx sc_ctx;
typedef struct sc_bvh sc_bvh;

/* Materials: one per object id.  DIFFUSE is Lambertian (two-sided);
 * DIELECTRIC is smooth glass with n(lambda) = cauchy_a + cauchy_b /
 * lambda_um^2 (dispersion, Abstract); EMISSIVE emits radiance `le` from
 * its front face (counter-clockwise winding).
 *
 * Glass colour and thickness (scene variations of Sec. III-C): a segment
 * of length t inside a dielectric keeps exp(-sigma(lambda) t) of its
 * weight (Beer-Lambert), sigma given in 1/m at 450, 550 and 650 nm,
 * piecewise linear in lambda between them and constant outside; all zero
 * is clear glass.  Nested and overlapping dielectrics follow Schmidt and
 * Budge (J. Graphics Tools 7(2), 2002): each camera path and photon keeps
 * the set of dielectrics it is inside (at most 4); the medium at a point
 * is the member of highest `priority` (ties: larger object id); a surface
 * is an interface only where its object is that medium on the inner side,
 * and there the outer index is that of the next medium (air if none);
 * other surfaces are crossed unchanged.  Cameras and lights are in air.
 * Glass roughness (Sec. III-C): `roughness` > 0 is the GGX width alpha of
 * a microfacet interface (Walter et al., EGSR 2007): a microfacet normal
 * drawn from the distribution of visible normals (Heitz, JCGT 2018),
 * reflection or refraction at it chosen by its Fresnel reflectance, path
 * weight G1(o) <= 1 (Smith); 0 is smooth glass. */
#define SC_MAT_DIFFUSE 0u
#define SC_MAT_DIELECTRIC 1u
#define SC_MAT_EMISSIVE 2u
#define SC_ALBEDO_CONST 0u    /* rho_a */
#define SC_ALBEDO_CHECKER 1u  /* 1 m squares on x,y: rho_a where floor(x)+floor(y) is even, else rho_b */
#define SC_ALBEDO_TEXTURE 2u  /* the scene texture, nearest texel over its rectangle */
#define SC_ALBEDO_TEXTURE_RGB 3u /* the scene's RGB texture, nearest texel: reflectance B at 450 nm,
                                    G at 550 nm, R at 650 nm, linear in lambda between them and
                                    constant outside; grey albedo output = (R + G + B) / 3 */

typedef struct {
    uint32_t type, albedo_mode;
    float rho_a, rho_b;
    float cauchy_a, cauchy_b;
    float le;
    uint32_t priority;  /* dielectric nesting priority */
    float sigma[3];     /* dielectric absorption (1/m) at 450, 550, 650 nm; finite, >= 0 */
    float roughness;    /* dielectric GGX alpha in [0, 1]; 0 = smooth */
} sc_material; /* 48 bytes */

typedef struct {
    const float* V;          /* device [nv][3] vertex positions */
    const uint32_t* I;       /* device [nt][3] vertex indices */
    const float* VN;         /* device [nv][3] unit vertex normals, or NULL for flat shading */
    const uint32_t* tri_obj; /* device [nt] object id of each triangle, 1..n_mat-1 */
    uint32_t nv, nt;
    const sc_material* mat;  /* host [n_mat], n_mat <= 65536; index = object id, row 0 unused */
    uint32_t n_mat;
    const float* point_lights; /* host [n_pl][4]: x, y, z, intensity (W/sr, flat spectrum) */
    uint32_t n_pl;
    const uint32_t* targets_obj; /* host [n_tg] object ids that photons are aimed at */
    const float* targets_sphere; /* host [n_tg][4]: bounding sphere cx, cy, cz, r */
    uint32_t n_tg;
    const float* tex;          /* device [tex_h][tex_w] grey albedo, or NULL */
    uint32_t tex_w, tex_h;
    float tex_x0, tex_y0, tex_ext_u, tex_ext_v; /* texture rectangle on x,y */
    uint32_t recv_obj;         /* receiver object of the caustic map, 0 = none */
    uint32_t recv_wc, recv_hc; /* caustic-map cells along x and y */
    float recv_x0, recv_y0, recv_ext_u, recv_ext_v; /* receiver rectangle on x,y */
    const float* tex_rgb;      /* device [tex_h][tex_w][3] RGB albedo, or NULL; same size and
                                  rectangle as tex (which may then be NULL) */
} sc_scene;

typedef struct {
    uint32_t width;     /* 4 or 8 (children per node); 0 = 8 */
    uint32_t leaf_max;  /* triangles per leaf, 1..8; 0 = 4 */
} sc_bvh_opts;

typedef struct {
    uint32_t width, leaf_max;
    uint32_t n_nodes, depth;   /* wide nodes and levels below the root */
    uint64_t node_bytes, tri_bytes;
    uint32_t max_stack;        /* traversal stack entries a ray can need */
} sc_bvh_info;

/* Pinhole camera: the ray through film point (sx, sy) in [-1,1]^2 (row 0
 * at the top) has direction fwd + sx*right + sy*up, normalised; right and
 * up already carry tan(vfov/2) and the aspect ratio. */
typedef struct {
    float eye[3], fwd[3], right[3], up[3];
    uint32_t w, h;
} sc_camera;

/* Wavelength sampling.  FIXED: k = 1 or 3 slots with wavelengths nm[]
 * (channel order R, G, B when k = 3); every (pixel, sample) traces k paths;
 * the caustic map has k channels.  UNIFORM: one path per (pixel, sample)
 * with lambda uniform in [lo, hi]; Gaussian sensor curves (40 nm wide at
 * 650/550/450 nm, mean 1 over [lo, hi]) map it to RGB; the caustic map
 * has `bins` spectral bins. */
#define SC_WL_FIXED 0u
#define SC_WL_UNIFORM 1u
typedef struct {
    uint32_t mode, k;
    float nm[4];
    float lo, hi;
    uint32_t bins;
} sc_wavelengths;

/* Outputs of sc_render, each a device array or NULL (not written):
 *   rgb        [h][w][3] f32  linear radiance, mean over samples
 *   obj        [h][w]    u32  object id of the first surface (0 = miss)
 *   trans      [h][w]    u8   1 if that object is DIELECTRIC
 *   tri        [h][w]    u32  triangle index (0xffffffff = miss)
 *   depth      [h][w]    f32  distance along the unit ray (+inf = miss)
 *   depthn     [h][w]    f32  min(depth / 10 m, 1)
 *   normal     [h][w][3] f32  world-space shading normal facing the camera
 *   normal_cam [h][w][3] f32  the same in camera space (x right, y up, z back)
 *   albedo     [h][w]    f32  diffuse albedo (glass 1, emitter 0, miss 0)
 * The last seven come from the ray through the pixel centre. */
typedef struct {
    float* rgb;
    uint32_t* obj;
    uint8_t* trans;
    uint32_t* tri;
    float* depth;
    float* depthn;
    float* normal;
    float* normal_cam;
    float* albedo;
} sc_aov;

/* Photon outcome statistics (host struct filled by sc_trace_photons when
 * requested; the call then synchronises). */
#define SC_PH_DEPOSITED 0
#define SC_PH_OUTSIDE 1
#define SC_PH_DIRECT 2
#define SC_PH_ELSEWHERE 3
#define SC_PH_ESCAPED 4
#define SC_PH_ABSORBED 5
#define SC_PH_TRUNCATED 6
#define SC_PH_LOST 7
#define SC_PH_EMIT_DEAD 8
typedef struct {
    double flux[9];
    uint64_t count[9];
    uint64_t segments;
} sc_photon_stats;

/* Cumulative counters of a context (sc_get_counters synchronises). */
typedef struct {
    uint64_t rays_closest;    /* closest-hit queries (camera, ground truth, photons) */
    uint64_t rays_shadow;     /* any-hit queries */
    uint64_t node_visits;     /* wide nodes fetched by the staged closest-hit kernel (visit counting on) */
    uint64_t tri_tests;       /* triangles tested by the staged closest-hit kernel (visit counting on) */
    uint64_t closest_launches;/* staged closest-hit kernel launches timed (profiling on) */
    double closest_ms;        /* their summed duration from HIP events (profiling on) */
    uint64_t closest_rays_timed; /* closest-hit rays traced by the staged kernel (the rest of
                                  * rays_closest by the per-lane path finishing kernels) */
    uint64_t finish_launches; /* photon path finishing kernel launches timed (profiling on) */
    double finish_ms;         /* their summed duration from HIP events (profiling on) */
    uint64_t finish_paths;    /* photon paths the finishing kernel took over */
    uint64_t finish_rays;     /* closest-hit rays it traced for them */
    uint64_t finish_node_visits; /* wide nodes it fetched (visit counting on) */
    uint64_t finish_tri_tests;   /* triangles it tested (visit counting on) */
    uint64_t anyhit_launches;    /* any-hit kernel launches timed (profiling on) */
    double anyhit_ms;            /* their summed duration from HIP events (profiling on) */
    uint64_t anyhit_rays;        /* shadow rays the any-hit kernel traced (the rest of rays_shadow by
                                  * the camera path finishing kernel) */
    uint64_t anyhit_node_visits; /* wide nodes it fetched (visit counting on) */
    uint64_t anyhit_tri_tests;   /* triangles it tested (visit counting on) */
    uint64_t cam_finish_launches;  /* camera path finishing kernel launches timed (profiling on) */
    double cam_finish_ms;          /* their summed duration from HIP events (profiling on) */
    uint64_t cam_finish_paths;     /* camera paths it took over */
    uint64_t cam_finish_rays;      /* closest-hit rays it traced for them */
    uint64_t cam_finish_shadow_rays; /* shadow rays it traced for them */
    uint64_t cam_finish_node_visits; /* wide nodes both kinds of ray fetched (visit counting on) */
    uint64_t cam_finish_tri_tests;   /* triangles both kinds tested (visit counting on) */
} sc_counters;

#define SC_OPT_COUNT_VISITS 1 /* 0/1: the traversal kernels count node and triangle visits */
#define SC_OPT_PROFILE 2      /* 0/1: time every traversal launch (closest hit, any hit, path
                               * finishing) with HIP events */
#define SC_OPT_QUEUE_CAP 3    /* camera paths per wavefront chunk (1024..2^30, default 1<<27) */
#define SC_OPT_STAGED_DEPTH 4 /* camera-path bounces traced as one launch per stage before the
                               * remaining paths are each finished by one lane (default 2; 0 = none,
                               * every path finished by one lane from its camera ray; a value of
                               * max_depth or more = every bounce staged); any value gives the same
                               * output bit for bit */
#define SC_OPT_CONV_BIG_TILE 5 /* U-Net 3x3 convolutions use 12-row pixel tiles when a layer has at
                                * least this many of them (default 2048; 0 = always), 8-row tiles
                                * otherwise; any value gives the same output bit for bit */
#define SC_OPT_PHOTON_STAGED_DEPTH 6 /* the same switch for photon paths (default 0: every photon
                                      * is finished by one lane from its emission) */
#define SC_OPT_PHOTON_CAP 7   /* photons per photon-pass chunk (1024..2^28, default 1<<24) */
#define SC_OPT_BVH_BUILDER 8  /* tree of later sc_build_bvh / sc_bvh_rebuild calls: 0 = binary radix
                               * tree over 36-bit Morton codes (Karras, HPG 2012), 1 = parallel
                               * locally-ordered clustering (Meister and Bittner, IEEE TVCG 2018),
                               * 2 = clustering from 2^20 triangles up, radix tree below (default);
                               * both trees are collapsed to the same wide-node layout and give
                               * the same hits bit for bit */
#define SC_OPT_TRACE_BLOCKS 9 /* blocks of 128 threads per compute unit in the persistent traversal
                               * grids (closest hit, any hit, path finishing; 1..16, default 8: what
                               * the chip holds at once).  Lower values leave room for work on
                               * another stream at the cost of this context's traversal rate; any
                               * value gives the same output bit for bit */

uint32_t sc_abi_version(void);
const char* sc_last_error(void);

/* Context on HIP device `device` using stream `hip_stream` (a hipStream_t,
 * NULL = the null stream).  The context owns its work buffers. */
sc_status sc_create(int device, void* hip_stream, sc_ctx** out);
sc_status sc_destroy(sc_ctx* ctx);
sc_status sc_set_stream(sc_ctx* ctx, void* hip_stream);
sc_status sc_set_option(sc_ctx* ctx, int32_t option, int64_t value);
sc_status sc_sync(sc_ctx* ctx);
sc_status sc_get_counters(sc_ctx* ctx, sc_counters* out);
sc_status sc_reset_counters(sc_ctx* ctx);

/* Build the wide BVH of a scene on the GPU (Morton codes, bitonic sort,
 * radix-tree hierarchy, bottom-up bounds, greedy collapse to `width`
 * children) and prepare its light and material tables.  The handle
 * references the scene's device arrays.  Synchronises.  EINVAL on null
 * pointers, nt == 0, an object id outside [1, n_mat) or an unknown
 * material; EUNSUPPORTED if the tree is too deep for the traversal stack. */
sc_status sc_build_bvh(sc_ctx* ctx, const sc_scene* scene, const sc_bvh_opts* opts, sc_bvh** out);
/* Rebuild an existing handle for `scene` (the same scene with moved
 * vertices, or another one) with the options it was built with, as
 * sc_build_bvh would, reusing the handle's device memory where it is large
 * enough: the per-frame rebuild of dynamic geometry.  Work already enqueued
 * on the context's stream that reads the old tree finishes first (stream
 * order).  Synchronises.  EINVAL on null pointers, a handle of another
 * context or an invalid scene (as sc_build_bvh); after any failure the
 * handle holds no tree and tracing calls on it fail with EINVAL until a
 * rebuild succeeds. */
sc_status sc_bvh_rebuild(sc_ctx* ctx, sc_bvh* bvh, const sc_scene* scene);
sc_status sc_bvh_get_info(const sc_bvh* bvh, sc_bvh_info* out);
sc_status sc_bvh_free(sc_bvh* bvh);
/* Copy the built structure to host memory for inspection (synchronises):
 * nodes_host receives node_bytes bytes (256-byte nodes: child boxes as
 * lo_x[8], hi_x[8], lo_y[8], hi_y[8], lo_z[8], hi_z[8], then child[8];
 * child 0xffffffff = empty, bit 31 set = leaf of (bits 28..30) + 1
 * triangles starting at bits 0..27, else a node index); tris_host receives
 * tri_bytes bytes (per leaf-ordered triangle three float4: vertex 0 with
 * the triangle index in .w as bits, vertex 1, vertex 2).  Either may be
 * NULL. */
sc_status sc_bvh_export(const sc_bvh* bvh, void* nodes_host, void* tris_host);

/* Closest hit of n rays (device O, D: [n][3], D unit length): the
 * lexicographic minimum of (t, triangle index) over all triangles with
 * t > 0 under the watertight test of Woop et al. (JCGT 2013).  Outputs
 * device t, prim (0xffffffff and +inf on a miss), barycentrics u, v of
 * vertices 1 and 2 (u, v may be NULL). */
sc_status sc_trace_rays(sc_ctx* ctx, const sc_bvh* bvh, uint32_t n, const float* O, const float* D,
                        float* t, uint32_t* prim, float* u, float* v);
/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the
 * closest hits of sc_trace_rays, bit for bit, without any allocation by
 * the library.  The rays are staged in a fixed array of device memory that
 * the library holds on every GPU it runs on until the process ends
 * (6 x 4 MiB: at most sc_trace_rays_noalloc_max() = 2^20 rays per call;
 * more is EINVAL, reported before anything is enqueued).  Every call on a
 * GPU shares that GPU's array, so calls that overlap on one GPU (other
 * streams, other contexts, other threads) race; calls in stream order on
 * one stream do not.  Arguments and outputs as sc_trace_rays. */
sc_status sc_trace_rays_noalloc(sc_ctx* ctx, const sc_bvh* bvh, uint32_t n, const float* O, const float* D,
                                float* t, uint32_t* prim, float* u, float* v);
uint32_t sc_trace_rays_noalloc_max(void);
/* Any hit with 0 < t < tmax[i], ignoring triangle excl[i] (excl may be
 * NULL); occluded[i] = 0/1.  All device arrays. */
sc_status sc_occluded(sc_ctx* ctx, const sc_bvh* bvh, uint32_t n, const float* O, const float* D,
                      const float* tmax, const uint32_t* excl, uint8_t* occluded);

/* Photon pass (the caustic side of the ground truth, Sec. III-D-6):
 * n_photons photons from the lights aimed at the photon target spheres,
 * carried through dielectrics (Cauchy IOR, Fresnel, total internal
 * reflection) and stored on the receiver at the first diffuse hit after at
 * least one dielectric event.  caustic_map: device f32 [recv_hc][recv_wc][C]
 * (C = k for FIXED, bins for UNIFORM) holding flux per cell; overwritten.
 * count_map: device u32 of the same shape with deposits per cell, or NULL.
 * stats: host, or NULL (non-NULL synchronises).  EINVAL if the scene has
 * no receiver, max_depth == 0 or the wavelength setting is invalid. */
sc_status sc_trace_photons(sc_ctx* ctx, const sc_bvh* bvh, uint64_t n_photons, uint32_t max_depth,
                           const sc_wavelengths* wl, uint64_t seed, float* caustic_map, uint32_t* count_map,
                           sc_photon_stats* stats);

/* General photon map (caustics on every diffuse surface, Sec. III-D-6):
 * the photon pass of sc_trace_photons, but every photon that reaches a
 * diffuse surface of any object after at least one dielectric event is
 * stored there (position, geometric normal on its side, flux, map
 * channel, photon index) in a hashed grid of cells 2.25 * radius wide
 * (offset by half a cell).  The
 * irradiance of channel c at a surface point x with facing normal n is
 * the flux of the stored photons of channel c within `radius` of x on the
 * same side (n_p . n > 0), over pi radius^2 (Jensen's density estimate
 * with a fixed radius).  The sum is exact and order independent: each flux
 * is taken as round(phi 2^S) in 64-bit fixed point, 2^S the largest power
 * of two with n_stored * max(phi) * 2^S <= 2^62, and
 * E = (float)(sum * (1 / (2^S pi radius^2))) in double.
 * Up to 2^24 photons; radius > 0 and no stored coordinate beyond about
 * 2^16 * 2.25 * radius from the origin (else EUNSUPPORTED).  Synchronises.
 * stats: host, or NULL.  The handle owns its device memory until
 * sc_pmap_free. */
typedef struct sc_pmap sc_pmap;
typedef struct {
    uint64_t n_stored;   /* photons stored */
    float radius;
    uint32_t channels;   /* as the wavelength setting of the pass */
    double scale;        /* 2^S */
    uint32_t buckets;    /* hash table size (a power of two) */
    uint64_t bytes;      /* device memory held */
} sc_pmap_info;
sc_status sc_pmap_trace(sc_ctx* ctx, const sc_bvh* bvh, uint64_t n_photons, uint32_t max_depth,
                        const sc_wavelengths* wl, uint64_t seed, float radius, sc_pmap** out,
                        sc_photon_stats* stats);
/* sc_pmap_trace into an existing handle, reusing its device memory where
 * it is large enough (the per-frame rebuild).  After a failure the handle
 * holds no map: gathers and renders with it fail with EINVAL until a
 * rebuild succeeds. */
sc_status sc_pmap_retrace(sc_ctx* ctx, const sc_bvh* bvh, uint64_t n_photons, uint32_t max_depth,
                          const sc_wavelengths* wl, uint64_t seed, float radius, sc_pmap* pm,
                          sc_photon_stats* stats);
sc_status sc_pmap_get_info(const sc_pmap* pm, sc_pmap_info* out);
/* Host copies of the stored photons in photon-index order (any may be
 * NULL): pos [n][3], nrm [n][3], phi [n], channel [n], photon [n]. */
sc_status sc_pmap_export(const sc_pmap* pm, float* pos, float* nrm, float* phi, uint32_t* channel,
                         uint64_t* photon);
/* Irradiance estimates at n device points P [n][3] with facing normals
 * N [n][3] for channels ch [n] into device E [n]. */
sc_status sc_pmap_gather(sc_ctx* ctx, const sc_pmap* pm, uint32_t n, const float* P, const float* N,
                         const uint32_t* ch, float* E);
sc_status sc_pmap_free(sc_pmap* pm);
/* sc_render with the caustic gather taken from the general photon map at
 * every diffuse vertex (instead of the receiver map).  EINVAL if the map's
 * channels differ from the wavelength setting's. */
sc_status sc_render_pmap(sc_ctx* ctx, const sc_bvh* bvh, const sc_camera* cam, uint32_t spp, uint32_t max_depth,
                         const sc_wavelengths* wl, uint64_t seed, const sc_pmap* pm, const sc_aov* out);

/* Render spp samples per pixel with at most max_depth surface hits per
 * path.  caustic_map: device map from sc_trace_photons with the same
 * wavelength setting, or NULL (caustic gather off).  With out->rgb NULL
 * only the ground truth of the pixel-centre rays is written.  The BVH is
 * only read: a context on the same device other than the one that built it
 * may render from it (on its own stream) while it is not being rebuilt.
 * EINVAL on spp == 0, max_depth == 0, w*h == 0, an invalid wavelength
 * setting or a NULL out. */
sc_status sc_render(sc_ctx* ctx, const sc_bvh* bvh, const sc_camera* cam, uint32_t spp, uint32_t max_depth,
                    const sc_wavelengths* wl, uint64_t seed, const float* caustic_map, const sc_aov* out);

/* sc_render gathering from a caustic map whose photon pass may still be
 * running on another stream (another context's sc_trace_photons): the
 * render's stream waits for map_ready (a hipEvent_t recorded on that
 * stream after the pass) only before its first kernel that reads the map,
 * the diffuse shading of the first bounce; camera ray generation, the
 * ground-truth rays and the first traversal overlap the photon pass.  The
 * output is that of sc_render with the finished map.  The event must be
 * recorded before this call (stream order, as hipStreamWaitEvent).  EINVAL
 * as sc_render, and on a NULL caustic_map or map_ready. */
sc_status sc_render_overlap(sc_ctx* ctx, const sc_bvh* bvh, const sc_camera* cam, uint32_t spp, uint32_t max_depth,
                            const sc_wavelengths* wl, uint64_t seed, const float* caustic_map, void* map_ready,
                            const sc_aov* out);

/* ------------------------------------------------------------------
 * Ground-truth passes over sc_render's buffers (Sec. III-D).  Each is a
 * plain per-pixel definition; device arrays [h][w].
 * ------------------------------------------------------------------ */
/* Local / non-local caustic mask (Sec. III-D-6): the luminance (Rec. 709:
 * (0.2126 R + 0.7152 G) + 0.0722 B) of a render with the caustic gather
 * minus that of the same render without it (same seeds, so the paths are
 * identical apart from the gathered light); mask = 0 if the difference is
 * <= threshold, 1 (local: the pixel's first surface is transparent, trans
 * may be NULL = never) or 2 (non-local) otherwise. */
sc_status sc_caustic_mask(sc_ctx* ctx, const float* rgb_with, const float* rgb_without, const uint8_t* trans,
                          uint32_t w, uint32_t h, float threshold, uint8_t* mask);
/* Outlines (Sec. III-D-4): out = 1 for a pixel of an object (obj != 0) whose
 * window of Chebyshev radius `thickness` (1..64, clipped at the image
 * border) contains another id; a band `thickness` pixels wide inside every
 * object edge. */
sc_status sc_outline(sc_ctx* ctx, const uint32_t* obj, uint32_t w, uint32_t h, uint32_t thickness, uint8_t* out);
/* Occlusion boundaries (Sec. III-D-5, depth discontinuities): out = 1 for a
 * pixel with finite depth d that has an 8-neighbour q with depth(q) - d >
 * rel_jump * d (the near side of the jump; a miss counts as infinitely
 * far). */
sc_status sc_occlusion_boundary(sc_ctx* ctx, const float* depth, uint32_t w, uint32_t h, float rel_jump,
                                uint8_t* out);

/* ------------------------------------------------------------------
 * Batched form: many scenes of uneven size rendered by persistent kernels
 * whose waves pull work items (64*m photons or pixels of one scene) from a
 * global counter; each lane follows its photon or its pixel's paths to the
 * end with the same per-path code as sc_trace_photons / sc_render, so every
 * output equals the one-scene result bit for bit.  The batch (clears,
 * photon pass, map conversion, rendering) is captured once in a hipGraph.
 * The paper's dataset is many such scenes (Sec. IV-A-2).
 * ------------------------------------------------------------------ */
typedef struct sc_batch sc_batch;

typedef struct {
    const sc_bvh* bvh;        /* scene and its BVH (built by sc_build_bvh) */
    sc_camera cam;
    uint32_t spp, max_depth;
    sc_wavelengths wl;
    uint64_t seed;            /* camera paths */
    uint64_t photon_seed;
    uint64_t n_photons;       /* 0: no photon pass; caustic_map (if not NULL) is then only gathered */
    float* caustic_map;       /* device [hc][wc][C], written by the photon pass; NULL with n_photons > 0
                                 = held by the batch */
    sc_aov out;               /* device outputs as in sc_render (NULL fields are skipped) */
} sc_batch_item;

typedef struct {
    uint32_t block_size;      /* threads per block: 64, 128 or 256 */
    uint32_t blocks_per_cu;   /* persistent blocks per compute unit, 1..32 */
    uint32_t px_per_item;     /* pixels per work item (the tile a wave takes): a multiple of 64, <= 4096 */
    uint32_t use_graph;       /* 1: capture in a hipGraph at creation, replay at every run */
    uint32_t ph_per_item;     /* photons per work item (the grain a wave takes from the photon queue): a
                                 multiple of 64, <= 65536; 0 = px_per_item */
    uint32_t bvh_width;       /* sc_autotune's choice of BVH width (4 or 8) for the items' trees;
                                 sc_batch_create ignores it (the trees are built by the caller) */
} sc_tune;

/* Prepare a batch (the items' device buffers must outlive it).  tune NULL
 * = {128, 8, 64, 1, 0, 8}.  EINVAL on an invalid item or tuning value. */
sc_status sc_batch_create(sc_ctx* ctx, uint32_t n, const sc_batch_item* items, const sc_tune* tune, sc_batch** out);
/* Run every photon pass and render of the batch (one graph launch). */
sc_status sc_batch_run(sc_ctx* ctx, sc_batch* batch);
sc_status sc_batch_free(sc_batch* batch);
/* create + run + free; synchronises. */
sc_status sc_render_batch(sc_ctx* ctx, uint32_t n, const sc_batch_item* items, const sc_tune* tune);
/* Autotuner of the batched form (the many-scene capture of Sec. IV-A-2):
 * chooses the persistent grid (block_size, blocks_per_cu), the pixel tile
 * (px_per_item), the photon queue grain (ph_per_item) and the BVH width
 * for this batch by timing candidates with HIP events on reduced copies
 * of it (1 sample per pixel, 1/8 of the photons, the items' own output
 * buffers, which hold unspecified values afterwards), one dimension at a
 * time from {128, 8, 64, 1, 256, 8}: the grid over {64, 128, 256} x {2, 4,
 * 8}, then the tile over {64, 128, 256, 512}, the grain over {64, 256,
 * 1024, 4096}, then width 4 (trees rebuilt from the items' scenes) against
 * the items' own trees.  No choice changes any output: the batch is the
 * one-scene result bit for bit for every setting.  out receives the
 * fastest setting (use_graph = 1).  Synchronises.  EINVAL on invalid
 * items (as sc_batch_create); SC_EABORTED when a candidate's run fails
 * (sc_last_error names it; out is left unchanged). */
sc_status sc_autotune(sc_ctx* ctx, uint32_t n, const sc_batch_item* items, sc_tune* out);

/* ------------------------------------------------------------------
 * Learned denoiser.  A U-Net (the network family the paper trains for
 * segmentation, Sec. IV-A-3; Ronneberger et al. 2015) maps a low-sample
 * render and its ground-truth buffers to a clean image.  Per level two 3x3
 * convolutions with ReLU; 2x2 max pooling down, nearest 2x upsampling and
 * skip concatenation up; a 1x1 output convolution predicting log(1 + rgb).
 * Input features per pixel (9): log(1+rgb) x3, albedo, world normal x3,
 * normalised depth, transparent bit.  Weights and activations are bfloat16
 * on the matrix cores with float accumulation; float master weights are
 * updated by Adam (beta 0.9/0.999, eps 1e-8); loss = mean |pred -
 * log(1 + target)|.
 *
 * Parameters are a float vector: layer by layer (encoder levels shallow to
 * deep, decoder levels deep to shallow, output layer), weights as
 * [cout][ky][kx][cin] followed by the biases.
 * ------------------------------------------------------------------ */
typedef struct sc_unet sc_unet;

/* widths[levels] channels per level, multiples of 16 (<= 256), 2 <= levels
 * <= 6; parameters start at zero (set them with sc_unet_set_params). */
sc_status sc_unet_create(sc_ctx* ctx, const uint32_t* widths, uint32_t levels, sc_unet** out);
sc_status sc_unet_free(sc_unet* net);
sc_status sc_unet_num_params(const sc_unet* net, uint64_t* n);
/* host float[n_params] in and out; set resets the Adam moments and step. */
sc_status sc_unet_set_params(sc_unet* net, const float* host_params);
sc_status sc_unet_get_params(sc_unet* net, float* host_params);
/* Forward pass of n images: device feat [n][h][w][9] f32 -> device pred
 * [n][h][w][3] f32 (log domain).  h and w must be multiples of
 * 2^(levels-1).  Keeps the activations for sc_unet_backward. */
sc_status sc_unet_forward(sc_ctx* ctx, sc_unet* net, const float* feat, uint32_t n, uint32_t w, uint32_t h,
                          float* pred);
/* Gradient of a loss w.r.t. all parameters, given device dpred [n][h][w][3]
 * (the loss gradient w.r.t. the last sc_unet_forward's prediction);
 * writes device grad f32 [n_params]. */
sc_status sc_unet_backward(sc_ctx* ctx, sc_unet* net, const float* dpred, float* grad);
/* One Adam step on the L1-log loss of n images: device feat [n][h][w][9],
 * device target [n][h][w][3] linear rgb.  loss (host, may be NULL; then
 * the call does not synchronise) receives the loss before the update. */
sc_status sc_unet_train_step(sc_ctx* ctx, sc_unet* net, const float* feat, const float* target, uint32_t n,
                             uint32_t w, uint32_t h, float lr, float* loss);
/* One convolution layer of a network alone, on the same kernels the
 * network runs (per-layer checks; a building block).  layer = index in
 * parameter order (encoder levels two 3x3 layers each, decoder levels two
 * 3x3 layers each, the 1x1 output layer last).  X: device f32
 * [n][h][w][cin], rounded to bfloat16 on entry as the network stores
 * activations (bfloat16-representable inputs are taken exactly).
 * Forward: Y device f32 [n][h][w][cout] = act(conv(X, W) + b), act = ReLU
 * if relu, else identity; a 3x3 layer's output is the bfloat16 value the
 * network stores, the 1x1 layer's the float prediction.  Backward, given
 * dZ = dL/d(conv output before act), device f32 [n][h][w][cout] rounded to
 * bfloat16 on entry: dX device f32 [n][h][w][cin] (the bfloat16 input
 * gradient the network feeds back; may be NULL) and dW device f32
 * [cout*k*k*cin + cout], weights [cout][k][k][cin] then bias, float
 * accumulation.  The backward call overwrites that layer's part of the
 * network's gradient buffer.  Both synchronise (they hold temporaries).
 * n*h*w <= 2^26; EINVAL on a bad layer index or empty shape. */
sc_status sc_unet_layer_forward(sc_ctx* ctx, sc_unet* net, uint32_t layer, const float* X, uint32_t n, uint32_t h,
                                uint32_t w, int32_t relu, float* Y);
sc_status sc_unet_layer_backward(sc_ctx* ctx, sc_unet* net, uint32_t layer, const float* X, const float* dZ,
                                 uint32_t n, uint32_t h, uint32_t w, float* dX, float* dW);
/* The network's input features of a w x h render (the buffers of
 * sc_render: in->rgb required, albedo, normal, depthn, trans may be NULL
 * = 0): device feat [h][w][9] f32 = log(1 + max(rgb, 0)) x3, albedo,
 * normal x3, depthn, trans.  The same per-pixel function builds the
 * denoiser's input inside sc_denoise, so training pairs made with it see
 * exactly the inference features. */
sc_status sc_unet_features(sc_ctx* ctx, const sc_aov* in, uint32_t w, uint32_t h, float* feat);
/* Denoise a render: in->rgb, albedo, normal, depthn, trans (device, as
 * written by sc_render; albedo/normal/depthn/trans may be NULL) of size
 * w x h -> device out_rgb [h][w][3] linear rgb.  Any w, h (padded inside). */
sc_status sc_denoise(sc_ctx* ctx, sc_unet* net, const sc_aov* in, uint32_t w, uint32_t h, float* out_rgb);

#ifdef __cplusplus
}
#endif
#endif
