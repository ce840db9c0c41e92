/*
 * sco.h -- CPU oracle of the SuperCaustics rendering hot path.
 *
 * TEST INFRASTRUCTURE ONLY.  This library is the plain, slow, single
 * threaded reference that the HIP path is checked against.  Only the test
 * suite, the smoke check and the CPU-baseline leg of the benchmark may load
 * it; the product path never does.  It shares no code and no header with
 * the HIP library: the struct layouts below are restated independently.
 *
 * What it computes (the paper defines the outputs, Sec. III-D; the light
 * transport behind them is the textbook reading stated in the design
 * notes):
 *   - depth, the distance from the camera to the first surface, also
 *     normalised over a 10 m range (Sec. III-D-1);
 *   - surface normals in world and camera space (Sec. III-D-2);
 *   - the object mask: the object each pixel sees first (Sec. III-D-3);
 *   - the image with refraction, dispersion and caustics (Abstract, Sec. I),
 *     traced as spectral paths through smooth dielectric meshes with
 *     Cauchy dispersion, exact Fresnel and total internal reflection, next
 *     event estimation on diffuse surfaces, and a photon-traced caustic map
 *     on a receiver plane;
 *   - glass colour, thickness and roughness (Sec. III-C lists them among
 *     the scene variations) as Beer-Lambert absorption inside each
 *     dielectric, GGX microfacet refraction, and nested and overlapping
 *     dielectrics resolved by priority.
 *
 * All pointers are host pointers.  Functions return 0 on success and a
 * negative value on invalid arguments.
 */
#ifndef SCO_H
#define SCO_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
    uint32_t type;         /* 0 diffuse, 1 dielectric, 2 emissive */
    uint32_t albedo_mode;  /* 0 constant rho_a, 1 checker (1 m, rho_a even), 2 grey texture, 3 RGB texture */
    float rho_a, rho_b;
    float cauchy_a, cauchy_b;  /* n(lambda) = a + b / lambda_um^2 */
    float le;                  /* emitted radiance (front face only) */
    uint32_t priority;         /* dielectric: nesting priority (ties: larger object id wins) */
    float sigma[3];            /* dielectric: absorption coefficient (1/m) at 450, 550, 650 nm */
    float roughness;           /* dielectric: GGX alpha in [0, 1]; 0 = smooth */
} sco_material;

typedef struct {
    const float* V;           /* [nv][3] */
    const uint32_t* I;        /* [nt][3] */
    const float* VN;          /* [nv][3] or NULL */
    const uint32_t* tri_obj;  /* [nt], object id >= 1 */
    uint32_t nv, nt;
    const sco_material* mat;  /* [n_mat], index = object id */
    uint32_t n_mat;
    const float* pl;          /* [n_pl][4] x,y,z,intensity */
    uint32_t n_pl;
    const uint32_t* tg_obj;   /* [n_tg] */
    const float* tg_sph;      /* [n_tg][4] cx,cy,cz,r */
    uint32_t n_tg;
    const float* tex;         /* [tex_h][tex_w] or NULL */
    uint32_t tex_w, tex_h;
    float tex_x0, tex_y0, tex_ext_u, tex_ext_v;
    uint32_t recv_obj;        /* 0 = no receiver */
    uint32_t recv_wc, recv_hc;
    float recv_x0, recv_y0, recv_ext_u, recv_ext_v;
    const float* tex_rgb;     /* [tex_h][tex_w][3] RGB albedo or NULL (same size and rectangle as tex) */
} sco_scene;

typedef struct {
    float eye[3], fwd[3], right[3], up[3];
    uint32_t w, h;
} sco_camera;

typedef struct {
    uint32_t mode;   /* 0 fixed, 1 uniform */
    uint32_t k;      /* fixed: number of slots, 1 or 3 */
    float nm[4];     /* fixed: wavelengths in channel order */
    float lo, hi;    /* uniform range in nm */
    uint32_t bins;   /* uniform: caustic-map spectral bins */
} sco_wavelengths;

typedef struct {
    float* rgb;        /* [h*w*3] */
    uint32_t* obj;     /* [h*w] */
    uint8_t* trans;    /* [h*w] */
    uint32_t* tri;     /* [h*w] */
    float* depth;      /* [h*w] */
    float* depthn;     /* [h*w] */
    float* normal;     /* [h*w*3] */
    float* normal_cam; /* [h*w*3] */
    float* albedo;     /* [h*w] */
    uint8_t* tie;      /* [h*w] second distinct hit within 1e-6 t */
} sco_aov;

typedef struct {
    double flux[9];     /* by outcome, see SCO_PH_* */
    uint64_t count[9];
    uint64_t segments;  /* closest-hit queries made */
} sco_photon_stats;

enum {
    SCO_PH_DEPOSITED = 0, SCO_PH_OUTSIDE = 1, SCO_PH_DIRECT = 2, SCO_PH_ELSEWHERE = 3,
    SCO_PH_ESCAPED = 4, SCO_PH_ABSORBED = 5, SCO_PH_TRUNCATED = 6, SCO_PH_LOST = 7,
    SCO_PH_EMIT_DEAD = 8
};

/* One photon of the general photon map (40 bytes). */
typedef struct {
    float pos[3];       /* deposit point */
    float nrm[3];       /* geometric normal on the side the photon arrived from */
    float phi;          /* flux */
    uint32_t channel;   /* map channel: wavelength slot or spectral bin */
    uint64_t photon;    /* photon index */
} sco_pm_rec;
typedef struct sco_bvh sco_bvh;

/* Counter-based generator (Salmon et al., SC'11): 10 rounds of Philox4x32. */
void sco_philox(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);
void sco_sincos2pi(float u, float* s, float* c);

/* Object-median binary BVH over the scene (the oracle's own); NULL on error. */
sco_bvh* sco_bvh_build(const sco_scene* s);
void sco_bvh_free(sco_bvh* b);

/* Closest hit for n rays: lexicographic minimum of (t, prim) over all
 * triangles with 0 < t.  bvh == NULL means brute force over all triangles.
 * prim = 0xffffffff on a miss (t = +inf). */
int sco_closest(const sco_scene* s, const sco_bvh* bvh, uint32_t n, const float* O, const float* D,
                float* t, uint32_t* prim, float* u, float* v);
/* Any hit with 0 < t < tmax[i], ignoring triangle excl[i] (may be NULL). */
int sco_any(const sco_scene* s, const sco_bvh* bvh, uint32_t n, const float* O, const float* D,
            const float* tmax, const uint32_t* excl, uint8_t* occluded);

/* One dielectric interaction, exposed for the optics pins. */
int sco_dielectric(const float d[3], const float Ng[3], const float Ns[3], const float P[3],
                   float lambda_nm, float ca, float cb, float u_fresnel,
                   float o_out[3], float d_out[3], int* reflected, float* R_out);
float sco_fresnel(float n1, float n2, float ci, float ct);
/* Rough (GGX) dielectric interface, exposed for the microfacet pins:
 * direction d arriving at a surface of normal n (either orientation),
 * index n1 on the incoming side and n2 across, GGX alpha in (0, 1];
 * count draws u[i][3] = (u0, u1, uF).  Out: direction, reflected flag
 * (1 reflected, 0 refracted, -1 no valid direction) and path weight. */
int sco_rough_dielectric(const float d[3], const float n[3], float n1, float n2, float alpha, uint32_t count,
                         const float* u, float* d_out, int32_t* reflected, float* weight);
/* exp(-x) for x >= 0 in the oracle's own float arithmetic (Beer-Lambert
 * weights); 1 for x <= 0, 0 for x > 87. */
float sco_exp_neg(float x);
/* One surface crossing of nested dielectrics: the set ids[0..n) of media
 * the path is inside, a hit on dielectric object k from its front
 * (entering = 1) or back.  Returns the set after crossing, whether the
 * surface is a real interface, and the indices n1 (the side the path comes
 * from) and n2 (across) at lambda. */
int sco_media_step(const sco_scene* s, const uint32_t* ids, uint32_t n, uint32_t k, int entering, float lam,
                   uint32_t* ids_after, uint32_t* n_after, int* real, float* n1, float* n2);
/* The frame and the Lambert bounce of diffuse vertices, exposed for the
 * pins: Duff et al.'s orthonormal basis (t1, t2) about unit n, and count
 * cosine-weighted directions about unit n from draws u[i] = (u0, u1). */
void sco_onb(const float n[3], float t1[3], float t2[3]);
void sco_cosine_dir(const float n[3], uint32_t count, const float* u, float* d_out);
void sco_camera_ray(const sco_camera* cam, uint32_t x, uint32_t y, float jx, float jy, float o[3], float d[3]);

/* Photon pass over photon indices [p0, p1) of a pass of n_photons.
 * map_sum: FP64 [recv_hc][recv_wc][C] accumulated in photon order (caller
 * zeroes it); count: u32 deposits per cell (may be NULL); stats may be NULL. */
int sco_trace_photons(const sco_scene* s, const sco_bvh* bvh, uint64_t n_photons, uint64_t p0, uint64_t p1,
                      uint32_t max_depth, const sco_wavelengths* wl, uint64_t seed,
                      double* map_sum, uint32_t* count, sco_photon_stats* stats);

/* Photon pass into the general photon map: every photon that reaches a
 * diffuse surface (any object) after at least one dielectric event is
 * stored there, in photon order, up to cap records (-1 beyond). */
int sco_pm_trace(const sco_scene* s, const sco_bvh* bvh, uint64_t n_photons, uint64_t p0, uint64_t p1,
                 uint32_t max_depth, const sco_wavelengths* wl, uint64_t seed,
                 sco_pm_rec* recs, uint64_t cap, uint64_t* n_rec, sco_photon_stats* stats);
/* Fixed-point scale 2^S of the disc sums: the largest power of two with
 * n * max(phi) * 2^S <= 2^62 (1 if there is no positive flux). */
double sco_pm_scale(const sco_pm_rec* recs, uint64_t n);
/* Irradiance estimate of channel at P (facing normal N) over the disc of
 * the given radius: sum of round(phi 2^S) of the records of that channel
 * on the same side within the radius, times 1 / (2^S pi r^2). */
float sco_pm_gather(const sco_pm_rec* recs, uint64_t n, float radius, const float P[3], const float N[3],
                    uint32_t channel);
/* sco_render with caustics gathered from the general photon map on every
 * diffuse surface instead of the receiver map. */
int sco_render_pm(const sco_scene* s, const sco_bvh* bvh, const sco_camera* cam, uint32_t spp, uint32_t max_depth,
                  const sco_wavelengths* wl, uint64_t seed, const sco_pm_rec* recs, uint64_t n_rec, float radius,
                  const uint32_t* pix, uint32_t n_pix, sco_aov* out, uint64_t* segments);
/* Render the listed pixels (all if pix == NULL).  caustic_map: float
 * [recv_hc][recv_wc][C] or NULL (caustics off).  Output arrays are full
 * size and may individually be NULL.  segments (may be NULL) receives the
 * number of closest-hit and any-hit queries made. */
int sco_render(const sco_scene* s, const sco_bvh* bvh, const sco_camera* cam, uint32_t spp, uint32_t max_depth,
               const sco_wavelengths* wl, uint64_t seed, const float* caustic_map,
               const uint32_t* pix, uint32_t n_pix, sco_aov* out, uint64_t* segments);

/* Per-path radiance samples (for debugging parity): L[(s*n_pix + i)*K + slot]. */
int sco_path_samples(const sco_scene* s, const sco_bvh* bvh, const sco_camera* cam, uint32_t spp,
                     uint32_t max_depth, const sco_wavelengths* wl, uint64_t seed, const float* caustic_map,
                     const uint32_t* pix, uint32_t n_pix, float* L, float* lambda);

#ifdef __cplusplus
}
#endif
#endif
