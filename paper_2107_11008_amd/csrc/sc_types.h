// sc_types.h -- structures shared by the host side and the kernels of the
// library (not part of the public ABI).
#pragma once
#include <stdint.h>

#include "../../include/sc.h"

// Wide BVH node: up to 8 children, child boxes stored as structure of
// arrays so a lane reads each box plane with one 32-byte run.
// child[i]: 0xffffffff = empty; bit 31 set = leaf with triangles
// [first, first + count) of the leaf-ordered triangle array, first in bits
// 0..27 and count-1 in bits 28..30; otherwise the index of a child node.
struct alignas(16) BNode {
    float lox[8], hix[8], loy[8], hiy[8], loz[8], hiz[8];
    uint32_t child[8];
    uint32_t pad[8];
};
static_assert(sizeof(BNode) == 256, "node layout");

#define SC_CHILD_EMPTY 0xffffffffu
#define SC_LEAF_BIT 0x80000000u
#define SC_LEAF_FIRST_MASK 0x0fffffffu

// device view of a prepared scene
struct DevScene {
    const float* V;
    const uint32_t* I;
    const float* VN;
    const uint32_t* tri_obj;
    uint32_t nt;
    const sc_material* mat;
    uint32_t n_mat;
    const float* pl;      // [n_pl][4]
    uint32_t n_pl;
    const float* tg;      // [n_tg][4]
    uint32_t n_tg;
    const float* tex;
    const float* tex_rgb;   // [tex_h][tex_w][3] or null
    uint32_t tex_w, tex_h;
    float tex_x0, tex_y0, tex_sx, tex_sy;
    uint32_t recv_obj, recv_wc, recv_hc;
    float recv_x0, recv_y0, cell_sx, cell_sy, inv_cell_area;
    const uint32_t* emit_prim;
    const float* emit_cdf;
    uint32_t n_emit;
    float a_tot;
    uint32_t n_entries;
    // acceleration structure
    const BNode* nodes;
    const float4* tris;   // 3 float4 per leaf-ordered triangle, prim id in .w of the first
    uint32_t n_nodes;
};

// device view of a wavelength setting
struct WaveDev {
    uint32_t mode, k;
    float nm[4];
    float lo, hi;
    uint32_t bins;
    float bin_scale;      // bins / (hi - lo)
    const float* tab;     // [3][n_tab] sensor curves every 0.25 nm (uniform mode)
    uint32_t n_tab;
    uint32_t channels;    // caustic-map channels
};

// wavefront state of camera paths, indexed by path id
struct PathState {
    float *ox, *oy, *oz, *dx, *dy, *dz;  // current ray
    float* T;                            // throughput
    float* L;                            // accumulated radiance
    float* lambda;
    uint32_t* flags;                     // bit0: a diffuse vertex was seen
    uint64_t* med;                       // media set (nested dielectrics)
    // hit of the current ray
    float *t, *u, *v;
    uint32_t* prim;
    // shadow ray of the current vertex
    float *sox, *soy, *soz, *sdx, *sdy, *sdz, *stmax, *scontrib;
    uint32_t* sexcl;
};

// wavefront state of photons, indexed by photon id within a chunk
struct PhotonState {
    float *ox, *oy, *oz, *dx, *dy, *dz;
    float* phi;
    float* lambda;
    uint32_t* slot;   // map channel
    uint32_t* spec;   // dielectric events so far
    uint64_t* med;    // media set (nested dielectrics)
    float *t, *u, *v;
    uint32_t* prim;
};

// device view of a general photon map: stored photons sorted into hash
// buckets of (cell, channel), cells 2.25 r wide
struct PMapDev {
    const float4* rec;             // [n][2]: (x, y, z, cell tag low bits), (nx, ny, nz, cell tag high bits)
    const unsigned long long* q;   // flux in fixed point, round(phi 2^S)
    const uint32_t* start;         // [buckets + 1] first record of each bucket
    uint32_t mask;                 // buckets - 1
    uint32_t cbits;                // channel bits at the bottom of a bucket index
    uint32_t on;                   // 0: caustics from the receiver map instead
    float r, r2, inv_h;            // radius, radius^2, 1 / cell width
    double c;                      // 1 / (2^S pi r^2)
};

// photons appended by a general-map photon pass
struct PmRecords {
    float *px, *py, *pz, *nx, *ny, *nz, *phi;
    uint32_t* ch;
    unsigned long long* photon;
    uint32_t* stat;   // [0] records, [1] largest flux (bits), [2] largest |coordinate| (bits)
    uint32_t cap;
};

struct Queues {
    uint32_t* cur;
    uint32_t* next;
    uint32_t* diffuse;
    uint32_t* dielectric;
    uint32_t* shadow;
    uint32_t* counts;  // one frame of counters per bounce depth (see QC_*)
};
// Queue counters: one frame of QC_FRAME words per bounce depth, each counter
// on its own cache line so that appends to different queues do not contend
// for one line.  Frame d holds the length of the depth-d queue (QC_CUR) and
// of the diffuse, dielectric and shadow queues made at depth d; appends to
// the next depth's queue go to frame d + 1 (QC_NEXT from frame d), so the
// frames never need to be rotated between launches.
constexpr uint32_t QC_CUR = 0, QC_DIFF = 64, QC_DIEL = 128, QC_SHADOW = 192, QC_FRAME = 256, QC_NEXT = QC_FRAME;

// counters incremented by kernels
struct DevCounters {
    unsigned long long rays_closest;
    unsigned long long rays_shadow;
    unsigned long long rays_staged;   // closest-hit rays of the k_closest launches
    unsigned long long node_visits;
    unsigned long long tri_tests;
    unsigned long long fin_paths;    // photon paths taken over by k_finish_photons
    unsigned long long fin_rays;     // closest-hit rays it traced
    unsigned long long fin_nodes;    // wide nodes it fetched (visit counting on)
    unsigned long long fin_tris;     // triangles it tested (visit counting on)
    unsigned long long any_rays;     // shadow rays of the k_anyhit launches
    unsigned long long any_nodes;    // wide nodes they fetched (visit counting on)
    unsigned long long any_tris;     // triangles they tested (visit counting on)
    unsigned long long cf_paths;     // camera paths taken over by k_finish_camera
    unsigned long long cf_rays;      // closest-hit rays it traced
    unsigned long long cf_shadow;    // shadow rays it traced
    unsigned long long cf_nodes;     // wide nodes both kinds fetched (visit counting on)
    unsigned long long cf_tris;      // triangles both kinds tested (visit counting on)
    unsigned long long ph_count[9];
    double ph_flux[9];
};
