/*
 * sco.c -- CPU oracle of the SuperCaustics rendering hot path.
 *
 * TEST INFRASTRUCTURE ONLY (see sco.h).  Plain single-threaded C, built
 * with -ffp-contract=off: every float operation below is one IEEE-754
 * binary32 operation rounded to nearest, in the order written, with
 * division and square root correctly rounded and denormals kept.  No
 * transcendental function of libm is used inside a traced decision.
 *
 * The paper (Sec. III and III-D) fixes what the outputs mean, not how light
 * transport is computed; each function below names the textbook method it
 * restates.  Ties in the closest hit go to the smaller triangle index, so
 * the result is one well-defined value that any acceleration structure
 * must reproduce.
 */
#include "sco.h"

#include <float.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------ */
/* small float vector helpers                                          */
/* ------------------------------------------------------------------ */

typedef struct { float x, y, z; } v3;

static v3 mk(float x, float y, float z) { v3 r; r.x = x; r.y = y; r.z = z; return r; }
static v3 vadd(v3 a, v3 b) { return mk(a.x + b.x, a.y + b.y, a.z + b.z); }
static v3 vsub(v3 a, v3 b) { return mk(a.x - b.x, a.y - b.y, a.z - b.z); }
static v3 vscale(v3 a, float s) { return mk(a.x * s, a.y * s, a.z * s); }
static v3 vneg(v3 a) { return mk(-a.x, -a.y, -a.z); }
static float vdot(v3 a, v3 b) { return (a.x * b.x + a.y * b.y) + a.z * b.z; }
static v3 vcross(v3 a, v3 b) {
    return mk(a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x);
}
static v3 vnorm(v3 a) {
    float inv = 1.0f / sqrtf(vdot(a, a));
    return vscale(a, inv);
}
static float vget(v3 a, int k) { return k == 0 ? a.x : (k == 1 ? a.y : a.z); }
static v3 ld3(const float* p, uint32_t i) { return mk(p[3 * (size_t)i], p[3 * (size_t)i + 1], p[3 * (size_t)i + 2]); }

static const float INV_PI_F = 0.31830988618379067154f;
static const float TWO_PI_F = 6.28318530717958647692f;

/* ------------------------------------------------------------------ */
/* Philox4x32-10 (Salmon, Moraes, Dror, Shaw: "Parallel random numbers:  */
/* as easy as 1, 2, 3", SC'11).  Each round multiplies counter words 0   */
/* and 2 by the two round multipliers, swaps the halves and mixes in the */
/* key, which is bumped by the two Weyl constants between rounds.       */
/* ------------------------------------------------------------------ */

void sco_philox(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
    uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int r = 0; r < 10; r++) {
        if (r > 0) { k0 += 0x9E3779B9u; k1 += 0xBB67AE85u; }
        uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c0;
        uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t n0 = hi1 ^ c1 ^ k0;
        uint32_t n2 = hi0 ^ c3 ^ k1;
        c0 = n0; c1 = lo1; c2 = n2; c3 = lo0;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* 24 high bits to a float in [0, 1 - 2^-24]. */
static float u01(uint32_t x) { return (float)(x >> 8) * 5.9604644775390625e-08f; }

/* Camera stream: counter (pixel, sample, depth<<4 | purpose, slot<<8 | 0). */
static void rng_cam(uint64_t seed, uint32_t pix, uint32_t sample, uint32_t depth, uint32_t purpose,
                    uint32_t slot, uint32_t out[4]) {
    uint32_t ctr[4] = {pix, sample, (depth << 4) | purpose, (slot << 8) | 0u};
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    sco_philox(ctr, key, out);
}
/* Photon stream: counter (p lo, p hi, depth<<4 | purpose, 1). */
static void rng_ph(uint64_t seed, uint64_t p, uint32_t depth, uint32_t purpose, uint32_t out[4]) {
    uint32_t ctr[4] = {(uint32_t)p, (uint32_t)(p >> 32), (depth << 4) | purpose, 1u};
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    sco_philox(ctr, key, out);
}

/* ------------------------------------------------------------------ */
/* sin and cos of 2*pi*u without libm: the quarter turn q = floor(4u) is  */
/* exact, f = 4u - q is exact, and sin/cos of f*pi/2 on [0,1) come from   */
/* their Taylor series (odd terms to f^13, even to f^14), coefficients    */
/* formed in double and rounded once to float, evaluated by Horner.       */
/* ------------------------------------------------------------------ */

static float SC_S[7], SC_C[8];
static int sc_init_done = 0;

static void sincos_init(void) {
    if (sc_init_done) return;
    const double h = 1.57079632679489661923; /* pi/2 */
    double p = h, fact = 1.0;
    /* sin: h^(2i+1)/(2i+1)! with alternating sign */
    for (int i = 0; i < 7; i++) {
        int n = 2 * i + 1;
        if (i > 0) { p = p * h * h; fact = fact * (double)(n - 1) * (double)n; }
        double c = p / fact;
        SC_S[i] = (float)((i & 1) ? -c : c);
    }
    p = 1.0; fact = 1.0;
    for (int i = 0; i < 8; i++) {
        int n = 2 * i;
        if (i > 0) { p = p * h * h; fact = fact * (double)(n - 1) * (double)n; }
        double c = p / fact;
        SC_C[i] = (float)((i & 1) ? -c : c);
    }
    sc_init_done = 1;
}

void sco_sincos2pi(float u, float* s, float* c) {
    sincos_init();
    float u4 = u * 4.0f;
    float qf = floorf(u4);
    int q = (int)qf;
    float f = u4 - qf;
    float f2 = f * f;
    float ps = SC_S[6];
    for (int i = 5; i >= 0; i--) ps = SC_S[i] + f2 * ps;
    ps = f * ps;
    float pc = SC_C[7];
    for (int i = 6; i >= 0; i--) pc = SC_C[i] + f2 * pc;
    q &= 3;
    if (q == 0) { *s = ps; *c = pc; }
    else if (q == 1) { *s = pc; *c = -ps; }
    else if (q == 2) { *s = -ps; *c = -pc; }
    else { *s = -pc; *c = ps; }
}

/* ------------------------------------------------------------------ */
/* Camera (pinhole).  Film coordinates in [-1,1], row 0 at the top.       */
/* ------------------------------------------------------------------ */

static void camera_ray(const sco_camera* cam, uint32_t x, uint32_t y, float jx, float jy, v3* o, v3* d) {
    float px = (float)x + jx;
    float py = (float)y + jy;
    float sx = (px + px) / (float)cam->w - 1.0f;
    float sy = 1.0f - (py + py) / (float)cam->h;
    v3 dd;
    dd.x = (cam->fwd[0] + sx * cam->right[0]) + sy * cam->up[0];
    dd.y = (cam->fwd[1] + sx * cam->right[1]) + sy * cam->up[1];
    dd.z = (cam->fwd[2] + sx * cam->right[2]) + sy * cam->up[2];
    *d = vnorm(dd);
    *o = mk(cam->eye[0], cam->eye[1], cam->eye[2]);
}

void sco_camera_ray(const sco_camera* cam, uint32_t x, uint32_t y, float jx, float jy, float o[3], float d[3]) {
    v3 oo, dd;
    camera_ray(cam, x, y, jx, jy, &oo, &dd);
    o[0] = oo.x; o[1] = oo.y; o[2] = oo.z;
    d[0] = dd.x; d[1] = dd.y; d[2] = dd.z;
}

/* ------------------------------------------------------------------ */
/* Watertight ray/triangle test (Woop, Benthin, Wald, JCGT 2(1), 2013).   */
/* The largest direction component becomes z; a shear maps the ray onto  */
/* the +z axis; the three 2D edge functions decide the hit (edges count); */
/* an edge function that is exactly zero is recomputed in double.        */
/* ------------------------------------------------------------------ */

typedef struct { v3 o, d; int kx, ky, kz; float sx, sy, sz; } ray_t;

static void ray_prep(ray_t* r, v3 o, v3 d) {
    r->o = o; r->d = d;
    float ax = fabsf(d.x), ay = fabsf(d.y), az = fabsf(d.z);
    int kz = 0;
    float m = ax;
    if (ay > m) { kz = 1; m = ay; }
    if (az > m) { kz = 2; }
    int kx = kz + 1; if (kx == 3) kx = 0;
    int ky = kx + 1; if (ky == 3) ky = 0;
    float dz = vget(d, kz);
    if (dz < 0.0f) { int t = kx; kx = ky; ky = t; }
    r->kx = kx; r->ky = ky; r->kz = kz;
    r->sx = vget(d, kx) / dz;
    r->sy = vget(d, ky) / dz;
    r->sz = 1.0f / dz;
}

/* Returns 1 and (t, u, v) on a hit with t > 0; u, v weight vertices 1 and 2. */
static int tri_hit(const ray_t* r, v3 p0, v3 p1, v3 p2, float* t_out, float* u_out, float* v_out) {
    v3 A = vsub(p0, r->o), B = vsub(p1, r->o), C = vsub(p2, r->o);
    float Akz = vget(A, r->kz), Bkz = vget(B, r->kz), Ckz = vget(C, r->kz);
    float Ax = vget(A, r->kx) - r->sx * Akz;
    float Ay = vget(A, r->ky) - r->sy * Akz;
    float Bx = vget(B, r->kx) - r->sx * Bkz;
    float By = vget(B, r->ky) - r->sy * Bkz;
    float Cx = vget(C, r->kx) - r->sx * Ckz;
    float Cy = vget(C, r->ky) - r->sy * Ckz;
    float U = Cx * By - Cy * Bx;
    float V = Ax * Cy - Ay * Cx;
    float W = Bx * Ay - By * Ax;
    if (U == 0.0f || V == 0.0f || W == 0.0f) {
        double CxBy = (double)Cx * (double)By, CyBx = (double)Cy * (double)Bx;
        double AxCy = (double)Ax * (double)Cy, AyCx = (double)Ay * (double)Cx;
        double BxAy = (double)Bx * (double)Ay, ByAx = (double)By * (double)Ax;
        U = (float)(CxBy - CyBx);
        V = (float)(AxCy - AyCx);
        W = (float)(BxAy - ByAx);
    }
    if ((U < 0.0f || V < 0.0f || W < 0.0f) && (U > 0.0f || V > 0.0f || W > 0.0f)) return 0;
    float det = (U + V) + W;
    if (det == 0.0f) return 0;
    float Az = r->sz * Akz, Bz = r->sz * Bkz, Cz = r->sz * Ckz;
    float T = (U * Az + V * Bz) + W * Cz;
    float rcp = 1.0f / det;
    float t = T * rcp;
    if (!(t > 0.0f)) return 0;
    *t_out = t;
    *u_out = V * rcp;
    *v_out = W * rcp;
    return 1;
}

static void tri_verts(const sco_scene* s, uint32_t prim, v3* p0, v3* p1, v3* p2) {
    const uint32_t* idx = s->I + 3 * (size_t)prim;
    *p0 = ld3(s->V, idx[0]); *p1 = ld3(s->V, idx[1]); *p2 = ld3(s->V, idx[2]);
}

/* ------------------------------------------------------------------ */
/* The oracle's own acceleration structure: a binary BVH split at the    */
/* object median along the widest centroid axis.  Its boxes are tested   */
/* in double with a generous margin, so it can only visit more nodes     */
/* than necessary, never fewer; the result equals brute force.          */
/* ------------------------------------------------------------------ */

typedef struct { float lo[3], hi[3]; int32_t left, right; uint32_t first, count; } bnode;
struct sco_bvh { bnode* nodes; uint32_t n_nodes; uint32_t* prims; };

typedef struct { float c[3]; float lo[3], hi[3]; uint32_t prim; } bprim;

static int cmp_axis;
static int cmp_bprim(const void* a, const void* b) {
    const bprim* x = (const bprim*)a; const bprim* y = (const bprim*)b;
    float cx = x->c[cmp_axis], cy = y->c[cmp_axis];
    if (cx < cy) return -1;
    if (cx > cy) return 1;
    return (x->prim < y->prim) ? -1 : (x->prim > y->prim);
}

static uint32_t bvh_rec(sco_bvh* b, bprim* P, uint32_t first, uint32_t count, uint32_t* next) {
    uint32_t id = (*next)++;
    bnode* n = &b->nodes[id];
    for (int k = 0; k < 3; k++) { n->lo[k] = INFINITY; n->hi[k] = -INFINITY; }
    float clo[3] = {INFINITY, INFINITY, INFINITY}, chi[3] = {-INFINITY, -INFINITY, -INFINITY};
    for (uint32_t i = first; i < first + count; i++) {
        for (int k = 0; k < 3; k++) {
            if (P[i].lo[k] < n->lo[k]) n->lo[k] = P[i].lo[k];
            if (P[i].hi[k] > n->hi[k]) n->hi[k] = P[i].hi[k];
            if (P[i].c[k] < clo[k]) clo[k] = P[i].c[k];
            if (P[i].c[k] > chi[k]) chi[k] = P[i].c[k];
        }
    }
    if (count <= 4) {
        n->left = n->right = -1; n->first = first; n->count = count;
        return id;
    }
    int ax = 0;
    float ext = chi[0] - clo[0];
    if (chi[1] - clo[1] > ext) { ax = 1; ext = chi[1] - clo[1]; }
    if (chi[2] - clo[2] > ext) { ax = 2; }
    cmp_axis = ax;
    qsort(P + first, count, sizeof(bprim), cmp_bprim);
    uint32_t half = count / 2;
    n->count = 0; n->first = 0;
    int32_t l = (int32_t)bvh_rec(b, P, first, half, next);
    int32_t r = (int32_t)bvh_rec(b, P, first + half, count - half, next);
    b->nodes[id].left = l; b->nodes[id].right = r;
    return id;
}

sco_bvh* sco_bvh_build(const sco_scene* s) {
    if (!s || s->nt == 0) return NULL;
    bprim* P = (bprim*)malloc(sizeof(bprim) * s->nt);
    sco_bvh* b = (sco_bvh*)calloc(1, sizeof(sco_bvh));
    b->nodes = (bnode*)malloc(sizeof(bnode) * 2 * (size_t)s->nt);
    b->prims = (uint32_t*)malloc(sizeof(uint32_t) * s->nt);
    for (uint32_t i = 0; i < s->nt; i++) {
        v3 a, c, d;
        tri_verts(s, i, &a, &c, &d);
        float xs[3] = {a.x, c.x, d.x}, ys[3] = {a.y, c.y, d.y}, zs[3] = {a.z, c.z, d.z};
        const float* cs[3] = {xs, ys, zs};
        for (int k = 0; k < 3; k++) {
            float lo = cs[k][0], hi = cs[k][0];
            for (int j = 1; j < 3; j++) { if (cs[k][j] < lo) lo = cs[k][j]; if (cs[k][j] > hi) hi = cs[k][j]; }
            P[i].lo[k] = lo; P[i].hi[k] = hi;
            P[i].c[k] = (float)(0.5 * ((double)lo + (double)hi));
        }
        P[i].prim = i;
    }
    uint32_t next = 0;
    bvh_rec(b, P, 0, s->nt, &next);
    b->n_nodes = next;
    for (uint32_t i = 0; i < s->nt; i++) b->prims[i] = P[i].prim;
    free(P);
    return b;
}

void sco_bvh_free(sco_bvh* b) {
    if (!b) return;
    free(b->nodes); free(b->prims); free(b);
}

/* Entry distance of the ray into the box, in double; +inf when missed. */
static double box_entry(const bnode* n, v3 o, v3 d, double tlim) {
    double t0 = 0.0, t1 = tlim;
    double oo[3] = {o.x, o.y, o.z}, dd[3] = {d.x, d.y, d.z};
    for (int k = 0; k < 3; k++) {
        double lo = n->lo[k], hi = n->hi[k];
        if (dd[k] == 0.0) {
            if (oo[k] < lo || oo[k] > hi) return INFINITY;
            continue;
        }
        double a = (lo - oo[k]) / dd[k], b = (hi - oo[k]) / dd[k];
        if (a > b) { double t = a; a = b; b = t; }
        if (a > t0) t0 = a;
        if (b < t1) t1 = b;
    }
    /* widen by a relative and an absolute margin before comparing */
    double slack = 1e-4 * fabs(t1) + 1e-5;
    if (t0 > t1 + slack) return INFINITY;
    return t0;
}

static double tlimit(float tbest) {
    if (isinf(tbest)) return INFINITY;
    return (double)tbest * (1.0 + 1e-4) + 1e-5;
}

/* closest: keep lexicographic minimum of (t, prim) */
static void consider(const sco_scene* s, const ray_t* r, uint32_t prim, float* tb, uint32_t* pb, float* ub, float* vb) {
    v3 a, b, c;
    tri_verts(s, prim, &a, &b, &c);
    float t, u, v;
    if (!tri_hit(r, a, b, c, &t, &u, &v)) return;
    if (t < *tb || (t == *tb && prim < *pb)) { *tb = t; *pb = prim; *ub = u; *vb = v; }
}

static void closest_one(const sco_scene* s, const sco_bvh* bvh, v3 o, v3 d, float* t, uint32_t* prim, float* u, float* v) {
    ray_t r;
    ray_prep(&r, o, d);
    float tb = INFINITY, ub = 0.0f, vb = 0.0f;
    uint32_t pb = 0xffffffffu;
    if (!bvh) {
        for (uint32_t i = 0; i < s->nt; i++) consider(s, &r, i, &tb, &pb, &ub, &vb);
    } else {
        uint32_t stack[128];
        int sp = 0;
        stack[sp++] = 0;
        while (sp > 0) {
            const bnode* n = &bvh->nodes[stack[--sp]];
            double te = box_entry(n, o, d, INFINITY);
            if (isinf(te) || te > tlimit(tb)) continue;
            if (n->left < 0) {
                for (uint32_t k = 0; k < n->count; k++) consider(s, &r, bvh->prims[n->first + k], &tb, &pb, &ub, &vb);
            } else {
                if (sp + 2 > 128) abort();
                stack[sp++] = (uint32_t)n->right;
                stack[sp++] = (uint32_t)n->left;
            }
        }
    }
    *t = tb; *prim = pb; *u = ub; *v = vb;
}

/* Distance of the nearest hit on any triangle other than excl (+inf if
 * none): brute force without a tree, else the tree walk of closest_one
 * with excl skipped. */
static float nearest_other(const sco_scene* s, const sco_bvh* bvh, v3 o, v3 d, uint32_t excl) {
    ray_t r;
    ray_prep(&r, o, d);
    float tb = INFINITY, ub = 0.0f, vb = 0.0f;
    uint32_t pb = 0xffffffffu;
    if (!bvh) {
        for (uint32_t i = 0; i < s->nt; i++)
            if (i != excl) consider(s, &r, i, &tb, &pb, &ub, &vb);
        return tb;
    }
    uint32_t stack[128];
    int sp = 0;
    stack[sp++] = 0;
    while (sp > 0) {
        const bnode* n = &bvh->nodes[stack[--sp]];
        double te = box_entry(n, o, d, INFINITY);
        if (isinf(te) || te > tlimit(tb)) continue;
        if (n->left < 0) {
            for (uint32_t k = 0; k < n->count; k++) {
                uint32_t i = bvh->prims[n->first + k];
                if (i != excl) consider(s, &r, i, &tb, &pb, &ub, &vb);
            }
        } else {
            if (sp + 2 > 128) abort();
            stack[sp++] = (uint32_t)n->right;
            stack[sp++] = (uint32_t)n->left;
        }
    }
    return tb;
}

static int any_one(const sco_scene* s, const sco_bvh* bvh, v3 o, v3 d, float tmax, uint32_t excl) {
    ray_t r;
    ray_prep(&r, o, d);
    if (!bvh) {
        for (uint32_t i = 0; i < s->nt; i++) {
            if (i == excl) continue;
            v3 a, b, c; float t, u, v;
            tri_verts(s, i, &a, &b, &c);
            if (tri_hit(&r, a, b, c, &t, &u, &v) && t < tmax) return 1;
        }
        return 0;
    }
    uint32_t stack[128];
    int sp = 0;
    stack[sp++] = 0;
    while (sp > 0) {
        const bnode* n = &bvh->nodes[stack[--sp]];
        double te = box_entry(n, o, d, INFINITY);
        if (isinf(te) || te > tlimit(tmax)) continue;
        if (n->left < 0) {
            for (uint32_t k = 0; k < n->count; k++) {
                uint32_t i = bvh->prims[n->first + k];
                if (i == excl) continue;
                v3 a, b, c; float t, u, v;
                tri_verts(s, i, &a, &b, &c);
                if (tri_hit(&r, a, b, c, &t, &u, &v) && t < tmax) return 1;
            }
        } else {
            if (sp + 2 > 128) abort();
            stack[sp++] = (uint32_t)n->right;
            stack[sp++] = (uint32_t)n->left;
        }
    }
    return 0;
}

int sco_closest(const sco_scene* s, const sco_bvh* bvh, uint32_t n, const float* O, const float* D,
                float* t, uint32_t* prim, float* u, float* v) {
    if (!s || !O || !D || !t || !prim) return -1;
    for (uint32_t i = 0; i < n; i++) {
        float uu, vv;
        closest_one(s, bvh, ld3(O, i), ld3(D, i), &t[i], &prim[i], &uu, &vv);
        if (u) u[i] = uu;
        if (v) v[i] = vv;
    }
    return 0;
}

int sco_any(const sco_scene* s, const sco_bvh* bvh, uint32_t n, const float* O, const float* D,
            const float* tmax, const uint32_t* excl, uint8_t* occluded) {
    if (!s || !O || !D || !tmax || !occluded) return -1;
    for (uint32_t i = 0; i < n; i++)
        occluded[i] = (uint8_t)any_one(s, bvh, ld3(O, i), ld3(D, i), tmax[i], excl ? excl[i] : 0xffffffffu);
    return 0;
}

/* ------------------------------------------------------------------ */
/* Hit frame and self-intersection-free ray origins.                    */
/* ------------------------------------------------------------------ */

typedef struct { v3 P, Ng, Nf, Ns; int entering; } frame_t;

static void hit_frame(const sco_scene* s, uint32_t prim, float u, float v, v3 d, frame_t* f) {
    v3 p0, p1, p2;
    tri_verts(s, prim, &p0, &p1, &p2);
    v3 n = vcross(vsub(p1, p0), vsub(p2, p0));
    f->Ng = vnorm(n);
    float w = (1.0f - u) - v;
    f->P = vadd(vadd(vscale(p0, w), vscale(p1, u)), vscale(p2, v));
    f->entering = vdot(d, f->Ng) < 0.0f;
    f->Nf = f->entering ? f->Ng : vneg(f->Ng);
    if (s->VN) {
        const uint32_t* idx = s->I + 3 * (size_t)prim;
        v3 n0 = ld3(s->VN, idx[0]), n1 = ld3(s->VN, idx[1]), n2 = ld3(s->VN, idx[2]);
        v3 ns = vnorm(vadd(vadd(vscale(n0, w), vscale(n1, u)), vscale(n2, v)));
        if (vdot(ns, f->Nf) < 0.0f) ns = vneg(ns);
        f->Ns = ns;
    } else {
        f->Ns = f->Nf;
    }
}

static int32_t f2i_bits(float f) { int32_t i; memcpy(&i, &f, 4); return i; }
static float i2f_bits(int32_t i) { float f; memcpy(&f, &i, 4); return f; }

/* Offset a surface point along n by a few ULPs (Waechter and Binder, "A
 * Fast and Robust Method for Avoiding Self-Intersection", Ray Tracing
 * Gems, ch. 6, 2019): integer ULP steps away from the origin region, a
 * small fixed step near it. */
static float offset_c(float p, float n) {
    const float origin = 1.0f / 32.0f, float_scale = 1.0f / 65536.0f, int_scale = 256.0f;
    int32_t of = (int32_t)(int_scale * n);
    int32_t pi = f2i_bits(p);
    pi = pi + ((p < 0.0f) ? -of : of);
    if (fabsf(p) < origin) return p + float_scale * n;
    return i2f_bits(pi);
}
static v3 offset_ray(v3 p, v3 n) { return mk(offset_c(p.x, n.x), offset_c(p.y, n.y), offset_c(p.z, n.z)); }

/* Orthonormal basis around unit n (Duff et al., "Building an Orthonormal
 * Basis, Revisited", JCGT 6(1), 2017). */
static void onb(v3 n, v3* t1, v3* t2) {
    float sign = copysignf(1.0f, n.z);
    float a = -1.0f / (sign + n.z);
    float b = (n.x * n.y) * a;
    *t1 = mk(1.0f + ((sign * n.x) * n.x) * a, sign * b, -(sign * n.x));
    *t2 = mk(b, sign + (n.y * n.y) * a, -n.y);
}

/* Cosine-weighted direction about unit n (Lambert bounce): a uniform
 * point of the unit disc, radius sqrt(u0) and angle 2 pi u1, lifted to
 * the hemisphere by z = sqrt(1 - u0) (Malley's method), expressed in the
 * frame above.  The density is cos(theta) / pi, so sin^2(theta) = u0 and
 * the azimuth 2 pi u1 are both uniform. */
static v3 cosine_dir(v3 n, float u0, float u1) {
    float rr = sqrtf(u0);
    float sp, cp;
    sco_sincos2pi(u1, &sp, &cp);
    float x = rr * cp, y = rr * sp;
    float z = sqrtf(fmaxf(0.0f, 1.0f - u0));
    v3 t1, t2;
    onb(n, &t1, &t2);
    return vnorm(vadd(vadd(vscale(t1, x), vscale(t2, y)), vscale(n, z)));
}

void sco_onb(const float n[3], float t1[3], float t2[3]) {
    v3 a, b;
    onb(mk(n[0], n[1], n[2]), &a, &b);
    t1[0] = a.x; t1[1] = a.y; t1[2] = a.z;
    t2[0] = b.x; t2[1] = b.y; t2[2] = b.z;
}

void sco_cosine_dir(const float n[3], uint32_t count, const float* u, float* d_out) {
    v3 nn = mk(n[0], n[1], n[2]);
    for (uint32_t i = 0; i < count; i++) {
        v3 d = cosine_dir(nn, u[2 * (size_t)i], u[2 * (size_t)i + 1]);
        d_out[3 * (size_t)i] = d.x; d_out[3 * (size_t)i + 1] = d.y; d_out[3 * (size_t)i + 2] = d.z;
    }
}

/* ------------------------------------------------------------------ */
/* Smooth dielectric interface.                                         */
/*   n(lambda) = A + B / lambda_um^2       (two-term Cauchy dispersion)  */
/*   Snell: eta = n_incident / n_transmitted; cos_t^2 = 1 - eta^2 sin_i^2 */
/*   total internal reflection when cos_t^2 <= 0                        */
/*   unpolarised Fresnel reflectance R = (Rs^2 + Rp^2)/2 with           */
/*   Rs = (n1 ci - n2 ct)/(n1 ci + n2 ct), Rp = (n1 ct - n2 ci)/(n1 ct + n2 ci) */
/*   the event is reflection iff u < R (weight 1 either way).           */
/* ------------------------------------------------------------------ */

float sco_fresnel(float n1, float n2, float ci, float ct) {
    float a1 = n1 * ci, b1 = n2 * ct;
    float rs = (a1 - b1) / (a1 + b1);
    float a2 = n1 * ct, b2 = n2 * ci;
    float rp = (a2 - b2) / (a2 + b2);
    return 0.5f * (rs * rs + rp * rp);
}

/* Refractive index from the two-term Cauchy law, lambda in nm. */
static float cauchy_n(float ca, float cb, float lambda_nm) {
    float l = lambda_nm * 0.001f;
    return ca + cb / (l * l);
}

/* Returns 1 with the new direction and reflected flag, 0 if no valid
 * outgoing direction exists even with the geometric normal.  n1 is the
 * index on the side the ray comes from, n2 the one across the surface. */
static int dielectric_dir(const frame_t* f, v3 d, float n1, float n2, float uF,
                          v3* dout, int* refl_out, float* R_out) {
    float eta = n1 / n2;
    v3 N = f->Ns;
    float ci = -vdot(d, N);
    int geometric = 0;
    if (!(ci > 0.0f)) { N = f->Nf; ci = -vdot(d, N); geometric = 1; }
    for (;;) {
        float e2 = eta * eta;
        float s2 = 1.0f - ci * ci;
        float k = 1.0f - e2 * s2;
        int refl;
        float ct = 0.0f, R = 1.0f;
        if (k <= 0.0f) {
            refl = 1;
        } else {
            ct = sqrtf(k);
            R = sco_fresnel(n1, n2, ci, ct);
            refl = uF < R;
        }
        v3 out;
        if (refl) out = vadd(d, vscale(N, ci + ci));
        else out = vadd(vscale(d, eta), vscale(N, eta * ci - ct));
        out = vnorm(out);
        float side = vdot(out, f->Nf);
        int ok = refl ? (side > 0.0f) : (side < 0.0f);
        if (ok) { *dout = out; *refl_out = refl; if (R_out) *R_out = R; return 1; }
        if (geometric) return 0;
        N = f->Nf; ci = -vdot(d, N); geometric = 1;
    }
}

int sco_dielectric(const float d[3], const float Ng[3], const float Ns[3], const float P[3],
                   float lambda_nm, float ca, float cb, float u_fresnel,
                   float o_out[3], float d_out[3], int* reflected, float* R_out) {
    frame_t f;
    v3 dd = mk(d[0], d[1], d[2]);
    f.P = mk(P[0], P[1], P[2]);
    f.Ng = mk(Ng[0], Ng[1], Ng[2]);
    f.entering = vdot(dd, f.Ng) < 0.0f;
    f.Nf = f.entering ? f.Ng : vneg(f.Ng);
    v3 ns = mk(Ns[0], Ns[1], Ns[2]);
    if (vdot(ns, f.Nf) < 0.0f) ns = vneg(ns);
    f.Ns = ns;
    v3 out;
    int refl;
    float n = cauchy_n(ca, cb, lambda_nm);
    float n1 = f.entering ? 1.0f : n, n2 = f.entering ? n : 1.0f;
    if (!dielectric_dir(&f, dd, n1, n2, u_fresnel, &out, &refl, R_out)) return 0;
    v3 o = offset_ray(f.P, refl ? f.Nf : vneg(f.Nf));
    o_out[0] = o.x; o_out[1] = o.y; o_out[2] = o.z;
    d_out[0] = out.x; d_out[1] = out.y; d_out[2] = out.z;
    *reflected = refl;
    return 1;
}

/* ------------------------------------------------------------------ */
/* Rough dielectric interface: the GGX microfacet model of Walter,       */
/* Marschner, Li and Torrance ("Microfacet Models for Refraction through */
/* Rough Surfaces", EGSR 2007) with width alpha, Smith shadowing          */
/*   G1(v) = 2 / (1 + sqrt(1 + alpha^2 tan^2 theta_v)),                  */
/* sampled through the distribution of visible normals (Heitz,           */
/* "Sampling the GGX Distribution of Visible Normals", JCGT 7(4), 2018): */
/* m is drawn with density G1(i) max(0, i.m) D(m) / (i.n) by stretching  */
/* i into the alpha = 1 configuration, drawing a point on the projected   */
/* hemisphere seen from there (r = sqrt(u0), phi = 2 pi u1, the second   */
/* coordinate warped towards the visible half) and stretching its normal */
/* back.  The Fresnel reflectance at m then picks reflection (uF < F) or  */
/* refraction across m, and the path weight is G1(o) <= 1 either way.    */
/* The macro normal n is the shading normal on the incoming side, else   */
/* the geometric one.  A draw whose outgoing direction lies on the wrong */
/* side of the surface or of m has weight 0: the path ends.              */
/* ------------------------------------------------------------------ */

static float smith_g1(float c, float a2) {
    float c2 = c * c;
    float t2 = (1.0f - c2) / c2;
    return 2.0f / (1.0f + sqrtf(1.0f + a2 * t2));
}

static int rough_dir(const frame_t* f, v3 d, float n1, float n2, float alpha, float u0, float u1, float uF,
                     v3* dout, int* refl_out, float* w_out) {
    float eta = n1 / n2;
    v3 N = f->Ns;
    if (!(-vdot(d, N) > 0.0f)) N = f->Nf;
    float a2 = alpha * alpha;
    /* the incoming direction in the frame (t1, t2, N), stretched */
    v3 t1, t2;
    onb(N, &t1, &t2);
    v3 iw = vneg(d);
    v3 vh = vnorm(mk(alpha * vdot(iw, t1), alpha * vdot(iw, t2), vdot(iw, N)));
    float lensq = vh.x * vh.x + vh.y * vh.y;
    v3 b1 = lensq > 0.0f ? vscale(mk(-vh.y, vh.x, 0.0f), 1.0f / sqrtf(lensq)) : mk(1.0f, 0.0f, 0.0f);
    v3 b2 = vcross(vh, b1);
    /* a point of the projected disc, warped to the visible half */
    float r = sqrtf(u0);
    float sp, cp;
    sco_sincos2pi(u1, &sp, &cp);
    float p1 = r * cp, p2 = r * sp;
    float h = 0.5f * (1.0f + vh.z);
    p2 = (1.0f - h) * sqrtf(fmaxf(0.0f, 1.0f - p1 * p1)) + h * p2;
    float p3 = sqrtf(fmaxf(0.0f, (1.0f - p1 * p1) - p2 * p2));
    v3 nh = vadd(vadd(vscale(b1, p1), vscale(b2, p2)), vscale(vh, p3));
    /* back to the alpha configuration and to world space */
    v3 ne = vnorm(mk(alpha * nh.x, alpha * nh.y, fmaxf(0.0f, nh.z)));
    v3 m = vnorm(vadd(vadd(vscale(t1, ne.x), vscale(t2, ne.y)), vscale(N, ne.z)));
    float ci = -vdot(d, m);
    if (!(ci > 0.0f)) return 0;
    float k = 1.0f - (eta * eta) * (1.0f - ci * ci);
    int refl;
    float ct = 0.0f;
    if (k <= 0.0f) {
        refl = 1;
    } else {
        ct = sqrtf(k);
        refl = uF < sco_fresnel(n1, n2, ci, ct);
    }
    v3 out;
    if (refl) out = vadd(d, vscale(m, ci + ci));
    else out = vadd(vscale(d, eta), vscale(m, eta * ci - ct));
    out = vnorm(out);
    float side = vdot(out, f->Nf);
    float on = vdot(out, N), om = vdot(out, m);
    int ok = refl ? (side > 0.0f && on > 0.0f && om > 0.0f) : (side < 0.0f && on < 0.0f && om < 0.0f);
    if (!ok) return 0;
    *dout = out;
    *refl_out = refl;
    *w_out = smith_g1(fabsf(on), a2);
    return 1;
}

int sco_rough_dielectric(const float d[3], const float n[3], float n1, float n2, float alpha, uint32_t count,
                         const float* u, float* d_out, int32_t* reflected, float* weight) {
    if (!d || !n || !u || !d_out || !reflected || !weight || !(alpha > 0.0f && alpha <= 1.0f)) return -1;
    frame_t f;
    v3 dd = mk(d[0], d[1], d[2]);
    f.P = mk(0.0f, 0.0f, 0.0f);
    f.Ng = mk(n[0], n[1], n[2]);
    f.entering = vdot(dd, f.Ng) < 0.0f;
    f.Nf = f.entering ? f.Ng : vneg(f.Ng);
    f.Ns = f.Nf;
    for (uint32_t i = 0; i < count; i++) {
        v3 out = mk(0.0f, 0.0f, 0.0f);
        int refl = 0;
        float w = 0.0f;
        if (!rough_dir(&f, dd, n1, n2, alpha, u[3 * (size_t)i], u[3 * (size_t)i + 1], u[3 * (size_t)i + 2],
                       &out, &refl, &w)) {
            refl = -1;
            w = 0.0f;
        }
        d_out[3 * (size_t)i] = out.x; d_out[3 * (size_t)i + 1] = out.y; d_out[3 * (size_t)i + 2] = out.z;
        reflected[i] = refl;
        weight[i] = w;
    }
    return 0;
}

/* ------------------------------------------------------------------ */
/* Absorption inside glass (Beer-Lambert): over a path length t in a    */
/* medium of absorption coefficient sigma the weight drops by            */
/* exp(-sigma t).  sigma is given at 450, 550 and 650 nm and taken       */
/* piecewise linear in lambda in between, constant outside.             */
/* ------------------------------------------------------------------ */

/* exp(-x) for x >= 0 with its own arithmetic, so that both sides of a
 * parity check compute the same bits: Cody-Waite reduction
 * x = k ln2 + r with |r| <= ln2 / 2 (ln2 split in a 16-bit head and a
 * tail, so k * head is exact), e^-r from its degree-7 Taylor polynomial
 * (truncation below 6e-9 relative on that interval), then the exact
 * scaling by 2^-k.  Results below 2^-125 are returned as 0. */
float sco_exp_neg(float x) {
    if (!(x > 0.0f)) return 1.0f;
    if (x > 87.0f) return 0.0f;
    float kf = floorf(x * 1.44269504f + 0.5f);
    int k = (int)kf;
    float r = (x - kf * 0.693145751953125f) - kf * 1.428606765330187e-06f;
    float q = -r;
    float p = (float)(1.0 / 5040.0) + q * (float)(1.0 / 40320.0);
    p = (float)(1.0 / 720.0) + q * p;
    p = (float)(1.0 / 120.0) + q * p;
    p = (float)(1.0 / 24.0) + q * p;
    p = (float)(1.0 / 6.0) + q * p;
    p = 0.5f + q * p;
    p = 1.0f + q * p;
    p = 1.0f + q * p;
    return p * i2f_bits((127 - k) << 23);
}

static float sigma_at(const sco_material* m, float lam) {
    if (lam <= 450.0f) return m->sigma[0];
    if (lam >= 650.0f) return m->sigma[2];
    if (lam < 550.0f) return m->sigma[0] + (m->sigma[1] - m->sigma[0]) * ((lam - 450.0f) / 100.0f);
    return m->sigma[1] + (m->sigma[2] - m->sigma[1]) * ((lam - 550.0f) / 100.0f);
}

/* ------------------------------------------------------------------ */
/* Nested and overlapping dielectrics (Schmidt and Budge, "Simple Nested */
/* Dielectrics in Ray Traced Images", J. Graphics Tools 7(2), 2002).     */
/* A path carries the set of dielectric objects it is inside, at most    */
/* MEDIA_CAP of them.  The medium at a point is the member of highest    */
/* priority (ties: the larger object id).  A surface of object k is a    */
/* real interface only if k is that member on the surface's inner side;  */
/* otherwise it lies inside a medium of higher priority and the path     */
/* crosses it unchanged, only the set changes (a false hit).  At a real  */
/* interface the index on the outer side is that of the medium left      */
/* when k is removed (air, n = 1, if none).  Refraction updates the set; */
/* reflection keeps it.  When the set is full, an object of lower        */
/* priority than every member is not added, else the lowest member is    */
/* replaced.                                                            */
/* ------------------------------------------------------------------ */

#define MEDIA_CAP 4
typedef struct { uint32_t id[MEDIA_CAP]; uint32_t n; } media_t;

static uint64_t med_key(const sco_scene* s, uint32_t k) { return ((uint64_t)s->mat[k].priority << 32) | k; }

static uint32_t med_top(const sco_scene* s, const media_t* L) {
    uint32_t best = 0;
    for (uint32_t i = 0; i < L->n; i++)
        if (best == 0 || med_key(s, L->id[i]) > med_key(s, best)) best = L->id[i];
    return best;
}

static void med_add(const sco_scene* s, media_t* L, uint32_t k) {
    for (uint32_t i = 0; i < L->n; i++) if (L->id[i] == k) return;
    if (L->n < MEDIA_CAP) { L->id[L->n++] = k; return; }
    uint32_t lo = 0;
    for (uint32_t i = 1; i < MEDIA_CAP; i++) if (med_key(s, L->id[i]) < med_key(s, L->id[lo])) lo = i;
    if (med_key(s, k) > med_key(s, L->id[lo])) L->id[lo] = k;
}

static void med_remove(media_t* L, uint32_t k) {
    for (uint32_t i = 0; i < L->n; i++)
        if (L->id[i] == k) { L->id[i] = L->id[L->n - 1]; L->n--; return; }
}

typedef struct { int real; float n1, n2; media_t after; } iface_t;

static void interface_at(const sco_scene* s, const media_t* L, uint32_t k, int entering, float lam, iface_t* I) {
    media_t in = *L, out = *L;
    med_add(s, &in, k);
    med_remove(&out, k);
    I->after = entering ? in : out;
    I->real = med_top(s, &in) == k;
    uint32_t o = med_top(s, &out);
    const sco_material* mk_ = &s->mat[k];
    float nk = cauchy_n(mk_->cauchy_a, mk_->cauchy_b, lam);
    float no = o ? cauchy_n(s->mat[o].cauchy_a, s->mat[o].cauchy_b, lam) : 1.0f;
    I->n1 = entering ? no : nk;
    I->n2 = entering ? nk : no;
}

/* Weight left after a segment of length t in the current medium. */
static float medium_weight(const sco_scene* s, const media_t* L, float lam, float t) {
    uint32_t o = med_top(s, L);
    if (!o) return 1.0f;
    float sg = sigma_at(&s->mat[o], lam);
    if (!(sg > 0.0f)) return 1.0f;
    return sco_exp_neg(sg * t);
}

int sco_media_step(const sco_scene* s, const uint32_t* ids, uint32_t n, uint32_t k, int entering, float lam,
                   uint32_t* ids_after, uint32_t* n_after, int* real, float* n1, float* n2) {
    if (!s || !s->mat || n > MEDIA_CAP || k == 0 || k >= s->n_mat) return -1;
    media_t L;
    L.n = n;
    for (uint32_t i = 0; i < n; i++) {
        if (ids[i] == 0 || ids[i] >= s->n_mat) return -1;
        L.id[i] = ids[i];
    }
    iface_t I;
    interface_at(s, &L, k, entering, lam, &I);
    for (uint32_t i = 0; i < I.after.n; i++) ids_after[i] = I.after.id[i];
    *n_after = I.after.n;
    *real = I.real;
    *n1 = I.n1;
    *n2 = I.n2;
    return 0;
}

/* ------------------------------------------------------------------ */
/* Scene-derived tables computed on the host in double.                 */
/* ------------------------------------------------------------------ */

typedef struct {
    uint32_t n_emit;
    uint32_t* emit_prim;
    float* emit_cdf;
    float a_tot;
    float cell_sx, cell_sy, inv_cell_area;
    float tex_sx, tex_sy;
    uint32_t n_entries;
} derived_t;

static void derive(const sco_scene* s, derived_t* D) {
    memset(D, 0, sizeof(*D));
    uint32_t ne = 0;
    for (uint32_t i = 0; i < s->nt; i++) if (s->mat[s->tri_obj[i]].type == 2) ne++;
    D->n_emit = ne;
    if (ne) {
        D->emit_prim = (uint32_t*)malloc(sizeof(uint32_t) * ne);
        D->emit_cdf = (float*)malloc(sizeof(float) * ne);
        double* area = (double*)malloc(sizeof(double) * ne);
        double tot = 0.0;
        uint32_t k = 0;
        for (uint32_t i = 0; i < s->nt; i++) {
            if (s->mat[s->tri_obj[i]].type != 2) continue;
            const uint32_t* idx = s->I + 3 * (size_t)i;
            double a[3], b[3], c[3];
            for (int j = 0; j < 3; j++) {
                a[j] = s->V[3 * (size_t)idx[0] + j]; b[j] = s->V[3 * (size_t)idx[1] + j]; c[j] = s->V[3 * (size_t)idx[2] + j];
            }
            double e1[3] = {b[0] - a[0], b[1] - a[1], b[2] - a[2]};
            double e2[3] = {c[0] - a[0], c[1] - a[1], c[2] - a[2]};
            double cx = e1[1] * e2[2] - e1[2] * e2[1];
            double cy = e1[2] * e2[0] - e1[0] * e2[2];
            double cz = e1[0] * e2[1] - e1[1] * e2[0];
            area[k] = 0.5 * sqrt(cx * cx + cy * cy + cz * cz);
            tot += area[k];
            D->emit_prim[k] = i;
            k++;
        }
        double cum = 0.0;
        for (uint32_t j = 0; j < ne; j++) {
            cum += area[j];
            D->emit_cdf[j] = (float)(cum / tot);
        }
        D->emit_cdf[ne - 1] = 1.0f;
        D->a_tot = (float)tot;
        free(area);
    }
    D->n_entries = s->n_pl + (ne > 0 ? 1u : 0u);
    if (s->recv_obj) {
        D->cell_sx = (float)s->recv_wc / s->recv_ext_u;
        D->cell_sy = (float)s->recv_hc / s->recv_ext_v;
        D->inv_cell_area = (float)(((double)s->recv_wc * (double)s->recv_hc) /
                                   ((double)s->recv_ext_u * (double)s->recv_ext_v));
    }
    if (s->tex || s->tex_rgb) {
        D->tex_sx = (float)s->tex_w / s->tex_ext_u;
        D->tex_sy = (float)s->tex_h / s->tex_ext_v;
    }
}

static void derive_free(derived_t* D) { free(D->emit_prim); free(D->emit_cdf); }

/* first index whose cdf exceeds u */
static uint32_t cdf_pick(const float* cdf, uint32_t n, float u) {
    for (uint32_t i = 0; i < n; i++) if (cdf[i] > u) return i;
    return n - 1;
}

/* nearest texel of the texture rectangle under P (edges clamped) */
static size_t texel_at(const sco_scene* s, const derived_t* D, v3 P) {
    float fx = (P.x - s->tex_x0) * D->tex_sx;
    float fy = (P.y - s->tex_y0) * D->tex_sy;
    int i = (int)floorf(fx), j = (int)floorf(fy);
    if (i < 0) i = 0;
    if (i > (int)s->tex_w - 1) i = (int)s->tex_w - 1;
    if (j < 0) j = 0;
    if (j > (int)s->tex_h - 1) j = (int)s->tex_h - 1;
    return (size_t)j * s->tex_w + (size_t)i;
}

/* Albedo at P for wavelength lam.  An RGB texel is read as reflectance
 * B at 450 nm, G at 550 nm and R at 650 nm, linear in lambda between
 * them and constant outside (the same rule as the absorption knots). */
static float albedo_at(const sco_scene* s, const derived_t* D, const sco_material* m, v3 P, float lam) {
    if (m->albedo_mode == 1) {
        int ix = (int)floorf(P.x), iy = (int)floorf(P.y);
        return ((ix + iy) & 1) == 0 ? m->rho_a : m->rho_b;
    }
    if (m->albedo_mode == 2 && s->tex) return s->tex[texel_at(s, D, P)];
    if (m->albedo_mode == 3 && s->tex_rgb) {
        const float* c = s->tex_rgb + 3 * texel_at(s, D, P);
        float r = c[0], g = c[1], b = c[2];
        if (lam <= 450.0f) return b;
        if (lam >= 650.0f) return r;
        if (lam < 550.0f) return b + (g - b) * ((lam - 450.0f) / 100.0f);
        return g + (r - g) * ((lam - 550.0f) / 100.0f);
    }
    return m->rho_a;
}

/* Grey albedo of the ground-truth output: the mean of an RGB texel. */
static float albedo_grey(const sco_scene* s, const derived_t* D, const sco_material* m, v3 P) {
    if (m->albedo_mode == 3 && s->tex_rgb) {
        const float* c = s->tex_rgb + 3 * texel_at(s, D, P);
        return ((c[0] + c[1]) + c[2]) / 3.0f;
    }
    return albedo_at(s, D, m, P, 550.0f);
}

/* Receiver cell of a point: floor of the scaled offset, the upper edge
 * clamped into the last cell; -1 outside the rectangle. */
static int64_t recv_cell(const sco_scene* s, const derived_t* D, v3 P) {
    float fx = (P.x - s->recv_x0) * D->cell_sx;
    float fy = (P.y - s->recv_y0) * D->cell_sy;
    if (!(fx >= 0.0f) || !(fy >= 0.0f) || fx > (float)s->recv_wc || fy > (float)s->recv_hc) return -1;
    uint32_t i = (uint32_t)fx, j = (uint32_t)fy;
    if (i >= s->recv_wc) i = s->recv_wc - 1;
    if (j >= s->recv_hc) j = s->recv_hc - 1;
    return (int64_t)j * s->recv_wc + i;
}

static uint32_t map_channels(const sco_wavelengths* wl) { return wl->mode == 0 ? wl->k : wl->bins; }

static uint32_t lambda_bin(const sco_wavelengths* wl, float lam) {
    float scale = (float)wl->bins / (wl->hi - wl->lo);
    float f = (lam - wl->lo) * scale;
    int b = (int)f;
    if (b < 0) b = 0;
    if (b > (int)wl->bins - 1) b = (int)wl->bins - 1;
    return (uint32_t)b;
}

static float lambda_uniform(const sco_wavelengths* wl, float u) { return wl->lo + u * (wl->hi - wl->lo); }

/* ------------------------------------------------------------------ */
/* Sensor curves for spectral samples: Gaussians of 40 nm width at 650,  */
/* 550 and 450 nm, each normalised to mean 1 over [lo, hi] so that a     */
/* flat spectrum maps to white; tabulated every 0.25 nm in double and    */
/* interpolated linearly in float.                                       */
/* ------------------------------------------------------------------ */

typedef struct { uint32_t n; float* tab[3]; float lo; } sensor_t;

static void sensor_make(const sco_wavelengths* wl, sensor_t* S) {
    const double mu[3] = {650.0, 550.0, 450.0};
    const double sigma = 40.0;
    uint32_t n = (uint32_t)((double)(wl->hi - wl->lo) * 4.0 + 0.5) + 1;
    S->n = n; S->lo = wl->lo;
    for (int c = 0; c < 3; c++) {
        double* g = (double*)malloc(sizeof(double) * n);
        for (uint32_t i = 0; i < n; i++) {
            double lam = (double)wl->lo + 0.25 * (double)i;
            double x = (lam - mu[c]) / sigma;
            g[i] = exp(-0.5 * x * x);
        }
        double sum = 0.0;
        for (uint32_t i = 0; i + 1 < n; i++) sum += 0.5 * (g[i] + g[i + 1]) * 0.25;
        double mean = sum / ((double)(n - 1) * 0.25);
        S->tab[c] = (float*)malloc(sizeof(float) * n);
        for (uint32_t i = 0; i < n; i++) S->tab[c][i] = (float)(g[i] / mean);
        free(g);
    }
}
static void sensor_free(sensor_t* S) { for (int c = 0; c < 3; c++) free(S->tab[c]); }

static float sensor_w(const sensor_t* S, int c, float lam) {
    float f = (lam - S->lo) * 4.0f;
    int i = (int)f;
    if (i < 0) i = 0;
    if (i > (int)S->n - 2) i = (int)S->n - 2;
    float fr = f - (float)i;
    float a = S->tab[c][i], b = S->tab[c][i + 1];
    return a + fr * (b - a);
}

/* ------------------------------------------------------------------ */
/* Light sampling shared by next-event estimation and photon emission.  */
/* A light "entry" is one point light or the set of emissive triangles; */
/* entries are picked uniformly, triangles proportionally to area, and  */
/* a point on a triangle uniformly (b0 = 1 - sqrt(u0), b2 = sqrt(u0) u1). */
/* ------------------------------------------------------------------ */

static v3 tri_point(const sco_scene* s, uint32_t prim, float u0, float u1, v3* Nl) {
    v3 p0, p1, p2;
    tri_verts(s, prim, &p0, &p1, &p2);
    float su = sqrtf(u0);
    float b0 = 1.0f - su;
    float b1 = su * (1.0f - u1);
    float b2 = su * u1;
    *Nl = vnorm(vcross(vsub(p1, p0), vsub(p2, p0)));
    return vadd(vadd(vscale(p0, b0), vscale(p1, b1)), vscale(p2, b2));
}

static uint32_t entry_pick(uint32_t n_entries, float u) {
    if (n_entries <= 1) return 0;
    uint32_t e = (uint32_t)(u * (float)n_entries);
    if (e > n_entries - 1) e = n_entries - 1;
    return e;
}

/* ------------------------------------------------------------------ */
/* Camera path (one pixel, sample, wavelength slot).                    */
/* ------------------------------------------------------------------ */

typedef struct {
    const sco_scene* s; const sco_bvh* bvh; const derived_t* D; const sco_wavelengths* wl;
    const float* map; uint32_t C; uint64_t seed; uint32_t max_depth;
    uint64_t segments;
    const sco_pm_rec* pm; uint64_t n_pm; double pm_scale; float pm_radius;   /* general photon map, or pm == NULL */
} pt_ctx;

static float pm_gather(const sco_pm_rec* recs, uint64_t n, double scale, float radius, v3 P, v3 N, uint32_t ch);

static float trace_path(pt_ctx* X, v3 o, v3 d, uint32_t pix, uint32_t sample, uint32_t slot, float lam) {
    const sco_scene* s = X->s;
    const derived_t* D = X->D;
    float T = 1.0f, L = 0.0f;
    int diffuse_seen = 0;
    media_t med;
    med.n = 0;   /* the camera is in air */
    for (uint32_t depth = 1; depth <= X->max_depth; depth++) {
        float t, u, v;
        uint32_t prim;
        closest_one(s, X->bvh, o, d, &t, &prim, &u, &v);
        X->segments++;
        if (prim == 0xffffffffu) break;
        T = T * medium_weight(s, &med, lam, t);
        uint32_t obj = s->tri_obj[prim];
        const sco_material* m = &s->mat[obj];
        frame_t f;
        hit_frame(s, prim, u, v, d, &f);
        if (m->type == 2) {
            if (!diffuse_seen && f.entering) L = L + T * m->le;
            break;
        }
        if (m->type == 1) {
            iface_t I;
            interface_at(s, &med, obj, f.entering, lam, &I);
            if (!I.real) {
                med = I.after;
                o = offset_ray(f.P, vneg(f.Nf));
                continue;
            }
            uint32_t r[4];
            rng_cam(X->seed, pix, sample, depth, 1, slot, r);
            v3 nd; int refl;
            if (m->roughness > 0.0f) {
                float w;
                if (!rough_dir(&f, d, I.n1, I.n2, m->roughness, u01(r[0]), u01(r[1]), u01(r[2]), &nd, &refl, &w))
                    break;
                T = T * w;
            } else if (!dielectric_dir(&f, d, I.n1, I.n2, u01(r[2]), &nd, &refl, NULL)) {
                break;
            }
            if (!refl) med = I.after;
            o = offset_ray(f.P, refl ? f.Nf : vneg(f.Nf));
            d = nd;
            continue;
        }
        /* diffuse (Lambertian, two-sided through the facing normal) */
        float rho = albedo_at(s, D, m, f.P, lam);
        diffuse_seen = 1;
        v3 os = offset_ray(f.P, f.Nf);
        /* caustic gather: the general photon map on every diffuse surface,
         * else the receiver map cell under the point */
        if (X->pm) {
            uint32_t b = (X->wl->mode == 0) ? slot : lambda_bin(X->wl, lam);
            float E = pm_gather(X->pm, X->n_pm, X->pm_scale, X->pm_radius, f.P, f.Nf, b);
            float g = ((T * rho) * INV_PI_F) * E;
            L = L + g;
        } else if (X->map && s->recv_obj && obj == s->recv_obj) {
            int64_t cell = recv_cell(s, D, f.P);
            if (cell >= 0) {
                uint32_t b = (X->wl->mode == 0) ? slot : lambda_bin(X->wl, lam);
                float E = X->map[(size_t)cell * X->C + b] * D->inv_cell_area;
                float g = ((T * rho) * INV_PI_F) * E;
                L = L + g;
            }
        }
        /* next event estimation: one light sample, one shadow ray */
        if (D->n_entries > 0) {
            uint32_t r[4];
            rng_cam(X->seed, pix, sample, depth, 2, slot, r);
            uint32_t e = entry_pick(D->n_entries, u01(r[2]));
            float contrib = 0.0f, tmax = 0.0f;
            uint32_t excl = 0xffffffffu;
            v3 om = mk(0, 0, 0);
            int shoot = 0;
            if (e < s->n_pl) {
                const float* lp = s->pl + 4 * (size_t)e;
                v3 w = vsub(mk(lp[0], lp[1], lp[2]), os);
                float r2 = vdot(w, w);
                float dist = sqrtf(r2);
                om = vscale(w, 1.0f / dist);
                float cosx = vdot(f.Nf, om);
                if (cosx > 0.0f) {
                    contrib = ((((T * rho) * INV_PI_F) * lp[3]) * cosx) / r2;
                    contrib = contrib * (float)D->n_entries;
                    contrib = contrib * medium_weight(s, &med, lam, dist);
                    tmax = dist;
                    shoot = 1;
                }
            } else {
                uint32_t k = cdf_pick(D->emit_cdf, D->n_emit, u01(r[3]));
                uint32_t lprim = D->emit_prim[k];
                v3 Nl;
                v3 y = tri_point(s, lprim, u01(r[0]), u01(r[1]), &Nl);
                v3 w = vsub(y, os);
                float r2 = vdot(w, w);
                float dist = sqrtf(r2);
                om = vscale(w, 1.0f / dist);
                float cosx = vdot(f.Nf, om);
                float cosl = -vdot(Nl, om);
                if (cosx > 0.0f && cosl > 0.0f) {
                    float le = s->mat[s->tri_obj[lprim]].le;
                    contrib = ((((((T * rho) * INV_PI_F) * le) * cosx) * cosl) / r2) * D->a_tot;
                    contrib = contrib * (float)D->n_entries;
                    contrib = contrib * medium_weight(s, &med, lam, dist);
                    tmax = dist * 0.9999f;
                    excl = lprim;
                    shoot = 1;
                }
            }
            if (shoot) {
                X->segments++;
                if (!any_one(s, X->bvh, os, om, tmax, excl)) L = L + contrib;
            }
        }
        if (depth == X->max_depth) break;
        /* cosine-weighted bounce */
        uint32_t r[4];
        rng_cam(X->seed, pix, sample, depth, 1, slot, r);
        d = cosine_dir(f.Nf, u01(r[0]), u01(r[1]));
        o = os;
        T = T * rho;
    }
    return L;
}

static int check_common(const sco_scene* s, const sco_wavelengths* wl, uint32_t max_depth) {
    if (!s || !wl || !s->V || !s->I || !s->tri_obj || !s->mat || s->nt == 0) return -1;
    if (max_depth == 0) return -1;
    if (wl->mode == 0 && !(wl->k == 1 || wl->k == 3)) return -1;
    if (wl->mode == 1 && (wl->bins == 0 || !(wl->hi > wl->lo))) return -1;
    if (wl->mode > 1) return -1;
    for (uint32_t i = 0; i < s->nt; i++) if (s->tri_obj[i] == 0 || s->tri_obj[i] >= s->n_mat) return -1;
    for (uint32_t k = 1; k < s->n_mat; k++) {
        const sco_material* m = &s->mat[k];
        if (m->type == 0 && m->albedo_mode == 3 && !s->tex_rgb) return -1;
        if (m->type != 1) continue;
        for (int c = 0; c < 3; c++) if (!(m->sigma[c] >= 0.0f && m->sigma[c] <= FLT_MAX)) return -1;
        if (!(m->roughness >= 0.0f && m->roughness <= 1.0f)) return -1;
    }
    return 0;
}

int sco_path_samples(const sco_scene* s, const sco_bvh* bvh, const sco_camera* cam, uint32_t spp,
                     uint32_t max_depth, const sco_wavelengths* wl, uint64_t seed, const float* caustic_map,
                     const uint32_t* pix, uint32_t n_pix, float* L, float* lambda) {
    if (check_common(s, wl, max_depth) || !cam || spp == 0 || !L) return -1;
    derived_t D;
    derive(s, &D);
    pt_ctx X = {s, bvh, &D, wl, caustic_map, map_channels(wl), seed, max_depth, 0, NULL, 0, 1.0, 0.0f};
    uint32_t K = wl->mode == 0 ? wl->k : 1;
    for (uint32_t sm = 0; sm < spp; sm++) {
        for (uint32_t i = 0; i < n_pix; i++) {
            uint32_t p = pix[i];
            uint32_t x = p % cam->w, y = p / cam->w;
            for (uint32_t slot = 0; slot < K; slot++) {
                uint32_t r[4];
                rng_cam(seed, p, sm, 0, 0, slot, r);
                float lam = wl->mode == 0 ? wl->nm[slot] : lambda_uniform(wl, u01(r[2]));
                v3 o, d;
                camera_ray(cam, x, y, u01(r[0]), u01(r[1]), &o, &d);
                size_t idx = ((size_t)sm * n_pix + i) * K + slot;
                L[idx] = trace_path(&X, o, d, p, sm, slot, lam);
                if (lambda) lambda[idx] = lam;
            }
        }
    }
    derive_free(&D);
    return 0;
}

/* ------------------------------------------------------------------ */
/* Render: film (ordered per-pixel sum over samples) and the ground-truth */
/* outputs of the pixel-centre ray.                                      */
/* ------------------------------------------------------------------ */

static int render_impl(const sco_scene* s, const sco_bvh* bvh, const sco_camera* cam, uint32_t spp,
                       uint32_t max_depth, const sco_wavelengths* wl, uint64_t seed, const float* caustic_map,
                       const sco_pm_rec* pm, uint64_t n_pm, float pm_radius,
                       const uint32_t* pix, uint32_t n_pix, sco_aov* out, uint64_t* segments) {
    if (check_common(s, wl, max_depth) || !cam || !out || spp == 0 || cam->w == 0 || cam->h == 0) return -1;
    derived_t D;
    derive(s, &D);
    sensor_t S;
    memset(&S, 0, sizeof(S));
    int spectral = wl->mode == 1;
    if (spectral) sensor_make(wl, &S);
    pt_ctx X = {s, bvh, &D, wl, caustic_map, map_channels(wl), seed, max_depth, 0,
                pm, n_pm, pm ? sco_pm_scale(pm, n_pm) : 1.0, pm_radius};
    uint32_t npx = pix ? n_pix : cam->w * cam->h;
    float inv_spp = 1.0f / (float)spp;
    v3 R = vnorm(mk(cam->right[0], cam->right[1], cam->right[2]));
    v3 U = vnorm(mk(cam->up[0], cam->up[1], cam->up[2]));
    v3 F = vnorm(mk(cam->fwd[0], cam->fwd[1], cam->fwd[2]));
    for (uint32_t i = 0; i < npx; i++) {
        uint32_t p = pix ? pix[i] : i;
        uint32_t x = p % cam->w, y = p / cam->w;
        if (out->rgb) {
            float acc[3] = {0.0f, 0.0f, 0.0f};
            for (uint32_t sm = 0; sm < spp; sm++) {
                if (!spectral) {
                    for (uint32_t slot = 0; slot < wl->k; slot++) {
                        uint32_t r[4];
                        rng_cam(seed, p, sm, 0, 0, slot, r);
                        v3 o, d;
                        camera_ray(cam, x, y, u01(r[0]), u01(r[1]), &o, &d);
                        float L = trace_path(&X, o, d, p, sm, slot, wl->nm[slot]);
                        if (wl->k == 3) acc[slot] = acc[slot] + L;
                        else { acc[0] = acc[0] + L; acc[1] = acc[1] + L; acc[2] = acc[2] + L; }
                    }
                } else {
                    uint32_t r[4];
                    rng_cam(seed, p, sm, 0, 0, 0, r);
                    float lam = lambda_uniform(wl, u01(r[2]));
                    v3 o, d;
                    camera_ray(cam, x, y, u01(r[0]), u01(r[1]), &o, &d);
                    float L = trace_path(&X, o, d, p, sm, 0, lam);
                    for (int c = 0; c < 3; c++) acc[c] = acc[c] + sensor_w(&S, c, lam) * L;
                }
            }
            for (int c = 0; c < 3; c++) out->rgb[3 * (size_t)p + c] = acc[c] * inv_spp;
        }
        /* pixel-centre ray: first surface, glass included */
        v3 o, d;
        camera_ray(cam, x, y, 0.5f, 0.5f, &o, &d);
        float t, u, v;
        uint32_t prim;
        closest_one(s, bvh, o, d, &t, &prim, &u, &v);
        X.segments++;
        uint32_t obj = 0;
        float dep = INFINITY, depn = 1.0f, alb = 0.0f;
        v3 N = mk(0, 0, 0), Nc = mk(0, 0, 0);
        if (prim != 0xffffffffu) {
            obj = s->tri_obj[prim];
            const sco_material* m = &s->mat[obj];
            frame_t f;
            hit_frame(s, prim, u, v, d, &f);
            dep = t;
            depn = fminf(t / 10.0f, 1.0f);
            N = f.Ns;
            Nc = mk(vdot(N, R), vdot(N, U), -vdot(N, F));
            alb = m->type == 0 ? albedo_grey(s, &D, m, f.P) : (m->type == 1 ? 1.0f : 0.0f);
        }
        if (out->obj) out->obj[p] = obj;
        if (out->trans) out->trans[p] = (uint8_t)(obj && s->mat[obj].type == 1);
        if (out->tri) out->tri[p] = prim;
        if (out->depth) out->depth[p] = dep;
        if (out->depthn) out->depthn[p] = depn;
        if (out->normal) { out->normal[3 * (size_t)p] = N.x; out->normal[3 * (size_t)p + 1] = N.y; out->normal[3 * (size_t)p + 2] = N.z; }
        if (out->normal_cam) { out->normal_cam[3 * (size_t)p] = Nc.x; out->normal_cam[3 * (size_t)p + 1] = Nc.y; out->normal_cam[3 * (size_t)p + 2] = Nc.z; }
        if (out->albedo) out->albedo[p] = alb;
        if (out->tie) {
            /* second-nearest distinct triangle along the same ray */
            uint8_t tie = 0;
            if (prim != 0xffffffffu) {
                double t2 = (double)nearest_other(s, bvh, o, d, prim);
                tie = (t2 - (double)t) < 1e-6 * (double)t;
            }
            out->tie[p] = tie;
        }
    }
    if (segments) *segments = X.segments;
    if (spectral) sensor_free(&S);
    derive_free(&D);
    return 0;
}

int sco_render(const sco_scene* s, const sco_bvh* bvh, const sco_camera* cam, uint32_t spp, uint32_t max_depth,
               const sco_wavelengths* wl, uint64_t seed, const float* caustic_map,
               const uint32_t* pix, uint32_t n_pix, sco_aov* out, uint64_t* segments) {
    return render_impl(s, bvh, cam, spp, max_depth, wl, seed, caustic_map, NULL, 0, 0.0f, pix, n_pix, out, segments);
}

int sco_render_pm(const sco_scene* s, const sco_bvh* bvh, const sco_camera* cam, uint32_t spp, uint32_t max_depth,
                  const sco_wavelengths* wl, uint64_t seed, const sco_pm_rec* recs, uint64_t n_rec, float radius,
                  const uint32_t* pix, uint32_t n_pix, sco_aov* out, uint64_t* segments) {
    if ((!recs && n_rec) || !(radius > 0.0f && radius <= FLT_MAX)) return -1;
    static const sco_pm_rec none;
    return render_impl(s, bvh, cam, spp, max_depth, wl, seed, NULL, recs ? recs : &none, n_rec, radius, pix, n_pix,
                       out, segments);
}

/* ------------------------------------------------------------------ */
/* Photons: emitted from the lights into cones around the photon target  */
/* spheres (one cone per target, picked in proportion to its solid angle */
/* 2 pi (1 - cos theta_k), direction uniform inside the cone), carried    */
/* through dielectrics, and stored on the receiver at the first diffuse   */
/* hit that follows at least one dielectric event.  The flux of a photon  */
/* is the light's power into all cones divided by the photon count of     */
/* its wavelength slot and by the number of cones containing its          */
/* direction (the exact mixture density).                               */
/* ------------------------------------------------------------------ */

/* The photon pass.  With recs == NULL, deposits go to the receiver map
 * (map_sum, count); otherwise every deposit, on any diffuse object, is
 * appended to recs in photon order (general photon map). */
static int photon_pass(const sco_scene* s, const sco_bvh* bvh, uint64_t n_photons, uint64_t p0, uint64_t p1,
                       uint32_t max_depth, const sco_wavelengths* wl, uint64_t seed,
                       double* map_sum, uint32_t* count, sco_pm_rec* recs, uint64_t cap, uint64_t* n_rec,
                       sco_photon_stats* stats) {
    derived_t D;
    derive(s, &D);
    uint32_t C = map_channels(wl);
    sco_photon_stats st;
    memset(&st, 0, sizeof(st));
    if (s->n_tg == 0 || D.n_entries == 0 || n_photons == 0) {
        if (stats) *stats = st;
        derive_free(&D);
        return 0;
    }
    uint32_t ntg = s->n_tg;
    float* cum = (float*)malloc(sizeof(float) * ntg);
    for (uint64_t p = p0; p < p1; p++) {
        uint32_t r0[4];
        rng_ph(seed, p, 0, 0, r0);
        uint32_t slot;
        float lam, nslot;
        if (wl->mode == 0) {
            slot = (uint32_t)(p % wl->k);
            lam = wl->nm[slot];
            uint64_t cnt = n_photons / wl->k + ((p % wl->k) < (n_photons % wl->k) ? 1u : 0u);
            (void)slot;
            nslot = (float)cnt;
        } else {
            lam = lambda_uniform(wl, u01(r0[3]));
            slot = lambda_bin(wl, lam);
            nslot = (float)n_photons / (float)wl->bins;
        }
        /* light point */
        uint32_t r2[4];
        rng_ph(seed, p, 0, 2, r2);
        uint32_t e = entry_pick(D.n_entries, u01(r2[2]));
        v3 y, Nl = mk(0, 0, 0);
        float power;
        int area = 0;
        if (e < s->n_pl) {
            const float* lp = s->pl + 4 * (size_t)e;
            y = mk(lp[0], lp[1], lp[2]);
            power = lp[3];
        } else {
            uint32_t k = cdf_pick(D.emit_cdf, D.n_emit, u01(r2[3]));
            uint32_t lprim = D.emit_prim[k];
            y = tri_point(s, lprim, u01(r2[0]), u01(r2[1]), &Nl);
            power = s->mat[s->tri_obj[lprim]].le * D.a_tot;
            area = 1;
        }
        /* cones towards the targets */
        float osum = 0.0f;
        for (uint32_t k = 0; k < ntg; k++) {
            const float* sp = s->tg_sph + 4 * (size_t)k;
            v3 dk = vsub(mk(sp[0], sp[1], sp[2]), y);
            float dist2 = vdot(dk, dk);
            float rr = sp[3] * sp[3];
            float q = rr / dist2;
            /* 1 - cos(theta_k), in a form without cancellation */
            float h = (q >= 1.0f) ? 2.0f : q / (1.0f + sqrtf(1.0f - q));
            osum = osum + TWO_PI_F * h;
            cum[k] = osum;
        }
        float target = u01(r0[0]) * osum;
        uint32_t kk = ntg - 1;
        for (uint32_t k = 0; k < ntg; k++) if (cum[k] > target) { kk = k; break; }
        const float* spk = s->tg_sph + 4 * (size_t)kk;
        v3 dkk = vsub(mk(spk[0], spk[1], spk[2]), y);
        float d2k = vdot(dkk, dkk);
        float qk = (spk[3] * spk[3]) / d2k;
        float hk = (qk >= 1.0f) ? 2.0f : qk / (1.0f + sqrtf(1.0f - qk));
        v3 axis = vscale(dkk, 1.0f / sqrtf(d2k));
        /* uniform in the cap: 1 - cos(theta) = u * h_k; sin^2 = g (2 - g) */
        float g = u01(r0[1]) * hk;
        float cost = 1.0f - g;
        float sint = sqrtf(fmaxf(0.0f, g * (2.0f - g)));
        float sp_, cp_;
        sco_sincos2pi(u01(r0[2]), &sp_, &cp_);
        v3 t1, t2;
        onb(axis, &t1, &t2);
        v3 om = vnorm(vadd(vadd(vscale(t1, cp_ * sint), vscale(t2, sp_ * sint)), vscale(axis, cost)));
        uint32_t m = 1;
        for (uint32_t k = 0; k < ntg; k++) {
            if (k == kk) continue;
            const float* sp = s->tg_sph + 4 * (size_t)k;
            v3 dk = vsub(mk(sp[0], sp[1], sp[2]), y);
            float dist2 = vdot(dk, dk);
            float q = (sp[3] * sp[3]) / dist2;
            v3 ax = vscale(dk, 1.0f / sqrtf(dist2));
            /* inside the cone: angle to the axis below theta_k, i.e. a
             * positive cosine and sin^2 = |om x ax|^2 <= sin^2 theta_k = q */
            v3 cr = vcross(om, ax);
            if (q >= 1.0f || (vdot(om, ax) > 0.0f && vdot(cr, cr) <= q)) m++;
        }
        float phi;
        v3 o;
        if (area) {
            float cy = vdot(Nl, om);
            if (!(cy > 0.0f)) { st.count[SCO_PH_EMIT_DEAD]++; continue; }
            phi = (((power * cy) * osum) * (float)D.n_entries) / (nslot * (float)m);
            o = offset_ray(y, Nl);
        } else {
            phi = ((power * osum) * (float)D.n_entries) / (nslot * (float)m);
            o = y;
        }
        v3 d = om;
        uint32_t spec = 0;
        media_t med;
        med.n = 0;   /* lights are in air */
        int outcome = SCO_PH_TRUNCATED;
        for (uint32_t depth = 1; depth <= max_depth; depth++) {
            float t, u, v;
            uint32_t prim;
            closest_one(s, bvh, o, d, &t, &prim, &u, &v);
            st.segments++;
            if (prim == 0xffffffffu) { outcome = SCO_PH_ESCAPED; break; }
            phi = phi * medium_weight(s, &med, lam, t);
            uint32_t obj = s->tri_obj[prim];
            const sco_material* mt = &s->mat[obj];
            frame_t f;
            hit_frame(s, prim, u, v, d, &f);
            if (mt->type == 2) { outcome = SCO_PH_ABSORBED; break; }
            if (mt->type == 1) {
                iface_t I;
                interface_at(s, &med, obj, f.entering, lam, &I);
                if (!I.real) {
                    med = I.after;
                    o = offset_ray(f.P, vneg(f.Nf));
                    continue;
                }
                uint32_t r1[4];
                rng_ph(seed, p, depth, 1, r1);
                v3 nd; int refl;
                if (mt->roughness > 0.0f) {
                    float w;
                    if (!rough_dir(&f, d, I.n1, I.n2, mt->roughness, u01(r1[0]), u01(r1[1]), u01(r1[2]), &nd, &refl,
                                   &w)) {
                        outcome = SCO_PH_LOST; break;
                    }
                    phi = phi * w;
                } else if (!dielectric_dir(&f, d, I.n1, I.n2, u01(r1[2]), &nd, &refl, NULL)) {
                    outcome = SCO_PH_LOST; break;
                }
                if (!refl) med = I.after;
                o = offset_ray(f.P, refl ? f.Nf : vneg(f.Nf));
                d = nd;
                spec++;
                continue;
            }
            if (spec == 0) { outcome = SCO_PH_DIRECT; break; }
            if (recs) {
                if (*n_rec >= cap) { free(cum); derive_free(&D); return -1; }
                sco_pm_rec* q = &recs[(*n_rec)++];
                q->pos[0] = f.P.x; q->pos[1] = f.P.y; q->pos[2] = f.P.z;
                q->nrm[0] = f.Nf.x; q->nrm[1] = f.Nf.y; q->nrm[2] = f.Nf.z;
                q->phi = phi;
                q->channel = slot;
                q->photon = p;
                outcome = SCO_PH_DEPOSITED;
                break;
            }
            if (obj != s->recv_obj) { outcome = SCO_PH_ELSEWHERE; break; }
            int64_t cell = recv_cell(s, &D, f.P);
            if (cell < 0) { outcome = SCO_PH_OUTSIDE; break; }
            size_t idx = (size_t)cell * C + slot;
            map_sum[idx] += (double)phi;
            if (count) count[idx]++;
            outcome = SCO_PH_DEPOSITED;
            break;
        }
        st.flux[outcome] += (double)phi;
        st.count[outcome]++;
    }
    free(cum);
    if (stats) *stats = st;
    derive_free(&D);
    return 0;
}

int sco_trace_photons(const sco_scene* s, const sco_bvh* bvh, uint64_t n_photons, uint64_t p0, uint64_t p1,
                      uint32_t max_depth, const sco_wavelengths* wl, uint64_t seed,
                      double* map_sum, uint32_t* count, sco_photon_stats* stats) {
    if (check_common(s, wl, max_depth) || !map_sum || !s->recv_obj || p1 > n_photons || p0 > p1) return -1;
    return photon_pass(s, bvh, n_photons, p0, p1, max_depth, wl, seed, map_sum, count, NULL, 0, NULL, stats);
}

int sco_pm_trace(const sco_scene* s, const sco_bvh* bvh, uint64_t n_photons, uint64_t p0, uint64_t p1,
                 uint32_t max_depth, const sco_wavelengths* wl, uint64_t seed,
                 sco_pm_rec* recs, uint64_t cap, uint64_t* n_rec, sco_photon_stats* stats) {
    if (check_common(s, wl, max_depth) || !recs || !n_rec || p1 > n_photons || p0 > p1) return -1;
    *n_rec = 0;
    return photon_pass(s, bvh, n_photons, p0, p1, max_depth, wl, seed, NULL, NULL, recs, cap, n_rec, stats);
}

/* ------------------------------------------------------------------ */
/* General photon map: density estimation over a disc.  The irradiance   */
/* of channel c at a surface point x with facing normal n is the flux of */
/* the stored photons of that channel within distance r of x, deposited  */
/* on the same side (n_p . n > 0), over the disc area pi r^2 (Jensen,     */
/* "Global Illumination using Photon Maps", EGWR 1996, with a fixed      */
/* radius).  The flux sum is exact: each photon's flux is taken in 64-bit */
/* fixed point, q = round(phi 2^S), with 2^S the largest power of two     */
/* such that n_stored * max(phi) * 2^S <= 2^62, so that no subset sum can */
/* overflow and the order of summation does not matter; then             */
/*   E = (float)(sum q * (1 / (2^S pi r^2)))  in double.                   */
/* ------------------------------------------------------------------ */

double sco_pm_scale(const sco_pm_rec* recs, uint64_t n) {
    float pmax = 0.0f;
    for (uint64_t i = 0; i < n; i++) if (recs[i].phi > pmax) pmax = recs[i].phi;
    if (n == 0 || !(pmax > 0.0f)) return 1.0;
    int e;
    frexp(ldexp(1.0, 62) / ((double)n * (double)pmax), &e);
    return ldexp(1.0, e - 1);
}

static float pm_gather(const sco_pm_rec* recs, uint64_t n, double scale, float radius, v3 P, v3 N, uint32_t ch) {
    float r2 = radius * radius;
    uint64_t sum = 0;
    for (uint64_t i = 0; i < n; i++) {
        const sco_pm_rec* q = &recs[i];
        if (q->channel != ch) continue;
        if (!(vdot(mk(q->nrm[0], q->nrm[1], q->nrm[2]), N) > 0.0f)) continue;
        v3 dlt = vsub(mk(q->pos[0], q->pos[1], q->pos[2]), P);
        if (vdot(dlt, dlt) < r2) sum += (uint64_t)nearbyint((double)q->phi * scale);
    }
    double c = 1.0 / ((scale * 3.14159265358979323846) * ((double)radius * (double)radius));
    return (float)((double)sum * c);
}

float sco_pm_gather(const sco_pm_rec* recs, uint64_t n, float radius, const float P[3], const float N[3],
                    uint32_t channel) {
    return pm_gather(recs, n, sco_pm_scale(recs, n), radius, mk(P[0], P[1], P[2]), mk(N[0], N[1], N[2]), channel);
}
