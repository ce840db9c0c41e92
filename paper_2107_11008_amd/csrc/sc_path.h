// sc_path.h -- per-ray and per-path device functions shared by the
// wavefront kernels (one stage per launch, queues between stages) and the
// persistent batched kernels (one lane follows a path to its end).  Both
// call exactly these functions, so their results are bit-identical.
#pragma once
#pragma clang fp contract(off)

#include "sc_device.h"

namespace scd {

constexpr int kLdsStack = 16;
constexpr int kStackMax = 160;   // maximum traversal stack entries per ray

// ---------------------------------------------------------------- traversal
// Reciprocal direction for the box tests only (the triangle test has its
// own exactly rounded divisions): the hardware reciprocal, within one ulp,
// scales an axis's crossing distances by at most 2^-23, far inside the
// relative margin of the box test.
__device__ __forceinline__ float safe_inv(float d) {
    const float a = fabsf(d) < 1e-20f ? copysignf(1e-20f, d) : d;
    return __builtin_amdgcn_rcpf(a);
}

// search bound: a node is visited if its entry distance is within a
// relative margin of the best hit, so equal-distance triangles with a
// smaller index in other nodes are still found
__device__ __forceinline__ float search_limit(float t) { return t + t * 9.765625e-04f; }

// traversal stack: the first kLdsStack entries of each lane in LDS, deeper
// entries in a private (scratch) array
struct Spill {
    uint2 e[kStackMax - kLdsStack];
};

template <int BS>
__device__ __forceinline__ void push(uint2 (*lds)[BS], Spill& s, int& sp, uint2 e) {
    if (sp < kLdsStack) lds[sp][threadIdx.x] = e;
    else s.e[sp - kLdsStack] = e;
    ++sp;
}
// The spill side is read through a volatile reference: otherwise the
// compiler merges both reads into one generic (flat) load through a
// selected address, which is slower than an LDS read and waits for every
// outstanding memory operation.
template <int BS>
__device__ __forceinline__ uint2 pop(uint2 (*lds)[BS], Spill& s, int& sp) {
    --sp;
    if (sp < kLdsStack) return lds[sp][threadIdx.x];
    const volatile uint2& v = s.e[sp - kLdsStack];
    return make_uint2(v.x, v.y);
}

__device__ __forceinline__ void cswap(uint32_t& ka, uint32_t& va, uint32_t& kb, uint32_t& vb) {
    const bool sw = kb < ka;
    const uint32_t k0 = sw ? kb : ka, k1 = sw ? ka : kb;
    const uint32_t v0 = sw ? vb : va, v1 = sw ? va : vb;
    ka = k0; kb = k1; va = v0; vb = v1;
}

// Batcher's odd-even merge sort of 8 (key, value) pairs, ascending keys
__device__ __forceinline__ void sort8(uint32_t* k, uint32_t* v) {
#define SC_CS(a, b) cswap(k[a], v[a], k[b], v[b])
    SC_CS(0, 1); SC_CS(2, 3); SC_CS(4, 5); SC_CS(6, 7);
    SC_CS(0, 2); SC_CS(1, 3); SC_CS(4, 6); SC_CS(5, 7);
    SC_CS(1, 2); SC_CS(5, 6);
    SC_CS(0, 4); SC_CS(1, 5); SC_CS(2, 6); SC_CS(3, 7);
    SC_CS(2, 4); SC_CS(3, 5);
    SC_CS(1, 2); SC_CS(3, 4); SC_CS(5, 6);
#undef SC_CS
}

struct NodeTest {
    uint32_t key[8];
    uint32_t ref[8];
};

// One fetch serves both kinds of step: 14 float4 from the step's base, a
// node (its child boxes and child words) or a leaf (up to 4 triangles of 48
// bytes, contiguous in the leaf-ordered array; the array is padded so the
// fetch stays inside it).  Every lane issues the same loads, so a wave whose
// lanes are at nodes and at leaves waits for one memory round trip, not
// two.  For a node the plane pairs of each axis are fetched near first:
// word index j ^ flip, flip = 2 on axes with a negative direction
// component (the node stores lower planes in words 0-1 of each axis and
// upper planes in words 2-3); leaves use flip = 0.
struct Fetch {
    float4 q[14];
};

__device__ __forceinline__ void fetch14(const float4* __restrict__ base, uint32_t fx, uint32_t fy, uint32_t fz,
                                        Fetch& f) {
#pragma unroll
    for (int j = 0; j < 4; ++j) f.q[j] = base[j ^ fx];
#pragma unroll
    for (int j = 4; j < 8; ++j) f.q[j] = base[j ^ fy];
#pragma unroll
    for (int j = 8; j < 12; ++j) f.q[j] = base[j ^ fz];
    f.q[12] = base[12];
    f.q[13] = base[13];
    // all 14 values are taken here, before the node/leaf branch: otherwise
    // the compiler moves the loads only one branch reads into that branch,
    // which brings back the second round trip (the asm is empty)
#pragma unroll
    for (int j = 0; j < 14; ++j) asm volatile("" ::"v"(f.q[j].x), "v"(f.q[j].y), "v"(f.q[j].z), "v"(f.q[j].w));
}

// Box tests of the 8 children of a fetched node.  A plane p is crossed at
// t = p * inv + c with c = -o * inv (one fused multiply-add per plane).
// Against t = (p - o) * inv its absolute error is at most 2^-23 |c| plus a
// relative 2^-24, so the near offsets are lowered and the far offsets
// raised by 2^-21 |c| per axis: every box the two-operation form admits is
// admitted (the relative margin on the far distance covers the rest, as it
// covers the rounding of the triangle test), and the hits do not change.
// key = entry distance bits, or 0xffffffff when the child is missed or
// lies beyond tlim.
__device__ __forceinline__ void test_node(const Fetch& f, F3 c, F3 inv, float tlim, NodeTest& r) {
    const float4* q = f.q;
    const float nx[8] = {q[0].x, q[0].y, q[0].z, q[0].w, q[1].x, q[1].y, q[1].z, q[1].w};
    const float fx[8] = {q[2].x, q[2].y, q[2].z, q[2].w, q[3].x, q[3].y, q[3].z, q[3].w};
    const float ny[8] = {q[4].x, q[4].y, q[4].z, q[4].w, q[5].x, q[5].y, q[5].z, q[5].w};
    const float fy[8] = {q[6].x, q[6].y, q[6].z, q[6].w, q[7].x, q[7].y, q[7].z, q[7].w};
    const float nz[8] = {q[8].x, q[8].y, q[8].z, q[8].w, q[9].x, q[9].y, q[9].z, q[9].w};
    const float fz[8] = {q[10].x, q[10].y, q[10].z, q[10].w, q[11].x, q[11].y, q[11].z, q[11].w};
    const uint32_t ch[8] = {__float_as_uint(q[12].x), __float_as_uint(q[12].y), __float_as_uint(q[12].z),
                            __float_as_uint(q[12].w), __float_as_uint(q[13].x), __float_as_uint(q[13].y),
                            __float_as_uint(q[13].z), __float_as_uint(q[13].w)};
    const float mx = fabsf(c.x) * 4.76837158203125e-07f, my = fabsf(c.y) * 4.76837158203125e-07f,
                mz = fabsf(c.z) * 4.76837158203125e-07f;   // 2^-21 |c|
    const F3 cn{c.x - mx, c.y - my, c.z - mz}, cf{c.x + mx, c.y + my, c.z + mz};
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        const float tnx = fmaf(nx[k], inv.x, cn.x), tfx = fmaf(fx[k], inv.x, cf.x);
        const float tny = fmaf(ny[k], inv.y, cn.y), tfy = fmaf(fy[k], inv.y, cf.y);
        const float tnz = fmaf(nz[k], inv.z, cn.z), tfz = fmaf(fz[k], inv.z, cf.z);
        const float tn = fmaxf(fmaxf(tnx, tny), fmaxf(tnz, 0.0f));
        const float tf = fminf(fminf(tfx, tfy), tfz);
        const bool hit = (tn <= fmaf(fabsf(tf), 9.765625e-04f, tf)) && (tn <= tlim);
        r.key[k] = hit ? __float_as_uint(tn) : 0xffffffffu;
        r.ref[k] = ch[k];
    }
}

__device__ __forceinline__ F3 perm(const RayPre& r, float4 p) { return permute(r, F3{p.x, p.y, p.z}); }

struct HitRec {
    float t, u, v;
    uint32_t prim;
};

struct VisitCount {
    unsigned long long nodes = 0, tris = 0;
};

// Resumable traversal of one ray, closest hit or any hit.
//  * closest hit: the lexicographic minimum of (t, triangle) over the scene;
//  * any hit: is there a triangle other than excl with 0 < t < tmax?
// A step visits one node or one leaf and returns true when the ray is done
// (then trav_result, or Trav::hit for an any-hit ray, is final).  Any
// visiting order gives the same result: boxes are tested conservatively
// and closest hits are compared by (t, triangle).  MODE fixes the kind at
// compile time (kClosest, kAny) or reads it from the state (kEither), so
// one kernel can follow camera rays and shadow rays with the same code.
enum TravMode { kClosest = 0, kAny = 1, kEither = 2 };

struct Trav {
    RayPre rp;
    F3 c, inv;         // a plane p is crossed at p * inv + c (see test_node)
    float tb;          // closest: best t so far; any: tmax
    float bV, bW, brcp;
    uint32_t pb;       // closest: best triangle; any: the excluded triangle
    uint32_t ref;
    uint32_t flip;     // per-axis node word flips, 2 bits each (see fetch14)
    int sp;
    bool any, hit;
};

__device__ __forceinline__ uint32_t axis_flips(F3 inv) {
    return (inv.x >= 0.0f ? 0u : 2u) | (inv.y >= 0.0f ? 0u : 2u) << 2 | (inv.z >= 0.0f ? 0u : 2u) << 4;
}

// base of a step's fetch and its word flips: the node, or the leaf's
// first triangle with no flips
__device__ __forceinline__ const float4* step_base(const DevScene& S, uint32_t ref, uint32_t flip, uint32_t& fl) {
    if (ref & SC_LEAF_BIT) {
        fl = 0u;
        return S.tris + 3 * (size_t)(ref & SC_LEAF_FIRST_MASK);
    }
    fl = flip;
    return reinterpret_cast<const float4*>(S.nodes + ref);
}

__device__ __forceinline__ void trav_begin(Trav& t, F3 o, F3 d, bool any, float tmax, uint32_t excl) {
    t.rp = ray_prepare(o, d);
    t.inv = F3{safe_inv(d.x), safe_inv(d.y), safe_inv(d.z)};
    t.c = F3{-(o.x * t.inv.x), -(o.y * t.inv.y), -(o.z * t.inv.z)};
    t.flip = axis_flips(t.inv);
    t.tb = any ? tmax : INFINITY;
    t.pb = any ? excl : 0xffffffffu;
    t.bV = 0.0f; t.bW = 0.0f; t.brcp = 0.0f;
    t.ref = 0;   // root node
    t.sp = 0;
    t.any = any;
    t.hit = false;
}

__device__ __forceinline__ void trav_init(Trav& t, F3 o, F3 d) { trav_begin(t, o, d, false, 0.0f, 0u); }
__device__ __forceinline__ void any_init(Trav& t, F3 o, F3 d, float tmax, uint32_t excl) {
    trav_begin(t, o, d, true, tmax, excl);
}

// Triangle k of a leaf fetch (k < 4) or, past the fetch, from memory.
__device__ __forceinline__ void leaf_tri(const DevScene& S, const Fetch& f, uint32_t first, uint32_t k, float4& a,
                                         float4& b, float4& c) {
    if (k < 4) {
        a = f.q[3 * k]; b = f.q[3 * k + 1]; c = f.q[3 * k + 2];
    } else {
        const float4* tp = S.tris + 3 * (size_t)(first + k);
        a = tp[0]; b = tp[1]; c = tp[2];
    }
}

// LDS-staged top of the tree: the collapse numbers nodes level by level,
// so nodes [0, kTopNodes) are the root and its children; a kernel may copy
// them into LDS once per block and pass the copy as `top` (then their
// fetches read LDS), or pass nullptr.
constexpr uint32_t kTopNodes = 9;
constexpr uint32_t kTopMinNodes = 65536;   // trees smaller than this keep their top in cache anyway

template <int BS, bool COUNT, int MODE>
__device__ __forceinline__ bool tstep(const DevScene& S, Trav& t, uint2 (*lds)[BS], Spill& st, VisitCount& vc,
                                      const float4* top = nullptr) {
    const bool any = MODE == kAny ? true : (MODE == kClosest ? false : t.any);
    uint32_t fl;
    const float4* base = step_base(S, t.ref, t.flip, fl);
    Fetch f;
    if (top && !(t.ref & SC_LEAF_BIT) && t.ref < kTopNodes) {
        const float4* q = top + 16 * t.ref;
        const uint32_t fx = fl & 3u, fy = (fl >> 2) & 3u, fz = fl >> 4;
#pragma unroll
        for (int j = 0; j < 4; ++j) f.q[j] = q[j ^ fx];
#pragma unroll
        for (int j = 4; j < 8; ++j) f.q[j] = q[j ^ fy];
#pragma unroll
        for (int j = 8; j < 12; ++j) f.q[j] = q[j ^ fz];
        f.q[12] = q[12];
        f.q[13] = q[13];
    } else {
        fetch14(base, fl & 3u, (fl >> 2) & 3u, fl >> 4, f);
    }
    if (!(t.ref & SC_LEAF_BIT)) {
        NodeTest nt;
        test_node(f, t.c, t.inv, search_limit(t.tb), nt);
        if (COUNT) ++vc.nodes;
        if (MODE == kAny) {
            // order does not matter for a yes/no answer
#pragma unroll
            for (int c = 0; c < 8; ++c)
                if (nt.key[c] != 0xffffffffu) push<BS>(lds, st, t.sp, make_uint2(nt.ref[c], nt.key[c]));
        } else {
            sort8(nt.key, nt.ref);
            if (nt.key[0] != 0xffffffffu) {
#pragma unroll
                for (int c = 7; c >= 1; --c)
                    if (nt.key[c] != 0xffffffffu) push<BS>(lds, st, t.sp, make_uint2(nt.ref[c], nt.key[c]));
                t.ref = nt.ref[0];
                return false;
            }
        }
    } else {
        const uint32_t first = t.ref & SC_LEAF_FIRST_MASK;
        const uint32_t cnt = ((t.ref >> 28) & 7u) + 1u;
        if (COUNT) vc.tris += cnt;
        for (uint32_t k = 0; k < cnt; ++k) {
            float4 a, b, c;
            leaf_tri(S, f, first, k, a, b, c);
            const uint32_t prim = __float_as_uint(a.w);
            if (any && prim == t.pb) continue;
            TriHit h;
            if (tri_test(t.rp, perm(t.rp, a), perm(t.rp, b), perm(t.rp, c), h)) {
                if (any) {
                    if (h.t < t.tb) {
                        t.hit = true;
                        return true;
                    }
                } else if (h.t < t.tb || (h.t == t.tb && prim < t.pb)) {
                    t.tb = h.t; t.pb = prim; t.bV = h.V; t.bW = h.W; t.brcp = h.rcp;
                }
            }
        }
    }
    if (MODE == kAny) {
        if (t.sp == 0) return true;
        t.ref = pop<BS>(lds, st, t.sp).x;
        return false;
    }
    // next entry from the stack that is still within reach (an any-hit
    // ray pushed only entries within reach of tmax)
    while (t.sp > 0) {
        const uint2 e = pop<BS>(lds, st, t.sp);
        if (__uint_as_float(e.y) <= search_limit(t.tb)) {
            t.ref = e.x;
            return false;
        }
    }
    return true;
}

template <int BS, bool COUNT>
__device__ __forceinline__ bool trav_step(const DevScene& S, Trav& t, uint2 (*lds)[BS], Spill& st, VisitCount& vc,
                                          const float4* top = nullptr) {
    return tstep<BS, COUNT, kClosest>(S, t, lds, st, vc, top);
}

__device__ __forceinline__ HitRec trav_result(const Trav& t) {
    return HitRec{t.tb, t.bV * t.brcp, t.bW * t.brcp, t.pb};
}

template <int BS, bool COUNT>
__device__ __forceinline__ HitRec trace_closest(const DevScene& S, F3 o, F3 d, uint2 (*lds)[BS], Spill& st,
                                                VisitCount& vc) {
    Trav t;
    trav_init(t, o, d);
    while (!tstep<BS, COUNT, kClosest>(S, t, lds, st, vc)) {
    }
    return trav_result(t);
}

template <int BS, bool COUNT>
__device__ __forceinline__ bool trace_any(const DevScene& S, F3 o, F3 d, float tmax, uint32_t excl, uint2 (*lds)[BS],
                                          Spill& st, VisitCount& vc) {
    Trav t;
    any_init(t, o, d, tmax, excl);
    while (!tstep<BS, COUNT, kAny>(S, t, lds, st, vc)) {
    }
    return t.hit;
}
template <int BS>
__device__ __forceinline__ bool trace_any(const DevScene& S, F3 o, F3 d, float tmax, uint32_t excl, uint2 (*lds)[BS],
                                          Spill& st) {
    VisitCount vc;
    return trace_any<BS, false>(S, o, d, tmax, excl, lds, st, vc);
}

// ---------------------------------------------------------------- camera paths
// ---------------------------------------------------------------- nested dielectrics
// Each path carries the set of dielectric objects it is inside (the
// nested-dielectric rules of Schmidt and Budge, J. Graphics Tools 7(2),
// 2002): up to kMedia object ids of 16 bits in one 64-bit word, ordered by
// descending (priority, object id), unused entries 0.  The medium at the
// path is the first entry.  A surface of object k is a real interface only
// where k heads the set on its inner side; elsewhere it lies inside a
// medium of higher priority and the path crosses it unchanged, only the
// set changes.  At a real interface the index on the outer side is that of
// the set's head once k is removed (air, n = 1, if none).  Refraction takes
// the set across the surface, reflection keeps the old one.  A full set
// drops its last entry to admit a higher-ranked object and ignores a lower
// one.
constexpr int kMedia = 4;

__device__ __forceinline__ uint64_t media_key(const DevScene& S, uint32_t id) {
    return ((uint64_t)S.mat[id].priority << 32) | id;
}
__device__ __forceinline__ uint32_t media_entry(uint64_t M, int i) { return (uint32_t)(M >> (16 * i)) & 0xffffu; }

__device__ __forceinline__ uint64_t media_add(const DevScene& S, uint64_t M, uint32_t k) {
    const uint64_t kk = media_key(S, k);
    uint32_t e[kMedia];
    int pos = 0;
    for (int i = 0; i < kMedia; ++i) {
        e[i] = media_entry(M, i);
        if (e[i] == k) return M;
        if (e[i] != 0u && media_key(S, e[i]) > kk) pos = i + 1;
    }
    if (pos == kMedia) return M;
    uint64_t out = 0ull;
    for (int j = 0, i = 0; j < kMedia; ++j) {
        const uint32_t v = j == pos ? k : e[i++];
        out |= (uint64_t)v << (16 * j);
    }
    return out;
}

__device__ __forceinline__ uint64_t media_remove(uint64_t M, uint32_t k) {
    for (int i = 0; i < kMedia; ++i) {
        if (media_entry(M, i) == k) {
            const uint64_t low = M & ((1ull << (16 * i)) - 1ull);
            const uint64_t high = i + 1 < kMedia ? (M >> (16 * (i + 1))) << (16 * i) : 0ull;
            return low | high;
        }
    }
    return M;
}

struct Crossing {
    bool real;        // a true interface (else the path passes straight on)
    float n1, n2;     // index on the incoming side and across
    uint64_t after;   // the set on the far side
};

__device__ __forceinline__ Crossing media_cross(const DevScene& S, uint64_t M, uint32_t k, bool entering, float lam) {
    const uint64_t in = media_add(S, M, k), out = media_remove(M, k);
    Crossing c;
    c.after = entering ? in : out;
    c.real = media_entry(in, 0) == k;
    const uint32_t o = media_entry(out, 0);
    const sc_material mk = S.mat[k];
    const float nk = cauchy_index(mk.cauchy_a, mk.cauchy_b, lam);
    float no = 1.0f;
    if (o != 0u) {
        const sc_material mo = S.mat[o];
        no = cauchy_index(mo.cauchy_a, mo.cauchy_b, lam);
    }
    c.n1 = entering ? no : nk;
    c.n2 = entering ? nk : no;
    return c;
}

// weight kept over a segment of length t in the medium heading set M
__device__ __forceinline__ float medium_weight(const DevScene& S, uint64_t M, float lam, float t) {
    const uint32_t o = media_entry(M, 0);
    if (o == 0u) return 1.0f;
    const float sg = absorption(S.mat[o], lam);
    if (!(sg > 0.0f)) return 1.0f;
    return exp_neg(sg * t);
}

// ---------------------------------------------------------------- general photon map
// Irradiance of channel ch at P (facing normal N): the fixed-point flux of
// the stored photons of that channel on the same side (n_p . N > 0) within
// r of P, times 1 / (2^S pi r^2).  Cells are 2.25 r wide and offset by half
// a cell (a floor at a multiple of the width lies mid-cell); the cells
// overlapping the box P +- 1.1 r, at most 2 per axis, are visited through
// their buckets, whose ranges are all loaded before any record so the
// misses overlap.  A bucket holds one channel only (its low bits), and a
// record counts only in its own cell (its packed cell coordinates are
// stored with it), so a bucket shared by two visited cells is not counted
// twice.  The integer sum does not depend on the order of the records.
// Points more than 2^20 cells from the origin are far from every stored
// photon (those lie within 2^16 cells).
__device__ __forceinline__ int pm_cell(float v, float inv_h) { return (int)floorf(v * inv_h + 0.5f); }

// packed cell coordinates (18 bits each, offset by 2^17): low 32 bits and high 22
__device__ __forceinline__ uint64_t pm_tag(int x, int y, int z) {
    return (uint64_t)((uint32_t)(x + 131072) & 0x3ffffu) | ((uint64_t)((uint32_t)(y + 131072) & 0x3ffffu) << 18) |
           ((uint64_t)((uint32_t)(z + 131072) & 0x3ffffu) << 36);
}

// the channel is the low cbits of the bucket, so a bucket holds one
// channel and the buckets of one cell's channels are adjacent
__device__ __forceinline__ uint32_t pm_bucket(int x, int y, int z, uint32_t ch, uint32_t cbits, uint32_t mask) {
    const uint32_t h = ((uint32_t)x * 73856093u) ^ ((uint32_t)y * 19349663u) ^ ((uint32_t)z * 83492791u);
    return ((h << cbits) | ch) & mask;
}

__device__ __forceinline__ float pmap_gather(const PMapDev& pm, F3 P, F3 N, uint32_t ch) {
    const float lim = 1048576.0f;
    if (!(fabsf(P.x * pm.inv_h) < lim && fabsf(P.y * pm.inv_h) < lim && fabsf(P.z * pm.inv_h) < lim)) return 0.0f;
    const float rr = pm.r * 1.1f;
    const int x0 = pm_cell(P.x - rr, pm.inv_h), nx = min(pm_cell(P.x + rr, pm.inv_h) - x0, 1);
    const int y0 = pm_cell(P.y - rr, pm.inv_h), ny = min(pm_cell(P.y + rr, pm.inv_h) - y0, 1);
    const int z0 = pm_cell(P.z - rr, pm.inv_h), nz = min(pm_cell(P.z + rr, pm.inv_h) - z0, 1);
    uint32_t s0[8], s1[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) {
        const int dx = j & 1, dy = (j >> 1) & 1, dz = j >> 2;
        s0[j] = 0u;
        s1[j] = 0u;
        if (dx <= nx && dy <= ny && dz <= nz) {
            const uint32_t b = pm_bucket(x0 + dx, y0 + dy, z0 + dz, ch, pm.cbits, pm.mask);
            s0[j] = pm.start[b];
            s1[j] = pm.start[b + 1];
        }
    }
    unsigned long long sum = 0ull;
    for (int j = 0; j < 8; ++j) {
        const uint64_t tag = pm_tag(x0 + (j & 1), y0 + ((j >> 1) & 1), z0 + (j >> 2));
        const uint32_t tlo = (uint32_t)tag, thi = (uint32_t)(tag >> 32);
        for (uint32_t k = s0[j]; k < s1[j]; ++k) {
            const float4 a = pm.rec[2 * (size_t)k];
            const float4 b = pm.rec[2 * (size_t)k + 1];
            if (__float_as_uint(a.w) != tlo || __float_as_uint(b.w) != thi) continue;
            const F3 dl = F3{a.x, a.y, a.z} - P;
            if (!(dot(dl, dl) < pm.r2)) continue;
            const F3 n{b.x, b.y, b.z};
            if (dot(n, N) > 0.0f) sum += pm.q[k];
        }
    }
    return (float)((double)sum * pm.c);
}

struct CamPath {
    F3 o, d;
    float T, L, lam;
    uint32_t flags;   // bit 0: a diffuse vertex was seen
    uint64_t med;     // media set (the camera is in air)
};

struct ShadowReq {
    F3 o, d;
    float tmax, contrib;
    uint32_t excl;
    bool shoot;
};

// ray through the jittered film point; wavelength of the slot (fixed) or
// drawn uniformly (spectral); throughput 1, radiance 0
__device__ __forceinline__ CamPath camera_start(const sc_camera& cam, const WaveDev& wl, uint64_t seed, uint32_t pix,
                                                uint32_t sample, uint32_t slot) {
    CamPath P;
    const uint32_t x = pix % cam.w, y = pix / cam.w;
    const U4 r = rng_camera(seed, pix, sample, 0, 0, slot);
    P.lam = wl.mode == SC_WL_FIXED ? wl.nm[slot] : lambda_from(wl, unit(r.c));
    camera_ray(cam, x, y, unit(r.a), unit(r.b), P.o, P.d);
    P.T = 1.0f;
    P.L = 0.0f;
    P.flags = 0u;
    P.med = 0ull;
    return P;
}

// emitter hit: its front-face radiance counts only before any diffuse vertex
__device__ __forceinline__ void camera_emission(const DevScene& S, const HitRec& h, CamPath& P) {
    if (P.flags & 1u) return;
    const sc_material m = S.mat[S.tri_obj[h.prim]];
    F3 p0, p1, p2;
    tri_vertices(S, h.prim, p0, p1, p2);
    const F3 Ng = normalize(cross(p1 - p0, p2 - p0));
    const float T = P.T * medium_weight(S, P.med, P.lam, h.t);
    if (dot(P.d, Ng) < 0.0f) P.L = P.L + T * m.le;
}

// dielectric hit: absorption over the segment, then reflect, refract
// (smooth, or through a GGX microfacet with its weight) or, for a surface
// hidden inside a higher-priority medium, pass straight on; false if the
// path ends here
__device__ __forceinline__ bool camera_dielectric(const DevScene& S, uint64_t seed, uint32_t pix, uint32_t sample,
                                                  uint32_t slot, uint32_t depth, uint32_t max_depth, const HitRec& h,
                                                  CamPath& P) {
    P.T = P.T * medium_weight(S, P.med, P.lam, h.t);
    const Frame f = hit_frame(S, h.prim, h.u, h.v, P.d);
    const Crossing c = media_cross(S, P.med, S.tri_obj[h.prim], f.entering, P.lam);
    if (!c.real) {
        P.med = c.after;
        P.o = offset_ray(f.P, neg(f.Nf));
        return depth < max_depth;
    }
    const U4 r = rng_camera(seed, pix, sample, depth, 1, slot);
    F3 nd;
    bool refl;
    const float alpha = S.mat[S.tri_obj[h.prim]].roughness;
    if (alpha > 0.0f) {
        float w;
        if (!rough_dielectric(f, P.d, c.n1, c.n2, alpha, unit(r.a), unit(r.b), unit(r.c), nd, refl, w)) return false;
        P.T = P.T * w;
    } else if (!dielectric(f, P.d, c.n1, c.n2, unit(r.c), nd, refl)) {
        return false;
    }
    if (!refl) P.med = c.after;
    P.o = offset_ray(f.P, refl ? f.Nf : neg(f.Nf));
    P.d = nd;
    return depth < max_depth;
}

// diffuse hit: caustic gather added to L, one light sample prepared as a
// shadow ray (its contribution is added if unoccluded), cosine-weighted
// bounce; false if the path ends here
__device__ __forceinline__ bool camera_diffuse(const DevScene& S, const WaveDev& wl, const float* __restrict__ cmap,
                                               const PMapDev& pm, uint64_t seed, uint32_t pix, uint32_t sample,
                                               uint32_t slot, uint32_t depth, uint32_t max_depth, const HitRec& h,
                                               CamPath& P, ShadowReq& sr) {
    const uint32_t obj = S.tri_obj[h.prim];
    const Frame f = hit_frame(S, h.prim, h.u, h.v, P.d);
    const sc_material m = S.mat[obj];
    const float rho = albedo(S, m, f.P, P.lam);
    const float T = P.T * medium_weight(S, P.med, P.lam, h.t);
    P.flags = P.flags | 1u;
    const F3 os = offset_ray(f.P, f.Nf);
    sr.shoot = false;
    // caustic gather: the general photon map on every diffuse surface, else
    // the receiver map cell under the point
    if (pm.on) {
        const uint32_t b = wl.mode == SC_WL_FIXED ? slot : spectral_bin(wl, P.lam);
        const float E = pmap_gather(pm, f.P, f.Nf, b);
        const float g = ((T * rho) * kInvPi) * E;
        P.L = P.L + g;
    } else if (cmap && S.recv_obj && obj == S.recv_obj) {
        const int64_t cell = receiver_cell(S, f.P);
        if (cell >= 0) {
            const uint32_t b = wl.mode == SC_WL_FIXED ? slot : spectral_bin(wl, P.lam);
            const float E = cmap[(size_t)cell * wl.channels + b] * S.inv_cell_area;
            const float g = ((T * rho) * kInvPi) * E;
            P.L = P.L + g;
        }
    }
    // next event estimation
    if (S.n_entries > 0) {
        const U4 r = rng_camera(seed, pix, sample, depth, 2, slot);
        const uint32_t e = pick_entry(S.n_entries, unit(r.c));
        if (e < S.n_pl) {
            const float* lp = S.pl + 4 * (size_t)e;
            const F3 w = F3{lp[0], lp[1], lp[2]} - os;
            const float r2 = dot(w, w);
            const float dist = sqrtf(r2);
            const F3 om = w * (1.0f / dist);
            const float cosx = dot(f.Nf, om);
            if (cosx > 0.0f) {
                float contrib = ((((T * rho) * kInvPi) * lp[3]) * cosx) / r2;
                contrib = contrib * (float)S.n_entries;
                contrib = contrib * medium_weight(S, P.med, P.lam, dist);
                sr = ShadowReq{os, om, dist, contrib, 0xffffffffu, true};
            }
        } else {
            const uint32_t k = cdf_first_above(S.emit_cdf, S.n_emit, unit(r.d));
            const uint32_t lprim = S.emit_prim[k];
            F3 Nl;
            const F3 y = light_point(S, lprim, unit(r.a), unit(r.b), Nl);
            const F3 w = y - os;
            const float r2 = dot(w, w);
            const float dist = sqrtf(r2);
            const F3 om = w * (1.0f / dist);
            const float cosx = dot(f.Nf, om);
            const float cosl = -dot(Nl, om);
            if (cosx > 0.0f && cosl > 0.0f) {
                const float le = S.mat[S.tri_obj[lprim]].le;
                float contrib = ((((((T * rho) * kInvPi) * le) * cosx) * cosl) / r2) * S.a_tot;
                contrib = contrib * (float)S.n_entries;
                contrib = contrib * medium_weight(S, P.med, P.lam, dist);
                sr = ShadowReq{os, om, dist * 0.9999f, contrib, lprim, true};
            }
        }
    }
    // cosine-weighted bounce
    if (depth < max_depth) {
        const U4 r = rng_camera(seed, pix, sample, depth, 1, slot);
        const float u0 = unit(r.a), u1 = unit(r.b);
        const float rr = sqrtf(u0);
        float sp, cp;
        sincos_turn(u1, sp, cp);
        const float x = rr * cp, y = rr * sp;
        const float z = sqrtf(fmaxf(0.0f, 1.0f - u0));
        F3 t1, t2;
        basis(f.Nf, t1, t2);
        P.d = normalize((t1 * x + t2 * y) + f.Nf * z);
        P.o = os;
        P.T = T * rho;
        return true;
    }
    return false;
}

// film: samples added in sample order (then slot order)
__device__ __forceinline__ void film_add(const WaveDev& wl, uint32_t K, uint32_t slot, float L, float lam, float* acc) {
    if (wl.mode == SC_WL_FIXED) {
        if (K == 3) {
            acc[slot] = acc[slot] + L;
        } else {
            acc[0] = acc[0] + L; acc[1] = acc[1] + L; acc[2] = acc[2] + L;
        }
    } else {
        acc[0] = acc[0] + sensor(wl, 0, lam) * L;
        acc[1] = acc[1] + sensor(wl, 1, lam) * L;
        acc[2] = acc[2] + sensor(wl, 2, lam) * L;
    }
}

// ground truth of the pixel-centre ray
__device__ __forceinline__ void aov_write(const DevScene& S, const sc_camera& cam, uint32_t pix, F3 d, const HitRec& h,
                                          const sc_aov& out) {
    const F3 Rh = normalize(F3{cam.right[0], cam.right[1], cam.right[2]});
    const F3 Uh = normalize(F3{cam.up[0], cam.up[1], cam.up[2]});
    const F3 Fh = normalize(F3{cam.fwd[0], cam.fwd[1], cam.fwd[2]});
    uint32_t obj = 0;
    float dep = INFINITY, depn = 1.0f, alb = 0.0f;
    F3 N{0.0f, 0.0f, 0.0f}, Nc{0.0f, 0.0f, 0.0f};
    uint8_t trans = 0;
    if (h.prim != 0xffffffffu) {
        obj = S.tri_obj[h.prim];
        const sc_material m = S.mat[obj];
        const Frame f = hit_frame(S, h.prim, h.u, h.v, d);
        dep = h.t;
        depn = fminf(h.t / 10.0f, 1.0f);
        N = f.Ns;
        Nc = F3{dot(N, Rh), dot(N, Uh), -dot(N, Fh)};
        alb = m.type == SC_MAT_DIFFUSE ? albedo_grey(S, m, f.P) : (m.type == SC_MAT_DIELECTRIC ? 1.0f : 0.0f);
        trans = m.type == SC_MAT_DIELECTRIC ? 1 : 0;
    }
    if (out.obj) out.obj[pix] = obj;
    if (out.trans) out.trans[pix] = trans;
    if (out.tri) out.tri[pix] = h.prim;
    if (out.depth) out.depth[pix] = dep;
    if (out.depthn) out.depthn[pix] = depn;
    if (out.normal) store3(out.normal, pix, N);
    if (out.normal_cam) store3(out.normal_cam, pix, Nc);
    if (out.albedo) out.albedo[pix] = alb;
}

// ---------------------------------------------------------------- photons
struct PhotonPath {
    F3 o, d;
    float phi, lam;
    uint32_t slot, spec;
    uint64_t med;     // media set (lights are in air)
};

// 1 - cos(theta) of the cone subtended by a sphere of squared radius rr at
// squared distance dist2, without cancellation
__device__ __forceinline__ float cap_height(float rr, float dist2) {
    const float q = rr / dist2;
    return q >= 1.0f ? 2.0f : q / (1.0f + sqrtf(1.0f - q));
}

// Photon p of a pass of n_total: light point, cone towards a target sphere
// picked by solid angle, direction uniform in the cone, flux = light power
// x total solid angle x light entries / (photons in its slot x cones that
// contain the direction).  False if the photon leaves an area light's back.
__device__ __forceinline__ bool photon_emit(const DevScene& S, const WaveDev& wl, uint64_t seed, uint64_t n_total,
                                            uint64_t p, PhotonPath& ph) {
    const U4 r0 = rng_photon(seed, p, 0, 0);
    uint32_t slot;
    float lam, nslot;
    if (wl.mode == SC_WL_FIXED) {
        slot = (uint32_t)(p % wl.k);
        lam = wl.nm[slot];
        const uint64_t cnt = n_total / wl.k + ((p % wl.k) < (n_total % wl.k) ? 1u : 0u);
        nslot = (float)cnt;
    } else {
        lam = lambda_from(wl, unit(r0.d));
        slot = spectral_bin(wl, lam);
        nslot = (float)n_total / (float)wl.bins;
    }
    const U4 r2 = rng_photon(seed, p, 0, 2);
    const uint32_t e = pick_entry(S.n_entries, unit(r2.c));
    F3 y, Nl{0.0f, 0.0f, 0.0f};
    float power;
    bool area = false;
    if (e < S.n_pl) {
        const float* lp = S.pl + 4 * (size_t)e;
        y = F3{lp[0], lp[1], lp[2]};
        power = lp[3];
    } else {
        const uint32_t k = cdf_first_above(S.emit_cdf, S.n_emit, unit(r2.d));
        const uint32_t lprim = S.emit_prim[k];
        y = light_point(S, lprim, unit(r2.a), unit(r2.b), Nl);
        power = S.mat[S.tri_obj[lprim]].le * S.a_tot;
        area = true;
    }
    float osum = 0.0f;
    for (uint32_t k = 0; k < S.n_tg; ++k) {
        const float* sp = S.tg + 4 * (size_t)k;
        const F3 dk = F3{sp[0], sp[1], sp[2]} - y;
        osum = osum + kTwoPi * cap_height(sp[3] * sp[3], dot(dk, dk));
    }
    const float target = unit(r0.a) * osum;
    uint32_t kk = S.n_tg - 1;
    float cum = 0.0f;
    for (uint32_t k = 0; k < S.n_tg; ++k) {
        const float* sp = S.tg + 4 * (size_t)k;
        const F3 dk = F3{sp[0], sp[1], sp[2]} - y;
        cum = cum + kTwoPi * cap_height(sp[3] * sp[3], dot(dk, dk));
        if (cum > target) {
            kk = k;
            break;
        }
    }
    const float* spk = S.tg + 4 * (size_t)kk;
    const F3 dkk = F3{spk[0], spk[1], spk[2]} - y;
    const float d2k = dot(dkk, dkk);
    const float hk = cap_height(spk[3] * spk[3], d2k);
    const F3 axis = dkk * (1.0f / sqrtf(d2k));
    const float g = unit(r0.b) * hk;
    const float cost = 1.0f - g;
    const float sint = sqrtf(fmaxf(0.0f, g * (2.0f - g)));
    float sp_, cp_;
    sincos_turn(unit(r0.c), sp_, cp_);
    F3 t1, t2;
    basis(axis, t1, t2);
    const F3 om = normalize((t1 * (cp_ * sint) + t2 * (sp_ * sint)) + axis * cost);
    uint32_t m = 1;
    for (uint32_t k = 0; k < S.n_tg; ++k) {
        if (k == kk) continue;
        const float* sp = S.tg + 4 * (size_t)k;
        const F3 dk = F3{sp[0], sp[1], sp[2]} - y;
        const float dist2 = dot(dk, dk);
        const float q = (sp[3] * sp[3]) / dist2;
        const F3 ax = dk * (1.0f / sqrtf(dist2));
        const F3 cr = cross(om, ax);
        if (q >= 1.0f || (dot(om, ax) > 0.0f && dot(cr, cr) <= q)) ++m;
    }
    bool alive = true;
    if (area) {
        const float cy = dot(Nl, om);
        if (!(cy > 0.0f)) alive = false;
        ph.phi = (((power * cy) * osum) * (float)S.n_entries) / (nslot * (float)m);
        ph.o = offset_ray(y, Nl);
    } else {
        ph.phi = ((power * osum) * (float)S.n_entries) / (nslot * (float)m);
        ph.o = y;
    }
    ph.d = om;
    ph.lam = lam;
    ph.slot = slot;
    ph.spec = 0u;
    ph.med = 0ull;
    return alive;
}

// A deposit: receiver-map index (cell * channels + channel), or for the
// general map the channel with the point and the geometric normal on the
// photon's side; cell_ch = -1 for none.
struct Deposit {
    int64_t cell_ch;
    F3 P, N;
};

// One photon interaction.  Returns true if the photon continues; sets
// outcome (SC_PH_*) when it ends, and dp.cell_ch >= 0 for a deposit (on the
// receiver, or with `general` on any diffuse surface).
__device__ __forceinline__ bool photon_event(const DevScene& S, const WaveDev& wl, uint64_t seed, uint64_t p,
                                             uint32_t depth, uint32_t max_depth, bool general, const HitRec& h,
                                             PhotonPath& ph, int& outcome, Deposit& dp) {
    dp.cell_ch = -1;
    if (h.prim == 0xffffffffu) {
        outcome = SC_PH_ESCAPED;
        return false;
    }
    ph.phi = ph.phi * medium_weight(S, ph.med, ph.lam, h.t);
    const uint32_t obj = S.tri_obj[h.prim];
    const sc_material m = S.mat[obj];
    const Frame f = hit_frame(S, h.prim, h.u, h.v, ph.d);
    if (m.type == SC_MAT_EMISSIVE) {
        outcome = SC_PH_ABSORBED;
        return false;
    }
    if (m.type == SC_MAT_DIELECTRIC) {
        const Crossing c = media_cross(S, ph.med, obj, f.entering, ph.lam);
        if (!c.real) {
            ph.med = c.after;
            ph.o = offset_ray(f.P, neg(f.Nf));
            if (depth < max_depth) return true;
            outcome = SC_PH_TRUNCATED;
            return false;
        }
        const U4 r = rng_photon(seed, p, depth, 1);
        F3 nd;
        bool refl;
        if (m.roughness > 0.0f) {
            float w;
            if (!rough_dielectric(f, ph.d, c.n1, c.n2, m.roughness, unit(r.a), unit(r.b), unit(r.c), nd, refl, w)) {
                outcome = SC_PH_LOST;
                return false;
            }
            ph.phi = ph.phi * w;
        } else if (!dielectric(f, ph.d, c.n1, c.n2, unit(r.c), nd, refl)) {
            outcome = SC_PH_LOST;
            return false;
        }
        if (!refl) ph.med = c.after;
        ph.o = offset_ray(f.P, refl ? f.Nf : neg(f.Nf));
        ph.d = nd;
        ph.spec = ph.spec + 1u;
        if (depth < max_depth) return true;
        outcome = SC_PH_TRUNCATED;
        return false;
    }
    if (ph.spec == 0u) {
        outcome = SC_PH_DIRECT;
    } else if (general) {
        outcome = SC_PH_DEPOSITED;
        dp.cell_ch = (int64_t)ph.slot;
        dp.P = f.P;
        dp.N = f.Nf;
    } else if (obj != S.recv_obj) {
        outcome = SC_PH_ELSEWHERE;
    } else {
        const int64_t cell = receiver_cell(S, f.P);
        if (cell < 0) {
            outcome = SC_PH_OUTSIDE;
        } else {
            outcome = SC_PH_DEPOSITED;
            dp.cell_ch = cell * (int64_t)wl.channels + (int64_t)ph.slot;
        }
    }
    return false;
}

// ---------------------------------------------------------------- whole paths
// A camera path from its current ray at surface hit depth0 to its end, one
// bounce after another in the same order as the staged kernels (closest
// hit; emission, dielectric event, or diffuse event with its shadow ray
// and caustic gather): P.L is final on return.  n_closest and n_shadow
// count the rays traced.
template <int BS, bool COUNT>
__device__ __forceinline__ void camera_continue(const DevScene& S, const WaveDev& wl, const float* cmap,
                                                const PMapDev& pm, uint64_t seed, uint32_t pix, uint32_t sample,
                                                uint32_t slot, uint32_t depth0, uint32_t max_depth, CamPath& P,
                                                uint2 (*lds)[BS], Spill& st, VisitCount& vc, uint32_t& n_closest,
                                                uint32_t& n_shadow) {
    for (uint32_t depth = depth0; depth <= max_depth; ++depth) {
        const HitRec h = trace_closest<BS, COUNT>(S, P.o, P.d, lds, st, vc);
        ++n_closest;
        if (h.prim == 0xffffffffu) break;
        const uint32_t type = S.mat[S.tri_obj[h.prim]].type;
        if (type == SC_MAT_EMISSIVE) {
            camera_emission(S, h, P);
            break;
        }
        if (type == SC_MAT_DIELECTRIC) {
            if (!camera_dielectric(S, seed, pix, sample, slot, depth, max_depth, h, P)) break;
            continue;
        }
        ShadowReq sr;
        const bool cont = camera_diffuse(S, wl, cmap, pm, seed, pix, sample, slot, depth, max_depth, h, P, sr);
        if (sr.shoot) {
            ++n_shadow;
            if (!trace_any<BS>(S, sr.o, sr.d, sr.tmax, sr.excl, lds, st)) P.L = P.L + sr.contrib;
        }
        if (!cont) break;
    }
}

// A photon from its current ray at surface hit depth0 to its end; every
// deposit is handed to dep(deposit, photon).  Returns the outcome of the
// last event; n_closest counts the rays traced.
template <int BS, class Dep>
__device__ __forceinline__ int photon_continue(const DevScene& S, const WaveDev& wl, uint64_t seed, uint64_t p,
                                               uint32_t depth0, uint32_t max_depth, bool general, PhotonPath& ph,
                                               uint2 (*lds)[BS], Spill& st, VisitCount& vc, uint32_t& n_closest,
                                               Dep dep) {
    for (uint32_t depth = depth0; depth <= max_depth; ++depth) {
        const HitRec h = trace_closest<BS, false>(S, ph.o, ph.d, lds, st, vc);
        ++n_closest;
        int outcome = -1;
        Deposit dp;
        const bool cont = photon_event(S, wl, seed, p, depth, max_depth, general, h, ph, outcome, dp);
        if (dp.cell_ch >= 0) dep(dp, ph);
        if (!cont) return outcome;
    }
    return -1;
}

}  // namespace scd
