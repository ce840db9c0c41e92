// sc_device.h -- device-side numerics of the rendering path (gfx950).
//
// Every float expression here is a single IEEE binary32 operation per
// operator, evaluated in the written order: the library is compiled with
// -ffp-contract=off (and the pragma below), division and square root are
// correctly rounded (HIP's default), denormals are kept.  That makes each
// traced path a deterministic function of its inputs and seeds.
#pragma once
#pragma clang fp contract(off)

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "sc_types.h"

namespace scd {

struct F3 {
    float x, y, z;
};

__device__ __forceinline__ F3 f3(float x, float y, float z) { return F3{x, y, z}; }
__device__ __forceinline__ F3 operator+(F3 a, F3 b) { return F3{a.x + b.x, a.y + b.y, a.z + b.z}; }
__device__ __forceinline__ F3 operator-(F3 a, F3 b) { return F3{a.x - b.x, a.y - b.y, a.z - b.z}; }
__device__ __forceinline__ F3 operator*(F3 a, float s) { return F3{a.x * s, a.y * s, a.z * s}; }
__device__ __forceinline__ F3 neg(F3 a) { return F3{-a.x, -a.y, -a.z}; }
__device__ __forceinline__ float dot(F3 a, F3 b) { return (a.x * b.x + a.y * b.y) + a.z * b.z; }
__device__ __forceinline__ F3 cross(F3 a, F3 b) {
    return F3{a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x};
}
__device__ __forceinline__ F3 normalize(F3 a) {
    float inv = 1.0f / sqrtf(dot(a, a));
    return a * inv;
}
__device__ __forceinline__ F3 load3(const float* p, uint32_t i) {
    const float* q = p + 3 * (size_t)i;
    return F3{q[0], q[1], q[2]};
}
__device__ __forceinline__ void store3(float* p, uint32_t i, F3 v) {
    float* q = p + 3 * (size_t)i;
    q[0] = v.x; q[1] = v.y; q[2] = v.z;
}

constexpr float kInvPi = 0.31830988618379067154f;
constexpr float kTwoPi = 6.28318530717958647692f;

// ---------------------------------------------------------------- Philox4x32-10
// Salmon et al. (SC'11): ten rounds of two 32x32->64 multiplies per round,
// halves swapped and xored with the key, key bumped by the Weyl constants.
struct U4 {
    uint32_t a, b, c, d;
};

__device__ __forceinline__ U4 philox(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3, uint32_t k0, uint32_t k1) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        if (r) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        const uint32_t lo0 = 0xD2511F53u * c0, hi0 = __umulhi(0xD2511F53u, c0);
        const uint32_t lo1 = 0xCD9E8D57u * c2, hi1 = __umulhi(0xCD9E8D57u, c2);
        const uint32_t n0 = hi1 ^ c1 ^ k0;
        const uint32_t n2 = hi0 ^ c3 ^ k1;
        c0 = n0; c1 = lo1; c2 = n2; c3 = lo0;
    }
    return U4{c0, c1, c2, c3};
}

// top 24 bits to [0, 1 - 2^-24]
__device__ __forceinline__ float unit(uint32_t x) { return (float)(x >> 8) * 5.9604644775390625e-08f; }

// camera stream: (pixel, sample, depth<<4|purpose, slot<<8|0)
__device__ __forceinline__ U4 rng_camera(uint64_t seed, uint32_t pix, uint32_t sample, uint32_t depth,
                                         uint32_t purpose, uint32_t slot) {
    return philox(pix, sample, (depth << 4) | purpose, slot << 8, (uint32_t)seed, (uint32_t)(seed >> 32));
}
// photon stream: (p lo, p hi, depth<<4|purpose, 1)
__device__ __forceinline__ U4 rng_photon(uint64_t seed, uint64_t p, uint32_t depth, uint32_t purpose) {
    return philox((uint32_t)p, (uint32_t)(p >> 32), (depth << 4) | purpose, 1u, (uint32_t)seed,
                  (uint32_t)(seed >> 32));
}

// ---------------------------------------------------------------- sin/cos of 2 pi u
// Quarter-turn reduction (exact), then Taylor polynomials of sin and cos of
// f*pi/2 for f in [0,1): odd powers to 13, even powers to 14; coefficients
// formed in double at compile time and rounded once to float.
struct TaylorCoeffs {
    float s[7];
    float c[8];
};
constexpr TaylorCoeffs make_taylor() {
    TaylorCoeffs t{};
    const double h = 1.57079632679489661923;
    double p = h, fact = 1.0;
    for (int i = 0; i < 7; ++i) {
        const int n = 2 * i + 1;
        if (i > 0) {
            p = p * h * h;
            fact = fact * (double)(n - 1) * (double)n;
        }
        const double v = p / fact;
        t.s[i] = (float)((i & 1) ? -v : v);
    }
    p = 1.0;
    fact = 1.0;
    for (int i = 0; i < 8; ++i) {
        const int n = 2 * i;
        if (i > 0) {
            p = p * h * h;
            fact = fact * (double)(n - 1) * (double)n;
        }
        const double v = p / fact;
        t.c[i] = (float)((i & 1) ? -v : v);
    }
    return t;
}
constexpr TaylorCoeffs kTaylor = make_taylor();

__device__ __forceinline__ void sincos_turn(float u, float& s, float& c) {
    const float u4 = u * 4.0f;
    const float qf = floorf(u4);
    const int q = ((int)qf) & 3;
    const float f = u4 - qf;
    const float f2 = f * f;
    float ps = kTaylor.s[6];
#pragma unroll
    for (int i = 5; i >= 0; --i) ps = kTaylor.s[i] + f2 * ps;
    ps = f * ps;
    float pc = kTaylor.c[7];
#pragma unroll
    for (int i = 6; i >= 0; --i) pc = kTaylor.c[i] + f2 * pc;
    if (q == 0) { s = ps; c = pc; }
    else if (q == 1) { s = pc; c = -ps; }
    else if (q == 2) { s = -ps; c = -pc; }
    else { s = -pc; c = ps; }
}

// ---------------------------------------------------------------- camera
__device__ __forceinline__ void camera_ray(const sc_camera& cam, uint32_t x, uint32_t y, float jx, float jy, F3& o,
                                           F3& d) {
    const float px = (float)x + jx;
    const float py = (float)y + jy;
    const float sx = (px + px) / (float)cam.w - 1.0f;
    const float sy = 1.0f - (py + py) / (float)cam.h;
    F3 dd;
    dd.x = (cam.fwd[0] + sx * cam.right[0]) + sy * cam.up[0];
    dd.y = (cam.fwd[1] + sx * cam.right[1]) + sy * cam.up[1];
    dd.z = (cam.fwd[2] + sx * cam.right[2]) + sy * cam.up[2];
    d = normalize(dd);
    o = F3{cam.eye[0], cam.eye[1], cam.eye[2]};
}

// ---------------------------------------------------------------- watertight triangle test
// Woop, Benthin, Wald (JCGT 2013): permute so the dominant direction axis is
// z, shear the triangle into ray space, decide with the three 2D edge
// functions (inclusive), recompute exact zeros in double.
struct RayPre {
    F3 o;         // origin permuted to (kx, ky, kz)
    float sx, sy, sz;
    int kx, ky, kz;
};

__device__ __forceinline__ float pick(F3 v, int k) { return k == 0 ? v.x : (k == 1 ? v.y : v.z); }

__device__ __forceinline__ RayPre ray_prepare(F3 o, F3 d) {
    RayPre r;
    const float ax = fabsf(d.x), ay = fabsf(d.y), az = fabsf(d.z);
    int kz = 0;
    float m = ax;
    if (ay > m) { kz = 1; m = ay; }
    if (az > m) { kz = 2; }
    int kx = kz + 1;
    if (kx == 3) kx = 0;
    int ky = kx + 1;
    if (ky == 3) ky = 0;
    const float dz = pick(d, kz);
    if (dz < 0.0f) {
        const int t = kx;
        kx = ky;
        ky = t;
    }
    r.kx = kx; r.ky = ky; r.kz = kz;
    r.sx = pick(d, kx) / dz;
    r.sy = pick(d, ky) / dz;
    r.sz = 1.0f / dz;
    r.o = F3{pick(o, kx), pick(o, ky), pick(o, kz)};
    return r;
}

__device__ __forceinline__ F3 permute(const RayPre& r, F3 p) { return F3{pick(p, r.kx), pick(p, r.ky), pick(p, r.kz)}; }

// Vertices already permuted into the ray's (kx, ky, kz) order.  On a hit
// with t > 0 returns true with t and the edge weights (U, V, W, det) so that
// barycentrics can be formed only for accepted hits.
struct TriHit {
    float t, V, W, rcp;
};

__device__ __forceinline__ bool tri_test(const RayPre& r, F3 p0, F3 p1, F3 p2, TriHit& h) {
    const F3 A = p0 - r.o, B = p1 - r.o, C = p2 - r.o;
    const float Ax = A.x - r.sx * A.z;
    const float Ay = A.y - r.sy * A.z;
    const float Bx = B.x - r.sx * B.z;
    const float By = B.y - r.sy * B.z;
    const float Cx = C.x - r.sx * C.z;
    const float Cy = C.y - r.sy * C.z;
    float U = Cx * By - Cy * Bx;
    float V = Ax * Cy - Ay * Cx;
    float W = Bx * Ay - By * Ax;
    if (U == 0.0f || V == 0.0f || W == 0.0f) {
        const double CxBy = (double)Cx * (double)By, CyBx = (double)Cy * (double)Bx;
        const double AxCy = (double)Ax * (double)Cy, AyCx = (double)Ay * (double)Cx;
        const double BxAy = (double)Bx * (double)Ay, ByAx = (double)By * (double)Ax;
        U = (float)(CxBy - CyBx);
        V = (float)(AxCy - AyCx);
        W = (float)(BxAy - ByAx);
    }
    if ((U < 0.0f || V < 0.0f || W < 0.0f) && (U > 0.0f || V > 0.0f || W > 0.0f)) return false;
    const float det = (U + V) + W;
    if (det == 0.0f) return false;
    const float Az = r.sz * A.z, Bz = r.sz * B.z, Cz = r.sz * C.z;
    const float T = (U * Az + V * Bz) + W * Cz;
    const float rcp = 1.0f / det;
    const float t = T * rcp;
    if (!(t > 0.0f)) return false;
    h.t = t; h.V = V; h.W = W; h.rcp = rcp;
    return true;
}

// ---------------------------------------------------------------- hit frame
struct Frame {
    F3 P, Ng, Nf, Ns;
    bool entering;
};

__device__ __forceinline__ void tri_vertices(const DevScene& S, uint32_t prim, F3& p0, F3& p1, F3& p2) {
    const uint32_t* idx = S.I + 3 * (size_t)prim;
    const uint32_t i0 = idx[0], i1 = idx[1], i2 = idx[2];
    p0 = load3(S.V, i0); p1 = load3(S.V, i1); p2 = load3(S.V, i2);
}

__device__ __forceinline__ Frame hit_frame(const DevScene& S, uint32_t prim, float u, float v, F3 d) {
    Frame f;
    const uint32_t* idx = S.I + 3 * (size_t)prim;
    const uint32_t i0 = idx[0], i1 = idx[1], i2 = idx[2];
    const F3 p0 = load3(S.V, i0), p1 = load3(S.V, i1), p2 = load3(S.V, i2);
    f.Ng = normalize(cross(p1 - p0, p2 - p0));
    const float w = (1.0f - u) - v;
    f.P = (p0 * w + p1 * u) + p2 * v;
    f.entering = dot(d, f.Ng) < 0.0f;
    f.Nf = f.entering ? f.Ng : neg(f.Ng);
    if (S.VN) {
        const F3 n0 = load3(S.VN, i0), n1 = load3(S.VN, i1), n2 = load3(S.VN, i2);
        F3 ns = normalize((n0 * w + n1 * u) + n2 * v);
        if (dot(ns, f.Nf) < 0.0f) ns = neg(ns);
        f.Ns = ns;
    } else {
        f.Ns = f.Nf;
    }
    return f;
}

// Ray origin pushed off the surface (Waechter and Binder, Ray Tracing Gems
// ch. 6): integer ULP steps proportional to the normal, a fixed small step
// near the coordinate origin.
__device__ __forceinline__ float offset1(float p, float n) {
    const int32_t of = (int32_t)(256.0f * n);
    const int32_t pi = __float_as_int(p) + ((p < 0.0f) ? -of : of);
    if (fabsf(p) < 0.03125f) return p + 1.52587890625e-05f * n;
    return __int_as_float(pi);
}
__device__ __forceinline__ F3 offset_ray(F3 p, F3 n) { return F3{offset1(p.x, n.x), offset1(p.y, n.y), offset1(p.z, n.z)}; }

// Orthonormal frame around unit n (Duff et al., JCGT 2017).
__device__ __forceinline__ void basis(F3 n, F3& t1, F3& t2) {
    const float sign = copysignf(1.0f, n.z);
    const float a = -1.0f / (sign + n.z);
    const float b = (n.x * n.y) * a;
    t1 = F3{1.0f + ((sign * n.x) * n.x) * a, sign * b, -(sign * n.x)};
    t2 = F3{b, sign + (n.y * n.y) * a, -n.y};
}

// ---------------------------------------------------------------- smooth dielectric
// Cauchy index, Snell refraction, unpolarised Fresnel, total internal
// reflection; reflect iff u < R.  Falls back to the geometric normal when
// the shading normal gives no valid outgoing side.
__device__ __forceinline__ float fresnel(float n1, float n2, float ci, float ct) {
    const float a1 = n1 * ci, b1 = n2 * ct;
    const float rs = (a1 - b1) / (a1 + b1);
    const float a2 = n1 * ct, b2 = n2 * ci;
    const float rp = (a2 - b2) / (a2 + b2);
    return 0.5f * (rs * rs + rp * rp);
}

// two-term Cauchy law, lambda in nm
__device__ __forceinline__ float cauchy_index(float ca, float cb, float lambda_nm) {
    const float l = lambda_nm * 0.001f;
    return ca + cb / (l * l);
}

// n1: index on the side the ray comes from, n2: index across the surface
__device__ __forceinline__ bool dielectric(const Frame& f, F3 d, float n1, float n2, float uF, F3& out, bool& refl) {
    const float eta = n1 / n2;
    F3 N = f.Ns;
    float ci = -dot(d, N);
    bool geometric = false;
    if (!(ci > 0.0f)) {
        N = f.Nf;
        ci = -dot(d, N);
        geometric = true;
    }
    for (int attempt = 0; attempt < 2; ++attempt) {
        const float e2 = eta * eta;
        const float s2 = 1.0f - ci * ci;
        const float k = 1.0f - e2 * s2;
        bool r;
        float ct = 0.0f;
        if (k <= 0.0f) {
            r = true;
        } else {
            ct = sqrtf(k);
            r = uF < fresnel(n1, n2, ci, ct);
        }
        F3 o;
        if (r) o = d + N * (ci + ci);
        else o = d * eta + N * (eta * ci - ct);
        o = normalize(o);
        const float side = dot(o, f.Nf);
        if (r ? (side > 0.0f) : (side < 0.0f)) {
            out = o;
            refl = r;
            return true;
        }
        if (geometric) return false;
        N = f.Nf;
        ci = -dot(d, N);
        geometric = true;
    }
    return false;
}

// ---------------------------------------------------------------- rough dielectric
// GGX microfacet refraction (Walter, Marschner, Li and Torrance, EGSR 2007)
// with Smith G1(v) = 2 / (1 + sqrt(1 + alpha^2 tan^2 theta_v)), sampled
// from the distribution of visible normals (Heitz, JCGT 7(4), 2018): the
// incoming direction is stretched to the alpha = 1 configuration, a point
// of the projected hemisphere is drawn (r = sqrt(u0), phi = 2 pi u1, the
// second coordinate warped towards the visible half), and its normal is
// stretched back.  Fresnel at m picks reflection (uF < F) or refraction;
// the weight is G1(o) <= 1.  The macro normal is the shading normal on the
// incoming side, else the geometric one.  False when the outgoing
// direction lies on the wrong side of the surface or of m.
__device__ __forceinline__ float smith_g1(float c, float a2) {
    const float c2 = c * c;
    const float t2 = (1.0f - c2) / c2;
    return 2.0f / (1.0f + sqrtf(1.0f + a2 * t2));
}

__device__ __forceinline__ bool rough_dielectric(const Frame& f, F3 d, float n1, float n2, float alpha, float u0,
                                                 float u1, float uF, F3& out, bool& refl, float& w) {
    const float eta = n1 / n2;
    F3 N = f.Ns;
    if (!(-dot(d, N) > 0.0f)) N = f.Nf;
    const float a2 = alpha * alpha;
    F3 t1, t2;
    basis(N, t1, t2);
    const F3 iw = neg(d);
    const F3 vh = normalize(F3{alpha * dot(iw, t1), alpha * dot(iw, t2), dot(iw, N)});
    const float lensq = vh.x * vh.x + vh.y * vh.y;
    const F3 b1 = lensq > 0.0f ? F3{-vh.y, vh.x, 0.0f} * (1.0f / sqrtf(lensq)) : F3{1.0f, 0.0f, 0.0f};
    const F3 b2 = cross(vh, b1);
    const float r = sqrtf(u0);
    float sp, cp;
    sincos_turn(u1, sp, cp);
    const float p1 = r * cp;
    float p2 = r * sp;
    const float h = 0.5f * (1.0f + vh.z);
    p2 = (1.0f - h) * sqrtf(fmaxf(0.0f, 1.0f - p1 * p1)) + h * p2;
    const float p3 = sqrtf(fmaxf(0.0f, (1.0f - p1 * p1) - p2 * p2));
    const F3 nh = (b1 * p1 + b2 * p2) + vh * p3;
    const F3 ne = normalize(F3{alpha * nh.x, alpha * nh.y, fmaxf(0.0f, nh.z)});
    const F3 m = normalize((t1 * ne.x + t2 * ne.y) + N * ne.z);
    const float ci = -dot(d, m);
    if (!(ci > 0.0f)) return false;
    const float k = 1.0f - (eta * eta) * (1.0f - ci * ci);
    float ct = 0.0f;
    if (k <= 0.0f) {
        refl = true;
    } else {
        ct = sqrtf(k);
        refl = uF < fresnel(n1, n2, ci, ct);
    }
    F3 o;
    if (refl) o = d + m * (ci + ci);
    else o = d * eta + m * (eta * ci - ct);
    o = normalize(o);
    const float side = dot(o, f.Nf), on = dot(o, N), om = dot(o, m);
    const bool ok = refl ? (side > 0.0f && on > 0.0f && om > 0.0f) : (side < 0.0f && on < 0.0f && om < 0.0f);
    if (!ok) return false;
    w = smith_g1(fabsf(on), a2);
    out = o;
    return true;
}

// ---------------------------------------------------------------- absorbing glass
// Beer-Lambert: a path segment of length t inside a medium keeps
// exp(-sigma t) of its weight.  sigma is given at 450, 550 and 650 nm and
// taken piecewise linear in lambda between them, constant outside.

// exp(-x) for x >= 0 without libm: Cody-Waite reduction x = k ln2 + r,
// |r| <= ln2/2 (ln2 split into a 16-bit head, exact when multiplied by k,
// and a tail); e^-r from its degree-7 Taylor polynomial (truncation below
// 6e-9 relative); exact scaling by 2^-k, which stays a normal number for
// x <= 87.  1 for x <= 0, 0 for x > 87.
__device__ __forceinline__ float exp_neg(float x) {
    if (!(x > 0.0f)) return 1.0f;
    if (x > 87.0f) return 0.0f;
    const float kf = floorf(x * 1.44269504f + 0.5f);
    const int k = (int)kf;
    const float r = (x - kf * 0.693145751953125f) - kf * 1.428606765330187e-06f;
    const float q = -r;
    float p = (float)(1.0 / 5040.0) + q * (float)(1.0 / 40320.0);
    p = (float)(1.0 / 720.0) + q * p;
    p = (float)(1.0 / 120.0) + q * p;
    p = (float)(1.0 / 24.0) + q * p;
    p = (float)(1.0 / 6.0) + q * p;
    p = 0.5f + q * p;
    p = 1.0f + q * p;
    p = 1.0f + q * p;
    return p * __int_as_float((127 - k) << 23);
}

__device__ __forceinline__ float absorption(const sc_material& m, float lam) {
    if (lam <= 450.0f) return m.sigma[0];
    if (lam >= 650.0f) return m.sigma[2];
    if (lam < 550.0f) return m.sigma[0] + (m.sigma[1] - m.sigma[0]) * ((lam - 450.0f) / 100.0f);
    return m.sigma[1] + (m.sigma[2] - m.sigma[1]) * ((lam - 550.0f) / 100.0f);
}

// ---------------------------------------------------------------- scene lookups
// nearest texel of the texture rectangle under P, edges clamped
__device__ __forceinline__ size_t texel(const DevScene& S, F3 P) {
    const float fx = (P.x - S.tex_x0) * S.tex_sx;
    const float fy = (P.y - S.tex_y0) * S.tex_sy;
    int i = (int)floorf(fx), j = (int)floorf(fy);
    i = i < 0 ? 0 : (i > (int)S.tex_w - 1 ? (int)S.tex_w - 1 : i);
    j = j < 0 ? 0 : (j > (int)S.tex_h - 1 ? (int)S.tex_h - 1 : j);
    return (size_t)j * S.tex_w + (size_t)i;
}

// albedo at P for wavelength lam; an RGB texel is reflectance B at 450 nm,
// G at 550 nm and R at 650 nm, linear in lambda between, constant outside
__device__ __forceinline__ float albedo(const DevScene& S, const sc_material& m, F3 P, float lam) {
    if (m.albedo_mode == SC_ALBEDO_CHECKER) {
        const int ix = (int)floorf(P.x), iy = (int)floorf(P.y);
        return ((ix + iy) & 1) == 0 ? m.rho_a : m.rho_b;
    }
    if (m.albedo_mode == SC_ALBEDO_TEXTURE && S.tex) return S.tex[texel(S, P)];
    if (m.albedo_mode == SC_ALBEDO_TEXTURE_RGB && S.tex_rgb) {
        const float* c = S.tex_rgb + 3 * texel(S, P);
        const float r = c[0], g = c[1], b = c[2];
        if (lam <= 450.0f) return b;
        if (lam >= 650.0f) return r;
        if (lam < 550.0f) return b + (g - b) * ((lam - 450.0f) / 100.0f);
        return g + (r - g) * ((lam - 550.0f) / 100.0f);
    }
    return m.rho_a;
}

// grey albedo of the ground-truth output: the mean of an RGB texel
__device__ __forceinline__ float albedo_grey(const DevScene& S, const sc_material& m, F3 P) {
    if (m.albedo_mode == SC_ALBEDO_TEXTURE_RGB && S.tex_rgb) {
        const float* c = S.tex_rgb + 3 * texel(S, P);
        return ((c[0] + c[1]) + c[2]) / 3.0f;
    }
    return albedo(S, m, P, 550.0f);
}

// receiver cell (floor rule, upper edge clamped); -1 outside the rectangle
__device__ __forceinline__ int64_t receiver_cell(const DevScene& S, F3 P) {
    const float fx = (P.x - S.recv_x0) * S.cell_sx;
    const float fy = (P.y - S.recv_y0) * S.cell_sy;
    if (!(fx >= 0.0f) || !(fy >= 0.0f) || fx > (float)S.recv_wc || fy > (float)S.recv_hc) return -1;
    uint32_t i = (uint32_t)fx, j = (uint32_t)fy;
    if (i >= S.recv_wc) i = S.recv_wc - 1;
    if (j >= S.recv_hc) j = S.recv_hc - 1;
    return (int64_t)j * S.recv_wc + i;
}

__device__ __forceinline__ uint32_t spectral_bin(const WaveDev& wl, float lam) {
    const float f = (lam - wl.lo) * wl.bin_scale;
    int b = (int)f;
    b = b < 0 ? 0 : (b > (int)wl.bins - 1 ? (int)wl.bins - 1 : b);
    return (uint32_t)b;
}
__device__ __forceinline__ float lambda_from(const WaveDev& wl, float u) { return wl.lo + u * (wl.hi - wl.lo); }

__device__ __forceinline__ uint32_t cdf_first_above(const float* cdf, uint32_t n, float u) {
    // smallest i with cdf[i] > u (cdf non-decreasing, cdf[n-1] = 1)
    uint32_t lo = 0, hi = n - 1;
    while (lo < hi) {
        const uint32_t mid = (lo + hi) >> 1;
        if (cdf[mid] > u) hi = mid;
        else lo = mid + 1;
    }
    return lo;
}

__device__ __forceinline__ uint32_t pick_entry(uint32_t n, float u) {
    if (n <= 1) return 0;
    uint32_t e = (uint32_t)(u * (float)n);
    return e > n - 1 ? n - 1 : e;
}

// uniform point on an emitting triangle and its unit geometric normal
__device__ __forceinline__ F3 light_point(const DevScene& S, uint32_t prim, float u0, float u1, F3& Nl) {
    F3 p0, p1, p2;
    tri_vertices(S, prim, p0, p1, p2);
    const float su = sqrtf(u0);
    const float b0 = 1.0f - su;
    const float b1 = su * (1.0f - u1);
    const float b2 = su * u1;
    Nl = normalize(cross(p1 - p0, p2 - p0));
    return (p0 * b0 + p1 * b1) + p2 * b2;
}

__device__ __forceinline__ float sensor(const WaveDev& wl, int c, float lam) {
    const float f = (lam - wl.lo) * 4.0f;
    int i = (int)f;
    i = i < 0 ? 0 : (i > (int)wl.n_tab - 2 ? (int)wl.n_tab - 2 : i);
    const float fr = f - (float)i;
    const float* tab = wl.tab + (size_t)c * wl.n_tab;
    const float a = tab[i], b = tab[i + 1];
    return a + fr * (b - a);
}

}  // namespace scd
