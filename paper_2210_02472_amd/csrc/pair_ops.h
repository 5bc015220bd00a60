// Pair operations shared by the single-set kernels (pairs.hip) and the batched persistent
// kernel (batch.hip): per-pair arithmetic of the acceleration, force-gradient and time-step passes
// in mixed and FP64 precision, the FP64 re-evaluation of close-pair tiles, and the tile sweep.
//
// Mixed precision, as used here: every difference of FP64 master quantities (positions,
// velocities, accelerations) is taken in FP64 and rounded once to FP32; all arithmetic after
// that (s^2, rsqrt, mass products, the pair term) is FP32; each LDS tile is summed in FP32
// and merged into FP64 accumulators.  The acceleration and gradient passes also accumulate a
// magnitude estimate M of sum_j |term_j| (the pair weight times the max-norm of the pair's
// difference vector: r for the acceleration, a_ji for the gradient); a target whose result is
// small against M (cancellation) is re-evaluated entirely in FP64 afterwards.
#pragma once

#include "bf_internal.h"

namespace bf {

// ---- helpers -------------------------------------------------------------------------------

__device__ __forceinline__ int32_t particle_of(const DevSet& s, int32_t k, int64_t n, uint32_t* flags) {
    if (s.idx == nullptr) return s.begin + k;  // ranges are validated on the host
    int32_t p = s.idx[k];
    if (p < 0 || p >= n) {
        atomicOr(flags, BF_FLAG_BADINDEX);
        p = 0;
    }
    return p;
}

// 1/sqrt(r2) in FP64: the hardware estimate (about 24 correct bits) refined by one
// third-order step of y (1 - e)^(-1/2) = y (1 + e/2 + 3e^2/8 + ...), e = 1 - r2 y^2.
__device__ __forceinline__ double rsqrt64(double r2) {
    const double y = __builtin_amdgcn_rsq(r2);
    const double h = r2 * y;
    const double e = __builtin_fma(-h, y, 1.0);
    const double t = __builtin_fma(e, 0.375, 0.5);
    return __builtin_fma(y * e, t, y);
}

__device__ __forceinline__ float rsqrt32(float r2) { return __builtin_amdgcn_rsqf(r2); }

// pairs inside one subsystem (equal labels) are left out of every pair sum (Alg. 1: the
// accelerations ignore intra-subsystem contributions)
__device__ __forceinline__ bool same_sub(const int32_t* sub, int pi, int pj) { return sub != nullptr && sub[pi] == sub[pj]; }

__device__ __forceinline__ float dif32(double a, double b) { return (float)(a - b); }
__device__ __forceinline__ float max3abs(float a, float b, float c) {
    return __builtin_fmaxf(__builtin_fabsf(a), __builtin_fmaxf(__builtin_fabsf(b), __builtin_fabsf(c)));
}

// G m stored as FP32 in the low half of the fourth FP64 slot of a packed position
__device__ __forceinline__ double pack_gm(float gm) { return __builtin_bit_cast(double, make_float2(gm, 0.f)); }
__device__ __forceinline__ float unpack_gm(double w) { return __builtin_bit_cast(float2, w).x; }

constexpr int kFold = 64;           // sources per FP32 partial before the FP64 merge

// Read-only data whose address is the same for every lane of a wavefront (a source of the
// sorted far stream, tile metadata): read through the constant address space, so that the
// compiler issues scalar loads and the operands arrive in SGPRs, once per wavefront, with no
// LDS staging.  The data must not be written while the kernel runs.
typedef __attribute__((address_space(4))) const float cfloat;
typedef __attribute__((address_space(4))) const double cdouble;
__device__ __forceinline__ float4 load_uniform4(const void* base, int q) {
    const cfloat* f = (const cfloat*)(base) + 4 * (size_t)q;
    return make_float4(f[0], f[1], f[2], f[3]);
}
__device__ __forceinline__ double4 load_uniform4d(const void* base, int q) {
    const cdouble* f = (const cdouble*)(base) + 4 * (size_t)q;
    return make_double4(f[0], f[1], f[2], f[3]);
}
constexpr float kTiny32 = 1e-20f;   // added to s^2 in FP32: keeps the self pair finite (and zero)
constexpr double kTiny64 = 1e-150;  // same in FP64

// FP64 contributions of one pair, straight from the masters (re-evaluation and fix-up paths).
// r = x_j - x_i, s2 = |r|^2 + eps2 > 0.  The target's values come in registers (T64), so a
// loop over sources loads them once.
struct T64 {
    double x, y, z, ax, ay, az;
};
template <bool GRAD>
__device__ __forceinline__ T64 target64(const Masters& P, int pi) {
    T64 t{P.x[pi], P.y[pi], P.z[pi], 0.0, 0.0, 0.0};
    if constexpr (GRAD) { t.ax = P.ax[pi]; t.ay = P.ay[pi]; t.az = P.az[pi]; }
    return t;
}

__device__ __forceinline__ void acc_pair64(const Masters& P, const T64& t, int pj, double G, double eps2, double& sx,
                                           double& sy, double& sz, double& sm, uint32_t* flags) {
    const double dx = P.x[pj] - t.x, dy = P.y[pj] - t.y, dz = P.z[pj] - t.z;
    const double r2 = dx * dx + dy * dy + dz * dz + eps2;
    if (r2 == 0.0) { atomicOr(flags, BF_FLAG_COINCIDENT); return; }
    const double ri = rsqrt64(r2);
    const double w = G * P.m[pj] * ri * ri * ri;
    sx += w * dx; sy += w * dy; sz += w * dz;
    sm += w * fmax(fabs(dx), fmax(fabs(dy), fabs(dz)));
}

__device__ __forceinline__ void grad_pair64(const Masters& P, const T64& t, int pj, double G, double eps2, double& sx,
                                            double& sy, double& sz, double& sm, uint32_t* flags) {
    const double dx = P.x[pj] - t.x, dy = P.y[pj] - t.y, dz = P.z[pj] - t.z;
    const double r2 = dx * dx + dy * dy + dz * dz + eps2;
    if (r2 == 0.0) { atomicOr(flags, BF_FLAG_COINCIDENT); return; }
    const double dax = P.ax[pj] - t.ax, day = P.ay[pj] - t.ay, daz = P.az[pj] - t.az;
    const double ri = rsqrt64(r2);
    const double ri2 = ri * ri;
    const double w = G * P.m[pj] * ri * ri2;
    const double q3 = 3.0 * (dax * dx + day * dy + daz * dz) * ri2;
    sx += w * (dax - q3 * dx); sy += w * (day - q3 * dy); sz += w * (daz - q3 * dz);
    sm += w * fmax(fabs(dax), fmax(fabs(day), fabs(daz)));
}

// ---- operations ----------------------------------------------------------------------------
// Each operation provides: Src (LDS element), Tgt (per-target registers), A32 (per-tile
// partial), A64 (running result), NC result components plus kCond magnitude components, and
// the steps used by the skeleton.

// Newtonian acceleration, mixed precision.  Pack: double4 (x, y, z, [G m as FP32]).
struct AccMixed {
    static constexpr int NC = 3;
    static constexpr bool kMixed = true, kMax = false, kCond = true;
    struct Src { double4 p; };
    struct Tgt { double x, y, z; };
    struct A32 { float x, y, z, m; };
    struct A64 { double x, y, z, m; };
    __device__ static Src load(const PairArgs& a, int q) { return {static_cast<const double4*>(a.pack)[q]}; }
    __device__ static void target(const PairArgs& a, int p, Tgt& t) { t.x = a.P.x[p]; t.y = a.P.y[p]; t.z = a.P.z[p]; }
    __device__ static void zero(A32& r) { r.x = r.y = r.z = r.m = 0.f; }
    __device__ static void zero(A64& r) { r.x = r.y = r.z = r.m = 0.0; }
    __device__ static void exclude(Src& s) { s.p.w = 0.0; }  // zero mass: no term
    __device__ static float pair(A32& r, const Tgt& t, const Src& s, float eps2f) {
        const float dx = dif32(s.p.x, t.x), dy = dif32(s.p.y, t.y), dz = dif32(s.p.z, t.z);
        const float r2 = __builtin_fmaf(dx, dx, __builtin_fmaf(dy, dy, __builtin_fmaf(dz, dz, eps2f)));
        const float ri = rsqrt32(r2);
        const float ri2 = ri * ri;
        const float w = (unpack_gm(s.p.w) * ri) * ri2;
        r.x = __builtin_fmaf(w, dx, r.x);
        r.y = __builtin_fmaf(w, dy, r.y);
        r.z = __builtin_fmaf(w, dz, r.z);
        // the self pair has dx = 0 and adds nothing here (a form without dx would count it)
        r.m = __builtin_fmaf(w, max3abs(dx, dy, dz), r.m);
        return r2;
    }
    __device__ static void fold(A64& o, const A32& i) {
        o.x += (double)i.x; o.y += (double)i.y; o.z += (double)i.z; o.m += (double)i.m;
    }
    __device__ static void redo(A64& o, const PairArgs& a, int pi, int q0, int len) {
        double sx = 0.0, sy = 0.0, sz = 0.0, sm = 0.0;
        const T64 t = target64<false>(a.P, pi);
        for (int q = q0; q < q0 + len; ++q) {
            const int pj = particle_of(a.src, q, a.P.n, a.flags);
            if (pj != pi && !same_sub(a.sub, pi, pj)) acc_pair64(a.P, t, pj, a.G, a.eps2, sx, sy, sz, sm, a.flags);
        }
        o.x += sx; o.y += sy; o.z += sz; o.m += sm;
    }
    __device__ static void comps(const A64& o, double* v) { v[0] = o.x; v[1] = o.y; v[2] = o.z; v[3] = o.m; }
};

// Force-gradient sum, mixed precision.  Pack: double4 (x, y, z, [G m as FP32]) and
// double4 (ax, ay, az, 0).  a_ji = a_j - a_i cancels strongly for near neighbours, whose 1/r^3
// weight dominates the sum, so it is formed in FP64 like the position difference.  Per pair:
// Gsum += w (a_ji - 3 (a_ji . r) r / s^2) with w = G m / s^3, accumulated as two sums
// S1 = sum w a_ji and S2 = sum w (a_ji . r)/s^2 r, Gsum = S1 - 3 S2.
struct GradMixed {
    static constexpr int NC = 3;
    static constexpr bool kMixed = true, kMax = false, kCond = true;
    struct Src { double4 p, a; };
    struct Tgt { double x, y, z, ax, ay, az; };
    struct A32 { float x, y, z, u, v, w, m; };
    struct A64 { double x, y, z, m; };
    __device__ static Src load(const PairArgs& a, int q) {
        const double4* pk = static_cast<const double4*>(a.pack);
        return {pk[2 * q], pk[2 * q + 1]};
    }
    __device__ static void target(const PairArgs& a, int p, Tgt& t) {
        t.x = a.P.x[p]; t.y = a.P.y[p]; t.z = a.P.z[p];
        t.ax = a.P.ax[p]; t.ay = a.P.ay[p]; t.az = a.P.az[p];
    }
    __device__ static void zero(A32& r) { r.x = r.y = r.z = r.u = r.v = r.w = r.m = 0.f; }
    __device__ static void zero(A64& r) { r.x = r.y = r.z = r.m = 0.0; }
    __device__ static void exclude(Src& s) { s.p.w = 0.0; }
    __device__ static float pair(A32& r, const Tgt& t, const Src& s, float eps2f) {
        const float dx = dif32(s.p.x, t.x), dy = dif32(s.p.y, t.y), dz = dif32(s.p.z, t.z);
        const float r2 = __builtin_fmaf(dx, dx, __builtin_fmaf(dy, dy, __builtin_fmaf(dz, dz, eps2f)));
        const float ri = rsqrt32(r2);
        const float ri2 = ri * ri;
        const float dax = dif32(s.a.x, t.ax), day = dif32(s.a.y, t.ay), daz = dif32(s.a.z, t.az);
        const float q = __builtin_fmaf(dax, dx, __builtin_fmaf(day, dy, daz * dz));
        const float w = (unpack_gm(s.p.w) * ri) * ri2;
        const float w5 = (w * q) * ri2;
        r.x = __builtin_fmaf(w, dax, r.x);
        r.y = __builtin_fmaf(w, day, r.y);
        r.z = __builtin_fmaf(w, daz, r.z);
        r.u = __builtin_fmaf(w5, dx, r.u);
        r.v = __builtin_fmaf(w5, dy, r.v);
        r.w = __builtin_fmaf(w5, dz, r.w);
        r.m = __builtin_fmaf(w, max3abs(dax, day, daz), r.m);
        return r2;
    }
    __device__ static void fold(A64& o, const A32& i) {
        o.x += (double)i.x - 3.0 * (double)i.u;
        o.y += (double)i.y - 3.0 * (double)i.v;
        o.z += (double)i.z - 3.0 * (double)i.w;
        o.m += (double)i.m;
    }
    __device__ static void redo(A64& o, const PairArgs& a, int pi, int q0, int len) {
        double sx = 0.0, sy = 0.0, sz = 0.0, sm = 0.0;
        const T64 t = target64<true>(a.P, pi);
        for (int q = q0; q < q0 + len; ++q) {
            const int pj = particle_of(a.src, q, a.P.n, a.flags);
            if (pj != pi && !same_sub(a.sub, pi, pj)) grad_pair64(a.P, t, pj, a.G, a.eps2, sx, sy, sz, sm, a.flags);
        }
        o.x += sx; o.y += sy; o.z += sz; o.m += sm;
    }
    __device__ static void comps(const A64& o, double* v) { v[0] = o.x; v[1] = o.y; v[2] = o.z; v[3] = o.m; }
};

// Time-step maxima, mixed precision.  Pack: double4 (x, y, z, [G m as FP32]) and
// double4 (vx, vy, vz, 0).  Per pair: Wff = max G(m_i + m_j)/r^3, Wfb = max |v_ij|^2/r^2
// (unsoftened); then dt_ff = eta_ff Wff^(-1/2), dt_fb = eta_fb Wfb^(-1/2).  The self pair has
// r^2 = 0 and always sends its tile to the FP64 re-evaluation, which excludes it by index.
struct DtMixed {
    static constexpr int NC = 2;
    static constexpr bool kMixed = true, kMax = true, kCond = false;
    struct Src { double4 p, v; };  // v.w: the source's particle index
    struct Tgt { double x, y, z, vx, vy, vz; float gm; int pi; };
    struct A32 { float ff, fb; };
    struct A64 { double ff, fb; };
    __device__ static Src load(const PairArgs& a, int q) {
        const double4* pk = static_cast<const double4*>(a.pack);
        return {pk[2 * q], pk[2 * q + 1]};
    }
    __device__ static void target(const PairArgs& a, int p, Tgt& t) {
        t.x = a.P.x[p]; t.y = a.P.y[p]; t.z = a.P.z[p];
        t.vx = a.P.vx[p]; t.vy = a.P.vy[p]; t.vz = a.P.vz[p];
        t.gm = (float)(a.G * a.P.m[p]);
        t.pi = p;
    }
    __device__ static void zero(A32& r) { r.ff = r.fb = 0.f; }
    __device__ static void zero(A64& r) { r.ff = r.fb = 0.0; }
    // moved out of reach: s^2 overflows to +inf in FP32, so both maxima get zero
    __device__ static void exclude(Src& s) { s.p.x = 1e150; }
    // The target itself (matched by index) adds nothing and reports an infinite separation, so
    // the close-pair re-evaluation (a threshold of 1e-30 on s^2, which a coincident distinct
    // pair meets) does not fire on it.
    __device__ static float pair(A32& r, const Tgt& t, const Src& s, float /*eps2f*/) {
        const bool self = (int)s.v.w == t.pi;
        const float dx = dif32(s.p.x, t.x), dy = dif32(s.p.y, t.y), dz = dif32(s.p.z, t.z);
        const float r2 = __builtin_fmaf(dx, dx, __builtin_fmaf(dy, dy, dz * dz));
        const float ux = dif32(s.v.x, t.vx), uy = dif32(s.v.y, t.vy), uz = dif32(s.v.z, t.vz);
        const float u2 = __builtin_fmaf(ux, ux, __builtin_fmaf(uy, uy, uz * uz));
        const float ri = rsqrt32(r2);
        const float ri2 = ri * ri;
        r.fb = fmaxf(r.fb, self ? 0.f : u2 * ri2);
        r.ff = fmaxf(r.ff, self ? 0.f : ((unpack_gm(s.p.w) + t.gm) * ri2) * ri);
        return self ? __builtin_huge_valf() : r2;
    }
    __device__ static void fold(A64& o, const A32& i) { o.ff = fmax(o.ff, (double)i.ff); o.fb = fmax(o.fb, (double)i.fb); }
    __device__ static bool beyond(const A32& r) { return !(fmaxf(r.ff, r.fb) < __builtin_huge_valf()); }
    __device__ static void redo(A64& o, const PairArgs& a, int pi, int q0, int len) {
        const double xi = a.P.x[pi], yi = a.P.y[pi], zi = a.P.z[pi];
        const double vxi = a.P.vx[pi], vyi = a.P.vy[pi], vzi = a.P.vz[pi], mi = a.P.m[pi];
        double ff = o.ff, fb = o.fb;
        for (int q = q0; q < q0 + len; ++q) {
            const int pj = particle_of(a.src, q, a.P.n, a.flags);
            if (pj == pi || same_sub(a.sub, pi, pj)) continue;
            const double dx = a.P.x[pj] - xi, dy = a.P.y[pj] - yi, dz = a.P.z[pj] - zi;
            const double r2 = dx * dx + dy * dy + dz * dz;
            if (r2 == 0.0) { atomicOr(a.flags, BF_FLAG_COINCIDENT); continue; }
            const double ux = a.P.vx[pj] - vxi, uy = a.P.vy[pj] - vyi, uz = a.P.vz[pj] - vzi;
            const double ri = rsqrt64(r2);
            fb = fmax(fb, (ux * ux + uy * uy + uz * uz) * ri * ri);
            ff = fmax(ff, a.G * (mi + a.P.m[pj]) * ri * ri * ri);
        }
        o.ff = ff; o.fb = fb;
    }
    __device__ static void comps(const A64& o, double* v) { v[0] = o.ff; v[1] = o.fb; }
};

// FP64 variants.  Packs: double4 (x, y, z, G m) [+ double4 (ax, ay, az, 0) | (vx, vy, vz, j)].
struct Acc64 {
    static constexpr int NC = 3;
    static constexpr bool kMixed = false, kMax = false, kCond = false;
    struct Src { double4 p; };
    struct Tgt { double x, y, z; };
    using A32 = int;  // unused
    struct A64 { double x, y, z; };
    __device__ static Src load(const PairArgs& a, int q) { return {static_cast<const double4*>(a.pack)[q]}; }
    // source q straight from the masters (the one-launch small pass has no pack)
    __device__ static Src load_master(const PairArgs& a, int q) {
        const int p = particle_of(a.src, q, a.P.n, a.flags);
        return {make_double4(a.P.x[p], a.P.y[p], a.P.z[p], a.G * a.P.m[p])};
    }
    __device__ static void target(const PairArgs& a, int p, Tgt& t) { t.x = a.P.x[p]; t.y = a.P.y[p]; t.z = a.P.z[p]; }
    __device__ static void zero(A64& r) { r.x = r.y = r.z = 0.0; }
    __device__ static void pair64(A64& r, const Tgt& t, const Src& s, double eps2t, int /*pi*/) {
        const double dx = s.p.x - t.x, dy = s.p.y - t.y, dz = s.p.z - t.z;
        const double r2 = __builtin_fma(dx, dx, __builtin_fma(dy, dy, __builtin_fma(dz, dz, eps2t)));
        const double ri = rsqrt64(r2);
        const double ri2 = ri * ri;
        const double w = (s.p.w * ri) * ri2;
        r.x = __builtin_fma(w, dx, r.x);
        r.y = __builtin_fma(w, dy, r.y);
        r.z = __builtin_fma(w, dz, r.z);
    }
    __device__ static void comps(const A64& o, double* v) { v[0] = o.x; v[1] = o.y; v[2] = o.z; }
};

struct Grad64 {
    static constexpr int NC = 3;
    static constexpr bool kMixed = false, kMax = false, kCond = false;
    struct Src { double4 p, a; };
    struct Tgt { double x, y, z, ax, ay, az; };
    using A32 = int;
    struct A64 { double x, y, z; };
    __device__ static Src load(const PairArgs& a, int q) {
        const double4* pk = static_cast<const double4*>(a.pack);
        return {pk[2 * q], pk[2 * q + 1]};
    }
    __device__ static Src load_master(const PairArgs& a, int q) {
        const int p = particle_of(a.src, q, a.P.n, a.flags);
        return {make_double4(a.P.x[p], a.P.y[p], a.P.z[p], a.G * a.P.m[p]),
                make_double4(a.P.ax[p], a.P.ay[p], a.P.az[p], 0.0)};
    }
    __device__ static void target(const PairArgs& a, int p, Tgt& t) {
        t.x = a.P.x[p]; t.y = a.P.y[p]; t.z = a.P.z[p];
        t.ax = a.P.ax[p]; t.ay = a.P.ay[p]; t.az = a.P.az[p];
    }
    __device__ static void zero(A64& r) { r.x = r.y = r.z = 0.0; }
    __device__ static void pair64(A64& r, const Tgt& t, const Src& s, double eps2t, int /*pi*/) {
        const double dx = s.p.x - t.x, dy = s.p.y - t.y, dz = s.p.z - t.z;
        const double r2 = __builtin_fma(dx, dx, __builtin_fma(dy, dy, __builtin_fma(dz, dz, eps2t)));
        const double ri = rsqrt64(r2);
        const double ri2 = ri * ri;
        const double dax = s.a.x - t.ax, day = s.a.y - t.ay, daz = s.a.z - t.az;
        const double q = __builtin_fma(dax, dx, __builtin_fma(day, dy, daz * dz));
        const double w = (s.p.w * ri) * ri2;
        const double w5 = (-3.0 * w * q) * ri2;
        r.x = __builtin_fma(w, dax, __builtin_fma(w5, dx, r.x));
        r.y = __builtin_fma(w, day, __builtin_fma(w5, dy, r.y));
        r.z = __builtin_fma(w, daz, __builtin_fma(w5, dz, r.z));
    }
    __device__ static void comps(const A64& o, double* v) { v[0] = o.x; v[1] = o.y; v[2] = o.z; }
};

struct Dt64 {
    static constexpr int NC = 2;
    static constexpr bool kMixed = false, kMax = true, kCond = false;
    struct Src { double4 p, v; };   // v.w = source particle index (exact in FP64)
    struct Tgt { double x, y, z, vx, vy, vz, gm; };
    using A32 = int;
    struct A64 { double ff, fb; };
    __device__ static Src load(const PairArgs& a, int q) {
        const double4* pk = static_cast<const double4*>(a.pack);
        return {pk[2 * q], pk[2 * q + 1]};
    }
    __device__ static void target(const PairArgs& a, int p, Tgt& t) {
        t.x = a.P.x[p]; t.y = a.P.y[p]; t.z = a.P.z[p];
        t.vx = a.P.vx[p]; t.vy = a.P.vy[p]; t.vz = a.P.vz[p];
        t.gm = a.G * a.P.m[p];
    }
    __device__ static void zero(A64& r) { r.ff = r.fb = 0.0; }
    __device__ static void pair64(A64& r, const Tgt& t, const Src& s, double /*eps2t*/, int pi) {
        const double dx = s.p.x - t.x, dy = s.p.y - t.y, dz = s.p.z - t.z;
        double r2 = __builtin_fma(dx, dx, __builtin_fma(dy, dy, __builtin_fma(dz, dz, kTiny64)));
        // the self pair is moved out of reach (its maxima underflow to zero); a coincident
        // distinct pair keeps s^2 = kTiny64 and drives the time-steps to zero
        r2 = ((double)pi == s.v.w) ? 1e300 : r2;
        const double ux = s.v.x - t.vx, uy = s.v.y - t.vy, uz = s.v.z - t.vz;
        const double u2 = __builtin_fma(ux, ux, __builtin_fma(uy, uy, uz * uz));
        const double ri = rsqrt64(r2);
        const double ri2 = ri * ri;
        r.fb = fmax(r.fb, u2 * ri2);
        r.ff = fmax(r.ff, ((s.p.w + t.gm) * ri2) * ri);
    }
    __device__ static void comps(const A64& o, double* v) { v[0] = o.ff; v[1] = o.fb; }
};

// ---- far-tile operations of the spatially sorted mode ----------------------------------------
// Sources of a tile are stored as FP32 offsets from the tile centre c (rounded once from FP64);
// a lane forms its target's offset from the same centre once per tile.  For a pair in a tile
// whose gap to every target of the workgroup is at least kappa times the tile half-extent h,
// the rounding error of dx is at most u (|x_j - c| + |x_i - c|) <= u (r + 2 sqrt(3) h), i.e.
// relative error u (1 + 2 sqrt(3) / kappa): the FP64 differences are only needed for near tiles.

struct AccRel {
    struct Src { float4 p; };             // (x - cx, y - cy, z - cz, G m)
    struct Tgt { float x, y, z; };
    using A32 = AccMixed::A32;
    __device__ static Src load(const PairArgs& a, int q) { return {static_cast<const float4*>(a.pack_far)[q]}; }
    __device__ static Src load_uniform(const PairArgs& a, int q) { return {load_uniform4(a.pack_far, q)}; }
    __device__ static void rel(Tgt& t, const AccMixed::Tgt& g, const double4& c, const double4&) {
        t.x = (float)(g.x - c.x); t.y = (float)(g.y - c.y); t.z = (float)(g.z - c.z);
    }
    // upper bound of sum_j |term_j| over the tile for this target: every source lies in the
    // cube of half-extent h about the centre, so r is at least the target's distance to that
    // cube (positive for a far tile) and |term| = G m r / s^3 <= G m / r^2
    static constexpr bool kTileBound = true, kWeightSum = false;
    __device__ static float factor(const Tgt&, float) { return 1.f; }
    __device__ static float bound(const Tgt& t, float h, float gm_tile, float) {
        const float gx = fmaxf(__builtin_fabsf(t.x) - h, 0.f), gy = fmaxf(__builtin_fabsf(t.y) - h, 0.f),
                    gz = fmaxf(__builtin_fabsf(t.z) - h, 0.f);
        const float r2 = fmaxf(__builtin_fmaf(gx, gx, __builtin_fmaf(gy, gy, gz * gz)), 1e-30f);
        return gm_tile / r2;
    }
    __device__ static void pair(A32& r, const Tgt& t, const Src& s, float eps2f) {
        const float dx = s.p.x - t.x, dy = s.p.y - t.y, dz = s.p.z - t.z;
        const float r2 = __builtin_fmaf(dx, dx, __builtin_fmaf(dy, dy, __builtin_fmaf(dz, dz, eps2f)));
        const float ri = rsqrt32(r2);
        const float ri2 = ri * ri;
        const float w = (s.p.w * ri) * ri2;
        r.x = __builtin_fmaf(w, dx, r.x);
        r.y = __builtin_fmaf(w, dy, r.y);
        r.z = __builtin_fmaf(w, dz, r.z);
    }
};

struct GradRel {
    struct Src { float4 p, a; };          // (x - cx, ..., G m), (ax - acx, ay - acy, az - acz, 0)
    struct Tgt { float x, y, z, ax, ay, az; };
    using A32 = GradMixed::A32;
    __device__ static Src load(const PairArgs& a, int q) {
        const float4* pk = static_cast<const float4*>(a.pack_far);
        return {pk[2 * q], pk[2 * q + 1]};
    }
    __device__ static Src load_uniform(const PairArgs& a, int q) {
        return {load_uniform4(a.pack_far, 2 * q), load_uniform4(a.pack_far, 2 * q + 1)};
    }
    __device__ static void rel(Tgt& t, const GradMixed::Tgt& g, const double4& c, const double4& ca) {
        t.x = (float)(g.x - c.x); t.y = (float)(g.y - c.y); t.z = (float)(g.z - c.z);
        t.ax = (float)(g.ax - ca.x); t.ay = (float)(g.ay - ca.y); t.az = (float)(g.az - ca.z);
    }
    // magnitude estimate per pair, as in the FP64-difference operation: a tile-wide bound (sum
    // of w times h_a + |a_c - a_i|) sent 60 times as many targets of a King W0 = 6 cluster to
    // the FP64 fix-up
    static constexpr bool kTileBound = false, kWeightSum = false;
    __device__ static float bound(const Tgt&, float, float, float) { return 0.f; }
    __device__ static float factor(const Tgt&, float) { return 1.f; }
    __device__ static void pair(A32& r, const Tgt& t, const Src& s, float eps2f) {
        const float dx = s.p.x - t.x, dy = s.p.y - t.y, dz = s.p.z - t.z;
        const float r2 = __builtin_fmaf(dx, dx, __builtin_fmaf(dy, dy, __builtin_fmaf(dz, dz, eps2f)));
        const float ri = rsqrt32(r2);
        const float ri2 = ri * ri;
        const float dax = s.a.x - t.ax, day = s.a.y - t.ay, daz = s.a.z - t.az;
        const float q = __builtin_fmaf(dax, dx, __builtin_fmaf(day, dy, daz * dz));
        const float w = (s.p.w * ri) * ri2;
        const float w5 = (w * q) * ri2;
        r.x = __builtin_fmaf(w, dax, r.x);
        r.y = __builtin_fmaf(w, day, r.y);
        r.z = __builtin_fmaf(w, daz, r.z);
        r.u = __builtin_fmaf(w5, dx, r.u);
        r.v = __builtin_fmaf(w5, dy, r.v);
        r.w = __builtin_fmaf(w5, dz, r.w);
        r.m = __builtin_fmaf(w, max3abs(dax, day, daz), r.m);
    }
};

template <class Near> struct FarOf;
template <> struct FarOf<AccMixed> { using type = AccRel; static constexpr int kMeta = 1; };
template <> struct FarOf<GradMixed> { using type = GradRel; static constexpr int kMeta = 2; };

// workgroup-wide min/max of the K targets of every lane (FP32 box)
template <int W>
__device__ __forceinline__ void block_box(float lo[3], float hi[3], float* sbox /* [2][3][W] */) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            lo[d] = fminf(lo[d], __shfl_xor(lo[d], off));
            hi[d] = fmaxf(hi[d], __shfl_xor(hi[d], off));
        }
    }
    if (lane == 0) {
#pragma unroll
        for (int d = 0; d < 3; ++d) { sbox[d * W + wave] = lo[d]; sbox[(3 + d) * W + wave] = hi[d]; }
    }
    __syncthreads();
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        lo[d] = sbox[d * W];
        hi[d] = sbox[(3 + d) * W];
        for (int w = 1; w < W; ++w) {
            lo[d] = fminf(lo[d], sbox[d * W + w]);
            hi[d] = fmaxf(hi[d], sbox[(3 + d) * W + w]);
        }
    }
}

// Sweep of sorted sources [j0, j1) (tile aligned) for the K targets of each lane.  Per tile the
// workgroup decides from the tile metadata whether the tile is near its target box; near tiles
// run the FP64-difference operation, far tiles the FP32 tile-relative one.
template <class Near, int K, int W>
__device__ __forceinline__ void sweep_sorted(const PairArgs& a, char* tile_raw, float* sbox, int tbase, int j0, int j1,
                                             typename Near::A64 (&acc)[K], int (&slot)[K], int (&pidx)[K]) {
    using Far = typename FarOf<Near>::type;
    constexpr int T = 64 * W;
    constexpr int kMeta = FarOf<Near>::kMeta;
    const int lane = threadIdx.x & 63;
    const int nt = a.tgt.count;
    typename Near::Tgt tg[K];
    float lo[3] = {__builtin_huge_valf(), __builtin_huge_valf(), __builtin_huge_valf()};
    float hi[3] = {-__builtin_huge_valf(), -__builtin_huge_valf(), -__builtin_huge_valf()};
#pragma unroll
    for (int k = 0; k < K; ++k) {
        slot[k] = tbase + k * 64 + lane;
        const int s = slot[k] < nt ? slot[k] : nt - 1;
        pidx[k] = particle_of(a.tgt, s, a.P.n, a.flags);
        Near::target(a, pidx[k], tg[k]);
        Near::zero(acc[k]);
        const float px = (float)tg[k].x, py = (float)tg[k].y, pz = (float)tg[k].z;
        lo[0] = fminf(lo[0], px); lo[1] = fminf(lo[1], py); lo[2] = fminf(lo[2], pz);
        hi[0] = fmaxf(hi[0], px); hi[1] = fmaxf(hi[1], py); hi[2] = fmaxf(hi[2], pz);
    }
    block_box<W>(lo, hi, sbox);
    typename Near::Src* tnear = reinterpret_cast<typename Near::Src*>(tile_raw);
    unsigned long long n_near = 0, n_far = 0;
    for (int jt = j0; jt < j1; jt += T) {
        const int len = min(T, j1 - jt);
        const int tix = jt / T;
        const double4 c = load_uniform4d(a.tile_meta, kMeta * tix);
        const double4 ca = kMeta > 1 ? load_uniform4d(a.tile_meta, kMeta * tix + 1) : c;
        const float2 hm = __builtin_bit_cast(float2, c.w);  // (tile half-extent, G * tile mass)
        const float h = hm.x;
        const float ha = kMeta > 1 ? unpack_gm(ca.w) : 0.f;  // half-extent of the tile's accelerations
        float gap2 = 0.f;
        {
            const float cc[3] = {(float)c.x, (float)c.y, (float)c.z};
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                const float g = fmaxf(0.f, fmaxf(cc[d] - h - hi[d], lo[d] - (cc[d] + h)));
                gap2 = __builtin_fmaf(g, g, gap2);
            }
        }
        const bool near = gap2 < (a.kappa * h) * (a.kappa * h);
        n_near += near ? 1 : 0;
        n_far += near ? 0 : 1;
        if (near) {
            // near tiles are staged through LDS (FP64 sources); the decision is uniform over
            // the workgroup, so the barriers are too
            __syncthreads();
            if ((int)threadIdx.x < len) tnear[threadIdx.x] = Near::load(a, jt + threadIdx.x);
            __syncthreads();
            for (int js = 0; js < len; js += kFold) {
                const int je = min(len, js + kFold);
                typename Near::A32 part[K];
#pragma unroll
                for (int k = 0; k < K; ++k) Near::zero(part[k]);
#pragma unroll 2
                for (int j = js; j < je; ++j) {
                    const typename Near::Src s = tnear[j];
#pragma unroll
                    for (int k = 0; k < K; ++k) Near::pair(part[k], tg[k], s, a.eps2f);
                }
#pragma unroll
                for (int k = 0; k < K; ++k) Near::fold(acc[k], part[k]);
            }
        } else {
            typename Far::Tgt tf[K];
            float fac[K];
#pragma unroll
            for (int k = 0; k < K; ++k) {
                Far::rel(tf[k], tg[k], c, ca);
                if (Far::kTileBound) acc[k].m += (double)Far::bound(tf[k], h, hm.y, ha);  // the whole tile
                fac[k] = Far::factor(tf[k], ha);
            }
            for (int js = 0; js < len; js += kFold) {
                const int je = min(len, js + kFold);
                typename Near::A32 part[K];
#pragma unroll
                for (int k = 0; k < K; ++k) Near::zero(part[k]);
#pragma unroll 4
                for (int j = js; j < je; ++j) {
                    const typename Far::Src s = Far::load_uniform(a, jt + j);  // scalar loads
#pragma unroll
                    for (int k = 0; k < K; ++k) Far::pair(part[k], tf[k], s, a.eps2f);
                }
#pragma unroll
                for (int k = 0; k < K; ++k) {
                    if (Far::kWeightSum) part[k].m *= fac[k];
                    Near::fold(acc[k], part[k]);
                }
            }
        }
    }
    if (a.tile_stats && threadIdx.x == 0) {
        atomicAdd(&a.tile_stats[0], n_near);
        atomicAdd(&a.tile_stats[1], n_far);
    }
}

// number of stored components of an operation (results + magnitude estimate)
template <class Op>
constexpr int ncomp_of() { return Op::NC + (Op::kCond ? 1 : 0); }

// ---- sweep of one source range for the K targets of each lane -------------------------------
// Loads the lane's targets (slots tbase + k*64 + lane of a.tgt; slots past nt duplicate the last
// target and are not written by the caller), then walks sources [j0, j1) of the packed stream
// in LDS tiles of 64*W.  DETECT: track min s^2 per tile and re-evaluate the wavefront's tile in
// FP64 when a lane saw s^2 < a.rfb2f.  All threads of the workgroup must call it (it
// synchronises).

template <class Op, int K, int W, bool DETECT, bool EXCL = false>
__device__ __forceinline__ void sweep(const PairArgs& a, typename Op::Src* tile, int tbase, int j0, int j1,
                                      typename Op::A64 (&acc)[K], int (&slot)[K], int (&pidx)[K],
                                      int32_t* tsub = nullptr) {
    constexpr int T = 64 * W;
    const int lane = threadIdx.x & 63;
    const int nt = a.tgt.count;
    typename Op::Tgt tg[K];
    int32_t sid[K];
#pragma unroll
    for (int k = 0; k < K; ++k) {
        slot[k] = tbase + k * 64 + lane;
        const int s = slot[k] < nt ? slot[k] : nt - 1;  // ragged tail: duplicate the last target
        pidx[k] = particle_of(a.tgt, s, a.P.n, a.flags);
        Op::target(a, pidx[k], tg[k]);
        Op::zero(acc[k]);
        if constexpr (EXCL) sid[k] = a.sub[pidx[k]];
    }
    for (int jt = j0; jt < j1; jt += T) {
        const int len = min(T, j1 - jt);
        // The tile is staged through LDS.  (Wavefront-uniform scalar loads, which the sorted far
        // path uses, measured slower here: the FP64 sources take twice the SGPR traffic and the
        // close-pair variants lost occupancy.)
        __syncthreads();
        if ((int)threadIdx.x < len) {
            tile[threadIdx.x] = Op::load(a, jt + threadIdx.x);
            if constexpr (EXCL) tsub[threadIdx.x] = a.sub[particle_of(a.src, jt + threadIdx.x, a.P.n, a.flags)];
        }
        __syncthreads();
        if constexpr (Op::kMixed) {
            // FP32 partials span at most kFold sources before they are merged in FP64; a
            // close pair re-evaluates only its kFold-source slice in FP64
            for (int js = 0; js < len; js += kFold) {
                const int je = min(len, js + kFold);
                typename Op::A32 part[K];
#pragma unroll
                for (int k = 0; k < K; ++k) Op::zero(part[k]);
                float dmin = __builtin_huge_valf();
#pragma unroll 4
                for (int j = js; j < je; ++j) {
                    const typename Op::Src s = tile[j];
                    float r2[K];
                    if constexpr (EXCL) {
                        const int32_t sj = tsub[j];
#pragma unroll
                        for (int k = 0; k < K; ++k) {
                            typename Op::Src sk = s;
                            if (sj == sid[k]) Op::exclude(sk);
                            r2[k] = Op::pair(part[k], tg[k], sk, a.eps2f);
                        }
                    } else {
#pragma unroll
                        for (int k = 0; k < K; ++k) r2[k] = Op::pair(part[k], tg[k], s, a.eps2f);
                    }
                    if constexpr (DETECT) {
#pragma unroll
                        for (int k = 0; k < K; k += 2) {
                            if (k + 1 < K) dmin = fminf(dmin, fminf(r2[k], r2[k + 1]));
                            else dmin = fminf(dmin, r2[k]);
                        }
                    }
                }
                bool redo = false;
                if constexpr (DETECT) {
                    bool close = dmin < a.rfb2f;
                    if constexpr (Op::kMax) {  // a rate beyond the FP32 range (overflow or r = 0)
#pragma unroll
                        for (int k = 0; k < K; ++k) close = close || Op::beyond(part[k]);
                    }
                    redo = __any(close);
                }
                if (redo) {
#pragma unroll
                    for (int k = 0; k < K; ++k) Op::redo(acc[k], a, pidx[k], jt + js, je - js);
                } else {
#pragma unroll
                    for (int k = 0; k < K; ++k) Op::fold(acc[k], part[k]);
                }
            }
        } else {
            const double eps2t = a.eps2 + kTiny64;
#pragma unroll 2
            for (int j = 0; j < len; ++j) {
                const typename Op::Src s = tile[j];
                if constexpr (EXCL) {
                    const int32_t sj = tsub[j];
#pragma unroll
                    for (int k = 0; k < K; ++k)
                        if (sj != sid[k]) Op::pair64(acc[k], tg[k], s, eps2t, pidx[k]);
                } else {
#pragma unroll
                    for (int k = 0; k < K; ++k) Op::pair64(acc[k], tg[k], s, eps2t, pidx[k]);
                }
            }
        }
    }
}

// ---- conditioning check and FP64 fix-up --------------------------------------------------------
// A mixed result y with magnitude estimate M is re-evaluated in FP64 when M > cond_max |y|:
// the FP32 error of a pair term is bounded relative to that term, so the relative error of y
// grows with M / |y| (cancellation).

__device__ __forceinline__ void cond_check(const PairArgs& a, int slot, const double* v) {
    const double ny = sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
    if (v[3] > a.cond_max * ny) {
        const int e = atomicAdd(a.fix_count, 1);
        if (e < a.tgt.count) a.fix_list[e] = slot;
    }
}

// ---- output of one target ------------------------------------------------------------------

template <class Op>
__device__ __forceinline__ void write_result(const PairArgs& a, int slot, int pi, const double* v) {
    if constexpr (Op::kMax) {
        // dt = eta W^(-1/2); W = 0 (no valid source) gives +inf
        const double dff = a.eta0 / sqrt(v[0]), dfb = a.eta1 / sqrt(v[1]);
        if (__builtin_isnan(dff) || __builtin_isnan(dfb)) atomicOr(a.flags, BF_FLAG_NONFINITE);
        a.o0[pi] = dff;
        a.o1[pi] = dfb;
    } else {
        if (!__builtin_isfinite(v[0]) || !__builtin_isfinite(v[1]) || !__builtin_isfinite(v[2]))
            atomicOr(a.flags, BF_FLAG_NONFINITE);
        a.o0[pi] = v[0];
        a.o1[pi] = v[1];
        a.o2[pi] = v[2];
        if constexpr (Op::kCond) cond_check(a, slot, v);
    }
}

// FP64 sum over the sources q0 <= q < q1 of `src` for target particle pi, one workgroup of 256
// threads (each takes every 256th source, then a fixed tree in LDS); the result in thread 0.
template <int OP>
__device__ __forceinline__ void fix_range(const Masters& P, const DevSet& src, const int32_t* sub, int pi, double G,
                                          double eps2, uint32_t* flags, int q0, int q1, double* out3) {
    __shared__ double red[3][256];
    double sx = 0.0, sy = 0.0, sz = 0.0, sm = 0.0;
    const T64 t = target64<OP == OP_GRAD>(P, pi);
#pragma unroll 2
    for (int q = q0 + (int)threadIdx.x; q < q1; q += 256) {
        const int pj = particle_of(src, q, P.n, flags);
        if (pj == pi || same_sub(sub, pi, pj)) continue;
        if constexpr (OP == OP_ACC) acc_pair64(P, t, pj, G, eps2, sx, sy, sz, sm, flags);
        else grad_pair64(P, t, pj, G, eps2, sx, sy, sz, sm, flags);
    }
    __syncthreads();
    red[0][threadIdx.x] = sx; red[1][threadIdx.x] = sy; red[2][threadIdx.x] = sz;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) {
            red[0][threadIdx.x] += red[0][threadIdx.x + s];
            red[1][threadIdx.x] += red[1][threadIdx.x + s];
            red[2][threadIdx.x] += red[2][threadIdx.x + s];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) { out3[0] = red[0][0]; out3[1] = red[1][0]; out3[2] = red[2][0]; }
}

template <int OP>
__device__ __forceinline__ void fix_one(const Masters& P, const DevSet& src, const int32_t* sub, int pi, double G,
                                        double eps2, uint32_t* flags, double* out3) {
    fix_range<OP>(P, src, sub, pi, G, eps2, flags, 0, src.count, out3);
}

}  // namespace bf
