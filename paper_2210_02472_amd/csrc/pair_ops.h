// Pair operations shared by the single-set kernels (pairs.hip) and the batched persistent
// kernel (batch.hip): per-pair arithmetic of the acceleration, force-gradient and time-step passes
// in mixed and FP64 precision, the FP64 re-evaluation of close-pair tiles, and the tile sweep.
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

constexpr float kTiny32 = 1e-20f;   // added to s^2 in FP32: keeps the self pair finite (and zero)
constexpr double kTiny64 = 1e-150;  // same in FP64

// ---- operations ----------------------------------------------------------------------------
// Each operation provides: Src (LDS element), Tgt (per-target registers), A32 (per-tile
// partial), A64 (running result), and the steps used by the skeleton.

// Newtonian acceleration, mixed precision.  Pack: float4 (x, y, z, G m).
struct AccMixed {
    static constexpr int NC = 3;
    static constexpr bool kMixed = true;
    static constexpr bool kMax = false;
    struct Src { float4 p; };
    struct Tgt { float x, y, z; };
    struct A32 { float x, y, z; };
    struct A64 { double x, y, z; };
    __device__ static Src load(const PairArgs& a, int q) { return {static_cast<const float4*>(a.pack)[q]}; }
    __device__ static void target(const PairArgs& a, int p, Tgt& t) {
        t.x = (float)a.P.x[p]; t.y = (float)a.P.y[p]; t.z = (float)a.P.z[p];
    }
    __device__ static void zero(A32& r) { r.x = r.y = r.z = 0.f; }
    __device__ static void zero(A64& r) { r.x = r.y = r.z = 0.0; }
    __device__ static float pair(A32& r, const Tgt& t, const Src& s, float eps2f) {
        const float dx = s.p.x - t.x, dy = s.p.y - t.y, dz = s.p.z - t.z;
        const float r2 = __builtin_fmaf(dx, dx, __builtin_fmaf(dy, dy, __builtin_fmaf(dz, dz, eps2f)));
        const float ri = rsqrt32(r2);
        const float ri2 = ri * ri;
        const float w = (s.p.w * ri) * ri2;
        r.x = __builtin_fmaf(w, dx, r.x);
        r.y = __builtin_fmaf(w, dy, r.y);
        r.z = __builtin_fmaf(w, dz, r.z);
        return r2;
    }
    __device__ static void fold(A64& o, const A32& i) { o.x += (double)i.x; o.y += (double)i.y; o.z += (double)i.z; }
    // FP64 re-evaluation of sources [q0, q0 + len) for target particle pi.
    __device__ static void redo(A64& o, const PairArgs& a, int pi, int q0, int len) {
        const double xi = a.P.x[pi], yi = a.P.y[pi], zi = a.P.z[pi];
        double sx = 0.0, sy = 0.0, sz = 0.0;
        for (int q = q0; q < q0 + len; ++q) {
            const int pj = particle_of(a.src, q, a.P.n, a.flags);
            if (pj == pi) continue;
            const double dx = a.P.x[pj] - xi, dy = a.P.y[pj] - yi, dz = a.P.z[pj] - zi;
            const double r2 = dx * dx + dy * dy + dz * dz + a.eps2;
            if (r2 == 0.0) { atomicOr(a.flags, BF_FLAG_COINCIDENT); continue; }
            const double ri = rsqrt64(r2);
            const double w = a.G * a.P.m[pj] * ri * ri * ri;
            sx += w * dx; sy += w * dy; sz += w * dz;
        }
        o.x += sx; o.y += sy; o.z += sz;
    }
    __device__ static void comps(const A64& o, double* v) { v[0] = o.x; v[1] = o.y; v[2] = o.z; }
};

// Force-gradient sum, mixed precision.  Pack: double4 (x, y, z, [G m as float | 0]) and
// double4 (ax, ay, az, 0).  The position and acceleration differences are taken in FP64 and
// rounded once to FP32 (a_ji = a_j - a_i cancels strongly for near neighbours, whose 1/r^3
// weight dominates the sum); everything after that is FP32.  Per pair:
// Gsum += w (a_ji - 3 (a_ji . r) r / s^2) with w = G m / s^3, accumulated as two sums
// S1 = sum w a_ji and S2 = sum w (a_ji . r)/s^2 r, Gsum = S1 - 3 S2.
struct GradMixed {
    static constexpr int NC = 3;
    static constexpr bool kMixed = true;
    static constexpr bool kMax = false;
    struct Src { double4 p, a; };
    struct Tgt { double x, y, z, ax, ay, az; };
    struct A32 { float x, y, z, u, v, w; };
    struct A64 { double x, y, z; };
    __device__ static Src load(const PairArgs& a, int q) {
        const double4* pk = static_cast<const double4*>(a.pack);
        return {pk[2 * q], pk[2 * q + 1]};
    }
    __device__ static void target(const PairArgs& a, int p, Tgt& t) {
        t.x = a.P.x[p]; t.y = a.P.y[p]; t.z = a.P.z[p];
        t.ax = a.P.ax[p]; t.ay = a.P.ay[p]; t.az = a.P.az[p];
    }
    __device__ static void zero(A32& r) { r.x = r.y = r.z = r.u = r.v = r.w = 0.f; }
    __device__ static void zero(A64& r) { r.x = r.y = r.z = 0.0; }
    __device__ static float pair(A32& r, const Tgt& t, const Src& s, float eps2f) {
        const float dx = (float)(s.p.x - t.x), dy = (float)(s.p.y - t.y), dz = (float)(s.p.z - t.z);
        const float gm = __builtin_bit_cast(float2, s.p.w).x;
        const float r2 = __builtin_fmaf(dx, dx, __builtin_fmaf(dy, dy, __builtin_fmaf(dz, dz, eps2f)));
        const float ri = rsqrt32(r2);
        const float ri2 = ri * ri;
        const float dax = (float)(s.a.x - t.ax), day = (float)(s.a.y - t.ay), daz = (float)(s.a.z - t.az);
        const float q = __builtin_fmaf(dax, dx, __builtin_fmaf(day, dy, daz * dz));
        const float w = (gm * ri) * ri2;
        const float w5 = (w * q) * ri2;
        r.x = __builtin_fmaf(w, dax, r.x);
        r.y = __builtin_fmaf(w, day, r.y);
        r.z = __builtin_fmaf(w, daz, r.z);
        r.u = __builtin_fmaf(w5, dx, r.u);
        r.v = __builtin_fmaf(w5, dy, r.v);
        r.w = __builtin_fmaf(w5, dz, r.w);
        return r2;
    }
    __device__ static void fold(A64& o, const A32& i) {
        o.x += (double)i.x - 3.0 * (double)i.u;
        o.y += (double)i.y - 3.0 * (double)i.v;
        o.z += (double)i.z - 3.0 * (double)i.w;
    }
    __device__ static void redo(A64& o, const PairArgs& a, int pi, int q0, int len) {
        const double xi = a.P.x[pi], yi = a.P.y[pi], zi = a.P.z[pi];
        const double axi = a.P.ax[pi], ayi = a.P.ay[pi], azi = a.P.az[pi];
        double sx = 0.0, sy = 0.0, sz = 0.0;
        for (int q = q0; q < q0 + len; ++q) {
            const int pj = particle_of(a.src, q, a.P.n, a.flags);
            if (pj == pi) continue;
            const double dx = a.P.x[pj] - xi, dy = a.P.y[pj] - yi, dz = a.P.z[pj] - zi;
            const double r2 = dx * dx + dy * dy + dz * dz + a.eps2;
            if (r2 == 0.0) { atomicOr(a.flags, BF_FLAG_COINCIDENT); continue; }
            const double dax = a.P.ax[pj] - axi, day = a.P.ay[pj] - ayi, daz = a.P.az[pj] - azi;
            const double ri = rsqrt64(r2);
            const double ri2 = ri * ri;
            const double w = a.G * a.P.m[pj] * ri * ri2;
            const double q3 = 3.0 * (dax * dx + day * dy + daz * dz) * ri2;
            sx += w * (dax - q3 * dx); sy += w * (day - q3 * dy); sz += w * (daz - q3 * dz);
        }
        o.x += sx; o.y += sy; o.z += sz;
    }
    __device__ static void comps(const A64& o, double* v) { v[0] = o.x; v[1] = o.y; v[2] = o.z; }
};

// Time-step maxima, mixed precision.  Pack: float4 (x, y, z, G m), float4 (vx, vy, vz, 0).
// Per pair: Wff = max G(m_i + m_j)/r^3, Wfb = max |v_ij|^2/r^2 (unsoftened); then
// dt_ff = eta_ff Wff^(-1/2), dt_fb = eta_fb Wfb^(-1/2).
struct DtMixed {
    static constexpr int NC = 2;
    static constexpr bool kMixed = true;
    static constexpr bool kMax = true;
    struct Src { float4 p, v; };
    struct Tgt { float x, y, z, vx, vy, vz, gm; };
    struct A32 { float ff, fb; };
    struct A64 { double ff, fb; };
    __device__ static Src load(const PairArgs& a, int q) {
        const float4* pk = static_cast<const float4*>(a.pack);
        return {pk[2 * q], pk[2 * q + 1]};
    }
    __device__ static void target(const PairArgs& a, int p, Tgt& t) {
        t.x = (float)a.P.x[p]; t.y = (float)a.P.y[p]; t.z = (float)a.P.z[p];
        t.vx = (float)a.P.vx[p]; t.vy = (float)a.P.vy[p]; t.vz = (float)a.P.vz[p];
        t.gm = (float)(a.G * a.P.m[p]);
    }
    __device__ static void zero(A32& r) { r.ff = r.fb = 0.f; }
    __device__ static void zero(A64& r) { r.ff = r.fb = 0.0; }
    __device__ static float pair(A32& r, const Tgt& t, const Src& s, float /*eps2f*/) {
        const float dx = s.p.x - t.x, dy = s.p.y - t.y, dz = s.p.z - t.z;
        const float r2 = __builtin_fmaf(dx, dx, __builtin_fmaf(dy, dy, dz * dz));
        const float ux = s.v.x - t.vx, uy = s.v.y - t.vy, uz = s.v.z - t.vz;
        const float u2 = __builtin_fmaf(ux, ux, __builtin_fmaf(uy, uy, uz * uz));
        const float ri = rsqrt32(r2);
        const float ri2 = ri * ri;
        r.fb = fmaxf(r.fb, u2 * ri2);
        r.ff = fmaxf(r.ff, ((s.p.w + t.gm) * ri2) * ri);
        return r2;
    }
    __device__ static void fold(A64& o, const A32& i) { o.ff = fmax(o.ff, (double)i.ff); o.fb = fmax(o.fb, (double)i.fb); }
    __device__ static void redo(A64& o, const PairArgs& a, int pi, int q0, int len) {
        const double xi = a.P.x[pi], yi = a.P.y[pi], zi = a.P.z[pi];
        const double vxi = a.P.vx[pi], vyi = a.P.vy[pi], vzi = a.P.vz[pi], mi = a.P.m[pi];
        double ff = o.ff, fb = o.fb;
        for (int q = q0; q < q0 + len; ++q) {
            const int pj = particle_of(a.src, q, a.P.n, a.flags);
            if (pj == pi) continue;
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
    static constexpr bool kMixed = false;
    static constexpr bool kMax = false;
    struct Src { double4 p; };
    struct Tgt { double x, y, z; };
    using A32 = int;  // unused
    struct A64 { double x, y, z; };
    __device__ static Src load(const PairArgs& a, int q) { return {static_cast<const double4*>(a.pack)[q]}; }
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
    static constexpr bool kMixed = false;
    static constexpr bool kMax = false;
    struct Src { double4 p, a; };
    struct Tgt { double x, y, z, ax, ay, az; };
    using A32 = int;
    struct A64 { double x, y, z; };
    __device__ static Src load(const PairArgs& a, int q) {
        const double4* pk = static_cast<const double4*>(a.pack);
        return {pk[2 * q], pk[2 * q + 1]};
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
    static constexpr bool kMixed = false;
    static constexpr bool kMax = true;
    struct Src { double4 p, v; };   // v.w = source particle index (exact in FP64)
    struct Tgt { double x, y, z, vx, vy, vz, gm; int p; };
    using A32 = int;
    struct A64 { double ff, fb; };
    __device__ static Src load(const PairArgs& a, int q) {
        const double4* pk = static_cast<const double4*>(a.pack);
        return {pk[2 * q], pk[2 * q + 1]};
    }
    __device__ static void target(const PairArgs& a, int p, Tgt& t) {
        t.x = a.P.x[p]; t.y = a.P.y[p]; t.z = a.P.z[p];
        t.vx = a.P.vx[p]; t.vy = a.P.vy[p]; t.vz = a.P.vz[p];
        t.gm = a.G * a.P.m[p]; t.p = p;
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

// ---- sweep of one source range for the K targets of each lane -------------------------------
// Loads the lane's targets (slots tbase + k*64 + lane of a.tgt; slots past nt duplicate the last
// target and are not written by the caller), then walks sources [j0, j1) of the packed stream
// in LDS tiles of 64*W.  All threads of the workgroup must call it (it synchronises).

template <class Op, int K, int W>
__device__ __forceinline__ void sweep(const PairArgs& a, typename Op::Src* tile, int tbase, int j0, int j1,
                                      typename Op::A64 (&acc)[K], int (&slot)[K], int (&pidx)[K]) {
    constexpr int T = 64 * W;
    const int lane = threadIdx.x & 63;
    const int nt = a.tgt.count;
    typename Op::Tgt tg[K];
#pragma unroll
    for (int k = 0; k < K; ++k) {
        slot[k] = tbase + k * 64 + lane;
        const int s = slot[k] < nt ? slot[k] : nt - 1;  // ragged tail: duplicate the last target
        pidx[k] = particle_of(a.tgt, s, a.P.n, a.flags);
        Op::target(a, pidx[k], tg[k]);
        Op::zero(acc[k]);
    }
    for (int jt = j0; jt < j1; jt += T) {
        const int len = min(T, j1 - jt);
        __syncthreads();
        if ((int)threadIdx.x < len) tile[threadIdx.x] = Op::load(a, jt + threadIdx.x);
        __syncthreads();
        if constexpr (Op::kMixed) {
            typename Op::A32 part[K];
#pragma unroll
            for (int k = 0; k < K; ++k) Op::zero(part[k]);
            float dmin = __builtin_huge_valf();
#pragma unroll 4
            for (int j = 0; j < len; ++j) {
                const typename Op::Src s = tile[j];
                float r2[K];
#pragma unroll
                for (int k = 0; k < K; ++k) r2[k] = Op::pair(part[k], tg[k], s, a.eps2f);
#pragma unroll
                for (int k = 0; k < K; k += 2) {
                    if (k + 1 < K) dmin = fminf(dmin, fminf(r2[k], r2[k + 1]));
                    else dmin = fminf(dmin, r2[k]);
                }
            }
            if (__any(dmin < a.rfb2f)) {
#pragma unroll
                for (int k = 0; k < K; ++k) Op::redo(acc[k], a, pidx[k], jt, len);
            } else {
#pragma unroll
                for (int k = 0; k < K; ++k) Op::fold(acc[k], part[k]);
            }
        } else {
            const double eps2t = a.eps2 + kTiny64;
#pragma unroll 2
            for (int j = 0; j < len; ++j) {
                const typename Op::Src s = tile[j];
#pragma unroll
                for (int k = 0; k < K; ++k) Op::pair64(acc[k], tg[k], s, eps2t, pidx[k]);
            }
        }
    }
}

}  // namespace bf
