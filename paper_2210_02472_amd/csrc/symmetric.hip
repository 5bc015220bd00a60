// Pair-symmetric sweep of the spatially sorted mixed acceleration and force-gradient passes, for
// passes whose targets and sources are one set (every particle active: a plain FSI step, level
// 0 of the hierarchy).
//
// The two terms of a pair differ only by the mass factor and the sign (Sec. 2.1, Eqs.
// new-newton-acc and new-grad-acc; r = x_j - x_i, a_ji = a_j - a_i, s^2 = r^2 + eps^2):
//   acceleration:   +G m_j r / s^3 on i,   -G m_i r / s^3 on j;
//   force gradient: +G m_j U / s^3 on i,   -G m_i U / s^3 on j,  U = a_ji - 3 (a_ji . r) r / s^2
// (swapping i and j flips both r and a_ji).  Each unordered pair is evaluated once and both
// terms are kept: the shared part (differences, s^2, rsqrt, U) is paid once per pair.
//
// Decomposition.  Particles are in Morton order, in tiles of 64; a block is B = kSymBlockTiles
// tiles.
//  * Workgroup w owns block w as rows: its W wavefronts hold R row tiles each (W R = B), one
//    particle of each row tile per lane.
//  * It sweeps the column blocks w, w+1, ..., w + nb/2 (cyclically, nb blocks), so that every
//    unordered pair of blocks is visited once; the pair at distance exactly nb/2 (nb even) is
//    visited by the lower-numbered block only.  Inside its own block a row tile pairs with the
//    column tiles after it and, in the diagonal tile, with the later particles only.
//  * All wavefronts of the workgroup work on the same column tile at a time.  The tile is staged
//    in LDS (FP32 offsets from the tile centre and FP64 values, each plane stored twice so that
//    index lane + k never wraps), prefetched one tile ahead through registers.
//  * Rotation: at step k = 0..63 lane l pairs its row particles with column particle (l + k) mod
//    64.  Row terms accumulate in registers (FP32 over the tile, then merged into FP64).  The
//    column particle's accumulator travels with it: every step moves the accumulators one lane
//    down (DPP wave_rol:1, fused into the add), so that after step k lane l holds the accumulator
//    of column (l + k) mod 64; the R row particles of a lane add their column terms before the
//    move.  No cross-lane reduction is needed.
//  * After a tile the W wavefronts' column sums go through LDS, are added in FP64 in wavefront
//    order and stored as one FP32 partial per (column particle, block distance).  A second
//    kernel adds, per particle, the row sum and the partials of all distances in a fixed order.
//    No atomics touch the results, so they are bitwise repeatable.
//
// Precision follows the directed sorted sweep: a tile near the wavefront's rows (gap below
// kappa times the tile half-extent, and the tiles of the workgroup's own block with a diagonal
// or skipped row tile) uses FP64 differences rounded once to FP32; a far tile uses FP32 offsets
// from the column tile's centre for both particles.  The magnitude estimates that drive the
// FP64 fix-up: the force gradient carries w max|a_ji| per pair on both sides; the acceleration
// carries w max|r| per pair on near tiles, and on far tiles the bound G m_tile / d^2 (d: the
// particle's distance to the other tile's box) on both sides.
#include "pair_ops.h"

namespace bf {

namespace {

// x taken from lane (l + 1) mod 64, fused by the compiler into the consuming add
__device__ __forceinline__ float rol1(float x) {
    return __builtin_bit_cast(float, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, x), 0x134 /* wave_rol:1 */, 0xf,
                                                              0xf, true));
}

__device__ __forceinline__ float wave_min(float v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v = fminf(v, __shfl_xor(v, off));
    return v;
}
__device__ __forceinline__ float wave_max(float v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v = fmaxf(v, __shfl_xor(v, off));
    return v;
}
__device__ __forceinline__ float wave_sum_xor(float v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
    return v;
}

struct P32 { float x, y, z, m; };
struct P64 { double x, y, z, m; };
__device__ __forceinline__ void fold(P64& o, const P32& i) {
    o.x += (double)i.x; o.y += (double)i.y; o.z += (double)i.z; o.m += (double)i.m;
}

// Particles past the last one sit far away with zero mass and zero acceleration: every term
// they take part in vanishes (their own pairs give 0 * finite).
constexpr double kFarAway = 1e18;

// LDS planes of one staged column tile: 16-byte elements, 128 per plane (two copies of the 64)
constexpr int kPlaneLen = 128;

// ---- the acceleration ----------------------------------------------------------------------
// planes: 0 far (x - cx, y - cy, z - cz, G m) FP32; 1 near (x, y) FP64; 2 near (z, [G m]) FP64
struct SymAcc {
    static constexpr int kS = 1, kMeta = 1, kPlanes = 3, kFarPlanes = 1, kRedNear = 4, kRedFar = 3;
    static constexpr bool kAcc = true;
    struct Row { double x, y, z; float gm; };
    struct Rel { float x, y, z; };
    __device__ static void load_row(const SymArgs& g, int s, bool live, Row& t) {
        if (live) {
            const double4 p = static_cast<const double4*>(g.row_pack)[s];
            t.x = p.x; t.y = p.y; t.z = p.z; t.gm = unpack_gm(p.w);
        } else {
            t.x = t.y = t.z = kFarAway; t.gm = 0.f;
        }
    }
    // 16-byte element `plane` of sorted particle s, or the far-away filler
    __device__ static uint4 stage_elem(const SymArgs& g, int plane, int s, bool ok) {
        if (ok) {
            if (plane == 0) return static_cast<const uint4*>(g.far_pack)[s];
            return static_cast<const uint4*>(g.near_pack)[2 * s + (plane - 1)];
        }
        if (plane == 0) return __builtin_bit_cast(uint4, make_float4(1e18f, 1e18f, 1e18f, 0.f));
        if (plane == 1) return __builtin_bit_cast(uint4, make_double2(kFarAway, kFarAway));
        return __builtin_bit_cast(uint4, make_double2(kFarAway, 0.0));
    }
    __device__ static void rel(Rel& t, const Row& r, const double4& c, const double4&) {
        t.x = (float)(r.x - c.x); t.y = (float)(r.y - c.y); t.z = (float)(r.z - c.z);
    }
    template <bool MASK>
    __device__ static void near(P32& r, float (&c)[4], const Row& t, const uint4* pl, int j, float eps2f, bool ok) {
        const double2 xy = __builtin_bit_cast(double2, pl[kPlaneLen + j]);
        const double2 zw = __builtin_bit_cast(double2, pl[2 * kPlaneLen + j]);
        const float dx = dif32(xy.x, t.x), dy = dif32(xy.y, t.y), dz = dif32(zw.x, t.z);
        const float r2 = __builtin_fmaf(dx, dx, __builtin_fmaf(dy, dy, __builtin_fmaf(dz, dz, eps2f)));
        float ri = rsqrt32(r2);
        if (MASK) ri = ok ? ri : 0.f;
        const float ri3 = (ri * ri) * ri;
        const float wj = unpack_gm(zw.y) * ri3, wi = t.gm * ri3;
        const float mx = max3abs(dx, dy, dz);
        r.x = __builtin_fmaf(wj, dx, r.x);
        r.y = __builtin_fmaf(wj, dy, r.y);
        r.z = __builtin_fmaf(wj, dz, r.z);
        r.m = __builtin_fmaf(wj, mx, r.m);
        c[0] = wi * dx; c[1] = wi * dy; c[2] = wi * dz; c[3] = wi * mx;
    }
    __device__ static void far(P32& r, float (&c)[4], const Rel& t, const uint4* pl, int j, float gmi, float eps2f) {
        const float4 sp = __builtin_bit_cast(float4, pl[j]);
        const float dx = sp.x - t.x, dy = sp.y - t.y, dz = sp.z - t.z;
        const float r2 = __builtin_fmaf(dx, dx, __builtin_fmaf(dy, dy, __builtin_fmaf(dz, dz, eps2f)));
        const float ri = rsqrt32(r2);
        const float ri3 = (ri * ri) * ri;
        const float wj = sp.w * ri3, wi = gmi * ri3;
        r.x = __builtin_fmaf(wj, dx, r.x);
        r.y = __builtin_fmaf(wj, dy, r.y);
        r.z = __builtin_fmaf(wj, dz, r.z);
        c[0] = wi * dx; c[1] = wi * dy; c[2] = wi * dz;
    }
};

// ---- the force gradient --------------------------------------------------------------------
// planes: 0 far position offsets + G m, 1 far acceleration offsets (FP32); 2 near (x, y),
// 3 near (z, [G m]), 4 near (ax, ay), 5 near (az, 0) (FP64)
struct SymGrad {
    static constexpr int kS = 2, kMeta = 2, kPlanes = 6, kFarPlanes = 2, kRedNear = 4, kRedFar = 4;
    static constexpr bool kAcc = false;
    struct Row { double x, y, z, ax, ay, az; float gm; };
    struct Rel { float x, y, z, ax, ay, az; };
    __device__ static void load_row(const SymArgs& g, int s, bool live, Row& t) {
        if (live) {
            const double4* pk = static_cast<const double4*>(g.row_pack);
            const double4 p = pk[2 * s], a = pk[2 * s + 1];
            t.x = p.x; t.y = p.y; t.z = p.z; t.gm = unpack_gm(p.w);
            t.ax = a.x; t.ay = a.y; t.az = a.z;
        } else {
            t.x = t.y = t.z = kFarAway; t.gm = 0.f;
            t.ax = t.ay = t.az = 0.0;
        }
    }
    __device__ static uint4 stage_elem(const SymArgs& g, int plane, int s, bool ok) {
        if (ok) {
            if (plane < 2) return static_cast<const uint4*>(g.far_pack)[2 * s + plane];
            return static_cast<const uint4*>(g.near_pack)[4 * s + (plane - 2)];
        }
        if (plane == 0) return __builtin_bit_cast(uint4, make_float4(1e18f, 1e18f, 1e18f, 0.f));
        if (plane == 2) return __builtin_bit_cast(uint4, make_double2(kFarAway, kFarAway));
        if (plane == 3) return __builtin_bit_cast(uint4, make_double2(kFarAway, 0.0));
        return make_uint4(0u, 0u, 0u, 0u);
    }
    __device__ static void rel(Rel& t, const Row& r, const double4& c, const double4& ca) {
        t.x = (float)(r.x - c.x); t.y = (float)(r.y - c.y); t.z = (float)(r.z - c.z);
        t.ax = (float)(r.ax - ca.x); t.ay = (float)(r.ay - ca.y); t.az = (float)(r.az - ca.z);
    }
    // shared part of a pair from FP32 differences: U, 1/s^3, both terms
    __device__ static void core(P32& r, float (&c)[4], float dx, float dy, float dz, float dax, float day, float daz,
                                float ri, float gmj, float gmi) {
        const float ri2 = ri * ri;
        const float ri3 = ri2 * ri;
        const float q = __builtin_fmaf(dax, dx, __builtin_fmaf(day, dy, daz * dz));
        const float sq = (-3.f * q) * ri2;
        const float ux = __builtin_fmaf(sq, dx, dax), uy = __builtin_fmaf(sq, dy, day), uz = __builtin_fmaf(sq, dz, daz);
        const float wj = gmj * ri3, wi = gmi * ri3;
        const float mx = max3abs(dax, day, daz);
        r.x = __builtin_fmaf(wj, ux, r.x);
        r.y = __builtin_fmaf(wj, uy, r.y);
        r.z = __builtin_fmaf(wj, uz, r.z);
        r.m = __builtin_fmaf(wj, mx, r.m);
        c[0] = wi * ux; c[1] = wi * uy; c[2] = wi * uz; c[3] = wi * mx;
    }
    template <bool MASK>
    __device__ static void near(P32& r, float (&c)[4], const Row& t, const uint4* pl, int j, float eps2f, bool ok) {
        const double2 xy = __builtin_bit_cast(double2, pl[2 * kPlaneLen + j]);
        const double2 zw = __builtin_bit_cast(double2, pl[3 * kPlaneLen + j]);
        const double2 axy = __builtin_bit_cast(double2, pl[4 * kPlaneLen + j]);
        const double2 az0 = __builtin_bit_cast(double2, pl[5 * kPlaneLen + j]);
        const float dx = dif32(xy.x, t.x), dy = dif32(xy.y, t.y), dz = dif32(zw.x, t.z);
        const float r2 = __builtin_fmaf(dx, dx, __builtin_fmaf(dy, dy, __builtin_fmaf(dz, dz, eps2f)));
        float ri = rsqrt32(r2);
        if (MASK) ri = ok ? ri : 0.f;
        core(r, c, dx, dy, dz, dif32(axy.x, t.ax), dif32(axy.y, t.ay), dif32(az0.x, t.az), ri, unpack_gm(zw.y), t.gm);
    }
    __device__ static void far(P32& r, float (&c)[4], const Rel& t, const uint4* pl, int j, float gmi, float eps2f) {
        const float4 sp = __builtin_bit_cast(float4, pl[j]);
        const float4 sa = __builtin_bit_cast(float4, pl[kPlaneLen + j]);
        const float dx = sp.x - t.x, dy = sp.y - t.y, dz = sp.z - t.z;
        const float r2 = __builtin_fmaf(dx, dx, __builtin_fmaf(dy, dy, __builtin_fmaf(dz, dz, eps2f)));
        core(r, c, dx, dy, dz, sa.x - t.ax, sa.y - t.ay, sa.z - t.az, rsqrt32(r2), sp.w, gmi);
    }
};

// G m / d^2 with d the distance of point p to the box [lo, hi] (FP32, same frame)
__device__ __forceinline__ float box_bound(const float p[3], const float lo[3], const float hi[3], float gm) {
    float d2 = 0.f;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        const float g = fmaxf(0.f, fmaxf(lo[d] - p[d], p[d] - hi[d]));
        d2 = __builtin_fmaf(g, g, d2);
    }
    return gm / fmaxf(d2, 1e-30f);
}

// The column tiles a workgroup visits, in order (uniform over the workgroup).  One set: block
// distance d = 0..nb/2, tile t of block (wg + d) mod nb.
// Two sets: the column tiles [t, d_end) of the workgroup's share in order, d = the row block (the
// partial row).
struct TileWalk {
    int d = 0, t = 0, ct = -1;
    int d_end = 0;  // first distance (one set) or column tile (two sets) past this workgroup's share
    __device__ void next(const SymArgs& g, int wg) {
        const int nb = g.n_blocks, W = kSymBlockTiles;
        if (g.between) {
            ct = ct < 0 ? t : ct + 1;
            if (ct >= d_end) ct = -1;
            return;
        }
        if (ct >= 0) ++t;
        for (;;) {
            if (d >= d_end || 2 * d > nb || (d > 0 && 2 * d == nb && wg >= d)) { ct = -1; return; }
            const int b = wg + d < nb ? wg + d : wg + d - nb;
            if (t < W && b * W + t < g.n_tiles) { ct = b * W + t; return; }
            ++d;
            t = 0;
        }
    }
};

// Row modes of a (row tile, column tile) visit: the tile pair is skipped, it is the diagonal
// tile (pairs whose column index within the tile exceeds the row index), or it is counted whole.
enum { kSkip = 0, kDiag = 1, kFull = 2 };

// pair (lane, column (lane + k) mod 64) counts for a row in `mode`
__device__ __forceinline__ bool counts(int mode, int lane, int k) {
    return mode == kFull || (mode == kDiag && k > 0 && lane + k < 64);
}

// Is column tile ct near the box [lo, hi] (gap below kappa times the tile's half-extent)?
template <class S>
__device__ __forceinline__ bool tile_near(const SymArgs& g, int ct, const float (&lo)[3], const float (&hi)[3]) {
    const double4 c = load_uniform4d(g.tile_meta, S::kMeta * ct);
    const float h = __builtin_bit_cast(float2, c.w).x;
    const float cc[3] = {(float)c.x, (float)c.y, (float)c.z};
    float gap2 = 0.f;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        const float gg = fmaxf(0.f, fmaxf(cc[d] - h - hi[d], lo[d] - (cc[d] + h)));
        gap2 = __builtin_fmaf(gg, gg, gap2);
    }
    return gap2 < (g.kappa * h) * (g.kappa * h);
}

// One column tile for the R row particles of each lane: row terms into own[r]; the column sums
// end in xs[q][slot], slot = the column each lane holds after the 64 steps.
template <class S, int R>
__device__ __forceinline__ void sym_tile(const SymArgs& g, int ct, const int (&mode)[R], bool masked,
                                         const typename S::Row (&row)[R], const float (&lo)[3], const float (&hi)[3],
                                         float gm_rows, P64 (&own)[R], const uint4* pl, float (*xs)[64],
                                         unsigned& n_near, unsigned& n_far) {
    const int lane = threadIdx.x & 63;
    const double4 c = load_uniform4d(g.tile_meta, S::kMeta * ct);
    const double4 ca = S::kMeta > 1 ? load_uniform4d(g.tile_meta, S::kMeta * ct + 1) : c;
    const float2 hm = __builtin_bit_cast(float2, c.w);  // (half-extent, G * tile mass)
    const float h = hm.x;
    const float cc[3] = {(float)c.x, (float)c.y, (float)c.z};
    float gap2 = 0.f;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        const float gg = fmaxf(0.f, fmaxf(cc[d] - h - hi[d], lo[d] - (cc[d] + h)));
        gap2 = __builtin_fmaf(gg, gg, gap2);
    }
    // tiles with a diagonal or skipped row (own block only) take the masked FP64-difference loop
    const bool near = masked || gap2 < (g.kappa * h) * (g.kappa * h);
    n_near += near ? 1u : 0u;
    n_far += near ? 0u : 1u;
    P32 part[R];
#pragma unroll
    for (int r = 0; r < R; ++r) part[r] = P32{0.f, 0.f, 0.f, 0.f};
    float ja[4] = {0.f, 0.f, 0.f, 0.f};  // accumulator of column (lane + k) mod 64 after step k
    if (near) {
        if (masked) {
            for (int k = 0; k < 64; ++k) {
                float cs[4] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    float cv[4];
                    S::template near<true>(part[r], cv, row[r], pl, lane + k, g.eps2f, counts(mode[r], lane, k));
#pragma unroll
                    for (int q = 0; q < S::kRedNear; ++q) cs[q] += cv[q];
                }
#pragma unroll
                for (int q = 0; q < S::kRedNear; ++q) ja[q] = rol1(ja[q]) + cs[q];
            }
        } else {
#pragma unroll 2
            for (int k = 0; k < 64; ++k) {
                float cs[4];
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    float cv[4];
                    S::template near<false>(part[r], cv, row[r], pl, lane + k, g.eps2f, true);
#pragma unroll
                    for (int q = 0; q < S::kRedNear; ++q) cs[q] = r == 0 ? cv[q] : cs[q] + cv[q];
                }
#pragma unroll
                for (int q = 0; q < S::kRedNear; ++q) ja[q] = rol1(ja[q]) + cs[q];
            }
        }
    } else {
        typename S::Rel tr[R];
#pragma unroll
        for (int r = 0; r < R; ++r) S::rel(tr[r], row[r], c, ca);
#pragma unroll 2
        for (int k = 0; k < 64; ++k) {
            float cs[4];
#pragma unroll
            for (int r = 0; r < R; ++r) {
                float cv[4];
                S::far(part[r], cv, tr[r], pl, lane + k, row[r].gm, g.eps2f);
#pragma unroll
                for (int q = 0; q < S::kRedFar; ++q) cs[q] = r == 0 ? cv[q] : cs[q] + cv[q];
            }
#pragma unroll
            for (int q = 0; q < S::kRedFar; ++q) ja[q] = rol1(ja[q]) + cs[q];
        }
        if constexpr (S::kAcc) {
            // row side: every source of the tile lies in the cube of half-extent h about c
            const float clo[3] = {-h, -h, -h}, chi[3] = {h, h, h};
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const float p[3] = {tr[r].x, tr[r].y, tr[r].z};
                own[r].m += (double)box_bound(p, clo, chi, hm.y);
            }
            // column side: the column this lane holds, against the box of the wavefront's rows
            // (a filler column gets a bound too; it is never stored)
            const float4 f = __builtin_bit_cast(float4, pl[(lane + 63) & 63]);
            const float ps[3] = {f.x, f.y, f.z};
            const float rlo[3] = {lo[0] - cc[0], lo[1] - cc[1], lo[2] - cc[2]};
            const float rhi[3] = {hi[0] - cc[0], hi[1] - cc[1], hi[2] - cc[2]};
            ja[3] = box_bound(ps, rlo, rhi, gm_rows);
        }
    }
#pragma unroll
    for (int r = 0; r < R; ++r) fold(own[r], part[r]);
    const int slot = (lane + 63) & 63;
#pragma unroll
    for (int q = 0; q < 4; ++q) xs[q][slot] = ja[q];
}

// Workgroup of W wavefronts; wavefront v holds row tiles B R W + R v + r (r < R) of block B.
template <class S, int W, int R>
__global__ __launch_bounds__(64 * W) void k_pairs_sym(const SymArgs g) {
    static_assert(W * R == kSymBlockTiles, "a workgroup covers one block");
    constexpr int NPL = S::kPlanes;
    __shared__ uint4 colbuf[2][NPL * kPlaneLen];
    __shared__ float xch[2][W][4][64];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    // workgroup (chunk, block): block wg's rows against its share [d0, d1) of the distances (one
    // set) or of the column tiles (two sets)
    const int wg = blockIdx.x % g.n_blocks, chunk = g.chunk0 + (int)(blockIdx.x / g.n_blocks);
    const int d0 = chunk * g.chunk_len, d1 = d0 + g.chunk_len;
    const int rbase = wg * (W * R) + wave * R;
    typename S::Row row[R];
    bool tile_live[R];
    int rs[R];
    float lo[3] = {__builtin_huge_valf(), __builtin_huge_valf(), __builtin_huge_valf()};
    float hi[3] = {-__builtin_huge_valf(), -__builtin_huge_valf(), -__builtin_huge_valf()};
    float gm_lane = 0.f;
#pragma unroll
    for (int r = 0; r < R; ++r) {
        tile_live[r] = rbase + r < g.n_row_tiles;
        rs[r] = (rbase + r) * 64 + lane;
        const bool live = tile_live[r] && rs[r] < g.n_rows;
        S::load_row(g, rs[r], live, row[r]);
        if (live) {
            const float p[3] = {(float)row[r].x, (float)row[r].y, (float)row[r].z};
#pragma unroll
            for (int d = 0; d < 3; ++d) { lo[d] = fminf(lo[d], p[d]); hi[d] = fmaxf(hi[d], p[d]); }
        }
        gm_lane += row[r].gm;
    }
#pragma unroll
    for (int d = 0; d < 3; ++d) { lo[d] = wave_min(lo[d]); hi[d] = wave_max(hi[d]); }
    const float gm_rows = S::kAcc ? wave_sum_xor(gm_lane) * (1.0f + 1e-5f) : 0.f;
    P64 own[R];
#pragma unroll
    for (int r = 0; r < R; ++r) own[r] = P64{0.0, 0.0, 0.0, 0.0};
    unsigned n_near = 0, n_far = 0;
    // The workgroup's box (the union of its wavefronts' boxes): a column tile far from it is far
    // from every wavefront, which then read only its FP32 planes; the FP64 planes are staged only
    // when some wavefront may take the near path.  A workgroup with dead row tiles (the ragged last
    // block) masks, and so reads the FP64 planes, on every tile.
    __shared__ float wbox[W][6];
    __shared__ float ubox[6];
    if (lane == 0) {
#pragma unroll
        for (int d = 0; d < 3; ++d) { wbox[wave][d] = lo[d]; wbox[wave][3 + d] = hi[d]; }
    }
    __syncthreads();
    if (threadIdx.x < 6) {
        const int q = threadIdx.x;
        float u = wbox[0][q];
        for (int v = 1; v < W; ++v) u = q < 3 ? fminf(u, wbox[v][q]) : fmaxf(u, wbox[v][q]);
        ubox[q] = u;
    }
    __syncthreads();
    const bool all_near = (wg + 1) * (W * R) > g.n_row_tiles;
    // FP64 planes needed for the visit of column tile ct at distance d (one set: the own block masks)
    auto wants_near = [&](const TileWalk& t) {
        if (all_near || (!g.between && t.d == 0)) return true;
        const float ulo[3] = {ubox[0], ubox[1], ubox[2]}, uhi[3] = {ubox[3], ubox[4], ubox[5]};
        return tile_near<S>(g, t.ct, ulo, uhi);
    };

    // staging: element k of plane p is copied (twice) by thread 64 p' + k, p = p' + W u
    constexpr int SPT = (NPL + W - 1) / W;  // planes per staging thread
    const int st_k = threadIdx.x & 63;
    TileWalk cur, pre;
    if (g.between) {
        cur.d = wg;
        cur.t = d0;
        cur.d_end = min(d1, g.n_tiles);
    } else {
        cur.d = d0;
        cur.d_end = d1;
    }
    cur.next(g, wg);
    pre = cur;
    pre.next(g, wg);
    const bool cur_near = cur.ct >= 0 && wants_near(cur);
    bool pre_near = pre.ct >= 0 && wants_near(pre);
    uint4 held[SPT];
#pragma unroll
    for (int u = 0; u < SPT; ++u) {
        const int pl = wave + W * u;
        if (pl < NPL && cur.ct >= 0 && (pl < S::kFarPlanes || cur_near)) {
            const int s = cur.ct * 64 + st_k;
            const uint4 e = S::stage_elem(g, pl, s, s < g.n);
            colbuf[0][pl * kPlaneLen + st_k] = e;
            colbuf[0][pl * kPlaneLen + st_k + 64] = e;
        }
        held[u] = make_uint4(0u, 0u, 0u, 0u);
        if (pl < NPL && pre.ct >= 0 && (pl < S::kFarPlanes || pre_near)) {
            const int s = pre.ct * 64 + st_k;
            held[u] = S::stage_elem(g, pl, s, s < g.n);
        }
    }
    __syncthreads();
    for (int i = 0; cur.ct >= 0; ++i) {
        const int buf = i & 1;
        const int ct = cur.ct;
        float (*xs)[64] = xch[buf][wave];
        int mode[R];
        bool any = false, masked = false;
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int rt = rbase + r;
            mode[r] = !tile_live[r] ? kSkip : (g.between || cur.d > 0 || ct > rt) ? kFull : ct == rt ? kDiag : kSkip;
            any = any || mode[r] != kSkip;
            masked = masked || mode[r] != kFull;
        }
        if (any) {
            sym_tile<S, R>(g, ct, mode, masked, row, lo, hi, gm_rows, own, colbuf[buf], xs, n_near, n_far);
        } else {
#pragma unroll
            for (int q = 0; q < 4; ++q) xs[q][lane] = 0.f;
        }
#pragma unroll
        for (int u = 0; u < SPT; ++u) {
            const int pl = wave + W * u;
            if (pl < NPL && pre.ct >= 0 && (pl < S::kFarPlanes || pre_near)) {
                colbuf[buf ^ 1][pl * kPlaneLen + st_k] = held[u];
                colbuf[buf ^ 1][pl * kPlaneLen + st_k + 64] = held[u];
            }
        }
        __syncthreads();
        if (threadIdx.x < 4 * 64) {
            const int q = threadIdx.x >> 6, k = threadIdx.x & 63;
            double s = 0.0;
#pragma unroll
            for (int v = 0; v < W; ++v) s += (double)xch[buf][v][q][k];
            const int col = ct * 64 + k;
            // the column term carries the opposite sign (the estimate M does not)
            if (col < g.n) g.part[((size_t)(cur.d - g.d_base) * 4 + q) * g.n_pad + col] = (float)(q < 3 ? -s : s);
        }
        cur = pre;
        pre.next(g, wg);
        pre_near = pre.ct >= 0 && wants_near(pre);
#pragma unroll
        for (int u = 0; u < SPT; ++u) {
            const int pl = wave + W * u;
            if (pl < NPL && pre.ct >= 0 && (pl < S::kFarPlanes || pre_near)) {
                const int s = pre.ct * 64 + st_k;
                held[u] = S::stage_elem(g, pl, s, s < g.n);
            }
        }
    }
#pragma unroll
    for (int r = 0; r < R; ++r) {
        if (tile_live[r] && rs[r] < g.n_rows) {
            double* o = g.own + (size_t)(chunk - g.chunk0) * 4 * g.n_row_pad;  // every chunk writes its row sums
            o[rs[r]] = own[r].x;
            o[(size_t)g.n_row_pad + rs[r]] = own[r].y;
            o[(size_t)2 * g.n_row_pad + rs[r]] = own[r].z;
            o[(size_t)3 * g.n_row_pad + rs[r]] = own[r].m;
        }
    }
    if (g.tile_stats && lane == 0) {
        atomicAdd(&g.tile_stats[0], (unsigned long long)n_near);
        atomicAdd(&g.tile_stats[1], (unsigned long long)n_far);
    }
}

// Adds, per particle, the shares of this pass in order, each share's row sum and then its
// distances' column partials, onto the running sum of the earlier passes (g.acc); the last pass
// writes the result.  One pass or several: the same additions in the same order.
// (row sums of type TO, partials of type TP)
template <int NC, class TO, class TP, class V>
__device__ __forceinline__ void sym_gather(const SymArgs& g, int s, V (&v)[NC], bool mx) {
    const int b = (s >> 6) / kSymBlockTiles;
    const int nb = g.n_blocks, D = nb / 2;
    const TO* own = reinterpret_cast<const TO*>(g.own);
    const TP* part = reinterpret_cast<const TP*>(g.part);
    for (int c = g.chunk0; c < g.chunk0 + g.pass_chunks; ++c) {
#pragma unroll
        for (int q = 0; q < NC; ++q) {
            const V x = (V)own[((size_t)(c - g.chunk0) * NC + q) * g.n_row_pad + s];
            v[q] = mx ? fmax(v[q], x) : v[q] + x;
        }
        const int e = min(D + 1, (c + 1) * g.chunk_len);
        for (int d = c * g.chunk_len; d < e; ++d) {
            if (d > 0 && 2 * d == nb && b < d) continue;  // no partial: this block pair was swept from here
#pragma unroll
            for (int q = 0; q < NC; ++q) {
                const V x = (V)part[((size_t)(d - g.d_base) * NC + q) * g.n_pad + s];
                v[q] = mx ? fmax(v[q], x) : v[q] + x;
            }
        }
    }
}

// the running sums of the passes before (zero for the first) and after (stored unless last)
template <int NC, class V>
__device__ __forceinline__ void sym_acc_load(const SymArgs& g, int s, V (&v)[NC]) {
#pragma unroll
    for (int q = 0; q < NC; ++q) v[q] = g.first ? (V)0 : reinterpret_cast<const V*>(g.acc)[(size_t)q * g.n_pad + s];
}
template <int NC, class V>
__device__ __forceinline__ void sym_acc_store(const SymArgs& g, int s, const V (&v)[NC]) {
#pragma unroll
    for (int q = 0; q < NC; ++q) reinterpret_cast<V*>(g.acc)[(size_t)q * g.n_pad + s] = v[q];
}

template <class Op>
__global__ __launch_bounds__(256) void k_sym_reduce(const PairArgs a, const SymArgs g) {
    const int s = blockIdx.x * 256 + threadIdx.x;
    if (s >= g.n) return;
    double v[4];
    sym_acc_load<4>(g, s, v);
    sym_gather<4, double, float>(g, s, v, false);
    if (g.last) write_result<Op>(a, s, particle_of(a.tgt, s, a.P.n, a.flags), v);
    else sym_acc_store<4>(g, s, v);
}

// ---- FP64 -----------------------------------------------------------------------------------
// The same walk with every pair in FP64: the set in its own order (no near / far split, so no
// sort), the columns staged from the FP64 pack (double4 (x, y, z, G m) [+ (ax, ay, az, 0)]),
// FP64 row sums, FP64 column accumulators moved by two DPP moves each, FP64 partials (3
// components, no magnitude estimate: the FP64 pass has no fix-up).

__device__ __forceinline__ double rol1d(double x) {
    const int2 v = __builtin_bit_cast(int2, x);
    return __builtin_bit_cast(double, make_int2(__builtin_amdgcn_mov_dpp(v.x, 0x134, 0xf, 0xf, true),
                                                __builtin_amdgcn_mov_dpp(v.y, 0x134, 0xf, 0xf, true)));
}

struct Sym64Acc {
    static constexpr int kPlanes = 2;  // (x, y), (z, G m)
    struct Row { double x, y, z, gm; };
    __device__ static void load_row(const SymArgs& g, int s, bool live, Row& t) {
        if (live) {
            const double4 p = static_cast<const double4*>(g.row_pack)[s];
            t.x = p.x; t.y = p.y; t.z = p.z; t.gm = p.w;
        } else {
            t.x = t.y = t.z = kFarAway; t.gm = 0.0;
        }
    }
    __device__ static uint4 stage_elem(const SymArgs& g, int plane, int s, bool ok) {
        if (ok) return static_cast<const uint4*>(g.near_pack)[2 * s + plane];
        return __builtin_bit_cast(uint4, plane == 0 ? make_double2(kFarAway, kFarAway) : make_double2(kFarAway, 0.0));
    }
    template <bool MASK>
    __device__ static void pair(double (&r)[3], double (&c)[3], const Row& t, const uint4* pl, int j, double eps2t,
                                bool ok) {
        const double2 xy = __builtin_bit_cast(double2, pl[j]);
        const double2 zw = __builtin_bit_cast(double2, pl[kPlaneLen + j]);
        const double dx = xy.x - t.x, dy = xy.y - t.y, dz = zw.x - t.z;
        const double r2 = __builtin_fma(dx, dx, __builtin_fma(dy, dy, __builtin_fma(dz, dz, eps2t)));
        double ri = rsqrt64(r2);
        if (MASK) ri = ok ? ri : 0.0;
        const double ri3 = (ri * ri) * ri;
        const double wj = zw.y * ri3, wi = t.gm * ri3;
        r[0] = __builtin_fma(wj, dx, r[0]);
        r[1] = __builtin_fma(wj, dy, r[1]);
        r[2] = __builtin_fma(wj, dz, r[2]);
        c[0] = wi * dx; c[1] = wi * dy; c[2] = wi * dz;
    }
};

struct Sym64Grad {
    static constexpr int kPlanes = 4;  // (x, y), (z, G m), (ax, ay), (az, 0)
    struct Row { double x, y, z, gm, ax, ay, az; };
    __device__ static void load_row(const SymArgs& g, int s, bool live, Row& t) {
        if (live) {
            const double4* pk = static_cast<const double4*>(g.row_pack);
            const double4 p = pk[2 * s], a = pk[2 * s + 1];
            t.x = p.x; t.y = p.y; t.z = p.z; t.gm = p.w;
            t.ax = a.x; t.ay = a.y; t.az = a.z;
        } else {
            t.x = t.y = t.z = kFarAway; t.gm = 0.0;
            t.ax = t.ay = t.az = 0.0;
        }
    }
    __device__ static uint4 stage_elem(const SymArgs& g, int plane, int s, bool ok) {
        if (ok) return static_cast<const uint4*>(g.near_pack)[4 * s + plane];
        if (plane == 0) return __builtin_bit_cast(uint4, make_double2(kFarAway, kFarAway));
        if (plane == 1) return __builtin_bit_cast(uint4, make_double2(kFarAway, 0.0));
        return make_uint4(0u, 0u, 0u, 0u);
    }
    template <bool MASK>
    __device__ static void pair(double (&r)[3], double (&c)[3], const Row& t, const uint4* pl, int j, double eps2t,
                                bool ok) {
        const double2 xy = __builtin_bit_cast(double2, pl[j]);
        const double2 zw = __builtin_bit_cast(double2, pl[kPlaneLen + j]);
        const double2 axy = __builtin_bit_cast(double2, pl[2 * kPlaneLen + j]);
        const double2 az0 = __builtin_bit_cast(double2, pl[3 * kPlaneLen + j]);
        const double dx = xy.x - t.x, dy = xy.y - t.y, dz = zw.x - t.z;
        const double r2 = __builtin_fma(dx, dx, __builtin_fma(dy, dy, __builtin_fma(dz, dz, eps2t)));
        double ri = rsqrt64(r2);
        if (MASK) ri = ok ? ri : 0.0;
        const double ri2 = ri * ri;
        const double ri3 = ri2 * ri;
        const double dax = axy.x - t.ax, day = axy.y - t.ay, daz = az0.x - t.az;
        const double q = __builtin_fma(dax, dx, __builtin_fma(day, dy, daz * dz));
        const double sq = (-3.0 * q) * ri2;
        const double ux = __builtin_fma(sq, dx, dax), uy = __builtin_fma(sq, dy, day), uz = __builtin_fma(sq, dz, daz);
        const double wj = zw.y * ri3, wi = t.gm * ri3;
        r[0] = __builtin_fma(wj, ux, r[0]);
        r[1] = __builtin_fma(wj, uy, r[1]);
        r[2] = __builtin_fma(wj, uz, r[2]);
        c[0] = wi * ux; c[1] = wi * uy; c[2] = wi * uz;
    }
};

template <class S, int W, int R>
__global__ __launch_bounds__(64 * W) void k_pairs_sym64(const SymArgs g, double eps2t) {
    static_assert(W * R == kSymBlockTiles, "a workgroup covers one block");
    constexpr int NPL = S::kPlanes;
    __shared__ uint4 colbuf[2][NPL * kPlaneLen];
    __shared__ double xch[2][W][3][64];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int wg = blockIdx.x % g.n_blocks, chunk = g.chunk0 + (int)(blockIdx.x / g.n_blocks);
    const int d0 = chunk * g.chunk_len, d1 = d0 + g.chunk_len;
    const int rbase = wg * (W * R) + wave * R;
    typename S::Row row[R];
    bool tile_live[R];
    int rs[R];
    double own[R][3];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        tile_live[r] = rbase + r < g.n_row_tiles;
        rs[r] = (rbase + r) * 64 + lane;
        S::load_row(g, rs[r], tile_live[r] && rs[r] < g.n_rows, row[r]);
        own[r][0] = own[r][1] = own[r][2] = 0.0;
    }
    constexpr int SPT = (NPL + W - 1) / W;
    const int st_k = threadIdx.x & 63;
    TileWalk cur, pre;
    cur.d = d0;
    cur.d_end = d1;
    cur.next(g, wg);
    pre = cur;
    pre.next(g, wg);
    uint4 held[SPT];
#pragma unroll
    for (int u = 0; u < SPT; ++u) {
        const int pl = wave + W * u;
        if (pl < NPL && cur.ct >= 0) {
            const int s = cur.ct * 64 + st_k;
            const uint4 e = S::stage_elem(g, pl, s, s < g.n);
            colbuf[0][pl * kPlaneLen + st_k] = e;
            colbuf[0][pl * kPlaneLen + st_k + 64] = e;
        }
        held[u] = make_uint4(0u, 0u, 0u, 0u);
        if (pl < NPL && pre.ct >= 0) {
            const int s = pre.ct * 64 + st_k;
            held[u] = S::stage_elem(g, pl, s, s < g.n);
        }
    }
    __syncthreads();
    for (int i = 0; cur.ct >= 0; ++i) {
        const int buf = i & 1;
        const int ct = cur.ct;
        const uint4* pls = colbuf[buf];
        int mode[R];
        bool any = false, masked = false;
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int rt = rbase + r;
            mode[r] = !tile_live[r] ? kSkip : (cur.d > 0 || ct > rt) ? kFull : ct == rt ? kDiag : kSkip;
            any = any || mode[r] != kSkip;
            masked = masked || mode[r] != kFull;
        }
        double ja[3] = {0.0, 0.0, 0.0};  // accumulator of column (lane + k) mod 64 after step k
        if (any) {
            if (masked) {
                for (int k = 0; k < 64; ++k) {
                    double cs[3] = {0.0, 0.0, 0.0};
#pragma unroll
                    for (int r = 0; r < R; ++r) {
                        double cv[3];
                        S::template pair<true>(own[r], cv, row[r], pls, lane + k, eps2t, counts(mode[r], lane, k));
#pragma unroll
                        for (int q = 0; q < 3; ++q) cs[q] += cv[q];
                    }
#pragma unroll
                    for (int q = 0; q < 3; ++q) ja[q] = rol1d(ja[q]) + cs[q];
                }
            } else {
#pragma unroll 2
                for (int k = 0; k < 64; ++k) {
                    double cs[3];
#pragma unroll
                    for (int r = 0; r < R; ++r) {
                        double cv[3];
                        S::template pair<false>(own[r], cv, row[r], pls, lane + k, eps2t, true);
#pragma unroll
                        for (int q = 0; q < 3; ++q) cs[q] = r == 0 ? cv[q] : cs[q] + cv[q];
                    }
#pragma unroll
                    for (int q = 0; q < 3; ++q) ja[q] = rol1d(ja[q]) + cs[q];
                }
            }
        }
        const int slot = any ? (lane + 63) & 63 : lane;
#pragma unroll
        for (int q = 0; q < 3; ++q) xch[buf][wave][q][slot] = ja[q];
#pragma unroll
        for (int u = 0; u < SPT; ++u) {
            const int pl = wave + W * u;
            if (pl < NPL && pre.ct >= 0) {
                colbuf[buf ^ 1][pl * kPlaneLen + st_k] = held[u];
                colbuf[buf ^ 1][pl * kPlaneLen + st_k + 64] = held[u];
            }
        }
        __syncthreads();
        if (threadIdx.x < 3 * 64) {
            const int q = threadIdx.x >> 6, k = threadIdx.x & 63;
            double s = 0.0;
#pragma unroll
            for (int v = 0; v < W; ++v) s += xch[buf][v][q][k];
            const int col = ct * 64 + k;
            if (col < g.n) reinterpret_cast<double*>(g.part)[((size_t)(cur.d - g.d_base) * 3 + q) * g.n_pad + col] = -s;
        }
        cur = pre;
        pre.next(g, wg);
#pragma unroll
        for (int u = 0; u < SPT; ++u) {
            const int pl = wave + W * u;
            if (pl < NPL && pre.ct >= 0) {
                const int s = pre.ct * 64 + st_k;
                held[u] = S::stage_elem(g, pl, s, s < g.n);
            }
        }
    }
#pragma unroll
    for (int r = 0; r < R; ++r) {
        if (tile_live[r] && rs[r] < g.n_rows) {
            double* o = g.own + (size_t)(chunk - g.chunk0) * 3 * g.n_row_pad;
#pragma unroll
            for (int q = 0; q < 3; ++q) o[(size_t)q * g.n_row_pad + rs[r]] = own[r][q];
        }
    }
}

template <class Op>
__global__ __launch_bounds__(256) void k_sym_reduce64(const PairArgs a, const SymArgs g) {
    const int s = blockIdx.x * 256 + threadIdx.x;
    if (s >= g.n) return;
    double v[3];
    sym_acc_load<3>(g, s, v);
    sym_gather<3, double, double>(g, s, v, false);
    if (g.last) write_result<Op>(a, s, particle_of(a.tgt, s, a.P.n, a.flags), v);
    else sym_acc_store<3>(g, s, v);
}

// Two sets: threads [0, n_rows) finish the rows (sums over the shares), threads [n_rows,
// n_rows + n) the columns (sums over the row blocks, with the opposite sign for the terms).
template <class Op>
__global__ __launch_bounds__(256) void k_between_reduce(const PairArgs ar, const PairArgs ac, const SymArgs g) {
    const int t = blockIdx.x * 256 + threadIdx.x;
    double v[4] = {0.0, 0.0, 0.0, 0.0};
    if (t < g.n_rows) {
        for (int c = 0; c < g.n_chunks; ++c) {
#pragma unroll
            for (int q = 0; q < 4; ++q) v[q] += g.own[((size_t)c * 4 + q) * g.n_row_pad + t];
        }
        write_result<Op>(ar, t, particle_of(ar.tgt, t, ar.P.n, ar.flags), v);
    } else if (t < g.n_rows + g.n) {
        const int s = t - g.n_rows;
        for (int w = 0; w < g.n_blocks; ++w) {
#pragma unroll
            for (int q = 0; q < 4; ++q) v[q] += (double)g.part[((size_t)w * 4 + q) * g.n_pad + s];
        }
        write_result<Op>(ac, s, particle_of(ac.tgt, s, ac.P.n, ac.flags), v);
    }
}


// ---- the time-step rates ---------------------------------------------------------------------
// The pairwise free-fall and fly-by rates (Sec. 3.5.3, Eqs. dt-freefall and dt-flyby):
//   W_ff = G (m_i + m_j) / r^3,   W_fb = |v_ij|^2 / r^2,
// are the same number for i and for j, so one evaluation of an unordered pair serves the row
// maximum and the column maximum.  The walk is the one above, the set in its own order (no
// sort), the columns staged from the time-step pack (double4 (x, y, z, [G m]), double4 (vx, vy,
// vz, particle index)).  FP64 differences rounded once to FP32 and FP32 rates, with the same
// operations as the directed mixed pass, so a pair gives the same FP32 rates in either
// orientation.  A maximum is exact in any order, so the row maxima, the column accumulators
// (moved by DPP, as above) and the partials all stay FP32.
// A rate has no cancellation: its FP32 value is good to a few units of rounding unless it
// overflows (pairs closer than about (G m)^(1/3) 1e-13) or r = 0.  A wavefront whose tile
// produced a non-finite maximum evaluates that tile again in FP64, drops its FP32 values and
// puts the FP64 maxima of its rows and columns into hi (64-bit atomic maximum on the bit
// patterns: the rates are >= 0, so their order is that of the integers); a pair at r = 0 in
// FP64 is left out and flagged.  (A NaN rate, from 0 * inf, is dropped by the maximum: a
// coincident pair of massless particles with equal velocities adds nothing and may go
// unflagged.)  Self-pairs (diagonal tiles) and the fillers past the last particle are masked out.

struct DtRow { double x, y, z, vx, vy, vz; float gm; int pi; };

__device__ __forceinline__ void dt_load_row(const SymArgs& g, int s, bool live, DtRow& t) {
    if (live) {
        const double4* pk = static_cast<const double4*>(g.row_pack);
        const double4 p = pk[2 * s], v = pk[2 * s + 1];
        t.x = p.x; t.y = p.y; t.z = p.z; t.gm = unpack_gm(p.w);
        t.vx = v.x; t.vy = v.y; t.vz = v.z; t.pi = (int)v.w;
    } else {
        t.x = t.y = t.z = 0.0; t.gm = 0.f;
        t.vx = t.vy = t.vz = 0.0; t.pi = -1;
    }
}

// planes: (x, y), (z, [G m]), (vx, vy), (vz, index) of the pack; zeros past the last particle
__device__ __forceinline__ uint4 dt_stage_elem(const SymArgs& g, int plane, int s, bool ok) {
    return ok ? static_cast<const uint4*>(g.near_pack)[4 * s + plane] : make_uint4(0u, 0u, 0u, 0u);
}

// One pair in FP32: maxima of the row (r) and the column terms (c).  MASK: a pair that does not
// count (ok false) gives zero rates.
template <bool MASK>
__device__ __forceinline__ void dt_pair(float (&r)[2], float (&c)[2], const DtRow& t, const uint4* pl, int j,
                                        bool ok) {
    const double2 xy = __builtin_bit_cast(double2, pl[j]);
    const double2 zw = __builtin_bit_cast(double2, pl[kPlaneLen + j]);
    const double2 vxy = __builtin_bit_cast(double2, pl[2 * kPlaneLen + j]);
    const double2 vz = __builtin_bit_cast(double2, pl[3 * kPlaneLen + j]);
    const float dx = dif32(xy.x, t.x), dy = dif32(xy.y, t.y), dz = dif32(zw.x, t.z);
    const float ux = dif32(vxy.x, t.vx), uy = dif32(vxy.y, t.vy), uz = dif32(vz.x, t.vz);
    const float r2 = __builtin_fmaf(dx, dx, __builtin_fmaf(dy, dy, dz * dz));
    const float u2 = __builtin_fmaf(ux, ux, __builtin_fmaf(uy, uy, uz * uz));
    float ri = rsqrt32(r2);
    if (MASK) ri = ok ? ri : 0.f;
    const float ri2 = ri * ri;
    const float fb = u2 * ri2;
    const float ff = ((unpack_gm(zw.y) + t.gm) * ri2) * ri;
    r[0] = fmaxf(r[0], ff);
    r[1] = fmaxf(r[1], fb);
    c[0] = ff;
    c[1] = fb;
}

__device__ __forceinline__ void max_bits(double* p, double v) {
    atomicMax(reinterpret_cast<unsigned long long*>(p), (unsigned long long)__double_as_longlong(v));
}

// The wavefront's tile again in FP64 (rare): row and column maxima into hi, one row tile at a
// time (few registers).  Masses from g.m (the particle indices ride in the pack).
template <int R>
__device__ __forceinline__ void dt_redo(const SymArgs& g, int ct, const int (&mode)[R], const bool (&rok)[R],
                                        const int (&rs)[R], const DtRow (&row)[R], const uint4* pl) {
    const int lane = threadIdx.x & 63;
    double cmax[2] = {0.0, 0.0};  // column (lane + 63) mod 64, over the row tiles
#pragma unroll
    for (int r = 0; r < R; ++r) {
        if (mode[r] == kSkip) continue;  // uniform over the wavefront
        const double mi = rok[r] ? g.m[row[r].pi] : 0.0;
        double rmax[2] = {0.0, 0.0}, acc[2] = {0.0, 0.0};
        for (int k = 0; k < 64; ++k) {
            const int j = lane + k;
            double ff = 0.0, fb = 0.0;
            if (rok[r] && ct * 64 + (j & 63) < g.n && counts(mode[r], lane, k)) {
                const double2 xy = __builtin_bit_cast(double2, pl[j]);
                const double2 zw = __builtin_bit_cast(double2, pl[kPlaneLen + j]);
                const double dx = xy.x - row[r].x, dy = xy.y - row[r].y, dz = zw.x - row[r].z;
                const double r2 = dx * dx + dy * dy + dz * dz;
                if (r2 == 0.0) {
                    atomicOr(g.flags, BF_FLAG_COINCIDENT);
                } else {
                    const double2 vxy = __builtin_bit_cast(double2, pl[2 * kPlaneLen + j]);
                    const double2 vz = __builtin_bit_cast(double2, pl[3 * kPlaneLen + j]);
                    const double ux = vxy.x - row[r].vx, uy = vxy.y - row[r].vy, uz = vz.x - row[r].vz;
                    const double ri = rsqrt64(r2);
                    fb = (ux * ux + uy * uy + uz * uz) * ri * ri;
                    ff = g.G * (mi + g.m[(int)vz.y]) * ri * ri * ri;
                }
            }
            rmax[0] = fmax(rmax[0], ff);
            rmax[1] = fmax(rmax[1], fb);
            acc[0] = fmax(rol1d(acc[0]), ff);
            acc[1] = fmax(rol1d(acc[1]), fb);
        }
        if (rok[r]) {
            max_bits(g.hi + rs[r], rmax[0]);
            max_bits(g.hi + g.n_pad + rs[r], rmax[1]);
        }
        cmax[0] = fmax(cmax[0], acc[0]);
        cmax[1] = fmax(cmax[1], acc[1]);
    }
    const int col = ct * 64 + ((lane + 63) & 63);
    if (col < g.n) {
        max_bits(g.hi + col, cmax[0]);
        max_bits(g.hi + g.n_pad + col, cmax[1]);
    }
}

template <int W, int R>
__global__ __launch_bounds__(64 * W) void k_pairs_symdt(const SymArgs g) {
    static_assert(W * R == kSymBlockTiles, "a workgroup covers one block");
    constexpr int NPL = 4;
    __shared__ uint4 colbuf[2][NPL * kPlaneLen];
    __shared__ float xch[2][W][2][64];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int wg = blockIdx.x % g.n_blocks, chunk = g.chunk0 + (int)(blockIdx.x / g.n_blocks);
    const int d0 = chunk * g.chunk_len, d1 = d0 + g.chunk_len;
    const int rbase = wg * (W * R) + wave * R;
    DtRow row[R];
    bool tile_live[R], rok[R], ragged_rows = false;
    int rs[R];
    float own[R][2];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        tile_live[r] = rbase + r < g.n_row_tiles;
        rs[r] = (rbase + r) * 64 + lane;
        rok[r] = tile_live[r] && rs[r] < g.n_rows;
        ragged_rows = ragged_rows || (tile_live[r] && (rbase + r + 1) * 64 > g.n_rows);
        dt_load_row(g, rs[r], rok[r], row[r]);
        own[r][0] = own[r][1] = 0.f;
    }
    constexpr int SPT = (NPL + W - 1) / W;
    const int st_k = threadIdx.x & 63;
    TileWalk cur, pre;
    cur.d = d0;
    cur.d_end = d1;
    cur.next(g, wg);
    pre = cur;
    pre.next(g, wg);
    uint4 held[SPT];
#pragma unroll
    for (int u = 0; u < SPT; ++u) {
        const int pl = wave + W * u;
        if (pl < NPL && cur.ct >= 0) {
            const int s = cur.ct * 64 + st_k;
            const uint4 e = dt_stage_elem(g, pl, s, s < g.n);
            colbuf[0][pl * kPlaneLen + st_k] = e;
            colbuf[0][pl * kPlaneLen + st_k + 64] = e;
        }
        held[u] = make_uint4(0u, 0u, 0u, 0u);
        if (pl < NPL && pre.ct >= 0) {
            const int s = pre.ct * 64 + st_k;
            held[u] = dt_stage_elem(g, pl, s, s < g.n);
        }
    }
    __syncthreads();
    for (int i = 0; cur.ct >= 0; ++i) {
        const int buf = i & 1;
        const int ct = cur.ct;
        const uint4* pls = colbuf[buf];
        int mode[R];
        bool any = false;
        bool masked = ragged_rows || (ct + 1) * 64 > g.n;  // fillers among the rows or the columns
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int rt = rbase + r;
            mode[r] = !tile_live[r] ? kSkip : (cur.d > 0 || ct > rt) ? kFull : ct == rt ? kDiag : kSkip;
            any = any || mode[r] != kSkip;
            masked = masked || mode[r] != kFull;
        }
        float ja[2] = {0.f, 0.f};  // accumulator of column (lane + k) mod 64 after step k
        if (any) {
            float part[R][2];
#pragma unroll
            for (int r = 0; r < R; ++r) part[r][0] = part[r][1] = 0.f;
            if (masked) {
                for (int k = 0; k < 64; ++k) {
                    float cs[2] = {0.f, 0.f};
#pragma unroll
                    for (int r = 0; r < R; ++r) {
                        float cv[2];
                        const bool ok = rok[r] && ct * 64 + ((lane + k) & 63) < g.n && counts(mode[r], lane, k);
                        dt_pair<true>(part[r], cv, row[r], pls, lane + k, ok);
                        cs[0] = fmaxf(cs[0], cv[0]);
                        cs[1] = fmaxf(cs[1], cv[1]);
                    }
                    ja[0] = fmaxf(rol1(ja[0]), cs[0]);
                    ja[1] = fmaxf(rol1(ja[1]), cs[1]);
                }
            } else {
#pragma unroll 2
                for (int k = 0; k < 64; ++k) {
                    float cs[2];
#pragma unroll
                    for (int r = 0; r < R; ++r) {
                        float cv[2];
                        dt_pair<false>(part[r], cv, row[r], pls, lane + k, true);
                        cs[0] = r == 0 ? cv[0] : fmaxf(cs[0], cv[0]);
                        cs[1] = r == 0 ? cv[1] : fmaxf(cs[1], cv[1]);
                    }
                    ja[0] = fmaxf(rol1(ja[0]), cs[0]);
                    ja[1] = fmaxf(rol1(ja[1]), cs[1]);
                }
            }
            // non-finite maxima (overflow, r = 0): the tile again in FP64
            float top = fmaxf(ja[0], ja[1]);
#pragma unroll
            for (int r = 0; r < R; ++r) top = fmaxf(top, fmaxf(part[r][0], part[r][1]));
            if (__any(!(top < __builtin_huge_valf()))) {
                dt_redo<R>(g, ct, mode, rok, rs, row, pls);
                ja[0] = ja[1] = 0.f;
            } else {
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    own[r][0] = fmaxf(own[r][0], part[r][0]);
                    own[r][1] = fmaxf(own[r][1], part[r][1]);
                }
            }
        }
        const int slot = any ? (lane + 63) & 63 : lane;
        xch[buf][wave][0][slot] = ja[0];
        xch[buf][wave][1][slot] = ja[1];
#pragma unroll
        for (int u = 0; u < SPT; ++u) {
            const int pl = wave + W * u;
            if (pl < NPL && pre.ct >= 0) {
                colbuf[buf ^ 1][pl * kPlaneLen + st_k] = held[u];
                colbuf[buf ^ 1][pl * kPlaneLen + st_k + 64] = held[u];
            }
        }
        __syncthreads();
        if (threadIdx.x < 2 * 64) {
            const int q = threadIdx.x >> 6, k = threadIdx.x & 63;
            float s = 0.f;
#pragma unroll
            for (int v = 0; v < W; ++v) s = fmaxf(s, xch[buf][v][q][k]);
            const int col = ct * 64 + k;
            if (col < g.n) g.part[((size_t)(cur.d - g.d_base) * 2 + q) * g.n_pad + col] = s;
        }
        cur = pre;
        pre.next(g, wg);
#pragma unroll
        for (int u = 0; u < SPT; ++u) {
            const int pl = wave + W * u;
            if (pl < NPL && pre.ct >= 0) {
                const int s = pre.ct * 64 + st_k;
                held[u] = dt_stage_elem(g, pl, s, s < g.n);
            }
        }
    }
    float* o = reinterpret_cast<float*>(g.own) + (size_t)(chunk - g.chunk0) * 2 * g.n_row_pad;
#pragma unroll
    for (int r = 0; r < R; ++r) {
        if (rok[r]) {
            o[rs[r]] = own[r][0];
            o[(size_t)g.n_row_pad + rs[r]] = own[r][1];
        }
    }
}

__global__ __launch_bounds__(256) void k_symdt_clear(double* hi, int n) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i < n) hi[i] = 0.0;
}

__global__ __launch_bounds__(256) void k_symdt_reduce(const PairArgs a, const SymArgs g) {
    const int s = blockIdx.x * 256 + threadIdx.x;
    if (s >= g.n) return;
    float v[2];
    sym_acc_load<2>(g, s, v);
    sym_gather<2, float, float>(g, s, v, true);
    if (!g.last) {
        sym_acc_store<2>(g, s, v);
        return;
    }
    const double w[2] = {fmax((double)v[0], g.hi[s]), fmax((double)v[1], g.hi[g.n_pad + s])};
    write_result<DtMixed>(a, s, particle_of(a.tgt, s, a.P.n, a.flags), w);
}
}  // namespace

size_t between_scratch_bytes(int64_t n_rows, int64_t n_cols, int chunks) {
    const int64_t row_tiles = (n_rows + 63) / 64, col_tiles = (n_cols + 63) / 64;
    const int64_t nb = (row_tiles + kSymBlockTiles - 1) / kSymBlockTiles;
    return sym_own_bytes(n_rows, chunks) + (size_t)nb * 4 * 64 * col_tiles * sizeof(float);
}

hipError_t launch_between_reduce(int op, const PairArgs& ar, const PairArgs& ac, const SymArgs& g, hipStream_t st) {
    const int64_t n = (int64_t)g.n_rows + g.n;
    if (n <= 0) return hipSuccess;
    const dim3 grid((unsigned)((n + 255) / 256));
    if (op == OP_ACC) hipLaunchKernelGGL(k_between_reduce<AccMixed>, grid, dim3(256), 0, st, ar, ac, g);
    else if (op == OP_GRAD) hipLaunchKernelGGL(k_between_reduce<GradMixed>, grid, dim3(256), 0, st, ar, ac, g);
    else return hipErrorInvalidValue;
    return hipGetLastError();
}

size_t sym_own_bytes(int64_t n, int chunks) {
    return ((size_t)chunks * 4 * 64 * ((n + 63) / 64) * sizeof(double) + 255) & ~size_t(255);
}


// Launch shapes.  Defaults, measured at N = 2^20: 8 wavefronts of 2 row tiles for the
// acceleration, 4 of 4 for the gradient (more row tiles per lane share each column read and
// rotation; fewer fit the VGPRs); 8 of 2 for the time-step rates (341 ms against 349 ms with 4
// of 4 and 472 ms with 16 of 1).  The other shapes (W wavefronts of R row tiles, W R =
// kSymBlockTiles) are there for the autotuner and for forced configurations.
constexpr int kAccWaves = 8, kAccRows = 2, kGradWaves = 4, kGradRows = 4, kDtWaves = 8, kDtRows = 2;
int sym_default_waves(int op) { return op == OP_ACC ? kAccWaves : op == OP_GRAD ? kGradWaves : kDtWaves; }
int sym_default_rows(int op) { return op == OP_ACC ? kAccRows : op == OP_GRAD ? kGradRows : kDtRows; }

using SymKernel = void (*)(const SymArgs);

static SymKernel sym_kernel(int op, int waves, int rows) {
#define BF_SYM(S, W, R) \
    if (waves == W && rows == R) return k_pairs_sym<S, W, R>;
    if (op == OP_ACC) { BF_SYM(SymAcc, 16, 1) BF_SYM(SymAcc, 8, 2) BF_SYM(SymAcc, 4, 4) }
    if (op == OP_GRAD) { BF_SYM(SymGrad, 16, 1) BF_SYM(SymGrad, 8, 2) BF_SYM(SymGrad, 4, 4) }
#undef BF_SYM
    if (op == OP_DT) {
        if (waves == 16 && rows == 1) return k_pairs_symdt<16, 1>;
        if (waves == 8 && rows == 2) return k_pairs_symdt<8, 2>;
        if (waves == 4 && rows == 4) return k_pairs_symdt<4, 4>;
    }
    return nullptr;
}

bool sym_variant_exists(int op, int waves, int rows) { return sym_kernel(op, waves, rows) != nullptr; }

int sym_blocks_per_cu(int op, int waves, int rows) {
    const SymKernel f = sym_kernel(op, waves, rows);
    if (!f) return 1;
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, reinterpret_cast<const void*>(f), 64 * waves, 0) !=
        hipSuccess)
        return 1;
    return nb > 0 ? nb : 1;
}

hipError_t launch_pairs_sym(int op, int waves, int rows, const SymArgs& g, hipStream_t st) {
    if (g.n <= 0) return hipSuccess;
    const SymKernel f = sym_kernel(op, waves, rows);
    if (!f) return hipErrorInvalidValue;
    if (op == OP_DT && g.first) {  // the FP64 maxima of re-evaluated tiles start at zero (a fill kernel: capturable)
        const int nh = 2 * g.n_pad;
        hipLaunchKernelGGL(k_symdt_clear, dim3((nh + 255) / 256), dim3(256), 0, st, g.hi, nh);
    }
    const dim3 grid((unsigned)g.n_blocks * (unsigned)(g.between ? g.n_chunks : g.pass_chunks));
    hipLaunchKernelGGL(f, grid, dim3(64 * waves), 0, st, g);
    return hipGetLastError();
}

// FP64: 4 wavefronts of 4 row tiles for both passes
constexpr int kSym64Waves = 4, kSym64Rows = 4;

int sym64_blocks_per_cu(int op) {
    const void* f = op == OP_ACC ? reinterpret_cast<const void*>(k_pairs_sym64<Sym64Acc, kSym64Waves, kSym64Rows>)
                                 : reinterpret_cast<const void*>(k_pairs_sym64<Sym64Grad, kSym64Waves, kSym64Rows>);
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, f, 64 * kSym64Waves, 0) != hipSuccess) return 1;
    return nb > 0 ? nb : 1;
}

hipError_t launch_pairs_sym64(int op, const SymArgs& g, double eps2t, hipStream_t st) {
    if (g.n <= 0) return hipSuccess;
    const dim3 grid((unsigned)g.n_blocks * (unsigned)g.pass_chunks);
    if (op == OP_ACC)
        hipLaunchKernelGGL((k_pairs_sym64<Sym64Acc, kSym64Waves, kSym64Rows>), grid, dim3(64 * kSym64Waves), 0, st, g, eps2t);
    else if (op == OP_GRAD)
        hipLaunchKernelGGL((k_pairs_sym64<Sym64Grad, kSym64Waves, kSym64Rows>), grid, dim3(64 * kSym64Waves), 0, st, g, eps2t);
    else return hipErrorInvalidValue;
    return hipGetLastError();
}

hipError_t launch_sym_reduce64(int op, const PairArgs& a, const SymArgs& g, hipStream_t st) {
    if (g.n <= 0) return hipSuccess;
    const dim3 grid((g.n + 255) / 256);
    if (op == OP_ACC) hipLaunchKernelGGL(k_sym_reduce64<Acc64>, grid, dim3(256), 0, st, a, g);
    else if (op == OP_GRAD) hipLaunchKernelGGL(k_sym_reduce64<Grad64>, grid, dim3(256), 0, st, a, g);
    else return hipErrorInvalidValue;
    return hipGetLastError();
}

hipError_t launch_sym_reduce(int op, const PairArgs& a, const SymArgs& g, hipStream_t st) {
    if (g.n <= 0) return hipSuccess;
    const dim3 grid((g.n + 255) / 256);
    if (op == OP_ACC) hipLaunchKernelGGL(k_sym_reduce<AccMixed>, grid, dim3(256), 0, st, a, g);
    else if (op == OP_GRAD) hipLaunchKernelGGL(k_sym_reduce<GradMixed>, grid, dim3(256), 0, st, a, g);
    else if (op == OP_DT) hipLaunchKernelGGL(k_symdt_reduce, grid, dim3(256), 0, st, a, g);
    else return hipErrorInvalidValue;
    return hipGetLastError();
}

}  // namespace bf
