// Direct-summation pair kernels for gfx950: Newtonian acceleration, force gradient and the
// pairwise time-step maxima, each in a mixed and an FP64 flavour, sharing one tiled skeleton.
//
// Skeleton (one workgroup = W wavefronts):
//  * the workgroup owns a slab of 64*K*W target slots (K per lane, lane-strided) and one of
//    `split` chunks of the source list; block b takes chunk b % split, so with split = 8 all
//    workgroups on one XCD (dispatch is round-robin over the 8 XCDs) stream the same chunk
//    and it stays in that XCD's L2;
//  * sources are staged tile by tile (64*W per tile, one per thread) from a packed stream into
//    LDS; every lane then walks the tile with a broadcast LDS read per source and updates its
//    K targets in registers;
//  * mixed precision (pair_ops.h): FP64 differences rounded once to FP32, FP32 arithmetic,
//    per-tile FP32 partials merged into FP64, optional FP64 re-evaluation of tiles holding
//    close pairs, and an FP64 fix-up of targets whose result cancels strongly;
//  * results go straight to the particle-indexed outputs (split == 1) or to per-chunk
//    partials that a second kernel reduces in chunk order (deterministic).
#include "pair_ops.h"

namespace bf {

template <class Op>
__device__ __forceinline__ void emit(const PairArgs& a, int c, int slot, int pi, const typename Op::A64& acc) {
    constexpr int NP = ncomp_of<Op>();
    double v[NP];
    Op::comps(acc, v);
    if (a.split == 1) {
        write_result<Op>(a, slot, pi, v);
    } else {
        const int nt = a.tgt.count;
#pragma unroll
        for (int comp = 0; comp < NP; ++comp) a.part[((size_t)c * NP + comp) * nt + slot] = v[comp];
    }
}

// ---- the skeleton --------------------------------------------------------------------------

template <class Op, int K, int W, bool DETECT, bool EXCL = false>
__global__ __launch_bounds__(64 * W) void k_pairs(const PairArgs a) {
    __shared__ typename Op::Src tile[64 * W];
    __shared__ int32_t tsub[EXCL ? 64 * W : 1];
    const int wave = threadIdx.x >> 6;
    const int c = blockIdx.x % a.split;
    const int slab = blockIdx.x / a.split;
    const int tbase = slab * (64 * K * W) + wave * (64 * K);
    const int j0 = c * a.chunk;
    const int j1 = min(a.src.count, j0 + a.chunk);
    typename Op::A64 acc[K];
    int slot[K], pidx[K];
    sweep<Op, K, W, DETECT, EXCL>(a, tile, tbase, j0, j1, acc, slot, pidx, tsub);
#pragma unroll
    for (int k = 0; k < K; ++k)
        if (slot[k] < a.tgt.count) emit<Op>(a, c, slot[k], pidx[k], acc[k]);
}

// ---- small passes: one launch, no partials in memory ----------------------------------------
// A workgroup of kSmallWaves wavefronts takes kSmallT targets.  Wavefront w sweeps the w-th
// slice of the sources in tiles of 64 staged in its own LDS region; within a wavefront lane
// (t, g) = (lane % kSmallT, lane / kSmallT) pairs target t with entries [16 g, 16 g + 16) of
// each tile (so an FP32 partial spans 16 sources, folded into FP64 after every tile).  At the
// end the workgroup adds the 16 x 4 FP64 sums of each target in a fixed order (wavefront,
// then lane group) and writes the result with the cancellation check, as the split kernels'
// reduction does.  All wavefronts take the same number of tile steps, so the barriers are
// uniform.
constexpr int kSmallWaves = 16, kSmallG = 4, kSmallT = 64 / kSmallG;

template <class Op>
__global__ __launch_bounds__(64 * kSmallWaves) void k_pairs_small(const PairArgs a) {
    constexpr int NP = ncomp_of<Op>();
    constexpr int kTileBytes = kSmallWaves * 64 * (int)sizeof(typename Op::Src);
    constexpr int kRedBytes = kSmallWaves * kSmallG * NP * kSmallT * (int)sizeof(double);
    __shared__ __align__(16) unsigned char lds[kTileBytes > kRedBytes ? kTileBytes : kRedBytes];
    typename Op::Src* tile = reinterpret_cast<typename Op::Src*>(lds) + (threadIdx.x >> 6) * 64;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int t = lane % kSmallT, grp = lane / kSmallT;
    const int nt = a.tgt.count, ns = a.src.count;
    const int slot = blockIdx.x * kSmallT + t;
    const int pi = particle_of(a.tgt, slot < nt ? slot : nt - 1, a.P.n, a.flags);
    typename Op::Tgt tg;
    Op::target(a, pi, tg);
    typename Op::A64 acc;
    Op::zero(acc);
    const int per = (ns + kSmallWaves - 1) / kSmallWaves;  // sources per wavefront
    const int j0 = wave * per, j1 = min(ns, j0 + per);
    const int steps = (per + 63) / 64;  // the same for every wavefront
    for (int st = 0; st < steps; ++st) {
        const int jt = j0 + st * 64;
        const int len = min(64, j1 - jt);  // <= 0 past this wavefront's slice
        __syncthreads();
        if (lane < len) tile[lane] = Op::load(a, jt + lane);
        __syncthreads();
        const int e0 = grp * (64 / kSmallG), e1 = min(len, e0 + 64 / kSmallG);
        if (e0 < e1) {
            typename Op::A32 part;
            Op::zero(part);
#pragma unroll 2
            for (int e = e0; e < e1; ++e) Op::pair(part, tg, tile[e], a.eps2f);
            Op::fold(acc, part);
        }
    }
    double v[NP];
    Op::comps(acc, v);
    __syncthreads();  // the tiles are done with: the LDS now holds the sums
    double* red = reinterpret_cast<double*>(lds);  // [wave][group][comp][target]
#pragma unroll
    for (int c = 0; c < NP; ++c) red[((wave * kSmallG + grp) * NP + c) * kSmallT + t] = v[c];
    __syncthreads();
    if ((int)threadIdx.x < kSmallT && slot < nt) {
        double r[NP];
#pragma unroll
        for (int c = 0; c < NP; ++c) r[c] = 0.0;
#pragma unroll 4
        for (int q = 0; q < kSmallWaves * kSmallG; ++q)
#pragma unroll
            for (int c = 0; c < NP; ++c) r[c] += red[(q * NP + c) * kSmallT + t];
        write_result<Op>(a, slot, pi, r);
    }
}

// The same in FP64 for the FP64 passes: sources straight from the masters (no pack kernel),
// FP64 pairs with the FP64 kernels' tiny added to s^2, and the pass statistics cleared here (an
// FP64 pass queues no fix-up): one launch per pass.
template <class Op>
__global__ __launch_bounds__(64 * kSmallWaves) void k_pairs_small64(const PairArgs a) {
    constexpr int NP = Op::NC;
    constexpr int kTileBytes = kSmallWaves * 64 * (int)sizeof(typename Op::Src);
    constexpr int kRedBytes = kSmallWaves * kSmallG * NP * kSmallT * (int)sizeof(double);
    __shared__ __align__(16) unsigned char lds[kTileBytes > kRedBytes ? kTileBytes : kRedBytes];
    if (blockIdx.x == 0 && threadIdx.x < 3 && a.pass_stats) a.pass_stats[threadIdx.x] = 0;
    typename Op::Src* tile = reinterpret_cast<typename Op::Src*>(lds) + (threadIdx.x >> 6) * 64;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int t = lane % kSmallT, grp = lane / kSmallT;
    const int nt = a.tgt.count, ns = a.src.count;
    const int slot = blockIdx.x * kSmallT + t;
    const int pi = particle_of(a.tgt, slot < nt ? slot : nt - 1, a.P.n, a.flags);
    typename Op::Tgt tg;
    Op::target(a, pi, tg);
    typename Op::A64 acc;
    Op::zero(acc);
    const double eps2t = a.eps2 + kTiny64;
    const int per = (ns + kSmallWaves - 1) / kSmallWaves;  // sources per wavefront
    const int j0 = wave * per, j1 = min(ns, j0 + per);
    const int steps = (per + 63) / 64;  // the same for every wavefront
    for (int st = 0; st < steps; ++st) {
        const int jt = j0 + st * 64;
        const int len = min(64, j1 - jt);  // <= 0 past this wavefront's slice
        __syncthreads();
        if (lane < len) tile[lane] = Op::load_master(a, jt + lane);
        __syncthreads();
        const int e0 = grp * (64 / kSmallG), e1 = min(len, e0 + 64 / kSmallG);
#pragma unroll 2
        for (int e = e0; e < e1; ++e) Op::pair64(acc, tg, tile[e], eps2t, pi);
    }
    double v[NP];
    Op::comps(acc, v);
    __syncthreads();  // the tiles are done with: the LDS now holds the sums
    double* red = reinterpret_cast<double*>(lds);  // [wave][group][comp][target]
#pragma unroll
    for (int c = 0; c < NP; ++c) red[((wave * kSmallG + grp) * NP + c) * kSmallT + t] = v[c];
    __syncthreads();
    if ((int)threadIdx.x < kSmallT && slot < nt) {
        double r[NP];
#pragma unroll
        for (int c = 0; c < NP; ++c) r[c] = 0.0;
#pragma unroll 4
        for (int q = 0; q < kSmallWaves * kSmallG; ++q)
#pragma unroll
            for (int c = 0; c < NP; ++c) r[c] += red[(q * NP + c) * kSmallT + t];
        write_result<Op>(a, slot, pi, r);
    }
}

hipError_t launch_pairs_small64(int op, const PairArgs& a, hipStream_t st) {
    const int nt = a.tgt.count;
    if (nt <= 0) return hipSuccess;
    const dim3 grid((nt + kSmallT - 1) / kSmallT), block(64 * kSmallWaves);
    if (op == OP_ACC) hipLaunchKernelGGL(k_pairs_small64<Acc64>, grid, block, 0, st, a);
    else if (op == OP_GRAD) hipLaunchKernelGGL(k_pairs_small64<Grad64>, grid, block, 0, st, a);
    else return hipErrorInvalidValue;
    return hipGetLastError();
}

hipError_t launch_pairs_small(int op, const PairArgs& a, hipStream_t st) {
    const int nt = a.tgt.count;
    if (nt <= 0) return hipSuccess;
    const dim3 grid((nt + kSmallT - 1) / kSmallT), block(64 * kSmallWaves);
    if (op == OP_ACC) hipLaunchKernelGGL(k_pairs_small<AccMixed>, grid, block, 0, st, a);
    else if (op == OP_GRAD) hipLaunchKernelGGL(k_pairs_small<GradMixed>, grid, block, 0, st, a);
    else return hipErrorInvalidValue;
    return hipGetLastError();
}

// ---- packing the source stream -------------------------------------------------------------

// begin > 0: this launch also starts the pass (the three pass statistics; begin == 2: and the
// fix-up queue counter), which saves a launch
template <int OP, bool MIXED>
__global__ __launch_bounds__(256) void k_pack(const PairArgs a, int begin) {
    if (begin > 0 && blockIdx.x == 0) {
        if (threadIdx.x < 3) a.pass_stats[threadIdx.x] = 0;
        if (threadIdx.x == 3 && begin == 2) *a.fix_count = 0;
    }
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= a.src.count) return;
    const int p = particle_of(a.src, q, a.P.n, a.flags);
    const double gm = a.G * a.P.m[p];
    double4* pk = static_cast<double4*>(const_cast<void*>(a.pack));
    // mixed: G m as FP32 in the low half of the fourth slot; FP64: G m as FP64
    const double4 pos = make_double4(a.P.x[p], a.P.y[p], a.P.z[p], MIXED ? pack_gm((float)gm) : gm);
    if constexpr (OP == OP_ACC) {
        pk[q] = pos;
    } else if constexpr (OP == OP_GRAD) {
        pk[2 * q] = pos;
        pk[2 * q + 1] = make_double4(a.P.ax[p], a.P.ay[p], a.P.az[p], 0.0);
    } else {
        pk[2 * q] = pos;
        pk[2 * q + 1] = make_double4(a.P.vx[p], a.P.vy[p], a.P.vz[p], (double)p);
    }
}

// ---- reduction over source chunks (fixed order) --------------------------------------------

template <class Op>
__global__ __launch_bounds__(256) void k_reduce(const PairArgs a) {
    constexpr int NP = ncomp_of<Op>();
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    const int nt = a.tgt.count;
    if (k >= nt) return;
    double v[NP];
#pragma unroll
    for (int comp = 0; comp < NP; ++comp) v[comp] = 0.0;
    for (int c = 0; c < a.split; ++c) {
#pragma unroll
        for (int comp = 0; comp < NP; ++comp) {
            const double x = a.part[((size_t)c * NP + comp) * nt + k];
            v[comp] = Op::kMax ? fmax(v[comp], x) : v[comp] + x;
        }
    }
    write_result<Op>(a, k, particle_of(a.tgt, k, a.P.n, a.flags), v);
}

// many chunks: one wavefront per target, lane l combining chunks l, l + 64, ... in order, then
// a fixed butterfly over the lanes
template <class Op>
__global__ __launch_bounds__(256) void k_reduce_wave(const PairArgs a) {
    constexpr int NP = ncomp_of<Op>();
    const int k = blockIdx.x * 4 + (int)(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    const int nt = a.tgt.count;
    if (k >= nt) return;  // uniform over the wavefront
    double v[NP];
#pragma unroll
    for (int comp = 0; comp < NP; ++comp) v[comp] = 0.0;
    for (int c = lane; c < a.split; c += 64) {
#pragma unroll
        for (int comp = 0; comp < NP; ++comp) {
            const double x = a.part[((size_t)c * NP + comp) * nt + k];
            v[comp] = Op::kMax ? fmax(v[comp], x) : v[comp] + x;
        }
    }
    for (int m = 32; m > 0; m >>= 1) {
#pragma unroll
        for (int comp = 0; comp < NP; ++comp) {
            const double x = __shfl_xor(v[comp], m, 64);
            v[comp] = Op::kMax ? fmax(v[comp], x) : v[comp] + x;
        }
    }
    if (lane == 0) write_result<Op>(a, k, particle_of(a.tgt, k, a.P.n, a.flags), v);
}

// ---- FP64 fix-up of ill-conditioned targets ------------------------------------------------

__global__ void k_zero_count(int32_t* c) { *c = 0; }
__global__ void k_zero_u64(unsigned long long* c, int n) {
    if ((int)threadIdx.x < n) c[threadIdx.x] = 0;
}
// start of a pass: the fix-up queue counter (if any) and the three pass statistics
__global__ void k_pass_begin(int32_t* fix_count, unsigned long long* stats) {
    if (threadIdx.x < 3) stats[threadIdx.x] = 0;
    if (threadIdx.x == 3 && fix_count) *fix_count = 0;
}

// The queue is worked in rounds of up to kFixTiled targets, each round split into source chunks
// so that the grid (wgs workgroups) fills.  Where a round has at least kFixWide targets and
// kFixWidePairs target-source pairs, each thread takes one target and every source chunk is
// staged through LDS for 256 targets at once; otherwise each workgroup takes one (target,
// chunk) item, its threads splitting the chunk.  Both write FP64 partial sums per chunk, which
// k_fixup_reduce adds in chunk order.  The plan depends only on the round's length, the source
// count, wgs and the partial buffer's capacity `cap` (doubles per component, at least
// kFixTiled), so the two kernels agree on it and the sums are repeatable.  Rounds past the
// queue's end exit at once.
constexpr int kFixWide = 64;
constexpr int64_t kFixWidePairs = 1 << 22;

struct FixPlan {
    bool wide;   // thread per target (else workgroup per (target, chunk))
    int nch;     // source chunks
    int chunk;   // sources per chunk
    int stride;  // partial-sum stride between chunk components
};

__device__ __forceinline__ FixPlan fix_plan(int count, int ns, int wgs, int cap) {
    FixPlan f;
    f.wide = count >= kFixWide && (int64_t)count * ns >= kFixWidePairs;
    if (f.wide) {
        const int slabs = (count + 255) / 256;
        f.stride = slabs * 256;
        f.nch = max(1, min(wgs / slabs, (ns + 255) / 256));  // chunks of at least 256 sources
    } else {
        f.stride = (count + 63) / 64 * 64;
        f.nch = max(1, min((wgs + count - 1) / count, (ns + 255) / 256));
    }
    f.nch = max(1, min(f.nch, cap / f.stride));  // the partial-sum buffer (stride <= kFixTiled <= cap)
    f.chunk = (ns + f.nch - 1) / f.nch;
    return f;
}

__device__ __forceinline__ int fix_round_count(const PairArgs& a, int base) {
    return min(min(*a.fix_count, a.tgt.count) - base, kFixTiled);
}

template <int OP>
__global__ __launch_bounds__(256) void k_fixup_tiled(const PairArgs a, double* part, int base, int wgs, int cap) {
    const int count = fix_round_count(a, base);
    if (count <= 0) return;
    const int ns = a.src.count;
    const FixPlan f = fix_plan(count, ns, wgs, cap);
    if (!f.wide) {
        for (int it = blockIdx.x; it < count * f.nch; it += gridDim.x) {  // uniform over the workgroup
            const int e = it / f.nch, c = it % f.nch;
            const int pi = particle_of(a.tgt, a.fix_list[base + e], a.P.n, a.flags);
            const int q0 = c * f.chunk, q1 = min(ns, q0 + f.chunk);
            double v[3];
            fix_range<OP>(a.P, a.src, a.sub, pi, a.G, a.eps2, a.flags, q0, q1, v);
            if (threadIdx.x == 0) {
                part[((size_t)c * 3 + 0) * f.stride + e] = v[0];
                part[((size_t)c * 3 + 1) * f.stride + e] = v[1];
                part[((size_t)c * 3 + 2) * f.stride + e] = v[2];
            }
            __syncthreads();  // fix_range's LDS is reused by the next item
        }
        return;
    }
    const int nch = f.nch, items = (count + 255) / 256 * nch, chunk = f.chunk;
    __shared__ double4 sp[256];  // (x, y, z, G m)
    __shared__ double4 sa[256];  // (ax, ay, az, particle index)
    for (int it = blockIdx.x; it < items; it += gridDim.x) {
        const int slab = it / nch, c = it % nch;
        const int e = slab * 256 + (int)threadIdx.x;
        const bool act = e < count;
        const int pi = particle_of(a.tgt, a.fix_list[base + (act ? e : 0)], a.P.n, a.flags);
        const double xi = a.P.x[pi], yi = a.P.y[pi], zi = a.P.z[pi];
        double axi = 0.0, ayi = 0.0, azi = 0.0;
        if constexpr (OP == OP_GRAD) { axi = a.P.ax[pi]; ayi = a.P.ay[pi]; azi = a.P.az[pi]; }
        double sx = 0.0, sy = 0.0, sz = 0.0;
        const int j0 = c * chunk, j1 = min(ns, j0 + chunk);
        for (int jt = j0; jt < j1; jt += 256) {
            const int len = min(256, j1 - jt);
            __syncthreads();
            if ((int)threadIdx.x < len) {
                const int p = particle_of(a.src, jt + threadIdx.x, a.P.n, a.flags);
                sp[threadIdx.x] = make_double4(a.P.x[p], a.P.y[p], a.P.z[p], a.G * a.P.m[p]);
                if constexpr (OP == OP_GRAD) sa[threadIdx.x] = make_double4(a.P.ax[p], a.P.ay[p], a.P.az[p], (double)p);
                else sa[threadIdx.x] = make_double4(0.0, 0.0, 0.0, (double)p);
            }
            __syncthreads();
            if (!act) continue;
            // Without subsystem labels the loop has no branch: a skipped pair (the target
            // itself, or a coincident pair, which raises the flag once per tile) adds w = 0.
            if (a.sub == nullptr) {
                bool coincident = false;
#pragma unroll 4
                for (int j = 0; j < len; ++j) {
                    const double4 q = sp[j];
                    const double4 qa = sa[j];
                    const double dx = q.x - xi, dy = q.y - yi, dz = q.z - zi;
                    const double r2 = dx * dx + dy * dy + dz * dz + a.eps2;
                    const bool self = (int)qa.w == pi, zero = r2 == 0.0;
                    coincident = coincident || (zero && !self);
                    const bool off = self || zero;
                    const double ri = rsqrt64(off ? 1.0 : r2);
                    const double ri2 = ri * ri;
                    const double w = off ? 0.0 : q.w * ri * ri2;
                    if constexpr (OP == OP_ACC) {
                        sx += w * dx; sy += w * dy; sz += w * dz;
                    } else {
                        const double dax = qa.x - axi, day = qa.y - ayi, daz = qa.z - azi;
                        const double q3 = 3.0 * (dax * dx + day * dy + daz * dz) * ri2;
                        sx += w * (dax - q3 * dx); sy += w * (day - q3 * dy); sz += w * (daz - q3 * dz);
                    }
                }
                if (coincident) atomicOr(a.flags, BF_FLAG_COINCIDENT);
                continue;
            }
            for (int j = 0; j < len; ++j) {
                const int pj = (int)sa[j].w;
                if (pj == pi || same_sub(a.sub, pi, pj)) continue;
                const double4 q = sp[j];
                const double dx = q.x - xi, dy = q.y - yi, dz = q.z - zi;
                const double r2 = dx * dx + dy * dy + dz * dz + a.eps2;
                if (r2 == 0.0) { atomicOr(a.flags, BF_FLAG_COINCIDENT); continue; }
                const double ri = rsqrt64(r2);
                const double ri2 = ri * ri;
                const double w = q.w * ri * ri2;
                if constexpr (OP == OP_ACC) {
                    sx += w * dx; sy += w * dy; sz += w * dz;
                } else {
                    const double dax = sa[j].x - axi, day = sa[j].y - ayi, daz = sa[j].z - azi;
                    const double q3 = 3.0 * (dax * dx + day * dy + daz * dz) * ri2;
                    sx += w * (dax - q3 * dx); sy += w * (day - q3 * dy); sz += w * (daz - q3 * dz);
                }
            }
        }
        if (act) {
            part[((size_t)c * 3 + 0) * f.stride + e] = sx;
            part[((size_t)c * 3 + 1) * f.stride + e] = sy;
            part[((size_t)c * 3 + 2) * f.stride + e] = sz;
        }
    }
}

// one wavefront per queued target: lane l adds chunks l, l + 64, ... in order, then a fixed
// butterfly over the lanes
__global__ __launch_bounds__(256) void k_fixup_reduce(const PairArgs a, const double* part, int base, int wgs,
                                                      int cap) {
    if (base == 0 && a.pass_stats && blockIdx.x == 0 && threadIdx.x == 0)
        a.pass_stats[0] = (unsigned long long)min(*a.fix_count, a.tgt.count);
    const int count = fix_round_count(a, base);
    if (count <= 0) return;
    const FixPlan f = fix_plan(count, a.src.count, wgs, cap);
    const int lane = threadIdx.x & 63;
    for (int e = blockIdx.x * 4 + (int)(threadIdx.x >> 6); e < count; e += gridDim.x * 4) {  // uniform per wave
        double v[3] = {0.0, 0.0, 0.0};
        for (int c = lane; c < f.nch; c += 64)
            for (int k = 0; k < 3; ++k) v[k] += part[((size_t)c * 3 + k) * f.stride + e];
        for (int m = 32; m > 0; m >>= 1)
            for (int k = 0; k < 3; ++k) v[k] += __shfl_xor(v[k], m, 64);
        if (lane == 0) {
            const int pi = particle_of(a.tgt, a.fix_list[base + e], a.P.n, a.flags);
            a.o0[pi] = v[0];
            a.o1[pi] = v[1];
            a.o2[pi] = v[2];
        }
    }
}

// ---- launch tables -------------------------------------------------------------------------

using KernelFn = void (*)(const PairArgs);

template <class Op, bool D>
static KernelFn pick(int k, int w) {
#define BF_PICK(KK, WW) \
    if (k == KK && w == WW) return k_pairs<Op, KK, WW, D>;
    BF_PICK(1, 2) BF_PICK(2, 2) BF_PICK(4, 2)
    BF_PICK(1, 4) BF_PICK(2, 4) BF_PICK(4, 4)
    BF_PICK(1, 8) BF_PICK(2, 8) BF_PICK(4, 8)
#undef BF_PICK
    return nullptr;
}

// variants with intra-subsystem exclusion: one block shape (4 waves), 1 or 2 targets per lane
template <class Op, bool D>
static KernelFn pick_excl(int k, int w) {
    if (w != 4) return nullptr;
    if (k == 1) return k_pairs<Op, 1, 4, D, true>;
    if (k == 2) return k_pairs<Op, 2, 4, D, true>;
    return nullptr;
}

static KernelFn kernel_for_excl(int op, int prec, int k, int w, bool detect) {
    const bool mixed = prec == BF_PREC_MIXED;
    switch (op) {
        case OP_ACC:
            if (!mixed) return pick_excl<Acc64, false>(k, w);
            return detect ? pick_excl<AccMixed, true>(k, w) : pick_excl<AccMixed, false>(k, w);
        case OP_GRAD:
            if (!mixed) return pick_excl<Grad64, false>(k, w);
            return detect ? pick_excl<GradMixed, true>(k, w) : pick_excl<GradMixed, false>(k, w);
        case OP_DT: return mixed ? pick_excl<DtMixed, true>(k, w) : pick_excl<Dt64, false>(k, w);
    }
    return nullptr;
}

static KernelFn kernel_for(int op, int prec, int k, int w, bool detect, bool excl = false) {
    if (excl) return kernel_for_excl(op, prec, k, w, detect);
    const bool mixed = prec == BF_PREC_MIXED;
    switch (op) {
        case OP_ACC:
            if (!mixed) return pick<Acc64, false>(k, w);
            return detect ? pick<AccMixed, true>(k, w) : pick<AccMixed, false>(k, w);
        case OP_GRAD:
            if (!mixed) return pick<Grad64, false>(k, w);
            return detect ? pick<GradMixed, true>(k, w) : pick<GradMixed, false>(k, w);
        case OP_DT: return mixed ? pick<DtMixed, true>(k, w) : pick<Dt64, false>(k, w);
    }
    return nullptr;
}

bool variant_exists(int op, int prec, int k, int waves, bool excl) {
    return kernel_for(op, prec, k, waves, false, excl) != nullptr;
}

int variant_blocks_per_cu(int op, int prec, int k, int waves, bool excl) {
    KernelFn f = kernel_for(op, prec, k, waves, op == OP_DT, excl);
    if (!f) return 0;
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, reinterpret_cast<const void*>(f), 64 * waves, 0) != hipSuccess)
        return 0;
    return nb;
}

hipError_t launch_pairs(int op, int prec, const KernelConfig& cfg, const PairArgs& a, int nblocks, hipStream_t st) {
    const bool detect = prec == BF_PREC_MIXED && a.rfb2f > 0.0f;
    KernelFn f = kernel_for(op, prec, cfg.k, cfg.waves, detect || op == OP_DT, a.sub != nullptr);
    if (!f) return hipErrorInvalidValue;
    hipLaunchKernelGGL(f, dim3(nblocks), dim3(64 * cfg.waves), 0, st, a);
    return hipGetLastError();
}

int pack_bytes(int op, int /*prec*/) { return op == OP_ACC ? 32 : 64; }

int stored_components(int op, int prec) {
    if (op == OP_DT) return 2;
    return prec == BF_PREC_MIXED ? 4 : 3;
}

template <int OP, bool MIXED>
static void pack_one(const PairArgs& a, int begin, hipStream_t st) {
    const int n = a.src.count;
    hipLaunchKernelGGL((k_pack<OP, MIXED>), dim3((n + 255) / 256), dim3(256), 0, st, a, begin);
}

hipError_t launch_pack(int op, int prec, const PairArgs& a, hipStream_t st, int begin) {
    if (a.src.count <= 0) return hipSuccess;
    const bool mixed = prec == BF_PREC_MIXED;
    if (op == OP_ACC) mixed ? pack_one<OP_ACC, true>(a, begin, st) : pack_one<OP_ACC, false>(a, begin, st);
    else if (op == OP_GRAD) mixed ? pack_one<OP_GRAD, true>(a, begin, st) : pack_one<OP_GRAD, false>(a, begin, st);
    else mixed ? pack_one<OP_DT, true>(a, begin, st) : pack_one<OP_DT, false>(a, begin, st);
    return hipGetLastError();
}

template <class Op>
static void reduce_one(const PairArgs& a, hipStream_t st) {
    const int n = a.tgt.count;
    if (a.split > kReduceWaveSplit) hipLaunchKernelGGL(k_reduce_wave<Op>, dim3((n + 3) / 4), dim3(256), 0, st, a);
    else hipLaunchKernelGGL(k_reduce<Op>, dim3((n + 255) / 256), dim3(256), 0, st, a);
}

hipError_t launch_reduce(int op, int prec, const PairArgs& a, hipStream_t st) {
    if (a.tgt.count <= 0) return hipSuccess;
    const bool mixed = prec == BF_PREC_MIXED;
    if (op == OP_ACC) mixed ? reduce_one<AccMixed>(a, st) : reduce_one<Acc64>(a, st);
    else if (op == OP_GRAD) mixed ? reduce_one<GradMixed>(a, st) : reduce_one<Grad64>(a, st);
    else mixed ? reduce_one<DtMixed>(a, st) : reduce_one<Dt64>(a, st);
    return hipGetLastError();
}

hipError_t launch_zero_count(int32_t* c, hipStream_t st) {
    hipLaunchKernelGGL(k_zero_count, dim3(1), dim3(1), 0, st, c);
    return hipGetLastError();
}

hipError_t launch_pass_begin(int32_t* fix_count, unsigned long long* stats, hipStream_t st) {
    hipLaunchKernelGGL(k_pass_begin, dim3(1), dim3(64), 0, st, fix_count, stats);
    return hipGetLastError();
}

hipError_t launch_zero_u64(unsigned long long* c, int n, hipStream_t st) {
    hipLaunchKernelGGL(k_zero_u64, dim3(1), dim3(64), 0, st, c, n);
    return hipGetLastError();
}

hipError_t launch_fixup(int op, const PairArgs& a, double* part, int cap, int num_cu, hipStream_t st) {
    const int nt = a.tgt.count;
    if (nt <= 0) return hipSuccess;
    if ((op != OP_ACC && op != OP_GRAD) || cap < kFixTiled) return hipErrorInvalidValue;
    const int64_t ns = a.src.count;
    for (int base = 0; base < nt; base += kFixTiled) {  // rounds past the queue's end exit at once
        const int len = std::min(nt - base, kFixTiled);
        // enough workgroups for the longest possible round, at most 8 per CU
        const int64_t most = (int64_t)len * ((ns + 255) / 256);
        const int g1 = (int)std::max<int64_t>(1, std::min<int64_t>(most, 8 * num_cu));
        const int g2 = std::min((len + 3) / 4, 8 * num_cu);
        if (op == OP_ACC) hipLaunchKernelGGL(k_fixup_tiled<OP_ACC>, dim3(g1), dim3(256), 0, st, a, part, base, g1, cap);
        else hipLaunchKernelGGL(k_fixup_tiled<OP_GRAD>, dim3(g1), dim3(256), 0, st, a, part, base, g1, cap);
        hipLaunchKernelGGL(k_fixup_reduce, dim3(g2), dim3(256), 0, st, a, (const double*)part, base, g1, cap);
    }
    return hipGetLastError();
}

}  // namespace bf
