// Direct-summation pair kernels for gfx950: Newtonian acceleration, force gradient and the
// pairwise time-step maxima, each in a mixed (FP32 pair arithmetic, FP64 merge) and an FP64
// flavour, sharing one tiled skeleton.
//
// Skeleton (one workgroup = W wavefronts):
//  * the workgroup owns a slab of 64*K*W target slots (K per lane, lane-strided) and one of
//    `split` chunks of the source list; block b takes chunk b % split, so with split = 8 all
//    workgroups on one XCD (dispatch is round-robin over the 8 XCDs) stream the same chunk
//    and it stays in that XCD's L2;
//  * sources are staged tile by tile (64*W per tile, one per thread) from a packed stream into
//    LDS; every lane then walks the tile with a broadcast LDS read per source and updates its
//    K targets in registers;
//  * mixed precision: each tile is summed into FP32 partials that start at zero, and merged
//    into FP64 accumulators after the tile (cascade summation: the FP32 sum never spans more
//    than one tile).  The per-lane minimum of s^2 over the tile is tracked; if any lane of the
//    wavefront saw s^2 < r_fb^2 the wavefront re-evaluates that tile in FP64 from the FP64
//    masters with explicit self-exclusion and uses that instead (close pairs, coincident
//    FP32 positions and the self pair all land there);
//  * results go straight to the particle-indexed outputs (split == 1) or to per-chunk
//    partials that a second kernel reduces in chunk order (deterministic).
#include "pair_ops.h"

namespace bf {

// ---- output of one target ------------------------------------------------------------------

template <class Op>
__device__ __forceinline__ void emit(const PairArgs& a, int c, int slot, int pi, const typename Op::A64& acc) {
    double v[Op::NC];
    Op::comps(acc, v);
    if (a.split == 1) {
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
        }
    } else {
        const int nt = a.tgt.count;
#pragma unroll
        for (int comp = 0; comp < Op::NC; ++comp) a.part[((size_t)c * Op::NC + comp) * nt + slot] = v[comp];
    }
}

// ---- the skeleton --------------------------------------------------------------------------

template <class Op, int K, int W>
__global__ __launch_bounds__(64 * W) void k_pairs(const PairArgs a) {
    __shared__ typename Op::Src tile[64 * W];
    const int wave = threadIdx.x >> 6;
    const int c = blockIdx.x % a.split;
    const int slab = blockIdx.x / a.split;
    const int tbase = slab * (64 * K * W) + wave * (64 * K);
    const int j0 = c * a.chunk;
    const int j1 = min(a.src.count, j0 + a.chunk);
    typename Op::A64 acc[K];
    int slot[K], pidx[K];
    sweep<Op, K, W>(a, tile, tbase, j0, j1, acc, slot, pidx);
#pragma unroll
    for (int k = 0; k < K; ++k)
        if (slot[k] < a.tgt.count) emit<Op>(a, c, slot[k], pidx[k], acc[k]);
}

// ---- packing the source stream -------------------------------------------------------------

template <int OP, bool MIXED>
__global__ __launch_bounds__(256) void k_pack(const PairArgs a) {
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= a.src.count) return;
    const int p = particle_of(a.src, q, a.P.n, a.flags);
    const double gm = a.G * a.P.m[p];
    if constexpr (MIXED) {
        float4* pk = static_cast<float4*>(const_cast<void*>(a.pack));
        const float4 pos = make_float4((float)a.P.x[p], (float)a.P.y[p], (float)a.P.z[p], (float)gm);
        if constexpr (OP == OP_ACC) {
            pk[q] = pos;
        } else if constexpr (OP == OP_GRAD) {
            // FP64 positions and accelerations; G m as FP32 in the low half of the fourth slot
            double4* pd = static_cast<double4*>(const_cast<void*>(a.pack));
            pd[2 * q] = make_double4(a.P.x[p], a.P.y[p], a.P.z[p],
                                     __builtin_bit_cast(double, make_float2((float)gm, 0.f)));
            pd[2 * q + 1] = make_double4(a.P.ax[p], a.P.ay[p], a.P.az[p], 0.0);
        } else {
            pk[2 * q] = pos;
            pk[2 * q + 1] = make_float4((float)a.P.vx[p], (float)a.P.vy[p], (float)a.P.vz[p], 0.f);
        }
    } else {
        double4* pk = static_cast<double4*>(const_cast<void*>(a.pack));
        const double4 pos = make_double4(a.P.x[p], a.P.y[p], a.P.z[p], gm);
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
}

// ---- reduction over source chunks (fixed order) --------------------------------------------

template <int NC, bool MAX>
__global__ __launch_bounds__(256) void k_reduce(const PairArgs a) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    const int nt = a.tgt.count;
    if (k >= nt) return;
    double v[NC];
#pragma unroll
    for (int comp = 0; comp < NC; ++comp) v[comp] = 0.0;
    for (int c = 0; c < a.split; ++c) {
#pragma unroll
        for (int comp = 0; comp < NC; ++comp) {
            const double x = a.part[((size_t)c * NC + comp) * nt + k];
            v[comp] = MAX ? fmax(v[comp], x) : v[comp] + x;
        }
    }
    const int p = particle_of(a.tgt, k, a.P.n, a.flags);
    if constexpr (MAX) {
        const double dff = a.eta0 / sqrt(v[0]), dfb = a.eta1 / sqrt(v[1]);
        if (__builtin_isnan(dff) || __builtin_isnan(dfb)) atomicOr(a.flags, BF_FLAG_NONFINITE);
        a.o0[p] = dff;
        a.o1[p] = dfb;
    } else {
        if (!__builtin_isfinite(v[0]) || !__builtin_isfinite(v[1]) || !__builtin_isfinite(v[2]))
            atomicOr(a.flags, BF_FLAG_NONFINITE);
        a.o0[p] = v[0];
        a.o1[p] = v[1];
        a.o2[p] = v[2];
    }
}

// ---- launch tables -------------------------------------------------------------------------

using KernelFn = void (*)(const PairArgs);

template <class Op>
static KernelFn pick(int k, int w) {
    if (w == 4) {
        if (k == 1) return k_pairs<Op, 1, 4>;
        if (k == 2) return k_pairs<Op, 2, 4>;
        if (k == 4) return k_pairs<Op, 4, 4>;
    } else if (w == 8) {
        if (k == 1) return k_pairs<Op, 1, 8>;
        if (k == 2) return k_pairs<Op, 2, 8>;
        if (k == 4) return k_pairs<Op, 4, 8>;
    } else if (w == 2) {
        if (k == 1) return k_pairs<Op, 1, 2>;
        if (k == 2) return k_pairs<Op, 2, 2>;
        if (k == 4) return k_pairs<Op, 4, 2>;
    }
    return nullptr;
}

static KernelFn kernel_for(int op, int prec, int k, int w) {
    const bool mixed = prec == BF_PREC_MIXED;
    switch (op) {
        case OP_ACC: return mixed ? pick<AccMixed>(k, w) : pick<Acc64>(k, w);
        case OP_GRAD: return mixed ? pick<GradMixed>(k, w) : pick<Grad64>(k, w);
        case OP_DT: return mixed ? pick<DtMixed>(k, w) : pick<Dt64>(k, w);
    }
    return nullptr;
}

bool variant_exists(int op, int prec, int k, int waves) { return kernel_for(op, prec, k, waves) != nullptr; }

int variant_blocks_per_cu(int op, int prec, int k, int waves) {
    KernelFn f = kernel_for(op, prec, k, waves);
    if (!f) return 0;
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, reinterpret_cast<const void*>(f), 64 * waves, 0) != hipSuccess)
        return 0;
    return nb;
}

hipError_t launch_pairs(int op, int prec, const KernelConfig& cfg, const PairArgs& a, int nblocks, hipStream_t st) {
    KernelFn f = kernel_for(op, prec, cfg.k, cfg.waves);
    if (!f) return hipErrorInvalidValue;
    hipLaunchKernelGGL(f, dim3(nblocks), dim3(64 * cfg.waves), 0, st, a);
    return hipGetLastError();
}

int pack_bytes(int op, int prec) {
    if (op == OP_GRAD) return 64;  // FP64 differences in both precisions
    const int base = prec == BF_PREC_MIXED ? 16 : 32;
    return op == OP_ACC ? base : 2 * base;
}

template <int OP, bool MIXED>
static void pack_one(const PairArgs& a, hipStream_t st) {
    const int n = a.src.count;
    hipLaunchKernelGGL((k_pack<OP, MIXED>), dim3((n + 255) / 256), dim3(256), 0, st, a);
}

hipError_t launch_pack(int op, int prec, const PairArgs& a, hipStream_t st) {
    if (a.src.count <= 0) return hipSuccess;
    const bool mixed = prec == BF_PREC_MIXED;
    if (op == OP_ACC) mixed ? pack_one<OP_ACC, true>(a, st) : pack_one<OP_ACC, false>(a, st);
    else if (op == OP_GRAD) mixed ? pack_one<OP_GRAD, true>(a, st) : pack_one<OP_GRAD, false>(a, st);
    else mixed ? pack_one<OP_DT, true>(a, st) : pack_one<OP_DT, false>(a, st);
    return hipGetLastError();
}

hipError_t launch_reduce(int op, const PairArgs& a, hipStream_t st) {
    const int n = a.tgt.count;
    if (n <= 0) return hipSuccess;
    const dim3 g((n + 255) / 256), b(256);
    if (op == OP_DT) hipLaunchKernelGGL((k_reduce<2, true>), g, b, 0, st, a);
    else hipLaunchKernelGGL((k_reduce<3, false>), g, b, 0, st, a);
    return hipGetLastError();
}

}  // namespace bf
