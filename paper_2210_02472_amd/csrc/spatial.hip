// Spatially sorted mode of the mixed acceleration and force-gradient passes.
//
// Sources and targets are ordered along a Morton (Z-order) curve over the sources' bounding box,
// so that a tile of 64*W consecutive sources and a workgroup's targets each occupy a compact
// region.  Each tile is packed twice: with FP64 positions (and accelerations) for tiles that lie
// near a workgroup's targets, and as FP32 offsets from the tile centre for all other tiles; the
// sorted sweep (pair_ops.h) picks per tile.  Outputs stay particle-indexed, so the ordering is
// invisible to the caller.
#include <algorithm>

#include <rocprim/device/device_merge_sort.hpp>
#include <rocprim/device/device_radix_sort.hpp>

#include "pair_ops.h"

namespace bf {

// ---- bounding box and Morton keys -----------------------------------------------------------

// order-preserving map of FP32 onto unsigned integers (min/max by integer atomics)
__device__ __forceinline__ uint32_t ord32(float f) {
    const uint32_t u = __float_as_uint(f);
    return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}
__device__ __forceinline__ float unord32(uint32_t u) {
    return __uint_as_float((u & 0x80000000u) ? (u & 0x7fffffffu) : ~u);
}

__global__ void k_box_init(uint32_t* box) {
    if (threadIdx.x < 3) box[threadIdx.x] = 0xffffffffu;
    else if (threadIdx.x < 6) box[threadIdx.x] = 0u;
}

__global__ __launch_bounds__(256) void k_box(Masters P, DevSet set, uint32_t* box, uint32_t* flags) {
    __shared__ uint32_t red[6][4];
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    uint32_t v[6] = {0xffffffffu, 0xffffffffu, 0xffffffffu, 0u, 0u, 0u};
    if (k < set.count) {
        const int p = particle_of(set, k, P.n, flags);
        const uint32_t x = ord32((float)P.x[p]), y = ord32((float)P.y[p]), z = ord32((float)P.z[p]);
        v[0] = v[3] = x; v[1] = v[4] = y; v[2] = v[5] = z;
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            v[d] = min(v[d], (uint32_t)__shfl_xor((int)v[d], off));
            v[3 + d] = max(v[3 + d], (uint32_t)__shfl_xor((int)v[3 + d], off));
        }
    }
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0)
        for (int d = 0; d < 6; ++d) red[d][wave] = v[d];
    __syncthreads();
    if (threadIdx.x < 6) {
        const int d = threadIdx.x;
        uint32_t r = red[d][0];
        for (int w = 1; w < 4; ++w) r = d < 3 ? min(r, red[d][w]) : max(r, red[d][w]);
        if (d < 3) atomicMin(&box[d], r);
        else atomicMax(&box[d], r);
    }
}

// spread the low 10 bits of v to every third bit
__device__ __forceinline__ uint32_t spread3(uint32_t v) {
    v &= 0x3ffu;
    v = (v | (v << 16)) & 0x030000ffu;
    v = (v | (v << 8)) & 0x0300f00fu;
    v = (v | (v << 4)) & 0x030c30c3u;
    v = (v | (v << 2)) & 0x09249249u;
    return v;
}

__global__ __launch_bounds__(256) void k_keys(Masters P, DevSet set, const uint32_t* box, uint32_t* keys,
                                              int32_t* vals, uint32_t* flags) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= set.count) return;
    const int p = particle_of(set, k, P.n, flags);
    const float c[3] = {(float)P.x[p], (float)P.y[p], (float)P.z[p]};
    uint32_t q[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        const float lo = unord32(box[d]), hi = unord32(box[3 + d]);
        const float span = hi - lo;
        float t = span > 0.f ? (c[d] - lo) / span : 0.f;
        t = fminf(fmaxf(t, 0.f), 1.f);  // targets outside the sources' box clamp to its faces
        q[d] = (uint32_t)(t * 1023.0f);
    }
    keys[k] = spread3(q[0]) | (spread3(q[1]) << 1) | (spread3(q[2]) << 2);
    vals[k] = k;
}

__global__ __launch_bounds__(256) void k_sorted_list(DevSet set, const int32_t* order, int32_t* out, int64_t n,
                                                     uint32_t* flags) {
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= set.count) return;
    int k = order[s];
    if (k < 0 || k >= set.count) k = 0;  // cannot happen: the sort permutes 0..count-1
    out[s] = particle_of(set, k, n, flags);
}

// Temporary storage of either sort below (the larger of the two).
size_t sort_tmp_bytes(int n) {
    size_t radix = 0, merge = 0;
    rocprim::radix_sort_pairs(nullptr, radix, (const uint32_t*)nullptr, (uint32_t*)nullptr, (const int32_t*)nullptr,
                              (int32_t*)nullptr, (unsigned)n, 0, 30, (hipStream_t)0);
    rocprim::merge_sort(nullptr, merge, (const uint32_t*)nullptr, (uint32_t*)nullptr, (const int32_t*)nullptr,
                        (int32_t*)nullptr, (size_t)n, rocprim::less<uint32_t>(), (hipStream_t)0);
    return std::max(radix, merge);
}

// The Morton order of a set.  Both sorts are stable, so they give the same order; the radix sort
// is the faster, but it clears its counters with memset operations, which a captured graph must
// not hold (graph_safe: the merge sort, which launches kernels only).
hipError_t launch_sort_set(const Masters& P, const DevSet& set, const DevSet& box_set, const SortBuffers& sb,
                           int32_t* out, uint32_t* flags, hipStream_t st, bool graph_safe) {
    const int n = set.count;
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_box_init, dim3(1), dim3(64), 0, st, sb.bbox);
    if (box_set.count > 0)
        hipLaunchKernelGGL(k_box, dim3((box_set.count + 255) / 256), dim3(256), 0, st, P, box_set, sb.bbox, flags);
    hipLaunchKernelGGL(k_keys, dim3((n + 255) / 256), dim3(256), 0, st, P, set, (const uint32_t*)sb.bbox, sb.keys_in,
                       sb.vals_in, flags);
    size_t bytes = sb.tmp_bytes;
    hipError_t e = graph_safe ? rocprim::merge_sort(sb.tmp, bytes, sb.keys_in, sb.keys_out, sb.vals_in, sb.vals_out,
                                                    (size_t)n, rocprim::less<uint32_t>(), st)
                              : rocprim::radix_sort_pairs(sb.tmp, bytes, sb.keys_in, sb.keys_out, sb.vals_in,
                                                          sb.vals_out, (unsigned)n, 0, 30, st);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_sorted_list, dim3((n + 255) / 256), dim3(256), 0, st, set, (const int32_t*)sb.vals_out, out,
                       P.n, flags);
    return hipGetLastError();
}

// ---- tile packing ----------------------------------------------------------------------------
// One workgroup of T = 64*W threads per tile of sorted sources.  Near stream: the FP64 pack of the
// mixed pass; far stream: FP32 offsets from the tile centre; metadata per tile: (centre, half
// extent as FP32 in the fourth slot) and, for the gradient, (acceleration centre, 0).

template <int OP, int T>
__global__ __launch_bounds__(T) void k_pack_tiles(const PairArgs a, double4* near_pack, float4* far_pack,
                                                 double4* meta) {
    __shared__ float red[6][T / 64];
    __shared__ float redA[6][T / 64];
    const int s = blockIdx.x * T + threadIdx.x;
    const bool ok = s < a.src.count;
    const int p = particle_of(a.src, ok ? s : a.src.count - 1, a.P.n, a.flags);
    const double x = a.P.x[p], y = a.P.y[p], z = a.P.z[p];
    double ax = 0.0, ay = 0.0, az = 0.0;
    if constexpr (OP == OP_GRAD) { ax = a.P.ax[p]; ay = a.P.ay[p]; az = a.P.az[p]; }
    // tile box of positions (and accelerations), FP32
    float v[6] = {(float)x, (float)y, (float)z, (float)x, (float)y, (float)z};
    float w[6] = {(float)ax, (float)ay, (float)az, (float)ax, (float)ay, (float)az};
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            v[d] = fminf(v[d], __shfl_xor(v[d], off));
            v[3 + d] = fmaxf(v[3 + d], __shfl_xor(v[3 + d], off));
            if constexpr (OP == OP_GRAD) {
                w[d] = fminf(w[d], __shfl_xor(w[d], off));
                w[3 + d] = fmaxf(w[3 + d], __shfl_xor(w[3 + d], off));
            }
        }
    }
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0) {
#pragma unroll
        for (int d = 0; d < 6; ++d) { red[d][wave] = v[d]; redA[d][wave] = w[d]; }
    }
    __syncthreads();
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        for (int u = 0; u < T / 64; ++u) {
            v[d] = fminf(v[d], red[d][u]);
            v[3 + d] = fmaxf(v[3 + d], red[3 + d][u]);
            w[d] = fminf(w[d], redA[d][u]);
            w[3 + d] = fmaxf(w[3 + d], redA[3 + d][u]);
        }
    }
    const double cx = 0.5 * ((double)v[0] + (double)v[3]);
    const double cy = 0.5 * ((double)v[1] + (double)v[4]);
    const double cz = 0.5 * ((double)v[2] + (double)v[5]);
    // half extent: covers the FP32 box, plus a margin for the rounding of the box corners
    float h = fmaxf(fmaxf(v[3] - v[0], v[4] - v[1]), v[5] - v[2]) * 0.5f;
    const float amax = fmaxf(fmaxf(fabsf(v[0]), fabsf(v[3])),
                             fmaxf(fmaxf(fabsf(v[1]), fabsf(v[4])), fmaxf(fabsf(v[2]), fabsf(v[5]))));
    h = h * (1.0f + 1e-6f) + amax * 1.2e-7f;
    const double acx = 0.5 * ((double)w[0] + (double)w[3]);
    const double acy = 0.5 * ((double)w[1] + (double)w[4]);
    const double acz = 0.5 * ((double)w[2] + (double)w[5]);
    constexpr int kMeta = OP == OP_GRAD ? 2 : 1;
    // G * tile mass (for the far-tile magnitude bound) and the half-extent of the accelerations
    const float gm = (float)(a.G * a.P.m[p]);
    float gsum = ok ? gm : 0.f;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) gsum += __shfl_xor(gsum, off);
    __shared__ float redM[T / 64];
    if (lane == 0) redM[wave] = gsum;
    __syncthreads();
    float gm_tile = 0.f;
    for (int u = 0; u < T / 64; ++u) gm_tile += redM[u];
    gm_tile *= 1.0f + 1e-5f;  // rounding margin of the FP32 sum
    float ha = fmaxf(fmaxf(w[3] - w[0], w[4] - w[1]), w[5] - w[2]) * 0.5f;
    const float amaxa = fmaxf(fmaxf(fabsf(w[0]), fabsf(w[3])),
                              fmaxf(fmaxf(fabsf(w[1]), fabsf(w[4])), fmaxf(fabsf(w[2]), fabsf(w[5]))));
    ha = ha * (1.0f + 1e-6f) + amaxa * 1.2e-7f;
    if (threadIdx.x == 0) {
        meta[kMeta * blockIdx.x] = make_double4(cx, cy, cz, __builtin_bit_cast(double, make_float2(h, gm_tile)));
        if constexpr (OP == OP_GRAD) meta[kMeta * blockIdx.x + 1] = make_double4(acx, acy, acz, pack_gm(ha));
    }
    if (!ok) return;
    constexpr int S = OP == OP_GRAD ? 2 : 1;
    near_pack[S * s] = make_double4(x, y, z, pack_gm(gm));
    far_pack[S * s] = make_float4((float)(x - cx), (float)(y - cy), (float)(z - cz), gm);
    if constexpr (OP == OP_GRAD) {
        near_pack[S * s + 1] = make_double4(ax, ay, az, 0.0);
        far_pack[S * s + 1] = make_float4((float)(ax - acx), (float)(ay - acy), (float)(az - acz), 0.f);
    }
}

hipError_t launch_pack_tiles(int op, int waves, const PairArgs& a, void* near_pack, void* far_pack, double4* meta,
                             hipStream_t st) {
    const int n = a.src.count;
    if (n <= 0) return hipSuccess;
    const int T = 64 * waves;
    const dim3 g((n + T - 1) / T);
    double4* np = static_cast<double4*>(near_pack);
    float4* fp = static_cast<float4*>(far_pack);
#define BF_PT(OPV, TV) hipLaunchKernelGGL((k_pack_tiles<OPV, TV>), g, dim3(TV), 0, st, a, np, fp, meta)
    if (op == OP_ACC) {
        if (T == 64) BF_PT(OP_ACC, 64); else if (T == 128) BF_PT(OP_ACC, 128); else if (T == 256) BF_PT(OP_ACC, 256); else if (T == 512) BF_PT(OP_ACC, 512);
        else return hipErrorInvalidValue;
    } else {
        if (T == 64) BF_PT(OP_GRAD, 64); else if (T == 128) BF_PT(OP_GRAD, 128); else if (T == 256) BF_PT(OP_GRAD, 256); else if (T == 512) BF_PT(OP_GRAD, 512);
        else return hipErrorInvalidValue;
    }
#undef BF_PT
    return hipGetLastError();
}

// ---- the sorted pair kernel ------------------------------------------------------------------

template <class Op>
__device__ __forceinline__ void emit_sorted(const PairArgs& a, int c, int slot, int pi, const typename Op::A64& acc) {
    constexpr int NP = ncomp_of<Op>();
    double v[NP];
    Op::comps(acc, v);
    if (a.split == 1) {
        if (!__builtin_isfinite(v[0]) || !__builtin_isfinite(v[1]) || !__builtin_isfinite(v[2]))
            atomicOr(a.flags, BF_FLAG_NONFINITE);
        a.o0[pi] = v[0];
        a.o1[pi] = v[1];
        a.o2[pi] = v[2];
        cond_check(a, slot, v);
    } else {
        const int nt = a.tgt.count;
#pragma unroll
        for (int comp = 0; comp < NP; ++comp) a.part[((size_t)c * NP + comp) * nt + slot] = v[comp];
    }
}

template <class Op, int K, int W>
// one target per lane: ask for six waves per SIMD (the gradient variant then fits 76 VGPRs
// without spills, 2% faster at N = 2^20 than at its natural 92)
__global__ __launch_bounds__(64 * W) __attribute__((amdgpu_waves_per_eu(K == 1 ? 6 : 1))) void k_pairs_sorted(
    const PairArgs a) {
    constexpr int T = 64 * W;
    using Far = typename FarOf<Op>::type;
    constexpr size_t kBytes = sizeof(typename Op::Src) > sizeof(typename Far::Src) ? sizeof(typename Op::Src)
                                                                                    : sizeof(typename Far::Src);
    __shared__ __attribute__((aligned(16))) char tile_raw[T * kBytes];
    __shared__ float sbox[6 * W];
    const int wave = threadIdx.x >> 6;
    const int c = blockIdx.x % a.split;
    const int slab = blockIdx.x / a.split;
    const int tbase = slab * (64 * K * W) + wave * (64 * K);
    const int j0 = c * a.chunk;
    const int j1 = min(a.src.count, j0 + a.chunk);
    typename Op::A64 acc[K];
    int slot[K], pidx[K];
    sweep_sorted<Op, K, W>(a, tile_raw, sbox, tbase, j0, j1, acc, slot, pidx);
#pragma unroll
    for (int k = 0; k < K; ++k)
        if (slot[k] < a.tgt.count) emit_sorted<Op>(a, c, slot[k], pidx[k], acc[k]);
}

using KernelFn = void (*)(const PairArgs);

template <class Op>
static KernelFn pick_sorted(int k, int w) {
#define BF_PICK(KK, WW) \
    if (k == KK && w == WW) return k_pairs_sorted<Op, KK, WW>;
    BF_PICK(1, 2) BF_PICK(2, 2) BF_PICK(4, 2)
    BF_PICK(1, 4) BF_PICK(2, 4) BF_PICK(4, 4)
    BF_PICK(1, 8) BF_PICK(2, 8) BF_PICK(4, 8)
#undef BF_PICK
    return nullptr;
}

static KernelFn sorted_kernel(int op, int k, int w) {
    if (op == OP_ACC) return pick_sorted<AccMixed>(k, w);
    if (op == OP_GRAD) return pick_sorted<GradMixed>(k, w);
    return nullptr;
}

bool sorted_variant_exists(int op, int k, int waves) { return sorted_kernel(op, k, waves) != nullptr; }

int sorted_blocks_per_cu(int op, int k, int waves) {
    KernelFn f = sorted_kernel(op, k, waves);
    if (!f) return 0;
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, reinterpret_cast<const void*>(f), 64 * waves, 0) != hipSuccess)
        return 0;
    return nb;
}

hipError_t launch_pairs_sorted(int op, const KernelConfig& cfg, const PairArgs& a, int nblocks, hipStream_t st) {
    KernelFn f = sorted_kernel(op, cfg.k, cfg.waves);
    if (!f) return hipErrorInvalidValue;
    hipLaunchKernelGGL(f, dim3(nblocks), dim3(64 * cfg.waves), 0, st, a);
    return hipGetLastError();
}

}  // namespace bf
