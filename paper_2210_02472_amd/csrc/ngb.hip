// Subsystem neighbour search and subsystem labels (Sec. 3.3).
//
//  * k_ngb: tiled pass over target x source pairs, kNgbK targets per thread.  Only pairs closer
//    than r_max are examined
//    further; for those the two-body elements of the relative orbit decide (Eqs. ngb-bound,
//    ngb-unbound): with mu = G (m_i + m_j), specific energy E = v^2/2 - mu/r and specific
//    angular momentum h, a bound pair (E < 0, a = -mu / 2E) is a neighbour when a < r_ngb or
//    r < r_ngb; an unbound pair when r < r_ngb, or when its periapsis h^2 / (mu (1 + e)) is
//    below r_ngb and C r / |v| < tau.  FP64 throughout.  Found pairs are appended as 64-bit keys
//    (i << 32 | j) and sorted afterwards, so the output does not depend on the order in which
//    workgroups found them.
//  * subsystem labels: the connected components of the neighbour graph by label propagation
//    (every particle starts with its own index; along every edge the larger label takes the
//    smaller one; labels jump to their label's label) until nothing changes.  Each component
//    ends labelled by its smallest particle index, the same labelling a depth-first search
//    from the smallest unvisited particle gives.
#include <rocprim/device/device_radix_sort.hpp>

#include "pair_ops.h"

namespace bf {

__device__ __forceinline__ bool ngb_criterion(double rx, double ry, double rz, double ux, double uy, double uz,
                                              double mu, const NgbArgs& a) {
    const double r = sqrt(rx * rx + ry * ry + rz * rz);
    const double v2 = ux * ux + uy * uy + uz * uz;
    const double E = 0.5 * v2 - mu / r;
    if (E < 0.0) {
        const double sma = -mu / (2.0 * E);
        return sma < a.r_ngb || r < a.r_ngb;
    }
    if (r < a.r_ngb) return true;
    const double hx = ry * uz - rz * uy, hy = rz * ux - rx * uz, hz = rx * uy - ry * ux;
    const double h2 = hx * hx + hy * hy + hz * hz;
    const double e = sqrt(1.0 + 2.0 * E * h2 / (mu * mu));
    const double rp = h2 / (mu * (1.0 + e));
    return rp < a.r_ngb && a.C * r < a.tau * sqrt(v2);
}

// A workgroup of W wavefronts stages T = 64 W sources at a time in LDS; each thread takes K
// targets (slots slab T K + t + T k), so every source read from LDS serves K pairs.
template <int W, int K>
__global__ __launch_bounds__(64 * W) void k_ngb(const NgbArgs a) {
    constexpr int T = 64 * W;
    __shared__ double4 tp[T];  // (x, y, z, m)
    __shared__ double4 tv[T];  // (vx, vy, vz, particle index)
    const int c = blockIdx.x % a.split;
    const int slab = blockIdx.x / a.split;
    int pi[K];
    bool active[K];
    double xi[K], yi[K], zi[K];
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const int slot = slab * (T * K) + (int)threadIdx.x + T * k;
        active[k] = slot < a.tgt.count;
        pi[k] = particle_of(a.tgt, active[k] ? slot : 0, a.P.n, a.flags);
        xi[k] = a.P.x[pi[k]]; yi[k] = a.P.y[pi[k]]; zi[k] = a.P.z[pi[k]];
    }
    const int j0 = c * a.chunk, j1 = min(a.src.count, j0 + a.chunk);
    for (int jt = j0; jt < j1; jt += T) {
        const int len = min(T, j1 - jt);
        __syncthreads();
        if ((int)threadIdx.x < len) {
            const int p = particle_of(a.src, jt + threadIdx.x, a.P.n, a.flags);
            tp[threadIdx.x] = make_double4(a.P.x[p], a.P.y[p], a.P.z[p], a.P.m[p]);
            tv[threadIdx.x] = make_double4(a.P.vx[p], a.P.vy[p], a.P.vz[p], (double)p);
        }
        __syncthreads();
        if (!(active[0])) continue;  // slots past the end come last
        for (int j = 0; j < len; ++j) {
            const double4 s = tp[j];
#pragma unroll
            for (int k = 0; k < K; ++k) {
                const double rx = s.x - xi[k], ry = s.y - yi[k], rz = s.z - zi[k];
                const double r2 = __builtin_fma(rx, rx, __builtin_fma(ry, ry, rz * rz));
                if (r2 >= a.r_max2 || !active[k]) continue;
                const double4 u = tv[j];
                const int pj = (int)u.w;
                const int i = pi[k];
                if (pj == i) continue;
                if (r2 == 0.0) {  // coincident: no orbit; reported, not linked
                    atomicOr(a.flags, BF_FLAG_COINCIDENT);
                    continue;
                }
                if (ngb_criterion(rx, ry, rz, u.x - a.P.vx[i], u.y - a.P.vy[i], u.z - a.P.vz[i],
                                  a.G * (a.P.m[i] + s.w), a)) {
                    const unsigned long long e = atomicAdd(a.count, 1ull);
                    if ((int64_t)e < a.cap) a.keys[e] = (unsigned long long)(uint32_t)i << 32 | (uint32_t)pj;
                }
            }
        }
    }
}

hipError_t launch_ngb(const NgbArgs& a, int waves, int nblocks, hipStream_t st) {
    if (waves == 4) hipLaunchKernelGGL((k_ngb<4, kNgbK>), dim3(nblocks), dim3(256), 0, st, a);
    else return hipErrorInvalidValue;
    return hipGetLastError();
}

size_t ngb_sort_tmp_bytes(int64_t m) {
    size_t bytes = 0;
    rocprim::radix_sort_keys(nullptr, bytes, (const unsigned long long*)nullptr, (unsigned long long*)nullptr,
                             (unsigned)std::max<int64_t>(m, 1), 0, 64, (hipStream_t)0);
    return bytes;
}

__global__ __launch_bounds__(256) void k_unpack_edges(const unsigned long long* keys, int64_t m, int32_t* edges) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= m) return;
    const unsigned long long k = keys[e];
    edges[2 * e] = (int32_t)(k >> 32);
    edges[2 * e + 1] = (int32_t)(k & 0xffffffffull);
}

hipError_t launch_ngb_finish(unsigned long long* keys_in, unsigned long long* keys_out, int64_t m, void* tmp,
                             size_t tmp_bytes, int32_t* edges, hipStream_t st) {
    if (m <= 0) return hipSuccess;
    size_t bytes = tmp_bytes;
    hipError_t e = rocprim::radix_sort_keys(tmp, bytes, keys_in, keys_out, (unsigned)m, 0, 64, st);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_unpack_edges, dim3((unsigned)((m + 255) / 256)), dim3(256), 0, st, keys_out, m, edges);
    return hipGetLastError();
}

// ---- subsystem labels ------------------------------------------------------------------------

__global__ __launch_bounds__(256) void k_label_init(int32_t* label, int64_t n, int32_t* word) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p == 0) *word = 0;
    if (p < n) label[p] = (int32_t)p;
}

__global__ __launch_bounds__(256) void k_label_edges(const int32_t* edges, int64_t m, int64_t n, int32_t* label,
                                                     int32_t* changed, uint32_t* flags) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= m) return;
    const int32_t i = edges[2 * e], j = edges[2 * e + 1];
    if (i < 0 || i >= n || j < 0 || j >= n) {
        atomicOr(flags, BF_FLAG_BADINDEX);
        return;
    }
    const int32_t li = label[i], lj = label[j];
    if (li < lj) {
        atomicMin(&label[j], li);
        *changed = 1;
    } else if (lj < li) {
        atomicMin(&label[i], lj);
        *changed = 1;
    }
}

__global__ __launch_bounds__(256) void k_label_jump(int32_t* label, int64_t n) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n) return;
    const int32_t l = label[p];
    const int32_t ll = label[l];
    if (ll < l) atomicMin(&label[p], ll);
}

__global__ __launch_bounds__(256) void k_clear_word(int32_t* w) { *w = 0; }

// components with at least two members: mark every label that some other particle carries
__global__ __launch_bounds__(256) void k_label_mark(const int32_t* label, int64_t n, int32_t* mark) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p < n && label[p] != (int32_t)p) mark[label[p]] = 1;
}

__global__ __launch_bounds__(256) void k_label_clear(int32_t* mark, int64_t n) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p < n) mark[p] = 0;
}

__global__ __launch_bounds__(256) void k_label_count(const int32_t* mark, int64_t n, int32_t* count) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p < n && mark[p]) atomicAdd(count, 1);
}

hipError_t launch_label_init(int32_t* label, int64_t n, int32_t* changed, hipStream_t st) {
    hipLaunchKernelGGL(k_label_init, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, label, n, changed);
    return hipGetLastError();
}

hipError_t launch_label_round(const int32_t* edges, int64_t m, int64_t n, int32_t* label, int32_t* changed,
                              uint32_t* flags, hipStream_t st) {
    hipLaunchKernelGGL(k_clear_word, dim3(1), dim3(1), 0, st, changed);
    if (m > 0)
        hipLaunchKernelGGL(k_label_edges, dim3((unsigned)((m + 255) / 256)), dim3(256), 0, st, edges, m, n, label,
                           changed, flags);
    hipLaunchKernelGGL(k_label_jump, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, label, n);
    return hipGetLastError();
}

hipError_t launch_label_count(const int32_t* label, int64_t n, int32_t* mark, int32_t* count, hipStream_t st) {
    const dim3 g((unsigned)((n + 255) / 256));
    hipLaunchKernelGGL(k_label_clear, g, dim3(256), 0, st, mark, n);
    hipLaunchKernelGGL(k_clear_word, dim3(1), dim3(1), 0, st, count);
    hipLaunchKernelGGL(k_label_mark, g, dim3(256), 0, st, label, n, mark);
    hipLaunchKernelGGL(k_label_count, g, dim3(256), 0, st, mark, n, count);
    return hipGetLastError();
}

}  // namespace bf
