// Time-step assignment epilogue and level partition.
//
//  * k_timestep: per target, the minimum of the pairwise free-fall / fly-by time-steps and the
//    per-particle gradient and jerk criteria (Sec. 3.5.4, Eqs. dt-nabla1, dt-nabla2; Sec. 3.5.5),
//    then the level of the power-of-two hierarchy: the smallest k with dt >= tau / 2^k
//    (Sec. 2.2: a particle is slow on a level when its time-step is at least the pivot).
//  * level partition: a stable radix sort of the set by level (levels are small integers), so
//    that every level, and every "level >= k" fast set, is a contiguous segment.
#include <rocprim/device/device_radix_sort.hpp>

#include "pair_ops.h"

namespace bf {

__global__ __launch_bounds__(256) void k_timestep(const TimestepArgs t) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= t.set.count) return;
    const int p = particle_of(t.set, k, t.P.n, t.flags);
    double dt = fmin(t.dt_ff[p], t.dt_fb[p]);
    const double v = sqrt(t.P.vx[p] * t.P.vx[p] + t.P.vy[p] * t.P.vy[p] + t.P.vz[p] * t.P.vz[p]);
    const double a = sqrt(t.ax[p] * t.ax[p] + t.ay[p] * t.ay[p] + t.az[p] * t.az[p]);
    if (t.gx) {
        // g' = Gsum / 24 (the gradient acceleration is a + eps^2 g')
        const double g = sqrt(t.gx[p] * t.gx[p] + t.gy[p] * t.gy[p] + t.gz[p] * t.gz[p]) / 24.0;
        if (t.eta_grad > 0.0 && g > 0.0) {
            dt = fmin(dt, t.eta_grad * cbrt(v / g));
            dt = fmin(dt, t.eta_grad * sqrt(a / g));
        }
    }
    if (t.jx && t.eta_jerk > 0.0) {
        const double j = sqrt(t.jx[p] * t.jx[p] + t.jy[p] * t.jy[p] + t.jz[p] * t.jz[p]);
        if (j > 0.0) dt = fmin(dt, t.eta_jerk * a / j);
    }
    // level: smallest k in [0, kmax] with dt >= tau 2^-k (exact powers of two)
    int lv = 0;
    while (lv < t.kmax && dt < ldexp(t.tau, -lv)) ++lv;
    if (__builtin_isnan(dt)) atomicOr(t.flags, BF_FLAG_NONFINITE);
    t.dt[p] = dt;
    if (t.level) t.level[p] = lv;
}

hipError_t launch_timestep(const TimestepArgs& t, hipStream_t st) {
    if (t.set.count <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_timestep, dim3((t.set.count + 255) / 256), dim3(256), 0, st, t);
    return hipGetLastError();
}

// ---- pivot split of one hierarchy level (adaptive HHS) ------------------------------------------
// flag[p] = 0 (slow) when the particle's time-step reaches the pivot tau, else 1 (fast).  The
// time-step is dt0[p], capped by dtl[p] (the time-step the level assigned from its own
// particles) when that is given; all_slow keeps every particle on this level (the deepest level).

__global__ __launch_bounds__(256) void k_pivot_flags(const DevSet set, int64_t n, const double* dt0, const double* dtl,
                                                     double tau, int all_slow, int32_t* flag, uint32_t* flags) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= set.count) return;
    const int p = particle_of(set, k, n, flags);
    double dt = dt0[p];
    if (dtl) dt = fmin(dt, dtl[p]);
    if (__builtin_isnan(dt)) atomicOr(flags, BF_FLAG_NONFINITE);
    flag[p] = (all_slow || dt >= tau) ? 0 : 1;
}

hipError_t launch_pivot_flags(const DevSet& set, int64_t n, const double* dt0, const double* dtl, double tau,
                              bool all_slow, int32_t* flag, uint32_t* flags, hipStream_t st) {
    if (set.count <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_pivot_flags, dim3((set.count + 255) / 256), dim3(256), 0, st, set, n, dt0, dtl, tau,
                       all_slow ? 1 : 0, flag, flags);
    return hipGetLastError();
}

// ---- level partition -------------------------------------------------------------------------

// Sort keys and the count per level.  The counts are gathered in an LDS histogram per
// workgroup and added to memory once per level and workgroup: one global atomic per particle
// on the same few addresses serialises (1.7 ms for 262,144 particles).  kmax <= 63.
__global__ __launch_bounds__(256) void k_level_keys(const DevSet set, int64_t n, const int32_t* level, int kmax,
                                                    uint32_t* keys, int32_t* vals, int32_t* counts, uint32_t* flags) {
    __shared__ int32_t hist[64];
    if ((int)threadIdx.x <= kmax) hist[threadIdx.x] = 0;
    __syncthreads();
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k < set.count) {
        const int p = particle_of(set, k, n, flags);
        int lv = level[p];
        if (lv < 0 || lv > kmax) {
            atomicOr(flags, BF_FLAG_BADINDEX);
            lv = lv < 0 ? 0 : kmax;
        }
        keys[k] = (uint32_t)lv;
        vals[k] = p;
        atomicAdd(&hist[lv], 1);
    }
    __syncthreads();
    if ((int)threadIdx.x <= kmax && hist[threadIdx.x] != 0) atomicAdd(&counts[threadIdx.x], hist[threadIdx.x]);
}

__global__ void k_clear_i32(int32_t* v, int n) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k < n) v[k] = 0;
}

// Is a new split of a set the same as the previous one?  cur and prev hold n and n_prev
// entries, the first counts[0] (device) and n0_prev (host) of them slow.  diff[0] = 1 if the slow
// parts differ, diff[1] = 1 if the whole lists differ (diff must be cleared before).
__global__ void k_split_diff(const int32_t* cur, int n, const int32_t* counts, const int32_t* prev, int n_prev,
                             int n0_prev, int32_t* diff) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    const int n0 = counts[0];
    if (k == 0) {
        if (n0 != n0_prev) diff[0] = 1;
        if (n0 != n0_prev || n != n_prev) diff[1] = 1;
    }
    if (k < n && k < n_prev && cur[k] != prev[k]) {
        if (k < n0) diff[0] = 1;
        diff[1] = 1;
    }
}

hipError_t launch_split_diff(const int32_t* cur, int n, const int32_t* counts, const int32_t* prev, int n_prev,
                             int n0_prev, int32_t* diff, hipStream_t st) {
    hipLaunchKernelGGL(k_clear_i32, dim3(1), dim3(64), 0, st, diff, 2);
    const int m = std::max(1, std::min(n, n_prev));
    hipLaunchKernelGGL(k_split_diff, dim3((m + 255) / 256), dim3(256), 0, st, cur, n, counts, prev, n_prev, n0_prev,
                       diff);
    return hipGetLastError();
}

size_t level_sort_tmp_bytes(int n) {
    size_t bytes = 0;
    rocprim::radix_sort_pairs(nullptr, bytes, (const uint32_t*)nullptr, (uint32_t*)nullptr, (const int32_t*)nullptr,
                              (int32_t*)nullptr, (unsigned)n, 0, 6, (hipStream_t)0);
    return bytes;
}

hipError_t launch_level_partition(const DevSet& set, int64_t n, const int32_t* level, int kmax, uint32_t* keys_in,
                                  uint32_t* keys_out, int32_t* vals_in, int32_t* out_order, int32_t* counts,
                                  void* tmp, size_t tmp_bytes, uint32_t* flags, hipStream_t st) {
    const int cnt = set.count;
    hipLaunchKernelGGL(k_clear_i32, dim3(1), dim3(64), 0, st, counts, kmax + 1);
    if (cnt <= 0) return hipGetLastError();
    hipLaunchKernelGGL(k_level_keys, dim3((cnt + 255) / 256), dim3(256), 0, st, set, n, level, kmax, keys_in, vals_in,
                       counts, flags);
    size_t bytes = tmp_bytes;
    hipError_t e = rocprim::radix_sort_pairs(tmp, bytes, keys_in, keys_out, vals_in, out_order, (unsigned)cnt, 0, 6, st);
    if (e != hipSuccess) return e;
    return hipGetLastError();
}

}  // namespace bf
