// FP64 energy of a particle set, elementwise kicks and drifts, and index-list validation.
#include "bf_internal.h"

namespace bf {

__device__ __forceinline__ int32_t upd_particle(const DevSet& s, int32_t k, int64_t n, uint32_t* flags) {
    if (s.idx == nullptr) return s.begin + k;
    int32_t p = s.idx[k];
    if (p < 0 || p >= n) {
        atomicOr(flags, BF_FLAG_BADINDEX);
        return -1;
    }
    return p;
}

// list entries outside [0, n) read particle 0 (bf_energy validates lists before the launch)
__device__ __forceinline__ int32_t clamp_particle(const DevSet& s, int32_t k, int64_t n) {
    const int32_t p = s.idx ? s.idx[k] : s.begin + k;
    return (p < 0 || p >= n) ? 0 : p;
}

__device__ __forceinline__ void neumaier(double& s, double& c, double v) {
    const double t = s + v;
    c += (fabs(s) >= fabs(v)) ? ((s - t) + v) : ((v - t) + s);
    s = t;
}

// Row sums: rows[a] = m_a * sum_{b != a} G m_b / s_ab (every pair appears in two rows), and the
// kinetic terms.  One thread per row, sources staged through LDS in tiles of 256.
__global__ __launch_bounds__(256) void k_energy_rows(const EnergyArgs e) {
    __shared__ double4 tile[256];
    const int n = e.set.count;
    const int a = blockIdx.x * blockDim.x + threadIdx.x;
    const int ac = a < n ? a : n - 1;
    const int32_t p = clamp_particle(e.set, ac, e.P.n);
    const double xi = e.P.x[p], yi = e.P.y[p], zi = e.P.z[p];
    double s = 0.0, c = 0.0;
    for (int t0 = 0; t0 < n; t0 += 256) {
        const int len = min(256, n - t0);
        __syncthreads();
        if ((int)threadIdx.x < len) {
            const int q = t0 + threadIdx.x;
            const int32_t pj = clamp_particle(e.set, q, e.P.n);
            tile[threadIdx.x] = make_double4(e.P.x[pj], e.P.y[pj], e.P.z[pj], e.P.m[pj]);
        }
        __syncthreads();
        for (int j = 0; j < len; ++j) {
            if (t0 + j == a) continue;
            const double4 q = tile[j];
            const double dx = q.x - xi, dy = q.y - yi, dz = q.z - zi;
            const double r2 = dx * dx + dy * dy + dz * dz + e.eps2;
            if (r2 == 0.0) continue;
            neumaier(s, c, q.w / sqrt(r2));
        }
    }
    if (a < n) {
        e.rows[a] = e.G * e.P.m[p] * (s + c);
        const double v2 = e.P.vx[p] * e.P.vx[p] + e.P.vy[p] * e.P.vy[p] + e.P.vz[p] * e.P.vz[p];
        e.kin[a] = 0.5 * e.P.m[p] * v2;
    }
}

// Single workgroup: compensated sums over fixed contiguous ranges, then thread 0 combines them in
// order.  out[0] = kinetic, out[1] = potential = -1/2 sum rows.
__global__ __launch_bounds__(1024) void k_energy_final(const EnergyArgs e) {
    __shared__ double ps[1024], pc[1024], ks[1024], kc[1024];
    const int n = e.set.count;
    const int per = (n + 1023) / 1024;
    const int lo = threadIdx.x * per, hi = min(n, lo + per);
    double s = 0.0, c = 0.0, s2 = 0.0, c2 = 0.0;
    for (int a = lo; a < hi; ++a) {
        neumaier(s, c, e.rows[a]);
        neumaier(s2, c2, e.kin[a]);
    }
    ps[threadIdx.x] = s; pc[threadIdx.x] = c; ks[threadIdx.x] = s2; kc[threadIdx.x] = c2;
    __syncthreads();
    if (threadIdx.x == 0) {
        double S = 0.0, C = 0.0, K = 0.0, KC = 0.0;
        for (int t = 0; t < 1024; ++t) {
            neumaier(S, C, ps[t]);
            neumaier(S, C, pc[t]);
            neumaier(K, KC, ks[t]);
            neumaier(K, KC, kc[t]);
        }
        e.out[0] = K + KC;
        e.out[1] = -0.5 * (S + C);
    }
}

hipError_t launch_energy(const EnergyArgs& e, hipStream_t st) {
    const int n = e.set.count;
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_energy_rows, dim3((n + 255) / 256), dim3(256), 0, st, e);
    hipLaunchKernelGGL(k_energy_final, dim3(1), dim3(1024), 0, st, e);
    return hipGetLastError();
}

// v_i += h (a_i + h2 g_i); with drift, then x_i += hd v_i (the kick and the drift that follows it
// in the FSI cycle, one launch)
__global__ __launch_bounds__(256) void k_kick(bf_state S, DevSet set, double h, const double* __restrict__ ax,
                                              const double* __restrict__ ay, const double* __restrict__ az, double h2,
                                              const double* __restrict__ gx, const double* __restrict__ gy,
                                              const double* __restrict__ gz, bool drift, double hd, uint32_t* flags) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= set.count) return;
    const int p = upd_particle(set, k, S.n, flags);
    if (p < 0) return;
    double kx = ax[p], ky = ay[p], kz = az[p];
    if (gx) {
        kx = __builtin_fma(h2, gx[p], kx);
        ky = __builtin_fma(h2, gy[p], ky);
        kz = __builtin_fma(h2, gz[p], kz);
    }
    const double vx = __builtin_fma(h, kx, S.vx[p]), vy = __builtin_fma(h, ky, S.vy[p]),
                 vz = __builtin_fma(h, kz, S.vz[p]);
    S.vx[p] = vx;
    S.vy[p] = vy;
    S.vz[p] = vz;
    if (drift) {
        S.x[p] = __builtin_fma(hd, vx, S.x[p]);
        S.y[p] = __builtin_fma(hd, vy, S.y[p]);
        S.z[p] = __builtin_fma(hd, vz, S.z[p]);
    }
}

// x_i += h v_i
__global__ __launch_bounds__(256) void k_drift(bf_state S, DevSet set, double h, uint32_t* flags) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= set.count) return;
    const int p = upd_particle(set, k, S.n, flags);
    if (p < 0) return;
    S.x[p] = __builtin_fma(h, S.vx[p], S.x[p]);
    S.y[p] = __builtin_fma(h, S.vy[p], S.y[p]);
    S.z[p] = __builtin_fma(h, S.vz[p], S.z[p]);
}

__global__ __launch_bounds__(256) void k_validate(DevSet set, int64_t n, uint32_t* flags) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= set.count) return;
    const int32_t p = set.idx[k];
    if (p < 0 || p >= n) atomicOr(flags, BF_FLAG_BADINDEX);
}

hipError_t launch_kick(const bf_state& S, const DevSet& set, double h, const double* ax, const double* ay,
                       const double* az, double h2, const double* gx, const double* gy, const double* gz,
                       uint32_t* flags, hipStream_t st) {
    if (set.count <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_kick, dim3((set.count + 255) / 256), dim3(256), 0, st, S, set, h, ax, ay, az, h2, gx, gy,
                       gz, false, 0.0, flags);
    return hipGetLastError();
}

hipError_t launch_kick_drift(const bf_state& S, const DevSet& set, double h, const double* ax, const double* ay,
                             const double* az, double h2, const double* gx, const double* gy, const double* gz,
                             double hd, uint32_t* flags, hipStream_t st) {
    if (set.count <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_kick, dim3((set.count + 255) / 256), dim3(256), 0, st, S, set, h, ax, ay, az, h2, gx, gy,
                       gz, true, hd, flags);
    return hipGetLastError();
}

hipError_t launch_drift(const bf_state& S, const DevSet& set, double h, uint32_t* flags, hipStream_t st) {
    if (set.count <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_drift, dim3((set.count + 255) / 256), dim3(256), 0, st, S, set, h, flags);
    return hipGetLastError();
}

hipError_t launch_validate(const DevSet& set, int64_t n, uint32_t* flags, hipStream_t st) {
    if (set.count <= 0 || set.idx == nullptr) return hipSuccess;
    hipLaunchKernelGGL(k_validate, dim3((set.count + 255) / 256), dim3(256), 0, st, set, n, flags);
    return hipGetLastError();
}

}  // namespace bf
