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

// 1/sqrt(r2) in FP64: the hardware estimate (about 24 correct bits) refined by one third-order
// step of y (1 - e)^(-1/2) = y (1 + e/2 + 3e^2/8 + ...), e = 1 - r2 y^2 (about 69 bits before
// rounding).  r2 = 0 (a coincident pair at eps = 0) gives NaN here ...
__device__ __forceinline__ double energy_rsqrt_raw(double r2) {
    const double y = __builtin_amdgcn_rsq(r2);
    const double h = r2 * y;
    const double e = __builtin_fma(-h, y, 1.0);
    const double t = __builtin_fma(e, 0.375, 0.5);
    return __builtin_fma(y * e, t, y);
}
// ... and 0 here: the pair is left out
__device__ __forceinline__ double energy_rsqrt(double r2) { return r2 > 0.0 ? energy_rsqrt_raw(r2) : 0.0; }

// (x, y, z, m) of set position k, packed for the pair kernel
__global__ __launch_bounds__(256) void k_energy_pack(const EnergyArgs e) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= e.set.count) return;
    const int32_t p = clamp_particle(e.set, k, e.P.n);
    e.pack[k] = make_double4(e.P.x[p], e.P.y[p], e.P.z[p], e.P.m[p]);
}

// Column data the same for every lane of a wavefront, read through the constant address space:
// the compiler issues scalar loads and the operands arrive in SGPRs (no LDS staging, no
// barrier).  The pack is not written while the pair kernel runs.
typedef const double __attribute__((address_space(4))) cdouble_e;
__device__ __forceinline__ double4 column(const double4* pack, int q) {
    const cdouble_e* f = (const cdouble_e*)(pack) + 4 * (size_t)q;
    return make_double4(f[0], f[1], f[2], f[3]);
}

// The potential U = -sum_{a<b} G m_a m_b / s_ab (Sec. 2.1) with every unordered pair evaluated
// once.  Set positions are cut into blocks of kEB = 512; workgroup w takes the w-th pair (rb, q)
// with q >= rb in row-major order: rows a of block rb (two per thread, a0 + t and a0 + t + 256)
// against the columns b > a of block q.  Only those pairs are launched, and short workgroups
// keep the chip filled to the end (chunks of 8,192 columns took 36 ms at N = 262,144, of 512
// 19 ms).  Every column, read through scalar loads, serves the thread's two rows.  Each row sums
// 64-column slices in plain FP64 and folds every slice into a compensated (Neumaier) row sum;
// the rows are added in a fixed tree and the workgroup writes part[w].  Workgroups with q == rb
// also write their rows' kinetic terms.
constexpr int kEB = 512, kER = 2;
static_assert(kEB == 256 * kER, "a workgroup's 256 threads cover its row block");

// (rb, q) of the w-th upper-triangular block pair of nb blocks: rows rb before hold
// nb + (nb - 1) + ... pairs
__device__ __forceinline__ void block_pair(int w, int nb, int& rb, int& q) {
    int lo = 0, hi = nb - 1;  // largest rb with first(rb) <= w, first(rb) = rb nb - rb (rb - 1) / 2
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        const long long first = (long long)mid * nb - (long long)mid * (mid - 1) / 2;
        if (first <= w) lo = mid;
        else hi = mid - 1;
    }
    rb = lo;
    q = rb + (int)(w - ((long long)rb * nb - (long long)rb * (rb - 1) / 2));
}

__global__ __launch_bounds__(256) void k_energy_pairs(const EnergyArgs e, int nb) {
    __shared__ double red[256];
    const int n = e.set.count;
    int rb, q;
    block_pair(blockIdx.x, nb, rb, q);
    const int a0 = rb * kEB, b0 = q * kEB, b1 = min(n, b0 + kEB);
    int a[kER];
#pragma unroll
    for (int r = 0; r < kER; ++r) a[r] = a0 + threadIdx.x + 256 * r;
    if (q == rb) {
#pragma unroll
        for (int r = 0; r < kER; ++r) {
            if (a[r] < n) {
                const int32_t p = clamp_particle(e.set, a[r], e.P.n);
                const double v2 = e.P.vx[p] * e.P.vx[p] + e.P.vy[p] * e.P.vy[p] + e.P.vz[p] * e.P.vz[p];
                e.kin[a[r]] = 0.5 * e.P.m[p] * v2;
            }
        }
    }
    double4 me[kER];
    double s[kER], c[kER];
#pragma unroll
    for (int r = 0; r < kER; ++r) {
        me[r] = e.pack[a[r] < n ? a[r] : n - 1];
        s[r] = c[r] = 0.0;
    }
    for (int j0 = b0; j0 < b1; j0 += 64) {
        double slice[kER];
#pragma unroll
        for (int r = 0; r < kER; ++r) slice[r] = 0.0;
        if (q > rb && b1 - j0 >= 64) {  // past every row of the block: every pair counts, unrolled
#pragma unroll 4
            for (int j = 0; j < 64; ++j) {
                const double4 o = column(e.pack, j0 + j);
#pragma unroll
                for (int r = 0; r < kER; ++r) {
                    const double dx = o.x - me[r].x, dy = o.y - me[r].y, dz = o.z - me[r].z;
                    const double r2 = __builtin_fma(dx, dx, __builtin_fma(dy, dy, __builtin_fma(dz, dz, e.eps2)));
                    slice[r] = __builtin_fma(o.w, energy_rsqrt_raw(r2), slice[r]);
                }
            }
            // a coincident pair made the slice NaN: that row's slice again, leaving the pair out
#pragma unroll
            for (int r = 0; r < kER; ++r) {
                if (__builtin_isfinite(slice[r])) continue;
                slice[r] = 0.0;
                for (int j = 0; j < 64; ++j) {
                    const double4 o = column(e.pack, j0 + j);
                    const double dx = o.x - me[r].x, dy = o.y - me[r].y, dz = o.z - me[r].z;
                    const double r2 = __builtin_fma(dx, dx, __builtin_fma(dy, dy, __builtin_fma(dz, dz, e.eps2)));
                    slice[r] = __builtin_fma(o.w, energy_rsqrt(r2), slice[r]);
                }
            }
        } else {  // the block's own rows or a ragged end: columns b > a only
            const int j1 = min(b1, j0 + 64);
            for (int j = j0; j < j1; ++j) {
                const double4 o = column(e.pack, j);
#pragma unroll
                for (int r = 0; r < kER; ++r) {
                    const double dx = o.x - me[r].x, dy = o.y - me[r].y, dz = o.z - me[r].z;
                    const double r2 = __builtin_fma(dx, dx, __builtin_fma(dy, dy, __builtin_fma(dz, dz, e.eps2)));
                    const double w = j > a[r] ? o.w : 0.0;
                    slice[r] = __builtin_fma(w, energy_rsqrt(r2), slice[r]);
                }
            }
        }
#pragma unroll
        for (int r = 0; r < kER; ++r) neumaier(s[r], c[r], slice[r]);
    }
    double row = 0.0;
#pragma unroll
    for (int r = 0; r < kER; ++r)
        if (a[r] < n) row += e.G * me[r].w * (s[r] + c[r]);
    red[threadIdx.x] = row;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) e.rows[blockIdx.x] = red[0];
}

// Single workgroup: compensated sums over fixed contiguous ranges of the workgroup partials and
// of the kinetic terms, then thread 0 combines them in order.  out[0] = kinetic, out[1] =
// potential = -(sum of the partials).
__global__ __launch_bounds__(1024) void k_energy_final(const EnergyArgs e, int nparts) {
    __shared__ double ps[1024], pc[1024], ks[1024], kc[1024];
    const int n = e.set.count;
    double s = 0.0, c = 0.0, s2 = 0.0, c2 = 0.0;
    {
        const int per = (nparts + 1023) / 1024;
        const int lo = threadIdx.x * per, hi = min(nparts, lo + per);
        for (int a = lo; a < hi; ++a) neumaier(s, c, e.rows[a]);
    }
    {
        const int per = (n + 1023) / 1024;
        const int lo = threadIdx.x * per, hi = min(n, lo + per);
        for (int a = lo; a < hi; ++a) neumaier(s2, c2, e.kin[a]);
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
        e.out[1] = -(S + C);
    }
}

int energy_partials(int n) {
    const long long nb = (n + kEB - 1) / kEB;
    return (int)(nb * (nb + 1) / 2);
}

hipError_t launch_energy(const EnergyArgs& e, hipStream_t st) {
    const int n = e.set.count;
    if (n <= 0) return hipSuccess;
    const int nb = (n + kEB - 1) / kEB;
    const int parts = energy_partials(n);
    hipLaunchKernelGGL(k_energy_pack, dim3((n + 255) / 256), dim3(256), 0, st, e);
    hipLaunchKernelGGL(k_energy_pairs, dim3(parts), dim3(256), 0, st, e, nb);
    hipLaunchKernelGGL(k_energy_final, dim3(1), dim3(1024), 0, st, e, parts);
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
