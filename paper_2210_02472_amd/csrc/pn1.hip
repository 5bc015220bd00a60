// Global PN1.0 acceleration for pairs that involve a flagged massive particle (black hole),
// in FP64.  The pair set is {(i, j): i target, j source, j != i, i or j in the BH list}.
//  * k_pn_bh_sums:  for every BH b and source chunk, a workgroup sums the PN1.0 acceleration
//                   of b from all sources of the chunk (fixed-order LDS tree) -> partials, and
//                   records whether b is one of the chunk's sources;
//  * k_pn_targets:  which BHs are sources (a range test, or those records), then per target: a
//                   BH target adds its partials in chunk order, any other target sums over the
//                   BH sources directly.
// Two launches per pass.  Lists of more than kPnInLds BHs take two more (k_pn_clear and
// k_pn_flags mark the BH sources in memory).
#include "pair_ops.h"

namespace bf {

constexpr int kPnInLds = 4096;

__device__ __forceinline__ int32_t pn_particle(const DevSet& s, int32_t k, int64_t n, uint32_t* flags) {
    if (s.idx == nullptr) return s.begin + k;
    int32_t p = s.idx[k];
    if (p < 0 || p >= n) {
        atomicOr(flags, BF_FLAG_BADINDEX);
        p = 0;
    }
    return p;
}

// Two-body 1PN acceleration of i due to j (harmonic gauge), n = (x_i - x_j)/r, v_ij = v_i - v_j:
//   G m_j/(c^2 r^2) {[G(5 m_i + 4 m_j)/r + 3/2 (n.v_j)^2 - v_i^2 + 4 v_i.v_j - 2 v_j^2] n
//                    + [4 n.v_i - 3 n.v_j] v_ij}
__device__ __forceinline__ void pn_pair(const Masters& P, int i, int j, double G, double c2inv, double& sx,
                                        double& sy, double& sz, uint32_t* flags) {
    const double rx = P.x[i] - P.x[j], ry = P.y[i] - P.y[j], rz = P.z[i] - P.z[j];
    const double r2 = rx * rx + ry * ry + rz * rz;
    if (r2 == 0.0) {
        atomicOr(flags, BF_FLAG_COINCIDENT);
        return;
    }
    const double ir = rsqrt64(r2);
    const double nx = rx * ir, ny = ry * ir, nz = rz * ir;
    const double vix = P.vx[i], viy = P.vy[i], viz = P.vz[i];
    const double vjx = P.vx[j], vjy = P.vy[j], vjz = P.vz[j];
    const double vi2 = vix * vix + viy * viy + viz * viz;
    const double vj2 = vjx * vjx + vjy * vjy + vjz * vjz;
    const double vivj = vix * vjx + viy * vjy + viz * vjz;
    const double nvi = nx * vix + ny * viy + nz * viz;
    const double nvj = nx * vjx + ny * vjy + nz * vjz;
    const double A = G * (5.0 * P.m[i] + 4.0 * P.m[j]) * ir + 1.5 * nvj * nvj - vi2 + 4.0 * vivj - 2.0 * vj2;
    const double B = 4.0 * nvi - 3.0 * nvj;
    const double pre = G * P.m[j] * c2inv * ir * ir;
    sx += pre * (A * nx + B * (vix - vjx));
    sy += pre * (A * ny + B * (viy - vjy));
    sz += pre * (A * nz + B * (viz - vjz));
}

__global__ __launch_bounds__(256) void k_pn_flags(const PnArgs a) {
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (a.src.idx == nullptr) {
        if (q < a.nbh) {
            const int b = a.bh[q];
            a.bh_in_src[q] = (b >= a.src.begin && b < a.src.begin + a.src.count) ? 1 : 0;
        }
        return;
    }
    if (q >= a.src.count) return;
    const int p = pn_particle(a.src, q, a.P.n, a.flags);
    for (int k = 0; k < a.nbh; ++k)
        if (a.bh[k] == p) atomicMax(&a.bh_in_src[k], 1);
}

__global__ __launch_bounds__(256) void k_pn_clear(int32_t* v, int n) {
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q < n) v[q] = 0;
}

// grid (nchunk, nbh); 256 threads.  part: [nbh][nchunk][4], the fourth value 1 when b is one of
// the chunk's sources
__global__ __launch_bounds__(256) void k_pn_bh_sums(const PnArgs a) {
    __shared__ double red[3][256];
    const int kb = blockIdx.y;
    const int c = blockIdx.x;
    int b = a.bh[kb];
    if (b < 0 || b >= a.P.n) { if (threadIdx.x == 0) atomicOr(a.flags, BF_FLAG_BADINDEX); b = 0; }
    const int q0 = c * a.chunk;
    const int q1 = min(a.src.count, q0 + a.chunk);
    double sx = 0.0, sy = 0.0, sz = 0.0;
    int found = 0;
    for (int q = q0 + threadIdx.x; q < q1; q += 256) {
        const int j = pn_particle(a.src, q, a.P.n, a.flags);
        if (j == b) {
            found = 1;
            continue;
        }
        pn_pair(a.P, b, j, a.G, a.c2inv, sx, sy, sz, a.flags);
    }
    red[0][threadIdx.x] = sx; red[1][threadIdx.x] = sy; red[2][threadIdx.x] = sz;
    found = __syncthreads_or(found);
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) {
            red[0][threadIdx.x] += red[0][threadIdx.x + s];
            red[1][threadIdx.x] += red[1][threadIdx.x + s];
            red[2][threadIdx.x] += red[2][threadIdx.x + s];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        double* o = a.part + ((size_t)kb * a.nchunk + c) * 4;
        o[0] = red[0][0]; o[1] = red[1][0]; o[2] = red[2][0]; o[3] = found ? 1.0 : 0.0;
    }
}

__global__ __launch_bounds__(256) void k_pn_targets(const PnArgs a) {
    __shared__ int in_src[kPnInLds];  // which BHs are sources (lists of up to kPnInLds BHs)
    const bool lds = a.nbh <= kPnInLds;
    if (lds) {
        for (int kb = threadIdx.x; kb < a.nbh; kb += 256) {
            int v = 0;
            if (a.src.idx == nullptr) {
                const int b = a.bh[kb];
                v = b >= a.src.begin && b < a.src.begin + a.src.count;
            } else {
                for (int c = 0; c < a.nchunk; ++c) v |= a.part[((size_t)kb * a.nchunk + c) * 4 + 3] != 0.0;
            }
            in_src[kb] = v;
        }
        __syncthreads();
    }
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= a.tgt.count) return;
    const int i = pn_particle(a.tgt, k, a.P.n, a.flags);
    int self = -1;
    for (int kb = 0; kb < a.nbh; ++kb)
        if (a.bh[kb] == i) { self = kb; break; }
    double sx = 0.0, sy = 0.0, sz = 0.0;
    if (self >= 0) {
        for (int c = 0; c < a.nchunk; ++c) {
            const double* o = a.part + ((size_t)self * a.nchunk + c) * 4;
            sx += o[0]; sy += o[1]; sz += o[2];
        }
    } else {
        for (int kb = 0; kb < a.nbh; ++kb) {
            if (!(lds ? in_src[kb] : a.bh_in_src[kb])) continue;
            int j = a.bh[kb];
            if (j < 0 || j >= a.P.n) continue;  // flagged by k_pn_bh_sums
            pn_pair(a.P, i, j, a.G, a.c2inv, sx, sy, sz, a.flags);
        }
    }
    if (!__builtin_isfinite(sx) || !__builtin_isfinite(sy) || !__builtin_isfinite(sz))
        atomicOr(a.flags, BF_FLAG_NONFINITE);
    a.o0[i] = sx; a.o1[i] = sy; a.o2[i] = sz;
}

hipError_t launch_pn1(const PnArgs& a, hipStream_t st) {
    if (a.tgt.count <= 0) return hipSuccess;
    if (a.nbh > 0) {
        if (a.nbh > kPnInLds) {
            if (a.src.idx != nullptr) {
                hipLaunchKernelGGL(k_pn_clear, dim3((a.nbh + 255) / 256), dim3(256), 0, st, a.bh_in_src, a.nbh);
                if (a.src.count > 0)
                    hipLaunchKernelGGL(k_pn_flags, dim3((a.src.count + 255) / 256), dim3(256), 0, st, a);
            } else {
                hipLaunchKernelGGL(k_pn_flags, dim3((a.nbh + 255) / 256), dim3(256), 0, st, a);
            }
        }
        hipLaunchKernelGGL(k_pn_bh_sums, dim3(a.nchunk, a.nbh), dim3(256), 0, st, a);
    }
    hipLaunchKernelGGL(k_pn_targets, dim3((a.tgt.count + 255) / 256), dim3(256), 0, st, a);
    return hipGetLastError();
}

}  // namespace bf
