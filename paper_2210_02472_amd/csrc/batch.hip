// Batched ensembles of independent clusters in one persistent launch.
//
// Cluster c owns particles [coff[c], coff[c+1]) and active particles aidx[aoff[c] .. aoff[c+1]).
// A work item is (cluster, slab of 64*K*W active targets, chunk of `chunk` sources of that
// cluster); K, W and chunk are the launch shape (default 2, 4, 4096; tuned per size bucket).  k_batch_plan counts items per cluster and scans them (one workgroup); the persistent
// workgroups of k_batch_pairs pull items from an atomic counter until the queue is empty and
// write per-chunk partials; k_batch_reduce adds each target's chunks in chunk order.  Every
// item's result and output location are fixed, so the outcome does not depend on which
// workgroup ran it.  All sizes of the launches depend only on host-side bounds, so the whole
// sequence can be captured in a HIP graph and replayed while the offsets and lists change.
#include <algorithm>
#include <string>

#include "pair_ops.h"

namespace bf {

// default shape: 2 targets per lane, 4 waves per workgroup, 4096 sources per work item (16 tiles
// of 256); the sources per item are a multiple of every tile (64 W)
constexpr int kBatchChunk = 4096;
constexpr int kBK = 2, kBW = 4;

struct Batch {
    PairArgs base;        // masters, constants, flags; tgt/src/pack are set per item
    int32_t nclusters;
    const int64_t* coff;  // [nclusters + 1]
    const int32_t* aidx;  // active particle indices
    const int64_t* aoff;  // [nclusters + 1]
    int64_t max_active;
    int64_t max_cluster_n;
    int32_t max_chunks;
    int32_t pack_bytes;   // bytes per packed source
    int32_t kk, ww;       // targets per lane, waves per workgroup
    int32_t chunk;        // sources per work item
    int32_t slab;         // active targets per work item: 64 kk ww
    int32_t* item_off;    // [nclusters + 1]
    int32_t* counter;
    int32_t* bad;         // [nclusters] 1 if the cluster's offsets are invalid
    double* part;         // [max_chunks][NC][max_active]
    double *o0, *o1, *o2;
};

// cluster bounds with validation (invalid clusters are skipped and flagged)
__device__ __forceinline__ bool cluster_bounds(const Batch& b, int c, int64_t& cb, int64_t& ce, int64_t& a0,
                                               int64_t& a1) {
    cb = b.coff[c]; ce = b.coff[c + 1];
    a0 = b.aoff[c]; a1 = b.aoff[c + 1];
    return cb >= 0 && ce >= cb && ce <= b.base.P.n && ce - cb <= b.max_cluster_n && a0 >= 0 && a1 >= a0 &&
           a1 <= b.max_active;
}

// One workgroup of 1024 threads: per-cluster item counts, exclusive scan, reset of the queue.
__global__ __launch_bounds__(1024) void k_batch_plan(const Batch b) {
    __shared__ int32_t sums[1024];
    const int nc = b.nclusters;
    const int per = (nc + 1023) / 1024;
    const int lo = threadIdx.x * per, hi = min(nc, lo + per);
    int32_t s = 0;
    for (int c = lo; c < hi; ++c) {
        int64_t cb, ce, a0, a1;
        int32_t items = 0;
        const bool ok = cluster_bounds(b, c, cb, ce, a0, a1);
        if (!ok) atomicOr(b.base.flags, BF_FLAG_BADINDEX);
        b.bad[c] = ok ? 0 : 1;
        if (ok && a1 > a0 && ce > cb) {
            const int64_t nslab = (a1 - a0 + b.slab - 1) / b.slab;
            const int64_t nch = (ce - cb + b.chunk - 1) / b.chunk;
            items = (int32_t)(nslab * nch);
        }
        b.item_off[c] = items;  // counts for now
        s += items;
    }
    sums[threadIdx.x] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        int32_t run = 0;
        for (int t = 0; t < 1024; ++t) {
            const int32_t v = sums[t];
            sums[t] = run;
            run += v;
        }
        b.item_off[nc] = run;
        *b.counter = 0;
        *b.base.fix_count = 0;
    }
    __syncthreads();
    int32_t run = sums[threadIdx.x];
    for (int c = lo; c < hi; ++c) {
        const int32_t v = b.item_off[c];
        b.item_off[c] = run;
        run += v;
    }
}

template <class Op, int K, int W>
__global__ __launch_bounds__(64 * W) void k_batch_pairs(const Batch b) {
    __shared__ typename Op::Src tile[64 * W];
    __shared__ int32_t s_item;
    const int wave = threadIdx.x >> 6;
    const int32_t total = b.item_off[b.nclusters];
    for (;;) {
        __syncthreads();
        if (threadIdx.x == 0) s_item = atomicAdd(b.counter, 1);
        __syncthreads();
        const int32_t item = s_item;
        if (item >= total) break;
        // cluster of the item: largest c with item_off[c] <= item (empty clusters share offsets)
        int lo = 0, hi = b.nclusters - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (b.item_off[mid] <= item) lo = mid;
            else hi = mid - 1;
        }
        const int c = lo;
        int64_t cb, ce, a0, a1;
        cluster_bounds(b, c, cb, ce, a0, a1);  // validated by k_batch_plan (bad clusters have no items)
        const int32_t na = (int32_t)(a1 - a0), ns = (int32_t)(ce - cb);
        const int32_t nch = (ns + b.chunk - 1) / b.chunk;
        const int32_t local = item - b.item_off[c];
        const int32_t slab = local / nch, q = local % nch;
        PairArgs a = b.base;
        a.tgt = DevSet{b.aidx + a0, na, 0};
        a.src = DevSet{nullptr, ns, (int32_t)cb};
        a.pack = static_cast<const char*>(b.base.pack) + cb * b.pack_bytes;
        const int j0 = q * b.chunk;
        const int j1 = min(ns, j0 + b.chunk);
        typename Op::A64 acc[K];
        int slot[K], pidx[K];
        sweep<Op, K, W, false>(a, tile, slab * (64 * K * W) + wave * (64 * K), j0, j1, acc, slot, pidx);
#pragma unroll
        for (int k = 0; k < K; ++k) {
            if (slot[k] < na) {
                constexpr int NP = ncomp_of<Op>();
                double v[NP];
                Op::comps(acc[k], v);
#pragma unroll
                for (int comp = 0; comp < NP; ++comp)
                    b.part[((size_t)q * NP + comp) * b.max_active + a0 + slot[k]] = v[comp];
            }
        }
    }
}

template <int NP>
__global__ __launch_bounds__(256) void k_batch_reduce(const Batch b) {
    const int64_t a = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (a >= b.max_active) return;
    const int64_t atot = b.aoff[b.nclusters];
    if (a >= atot) return;
    int lo = 0, hi = b.nclusters - 1;  // cluster with aoff[c] <= a < aoff[c+1]
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (b.aoff[mid] <= a) lo = mid;
        else hi = mid - 1;
    }
    const int c = lo;
    if (b.bad[c]) return;
    int64_t cb, ce, a0, a1;
    cluster_bounds(b, c, cb, ce, a0, a1);
    if (a < a0 || a >= a1) return;
    const int32_t nch = (int32_t)((ce - cb + b.chunk - 1) / b.chunk);
    double v[NP];
#pragma unroll
    for (int comp = 0; comp < NP; ++comp) v[comp] = 0.0;
    for (int q = 0; q < nch; ++q)
#pragma unroll
        for (int comp = 0; comp < NP; ++comp) v[comp] += b.part[((size_t)q * NP + comp) * b.max_active + a];
    int32_t p = b.aidx[a];
    if (p < cb || p >= ce) {
        atomicOr(b.base.flags, BF_FLAG_BADINDEX);
        return;
    }
    if (!__builtin_isfinite(v[0]) || !__builtin_isfinite(v[1]) || !__builtin_isfinite(v[2]))
        atomicOr(b.base.flags, BF_FLAG_NONFINITE);
    b.o0[p] = v[0]; b.o1[p] = v[1]; b.o2[p] = v[2];
    if constexpr (NP == 4) {  // mixed: queue ill-conditioned targets for the FP64 fix-up
        const double ny = sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
        if (v[3] > b.base.cond_max * ny) {
            const int e = atomicAdd(b.base.fix_count, 1);
            if (e < b.max_active) b.base.fix_list[e] = (int32_t)a;
        }
    }
}

// FP64 re-evaluation of the queued active slots over their cluster's sources
template <int OP>
__global__ __launch_bounds__(256) void k_batch_fixup(const Batch b) {
    const int count = (int)min((int64_t)*b.base.fix_count, b.max_active);
    for (int e = blockIdx.x; e < count; e += gridDim.x) {
        const int32_t a = b.base.fix_list[e];
        int lo = 0, hi = b.nclusters - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (b.aoff[mid] <= a) lo = mid;
            else hi = mid - 1;
        }
        int64_t cb, ce, a0, a1;
        cluster_bounds(b, lo, cb, ce, a0, a1);  // queued slots come from valid clusters
        const int32_t p = b.aidx[a];            // checked by the reduction before queueing
        const DevSet src{nullptr, (int32_t)(ce - cb), (int32_t)cb};
        double r[3];
        fix_one<OP>(b.base.P, src, nullptr, p, b.base.G, b.base.eps2, b.base.flags, r);
        if (threadIdx.x == 0) { b.o0[p] = r[0]; b.o1[p] = r[1]; b.o2[p] = r[2]; }
        __syncthreads();
    }
}

// kick / drift of the active particles of every cluster
__global__ __launch_bounds__(256) void k_batch_kick(bf_state S, const Batch b, double h, const double* ax,
                                                    const double* ay, const double* az, double h2, const double* gx,
                                                    const double* gy, const double* gz) {
    const int64_t a = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (a >= b.max_active || a >= b.aoff[b.nclusters]) return;
    const int32_t p = b.aidx[a];
    if (p < 0 || p >= S.n) return;  // flagged by the reduction
    double kx = ax[p], ky = ay[p], kz = az[p];
    if (gx) {
        kx = __builtin_fma(h2, gx[p], kx);
        ky = __builtin_fma(h2, gy[p], ky);
        kz = __builtin_fma(h2, gz[p], kz);
    }
    S.vx[p] = __builtin_fma(h, kx, S.vx[p]);
    S.vy[p] = __builtin_fma(h, ky, S.vy[p]);
    S.vz[p] = __builtin_fma(h, kz, S.vz[p]);
}

__global__ __launch_bounds__(256) void k_batch_drift(bf_state S, const Batch b, double h) {
    const int64_t a = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (a >= b.max_active || a >= b.aoff[b.nclusters]) return;
    const int32_t p = b.aidx[a];
    if (p < 0 || p >= S.n) return;
    S.x[p] = __builtin_fma(h, S.vx[p], S.x[p]);
    S.y[p] = __builtin_fma(h, S.vy[p], S.y[p]);
    S.z[p] = __builtin_fma(h, S.vz[p], S.z[p]);
}

using BatchKernel = void (*)(const Batch);

// the shapes: K in {1, 2, 4} targets per lane, W in {4, 8} waves per workgroup
template <class Op>
static BatchKernel batch_kernel_of(int k, int w) {
#define BF_BK(K, W) \
    if (k == K && w == W) return k_batch_pairs<Op, K, W>;
    BF_BK(1, 4) BF_BK(2, 4) BF_BK(4, 4) BF_BK(1, 8) BF_BK(2, 8) BF_BK(4, 8)
#undef BF_BK
    return nullptr;
}

static BatchKernel batch_kernel(int op, int prec, int k, int w) {
    const bool mixed = prec == BF_PREC_MIXED;
    if (op == OP_ACC) return mixed ? batch_kernel_of<AccMixed>(k, w) : batch_kernel_of<Acc64>(k, w);
    if (op == OP_GRAD) return mixed ? batch_kernel_of<GradMixed>(k, w) : batch_kernel_of<Grad64>(k, w);
    return nullptr;
}

}  // namespace bf

bool bf_internal_batch_shape_ok(int op, int prec, int k, int waves, int chunk) {
    return bf::batch_kernel(op, prec, k, waves) != nullptr && chunk > 0 && chunk % (64 * waves) == 0 &&
           chunk <= (1 << 20);
}

namespace bf {

static hipError_t launch_batch_op(BatchKernel f, const Batch& b, int num_cu, hipStream_t st) {
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, reinterpret_cast<const void*>(f), 64 * b.ww, 0) !=
        hipSuccess)
        nb = 1;
    hipLaunchKernelGGL(f, dim3(num_cu * std::max(nb, 1)), dim3(64 * b.ww), 0, st, b);
    return hipGetLastError();
}

}  // namespace bf

// =============================================================================================
using namespace bf;

// Implemented in capi.hip: scratch growth and error recording shared with the other entry points.
int bf_internal_ensure(bf_ctx* ctx, int which, size_t need);
void* bf_internal_scratch(bf_ctx* ctx, int which);
int bf_internal_fail(int code, const char* msg);
void bf_internal_swap_scratch(bf_ctx* ctx, void* bufs[3], size_t bytes[3]);
std::pair<hipEvent_t, hipEvent_t> bf_internal_timer_begin(bf_ctx* c);
void bf_internal_timer_end(bf_ctx* c, int op, std::pair<hipEvent_t, hipEvent_t> ev);
int bf_internal_bucket(int64_t v);

// launch shape of a batched pass: forced, tuned for (active total, largest cluster), or the
// default
static KernelConfig batch_shape(bf_ctx* c, int op, int prec, int64_t max_active, int64_t max_cluster_n) {
    KernelConfig bc = c->batch_forced[op];
    if (bc.k == 0) {
        auto it = c->tuned.find(std::make_tuple(op, prec, (int)kTuneBatched, bf_internal_bucket(max_active),
                                                bf_internal_bucket(max_cluster_n)));
        if (it != c->tuned.end()) bc = it->second;
    }
    if (!bf_internal_batch_shape_ok(op, prec, bc.k, bc.waves, bc.split)) bc = KernelConfig{kBK, kBW, kBatchChunk};
    return bc;
}

static int batch_setup(bf_ctx* c, const bf_particles* P, int32_t nclusters, const int64_t* coff, const int32_t* aidx,
                       const int64_t* aoff, int64_t max_active, int64_t max_cluster_n, double G, double eps2, int prec,
                       double r_fb, int op, Batch& b) {
    if (!c || !P) return bf_internal_fail(BF_ERR_ARG, "NULL context or particles");
    if (P->n <= 0 || P->n > INT32_MAX || !P->x || !P->y || !P->z || !P->m)
        return bf_internal_fail(BF_ERR_ARG, "bad particle arrays");
    if (nclusters <= 0 || !coff || !aoff || (max_active > 0 && !aidx))
        return bf_internal_fail(BF_ERR_ARG, "bad cluster description");
    if (max_active < 0 || max_active > INT32_MAX || max_cluster_n <= 0 || max_cluster_n > P->n)
        return bf_internal_fail(BF_ERR_ARG, "bad bounds");
    if (prec != BF_PREC_FP64 && prec != BF_PREC_MIXED) return bf_internal_fail(BF_ERR_ARG, "bad prec");
    if (c->sub)
        return bf_internal_fail(BF_ERR_UNSUPPORTED, "batched ensembles take no subsystem exclusion "
                                                    "(clear it with bf_set_subsystems(ctx, NULL, 0))");
    if (!(eps2 >= 0 && eps2 < INFINITY) || !(r_fb >= 0 && r_fb < INFINITY) || !(G > -INFINITY && G < INFINITY))
        return bf_internal_fail(BF_ERR_ARG, "bad G, eps2 or r_fb");
    b = Batch{};
    b.base.P.x = P->x; b.base.P.y = P->y; b.base.P.z = P->z;
    b.base.P.vx = P->vx; b.base.P.vy = P->vy; b.base.P.vz = P->vz;
    b.base.P.m = P->m; b.base.P.n = P->n;
    b.base.G = G;
    b.base.eps2 = eps2;
    b.base.eps2f = (float)eps2 + 1e-20f;
    b.base.rfb2f = prec == BF_PREC_MIXED ? (float)(r_fb * r_fb) : -1.0f;
    b.base.split = 1;
    b.nclusters = nclusters;
    b.coff = coff; b.aidx = aidx; b.aoff = aoff;
    b.max_active = max_active;
    b.max_cluster_n = max_cluster_n;
    const KernelConfig bc = batch_shape(c, op, prec, max_active, max_cluster_n);
    b.kk = bc.k;
    b.ww = bc.waves;
    b.chunk = bc.split;
    b.slab = 64 * bc.k * bc.waves;
    b.max_chunks = (int32_t)((max_cluster_n + b.chunk - 1) / b.chunk);
    b.pack_bytes = pack_bytes(op, prec);
    const size_t pack_total = (size_t)P->n * b.pack_bytes;
    const size_t part_bytes = (size_t)b.max_chunks * stored_components(op, prec) *
                              std::max<int64_t>(max_active, 1) * sizeof(double);
    const size_t off_bytes = ((size_t)(2 * nclusters + 3 + std::max<int64_t>(max_active, 1)) * sizeof(int32_t) + 255) &
                             ~size_t(255);
    if (int rc = bf_internal_ensure(c, 2, pack_total)) return rc;
    if (int rc = bf_internal_ensure(c, 4, part_bytes + off_bytes)) return rc;
    b.base.pack = bf_internal_scratch(c, 2);
    char* s4 = static_cast<char*>(bf_internal_scratch(c, 4));
    b.part = reinterpret_cast<double*>(s4);
    b.item_off = reinterpret_cast<int32_t*>(s4 + part_bytes);
    b.counter = b.item_off + nclusters + 1;
    b.bad = b.counter + 1;
    b.base.fix_count = b.bad + nclusters;
    b.base.fix_list = b.base.fix_count + 1;
    b.base.cond_max = cond_max_for(op);
    return BF_OK;
}

// enqueue one batched pass (no allocation, no synchronisation: safe under stream capture)
static int batch_enqueue(bf_ctx* c, Batch& b, int op, int prec) {
    hipStream_t st = c->stream;
    // pack every particle (the clusters' source ranges are sub-ranges of this stream)
    PairArgs pk = b.base;
    pk.src = DevSet{nullptr, (int32_t)b.base.P.n, 0};
    hipError_t e = launch_pack(op, prec, pk, st);
    if (e != hipSuccess) return bf_internal_fail(BF_ERR_HIP, hipGetErrorString(e));
    hipLaunchKernelGGL(k_batch_plan, dim3(1), dim3(1024), 0, st, b);
    const bool mixed = prec == BF_PREC_MIXED;
    const BatchKernel f = batch_kernel(op, prec, b.kk, b.ww);
    if (!f) return bf_internal_fail(BF_ERR_UNSUPPORTED, "no batched kernel of this shape");
    const auto ev = bf_internal_timer_begin(c);  // the persistent pair kernel, when timing is on
    e = launch_batch_op(f, b, c->num_cu, st);
    if (e != hipSuccess) return bf_internal_fail(BF_ERR_HIP, hipGetErrorString(e));
    bf_internal_timer_end(c, op, ev);
    if (b.max_active > 0) {
        const dim3 g((unsigned)((b.max_active + 255) / 256));
        if (mixed) hipLaunchKernelGGL(k_batch_reduce<4>, g, dim3(256), 0, st, b);
        else hipLaunchKernelGGL(k_batch_reduce<3>, g, dim3(256), 0, st, b);
        if (mixed) {
            const unsigned nfix = (unsigned)std::min<int64_t>(b.max_active, 4 * c->num_cu);
            if (op == OP_ACC) hipLaunchKernelGGL(k_batch_fixup<OP_ACC>, dim3(nfix), dim3(256), 0, st, b);
            else hipLaunchKernelGGL(k_batch_fixup<OP_GRAD>, dim3(nfix), dim3(256), 0, st, b);
        }
    }
    e = hipGetLastError();
    if (e != hipSuccess) return bf_internal_fail(BF_ERR_HIP, hipGetErrorString(e));
    return BF_OK;
}

extern "C" {

BF_API int bf_query_batched_config(bf_ctx* c, int op, int prec, int64_t max_active, int64_t max_cluster_n, int* k,
                                   int* waves, int* chunk) {
    if (!c) return bf_internal_fail(BF_ERR_ARG, "NULL context");
    if (op != OP_ACC && op != OP_GRAD) return bf_internal_fail(BF_ERR_ARG, "BF_OP_FORCES or BF_OP_GRADIENT");
    if (prec != BF_PREC_FP64 && prec != BF_PREC_MIXED) return bf_internal_fail(BF_ERR_ARG, "bad prec");
    const KernelConfig bc = batch_shape(c, op, prec, max_active, max_cluster_n);
    if (k) *k = bc.k;
    if (waves) *waves = bc.waves;
    if (chunk) *chunk = bc.split;
    return BF_OK;
}

BF_API int bf_forces_batched(bf_ctx* c, const bf_particles* P, int32_t nclusters, const int64_t* coff,
                             const int32_t* aidx, const int64_t* aoff, int64_t max_active, int64_t max_cluster_n,
                             double G, double eps2, int prec, double r_fb, double* ax, double* ay, double* az) {
    Batch b{};
    if (int rc = batch_setup(c, P, nclusters, coff, aidx, aoff, max_active, max_cluster_n, G, eps2, prec, r_fb, OP_ACC, b))
        return rc;
    if (!ax || !ay || !az) return bf_internal_fail(BF_ERR_ARG, "output pointer NULL");
    b.base.flags = c->d_flags;
    b.o0 = ax; b.o1 = ay; b.o2 = az;
    return batch_enqueue(c, b, OP_ACC, prec);
}

BF_API int bf_force_gradient_batched(bf_ctx* c, const bf_particles* P, int32_t nclusters, const int64_t* coff,
                                     const int32_t* aidx, const int64_t* aoff, int64_t max_active,
                                     int64_t max_cluster_n, const double* ax, const double* ay, const double* az,
                                     double G, double eps2, int prec, double r_fb, double* gx, double* gy,
                                     double* gz) {
    Batch b{};
    if (int rc = batch_setup(c, P, nclusters, coff, aidx, aoff, max_active, max_cluster_n, G, eps2, prec, r_fb, OP_GRAD, b))
        return rc;
    if (!ax || !ay || !az || !gx || !gy || !gz) return bf_internal_fail(BF_ERR_ARG, "array pointer NULL");
    b.base.P.ax = ax; b.base.P.ay = ay; b.base.P.az = az;
    b.base.flags = c->d_flags;
    b.o0 = gx; b.o1 = gy; b.o2 = gz;
    return batch_enqueue(c, b, OP_GRAD, prec);
}

// A captured graph owns the scratch its kernels use, so later growth of the context's scratch
// can never leave a replay pointing at freed memory.

// prepare the two batch descriptors of a batched FSI cycle (sizes every scratch buffer)
static int batched_fsi_setup(bf_ctx* c, const bf_state* S, int32_t nclusters, const int64_t* coff, const int32_t* aidx,
                             const int64_t* aoff, int64_t max_active, int64_t max_cluster_n, double G, double eps2,
                             int prec, double r_fb, double dt, double* ax, double* ay, double* az, Batch& ba,
                             Batch& bg) {
    if (!S) return bf_internal_fail(BF_ERR_ARG, "NULL state");
    if (!S->x || !S->y || !S->z || !S->vx || !S->vy || !S->vz || !S->m) return bf_internal_fail(BF_ERR_ARG, "state NULL");
    if (!ax || !ay || !az) return bf_internal_fail(BF_ERR_ARG, "acceleration pointer NULL");
    if (!(dt > -INFINITY && dt < INFINITY)) return bf_internal_fail(BF_ERR_ARG, "dt not finite");
    bf_particles P{S->x, S->y, S->z, S->vx, S->vy, S->vz, S->m, S->n};
    // both passes share the pack and partial buffers: size them for both, then take the
    // gradient pass's pointers again (the acceleration sizing may have grown the buffers)
    if (int rc = batch_setup(c, &P, nclusters, coff, aidx, aoff, max_active, max_cluster_n, G, eps2, prec, r_fb, OP_GRAD, bg))
        return rc;
    if (int rc = batch_setup(c, &P, nclusters, coff, aidx, aoff, max_active, max_cluster_n, G, eps2, prec, r_fb, OP_ACC, ba))
        return rc;
    if (int rc = batch_setup(c, &P, nclusters, coff, aidx, aoff, max_active, max_cluster_n, G, eps2, prec, r_fb, OP_GRAD, bg))
        return rc;
    if (int rc = bf_internal_ensure(c, 3, (size_t)3 * S->n * sizeof(double))) return rc;
    double* gx = static_cast<double*>(bf_internal_scratch(c, 3));
    ba.base.flags = bg.base.flags = c->d_flags;
    ba.o0 = ax; ba.o1 = ay; ba.o2 = az;
    bg.base.P.ax = ax; bg.base.P.ay = ay; bg.base.P.az = az;
    bg.o0 = gx; bg.o1 = gx + S->n; bg.o2 = gx + 2 * S->n;
    return BF_OK;
}

// enqueue the FSI cycle of the active particles (no allocation, no synchronisation)
static int batched_fsi_enqueue(bf_ctx* c, const bf_state* S, Batch& ba, Batch& bg, int prec, double dt) {
    hipStream_t st = c->stream;
    const unsigned nb = (unsigned)std::max<int64_t>(1, (ba.max_active + 255) / 256);
    const double *ax = ba.o0, *ay = ba.o1, *az = ba.o2;
    const double *gx = bg.o0, *gy = bg.o1, *gz = bg.o2;
    const double* nul = nullptr;
    hipLaunchKernelGGL(k_batch_kick, dim3(nb), dim3(256), 0, st, *S, ba, dt / 6.0, ax, ay, az, 0.0, nul, nul, nul);
    hipLaunchKernelGGL(k_batch_drift, dim3(nb), dim3(256), 0, st, *S, ba, 0.5 * dt);
    if (int rc = batch_enqueue(c, ba, OP_ACC, prec)) return rc;
    if (int rc = batch_enqueue(c, bg, OP_GRAD, prec)) return rc;
    hipLaunchKernelGGL(k_batch_kick, dim3(nb), dim3(256), 0, st, *S, ba, 2.0 * dt / 3.0, ax, ay, az, dt * dt / 24.0, gx,
                       gy, gz);
    hipLaunchKernelGGL(k_batch_drift, dim3(nb), dim3(256), 0, st, *S, ba, 0.5 * dt);
    if (int rc = batch_enqueue(c, ba, OP_ACC, prec)) return rc;
    hipLaunchKernelGGL(k_batch_kick, dim3(nb), dim3(256), 0, st, *S, ba, dt / 6.0, ax, ay, az, 0.0, nul, nul, nul);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return bf_internal_fail(BF_ERR_HIP, hipGetErrorString(e));
    return BF_OK;
}

BF_API int bf_fsi_step_batched(bf_ctx* c, const bf_state* S, int32_t nclusters, const int64_t* coff,
                               const int32_t* aidx, const int64_t* aoff, int64_t max_active, int64_t max_cluster_n,
                               double G, double eps2, int prec, double r_fb, double dt, double* ax, double* ay,
                               double* az) {
    if (!c) return bf_internal_fail(BF_ERR_ARG, "NULL context");
    Batch ba{}, bg{};
    if (int rc = batched_fsi_setup(c, S, nclusters, coff, aidx, aoff, max_active, max_cluster_n, G, eps2, prec, r_fb, dt,
                                   ax, ay, az, ba, bg))
        return rc;
    return batched_fsi_enqueue(c, S, ba, bg, prec, dt);
}

BF_API int bf_graph_capture_batched_fsi(bf_ctx* c, const bf_state* S, int32_t nclusters, const int64_t* coff,
                                        const int32_t* aidx, const int64_t* aoff, int64_t max_active,
                                        int64_t max_cluster_n, double G, double eps2, int prec, double r_fb, double dt,
                                        double* ax, double* ay, double* az, void** graph_exec) {
    if (!c || !graph_exec) return bf_internal_fail(BF_ERR_ARG, "NULL context or graph pointer");
    *graph_exec = nullptr;
    // the graph gets fresh scratch buffers: park the context's own while they are allocated
    void* saved[3] = {nullptr, nullptr, nullptr};
    size_t saved_bytes[3] = {0, 0, 0};
    bf_internal_swap_scratch(c, saved, saved_bytes);
    Batch ba{}, bg{};
    if (int rc = batched_fsi_setup(c, S, nclusters, coff, aidx, aoff, max_active, max_cluster_n, G, eps2, prec, r_fb, dt,
                                   ax, ay, az, ba, bg)) {
        bf_internal_swap_scratch(c, saved, saved_bytes);  // context buffers back, graph ones out
        for (void* p : saved) if (p) hipFree(p);
        return rc;
    }
    void* mine[3];
    size_t mine_bytes[3];
    for (int i = 0; i < 3; ++i) { mine[i] = saved[i]; mine_bytes[i] = saved_bytes[i]; }
    bf_internal_swap_scratch(c, mine, mine_bytes);  // context has its buffers again; mine = graph's
    auto free_mine = [&]() { for (void* p : mine) if (p) hipFree(p); };
    hipStream_t user = c->stream;
    hipStream_t cap = nullptr;
    if (hipStreamCreateWithFlags(&cap, hipStreamNonBlocking) != hipSuccess) {
        free_mine();
        return bf_internal_fail(BF_ERR_HIP, "capture stream creation failed");
    }
    if (hipStreamSynchronize(user) != hipSuccess) {
        hipStreamDestroy(cap);
        free_mine();
        return bf_internal_fail(BF_ERR_HIP, "stream synchronisation failed");
    }
    int rc = BF_OK;
    hipError_t e = hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) {
        hipStreamDestroy(cap);
        free_mine();
        return bf_internal_fail(BF_ERR_HIP, hipGetErrorString(e));
    }
    c->stream = cap;
    c->capturing = true;  // no timing events inside the graph
    rc = batched_fsi_enqueue(c, S, ba, bg, prec, dt);
    c->capturing = false;
    c->stream = user;
    hipGraph_t g = nullptr;
    e = hipStreamEndCapture(cap, &g);
    hipStreamDestroy(cap);
    if (!rc && e != hipSuccess) rc = bf_internal_fail(BF_ERR_HIP, hipGetErrorString(e));
    if (rc) {
        if (g) hipGraphDestroy(g);
        free_mine();
        return rc;
    }
    bf_graph* h = new bf_graph();
    h->graph = g;
    for (int i = 0; i < 3; ++i) h->owned[i] = mine[i];
    if (hipGraphInstantiate(&h->exec, g, nullptr, nullptr, 0) != hipSuccess) {
        hipGraphDestroy(g);
        free_mine();
        delete h;
        return bf_internal_fail(BF_ERR_HIP, "graph instantiation failed");
    }
    *graph_exec = h;
    return BF_OK;
}

BF_API int bf_graph_launch(bf_ctx* c, void* graph_exec) {
    if (!c || !graph_exec) return bf_internal_fail(BF_ERR_ARG, "NULL context or graph");
    bf_graph* h = static_cast<bf_graph*>(graph_exec);
    hipError_t e = hipGraphLaunch(h->exec, c->stream);
    if (e != hipSuccess) return bf_internal_fail(BF_ERR_HIP, hipGetErrorString(e));
    return BF_OK;
}

BF_API int bf_graph_destroy(void* graph_exec) {
    if (!graph_exec) return BF_OK;
    bf_graph* h = static_cast<bf_graph*>(graph_exec);
    if (h->exec) hipGraphExecDestroy(h->exec);
    if (h->graph) hipGraphDestroy(h->graph);
    hipDeviceSynchronize();  // a replay may still be running on some stream
    for (void* p : h->owned)
        if (p) hipFree(p);
    delete h;
    return BF_OK;
}

}  // extern "C"
