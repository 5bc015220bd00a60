// C ABI of libbifrost_hip: argument checks, context and scratch management, launch planning,
// the FSI cycle driver and the autotuner.  Every numerical step runs in the kernels of
// pairs.hip, pn1.hip, energy_update.hip and batch.hip.
#include <math.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <fstream>
#include <mutex>
#include <sstream>
#include <string>
#include <vector>

#include "bf_internal.h"

using namespace bf;

// ---- scratch of the allocation-free entry point (bf_forces_noalloc) -------------------------
// Every buffer of that entry point's pass is carved from this array; each device holds its own
// copy until the process ends.  On the host the name stands in for the array and is not a
// device address: bf_create resolves the address once per device, with that device current,
// and only that address is handed to kernels.
constexpr size_t kStaticScratchBytes = (size_t)64 << 20;
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

namespace {

thread_local std::string g_err;

int fail(int code, const std::string& msg) {
    g_err = msg;
    return code;
}

#define BF_HIP(call)                                                                         \
    do {                                                                                     \
        hipError_t e_ = (call);                                                              \
        if (e_ != hipSuccess)                                                                \
            return fail(BF_ERR_HIP, std::string(#call " failed: ") + hipGetErrorString(e_)); \
    } while (0)

bool finite_nonneg(double v) { return isfinite(v) && v >= 0.0; }

int check_set(const bf_set* s, int64_t n, const char* what) {
    if (!s) return fail(BF_ERR_ARG, std::string(what) + " set is NULL");
    if (s->count < 0) return fail(BF_ERR_ARG, std::string(what) + " count < 0");
    if (s->idx == nullptr) {
        if (s->begin < 0 || (int64_t)s->begin + s->count > n)
            return fail(BF_ERR_ARG, std::string(what) + " range outside [0, n)");
    }
    return BF_OK;
}

int check_particles(const bf_particles* P, bool need_v) {
    if (!P) return fail(BF_ERR_ARG, "particles NULL");
    if (P->n <= 0 || P->n > INT32_MAX) return fail(BF_ERR_ARG, "n must be in [1, 2^31)");
    if (!P->x || !P->y || !P->z || !P->m) return fail(BF_ERR_ARG, "position/mass pointer NULL");
    if (need_v && (!P->vx || !P->vy || !P->vz)) return fail(BF_ERR_ARG, "velocity pointer NULL");
    return BF_OK;
}

Masters masters_of(const bf_particles* P) {
    Masters M{};
    M.x = P->x; M.y = P->y; M.z = P->z;
    M.vx = P->vx; M.vy = P->vy; M.vz = P->vz;
    M.m = P->m;
    M.n = P->n;
    return M;
}

DevSet devset(const bf_set* s) { return DevSet{s->idx, s->count, s->begin}; }

// the static scratch's device address per device (resolved once, by bf_create)
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
bool g_scratch_done[kMaxDevices];
void* g_scratch_ptr[kMaxDevices];
hipError_t g_scratch_err[kMaxDevices];

void static_scratch_init(int device) {  // the device is current
    if (device < 0 || device >= kMaxDevices) return;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (g_scratch_done[device]) return;
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) (void)hipGetLastError();  // not left for the next launch check to report
    g_scratch_ptr[device] = e == hipSuccess ? ptr : nullptr;
    g_scratch_err[device] = e;
    g_scratch_done[device] = true;
}

void* static_scratch_of(int device, std::string* why) {
    if (device < 0 || device >= kMaxDevices) {
        *why = "device index beyond the static scratch table";
        return nullptr;
    }
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_done[device]) {
        *why = "static scratch not set up on this device";
        return nullptr;
    }
    if (!g_scratch_ptr[device]) *why = std::string("hipGetSymbolAddress failed: ") + hipGetErrorString(g_scratch_err[device]);
    return g_scratch_ptr[device];
}

int ensure(void** buf, size_t* have, size_t need, hipStream_t st) {
    if (need <= *have) return BF_OK;
    size_t want = std::max(need, *have + *have / 2);
    want = (want + 4095) & ~size_t(4095);
    if (*buf) {
        BF_HIP(hipStreamSynchronize(st));
        BF_HIP(hipFree(*buf));
        *buf = nullptr;
        *have = 0;
    }
    if (hipMalloc(buf, want) != hipSuccess) {
        *buf = nullptr;
        (void)hipGetLastError();  // not left for the next launch check to report
        return fail(BF_ERR_NOMEM, "scratch allocation of " + std::to_string(want) + " bytes failed");
    }
    *have = want;
    return BF_OK;
}

int ilog2_bucket(int64_t v) {
    int b = 0;
    while (v > 1) { v >>= 1; ++b; }
    return b;
}

// Default kernel shape: K targets per lane and W waves per workgroup.
KernelConfig default_config(int op, int prec, int64_t nt) {
    KernelConfig c;
    c.waves = 4;
    if (nt >= 64 * 2 * 4 * 512) c.k = 2;
    else c.k = 1;
    // mixed time-step passes: two targets per lane from 32,768 targets (5-8% faster at 32,768
    // and 131,072 targets against themselves; one is faster at 8,192)
    if (op == OP_DT && prec == BF_PREC_MIXED && nt >= 32768) c.k = 2;
    if (prec == BF_PREC_FP64 && op != OP_ACC) c.k = 1;
    return c;
}

struct Plan {
    KernelConfig cfg;
    int split = 1, chunk = 0, nblocks = 0;
};

// Spatially sorted mode: mixed acceleration / gradient passes on large enough sets.
// Below these sizes the sort, the tile packs and their launches cost more than the far tiles
// save (measured on a 262,144-body HHS interval, whose deep levels are small).
constexpr int64_t kSortMinSources = 16384, kSortMinTargets = 16384, kSortMinPairs = (int64_t)1 << 31;
// The two-set sweep replaces two directed passes and pays off from a quarter of that size.
constexpr int64_t kSortMinPairsBetween = kSortMinPairs / 4;
constexpr int64_t kAutoSplitCap = 32, kAutoChunkMin = 512;
// Up to these sizes a mixed unsorted pass runs as one launch of the small kernel (measured on
// the HHS levels: 5-20% faster per pass up to 4,221 bodies, slower from 8,176).
constexpr int64_t kSmallMaxTargets = 6144, kSmallMaxSources = 6144;
constexpr double kKappaMin = 0.5, kKappaMax = 64.0;
// Pair-symmetric sweep: its column partials take (n / 2048 + 1) * 16 bytes per particle
// (8.6 GB at n = 2^20); above this size the directed sorted sweep runs instead.
constexpr size_t kSymMaxScratch = (size_t)32 << 30;

bool same_set(const bf_set* t, const bf_set* s) {
    return t->idx == s->idx && t->count == s->count && (t->idx != nullptr || t->begin == s->begin);
}

// Shape of the pair-symmetric sweep of op over na rows and nb columns: forced, tuned for the
// size bucket, or the default (k = row tiles per wavefront, split = rounds of resident
// workgroups, 0 meaning kSymRounds).
KernelConfig sym_config(bf_ctx* ctx, int op, int64_t na, int64_t nb) {
    if (ctx->sym_forced[op].k) return ctx->sym_forced[op];
    auto it = ctx->tuned.find(std::make_tuple(op, (int)BF_PREC_MIXED, (int)kTuneSymmetric, ilog2_bucket(na),
                                              ilog2_bucket(nb)));
    if (it != ctx->tuned.end() && sym_variant_exists(op, it->second.waves, it->second.k)) return it->second;
    return KernelConfig{sym_default_rows(op), sym_default_waves(op), 0};
}

// One-set pair-symmetric sweeps run their distance shares in passes whose scratch fits the
// limit (kSymMaxScratch, or the context's): the share count grows until one share's column
// partials fit, and a pass takes as many shares as fit beside the running sums.  Scratch of a
// pass: [row sums of its shares | partials of its distances | running sums (several passes) |
// FP64 maxima (time-step)].
struct SymKind {
    int comps;         // components per particle
    size_t own_elem;   // bytes of a row sum and of a running sum
    size_t part_elem;  // bytes of a partial
    bool hi;           // time-step rates: the FP64 maxima of re-evaluated tiles
};
constexpr SymKind kSymMixed{4, sizeof(double), sizeof(float), false};
constexpr SymKind kSym64{3, sizeof(double), sizeof(double), false};
constexpr SymKind kSymDt{2, sizeof(float), sizeof(float), true};

struct SymPasses {
    int chunks = 1, chunk_len = 1, per_pass = 1, passes = 1;
    size_t own = 0, part = 0, acc = 0, hi = 0;  // region bytes, each a multiple of 256
    size_t total() const { return own + part + acc + hi; }
};

size_t align256(size_t b) { return (b + 255) & ~size_t(255); }

SymPasses sym_passes(bf_ctx* ctx, int64_t n, int chunks, const SymKind& k) {
    const int64_t n_tiles = (n + 63) / 64, n_pad = 64 * n_tiles;
    const int64_t nb = (n_tiles + kSymBlockTiles - 1) / kSymBlockTiles, D = nb / 2 + 1;
    const size_t limit = ctx->sym_limit ? ctx->sym_limit : kSymMaxScratch;
    const size_t per_d = (size_t)k.comps * n_pad * k.part_elem;   // one distance's partials
    const size_t per_c = (size_t)k.comps * n_pad * k.own_elem;    // one share's row sums
    const size_t acc = align256((size_t)k.comps * n_pad * k.own_elem);
    const size_t hi = k.hi ? align256((size_t)2 * n_pad * sizeof(double)) : 0;
    const size_t fixed = acc + hi + per_c + 512;
    const int64_t len_max = limit > fixed ? std::max<int64_t>(1, (int64_t)((limit - fixed) / per_d)) : 1;
    SymPasses sp;
    int64_t c = std::max<int64_t>(std::max(1, chunks), (D + len_max - 1) / len_max);
    c = std::min(c, D);
    sp.chunk_len = (int)((D + c - 1) / c);
    sp.chunks = (int)((D + sp.chunk_len - 1) / sp.chunk_len);
    const size_t one = align256(sp.chunks * per_c) + align256(D * per_d) + hi;
    if (one <= limit) {
        sp.per_pass = sp.chunks;
    } else {
        const size_t per_share = per_c + sp.chunk_len * per_d;
        sp.per_pass = (int)std::max<int64_t>(1, limit > acc + hi + 512 ? (int64_t)((limit - acc - hi - 512) / per_share) : 1);
        sp.per_pass = std::min(sp.per_pass, sp.chunks);
    }
    sp.passes = (sp.chunks + sp.per_pass - 1) / sp.per_pass;
    sp.own = align256(sp.per_pass * per_c);
    sp.part = align256(std::min<int64_t>(D, (int64_t)sp.per_pass * sp.chunk_len) * per_d);
    sp.acc = sp.passes > 1 ? acc : 0;
    sp.hi = hi;
    return sp;
}

// Default rounds of resident workgroups: 64.  At N = 2^20 the gradient sweep takes 414 ms with
// 2 rounds (1 share of the distances per row block), 396 ms with 4 (2 shares), 389 ms with 8,
// 381-383 ms with 16, 375 ms with 32 (16 shares) and 373 ms with 64 (32 shares); the
// acceleration 254, 246, 244, 240, 241 and 239 ms: the shares even out the workgroups' lengths
// and the last round is shorter.  The 262,144-body HHS interval takes the same time with 32 and
// 64 (258 ms without PN).
constexpr int kSymRounds = 64;

// resident workgroups the shares of a sweep aim at
int64_t sym_want(bf_ctx* ctx, int op, const KernelConfig& sc) {
    return (int64_t)(sc.split > 0 ? sc.split : kSymRounds) * ctx->num_cu * sym_blocks_per_cu(op, sc.waves, sc.k);
}

// Shares of the block distances per row block: at least the configured rounds of resident
// workgroups.
int sym_chunks(bf_ctx* ctx, int op, int64_t n, const KernelConfig& sc) {
    const int64_t n_tiles = (n + 63) / 64;
    const int64_t nb = (n_tiles + kSymBlockTiles - 1) / kSymBlockTiles;
    const int64_t want = sym_want(ctx, op, sc);
    return (int)std::max<int64_t>(1, std::min<int64_t>(nb / 2 + 1, (want + nb - 1) / nb));
}

// The one-set sweeps in the set's own order (FP64, time-step rates) need no sort; their
// smallest grain is one pair of 1,024-particle blocks per workgroup, about 0.27 ms, so below
// some 20,000 particles the directed pass is faster.  Measured (ms per pass, symmetric /
// directed): time-step rates 0.29 / 0.24 at 16,384, 0.59 / 0.76 at 32,768, 0.88 / 1.50 at
// 46,340; FP64 acceleration 0.30 / 0.20, 0.67 / 0.71, 1.07 / 1.39 (0.45 at 24,576 against
// about 0.42 directed).
constexpr int64_t kSymSetMin = 24576, kSym64Min = 32768;

// FP64 passes over one set: the symmetric sweep in the set's own order (no sort needed)
bool use_symmetric64(bf_ctx* ctx, int op, int prec, const bf_set* tg, const bf_set* sr) {
    const int64_t n = sr->count;
    return prec == BF_PREC_FP64 && (op == OP_ACC || op == OP_GRAD) && (ctx->sort_ops >> op & 1) &&
           !(ctx->sort_ops & BF_SORT_DIRECTED) && same_set(tg, sr) && ctx->sub == nullptr && n >= 64 &&
           ((ctx->sort_ops & BF_SORT_ANY_SIZE) || n >= kSym64Min);
}

int sym64_chunks(bf_ctx* ctx, int op, int64_t n) {
    const int64_t n_tiles = (n + 63) / 64;
    const int64_t nb = (n_tiles + kSymBlockTiles - 1) / kSymBlockTiles;
    const int64_t want = 2 * (int64_t)ctx->num_cu * sym64_blocks_per_cu(op);
    return (int)std::max<int64_t>(1, std::min<int64_t>(nb / 2 + 1, (want + nb - 1) / nb));
}

// Mixed time-step passes over one set, r_fb = 0: each unordered pair once, in the set's own order
bool use_symmetric_dt(bf_ctx* ctx, int op, int prec, const bf_set* tg, const bf_set* sr, double r_fb) {
    const int64_t n = sr->count;
    return op == OP_DT && prec == BF_PREC_MIXED && r_fb == 0.0 && (ctx->sort_ops >> OP_DT & 1) &&
           !(ctx->sort_ops & BF_SORT_DIRECTED) &&
           same_set(tg, sr) && ctx->sub == nullptr && n >= 64 &&
           ((ctx->sort_ops & BF_SORT_ANY_SIZE) || n >= kSymSetMin);
}

bool use_symmetric(bf_ctx* ctx, int op, bool sorted, const bf_set* tg, const bf_set* sr) {
    (void)ctx; (void)op;
    return sorted && !(ctx->sort_ops & BF_SORT_DIRECTED) && same_set(tg, sr);
}

bool use_sorted(bf_ctx* ctx, int op, int prec, int64_t nt, int64_t ns, double r_fb,
                int64_t min_pairs = kSortMinPairs) {
    return (ctx->sort_ops >> op & 1) && ctx->sub == nullptr && prec == BF_PREC_MIXED &&
           (op == OP_ACC || op == OP_GRAD) &&
           r_fb == 0.0 &&
           ((ctx->sort_ops & BF_SORT_ANY_SIZE) ||
            (ns >= kSortMinSources && nt >= kSortMinTargets && nt * ns >= min_pairs)) &&
           ns >= 64 && nt >= 64;
}

int plan(bf_ctx* ctx, int op, int prec, int64_t nt, int64_t ns, Plan& p, bool sorted = false) {
    KernelConfig c = ctx->forced[op][prec];
    if (c.k == 0) {
        auto it = ctx->tuned.find(std::make_tuple(op, prec, (int)kTuneDirected, ilog2_bucket(nt), ilog2_bucket(ns)));
        if (it != ctx->tuned.end()) c = it->second;
        else c = default_config(op, prec, nt);
        if (it == ctx->tuned.end() && sorted) c.k = 1;  // measured best for the sorted kernels
    }
    const bool excl = ctx->sub != nullptr && !sorted;
    if (excl) {  // the exclusion variants exist for 4 waves and 1 or 2 targets per lane
        c.waves = 4;
        c.k = std::min(c.k, 2);
    }
    if (!variant_exists(op, prec, c.k, c.waves, excl))
        return fail(BF_ERR_UNSUPPORTED, "no kernel variant for k=" + std::to_string(c.k) + " waves=" + std::to_string(c.waves));
    // Source chunks are whole groups of G sources: the LDS tile (T) in sorted mode, which walks
    // tiles; 64 in unsorted mode, whose sweep takes any chunk, so that passes over few sources
    // still split into enough workgroups.
    const int T = 64 * c.waves;
    const int G = sorted ? T : 64;
    const int64_t slab = (int64_t)64 * c.k * c.waves;
    const int64_t nslabs = std::max<int64_t>(1, (nt + slab - 1) / slab);
    const int64_t ntiles = std::max<int64_t>(1, (ns + G - 1) / G);
    int64_t split = c.split;
    if (split <= 0) {
        int bpc = sorted ? sorted_blocks_per_cu(op, c.k, c.waves) : variant_blocks_per_cu(op, prec, c.k, c.waves, excl);
        if (bpc <= 0) bpc = 1;
        const int64_t resident = (int64_t)ctx->num_cu * bpc;
        // At least four full rounds of resident workgroups.  The split is a multiple of the 8 XCDs
        // whenever there is enough work, so that (with round-robin dispatch) every workgroup on
        // one XCD streams the same source chunk and the chunk is served from that XCD's L2.
        const int64_t want = 4 * resident;
        split = (want + nslabs - 1) / nslabs;
        split = std::max<int64_t>(8, (split + 7) / 8 * 8);
        // unsorted passes over few targets: beyond max(32, ns / 512) chunks the partial sums
        // cost more than the extra workgroups gain (measured on the levels of a 262,144-body
        // HHS interval, 2,083 to 32,701 bodies, and on 6,554 targets x 65,536 sources)
        if (!sorted) split = std::min<int64_t>(split, std::max<int64_t>(kAutoSplitCap, ns / kAutoChunkMin));
    }
    split = std::min<int64_t>(split, ntiles);
    split = std::max<int64_t>(split, 1);
    // sources per chunk: whole groups
    const int64_t tiles_per_chunk = (ntiles + split - 1) / split;
    split = (ntiles + tiles_per_chunk - 1) / tiles_per_chunk;
    p.cfg = c;
    p.split = (int)split;
    p.chunk = (int)(tiles_per_chunk * G);
    if (nslabs * split > INT32_MAX) return fail(BF_ERR_UNSUPPORTED, "grid too large");
    p.nblocks = (int)(nslabs * split);
    return BF_OK;
}

// A fixed block of device memory that a pass takes all of its scratch from, instead of the
// context's buffers (which grow by allocation).
struct Arena {
    char* base;
    size_t bytes;
};
// fix-up partials of a pass run in an arena: 3 * kArenaFixCap doubles
constexpr int kArenaFixCap = 4 * kFixTiled;

// Lower a plan's source split to at most `most` chunks of whole 64-source groups (unsorted).
void cap_split(Plan& p, int64_t ns, int64_t most) {
    if (p.split <= most) return;
    const int64_t nslabs = p.nblocks / p.split;
    const int64_t ngroups = std::max<int64_t>(1, (ns + 63) / 64);
    const int64_t per = (ngroups + most - 1) / most;
    p.split = (int)((ngroups + per - 1) / per);
    p.chunk = (int)(per * 64);
    p.nblocks = (int)(nslabs * p.split);
}

// Run one pair pass (acc, grad or dt) end to end on the context stream.  With an arena the pass
// allocates nothing: it takes the unsorted directed sweep, carves every buffer from the arena
// (lowering the source split until the partials fit) and records no timing events.
int run_pairs(bf_ctx* ctx, int op, int prec, const Masters& M, const bf_set* tg, const bf_set* sr, double G, double eps2,
              double r_fb, double eta0, double eta1, double* o0, double* o1, double* o2,
              const Arena* arena = nullptr) {
    if (tg->count == 0) return BF_OK;
    if (ctx->sub && ctx->sub_n != M.n)
        return fail(BF_ERR_ARG, "subsystem labels were set for n=" + std::to_string(ctx->sub_n) +
                                    " particles, this pass has n=" + std::to_string(M.n));
    const bool sorted = !arena && use_sorted(ctx, op, prec, tg->count, sr->count, r_fb);
    Plan p;
    int rc = plan(ctx, op, prec, tg->count, sr->count, p, sorted);
    if (rc) return rc;
    if (sorted && !sorted_variant_exists(op, p.cfg.k, p.cfg.waves))
        return fail(BF_ERR_UNSUPPORTED, "no sorted kernel variant for this configuration");
    bool sym = !arena && use_symmetric(ctx, op, sorted, tg, sr);
    bool symdt = !arena && use_symmetric_dt(ctx, op, prec, tg, sr, r_fb);
    bool sym64 = !arena && use_symmetric64(ctx, op, prec, tg, sr);
    const KernelConfig sc = sym || symdt ? sym_config(ctx, op, sr->count, sr->count) : KernelConfig{};
    SymPasses sp;
    if (sym || symdt || sym64) {
        // the column partials are large (8.6 GB in one pass at n = 2^20): without the memory,
        // the directed sweep runs instead
        const int shares = sym64 ? sym64_chunks(ctx, op, sr->count) : sym_chunks(ctx, op, sr->count, sc);
        sp = sym_passes(ctx, sr->count, shares, sym64 ? kSym64 : symdt ? kSymDt : kSymMixed);
        if (ensure(&ctx->scratch9, &ctx->scratch9_bytes, sp.total(), ctx->stream)) {
            g_err.clear();
            sym = symdt = sym64 = false;
        }
    }
    // few targets and sources, mixed, unsorted, no exclusion or close-pair re-evaluation, no
    // forced or tuned configuration: the one-launch small kernel
    const bool small = !sorted && !sym && !sym64 && prec == BF_PREC_MIXED && (op == OP_ACC || op == OP_GRAD) &&
                       ctx->sub == nullptr && r_fb == 0.0 && tg->count <= kSmallMaxTargets &&
                       sr->count <= kSmallMaxSources && ctx->forced[op][prec].k == 0 &&
                       ctx->tuned.find(std::make_tuple(op, prec, (int)kTuneDirected, ilog2_bucket(tg->count),
                                                       ilog2_bucket(sr->count))) == ctx->tuned.end();
    // the same for FP64 passes: one launch, sources straight from the masters, no pack
    const bool small64 = !sorted && !sym && !sym64 && prec == BF_PREC_FP64 && (op == OP_ACC || op == OP_GRAD) &&
                         ctx->sub == nullptr && tg->count <= kSmallMaxTargets && sr->count <= kSmallMaxSources &&
                         ctx->forced[op][prec].k == 0 &&
                         ctx->tuned.find(std::make_tuple(op, prec, (int)kTuneDirected, ilog2_bucket(tg->count),
                                                         ilog2_bucket(sr->count))) == ctx->tuned.end();
    if (sym || sym64 || symdt || small || small64) p.split = 1;  // no source split in memory
    // scratch: [fix counter | fix list (one slot per target)], the split partials, the packed
    // sources (unsorted) and the fix-up partials: from the context's buffers, or the arena
    const bool fix = prec == BF_PREC_MIXED && op != OP_DT;
    const size_t head = 256 + (((size_t)tg->count * sizeof(int32_t) + 255) & ~size_t(255));
    const size_t chunk_bytes = (size_t)stored_components(op, prec) * tg->count * sizeof(double);
    char* head_buf = nullptr;
    double* part_buf = nullptr;
    void* pack_buf = nullptr;
    double* fix_buf = nullptr;
    int fix_cap = kFixChunks * kFixTiled;
    if (arena) {
        // [head | packed sources | fix-up partials | split partials], each 256-byte aligned
        const size_t pack = (((size_t)sr->count * pack_bytes(op, prec)) + 255) & ~size_t(255);
        const size_t fixb = fix ? (size_t)3 * kArenaFixCap * sizeof(double) : 0;
        const size_t fixed = head + pack + fixb;
        if (fixed > arena->bytes)
            return fail(BF_ERR_ARG, "the pass needs " + std::to_string(fixed) + " bytes of scratch; the static buffer holds " +
                                        std::to_string(arena->bytes));
        if (p.split > 1) cap_split(p, sr->count, (int64_t)std::max<size_t>(1, (arena->bytes - fixed) / chunk_bytes));
        head_buf = arena->base;
        pack_buf = arena->base + head;
        fix_buf = reinterpret_cast<double*>(arena->base + head + pack);
        fix_cap = kArenaFixCap;
        part_buf = reinterpret_cast<double*>(arena->base + fixed);
    } else {
        const size_t part_bytes = p.split > 1 ? (size_t)p.split * chunk_bytes : 0;
        rc = ensure(&ctx->scratch, &ctx->scratch_bytes, head + part_bytes, ctx->stream);
        if (rc) return rc;
        if (fix) {
            rc = ensure(&ctx->scratch8, &ctx->scratch8_bytes, (size_t)kFixChunks * 3 * kFixTiled * sizeof(double),
                        ctx->stream);
            if (rc) return rc;
        }
        if (!sorted && !small64 && sr->count > 0) {
            rc = ensure(&ctx->scratch2, &ctx->scratch2_bytes, (size_t)sr->count * pack_bytes(op, prec), ctx->stream);
            if (rc) return rc;
        }
    }
    PairArgs a{};
    a.P = M;
    a.tgt = devset(tg);
    a.src = devset(sr);
    a.G = G;
    a.eps2 = eps2;
    a.eps2f = (float)eps2 + 1e-20f;
    float rfb2 = (float)(r_fb * r_fb);
    if (op == OP_DT) rfb2 = std::max(rfb2, 1e-30f);  // coincident pairs of the FP32 time-step pass
    a.rfb2f = prec == BF_PREC_MIXED ? rfb2 : -1.0f;
    a.split = p.split;
    a.chunk = p.chunk;
    a.eta0 = eta0;
    a.eta1 = eta1;
    a.o0 = o0; a.o1 = o1; a.o2 = o2;
    a.flags = ctx->d_flags;
    a.cond_max = cond_max_for(op);
    a.sub = ctx->sub;
    // sorted mode: sort lists and temporaries, near and far streams, tile metadata
    const int64_t s_nt = tg->count, s_ns = sr->count, s_nmax = std::max(s_nt, s_ns);
    const size_t s_tmp = sorted ? sort_tmp_bytes((int)s_nmax) : 0;
    const size_t s_list = ((size_t)s_nmax * 4 + 255) & ~size_t(255);
    const int s_waves = sym ? 1 : p.cfg.waves;  // the symmetric sweep packs tiles of 64
    const int64_t s_ntiles = (s_ns + 64 * s_waves - 1) / (64 * s_waves);
    const int s_kmeta = op == OP_GRAD ? 2 : 1;
    const size_t s_far = (((size_t)s_ns * (op == OP_GRAD ? 32 : 16)) + 255) & ~size_t(255);
    if (sorted) {
        rc = ensure(&ctx->scratch5, &ctx->scratch5_bytes, 256 + 6 * s_list + ((s_tmp + 255) & ~size_t(255)),
                    ctx->stream);
        if (rc) return rc;
        rc = ensure(&ctx->scratch2, &ctx->scratch2_bytes, (size_t)s_ns * pack_bytes(op, prec), ctx->stream);
        if (rc) return rc;
        rc = ensure(&ctx->scratch6, &ctx->scratch6_bytes, s_far + (size_t)s_ntiles * s_kmeta * sizeof(double4),
                    ctx->stream);
        if (rc) return rc;
    }
    if (ctx->dry) return BF_OK;  // sizing before a capture: every buffer of this pass now exists
    if (!arena) {
        head_buf = static_cast<char*>(ctx->scratch);
        part_buf = reinterpret_cast<double*>(head_buf + head);
        pack_buf = ctx->scratch2;
        fix_buf = static_cast<double*>(ctx->scratch8);
    }
    a.fix_count = reinterpret_cast<int32_t*>(head_buf);
    a.fix_list = reinterpret_cast<int32_t*>(head_buf + 256);
    if (p.split > 1) a.part = part_buf;
    a.tile_stats = ctx->d_stats + 1;
    a.pass_stats = ctx->d_stats;
    const bool pack_begins = !sorted && !small64 && sr->count > 0;  // the pack kernel starts the pass
    // (the FP64 one-launch kernel clears the pass statistics itself)
    if (!pack_begins && !small64) BF_HIP(launch_pass_begin(fix ? a.fix_count : nullptr, ctx->d_stats, ctx->stream));
    SymArgs g{};
    if (sorted) {
        // order targets and sources along a Morton curve, then pack the sorted sources into tiles
        const int64_t nt = s_nt, ns = s_ns;
        const size_t tmp = s_tmp, list_bytes = s_list;
        char* b5 = static_cast<char*>(ctx->scratch5);
        SortBuffers sb;
        sb.bbox = reinterpret_cast<uint32_t*>(b5);
        sb.keys_in = reinterpret_cast<uint32_t*>(b5 + 256);
        sb.keys_out = reinterpret_cast<uint32_t*>(b5 + 256 + list_bytes);
        sb.vals_in = reinterpret_cast<int32_t*>(b5 + 256 + 2 * list_bytes);
        sb.vals_out = reinterpret_cast<int32_t*>(b5 + 256 + 3 * list_bytes);
        int32_t* src_sorted = reinterpret_cast<int32_t*>(b5 + 256 + 4 * list_bytes);
        int32_t* tgt_sorted = reinterpret_cast<int32_t*>(b5 + 256 + 5 * list_bytes);
        sb.tmp = b5 + 256 + 6 * list_bytes;
        sb.tmp_bytes = tmp;
        const DevSet ds = devset(sr), dt = devset(tg);
        BF_HIP(launch_sort_set(M, ds, ds, sb, src_sorted, ctx->d_flags, ctx->stream, ctx->capturing));
        const bool same = same_set(tg, sr);
        if (!same) BF_HIP(launch_sort_set(M, dt, ds, sb, tgt_sorted, ctx->d_flags, ctx->stream, ctx->capturing));
        a.src = DevSet{src_sorted, (int32_t)ns, 0};
        a.tgt = DevSet{same ? src_sorted : tgt_sorted, (int32_t)nt, 0};
        const int tile_waves = s_waves;
        const int64_t ntiles = s_ntiles;
        const size_t far_bytes = s_far;
        a.pack = ctx->scratch2;
        a.pack_far = ctx->scratch6;
        a.tile_meta = reinterpret_cast<const double4*>(static_cast<char*>(ctx->scratch6) + far_bytes);
        a.kappa = ctx->kappa;
        BF_HIP(launch_pack_tiles(op, tile_waves, a, ctx->scratch2, ctx->scratch6,
                                 reinterpret_cast<double4*>(static_cast<char*>(ctx->scratch6) + far_bytes), ctx->stream));
        if (sym) {
            g.near_pack = a.pack;
            g.far_pack = a.pack_far;
            g.tile_meta = a.tile_meta;
            g.row_pack = a.pack;
            g.n = g.n_rows = (int32_t)ns;
            g.n_tiles = g.n_row_tiles = (int32_t)ntiles;
            g.n_blocks = (int32_t)((ntiles + kSymBlockTiles - 1) / kSymBlockTiles);
            g.n_pad = g.n_row_pad = (int32_t)(64 * ntiles);
            g.between = 0;
            g.eps2f = a.eps2f;
            g.kappa = a.kappa;
            g.tile_stats = a.tile_stats;
        }
    } else if (sr->count > 0 && !small64) {
        a.pack = pack_buf;
        BF_HIP(launch_pack(op, prec, a, ctx->stream, fix ? 2 : 1));
        if (sym64) {  // rows and columns: the FP64 pack in the set's order
            const int64_t ns = sr->count, ntiles = (ns + 63) / 64;
            g.near_pack = g.row_pack = a.pack;
            g.n = g.n_rows = (int32_t)ns;
            g.n_tiles = g.n_row_tiles = (int32_t)ntiles;
            g.n_blocks = (int32_t)((ntiles + kSymBlockTiles - 1) / kSymBlockTiles);
            g.n_pad = g.n_row_pad = (int32_t)(64 * ntiles);
            g.between = 0;
        }
        if (symdt) {  // rows and columns: the time-step pack in the set's order
            const int64_t ns = sr->count, ntiles = (ns + 63) / 64;
            g.near_pack = g.row_pack = a.pack;
            g.n = g.n_rows = (int32_t)ns;
            g.n_tiles = g.n_row_tiles = (int32_t)ntiles;
            g.n_blocks = (int32_t)((ntiles + kSymBlockTiles - 1) / kSymBlockTiles);
            g.n_pad = g.n_row_pad = (int32_t)(64 * ntiles);
            g.between = 0;
            g.m = M.m;
            g.G = G;
            g.flags = ctx->d_flags;
        }
    }
    if (sym || sym64 || symdt) {  // the shares and the scratch regions of the passes
        char* base = static_cast<char*>(ctx->scratch9);
        g.n_chunks = sp.chunks;
        g.chunk_len = sp.chunk_len;
        g.own = reinterpret_cast<double*>(base);  // the time-step sweep keeps floats
        g.part = reinterpret_cast<float*>(base + sp.own);
        g.acc = sp.acc ? reinterpret_cast<double*>(base + sp.own + sp.part) : nullptr;
        g.hi = sp.hi ? reinterpret_cast<double*>(base + sp.own + sp.part + sp.acc) : nullptr;
    }
    // pass q of the shares
    auto sym_pass = [&](int q) {
        g.chunk0 = q * sp.per_pass;
        g.pass_chunks = std::min(sp.per_pass, sp.chunks - g.chunk0);
        g.d_base = g.chunk0 * sp.chunk_len;
        g.first = q == 0;
        g.last = q == sp.passes - 1;
    };
    std::pair<hipEvent_t, hipEvent_t> ev{nullptr, nullptr};
    const bool timed = ctx->timing && !ctx->capturing && !arena;
    if (timed) {
        if (!ctx->tpool.empty()) {
            ev = ctx->tpool.back();
            ctx->tpool.pop_back();
        } else {
            BF_HIP(hipEventCreate(&ev.first));
            BF_HIP(hipEventCreate(&ev.second));
        }
        BF_HIP(hipEventRecord(ev.first, ctx->stream));
    }
    if (sym || symdt || sym64) {
        // every pass but the last adds its partials onto the running sums between the sweeps
        for (int q = 0; q < sp.passes; ++q) {
            sym_pass(q);
            if (sym64) BF_HIP(launch_pairs_sym64(op, g, eps2 + 1e-150 /* the FP64 kernels' tiny */, ctx->stream));
            else BF_HIP(launch_pairs_sym(op, sc.waves, sc.k, g, ctx->stream));
            if (q + 1 < sp.passes) {
                if (sym64) BF_HIP(launch_sym_reduce64(op, a, g, ctx->stream));
                else BF_HIP(launch_sym_reduce(op, a, g, ctx->stream));
            }
        }
    } else if (sorted) BF_HIP(launch_pairs_sorted(op, p.cfg, a, p.nblocks, ctx->stream));
    else if (small) BF_HIP(launch_pairs_small(op, a, ctx->stream));
    else if (small64) BF_HIP(launch_pairs_small64(op, a, ctx->stream));
    else BF_HIP(launch_pairs(op, prec, p.cfg, a, p.nblocks, ctx->stream));
    // credit: every (target, source) pair, less the self-pairs when targets and sources are one set
    ctx->pair_credit[op] += (int64_t)tg->count * (same_set(tg, sr) ? sr->count - 1 : sr->count);
    ctx->last_kind = sym || sym64 || symdt ? BF_PASS_SYMMETRIC : sorted ? BF_PASS_SORTED : BF_PASS_UNSORTED;
    ctx->last_k = sym || symdt ? sc.k : sym64 ? 4 : small || small64 ? 1 : p.cfg.k;
    ctx->last_waves = sym || symdt ? sc.waves : sym64 ? 4 : small || small64 ? 16 : p.cfg.waves;
    ctx->last_split = sym || sym64 || symdt ? g.n_chunks : p.split;
    ctx->last_passes = sym || sym64 || symdt ? sp.passes : 1;
    if (timed) {
        BF_HIP(hipEventRecord(ev.second, ctx->stream));
        ctx->tev[op].push_back(ev);
    }
    if (sym || symdt) BF_HIP(launch_sym_reduce(op, a, g, ctx->stream));
    else if (sym64) BF_HIP(launch_sym_reduce64(op, a, g, ctx->stream));
    else if (p.split > 1) BF_HIP(launch_reduce(op, prec, a, ctx->stream));
    if (fix) BF_HIP(launch_fixup(op, a, fix_buf, fix_cap, ctx->num_cu, ctx->stream));
    return BF_OK;
}

// Both inter-set passes A <- B and B <- A (Sec. 2.2: the inter-level sums of the hierarchy are
// the same pairs seen from either side), written into the same particle-indexed outputs.  When
// the spatially sorted mode applies to both and the sets are disjoint (the caller's guarantee),
// one two-set symmetric sweep evaluates every pair (a, b) once; otherwise two passes run.
int run_pairs_between(bf_ctx* ctx, int op, int prec, const Masters& M, const bf_set* A, const bf_set* B, double G,
                      double eps2, double r_fb, double* o0, double* o1, double* o2) {
    auto two_passes = [&]() -> int {
        if (int rc = run_pairs(ctx, op, prec, M, A, B, G, eps2, r_fb, 0, 0, o0, o1, o2)) return rc;
        return run_pairs(ctx, op, prec, M, B, A, G, eps2, r_fb, 0, 0, o0, o1, o2);
    };
    const int64_t na = A->count, nb = B->count;
    if (na == 0 || nb == 0 || (ctx->sort_ops & BF_SORT_DIRECTED) ||
        !use_sorted(ctx, op, prec, na, nb, r_fb, kSortMinPairsBetween) ||
        !use_sorted(ctx, op, prec, nb, na, r_fb, kSortMinPairsBetween))
        return two_passes();
    // shares of each row block's column tiles: at least two rounds of resident workgroups
    const int64_t a_tiles = (na + 63) / 64, b_tiles = (nb + 63) / 64;
    const int64_t rblocks = (a_tiles + kSymBlockTiles - 1) / kSymBlockTiles;
    const KernelConfig sc = sym_config(ctx, op, na, nb);
    const int64_t want = sym_want(ctx, op, sc);
    // at least a block of column tiles per share, the granularity of the one-set sweep's
    // distances: each share writes row sums of its own (32 B per row particle), and with one
    // tile per share those writes and their reduction outweigh the sweep (a 32,768 x 32,768
    // level of the 262,144-body interval took 512 shares of one tile at 32 rounds)
    const int64_t most = std::max<int64_t>(1, b_tiles / kSymBlockTiles);
    const int shares = (int)std::max<int64_t>(1, std::min<int64_t>(most, (want + rblocks - 1) / rblocks));
    if (between_scratch_bytes(na, nb, shares) > kSymMaxScratch ||
        ensure(&ctx->scratch9, &ctx->scratch9_bytes, between_scratch_bytes(na, nb, shares), ctx->stream)) {
        g_err.clear();
        return two_passes();
    }
    // scratch: two fix-up queues [counter | list] for A and B
    const size_t qa = 256 + (((size_t)na * sizeof(int32_t) + 255) & ~size_t(255));
    const size_t qb = 256 + (((size_t)nb * sizeof(int32_t) + 255) & ~size_t(255));
    if (int rc = ensure(&ctx->scratch, &ctx->scratch_bytes, qa + qb, ctx->stream)) return rc;
    if (int rc = ensure(&ctx->scratch8, &ctx->scratch8_bytes, (size_t)kFixChunks * 3 * kFixTiled * sizeof(double),
                        ctx->stream))
        return rc;
    // sort both sets, pack B as column tiles of 64 and A as the FP64 row stream
    const int64_t nmax = std::max(na, nb);
    const size_t tmp = sort_tmp_bytes((int)nmax);
    const size_t list_bytes = ((size_t)nmax * 4 + 255) & ~size_t(255);
    if (int rc = ensure(&ctx->scratch5, &ctx->scratch5_bytes, 256 + 6 * list_bytes + ((tmp + 255) & ~size_t(255)),
                        ctx->stream))
        return rc;
    char* b5 = static_cast<char*>(ctx->scratch5);
    SortBuffers sb;
    sb.bbox = reinterpret_cast<uint32_t*>(b5);
    sb.keys_in = reinterpret_cast<uint32_t*>(b5 + 256);
    sb.keys_out = reinterpret_cast<uint32_t*>(b5 + 256 + list_bytes);
    sb.vals_in = reinterpret_cast<int32_t*>(b5 + 256 + 2 * list_bytes);
    sb.vals_out = reinterpret_cast<int32_t*>(b5 + 256 + 3 * list_bytes);
    int32_t* b_sorted = reinterpret_cast<int32_t*>(b5 + 256 + 4 * list_bytes);
    int32_t* a_sorted = reinterpret_cast<int32_t*>(b5 + 256 + 5 * list_bytes);
    sb.tmp = b5 + 256 + 6 * list_bytes;
    sb.tmp_bytes = tmp;
    const int pb = pack_bytes(op, prec);
    const size_t far_bytes = (((size_t)nb * (op == OP_GRAD ? 32 : 16)) + 255) & ~size_t(255);
    const int kmeta = op == OP_GRAD ? 2 : 1;
    if (int rc = ensure(&ctx->scratch2, &ctx->scratch2_bytes, (size_t)nb * pb, ctx->stream)) return rc;
    if (int rc = ensure(&ctx->scratch6, &ctx->scratch6_bytes, far_bytes + (size_t)b_tiles * kmeta * sizeof(double4),
                        ctx->stream))
        return rc;
    if (int rc = ensure(&ctx->scratch10, &ctx->scratch10_bytes, (size_t)na * pb, ctx->stream)) return rc;
    if (ctx->dry) return BF_OK;  // sizing before a capture: every buffer of this sweep now exists

    PairArgs ab{};  // A targets, B sources
    ab.P = M;
    ab.G = G;
    ab.eps2 = eps2;
    ab.eps2f = (float)eps2 + 1e-20f;
    ab.rfb2f = 0.0f;
    ab.split = 1;
    ab.o0 = o0; ab.o1 = o1; ab.o2 = o2;
    ab.flags = ctx->d_flags;
    ab.cond_max = cond_max_for(op);
    ab.kappa = ctx->kappa;
    PairArgs ba = ab;  // B targets, A sources
    ab.fix_count = static_cast<int32_t*>(ctx->scratch);
    ab.fix_list = reinterpret_cast<int32_t*>(static_cast<char*>(ctx->scratch) + 256);
    ba.fix_count = reinterpret_cast<int32_t*>(static_cast<char*>(ctx->scratch) + qa);
    ba.fix_list = reinterpret_cast<int32_t*>(static_cast<char*>(ctx->scratch) + qa + 256);
    BF_HIP(launch_pass_begin(ab.fix_count, ctx->d_stats, ctx->stream));
    BF_HIP(launch_zero_count(ba.fix_count, ctx->stream));
    ab.tile_stats = ctx->d_stats + 1;
    ab.pass_stats = ctx->d_stats;  // the count of A's queue is reported
    const DevSet dA = devset(A), dB = devset(B);
    BF_HIP(launch_sort_set(M, dB, dB, sb, b_sorted, ctx->d_flags, ctx->stream, ctx->capturing));
    BF_HIP(launch_sort_set(M, dA, dA, sb, a_sorted, ctx->d_flags, ctx->stream, ctx->capturing));
    ab.tgt = ba.src = DevSet{a_sorted, (int32_t)na, 0};
    ab.src = ba.tgt = DevSet{b_sorted, (int32_t)nb, 0};
    double4* meta = reinterpret_cast<double4*>(static_cast<char*>(ctx->scratch6) + far_bytes);
    ab.pack = ctx->scratch2;
    ab.pack_far = ctx->scratch6;
    ab.tile_meta = meta;
    BF_HIP(launch_pack_tiles(op, 1, ab, ctx->scratch2, ctx->scratch6, meta, ctx->stream));
    PairArgs pa = ab;  // the rows' FP64 stream: the mixed pack of the sorted A list
    pa.src = ab.tgt;
    pa.pack = ctx->scratch10;
    BF_HIP(launch_pack(op, BF_PREC_MIXED, pa, ctx->stream));

    SymArgs g{};
    g.near_pack = ctx->scratch2;
    g.far_pack = ctx->scratch6;
    g.tile_meta = meta;
    g.row_pack = ctx->scratch10;
    g.n = (int32_t)nb;
    g.n_tiles = (int32_t)b_tiles;
    g.n_pad = (int32_t)(64 * b_tiles);
    g.n_rows = (int32_t)na;
    g.n_row_tiles = (int32_t)a_tiles;
    g.n_row_pad = (int32_t)(64 * a_tiles);
    g.n_blocks = (int32_t)rblocks;
    g.between = 1;
    g.eps2f = ab.eps2f;
    g.kappa = ctx->kappa;
    g.n_chunks = shares;
    g.chunk_len = (int32_t)((b_tiles + shares - 1) / shares);
    g.own = static_cast<double*>(ctx->scratch9);
    g.part = reinterpret_cast<float*>(static_cast<char*>(ctx->scratch9) + sym_own_bytes(na, shares));
    g.tile_stats = ab.tile_stats;

    std::pair<hipEvent_t, hipEvent_t> ev{nullptr, nullptr};
    const bool timed = ctx->timing && !ctx->capturing;
    if (timed) {
        if (!ctx->tpool.empty()) {
            ev = ctx->tpool.back();
            ctx->tpool.pop_back();
        } else {
            BF_HIP(hipEventCreate(&ev.first));
            BF_HIP(hipEventCreate(&ev.second));
        }
        BF_HIP(hipEventRecord(ev.first, ctx->stream));
    }
    BF_HIP(launch_pairs_sym(op, sc.waves, sc.k, g, ctx->stream));
    if (timed) {
        BF_HIP(hipEventRecord(ev.second, ctx->stream));
        ctx->tev[op].push_back(ev);
    }
    ctx->pair_credit[op] += 2 * (int64_t)A->count * B->count;  // a <- b and b <- a
    ctx->last_kind = BF_PASS_BETWEEN;
    ctx->last_k = sc.k;
    ctx->last_waves = sc.waves;
    ctx->last_split = shares;
    BF_HIP(launch_between_reduce(op, ab, ba, g, ctx->stream));
    BF_HIP(launch_fixup(op, ab, static_cast<double*>(ctx->scratch8), kFixChunks * kFixTiled, ctx->num_cu, ctx->stream));
    BF_HIP(launch_fixup(op, ba, static_cast<double*>(ctx->scratch8), kFixChunks * kFixTiled, ctx->num_cu, ctx->stream));
    return BF_OK;
}

int check_ctx(bf_ctx* ctx) {
    if (!ctx) return fail(BF_ERR_ARG, "context NULL");
    return BF_OK;
}

int check_prec(int prec) {
    if (prec != BF_PREC_FP64 && prec != BF_PREC_MIXED) return fail(BF_ERR_ARG, "prec must be BF_PREC_FP64 or BF_PREC_MIXED");
    return BF_OK;
}

}  // namespace

// shared with batch.hip
int bf_internal_fail(int code, const char* msg) { return fail(code, msg); }

// HIP events around a kernel launch of op on the context stream (when timing is on and nothing
// is being captured): begin returns the pair (or two null events), end records it
std::pair<hipEvent_t, hipEvent_t> bf_internal_timer_begin(bf_ctx* c) {
    std::pair<hipEvent_t, hipEvent_t> ev{nullptr, nullptr};
    if (!c->timing || c->capturing) return ev;
    if (!c->tpool.empty()) {
        ev = c->tpool.back();
        c->tpool.pop_back();
    } else if (hipEventCreate(&ev.first) != hipSuccess || hipEventCreate(&ev.second) != hipSuccess) {
        return {nullptr, nullptr};
    }
    if (hipEventRecord(ev.first, c->stream) != hipSuccess) return {nullptr, nullptr};
    return ev;
}
void bf_internal_timer_end(bf_ctx* c, int op, std::pair<hipEvent_t, hipEvent_t> ev) {
    if (!ev.first || !ev.second) return;
    if (hipEventRecord(ev.second, c->stream) == hipSuccess) c->tev[op].push_back(ev);
}
void bf_internal_credit(bf_ctx* c, int op, int64_t pairs) { c->pair_credit[op] += pairs; }
int bf_internal_bucket(int64_t v) { return ilog2_bucket(v); }
bool bf_internal_batch_shape_ok(int op, int prec, int k, int waves, int chunk);  // batch.hip

int bf_internal_ensure(bf_ctx* c, int which, size_t need) {
    switch (which) {
        case 1: return ensure(&c->scratch, &c->scratch_bytes, need, c->stream);
        case 2: return ensure(&c->scratch2, &c->scratch2_bytes, need, c->stream);
        case 3: return ensure(&c->scratch3, &c->scratch3_bytes, need, c->stream);
        case 4: return ensure(&c->scratch4, &c->scratch4_bytes, need, c->stream);
    }
    return fail(BF_ERR_ARG, "bad scratch id");
}

// exchange scratch buffers 2, 3 and 4 of the context with bufs (used to give graphs their own)
void bf_internal_swap_scratch(bf_ctx* c, void* bufs[3], size_t bytes[3]) {
    std::swap(c->scratch2, bufs[0]); std::swap(c->scratch2_bytes, bytes[0]);
    std::swap(c->scratch3, bufs[1]); std::swap(c->scratch3_bytes, bytes[1]);
    std::swap(c->scratch4, bufs[2]); std::swap(c->scratch4_bytes, bytes[2]);
}

void* bf_internal_scratch(bf_ctx* c, int which) {
    switch (which) {
        case 1: return c->scratch;
        case 2: return c->scratch2;
        case 3: return c->scratch3;
        case 4: return c->scratch4;
    }
    return nullptr;
}

// =============================================================================================
extern "C" {

BF_API const char* bf_version(void) { return "bifrost-hip 0.1 (gfx950)"; }

BF_API const char* bf_status_string(int s) {
    switch (s) {
        case BF_OK: return "ok";
        case BF_ERR_ARG: return "invalid argument";
        case BF_ERR_HIP: return "HIP runtime error";
        case BF_ERR_NONFINITE: return "non-finite result";
        case BF_ERR_UNSUPPORTED: return "unsupported request";
        case BF_ERR_NOMEM: return "out of device memory";
    }
    return "unknown status";
}

BF_API const char* bf_last_error(void) { return g_err.c_str(); }

BF_API int bf_create(bf_ctx** out, int device, void* stream) {
    g_err.clear();
    if (!out) return fail(BF_ERR_ARG, "ctx pointer NULL");
    *out = nullptr;
    int ndev = 0;
    BF_HIP(hipGetDeviceCount(&ndev));
    if (device < 0 || device >= ndev) return fail(BF_ERR_ARG, "device out of range");
    BF_HIP(hipSetDevice(device));
    static_scratch_init(device);
    hipDeviceProp_t prop;
    BF_HIP(hipGetDeviceProperties(&prop, device));
    bf_ctx* c = new bf_ctx();
    c->device = device;
    c->stream = static_cast<hipStream_t>(stream);
    c->num_cu = prop.multiProcessorCount;
    if (hipMalloc(&c->d_stats, 8 * sizeof(unsigned long long)) != hipSuccess ||
        hipMalloc(&c->d_flags, sizeof(uint32_t)) != hipSuccess ||
        hipHostMalloc(&c->h_flags, sizeof(uint32_t), hipHostMallocDefault) != hipSuccess) {
        delete c;
        return fail(BF_ERR_NOMEM, "flag allocation failed");
    }
    if (hipMemsetAsync(c->d_flags, 0, sizeof(uint32_t), c->stream) != hipSuccess ||
        hipStreamSynchronize(c->stream) != hipSuccess) {
        hipFree(c->d_flags);
        hipHostFree(c->h_flags);
        delete c;
        return fail(BF_ERR_HIP, "flag initialisation failed");
    }
    *out = c;
    return BF_OK;
}

static void drop_timing(bf_ctx* c) {
    for (auto& v : c->tev) {
        for (auto& e : v) c->tpool.push_back(e);
        v.clear();
    }
}

BF_API int bf_destroy(bf_ctx* c) {
    if (!c) return BF_OK;
    hipSetDevice(c->device);
    hipStreamSynchronize(c->stream);
    drop_timing(c);
    for (auto& e : c->tpool) {
        hipEventDestroy(e.first);
        hipEventDestroy(e.second);
    }
    if (c->scratch) hipFree(c->scratch);
    if (c->scratch2) hipFree(c->scratch2);
    if (c->scratch3) hipFree(c->scratch3);
    if (c->scratch4) hipFree(c->scratch4);
    if (c->scratch5) hipFree(c->scratch5);
    if (c->scratch6) hipFree(c->scratch6);
    if (c->scratch7) hipFree(c->scratch7);
    if (c->scratch8) hipFree(c->scratch8);
    if (c->scratch9) hipFree(c->scratch9);
    if (c->scratch10) hipFree(c->scratch10);
    if (c->scratch11) hipFree(c->scratch11);
    if (c->d_flags) hipFree(c->d_flags);
    if (c->d_stats) hipFree(c->d_stats);
    if (c->h_flags) hipHostFree(c->h_flags);
    delete c;
    return BF_OK;
}

BF_API int bf_release_scratch(bf_ctx* c, size_t* freed) {
    if (int rc = check_ctx(c)) return rc;
    BF_HIP(hipStreamSynchronize(c->stream));
    size_t total = 0;
    void** bufs[] = {&c->scratch, &c->scratch2, &c->scratch3, &c->scratch4, &c->scratch5,
                     &c->scratch6, &c->scratch7, &c->scratch8, &c->scratch9, &c->scratch10, &c->scratch11};
    size_t* sizes[] = {&c->scratch_bytes, &c->scratch2_bytes, &c->scratch3_bytes, &c->scratch4_bytes,
                       &c->scratch5_bytes, &c->scratch6_bytes, &c->scratch7_bytes, &c->scratch8_bytes,
                       &c->scratch9_bytes, &c->scratch10_bytes, &c->scratch11_bytes};
    for (int i = 0; i < 11; ++i) {
        if (*bufs[i]) BF_HIP(hipFree(*bufs[i]));
        *bufs[i] = nullptr;
        total += *sizes[i];
        *sizes[i] = 0;
    }
    if (freed) *freed = total;
    return BF_OK;
}

BF_API int bf_enable_timing(bf_ctx* c, int on) {
    if (int rc = check_ctx(c)) return rc;
    BF_HIP(hipStreamSynchronize(c->stream));
    drop_timing(c);
    c->timing = on != 0;
    return BF_OK;
}

BF_API int bf_kernel_times(bf_ctx* c, int op, float* ms, int cap, int* count) {
    if (int rc = check_ctx(c)) return rc;
    if (op < 0 || op >= OP_COUNT) return fail(BF_ERR_ARG, "bad op");
    if (!count || (cap > 0 && !ms) || cap < 0) return fail(BF_ERR_ARG, "bad output buffer");
    BF_HIP(hipStreamSynchronize(c->stream));
    auto& v = c->tev[op];
    *count = (int)v.size();
    for (int i = 0; i < (int)v.size() && i < cap; ++i) BF_HIP(hipEventElapsedTime(&ms[i], v[i].first, v[i].second));
    for (auto& e : v) c->tpool.push_back(e);
    v.clear();
    return BF_OK;
}

BF_API int bf_set_stream(bf_ctx* c, void* stream) {
    if (int rc = check_ctx(c)) return rc;
    c->stream = static_cast<hipStream_t>(stream);
    return BF_OK;
}

BF_API int bf_read_flags(bf_ctx* c, uint32_t* flags, int clear) {
    if (int rc = check_ctx(c)) return rc;
    if (!flags) return fail(BF_ERR_ARG, "flags NULL");
    BF_HIP(hipMemcpyAsync(c->h_flags, c->d_flags, sizeof(uint32_t), hipMemcpyDeviceToHost, c->stream));
    BF_HIP(hipStreamSynchronize(c->stream));
    *flags = *c->h_flags;
    if (clear) {
        BF_HIP(hipMemsetAsync(c->d_flags, 0, sizeof(uint32_t), c->stream));
        BF_HIP(hipStreamSynchronize(c->stream));
    }
    return BF_OK;
}

BF_API int bf_validate_set(bf_ctx* c, const bf_set* s, int64_t n) {
    if (int rc = check_ctx(c)) return rc;
    if (n <= 0) return fail(BF_ERR_ARG, "n <= 0");
    if (int rc = check_set(s, n, "validated")) return rc;
    if (s->idx == nullptr || s->count == 0) return BF_OK;
    uint32_t before = 0;
    if (int rc = bf_read_flags(c, &before, 0)) return rc;
    BF_HIP(hipMemsetAsync(c->d_flags, 0, sizeof(uint32_t), c->stream));
    BF_HIP(launch_validate(devset(s), n, c->d_flags, c->stream));
    uint32_t f = 0;
    if (int rc = bf_read_flags(c, &f, 0)) return rc;
    // restore the earlier flags (plus nothing else: the validation itself is not an error source)
    *c->h_flags = before;
    BF_HIP(hipMemcpyAsync(c->d_flags, c->h_flags, sizeof(uint32_t), hipMemcpyHostToDevice, c->stream));
    BF_HIP(hipStreamSynchronize(c->stream));
    if (f & BF_FLAG_BADINDEX) return fail(BF_ERR_ARG, "index list has entries outside [0, n)");
    return BF_OK;
}

BF_API int bf_forces(bf_ctx* c, const bf_particles* P, const bf_set* t, const bf_set* s, double G, double eps2,
                     int prec, double r_fb, double* ax, double* ay, double* az) {
    g_err.clear();
    if (int rc = check_ctx(c)) return rc;
    if (int rc = check_particles(P, false)) return rc;
    if (int rc = check_set(t, P->n, "target")) return rc;
    if (int rc = check_set(s, P->n, "source")) return rc;
    if (int rc = check_prec(prec)) return rc;
    if (!isfinite(G)) return fail(BF_ERR_ARG, "G not finite");
    if (!finite_nonneg(eps2)) return fail(BF_ERR_ARG, "eps2 must be finite and >= 0");
    if (!finite_nonneg(r_fb)) return fail(BF_ERR_ARG, "r_fb must be finite and >= 0");
    if (!ax || !ay || !az) return fail(BF_ERR_ARG, "output pointer NULL");
    return run_pairs(c, OP_ACC, prec, masters_of(P), t, s, G, eps2, r_fb, 0, 0, ax, ay, az);
}

BF_API int bf_forces_noalloc(bf_ctx* c, const bf_particles* P, const bf_set* t, const bf_set* s, double G,
                             double eps2, int prec, double r_fb, double* ax, double* ay, double* az) {
    g_err.clear();
    if (int rc = check_ctx(c)) return rc;
    if (int rc = check_particles(P, false)) return rc;
    if (int rc = check_set(t, P->n, "target")) return rc;
    if (int rc = check_set(s, P->n, "source")) return rc;
    if (int rc = check_prec(prec)) return rc;
    if (!isfinite(G)) return fail(BF_ERR_ARG, "G not finite");
    if (!finite_nonneg(eps2)) return fail(BF_ERR_ARG, "eps2 must be finite and >= 0");
    if (!finite_nonneg(r_fb)) return fail(BF_ERR_ARG, "r_fb must be finite and >= 0");
    if (!ax || !ay || !az) return fail(BF_ERR_ARG, "output pointer NULL");
    std::string why;
    void* base = static_scratch_of(c->device, &why);
    if (!base) return fail(BF_ERR_HIP, why);
    const Arena arena{static_cast<char*>(base), kStaticScratchBytes};
    return run_pairs(c, OP_ACC, prec, masters_of(P), t, s, G, eps2, r_fb, 0, 0, ax, ay, az, &arena);
}

BF_API int bf_force_gradient(bf_ctx* c, const bf_particles* P, const bf_set* t, const bf_set* s, const double* ax,
                             const double* ay, const double* az, double G, double eps2, int prec, double r_fb,
                             double* gx, double* gy, double* gz) {
    g_err.clear();
    if (int rc = check_ctx(c)) return rc;
    if (int rc = check_particles(P, false)) return rc;
    if (int rc = check_set(t, P->n, "target")) return rc;
    if (int rc = check_set(s, P->n, "source")) return rc;
    if (int rc = check_prec(prec)) return rc;
    if (!isfinite(G)) return fail(BF_ERR_ARG, "G not finite");
    if (!finite_nonneg(eps2)) return fail(BF_ERR_ARG, "eps2 must be finite and >= 0");
    if (!finite_nonneg(r_fb)) return fail(BF_ERR_ARG, "r_fb must be finite and >= 0");
    if (!ax || !ay || !az) return fail(BF_ERR_ARG, "acceleration pointer NULL");
    if (!gx || !gy || !gz) return fail(BF_ERR_ARG, "output pointer NULL");
    Masters M = masters_of(P);
    M.ax = ax; M.ay = ay; M.az = az;
    return run_pairs(c, OP_GRAD, prec, M, t, s, G, eps2, r_fb, 0, 0, gx, gy, gz);
}

// ranges can be checked for overlap on the host; index lists are the caller's promise
static int check_disjoint(const bf_set* a, const bf_set* b) {
    if (a->idx == nullptr && b->idx == nullptr && a->count > 0 && b->count > 0 &&
        a->begin < b->begin + b->count && b->begin < a->begin + a->count)
        return fail(BF_ERR_ARG, "the two sets overlap");
    if (a->idx != nullptr && a->idx == b->idx && a->count > 0 && b->count > 0)
        return fail(BF_ERR_ARG, "the two sets share their index list");
    return BF_OK;
}

BF_API int bf_forces_between(bf_ctx* c, const bf_particles* P, const bf_set* a, const bf_set* b, double G,
                             double eps2, int prec, double r_fb, double* ax, double* ay, double* az) {
    g_err.clear();
    if (int rc = check_ctx(c)) return rc;
    if (int rc = check_particles(P, false)) return rc;
    if (int rc = check_set(a, P->n, "first")) return rc;
    if (int rc = check_set(b, P->n, "second")) return rc;
    if (int rc = check_disjoint(a, b)) return rc;
    if (int rc = check_prec(prec)) return rc;
    if (!isfinite(G)) return fail(BF_ERR_ARG, "G not finite");
    if (!finite_nonneg(eps2)) return fail(BF_ERR_ARG, "eps2 must be finite and >= 0");
    if (!finite_nonneg(r_fb)) return fail(BF_ERR_ARG, "r_fb must be finite and >= 0");
    if (!ax || !ay || !az) return fail(BF_ERR_ARG, "output pointer NULL");
    return run_pairs_between(c, OP_ACC, prec, masters_of(P), a, b, G, eps2, r_fb, ax, ay, az);
}

BF_API int bf_force_gradient_between(bf_ctx* c, const bf_particles* P, const bf_set* a, const bf_set* b,
                                     const double* ax, const double* ay, const double* az, double G, double eps2,
                                     int prec, double r_fb, double* gx, double* gy, double* gz) {
    g_err.clear();
    if (int rc = check_ctx(c)) return rc;
    if (int rc = check_particles(P, false)) return rc;
    if (int rc = check_set(a, P->n, "first")) return rc;
    if (int rc = check_set(b, P->n, "second")) return rc;
    if (int rc = check_disjoint(a, b)) return rc;
    if (int rc = check_prec(prec)) return rc;
    if (!isfinite(G)) return fail(BF_ERR_ARG, "G not finite");
    if (!finite_nonneg(eps2)) return fail(BF_ERR_ARG, "eps2 must be finite and >= 0");
    if (!finite_nonneg(r_fb)) return fail(BF_ERR_ARG, "r_fb must be finite and >= 0");
    if (!ax || !ay || !az) return fail(BF_ERR_ARG, "acceleration pointer NULL");
    if (!gx || !gy || !gz) return fail(BF_ERR_ARG, "output pointer NULL");
    Masters M = masters_of(P);
    M.ax = ax; M.ay = ay; M.az = az;
    return run_pairs_between(c, OP_GRAD, prec, M, a, b, G, eps2, r_fb, gx, gy, gz);
}

BF_API int bf_dt_min(bf_ctx* c, const bf_particles* P, const bf_set* t, const bf_set* s, double G, double eta_ff,
                     double eta_fb, int prec, double r_fb, double* dt_ff, double* dt_fb) {
    g_err.clear();
    if (int rc = check_ctx(c)) return rc;
    if (int rc = check_particles(P, true)) return rc;
    if (int rc = check_set(t, P->n, "target")) return rc;
    if (int rc = check_set(s, P->n, "source")) return rc;
    if (int rc = check_prec(prec)) return rc;
    if (!(isfinite(G) && G > 0)) return fail(BF_ERR_ARG, "G must be finite and > 0");
    if (!finite_nonneg(eta_ff) || !finite_nonneg(eta_fb)) return fail(BF_ERR_ARG, "eta must be finite and >= 0");
    if (!finite_nonneg(r_fb)) return fail(BF_ERR_ARG, "r_fb must be finite and >= 0");
    if (!dt_ff || !dt_fb) return fail(BF_ERR_ARG, "output pointer NULL");
    return run_pairs(c, OP_DT, prec, masters_of(P), t, s, G, 0.0, r_fb, eta_ff, eta_fb, dt_ff, dt_fb, nullptr);
}

static int pn1_impl(bf_ctx* c, const Masters& M, const bf_set* t, const bf_set* s, const int32_t* bh, int32_t nbh,
                    double G, double cl, double* o0, double* o1, double* o2) {
    if (t->count == 0) return BF_OK;
    PnArgs a{};
    a.P = M;
    a.tgt = devset(t);
    a.src = devset(s);
    a.bh = bh;
    a.nbh = nbh;
    a.G = G;
    a.c2inv = 1.0 / (cl * cl);
    a.chunk = 4096;
    a.nchunk = std::max(1, (s->count + a.chunk - 1) / a.chunk);
    a.o0 = o0; a.o1 = o1; a.o2 = o2;
    a.flags = c->d_flags;
    if (nbh > 0) {
        const size_t part_bytes = (size_t)nbh * a.nchunk * 4 * sizeof(double);
        const size_t need = part_bytes + (size_t)nbh * sizeof(int32_t) + 256;
        if (int rc = ensure(&c->scratch, &c->scratch_bytes, need, c->stream)) return rc;
        a.part = static_cast<double*>(c->scratch);
        a.bh_in_src = reinterpret_cast<int32_t*>(static_cast<char*>(c->scratch) + ((part_bytes + 255) & ~size_t(255)));
    }
    if (c->dry) return BF_OK;  // sizing before a capture: the scratch now exists
    BF_HIP(launch_pn1(a, c->stream));
    return BF_OK;
}

BF_API int bf_pn1_bh(bf_ctx* c, const bf_particles* P, const bf_set* t, const bf_set* s, const int32_t* bh_idx,
                     int32_t n_bh, double G, double cl, double* apx, double* apy, double* apz) {
    g_err.clear();
    if (int rc = check_ctx(c)) return rc;
    if (int rc = check_particles(P, true)) return rc;
    if (int rc = check_set(t, P->n, "target")) return rc;
    if (int rc = check_set(s, P->n, "source")) return rc;
    if (n_bh < 0 || (n_bh > 0 && !bh_idx)) return fail(BF_ERR_ARG, "bad black-hole list");
    if (!(isfinite(cl) && cl > 0)) return fail(BF_ERR_ARG, "c must be finite and > 0");
    if (!isfinite(G)) return fail(BF_ERR_ARG, "G not finite");
    if (!apx || !apy || !apz) return fail(BF_ERR_ARG, "output pointer NULL");
    return pn1_impl(c, masters_of(P), t, s, bh_idx, n_bh, G, cl, apx, apy, apz);
}

BF_API int bf_energy(bf_ctx* c, const bf_particles* P, const bf_set* s, double G, double eps2, double* kinetic,
                     double* potential) {
    g_err.clear();
    if (int rc = check_ctx(c)) return rc;
    if (int rc = check_particles(P, true)) return rc;
    if (int rc = check_set(s, P->n, "energy")) return rc;
    if (!finite_nonneg(eps2)) return fail(BF_ERR_ARG, "eps2 must be finite and >= 0");
    if (!kinetic || !potential) return fail(BF_ERR_ARG, "output pointer NULL");
    if (s->count == 0) { *kinetic = 0; *potential = 0; return BF_OK; }
    // one partial per upper-triangular pair of 512-particle blocks: at most 2^24 particles
    if (s->count > (1 << 24)) return fail(BF_ERR_UNSUPPORTED, "bf_energy takes at most 2^24 particles");
    if (s->idx) {
        if (int rc = bf_validate_set(c, s, P->n)) return rc;
    }
    EnergyArgs e{};
    e.P = masters_of(P);
    e.set = devset(s);
    e.G = G;
    e.eps2 = eps2;
    const size_t np = (size_t)energy_partials(s->count);
    const size_t packb = ((size_t)s->count * sizeof(double4) + 255) & ~size_t(255);
    const size_t need = packb + (np + (size_t)s->count + 2) * sizeof(double);
    if (int rc = ensure(&c->scratch, &c->scratch_bytes, need, c->stream)) return rc;
    e.pack = static_cast<double4*>(c->scratch);
    e.rows = reinterpret_cast<double*>(static_cast<char*>(c->scratch) + packb);
    e.kin = e.rows + np;
    e.out = e.kin + s->count;
    BF_HIP(launch_energy(e, c->stream));
    double h[2];
    BF_HIP(hipMemcpyAsync(h, e.out, sizeof(h), hipMemcpyDeviceToHost, c->stream));
    BF_HIP(hipStreamSynchronize(c->stream));
    *kinetic = h[0];
    *potential = h[1];
    return BF_OK;
}

static int check_state(const bf_state* S) {
    if (!S) return fail(BF_ERR_ARG, "state NULL");
    if (S->n <= 0 || S->n > INT32_MAX) return fail(BF_ERR_ARG, "n must be in [1, 2^31)");
    if (!S->x || !S->y || !S->z || !S->vx || !S->vy || !S->vz || !S->m) return fail(BF_ERR_ARG, "state pointer NULL");
    return BF_OK;
}

BF_API int bf_kick(bf_ctx* c, const bf_state* S, const bf_set* set, double h, const double* ax, const double* ay,
                   const double* az, double h2, const double* gx, const double* gy, const double* gz) {
    g_err.clear();
    if (int rc = check_ctx(c)) return rc;
    if (int rc = check_state(S)) return rc;
    if (int rc = check_set(set, S->n, "kick")) return rc;
    if (!ax || !ay || !az) return fail(BF_ERR_ARG, "acceleration pointer NULL");
    if ((gx || gy || gz) && !(gx && gy && gz)) return fail(BF_ERR_ARG, "gradient pointers must be all NULL or all set");
    if (!isfinite(h) || !isfinite(h2)) return fail(BF_ERR_ARG, "h not finite");
    BF_HIP(launch_kick(*S, devset(set), h, ax, ay, az, h2, gx, gy, gz, c->d_flags, c->stream));
    return BF_OK;
}

BF_API int bf_drift(bf_ctx* c, const bf_state* S, const bf_set* set, double h) {
    g_err.clear();
    if (int rc = check_ctx(c)) return rc;
    if (int rc = check_state(S)) return rc;
    if (int rc = check_set(set, S->n, "drift")) return rc;
    if (!isfinite(h)) return fail(BF_ERR_ARG, "h not finite");
    BF_HIP(launch_drift(*S, devset(set), h, c->d_flags, c->stream));
    return BF_OK;
}

static int check_fsi_params(const bf_fsi_params* prm) {
    if (!prm) return fail(BF_ERR_ARG, "params NULL");
    if (int rc = check_prec(prm->prec)) return rc;
    if (!isfinite(prm->G) || !finite_nonneg(prm->eps2) || !finite_nonneg(prm->r_fb))
        return fail(BF_ERR_ARG, "bad G, eps2 or r_fb");
    if (prm->n_bh < 0 || (prm->n_bh > 0 && (!prm->bh_idx || !(isfinite(prm->c) && prm->c > 0))))
        return fail(BF_ERR_ARG, "bad PN parameters");
    return BF_OK;
}

// One FSI cycle (Sec. 2.1, Eq. fsi-cycle) over `set`, optionally wrapped in PN1.0 half-kicks;
// g* is scratch for the gradient sums (and the PN accelerations), particle-indexed.
static int fsi_impl(bf_ctx* c, const bf_state* S, const bf_set* set, double dt, const bf_fsi_params* prm, double* ax,
                    double* ay, double* az, int flags, double* gx, double* gy, double* gz) {
    if (set->count == 0) return BF_OK;
    const int64_t n = S->n;
    bf_particles P{S->x, S->y, S->z, S->vx, S->vy, S->vz, S->m, n};
    const Masters M = masters_of(&P);
    const DevSet ds = devset(set);
    const double G = prm->G, e2 = prm->eps2, rfb = prm->r_fb;
    const int prec = prm->prec;
    int rc;

    auto pn_half_kick = [&]() -> int {
        if (prm->n_bh == 0) return BF_OK;
        if (int r = pn1_impl(c, M, set, set, prm->bh_idx, prm->n_bh, G, prm->c, gx, gy, gz)) return r;
        if (!c->dry)
            BF_HIP(launch_kick(*S, ds, 0.5 * dt, gx, gy, gz, 0.0, nullptr, nullptr, nullptr, c->d_flags, c->stream));
        return BF_OK;
    };
    auto acc = [&]() { return run_pairs(c, OP_ACC, prec, M, set, set, G, e2, rfb, 0, 0, ax, ay, az); };

    if ((rc = pn_half_kick())) return rc;
    if (!(flags & BF_A_VALID))
        if ((rc = acc())) return rc;
    const bool go = !c->dry;  // a sizing pass before a capture launches nothing
    if (go)
        BF_HIP(launch_kick_drift(*S, ds, dt / 6.0, ax, ay, az, 0.0, nullptr, nullptr, nullptr, 0.5 * dt, c->d_flags,
                                 c->stream));
    if ((rc = acc())) return rc;
    Masters Mg = M;
    Mg.ax = ax; Mg.ay = ay; Mg.az = az;
    if ((rc = run_pairs(c, OP_GRAD, prec, Mg, set, set, G, e2, rfb, 0, 0, gx, gy, gz))) return rc;
    if (go)
        BF_HIP(launch_kick_drift(*S, ds, 2.0 * dt / 3.0, ax, ay, az, dt * dt / 24.0, gx, gy, gz, 0.5 * dt, c->d_flags,
                                 c->stream));
    if ((rc = acc())) return rc;
    if (go) BF_HIP(launch_kick(*S, ds, dt / 6.0, ax, ay, az, 0.0, nullptr, nullptr, nullptr, c->d_flags, c->stream));
    if ((rc = pn_half_kick())) return rc;
    return BF_OK;
}

BF_API int bf_fsi_step(bf_ctx* c, const bf_state* S, const bf_set* set, double dt, const bf_fsi_params* prm, double* ax,
                       double* ay, double* az, int flags) {
    g_err.clear();
    if (int rc = check_ctx(c)) return rc;
    if (int rc = check_state(S)) return rc;
    if (int rc = check_set(set, S->n, "fsi")) return rc;
    if (int rc = check_fsi_params(prm)) return rc;
    if (!isfinite(dt)) return fail(BF_ERR_ARG, "dt not finite");
    if (!ax || !ay || !az) return fail(BF_ERR_ARG, "acceleration pointer NULL");
    if (set->count == 0) return BF_OK;
    const int64_t n = S->n;
    if (int rc = ensure(&c->scratch3, &c->scratch3_bytes, (size_t)3 * n * sizeof(double), c->stream)) return rc;
    double* g = static_cast<double*>(c->scratch3);
    return fsi_impl(c, S, set, dt, prm, ax, ay, az, flags, g, g + n, g + 2 * n);
}

// ---- time-step assignment, level partition, HHS-FSI interval ------------------------------------

BF_API int bf_jerk(bf_ctx* c, const bf_particles* P, const bf_set* t, const bf_set* s, double G, double eps2, int prec,
                   double* jx, double* jy, double* jz) {
    g_err.clear();
    if (int rc = check_ctx(c)) return rc;
    if (int rc = check_particles(P, true)) return rc;
    if (int rc = check_set(t, P->n, "target")) return rc;
    if (int rc = check_set(s, P->n, "source")) return rc;
    if (int rc = check_prec(prec)) return rc;
    if (!isfinite(G)) return fail(BF_ERR_ARG, "G not finite");
    if (!finite_nonneg(eps2)) return fail(BF_ERR_ARG, "eps2 must be finite and >= 0");
    if (!jx || !jy || !jz) return fail(BF_ERR_ARG, "output pointer NULL");
    // the jerk is the tidal contraction of the gradient pass with velocities in place of accelerations
    Masters M = masters_of(P);
    M.ax = P->vx; M.ay = P->vy; M.az = P->vz;
    return run_pairs(c, OP_GRAD, prec, M, t, s, G, eps2, 0.0, 0, 0, jx, jy, jz);
}

BF_API int bf_timestep_assign(bf_ctx* c, const bf_particles* P, const bf_set* set, const double* dt_ff,
                              const double* dt_fb, const double* ax, const double* ay, const double* az,
                              const double* gx, const double* gy, const double* gz, const double* jx, const double* jy,
                              const double* jz, double eta_grad, double eta_jerk, double tau, int kmax, double* dt,
                              int32_t* level) {
    g_err.clear();
    if (int rc = check_ctx(c)) return rc;
    if (int rc = check_particles(P, true)) return rc;
    if (int rc = check_set(set, P->n, "timestep")) return rc;
    if (!dt_ff || !dt_fb || !ax || !ay || !az || !dt) return fail(BF_ERR_ARG, "array pointer NULL");
    if ((gx || gy || gz) && !(gx && gy && gz)) return fail(BF_ERR_ARG, "gradient pointers must be all NULL or all set");
    if ((jx || jy || jz) && !(jx && jy && jz)) return fail(BF_ERR_ARG, "jerk pointers must be all NULL or all set");
    if (!isfinite(eta_grad) || !isfinite(eta_jerk)) return fail(BF_ERR_ARG, "eta not finite");
    if (!(isfinite(tau) && tau > 0)) return fail(BF_ERR_ARG, "tau must be finite and > 0");
    if (kmax < 0 || kmax > 63) return fail(BF_ERR_ARG, "kmax must be in [0, 63]");
    TimestepArgs t{};
    t.P = masters_of(P);
    t.set = devset(set);
    t.dt_ff = dt_ff; t.dt_fb = dt_fb;
    t.ax = ax; t.ay = ay; t.az = az;
    t.gx = gx; t.gy = gy; t.gz = gz;
    t.jx = jx; t.jy = jy; t.jz = jz;
    t.eta_grad = eta_grad; t.eta_jerk = eta_jerk; t.tau = tau; t.kmax = kmax;
    t.dt = dt; t.level = level;
    t.flags = c->d_flags;
    BF_HIP(launch_timestep(t, c->stream));
    return BF_OK;
}

// stable partition of a set by level into `order`; level counts copied to the host (synchronising)
// Stable partition of `set` by level; counts to the host (synchronising).  With prev, also
// whether the new order equals the previous one (prev[0..n_prev), n0_prev of them at level 0):
// same_host[0] = same level-0 part, same_host[1] = same list (diff_dev: two device ints).
static int partition_impl(bf_ctx* c, const bf_set* set, int64_t n, const int32_t* level, int kmax, int32_t* order,
                          int64_t* counts_host, const int32_t* prev = nullptr, int n_prev = 0, int n0_prev = 0,
                          int32_t* diff_dev = nullptr, bool* same_host = nullptr) {
    const int cnt = set->count;
    const size_t lb = ((size_t)std::max(cnt, 1) * 4 + 255) & ~size_t(255);
    const size_t tmp = level_sort_tmp_bytes(std::max(cnt, 1));
    if (int rc = ensure(&c->scratch5, &c->scratch5_bytes, 256 + 3 * lb + tmp, c->stream)) return rc;
    char* b = static_cast<char*>(c->scratch5);
    int32_t* counts = reinterpret_cast<int32_t*>(b);
    uint32_t* kin = reinterpret_cast<uint32_t*>(b + 256);
    uint32_t* kout = reinterpret_cast<uint32_t*>(b + 256 + lb);
    int32_t* vin = reinterpret_cast<int32_t*>(b + 256 + 2 * lb);
    BF_HIP(launch_level_partition(devset(set), n, level, kmax, kin, kout, vin, order, counts, b + 256 + 3 * lb, tmp,
                                  c->d_flags, c->stream));
    int32_t h[64], d[2] = {1, 1};
    if (prev) {
        BF_HIP(launch_split_diff(order, cnt, counts, prev, n_prev, n0_prev, diff_dev, c->stream));
        BF_HIP(hipMemcpyAsync(d, diff_dev, sizeof(d), hipMemcpyDeviceToHost, c->stream));
    }
    BF_HIP(hipMemcpyAsync(h, counts, sizeof(int32_t) * (kmax + 1), hipMemcpyDeviceToHost, c->stream));
    BF_HIP(hipStreamSynchronize(c->stream));
    for (int k = 0; k <= kmax; ++k) counts_host[k] = h[k];
    if (same_host) {
        same_host[0] = prev && d[0] == 0;
        same_host[1] = prev && d[1] == 0;
    }
    return BF_OK;
}

BF_API int bf_level_partition(bf_ctx* c, const bf_set* set, int64_t n, const int32_t* level, int kmax, int32_t* order,
                              int64_t* counts) {
    g_err.clear();
    if (int rc = check_ctx(c)) return rc;
    if (n <= 0 || n > INT32_MAX) return fail(BF_ERR_ARG, "n must be in [1, 2^31)");
    if (int rc = check_set(set, n, "partition")) return rc;
    if (!level || !order || !counts) return fail(BF_ERR_ARG, "array pointer NULL");
    if (kmax < 0 || kmax > 63) return fail(BF_ERR_ARG, "kmax must be in [0, 63]");
    return partition_impl(c, set, n, level, kmax, order, counts);
}

namespace {

// bit l of *mask set when a listed black hole sits on level l (an entry outside the particle
// range or the levels sets every bit); one workgroup
__global__ __launch_bounds__(256) void k_bh_level_mask(const int32_t* bh, int32_t nbh, const int32_t* level, int64_t n,
                                                      unsigned long long* mask) {
    if (threadIdx.x == 0) *mask = 0ull;
    __syncthreads();
    for (int i = threadIdx.x; i < nbh; i += blockDim.x) {
        const int32_t p = bh[i];
        unsigned long long b = ~0ull;
        if (p >= 0 && p < n) {
            const int32_t l = level[p];
            if (l >= 0 && l < 64) b = 1ull << l;
        }
        atomicOr(mask, b);
    }
}

struct HhsCtx {
    bf_ctx* c;
    const bf_state* S;
    const bf_fsi_params* prm;
    Masters M;
    const int32_t* order;
    int64_t begin[65];  // begin[k] = first position of level k in `order`; begin[kmax+1] = total
    int kmax;
    double *asf, *gsf, *afsi, *gfsi;  // each 3n
    // Results a later visit of the same level may take instead of recomputing.  A particle
    // drifts only in the FSI cycles of its own level, and those run only inside visits of its
    // level, so between two visits of level k no particle of level >= k moves (with levels
    // reassigned per visit the driver also checks that the level's sets are unchanged):
    //  - afsi holds level k's own accelerations at its final positions after each of its FSI
    //    cycles (the sets of the levels are disjoint), valid for the next one (a_ok[k]);
    //  - asf_lv[k] (3n, particle-indexed) holds level k's inter-level accelerations; the last
    //    ones of a visit equal the first ones of the next visit (il_ok[k]).
    // Kernels are deterministic, so an interval with reuse equals one without, bit for bit.
    double* asf_lv[64];
    mutable bool a_ok[64], il_ok[64];
    bool reuse = false;
    // fixed levels with PN1.0: bit l set when a black hole sits on level l.  A PN kick over sets
    // with no black hole adds exactly zero, so it is not launched (unknown: every kick runs).
    bool bh_known = false;
    unsigned long long bh_levels = ~0ull;
};

bf_set segment(const HhsCtx& h, int64_t b, int64_t e) { return bf_set{h.order + b, (int32_t)(e - b), 0}; }

// inter-level accelerations (Sec. 2.2): S <- F and F <- S into as (3n, particle-indexed)
int interlevel_acc(const HhsCtx& h, const bf_set& Sset, const bf_set& Fset, double* as) {
    const int64_t n = h.S->n;
    const bf_fsi_params* p = h.prm;
    return run_pairs_between(h.c, OP_ACC, p->prec, h.M, &Sset, &Fset, p->G, p->eps2, p->r_fb, as, as + n, as + 2 * n);
}

// One level of the HHS-FSI cycle (Sec. 2.2, Eq. hhsfsi-cycle) for slow set Sset and fast set
// Fset (Bset = both, contiguous); `fast` advances F by tau/2 (the next level).  k is the level
// (results reused between its visits while h.a_ok / h.il_ok say so) or -1 (nothing reused).
extern "C++" {
template <class Fast>
int hhs_cycle(const HhsCtx& h, const bf_set& Sset, const bf_set& Fset, const bf_set& Bset, double tau, int k,
              Fast&& fast) {
    const int64_t n = h.S->n;
    bf_ctx* c = h.c;
    const bf_fsi_params* p = h.prm;
    const bool keep = h.reuse && k >= 0;
    double* const as = keep && h.asf_lv[k] ? h.asf_lv[k] : h.asf;
    // which of S (level k) and F (deeper) hold a black hole
    const bool known = h.bh_known && k >= 0 && k < 64;
    const unsigned long long deeper = known && k < 63 ? ~((2ull << k) - 1ull) : 0ull;
    const bool s_bh = !known || (h.bh_levels >> k & 1ull), f_bh = !known || (h.bh_levels & deeper);
    bf_fsi_params pf = *p;
    if (!s_bh) pf.n_bh = 0;  // no PN pair inside S
    auto fsi = [&](double dt) {
        const int fl = keep && h.a_ok[k] ? BF_A_VALID : 0;
        const int r = fsi_impl(c, h.S, &Sset, dt, &pf, h.afsi, h.afsi + n, h.afsi + 2 * n, fl, h.gfsi, h.gfsi + n,
                               h.gfsi + 2 * n);
        if (keep) h.a_ok[k] = r == BF_OK;
        return r;
    };
    auto inter = [&]() {
        const int r = interlevel_acc(h, Sset, Fset, as);
        if (keep) h.il_ok[k] = r == BF_OK && as != h.asf;
        return r;
    };
    if (Fset.count == 0) return Sset.count ? fsi(tau) : BF_OK;  // no split at the last level
    if (Sset.count == 0) {
        if (int rc = fast()) return rc;
        return fast();
    }
    const DevSet dB = devset(&Bset);
    const double* nul = nullptr;
    int rc;
    const bool go = !c->dry;
    // PN1.0 (Sec. 3.8) in the hierarchy, a reading: every plain FSI cycle carries half-kicks
    // over its own pairs (fsi_impl), and each level's cycle is wrapped in half-kicks over its
    // inter-level pairs with a flagged particle
    auto pn_interlevel_half_kick = [&]() -> int {
        if (p->n_bh == 0 || !(s_bh || f_bh)) return BF_OK;
        if (int r = pn1_impl(c, h.M, &Sset, &Fset, p->bh_idx, p->n_bh, p->G, p->c, h.gsf, h.gsf + n, h.gsf + 2 * n))
            return r;
        if (int r = pn1_impl(c, h.M, &Fset, &Sset, p->bh_idx, p->n_bh, p->G, p->c, h.gsf, h.gsf + n, h.gsf + 2 * n))
            return r;
        if (go)
            BF_HIP(launch_kick(*h.S, dB, 0.5 * tau, h.gsf, h.gsf + n, h.gsf + 2 * n, 0.0, nul, nul, nul, c->d_flags,
                               c->stream));
        return BF_OK;
    };
    if ((rc = pn_interlevel_half_kick())) return rc;
    if (!(keep && h.il_ok[k]))
        if ((rc = inter())) return rc;
    if (go) BF_HIP(launch_kick(*h.S, dB, tau / 6.0, as, as + n, as + 2 * n, 0.0, nul, nul, nul, c->d_flags, c->stream));
    if ((rc = fsi(0.5 * tau))) return rc;
    if ((rc = fast())) return rc;
    if ((rc = inter())) return rc;
    Masters Mg = h.M;
    Mg.ax = as; Mg.ay = as + n; Mg.az = as + 2 * n;
    if ((rc = run_pairs_between(c, OP_GRAD, p->prec, Mg, &Sset, &Fset, p->G, p->eps2, p->r_fb, h.gsf, h.gsf + n,
                                h.gsf + 2 * n)))
        return rc;
    if (go)
        BF_HIP(launch_kick(*h.S, dB, 2.0 * tau / 3.0, as, as + n, as + 2 * n, tau * tau / 24.0, h.gsf, h.gsf + n,
                           h.gsf + 2 * n, c->d_flags, c->stream));
    if ((rc = fast())) return rc;
    if ((rc = fsi(0.5 * tau))) return rc;
    if ((rc = inter())) return rc;
    if (go) BF_HIP(launch_kick(*h.S, dB, tau / 6.0, as, as + n, as + 2 * n, 0.0, nul, nul, nul, c->d_flags, c->stream));
    return pn_interlevel_half_kick();
}
}  // extern "C++"

// fixed levels: level k's slow set is the k-th segment of the level order
int hhs_rec(const HhsCtx& h, int k, double tau) {
    const int64_t total = h.begin[h.kmax + 1];
    const int64_t sb = h.begin[k], fb = k < h.kmax ? h.begin[k + 1] : total;
    const bf_set Sset = segment(h, sb, fb), Fset = segment(h, fb, total), Bset = segment(h, sb, total);
    return hhs_cycle(h, Sset, Fset, Bset, tau, k, [&]() { return hhs_rec(h, k + 1, 0.5 * tau); });
}

// one fixed-level interval: nothing is valid at its start
int hhs_run(const HhsCtx& h, double tau) {
    for (int k = 0; k < 64; ++k) h.a_ok[k] = h.il_ok[k] = false;
    return hhs_rec(h, 0, tau);
}

// adaptive levels: every level assigns time-steps to its particles P and splits them at the
// pivot tau (Sec. 2.2).  Below the top level every criterion is evaluated again over P alone:
// the pairwise free-fall / fly-by time-steps (Sec. 3.5.3), both gradient criteria (Sec. 3.5.4,
// Eqs. dt-nabla1, dt-nabla2, with the acceleration and gradient sum over P) and the jerk
// criterion (Sec. 3.5.5, the jerk over P); the result is capped by the interval's initial
// time-step (Sec. 3.5.1, the level-0 minimum).
struct HhsAdapt {
    const double* dt0;
    double eta_ff, eta_fb, eta_grad, eta_jerk;
    double *dtff, *dtfb, *dtl;  // particle-indexed: pairwise criteria, the level's time-step
    double *alv, *glv, *jlv;    // 3n each: acceleration, gradient sum and jerk over the level's set
    int32_t* flag;              // particle-indexed: 0 slow, 1 fast
    int32_t* lists;             // 2 (kmax + 1) buffers of `cap` entries: the splits of the level-k set,
                                // this visit's and the previous visit's
    int32_t* diff;              // two device ints: does this split differ from the previous one
    int which[64];              // buffer of level k's latest split
    int64_t prev_n[64], prev_n0[64];  // its size and slow count (-1: none, nothing kept)
    int64_t cap;
    int max_level;
    int64_t nodes;
};

// time-steps of the particles of P from P alone (all criteria), into A.dtl
int level_timesteps(const HhsCtx& h, HhsAdapt& A, const bf_set& P) {
    bf_ctx* c = h.c;
    const int64_t n = h.S->n;
    const bf_fsi_params* p = h.prm;
    if (int rc = run_pairs(c, OP_DT, p->prec, h.M, &P, &P, p->G, 0.0, 0.0, A.eta_ff, A.eta_fb, A.dtff, A.dtfb,
                           nullptr))
        return rc;
    if (int rc = run_pairs(c, OP_ACC, p->prec, h.M, &P, &P, p->G, p->eps2, p->r_fb, 0, 0, A.alv, A.alv + n,
                           A.alv + 2 * n))
        return rc;
    const bool grad = A.eta_grad > 0.0, jerk = A.eta_jerk > 0.0;
    if (grad) {
        Masters Mg = h.M;
        Mg.ax = A.alv; Mg.ay = A.alv + n; Mg.az = A.alv + 2 * n;
        if (int rc = run_pairs(c, OP_GRAD, p->prec, Mg, &P, &P, p->G, p->eps2, p->r_fb, 0, 0, A.glv, A.glv + n,
                               A.glv + 2 * n))
            return rc;
    }
    if (jerk) {
        // the jerk is the tidal contraction with the velocities in place of the accelerations
        Masters Mj = h.M;
        Mj.ax = h.S->vx; Mj.ay = h.S->vy; Mj.az = h.S->vz;
        if (int rc = run_pairs(c, OP_GRAD, p->prec, Mj, &P, &P, p->G, p->eps2, 0.0, 0, 0, A.jlv, A.jlv + n,
                               A.jlv + 2 * n))
            return rc;
    }
    if (c->dry) return BF_OK;
    TimestepArgs t{};
    t.P = h.M;
    t.set = devset(&P);
    t.dt_ff = A.dtff; t.dt_fb = A.dtfb;
    t.ax = A.alv; t.ay = A.alv + n; t.az = A.alv + 2 * n;
    if (grad) { t.gx = A.glv; t.gy = A.glv + n; t.gz = A.glv + 2 * n; }
    if (jerk) { t.jx = A.jlv; t.jy = A.jlv + n; t.jz = A.jlv + 2 * n; }
    t.eta_grad = A.eta_grad; t.eta_jerk = A.eta_jerk; t.tau = 1.0; t.kmax = 0;
    t.dt = A.dtl; t.level = nullptr;
    t.flags = c->d_flags;
    BF_HIP(launch_timestep(t, c->stream));
    return BF_OK;
}

int hhs_adapt(const HhsCtx& h, HhsAdapt& A, const bf_set& P, int k, double tau) {
    if (P.count == 0) return BF_OK;
    bf_ctx* c = h.c;
    const int64_t n = h.S->n;
    const bool top = k == 0;
    if (!top)
        if (int rc = level_timesteps(h, A, P)) return rc;
    BF_HIP(launch_pivot_flags(devset(&P), n, A.dt0, top ? nullptr : A.dtl, tau, k >= h.kmax, A.flag, c->d_flags,
                              c->stream));
    // Level k's split goes to the buffer its previous split is not in, and is compared with it.
    // Between two visits of level k only FSI cycles of shallower levels drift particles, each
    // over its own slow set (or its whole set when its fast set is empty).  While every
    // shallower level keeps its split and its fast set, the particles of level k and deeper
    // therefore stay where they were, and equal lists keep level k's own accelerations (same
    // slow set) and its inter-level accelerations (same slow and fast sets) valid, as for fixed
    // levels.  A level whose split changes, or whose fast set is empty, drops what every deeper
    // level kept: the next visit of a deeper level starts afresh.
    const bool had = A.prev_n[k] >= 0;
    const int cur = had ? 1 - A.which[k] : 0;
    int32_t* mine = A.lists + ((size_t)k * 2 + cur) * A.cap;
    const int32_t* prev = had ? A.lists + ((size_t)k * 2 + (1 - cur)) * A.cap : nullptr;
    int64_t cnt[2];
    bool same[2] = {false, false};
    if (int rc = partition_impl(c, &P, n, A.flag, 1, mine, cnt, prev, had ? (int)A.prev_n[k] : 0,
                                had ? (int)A.prev_n0[k] : 0, A.diff, same))
        return rc;
    A.which[k] = cur;
    A.prev_n[k] = P.count;
    A.prev_n0[k] = cnt[0];
    if (!same[0]) h.a_ok[k] = false;
    if (!same[1]) h.il_ok[k] = false;
    if (!same[1] || cnt[1] == 0)
        for (int d = k + 1; d < 64; ++d) {
            A.prev_n[d] = -1;
            h.a_ok[d] = h.il_ok[d] = false;
        }
    A.max_level = std::max(A.max_level, k);
    ++A.nodes;
    const bf_set Sset{mine, (int32_t)cnt[0], 0}, Fset{mine + cnt[0], (int32_t)cnt[1], 0};
    const bf_set Bset{mine, (int32_t)(cnt[0] + cnt[1]), 0};
    return hhs_cycle(h, Sset, Fset, Bset, tau, k, [&]() { return hhs_adapt(h, A, Fset, k + 1, 0.5 * tau); });
}

}  // namespace

static int hhs_setup(bf_ctx* c, const bf_state* S, const bf_set* set, const int32_t* level, int kmax, double tau,
                     const bf_fsi_params* prm, HhsCtx& h) {
    if (int rc = check_ctx(c)) return rc;
    if (int rc = check_state(S)) return rc;
    if (int rc = check_set(set, S->n, "hhs")) return rc;
    if (int rc = check_fsi_params(prm)) return rc;
    if (!level) return fail(BF_ERR_ARG, "level NULL");
    if (kmax < 0 || kmax > 63) return fail(BF_ERR_ARG, "kmax must be in [0, 63]");
    if (!(isfinite(tau) && tau > 0)) return fail(BF_ERR_ARG, "tau must be finite and > 0");
    const int64_t n = S->n;
    const size_t ob = ((size_t)std::max(set->count, 1) * 4 + 255) & ~size_t(255);
    if (int rc = ensure(&c->scratch7, &c->scratch7_bytes, ob + (size_t)12 * n * sizeof(double), c->stream)) return rc;
    h.c = c;
    h.S = S;
    h.prm = prm;
    bf_particles P{S->x, S->y, S->z, S->vx, S->vy, S->vz, S->m, n};
    h.M = masters_of(&P);
    int32_t* order = static_cast<int32_t*>(c->scratch7);
    double* d = reinterpret_cast<double*>(static_cast<char*>(c->scratch7) + ob);
    h.asf = d; h.gsf = d + 3 * n; h.afsi = d + 6 * n; h.gfsi = d + 9 * n;
    h.order = order;
    h.kmax = kmax;
    int64_t counts[64];
    for (int k = 0; k < 64; ++k) counts[k] = 0;
    if (set->count > 0)
        if (int rc = partition_impl(c, set, n, level, kmax, order, counts)) return rc;
    h.begin[0] = 0;
    for (int k = 0; k <= kmax; ++k) h.begin[k + 1] = h.begin[k] + counts[k];
    // inter-level accelerations kept per level: one 3n array for each level with S and F
    const int64_t total = h.begin[kmax + 1];
    int nl = 0;
    for (int k = 0; k < kmax; ++k) nl += counts[k] > 0 && h.begin[k + 1] < total;
    if (nl > 0)
        if (int rc = ensure(&c->scratch11, &c->scratch11_bytes, (size_t)nl * 3 * n * sizeof(double), c->stream))
            return rc;
    for (int k = 0, i = 0; k < 64; ++k) {
        const bool split = k < kmax && counts[k] > 0 && h.begin[k + 1] < total;
        h.asf_lv[k] = split ? static_cast<double*>(c->scratch11) + (size_t)(i++) * 3 * n : nullptr;
    }
    h.reuse = c->hhs_reuse;
    if (prm->n_bh > 0 && set->count > 0) {
        // the levels of the black holes, once per interval (the partition has synchronised)
        unsigned long long mask = ~0ull;
        hipLaunchKernelGGL(k_bh_level_mask, dim3(1), dim3(256), 0, c->stream, prm->bh_idx, prm->n_bh, level, n,
                           c->d_stats + 4);
        BF_HIP(hipGetLastError());
        BF_HIP(hipMemcpyAsync(&mask, c->d_stats + 4, sizeof(mask), hipMemcpyDeviceToHost, c->stream));
        BF_HIP(hipStreamSynchronize(c->stream));
        h.bh_known = true;
        h.bh_levels = mask;
    }
    return BF_OK;
}

BF_API int bf_hhs_interval(bf_ctx* c, const bf_state* S, const bf_set* set, const int32_t* level, int kmax, double tau,
                           const bf_fsi_params* prm) {
    g_err.clear();
    HhsCtx h;
    if (int rc = hhs_setup(c, S, set, level, kmax, tau, prm, h)) return rc;
    if (set->count == 0) return BF_OK;
    return hhs_run(h, tau);
}

BF_API int bf_graph_capture_hhs_interval(bf_ctx* c, const bf_state* S, const bf_set* set, const int32_t* level,
                                         int kmax, double tau, const bf_fsi_params* prm, void** graph_exec) {
    g_err.clear();
    if (int rc = check_ctx(c)) return rc;
    if (!graph_exec) return fail(BF_ERR_ARG, "graph pointer NULL");
    *graph_exec = nullptr;
    // The graph gets buffers of its own: park the context's while the interval is sized and
    // captured, then hand the new ones to the graph and give the context its own back.
    constexpr int kSlots = 9;
    void** slot[kSlots] = {&c->scratch,  &c->scratch2, &c->scratch5,  &c->scratch6, &c->scratch7,
                           &c->scratch8, &c->scratch9, &c->scratch10, &c->scratch11};
    size_t* slot_bytes[kSlots] = {&c->scratch_bytes,  &c->scratch2_bytes, &c->scratch5_bytes,
                                  &c->scratch6_bytes, &c->scratch7_bytes, &c->scratch8_bytes,
                                  &c->scratch9_bytes, &c->scratch10_bytes, &c->scratch11_bytes};
    void* parked[kSlots];
    size_t parked_bytes[kSlots];
    for (int i = 0; i < kSlots; ++i) {
        parked[i] = *slot[i];
        parked_bytes[i] = *slot_bytes[i];
        *slot[i] = nullptr;
        *slot_bytes[i] = 0;
    }
    auto unpark = [&](bool free_new) {
        for (int i = 0; i < kSlots; ++i) {
            if (free_new && *slot[i]) hipFree(*slot[i]);
            *slot[i] = parked[i];
            *slot_bytes[i] = parked_bytes[i];
        }
    };
    HhsCtx h;
    int rc = hhs_setup(c, S, set, level, kmax, tau, prm, h);
    if (!rc && set->count == 0) rc = fail(BF_ERR_ARG, "empty set: nothing to capture");
    if (rc) {
        hipStreamSynchronize(c->stream);
        unpark(true);
        return rc;
    }
    c->capturing = true;  // no timing events inside the graph; graph-safe sorts
    c->dry = true;
    rc = hhs_run(h, tau);
    c->dry = false;
    hipStream_t user = c->stream, cap = nullptr;
    hipGraph_t g = nullptr;
    if (!rc && hipStreamSynchronize(user) != hipSuccess) rc = fail(BF_ERR_HIP, "stream synchronisation failed");
    if (!rc && hipStreamCreateWithFlags(&cap, hipStreamNonBlocking) != hipSuccess)
        rc = fail(BF_ERR_HIP, "capture stream creation failed");
    if (!rc) {
        hipError_t e = hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal);
        if (e != hipSuccess) {
            rc = fail(BF_ERR_HIP, hipGetErrorString(e));
        } else {
            c->stream = cap;
            rc = hhs_run(h, tau);
            c->stream = user;
            e = hipStreamEndCapture(cap, &g);
            if (!rc && e != hipSuccess) rc = fail(BF_ERR_HIP, hipGetErrorString(e));
        }
    }
    if (cap) hipStreamDestroy(cap);
    c->capturing = false;
    bf_graph* gr = nullptr;
    if (!rc) {
        gr = new bf_graph();
        gr->graph = g;
        if (hipGraphInstantiate(&gr->exec, g, nullptr, nullptr, 0) != hipSuccess) {
            rc = fail(BF_ERR_HIP, "graph instantiation failed");
            delete gr;
            gr = nullptr;
        }
    }
    if (rc) {
        if (g) hipGraphDestroy(g);
        hipStreamSynchronize(user);
        unpark(true);
        return rc;
    }
    for (int i = 0; i < kSlots; ++i) gr->owned[i] = *slot[i];
    unpark(false);
    *graph_exec = gr;
    return BF_OK;
}

BF_API int bf_hhs_interval_adaptive(bf_ctx* c, const bf_state* S, const bf_set* set, const double* dt0, int kmax,
                                    double tau, double eta_ff, double eta_fb, double eta_grad, double eta_jerk,
                                    const bf_fsi_params* prm, int* max_level, int64_t* n_levels) {
    g_err.clear();
    if (int rc = check_ctx(c)) return rc;
    if (int rc = check_state(S)) return rc;
    if (int rc = check_set(set, S->n, "hhs")) return rc;
    if (int rc = check_fsi_params(prm)) return rc;
    if (!dt0) return fail(BF_ERR_ARG, "dt0 NULL");
    if (kmax < 0 || kmax > 63) return fail(BF_ERR_ARG, "kmax must be in [0, 63]");
    if (!(isfinite(tau) && tau > 0)) return fail(BF_ERR_ARG, "tau must be finite and > 0");
    if (!(isfinite(eta_ff) && eta_ff > 0) || !(isfinite(eta_fb) && eta_fb > 0))
        return fail(BF_ERR_ARG, "eta_ff and eta_fb must be finite and > 0");
    if (!finite_nonneg(eta_grad) || !finite_nonneg(eta_jerk))
        return fail(BF_ERR_ARG, "eta_grad and eta_jerk must be finite and >= 0");
    if (max_level) *max_level = -1;
    if (n_levels) *n_levels = 0;
    if (set->count == 0) return BF_OK;
    const int64_t n = S->n, cap = set->count;
    const size_t lb = ((size_t)2 * (kmax + 1) * cap * 4 + 255) & ~size_t(255);
    const size_t fb = (((size_t)n * 4 + 255) & ~size_t(255)) + 256;  // the flags, then the split diff
    if (int rc = ensure(&c->scratch7, &c->scratch7_bytes, lb + fb + (size_t)24 * n * sizeof(double), c->stream))
        return rc;
    // every level may split: an inter-level acceleration array (3n) for each
    if (int rc = ensure(&c->scratch11, &c->scratch11_bytes, (size_t)(kmax + 1) * 3 * n * sizeof(double), c->stream))
        return rc;
    HhsCtx h;
    h.c = c;
    h.S = S;
    h.prm = prm;
    bf_particles P{S->x, S->y, S->z, S->vx, S->vy, S->vz, S->m, n};
    h.M = masters_of(&P);
    h.order = nullptr;
    h.kmax = kmax;
    char* base = static_cast<char*>(c->scratch7);
    double* d = reinterpret_cast<double*>(base + lb + fb);
    h.asf = d; h.gsf = d + 3 * n; h.afsi = d + 6 * n; h.gfsi = d + 9 * n;
    HhsAdapt A;
    A.dt0 = dt0;
    A.eta_ff = eta_ff;
    A.eta_fb = eta_fb;
    A.eta_grad = eta_grad;
    A.eta_jerk = eta_jerk;
    A.dtff = d + 12 * n;
    A.dtfb = d + 13 * n;
    A.dtl = d + 14 * n;
    A.alv = d + 15 * n;
    A.glv = d + 18 * n;
    A.jlv = d + 21 * n;
    A.flag = reinterpret_cast<int32_t*>(base + lb);
    A.diff = reinterpret_cast<int32_t*>(base + lb + fb - 256);
    A.lists = reinterpret_cast<int32_t*>(base);
    A.cap = cap;
    A.max_level = -1;
    A.nodes = 0;
    for (int k = 0; k < 64; ++k) {
        A.which[k] = 0;
        A.prev_n[k] = A.prev_n0[k] = -1;
        h.a_ok[k] = h.il_ok[k] = false;
        h.asf_lv[k] = k <= kmax ? static_cast<double*>(c->scratch11) + (size_t)k * 3 * n : nullptr;
    }
    h.reuse = c->hhs_reuse;
    const int rc = hhs_adapt(h, A, *set, 0, tau);
    if (max_level) *max_level = A.max_level;
    if (n_levels) *n_levels = A.nodes;
    return rc;
}

// ---- configuration, tuning -------------------------------------------------------------------

BF_API int bf_last_pass_stats(bf_ctx* c, int64_t* fixups, int64_t* near_tiles, int64_t* far_tiles) {
    if (int rc = check_ctx(c)) return rc;
    unsigned long long h[3];
    BF_HIP(hipMemcpyAsync(h, c->d_stats, sizeof(h), hipMemcpyDeviceToHost, c->stream));
    BF_HIP(hipStreamSynchronize(c->stream));
    if (fixups) *fixups = (int64_t)(h[0] & 0xffffffffull);
    if (near_tiles) *near_tiles = (int64_t)h[1];
    if (far_tiles) *far_tiles = (int64_t)h[2];
    return BF_OK;
}

BF_API int bf_pair_credit(bf_ctx* c, int op, int64_t* pairs, int reset) {
    if (int rc = check_ctx(c)) return rc;
    if (op < 0 || op >= OP_COUNT) return fail(BF_ERR_ARG, "bad op");
    if (!pairs) return fail(BF_ERR_ARG, "pairs NULL");
    *pairs = c->pair_credit[op];
    if (reset) c->pair_credit[op] = 0;
    return BF_OK;
}

BF_API int bf_last_pass_config(bf_ctx* c, int* kind, int* k, int* waves, int* split) {
    if (int rc = check_ctx(c)) return rc;
    if (kind) *kind = c->last_kind;
    if (k) *k = c->last_k;
    if (waves) *waves = c->last_waves;
    if (split) *split = c->last_split;
    return BF_OK;
}

BF_API int bf_set_spatial_sort(bf_ctx* c, int ops_mask, double kappa) {
    if (int rc = check_ctx(c)) return rc;
    if (ops_mask & ~((1 << OP_ACC) | (1 << OP_GRAD) | (1 << OP_DT) | BF_SORT_ANY_SIZE | BF_SORT_DIRECTED))
        return fail(BF_ERR_ARG, "ops_mask: only the force, gradient and time-step passes, BF_SORT_ANY_SIZE and "
                                "BF_SORT_DIRECTED");
    if (kappa != 0.0 && !(kappa >= kKappaMin && kappa <= kKappaMax))
        return fail(BF_ERR_ARG, "kappa must be 0 (keep) or in [0.5, 64]");
    c->sort_ops = ops_mask;
    if (kappa != 0.0) c->kappa = (float)kappa;
    return BF_OK;
}

BF_API int bf_set_hhs_reuse(bf_ctx* c, int on) {
    if (int rc = check_ctx(c)) return rc;
    c->hhs_reuse = on != 0;
    return BF_OK;
}

BF_API int bf_neighbours(bf_ctx* c, const bf_particles* P, const bf_set* t, const bf_set* s, double G, double r_ngb,
                         double r_max, double C, double tau, int32_t* edges, int64_t cap, int64_t* n_edges) {
    g_err.clear();
    if (int rc = check_ctx(c)) return rc;
    if (int rc = check_particles(P, true)) return rc;
    if (int rc = check_set(t, P->n, "target")) return rc;
    if (int rc = check_set(s, P->n, "source")) return rc;
    if (!(isfinite(G) && G > 0)) return fail(BF_ERR_ARG, "G must be finite and > 0");
    if (!(isfinite(r_ngb) && r_ngb > 0) || !(isfinite(r_max) && r_max > 0))
        return fail(BF_ERR_ARG, "r_ngb and r_max must be finite and > 0");
    if (!(isfinite(C) && C > 0) || !(isfinite(tau) && tau > 0)) return fail(BF_ERR_ARG, "C and tau must be finite and > 0");
    if (!n_edges) return fail(BF_ERR_ARG, "n_edges NULL");
    if (cap < 0 || (cap > 0 && !edges)) return fail(BF_ERR_ARG, "bad edge buffer");
    *n_edges = 0;
    if (t->count == 0 || s->count == 0) return BF_OK;
    const int64_t capk = std::max<int64_t>(cap, 1);
    const size_t kb = ((size_t)capk * 8 + 255) & ~size_t(255);
    const size_t tmp = ngb_sort_tmp_bytes(capk);
    if (int rc = ensure(&c->scratch4, &c->scratch4_bytes, 256 + 2 * kb + tmp, c->stream)) return rc;
    char* b = static_cast<char*>(c->scratch4);
    NgbArgs a{};
    a.P = masters_of(P);
    a.tgt = devset(t);
    a.src = devset(s);
    a.G = G;
    a.r_ngb = r_ngb;
    a.r_max2 = r_max * r_max;
    a.C = C;
    a.tau = tau;
    a.count = reinterpret_cast<unsigned long long*>(b);
    a.keys = reinterpret_cast<unsigned long long*>(b + 256);
    a.cap = cap;
    a.flags = c->d_flags;
    constexpr int T = 256;
    const int64_t nslabs = (t->count + T * kNgbK - 1) / (T * kNgbK), ntiles = (s->count + T - 1) / T;
    int64_t split = std::max<int64_t>(1, (8 * (int64_t)c->num_cu + nslabs - 1) / nslabs);
    split = std::min(split, ntiles);
    const int64_t tiles_per_chunk = (ntiles + split - 1) / split;
    split = (ntiles + tiles_per_chunk - 1) / tiles_per_chunk;
    a.split = (int32_t)split;
    a.chunk = (int32_t)(tiles_per_chunk * T);
    if (nslabs * split > INT32_MAX) return fail(BF_ERR_UNSUPPORTED, "grid too large");
    BF_HIP(launch_zero_u64(a.count, 1, c->stream));
    BF_HIP(launch_ngb(a, 4, (int)(nslabs * split), c->stream));
    unsigned long long found = 0;
    BF_HIP(hipMemcpyAsync(&found, a.count, sizeof(found), hipMemcpyDeviceToHost, c->stream));
    BF_HIP(hipStreamSynchronize(c->stream));
    *n_edges = (int64_t)found;
    if ((int64_t)found > cap) return fail(BF_ERR_NOMEM, "edge buffer too small: " + std::to_string(found) + " pairs found");
    BF_HIP(launch_ngb_finish(a.keys, reinterpret_cast<unsigned long long*>(b + 256 + kb), (int64_t)found,
                             b + 256 + 2 * kb, tmp, edges, c->stream));
    return BF_OK;
}

BF_API int bf_subsystems(bf_ctx* c, int64_t n, const int32_t* edges, int64_t m, int32_t* label, int64_t* n_sub) {
    g_err.clear();
    if (int rc = check_ctx(c)) return rc;
    if (n <= 0 || n > INT32_MAX) return fail(BF_ERR_ARG, "n must be in [1, 2^31)");
    if (m < 0 || (m > 0 && !edges)) return fail(BF_ERR_ARG, "bad edge list");
    if (!label) return fail(BF_ERR_ARG, "label NULL");
    const size_t mb = ((size_t)n * 4 + 255) & ~size_t(255);
    if (int rc = ensure(&c->scratch4, &c->scratch4_bytes, 256 + mb, c->stream)) return rc;
    int32_t* word = static_cast<int32_t*>(c->scratch4);
    int32_t* mark = reinterpret_cast<int32_t*>(static_cast<char*>(c->scratch4) + 256);
    BF_HIP(launch_label_init(label, n, word, c->stream));
    // every round that changes something lowers at least one label, so this ends
    for (int64_t round = 0;; ++round) {
        if (round > n + 64) return fail(BF_ERR_HIP, "label propagation did not settle");
        BF_HIP(launch_label_round(edges, m, n, label, word, c->d_flags, c->stream));
        int32_t changed = 0;
        BF_HIP(hipMemcpyAsync(&changed, word, sizeof(changed), hipMemcpyDeviceToHost, c->stream));
        BF_HIP(hipStreamSynchronize(c->stream));
        if (!changed) break;
    }
    if (n_sub) {
        BF_HIP(launch_label_count(label, n, mark, word, c->stream));
        int32_t cnt = 0;
        BF_HIP(hipMemcpyAsync(&cnt, word, sizeof(cnt), hipMemcpyDeviceToHost, c->stream));
        BF_HIP(hipStreamSynchronize(c->stream));
        *n_sub = cnt;
    }
    return BF_OK;
}

BF_API int bf_set_subsystems(bf_ctx* c, const int32_t* label, int64_t n) {
    if (int rc = check_ctx(c)) return rc;
    if (label && (n <= 0 || n > INT32_MAX)) return fail(BF_ERR_ARG, "n must be in [1, 2^31)");
    c->sub = label;
    c->sub_n = label ? n : 0;
    return BF_OK;
}

BF_API int bf_query_config(bf_ctx* c, int op, int prec, int64_t nt, int64_t ns, int* k, int* waves, int* split) {
    if (int rc = check_ctx(c)) return rc;
    if (op < 0 || op >= OP_COUNT) return fail(BF_ERR_ARG, "bad op");
    if (int rc = check_prec(prec)) return rc;
    if (nt <= 0 || ns <= 0) return fail(BF_ERR_ARG, "sizes must be > 0");
    Plan p;
    if (int rc = plan(c, op, prec, nt, ns, p, use_sorted(c, op, prec, nt, ns, 0.0))) return rc;
    if (k) *k = p.cfg.k;
    if (waves) *waves = p.cfg.waves;
    if (split) *split = p.split;
    return BF_OK;
}

BF_API int bf_set_config(bf_ctx* c, int op, int prec, int k, int waves, int split) {
    if (int rc = check_ctx(c)) return rc;
    if (op < 0 || op >= OP_COUNT) return fail(BF_ERR_ARG, "bad op");
    if (int rc = check_prec(prec)) return rc;
    if (k == 0) { c->forced[op][prec] = KernelConfig{}; return BF_OK; }
    if (!variant_exists(op, prec, k, waves)) return fail(BF_ERR_UNSUPPORTED, "no such kernel variant");
    if (split < 0) return fail(BF_ERR_ARG, "split < 0");
    c->forced[op][prec] = KernelConfig{k, waves, split};
    return BF_OK;
}

static int write_cache(bf_ctx* c, const char* path) {
    std::ofstream f(path);
    if (!f) return fail(BF_ERR_ARG, std::string("cannot write ") + path);
    f << "[\n";
    size_t i = 0;
    for (const auto& kv : c->tuned) {
        f << "  {\"op\": " << std::get<0>(kv.first) << ", \"prec\": " << std::get<1>(kv.first)
          << ", \"sweep\": " << std::get<2>(kv.first) << ", \"nt_log2\": " << std::get<3>(kv.first)
          << ", \"ns_log2\": " << std::get<4>(kv.first) << ", \"k\": " << kv.second.k
          << ", \"waves\": " << kv.second.waves << ", \"split\": " << kv.second.split << "}"
          << (++i < c->tuned.size() ? ",\n" : "\n");
    }
    f << "]\n";
    return BF_OK;
}

// a table entry names an instantiated shape
static bool tuned_entry_ok(int op, int prec, int sweep, int k, int w, int sp) {
    if (op < 0 || op >= OP_COUNT || (prec != 0 && prec != 1) || sp < 0) return false;
    if (sweep == kTuneDirected) return variant_exists(op, prec, k, w);
    if (sweep == kTuneSymmetric) return prec == BF_PREC_MIXED && sym_variant_exists(op, w, k);
    if (sweep == kTuneBatched) return bf_internal_batch_shape_ok(op, prec, k, w, sp);
    return false;
}

BF_API int bf_autotune_load(bf_ctx* c, const char* path) {
    if (int rc = check_ctx(c)) return rc;
    if (!path) return fail(BF_ERR_ARG, "path NULL");
    std::ifstream f(path);
    if (!f) return fail(BF_ERR_ARG, std::string("cannot read ") + path);
    std::string line;
    while (std::getline(f, line)) {
        int op, prec, sw = kTuneDirected, bt, bs, k, w, sp;
        const bool v2 = sscanf(line.c_str(), " {\"op\": %d, \"prec\": %d, \"sweep\": %d, \"nt_log2\": %d, \"ns_log2\": "
                                             "%d, \"k\": %d, \"waves\": %d, \"split\": %d",
                               &op, &prec, &sw, &bt, &bs, &k, &w, &sp) == 8;
        // tables written before the sweep kind existed hold directed entries only
        const bool v1 = !v2 && sscanf(line.c_str(), " {\"op\": %d, \"prec\": %d, \"nt_log2\": %d, \"ns_log2\": %d, "
                                                    "\"k\": %d, \"waves\": %d, \"split\": %d",
                                      &op, &prec, &bt, &bs, &k, &w, &sp) == 7;
        if (v1) sw = kTuneDirected;
        if ((v1 || v2) && tuned_entry_ok(op, prec, sw, k, w, sp))
            c->tuned[std::make_tuple(op, prec, sw, bt, bs)] = KernelConfig{k, w, sp};
    }
    return BF_OK;
}

// synthetic particles for tuning: uniform in the unit cube
__global__ void k_tune_fill(double* x, double* y, double* z, double* v, double* m, int64_t n) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    uint64_t h = (uint64_t)i * 0x9E3779B97F4A7C15ull + 0x1234567ull;
    auto nxt = [&h]() {
        h ^= h >> 33; h *= 0xff51afd7ed558ccdull; h ^= h >> 33; h *= 0xc4ceb9fe1a85ec53ull; h ^= h >> 33;
        return (double)(h >> 11) * (1.0 / 9007199254740992.0);
    };
    x[i] = nxt(); y[i] = nxt(); z[i] = nxt();
    v[i] = nxt() - 0.5; v[n + i] = nxt() - 0.5; v[2 * n + i] = nxt() - 0.5;
    m[i] = 1.0 / (double)n;
}

extern "C++" {
namespace {

// Time `run` once after one warm-up call (HIP events on the context stream), in ms; < 0 on error
// (the error is left in rc).
template <class Run>
float time_candidate(bf_ctx* c, Run&& run, int& rc) {
    rc = run();
    if (rc) return -1.f;
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess) return -1.f;
    if (hipEventCreate(&e1) != hipSuccess) {
        hipEventDestroy(e0);
        return -1.f;
    }
    hipEventRecord(e0, c->stream);
    rc = run();
    hipEventRecord(e1, c->stream);
    float ms = -1.f;
    if (!rc && hipEventSynchronize(e1) == hipSuccess) hipEventElapsedTime(&ms, e0, e1);
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    return rc ? -1.f : ms;
}

// Directed passes: targets per lane x waves per workgroup x source split (the automatic split
// and 1/4, 1/2 and 2 times it).  The pass is timed on tg (the caller's sample) against sr; the
// winner is stored for the bucket of (nt_bucket, ns_bucket).
int tune_directed(bf_ctx* c, int op, int prec, const Masters& M, const bf_set& tg, const bf_set& sr, int64_t nt_bucket,
                  int64_t ns_bucket, double* o) {
    const int64_t n = M.n;
    const KernelConfig saved = c->forced[op][prec];
    KernelConfig best{};
    float best_ms = 1e30f;
    int rc = BF_OK;
    const bool sorted = use_sorted(c, op, prec, tg.count, sr.count, 0.0);
    const int ks[] = {1, 2, 4};
    const int ws[] = {2, 4, 8};
    for (int k : ks) {
        for (int w : ws) {
            if (!variant_exists(op, prec, k, w) || (sorted && !sorted_variant_exists(op, k, w))) continue;
            c->forced[op][prec] = KernelConfig{k, w, 0};
            Plan p;
            if ((rc = plan(c, op, prec, tg.count, sr.count, p, sorted))) break;
            const int s0 = p.split;
            const int cand[] = {0, std::max(1, s0 / 4), std::max(1, s0 / 2), 2 * s0};
            int tried[4];
            int nt_ = 0;
            for (int ci = 0; ci < 4; ++ci) {
                // the split a forced value turns into (whole groups, at most one chunk per group)
                c->forced[op][prec] = KernelConfig{k, w, cand[ci]};
                Plan q;
                if ((rc = plan(c, op, prec, tg.count, sr.count, q, sorted))) break;
                const int es = q.split;
                bool dup = false;
                for (int t = 0; t < nt_; ++t) dup = dup || tried[t] == es;
                if (dup) continue;
                tried[nt_++] = es;
                const float ms = time_candidate(c, [&]() {
                    return run_pairs(c, op, prec, M, &tg, &sr, 1.0, 0.0, 0.0, 0.2, 0.2, o, o + n, o + 2 * n);
                }, rc);
                if (rc) break;
                if (ms >= 0.f && ms < best_ms) {
                    best_ms = ms;
                    best = KernelConfig{k, w, ci == 0 ? 0 : es};  // 0: automatic for each size
                }
            }
            if (rc) break;
        }
        if (rc) break;
    }
    c->forced[op][prec] = saved;
    if (rc) return rc;
    if (best.k == 0) return fail(BF_ERR_UNSUPPORTED, "no variant ran");
    c->tuned[std::make_tuple(op, prec, (int)kTuneDirected, (int)nt_bucket, (int)ns_bucket)] = best;
    return BF_OK;
}

// Pair-symmetric sweeps over one set: (row tiles, waves) shapes x rounds of resident workgroups
// (1, 2, 4), timed on the caller's whole set.
int tune_symmetric(bf_ctx* c, int op, const Masters& M, const bf_set& set, double* o) {
    const int64_t n = M.n;
    const KernelConfig saved = c->sym_forced[op];
    KernelConfig best{};
    float best_ms = 1e30f;
    int rc = BF_OK;
    const int shapes[][2] = {{16, 1}, {8, 2}, {4, 4}};  // (waves, rows)
    for (const auto& sh : shapes) {
        if (!sym_variant_exists(op, sh[0], sh[1])) continue;
        for (int rounds : {4, 8, 16, 32, 64}) {
            c->sym_forced[op] = KernelConfig{sh[1], sh[0], rounds};
            const float ms = time_candidate(c, [&]() {
                return run_pairs(c, op, BF_PREC_MIXED, M, &set, &set, 1.0, 0.0, 0.0, 0.2, 0.2, o, o + n, o + 2 * n);
            }, rc);
            if (rc) break;
            if (c->last_kind != BF_PASS_SYMMETRIC) {  // the sweep did not apply (size, memory)
                c->sym_forced[op] = saved;
                return fail(BF_ERR_UNSUPPORTED, "this pass does not take the pair-symmetric sweep");
            }
            if (ms >= 0.f && ms < best_ms) {
                best_ms = ms;
                best = KernelConfig{sh[1], sh[0], rounds};
            }
        }
        if (rc) break;
    }
    c->sym_forced[op] = saved;
    if (rc) return rc;
    if (best.k == 0) return fail(BF_ERR_UNSUPPORTED, "no variant ran");
    c->tuned[std::make_tuple(op, (int)BF_PREC_MIXED, (int)kTuneSymmetric, ilog2_bucket(set.count),
                             ilog2_bucket(set.count))] = best;
    return BF_OK;
}

}  // namespace
}  // extern "C++"

BF_API int bf_autotune(bf_ctx* c, int op, int prec, int64_t nt, int64_t ns, const char* cache_path) {
    g_err.clear();
    if (int rc = check_ctx(c)) return rc;
    if (op < 0 || op >= OP_COUNT) return fail(BF_ERR_ARG, "bad op");
    if (int rc = check_prec(prec)) return rc;
    if (nt <= 0 || ns <= 0 || nt > INT32_MAX || ns > INT32_MAX) return fail(BF_ERR_ARG, "bad sizes");
    if (cache_path) {
        std::ifstream probe(cache_path);
        if (probe) bf_autotune_load(c, cache_path);
    }
    const int64_t n = std::max(nt, ns);
    double* buf = nullptr;
    // x y z vx vy vz m ax ay az out0 out1 out2
    if (hipMalloc(&buf, (size_t)13 * n * sizeof(double)) != hipSuccess) return fail(BF_ERR_NOMEM, "tuning buffers");
    double *x = buf, *y = x + n, *z = y + n, *v = z + n, *m = v + 3 * n, *a = m + n, *o = a + 3 * n;
    hipLaunchKernelGGL(k_tune_fill, dim3((n + 255) / 256), dim3(256), 0, c->stream, x, y, z, v, m, n);
    hipLaunchKernelGGL(k_tune_fill, dim3((n + 255) / 256), dim3(256), 0, c->stream, a, a + n, a + 2 * n, o, o + n, n);
    Masters M{};
    M.x = x; M.y = y; M.z = z; M.vx = v; M.vy = v + n; M.vz = v + 2 * n; M.m = m;
    M.ax = a; M.ay = a + n; M.az = a + 2 * n; M.n = n;
    // Large target sets are timed on a leading sample of targets (the rate per pair is what is
    // compared); an automatic split is recomputed for the real size when the entry is used.
    const int64_t nt_time = std::min<int64_t>(nt, (int64_t)1 << 17);
    const bf_set tg{nullptr, (int32_t)nt_time, 0}, sr{nullptr, (int32_t)ns, 0};
    const int32_t* saved_sub = c->sub;
    c->sub = nullptr;  // tuning runs on its own synthetic particles
    int rc = tune_directed(c, op, prec, M, tg, sr, ilog2_bucket(nt), ilog2_bucket(ns), o);
    c->sub = saved_sub;
    hipStreamSynchronize(c->stream);
    hipFree(buf);
    if (rc) return rc;
    if (cache_path) return write_cache(c, cache_path);
    return BF_OK;
}

BF_API int bf_autotune_pass(bf_ctx* c, int op, int prec, const bf_particles* P, const bf_set* targets,
                            const bf_set* sources, const double* ax, const double* ay, const double* az,
                            const char* cache_path) {
    g_err.clear();
    if (int rc = check_ctx(c)) return rc;
    if (op < 0 || op >= OP_COUNT) return fail(BF_ERR_ARG, "bad op");
    if (int rc = check_prec(prec)) return rc;
    if (int rc = check_particles(P, op == OP_DT)) return rc;
    if (int rc = check_set(targets, P->n, "target")) return rc;
    if (int rc = check_set(sources, P->n, "source")) return rc;
    if (targets->count == 0 || sources->count == 0) return fail(BF_ERR_ARG, "empty set");
    if (op == OP_GRAD && (!ax || !ay || !az)) return fail(BF_ERR_ARG, "the gradient needs the accelerations");
    if (cache_path) {
        std::ifstream probe(cache_path);
        if (probe) bf_autotune_load(c, cache_path);
    }
    const int64_t n = P->n;
    double* o = nullptr;
    if (hipMalloc(&o, (size_t)3 * n * sizeof(double)) != hipSuccess) return fail(BF_ERR_NOMEM, "tuning buffers");
    Masters M = masters_of(P);
    M.ax = ax; M.ay = ay; M.az = az;
    int rc = BF_OK;
    // the pass takes the pair-symmetric sweep: tune its shapes on the whole set
    const bool sorted = use_sorted(c, op, prec, targets->count, sources->count, 0.0);
    if ((sorted && use_symmetric(c, op, sorted, targets, sources)) || use_symmetric_dt(c, op, prec, targets, sources, 0.0)) {
        rc = tune_symmetric(c, op, M, *targets, o);
    } else {
        // directed: a leading sample of the targets (a sub-range or the head of the list)
        const int64_t nt_time = std::min<int64_t>(targets->count, (int64_t)1 << 17);
        bf_set tg = *targets;
        tg.count = (int32_t)nt_time;
        rc = tune_directed(c, op, prec, M, tg, *sources, ilog2_bucket(targets->count), ilog2_bucket(sources->count), o);
    }
    hipStreamSynchronize(c->stream);
    hipFree(o);
    if (rc) return rc;
    if (cache_path) return write_cache(c, cache_path);
    return BF_OK;
}

BF_API int bf_autotune_batched(bf_ctx* c, int op, int prec, const bf_particles* P, int32_t n_clusters,
                               const int64_t* cluster_off, const int32_t* active_idx, const int64_t* active_off,
                               int64_t max_active, int64_t max_cluster_n, const double* ax, const double* ay,
                               const double* az, const char* cache_path) {
    g_err.clear();
    if (int rc = check_ctx(c)) return rc;
    if (op != OP_ACC && op != OP_GRAD) return fail(BF_ERR_ARG, "batched passes: BF_OP_FORCES or BF_OP_GRADIENT");
    if (int rc = check_prec(prec)) return rc;
    if (int rc = check_particles(P, false)) return rc;
    if (op == OP_GRAD && (!ax || !ay || !az)) return fail(BF_ERR_ARG, "the gradient needs the accelerations");
    if (max_active <= 0 || max_cluster_n <= 0) return fail(BF_ERR_ARG, "bad bounds");
    if (cache_path) {
        std::ifstream probe(cache_path);
        if (probe) bf_autotune_load(c, cache_path);
    }
    const int64_t n = P->n;
    double* o = nullptr;
    if (hipMalloc(&o, (size_t)3 * n * sizeof(double)) != hipSuccess) return fail(BF_ERR_NOMEM, "tuning buffers");
    const KernelConfig saved = c->batch_forced[op];
    KernelConfig best{};
    float best_ms = 1e30f;
    int rc = BF_OK;
    for (int k : {1, 2, 4}) {
        for (int w : {4, 8}) {
            for (int chunk : {2048, 4096, 8192}) {
                if (!bf_internal_batch_shape_ok(op, prec, k, w, chunk)) continue;
                c->batch_forced[op] = KernelConfig{k, w, chunk};
                const float ms = time_candidate(c, [&]() {
                    return op == OP_ACC ? bf_forces_batched(c, P, n_clusters, cluster_off, active_idx, active_off,
                                                            max_active, max_cluster_n, 1.0, 0.0, prec, 0.0, o, o + n,
                                                            o + 2 * n)
                                        : bf_force_gradient_batched(c, P, n_clusters, cluster_off, active_idx,
                                                                    active_off, max_active, max_cluster_n, ax, ay, az,
                                                                    1.0, 0.0, prec, 0.0, o, o + n, o + 2 * n);
                }, rc);
                if (rc) break;
                if (ms >= 0.f && ms < best_ms) {
                    best_ms = ms;
                    best = KernelConfig{k, w, chunk};
                }
            }
            if (rc) break;
        }
        if (rc) break;
    }
    c->batch_forced[op] = saved;
    hipStreamSynchronize(c->stream);
    hipFree(o);
    if (rc) return rc;
    if (best.k == 0) return fail(BF_ERR_UNSUPPORTED, "no variant ran");
    c->tuned[std::make_tuple(op, prec, (int)kTuneBatched, ilog2_bucket(max_active), ilog2_bucket(max_cluster_n))] =
        best;
    if (cache_path) return write_cache(c, cache_path);
    return BF_OK;
}

BF_API int bf_set_symmetric_config(bf_ctx* c, int op, int rows, int waves, int rounds) {
    if (int rc = check_ctx(c)) return rc;
    if (op < 0 || op >= OP_COUNT) return fail(BF_ERR_ARG, "bad op");
    if (rows == 0) { c->sym_forced[op] = KernelConfig{}; return BF_OK; }
    if (!sym_variant_exists(op, waves, rows)) return fail(BF_ERR_UNSUPPORTED, "no such symmetric shape");
    if (rounds < 0 || rounds > 64) return fail(BF_ERR_ARG, "rounds must be in [0, 64]");
    c->sym_forced[op] = KernelConfig{rows, waves, rounds};
    return BF_OK;
}

BF_API int bf_set_symmetric_scratch_limit(bf_ctx* c, size_t bytes) {
    if (int rc = check_ctx(c)) return rc;
    c->sym_limit = bytes;
    return BF_OK;
}

BF_API int bf_last_symmetric_passes(bf_ctx* c, int* passes) {
    if (int rc = check_ctx(c)) return rc;
    if (!passes) return fail(BF_ERR_ARG, "passes NULL");
    *passes = c->last_passes;
    return BF_OK;
}

BF_API int bf_set_batched_config(bf_ctx* c, int op, int prec, int k, int waves, int chunk) {
    if (int rc = check_ctx(c)) return rc;
    if (op != OP_ACC && op != OP_GRAD) return fail(BF_ERR_ARG, "batched passes: BF_OP_FORCES or BF_OP_GRADIENT");
    if (int rc = check_prec(prec)) return rc;
    if (k == 0) { c->batch_forced[op] = KernelConfig{}; return BF_OK; }
    if (!bf_internal_batch_shape_ok(op, prec, k, waves, chunk))
        return fail(BF_ERR_UNSUPPORTED, "no such batched shape (chunk: a positive multiple of 64 * waves)");
    c->batch_forced[op] = KernelConfig{k, waves, chunk};
    return BF_OK;
}

}  // extern "C"
