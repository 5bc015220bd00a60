// Internal declarations of libbifrost_hip: context, kernel argument blocks, launchers.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <map>
#include <string>
#include <tuple>
#include <utility>
#include <vector>

#include "bifrost.h"

namespace bf {

// ---- argument blocks (passed by value to kernels) ----------------------------------------

// A set as the kernels see it: slot k -> particle idx ? idx[k] : begin + k.
struct DevSet {
    const int32_t* idx;
    int32_t count;
    int32_t begin;
};

// FP64 master arrays.
struct Masters {
    const double *x, *y, *z, *vx, *vy, *vz, *m;
    const double *ax, *ay, *az;  // gradient input (particle-indexed), else null
    int64_t n;
};

// Everything a pair kernel needs.
struct PairArgs {
    Masters P;
    DevSet tgt;       // targets
    DevSet src;       // sources
    const void* pack; // packed source stream (op/precision dependent layout), length src.count
    double G;
    double eps2;      // softening (FP64 path)
    float eps2f;      // eps2 + tiny (FP32 path; tiny keeps the self pair finite)
    float rfb2f;      // close-pair threshold on s^2 for the FP64 re-evaluation
    int32_t split;    // number of source chunks
    int32_t chunk;    // sources per chunk (multiple of the tile size)
    double* part;     // [split][ncomp][tgt.count] partial results when split > 1
    double *o0, *o1, *o2;  // particle-indexed outputs when split == 1
    double eta0, eta1;     // dt_min: eta_ff, eta_fb
    const void* pack_far;     // spatially sorted mode: FP32 tile-relative source stream
    const double4* tile_meta; // spatially sorted mode: per tile (centre, extent) [, (a centre, 0)]
    float kappa;              // spatially sorted mode: a tile is near when gap < kappa * extent
    double cond_max;       // mixed acc/grad: FP64 fix-up when magnitude estimate > cond_max |result|
    int32_t* fix_list;     // [tgt.count] target slots queued for the FP64 fix-up
    int32_t* fix_count;    // number of queued slots
    unsigned long long* tile_stats;  // sorted mode: [near tiles, far tiles] visited (NULL: not counted)
    unsigned long long* pass_stats;  // [fix-ups, near, far] of the pass: the fix-up writes entry 0 (NULL: not)
    const int32_t* sub;    // particle-indexed subsystem labels (NULL: no exclusion)
    uint32_t* flags;
};

enum Op { OP_ACC = 0, OP_GRAD = 1, OP_DT = 2, OP_COUNT = 3 };

struct KernelConfig {
    int k = 0;      // targets per lane (symmetric sweep: row tiles per wavefront)
    int waves = 0;  // waves per workgroup
    int split = 0;  // source chunks (0 = automatic); symmetric: rounds of resident workgroups the
                    // distance shares aim at (0 = 2); batched: sources per work item (0 = 4096)
};
enum { kTuneDirected = 0, kTuneSymmetric = 1, kTuneBatched = 2 };

// Launch one pair kernel (returns the hip error of the launch).
hipError_t launch_pairs(int op, int prec, const KernelConfig& cfg, const PairArgs& a, int nblocks,
                        hipStream_t st);
// Is (k, waves) an instantiated variant?
bool variant_exists(int op, int prec, int k, int waves, bool excl = false);
// Resident workgroups per CU for a variant (occupancy API), 0 if unknown.
int variant_blocks_per_cu(int op, int prec, int k, int waves, bool excl = false);
// Bytes per packed source for op/prec.
int pack_bytes(int op, int prec);

// Stored components per target (results, plus the magnitude estimate of the mixed acc/grad).
int stored_components(int op, int prec);

// begin: 0, or start the pass as well (1: clear a.pass_stats; 2: and *a.fix_count)
hipError_t launch_pack(int op, int prec, const PairArgs& a, hipStream_t st, int begin = 0);
hipError_t launch_reduce(int op, int prec, const PairArgs& a, hipStream_t st);
// Mixed acceleration / gradient pass over few targets and sources in one launch (no source
// split in memory): results and the fix-up queue written directly.
hipError_t launch_pairs_small(int op, const PairArgs& a, hipStream_t st);
// FP64 acceleration / gradient, the same limits: sources read from the masters, no pack, the pass
// statistics cleared by the kernel (one launch)
hipError_t launch_pairs_small64(int op, const PairArgs& a, hipStream_t st);
hipError_t launch_zero_count(int32_t* c, hipStream_t st);
hipError_t launch_zero_u64(unsigned long long* c, int n, hipStream_t st);
// one kernel: zero the fix-up counter (if not NULL) and the three pass statistics
hipError_t launch_pass_begin(int32_t* fix_count, unsigned long long* stats, hipStream_t st);
// A captured graph and the scratch buffers it owns (freed with it).
struct bf_graph {
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    void* owned[12] = {};
};

// FP64 fix-up of queued targets; part: 3 * cap doubles of scratch (cap >= kFixTiled; the
// context's buffer holds cap = kFixChunks * kFixTiled).
constexpr int kFixTiled = 32768, kFixChunks = 64;
// source-chunk partials: more chunks than this are added by one wavefront per target
constexpr int kReduceWaveSplit = 16;
hipError_t launch_fixup(int op, const PairArgs& a, double* part, int cap, int num_cu, hipStream_t st);

// Spatially sorted mixed acc/grad (spatial.hip).
struct SortBuffers {
    uint32_t* bbox;      // 6 ordered-uint words: min x, y, z then max x, y, z
    uint32_t* keys_in;   // [n]
    uint32_t* keys_out;  // [n]
    int32_t* vals_in;    // [n]
    int32_t* vals_out;   // [n]
    void* tmp;           // sort temporary storage
    size_t tmp_bytes;
};
// bytes of sort temporary storage for n keys
size_t sort_tmp_bytes(int n);
// sort the particles of `set` along a Morton curve over the box of `box_set`; writes the sorted
// particle list to out[0..set.count).  graph_safe: a sort made of kernel launches only (for
// graph capture); the same order.
hipError_t launch_sort_set(const Masters& P, const DevSet& set, const DevSet& box_set, const SortBuffers& sb,
                           int32_t* out, uint32_t* flags, hipStream_t st, bool graph_safe = false);
// pack sorted sources into tiles of 64*waves: near (FP64) stream, far (FP32 tile-relative)
// stream and tile metadata
hipError_t launch_pack_tiles(int op, int waves, const PairArgs& a, void* near_pack, void* far_pack,
                             double4* meta, hipStream_t st);
// launch the spatially sorted pair kernel
hipError_t launch_pairs_sorted(int op, const KernelConfig& cfg, const PairArgs& a, int nblocks, hipStream_t st);
bool sorted_variant_exists(int op, int k, int waves);
int sorted_blocks_per_cu(int op, int k, int waves);

// Pair-symmetric sorted sweep (symmetric.hip): targets and sources are one set, sorted and
// packed in tiles of 64; a workgroup owns a block of kSymBlockTiles row tiles (W wavefronts of R
// row tiles each, W R = kSymBlockTiles).
constexpr int kSymBlockTiles = 16;
// Two modes:
//  * one set (between == 0): rows and columns are the same sorted set; each unordered pair once;
//  * two sets (between == 1): rows are set A, columns set B (disjoint); every pair (a, b) once.
struct SymArgs {
    const void* near_pack;     // sorted columns, FP64 (the near stream of launch_pack_tiles)
    const void* far_pack;      // sorted columns, FP32 offsets from their tile's centre
    const double4* tile_meta;  // per column tile: (centre, [half-extent, G tile mass]) [, (a centre, [a half-extent])]
    const void* row_pack;      // sorted rows, FP64, same layout as near_pack (one set: near_pack)
    int32_t n;                 // columns
    int32_t n_tiles;           // ceil(n / 64)
    int32_t n_pad;             // 64 n_tiles: stride of part
    int32_t n_rows, n_row_tiles, n_row_pad;  // rows: count, ceil(count / 64), 64 n_row_tiles (stride of own)
    int32_t n_blocks;          // row blocks: ceil(n_row_tiles / kSymBlockTiles)
    int32_t between;           // 0: one set, 1: two sets
    float eps2f, kappa;
    int32_t n_chunks;          // the column range of a row block is split into n_chunks shares of
    int32_t chunk_len;         // chunk_len block distances (one set) or column tiles (two sets)
    float* part;               // one set: [distances of the pass][4][n_pad] column partials per block
                               // distance (slot d - d_base); two sets: [n_blocks][4][n_pad] per row block
    double* own;               // [shares of the pass][4][n_row_pad] row sums, one row per share
    // One set: the shares run in passes whose partials fit the scratch limit.  This pass covers
    // shares [chunk0, chunk0 + pass_chunks), distances from d_base = chunk0 chunk_len; acc holds
    // the running per-particle sums between passes (NULL for a single pass); first / last: this
    // is the first / last pass.  Two sets: chunk0 = d_base = 0, one pass.
    int32_t chunk0, pass_chunks, d_base;
    int32_t first, last;
    double* acc;
    unsigned long long* tile_stats;  // [near, far] wavefront-tile visits (NULL: not counted)
    // time-step sweep only: the masses and G of the FP64 re-evaluation, the device flags
    // (coincident pairs), the FP64 maxima of re-evaluated tiles [2][n_pad]
    const double* m;
    double G;
    uint32_t* flags;
    double* hi;
};
// bytes of own (256-byte aligned) for n rows and `chunks` shares (two sets)
size_t sym_own_bytes(int64_t n, int chunks);
// the same for rows of n_rows particles against columns of n_cols (two sets)
size_t between_scratch_bytes(int64_t n_rows, int64_t n_cols, int chunks);
// adds the row sums (rows: a_rows.tgt, sorted) and the column partials (columns: a_cols.tgt) in a
// fixed order, writes both sets' particle-indexed outputs and queues ill-conditioned targets
hipError_t launch_between_reduce(int op, const PairArgs& a_rows, const PairArgs& a_cols, const SymArgs& g,
                                 hipStream_t st);
// FP64 one-set sweep: the set in its own order, FP64 pack (launch_pack, FP64) as columns and
// rows, FP64 row sums [shares][3][n_pad] and partials [distances][3][n_pad] (part holds
// doubles), no fix-up
int sym64_blocks_per_cu(int op);
hipError_t launch_pairs_sym64(int op, const SymArgs& g, double eps2t, hipStream_t st);
hipError_t launch_sym_reduce64(int op, const PairArgs& a, const SymArgs& g, hipStream_t st);
// mixed time-step one-set sweep: the time-step pack (launch_pack, mixed) in the set's own order as
// columns and rows, FP32 row maxima [shares][2][n_pad] (own and acc hold floats), FP64 maxima
// of the tiles evaluated again in FP64 (hi) and FP32 partials [distances][2][n_pad]; launched by
// launch_pairs_sym / launch_sym_reduce with op OP_DT
// resident workgroups per CU of the symmetric kernel of op with a given shape, the default
// shape, and the launch
// shapes: W wavefronts of R row tiles each (W R = kSymBlockTiles): (16, 1), (8, 2), (4, 4);
// op OP_ACC, OP_GRAD (sorted, mixed) or OP_DT (set order, mixed)
int sym_default_waves(int op);
int sym_default_rows(int op);
bool sym_variant_exists(int op, int waves, int rows);
int sym_blocks_per_cu(int op, int waves, int rows);
hipError_t launch_pairs_sym(int op, int waves, int rows, const SymArgs& g, hipStream_t st);
// adds the row-side sums and the partials in a fixed order and writes the particle-indexed
// outputs of a.tgt (the sorted list), queueing ill-conditioned targets for the fix-up
hipError_t launch_sym_reduce(int op, const PairArgs& a, const SymArgs& g, hipStream_t st);

// time-step assignment epilogue (timestep.hip)
struct TimestepArgs {
    Masters P;
    DevSet set;
    const double *dt_ff, *dt_fb;            // pairwise criteria (particle-indexed)
    const double *ax, *ay, *az;             // accelerations
    const double *gx, *gy, *gz;             // force-gradient sums (NULL: no gradient criteria)
    const double *jx, *jy, *jz;             // jerks (NULL: no jerk criterion)
    double eta_grad, eta_jerk, tau;
    int kmax;
    double* dt;                             // out: time-step
    int32_t* level;                         // out: level (NULL: not assigned)
    uint32_t* flags;
};
hipError_t launch_timestep(const TimestepArgs& t, hipStream_t st);
// Subsystem neighbour search (ngb.hip).
struct NgbArgs {
    Masters P;
    DevSet tgt, src;
    double G, r_ngb, r_max2, C, tau;
    int32_t split, chunk;         // source chunks per target slab, sources per chunk
    unsigned long long* keys;     // [cap] found pairs (i << 32 | j), unordered
    int64_t cap;
    unsigned long long* count;    // pairs found (may exceed cap)
    uint32_t* flags;
};
// targets per thread of the neighbour kernel (a workgroup of 64 waves threads takes 64 waves kNgbK)
constexpr int kNgbK = 2;
hipError_t launch_ngb(const NgbArgs& a, int waves, int nblocks, hipStream_t st);
size_t ngb_sort_tmp_bytes(int64_t m);
hipError_t launch_ngb_finish(unsigned long long* keys_in, unsigned long long* keys_out, int64_t m, void* tmp,
                             size_t tmp_bytes, int32_t* edges, hipStream_t st);
hipError_t launch_label_init(int32_t* label, int64_t n, int32_t* changed, hipStream_t st);
hipError_t launch_label_round(const int32_t* edges, int64_t m, int64_t n, int32_t* label, int32_t* changed,
                              uint32_t* flags, hipStream_t st);
hipError_t launch_label_count(const int32_t* label, int64_t n, int32_t* mark, int32_t* count, hipStream_t st);

size_t level_sort_tmp_bytes(int n);
// Compare the split cur[0..n) (slow part counts[0], on the device) with the previous split
// prev[0..n_prev) (slow part n0_prev): diff[0] = slow parts differ, diff[1] = lists differ.
hipError_t launch_split_diff(const int32_t* cur, int n, const int32_t* counts, const int32_t* prev, int n_prev,
                             int n0_prev, int32_t* diff, hipStream_t st);
// slow (0) / fast (1) flag per particle of a level: time-step min(dt0, dtl) (dtl may be NULL)
// against the pivot tau; all_slow: every particle slow (the deepest level)
hipError_t launch_pivot_flags(const DevSet& set, int64_t n, const double* dt0, const double* dtl, double tau,
                              bool all_slow, int32_t* flag, uint32_t* flags, hipStream_t st);
hipError_t launch_level_partition(const DevSet& set, int64_t n, const int32_t* level, int kmax, uint32_t* keys_in,
                                  uint32_t* keys_out, int32_t* vals_in, int32_t* out_order, int32_t* counts,
                                  void* tmp, size_t tmp_bytes, uint32_t* flags, hipStream_t st);

// Mixed acc / grad: a target is re-evaluated in FP64 when its magnitude estimate M exceeds
// cond_max times the norm of its result.  Acceleration: M = sum w max|r| lies within a factor
// sqrt(3) of the sum of the term norms; threshold 16.  Gradient: M = sum w max|a_ji| falls
// short of the sum of the term norms by up to a factor 2 sqrt(3) (|term| <= 2 w |a_ji|), and
// the two partial sums S1 = sum w a_ji and S2 = sum w (a_ji . r) r / s^2 are carried
// separately; threshold 8.
constexpr double kCondMax = 16.0;
constexpr double kCondMaxGrad = 8.0;
inline double cond_max_for(int op) { return op == OP_GRAD ? kCondMaxGrad : kCondMax; }

// PN1.0
struct PnArgs {
    Masters P;
    DevSet tgt, src;
    const int32_t* bh;
    int32_t nbh;
    double G, c2inv;
    double* part;        // [nbh][nchunk][4] partial sums of BH targets over all sources, BH-is-source record
    int32_t nchunk, chunk;
    int32_t* bh_in_src;  // [nbh] 1 if bh[k] is a source (lists of more than 4096 BHs)
    double *o0, *o1, *o2;
    uint32_t* flags;
};
hipError_t launch_pn1(const PnArgs& a, hipStream_t st);

// energy
struct EnergyArgs {
    Masters P;
    DevSet set;
    double G, eps2;
    double* rows;   // [energy_partials(count)] potential partials of the pair workgroups
    double* kin;    // [count] per-particle kinetic terms
    double* out;    // [2] final kinetic, potential
    double4* pack;  // [count] (x, y, z, m) of the set, in set order
};
// number of pair workgroups (and potential partials) of the energy of a set of n
int energy_partials(int n);
hipError_t launch_energy(const EnergyArgs& a, hipStream_t st);

// elementwise updates
hipError_t launch_kick(const bf_state& S, const DevSet& set, double h, const double* ax, const double* ay,
                       const double* az, double h2, const double* gx, const double* gy, const double* gz,
                       uint32_t* flags, hipStream_t st);
// launch_kick followed by x += hd v over the same set, in one launch
hipError_t launch_kick_drift(const bf_state& S, const DevSet& set, double h, const double* ax, const double* ay,
                             const double* az, double h2, const double* gx, const double* gy, const double* gz,
                             double hd, uint32_t* flags, hipStream_t st);
hipError_t launch_drift(const bf_state& S, const DevSet& set, double h, uint32_t* flags, hipStream_t st);
hipError_t launch_validate(const DevSet& set, int64_t n, uint32_t* flags, hipStream_t st);

}  // namespace bf

// ---- the context -------------------------------------------------------------------------

struct bf_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    int num_cu = 0;
    uint32_t* d_flags = nullptr;      // device flag word
    uint32_t* h_flags = nullptr;      // pinned host mirror
    void* scratch = nullptr;          // general scratch (partials, packs)
    size_t scratch_bytes = 0;
    void* scratch2 = nullptr;         // second scratch (packed sources)
    size_t scratch2_bytes = 0;
    void* scratch3 = nullptr;         // third scratch (intermediate gradient / a arrays)
    size_t scratch3_bytes = 0;
    void* scratch4 = nullptr;         // batched partials, work-item offsets, queue counter
    size_t scratch4_bytes = 0;
    void* scratch5 = nullptr;         // spatial sort: box, keys, values, sorted lists, sort temporaries
    size_t scratch5_bytes = 0;
    void* scratch6 = nullptr;         // spatial sort: far (FP32 tile-relative) stream and tile metadata
    size_t scratch6_bytes = 0;
    void* scratch7 = nullptr;         // HHS driver: level order and inter-level / FSI arrays
    size_t scratch7_bytes = 0;
    void* scratch8 = nullptr;         // FP64 fix-up partial sums
    size_t scratch8_bytes = 0;
    void* scratch9 = nullptr;         // pair-symmetric sweep: row sums and column partials
    size_t scratch9_bytes = 0;
    void* scratch10 = nullptr;        // two-set symmetric sweep: FP64 stream of the row set
    size_t scratch10_bytes = 0;
    void* scratch11 = nullptr;        // HHS driver: inter-level accelerations kept per level
    size_t scratch11_bytes = 0;
    bool capturing = false;           // a graph capture is recording this context's work
    bool dry = false;                 // size scratch only, launch nothing (before a capture)
    unsigned long long* d_stats = nullptr;  // [fix-ups, near tiles, far tiles] of the last pass, [4]: HHS
                                            // black-hole level mask
    int last_kind = 0, last_k = 0, last_waves = 0, last_split = 0;  // how the last pass ran
    int last_passes = 1;     // sweeps of the last pair-symmetric pass (its shares in passes)
    size_t sym_limit = 0;    // scratch limit of a pair-symmetric pass (0: the default)
    // spatially sorted mixed passes: bit op set = use them for that operation when large enough
    int sort_ops = (1 << 0) | (1 << 1) | (1 << 2);  // acceleration, force-gradient and time-step passes
    const int32_t* sub = nullptr;     // subsystem labels applied to acc / grad / dt passes (NULL: none)
    int64_t sub_n = 0;
    float kappa = 1.0f;               // a tile is near a workgroup when their gap < kappa * tile half-extent
    bool hhs_reuse = true;            // HHS drivers keep accelerations between visits of a level
    int64_t pair_credit[bf::OP_COUNT] = {};  // pair interactions credited by the passes of each op
    // kernel timing: event pairs around pair-kernel launches, per op
    bool timing = false;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> tev[bf::OP_COUNT];
    std::vector<std::pair<hipEvent_t, hipEvent_t>> tpool;
    // (op, prec) -> forced configuration
    bf::KernelConfig forced[bf::OP_COUNT][2];
    // (op, prec, log2 bucket nt, log2 bucket ns) -> tuned configuration
    // (op, prec, sweep kind, log2 bucket nt, log2 bucket ns) -> tuned configuration; sweep kinds:
    // kTuneDirected (k per lane, waves, split), kTuneSymmetric (row tiles per wavefront, waves,
    // rounds of resident workgroups), kTuneBatched (k per lane, waves, sources per work item;
    // buckets of the active total and the largest cluster)
    std::map<std::tuple<int, int, int, int, int>, bf::KernelConfig> tuned;
    bf::KernelConfig sym_forced[bf::OP_COUNT];    // forced symmetric shape (k = 0: none)
    bf::KernelConfig batch_forced[bf::OP_COUNT];  // forced batched shape (k = 0: none)
};
