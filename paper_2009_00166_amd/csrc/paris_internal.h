// Internal declarations shared by the kernel and host translation units of libparis.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

namespace paris {

constexpr int kSeg = 16;           // w, segments per iSAX word
constexpr int kSym = 256;          // 8-bit symbols
constexpr int kMaxLength = 2048;   // longest series the summarise kernel stages in LDS
constexpr int kSeedChunk = 512;    // sorted positions per seed block: its smallest bound is refined
constexpr int kSeedBatchChunks = 32;  // seed chunks per block of the batched seed
constexpr int kSeedGroup = 4;         // batched seed: chunks whose positions are loaded together
constexpr int kTimingEvery = 8;       // timing mode 3: the scan of every 8th query is timed
constexpr int kResolveList = 256;  // in-band candidates resolved block-cooperatively
constexpr int kRefineBlocks = 512; // default refine grid (16 lane groups of 16 lanes per block)
constexpr int kRefineMinBlocks = 128;  // refine blocks taking part with few survivors
constexpr int kRefinePerBlock = 512;   // survivors per taking-part refine block
constexpr int kRefineBatch = 4;    // refine: survivors a lane group takes at once
constexpr int kRefineVec = 4;      // float4 per lane per refine chunk (a 1 KiB piece of a row per group)

// Best-so-far key: float32 bits of the squared distance (non-negative, so the bit pattern
// orders like the value) in the high word, series index in the low word. atomicMin on it keeps
// the smallest distance and, among equal float32 distances, the lowest index.
constexpr unsigned long long kBsfInit = (0x7F800000ull << 32) | 0xFFFFFFFFull;  // (+inf, max)

enum ErrBits : uint32_t {
    kErrNonFinite = 1u,      // NaN or Inf in the data or the query
    kErrSurvOverflow = 2u,   // more LB survivors than capacity
    kErrDoneOverflow = 4u,   // more completed candidates than capacity
};

constexpr int kKnnMax = 64;          // largest k of the exact k-NN
constexpr int kKnnResolve = 2048;    // k-NN: completed candidates re-scored in float64 at most
constexpr int kKnnWindow = 16384;    // k-NN: sorted positions of the approximate search's window
constexpr int kKnnSeedCap = 4096;    // k-NN: seed distances kept for the selection of the k best

// One answer of the exact k-NN: series index and float64 squared distance.
struct KnnHit {
    long long idx;
    double d2;
};

// Result of one query, written by the last kernel of the query.
struct QResult {
    long long idx;            // -1 if none (non-finite query)
    double d2;                // float64 squared distance
    unsigned long long seed_key;
    long long win_lo, win_hi;
    uint32_t n_surv, n_refined, n_abandon, n_bsf_upd, n_resolved, err;
    uint32_t n_read;          // series whose 8-bit words the scan read (runs it did not prune)
};

// Per-query device state. The last kernel of every query snapshots the result and leaves the
// working fields reset for the next query (so no kernel has to clear them before the seed's
// atomics); the build initialises them.
struct alignas(256) QState {
    // summaries of the current query (written by block 0 of the prepare kernel)
    double paa[kSeg];
    uint8_t sym[kSeg];
    uint32_t root;
    uint32_t pad0;
    unsigned long long k64;
    long long win_lo, win_hi;
    // working fields (reset after every query)
    unsigned long long seed_key;
    unsigned long long head_key;   // (fine bound bits, index) of the survivor with the smallest bound
    uint32_t n_surv, n_refined, n_abandon, n_bsf_upd, n_done, n_read;
    uint32_t err;
    uint32_t blocks_done;
    uint32_t pad1;
    // the best-so-far on a line of its own: the seed's and refine's atomics and the refine's
    // re-reads of it do not queue behind the counters' atomics on one memory channel line
    alignas(128) unsigned long long bsf_key;
    QResult res;
};

// Pruning margins, derived on the host from the series length (see margins_for_length).
struct Margins {
    double prune_rel;   // prune / abandon only when value > bsf * (1 + prune_rel)
    double band_rel;    // float64 resolve of every candidate with d32 <= best32 * (1 + band_rel)
};

// ---- build kernels ----
hipError_t launch_summarise(const float* X, long long N, int n, uint8_t* sax, unsigned long long* keys,
                            uint32_t* perm, uint32_t* err, hipStream_t st);
size_t sort_hist_words(long long N);
hipError_t launch_sort_keys(unsigned long long* keys, uint32_t* perm, unsigned long long* keys_alt,
                            uint32_t* perm_alt, uint32_t* hist, long long N, hipStream_t st);
hipError_t launch_root_offsets(const unsigned long long* keys, long long N, uint32_t* roff,
                               hipStream_t st);
hipError_t launch_gather_sax(const uint8_t* sax, const uint32_t* perm, long long N, uint8_t* saxs, hipStream_t st);

// ---- ADS+ tree (leaf mode 2) ----
constexpr int kRoots = 65536;       // root subtrees: node r is root key r
constexpr int kTreeChunk = 4096;    // positions per work item of a tree-building round
constexpr int kTreeMaxDepth = 112;  // 16 segments x 7 extra bits: splits along any path

// A node of the tree (32 bytes): its range of the leaf order, its children (child0 and
// child0 + 1, the bit-0 and bit-1 children; -1 for a leaf), the segment its split refines and
// the bits it fixes per segment.
struct AdsNode {
    uint32_t start, end;
    int32_t child0;
    int32_t split;
    uint8_t card[kSeg];
};
static_assert(sizeof(AdsNode) == 32, "tree nodes are 32 bytes");

struct TreeChunk {
    uint32_t slot;          // index of its node in the round's list
    uint32_t start, end;    // positions of the leaf order
    uint32_t pad;
};

// One round of the tree build: the nodes that split (ascending ids), their chunks, the scratch.
struct TreeRound {
    AdsNode* nodes;
    const int32_t* todo;          // [n_todo] node ids
    const uint32_t* todo_chunks;  // [n_todo + 1] first chunk of every node
    int32_t* todo_split;          // [n_todo] chosen segment
    int n_todo;
    int next;                     // id of the first child created in this round
    const TreeChunk* chunks;
    uint32_t* chunk_ones;         // [chunks][16] series whose next bit is 1
    uint2* chunk_dst;             // [chunks] first destination of a zero / of a one
    const uint8_t* sax;
    uint32_t* perm;
    uint32_t* perm_tmp;
};

hipError_t launch_tree_roots(const uint32_t* roff, AdsNode* nodes, hipStream_t st);
hipError_t launch_tree_round(const TreeRound& r, int n_chunks, hipStream_t st);
hipError_t launch_tree_keys(const uint8_t* sax, const uint32_t* perm, long long N, unsigned long long* keys,
                            hipStream_t st);

// ---- query kernels ----
struct QueryArgs {
    const float* X;
    long long N;
    int n;
    const uint8_t* sax;
    const uint8_t* saxs;          // the same words in leaf order (saxs[p] = sax[perm[p]])
    const uint8_t* env;           // [ceil(N / 32)][32] symbol envelope of every run of 32
                                  // leaf-order positions: the smallest symbol of each segment,
                                  // then the largest
    const unsigned long long* keys;
    const uint32_t* perm;
    const uint32_t* roff;
    int leaf_mode, n_leaves, seed_cap;
    QState* qs;
    float* t8;        // [16][256]
    uint2* surv;      // (index, lb2 bits)
    uint32_t surv_cap;
    uint2* done;      // (index, d2 fp32 bits)
    uint32_t done_cap;
    Margins mg;
    QResult* host_res;  // pinned host memory mapped for the device (may be null): the result is
                        // also stored there, so the host needs no copy after synchronising
    const unsigned long long* leaf_keys;  // learned seed, per-query path: best (logit, leaf) keys
    int leaf_key_count;                   // of the network's blocks, merged by the seed kernel
    int learned_cpl;        // > 0: learned seed over kTopLeaves leaves of up to this many chunks
    int refine_blocks;      // refine grid (0: kRefineBlocks)
    int refine_lanes;       // lanes per refined row: 4, 8 (default) or 16
    int bsf_private;        // 1: every lane group prunes with its own best-so-far copy only
    // exact k-NN (knn_k > 0): the best-so-far key of QState is the k-th best key found so far,
    // the k best keys live in knn_slots, and the seed refines knn_r * knn_k smallest-bound
    // members of the approximate search's window (spread evenly over its chunks)
    int knn_k;
    int knn_r;
    unsigned long long* knn_slots;  // [kKnnMax] (float32 bits of ED^2, index) keys
    unsigned long long* knn_seed;   // [kKnnSeedCap] the seed blocks' keys (slot = block r + t)
    KnnHit* knn_out;                // [kKnnMax] answers of the last block (mapped host memory)
    // leaf mode 2 (ADS+ tree): the nodes, and the largest window the approximate search reaches
    const AdsNode* tree;
    int tree_window;
};

// ---- batched path ----
constexpr int kBandCap = 4;        // float64-resolve candidates kept per query in a batch

// Per-query state of a batch (64 bytes).
struct alignas(64) BQuery {
    unsigned long long bsf_key;    // (float32 bits of ED^2, index), atomicMin
    float qn;                      // float32 squared norm of the query
    float a;                       // screen threshold constant (see k_screen)
    uint32_t n_band;               // entries appended to band[] (may exceed kBandCap)
    uint32_t err;                  // kErrNonFinite
    uint32_t ub;                   // float32 bits: the screen's largest survivor accumulator
                                   // (atomicMax), then the certified upper bound on the nearest
                                   // squared distance derived from it (+inf: none)
    float u_lo;                    // the screen's threshold U_q, rounded down
    uint2 band[kBandCap];          // (index, ED^2 float32 bits) within the resolve band
};

// Batch-mode arguments of the prepare+seed kernel (bq == nullptr: the plain path).
struct SeedBatch {
    const float* Q;       // [M][n] float32 queries
    BQuery* bq;           // [M]
    uint16_t* qb;         // [M][np] bfloat16 copies, zero padded
    int np;               // screened dimensions (n / P) rounded up to a multiple of 32
    int P;                // segment length of the screen's projection (1: the series itself)
    const int32_t* leaves;  // learned seed: [M][kTopLeaves] leaf ids (used when learned_cpl > 0)
    double* qpaa;         // [M][16] float64 PAA of every query (for the screen's block bound)
    int chunks;           // seed chunks of a query's window(s) (set by the launcher)
};

struct BatchHdr {
    uint32_t next_item;    // screen work counter (series work items)
    uint32_t n_cand;       // screen candidates appended (may exceed the capacity)
    uint32_t n_fallback;   // queries handed back to the per-query path
    uint32_t flags;
    uint32_t n_tiles;      // query tiles the screen ran (summed over its work items)
    uint32_t n_rescored;   // candidates the re-score read rows for (the others were skipped)
    uint32_t xn_max;       // float32 bits: largest series squared norm (set at attach, kept)
    uint32_t pad;
};

constexpr int kEnvRun = 32;          // sorted positions per stored symbol envelope
constexpr int kScreenGroup = 4096;   // queries per alive list of the screen
constexpr int kAmaxQueries = 4096;   // batch size up to which the screen gathers survivor maxima

struct ScreenArgs {
    const uint16_t* Xb;    // [N][np] bfloat16 collection
    const float* xn;       // [N] float32 squared norms
    long long N;
    const uint16_t* Qb;    // [M][np] bfloat16 queries
    BQuery* bq;
    uint16_t* qbias;       // [M][16] bfloat16 bias row of every query (written by launch_screen)
    int M;
    uint2* cand;           // (query, series)
    float* cand_d2;        // per candidate: the screen's accumulator, truncated (re-score input)
    uint32_t cand_cap;
    BatchHdr* hdr;
    float c_screen;        // relative margin c of E = c (qn + xn)
    float* dump;           // optional [M][N] float32 dot products (tests)
    const uint32_t* perm;  // [N] series at each sorted position (Xb and xn are in leaf order)
    // block bound (nullptr mask: every pair is screened)
    unsigned long long* mask;  // [items][ceil(M / 64)] alive bits, written by k_block_mask
    const uint8_t* env;    // [ceil(N / kEnvRun)][32] symbol envelopes (min[16], max[16])
    const double* qpaa;    // [M][16] float64 query PAA
    double seg_len;        // L = n / 16
    double seed_rel, prune_rel;
};

struct RescoreArgs {
    const float* X;
    const float* Q;        // [M][n] float32 queries
    int n, M;
    BQuery* bq;
    const uint2* cand;
    float* cand_d2;        // float32 squared distance of each candidate (+inf: abandoned)
    uint32_t cand_cap;
    BatchHdr* hdr;
    double prune_rel, band_rel;
    uint32_t* fallback;    // [M] queries to answer on the per-query path
    int ub_on;             // skip candidates whose screened lower bound exceeds the query's ub
    float c_screen;        // the screen's relative margin (for the candidates' upper bounds)
    double seed_rel;
    int lb_on;             // cand_d2 holds screen accumulators: head pass + lower-bound pre-check
    int P;                 // segment length of the screen's projection (1: the series itself)
};

struct ScreenShape {
    int qt;     // queries per LDS tile: 32 or 64
    int grid;   // persistent blocks
    int subs;   // series subtiles per wave held in registers (16 wide: 2 or 4; 32 wide: 1 or 2)
    int mfma;   // 16: v_mfma_f32_16x16x32_bf16; 32: v_mfma_f32_32x32x16_bf16
};

hipError_t launch_to_bf16(const float* X, const uint32_t* perm, long long N, int n, int np, int P, uint16_t* Xb,
                          float* xn, hipStream_t st);
hipError_t launch_block_env(const uint8_t* saxs, long long N, uint8_t* env, hipStream_t st);
int screen_item_series(ScreenShape shape);
hipError_t launch_batch_init(BQuery* bq, int M, BatchHdr* hdr, hipStream_t st);
hipError_t launch_batch_thresholds(BQuery* bq, int M, float c_screen, double seed_rel, int P, hipStream_t st);
hipError_t launch_set_bsf(BQuery* bq, const float* sqdist, int M, hipStream_t st);
hipError_t launch_xn_max(const float* xn, long long N, BatchHdr* hdr, hipStream_t st);
// alive bits of the block bound (no launch when the shape or arguments do not use them)
hipError_t launch_block_mask(const ScreenArgs& s, ScreenShape shape, hipStream_t st);
hipError_t launch_screen(const ScreenArgs& s, int np, ScreenShape shape, hipStream_t st);
hipError_t launch_rescore(const RescoreArgs& r, hipStream_t st);
hipError_t launch_batch_resolve(const RescoreArgs& r, long long* out_idx, double* out_dist, hipStream_t st);

// ---- learned seed ----
constexpr int kMlpIn = 16;          // PAA features
constexpr int kMlpHid = 256;        // hidden width
constexpr int kTopLeaves = 8;       // leaves visited by the learned seed
constexpr int kMaxLeaves = 65536;   // largest leaf count the network can score

// Offsets (in elements) of the packed parameter vector [W1 (256x16), b1, W2 (256x256), b2,
// W3 (n_out x 256), b3], rows indexed by output unit.
struct MlpOffsets {
    long long w1, b1, w2, b2, w3, b3, total;
};

inline MlpOffsets mlp_offsets(int n_out)
{
    MlpOffsets o;
    o.w1 = 0;
    o.b1 = o.w1 + (long long)kMlpHid * kMlpIn;
    o.w2 = o.b1 + kMlpHid;
    o.b2 = o.w2 + (long long)kMlpHid * kMlpHid;
    o.w3 = o.b2 + kMlpHid;
    o.b3 = o.w3 + (long long)n_out * kMlpHid;
    o.total = o.b3 + n_out;
    return o;
}

struct MlpNet {
    const float* master;    // float32 parameters (biases are read from here)
    const uint16_t* wb;     // bfloat16 mirror of the same vector (weights are read from here)
    int n_out;
    MlpOffsets off;
};

struct MlpQueryScratch {
    unsigned long long* part;  // [blocks][kTopLeaves] every block's best (logit, leaf) keys
};

// (logit, leaf) order key of the top-leaf selections: float bits mapped to an unsigned order
// (NaN lowest), leaf id complemented so that among equal logits the lower id has the larger key.
__device__ __forceinline__ unsigned long long top_key(float v, uint32_t c)
{
    uint32_t u = __float_as_uint(v);
    u = (u >> 31) ? ~u : (u | 0x80000000u);
    if (v != v) u = 0u;
    return ((unsigned long long)u << 32) | (uint32_t)(~c);
}

enum GemmEpilogue { kEpiBiasReluBf16 = 0, kEpiBiasF32 = 1, kEpiMask = 2, kEpiF32 = 3 };

struct GemmArgs {
    const uint16_t* A;
    long long lda;
    const uint16_t* B;
    long long ldb;
    int M, N, K;
    const float* bias;      // kEpiBiasReluBf16, kEpiBiasF32: [N]
    const uint16_t* mask;   // kEpiMask: bfloat16 activation [M][ldm]; zero entries zero the output
    long long ldm;
    float* Cf;              // float32 output (kEpiBiasF32, kEpiMask, kEpiF32)
    uint16_t* Cb;           // bfloat16 output (kEpiBiasReluBf16, kEpiMask)
    long long ldc;
};

struct AdamArgs {
    float lr, beta1, beta2, eps;
    float bc1, bc2;         // 1 - beta1^t, 1 - beta2^t
};

hipError_t launch_paa_features(const float* Q, long long M, long long Mpad, int n, float* P, hipStream_t st);
hipError_t launch_l1_fwd(const MlpNet& net, const float* P, const int32_t* sel, int rows_real, int rows_pad,
                         uint16_t* H1, hipStream_t st);
hipError_t launch_l1_bwd(const float* G1, const float* P, const int32_t* sel, int rows_real, float* dW1,
                         hipStream_t st);
hipError_t launch_gemm(const GemmArgs& g, int ta, int tb, int epi, hipStream_t st);
hipError_t launch_softmax_ce(const float* Z, int n_out, const int32_t* y, const int32_t* sel, int rows_real,
                             int rows_pad, float* G, uint16_t* Gb, float* loss_row, hipStream_t st);
hipError_t launch_colsum(const float* G, int rows, int cols, float* out, hipStream_t st);
hipError_t launch_mean_loss(const float* loss_row, int rows, float* out, hipStream_t st);
hipError_t launch_adam(float* p, const float* g, float* m, float* v, uint16_t* wb, long long count,
                       const AdamArgs& a, hipStream_t st);
hipError_t launch_mirror(const float* p, uint16_t* wb, long long count, hipStream_t st);
hipError_t launch_topk(const float* Z, int rows, int n_out, int k, int32_t* out, hipStream_t st);
hipError_t launch_mlp_query(const MlpNet& net, const float* q, int n, const MlpQueryScratch& s, hipStream_t st);
hipError_t launch_leaf_of(const uint8_t* sax, const unsigned long long* keys, const uint32_t* perm, long long N,
                          int n_leaves, const long long* idx, long long count, int32_t* out, hipStream_t st);

// Launch shape of the lower-bound scan (chosen by the autotuner on first use).
struct ScanShape {
    int threads;   // 256 or 512
    int per_cu;    // blocks per compute unit
    int unroll;    // run envelopes per thread in flight: 1, 2 or 4
};

hipError_t launch_reset(const QueryArgs& a, hipStream_t st);
hipError_t launch_scan_again(const QueryArgs& a, hipStream_t st);
hipError_t launch_touch(const void* p, size_t bytes, uint32_t* sink, hipStream_t st);
// query summaries, tables, window, and the lower-bound-guided approximate-search seed
hipError_t launch_prepare_seed(const QueryArgs& a, const float* q, hipStream_t st);
hipError_t launch_prepare_seed_batch(const QueryArgs& a, const SeedBatch& b, int n_queries, hipStream_t st);
// threshold_sq < 0: use the best-so-far in QState; otherwise a fixed threshold.
// ev_start / ev_stop (optional): HIP events bound to the scan kernel's own dispatch, so that
// their elapsed time is the kernel's start-to-end duration without the gaps around it.
hipError_t launch_lbscan(const QueryArgs& a, float threshold_sq, ScanShape shape, hipStream_t st,
                         hipEvent_t ev_start = nullptr, hipEvent_t ev_stop = nullptr);
// refinement; its last block resolves in float64, writes the result (and element qi of
// out_idx / out_dist when they are not null) and resets the state for the next query.
hipError_t launch_refine_resolve(const QueryArgs& a, const float* q, long long* out_idx, double* out_dist,
                                 long long qi, hipStream_t st);
int seed_grid(const QueryArgs& a);
// exact k-NN: the k best slots set to (+inf, no index) and the state's k-th key to +inf
hipError_t launch_knn_reset(const QueryArgs& a, hipStream_t st);
// the k smallest seed keys into the slots, the k-th of them as the best-so-far
hipError_t launch_knn_select(const QueryArgs& a, hipStream_t st);

}  // namespace paris
