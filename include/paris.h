/*
 * paris.h — C ABI of the MI355X exact 1-NN search over iSAX summaries (ParIS+, arXiv 2009.00166).
 *
 * Problem (Section 2.1, "Similarity Search"): given a query series of length n and a collection
 * of series of the same length, return the series of the collection with the smallest Euclidean
 * distance to the query. Ties go to the lowest series index. The paper's ExactSearch returns
 * only the best-so-far distance (Section 3.3.3); these calls return the index and the distance.
 *
 * Method: every series is summarised once (paris_build) into a 16-segment, 8-bit iSAX word
 * (Section 2.2: PAA segment means quantised against 255 Gaussian boundaries); the words are also
 * kept in leaf order with the symbol envelope (per-segment smallest and largest symbol) of every
 * run of 32 consecutive positions. A query (paris_query_exact) takes an approximate-search seed
 * as its first best-so-far distance (Section 3.3), scans the collection with the iSAX lower bound
 * (every run's bound over its envelope first, then the words of the series of the runs it does
 * not prune) and keeps the series the bound cannot prune (the LBC workers of Section 3.3.3),
 * computes real distances of the
 * survivors with early abandoning while an atomic minimum tightens the best-so-far (the RDC
 * workers), and resolves the final comparison in float64.
 *
 * Conventions for every call:
 *   - Return value: PARIS_OK (0) or a negative paris_status. No exception, abort or exit ever
 *     crosses this boundary.
 *   - "_dev" pointers are device (HBM) addresses on the current HIP device; others are host.
 *   - hip_stream is a hipStream_t passed as void* (NULL = the default stream).
 *   - Argument errors are detected on the host before anything is launched; outputs are then
 *     left untouched.
 *   - Series indices are 0-based positions in the collection array. n_series must be in
 *     [1, 2^32 - 2]; length must be a positive multiple of 16.
 *   - Floating-point data are IEEE float32, row-major [n_series][length], 16-byte aligned.
 *     The library does not z-normalise; it searches the values as given.
 */
#ifndef PARIS_H
#define PARIS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum paris_status {
    PARIS_OK = 0,
    PARIS_EINVAL = -1,     /* bad argument, or NaN/Inf found in the data or the query      */
    PARIS_ENOMEM = -2,     /* workspace smaller than paris_workspace_size()                  */
    PARIS_ENODEV = -3,     /* no usable HIP device                                           */
    PARIS_EHIP = -4,       /* a HIP runtime call failed; the handle must then be freed       */
    PARIS_EOVERFLOW = -5,  /* a device buffer overflowed (cannot happen at default capacity) */
    PARIS_ESTATE = -6      /* invalid or freed handle                                        */
} paris_status;

enum { PARIS_LEAF_ROOT16 = 0, PARIS_LEAF_EQUAL_COUNT = 1, PARIS_LEAF_ADS = 2 };

/* Index configuration. Start from paris_default_config(). */
typedef struct paris_config {
    int32_t segments;   /* w: must be 16 (Section 3 fixes w = 16)                              */
    int32_t card_bits;  /* must be 8: 256 symbols, the maximum cardinality (Section 2.2)        */
    int32_t leaf_mode;  /* PARIS_LEAF_ROOT16: leaves are the root subtrees, i.e. runs of equal
                           first bits of the 16 symbols (Section 3, pipeline overview).
                           PARIS_LEAF_EQUAL_COUNT: n_leaves equal slices of the key order.
                           PARIS_LEAF_ADS: the ADS+ tree (Section 2.2): root subtrees whose
                           leaves split while they hold more than leaf_cap series, each split
                           fixing one more bit of the segment that divides the leaf most evenly
                           (ties: the lowest segment); bulk loaded on the GPU.                 */
    int32_t n_leaves;   /* EQUAL_COUNT only: 1 .. 65536 (default 4096)                          */
    int32_t seed_cap;   /* ROOT16 only: the approximate search examines at most this many
                           members of the query's subtree (default 16384), consecutive in key
                           order and centred on the query's key; in every 512 of them the one
                           with the smallest lower bound gets its real distance computed, and
                           the smallest of those is the first best-so-far. 0 disables the seed:
                           the best-so-far starts at +inf (the answer is unchanged).           */
    int32_t leaf_cap;   /* PARIS_LEAF_ADS only: leaf capacity, 1 .. 2^20 (default 2048; the paper
                           gives none). The approximate search reaches the query's leaf by the
                           query's bits and examines at most seed_cap of its positions.        */
    int32_t reserved[2];
} paris_config;

/* Per-query counters (paris_query_batch sums them over the batch). */
typedef struct paris_stats {
    int64_t lb_survivors;  /* series whose lower bound did not prune them                     */
    int64_t refined;       /* survivors whose distance computation started                   */
    int64_t abandoned;     /* of those, stopped early because the partial sum passed the BSF */
    int64_t bsf_updates;   /* times the atomic best-so-far went down during refinement       */
    int64_t resolved;      /* candidates re-scored in float64 for the final comparison       */
    int64_t seed_index;    /* series found by the approximate search (-1 if none)            */
    double  seed_dist;     /* its float32-computed distance (+inf if none)                   */
    int64_t seed_lo, seed_hi;  /* sorted-position window examined by the approximate search  */
    int64_t words_read;        /* series whose 8-bit words the scan read: the series of the
                                  runs whose envelope bound did not prune them                */
} paris_stats;

typedef struct paris_index paris_index;  /* opaque, library-owned host handle */

/* Device-buffer addresses inside a built index's workspace (for inspection and tests). */
typedef struct paris_layout {
    const uint8_t  *sax_dev;    /* uint8  [n_series][16]: iSAX word of series i at row i       */
    const uint64_t *keys_dev;   /* uint64 [n_series]: leaf keys in ascending (key, index) order */
    const uint32_t *perm_dev;   /* uint32 [n_series]: series index at each sorted position      */
    const uint32_t *roff_dev;   /* uint32 [65537]: first sorted position of each root subtree  */
    int64_t n_series;
    int32_t length;
    int32_t leaf_mode, n_leaves, seed_cap;
    int32_t scan_threads, scan_blocks_per_cu, scan_unroll;  /* lower-bound scan launch shape
                                                               picked at build                */
    /* PARIS_LEAF_ADS only (else NULL / 0): the tree's nodes, 32 bytes each: uint32 start, end
       (range of the leaf order), int32 child0 (-1: leaf; the bit-1 child is child0 + 1), int32
       split (segment refined by the split, -1: leaf), uint8 card[16] (bits fixed per segment).
       Nodes 0 .. 65535 are the root subtrees (node r: root key r); every round of the build
       splits the leaves that must split in ascending id, the i-th getting children next + 2i and
       next + 2i + 1 (next: the node count before the round). In this mode perm_dev is the tree's
       leaf order (a stable partition of the key order per split, bit 0 first) and keys_dev[p] is
       the leaf key of series perm_dev[p] (no longer ascending).                                */
    const void *tree_nodes_dev;
    int64_t n_tree_nodes;
    int64_t tree_max_leaf;      /* series in the largest leaf                                   */
    /* distance screen launch shape picked at paris_batch_attach (all 0 without a batch
       workspace): query-tile rows, persistent blocks per CU, series subtiles per wave, MFMA
       form (16: 16x16x32, 32: 32x32x16)                                                      */
    int32_t screen_rows, screen_blocks_per_cu, screen_subtiles, screen_mfma;
} paris_layout;

/* Query summaries as computed on the device (inspection and tests). */
typedef struct paris_query_info {
    double   paa[16];       /* segment means (float64, ascending sum, divided by L)          */
    uint8_t  sym[16];       /* 8-bit iSAX symbols                                            */
    uint32_t root;          /* 16-bit root key: first bit of every symbol, segment 0 = MSB   */
    uint32_t pad;
    uint64_t k64;           /* leaf key: bit planes 7..4 of the symbols, segment 0 first     */
    int64_t  win_lo, win_hi;  /* approximate-search window (sorted positions)                */
} paris_query_info;

/* Fills *cfg with the defaults (16 segments, 8 bits, ROOT16, 4096 leaves, seed_cap 16384). */
paris_status paris_default_config(paris_config *cfg);

/*
 * Tuned launch shapes. paris_build times the scan's candidate shapes and then refines the
 * choice on the first 48 queries; paris_batch_attach times the screen's. When the environment
 * variable PARIS_TUNE_CACHE names a file, both decisions are appended to it (one text line
 * each, keyed by kind, device architecture, series length, floor(log2 n_series) and, for the
 * scan, collection in host memory, for the screen, 2 * max_batch + block bound on), and a
 * later build or attach with a matching line takes that shape without timing anything.
 * PARIS_SCAN_SHAPE / PARIS_SCREEN_SHAPE, when set, override the cache.
 */

/* Bytes of device workspace paris_build needs for this collection shape (host-only call). */
paris_status paris_workspace_size(int64_t n_series, int32_t length, const paris_config *cfg,
                                  size_t *bytes);

/*
 * Summarise the collection and build the leaf order (Section 3.1, IndexBulkLoading: the iSAX
 * word of the series at position p is stored at SAX[p]; root subtrees are the RecBufs). The
 * grouping into subtrees is a stable sort by leaf key instead of locked buffer inserts.
 *   series_dev      float32 [n_series][length], BORROWED: must stay alive and unmodified until
 *                   paris_free. Every value must be finite (else PARIS_EINVAL).
 *   workspace_dev   at least paris_workspace_size() bytes of device memory, 256-byte aligned,
 *                   BORROWED for the life of the handle; the library owns its contents.
 *   out             receives the handle (library-owned host memory; release with paris_free).
 * Synchronous: returns after the build finished on hip_stream (including a short timing of
 * candidate launch shapes for the lower-bound scan).
 */
paris_status paris_build(const float *series_dev, int64_t n_series, int32_t length,
                         const paris_config *cfg, void *workspace_dev, size_t workspace_bytes,
                         void *hip_stream, paris_index **out);

/*
 * Out-of-core collections (the paper's setting of Section 3: the raw data stay outside the memory
 * that holds the index, and only the series the lower bound cannot prune are read). A collection
 * in host memory from paris_host_alloc can be passed to paris_build as series_dev (its device
 * address): the index (iSAX words, leaf order, tree, workspaces, the batched path's bfloat16
 * copy) lives in HBM, while the summarisation, the approximate search, the refinement, the
 * batched re-score and the float64 resolve read the raw series over PCIe. Answers are identical.
 *   paris_host_alloc   pinned host memory of `bytes` (256-byte aligned), mapped for the current
 *                      device: *host_ptr for the host, *dev_ptr for the kernels. PARIS_ENOMEM if
 *                      the allocation fails.
 *   paris_host_free    releases it (after every index built on it is freed).
 */
paris_status paris_host_alloc(size_t bytes, void **host_ptr, void **dev_ptr);
paris_status paris_host_free(void *host_ptr);

/* Addresses and shape of a built index (host-only call). */
paris_status paris_get_layout(const paris_index *idx, paris_layout *out);

/*
 * Exact 1-NN of one query (Section 3.3.3, ExactSearch with its LBC and RDC workers).
 *   query_dev   float32 [length] on the device; must be finite (else PARIS_EINVAL).
 *   nn_index    host out: index of the nearest series (lowest index among exact ties).
 *   nn_dist     host out: its Euclidean distance, from the float64 squared distance
 *               (ascending-order sum of float64 squared differences), correctly rounded sqrt.
 *   stats       optional host out (may be NULL).
 * Synchronous. One call in flight per handle.
 */
paris_status paris_query_exact(paris_index *idx, const float *query_dev, int64_t *nn_index,
                               double *nn_dist, paris_stats *stats, void *hip_stream);

/*
 * Exact k-NN of one query: the k series nearest to the query (the k-NN classification
 * experiment of Section 4 uses the k nearest series), in ascending (distance, index) order;
 * among equal float64 squared distances the lower index comes first.
 *   k           1 .. 64 (else PARIS_EINVAL).
 *   nn_index    host out [k]: indices of the answers; nn_dist host out [k]: their Euclidean
 *               distances (float64 squared distance in the oracle's operation order, correctly
 *               rounded sqrt).
 *   n_found     host out: min(k, n_series) answers written.
 *   stats       optional host out: lb_survivors, refined, abandoned; bsf_updates = times a
 *               completed distance entered the k best; resolved = candidates re-scored in float64.
 * The method is the exact search with the k-th best distance in the role of the best-so-far
 * (Section 3.3.3): the approximate search's window, 16384 sorted positions centred on the query's
 * leaf key (or the learned seed's leaves), gives the first k-th best (8k of its members, the
 * smallest-bound ones of every 512 positions in equal numbers, get their distance; the environment
 * variable PARIS_KNN_SEED = 1 .. 16 sets the 8), the lower-bound scan
 * keeps the series whose bound does not exceed it, the refinement abandons a distance once its
 * partial sum passes it while completed distances replace the largest of the k best, and the last
 * block re-scores in float64 every completed candidate within the rounding band of the final k-th
 * distance. PARIS_EOVERFLOW if more than 2048 candidates fall in that band (only with massive
 * exact ties). k = 1 runs paris_query_exact. Synchronous; one call in flight per handle; uses the
 * learned seed when one is set.
 */
paris_status paris_query_knn(paris_index *idx, const float *query_dev, int32_t k, int64_t *nn_index,
                             double *nn_dist, int32_t *n_found, paris_stats *stats, void *hip_stream);

/*
 * Allocation-free variant of paris_query_exact, for callers that cannot allocate device memory
 * while they run: code under HIP graph capture, tight serving loops, harnesses that forbid
 * allocation. Same arguments, outputs, answer and synchrony as paris_query_exact. The per-query
 * scratch (query state, lower-bound tables, survivor list, completed-candidate list) is taken
 * from one library-held device array of at most 20 MiB per GPU (a static device array of the
 * library's code object, held by each GPU it runs on until the process ends) instead of the
 * index workspace; the call allocates and frees nothing.
 *   Limits: at most PARIS_NOALLOC_MAX_SURVIVORS series may survive the lower-bound scan and at
 *   most PARIS_NOALLOC_MAX_COMPLETED completed distances may fall in the float64 resolve band
 *   (only exact or near ties reach it). A query beyond either returns PARIS_EOVERFLOW with the
 *   outputs untouched (paris_query_exact, whose lists hold n_series entries, answers it). An
 *   index of at most PARIS_NOALLOC_MAX_SURVIVORS series can never exceed the first limit.
 *   The index's device must be the current device (else PARIS_EINVAL).
 *   The array is shared by every index on that GPU and keeps the last call's contents (each call
 *   first resets the state it needs): calls that overlap on one GPU (other streams, other host
 *   threads) race and must be serialised by the caller. Timing (paris_set_timing) is ignored.
 */
#define PARIS_NOALLOC_MAX_SURVIVORS (1u << 21)
#define PARIS_NOALLOC_MAX_COMPLETED (1u << 18)
paris_status paris_query_exact_noalloc(paris_index *idx, const float *query_dev, int64_t *nn_index,
                                       double *nn_dist, paris_stats *stats, void *hip_stream);

/*
 * Exact 1-NN of n_queries queries.
 *   queries_dev   float32 [n_queries][length] on the device, finite.
 *   nn_index_dev  int64 [n_queries] device out;  nn_dist_dev  float64 [n_queries] device out.
 *   stats         optional host out, summed over the batch (may be NULL).
 * With a batch workspace attached (paris_batch_attach), the queries go in chunks of max_batch
 * through the batched pipeline (one HIP graph per chunk): per-query seeds; a block bound that
 * drops every (query, run of 128 or 256 consecutive series in leaf order) pair whose iSAX
 * lower bound (Section 3.3.1) over the run's symbol envelope exceeds the query's seed distance;
 * the bfloat16 MFMA distance screen with a certified margin over the remaining pairs (series
 * longer than 512 points are screened on segment means); float32 re-scoring of its survivors
 * and the float64 resolve; each chunk is synchronised
 * once, and a query whose candidate or resolve buffers overflow is answered by the per-query
 * path. Without one, the queries run one after another through the per-query kernels and the
 * call is asynchronous unless stats is requested. A NaN/Inf query yields index -1 and distance
 * NaN. stats for the batched pipeline: lb_survivors = screen survivors, refined = survivors
 * whose rows the float32 re-score read (the others were skipped: their screened lower bound
 * exceeded a certified upper bound on the query's nearest distance from the other survivors,
 * or the re-score's running threshold after the head pass had scored the survivors with the
 * largest screen accumulators), resolved = queries answered on the per-query fallback path.
 */
paris_status paris_query_batch(paris_index *idx, const float *queries_dev, int64_t n_queries,
                               int64_t *nn_index_dev, double *nn_dist_dev, paris_stats *stats,
                               void *hip_stream);

/*
 * Several collections in one call (batches mixing collections of different lengths): for every
 * c < n_idx, the n_queries[c] queries at queries_dev[c] (float32 [n_queries[c]][length of
 * idx[c]], device, 16-byte aligned) are answered against idx[c] as by paris_query_batch, into
 * nn_index_dev[c] / nn_dist_dev[c] (device, [n_queries[c]]). idx, queries_dev, n_queries,
 * nn_index_dev and nn_dist_dev are host arrays of n_idx entries; the handles must be distinct.
 * Each collection uses its own attached batch workspace, screen shape (tuned per length) and
 * captured graph. stats (host, may be NULL) sums the counters over all collections. Errors as
 * for paris_query_batch; arguments of every collection are checked before any launch.
 */
paris_status paris_query_batch_multi(paris_index *const *idx, int32_t n_idx, const float *const *queries_dev,
                                     const int64_t *n_queries, int64_t *const *nn_index_dev,
                                     double *const *nn_dist_dev, paris_stats *stats, void *hip_stream);

/*
 * Batched pipeline resources (the batched pattern of the paper's worker pools: many queries,
 * one launch). paris_batch_workspace_size gives the bytes for chunks of up to max_batch queries
 * (1 .. 65536): a bfloat16 copy of the collection in leaf order (np = the screened dimensions
 * rounded up to 32; stored in MFMA fragment order, ceil(N / 32) blocks of 32 rows x np), its norms, the query buffers, per-query states, per-query
 * bias rows of the screen (32 bytes each), a candidate list of min(4096 * max_batch, 2^32 - 16) entries (12 bytes each: query, series, float32
 * re-scored distance), per-query learned-seed leaves and PAA and the block bound's alive bits
 * (ceil(N / 128) * ceil(max_batch / 64) words of 8 bytes).
 * paris_batch_attach borrows that device memory (256-byte aligned) for the life of the handle
 * (or until the next attach), converts the collection, times the screen's tile shapes (on a
 * screen of every pair) and captures the pipeline into a HIP graph. Synchronous on hip_stream.
 * The environment variable PARIS_BLOCK_LB=0, read at attach, turns the block bound off.
 */
paris_status paris_batch_workspace_size(const paris_index *idx, int32_t max_batch, size_t *bytes);
paris_status paris_batch_attach(paris_index *idx, void *workspace_dev, size_t workspace_bytes,
                                int32_t max_batch, void *hip_stream);

/*
 * The screen's float32 dot products of bfloat16 query and series rows, for inspection and
 * tests: dots_dev float32 [n_queries][n_series] (device out) receives q~ . x~ as accumulated
 * by the MFMA screen kernel. Needs an attached batch workspace; n_queries <= max_batch.
 */
paris_status paris_screen_dots(paris_index *idx, const float *queries_dev, int32_t n_queries,
                               float *dots_dev, void *hip_stream);

/*
 * Screen work counters of the batched pipeline since the last attach or reset (host outs):
 * tiles_run = query tiles the MFMA screen ran, tiles_dense = tiles a screen of every pair
 * would have run for the same chunks (their ratio is the share of pairs the block bound kept,
 * rounded up to whole tiles). reset != 0 zeroes both after reading. Errors: PARIS_ESTATE
 * (bad handle), PARIS_EINVAL (NULL out).
 */
paris_status paris_batch_screen_tiles(paris_index *idx, int64_t *tiles_run, int64_t *tiles_dense, int32_t reset);

/*
 * The block bound's alive bits for given thresholds (inspection and tests; the Section 3.3.1
 * lower bound taken over the symbol envelope of a run of item_series consecutive sorted
 * positions, 128 or 256):
 *   queries_dev  float32 [n_queries][length] on the device, 16-byte aligned;
 *   sqdist_dev   float32 [n_queries] on the device: U_q, each query's threshold as a squared
 *                distance (it takes the place of the seed's distance);
 *   bits_dev     uint64 [ceil(N / item_series)][ceil(n_queries / 64)] device out: bit q % 64 of
 *                word (run, q / 64) is set iff the run's bound, in float64, is at most
 *                U_q (1 + seed margin)(1 + prune margin) (both margins below 1e-4 relative);
 *                non-finite queries have no bits.
 * Needs an attached batch workspace (n_queries <= max_batch); overwrites its query buffers.
 * Synchronous. Errors: PARIS_ESTATE (bad handle, no workspace), PARIS_EINVAL (arguments).
 */
paris_status paris_block_bound_bits(paris_index *idx, const float *queries_dev, const float *sqdist_dev,
                                    int32_t n_queries, int32_t item_series, uint64_t *bits_dev, void *hip_stream);

/*
 * Query summaries as the device computes them (Section 2.2 on the query; Section 3.3.1 table):
 *   info          host out (may be NULL).
 *   table_dev     optional device out float32 [16][256]: per-segment lower-bound terms
 *                 L * delta(q_s, c)^2, rounded toward zero (so their sum never exceeds the bound).
 * Synchronous.
 */
paris_status paris_query_info_get(paris_index *idx, const float *query_dev, paris_query_info *info,
                                  float *table_dev, void *hip_stream);

/*
 * The lower-bound scan alone (Section 3.3.3, LBC worker) against a caller-given threshold on
 * the squared bound: every series whose float32 bound is <= threshold_sq is written, in no
 * particular order, as (index, bound) to idx_dev[0..) / lb_dev[0..).
 *   capacity      entries available in idx_dev / lb_dev.
 *   count         host out: number of series that passed (may exceed capacity; then only
 *                 capacity entries were written and PARIS_EOVERFLOW is returned).
 * Synchronous.
 */
paris_status paris_lb_scan(paris_index *idx, const float *query_dev, float threshold_sq,
                           uint32_t *idx_dev, float *lb_dev, int64_t capacity, int64_t *count,
                           void *hip_stream);

/*
 * Best-so-far sharing during refinement (Section 3.3: ParIS+ keeps one best-so-far that every
 * distance worker reads and lowers; nb-ParIS+ gives each worker its own copy, initialised with
 * the approximate answer, and takes the minimum over the copies at the end).
 *   shared  1: every lane group of the refine kernel re-reads the shared best-so-far as other
 *           groups lower it (ParIS+'s design). 0 (the default set by paris_build): each lane
 *           group (one survivor at a time, the GPU's distance worker) prunes only against the
 *           approximate search's best-so-far and the smallest distance it has itself completed;
 *           the answer is still the minimum over all groups. Results are identical either way;
 *           only the number of rows refined (paris_stats.refined) and the time change: private
 *           copies refine a few percent more rows but skip the re-reads of one hot address,
 *           and on hard queries run faster. Affects paris_query_exact (and the per-query
 *           fallback of batches).
 * Returns PARIS_EINVAL for any other value, PARIS_ESTATE for a bad handle. Host only.
 */
paris_status paris_set_bsf_sharing(paris_index *idx, int32_t shared);

/*
 * Per-phase device timing of paris_query_exact, with HIP events on the call's stream:
 * [0] query summaries + approximate-search seed (+ the seed network), [1] lower-bound scan,
 * [2] refinement + float64 resolve. paris_set_timing(idx, 1) times all three phases with events
 * recorded between them (each phase then includes the dispatch gap before its first kernel);
 * paris_set_timing(idx, 2) times only the scan, with a start and a stop event bound to the scan
 * kernel's own dispatch (its start-to-end duration); paris_set_timing(idx, 3) does the same for
 * the scan of every 8th paris_query_exact call (a sample that leaves the other calls without
 * events); 0 turns timing off; each call zeroes the totals. With timing on, paris_lb_scan adds
 * its scan kernel's duration (events bound to its dispatch) to [1]. Events are read back
 * one query late (two event sets alternate), so timing adds no synchronisation to a query.
 * paris_get_timing waits for the outstanding events and returns the summed milliseconds
 * (ms_out3[3]) and the number of timed calls.
 */
paris_status paris_set_timing(paris_index *idx, int32_t enable);
paris_status paris_get_timing(paris_index *idx, double *ms_out3, int64_t *n_queries);

/*
 * With timing on, paris_query_batch launches its pipeline directly (not through the captured
 * graph) with HIP events between the stages; ms_out5 receives the summed milliseconds of
 * [0] reset + seeds + screen thresholds, [1] block bound (alive bits), [2] bfloat16 MFMA
 * screen, [3] float32 re-score, [4] float64 resolve, and n_chunks the number of timed chunks.
 */
paris_status paris_get_batch_timing(const paris_index *idx, double *ms_out5, int64_t *n_chunks);

/* Release the handle (the borrowed buffers are not touched). NULL is accepted. */
paris_status paris_free(paris_index *idx);

/*
 * ---- Learned best-so-far seed ------------------------------------------------------------
 * The approximate search that opens exact search (Section 3.3) visits the one leaf selected by
 * the query's own iSAX word. With a seed network attached to an EQUAL_COUNT index, it instead
 * visits the 8 leaves with the highest scores of a 16 -> 256 -> 256 -> n_leaves perceptron on
 * the query's PAA (ReLU hidden layers; ties by lowest leaf id), refining in every run of 512
 * sorted positions of those leaves the member with the smallest lower bound. The seed stays a
 * true distance, so answers are unchanged; only the pruning power of the first best-so-far
 * changes. The network is not part of the paper: it is trained with the calls below on
 * (query features, leaf of the query's exact nearest neighbour) pairs from the exact search.
 *
 * Parameters: one float32 vector of paris_mlp_param_count() values, packed as
 *   W1 [256][16], b1 [256], W2 [256][256], b2 [256], W3 [n_leaves][256], b3 [n_leaves]
 * (row-major, rows indexed by output unit; 1,122,816 values at 4096 leaves).
 * Arithmetic: products take bfloat16 operands (weights rounded to nearest even from the
 * float32 master copy, hidden activations and back-propagated gradients likewise; the
 * 16 features stay float32) with float32 accumulation; biases are float32. Loss: mean softmax
 * cross-entropy. Optimiser: Adam (Kingma and Ba 2015, Algorithm 1) on the master copy.
 * A network keeps its parameters, Adam moments and the activations of max_rows rows in a
 * caller-owned device workspace of paris_mlp_workspace_size() bytes; the library allocates no
 * device memory for it. One call at a time per network and per index using it.
 */
typedef struct paris_mlp paris_mlp;  /* opaque, library-owned host handle */

typedef struct paris_adam {
    float lr;      /* step size, > 0                    */
    float beta1;   /* first-moment decay, in [0, 1)     */
    float beta2;   /* second-moment decay, in [0, 1)    */
    float eps;     /* denominator offset, > 0           */
} paris_adam;

/* count (host out): parameters of a network scoring n_leaves leaves (multiple of 64,
   64 .. 65536). */
paris_status paris_mlp_param_count(int32_t n_leaves, int64_t *count);

/* bytes (host out): the device workspace a network of n_leaves leaves and max_rows rows needs. */
paris_status paris_mlp_workspace_size(int32_t n_leaves, int32_t max_rows, int64_t *bytes);

/* Create a network with all-zero parameters in workspace_dev (device, caller-owned, 256-byte
   aligned, at least paris_mlp_workspace_size() bytes; it must outlive the network and is
   zeroed here). max_rows (multiple of 64, 64 .. 65536) bounds the rows of one training step;
   inference on more rows runs in pieces of max_rows. Synchronous. PARIS_EINVAL for a bad
   shape, a NULL, misaligned or short workspace. Release with paris_mlp_free, which leaves the
   workspace to its owner. */
paris_status paris_mlp_create(int32_t n_leaves, int32_t max_rows, void *workspace_dev, int64_t workspace_bytes,
                              paris_mlp **out);

/* Copy parameters in (params_dev float32 [count], device) and reset Adam's moments and step
   count; or copy them out. Asynchronous on hip_stream. */
paris_status paris_mlp_set_params(paris_mlp *net, const float *params_dev, void *hip_stream);
paris_status paris_mlp_get_params(const paris_mlp *net, float *params_dev, void *hip_stream);

/* Features of queries [n_queries][length] (device, float32; length a multiple of 16, <= 2048):
   features_dev float32 [n_queries][16] receives each query's PAA (Section 2.2), summed in
   float64 in ascending position and divided by length / 16, then rounded to float32.
   Asynchronous. */
paris_status paris_query_features(const float *queries_dev, int64_t n_queries, int32_t length,
                                  float *features_dev, void *hip_stream);

/* logits_dev float32 [rows][n_leaves] (device out) of features_dev float32 [rows][16].
   Asynchronous. */
paris_status paris_mlp_forward(paris_mlp *net, const float *features_dev, int64_t rows,
                               float *logits_dev, void *hip_stream);

/* leaves_dev int32 [rows][8] (device out): the 8 best-scoring leaves of every row, best first,
   equal logits by lowest leaf id. Asynchronous. */
paris_status paris_mlp_top_leaves(paris_mlp *net, const float *features_dev, int64_t rows,
                                  int32_t *leaves_dev, void *hip_stream);

/* Gradient of the mean loss over rows (1 .. max_rows) examples, packed like the parameters,
   into grad_dev float32 [count] (device out); loss_dev (device out, may be NULL) receives the
   mean loss. Example r is features_dev[s] with label labels_dev[s] (leaf id, int32), where
   s = rows_sel_dev[r] if rows_sel_dev (device int32 [rows]) is not NULL, else s = r.
   Asynchronous. */
paris_status paris_mlp_grad(paris_mlp *net, const float *features_dev, const int32_t *labels_dev,
                            const int32_t *rows_sel_dev, int64_t rows, float *grad_dev,
                            float *loss_dev, void *hip_stream);

/* One training step: the gradient as in paris_mlp_grad, then one Adam update of the master
   parameters and their bfloat16 copy. Asynchronous. */
paris_status paris_mlp_train_step(paris_mlp *net, const float *features_dev, const int32_t *labels_dev,
                                  const int32_t *rows_sel_dev, int64_t rows, const paris_adam *opt,
                                  float *loss_dev, void *hip_stream);

/* One Adam update of the master parameters (and their bfloat16 copy) with a caller-supplied
   gradient grad_dev float32 [count] (device), packed like the parameters: e.g. a gradient
   summed over several devices' paris_mlp_grad results. Asynchronous. */
paris_status paris_mlp_apply(paris_mlp *net, const float *grad_dev, const paris_adam *opt, void *hip_stream);

/* Release a network; indexes using it go back to the plain seed. NULL is accepted. */
paris_status paris_mlp_free(paris_mlp *net);

/* Training labels: leaves_dev int32 [count] (device out) receives the EQUAL_COUNT leaf holding
   each series index of series_dev int64 [count] (device; -1 for an index outside the
   collection): the leaf whose slice [floor(l N / n_leaves), floor((l+1) N / n_leaves)) of the
   order sorted by (leaf key, index) contains the series. PARIS_EINVAL on a ROOT16 index.
   Asynchronous. */
paris_status paris_leaf_of(const paris_index *idx, const int64_t *series_dev, int64_t count,
                           int32_t *leaves_dev, void *hip_stream);

/* Attach (enabled = 1) or detach (enabled = 0, or net = NULL) the learned seed for both
   paris_query_exact and paris_query_batch. The index must be EQUAL_COUNT with n_leaves equal
   to the network's, on the same device (else PARIS_EINVAL). The network is borrowed: it must
   outlive its use. With a batch workspace attached, the pipeline graph is captured again
   (synchronous). */
paris_status paris_set_seed_model(paris_index *idx, paris_mlp *net, int32_t enabled);

/* Static English text for a status code. */
const char *paris_status_string(paris_status s);

#ifdef __cplusplus
}
#endif

#endif /* PARIS_H */
