// Host side of the C ABI declared in include/paris.h: argument checks, workspace planning,
// kernel sequencing, launch-shape autotuning and read-back. No exception or abort crosses the
// boundary.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <atomic>
#include <mutex>
#include <new>
#include <unordered_set>
#include <vector>

#include "paris.h"
#include "paris_internal.h"

using namespace paris;

namespace {

constexpr uint32_t kMagic = 0x50415249u;  // "PARI"
// launch shapes of the lower-bound scan: (threads, blocks per CU, run envelopes per thread in
// flight)
constexpr int kScanCands = 8;
constexpr ScanShape kScanCandidates[kScanCands] = {{512, 2, 1}, {512, 2, 2}, {512, 4, 1}, {512, 1, 4},
                                                   {256, 4, 1}, {256, 4, 2}, {256, 8, 1}, {256, 3, 4}};
constexpr int kTunePer = 6;   // queries of the online phase (each scanned with every candidate)
// mapped host buffer of an index: the query result, then the k-NN answers 256 bytes on
constexpr size_t kHostResBytes = 256 + kKnnMax * sizeof(KnnHit);
static_assert(sizeof(QResult) <= 256, "the k-NN answers follow the result at 256 bytes");
constexpr size_t kAlign = 256;

size_t align_up(size_t v) { return (v + kAlign - 1) & ~(kAlign - 1); }

// Workspace layout. The radix-sort scratch (alternate keys / positions / histograms) is only
// needed during the build and aliases the survivor and completed-candidate buffers.
struct Plan {
    size_t hdr, sax, saxs, env, keys, perm, roff, qs, t8, knn, surv, done, total;
    size_t keys_alt, perm_alt, hist;
    // ADS+ tree (leaf mode 2): nodes, and the scratch of a build round (todo ids, chunk starts,
    // splits; chunks, their counts and destinations); 0 otherwise
    size_t tree, tree_todo, tree_todo_chunks, tree_split, tree_chunks, tree_ones, tree_dst;
    long long node_cap, todo_cap, chunk_cap;
};

// Largest number of nodes a tree over N series with leaf capacity cap is given: the root
// subtrees, twice a generous count of splits (every split node holds more than cap series, so
// the nodes split in one round number at most N / (cap + 1)), and room for chains of splits of
// a group of identical words. A build that would need more stops splitting (its leaves stay
// larger than cap; the search only reads a larger window).
long long tree_node_cap(long long N, int cap)
{
    const long long per_round = N / ((long long)cap + 1) + 1;
    return kRoots + 8 * per_round + 2 * kTreeMaxDepth * 64;
}

void make_plan(long long N, Plan* p, const paris_config* cfg)
{
    size_t off = 0;
    auto take = [&off](size_t bytes) { const size_t at = off; off = align_up(off + bytes); return at; };
    p->hdr = take(256);
    p->sax = take((size_t)N * 16);
    p->saxs = take((size_t)N * 16);
    p->env = take((size_t)(N + kEnvRun - 1) / kEnvRun * 32);
    p->keys = take((size_t)N * 8);
    p->perm = take((size_t)N * 4);
    p->roff = take(65537 * 4);
    p->qs = take(sizeof(QState));
    p->t8 = take(kSeg * kSym * 4);
    p->knn = take((size_t)(kKnnMax + kKnnSeedCap) * 8);
    p->surv = take((size_t)N * 8);
    // every survivor completes at most once, plus the head survivor computed first (it is also
    // met again in the list): N + 1 entries
    p->done = take((size_t)(N + 1) * 8);
    p->tree = p->tree_todo = p->tree_todo_chunks = p->tree_split = p->tree_chunks = p->tree_ones = p->tree_dst = 0;
    p->node_cap = p->todo_cap = p->chunk_cap = 0;
    if (cfg && cfg->leaf_mode == PARIS_LEAF_ADS) {
        p->node_cap = tree_node_cap(N, cfg->leaf_cap);
        p->todo_cap = N / ((long long)cfg->leaf_cap + 1) + 1;
        p->chunk_cap = N / kTreeChunk + p->todo_cap + 1;
        p->tree = take((size_t)p->node_cap * sizeof(AdsNode));
        p->tree_todo = take((size_t)p->todo_cap * 4);
        p->tree_todo_chunks = take((size_t)(p->todo_cap + 1) * 4);
        p->tree_split = take((size_t)p->todo_cap * 4);
        p->tree_chunks = take((size_t)p->chunk_cap * sizeof(TreeChunk));
        p->tree_ones = take((size_t)p->chunk_cap * kSeg * 4);
        p->tree_dst = take((size_t)p->chunk_cap * 8);
    }
    p->total = off;
    p->keys_alt = p->surv;  // 8N bytes
    p->perm_alt = p->done;  // 4N bytes
    p->hist = align_up(p->done + (size_t)N * 4);
    if (p->hist + sort_hist_words(N) * 4 > p->total) {
        // histogram does not fit behind the alternate positions: give it its own space
        p->hist = p->total;
        p->total = align_up(p->total + sort_hist_words(N) * 4);
    }
}

bool config_ok(const paris_config* c)
{
    if (!c) return false;
    if (c->segments != 16 || c->card_bits != 8) return false;
    if (c->leaf_mode != PARIS_LEAF_ROOT16 && c->leaf_mode != PARIS_LEAF_EQUAL_COUNT &&
        c->leaf_mode != PARIS_LEAF_ADS)
        return false;
    if (c->leaf_mode == PARIS_LEAF_ADS && (c->leaf_cap < 1 || c->leaf_cap > (1 << 20))) return false;
    if (c->leaf_mode == PARIS_LEAF_EQUAL_COUNT && (c->n_leaves < 1 || c->n_leaves > 65536)) return false;
    if (c->seed_cap < 0 || c->seed_cap > (1 << 24)) return false;
    return true;
}

bool shape_ok(long long N, int n)
{
    return N >= 1 && N <= 0xFFFFFFFELL && n >= 16 && n % 16 == 0 && n <= kMaxLength;
}

double gamma_k(int k)
{
    const double u = std::ldexp(1.0, -24);
    return k * u / (1.0 - k * u);
}

// prune_rel: a series is dropped (bound or partial distance above bsf * (1 + prune_rel)) only
// when its exact distance provably exceeds the exact nearest distance: covers the float32 error
// of the best-so-far (gamma_{n+2}), of a partial distance (gamma_n) and of the 16-term bound sum
// (gamma_16), twice over, plus slack for the rounded PAA of the bound.
// band_rel: the exact nearest neighbour's float32 distance is within (1 + gamma)/(1 - gamma) of
// the final float32 best, so everything within 4 gamma_{n+2} is re-scored in float64.
Margins margins_for_length(int n)
{
    Margins m;
    m.prune_rel = 2.0 * (gamma_k(n + 2) + gamma_k(n) + gamma_k(16)) + std::ldexp(1.0, -30);
    m.band_rel = 4.0 * gamma_k(n + 2) + std::ldexp(1.0, -30);
    return m;
}

// Relative margin c of the bfloat16 screen, |d~^2 - d^2| <= c (qn + xn): bfloat16 rounding of
// both operands (2 u_b + u_b^2, u_b = 2^-8), the float32 norms (gamma_n), and the MFMA's float32
// accumulation of the np products plus the two folded threshold terms, whose magnitudes are
// below 2 (qn + xn) (unit roundoff taken as 2^-23 so truncating accumulation is covered:
// 2 gamma (1/2 (1 + u_b)^2 + 2) <= 6 gamma); inflated by 5%.
float screen_margin(int n, int np)
{
    const double ub = std::ldexp(1.0, -8);
    const double u23 = std::ldexp(1.0, -23);
    const double u24 = std::ldexp(1.0, -24);
    auto gam = [](int k, double u) { return k * u / (1.0 - k * u); };
    const double c = (2.0 * ub + ub * ub) + 6.0 * gam(np + 48, u23) * (1.0 + ub) * (1.0 + ub) +
                     2.0 * gam(n, u24) + 16.0 * u24;
    return (float)(1.05 * c + 32.0 * u24);
}

paris_status device_ok()
{
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || count <= 0) return PARIS_ENODEV;
    return PARIS_OK;
}

}  // namespace

// The learned-seed network: float32 master weights, their bfloat16 mirror, Adam moments and the
// activation / gradient buffers of up to max_rows rows, all in one device allocation.
struct paris_mlp {
    uint32_t magic;
    int device;
    int n_out, max_rows;
    MlpOffsets off;
    uint8_t* mem;
    float* master;
    uint16_t* wb;
    float* grad;
    float* am;
    float* av;
    float* P;          // [max_rows][16] features of the current rows (inference from queries)
    uint16_t* H1;      // [max_rows][256]
    uint16_t* H2;      // [max_rows][256]
    float* Z;          // [max_rows][n_out] logits
    float* G3;         // [max_rows][n_out]
    uint16_t* G3b;
    float* G2;         // [max_rows][256]
    uint16_t* G2b;
    float* G1;         // [max_rows][256]
    uint16_t* G1b;
    float* loss_row;   // [max_rows]
    unsigned long long* partq;  // [n_out / 256 + 1][8] per-query block keys
    long long step;    // Adam steps taken
};

struct paris_index {
    uint32_t magic;
    int device;
    const float* X;
    long long N;
    int n;
    paris_config cfg;
    uint8_t* ws;
    size_t ws_bytes;
    Plan plan;
    QState* host_qs;   // pinned read-back buffer
    QResult* host_res;       // pinned, device-mapped: the query result lands here directly
    QResult* host_res_dev;   // its device address
    KnnHit* host_knn;        // the k-NN answers, in the same mapped allocation (256 bytes on)
    KnnHit* host_knn_dev;
    Margins mg;
    ScanShape scan;
    // online scan tuning: each of the first kTunePer queries is scanned with every candidate
    // shape, each scan timed by events bound to its dispatch; the smallest total wins
    int scan_online;        // queries left in the online phase (0: done or off)
    bool scan_decide;       // the phase is over and its events await reading
    hipEvent_t tune_ev[kScanCands * kTunePer][2];
    int refine_blocks;
    int refine_lanes;
    int bsf_private;        // 1 (default): per-group best-so-far copies; 0: one shared best-so-far
    bool timing;
    int timing_mode;        // paris_set_timing: 1 all three phases, 2 the scan only, 3 the scan of every 8th call
    long long timing_calls; // paris_query_exact calls since timing was set (mode 3 sampling)
    hipEvent_t ev[2][4];    // two event sets, used alternately: a set is read back one query later
    bool ev_pending[2];
    int ev_set;
    double phase_ms[3];
    long long timed_queries;
    // batched path (paris_batch_attach)
    uint8_t* bws;
    size_t bws_bytes;
    int max_batch;
    int np;     // screened dimensions rounded up to 32
    int proj;   // segment length of the screen's projection (1: n <= 256, the series itself)
    bool screen_ok;
    struct {
        size_t hdr, xb, xn, qin, qb, bq, qbias, cand, cand_d2, oidx, odist, fb, leaves, qpaa, mask, total;
        uint32_t cand_cap;
    } bp;
    ScreenShape screen;
    float c_screen;
    double seed_rel;
    hipGraph_t graph;
    hipGraphExec_t graph_exec;
    BatchHdr* host_hdr;   // pinned read-back of the batch header
    uint32_t* host_fb;    // pinned read-back of the fallback list
    long long batch_candidates;
    bool block_lb;        // screen only the (query, work item) pairs that the block bound keeps
    long long tiles_run, tiles_dense;   // screen query tiles run / a dense screen's count
    hipEvent_t bev[6];    // batch stage events (timing on): seeds | block bound | screen | re-score | resolve
    double batch_ms[5];
    long long timed_chunks;
    // learned seed (paris_set_seed_model): the network is borrowed, not owned
    paris_mlp* model;
    bool learned;
    // ADS+ tree (leaf mode 2)
    long long n_tree_nodes;
    long long tree_max_leaf;
};

namespace {

QueryArgs args_for(const paris_index* h)
{
    QueryArgs a;
    uint8_t* ws = h->ws;
    a.X = h->X;
    a.N = h->N;
    a.n = h->n;
    a.sax = ws + h->plan.sax;
    a.saxs = ws + h->plan.saxs;
    a.env = ws + h->plan.env;
    a.keys = reinterpret_cast<const unsigned long long*>(ws + h->plan.keys);
    a.perm = reinterpret_cast<const uint32_t*>(ws + h->plan.perm);
    a.roff = reinterpret_cast<const uint32_t*>(ws + h->plan.roff);
    a.leaf_mode = h->cfg.leaf_mode;
    a.n_leaves = h->cfg.n_leaves;
    a.seed_cap = h->cfg.seed_cap;
    a.qs = reinterpret_cast<QState*>(ws + h->plan.qs);
    a.t8 = reinterpret_cast<float*>(ws + h->plan.t8);
    a.surv = reinterpret_cast<uint2*>(ws + h->plan.surv);
    a.surv_cap = (uint32_t)h->N;
    a.done = reinterpret_cast<uint2*>(ws + h->plan.done);
    a.done_cap = (uint32_t)h->N + 1u;
    a.mg = h->mg;
    a.host_res = nullptr;
    a.knn_k = 0;
    a.knn_r = 0;
    a.knn_slots = reinterpret_cast<unsigned long long*>(ws + h->plan.knn);
    a.knn_seed = a.knn_slots + kKnnMax;
    a.knn_out = nullptr;
    a.tree = h->cfg.leaf_mode == PARIS_LEAF_ADS ? reinterpret_cast<const AdsNode*>(ws + h->plan.tree) : nullptr;
    a.tree_window = (int)(h->tree_max_leaf < 0x7FFFFFFF ? h->tree_max_leaf : 0x7FFFFFFF);
    a.leaf_keys = nullptr;
    a.leaf_key_count = 0;
    a.learned_cpl = 0;
    a.refine_blocks = h->refine_blocks;
    a.refine_lanes = h->refine_lanes;
    a.bsf_private = h->bsf_private;
    return a;
}

MlpNet net_of(const paris_mlp* m)
{
    MlpNet net;
    net.master = m->master;
    net.wb = m->wb;
    net.n_out = m->n_out;
    net.off = m->off;
    return net;
}

// chunks of kSeedChunk sorted positions in the largest equal-count leaf
int learned_chunks(const paris_index* h)
{
    const long long leaf = (h->N + h->cfg.n_leaves - 1) / h->cfg.n_leaves;
    const long long c = (leaf + kSeedChunk - 1) / kSeedChunk;
    return (int)(c < 1 ? 1 : c);
}

// Live handles: a freed or foreign pointer is rejected without being dereferenced.
std::mutex g_live_mu;
std::unordered_set<const paris_index*> g_live;

bool handle_ok(const paris_index* h)
{
    if (!h) return false;
    std::lock_guard<std::mutex> g(g_live_mu);
    return g_live.count(h) != 0 && h->magic == kMagic;
}

#define HIP_TRY(expr)                                  \
    do {                                               \
        if ((expr) != hipSuccess) return PARIS_EHIP;   \
    } while (0)

// Add the durations recorded in event set `set` to the totals (waits for its last event, which
// the queries issued since have normally long passed).
paris_status collect_timing(paris_index* h, int set)
{
    hipEvent_t* ev = h->ev[set];
    if (h->timing_mode == 1) {
        HIP_TRY(hipEventSynchronize(ev[3]));
        for (int k = 0; k < 3; ++k) {
            float ms = 0.f;
            HIP_TRY(hipEventElapsedTime(&ms, ev[k], ev[k + 1]));
            h->phase_ms[k] += ms;
        }
    } else {
        HIP_TRY(hipEventSynchronize(ev[2]));
        float ms = 0.f;
        HIP_TRY(hipEventElapsedTime(&ms, ev[1], ev[2]));
        h->phase_ms[1] += ms;
    }
    h->ev_pending[set] = false;
    h->timed_queries += 1;
    return PARIS_OK;
}

paris_status collect_pending(paris_index* h)
{
    for (int set = 0; set < 2; ++set)
        if (h->ev_pending[set]) {
            paris_status s = collect_timing(h, set);
            if (s != PARIS_OK) return s;
        }
    return PARIS_OK;
}

// ADS+ tree build (leaf mode 2): the root subtrees from the root offsets, then rounds that split,
// in ascending node id, every leaf holding more than cap series with a segment below 8 bits
// (the kernels choose the segment and partition the leaf order). The host lists each round's
// nodes and cuts them into chunks; after the round it reads the new children back to list the
// next round. Returns the node count and the size of the largest leaf.
paris_status build_tree(const Plan& plan, uint8_t* ws, long long N, int cap, hipStream_t st, long long* n_nodes,
                        long long* max_leaf_out)
{
    AdsNode* nodes = reinterpret_cast<AdsNode*>(ws + plan.tree);
    const uint32_t* roff = reinterpret_cast<const uint32_t*>(ws + plan.roff);
    HIP_TRY(launch_tree_roots(roff, nodes, st));
    std::vector<uint32_t> hroff(kRoots + 1);
    HIP_TRY(hipMemcpyAsync(hroff.data(), roff, (size_t)(kRoots + 1) * 4, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    struct Item {
        int32_t id;
        uint32_t start, end;
    };
    std::vector<Item> todo, nt;
    long long max_leaf = 0;
    for (int r = 0; r < kRoots; ++r) {
        const long long sz = (long long)hroff[r + 1] - hroff[r];
        if (sz > cap) todo.push_back({r, hroff[r], hroff[r + 1]});
        else if (sz > max_leaf) max_leaf = sz;
    }
    TreeRound R;
    R.nodes = nodes;
    R.todo = reinterpret_cast<const int32_t*>(ws + plan.tree_todo);
    R.todo_chunks = reinterpret_cast<const uint32_t*>(ws + plan.tree_todo_chunks);
    R.todo_split = reinterpret_cast<int32_t*>(ws + plan.tree_split);
    R.chunks = reinterpret_cast<const TreeChunk*>(ws + plan.tree_chunks);
    R.chunk_ones = reinterpret_cast<uint32_t*>(ws + plan.tree_ones);
    R.chunk_dst = reinterpret_cast<uint2*>(ws + plan.tree_dst);
    R.sax = ws + plan.sax;
    R.perm = reinterpret_cast<uint32_t*>(ws + plan.perm);
    R.perm_tmp = reinterpret_cast<uint32_t*>(ws + plan.surv);   // 4N of the 8N survivor bytes
    long long next = kRoots;
    std::vector<int32_t> h_todo;
    std::vector<uint32_t> h_tc;
    std::vector<TreeChunk> h_chunks;
    std::vector<AdsNode> kids;
    while (!todo.empty()) {
        const long long n = (long long)todo.size();
        long long chunks = 0;
        for (const Item& it : todo) chunks += ((long long)it.end - it.start + kTreeChunk - 1) / kTreeChunk;
        if (next + 2 * n > plan.node_cap || n > plan.todo_cap || chunks > plan.chunk_cap) {
            // out of node room: these stay leaves
            for (const Item& it : todo)
                if ((long long)it.end - it.start > max_leaf) max_leaf = (long long)it.end - it.start;
            break;
        }
        h_todo.resize(n);
        h_tc.resize(n + 1);
        h_chunks.clear();
        for (long long i = 0; i < n; ++i) {
            h_todo[i] = todo[i].id;
            h_tc[i] = (uint32_t)h_chunks.size();
            for (uint32_t a = todo[i].start; a < todo[i].end; a += kTreeChunk) {
                const uint32_t b = todo[i].end - a > (uint32_t)kTreeChunk ? a + kTreeChunk : todo[i].end;
                h_chunks.push_back(TreeChunk{(uint32_t)i, a, b, 0u});
            }
        }
        h_tc[n] = (uint32_t)h_chunks.size();
        HIP_TRY(hipMemcpyAsync(ws + plan.tree_todo, h_todo.data(), (size_t)n * 4, hipMemcpyHostToDevice, st));
        HIP_TRY(hipMemcpyAsync(ws + plan.tree_todo_chunks, h_tc.data(), (size_t)(n + 1) * 4, hipMemcpyHostToDevice, st));
        HIP_TRY(hipMemcpyAsync(ws + plan.tree_chunks, h_chunks.data(), h_chunks.size() * sizeof(TreeChunk),
                               hipMemcpyHostToDevice, st));
        R.n_todo = (int)n;
        R.next = (int)next;
        HIP_TRY(launch_tree_round(R, (int)h_chunks.size(), st));
        kids.resize(2 * n);
        HIP_TRY(hipMemcpyAsync(kids.data(), nodes + next, (size_t)(2 * n) * sizeof(AdsNode), hipMemcpyDeviceToHost, st));
        HIP_TRY(hipStreamSynchronize(st));
        nt.clear();
        for (long long j = 0; j < 2 * n; ++j) {
            const AdsNode& k = kids[j];
            const long long sz = (long long)k.end - k.start;
            bool open = false;
            for (int sg = 0; sg < kSeg; ++sg) open |= k.card[sg] < 8;
            if (sz > cap && open) nt.push_back({(int32_t)(next + j), k.start, k.end});
            else if (sz > max_leaf) max_leaf = sz;
        }
        next += 2 * n;
        todo.swap(nt);
    }
    *n_nodes = next;
    *max_leaf_out = max_leaf;
    return PARIS_OK;
}

// Per-query scratch taken from somewhere other than the index workspace (the allocation-free
// entry point): query state, lower-bound tables, survivor and completed-candidate lists.
struct QueryScratch {
    QState* qs;
    float* t8;
    uint2* surv;
    uint32_t surv_cap;
    uint2* done;
    uint32_t done_cap;
};

// ---- tuned launch shapes, kept across processes ------------------------------------------
// PARIS_TUNE_CACHE names a text file with one tuned shape per line,
//   <kind> <arch> <a> <b> <c> : <v0> <v1> <v2> <v3>
// kind "scan": a = series length, b = floor(log2 N), c = 1 for a collection in host memory;
//              values threads, blocks per CU, unroll, 0 (the online phase's decision);
// kind "screen": a = screened dimensions, b = floor(log2 N), c = 2 * max_batch + block bound;
//              values query-tile rows, blocks per CU, subtiles, MFMA form.
// The last line with a matching key wins; other lines are ignored. Decisions are appended.
std::mutex g_tune_mu;

const char* tune_cache_path()
{
    const char* p = std::getenv("PARIS_TUNE_CACHE");
    return p && p[0] ? p : nullptr;
}

// the device's architecture name up to its first feature flag (e.g. "gfx950")
void arch_name(char* out, size_t cap)
{
    std::snprintf(out, cap, "unknown");
    int dev = 0;
    hipDeviceProp_t p;
    if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&p, dev) != hipSuccess) return;
    size_t i = 0;
    for (; i + 1 < cap && p.gcnArchName[i] && p.gcnArchName[i] != ':' && p.gcnArchName[i] != ' '; ++i)
        out[i] = p.gcnArchName[i];
    out[i] = 0;
    if (i == 0) std::snprintf(out, cap, "unknown");
}

int floor_log2(long long v)
{
    int b = 0;
    while (v > 1) { v >>= 1; ++b; }
    return b;
}

bool tune_cache_get(const char* kind, long long a, long long b, long long c, int v[4])
{
    const char* path = tune_cache_path();
    if (!path) return false;
    char arch[64];
    arch_name(arch, sizeof arch);
    std::lock_guard<std::mutex> g(g_tune_mu);
    FILE* f = std::fopen(path, "r");
    if (!f) return false;
    bool found = false;
    char line[256];
    while (std::fgets(line, sizeof line, f)) {
        char k[32], ar[64];
        long long la, lb, lc;
        int w[4];
        if (std::sscanf(line, "%31s %63s %lld %lld %lld : %d %d %d %d", k, ar, &la, &lb, &lc, &w[0], &w[1], &w[2],
                        &w[3]) != 9)
            continue;
        if (std::strcmp(k, kind) || std::strcmp(ar, arch) || la != a || lb != b || lc != c) continue;
        for (int i = 0; i < 4; ++i) v[i] = w[i];
        found = true;
    }
    std::fclose(f);
    return found;
}

void tune_cache_put(const char* kind, long long a, long long b, long long c, const int v[4])
{
    const char* path = tune_cache_path();
    if (!path) return;
    char arch[64];
    arch_name(arch, sizeof arch);
    std::lock_guard<std::mutex> g(g_tune_mu);
    FILE* f = std::fopen(path, "a");
    if (!f) return;   // an unwritable cache only costs the next process a tuning run
    std::fprintf(f, "%s %s %lld %lld %lld : %d %d %d %d\n", kind, arch, a, b, c, v[0], v[1], v[2], v[3]);
    std::fclose(f);
}

bool collection_in_host(const paris_index* h)
{
    hipPointerAttribute_t pa;
    const bool host = hipPointerGetAttributes(&pa, h->X) == hipSuccess && pa.type == hipMemoryTypeHost;
    (void)hipGetLastError();
    return host;
}

// a cached scan shape for this collection, if the cache holds a valid one
bool scan_from_cache(paris_index* h)
{
    int v[4];
    if (!tune_cache_get("scan", h->n, floor_log2(h->N), collection_in_host(h) ? 1 : 0, v)) return false;
    for (int c = 0; c < kScanCands; ++c)
        if (kScanCandidates[c].threads == v[0] && kScanCandidates[c].per_cu == v[1] &&
            kScanCandidates[c].unroll == v[2]) {
            h->scan = kScanCandidates[c];
            return true;
        }
    return false;
}

void scan_to_cache(const paris_index* h)
{
    const int v[4] = {h->scan.threads, h->scan.per_cu, h->scan.unroll, 0};
    tune_cache_put("scan", h->n, floor_log2(h->N), collection_in_host(h) ? 1 : 0, v);
}

paris_status run_query(paris_index* h, const float* q, hipStream_t st, long long* out_idx,
                       double* out_dist, long long qi, bool timed, QResult* host_res = nullptr,
                       const QueryScratch* scratch_in = nullptr)
{
    QueryArgs a = args_for(h);
    a.host_res = host_res;
    if (scratch_in) {
        a.qs = scratch_in->qs;
        a.t8 = scratch_in->t8;
        a.surv = scratch_in->surv;
        a.surv_cap = scratch_in->surv_cap;
        a.done = scratch_in->done;
        a.done_cap = scratch_in->done_cap;
        // the array keeps whatever the previous call on this device left: start from a clean
        // state (a kernel, not a memset, so the sequence stays capturable)
        HIP_TRY(launch_reset(a, st));
    }
    int set = 0;
    const bool all = h->timing_mode == 1;
    if (timed) {
        set = h->ev_set;
        if (h->ev_pending[set]) {
            paris_status cs = collect_timing(h, set);
            if (cs != PARIS_OK) return cs;
        }
    }
    hipEvent_t* ev = h->ev[set];
    if (h->scan_decide) {
        // the online phase's scans finished before their queries' results were read back
        HIP_TRY(hipEventSynchronize(h->tune_ev[kScanCands * kTunePer - 1][1]));
        // paired comparison: every candidate scanned the same queries; the smallest total wins
        float best = 1e30f;
        for (int c = 0; c < kScanCands; ++c) {
            float total = 0.f;
            for (int k = 0; k < kTunePer; ++k) {
                const int slot = k * kScanCands + c;
                float ms = 0.f;
                total += hipEventElapsedTime(&ms, h->tune_ev[slot][0], h->tune_ev[slot][1]) == hipSuccess ? ms : 1e30f;
            }
            if (total < best) { best = total; h->scan = kScanCandidates[c]; }
        }
        h->scan_decide = false;
        scan_to_cache(h);
    }
    const ScanShape shape = h->scan;
    // online phase: this query is scanned once with every candidate shape (in an order rotated
    // per query, so that no candidate always runs first on a cold cache), each run bound to its
    // own events; the last run's survivors are the ones refined
    const int online = (!timed && h->scan_online > 0) ? kTunePer - h->scan_online : -1;
    if (online >= 0 && --h->scan_online == 0) h->scan_decide = true;
    if (timed && all) HIP_TRY(hipEventRecord(ev[0], st));
    if (h->learned) {
        const paris_mlp* m = h->model;
        MlpQueryScratch sc{m->partq};
        HIP_TRY(launch_mlp_query(net_of(m), q, h->n, sc, st));
        a.leaf_keys = m->partq;
        a.leaf_key_count = (m->n_out + 255) / 256 * kTopLeaves;
        a.learned_cpl = learned_chunks(h);
    }
    HIP_TRY(launch_prepare_seed(a, q, st));
    // all phases: events recorded between the phases (each phase includes the gap before its
    // first kernel); the scan alone: events bound to the scan kernel's dispatch
    if (timed && all) HIP_TRY(hipEventRecord(ev[1], st));
    const bool bind = timed && !all;
    if (online >= 0) {
        for (int r = 0; r < kScanCands; ++r) {
            const int c = (r + online) % kScanCands;
            if (r > 0) HIP_TRY(launch_scan_again(a, st));
            const int slot = online * kScanCands + c;
            HIP_TRY(launch_lbscan(a, -1.f, kScanCandidates[c], st, h->tune_ev[slot][0], h->tune_ev[slot][1]));
        }
    } else {
        HIP_TRY(launch_lbscan(a, -1.f, shape, st, bind ? ev[1] : nullptr, bind ? ev[2] : nullptr));
    }
    if (timed && all) HIP_TRY(hipEventRecord(ev[2], st));
    HIP_TRY(launch_refine_resolve(a, q, out_idx, out_dist, qi, st));
    if (timed && all) HIP_TRY(hipEventRecord(ev[3], st));
    if (timed) {
        h->ev_pending[set] = true;
        h->ev_set = set ^ 1;
    }
    return PARIS_OK;
}

void fill_stats(const QResult& r, paris_stats* o)
{
    o->lb_survivors = r.n_surv;
    o->refined = r.n_refined;
    o->abandoned = r.n_abandon;
    o->bsf_updates = r.n_bsf_upd;
    o->resolved = r.n_resolved;
    if (r.seed_key == kBsfInit) {
        o->seed_index = -1;
        o->seed_dist = INFINITY;
    } else {
        uint32_t bits = (uint32_t)(r.seed_key >> 32);
        float d2;
        std::memcpy(&d2, &bits, 4);
        o->seed_index = (int64_t)(uint32_t)(r.seed_key & 0xFFFFFFFFu);
        o->seed_dist = std::sqrt((double)d2);
    }
    o->seed_lo = r.win_lo;
    o->seed_hi = r.win_hi;
    o->words_read = r.n_read;
}

// Launch-shape autotuner for the lower-bound scan: every candidate shape scans the whole SAX
// array at a zero threshold (the series' own word as the query: nothing but that row survives),
// timed with HIP events, back to back (array in cache) and, for large arrays, after a cache
// sweep (array in HBM); the smallest sum of the two medians wins.
// PARIS_SCAN_SHAPE="threads,blocks_per_cu,unroll" overrides the choice.
paris_status tune_scan(paris_index* h, hipStream_t st)
{
    const char* env = std::getenv("PARIS_SCAN_SHAPE");
    if (env) {
        int t = 0, b = 0, u = 4;
        const int got = std::sscanf(env, "%d,%d,%d", &t, &b, &u);
        if (got >= 2 && (t == 256 || t == 512) && b >= 1 && b <= 32 && (u == 1 || u == 2 || u == 4)) {
            h->scan = ScanShape{t, b, u};
            return PARIS_OK;
        }
    }
    // (threads, blocks per CU, run envelopes per thread in flight)
    const ScanShape* cands = kScanCandidates;
    const QueryArgs a = args_for(h);
    HIP_TRY(launch_prepare_seed(a, h->X, st));  // tables of series 0
    // Cold runs matter when the iSAX array outgrows the L2s; they are preceded by a read-only
    // sweep of up to 1 GiB of the raw collection, which evicts the array from the 256 MB
    // Infinity Cache (only possible when the collection is that large).
    const size_t raw = (size_t)h->N * h->n * 4;
    const size_t sweep = raw < ((size_t)1 << 30) ? raw : ((size_t)1 << 30);
    // (a collection in host memory is read over PCIe and never evicts the device caches)
    const bool host_coll = collection_in_host(h);
    const bool cold = !host_coll && (size_t)h->N * 16 > ((size_t)32 << 20) && sweep >= ((size_t)512 << 20);
    uint32_t* sink = reinterpret_cast<uint32_t*>(h->ws + h->plan.hdr) + 16;
    hipEvent_t e0, e1;
    HIP_TRY(hipEventCreate(&e0));
    HIP_TRY(hipEventCreate(&e1));
    float best = 1e30f;
    ScanShape pick = cands[1];
    constexpr int kReps = 9;
    auto median = [](float* t) {
        for (int i = 1; i < kReps; ++i)  // insertion sort
            for (int j = i; j > 0 && t[j] < t[j - 1]; --j) { const float x = t[j]; t[j] = t[j - 1]; t[j - 1] = x; }
        return t[kReps / 2];
    };
    for (int ci = 0; ci < kScanCands; ++ci) {
        const ScanShape& s = cands[ci];
        float score = 0.f;
        for (int pass = 0; pass < (cold ? 2 : 1); ++pass) {
            float t[kReps];
            for (int r = 0; r <= kReps; ++r) {
                if (pass == 1) HIP_TRY(launch_touch(h->X, sweep, sink, st));
                HIP_TRY(hipEventRecord(e0, st));
                HIP_TRY(launch_lbscan(a, 0.f, s, st));
                HIP_TRY(hipEventRecord(e1, st));
                HIP_TRY(hipEventSynchronize(e1));
                float ms = 0.f;
                HIP_TRY(hipEventElapsedTime(&ms, e0, e1));
                if (r > 0) t[r - 1] = ms;  // first run warms up
            }
            score += median(t);
        }
        if (score < best) { best = score; pick = s; }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    h->scan = pick;
    HIP_TRY(launch_reset(a, st));
    HIP_TRY(hipStreamSynchronize(st));
    return PARIS_OK;
}

// ---- batched path ------------------------------------------------------------------------
void make_batch_plan(paris_index* h, int max_batch)
{
    size_t off = 0;
    auto take = [&off](size_t bytes) { const size_t at = off; off = align_up(off + bytes); return at; };
    const size_t N = (size_t)h->N, M = (size_t)max_batch;
    h->bp.hdr = take(256);
    h->bp.xb = take((N + 31) / 32 * 32 * h->np * 2);   // whole 32-row fragment blocks
    h->bp.xn = take(N * 4);
    h->bp.qin = take(M * h->n * 4);
    h->bp.qb = take(M * h->np * 2);
    h->bp.bq = take(M * sizeof(BQuery));
    h->bp.qbias = take(M * 32);
    const size_t cap = M * 4096 < (size_t)0xFFFFFFF0u ? M * 4096 : (size_t)0xFFFFFFF0u;
    h->bp.cand_cap = (uint32_t)cap;
    h->bp.cand = take(cap * 8);
    h->bp.cand_d2 = take(cap * 4);
    h->bp.oidx = take(M * 8);
    h->bp.odist = take(M * 8);
    h->bp.fb = take(M * 4);
    h->bp.leaves = take(M * kTopLeaves * 4);
    h->bp.qpaa = take(M * kSeg * 8);
    // alive bits for the smallest work item of the 32-wide screen (128 sorted positions)
    h->bp.mask = take((N + 127) / 128 * ((M + 63) / 64) * 8);
    h->bp.total = off;
}

bool batch_screen_usable(const paris_index* h)
{
    return h->bws != nullptr && h->screen_ok && (h->cfg.seed_cap > 0 || h->cfg.leaf_mode == PARIS_LEAF_EQUAL_COUNT);
}

BatchHdr* bhdr(paris_index* h) { return reinterpret_cast<BatchHdr*>(h->bws + h->bp.hdr); }
BQuery* bqs(paris_index* h) { return reinterpret_cast<BQuery*>(h->bws + h->bp.bq); }

// The screen's accumulators bound each candidate's distance (the re-score's skip test) when the
// screen works on the series themselves (no projection) with the 32-wide form, which stores them.
int candidate_bounds_on(const paris_index* h) { return h->proj == 1 && h->screen.mfma == 32 ? 1 : 0; }

ScreenArgs screen_args(paris_index* h, int m, float* dump, bool masked = true)
{
    ScreenArgs s;
    s.Xb = reinterpret_cast<const uint16_t*>(h->bws + h->bp.xb);
    s.xn = reinterpret_cast<const float*>(h->bws + h->bp.xn);
    s.N = h->N;
    s.Qb = reinterpret_cast<const uint16_t*>(h->bws + h->bp.qb);
    s.bq = bqs(h);
    s.qbias = reinterpret_cast<uint16_t*>(h->bws + h->bp.qbias);
    s.M = m;
    s.cand = reinterpret_cast<uint2*>(h->bws + h->bp.cand);
    s.cand_d2 = reinterpret_cast<float*>(h->bws + h->bp.cand_d2);
    s.cand_cap = h->bp.cand_cap;
    s.hdr = bhdr(h);
    s.c_screen = h->c_screen;
    s.dump = dump;
    s.perm = reinterpret_cast<const uint32_t*>(h->ws + h->plan.perm);
    s.mask = masked && h->block_lb ? reinterpret_cast<unsigned long long*>(h->bws + h->bp.mask) : nullptr;
    s.env = h->ws + h->plan.env;
    s.qpaa = reinterpret_cast<const double*>(h->bws + h->bp.qpaa);
    s.seg_len = (double)(h->n / kSeg);
    s.seed_rel = h->seed_rel;
    s.prune_rel = h->mg.prune_rel;
    return s;
}

RescoreArgs rescore_args(paris_index* h, int m)
{
    RescoreArgs r;
    r.X = h->X;
    r.Q = reinterpret_cast<const float*>(h->bws + h->bp.qin);
    r.n = h->n;
    r.M = m;
    r.bq = bqs(h);
    r.cand = reinterpret_cast<const uint2*>(h->bws + h->bp.cand);
    r.cand_d2 = reinterpret_cast<float*>(h->bws + h->bp.cand_d2);
    r.cand_cap = h->bp.cand_cap;
    r.hdr = bhdr(h);
    r.prune_rel = h->mg.prune_rel;
    r.band_rel = h->mg.band_rel;
    r.fallback = reinterpret_cast<uint32_t*>(h->bws + h->bp.fb);
    r.ub_on = candidate_bounds_on(h);
    r.c_screen = h->c_screen;
    r.seed_rel = h->seed_rel;
    r.lb_on = h->screen.mfma == 32 ? 1 : 0;   // only the 32-wide screen stores accumulators
    r.P = h->proj;
    return r;
}

// ---- learned seed: network passes on up to max_rows rows --------------------------------
long long pad64(long long r) { return (r + 63) / 64 * 64; }

// forward: H1, H2 and the logits Z of `rows` rows of features (row r = P[sel ? sel[r] : r])
paris_status mlp_forward_rows(paris_mlp* m, const float* P, const int32_t* sel, int rows, hipStream_t st)
{
    const MlpNet net = net_of(m);
    const int mp = (int)pad64(rows);
    HIP_TRY(launch_l1_fwd(net, P, sel, rows, mp, m->H1, st));
    GemmArgs g{};
    g.A = m->H1; g.lda = kMlpHid; g.B = m->wb + m->off.w2; g.ldb = kMlpHid;
    g.M = mp; g.N = kMlpHid; g.K = kMlpHid; g.bias = m->master + m->off.b2; g.Cb = m->H2; g.ldc = kMlpHid;
    HIP_TRY(launch_gemm(g, 0, 0, kEpiBiasReluBf16, st));
    g = GemmArgs{};
    g.A = m->H2; g.lda = kMlpHid; g.B = m->wb + m->off.w3; g.ldb = kMlpHid;
    g.M = mp; g.N = m->n_out; g.K = kMlpHid; g.bias = m->master + m->off.b3; g.Cf = m->Z; g.ldc = m->n_out;
    HIP_TRY(launch_gemm(g, 0, 0, kEpiBiasF32, st));
    return PARIS_OK;
}

// forward + back-propagation into m->grad (packed like the parameters) and the mean loss
paris_status mlp_grad_rows(paris_mlp* m, const float* P, const int32_t* y, const int32_t* sel, int rows,
                           float* loss_out, hipStream_t st)
{
    paris_status s = mlp_forward_rows(m, P, sel, rows, st);
    if (s != PARIS_OK) return s;
    const int mp = (int)pad64(rows), no = m->n_out;
    HIP_TRY(launch_softmax_ce(m->Z, no, y, sel, rows, mp, m->G3, m->G3b, m->loss_row, st));
    GemmArgs g{};
    // dL/dA2 = (G3 W3) masked by the ReLU of layer 2
    g.A = m->G3b; g.lda = no; g.B = m->wb + m->off.w3; g.ldb = kMlpHid;
    g.M = mp; g.N = kMlpHid; g.K = no; g.mask = m->H2; g.ldm = kMlpHid; g.Cf = m->G2; g.Cb = m->G2b; g.ldc = kMlpHid;
    HIP_TRY(launch_gemm(g, 0, 1, kEpiMask, st));
    // dW3 = G3^T H2
    g = GemmArgs{};
    g.A = m->G3b; g.lda = no; g.B = m->H2; g.ldb = kMlpHid;
    g.M = no; g.N = kMlpHid; g.K = mp; g.Cf = m->grad + m->off.w3; g.ldc = kMlpHid;
    HIP_TRY(launch_gemm(g, 1, 1, kEpiF32, st));
    // dL/dA1 = (G2 W2) masked by the ReLU of layer 1
    g = GemmArgs{};
    g.A = m->G2b; g.lda = kMlpHid; g.B = m->wb + m->off.w2; g.ldb = kMlpHid;
    g.M = mp; g.N = kMlpHid; g.K = kMlpHid; g.mask = m->H1; g.ldm = kMlpHid; g.Cf = m->G1; g.Cb = m->G1b; g.ldc = kMlpHid;
    HIP_TRY(launch_gemm(g, 0, 1, kEpiMask, st));
    // dW2 = G2^T H1
    g = GemmArgs{};
    g.A = m->G2b; g.lda = kMlpHid; g.B = m->H1; g.ldb = kMlpHid;
    g.M = kMlpHid; g.N = kMlpHid; g.K = mp; g.Cf = m->grad + m->off.w2; g.ldc = kMlpHid;
    HIP_TRY(launch_gemm(g, 1, 1, kEpiF32, st));
    HIP_TRY(launch_l1_bwd(m->G1, P, sel, rows, m->grad + m->off.w1, st));
    HIP_TRY(launch_colsum(m->G3, mp, no, m->grad + m->off.b3, st));
    HIP_TRY(launch_colsum(m->G2, mp, kMlpHid, m->grad + m->off.b2, st));
    HIP_TRY(launch_colsum(m->G1, mp, kMlpHid, m->grad + m->off.b1, st));
    if (loss_out) HIP_TRY(launch_mean_loss(m->loss_row, rows, loss_out, st));
    return PARIS_OK;
}

// top leaves of M queries [M][n] (features, forward and selection in chunks of max_rows rows)
paris_status mlp_top_leaves_of_queries(paris_mlp* m, const float* Q, long long M, int n, int32_t* leaves,
                                       hipStream_t st)
{
    for (long long r0 = 0; r0 < M; r0 += m->max_rows) {
        const int rows = (int)(M - r0 < m->max_rows ? M - r0 : m->max_rows);
        HIP_TRY(launch_paa_features(Q + r0 * n, rows, pad64(rows), n, m->P, st));
        paris_status s = mlp_forward_rows(m, m->P, nullptr, rows, st);
        if (s != PARIS_OK) return s;
        HIP_TRY(launch_topk(m->Z, rows, m->n_out, kTopLeaves, leaves + r0 * kTopLeaves, st));
    }
    return PARIS_OK;
}

bool adam_ok(const paris_adam* o)
{
    return o && o->lr > 0.f && o->beta1 >= 0.f && o->beta1 < 1.f && o->beta2 >= 0.f && o->beta2 < 1.f &&
           o->eps > 0.f;
}

// one Adam step (Kingma and Ba 2015, Algorithm 1) with the given gradient
paris_status mlp_adam(paris_mlp* m, const float* grad, const paris_adam& o, hipStream_t st)
{
    m->step += 1;
    AdamArgs a;
    a.lr = o.lr;
    a.beta1 = o.beta1;
    a.beta2 = o.beta2;
    a.eps = o.eps;
    a.bc1 = (float)(1.0 - std::pow((double)o.beta1, (double)m->step));
    a.bc2 = (float)(1.0 - std::pow((double)o.beta2, (double)m->step));
    HIP_TRY(launch_adam(m->master, grad, m->am, m->av, m->wb, m->off.total, a, st));
    return PARIS_OK;
}

std::mutex g_mlp_mu;
std::unordered_set<const paris_mlp*> g_mlp_live;

bool mlp_ok(const paris_mlp* m)
{
    if (!m) return false;
    std::lock_guard<std::mutex> g(g_mlp_mu);
    return g_mlp_live.count(m) != 0 && m->magic == kMagic + 1;
}

// The batch pipeline on queries already copied to the internal query buffer: reset, seeds,
// screen thresholds, the MFMA screen, float32 re-score, float64 resolve.
paris_status launch_batch_pipeline(paris_index* h, int m, hipStream_t st, bool timed = false)
{
    const QueryArgs a = args_for(h);
    SeedBatch sb;
    sb.Q = reinterpret_cast<const float*>(h->bws + h->bp.qin);
    sb.bq = bqs(h);
    sb.qb = reinterpret_cast<uint16_t*>(h->bws + h->bp.qb);
    sb.np = h->np;
    sb.P = h->proj;
    sb.leaves = nullptr;
    sb.qpaa = reinterpret_cast<double*>(h->bws + h->bp.qpaa);
    if (timed) HIP_TRY(hipEventRecord(h->bev[0], st));
    HIP_TRY(launch_batch_init(bqs(h), m, bhdr(h), st));
    QueryArgs al = a;
    if (h->learned) {
        int32_t* lv = reinterpret_cast<int32_t*>(h->bws + h->bp.leaves);
        paris_status ls = mlp_top_leaves_of_queries(h->model, sb.Q, m, h->n, lv, st);
        if (ls != PARIS_OK) return ls;
        sb.leaves = lv;
        al.learned_cpl = learned_chunks(h);
    }
    HIP_TRY(launch_prepare_seed_batch(al, sb, m, st));
    HIP_TRY(launch_batch_thresholds(bqs(h), m, h->c_screen, h->seed_rel, h->proj, st));
    if (timed) HIP_TRY(hipEventRecord(h->bev[1], st));
    const ScreenArgs sa = screen_args(h, m, nullptr);
    HIP_TRY(launch_block_mask(sa, h->screen, st));
    if (timed) HIP_TRY(hipEventRecord(h->bev[2], st));
    HIP_TRY(launch_screen(sa, h->np, h->screen, st));
    if (timed) HIP_TRY(hipEventRecord(h->bev[3], st));
    const RescoreArgs r = rescore_args(h, m);
    HIP_TRY(launch_rescore(r, st));
    if (timed) HIP_TRY(hipEventRecord(h->bev[4], st));
    HIP_TRY(launch_batch_resolve(r, reinterpret_cast<long long*>(h->bws + h->bp.oidx),
                                 reinterpret_cast<double*>(h->bws + h->bp.odist), st));
    if (timed) HIP_TRY(hipEventRecord(h->bev[5], st));
    return PARIS_OK;
}

// Capture the full-size pipeline once into a HIP graph (on a private stream).
paris_status capture_batch_graph(paris_index* h)
{
    hipStream_t cs = nullptr;
    HIP_TRY(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
    paris_status s = PARIS_OK;
    if (hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal) != hipSuccess) s = PARIS_EHIP;
    if (s == PARIS_OK) {
        paris_status ls = launch_batch_pipeline(h, h->max_batch, cs);
        hipGraph_t g = nullptr;
        if (hipStreamEndCapture(cs, &g) != hipSuccess || ls != PARIS_OK) s = PARIS_EHIP;
        if (s == PARIS_OK && hipGraphInstantiate(&h->graph_exec, g, nullptr, nullptr, 0) != hipSuccess)
            s = PARIS_EHIP;
        if (s == PARIS_OK) h->graph = g;
        else if (g) (void)hipGraphDestroy(g);
    }
    (void)hipStreamDestroy(cs);
    return s;
}

paris_status run_batch_chunk(paris_index* h, const float* queries, long long q0, int m, long long* out_idx,
                             double* out_dist, hipStream_t st, long long* cands, long long* fallbacks,
                             long long* rescored)
{
    const size_t qbytes = (size_t)m * h->n * 4;
    HIP_TRY(hipMemcpyAsync(h->bws + h->bp.qin, queries + q0 * h->n, qbytes, hipMemcpyDeviceToDevice, st));
    const bool timed = h->timing && h->bev[0];
    if (m == h->max_batch && h->graph_exec && !timed) {
        HIP_TRY(hipGraphLaunch(h->graph_exec, st));
    } else {
        paris_status s = launch_batch_pipeline(h, m, st, timed);
        if (s != PARIS_OK) return s;
    }
    HIP_TRY(hipMemcpyAsync(out_idx + q0, h->bws + h->bp.oidx, (size_t)m * 8, hipMemcpyDeviceToDevice, st));
    HIP_TRY(hipMemcpyAsync(out_dist + q0, h->bws + h->bp.odist, (size_t)m * 8, hipMemcpyDeviceToDevice, st));
    HIP_TRY(hipMemcpyAsync(h->host_hdr, bhdr(h), sizeof(BatchHdr), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    if (timed) {
        for (int k = 0; k < 5; ++k) {
            float ms = 0.f;
            HIP_TRY(hipEventElapsedTime(&ms, h->bev[k], h->bev[k + 1]));
            h->batch_ms[k] += ms;
        }
        h->timed_chunks += 1;
    }
    const BatchHdr hd = *h->host_hdr;
    *cands += hd.n_cand;
    *rescored += hd.n_rescored;
    {
        const long long xb = screen_item_series(h->screen);
        h->tiles_run += hd.n_tiles;
        h->tiles_dense += (h->N + xb - 1) / xb * ((m + h->screen.qt - 1) / h->screen.qt);
    }
    if (hd.n_fallback) {
        // queries whose screen candidates or resolve band overflowed: the per-query path
        HIP_TRY(hipMemcpyAsync(h->host_fb, h->bws + h->bp.fb, (size_t)hd.n_fallback * 4, hipMemcpyDeviceToHost, st));
        HIP_TRY(hipStreamSynchronize(st));
        for (uint32_t k = 0; k < hd.n_fallback; ++k) {
            const long long qi = q0 + h->host_fb[k];
            paris_status s = run_query(h, queries + qi * h->n, st, out_idx, out_dist, qi, false);
            if (s != PARIS_OK) return s;
        }
        *fallbacks += hd.n_fallback;
    }
    return PARIS_OK;
}

// Screen autotuner: MFMA form (16x16x32 or 32x32x16) x query-tile height (32 or 64 rows) x
// series per wave, every threshold at +inf (no candidate) and every pair screened (no block
// bound: before the first batch there are no thresholds to bound against), timed over
// full-size batches; the median of three runs decides. PARIS_SCREEN_SHAPE="qt,subs[,mfma[,blocks
// per CU]]" overrides. More than 256 dimensions always take the 32-wide form with one subtile per wave.
paris_status tune_screen(paris_index* h, hipStream_t st)
{
    const char* env = std::getenv("PARIS_SCREEN_SHAPE");
    int cus = 256, dev = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        cus = 256;
    if (h->np > 256) {   // one form serves more than 256 dimensions
        h->screen = ScreenShape{32, cus * 2, 1, 32};
        return PARIS_OK;
    }
    if (env) {
        int qt = 0, subs = 0, mf = 16, per_cu = 0;
        const int got = std::sscanf(env, "%d,%d,%d,%d", &qt, &subs, &mf, &per_cu);
        if (per_cu < 0 || per_cu > 8) per_cu = 0;
        if (got >= 2 && mf == 16 && (qt == 32 || qt == 64) && (subs == 2 || subs == 4)) {
            h->screen = ScreenShape{qt, cus * (per_cu ? per_cu : (subs == 2 ? 2 : 1)), subs, 16};
            return PARIS_OK;
        }
        if (got >= 3 && mf == 32 && (qt == 32 || qt == 64) && (subs == 1 || subs == 2)) {
            h->screen = ScreenShape{qt, cus * (per_cu ? per_cu : (qt * subs > 64 ? 1 : 2)), subs, 32};
            return PARIS_OK;
        }
    }
    const int m = h->max_batch;
    const long long variant = 2LL * m + (h->block_lb ? 1 : 0);
    {
        int v[4];
        if (tune_cache_get("screen", h->np, floor_log2(h->N), variant, v)) {
            const bool ok16 = v[3] == 16 && (v[0] == 32 || v[0] == 64) && (v[2] == 2 || v[2] == 4) && !h->block_lb;
            const bool ok32 = v[3] == 32 && (v[0] == 32 || v[0] == 64) && (v[2] == 1 || v[2] == 2);
            if ((ok16 || ok32) && v[1] >= 1 && v[1] <= 8) {
                h->screen = ScreenShape{v[0], cus * v[1], v[2], v[3]};
                return PARIS_OK;
            }
        }
    }
    HIP_TRY(hipMemsetAsync(h->bws + h->bp.qb, 0, (size_t)m * h->np * 2, st));
    hipEvent_t e0, e1;
    HIP_TRY(hipEventCreate(&e0));
    HIP_TRY(hipEventCreate(&e1));
    float best = 1e30f;
    ScreenShape pick{32, cus * 2, 2, 32};
    const ScreenShape cands[] = {{32, cus * 2, 2, 16}, {64, cus * 2, 2, 16}, {32, cus, 4, 16}, {64, cus, 4, 16},
                                 {32, cus * 2, 2, 32}, {64, cus * 2, 1, 32}, {32, cus * 2, 1, 32}};
    for (const ScreenShape& sh : cands) {
        if (h->block_lb && sh.mfma != 32) continue;   // the block bound needs the 32-wide form
        float t[3];
        for (int r = 0; r < 4; ++r) {
            HIP_TRY(launch_batch_init(bqs(h), m, bhdr(h), st));  // thresholds +inf
            HIP_TRY(hipEventRecord(e0, st));
            HIP_TRY(launch_screen(screen_args(h, m, nullptr, false), h->np, sh, st));
            HIP_TRY(hipEventRecord(e1, st));
            HIP_TRY(hipEventSynchronize(e1));
            float ms = 0.f;
            HIP_TRY(hipEventElapsedTime(&ms, e0, e1));
            if (r > 0) t[r - 1] = ms;
        }
        const float lo = std::fmin(t[0], std::fmin(t[1], t[2])), hi = std::fmax(t[0], std::fmax(t[1], t[2]));
        const float med = t[0] + t[1] + t[2] - lo - hi;
        if (med < best) { best = med; pick = sh; }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    h->screen = pick;
    const int v[4] = {pick.qt, pick.grid / cus, pick.subs, pick.mfma};
    tune_cache_put("screen", h->np, floor_log2(h->N), variant, v);
    return PARIS_OK;
}

void release_batch(paris_index* h)
{
    if (h->graph_exec) (void)hipGraphExecDestroy(h->graph_exec);
    if (h->graph) (void)hipGraphDestroy(h->graph);
    if (h->host_hdr) (void)hipHostFree(h->host_hdr);
    if (h->host_fb) (void)hipHostFree(h->host_fb);
    h->graph_exec = nullptr;
    h->graph = nullptr;
    h->host_hdr = nullptr;
    h->host_fb = nullptr;
    h->bws = nullptr;
    h->screen_ok = false;
}

// All queries of one collection: chunks of max_batch through the batched pipeline, or one by one
// through the per-query path when no batch workspace is attached. Counters are added to *agg.
paris_status batch_core(paris_index* h, const float* queries_dev, long long n_queries, int64_t* nn_index_dev,
                        double* nn_dist_dev, bool want_stats, paris_stats* agg, hipStream_t st)
{
    if (batch_screen_usable(h)) {
        long long cands = 0, fallbacks = 0, rescored = 0;
        for (long long q0 = 0; q0 < n_queries; q0 += h->max_batch) {
            const int m = (int)((n_queries - q0) < h->max_batch ? (n_queries - q0) : h->max_batch);
            paris_status s = run_batch_chunk(h, queries_dev, q0, m, reinterpret_cast<long long*>(nn_index_dev),
                                             nn_dist_dev, st, &cands, &fallbacks, &rescored);
            if (s != PARIS_OK) return s;
        }
        h->batch_candidates += cands;
        agg->lb_survivors += cands;
        agg->refined += rescored;
        agg->resolved += fallbacks;
        return PARIS_OK;
    }
    for (long long i = 0; i < n_queries; ++i) {
        const float* q = queries_dev + i * (long long)h->n;
        paris_status s = run_query(h, q, st, reinterpret_cast<long long*>(nn_index_dev), nn_dist_dev, i, false);
        if (s != PARIS_OK) return s;
        if (want_stats) {
            HIP_TRY(hipMemcpyAsync(&h->host_qs->res, &reinterpret_cast<QState*>(h->ws + h->plan.qs)->res,
                                   sizeof(QResult), hipMemcpyDeviceToHost, st));
            HIP_TRY(hipStreamSynchronize(st));
            paris_stats one;
            fill_stats(h->host_qs->res, &one);
            agg->lb_survivors += one.lb_survivors;
            agg->refined += one.refined;
            agg->abandoned += one.abandoned;
            agg->bsf_updates += one.bsf_updates;
            agg->resolved += one.resolved;
            agg->words_read += one.words_read;
        }
    }
    return PARIS_OK;
}

}  // namespace

extern "C" {

paris_status paris_batch_workspace_size(const paris_index* h, int32_t max_batch, size_t* bytes)
{
    if (!handle_ok(h)) return PARIS_ESTATE;
    if (!bytes || max_batch < 1 || max_batch > 65536) return PARIS_EINVAL;
    paris_index tmp = *h;
    make_batch_plan(&tmp, max_batch);
    *bytes = tmp.bp.total;
    return PARIS_OK;
}

paris_status paris_batch_attach(paris_index* h, void* workspace_dev, size_t workspace_bytes, int32_t max_batch,
                                void* hip_stream)
{
    if (!handle_ok(h)) return PARIS_ESTATE;
    if (!workspace_dev || max_batch < 1 || max_batch > 65536 ||
        reinterpret_cast<uintptr_t>(workspace_dev) % kAlign != 0)
        return PARIS_EINVAL;
    paris_index tmp = *h;
    make_batch_plan(&tmp, max_batch);
    if (workspace_bytes < tmp.bp.total) return PARIS_ENOMEM;
    hipStream_t st = reinterpret_cast<hipStream_t>(hip_stream);
    release_batch(h);
    h->bp = tmp.bp;
    h->bws = static_cast<uint8_t*>(workspace_dev);
    h->bws_bytes = workspace_bytes;
    h->max_batch = max_batch;
    if (hipHostMalloc(reinterpret_cast<void**>(&h->host_hdr), sizeof(BatchHdr), hipHostMallocDefault) != hipSuccess ||
        hipHostMalloc(reinterpret_cast<void**>(&h->host_fb), (size_t)max_batch * 4, hipHostMallocDefault) != hipSuccess) {
        release_batch(h);
        return PARIS_EHIP;
    }
    // the screen keeps a wave's series fragments in registers: up to 512 dimensions (longer
    // series are screened on segment means)
    h->screen_ok = h->np <= 512;
    if (!h->screen_ok) return PARIS_OK;  // batches then use the per-query path
    paris_status s = PARIS_OK;
    const char* blb = std::getenv("PARIS_BLOCK_LB");
    h->block_lb = !(blb && blb[0] == '0');
    h->tiles_run = h->tiles_dense = 0;
    if (launch_to_bf16(h->X, reinterpret_cast<const uint32_t*>(h->ws + h->plan.perm), h->N, h->n, h->np, h->proj,
                       reinterpret_cast<uint16_t*>(h->bws + h->bp.xb), reinterpret_cast<float*>(h->bws + h->bp.xn),
                       st) != hipSuccess ||
        launch_xn_max(reinterpret_cast<const float*>(h->bws + h->bp.xn), h->N, bhdr(h), st) != hipSuccess)
        s = PARIS_EHIP;
    if (s == PARIS_OK) s = tune_screen(h, st);
    if (s == PARIS_OK && hipStreamSynchronize(st) != hipSuccess) s = PARIS_EHIP;
    if (s == PARIS_OK && std::getenv("PARIS_NO_GRAPH") == nullptr) s = capture_batch_graph(h);
    if (s != PARIS_OK) release_batch(h);
    return s;
}

paris_status paris_screen_dots(paris_index* h, const float* queries_dev, int32_t n_queries, float* dots_dev,
                               void* hip_stream)
{
    if (!handle_ok(h)) return PARIS_ESTATE;
    if (!h->bws || !h->screen_ok) return PARIS_ESTATE;
    if (!queries_dev || !dots_dev || n_queries < 1 || n_queries > h->max_batch ||
        reinterpret_cast<uintptr_t>(queries_dev) % 16 != 0)
        return PARIS_EINVAL;
    hipStream_t st = reinterpret_cast<hipStream_t>(hip_stream);
    const int m = n_queries;
    const QueryArgs a = args_for(h);
    SeedBatch sb;
    sb.Q = reinterpret_cast<const float*>(h->bws + h->bp.qin);
    sb.bq = bqs(h);
    sb.qb = reinterpret_cast<uint16_t*>(h->bws + h->bp.qb);
    sb.np = h->np;
    sb.P = h->proj;
    sb.leaves = nullptr;
    sb.qpaa = reinterpret_cast<double*>(h->bws + h->bp.qpaa);
    HIP_TRY(hipMemcpyAsync(h->bws + h->bp.qin, queries_dev, (size_t)m * h->n * 4, hipMemcpyDeviceToDevice, st));
    HIP_TRY(launch_batch_init(bqs(h), m, bhdr(h), st));
    HIP_TRY(launch_prepare_seed_batch(a, sb, m, st));  // bfloat16 queries and norms (thresholds stay +inf)
    HIP_TRY(launch_screen(screen_args(h, m, dots_dev), h->np, h->screen, st));
    HIP_TRY(hipStreamSynchronize(st));
    return PARIS_OK;
}

paris_status paris_block_bound_bits(paris_index* h, const float* queries_dev, const float* sqdist_dev,
                                    int32_t n_queries, int32_t item_series, uint64_t* bits_dev, void* hip_stream)
{
    if (!handle_ok(h)) return PARIS_ESTATE;
    if (!h->bws || !h->screen_ok) return PARIS_ESTATE;
    if (!queries_dev || !sqdist_dev || !bits_dev || n_queries < 1 || n_queries > h->max_batch ||
        (item_series != 128 && item_series != 256) || reinterpret_cast<uintptr_t>(queries_dev) % 16 != 0)
        return PARIS_EINVAL;
    hipStream_t st = reinterpret_cast<hipStream_t>(hip_stream);
    const int m = n_queries;
    const QueryArgs a = args_for(h);
    SeedBatch sb;
    sb.Q = reinterpret_cast<const float*>(h->bws + h->bp.qin);
    sb.bq = bqs(h);
    sb.qb = reinterpret_cast<uint16_t*>(h->bws + h->bp.qb);
    sb.np = h->np;
    sb.P = h->proj;
    sb.leaves = nullptr;
    sb.qpaa = reinterpret_cast<double*>(h->bws + h->bp.qpaa);
    HIP_TRY(hipMemcpyAsync(h->bws + h->bp.qin, queries_dev, (size_t)m * h->n * 4, hipMemcpyDeviceToDevice, st));
    HIP_TRY(launch_batch_init(bqs(h), m, bhdr(h), st));
    HIP_TRY(launch_prepare_seed_batch(a, sb, m, st));   // query PAA (and a seed, replaced below)
    HIP_TRY(launch_set_bsf(bqs(h), sqdist_dev, m, st));
    ScreenArgs s = screen_args(h, m, nullptr, true);
    s.mask = reinterpret_cast<unsigned long long*>(bits_dev);
    HIP_TRY(launch_block_mask(s, ScreenShape{32, 0, item_series / 128, 32}, st));
    HIP_TRY(hipStreamSynchronize(st));
    return PARIS_OK;
}

paris_status paris_batch_screen_tiles(paris_index* h, int64_t* tiles_run, int64_t* tiles_dense, int32_t reset)
{
    if (!handle_ok(h)) return PARIS_ESTATE;
    if (!tiles_run || !tiles_dense) return PARIS_EINVAL;
    *tiles_run = h->tiles_run;
    *tiles_dense = h->tiles_dense;
    if (reset) h->tiles_run = h->tiles_dense = 0;
    return PARIS_OK;
}

paris_status paris_default_config(paris_config* cfg)
{
    if (!cfg) return PARIS_EINVAL;
    std::memset(cfg, 0, sizeof(*cfg));
    cfg->segments = 16;
    cfg->card_bits = 8;
    cfg->leaf_mode = PARIS_LEAF_ROOT16;
    cfg->n_leaves = 4096;
    cfg->seed_cap = 16384;
    cfg->leaf_cap = 2048;
    return PARIS_OK;
}

paris_status paris_workspace_size(int64_t n_series, int32_t length, const paris_config* cfg, size_t* bytes)
{
    if (!bytes || !config_ok(cfg) || !shape_ok(n_series, length)) return PARIS_EINVAL;
    Plan p;
    make_plan(n_series, &p, cfg);
    *bytes = p.total;
    return PARIS_OK;
}

paris_status paris_build(const float* series_dev, int64_t n_series, int32_t length, const paris_config* cfg,
                         void* workspace_dev, size_t workspace_bytes, void* hip_stream, paris_index** out)
{
    if (!out || !series_dev || !workspace_dev || !config_ok(cfg) || !shape_ok(n_series, length))
        return PARIS_EINVAL;
    if (reinterpret_cast<uintptr_t>(series_dev) % 16 != 0 ||
        reinterpret_cast<uintptr_t>(workspace_dev) % kAlign != 0)
        return PARIS_EINVAL;
    Plan plan;
    make_plan(n_series, &plan, cfg);
    if (workspace_bytes < plan.total) return PARIS_ENOMEM;
    paris_status ds = device_ok();
    if (ds != PARIS_OK) return ds;

    hipStream_t st = reinterpret_cast<hipStream_t>(hip_stream);
    uint8_t* ws = static_cast<uint8_t*>(workspace_dev);
    uint32_t* err = reinterpret_cast<uint32_t*>(ws + plan.hdr);
    auto* keys = reinterpret_cast<unsigned long long*>(ws + plan.keys);
    auto* perm = reinterpret_cast<uint32_t*>(ws + plan.perm);
    HIP_TRY(hipMemsetAsync(err, 0, 256, st));
    HIP_TRY(launch_summarise(series_dev, n_series, length, ws + plan.sax, keys, perm, err, st));
    HIP_TRY(launch_sort_keys(keys, perm, reinterpret_cast<unsigned long long*>(ws + plan.keys_alt),
                             reinterpret_cast<uint32_t*>(ws + plan.perm_alt),
                             reinterpret_cast<uint32_t*>(ws + plan.hist), n_series, st));
    HIP_TRY(launch_root_offsets(keys, n_series, reinterpret_cast<uint32_t*>(ws + plan.roff), st));
    long long tree_nodes = 0, tree_max_leaf = 0;
    if (cfg->leaf_mode == PARIS_LEAF_ADS) {
        paris_status ts = build_tree(plan, ws, n_series, cfg->leaf_cap, st, &tree_nodes, &tree_max_leaf);
        if (ts != PARIS_OK) return ts;
        HIP_TRY(launch_tree_keys(ws + plan.sax, perm, n_series, keys, st));
    }
    HIP_TRY(launch_gather_sax(ws + plan.sax, perm, n_series, ws + plan.saxs, st));
    HIP_TRY(launch_block_env(ws + plan.saxs, n_series, ws + plan.env, st));
    uint32_t herr = 0;
    HIP_TRY(hipMemcpyAsync(&herr, err, 4, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    if (herr & kErrNonFinite) return PARIS_EINVAL;

    paris_index* h = new (std::nothrow) paris_index();
    if (!h) return PARIS_ENOMEM;
    h->magic = kMagic;
    if (hipGetDevice(&h->device) != hipSuccess) h->device = 0;
    h->X = series_dev;
    h->N = n_series;
    h->n = length;
    h->cfg = *cfg;
    h->ws = ws;
    h->ws_bytes = workspace_bytes;
    h->plan = plan;
    h->mg = margins_for_length(length);
    h->scan = ScanShape{512, 2, 2};
    h->refine_blocks = kRefineBlocks;
    if (const char* rb = std::getenv("PARIS_REFINE_BLOCKS")) {
        const int v = std::atoi(rb);
        if (v >= 16 && v <= 4096) h->refine_blocks = v;
    }
    h->refine_lanes = 8;
    if (const char* rl = std::getenv("PARIS_REFINE_LANES")) {
        const int v = std::atoi(rl);
        if (v == 4 || v == 8 || v == 16) h->refine_lanes = v;
    }
    h->scan_online = 0;
    h->scan_decide = false;
    for (int k = 0; k < kScanCands * kTunePer; ++k) h->tune_ev[k][0] = h->tune_ev[k][1] = nullptr;
    h->bsf_private = 1;   // measured faster on the GPU; paris_set_bsf_sharing(h, 1) for ParIS+'s
    h->timing = false;
    h->timing_mode = 0;
    for (int set = 0; set < 2; ++set) {
        for (int k = 0; k < 4; ++k) h->ev[set][k] = nullptr;
        h->ev_pending[set] = false;
    }
    h->ev_set = 0;
    for (int k = 0; k < 3; ++k) h->phase_ms[k] = 0.0;
    h->timed_queries = 0;
    h->host_qs = nullptr;
    h->host_res = nullptr;
    h->host_res_dev = nullptr;
    h->bws = nullptr;
    h->bws_bytes = 0;
    h->max_batch = 0;
    h->proj = 1;
    while (length / h->proj > 512 || length % h->proj != 0) ++h->proj;   // n / P <= 512 dimensions
    h->np = (length / h->proj + 31) / 32 * 32;
    h->screen_ok = false;
    std::memset(&h->bp, 0, sizeof(h->bp));
    h->screen = ScreenShape{64, 0, 4, 16};
    h->c_screen = screen_margin(length / h->proj, h->np);
    // the seed series' exact squared distance is at most d32 (1 + g) / (1 - g) < d32 (1 + 3 g)
    h->seed_rel = 3.0 * gamma_k(length + 2) + std::ldexp(1.0, -30);
    h->graph = nullptr;
    h->graph_exec = nullptr;
    h->host_hdr = nullptr;
    h->host_fb = nullptr;
    h->batch_candidates = 0;
    for (int k = 0; k < 6; ++k) h->bev[k] = nullptr;
    for (int k = 0; k < 5; ++k) h->batch_ms[k] = 0.0;
    h->timed_chunks = 0;
    h->model = nullptr;
    h->learned = false;
    h->n_tree_nodes = tree_nodes;
    h->tree_max_leaf = tree_max_leaf;
    if (hipHostMalloc(reinterpret_cast<void**>(&h->host_qs), sizeof(QState), hipHostMallocDefault) != hipSuccess ||
        hipHostMalloc(reinterpret_cast<void**>(&h->host_res), kHostResBytes, hipHostMallocMapped) != hipSuccess ||
        hipHostGetDevicePointer(reinterpret_cast<void**>(&h->host_res_dev), h->host_res, 0) != hipSuccess) {
        if (h->host_qs) (void)hipHostFree(h->host_qs);
        if (h->host_res) (void)hipHostFree(h->host_res);
        delete h;
        return PARIS_EHIP;
    }
    h->host_knn = reinterpret_cast<KnnHit*>(reinterpret_cast<uint8_t*>(h->host_res) + 256);
    h->host_knn_dev = reinterpret_cast<KnnHit*>(reinterpret_cast<uint8_t*>(h->host_res_dev) + 256);
    const QueryArgs a = args_for(h);
    paris_status ts = PARIS_OK;
    if (launch_reset(a, st) != hipSuccess) ts = PARIS_EHIP;
    const bool cached = std::getenv("PARIS_SCAN_SHAPE") == nullptr && scan_from_cache(h);
    if (ts == PARIS_OK && !cached) ts = tune_scan(h, st);
    if (ts == PARIS_OK && !cached && std::getenv("PARIS_SCAN_SHAPE") == nullptr) {
        // the build's choice (on a threshold of 0) is refined on the first real queries
        bool ok = true;
        for (int k = 0; k < kScanCands * kTunePer && ok; ++k)
            ok = hipEventCreate(&h->tune_ev[k][0]) == hipSuccess && hipEventCreate(&h->tune_ev[k][1]) == hipSuccess;
        if (ok) h->scan_online = kTunePer;
    }
    if (ts != PARIS_OK) {
        (void)hipHostFree(h->host_qs);
        (void)hipHostFree(h->host_res);
        delete h;
        return ts;
    }
    {
        std::lock_guard<std::mutex> g(g_live_mu);
        g_live.insert(h);
    }
    *out = h;
    return PARIS_OK;
}

paris_status paris_host_alloc(size_t bytes, void** host_ptr, void** dev_ptr)
{
    if (!host_ptr || !dev_ptr || bytes == 0) return PARIS_EINVAL;
    paris_status ds = device_ok();
    if (ds != PARIS_OK) return ds;
    void* hp = nullptr;
    if (hipHostMalloc(&hp, bytes, hipHostMallocMapped) != hipSuccess || !hp) return PARIS_ENOMEM;
    void* dp = nullptr;
    if (hipHostGetDevicePointer(&dp, hp, 0) != hipSuccess || !dp) {
        (void)hipHostFree(hp);
        return PARIS_EHIP;
    }
    *host_ptr = hp;
    *dev_ptr = dp;
    return PARIS_OK;
}

paris_status paris_host_free(void* host_ptr)
{
    if (!host_ptr) return PARIS_OK;
    return hipHostFree(host_ptr) == hipSuccess ? PARIS_OK : PARIS_EHIP;
}

paris_status paris_get_layout(const paris_index* h, paris_layout* o)
{
    if (!handle_ok(h)) return PARIS_ESTATE;
    if (!o) return PARIS_EINVAL;
    *o = paris_layout{};
    o->sax_dev = h->ws + h->plan.sax;
    o->keys_dev = reinterpret_cast<const uint64_t*>(h->ws + h->plan.keys);
    o->perm_dev = reinterpret_cast<const uint32_t*>(h->ws + h->plan.perm);
    o->roff_dev = reinterpret_cast<const uint32_t*>(h->ws + h->plan.roff);
    o->n_series = h->N;
    o->length = h->n;
    o->leaf_mode = h->cfg.leaf_mode;
    o->n_leaves = h->cfg.n_leaves;
    o->seed_cap = h->cfg.seed_cap;
    o->scan_threads = h->scan.threads;
    o->scan_blocks_per_cu = h->scan.per_cu;
    o->scan_unroll = h->scan.unroll;
    if (h->screen_ok) {
        int cus = 256, dev = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
            cus = 256;
        o->screen_rows = h->screen.qt;
        o->screen_blocks_per_cu = h->screen.grid / cus;
        o->screen_subtiles = h->screen.subs;
        o->screen_mfma = h->screen.mfma;
    }
    const bool tree = h->cfg.leaf_mode == PARIS_LEAF_ADS;
    o->tree_nodes_dev = tree ? static_cast<const void*>(h->ws + h->plan.tree) : nullptr;
    o->n_tree_nodes = tree ? h->n_tree_nodes : 0;
    o->tree_max_leaf = tree ? h->tree_max_leaf : 0;
    return PARIS_OK;
}

}  // extern "C"

namespace {

// Waits for the result of the query just launched on st (it lands in the index's mapped host
// buffer) and copies it out.
paris_status finish_query(paris_index* h, hipStream_t st, int64_t* nn_index, double* nn_dist, paris_stats* stats)
{
    volatile long long* flag = &h->host_res->idx;
    // The result lands in mapped host memory: wait for it there (a stream synchronisation costs
    // a few microseconds more). Every 1024 polls the stream is asked whether it failed or
    // drained without producing the result.
    for (unsigned it = 1;; ++it) {
        if (*flag != -2) break;
        if ((it & 1023u) == 0u) {
            const hipError_t e = hipStreamQuery(st);
            if (e == hipSuccess) break;          // drained: the flag is read once more below
            if (e != hipErrorNotReady) return PARIS_EHIP;
        }
        __builtin_ia32_pause();
    }
    std::atomic_thread_fence(std::memory_order_acquire);
    const QResult r = *h->host_res;
    if (r.idx == -2) return PARIS_EHIP;
    if (r.err & kErrNonFinite) return PARIS_EINVAL;
    if (r.err & (kErrSurvOverflow | kErrDoneOverflow)) return PARIS_EOVERFLOW;
    if (r.idx < 0) return PARIS_EINVAL;
    *nn_index = r.idx;
    *nn_dist = std::sqrt(r.d2);
    if (stats) fill_stats(r, stats);
    return PARIS_OK;
}

}  // namespace

extern "C" {

paris_status paris_query_exact(paris_index* h, const float* query_dev, int64_t* nn_index, double* nn_dist,
                               paris_stats* stats, void* hip_stream)
{
    if (!handle_ok(h)) return PARIS_ESTATE;
    if (!query_dev || !nn_index || !nn_dist || reinterpret_cast<uintptr_t>(query_dev) % 16 != 0)
        return PARIS_EINVAL;
    hipStream_t st = reinterpret_cast<hipStream_t>(hip_stream);
    *reinterpret_cast<volatile long long*>(&h->host_res->idx) = -2;  // the resolve writes it last
    const bool timed = h->timing && (h->timing_mode != 3 || (h->timing_calls++ % kTimingEvery) == 0);
    paris_status s = run_query(h, query_dev, st, nullptr, nullptr, 0, timed, h->host_res_dev);
    if (s != PARIS_OK) return s;
    return finish_query(h, st, nn_index, nn_dist, stats);
}

}  // extern "C"

// ---- exact k-NN --------------------------------------------------------------------------
namespace {
// seed distances per answer (PARIS_KNN_SEED overrides, 1 .. 16)
int knn_seed_per_answer()
{
    if (const char* e = std::getenv("PARIS_KNN_SEED")) {
        const int v = std::atoi(e);
        if (v >= 1 && v <= 16) return v;
    }
    return 8;   // measured at 10M x 256 over 1, 2, 4, 8 and 16 (k = 10 and 64)
}
}  // namespace

extern "C" paris_status paris_query_knn(paris_index* h, const float* query_dev, int32_t k, int64_t* nn_index,
                             double* nn_dist, int32_t* n_found, paris_stats* stats, void* hip_stream)
{
    if (!handle_ok(h)) return PARIS_ESTATE;
    if (!query_dev || !nn_index || !nn_dist || !n_found || k < 1 || k > kKnnMax ||
        reinterpret_cast<uintptr_t>(query_dev) % 16 != 0)
        return PARIS_EINVAL;
    hipStream_t st = reinterpret_cast<hipStream_t>(hip_stream);
    if (k == 1) {   // the 1-NN search itself
        paris_status s1 = paris_query_exact(h, query_dev, nn_index, nn_dist, stats, hip_stream);
        if (s1 == PARIS_OK) *n_found = 1;
        return s1;
    }
    QueryArgs a = args_for(h);
    a.host_res = h->host_res_dev;
    a.knn_k = k;
    a.knn_out = h->host_knn_dev;
    const paris_mlp* m = h->learned ? h->model : nullptr;
    if (m) {
        a.leaf_keys = m->partq;
        a.leaf_key_count = (m->n_out + 255) / 256 * kTopLeaves;
        a.learned_cpl = learned_chunks(h);
    }
    // seed distances per answer: the smallest-bound members of every chunk of the approximate
    // search's window(s), kKnnSeedPerAnswer * k of them spread over its chunks
    a.knn_r = knn_seed_per_answer();
    *reinterpret_cast<volatile long long*>(&h->host_res->idx) = -2;
    HIP_TRY(launch_knn_reset(a, st));
    if (m) {
        MlpQueryScratch sc{m->partq};
        HIP_TRY(launch_mlp_query(net_of(m), query_dev, h->n, sc, st));
    }
    HIP_TRY(launch_prepare_seed(a, query_dev, st));
    HIP_TRY(launch_knn_select(a, st));
    HIP_TRY(launch_lbscan(a, -1.f, h->scan, st));
    HIP_TRY(launch_refine_resolve(a, query_dev, nullptr, nullptr, 0, st));
    int64_t top_i = -1;
    double top_d = 0.0;
    paris_status s = finish_query(h, st, &top_i, &top_d, stats);
    if (s != PARIS_OK) return s;
    const QResult r = *h->host_res;
    const int found = (int)(r.n_resolved < (uint32_t)k ? r.n_resolved : (uint32_t)k);
    for (int j = 0; j < found; ++j) {
        nn_index[j] = h->host_knn[j].idx;
        nn_dist[j] = std::sqrt(h->host_knn[j].d2);
    }
    *n_found = found;
    return PARIS_OK;
}

// ---- allocation-free per-query entry point ----------------------------------------------
// The per-query scratch of paris_query_exact_noalloc lives in one file-scope device array per
// GPU (the code object's copy on that device), never allocated or freed by any call.
namespace {
constexpr size_t na_align(size_t v) { return (v + 255) & ~(size_t)255; }
constexpr size_t kNaSurvCap = (size_t)PARIS_NOALLOC_MAX_SURVIVORS;
constexpr size_t kNaDoneCap = (size_t)PARIS_NOALLOC_MAX_COMPLETED;
constexpr size_t kNaQs = 0;
constexpr size_t kNaT8 = na_align(kNaQs + sizeof(QState));
constexpr size_t kNaSurv = na_align(kNaT8 + (size_t)kSeg * kSym * 4);
constexpr size_t kNaDone = na_align(kNaSurv + kNaSurvCap * 8);
constexpr size_t kNaBytes = na_align(kNaDone + kNaDoneCap * 8);
static_assert(kNaBytes <= ((size_t)20 << 20), "the allocation-free scratch stays below 20 MiB");
}  // namespace

static __device__ __align__(256) uint8_t scratch[kNaBytes];

namespace {
constexpr int kNaMaxDevices = 64;
std::mutex g_na_mu;
uint8_t* g_na_ptr[kNaMaxDevices] = {};   // device address of `scratch` on each GPU

// Device address of this GPU's copy of the scratch array (looked up once per device, with that
// device current; the array's host-side name is not a device address).
paris_status noalloc_scratch(int dev, uint8_t** out)
{
    if (dev < 0 || dev >= kNaMaxDevices) return PARIS_ENODEV;
    std::lock_guard<std::mutex> g(g_na_mu);
    if (!g_na_ptr[dev]) {
        void* p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return PARIS_EHIP;
        g_na_ptr[dev] = static_cast<uint8_t*>(p);
    }
    *out = g_na_ptr[dev];
    return PARIS_OK;
}
}  // namespace

extern "C" {

paris_status paris_query_exact_noalloc(paris_index* h, const float* query_dev, int64_t* nn_index,
                                       double* nn_dist, paris_stats* stats, void* hip_stream)
{
    if (!handle_ok(h)) return PARIS_ESTATE;
    if (!query_dev || !nn_index || !nn_dist || reinterpret_cast<uintptr_t>(query_dev) % 16 != 0)
        return PARIS_EINVAL;
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess) return PARIS_EHIP;
    if (dev != h->device) return PARIS_EINVAL;   // the index's device must be current
    uint8_t* base = nullptr;
    paris_status ps = noalloc_scratch(dev, &base);
    if (ps != PARIS_OK) return ps;
    QueryScratch sc;
    sc.qs = reinterpret_cast<QState*>(base + kNaQs);
    sc.t8 = reinterpret_cast<float*>(base + kNaT8);
    sc.surv = reinterpret_cast<uint2*>(base + kNaSurv);
    sc.surv_cap = (uint32_t)kNaSurvCap;
    sc.done = reinterpret_cast<uint2*>(base + kNaDone);
    sc.done_cap = (uint32_t)kNaDoneCap;
    hipStream_t st = reinterpret_cast<hipStream_t>(hip_stream);
    *reinterpret_cast<volatile long long*>(&h->host_res->idx) = -2;
    paris_status s = run_query(h, query_dev, st, nullptr, nullptr, 0, false, h->host_res_dev, &sc);
    if (s != PARIS_OK) return s;
    return finish_query(h, st, nn_index, nn_dist, stats);
}

paris_status paris_query_batch(paris_index* h, const float* queries_dev, int64_t n_queries, int64_t* nn_index_dev,
                               double* nn_dist_dev, paris_stats* stats, void* hip_stream)
{
    if (!handle_ok(h)) return PARIS_ESTATE;
    if (!queries_dev || !nn_index_dev || !nn_dist_dev || n_queries < 0 ||
        reinterpret_cast<uintptr_t>(queries_dev) % 16 != 0)
        return PARIS_EINVAL;
    paris_stats agg;
    std::memset(&agg, 0, sizeof(agg));
    paris_status s = batch_core(h, queries_dev, n_queries, nn_index_dev, nn_dist_dev, stats != nullptr, &agg,
                                reinterpret_cast<hipStream_t>(hip_stream));
    if (s != PARIS_OK) return s;
    if (stats) {
        agg.seed_index = -1;
        agg.seed_dist = INFINITY;
        *stats = agg;
    }
    return PARIS_OK;
}

paris_status paris_query_batch_multi(paris_index* const* idx, int32_t n_idx, const float* const* queries_dev,
                                     const int64_t* n_queries, int64_t* const* nn_index_dev,
                                     double* const* nn_dist_dev, paris_stats* stats, void* hip_stream)
{
    if (!idx || n_idx < 1 || !queries_dev || !n_queries || !nn_index_dev || !nn_dist_dev) return PARIS_EINVAL;
    for (int32_t c = 0; c < n_idx; ++c) {
        if (!handle_ok(idx[c])) return PARIS_ESTATE;
        for (int32_t d = 0; d < c; ++d)
            if (idx[d] == idx[c]) return PARIS_EINVAL;   // one in-flight call per handle
        if (n_queries[c] < 0) return PARIS_EINVAL;
        if (n_queries[c] > 0 && (!queries_dev[c] || !nn_index_dev[c] || !nn_dist_dev[c] ||
                                 reinterpret_cast<uintptr_t>(queries_dev[c]) % 16 != 0))
            return PARIS_EINVAL;
    }
    hipStream_t st = reinterpret_cast<hipStream_t>(hip_stream);
    paris_stats agg;
    std::memset(&agg, 0, sizeof(agg));
    for (int32_t c = 0; c < n_idx; ++c) {
        if (n_queries[c] == 0) continue;
        paris_status s = batch_core(idx[c], queries_dev[c], n_queries[c], nn_index_dev[c], nn_dist_dev[c],
                                    stats != nullptr, &agg, st);
        if (s != PARIS_OK) return s;
    }
    if (stats) {
        agg.seed_index = -1;
        agg.seed_dist = INFINITY;
        *stats = agg;
    }
    return PARIS_OK;
}

paris_status paris_query_info_get(paris_index* h, const float* query_dev, paris_query_info* info, float* table_dev,
                                  void* hip_stream)
{
    if (!handle_ok(h)) return PARIS_ESTATE;
    if (!query_dev || reinterpret_cast<uintptr_t>(query_dev) % 16 != 0) return PARIS_EINVAL;
    hipStream_t st = reinterpret_cast<hipStream_t>(hip_stream);
    const QueryArgs a = args_for(h);
    HIP_TRY(launch_prepare_seed(a, query_dev, st));
    if (table_dev) HIP_TRY(hipMemcpyAsync(table_dev, a.t8, kSeg * kSym * 4, hipMemcpyDeviceToDevice, st));
    HIP_TRY(hipMemcpyAsync(h->host_qs, a.qs, sizeof(QState), hipMemcpyDeviceToHost, st));
    HIP_TRY(launch_reset(a, st));
    HIP_TRY(hipStreamSynchronize(st));
    const QState& q = *h->host_qs;
    if (info) {
        for (int s = 0; s < 16; ++s) { info->paa[s] = q.paa[s]; info->sym[s] = q.sym[s]; }
        info->root = q.root;
        info->pad = 0;
        info->k64 = q.k64;
        info->win_lo = q.win_lo;
        info->win_hi = q.win_hi;
    }
    if (q.err & kErrNonFinite) return PARIS_EINVAL;
    return PARIS_OK;
}

paris_status paris_lb_scan(paris_index* h, const float* query_dev, float threshold_sq, uint32_t* idx_dev,
                           float* lb_dev, int64_t capacity, int64_t* count, void* hip_stream)
{
    if (!handle_ok(h)) return PARIS_ESTATE;
    if (!query_dev || !count || capacity < 0 || (capacity > 0 && (!idx_dev || !lb_dev)) ||
        !(threshold_sq >= 0.f) || reinterpret_cast<uintptr_t>(query_dev) % 16 != 0)
        return PARIS_EINVAL;
    hipStream_t st = reinterpret_cast<hipStream_t>(hip_stream);
    QueryArgs a = args_for(h);
    if (h->timing) {
        paris_status ps = collect_pending(h);
        if (ps != PARIS_OK) return ps;
    }
    HIP_TRY(launch_prepare_seed(a, query_dev, st));
    HIP_TRY(launch_lbscan(a, threshold_sq, h->scan, st, h->timing ? h->ev[0][1] : nullptr,
                          h->timing ? h->ev[0][2] : nullptr));
    HIP_TRY(hipMemcpyAsync(h->host_qs, a.qs, sizeof(QState), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    const QState& q = *h->host_qs;
    const long long n = q.n_surv;
    const uint32_t qerr = q.err;
    if (h->timing) {  // the scan alone is added to phase [1]
        float ms = 0.f;
        HIP_TRY(hipEventElapsedTime(&ms, h->ev[0][1], h->ev[0][2]));
        h->phase_ms[1] += ms;
        h->timed_queries += 1;
    }
    const long long k = n < capacity ? n : capacity;
    if (k > 0) {
        // survivors are (index, bound) pairs in the survivor buffer; split them for the caller
        HIP_TRY(hipMemcpy2DAsync(idx_dev, 4, a.surv, 8, 4, (size_t)k, hipMemcpyDeviceToDevice, st));
        HIP_TRY(hipMemcpy2DAsync(lb_dev, 4, reinterpret_cast<uint8_t*>(a.surv) + 4, 8, 4, (size_t)k,
                                 hipMemcpyDeviceToDevice, st));
    }
    HIP_TRY(launch_reset(a, st));
    HIP_TRY(hipStreamSynchronize(st));
    if (qerr & kErrNonFinite) return PARIS_EINVAL;
    *count = n;
    return n > capacity ? PARIS_EOVERFLOW : PARIS_OK;
}

paris_status paris_set_bsf_sharing(paris_index* h, int32_t shared)
{
    if (!handle_ok(h)) return PARIS_ESTATE;
    if (shared != 0 && shared != 1) return PARIS_EINVAL;
    h->bsf_private = shared ? 0 : 1;
    return PARIS_OK;
}

paris_status paris_set_timing(paris_index* h, int32_t enable)
{
    if (!handle_ok(h)) return PARIS_ESTATE;
    if (enable < 0 || enable > 3) return PARIS_EINVAL;
    if (enable && !h->ev[0][0]) {
        for (int set = 0; set < 2; ++set)
            for (int k = 0; k < 4; ++k) HIP_TRY(hipEventCreate(&h->ev[set][k]));
        for (int k = 0; k < 6; ++k) HIP_TRY(hipEventCreate(&h->bev[k]));
    }
    h->timing = enable != 0;
    h->timing_mode = enable;
    h->timing_calls = 0;
    h->ev_pending[0] = h->ev_pending[1] = false;
    h->ev_set = 0;
    for (int k = 0; k < 3; ++k) h->phase_ms[k] = 0.0;
    h->timed_queries = 0;
    for (int k = 0; k < 5; ++k) h->batch_ms[k] = 0.0;
    h->timed_chunks = 0;
    return PARIS_OK;
}

paris_status paris_get_batch_timing(const paris_index* h, double* ms_out5, int64_t* n_chunks)
{
    if (!handle_ok(h)) return PARIS_ESTATE;
    if (!ms_out5 || !n_chunks) return PARIS_EINVAL;
    for (int k = 0; k < 5; ++k) ms_out5[k] = h->batch_ms[k];
    *n_chunks = h->timed_chunks;
    return PARIS_OK;
}

paris_status paris_get_timing(paris_index* h, double* ms_out3, int64_t* n_queries)
{
    if (!handle_ok(h)) return PARIS_ESTATE;
    if (!ms_out3 || !n_queries) return PARIS_EINVAL;
    if (h->timing) {
        paris_status s = collect_pending(h);
        if (s != PARIS_OK) return s;
    }
    for (int k = 0; k < 3; ++k) ms_out3[k] = h->phase_ms[k];
    *n_queries = h->timed_queries;
    return PARIS_OK;
}

paris_status paris_free(paris_index* h)
{
    if (!h) return PARIS_OK;
    {
        std::lock_guard<std::mutex> g(g_live_mu);
        if (g_live.erase(h) == 0) return PARIS_ESTATE;
    }
    h->magic = 0;
    release_batch(h);
    if (h->host_qs) (void)hipHostFree(h->host_qs);
    if (h->host_res) (void)hipHostFree(h->host_res);
    for (int set = 0; set < 2; ++set)
        for (int k = 0; k < 4; ++k)
            if (h->ev[set][k]) (void)hipEventDestroy(h->ev[set][k]);
    for (int k = 0; k < 6; ++k)
        if (h->bev[k]) (void)hipEventDestroy(h->bev[k]);
    for (int k = 0; k < kScanCands * kTunePer; ++k)
        for (int e = 0; e < 2; ++e)
            if (h->tune_ev[k][e]) (void)hipEventDestroy(h->tune_ev[k][e]);
    delete h;
    return PARIS_OK;
}

// ---- learned seed -------------------------------------------------------------------------
paris_status paris_mlp_param_count(int32_t n_leaves, int64_t* count)
{
    if (!count || n_leaves < 64 || n_leaves > kMaxLeaves || n_leaves % 64 != 0) return PARIS_EINVAL;
    *count = mlp_offsets(n_leaves).total;
    return PARIS_OK;
}

}  // extern "C"

namespace {

// byte offsets of a network's arrays in its workspace (each 256-byte aligned); returns the total
struct MlpArrays {
    size_t master, wb, grad, m, v, P, H1, H2, Z, G3, G3b, G2, G2b, G1, G1b, lr, zq, total;
};

bool mlp_shape_ok(int32_t n_leaves, int32_t max_rows)
{
    return n_leaves >= 64 && n_leaves <= kMaxLeaves && n_leaves % 64 == 0 && max_rows >= 64 && max_rows <= 65536 &&
           max_rows % 64 == 0;
}

MlpArrays mlp_arrays(int32_t n_leaves, int32_t max_rows)
{
    const size_t np = (size_t)mlp_offsets(n_leaves).total, R = (size_t)max_rows, no = (size_t)n_leaves, H = kMlpHid;
    MlpArrays a{};
    size_t off = 0;
    auto take = [&off](size_t bytes) { const size_t at = off; off = align_up(off + bytes); return at; };
    a.master = take(np * 4);
    a.wb = take(np * 2);
    a.grad = take(np * 4);
    a.m = take(np * 4);
    a.v = take(np * 4);
    a.P = take(R * kMlpIn * 4);
    a.H1 = take(R * H * 2);
    a.H2 = take(R * H * 2);
    a.Z = take(R * no * 4);
    a.G3 = take(R * no * 4);
    a.G3b = take(R * no * 2);
    a.G2 = take(R * H * 4);
    a.G2b = take(R * H * 2);
    a.G1 = take(R * H * 4);
    a.G1b = take(R * H * 2);
    a.lr = take(R * 4);
    a.zq = take((no / 256 + 1) * kTopLeaves * 8);
    a.total = off;
    return a;
}

}  // namespace

extern "C" {

paris_status paris_mlp_workspace_size(int32_t n_leaves, int32_t max_rows, int64_t* bytes)
{
    if (!bytes || !mlp_shape_ok(n_leaves, max_rows)) return PARIS_EINVAL;
    *bytes = (int64_t)mlp_arrays(n_leaves, max_rows).total;
    return PARIS_OK;
}

paris_status paris_mlp_create(int32_t n_leaves, int32_t max_rows, void* workspace_dev, int64_t workspace_bytes,
                              paris_mlp** out)
{
    if (!out || !mlp_shape_ok(n_leaves, max_rows) || !workspace_dev) return PARIS_EINVAL;
    if (reinterpret_cast<uintptr_t>(workspace_dev) % kAlign != 0) return PARIS_EINVAL;
    const MlpArrays a = mlp_arrays(n_leaves, max_rows);
    if (workspace_bytes < (int64_t)a.total) return PARIS_EINVAL;
    paris_status ds = device_ok();
    if (ds != PARIS_OK) return ds;
    paris_mlp* m = new (std::nothrow) paris_mlp();
    if (!m) return PARIS_ENOMEM;
    m->magic = kMagic + 1;
    if (hipGetDevice(&m->device) != hipSuccess) m->device = 0;
    m->n_out = n_leaves;
    m->max_rows = max_rows;
    m->off = mlp_offsets(n_leaves);
    m->step = 0;
    m->mem = static_cast<uint8_t*>(workspace_dev);
    uint8_t* b = m->mem;
    m->master = reinterpret_cast<float*>(b + a.master);
    m->wb = reinterpret_cast<uint16_t*>(b + a.wb);
    m->grad = reinterpret_cast<float*>(b + a.grad);
    m->am = reinterpret_cast<float*>(b + a.m);
    m->av = reinterpret_cast<float*>(b + a.v);
    m->P = reinterpret_cast<float*>(b + a.P);
    m->H1 = reinterpret_cast<uint16_t*>(b + a.H1);
    m->H2 = reinterpret_cast<uint16_t*>(b + a.H2);
    m->Z = reinterpret_cast<float*>(b + a.Z);
    m->G3 = reinterpret_cast<float*>(b + a.G3);
    m->G3b = reinterpret_cast<uint16_t*>(b + a.G3b);
    m->G2 = reinterpret_cast<float*>(b + a.G2);
    m->G2b = reinterpret_cast<uint16_t*>(b + a.G2b);
    m->G1 = reinterpret_cast<float*>(b + a.G1);
    m->G1b = reinterpret_cast<uint16_t*>(b + a.G1b);
    m->loss_row = reinterpret_cast<float*>(b + a.lr);
    m->partq = reinterpret_cast<unsigned long long*>(b + a.zq);
    // all-zero parameters and moments until the caller sets parameters
    if (hipMemset(m->mem, 0, a.total) != hipSuccess || hipDeviceSynchronize() != hipSuccess) {
        delete m;
        return PARIS_EHIP;
    }
    {
        std::lock_guard<std::mutex> g(g_mlp_mu);
        g_mlp_live.insert(m);
    }
    *out = m;
    return PARIS_OK;
}

paris_status paris_mlp_set_params(paris_mlp* m, const float* params_dev, void* hip_stream)
{
    if (!mlp_ok(m)) return PARIS_ESTATE;
    if (!params_dev) return PARIS_EINVAL;
    hipStream_t st = reinterpret_cast<hipStream_t>(hip_stream);
    const size_t np = (size_t)m->off.total;
    HIP_TRY(hipMemcpyAsync(m->master, params_dev, np * 4, hipMemcpyDeviceToDevice, st));
    HIP_TRY(hipMemsetAsync(m->am, 0, np * 4, st));
    HIP_TRY(hipMemsetAsync(m->av, 0, np * 4, st));
    HIP_TRY(launch_mirror(m->master, m->wb, (long long)np, st));
    m->step = 0;
    return PARIS_OK;
}

paris_status paris_mlp_get_params(const paris_mlp* m, float* params_dev, void* hip_stream)
{
    if (!mlp_ok(m)) return PARIS_ESTATE;
    if (!params_dev) return PARIS_EINVAL;
    HIP_TRY(hipMemcpyAsync(params_dev, m->master, (size_t)m->off.total * 4, hipMemcpyDeviceToDevice,
                           reinterpret_cast<hipStream_t>(hip_stream)));
    return PARIS_OK;
}

paris_status paris_query_features(const float* queries_dev, int64_t n_queries, int32_t length, float* features_dev,
                                  void* hip_stream)
{
    if (!queries_dev || !features_dev || n_queries < 0 || length < 16 || length > kMaxLength || length % 16 != 0)
        return PARIS_EINVAL;
    HIP_TRY(launch_paa_features(queries_dev, n_queries, n_queries, length, features_dev,
                                reinterpret_cast<hipStream_t>(hip_stream)));
    return PARIS_OK;
}

paris_status paris_mlp_forward(paris_mlp* m, const float* features_dev, int64_t rows, float* logits_dev,
                               void* hip_stream)
{
    if (!mlp_ok(m)) return PARIS_ESTATE;
    if (!features_dev || !logits_dev || rows < 0) return PARIS_EINVAL;
    hipStream_t st = reinterpret_cast<hipStream_t>(hip_stream);
    for (long long r0 = 0; r0 < rows; r0 += m->max_rows) {
        const int rr = (int)(rows - r0 < m->max_rows ? rows - r0 : m->max_rows);
        paris_status s = mlp_forward_rows(m, features_dev + r0 * kMlpIn, nullptr, rr, st);
        if (s != PARIS_OK) return s;
        HIP_TRY(hipMemcpyAsync(logits_dev + r0 * m->n_out, m->Z, (size_t)rr * m->n_out * 4, hipMemcpyDeviceToDevice, st));
    }
    return PARIS_OK;
}

paris_status paris_mlp_top_leaves(paris_mlp* m, const float* features_dev, int64_t rows, int32_t* leaves_dev,
                                  void* hip_stream)
{
    if (!mlp_ok(m)) return PARIS_ESTATE;
    if (!features_dev || !leaves_dev || rows < 0) return PARIS_EINVAL;
    hipStream_t st = reinterpret_cast<hipStream_t>(hip_stream);
    for (long long r0 = 0; r0 < rows; r0 += m->max_rows) {
        const int rr = (int)(rows - r0 < m->max_rows ? rows - r0 : m->max_rows);
        paris_status s = mlp_forward_rows(m, features_dev + r0 * kMlpIn, nullptr, rr, st);
        if (s != PARIS_OK) return s;
        HIP_TRY(launch_topk(m->Z, rr, m->n_out, kTopLeaves, leaves_dev + r0 * kTopLeaves, st));
    }
    return PARIS_OK;
}

paris_status paris_mlp_grad(paris_mlp* m, const float* features_dev, const int32_t* labels_dev,
                            const int32_t* rows_sel_dev, int64_t rows, float* grad_dev, float* loss_dev,
                            void* hip_stream)
{
    if (!mlp_ok(m)) return PARIS_ESTATE;
    if (!features_dev || !labels_dev || !grad_dev || rows < 1 || rows > m->max_rows) return PARIS_EINVAL;
    hipStream_t st = reinterpret_cast<hipStream_t>(hip_stream);
    paris_status s = mlp_grad_rows(m, features_dev, labels_dev, rows_sel_dev, (int)rows, loss_dev, st);
    if (s != PARIS_OK) return s;
    HIP_TRY(hipMemcpyAsync(grad_dev, m->grad, (size_t)m->off.total * 4, hipMemcpyDeviceToDevice, st));
    return PARIS_OK;
}

paris_status paris_mlp_train_step(paris_mlp* m, const float* features_dev, const int32_t* labels_dev,
                                  const int32_t* rows_sel_dev, int64_t rows, const paris_adam* opt,
                                  float* loss_dev, void* hip_stream)
{
    if (!mlp_ok(m)) return PARIS_ESTATE;
    if (!features_dev || !labels_dev || !adam_ok(opt) || rows < 1 || rows > m->max_rows) return PARIS_EINVAL;
    hipStream_t st = reinterpret_cast<hipStream_t>(hip_stream);
    paris_status s = mlp_grad_rows(m, features_dev, labels_dev, rows_sel_dev, (int)rows, loss_dev, st);
    if (s != PARIS_OK) return s;
    return mlp_adam(m, m->grad, *opt, st);
}

paris_status paris_mlp_apply(paris_mlp* m, const float* grad_dev, const paris_adam* opt, void* hip_stream)
{
    if (!mlp_ok(m)) return PARIS_ESTATE;
    if (!grad_dev || !adam_ok(opt)) return PARIS_EINVAL;
    return mlp_adam(m, grad_dev, *opt, reinterpret_cast<hipStream_t>(hip_stream));
}

paris_status paris_mlp_free(paris_mlp* m)
{
    if (!m) return PARIS_OK;
    {
        std::lock_guard<std::mutex> g(g_mlp_mu);
        if (g_mlp_live.erase(m) == 0) return PARIS_ESTATE;
    }
    {
        // indexes still pointing at this network fall back to the plain seed
        std::lock_guard<std::mutex> g(g_live_mu);
        for (const paris_index* hc : g_live) {
            paris_index* h = const_cast<paris_index*>(hc);
            if (h->model == m) {
                h->model = nullptr;
                h->learned = false;
                if (h->graph_exec) {
                    (void)hipGraphExecDestroy(h->graph_exec);
                    h->graph_exec = nullptr;
                }
                if (h->graph) {
                    (void)hipGraphDestroy(h->graph);
                    h->graph = nullptr;
                }
            }
        }
    }
    m->magic = 0;
    (void)hipDeviceSynchronize();   // the workspace goes back to its owner idle
    delete m;
    return PARIS_OK;
}

paris_status paris_leaf_of(const paris_index* h, const int64_t* series_dev, int64_t count, int32_t* leaves_dev,
                           void* hip_stream)
{
    if (!handle_ok(h)) return PARIS_ESTATE;
    if (h->cfg.leaf_mode != PARIS_LEAF_EQUAL_COUNT) return PARIS_EINVAL;
    if (!series_dev || !leaves_dev || count < 0) return PARIS_EINVAL;
    const QueryArgs a = args_for(h);
    HIP_TRY(launch_leaf_of(a.sax, a.keys, a.perm, h->N, h->cfg.n_leaves, reinterpret_cast<const long long*>(series_dev),
                           count, leaves_dev, reinterpret_cast<hipStream_t>(hip_stream)));
    return PARIS_OK;
}

paris_status paris_set_seed_model(paris_index* h, paris_mlp* m, int32_t enabled)
{
    if (!handle_ok(h)) return PARIS_ESTATE;
    if (m && !mlp_ok(m)) return PARIS_ESTATE;
    if (enabled && !m) return PARIS_EINVAL;
    if (m && (h->cfg.leaf_mode != PARIS_LEAF_EQUAL_COUNT || h->cfg.n_leaves != m->n_out || m->device != h->device))
        return PARIS_EINVAL;
    const bool was = h->learned;
    h->model = m;
    h->learned = enabled != 0 && m != nullptr;
    if (h->graph_exec && (was != h->learned || h->learned)) {
        // the captured batch pipeline changes with the seed: capture it again
        (void)hipGraphExecDestroy(h->graph_exec);
        h->graph_exec = nullptr;
        if (h->graph) (void)hipGraphDestroy(h->graph);
        h->graph = nullptr;
        if (std::getenv("PARIS_NO_GRAPH") == nullptr) return capture_batch_graph(h);
    }
    return PARIS_OK;
}

const char* paris_status_string(paris_status s)
{
    switch (s) {
    case PARIS_OK: return "ok";
    case PARIS_EINVAL: return "invalid argument or non-finite value";
    case PARIS_ENOMEM: return "workspace too small";
    case PARIS_ENODEV: return "no HIP device";
    case PARIS_EHIP: return "HIP runtime error";
    case PARIS_EOVERFLOW: return "device buffer overflow";
    case PARIS_ESTATE: return "invalid handle";
    }
    return "unknown status";
}

}  // extern "C"
