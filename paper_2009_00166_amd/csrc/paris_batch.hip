// Batched exact 1-NN (many queries per launch): per-query lower-bound-guided seeds, a dense
// bfloat16 MFMA screen of every (query, series) pair with a certified error margin, float32
// re-scoring of the screen's survivors with early abandoning, and the float64 resolve.
//
// Screen. The squared distance is ||q||^2 + ||x||^2 - 2 q.x; q.x over all pairs is a dense
// contraction (queries x dimensions x series) computed with v_mfma_f32_16x16x32_bf16 on
// round-to-nearest bfloat16 copies of q and x, float32 accumulation. With u_b = 2^-8 the
// bfloat16 products are within (2 u_b + u_b^2) sum_j |q_j x_j| <= (2 u_b + u_b^2)(qn + xn)/2 of
// q.x; the float32 accumulation and the float32 norms add gamma-terms of the same form. So
// |d~^2 - d^2| <= E = c (qn + xn) with c set on the host (screen_margin). A series is kept for
// query q iff d~^2 - E <= U_q, where U_q is an upper bound on the nearest squared distance (the
// seed's distance, rounded up). The nearest neighbour and every series tied with it always pass.
// The test is folded into per-row and per-column constants: keep iff
//     dot >= a_q + b_x,  a_q = ((1 - c) qn - U_q) / 2,  b_x = (1 - c) xn / 2
// (both rounded down, c inflated for the evaluation of the test itself). The constants enter
// the contraction itself through one extra k-step: the query row carries [hi, lo, 1, 1] and the
// series row [1, 1, hi', lo'], where hi + lo >= -a_q and hi' + lo' >= -b_x are pairs of
// bfloat16 values (hi rounded down, the exact float32 remainder rounded up: bias_pair), so
// every accumulator ends as dot - a_q - b_x or more, within about 2^-16 relative of it, and a
// series survives iff its accumulator is >= 0.
#include <type_traits>

#include "paris_internal.h"

namespace paris {

// Gaussian region boundaries beta_1..beta_255 (index 0 unused): the k/256 quantiles of N(0,1).
static __constant__ double c_beta[256] = {
    0.0,
#include "breakpoints.inc"
};

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

__device__ __forceinline__ uint16_t to_bf16(float f)
{
    const uint32_t b = __float_as_uint(f);
    return (uint16_t)((b + 0x7FFFu + ((b >> 16) & 1u)) >> 16);
}

// bfloat16 of a finite float32, rounded toward +inf
__device__ __forceinline__ uint16_t to_bf16_up(float f)
{
    const uint32_t b = __float_as_uint(f);
    uint32_t h = b >> 16;
    if ((b & 0xFFFFu) != 0u && !(b >> 31)) h += 1u;  // positive with dropped bits: away from 0
    return (uint16_t)h;                               // negative: truncation is toward +inf
}

__device__ __forceinline__ float key_dist_b(unsigned long long k) { return __uint_as_float((uint32_t)(k >> 32)); }

__device__ __forceinline__ unsigned long long pack_key_b(float d2, uint32_t idx)
{
    return ((unsigned long long)__float_as_uint(d2) << 32) | idx;
}

constexpr float kNoPass = -1.0e30f;  // bias of absent rows / columns: never >= 0
constexpr int kCandStage = 512;      // screen candidates staged per block in LDS
constexpr int kRescoreBlocks = 2048;  // re-score blocks (8 per CU: latency-bound row reads)
constexpr int kHeadBlocks = 1024;     // head-pass blocks (one lane per candidate test)

// bfloat16 of a finite float32, rounded toward -inf
__device__ __forceinline__ uint16_t to_bf16_down(float f)
{
    const uint32_t b = __float_as_uint(f);
    uint32_t h = b >> 16;
    if ((b & 0xFFFFu) != 0u && (b >> 31)) h += 1u;  // negative with dropped bits: away from 0
    return (uint16_t)h;
}

// A bias t as two bfloat16 terms hi + lo >= t: hi = t rounded down (t - hi is then exact in
// float32 and non-negative), lo = that remainder rounded up. Packed as [hi, lo].
__device__ __forceinline__ uint2 bias_pair(float t)
{
    const uint16_t hi = to_bf16_down(t);
    const float rem = t - __uint_as_float((uint32_t)hi << 16);
    const uint16_t lo = to_bf16_up(rem);
    return make_uint2((uint32_t)hi | ((uint32_t)lo << 16), 0u);
}

// ------------------------------------------------------------------------------------------
// Collection -> zero-padded bfloat16 rows [N][np] and float32 squared norms (one wave per row).
// ------------------------------------------------------------------------------------------
// Series longer than the screen's 512 dimensions are screened on their segment means over
// segments of P points (P the smallest divisor of n with n / P <= 512): for the mean vectors p,
// P ||p_q - p_x||^2 <= ||q - x||^2 (Cauchy-Schwarz on every segment), so the projected distance
// is a lower bound and pruning on it stays exact; the threshold is divided by P instead of
// scaling the vectors (k_batch_thresholds). P = 1 is the series itself.
__device__ __forceinline__ float seg_mean(const float* __restrict__ x, int j, int P)
{
    if (P == 1) return x[j];
    double acc = 0.0;
    for (int i = 0; i < P; ++i) acc = acc + (double)x[j * P + i];
    return (float)(acc / (double)P);
}

// Element offset of dimension d of row p in the bfloat16 copy. Rows are stored in fragment
// order: blocks of 32 rows, each a run of np / 16 k-steps of 64 lanes x 8 values, lane
// 32 h + c holding dimensions 16 s + 8 h .. + 7 of row 32 b + c. That is the B operand of
// v_mfma_f32_32x32x16_bf16 for k-step s of the 32 series of block b, so the screen reads a
// wave's series fragments with loads of 1 KiB contiguous; 8 consecutive dimensions of a row
// (a 16-byte chunk starting at a multiple of 8) stay contiguous for the 16-wide form.
__host__ __device__ __forceinline__ long long xb_off(long long p, int d, int np)
{
    return ((((p >> 5) * (np >> 4) + (d >> 4)) * 64) + ((d >> 3) & 1) * 32 + (p & 31)) * 8 + (d & 7);
}

// Row p of the copy is series perm[p] (leaf order), so that a run of consecutive rows shares
// long iSAX prefixes and the block bound of the screen (k_block_mask) stays tight.
__global__ __launch_bounds__(256) void k_to_bf16(const float* __restrict__ X, const uint32_t* __restrict__ perm,
                                                 long long N, int n, int np, int P,
                                                 uint16_t* __restrict__ Xb, float* __restrict__ xn)
{
    const int lane = threadIdx.x & 63;
    const long long wave = ((long long)blockIdx.x * 256 + threadIdx.x) >> 6;
    const long long nw = (long long)gridDim.x * 4;
    const int nd = n / P;
    for (long long i = wave; i < N; i += nw) {
        const float* row = X + (long long)perm[i] * n;
        float sq = 0.f;
        for (int j = lane; j < np; j += 64) {
            const float v = j < nd ? seg_mean(row, j, P) : 0.f;
            Xb[xb_off(i, j, np)] = to_bf16(v);
            sq += v * v;
        }
        for (int off = 32; off > 0; off >>= 1) sq += __shfl_xor(sq, off);
        if (lane == 0) xn[i] = sq;
    }
}

hipError_t launch_to_bf16(const float* X, const uint32_t* perm, long long N, int n, int np, int P, uint16_t* Xb,
                          float* xn, hipStream_t st)
{
    long long blocks = (N + 3) / 4;
    if (blocks > 65536) blocks = 65536;
    k_to_bf16<<<(unsigned)blocks, 256, 0, st>>>(X, perm, N, n, np, P, Xb, xn);
    return hipGetLastError();
}

// ------------------------------------------------------------------------------------------
// Block bound of the screen.
// Every series of a run of consecutive sorted positions has, in each segment, a symbol between
// the run's smallest and largest symbol of that segment, so its PAA value lies in the union of
// those regions. The distance from the query's PAA value to that union is at most the distance
// to the series' own region, and the iSAX lower bound (Section 3.3.1: L times the sum over the
// 16 segments of the squared distance from the query mean to the region) built from it is at
// most the bound of every series of the run, hence at most their Euclidean distances. A (query,
// run) pair whose block bound exceeds the query's threshold U_q holds no series that the screen
// would have to keep: the screen skips it.
// ------------------------------------------------------------------------------------------
// Symbol envelope of every run of kEnvRun sorted positions: bytes 0..15 the smallest symbol of
// each segment, bytes 16..31 the largest. One wave per run: lane l reads the 8 symbols of
// segments 8 (l / 32) .. +7 of position l % 32 of the run.
__global__ __launch_bounds__(256) void k_block_env(const uint8_t* __restrict__ saxs, long long N,
                                                   uint8_t* __restrict__ env)
{
    const int lane = threadIdx.x & 63, half = lane >> 5;
    const long long runs = (N + kEnvRun - 1) / kEnvRun;
    const long long run = ((long long)blockIdx.x * 256 + threadIdx.x) >> 6;
    if (run >= runs) return;   // whole waves leave together
    const long long p = run * kEnvRun + (lane & 31);
    uint32_t mn[8], mx[8];
    const uint2 v = p < N ? *reinterpret_cast<const uint2*>(saxs + p * 16 + half * 8) : make_uint2(0u, 0u);
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        const uint32_t b = ((k < 4 ? v.x : v.y) >> (8 * (k & 3))) & 0xFFu;
        mn[k] = p < N ? b : 255u;
        mx[k] = p < N ? b : 0u;
    }
#pragma unroll
    for (int o = 1; o < 32; o <<= 1) {
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            mn[k] = min(mn[k], (uint32_t)__shfl_xor((int)mn[k], o));
            mx[k] = max(mx[k], (uint32_t)__shfl_xor((int)mx[k], o));
        }
    }
    if ((lane & 31) == 0) {
        uint2 lo = make_uint2(0u, 0u), hi = make_uint2(0u, 0u);
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            lo.x |= mn[k] << (8 * k);
            lo.y |= mn[k + 4] << (8 * k);
            hi.x |= mx[k] << (8 * k);
            hi.y |= mx[k + 4] << (8 * k);
        }
        *reinterpret_cast<uint2*>(env + run * 32 + half * 8) = lo;
        *reinterpret_cast<uint2*>(env + run * 32 + 16 + half * 8) = hi;
    }
}

hipError_t launch_block_env(const uint8_t* saxs, long long N, uint8_t* env, hipStream_t st)
{
    const long long runs = (N + kEnvRun - 1) / kEnvRun;
    const long long blocks = (runs + 3) / 4;
    k_block_env<<<(unsigned)blocks, 256, 0, st>>>(saxs, N, env);
    return hipGetLastError();
}

// Alive bits of every (work item of XB sorted positions, query): bit q % 64 of word
// item * ceil(M / 64) + q / 64 is set unless the item's block bound provably exceeds
// V_q = U_q (1 + seed_rel)(1 + prune_rel) (U_q the seed's squared distance, as in
// k_batch_thresholds before any projection). A query without a threshold (non-finite, or no
// seed) has no bits. One thread per query (so a wave ballot is one word); a block takes
// kMaskItems items, whose envelopes it merges and stages in LDS.
//
// Arithmetic in float32, certified: region edges rounded outward (lower edge down, upper edge
// up), the query's float64 segment means rounded to nearest (error at most u |p_s|, u = 2^-24),
// gaps and their squares and the 16-term sum rounded to nearest. Then the computed bound B~
// satisfies B~ <= (1 + e)(sqrt(B) + u sqrt(A))^2 (Cauchy-Schwarz on the cross term), with B
// the exact bound over the widened intervals (at most the envelope's bound, hence at most
// every member's distance), A = L sum_s p_s^2 and e = 24 u for the products, the sum and the
// factor L. A pair is dropped only when B~ > T_q = RU((1 + e)(sqrt(V_q) + u sqrt(A))^2),
// which implies B > V_q.
constexpr int kMaskItems = 64;

__global__ __launch_bounds__(256) void k_block_mask(ScreenArgs Sa, int XB)
{
    __shared__ double beta[257];
    __shared__ float s_lo[kMaskItems][kSeg], s_hi[kMaskItems][kSeg];
    const int tid = threadIdx.x, lane = tid & 63;
    const int M = Sa.M, words = (M + 63) >> 6;
    const long long N = Sa.N;
    const long long n_items = (N + XB - 1) / XB;
    const long long it0 = (long long)blockIdx.x * kMaskItems;
    const long long runs = (N + kEnvRun - 1) / kEnvRun;
    const int rpi = XB / kEnvRun;
    if (tid == 0) { beta[0] = -__builtin_inf(); beta[256] = __builtin_inf(); }
    if (tid >= 1) beta[tid] = c_beta[tid];
    __syncthreads();
    for (int e = tid; e < kMaskItems * kSeg; e += 256) {
        const int ii = e >> 4, sg = e & 15;
        const long long item = it0 + ii;
        uint32_t mn = 255u, mx = 0u;
        for (int r = 0; r < rpi; ++r) {
            const long long run = item * rpi + r;
            if (item < n_items && run < runs) {
                mn = min(mn, (uint32_t)Sa.env[run * 32 + sg]);
                mx = max(mx, (uint32_t)Sa.env[run * 32 + 16 + sg]);
            }
        }
        s_lo[ii][sg] = __double2float_rd(beta[mn]);       // lower edge of the smallest symbol, rounded down
        s_hi[ii][sg] = __double2float_ru(beta[mx + 1]);   // upper edge of the largest symbol, rounded up
    }
    const int q = blockIdx.y * 256 + tid;
    float pq[kSeg];
    float thr = -1.f;   // no bit
#pragma unroll
    for (int sg = 0; sg < kSeg; ++sg) pq[sg] = 0.f;
    if (q < M) {
        const BQuery& b = Sa.bq[q];
        if (!b.err && b.bsf_key != kBsfInit) {
            double A = 0.0;
#pragma unroll
            for (int sg = 0; sg < kSeg; ++sg) {
                const double p = Sa.qpaa[(long long)q * kSeg + sg];
                pq[sg] = (float)p;
                A = A + p * p;
            }
            A = A * Sa.seg_len;
            const double u = 0x1p-24;
            const double V = ((double)key_dist_b(b.bsf_key) * (1.0 + Sa.seed_rel) + 1e-20) * (1.0 + Sa.prune_rel);
            const double r = sqrt(V) * (1.0 + 2.0 * u) + u * sqrt(A) * (1.0 + 2.0 * u);
            thr = __double2float_ru((1.0 + 24.0 * u) * r * r * (1.0 + 4.0 * u));
        }
    }
    const float L = (float)Sa.seg_len;
    __syncthreads();
    const int word = (blockIdx.y * 256 + (tid & ~63)) >> 6;
    for (int ii = 0; ii < kMaskItems; ++ii) {
        const long long item = it0 + ii;
        if (item >= n_items) break;   // uniform
        float acc = 0.f;
#pragma unroll
        for (int sg = 0; sg < kSeg; ++sg) {
            const float g = fmaxf(fmaxf(s_lo[ii][sg] - pq[sg], pq[sg] - s_hi[ii][sg]), 0.f);
            acc = fmaf(g, g, acc);
        }
        const bool alive = thr >= 0.f && acc * L <= thr;
        const unsigned long long bits = __ballot(alive);
        if (lane == 0 && word < words) Sa.mask[item * words + word] = bits;
    }
}

// ------------------------------------------------------------------------------------------
// Per-batch reset (a fill kernel, so the sequence can be captured in a graph).
// ------------------------------------------------------------------------------------------
__global__ void k_batch_init(BQuery* __restrict__ bq, int M, BatchHdr* __restrict__ hdr)
{
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q < M) {
        BQuery& b = bq[q];
        b.bsf_key = kBsfInit;
        b.qn = 0.f;
        b.a = __builtin_inff();
        b.n_band = 0;
        b.err = 0;
        b.ub = 0u;   // largest survivor accumulator (bits) until k_query_ub
        b.u_lo = 0.f;
    }
    if (q == 0) {
        hdr->next_item = 0;
        hdr->n_cand = 0;
        hdr->n_fallback = 0;
        hdr->flags = 0;
        hdr->n_tiles = 0;
        hdr->n_rescored = 0;
    }
}

// Screen threshold constant of every query from its seed (U_q = seed distance rounded up, in
// units of the screened vectors: divided by the segment length P of a projected screen).
__global__ void k_batch_thresholds(BQuery* __restrict__ bq, int M, float c_screen, double seed_rel, int P)
{
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= M) return;
    BQuery& b = bq[q];
    if (b.err || b.bsf_key == kBsfInit) { b.a = __builtin_inff(); return; }  // nothing to screen
    double U = (double)key_dist_b(b.bsf_key) * (1.0 + seed_rel) + 1e-20;
    if (P > 1) U = U / (double)P * (1.0 + 0x1p-50);
    const double a = ((1.0 - (double)c_screen) * (double)b.qn - U) * 0.5;
    b.a = __double2float_rd(a);
    b.u_lo = __double2float_rd(U);
}

// ------------------------------------------------------------------------------------------
// The screen. Persistent blocks of 4 waves take series tiles of 256 (64 per wave) from an
// atomic work counter. A wave keeps its 64 series' bfloat16 fragments (np/32 k-steps plus the
// bias step) in registers for the whole item and streams every query tile (QT queries,
// double-buffered in LDS, rows padded by 16 bytes so the 16 rows read by a quarter-wave hit
// distinct banks) through v_mfma_f32_16x16x32_bf16: per k-step QT/16 x 4 MFMAs, with the next
// k-step's query operands read from LDS before the current MFMAs issue. Operand layout
// (16x16x32): lane l holds row/column (l % 16) and the 8 k-elements 8 (l / 16) .. +7 of the
// k-step, for both A (queries) and B (series); the accumulator of lane l holds rows
// 4 (l / 16) + r, r = 0..3, of column l % 16. A wave takes the append path only when the
// maximum over its accumulators is >= 0 (rare).
// ------------------------------------------------------------------------------------------
template <int KS, int QT, int SUBS>
__global__ __launch_bounds__(256, SUBS == 2 ? 2 : 1) void k_screen(ScreenArgs S)
{
    constexpr int XW = 16 * SUBS;       // series per wave (kept in registers)
    constexpr int XB = 4 * XW;          // series per work item (block)
    constexpr int NP = KS * 32;
    constexpr int KT = KS + 1;          // k-steps including the bias step
    constexpr int RS = KT * 32 + 8;     // LDS row stride (bfloat16 elements)
    constexpr int QS = QT / 16;         // query subtiles per tile
    constexpr int V8 = NP / 8;          // 16-byte vectors per data row
    constexpr int STAGE = (QT * V8 + 255) / 256;
    __shared__ __attribute__((aligned(16))) uint16_t qtile[2][QT * RS];
    __shared__ long long s_item;
    // candidates are staged per block (LDS atomics) and flushed with one global atomic
    __shared__ uint2 cbuf[kCandStage];
    __shared__ uint32_t ccount, cbase;
    const int tid = threadIdx.x, w = tid >> 6, l = tid & 63;
    if (tid == 0) ccount = 0;
    auto flush_cands = [&]() {
        const uint32_t cnt = min(ccount, (uint32_t)kCandStage);
        if (tid == 0) cbase = atomicAdd(&S.hdr->n_cand, cnt);
        __syncthreads();
        for (uint32_t k = tid; k < cnt; k += 256) {
            const uint32_t pos = cbase + k;
            if (pos < S.cand_cap) S.cand[pos] = cbuf[k];
        }
        __syncthreads();
        if (tid == 0) ccount = 0;
        __syncthreads();
    };

    const int col = l & 15, kg = l >> 4;
    const int M = S.M;
    const long long N = S.N;
    const int n_qt = (M + QT - 1) / QT;
    const long long n_items = (N + XB - 1) / XB;
    const bool dump = S.dump != nullptr;

    // bias block of every row: chunk 0 = [hi(-a_q), lo(-a_q), 1, 1, 0 ...] is rewritten with
    // each tile, chunks 1..3 stay zero
    for (int e = tid; e < 2 * QT * 4; e += 256) {
        const int buf = e / (QT * 4), rem = e - buf * QT * 4, row = rem >> 2, ch = rem & 3;
        *reinterpret_cast<uint4*>(&qtile[buf][row * RS + NP + ch * 8]) = make_uint4(0, 0, 0, 0);
    }

    auto stage_load = [&](int t, uint4* pre, uint2& bias) {
#pragma unroll
        for (int s = 0; s < STAGE; ++s) {
            const int e = tid + s * 256;
            const int row = e / V8, v = e - row * V8;
            const int q = t * QT + row;
            pre[s] = (e < QT * V8 && q < M)
                         ? *reinterpret_cast<const uint4*>(S.Qb + (long long)q * NP + v * 8)
                         : make_uint4(0, 0, 0, 0);
        }
        if (tid < QT) {
            const int q = t * QT + tid;
            const float a = (q < M && !dump) ? S.bq[q].a : (dump ? 0.f : __builtin_inff());
            const float t1 = a < __builtin_inff() ? -a : kNoPass;
            bias = bias_pair(t1);  // [hi(-a_q), lo(-a_q), 1.0, 1.0]
            bias.y = 0x3F803F80u;
        }
    };
    auto stage_store = [&](int buf, const uint4* pre, uint2 bias) {
#pragma unroll
        for (int s = 0; s < STAGE; ++s) {
            const int e = tid + s * 256;
            if (e < QT * V8) {
                const int row = e / V8, v = e - row * V8;
                *reinterpret_cast<uint4*>(&qtile[buf][row * RS + v * 8]) = pre[s];
            }
        }
        if (tid < QT) *reinterpret_cast<uint2*>(&qtile[buf][tid * RS + NP]) = bias;
    };

    for (;;) {
        __syncthreads();
        if (tid == 0) s_item = (long long)atomicAdd(&S.hdr->next_item, 1u);
        __syncthreads();
        const long long item = s_item;
        if (item >= n_items) break;  // uniform: every wave reaches this exit
        const long long xb0 = item * XB + w * XW;
        if (tid == 0) atomicAdd(&S.hdr->n_tiles, (uint32_t)n_qt);

        bf16x8 bfr[SUBS][KT];
#pragma unroll
        for (int sub = 0; sub < SUBS; ++sub) {
            const long long x = xb0 + sub * 16 + col;
            const bool ok = x < N;
#pragma unroll
            for (int ks = 0; ks < KS; ++ks) {
                if (ok) bfr[sub][ks] = *reinterpret_cast<const bf16x8*>(S.Xb + xb_off(x, ks * 32 + kg * 8, NP));
                else bfr[sub][ks] = bf16x8{};
            }
            // bias step: lanes of k-group 0 carry [1, RU(-b_x), 0 ...]
            float t2 = kNoPass;
            if (ok) t2 = dump ? 0.f : -__double2float_rd((1.0 - (double)S.c_screen) * (double)S.xn[x] * 0.5);
            uint4 bb = make_uint4(0, 0, 0, 0);
            if (kg == 0) {
                bb.x = 0x3F803F80u;   // [1.0, 1.0, hi(-b_x), lo(-b_x)]
                const uint2 hl = bias_pair(t2);
                bb.y = hl.x;
            }
            bfr[sub][KS] = __builtin_bit_cast(bf16x8, bb);
        }

        {
            uint4 pre[STAGE];
            uint2 bias = make_uint2(0u, 0u);
            stage_load(0, pre, bias);
            stage_store(0, pre, bias);
        }
        __syncthreads();

        for (int t = 0; t < n_qt; ++t) {
            const int buf = t & 1;
            uint4 pre[STAGE];
            uint2 bias = make_uint2(0u, 0u);
            const bool more = t + 1 < n_qt;
            if (more) stage_load(t + 1, pre, bias);  // in flight during the MFMAs

            f32x4 acc[QS][SUBS];
#pragma unroll
            for (int qs = 0; qs < QS; ++qs)
#pragma unroll
                for (int sub = 0; sub < SUBS; ++sub) acc[qs][sub] = f32x4{0.f, 0.f, 0.f, 0.f};
            const uint16_t* tb = qtile[buf] + col * RS + kg * 8;
            bf16x8 a[QS], an[QS];
#pragma unroll
            for (int qs = 0; qs < QS; ++qs) a[qs] = *reinterpret_cast<const bf16x8*>(tb + qs * 16 * RS);
#pragma unroll
            for (int ks = 0; ks < KT; ++ks) {
                if (ks + 1 < KT) {
#pragma unroll
                    for (int qs = 0; qs < QS; ++qs)
                        an[qs] = *reinterpret_cast<const bf16x8*>(tb + qs * 16 * RS + (ks + 1) * 32);
                }
#pragma unroll
                for (int qs = 0; qs < QS; ++qs)
#pragma unroll
                    for (int sub = 0; sub < SUBS; ++sub)
                        acc[qs][sub] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[qs], bfr[sub][ks], acc[qs][sub],
                                                                               0, 0, 0);
                if (ks + 1 < KT) {
#pragma unroll
                    for (int qs = 0; qs < QS; ++qs) a[qs] = an[qs];
                }
            }

            if (dump) {
#pragma unroll
                for (int qs = 0; qs < QS; ++qs)
#pragma unroll
                    for (int sub = 0; sub < SUBS; ++sub)
#pragma unroll
                        for (int r = 0; r < 4; ++r) {
                            const int q = t * QT + qs * 16 + kg * 4 + r;
                            const long long x = xb0 + sub * 16 + col;
                            if (q < M && x < N) S.dump[(long long)q * N + (S.perm ? S.perm[x] : x)] = acc[qs][sub][r];
                        }
            } else {
                float m = kNoPass;
#pragma unroll
                for (int qs = 0; qs < QS; ++qs)
#pragma unroll
                    for (int sub = 0; sub < SUBS; ++sub)
                        m = fmaxf(m, fmaxf(fmaxf(acc[qs][sub][0], acc[qs][sub][1]),
                                           fmaxf(acc[qs][sub][2], acc[qs][sub][3])));
                const bool hit = m >= 0.f;
                if (__ballot(hit) && hit) {
#pragma unroll
                    for (int qs = 0; qs < QS; ++qs)
#pragma unroll
                        for (int sub = 0; sub < SUBS; ++sub)
#pragma unroll
                            for (int r = 0; r < 4; ++r) {
                                if (acc[qs][sub][r] >= 0.f) {
                                    const int q = t * QT + qs * 16 + kg * 4 + r;
                                    const long long x = xb0 + sub * 16 + col;
                                    if (q < M && x < N) {
                                        const uint2 c = make_uint2((uint32_t)q, S.perm ? S.perm[x] : (uint32_t)x);
                                        const uint32_t p = atomicAdd(&ccount, 1u);
                                        if (p < (uint32_t)kCandStage) {
                                            cbuf[p] = c;
                                        } else {  // more than the stage holds in one tile
                                            const uint32_t pos = atomicAdd(&S.hdr->n_cand, 1u);
                                            if (pos < S.cand_cap) S.cand[pos] = c;
                                        }
                                    }
                                }
                            }
                }
            }
            if (more) stage_store(buf ^ 1, pre, bias);
            __syncthreads();
            if (ccount >= (uint32_t)(kCandStage / 2)) flush_cands();  // uniform: read after the barrier
        }
    }
    __syncthreads();
    if (ccount) flush_cands();
}

// 16 bytes per lane from base + voffset (bytes) into LDS at lds + 8 lane (bfloat16 elements; lds
// is wave-uniform): buffer_load_dwordx4 ... lds through a raw descriptor of `bytes` bytes, so a
// read past the end returns zeros.
__device__ __forceinline__ void lds_dma16(const uint16_t* base, int bytes, int voffset, uint16_t* lds)
{
    const __amdgpu_buffer_rsrc_t rs =
        __builtin_amdgcn_make_buffer_rsrc(const_cast<uint16_t*>(base), (short)0, bytes, 0x00020000);
    __builtin_amdgcn_raw_ptr_buffer_load_lds(rs, (__attribute__((address_space(3))) void*)lds, 16, voffset, 0, 0, 0);
}

// The same screen on v_mfma_f32_32x32x16_bf16: a 32 x 32 output tile per instruction doubles
// the work per operand byte, so a query fragment read from LDS feeds twice the arithmetic of
// the 16 x 16 form. A wave holds S subtiles of 32 series (k-steps of 16, plus the bias step) in
// registers; query tiles of QT rows stream through LDS. Operand layout (32x32x16): lane l holds
// row/column (l % 32) and the 8 k-elements 8 (l / 32) .. +7 of the k-step for both A (queries)
// and B (series); accumulator element i of lane l is row 8 (i / 4) + 4 (l / 32) + i % 4, column
// l % 32. Bias step: query rows carry [hi(-a_q), lo(-a_q), 1, 1] and series rows
// [1, 1, hi(-b_x), lo(-b_x)] in k-elements 0..3, zeros elsewhere.
// Work units are (work item of 4 S 32 sorted positions, group of queries), claimed from a
// counter one ahead; a unit builds its alive list, reads its series fragments (1 KiB contiguous
// per load: the copy is in fragment order), then runs its query tiles. The register budget of
// two waves per SIMD (256) holds the S series fragment sets, the accumulators and a query
// fragment pipeline two k-steps deep with nothing live across units.
template <int KS16, int QT, int S, bool DUMP>
__global__ __launch_bounds__(256, 2) void k_screen32(ScreenArgs Sa)
{
    static_assert(S == 1 || S == 2, "one or two 32-series subtiles per wave");
    constexpr int XW = 32 * S;          // series per wave (kept in registers)
    constexpr int XB = 4 * XW;          // series per work item (block)
    constexpr int NP = KS16 * 16;
    constexpr int KT = KS16 + 1;        // k-steps including the bias step
    constexpr int QS = QT / 32;         // query subtiles per tile
    constexpr int CH = NP / 8;          // 16-byte chunks per query row
    // chunk swizzle mask: c ^ (row & SWM) must stay inside the row, so SWM + 1 divides CH
    // (CH = 2 KS16 is a multiple of 4; a multiple of 8 takes the 8-row mask)
    constexpr int SWM = CH % 8 == 0 ? 7 : 3;
    static_assert(CH % (SWM + 1) == 0, "the swizzle must permute the chunks of a row");
    constexpr int TCH = QT * CH;        // chunks per query tile
    static_assert(TCH % 64 == 0, "a wave's 64 chunk positions are all inside the tile or all past it");
    constexpr int LOADS = (TCH + 255) / 256;    // direct-to-LDS loads per lane per tile
    // queries per alive list: two blocks per CU must fit in LDS next to the two tile buffers
    constexpr int GROUP = QT * NP >= 64 * 256 ? kScreenGroup / 2 : kScreenGroup;
    static_assert(GROUP % QT == 0, "a tile never reads past the list");
    // Query tiles go from global memory straight into LDS (global_load_lds_dwordx4: no staging
    // registers, so nothing holds the MFMAs back while the next tile is in flight). A row's
    // 16-byte chunk c sits at chunk c ^ (row & SWM) of the row, so the 8 rows that one LDS cycle
    // serves hit 8 distinct bank groups. The bias columns live in their own small array.
    __shared__ __attribute__((aligned(16))) uint16_t qd0[QT * NP];
    __shared__ __attribute__((aligned(16))) uint16_t qd1[QT * NP];
    __shared__ __attribute__((aligned(16))) uint16_t qb0[QT * 16];
    __shared__ __attribute__((aligned(16))) uint16_t qb1[QT * 16];
    // queries of the current group whose block bound did not prune the item (ascending)
    __shared__ uint16_t s_list[GROUP];
    __shared__ uint32_t s_cnt;
    __shared__ long long s_item, s_next;
    __shared__ uint2 cbuf[kCandStage];
    __shared__ uint32_t ccount, cbase;
    // largest survivor accumulator of every query seen by this block (batches of at most
    // kAmaxQueries; where two blocks per CU leave LDS room for it): gives the re-score a
    // certified upper bound on the nearest distance
    constexpr int LDS_BASE = 4 * QT * NP + 64 * QT + 2 * GROUP + 8 * kCandStage + 256;   // bytes
    constexpr int AQ = LDS_BASE + 4 * kAmaxQueries <= 80 * 1024 - 512 ? kAmaxQueries : 1;
    __shared__ uint32_t s_amax[AQ];
    const int tid = threadIdx.x, l = tid & 63;
    // the wave index, known to the compiler as uniform: per-wave addresses stay in scalar registers
    const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
    if (tid == 0) ccount = 0;
    const bool track = AQ > 1 && Sa.M <= AQ && !DUMP;
    if (track)
        for (int e = tid; e < Sa.M; e += 256) s_amax[e] = 0u;
    // A candidate at list position pos: (query, series) and its accumulator truncated to the top
    // 16 bits (so at most the accumulator), from which the re-score derives distance bounds.
    // Staged entries carry (query | top 16 bits of the accumulator, sorted position).
    auto store_cand = [&](uint32_t pos, uint32_t qa, uint32_t p) __attribute__((always_inline)) {
        if (pos < Sa.cand_cap) {
            Sa.cand[pos] = make_uint2(qa & 0xFFFFu, Sa.perm ? Sa.perm[p] : p);
            Sa.cand_d2[pos] = __uint_as_float(qa & 0xFFFF0000u);
        }
    };
    auto flush_cands = [&]() __attribute__((always_inline)) {
        const uint32_t cnt = min(ccount, (uint32_t)kCandStage);
        if (tid == 0) cbase = atomicAdd(&Sa.hdr->n_cand, cnt);
        __syncthreads();
        for (uint32_t k = tid; k < cnt; k += 256) store_cand(cbase + k, cbuf[k].x, cbuf[k].y);
        __syncthreads();
        if (tid == 0) ccount = 0;
        __syncthreads();
    };

    const int col = l & 31, kh = l >> 5;
    const int M = Sa.M;
    const long long N = Sa.N;
    const long long n_items = (N + XB - 1) / XB;
    const bool masked = Sa.mask != nullptr && !DUMP;
    const int words = (M + 63) >> 6;
    // work units: (work item, group of GROUP queries), item-major; one group for M <= GROUP
    const int n_groups = (M + GROUP - 1) / GROUP;
    const long long n_units = n_items * n_groups;
    int g0 = 0, cnt = 0;   // current query group and its number of listed queries

    // query of list entry i of the current group; entries past the list (i >= cnt, i < GROUP)
    // read query g0, whose rows then carry a bias that never passes. The list is read at a
    // clamped index whether or not it is in use, so the reads need no branch.
    auto query_at = [&](int i) __attribute__((always_inline)) -> int {
        const int ic = i < cnt ? i : 0;
        const int li = (int)s_list[ic];
        return i < cnt ? g0 + (masked ? li : ic) : g0;
    };
    // series index of sorted position p (the bfloat16 rows are stored in leaf order)
    auto series_of = [&](uint32_t p) __attribute__((always_inline)) -> uint32_t { return Sa.perm ? Sa.perm[p] : p; };

    // The queries of tile t's rows that this lane loads, data chunks and (in the first 2 QT / 64
    // waves) the bias-row chunk w 64 + l, half a row each: every list read is issued before any
    // of them is used.
    struct TileRows {
        int q[LOADS];
        int qb;
    };
    auto tile_rows = [&](int t) __attribute__((always_inline)) {
        TileRows r;
#pragma unroll
        for (int j = 0; j < LOADS; ++j) {
            const int pos = (j * 4 + w) * 64 + l;
            r.q[j] = query_at(t * QT + min(pos / CH, QT - 1));
        }
        r.qb = query_at(t * QT + min((w * 64 + l) >> 1, QT - 1));
        return r;
    };
    // tile t into qd[BUF] (asynchronous: complete after the next full wait) and its raw bias
    // constants into registers. The two tile buffers are distinct arrays addressed with a
    // compile-time index (the tile loop is unrolled by two), so the compiler can see that the
    // next tile's direct loads never write the buffer being read and need not wait for them
    // before the LDS reads. The loads are buffer loads (buffer_load_dwordx4 ... lds) through a
    // descriptor covering the M query rows: unlike the flat-encoded global form, they leave the
    // LDS reads' counter in order, so a fragment read waits only for itself.
    auto tile_issue = [&](const TileRows& r, auto BUF) __attribute__((always_inline)) {
        uint16_t* dst = decltype(BUF)::value == 0 ? qd0 : qd1;
        if (w * 64 < 2 * QT)   // uniform: bias rows, [hi(-a_q), lo(-a_q), 1, 1, 0 ...], 32 bytes each
            lds_dma16(Sa.qbias, M * 32, (r.qb * 16 + (l & 1) * 8) * 2,
                      (decltype(BUF)::value == 0 ? qb0 : qb1) + w * 64 * 8);
#pragma unroll
        for (int j = 0; j < LOADS; ++j) {
            const int pos = (j * 4 + w) * 64 + l;             // chunk position in the tile
            if ((j * 4 + w) * 64 < TCH) {                     // uniform per wave
                const int row = pos / CH, pc = pos - row * CH;
                const int c = pc ^ (row & SWM);
                lds_dma16(Sa.Qb, M * NP * 2, (r.q[j] * NP + c * 8) * 2, dst + (j * 4 + w) * 64 * 8);
            }
        }
    };

    // Work units are claimed one ahead (the claim's latency is off the path between units).
    if (tid == 0) s_next = (long long)atomicAdd(&Sa.hdr->next_item, 1u);
    for (;;) {
        __syncthreads();
        if (tid == 0) {
            s_item = s_next;
            s_next = s_next < n_units ? (long long)atomicAdd(&Sa.hdr->next_item, 1u) : n_units;
        }
        __syncthreads();
        // values read from LDS, made wave-uniform for the compiler (scalar registers, uniform
        // branches): every lane read the same word (units fit 31 bits: N / 128 items x 16 groups)
        const int unit = __builtin_amdgcn_readfirstlane((int)s_item);
        if (unit >= n_units) break;  // uniform: every wave reaches this exit
        const long long item = unit / n_groups;
        g0 = (unit - (int)item * n_groups) * GROUP;
        // this wave's first sorted position (sorted positions fit 32 bits: N <= 2^32 - 1) and the
        // wave-uniform bases its rows are addressed from with 32-bit lane offsets
        const uint32_t xw0 = (uint32_t)(item * XB + w * XW);
        // the wave's fragments of series block b = xw0 / 32 + sub start at Xb + b KS16 512
        const uint16_t* xfrag = Sa.Xb + (long long)(xw0 >> 5) * KS16 * 512 + l * 8;
        const float* xnorm = Sa.xn + xw0;

        bf16x8 bfr[S][KT];
        {
            if (masked) {
                // the group's alive bits -> ascending list of queries (one wave, prefix sum of
                // the word popcounts); the barrier first: every wave has read the last count
                __syncthreads();
                if (w == 0) {
                    const int w0 = g0 >> 6, gw = min(GROUP / 64, words - w0);
                    const unsigned long long* mrow = Sa.mask + item * words + w0;
                    unsigned long long bits = l < gw ? mrow[l] : 0ull;
                    const uint32_t pc = (uint32_t)__popcll(bits);
                    uint32_t inc = pc;
#pragma unroll
                    for (int o = 1; o < 64; o <<= 1) {
                        const uint32_t v = __shfl_up(inc, o);
                        if (l >= o) inc += v;
                    }
                    uint32_t pos = inc - pc;
                    while (bits) {
                        s_list[pos++] = (uint16_t)(l * 64 + __builtin_ctzll(bits));
                        bits &= bits - 1ull;
                    }
                    if (l == 63) s_cnt = inc;
                }
                __syncthreads();
                cnt = __builtin_amdgcn_readfirstlane((int)s_cnt);
            } else {
                cnt = min(GROUP, M - g0);
            }
            if (cnt == 0) continue;   // uniform
            {
#pragma unroll
                for (int sub = 0; sub < S; ++sub) {
                    const uint32_t xl = sub * 32 + col;
                    const bool ok = xw0 + xl < N;
                    const uint16_t* xr = xfrag + sub * KS16 * 512;
#pragma unroll
                    for (int ks = 0; ks < KS16; ++ks) {
                        if (ok) bfr[sub][ks] = *reinterpret_cast<const bf16x8*>(xr + ks * 512);
                        else bfr[sub][ks] = bf16x8{};
                    }
                    float t2 = kNoPass;
                    if (ok) t2 = DUMP ? 0.f : -__double2float_rd((1.0 - (double)Sa.c_screen) * (double)xnorm[xl] * 0.5);
                    uint4 bb = make_uint4(0, 0, 0, 0);
                    if (kh == 0) {
                        bb.x = 0x3F803F80u;   // [1.0, 1.0, hi(-b_x), lo(-b_x)]
                        bb.y = bias_pair(t2).x;
                    }
                    bfr[sub][KS16] = __builtin_bit_cast(bf16x8, bb);
                }
            }
            const int n_qt = (cnt + QT - 1) / QT;

            tile_issue(tile_rows(0), std::integral_constant<int, 0>{});
            __builtin_amdgcn_s_waitcnt(0);
            __syncthreads();

            auto tile = [&](int t, auto CUR) __attribute__((always_inline)) {
                constexpr int B = decltype(CUR)::value;
                const std::integral_constant<int, 1 - B> NEXT{};
                const bool more = t + 1 < n_qt;
                // the next tile's list entries now; its loads go out after the first k-step's
                // MFMAs, by when the list reads have returned
                TileRows nr;
                if (more) nr = tile_rows(t + 1);

                f32x16 acc[QS][S];
#pragma unroll
                for (int qs = 0; qs < QS; ++qs)
#pragma unroll
                    for (int sub = 0; sub < S; ++sub)
#pragma unroll
                        for (int i = 0; i < 16; ++i) acc[qs][sub][i] = 0.f;
                const uint16_t* tb = B == 0 ? qd0 : qd1;
                const uint16_t* tbb = (B == 0 ? qb0 : qb1) + col * 16 + kh * 8;
                // chunk (2 ks + kh) ^ (row & SWM) of row qs 32 + col: with SWM = 7 the bits above
                // bit 2 of 2 ks pass the XOR unchanged, so it is a lane offset for ks mod 4 plus
                // the constant 8 (ks / 4) chunks (an immediate offset of the LDS read)
                auto a_frag = [&](int qs, int ks) __attribute__((always_inline)) -> bf16x8 {
                    const int row = qs * 32 + col;
                    if (ks == KS16) return *reinterpret_cast<const bf16x8*>(tbb + qs * 32 * 16);
                    if constexpr (SWM == 7) {
                        const int c = ((2 * (ks & 3) + kh) ^ (col & 7)) + 8 * (ks >> 2);
                        return *reinterpret_cast<const bf16x8*>(tb + row * NP + c * 8);
                    } else {
                        const int c = (2 * ks + kh) ^ (row & SWM);
                        return *reinterpret_cast<const bf16x8*>(tb + row * NP + c * 8);
                    }
                };
                // query fragments read two k-steps ahead of their MFMAs; the scheduling barriers
                // keep each read issued before the MFMAs of the step it runs ahead of
                bf16x8 fa[KT][QS];
#pragma unroll
                for (int qs = 0; qs < QS; ++qs) fa[0][qs] = a_frag(qs, 0);
                if constexpr (KT > 1) {
#pragma unroll
                    for (int qs = 0; qs < QS; ++qs) fa[1][qs] = a_frag(qs, 1);
                }
#pragma unroll
                for (int ks = 0; ks < KT; ++ks) {
                    if (ks + 2 < KT) {
#pragma unroll
                        for (int qs = 0; qs < QS; ++qs) fa[ks + 2][qs] = a_frag(qs, ks + 2);
                    }
                    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
                    for (int qs = 0; qs < QS; ++qs)
#pragma unroll
                        for (int sub = 0; sub < S; ++sub)
                            acc[qs][sub] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(fa[ks][qs], bfr[sub][ks],
                                                                                   acc[qs][sub], 0, 0, 0);
                    __builtin_amdgcn_sched_barrier(0);
                    if (ks == 0 && more) tile_issue(nr, NEXT);   // lands in LDS during the MFMAs
                }

                if constexpr (DUMP) {
#pragma unroll
                    for (int qs = 0; qs < QS; ++qs)
#pragma unroll
                        for (int sub = 0; sub < S; ++sub)
#pragma unroll
                            for (int i = 0; i < 16; ++i) {
                                const int r = t * QT + qs * 32 + 8 * (i >> 2) + 4 * kh + (i & 3);
                                const uint32_t p = xw0 + sub * 32 + col;
                                if (r < cnt && p < N)
                                    Sa.dump[(long long)query_at(r) * N + series_of(p)] = acc[qs][sub][i];
                            }
                } else {
                    // One wave-wide test (the lanes' largest accumulators) for the common tile
                    // without a passing pair. Otherwise every accumulator slot (qs, sub, i) is
                    // tested with its own ballot (a scalar branch per slot); a slot with passing
                    // lanes drops rows past the list and series past N, reserves the remaining
                    // lanes' cbuf entries with one LDS atomic (ranks from mbcnt) and writes them.
                    float m = kNoPass;
#pragma unroll
                    for (int qs = 0; qs < QS; ++qs)
#pragma unroll
                        for (int sub = 0; sub < S; ++sub)
#pragma unroll
                            for (int i = 0; i < 16; i += 4)
                                m = fmaxf(m, fmaxf(fmaxf(acc[qs][sub][i], acc[qs][sub][i + 1]),
                                                   fmaxf(acc[qs][sub][i + 2], acc[qs][sub][i + 3])));
                    if (__ballot(m >= 0.f)) {
#pragma unroll
                        for (int qs = 0; qs < QS; ++qs)
#pragma unroll
                            for (int sub = 0; sub < S; ++sub)
#pragma unroll
                                for (int i = 0; i < 16; ++i) {
                                    const float av = acc[qs][sub][i];
                                    if (__ballot(av >= 0.f) == 0ull) continue;   // uniform
                                    const int r = t * QT + qs * 32 + 8 * (i >> 2) + 4 * kh + (i & 3);
                                    const uint32_t p = xw0 + sub * 32 + col;
                                    const bool take = av >= 0.f && r < cnt && p < N;
                                    const unsigned long long mk = __ballot(take);
                                    if (take) {
                                        const uint32_t rank = __builtin_amdgcn_mbcnt_hi(
                                            (uint32_t)(mk >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)mk, 0u));
                                        uint32_t base = 0;
                                        if (rank == 0) base = atomicAdd(&ccount, (uint32_t)__popcll(mk));
                                        base = __builtin_amdgcn_readlane(base, __builtin_ctzll(mk));
                                        const uint32_t qh = (uint32_t)query_at(r);
                                        // av >= 0: its bits order as its values
                                        if (track) atomicMax(&s_amax[qh], __float_as_uint(av));
                                        const uint2 c = make_uint2(qh | (__float_as_uint(av) & 0xFFFF0000u), p);
                                        const uint32_t kk = base + rank;
                                        if (kk < (uint32_t)kCandStage) {
                                            cbuf[kk] = c;
                                        } else {  // more than the stage holds in one tile
                                            store_cand(atomicAdd(&Sa.hdr->n_cand, 1u), c.x, c.y);
                                        }
                                    }
                                }
                    }
                }
                __builtin_amdgcn_s_waitcnt(0);   // this wave's direct-to-LDS loads have landed
                __syncthreads();
                if (ccount >= (uint32_t)(kCandStage / 2)) flush_cands();  // uniform: read after the barrier
            };
            if (tid == 0) atomicAdd(&Sa.hdr->n_tiles, (uint32_t)n_qt);
            for (int t = 0; t < n_qt; t += 2) {
                tile(t, std::integral_constant<int, 0>{});
                if (t + 1 < n_qt) tile(t + 1, std::integral_constant<int, 1>{});
            }
        }
    }
    __syncthreads();
    if (ccount) flush_cands();
    if (track)
        for (int q = tid; q < Sa.M; q += 256)
            if (s_amax[q]) atomicMax(&Sa.bq[q].ub, s_amax[q]);
}

template <int KS16, int QT, int S>
static void launch_screen32_shape(const ScreenArgs& s, int grid, hipStream_t st)
{
    if (s.dump) k_screen32<KS16, QT, S, true><<<grid, 256, 0, st>>>(s);
    else k_screen32<KS16, QT, S, false><<<grid, 256, 0, st>>>(s);
}

template <int KS16>
static hipError_t launch_screen32_ks(const ScreenArgs& s, ScreenShape shape, hipStream_t st)
{
    const int grid = shape.grid > 0 ? shape.grid : 512;
    if constexpr (KS16 > 16) {
        // more than 256 dimensions: one 32-series subtile per wave and 32-row query tiles (the
        // series fragments alone take 4 (KS16 + 1) registers)
        launch_screen32_shape<KS16, 32, 1>(s, grid, st);
    } else {
        if (shape.subs == 1) {
            if (shape.qt == 64) launch_screen32_shape<KS16, 64, 1>(s, grid, st);
            else launch_screen32_shape<KS16, 32, 1>(s, grid, st);
        } else {
            if (shape.qt == 64) launch_screen32_shape<KS16, 64, 2>(s, grid, st);
            else launch_screen32_shape<KS16, 32, 2>(s, grid, st);
        }
    }
    return hipGetLastError();
}

template <int KS>
static hipError_t launch_screen_ks(const ScreenArgs& s, ScreenShape shape, hipStream_t st)
{
    const int grid = shape.grid > 0 ? shape.grid : 256;
    if (shape.subs == 2) {
        if (shape.qt == 64) k_screen<KS, 64, 2><<<grid, 256, 0, st>>>(s);
        else k_screen<KS, 32, 2><<<grid, 256, 0, st>>>(s);
    } else {
        if (shape.qt == 64) k_screen<KS, 64, 4><<<grid, 256, 0, st>>>(s);
        else k_screen<KS, 32, 4><<<grid, 256, 0, st>>>(s);
    }
    return hipGetLastError();
}

// Work-item size (sorted positions) of a screen shape.
int screen_item_series(ScreenShape shape) { return shape.mfma == 32 ? 128 * shape.subs : 64 * shape.subs; }

// The block bound serves the 32-wide form (the 16-wide one screens every pair).
bool screen_uses_mask(const ScreenArgs& s, ScreenShape shape) { return s.mask && !s.dump && shape.mfma == 32; }

hipError_t launch_block_mask(const ScreenArgs& s, ScreenShape shape, hipStream_t st)
{
    if (!screen_uses_mask(s, shape)) return hipSuccess;
    const int XB = screen_item_series(shape);
    const long long items = (s.N + XB - 1) / XB;
    const dim3 grid((unsigned)((items + kMaskItems - 1) / kMaskItems), (unsigned)((s.M + 255) / 256));
    k_block_mask<<<grid, 256, 0, st>>>(s, XB);
    return hipGetLastError();
}

// The 32-wide screen's bias row of every query: [hi(-a_q), lo(-a_q), 1, 1, 0 x 12] in bfloat16
// (a query without a threshold, a_q = +inf, takes kNoPass: never passes); with dump, a_q = 0.
__global__ __launch_bounds__(256) void k_query_bias(const BQuery* __restrict__ bq, int M, bool dump,
                                                    uint16_t* __restrict__ rows)
{
    const int q = blockIdx.x * 256 + threadIdx.x;
    if (q >= M) return;
    const float a = dump ? 0.f : bq[q].a;
    const float t1 = a < __builtin_inff() ? -a : kNoPass;
    const uint2 bp = bias_pair(t1);
    uint4* r = reinterpret_cast<uint4*>(rows + (long long)q * 16);
    r[0] = make_uint4(bp.x, 0x3F803F80u, 0u, 0u);
    r[1] = make_uint4(0u, 0u, 0u, 0u);
}

hipError_t launch_screen(const ScreenArgs& s_in, int np, ScreenShape shape, hipStream_t st)
{
    ScreenArgs s = s_in;
    if (!screen_uses_mask(s, shape)) s.mask = nullptr;
    if (shape.mfma == 32) {
        if (s.M > 0) k_query_bias<<<(s.M + 255) / 256, 256, 0, st>>>(s.bq, s.M, s.dump != nullptr, s.qbias);
        switch (np / 32) {
        case 1: return launch_screen32_ks<2>(s, shape, st);
        case 2: return launch_screen32_ks<4>(s, shape, st);
        case 3: return launch_screen32_ks<6>(s, shape, st);
        case 4: return launch_screen32_ks<8>(s, shape, st);
        case 5: return launch_screen32_ks<10>(s, shape, st);
        case 6: return launch_screen32_ks<12>(s, shape, st);
        case 7: return launch_screen32_ks<14>(s, shape, st);
        case 8: return launch_screen32_ks<16>(s, shape, st);
        case 9: return launch_screen32_ks<18>(s, shape, st);
        case 10: return launch_screen32_ks<20>(s, shape, st);
        case 11: return launch_screen32_ks<22>(s, shape, st);
        case 12: return launch_screen32_ks<24>(s, shape, st);
        case 13: return launch_screen32_ks<26>(s, shape, st);
        case 14: return launch_screen32_ks<28>(s, shape, st);
        case 15: return launch_screen32_ks<30>(s, shape, st);
        case 16: return launch_screen32_ks<32>(s, shape, st);
        default: return hipErrorInvalidValue;
        }
    }
    if (np > 256) return hipErrorInvalidValue;   // the 16-wide form holds at most 256 dimensions
    switch (np / 32) {
    case 1: return launch_screen_ks<1>(s, shape, st);
    case 2: return launch_screen_ks<2>(s, shape, st);
    case 3: return launch_screen_ks<3>(s, shape, st);
    case 4: return launch_screen_ks<4>(s, shape, st);
    case 5: return launch_screen_ks<5>(s, shape, st);
    case 6: return launch_screen_ks<6>(s, shape, st);
    case 7: return launch_screen_ks<7>(s, shape, st);
    case 8: return launch_screen_ks<8>(s, shape, st);
    default: return hipErrorInvalidValue;
    }
}

// ------------------------------------------------------------------------------------------
// Re-score: float32 squared distance of every screen candidate (16 lanes per candidate, 64
// points per step, early abandoning against the query's best-so-far), stored per candidate
// and folded into the query's key with atomicMin. Then the band pass selects, against the
// final best of each query, the candidates within the resolve band.
// ------------------------------------------------------------------------------------------
__device__ __forceinline__ float group16_sum_b(float v)
{
    v += __shfl_xor(v, 8, 16);
    v += __shfl_xor(v, 4, 16);
    v += __shfl_xor(v, 2, 16);
    v += __shfl_xor(v, 1, 16);
    return v;
}

// Upper bound on every query's nearest squared distance from its screen survivors. A kept pair
// with accumulator A has d^2 <= U_q - 2 A + 2 c (qn + xn); for the survivor holding the query's
// largest accumulator A_max (gathered by the screen) that is at most
// U_q - 2 A_max + 2 c (qn + xn_max), xn_max the largest series norm, and the nearest squared
// distance is at most this survivor's. Evaluated in float64, rounded up, stored in place of
// A_max (+inf: none).
__global__ void k_query_ub(RescoreArgs R)
{
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= R.M) return;
    BQuery& b = R.bq[q];
    const float amax = __uint_as_float(b.ub);
    float ubf = __builtin_inff();
    if (R.ub_on && amax > 0.f && !b.err && b.bsf_key != kBsfInit) {
        const double xn_max = (double)__uint_as_float(R.hdr->xn_max);
        // U_q from its rounded-down copy (u_lo <= U_q < u_lo (1 + 2^-23)); the best-so-far may
        // already be lower than the seed the screen's thresholds came from (head pass)
        const double U = (double)b.u_lo * (1.0 + 0x1p-23);
        const double ub = (U - 2.0 * (double)amax + 2.0 * (double)R.c_screen * ((double)b.qn + xn_max)) * (1.0 + 0x1p-40);
        if (ub >= 0.0) ubf = __double2float_ru(ub);
    }
    b.ub = __float_as_uint(ubf);
}

// Largest series squared norm of the screened copy (for the candidates' upper bounds).
__global__ __launch_bounds__(256) void k_xn_max(const float* __restrict__ xn, long long N, uint32_t* __restrict__ out)
{
    float m = 0.f;
    for (long long i = (long long)blockIdx.x * 256 + threadIdx.x; i < N; i += (long long)gridDim.x * 256)
        m = fmaxf(m, xn[i]);
    for (int off = 32; off > 0; off >>= 1) m = fmaxf(m, __shfl_xor(m, off));
    if ((threadIdx.x & 63) == 0) atomicMax(out, __float_as_uint(m));   // non-negative: bits order as values
}

hipError_t launch_xn_max(const float* xn, long long N, BatchHdr* hdr, hipStream_t st)
{
    hipError_t e = hipMemsetAsync(&hdr->xn_max, 0, 4, st);
    if (e != hipSuccess) return e;
    long long blocks = (N + 255) / 256;
    if (blocks > 2048) blocks = 2048;
    k_xn_max<<<(unsigned)blocks, 256, 0, st>>>(xn, N, &hdr->xn_max);
    return hipGetLastError();
}

// A candidate whose screened lower bound u_lo - 2 A (A: its accumulator, stored truncated, so
// at most A (1 + 2^-7)) exceeds the query's certified upper bound ub is farther than the nearest
// neighbour and is skipped without reading its row.
__global__ __launch_bounds__(256) void k_rescore(RescoreArgs R)
{
    const int tid = threadIdx.x, l = tid & 15, lane = tid & 63;
    const uint32_t count = min(R.hdr->n_cand, R.cand_cap);
    const uint32_t grp = (blockIdx.x * 256u + tid) >> 4;
    const uint32_t ngrp = gridDim.x * 16u;
    const int n = R.n, nv = n >> 2;
    uint32_t rescored = 0;
    // the next candidate's entry (and screened accumulator) is fetched while the current one is scored
    uint2 e = grp < count ? R.cand[grp] : make_uint2(0u, 0u);
    float ea = grp < count ? R.cand_d2[grp] : 0.f;
    for (uint32_t c = grp; c < count; c += ngrp) {
        const uint2 cur = e;
        const float at = ea;
        if (c + ngrp < count) {
            e = R.cand[c + ngrp];
            ea = R.cand_d2[c + ngrp];
        }
        BQuery& b = R.bq[cur.x];
        // at keeps the top 16 bits of A, so A <= at(1 + 2^-7) when at > 0 and A <= at otherwise;
        // P (u_lo - 2 A) <= P d_P^2 <= d^2 (d_P: the screened, projected distance)
        const double a_hi = at > 0.f ? (double)at * (1.0 + 0x1p-7) : (double)at;
        const double lb = (double)b.u_lo - 2.0 * a_hi;
        if (R.ub_on && lb > (double)__uint_as_float(b.ub)) {   // uniform in the group
            if (l == 0) R.cand_d2[c] = __builtin_inff();
            continue;
        }
        unsigned long long key = 0;
        if (l == 0) key = __hip_atomic_load(&b.bsf_key, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        key = __shfl(key, lane & ~15);
        const float thr = __double2float_ru((double)key_dist_b(key) * (1.0 + R.prune_rel) + 1e-25);
        if (R.lb_on && (double)R.P * lb * (1.0 - 0x1p-40) > (double)thr) {   // as an abandon at 0 points
            if (l == 0) R.cand_d2[c] = __builtin_inff();
            continue;
        }
        ++rescored;
        const float4* r4 = reinterpret_cast<const float4*>(R.X + (long long)cur.y * n);
        const float4* q4 = reinterpret_cast<const float4*>(R.Q + (long long)cur.x * n);
        float acc = 0.f;
        bool ab = false;
        for (int v0 = 0; v0 < nv; v0 += 16) {
            const int v = v0 + l;
            float part = 0.f;
            if (v < nv) {
                const float4 a = r4[v], bq = q4[v];
                const float dx = bq.x - a.x, dy = bq.y - a.y, dz = bq.z - a.z, dw = bq.w - a.w;
                part = (dx * dx + dy * dy) + (dz * dz + dw * dw);
            }
            acc += group16_sum_b(part);
            if (acc > thr) { ab = true; break; }
        }
        if (l != 0) continue;
        R.cand_d2[c] = ab ? __builtin_inff() : acc;
        if (!ab) atomicMin(&b.bsf_key, pack_key_b(acc, cur.y));
    }
    // candidates read per block (lane 0 of every group counted its own)
    uint32_t r = l == 0 ? rescored : 0u;
    for (int off = 32; off > 0; off >>= 1) r += __shfl_xor(r, off);
    if (lane == 0 && r) atomicAdd(&R.hdr->n_rescored, r);
}

__global__ __launch_bounds__(256) void k_band(RescoreArgs R)
{
    const uint32_t count = min(R.hdr->n_cand, R.cand_cap);
    for (uint32_t c = blockIdx.x * 256u + threadIdx.x; c < count; c += gridDim.x * 256u) {
        const float d = R.cand_d2[c];
        if (!(d < __builtin_inff())) continue;
        const uint2 e = R.cand[c];
        BQuery& b = R.bq[e.x];
        if ((double)d <= (double)key_dist_b(b.bsf_key) * (1.0 + R.band_rel) + 1e-25) {
            const uint32_t pos = atomicAdd(&b.n_band, 1u);
            if (pos < kBandCap) b.band[pos] = make_uint2(e.y, __float_as_uint(d));
        }
    }
}

// Head pass (before the re-score): every survivor whose truncated accumulator equals the top 16
// bits of its query's largest one (the smallest screened lower bound; usually the nearest
// neighbour) gets its float32 distance computed by one wave and folded into the query's
// best-so-far, so that the re-score's thresholds start near the answer. One lane per candidate
// tests; the wave then scores the hits one after another (a few per query).
__global__ __launch_bounds__(256) void k_heads(RescoreArgs R)
{
    const int lane = threadIdx.x & 63;
    const uint32_t count = min(R.hdr->n_cand, R.cand_cap);
    const uint32_t wid = (blockIdx.x * 256u + threadIdx.x) >> 6, nw = gridDim.x * 4u;
    const int nv = R.n >> 2;
    for (uint32_t c0 = wid * 64u; c0 < count; c0 += nw * 64u) {
        const uint32_t c = c0 + (uint32_t)lane;
        bool hit = false;
        uint2 e = make_uint2(0u, 0u);
        if (c < count) {
            const float at = R.cand_d2[c];
            if (at > 0.f) {
                e = R.cand[c];
                hit = (R.bq[e.x].ub & 0xFFFF0000u) == __float_as_uint(at);
            }
        }
        unsigned long long m = __ballot(hit);
        while (m) {
            const int src = __ffsll((long long)m) - 1;
            m &= m - 1ull;
            const uint32_t qx = __shfl(e.x, src), row = __shfl(e.y, src);
            const float4* r4 = reinterpret_cast<const float4*>(R.X + (long long)row * R.n);
            const float4* q4 = reinterpret_cast<const float4*>(R.Q + (long long)qx * R.n);
            float part = 0.f;
            for (int v = lane; v < nv; v += 64) {
                const float4 a = r4[v], bq = q4[v];
                const float dx = bq.x - a.x, dy = bq.y - a.y, dz = bq.z - a.z, dw = bq.w - a.w;
                part += (dx * dx + dy * dy) + (dz * dz + dw * dw);
            }
            for (int off = 32; off > 0; off >>= 1) part += __shfl_xor(part, off);
            if (lane == 0) atomicMin(&R.bq[qx].bsf_key, pack_key_b(part, row));
        }
    }
}

hipError_t launch_rescore(const RescoreArgs& r, hipStream_t st)
{
    if (r.lb_on) {
        k_heads<<<kHeadBlocks, 256, 0, st>>>(r);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    k_query_ub<<<(r.M + 255) / 256, 256, 0, st>>>(r);
    {
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    k_rescore<<<kRescoreBlocks, 256, 0, st>>>(r);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    k_band<<<256, 256, 0, st>>>(r);
    return hipGetLastError();
}

// ------------------------------------------------------------------------------------------
// Resolve: one wave per query (lane 0 works). Every band entry within band_rel of the final
// float32 best is re-scored in float64 with the fixed operation order (ascending j:
// d = q_j - x_j; t = d * d; acc = acc + t); the smallest (squared distance, index) is written
// out. A query whose band list overflowed (exact ties beyond its capacity) or whose candidate
// list overflowed is handed back to the host (fallback list) and answered by the per-query path.
// ------------------------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_batch_resolve(RescoreArgs R, long long* __restrict__ out_idx,
                                                       double* __restrict__ out_dist)
{
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int q = blockIdx.x * 4 + w;
    if (q >= R.M || lane != 0) return;
    BQuery& b = R.bq[q];
    const int n = R.n;
    if (b.err) {
        out_idx[q] = -1;
        out_dist[q] = __builtin_nan("");
        return;
    }
    const unsigned long long key = b.bsf_key;
    const double band = (double)key_dist_b(key) * (1.0 + R.band_rel) + 1e-25;
    double bd = __builtin_inf();
    long long bi = -1;
    const bool overflow = b.n_band > (uint32_t)kBandCap || R.hdr->n_cand > R.cand_cap;
    if (!overflow) {
        const float* qv = R.Q + (long long)q * n;
        for (uint32_t e = 0; e < b.n_band; ++e) {
            const uint2 v = b.band[e];
            if ((double)__uint_as_float(v.y) > band) continue;
            const float* x = R.X + (long long)v.x * n;
            double acc = 0.0;
#pragma unroll 8
            for (int j = 0; j < n; ++j) {
                const double d = (double)qv[j] - (double)x[j];
                const double t = d * d;
                acc = acc + t;
            }
            if (acc < bd || (acc == bd && (long long)v.x < bi)) { bd = acc; bi = v.x; }
        }
    }
    if (bi < 0) {  // overflow, or no completed candidate (cannot happen with a seed)
        out_idx[q] = -2;
        const uint32_t p = atomicAdd(&R.hdr->n_fallback, 1u);
        R.fallback[p] = (uint32_t)q;
    } else {
        out_idx[q] = bi;
        out_dist[q] = sqrt(bd);
    }
}

hipError_t launch_batch_resolve(const RescoreArgs& r, long long* out_idx, double* out_dist, hipStream_t st)
{
    k_batch_resolve<<<(r.M + 3) / 4, 256, 0, st>>>(r, out_idx, out_dist);
    return hipGetLastError();
}

hipError_t launch_batch_init(BQuery* bq, int M, BatchHdr* hdr, hipStream_t st)
{
    k_batch_init<<<(M + 255) / 256, 256, 0, st>>>(bq, M, hdr);
    return hipGetLastError();
}

// Inspection: a given squared distance per query as its best-so-far (series 0), in place of
// the seed's.
__global__ void k_set_bsf(BQuery* __restrict__ bq, const float* __restrict__ sqdist, int M)
{
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q < M) bq[q].bsf_key = pack_key_b(sqdist[q], 0u);
}

hipError_t launch_set_bsf(BQuery* bq, const float* sqdist, int M, hipStream_t st)
{
    k_set_bsf<<<(M + 255) / 256, 256, 0, st>>>(bq, sqdist, M);
    return hipGetLastError();
}

hipError_t launch_batch_thresholds(BQuery* bq, int M, float c_screen, double seed_rel, int P, hipStream_t st)
{
    k_batch_thresholds<<<(M + 255) / 256, 256, 0, st>>>(bq, M, c_screen, seed_rel, P);
    return hipGetLastError();
}

}  // namespace paris
