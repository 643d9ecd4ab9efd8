// Build-side kernels: iSAX summarisation and the leaf order (stable LSD radix sort by leaf key).
//
// Section 3.1 (IndexBulkLoading): every series is converted to its iSAX word, which is stored at
// the series' own position of the SAX array, and the (word, position) pair is routed to the
// buffer of its root subtree (the first bit of each of the 16 symbols). Here the routing is a
// stable sort by a 64-bit leaf key whose top 16 bits are that root key; no locks are needed.
#include "paris_internal.h"

namespace paris {

// Gaussian region boundaries beta_1..beta_255 (index 0 unused): the k/256 quantiles of N(0,1).
static __constant__ double c_beta[256] = {
    0.0,
#include "breakpoints.inc"
};

// ------------------------------------------------------------------------------------------
// summarise: PAA (segment means) and 8-bit symbols for 16 series per 256-thread block.
//   * the block's 16 rows are staged in LDS with coalesced float4 loads; each segment gets
//     L + 1 floats so that the 16 x 16 threads reading their segments hit distinct banks;
//   * thread (row r, segment s) sums its L values in float64 in ascending order and divides
//     by L (the oracle's arithmetic, bit for bit), then counts the boundaries <= the mean with
//     an 8-step binary search in LDS;
//   * symbols are packed 4 per 32-bit store; the leaf key (bit planes 7..4, segment 0 first)
//     comes from four wave ballots, each 16-lane group of a wave being one row.
// ------------------------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_summarise(const float* __restrict__ X, long long N, int n,
                                                   uint8_t* __restrict__ sax,
                                                   unsigned long long* __restrict__ keys,
                                                   uint32_t* __restrict__ perm,
                                                   uint32_t* __restrict__ err)
{
    extern __shared__ float tile[];
    __shared__ double beta[256];
    const int tid = threadIdx.x;
    beta[tid] = c_beta[tid];
    const int L = n >> 4;
    const int LP = L + 1;
    const int r = tid >> 4, s = tid & 15, lane = tid & 63;
    const bool vec_ok = (L & 3) == 0;

    for (long long base = (long long)blockIdx.x * 16; base < N; base += (long long)gridDim.x * 16) {
        const int rows = (int)((N - base) < 16 ? (N - base) : 16);
        __syncthreads();  // previous tile fully consumed (and beta visible on the first pass)
        const float* src = X + base * (long long)n;
        if (vec_ok) {
            const float4* src4 = reinterpret_cast<const float4*>(src);
            const int nv = rows * (n >> 2);
            for (int v = tid; v < nv; v += 256) {
                const float4 f = src4[v];
                const int e = v << 2;
                const int seg = e / L;        // row * 16 + segment
                float* d = tile + seg * LP + (e - seg * L);
                d[0] = f.x; d[1] = f.y; d[2] = f.z; d[3] = f.w;
            }
        } else {
            const int ne = rows * n;
            for (int e = tid; e < ne; e += 256) {
                const int seg = e / L;
                tile[seg * LP + (e - seg * L)] = src[e];
            }
        }
        __syncthreads();

        const bool valid = r < rows;
        double acc = 0.0;
        bool bad = false;
        if (valid) {
            const float* p = tile + (r * 16 + s) * LP;
            for (int j = 0; j < L; ++j) {
                const float v = p[j];
                bad |= !__builtin_isfinite(v);
                acc = acc + (double)v;
            }
        }
        const double m = acc / (double)L;
        int c = 0;
#pragma unroll
        for (int bit = 128; bit; bit >>= 1) {
            const int t = c | bit;
            if (beta[t] <= m) c = t;
        }

        uint32_t packed = (uint32_t)c << (8 * (s & 3));
        packed |= __shfl_xor(packed, 1);
        packed |= __shfl_xor(packed, 2);
        if (valid && (s & 3) == 0)
            *reinterpret_cast<uint32_t*>(sax + (base + r) * 16 + s) = packed;

        const unsigned long long b7 = __ballot(valid && (c & 0x80));
        const unsigned long long b6 = __ballot(valid && (c & 0x40));
        const unsigned long long b5 = __ballot(valid && (c & 0x20));
        const unsigned long long b4 = __ballot(valid && (c & 0x10));
        if (valid && s == 0) {
            const int g = lane >> 4;
            auto plane = [g](unsigned long long b) -> unsigned long long {
                const uint32_t x = (uint32_t)(b >> (16 * g)) & 0xFFFFu;
                return (unsigned long long)(__brev(x) >> 16);  // segment 0 -> bit 15
            };
            keys[base + r] = (plane(b7) << 48) | (plane(b6) << 32) | (plane(b5) << 16) | plane(b4);
            perm[base + r] = (uint32_t)(base + r);
        }
        const unsigned long long anybad = __ballot(bad);
        if (anybad && lane == 0) atomicOr(err, (uint32_t)kErrNonFinite);
    }
}

hipError_t launch_summarise(const float* X, long long N, int n, uint8_t* sax, unsigned long long* keys,
                            uint32_t* perm, uint32_t* err, hipStream_t st)
{
    const int L = n >> 4;
    const size_t lds = (size_t)16 * 16 * (L + 1) * sizeof(float);
    if (lds > 64 * 1024) {
        hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(k_summarise),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
    }
    const long long groups = (N + 15) / 16;
    const int grid = (int)(groups < 65536 ? groups : 65536);
    k_summarise<<<grid, 256, lds, st>>>(X, N, n, sax, keys, perm, err);
    return hipGetLastError();
}

// ------------------------------------------------------------------------------------------
// Stable LSD radix sort of (key, position) pairs, 8 bits per pass, 8 passes. Each pass:
// per-tile digit histograms (digit-major), one exclusive scan, and a stable scatter in which a
// tile is processed in rounds of 256 elements: the rank of an element among equal digits of
// its wave comes from 8 ballots (match of all digit bits), waves are ordered through LDS.
// ------------------------------------------------------------------------------------------
constexpr int kTile = 4096;  // 256 threads x 16 rounds

static long long num_tiles(long long N) { return (N + kTile - 1) / kTile; }

size_t sort_hist_words(long long N) { return (size_t)num_tiles(N) * 256 + 256; }

__global__ __launch_bounds__(256) void k_rs_hist(const unsigned long long* __restrict__ keys, long long N,
                                                 int shift, uint32_t* __restrict__ hist, long long ntiles)
{
    __shared__ uint32_t h[256];
    h[threadIdx.x] = 0;
    __syncthreads();
    const long long t0 = (long long)blockIdx.x * kTile;
#pragma unroll 4
    for (int k = 0; k < 16; ++k) {
        const long long i = t0 + k * 256 + threadIdx.x;
        if (i < N) atomicAdd(&h[(uint32_t)(keys[i] >> shift) & 255u], 1u);
    }
    __syncthreads();
    hist[(long long)threadIdx.x * ntiles + blockIdx.x] = h[threadIdx.x];
}

// Exclusive scan of the digit-major histogram in two launches: the total of every digit row,
// then each row scanned by its own block starting from the sum of the rows before it.
__device__ __forceinline__ uint32_t block_sum_256(uint32_t v, uint32_t* red)
{
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    const uint32_t s = red[0] + red[1] + red[2] + red[3];
    __syncthreads();
    return s;
}

__global__ __launch_bounds__(256) void k_rs_rowsum(const uint32_t* __restrict__ hist, long long ntiles,
                                                   uint32_t* __restrict__ totals)
{
    __shared__ uint32_t red[4];
    const uint32_t* row = hist + (long long)blockIdx.x * ntiles;
    uint32_t s = 0;
    for (long long t = threadIdx.x; t < ntiles; t += 256) s += row[t];
    s = block_sum_256(s, red);
    if (threadIdx.x == 0) totals[blockIdx.x] = s;
}

__global__ __launch_bounds__(256) void k_rs_rowscan(uint32_t* __restrict__ hist, long long ntiles,
                                                    const uint32_t* __restrict__ totals)
{
    __shared__ uint32_t red[4];
    __shared__ uint32_t part[256];
    const int tid = threadIdx.x, d = blockIdx.x;
    uint32_t carry = block_sum_256(tid < d ? totals[tid] : 0u, red);  // rows before this one
    uint32_t* row = hist + (long long)d * ntiles;
    for (long long c = 0; c < ntiles; c += 256) {
        const long long t = c + tid;
        const uint32_t v = t < ntiles ? row[t] : 0u;
        part[tid] = v;
        __syncthreads();
        for (int off = 1; off < 256; off <<= 1) {  // inclusive Hillis-Steele scan
            const uint32_t o = tid >= off ? part[tid - off] : 0u;
            __syncthreads();
            part[tid] += o;
            __syncthreads();
        }
        if (t < ntiles) row[t] = carry + part[tid] - v;
        carry += part[255];
        __syncthreads();
    }
}

__global__ __launch_bounds__(256) void k_rs_scatter(const unsigned long long* __restrict__ kin,
                                                    const uint32_t* __restrict__ vin,
                                                    unsigned long long* __restrict__ kout,
                                                    uint32_t* __restrict__ vout, long long N, int shift,
                                                    const uint32_t* __restrict__ hist, long long ntiles)
{
    __shared__ uint32_t run[256];
    __shared__ uint32_t wc[4][256];
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    run[tid] = hist[(long long)tid * ntiles + blockIdx.x];
    wc[0][tid] = wc[1][tid] = wc[2][tid] = wc[3][tid] = 0;
    __syncthreads();
    const unsigned long long lt = lane ? (~0ull >> (64 - lane)) : 0ull;
    const long long t0 = (long long)blockIdx.x * kTile;
    for (int k = 0; k < 16; ++k) {
        const long long i = t0 + k * 256 + tid;
        const bool ok = i < N;
        const unsigned long long key = ok ? kin[i] : 0ull;
        const uint32_t val = ok ? vin[i] : 0u;
        const uint32_t d = (uint32_t)(key >> shift) & 255u;
        unsigned long long peers = __ballot(ok);
#pragma unroll
        for (int b = 0; b < 8; ++b) {
            const bool bit = (d >> b) & 1u;
            const unsigned long long m = __ballot(bit);
            peers &= bit ? m : ~m;
        }
        const uint32_t rank = (uint32_t)__popcll(peers & lt);
        if (ok && (peers & lt) == 0) wc[wv][d] = (uint32_t)__popcll(peers);
        __syncthreads();
        if (ok) {
            uint32_t off = run[d] + rank;
            for (int w = 0; w < wv; ++w) off += wc[w][d];
            kout[off] = key;
            vout[off] = val;
        }
        __syncthreads();
        run[tid] += wc[0][tid] + wc[1][tid] + wc[2][tid] + wc[3][tid];
        wc[0][tid] = wc[1][tid] = wc[2][tid] = wc[3][tid] = 0;
        __syncthreads();
    }
}

hipError_t launch_sort_keys(unsigned long long* keys, uint32_t* perm, unsigned long long* keys_alt,
                            uint32_t* perm_alt, uint32_t* hist, long long N, hipStream_t st)
{
    const long long nt = num_tiles(N);
    unsigned long long *ka = keys, *kb = keys_alt;
    uint32_t *va = perm, *vb = perm_alt;
    for (int pass = 0; pass < 8; ++pass) {  // even pass count: the result ends in keys / perm
        const int shift = 8 * pass;
        k_rs_hist<<<(unsigned)nt, 256, 0, st>>>(ka, N, shift, hist, nt);
        k_rs_rowsum<<<256, 256, 0, st>>>(hist, nt, hist + nt * 256);
        k_rs_rowscan<<<256, 256, 0, st>>>(hist, nt, hist + nt * 256);
        k_rs_scatter<<<(unsigned)nt, 256, 0, st>>>(ka, va, kb, vb, N, shift, hist, nt);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        unsigned long long* tk = ka; ka = kb; kb = tk;
        uint32_t* tv = va; va = vb; vb = tv;
    }
    return hipSuccess;
}

// First sorted position of every root subtree: lower bound of (r << 48) in the sorted keys.
__global__ __launch_bounds__(256) void k_root_offsets(const unsigned long long* __restrict__ keys, long long N,
                                                      uint32_t* __restrict__ roff)
{
    const int r = blockIdx.x * 256 + threadIdx.x;
    if (r > 65536) return;
    if (r == 65536) { roff[r] = (uint32_t)N; return; }
    const unsigned long long target = (unsigned long long)r << 48;
    long long lo = 0, hi = N;
    while (lo < hi) {
        const long long mid = (lo + hi) >> 1;
        if (keys[mid] < target) lo = mid + 1; else hi = mid;
    }
    roff[r] = (uint32_t)lo;
}

// iSAX words in leaf order (saxs[p] = sax[perm[p]]): the approximate search reads a window of
// consecutive sorted positions, which this copy turns into contiguous reads.
__global__ __launch_bounds__(256) void k_gather_sax(const uint4* __restrict__ sax, const uint32_t* __restrict__ perm,
                                                    long long N, uint4* __restrict__ saxs)
{
    for (long long p = (long long)blockIdx.x * 256 + threadIdx.x; p < N; p += (long long)gridDim.x * 256)
        saxs[p] = sax[perm[p]];
}

hipError_t launch_gather_sax(const uint8_t* sax, const uint32_t* perm, long long N, uint8_t* saxs, hipStream_t st)
{
    long long blocks = (N + 255) / 256;
    if (blocks > 8192) blocks = 8192;
    k_gather_sax<<<(unsigned)blocks, 256, 0, st>>>(reinterpret_cast<const uint4*>(sax), perm, N,
                                                   reinterpret_cast<uint4*>(saxs));
    return hipGetLastError();
}

hipError_t launch_root_offsets(const unsigned long long* keys, long long N, uint32_t* roff, hipStream_t st)
{
    k_root_offsets<<<(65537 + 255) / 256, 256, 0, st>>>(keys, N, roff);
    return hipGetLastError();
}

}  // namespace paris
