// Query-side kernels of the exact 1-NN search (Section 3.3): prepare, approximate-search seed,
// lower-bound scan (LBC workers), early-abandoning refinement (RDC workers), float64 resolve.
#include "paris_internal.h"

namespace paris {

static __constant__ double c_beta[256] = {
    0.0,
#include "breakpoints.inc"
};

__device__ __forceinline__ unsigned long long pack_key(float d2, uint32_t idx)
{
    return ((unsigned long long)__float_as_uint(d2) << 32) | idx;
}

__device__ __forceinline__ float key_dist(unsigned long long k) { return __uint_as_float((uint32_t)(k >> 32)); }

__device__ __forceinline__ unsigned long long load_key(const unsigned long long* p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// threshold on a float32 squared quantity, rounded up so the comparison never prunes early
__device__ __forceinline__ float prune_threshold(float bsf, double rel)
{
    return __double2float_ru((double)bsf * (1.0 + rel) + 1e-25);
}

// all-reduce of a float over the 16 lanes of a lane group (butterfly: identical on all lanes)
__device__ __forceinline__ float group16_sum(float v)
{
    v += __shfl_xor(v, 8, 16);
    v += __shfl_xor(v, 4, 16);
    v += __shfl_xor(v, 2, 16);
    v += __shfl_xor(v, 1, 16);
    return v;
}

// ------------------------------------------------------------------------------------------
// prepare (one 256-thread block): query PAA and symbols (same arithmetic as the build), root and
// leaf keys, the lower-bound tables, the approximate-search window, and a fresh search state.
//   T8[s][c] = L * delta(q_s, region c)^2 in float64, rounded toward zero to float32;
//   T5[s][g] = min_{k<8} T8[s][8g+k] = the same term at 32 symbols (5-bit prefix).
// ------------------------------------------------------------------------------------------
// Lower bound of key in sorted keys[a, b) found by the whole block with 256-way splits.
__device__ long long block_lower_bound(const unsigned long long* __restrict__ keys, long long a, long long b,
                                       unsigned long long key, int* s_cnt)
{
    const int tid = threadIdx.x;
    for (;;) {
        const long long len = b - a;
        if (len <= 0) return a;
        const long long step = (len + 255) / 256;
        const long long nsamp = (len + step - 1) / step;
        const long long p = a + (long long)tid * step;
        const bool less = (tid < nsamp) && keys[p] < key;
        __syncthreads();
        if (tid == 0) *s_cnt = 0;
        __syncthreads();
        const unsigned long long m = __ballot(less);
        if ((tid & 63) == 0 && m) atomicAdd(s_cnt, __popcll(m));
        __syncthreads();
        const long long k = *s_cnt;  // samples below key form a prefix
        if (step == 1) return a + k;
        if (k == 0) return a;
        const long long na = a + (k - 1) * step + 1;
        const long long nb = (k < nsamp) ? a + k * step : b;
        a = na;
        b = nb;
    }
}

__global__ __launch_bounds__(256) void k_prepare(QueryArgs A, const float* __restrict__ q)
{
    extern __shared__ float qv[];
    __shared__ double beta[257];
    __shared__ double qpaa[kSeg];
    __shared__ int qsym[kSeg];
    __shared__ float t8[kSeg * kSym];
    __shared__ uint32_t s_bad;
    __shared__ unsigned long long s_k64;
    __shared__ uint32_t s_root;
    __shared__ int s_cnt;
    __shared__ double red_lb[256];
    __shared__ int red_r[256];

    const int tid = threadIdx.x;
    const int n = A.n, L = n >> 4;
    if (tid == 0) { s_bad = 0; beta[0] = -__builtin_inf(); beta[256] = __builtin_inf(); }
    if (tid >= 1) beta[tid] = c_beta[tid];
    for (int j = tid; j < n; j += 256) qv[j] = q[j];
    __syncthreads();
    if (tid < kSeg) {
        double acc = 0.0;
        bool bad = false;
        for (int j = 0; j < L; ++j) {
            const float v = qv[tid * L + j];
            bad |= !__builtin_isfinite(v);
            acc = acc + (double)v;
        }
        const double m = acc / (double)L;
        int c = 0;
        for (int bit = 128; bit; bit >>= 1) {
            const int t = c | bit;
            if (beta[t] <= m) c = t;
        }
        qpaa[tid] = m;
        qsym[tid] = c;
        A.qs->paa[tid] = m;
        A.qs->sym[tid] = (uint8_t)c;
        if (bad) atomicOr(&s_bad, 1u);
    }
    __syncthreads();
    if (tid == 0) {
        unsigned long long k = 0;
        for (int p = 7; p >= 4; --p)
            for (int s = 0; s < kSeg; ++s) k = (k << 1) | (unsigned long long)((qsym[s] >> p) & 1);
        s_k64 = k;
        s_root = (uint32_t)(k >> 48);
    }
    for (int e = tid; e < kSeg * kSym; e += 256) {
        const int s = e >> 8, c = e & 255;
        const double x = qpaa[s], lo = beta[c], hi = beta[c + 1];
        double d = 0.0;
        if (x < lo) d = lo - x;          // query mean BELOW the region
        else if (x > hi) d = x - hi;     // ABOVE the region
        const double v = (double)L * (d * d);
        const float f = __double2float_rz(v);
        t8[e] = f;
        A.t8[e] = f;
    }
    __syncthreads();
    for (int e = tid; e < kSeg * kCoarse; e += 256) {
        const int s = e >> 5, g = e & 31;
        const float* p = t8 + s * kSym + g * 8;
        float m = p[0];
        for (int k = 1; k < 8; ++k) m = fminf(m, p[k]);
        A.t5[e] = m;
    }

    // approximate-search window (sorted positions)
    long long lo = 0, hi = 0;
    const unsigned long long kq = s_k64;
    if (A.leaf_mode == 0) {
        if (A.seed_cap > 0) {
            uint32_t R = s_root;
            lo = A.roff[R];
            hi = A.roff[R + 1];
            if (lo == hi) {
                // empty subtree: the non-empty one with the smallest cardinality-2 lower bound
                // L * sum over segments whose top bit differs from the query's of q_s^2
                double best = __builtin_inf();
                int br = 0x7FFFFFFF;
                for (int r = tid * 256; r < tid * 256 + 256; ++r) {
                    if (A.roff[r + 1] == A.roff[r]) continue;
                    double acc = 0.0;
                    for (int s = 0; s < kSeg; ++s) {
                        const int bx = (r >> (15 - s)) & 1;
                        const double x = qpaa[s];
                        double d = 0.0;
                        if (bx == 1 && x < 0.0) d = 0.0 - x;       // region [0, +inf)
                        else if (bx == 0 && x > 0.0) d = x - 0.0;  // region (-inf, 0)
                        acc = acc + d * d;
                    }
                    const double lbv = (double)L * acc;
                    if (lbv < best) { best = lbv; br = r; }  // ascending r: ties keep the lowest
                }
                red_lb[tid] = best;
                red_r[tid] = br;
                __syncthreads();
                for (int off = 128; off > 0; off >>= 1) {
                    if (tid < off) {
                        const double b2 = red_lb[tid + off];
                        const int r2 = red_r[tid + off];
                        if (b2 < red_lb[tid] || (b2 == red_lb[tid] && r2 < red_r[tid])) {
                            red_lb[tid] = b2;
                            red_r[tid] = r2;
                        }
                    }
                    __syncthreads();
                }
                R = (uint32_t)red_r[0];
                lo = A.roff[R];
                hi = A.roff[R + 1];
            }
            if (hi - lo > A.seed_cap) {
                const long long c = block_lower_bound(A.keys, lo, hi, kq, &s_cnt);
                long long a = c - A.seed_cap / 2;
                if (a < lo) a = lo;
                if (a > hi - A.seed_cap) a = hi - A.seed_cap;
                lo = a;
                hi = a + A.seed_cap;
            }
        }
    } else {
        const long long N = A.N, nl = A.n_leaves;
        const long long c = block_lower_bound(A.keys, 0, N, kq, &s_cnt);
        long long ell = ((c + 1) * nl + N - 1) / N - 1;
        if (ell < 0) ell = 0;
        if (ell > nl - 1) ell = nl - 1;
        lo = ell * N / nl;
        hi = (ell + 1) * N / nl;
    }
    if (tid == 0) {
        QState* qs = A.qs;
        qs->root = s_root;
        qs->k64 = kq;
        qs->win_lo = lo;
        qs->win_hi = hi;
        qs->bsf_key = kBsfInit;
        qs->seed_key = kBsfInit;
        qs->n_surv = qs->n_refined = qs->n_abandon = qs->n_bsf_upd = qs->n_done = qs->n_resolved = 0;
        qs->err = s_bad ? (uint32_t)kErrNonFinite : 0u;
        qs->res_idx = -1;
        qs->res_d2 = __builtin_inf();
    }
}

hipError_t launch_prepare(const QueryArgs& a, const float* q, hipStream_t st)
{
    k_prepare<<<1, 256, (size_t)a.n * sizeof(float), st>>>(a, q);
    return hipGetLastError();
}

// ------------------------------------------------------------------------------------------
// seed: float32 squared distance from the query to every member of the approximate-search
// window (16 lanes per member), folded into the best-so-far key with atomicMin.
// ------------------------------------------------------------------------------------------
__device__ __forceinline__ float ed2_group16(const float* __restrict__ row, const float* __restrict__ q,
                                             int nv, int l)
{
    const float4* r4 = reinterpret_cast<const float4*>(row);
    const float4* q4 = reinterpret_cast<const float4*>(q);
    float acc = 0.f;
    for (int v = l; v < nv; v += 16) {
        const float4 a = r4[v], b = q4[v];
        const float dx = b.x - a.x, dy = b.y - a.y, dz = b.z - a.z, dw = b.w - a.w;
        acc += (dx * dx + dy * dy) + (dz * dz + dw * dw);
    }
    return group16_sum(acc);
}

__global__ __launch_bounds__(256) void k_seed(QueryArgs A, const float* __restrict__ q)
{
    const long long lo = A.qs->win_lo, hi = A.qs->win_hi;
    const int l = threadIdx.x & 15;
    const long long grp = ((long long)blockIdx.x * 256 + threadIdx.x) >> 4;
    const long long ngrp = (long long)gridDim.x * 16;
    const int nv = A.n >> 2;
    for (long long p = lo + grp; p < hi; p += ngrp) {
        const uint32_t row = A.perm[p];
        const float d = ed2_group16(A.X + (long long)row * A.n, q, nv, l);
        if (l == 0) atomicMin(&A.qs->bsf_key, pack_key(d, row));
    }
}

hipError_t launch_seed(const QueryArgs& a, const float* q, hipStream_t st)
{
    k_seed<<<128, 256, 0, st>>>(a, q);
    return hipGetLastError();
}

// ------------------------------------------------------------------------------------------
// lbscan (LBC workers): one 16-byte iSAX word per lane per step.
//   coarse bound: sum over s of T5[s][sym_s >> 3] from LDS. All lanes of a wave read table s at
//   the same time, and table s is 32 consecutive words, so every LDS read is conflict-free
//   (distinct banks or broadcasts) whatever the symbols are;
//   fine bound (only for lanes the coarse bound did not prune): sum of T8[s][sym_s] from the
//   L1/L2-resident global table;
//   survivors (fine bound <= threshold) are appended with one atomicAdd per wave: ballot, then
//   each lane's rank among the set lanes below it (mbcnt).
// ------------------------------------------------------------------------------------------
__device__ __forceinline__ float coarse_lb(const uint4 w, const float* __restrict__ t5)
{
    float part[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const uint32_t x = (k == 0) ? w.x : (k == 1) ? w.y : (k == 2) ? w.z : w.w;
        const float a = t5[(4 * k + 0) * 32 + ((x >> 3) & 31)];
        const float b = t5[(4 * k + 1) * 32 + ((x >> 11) & 31)];
        const float c = t5[(4 * k + 2) * 32 + ((x >> 19) & 31)];
        const float d = t5[(4 * k + 3) * 32 + ((x >> 27) & 31)];
        part[k] = (a + b) + (c + d);
    }
    return (part[0] + part[1]) + (part[2] + part[3]);
}

__device__ __forceinline__ float fine_lb(const uint4 w, const float* __restrict__ t8)
{
    float part[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const uint32_t x = (k == 0) ? w.x : (k == 1) ? w.y : (k == 2) ? w.z : w.w;
        const float a = t8[(4 * k + 0) * 256 + (x & 255)];
        const float b = t8[(4 * k + 1) * 256 + ((x >> 8) & 255)];
        const float c = t8[(4 * k + 2) * 256 + ((x >> 16) & 255)];
        const float d = t8[(4 * k + 3) * 256 + (x >> 24)];
        part[k] = (a + b) + (c + d);
    }
    return (part[0] + part[1]) + (part[2] + part[3]);
}

constexpr int kScanUnroll = 4;

__global__ __launch_bounds__(256) void k_lbscan(QueryArgs A, float fixed_thr)
{
    __shared__ float t5[kSeg * kCoarse];
    const int tid = threadIdx.x, lane = tid & 63;
    t5[tid] = A.t5[tid];
    t5[tid + 256] = A.t5[tid + 256];
    float thr;
    if (fixed_thr >= 0.f) {
        thr = fixed_thr;
    } else {
        const unsigned long long key = A.qs->bsf_key;
        thr = prune_threshold(key_dist(key), A.mg.prune_rel);
        if (blockIdx.x == 0 && tid == 0) A.qs->seed_key = key;
    }
    __syncthreads();
    const uint4* __restrict__ sax = reinterpret_cast<const uint4*>(A.sax);
    const long long N = A.N;
    const long long stride = (long long)gridDim.x * 256;
    for (long long base = (long long)blockIdx.x * 256; base < N; base += stride * kScanUnroll) {
        uint4 w[kScanUnroll];
#pragma unroll
        for (int u = 0; u < kScanUnroll; ++u) {
            const long long i = base + u * stride + tid;
            w[u] = (i < N) ? sax[i] : make_uint4(0, 0, 0, 0);
        }
#pragma unroll
        for (int u = 0; u < kScanUnroll; ++u) {
            const long long i = base + u * stride + tid;
            const float lb5 = coarse_lb(w[u], t5);
            bool pass = (i < N) && (lb5 <= thr);
            float lb8 = 0.f;
            if (pass) {
                lb8 = fine_lb(w[u], A.t8);
                pass = lb8 <= thr;
            }
            const unsigned long long m = __ballot(pass);
            if (m) {
                const uint32_t rank = __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32),
                                                                __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
                const int leader = __ffsll((long long)m) - 1;
                uint32_t basepos = 0;
                if (lane == leader) basepos = atomicAdd(&A.qs->n_surv, (uint32_t)__popcll(m));
                basepos = __shfl(basepos, leader);
                if (pass) {
                    const uint32_t pos = basepos + rank;
                    if (pos < A.surv_cap) A.surv[pos] = make_uint2((uint32_t)i, __float_as_uint(lb8));
                }
            }
        }
    }
}

static int g_scan_grid = 0;

hipError_t launch_lbscan(const QueryArgs& a, float threshold_sq, hipStream_t st)
{
    if (g_scan_grid == 0) {
        int dev = 0, cus = 256;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
            cus = 256;
        g_scan_grid = cus * 8;
    }
    const long long need = (a.N + 256LL * kScanUnroll - 1) / (256LL * kScanUnroll);
    const int grid = (int)(need < g_scan_grid ? need : g_scan_grid);
    k_lbscan<<<grid > 0 ? grid : 1, 256, 0, st>>>(a, threshold_sq);
    return hipGetLastError();
}

// ------------------------------------------------------------------------------------------
// refine (RDC workers): 16 lanes per survivor, 64 points (16 float4) per step. Before starting,
// the survivor's bound is checked again against the current best-so-far; after every step the
// partial float32 sum is compared with it (early abandoning). A completed distance is folded
// into the best-so-far with atomicMin and, when it lies within the resolve band of the current
// best, recorded for the float64 resolve.
// ------------------------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_refine(QueryArgs A, const float* __restrict__ q)
{
    const int tid = threadIdx.x, l = tid & 15, lane = tid & 63;
    const uint32_t count = min(A.qs->n_surv, A.surv_cap);
    const uint32_t grp = (blockIdx.x * 256u + tid) >> 4;
    const uint32_t ngrp = gridDim.x * 16u;
    const int nv = A.n >> 2;
    const float4* q4 = reinterpret_cast<const float4*>(q);
    uint32_t refined = 0, abandoned = 0;
    for (uint32_t c = grp; c < count; c += ngrp) {
        const uint2 e = A.surv[c];
        const float lb = __uint_as_float(e.y);
        unsigned long long key = 0;
        if (l == 0) key = load_key(&A.qs->bsf_key);
        key = __shfl(key, lane & ~15);
        float thr = prune_threshold(key_dist(key), A.mg.prune_rel);
        if (lb > thr) continue;
        ++refined;
        const float4* r4 = reinterpret_cast<const float4*>(A.X + (long long)e.x * A.n);
        float acc = 0.f;
        bool ab = false;
        for (int v0 = 0; v0 < nv; v0 += 16) {
            const int v = v0 + l;
            float part = 0.f;
            if (v < nv) {
                const float4 a = r4[v], b = q4[v];
                const float dx = b.x - a.x, dy = b.y - a.y, dz = b.z - a.z, dw = b.w - a.w;
                part = (dx * dx + dy * dy) + (dz * dz + dw * dw);
            }
            acc += group16_sum(part);
            if (acc > thr) { ab = true; break; }
            if (l == 0) key = load_key(&A.qs->bsf_key);
            key = __shfl(key, lane & ~15);
            thr = prune_threshold(key_dist(key), A.mg.prune_rel);
        }
        if (ab) { ++abandoned; continue; }
        if (l == 0) {
            const unsigned long long mine = pack_key(acc, e.x);
            const unsigned long long old = atomicMin(&A.qs->bsf_key, mine);
            if (mine < old) atomicAdd(&A.qs->n_bsf_upd, 1u);
            const unsigned long long now = mine < old ? mine : old;
            if ((double)acc <= (double)key_dist(now) * (1.0 + A.mg.band_rel) + 1e-25) {
                const uint32_t pos = atomicAdd(&A.qs->n_done, 1u);
                if (pos < A.done_cap) A.done[pos] = make_uint2(e.x, __float_as_uint(acc));
            }
        }
    }
    // per-wave counter aggregation (only lane 0 of each group counted)
    uint32_t r = (l == 0) ? refined : 0u, ab = (l == 0) ? abandoned : 0u;
    for (int off = 32; off > 0; off >>= 1) {
        r += __shfl_xor(r, off);
        ab += __shfl_xor(ab, off);
    }
    if (lane == 0) {
        if (r) atomicAdd(&A.qs->n_refined, r);
        if (ab) atomicAdd(&A.qs->n_abandon, ab);
    }
}

hipError_t launch_refine(const QueryArgs& a, const float* q, hipStream_t st)
{
    k_refine<<<512, 256, 0, st>>>(a, q);
    return hipGetLastError();
}

// ------------------------------------------------------------------------------------------
// resolve (one block): every recorded candidate within the band of the final float32 best is
// re-scored in float64 with the fixed operation order (ascending j: d = q_j - x_j; t = d * d;
// acc = acc + t; no contraction, the library is built with -ffp-contract=off); the answer is
// the smallest float64 squared distance, ties to the lowest index.
// ------------------------------------------------------------------------------------------
__device__ double ed2_f64(const float* __restrict__ row, const float* __restrict__ q, int n)
{
    double acc = 0.0;
    for (int j = 0; j < n; ++j) {
        const double d = (double)q[j] - (double)row[j];
        const double t = d * d;
        acc = acc + t;
    }
    return acc;
}

__global__ __launch_bounds__(256) void k_resolve(QueryArgs A, const float* __restrict__ q, long long* out_idx,
                                                 double* out_dist, long long qi)
{
    __shared__ double rd[256];
    __shared__ long long ri[256];
    __shared__ uint32_t rcount;
    const int tid = threadIdx.x;
    if (tid == 0) rcount = 0;
    const unsigned long long key = A.qs->bsf_key;
    const double band = (double)key_dist(key) * (1.0 + A.mg.band_rel) + 1e-25;
    const uint32_t count = min(A.qs->n_done, A.done_cap);
    double bd = __builtin_inf();
    long long bi = 0x7FFFFFFFFFFFFFFFll;
    uint32_t nres = 0;
    __syncthreads();
    for (uint32_t e = tid; e < count; e += 256) {
        const uint2 v = A.done[e];
        if ((double)__uint_as_float(v.y) <= band) {
            const double d = ed2_f64(A.X + (long long)v.x * A.n, q, A.n);
            ++nres;
            if (d < bd || (d == bd && (long long)v.x < bi)) { bd = d; bi = v.x; }
        }
    }
    rd[tid] = bd;
    ri[tid] = bi;
    if (nres) atomicAdd(&rcount, nres);
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if (tid < off) {
            const double d2 = rd[tid + off];
            const long long i2 = ri[tid + off];
            if (d2 < rd[tid] || (d2 == rd[tid] && i2 < ri[tid])) { rd[tid] = d2; ri[tid] = i2; }
        }
        __syncthreads();
    }
    if (tid == 0) {
        QState* qs = A.qs;
        const bool found = ri[0] != 0x7FFFFFFFFFFFFFFFll && qs->err == 0u;
        if (A.qs->n_surv > A.surv_cap) qs->err |= kErrSurvOverflow;
        if (A.qs->n_done > A.done_cap) qs->err |= kErrDoneOverflow;
        qs->res_idx = found ? ri[0] : -1;
        qs->res_d2 = found ? rd[0] : __builtin_nan("");
        qs->n_resolved = rcount;
        if (out_idx) {
            out_idx[qi] = found ? ri[0] : -1;
            out_dist[qi] = found ? sqrt(rd[0]) : __builtin_nan("");
        }
    }
}

hipError_t launch_resolve(const QueryArgs& a, const float* q, long long* out_idx, double* out_dist,
                          long long qi, hipStream_t st)
{
    k_resolve<<<1, 256, 0, st>>>(a, q, out_idx, out_dist, qi);
    return hipGetLastError();
}

}  // namespace paris
