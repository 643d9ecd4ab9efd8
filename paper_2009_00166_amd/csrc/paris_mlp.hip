// Learned best-so-far seed: a 16 -> 256 -> 256 -> n_out perceptron on the query PAA scores every
// equal-count leaf, and the approximate search (the first step of exact search, Section 3.3) is
// run over the best-scoring leaves instead of the single leaf the query's own iSAX word selects.
// The network is not part of the paper; it is trained on (query, leaf of its exact nearest
// neighbour) pairs that the exact search itself produces.
//
// Arithmetic: bfloat16 operands (weights rounded to nearest even from float32 master weights,
// hidden activations and back-propagated gradients rounded where they enter a product), float32
// accumulation, float32 biases. The first layer (16 inputs) and its gradient run on the vector
// units with float32 features; the larger products run on the bf16 MFMA of gfx950
// (v_mfma_f32_16x16x32_bf16) in one LDS-tiled kernel that reads either operand in either layout.
// Training: mean softmax cross-entropy, back-propagation, Adam (Kingma and Ba 2015, Algorithm 1).
#include "paris_internal.h"

namespace paris {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ uint16_t rne16(float f)
{
    const uint32_t b = __float_as_uint(f);
    return (uint16_t)((b + 0x7FFFu + ((b >> 16) & 1u)) >> 16);
}

__device__ __forceinline__ float bf2f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

__device__ __forceinline__ float wsum(float v)
{
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
    return v;
}

// ---- features: float32 of the float64 PAA (ascending sum per segment, divided by L) ---------
__global__ __launch_bounds__(256) void k_paa_features(const float* __restrict__ Q, long long M,
                                                      long long Mpad, int n, float* __restrict__ P)
{
    const long long e = (long long)blockIdx.x * 256 + threadIdx.x;
    if (e >= Mpad * kMlpIn) return;
    const long long r = e >> 4;
    const int s = (int)(e & 15);
    if (r >= M) { P[e] = 0.f; return; }
    const int L = n >> 4;
    const float* x = Q + r * n + (long long)s * L;
    double acc = 0.0;
    for (int j = 0; j < L; ++j) acc = acc + (double)x[j];
    P[e] = (float)(acc / (double)L);
}

hipError_t launch_paa_features(const float* Q, long long M, long long Mpad, int n, float* P, hipStream_t st)
{
    const long long total = Mpad * kMlpIn;
    if (total == 0) return hipSuccess;
    k_paa_features<<<(unsigned)((total + 255) / 256), 256, 0, st>>>(Q, M, Mpad, n, P);
    return hipGetLastError();
}

// ---- layer 1: H1 = bf16(relu(P W1^T + b1)), rows >= rows_real are zero ----------------------
// sel (nullable): row r reads feature row sel[r].
__global__ __launch_bounds__(256) void k_l1_fwd(MlpNet net, const float* __restrict__ P,
                                                const int32_t* __restrict__ sel, int rows_real,
                                                int rows_pad, uint16_t* __restrict__ H1)
{
    const long long e = (long long)blockIdx.x * 256 + threadIdx.x;
    if (e >= (long long)rows_pad * kMlpHid) return;
    const int r = (int)(e >> 8), j = (int)(e & 255);
    if (r >= rows_real) { H1[e] = 0; return; }
    const long long pr = sel ? (long long)sel[r] : (long long)r;
    const float* p = P + pr * kMlpIn;
    const uint16_t* w = net.wb + net.off.w1 + (long long)j * kMlpIn;
    float acc = 0.f;
    for (int i = 0; i < kMlpIn; ++i) acc = acc + p[i] * bf2f(w[i]);
    acc = acc + net.master[net.off.b1 + j];
    H1[e] = rne16(fmaxf(acc, 0.f));
}

// ---- dW1 = G1^T P (float32 on the vector units) ----------------------------------------------
// dW1[j][i] = sum_r G1[r][j] P[sel(r)][i] (float32: the features enter unrounded). A block
// takes 64 outputs (4 hidden units x 16 features); its 16 waves split the rows (wave w sums
// rows w, w + 16, ...) and the 16 partial sums are added in wave order (deterministic).
__global__ __launch_bounds__(1024) void k_l1_bwd(const float* __restrict__ G1, const float* __restrict__ P,
                                                 const int32_t* __restrict__ sel, int rows_real,
                                                 float* __restrict__ dW1)
{
    __shared__ float part[16][64];
    const int tid = threadIdx.x, o = tid & 63, rw = tid >> 6;
    const int j = blockIdx.x * 4 + (o >> 4), i = o & 15;
    float acc = 0.f;
    for (int r = rw; r < rows_real; r += 16) {
        const long long pr = sel ? (long long)sel[r] : (long long)r;
        acc = acc + G1[(long long)r * kMlpHid + j] * P[pr * kMlpIn + i];
    }
    part[rw][o] = acc;
    __syncthreads();
    if (tid < 64) {
        float t = 0.f;
        for (int k = 0; k < 16; ++k) t = t + part[k][o];
        dW1[j * kMlpIn + i] = t;
    }
}

// ---- generic product on the MFMA: C[m][n] = sum_k A(m,k) B(n,k) ----------------------------
// A(m,k) = TA ? A[k*lda + m] : A[m*lda + k];  B(n,k) = TB ? B[k*ldb + n] : B[n*ldb + k].
// Tiles 64 x 64 x 32, 4 waves as 2 x 2, each wave 32 x 32 = 2 x 2 MFMA tiles of 16 x 16.
// Operand tiles are staged in LDS k-contiguous (a row-contiguous operand is transposed on the
// way in), so every lane reads its 8 consecutive k of one row with one 16-byte LDS read.
// MFMA 16x16x32 bf16 lane layout: lane l supplies row (l % 16), k = 8 (l / 16) .. + 7 of A and
// the same of B (column l % 16); it receives D rows 4 (l / 16) + r, r = 0..3, column l % 16.
constexpr int kBM = 64, kBN = 64, kBK = 32, kLS = kBK + 8;   // LDS row stride: 80 bytes

template <int T>
__device__ __forceinline__ void load_tile(const uint16_t* __restrict__ X, long long ld, int r0, int k0,
                                          uint16_t* S, int tid)
{
    if (T == 0) {
        const int r = tid >> 2, kk = (tid & 3) * 8;
        const uint4 v = *reinterpret_cast<const uint4*>(X + (long long)(r0 + r) * ld + k0 + kk);
        *reinterpret_cast<uint4*>(S + r * kLS + kk) = v;
    } else {
        const int kk = tid >> 3, r8 = (tid & 7) * 8;
        const uint4 v = *reinterpret_cast<const uint4*>(X + (long long)(k0 + kk) * ld + r0 + r8);
        const uint32_t w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            S[(r8 + 2 * e) * kLS + kk] = (uint16_t)(w[e] & 0xFFFFu);
            S[(r8 + 2 * e + 1) * kLS + kk] = (uint16_t)(w[e] >> 16);
        }
    }
}

template <int TA, int TB, int EPI>
__global__ __launch_bounds__(256) void k_gemm(GemmArgs g)
{
    __shared__ __attribute__((aligned(16))) uint16_t As[kBM * kLS];
    __shared__ __attribute__((aligned(16))) uint16_t Bs[kBN * kLS];
    const int tid = threadIdx.x, w = tid >> 6, l = tid & 63;
    const int m0 = blockIdx.y * kBM, n0 = blockIdx.x * kBN;
    const int wm = (w >> 1) * 32, wn = (w & 1) * 32;
    f32x4 acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
    for (int k0 = 0; k0 < g.K; k0 += kBK) {
        load_tile<TA>(g.A, g.lda, m0, k0, As, tid);
        load_tile<TB>(g.B, g.ldb, n0, k0, Bs, tid);
        __syncthreads();
        bf16x8 a[2], b[2];
#pragma unroll
        for (int i = 0; i < 2; ++i)
            a[i] = *reinterpret_cast<const bf16x8*>(As + (wm + i * 16 + (l & 15)) * kLS + (l >> 4) * 8);
#pragma unroll
        for (int j = 0; j < 2; ++j)
            b[j] = *reinterpret_cast<const bf16x8*>(Bs + (wn + j * 16 + (l & 15)) * kLS + (l >> 4) * 8);
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int j = 0; j < 2; ++j)
                acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i], b[j], acc[i][j], 0, 0, 0);
        __syncthreads();
    }
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const long long m = m0 + wm + i * 16 + 4 * (l >> 4) + r;
                const int n = n0 + wn + j * 16 + (l & 15);
                float v = acc[i][j][r];
                const long long o = m * g.ldc + n;
                if (EPI == kEpiBiasReluBf16) {
                    g.Cb[o] = rne16(fmaxf(v + g.bias[n], 0.f));
                } else if (EPI == kEpiBiasF32) {
                    g.Cf[o] = v + g.bias[n];
                } else if (EPI == kEpiMask) {
                    v = (g.mask[m * g.ldm + n] != 0) ? v : 0.f;
                    g.Cf[o] = v;
                    g.Cb[o] = rne16(v);
                } else {
                    g.Cf[o] = v;
                }
            }
}

template <int TA, int TB, int EPI>
static hipError_t gemm_t(const GemmArgs& g, hipStream_t st)
{
    dim3 grid((unsigned)(g.N / kBN), (unsigned)(g.M / kBM));
    k_gemm<TA, TB, EPI><<<grid, 256, 0, st>>>(g);
    return hipGetLastError();
}

// ---- softmax cross-entropy: G = (softmax(z) - onehot(y)) / rows_real, one block per row -----
__global__ __launch_bounds__(256) void k_softmax_ce(const float* __restrict__ Z, int n_out,
                                                    const int32_t* __restrict__ y,
                                                    const int32_t* __restrict__ sel, int rows_real,
                                                    float* __restrict__ G, uint16_t* __restrict__ Gb,
                                                    float* __restrict__ loss_row)
{
    __shared__ float red[4];
    const int r = blockIdx.x, tid = threadIdx.x, w = tid >> 6, l = tid & 63;
    const float* z = Z + (long long)r * n_out;
    float* g = G + (long long)r * n_out;
    uint16_t* gb = Gb + (long long)r * n_out;
    const int label = r < rows_real ? y[sel ? sel[r] : r] : -1;
    if (label < 0 || label >= n_out) {   // padding row (or an example without a valid label)
        for (int c = tid; c < n_out; c += 256) { g[c] = 0.f; gb[c] = 0; }
        if (tid == 0) loss_row[r] = 0.f;
        return;
    }
    float mx = -__builtin_inff();
    for (int c = tid; c < n_out; c += 256) mx = fmaxf(mx, z[c]);
    for (int off = 32; off > 0; off >>= 1) mx = fmaxf(mx, __shfl_xor(mx, off));
    if (l == 0) red[w] = mx;
    __syncthreads();
    mx = fmaxf(fmaxf(red[0], red[1]), fmaxf(red[2], red[3]));
    __syncthreads();
    float s = 0.f;
    for (int c = tid; c < n_out; c += 256) s += __expf(z[c] - mx);
    s = wsum(s);
    if (l == 0) red[w] = s;
    __syncthreads();
    s = (red[0] + red[1]) + (red[2] + red[3]);
    const float lse = mx + __logf(s);
    const float inv = 1.0f / (float)rows_real;
    for (int c = tid; c < n_out; c += 256) {
        float v = __expf(z[c] - lse);
        if (c == label) v -= 1.f;
        v *= inv;
        g[c] = v;
        gb[c] = rne16(v);
    }
    if (tid == 0) loss_row[r] = lse - z[label];
}

// ---- column sums (bias gradients) and the mean loss -----------------------------------------
// Column sums of G [rows][cols] (bias gradients). A block takes 64 columns; its 16 waves
// split the rows (wave w sums rows w, w + 16, ...) and the partial sums are added in wave
// order, so the result does not depend on scheduling.
__global__ __launch_bounds__(1024) void k_colsum(const float* __restrict__ G, int rows, int cols,
                                                 float* __restrict__ out)
{
    __shared__ float part[16][64];
    const int tid = threadIdx.x, cl = tid & 63, rw = tid >> 6;
    const int c = blockIdx.x * 64 + cl;
    float acc = 0.f;
    if (c < cols)
        for (int r = rw; r < rows; r += 16) acc += G[(long long)r * cols + c];
    part[rw][cl] = acc;
    __syncthreads();
    if (tid < 64 && c < cols) {
        float t = 0.f;
        for (int k = 0; k < 16; ++k) t += part[k][cl];
        out[c] = t;
    }
}

__global__ __launch_bounds__(256) void k_mean_loss(const float* __restrict__ lr, int rows, float* __restrict__ out)
{
    __shared__ float red[4];
    float s = 0.f;
    for (int r = threadIdx.x; r < rows; r += 256) s += lr[r];
    s = wsum(s);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) out[0] = ((red[0] + red[1]) + (red[2] + red[3])) / (float)rows;
}

// ---- Adam on the float32 master weights, then the bfloat16 mirror ---------------------------
__global__ __launch_bounds__(256) void k_adam(float* __restrict__ p, const float* __restrict__ g,
                                              float* __restrict__ m, float* __restrict__ v,
                                              uint16_t* __restrict__ wb, long long count, AdamArgs a)
{
    const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
    if (i >= count) return;
    const float gi = g[i];
    const float mi = a.beta1 * m[i] + (1.f - a.beta1) * gi;
    const float vi = a.beta2 * v[i] + (1.f - a.beta2) * (gi * gi);
    m[i] = mi;
    v[i] = vi;
    const float mhat = mi / a.bc1, vhat = vi / a.bc2;
    const float pi = p[i] - a.lr * mhat / (sqrtf(vhat) + a.eps);
    p[i] = pi;
    wb[i] = rne16(pi);
}

__global__ __launch_bounds__(256) void k_mirror(const float* __restrict__ p, uint16_t* __restrict__ wb, long long count)
{
    const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
    if (i < count) wb[i] = rne16(p[i]);
}

// ---- top leaves: the k largest logits of a row, equal logits by lowest leaf id --------------
__device__ void block_top(const float* __restrict__ z, int n_out, int k, int32_t* __restrict__ out)
{
    __shared__ uint32_t taken[kMaxLeaves / 32];
    __shared__ unsigned long long red[4];
    const int tid = threadIdx.x, w = tid >> 6, l = tid & 63;
    for (int e = tid; e < (n_out + 31) / 32; e += 256) taken[e] = 0u;
    __syncthreads();
    for (int t = 0; t < k; ++t) {
        unsigned long long best = 0ull;
        for (int c = tid; c < n_out; c += 256) {
            if ((taken[c >> 5] >> (c & 31)) & 1u) continue;
            const unsigned long long key = top_key(z[c], (uint32_t)c);
            best = key > best ? key : best;
        }
        for (int off = 32; off > 0; off >>= 1) {
            const unsigned long long o = __shfl_xor(best, off);
            best = o > best ? o : best;
        }
        if (l == 0) red[w] = best;
        __syncthreads();
        best = red[0];
        for (int q = 1; q < 4; ++q) best = red[q] > best ? red[q] : best;
        const uint32_t c = ~(uint32_t)(best & 0xFFFFFFFFu);
        if (tid == 0) {
            out[t] = (int32_t)c;
            taken[c >> 5] |= 1u << (c & 31);
        }
        __syncthreads();
    }
}

__global__ __launch_bounds__(256) void k_topk(const float* __restrict__ Z, int n_out, int k,
                                              int32_t* __restrict__ out)
{
    block_top(Z + (long long)blockIdx.x * n_out, n_out, k, out + (long long)blockIdx.x * k);
}

// ---- one query (per-query search path): PAA, the three layers and the top leaves ------------
// Every block (1024 threads) recomputes the two hidden layers (65k multiply-adds) and scores 256
// leaves, then stores its 8 best (logit, leaf) keys; the seed kernel that runs next merges the
// blocks' keys (after the kernel boundary, so no fence or completion counter is needed here).
// All weight reads are issued at the start, before the query is summarised, so their latency
// overlaps the first layer: a wave owns 16 rows of a layer, a row (256 bfloat16) is read by 32
// lanes with 16 bytes each, and a lane's 8 partial dot products are combined by a butterfly
// that halves the set at each step (a reduce-scatter over the half-wave).
__device__ __forceinline__ float dot8_bf(const uint4 w, const float* hv)
{
    const uint32_t u[4] = {w.x, w.y, w.z, w.w};
    float acc = 0.f;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        acc = acc + hv[2 * e] * __uint_as_float(u[e] << 16);
        acc = acc + hv[2 * e + 1] * __uint_as_float(u[e] & 0xFFFF0000u);
    }
    return acc;
}

// sum over the 32 lanes of a half-wave of 8 partials per lane; lane l returns the sum of
// partial index (l % 32) / 4 (the 4 lanes of a quad return the same sum)
__device__ __forceinline__ float reduce_scatter8(float (&part)[8], int lane)
{
#pragma unroll
    for (int off = 16, cnt = 4; off >= 4; off >>= 1, cnt >>= 1) {
        const bool upper = (lane & off) != 0;
#pragma unroll
        for (int i = 0; i < cnt; ++i) {
            const float send = upper ? part[i] : part[i + cnt];
            const float keep = upper ? part[i + cnt] : part[i];
            part[i] = keep + __shfl_xor(send, off);
        }
    }
    float v = part[0];
    v += __shfl_xor(v, 2);
    v += __shfl_xor(v, 1);
    return v;
}

__global__ __launch_bounds__(1024) void k_mlp_query(MlpNet net, const float* __restrict__ q, int n,
                                                    MlpQueryScratch s)
{
    __shared__ float qv[kMaxLength];
    __shared__ float f[kMlpIn];
    __shared__ float h1[kMlpHid];
    __shared__ float h2[kMlpHid];
    __shared__ unsigned long long bk[256];
    const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63, half = lane >> 5, kk = (lane & 31) * 8;
    // the query, then every weight this thread needs (issued together)
    float qr[2];
#pragma unroll
    for (int i = 0; i < 2; ++i) {
        const int j = tid + i * 1024;
        qr[i] = j < n ? q[j] : 0.f;
    }
    const int hu = tid & 255;   // layer-1 unit of this thread (threads >= 256 repeat a row, unused)
    const uint4 w1a = *reinterpret_cast<const uint4*>(net.wb + net.off.w1 + (long long)hu * kMlpIn);
    const uint4 w1b = *reinterpret_cast<const uint4*>(net.wb + net.off.w1 + (long long)hu * kMlpIn + 8);
    uint4 w2v[8], w3v[8];
#pragma unroll
    for (int p = 0; p < 8; ++p)
        w2v[p] = *reinterpret_cast<const uint4*>(net.wb + net.off.w2 + (long long)(16 * w + 2 * p + half) * kMlpHid + kk);
    const long long u0 = (long long)blockIdx.x * 256 + 16 * w;
#pragma unroll
    for (int p = 0; p < 8; ++p) {
        long long u = u0 + 2 * p + half;
        u = u < net.n_out ? u : net.n_out - 1;   // rows past the last leaf: read a valid row, unused
        w3v[p] = *reinterpret_cast<const uint4*>(net.wb + net.off.w3 + u * kMlpHid + kk);
    }
    // biases too: every read of this kernel is in flight before the first wait
    const int pr = (lane & 31) >> 2;          // this lane's row pair after the reduce-scatter
    const int row = 16 * w + 2 * pr + half;   // its row of the layer (block-local for layer 3)
    const long long u3 = u0 + 2 * pr + half;
    const float bias1 = net.master[net.off.b1 + hu];
    const float bias2 = net.master[net.off.b2 + row];
    const float bias3 = net.master[net.off.b3 + (u3 < net.n_out ? u3 : net.n_out - 1)];
#pragma unroll
    for (int i = 0; i < 2; ++i) {
        const int j = tid + i * 1024;
        if (j < n) qv[j] = qr[i];
    }
    __syncthreads();
    if (tid < kMlpIn) {
        const int L = n >> 4;
        double acc = 0.0;
        for (int j = 0; j < L; ++j) acc = acc + (double)qv[tid * L + j];
        f[tid] = (float)(acc / (double)L);
    }
    __syncthreads();
    if (tid < kMlpHid) {
        const uint32_t u[8] = {w1a.x, w1a.y, w1a.z, w1a.w, w1b.x, w1b.y, w1b.z, w1b.w};
        float acc = 0.f;
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            acc = acc + f[2 * e] * __uint_as_float(u[e] << 16);
            acc = acc + f[2 * e + 1] * __uint_as_float(u[e] & 0xFFFF0000u);
        }
        acc = acc + bias1;
        h1[tid] = bf2f(rne16(fmaxf(acc, 0.f)));
    }
    __syncthreads();
    {
        float hv[8], part[8];
#pragma unroll
        for (int e = 0; e < 8; ++e) hv[e] = h1[kk + e];
#pragma unroll
        for (int p = 0; p < 8; ++p) part[p] = dot8_bf(w2v[p], hv);
        const float acc = reduce_scatter8(part, lane);
        if ((lane & 3) == 0) h2[row] = bf2f(rne16(fmaxf(acc + bias2, 0.f)));
    }
    __syncthreads();
    {
        float hv[8], part[8];
#pragma unroll
        for (int e = 0; e < 8; ++e) hv[e] = h2[kk + e];
#pragma unroll
        for (int p = 0; p < 8; ++p) part[p] = dot8_bf(w3v[p], hv);
        const float acc = reduce_scatter8(part, lane);
        if ((lane & 3) == 0) bk[row] = u3 < net.n_out ? top_key(acc + bias3, (uint32_t)u3) : 0ull;
    }
    __syncthreads();
    // the block's 8 largest keys, by rank (valid keys are distinct; absent leaves have key 0 and
    // are never among the 8, as every block holds at least 64 leaves)
    if (tid < 256) {
        const unsigned long long key = bk[tid];
        if (key != 0ull) {
            int r = 0;
            for (int i = 0; i < 256; ++i) r += bk[i] > key ? 1 : 0;
            if (r < kTopLeaves) s.part[blockIdx.x * kTopLeaves + r] = key;
        }
    }
}

// ---- labels: the equal-count leaf of a series ---------------------------------------------
// The series' leaf key is rebuilt from its iSAX word (bit planes 7..4 of the 16 symbols,
// segment 0 first; byte s of the word is symbol s); its position in the order sorted by
// (key, index) is found by binary search; the leaf is the slice of that order containing it.
__global__ __launch_bounds__(256) void k_leaf_of(const uint8_t* __restrict__ sax,
                                                 const unsigned long long* __restrict__ keys,
                                                 const uint32_t* __restrict__ perm, long long N, int n_leaves,
                                                 const long long* __restrict__ idx, long long count,
                                                 int32_t* __restrict__ out)
{
    const long long t = (long long)blockIdx.x * 256 + threadIdx.x;
    if (t >= count) return;
    const long long i = idx[t];
    if (i < 0 || i >= N) { out[t] = -1; return; }
    const uint4 w = reinterpret_cast<const uint4*>(sax)[i];
    const uint32_t wd[4] = {w.x, w.y, w.z, w.w};
    unsigned long long k = 0;
    for (int p = 7; p >= 4; --p)
        for (int s = 0; s < 16; ++s) {
            const uint32_t sym = (wd[s >> 2] >> ((s & 3) * 8)) & 255u;
            k = (k << 1) | (unsigned long long)((sym >> p) & 1u);
        }
    long long lo = 0, hi = N;   // first position whose (key, index) is not below (k, i)
    while (lo < hi) {
        const long long mid = (lo + hi) >> 1;
        const unsigned long long km = keys[mid];
        const bool below = km < k || (km == k && (long long)perm[mid] < i);
        if (below) lo = mid + 1;
        else hi = mid;
    }
    out[t] = (int32_t)(((lo + 1) * n_leaves + N - 1) / N - 1);
}

hipError_t launch_leaf_of(const uint8_t* sax, const unsigned long long* keys, const uint32_t* perm, long long N,
                          int n_leaves, const long long* idx, long long count, int32_t* out, hipStream_t st)
{
    if (count <= 0) return hipSuccess;
    k_leaf_of<<<(unsigned)((count + 255) / 256), 256, 0, st>>>(sax, keys, perm, N, n_leaves, idx, count, out);
    return hipGetLastError();
}

// ---- host launchers ----------------------------------------------------------------------
hipError_t launch_l1_fwd(const MlpNet& net, const float* P, const int32_t* sel, int rows_real,
                         int rows_pad, uint16_t* H1, hipStream_t st)
{
    const long long total = (long long)rows_pad * kMlpHid;
    k_l1_fwd<<<(unsigned)((total + 255) / 256), 256, 0, st>>>(net, P, sel, rows_real, rows_pad, H1);
    return hipGetLastError();
}

hipError_t launch_l1_bwd(const float* G1, const float* P, const int32_t* sel, int rows_real, float* dW1,
                         hipStream_t st)
{
    k_l1_bwd<<<kMlpHid / 4, 1024, 0, st>>>(G1, P, sel, rows_real, dW1);
    return hipGetLastError();
}

hipError_t launch_gemm(const GemmArgs& g, int ta, int tb, int epi, hipStream_t st)
{
    if (g.M % kBM || g.N % kBN || g.K % kBK || g.M <= 0 || g.N <= 0 || g.K <= 0) return hipErrorInvalidValue;
    if (ta == 0 && tb == 0 && epi == kEpiBiasReluBf16) return gemm_t<0, 0, kEpiBiasReluBf16>(g, st);
    if (ta == 0 && tb == 0 && epi == kEpiBiasF32) return gemm_t<0, 0, kEpiBiasF32>(g, st);
    if (ta == 0 && tb == 1 && epi == kEpiMask) return gemm_t<0, 1, kEpiMask>(g, st);
    if (ta == 1 && tb == 1 && epi == kEpiF32) return gemm_t<1, 1, kEpiF32>(g, st);
    return hipErrorInvalidValue;
}

hipError_t launch_softmax_ce(const float* Z, int n_out, const int32_t* y, const int32_t* sel, int rows_real,
                             int rows_pad, float* G, uint16_t* Gb, float* loss_row, hipStream_t st)
{
    k_softmax_ce<<<rows_pad, 256, 0, st>>>(Z, n_out, y, sel, rows_real, G, Gb, loss_row);
    return hipGetLastError();
}

hipError_t launch_colsum(const float* G, int rows, int cols, float* out, hipStream_t st)
{
    k_colsum<<<(cols + 63) / 64, 1024, 0, st>>>(G, rows, cols, out);
    return hipGetLastError();
}

hipError_t launch_mean_loss(const float* loss_row, int rows, float* out, hipStream_t st)
{
    k_mean_loss<<<1, 256, 0, st>>>(loss_row, rows, out);
    return hipGetLastError();
}

hipError_t launch_adam(float* p, const float* g, float* m, float* v, uint16_t* wb, long long count,
                       const AdamArgs& a, hipStream_t st)
{
    k_adam<<<(unsigned)((count + 255) / 256), 256, 0, st>>>(p, g, m, v, wb, count, a);
    return hipGetLastError();
}

hipError_t launch_mirror(const float* p, uint16_t* wb, long long count, hipStream_t st)
{
    k_mirror<<<(unsigned)((count + 255) / 256), 256, 0, st>>>(p, wb, count);
    return hipGetLastError();
}

hipError_t launch_topk(const float* Z, int rows, int n_out, int k, int32_t* out, hipStream_t st)
{
    if (rows <= 0) return hipSuccess;
    k_topk<<<rows, 256, 0, st>>>(Z, n_out, k, out);
    return hipGetLastError();
}

hipError_t launch_mlp_query(const MlpNet& net, const float* q, int n, const MlpQueryScratch& s, hipStream_t st)
{
    k_mlp_query<<<(net.n_out + 255) / 256, 1024, 0, st>>>(net, q, n, s);
    return hipGetLastError();
}

}  // namespace paris
