// ADS+ tree build (Section 2.2, the ADS+ index; Section 3.1, IndexConstruction and SplitNode):
// the root subtrees (first bit of every segment) are the runs of equal root key in the leaf order
// of the build's radix sort; a node holding more than the leaf capacity splits into two children
// that fix one more bit of one segment, the segment whose extra bit divides the node's series most
// evenly (ties: the lowest segment; a node with all 8 bits of every segment fixed stays a leaf).
//
// Every word is known before the tree grows, so the tree is bulk loaded level by level: in every
// round the host lists the nodes that must split (ascending node id) and cuts their position
// ranges into chunks of kTreeChunk; then
//   k_tree_count      per chunk, the number of series whose next bit is 1, for every segment;
//   k_tree_choose     per node, the most even segment, the two children (ids next + 2i, +2i+1),
//                     and every chunk's offsets among the node's zeros and ones;
//   k_tree_partition  per chunk, a stable partition by that bit (wave ballots, ranks in order)
//                     into a scratch copy of the positions;
//   k_tree_copy       the partitioned ranges back.
// A node's series stay contiguous in the leaf order (bit 0 first), so the leaves are ranges of it.
#include "paris_internal.h"

namespace paris {

__global__ void k_tree_roots(const uint32_t* __restrict__ roff, AdsNode* __restrict__ nodes)
{
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= kRoots) return;
    AdsNode v;
    v.start = roff[r];
    v.end = roff[r + 1];
    v.child0 = -1;
    v.split = -1;
#pragma unroll
    for (int s = 0; s < kSeg; ++s) v.card[s] = 1;
    nodes[r] = v;
}

hipError_t launch_tree_roots(const uint32_t* roff, AdsNode* nodes, hipStream_t st)
{
    k_tree_roots<<<kRoots / 256, 256, 0, st>>>(roff, nodes);
    return hipGetLastError();
}

// next bit of every segment of one word at the node's cardinalities (bit s of the result)
__device__ __forceinline__ uint32_t next_bits(const uint4 w, const uint8_t* card)
{
    uint32_t m = 0;
#pragma unroll
    for (int s = 0; s < kSeg; ++s) {
        const uint32_t word = s < 4 ? w.x : s < 8 ? w.y : s < 12 ? w.z : w.w;
        const uint32_t sym = (word >> (8 * (s & 3))) & 255u;
        const int c = card[s];
        m |= (c < 8 ? ((sym >> (7 - c)) & 1u) : 0u) << s;
    }
    return m;
}

__global__ __launch_bounds__(256) void k_tree_count(TreeRound R)
{
    __shared__ uint32_t part[4][kSeg];
    __shared__ uint8_t card[kSeg];
    const TreeChunk c = R.chunks[blockIdx.x];
    const int tid = threadIdx.x, lane = tid & 63;
    if (tid < kSeg) card[tid] = R.nodes[R.todo[c.slot]].card[tid];
    __syncthreads();
    uint32_t cnt[kSeg];
#pragma unroll
    for (int s = 0; s < kSeg; ++s) cnt[s] = 0;
    for (uint32_t p = c.start + tid; p < c.end; p += 256) {
        const uint4 w = reinterpret_cast<const uint4*>(R.sax)[R.perm[p]];
        const uint32_t m = next_bits(w, card);
#pragma unroll
        for (int s = 0; s < kSeg; ++s) cnt[s] += (m >> s) & 1u;
    }
#pragma unroll
    for (int s = 0; s < kSeg; ++s) {
        uint32_t v = cnt[s];
        for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
        if (lane == 0) part[tid >> 6][s] = v;
    }
    __syncthreads();
    if (tid < kSeg)
        R.chunk_ones[(long long)blockIdx.x * kSeg + tid] = part[0][tid] + part[1][tid] + part[2][tid] + part[3][tid];
}

__global__ __launch_bounds__(256) void k_tree_choose(TreeRound R)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= R.n_todo) return;
    const int v = R.todo[i];
    AdsNode node = R.nodes[v];
    const uint32_t c0 = R.todo_chunks[i], c1 = R.todo_chunks[i + 1];
    uint32_t ones[kSeg];
#pragma unroll
    for (int s = 0; s < kSeg; ++s) ones[s] = 0;
    for (uint32_t c = c0; c < c1; ++c)
#pragma unroll
        for (int s = 0; s < kSeg; ++s) ones[s] += R.chunk_ones[(long long)c * kSeg + s];
    const long long m = (long long)node.end - node.start;
    int best = -1;
    long long gap_best = 0;
    for (int s = 0; s < kSeg; ++s) {
        if (node.card[s] >= 8) continue;
        long long gap = 2 * (long long)ones[s] - m;
        gap = gap < 0 ? -gap : gap;
        if (best < 0 || gap < gap_best) { best = s; gap_best = gap; }   // ties keep the lowest
    }
    // the host lists only nodes with a segment below 8 bits, so best >= 0
    const uint32_t n0 = (uint32_t)(m - ones[best]);
    const int child = R.next + 2 * i;
    node.child0 = child;
    node.split = best;
    R.nodes[v] = node;
    AdsNode k0 = node, k1 = node;
    k0.child0 = k1.child0 = -1;
    k0.split = k1.split = -1;
    k0.card[best] = k1.card[best] = (uint8_t)(node.card[best] + 1);
    k0.end = node.start + n0;
    k1.start = node.start + n0;
    R.nodes[child] = k0;
    R.nodes[child + 1] = k1;
    // every chunk's first destination among the node's zeros and ones
    uint32_t z = 0, o = 0;
    for (uint32_t c = c0; c < c1; ++c) {
        const TreeChunk ch = R.chunks[c];
        const uint32_t oc = R.chunk_ones[(long long)c * kSeg + best];
        const uint32_t zc = (ch.end - ch.start) - oc;
        R.chunk_dst[c] = make_uint2(node.start + z, node.start + n0 + o);
        z += zc;
        o += oc;
    }
    R.todo_split[i] = best;
}

__global__ __launch_bounds__(256) void k_tree_partition(TreeRound R)
{
    __shared__ uint32_t wz[4], wo[4];
    __shared__ uint8_t card[kSeg];
    __shared__ int s_split;
    const TreeChunk c = R.chunks[blockIdx.x];
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    if (tid < kSeg) card[tid] = R.nodes[R.todo[c.slot]].card[tid];
    if (tid == 0) s_split = R.todo_split[c.slot];
    __syncthreads();
    const int s = s_split;
    const int cs = card[s];
    const uint2 dst = R.chunk_dst[blockIdx.x];
    uint32_t zb = dst.x, ob = dst.y;   // next destinations of a zero and of a one
    for (uint32_t base = c.start; base < c.end; base += 256) {
        const uint32_t p = base + tid;
        const bool in = p < c.end;
        uint32_t row = 0, bit = 0;
        if (in) {
            row = R.perm[p];
            const uint4 w = reinterpret_cast<const uint4*>(R.sax)[row];
            const uint32_t word = s < 4 ? w.x : s < 8 ? w.y : s < 12 ? w.z : w.w;
            bit = (((word >> (8 * (s & 3))) & 255u) >> (7 - cs)) & 1u;
        }
        const unsigned long long m1 = __ballot(in && bit);
        const unsigned long long m0 = __ballot(in && !bit);
        const uint32_t r1 = __builtin_amdgcn_mbcnt_hi((uint32_t)(m1 >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m1, 0u));
        const uint32_t r0 = __builtin_amdgcn_mbcnt_hi((uint32_t)(m0 >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m0, 0u));
        if (lane == 0) { wz[wv] = (uint32_t)__popcll(m0); wo[wv] = (uint32_t)__popcll(m1); }
        __syncthreads();
        uint32_t pz = 0, po = 0, tz = 0, to = 0;
        for (int k = 0; k < 4; ++k) {
            if (k < wv) { pz += wz[k]; po += wo[k]; }
            tz += wz[k];
            to += wo[k];
        }
        if (in) R.perm_tmp[bit ? ob + po + r1 : zb + pz + r0] = row;
        zb += tz;
        ob += to;
        __syncthreads();   // wz / wo are rewritten by the next step
    }
}

__global__ __launch_bounds__(256) void k_tree_copy(TreeRound R)
{
    const TreeChunk c = R.chunks[blockIdx.x];
    for (uint32_t p = c.start + threadIdx.x; p < c.end; p += 256) R.perm[p] = R.perm_tmp[p];
}

hipError_t launch_tree_round(const TreeRound& r, int n_chunks, hipStream_t st)
{
    k_tree_count<<<n_chunks, 256, 0, st>>>(r);
    k_tree_choose<<<(r.n_todo + 255) / 256, 256, 0, st>>>(r);
    k_tree_partition<<<n_chunks, 256, 0, st>>>(r);
    k_tree_copy<<<n_chunks, 256, 0, st>>>(r);
    return hipGetLastError();
}

// leaf keys of the series at every position of the tree's leaf order (bit planes 7..4 of the 16
// symbols, segment 0 first), so that keys[p] belongs to the series perm[p] in every leaf mode
__global__ __launch_bounds__(256) void k_tree_keys(const uint8_t* __restrict__ sax, const uint32_t* __restrict__ perm,
                                                   long long N, unsigned long long* __restrict__ keys)
{
    for (long long p = (long long)blockIdx.x * 256 + threadIdx.x; p < N; p += (long long)gridDim.x * 256) {
        const uint4 w = reinterpret_cast<const uint4*>(sax)[perm[p]];
        const uint32_t ws[4] = {w.x, w.y, w.z, w.w};
        unsigned long long k = 0;
        for (int b = 7; b >= 4; --b)
            for (int s = 0; s < kSeg; ++s) k = (k << 1) | (unsigned long long)((ws[s >> 2] >> (8 * (s & 3) + b)) & 1u);
        keys[p] = k;
    }
}

hipError_t launch_tree_keys(const uint8_t* sax, const uint32_t* perm, long long N, unsigned long long* keys,
                            hipStream_t st)
{
    long long blocks = (N + 255) / 256;
    if (blocks > 8192) blocks = 8192;
    k_tree_keys<<<(unsigned)blocks, 256, 0, st>>>(sax, perm, N, keys);
    return hipGetLastError();
}

}  // namespace paris
