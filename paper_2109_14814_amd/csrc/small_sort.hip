// small_sort.hip -- sort of a few distinct 64-bit keys (the hit list of a
// search): chunks of SORT_TILE keys are sorted completely in LDS by stable
// LSD passes, each key ranked within its wave with ballots; then every key
// is placed by its rank in the other chunks.  Up to TINY_SORT keys, one
// block ranks each key by counting the smaller ones.
#include <string.h>

#include "ms_internal.hpp"

namespace ms {

namespace {

constexpr int RB = 8;                 // radix bits per pass
constexpr int RADIX = 1 << RB;
constexpr int SORT_BLOCK = 256;       // 4 waves
constexpr int SORT_WAVES = SORT_BLOCK / WAVE;
constexpr int SORT_ITEMS = 16;
constexpr int SORT_TILE = SORT_BLOCK * SORT_ITEMS;      // 4096 keys
constexpr int WAVE_TILE = WAVE * SORT_ITEMS;            // 1024 keys per wave

__device__ __forceinline__ uint32_t digit_of(uint64_t k, int shift) { return (uint32_t)(k >> shift) & (RADIX - 1); }

// Exclusive scan over the 256 threads of a block (one value each).
__device__ __forceinline__ uint32_t block_excl_scan_256(uint32_t v, uint32_t *s_tmp /* >= 4 */, uint32_t *total)
{
    int lane = threadIdx.x & (WAVE - 1), w = threadIdx.x / WAVE;
    uint32_t x = v;
    for (int o = 1; o < WAVE; o <<= 1) {
        uint32_t y = __shfl_up(x, o);
        if (lane >= o) x += y;
    }
    if (lane == WAVE - 1) s_tmp[w] = x;
    __syncthreads();
    uint32_t add = 0, tot = 0;
    for (int i = 0; i < SORT_WAVES; ++i) {
        uint32_t t = s_tmp[i];
        if (i < w) add += t;
        tot += t;
    }
    __syncthreads();
    if (total) *total = tot;
    return add + x - v;
}

// Each block sorts one chunk of SORT_TILE keys completely in LDS (stable
// LSD passes; within a wave, the lanes holding the same digit are found with
// RB ballots and ranked by their position).
constexpr int TINY_SORT = 1024;

__global__ void __launch_bounds__(SORT_BLOCK) k_sort_chunks(const uint64_t *__restrict__ in, uint64_t *__restrict__ out,
                                                            uint64_t *__restrict__ final_out, const int64_t *n_dev,
                                                            int64_t cap, int lo_bit, int passes)
{
    __shared__ uint64_t s_buf[2][SORT_TILE];
    __shared__ uint32_t s_wcnt[SORT_WAVES][RADIX];
    __shared__ uint32_t s_tstart[RADIX];
    __shared__ uint32_t s_tmp[SORT_WAVES];
    const int tid = threadIdx.x, lane = tid & (WAVE - 1), w = tid / WAVE;
    const int64_t n = *n_dev < cap ? *n_dev : cap;
    if (n <= TINY_SORT) {
        // few keys: block 0 ranks each key by counting the smaller ones
        if (blockIdx.x != 0) return;
        for (int i = tid; i < n; i += SORT_BLOCK) s_buf[0][i] = in[i];
        __syncthreads();
        for (int i = tid; i < n; i += SORT_BLOCK) {
            const uint64_t k = s_buf[0][i];
            int r = 0;
            for (int j = 0; j < n; ++j) r += s_buf[0][j] < k;
            final_out[r] = k;
        }
        return;
    }
    const int64_t base = (int64_t)blockIdx.x * SORT_TILE;
    if (base >= n) return;
    const int cnt = (int)((n - base) < SORT_TILE ? (n - base) : SORT_TILE);
    uint64_t key[SORT_ITEMS];
#pragma unroll
    for (int i = 0; i < SORT_ITEMS; ++i) {
        int idx = w * WAVE_TILE + i * WAVE + lane;
        key[i] = idx < cnt ? in[base + idx] : ~0ull;
    }
    int cur = 0;
    for (int p = 0; p < passes; ++p) {
        const int shift = lo_bit + RB * p;
        s_wcnt[0][tid] = 0; s_wcnt[1][tid] = 0; s_wcnt[2][tid] = 0; s_wcnt[3][tid] = 0;
        __syncthreads();
        uint32_t rank[SORT_ITEMS];
#pragma unroll
        for (int i = 0; i < SORT_ITEMS; ++i) {
            int idx = w * WAVE_TILE + i * WAVE + lane;
            bool valid = idx < cnt;
            uint32_t d = digit_of(key[i], shift);
            uint64_t peers = ballot(valid);
#pragma unroll
            for (int b = 0; b < RB; ++b) {
                uint64_t m = ballot((d >> b) & 1u);
                peers &= ((d >> b) & 1u) ? m : ~m;
            }
            uint32_t prev = valid ? s_wcnt[w][d] : 0u;
            rank[i] = prev + (uint32_t)mbcnt(peers);
            bool leader = valid && (peers != 0) && (lane == __builtin_ctzll(peers));
            if (leader) s_wcnt[w][d] = prev + (uint32_t)__builtin_popcountll(peers);
        }
        __syncthreads();
        uint32_t c0 = s_wcnt[0][tid], c1 = s_wcnt[1][tid], c2 = s_wcnt[2][tid], c3 = s_wcnt[3][tid];
        uint32_t tstart = block_excl_scan_256(c0 + c1 + c2 + c3, s_tmp, nullptr);
        s_wcnt[0][tid] = 0; s_wcnt[1][tid] = c0; s_wcnt[2][tid] = c0 + c1; s_wcnt[3][tid] = c0 + c1 + c2;
        s_tstart[tid] = tstart;
        __syncthreads();
#pragma unroll
        for (int i = 0; i < SORT_ITEMS; ++i) {
            int idx = w * WAVE_TILE + i * WAVE + lane;
            if (idx < cnt) {
                uint32_t d = digit_of(key[i], shift);
                s_buf[cur][s_tstart[d] + s_wcnt[w][d] + rank[i]] = key[i];
            }
        }
        __syncthreads();
#pragma unroll
        for (int i = 0; i < SORT_ITEMS; ++i) {
            int idx = w * WAVE_TILE + i * WAVE + lane;
            key[i] = idx < cnt ? s_buf[cur][idx] : ~0ull;
        }
        cur ^= 1;
    }
#pragma unroll
    for (int i = 0; i < SORT_ITEMS; ++i) {
        int idx = w * WAVE_TILE + i * WAVE + lane;
        if (idx < cnt) out[base + idx] = key[i];
    }
}

// Final position of each key of the sorted chunks: its index in its own chunk
// plus, for every other chunk, the number of keys there that are smaller
// (keys are distinct).
__global__ void __launch_bounds__(SORT_BLOCK) k_merge_rank(const uint64_t *__restrict__ chunks,
                                                           uint64_t *__restrict__ out, const int64_t *n_dev, int64_t cap)
{
    const int64_t n = *n_dev < cap ? *n_dev : cap;
    if (n <= TINY_SORT) return;   // already placed by k_sort_chunks
    const int64_t nch = (n + SORT_TILE - 1) / SORT_TILE;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        const uint64_t k = chunks[i];
        const int64_t c = i / SORT_TILE;
        int64_t pos = i - c * SORT_TILE;
        for (int64_t o = 0; o < nch; ++o) {
            if (o == c) continue;
            int64_t lo = o * SORT_TILE, hi = lo + SORT_TILE < n ? lo + SORT_TILE : n;
            const int64_t b = lo;
            while (lo < hi) {
                int64_t mid = lo + ((hi - lo) >> 1);
                if (chunks[mid] < k) lo = mid + 1;
                else hi = mid;
            }
            pos += lo - b;
        }
        out[pos] = k;
    }
}

}  // namespace

int sort_unique_small(const uint64_t *in, uint64_t *tmp, uint64_t *out, const int64_t *n_dev, int64_t cap,
                      int lo_bit, int n_bits, hipStream_t st)
{
    if (cap <= 0) return MS_OK;
    int passes = n_bits <= 0 ? 0 : (n_bits + RB - 1) / RB;
    int64_t chunks = ceil_div(cap, SORT_TILE);
    MS_LAUNCH("k_sort_chunks", k_sort_chunks, dim3((unsigned)chunks), dim3(SORT_BLOCK), 0, st, in, tmp, out, n_dev, cap, lo_bit,
                       passes);
    int64_t g = ceil_div(cap, SORT_BLOCK);
    if (g > 1024) g = 1024;
    MS_LAUNCH("k_merge_rank", k_merge_rank, dim3((unsigned)g), dim3(SORT_BLOCK), 0, st, tmp, out, n_dev, cap);
    MS_HIP(hipGetLastError());
    return MS_OK;
}

}  // namespace ms
