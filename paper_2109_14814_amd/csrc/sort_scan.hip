// sort_scan.hip -- device-wide primitives of the search pipeline:
//   * LSD radix sort of 64-bit keys (8-bit digits), one kernel per digit in
//     "onesweep" form: tiles are ranked in LDS with wave ballots, each tile's
//     per-digit offset comes from a decoupled look-back over earlier tiles,
//     and the tile is staged in LDS so that the scatter writes runs of
//     consecutive addresses;
//   * exclusive scans (reduce / scan partials / rescan) with host- or
//     device-side element counts, so they can run inside captured graphs.
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
constexpr uint32_t FLAG_AGG = 1u << 30;
constexpr uint32_t FLAG_PRE = 2u << 30;
constexpr uint32_t VAL_MASK = (1u << 30) - 1;
constexpr int MAX_SORT_GRID = 1024;
constexpr int LB_W = 16;            // look-back window (statuses read per round trip)

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

__global__ void __launch_bounds__(256) k_fill_u64(uint64_t *p, uint64_t v, int64_t n)
{
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) p[i] = v;
}

// One stable counting pass on RB-bit digit `shift` from `in` to `out`
// (RB = 8, 9 or 10; each of the 256 threads owns RADIX / 256 digits).
// Besides its own look-back words, each block clears, for the tile it
// processes, the look-back words of the next pass (status_next) and
// `extra_per_tile` words of `extra` (a later kernel's look-back words), so
// no separate clearing kernel is needed.
template <int RBT>
__global__ void __launch_bounds__(SORT_BLOCK) k_radix_onesweep(const uint64_t *__restrict__ in,
                                                               uint64_t *__restrict__ out, const int64_t *n_dev,
                                                               int shift, const uint32_t *__restrict__ hist_pass,
                                                               uint32_t *status, uint32_t *status_next,
                                                               uint32_t *tile_ctr, uint64_t *extra,
                                                               int extra_per_tile, int64_t cap)
{
    constexpr int R = 1 << RBT;
    constexpr int DPT = R / SORT_BLOCK;
    __shared__ uint64_t s_keys[SORT_TILE];
    __shared__ uint32_t s_wcnt[SORT_WAVES][R];
    __shared__ uint32_t s_tstart[R];
    __shared__ uint32_t s_gbase[R];
    __shared__ uint32_t s_dbase[R];
    __shared__ uint32_t s_tmp[SORT_WAVES];
    __shared__ uint32_t s_tile;

    const int tid = threadIdx.x, lane = tid & (WAVE - 1), w = tid / WAVE;
    const int64_t n = *n_dev < cap ? *n_dev : cap;
    const int64_t ntiles = (n + SORT_TILE - 1) / SORT_TILE;
    if ((int64_t)blockIdx.x >= ntiles) return;   // no tile for this block: leave the counter alone

    // global exclusive offsets of the digits (the same for every tile)
    {
        uint32_t v[DPT], sum = 0;
#pragma unroll
        for (int j = 0; j < DPT; ++j) { v[j] = hist_pass[tid * DPT + j]; sum += v[j]; }
        uint32_t ex = block_excl_scan_256(sum, s_tmp, nullptr);
#pragma unroll
        for (int j = 0; j < DPT; ++j) { s_dbase[tid * DPT + j] = ex; ex += v[j]; }
    }

    for (;;) {
        if (tid == 0) s_tile = atomicAdd(tile_ctr, 1u);
#pragma unroll
        for (int j = 0; j < DPT; ++j) {
            s_wcnt[0][tid * DPT + j] = 0; s_wcnt[1][tid * DPT + j] = 0;
            s_wcnt[2][tid * DPT + j] = 0; s_wcnt[3][tid * DPT + j] = 0;
        }
        __syncthreads();
        const int64_t tile = s_tile;
        if (tile >= ntiles) break;
        const int64_t base = tile * SORT_TILE;
        const int64_t wbase = base + (int64_t)w * WAVE_TILE;
        if (status_next)
            for (int j = tid; j < R; j += SORT_BLOCK) status_next[tile * R + j] = 0;
        if (extra)
            for (int j = tid; j < extra_per_tile; j += SORT_BLOCK) extra[tile * extra_per_tile + j] = 0;

        uint64_t key[SORT_ITEMS];
        uint32_t rank[SORT_ITEMS];
#pragma unroll
        for (int i = 0; i < SORT_ITEMS; ++i) {
            int64_t idx = wbase + i * WAVE + lane;
            key[i] = idx < n ? __builtin_nontemporal_load(in + idx) : ~0ull;
        }
        // wave-level stable ranking: the lanes holding the same digit are
        // found with RB ballots; the lowest of them bumps the wave's counter
#pragma unroll
        for (int i = 0; i < SORT_ITEMS; ++i) {
            int64_t idx = wbase + i * WAVE + lane;
            bool valid = idx < n;
            uint32_t d = (uint32_t)(key[i] >> shift) & (R - 1);
            uint64_t peers = ballot(valid);
#pragma unroll
            for (int b = 0; b < RBT; ++b) {
                uint64_t m = ballot((d >> b) & 1u);
                peers &= ((d >> b) & 1u) ? m : ~m;
            }
            uint32_t prev = valid ? s_wcnt[w][d] : 0u;
            rank[i] = prev + (uint32_t)mbcnt(peers);
            bool leader = valid && (peers != 0) && (lane == __builtin_ctzll(peers));
            if (leader) s_wcnt[w][d] = prev + (uint32_t)__builtin_popcountll(peers);
        }
        __syncthreads();
        // per digit: the waves' exclusive offsets, the tile count and start
        uint32_t tcount[DPT], tsum = 0;
#pragma unroll
        for (int j = 0; j < DPT; ++j) {
            const int d = tid * DPT + j;
            uint32_t c0 = s_wcnt[0][d], c1 = s_wcnt[1][d], c2 = s_wcnt[2][d], c3 = s_wcnt[3][d];
            tcount[j] = c0 + c1 + c2 + c3;
            tsum += tcount[j];
            s_wcnt[0][d] = 0; s_wcnt[1][d] = c0; s_wcnt[2][d] = c0 + c1; s_wcnt[3][d] = c0 + c1 + c2;
        }
        uint32_t tstart = block_excl_scan_256(tsum, s_tmp, nullptr);
#pragma unroll
        for (int j = 0; j < DPT; ++j) { s_tstart[tid * DPT + j] = tstart; tstart += tcount[j]; }
        // decoupled look-back, one chain per digit
#pragma unroll
        for (int j = 0; j < DPT; ++j) {
            const int d = tid * DPT + j;
            uint32_t *my = status + tile * R + d;
            if (tile == 0) {
                __hip_atomic_store(my, FLAG_PRE | tcount[j], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                s_gbase[d] = s_dbase[d];
            } else {
                __hip_atomic_store(my, FLAG_AGG | tcount[j], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            }
        }
        if (tile > 0) {
#pragma unroll
            for (int j = 0; j < DPT; ++j) {
                const int d = tid * DPT + j;
                // read LB_W predecessors per round trip; stop at the first
                // inclusive prefix; re-read from a predecessor not yet published
                uint32_t excl = 0;
                int64_t t = tile - 1;
                for (;;) {
                    uint32_t sv[LB_W];
#pragma unroll
                    for (int k = 0; k < LB_W; ++k)
                        sv[k] = (t - k >= 0) ? __hip_atomic_load(status + (t - k) * R + d, __ATOMIC_RELAXED,
                                                                 __HIP_MEMORY_SCOPE_AGENT)
                                             : FLAG_PRE;
                    bool done = false;
                    int used = 0;
#pragma unroll
                    for (int k = 0; k < LB_W; ++k) {
                        if (!done && used == k) {
                            uint32_t fl = sv[k] & ~VAL_MASK;
                            if (fl != 0) {
                                excl += sv[k] & VAL_MASK;
                                if (fl == FLAG_PRE) done = true;
                                else used = k + 1;
                            }
                        }
                    }
                    if (done) break;
                    t -= used;
                }
                __hip_atomic_store(status + tile * R + d, FLAG_PRE | (excl + tcount[j]), __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_AGENT);
                s_gbase[d] = s_dbase[d] + excl;
            }
        }
        __syncthreads();
        // stage the tile in LDS in digit order, then write runs out
#pragma unroll
        for (int i = 0; i < SORT_ITEMS; ++i) {
            int64_t idx = wbase + i * WAVE + lane;
            if (idx < n) {
                uint32_t d = (uint32_t)(key[i] >> shift) & (R - 1);
                s_keys[s_tstart[d] + s_wcnt[w][d] + rank[i]] = key[i];
            }
        }
        __syncthreads();
        const int valid_in_tile = (int)((n - base) < SORT_TILE ? (n - base) : SORT_TILE);
        for (int j = tid; j < valid_in_tile; j += SORT_BLOCK) {
            uint64_t k = s_keys[j];
            uint32_t d = (uint32_t)(k >> shift) & (R - 1);
            out[(int64_t)s_gbase[d] + (j - (int64_t)s_tstart[d])] = k;
        }
        __syncthreads();
    }
}

// ----------------------------------------------- small sorts of unique keys

// Each block sorts one chunk of SORT_TILE keys completely in LDS (stable
// LSD passes with the same wave-ballot ranking as the onesweep kernel).
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

// ------------------------------------------------------------------ scans

constexpr int SCAN_BLOCK = 256;
constexpr int MAX_SCAN_GRID = 1024;

template <typename T>
__device__ __forceinline__ int64_t block_sum_i64(T v, int64_t *s_red)
{
    int64_t x = (int64_t)v;
    for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o);
    int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (lane == 0) s_red[w] = x;
    __syncthreads();
    int64_t t = 0;
    for (int i = 0; i < SCAN_BLOCK / WAVE; ++i) t += s_red[i];
    __syncthreads();
    return t;
}

// Inclusive scan of one value per thread across the block; returns the
// exclusive prefix and the block total.
__device__ __forceinline__ int64_t block_excl_scan_i64(int64_t v, int64_t *s_red, int64_t *total)
{
    int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    int64_t x = v;
    for (int o = 1; o < WAVE; o <<= 1) {
        int64_t y = __shfl_up(x, o);
        if (lane >= o) x += y;
    }
    if (lane == WAVE - 1) s_red[w] = x;
    __syncthreads();
    int64_t add = 0, tot = 0;
    for (int i = 0; i < SCAN_BLOCK / WAVE; ++i) {
        int64_t t = s_red[i];
        if (i < w) add += t;
        tot += t;
    }
    __syncthreads();
    *total = tot;
    return add + x - v;
}

template <typename T>
__device__ __forceinline__ void range_of_block(int64_t n, int64_t &b, int64_t &e)
{
    int64_t per = (n + gridDim.x - 1) / gridDim.x;
    b = per * blockIdx.x;
    e = b + per;
    if (b > n) b = n;
    if (e > n) e = n;
}

template <typename T>
__global__ void __launch_bounds__(SCAN_BLOCK) k_scan_reduce(const T *in, const int64_t *n_dev, int64_t n_host,
                                                            int64_t *partial)
{
    __shared__ int64_t s_red[SCAN_BLOCK / WAVE];
    int64_t n = n_dev ? *n_dev : n_host;
    int64_t b, e;
    range_of_block<T>(n, b, e);
    int64_t acc = 0;
    for (int64_t i = b + threadIdx.x; i < e; i += SCAN_BLOCK) acc += (int64_t)in[i];
    int64_t t = block_sum_i64(acc, s_red);
    if (threadIdx.x == 0) partial[blockIdx.x] = t;
}

__global__ void __launch_bounds__(SCAN_BLOCK) k_scan_partials(int64_t *partial, int nparts)
{
    __shared__ int64_t s_red[SCAN_BLOCK / WAVE];
    // nparts <= MAX_SCAN_GRID = 4 per thread
    constexpr int PER = MAX_SCAN_GRID / SCAN_BLOCK;
    int64_t v[PER], loc = 0;
    for (int j = 0; j < PER; ++j) {
        int idx = threadIdx.x * PER + j;
        v[j] = idx < nparts ? partial[idx] : 0;
        loc += v[j];
    }
    int64_t tot;
    int64_t ex = block_excl_scan_i64(loc, s_red, &tot);
    for (int j = 0; j < PER; ++j) {
        int idx = threadIdx.x * PER + j;
        if (idx < nparts) partial[idx] = ex;
        ex += v[j];
    }
    if (threadIdx.x == 0) partial[MAX_SCAN_GRID] = tot;
}

template <typename T>
__global__ void __launch_bounds__(SCAN_BLOCK) k_scan_apply(const T *in, int64_t *out, const int64_t *n_dev,
                                                           int64_t n_host, const int64_t *partial,
                                                           int64_t *total_dev)
{
    __shared__ int64_t s_red[SCAN_BLOCK / WAVE];
    int64_t n = n_dev ? *n_dev : n_host;
    int64_t b, e;
    range_of_block<T>(n, b, e);
    int64_t run = partial[blockIdx.x];
    for (int64_t c = b; c < e; c += SCAN_BLOCK) {
        int64_t i = c + threadIdx.x;
        int64_t v = i < e ? (int64_t)in[i] : 0;
        int64_t tot;
        int64_t ex = block_excl_scan_i64(v, s_red, &tot);
        if (i < e) out[i] = run + ex;
        run += tot;
    }
    if (blockIdx.x == gridDim.x - 1 && threadIdx.x == 0) {
        out[n] = partial[MAX_SCAN_GRID];
        if (total_dev) *total_dev = partial[MAX_SCAN_GRID];
    }
}

}  // namespace

int launch_fill_u64(uint64_t *p, uint64_t v, int64_t n, hipStream_t st)
{
    if (n <= 0) return MS_OK;
    int64_t blocks = ceil_div(n, 256);
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(k_fill_u64, dim3((unsigned)blocks), dim3(256), 0, st, p, v, n);
    MS_HIP(hipGetLastError());
    return MS_OK;
}

RadixPlan radix_plan(int lo_bit, int n_bits, int64_t cap)
{
    RadixPlan p;
    memset(&p, 0, sizeof p);
    p.lo_bit = lo_bit;
    p.n_bits = n_bits < 0 ? 0 : n_bits;
    p.cap = cap > 0 ? cap : 0;
    p.tiles_cap = ceil_div(p.cap > 0 ? p.cap : 1, SORT_TILE);
    if (p.n_bits == 0) { p.passes = 0; p.rb = 8; return p; }
    p.passes = (p.n_bits + 9) / 10;
    int rb = (p.n_bits + p.passes - 1) / p.passes;
    p.rb = rb < 8 ? 8 : rb;
    return p;
}

size_t radix_ws_bytes(const RadixPlan &p)
{
    size_t r = (size_t)1 << p.rb;
    size_t words = (size_t)p.passes * r + (size_t)p.passes * p.tiles_cap * r + (size_t)p.passes + 2;
    return (words * sizeof(uint32_t) + 255) & ~(size_t)255;
}

void radix_ws_carve(RadixPlan &p, void *base)
{
    size_t r = (size_t)1 << p.rb;
    uint32_t *w = (uint32_t *)base;
    p.hist = w;
    p.status = w + (size_t)p.passes * r;
    p.tile_ctr = p.status + (size_t)p.passes * p.tiles_cap * r;
}

int radix_sort(const RadixPlan &p, uint64_t *keys, uint64_t *alt, const int64_t *n_dev, uint64_t *extra,
               int extra_per_tile, hipStream_t st, uint64_t **result)
{
    *result = keys;
    if (p.passes == 0 || p.cap == 0) return MS_OK;
    if (p.cap >= (int64_t)VAL_MASK) return fail(MS_E_CAPACITY, "radix sort: more than 2^30 keys");
    const size_t r = (size_t)1 << p.rb;
    int64_t g = p.tiles_cap < MAX_SORT_GRID ? p.tiles_cap : MAX_SORT_GRID;
    uint64_t *src = keys, *dst = alt;
    for (int q = 0; q < p.passes; ++q) {
        uint32_t *stat = p.status + (size_t)q * p.tiles_cap * r;
        uint32_t *next = q + 1 < p.passes ? stat + (size_t)p.tiles_cap * r : nullptr;
        uint64_t *ex = q + 1 == p.passes ? extra : nullptr;
        int shift = p.lo_bit + p.rb * q;
        if (p.rb == 8)
            MS_LAUNCH("k_radix_onesweep", k_radix_onesweep<8>, dim3((unsigned)g), dim3(SORT_BLOCK), 0, st, src, dst, n_dev, shift,
                               p.hist + q * r, stat, next, p.tile_ctr + q, ex, extra_per_tile, p.cap);
        else if (p.rb == 9)
            MS_LAUNCH("k_radix_onesweep", k_radix_onesweep<9>, dim3((unsigned)g), dim3(SORT_BLOCK), 0, st, src, dst, n_dev, shift,
                               p.hist + q * r, stat, next, p.tile_ctr + q, ex, extra_per_tile, p.cap);
        else
            MS_LAUNCH("k_radix_onesweep", k_radix_onesweep<10>, dim3((unsigned)g), dim3(SORT_BLOCK), 0, st, src, dst, n_dev,
                               shift, p.hist + q * r, stat, next, p.tile_ctr + q, ex, extra_per_tile, p.cap);
        MS_HIP(hipGetLastError());
        uint64_t *t = src; src = dst; dst = t;
    }
    *result = src;
    return MS_OK;
}

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

size_t scan_ws_bytes() { return (MAX_SCAN_GRID + 8) * sizeof(int64_t); }

int scan_u32_to_i64(const uint32_t *in, int64_t *out, int64_t n, int64_t *total_dev, void *ws, hipStream_t st)
{
    int64_t *partial = (int64_t *)ws;
    int64_t g = ceil_div(n > 0 ? n : 1, 2048);
    if (g > MAX_SCAN_GRID) g = MAX_SCAN_GRID;
    hipLaunchKernelGGL(k_scan_reduce<uint32_t>, dim3((unsigned)g), dim3(SCAN_BLOCK), 0, st, in, nullptr, n, partial);
    hipLaunchKernelGGL(k_scan_partials, dim3(1), dim3(SCAN_BLOCK), 0, st, partial, (int)g);
    hipLaunchKernelGGL(k_scan_apply<uint32_t>, dim3((unsigned)g), dim3(SCAN_BLOCK), 0, st, in, out, nullptr, n,
                       partial, total_dev);
    MS_HIP(hipGetLastError());
    return MS_OK;
}

int scan_i64_dev(const int64_t *in, int64_t *out, const int64_t *n_dev, int64_t cap, int64_t *total_dev, void *ws,
                 hipStream_t st)
{
    int64_t *partial = (int64_t *)ws;
    int64_t g = ceil_div(cap > 0 ? cap : 1, 2048);
    if (g > MAX_SCAN_GRID) g = MAX_SCAN_GRID;
    hipLaunchKernelGGL(k_scan_reduce<int64_t>, dim3((unsigned)g), dim3(SCAN_BLOCK), 0, st, in, n_dev, (int64_t)0,
                       partial);
    hipLaunchKernelGGL(k_scan_partials, dim3(1), dim3(SCAN_BLOCK), 0, st, partial, (int)g);
    hipLaunchKernelGGL(k_scan_apply<int64_t>, dim3((unsigned)g), dim3(SCAN_BLOCK), 0, st, in, out, n_dev, (int64_t)0,
                       partial, total_dev);
    MS_HIP(hipGetLastError());
    return MS_OK;
}

}  // namespace ms
