// sort_scan.hip -- device-wide primitives of the search pipeline:
//   * LSD radix sort of 64-bit keys (8-bit digits), one kernel per digit in
//     "onesweep" form: tiles are ranked in LDS with wave ballots, each tile's
//     per-digit offset comes from a decoupled look-back over earlier tiles,
//     and the tile is staged in LDS so that the scatter writes runs of
//     consecutive addresses;
//   * exclusive scans (reduce / scan partials / rescan) with host- or
//     device-side element counts, so they can run inside captured graphs.
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
constexpr int MAX_PASSES = 8;
constexpr uint32_t FLAG_AGG = 1u << 30;
constexpr uint32_t FLAG_PRE = 2u << 30;
constexpr uint32_t VAL_MASK = (1u << 30) - 1;
constexpr int MAX_SORT_GRID = 1024;

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

// Digit histograms of every pass in one read of the keys.
__global__ void __launch_bounds__(SORT_BLOCK) k_radix_hist(const uint64_t *keys, const int64_t *n_dev, int lo_bit,
                                                           int passes, uint32_t *hist)
{
    __shared__ uint32_t s_h[MAX_PASSES * RADIX];
    for (int i = threadIdx.x; i < passes * RADIX; i += SORT_BLOCK) s_h[i] = 0;
    __syncthreads();
    int64_t n = *n_dev;
    int64_t stride = (int64_t)gridDim.x * SORT_BLOCK;
    for (int64_t i = (int64_t)blockIdx.x * SORT_BLOCK + threadIdx.x; i < n; i += stride) {
        uint64_t k = __builtin_nontemporal_load(keys + i);
        for (int p = 0; p < passes; ++p) atomicAdd(&s_h[p * RADIX + digit_of(k, lo_bit + RB * p)], 1u);
    }
    __syncthreads();
    for (int i = threadIdx.x; i < passes * RADIX; i += SORT_BLOCK)
        if (s_h[i]) atomicAdd(&hist[i], s_h[i]);
}

// One stable counting pass on digit (shift .. shift+7) from `in` to `out`.
__global__ void __launch_bounds__(SORT_BLOCK) k_radix_onesweep(const uint64_t *__restrict__ in,
                                                               uint64_t *__restrict__ out, const int64_t *n_dev,
                                                               int shift, const uint32_t *__restrict__ hist_pass,
                                                               uint32_t *status, uint32_t *tile_ctr)
{
    __shared__ uint64_t s_keys[SORT_TILE];
    __shared__ uint32_t s_wcnt[SORT_WAVES][RADIX];
    __shared__ uint32_t s_tstart[RADIX];
    __shared__ int64_t s_gbase[RADIX];
    __shared__ int64_t s_dbase[RADIX];
    __shared__ uint32_t s_tmp[SORT_WAVES];
    __shared__ uint32_t s_tile;

    const int tid = threadIdx.x, lane = tid & (WAVE - 1), w = tid / WAVE;
    const int64_t n = *n_dev;
    const int64_t ntiles = (n + SORT_TILE - 1) / SORT_TILE;

    // global exclusive offsets of each digit (same for every tile)
    {
        uint32_t c = hist_pass[tid];
        uint32_t ex = block_excl_scan_256(c, s_tmp, nullptr);
        s_dbase[tid] = ex;
    }

    for (;;) {
        if (tid == 0) s_tile = atomicAdd(tile_ctr, 1u);
        s_wcnt[0][tid] = 0; s_wcnt[1][tid] = 0; s_wcnt[2][tid] = 0; s_wcnt[3][tid] = 0;
        __syncthreads();
        const int64_t tile = s_tile;
        if (tile >= ntiles) break;
        const int64_t base = tile * SORT_TILE;
        const int64_t wbase = base + (int64_t)w * WAVE_TILE;

        uint64_t key[SORT_ITEMS];
        uint32_t rank[SORT_ITEMS];
#pragma unroll
        for (int i = 0; i < SORT_ITEMS; ++i) {
            int64_t idx = wbase + i * WAVE + lane;
            key[i] = idx < n ? __builtin_nontemporal_load(in + idx) : ~0ull;
        }
        // wave-level stable ranking: for each item, the lanes holding the
        // same digit are found with 8 ballots; the lowest of them bumps the
        // wave's counter for that digit
#pragma unroll
        for (int i = 0; i < SORT_ITEMS; ++i) {
            int64_t idx = wbase + i * WAVE + lane;
            bool valid = idx < n;
            uint32_t d = digit_of(key[i], shift);
            uint64_t peers = ballot(valid);
#pragma unroll
            for (int b = 0; b < RB; ++b) {
                uint64_t m = ballot((d >> b) & 1u);
                peers &= ((d >> b) & 1u) ? m : ~m;
            }
            uint32_t before = (uint32_t)mbcnt(peers);
            uint32_t prev = valid ? s_wcnt[w][d] : 0u;
            rank[i] = prev + before;
            bool leader = valid && (peers != 0) && (lane == __builtin_ctzll(peers));
            if (leader) s_wcnt[w][d] = prev + (uint32_t)__builtin_popcountll(peers);
        }
        __syncthreads();
        // per digit: waves' exclusive offsets, tile count, tile-local start
        uint32_t c0 = s_wcnt[0][tid], c1 = s_wcnt[1][tid], c2 = s_wcnt[2][tid], c3 = s_wcnt[3][tid];
        uint32_t tcount = c0 + c1 + c2 + c3;
        uint32_t tstart = block_excl_scan_256(tcount, s_tmp, nullptr);
        s_wcnt[0][tid] = 0; s_wcnt[1][tid] = c0; s_wcnt[2][tid] = c0 + c1; s_wcnt[3][tid] = c0 + c1 + c2;
        s_tstart[tid] = tstart;
        // decoupled look-back for this digit
        uint32_t *my = status + tile * RADIX + tid;
        if (tile == 0) {
            __hip_atomic_store(my, FLAG_PRE | tcount, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            s_gbase[tid] = s_dbase[tid];
        } else {
            __hip_atomic_store(my, FLAG_AGG | tcount, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            uint32_t excl = 0;
            int64_t t = tile - 1;
            for (;;) {
                uint32_t sv = __hip_atomic_load(status + t * RADIX + tid, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                uint32_t fl = sv & ~VAL_MASK;
                if (fl == 0) continue;            // predecessor not published yet (it is running)
                excl += sv & VAL_MASK;
                if (fl == FLAG_PRE) break;
                --t;
            }
            __hip_atomic_store(my, FLAG_PRE | (excl + tcount), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            s_gbase[tid] = s_dbase[tid] + excl;
        }
        __syncthreads();
        // stage the tile in LDS in digit order
#pragma unroll
        for (int i = 0; i < SORT_ITEMS; ++i) {
            int64_t idx = wbase + i * WAVE + lane;
            if (idx < n) {
                uint32_t d = digit_of(key[i], shift);
                s_keys[s_tstart[d] + s_wcnt[w][d] + rank[i]] = key[i];
            }
        }
        __syncthreads();
        const int valid_in_tile = (int)((n - base) < SORT_TILE ? (n - base) : SORT_TILE);
        for (int j = tid; j < valid_in_tile; j += SORT_BLOCK) {
            uint64_t k = s_keys[j];
            uint32_t d = digit_of(k, shift);
            out[s_gbase[d] + (j - (int64_t)s_tstart[d])] = k;
        }
        __syncthreads();
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

size_t sort_ws_bytes(int64_t cap, int max_passes)
{
    int64_t tiles = ceil_div(cap > 0 ? cap : 1, SORT_TILE);
    size_t words = (size_t)max_passes * RADIX + (size_t)max_passes * tiles * RADIX + (size_t)max_passes;
    words = (words + 1) & ~(size_t)1;   // even count of u32 -> 8-byte multiple
    return words * sizeof(uint32_t);
}

void sort_ws_carve(void *base, int64_t cap, int max_passes, SortWs &ws)
{
    int64_t tiles = ceil_div(cap > 0 ? cap : 1, SORT_TILE);
    uint32_t *p = (uint32_t *)base;
    ws.hist = p;
    ws.status = p + (size_t)max_passes * RADIX;
    ws.tile_ctr = ws.status + (size_t)max_passes * tiles * RADIX;
}

int radix_sort_u64(uint64_t *keys, uint64_t *alt, const int64_t *n_dev, int64_t cap, int lo_bit, int n_bits,
                   const SortWs &ws, hipStream_t st, uint64_t **result)
{
    *result = keys;
    if (cap <= 0 || n_bits <= 0) return MS_OK;
    if (cap >= (int64_t)VAL_MASK) return fail(MS_E_CAPACITY, "radix sort: more than 2^30 keys");
    int passes = (n_bits + RB - 1) / RB;
    if (passes > MAX_PASSES) return fail(MS_E_KEYBITS, "radix sort: more than 64 key bits");
    int64_t tiles = ceil_div(cap, SORT_TILE);
    // clear histograms, look-back status words and tile counters of every pass
    size_t words = (size_t)passes * RADIX + (size_t)passes * tiles * RADIX + (size_t)passes;
    // status and counters follow the histograms contiguously only when the
    // workspace was carved for exactly `passes`; clear each region instead
    int rc;
    if ((rc = launch_fill_u64((uint64_t *)ws.hist, 0, (int64_t)((size_t)passes * RADIX / 2), st))) return rc;
    if ((rc = launch_fill_u64((uint64_t *)ws.status, 0, (int64_t)((size_t)passes * tiles * RADIX / 2), st))) return rc;
    (void)words;
    {
        int64_t g = tiles < MAX_SORT_GRID ? tiles : MAX_SORT_GRID;
        hipLaunchKernelGGL(k_radix_hist, dim3((unsigned)g), dim3(SORT_BLOCK), 0, st, keys, n_dev, lo_bit, passes,
                           ws.hist);
        MS_HIP(hipGetLastError());
    }
    // tile counters: one u32 per pass, cleared with a tiny fill (2 per u64)
    if ((rc = launch_fill_u64((uint64_t *)ws.tile_ctr, 0, (passes + 1) / 2, st))) return rc;
    uint64_t *src = keys, *dst = alt;
    int64_t g = tiles < MAX_SORT_GRID ? tiles : MAX_SORT_GRID;
    for (int p = 0; p < passes; ++p) {
        hipLaunchKernelGGL(k_radix_onesweep, dim3((unsigned)g), dim3(SORT_BLOCK), 0, st, src, dst, n_dev,
                           lo_bit + RB * p, ws.hist + p * RADIX, ws.status + (size_t)p * tiles * RADIX,
                           ws.tile_ctr + p);
        MS_HIP(hipGetLastError());
        uint64_t *t = src; src = dst; dst = t;
    }
    *result = src;
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
