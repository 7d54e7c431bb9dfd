// search.hip -- the mesh-intersection search of Sec. 6.2 on one GPU, for one
// mesh pair or a batch of pairs searched together.
//
// Every kernel reads its sizes from device memory, so one call queues a fixed
// sequence of kernels with no host round trip (and can be captured in a HIP
// graph):
//   k_mark        per quad (two triangles): the cells of its four vertices,
//                 each triangle's cell range as the min / max of its
//                 vertices' cells (the cell map is monotone), one occupancy
//                 byte per (hashed) cell and side of the union of the two
//                 ranges, holding the search's epoch value (no clearing
//                 between searches); compact ranges; per-block totals;
//                 block 0 clears the counters
//   k_pack        hashed cells occupied by both meshes as bit tables (fine
//                 and coarse); each both-occupied fine cell is a group whose
//                 counters are cleared here
//   k_keys        per triangle: the cells of its range in a both-occupied
//                 group (a cell holding one mesh only cannot hold a pair);
//                 entries [cell | side | triangle] at offsets reserved per
//                 block, each with its group and its rank in the group
//   k_groups      groups holding A and B entries: entry ranges and slot
//                 offsets sum(nA * nB) (scan with decoupled look-back)
//   k_scatter     entries to their group's range, A's before B's, each with
//                 its triangle's box (Sec. 6.2.2)
//   k_enum        slot -> (group, iA, iB); a pair is kept only when both
//                 entries are of one cell, in its home cell (cell of the
//                 componentwise max of the boxes' lower corners) and only if
//                 the closed boxes overlap (Sec. 6.2.2); then, on the chunk's
//                 candidates, the Moller quick test (Sec. 6.2.3), the 4x4
//                 solve and inclusion (Sec. 6.2.4), hit records; last, the
//                 exact cell statistics into sharded counters
//   k_finish      the statistics, the next epoch value, and the hits sorted
//                 by (pair, triA, triB) when there are at most 1024 of them
//                 (above, a chunk sort, merge rank and placement first)
// A batch numbers its cells with a per-pair cell offset, so entries of
// different pairs never share a cell (they may share a group).
#include <math.h>
#include <string.h>

#include <mutex>
#include <string>
#include <utility>
#include <vector>

#include "ms_internal.hpp"
#include "predicate.hpp"

namespace ms {

namespace {

constexpr int BLOCK = 256;
constexpr int MAX_GRID = 2048;
// k_mark: runs of tiles per block, at most MARK_GRID_CAP blocks.  Many short
// runs balance the CUs better than few long ones (the 256-pair family's
// 29,700 tiles: 280 us as one tile per block, 443 us as 2048 runs); the
// grid is the number of runs (rounded up to whole XCDs), so that no XCD is
// left with only empty runs.
constexpr int64_t MARK_GRID_CAP = 32768;

inline unsigned mark_grid(int64_t n_tiles)
{
    if (n_tiles <= 0) return 1;
    const int64_t per = (n_tiles + MARK_GRID_CAP - 1) / MARK_GRID_CAP;
    int64_t g = (n_tiles + per - 1) / per;
    if (g > 8) g = (g + 7) / 8 * 8;
    return (unsigned)g;
}
static_assert(MAX_GRID <= MS_COUNT_PARTIALS, "count partials fit the mesh scratch");
constexpr int TILE_TRIS = 2 * BLOCK;                  // triangles of a tile: one quad per thread
// Counter lines of the enumeration (cand, moller, degen, outside, cells,
// slots, unstaged chunks), one 128-byte line each.
constexpr int STAT_SHARDS = 8;
constexpr int SHARD_WORDS = 16;
constexpr uint64_t SFLAG_AGG = 1ull << 62;
constexpr uint64_t SFLAG_PRE = 2ull << 62;
constexpr uint64_t SVAL_MASK = (1ull << 62) - 1;

static_assert(sizeof(search_stats_t) == 16 * 8, "search_stats_t is 16 int64 words");

inline unsigned grid_for(int64_t n, int64_t cap = MAX_GRID)
{
    int64_t g = ceil_div(n > 0 ? n : 1, BLOCK);
    return (unsigned)(g < cap ? g : cap);
}

struct KeyLayout {
    int tb;            // triangle bits
    int cell_shift;    // tb + 1
    uint64_t tmask;
};

// One mesh pair with its grid.  Cells of this pair have global ids
// cell_base + linear cell.  Its triangles are cut into tiles of TILE_TRIS
// triangles (BLOCK quads) of one mesh each: tiles tile_off + [0, tilesA)
// hold A's, the next ceil(nB / TILE_TRIS) hold B's, so that the pair and
// the side are the same for every thread of a block that works on one tile.
struct PairDesc {
    MeshView A, B;
    GridView g;
    uint64_t cell_base;
    int64_t tile_off;
    int32_t nA, nB;
    int32_t tilesA, prune;     // prune: MS_SEARCH_PRUNE
    uint64_t st[4];     // linear-id strides of the cells: n1 n2 n3, n2 n3, n3, 1
    uint32_t fbs[4];    // fine table: linear-id strides of its blocks (cell index / 2 per axis), mod 2^32
    uint32_t fbh[4];    //   and fbs * HASH_MUL mod 2^32
    uint32_t cbs[4];    // coarse table (cell index / 2 per axis): strides of its blocks, mod 2^32
    uint32_t cbh[4];    //   (cell index / 4 per axis) and cbs * HASH_MUL mod 2^32
    double nm1[4];      // n_d - 1
};

struct BatchView {
    PairDesc p0;                 // the pair of a single search
    const PairDesc *pairs;       // device array of a batch
    const int64_t *tile_off;     // n_pairs + 1 (batch): first triangle tile of each pair
    const uint64_t *cell_base;   // n_pairs + 1 (batch)
    int64_t n_tiles;             // triangle tiles of all pairs
    int32_t n_pairs;
    int32_t bm_log2;             // occupancy flags per side: 2^bm_log2 bytes, then as many bits
    int32_t bc_log2;             // the same for the coarse cells (2x the edge): 2^bc_log2 per side
    int32_t packable;            // every grid has <= 4096 cells per axis
    int32_t c32;                 // every grid has < 2^31 cells per axis (32-bit cell ranges)
    int32_t pb, tbA, tbB;        // bits of the pair, A- and B-triangle fields of hit keys
    KeyLayout kl;
};

template <bool ONE>
MS_D const PairDesc &pair_desc(const BatchView &bv, int p)
{
    if constexpr (ONE) return bv.p0;
    else return bv.pairs[p];
}

// Last index i in [0, n) with a[i] <= x (a ascending, a[0] <= x).
template <typename T>
MS_D int64_t last_le(const T *a, int64_t n, T x)
{
    int64_t lo = 0, hi = n;
    while (hi - lo > 1) {
        int64_t mid = lo + ((hi - lo) >> 1);
        if (a[mid] <= x) lo = mid;
        else hi = mid;
    }
    return lo;
}


// Multiplier of the hashed tables (the odd 32-bit constant nearest 2^32 / phi).
constexpr uint32_t HASH_MUL = 0x9E3779B1u;


// The top log2 bits (1 <= log2 <= 31) of a product id * HASH_MUL mod 2^32 (of
// the id mod 2^32: ids that differ by a multiple of 2^32 share a hash, which
// only costs work).  The product is linear in the id, so the products of
// neighbouring ids follow from one of them by adding per-axis products
// (stride_d * HASH_MUL), with no multiplication per cell.
MS_D uint32_t hash_of_product(uint32_t prod, int log2)
{
    return prod >> (32 - log2);
}

struct CellRange {
    int64_t lo[4], hi[4];
};

// Overlapped cell range of triangle t of mesh m (its box from the vertices),
// or false for a non-finite triangle.
MS_D bool tri_cells(const MeshView &m, int32_t t, const GridView &g, CellRange &r)
{
    double lo[4], hi[4];
    if (!tri_box(m, t, lo, hi)) return false;
#pragma unroll
    for (int d = 0; d < 4; ++d) {
        r.lo[d] = cell_of(lo[d], g.wlo[d], g.inv, g.n[d]);
        r.hi[d] = cell_of(hi[d], g.wlo[d], g.inv, g.n[d]);
    }
    return true;
}

MS_D int64_t range_count(const CellRange &r)
{
    return (r.hi[0] - r.lo[0] + 1) * (r.hi[1] - r.lo[1] + 1) * (r.hi[2] - r.lo[2] + 1) * (r.hi[3] - r.lo[3] + 1);
}

// The cells of a grid with twice the edge (cell index / 2 per axis), used to
// skip at once the triangles whose neighbourhood holds no cell of the other
// mesh.
MS_D void coarse_of(const CellRange &r, const int64_t n[4], CellRange &rc, int64_t nc[4])
{
#pragma unroll
    for (int d = 0; d < 4; ++d) {
        rc.lo[d] = r.lo[d] >> 1;
        rc.hi[d] = r.hi[d] >> 1;
        nc[d] = (n[d] + 1) >> 1;
    }
}

// Visit every cell of a range in lexicographic order (linear cell ids).
template <typename F>
MS_D void for_cells(const CellRange &r, const int64_t n[4], F &&f)
{
    for (int64_t c0 = r.lo[0]; c0 <= r.hi[0]; ++c0)
        for (int64_t c1 = r.lo[1]; c1 <= r.hi[1]; ++c1)
            for (int64_t c2 = r.lo[2]; c2 <= r.hi[2]; ++c2) {
                int64_t base = ((c0 * n[1] + c1) * n[2] + c2) * n[3];
                for (int64_t c3 = r.lo[3]; c3 <= r.hi[3]; ++c3) f((uint64_t)(base + c3));
            }
}

// The same with the coordinates of each cell: f(c, linear id).
template <typename F>
MS_D void for_cells_xy(const CellRange &r, const int64_t n[4], F &&f)
{
    int64_t c[4];
    for (c[0] = r.lo[0]; c[0] <= r.hi[0]; ++c[0])
        for (c[1] = r.lo[1]; c[1] <= r.hi[1]; ++c[1])
            for (c[2] = r.lo[2]; c[2] <= r.hi[2]; ++c[2]) {
                const int64_t base = ((c[0] * n[1] + c[1]) * n[2] + c[2]) * n[3];
                for (c[3] = r.lo[3]; c[3] <= r.hi[3]; ++c[3]) f(c, (uint64_t)(base + c[3]));
            }
}

// Occupancy bit of hashed cell h in a side's bit table.
MS_D uint32_t occ_bit(const uint32_t *bits, uint32_t h) { return (bits[h >> 5] >> (h & 31)) & 1u; }

// ------------------------------------------- 32-bit cell ranges (the usual grids)

// Cell of coordinate x on an axis of n < 2^31 cells (nm1 = n - 1):
// clamp(floor((x - wlo) * inv), 0, n - 1), equal to cell_of.  The clamp is
// taken in FP64 before one 32-bit conversion, and the floor is left to that
// conversion: it truncates, which is the floor on [0, n - 1], and whatever
// lies below 0 (or is NaN) clamps to 0 either way.
MS_D int32_t cell_of32(double x, double wlo, double inv, double nm1)
{
    const double t = (x - wlo) * inv;
    return (int32_t)fmin(fmax(t, 0.0), nm1);
}

// A triangle's cell range: lowest cell and extent (hi - lo) per axis.
struct Range32 {
    int32_t lo[4], e[4];
};

// 4D box of triangle t (as tri_box), its vertex ids found without an
// integer division.
MS_D bool tri_box_d(const MeshView &m, int32_t t, double lo[4], double hi[4])
{
    int32_t i1, i2, i3;
    tri_vertex_ids_d(m, t, i1, i2, i3);
    const d4 a = load_d4(m.V + 4 * (int64_t)i1), b = load_d4(m.V + 4 * (int64_t)i2),
             c = load_d4(m.V + 4 * (int64_t)i3);
    const double va[4] = {a.x, a.y, a.z, a.w}, vb[4] = {b.x, b.y, b.z, b.w}, vc[4] = {c.x, c.y, c.z, c.w};
    bool fin = true;
#pragma unroll
    for (int d = 0; d < 4; ++d) {
        lo[d] = fmin(fmin(va[d], vb[d]), vc[d]);
        hi[d] = fmax(fmax(va[d], vb[d]), vc[d]);
        fin = fin && isfinite(va[d]) && isfinite(vb[d]) && isfinite(vc[d]);
    }
    return fin;
}

// The range on the coarse grid (cell index / 2 per axis).
MS_D Range32 coarse_range(const Range32 &r)
{
    Range32 c;
#pragma unroll
    for (int d = 0; d < 4; ++d) {
        c.lo[d] = r.lo[d] >> 1;
        c.e[d] = ((r.lo[d] + r.e[d]) >> 1) - c.lo[d];
    }
    return c;
}

// True when every axis of the range has one or two cells: its cells are then
// lo + b for the positions b in {0,1}^4 (bit 3 - d of b for axis d, so that
// ascending b is the lexicographic order) with b inside the extent mask.
MS_D bool range_small(const Range32 &r) { return (r.e[0] | r.e[1] | r.e[2] | r.e[3]) <= 1; }

// Cells of a range: 2^(sum of the extents) when each is 0 or 1 (the usual
// case, a shift), else the product of the cell counts per axis.
MS_D unsigned long long range_cells(const Range32 &r)
{
    if (range_small(r)) return 1ull << (r.e[0] + r.e[1] + r.e[2] + r.e[3]);
    return (unsigned long long)(r.e[0] + 1) * (unsigned long long)(r.e[1] + 1) * (unsigned long long)(r.e[2] + 1) *
           (unsigned long long)(r.e[3] + 1);
}


// ------------------------------------------------- blocked hashed tables
//
// The occupancy tables (fine cells, and coarse cells of twice the edge) are
// hashed by blocks: a cell's 2x2x2x2 block (cell index / 2 per axis) picks a
// 16-byte line of the table -- the top lg - 4 bits of (pair's cell base +
// the block's linear id) * HASH_MUL mod 2^32 -- and the low bit of each cell index
// the byte in it.  Neighbouring cells thus share cache lines, so that the
// marks and tests of a wave touch few lines; two cells share a hashed index
// only when their blocks' hashes collide.  bs: linear-id strides of the
// blocks of the table's grid.

// Hashed index of cell c (coordinates on the table's grid).
MS_D uint32_t blocked_index(const int64_t c[4], const uint32_t bs[4], uint64_t cb, int lg)
{
    uint32_t lin = (uint32_t)cb;
#pragma unroll
    for (int d = 0; d < 4; ++d) lin += (uint32_t)(c[d] >> 1) * (uint32_t)bs[d];
    const uint32_t par = (uint32_t)((c[0] & 1) << 3 | (c[1] & 1) << 2 | (c[2] & 1) << 1 | (c[3] & 1));
    return hash_of_product(lin * HASH_MUL, lg - 4) << 4 | par;
}

// The 16 positions of a small range in Gray-code order (each step moves one
// axis by one cell): step k visits position k ^ (k >> 1).
template <int K>
struct GrayStep {
    static constexpr int b = K ^ (K >> 1);
    static constexpr int flip = K == 0 ? 0 : b ^ ((K - 1) ^ ((K - 1) >> 1));
    static constexpr int axis = flip == 8 ? 0 : flip == 4 ? 1 : flip == 2 ? 2 : 3;
    static constexpr bool up = (b & flip) != 0;
};

// Walk over the positions of a small range u: the hash product of the
// current block and the parity bits of the range's lowest cell.  Moving up
// along axis d enters the next block only from an odd cell index, so the
// per-axis steps of the product are bh[d] or 0 per range.
struct BlockWalk {
    uint32_t p;
    uint32_t up[4], dn[4];
    uint32_t par0;
};

MS_D void walk_init(BlockWalk &w, const Range32 &u, const uint32_t bs[4], const uint32_t bh[4], uint64_t cb)
{
    uint32_t lin = (uint32_t)cb;
    w.par0 = 0;
#pragma unroll
    for (int d = 0; d < 4; ++d) {
        lin += (uint32_t)(u.lo[d] >> 1) * (uint32_t)bs[d];
        const bool odd = (u.lo[d] & 1) != 0;
        w.up[d] = odd ? bh[d] : 0u;
        w.dn[d] = odd ? 0u - bh[d] : 0u;
        w.par0 |= (uint32_t)(u.lo[d] & 1) << (3 - d);
    }
    w.p = lin * HASH_MUL;
}

template <int K>
MS_D uint32_t walk_index(BlockWalk &w, int lg)
{
    if constexpr (K > 0) w.p += GrayStep<K>::up ? w.up[GrayStep<K>::axis] : w.dn[GrayStep<K>::axis];
    return hash_of_product(w.p, lg - 4) << 4 | (w.par0 ^ (uint32_t)GrayStep<K>::b);
}

// A side's occupancy table inside the byte region at base: the table at
// base + off (2^lg bytes).  The same for a bit table of 2^lg bits at w.
struct TabRef {
    uint8_t *base;
    uint32_t off;
    int lg;
};

struct BitRef {
    const uint32_t *w;
    int lg;
};

// Marks (value v) the cells of the small range u whose positions are in m.
template <int... Ks>
MS_D void mark_walk(const TabRef &t, BlockWalk w, uint32_t m, uint8_t v, std::integer_sequence<int, Ks...>)
{
    ((void)[&] {
        const uint32_t i = walk_index<Ks>(w, t.lg);
        if ((m >> GrayStep<Ks>::b) & 1u) t.base[t.off + i] = v;
    }(), ...);
}

// Both-occupied bits of the cells of the small range u whose positions are
// in m, as a mask over the positions (bit b for position b); the loads are
// independent, so they are in flight together.
template <int... Ks>
MS_D uint32_t bits_walk(const BitRef &t, BlockWalk w, uint32_t m, std::integer_sequence<int, Ks...>)
{
    uint32_t r = 0;
    ((void)[&] {
        const uint32_t i = walk_index<Ks>(w, t.lg);
        if ((m >> GrayStep<Ks>::b) & 1u) r |= ((t.w[i >> 5] >> (i & 31)) & 1u) << GrayStep<Ks>::b;
    }(), ...);
    return r;
}

// The cells of a range of any size, in lexicographic order, with their
// coordinates (Range32 form).
template <typename F>
MS_D void for_cells32(const Range32 &r, F &&f)
{
    int64_t c[4];
    for (c[0] = r.lo[0]; c[0] <= r.lo[0] + r.e[0]; ++c[0])
        for (c[1] = r.lo[1]; c[1] <= r.lo[1] + r.e[1]; ++c[1])
            for (c[2] = r.lo[2]; c[2] <= r.lo[2] + r.e[2]; ++c[2])
                for (c[3] = r.lo[3]; c[3] <= r.lo[3] + r.e[3]; ++c[3]) f(c);
}

// The positions of a small range r inside its own extent: starting from
// position 0, each axis of extent 1 adds the copy of the set moved one cell
// along it (bit 3 - d of the position).
MS_D uint32_t range_positions(const Range32 &r)
{
    uint32_t m = 1u;
    m |= (m << 8) & (0u - (uint32_t)r.e[0]);
    m |= (m << 4) & (0u - (uint32_t)r.e[1]);
    m |= (m << 2) & (0u - (uint32_t)r.e[2]);
    m |= (m << 1) & (0u - (uint32_t)r.e[3]);
    return m;
}

// Marks every cell of range r (any size).
MS_D void mark_range(const TabRef &t, const Range32 &r, const uint32_t bs[4], const uint32_t bh[4], uint64_t cb,
                     uint8_t v)
{
    if (range_small(r)) {
        BlockWalk w;
        walk_init(w, r, bs, bh, cb);
        mark_walk(t, w, range_positions(r), v, std::make_integer_sequence<int, 16>{});
        return;
    }
    for_cells32(r, [&](const int64_t *c) { t.base[t.off + blocked_index(c, bs, cb, t.lg)] = v; });
}

// Number of cells of range r whose both-occupied bit is set (any range).
MS_D uint32_t count_both(const BitRef &t, const Range32 &r, const uint32_t bs[4], const uint32_t bh[4], uint64_t cb)
{
    if (range_small(r)) {
        BlockWalk w;
        walk_init(w, r, bs, bh, cb);
        return (uint32_t)__builtin_popcount(bits_walk(t, w, range_positions(r), std::make_integer_sequence<int, 16>{}));
    }
    uint32_t n = 0;
    for_cells32(r, [&](const int64_t *c) { n += occ_bit(t.w, blocked_index(c, bs, cb, t.lg)); });
    return n;
}

// Compact cell range: lo cell per axis in 12 bits (bits 0..47), extent per
// axis in 4 bits (48..63).  Two values no range can take mark a non-finite
// triangle and a range too large to pack (recomputed from the box).
constexpr uint64_t RNG_NONFINITE = ~0ull;   // no entries: a non-finite or pruned triangle
constexpr uint64_t RNG_FROM_BOX = ~0ull - 1;

MS_D uint64_t pack_range(const CellRange &r, bool packable)
{
    if (!packable) return RNG_FROM_BOX;
    uint64_t v = 0;
#pragma unroll
    for (int d = 0; d < 4; ++d) {
        int64_t e = r.hi[d] - r.lo[d];
        if (e > 15) return RNG_FROM_BOX;
        v |= (uint64_t)r.lo[d] << (12 * d);
        v |= (uint64_t)e << (48 + 4 * d);
    }
    return v;
}

MS_D void unpack_range(uint64_t v, CellRange &r)
{
#pragma unroll
    for (int d = 0; d < 4; ++d) {
        r.lo[d] = (int64_t)((v >> (12 * d)) & 4095);
        r.hi[d] = r.lo[d] + (int64_t)((v >> (48 + 4 * d)) & 15);
    }
}

MS_D const MeshView &side_mesh(const PairDesc &P, int side) { return side ? P.B : P.A; }

// Where a triangle tile lives: pair, side, its first local triangle and the
// side's triangle count.  Every value is the same for the whole block.
struct TileLoc {
    int p, side;
    int32_t t0, n;
};

// The pair of a batch tile, found by all threads of the block at once (a
// block-wide call); the pair of a single search is 0.
template <bool ONE, int NT = BLOCK>
MS_D int tile_pair_search(const BatchView &bv, int64_t tile, int *s_p)
{
    if constexpr (ONE) {
        return 0;
    } else {
        __syncthreads();          // the previous search's result is no longer read
        for (int p = threadIdx.x; p < bv.n_pairs; p += NT)
            if (bv.tile_off[p] <= tile && tile < bv.tile_off[p + 1]) *s_p = p;
        __syncthreads();
        return __builtin_amdgcn_readfirstlane(*s_p);
    }
}

// Location of tile `tile` given a pair p with tile_off[p] <= tile (the pairs
// after p are stepped through, empty ones included).
template <bool ONE>
MS_D TileLoc tile_loc(const BatchView &bv, int64_t tile, int p)
{
    TileLoc L;
    if constexpr (!ONE)
        while (bv.tile_off[p + 1] <= tile) ++p;
    const PairDesc &P = pair_desc<ONE>(bv, p);
    const int64_t lt = tile - P.tile_off;
    L.p = p;
    L.side = lt >= P.tilesA;
    L.t0 = (int32_t)((L.side ? lt - P.tilesA : lt) * TILE_TRIS);
    L.n = L.side ? P.nB : P.nA;
    return L;
}

// Cell range of triangle t (global index gt) from its compact record, or from
// its vertices when the range did not pack.
MS_D bool range_at(const uint64_t *rng, int64_t gt, const MeshView &m, int32_t t, const GridView &g, CellRange &r)
{
    uint64_t v = rng[gt];
    if (v == RNG_NONFINITE) return false;
    if (v != RNG_FROM_BOX) {
        unpack_range(v, r);
        return true;
    }
    return tri_cells(m, t, g, r);
}


MS_D uint64_t pack_range32(const Range32 &r, bool packable)
{
    if (!packable || (r.e[0] | r.e[1] | r.e[2] | r.e[3]) > 15) return RNG_FROM_BOX;
    return (uint64_t)r.lo[0] | (uint64_t)r.lo[1] << 12 | (uint64_t)r.lo[2] << 24 | (uint64_t)r.lo[3] << 36 |
           (uint64_t)r.e[0] << 48 | (uint64_t)r.e[1] << 52 | (uint64_t)r.e[2] << 56 | (uint64_t)r.e[3] << 60;
}

MS_D void unpack_range32(uint64_t v, Range32 &r)
{
#pragma unroll
    for (int d = 0; d < 4; ++d) {
        r.lo[d] = (int32_t)((v >> (12 * d)) & 4095);
        r.e[d] = (int32_t)((v >> (48 + 4 * d)) & 15);
    }
}

// Cell range of triangle t of mesh m on grid P (32-bit form), or false for a
// non-finite triangle.
MS_D bool tri_range32(const MeshView &m, int32_t t, const PairDesc &P, Range32 &r)
{
    double lo[4], hi[4];
    if (!tri_box_d(m, t, lo, hi)) return false;
#pragma unroll
    for (int d = 0; d < 4; ++d) {
        r.lo[d] = cell_of32(lo[d], P.g.wlo[d], P.g.inv, P.nm1[d]);
        r.e[d] = cell_of32(hi[d], P.g.wlo[d], P.g.inv, P.nm1[d]) - r.lo[d];
    }
    return true;
}

// The same from the compact record written by k_mark, or from the vertices
// when the range did not pack.
MS_D bool range32_at(const uint64_t *rng, int64_t gt, const MeshView &m, int32_t t, const PairDesc &P, Range32 &r)
{
    const uint64_t v = rng[gt];
    if (v == RNG_NONFINITE) return false;
    if (v != RNG_FROM_BOX) {
        unpack_range32(v, r);
        return true;
    }
    return tri_range32(m, t, P, r);
}

// Logical block index that gives each XCD a contiguous run of the grid's
// blocks (workgroups are dealt to the 8 XCDs in turn, so block b runs on XCD
// b mod 8): neighbouring tiles, which share vertex rows, then share an L2.
MS_D int64_t xcd_block(int64_t b, int64_t nb)
{
    if (nb % 8 != 0) return b;
    return (b % 8) * (nb / 8) + b / 8;
}

// Decoupled look-back over 64-bit status words [flag:2 | value:62] of the
// tiles before `tile` (word of tile i at status[i * stride]), run by all 64
// lanes of one wave: each round reads 64 predecessors at once, finds the
// nearest inclusive prefix with a ballot and re-reads when a predecessor
// before it has not published yet.  Returns the exclusive prefix in every
// lane.
MS_D uint64_t wave_lookback_s(const uint64_t *status, int64_t stride, int64_t tile)
{
    const int lane = lane_id();
    uint64_t excl = 0;
    int64_t t = tile - 1;
    for (;;) {
        const int64_t idx = t - lane;
        const uint64_t v = idx >= 0 ? __hip_atomic_load(status + idx * stride, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)
                                    : SFLAG_PRE;
        const uint64_t fl = v & ~SVAL_MASK;
        const uint64_t pre = ballot(fl == SFLAG_PRE);
        const uint64_t zero = ballot(fl == 0);
        const int k = pre ? __builtin_ctzll(pre) : 63;
        const uint64_t upto = (2ull << k) - 1;     // lanes 0..k
        if (zero & upto) continue;
        excl += wave_sum_u64(lane <= k ? (v & SVAL_MASK) : 0ull);
        if (pre) return excl;
        t -= 64;
    }
}

MS_D uint64_t wave_lookback(const uint64_t *status, int64_t tile) { return wave_lookback_s(status, 1, tile); }

// The same over pairs of words (a, b) published together (tile i's pair at
// status[i * stride], status[i * stride + 1]): a predecessor is ready when
// both words carry the same non-zero flag.
MS_D void wave_lookback2(const uint64_t *status, int64_t stride, int64_t tile, uint64_t &ea, uint64_t &eb)
{
    const int lane = lane_id();
    ea = eb = 0;
    int64_t t = tile - 1;
    for (;;) {
        const int64_t idx = t - lane;
        uint64_t va = SFLAG_PRE, vb = SFLAG_PRE;
        if (idx >= 0) {
            va = __hip_atomic_load(status + stride * idx, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            vb = __hip_atomic_load(status + stride * idx + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        const uint64_t fa = va & ~SVAL_MASK, fb = vb & ~SVAL_MASK;
        const bool ready = fa != 0 && fa == fb;
        const uint64_t pre = ballot(ready && fa == SFLAG_PRE);
        const uint64_t notready = ballot(!ready);
        const int k = pre ? __builtin_ctzll(pre) : 63;
        const uint64_t upto = (2ull << k) - 1;
        if (notready & upto) continue;
        ea += wave_sum_u64(lane <= k ? (va & SVAL_MASK) : 0ull);
        eb += wave_sum_u64(lane <= k ? (vb & SVAL_MASK) : 0ull);
        if (pre) return;
        t -= 64;
    }
}

MS_D void publish_u64(uint64_t *w, uint64_t flag, uint64_t v)
{
    __hip_atomic_store(w, flag | v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

template <int NT = BLOCK, typename T>
MS_D T block_sum(T v, T *s_tmp)
{
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    __syncthreads();
    if (lane_id() == 0) s_tmp[threadIdx.x / WAVE] = v;
    __syncthreads();
    T t = 0;
    for (int i = 0; i < NT / WAVE; ++i) t += s_tmp[i];
    return t;
}

// Exclusive scan of one value per thread over the block (NT threads); *total = sum.
template <int NT = BLOCK, typename T>
MS_D T block_excl(T v, T *s_tmp, T *total)
{
    const int lane = lane_id(), w = threadIdx.x / WAVE;
    T x = v;
    for (int o = 1; o < WAVE; o <<= 1) {
        T y = __shfl_up(x, o);
        if (lane >= o) x += y;
    }
    __syncthreads();
    if (lane == WAVE - 1) s_tmp[w] = x;
    __syncthreads();
    T add = 0, tot = 0;
    for (int i = 0; i < NT / WAVE; ++i) {
        T t = s_tmp[i];
        if (i < w) add += t;
        tot += t;
    }
    *total = tot;
    return add + x - v;
}

// ---------------------------------------------------------------- kernels

// Counters to clear at the start of a search (by k_mark's first block) or of
// the all-pairs test (by k_prepare).
struct ClearSpec {
    search_stats_t *stats;
    uint64_t *w[3];    int64_t n[3];             // look-back words, counters
};

__global__ void __launch_bounds__(BLOCK) k_prepare(ClearSpec c)
{
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const int64_t g0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c.stats && g0 < (int64_t)(sizeof(search_stats_t) / 8)) ((int64_t *)c.stats)[g0] = 0;
#pragma unroll
    for (int k = 0; k < 3; ++k)
        for (int64_t i = g0; i < c.n[k]; i += stride) c.w[k][i] = 0;
}

// Occupancy marks carry the search's epoch value v in 1..255 (the search
// count mod 255, plus one), so that the tables need no clearing between
// searches: a byte counts as set only when it holds v.  The search whose v
// wraps back to 1 finds the tables cleared by the one before it.  A byte
// left over from another use of the workspace can only add occupancy, which
// adds work but never changes a result.
MS_D uint8_t epoch_value(const uint64_t *epoch) { return (uint8_t)(*epoch % 255u + 1u); }

// ---------------------------------------------------------------- quad tiles
//
// k_mark and k_keys give each thread one quad of the vertex grid, i.e. both
// its triangles: T1 = (W(i+1,k), W(i,k), W(i,k+1)) and T2 = (W(i,k+1),
// W(i+1,k+1), W(i+1,k)) share the vertices W(i+1,k) and W(i,k+1).  The cell
// map is monotone, so a triangle's cell range is the min / max of its
// vertices' cells: each of the four vertices is converted once.

// The positions of the range u (range_small) that lie in range r, a range
// inside u: r's own positions, moved by r's offset from u's lowest cell.
MS_D uint32_t position_mask(const Range32 &u, const Range32 &r)
{
    const uint32_t sh = (uint32_t)(r.lo[0] - u.lo[0]) << 3 | (uint32_t)(r.lo[1] - u.lo[1]) << 2 |
                        (uint32_t)(r.lo[2] - u.lo[2]) << 1 | (uint32_t)(r.lo[3] - u.lo[3]);
    return range_positions(r) << sh;
}

// Smallest range holding both ranges.
MS_D Range32 range_union(const Range32 &a, const Range32 &b)
{
    Range32 u;
#pragma unroll
    for (int d = 0; d < 4; ++d) {
        u.lo[d] = min(a.lo[d], b.lo[d]);
        u.e[d] = max(a.lo[d] + a.e[d], b.lo[d] + b.e[d]) - u.lo[d];
    }
    return u;
}

// Marks, in one pass over the 16 positions of their union, the cells of the
// quad's finite triangles (ok1, ok2); a union wider than two cells on some
// axis marks each triangle on its own.
MS_D void mark_quad(const TabRef &t, const Range32 &r1, bool ok1, const Range32 &r2, bool ok2,
                    const uint32_t bs[4], const uint32_t bh[4], uint64_t cb, uint8_t v)
{
    if (!ok1 && !ok2) return;
    const Range32 u = ok1 && ok2 ? range_union(r1, r2) : (ok1 ? r1 : r2);
    if (range_small(u)) {
        const uint32_t m = (ok1 ? position_mask(u, r1) : 0u) | (ok2 ? position_mask(u, r2) : 0u);
        BlockWalk w;
        walk_init(w, u, bs, bh, cb);
        mark_walk(t, w, m, v, std::make_integer_sequence<int, 16>{});
        return;
    }
    if (ok1) mark_range(t, r1, bs, bh, cb, v);
    if (ok2) mark_range(t, r2, bs, bh, cb, v);
}

// Cells of the four vertices of a quad (a = W(i,k), b = W(i+1,k),
// c = W(i,k+1), d = W(i+1,k+1)) and whether each vertex is finite.
struct QuadVerts {
    int32_t c[4][4];
    bool fin[4];
};

// Whether the box of the triangle with vertices u, v, w meets the box ob
// (lo[4], hi[4]): closed intervals, per axis.
MS_D bool tri_meets_box(const d4 &u, const d4 &v, const d4 &w, const double *ob)
{
    const double a[4] = {u.x, u.y, u.z, u.w}, b[4] = {v.x, v.y, v.z, v.w}, c[4] = {w.x, w.y, w.z, w.w};
    bool meet = true;
#pragma unroll
    for (int d = 0; d < 4; ++d) {
        const double lo = fmin(fmin(a[d], b[d]), c[d]), hi = fmax(fmax(a[d], b[d]), c[d]);
        meet = meet && lo <= ob[4 + d] && ob[d] <= hi;
    }
    return meet;
}

// ob: the other mesh's box (MS_SEARCH_PRUNE) or null; keep1 / keep2: the
// quad's triangles meet it (always true without pruning).
MS_D void quad_vertices(const MeshView &m, int32_t q, const PairDesc &P, QuadVerts &qv, const double *ob,
                        bool &keep1, bool &keep2)
{
    int32_t k, i;
    quad_row_col(m, q, k, i);
    int32_t i1 = i + 1;
    if (i1 == m.n_theta_v) i1 = 0;
    const int32_t r0 = k * m.n_theta_v, r1 = r0 + m.n_theta_v;
    const int32_t id[4] = {r0 + i, r0 + i1, r1 + i, r1 + i1};
    d4 x[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) x[j] = load_d4(m.V + 4 * (int64_t)id[j]);
    keep1 = keep2 = true;
    if (ob) {
        keep1 = tri_meets_box(x[1], x[0], x[2], ob);    // T1 = (b, a, c)
        keep2 = tri_meets_box(x[2], x[3], x[1], ob);    // T2 = (c, d, b)
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const double w[4] = {x[j].x, x[j].y, x[j].z, x[j].w};
        qv.fin[j] = (int)isfinite(w[0]) & (int)isfinite(w[1]) & (int)isfinite(w[2]) & (int)isfinite(w[3]);
#pragma unroll
        for (int d = 0; d < 4; ++d) qv.c[j][d] = cell_of32(w[d], P.g.wlo[d], P.g.inv, P.nm1[d]);
    }
}

// The cell ranges of the quad's triangles T1 (vertices b, a, c) and T2
// (c, d, b); ok1 / ok2: the triangle is finite.
MS_D void quad_ranges(const QuadVerts &qv, Range32 &r1, bool &ok1, Range32 &r2, bool &ok2)
{
#pragma unroll
    for (int d = 0; d < 4; ++d) {
        const int32_t mn = min(qv.c[1][d], qv.c[2][d]), mx = max(qv.c[1][d], qv.c[2][d]);
        r1.lo[d] = min(mn, qv.c[0][d]);
        r1.e[d] = max(mx, qv.c[0][d]) - r1.lo[d];
        r2.lo[d] = min(mn, qv.c[3][d]);
        r2.e[d] = max(mx, qv.c[3][d]) - r2.lo[d];
    }
    ok1 = qv.fin[0] & qv.fin[1] & qv.fin[2];
    ok2 = qv.fin[1] & qv.fin[2] & qv.fin[3];
}

// World-bound pruning (MS_SEARCH_PRUNE, Sec. 6.2.1): the box of each mesh of
// each pair over its finite vertices (lo = +inf, hi = -inf without one), one
// block per (pair, side), written to pbox[8 (2 p + side) ..] as lo[4], hi[4].
// Every finite triangle lies in it.  Pairs without the flag write nothing.
constexpr int BOUNDS_BLOCK = 1024;

template <bool ONE>
__global__ void __launch_bounds__(BOUNDS_BLOCK) k_bounds(BatchView bv, double *pbox)
{
    __shared__ double s_red[8][BOUNDS_BLOCK / WAVE];
    const int p = (int)(blockIdx.x >> 1), side = (int)(blockIdx.x & 1);
    const PairDesc &P = pair_desc<ONE>(bv, p);
    if (!P.prune) return;
    const MeshView &m = side_mesh(P, side);
    double v[8];
#pragma unroll
    for (int d = 0; d < 4; ++d) {
        v[d] = INFINITY;
        v[4 + d] = -INFINITY;
    }
    const int64_t nv = m.n_tris > 0 ? (int64_t)m.n_theta_v * m.n_s_v : 0;
    constexpr int U = 4;     // loads in flight per thread
    for (int64_t base = 0; base < nv; base += (int64_t)U * BOUNDS_BLOCK) {
        d4 x[U];
        bool in[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t j = base + (int64_t)u * BOUNDS_BLOCK + threadIdx.x;
            in[u] = j < nv;
            if (in[u]) x[u] = load_d4(m.V + 4 * j);
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            if (!in[u]) continue;
            const double w[4] = {x[u].x, x[u].y, x[u].z, x[u].w};
            if (!(isfinite(w[0]) && isfinite(w[1]) && isfinite(w[2]) && isfinite(w[3]))) continue;
#pragma unroll
            for (int d = 0; d < 4; ++d) {
                v[d] = fmin(v[d], w[d]);
                v[4 + d] = fmax(v[4 + d], w[d]);
            }
        }
    }
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        for (int o = WAVE / 2; o > 0; o >>= 1) {
            const double u = __shfl_xor(v[k], o);
            v[k] = k < 4 ? fmin(v[k], u) : fmax(v[k], u);
        }
        if (lane_id() == 0) s_red[k][threadIdx.x / WAVE] = v[k];
    }
    __syncthreads();
    if (threadIdx.x < 8) {
        const int k = threadIdx.x;
        double r = s_red[k][0];
        for (int w = 1; w < BOUNDS_BLOCK / WAVE; ++w) r = k < 4 ? fmin(r, s_red[k][w]) : fmax(r, s_red[k][w]);
        pbox[8 * (int64_t)blockIdx.x + k] = r;
    }
}

// Occupancy: one byte per hashed global cell and side, set with plain stores
// (all writers store the same value), fine and coarse.  Stores each
// triangle's compact cell range and per-block entry / non-finite totals.
// Block 0 also clears the search's counters.  One thread per quad; each
// block takes a contiguous run of quad tiles, and the runs of neighbouring
// blocks share an XCD (xcd_block).
template <bool ONE, bool C32>
__global__ void __launch_bounds__(BLOCK) k_mark(BatchView bv, uint8_t *flags, const uint64_t *epoch, uint64_t *rng,
                                                const double *pbox, unsigned long long *partial, ClearSpec c)
{
    __shared__ unsigned long long s_tmp[BLOCK / WAVE];
    if (blockIdx.x == 0) {
        if (threadIdx.x < (int)(sizeof(search_stats_t) / 8)) ((int64_t *)c.stats)[threadIdx.x] = 0;
#pragma unroll
        for (int k = 0; k < 3; ++k)
            for (int64_t i = threadIdx.x; i < c.n[k]; i += BLOCK) c.w[k][i] = 0;
    }
    const uint8_t v = epoch_value(epoch);
    unsigned long long all = 0, bad = 0;
    const int lg = bv.bm_log2, lc = bv.bc_log2;
    const int64_t ntiles = bv.n_tiles;
    const int64_t per = ceil_div(ntiles, gridDim.x);
    const int64_t t0 = xcd_block(blockIdx.x, gridDim.x) * per;
    const int64_t t1 = t0 + per < ntiles ? t0 + per : ntiles;
    __shared__ int s_p;
    int p = t0 < t1 ? tile_pair_search<ONE>(bv, t0, &s_p) : 0;
    for (int64_t tile = t0; tile < t1; ++tile) {
        const TileLoc L = tile_loc<ONE>(bv, tile, p);
        p = L.p;
        const int32_t q = (L.t0 >> 1) + (int32_t)threadIdx.x;
        if (2 * q >= L.n) continue;
        const int64_t g = tile * TILE_TRIS + 2 * (int64_t)threadIdx.x;
        const PairDesc &P = pair_desc<ONE>(bv, L.p);
        const MeshView &m = side_mesh(P, L.side);
        uint8_t *fine = flags + ((size_t)L.side << lg);
        uint8_t *coarse = flags + ((size_t)2 << lg) + ((size_t)L.side << lc);
        // the other mesh's box when pruning: a triangle that misses it is
        // counted (its cells) but neither marked nor keyed
        const double *ob = P.prune ? pbox + 8 * (2 * (int64_t)L.p + (1 - L.side)) : nullptr;
        if constexpr (C32) {
            QuadVerts qv;
            bool keep1, keep2;
            quad_vertices(m, q, P, qv, ob, keep1, keep2);
            Range32 r1, r2;
            bool ok1, ok2;
            quad_ranges(qv, r1, ok1, r2, ok2);
            const bool k1 = ok1 && keep1, k2 = ok2 && keep2;
            ulonglong2 rr;
            rr.x = k1 ? pack_range32(r1, bv.packable != 0) : RNG_NONFINITE;
            rr.y = k2 ? pack_range32(r2, bv.packable != 0) : RNG_NONFINITE;
            *reinterpret_cast<ulonglong2 *>(rng + g) = rr;
            bad += (unsigned long long)(!ok1) + (unsigned long long)(!ok2);
            if (ok1) all += range_cells(r1);
            if (ok2) all += range_cells(r2);
            mark_quad(TabRef{flags, (uint32_t)L.side << lg, lg}, r1, k1, r2, k2, P.fbs, P.fbh, P.cell_base, v);
            mark_quad(TabRef{flags, ((uint32_t)2 << lg) + ((uint32_t)L.side << lc), lc}, coarse_range(r1), k1,
                      coarse_range(r2), k2, P.cbs, P.cbh, P.cell_base, v);
        } else {
            // grids of 2^31 cells or more along an axis: 64-bit cells, one triangle at a time
            const uint64_t cb = P.cell_base;
            for (int h = 0; h < 2; ++h) {
                CellRange r;
                if (!tri_cells(m, 2 * q + h, P.g, r)) {
                    ++bad;
                    rng[g + h] = RNG_NONFINITE;
                    continue;
                }
                all += (unsigned long long)range_count(r);
                if (ob) {
                    double lo[4], hi[4];
                    tri_box(m, 2 * q + h, lo, hi);
                    bool meet = true;
#pragma unroll
                    for (int d = 0; d < 4; ++d) meet = meet && lo[d] <= ob[4 + d] && ob[d] <= hi[d];
                    if (!meet) {
                        rng[g + h] = RNG_NONFINITE;
                        continue;
                    }
                }
                rng[g + h] = RNG_FROM_BOX;
                for_cells_xy(r, P.g.n, [&](const int64_t *c, uint64_t) { fine[blocked_index(c, P.fbs, cb, lg)] = v; });
                CellRange rc;
                int64_t nc[4];
                coarse_of(r, P.g.n, rc, nc);
                for_cells_xy(rc, nc, [&](const int64_t *c, uint64_t) { coarse[blocked_index(c, P.cbs, cb, lc)] = v; });
            }
        }
    }
    all = block_sum(all, s_tmp);
    bad = block_sum(bad, s_tmp);
    if (threadIdx.x == 0) {
        partial[2 * blockIdx.x] = all;
        partial[2 * blockIdx.x + 1] = bad;
    }
}

// 32 occupancy bytes -> one word of flags (bytes equal to v).
MS_D uint32_t byte_mask(const uint8_t *f, uint32_t v)
{
    const uint4 *p = reinterpret_cast<const uint4 *>(f);
    const uint4 a = p[0], b = p[1];
    const uint32_t q[8] = {a.x, a.y, a.z, a.w, b.x, b.y, b.z, b.w};
    uint32_t m = 0;
#pragma unroll
    for (int i = 0; i < 8; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) m |= (uint32_t)(((q[i] >> (8 * j)) & 0xffu) == v) << (4 * i + j);
    return m;
}

// The hashed cells that both meshes occupy, as bit tables (fine, then
// coarse): the AND of the two sides' occupancy bytes.  Every set fine bit is
// a cell group, whose entry counters and several-cells flag are cleared here.
__global__ void __launch_bounds__(BLOCK) k_pack(const uint8_t *flags, const uint64_t *epoch, int bm_log2, int bc_log2,
                                                uint32_t *both, uint64_t *grp, uint32_t *mix, int64_t n_fwords,
                                                int64_t n_cwords)
{
    const uint32_t v = epoch_value(epoch);
    const size_t side = (size_t)1 << bm_log2, cside = (size_t)1 << bc_log2;
    const int64_t n = n_fwords + n_cwords;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t w = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; w < n; w += stride) {
        if (w < n_fwords) {
            uint32_t m = byte_mask(flags + 32 * w, v) & byte_mask(flags + side + 32 * w, v);
            both[w] = m;
            while (m) {
                const int64_t h = 32 * w + __builtin_ctz(m);
                grp[h] = 0;
                mix[h] = 0;
                m &= m - 1;
            }
        } else {
            const uint8_t *c = flags + 2 * side + 32 * (w - n_fwords);
            both[w] = byte_mask(c, v) & byte_mask(c + cside, v);
        }
    }
}

// Whether any coarse cell of the range is occupied by both meshes (a
// triangle whose coarse neighbourhood holds no cell of the other mesh has no
// entry at all).
MS_D bool coarse_any(const BatchView &bv, const uint32_t *cboth, const PairDesc &P, const Range32 &rc)
{
    return count_both(BitRef{cboth, bv.bc_log2}, rc, P.cbs, P.cbh, P.cell_base) != 0;
}

struct KeysOut {
    uint64_t *ent;                // [cell | side | triangle]
    int32_t *epair;               // pair of the entry (batch)
    uint32_t *erank;              // rank of the entry among its group's entries of its side
    uint32_t *ehash;              // the entry's hashed cell (its group)
    int64_t cap;
    unsigned long long *n_keys;   // entries reserved (cleared)
    uint32_t *grp;                // per hashed cell h: [2 h] A entries, [2 h + 1] B entries
    uint64_t *own;                // per hashed cell: the cell of one of its entries (any)
    search_stats_t *stats;
};

// Entries of each triangle: the cells of its range whose hashed cell both
// meshes occupy (a cell holding one mesh only cannot hold a pair), after the
// same test on the coarse cells.  One thread per triangle (KEYS_BLOCK =
// TILE_TRIS threads: one tile per block).  Each block counts the entries of
// its tile, reserves that many output slots with one atomic add (blocks
// without entries take none) and writes the entries, listed in LDS first
// when they are few enough, so that all threads write them together; every
// stored entry is counted in its group and side (its rank there is kept for
// the placement, its hashed cell with it), and the first of each side
// leaves its cell as the group's sample.  One block more than the tiles
// sums k_mark's per-block totals and clears the enumeration's counter
// lines, beside the others.
constexpr int KEYS_BLOCK = TILE_TRIS;
constexpr int KEYS_STAGE = 2048;          // entries of a block staged in LDS (more: each thread writes its own)

struct KeysTotals {
    const unsigned long long *mark_partial;   // per k_mark block: entries, non-finite triangles
    int n_mark_partial;
    unsigned long long *shards;               // the enumeration's counter lines, cleared here
};

// Eight waves per SIMD (at most 64 registers; the batch forms spill a few
// bytes): its blocks wait on dependent loads and atomics, and more of them
// in flight shortened the family batch's k_keys from 648 to 609 us.
template <bool ONE, bool C32>
__global__ void __launch_bounds__(KEYS_BLOCK) __attribute__((amdgpu_waves_per_eu(8, 8))) k_keys(BatchView bv, const uint32_t *both, const uint64_t *rng, KeysOut o,
                                                     KeysTotals kt)
{
    __shared__ uint64_t s_tmp[KEYS_BLOCK / WAVE];
    __shared__ unsigned long long s_blk0;
    __shared__ uint32_t s_kh[KEYS_STAGE];     // staged entries: hashed cell, cell, thread
    __shared__ uint64_t s_kc[KEYS_STAGE];
    __shared__ uint16_t s_kt[KEYS_STAGE];
    const int lg = bv.bm_log2, lc = bv.bc_log2;
    const uint32_t *cboth = both + ((size_t)1 << lg) / 32;
    const int64_t tile = blockIdx.x;
    if (tile >= bv.n_tiles) {
        if (tile == (bv.n_tiles > 0 ? bv.n_tiles : 1)) {
            unsigned long long all = 0, bad = 0;
            for (int i0 = threadIdx.x; i0 < kt.n_mark_partial; i0 += 4 * KEYS_BLOCK) {
                unsigned long long a[4] = {0, 0, 0, 0}, b[4] = {0, 0, 0, 0};
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const int i = i0 + u * KEYS_BLOCK;
                    if (i < kt.n_mark_partial) {
                        a[u] = kt.mark_partial[2 * i];
                        b[u] = kt.mark_partial[2 * i + 1];
                    }
                }
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    all += a[u];
                    bad += b[u];
                }
            }
            all = block_sum<KEYS_BLOCK>(all, (unsigned long long *)s_tmp);
            bad = block_sum<KEYS_BLOCK>(bad, (unsigned long long *)s_tmp);
            if (threadIdx.x == 0) {
                o.stats->n_entries_all = (int64_t)all;
                o.stats->n_nonfinite = (int64_t)bad;
            }
            if (threadIdx.x < STAT_SHARDS * SHARD_WORDS) kt.shards[threadIdx.x] = 0;
        }
        return;
    }
    __shared__ int s_p;
    const TileLoc L = tile_loc<ONE>(bv, tile, tile_pair_search<ONE, KEYS_BLOCK>(bv, tile, &s_p));
    const int32_t t = L.t0 + (int32_t)threadIdx.x;
    const int64_t g = tile * TILE_TRIS + threadIdx.x;
    const PairDesc &P = pair_desc<ONE>(bv, L.p);
    const MeshView &m = side_mesh(P, L.side);
    const uint64_t cb = P.cell_base;
    uint32_t cnt = 0;
    Range32 r;
    if (t < L.n) {
        if constexpr (C32) {
            if (range32_at(rng, g, m, t, P, r) && coarse_any(bv, cboth, P, coarse_range(r)))
                cnt = count_both(BitRef{both, lg}, r, P.fbs, P.fbh, cb);
        } else {
            CellRange rr;
            if (range_at(rng, g, m, t, P.g, rr)) {
                CellRange rc;
                int64_t nc[4];
                coarse_of(rr, P.g.n, rc, nc);
                uint32_t any = 0;
                for_cells_xy(rc, nc, [&](const int64_t *c, uint64_t) {
                    any |= occ_bit(cboth, blocked_index(c, P.cbs, cb, lc));
                });
                if (any)
                    for_cells_xy(rr, P.g.n, [&](const int64_t *c, uint64_t) {
                        cnt += occ_bit(both, blocked_index(c, P.fbs, cb, lg));
                    });
            }
        }
    }
    uint64_t btotal;
    const uint64_t texcl = block_excl<KEYS_BLOCK>((uint64_t)cnt, s_tmp, &btotal);
    if (btotal == 0) return;                      // uniform: every thread saw the same total
    if (threadIdx.x == 0) {
        const unsigned long long b0 = atomicAdd(o.n_keys, (unsigned long long)btotal);
        s_blk0 = b0;
        if ((int64_t)(b0 + btotal) > o.cap) atomicOr((unsigned long long *)&o.stats->overflow, 1ull);
    }
    __syncthreads();
    const uint64_t blk0 = s_blk0;
    if (btotal <= KEYS_STAGE) {
        // the block's entries through LDS: each thread lists its own at its
        // offset, then every thread takes every KEYS_BLOCK-th entry, so
        // that the group counters are advanced by all threads at once and
        // the entry stores are contiguous
        if (cnt) {
            uint32_t k = (uint32_t)texcl;
            auto stage = [&](uint64_t gc, uint32_t hh) {
                s_kh[k] = hh;
                s_kc[k] = gc;
                s_kt[k] = (uint16_t)threadIdx.x;
                ++k;
            };
            if constexpr (C32) {
                for_cells32(r, [&](const int64_t *c) {
                    const uint32_t hh = blocked_index(c, P.fbs, cb, lg);
                    if (occ_bit(both, hh))
                        stage(cb + (uint64_t)c[0] * P.st[0] + (uint64_t)c[1] * P.st[1] + (uint64_t)c[2] * P.st[2] +
                                  (uint64_t)c[3],
                              hh);
                });
            } else {
                CellRange rr;
                range_at(rng, g, m, t, P.g, rr);
                for_cells_xy(rr, P.g.n, [&](const int64_t *c, uint64_t cell) {
                    const uint32_t hh = blocked_index(c, P.fbs, cb, lg);
                    if (occ_bit(both, hh)) stage(cb + cell, hh);
                });
            }
        }
        __syncthreads();
        const uint64_t side_bits = (uint64_t)L.side << bv.kl.tb;
        for (uint32_t i = threadIdx.x; i < (uint32_t)btotal; i += KEYS_BLOCK) {
            const int64_t pos = (int64_t)(blk0 + i);
            if (pos >= o.cap) break;           // only stored entries are counted in their group
            const uint32_t hh = s_kh[i];
            const uint64_t gc = s_kc[i];
            const uint32_t rank = atomicAdd(&o.grp[2 * (size_t)hh + L.side], 1u);
            o.erank[pos] = rank;
            o.ehash[pos] = hh;
            if (rank == 0) o.own[hh] = gc;     // the first entry of each side: the group's sample
            o.ent[pos] = (gc << bv.kl.cell_shift) | side_bits | (uint64_t)(uint32_t)(L.t0 + s_kt[i]);
            if (!ONE) o.epair[pos] = L.p;
        }
        return;
    }
    if (cnt == 0) return;
    int64_t pos = (int64_t)(blk0 + texcl);
    const uint64_t low = ((uint64_t)L.side << bv.kl.tb) | (uint64_t)t;
    // only stored entries are counted in their group; the first entry of
    // each side leaves its cell as the group's sample
    auto put = [&](uint64_t gc, uint32_t hh) {
        if (pos < o.cap) {
            const uint32_t rank = atomicAdd(&o.grp[2 * (size_t)hh + L.side], 1u);
            o.erank[pos] = rank;
            o.ehash[pos] = hh;
            if (rank == 0) o.own[hh] = gc;
            o.ent[pos] = (gc << bv.kl.cell_shift) | low;
            if (!ONE) o.epair[pos] = L.p;
        }
        ++pos;
    };
    if constexpr (C32) {
        for_cells32(r, [&](const int64_t *c) {
            const uint32_t hh = blocked_index(c, P.fbs, cb, lg);
            if (occ_bit(both, hh))
                put(cb + (uint64_t)c[0] * P.st[0] + (uint64_t)c[1] * P.st[1] + (uint64_t)c[2] * P.st[2] + (uint64_t)c[3],
                    hh);
        });
    } else {
        CellRange rr;
        range_at(rng, g, m, t, P.g, rr);
        for_cells_xy(rr, P.g.n, [&](const int64_t *c, uint64_t cell) {
            const uint32_t hh = blocked_index(c, P.fbs, cb, lg);
            if (occ_bit(both, hh)) put(cb + cell, hh);
        });
    }
}

// A kept cell group: its entries, A's then B's, from `start`; h is its
// hashed cell.
struct CellRec {
    int64_t start;
    int32_t nA, nB;
    int64_t h;
};

// First index in [lo, hi) whose key is >= k (keys ascending).
MS_D int64_t lower_bound_u64(const uint64_t *a, int64_t lo, int64_t hi, uint64_t k)
{
    while (lo < hi) {
        int64_t mid = lo + ((hi - lo) >> 1);
        if (a[mid] < k) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

// The groups holding both meshes, in order of their hashed cells.  A group
// is kept when it has A and B entries; kept groups get consecutive records,
// entry ranges (sum of nA + nB before them) and slot offsets (sum of
// nA * nB), from one block scan and a decoupled look-back per tile of
// GROUP_WORDS words of the both-occupied table.  Each group's counter word
// becomes its two placement cursors: start (A entries) in the low half,
// start + nA (B entries) in the high half; a group not kept gets the
// cursors' high bits set.
constexpr int GROUP_ITEMS = 16;                  // words of the fine table per thread
constexpr int GROUP_WORDS = BLOCK * GROUP_ITEMS;
constexpr int GROUP_SEG = 8;                     // set bits per thread when the tile's are listed
constexpr int GROUP_LIST = BLOCK * GROUP_SEG;
constexpr uint64_t GRP_DROP = 0x8000000080000000ull;

struct GroupsOut {
    const uint32_t *both;     // fine both-occupied bits
    uint64_t *grp;            // per hashed cell: counters in, cursors out
    int64_t n_fwords;
    CellRec *cells;           // kept groups
    int64_t *pstart;          // kept groups + 1
    int64_t *kept;            // [0] kept groups, [1] their slots
    uint64_t *stat;           // 2 look-back words per tile (cleared)
    uint32_t *tile_ctr;       // (cleared)
    search_stats_t *stats;
};

// Tiles at most this many take their tile from the block index: every block
// is then resident at once (one per CU suffices), so the look-back cannot wait
// on a tile that never starts; more tiles take theirs from a counter.
constexpr int GROUP_DIRECT_TILES = 256;

__global__ void __launch_bounds__(BLOCK) k_groups(GroupsOut o)
{
    __shared__ uint64_t s_tk[BLOCK / WAVE], s_tp[BLOCK / WAVE], s_tn[BLOCK / WAVE];
    __shared__ uint64_t s_kbase, s_pbase;
    __shared__ uint32_t s_tile;
    __shared__ uint32_t s_list[GROUP_LIST];
    const int64_t ntiles = (o.n_fwords + GROUP_WORDS - 1) / GROUP_WORDS;
    const bool direct = ntiles <= GROUP_DIRECT_TILES;
    for (int round = 0;; ++round) {
        int64_t tile;
        if (direct) {
            if (round > 0) break;
            tile = blockIdx.x;
        } else {
            if (threadIdx.x == 0) s_tile = atomicAdd(o.tile_ctr, 1u);
            __syncthreads();
            tile = s_tile;
            __syncthreads();
        }
        if (tile >= ntiles) break;
        const int64_t w0 = tile * GROUP_WORDS + (int64_t)threadIdx.x * GROUP_ITEMS;
        uint32_t m[GROUP_ITEMS];
        uint64_t kc = 0, pc = 0;     // (kept << 32) | entries; slots
        uint32_t nb = 0;
#pragma unroll
        for (int j = 0; j < GROUP_ITEMS; ++j) {
            m[j] = w0 + j < o.n_fwords ? o.both[w0 + j] : 0u;
            nb += (uint32_t)__builtin_popcount(m[j]);
        }
        // The tile's set bits, in order, split evenly over the threads
        // (GROUP_SEG at most each), so that every thread issues the loads of
        // its groups' counters together; a denser tile is walked word by
        // word by each thread.
        uint64_t nbt;
        const uint64_t nboff = block_excl((uint64_t)nb, s_tn, &nbt);
        const bool listed = nbt <= (uint64_t)GROUP_LIST;
        uint32_t seg0 = 0, segn = 0;
        uint32_t gh[GROUP_SEG];
        uint64_t gv[GROUP_SEG];
        if (listed) {
            uint32_t k = (uint32_t)nboff;
#pragma unroll
            for (int j = 0; j < GROUP_ITEMS; ++j)
                for (uint32_t q = m[j]; q; q &= q - 1) s_list[k++] = (uint32_t)(32 * (w0 + j)) + (uint32_t)__builtin_ctz(q);
            __syncthreads();
            const uint32_t per = ((uint32_t)nbt + BLOCK - 1) / BLOCK;
            seg0 = threadIdx.x * per;
            segn = seg0 < (uint32_t)nbt ? ((uint32_t)nbt - seg0 < per ? (uint32_t)nbt - seg0 : per) : 0u;
#pragma unroll
            for (int k2 = 0; k2 < GROUP_SEG; ++k2) {
                gh[k2] = (uint32_t)k2 < segn ? s_list[seg0 + k2] : 0u;
                gv[k2] = (uint32_t)k2 < segn ? o.grp[gh[k2]] : 0ull;
            }
#pragma unroll
            for (int k2 = 0; k2 < GROUP_SEG; ++k2) {
                const uint64_t a = gv[k2] & 0xffffffffull, b = gv[k2] >> 32;
                if (a && b) {
                    kc += (1ull << 32) + a + b;
                    pc += a * b;
                }
            }
        } else {
#pragma unroll
            for (int j = 0; j < GROUP_ITEMS; ++j) {
                for (uint32_t q = m[j]; q; q &= q - 1) {
                    const uint64_t v = o.grp[32 * (w0 + j) + __builtin_ctz(q)];
                    const uint64_t a = v & 0xffffffffull, b = v >> 32;
                    if (a && b) {
                        kc += (1ull << 32) + a + b;
                        pc += a * b;
                    }
                }
            }
        }
        uint64_t ktot, ptot;
        const uint64_t kex = block_excl(kc, s_tk, &ktot);
        const uint64_t pex = block_excl(pc, s_tp, &ptot);
        if (threadIdx.x < WAVE) {
            uint64_t kb = 0, pb = 0;
            uint64_t *sk = o.stat + 2 * tile, *sp = sk + 1;
            if (tile == 0) {
                if (threadIdx.x == 0) {
                    publish_u64(sp, SFLAG_PRE, ptot);
                    publish_u64(sk, SFLAG_PRE, ktot);
                }
            } else {
                if (threadIdx.x == 0) {
                    publish_u64(sp, SFLAG_AGG, ptot);
                    publish_u64(sk, SFLAG_AGG, ktot);
                }
                wave_lookback2(o.stat, 2, tile, kb, pb);
                if (threadIdx.x == 0) {
                    publish_u64(sp, SFLAG_PRE, pb + ptot);
                    publish_u64(sk, SFLAG_PRE, kb + ktot);
                }
            }
            if (threadIdx.x == 0) {
                s_kbase = kb;
                s_pbase = pb;
                if (tile == ntiles - 1) {
                    const int64_t nk = (int64_t)((kb + ktot) >> 32), P = (int64_t)(pb + ptot);
                    o.kept[0] = nk;
                    o.kept[1] = P;
                    o.pstart[nk] = P;
                    o.stats->n_groups = nk;
                    o.stats->n_group_slots = P;
                }
            }
        }
        __syncthreads();
        uint64_t kr = s_kbase + kex, pr = s_pbase + pex;
        // each group's record and cursors, in the order of the scan
        auto place = [&](int64_t h, uint64_t v) {
            uint64_t *gw = o.grp + h;
            const uint64_t a = v & 0xffffffffull, b = v >> 32;
            if (a && b) {
                const int64_t ki = (int64_t)(kr >> 32), start = (int64_t)(kr & 0xffffffffull);
                CellRec cr;
                cr.start = start;
                cr.nA = (int32_t)a;
                cr.nB = (int32_t)b;
                cr.h = h;
                o.cells[ki] = cr;
                o.pstart[ki] = (int64_t)pr;
                *gw = (((uint64_t)start + a) << 32) | (uint64_t)start;
                kr += (1ull << 32) + a + b;
                pr += a * b;
            } else {
                *gw = GRP_DROP;
            }
        };
        if (listed) {
#pragma unroll
            for (int k2 = 0; k2 < GROUP_SEG; ++k2)
                if ((uint32_t)k2 < segn) place(gh[k2], gv[k2]);
        } else {
#pragma unroll
            for (int j = 0; j < GROUP_ITEMS; ++j)
                for (uint32_t q = m[j]; q; q &= q - 1) {
                    const int64_t h = 32 * (w0 + j) + __builtin_ctz(q);
                    place(h, o.grp[h]);
                }
        }
        __syncthreads();
    }
}

// Entries to their group's range: the group's start for the entry's side
// plus the entry's rank among them (A entries first), each with its
// triangle's box (from the vertices), so that the enumeration reads the box
// with the entry.  Entries of groups holding one mesh only are dropped.  An
// entry whose cell differs from its group's sample flags the group as
// holding several cells.  When the next search's epoch value wraps to 1,
// the occupancy tables are cleared here.
template <bool ONE>
__global__ void __launch_bounds__(BLOCK) k_scatter(BatchView bv, const uint64_t *ent, const int32_t *epair,
                                                   const uint32_t *erank, const uint32_t *ehash,
                                                   const unsigned long long *n_keys, int64_t cap,
                                                   const uint32_t *grp, const uint64_t *own, uint32_t *mix,
                                                   uint64_t *out, int32_t *opair, double *sbox, const uint64_t *epoch,
                                                   uint4 *flags, int64_t flag_vecs)
{
    const uint64_t ep = *epoch;                 // (read early, used last)
    const int64_t nk = (int64_t)*n_keys;
    const int64_t n = nk < cap ? nk : cap;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const int tb = bv.kl.tb;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        const uint64_t e = ent[i];
        const uint32_t r = erank[i];
        const int p = ONE ? 0 : epair[i];
        const uint64_t gc = e >> bv.kl.cell_shift;
        const uint32_t h = ehash[i];
        const int side = (int)((e >> tb) & 1);
        const uint32_t c = grp[2 * (size_t)h + side];
        double lo[4], hi[4];
        const PairDesc &Pd = pair_desc<ONE>(bv, p);
        tri_box_d(side_mesh(Pd, side), (int32_t)(e & bv.kl.tmask), lo, hi);
        if (c & 0x80000000u) continue;
        const uint32_t pos = c + r;
        out[pos] = e;
        if (!ONE) opair[pos] = p;
        double2 *b = reinterpret_cast<double2 *>(sbox + 8 * (size_t)pos);
        b[0] = make_double2(lo[0], lo[1]);
        b[1] = make_double2(lo[2], lo[3]);
        b[2] = make_double2(hi[0], hi[1]);
        b[3] = make_double2(hi[2], hi[3]);
        if (own[h] != gc) mix[h] = 1u;    // every writer stores the same value
    }
    if ((ep + 1) % 255u == 0) {          // the next search's value wraps to 1 (k_finish advances the epoch)
        const uint4 z = make_uint4(0u, 0u, 0u, 0u);
        for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < flag_vecs; i += stride) flags[i] = z;
    }
}

// Box of grouped entry e (lo in [0..3], hi in [4..7]).
MS_D void entry_box(const double *sbox, int64_t e, double lo[4], double hi[4])
{
    const double2 *b = reinterpret_cast<const double2 *>(sbox + 8 * e);
    const double2 a0 = b[0], a1 = b[1], a2 = b[2], a3 = b[3];
    lo[0] = a0.x; lo[1] = a0.y; lo[2] = a1.x; lo[3] = a1.y;
    hi[0] = a2.x; hi[1] = a2.y; hi[2] = a3.x; hi[3] = a3.y;
}

MS_D void wave_count(bool p, int64_t *ctr)
{
    uint64_t m = ballot(p);
    if (m && lane_id() == __builtin_ctzll(m)) atomicAdd((unsigned long long *)ctr, (unsigned long long)__builtin_popcountll(m));
}

MS_D void emit_hit(bool hit, const hit_t &h, uint64_t key, hit_t *hits, uint64_t *hkeys, int64_t cap,
                   search_stats_t *stats)
{
    int64_t idx = wave_reserve(hit, (unsigned long long *)&stats->n_hits);
    if (hit) {
        if (idx < cap) {
            hits[idx] = h;
            if (hkeys) hkeys[idx] = key;
        } else {
            atomicOr((unsigned long long *)&stats->overflow, 4ull);
        }
    }
}

// Slot -> (group, iA, iB), iA = slot mod nA, iB = slot / nA (Alg. 1).  A
// group holds the entries of every cell with the same hashed id, so a pair
// of entries counts only when both are entries of the same cell; the pair
// is then kept only in its home cell, the cell of the componentwise max of
// the two boxes' lower corners (the one cell of both ranges that every
// overlapping pair has, by monotonicity of the cell map), and only if the
// closed boxes overlap (Sec. 6.2.2).
//
// Each block takes a chunk of consecutive slots: ITEMS per thread, or up to
// ITEMS_MAX when that is enough for every chunk to have a block in the first
// round of resident blocks (otherwise a few chunks past a full round would
// wait for a second round, doubling the kernel's time).  Of every group the
// chunk touches it needs only the A entries of the rows it covers (all of
// them once it spans more than one row) and the B entries of those rows; when
// these are at most S::stage in all, the block stages their cells, triangle
// indices and boxes in LDS, so that every slot reads LDS only.  Otherwise each slot gathers its two triangles from global
// memory.  One atomic reservation per chunk for the candidates, then the
// narrow phase on the chunk's candidates.  Last, the exact cell statistics
// (Alg. 1's boxes and slots) of the groups that start in the chunk.
//
// The work-tile shape: NT threads per block, ITEMS (up to ITEMS_MAX) slots
// per thread (a chunk is NT * ITEMS slots), STAGE staged entries (their LDS
// also holds a chunk's candidates), CELLS groups per chunk held in LDS,
// PSTART slot offsets held in LDS, GRID blocks.  The narrow phase needs
// about 200 registers, so a SIMD holds two waves: one 512-thread block per
// CU, or two 256-thread blocks when their LDS fits twice.  Results do not
// depend on the shape, only the time.
template <int NT, int ITEMS, int ITEMS_MAX, int STAGE, int CELLS, int PSTART, int GRID>
struct EnumShape {
    static constexpr int block = NT, items = ITEMS, items_max = ITEMS_MAX, slots_max = NT * ITEMS_MAX, stage = STAGE,
                         cells = CELLS, pstart = PSTART, grid = GRID;
    static_assert(ITEMS <= ITEMS_MAX && ITEMS_MAX <= 32 && CELLS <= NT, "keep bits per thread; one group per thread");
};
using EnumWide = EnumShape<512, 8, 10, 960, 256, 4096, 512>;     // one block per CU, two rounds
using EnumHalf = EnumShape<256, 8, 10, 480, 128, 2048, 1024>;    // two blocks per CU, two rounds
using EnumQuarter = EnumShape<128, 8, 10, 240, 64, 1024, 2048>;  // four blocks per CU, two rounds

template <bool ONE>
MS_D bool enum_pair(const PairDesc &Pd, uint64_t cell, const double alo[4], const double ahi[4], const double blo[4],
                    const double bhi[4])
{
    bool ov = true;
#pragma unroll
    for (int d = 0; d < 4; ++d) ov = ov && (alo[d] <= bhi[d]) && (blo[d] <= ahi[d]);
    if (!ov) return false;
    int64_t h[4];
#pragma unroll
    for (int d = 0; d < 4; ++d) {
        const double m = alo[d] > blo[d] ? alo[d] : blo[d];
        h[d] = cell_of(m, Pd.g.wlo[d], Pd.g.inv, Pd.g.n[d]);
    }
    return (uint64_t)cell_linear(h, Pd.g.n) == cell;
}

// Bounds of local cell `cell` in t = (x - wlo) * inv per axis, such that
// cell_of(x) == that axis's coordinate exactly when lo <= t and not t >= hi:
// lo = -inf on the first cell, hi = NaN on the last (no upper bound), else
// the cell's integer edges (floor(t) == c <=> c <= t < c + 1 in FP64).
template <int CELLS>
MS_D void home_bounds(const GridView &g, uint64_t cell, double (*gb)[CELLS], int k)
{
    int64_t c[4];
    uint64_t r = cell;
#pragma unroll
    for (int d = 3; d >= 0; --d) {
        c[d] = (int64_t)(r % (uint64_t)g.n[d]);
        r /= (uint64_t)g.n[d];
    }
#pragma unroll
    for (int d = 0; d < 4; ++d) {
        gb[d][k] = c[d] == 0 ? -INFINITY : (double)c[d];
        gb[4 + d][k] = c[d] == g.n[d] - 1 ? (double)NAN : (double)(c[d] + 1);
    }
}

// Slot offset inside a group -> (row iB, column iA) for rows of nA; the
// 32-bit division is much cheaper and covers every group below 2^32 slots.
MS_D void split_slot(uint64_t local, uint32_t nA, uint64_t &iB, uint64_t &iA)
{
    if (local <= 0xffffffffull) {
        const uint32_t l = (uint32_t)local, q = l / nA;
        iB = q;
        iA = l - q * nA;
    } else {
        iB = local / nA;
        iA = local - iB * nA;
    }
}

template <bool ONE>
MS_D int entry_pair(const int32_t *kpair, int64_t e)
{
    if constexpr (ONE) return 0;
    else return kpair[e];
}

// Exact cell statistics of a group holding several cells (cells whose hashes
// collide), by the whole block of NT threads: each cell's A and B entries are
// counted in an LDS table keyed by the cell (s_tab: GS_SLOTS keys, then as
// many count words, then an overflow flag), then every cell with entries of
// both meshes adds itself and nA * nB slots.  A group of more distinct cells
// than the table holds is counted per A entry instead.
constexpr int GS_SLOTS = 64;

template <int NT>
MS_D void group_stats(const uint64_t *keys, const CellRec &cr, int sh, uint64_t *s_tab, unsigned long long &xc,
                      unsigned long long &xs)
{
    constexpr uint64_t EMPTY = ~0ull;
    uint64_t *s_key = s_tab, *s_cnt = s_tab + GS_SLOTS, *s_full = s_tab + 2 * GS_SLOTS;
    for (int i = threadIdx.x; i < GS_SLOTS; i += NT) {
        s_key[i] = EMPTY;
        s_cnt[i] = 0;
    }
    if (threadIdx.x == 0) *s_full = 0;
    __syncthreads();
    const int n = cr.nA + cr.nB;
    for (int i = threadIdx.x; i < n; i += NT) {
        const uint64_t c = keys[cr.start + i] >> sh;
        const unsigned long long add = i < cr.nA ? 1ull : (1ull << 32);   // nA in the low half, nB in the high
        uint32_t slot = (uint32_t)((c * 0x9E3779B97F4A7C15ull) >> 58);
        bool done = false;
        for (int probe = 0; probe < GS_SLOTS && !done; ++probe) {
            const unsigned long long k =
                atomicCAS((unsigned long long *)&s_key[slot], (unsigned long long)EMPTY, (unsigned long long)c);
            if (k == EMPTY || k == c) {
                atomicAdd((unsigned long long *)&s_cnt[slot], add);
                done = true;
            } else {
                slot = (slot + 1) & (GS_SLOTS - 1);
            }
        }
        if (!done) *s_full = 1;
    }
    __syncthreads();
    if (*s_full == 0) {
        for (int i = threadIdx.x; i < GS_SLOTS; i += NT) {
            if (s_key[i] == EMPTY) continue;
            const uint64_t v = s_cnt[i], a = v & 0xffffffffull, b = v >> 32;
            xs += a * b;
            xc += (a > 0 && b > 0);
        }
    } else {
        for (int i = threadIdx.x; i < cr.nA; i += NT) {
            const uint64_t ci = keys[cr.start + i] >> sh;
            uint32_t nb = 0, before = 0;
            for (int j = 0; j < cr.nB; ++j) nb += (keys[cr.start + cr.nA + j] >> sh) == ci;
            for (int j = 0; j < i; ++j) before += (keys[cr.start + j] >> sh) == ci;
            xs += nb;
            xc += (nb > 0 && before == 0);
        }
    }
    __syncthreads();
}

// A staged slot: its group c (last with s_pre[c] <= slot) and the staged
// indices of its A and B entries.
struct StagedSlot {
    int c, ia, ib;
};

MS_D StagedSlot staged_slot(int64_t slot, int nc, const int64_t *s_pre, const int32_t *s_nA, const int32_t *s_aoff,
                            const int32_t *s_ia0, const int32_t *s_boff, const int32_t *s_ib0)
{
    int lo = 0, hi = nc;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (s_pre[mid] <= slot) lo = mid;
        else hi = mid;
    }
    uint64_t iB, iA;
    split_slot((uint64_t)(slot - s_pre[lo]), (uint32_t)s_nA[lo], iB, iA);
    StagedSlot q;
    q.c = lo;
    q.ia = s_aoff[lo] + (int)((int64_t)iA - s_ia0[lo]);
    q.ib = s_boff[lo] + (int)((int64_t)iB - s_ib0[lo]);
    return q;
}

// One slot from global memory (chunks whose entries do not fit the LDS
// stage): its group by binary search, both entries, both boxes from the
// vertices.
struct SlotOut {
    uint64_t packed;    // (triA << 32) | triB
    int32_t pr;         // pair
    int32_t keep;
};

template <bool ONE>
MS_D SlotOut global_slot(const BatchView &bv, const uint64_t *keys, const int32_t *kpair, const double *sbox,
                         const CellRec *cells, const int64_t *pstart, int64_t c0, int64_t nc, const int64_t *s_pre,
                         int64_t slot)
{
    SlotOut o;
    o.packed = 0;
    o.pr = 0;
    o.keep = 0;
    const int sh = bv.kl.cell_shift;
    // the slot's group among the chunk's nc groups from c0: their slot
    // starts in LDS (s_pre) when they are few, else in global memory
    const int64_t c = s_pre ? c0 + last_le<int64_t>(s_pre, nc, slot) : c0 + last_le<int64_t>(pstart + c0, nc, slot);
    const CellRec cr = cells[c];
    uint64_t iB, iA;
    split_slot((uint64_t)(slot - pstart[c]), (uint32_t)cr.nA, iB, iA);
    const int64_t eA = cr.start + (int64_t)iA, eB = cr.start + cr.nA + (int64_t)iB;
    const uint64_t kA = keys[eA];
    const uint64_t kB = keys[eB];
    const uint64_t ca = kA >> sh;
    const int32_t ta = (int32_t)(kA & bv.kl.tmask), tb = (int32_t)(kB & bv.kl.tmask);
    o.packed = ((uint64_t)(uint32_t)ta << 32) | (uint32_t)tb;
    if (ca != (kB >> sh)) return o;
    o.pr = entry_pair<ONE>(kpair, eA);
    const PairDesc &Pd = pair_desc<ONE>(bv, o.pr);
    double alo[4], ahi[4], blo[4], bhi[4];
    entry_box(sbox, eA, alo, ahi);
    entry_box(sbox, eB, blo, bhi);
    o.keep = enum_pair<ONE>(Pd, ca - Pd.cell_base, alo, ahi, blo, bhi);
    return o;
}

// For x0 <= x1, the last i0 and i1 in [0, n) with a[i] <= x (a ascending,
// a[0] <= x0), found by the whole block at once: each round splits every
// open range [lo, hi) into NT parts, one per thread, and keeps the part
// where a[i] <= x stops holding (two loads per thread and round; log_NT(n)
// rounds).  s_r[0..1] = [lo, hi) for x0, s_r[2..3] for x1; the results are
// s_r[0] and s_r[2].  Ends with a barrier.
template <int NT>
MS_D void block_last_le2(const int64_t *a, int64_t n, int64_t x0, int64_t x1, int64_t *s_r)
{
    if (threadIdx.x == 0) {
        s_r[0] = 0;
        s_r[1] = n;
        s_r[2] = 0;
        s_r[3] = n;
    }
    __syncthreads();
    for (;;) {
        const int64_t lo0 = s_r[0], hi0 = s_r[1], lo1 = s_r[2], hi1 = s_r[3];
        if (hi0 - lo0 <= 1 && hi1 - lo1 <= 1) break;
        __syncthreads();      // every thread has read the ranges
#pragma unroll
        for (int k = 0; k < 2; ++k) {
            const int64_t lo = k ? lo1 : lo0, hi = k ? hi1 : hi0, x = k ? x1 : x0;
            if (hi - lo <= 1) continue;
            const int64_t step = (hi - lo + NT - 1) / NT;
            const int64_t i = lo + (int64_t)threadIdx.x * step;
            if (i < hi && a[i] <= x) {
                const int64_t j = i + step;
                if (j >= hi || a[j] > x) {
                    s_r[2 * k] = i;
                    s_r[2 * k + 1] = j < hi ? j : hi;
                }
            }
        }
        __syncthreads();
    }
    __syncthreads();
}

template <bool ONE, class S>
__global__ void __launch_bounds__(S::block) k_enum(BatchView bv, const uint64_t *keys, const int32_t *kpair,
                                                const double *sbox, const CellRec *cells, const int64_t *pstart_g, const int64_t *kept,
                                                const uint32_t *mix,
                                                search_stats_t *stats, uint64_t *cand, int32_t *cand_pair,
                                                int64_t cand_cap, hit_t *hits, uint64_t *hkeys, int64_t hits_cap,
                                                unsigned long long *epart, int resident)
{
    constexpr int ENUM_BLOCK = S::block, ENUM_ITEMS = S::items, ENUM_ITEMS_MAX = S::items_max,
                  ENUM_SLOTS_MAX = S::slots_max, ENUM_STAGE = S::stage, ENUM_CELLS = S::cells,
                  ENUM_PSTART = S::pstart;
    static_assert(ENUM_STAGE > 2 * GS_SLOTS, "the staged cells hold a group's statistics table");
    __shared__ int64_t s_pstart[ENUM_PSTART + 1];
    // the staged boxes during enumeration (component-major, so that lanes
    // reading consecutive entries hit distinct banks), then the chunk's
    // compacted candidates
    __shared__ union {
        double box[8][ENUM_STAGE];
        struct {
            uint64_t tt[ENUM_SLOTS_MAX];
            int32_t pair[ENUM_SLOTS_MAX];
        } c;
    } s_u;
    static_assert(sizeof(double) * ENUM_STAGE * 8 >= 12 * ENUM_SLOTS_MAX, "candidate list overlays the staged boxes");
    double (*s_box)[ENUM_STAGE] = s_u.box;
    __shared__ int32_t s_t[ENUM_STAGE];
    __shared__ uint64_t s_ec[ENUM_STAGE];
    __shared__ int32_t s_ep[ONE ? 1 : ENUM_STAGE];
    __shared__ int64_t s_pre[ENUM_CELLS + 1];
    __shared__ int64_t s_start[ENUM_CELLS];
    __shared__ int32_t s_aoff[ENUM_CELLS + 1], s_boff[ENUM_CELLS], s_ia0[ENUM_CELLS], s_ib0[ENUM_CELLS];
    __shared__ int32_t s_nA[ENUM_CELLS];
    __shared__ int64_t s_c0, s_c1;
    __shared__ int64_t s_rng[4];
    __shared__ uint32_t s_kscan[ENUM_BLOCK / WAVE];
    __shared__ unsigned long long s_kbase;
    __shared__ unsigned long long s_st[ENUM_BLOCK / WAVE];
    __shared__ uint32_t s_nmix;
    __shared__ uint64_t s_gcell[ENUM_CELLS];
    __shared__ double s_gb[8][ENUM_CELLS];            // per staged group: t-bounds of its cell
    __shared__ double s_gw[ONE ? 1 : 5][ENUM_CELLS];  // per staged group: wlo, inv (batch)
    unsigned long long xc = 0, xs = 0;      // exact cells and slots
    // the block's counts (thread 0), added at its end to one of STAT_SHARDS
    // counter lines (block index mod STAT_SHARDS): same-line atomics of
    // hundreds of blocks would serialise; k_finish sums the lines
    unsigned long long b_cand = 0, b_moller = 0, b_degen = 0, b_outside = 0, b_unstaged = 0;
    const int64_t ncells = kept[0];
    const int64_t P = kept[1];
    // slots per thread: ENUM_ITEMS, or more (up to ENUM_ITEMS_MAX) when that
    // gives every chunk a block among the `resident` ones of the first round
    int items = ENUM_ITEMS;
    if (resident > 0) {
        const int64_t per = ceil_div(P, (int64_t)resident * ENUM_BLOCK);
        if (per > ENUM_ITEMS && per <= ENUM_ITEMS_MAX) items = (int)per;
    }
    const int64_t chunk_slots = (int64_t)items * ENUM_BLOCK;
    const int64_t nchunks = ceil_div(P, chunk_slots);
    if ((int64_t)blockIdx.x >= nchunks) return;     // no chunk, nothing to count (the whole block)
    const int sh = bv.kl.cell_shift;
    const bool lds_pre = ncells <= ENUM_PSTART;
    {
    if (lds_pre) {
        for (int64_t i = threadIdx.x; i <= ncells; i += ENUM_BLOCK) s_pstart[i] = pstart_g[i];
        __syncthreads();
    }
    const int64_t *pstart = lds_pre ? s_pstart : pstart_g;
    for (int64_t chunk = blockIdx.x; chunk < nchunks; chunk += gridDim.x) {
        const int64_t S0 = chunk * chunk_slots;
        const int64_t S1 = S0 + chunk_slots < P ? S0 + chunk_slots : P;
        if (lds_pre) {
            // the one i with pstart[i] <= x < pstart[i + 1], for x = S0, S1 - 1
            for (int64_t i = threadIdx.x; i < ncells; i += ENUM_BLOCK) {
                const int64_t a = s_pstart[i], b = s_pstart[i + 1];
                if (a <= S0 && S0 < b) s_c0 = i;
                if (a <= S1 - 1 && S1 - 1 < b) s_c1 = i;
            }
            if (threadIdx.x == 0) s_nmix = 0;
        } else {
            block_last_le2<ENUM_BLOCK>(pstart, ncells, S0, S1 - 1, s_rng);
            if (threadIdx.x == 0) {
                s_c0 = s_rng[0];
                s_c1 = s_rng[2];
                s_nmix = 0;
            }
        }
        __syncthreads();
        const int64_t c0 = s_c0, nc = s_c1 - s_c0 + 1;
        const int64_t *pre_lds = nc <= ENUM_CELLS ? s_pre : nullptr;
        // the rows of every touched group that the chunk covers, and the entries they need
        uint32_t need = 0;
        bool first_here = false;     // the group's first slot is in this chunk (it is counted here)
        uint32_t mixv = 0;
        uint64_t gslots = 0;
        if (nc <= ENUM_CELLS && threadIdx.x < nc) {
            const int64_t c = c0 + threadIdx.x;
            const CellRec cr = cells[c];
            const int64_t p0 = pstart[c], p1 = pstart[c + 1];
            first_here = p0 >= S0;
            if (first_here) mixv = mix[cr.h];      // used after the narrow phase
            gslots = (uint64_t)cr.nA * (uint64_t)cr.nB;
            const int64_t l0 = (S0 > p0 ? S0 : p0) - p0, l1 = (S1 < p1 ? S1 : p1) - p0;
            const int64_t ib0 = l0 / cr.nA, ib1 = (l1 - 1) / cr.nA;
            int64_t ia0 = 0, ia1 = cr.nA;
            if (ib0 == ib1) {
                ia0 = l0 - ib0 * cr.nA;
                ia1 = (l1 - 1) - ib1 * cr.nA + 1;
            }
            need = (uint32_t)((ia1 - ia0) + (ib1 - ib0 + 1));
            s_pre[threadIdx.x] = p0;
            s_start[threadIdx.x] = cr.start;
            s_ia0[threadIdx.x] = (int32_t)ia0;
            s_ib0[threadIdx.x] = (int32_t)ib0;
            s_nA[threadIdx.x] = cr.nA;
            s_boff[threadIdx.x] = (int32_t)(ia1 - ia0);     // made absolute below
            if (threadIdx.x == nc - 1) s_pre[nc] = p1;
        }
        uint32_t tot;
        const uint32_t off = block_excl<ENUM_BLOCK>(need, s_kscan, &tot);
        const bool staged = nc <= ENUM_CELLS && tot <= ENUM_STAGE;
        if (!staged && threadIdx.x == 0) ++b_unstaged;
        if (staged) {
            if (threadIdx.x < nc) {
                s_aoff[threadIdx.x] = (int32_t)off;
                s_boff[threadIdx.x] += (int32_t)off;
            }
            if (threadIdx.x == 0) s_aoff[nc] = (int32_t)tot;
            __syncthreads();
            for (int i = threadIdx.x; i < (int)tot; i += ENUM_BLOCK) {
                int lo = 0, hi = (int)nc;             // the group whose staged range holds i
                while (hi - lo > 1) {
                    const int mid = (lo + hi) >> 1;
                    if (s_aoff[mid] <= i) lo = mid;
                    else hi = mid;
                }
                const bool isB = i >= s_boff[lo];
                const int64_t e = isB ? s_start[lo] + s_nA[lo] + s_ib0[lo] + (i - s_boff[lo])
                                      : s_start[lo] + s_ia0[lo] + (i - s_aoff[lo]);
                const uint64_t key = keys[e];
                const int32_t t = (int32_t)(key & bv.kl.tmask);
                const int p = entry_pair<ONE>(kpair, e);
                double blo[4], bhi[4];
                entry_box(sbox, e, blo, bhi);
#pragma unroll
                for (int d = 0; d < 4; ++d) { s_box[d][i] = blo[d]; s_box[4 + d][i] = bhi[d]; }
                s_t[i] = t;
                s_ec[i] = key >> sh;
                if (!ONE) s_ep[i] = p;
            }
            __syncthreads();
            // per group: the cell of its first staged entry (every entry's
            // cell, unless the group holds several) and that cell's bounds
            // in the grid's coordinate t = (x - wlo) * inv
            if (threadIdx.x < nc) {
                const int i0 = s_aoff[threadIdx.x];
                const uint64_t gc = s_ec[i0];
                const PairDesc &Pd = pair_desc<ONE>(bv, ONE ? 0 : s_ep[i0]);
                home_bounds<ENUM_CELLS>(Pd.g, gc - Pd.cell_base, s_gb, threadIdx.x);
                s_gcell[threadIdx.x] = gc;
                if constexpr (!ONE) {
#pragma unroll
                    for (int d = 0; d < 4; ++d) s_gw[d][threadIdx.x] = Pd.g.wlo[d];
                    s_gw[4][threadIdx.x] = Pd.g.inv;
                }
            }
            __syncthreads();
        }
        // pass 1: the keep bit of each slot (the pair of a kept slot is
        // found again in pass 2, so that no per-slot state is held)
        uint32_t keepm = 0;
        // a thread's slots lie ENUM_BLOCK apart: the group and the (iB, iA)
        // split are found once per group entered, then advanced by
        // ENUM_BLOCK = qa * nA + ra slots at a time
        int c = 0, ia = 0, ib = 0;
        int64_t pend = 0;
        uint32_t nAc = 1, iA = 0, qa = 0, ra = 0;
#pragma unroll 1
        for (int j = 0; j < items; ++j) {
            const int64_t slot = S0 + (int64_t)j * ENUM_BLOCK + threadIdx.x;
            bool keep = false;
            if (slot < S1) {
                if (staged) {
                    if (j == 0 || slot >= pend) {
                        const StagedSlot q = staged_slot(slot, (int)nc, s_pre, s_nA, s_aoff, s_ia0, s_boff, s_ib0);
                        c = q.c;
                        ia = q.ia;
                        ib = q.ib;
                        nAc = (uint32_t)s_nA[c];
                        pend = s_pre[c + 1];
                        iA = (uint32_t)(ia - s_aoff[c] + s_ia0[c]);
                        qa = (uint32_t)ENUM_BLOCK / nAc;
                        ra = (uint32_t)ENUM_BLOCK - qa * nAc;
                    } else {
                        iA += ra;
                        ia += (int)ra;
                        ib += (int)qa;
                        if (iA >= nAc) {
                            iA -= nAc;
                            ia -= (int)nAc;
                            ++ib;
                        }
                    }
                    const uint64_t ca = s_ec[ia];
                    if (ca == s_ec[ib]) {
                        double alo[4], ahi[4], blo[4], bhi[4];
                        bool ov = true;
#pragma unroll
                        for (int d = 0; d < 4; ++d) {
                            alo[d] = s_box[d][ia]; ahi[d] = s_box[4 + d][ia];
                            blo[d] = s_box[d][ib]; bhi[d] = s_box[4 + d][ib];
                            ov = ov && (alo[d] <= bhi[d]) && (blo[d] <= ahi[d]);
                        }
                        if (ov) {
                            if (ca == s_gcell[c]) {
                                // home cell = the group's cell: per axis, the
                                // max of the lower corners falls in its bounds
                                bool in = true;
#pragma unroll
                                for (int d = 0; d < 4; ++d) {
                                    const double m = alo[d] > blo[d] ? alo[d] : blo[d];
                                    double wl, iv;
                                    if constexpr (ONE) {
                                        wl = bv.p0.g.wlo[d];
                                        iv = bv.p0.g.inv;
                                    } else {
                                        wl = s_gw[d][c];
                                        iv = s_gw[4][c];
                                    }
                                    const double t = (m - wl) * iv;
                                    in = in && (t >= s_gb[d][c]) && !(t >= s_gb[4 + d][c]);
                                }
                                keep = in;
                            } else {
                                const PairDesc &Pd = pair_desc<ONE>(bv, ONE ? 0 : s_ep[ia]);
                                keep = enum_pair<ONE>(Pd, ca - Pd.cell_base, alo, ahi, blo, bhi);
                            }
                        }
                    }
                } else {
                    keep = global_slot<ONE>(bv, keys, kpair, sbox, cells, pstart, c0, nc, pre_lds, slot).keep != 0;
                }
            }
            keepm |= (uint32_t)keep << j;
        }
        // the candidates: counted with one atomic per chunk, stored when asked
        // for, and compacted into LDS for the narrow phase
        uint32_t ktot;
        const uint32_t kex = block_excl<ENUM_BLOCK>((uint32_t)__builtin_popcount(keepm), s_kscan, &ktot);
        if (threadIdx.x == 0) {
            // the chunk's place in the candidate list matters only when the
            // list is stored; otherwise the count needs no reply
            unsigned long long b = 0;
            if (ktot) {
                if (cand) b = atomicAdd((unsigned long long *)&stats->n_cand, (unsigned long long)ktot);
                else b_cand += ktot;
            }
            s_kbase = b;
        }
        __syncthreads();        // (also: every slot is done reading the staged boxes)
        {
            uint32_t li = kex;
            int64_t idx = (int64_t)s_kbase + kex;
#pragma unroll 1
            for (uint32_t m = keepm; m; m &= m - 1) {
                const int64_t slot = S0 + (int64_t)__builtin_ctz(m) * ENUM_BLOCK + threadIdx.x;
                uint64_t packed;
                int32_t pr;
                if (staged) {
                    const StagedSlot q = staged_slot(slot, (int)nc, s_pre, s_nA, s_aoff, s_ia0, s_boff, s_ib0);
                    packed = ((uint64_t)(uint32_t)s_t[q.ia] << 32) | (uint32_t)s_t[q.ib];
                    pr = ONE ? 0 : s_ep[q.ia];
                } else {
                    const SlotOut so = global_slot<ONE>(bv, keys, kpair, sbox, cells, pstart, c0, nc, pre_lds, slot);
                    packed = so.packed;
                    pr = so.pr;
                }
                s_u.c.tt[li] = packed;
                s_u.c.pair[li] = pr;
                if (cand) {
                    if (idx < cand_cap) {
                        cand[idx] = packed;
                        if (cand_pair) cand_pair[idx] = pr;
                    } else {
                        atomicOr((unsigned long long *)&stats->overflow, 2ull);
                    }
                }
                ++li;
                ++idx;
            }
        }
        __syncthreads();
        // the narrow phase on the chunk's candidates: Moller quick test
        // (Sec. 6.2.3), 4x4 solve and inclusion (Sec. 6.2.4), hit records
        if (ktot) {
            uint32_t nm = 0, nd = 0, no = 0;
            for (uint32_t base = 0; base < ktot; base += ENUM_BLOCK) {
                const uint32_t i = base + threadIdx.x;
                int stt = PS_AABB;
                int32_t ta = 0, tb = 0, p = 0;
                double z[4] = {0, 0, 0, 0};
                Tri Pt;
                if (i < ktot) {
                    const uint64_t tt = s_u.c.tt[i];
                    ta = (int32_t)(tt >> 32);
                    tb = (int32_t)(tt & 0xffffffffu);
                    p = s_u.c.pair[i];
                    const PairDesc &Pd = pair_desc<ONE>(bv, p);
                    Pt = load_tri(Pd.A, ta);
                    const Tri Q = load_tri(Pd.B, tb);
                    if (same_side(Pt, Q) || same_side(Q, Pt)) {
                        stt = PS_MOLLER;
                    } else {
                        const bool ok = solve_pair(Pt, Q, z);
                        stt = !ok ? PS_DEGEN : !inside(z) ? PS_OUTSIDE : PS_HIT;
                    }
                }
                nm += stt == PS_MOLLER;
                nd += stt == PS_DEGEN;
                no += stt == PS_OUTSIDE;
                hit_t h;
                uint64_t key = 0;
                if (stt == PS_HIT) {
                    const PairDesc &Pd = pair_desc<ONE>(bv, p);
                    make_hit(Pd.A, Pd.B, ta, tb, (uint32_t)p, Pt, z, h);
                    key = ((uint64_t)p << (bv.tbA + bv.tbB)) | ((uint64_t)(uint32_t)ta << bv.tbB) | (uint32_t)tb;
                }
                emit_hit(stt == PS_HIT, h, key, hits, hkeys, hits_cap, stats);
            }
            const uint32_t sm = block_sum<ENUM_BLOCK>(nm, s_kscan), sd = block_sum<ENUM_BLOCK>(nd, s_kscan), so = block_sum<ENUM_BLOCK>(no, s_kscan);
            if (threadIdx.x == 0) {
                b_moller += sm;
                b_degen += sd;
                b_outside += so;
            }
        }
        // exact statistics of the groups that start in this chunk: a group of
        // one cell adds the cell and nA * nB slots; the groups of several
        // cells are listed and counted by the whole block
        __syncthreads();
        if (nc <= ENUM_CELLS) {
            if (first_here) {
                if (mixv) {
                    s_u.c.pair[atomicAdd(&s_nmix, 1u)] = (int32_t)threadIdx.x;
                } else {
                    xc += 1;
                    xs += gslots;
                }
            }
        } else {
            for (int64_t c = c0 + threadIdx.x; c < c0 + nc; c += ENUM_BLOCK) {
                if (pstart[c] < S0) continue;
                const CellRec cr = cells[c];
                if (mix[cr.h]) {
                    s_u.c.pair[atomicAdd(&s_nmix, 1u)] = (int32_t)(c - c0);
                } else {
                    xc += 1;
                    xs += (unsigned long long)cr.nA * (unsigned long long)cr.nB;
                }
            }
        }
        __syncthreads();
        for (uint32_t k = 0; k < s_nmix; ++k) {
            const CellRec cr = cells[c0 + s_u.c.pair[k]];
            group_stats<ENUM_BLOCK>(keys, cr, sh, s_ec, xc, xs);
        }
        __syncthreads();
    }
    }
    const unsigned long long sc = block_sum<ENUM_BLOCK>(xc, s_st), ss = block_sum<ENUM_BLOCK>(xs, s_st);
    if (threadIdx.x == 0) {
        unsigned long long *w = epart + SHARD_WORDS * (blockIdx.x % STAT_SHARDS);
        const unsigned long long c[7] = {b_cand, b_moller, b_degen, b_outside, sc, ss, b_unstaged};
#pragma unroll
        for (int k = 0; k < 7; ++k)
            if (c[k]) atomicAdd(w + k, c[k]);
    }
}

__global__ void __launch_bounds__(BLOCK) k_hits_place(const hit_t *tmp, const uint64_t *sorted, const int64_t *n_dev,
                                                      int64_t cap, int tbA, int tbB, hit_t *out)
{
    const int64_t n = *n_dev < cap ? *n_dev : cap;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        const hit_t &h = tmp[i];
        const uint64_t key = ((uint64_t)h.flags << (tbA + tbB)) | ((uint64_t)(uint32_t)h.triA << tbB) | (uint32_t)h.triB;
        out[lower_bound_u64(sorted, 0, n, key)] = h;
    }
}

// The end of a search, one block: the enumeration's counter lines summed
// into the statistics, the epoch advanced (the occupancy tables of this
// search are no longer read), and, for a hit capacity of at most HITS_TINY,
// the hits ranked by counting the smaller keys (the keys are distinct) and
// placed, key and record together.
constexpr int HITS_TINY = 1024;
constexpr int FIN_BLOCK = 256;

struct FinishArgs {
    search_stats_t *stats;
    uint64_t *epoch;
    const unsigned long long *n_keys;
    const unsigned long long *shards;
    int tiny;                  // sort the hits here
    const hit_t *tmp;
    uint64_t *keys;
    int64_t cap;
    hit_t *out;
};

__global__ void __launch_bounds__(FIN_BLOCK) k_finish(FinishArgs a)
{
    __shared__ uint64_t s_k[HITS_TINY];
    if (threadIdx.x < 7) {
        unsigned long long v = 0;
        for (int i = 0; i < STAT_SHARDS; ++i) v += a.shards[SHARD_WORDS * i + threadIdx.x];
        search_stats_t *st = a.stats;
        switch (threadIdx.x) {
        case 0: st->n_cand += (int64_t)v; break;
        case 1: st->n_moller = (int64_t)v; break;
        case 2: st->n_degenerate = (int64_t)v; break;
        case 3: st->n_outside = (int64_t)v; break;
        case 4: st->n_cells = (int64_t)v; break;
        case 5: st->n_slots = (int64_t)v; break;
        default: st->n_chunks_unstaged = (int64_t)v; break;
        }
    } else if (threadIdx.x == 7) {
        *a.epoch += 1;
        a.stats->n_entries = (int64_t)*a.n_keys;
    }
    if (!a.tiny) return;
    const int n = (int)(a.stats->n_hits < a.cap ? a.stats->n_hits : a.cap);
    for (int i = threadIdx.x; i < n; i += FIN_BLOCK) s_k[i] = a.keys[i];
    __syncthreads();
    for (int i = threadIdx.x; i < n; i += FIN_BLOCK) {
        const uint64_t k = s_k[i];
        int r = 0;
        for (int j = 0; j < n; ++j) r += s_k[j] < k;
        a.keys[r] = k;
        a.out[r] = a.tmp[i];
    }
}

// Per-pair hit offsets of a batch from the sorted hit keys.
__global__ void __launch_bounds__(BLOCK) k_pair_offsets(const uint64_t *sorted, const int64_t *n_dev, int64_t cap,
                                                        int n_pairs, int shift, int64_t *offs)
{
    const int64_t n = *n_dev < cap ? *n_dev : cap;
    for (int p = blockIdx.x * blockDim.x + threadIdx.x; p <= n_pairs; p += gridDim.x * blockDim.x)
        offs[p] = p == n_pairs ? n : lower_bound_u64(sorted, 0, n, (uint64_t)p << shift);
}

// All pairs, tiled: each thread holds one triangle of A, tiles of B are
// staged in LDS; every stage of the test runs on every pair.
constexpr int AP_TILE = 128;

__global__ void __launch_bounds__(BLOCK) k_allpairs(PairDesc pd, hit_t *hits, int64_t hits_cap, search_stats_t *stats)
{
    __shared__ double s_tri[AP_TILE][12];
    __shared__ double s_box[AP_TILE][8];
    __shared__ int s_fin[AP_TILE];
    const int64_t a_tiles = ceil_div(pd.nA, BLOCK);
    const int64_t b_tiles = ceil_div(pd.nB, AP_TILE);
    const int64_t n_work = a_tiles * b_tiles;
    for (int64_t w = blockIdx.x; w < n_work; w += gridDim.x) {
        const int64_t at = w % a_tiles, bt = w / a_tiles;
        const int32_t ta = (int32_t)(at * BLOCK + threadIdx.x);
        const bool a_ok = ta < pd.nA;
        Tri P = a_ok ? load_tri(pd.A, ta) : Tri{};
        double alo[4] = {0, 0, 0, 0}, ahi[4] = {0, 0, 0, 0};
        const bool a_fin = a_ok && tri_box(pd.A, ta, alo, ahi);
        const int32_t tb0 = (int32_t)(bt * AP_TILE);
        __syncthreads();
        if (threadIdx.x < AP_TILE) {
            int32_t tb = tb0 + threadIdx.x;
            if (tb < pd.nB) {
                Tri Q = load_tri(pd.B, tb);
                double blo[4], bhi[4];
                s_fin[threadIdx.x] = tri_box(pd.B, tb, blo, bhi) ? 1 : 0;
                for (int j = 0; j < 3; ++j)
                    for (int d = 0; d < 4; ++d) s_tri[threadIdx.x][4 * j + d] = Q.p[j][d];
                for (int d = 0; d < 4; ++d) { s_box[threadIdx.x][d] = blo[d]; s_box[threadIdx.x][4 + d] = bhi[d]; }
            }
        }
        __syncthreads();
        const int nb = (int)((pd.nB - tb0) < AP_TILE ? (pd.nB - tb0) : AP_TILE);
        for (int j = 0; j < nb; ++j) {
            Tri Q;
#pragma unroll
            for (int v = 0; v < 3; ++v)
#pragma unroll
                for (int d = 0; d < 4; ++d) Q.p[v][d] = s_tri[j][4 * v + d];
            const bool b_fin = s_fin[j] != 0;
            bool box = true;
#pragma unroll
            for (int d = 0; d < 4; ++d) box = box && (alo[d] <= s_box[j][4 + d]) && (s_box[j][d] <= ahi[d]);
            double z[4];
            int st = pair_status_forced(P, Q, box, z);
            const bool live = a_fin && b_fin;
            if (!live) st = PS_AABB;
            wave_count(live && st != PS_AABB, &stats->n_cand);
            wave_count(st == PS_MOLLER, &stats->n_moller);
            wave_count(st == PS_DEGEN, &stats->n_degenerate);
            wave_count(st == PS_OUTSIDE, &stats->n_outside);
            hit_t h;
            if (st == PS_HIT) make_hit(pd.A, pd.B, ta, tb0 + j, 0u, P, z, h);
            emit_hit(st == PS_HIT, h, 0, hits, nullptr, hits_cap, stats);
        }
    }
}

__global__ void k_copy_i64(const int64_t *a, int64_t *out) { *out = *a; }

// Entry count of one pair's grid (workspace sizing): per-block partials.
__global__ void __launch_bounds__(BLOCK) k_count_all(PairDesc pd, unsigned long long *partial)
{
    __shared__ unsigned long long s_tmp[BLOCK / WAVE];
    const int64_t ntot = (int64_t)pd.nA + pd.nB;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    unsigned long long all = 0;
    for (int64_t gt = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; gt < ntot; gt += stride) {
        const bool side = gt >= pd.nA;
        const int64_t t = side ? gt - pd.nA : gt;
        CellRange r;
        if (tri_cells(side ? pd.B : pd.A, (int32_t)t, pd.g, r)) all += (unsigned long long)range_count(r);
    }
    all = block_sum(all, s_tmp);
    if (threadIdx.x == 0) partial[blockIdx.x] = all;
}

// ------------------------------------------------------------- host side

struct Geometry {
    int64_t n_pairs, n_tri, n_tiles, max_nA, max_nB;
    int tb, tbA, tbB, pb;
    int cell_bits;
    int bm_log2, bc_log2;
    int packable, c32;
    int enum_shape;
    int prune;          // some pair asks for world-bound pruning
    uint64_t total_cells;
};

struct Layout {
    int64_t ent_cap, cand_cap, hits_cap;
    size_t o_epoch, o_flags, o_both, o_pbox, o_grp, o_own, o_mix, o_gstat, o_ctrs, o_part, o_epart, o_rng, o_ent, o_epair, o_erank, o_ehash, o_sorted,
        o_spair, o_sbox,
        o_cells, o_pstart, o_htmp, o_hkeys, o_halt, o_misc, o_desc, o_toff, o_cbase, total;
    int64_t n_kblocks, cell_cap, n_fwords, n_cwords, n_gtiles;
};

inline size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

int pair_cells(const search_params_t *p, uint64_t &cells)
{
    unsigned __int128 c = 1;
    for (int d = 0; d < 4; ++d) {
        if (p->n_cells[d] < 1) return fail(MS_E_ARG, "search: n_cells must be >= 1");
        c *= (unsigned __int128)p->n_cells[d];
        if (c > ((unsigned __int128)1 << 62)) return fail(MS_E_KEYBITS, "search: grid has more than 2^62 cells");
    }
    if (!(p->inv_edge > 0.0) || !isfinite(p->inv_edge)) return fail(MS_E_ARG, "search: inv_edge must be > 0 and finite");
    for (int d = 0; d < 4; ++d)
        if (!isfinite(p->world_lo[d])) return fail(MS_E_ARG, "search: world_lo must be finite");
    cells = (uint64_t)c;
    return MS_OK;
}

int geometry(int64_t n_pairs, const ms_mesh *const *A, const ms_mesh *const *B, const search_params_t *prm,
             Geometry &G)
{
    memset(&G, 0, sizeof G);
    G.n_pairs = n_pairs;
    G.packable = 1;
    G.c32 = 1;
    unsigned __int128 total = 0;
    for (int64_t i = 0; i < n_pairs; ++i) {
        if (!A[i] || !B[i]) return fail(MS_E_ARG, "search: NULL mesh");
        uint64_t c = 0;
        int rc = pair_cells(&prm[i], c);
        if (rc) return rc;
        total += c;
        G.n_tri += (int64_t)A[i]->view.n_tris + B[i]->view.n_tris;
        G.n_tiles += ceil_div(A[i]->view.n_tris, TILE_TRIS) + ceil_div(B[i]->view.n_tris, TILE_TRIS);
        if (A[i]->view.n_tris > G.max_nA) G.max_nA = A[i]->view.n_tris;
        if (B[i]->view.n_tris > G.max_nB) G.max_nB = B[i]->view.n_tris;
        for (int d = 0; d < 4; ++d) {
            if (prm[i].n_cells[d] > 4096) G.packable = 0;
            if (prm[i].n_cells[d] > (int64_t)0x7fffffff) G.c32 = 0;
        }
    }
    if (total > ((unsigned __int128)1 << 62)) return fail(MS_E_KEYBITS, "search: the grids have more than 2^62 cells");
    G.total_cells = (uint64_t)total;
    int64_t mx = G.max_nA > G.max_nB ? G.max_nA : G.max_nB;
    G.tb = bits_for(mx > 0 ? (uint64_t)(mx - 1) : 0);
    if (G.tb == 0) G.tb = 1;
    G.tbA = bits_for(G.max_nA > 0 ? (uint64_t)(G.max_nA - 1) : 0);
    G.tbB = bits_for(G.max_nB > 0 ? (uint64_t)(G.max_nB - 1) : 0);
    if (G.tbB == 0) G.tbB = 1;
    G.pb = bits_for(n_pairs > 1 ? (uint64_t)(n_pairs - 1) : 0);
    G.cell_bits = bits_for(G.total_cells > 0 ? G.total_cells - 1 : 0);
    if (G.cell_bits + 1 + G.tb > 63)
        return fail(MS_E_KEYBITS, "search: cell index + side + triangle needs more than 63 key bits; coarsen the grid");
    if (G.pb + G.tbA + G.tbB > 64) return fail(MS_E_KEYBITS, "search: pair + triangle indices exceed 64 bits");
    int lg = bits_for((uint64_t)(G.n_tri > 0 ? G.n_tri : 1)) + 2;
    G.bm_log2 = lg < 12 ? 12 : (lg > 25 ? 25 : lg);
    int req = 0;     // a table size asked for by any pair (the largest)
    for (int64_t i = 0; i < n_pairs; ++i)
        if (prm[i].table_log2 > req) req = prm[i].table_log2;
    if (req > 0) G.bm_log2 = req < 8 ? 8 : (req > 27 ? 27 : req);   // the automatic size stays within [12, 25]
    G.bc_log2 = G.bm_log2 - 3;
    G.enum_shape = 0;    // the shape of the first pair that asks for one, else MS_ENUM_HALF
    for (int64_t i = 0; i < n_pairs; ++i) {
        if (prm[i].enum_shape < 0 || prm[i].enum_shape > MS_ENUM_QUARTER)
            return fail(MS_E_ARG, "search: enum_shape must be 0 or an MS_ENUM_* value");
        if (G.enum_shape == 0) G.enum_shape = prm[i].enum_shape;
    }
    if (G.enum_shape == 0) G.enum_shape = MS_ENUM_HALF;
    for (int64_t i = 0; i < n_pairs; ++i)
        if (prm[i].flags & MS_SEARCH_PRUNE) G.prune = 1;
    return MS_OK;
}

// Occupancy bytes: fine table (2 sides x 2^bm_log2), then coarse (2 x 2^bc_log2).
inline size_t flag_bytes(const Geometry &G) { return ((size_t)2 << G.bm_log2) + ((size_t)2 << G.bc_log2); }

void layout(const Geometry &G, Layout &L)
{
    size_t o = 0;
    auto take = [&](size_t bytes) { size_t at = o; o = align256(o + bytes); return at; };
    const int64_t n_ids = (int64_t)1 << G.bm_log2;       // groups: fine hashed cells
    L.n_kblocks = G.n_tiles > 0 ? G.n_tiles : 1;
    L.cell_cap = L.ent_cap / 2 + 1;
    L.n_fwords = n_ids / 32;
    L.n_cwords = ((int64_t)1 << G.bc_log2) / 32;
    L.n_gtiles = ceil_div(L.n_fwords, GROUP_WORDS);
    L.o_epoch = take(64);         // first, so that every layout of a workspace shares it
    L.o_flags = take(flag_bytes(G));
    L.o_both = take((size_t)(L.n_fwords + L.n_cwords) * 4);
    L.o_grp = take((size_t)n_ids * 8);
    L.o_own = take((size_t)n_ids * 8);
    L.o_mix = take((size_t)n_ids * 4);
    L.o_gstat = take((size_t)L.n_gtiles * 16);
    L.o_ctrs = take(64);
    L.o_part = take((size_t)MARK_GRID_CAP * 16);
    L.o_pbox = take((size_t)(G.n_pairs > 0 ? G.n_pairs : 1) * 2 * 8 * sizeof(double));
    L.o_epart = take((size_t)STAT_SHARDS * SHARD_WORDS * 8);
    L.o_rng = take((size_t)(G.n_tiles * TILE_TRIS + 1) * 8);
    L.o_ent = take((size_t)(L.ent_cap + 1) * 8);
    L.o_epair = take((size_t)(L.ent_cap + 1) * 4);
    L.o_erank = take((size_t)(L.ent_cap + 1) * 4);
    L.o_ehash = take((size_t)(L.ent_cap + 1) * 4);
    L.o_sorted = take((size_t)(L.ent_cap + 1) * 8);
    L.o_spair = take((size_t)(L.ent_cap + 1) * 4);
    L.o_sbox = take((size_t)(L.ent_cap + 1) * 64);
    L.o_cells = take((size_t)L.cell_cap * sizeof(CellRec));
    L.o_pstart = take((size_t)(L.cell_cap + 1) * 8);
    L.o_htmp = take((size_t)(L.hits_cap > 0 ? L.hits_cap : 1) * sizeof(hit_t));
    L.o_hkeys = take((size_t)(L.hits_cap + 1) * 8);
    L.o_halt = take((size_t)(L.hits_cap + 1) * 8);
    L.o_misc = take(64);
    L.o_desc = take((size_t)(G.n_pairs > 1 ? G.n_pairs : 1) * sizeof(PairDesc));
    L.o_toff = take((size_t)(G.n_pairs + 1) * 8);
    L.o_cbase = take((size_t)(G.n_pairs + 1) * 8);
    L.total = o;
}

// Largest entry capacity whose layout fits ws_bytes (other capacities fixed).
bool fit_entries(const Geometry &G, Layout &L, size_t ws_bytes)
{
    L.ent_cap = 0;
    layout(G, L);
    if (L.total > ws_bytes) return false;
    int64_t lo = 0, hi = (int64_t)(ws_bytes / 16) + 1;
    while (hi - lo > 1) {
        int64_t mid = lo + (hi - lo) / 2;
        Layout t = L;
        t.ent_cap = mid;
        layout(G, t);
        if (t.total <= ws_bytes) lo = mid; else hi = mid;
    }
    L.ent_cap = lo < ((int64_t)1 << 30) - 2 ? lo : ((int64_t)1 << 30) - 2;
    layout(G, L);
    return true;
}

PairDesc make_desc(const ms_mesh *A, const ms_mesh *B, const search_params_t *p, uint64_t cell_base, int64_t tile_off)
{
    PairDesc d;
    memset(&d, 0, sizeof d);
    d.A = A->view;
    d.B = B->view;
    for (int k = 0; k < 4; ++k) { d.g.wlo[k] = p->world_lo[k]; d.g.n[k] = p->n_cells[k]; }
    d.g.inv = p->inv_edge;
    d.cell_base = cell_base;
    d.tile_off = tile_off;
    d.nA = A->view.n_tris;
    d.nB = B->view.n_tris;
    d.tilesA = (int32_t)ceil_div(d.nA, TILE_TRIS);
    d.prune = (p->flags & MS_SEARCH_PRUNE) != 0;
    const uint64_t n1 = (uint64_t)p->n_cells[1], n2 = (uint64_t)p->n_cells[2], n3 = (uint64_t)p->n_cells[3];
    d.st[0] = n1 * n2 * n3;
    d.st[1] = n2 * n3;
    d.st[2] = n3;
    d.st[3] = 1;
    // blocks of the fine table: (n + 1) / 2 per axis; of the coarse table: (n + 3) / 4
    const uint64_t f1 = (n1 + 1) >> 1, f2 = (n2 + 1) >> 1, f3 = (n3 + 1) >> 1;
    const uint64_t c1 = (n1 + 3) >> 2, c2 = (n2 + 3) >> 2, c3 = (n3 + 3) >> 2;
    d.fbs[0] = (uint32_t)(f1 * f2 * f3);
    d.fbs[1] = (uint32_t)(f2 * f3);
    d.fbs[2] = (uint32_t)f3;
    d.fbs[3] = 1;
    d.cbs[0] = (uint32_t)(c1 * c2 * c3);
    d.cbs[1] = (uint32_t)(c2 * c3);
    d.cbs[2] = (uint32_t)c3;
    d.cbs[3] = 1;
    for (int k = 0; k < 4; ++k) {
        d.fbh[k] = d.fbs[k] * HASH_MUL;
        d.cbh[k] = d.cbs[k] * HASH_MUL;
        d.nm1[k] = (double)(p->n_cells[k] - 1);
    }
    return d;
}

BatchView make_view(const Geometry &G, const PairDesc &p0, char *ws, const Layout &L)
{
    BatchView bv;
    memset(&bv, 0, sizeof bv);
    bv.p0 = p0;
    bv.pairs = (const PairDesc *)(ws + L.o_desc);
    bv.tile_off = (const int64_t *)(ws + L.o_toff);
    bv.cell_base = (const uint64_t *)(ws + L.o_cbase);
    bv.n_tiles = G.n_tiles;
    bv.n_pairs = (int32_t)G.n_pairs;
    bv.bm_log2 = G.bm_log2;
    bv.bc_log2 = G.bc_log2;
    bv.packable = G.packable;
    bv.c32 = G.c32;
    bv.pb = G.pb;
    bv.tbA = G.tbA;
    bv.tbB = G.tbB;
    bv.kl.tb = G.tb;
    bv.kl.cell_shift = G.tb + 1;
    bv.kl.tmask = (1ull << G.tb) - 1;
    return bv;
}

// Blocks of kernel fn (nt threads each) resident at once on the current
// device, 0 when the runtime cannot say; asked once per kernel and device
// (a fixed table: no allocation on this path).
inline int resident_blocks(const void *fn, int nt)
{
    struct Known {
        const void *fn;
        int dev, blocks;
    };
    static std::mutex mu;
    static Known known[64];
    static int n_known = 0;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) {
        (void)hipGetLastError();
        return 0;
    }
    std::lock_guard<std::mutex> lock(mu);
    for (int i = 0; i < n_known; ++i)
        if (known[i].fn == fn && known[i].dev == dev) return known[i].blocks;
    int per_cu = 0, cus = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, nt, 0) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) {
        (void)hipGetLastError();
        per_cu = cus = 0;
    }
    if (n_known < 64) known[n_known++] = Known{fn, dev, per_cu * cus};
    return per_cu * cus;
}

template <bool ONE, class S>
int enum_resident()
{
    return resident_blocks(reinterpret_cast<const void *>(&k_enum<ONE, S>), S::block);
}

// Queue the whole pipeline (no host synchronisation).
template <bool ONE>
int enqueue(const Geometry &G, const Layout &L, const BatchView &bv, char *ws, hit_t *hits_dev, int64_t hits_cap,
            search_stats_t *stats, uint64_t *cand_user, int64_t cand_cap, int64_t *pair_offs, hipStream_t st)
{
    int rc;
    uint64_t *epoch = (uint64_t *)(ws + L.o_epoch);
    uint8_t *flags = (uint8_t *)(ws + L.o_flags);
    uint32_t *both = (uint32_t *)(ws + L.o_both);
    uint64_t *grp = (uint64_t *)(ws + L.o_grp);
    uint64_t *own = (uint64_t *)(ws + L.o_own);
    uint32_t *mix = (uint32_t *)(ws + L.o_mix);
    uint64_t *gstat = (uint64_t *)(ws + L.o_gstat);
    uint32_t *ctrs = (uint32_t *)(ws + L.o_ctrs);     // [1] k_groups tile counter
    unsigned long long *n_keys = (unsigned long long *)(ctrs + 4);   // entries reserved by k_keys
    unsigned long long *mpart = (unsigned long long *)(ws + L.o_part);
    double *pbox = (double *)(ws + L.o_pbox);
    unsigned long long *epart = (unsigned long long *)(ws + L.o_epart);
    uint64_t *rng = (uint64_t *)(ws + L.o_rng);
    uint64_t *ent = (uint64_t *)(ws + L.o_ent);
    int32_t *epair = (int32_t *)(ws + L.o_epair);
    uint32_t *erank = (uint32_t *)(ws + L.o_erank);
    uint32_t *ehash = (uint32_t *)(ws + L.o_ehash);
    uint64_t *sorted = (uint64_t *)(ws + L.o_sorted);
    int32_t *spair = (int32_t *)(ws + L.o_spair);
    double *sbox = (double *)(ws + L.o_sbox);
    CellRec *cells = (CellRec *)(ws + L.o_cells);
    int64_t *pstart = (int64_t *)(ws + L.o_pstart);
    hit_t *htmp = (hit_t *)(ws + L.o_htmp);
    uint64_t *hkeys = (uint64_t *)(ws + L.o_hkeys);
    uint64_t *halt = (uint64_t *)(ws + L.o_halt);
    int64_t *misc = (int64_t *)(ws + L.o_misc);       // [1..2] kept groups and their slots

    // counters and look-back words: cleared by k_mark's block 0; the
    // occupancy tables need no clearing (epoch-valued marks)
    ClearSpec cs;
    memset(&cs, 0, sizeof cs);
    cs.stats = stats;
    cs.w[0] = gstat;
    cs.n[0] = 2 * L.n_gtiles;
    cs.w[1] = (uint64_t *)ctrs;
    cs.n[1] = 8;
    const unsigned g_tri = mark_grid(G.n_tiles);
    if (G.prune)
        MS_LAUNCH("k_bounds", k_bounds<ONE>, dim3((unsigned)(2 * (G.n_pairs > 0 ? G.n_pairs : 1))),
                  dim3(BOUNDS_BLOCK), 0, st, bv, pbox);
    if (G.c32)
        MS_LAUNCH("k_mark", (k_mark<ONE, true>), dim3(g_tri), dim3(BLOCK), 0, st, bv, flags, epoch, rng, pbox, mpart,
                  cs);
    else
        MS_LAUNCH("k_mark", (k_mark<ONE, false>), dim3(g_tri), dim3(BLOCK), 0, st, bv, flags, epoch, rng, pbox, mpart,
                  cs);
    MS_LAUNCH("k_pack", k_pack, dim3(grid_for(L.n_fwords + L.n_cwords, 4096)), dim3(BLOCK), 0, st, flags, epoch,
              G.bm_log2, G.bc_log2, both, grp, mix, L.n_fwords, L.n_cwords);
    KeysOut ko;
    ko.ent = ent;
    ko.epair = epair;
    ko.erank = erank;
    ko.ehash = ehash;
    ko.cap = L.ent_cap;
    ko.n_keys = n_keys;
    ko.grp = (uint32_t *)grp;
    ko.own = own;
    ko.stats = stats;
    KeysTotals kt;
    kt.mark_partial = mpart;
    kt.n_mark_partial = (int)g_tri;
    kt.shards = epart;
    const unsigned n_kb = (unsigned)(G.n_tiles > 0 ? G.n_tiles : 1) + 1;   // + the totals block
    if (G.c32)
        MS_LAUNCH("k_keys", (k_keys<ONE, true>), dim3(n_kb), dim3(KEYS_BLOCK), 0, st, bv, both, rng, ko, kt);
    else
        MS_LAUNCH("k_keys", (k_keys<ONE, false>), dim3(n_kb), dim3(KEYS_BLOCK), 0, st, bv, both, rng, ko, kt);
    GroupsOut go;
    go.both = both;
    go.grp = grp;
    go.n_fwords = L.n_fwords;
    go.cells = cells;
    go.pstart = pstart;
    go.kept = misc + 1;
    go.stat = gstat;
    go.tile_ctr = ctrs + 1;
    go.stats = stats;
    MS_LAUNCH("k_groups", k_groups, dim3((unsigned)(L.n_gtiles < 1024 ? L.n_gtiles : 1024)), dim3(BLOCK), 0, st, go);
    static_assert(GROUP_DIRECT_TILES <= 1024, "a direct k_groups launch has one block per tile");
    MS_LAUNCH("k_scatter", k_scatter<ONE>, dim3(grid_for(L.ent_cap, 8192)), dim3(BLOCK), 0, st, bv, ent, epair, erank,
              ehash, n_keys, L.ent_cap, (uint32_t *)grp, own, mix, sorted, spair, sbox, epoch, (uint4 *)flags,
              (int64_t)(flag_bytes(G) / 16));
    if (G.enum_shape == MS_ENUM_QUARTER)
        MS_LAUNCH("k_enum", (k_enum<ONE, EnumQuarter>), dim3(EnumQuarter::grid), dim3(EnumQuarter::block), 0, st, bv,
                  sorted, spair, sbox, cells, pstart, misc + 1, mix, stats, cand_user, (int32_t *)nullptr,
                  cand_user ? cand_cap : (int64_t)0, htmp, hkeys, hits_cap, epart, enum_resident<ONE, EnumQuarter>());
    else if (G.enum_shape == MS_ENUM_HALF)
        MS_LAUNCH("k_enum", (k_enum<ONE, EnumHalf>), dim3(EnumHalf::grid), dim3(EnumHalf::block), 0, st, bv, sorted,
                  spair, sbox, cells, pstart, misc + 1, mix, stats, cand_user, (int32_t *)nullptr,
                  cand_user ? cand_cap : (int64_t)0, htmp, hkeys, hits_cap, epart, enum_resident<ONE, EnumHalf>());
    else
        MS_LAUNCH("k_enum", (k_enum<ONE, EnumWide>), dim3(EnumWide::grid), dim3(EnumWide::block), 0, st, bv, sorted,
                  spair, sbox, cells, pstart, misc + 1, mix, stats, cand_user, (int32_t *)nullptr,
                  cand_user ? cand_cap : (int64_t)0, htmp, hkeys, hits_cap, epart, enum_resident<ONE, EnumWide>());
    MS_HIP(hipGetLastError());
    const bool tiny = hits_cap > 0 && hits_cap <= HITS_TINY;
    if (hits_cap > HITS_TINY) {
        if ((rc = sort_unique_small(hkeys, halt, hkeys, &stats->n_hits, hits_cap, 0, G.pb + G.tbA + G.tbB, st)))
            return rc;
        MS_LAUNCH("k_hits_place", k_hits_place, dim3(grid_for(hits_cap, 256)), dim3(BLOCK), 0, st, htmp, hkeys,
                  &stats->n_hits, hits_cap, G.tbA, G.tbB, hits_dev);
    }
    FinishArgs fa;
    fa.stats = stats;
    fa.epoch = epoch;
    fa.n_keys = n_keys;
    fa.shards = epart;
    fa.tiny = tiny ? 1 : 0;
    fa.tmp = htmp;
    fa.keys = hkeys;
    fa.cap = hits_cap;
    fa.out = hits_dev;
    MS_LAUNCH("k_finish", k_finish, dim3(1), dim3(FIN_BLOCK), 0, st, fa);
    if (hits_cap > 0 && pair_offs)
        MS_LAUNCH("k_pair_offsets", k_pair_offsets, dim3(grid_for(G.n_pairs + 1, 64)), dim3(BLOCK), 0, st, hkeys,
                  &stats->n_hits, hits_cap, (int)G.n_pairs, G.tbA + G.tbB, pair_offs);
    MS_HIP(hipGetLastError());
    return MS_OK;
}

int check_status(const search_stats_t &hs, const Geometry &G, const Layout &L, int64_t hits_cap, int64_t cand_cap,
                 bool want_cand, int64_t *needed)
{
    if (!hs.overflow) return MS_OK;
    if (needed) {
        needed[0] = hs.n_hits;
        needed[1] = hs.n_cand;
        Layout t = L;
        t.ent_cap = hs.n_entries;
        t.hits_cap = hs.n_hits > hits_cap ? hs.n_hits : hits_cap;
        t.cand_cap = want_cand ? 0 : (hs.n_cand > cand_cap ? hs.n_cand : cand_cap);
        layout(G, t);
        needed[2] = (int64_t)t.total;
    }
    if (hs.overflow & 1) return fail(MS_E_WORKSPACE, "search: entries exceed the workspace");
    return fail(MS_E_CAPACITY, "search: candidate or hit capacity exceeded");
}

// Entries of all pairs before filtering (workspace sizing); synchronises.
int count_entries(int64_t n_pairs, const ms_mesh *const *A, const ms_mesh *const *B, const search_params_t *prm,
                  unsigned long long *dev_partial, hipStream_t st, int64_t &total)
{
    total = 0;
    std::vector<unsigned long long> host(MAX_GRID);
    for (int64_t i = 0; i < n_pairs; ++i) {
        PairDesc pd = make_desc(A[i], B[i], &prm[i], 0, 0);
        const int64_t nt = (int64_t)pd.nA + pd.nB;
        const unsigned g = grid_for(nt);
        hipLaunchKernelGGL(k_count_all, dim3(g), dim3(BLOCK), 0, st, pd, dev_partial);
        MS_HIP(hipGetLastError());
        MS_HIP(hipMemcpyAsync(host.data(), dev_partial, (size_t)g * 8, hipMemcpyDeviceToHost, st));
        MS_HIP(hipStreamSynchronize(st));
        for (unsigned b = 0; b < g; ++b) total += (int64_t)host[b];
    }
    return MS_OK;
}

}  // namespace
}  // namespace ms

using namespace ms;

// ------------------------------------------------------------ single pair

extern "C" int search_workspace_size(const ms_mesh *A, const ms_mesh *B, const search_params_t *params,
                                     int64_t cand_cap, int64_t hits_cap, void *stream, size_t *bytes)
{
    if (!A || !B || !params || !bytes) return fail(MS_E_ARG, "search_workspace_size: NULL argument");
    if (cand_cap < 0 || hits_cap < 0) return fail(MS_E_ARG, "search_workspace_size: negative capacity");
    Geometry G;
    int rc = geometry(1, &A, &B, params, G);
    if (rc) return rc;
    int64_t E = 0;
    if ((rc = count_entries(1, &A, &B, params, (unsigned long long *)A->counter, (hipStream_t)stream, E))) return rc;
    Layout L;
    memset(&L, 0, sizeof L);
    L.ent_cap = E;
    L.cand_cap = cand_cap;
    L.hits_cap = hits_cap;
    layout(G, L);
    *bytes = L.total;
    return MS_OK;
}

namespace ms {
namespace {

// Checks the arguments and queues one plain search (shared by the
// synchronous and the asynchronous entry points).
int search_queue(const ms_mesh *A, const ms_mesh *B, const search_params_t *params, void *ws_dev, size_t ws_bytes,
                 hit_t *hits_dev, int64_t hits_cap, search_stats_t *stats_dev, int64_t *cand_dev, int64_t cand_cap,
                 int64_t *needed, void *stream, Geometry &G, Layout &L, bool &want_cand)
{
    if (!A || !B || !params || !stats_dev || (!ws_dev && ws_bytes)) return fail(MS_E_ARG, "search_intersections: NULL argument");
    if (hits_cap < 0 || cand_cap < 0) return fail(MS_E_ARG, "search_intersections: negative capacity");
    if (hits_cap > 0 && !hits_dev) return fail(MS_E_ARG, "search_intersections: hits_dev is NULL");
    want_cand = (params->flags & MS_SEARCH_CANDIDATES) != 0;
    if (want_cand && cand_cap > 0 && !cand_dev) return fail(MS_E_ARG, "search_intersections: cand_dev is NULL");
    if (params->flags & MS_SEARCH_STRICT) {
        ms_mesh_info_t ia, ib;
        int r0 = mesh_info(A, &ia);
        if (r0) return r0;
        if ((r0 = mesh_info(B, &ib))) return r0;
        if (ia.n_nonfinite || ib.n_nonfinite)
            return fail(MS_E_NONFINITE, "search_intersections: non-finite triangles with MS_SEARCH_STRICT");
    }
    int rc = geometry(1, &A, &B, params, G);
    if (rc) return rc;
    hipStream_t st = (hipStream_t)stream;
    memset(&L, 0, sizeof L);
    L.cand_cap = want_cand ? 0 : cand_cap;
    L.hits_cap = hits_cap;
    if (!fit_entries(G, L, ws_bytes)) {
        if (needed) { needed[0] = hits_cap; needed[1] = cand_cap; needed[2] = (int64_t)L.total; }
        return fail(MS_E_WORKSPACE, "search_intersections: workspace smaller than the fixed part");
    }
    char *ws = (char *)ws_dev;
    const PairDesc p0 = make_desc(A, B, params, 0, 0);
    const BatchView bv = make_view(G, p0, ws, L);
    return enqueue<true>(G, L, bv, ws, hits_dev, hits_cap, stats_dev, want_cand ? (uint64_t *)cand_dev : nullptr,
                         cand_cap, nullptr, st);
}

}  // namespace
}  // namespace ms

extern "C" int search_intersections(const ms_mesh *A, const ms_mesh *B, const search_params_t *params, void *ws_dev,
                                    size_t ws_bytes, hit_t *hits_dev, int64_t hits_cap, search_stats_t *stats_dev,
                                    int64_t *cand_dev, int64_t cand_cap, int64_t *needed, void *stream)
{
    Geometry G;
    Layout L;
    bool want_cand = false;
    int rc = search_queue(A, B, params, ws_dev, ws_bytes, hits_dev, hits_cap, stats_dev, cand_dev, cand_cap, needed,
                          stream, G, L, want_cand);
    if (rc) return rc;
    hipStream_t st = (hipStream_t)stream;
    search_stats_t hs;
    MS_HIP(hipMemcpyAsync(&hs, stats_dev, sizeof hs, hipMemcpyDeviceToHost, st));
    MS_HIP(hipStreamSynchronize(st));
    return check_status(hs, G, L, hits_cap, cand_cap, want_cand, needed);
}

extern "C" int search_intersections_async(const ms_mesh *A, const ms_mesh *B, const search_params_t *params,
                                          void *ws_dev, size_t ws_bytes, hit_t *hits_dev, int64_t hits_cap,
                                          search_stats_t *stats_dev, int64_t *cand_dev, int64_t cand_cap, void *stream)
{
    Geometry G;
    Layout L;
    bool want_cand = false;
    return search_queue(A, B, params, ws_dev, ws_bytes, hits_dev, hits_cap, stats_dev, cand_dev, cand_cap, nullptr,
                        stream, G, L, want_cand);
}

// ----------------------------------------------- search without allocation

namespace ms {
namespace {

// The workspace of search_intersections_noalloc: one fixed array per GPU,
// from library load to process end.  Host code never passes the array's
// name to a kernel (on the host it is only a stand-in for the symbol): it
// uses the device address that hipGetSymbolAddress returns for the current
// device, looked up once per device.
static __device__ __align__(256) unsigned char scratch[MS_NOALLOC_SCRATCH_BYTES];

constexpr int SCRATCH_DEVICES = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[SCRATCH_DEVICES];

int scratch_address(void **out)
{
    int dev = 0;
    MS_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= SCRATCH_DEVICES) return fail(MS_E_ARG, "search_intersections_noalloc: device index too large");
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
        if (!p) return fail(MS_E_HIP, "hipGetSymbolAddress(scratch) returned NULL");
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return MS_OK;
}

// Size of a layout without entries (tables, per-triangle ranges, hit
// buffers) for the table size in G.
size_t fixed_bytes(const Geometry &G, int64_t hits_cap)
{
    Layout L;
    memset(&L, 0, sizeof L);
    L.hits_cap = hits_cap;
    layout(G, L);
    return L.total;
}

}  // namespace
}  // namespace ms

extern "C" int search_intersections_noalloc(const ms_mesh *A, const ms_mesh *B, const search_params_t *params,
                                            hit_t *hits_dev, int64_t hits_cap, search_stats_t *stats_dev,
                                            int64_t *cand_dev, int64_t cand_cap, void *stream)
{
    if (!A || !B || !params || !stats_dev) return fail(MS_E_ARG, "search_intersections_noalloc: NULL argument");
    if (hits_cap < 0 || cand_cap < 0) return fail(MS_E_ARG, "search_intersections_noalloc: negative capacity");
    if (hits_cap > (int64_t)(MS_NOALLOC_SCRATCH_BYTES / sizeof(hit_t)))
        return fail(MS_E_WORKSPACE, "search_intersections_noalloc: hits_cap does not fit the fixed scratch");
    // The automatic hashed-table size is lowered until tables, per-triangle
    // ranges and hit buffers take at most half of the scratch (the rest holds
    // the entries); the results do not depend on the table size.
    search_params_t p = *params;
    if (p.table_log2 == 0) {
        Geometry G;
        int rc = geometry(1, &A, &B, &p, G);
        if (rc) return rc;
        int lg = G.bm_log2;
        for (; lg > 12; --lg) {
            G.bm_log2 = lg;
            G.bc_log2 = lg - 3;
            if (fixed_bytes(G, hits_cap) <= MS_NOALLOC_SCRATCH_BYTES / 2) break;
        }
        p.table_log2 = lg;
    }
    {
        Geometry G;
        int rc = geometry(1, &A, &B, &p, G);
        if (rc) return rc;
        const size_t need = fixed_bytes(G, hits_cap);
        if (need > MS_NOALLOC_SCRATCH_BYTES)
            return fail(MS_E_WORKSPACE, "search_intersections_noalloc: the meshes need " + std::to_string(need) +
                                            " bytes of tables before any entry, above the fixed scratch of " +
                                            std::to_string((size_t)MS_NOALLOC_SCRATCH_BYTES) + " bytes");
    }
    void *ws = nullptr;
    int rc = scratch_address(&ws);
    if (rc) return rc;
    Geometry G;
    Layout L;
    bool want_cand = false;
    return search_queue(A, B, &p, ws, MS_NOALLOC_SCRATCH_BYTES, hits_dev, hits_cap, stats_dev, cand_dev, cand_cap,
                        nullptr, stream, G, L, want_cand);
}

extern "C" int narrow_allpairs(const ms_mesh *A, const ms_mesh *B, hit_t *hits_dev, int64_t hits_cap,
                               int64_t *n_hits_dev, search_stats_t *stats_dev, void *stream)
{
    if (!A || !B || !n_hits_dev || !stats_dev) return fail(MS_E_ARG, "narrow_allpairs: NULL argument");
    if (hits_cap < 0 || (hits_cap > 0 && !hits_dev)) return fail(MS_E_ARG, "narrow_allpairs: bad hits buffer");
    hipStream_t st = (hipStream_t)stream;
    search_params_t p;
    memset(&p, 0, sizeof p);
    p.inv_edge = 1.0;
    for (int d = 0; d < 4; ++d) p.n_cells[d] = 1;
    PairDesc pd = make_desc(A, B, &p, 0, 0);
    ClearSpec cs;
    memset(&cs, 0, sizeof cs);
    cs.stats = stats_dev;
    hipLaunchKernelGGL(k_prepare, dim3(1), dim3(64), 0, st, cs);
    int64_t work = ceil_div(pd.nA, BLOCK) * ceil_div(pd.nB, AP_TILE);
    if (work > 0) {
        int64_t g = work < 8192 ? work : 8192;
        hipLaunchKernelGGL(k_allpairs, dim3((unsigned)g), dim3(BLOCK), 0, st, pd, hits_dev, hits_cap, stats_dev);
    }
    hipLaunchKernelGGL(k_copy_i64, dim3(1), dim3(1), 0, st, &stats_dev->n_hits, n_hits_dev);
    MS_HIP(hipGetLastError());
    return MS_OK;
}

// ------------------------------------------------------------------ batch

struct ms_batch {
    ms::Geometry G;
    std::vector<ms::PairDesc> desc;
    std::vector<int64_t> tile_off;
    std::vector<uint64_t> cell_base;
    int64_t ent_all;             // entries before filtering (workspace sizing)
    int64_t hits_cap, cand_cap;
    // captured graph and the buffers it was captured with; capture runs on a
    // stream of the batch's own (the caller's may be the legacy default
    // stream, which cannot be captured); the graph is launched on the
    // caller's stream
    hipStream_t cap_stream;
    hipGraph_t graph;
    hipGraphExec_t exec;
    void *g_ws;
    size_t g_ws_bytes;
    void *g_hits, *g_offs, *g_stats;
    int64_t g_hits_cap;
};

namespace ms {
namespace {

int batch_upload(ms_batch *b, char *ws, const Layout &L, hipStream_t st)
{
    const int64_t np = b->G.n_pairs;
    MS_HIP(hipMemcpyAsync(ws + L.o_desc, b->desc.data(), (size_t)np * sizeof(PairDesc), hipMemcpyHostToDevice, st));
    MS_HIP(hipMemcpyAsync(ws + L.o_toff, b->tile_off.data(), (size_t)(np + 1) * 8, hipMemcpyHostToDevice, st));
    MS_HIP(hipMemcpyAsync(ws + L.o_cbase, b->cell_base.data(), (size_t)(np + 1) * 8, hipMemcpyHostToDevice, st));
    return MS_OK;
}

}  // namespace
}  // namespace ms

namespace ms {
namespace {

// A batch plan: geometry, pair descriptors and offsets; with `count`, the
// entries before filtering are counted (kernels, synchronises) and *ws_bytes
// is the workspace for them.
int plan_batch(int32_t n_pairs, const ms_mesh *const *A, const ms_mesh *const *B, const search_params_t *params,
               int64_t hits_cap, int64_t cand_cap, bool count, void *stream, ms_batch **out, size_t *ws_bytes);

}  // namespace
}  // namespace ms

extern "C" int batch_create(int32_t n_pairs, const ms_mesh *const *A, const ms_mesh *const *B,
                            const search_params_t *params, int64_t hits_cap, int64_t cand_cap, void *stream,
                            ms_batch **out, size_t *ws_bytes)
{
    if (!out || !ws_bytes || n_pairs < 1 || !A || !B || !params || hits_cap < 0 || cand_cap < 0)
        return fail(MS_E_ARG, "batch_create: bad argument");
    return plan_batch(n_pairs, A, B, params, hits_cap, cand_cap, true, stream, out, ws_bytes);
}

namespace ms {
namespace {

int plan_batch(int32_t n_pairs, const ms_mesh *const *A, const ms_mesh *const *B, const search_params_t *params,
               int64_t hits_cap, int64_t cand_cap, bool count, void *stream, ms_batch **out, size_t *ws_bytes)
{
    *out = nullptr;
    ms_batch *b = new ms_batch();
    b->graph = nullptr;
    b->exec = nullptr;
    b->g_ws = nullptr;
    b->cap_stream = nullptr;
    int rc = geometry(n_pairs, A, B, params, b->G);
    if (rc) { delete b; return rc; }
    {
        hipError_t e = hipStreamCreateWithFlags(&b->cap_stream, hipStreamNonBlocking);
        if (e != hipSuccess) { delete b; return hip_fail(e, "hipStreamCreate"); }
    }
    b->desc.resize((size_t)n_pairs);
    b->tile_off.resize((size_t)n_pairs + 1);
    b->cell_base.resize((size_t)n_pairs + 1);
    uint64_t cb = 0;
    int64_t to = 0;
    for (int32_t i = 0; i < n_pairs; ++i) {
        uint64_t c = 0;
        pair_cells(&params[i], c);
        b->desc[(size_t)i] = make_desc(A[i], B[i], &params[i], cb, to);
        b->cell_base[(size_t)i] = cb;
        b->tile_off[(size_t)i] = to;
        cb += c;
        to += ceil_div(A[i]->view.n_tris, TILE_TRIS) + ceil_div(B[i]->view.n_tris, TILE_TRIS);
    }
    b->cell_base[(size_t)n_pairs] = cb;
    b->tile_off[(size_t)n_pairs] = to;
    int64_t E = 0;
    if (count && (rc = count_entries(n_pairs, A, B, params, (unsigned long long *)A[0]->counter, (hipStream_t)stream, E))) {
        batch_free(b);
        return rc;
    }
    b->ent_all = E;
    b->hits_cap = hits_cap;
    b->cand_cap = cand_cap;
    Layout L;
    memset(&L, 0, sizeof L);
    L.ent_cap = E;
    L.cand_cap = cand_cap;
    L.hits_cap = hits_cap;
    layout(b->G, L);
    if (ws_bytes) *ws_bytes = L.total;
    *out = b;
    return MS_OK;
}

}  // namespace
}  // namespace ms

extern "C" int batch_free(ms_batch *b)
{
    if (!b) return MS_OK;
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    if (b->cap_stream) (void)hipStreamDestroy(b->cap_stream);
    delete b;
    return MS_OK;
}

extern "C" int batch_search(ms_batch *b, void *ws_dev, size_t ws_bytes, hit_t *hits_dev, int64_t hits_cap,
                            int64_t *pair_hit_offsets_dev, search_stats_t *stats_dev, int32_t use_graph, void *stream)
{
    if (!b || !ws_dev || !stats_dev || !pair_hit_offsets_dev || hits_cap < 0 || (hits_cap > 0 && !hits_dev))
        return fail(MS_E_ARG, "batch_search: bad argument");
    if (hits_cap > b->hits_cap) return fail(MS_E_ARG, "batch_search: hits_cap above the value the batch was sized for");
    hipStream_t st = (hipStream_t)stream;
    Layout L;
    memset(&L, 0, sizeof L);
    L.cand_cap = b->cand_cap;
    L.hits_cap = hits_cap;
    if (!fit_entries(b->G, L, ws_bytes)) return fail(MS_E_WORKSPACE, "batch_search: workspace smaller than the fixed part");
    char *ws = (char *)ws_dev;
    const BatchView bv = make_view(b->G, b->desc[0], ws, L);
    int rc;
    if (!use_graph) {
        if ((rc = batch_upload(b, ws, L, st))) return rc;
        return enqueue<false>(b->G, L, bv, ws, hits_dev, hits_cap, stats_dev, nullptr, L.cand_cap,
                              pair_hit_offsets_dev, st);
    }
    const bool same = b->exec && b->g_ws == ws_dev && b->g_ws_bytes == ws_bytes && b->g_hits == (void *)hits_dev &&
                      b->g_offs == (void *)pair_hit_offsets_dev && b->g_stats == (void *)stats_dev &&
                      b->g_hits_cap == hits_cap;
    if (!same) {
        if (b->exec) { (void)hipGraphExecDestroy(b->exec); b->exec = nullptr; }
        if (b->graph) { (void)hipGraphDestroy(b->graph); b->graph = nullptr; }
        // the descriptors go to the workspace once, outside the graph
        if ((rc = batch_upload(b, ws, L, st))) return rc;
        MS_HIP(hipStreamSynchronize(st));
        hipStream_t cs = b->cap_stream;
        MS_HIP(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
        rc = enqueue<false>(b->G, L, bv, ws, hits_dev, hits_cap, stats_dev, nullptr, L.cand_cap, pair_hit_offsets_dev,
                            cs);
        hipGraph_t g = nullptr;
        hipError_t e = hipStreamEndCapture(cs, &g);
        if (rc) { if (g) (void)hipGraphDestroy(g); return rc; }
        if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture");
        hipGraphExec_t x = nullptr;
        e = hipGraphInstantiate(&x, g, nullptr, nullptr, 0);
        if (e != hipSuccess) { (void)hipGraphDestroy(g); return hip_fail(e, "hipGraphInstantiate"); }
        b->graph = g;
        b->exec = x;
        b->g_ws = ws_dev;
        b->g_ws_bytes = ws_bytes;
        b->g_hits = hits_dev;
        b->g_offs = pair_hit_offsets_dev;
        b->g_stats = stats_dev;
        b->g_hits_cap = hits_cap;
    }
    MS_HIP(hipGraphLaunch(b->exec, st));
    return MS_OK;
}

extern "C" int batch_needed(const ms_batch *b, const search_stats_t *stats_host, int64_t *needed)
{
    if (!b || !stats_host || !needed) return fail(MS_E_ARG, "batch_needed: NULL argument");
    Layout L;
    memset(&L, 0, sizeof L);
    L.ent_cap = stats_host->n_entries > b->ent_all ? stats_host->n_entries : b->ent_all;
    L.hits_cap = stats_host->n_hits > b->hits_cap ? stats_host->n_hits : b->hits_cap;
    L.cand_cap = stats_host->n_cand > b->cand_cap ? stats_host->n_cand : b->cand_cap;
    layout(b->G, L);
    needed[0] = L.hits_cap;
    needed[1] = L.cand_cap;
    needed[2] = (int64_t)L.total;
    return MS_OK;
}

// ------------------------------------------------------ one-call batched form

namespace ms {
namespace {

// Plans of search_intersections_batched, reused by calls with the same
// pairs (descriptor bytes: vertex pointers, grid sizes, cell grids), the
// same buffers and the same device, so that a repeated call launches the
// graph it captured.  A few are kept; the oldest is released when a new one
// is needed (after its last launch has finished).
struct BatchedPlan {
    std::vector<PairDesc> key;
    int device;
    void *ws, *hits, *offs, *stats;
    size_t ws_bytes;
    int64_t hits_cap;
    ms_batch *plan;
    hipEvent_t done;
};

constexpr size_t BATCHED_PLANS = 8;
std::mutex g_bp_mu;
std::vector<BatchedPlan> g_bp;

bool same_plan(const BatchedPlan &p, const std::vector<PairDesc> &key, int dev, void *ws, size_t ws_bytes,
               void *hits, int64_t hits_cap, void *offs, void *stats)
{
    return p.device == dev && p.ws == ws && p.ws_bytes == ws_bytes && p.hits == hits && p.hits_cap == hits_cap &&
           p.offs == offs && p.stats == stats && p.key.size() == key.size() &&
           memcmp(p.key.data(), key.data(), key.size() * sizeof(PairDesc)) == 0;
}

}  // namespace
}  // namespace ms

extern "C" int search_batched_workspace_size(int32_t n_pairs, const ms_mesh *const *A, const ms_mesh *const *B,
                                             const search_params_t *per_pair, int64_t hits_cap, void *stream,
                                             size_t *bytes)
{
    if (!bytes || n_pairs < 1 || !A || !B || !per_pair || hits_cap < 0)
        return fail(MS_E_ARG, "search_batched_workspace_size: bad argument");
    ms_batch *b = nullptr;
    int rc = plan_batch(n_pairs, A, B, per_pair, hits_cap, 0, true, stream, &b, bytes);
    batch_free(b);
    return rc;
}

extern "C" int search_intersections_batched(int32_t n_pairs, const ms_mesh *const *A, const ms_mesh *const *B,
                                            const search_params_t *per_pair, void *ws_dev, size_t ws_bytes,
                                            hit_t *hits_dev, int64_t hits_cap, int64_t *pair_hit_offsets_dev,
                                            search_stats_t *stats_dev, int32_t use_graph, void *stream)
{
    if (n_pairs < 1 || !A || !B || !per_pair || !ws_dev || !stats_dev || !pair_hit_offsets_dev || hits_cap < 0 ||
        (hits_cap > 0 && !hits_dev))
        return fail(MS_E_ARG, "search_intersections_batched: bad argument");
    Geometry G;
    int rc = geometry(n_pairs, A, B, per_pair, G);
    if (rc) return rc;
    std::vector<PairDesc> key((size_t)n_pairs);
    {
        uint64_t cb = 0;
        int64_t to = 0;
        for (int32_t i = 0; i < n_pairs; ++i) {
            uint64_t c = 0;
            pair_cells(&per_pair[i], c);
            key[(size_t)i] = make_desc(A[i], B[i], &per_pair[i], cb, to);
            cb += c;
            to += ceil_div(A[i]->view.n_tris, TILE_TRIS) + ceil_div(B[i]->view.n_tris, TILE_TRIS);
        }
    }
    int dev = 0;
    MS_HIP(hipGetDevice(&dev));
    hipStream_t st = (hipStream_t)stream;
    std::lock_guard<std::mutex> lk(g_bp_mu);
    BatchedPlan *bp = nullptr;
    for (BatchedPlan &p : g_bp)
        if (same_plan(p, key, dev, ws_dev, ws_bytes, hits_dev, hits_cap, pair_hit_offsets_dev, stats_dev)) bp = &p;
    if (!bp) {
        if (g_bp.size() >= BATCHED_PLANS) {
            BatchedPlan &old = g_bp.front();
            (void)hipEventSynchronize(old.done);
            (void)hipEventDestroy(old.done);
            batch_free(old.plan);
            g_bp.erase(g_bp.begin());
        }
        BatchedPlan np;
        np.key = key;
        np.device = dev;
        np.ws = ws_dev;
        np.ws_bytes = ws_bytes;
        np.hits = hits_dev;
        np.hits_cap = hits_cap;
        np.offs = pair_hit_offsets_dev;
        np.stats = stats_dev;
        if ((rc = plan_batch(n_pairs, A, B, per_pair, hits_cap, 0, false, stream, &np.plan, nullptr))) return rc;
        hipError_t e = hipEventCreateWithFlags(&np.done, hipEventDisableTiming);
        if (e != hipSuccess) { batch_free(np.plan); return hip_fail(e, "hipEventCreate"); }
        g_bp.push_back(np);
        bp = &g_bp.back();
    }
    if ((rc = batch_search(bp->plan, ws_dev, ws_bytes, hits_dev, hits_cap, pair_hit_offsets_dev, stats_dev, use_graph,
                           stream)))
        return rc;
    MS_HIP(hipEventRecord(bp->done, st));
    return MS_OK;
}

// ---------------------------------------------------------------- profiling

namespace ms {
namespace {

struct Profiler {
    bool on = false;
    std::vector<const char *> names;
    std::vector<hipEvent_t> events;   // start / stop pairs, grows on demand
    size_t used = 0;                  // pairs handed out since the last read
};

thread_local Profiler g_prof;

}  // namespace

bool prof_pair(const char *name, hipStream_t st, hipEvent_t *start, hipEvent_t *stop)
{
    Profiler &P = g_prof;
    if (!P.on) return false;
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(st, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone) return false;
    while (P.events.size() < 2 * (P.used + 1)) {
        hipEvent_t e;
        if (hipEventCreate(&e) != hipSuccess) { P.on = false; return false; }
        P.events.push_back(e);
    }
    if (P.names.size() < P.used + 1) P.names.resize(P.used + 1);
    P.names[P.used] = name;
    *start = P.events[2 * P.used];
    *stop = P.events[2 * P.used + 1];
    ++P.used;
    return true;
}

}  // namespace ms

extern "C" int search_profile_enable(int on)
{
    ms::g_prof.on = on != 0;
    ms::g_prof.used = 0;
    return MS_OK;
}

extern "C" int search_profile_read(char *names, size_t names_len, double *ms_out, int cap, int *n_out)
{
    if (!n_out || (cap > 0 && !ms_out)) return ms::fail(MS_E_ARG, "search_profile_read: NULL argument");
    ms::Profiler &P = ms::g_prof;
    int n = (int)P.used;
    *n_out = n;
    if (n == 0) return MS_OK;
    MS_HIP(hipEventSynchronize(P.events[2 * (P.used - 1) + 1]));
    std::string csv;
    for (int i = 0; i < n && i < cap; ++i) {
        float t = 0.f;
        MS_HIP(hipEventElapsedTime(&t, P.events[2 * i], P.events[2 * i + 1]));
        ms_out[i] = t;
        if (i) csv += ",";
        csv += P.names[i];
    }
    P.used = 0;
    if (names && names_len) {
        size_t k = csv.size() < names_len - 1 ? csv.size() : names_len - 1;
        memcpy(names, csv.data(), k);
        names[k] = 0;
    }
    return MS_OK;
}
