/*
 * msearch.h -- C ABI of the MI355X (gfx950) manifold-mesh intersection
 * search and stroboscopic-map library (libmsearch.so).
 *
 * Method: Kumar, Anderson, de la Llave, "Rapid GPU-assisted search and
 * parameterization-based refinement and continuation of connections between
 * tori in periodically perturbed planar circular restricted 3-body problems",
 * arXiv 2109.14814.  Section numbers below refer to that paper.
 *
 * Conventions for every entry point
 *   - Return value: MS_OK (0) or a negative MS_E_* code.  After an error,
 *     last_error() returns a thread-local description.  No C++ exception
 *     crosses this boundary.
 *   - Pointers named *_dev are device (HBM) pointers owned by the caller; the
 *     library borrows them for the duration of the call (and, for vertices
 *     passed to mesh_build, for the lifetime of the mesh handle).  Pointers
 *     named *_host are host pointers.
 *   - `stream` is a hipStream_t (passed as void* so that this header needs no
 *     HIP include); NULL means the default stream.  All device work is queued
 *     on that stream.  Unless stated otherwise a call returns once its work is
 *     queued.
 *   - FP64 throughout.  The search kernels are built with contraction off,
 *     so each operation of the pair predicate rounds once as written (the
 *     oracle does the same, and the decisions agree bit for bit).  The
 *     Runge-Kutta and refinement kernels let the compiler fuse multiply-adds;
 *     their results agree with the oracle within the stated tolerances.
 */
#ifndef MSEARCH_H
#define MSEARCH_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---------------------------------------------------------------- status */
enum {
    MS_OK = 0,
    MS_E_ARG = -1,        /* invalid argument (NULL, negative size, bad flag) */
    MS_E_CAPACITY = -2,   /* an output buffer is too small; *needed says how large */
    MS_E_HIP = -3,        /* a HIP runtime call failed (text in last_error) */
    MS_E_NONFINITE = -4,  /* non-finite vertex with MS_SEARCH_STRICT */
    MS_E_KEYBITS = -5,    /* grid too fine: cell index does not fit the entry word */
    MS_E_WORKSPACE = -6   /* workspace too small for this search; query again */
};

/* Thread-local text of the last error (never NULL). */
const char *last_error(void);

/* ------------------------------------------------------------------ mesh */

/* Opaque mesh handle: triangle table and per-triangle 4D boxes in HBM. */
typedef struct ms_mesh ms_mesh;

/* Vertex layouts accepted by mesh_build. */
enum {
    MS_LAYOUT_AOS = 0,    /* (n_s_v * n_theta_v) x 4 doubles, theta index fastest,
                             (x, y, p_x, p_y) of one vertex contiguous (32 B).
                             Borrowed: must outlive the handle. */
    MS_LAYOUT_SOA = 1     /* four planes x[n_s_v][n_theta_v], y, p_x, p_y, back to
                             back (the four N x M arrays of Sec. 6.1, stored with
                             theta fastest).  Copied into an owned AoS buffer by
                             mesh_build and again by every mesh_update, which reads
                             the planes at the pointer given to mesh_build (keep them
                             valid while the handle may be updated). */
};

/*
 * mesh_build -- triangulate a vertex grid W(theta_i, s_k) (Sec. 6.1).
 *
 * Quad (i, k) joins W(i,k), W(i+1,k), W(i,k+1), W(i+1,k+1); when periodic
 * != 0, i+1 is taken mod n_theta_v (theta_N = theta_0 + 2 pi) so there are
 * n_theta_v quads per s-row, otherwise n_theta_v - 1.  Quad q = i + k*Nq is
 * split along W(i+1,k)-W(i,k+1) into triangles 2q (T1) and 2q+1 (T2), with
 * the vertex order of the narrow phase (Sec. 6.2.4):
 *   T1: p1 = W(i+1,k), p2 = W(i,k),     p3 = W(i,k+1)
 *   T2: p1 = W(i,k+1), p2 = W(i+1,k+1), p3 = W(i+1,k)
 * theta_host[n_theta_v] and s_host[n_s_v] are the sample values used for the
 * (theta, s) estimates of hits; they are copied.  A triangle with a
 * non-finite coordinate takes no part in any search.  The triangles' 4D
 * boxes (Sec. 6.2.2) are not stored: every kernel that needs one computes it
 * from the three vertices.  Runs the statistics pass of mesh_info and
 * synchronises `stream` before returning.  A grid with fewer than 2 vertices
 * along s (or along a non-periodic theta) has no triangles and is valid.
 */
int mesh_build(const double *verts_dev, int32_t n_theta_v, int32_t n_s_v, int32_t periodic,
               int32_t layout, const double *theta_host, const double *s_host, void *stream,
               ms_mesh **out);

/* Release a handle and its device buffers (NULL is accepted). */
int mesh_free(ms_mesh *mesh);

typedef struct {
    int64_t n_tris;        /* 2 * Nq * (n_s_v - 1) */
    int64_t n_nonfinite;   /* triangles excluded for non-finite coordinates */
    double lo[4], hi[4];   /* bounds of the finite triangles (+inf/-inf if none) */
    double mean_diam;      /* mean over finite triangles of the longest 4D edge */
} ms_mesh_info_t;

/* Bounds, diameter and counts of a mesh.  After mesh_update this runs the
 * statistics pass on the stream given there and synchronises it. */
int mesh_info(const ms_mesh *mesh, ms_mesh_info_t *out);

/*
 * mesh_update -- tell the handle that the caller changed the vertex values
 * in place (same grid, same buffer; e.g. after propagate_vertices on
 * `stream`).  An AoS mesh's searches read the caller's vertices directly, so
 * for it this only marks the statistics of mesh_info (and so
 * search_default_params) for recomputation on `stream`, and queues nothing.
 * An SoA mesh's searches read the handle's AoS copy: mesh_update queues the
 * conversion of the current planes into that copy on `stream`.  Allocates
 * nothing.
 */
int mesh_update(ms_mesh *mesh, void *stream);

/* --------------------------------------------------------------- search */

/* Search flags. */
enum {
    MS_SEARCH_CANDIDATES = 1,   /* also write the candidate set C to cand_dev */
    MS_SEARCH_STRICT = 2,       /* fail with MS_E_NONFINITE if a mesh has non-finite triangles */
    MS_SEARCH_PRUNE = 4         /* world-bound pruning (Sec. 6.2.1): a triangle whose box misses the
                                   other mesh's box (over its finite vertices, computed by the search
                                   itself: one block per mesh, so it pays for small meshes such as
                                   half-layers) takes no part in the grid.  Hits and candidates do not
                                   change; n_cells and n_slots then describe the pruned grid
                                   (n_entries_all still counts every finite triangle's cells). */
};

/*
 * Uniform grid of Sec. 6.2.1 in the 0-based form: cell of coordinate x on
 * axis d is clamp(floor((x - world_lo[d]) * inv_edge), 0, n_cells[d] - 1),
 * evaluated in FP64.  The grid only decides which pairs are examined; the
 * hit set does not depend on it (every box-overlapping pair shares the cell
 * of the componentwise max of the two boxes' lower corners and is examined
 * there exactly once).
 */
typedef struct {
    double world_lo[4];
    double inv_edge;        /* 1 / cell edge, > 0 and finite */
    int64_t n_cells[4];     /* cells per axis, >= 1 */
    int32_t flags;          /* MS_SEARCH_* */
    int32_t table_log2;     /* 0: automatic; else log2 of the hashed occupancy table per
                               side, clamped to [8, 27]; the automatic size is within
                               [12, 25] (smaller: more cells share a group;
                               results do not change, only the work) */
    int32_t enum_shape;     /* work tile of the pair enumeration (MS_ENUM_*; 0: MS_ENUM_HALF;
                               a batch takes its first pair's); results do not change,
                               only the time */
    int32_t reserved;       /* 0 */
} search_params_t;

/* Enumeration work tiles: a block takes a chunk of consecutive slots and
 * stages the entries they need in LDS. */
enum {
    MS_ENUM_WIDE = 1,       /* 512 threads x 8 slots, up to 768 staged entries: one block per CU */
    MS_ENUM_HALF = 2,       /* 256 threads x 8 slots, up to 384 staged entries: two blocks per CU */
    MS_ENUM_QUARTER = 3     /* 128 threads x 8 slots, up to 192 staged entries: four blocks per CU */
};

/* World = box of both meshes' finite triangles, edge = kappa * the geometric
 * mean of the two meshes' mean triangle diameters (longest edge; one mesh's
 * alone when the other has no finite triangle), n_cells[d] = max(1,
 * ceil(span_d * inv_edge)); table_log2 = 0, enum_shape = 0. */
int search_default_params(const ms_mesh *A, const ms_mesh *B, double kappa, search_params_t *out);

/*
 * Hit record (120 B).  (u, v) are the coordinates of the intersection point
 * on A's triangle and (a, b) on B's, in the form of the narrow-phase system
 * p2 + (p1 - p2) u + (p3 - p2) v = q2 + (q1 - q2) a + (q3 - q2) b
 * (Sec. 6.2.4; the paper writes (a, b, c, d)).  X is the point
 * (p2 + u (p1 - p2)) + v (p3 - p2); (thA, sA) and (thB, sB) the parameter
 * estimates of Sec. 6.2.4; margin = min(u, v, a, b, 1-(u+v), 1-(a+b)).
 */
typedef struct {
    int32_t triA, triB;
    uint32_t flags, pad;
    double u, v, a, b;
    double X[4];
    double thA, sA, thB, sB;
    double margin;
} hit_t;

/* Counters written by a search (device memory, int64 each). */
typedef struct {
    int64_t n_entries;       /* (cell, triangle) entries after the both-sides filter on hashed cells */
    int64_t n_entries_all;   /* entries before the filter */
    int64_t n_cells;         /* distinct cells holding both meshes (Alg. 1's boxes, exact) */
    int64_t n_slots;         /* sum over those cells of nA * nB (exact) */
    int64_t n_cand;          /* |C|: distinct box-overlapping pairs */
    int64_t n_moller;        /* candidates rejected by the Moller test */
    int64_t n_degenerate;    /* candidates with a singular 4x4 system */
    int64_t n_outside;       /* solved, intersection outside a triangle */
    int64_t n_hits;          /* |H| */
    int64_t n_nonfinite;     /* triangles of A and B excluded */
    int64_t overflow;        /* bit 0: entries > capacity, bit 1: cand, bit 2: hits */
    int64_t n_groups;        /* groups enumerated: hashed cells with A and B entries (>= n_cells) */
    int64_t n_group_slots;   /* sum over those groups of nA * nB (>= n_slots) */
    int64_t n_chunks_unstaged; /* enumeration chunks whose entries did not fit on-chip (crowded
                                  cells; their slots were read from device memory) */
    int64_t reserved[2];     /* zero */
} search_stats_t;

/*
 * search_workspace_size -- bytes of device workspace that search_intersections
 * needs for this pair and grid, with room for cand_cap candidates and
 * hits_cap hits.  Runs an entry-count kernel on `stream` and synchronises it.
 * Returns MS_E_KEYBITS when the entry word [cell | side | triangle] needs
 * more than 63 bits (prod(n_cells) too large for the triangle counts).
 */
int search_workspace_size(const ms_mesh *A, const ms_mesh *B, const search_params_t *params,
                          int64_t cand_cap, int64_t hits_cap, void *stream, size_t *bytes);

/*
 * search_intersections -- H = { (A_i, B_j) : triangles intersect } (Sec. 6.2),
 * by the GPU pipeline: one entry per covered cell that both meshes occupy,
 * entries grouped by hashed cell (counted and scattered, no sort), pair
 * enumeration inside each group with the same-cell, home-cell and box tests
 * (Sec. 6.2.2), Moller quick test (Sec. 6.2.3) and the 4x4 narrow phase
 * (Sec. 6.2.4), hits sorted by (triA, triB).
 *   ws_dev/ws_bytes: workspace from search_workspace_size (not shared with a
 *     concurrent call); cand_cap and hits_cap must not exceed the values the
 *     workspace was sized for.  The workspace keeps state from one search to
 *     the next (occupancy marks tagged with a search counter, so that no
 *     clearing pass runs); results never depend on its contents, but zero it
 *     once after allocation so that the work counters of its first search
 *     (n_entries, n_groups, n_group_slots) carry no leftover marks.
 *   hits_dev/hits_cap: output records, sorted by (triA, triB).
 *   stats_dev: one search_stats_t in device memory, written by the search.
 *   cand_dev/cand_cap: with MS_SEARCH_CANDIDATES, receives C as packed
 *     (triA << 32 | triB), unordered; else ignored (may be NULL).
 *   needed (host, may be NULL): on MS_E_CAPACITY / MS_E_WORKSPACE, needed[0] =
 *     hits, needed[1] = candidates, needed[2] = workspace bytes required.
 * Synchronises `stream` at the end to check capacities and returns
 * MS_E_CAPACITY or MS_E_WORKSPACE when a buffer overflowed (outputs are then
 * incomplete but every write stayed in bounds).
 */
int search_intersections(const ms_mesh *A, const ms_mesh *B, const search_params_t *params,
                         void *ws_dev, size_t ws_bytes, hit_t *hits_dev, int64_t hits_cap,
                         search_stats_t *stats_dev, int64_t *cand_dev, int64_t cand_cap,
                         int64_t *needed, void *stream);

/*
 * search_intersections_async -- the same search without the final
 * synchronisation: returns once the kernels are queued on `stream`.  A buffer
 * overflow is reported only in stats_dev->overflow (bit 0 entries, bit 1
 * candidates, bit 2 hits); read it after the stream has completed and, if
 * set, call search_intersections to learn the sizes needed.  For loops that
 * search repeatedly without host round trips.
 */
int search_intersections_async(const ms_mesh *A, const ms_mesh *B, const search_params_t *params, void *ws_dev,
                               size_t ws_bytes, hit_t *hits_dev, int64_t hits_cap, search_stats_t *stats_dev,
                               int64_t *cand_dev, int64_t cand_cap, void *stream);

/*
 * search_intersections_noalloc -- for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc): search_intersections_async with no workspace argument.
 * The workspace is a fixed device array inside the library,
 * MS_NOALLOC_SCRATCH_BYTES per GPU, held from library load to process end;
 * the call allocates nothing (no hipMalloc, no hipFree).  The caller still
 * passes the outputs (hits, stats, candidates), as for the other searches.
 *   - Every call on a GPU shares that GPU's array, which keeps the last
 *     call's contents (results never depend on them; the counters the
 *     search needs cleared are cleared by its first kernel).  Calls that
 *     overlap on one GPU (other streams, other threads) race: serialise them.
 *   - table_log2 = 0 picks the largest hashed table whose fixed part (tables,
 *     per-triangle ranges, hit buffers) takes at most half of the array; the
 *     rest holds the entries.  Returns MS_E_WORKSPACE, with the bytes needed
 *     in last_error(), when the fixed part alone exceeds the array (meshes of
 *     more than a few million triangles, or a large explicit table_log2 or
 *     hits_cap).  Entries beyond the rest set stats_dev->overflow bit 0, like
 *     the other asynchronous search; read it after the stream completes.
 *   - Asynchronous (returns once queued); with MS_SEARCH_STRICT it first
 *     waits for the meshes' statistics (mesh_info).  The first call on a
 *     device looks up the array's device address (no allocation).
 */
#define MS_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
int search_intersections_noalloc(const ms_mesh *A, const ms_mesh *B, const search_params_t *params,
                                 hit_t *hits_dev, int64_t hits_cap, search_stats_t *stats_dev,
                                 int64_t *cand_dev, int64_t cand_cap, void *stream);

/*
 * narrow_allpairs -- the full pair test (Moller, 4x4 solve, inclusion) on every
 * pair of A x B with no grid and no early exit (the box test is evaluated and
 * folded into the decision): the "tri-pair tests/s" workload.  Hits are
 * written unordered to hits_dev; *n_hits_dev (device int64) receives |H|;
 * stats_dev (optional) receives the per-stage counters.  Asynchronous.
 */
int narrow_allpairs(const ms_mesh *A, const ms_mesh *B, hit_t *hits_dev, int64_t hits_cap,
                    int64_t *n_hits_dev, search_stats_t *stats_dev, void *stream);

/*
 * Batched search: many mesh pairs (e.g. the members of a torus family or the
 * half-layer pairs of Sec. 5 / Sec. 6.4) searched together by one pass of
 * the pipeline.  Each pair keeps its own grid; the cells of pair i are
 * offset so that no two pairs share a cell.  Hits come out sorted by (pair,
 * triA, triB); hit_t.flags holds the pair index.
 *
 * batch_create -- plan a batch: copies the pair descriptors (the meshes
 *   must stay alive and unchanged in topology), counts entries (runs kernels
 *   on `stream`, synchronises) and returns the workspace size for hits_cap
 *   hits and cand_cap internal candidates.
 * batch_search -- queue the search of every pair (asynchronous; no host
 *   synchronisation).  pair_hit_offsets_dev receives n_pairs + 1 int64 offsets
 *   into hits_dev.  With use_graph != 0 the kernel sequence is captured into a
 *   HIP graph on the first call (and again whenever a buffer argument
 *   changes) and later calls launch the graph.  Capacity overflow is
 *   reported in stats_dev->overflow (check it after synchronising);
 *   batch_needed then gives the sizes to re-plan with.
 * batch_free -- release the plan and its graph.
 */
typedef struct ms_batch ms_batch;
int batch_create(int32_t n_pairs, const ms_mesh *const *A, const ms_mesh *const *B, const search_params_t *params,
                 int64_t hits_cap, int64_t cand_cap, void *stream, ms_batch **out, size_t *ws_bytes);
int batch_search(ms_batch *batch, void *ws_dev, size_t ws_bytes, hit_t *hits_dev, int64_t hits_cap,
                 int64_t *pair_hit_offsets_dev, search_stats_t *stats_dev, int32_t use_graph, void *stream);
/* needed[0] hits, needed[1] candidates, needed[2] workspace bytes for the
 * counts of a finished search (stats copied to the host). */
int batch_needed(const ms_batch *batch, const search_stats_t *stats_host, int64_t *needed);
int batch_free(ms_batch *batch);

/*
 * One-call form of the batched search (the independent searches of many
 * half-layer pairs of Sec. 6.4, or of a torus family, in one call).
 * search_batched_workspace_size -- workspace bytes for these pairs with
 *   room for hits_cap hits (counts entries: runs kernels on `stream` and
 *   synchronises it).
 * search_intersections_batched -- search every pair: hits sorted by (pair,
 *   triA, triB) with hit_t.flags = pair index, pair_hit_offsets_dev[n_pairs +
 *   1] (int64, device) the offsets of each pair's hits, stats_dev the totals.
 *   Every pair keeps its own grid (per_pair[i]).  The library keeps the plans
 *   of its last 8 distinct calls (keyed by the pairs' meshes, vertex
 *   pointers and grids, and by the buffers): a repeated call reuses its plan
 *   and, with use_graph != 0, launches the HIP graph captured by its first
 *   call.  Asynchronous, except that the first call of a plan with
 *   use_graph != 0 synchronises `stream` once before capturing (so capture
 *   such a call into a graph of your own only with use_graph = 0).
 *   Overflow is reported in stats_dev->overflow (check after synchronising);
 *   call search_batched_workspace_size again with the counts to size anew.
 *   Releasing an old plan waits for its last launch.  Calls that overlap on
 *   one workspace race.
 */
int search_batched_workspace_size(int32_t n_pairs, const ms_mesh *const *A, const ms_mesh *const *B,
                                  const search_params_t *per_pair, int64_t hits_cap, void *stream, size_t *bytes);
int search_intersections_batched(int32_t n_pairs, const ms_mesh *const *A, const ms_mesh *const *B,
                                 const search_params_t *per_pair, void *ws_dev, size_t ws_bytes, hit_t *hits_dev,
                                 int64_t hits_cap, int64_t *pair_hit_offsets_dev, search_stats_t *stats_dev,
                                 int32_t use_graph, void *stream);

/*
 * Kernel timing for benchmarks.  While enabled (per calling thread), every
 * kernel that mesh_info and the searches queue on an uncaptured stream is
 * launched with a start and a stop event that take that dispatch's own begin
 * and end timestamps.  search_profile_read waits for the last of them and
 * returns the names (comma separated) and durations in ms of the kernels
 * launched since the previous read (at most cap of them; *n receives the
 * number), then starts a new record.
 */
int search_profile_enable(int on);
int search_profile_read(char *names, size_t names_len, double *ms, int cap, int *n);

/* ------------------------------------------------------------------ map */

/* Planar elliptic restricted three-body problem in pulsating rotating
 * coordinates with the true anomaly f as independent variable (the model
 * family of Sec. 3.2-3.3):
 *   x'' - 2 y' = w(f) dOmega/dx,  y'' + 2 x' = w(f) dOmega/dy,
 *   w = 1 / (1 + e cos f), Omega = (x^2+y^2)/2 + (1-mu)/r1 + mu/r2.
 * The stroboscopic map F advances f by 2 pi (Sec. 4.1). */
typedef struct {
    double mu, e;
    int32_t steps_per_period;   /* fixed RK8 steps per 2 pi of f */
    int32_t n_periods;          /* F^n_periods; negative = backwards */
} map_params_t;

/*
 * propagate_vertices -- out = F^n(in) for n_vertices states (x, y, x', y'),
 * AoS 4 doubles each, by the 11-stage order-8 explicit Runge-Kutta method of
 * Cooper & Verner (1972) with fixed steps (the globalization maps
 * F^{+-k} of Sec. 4.3).  in_dev may equal out_dev.  Asynchronous: queues one
 * kernel (the stage weights w(f) are computed on the GPU inside it), allocates
 * nothing, never synchronises, and can be captured into a HIP graph.
 */
int propagate_vertices(const double *in_dev, double *out_dev, int64_t n_vertices,
                       const map_params_t *params, void *stream);

/*
 * The same problem in the position-momentum coordinates of Sec. 3.3: time t,
 * primaries on a Kepler ellipse of semi-major axis 1, eccentricity
 * params->e and period 2 pi with periapse at t = 0, 2 pi, ...; the frame
 * turns with the primaries but is not rescaled, so they sit at (-mu rho, 0)
 * and ((1 - mu) rho, 0) with rho(t) = 1 - e cos E(t), E - e sin E = t.  The
 * state z = (x, y, px, py) follows Hamilton's equations of
 *   H = (px^2 + py^2)/2 + n(t) (px y - py x) - (1 - mu)/r1 - mu/r2,
 *   r1 = |(x + mu rho, y)|, r2 = |(x - (1 - mu) rho, y)|,
 * n(t) the rate of the primaries' true anomaly.  The stroboscopic map F
 * advances t by 2 pi from a periapse (Sec. 4.1); steps_per_period RK8 steps
 * (Cooper & Verner) per period, F^n_periods, negative = backwards.
 */

/* pertbp_map -- out = F^n(in) for n_states states (x, y, px, py), AoS 4
 * doubles each, device arrays.  in_dev may equal out_dev.  Asynchronous on
 * stream; MS_E_ARG for a bad pointer, steps_per_period <= 0, e outside
 * [0, 1) or mu outside [0, 1].  The kernel solves Kepler's equation for the
 * stage times on the GPU; the call allocates nothing, never synchronises and
 * can be captured into a HIP graph. */
int pertbp_map(const double *in_dev, double *out_dev, int64_t n_states, const map_params_t *params,
               void *stream);

/* pertbp_map_stm -- F^n(in) and its state transition matrix DF^n (the
 * matrices of the derivative formulas of Sec. 7), from the variational
 * equations integrated with the same RK8 stages (the exact derivative of the
 * discrete map).
 *   out_dev  n_states x 4 (may be NULL; may equal in_dev)
 *   stm_dev  n_states x 16, row-major per state: stm[16 p + 4 i + j] =
 *            d out_i / d in_j; must not overlap in_dev or out_dev.
 *   cols_per_thread  1, 2 or 4 columns of DF per GPU thread (4 / cols
 *            threads per state), or 0 for the default (4 from 131,072 states
 *            up, 2 from 65,536, else 1); a tuning choice only, the results
 *            are identical.
 * Asynchronous; errors as pertbp_map. */
int pertbp_map_stm(const double *in_dev, double *out_dev, double *stm_dev, int64_t n_states,
                   const map_params_t *params, int32_t cols_per_thread, void *stream);

/* ------------------------------------------------------- theta spectral */

/*
 * Periodic functions of theta sampled at theta_i = 2 pi i / n_theta (Sec. 6.1):
 * a "row" is the n_theta vertices of one s-value of a mesh grid, AoS 4
 * doubles per vertex (x, y, px, py), theta fastest, rows back to back: element
 * (r, i) at 4 (r n_theta + i).  The operations act on each coordinate
 * separately through the discrete Fourier series over the signed
 * frequencies k in (-n_theta/2, n_theta/2]; for even n_theta the term at
 * n_theta/2 is the real mode cos(n_theta theta / 2), so real rows give real
 * results.
 */

/* theta_shift -- for each row r,
 *   out(r, i) = d^order/dtheta^order of a_r(theta_i + rho_r),
 * by an FFT, multiplication of coefficient k by (j k)^order e^{j k rho_r} and
 * the inverse FFT (the translation of Sec. 6.1, used with rho = -n omega to
 * put the points F^n(W(theta_i, s)) = W(theta_i + n omega, lambda^n s) back on
 * the theta grid; order 1 is the theta derivative of Sec. 7).
 *   rho_dev  n_rows doubles (one shift per row), or NULL to use rho for all.
 *   n_theta  a power of two, 2 ... 2048; order 0, 1 or 2.
 * in_dev may equal out_dev.  Asynchronous; MS_E_ARG for bad sizes or
 * pointers.  The first call for a given (device, n_theta) builds the
 * table of twiddle factors (synchronous allocation and copy, kept for the
 * life of the process: make that call before capturing a graph). */
int theta_shift(const double *in_dev, double *out_dev, int32_t n_theta, int64_t n_rows, const double *rho_dev,
                double rho, int32_t order, void *stream);

/* theta_spectrum -- the forward transform of each row (the FFT step of
 * Sec. 6.1 and Sec. 7): out(r, j) = (Z0(j), Z1(j)) / n_theta for the
 * frequencies j = 0..n_theta-1 in natural order, where z0 = x + i y and
 * z1 = px + i py are a row's coordinate pairs as complex sequences; stored
 * as 4 doubles per frequency (Re Z0, Im Z0, Re Z1, Im Z1), the layout of the
 * rows.  n_theta a power of two, 2 ... 2048.  Asynchronous; the first call
 * per (device, n_theta) builds the twiddle table as theta_shift does. */
int theta_spectrum(const double *in_dev, double *out_dev, int32_t n_theta, int64_t n_rows, void *stream);

/*
 * globalize_manifold -- the globalized mesh of a manifold (Sec. 6.1).  From
 * the fundamental-domain grid W(theta_i, s_k) (grid_dev: n_s rows of
 * n_theta vertices, AoS 4 doubles, s_host[k] strictly increasing), for
 * n = 1..n_max the points F^(d n)(W(theta_i, s_k)) = W(theta_i + d n omega,
 * lambda^(d n) s_k) are shifted back by -d n omega (theta_shift), giving
 * W(theta_i, lambda^(d n) s_k); d = map->n_periods = +1 for an unstable
 * manifold (the map F, multiplier lambda > 1) or -1 for a stable one (F^-1,
 * its multiplier lambda < 1).  F is the position-momentum map of pertbp_map
 * with map's mu, e and steps_per_period, applied once per layer to the
 * previous layer's points.  The rows, s = lambda^(d n) s_k, are written to
 * out_dev sorted by s (the row s = 0, the torus, once), with their s values
 * in s_out_host and their number in *n_rows_out; MS_E_CAPACITY (with
 * *n_rows_out set) when out_rows_cap is smaller.  n_theta a power of two,
 * 2 ... 2048.  Workspace: globalize_workspace_size bytes.  Synchronous (the
 * sorted order is computed on the host).
 */
int globalize_workspace_size(int32_t n_theta, int32_t n_s, int32_t n_max, size_t *bytes);
int globalize_manifold(const double *grid_dev, const double *s_host, int32_t n_theta, int32_t n_s, int32_t n_max,
                       double omega, double lambda, const map_params_t *map, double *out_dev, int64_t out_rows_cap,
                       double *s_out_host, int64_t *n_rows_out, void *ws, size_t ws_bytes, void *stream);

/* theta_interp -- trigonometric interpolation (Sec. 7): out_dev[4 q + c] is
 * the value at theta_dev[q] of the trigonometric polynomial through the
 * samples of row row_dev[q] (coordinate c).  Any n_theta >= 1.  A query with
 * a row outside [0, n_rows), a non-finite theta, or a theta so large that
 * theta n_theta / (2 pi) overflows yields NaN.  Asynchronous. */
int theta_interp(const double *rows_dev, int32_t n_theta, int64_t n_rows, const int64_t *row_dev,
                 const double *theta_dev, int64_t n_query, double *out_dev, void *stream);

/* ------------------------------------------------- Fourier-Taylor charts */

/*
 * ft_partials -- points and partial derivatives of a Fourier-Taylor
 * parameterization W(theta, s) = sum_{k=0}^{order} W_k(theta) s^k of a
 * manifold (Sec. 7), locally or globalized through the stroboscopic map:
 *   W_glob(theta, s) = F^m(W(theta - m omega, lambda^-m s)),
 *   dW_glob/dtheta = DF^m dW/dtheta,   dW_glob/ds = lambda^-m DF^m dW/ds,
 * with the partials of W taken at (theta - m omega, lambda^-m s) (the s
 * series differentiated term by term, the theta derivative by multiplying
 * the spectrum by i j, both interpolated trigonometrically at theta).
 *   spec_dev   the coefficients' spectra: theta_spectrum of the (order + 1)
 *              rows W_k(theta_i), i = 0..n_theta-1 (so (order + 1) x n_theta
 *              x 4 doubles).  Any n_theta >= 1 is accepted here.
 *   theta_dev, s_dev  n_query parameters.
 *   map        NULL or n_periods == 0: the local chart (omega, lambda
 *              unused).  Else m = map->n_periods (negative for a stable
 *              manifold, with its multiplier lambda) and F, DF are those of
 *              pertbp_map_stm with map's mu, e and steps.
 *   w_dev, dth_dev, ds_dev  n_query x 4 outputs.
 *   stm_dev    n_query x 16 doubles of workspace (DF^m per query, row-major;
 *              left there on return); required when m != 0.
 * Asynchronous.  A query with a non-finite theta or s yields NaN. */
int ft_partials(const double *spec_dev, int32_t n_theta, int32_t order, const double *theta_dev,
                const double *s_dev, int64_t n_query, double omega, double lambda, const map_params_t *map,
                double *w_dev, double *dth_dev, double *ds_dev, double *stm_dev, void *stream);

/* ------------------------------------------------------------ refinement */

/*
 * The refinement problem of Sec. 7.  A hit of the search gives approximate
 * parameters x = (th1, s1, th2, s2) of a point where the unstable and stable
 * manifold meshes meet.  With the manifolds represented near the hit by
 * patches
 *   x_u(th, s) = U.base + th U.d1 + s U.d2,   x_s(th, s) = S.base + th S.d1 + s S.d2
 * and pushed by the stroboscopic map (F^{fwd.n_periods} on the unstable side,
 * F^{bwd.n_periods} on the stable side, usually +3 and -3; the
 * globalisations of Sec. 4.3), the mismatch is
 *   f(x) = F^{fwd.n_periods}(x_u(th1, s1)) - F^{bwd.n_periods}(x_s(th2, s2)),
 * r = |f|^2, and Df = [df/dth1 df/ds1 df/dth2 df/ds2] (Sec. 7).  The
 * derivative with respect to the eccentricity e (shared by both maps, which
 * must have the same mu and e) is the fifth column.
 *
 * patch_t arrays are device arrays: one patch per hit (patch_stride = 1) or
 * one patch shared by all hits (patch_stride = 0).
 */
typedef struct {
    double base[4], d1[4], d2[4];
} patch_t;

enum {
    MS_REFINE_RESIDUAL = 0,   /* f, r */
    MS_REFINE_ADJOINT = 1,    /* f, r, grad = dr/d(th1, s1, th2, s2, e) by the discrete adjoint */
    MS_REFINE_TANGENT = 2,    /* f, r, J = df/d(th1, s1, th2, s2, e) by the variational
                                 equations, grad = 2 J^T f */
    MS_REFINE_NEWTON = 3      /* (workspace sizing of refine_newton only) */
};

/* Workspace bytes of refine_grad (mode 0-2) or refine_newton (mode 3) for K
 * hits.  Holds the stage values of one period per side (steps_per_period x 11
 * doubles of w(f), and as many of dw/de except in residual mode, computed by
 * the call itself); the adjoint also needs K x 2 x (steps / ckpt_every) x 32 B
 * of checkpoints plus a window of recomputed states and step Jacobians (at
 * most 256 MiB, at least one checkpoint segment). */
int refine_workspace_size(int64_t K, const map_params_t *fwd, const map_params_t *bwd, int32_t ckpt_every,
                          int32_t mode, size_t *bytes);

/*
 * refine_grad -- mismatch and derivatives for K parameter vectors.
 *   params_dev  K x 4 doubles (th1, s1, th2, s2).
 *   f_dev       K x 4 (required for MS_REFINE_ADJOINT, else optional);
 *   r_dev       K (optional);
 *   grad_dev    K x 5: dr/d(th1, s1, th2, s2, e) (adjoint and tangent modes);
 *   J_dev       K x 4 x 5, row-major (tangent mode, optional).
 * The adjoint runs the map forwards keeping the state every ckpt_every steps,
 * then goes backwards over windows of whole checkpoint segments: the states of
 * a window are recomputed from their checkpoints, the Jacobian of every step
 * of the window (and its derivative with respect to e) is formed in parallel,
 * and the cotangent is carried back through the transposed steps; the result
 * does not depend on ckpt_every (bit for bit).  The tangent integrates the
 * variational equations with the same method, so both give the derivative of
 * the discrete map.  ws: refine_workspace_size bytes (the call writes every
 * part it reads).  Asynchronous on `stream`: queues kernels only, allocates
 * nothing, never synchronises, and can be captured into a HIP graph whatever
 * the values of e and steps_per_period.
 */
int refine_grad(const double *params_dev, int64_t K, const patch_t *U_dev, const patch_t *S_dev,
                int32_t patch_stride, const map_params_t *fwd, const map_params_t *bwd, int32_t ckpt_every,
                int32_t mode, double *f_dev, double *r_dev, double *grad_dev, double *J_dev, void *ws,
                size_t ws_bytes, void *stream);

/*
 * refine_newton -- damped Newton iteration of Sec. 7,
 *   x <- x - alpha Df(x)^{-1} f(x),
 * per hit, from params_in_dev (K x 4) to params_out_dev (K x 4).  alpha
 * starts at alpha0 after every accepted step and is halved after every trial
 * point whose r is not below the current one (the current point is kept).
 * Df is solved by Gaussian elimination with partial pivoting (first row of
 * largest magnitude).  Per hit the iteration stops with status
 *   0 converged (|f|^2 <= tol^2), 1 max_trials trial points evaluated,
 *   2 alpha < alpha_min, 3 Df singular (exact zero pivot),
 *   4 non-finite mismatch at the start point.
 * Outputs: the final point, its f (K x 4) and r (K), status and the number of
 * trial points (K int32 each; f_dev, r_dev, status_dev, trials_dev optional).
 * Every trial evaluates f and Df at once (tangent pass); the whole iteration
 * is queued without host synchronisation (max_trials + 1 passes).
 */
typedef struct {
    int32_t max_trials;
    double tol;
    double alpha0;
    double alpha_min;
} newton_params_t;

int refine_newton(const double *params_in_dev, double *params_out_dev, int64_t K, const patch_t *U_dev,
                  const patch_t *S_dev, int32_t patch_stride, const map_params_t *fwd, const map_params_t *bwd,
                  const newton_params_t *np, double *f_dev, double *r_dev, int32_t *status_dev,
                  int32_t *trials_dev, void *ws, size_t ws_bytes, void *stream);

/*
 * ft_newton -- the same damped Newton iteration (same alpha rule, stopping
 * rules and status codes) for two globalized Fourier-Taylor charts (Sec. 7):
 *   f(x) = W_U(theta_u, s_u) - W_S(theta_s, s_s),
 *   Df = [dW_U/dtheta, dW_U/ds, -dW_S/dtheta, -dW_S/ds],
 * x = (theta_u, s_u, theta_s, s_s), each chart evaluated by ft_partials
 * with its own m, omega and lambda and the map's mu, e and steps_per_period
 * (map->n_periods is ignored).  One iteration evaluates both charts at the
 * trial points of the running problems; the stream is synchronised once per
 * iteration to stop as soon as no problem is running.  Workspace:
 * ft_newton_workspace_size(K) bytes. */
typedef struct {
    const double *spec_dev;   /* theta_spectrum of the chart's order + 1 coefficient rows */
    int32_t n_theta;
    int32_t order;
    int32_t n_periods;        /* m of the globalization: > 0 unstable, < 0 stable, 0 local */
    int32_t reserved;
    double omega;             /* rotation number of the chart's circle */
    double lambda;            /* multiplier of the chart's s direction */
} ft_chart_t;

int ft_newton_workspace_size(int64_t K, size_t *bytes);

/* continuation_predict -- initial guesses for a continuation step along a
 * line of rotation numbers (Sec. 8): for row k, x = x0 on a first step
 * (x1_dev == NULL), else
 *   x = x0 + q (x0 - x1),  q = domega_u / (omega_u0 - omega_u1),
 * or q = domega_s / (omega_s0 - omega_s1) when domega_u == 0 (q = 0 when
 * both are 0).  x0, x1, out: K x 4 (theta_u, s_u, theta_s, s_s); omega0,
 * omega1, domega: K x 2 (omega_u, omega_s).  out may equal x0.  A zero
 * denominator gives non-finite rows.  Asynchronous. */
int continuation_predict(const double *x0_dev, const double *omega0_dev, const double *domega_dev,
                         const double *x1_dev, const double *omega1_dev, int64_t K, double *out_dev, void *stream);
int ft_newton(const double *params_in_dev, double *params_out_dev, int64_t K, const ft_chart_t *U,
              const ft_chart_t *S, const map_params_t *map, const newton_params_t *np, double *f_dev,
              double *r_dev, int32_t *status_dev, int32_t *trials_dev, void *ws, size_t ws_bytes, void *stream);

/*
 * The method of layers (Sec. 5).  With lambda_u and lambda_s the multipliers
 * of the internal dynamics on the unstable and stable manifolds and
 * T x (-D, D) their fundamental domains, the half-layers are
 *   U_n^+ : s in [D lambda_u^(n-1), D lambda_u^n],   U_n^- : the same with -s,
 *   S_n^+ : s in [D / lambda_s^(n-1), D / lambda_s^n], S_n^- : the same with -s.
 * Since F maps U_n onto U_(n+1) and S_n onto S_(n-1), every heteroclinic
 * orbit meets some pair (U_n, S_n) or (U_n, S_(n-1)) with n >= 1, so a search
 * up to layer L examines the 8 half-layer pairs of each layer: U_n^a against
 * S_n^b and S_(n-1)^b, a, b in {+, -} (the paper: 14 layers, 112 pairs).
 * Host functions; no device work, no stream.
 */
typedef struct {
    int32_t u_layer, u_sign;   /* U_n^(+/-): n >= 1, sign +1 or -1 */
    int32_t s_layer, s_sign;   /* S_m^(+/-): m = n or n - 1 */
} layer_pair_t;

/*
 * layer_pairs -- the 8 * n_layers half-layer pairs for layers 1..n_layers,
 * ordered by n, then U's sign (+ first), then S_n before S_(n-1), then S's
 * sign (+ first).  *n_out = 8 * n_layers; MS_E_CAPACITY (out untouched)
 * when cap is smaller; MS_E_ARG for n_layers < 0 or a NULL pointer.
 */
int layer_pairs(int32_t n_layers, layer_pair_t *out, int32_t cap, int32_t *n_out);

/*
 * half_layer_bounds -- [lo, hi] of |s| for half-layer `layer` (unstable:
 * D lambda^(layer-1) and D lambda^layer; stable: D / lambda^(layer-1) and
 * D / lambda^layer), ordered lo < hi.  MS_E_ARG unless D > 0, lambda > 0,
 * lambda != 1 and both bounds finite.
 */
int half_layer_bounds(double D, double lambda, int32_t stable, int32_t layer, double *lo, double *hi);

/*
 * half_layer_columns -- the columns [*k0, *k1] of a mesh with s samples
 * s_host[0..n_s_v) (strictly increasing) that form the half-layer of sign
 * `sign` (+1 or -1): the columns from the sample equal to one boundary to
 * the sample equal to the other (equality within a relative 1e-12; the
 * manifold's globalization produces the boundaries as samples, Sec. 6.2).
 * A mesh over columns [k0, k1] of an AoS vertex grid starts at vertex
 * k0 * n_theta_v, with n_s_v = k1 - k0 + 1 (no copy).  MS_E_ARG when a
 * boundary is not a sample or the samples do not increase.
 */
int half_layer_columns(const double *s_host, int32_t n_s_v, double D, double lambda, int32_t stable, int32_t layer,
                       int32_t sign, int32_t *k0, int32_t *k1);

#ifdef __cplusplus
}
#endif

#endif /* MSEARCH_H */
