/*
 * tc.h - C ABI of the MI355X triangle-counting library (libtc.so).
 *
 * Method: exact triangle counting as matching of a triangle query Q against an
 * undirected data graph G (Wang & Owens, "Fast BFS-Based Triangle Counting on
 * GPUs", Sec. II-A problem definition, Def. 1-2; Sec. III-A, Alg. 1).
 *
 *   tc_build_csr         input cleaning: pairs -> symmetric, deduplicated,
 *                        self-loop-free CSR with ascending rows (Sec. II-A: the
 *                        graphs are undirected and unlabeled; Sec. III-B: CSR).
 *   tc_orient            unique mapping order (Alg. 1 "Generate_UMO", Sec. III-A
 *                        NEC ordering): keep each undirected edge once, from the
 *                        lower-ranked to the higher-ranked endpoint.
 *   tc_count             all-source advance over the oriented graph (Alg. 1
 *                        "Advance", Sec. III-B) enumerating wedges u->v->w, the
 *                        filter that keeps wedges closed by the stored non-tree
 *                        edge (u,w) (Alg. 1 "Store_none_tree_connection"), and
 *                        the reduction to |M|/|Q| (Alg. 1 return value).
 *   tc_count_per_vertex  the same, plus t(v) = number of triangles containing v.
 *   tc_count_batched     per-graph counts of many graphs packed as one disjoint
 *                        union, in one launch sequence.
 *   tc_source_work       the wedge work w(u) of every source and its prefix
 *                        (equal-work ranges of sources).
 *   tc_list_triangles    the match set M itself: every triangle as one row
 *                        (u, v, w) of the oriented graph.
 *   tc_edge_support      for every edge, the number of matches (triangles)
 *                        that use it.
 *   tc_count_k4          the 4-clique query (the next clique after the triangle).
 *   tc_segmented_intersect  the segmented-intersection operator: a merge of
 *                        N+(u) and N+(v) for every oriented edge (count and
 *                        per-edge support).
 *   tc_count_diamonds    the diamond query (two triangles sharing an edge), a
 *                        query with two neighbourhood-equivalence classes.
 *   tc_ne_filter,        the paper's own pipeline, kept for comparison: the NE
 *   tc_count_bfs         candidate filter and the two-iteration advance with
 *                        its partial and complete matches written out.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - All array arguments are DEVICE pointers on the current HIP device, owned
 *    by the caller.  The library never allocates device memory: each entry
 *    point that needs scratch memory takes a caller-owned workspace.
 *  - Workspace protocol: call with ws == NULL to receive the required size in
 *    *ws_bytes (TC_OK, nothing is launched).  Call again with ws pointing to at
 *    least that many bytes (256-byte aligned) and *ws_bytes set to its size;
 *    a smaller *ws_bytes returns TC_ERR_WORKSPACE.
 *  - stream is a hipStream_t passed as void* (NULL = the default stream).  Work
 *    is enqueued asynchronously; no entry point synchronises the host.
 *  - Errors that can be seen from the host (bad sizes, null pointers, short
 *    workspace) are returned immediately and nothing is launched.  Errors that
 *    only the device can see (an out-of-range vertex id, an output capacity too
 *    small) are reported through the device-side size output of the call
 *    (nnz_out / m_out), which then holds -status; the CSR written in that case
 *    is the empty graph (all offsets 0), so later calls stay memory-safe.
 *  - Vertex ids are 0-based int32 in [0, n), n < 2^31.  Row offsets are int32
 *    or int64 (offset_bytes = 4 or 8); column indices are int32.
 *  - A CSR passed to tc_orient / tc_count must be well formed: row_ptr[0] = 0,
 *    non-decreasing, every column id in [0, n), rows strictly ascending.  The
 *    outputs of tc_build_csr and tc_orient are.  Malformed input is undefined
 *    behaviour (it may read out of bounds).
 *  - Counts are exact unsigned 64-bit integers.  Distinct streams may run calls
 *    concurrently as long as they use distinct workspaces and outputs.
 *  - tc_last_error() returns a thread-local message for the last non-OK status.
 */
#ifndef TC_H_
#define TC_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t tc_status;

#define TC_OK 0
#define TC_ERR_INVALID_ARG 1      /* bad size, null pointer, unknown option */
#define TC_ERR_ID_OUT_OF_RANGE 2  /* an input pair holds an id outside [0, n) */
#define TC_ERR_CAPACITY 3         /* an output array is too small */
#define TC_ERR_WORKSPACE 4        /* *ws_bytes is below the required size */
#define TC_ERR_HIP 5              /* a HIP runtime call or kernel launch failed */
#define TC_ERR_UNSUPPORTED 6      /* n >= 2^31, or int32 offsets too narrow */

#define TC_ORDER_DEGREE 0 /* rank(v) = (deg(v), v) lexicographic: the default */
#define TC_ORDER_ID 1     /* rank(v) = v: the paper's "destination id larger than source id" */

#define TC_PROBE_AUTO 0   /* LDS cuckoo table of N+(u), with stash and sorted fallbacks */
#define TC_PROBE_SORTED 1 /* binary search over the sorted N+(u) staged in LDS */

/*
 * Optional launch parameters of the count entry points (NULL = defaults).  They
 * change only the speed, never the counts.
 */
typedef struct tc_tune {
  int32_t small_max;     /* sources with 2 <= d+(u) <= small_max are handled by one wave,
                            larger ones by a workgroup; 0 = default (80), at most 96 */
  int32_t probe;         /* TC_PROBE_AUTO or TC_PROBE_SORTED */
  int32_t blocks_per_cu; /* persistent grid = blocks_per_cu x compute units, capped at the
                            occupancy limit; 0 = occupancy limit */
  int32_t max_kicks;     /* cuckoo placements per key before it goes to the stash
                            (the stash holds 32 keys; past it the slice is binary
                            searched instead): 0 = default (48), 1 to 1024 = that many,
                            -1 = none, so every key takes the stash or the sorted
                            fallback (exercises those probe modes) */
  int32_t split_log2;    /* equal-work quanta: a workgroup-mode source u whose work
                            w(u) = sum of d+(v) over v in N+(u) (its wedges; x8 when
                            N+(u) is too long for LDS and is searched in memory)
                            exceeds 2^split_log2 is cut into ceil(w(u) / 2^split_log2)
                            parts (at most 1024) that any workgroup may take;
                            0 = default (2^21), 1 to 40 = that quantum, -1 = never */
} tc_tune;

/* Read-only view of a CSR graph in device memory. */
typedef struct tc_csr {
  int64_t n;            /* number of vertices; ids are in [0, n) */
  int32_t offset_bytes; /* 4: row_ptr is int32_t[n+1]; 8: row_ptr is int64_t[n+1] */
  const void* row_ptr;  /* device; row_ptr[n] is the number of stored entries */
  const int32_t* col;   /* device; row_ptr[n] column ids, each row ascending */
} tc_csr;

/*
 * tc_build_csr - clean an undirected edge list into a symmetric CSR.
 *
 * Follows the problem statement (Sec. II-A): G is undirected, so (u,v) and
 * (v,u) are one edge; it has no labels or weights.  Self-loops cannot be part
 * of a triangle match under an injective mapping (Def. 2) and are dropped.
 *
 *   n            vertices, 0 <= n < 2^31
 *   num_pairs    number of input pairs (>= 0)
 *   src, dst     device int32[num_pairs]; pair i is {src[i], dst[i]}.
 *                Duplicates, both directions and self-loops are allowed.
 *   offset_bytes 4 or 8: width of row_ptr.  4 requires 2*num_pairs < 2^31.
 *   row_ptr      device, (n+1) offsets of width offset_bytes (written)
 *   col          device int32[col_capacity] (written): for every vertex u its
 *                distinct neighbours v != u in ascending order
 *   col_capacity entries available in col; the result needs 2m entries
 *                (m = distinct undirected non-loop edges <= num_pairs)
 *   nnz_out      device int64[1] (written): 2m, or -TC_ERR_ID_OUT_OF_RANGE if
 *                an id lies outside [0, n), or -TC_ERR_CAPACITY if 2m >
 *                col_capacity; on either error row_ptr is all zeros.
 *   ws, ws_bytes workspace (see protocol above); O(num_pairs + n) bytes.
 */
tc_status tc_build_csr(int64_t n, int64_t num_pairs, const int32_t* src, const int32_t* dst,
                       int32_t offset_bytes, void* row_ptr, int32_t* col, int64_t col_capacity,
                       int64_t* nnz_out, void* ws, size_t* ws_bytes, void* stream);

/*
 * tc_orient - keep each undirected edge once, oriented by a strict total order.
 *
 * The paper's unique mapping order (Alg. 1 "Generate_UMO"; Sec. III-A, NEC
 * ordering u1 < u2 < u3) visits equivalent query nodes in increasing order so
 * each triangle is matched once.  Any strict total order has that property;
 * TC_ORDER_DEGREE ranks by (degree, id), which bounds every out-degree by
 * O(sqrt(m)); TC_ORDER_ID is the paper's id order.
 *
 *   sym          symmetric CSR (as written by tc_build_csr)
 *   order        TC_ORDER_DEGREE or TC_ORDER_ID
 *   dag_row_ptr  device, (n+1) offsets of width sym->offset_bytes (written)
 *   dag_col      device int32[dag_col_capacity] (written): for each u the v with
 *                rank(u) < rank(v), ascending by id (a subsequence of u's row)
 *   dag_col_capacity  entries available in dag_col; m = row_ptr[n]/2 are needed
 *                (at most 2^40)
 *   m_out        device int64[1] (written): m, or -TC_ERR_CAPACITY when the DAG
 *                needs more than dag_col_capacity entries or row_ptr[n] exceeds
 *                2 * dag_col_capacity (then dag_row_ptr is all zeros)
 *   ws, ws_bytes workspace; depends on n and dag_col_capacity: about
 *                4 n + dag_col_capacity / 4 bytes (per-tile state for up to
 *                2 * dag_col_capacity symmetric entries).
 */
tc_status tc_orient(const tc_csr* sym, int32_t order, void* dag_row_ptr, int32_t* dag_col,
                    int64_t dag_col_capacity, int64_t* m_out, void* ws, size_t* ws_bytes,
                    void* stream);

/*
 * tc_count - number of triangles T of the oriented graph (Alg. 1 return value
 * |M|/|Q|: each triangle is matched exactly once under the orientation).
 *
 * For every source u (all-source traversal, Sec. III), every v in N+(u) and
 * every w in N+(v), the wedge u->v->w is a match iff w is in N+(u).  Sources
 * with out-degree < 2 and middles with out-degree 0 cannot complete a match
 * and are pruned (the 1- and 2-look-ahead of Sec. III-C).
 *
 *   dag      oriented CSR (as written by tc_orient; any DAG works)
 *   total    device uint64[1] (written, not accumulated)
 *   tune     launch parameters or NULL
 *   ws, ws_bytes  workspace; O(n) bytes.
 */
tc_status tc_count(const tc_csr* dag, uint64_t* total, const tc_tune* tune, void* ws,
                   size_t* ws_bytes, void* stream);

/*
 * tc_count_per_vertex - per-vertex triangle counts t(v) and the total.
 *
 * t(v) is the number of triangles that contain v; sum_v t(v) = 3T.  The paper
 * outputs the listing M of matched node sequences (Sec. II-A, Alg. 1); t(v) is
 * the number of times v appears in M.
 *
 *   dag         oriented CSR
 *   per_vertex  device uint64[dag->n] (written, not accumulated)
 *   total       device uint64[1] or NULL (written when non-NULL)
 *   tune        launch parameters or NULL
 *   ws, ws_bytes  workspace; O(n) bytes.
 */
tc_status tc_count_per_vertex(const tc_csr* dag, uint64_t* per_vertex, uint64_t* total,
                              const tc_tune* tune, void* ws, size_t* ws_bytes, void* stream);

/*
 * tc_count_per_vertex_noalloc - tc_count_per_vertex for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc): the same kernels and results, with the
 * scratch (class counters, the split table, the binned source list, a scratch
 * total) in one static device array of the library instead of a caller
 * workspace.  The caller still passes the DAG and the outputs.
 *
 *   dag         oriented CSR with n <= 2^22 vertices (the array holds 16.1 MiB
 *               per device); a larger n returns TC_ERR_CAPACITY, nothing launched
 *   per_vertex  device uint64[dag->n] (written, not accumulated)
 *   total       device uint64[1] or NULL (written when non-NULL)
 *   tune        launch parameters or NULL
 * Each device holds its own copy of the array (looked up on the first call on
 * that device) until the process ends.  Every call on one device shares it:
 * calls that overlap on one device, on any streams, race and give wrong counts;
 * serialise them.  Nothing is allocated and no allocating library routine is
 * called.
 */
tc_status tc_count_per_vertex_noalloc(const tc_csr* dag, uint64_t* per_vertex, uint64_t* total,
                                      const tc_tune* tune, void* stream);

/*
 * tc_count_batched - per-graph triangle counts of many independent graphs in
 * one launch.
 *
 * The batch is the disjoint union of its graphs: graph g owns the vertex ids
 * [vtx_off[g], vtx_off[g+1]) of one CSR (global ids, as a concatenation of the
 * graphs with shifted ids gives).  Every triangle lies inside one graph, so
 * counting the union with tc_count's method and adding each source's matches to
 * the total of the source's graph gives every graph's |M|/|Q| (Alg. 1 return
 * value) at once.  The union is oriented with tc_orient like any graph.
 *
 *   dag         oriented CSR of the union (n = vtx_off[num_graphs])
 *   num_graphs  number of graphs G >= 0
 *   vtx_off     device int64[G+1], vtx_off[0] = 0, non-decreasing; edges must not
 *               cross graph boundaries.  Offsets outside [0, n] are clamped;
 *               vertices outside every range add to no graph total.
 *   totals      device uint64[G] (written): triangles of each graph
 *   per_vertex  device uint64[n] or NULL: t(v) for every vertex of the union
 *   total       device uint64[1] or NULL: triangles of the whole batch
 *   tune        launch parameters or NULL
 *   ws, ws_bytes  workspace; O(n) bytes.
 * The call enqueues a fixed sequence of kernels and allocates nothing, so it can
 * be captured in a HIP graph and replayed while its buffers stay in place.
 */
tc_status tc_count_batched(const tc_csr* dag, int64_t num_graphs, const int64_t* vtx_off,
                           uint64_t* totals, uint64_t* per_vertex, uint64_t* total,
                           const tc_tune* tune, void* ws, size_t* ws_bytes, void* stream);

/*
 * tc_pack_pairs - the raw pairs of several graphs, concatenated, moved in place
 * to the vertex ids of their disjoint union, the input tc_build_csr takes to
 * build a batch for tc_count_batched (every triangle lies inside one graph, so
 * the union's matches are the graphs' matches, Alg. 1 run on each graph).
 *
 *   num_graphs  G >= 0
 *   pair_off    device int64[G+1]: graph g's pairs are [pair_off[g], pair_off[g+1])
 *               of src and dst, with local ids in [0, n_g)
 *   vtx_off     device int64[G+1]: graph g owns the union ids [vtx_off[g],
 *               vtx_off[g+1]), so n_g = vtx_off[g+1] - vtx_off[g]
 *   src, dst    device int32[pair_off[G]] (read and written): each local id x
 *               becomes vtx_off[g] + x, or -1 when x lies outside [0, n_g), which
 *               tc_build_csr then reports as TC_ERR_ID_OUT_OF_RANGE
 * Offsets must be non-decreasing; nothing is allocated and no workspace is used.
 */
tc_status tc_pack_pairs(int64_t num_graphs, const int64_t* pair_off, const int64_t* vtx_off,
                        int32_t* src, int32_t* dst, void* stream);

/*
 * tc_source_work - the wedge work of every source and its exclusive prefix.
 * In the all-source advance (Alg. 1 "Advance", Sec. III-B) source u enumerates
 * one wedge u -> v -> w per v in N+(u) and w in N+(v): w(u) = sum of d+(v) over
 * N+(u), and 0 when d+(u) < 2 (the 2-look-ahead of Sec. III-C).  The prefix
 * cuts the sources into contiguous ranges of equal work (how the count would be
 * sharded) and its last entry is the total W the count enumerates.
 *
 *   dag      oriented CSR
 *   work     device int64[n] or NULL: w(u) (written)
 *   prefix   device int64[n+1] (written): prefix[u] = sum of w over ids < u
 *   ws, ws_bytes  workspace; about 8 n bytes.
 */
tc_status tc_source_work(const tc_csr* dag, int64_t* work, int64_t* prefix, void* ws,
                         size_t* ws_bytes, void* stream);

/*
 * tc_list_triangles - the matches themselves.  Sec. II-A defines the output of
 * subgraph matching as every match; Alg. 1 collects the complete matches in M,
 * and under the unique mapping order each triangle is one match.  Each is
 * written as the row (u, v, w) = (u1, u2, u3) of the query path: v and w in
 * N+(u), w in N+(v).
 *
 *   dag        oriented CSR (as written by tc_orient)
 *   triples    device int32[3 * capacity] (written): rows (u, v, w).  The rows
 *              of one u are contiguous and sources come in increasing id order;
 *              within one u the order is unspecified (the set is unique).
 *   capacity   rows available in triples (at most 2^40)
 *   count_out  device int64[1] (written): T, or -TC_ERR_CAPACITY when T >
 *              capacity (then no row is written)
 *   tune       launch parameters or NULL (as for tc_count)
 *   ws, ws_bytes  workspace; O(n) bytes.
 * Two passes: the per-source counts (the tc_count enumeration), their
 * exclusive scan into row offsets, and the same enumeration writing rows.
 */
tc_status tc_list_triangles(const tc_csr* dag, int32_t* triples, int64_t capacity,
                            int64_t* count_out, const tc_tune* tune, void* ws, size_t* ws_bytes,
                            void* stream);

/*
 * tc_edge_support - per-edge support: for every oriented edge e, the number of
 * triangles (matches of the triangle query, Sec. II-A and Alg. 1) that contain
 * it.  A match u -> v -> w closed by (u, w) uses the three edges (u, v), (v, w)
 * and (u, w); each gets one.  Summed over the edges this is 3T.
 *
 *   dag       oriented CSR (as written by tc_orient)
 *   support   device uint32[capacity] (written): support[e] for e in [0, m),
 *             aligned with dag->col (entry e is the edge (u, dag->col[e]))
 *   capacity  entries available in support; m = dag row_ptr[n] are needed
 *   m_out     device int64[1] (written): m, or -TC_ERR_CAPACITY when m >
 *             capacity (then support is not written)
 *   total     device uint64[1] (written) or NULL: T
 *   tune      launch parameters or NULL (as for tc_count)
 *   ws, ws_bytes  workspace; O(n) bytes.
 * One launch of the count enumeration: each hit adds one to (v, w) with a
 * global atomic; the hits of each (u, v) list and of each slot w of the source's
 * LDS table are added once per source.
 */
tc_status tc_edge_support(const tc_csr* dag, uint32_t* support, int64_t capacity, int64_t* m_out,
                          uint64_t* total, const tc_tune* tune, void* ws, size_t* ws_bytes,
                          void* stream);

/*
 * tc_segmented_intersect - the segmented-intersection operator (Sec. II-B
 * lists it with advance, filter and compute) applied to the triangle query:
 * for every oriented edge (u, v) the sorted lists N+(u) and N+(v) are
 * intersected by a merge, and every common out-neighbour w closes the match
 * u -> v -> w (Alg. 1's non-tree edge (u, w) exists and so does (v, w)).  Under
 * the unique mapping order each triangle is found once, at its lowest edge, so
 * the number of common out-neighbours summed over the edges is |M|/|Q|.  The
 * edge-centric alternative to tc_count's wedge probe; same results.
 *
 *   dag           oriented CSR (as written by tc_orient, either order); rows
 *                 must be ascending
 *   edge_capacity upper bound on m = dag row_ptr[n] (e.g. the DAG column
 *                 capacity given to tc_orient); sizes the workspace
 *   total         device uint64[1] (written): T, or 0 on a capacity error
 *   support       device uint32[edge_capacity] or NULL: when non-NULL, entry e
 *                 (aligned with dag->col) receives the triangles on edge
 *                 (u, dag->col[e]), as tc_edge_support writes them
 *   m_out         device int64[1] (written): m, or -TC_ERR_CAPACITY when m >
 *                 edge_capacity (then nothing else is computed)
 *   ws, ws_bytes  workspace; 16 bytes per edge of capacity plus scan partials.
 * Load balance: the merge lengths d+(u) + d+(v) of all edges (0 where the
 * look-ahead of Sec. III-C rules the edge out) are scanned into one merge
 * space, cut into equal chunks of merge steps.
 */
tc_status tc_segmented_intersect(const tc_csr* dag, int64_t edge_capacity, uint64_t* total,
                                 uint32_t* support, int64_t* m_out, void* ws, size_t* ws_bytes,
                                 void* stream);

/*
 * tc_count_diamonds - number of diamonds: matches of the query made of two
 * triangles {a, b, c} and {b, c, d} sharing the edge {b, c}, counted as
 * subgraphs (a and d may be adjacent).  The query has two neighbourhood-
 * equivalence classes (Def. 3): {b, c} (adjacent to every other node) and
 * {a, d} (adjacent to b and c only).  The unique mapping order fixes one order
 * in each class (Alg. 1 "Generate_UMO"): {b, c} is matched as an oriented edge,
 * and the candidates for a and d are the common neighbours of b and c, of
 * which every pair a < d is one match.  So the count is the sum over the edges
 * of C(s, 2), s = the edge's support (triangles on it); an edge with s < 2
 * adds nothing (the look-ahead of Sec. III-C).
 *
 *   dag           oriented CSR (as written by tc_orient, either order)
 *   edge_capacity upper bound on m = dag row_ptr[n]; sizes the workspace
 *   total         device uint64[1] (written): the number of diamonds
 *   m_out         device int64[1] (written): m, or -TC_ERR_CAPACITY when m >
 *                 edge_capacity (then total is 0)
 *   tune          launch parameters of the support enumeration, or NULL
 *   ws, ws_bytes  workspace; O(n) bytes plus 4 bytes per edge of capacity.
 */
tc_status tc_count_diamonds(const tc_csr* dag, int64_t edge_capacity, uint64_t* total,
                            int64_t* m_out, const tc_tune* tune, void* ws, size_t* ws_bytes,
                            void* stream);

/*
 * tc_count_labelled - number of matches of a labelled triangle query: the
 * triangles {x, y, z} of the data graph whose vertex labels, as a multiset,
 * equal the query labels {a, b, c} (a match maps every query node onto a vertex
 * of the same label, Sec. I; queries with node labels are the extension that
 * Sec. II-A names).  Each such triangle is counted once, as tc_count counts
 * the unlabelled ones.
 * Alg. 1's candidate filtering (Filter+Compute) with labels: a DAG edge is
 * kept when its two labels form one of the query's edge label pairs (a
 * sub-multiset of {a, b, c}); the kept edges, compacted in row order, form a
 * DAG on the same vertices, which tc_count then counts.  For three equal or
 * three distinct query labels that count is the answer; for {a, a, b} the
 * count of {a, a, a} (also closed by kept edges only) is subtracted.
 *
 *   dag           oriented CSR (as written by tc_orient, either order)
 *   edge_capacity upper bound on m = dag row_ptr[n] (e.g. the DAG column
 *                 capacity given to tc_orient); sizes the workspace; at most
 *                 INT32_MAX with 4-byte offsets
 *   labels        device int32[n]: the label of every vertex (any values)
 *   a, b, c       the query labels, in any order
 *   total         device uint64[1] (written): the number of matches, 0 on a
 *                 capacity error
 *   kept_out      device int64[1] or NULL (written): the DAG edges whose labels
 *                 fit the query, or -TC_ERR_CAPACITY when m > edge_capacity
 *                 (then nothing is counted)
 *   tune          launch parameters of the count, or NULL (as for tc_count)
 *   ws, ws_bytes  workspace: the filtered DAG (offsets and 4 bytes per edge of
 *                 capacity), 1 byte per edge of capacity for the filter flags,
 *                 24 bytes per vertex, and tc_count's workspace.
 */
tc_status tc_count_labelled(const tc_csr* dag, int64_t edge_capacity, const int32_t* labels,
                            int32_t a, int32_t b, int32_t c, uint64_t* total, int64_t* kept_out,
                            const tc_tune* tune, void* ws, size_t* ws_bytes, void* stream);

/*
 * tc_edge_directions - the arc directions of a directed data graph on the DAG
 * of its underlying undirected graph (Sec. II-A: the method extends to directed
 * graphs; tc_build_csr and tc_orient keep the undirected edges, this records
 * which way each one points).
 *
 *   dag           oriented CSR built from the same pairs (tc_build_csr of src,
 *                 dst, then tc_orient)
 *   edge_capacity upper bound on m = dag row_ptr[n]
 *   num_pairs     arcs src[i] -> dst[i], device int32[num_pairs] each;
 *                 duplicates allowed, self-loops ignored
 *   dir           device uint8[edge_capacity rounded up to a multiple of 4],
 *                 4-byte aligned (written): dir[e], aligned with dag->col, has
 *                 bit 0 set when the data graph has the arc from e's row vertex
 *                 to dag->col[e], bit 1 when it has the reverse arc
 *   m_out         device int64[1] (written): m, or negative: -TC_ERR_CAPACITY
 *                 when m > edge_capacity (nothing else written),
 *                 -TC_ERR_ID_OUT_OF_RANGE for an id outside [0, n), or
 *                 -TC_ERR_INVALID_ARG for an arc whose pair is not a DAG edge
 * One thread per arc finds the edge by binary search of the two rows.  No
 * workspace.
 */
tc_status tc_edge_directions(const tc_csr* dag, int64_t edge_capacity, int64_t num_pairs,
                             const int32_t* src, const int32_t* dst, uint8_t* dir,
                             int64_t* m_out, void* stream);

/*
 * tc_count_directed - matches of a directed triangle query: a digraph on the
 * query nodes 0, 1, 2 with every pair joined by one arc or by both (the seven
 * such digraphs up to isomorphism include the 3-cycle and the transitive
 * triangle).  A match maps the query nodes one-to-one onto a triangle of the
 * underlying graph so that every query arc lands on an arc of the same
 * direction (induced = 0), or so that the arcs between every two matched
 * vertices are exactly the images of the query's (induced = 1); matches are
 * counted as subgraphs (maps divided by the query's automorphisms), as the
 * undirected count divides |M| by |Q| (Alg. 1).
 * The enumeration is tc_count's (Alg. 1's advance and non-tree-edge check,
 * each triangle found once as u -> v -> w): every closed wedge adds the
 * query's matches on its triangle, looked up in a 64-entry table (built on the
 * host from the query) by the direction codes of (u, v), (u, w) and (v, w).
 * The code of (u, w) is kept beside w in the LDS table of N+(u).
 *
 *   dag           oriented CSR (as written by tc_orient, either order)
 *   dir           device uint8[m] as tc_edge_directions writes it for this DAG
 *   p01, p02, p12 the query's node pairs 0-1, 0-2, 1-2, each 1 (lower -> higher),
 *                 2 (higher -> lower) or 3 (both)
 *   induced       0 or 1
 *   total         device uint64[1] (written): the number of matches
 *   tune          launch parameters or NULL (as for tc_count)
 *   ws, ws_bytes  workspace; as tc_count's.
 */
tc_status tc_count_directed(const tc_csr* dag, const uint8_t* dir, int32_t p01, int32_t p02,
                            int32_t p12, int32_t induced, uint64_t* total, const tc_tune* tune,
                            void* ws, size_t* ws_bytes, void* stream);

/*
 * tc_edge_labels - the labels of an edge-labelled data graph on the DAG of its
 * underlying undirected graph (Sec. II-A: matching with edge label
 * information), one byte per DAG edge.
 *
 *   dag           oriented CSR built from the same pairs
 *   edge_capacity upper bound on m = dag row_ptr[n]
 *   num_pairs     pairs {src[i], dst[i]} with label labels[i] (device int32,
 *                 int32, uint8 [num_pairs]); labels in 0..3; a pair given
 *                 several times (either direction) gives its edge the largest
 *                 of its labels; self-loops are ignored
 *   edge_labels   device uint8[edge_capacity rounded up to a multiple of 4],
 *                 4-byte aligned (written): the label of each DAG edge, aligned
 *                 with dag->col
 *   m_out         device int64[1] (written): m, or negative: -TC_ERR_CAPACITY
 *                 when m > edge_capacity, -TC_ERR_ID_OUT_OF_RANGE for an id
 *                 outside [0, n), -TC_ERR_INVALID_ARG for a label above 3 or a
 *                 pair that is not a DAG edge
 * No workspace.
 */
tc_status tc_edge_labels(const tc_csr* dag, int64_t edge_capacity, int64_t num_pairs,
                         const int32_t* src, const int32_t* dst, const uint8_t* labels,
                         uint8_t* edge_labels, int64_t* m_out, void* stream);

/*
 * tc_count_edge_labelled - matches of a triangle query with edge labels: the
 * query's edges 0-1, 0-2, 1-2 carry labels q01, q02, q12 (each 0..3, in any
 * order: the nodes' permutations permute a triangle's edges); a match maps the
 * query nodes one-to-one onto a triangle so that every query edge lands on a
 * data edge of the same label, counted as subgraphs (maps divided by the
 * query's label-preserving automorphisms): each triangle whose three edge
 * labels form the query's multiset counts once.
 * Alg. 1's candidate filtering with edge labels: the DAG edges whose label is
 * one of the query's are compacted (with their labels) into a DAG on the same
 * vertices; then the count kernel's coded launch (as tc_count_directed's, the
 * labels as the per-edge codes) adds, per closed wedge, the entry of a table
 * built on the host from the query for the labels of (u, v), (u, w), (v, w).
 *
 *   dag           oriented CSR (as written by tc_orient, either order)
 *   edge_capacity upper bound on m = dag row_ptr[n]; sizes the workspace; at
 *                 most INT32_MAX with 4-byte offsets
 *   edge_labels   device uint8[m] as tc_edge_labels writes it for this DAG
 *   total         device uint64[1] (written): the number of matches, 0 on a
 *                 capacity error
 *   kept_out      device int64[1] or NULL (written): the DAG edges whose label
 *                 is in the query, or -TC_ERR_CAPACITY when m > edge_capacity
 *   tune          launch parameters of the count, or NULL (as for tc_count)
 *   ws, ws_bytes  workspace: the filtered DAG and its labels (offsets and 6
 *                 bytes per edge of capacity), 24 bytes per vertex, and
 *                 tc_count's workspace.
 */
tc_status tc_count_edge_labelled(const tc_csr* dag, int64_t edge_capacity,
                                 const uint8_t* edge_labels, int32_t q01, int32_t q02,
                                 int32_t q12, uint64_t* total, int64_t* kept_out,
                                 const tc_tune* tune, void* ws, size_t* ws_bytes, void* stream);

/*
 * tc_ne_filter - the candidate filter of Alg. 1: a data vertex can stand for a
 * query node only if its neighbourhood encoding (NE = degree, Sec. III-C)
 * covers the node's; every node of the triangle query has degree 2.  Iterated:
 * a vertex is dropped while it keeps fewer than min_degree candidate
 * neighbours, which converges to the min_degree-core.  Any number of rounds
 * keeps every triangle (its vertices always keep two candidate neighbours).
 *
 *   sym          symmetric CSR (as written by tc_build_csr)
 *   min_degree   the query node degree (2 for the triangle), >= 0
 *   max_rounds   rounds launched, in [0, 4096]; a round after one that removed
 *                nothing does no work
 *   keep         device uint8[n] (written): 1 for the remaining candidates
 *   stats_out    device int64[3] (written): candidates kept, rounds that removed
 *                something, 1 if the last round removed nothing (converged)
 *   ws, ws_bytes workspace; 4 (max_rounds + 1) bytes.
 */
tc_status tc_ne_filter(const tc_csr* sym, int32_t min_degree, int32_t max_rounds, uint8_t* keep,
                       int64_t* stats_out, void* ws, size_t* ws_bytes, void* stream);

/*
 * tc_count_bfs - Alg. 1's verification as two BFS iterations with their
 * results written out (the comparison point for the fused tc_count).
 * Iteration 1 advances every candidate source u to v in N+(u) and compacts the
 * partial matches (u, v) that pass the 2-/1-look-ahead of Sec. III-C (d+(u) >=
 * 2, d+(v) >= 1) and the candidate mask; iteration 2 advances each to every w
 * in N+(v) that is a candidate and keeps it when the non-tree query edge (u, w)
 * exists ("Store_none_tree_connection"), i.e. w is in N+(u).
 *
 *   dag                oriented CSR (as written by tc_orient, either order)
 *   keep               device uint8[n] or NULL: candidate vertices
 *   frontier_capacity  partial matches the workspace holds; m = dag row_ptr[n]
 *                      always suffices
 *   matches            device int32[3 * match_capacity] or NULL: complete
 *                      matches as rows (u, v, w), in no particular order
 *   match_capacity     rows available in matches
 *   stats_out          device int64[4] (written): partial matches after
 *                      iteration 1, candidate wedges of iteration 2, complete
 *                      matches, status: 0, or TC_ERR_CAPACITY when the frontier
 *                      did not fit (then only the first entry is valid) or the
 *                      matches did not fit the rows (then the rows are partial)
 *   total              device uint64[1] or NULL (written): complete matches
 *   ws, ws_bytes       workspace; about 16 B per frontier_capacity entry.
 */
tc_status tc_count_bfs(const tc_csr* dag, const uint8_t* keep, int64_t frontier_capacity,
                       int32_t* matches, int64_t match_capacity, int64_t* stats_out,
                       uint64_t* total, void* ws, size_t* ws_bytes, void* stream);

/*
 * tc_count_k4 - number of 4-cliques: the matches of the 4-clique query (Sec.
 * II-A's subgraph matching with Q = K4; one node per BFS iteration of Alg. 1
 * under the unique mapping order, so each 4-clique is found once, as
 * u -> v -> w -> x with all six edges present).  Look-ahead (Sec. III-C):
 * d+(u) >= 3, d+(v) >= 2, d+(w) >= 1.
 *
 *   dag      oriented CSR (as written by tc_orient, either order)
 *   total    device uint64[1] (written)
 *   ws, ws_bytes  workspace: about 5 n + 33 KB bytes (a byte per vertex marking
 *            the sources whose middles are split over several workgroups, and
 *            8-byte entries listing their parts, n / 2 + 4096 of them).
 */
tc_status tc_count_k4(const tc_csr* dag, uint64_t* total, void* ws, size_t* ws_bytes,
                      void* stream);

/* Human-readable name of a status code (static storage). */
const char* tc_status_string(tc_status status);

/* Message for the last non-OK status returned on this thread ("" if none). */
const char* tc_last_error(void);

/* Library version as MAJOR*10000 + MINOR*100 + PATCH. */
int32_t tc_version(void);

#ifdef __cplusplus
}
#endif

#endif /* TC_H_ */
