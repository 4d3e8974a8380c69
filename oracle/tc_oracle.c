/*
 * tc_oracle.c - CPU oracle for exact triangle counting.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the library's product path may call,
 * link or load this file; only the tests, the smoke check and the CPU-baseline
 * leg of the benchmark use it.  It shares no code with the GPU path.
 *
 * It is deliberately plain and slow: every function follows a definition from
 * Wang & Owens, "Fast BFS-Based Triangle Counting on GPUs", written out.
 *
 *  - oracle_clean: Sec. II-A (problem definition) says both graphs are
 *    undirected with no labels or weights, so (u,v) and (v,u) are one edge.
 *    Def. 2 maps query nodes injectively, so a self-loop can never be part of a
 *    triangle match and is dropped.  The result is E = {{u,v} : u != v} as a
 *    symmetric CSR with ascending rows (Sec. III-B stores graphs as CSR).
 *  - oracle_orient: the unique mapping order of Alg. 1 ("Generate_UMO") and of
 *    Sec. III-A (the triangle is one neighbourhood-equivalence class; visit its
 *    nodes in increasing order u1 < u2 < u3).  Each undirected edge is kept
 *    once, from the lower to the higher rank, for a strict total order "rank".
 *  - oracle_count: the wedge u -> v -> w of the oriented graph is a match iff
 *    the non-tree query edge (u1, u3) is present (Alg. 1
 *    "Store_none_tree_connection"), i.e. w is also an out-neighbour of u.  With
 *    rank(u) < rank(v) < rank(w) forced by the orientation, every triangle
 *    {a,b,c} of G is found exactly once, so the count is |M|/|Q| of Alg. 1.
 *    Found by merging the two sorted out-neighbour lists (node iterator).
 *    Per-vertex counts t(x) = number of triangles containing x.
 *  - oracle_vertex_triangles: t(v) by its definition straight from the raw
 *    input pairs: the number of distinct edges among the neighbours of v.
 *  - oracle_list: the match set M itself (Sec. II-A: the output of subgraph
 *    matching is every match; Alg. 1 collects the complete matches in M).  Each
 *    triangle is one match under the orientation, written as the triple
 *    (u, v, w) = (u1, u2, u3) of the query path with its non-tree edge.
 *  - oracle_kcore: the NE (neighbourhood-encoding) candidate filter of Alg. 1
 *    and Sec. III-C, read as: a data vertex can stand for a query node of
 *    degree k only if it keeps at least k neighbours that are candidates too,
 *    applied until nothing changes (the k-core).  For the triangle k = 2.
 *  - oracle_count_k4: the same matching for the 4-clique query (the paper
 *    presents the triangle as one instance of subgraph matching; a 4-clique is
 *    the next clique query): with the orientation every 4-clique is found once
 *    as u -> v -> w -> x with all six edges present.
 *  - oracle_edge_support: for every edge, the number of matches (triangles)
 *    that use it, i.e. how many times it appears as a query edge among the
 *    matches of M.  Each match u -> v -> w, u -> w adds one to each of its
 *    three edges.
 *  - oracle_count_diamonds: the diamond query (two triangles sharing an edge),
 *    a query with two neighbourhood-equivalence classes (Def. 3), each with its
 *    own unique mapping order.
 *  - oracle_count_labelled: the labelled triangle query (Sec. II-A: matching
 *    with node label information): a triangle {a, b, c} of G matches the query
 *    with node labels {l0, l1, l2} when the multiset of its vertices' labels
 *    equals the query's; each matching triangle counts once (as a subgraph).
 *  - oracle_count_directed: the directed triangle query (Sec. II-A: the method
 *    extends to directed graphs): the data graph is a set of arcs, its
 *    triangles those of the underlying undirected graph; a match maps the
 *    query's three nodes one-to-one onto a triangle so that every query arc
 *    lands on an arc of the same direction (or, induced, so that the arcs
 *    between two matched vertices are exactly the images of the query's).
 *    Matches count as subgraphs: embeddings divided by the query's
 *    automorphisms.
 *  - oracle_count_edge_labelled: the triangle query with edge labels (Sec.
 *    II-A: matching with edge label information): the data graph's undirected
 *    edges carry labels (an edge given several times takes the largest of its
 *    labels); a match maps the query's nodes one-to-one onto a triangle so that
 *    each query edge lands on a data edge of the same label.  Counted as
 *    subgraphs: maps divided by the query's label-preserving automorphisms.
 *
 * Every function is pinned by the CPU test suite against brute force over
 * vertex triples, trace(A^3)/6 and diag(A^3)/2, closed forms and invariants.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

static int cmp_u64(const void* a, const void* b) {
  uint64_t x = *(const uint64_t*)a, y = *(const uint64_t*)b;
  return (x > y) - (x < y);
}

static int cmp_i32(const void* a, const void* b) {
  int32_t x = *(const int32_t*)a, y = *(const int32_t*)b;
  return (x > y) - (x < y);
}

/*
 * Clean num_pairs raw pairs into a symmetric CSR.
 * row_ptr: int64[n+1]; col: int32[cap].
 * Returns 2m (number of stored entries), -2 if an id is outside [0, n),
 * -3 if 2m > cap, -1 on allocation failure.
 */
int64_t oracle_clean(int64_t n, int64_t num_pairs, const int32_t* src, const int32_t* dst,
                     int64_t* row_ptr, int32_t* col, int64_t cap) {
  for (int64_t i = 0; i < num_pairs; ++i) {
    if (src[i] < 0 || src[i] >= n || dst[i] < 0 || dst[i] >= n) return -2;
  }
  /* one key per unordered pair {a, b}, a < b; self-loops are not edges */
  uint64_t* keys = (uint64_t*)malloc(sizeof(uint64_t) * (size_t)(num_pairs > 0 ? num_pairs : 1));
  if (!keys) return -1;
  int64_t k = 0;
  for (int64_t i = 0; i < num_pairs; ++i) {
    int64_t a = src[i], b = dst[i];
    if (a == b) continue;
    if (a > b) { int64_t t = a; a = b; b = t; }
    keys[k++] = ((uint64_t)a << 32) | (uint64_t)b;
  }
  qsort(keys, (size_t)k, sizeof(uint64_t), cmp_u64);
  int64_t m = 0;
  for (int64_t i = 0; i < k; ++i) {
    if (i == 0 || keys[i] != keys[i - 1]) keys[m++] = keys[i];
  }
  if (2 * m > cap) { free(keys); return -3; }
  /* degree of every vertex, then offsets */
  for (int64_t v = 0; v <= n; ++v) row_ptr[v] = 0;
  for (int64_t i = 0; i < m; ++i) {
    row_ptr[(keys[i] >> 32) + 1] += 1;
    row_ptr[(keys[i] & 0xFFFFFFFFu) + 1] += 1;
  }
  for (int64_t v = 0; v < n; ++v) row_ptr[v + 1] += row_ptr[v];
  int64_t* fill = (int64_t*)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
  if (!fill) { free(keys); return -1; }
  for (int64_t v = 0; v < n; ++v) fill[v] = row_ptr[v];
  for (int64_t i = 0; i < m; ++i) {
    int32_t a = (int32_t)(keys[i] >> 32), b = (int32_t)(keys[i] & 0xFFFFFFFFu);
    col[fill[a]++] = b;
    col[fill[b]++] = a;
  }
  for (int64_t v = 0; v < n; ++v) {
    qsort(col + row_ptr[v], (size_t)(row_ptr[v + 1] - row_ptr[v]), sizeof(int32_t), cmp_i32);
  }
  free(fill);
  free(keys);
  return 2 * m;
}

/*
 * rank(u) < rank(v) for the strict total order selected by `order`:
 *   0: (degree, id)   1: id   2: (key[v], id) for a caller-supplied key array.
 */
static int rank_less(int32_t order, const int64_t* row_ptr, const int64_t* key, int64_t u,
                     int64_t v) {
  int64_t ku = 0, kv = 0;
  if (order == 0) {
    ku = row_ptr[u + 1] - row_ptr[u];
    kv = row_ptr[v + 1] - row_ptr[v];
  } else if (order == 2) {
    ku = key[u];
    kv = key[v];
  }
  if (ku != kv) return ku < kv;
  return u < v;
}

/*
 * Orient a symmetric CSR: keep entry (u, v) iff rank(u) < rank(v).
 * dag_ptr: int64[n+1]; dag_col: int32[row_ptr[n] / 2].  Rows stay ascending
 * by id (a subsequence of the symmetric row).  Returns m, the kept entries.
 */
int64_t oracle_orient(int64_t n, const int64_t* row_ptr, const int32_t* col, int32_t order,
                      const int64_t* key, int64_t* dag_ptr, int32_t* dag_col) {
  int64_t m = 0;
  dag_ptr[0] = 0;
  for (int64_t u = 0; u < n; ++u) {
    for (int64_t e = row_ptr[u]; e < row_ptr[u + 1]; ++e) {
      if (rank_less(order, row_ptr, key, u, col[e])) dag_col[m++] = col[e];
    }
    dag_ptr[u + 1] = m;
  }
  return m;
}

/*
 * Count triangles of an oriented graph (rows ascending by id).
 * For each source u and each v in N+(u), every w common to N+(u) and N+(v)
 * closes the wedge u -> v -> w: one triangle {u, v, w}.
 * t (nullable): uint64[n], set to the per-vertex counts.
 * threads <= 0 uses the OpenMP default.  Only the sources u < sources are
 * enumerated (sources = n for the whole graph; fewer gives a timing sample).
 */
uint64_t oracle_count(int64_t n, int64_t sources, const int64_t* dag_ptr, const int32_t* dag_col,
                      uint64_t* t, int32_t threads) {
  uint64_t total = 0;
  if (t) memset(t, 0, sizeof(uint64_t) * (size_t)n);
  if (sources > n) sources = n;
#ifdef _OPENMP
  if (threads > 0) omp_set_num_threads(threads);
#else
  (void)threads;
#endif
#pragma omp parallel for schedule(dynamic, 64) reduction(+ : total)
  for (int64_t u = 0; u < sources; ++u) {
    for (int64_t e = dag_ptr[u]; e < dag_ptr[u + 1]; ++e) {
      int64_t v = dag_col[e];
      int64_t i = dag_ptr[u], iend = dag_ptr[u + 1];
      int64_t j = dag_ptr[v], jend = dag_ptr[v + 1];
      uint64_t found = 0;
      while (i < iend && j < jend) {
        int32_t a = dag_col[i], b = dag_col[j];
        if (a < b) {
          ++i;
        } else if (b < a) {
          ++j;
        } else {
          ++found;
          if (t) {
#pragma omp atomic
            t[a] += 1;
          }
          ++i;
          ++j;
        }
      }
      total += found;
      if (t && found) {
#pragma omp atomic
        t[u] += found;
#pragma omp atomic
        t[v] += found;
      }
    }
  }
  return total;
}

/* Threads an OpenMP parallel region of oracle_count would use. */
int32_t oracle_max_threads(void) {
#ifdef _OPENMP
  return (int32_t)omp_get_max_threads();
#else
  return 1;
#endif
}

/*
 * t(v) from the raw pairs, by definition: the number of distinct edges {a, b}
 * (a != b) with both a and b adjacent to v.  Returns -1 on a bad argument.
 */
int64_t oracle_vertex_triangles(int64_t n, int64_t num_pairs, const int32_t* src,
                                const int32_t* dst, int32_t v) {
  if (v < 0 || v >= n) return -1;
  unsigned char* nbr = (unsigned char*)calloc((size_t)(n > 0 ? n : 1), 1);
  if (!nbr) return -1;
  for (int64_t i = 0; i < num_pairs; ++i) {
    if (src[i] == v && dst[i] != v) nbr[dst[i]] = 1;
    if (dst[i] == v && src[i] != v) nbr[src[i]] = 1;
  }
  int64_t cap = 1024, k = 0;
  uint64_t* keys = (uint64_t*)malloc(sizeof(uint64_t) * (size_t)cap);
  if (!keys) { free(nbr); return -1; }
  for (int64_t i = 0; i < num_pairs; ++i) {
    int64_t a = src[i], b = dst[i];
    if (a == b || !nbr[a] || !nbr[b]) continue;
    if (a > b) { int64_t t = a; a = b; b = t; }
    if (k == cap) {
      cap *= 2;
      uint64_t* grown = (uint64_t*)realloc(keys, sizeof(uint64_t) * (size_t)cap);
      if (!grown) { free(keys); free(nbr); return -1; }
      keys = grown;
    }
    keys[k++] = ((uint64_t)a << 32) | (uint64_t)b;
  }
  qsort(keys, (size_t)k, sizeof(uint64_t), cmp_u64);
  int64_t distinct = 0;
  for (int64_t i = 0; i < k; ++i) {
    if (i == 0 || keys[i] != keys[i - 1]) ++distinct;
  }
  free(keys);
  free(nbr);
  return distinct;
}

/*
 * The triangles of an oriented graph as triples (u, v, w) with v and w in
 * N+(u) and w in N+(v): for every u in id order, every v in N+(u) in row
 * order, the common out-neighbours w of u and v in increasing order, so the
 * triples come out in lexicographic (u, v, w) order (rows are sorted).
 * out (nullable): int32[3 * cap], receives the first min(T, cap) triples.
 * Returns T.  Single-threaded.
 */
int64_t oracle_list(int64_t n, const int64_t* dag_ptr, const int32_t* dag_col, int32_t* out,
                    int64_t cap) {
  int64_t found = 0;
  for (int64_t u = 0; u < n; ++u) {
    for (int64_t e = dag_ptr[u]; e < dag_ptr[u + 1]; ++e) {
      int64_t v = dag_col[e];
      int64_t i = dag_ptr[u], iend = dag_ptr[u + 1];
      int64_t j = dag_ptr[v], jend = dag_ptr[v + 1];
      while (i < iend && j < jend) {
        int32_t a = dag_col[i], b = dag_col[j];
        if (a < b) {
          ++i;
        } else if (b < a) {
          ++j;
        } else {
          if (out && found < cap) {
            out[3 * found + 0] = (int32_t)u;
            out[3 * found + 1] = (int32_t)v;
            out[3 * found + 2] = a;
          }
          ++found;
          ++i;
          ++j;
        }
      }
    }
  }
  return found;
}

/*
 * Support of every oriented edge: sup[e] (e an index into dag_col) = number of
 * triangles containing that edge.  Every triangle found by merging N+(u) and
 * N+(v) for the edge e = (u, v) adds one to e, to (u, w) and to (v, w), whose
 * indices are the merge positions.  sup: uint32[dag_ptr[n]], overwritten.
 * Single-threaded.  Returns T.
 */
int64_t oracle_edge_support(int64_t n, const int64_t* dag_ptr, const int32_t* dag_col,
                            uint32_t* sup) {
  memset(sup, 0, sizeof(uint32_t) * (size_t)dag_ptr[n]);
  int64_t found = 0;
  for (int64_t u = 0; u < n; ++u) {
    for (int64_t e = dag_ptr[u]; e < dag_ptr[u + 1]; ++e) {
      int64_t v = dag_col[e];
      int64_t i = dag_ptr[u], iend = dag_ptr[u + 1];
      int64_t j = dag_ptr[v], jend = dag_ptr[v + 1];
      while (i < iend && j < jend) {
        int32_t a = dag_col[i], b = dag_col[j];
        if (a < b) {
          ++i;
        } else if (b < a) {
          ++j;
        } else {
          sup[e] += 1;  /* (u, v) */
          sup[i] += 1;  /* (u, w) */
          sup[j] += 1;  /* (v, w) */
          ++found;
          ++i;
          ++j;
        }
      }
    }
  }
  return found;
}

/*
 * k-core membership of a symmetric CSR: keep[v] = 1 iff v belongs to the
 * largest subgraph in which every vertex has at least k neighbours.  Peels with
 * a queue: a vertex whose count of surviving neighbours drops below k is removed
 * and its neighbours' counts drop by one.  Returns the number kept.
 */
int64_t oracle_kcore(int64_t n, const int64_t* row_ptr, const int32_t* col, int32_t k,
                     uint8_t* keep) {
  int64_t* cnt = (int64_t*)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
  int64_t* queue = (int64_t*)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
  if (!cnt || !queue) { free(cnt); free(queue); return -1; }
  int64_t head = 0, tail = 0;
  for (int64_t v = 0; v < n; ++v) {
    cnt[v] = row_ptr[v + 1] - row_ptr[v];
    keep[v] = 1;
    if (cnt[v] < k) { keep[v] = 0; queue[tail++] = v; }
  }
  while (head < tail) {
    int64_t v = queue[head++];
    for (int64_t e = row_ptr[v]; e < row_ptr[v + 1]; ++e) {
      int64_t w = col[e];
      if (keep[w] && --cnt[w] < k) { keep[w] = 0; queue[tail++] = w; }
    }
  }
  free(cnt);
  free(queue);
  return n - tail;
}

/*
 * Number of 4-cliques of an oriented graph: for every u, every v in N+(u), the
 * common out-neighbours S = N+(u) & N+(v) (sorted merge), and for every w in S
 * the size of S & N+(w) (another merge).  Single-threaded.
 */
uint64_t oracle_count_k4(int64_t n, const int64_t* dag_ptr, const int32_t* dag_col) {
  int64_t maxd = 0;
  for (int64_t u = 0; u < n; ++u)
    if (dag_ptr[u + 1] - dag_ptr[u] > maxd) maxd = dag_ptr[u + 1] - dag_ptr[u];
  int32_t* common = (int32_t*)malloc(sizeof(int32_t) * (size_t)(maxd > 0 ? maxd : 1));
  if (!common) return UINT64_MAX;
  uint64_t total = 0;
  for (int64_t u = 0; u < n; ++u) {
    for (int64_t e = dag_ptr[u]; e < dag_ptr[u + 1]; ++e) {
      int64_t v = dag_col[e];
      int64_t i = dag_ptr[u], iend = dag_ptr[u + 1];
      int64_t j = dag_ptr[v], jend = dag_ptr[v + 1];
      int64_t k = 0;
      while (i < iend && j < jend) {
        if (dag_col[i] < dag_col[j]) ++i;
        else if (dag_col[j] < dag_col[i]) ++j;
        else { common[k++] = dag_col[i]; ++i; ++j; }
      }
      for (int64_t a = 0; a < k; ++a) {
        int64_t w = common[a];
        int64_t p = 0, q = dag_ptr[w], qend = dag_ptr[w + 1];
        while (p < k && q < qend) {
          if (common[p] < dag_col[q]) ++p;
          else if (dag_col[q] < common[p]) ++q;
          else { ++total; ++p; ++q; }
        }
      }
    }
  }
  free(common);
  return total;
}

/*
 * Number of diamonds: matches of the 4-node query made of two triangles
 * {a,b,c} and {b,c,d} that share the edge {b,c}, counted as subgraphs (a and d
 * may or may not be adjacent; Def. 2 asks only that query edges map to data
 * edges).  The query's nodes form two neighbourhood-equivalence classes
 * (Def. 3): {b, c}, each adjacent to all three others, and {a, d}, each
 * adjacent to b and c only.  The unique mapping order fixes one order inside
 * each class, b < c and a < d (Alg. 1 "Generate_UMO"; vertex ids here), so each
 * diamond subgraph is matched once.  Matching order b, c, a, d: every edge
 * {b, c} with b < c; the candidates for a and for d are the vertices adjacent
 * to both b and c (the query edges a-b, a-c; d-b, d-c), found by merging the
 * two sorted rows of the symmetric CSR; every pair a < d of the k candidates
 * is one match: k(k-1)/2.  Only edges whose lower end b < sources take part
 * (sources = n: all).  Single-threaded.
 */
uint64_t oracle_count_diamonds(int64_t n, int64_t sources, const int64_t* row_ptr,
                               const int32_t* col) {
  uint64_t total = 0;
  if (sources > n) sources = n;
  for (int64_t b = 0; b < sources; ++b) {
    for (int64_t e = row_ptr[b]; e < row_ptr[b + 1]; ++e) {
      int64_t c = col[e];
      if (c <= b) continue;
      int64_t i = row_ptr[b], iend = row_ptr[b + 1];
      int64_t j = row_ptr[c], jend = row_ptr[c + 1];
      uint64_t k = 0;
      while (i < iend && j < jend) {
        if (col[i] < col[j]) ++i;
        else if (col[j] < col[i]) ++j;
        else { ++k; ++i; ++j; }
      }
      total += k * (k - 1) / 2;  /* k >= 2 only: 2-look-ahead on the candidates */
    }
  }
  return total;
}

/*
 * Labelled triangles: the triangles {a, b, c} of the oriented graph whose label
 * multiset {L(a), L(b), L(c)} equals {q0, q1, q2}.  Every triangle is found once
 * by the node iterator of oracle_count; its three labels are sorted and
 * compared with the sorted query.  Single-threaded.
 */
static void sort3(int32_t* x, int32_t* y, int32_t* z) {
  int32_t t;
  if (*x > *y) { t = *x; *x = *y; *y = t; }
  if (*y > *z) { t = *y; *y = *z; *z = t; }
  if (*x > *y) { t = *x; *x = *y; *y = t; }
}

uint64_t oracle_count_labelled(int64_t n, const int64_t* dag_ptr, const int32_t* dag_col,
                               const int32_t* labels, int32_t q0, int32_t q1, int32_t q2) {
  uint64_t total = 0;
  sort3(&q0, &q1, &q2);
  for (int64_t u = 0; u < n; ++u) {
    for (int64_t e = dag_ptr[u]; e < dag_ptr[u + 1]; ++e) {
      int64_t v = dag_col[e];
      int64_t i = dag_ptr[u], iend = dag_ptr[u + 1];
      int64_t j = dag_ptr[v], jend = dag_ptr[v + 1];
      while (i < iend && j < jend) {
        int32_t a = dag_col[i], b = dag_col[j];
        if (a < b) {
          ++i;
        } else if (b < a) {
          ++j;
        } else {
          int32_t x = labels[u], y = labels[v], z = labels[a];
          sort3(&x, &y, &z);
          if (x == q0 && y == q1 && z == q2) ++total;
          ++i;
          ++j;
        }
      }
    }
  }
  return total;
}

/*
 * oracle_count_directed - the directed triangle query.
 *
 * Arcs: the pairs (src[i] -> dst[i]) with src[i] != dst[i], duplicates allowed;
 * dag_ptr / dag_col orient the underlying undirected graph (as oracle_orient
 * writes it) and enumerate its triangles.  The query is a directed graph on the
 * nodes 0, 1, 2 with every pair connected: p01, p02, p12 hold bit 1 when the
 * lower node has an arc to the higher, bit 2 when the higher has one to the
 * lower (each in 1..3).  An embedding is a one-to-one map f of the query nodes
 * onto the three vertices of a triangle such that for every ordered pair
 * (i, j) of query nodes the query arc i -> j implies the arc f(i) -> f(j)
 * (induced = 0), or the two are present together (induced = 1).  The result
 * is the number of embeddings over all triangles divided by the number of
 * permutations of the query nodes that map its arcs onto its arcs.  Only the
 * triangles whose DAG source (first vertex) has an id below `sources` count
 * (sources = n: all of them).
 * Returns -2 if a pair holds an id outside [0, n), -3 for a code outside
 * 1..3, -1 on allocation failure.  Single-threaded.
 */
static int arc_of(int32_t p01, int32_t p02, int32_t p12, int i, int j) {
  int32_t code = (i == 0 && j == 1) || (i == 1 && j == 0) ? p01
               : (i == 0 && j == 2) || (i == 2 && j == 0) ? p02 : p12;
  return i < j ? (code & 1) != 0 : (code & 2) != 0;
}

static int has_arc(const uint64_t* keys, int64_t nk, int64_t x, int64_t y) {
  uint64_t want = ((uint64_t)x << 32) | (uint64_t)y;
  int64_t lo = 0, hi = nk;
  while (lo < hi) {
    int64_t mid = lo + (hi - lo) / 2;
    if (keys[mid] < want) lo = mid + 1;
    else hi = mid;
  }
  return lo < nk && keys[lo] == want;
}

int64_t oracle_count_directed(int64_t n, const int64_t* dag_ptr, const int32_t* dag_col,
                              int64_t num_pairs, const int32_t* src, const int32_t* dst,
                              int32_t p01, int32_t p02, int32_t p12, int32_t induced,
                              int64_t sources) {
  static const int perms[6][3] = {{0, 1, 2}, {0, 2, 1}, {1, 0, 2}, {1, 2, 0}, {2, 0, 1}, {2, 1, 0}};
  if (p01 < 1 || p01 > 3 || p02 < 1 || p02 > 3 || p12 < 1 || p12 > 3) return -3;
  for (int64_t i = 0; i < num_pairs; ++i)
    if (src[i] < 0 || src[i] >= n || dst[i] < 0 || dst[i] >= n) return -2;
  uint64_t* keys = (uint64_t*)malloc(sizeof(uint64_t) * (size_t)(num_pairs > 0 ? num_pairs : 1));
  if (!keys) return -1;
  int64_t nk = 0;
  for (int64_t i = 0; i < num_pairs; ++i)
    if (src[i] != dst[i]) keys[nk++] = ((uint64_t)(uint32_t)src[i] << 32) | (uint32_t)dst[i];
  qsort(keys, (size_t)nk, sizeof(uint64_t), cmp_u64);
  /* the query's automorphisms */
  int64_t aut = 0;
  for (int s = 0; s < 6; ++s) {
    int same = 1;
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j)
        if (i != j && arc_of(p01, p02, p12, i, j) != arc_of(p01, p02, p12, perms[s][i], perms[s][j]))
          same = 0;
    aut += same;
  }
  int64_t embeddings = 0;
  for (int64_t u = 0; u < sources; ++u) {
    for (int64_t e = dag_ptr[u]; e < dag_ptr[u + 1]; ++e) {
      int64_t v = dag_col[e];
      int64_t i = dag_ptr[u], iend = dag_ptr[u + 1];
      int64_t j = dag_ptr[v], jend = dag_ptr[v + 1];
      while (i < iend && j < jend) {
        int32_t a = dag_col[i], b = dag_col[j];
        if (a < b) {
          ++i;
        } else if (b < a) {
          ++j;
        } else {
          int64_t t[3] = {u, v, a};
          for (int s = 0; s < 6; ++s) {
            int ok = 1;
            for (int x = 0; x < 3 && ok; ++x)
              for (int y = 0; y < 3 && ok; ++y) {
                if (x == y) continue;
                int q = arc_of(p01, p02, p12, x, y);
                int g = has_arc(keys, nk, t[perms[s][x]], t[perms[s][y]]);
                if (induced ? q != g : (q && !g)) ok = 0;
              }
            embeddings += ok;
          }
          ++i;
          ++j;
        }
      }
    }
  }
  free(keys);
  return embeddings / aut;
}

/*
 * oracle_count_edge_labelled - the triangle query with edge labels.
 *
 * Pairs (src[i], dst[i]) with labels lab[i] (src != dst; duplicates and both
 * directions allowed): the undirected edge {a, b} has the largest label of its
 * pairs.  dag_ptr / dag_col orient the undirected graph (as oracle_orient
 * writes it) and enumerate its triangles.  The query's edges 0-1, 0-2, 1-2
 * carry the labels q01, q02, q12.  An embedding is a one-to-one map f of the
 * query nodes onto a triangle's vertices with label{f(i), f(j)} = q_ij for each
 * query edge; the result is the number of embeddings divided by the number of
 * permutations of the query nodes that keep every edge's label.  Only the
 * triangles whose DAG source has an id below `sources` count (n: all).
 * Returns -2 if a pair holds an id outside [0, n), -1 on allocation failure.
 * Single-threaded.
 */
static int32_t query_label(int32_t q01, int32_t q02, int32_t q12, int i, int j) {
  int lo = i < j ? i : j, hi = i < j ? j : i;
  return lo == 0 ? (hi == 1 ? q01 : q02) : q12;
}

/* label of edge {x, y} from the sorted (min << 32 | max) keys, or -1 */
static int32_t edge_label_of(const uint64_t* keys, const int32_t* labs, int64_t nk, int64_t x,
                             int64_t y) {
  int64_t a = x < y ? x : y, b = x < y ? y : x;
  uint64_t want = ((uint64_t)a << 32) | (uint64_t)b;
  int64_t lo = 0, hi = nk;
  while (lo < hi) {
    int64_t mid = lo + (hi - lo) / 2;
    if (keys[mid] < want) lo = mid + 1;
    else hi = mid;
  }
  return lo < nk && keys[lo] == want ? labs[lo] : -1;
}

typedef struct {
  uint64_t key;
  int32_t lab;
} keyed_label;

static int cmp_keyed(const void* a, const void* b) {
  const keyed_label* x = (const keyed_label*)a;
  const keyed_label* y = (const keyed_label*)b;
  if (x->key != y->key) return (x->key > y->key) - (x->key < y->key);
  return (x->lab > y->lab) - (x->lab < y->lab);
}

int64_t oracle_count_edge_labelled(int64_t n, const int64_t* dag_ptr, const int32_t* dag_col,
                                   int64_t num_pairs, const int32_t* src, const int32_t* dst,
                                   const int32_t* lab, int32_t q01, int32_t q02, int32_t q12,
                                   int64_t sources) {
  static const int perms[6][3] = {{0, 1, 2}, {0, 2, 1}, {1, 0, 2}, {1, 2, 0}, {2, 0, 1}, {2, 1, 0}};
  for (int64_t i = 0; i < num_pairs; ++i)
    if (src[i] < 0 || src[i] >= n || dst[i] < 0 || dst[i] >= n) return -2;
  keyed_label* kl = (keyed_label*)malloc(sizeof(keyed_label) * (size_t)(num_pairs > 0 ? num_pairs : 1));
  if (!kl) return -1;
  int64_t k = 0;
  for (int64_t i = 0; i < num_pairs; ++i) {
    int64_t a = src[i], b = dst[i];
    if (a == b) continue;
    if (a > b) { int64_t t = a; a = b; b = t; }
    kl[k].key = ((uint64_t)a << 32) | (uint64_t)b;
    kl[k].lab = lab[i];
    ++k;
  }
  qsort(kl, (size_t)k, sizeof(keyed_label), cmp_keyed);
  /* one entry per edge: the last of its run holds the largest label */
  uint64_t* keys = (uint64_t*)malloc(sizeof(uint64_t) * (size_t)(k > 0 ? k : 1));
  int32_t* labs = (int32_t*)malloc(sizeof(int32_t) * (size_t)(k > 0 ? k : 1));
  if (!keys || !labs) {
    free(kl); free(keys); free(labs);
    return -1;
  }
  int64_t nk = 0;
  for (int64_t i = 0; i < k; ++i) {
    if (i + 1 < k && kl[i + 1].key == kl[i].key) continue;
    keys[nk] = kl[i].key;
    labs[nk] = kl[i].lab;
    ++nk;
  }
  free(kl);
  int64_t aut = 0;
  for (int s = 0; s < 6; ++s) {
    int same = 1;
    for (int i = 0; i < 3; ++i)
      for (int j = i + 1; j < 3; ++j)
        if (query_label(q01, q02, q12, i, j) !=
            query_label(q01, q02, q12, perms[s][i], perms[s][j]))
          same = 0;
    aut += same;
  }
  int64_t embeddings = 0;
  for (int64_t u = 0; u < sources; ++u) {
    for (int64_t e = dag_ptr[u]; e < dag_ptr[u + 1]; ++e) {
      int64_t v = dag_col[e];
      int64_t i = dag_ptr[u], iend = dag_ptr[u + 1];
      int64_t j = dag_ptr[v], jend = dag_ptr[v + 1];
      while (i < iend && j < jend) {
        int32_t a = dag_col[i], b = dag_col[j];
        if (a < b) {
          ++i;
        } else if (b < a) {
          ++j;
        } else {
          int64_t t[3] = {u, v, a};
          for (int s = 0; s < 6; ++s) {
            int ok = 1;
            for (int x = 0; x < 3 && ok; ++x)
              for (int y = x + 1; y < 3 && ok; ++y)
                if (edge_label_of(keys, labs, nk, t[perms[s][x]], t[perms[s][y]]) !=
                    query_label(q01, q02, q12, x, y))
                  ok = 0;
            embeddings += ok;
          }
          ++i;
          ++j;
        }
      }
    }
  }
  free(keys);
  free(labs);
  return embeddings / aut;
}
