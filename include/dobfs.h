/*
 * dobfs.h -- direction-optimized breadth-first search on one AMD Instinct
 * MI355X (gfx950), exposed as a C ABI.
 *
 * Method: Yang, Buluc & Owens, "Implementing Push-Pull Efficiently in
 * GraphBLAS" (arXiv 1804.03327). One BFS level computes the masked Boolean
 * matvec f' = A^T f .* not(v) over the semiring ({0,1}, OR, AND, 0)
 * (Section 4, Algorithm 1) either column-based ("push", Equation 5,
 * Section 6.2) or row-based with a mask and early exit ("pull", Equation 4,
 * Algorithm 2, Sections 5.2-5.4); a per-level rule picks the direction
 * (Section 6.3).
 *
 * Conventions shared by every call
 * --------------------------------
 *  - Graph: A(u,v) = 1 for an edge u->v. CSR(A): csr_colind[csr_rowptr[u] ..
 *    csr_rowptr[u+1]) are the out-neighbours of u (used by push).
 *    CSC(A): csc_rowind[csc_colptr[v] .. csc_colptr[v+1]) are the
 *    in-neighbours of v (used by pull). Indices are int32; nnz <= 2^31-1.
 *    Rows need not be sorted; self-loops and duplicates are accepted. For an
 *    undirected graph pass the same arrays twice.
 *  - Bit vectors: bit i of a length-V vector is bit (i & 31) of uint32 word
 *    i >> 5; ceil(V/32) words. Bits at positions >= V are ignored on input
 *    and written as 0 on output.
 *  - Device pointers are HIP device memory of the graph's device. Host
 *    pointers are ordinary host memory. `stream` is a hipStream_t (NULL =
 *    the null stream); all device work of a call is ordered on it.
 *  - Every function returns a dobfs_status. Nothing aborts or throws across
 *    the ABI. On failure dobfs_last_error() gives a message for the calling
 *    thread, and no output has been written unless stated.
 *  - Thread safety: graphs are immutable after creation. Calls on one graph
 *    from several threads are safe when each passes its own workspace; calls
 *    that let the library use its internal workspace (workspace = NULL) must
 *    not overlap on one graph.
 */
#ifndef DOBFS_H
#define DOBFS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  DOBFS_OK = 0,
  DOBFS_ERR_INVALID_ARG = 1,         /* bad size, pointer, index or option */
  DOBFS_ERR_OUT_OF_MEMORY = 2,       /* device or pinned-host allocation failed */
  DOBFS_ERR_DEVICE = 3,              /* a HIP call failed (no GPU, launch error ...) */
  DOBFS_ERR_WORKSPACE_TOO_SMALL = 4, /* ws_bytes below the *_workspace_bytes figure */
  DOBFS_ERR_UNSUPPORTED = 5,         /* option combination not implemented */
  DOBFS_ERR_INTERNAL = 6,
  DOBFS_ERR_TIMEOUT = 7              /* dobfs_server_wait: the query was not done in time */
} dobfs_status;

typedef struct dobfs_graph_s *dobfs_graph;

/* ------------------------------------------------------------------ graphs */

enum {
  DOBFS_UPLOAD_VALIDATE = 1u,  /* accepted for compatibility; the checks below are always made */
  DOBFS_UPLOAD_HUBS_FIRST = 2u /* keep every CSC(A) column (a row's in-neighbours) ordered by
                                  decreasing out-degree of the neighbour, ties by id, in a copy
                                  the graph owns: the pull's early exit (Section 5.3) then tends
                                  to stop at the first entries. Depths are unchanged; a pull
                                  reports the first hit in this order as the parent. */
};

/*
 * Copy a graph from host memory to device `device` (Section 6: the matrix is
 * held as CSR for push and CSC for pull). The library owns the device copy
 * until dobfs_graph_destroy. Checked before anything is allocated: V >= 1,
 * 0 <= nnz <= 2^31-1, non-null arrays (colind/rowind may be NULL when
 * nnz = 0), offsets start at 0, never decrease and end at nnz, and every
 * index lies in [0, V) (O(V + nnz) on the host). flags: 0 or
 * DOBFS_UPLOAD_VALIDATE. Returns INVALID_ARG on a failed check, DEVICE /
 * OUT_OF_MEMORY on HIP failures; *out is set only on success. When the CSR
 * and CSC pointers are the same (an undirected graph), one copy is stored
 * (with DOBFS_UPLOAD_HUBS_FIRST the CSC side gets its own reordered copy).
 */
dobfs_status dobfs_graph_upload(int32_t V, int64_t nnz, const int32_t *csr_rowptr,
                                const int32_t *csr_colind, const int32_t *csc_colptr,
                                const int32_t *csc_rowind, int32_t device, uint32_t flags,
                                dobfs_graph *out);

/*
 * Same, from arrays already in device memory of `device`. The arrays are
 * BORROWED: the caller keeps them alive and unchanged until the graph is
 * destroyed. The same checks run on the device (offsets monotone from 0 to
 * nnz, indices in [0, V)). Work is ordered on `stream`; the call returns
 * after it completes.
 */
dobfs_status dobfs_graph_wrap_device(int32_t V, int64_t nnz, const int32_t *csr_rowptr,
                                     const int32_t *csr_colind, const int32_t *csc_colptr,
                                     const int32_t *csc_rowind, int32_t device, uint32_t flags,
                                     void *stream, dobfs_graph *out);

/* Free the graph's device memory and its internal workspace. NULL is a no-op. */
dobfs_status dobfs_graph_destroy(dobfs_graph g);

/* Vertex and edge counts of a graph (either pointer may be NULL). */
dobfs_status dobfs_graph_info(dobfs_graph g, int32_t *V, int64_t *nnz, int32_t *device);

/* ---------------------------------------------------------- BFS options */

enum {
  DOBFS_DIR_PUSH = 0, /* column-based masked matvec over CSR(A) (Algorithm 3, Equation 5) */
  DOBFS_DIR_PULL = 1  /* row-based masked matvec over CSC(A) (Algorithm 2, Equation 4) */
};

/* Which optimizations of Table 2 are active (each row adds to the previous). */
enum {
  DOBFS_MODE_FULL = 0,           /* direction change + masking + early exit + operand reuse */
  DOBFS_MODE_PUSH_ONLY = 1,      /* push at every level (Table 2 "Structure only") */
  DOBFS_MODE_PULL_UNMASKED = 2,  /* pull computes every row from the frontier, mask after */
  DOBFS_MODE_PULL_MASKED = 3,    /* pull computes unvisited rows only, scans whole rows */
  DOBFS_MODE_PULL_MASKED_EE = 4, /* as above, stopping at the first parent found */
  DOBFS_MODE_PULL_ONLY = 5,      /* FULL's pull at every level (no direction change) */
  DOBFS_MODE_PUSH_SORT = 6,      /* Table 2 "Baseline": push at every level as Algorithm 3 prints it:
                                    gather (neighbour, vertex) pairs, key-value radix sort, keep the
                                    first pair of each key, drop visited keys; the host reads each
                                    level's counts back. Needs the larger workspace that
                                    dobfs_bfs_workspace_bytes reports for this mode. */
  DOBFS_MODE_PUSH_SORT_KEYS = 7  /* Table 2 "Structure only" as the paper measures it (Section 5.5:
                                    a Boolean BFS needs the matrix's structure, not its values): the
                                    push of PUSH_SORT with the values dropped, a key-only radix sort
                                    of the gathered neighbours, unique keys, drop visited keys. It
                                    computes depths only: parent must be NULL (else INVALID_ARG).
                                    Same workspace as PUSH_SORT. */
};

enum {
  DOBFS_HEUR_RATIO = 0, /* Section 6.3: r = nnz(f)/V against alpha (up) and beta (down) */
  DOBFS_HEUR_EDGES = 1  /* Beamer's rule: push->pull when m_f/m_u > alpha; back when nnz(f)/V < beta */
};

enum {
  DOBFS_OPT_TIME_KERNELS = 1u, /* every kernel launch records its own start and end (HIP
                                  extended-launch events); fills the *_ms stats. In the
                                  persistent loop a level's time is the difference of the
                                  device clock at the starts of consecutive steps */
  DOBFS_OPT_PERSISTENT = 2u /* dobfs_bfs, dobfs_bfs_static and dobfs_bfs_batch: run the level
                               loop as a persistent kernel (one launch runs up to 64 steps,
                               co-resident blocks sized by the occupancy query, a grid barrier
                               between steps) instead of one launch per step. Same results. On MI355X the barrier needs an
                               agent-scope L2 write-back and invalidate per block (the XCDs' L2
                               caches are not coherent), which costs more than a kernel
                               boundary, so this is off by default. The environment variable
                               DOBFS_SPIN_LIMIT bounds every barrier wait (polls; exceeded ->
                               DOBFS_ERR_INTERNAL, every block leaves); DOBFS_PERSIST_BLOCKS
                               caps the grid */
};

typedef struct {
  int32_t mode;              /* DOBFS_MODE_* */
  int32_t heuristic;         /* DOBFS_HEUR_* */
  float alpha, beta;         /* switch points; 0.01 and 0.01 by default (Section 6.3) */
  const int8_t *forced_dirs; /* host, optional: direction of levels 0 .. n_forced-1 */
  int32_t n_forced;          /* levels past n_forced, or past the first 1024, follow the mode
                                and heuristic */
  uint32_t flags;            /* DOBFS_OPT_* */
  /* Schedule settings of the single-source kernels (results do not depend on them; 0 keeps
     the default; out-of-range values -> INVALID_ARG). The autotuner chooses them per graph. */
  int32_t pull_mid;          /* pull: in-neighbours a thread scans before a wave of 64 lanes takes
                                the row over, 4 .. 2^20 (default 32) */
  int32_t bitmap_rows;       /* push after a pull runs block-local over the pull's bits when no
                                4096-row tile found more rows than this, 0 .. 4096 (default 512) */
  int32_t local_unit;        /* block-local push: frontier vertices a block takes at once,
                                1 .. 256 (default 128) */
  int32_t local_chunks;      /* block-local push: most 1024-edge chunks of a unit one block may
                                get before the push needs the global degree scan, 1 .. 2^20
                                (default 4) */
} dobfs_options;

/* Fill *opt with the defaults (FULL, RATIO, alpha = beta = 0.01). */
dobfs_status dobfs_options_default(dobfs_options *opt);

/*
 * The direction rule of Section 6.3 as a pure host function. After a level
 * run in direction `dir` that turned a frontier of nf vertices into one of
 * n_new vertices, returns the direction for the next level:
 *   RATIO: push->pull when n_new > nf and n_new > alpha*V;
 *          pull->push when n_new < nf and n_new < beta*V; otherwise unchanged.
 *   EDGES: push->pull when m_f > alpha*m_u (m_f = out-edges of the new
 *          frontier, the push's next work; m_u = in-edges of the vertices
 *          still unvisited, the most a pull could scan; on an undirected
 *          graph both are plain degrees);
 *          pull->push when n_new < beta*V.
 * alpha and beta are compared in double precision.
 */
int32_t dobfs_next_direction(const dobfs_options *opt, int32_t dir, int64_t V, int64_t nf,
                             int64_t n_new, int64_t m_f, int64_t m_u);

/* ---------------------------------------------------------- statistics */

typedef struct {
  int32_t dir;     /* direction of this level */
  int32_t nf;      /* frontier size entering the level, nnz(f) */
  int32_t n_new;   /* vertices discovered by the level */
  int32_t variant; /* how a push level ran: 0 with a global scan of the frontier's degrees,
                      1 block-local over the frontier list, 2 block-local over the bits the
                      pull before it found; 0 for pull levels */
  int64_t edges;   /* push: nnz(m_f^+) adjacency entries read; pull: in-neighbours checked */
  int64_t m_f;     /* push: out-edges of the input frontier (0 on pull levels) */
  float ms_main;   /* execution time (DOBFS_OPT_TIME_KERNELS, else 0) of the level's pull or
                      push: the step that decides and runs the level (the expansion step
                      after a scan) */
  float ms_aux;    /* the scan step of a push level that needs the global degree scan (with
                      the bitmap-to-list conversion after a pull level), 0 otherwise; every
                      multi-source push level has one (it also merges the push before's
                      winners into the visited words and clears the next frontier) */
} dobfs_level_stats;

typedef struct {
  int32_t levels;           /* levels run (the last one discovers nothing) */
  int32_t cap;              /* capacity of `level` (caller sets; may be 0) */
  dobfs_level_stats *level; /* host array of cap entries, caller-owned, may be NULL */
  float ms_total;           /* device time of the whole call (events) */
  float ms_init;            /* init kernel execution time (DOBFS_OPT_TIME_KERNELS) */
  int64_t reached;          /* vertices with depth >= 0 (multi-source: (vertex, source) pairs) */
  /* Every launch of the per-level kernels in the call, counted the way a kernel profiler
     counts them, with their summed execution times (DOBFS_OPT_TIME_KERNELS, else 0).
     One step kernel, launched once per level, twice for a push level that needs the
     global degree scan (every multi-source push level does), once more for the step that
     finds the end, and for any steps enqueued past the end (they exit at once);
     launches_aux and ms_aux_all are 0. The sort-based push mode leaves all four at 0. */
  int32_t launches_main;
  int32_t launches_aux;
  float ms_main_all;
  float ms_aux_all;
  /* Single source: the traversed edges in the Graph500 count, i.e. the sum of out-degrees
     over the reached vertices, halved when the graph was given as undirected (the same
     arrays passed for CSR(A) and CSC(A)): every undirected edge with a reached endpoint
     counted once. Counted on the device after the traversal (outside ms_total).
     Multi-source: 0. */
  int64_t edges_g500;
} dobfs_stats;

/* ----------------------------------------------------------------- BFS */

/*
 * Device bytes of workspace one dobfs_bfs call on graph g needs (two visited
 * bitmaps, two frontier bitmaps, two frontier queues of V entries, the push
 * scan arrays and a small control block). opt may be NULL.
 */
dobfs_status dobfs_bfs_workspace_bytes(dobfs_graph g, const dobfs_options *opt, size_t *bytes);

/*
 * Breadth-first search from `source` (Algorithm 1). On return
 *   depth[v]  = hops on a shortest path source->v, -1 if unreachable
 *               (Algorithm 1's level numbers minus one: source 0);
 *   parent[v] = an in-neighbour u of v with depth[u] = depth[v]-1,
 *               parent[source] = source, -1 if unreachable. On pull levels
 *               it is the first such u in CSC order (early exit); on push
 *               levels any such u.
 * depth: device int32[V], required. parent: device int32[V] or NULL.
 * workspace: device memory of at least dobfs_bfs_workspace_bytes, or NULL
 * for a library-owned one. stats: host, optional (opt->flags may add
 * per-kernel times). The call blocks until results are final: each level's
 * direction is decided on the device, and the host reads the traversal state
 * back once per batch of levels. source outside [0,V) -> INVALID_ARG with
 * nothing written.
 * Workspace reuse: when the call returns, depth and parent are final, but
 * blocks of its last kernel may still be reading the workspace's control
 * block. A caller's workspace may be passed to a later call on the same
 * stream, or on another stream once the first stream has been synchronised
 * (or an event recorded on it waited for); the library-owned workspace is
 * ordered this way by the library.
 */
dobfs_status dobfs_bfs(dobfs_graph g, int32_t source, const dobfs_options *opt, int32_t *depth,
                       int32_t *parent, void *workspace, size_t ws_bytes, void *stream,
                       dobfs_stats *stats);

/*
 * For callers that cannot allocate device or pinned host memory (code that
 * must not call hipMalloc: tight serving loops, harnesses that forbid it):
 * dobfs_bfs with the workspace and the level report in a static device array
 * of the library, DOBFS_STATIC_SCRATCH_BYTES on every device the library runs
 * this call on, held until the process ends. The call makes no allocation
 * (no hipMalloc / hipFree / hipHostMalloc, no events): it copies each batch's
 * report into ordinary host memory after the stream has drained, so it
 * synchronises `stream` once per batch of levels.
 * Results, arguments and errors as dobfs_bfs, and:
 *  - the graph must fit: 16*V + 4*ceil(V/32)*4 + 4*(nnz/1024) bytes plus
 *    about 200 KB of control data (256-byte aligned regions) within the
 *    array; V <= 2^22 with nnz <= 2^28 always fits (RMAT scale 22, edge
 *    factor 16). Larger graphs -> INVALID_ARG, nothing written;
 *  - DOBFS_MODE_PUSH_SORT and DOBFS_OPT_TIME_KERNELS -> UNSUPPORTED (they
 *    need a larger workspace and events); stats receive no times (0);
 *  - every call on a device shares that device's array, which keeps the
 *    last call's contents (each call clears what it needs cleared). Calls
 *    that overlap on one device race: issue them on one stream, or
 *    synchronise the stream of the previous call first.
 */
#define DOBFS_STATIC_SCRATCH_BYTES ((size_t)68 << 20)
dobfs_status dobfs_bfs_static(dobfs_graph g, int32_t source, const dobfs_options *opt, int32_t *depth,
                              int32_t *parent, void *stream, dobfs_stats *stats);

/* ------------------------------------------------------ multi-source BFS */

/* Device bytes of workspace a dobfs_bfs_batch call with k sources needs
 * (k in [1, 64]): about 168 bytes per vertex for the visited and frontier
 * words (the frontiers of the first 16 levels are kept as their depth
 * record), plus 2*k bytes per vertex for the level table of deeper levels. */
dobfs_status dobfs_bfs_batch_workspace_bytes(dobfs_graph g, int32_t k, size_t *bytes);

/*
 * k breadth-first searches at once (1 <= k <= 64), one per entry of
 * `sources` (host int32[k], each in [0,V); repeats allowed). Algorithm 1
 * with the frontier vector widened to a k-column bit matrix: one level is the
 * masked Boolean matrix product F' = A^T F .* not(Vis) over (OR, AND), in
 * push form (column-based, Equation 5 per column) or pull form (row-based
 * with early exit once every missing source is found, Sections 5.2-5.4),
 * the direction chosen per level for the whole batch by opt's rule applied
 * to the batch's frontier (vertices with any frontier bit) and edge counts.
 * On return depth[b*V + v] is the hop count of a shortest path
 * sources[b] -> v, -1 if unreachable: row b equals what dobfs_bfs from
 * sources[b] returns in `depth`. No parents are produced.
 * depth: device int32[k*V], row-major, required. workspace: device memory
 * of at least dobfs_bfs_batch_workspace_bytes(g, k), 256-byte aligned, or
 * NULL for a library-owned one (shared with the other calls on g and
 * serialised with them). opt: modes FULL, PUSH_ONLY and PULL_ONLY (others
 * -> UNSUPPORTED), both heuristics, forced directions. stats: as for
 * dobfs_bfs, with nf and n_new counting vertices that carry any source bit
 * and `reached` counting (vertex, source) pairs. Blocks until depth is
 * final. Errors: k out of range, a source outside [0,V) or a NULL pointer
 * -> INVALID_ARG with nothing written; a traversal deeper than 65533 levels
 * -> UNSUPPORTED (levels are kept in 16 bits).
 */
dobfs_status dobfs_bfs_batch(dobfs_graph g, const int32_t *sources, int32_t k,
                             const dobfs_options *opt, int32_t *depth, void *workspace,
                             size_t ws_bytes, void *stream, dobfs_stats *stats);

/* --------------------------------------------------------------- serving */

/*
 * A query server over device-resident graphs: single-source BFS queries
 * arrive one at a time (dobfs_server_submit) and are answered by
 * multi-source traversals (dobfs_bfs_batch semantics) that take up to
 * max_batch queued queries of one graph at once, the graph whose oldest
 * query has waited longest first; a batch of one runs dobfs_bfs (depths
 * only, its own smaller workspace). `slots` batches run at the same time,
 * each on a host thread and HIP stream of its own, so queries that arrive
 * while a batch is on the GPU are admitted into the next free slot and run
 * beside it (continuous batching, not a single queue). Graphs whose batches
 * have taken more than 2 ms on average may occupy at most slots - 1 slots at
 * once, so a deep traversal never holds every slot, and their queries are
 * batched only once 8 of them are queued (fewer run one per slot). Admission by memory: the
 * server makes one device allocation of mem_budget bytes when it is created
 * and carves every batch's workspace out of it; a batch starts only when its
 * workspace fits in what the running batches leave free, and a batch is cut
 * down to the number of sources whose workspace fits in the whole budget
 * (queries of a graph for which not even one fits fail with
 * DOBFS_ERR_OUT_OF_MEMORY). Each query's depths are those dobfs_bfs returns
 * for its source (the server runs no other arithmetic). The server owns its
 * memory and streams; graphs stay owned by the caller and must outlive the
 * server. Thread-safe: any thread may submit and wait.
 */
typedef struct dobfs_server_s *dobfs_server;

typedef struct {
  int32_t slots;      /* batches in flight at once, 1..16 (default 4) */
  int32_t max_batch;  /* sources per batch, 1..64 (default 64) */
  size_t mem_budget;  /* device bytes the server allocates for all running batches' workspaces;
                         0 = slots x the largest batch workspace (default 0) */
  dobfs_options opt;  /* traversal options of every batch: modes FULL, PUSH_ONLY, PULL_ONLY */
} dobfs_server_options;

typedef struct {
  int32_t graph, source;
  int32_t batch_size;   /* queries answered by the same traversal */
  int32_t status;       /* dobfs_status of the traversal */
  double t_submit_ms;   /* steady-clock times in ms since the server was created */
  double t_start_ms;    /* the batch was admitted and launched */
  double t_done_ms;     /* depth is final in device memory */
} dobfs_query_info;

/* Defaults: 4 slots, batches of up to 64, no budget beyond the slots, default BFS options. */
dobfs_status dobfs_server_options_default(dobfs_server_options *opt);

/* graphs: host array of n_graphs handles on one device (copied). Allocates
 * the memory pool (mem_budget bytes) and one stream per slot. Errors:
 * INVALID_ARG, OUT_OF_MEMORY, DEVICE, UNSUPPORTED (options). */
dobfs_status dobfs_server_create(const dobfs_graph *graphs, int32_t n_graphs,
                                 const dobfs_server_options *opt, dobfs_server *out);

/* Queue a BFS from `source` on graphs[graph]; `depth` (device int32[V] of that
 * graph, caller-owned) receives the result and must stay valid until the
 * query is done. The slots run on streams of their own (non-blocking, not
 * ordered after any stream of the caller's): work the caller has queued that
 * writes or reads `depth` must be complete before the call, and the result
 * may be read once dobfs_server_wait reports the query done. *id identifies
 * the query. Never blocks on the GPU. */
dobfs_status dobfs_server_submit(dobfs_server s, int32_t graph, int32_t source, int32_t *depth,
                                 uint64_t *id);

/* Wait up to timeout_ms (< 0: no limit) for query `id`; DOBFS_ERR_TIMEOUT if
 * it is still queued or running. On return *info (optional) describes it;
 * the call returns the traversal's status once done. */
dobfs_status dobfs_server_wait(dobfs_server s, uint64_t id, int32_t timeout_ms, dobfs_query_info *info);

/* Answers every query already submitted, then frees the server. */
dobfs_status dobfs_server_destroy(dobfs_server s);

/* -------------------------------------------------------- standalone mxv */

enum {
  DOBFS_MXV_EARLY_EXIT = 1u, /* pull: stop a row at its first hit (Algorithm 2, break) */
  DOBFS_MXV_ACCUM_OR = 2u    /* y = y OR result instead of y = result (Algorithms 2-3, accum) */
};

/* Device bytes of workspace a dobfs_mxv call on g needs. */
dobfs_status dobfs_mxv_workspace_bytes(dobfs_graph g, size_t *bytes);

/*
 * y = (A^T x) .* m over ({0,1}, OR, AND, 0) (Equations 2-5, Section 3.2):
 *   t(i)    = OR over edges j->i of x(j)
 *   pass(i) = mask_bits == NULL ? 1 : (mask(i) XOR complement)
 *   y(i)    = ACCUM_OR ? y(i) OR (t(i) AND pass(i)) : t(i) AND pass(i)
 * The four variants of Section 6.3 / Table 1:
 *   direction PULL, mask NULL : ROW_MXV        (every row)
 *   direction PULL, mask      : ROW_MASKED_MXV (rows that pass only)
 *   direction PUSH, mask NULL : COL_MXV
 *   direction PUSH, mask      : COL_MASKED_MXV (expand, dedupe, then filter)
 * x is given as a device bit vector x_bits, or (x_bits NULL) as a device
 * index list x_idx[0..x_nnz) of distinct vertices; the call converts it to
 * the form its direction reads (dense for pull, sparse for push).
 * EARLY_EXIT applies to pull only (a column-based matvec cannot exit early).
 * Outputs (device): y_bits (required, ceil(V/32) words); y_idx (optional,
 * int32[V]): the set bits of y in ascending order; y_witness (optional,
 * int32[V]): for every i with t(i) AND pass(i), a j with x(j) = 1 and an edge
 * j->i (pull: the first in CSC order); other entries are left unchanged.
 * y_nnz (host, optional): popcount of y; when y_nnz or y_idx is given the
 * call blocks until done, otherwise it only enqueues work on `stream`.
 * Aliasing: x_bits and mask_bits may be the same buffer as y_bits (the
 * in-place BFS form v = v OR A^T v .* not(v) of Section 5.4 with ACCUM_OR):
 * the result is then computed from x and mask as they were before the call.
 * y_idx, y_witness and x_idx must not overlap each other or the bit vectors.
 */
dobfs_status dobfs_mxv(dobfs_graph g, const uint32_t *x_bits, const int32_t *x_idx,
                       int32_t x_nnz, const uint32_t *mask_bits, int32_t complement,
                       int32_t direction, uint32_t flags, uint32_t *y_bits, int32_t *y_idx,
                       int32_t *y_witness, int32_t *y_nnz, void *workspace, size_t ws_bytes,
                       void *stream);

/* ------------------------------------------------------------- errors */

/* Static name of a status code. */
const char *dobfs_status_string(dobfs_status s);

/* Message of the calling thread's last failure ("" if none). */
const char *dobfs_last_error(void);

/* Library version as major*10000 + minor*100 + patch. */
int32_t dobfs_version(void);

#ifdef __cplusplus
}
#endif

#endif /* DOBFS_H */
