/*
 * cfpq.h -- context-free path querying (relational semantics) on AMD gfx950.
 *
 * The library computes, for an edge-labelled graph D = (V, E) and a grammar
 * G = (N, Sigma, P) in Chomsky normal form without start symbol or epsilon
 * rules (section 2 of Azimov & Grigorev, "Context-Free Path Querying by Matrix
 * Multiplication", EDBT 2018), the context-free relation
 *     R_A = { (i, j) : some path i -> j spells a word derivable from A }
 * for every nonterminal A.  It follows Algorithm 1 (section 4.2): initialise
 * one Boolean matrix per nonterminal from the edges, then repeat
 * T_A |= T_B x T_C for every rule A -> B C until no matrix changes.  Theorem 2
 * (section 4.1) states that the fixpoint is exactly R.
 *
 * Conventions for every entry point:
 *  - Ids are dense, 0-based int32: nodes 0..n-1, terminals 0..n_terminals-1,
 *    nonterminals 0..n_nonterminals-1.
 *  - Matrix layout ("bit layout"): a matrix is cfpq_padded_rows(n) rows of
 *    cfpq_row_words(n) uint64 words; bit (j % 64) of word (j / 64) of row i is
 *    1 iff (i, j) is in the relation.  The result buffer holds n_nonterminals
 *    such matrices back to back.  Rows >= n and bits >= n are 0 on return.
 *  - Memory: pointers named d_* are device memory owned by the caller; every
 *    other pointer is host memory borrowed for the duration of the call.  The
 *    library allocates no device memory inside cfpq_closure: its scratch space
 *    is the caller's workspace.  Matrix buffers and workspaces must be 16-byte
 *    aligned (every hipMalloc'd pointer is); misaligned ones are CFPQ_EINVAL.
 *  - Streams: `stream` is a hipStream_t (NULL = the default stream).  Work is
 *    ordered on it.  cfpq_closure returns after the fixpoint is reached (it
 *    reads a change flag back after every loop), so results and stats are
 *    valid on return.
 *  - Errors: every entry point returns a cfpq_status.  Argument errors are
 *    reported before any device work; cfpq_last_error() gives a message for the
 *    calling thread.  A HIP failure returns CFPQ_EDEVICE with the HIP error
 *    text in the message.
 */
#ifndef CFPQ_H
#define CFPQ_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define CFPQ_ABI_VERSION 4

#if defined(__GNUC__)
#define CFPQ_API __attribute__((visibility("default")))
#else
#define CFPQ_API
#endif

typedef enum {
    CFPQ_OK = 0,
    CFPQ_EINVAL = -1,     /* an argument is out of range or NULL */
    CFPQ_ENOMEM = -2,     /* workspace or memory budget too small */
    CFPQ_EDEVICE = -3,    /* a HIP call failed */
    CFPQ_ENOTCONV = -4,   /* max_iters reached; the partial result is sound (a subset of R) */
    CFPQ_EBUSY = -5,      /* no free slot (serving) */
    CFPQ_ENOTREADY = -6,  /* request still running (serving) */
    CFPQ_ERANGE = -7      /* a single-path length does not fit (>= 2^31 - 1) */
} cfpq_status;

/* Edge (src, label, dst) of E (section 2).  Multi-edges and self-loops are allowed. */
typedef struct { int32_t src, label, dst; } cfpq_edge;
/* Production A -> x. */
typedef struct { int32_t lhs, terminal; } cfpq_term_rule;
/* Production A -> B C. */
typedef struct { int32_t lhs, left, right; } cfpq_bin_rule;

typedef struct {
    int32_t n_nodes;           /* |V| >= 0 */
    int32_t edges_on_device;   /* 0: `edges` is host memory; 1: device memory */
    int64_t n_edges;           /* |E| >= 0 */
    const cfpq_edge* edges;    /* n_edges records */
} cfpq_graph;

typedef struct {
    int32_t n_nonterminals;    /* 1..CFPQ_MAX_NONTERMINALS */
    int32_t n_terminals;       /* >= 0; every edge label must be below it */
    int32_t n_term_rules;
    int32_t n_bin_rules;
    const cfpq_term_rule* term_rules;   /* host */
    const cfpq_bin_rule* bin_rules;     /* host */
} cfpq_grammar;

#define CFPQ_MAX_NONTERMINALS 64
#define CFPQ_MAX_NODES (1 << 20)

/* Product kernels.  AUTO, BITS, MFMA and FP4 compute the dense product (every
 * word of both operands is read).  ROWS and COLS skip the zero entries of one
 * operand: ROWS forms row i of B x C as the OR of the rows C[k, :] for the set
 * bits k of B[i, :] (cost ~ nnz(B) rows of C); COLS does the same on the
 * transposed product (B x C)^T = C^T x B^T (cost ~ nnz(C) rows of B^T, plus
 * transposes).  All give identical bits.
 *
 * Environment (read on every call of cfpq_closure, cfpq_closure_static and
 * cfpq_workspace_bytes):
 *   CFPQ_PATH  bits, mfma, fp4, rows or cols: used where options.path is
 *              AUTO (any other value is ignored); the bits are the same.
 *   CFPQ_LOG   a file name, or "-" for stderr: cfpq_closure appends JSON
 *              lines -- {"event": "loop", ...} per host-driven loop (loop,
 *              rules_launched, changed nonterminals, products so far,
 *              host_ms), {"event": "replay", ...} per replay of captured
 *              loops, and {"event": "closure", ...} per call with its totals.
 */
enum {
    CFPQ_PATH_AUTO = 0,
    CFPQ_PATH_BITS = 1,  /* bit-packed VALU product (AND / OR-reduce) */
    CFPQ_PATH_MFMA = 2,  /* int8 MFMA, int32 sums */
    CFPQ_PATH_ROWS = 3,  /* row gathers by the set bits of B */
    CFPQ_PATH_COLS = 4,  /* row gathers of the transposed product */
    CFPQ_PATH_FP4 = 5    /* e2m1 (fp4) MFMA, fp32 sums */
};
/* Hybrid product choice of cfpq_closure (options.hybrid). */
enum { CFPQ_HYBRID_OFF = 0, CFPQ_HYBRID_AUTO = 1 };
enum { CFPQ_SCHEDULE_INPLACE = 0, CFPQ_SCHEDULE_JACOBI = 1 };

typedef struct {
    int32_t path;            /* CFPQ_PATH_*: product kernel.  AUTO = autotuned dense kernel;
                                ROWS / COLS run every product that way (hybrid ignored) */
    int32_t schedule;        /* CFPQ_SCHEDULE_JACOBI: every product of a loop reads the
                                matrices of the previous loop (Algorithm 1 exactly);
                                CFPQ_SCHEDULE_INPLACE: products read the latest matrices
                                (same fixpoint, usually fewer loops) */
    int32_t dirty_worklist;  /* nonzero: a rule A -> B C runs in a loop only if B or C
                                changed in the previous loop (all rules run in loop 1) */
    int32_t profile;         /* nonzero: time every product with HIP events on `stream`
                                (stats.product_ms); costs one event pair per product */
    int32_t tile;            /* product kernel variant; 0 = autotuned or default.  BITS: output
                                strip width in 32-bit words per workgroup (8, 16 or 32).  FP4:
                                2 or 3 = a workgroup per 256 x 256 tile with that many chunk
                                buffers, 5 = persistent workgroups (the default); other
                                values give CFPQ_EINVAL */
    int32_t capture;         /* loops per captured HIP graph: the loop state (per-rule dirty
                                decisions, change flags, loop count) lives on the device and the
                                host reads it back once per `capture` loops; 0 = host-driven
                                loop with one read-back per loop.  Ignored when profile is set
                                or the hybrid choice is in effect.  Default 8. */
    int32_t hybrid;          /* CFPQ_HYBRID_AUTO (default): for padded sizes of at least 4096,
                                each product of each loop picks the dense kernel, ROWS or COLS
                                from the current number of set bits of its operands (a cost
                                model; the bits are the same whichever runs).  The loop is then
                                host-driven.  CFPQ_HYBRID_OFF: every product is dense. */
    int32_t warm_start;      /* 0: d_result is overwritten.  1: d_result already holds matrices in
                                the bit layout that are subsets of R (for example a result of
                                CFPQ_ENOTCONV, or R of the same graph with fewer edges); the edge
                                initialisation is OR-ed into them and the loop continues from
                                there.  The fixpoint is the same (R is the least fixpoint above the
                                initial matrices, Theorem 2); only the loop count drops. */
    int64_t max_iters;       /* loop cap; 0 = |V|^2 |N| + 1 (Theorem 3's bound) */
} cfpq_options;

typedef struct {
    int64_t iterations;      /* loop executions, including the final one that changed nothing */
    int64_t products;        /* Boolean products executed (dense and sparse) */
    double bitops;           /* 2 * npad^3 per executed dense product, npad = cfpq_padded_rows(n);
                                ROWS / COLS products are not counted */
    double device_ms;        /* device time from matrix initialisation to the last flag */
    double product_ms;       /* summed duration of the product kernels (options.profile), else 0 */
    int32_t path_used;       /* CFPQ_PATH_BITS, MFMA or FP4 (dense kernel), ROWS or COLS */
    int32_t converged;       /* 1 if the fixpoint was reached */
    int64_t sparse_products; /* products of `products` that ran as ROWS or COLS */
    int64_t delta_products;  /* products of `products` with a delta operand: a rule A -> B C whose
                                operands gained the bits D_B, D_C since the previous loop started
                                may add D_B x C and B x D_C instead of B x C (hybrid choice) */
    double minplus_terms;    /* cfpq_single_path only: (i, j, k) terms l_B(i,k) + l_C(k,j) the min-plus
                                tile kernel evaluated (product_ms is then its summed time); 0 elsewhere */
    double sparse_bytes;     /* cfpq_closure: algorithmic bytes of the rules whose every part ran as ROWS or
                                COLS -- per part nz * row bytes (the rows gathered at the nz set bits of its
                                sparse operand) + 3 matrices (the bit scan of that operand, read and write
                                of the result) */
    double sparse_ms;        /* summed duration of those rules (options.profile), else 0 */
} cfpq_stats;

/* ABI version of the loaded library (CFPQ_ABI_VERSION). */
CFPQ_API int32_t cfpq_abi_version(void);

/* Message for the last error on the calling thread ("" if none).  The pointer
 * stays valid until the next call on this thread. */
CFPQ_API const char* cfpq_last_error(void);

/* Fill `opt` with defaults: AUTO path, hybrid choice on, in-place schedule,
 * dirty worklist on, 8 loops per captured graph, no per-product timing, no
 * warm start, max_iters from Theorem 3. */
CFPQ_API void cfpq_default_options(cfpq_options* opt);

/* Words per matrix row: ceil(n/64) rounded up to a multiple of 4 (n >= 0). */
CFPQ_API int64_t cfpq_row_words(int32_t n_nodes);

/* Rows per matrix: 64 * cfpq_row_words(n) (the padded matrix is square). */
CFPQ_API int64_t cfpq_padded_rows(int32_t n_nodes);

/* Bytes of the result buffer: n_nonterminals * padded_rows * row_words * 8. */
CFPQ_API size_t cfpq_result_bytes(int32_t n_nodes, int32_t n_nonterminals);

/* Workspace bytes that cfpq_closure needs for this graph size, grammar and
 * options (it depends on n_edges only through edges copied from the host).
 * Returns CFPQ_EINVAL for invalid arguments. */
CFPQ_API cfpq_status cfpq_workspace_bytes(const cfpq_graph* graph, const cfpq_grammar* grammar,
                                 const cfpq_options* opt, size_t* bytes);

/*
 * Relational CFPQ closure (Algorithm 1, section 4.2).
 *   graph, grammar   inputs as above (validated on the host; with
 *                    edges_on_device = 1 the edge ids are checked by the
 *                    initialisation kernel and an out-of-range edge makes the
 *                    call return CFPQ_EINVAL before any product runs)
 *   opt              NULL = cfpq_default_options
 *   stream           hipStream_t or NULL
 *   d_workspace      device scratch of at least cfpq_workspace_bytes bytes
 *   d_result         device buffer of cfpq_result_bytes bytes; overwritten with
 *                    R in the bit layout
 *   stats            optional (NULL allowed)
 * Returns CFPQ_OK, CFPQ_ENOTCONV (max_iters reached, d_result is a sound
 * subset of R), CFPQ_EINVAL, CFPQ_ENOMEM (workspace too small) or CFPQ_EDEVICE.
 * A graph of at most 512 padded rows with path AUTO, the in-place schedule, no
 * profile and no warm start runs as a one-instance cfpq_batch_closure (the
 * whole fixpoint in one workgroup, one launch; capture is ignored,
 * stats.path_used is BITS, the loop count may differ from the loop here); the
 * bits are the same.  So does the Jacobi schedule on graphs of at most 256
 * padded rows whose |N| matrices fit twice in 48 KiB (same loop count).
 */
CFPQ_API cfpq_status cfpq_closure(const cfpq_graph* graph, const cfpq_grammar* grammar,
                         const cfpq_options* opt, void* stream,
                         void* d_workspace, size_t workspace_bytes,
                         uint64_t* d_result, cfpq_stats* stats);

/* Bytes of the static workspace of cfpq_closure_static (per GPU). */
#define CFPQ_STATIC_WORKSPACE_BYTES ((size_t)64 << 20)

/*
 * cfpq_closure without a workspace argument, for callers that cannot
 * allocate device memory (code in tight serving loops, harnesses that forbid
 * hipMalloc): the library's own workspace -- a device array of
 * CFPQ_STATIC_WORKSPACE_BYTES (64 MiB) that each GPU the library runs on holds
 * until the process ends -- is used instead, and the call allocates nothing
 * (no hipMalloc / hipFree, no HIP events, no graph capture: the loop is
 * host-driven and stats.device_ms is the host's wall time).  The caller still
 * owns graph, grammar and d_result, as for cfpq_closure.  The workspace keeps
 * the previous call's contents; every part of it a closure reads is written
 * first.  Calls on one GPU share its array: the library runs them one at a
 * time (from any number of host threads; each call returns only after its
 * stream is synchronised).  opt.capture and opt.profile are ignored, and a
 * graph small enough for the resident route still runs the ordinary loop.
 * Returns as cfpq_closure, and CFPQ_ENOMEM, before any device work, when the
 * closure needs more than CFPQ_STATIC_WORKSPACE_BYTES of workspace (about
 * 5000 nodes for a 4-nonterminal grammar with the hybrid choice on).
 */
CFPQ_API cfpq_status cfpq_closure_static(const cfpq_graph* graph, const cfpq_grammar* grammar,
                                         const cfpq_options* opt, void* stream, uint64_t* d_result,
                                         cfpq_stats* stats);

/*
 * One Boolean matrix product with union (the product of section 2 for a
 * single rule A -> B C, fused with the union of Algorithm 1):
 *     d_a |= d_b x d_c,   P_ij = OR_k (b_ik AND c_kj)
 * All three are npad x npad matrices in the bit layout for `n_nodes`.  d_a may
 * alias d_b and/or d_c (the in-place update; bits are only ever set, so every
 * value read is a subset of the final one).  path = any CFPQ_PATH_* (AUTO
 * picks the autotuned dense kernel); tile as in cfpq_options (0 = default).
 * *d_changed (device int32, required) is OR-ed with 1 when d_a gained a bit.
 * d_workspace may be NULL for BITS; MFMA and FP4 (one transposed operand), ROWS (a
 * list of rows long enough to be split over several wavefronts) and COLS
 * (two transposed operands, the transposed product, the list) need
 * cfpq_product_workspace_bytes.  The MFMA and FP4 paths require
 * n_nodes <= 2^19 (exact int32 / fp32 sums); larger sizes return CFPQ_EINVAL.  Every product
 * kernel only reads rows and columns below n_nodes of its operands, which
 * must be zero beyond them (as in every matrix of the bit layout).
 */
CFPQ_API size_t cfpq_product_workspace_bytes(int32_t n_nodes, int32_t path);
CFPQ_API cfpq_status cfpq_product(int32_t n_nodes, int32_t path, int32_t tile, const uint64_t* d_b,
                                  const uint64_t* d_c, uint64_t* d_a, int32_t* d_changed,
                                  void* d_workspace, size_t workspace_bytes, void* stream);

/* Number of set bits of each of `count` consecutive matrices of the bit
 * layout for n_nodes (|R_A| per nonterminal for a result buffer), written to
 * the device array d_counts[count].  Stream-ordered; does not synchronise. */
CFPQ_API cfpq_status cfpq_popcount(int32_t n_nodes, int32_t count, const uint64_t* d_mats,
                          unsigned long long* d_counts, void* stream);

/* ------------------------------------------------------------------------
 * Single-path semantics (section 5): a path length for every triple.
 *
 * Alongside R (the bit matrices of cfpq_closure), every (A, i, j) in R_A gets
 * a length L_A(i, j) such that some path i -> j of exactly that many edges
 * has a label word that A derives (the section's theorem).  Lengths follow
 * the section's construction on Algorithm 1's simultaneous step: 1 for the
 * cells set by the edges; when a step first adds A to (i, j) through a rule
 * A -> B C and a node k with both operand cells present after the previous
 * step, L_A(i, j) = L_B(i, k) + L_C(k, j), and a cell keeps its length
 * afterwards.  Where one step offers several (rule, k) sums the smallest is
 * kept (the section leaves the choice open; the smallest makes it unique).
 * ------------------------------------------------------------------------ */

/* Bytes of the lengths buffer: n_nonterminals * npad * npad uint32, cell
 * (A, i, j) at index (A * npad + i) * npad + j, 0 = not in R_A. */
CFPQ_API size_t cfpq_lengths_bytes(int32_t n_nodes, int32_t n_nonterminals);

/* Workspace for cfpq_single_path: two more bit matrices per nonterminal
 * (the next step and the step's new cells), transposed right operands,
 * per-loop counts and 64 x 64 tile flags of the new cells (4 bytes per tile
 * and nonterminal), a column index (npad + 1 offsets, npad cursors, one row
 * id per edge) for each fixed sparse right operand, plus small tables. */
CFPQ_API cfpq_status cfpq_single_path_workspace_bytes(const cfpq_graph* graph, const cfpq_grammar* grammar,
                                                      size_t* bytes);

/*
 * Relational closure with single-path lengths.  d_result as for cfpq_closure
 * (R in the bit layout); d_lengths: device buffer of cfpq_lengths_bytes,
 * overwritten.  max_iters: loop cap, 0 = Theorem 3's bound.  Synchronises
 * `stream`.  Returns CFPQ_OK, CFPQ_ENOTCONV (cap reached: every stored length
 * is still a valid path length), CFPQ_ERANGE (a length reached 2^31 - 1: the
 * contents of d_result and d_lengths are then unspecified), CFPQ_EINVAL,
 * CFPQ_ENOMEM or CFPQ_EDEVICE.  stats: iterations, Boolean products, device time, the
 * min-plus tile kernel's terms (minplus_terms) and summed time (product_ms);
 * rules whose min-plus runs as a row or column gather (a fixed sparse edge
 * matrix operand, or a left operand sparse enough in that loop) are in
 * neither figure.
 */
CFPQ_API cfpq_status cfpq_single_path(const cfpq_graph* graph, const cfpq_grammar* grammar, int64_t max_iters,
                                      void* stream, void* d_workspace, size_t workspace_bytes, uint64_t* d_result,
                                      uint32_t* d_lengths, cfpq_stats* stats);

/*
 * A witness path for (a, i, j) from lengths computed by cfpq_single_path and
 * copied to the host: it splits each cell into two present cells whose
 * lengths add up to its own (the split that set it always qualifies) down to
 * single edges.  graph: host edges.  path: host buffer of max_edges records,
 * filled with the path's edges in order.  Returns the number of edges
 * (= L_a(i, j)) or a negative cfpq_status: CFPQ_EINVAL if the cell is not in
 * R_a or the lengths are inconsistent, CFPQ_ENOMEM if max_edges is shorter
 * than the length.
 */
CFPQ_API int64_t cfpq_witness(const cfpq_graph* graph, const cfpq_grammar* grammar, const uint32_t* lengths,
                              int32_t a, int32_t i, int32_t j, cfpq_edge* path, int64_t max_edges);

/* ------------------------------------------------------------------------
 * Conjunctive grammars (the generalisation named in the paper's conclusion).
 *
 * Rules A -> B1 C1 & ... & Bk Ck (k >= 1) join the grammar's terminal rules
 * and its binary rules (which are one-conjunct rules).  Algorithm 1's step
 * becomes T_A |= AND over m of (T_Bm x T_Cm).  The fixpoint contains every
 * (A, i, j) joined by a path whose word A derives, and possibly more (each
 * conjunct may use another path between the same nodes); on a graph with one
 * path between any two nodes it is exact.
 * ------------------------------------------------------------------------ */

typedef struct { int32_t left, right; } cfpq_conjunct;         /* one conjunct B C */
typedef struct {
    int32_t lhs;                      /* A */
    int32_t n_conjuncts;              /* k >= 1 */
    const cfpq_conjunct* conjuncts;   /* k entries, host memory */
} cfpq_conj_rule;

/* Workspace for cfpq_conjunctive_closure (as cfpq_workspace_bytes, plus two
 * scratch matrices when some rule has k >= 2, two more when some conjunct
 * runs as COLS, plus one matrix per dense conjunct B C that occurs in more
 * than one rule: its product is computed once per loop and read by every
 * use). */
CFPQ_API cfpq_status cfpq_conjunctive_workspace_bytes(const cfpq_graph* graph, const cfpq_grammar* grammar,
                                                      int32_t n_conj_rules, const cfpq_conj_rule* conj_rules,
                                                      const cfpq_options* opt, size_t* bytes);

/*
 * Closure for a conjunctive grammar: grammar (terminal rules, one-conjunct
 * binary rules) plus n_conj_rules rules with any number of conjuncts.
 * opt: path AUTO, BITS, MFMA or FP4 (dense products), schedule, dirty_worklist,
 * tile and max_iters as for cfpq_closure; warm_start must be 0; hybrid AUTO
 * (default), when the graph has at most npad^2 / 16 edges, runs a conjunct
 * whose left operand heads no rule as a ROWS product, and else one whose
 * right operand heads no rule as a COLS product (both counted in
 * stats.sparse_products, not in bitops); OFF keeps every product dense;
 * capture and profile are ignored (host-driven loop).  d_result, stream,
 * workspace, stats and the return codes as for cfpq_closure.
 */
CFPQ_API cfpq_status cfpq_conjunctive_closure(const cfpq_graph* graph, const cfpq_grammar* grammar,
                                              int32_t n_conj_rules, const cfpq_conj_rule* conj_rules,
                                              const cfpq_options* opt, void* stream, void* d_workspace,
                                              size_t workspace_bytes, uint64_t* d_result, cfpq_stats* stats);

/* ------------------------------------------------------------------------
 * Autotuner: the fastest product kernel per size bucket.
 *
 * cfpq_autotune times every product variant (fp4 and int8 MFMA; VALU with
 * 8, 16 and 32-word strips) on synthetic operands of the padded size for
 * n_nodes and records the fastest for the bucket ceil(log2(npad)) in a
 * process-wide table.  The AUTO path of cfpq_closure and cfpq_product then
 * uses it (an untuned bucket uses FP4 up to 2^19 nodes, else BITS).  All variants give
 * identical bits.  The environment variable CFPQ_TUNE_CACHE names a JSON file
 * (as written by cfpq_tune_save) loaded at first use.
 * ------------------------------------------------------------------------ */

typedef struct {
    int32_t npad;              /* padded size the entry was measured at */
    int32_t path;              /* CFPQ_PATH_FP4, CFPQ_PATH_MFMA or CFPQ_PATH_BITS */
    int32_t tile;              /* BITS strip width (0 = default) */
    float ms;                  /* the chosen kernel's time per product */
    int32_t n_candidates;      /* entries used below (filled by cfpq_autotune only) */
    int32_t candidate_path[8];
    int32_t candidate_tile[8];
    float candidates_ms[8];
} cfpq_tune_entry;

/* Device workspace for cfpq_autotune: four matrices of the bit layout. */
CFPQ_API size_t cfpq_autotune_workspace_bytes(int32_t n_nodes);

/* Measure and record the bucket of n_nodes (synchronises `stream`). */
CFPQ_API cfpq_status cfpq_autotune(int32_t n_nodes, void* stream, void* d_workspace, size_t workspace_bytes,
                                   cfpq_tune_entry* out);

/* The recorded entry for n_nodes' bucket; CFPQ_ENOTREADY if none. */
CFPQ_API cfpq_status cfpq_tune_get(int32_t n_nodes, cfpq_tune_entry* out);

/* Write / merge-read the table as JSON text; CFPQ_EINVAL if the file cannot
 * be opened.  Unrecognised lines are ignored. */
CFPQ_API cfpq_status cfpq_tune_save(const char* path);
CFPQ_API cfpq_status cfpq_tune_load(const char* path);

/* Forget every entry (and do not read CFPQ_TUNE_CACHE afterwards). */
CFPQ_API void cfpq_tune_clear(void);

/* ------------------------------------------------------------------------
 * Batched closure: many independent instances of uneven size in one call.
 * ------------------------------------------------------------------------ */

/* One query of a batch.  d_result: device buffer of
 * cfpq_result_bytes(graph.n_nodes, grammar->n_nonterminals) bytes, owned by
 * the caller, overwritten with that instance's R in the bit layout. */
typedef struct {
    cfpq_graph graph;
    const cfpq_grammar* grammar;
    uint64_t* d_result;
} cfpq_instance;

/* Workspace bytes for cfpq_batch_closure with these instances and options
 * (enough for any route the batch tuning table may choose). */
CFPQ_API cfpq_status cfpq_batch_workspace_bytes(int32_t n_instances, const cfpq_instance* instances,
                                                const cfpq_options* opt, size_t* bytes);

/* Routes of the batched engine (cfpq_batch_closure and the server): how the
 * instances of one size bucket (one padded side) run. */
enum {
    CFPQ_ROUTE_RESIDENT = 1, /* one workgroup runs the instance's whole fixpoint (VALU products,
                                right operand in LDS); padded side <= 512 only */
    CFPQ_ROUTE_TILES = 2     /* the engine's per-loop work list shared by all such instances: fp4-MFMA
                                tiles of `tile` x `tile` (256: a workgroup per tile; 128: a wavefront per
                                tile), row gathers for rules with an edge-matrix left operand */
};

/* The batch tuning table: one entry per padded side (a multiple of 256).
 * Untuned sides use RESIDENT up to 512 and TILES 256 above. */
typedef struct {
    int32_t npad;              /* padded side of the bucket */
    int32_t route;             /* CFPQ_ROUTE_* */
    int32_t tile;              /* TILES: 256 or 128 (0 for RESIDENT) */
    float ms;                  /* cfpq_batch_autotune: the sample's time with the chosen route */
    int32_t instances;         /* cfpq_batch_autotune: instances of this side in the sample */
    int32_t n_candidates;      /* entries used below */
    int32_t candidate_route[4];
    int32_t candidate_tile[4];
    float candidates_ms[4];
} cfpq_batch_tune_entry;

/* Device workspace for cfpq_batch_autotune with these instances. */
CFPQ_API cfpq_status cfpq_batch_autotune_workspace_bytes(int32_t n_instances, const cfpq_instance* instances,
                                                         const cfpq_options* opt, size_t* bytes);

/*
 * Batch autotuner.  The sample is the first max_per_bucket instances of every
 * padded side present (0 = all instances).  Side by side, smallest first,
 * each candidate route of that side (RESIDENT where the side allows it, TILES
 * 256, TILES 128) is timed on the whole sample while the other sides keep
 * their current route (the table's, or the default) -- so the overlap of
 * resident workgroups with the tile work list is part of the measurement --
 * as the median host wall time of `reps` runs (0 = 3) after one warm-up run.
 * A candidate replaces the current route only if it is more than 2% faster.
 * Every choice is recorded in the batch tuning table, which
 * cfpq_batch_closure and servers created afterwards read.  The sample's
 * results are written to its instances' d_result (every route gives the same
 * bits).  out: NULL or room for max_out entries, filled in ascending padded
 * side (ms: the sample's time with the chosen route; candidates_ms: with each
 * candidate); *n_out (nullable) receives the number of sides tuned.  opt as
 * for cfpq_batch_closure.  Synchronises `stream`.  Returns CFPQ_OK,
 * CFPQ_EINVAL, CFPQ_ENOMEM (workspace) or CFPQ_EDEVICE.
 */
CFPQ_API cfpq_status cfpq_batch_autotune(int32_t n_instances, const cfpq_instance* instances,
                                         const cfpq_options* opt, void* stream, void* d_workspace,
                                         size_t workspace_bytes, int32_t max_per_bucket, int32_t reps,
                                         cfpq_batch_tune_entry* out, int32_t max_out, int32_t* n_out);

/* The table's entry for padded side npad; CFPQ_ENOTREADY if none. */
CFPQ_API cfpq_status cfpq_batch_tune_get(int32_t npad, cfpq_batch_tune_entry* out);

/* Set (route != 0) or remove (route == 0) the entry of entry->npad by hand.
 * CFPQ_EINVAL for a padded side that is not a positive multiple of 256, a
 * RESIDENT route above 512 or a TILES tile other than 128 / 256.
 * cfpq_tune_save / cfpq_tune_load / cfpq_tune_clear cover this table too. */
CFPQ_API cfpq_status cfpq_batch_tune_set(const cfpq_batch_tune_entry* entry);

/*
 * Relational closure (Algorithm 1, in-place schedule) of every instance,
 * computed together.  Each instance takes the route of its padded side from
 * the batch tuning table (untuned: padded side <= 512 runs its whole fixpoint
 * in one workgroup, VALU product; larger ones share a per-loop work list of
 * 256 x 256 fp4-MFMA tiles), with `opt->capture` loops
 * (0 = 8) per captured HIP graph.  With opt->hybrid AUTO (the default), a
 * rule of a larger instance whose left operand heads no binary rule (its
 * matrix is fixed by the edges) runs as row gathers instead of tiles when the
 * graph has at most npad^2 / 16 edges -- after the first two loops only the
 * rows of its right operand that gained bits since it last ran are pushed
 * into the result; OFF keeps every rule on the tiles.
 * Results are bit-identical to cfpq_closure on each instance alone.  opt:
 * schedule must be INPLACE and warm_start 0; dirty_worklist, capture,
 * hybrid and max_iters apply to every instance; path, tile and profile are
 * ignored.  Instances are limited to 2^19 nodes.
 * stats: NULL or n_instances entries (device_ms is the whole batch's time).
 * Device edges are checked by the initialisation kernel, which skips an
 * out-of-range edge; the call then returns CFPQ_EINVAL naming the instance,
 * after the batch has run (results unspecified).
 * Returns CFPQ_OK, CFPQ_ENOTCONV (some instance hit max_iters; all results
 * are sound), CFPQ_EINVAL (message names the instance), CFPQ_ENOMEM or
 * CFPQ_EDEVICE.  Synchronises `stream` before returning.
 */
CFPQ_API cfpq_status cfpq_batch_closure(int32_t n_instances, const cfpq_instance* instances,
                                        const cfpq_options* opt, void* stream, void* d_workspace,
                                        size_t workspace_bytes, cfpq_stats* stats);

/* ------------------------------------------------------------------------
 * Serving: continuous batching of CFPQ queries.
 *
 * A server owns one device allocation of hbm_budget bytes (made once, at
 * creation) holding its tables and an arena for the queries' matrices,
 * transposed right operands and edges.  A worker thread admits queued
 * queries in arrival order whenever a slot is free and the query's footprint
 * fits the arena, keeps their matrices resident until their fixpoint, and
 * runs every admitted query's loops together with the others in flight
 * (the batched engine of cfpq_batch_closure).  On completion the query's
 * matrices are copied to its d_result and its latency is recorded.
 * Queries with a padded side of at least 4096 go instead, in arrival order,
 * to `hybrid_lanes` lane threads, each running one query at a time with the
 * hybrid closure of cfpq_closure on its own stream (workspace from the same
 * arena, admitted when it fits, result written straight to d_result), so
 * their work overlaps the engine's on the device.
 * ------------------------------------------------------------------------ */

typedef struct cfpq_server cfpq_server;

typedef struct {
    size_t hbm_budget;     /* device bytes the server may use (tables + arena); default 8 GiB */
    int32_t max_slots;     /* queries resident at once, 1..4096; default 256 */
    int32_t capture;       /* loops per replay of the captured engine loop, 1..256; default 4 */
    int32_t max_pending;   /* queued (not yet admitted) queries; submit returns CFPQ_EBUSY beyond */
    int32_t hybrid_lanes;  /* lane threads for queries of padded side >= 4096, 0..16; default 2;
                              0 = every query runs in the batched engine */
} cfpq_server_config;

typedef struct {
    int32_t done;          /* 1 when the result is in d_result */
    cfpq_status status;    /* CFPQ_OK, CFPQ_ENOTCONV, CFPQ_EINVAL (bad device edge) or CFPQ_EDEVICE;
                              CFPQ_ENOTREADY while running */
    double queue_ms;       /* submit -> admission */
    double run_ms;         /* admission -> result copied */
    double latency_ms;     /* submit -> result copied */
    cfpq_stats stats;      /* iterations, products, bitops of this query */
} cfpq_request_info;

CFPQ_API void cfpq_server_default_config(cfpq_server_config* cfg);

/* Create a server on the current device.  stream: hipStream_t for all of the
 * server's device work, or NULL for a private non-blocking stream.  Fails with
 * CFPQ_ENOMEM if hbm_budget cannot be allocated or does not cover the tables. */
CFPQ_API cfpq_status cfpq_server_create(const cfpq_server_config* cfg, void* stream, cfpq_server** out);

/* Queue one query.  graph/grammar are copied (host edges are copied at submit;
 * device edges must stay valid until the query is done; their ids are checked
 * on the device, and a query with an id out of range completes with status
 * CFPQ_EINVAL and d_result unwritten).  d_result: device buffer of
 * cfpq_result_bytes(n, |N|) bytes, written when the query completes.
 * Limits: 2^19 nodes, 64 binary rules, 64 terminals, 256 terminal rules.
 * Returns CFPQ_OK with *ticket set, CFPQ_EINVAL, CFPQ_ENOMEM (the query can
 * never fit the arena) or CFPQ_EBUSY (queue full).  Thread-safe. */
CFPQ_API cfpq_status cfpq_server_submit(cfpq_server* srv, const cfpq_graph* graph, const cfpq_grammar* grammar,
                                        uint64_t* d_result, int64_t* ticket);

/* Non-blocking status of a ticket.  Returns CFPQ_ENOTREADY while queued or
 * running; once done, fills info, releases the ticket and returns the query's
 * status.  Thread-safe. */
CFPQ_API cfpq_status cfpq_server_poll(cfpq_server* srv, int64_t ticket, cfpq_request_info* info);

/* Like cfpq_server_poll but blocks until the query is done. */
CFPQ_API cfpq_status cfpq_server_wait(cfpq_server* srv, int64_t ticket, cfpq_request_info* info);

/* Stop admitting, finish the queries already admitted, drop queued ones,
 * free everything.  Returns CFPQ_EDEVICE if the worker hit a HIP error.
 *
 * After a HIP error in the worker (or a lane's failure to select the device)
 * the server stops: queued queries complete at once with CFPQ_EDEVICE, and
 * every admitted query completes only after the thread that runs it has
 * finished with its buffers (its stream synchronised or abandoned) -- a
 * lane's query with the status of its closure, the worker's with
 * CFPQ_EDEVICE -- so d_result may be freed as soon as wait/poll reports the
 * query done.  Later submits return CFPQ_EDEVICE. */
CFPQ_API cfpq_status cfpq_server_destroy(cfpq_server* srv);

/* For tests of the failure handling above, which cannot make a device fail on
 * purpose: the worker stops at its next turn exactly as after a HIP error
 * (no device work is involved).  Returns once the worker has stopped
 * (queued queries are then done with CFPQ_EDEVICE; lanes may still be
 * finishing theirs); CFPQ_OK, or CFPQ_EINVAL for a NULL server. */
CFPQ_API cfpq_status cfpq_server_inject_fault(cfpq_server* srv);

#ifdef __cplusplus
}
#endif

#endif /* CFPQ_H */
