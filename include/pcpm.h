/*
 * pcpm.h -- C ABI of libpcpm: Partition-Centric Processing (PCPM) PageRank
 * on one AMD Instinct MI355X (gfx950).
 *
 * Method: Lakhotia, Kannan, Prasanna, "Accelerating PageRank using
 * Partition-Centric Processing" (arXiv 1709.07122).  Section references
 * below are to that paper.
 *
 * Conventions for every entry point
 *   - Pointers are HIP device pointers owned by the caller unless marked
 *     (host).  Inputs are never modified.
 *   - `stream` is a hipStream_t passed as void*; NULL is the null stream.
 *     All device work of a call is ordered on that stream.
 *   - Every call returns a pcpm_status_t and never aborts the process.  On an
 *     error the outputs are undefined, except PCPM_ERR_NOT_CONVERGED, which
 *     leaves valid ranks, iteration count and residual.  pcpm_last_error()
 *     returns a message for the calling thread's last failure.
 *   - A graph is a directed CSR: row_off[n+1] (int32, row_off[0] = 0,
 *     row_off[n] = m, non-decreasing) and col[m] (int32), every row sorted
 *     strictly ascending (no duplicate edges), no self-loops.  n < 2^31 because
 *     the top bit of a destination ID is reserved as the message flag
 *     (Sec. 3.2), and m < 2^31.
 *   - A handle may be used by one stream at a time; calls on one handle that
 *     overlap in time race on its scratch buffers.
 *   - Ranks are FP32; the L1 residual and the dangling mass are accumulated
 *     in FP64 on the device.  The gather adds the FP32 updates of a node
 *     exactly (64-bit fixed point), so ranks are reproducible run to run.
 */
#ifndef PCPM_H
#define PCPM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  PCPM_OK = 0,
  PCPM_ERR_INVALID_ARG = 1,  /* bad size, pointer, q, d, tol or iteration cap  */
  PCPM_ERR_GRAPH = 2,        /* CSR breaks the conventions above             */
  PCPM_ERR_OVERFLOW = 3,     /* n or m >= 2^31                               */
  PCPM_ERR_OOM = 4,          /* device allocation failed                     */
  PCPM_ERR_DEVICE = 5,       /* HIP runtime or launch failure                */
  PCPM_ERR_NOT_CONVERGED = 6,/* max_iters reached above tol (outputs valid)  */
  PCPM_ERR_NUMERIC = 7       /* residual or dangling mass became non-finite   */
} pcpm_status_t;

typedef struct pcpm_png* pcpm_png_t;

/* Build options.  Zero-initialise and set what you need. */
typedef struct {
  int32_t part_log2;     /* q = 2^part_log2 nodes per partition (Sec. 3.1),
                            1..14 (the gather keeps an 8-byte exact sum per
                            node of a partition in the LDS of one compute
                            unit) with k = ceil(n/q) <= 16384;
                            0 = autotune: the measured sweep of Sec. 5.3.2
                            (Figs. 11-14) on this GPU -- every candidate q
                            (tune_log2_mask) and update order is built and
                            timed over a few iterations, then the work-item
                            chunks of the fastest are varied and timed; the
                            fastest configuration is built and returned, and
                            remembered for the process (keyed by the graph's
                            content, the options and the device), so a
                            later build of the same graph skips the sweep.
                            pcpm_tune_table gives the measurements.         */
  int32_t num_graphs;    /* 0 or 1: one graph.  G > 1: the CSR is the block-
                            diagonal union of G graphs; graph g owns nodes
                            [graph_node_off[g], graph_node_off[g] +
                            graph_nodes[g]); every graph_node_off[g] is a
                            multiple of q (partitions never straddle graphs),
                            graph_node_off[G] = n, nodes between a graph's
                            last node and the next offset are padding without
                            edges, and no edge leaves its graph.  Each graph
                            gets its own uniform jump, dangling spread,
                            residual and convergence.                        */
  const int64_t* graph_node_off; /* (host) G+1, required when G > 1          */
  const int64_t* graph_nodes;    /* (host) G, required when G > 1            */
  int64_t scatter_chunk; /* PNG edges per scatter work item; 0 = automatic   */
  int64_t gather_chunk;  /* destination IDs per gather work item; 0 = auto   */
  int64_t build_chunk;   /* CSR edges per count/fill work item of the build;
                            0 = automatic (about m / max(k, 4096), >= 16384)  */
  const float* weights;  /* (device) m edge weights in CSR order (weights[e]
                            belongs to the edge row -> col[e]), finite, any
                            sign; NULL = unweighted.  Stored next to the
                            destination IDs in bin order (Sec. 3.5) and read
                            by pcpm_spmv only: PageRank always scales by
                            1/outdeg.  The caller keeps ownership.           */
  int64_t update_order;  /* storage order of the updates: 1 = bin order (the
                            bins of Sec. 3.1: the scatter writes one run per
                            (pair, bin) segment, the gather reads its bin in
                            sequence), 2 = PNG order (update e belongs to PNG
                            edge e: sequential scatter writes, the gather
                            reads one run per segment), 0 = automatic: PNG
                            order when the average non-empty segment holds
                            fewer than 360 updates.  Results are identical.
                            Under autotune, 0 times both orders.             */
  int64_t tune_vectors;  /* autotune objective: 0 or 1 = time per PageRank
                            iteration; v > 1 = time per vector-iteration of
                            pcpm_ppr_batch with min(v, tile width) vectors
                            (the tile width follows from q)                 */
  int64_t tune_log2_mask;/* autotune candidates: bit s set = try q = 2^s
                            (1 <= s <= 14); 0 = q in {2^12, 2^13, 2^14}.
                            Candidates with k > 16384, or that a graph
                            offset of a batch is not a multiple of, are
                            skipped.  Caller-set scatter_chunk and
                            gather_chunk are kept; 0 lets the sweep vary
                            them (the automatic value, half, double).        */
  int64_t num_cols;      /* generic SpMV (Sec. 3.5): the CSR is the n x
                            num_cols matrix A (rows 0..n-1, columns in
                            [0, num_cols)); the scatter runs over row
                            partitions and the gather over column partitions,
                            both of q rows / columns.  0 = num_cols = n.     */
  int64_t allow_diagonal;/* 1: keep entries A[i][i] (rejected as self-loops
                            otherwise).  A handle with allow_diagonal = 1 or
                            num_cols != n holds a matrix: only pcpm_spmv,
                            pcpm_png_info, pcpm_png_export_weights and
                            pcpm_png_free take it (PCPM_ERR_INVALID_ARG from
                            the PageRank calls); it cannot hold several
                            graphs.                                          */
} pcpm_build_opts_t;

typedef struct {
  int64_t n, m;          /* nodes (padding included), edges                   */
  int64_t q, k;          /* partition size and count, k = ceil(n/q)           */
  int64_t eprime;        /* |E'|: PNG edges = updates per iteration (Sec. 3.3) */
  int64_t nseg;          /* non-empty (source, destination) partition pairs   */
  int64_t n_dangling;    /* nodes without out-edges                           */
  int64_t scatter_items; /* scatter work items                                */
  int64_t gather_items;  /* gather work items                                 */
  int64_t split_bins;    /* destination bins gathered by more than one item   */
  int64_t device_bytes;  /* device memory held by the handle                  */
  int64_t num_graphs;    /* G (1 for a single graph)                          */
  double build_ms;       /* wall time of pcpm_build_png, device work included */
  int64_t weighted;      /* 1 if the build was given edge weights             */
  int64_t update_order;  /* 1 = bin order, 2 = PNG order (see the build opts) */
  int64_t num_cols;      /* columns of a matrix handle (n for a graph)        */
  int64_t matrix;        /* 1 for a matrix handle (SpMV only)                 */
} pcpm_png_info_t;

/*
 * Pre-processing (Sec. 3.1 partitioning and write offsets, Sec. 3.3 PNG
 * construction): partitions P_i = [i*q, (i+1)*q); for every source partition
 * p and destination partition p' the list U(p,p') of nodes of p with an
 * out-edge into p' (one update per node and destination partition,
 * Sec. 3.2), the update-bin write offsets ordered by source partition ID,
 * and the destination-ID bins with the top bit set on the first ID of each
 * message.  Validates the CSR (PCPM_ERR_GRAPH) and keeps every buffer the
 * iterations need, so the iteration calls allocate nothing.
 * Synchronises `stream`.  *out receives a handle owning its device memory.
 */
pcpm_status_t pcpm_build_png(int64_t n, int64_t m, const int32_t* row_off, const int32_t* col,
                             const pcpm_build_opts_t* opts /* (host) nullable */, void* stream,
                             pcpm_png_t* out /* (host) */);

/* Sizes and statistics of a built handle (host struct). */
pcpm_status_t pcpm_png_info(pcpm_png_t g, pcpm_png_info_t* out /* (host) */);

/*
 * Copy the layout to host arrays in its canonical form (any pointer may be
 * NULL to skip that array); all arrays are (host):
 *   png_off[k][k+1]  per source partition p: sum over p'' < j of |U(p,p'')|
 *   png_src[E']      U(p,p') concatenated over p, then p' (node IDs, no flag)
 *   upd_start[k+1]   first update slot of each destination bin
 *   wo[k][k]         write offset of partition p into bin p' (Sec. 3.1):
 *                    sum over p'' < p of |U(p'',p')|
 *   did_start[k+1]   first destination-ID position of each bin
 *   did[m]           destination IDs in bin order, top bit = first of message
 * Synchronises the device.
 */
pcpm_status_t pcpm_png_export(pcpm_png_t g, int64_t* png_off, int32_t* png_src,
                              int64_t* upd_start, int64_t* wo, int64_t* did_start,
                              uint32_t* did);

/* The build's edge weights in destination-ID bin order (Sec. 3.5): w[e]
 * (host, m floats) is the weight of the edge whose destination ID is did[e]
 * of pcpm_png_export.  PCPM_ERR_INVALID_ARG if the handle is unweighted.
 * Synchronises the device. */
pcpm_status_t pcpm_png_export_weights(pcpm_png_t g, float* w /* (host) m */);

/* Release a handle and its device memory (NULL is ignored). */
void pcpm_png_free(pcpm_png_t g);

/*
 * Sparse matrix-vector product over the PNG (Sec. 3.5, the extension of PCPM
 * to weighted graphs and SpMV):
 *   y(v) = sum over edges u->v of w(u,v) * x(u)
 * with w the build's weights (1 on every edge of an unweighted handle), i.e.
 * y = A^T x for the CSR matrix A of the build.  The scatter writes x(u) once
 * per (u, destination partition) (Alg. 3 without the 1/outdeg scaling); the
 * gather reads each weight with its destination ID and applies it to the
 * update before accumulating (Alg. 5).  x and y are device arrays of n floats
 * and must not overlap.  On a matrix handle (num_cols C, n = R rows) x has
 * R entries and y has C: y = A^T x, with the scatter over row partitions and
 * the gather over column partitions (Sec. 3.5); diagonal entries are
 * allowed there (allow_diagonal).
 * Accuracy: each product w*x(u) is formed exactly in FP64 and rounded to a
 * multiple of 2^-s, s = min(50 - ceil(log2(max|w| max|x|)), 62 -
 * ceil(log2(W max|x|))) with W the largest sum over v of |w(u,v)| (computed
 * once per handle: by the build when it has weights, by the first call
 * otherwise, on `stream`); the sum is exact (64-bit integers, independent of
 * order: y is bit-reproducible), then rounded once to FP32.  So |y(v) -
 * exact| <= indeg(v) 2^-(s+1) + FP32 rounding of y(v).  If x holds a
 * non-finite value, y is NaN everywhere.  Asynchronous on `stream`.
 * Works on multi-graph handles (block-diagonal).
 */
pcpm_status_t pcpm_spmv(pcpm_png_t g, const float* x /* (device) n */, float* y /* (device) n */,
                        void* stream);

/*
 * Degree-ordered relabelling of a CSR graph (Sec. 5.3.1 and Table 6: a node
 * labelling with more locality raises the compression ratio r of the PNG,
 * and with it lowers the traffic of Sec. 4).  New label i goes to the node of
 * i-th largest degree -- in-degree for key 0, out-degree for key 1 -- with
 * equal degrees in increasing old ID.  Outputs (device, caller-owned):
 * perm[old] = new label (n), and the relabelled CSR row_off_out (n + 1),
 * col_out (m): edge perm[u] -> perm[v] for every input edge u -> v, every row
 * in ascending column order.  Input: row_off (n + 1) non-decreasing from 0
 * to m, col (m) in [0, n) (PCPM_ERR_GRAPH otherwise); row order, self-loops
 * and duplicates are not checked and are carried over (pcpm_build_png
 * rejects them).  Outputs must not overlap inputs or each other.  Allocates
 * about 16.5 max(n, m) + 16 n bytes of device memory for the call.  Synchronises
 * `stream`.
 */
pcpm_status_t pcpm_relabel(int64_t n, int64_t m, const int32_t* row_off /* (device) n+1 */,
                           const int32_t* col /* (device) m */, int32_t key,
                           int32_t* perm /* (device) n */, int32_t* row_off_out /* (device) n+1 */,
                           int32_t* col_out /* (device) m */, void* stream);

/*
 * One PageRank iteration (Eq. 1, Sec. 2.1) carried out as PCPM scatter
 * (Alg. 3 over the PNG), gather (Alg. 5, branch-free) and apply (Alg. 2):
 *   pr_out(v) = (1-d)/n + d * ( sum_{u->v} pr_in(u)/outdeg(u) + D/n )
 * with D the FP64 sum of pr_in over dangling nodes (their mass is spread
 * uniformly).  pr_in and pr_out (n floats each) must not overlap.  If resid
 * is non-NULL the FP64 L1 distance sum_v |pr_out(v) - pr_in(v)| is written
 * there and the call synchronises `stream`; a non-finite value in pr_in then
 * returns PCPM_ERR_NUMERIC.  With resid NULL the call does not synchronise,
 * and a non-finite pr_in makes pr_out NaN everywhere.  pr_in may hold any
 * finite values (the fixed-point scale of the gather follows its largest
 * value and its L1 mass).  0 <= d < 1.
 */
pcpm_status_t pcpm_iterate(pcpm_png_t g, double d, const float* pr_in, float* pr_out,
                           double* resid /* (host) nullable */, void* stream);

/*
 * PageRank to convergence: starts from init (n floats, used as given) or,
 * when init is NULL, from 1/n everywhere; iterates as pcpm_iterate until the
 * FP64 L1 residual of an iteration is below tol (then pr_out holds that
 * iteration's output) or max_iters iterations have run.  tol <= 0 runs
 * exactly max_iters iterations and returns PCPM_OK.  *iters receives the
 * number of iterations run, *resid the last residual, res_hist (host,
 * nullable, max_iters entries) every residual.  1 <= max_iters <= 100000.
 * Synchronises `stream`.
 * For a handle of G > 1 graphs every graph runs Eq. 1 with its own n_g
 * (1/n_g start, jump and dangling spread on its own nodes, 0 on padding);
 * a graph whose residual falls below tol keeps that iterate while the others
 * go on; *iters and *resid are the largest over graphs, res_hist[i] is the
 * largest residual over graphs in iteration i (a graph that has converged
 * contributes its last residual), and pcpm_graph_results gives every graph's.
 */
pcpm_status_t pcpm_pagerank(pcpm_png_t g, double d, double tol, int32_t max_iters,
                            const float* init /* nullable */, float* pr_out,
                            int32_t* iters /* (host) */, double* resid /* (host) */,
                            double* res_hist /* (host) nullable */, void* stream);

/*
 * Personalised PageRank for k vectors on a single-graph handle.  Vector j
 * runs the recurrence of Eq. 1 with the uniform jump 1/n replaced by t_j,
 * uniform on its seed set S_j (the dangling mass D_j is spread by t_j too),
 * from x_0 = t_j:
 *   x'(v) = (1-d) t_j(v) + d * ( sum_{u->v} x(u)/outdeg(u) + D_j t_j(v) ).
 * S_j = seeds[seed_off[j] .. seed_off[j+1]) (host arrays; every set non-empty,
 * nodes in [0, n), no node twice in a set).  pcpm_ppr_tile_width(g) vectors
 * share every PNG edge and destination ID of the scatter and gather, one per
 * slot of an update; a vector whose FP64 L1 residual falls below tol (or
 * that has run max_iters iterations) is stored with that iterate and its
 * slot starts the next waiting vector, so each vector runs its own number of
 * iterations, the same as when it runs alone.  pr_out (device) receives the ranks as [n][k] row-major;
 * iters and resid (host, k each) every vector's iteration count and last
 * residual.  tol <= 0 runs exactly max_iters iterations.  Returns
 * PCPM_ERR_NOT_CONVERGED (outputs valid) when some vector stays above tol.
 * The first call on a handle allocates the working set for its tile width
 * and keeps it.  Synchronises `stream`.
 */
pcpm_status_t pcpm_ppr_batch(pcpm_png_t g, double d, int32_t k, const int32_t* seed_off /* (host) k+1 */,
                             const int32_t* seeds /* (host) */, double tol, int32_t max_iters,
                             float* pr_out /* [n][k] */, int32_t* iters /* (host) k */,
                             double* resid /* (host) k */, void* stream);

/* Vectors per tile of pcpm_ppr_batch on this handle: the largest power of two
 * (at most 16) whose q * width 8-byte sums fit the gather's LDS slice. */
int32_t pcpm_ppr_tile_width(pcpm_png_t g);

/* ---- learned warm start -------------------------------------------------
 * A start vector predicted from graph features by a 3-layer MLP (width 64,
 * ReLU), trained on PageRank vectors this library computes.  Compute is BF16
 * x BF16 with FP32 accumulation.  Parameters are one FP32 device array of
 * PCPM_WS_PARAMS floats: W1[64][8], b1[64], W2[64][64], b2[64], w3[64], b3.
 * Convergence is still certified by the FP64 residual of pcpm_pagerank; a
 * poor prediction costs iterations, never correctness. */
#define PCPM_WS_FEATURES 8
#define PCPM_WS_HIDDEN 64
#define PCPM_WS_PARAMS 4801

/* Features of every node of a single-graph handle into feat (device,
 * [n][8] FP32): log1p(indeg), log1p(outdeg), dangling flag, and
 * log(n * PR_1(v)) with PR_1 the first iterate of Eq. 1 from 1/n (the
 * one-SpMV aggregate sum_{u->v} 1/outdeg(u) of the in-neighbours' degrees),
 * then four zeros.  In-degrees are counted from the destination-ID bins on
 * the first call, and the first two features are kept in the handle from
 * then on (8 bytes per node; the time of that count and of forming them, in
 * ms, goes to *first_call_ms when non-NULL); every call runs one PCPM
 * iteration from the uniform vector. */
pcpm_status_t pcpm_ws_features(pcpm_png_t g, double d, float* feat, double* first_call_ms /* (host) nullable */,
                               void* stream);

/* yhat[v] = w3 . relu(W2 relu(W1 feat[v] + b1) + b2) + b3 for n nodes
 * (device arrays); the prediction of log(n * PR(v)).  Runs on MFMA. */
pcpm_status_t pcpm_ws_forward(const float* params, const float* feat, int64_t n, float* yhat, void* stream);

/* The warm-start prediction for the handle's nodes without a feature matrix:
 * yhat (device, n floats) equals pcpm_ws_forward(params, F) for the matrix F
 * that pcpm_ws_features(g, d, F) writes, bit for bit, with the features
 * formed in the forward kernel from the kept log-degrees, the dangling mask
 * and the first iterate (one PCPM iteration, as pcpm_ws_features runs).
 * Same handle requirements, in-degree count and *first_call_ms as
 * pcpm_ws_features. */
pcpm_status_t pcpm_ws_predict(pcpm_png_t g, const float* params, double d, float* yhat,
                              double* first_call_ms /* (host) nullable */, void* stream);

/* pr0 = softmax of yhat over the n nodes (max-shifted, FP64 sum): a start
 * vector of unit mass for pcpm_pagerank.  If any prediction is non-finite the
 * uniform vector 1/n is written instead and *fallback (host) is 1.  work:
 * device scratch of pcpm_ws_work_floats(1) floats. */
pcpm_status_t pcpm_ws_init(const float* yhat, int64_t n, float* pr0, float* work, int32_t* fallback /* (host) */,
                           void* stream);

/* Floats of device scratch pcpm_ws_backward needs for a minibatch of b. */
int64_t pcpm_ws_work_floats(int64_t b);

/* Gradient of the mean squared error (1/b) sum_i (yhat(idx[i]) - target(idx[i]))^2
 * with respect to params into grad (PCPM_WS_PARAMS floats), for the b rows
 * idx (device int64) of feat ([rows][8]) and target ([rows]); the forward
 * pass rounds as pcpm_ws_forward.  *loss (host) receives the loss.  Sums over
 * the minibatch run in a fixed order, so the result is deterministic.  An
 * index outside [0, rows) is not dereferenced: the call returns
 * PCPM_ERR_INVALID_ARG and grad is unspecified. */
pcpm_status_t pcpm_ws_backward(const float* params, const float* feat, const float* target, int64_t rows,
                               const int64_t* idx, int64_t b, float* grad, float* work, double* loss /* (host) */,
                               void* stream);

/* pcpm_ws_backward without a workspace argument and without allocating,
 * for callers that cannot allocate device memory (tight training loops,
 * harnesses that forbid hipMalloc).  The workspace is a fixed array of the
 * library in device memory (4.9 MB per GPU, held until the process ends),
 * so the minibatch is limited to b <= 16384 samples; a larger b returns
 * PCPM_ERR_INVALID_ARG before any device work.  Results are bit-identical to
 * pcpm_ws_backward's for the same inputs.  Every call on one GPU shares that
 * GPU's array: calls that overlap on one GPU (other threads, other streams)
 * race and must be serialised by the caller.  Synchronises `stream`. */
pcpm_status_t pcpm_ws_backward_noalloc(const float* params, const float* feat, const float* target, int64_t rows,
                                       const int64_t* idx, int64_t b, float* grad, double* loss /* (host) */,
                                       void* stream);

/* One Adam step (beta1 0.9, beta2 0.999, eps 1e-8, bias-corrected with step
 * >= 1) on the FP32 master parameters, moments m and v (device). */
pcpm_status_t pcpm_ws_adam(float* params, const float* grad, float* m, float* v, int32_t step, float lr,
                           void* stream);

/* Training target y[v] = log(n * pr[v]). */
pcpm_status_t pcpm_ws_targets(const float* pr, int64_t n, float* y, void* stream);

/* Per-graph outcome of the last pcpm_pagerank on a handle: iterations run and
 * last residual of each of the G graphs (host arrays of G). */
pcpm_status_t pcpm_graph_results(pcpm_png_t g, int32_t* iters /* (host) G */, double* resid /* (host) G */);

/* One measurement of an autotuned build. */
typedef struct {
  int32_t part_log2, update_order;     /* the candidate's q and update order   */
  int64_t scatter_chunk, gather_chunk; /* its work-item chunks (0 = automatic) */
  double ms_per_iter;                  /* per iteration (per vector-iteration
                                          for tune_vectors > 1)               */
  double build_ms;                     /* its PNG build (0 for chunk variants,
                                          which reuse the PNG)               */
} pcpm_tune_entry_t;

/* The measurements behind an autotuned handle (part_log2 = 0): up to
 * max_entries entries into out (host), in the order measured; returns the
 * number of entries (0 for a handle built with a given part_log2), and
 * *best (host, nullable) the index of the chosen one, *cached (host,
 * nullable) 1 if the sweep was taken from the process's cache (the table is
 * then the original sweep's). */
int32_t pcpm_tune_table(pcpm_png_t g, pcpm_tune_entry_t* out, int32_t max_entries, int32_t* best,
                        int32_t* cached);

/* Forget every configuration the autotuner remembers in this process. */
void pcpm_tune_cache_clear(void);

/* 64-bit content hash of a CSR graph (row_off n+1, col m, device arrays),
 * the one the autotuner's cache keys on; equal graphs give equal hashes.
 * Synchronises `stream`. */
pcpm_status_t pcpm_graph_hash(int64_t n, int64_t m, const int32_t* row_off, const int32_t* col, void* stream,
                              uint64_t* out /* (host) */);

/* Plain HBM streams, the measured ceiling the iteration kernels are compared
 * with (the part STREAM plays for the paper's CPU, Sec. 5.1): kind 0 reads
 * `bytes` from src (one float per workgroup, 4096 of them, goes to dst), 1
 * writes `bytes` to dst, 2 the same with non-temporal stores, 3 copies
 * `bytes` from src to dst, 4 the same with non-temporal stores.  bytes is a
 * positive multiple of 16; device buffers, 16-byte aligned, not
 * overlapping.  Asynchronous on `stream`. */
pcpm_status_t pcpm_hbm_stream(int32_t kind, const void* src /* (device) */, void* dst /* (device) */, int64_t bytes,
                              void* stream);

/* How pcpm_pagerank and pcpm_ppr_batch run their iterations on a handle.
 * mode 1: one launch per phase (scatter, gather, merge, finalize, refill)
 * per iteration, iterations queued in batches, two batches in flight while
 * the host reads the FP64 residual after the older one (iterations queued
 * past convergence return at once and change nothing).  mode 2: one persistent cooperative launch for the whole
 * solve or batch, one workgroup per resident slot (pcpm_launch_grid),
 * grid-wide barriers between the phases, convergence and refills decided on
 * the device.  mode 0 (the default) is mode 1, the faster on MI355X.
 * Results are bit-identical in both modes.  spin_limit bounds every
 * device-side wait of mode 2 (polls; 0 = the default, 2^22): a wait that
 * runs past it makes the call return PCPM_ERR_DEVICE with undefined output,
 * and the next call starts afresh.  PCPM_ERR_INVALID_ARG for another mode, or
 * mode 2 on a device without cooperative launches. */
pcpm_status_t pcpm_set_launch(pcpm_png_t g, int32_t mode, uint32_t spin_limit);

/* Workgroups of the persistent solve on this handle's device (0 if it
 * cannot run). */
int32_t pcpm_launch_grid(pcpm_png_t g);

/* Message of the calling thread's last failure ("" if none). */
const char* pcpm_last_error(void);

/*
 * Per-kernel device timing (HIP events recorded around every launch on the
 * launch stream).  pcpm_timing_enable(1) starts recording, (0) stops it.
 * pcpm_timing_collect synchronises the recorded events, fills up to
 * max_entries (host) records, returns how many kernels had launches and
 * clears the record.  The launches of iterations that pcpm_pagerank or
 * pcpm_ppr_batch queued past convergence (they return at once) are dropped
 * from the record, so a solve of c iterations records c launches of each
 * per-iteration kernel.  Meant for one recording thread at a time.
 */
typedef struct {
  char name[48];
  int64_t launches;
  double total_ms;
} pcpm_kernel_time_t;

void pcpm_timing_enable(int on);
int pcpm_timing_collect(pcpm_kernel_time_t* out /* (host) */, int max_entries);

#ifdef __cplusplus
}
#endif

#endif /* PCPM_H */
