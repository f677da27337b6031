/*
 * hanf.h — C ABI of the MI355X (gfx950) HyperANF library.
 *
 * HyperANF (Boldi, Rosa, Vigna, arXiv:1011.5599) approximates the neighbourhood
 * function N_G(t), the number of node pairs (x, y) with y reachable from x in at most
 * t arcs, by keeping one HyperLogLog counter per node (Section 3.1, Algorithm 1) and
 * replacing, at every iteration, each counter by the register-wise maximum of itself
 * and its successors' counters (Section 3.2, Algorithm 2), until no counter changes.
 * The statistics of Sections 4-5 (distance cdf, effective diameter, average distance,
 * spid) follow from the sequence N_hat(0..T).
 *
 * Conventions for every function:
 *   - Return value: HANF_OK (0), HANF_DONE (1, only hanf_iterate) or a negative error
 *     code. No exception or abort crosses the ABI. After an error the context stays
 *     valid for hanf_last_error and hanf_destroy; its run state may need a new
 *     hanf_init_counters.
 *   - The caller owns every buffer it passes in or receives into; the library owns the
 *     device memory it allocates and the context handle.
 *   - Work is ordered on the context's HIP stream. Calls that hand results to the
 *     host (hanf_iterate, hanf_read_*, hanf_stats, hanf_load_csr) return complete
 *     results: they synchronise that stream, unless nothing was queued since the values
 *     were last read with the run state (then they are served from that read).
 *   - A context is not thread-safe; distinct contexts are independent.
 *   - Device pointers are HIP device addresses on the context's device (for instance
 *     torch.Tensor.data_ptr() of a tensor on that device). Buffers passed with
 *     HANF_DEVICE_PTRS that are not device memory of that device are refused with
 *     HANF_EINVAL before any kernel touches them.
 */
#ifndef HANF_H
#define HANF_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes */
#define HANF_OK 0
#define HANF_DONE 1      /* hanf_iterate / hanf_poll: the fixpoint was reached */
#define HANF_BUSY 2      /* hanf_poll: enqueued passes are still running */
#define HANF_EINVAL -1   /* invalid argument or malformed graph */
#define HANF_ENOMEM -2   /* device or host allocation failed */
#define HANF_EDEVICE -3  /* HIP runtime error */
#define HANF_ESTATE -4   /* call out of order (e.g. iterate before init) */
#define HANF_ERANGE -5   /* output capacity too small */
#define HANF_EMAXITER -6 /* the pass cap was reached before the fixpoint */

/* ---- size limits: the most nodes and arcs of a graph, of a batch of graphs and of a
 * batch's row layout (2^31 - 2^20 each). Node ids and arc positions are 32-bit in the
 * kernels, which step up to a few thousand positions past the end of a range before
 * testing it, so both counts stay this far below 2^31 (HANF_EINVAL beyond). */
#define HANF_MAX_NODES 2146435072
#define HANF_MAX_ARCS 2146435072

/* ---- flags for buffers handed to the library */
#define HANF_HOST_PTRS 0u   /* host memory: copied */
#define HANF_DEVICE_PTRS 1u /* device memory: borrowed (load_csr) or copied (registers) */

/* ---- options (hanf_set_option) */
#define HANF_OPT_FRONTIER 1     /* 1 (default): skip successors whose counter did not change
                                   in the previous pass (Section 3.3, tracking modified
                                   counters); 0: every pass maximises with every successor */
#define HANF_OPT_MAX_PASSES 2   /* cap on passes before HANF_EMAXITER; default n + 1 */
#define HANF_OPT_LIGHT_MAX 3    /* nodes with at most this many arcs are handled by one lane
                                   group; default depends on m (0 = default) */
#define HANF_OPT_CHUNK_ARCS 4   /* arcs per wavefront chunk for the other nodes (0 = default) */
#define HANF_OPT_TIMING 5       /* 1: time every kernel with HIP events (hanf_read_pass_log) */
#define HANF_OPT_BATCH 6        /* passes enqueued between host checks of the fixpoint (default 4) */
#define HANF_OPT_TILE_NODES 7   /* nodes per light tile (multiple of the slots per wave; 0 = auto) */
#define HANF_OPT_DENSE_SWITCH 8 /* d: after a pass that changed >= n/d counters, the next pass
                                   maximises with every successor instead of testing each one's
                                   modified flag (same result; cheaper when most changed).
                                   Default 4; 0 = never */
#define HANF_OPT_SYSTOLIC 9     /* s: after a pass that changed < n/s counters, the next pass is
                                   systolic (Section 3.3, systolic computation): the modified
                                   counters signal their predecessors through the transposed
                                   graph and only signalled nodes are recomputed (same result).
                                   Needs a transposed graph (hanf_load_transpose or
                                   hanf_build_transpose); default 4 as in the paper; 0 = never */

#define HANF_OPT_SEEDS_PER_ROW 10 /* batched runs: counters of one graph's seeds side by side in a
                                   node's row (one successor scan and one gather serve them
                                   all). 0 (default): as many as fit, up to 32 and 1024 bytes
                                   per row; else a power of two up to 32. Results do not change */

#define HANF_OPT_PACKED5 11     /* register format, read by the next hanf_init_counters /
                                   hanf_init_batch. 1: 5-bit registers packed without gaps, as
                                   in Section 3.3 (register j of a counter at bits 5j..5j+4 of
                                   its little-endian bit string: 5m/8 bytes per counter instead
                                   of m), maximised with the paper's broadword multi-word max;
                                   needs m >= 64 (64 registers fill five 64-bit words). 0: one
                                   register per byte. 2 (default): 5-bit when a node's row
                                   holds at least 512 registers (m >= 64 and seeds side by side
                                   in a batch), else one per byte. Results are identical; register
                                   I/O stays one byte per register */
#define HANF_OPT_HUBS 12        /* node order of a single graph (a layout choice: every
                                   register, N_hat(t) up to the order of its sum, and T are those
                                   of the caller's order, and all I/O stays in the caller's node
                                   ids). K > 0: the K nodes with the largest in-degree (the
                                   counters the union step of Algorithm 2 reads most) first, by
                                   class of in-degree (8 per octave, largest first) and id, fewer
                                   when a class would cross K; every other node after them in id
                                   order. Their rows then share cache lines and stay in one XCD's
                                   L2: passes over every node run about 18% faster. In-degrees
                                   come from the transposed graph if one is set, else from a
                                   count of col_idx. Choosing the order rewrites the graph, which
                                   costs about 70% of a pass over every node (one rename per
                                   arc), once per ingest; K > 0 chooses it at the first
                                   hanf_init_counters after ingest. -1 (default): K = 4 MiB / row
                                   bytes (65536 at m = 64) when rows are shorter than a 128-byte
                                   L2 line (m <= 64 in bytes, m <= 128 packed: longer rows share
                                   no lines and gain nothing), for graphs of at least 16 K nodes
                                   with a transposed graph, chosen at the second
                                   hanf_init_counters on the same ingest (a single run keeps the
                                   caller's order; from the second run on, the rewrite pays for
                                   itself). 0: the caller's order */

#define HANF_OPT_FORWARD 14     /* systolic passes without a transposed graph (Section 3.3): when none
                                   is set, the pass after one that changed fewer than n/s counters
                                   (s = HANF_OPT_SYSTOLIC) finds the nodes to recompute by a
                                   forward scan of the successor lists in a kernel of its own
                                   (each node with a modified successor is marked), then
                                   recomputes only the marked nodes, as systolic passes do (pass
                                   records show systolic = 2). 0 (default) off: such passes test
                                   every successor's flag inside the union step, which on MI355X
                                   costs about as much as the scan alone (web24's last passes:
                                   0.68-0.71 ms, against 0.61 ms of scan plus the recomputation),
                                   and far less where many counters still change; 1 on. Results
                                   do not change */
#define HANF_OPT_STAGE 13       /* LDS staging of light tiles, in passes over every successor: the
                                   wavefront of a light tile (consecutive ids) first copies the
                                   tile's counters into LDS, then maximises successors inside
                                   the tile's id range from there (a tile holds 4 KiB of
                                   counters: 32 nodes at m = 128). 0 (default) never; 1 when
                                   the format allows (one register per byte, rows of at most
                                   256 bytes, 4 loads in flight). On MI355X the caches already
                                   serve such successors and staging is slower (fewer
                                   wavefronts per CU); it is kept as an option. Results do not
                                   change */

/* Tuning and test options (the results never change):
 *   103  LDS bytes per wavefront for the counters of a staged light tile (HANF_OPT_STAGE):
 *        2048, 4096 (default), 8192 or 16384;
 *   104  1: run the instrumented union kernels, which count arcs_near in the pass records
 *        (byte registers, rows of at most 256 bytes, 4 loads in flight; elsewhere -1);
 *   100  loads in flight per lane in the gather loops: 2, 4 or 8; 0 (default): 8 for one
 *        register per byte, 4 for 5-bit registers and for staged or instrumented kernels;
 *   101  the persistent union kernel over listed work units: 0 (default) for systolic
 *        passes, 1 never, 2 for every pass;
 *   102  hanf_build_transpose: 0 (default) the bucket sort up to 2^26 nodes and per-node
 *        counters above, 1 per-node counters always. */

/* ---- hanf_footprint flags */
#define HANF_FP_COPY_GRAPH 1    /* include the graph copy (HANF_HOST_PTRS ingest) */
#define HANF_FP_TRANSPOSE 2     /* include the transposed graph and the systolic signal buffers */
#define HANF_FP_PACKED5 4       /* 5-bit registers (HANF_OPT_PACKED5); needs log2m >= 6 */
#define HANF_FP_ORDER 8         /* the graph (and, with HANF_FP_TRANSPOSE, its transpose) rewritten
                                   in the library's node order, and the order tables
                                   (HANF_OPT_HUBS); an upper bound, a self-transpose needs no copy */

typedef struct hanf_ctx hanf_ctx;

/* Statistics of Sections 4-5 of the paper, from N_hat(0..T). */
typedef struct {
  double ed;       /* effective diameter at alpha: smallest t with H(t) >= alpha (Section 4) */
  double ied;      /* interpolated effective diameter: the alpha crossing of the linear
                      interpolation of (t, H(t)) (Section 4) */
  double avg_dist; /* E = sum_t t h(t), h(t) = H(t) - H(t-1) (Section 4, moments) */
  double var;      /* sum_t t^2 h(t) - E^2 (Section 4, moments) */
  double spid;     /* var / avg_dist, the shortest-paths index of dispersion (Section 5);
                      NaN when avg_dist = 0 */
  double n_max;    /* max_t N_hat(t), the normaliser of H */
  double d_lo;     /* Algorithm 3 with error eps: largest t with N_hat(t)/M <= alpha(1-2eps); -1 if none */
  double d_hi;     /* Algorithm 3: smallest t with N_hat(t)/M >= alpha(1+2eps); -1 if none */
  int32_t T;       /* the fixpoint iteration: N_hat has T+1 values */
  int32_t distinct;/* 1 if computed on pairs at distance >= 1 only (self-pairs dropped) */
} hanf_stats_t;

/* One record per executed pass (pass t turns c_t into c_{t+1}). */
typedef struct {
  int64_t changed;       /* counters that changed in the pass */
  int64_t arcs_scanned;  /* arcs whose successor was examined */
  int64_t arcs_gathered; /* arcs whose successor counter was maximised in (A_t) */
  int64_t rows_written;  /* counters written to the next buffer */
  int64_t rows_read;     /* own counters read to build a new counter */
  float union_ms;        /* union kernel time (HANF_OPT_TIMING), else 0 */
  float finalize_ms;     /* multi-chunk combine kernel time (and, with 5-bit registers, the
                            estimates of changed counters), else 0 */
  float reduce_ms;       /* estimate reduction kernels time, else 0 */
  int32_t gather_all;    /* 1 if the pass maximised with every successor */
  int32_t systolic;      /* 1 if only nodes signalled by a modified successor were recomputed
                            (signals through the transposed graph), 2 if so with the nodes
                            found by a forward scan of the successor lists (HANF_OPT_FORWARD) */
  int64_t arcs_signalled;/* systolic pass: predecessor arcs of the modified counters followed */
  float signal_ms;       /* systolic signal kernels time (HANF_OPT_TIMING), else 0 */
  int64_t arcs_local;    /* of arcs_gathered: successor counters read from a light tile's
                            counters staged in LDS (HANF_OPT_STAGE) instead of device memory */
  int64_t arcs_near;     /* of arcs_gathered: successors w of v with |w - v| < W, W = the rows
                            4 MiB (one XCD's L2) holds, halved: 16384 at 128-byte rows.
                            Counted by instrumented kernels only (option 104, or staging),
                            else -1 */
  int32_t flag_summary;  /* 1 if the pass read the modified-flag summary (a byte per 1024
                            nodes) before successors' flag words: a frontier pass after one
                            that modified counters in at most an eighth of those groups */
} hanf_pass_t;

/* Creates a context on HIP device `device`. `hip_stream` is a hipStream_t to order work
 * on, or NULL for a stream owned by the library. */
int hanf_create(int device, void *hip_stream, hanf_ctx **out);

/* Releases every device allocation of the context. Safe on NULL and after errors. */
void hanf_destroy(hanf_ctx *ctx);

/* Sets one HANF_OPT_* option. Schedule options take effect at the next initialisation
 * (hanf_init_counters / hanf_init_batch), which rebuilds the schedule when they changed. */
int hanf_set_option(hanf_ctx *ctx, int option, int64_t value);

/* Graph ingest (the graph G of Section 3.2, as successor lists). CSR: the successors of
 * v are col_idx[row_ptr[v] .. row_ptr[v+1]), 0 <= v < n. Requirements, checked on the
 * device: 1 <= n <= HANF_MAX_NODES, 0 <= arcs <= HANF_MAX_ARCS, row_ptr[0] = 0, row_ptr nondecreasing,
 * row_ptr[n] = arcs, 0 <= col_idx[a] < n (HANF_EINVAL otherwise). Duplicate arcs and
 * self-loops are allowed and change nothing. With HANF_HOST_PTRS the arrays are copied;
 * with HANF_DEVICE_PTRS they are borrowed and must stay alive and unchanged until the
 * context is destroyed or another graph is loaded. The degree-aware work schedule is
 * built on the device at the next initialisation (it depends on m). Discards any
 * previous run state. */
int hanf_load_csr(hanf_ctx *ctx, int32_t n, int64_t arcs, const int32_t *row_ptr,
                  const int32_t *col_idx, uint32_t flags);

/* Transposed graph for systolic passes (Section 3.3, systolic computation: a modified
 * counter signals the predecessors of its node). The predecessor lists of the loaded graph
 * as CSR: row_ptr_t[n + 1], col_idx_t[arcs], where n and arcs must be the graph's
 * (HANF_EINVAL otherwise); the order inside a list is free. With HANF_DEVICE_PTRS the
 * arrays are borrowed and must outlive the context's use of this graph; for a symmetric
 * graph the graph's own arrays may be passed. The CSR shape is checked on the device
 * (HANF_EINVAL); that it is the transpose is the caller's guarantee (otherwise the results
 * are undefined, though every access stays inside the context's arrays). Single graphs
 * only. Call after hanf_load_csr and before hanf_init_counters (a run in progress must be
 * initialised again). Replaced by the next graph ingest. */
int hanf_load_transpose(hanf_ctx *ctx, int32_t n, int64_t arcs, const int32_t *row_ptr_t,
                        const int32_t *col_idx_t, uint32_t flags);

/* Declares the loaded graph (every graph of a batch) symmetric: its successor lists are
 * also its predecessor lists, so they serve systolic passes as the transposed graph with no
 * copy. The symmetry is the caller's guarantee (otherwise the results are undefined, though
 * every access stays inside the context's arrays). Same call order as hanf_load_transpose;
 * single graphs and batches. */
int hanf_transpose_self(hanf_ctx *ctx);

/* Builds the transposed graph of the loaded graph (or batch) on the device: the arcs are
 * counting-sorted by target in two levels (per-bucket counts from LDS histograms over node
 * ranges, prefix sums, a scatter of (target, source) pairs, then a sort inside each bucket;
 * graphs beyond 2^26 nodes use per-node counters instead). The predecessor lists take
 * 4 (n + 1) + 4 arcs bytes, kept until the next graph ingest; the sort's buffers go back
 * to the context's pool before returning. Same call order as hanf_load_transpose. */
int hanf_build_transpose(hanf_ctx *ctx);

/* Counter initialisation (Algorithm 2: add v to c[v]; Algorithm 1 add). m = 2^log2m
 * registers per counter, 4 <= log2m <= 8. The item v is hashed with splitmix64:
 * h = output number v+1 of the generator started from state `seed`; register index =
 * the leftmost log2m bits of h; value = rho+ of the remaining bits (leading zeroes plus
 * one), saturated at 31. Computes N_hat(0) = sum_v size(c[v]) (Algorithm 1 size with the
 * HyperLogLog small-range rule). Asynchronous (no host synchronisation). */
int hanf_init_counters(hanf_ctx *ctx, int32_t log2m, uint64_t seed);

/* Runs up to max_steps passes of Algorithm 2's main loop (max_steps <= 0: until the
 * fixpoint). Each pass computes c_{t+1}[v] = register-wise max(c_t[v], c_t[w] for
 * v -> w) for every v, reading only c_t (synchronous update, as through the paper's
 * update file), then N_hat(t+1). Returns HANF_DONE when a pass left every counter
 * unchanged (the only sound stop, Section 3.2): T is then the last t, and N_hat has T+1
 * values. *steps_done (may be NULL) receives the passes run by this call, including
 * the final unchanged one; *changed_last (may be NULL) the changed count of the last
 * pass. HANF_EMAXITER if the pass cap is reached first. */
int hanf_iterate(hanf_ctx *ctx, int32_t max_steps, int32_t *steps_done, int64_t *changed_last);

/* Non-blocking form of hanf_iterate, for callers that keep several runs in flight on
 * different streams: enqueues `passes` passes and a copy of the run state, and returns at
 * once. Passes enqueued past the fixpoint do nothing. The pass log is not kept. */
int hanf_enqueue(hanf_ctx *ctx, int32_t passes);

/* Does not wait: HANF_BUSY while the work of the last hanf_enqueue runs; then HANF_DONE if
 * the fixpoint was reached, HANF_OK if more passes are needed, HANF_EMAXITER at the pass cap.
 * *t (may be NULL) receives the iteration reached. HANF_ESTATE if nothing was enqueued. */
int hanf_poll(hanf_ctx *ctx, int32_t *t);

/* Copies N_hat(0..t) to host `out` (FP64). *len receives t+1; HANF_ERANGE if cap < t+1. */
int hanf_read_nt(hanf_ctx *ctx, double *out, int32_t cap, int32_t *len);

/* Copies the current counters c_t (n*m bytes, node-major, m bytes per node, register j
 * of node v at v*m + j) to `out` (host or device per flags). `bytes` must be n*m. Packed
 * 5-bit registers are unpacked on the device (through a staging buffer of at most 64 MiB
 * when `out` is host memory). */
int hanf_read_registers(hanf_ctx *ctx, uint8_t *out, int64_t bytes, uint32_t flags);

/* The estimate size(c_t[v]) of every current counter (Algorithm 1, with the small-range
 * rule): out[v] for v < n, count = n. Single graphs. The same per-node values the pass
 * kernels sum into N_hat(t) (exposed so they can be checked one by one). */
int hanf_read_estimates(hanf_ctx *ctx, double *out, int64_t count, uint32_t flags);

/* The node order the library runs a single graph in (HANF_OPT_HUBS): out[i] = the caller's
 * id of the node whose counter is the library's row i (count = n int32, host or device per
 * flags). The identity until the initialisation that chooses the order (the first after
 * ingest with K > 0, the second with -1), and when that order is the caller's. HANF_EINVAL
 * for batches or a wrong count. */
int hanf_read_order(hanf_ctx *ctx, int32_t *out, int32_t count, uint32_t flags);

/* Resumes from a checkpoint: counters `in` (n*m bytes, layout of hanf_read_registers,
 * values <= 31; packed on the device when the run keeps 5-bit registers) taken at
 * iteration t, and N_hat(0..t) in nt_prefix (len = t+1, host).
 * Every counter is treated as modified for the next pass, so the continuation is
 * identical to an uninterrupted run. Requires a prior hanf_init_counters (fixes m).
 * Argument errors (sizes, t, flags, pointers) leave the run in progress untouched; a
 * register value above 31 (HANF_EINVAL) or a device error discards it, and the context
 * must then be initialised again. */
int hanf_write_registers(hanf_ctx *ctx, const uint8_t *in, int64_t bytes, int32_t t,
                         const double *nt_prefix, int32_t len, uint32_t flags);

/* Statistics of Sections 4-5 and Algorithm 3, computed on the device from the context's
 * N_hat(0..t): H(t) = N_hat(t)/max N_hat, h(t) = H(t) - H(t-1) (H(-1) = 0), ed, ied,
 * average distance, variance, spid, and Algorithm 3's interval with error eps. alpha in
 * (0, 1] (0.9 is the paper's default). distinct = 1 drops the self-pairs: H'(t) =
 * (N_hat(t) - N_hat(0)) / (max N_hat - N_hat(0)). */
int hanf_stats(hanf_ctx *ctx, double alpha, double eps, int32_t distinct, hanf_stats_t *out);

/* The same statistics from a caller's N_hat(0..len-1) (host memory, len >= 1, T = len-1):
 * a pure host function, no context or device (the code hanf_stats runs on the device).
 * HANF_EINVAL for NULL pointers, len < 1, alpha outside (0, 1] or eps < 0. */
int hanf_stats_nt(const double *nt, int32_t len, double alpha, double eps, int32_t distinct,
                  hanf_stats_t *out);

/* Per-pass records of the current run (one per executed pass). *len = passes so far. */
int hanf_read_pass_log(hanf_ctx *ctx, hanf_pass_t *out, int32_t cap, int32_t *len);

/* Device bytes a context needs for a graph of n nodes and `arcs` arcs at 2^log2m registers:
 * two register arrays (the counters and the update buffer, Section 3.2; 5m/8 bytes per
 * counter with HANF_FP_PACKED5 in `flags`), modified flags and their summary (a byte per
 * 1024 nodes), estimate sums, plus, by the bits of `flags` (HANF_FP_*): the graph copy
 * (HANF_FP_COPY_GRAPH), the transposed graph
 * with the systolic signal buffers and the lists of signalled successors (HANF_FP_TRANSPOSE;
 * systolic passes from a forward scan need the same buffers less the transposed graph) and
 * the reordered graph (HANF_FP_ORDER). Pure host function; the memory figure of Section 3.4
 * (O(n m) register bytes) is its dominant term. HANF_EINVAL for arguments out of range. */
int hanf_footprint(int32_t n, int64_t arcs, int32_t log2m, int32_t flags, int64_t *bytes);

/* Device memory the context holds (pure host function): *held (may be NULL) = every device
 * buffer it allocated and has not returned to HIP, in use or kept in its pool for reuse by
 * later runs (allocations are rounded up to size classes); *pooled (may be NULL) = the part
 * kept in the pool. What a caller budgeting device memory (a serving loop admitting graphs by
 * footprint, Section 3.4's memory bound) must count for this context. */
int hanf_device_bytes(const hanf_ctx *ctx, int64_t *held, int64_t *pooled);

/* Returns the pooled buffers (see hanf_device_bytes) to HIP. Waits for the context's stream;
 * freeing device memory also waits for the device. Buffers in use are kept. */
int hanf_trim(hanf_ctx *ctx);

/* ---- Batched runs: many independent HyperANF runs in the same passes.
 * Each input graph g is run with n_seeds hash seeds; component c = g * n_seeds + s is an
 * independent run of Algorithm 2 on graph g with seed seeds[c]. The components are laid
 * side by side as one graph (disjoint union, each starting on a 64-node boundary), so a
 * pass of Algorithm 2 over it is a pass of every component; a component's counters and
 * N_hat(t) are exactly those of its own run, and its fixpoint T is the first pass that left
 * it unchanged. hanf_iterate runs the passes until every component has stopped. This serves
 * the paper's protocol of many low-precision runs per graph (Section 4, moments; Section 6). */

/* Loads the graphs: graph_off[n_graphs+1] node offsets (graph g has nodes graph_off[g] ..
 * graph_off[g+1]-1, at least one) and arc_off[n_graphs+1] arc offsets (host memory), and
 * row_ptr[graph_off[n_graphs]+1], col_idx[arc_off[n_graphs]]: one CSR over all graphs with
 * global ids (host memory, copied, or device memory with HANF_DEVICE_PTRS, read only during
 * this call). row_ptr[graph_off[g]] must equal arc_off[g] and no arc may leave its graph
 * (HANF_EINVAL). Replaces any graph or batch the context held. */
int hanf_load_batch(hanf_ctx *ctx, int32_t n_graphs, const int32_t *graph_off, const int32_t *arc_off,
                    const int32_t *row_ptr, const int32_t *col_idx, int32_t n_seeds, uint32_t flags);

/* The same, with the graphs given separately, each as its own CSR with its own node ids
 * 0..n_nodes[g]-1: row_ptrs[g] (n_nodes[g]+1 entries) and col_idxs[g] (n_arcs[g] entries),
 * all host memory (copied) or all device memory (HANF_DEVICE_PTRS, read during the call).
 * The arrays of pointers and sizes are host memory. Each graph's CSR is checked as in
 * hanf_load_csr. */
int hanf_load_batch_list(hanf_ctx *ctx, int32_t n_graphs, const int32_t *const *row_ptrs,
                         const int32_t *const *col_idxs, const int32_t *n_nodes, const int64_t *n_arcs,
                         int32_t n_seeds, uint32_t flags);

/* Initialises every component (Algorithm 2's initialisation with the graph-local node id as
 * the item and seeds[c] as the hash seed; seeds has n_graphs * n_seeds entries, host). Passes
 * allowed default to the largest graph's n + 1 (every component then stops as it would alone),
 * lowered to what 64 MiB of per-component N_hat histories hold but never below 1024
 * (HANF_OPT_MAX_PASSES changes it). */
int hanf_init_batch(hanf_ctx *ctx, int32_t log2m, const uint64_t *seeds);

/* Number of components and, if T is non-NULL (n_components entries, host), each one's
 * fixpoint iteration, or -1 while it still changes. */
int hanf_batch_info(hanf_ctx *ctx, int32_t *n_components, int32_t *T);

/* N_hat(0..T) of component `comp` (or up to the current iteration while it still changes). */
int hanf_batch_read_nt(hanf_ctx *ctx, int32_t comp, double *out, int32_t cap, int32_t *len);

/* Current counters of component `comp`: n_g * m bytes, node-major (graph-local ids), one
 * byte per register (5-bit rows are unpacked on the device), to host or device memory per
 * flags. HANF_EINVAL for a bad component or size. */
int hanf_batch_read_registers(hanf_ctx *ctx, int32_t comp, uint8_t *out, int64_t bytes, uint32_t flags);

/* Per-node estimates of component comp (count = its graph's n), as hanf_read_estimates. */
int hanf_batch_read_estimates(hanf_ctx *ctx, int32_t comp, double *out, int64_t count, uint32_t flags);

/* hanf_stats of component `comp`. */
int hanf_batch_stats(hanf_ctx *ctx, int32_t comp, double alpha, double eps, int32_t distinct,
                     hanf_stats_t *out);

/* The paper's a-posteriori figures over many runs of one graph (Section 6; Table 2 reports
 * them as mean +- standard deviation over 100 runs): for every graph g of the batch, over its
 * n_seeds runs (components g * n_seeds + s), the mean and the sample standard deviation of
 * the effective diameter at alpha, the interpolated effective diameter, the average distance
 * and spid (Sections 4-5; distinct = 1 drops the self-pairs as in hanf_stats). */
typedef struct {
  double ed, ied, avg_dist, spid;              /* means over the graph's runs */
  double ed_sd, ied_sd, avg_dist_sd, spid_sd;  /* sample standard deviations (divisor runs - 1);
                                                  NaN with one run */
  int32_t runs;                                /* n_seeds */
  int32_t distinct;
} hanf_seed_summary_t;

/* Fills out[0 .. n_graphs-1] (host) for the loaded batch, computed on the device from every
 * component's N_hat (a component still changing contributes its N_hat so far). HANF_ESTATE
 * without an initialised batch, HANF_EINVAL for alpha outside (0, 1] or a NULL out. */
int hanf_batch_seed_summary(hanf_ctx *ctx, double alpha, int32_t distinct, hanf_seed_summary_t *out);

/* hanf_stats of every component in one launch; out has n_components entries (host). */
int hanf_batch_stats_all(hanf_ctx *ctx, double alpha, double eps, int32_t distinct, hanf_stats_t *out);

/* For callers that cannot allocate device memory (code under HIP graph capture, serving
 * loops and harnesses that forbid hipMalloc): hanf_batch_stats_all without any allocation.
 * The kernel stages the per-component records in a fixed device array of
 * HANF_NOALLOC_MAX_COMPONENTS records (72 bytes each, 4.5 MiB), one per device, allocated
 * with the library and held until the process ends; the records are then copied to `out`
 * (n_components hanf_stats_t, host memory, the caller's). Every record is written by each
 * call, so nothing needs clearing between calls. HANF_ERANGE, with a message, when the
 * batch has more components than that; HANF_EDEVICE if the array's device address could
 * not be obtained when the context was created. All calls on one device share its array:
 * calls that overlap on one device (for instance from two host threads) race. Synchronises
 * the context's stream. */
#define HANF_NOALLOC_MAX_COMPONENTS 65536
int hanf_batch_stats_all_noalloc(hanf_ctx *ctx, double alpha, double eps, int32_t distinct, hanf_stats_t *out);

/* Last error message of the context, or of the calling thread when ctx is NULL. */
const char *hanf_last_error(const hanf_ctx *ctx);

/* Section 3.3's broadword register-wise max on 5-bit fields, on its own: `groups` groups of
 * 64 registers packed in five 64-bit words (40 bytes, register j at bits 5j..5j+4 of the
 * group's little-endian bit string, so fields 12, 25, 38 and 51 straddle two words);
 * out = max(x, y) per register. Device pointers, 8-byte aligned, on device `device`.
 * The same function the union kernel uses with HANF_OPT_PACKED5; exposed for exhaustive
 * testing. Synchronous. */
int hanf_max5_groups(int device, const uint8_t *x, const uint8_t *y, uint8_t *out, int64_t groups);

/* Register-wise maximum of `count` 32-bit words, each holding four registers (values
 * <= 127): out[i] = bytewise max(x[i], y[i]), on device `device`. Device pointers. Exposes
 * the union kernel's packed maximum (Algorithm 2 union; Section 3.3's broadword idea) for
 * exhaustive testing. Synchronous. */
int hanf_bytemax_words(int device, const uint32_t *x, const uint32_t *y, uint32_t *out,
                       int64_t count);

/* The union step's accumulator for the successor counters it gathers (Algorithm 2 union),
 * on its own: `count` groups of k 16-byte lanes (16 registers each, one per byte),
 * out[i] = the register-wise max of x[i*k .. i*k+k), accumulated from empty (from_first 0)
 * or starting from the first lane (1), the two ways the union kernel starts it. Device
 * pointers, 16-byte aligned, on device `device`; x holds count * k lanes, out count lanes.
 * Exposed for exhaustive testing. Synchronous. */
int hanf_gathermax_lanes(int device, const uint32_t *x, int32_t k, int32_t from_first, uint32_t *out,
                         int64_t count);

#ifdef __cplusplus
}
#endif

#endif /* HANF_H */
