// Internal declarations shared by the HIP kernels (hanf_kernels.hip) and the C-ABI host
// layer (hanf_api.hip). Not part of the public interface.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace hanf {

constexpr int kWave = 64;         // CDNA wavefront width
constexpr int kBlockThreads = 256; // 4 wavefronts per workgroup
constexpr int kNodesPerBlock = 64; // estimate partial sums are cached per 64 consecutive nodes
constexpr int kMaxTile = 256;      // largest light tile (bitonic sort width)
constexpr int kXcds = 8;           // MI355X accelerator complex dies
constexpr int kReduceBlocks = 64;  // 64-node blocks per reduction workgroup (16 per wavefront)
constexpr int kSumShift = 10;      // modified-flag summary: one byte per 2^10 nodes (16 blocks,
                                   //   one reduction wavefront's)
constexpr int kSumDiv = 8;         // summary read when at most 1/8 of its bytes are set
constexpr int kMarkedShift = 40;   // per reduction workgroup, the marked summary bytes are
                                   //   added to its changed-counter count from this bit
constexpr int kStatSlots = 1024;   // rows of work counters, spread over workgroups
constexpr int kStatFields = 6;     // work counters per row: scanned, gathered, written, read, local, near
constexpr int64_t kL2Bytes = 4 << 20;  // L2 of one XCD
constexpr int kStageWaveBytes = 4096;  // LDS per wavefront for the rows of a staged light tile
constexpr int kCompChunkBlocks = 1024;  // blocks per chunk of a batch component's reduction
constexpr int kPacked5LaneBytes = 40;   // 64 registers of 5 bits: one lane of a packed counter
constexpr int kMaxPassesPerCheck = 1024;  // passes enqueued between host reads of the run state
constexpr int32_t kMaxLogRecords = 1 << 16;  // pass records kept per run (the first 65536 passes)

// Run state kept in device memory, so consecutive passes can be enqueued without a host
// round trip: kernels read the iteration t and stop early once the run has halted.
struct DevState {
  int32_t t;          // the counters in regs[t & 1] are c_t
  int32_t halted;     // 1 once a pass changed nothing (done) or the pass cap was reached
  int32_t done;       // 1 once a pass changed nothing
  int32_t capped;     // 1 if the pass cap stopped the run
  int32_t first_pass; // 1 after init/resume: both register buffers hold c_t, every
                      // successor is maximised in, and no copy is needed
  int32_t frontier;   // 1 = skip successors unchanged in the previous pass
  int32_t max_passes;
  int32_t passes;     // passes executed so far
  int32_t err;        // validation error bits
  int32_t dense_next; // 1: the next pass maximises with every successor (the previous pass
                      // changed at least dense_threshold counters)
  int32_t systolic;   // 1: this pass only recomputes nodes signalled through the transposed
                      // graph (the previous pass changed fewer than n / sys_div counters)
  int32_t sys_div;    // 0 = never systolic
  int64_t changed_last;
  int64_t dense_threshold;  // 0 = never
  uint64_t sys_acc;   // systolic pass: (signalling nodes << 32) | their predecessor arcs
  int32_t sys_units;  // systolic pass: work units listed for the union kernel
  int32_t use_sum;    // 1: the next pass reads a group's summary byte before a flag word
                      //   (set when at most 1 / kSumDiv of the groups are marked)
};

struct PassLog {  // per executed pass, filled on the device
  int64_t changed, scanned, gathered, written, read, gather_all, systolic, signalled;
  int64_t local;  // successor counters maximised in from a light tile's rows staged in LDS
  int64_t near;   // successor counters maximised in whose id is within near_window of the node's
                  //   (counted only by the instrumented kernels: count_near or stage)
  int64_t summary;  // 1 if the pass read the flag summary before flag words
};

struct Chunk {   // a run of at most `chunk_arcs` arcs of one node, handled by one wavefront
  int32_t v, a0, a1, part;  // part: partial-result slot for nodes split in several chunks, else -1
};

struct Heavy {   // a node split in several chunks, combined by the finalize kernel
  int32_t v, first, count, pad_;
};

enum ReduceMode : int32_t { kReduceInit = 0, kReducePass = 1 };

// Statistics of N_hat(0..T) into out[0..8]: ed, ied, avg_dist, var, spid, n_max, d_lo, d_hi,
// T (Sections 4-5 and Algorithm 3). Sequential O(T) work; the same code serves the device
// kernels (k_stats, k_stats_all) and the host entry point hanf_stats_nt.
__host__ __device__ inline void stats_of(const double *nt, int32_t T, double alpha, double eps, int32_t distinct,
                         double *out) {
  double M = nt[0];
  for (int32_t t = 1; t <= T; ++t) M = nt[t] > M ? nt[t] : M;
  const double base = distinct ? nt[0] : 0.0;
  const double den = M - base;
  const double nan = __builtin_nan("");
  double ed = nan, ied = nan, mean = 0.0, second = 0.0;
  double Hprev = 0.0;
  bool found = false;
  for (int32_t t = 0; t <= T; ++t) {
    const double H = den > 0.0 ? (nt[t] - base) / den : nan;
    const double h = H - Hprev;
    mean += (double)t * h;
    second += (double)t * (double)t * h;
    if (!found && H >= alpha) {
      found = true;
      ed = (double)t;
      ied = t == 0 ? 0.0 : (double)(t - 1) + (alpha - Hprev) / (H - Hprev);
    }
    Hprev = H;
  }
  const double var = second - mean * mean;
  double d_lo = -1.0, d_hi = -1.0;
  for (int32_t t = 0; t <= T; ++t) {
    const double r = nt[t] / M;
    if (r <= alpha * (1.0 - 2.0 * eps)) d_lo = (double)t;
    if (d_hi < 0.0 && r >= alpha * (1.0 + 2.0 * eps)) d_hi = (double)t;
  }
  out[0] = ed;
  out[1] = ied;
  out[2] = mean;
  out[3] = var;
  out[4] = mean != 0.0 ? var / mean : nan;
  out[5] = M;
  out[6] = d_lo;
  out[7] = d_hi;
  out[8] = (double)T;
}


// One component's statistics as the public hanf_stats_t lays them out (ed, ied, avg_dist,
// var, spid, n_max, d_lo, d_hi, then T and distinct), so records written on the device can
// be copied into the caller's array as they are.
struct StatsRec {
  double v[8];
  int32_t T;
  int32_t distinct;
};

// Per-graph summary of a batch's runs as the public hanf_seed_summary_t lays it out: means
// of ed, ied, avg_dist, spid, then their sample standard deviations, then runs and distinct.
struct SummaryRec {
  double v[8];
  int32_t runs;
  int32_t distinct;
};

// Layout of a batched run. Its results are components c = (graph g, seed s), independent
// runs. Every node row holds S = 2^seed_log2 counters ("row seeds" j = 0..S-1), so the
// graphs are laid side by side as one graph in copies ("layout components" L), each
// starting on a 64-node boundary so that no estimate block straddles two; copy L of graph g
// carries seeds q*S .. q*S+S-1 of g in its rows (q = L mod copies). Row seeds beyond the
// graph's seeds hold empty counters that never change.
struct BatchArgs {
  const int32_t *blk_comp;       // layout component of every 64-node block
  const int32_t *comp_node_off;  // first node of every layout component, n_lay + 1 entries
  const int32_t *comp_n;         // real nodes of every layout component (the rest are padding)
  const int32_t *slot_comp;      // result component of row seed j of layout component L at
                                 //   [L * S + j], or -1 for an empty row seed
  const int32_t *comp_row;       // L * S + j of every result component
  const uint64_t *comp_seed;     // hash seed of every result component
  int32_t *blkcnt;               // counters changed per (block, row seed) in the last pass
  int32_t *comp_T;               // fixpoint iteration of every result component, -1 while it changes
  double *comp_nt;               // N_hat history: comp_nt[c * nt_cap + t]
  const int32_t *comp_chunk0;    // first reduction chunk of every result component (n_comp + 1)
  const int32_t *cchunk_comp;    // result component of every chunk
  const int32_t *cchunk_b0;      // first block of every chunk
  double *cchunk_sum;            // per chunk: estimate sum and changed counters of the last pass
  int64_t *cchunk_cnt;
  int32_t n_cchunks;
  int32_t n_comp;                // result components
  int32_t n_lay;                 // layout components
  int32_t active;                // 1 for a batched run
};

// Kernel arguments of one pass (passed by value).
struct PassArgs {
  const int32_t *row_ptr;
  const int32_t *col_idx;
  uint8_t *regs0, *regs1;    // regs[t & 1] = c_t, regs[(t+1) & 1] = c_{t+1}; a row of S counters
                             //   of m bytes per node (row seed j at byte j * m)
  uint32_t *bits0, *bits1;   // changed flags, S bits per node (bit v * S + j): bits[t & 1] written
                             //   by pass t-1, bits[(t+1) & 1] by pass t
  uint8_t *mod_sum;          // per 2^kSumShift nodes: 1 if the last pass modified a counter there
  int32_t n_sum;             // its bytes
  double *est;               // estimate of every current counter, [v * S + j]
  double *blocksum;          // per 64 nodes and row seed, [b * S + j]
  double *wgsum;             // per reduce workgroup
  int64_t *wgcnt;            // per reduce workgroup: changed counters, plus its marked summary
                             //   bytes << kMarkedShift
  int64_t *stat_slots;       // kStatSlots x {scanned, gathered, written, read, local, near}
  const int32_t *light;      // light tiles: tile_nodes entries per tile, -1 = empty
  const Chunk *chunks;
  const Heavy *heavy;
  uint8_t *partial;          // m bytes per chunk of a multi-chunk node
  uint8_t *partial_any;      // 1 if the chunk maximised at least one successor
  const int32_t *trow_ptr;   // transposed graph (predecessor lists), systolic passes only
  const int32_t *tcol_idx;
  uint8_t *todo;             // systolic pass: 1 for nodes with a successor modified by the previous
                             //   pass (one byte per node, 64 per block: set with plain stores)
  uint8_t *tile_todo;        // systolic pass: 1 for light tiles holding such a node
  int32_t *unit_list;        // systolic pass: work units with something to do (chunks, then tiles)
  int32_t *sys_node;         // systolic pass: modified nodes with predecessors ...
  int32_t *sys_pos;          //   ... and the offset of their predecessor arcs in the signal list
  int32_t *sig_list;         // systolic pass: the signalled successors of node v (those whose
                             //   counter the previous pass modified, one entry per arc) at
                             //   sig_list[row_ptr[v] ..], in no particular order (arcs entries) ...
  int32_t *sig_cnt;          //   ... and how many (one per node, 64 per block; cleared with todo)
  DevState *st;
  double *nt;                // N_hat history
  PassLog *log;
  const double *lc;          // linear-counting table m ln(m/V), V = 0..m
  double K;                  // alpha_m m^2 2^31
  int32_t n;
  int32_t log2m;             // m = 2^log2m registers per counter
  int32_t seed_log2;         // S = 2^seed_log2 counters per node row (1 for a single run)
  int32_t gs;                // lanes per counter: m / 16, or m / 64 for 5-bit registers
                             // (a row has S * gs lanes)
  int32_t packed;            // 1: 5-bit registers packed without gaps (m >= 64)
  int32_t n_blocks;          // ceil(n / 64)
  int32_t n_chunks;
  int32_t n_chunk_wgs;       // union workgroups given to chunks (multiple of 8)
  int32_t n_light_wgs;
  int32_t n_tiles;
  int32_t tile_nodes;
  int32_t light_max;         // nodes with more arcs are handled by chunks
  int32_t stage;             // 1: in passes over every successor, a light tile's wavefront first
                             //   copies the rows of c_t of the tile's id range into LDS, and
                             //   successors in that range are maximised in from there
  int32_t lds_wave_bytes;    // dynamic LDS per wavefront of the union kernels: the list of
                             //   active nodes of a tile or, when staging, its rows (shared)
  int32_t near_window;       // a gathered successor w of v is counted as near if |w - v| < this
  int32_t count_near;        // 1: the union kernels count near successors (instrumented kernels)
  int32_t n_heavy;
  int32_t n_fin_wgs;
  int32_t n_reduce_wgs;
  int32_t nt_cap;             // N_hat history capacity (values)
  int32_t log_cap;            // pass records kept (passes beyond it run unrecorded)
  int64_t arcs;
  const int32_t *node_id;    // the caller's id of node v (hashed at initialisation) when the
                             //   library chose its own node order, else NULL (the same id)
  BatchArgs batch;
};

// ---- launchers (hanf_kernels.hip); all asynchronous on `s`
hipError_t launch_validate(const int32_t *row_ptr, const int32_t *col_idx, int32_t n, int64_t arcs,
                           DevState *st, hipStream_t s);
hipError_t launch_state_reset(DevState *st, int32_t t, int32_t frontier, int32_t max_passes,
                              int64_t dense_threshold, int32_t sys_div, hipStream_t s);
hipError_t launch_classify(const int32_t *row_ptr, int32_t n, int32_t light_max, int32_t chunk_arcs,
                           uint64_t *keys, hipStream_t s);
// exclusive scan of n uint64 values in place; `tmp` needs scan_tmp_elems(n) elements
int64_t scan_tmp_elems(int64_t n);
hipError_t launch_exclusive_scan_u64(uint64_t *data, int64_t n, uint64_t *tmp, hipStream_t s);
hipError_t launch_fill_chunks(const int32_t *row_ptr, int32_t n, const uint64_t *offs,
                              int32_t chunk_arcs, Chunk *chunks, Heavy *heavy, hipStream_t s);
hipError_t launch_build_tiles(const int32_t *row_ptr, int32_t n, int32_t light_max, int32_t tile_nodes,
                              int32_t n_tiles, int32_t *light, hipStream_t s);
hipError_t launch_init(const PassArgs &a, uint64_t seed, hipStream_t s);
hipError_t launch_estimate_all(const PassArgs &a, const uint8_t *regs, hipStream_t s);
// Pass launchers take optional events recorded at the start of their first kernel (e0) and
// the end of their last (e1).
hipError_t launch_signal(const PassArgs &a, int64_t arcs, hipStream_t s, hipEvent_t e0 = nullptr,
                         hipEvent_t e1 = nullptr);
// full: the kernel with one wavefront per work unit; list: the persistent kernel, which
// runs the systolic passes when both are launched and every pass when it runs alone
hipError_t launch_union(const PassArgs &a, int u, int full, int list, hipStream_t s, hipEvent_t e0 = nullptr,
                        hipEvent_t e1 = nullptr);
// transposed graph: in-degree counts into keys (n + 1 zeroed uint64), then, after their
// exclusive scan, the predecessor lists (keys are consumed as fill cursors)
hipError_t launch_transpose_count(const int32_t *col_idx, int64_t arcs, uint64_t *keys, hipStream_t s);
hipError_t launch_transpose_fill(const int32_t *row_ptr, const int32_t *col_idx, int32_t n, uint64_t *keys,
                                 int32_t *trow_ptr, int32_t *tcol_idx, hipStream_t s);
hipError_t launch_fill_u64(uint64_t *p, int64_t count, uint64_t value, hipStream_t s);
// transposed graph by buckets (graphs of at most kTpMaxNodes nodes): first level (per node
// range histograms into nb buckets of 2^bs ids, their scan, the pairs, bucket starts), then
// second level (light buckets one workgroup each; hub buckets in chunks)
constexpr int32_t kTpMaxNodes = 1 << 26;
constexpr int32_t kTpNumBuckets = 8192;
constexpr int64_t kTpLight = 1 << 18;   // pairs of a bucket sorted by one workgroup
constexpr int64_t kTpChunk = 1 << 16;   // pairs per chunk of a hub bucket
hipError_t launch_tp_first(const int32_t *row_ptr, const int32_t *col_idx, int32_t n, int32_t range, int32_t bs,
                           int32_t nb, int32_t n_ranges, uint64_t *hist, uint64_t *scan_tmp, uint64_t *pairs,
                           uint64_t *bstart, hipStream_t s);
hipError_t launch_tp_second(const uint64_t *pairs, const uint64_t *bstart, const int32_t *blist, int32_t n_light,
                            const int32_t *hlist, const int32_t *hchunk0, int32_t n_heavy, const int64_t *chunk_lo,
                            const int64_t *chunk_hi, const int64_t *chunk_s, int32_t n_hchunks, uint32_t *h2, int32_t bs,
                            int32_t n, int32_t *trow_ptr, int32_t *tcol_idx, hipStream_t s);
// ---- node order (hanf_order.hip): hubs first, by class of in-degree, then the other nodes
constexpr int kOrderLevels = 240;                 // in-degree classes 0..239 (0: no arcs in)
constexpr int kOrderTopLevel = kOrderLevels - 1;  // hub of level l has output class top - l
constexpr int kOrderRest = kOrderLevels;          // output class of the other nodes
constexpr int kOrderClasses = kOrderLevels + 1;
int64_t order_counts_elems(int32_t n);  // uint64 counters of launch_order_select
// in-degrees: from the transposed graph's rows when trp is set, else by counting targets
hipError_t launch_in_degrees(const int32_t *trp, const int32_t *ci, int32_t n, int64_t arcs, uint32_t *deg,
                             hipStream_t s);
// perm (new id -> old id) and inv (old -> new): at most K hubs by class of in-degree, then
// the rest by id. hist: kOrderLevels uint32; plan: 1 int32; counts: order_counts_elems(n)
// uint64 with scan_tmp of scan_tmp_elems of that many
hipError_t launch_order_select(const uint32_t *deg, int32_t n, int64_t K, uint32_t *hist, int32_t *plan,
                               uint64_t *counts, uint64_t *scan_tmp, int32_t *perm, int32_t *inv, hipStream_t s);
// the CSR (rp, ci) in the new order, whose first H ids are the hubs: keys n + 1 uint64 (with
// scan_tmp for n + 1), rec rename_groups(n) records and hub_new max(H, 1) int32 (the
// renaming table of the arcs' targets), wrow permute_windows(arcs) + 1 int32
int64_t rename_groups(int32_t n);
int64_t permute_windows(int64_t arcs);
hipError_t launch_permute_csr(const int32_t *rp, const int32_t *ci, int32_t n, int64_t arcs, const int32_t *perm,
                              const int32_t *inv, int32_t H, uint64_t *keys, uint64_t *scan_tmp, uint4 *rec,
                              int32_t *hub_new, int32_t *wrow, int32_t *rp_new, int32_t *ci_new, hipStream_t s);
// dst row i = src row idx[i]; row_bytes a multiple of 8
hipError_t launch_gather_rows(const uint8_t *src, uint8_t *dst, const int32_t *idx, int32_t n, int64_t row_bytes,
                              hipStream_t s);
hipError_t launch_iota(int32_t *p, int32_t n, hipStream_t s);
hipError_t launch_finalize(const PassArgs &a, hipStream_t s, hipEvent_t e0 = nullptr, hipEvent_t e1 = nullptr);
hipError_t launch_estimate_changed(const PassArgs &a, hipStream_t s, hipEvent_t e0 = nullptr,
                                   hipEvent_t e1 = nullptr);
hipError_t launch_reduce(const PassArgs &a, int32_t mode, int32_t force, hipStream_t s, hipEvent_t e0 = nullptr,
                         hipEvent_t e1 = nullptr);
hipError_t launch_stats(const double *nt, const int32_t *T_or_null, const DevState *st, double alpha,
                        double eps, int32_t distinct, double *out, hipStream_t s);
hipError_t launch_expand_local(const int32_t *graph_off, const int32_t *arc_off, const int32_t *rp_in,
                               const int32_t *ci_in, int32_t n_graphs, int32_t n_seeds, const PassArgs &a,
                               const int32_t *comp_arc_off, int32_t *rp_exp, int32_t *ci_exp, int64_t n_exp,
                               int64_t e_exp, DevState *st, hipStream_t s);
hipError_t launch_check_offsets(const int32_t *rp, const int32_t *goff, const int32_t *aoff, int32_t n_graphs,
                                DevState *st, hipStream_t s);
hipError_t launch_stats_all(const PassArgs &a, double alpha, double eps, int32_t distinct, StatsRec *out,
                            hipStream_t s);
hipError_t launch_seed_summary(const PassArgs &a, int32_t n_graphs, int32_t n_seeds, double alpha, int32_t distinct,
                               SummaryRec *out, hipStream_t s);
hipError_t launch_expand(const int32_t *graph_off, const int32_t *rp_in, const int32_t *ci_in,
                         int32_t n_seeds, const PassArgs &a, const int32_t *comp_arc_off, int32_t *rp_exp,
                         int32_t *ci_exp, int64_t n_exp, int64_t e_exp, DevState *st, hipStream_t s);
hipError_t launch_check_registers(const uint8_t *regs, int64_t bytes, DevState *st, hipStream_t s);
hipError_t launch_set_history(double *nt, const double *prefix, int32_t len, DevState *st,
                              int32_t t, hipStream_t s);
hipError_t launch_bytemax_words(const uint32_t *x, const uint32_t *y, uint32_t *out, int64_t count,
                                hipStream_t s);
hipError_t launch_gathermax_lanes(const uint4 *x, int32_t k, int32_t from_first, uint4 *out, int64_t count,
                                 hipStream_t s);
hipError_t launch_max5_groups(const uint8_t *x, const uint8_t *y, uint8_t *out, int64_t groups, hipStream_t s);
hipError_t launch_unpack5(const uint8_t *packed, uint8_t *out, int64_t groups, hipStream_t s);
hipError_t launch_pack5(const uint8_t *in, uint8_t *packed, int64_t groups, hipStream_t s);
hipError_t launch_unpack5_rows(const uint8_t *src, int64_t row_stride, int32_t gpr, int64_t rows, uint8_t *out,
                               hipStream_t s);

}  // namespace hanf
