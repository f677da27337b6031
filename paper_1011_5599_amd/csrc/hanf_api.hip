// C ABI of the HyperANF library (declared in include/hanf.h): context management, graph
// ingest and schedule construction, the host side of the iteration loop, checkpoints and
// statistics. Every computation on graph data runs in the HIP kernels of hanf_kernels.hip;
// this layer validates arguments, owns device memory and orders launches on the stream.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstddef>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "hanf.h"
#include "hanf_internal.h"

using namespace hanf;

// Device memory of hanf_batch_stats_all_noalloc: the per-component statistics records are
// staged here instead of in an allocation. One copy per device, held until the process
// ends. Host code must not use this name as a device address: every use goes through the
// address hipGetSymbolAddress returns on that device (g_scratch_dev).
static __device__ __align__(256) StatsRec scratch[HANF_NOALLOC_MAX_COMPONENTS];

namespace {

constexpr int kMaxDevices = 64;

// Bytes of the modified-flag summary: one per 2^kSumShift nodes (2^(kSumShift-6) blocks),
// padded to a multiple of 4.
int64_t sum_bytes(int64_t n_blocks) {
  const int64_t per = (int64_t)1 << (kSumShift - 6);
  return ((n_blocks + per - 1) / per + 3) / 4 * 4;
}
std::mutex g_scratch_mu;
StatsRec *g_scratch_dev[kMaxDevices] = {};  // device address of `scratch` on each device
hipError_t g_scratch_err[kMaxDevices] = {};  // the lookup's result where it failed

// Looks up the device address of `scratch` on `device` once (the device must be current).
void scratch_setup(int device) {
  if (device < 0 || device >= kMaxDevices) return;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch_dev[device]) return;
  void *p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e == hipSuccess && p) {
    g_scratch_dev[device] = static_cast<StatsRec *>(p);
    g_scratch_err[device] = hipSuccess;
  } else {
    (void)hipGetLastError();
    g_scratch_err[device] = e != hipSuccess ? e : hipErrorInvalidSymbol;
  }
}

StatsRec *scratch_of(int device, hipError_t *err) {
  if (device < 0 || device >= kMaxDevices) {
    *err = hipErrorInvalidDevice;
    return nullptr;
  }
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  *err = g_scratch_err[device];
  return g_scratch_dev[device];
}

}  // namespace

namespace {

thread_local std::string g_thread_error;

// Published HyperLogLog bias constants (the paper defers alpha_m to the HyperLogLog paper).
double alpha_for(int m) {
  if (m == 16) return 0.673;
  if (m == 32) return 0.697;
  if (m == 64) return 0.709;
  return 0.7213 / (1.0 + 1.079 / m);
}

struct Schedule {
  int G = 0;          // lanes per node row the schedule was built for
  int lane_bytes = 0; // bytes per lane of the register format (partial rows)
  int32_t light_max = 0, chunk_arcs = 0, tile_nodes = 0;
  int32_t tile_base = 0;   // nodes per light tile without staging (option or default)
  int32_t stage_tile = 0;  // nodes per light tile when staging (0: the format cannot stage)
  int stage_opt = 0;       // HANF_OPT_STAGE the schedule was built with
  int unroll = 4;              // loads in flight per lane in the union kernels
  int stage = 0;           // light tiles stage their rows in LDS (passes over every successor)
  int32_t lds_wave_bytes = 0;
  int32_t n_tiles = 0, n_chunks = 0, n_heavy = 0;
  int32_t n_chunk_wgs = 0, n_light_wgs = 0, n_fin_wgs = 0;
  int32_t *light = nullptr;
  Chunk *chunks = nullptr;
  Heavy *heavy = nullptr;
  uint8_t *partial = nullptr;
  uint8_t *partial_any = nullptr;
  uint8_t *tile_todo = nullptr;   // systolic flags of the light tiles
  int32_t *unit_list = nullptr;   // systolic work units
  int64_t *stat_slots = nullptr;  // kStatSlots x 4 work counters
};

}  // namespace

struct hanf_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  std::string err;
  int fail_alloc_at = 0;  // test hook (HANF_TEST_FAIL_ALLOC): make that allocation fail
  int alloc_count = 0;
  std::multimap<size_t, void *> pool;  // released device buffers, reused by exact size
  std::map<void *, size_t> sizes;      // byte size of every live or pooled buffer

  // options
  int frontier = 1;
  int64_t max_passes_opt = 0;
  int32_t light_max_opt = 0, chunk_opt = 0, tile_opt = 0;
  int timing = 0;
  int dense_div = 4;  // a pass after one that changed >= n/dense_div counters maximises with all successors
  int passes_per_check = 4;
  int unroll = 0;  // loads in flight per lane in the gather loops (option 100); 0: automatic
  int sys_div = 4;    // a pass after one that changed < n/sys_div counters is systolic (0 = never)
  int union_policy = 0;  // 0: persistent union kernel for systolic passes, 1: never, 2: always
  int packed_opt = 2;    // HANF_OPT_PACKED5: 0 bytes, 1 5-bit registers, 2 chosen by row width
  int tp_counting = 0;   // 1: build transposes by per-node counters even below kTpMaxNodes
  int64_t hubs_opt = -1; // HANF_OPT_HUBS: -1 auto, 0 the caller's order, K: up to K hubs first
  int stage_opt = 0;     // HANF_OPT_STAGE: 0 never, 1 whenever the format allows
  int32_t stage_bytes = kStageWaveBytes;  // LDS per wavefront for a staged tile's counters
  int count_near = 0;    // 1: instrumented union kernels count near successors (option 104)
  int forward = 0;       // HANF_OPT_FORWARD: systolic passes without a transposed graph
  bool sys_seen = false; // the last state read showed a systolic next pass
  bool first_enqueued = false;  // the first pass of the run (always over every successor) is queued

  // graph
  int32_t n = 0;
  int64_t arcs = 0;
  const int32_t *rp = nullptr, *ci = nullptr;
  int32_t *rp_own = nullptr, *ci_own = nullptr;
  bool graph_ok = false;
  // transposed graph (systolic passes): owned, or the caller's device arrays
  const int32_t *trp = nullptr, *tci = nullptr;
  int32_t *trp_own = nullptr, *tci_own = nullptr;
  // node order chosen at the first initialisation after ingest (single graphs): the graph
  // and its transpose above are then in that order, row v holding the caller's node perm[v]
  bool ordered = false;  // the order of this ingest is decided
  int32_t inits = 0;     // initialisations since ingest
  int32_t *perm = nullptr, *inv = nullptr;  // new id -> caller's id, and back; NULL: the same
  int32_t n_hubs = 0;                        // the order's hubs (new ids 0 .. n_hubs - 1)

  Schedule sch;

  // batched graph. Base (from ingest): every graph once, side by side, 64-node aligned.
  // Layout (chosen at initialisation, once m is known): rows of S = 2^sl counters, and
  // `copies` copies of every graph when its seeds need more than one row.
  bool batch = false;
  int32_t n_graphs = 0, n_seeds = 0, n_comp = 0, n_lay = 0;
  int32_t base_n = 0;
  int64_t base_arcs = 0;
  std::vector<int32_t> g_node_off_h, g_n_h, g_aoff_h;      // per graph in the base
  int32_t *blk_comp = nullptr, *comp_node_off = nullptr, *comp_n = nullptr;  // base tables
  int32_t copies = 1;
  bool layout_ok = false;
  std::vector<int32_t> lay_node_off_h, lay_n_h, comp_row_h;
  int32_t *lay_blk = nullptr, *lay_node_off = nullptr, *lay_n = nullptr;  // tables of an expanded layout
  int32_t *rp_lay = nullptr, *ci_lay = nullptr, *trp_lay = nullptr, *tci_lay = nullptr;
  int seeds_row_opt = 0;  // 0: as many counters per row as fit (<= 32, S * m <= 1024 bytes)
  // batched run state
  uint64_t *comp_seed = nullptr;
  int32_t *blkcnt = nullptr, *comp_T = nullptr, *slot_comp = nullptr, *comp_row = nullptr;
  double *comp_nt = nullptr;
  std::vector<int32_t> slot_h, chunk0_h, cchunk_comp_h, cchunk_b0_h;  // row and reduction tables
  int32_t *comp_chunk0 = nullptr, *cchunk_comp = nullptr, *cchunk_b0 = nullptr;
  double *cchunk_sum = nullptr;
  int64_t *cchunk_cnt = nullptr;

  // run state
  int log2m = 0;
  int sl = 0;  // log2 of the counters per node row
  int packed = 0;  // the run's registers are 5-bit packed
  bool inited = false;
  uint8_t *regs[2] = {nullptr, nullptr};
  uint32_t *bits[2] = {nullptr, nullptr};
  uint8_t *mod_sum = nullptr;  // summary of the modified flags (PassArgs::mod_sum)
  uint8_t *todo = nullptr;                             // systolic signals, one byte per node
  int32_t *sig_list = nullptr, *sig_cnt = nullptr;     // signalled successors per node
  int32_t *sys_node = nullptr, *sys_pos = nullptr;     // systolic signal list
  double *est = nullptr, *blocksum = nullptr, *wgsum = nullptr, *lc = nullptr, *nt = nullptr;
  double *stats_out = nullptr;
  int64_t *wgcnt = nullptr;
  PassLog *log = nullptr;
  DevState *st = nullptr;
  DevState *st_host = nullptr;  // pinned
  bool st_fresh = false;  // st_host equals the device state: nothing queued since could change it
  double *nt_host = nullptr;  // pinned: N_hat(0 .. nt_host_len - 1), read with the state
  int32_t nt_host_len = 0;
  std::vector<int32_t> comp_T_host;  // batches: every component's fixpoint, read with the state
  bool comp_T_fresh = false;         // valid while st_fresh also holds
  DevState *st_poll = nullptr;  // pinned, written by the copy hanf_enqueue leaves on the stream
  PassLog *log_host = nullptr;  // pinned, kMaxPassesPerCheck records read with the state
  hipEvent_t poll_ev = nullptr;
  // per-kernel timing events of hanf_iterate, created once and reused by every batch of
  // passes (the host then creates and destroys none between batches)
  std::vector<hipEvent_t> ev_pool;
  bool poll_pending = false;
  int32_t nt_cap = 0, log_cap = 0, max_passes = 0, n_blocks = 0, n_reduce_wgs = 0;
  std::vector<double> lc_host;
  std::vector<hanf_pass_t> host_log;
  PassArgs args{};
};

namespace {

int fail(hanf_ctx *c, int code, const std::string &msg) {
  if (c)
    c->err = msg;
  else
    g_thread_error = msg;
  return code;
}

int hip_fail(hanf_ctx *c, hipError_t e, const char *what) {
  std::string msg = std::string(what) + ": " + hipGetErrorString(e);
  return fail(c, e == hipErrorOutOfMemory ? HANF_ENOMEM : HANF_EDEVICE, msg);
}

#define HIP_TRY(ctx, expr, what)           \
  do {                                     \
    hipError_t e_ = (expr);                \
    if (e_ != hipSuccess) return hip_fail(ctx, e_, what); \
  } while (0)

// Allocation sizes above 64 KiB are rounded up to size classes 2^k and 1.5 * 2^k, so that
// runs on graphs of different sizes can reuse each other's buffers (at most a third wasted).
size_t size_class(size_t bytes) {
  if (bytes <= (64u << 10)) return (bytes + 255) / 256 * 256;
  size_t p = 1;
  while (p < bytes) p <<= 1;
  const size_t mid = p / 2 + p / 4;
  return bytes <= mid ? mid : p;
}

// Device allocations go through a per-context pool: a released buffer is kept and handed
// out again for a request of the same size class, so repeated runs allocate nothing after
// the first (hipFree also waits for the whole device, which would stall other streams).
// Everything is returned to HIP at hanf_destroy.
template <typename T>
int dev_alloc(hanf_ctx *c, T **p, size_t count, const char *what) {
  *p = nullptr;
  c->alloc_count++;
  if (c->fail_alloc_at > 0 && c->alloc_count == c->fail_alloc_at)
    return fail(c, HANF_ENOMEM, std::string("forced allocation failure: ") + what);
  const size_t bytes = size_class(std::max<size_t>(count, 1) * sizeof(T));
  auto it = c->pool.find(bytes);
  if (it != c->pool.end()) {
    *p = static_cast<T *>(it->second);
    c->pool.erase(it);
    return HANF_OK;
  }
  void *q = nullptr;
  hipError_t e = hipMalloc(&q, bytes);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    // release pooled buffers and retry once
    for (auto &kv : c->pool) {
      c->sizes.erase(kv.second);
      (void)hipFree(kv.second);
    }
    c->pool.clear();
    e = hipMalloc(&q, bytes);
  }
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return fail(c, HANF_ENOMEM, std::string("hipMalloc failed for ") + what + ": " + hipGetErrorString(e));
  }
  c->sizes[q] = bytes;
  *p = static_cast<T *>(q);
  return HANF_OK;
}

// Returns a buffer to the context's pool (the pointer is cleared).
template <typename T>
void dev_release(hanf_ctx *c, T *&p) {
  if (p) {
    auto it = c->sizes.find((void *)p);
    if (it != c->sizes.end())
      c->pool.emplace(it->second, (void *)p);
    else
      (void)hipFree(p);
  }
  p = nullptr;
}

template <typename T>
void dev_free(T *&p) {
  if (p) (void)hipFree(p);
  p = nullptr;
}

void free_schedule(hanf_ctx *c) {
  Schedule &s = c->sch;
  dev_release(c, s.light);
  dev_release(c, s.chunks);
  dev_release(c, s.heavy);
  dev_release(c, s.partial);
  dev_release(c, s.partial_any);
  dev_release(c, s.tile_todo);
  dev_release(c, s.unit_list);
  dev_release(c, s.stat_slots);
  s = Schedule();
}

void free_run(hanf_ctx *c) {
  for (int i = 0; i < 2; ++i) {
    dev_release(c, c->regs[i]);
    dev_release(c, c->bits[i]);
  }
  dev_release(c, c->mod_sum);
  dev_release(c, c->est);
  dev_release(c, c->blocksum);
  dev_release(c, c->wgsum);
  dev_release(c, c->wgcnt);
  dev_release(c, c->lc);
  dev_release(c, c->nt);
  dev_release(c, c->log);
  dev_release(c, c->stats_out);
  dev_release(c, c->comp_seed);
  dev_release(c, c->blkcnt);
  dev_release(c, c->comp_T);
  dev_release(c, c->comp_nt);
  dev_release(c, c->slot_comp);
  dev_release(c, c->comp_row);
  dev_release(c, c->comp_chunk0);
  dev_release(c, c->cchunk_comp);
  dev_release(c, c->cchunk_b0);
  dev_release(c, c->cchunk_sum);
  dev_release(c, c->cchunk_cnt);
  dev_release(c, c->todo);
  dev_release(c, c->sig_list);
  dev_release(c, c->sig_cnt);
  dev_release(c, c->sys_node);
  dev_release(c, c->sys_pos);
  c->inited = false;
  c->log2m = 0;
  c->packed = 0;
}

// Drops an expanded batch layout (the base remains).
void free_layout(hanf_ctx *c) {
  dev_release(c, c->lay_blk);
  dev_release(c, c->lay_node_off);
  dev_release(c, c->lay_n);
  dev_release(c, c->rp_lay);
  dev_release(c, c->ci_lay);
  dev_release(c, c->trp_lay);
  dev_release(c, c->tci_lay);
  c->layout_ok = false;
  c->copies = 1;
}

void free_transpose(hanf_ctx *c) {
  dev_release(c, c->trp_own);
  dev_release(c, c->tci_own);
  dev_release(c, c->trp_lay);
  dev_release(c, c->tci_lay);
  c->trp = c->tci = nullptr;
}

void free_graph(hanf_ctx *c) {
  free_transpose(c);
  free_layout(c);
  dev_release(c, c->perm);
  dev_release(c, c->inv);
  c->n_hubs = 0;
  c->ordered = false;
  c->inits = 0;
  dev_release(c, c->rp_own);
  dev_release(c, c->ci_own);
  dev_release(c, c->blk_comp);
  dev_release(c, c->comp_node_off);
  dev_release(c, c->comp_n);
  c->batch = false;
  c->n_graphs = c->n_seeds = c->n_comp = c->n_lay = 0;
  c->base_n = 0;
  c->base_arcs = 0;
  c->g_node_off_h.clear();
  c->g_n_h.clear();
  c->g_aoff_h.clear();
  c->lay_node_off_h.clear();
  c->lay_n_h.clear();
  c->comp_row_h.clear();
  c->rp = c->ci = nullptr;
  c->graph_ok = false;
  c->n = 0;
  c->arcs = 0;
}

// After batched ingest: the base (every graph once) is the graph until initialisation
// chooses the row layout.
void set_base(hanf_ctx *c, const std::vector<int32_t> &node_off, const std::vector<int32_t> &n,
              const std::vector<int32_t> &arc_off) {
  c->rp = c->rp_own;
  c->ci = c->ci_own;
  c->g_node_off_h = node_off;
  c->g_n_h = n;
  c->g_aoff_h = arc_off;
  c->base_n = c->n;
  c->base_arcs = c->arcs;
  c->lay_node_off_h = node_off;
  c->lay_n_h = n;
  c->copies = 1;
  c->layout_ok = true;
  c->graph_ok = true;
}

int sync(hanf_ctx *c, const char *what) {
  hipError_t e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) return hip_fail(c, e, what);
  return HANF_OK;
}

int read_state(hanf_ctx *c) {
  c->st_fresh = false;
  c->comp_T_fresh = false;
  HIP_TRY(c, hipMemcpyAsync(c->st_host, c->st, sizeof(DevState), hipMemcpyDeviceToHost, c->stream),
          "state read");
  const int rc = sync(c, "state read");
  c->st_fresh = rc == HANF_OK;
  return rc;
}

// A state reset whose result the host reads back before using it.
hipError_t reset_state_unread(hanf_ctx *c) {
  c->st_fresh = false;
  c->nt_host_len = 0;
  return launch_state_reset(c->st, 0, c->frontier, 1, 0, 0, c->stream);
}

// The run state, read from the device unless the host copy is current.
int current_state(hanf_ctx *c) { return c->st_fresh ? HANF_OK : read_state(c); }

// N_hat values kept on the host with the state (a prefix of the history).
constexpr int32_t kNtHostCache = 1024;

// The state k_state_reset writes (the host copy is current once it ran, as long as nothing
// queued after it changes the state).
void mirror_state_reset(hanf_ctx *c, int32_t t, int32_t max_passes, int64_t dense_threshold, int32_t sys_div) {
  DevState &s = *c->st_host;
  s.t = t;
  s.halted = 0;
  s.done = 0;
  s.capped = 0;
  s.first_pass = 1;
  s.frontier = c->frontier;
  s.max_passes = max_passes;
  s.passes = 0;
  s.err = 0;
  s.changed_last = -1;
  s.dense_next = 0;
  s.dense_threshold = dense_threshold;
  s.systolic = 0;
  s.sys_div = sys_div;
  s.sys_acc = 0ull;
  s.sys_units = 0;
  s.use_sum = 0;
  c->st_fresh = true;
  c->comp_T_fresh = false;
}

// Batches: the run state and every component's fixpoint T, from the device unless the host
// copies are current (one wait for all the components a caller then reads).
int batch_state(hanf_ctx *c) {
  if (c->st_fresh && c->comp_T_fresh && (int32_t)c->comp_T_host.size() == c->n_comp) return HANF_OK;
  c->st_fresh = false;
  c->comp_T_fresh = false;
  c->comp_T_host.resize((size_t)c->n_comp);
  HIP_TRY(c, hipMemcpyAsync(c->comp_T_host.data(), c->comp_T, sizeof(int32_t) * c->n_comp, hipMemcpyDeviceToHost,
                            c->stream),
          "fixpoint read");
  HIP_TRY(c, hipMemcpyAsync(c->st_host, c->st, sizeof(DevState), hipMemcpyDeviceToHost, c->stream), "state read");
  const int rc = sync(c, "state read");
  c->st_fresh = c->comp_T_fresh = rc == HANF_OK;
  return rc;
}

// Default schedule parameters for G lanes per counter (W = 64/G slots per wavefront).
void choose_schedule(hanf_ctx *c, int G, int lane_bytes, Schedule &s) {
  const int W = kWave / G;
  s.G = G;
  s.lane_bytes = lane_bytes;
  // defaults measured on MI355X over light_max 16..128 and chunk_arcs 256..2048: one arc per
  // register of the row (clamped to 32..128) and 16 arcs per slot and unrolled gather in a
  // chunk
  const int row_regs = G * (lane_bytes == kPacked5LaneBytes ? 64 : 16);
  s.light_max = c->light_max_opt > 0 ? c->light_max_opt : std::max(32, std::min(128, row_regs));
  // loads in flight per lane: 8 for byte registers (at 80 VGPRs or fewer, so 6 wavefronts per
  // SIMD still fit), 4 for 5-bit ones (ten VGPRs a counter) and for the staged and
  // instrumented kernels, which exist for 4 only
  s.unroll = c->unroll > 0 ? c->unroll : (lane_bytes != 16 || c->stage_opt == 1 || c->count_near) ? 4 : 8;
  s.chunk_arcs = c->chunk_opt > 0 ? c->chunk_opt : std::max(256, std::min(2048, W * s.unroll * 16));
  int32_t tile = c->tile_opt;
  if (tile <= 0) {
    // about 8 rounds of W nodes per wavefront on large graphs (measured best on MI355X for
    // m = 64 and 128), fewer on small graphs so that the chip still gets many wavefronts
    int64_t rounds = (int64_t)c->n / ((int64_t)W * 2048);
    rounds = std::max<int64_t>(1, std::min<int64_t>({rounds, (int64_t)8, (int64_t)(kMaxTile / W)}));
    tile = (int32_t)(rounds * W);
  }
  tile = std::max(W, std::min(kMaxTile, (tile / W) * W));
  s.tile_base = s.tile_nodes = tile;
  // staged tiles: as many rows as kStageWaveBytes of LDS hold, at least one round of W
  const int32_t row_bytes = G * lane_bytes;
  const int32_t st = std::min(kMaxTile, (c->stage_bytes / row_bytes) / W * W);
  s.stage_tile = (lane_bytes == 16 && G <= 16 && s.unroll == 4 && st >= W) ? st : 0;
  s.stage_opt = c->stage_opt;
}

int build_schedule(hanf_ctx *c, int G, int lane_bytes) {
  free_schedule(c);
  Schedule &s = c->sch;
  choose_schedule(c, G, lane_bytes, s);
  const int32_t n = c->n;
  int rc;
  // chunk counts, prefix sums, chunk and heavy lists
  uint64_t *keys = nullptr, *tmp = nullptr;
  if ((rc = dev_alloc(c, &keys, (size_t)n + 1, "schedule keys"))) return rc;
  if ((rc = dev_alloc(c, &tmp, (size_t)scan_tmp_elems((int64_t)n + 1), "scan scratch"))) {
    dev_release(c, keys);
    return rc;
  }
  hipError_t e = launch_classify(c->rp, n, s.light_max, s.chunk_arcs, keys, c->stream);
  if (e == hipSuccess) e = launch_exclusive_scan_u64(keys, (int64_t)n + 1, tmp, c->stream);
  uint64_t total[1] = {0};
  if (e == hipSuccess) e = hipMemcpyAsync(total, keys + n, sizeof(uint64_t), hipMemcpyDeviceToHost, c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) {
    dev_release(c, keys);
    dev_release(c, tmp);
    return hip_fail(c, e, "schedule scan");
  }
  s.stage = s.stage_tile > 0 && s.stage_opt == 1;
  if (s.stage) s.tile_nodes = s.stage_tile;
  {
    // One launch holds fewer than 2^32 threads: the union step runs a wavefront per work
    // unit (chunk or light tile) and the tile builder a workgroup of at least a wavefront
    // per tile. Only very small tiles or chunks on graphs of ~10^9 nodes or arcs exceed it.
    const int64_t chunks = (int64_t)(total[0] >> 32);
    const int64_t tiles = ((int64_t)n + s.tile_nodes - 1) / s.tile_nodes;
    int64_t width = kWave;
    while (width < s.tile_nodes) width <<= 1;
    const int64_t most = (int64_t)1 << 32;
    if ((chunks + tiles + 40) * kWave >= most || tiles * width >= most) {
      dev_release(c, keys);
      dev_release(c, tmp);
      return fail(c, HANF_EINVAL,
                  "schedule too large for one launch: raise HANF_OPT_TILE_NODES or HANF_OPT_CHUNK_ARCS");
    }
  }
  s.n_chunks = (int32_t)(total[0] >> 32);
  s.n_heavy = (int32_t)(total[0] & 0xffffffffull);
  s.lds_wave_bytes = s.stage ? s.tile_nodes * G * lane_bytes : ((s.tile_nodes * 4 + 15) / 16) * 16;
  s.n_tiles = (int32_t)(((int64_t)n + s.tile_nodes - 1) / s.tile_nodes);
  if ((rc = dev_alloc(c, &s.light, (size_t)s.n_tiles * s.tile_nodes, "light tiles"))) {
    dev_release(c, keys);
    dev_release(c, tmp);
    return rc;
  }
  e = launch_build_tiles(c->rp, n, s.light_max, s.tile_nodes, s.n_tiles, s.light, c->stream);
  if (e != hipSuccess) {
    dev_release(c, keys);
    dev_release(c, tmp);
    return hip_fail(c, e, "build tiles");
  }
  const size_t row_bytes = (size_t)G * s.lane_bytes;
  if ((rc = dev_alloc(c, &s.chunks, (size_t)s.n_chunks, "chunks")) ||
      (rc = dev_alloc(c, &s.heavy, (size_t)s.n_heavy, "heavy nodes")) ||
      (rc = dev_alloc(c, &s.partial, (size_t)s.n_chunks * row_bytes, "chunk partials")) ||
      (rc = dev_alloc(c, &s.partial_any, (size_t)s.n_chunks, "chunk flags"))) {
    dev_release(c, keys);
    dev_release(c, tmp);
    return rc;
  }
  e = launch_fill_chunks(c->rp, n, keys, s.chunk_arcs, s.chunks, s.heavy, c->stream);
  dev_release(c, keys);  // pooled: reused only by work queued later on the same stream
  dev_release(c, tmp);
  if (e != hipSuccess) return hip_fail(c, e, "fill chunks");
  s.n_chunk_wgs = (s.n_chunks + 3) / 4;
  s.n_chunk_wgs = ((s.n_chunk_wgs + kXcds - 1) / kXcds) * kXcds;  // light workgroups start on XCD 0
  s.n_light_wgs = (s.n_tiles + 3) / 4;
  s.n_fin_wgs = (s.n_heavy + 3) / 4;
  if ((rc = dev_alloc(c, &s.stat_slots, (size_t)kStatSlots * kStatFields, "work counters")) ||
      (rc = dev_alloc(c, &s.tile_todo, ((size_t)s.n_tiles + 3) / 4 * 4, "tile flags")) ||
      (rc = dev_alloc(c, &s.unit_list, (size_t)s.n_chunks + s.n_tiles, "work unit list")))
    return rc;
  return HANF_OK;
}

void fill_args(hanf_ctx *c) {
  PassArgs &a = c->args;
  a.row_ptr = c->rp;
  a.col_idx = c->ci;
  a.regs0 = c->regs[0];
  a.regs1 = c->regs[1];
  a.bits0 = c->bits[0];
  a.bits1 = c->bits[1];
  a.mod_sum = c->mod_sum;
  a.n_sum = sum_bytes(c->n_blocks);
  a.est = c->est;
  a.blocksum = c->blocksum;
  a.wgsum = c->wgsum;
  a.wgcnt = c->wgcnt;
  a.stat_slots = c->sch.stat_slots;
  a.light = c->sch.light;
  a.chunks = c->sch.chunks;
  a.heavy = c->sch.heavy;
  a.partial = c->sch.partial;
  a.partial_any = c->sch.partial_any;
  a.tile_todo = c->sch.tile_todo;
  a.unit_list = c->sch.unit_list;
  const bool sys = c->trp && c->todo;
  const bool lay_t = c->batch && c->copies > 1;  // the transposed graph of the expanded layout
  a.trow_ptr = sys ? (lay_t ? c->trp_lay : c->trp) : nullptr;
  a.tcol_idx = sys ? (lay_t ? c->tci_lay : c->tci) : nullptr;
  a.todo = c->todo;
  a.sys_node = c->sys_node;
  a.sys_pos = c->sys_pos;
  a.sig_list = c->sig_list;
  a.sig_cnt = c->sig_cnt;
  a.st = c->st;
  a.nt = c->nt;
  a.log = c->log;
  a.lc = c->lc;
  const int m = 1 << c->log2m;
  a.K = alpha_for(m) * m * m * 2147483648.0;
  a.n = c->n;
  a.log2m = c->log2m;
  a.seed_log2 = c->sl;
  a.packed = c->packed;
  a.gs = c->packed ? 1 << (c->log2m - 6) : 1 << (c->log2m - 4);
  a.n_blocks = c->n_blocks;
  a.n_chunks = c->sch.n_chunks;
  a.n_chunk_wgs = c->sch.n_chunk_wgs;
  a.n_light_wgs = c->sch.n_light_wgs;
  a.n_tiles = c->sch.n_tiles;
  a.tile_nodes = c->sch.tile_nodes;
  a.light_max = c->sch.light_max;
  a.stage = c->sch.stage;
  // the instrumented kernels exist where staging could run (byte rows up to 256 bytes, 4 loads
  // in flight); elsewhere near successors are not counted
  a.count_near = (c->count_near && c->sch.stage_tile > 0) ? 1 : 0;
  a.lds_wave_bytes = c->sch.lds_wave_bytes;
  // rows one XCD's 4 MiB L2 holds, half on either side of the node (see the pass record)
  const int64_t rb = (int64_t)c->sch.G * c->sch.lane_bytes;  // 0 until a schedule is built
  a.near_window = rb > 0 ? (int32_t)std::max<int64_t>(1, (int64_t)(kL2Bytes / 2) / rb) : 1;
  a.n_heavy = c->sch.n_heavy;
  a.n_fin_wgs = c->sch.n_fin_wgs;
  a.n_reduce_wgs = c->n_reduce_wgs;
  a.nt_cap = c->nt_cap;
  a.log_cap = c->log_cap;
  a.arcs = c->arcs;
  a.node_id = c->batch ? nullptr : c->perm;
  a.batch.active = c->batch ? 1 : 0;
  a.batch.n_comp = c->n_comp;
  a.batch.n_lay = c->n_lay;
  const bool lay = c->batch && c->copies > 1;
  a.batch.blk_comp = lay ? c->lay_blk : c->blk_comp;
  a.batch.comp_node_off = lay ? c->lay_node_off : c->comp_node_off;
  a.batch.comp_n = lay ? c->lay_n : c->comp_n;
  a.batch.slot_comp = c->slot_comp;
  a.batch.comp_row = c->comp_row;
  a.batch.comp_chunk0 = c->comp_chunk0;
  a.batch.cchunk_comp = c->cchunk_comp;
  a.batch.cchunk_b0 = c->cchunk_b0;
  a.batch.cchunk_sum = c->cchunk_sum;
  a.batch.cchunk_cnt = c->cchunk_cnt;
  a.batch.n_cchunks = (int32_t)c->cchunk_comp_h.size();
  a.batch.comp_seed = c->comp_seed;
  a.batch.blkcnt = c->blkcnt;
  a.batch.comp_T = c->comp_T;
  a.batch.comp_nt = c->comp_nt;
}

// Per-component N_hat histories of a batch are kept within this many bytes when the pass cap
// is the default.
constexpr int64_t kBatchHistoryBytes = 64 << 20;

// Passes allowed before HANF_EMAXITER: the option, else n + 1 for one graph (T is below the
// number of nodes). For a batch, the largest graph's n + 1, so every component stops as it
// would alone; its histories hold cap + 2 values per component, so the cap is lowered to
// what kBatchHistoryBytes holds, but never below 1024 passes.
int64_t default_max_passes(const hanf_ctx *c) {
  if (c->max_passes_opt > 0) return c->max_passes_opt;
  if (!c->batch) return (int64_t)c->n + 1;
  int64_t nmax = 1;
  for (int32_t g : c->g_n_h) nmax = std::max<int64_t>(nmax, g);
  const int64_t fits = kBatchHistoryBytes / 8 / std::max<int64_t>(1, c->n_comp) - 2;
  return std::min<int64_t>(nmax + 1, std::max<int64_t>(1024, fits));
}

// Packed registers move through a device staging buffer of at most this many 64-register
// groups (64 MiB unpacked) when the caller's buffer is in host memory.
constexpr int64_t kStageGroups = 1 << 20;

// The counters in `src` (the run's format) as one byte per register: n * m bytes at `out`.
int regs_to_bytes(hanf_ctx *c, const uint8_t *src, uint8_t *out, uint32_t flags) {
  const size_t bytes = (size_t)c->n << c->log2m;
  if (!c->packed) {
    HIP_TRY(c, hipMemcpyAsync(out, src, bytes,
                              flags == HANF_DEVICE_PTRS ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, c->stream),
            "register read");
    return sync(c, "register read");
  }
  const int64_t groups = (int64_t)(bytes / 64);
  if (flags == HANF_DEVICE_PTRS) {
    HIP_TRY(c, launch_unpack5(src, out, groups, c->stream), "register unpack");
    return sync(c, "register read");
  }
  const int64_t chunk = std::min<int64_t>(groups, kStageGroups);
  uint8_t *stage = nullptr;
  int rc;
  if ((rc = dev_alloc(c, &stage, (size_t)chunk * 64, "register staging"))) return rc;
  hipError_t e = hipSuccess;
  for (int64_t g0 = 0; g0 < groups && e == hipSuccess; g0 += chunk) {
    const int64_t cnt = std::min(chunk, groups - g0);
    e = launch_unpack5(src + g0 * kPacked5LaneBytes, stage, cnt, c->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(out + g0 * 64, stage, (size_t)cnt * 64, hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  }
  dev_release(c, stage);
  if (e != hipSuccess) return hip_fail(c, e, "register read");
  return HANF_OK;
}

// One byte per register (n * m bytes at `in`, each <= 31) into `dst` in the run's format.
// Sets DevState::err (16) when a register is above 31; the caller reads the state.
int bytes_to_regs(hanf_ctx *c, const uint8_t *in, uint8_t *dst, uint32_t flags) {
  const size_t bytes = (size_t)c->n << c->log2m;
  const hipMemcpyKind kind = flags == HANF_DEVICE_PTRS ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
  if (!c->packed) {
    HIP_TRY(c, hipMemcpyAsync(dst, in, bytes, kind, c->stream), "register upload");
    HIP_TRY(c, launch_check_registers(dst, (int64_t)bytes, c->st, c->stream), "register check");
    return HANF_OK;
  }
  const int64_t groups = (int64_t)(bytes / 64);
  if (flags == HANF_DEVICE_PTRS) {
    HIP_TRY(c, launch_check_registers(in, (int64_t)bytes, c->st, c->stream), "register check");
    HIP_TRY(c, launch_pack5(in, dst, groups, c->stream), "register pack");
    return HANF_OK;
  }
  const int64_t chunk = std::min<int64_t>(groups, kStageGroups);
  uint8_t *stage = nullptr;
  int rc;
  if ((rc = dev_alloc(c, &stage, (size_t)chunk * 64, "register staging"))) return rc;
  hipError_t e = hipSuccess;
  for (int64_t g0 = 0; g0 < groups && e == hipSuccess; g0 += chunk) {
    const int64_t cnt = std::min(chunk, groups - g0);
    e = hipMemcpyAsync(stage, in + g0 * 64, (size_t)cnt * 64, hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess) e = launch_check_registers(stage, cnt * 64, c->st, c->stream);
    if (e == hipSuccess) e = launch_pack5(stage, dst + g0 * kPacked5LaneBytes, cnt, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);  // the staging buffer is reused
  }
  dev_release(c, stage);
  if (e != hipSuccess) return hip_fail(c, e, "register upload");
  return HANF_OK;
}

// Bytes of one node's row of counters: S counters of m bytes, or one of 5m/8 bytes (packed).
size_t row_bytes(int log2m, int sl, int packed) {
  return (packed ? ((size_t)kPacked5LaneBytes << (log2m - 6)) : ((size_t)1 << log2m)) << sl;
}

bool device_pointer(const hanf_ctx *c, const void *p) {
  hipPointerAttribute_t attr;
  const hipError_t e = hipPointerGetAttributes(&attr, p);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return false;
  }
  return attr.type == hipMemoryTypeDevice && attr.device == c->device;
}

// (rp, ci) with rows and targets in the node order of perm / inv, into new buffers of the
// context's pool (queued on the stream; the caller synchronises).
int permute_graph(hanf_ctx *c, const int32_t *rp, const int32_t *ci, int32_t **rp_new, int32_t **ci_new) {
  const int32_t n = c->n;
  const int64_t arcs = c->arcs;
  uint64_t *keys = nullptr, *tmp = nullptr;
  uint4 *rec = nullptr;
  int32_t *hub_new = nullptr, *wrow = nullptr;
  int rc;
  if ((rc = dev_alloc(c, rp_new, (size_t)n + 1, "reordered row_ptr")) ||
      (rc = dev_alloc(c, ci_new, (size_t)arcs, "reordered col_idx")) ||
      (rc = dev_alloc(c, &keys, (size_t)n + 1, "reorder keys")) ||
      (rc = dev_alloc(c, &tmp, (size_t)scan_tmp_elems((int64_t)n + 1), "scan scratch")) ||
      (rc = dev_alloc(c, &rec, (size_t)rename_groups(n), "renaming table")) ||
      (rc = dev_alloc(c, &hub_new, (size_t)std::max(c->n_hubs, 1), "renaming table")) ||
      (rc = dev_alloc(c, &wrow, (size_t)permute_windows(arcs) + 1, "reorder windows"))) {
    dev_release(c, *rp_new);
    dev_release(c, *ci_new);
    dev_release(c, keys);
    dev_release(c, tmp);
    dev_release(c, rec);
    dev_release(c, hub_new);
    dev_release(c, wrow);
    return rc;
  }
  const hipError_t e = launch_permute_csr(rp, ci, n, arcs, c->perm, c->inv, c->n_hubs, keys, tmp, rec, hub_new,
                                          wrow, *rp_new, *ci_new, c->stream);
  dev_release(c, keys);  // pooled: reused only by work queued later on the same stream
  dev_release(c, tmp);
  dev_release(c, rec);
  dev_release(c, hub_new);
  dev_release(c, wrow);
  if (e != hipSuccess) {
    dev_release(c, *rp_new);
    dev_release(c, *ci_new);
    return hip_fail(c, e, "graph reorder");
  }
  return HANF_OK;
}

// Rows of the K most-read counters (the hubs: largest in-degree) fit one XCD's L2 together.
constexpr int64_t kHubCacheBytes = 4 << 20;
// The order gains only where rows are shorter than an L2 line (hubs then share lines); at a
// line or more per row, passes over every node run no faster (measured at m = 128).
constexpr int64_t kL2LineBytes = 128;

// Chooses the node order of a single graph once per ingest (HANF_OPT_HUBS): with K > 0,
// hubs first (by class of in-degree, then id) and the other nodes after them in id order;
// the graph and its transpose are rewritten in that order. Auto: K rows fill kHubCacheBytes,
// for rows shorter than an L2 line and graphs with at least 16 K nodes whose transposed
// graph gives the in-degrees, chosen at the second initialisation on the ingest (the
// rewrite costs about 70% of a pass over every node, which a second run earns back; a
// single run gains little more than the rewrite, so it keeps the caller's order).
int order_nodes(hanf_ctx *c, int32_t log2m, int packed) {
  c->ordered = true;
  const int32_t n = c->n;
  const int64_t arcs = c->arcs;
  int64_t K = c->hubs_opt;
  if (K < 0) {
    const int64_t rb = (int64_t)row_bytes(log2m, 0, packed);
    K = kHubCacheBytes / rb;
    if (!c->trp || rb >= kL2LineBytes || (int64_t)n < 16 * K) K = 0;
  }
  K = std::min<int64_t>(K, n);
  if (K == 0 || arcs == 0) return HANF_OK;
  const bool self_t = c->trp && c->trp == c->rp;
  uint32_t *deg = nullptr, *hist = nullptr;
  int32_t *plan = nullptr;
  uint64_t *counts = nullptr, *tmp = nullptr;
  const int64_t ncnt = order_counts_elems(n);
  int rc;
  if ((rc = dev_alloc(c, &c->perm, (size_t)n, "node order")) || (rc = dev_alloc(c, &c->inv, (size_t)n, "node order")) ||
      (rc = dev_alloc(c, &deg, (size_t)n, "in-degrees")) ||
      (rc = dev_alloc(c, &hist, (size_t)kOrderLevels, "in-degree classes")) ||
      (rc = dev_alloc(c, &plan, 1, "order plan")) || (rc = dev_alloc(c, &counts, (size_t)ncnt, "order counts")) ||
      (rc = dev_alloc(c, &tmp, (size_t)scan_tmp_elems(ncnt), "scan scratch"))) {
    dev_release(c, c->perm);
    dev_release(c, c->inv);
    dev_release(c, deg);
    dev_release(c, hist);
    dev_release(c, plan);
    dev_release(c, counts);
    dev_release(c, tmp);
    return rc;
  }
  hipError_t e = launch_in_degrees(c->trp, c->ci, n, arcs, deg, c->stream);
  if (e == hipSuccess) e = launch_order_select(deg, n, K, hist, plan, counts, tmp, c->perm, c->inv, c->stream);
  int32_t lstar = 0;  // kOrderLevels: no class of in-degree fits under K, the order is the caller's
  uint64_t hubs = 0;  // the first new id of the other nodes: the count of hubs
  if (e == hipSuccess) e = hipMemcpyAsync(&lstar, plan, sizeof(int32_t), hipMemcpyDeviceToHost, c->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(&hubs, counts + (int64_t)kOrderRest * (ncnt / kOrderClasses), sizeof(uint64_t),
                       hipMemcpyDeviceToHost, c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  c->n_hubs = (int32_t)hubs;
  dev_release(c, deg);
  dev_release(c, hist);
  dev_release(c, plan);
  dev_release(c, counts);
  dev_release(c, tmp);
  if (e == hipSuccess && lstar >= kOrderLevels) {
    dev_release(c, c->perm);
    dev_release(c, c->inv);
    return HANF_OK;
  }
  int32_t *rp_new = nullptr, *ci_new = nullptr, *trp_new = nullptr, *tci_new = nullptr;
  if (e != hipSuccess) rc = hip_fail(c, e, "node order");
  if (!rc) rc = permute_graph(c, c->rp, c->ci, &rp_new, &ci_new);
  if (!rc && c->trp && !self_t) rc = permute_graph(c, c->trp, c->tci, &trp_new, &tci_new);
  if (!rc && (e = hipStreamSynchronize(c->stream)) != hipSuccess) rc = hip_fail(c, e, "node order");
  if (rc) {
    (void)hipStreamSynchronize(c->stream);
    dev_release(c, rp_new);
    dev_release(c, ci_new);
    dev_release(c, trp_new);
    dev_release(c, tci_new);
    dev_release(c, c->perm);
    dev_release(c, c->inv);
    return rc;
  }
  // the reordered graph replaces the caller's arrays (or their copy)
  dev_release(c, c->rp_own);
  dev_release(c, c->ci_own);
  c->rp = c->rp_own = rp_new;
  c->ci = c->ci_own = ci_new;
  if (self_t) {
    c->trp = rp_new;
    c->tci = ci_new;
  } else if (c->trp) {
    dev_release(c, c->trp_own);
    dev_release(c, c->tci_own);
    c->trp = c->trp_own = trp_new;
    c->tci = c->tci_own = tci_new;
  }
  return HANF_OK;
}

int alloc_run(hanf_ctx *c, int log2m, int sl, int packed) {
  free_run(c);
  const int m = 1 << log2m;
  const size_t S = (size_t)1 << sl;  // counters per node row
  const size_t bytes = (size_t)c->n * row_bytes(log2m, sl, packed);
  c->n_blocks = (int32_t)(((int64_t)c->n + kNodesPerBlock - 1) / kNodesPerBlock);
  c->n_reduce_wgs = (c->n_blocks + kReduceBlocks - 1) / kReduceBlocks;
  c->max_passes = (int32_t)std::min<int64_t>(default_max_passes(c), INT32_MAX - 8);
  c->nt_cap = c->max_passes + 2;
  c->log_cap = std::min(c->nt_cap, kMaxLogRecords);
  int rc;
  if ((rc = dev_alloc(c, &c->regs[0], bytes, "counters")) || (rc = dev_alloc(c, &c->regs[1], bytes, "counters")) ||
      (rc = dev_alloc(c, &c->bits[0], (size_t)2 * c->n_blocks * S, "flags")) ||
      (rc = dev_alloc(c, &c->bits[1], (size_t)2 * c->n_blocks * S, "flags")) ||
      (rc = dev_alloc(c, &c->mod_sum, (size_t)sum_bytes(c->n_blocks), "flag summary")) ||
      (rc = dev_alloc(c, &c->est, (size_t)c->n * S, "estimates")) ||
      (rc = dev_alloc(c, &c->blocksum, (size_t)c->n_blocks * S, "block sums")) ||
      (rc = dev_alloc(c, &c->wgsum, (size_t)c->n_reduce_wgs, "partial sums")) ||
      (rc = dev_alloc(c, &c->wgcnt, (size_t)c->n_reduce_wgs, "partial counts")) ||
      (rc = dev_alloc(c, &c->lc, (size_t)m + 1, "linear-counting table")) ||
      (rc = dev_alloc(c, &c->nt, (size_t)c->nt_cap, "N history")) ||
      (rc = dev_alloc(c, &c->log, (size_t)c->log_cap, "pass log")) ||
      (rc = dev_alloc(c, &c->stats_out, 16, "statistics"))) {
    free_run(c);
    return rc;
  }
  if (c->batch) {
    if ((rc = dev_alloc(c, &c->comp_seed, (size_t)c->n_comp, "component seeds")) ||
        (rc = dev_alloc(c, &c->blkcnt, (size_t)c->n_blocks * S, "block change counts")) ||
        (rc = dev_alloc(c, &c->comp_T, (size_t)c->n_comp, "component fixpoints")) ||
        (rc = dev_alloc(c, &c->comp_nt, (size_t)c->n_comp * c->nt_cap, "component histories")) ||
        (rc = dev_alloc(c, &c->slot_comp, (size_t)c->n_lay * S, "row seed components")) ||
        (rc = dev_alloc(c, &c->comp_row, (size_t)c->n_comp, "component rows")) ||
        (rc = dev_alloc(c, &c->comp_chunk0, (size_t)c->n_comp + 1, "component chunks")) ||
        (rc = dev_alloc(c, &c->cchunk_comp, c->cchunk_comp_h.size(), "chunk components")) ||
        (rc = dev_alloc(c, &c->cchunk_b0, c->cchunk_b0_h.size(), "chunk blocks")) ||
        (rc = dev_alloc(c, &c->cchunk_sum, c->cchunk_comp_h.size(), "chunk sums")) ||
        (rc = dev_alloc(c, &c->cchunk_cnt, c->cchunk_comp_h.size(), "chunk counts"))) {
      free_run(c);
      return rc;
    }
  }
  // linear counting m ln(m/V), V = 1..m (entry 0 unused)
  c->lc_host.assign((size_t)m + 1, 0.0);
  for (int V = 1; V <= m; ++V) c->lc_host[V] = m * std::log((double)m / V);
  HIP_TRY(c, hipMemcpyAsync(c->lc, c->lc_host.data(), sizeof(double) * (m + 1), hipMemcpyHostToDevice, c->stream),
          "table upload");
  c->log2m = log2m;
  c->sl = sl;
  c->packed = packed;
  return HANF_OK;
}

// Batched runs: lays out `copies` copies of every graph of the base (copy q of graph g is
// layout component L = g * copies + q, with the graph's 64-node aligned size), expanded on
// the device from the base, and so its transposed graph if there is one. One copy is the
// base itself.
int set_layout(hanf_ctx *c, int32_t copies) {
  if (c->layout_ok && copies == c->copies) return HANF_OK;
  HIP_TRY(c, hipStreamSynchronize(c->stream), "sync");
  free_run(c);
  free_schedule(c);
  free_layout(c);
  const int32_t G = c->n_graphs;
  if (copies == 1) {
    c->rp = c->rp_own;
    c->ci = c->ci_own;
    c->n = c->base_n;
    c->arcs = c->base_arcs;
    c->n_lay = G;
    c->lay_node_off_h = c->g_node_off_h;
    c->lay_n_h = c->g_n_h;
    c->layout_ok = true;
    return HANF_OK;
  }
  const int32_t L = G * copies;
  std::vector<int32_t> off((size_t)L + 1), n((size_t)L), aoff((size_t)L + 1);
  int64_t nacc = 0, aacc = 0;
  for (int32_t g = 0; g < G; ++g)
    for (int32_t q = 0; q < copies; ++q) {
      const int32_t k = g * copies + q;
      off[k] = (int32_t)nacc;
      aoff[k] = (int32_t)aacc;
      n[k] = c->g_n_h[g];
      nacc += c->g_node_off_h[g + 1] - c->g_node_off_h[g];
      aacc += c->g_aoff_h[g + 1] - c->g_aoff_h[g];
      if (nacc > HANF_MAX_NODES || aacc > HANF_MAX_ARCS)
        return fail(c, HANF_EINVAL, "batch row layout above HANF_MAX_NODES nodes or HANF_MAX_ARCS arcs");
    }
  off[L] = (int32_t)nacc;
  aoff[L] = (int32_t)aacc;
  std::vector<int32_t> blk((size_t)(nacc / kNodesPerBlock));
  for (int32_t k = 0; k < L; ++k)
    for (int64_t b = off[k] / kNodesPerBlock; b < off[k + 1] / kNodesPerBlock; ++b) blk[(size_t)b] = k;
  int32_t *d_aoff = nullptr;
  const bool with_t = c->trp != nullptr;
  int rc;
  if ((rc = dev_alloc(c, &c->lay_blk, blk.size(), "layout blocks")) ||
      (rc = dev_alloc(c, &c->lay_node_off, (size_t)L + 1, "layout offsets")) ||
      (rc = dev_alloc(c, &c->lay_n, (size_t)L, "layout sizes")) ||
      (rc = dev_alloc(c, &d_aoff, (size_t)L + 1, "layout arc offsets")) ||
      (rc = dev_alloc(c, &c->rp_lay, (size_t)nacc + 1, "layout row_ptr")) ||
      (rc = dev_alloc(c, &c->ci_lay, (size_t)aacc, "layout col_idx")) ||
      (with_t && (rc = dev_alloc(c, &c->trp_lay, (size_t)nacc + 1, "layout transposed row_ptr"))) ||
      (with_t && (rc = dev_alloc(c, &c->tci_lay, (size_t)aacc, "layout transposed col_idx")))) {
    dev_release(c, d_aoff);
    free_layout(c);
    return rc;
  }
  int32_t *d_goff = c->comp_node_off;  // base offsets of the graphs (device)
  hipError_t e = hipMemcpyAsync(c->lay_blk, blk.data(), sizeof(int32_t) * blk.size(), hipMemcpyHostToDevice, c->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(c->lay_node_off, off.data(), sizeof(int32_t) * (L + 1), hipMemcpyHostToDevice, c->stream);
  if (e == hipSuccess) e = hipMemcpyAsync(c->lay_n, n.data(), sizeof(int32_t) * L, hipMemcpyHostToDevice, c->stream);
  if (e == hipSuccess) e = hipMemcpyAsync(d_aoff, aoff.data(), sizeof(int32_t) * (L + 1), hipMemcpyHostToDevice, c->stream);
  PassArgs la{};
  la.batch.blk_comp = c->lay_blk;
  la.batch.comp_node_off = c->lay_node_off;
  la.batch.n_lay = L;
  if (e == hipSuccess) e = reset_state_unread(c);
  if (e == hipSuccess)
    e = launch_expand(d_goff, c->rp_own, c->ci_own, copies, la, d_aoff, c->rp_lay, c->ci_lay, nacc, aacc, c->st,
                      c->stream);
  if (e == hipSuccess && with_t)
    e = launch_expand(d_goff, c->trp, c->tci, copies, la, d_aoff, c->trp_lay, c->tci_lay, nacc, aacc, c->st, c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  dev_release(c, d_aoff);
  if (e != hipSuccess) {
    free_layout(c);
    return hip_fail(c, e, "batch row layout");
  }
  c->rp = c->rp_lay;
  c->ci = c->ci_lay;
  c->n = (int32_t)nacc;
  c->arcs = aacc;
  c->n_lay = L;
  c->lay_node_off_h = off;
  c->lay_n_h = n;
  c->copies = copies;
  c->layout_ok = true;
  return HANF_OK;
}

// The switches compare changed counters with the number of counters, n S.
// The transposed graph of (rp, ci) into trp / tci by the two-level bucket sort of the
// kernels (graphs of at most kTpMaxNodes nodes). One host read of the bucket sizes splits
// the buckets into those one workgroup sorts and the hubs' buckets, sorted in chunks.
int transpose_buckets(hanf_ctx *c, const int32_t *rp, const int32_t *ci, int32_t n, int64_t arcs, int32_t *trp,
                      int32_t *tci) {
  int32_t bs = 10;
  while (((((int64_t)n - 1) >> bs) + 1) > kTpNumBuckets) ++bs;
  const int32_t nb = (int32_t)((((int64_t)n - 1) >> bs) + 1);
  const int32_t B = 1 << bs;
  int32_t n_ranges = (int32_t)std::min<int64_t>(512, ((int64_t)n + 63) / 64);
  const int32_t range = (int32_t)((((int64_t)n + n_ranges - 1) / n_ranges + 63) / 64 * 64);
  n_ranges = (int32_t)(((int64_t)n + range - 1) / range);
  const int64_t hn = (int64_t)nb * n_ranges + 1;
  uint64_t *hist = nullptr, *tmp = nullptr, *pairs = nullptr, *bstart = nullptr;
  int32_t *lists = nullptr;
  int64_t *chunks = nullptr;
  uint32_t *h2 = nullptr;
  auto release = [&]() {
    dev_release(c, hist);
    dev_release(c, tmp);
    dev_release(c, pairs);
    dev_release(c, bstart);
    dev_release(c, lists);
    dev_release(c, chunks);
    dev_release(c, h2);
  };
  int rc;
  if ((rc = dev_alloc(c, &hist, (size_t)hn, "transpose histogram")) ||
      (rc = dev_alloc(c, &tmp, (size_t)scan_tmp_elems(hn), "scan scratch")) ||
      (rc = dev_alloc(c, &pairs, (size_t)arcs, "transpose pairs")) ||
      (rc = dev_alloc(c, &bstart, (size_t)nb + 1, "bucket starts"))) {
    release();
    return rc;
  }
  std::vector<uint64_t> bs_h((size_t)nb + 1);
  hipError_t e = launch_tp_first(rp, ci, n, range, bs, nb, n_ranges, hist, tmp, pairs, bstart, c->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(bs_h.data(), bstart, sizeof(uint64_t) * (nb + 1), hipMemcpyDeviceToHost, c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) {
    release();
    return hip_fail(c, e, "transpose (first level)");
  }
  // light buckets, then hub buckets with their chunks
  std::vector<int32_t> light, heavy, hchunk0;
  std::vector<int64_t> clo, chi, cs;
  for (int32_t b = 0; b < nb; ++b) {
    const int64_t lo = (int64_t)bs_h[b], hi = (int64_t)bs_h[b + 1];
    if (hi - lo <= kTpLight) {
      light.push_back(b);
    } else {
      heavy.push_back(b);
      hchunk0.push_back((int32_t)clo.size());
      for (int64_t p = lo; p < hi; p += kTpChunk) {
        clo.push_back(p);
        chi.push_back(std::min(hi, p + kTpChunk));
        cs.push_back(lo);
      }
    }
  }
  hchunk0.push_back((int32_t)clo.size());
  const int32_t nl = (int32_t)light.size(), nh = (int32_t)heavy.size(), nc = (int32_t)clo.size();
  if ((rc = dev_alloc(c, &lists, (size_t)nl + nh + nh + 1, "bucket lists")) ||
      (rc = dev_alloc(c, &chunks, (size_t)3 * nc, "hub chunks")) ||
      (rc = dev_alloc(c, &h2, (size_t)nc * B, "hub chunk counts"))) {
    release();
    return rc;
  }
  std::vector<int32_t> lists_h(light);
  lists_h.insert(lists_h.end(), heavy.begin(), heavy.end());
  lists_h.insert(lists_h.end(), hchunk0.begin(), hchunk0.end());
  std::vector<int64_t> chunks_h(clo);
  chunks_h.insert(chunks_h.end(), chi.begin(), chi.end());
  chunks_h.insert(chunks_h.end(), cs.begin(), cs.end());
  const int32_t arcs32 = (int32_t)arcs;
  e = hipMemcpyAsync(lists, lists_h.data(), sizeof(int32_t) * lists_h.size(), hipMemcpyHostToDevice, c->stream);
  if (e == hipSuccess && nc > 0)
    e = hipMemcpyAsync(chunks, chunks_h.data(), sizeof(int64_t) * chunks_h.size(), hipMemcpyHostToDevice, c->stream);
  if (e == hipSuccess)
    e = launch_tp_second(pairs, bstart, lists, nl, lists + nl, lists + nl + nh, nh, chunks, chunks + nc, chunks + 2 * nc,
                         nc, h2, bs, n, trp, tci, c->stream);
  if (e == hipSuccess) e = hipMemcpyAsync(trp + n, &arcs32, sizeof(int32_t), hipMemcpyHostToDevice, c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  release();
  if (e != hipSuccess) return hip_fail(c, e, "transpose (second level)");
  return HANF_OK;
}

int64_t dense_threshold(const hanf_ctx *c) {
  if (c->dense_div <= 0) return 0;
  return std::max<int64_t>(1, ((int64_t)c->n << c->sl) / c->dense_div);
}

// Systolic passes need the signal buffers of the run, and the transposed graph or the forward
// scan (HANF_OPT_FORWARD).
bool has_signals(const hanf_ctx *c) { return c->args.trow_ptr || (c->forward && c->args.todo); }
int32_t systolic_div(const hanf_ctx *c) { return (has_signals(c) && c->frontier) ? c->sys_div : 0; }

// Timed passes: start and end of the signal kernels, the union step, finalize (with the
// estimates of packed rows) and the reduction, each pair taken from the kernels' own
// dispatches.
constexpr int kPassEvents = 8;

int enqueue_pass(hanf_ctx *c, hipEvent_t *ev) {
  hipStream_t s = c->stream;
  c->st_fresh = false;
  hipEvent_t e[kPassEvents] = {};
  if (ev)
    for (int i = 0; i < kPassEvents; ++i) e[i] = ev[i];
  // the first pass of a run maximises with every successor and is never systolic
  if (c->first_enqueued) {
    HIP_TRY(c, launch_signal(c->args, c->arcs, s, e[0], e[1]), "signal kernels");
  } else if (ev) {
    HIP_TRY(c, hipEventRecord(e[0], s), "event");
    HIP_TRY(c, hipEventRecord(e[1], s), "event");
  }
  c->first_enqueued = true;
  // The per-unit kernel is skipped once the last state read showed systolic passes (the
  // persistent kernel then runs every pass, whatever its kind); otherwise both are launched
  // and each leaves the passes that are not its own.
  const bool has_sys = has_signals(c);
  const int list = c->union_policy == 2 || (c->union_policy == 0 && has_sys);
  const int full = c->union_policy == 1 || (c->union_policy == 0 && !(has_sys && c->sys_seen));
  HIP_TRY(c, launch_union(c->args, c->sch.unroll, full, list, s, e[2], e[3]), "union kernel");
  const bool est = c->args.packed != 0;  // packed rows: estimates in a kernel of their own
  HIP_TRY(c, launch_finalize(c->args, s, e[4], est ? nullptr : e[5]), "finalize kernel");
  HIP_TRY(c, launch_estimate_changed(c->args, s, nullptr, est ? e[5] : nullptr), "estimate kernel");
  HIP_TRY(c, launch_reduce(c->args, kReducePass, 0, s, e[6], e[7]), "reduce kernels");
  return HANF_OK;
}

}  // namespace

// ===================================================================== C ABI

extern "C" {

int hanf_create(int device, void *hip_stream, hanf_ctx **out) {
  if (!out) return fail(nullptr, HANF_EINVAL, "hanf_create: out is NULL");
  *out = nullptr;
  int ndev = 0;
  hipError_t e = hipGetDeviceCount(&ndev);
  if (e != hipSuccess || ndev <= 0) {
    (void)hipGetLastError();
    return fail(nullptr, HANF_EDEVICE, "hanf_create: no HIP device available");
  }
  if (device < 0 || device >= ndev) return fail(nullptr, HANF_EINVAL, "hanf_create: bad device index");
  hanf_ctx *c = new (std::nothrow) hanf_ctx();
  if (!c) return fail(nullptr, HANF_ENOMEM, "hanf_create: out of host memory");
  c->device = device;
  if (const char *f = std::getenv("HANF_TEST_FAIL_ALLOC")) c->fail_alloc_at = std::atoi(f);
  e = hipSetDevice(device);
  if (e == hipSuccess) {
    scratch_setup(device);
    if (hip_stream) {
      c->stream = (hipStream_t)hip_stream;
    } else {
      e = hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking);
      c->own_stream = e == hipSuccess;
    }
  }
  if (e == hipSuccess) e = hipHostMalloc((void **)&c->st_host, sizeof(DevState), hipHostMallocDefault);
  if (e == hipSuccess) e = hipHostMalloc((void **)&c->st_poll, sizeof(DevState), hipHostMallocDefault);
  if (e == hipSuccess) e = hipHostMalloc((void **)&c->nt_host, sizeof(double) * kNtHostCache, hipHostMallocDefault);
  if (e == hipSuccess)
    e = hipHostMalloc((void **)&c->log_host, sizeof(PassLog) * kMaxPassesPerCheck, hipHostMallocDefault);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&c->poll_ev, hipEventDisableTiming);
  if (e != hipSuccess) {
    std::string msg = std::string("hanf_create: ") + hipGetErrorString(e);
    hanf_destroy(c);
    return fail(nullptr, HANF_EDEVICE, msg);
  }
  int rc = dev_alloc(c, &c->st, 1, "state");
  if (rc) {
    std::string msg = c->err;
    hanf_destroy(c);
    return fail(nullptr, rc, msg);
  }
  *out = c;
  return HANF_OK;
}

void hanf_destroy(hanf_ctx *c) {
  if (!c) return;
  (void)hipSetDevice(c->device);
  if (c->stream) (void)hipStreamSynchronize(c->stream);
  free_run(c);
  free_schedule(c);
  free_graph(c);
  dev_release(c, c->st);
  for (auto &kv : c->sizes) (void)hipFree(kv.first);
  c->sizes.clear();
  c->pool.clear();
  if (c->st_host) (void)hipHostFree(c->st_host);
  if (c->st_poll) (void)hipHostFree(c->st_poll);
  if (c->nt_host) (void)hipHostFree(c->nt_host);
  if (c->log_host) (void)hipHostFree(c->log_host);
  if (c->poll_ev) (void)hipEventDestroy(c->poll_ev);
  for (hipEvent_t e : c->ev_pool) (void)hipEventDestroy(e);
  if (c->own_stream && c->stream) (void)hipStreamDestroy(c->stream);
  delete c;
}

int hanf_set_option(hanf_ctx *c, int option, int64_t value) {
  if (!c) return fail(nullptr, HANF_EINVAL, "hanf_set_option: NULL context");
  switch (option) {
    case HANF_OPT_FRONTIER:
      if (value != 0 && value != 1) return fail(c, HANF_EINVAL, "frontier must be 0 or 1");
      c->frontier = (int)value;
      break;
    case HANF_OPT_MAX_PASSES:
      if (value < 0) return fail(c, HANF_EINVAL, "max passes must be >= 0");
      c->max_passes_opt = value;
      break;
    case HANF_OPT_LIGHT_MAX:
      if (value < 0 || value > (1 << 20)) return fail(c, HANF_EINVAL, "light max out of range");
      c->light_max_opt = (int32_t)value;
      break;
    case HANF_OPT_CHUNK_ARCS:
      if (value < 0 || value > (1 << 24)) return fail(c, HANF_EINVAL, "chunk arcs out of range");
      c->chunk_opt = (int32_t)value;
      break;
    case HANF_OPT_TIMING:
      c->timing = value ? 1 : 0;
      break;
    case HANF_OPT_BATCH:
      if (value < 1 || value > kMaxPassesPerCheck) return fail(c, HANF_EINVAL, "batch must be in 1..1024");
      c->passes_per_check = (int)value;
      break;
    case HANF_OPT_TILE_NODES:
      if (value < 0 || value > kMaxTile) return fail(c, HANF_EINVAL, "tile nodes must be in 0..256");
      c->tile_opt = (int32_t)value;
      break;
    case HANF_OPT_DENSE_SWITCH:
      if (value < 0 || value > (1 << 30)) return fail(c, HANF_EINVAL, "dense switch out of range");
      c->dense_div = (int)value;
      break;
    case HANF_OPT_SYSTOLIC:
      if (value < 0 || value > (1 << 30)) return fail(c, HANF_EINVAL, "systolic switch out of range");
      c->sys_div = (int)value;
      break;
    case HANF_OPT_SEEDS_PER_ROW:
      if (value < 0 || value > 32 || (value & (value - 1)) != 0)
        return fail(c, HANF_EINVAL, "seeds per row must be 0 or a power of two up to 32");
      c->seeds_row_opt = (int)value;
      break;
    case HANF_OPT_PACKED5:
      if (value < 0 || value > 2) return fail(c, HANF_EINVAL, "packed5 must be 0, 1 or 2");
      c->packed_opt = (int)value;
      break;
    case HANF_OPT_HUBS:
      if (value < -1 || value > INT32_MAX) return fail(c, HANF_EINVAL, "hubs must be -1 (auto), 0 or a count");
      c->hubs_opt = value;
      break;
    case HANF_OPT_FORWARD:
      if (value != 0 && value != 1) return fail(c, HANF_EINVAL, "forward must be 0 or 1");
      c->forward = (int)value;
      break;
    case HANF_OPT_STAGE:
      if (value < 0 || value > 1) return fail(c, HANF_EINVAL, "stage must be 0 or 1");
      c->stage_opt = (int)value;
      break;
    case 101:  // persistent union kernel: 0 for systolic passes, 1 never, 2 always; used by tests
      if (value < 0 || value > 2) return fail(c, HANF_EINVAL, "union policy must be 0, 1 or 2");
      c->union_policy = (int)value;
      break;
    case 102:  // transpose build: 0 bucket sort up to 2^26 nodes, 1 always per-node counters; used by tests
      if (value != 0 && value != 1) return fail(c, HANF_EINVAL, "transpose build must be 0 or 1");
      c->tp_counting = (int)value;
      break;
    case 104:  // instrumented union kernels that count near successors (0 or 1); used by the benchmark
      if (value != 0 && value != 1) return fail(c, HANF_EINVAL, "count_near must be 0 or 1");
      c->count_near = (int)value;
      break;
    case 103:  // LDS bytes per wavefront for a staged tile (2048, 4096, 8192 or 16384); used by the tuner
      if (value != 2048 && value != 4096 && value != 8192 && value != 16384)
        return fail(c, HANF_EINVAL, "stage bytes must be 2048, 4096, 8192 or 16384");
      c->stage_bytes = (int32_t)value;
      break;
    case 100:  // unroll of the gather loops (0 automatic, 2, 4 or 8); used by the tuner
      if (value != 0 && value != 2 && value != 4 && value != 8) return fail(c, HANF_EINVAL, "unroll must be 0, 2, 4 or 8");
      c->unroll = (int)value;
      break;
    default:
      return fail(c, HANF_EINVAL, "unknown option");
  }
  return HANF_OK;
}

int hanf_load_csr(hanf_ctx *c, int32_t n, int64_t arcs, const int32_t *row_ptr, const int32_t *col_idx,
                  uint32_t flags) {
  if (!c) return fail(nullptr, HANF_EINVAL, "hanf_load_csr: NULL context");
  if (n < 1 || n > HANF_MAX_NODES) return fail(c, HANF_EINVAL, "n must be in [1, HANF_MAX_NODES]");
  if (arcs < 0 || arcs > HANF_MAX_ARCS) return fail(c, HANF_EINVAL, "arcs must be in [0, HANF_MAX_ARCS]");
  if (!row_ptr || (arcs > 0 && !col_idx)) return fail(c, HANF_EINVAL, "NULL CSR array");
  if (flags != HANF_HOST_PTRS && flags != HANF_DEVICE_PTRS) return fail(c, HANF_EINVAL, "bad flags");
  HIP_TRY(c, hipSetDevice(c->device), "set device");
  HIP_TRY(c, hipStreamSynchronize(c->stream), "sync");
  free_run(c);
  free_schedule(c);
  free_graph(c);
  int rc;
  if (flags == HANF_DEVICE_PTRS) {
    for (const void *p : {(const void *)row_ptr, (const void *)col_idx}) {
      if (!p) continue;
      hipPointerAttribute_t attr;
      hipError_t e = hipPointerGetAttributes(&attr, p);
      if (e != hipSuccess || attr.type != hipMemoryTypeDevice || attr.device != c->device) {
        (void)hipGetLastError();
        return fail(c, HANF_EINVAL, "HANF_DEVICE_PTRS: pointer is not device memory of this device");
      }
    }
    c->rp = row_ptr;
    c->ci = arcs > 0 ? col_idx : nullptr;
  } else {
    if ((rc = dev_alloc(c, &c->rp_own, (size_t)n + 1, "row_ptr")) ||
        (rc = dev_alloc(c, &c->ci_own, (size_t)arcs, "col_idx"))) {
      free_graph(c);
      return rc;
    }
    HIP_TRY(c, hipMemcpyAsync(c->rp_own, row_ptr, sizeof(int32_t) * ((size_t)n + 1), hipMemcpyHostToDevice, c->stream),
            "row_ptr upload");
    if (arcs > 0)
      HIP_TRY(c, hipMemcpyAsync(c->ci_own, col_idx, sizeof(int32_t) * (size_t)arcs, hipMemcpyHostToDevice, c->stream),
              "col_idx upload");
    c->rp = c->rp_own;
    c->ci = c->ci_own;
  }
  c->n = n;
  c->arcs = arcs;
  HIP_TRY(c, reset_state_unread(c), "state reset");
  HIP_TRY(c, launch_validate(c->rp, c->ci, n, arcs, c->st, c->stream), "validate");
  if ((rc = read_state(c))) return rc;
  if (c->st_host->err) {
    const int e = c->st_host->err;
    std::string msg = "malformed CSR:";
    if (e & 1) msg += " row_ptr[0] != 0;";
    if (e & 2) msg += " row_ptr decreases;";
    if (e & 4) msg += " row_ptr[n] != arcs;";
    if (e & 8) msg += " col_idx out of [0, n);";
    free_graph(c);
    return fail(c, HANF_EINVAL, msg);
  }
  c->graph_ok = true;
  return HANF_OK;
}

int hanf_load_transpose(hanf_ctx *c, int32_t n_t, int64_t arcs_t, const int32_t *row_ptr_t, const int32_t *col_idx_t,
                        uint32_t flags) {
  if (!c) return fail(nullptr, HANF_EINVAL, "hanf_load_transpose: NULL context");
  if (!c->graph_ok) return fail(c, HANF_ESTATE, "no graph loaded");
  if (c->batch) return fail(c, HANF_EINVAL, "batched graph: use hanf_build_transpose");
  if (n_t != c->n || arcs_t != c->arcs)
    return fail(c, HANF_EINVAL, "the transposed graph must have the graph's n and arcs");
  if (!row_ptr_t || (c->arcs > 0 && !col_idx_t)) return fail(c, HANF_EINVAL, "NULL CSR array");
  if (flags != HANF_HOST_PTRS && flags != HANF_DEVICE_PTRS) return fail(c, HANF_EINVAL, "bad flags");
  HIP_TRY(c, hipSetDevice(c->device), "set device");
  HIP_TRY(c, hipStreamSynchronize(c->stream), "sync");
  free_transpose(c);
  c->inited = false;  // the signal buffers are sized at the next initialisation
  const int32_t n = c->n;
  const int64_t arcs = c->arcs;
  int rc;
  if (flags == HANF_DEVICE_PTRS) {
    for (const void *p : {(const void *)row_ptr_t, (const void *)col_idx_t}) {
      if (!p) continue;
      hipPointerAttribute_t attr;
      hipError_t e = hipPointerGetAttributes(&attr, p);
      if (e != hipSuccess || attr.type != hipMemoryTypeDevice || attr.device != c->device) {
        (void)hipGetLastError();
        return fail(c, HANF_EINVAL, "HANF_DEVICE_PTRS: pointer is not device memory of this device");
      }
    }
    c->trp = row_ptr_t;
    c->tci = arcs > 0 ? col_idx_t : nullptr;
  } else {
    if ((rc = dev_alloc(c, &c->trp_own, (size_t)n + 1, "transposed row_ptr")) ||
        (rc = dev_alloc(c, &c->tci_own, (size_t)arcs, "transposed col_idx"))) {
      free_transpose(c);
      return rc;
    }
    HIP_TRY(c, hipMemcpyAsync(c->trp_own, row_ptr_t, sizeof(int32_t) * ((size_t)n + 1), hipMemcpyHostToDevice,
                              c->stream),
            "transposed row_ptr upload");
    if (arcs > 0)
      HIP_TRY(c, hipMemcpyAsync(c->tci_own, col_idx_t, sizeof(int32_t) * (size_t)arcs, hipMemcpyHostToDevice,
                                c->stream),
              "transposed col_idx upload");
    c->trp = c->trp_own;
    c->tci = c->tci_own;
  }
  HIP_TRY(c, reset_state_unread(c), "state reset");
  HIP_TRY(c, launch_validate(c->trp, c->tci, n, arcs, c->st, c->stream), "validate");
  if ((rc = read_state(c))) return rc;
  if (c->st_host->err) {
    free_transpose(c);
    return fail(c, HANF_EINVAL, "malformed transposed CSR (it must have the graph's n and arcs)");
  }
  if (c->perm) {  // the caller's ids, into the node order already chosen
    int32_t *trp_new = nullptr, *tci_new = nullptr;
    if ((rc = permute_graph(c, c->trp, c->tci, &trp_new, &tci_new))) {
      free_transpose(c);
      return rc;
    }
    const hipError_t e = hipStreamSynchronize(c->stream);
    free_transpose(c);
    if (e != hipSuccess) {
      dev_release(c, trp_new);
      dev_release(c, tci_new);
      return hip_fail(c, e, "transpose reorder");
    }
    c->trp = c->trp_own = trp_new;
    c->tci = c->tci_own = tci_new;
  }
  return HANF_OK;
}

int hanf_transpose_self(hanf_ctx *c) {
  if (!c) return fail(nullptr, HANF_EINVAL, "hanf_transpose_self: NULL context");
  if (!c->graph_ok) return fail(c, HANF_ESTATE, "no graph loaded");
  HIP_TRY(c, hipSetDevice(c->device), "set device");
  HIP_TRY(c, hipStreamSynchronize(c->stream), "sync");
  free_transpose(c);
  c->inited = false;
  int rc;
  if (c->batch) {  // the base's own lists; the next initialisation lays them out with the graph
    if ((rc = set_layout(c, 1))) return rc;
    c->trp = c->rp_own;
    c->tci = c->ci_own;
  } else {
    c->trp = c->rp;
    c->tci = c->ci;
  }
  return HANF_OK;
}

int hanf_build_transpose(hanf_ctx *c) {
  if (!c) return fail(nullptr, HANF_EINVAL, "hanf_build_transpose: NULL context");
  if (!c->graph_ok) return fail(c, HANF_ESTATE, "no graph loaded");
  HIP_TRY(c, hipSetDevice(c->device), "set device");
  HIP_TRY(c, hipStreamSynchronize(c->stream), "sync");
  free_transpose(c);
  c->inited = false;
  int rc;
  // a batch's transpose is built on its base; the next initialisation lays it out with the graph
  if (c->batch && (rc = set_layout(c, 1))) return rc;
  const int32_t n = c->n;
  const int64_t arcs = c->arcs;
  uint64_t *keys = nullptr, *tmp = nullptr;
  if ((rc = dev_alloc(c, &c->trp_own, (size_t)n + 1, "transposed row_ptr")) ||
      (rc = dev_alloc(c, &c->tci_own, (size_t)arcs, "transposed col_idx")) ||
      (rc = dev_alloc(c, &keys, (size_t)n + 1, "in-degrees")) ||
      (rc = dev_alloc(c, &tmp, (size_t)scan_tmp_elems((int64_t)n + 1), "scan scratch"))) {
    dev_release(c, keys);
    dev_release(c, tmp);
    free_transpose(c);
    return rc;
  }
  if (arcs > 0 && n <= kTpMaxNodes && !c->tp_counting) {  // bucket sort; the counting build below is the fallback
    dev_release(c, keys);
    dev_release(c, tmp);
    if ((rc = transpose_buckets(c, c->rp, c->ci, n, arcs, c->trp_own, c->tci_own))) {
      free_transpose(c);
      return rc;
    }
    c->trp = c->trp_own;
    c->tci = c->tci_own;
    return HANF_OK;
  }
  hipError_t e = launch_fill_u64(keys, (int64_t)n + 1, 0ull, c->stream);
  if (e == hipSuccess) e = launch_transpose_count(c->ci, arcs, keys, c->stream);
  if (e == hipSuccess) e = launch_exclusive_scan_u64(keys, (int64_t)n + 1, tmp, c->stream);
  if (e == hipSuccess) e = launch_transpose_fill(c->rp, c->ci, n, keys, c->trp_own, c->tci_own, c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  dev_release(c, keys);
  dev_release(c, tmp);
  if (e != hipSuccess) {
    free_transpose(c);
    return hip_fail(c, e, "transpose");
  }
  c->trp = c->trp_own;
  c->tci = c->tci_own;
  return HANF_OK;
}

}  // extern "C"

namespace {

int init_common(hanf_ctx *c, int32_t log2m, uint64_t seed, const uint64_t *seeds) {
  if (!c->graph_ok) return fail(c, HANF_ESTATE, "no graph loaded");
  if (log2m < 4 || log2m > 8) return fail(c, HANF_EINVAL, "log2m must be in 4..8");
  if (c->packed_opt == 1 && log2m < 6) return fail(c, HANF_EINVAL, "5-bit registers need m >= 64 (log2m >= 6)");
  HIP_TRY(c, hipSetDevice(c->device), "set device");
  int rc;
  int sl = 0;
  if (c->batch) {
    // counters per row: as many seeds as fit, a power of two, at most 32, rows <= 1024
    // registers (1024 bytes, or 640 packed)
    const int m = 1 << log2m;
    int S = 1;
    while (S < c->n_seeds && S < 32 && 2 * S * m <= 1024 && (c->seeds_row_opt == 0 || S < c->seeds_row_opt)) S *= 2;
    while ((1 << sl) < S) ++sl;
    if ((rc = set_layout(c, (c->n_seeds + S - 1) / S))) return rc;
  }
  // Register format: rows of at least 512 registers (several seeds side by side) are bound
  // by their bytes, and 5-bit registers are faster there; narrower rows are bound by the
  // rate of row requests, and one register per byte is faster (measured on MI355X).
  const int packed = c->packed_opt == 1 || (c->packed_opt == 2 && log2m >= 6 && ((1 << log2m) << sl) >= 512);
  // lanes per node row: 16 byte registers or 64 packed ones per lane
  const int G = (packed ? 1 << (log2m - 6) : 1 << (log2m - 4)) << sl;
  const int lane_bytes = packed ? kPacked5LaneBytes : 16;
  if (!c->batch && !c->ordered && (c->hubs_opt >= 0 || c->inits > 0)) {
    if ((rc = order_nodes(c, log2m, packed))) return rc;
    if (c->perm) free_schedule(c);  // built on the caller's order
  }
  ++c->inits;
  Schedule want;
  choose_schedule(c, G, lane_bytes, want);
  if (c->sch.G != G || c->sch.lane_bytes != lane_bytes || !c->sch.light || want.light_max != c->sch.light_max ||
      want.chunk_arcs != c->sch.chunk_arcs || want.tile_base != c->sch.tile_base ||
      want.stage_opt != c->sch.stage_opt || want.stage_tile != c->sch.stage_tile ||
      want.unroll != c->sch.unroll) {
    if ((rc = build_schedule(c, G, lane_bytes))) return rc;
  }
  size_t n_cchunks_before = c->cchunk_comp_h.size();
  if (c->batch) {
    // which result component every row seed of every layout component runs, and the
    // reduction chunks of every result component (kCompChunkBlocks blocks each)
    const int32_t S = 1 << sl;
    c->slot_h.assign((size_t)c->n_lay * S, -1);
    c->comp_row_h.assign((size_t)c->n_comp, 0);
    c->chunk0_h.assign((size_t)c->n_comp + 1, 0);
    c->cchunk_comp_h.clear();
    c->cchunk_b0_h.clear();
    for (int32_t g = 0; g < c->n_graphs; ++g)
      for (int32_t sd = 0; sd < c->n_seeds; ++sd) {
        const int32_t comp = g * c->n_seeds + sd;
        const int32_t L = g * c->copies + sd / S;
        const int32_t row = L * S + sd % S;
        c->slot_h[(size_t)row] = comp;
        c->comp_row_h[(size_t)comp] = row;
        c->chunk0_h[(size_t)comp] = (int32_t)c->cchunk_comp_h.size();
        const int32_t b0 = c->lay_node_off_h[L] / kNodesPerBlock, b1 = c->lay_node_off_h[L + 1] / kNodesPerBlock;
        for (int32_t b = b0; b < b1; b += kCompChunkBlocks) {
          c->cchunk_comp_h.push_back(comp);
          c->cchunk_b0_h.push_back(b);
        }
      }
    c->chunk0_h[(size_t)c->n_comp] = (int32_t)c->cchunk_comp_h.size();
  }
  const int64_t want_cap = default_max_passes(c) + 2;
  if (c->log2m != log2m || c->sl != sl || c->packed != packed || !c->regs[0] || want_cap != c->nt_cap ||
      c->cchunk_comp_h.size() != n_cchunks_before) {
    if ((rc = alloc_run(c, log2m, sl, packed))) return rc;
  }
  if (c->batch) {
    HIP_TRY(c, hipMemcpyAsync(c->slot_comp, c->slot_h.data(), sizeof(int32_t) * c->slot_h.size(),
                              hipMemcpyHostToDevice, c->stream),
            "row seed upload");
    HIP_TRY(c, hipMemcpyAsync(c->comp_row, c->comp_row_h.data(), sizeof(int32_t) * c->n_comp, hipMemcpyHostToDevice,
                              c->stream),
            "component row upload");
    HIP_TRY(c, hipMemcpyAsync(c->comp_chunk0, c->chunk0_h.data(), sizeof(int32_t) * c->chunk0_h.size(),
                              hipMemcpyHostToDevice, c->stream),
            "chunk table upload");
    HIP_TRY(c, hipMemcpyAsync(c->cchunk_comp, c->cchunk_comp_h.data(), sizeof(int32_t) * c->cchunk_comp_h.size(),
                              hipMemcpyHostToDevice, c->stream),
            "chunk table upload");
    HIP_TRY(c, hipMemcpyAsync(c->cchunk_b0, c->cchunk_b0_h.data(), sizeof(int32_t) * c->cchunk_b0_h.size(),
                              hipMemcpyHostToDevice, c->stream),
            "chunk table upload");
  }
  if ((c->trp || c->forward) && !c->todo) {  // signal marks and lists for systolic passes
    if ((rc = dev_alloc(c, &c->todo, (size_t)kNodesPerBlock * c->n_blocks, "systolic signals")) ||
        (rc = dev_alloc(c, &c->sig_list, (size_t)std::max<int64_t>(1, c->arcs), "signalled successors")) ||
        (rc = dev_alloc(c, &c->sig_cnt, (size_t)kNodesPerBlock * c->n_blocks, "signalled successors"))) {
      free_run(c);
      return rc;
    }
    // zero before the first systolic pass; every pass clears the counts it used
    HIP_TRY(c, hipMemsetAsync(c->sig_cnt, 0, sizeof(int32_t) * kNodesPerBlock * c->n_blocks, c->stream),
            "signal counts");
  }
  if (c->trp && !c->sys_node) {  // the list of modified nodes that signal through the transpose
    if ((rc = dev_alloc(c, &c->sys_node, (size_t)c->n, "systolic list")) ||
        (rc = dev_alloc(c, &c->sys_pos, (size_t)c->n, "systolic list"))) {
      free_run(c);
      return rc;
    }
  }
  c->inited = false;
  c->sys_seen = false;
  c->first_enqueued = false;
  fill_args(c);
  c->host_log.clear();
  if (seeds)
    HIP_TRY(c, hipMemcpyAsync(c->comp_seed, seeds, sizeof(uint64_t) * c->n_comp, hipMemcpyHostToDevice, c->stream),
            "seed upload");
  c->nt_host_len = 0;
  HIP_TRY(c, launch_state_reset(c->st, 0, c->frontier, c->max_passes, dense_threshold(c), systolic_div(c),
                                c->stream),
          "state reset");
  // neither the init kernel nor the first reduction changes the state
  mirror_state_reset(c, 0, c->max_passes, dense_threshold(c), systolic_div(c));
  HIP_TRY(c, launch_init(c->args, seed, c->stream), "init kernel");
  HIP_TRY(c, launch_reduce(c->args, kReduceInit, 1, c->stream), "reduce kernels");
  if (seeds && (rc = sync(c, "batch init"))) return rc;  // the seed array is the caller's
  c->inited = true;
  return HANF_OK;
}

}  // namespace

extern "C" {

int hanf_init_counters(hanf_ctx *c, int32_t log2m, uint64_t seed) {
  if (!c) return fail(nullptr, HANF_EINVAL, "hanf_init_counters: NULL context");
  if (c->batch) return fail(c, HANF_EINVAL, "batched graph: use hanf_init_batch");
  return init_common(c, log2m, seed, nullptr);
}

int hanf_init_batch(hanf_ctx *c, int32_t log2m, const uint64_t *seeds) {
  if (!c) return fail(nullptr, HANF_EINVAL, "hanf_init_batch: NULL context");
  if (!c->batch) return fail(c, HANF_ESTATE, "no batch loaded (hanf_load_batch)");
  if (!seeds) return fail(c, HANF_EINVAL, "seeds is NULL");
  return init_common(c, log2m, 0, seeds);
}

int hanf_iterate(hanf_ctx *c, int32_t max_steps, int32_t *steps_done, int64_t *changed_last) {
  if (steps_done) *steps_done = 0;
  if (!c) return fail(nullptr, HANF_EINVAL, "hanf_iterate: NULL context");
  if (!c->inited) return fail(c, HANF_ESTATE, "counters not initialised");
  HIP_TRY(c, hipSetDevice(c->device), "set device");
  int rc;
  if ((rc = current_state(c))) return rc;
  int32_t steps = 0;
  std::vector<hipEvent_t> &ev = c->ev_pool;
  for (;;) {
    DevState s0 = *c->st_host;
    c->sys_seen = s0.systolic != 0;
    if (changed_last) *changed_last = s0.changed_last;
    if (s0.done) {
      if (steps_done) *steps_done = steps;
      return HANF_DONE;
    }
    if (s0.capped) {
      if (steps_done) *steps_done = steps;
      return fail(c, HANF_EMAXITER, "pass cap reached before the fixpoint");
    }
    if (max_steps > 0 && steps >= max_steps) break;
    int B = c->passes_per_check;
    if (max_steps > 0) B = std::min(B, max_steps - steps);
    if (c->timing)
      while (ev.size() < (size_t)B * kPassEvents) {
        hipEvent_t x = nullptr;
        if (hipEventCreate(&x) != hipSuccess) return fail(c, HANF_EDEVICE, "event create");
        ev.push_back(x);
      }
    for (int i = 0; i < B; ++i) {
      rc = enqueue_pass(c, c->timing ? &ev[(size_t)i * kPassEvents] : nullptr);
      if (rc) return rc;
    }
    // the run state, the records of every pass the batch may have run and the start of the
    // N_hat history, in one wait
    const int32_t cnt = (int32_t)std::max<int64_t>(0, std::min<int64_t>(B, (int64_t)c->log_cap - s0.passes));
    const int32_t nt_cnt = std::min(c->nt_cap, kNtHostCache);
    c->nt_host_len = 0;
    HIP_TRY(c, hipMemcpyAsync(c->st_host, c->st, sizeof(DevState), hipMemcpyDeviceToHost, c->stream),
            "state read");
    if (cnt > 0)
      HIP_TRY(c, hipMemcpyAsync(c->log_host, c->log + s0.passes, sizeof(PassLog) * cnt, hipMemcpyDeviceToHost,
                                c->stream),
              "pass log read");
    if (!c->batch)
      HIP_TRY(c, hipMemcpyAsync(c->nt_host, c->nt, sizeof(double) * nt_cnt, hipMemcpyDeviceToHost, c->stream),
              "history read");
    if ((rc = sync(c, "state read"))) return rc;
    c->st_fresh = true;
    c->comp_T_fresh = false;
    if (!c->batch) c->nt_host_len = std::min(c->st_host->t + 1, nt_cnt);
    const int32_t ran = c->st_host->passes - s0.passes;
    if (ran > B) return fail(c, HANF_EDEVICE, "more passes recorded than enqueued");
    if (ran > 0) {
      const PassLog *recs = c->log_host;
      for (int32_t i = 0; i < std::min(ran, cnt); ++i) {  // passes beyond log_cap are not recorded
        hanf_pass_t r{};
        r.changed = recs[i].changed;
        r.arcs_scanned = recs[i].scanned;
        r.arcs_gathered = recs[i].gathered;
        r.rows_written = recs[i].written;
        r.rows_read = recs[i].read;
        r.gather_all = (int32_t)recs[i].gather_all;
        r.systolic = (int32_t)recs[i].systolic;
        r.arcs_signalled = recs[i].signalled;
        r.arcs_local = recs[i].local;
        r.arcs_near = (c->args.count_near || c->args.stage) ? recs[i].near : -1;
        r.flag_summary = (int32_t)recs[i].summary;
        if (c->timing) {
          hipEvent_t *e = &ev[(size_t)i * kPassEvents];
          (void)hipEventElapsedTime(&r.signal_ms, e[0], e[1]);
          (void)hipEventElapsedTime(&r.union_ms, e[2], e[3]);
          (void)hipEventElapsedTime(&r.finalize_ms, e[4], e[5]);
          (void)hipEventElapsedTime(&r.reduce_ms, e[6], e[7]);
        }
        c->host_log.push_back(r);
      }
    }
    steps += ran;
    if (ran == 0 && !c->st_host->done && !c->st_host->capped)
      return fail(c, HANF_EDEVICE, "no pass completed (device state did not advance)");
  }
  if (steps_done) *steps_done = steps;
  return HANF_OK;
}

int hanf_enqueue(hanf_ctx *c, int32_t passes) {
  if (!c) return fail(nullptr, HANF_EINVAL, "hanf_enqueue: NULL context");
  if (!c->inited) return fail(c, HANF_ESTATE, "counters not initialised");
  if (passes < 1) return fail(c, HANF_EINVAL, "passes must be >= 1");
  HIP_TRY(c, hipSetDevice(c->device), "set device");
  int rc;
  for (int32_t i = 0; i < passes; ++i)
    if ((rc = enqueue_pass(c, nullptr))) return rc;
  HIP_TRY(c, hipMemcpyAsync(c->st_poll, c->st, sizeof(DevState), hipMemcpyDeviceToHost, c->stream), "state copy");
  HIP_TRY(c, hipEventRecord(c->poll_ev, c->stream), "event");
  c->poll_pending = true;
  return HANF_OK;
}

int hanf_poll(hanf_ctx *c, int32_t *t) {
  if (!c) return fail(nullptr, HANF_EINVAL, "hanf_poll: NULL context");
  if (!c->inited) return fail(c, HANF_ESTATE, "counters not initialised");
  if (!c->poll_pending) return fail(c, HANF_ESTATE, "nothing enqueued");
  HIP_TRY(c, hipSetDevice(c->device), "set device");
  const hipError_t e = hipEventQuery(c->poll_ev);
  if (e == hipErrorNotReady) {
    (void)hipGetLastError();
    return HANF_BUSY;
  }
  if (e != hipSuccess) return hip_fail(c, e, "poll");
  c->poll_pending = false;
  const DevState s0 = *c->st_poll;
  c->sys_seen = s0.systolic != 0;
  if (t) *t = s0.t;
  if (s0.done) return HANF_DONE;
  if (s0.capped) return fail(c, HANF_EMAXITER, "pass cap reached before the fixpoint");
  return HANF_OK;
}

int hanf_read_nt(hanf_ctx *c, double *out, int32_t cap, int32_t *len) {
  if (!c) return fail(nullptr, HANF_EINVAL, "hanf_read_nt: NULL context");
  if (!c->inited) return fail(c, HANF_ESTATE, "counters not initialised");
  if (!len) return fail(c, HANF_EINVAL, "len is NULL");
  HIP_TRY(c, hipSetDevice(c->device), "set device");
  int rc;
  if ((rc = current_state(c))) return rc;
  const int32_t have = c->st_host->t + 1;
  *len = have;
  if (cap < have) return fail(c, HANF_ERANGE, "output capacity below t+1");
  if (!out) return fail(c, HANF_EINVAL, "out is NULL");
  if (c->st_fresh && have <= c->nt_host_len) {  // read with the state by the last wait
    std::memcpy(out, c->nt_host, sizeof(double) * have);
    return HANF_OK;
  }
  HIP_TRY(c, hipMemcpyAsync(out, c->nt, sizeof(double) * have, hipMemcpyDeviceToHost, c->stream), "history read");
  return sync(c, "history read");
}

int hanf_read_registers(hanf_ctx *c, uint8_t *out, int64_t bytes, uint32_t flags) {
  if (!c) return fail(nullptr, HANF_EINVAL, "hanf_read_registers: NULL context");
  if (!c->inited) return fail(c, HANF_ESTATE, "counters not initialised");
  if (!out) return fail(c, HANF_EINVAL, "out is NULL");
  if (bytes != (int64_t)c->n << c->log2m) return fail(c, HANF_EINVAL, "bytes must be n * m");
  if (flags != HANF_HOST_PTRS && flags != HANF_DEVICE_PTRS) return fail(c, HANF_EINVAL, "bad flags");
  HIP_TRY(c, hipSetDevice(c->device), "set device");
  if (flags == HANF_DEVICE_PTRS && !device_pointer(c, out))
    return fail(c, HANF_EINVAL, "HANF_DEVICE_PTRS: out is not device memory of this device");
  int rc;
  if ((rc = current_state(c))) return rc;
  const uint8_t *src = c->regs[c->st_host->t & 1];
  if (!c->perm) return regs_to_bytes(c, src, out, flags);
  // rows back in the caller's order first
  const size_t rb = row_bytes(c->log2m, c->sl, c->packed);
  uint8_t *tmp = nullptr;
  if ((rc = dev_alloc(c, &tmp, (size_t)c->n * rb, "register reorder"))) return rc;
  const hipError_t e = launch_gather_rows(src, tmp, c->inv, c->n, (int64_t)rb, c->stream);
  rc = e != hipSuccess ? hip_fail(c, e, "register reorder") : regs_to_bytes(c, tmp, out, flags);
  (void)hipStreamSynchronize(c->stream);
  dev_release(c, tmp);
  return rc;
}

int hanf_read_estimates(hanf_ctx *c, double *out, int64_t count, uint32_t flags) {
  if (!c) return fail(nullptr, HANF_EINVAL, "hanf_read_estimates: NULL context");
  if (!c->inited) return fail(c, HANF_ESTATE, "counters not initialised");
  if (c->batch) return fail(c, HANF_EINVAL, "batched graph: use hanf_batch_read_estimates");
  if (!out) return fail(c, HANF_EINVAL, "out is NULL");
  if (count != c->n) return fail(c, HANF_EINVAL, "count must be n");
  if (flags != HANF_HOST_PTRS && flags != HANF_DEVICE_PTRS) return fail(c, HANF_EINVAL, "bad flags");
  HIP_TRY(c, hipSetDevice(c->device), "set device");
  if (flags == HANF_DEVICE_PTRS && !device_pointer(c, out))
    return fail(c, HANF_EINVAL, "HANF_DEVICE_PTRS: out is not device memory of this device");
  if (!c->perm) {
    HIP_TRY(c, hipMemcpyAsync(out, c->est, sizeof(double) * (size_t)count,
                              flags == HANF_DEVICE_PTRS ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, c->stream),
            "estimate read");
    return sync(c, "estimate read");
  }
  // estimates back in the caller's node order
  if (flags == HANF_DEVICE_PTRS) {
    HIP_TRY(c, launch_gather_rows((const uint8_t *)c->est, (uint8_t *)out, c->inv, c->n, 8, c->stream),
            "estimate reorder");
    return sync(c, "estimate read");
  }
  double *tmp = nullptr;
  int rc;
  if ((rc = dev_alloc(c, &tmp, (size_t)count, "estimate reorder"))) return rc;
  hipError_t e = launch_gather_rows((const uint8_t *)c->est, (uint8_t *)tmp, c->inv, c->n, 8, c->stream);
  if (e == hipSuccess) e = hipMemcpyAsync(out, tmp, sizeof(double) * (size_t)count, hipMemcpyDeviceToHost, c->stream);
  const hipError_t e2 = hipStreamSynchronize(c->stream);
  dev_release(c, tmp);
  if (e != hipSuccess || e2 != hipSuccess) return hip_fail(c, e != hipSuccess ? e : e2, "estimate read");
  return HANF_OK;
}

int hanf_read_order(hanf_ctx *c, int32_t *out, int32_t count, uint32_t flags) {
  if (!c) return fail(nullptr, HANF_EINVAL, "hanf_read_order: NULL context");
  if (!c->graph_ok) return fail(c, HANF_ESTATE, "no graph loaded");
  if (c->batch) return fail(c, HANF_EINVAL, "batched graphs keep the caller's order");
  if (!out) return fail(c, HANF_EINVAL, "out is NULL");
  if (count != c->n) return fail(c, HANF_EINVAL, "count must be n");
  if (flags != HANF_HOST_PTRS && flags != HANF_DEVICE_PTRS) return fail(c, HANF_EINVAL, "bad flags");
  HIP_TRY(c, hipSetDevice(c->device), "set device");
  if (flags == HANF_DEVICE_PTRS && !device_pointer(c, out))
    return fail(c, HANF_EINVAL, "HANF_DEVICE_PTRS: out is not device memory of this device");
  if (!c->perm) {
    if (flags == HANF_HOST_PTRS) {
      for (int32_t i = 0; i < count; ++i) out[i] = i;
      return HANF_OK;
    }
    HIP_TRY(c, launch_iota(out, count, c->stream), "order read");
    return sync(c, "order read");
  }
  HIP_TRY(c, hipMemcpyAsync(out, c->perm, sizeof(int32_t) * (size_t)count,
                            flags == HANF_DEVICE_PTRS ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, c->stream),
          "order read");
  return sync(c, "order read");
}

int hanf_write_registers(hanf_ctx *c, const uint8_t *in, int64_t bytes, int32_t t, const double *nt_prefix,
                         int32_t len, uint32_t flags) {
  if (!c) return fail(nullptr, HANF_EINVAL, "hanf_write_registers: NULL context");
  if (!c->inited) return fail(c, HANF_ESTATE, "counters not initialised (m unknown)");
  if (c->batch) return fail(c, HANF_EINVAL, "checkpoint resume is for single graphs");
  if (!in || !nt_prefix) return fail(c, HANF_EINVAL, "NULL input");
  if (bytes != (int64_t)c->n << c->log2m) return fail(c, HANF_EINVAL, "bytes must be n * m");
  if (t < 0 || len != t + 1) return fail(c, HANF_EINVAL, "len must be t + 1");
  if (t + 2 > c->nt_cap) return fail(c, HANF_ERANGE, "t beyond the pass cap");
  if (flags != HANF_HOST_PTRS && flags != HANF_DEVICE_PTRS) return fail(c, HANF_EINVAL, "bad flags");
  HIP_TRY(c, hipSetDevice(c->device), "set device");
  if (flags == HANF_DEVICE_PTRS && !device_pointer(c, in))
    return fail(c, HANF_EINVAL, "HANF_DEVICE_PTRS: in is not device memory of this device");
  // from here on the run in progress is replaced (on an error it must be initialised again)
  c->inited = false;
  c->sys_seen = false;
  c->first_enqueued = false;
  c->st_fresh = false;
  c->nt_host_len = 0;
  HIP_TRY(c, launch_state_reset(c->st, t, c->frontier, c->max_passes, dense_threshold(c), systolic_div(c),
                                c->stream),
          "state reset");
  int rc;
  if (!c->perm) {
    if ((rc = bytes_to_regs(c, in, c->regs[t & 1], flags))) return rc;
  } else {  // rows in the caller's order, then into the library's
    const size_t rb = row_bytes(c->log2m, c->sl, c->packed);
    uint8_t *tmp = nullptr;
    if ((rc = dev_alloc(c, &tmp, (size_t)c->n * rb, "register reorder"))) return rc;
    rc = bytes_to_regs(c, in, tmp, flags);
    if (!rc) {
      const hipError_t e = launch_gather_rows(tmp, c->regs[t & 1], c->perm, c->n, (int64_t)rb, c->stream);
      if (e != hipSuccess) rc = hip_fail(c, e, "register reorder");
    }
    (void)hipStreamSynchronize(c->stream);
    dev_release(c, tmp);
    if (rc) return rc;
  }
  if ((rc = read_state(c))) return rc;
  if (c->st_host->err) return fail(c, HANF_EINVAL, "register value above 31");
  HIP_TRY(c, hipMemcpyAsync(c->regs[(t + 1) & 1], c->regs[t & 1], (size_t)c->n * row_bytes(c->log2m, c->sl, c->packed),
                            hipMemcpyDeviceToDevice, c->stream),
          "register copy");
  fill_args(c);
  c->host_log.clear();
  HIP_TRY(c, launch_estimate_all(c->args, c->regs[t & 1], c->stream), "estimate kernel");
  HIP_TRY(c, launch_reduce(c->args, kReduceInit, 1, c->stream), "reduce kernels");
  HIP_TRY(c, hipMemcpyAsync(c->nt, nt_prefix, sizeof(double) * len, hipMemcpyHostToDevice, c->stream),
          "history upload");
  if ((rc = sync(c, "resume"))) return rc;
  c->inited = true;
  return HANF_OK;
}

int hanf_stats(hanf_ctx *c, double alpha, double eps, int32_t distinct, hanf_stats_t *out) {
  if (!c) return fail(nullptr, HANF_EINVAL, "hanf_stats: NULL context");
  if (!out) return fail(c, HANF_EINVAL, "out is NULL");
  if (!c->inited) return fail(c, HANF_ESTATE, "counters not initialised");
  if (!(alpha > 0.0 && alpha <= 1.0)) return fail(c, HANF_EINVAL, "alpha must be in (0, 1]");
  if (!(eps >= 0.0)) return fail(c, HANF_EINVAL, "eps must be >= 0");
  HIP_TRY(c, hipSetDevice(c->device), "set device");
  double buf[9];
  HIP_TRY(c, launch_stats(c->nt, nullptr, c->st, alpha, eps, distinct ? 1 : 0, c->stats_out, c->stream),
          "stats kernel");
  HIP_TRY(c, hipMemcpyAsync(buf, c->stats_out, sizeof(buf), hipMemcpyDeviceToHost, c->stream), "stats read");
  int rc;
  if ((rc = sync(c, "stats"))) return rc;
  out->ed = buf[0];
  out->ied = buf[1];
  out->avg_dist = buf[2];
  out->var = buf[3];
  out->spid = buf[4];
  out->n_max = buf[5];
  out->d_lo = buf[6];
  out->d_hi = buf[7];
  out->T = (int32_t)buf[8];
  out->distinct = distinct ? 1 : 0;
  return HANF_OK;
}

int hanf_stats_nt(const double *nt, int32_t len, double alpha, double eps, int32_t distinct, hanf_stats_t *out) {
  if (!nt || !out || len < 1) return fail(nullptr, HANF_EINVAL, "hanf_stats_nt: need nt, out and len >= 1");
  if (!(alpha > 0.0 && alpha <= 1.0)) return fail(nullptr, HANF_EINVAL, "alpha must be in (0, 1]");
  if (!(eps >= 0.0)) return fail(nullptr, HANF_EINVAL, "eps must be >= 0");
  double buf[9];
  stats_of(nt, len - 1, alpha, eps, distinct ? 1 : 0, buf);
  out->ed = buf[0];
  out->ied = buf[1];
  out->avg_dist = buf[2];
  out->var = buf[3];
  out->spid = buf[4];
  out->n_max = buf[5];
  out->d_lo = buf[6];
  out->d_hi = buf[7];
  out->T = len - 1;
  out->distinct = distinct ? 1 : 0;
  return HANF_OK;
}

int hanf_read_pass_log(hanf_ctx *c, hanf_pass_t *out, int32_t cap, int32_t *len) {
  if (!c) return fail(nullptr, HANF_EINVAL, "hanf_read_pass_log: NULL context");
  if (!len) return fail(c, HANF_EINVAL, "len is NULL");
  const int32_t have = (int32_t)c->host_log.size();
  *len = have;
  if (cap < have) return fail(c, HANF_ERANGE, "output capacity below the pass count");
  if (have > 0 && !out) return fail(c, HANF_EINVAL, "out is NULL");
  if (have > 0) std::memcpy(out, c->host_log.data(), sizeof(hanf_pass_t) * have);
  return HANF_OK;
}

int hanf_footprint(int32_t n, int64_t arcs, int32_t log2m, int32_t flags, int64_t *bytes) {
  if (!bytes) return fail(nullptr, HANF_EINVAL, "bytes is NULL");
  if (n < 1 || n > HANF_MAX_NODES || arcs < 0 || arcs > HANF_MAX_ARCS || log2m < 4 || log2m > 8)
    return fail(nullptr, HANF_EINVAL, "hanf_footprint: argument out of range");
  if ((flags & HANF_FP_PACKED5) && log2m < 6)
    return fail(nullptr, HANF_EINVAL, "hanf_footprint: 5-bit registers need log2m >= 6");
  const int64_t m = 1LL << log2m;
  const int64_t blocks = ((int64_t)n + kNodesPerBlock - 1) / kNodesPerBlock;
  // counters + update buffer: m bytes per counter, or 5m/8 with 5-bit registers
  int64_t b = 2 * (int64_t)n * ((flags & HANF_FP_PACKED5) ? m * 5 / 8 : m);
  b += 2 * 2 * blocks * 4;                               // modified flags
  b += sum_bytes(blocks);                                // their summary
  b += (int64_t)n * 8 + blocks * 8 + 2 * ((blocks + 3) / 4) * 8;  // estimates and sums
  b += (int64_t)n * 4 + 4096;                            // light tiles
  b += ((int64_t)n + 1) * 8 * 2;                         // schedule scan (transient)
  b += ((int64_t)n + 3) * 8;                             // N_hat history (pass cap n + 1)
  b += std::min<int64_t>((int64_t)n + 3, kMaxLogRecords) * (int64_t)sizeof(PassLog);  // pass records
  b += blocks * kNodesPerBlock;                          // systolic marks (forward scan or transpose)
  if (flags & HANF_FP_COPY_GRAPH) b += ((int64_t)n + 1) * 4 + arcs * 4;
  if (flags & HANF_FP_TRANSPOSE) {
    b += ((int64_t)n + 1) * 4 + arcs * 4;  // predecessor lists
    b += (int64_t)n * 8;                   // signal list
    b += arcs * 4 + blocks * kNodesPerBlock * 4;  // signalled successors and their counts
  }
  if (flags & HANF_FP_ORDER) {
    b += ((int64_t)n + 1) * 4 + arcs * 4 + (int64_t)n * 8;  // the reordered graph, perm and inv
    if (flags & HANF_FP_TRANSPOSE) b += ((int64_t)n + 1) * 4 + arcs * 4;  // a transpose of its own
  }
  *bytes = b;
  return HANF_OK;
}

int hanf_load_batch(hanf_ctx *c, int32_t n_graphs, const int32_t *graph_off, const int32_t *arc_off, const int32_t *row_ptr,
                    const int32_t *col_idx, int32_t n_seeds, uint32_t flags) {
  if (!c) return fail(nullptr, HANF_EINVAL, "hanf_load_batch: NULL context");
  if (n_graphs < 1 || n_seeds < 1 || !graph_off || !arc_off || !row_ptr)
    return fail(c, HANF_EINVAL, "bad batch arguments");
  if (flags != HANF_HOST_PTRS && flags != HANF_DEVICE_PTRS) return fail(c, HANF_EINVAL, "bad flags");
  const int64_t arcs = arc_off[n_graphs];
  if (arcs > 0 && !col_idx) return fail(c, HANF_EINVAL, "col_idx is NULL");
  if (flags == HANF_DEVICE_PTRS && (!device_pointer(c, row_ptr) || (arcs > 0 && !device_pointer(c, col_idx))))
    return fail(c, HANF_EINVAL, "HANF_DEVICE_PTRS: pointer is not device memory of this device");
  if (arc_off[0] != 0 || arcs < 0 || arcs > HANF_MAX_ARCS)
    return fail(c, HANF_EINVAL, "arcs must be in [0, HANF_MAX_ARCS]");
  if ((int64_t)n_graphs * n_seeds >= (int64_t)INT32_MAX) return fail(c, HANF_EINVAL, "too many components");
  if (graph_off[0] != 0) return fail(c, HANF_EINVAL, "graph_off[0] must be 0");
  for (int32_t g = 0; g < n_graphs; ++g) {
    if (graph_off[g + 1] <= graph_off[g]) return fail(c, HANF_EINVAL, "every graph needs at least one node");
    if (arc_off[g + 1] < arc_off[g]) return fail(c, HANF_EINVAL, "arc_off decreases");
  }
  const int32_t N = graph_off[n_graphs];
  // the base: every graph once, each starting on a 64-node boundary
  const int32_t C = n_graphs;
  std::vector<int32_t> node_off((size_t)C + 1), comp_aoff((size_t)C + 1), ncomp((size_t)C);
  int64_t nacc = 0, aacc = 0;
  for (int32_t g = 0; g < n_graphs; ++g) {
    const int64_t ng = graph_off[g + 1] - graph_off[g];
    const int64_t ag = (int64_t)arc_off[g + 1] - arc_off[g];
    node_off[g] = (int32_t)nacc;
    comp_aoff[g] = (int32_t)aacc;
    ncomp[g] = (int32_t)ng;
    nacc += (ng + kNodesPerBlock - 1) / kNodesPerBlock * kNodesPerBlock;
    aacc += ag;
    if (nacc > HANF_MAX_NODES || aacc > HANF_MAX_ARCS)
      return fail(c, HANF_EINVAL, "batch above HANF_MAX_NODES nodes or HANF_MAX_ARCS arcs");
  }
  node_off[C] = (int32_t)nacc;
  comp_aoff[C] = (int32_t)aacc;
  const int64_t n_exp = nacc, e_exp = aacc;
  std::vector<int32_t> blk((size_t)(n_exp / kNodesPerBlock));
  for (int32_t k = 0; k < C; ++k)
    for (int64_t b = node_off[k] / kNodesPerBlock; b < node_off[k + 1] / kNodesPerBlock; ++b) blk[(size_t)b] = k;

  HIP_TRY(c, hipSetDevice(c->device), "set device");
  HIP_TRY(c, hipStreamSynchronize(c->stream), "sync");
  free_run(c);
  free_schedule(c);
  free_graph(c);
  int rc;
  const bool dev_in = flags == HANF_DEVICE_PTRS;
  int32_t *d_goff = nullptr, *d_rp = nullptr, *d_ci = nullptr, *d_aoff = nullptr, *d_gaoff = nullptr;
  auto cleanup = [&]() {
    dev_release(c, d_goff);
    dev_release(c, d_gaoff);
    if (!dev_in) {
      dev_release(c, d_rp);
      dev_release(c, d_ci);
    }
    dev_release(c, d_aoff);
  };
  if (dev_in) {
    d_rp = const_cast<int32_t *>(row_ptr);
    d_ci = const_cast<int32_t *>(col_idx);
  }
  if ((rc = dev_alloc(c, &d_goff, (size_t)n_graphs + 1, "batch graph offsets")) ||
      (rc = dev_alloc(c, &d_gaoff, (size_t)n_graphs + 1, "batch arc offsets")) ||
      (!dev_in && (rc = dev_alloc(c, &d_rp, (size_t)N + 1, "batch row_ptr"))) ||
      (!dev_in && (rc = dev_alloc(c, &d_ci, (size_t)arcs, "batch col_idx"))) ||
      (rc = dev_alloc(c, &d_aoff, (size_t)C + 1, "component arc offsets")) ||
      (rc = dev_alloc(c, &c->blk_comp, blk.size(), "block components")) ||
      (rc = dev_alloc(c, &c->comp_node_off, (size_t)C + 1, "component offsets")) ||
      (rc = dev_alloc(c, &c->comp_n, (size_t)C, "component sizes")) ||
      (rc = dev_alloc(c, &c->rp_own, (size_t)n_exp + 1, "row_ptr")) ||
      (rc = dev_alloc(c, &c->ci_own, (size_t)e_exp, "col_idx"))) {
    cleanup();
    free_graph(c);
    return rc;
  }
  hipError_t e = hipMemcpyAsync(d_goff, graph_off, sizeof(int32_t) * (n_graphs + 1), hipMemcpyHostToDevice, c->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(d_gaoff, arc_off, sizeof(int32_t) * (n_graphs + 1), hipMemcpyHostToDevice, c->stream);
  if (e == hipSuccess && !dev_in)
    e = hipMemcpyAsync(d_rp, row_ptr, sizeof(int32_t) * ((size_t)N + 1), hipMemcpyHostToDevice, c->stream);
  if (e == hipSuccess && arcs > 0 && !dev_in)
    e = hipMemcpyAsync(d_ci, col_idx, sizeof(int32_t) * (size_t)arcs, hipMemcpyHostToDevice, c->stream);
  if (e == hipSuccess) e = hipMemcpyAsync(d_aoff, comp_aoff.data(), sizeof(int32_t) * (C + 1), hipMemcpyHostToDevice, c->stream);
  if (e == hipSuccess) e = hipMemcpyAsync(c->blk_comp, blk.data(), sizeof(int32_t) * blk.size(), hipMemcpyHostToDevice, c->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(c->comp_node_off, node_off.data(), sizeof(int32_t) * (C + 1), hipMemcpyHostToDevice, c->stream);
  if (e == hipSuccess) e = hipMemcpyAsync(c->comp_n, ncomp.data(), sizeof(int32_t) * C, hipMemcpyHostToDevice, c->stream);
  if (e == hipSuccess) e = reset_state_unread(c);
  if (e == hipSuccess) e = launch_validate(d_rp, d_ci, N, arcs, c->st, c->stream);
  if (e == hipSuccess) e = launch_check_offsets(d_rp, d_goff, d_gaoff, n_graphs, c->st, c->stream);
  c->batch = true;
  c->n_graphs = n_graphs;
  c->n_seeds = n_seeds;
  c->n_comp = n_graphs * n_seeds;
  c->n_lay = C;
  c->n = (int32_t)n_exp;
  c->arcs = e_exp;
  fill_args(c);
  if (e == hipSuccess)
    e = launch_expand(d_goff, d_rp, d_ci, 1, c->args, d_aoff, c->rp_own, c->ci_own, n_exp, e_exp, c->st, c->stream);
  if (e != hipSuccess) {
    cleanup();
    free_graph(c);
    return hip_fail(c, e, "batch ingest");
  }
  rc = read_state(c);
  cleanup();
  if (rc) {
    free_graph(c);
    return rc;
  }
  if (c->st_host->err) {
    const int er = c->st_host->err;
    free_graph(c);
    return fail(c, HANF_EINVAL, (er & 32) ? "an arc leaves its graph"
                                : (er & 64) ? "arc_off disagrees with row_ptr" : "malformed CSR");
  }
  set_base(c, node_off, ncomp, comp_aoff);
  return HANF_OK;
}

int hanf_load_batch_list(hanf_ctx *c, int32_t n_graphs, const int32_t *const *row_ptrs,
                         const int32_t *const *col_idxs, const int32_t *n_nodes, const int64_t *n_arcs,
                         int32_t n_seeds, uint32_t flags) {
  if (!c) return fail(nullptr, HANF_EINVAL, "hanf_load_batch_list: NULL context");
  if (n_graphs < 1 || n_seeds < 1 || !row_ptrs || !col_idxs || !n_nodes || !n_arcs)
    return fail(c, HANF_EINVAL, "bad batch arguments");
  if (flags != HANF_HOST_PTRS && flags != HANF_DEVICE_PTRS) return fail(c, HANF_EINVAL, "bad flags");
  if ((int64_t)n_graphs * n_seeds >= (int64_t)INT32_MAX) return fail(c, HANF_EINVAL, "too many components");
  std::vector<int32_t> goff((size_t)n_graphs + 1), aoff((size_t)n_graphs + 1);
  int64_t nacc = 0, aacc = 0;
  for (int32_t g = 0; g < n_graphs; ++g) {
    if (flags == HANF_DEVICE_PTRS && row_ptrs[g] &&
        (!device_pointer(c, row_ptrs[g]) || (n_arcs[g] > 0 && col_idxs[g] && !device_pointer(c, col_idxs[g]))))
      return fail(c, HANF_EINVAL, "HANF_DEVICE_PTRS: pointer is not device memory of this device");
    if (n_nodes[g] < 1 || n_arcs[g] < 0 || !row_ptrs[g] || (n_arcs[g] > 0 && !col_idxs[g]))
      return fail(c, HANF_EINVAL, "every graph needs at least one node and its arrays");
    goff[g] = (int32_t)nacc;
    aoff[g] = (int32_t)aacc;
    nacc += n_nodes[g];
    aacc += n_arcs[g];
    if (nacc + n_graphs > HANF_MAX_NODES || aacc > HANF_MAX_ARCS)
      return fail(c, HANF_EINVAL, "batch above HANF_MAX_NODES nodes or HANF_MAX_ARCS arcs");
  }
  goff[n_graphs] = (int32_t)nacc;
  aoff[n_graphs] = (int32_t)aacc;
  const int32_t C = n_graphs;  // the base: every graph once, 64-node aligned
  std::vector<int32_t> node_off((size_t)C + 1), comp_aoff((size_t)C + 1), ncomp((size_t)C);
  int64_t en = 0, ea = 0;
  for (int32_t g = 0; g < n_graphs; ++g) {
    node_off[g] = (int32_t)en;
    comp_aoff[g] = (int32_t)ea;
    ncomp[g] = n_nodes[g];
    en += ((int64_t)n_nodes[g] + kNodesPerBlock - 1) / kNodesPerBlock * kNodesPerBlock;
    ea += n_arcs[g];
    if (en > HANF_MAX_NODES || ea > HANF_MAX_ARCS)
      return fail(c, HANF_EINVAL, "batch above HANF_MAX_NODES nodes or HANF_MAX_ARCS arcs");
  }
  node_off[C] = (int32_t)en;
  comp_aoff[C] = (int32_t)ea;
  std::vector<int32_t> blk((size_t)(en / kNodesPerBlock));
  for (int32_t k = 0; k < C; ++k)
    for (int64_t b = node_off[k] / kNodesPerBlock; b < node_off[k + 1] / kNodesPerBlock; ++b) blk[(size_t)b] = k;

  HIP_TRY(c, hipSetDevice(c->device), "set device");
  HIP_TRY(c, hipStreamSynchronize(c->stream), "sync");
  free_run(c);
  free_schedule(c);
  free_graph(c);
  int rc;
  int32_t *d_goff = nullptr, *d_gaoff = nullptr, *d_rp = nullptr, *d_ci = nullptr, *d_aoff = nullptr;
  auto cleanup = [&]() {
    dev_release(c, d_goff);
    dev_release(c, d_gaoff);
    dev_release(c, d_rp);
    dev_release(c, d_ci);
    dev_release(c, d_aoff);
  };
  if ((rc = dev_alloc(c, &d_goff, (size_t)n_graphs + 1, "batch graph offsets")) ||
      (rc = dev_alloc(c, &d_gaoff, (size_t)n_graphs + 1, "batch arc offsets")) ||
      (rc = dev_alloc(c, &d_rp, (size_t)nacc + n_graphs, "batch row_ptr")) ||
      (rc = dev_alloc(c, &d_ci, (size_t)aacc, "batch col_idx")) ||
      (rc = dev_alloc(c, &d_aoff, (size_t)C + 1, "component arc offsets")) ||
      (rc = dev_alloc(c, &c->blk_comp, blk.size(), "block components")) ||
      (rc = dev_alloc(c, &c->comp_node_off, (size_t)C + 1, "component offsets")) ||
      (rc = dev_alloc(c, &c->comp_n, (size_t)C, "component sizes")) ||
      (rc = dev_alloc(c, &c->rp_own, (size_t)en + 1, "row_ptr")) ||
      (rc = dev_alloc(c, &c->ci_own, (size_t)ea, "col_idx"))) {
    cleanup();
    free_graph(c);
    return rc;
  }
  const hipMemcpyKind kind = flags == HANF_DEVICE_PTRS ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
  hipError_t e = hipSuccess;
  for (int32_t g = 0; g < n_graphs && e == hipSuccess; ++g) {
    e = hipMemcpyAsync(d_rp + goff[g] + g, row_ptrs[g], sizeof(int32_t) * ((size_t)n_nodes[g] + 1), kind, c->stream);
    if (e == hipSuccess && n_arcs[g] > 0)
      e = hipMemcpyAsync(d_ci + aoff[g], col_idxs[g], sizeof(int32_t) * (size_t)n_arcs[g], kind, c->stream);
  }
  if (e == hipSuccess) e = hipMemcpyAsync(d_goff, goff.data(), sizeof(int32_t) * (n_graphs + 1), hipMemcpyHostToDevice, c->stream);
  if (e == hipSuccess) e = hipMemcpyAsync(d_gaoff, aoff.data(), sizeof(int32_t) * (n_graphs + 1), hipMemcpyHostToDevice, c->stream);
  if (e == hipSuccess) e = hipMemcpyAsync(d_aoff, comp_aoff.data(), sizeof(int32_t) * (C + 1), hipMemcpyHostToDevice, c->stream);
  if (e == hipSuccess) e = hipMemcpyAsync(c->blk_comp, blk.data(), sizeof(int32_t) * blk.size(), hipMemcpyHostToDevice, c->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(c->comp_node_off, node_off.data(), sizeof(int32_t) * (C + 1), hipMemcpyHostToDevice, c->stream);
  if (e == hipSuccess) e = hipMemcpyAsync(c->comp_n, ncomp.data(), sizeof(int32_t) * C, hipMemcpyHostToDevice, c->stream);
  if (e == hipSuccess) e = reset_state_unread(c);
  c->batch = true;
  c->n_graphs = n_graphs;
  c->n_seeds = n_seeds;
  c->n_comp = n_graphs * n_seeds;
  c->n_lay = C;
  c->n = (int32_t)en;
  c->arcs = ea;
  fill_args(c);
  if (e == hipSuccess)
    e = launch_expand_local(d_goff, d_gaoff, d_rp, d_ci, n_graphs, 1, c->args, d_aoff, c->rp_own, c->ci_own, en, ea,
                            c->st, c->stream);
  if (e != hipSuccess) {
    cleanup();
    free_graph(c);
    return hip_fail(c, e, "batch ingest");
  }
  rc = read_state(c);
  cleanup();
  if (rc) {
    free_graph(c);
    return rc;
  }
  if (c->st_host->err) {
    free_graph(c);
    return fail(c, HANF_EINVAL, "malformed CSR in the batch");
  }
  set_base(c, node_off, ncomp, comp_aoff);
  return HANF_OK;
}

int hanf_batch_info(hanf_ctx *c, int32_t *n_components, int32_t *T) {
  if (!c) return fail(nullptr, HANF_EINVAL, "hanf_batch_info: NULL context");
  if (!c->batch) return fail(c, HANF_ESTATE, "no batch loaded");
  if (n_components) *n_components = c->n_comp;
  if (T) {
    if (!c->inited) return fail(c, HANF_ESTATE, "counters not initialised");
    HIP_TRY(c, hipMemcpyAsync(T, c->comp_T, sizeof(int32_t) * c->n_comp, hipMemcpyDeviceToHost, c->stream),
            "fixpoint read");
    return sync(c, "fixpoint read");
  }
  return HANF_OK;
}

int hanf_batch_read_nt(hanf_ctx *c, int32_t comp, double *out, int32_t cap, int32_t *len) {
  if (!c) return fail(nullptr, HANF_EINVAL, "hanf_batch_read_nt: NULL context");
  if (!c->batch || !c->inited) return fail(c, HANF_ESTATE, "no initialised batch");
  if (comp < 0 || comp >= c->n_comp || !len) return fail(c, HANF_EINVAL, "bad component or len");
  HIP_TRY(c, hipSetDevice(c->device), "set device");
  int rc;
  if ((rc = batch_state(c))) return rc;
  const int32_t Tc = c->comp_T_host[(size_t)comp];
  const int32_t have = (Tc >= 0 ? Tc : c->st_host->t) + 1;
  *len = have;
  if (cap < have) return fail(c, HANF_ERANGE, "output capacity below the history length");
  if (!out) return fail(c, HANF_EINVAL, "out is NULL");
  HIP_TRY(c, hipMemcpyAsync(out, c->comp_nt + (size_t)comp * c->nt_cap, sizeof(double) * have, hipMemcpyDeviceToHost,
                            c->stream),
          "history read");
  return sync(c, "history read");
}

int hanf_batch_read_registers(hanf_ctx *c, int32_t comp, uint8_t *out, int64_t bytes, uint32_t flags) {
  if (!c) return fail(nullptr, HANF_EINVAL, "hanf_batch_read_registers: NULL context");
  if (!c->batch || !c->inited) return fail(c, HANF_ESTATE, "no initialised batch");
  if (comp < 0 || comp >= c->n_comp || !out) return fail(c, HANF_EINVAL, "bad component or out");
  if (flags != HANF_HOST_PTRS && flags != HANF_DEVICE_PTRS) return fail(c, HANF_EINVAL, "bad flags");
  if (flags == HANF_DEVICE_PTRS && !device_pointer(c, out))
    return fail(c, HANF_EINVAL, "HANF_DEVICE_PTRS: out is not device memory of this device");
  const int32_t row = c->comp_row_h[comp];
  const int32_t L = row >> c->sl, j = row & ((1 << c->sl) - 1);
  const size_t m = (size_t)1 << c->log2m, R = row_bytes(c->log2m, c->sl, c->packed);
  const size_t cb = R >> c->sl;  // bytes of one counter
  const int32_t ng = c->lay_n_h[L];
  if (bytes != (int64_t)ng * (int64_t)m) return fail(c, HANF_EINVAL, "bytes must be n_graph * m");
  HIP_TRY(c, hipSetDevice(c->device), "set device");
  int rc;
  if ((rc = current_state(c))) return rc;
  // counter j of every row of the component's nodes: a strided copy (unpacked on the device)
  const uint8_t *src = c->regs[c->st_host->t & 1] + (size_t)c->lay_node_off_h[L] * R + (size_t)j * cb;
  if (!c->packed) {
    HIP_TRY(c, hipMemcpy2DAsync(out, m, src, R, m, (size_t)ng,
                                flags == HANF_DEVICE_PTRS ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, c->stream),
            "register read");
    return sync(c, "register read");
  }
  const int32_t gpr = (int32_t)(m / 64);
  if (flags == HANF_DEVICE_PTRS) {
    HIP_TRY(c, launch_unpack5_rows(src, (int64_t)R, gpr, ng, out, c->stream), "register unpack");
    return sync(c, "register read");
  }
  const int64_t rows_per = std::max<int64_t>(1, kStageGroups / gpr);
  const int64_t chunk = std::min<int64_t>(ng, rows_per);
  uint8_t *stage = nullptr;
  if ((rc = dev_alloc(c, &stage, (size_t)chunk * m, "register staging"))) return rc;
  hipError_t e = hipSuccess;
  for (int64_t r0 = 0; r0 < ng && e == hipSuccess; r0 += chunk) {
    const int64_t cnt = std::min<int64_t>(chunk, ng - r0);
    e = launch_unpack5_rows(src + r0 * (int64_t)R, (int64_t)R, gpr, cnt, stage, c->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(out + r0 * (int64_t)m, stage, (size_t)cnt * m, hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  }
  dev_release(c, stage);
  if (e != hipSuccess) return hip_fail(c, e, "register read");
  return HANF_OK;
}

int hanf_batch_read_estimates(hanf_ctx *c, int32_t comp, double *out, int64_t count, uint32_t flags) {
  if (!c) return fail(nullptr, HANF_EINVAL, "hanf_batch_read_estimates: NULL context");
  if (!c->batch || !c->inited) return fail(c, HANF_ESTATE, "no initialised batch");
  if (comp < 0 || comp >= c->n_comp || !out) return fail(c, HANF_EINVAL, "bad component or out");
  if (flags != HANF_HOST_PTRS && flags != HANF_DEVICE_PTRS) return fail(c, HANF_EINVAL, "bad flags");
  if (flags == HANF_DEVICE_PTRS && !device_pointer(c, out))
    return fail(c, HANF_EINVAL, "HANF_DEVICE_PTRS: out is not device memory of this device");
  const int32_t row = c->comp_row_h[comp];
  const int32_t L = row >> c->sl, j = row & ((1 << c->sl) - 1);
  const size_t S = (size_t)1 << c->sl;
  const int32_t ng = c->lay_n_h[L];
  if (count != ng) return fail(c, HANF_EINVAL, "count must be the graph's n");
  HIP_TRY(c, hipSetDevice(c->device), "set device");
  const double *src = c->est + (size_t)c->lay_node_off_h[L] * S + (size_t)j;  // counter j of each row
  HIP_TRY(c, hipMemcpy2DAsync(out, sizeof(double), src, sizeof(double) * S, sizeof(double), (size_t)ng,
                              flags == HANF_DEVICE_PTRS ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, c->stream),
          "estimate read");
  return sync(c, "estimate read");
}

int hanf_batch_stats(hanf_ctx *c, int32_t comp, double alpha, double eps, int32_t distinct, hanf_stats_t *out) {
  if (!c) return fail(nullptr, HANF_EINVAL, "hanf_batch_stats: NULL context");
  if (!c->batch || !c->inited) return fail(c, HANF_ESTATE, "no initialised batch");
  if (comp < 0 || comp >= c->n_comp || !out) return fail(c, HANF_EINVAL, "bad component or out");
  if (!(alpha > 0.0 && alpha <= 1.0) || !(eps >= 0.0)) return fail(c, HANF_EINVAL, "alpha or eps out of range");
  HIP_TRY(c, hipSetDevice(c->device), "set device");
  double buf[9];
  HIP_TRY(c, launch_stats(c->comp_nt + (size_t)comp * c->nt_cap, c->comp_T + comp, c->st, alpha, eps,
                          distinct ? 1 : 0, c->stats_out, c->stream),
          "stats kernel");
  HIP_TRY(c, hipMemcpyAsync(buf, c->stats_out, sizeof(buf), hipMemcpyDeviceToHost, c->stream), "stats read");
  int rc;
  if ((rc = sync(c, "stats"))) return rc;
  out->ed = buf[0];
  out->ied = buf[1];
  out->avg_dist = buf[2];
  out->var = buf[3];
  out->spid = buf[4];
  out->n_max = buf[5];
  out->d_lo = buf[6];
  out->d_hi = buf[7];
  out->T = (int32_t)buf[8];
  out->distinct = distinct ? 1 : 0;
  return HANF_OK;
}

int hanf_batch_stats_all(hanf_ctx *c, double alpha, double eps, int32_t distinct, hanf_stats_t *out) {
  if (!c) return fail(nullptr, HANF_EINVAL, "hanf_batch_stats_all: NULL context");
  if (!c->batch || !c->inited) return fail(c, HANF_ESTATE, "no initialised batch");
  if (!out) return fail(c, HANF_EINVAL, "out is NULL");
  if (!(alpha > 0.0 && alpha <= 1.0) || !(eps >= 0.0)) return fail(c, HANF_EINVAL, "alpha or eps out of range");
  HIP_TRY(c, hipSetDevice(c->device), "set device");
  StatsRec *dbuf = nullptr;
  int rc;
  if ((rc = dev_alloc(c, &dbuf, (size_t)c->n_comp, "statistics"))) return rc;
  hipError_t e = launch_stats_all(c->args, alpha, eps, distinct ? 1 : 0, dbuf, c->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(out, dbuf, sizeof(StatsRec) * (size_t)c->n_comp, hipMemcpyDeviceToHost, c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  dev_release(c, dbuf);
  if (e != hipSuccess) return hip_fail(c, e, "statistics");
  return HANF_OK;
}

int hanf_batch_seed_summary(hanf_ctx *c, double alpha, int32_t distinct, hanf_seed_summary_t *out) {
  if (!c) return fail(nullptr, HANF_EINVAL, "hanf_batch_seed_summary: NULL context");
  if (!c->batch || !c->inited) return fail(c, HANF_ESTATE, "no initialised batch");
  if (!out) return fail(c, HANF_EINVAL, "out is NULL");
  if (!(alpha > 0.0 && alpha <= 1.0)) return fail(c, HANF_EINVAL, "alpha must be in (0, 1]");
  HIP_TRY(c, hipSetDevice(c->device), "set device");
  SummaryRec *dbuf = nullptr;
  int rc;
  if ((rc = dev_alloc(c, &dbuf, (size_t)c->n_graphs, "seed summary"))) return rc;
  hipError_t e = launch_seed_summary(c->args, c->n_graphs, c->n_seeds, alpha, distinct ? 1 : 0, dbuf, c->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(out, dbuf, sizeof(SummaryRec) * (size_t)c->n_graphs, hipMemcpyDeviceToHost, c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  dev_release(c, dbuf);
  if (e != hipSuccess) return hip_fail(c, e, "seed summary");
  return HANF_OK;
}

static_assert(sizeof(SummaryRec) == sizeof(hanf_seed_summary_t), "SummaryRec must have hanf_seed_summary_t's layout");
static_assert(offsetof(SummaryRec, runs) == offsetof(hanf_seed_summary_t, runs),
              "SummaryRec must have hanf_seed_summary_t's layout");

int hanf_batch_stats_all_noalloc(hanf_ctx *c, double alpha, double eps, int32_t distinct, hanf_stats_t *out) {
  if (!c) return fail(nullptr, HANF_EINVAL, "hanf_batch_stats_all_noalloc: NULL context");
  if (!c->batch || !c->inited) return fail(c, HANF_ESTATE, "no initialised batch");
  if (!out) return fail(c, HANF_EINVAL, "out is NULL");
  if (!(alpha > 0.0 && alpha <= 1.0) || !(eps >= 0.0)) return fail(c, HANF_EINVAL, "alpha or eps out of range");
  if (c->n_comp > HANF_NOALLOC_MAX_COMPONENTS)
    return fail(c, HANF_ERANGE,
                "hanf_batch_stats_all_noalloc: the batch has " + std::to_string(c->n_comp) +
                    " components, more than HANF_NOALLOC_MAX_COMPONENTS (" +
                    std::to_string(HANF_NOALLOC_MAX_COMPONENTS) + "); use hanf_batch_stats_all");
  HIP_TRY(c, hipSetDevice(c->device), "set device");
  hipError_t e = hipSuccess;
  StatsRec *dbuf = scratch_of(c->device, &e);
  if (!dbuf) return hip_fail(c, e, "hanf_batch_stats_all_noalloc: device address of the statistics array");
  e = launch_stats_all(c->args, alpha, eps, distinct ? 1 : 0, dbuf, c->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(out, dbuf, sizeof(StatsRec) * (size_t)c->n_comp, hipMemcpyDeviceToHost, c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) return hip_fail(c, e, "statistics");
  return HANF_OK;
}

static_assert(sizeof(StatsRec) == sizeof(hanf_stats_t), "StatsRec must have hanf_stats_t's layout");
static_assert(offsetof(StatsRec, T) == offsetof(hanf_stats_t, T), "StatsRec must have hanf_stats_t's layout");
static_assert(offsetof(StatsRec, distinct) == offsetof(hanf_stats_t, distinct),
              "StatsRec must have hanf_stats_t's layout");

int hanf_device_bytes(const hanf_ctx *c, int64_t *held, int64_t *pooled) {
  if (!c) return fail(nullptr, HANF_EINVAL, "hanf_device_bytes: NULL context");
  int64_t h = 0, p = 0;
  for (const auto &kv : c->sizes) h += (int64_t)kv.second;
  for (const auto &kv : c->pool) p += (int64_t)kv.first;
  if (held) *held = h;
  if (pooled) *pooled = p;
  return HANF_OK;
}

int hanf_trim(hanf_ctx *c) {
  if (!c) return fail(nullptr, HANF_EINVAL, "hanf_trim: NULL context");
  HIP_TRY(c, hipSetDevice(c->device), "set device");
  HIP_TRY(c, hipStreamSynchronize(c->stream), "sync");
  for (auto &kv : c->pool) {
    c->sizes.erase(kv.second);
    (void)hipFree(kv.second);
  }
  c->pool.clear();
  return HANF_OK;
}

const char *hanf_last_error(const hanf_ctx *c) { return c ? c->err.c_str() : g_thread_error.c_str(); }

int hanf_max5_groups(int device, const uint8_t *x, const uint8_t *y, uint8_t *out, int64_t groups) {
  if (!x || !y || !out || groups < 0) return fail(nullptr, HANF_EINVAL, "hanf_max5_groups: bad argument");
  if (((uintptr_t)x | (uintptr_t)y | (uintptr_t)out) & 7u)
    return fail(nullptr, HANF_EINVAL, "hanf_max5_groups: buffers must be 8-byte aligned");
  hipError_t e = hipSetDevice(device);
  if (e == hipSuccess && groups > 0) e = launch_max5_groups(x, y, out, groups, nullptr);
  if (e == hipSuccess) e = hipDeviceSynchronize();
  if (e != hipSuccess) return hip_fail(nullptr, e, "hanf_max5_groups");
  return HANF_OK;
}

int hanf_gathermax_lanes(int device, const uint32_t *x, int32_t k, int32_t from_first, uint32_t *out, int64_t count) {
  if (!x || !out || k < 1 || count < 0 || (from_first != 0 && from_first != 1))
    return fail(nullptr, HANF_EINVAL, "hanf_gathermax_lanes: bad argument");
  if ((reinterpret_cast<uintptr_t>(x) | reinterpret_cast<uintptr_t>(out)) & 15)
    return fail(nullptr, HANF_EINVAL, "hanf_gathermax_lanes: buffers must be 16-byte aligned");
  hipError_t e = hipSetDevice(device);
  if (e == hipSuccess && count > 0)
    e = launch_gathermax_lanes(reinterpret_cast<const uint4 *>(x), k, from_first, reinterpret_cast<uint4 *>(out),
                               count, nullptr);
  if (e == hipSuccess) e = hipDeviceSynchronize();
  if (e != hipSuccess) return hip_fail(nullptr, e, "hanf_gathermax_lanes");
  return HANF_OK;
}

int hanf_bytemax_words(int device, const uint32_t *x, const uint32_t *y, uint32_t *out, int64_t count) {
  if (!x || !y || !out || count < 0) return fail(nullptr, HANF_EINVAL, "hanf_bytemax_words: bad argument");
  hipError_t e = hipSetDevice(device);
  if (e == hipSuccess && count > 0) e = launch_bytemax_words(x, y, out, count, nullptr);
  if (e == hipSuccess) e = hipDeviceSynchronize();
  if (e != hipSuccess) return hip_fail(nullptr, e, "hanf_bytemax_words");
  return HANF_OK;
}

}  // extern "C"
