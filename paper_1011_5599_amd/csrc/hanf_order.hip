// Node order chosen at ingest (hub grouping) and the row gathers that map between it and
// the caller's node ids.
//
// Every arc makes the union step read its target's counter (Algorithm 2), so a node of
// in-degree d has its row read d times per pass over every node. With 64-byte rows and
// 128-byte L2 lines, rows of the most-read nodes scattered over the id range waste half of
// every line they occupy, and each of them shares its line with a row that is rarely read.
// Giving the K most-read nodes the first K ids packs their rows into K/2 lines that stay in
// one XCD's L2. The order is a layout choice only: counters are still hashed from the
// caller's ids, so every register, every N_hat(t) and the fixpoint are those of the
// caller's labelling (N_hat up to the order of its floating-point sum).
//
// Order: hubs first, by class of in-degree (8 classes per octave), larger classes first,
// by id within a class; every other node after them, by id. Deterministic: the classes
// come from a histogram and the ranks from a stable scatter. Rewriting the graph renames
// every arc's target, so the order is chosen once per ingest and kept for every run on it.
#include "hanf_internal.h"

namespace hanf {

namespace {

constexpr int kOrderBlock = 1024;  // nodes per block of the stable scatter (16 rounds of a wavefront)
constexpr int kPermWindow = 1024;  // arc positions per wavefront of the CSR permutation
constexpr int kPermRows = 512;     // row starts a wavefront stages in LDS

// Class level of in-degree d >= 1: d itself below 8, then 8 levels per octave from the three
// bits below the leading one; nondecreasing in d, at most kOrderTopLevel (239). Level 0 is
// in-degree 0.
__device__ __forceinline__ int degree_level(uint32_t d) {
  if (d == 0) return 0;
  const int e = 31 - __clz(d);
  if (e < 3) return (int)d;
  return 8 * (e - 2) + (int)((d >> (e - 3)) & 7u);
}

// Output class of a node: hubs (level >= lstar) by decreasing level, then the rest.
__device__ __forceinline__ int order_class(uint32_t d, int lstar) {
  const int l = degree_level(d);
  return (d > 0 && l >= lstar) ? kOrderTopLevel - l : kOrderRest;
}

__global__ void k_degrees_rp(const int32_t *rp, int32_t n, uint32_t *deg) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += stride)
    deg[v] = (uint32_t)(rp[v + 1] - rp[v]);
}

__global__ void k_fill_u32(uint32_t *p, int64_t count, uint32_t value) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += stride) p[i] = value;
}

__global__ void k_degrees_count(const int32_t *ci, int64_t arcs, uint32_t *deg) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < arcs; p += stride)
    atomicAdd(&deg[ci[p]], 1u);
}

__global__ __launch_bounds__(kBlockThreads) void k_level_hist(const uint32_t *deg, int32_t n, uint32_t *hist) {
  __shared__ uint32_t h[kOrderLevels];
  for (int i = threadIdx.x; i < kOrderLevels; i += kBlockThreads) h[i] = 0;
  __syncthreads();
  const int64_t stride = (int64_t)gridDim.x * kBlockThreads;
  for (int64_t v = (int64_t)blockIdx.x * kBlockThreads + threadIdx.x; v < n; v += stride)
    atomicAdd(&h[degree_level(deg[v])], 1u);
  __syncthreads();
  for (int i = threadIdx.x; i < kOrderLevels; i += kBlockThreads)
    if (h[i]) atomicAdd(&hist[i], h[i]);
}

// lstar: the lowest level such that the nodes at this level or above number at most K
// (kOrderLevels when even the top level holds more than K nodes: no hubs).
__global__ __launch_bounds__(kWave) void k_order_plan(const uint32_t *hist, int64_t K, int32_t *plan) {
  __shared__ uint32_t h[kOrderLevels];
  for (int i = threadIdx.x; i < kOrderLevels; i += kWave) h[i] = hist[i];
  __syncthreads();
  if (threadIdx.x != 0) return;
  int64_t cum = 0;
  int lstar = kOrderLevels;
  for (int l = kOrderLevels - 1; l >= 1; --l) {
    cum += h[l];
    if (cum > K) break;
    lstar = l;
  }
  plan[0] = lstar;
}

// Per block of kOrderBlock nodes: nodes of each class, stored class-major (class c of block
// b at c * n_blk + b), so that one exclusive scan gives every class's first new id in
// every block.
__global__ __launch_bounds__(kBlockThreads) void k_order_count(const uint32_t *deg, int32_t n, const int32_t *plan,
                                                               int32_t n_blk, uint64_t *counts) {
  __shared__ uint32_t h[kOrderClasses];
  for (int i = threadIdx.x; i < kOrderClasses; i += kBlockThreads) h[i] = 0;
  __syncthreads();
  const int lstar = plan[0];
  const int64_t b0 = (int64_t)blockIdx.x * kOrderBlock;
  for (int i = threadIdx.x; i < kOrderBlock; i += kBlockThreads) {
    const int64_t v = b0 + i;
    if (v < n) atomicAdd(&h[order_class(deg[v], lstar)], 1u);
  }
  __syncthreads();
  for (int i = threadIdx.x; i < kOrderClasses; i += kBlockThreads)
    counts[(int64_t)i * n_blk + blockIdx.x] = h[i];
}

// One wavefront per block of kOrderBlock nodes, in id order, 64 at a time: the lanes of one
// class take consecutive new ids from that class's cursor in the block (stable ranks).
__global__ __launch_bounds__(kWave) void k_order_scatter(const uint32_t *deg, int32_t n, const int32_t *plan,
                                                          int32_t n_blk, const uint64_t *offs, int32_t *perm,
                                                          int32_t *inv) {
  __shared__ int32_t cur[kOrderClasses];
  const int lane = threadIdx.x;
  for (int i = lane; i < kOrderClasses; i += kWave) cur[i] = (int32_t)offs[(int64_t)i * n_blk + blockIdx.x];
  __syncthreads();
  const int lstar = plan[0];
  const uint64_t below = (1ull << lane) - 1ull;
  const int64_t b0 = (int64_t)blockIdx.x * kOrderBlock;
  for (int r = 0; r < kOrderBlock; r += kWave) {
    const int64_t v = b0 + r + lane;
    const bool valid = v < n;
    const int cls = valid ? order_class(deg[v], lstar) : -1;
    uint64_t pending = __ballot(valid);
    while (pending) {
      const int leader = __ffsll((long long)pending) - 1;
      const int c = __shfl(cls, leader);
      const uint64_t mask = __ballot(cls == c);
      const int32_t base = cur[c];
      if (cls == c) {
        const int32_t id = base + __popcll(mask & below);
        perm[id] = (int32_t)v;
        inv[v] = id;
      }
      __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
      __builtin_amdgcn_wave_barrier();
      if (lane == leader) cur[c] = base + __popcll(mask);
      __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
      __builtin_amdgcn_wave_barrier();
      pending &= ~mask;
    }
  }
}

// keys[v] = arcs of the node given id v (its old row perm[v]); keys[n] = 0.
__global__ void k_order_degrees(const int32_t *rp, const int32_t *perm, int32_t n, uint64_t *keys) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v <= n; v += stride) {
    if (v == n) {
      keys[v] = 0;
    } else {
      const int32_t u = perm[v];
      keys[v] = (uint64_t)(rp[u + 1] - rp[u]);
    }
  }
}

__global__ void k_keys_to_rp(const uint64_t *keys, int32_t n, int32_t *rp) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v <= n; v += stride) rp[v] = (int32_t)keys[v];
}

// Renaming table of the order, for the arcs' targets. The H hubs take new ids 0 .. H - 1 and
// every other node keeps its place among the others, so a non-hub w becomes H + w - (hubs
// with an id below w), and a hub becomes hub_new[hubs with an id below w], where hub_new
// lists the hubs' new ids in old-id order. Per group of 64 consecutive old ids a 16-byte
// record holds the group's hub bits and the hubs in earlier groups, so one record read and
// a popcount give the count. Records (n / 4 bytes) and hub_new (4 bytes per hub) stay in an
// XCD's L2 at sizes where inv (4 bytes per node, read at random) would not: 2^22 nodes take
// 1 MiB of records against 16 MiB of inv.
// First step: each group's hub bits (the nodes with inv < H) and hub count; gcount[n_groups]
// = 0 closes the array for an exclusive scan.
__global__ __launch_bounds__(kBlockThreads) void k_rename_bits(const int32_t *inv, int32_t n, int32_t H,
                                                               int64_t n_groups, uint4 *rec, uint64_t *gcount) {
  const int lane = threadIdx.x & 63;
  const int64_t waves = ((int64_t)gridDim.x * kBlockThreads) >> 6;
  if (blockIdx.x == 0 && threadIdx.x == 0) gcount[n_groups] = 0;
  for (int64_t g = ((int64_t)blockIdx.x * kBlockThreads + threadIdx.x) >> 6; g < n_groups; g += waves) {
    const int64_t v = g * kWave + lane;
    const uint64_t bits = __ballot(v < n && inv[v] < H);
    if (lane == 0) {
      rec[g] = make_uint4((uint32_t)bits, (uint32_t)(bits >> 32), 0u, 0u);
      gcount[g] = (uint64_t)__popcll(bits);
    }
  }
}

// Second step, after the exclusive scan of gcount: each record's count of earlier hubs, and
// every hub's new id at its rank in old-id order.
__global__ __launch_bounds__(kBlockThreads) void k_rename_hubs(const int32_t *inv, int32_t n, int64_t n_groups,
                                                               const uint64_t *gprefix, uint4 *rec,
                                                               int32_t *hub_new) {
  const int lane = threadIdx.x & 63;
  const int64_t waves = ((int64_t)gridDim.x * kBlockThreads) >> 6;
  for (int64_t g = ((int64_t)blockIdx.x * kBlockThreads + threadIdx.x) >> 6; g < n_groups; g += waves) {
    const uint4 r = rec[g];
    const uint64_t bits = ((uint64_t)r.y << 32) | r.x;
    const uint32_t before = (uint32_t)gprefix[g];
    const int64_t v = g * kWave + lane;
    if ((bits >> lane) & 1ull) hub_new[before + __popcll(bits & ((1ull << lane) - 1ull))] = inv[v];
    if (lane == 0) rec[g].z = before;
  }
}

// wrow[k]: the row that holds old position k * kPermWindow (every such position lies in
// exactly one row with arcs, so each entry is written once); wrow[windows] = n - 1 closes the
// last window.
__global__ void k_window_rows(const int32_t *rp, int32_t n, int64_t windows, int32_t *wrow) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (gid == 0) wrow[windows] = n - 1;
  for (int64_t r = gid; r < n; r += stride) {
    const int64_t a = rp[r], b = rp[r + 1];
    for (int64_t q = (a + kPermWindow - 1) / kPermWindow; q * kPermWindow < b; ++q) wrow[q] = (int32_t)r;
  }
}

// The arcs in the new order: the arc at old position p, in old row u, goes to new position
// rp_new[inv[u]] + (p - rp[u]) with its target renamed (inv[ci[p]], taken from the renaming
// table). One wavefront per window of kPermWindow consecutive old positions (reads in order;
// each row's arcs are written in order). The window's rows run from the row of its first
// position to the row of the next window's first position (k_window_rows); up to kPermRows
// of them are staged in LDS with their start and the shift to their new place, so an arc's
// row and destination come from an LDS search. The window's positions go in batches of
// kPermBatch steps of 64: first every successor id of the batch is loaded, then every
// renaming record, then the hub entries, so each kind of load has a batch in flight at once.
constexpr int kPermBatch = 8;
static_assert(kPermWindow % (kPermBatch * kWave) == 0, "whole batches per window");

__global__ __launch_bounds__(kBlockThreads) void k_permute_csr(const int32_t *__restrict__ rp,
                                                               const int32_t *__restrict__ ci, int32_t n,
                                                               int32_t arcs, const int32_t *__restrict__ inv,
                                                               const uint4 *__restrict__ rec,
                                                               const int32_t *__restrict__ hub_new, int32_t H,
                                                               const int32_t *__restrict__ wrow,
                                                               const int32_t *__restrict__ rp_new,
                                                               int32_t *__restrict__ ci_new) {
  __shared__ int32_t starts_all[kBlockThreads / kWave][kPermRows];
  __shared__ int32_t shift_all[kBlockThreads / kWave][kPermRows];
  const int lane = threadIdx.x & 63;
  int32_t *starts = starts_all[threadIdx.x >> 6];
  int32_t *shift = shift_all[threadIdx.x >> 6];
  const int64_t wave = ((int64_t)blockIdx.x * kBlockThreads + threadIdx.x) >> 6;
  const int64_t p0_64 = wave * kPermWindow;
  if (p0_64 >= arcs) return;  // wavefront-uniform
  const int32_t p0 = (int32_t)p0_64;
  const int32_t p1 = (int32_t)min((int64_t)arcs, p0_64 + kPermWindow) - 1;
  // rows r0 .. r0 + rows - 1 hold every position of the window (and possibly a row after it,
  // which starts past the window and is never the row of a position in it)
  const int32_t r0 = wrow[wave], rows = wrow[wave + 1] - r0 + 1;
  const bool staged = rows <= kPermRows;
  if (staged)
    for (int32_t i = lane; i < rows; i += kWave) {
      const int32_t st = rp[r0 + i];
      starts[i] = st;
      shift[i] = rp_new[inv[r0 + i]] - st;  // arc p of the row goes to p + shift
    }
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
  for (int s0 = 0; s0 < kPermWindow; s0 += kPermBatch * kWave) {
    int32_t w[kPermBatch], nw[kPermBatch];
    uint4 r[kPermBatch];
#pragma unroll
    for (int k = 0; k < kPermBatch; ++k) {
      const int32_t p = p0 + s0 + k * kWave + lane;
      w[k] = p <= p1 ? ci[p] : 0;  // (id 0 past the window: renamed, never stored)
    }
#pragma unroll
    for (int k = 0; k < kPermBatch; ++k) r[k] = rec[(uint32_t)w[k] >> 6];
#pragma unroll
    for (int k = 0; k < kPermBatch; ++k) {
      const uint64_t bits = ((uint64_t)r[k].y << 32) | r[k].x;
      const int b = w[k] & 63;
      const int32_t below = (int32_t)r[k].z + __popcll(bits & ((1ull << b) - 1ull));
      nw[k] = ((bits >> b) & 1ull) ? hub_new[below] : H + (w[k] - below);
    }
#pragma unroll
    for (int k = 0; k < kPermBatch; ++k) {
      const int32_t p = p0 + s0 + k * kWave + lane;
      if (p > p1) continue;
      // the last of rows r0 .. r0 + rows - 1 starting at or before p
      int32_t a = 0, b = rows;
      int32_t dst;
      if (staged) {
        while (b - a > 1) {
          const int32_t mid = (a + b) >> 1;
          if (starts[mid] <= p) a = mid; else b = mid;
        }
        dst = p + shift[a];
      } else {
        while (b - a > 1) {
          const int32_t mid = (a + b) >> 1;
          if (rp[r0 + mid] <= p) a = mid; else b = mid;
        }
        dst = rp_new[inv[r0 + a]] + (p - rp[r0 + a]);
      }
      ci_new[dst] = nw[k];
    }
  }
}

// dst row i = src row idx[i], rows of `words` 8-byte words.
__global__ void k_gather_rows(const uint2 *src, uint2 *dst, const int32_t *idx, int32_t n, int64_t words) {
  const int64_t total = (int64_t)n * words;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g < total; g += stride) {
    const int64_t i = g / words, w = g - i * words;
    dst[g] = src[(int64_t)idx[i] * words + w];
  }
}

__global__ void k_iota(int32_t *p, int32_t n) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) p[i] = (int32_t)i;
}

unsigned grid_of(int64_t items, int per_block, int64_t cap) {
  int64_t g = (items + per_block - 1) / per_block;
  if (g < 1) g = 1;
  if (g > cap) g = cap;
  return (unsigned)g;
}

}  // namespace

int64_t order_counts_elems(int32_t n) {
  return (int64_t)kOrderClasses * (((int64_t)n + kOrderBlock - 1) / kOrderBlock);
}

hipError_t launch_in_degrees(const int32_t *trp, const int32_t *ci, int32_t n, int64_t arcs, uint32_t *deg,
                             hipStream_t s) {
  if (trp) {
    hipLaunchKernelGGL(k_degrees_rp, dim3(grid_of(n, kBlockThreads, 4096)), dim3(kBlockThreads), 0, s, trp, n, deg);
    return hipGetLastError();
  }
  hipLaunchKernelGGL(k_fill_u32, dim3(grid_of(n, kBlockThreads, 4096)), dim3(kBlockThreads), 0, s, deg, (int64_t)n, 0u);
  if (arcs > 0)
    hipLaunchKernelGGL(k_degrees_count, dim3(grid_of(arcs, kBlockThreads, 8192)), dim3(kBlockThreads), 0, s, ci, arcs,
                       deg);
  return hipGetLastError();
}

hipError_t launch_order_select(const uint32_t *deg, int32_t n, int64_t K, uint32_t *hist, int32_t *plan,
                               uint64_t *counts, uint64_t *scan_tmp, int32_t *perm, int32_t *inv, hipStream_t s) {
  const int32_t n_blk = (int32_t)(((int64_t)n + kOrderBlock - 1) / kOrderBlock);
  hipLaunchKernelGGL(k_fill_u32, dim3(1), dim3(kBlockThreads), 0, s, hist, (int64_t)kOrderLevels, 0u);
  hipLaunchKernelGGL(k_level_hist, dim3(grid_of(n, kBlockThreads * 16, 1024)), dim3(kBlockThreads), 0, s, deg, n, hist);
  hipLaunchKernelGGL(k_order_plan, dim3(1), dim3(kWave), 0, s, hist, K, plan);
  hipLaunchKernelGGL(k_order_count, dim3((unsigned)n_blk), dim3(kBlockThreads), 0, s, deg, n, plan, n_blk, counts);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if ((e = launch_exclusive_scan_u64(counts, order_counts_elems(n), scan_tmp, s)) != hipSuccess) return e;
  hipLaunchKernelGGL(k_order_scatter, dim3((unsigned)n_blk), dim3(kWave), 0, s, deg, n, plan, n_blk, counts, perm, inv);
  return hipGetLastError();
}

int64_t rename_groups(int32_t n) { return ((int64_t)n + kWave - 1) / kWave; }
int64_t permute_windows(int64_t arcs) { return (arcs + kPermWindow - 1) / kPermWindow; }

hipError_t launch_permute_csr(const int32_t *rp, const int32_t *ci, int32_t n, int64_t arcs, const int32_t *perm,
                              const int32_t *inv, int32_t H, uint64_t *keys, uint64_t *scan_tmp, uint4 *rec,
                              int32_t *hub_new, int32_t *wrow, int32_t *rp_new, int32_t *ci_new, hipStream_t s) {
  hipLaunchKernelGGL(k_order_degrees, dim3(grid_of((int64_t)n + 1, kBlockThreads, 4096)), dim3(kBlockThreads), 0, s,
                     rp, perm, n, keys);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if ((e = launch_exclusive_scan_u64(keys, (int64_t)n + 1, scan_tmp, s)) != hipSuccess) return e;
  hipLaunchKernelGGL(k_keys_to_rp, dim3(grid_of((int64_t)n + 1, kBlockThreads, 4096)), dim3(kBlockThreads), 0, s,
                     keys, n, rp_new);
  if (arcs > 0) {
    // the renaming table; keys (n + 1 entries, read by k_keys_to_rp before) holds the group
    // counts (n_groups + 1 <= n + 1 entries)
    const int64_t n_groups = rename_groups(n);
    const unsigned wgs = grid_of(n_groups, kBlockThreads / kWave, 4096);
    hipLaunchKernelGGL(k_rename_bits, dim3(wgs), dim3(kBlockThreads), 0, s, inv, n, H, n_groups, rec, keys);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if ((e = launch_exclusive_scan_u64(keys, n_groups + 1, scan_tmp, s)) != hipSuccess) return e;
    hipLaunchKernelGGL(k_rename_hubs, dim3(wgs), dim3(kBlockThreads), 0, s, inv, n, n_groups, keys, rec, hub_new);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    const int64_t waves = permute_windows(arcs);
    hipLaunchKernelGGL(k_window_rows, dim3(grid_of(n, kBlockThreads, 4096)), dim3(kBlockThreads), 0, s, rp, n, waves,
                       wrow);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(k_permute_csr, dim3((unsigned)((waves + 3) / 4)), dim3(kBlockThreads), 0, s, rp, ci, n,
                       (int32_t)arcs, inv, rec, hub_new, H, wrow, rp_new, ci_new);
  }
  return hipGetLastError();
}

hipError_t launch_gather_rows(const uint8_t *src, uint8_t *dst, const int32_t *idx, int32_t n, int64_t row_bytes,
                              hipStream_t s) {
  const int64_t words = row_bytes / 8;
  hipLaunchKernelGGL(k_gather_rows, dim3(grid_of((int64_t)n * words, kBlockThreads, 16384)), dim3(kBlockThreads), 0, s,
                     (const uint2 *)src, (uint2 *)dst, idx, n, words);
  return hipGetLastError();
}

hipError_t launch_iota(int32_t *p, int32_t n, hipStream_t s) {
  hipLaunchKernelGGL(k_iota, dim3(grid_of(n, kBlockThreads, 4096)), dim3(kBlockThreads), 0, s, p, n);
  return hipGetLastError();
}

}  // namespace hanf
