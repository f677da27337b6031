// Seeded synthetic graph generators producing CSR int32 (row_ptr[n+1], col_idx[arcs]).
//
// This module only builds input graphs. It holds none of HyperANF's arithmetic
// (no counter hashing, no register maximisation, no estimator) and is shared by
// the tests and the benchmark to feed the same graph to the CPU oracle and to
// the GPU library.
//
// Determinism: every random draw comes from xoshiro256** streams whose state is
// expanded from (graph seed, stream id) with the MurmurHash3 64-bit finaliser.
// Streams are tied to fixed work units (sample chunks, node ids), never to
// threads, so the output bytes do not depend on the thread count.
//
// Successor lists are sorted ascending, self-loops and duplicate arcs removed.

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstdlib>
#include <cstring>
#include <numeric>
#include <vector>
#include <omp.h>

namespace {

inline uint64_t fmix64(uint64_t k) {  // MurmurHash3 finaliser, used only for seed expansion
  k ^= k >> 33;
  k *= 0xff51afd7ed558ccdULL;
  k ^= k >> 33;
  k *= 0xc4ceb9fe1a85ec53ULL;
  k ^= k >> 33;
  return k;
}

inline uint64_t rotl(uint64_t x, int k) { return (x << k) | (x >> (64 - k)); }

struct Rng {  // xoshiro256** (Blackman & Vigna)
  uint64_t s[4];
  Rng(uint64_t seed, uint64_t stream) {
    uint64_t x = fmix64(seed * 0x9ddfea08eb382d69ULL + 0x243f6a8885a308d3ULL) ^
                 fmix64(stream + 0x13198a2e03707344ULL);
    for (int i = 0; i < 4; i++) {
      x = fmix64(x + 0xa4093822299f31d0ULL * (uint64_t)(i + 1));
      s[i] = x | (i == 0 ? 1ULL : 0ULL);
    }
  }
  inline uint64_t next() {
    const uint64_t r = rotl(s[1] * 5, 7) * 9;
    const uint64_t t = s[1] << 17;
    s[2] ^= s[0];
    s[3] ^= s[1];
    s[1] ^= s[2];
    s[0] ^= s[3];
    s[2] ^= t;
    s[3] = rotl(s[3], 45);
    return r;
  }
  inline double uniform() { return (double)(next() >> 11) * 0x1.0p-53; }  // [0,1)
  inline uint64_t below(uint64_t bound) {  // unbiased integer in [0, bound)
    const uint64_t lim = (~0ULL) - ((~0ULL) % bound) - 1;
    uint64_t x;
    do { x = next(); } while (x > lim);
    return x % bound;
  }
  inline double normal() {  // Box-Muller, one output per call
    double u1 = uniform();
    while (u1 <= 0.0) u1 = uniform();
    const double u2 = uniform();
    return std::sqrt(-2.0 * std::log(u1)) * std::cos(6.283185307179586 * u2);
  }
};

// Open-addressing set of nonzero 64-bit keys; keeps first occurrences in insertion order.
struct KeySet {
  std::vector<uint64_t> slot;
  uint64_t mask;
  explicit KeySet(uint64_t expected) {
    uint64_t cap = 16;
    while (cap < expected * 2) cap <<= 1;
    slot.assign(cap, 0);
    mask = cap - 1;
  }
  bool insert(uint64_t key) {  // true if new
    uint64_t h = fmix64(key) & mask;
    for (;;) {
      const uint64_t s = slot[h];
      if (s == key) return false;
      if (s == 0) { slot[h] = key; return true; }
      h = (h + 1) & mask;
    }
  }
};

void random_permutation(int64_t n, uint64_t seed, uint64_t stream, std::vector<int32_t> &perm) {
  perm.resize(n);
  std::iota(perm.begin(), perm.end(), 0);
  Rng r(seed, stream);
  for (int64_t i = n - 1; i > 0; i--) {
    const int64_t j = (int64_t)r.below((uint64_t)i + 1);
    std::swap(perm[i], perm[j]);
  }
}

// Builds a CSR from (src, dst) pairs: counting sort by source, then sort + dedupe rows.
int build_csr(int32_t n, const std::vector<int32_t> &src, const std::vector<int32_t> &dst,
              int32_t **row_ptr_out, int32_t **col_out, int64_t *arcs_out) {
  const int64_t e = (int64_t)src.size();
  std::vector<int64_t> cnt((size_t)n + 1, 0);
  for (int64_t i = 0; i < e; i++) cnt[(size_t)src[i] + 1]++;
  for (int32_t v = 0; v < n; v++) cnt[(size_t)v + 1] += cnt[v];
  std::vector<int32_t> col((size_t)e);
  {
    std::vector<int64_t> pos(cnt.begin(), cnt.end() - 1);
    for (int64_t i = 0; i < e; i++) col[(size_t)pos[src[i]]++] = dst[i];
  }
  std::vector<int64_t> keep((size_t)n, 0);
#pragma omp parallel for schedule(dynamic, 4096)
  for (int32_t v = 0; v < n; v++) {
    int32_t *b = col.data() + cnt[v], *en = col.data() + cnt[(size_t)v + 1];
    std::sort(b, en);
    int32_t *w = b;
    for (int32_t *p = b; p < en; p++)
      if (*p != v && (w == b || *(w - 1) != *p)) *w++ = *p;
    keep[v] = w - b;
  }
  int32_t *rp = (int32_t *)std::malloc(sizeof(int32_t) * ((size_t)n + 1));
  int64_t total = 0;
  for (int32_t v = 0; v < n; v++) total += keep[v];
  if (total >= (int64_t)INT32_MAX) { std::free(rp); return -2; }
  int32_t *ci = (int32_t *)std::malloc(sizeof(int32_t) * (size_t)std::max<int64_t>(total, 1));
  if (!rp || !ci) { std::free(rp); std::free(ci); return -3; }
  int64_t acc = 0;
  for (int32_t v = 0; v < n; v++) { rp[v] = (int32_t)acc; acc += keep[v]; }
  rp[n] = (int32_t)acc;
#pragma omp parallel for schedule(dynamic, 4096)
  for (int32_t v = 0; v < n; v++)
    std::memcpy(ci + rp[v], col.data() + cnt[v], sizeof(int32_t) * (size_t)keep[v]);
  *row_ptr_out = rp;
  *col_out = ci;
  *arcs_out = total;
  return 0;
}

// One R-MAT endpoint pair on 2^scale ids; probabilities as 32-bit fixed-point thresholds.
struct RmatQ {
  uint64_t ta, tab, tabc;
  RmatQ(double a, double b, double c) {
    ta = (uint64_t)std::llround(a * 4294967296.0);
    tab = (uint64_t)std::llround((a + b) * 4294967296.0);
    tabc = (uint64_t)std::llround((a + b + c) * 4294967296.0);
  }
  inline void sample(Rng &r, int scale, uint64_t &u, uint64_t &v) const {
    u = 0; v = 0;
    uint64_t bits = 0;
    for (int l = 0; l < scale; l++) {
      if ((l & 1) == 0) bits = r.next();
      const uint64_t x = (l & 1) ? (bits >> 32) : (bits & 0xffffffffULL);
      u <<= 1; v <<= 1;
      if (x < ta) {
      } else if (x < tab) {
        v |= 1;
      } else if (x < tabc) {
        u |= 1;
      } else {
        u |= 1; v |= 1;
      }
    }
  }
};

const int64_t kChunk = 1 << 16;  // samples per RNG stream

}  // namespace

extern "C" {

// Directed or symmetric R-MAT on 2^scale ids (or on the first n_nodes of them, by rejection).
// Directed: distinct non-loop ordered pairs are taken in sample order until `target` arcs.
// Symmetric: distinct unordered non-loop pairs until `target` edges, each emitted in both
// directions (2*target arcs). Ids are relabelled by a seeded uniform permutation.
int gg_rmat(int scale, int64_t target, double a, double b, double c, int symmetric,
            uint64_t seed, int64_t n_nodes, int32_t *n_out, int64_t *arcs_out, int32_t **row_ptr,
            int32_t **col_idx) {
  if (scale < 1 || scale > 30 || target < 0) return -1;
  // n_nodes > 0: R-MAT on 2^scale ids, samples with an endpoint >= n_nodes rejected
  const int64_t n = n_nodes > 0 ? n_nodes : (1LL << scale);
  if (n > (1LL << scale)) return -1;
  const double max_pairs = symmetric ? (double)n * (double)(n - 1) / 2.0 : (double)n * (double)(n - 1);
  if ((double)target > 0.5 * max_pairs) return -1;
  RmatQ q(a, b, c);
  KeySet seen((uint64_t)target + 16);
  std::vector<int32_t> src, dst;
  src.reserve((size_t)target);
  dst.reserve((size_t)target);
  int64_t chunk_id = 0;
  std::vector<uint64_t> buf;
  while ((int64_t)src.size() < target) {
    // Draw a batch of chunks in parallel (each chunk its own stream), consume in order.
    const int64_t need = target - (int64_t)src.size();
    const int64_t nchunks = std::max<int64_t>(1, std::min<int64_t>(256, (need * 5 / 4) / kChunk + 1));
    buf.assign((size_t)(nchunks * kChunk), 0);
#pragma omp parallel for schedule(static)
    for (int64_t k = 0; k < nchunks; k++) {
      Rng r(seed, (uint64_t)(chunk_id + k));
      for (int64_t i = 0; i < kChunk; i++) {
        uint64_t u, v;
        q.sample(r, scale, u, v);
        if (symmetric && u > v) std::swap(u, v);
        buf[(size_t)(k * kChunk + i)] = (u == v || (int64_t)u >= n || (int64_t)v >= n) ? 0 : ((u << 32) | v) + 1;
      }
    }
    chunk_id += nchunks;
    for (size_t i = 0; i < buf.size() && (int64_t)src.size() < target; i++) {
      const uint64_t key = buf[i];
      if (key == 0 || !seen.insert(key)) continue;
      src.push_back((int32_t)((key - 1) >> 32));
      dst.push_back((int32_t)((key - 1) & 0xffffffffULL));
    }
  }
  std::vector<int32_t> perm;
  random_permutation(n, seed, 0xfeedULL << 32, perm);
  const int64_t e = (int64_t)src.size();
  for (int64_t i = 0; i < e; i++) { src[i] = perm[src[i]]; dst[i] = perm[dst[i]]; }
  if (symmetric) {
    src.resize((size_t)(2 * e));
    dst.resize((size_t)(2 * e));
    for (int64_t i = 0; i < e; i++) { src[e + i] = dst[i]; dst[e + i] = src[i]; }
  }
  *n_out = (int32_t)n;
  return build_csr((int32_t)n, src, dst, row_ptr, col_idx, arcs_out);
}

// Directed Erdos-Renyi with exactly `target` distinct non-loop arcs on n nodes.
int gg_er(int32_t n, int64_t target, uint64_t seed, int32_t *n_out, int64_t *arcs_out,
          int32_t **row_ptr, int32_t **col_idx) {
  if (n < 1 || target < 0) return -1;
  if ((double)target > 0.5 * (double)n * (double)(n - 1)) return -1;
  KeySet seen((uint64_t)target + 16);
  std::vector<int32_t> src, dst;
  src.reserve((size_t)target);
  dst.reserve((size_t)target);
  uint64_t stream = 0;
  while ((int64_t)src.size() < target) {
    Rng r(seed, stream++);
    for (int64_t i = 0; i < kChunk && (int64_t)src.size() < target; i++) {
      const uint64_t u = r.below((uint64_t)n), v = r.below((uint64_t)n);
      if (u == v) continue;
      if (!seen.insert(((u << 32) | v) + 1)) continue;
      src.push_back((int32_t)u);
      dst.push_back((int32_t)v);
    }
  }
  *n_out = n;
  return build_csr(n, src, dst, row_ptr, col_idx, arcs_out);
}

// Hosts of the web-like graph: contiguous id ranges with LogNormal sizes of mean
// host_mean (shape host_sigma), drawn from one sequential stream of the graph seed.
static void web_hosts(int32_t n, double host_mean, double host_sigma, uint64_t seed,
                      std::vector<int32_t> &host_lo, std::vector<int32_t> &host_hi) {
  host_lo.assign((size_t)n, 0);
  host_hi.assign((size_t)n, 0);
  Rng r(seed, 1);
  const double mu = std::log(host_mean) - 0.5 * host_sigma * host_sigma;
  int64_t lo = 0;
  while (lo < n) {
    int64_t sz = std::llround(std::exp(mu + host_sigma * r.normal()));
    if (sz < 1) sz = 1;
    const int64_t hi = std::min<int64_t>(n, lo + sz);
    for (int64_t v = lo; v < hi; v++) { host_lo[v] = (int32_t)lo; host_hi[v] = (int32_t)(hi - 1); }
    lo = hi;
  }
}

// First id of each node's host (n entries), as gg_web draws the hosts.
int gg_web_hosts(int32_t n, double host_mean, double host_sigma, uint64_t seed, int32_t *host_first) {
  if (n < 2 || host_mean < 1 || !host_first) return -1;
  std::vector<int32_t> lo, hi;
  web_hosts(n, host_mean, host_sigma, seed, lo, hi);
  std::memcpy(host_first, lo.data(), sizeof(int32_t) * (size_t)n);
  return 0;
}

// Web-like directed graph. Hosts are contiguous id ranges with LogNormal sizes of mean
// `host_mean` (shape host_sigma); out-degrees are round(LogNormal) with mean `deg_mean`
// (shape deg_sigma). Each arc is intra-host with probability p_intra, to v +/- a
// Geometric(geo_p) offset clamped into the host, else inter-host, to a node drawn with
// weight rank^(-1/(gamma-1)) over a seeded random ranking (Chung-Lu; power-law in-degree
// with exponent gamma) through a Vose alias table.
// A duplicate or self-loop target is drawn again. With keep_kind = 0 every draw takes a
// new intra/inter choice; nearby ids repeat far more often than power-law targets, so
// fewer than p_intra of the kept arcs are intra-host. With keep_kind = 1 the choice is
// taken once per arc and only the target is drawn again: an intra-host arc that finds no
// free nearby id draws over the whole host, and one that finds no free id in the host
// becomes inter-host, so p_intra holds for the kept arcs up to nodes whose host runs out.
int gg_web(int32_t n, double host_mean, double host_sigma, double deg_mean, double deg_sigma,
           double p_intra, double geo_p, double gamma, uint64_t seed, int32_t keep_kind,
           int32_t *n_out, int64_t *arcs_out, int32_t **row_ptr, int32_t **col_idx) {
  if (n < 2 || host_mean < 1 || deg_mean < 0 || geo_p <= 0 || geo_p > 1 || gamma <= 1) return -1;
  std::vector<int32_t> host_lo, host_hi;
  web_hosts(n, host_mean, host_sigma, seed, host_lo, host_hi);
  // Alias table over ranks; rank r (0-based) has weight (r+1)^(-1/(gamma-1)).
  std::vector<int32_t> rank_node;
  random_permutation(n, seed, 2, rank_node);
  std::vector<double> prob((size_t)n);
  std::vector<int32_t> alias((size_t)n);
  {
    const double ex = -1.0 / (gamma - 1.0);
    std::vector<double> w((size_t)n);
    double tot = 0;
    for (int32_t i = 0; i < n; i++) { w[i] = std::pow((double)i + 1.0, ex); tot += w[i]; }
    std::vector<int32_t> small, large;
    for (int32_t i = 0; i < n; i++) {
      w[i] = w[i] * (double)n / tot;
      (w[i] < 1.0 ? small : large).push_back(i);
    }
    while (!small.empty() && !large.empty()) {
      const int32_t s = small.back(), l = large.back();
      small.pop_back();
      prob[s] = w[s];
      alias[s] = l;
      w[l] = (w[l] + w[s]) - 1.0;
      if (w[l] < 1.0) { large.pop_back(); small.push_back(l); }
    }
    for (int32_t i : large) { prob[i] = 1.0; alias[i] = i; }
    for (int32_t i : small) { prob[i] = 1.0; alias[i] = i; }
  }
  // Out-degrees (per-node streams), provisional offsets.
  std::vector<int64_t> off((size_t)n + 1, 0);
  const double dmu = std::log(std::max(deg_mean, 1e-9)) - 0.5 * deg_sigma * deg_sigma;
#pragma omp parallel for schedule(static, 65536)
  for (int32_t v = 0; v < n; v++) {
    Rng r(seed, (1ULL << 40) + (uint64_t)v);
    int64_t d = deg_mean > 0 ? std::llround(std::exp(dmu + deg_sigma * r.normal())) : 0;
    if (d > n - 1) d = n - 1;
    off[(size_t)v + 1] = d;
  }
  for (int32_t v = 0; v < n; v++) off[(size_t)v + 1] += off[v];
  const int64_t prov = off[n];
  std::vector<int32_t> col((size_t)std::max<int64_t>(prov, 1));
  std::vector<int64_t> keep((size_t)n, 0);
  const double lq = std::log1p(-geo_p);
#pragma omp parallel for schedule(dynamic, 4096)
  for (int32_t v = 0; v < n; v++) {
    Rng r(seed, (1ULL << 40) + (uint64_t)v);
    (void)r.normal();  // the degree draw
    int32_t *b = col.data() + off[v];
    const int64_t d = off[(size_t)v + 1] - off[v];
    // Draw until d distinct non-loop targets (bounded retries), so the degree law holds
    // after duplicate removal.
    auto intra_target = [&]() -> int64_t {
      double u = r.uniform();
      while (u <= 0.0) u = r.uniform();
      const int64_t g = 1 + (int64_t)std::floor(std::log(u) / lq);  // Geometric on {1,2,...}
      const int64_t delta = (r.next() & 1) ? g : -g;
      return std::min<int64_t>(host_hi[v], std::max<int64_t>(host_lo[v], (int64_t)v + delta));
    };
    auto host_target = [&]() -> int64_t {  // uniform over v's host
      return host_lo[v] + (int64_t)r.below((uint64_t)(host_hi[v] - host_lo[v] + 1));
    };
    auto inter_target = [&]() -> int64_t {
      const uint64_t i2 = r.below((uint64_t)n);
      const int32_t rk = (r.uniform() < prob[i2]) ? (int32_t)i2 : alias[i2];
      return rank_node[rk];
    };
    int64_t k = 0;
    auto take = [&](int64_t t) -> bool {  // keeps t if it is new and not v itself
      if (t == v) return false;
      for (int64_t j = 0; j < k; j++)
        if (b[j] == (int32_t)t) return false;
      b[k++] = (int32_t)t;
      return true;
    };
    const int64_t max_draws = 8 * d + 64;
    if (!keep_kind) {
      for (int64_t draw = 0; k < d && draw < max_draws; draw++)
        take(r.uniform() < p_intra ? intra_target() : inter_target());
    } else {
      // An intra-host arc draws a nearby id up to 32 times, then any id of the host up to
      // 32 times, then becomes inter-host. Once the nearby ids of v are taken (a first
      // intra-host arc found none), later intra-host arcs start at the host-wide draws,
      // and once the host is taken, at the inter-host draws, so the draw budget still
      // covers d.
      int64_t draws = 0;
      int level_min = 0;  // 0 nearby, 1 host-wide, 2 inter-host
      while (k < d && draws < max_draws) {
        int level = r.uniform() < p_intra ? level_min : 2;
        bool kept = false;
        for (int tries = 0; !kept && draws < max_draws; tries++, draws++) {
          if (tries == 32 && level < 2) {
            level_min = std::max(level_min, ++level);
            tries = 0;
          } else if (tries == 32) {
            break;
          }
          kept = take(level == 0 ? intra_target() : level == 1 ? host_target() : inter_target());
        }
      }
    }
    std::sort(b, b + k);
    int32_t *w = b + k;
    keep[v] = w - b;
  }
  int64_t total = 0;
  for (int32_t v = 0; v < n; v++) total += keep[v];
  if (total >= (int64_t)INT32_MAX) return -2;
  int32_t *rp = (int32_t *)std::malloc(sizeof(int32_t) * ((size_t)n + 1));
  int32_t *ci = (int32_t *)std::malloc(sizeof(int32_t) * (size_t)std::max<int64_t>(total, 1));
  if (!rp || !ci) { std::free(rp); std::free(ci); return -3; }
  int64_t acc = 0;
  for (int32_t v = 0; v < n; v++) { rp[v] = (int32_t)acc; acc += keep[v]; }
  rp[n] = (int32_t)acc;
#pragma omp parallel for schedule(dynamic, 4096)
  for (int32_t v = 0; v < n; v++)
    std::memcpy(ci + rp[v], col.data() + off[v], sizeof(int32_t) * (size_t)keep[v]);
  *n_out = n;
  *arcs_out = total;
  *row_ptr = rp;
  *col_idx = ci;
  return 0;
}

void gg_free(void *p) { std::free(p); }

}  // extern "C"
