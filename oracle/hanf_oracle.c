/*
 * HyperANF CPU oracle — TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, deliberately unoptimised CPU HyperANF used to check the GPU
 * library. Only the tests, the smoke entry point and the benchmark's CPU-baseline
 * leg may load it; the product path never does. It shares no code, header, table
 * or constant generator with the GPU library.
 *
 * Every function follows Boldi, Rosa, Vigna, "HyperANF: Approximating the
 * Neighbourhood Function of Very Large Graphs on a Budget" (arXiv:1011.5599):
 *   - Section 3.1, Algorithm 1 (HyperLogLog add / size);
 *   - Section 3.2, Algorithm 2 (the HyperANF iteration, union = register max);
 *   - Section 3.3 (task decomposition; tracking modified counters);
 * and, where the paper defers to the HyperLogLog paper of Flajolet, Fusy,
 * Gandouet and Meunier (alpha_m, small-range correction), on that paper's
 * published algorithm. Readings of silent or ambiguous passages:
 *   - hash: h_s(x) is the (x+1)-th output of splitmix64 started from state s;
 *   - "leftmost" bits are the most significant bits of the 64-bit hash;
 *   - registers start at 0 (the paper's minus infinity; rho+ >= 1 so max is unaffected)
 *     and saturate at 31 (5-bit registers, ceil(log log n) for n <= 2^32);
 *   - size(): raw = alpha_m m^2 / sum_j 2^-M[j]; if raw <= 5m/2 and some register is 0,
 *     the linear-counting value m ln(m/V) is returned instead (V = zero registers);
 *   - the new counter of v includes v's own counter (Algorithm 2 starts m <- c[v]);
 *   - passes are synchronous (Jacobi): every read in a pass sees the old counters.
 */
#include <math.h>
#include <pthread.h>
#include <stdatomic.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* ---------------------------------------------------------------- hash (Section 3.1) */

/* h_seed(x): the (x+1)-th output of the splitmix64 generator whose state starts at
 * `seed` (Steele, Lea, Flood 2014). The generator adds the golden-ratio increment to its
 * state before each output and then mixes the state. */
uint64_t orc_hash(uint64_t seed, uint64_t x) {
  uint64_t state = seed + (x + 1) * 0x9E3779B97F4A7C15ULL;
  uint64_t z = state;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}

/* h_b(x): the integer value of the leftmost b bits of the hash (Section 3.1). */
int orc_register_index(uint64_t h, int b) { return (int)(h >> (64 - b)); }

/* rho+(h^b(x)): number of leading zeroes of the 64-b bits that follow the leftmost b
 * bits, plus one (Section 3.1; e.g. rho+(00101) = 3). If all of them are zero the
 * sequence has 64-b leading zeroes. */
int orc_rho_plus(uint64_t h, int b) {
  int zeros = 0;
  for (int bit = 63 - b; bit >= 0; bit--) {
    if ((h >> bit) & 1ULL) break;
    zeros++;
  }
  return zeros + 1;
}

/* ---------------------------------------------------------------- Algorithm 1 */

#define ORC_REGISTER_MAX 31 /* 5-bit registers */

/* add(M, x) given the hash h = h(x): i <- h_b(x); M[i] <- max(M[i], rho+(h^b(x))). */
void orc_add_hashed(uint8_t *M, int b, uint64_t h) {
  int i = orc_register_index(h, b);
  int r = orc_rho_plus(h, b);
  if (r > ORC_REGISTER_MAX) r = ORC_REGISTER_MAX;
  if (r > M[i]) M[i] = (uint8_t)r;
}

/* add(M, x) of Algorithm 1. */
void orc_add(uint8_t *M, int b, uint64_t seed, uint64_t x) { orc_add_hashed(M, b, orc_hash(seed, x)); }

/* alpha_m, the bias constant of the HyperLogLog estimator (values published with the
 * HyperLogLog algorithm; the paper defers to it). */
double orc_alpha(int m) {
  if (m == 16) return 0.673;
  if (m == 32) return 0.697;
  if (m == 64) return 0.709;
  return 0.7213 / (1.0 + 1.079 / m);
}

/* size(M): E = alpha_m m^2 (sum_j 2^-M[j])^-1, computed with the single division
 * (alpha_m m^2) / sum; with the small-range (linear counting) rule of the HyperLogLog
 * algorithm. The sum of powers of two is exact in double precision. */
double orc_size(const uint8_t *M, int b) {
  int m = 1 << b;
  double sum = 0.0;
  int zeros = 0;
  for (int j = 0; j < m; j++) {
    sum += ldexp(1.0, -(int)M[j]);
    if (M[j] == 0) zeros++;
  }
  double E = orc_alpha(m) * m * m / sum;
  if (E <= 2.5 * m && zeros > 0) E = m * log((double)m / zeros);
  return E;
}

/* ---------------------------------------------------------------- Algorithm 2 */

/* union(M, N): M[i] <- max(M[i], N[i]) for every i < m. */
void orc_union(uint8_t *M, const uint8_t *N, int m) {
  for (int i = 0; i < m; i++)
    if (N[i] > M[i]) M[i] = N[i];
}

/* Initialisation: every counter empty, then add v to c[v]. Counters are node-major,
 * m bytes each. */
void orc_init(int32_t n, int b, uint64_t seed, uint8_t *c) {
  int m = 1 << b;
  memset(c, 0, (size_t)n * (size_t)m);
  for (int32_t v = 0; v < n; v++) orc_add(c + (size_t)v * m, b, seed, (uint64_t)v);
}

/* N_hat(t) = sum over v of size(c[v]), summed in node order with Neumaier's
 * compensated summation. */
/* size() of every counter of c (n counters of m bytes): out[v]. */
void orc_sizes(int32_t n, int b, const uint8_t *c, double *out) {
  int m = 1 << b;
  for (int32_t v = 0; v < n; v++) out[v] = orc_size(c + (size_t)v * m, b);
}

double orc_sum_sizes(int32_t n, int b, const uint8_t *c) {
  int m = 1 << b;
  double s = 0.0, comp = 0.0;
  for (int32_t v = 0; v < n; v++) {
    double x = orc_size(c + (size_t)v * m, b);
    double t = s + x;
    if (fabs(s) >= fabs(x))
      comp += (s - t) + x;
    else
      comp += (x - t) + s;
    s = t;
  }
  return s + comp;
}

/* orc_sum_sizes with the per-node sizes computed by nthreads threads over contiguous
 * segments, then summed in node order exactly as orc_sum_sizes does (same value). */
typedef struct {
  int32_t n, seg;
  int b;
  const uint8_t *c;
  double *out;
  atomic_int next_task;
} sizes_job;

static void *sizes_worker(void *arg) {
  sizes_job *job = (sizes_job *)arg;
  int m = 1 << job->b;
  for (;;) {
    int task = atomic_fetch_add(&job->next_task, 1);
    int64_t lo = (int64_t)task * job->seg;
    if (lo >= job->n) break;
    int64_t hi = lo + job->seg < job->n ? lo + job->seg : job->n;
    for (int64_t v = lo; v < hi; v++) job->out[v] = orc_size(job->c + (size_t)v * m, job->b);
  }
  return NULL;
}

double orc_sum_sizes_mt(int32_t n, int b, const uint8_t *c, int nthreads) {
  double *x = (double *)malloc(sizeof(double) * (n ? (size_t)n : 1));
  pthread_t *th = (pthread_t *)malloc(sizeof(pthread_t) * (size_t)(nthreads > 0 ? nthreads : 1));
  if (!x || !th || nthreads <= 1) {
    free(x);
    free(th);
    return orc_sum_sizes(n, b, c);
  }
  sizes_job job;
  job.n = n;
  job.seg = 4096;
  job.b = b;
  job.c = c;
  job.out = x;
  atomic_init(&job.next_task, 0);
  int started = 0;
  for (int i = 0; i < nthreads; i++)
    if (pthread_create(&th[i], NULL, sizes_worker, &job) == 0) started++;
    else break;
  if (started == 0) sizes_worker(&job);
  for (int i = 0; i < started; i++) pthread_join(th[i], NULL);
  double s = 0.0, comp = 0.0;
  for (int32_t v = 0; v < n; v++) {
    double t = s + x[v];
    if (fabs(s) >= fabs(x[v]))
      comp += (s - t) + x[v];
    else
      comp += (x[v] - t) + s;
    s = t;
  }
  free(x);
  free(th);
  return s + comp;
}

/* One pass of the main loop for the nodes lo..hi-1: m <- c[v]; for each v -> w,
 * m <- union(c[w], m); the new counter goes to `next` (the update file), so every
 * read sees the counters of the previous iteration. With `modified` non-NULL, the
 * maximisation with successors whose counter did not change in the previous
 * iteration is skipped (Section 3.3, tracking modified counters). */
static void pass_range(int32_t lo, int32_t hi, const int32_t *row_ptr, const int32_t *col_idx,
                       int m, const uint8_t *cur, uint8_t *next, const uint8_t *modified,
                       uint8_t *modified_out, int64_t *changed, int64_t *maxed) {
  int64_t ch = 0, mx = 0;
  for (int32_t v = lo; v < hi; v++) {
    uint8_t *acc = next + (size_t)v * m;
    memcpy(acc, cur + (size_t)v * m, (size_t)m);
    for (int32_t a = row_ptr[v]; a < row_ptr[v + 1]; a++) {
      int32_t w = col_idx[a];
      if (modified && !modified[w]) continue;
      orc_union(acc, cur + (size_t)w * m, m);
      mx++;
    }
    int differs = memcmp(acc, cur + (size_t)v * m, (size_t)m) != 0;
    if (modified_out) modified_out[v] = (uint8_t)differs;
    ch += differs;
  }
  *changed += ch;
  *maxed += mx;
}

/* Task decomposition (Section 3.3): the nodes are cut into contiguous segments, in the
 * order of the thousands, and a pool of threads repeatedly takes the first segment not
 * yet taken. */
typedef struct {
  int32_t n, seg, ntasks;
  const int32_t *row_ptr, *col_idx;
  int m;
  const uint8_t *cur;
  uint8_t *next;
  const uint8_t *modified;
  uint8_t *modified_out;
  atomic_int next_task;
  atomic_llong changed, maxed;
} pass_job;

static void *pass_worker(void *arg) {
  pass_job *job = (pass_job *)arg;
  int64_t ch = 0, mx = 0;
  for (;;) {
    int task = atomic_fetch_add(&job->next_task, 1);
    if (task >= job->ntasks) break;
    int32_t lo = task * job->seg;
    int32_t hi = lo + job->seg < job->n ? lo + job->seg : job->n;
    pass_range(lo, hi, job->row_ptr, job->col_idx, job->m, job->cur, job->next, job->modified,
               job->modified_out, &ch, &mx);
  }
  atomic_fetch_add(&job->changed, ch);
  atomic_fetch_add(&job->maxed, mx);
  return NULL;
}

/* One full pass over all nodes; returns the number of counters that changed and, in
 * *maxed_out (if non-NULL), the number of unions performed with successor counters. */
int64_t orc_pass(int32_t n, const int32_t *row_ptr, const int32_t *col_idx, int b,
                 const uint8_t *cur, uint8_t *next, const uint8_t *modified,
                 uint8_t *modified_out, int nthreads, int64_t *maxed_out) {
  int m = 1 << b;
  int64_t changed = 0, maxed = 0;
  if (nthreads <= 1) {
    pass_range(0, n, row_ptr, col_idx, m, cur, next, modified, modified_out, &changed, &maxed);
  } else {
    pass_job job;
    job.n = n;
    job.seg = n / 4096 + 1;
    if (job.seg < 64) job.seg = 64;
    job.ntasks = (int)((n + job.seg - 1) / job.seg);
    job.row_ptr = row_ptr;
    job.col_idx = col_idx;
    job.m = m;
    job.cur = cur;
    job.next = next;
    job.modified = modified;
    job.modified_out = modified_out;
    atomic_init(&job.next_task, 0);
    atomic_init(&job.changed, 0);
    atomic_init(&job.maxed, 0);
    pthread_t *th = (pthread_t *)malloc(sizeof(pthread_t) * (size_t)nthreads);
    int started = 0;
    for (int i = 0; i < nthreads; i++)
      if (pthread_create(&th[i], NULL, pass_worker, &job) == 0) started++;
      else break;
    if (started == 0) pass_worker(&job);
    for (int i = 0; i < started; i++) pthread_join(th[i], NULL);
    free(th);
    changed = atomic_load(&job.changed);
    maxed = atomic_load(&job.maxed);
  }
  if (maxed_out) *maxed_out = maxed;
  return changed;
}

/* The whole of Algorithm 2: initialise, then repeat { N_hat(t) = sum of sizes; one pass;
 * t <- t+1 } until no counter changes. nt receives N_hat(0..T) (T+1 values, T = the
 * first t whose pass leaves every counter unchanged); with nt NULL the sums are skipped.
 * Returns 0, -5 if nt_cap is too small, -6 if max_passes passes did not stabilise, -2 on
 * allocation failure. If final_regs is non-NULL it receives the stable counters (n*m
 * bytes). */
int orc_run(int32_t n, const int32_t *row_ptr, const int32_t *col_idx, int b, uint64_t seed,
            int32_t max_passes, int skip_unmodified, int nthreads, double *nt, int32_t nt_cap,
            int32_t *T_out, uint8_t *final_regs) {
  int m = 1 << b;
  size_t bytes = (size_t)n * (size_t)m;
  uint8_t *cur = (uint8_t *)malloc(bytes ? bytes : 1);
  uint8_t *next = (uint8_t *)malloc(bytes ? bytes : 1);
  uint8_t *mod = skip_unmodified ? (uint8_t *)malloc(n ? (size_t)n : 1) : NULL;
  uint8_t *mod_out = skip_unmodified ? (uint8_t *)malloc(n ? (size_t)n : 1) : NULL;
  int rc = 0;
  if (!cur || !next || (skip_unmodified && (!mod || !mod_out))) {
    rc = -2;
    goto done;
  }
  orc_init(n, b, seed, cur);
  if (mod) memset(mod, 1, (size_t)n);
  int32_t t = 0;
  for (;;) {
    if (nt) {
      if (t >= nt_cap) { rc = -5; break; }
      nt[t] = orc_sum_sizes(n, b, cur);
    }
    if (t >= max_passes) { rc = -6; break; }
    int64_t changed = orc_pass(n, row_ptr, col_idx, b, cur, next, mod, mod_out, nthreads, NULL);
    if (changed == 0) break;
    uint8_t *tmp = cur; cur = next; next = tmp;
    if (mod) { uint8_t *tm = mod; mod = mod_out; mod_out = tm; }
    t++;
  }
  *T_out = t;
  if (final_regs && rc == 0) memcpy(final_regs, cur, bytes);
done:
  free(cur);
  free(next);
  free(mod);
  free(mod_out);
  return rc;
}

/* The counter that Section 3.2 says c_t[v] is equivalent to: a counter fed with every
 * node of the ball B(v, t) (nodes reachable from v in at most t arcs), found by
 * breadth-first search. *ball_size receives |B(v,t)|. Returns 0, or -2 on allocation
 * failure. */
int orc_ball_counter(int32_t n, const int32_t *row_ptr, const int32_t *col_idx, int b,
                     uint64_t seed, int32_t v, int32_t t, uint8_t *M, int64_t *ball_size) {
  int m = 1 << b;
  int32_t *dist = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
  int32_t *queue = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
  if (!dist || !queue) { free(dist); free(queue); return -2; }
  for (int32_t i = 0; i < n; i++) dist[i] = -1;
  memset(M, 0, (size_t)m);
  int64_t head = 0, tail = 0;
  dist[v] = 0;
  queue[tail++] = v;
  while (head < tail) {
    int32_t u = queue[head++];
    orc_add(M, b, seed, (uint64_t)u);
    if (dist[u] == t) continue;
    for (int32_t a = row_ptr[u]; a < row_ptr[u + 1]; a++) {
      int32_t w = col_idx[a];
      if (dist[w] < 0) {
        dist[w] = dist[u] + 1;
        queue[tail++] = w;
      }
    }
  }
  *ball_size = tail;
  free(dist);
  free(queue);
  return 0;
}

/* ---------------------------------------------------------------- broadword (Section 3.3) */

/* L_k: the lowest bit of every k-bit block of a 64-bit word set, over the floor(64/k)
 * whole blocks (the paper's example L_8 has a typo: 20 hex digits; the intended value is
 * 0x0101010101010101). H_k = L_k << (k-1): the highest bit of every block set. */
uint64_t orc_broadword_L(int k) {
  uint64_t L = 0;
  for (int i = 0; i + k <= 64; i += k) L |= 1ULL << i;
  return L;
}

/* x <_k^u y: per k-bit block, the block's high bit is set iff x's block is smaller than
 * y's (unsigned). The formula of Section 3.3, written out. */
uint64_t orc_broadword_less(uint64_t x, uint64_t y, int k) {
  uint64_t L = orc_broadword_L(k), H = L << (k - 1);
  return ((((x | H) - (y & ~H)) | (x ^ y)) ^ (x | ~y)) & H;
}

/* Block-wise maximum of x and y: the mask m is all ones where x's block is kept and all
 * zeroes where y's block is taken; the result is x & m | y & ~m (Section 3.3). */
uint64_t orc_broadword_max(uint64_t x, uint64_t y, int k) {
  uint64_t L = orc_broadword_L(k), H = L << (k - 1);
  uint64_t c = orc_broadword_less(x, y, k);
  uint64_t mask = ((((c >> (k - 1)) | H) - L) | H) ^ c;
  return (x & mask) | (y & ~mask);
}

/* ---------------------------------------------------------------- balls of every node (Section 3.2) */

/* Section 3.2: after t passes, c_t[v] is the counter of the ball B(v, t). This checks the
 * identity for every node and every t against counters the caller computed by iteration:
 * regs holds c_0 .. c_T one after another (T+1 arrays of n*m bytes). For each v a
 * breadth-first search visits the nodes in order of distance; a counter fed with them is
 * compared with c_d[v] each time the distance d is complete, and, once the search ends,
 * with c_d[v] for every remaining d <= T (the ball no longer grows). Distances beyond T
 * are compared with c_T[v] (the counters are stable from T on). The exact distance counts
 * go to hist (hist[d] = pairs at distance d, for d < hist_len; longer distances add to the
 * last slot), so N(t) is their running sum. Returns the number of (v, d) mismatches;
 * *bad_v / *bad_t receive the first one found by the lowest thread (or -1). nthreads
 * workers take segments of 64 nodes. -2 on allocation failure. */
typedef struct {
  int32_t n, T, hist_len;
  const int32_t *row_ptr, *col_idx;
  int b;
  uint64_t seed;
  const uint8_t *regs;
  int64_t *hist;
  atomic_int next_task;
  atomic_llong mismatches;
  atomic_int bad_v, bad_t;
  pthread_mutex_t lock;
  int failed;
} balls_job;

static void *balls_worker(void *arg) {
  balls_job *job = (balls_job *)arg;
  const int m = 1 << job->b;
  const size_t layer = (size_t)job->n * (size_t)m;
  int32_t *dist = (int32_t *)malloc(sizeof(int32_t) * (size_t)job->n);
  int32_t *queue = (int32_t *)malloc(sizeof(int32_t) * (size_t)job->n);
  int64_t *hist = (int64_t *)calloc((size_t)job->hist_len, sizeof(int64_t));
  uint8_t *M = (uint8_t *)malloc((size_t)m);
  if (!dist || !queue || !hist || !M) {
    pthread_mutex_lock(&job->lock);
    job->failed = 1;
    pthread_mutex_unlock(&job->lock);
    free(dist); free(queue); free(hist); free(M);
    return NULL;
  }
  for (int32_t i = 0; i < job->n; i++) dist[i] = -1;
  int64_t bad = 0;
  for (;;) {
    int task = atomic_fetch_add(&job->next_task, 1);
    int32_t lo = task * 64;
    if (lo >= job->n) break;
    int32_t hi = lo + 64 < job->n ? lo + 64 : job->n;
    for (int32_t v = lo; v < hi; v++) {
      memset(M, 0, (size_t)m);
      int64_t head = 0, tail = 0;
      int32_t level = 0;
      dist[v] = 0;
      queue[tail++] = v;
      while (head < tail) {
        int32_t u = queue[head];
        if (dist[u] != level) {  /* B(v, level) is complete */
          int32_t t = level < job->T ? level : job->T;
          if (memcmp(M, job->regs + (size_t)t * layer + (size_t)v * m, (size_t)m) != 0) {
            bad++;
            int expect = -1;
            if (atomic_compare_exchange_strong(&job->bad_v, &expect, v)) atomic_store(&job->bad_t, level);
          }
          level = dist[u];
        }
        head++;
        orc_add(M, job->b, job->seed, (uint64_t)u);
        hist[dist[u] < job->hist_len ? dist[u] : job->hist_len - 1]++;
        for (int32_t a = job->row_ptr[u]; a < job->row_ptr[u + 1]; a++) {
          int32_t w = job->col_idx[a];
          if (dist[w] < 0) {
            dist[w] = dist[u] + 1;
            queue[tail++] = w;
          }
        }
      }
      /* the ball stops growing at the last level: every later c_t[v] equals its counter */
      for (int32_t d = level; d <= job->T || d == level; d++) {
        int32_t t = d < job->T ? d : job->T;
        if (memcmp(M, job->regs + (size_t)t * layer + (size_t)v * m, (size_t)m) != 0) {
          bad++;
          int expect = -1;
          if (atomic_compare_exchange_strong(&job->bad_v, &expect, v)) atomic_store(&job->bad_t, d);
        }
        if (d >= job->T) break;
      }
      for (int64_t i = 0; i < tail; i++) dist[queue[i]] = -1;
    }
  }
  pthread_mutex_lock(&job->lock);
  for (int32_t d = 0; d < job->hist_len; d++) job->hist[d] += hist[d];
  pthread_mutex_unlock(&job->lock);
  atomic_fetch_add(&job->mismatches, bad);
  free(dist); free(queue); free(hist); free(M);
  return NULL;
}

int64_t orc_balls_check(int32_t n, const int32_t *row_ptr, const int32_t *col_idx, int b, uint64_t seed,
                        const uint8_t *regs, int32_t T, int nthreads, int64_t *hist, int32_t hist_len,
                        int32_t *bad_v, int32_t *bad_t) {
  balls_job job;
  job.n = n;
  job.T = T;
  job.hist_len = hist_len;
  job.row_ptr = row_ptr;
  job.col_idx = col_idx;
  job.b = b;
  job.seed = seed;
  job.regs = regs;
  job.hist = hist;
  job.failed = 0;
  memset(hist, 0, sizeof(int64_t) * (size_t)hist_len);
  atomic_init(&job.next_task, 0);
  atomic_init(&job.mismatches, 0);
  atomic_init(&job.bad_v, -1);
  atomic_init(&job.bad_t, -1);
  pthread_mutex_init(&job.lock, NULL);
  if (nthreads < 1) nthreads = 1;
  pthread_t *th = (pthread_t *)malloc(sizeof(pthread_t) * (size_t)nthreads);
  int started = 0;
  if (th)
    for (int i = 0; i < nthreads; i++)
      if (pthread_create(&th[i], NULL, balls_worker, &job) == 0) started++;
      else break;
  if (started == 0) balls_worker(&job);
  for (int i = 0; i < started; i++) pthread_join(th[i], NULL);
  free(th);
  pthread_mutex_destroy(&job.lock);
  *bad_v = atomic_load(&job.bad_v);
  *bad_t = atomic_load(&job.bad_t);
  if (job.failed) return -2;
  return atomic_load(&job.mismatches);
}
