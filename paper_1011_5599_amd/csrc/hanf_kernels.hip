// HIP kernels for gfx950 (CDNA4): HyperANF's iteration (Boldi, Rosa, Vigna, Algorithm 2)
// over HyperLogLog counters (Algorithm 1).
//
// Data layout in HBM (S = counters per node row: 1 for a single run, up to 32 seeds of a
// batched run side by side):
//   regs[2]   uint8 [n][S][m]  counters c_t and c_{t+1}, node-major, m = 2^log2m bytes each
//             (or [n][S][5m/8] with 5-bit registers packed without gaps)
//   bits[2]   uint32 [2 * S * ceil(n/64)]  modified-counter flags (S bits per node) of the
//             previous / current pass
//   est       double [n][S]    estimate of each current counter
//   blocksum  double [ceil(n/64)][S]  cached estimate sums per 64 consecutive nodes
//
// One pass (c_t -> c_{t+1}) is the signal kernels (systolic passes only do work), one
// union launch (k_union, or k_union_list over listed work units), k_finalize when a node's
// arcs are split over several wavefronts, k_estimate_changed for packed registers, and two
// reduction launches. The union's cost is its random gathers of successor counters: row
// requests through each compute unit's memory path (address and data units, L1 misses to
// L2) rather than HBM bytes, with the byte maxima's vector ALU work close behind.
// Lanes load counters 16 bytes at a time (40 bytes, 64 registers, when packed); a node row
// (S counters) is handled by G = S*m/16 lanes (S*m/64 packed), a "slot"; a wavefront holds
// W = 64/G slots. The max of a whole row serves its S counters at once (one successor id
// read, one row gather); changes, flags and estimates are kept per counter.
//   - light nodes (few arcs): one slot per node, nodes of a tile sorted by degree so the
//     slots of a wavefront finish together; tiles are assigned to XCDs in contiguous runs
//     so neighbouring ids (and their shared successors) meet in the same L2;
//   - other nodes: one wavefront per chunk of arcs, its W slots striding over the chunk;
//     nodes with several chunks leave per-chunk partial maxima combined by k_finalize.
#include <hip/hip_ext.h>

#include "hanf_internal.h"

namespace hanf {
namespace {

// ------------------------------------------------------------------ packed register max

// Register-wise max of four registers packed in a 32-bit word. Registers hold values <= 31
// (at most 127 is required), so the top bit of every byte is free: (x | 0x80808080) - y
// never borrows across bytes and leaves each byte's top bit set exactly where x_b >= y_b.
// That bit becomes a 0x7f byte mask selecting x, and bit-field insert takes y elsewhere.
// (The same idea as the paper's broadword maximisation, specialised to 8-bit blocks with a
// spare high bit.)
__device__ __forceinline__ uint32_t bytemax(uint32_t x, uint32_t y) {
  const uint32_t d = (x | 0x80808080u) - y;
  const uint32_t hi = d & 0x80808080u;
  const uint32_t keep_x = hi - (hi >> 7);
  return (x & keep_x) | (y & ~keep_x);
}

__device__ __forceinline__ uint4 bytemax4(uint4 a, uint4 b) {
  return make_uint4(bytemax(a.x, b.x), bytemax(a.y, b.y), bytemax(a.z, b.z), bytemax(a.w, b.w));
}

__device__ __forceinline__ uint4 zero4() { return make_uint4(0u, 0u, 0u, 0u); }

// Maxima of the two 16-bit halves of a and b (one v_pk_max_u16).
typedef unsigned short u16x2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ uint32_t max_u16x2(uint32_t a, uint32_t b) {
  return __builtin_bit_cast(uint32_t, __builtin_elementwise_max(__builtin_bit_cast(u16x2, a),
                                                                __builtin_bit_cast(u16x2, b)));
}

// Modified flags: S = 2^sl bits per node (sl <= 5, at most 32 counters per row), so a
// node's bits never cross a 32-bit word: word v >> (5 - sl), from bit (v << sl) mod 32.
// Loops load the words of all their nodes first (v clamped to a valid id where there is
// none), so the loads are in flight together instead of one round trip after another.
__device__ __forceinline__ uint32_t mod_word(const uint32_t *bits, int32_t v, int sl) {
  return bits[(uint32_t)v >> (5 - sl)];
}
__device__ __forceinline__ bool mod_in_word(uint32_t word, int32_t v, int sl) {
  const uint32_t field = sl == 5 ? 0xffffffffu : ((1u << (1u << sl)) - 1u);
  return ((word >> (((uint32_t)v << sl) & 31u)) & field) != 0u;
}
// Was any counter of node v's row modified?
__device__ __forceinline__ bool node_mod(const uint32_t *bits, int32_t v, int sl) {
  return mod_in_word(mod_word(bits, v, sl), v, sl);
}

__device__ __forceinline__ uint4 shfl_xor4(uint4 a, int off) {
  return make_uint4(__shfl_xor(a.x, off), __shfl_xor(a.y, off), __shfl_xor(a.z, off),
                    __shfl_xor(a.w, off));
}

// ------------------------------------------------------------------ register formats
//
// The kernels below are written once for a register format F: F::Lane is the part of a
// counter one lane holds (F::kRegs registers in F::kBytes bytes), a row of G lanes is
// G * F::kBytes bytes, and F supplies the load, store, register-wise max, comparison,
// cross-lane shuffle, the terms of the size estimate, and a lane with one register set.

// One register per byte; a lane holds 16 registers (one 16-byte load).
struct ByteRegs {
  using Lane = uint4;
  static constexpr int kRegs = 16;
  static constexpr int kBytes = 16;
  static constexpr bool kEstimateInUnion = true;  // the union kernel writes changed estimates
  static constexpr bool kStageable = true;        // light tiles may stage their rows in LDS
  static __device__ __forceinline__ Lane zero() { return zero4(); }
  static __device__ __forceinline__ Lane load(const uint8_t *regs, int64_t row, int G, int sub) {
    return *reinterpret_cast<const uint4 *>(regs + ((size_t)row * G + sub) * kBytes);
  }
  static __device__ __forceinline__ void store(uint8_t *regs, int64_t row, int G, int sub, Lane x) {
    *reinterpret_cast<uint4 *>(regs + ((size_t)row * G + sub) * kBytes) = x;
  }
  static __device__ __forceinline__ Lane max(Lane a, Lane b) { return bytemax4(a, b); }
  // The part of row `row` a lane holds, given lane_base = regs + sub * kBytes (of the lane's
  // row position) and G lanes per row.
  static __device__ __forceinline__ Lane load_at(const uint8_t *lane_base, uint32_t row, int G) {
    // (rows of G * 16 bytes, a power of two: one 64-bit shift-and-add per address)
    return *reinterpret_cast<const uint4 *>(lane_base + ((uint64_t)row << __builtin_ctz((uint32_t)(G * kBytes))));
  }
  // Accumulator of the register-wise max of many gathered counters. Two sets of 16-bit
  // maxima: `hi` over the 16-bit halves of each word as they are, `lo` over the words
  // shifted up by one byte. Of two pairs (h, l) of bytes the larger 16-bit value has the
  // larger h, so the high byte of a 16-bit maximum is the largest high byte: bytes 1 and 3
  // of the register-wise max are the high bytes of `hi`, bytes 0 and 2 those of `lo` (the low
  // bytes are not used). Three instructions per gathered 32-bit word (a shift and two
  // packed maxima) instead of the six of bytemax; the counter is put together once.
  struct Acc {
    uint4 hi, lo;
  };
  static __device__ __forceinline__ Acc acc_zero() { return Acc{zero4(), zero4()}; }
  static __device__ __forceinline__ Acc acc_from(Lane x) {
    return Acc{x, make_uint4(x.x << 8, x.y << 8, x.z << 8, x.w << 8)};
  }
  static __device__ __forceinline__ void acc_add(Acc &a, Lane x) {
    a.hi = make_uint4(max_u16x2(a.hi.x, x.x), max_u16x2(a.hi.y, x.y), max_u16x2(a.hi.z, x.z), max_u16x2(a.hi.w, x.w));
    a.lo = make_uint4(max_u16x2(a.lo.x, x.x << 8), max_u16x2(a.lo.y, x.y << 8), max_u16x2(a.lo.z, x.z << 8),
                      max_u16x2(a.lo.w, x.w << 8));
  }
  static __device__ __forceinline__ Lane acc_value(const Acc &a) {
    // bytes 3, 2, 1, 0 from hi.byte3, lo.byte3, hi.byte1, lo.byte1 (v_perm: bytes 4..7 are
    // the first operand's, 0..3 the second's)
    constexpr uint32_t sel = 0x07030501u;
    return make_uint4(__builtin_amdgcn_perm(a.hi.x, a.lo.x, sel), __builtin_amdgcn_perm(a.hi.y, a.lo.y, sel),
                      __builtin_amdgcn_perm(a.hi.z, a.lo.z, sel), __builtin_amdgcn_perm(a.hi.w, a.lo.w, sel));
  }
  static __device__ __forceinline__ bool differ(Lane a, Lane b) {
    return a.x != b.x || a.y != b.y || a.z != b.z || a.w != b.w;
  }
  static __device__ __forceinline__ Lane shfl_xor(Lane a, int off) { return shfl_xor4(a, off); }
  // sum of 2^(31 - M[j]) and number of zero registers over the lane's registers
  static __device__ __forceinline__ void size_terms(Lane a, uint64_t &S, uint32_t &V) {
    const uint32_t w[4] = {a.x, a.y, a.z, a.w};
#pragma unroll
    for (int i = 0; i < 4; ++i) {
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const uint32_t r = (w[i] >> (8 * k)) & 0xffu;
        S += (uint64_t)(1u << (31u - r));
        V += (r == 0u);
      }
    }
  }
  // register `j` (0..15) of the lane set to r, the others 0
  static __device__ __forceinline__ Lane single(uint32_t j, uint32_t r) {
    uint32_t w[4] = {0u, 0u, 0u, 0u};
#pragma unroll
    for (int i = 0; i < 4; ++i)
      if ((j >> 2) == (uint32_t)i) w[i] = r << (8 * (j & 3u));
    return make_uint4(w[0], w[1], w[2], w[3]);
  }
};

// Word `word` (64 bits) of the bit string with ones at positions 5i + bit.
constexpr uint64_t field_bits5(int word, int bit) {
  uint64_t x = 0;
  for (int b = 0; b < 64; ++b)
    if ((64 * word + b) % 5 == bit) x |= 1ull << b;
  return x;
}

// 5-bit registers packed without gaps (Section 3.3): register j of a counter is bits
// 5j .. 5j+4 of its little-endian bit string, so a counter of m registers is 5m/8 bytes and
// fields straddle the machine words. A lane holds 64 registers: 320 bits, which start on a
// 64-bit word boundary (the paper's "at least w registers per counter", w = 64). The lane
// keeps them as ten 32-bit words, the width of the GPU's carry chain.
struct Packed5Regs {
  struct Lane {
    uint32_t w[10];
  };
  static constexpr int kRegs = 64;
  static constexpr int kBytes = 40;
  static constexpr bool kStageable = false;
  // Estimates of changed counters come from k_estimate_changed after the union step: the
  // 64 field extractions would otherwise raise the union kernel's register count (and
  // lower its occupancy) for a step that runs once per changed node.
  static constexpr bool kEstimateInUnion = false;
  // the lowest (L) and the highest (H) bit of every 5-bit field, 64-bit word k of five
  static __host__ __device__ __forceinline__ constexpr uint64_t L64(int k) {
    return k == 0 ? 0x1084210842108421ull : k == 1 ? 0x2108421084210842ull : k == 2 ? 0x4210842108421084ull
         : k == 3 ? 0x8421084210842108ull : 0x0842108421084210ull;
  }
  static __host__ __device__ __forceinline__ constexpr uint64_t H64(int k) {
    return k == 0 ? 0x0842108421084210ull : k == 1 ? 0x1084210842108421ull : k == 2 ? 0x2108421084210842ull
         : k == 3 ? 0x4210842108421084ull : 0x8421084210842108ull;
  }
  // the same, 32-bit word i of ten
  static __host__ __device__ __forceinline__ constexpr uint32_t L(int i) {
    return (uint32_t)(L64(i >> 1) >> (32 * (i & 1)));
  }
  static __host__ __device__ __forceinline__ constexpr uint32_t H(int i) {
    return (uint32_t)(H64(i >> 1) >> (32 * (i & 1)));
  }
  static __device__ __forceinline__ Lane zero() {
    Lane z;
#pragma unroll
    for (int i = 0; i < 10; ++i) z.w[i] = 0u;
    return z;
  }
  static __device__ __forceinline__ Lane load(const uint8_t *regs, int64_t row, int G, int sub) {
    const uint2 *p = reinterpret_cast<const uint2 *>(regs + ((size_t)row * G + sub) * kBytes);
    Lane x;
#pragma unroll
    for (int k = 0; k < 5; ++k) {
      const uint2 t = p[k];
      x.w[2 * k] = t.x;
      x.w[2 * k + 1] = t.y;
    }
    return x;
  }
  static __device__ __forceinline__ void store(uint8_t *regs, int64_t row, int G, int sub, Lane x) {
    uint2 *p = reinterpret_cast<uint2 *>(regs + ((size_t)row * G + sub) * kBytes);
#pragma unroll
    for (int k = 0; k < 5; ++k) p[k] = make_uint2(x.w[2 * k], x.w[2 * k + 1]);
  }
  // Broadword register-wise max of Section 3.3 on k = 5-bit fields. The comparison
  //   lt = (((x | H) - (y & ~H)) | (x ^ y)) ^ (x | ~y)) & H
  // sets the high bit of every field where x < y. Per field the subtraction is
  // 2^4 + x_low - y_low >= 1, so it never borrows out of a field; a field that straddles two
  // words borrows from its low part into its high part, which is the multi-word borrow
  // (one subtract-with-borrow chain over the ten words). The selection mask moves each
  // result bit to its field's low bit (a multi-word shift right by 4), ors in H and
  // subtracts L (1 per field, again only borrowing inside a field): a field becomes 1 0000
  // where x < y and 0 1111 elsewhere; or-ing H and xor-ing lt turn those into all zeros and
  // all ones. The result takes x where the mask is set and y elsewhere.
  static __device__ __forceinline__ Lane max(Lane x, Lane y) {
    uint32_t lt[10];
    unsigned int borrow = 0u;
#pragma unroll
    for (int i = 0; i < 10; ++i) {
      unsigned int bo;
      const uint32_t d = __builtin_subc(x.w[i] | H(i), y.w[i] & ~H(i), borrow, &bo);
      borrow = bo;
      lt[i] = ((d | (x.w[i] ^ y.w[i])) ^ (x.w[i] | ~y.w[i])) & H(i);
    }
    Lane out;
    borrow = 0u;
#pragma unroll
    for (int i = 0; i < 10; ++i) {
      const uint32_t sh = (lt[i] >> 4) | (i < 9 ? lt[i + 1 < 10 ? i + 1 : 9] << 28 : 0u);
      unsigned int bo;
      const uint32_t d = __builtin_subc(sh | H(i), L(i), borrow, &bo);
      borrow = bo;
      const uint32_t mask = (d | H(i)) ^ lt[i];
      out.w[i] = (x.w[i] & mask) | (y.w[i] & ~mask);
    }
    return out;
  }
  static __device__ __forceinline__ Lane load_at(const uint8_t *lane_base, uint32_t row, int G) {
    const uint2 *p = reinterpret_cast<const uint2 *>(lane_base + (uint64_t)row * (uint32_t)(G * kBytes));
    Lane x;
#pragma unroll
    for (int k = 0; k < 5; ++k) {
      const uint2 t = p[k];
      x.w[2 * k] = t.x;
      x.w[2 * k + 1] = t.y;
    }
    return x;
  }
  // the gather accumulator is the lane itself (broadword max per counter gathered)
  using Acc = Lane;
  static __device__ __forceinline__ Acc acc_zero() { return zero(); }
  static __device__ __forceinline__ Acc acc_from(Lane x) { return x; }
  static __device__ __forceinline__ void acc_add(Acc &a, Lane x) { a = max(a, x); }
  static __device__ __forceinline__ Lane acc_value(const Acc &a) { return a; }
  static __device__ __forceinline__ bool differ(Lane a, Lane b) {
    uint32_t d = 0u;
#pragma unroll
    for (int i = 0; i < 10; ++i) d |= a.w[i] ^ b.w[i];
    return d != 0u;
  }
  static __device__ __forceinline__ Lane shfl_xor(Lane a, int off) {
    Lane r;
#pragma unroll
    for (int i = 0; i < 10; ++i) r.w[i] = __shfl_xor(a.w[i], off);
    return r;
  }
  // register j (0..63) of the lane
  static __device__ __forceinline__ uint32_t field(const Lane &a, int j) {
    const int p = 5 * j, i = p >> 5, o = p & 31;
    uint32_t f = a.w[i] >> o;
    if (o > 27) f |= a.w[i + 1 < 10 ? i + 1 : 9] << (32 - o);
    return f & 31u;
  }
  static __device__ __forceinline__ void size_terms(Lane a, uint64_t &S, uint32_t &V) {
#pragma unroll
    for (int j = 0; j < 64; ++j) {
      const uint32_t t = 0x80000000u >> field(a, j);  // 2^(31 - M[j])
      S += (uint64_t)t;
      V += t >> 31;  // M[j] == 0
    }
  }
  static __device__ __forceinline__ Lane single(uint32_t j, uint32_t r) {
    const uint32_t p = 5u * j, k = p >> 5, o = p & 31u;
    Lane x;
#pragma unroll
    for (int i = 0; i < 10; ++i) {
      uint32_t w = 0u;
      if ((uint32_t)i == k) w = r << o;
      if ((uint32_t)i == k + 1u && o > 27u) w = r >> (32u - o);
      x.w[i] = w;
    }
    return x;
  }
};
static_assert(Packed5Regs::kBytes == kPacked5LaneBytes, "packed lane size");
static_assert(Packed5Regs::L64(0) == field_bits5(0, 0) && Packed5Regs::L64(1) == field_bits5(1, 0) &&
                  Packed5Regs::L64(2) == field_bits5(2, 0) && Packed5Regs::L64(3) == field_bits5(3, 0) &&
                  Packed5Regs::L64(4) == field_bits5(4, 0),
              "low field bits");
static_assert(Packed5Regs::H64(0) == field_bits5(0, 4) && Packed5Regs::H64(1) == field_bits5(1, 4) &&
                  Packed5Regs::H64(2) == field_bits5(2, 4) && Packed5Regs::H64(3) == field_bits5(3, 4) &&
                  Packed5Regs::H64(4) == field_bits5(4, 4),
              "high field bits");

// ------------------------------------------------------------------ hash (Algorithm 1 add)

// Output number k (k >= 1) of the splitmix64 generator whose state starts at `seed`: the
// state advances by the golden-ratio increment before each output, then is mixed.
__device__ __forceinline__ uint64_t splitmix64_output(uint64_t seed, uint64_t k) {
  uint64_t z = seed + k * 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

// ------------------------------------------------------------------ estimator (Algorithm 1 size)

// size() of the counter held by an aligned group of gs lanes (F::kRegs registers per lane),
// with the HyperLogLog small-range rule. S = sum_j 2^(31 - M[j]) is an exact integer
// (<= 2^39), so raw = alpha m^2 / sum_j 2^-M[j] = K / S with K = alpha m^2 2^31 takes one
// IEEE division. All lanes of the group must be active; every lane returns the estimate.
template <class F>
__device__ __forceinline__ double slot_estimate(typename F::Lane acc, const double *lc, double K, int gs) {
  uint64_t S = 0;
  uint32_t V = 0;
  F::size_terms(acc, S, V);
  for (int off = 1; off < gs; off <<= 1) {
    const uint32_t lo = __shfl_xor((uint32_t)S, off);
    const uint32_t hi = __shfl_xor((uint32_t)(S >> 32), off);
    S += ((uint64_t)hi << 32) | lo;
    V += __shfl_xor(V, off);
  }
  const double m = (double)F::kRegs * gs;
  const double raw = K / (double)S;
  return (raw <= 2.5 * m && V > 0u) ? lc[V] : raw;
}

// ------------------------------------------------------------------ pass helpers

struct Flags {
  const uint8_t *cur;
  uint8_t *nxt;
  const uint32_t *prev_bits;  // counters modified by the previous pass
  uint32_t *cur_bits;         // counters modified by this pass
  bool gather_all;            // maximise with every successor (first pass, or frontier off)
  bool copy_check;            // next[v] may hold c_{t-1}[v] != c_t[v]: copy when v was modified
  bool systolic;              // only nodes in `todo` (signalled by a modified successor) may change
  bool use_sum;               // few groups were modified: test a group's summary byte first
  const uint8_t *todo;
  int sl;                     // log2 of the counters per node row
};

__device__ __forceinline__ Flags make_flags(const PassArgs &a, const DevState *st) {
  const int32_t t = st->t, first = st->first_pass;
  Flags f;
  const bool odd = t & 1;
  f.cur = odd ? a.regs1 : a.regs0;
  f.nxt = odd ? a.regs0 : a.regs1;
  f.prev_bits = odd ? a.bits1 : a.bits0;
  f.cur_bits = odd ? a.bits0 : a.bits1;
  f.gather_all = first || !st->frontier || st->dense_next;
  f.copy_check = !first;
  f.systolic = !f.gather_all && st->systolic;
  f.use_sum = !f.gather_all && !f.systolic && st->use_sum;
  f.todo = a.todo;
  f.sl = a.seed_log2;
  return f;
}

// The flag words of U successor ids (0 where a successor's counter cannot have changed).
// When few groups of 2^kSumShift nodes hold a counter the previous pass modified, each
// successor's group byte is read first (the summary is n / 1024 bytes, so it stays in the
// L1 cache) and only the words of marked groups are loaded: in the last passes of a run
// nearly every flag-word load, an L1 miss each, is skipped.
template <int U>
__device__ __forceinline__ void load_flag_words(const PassArgs &a, const Flags &f, const int32_t (&w)[U],
                                                uint32_t (&fw)[U]) {
  if (f.use_sum) {  // (the summary byte goes to the word's own register: no extra registers)
#pragma unroll
    for (int k = 0; k < U; ++k) fw[k] = a.mod_sum[(uint32_t)w[k] >> kSumShift];
#pragma unroll
    for (int k = 0; k < U; ++k) fw[k] = fw[k] ? mod_word(f.prev_bits, w[k], f.sl) : 0u;
  } else {
#pragma unroll
    for (int k = 0; k < U; ++k) fw[k] = mod_word(f.prev_bits, w[k], f.sl);
  }
}

struct Counters {
  int32_t scanned = 0, gathered = 0, written = 0, read = 0, local = 0;
  int32_t near = 0;  // per lane: the lane's own gathered successor ids within near_window
};

// A lane's part of row r of a light tile staged in LDS (byte registers, rows of G lanes).
__device__ __forceinline__ uint4 stage_row(const uint8_t *stage, int32_t r, int G, int sub) {
  return *reinterpret_cast<const uint4 *>(stage + ((size_t)r * G + sub) * 16);
}

// Writes c_{t+1}[v] for the node of a slot, given `acc`, the max over the successors
// maximised in (and over c_t[v] when own_loaded). Called with all 64 lanes active; idle
// slots pass v < 0. Keeps the two register buffers consistent without copying unchanged
// rows: next[v] already equals c_t[v] unless v was modified by the previous pass. Changes
// and estimates are per counter: counter j of the row is lanes j*gs .. j*gs+gs-1.
template <class F, int G>
__device__ __forceinline__ void finalize_slot(const PassArgs &a, const Flags &f, int32_t v, int lane,
                                              typename F::Lane acc, bool any, bool own_loaded,
                                              typename F::Lane own, Counters &cnt) {
  const int sub = lane % G;
  const bool pv = (v >= 0 && f.copy_check) ? node_mod(f.prev_bits, v, f.sl) : false;
  const bool work = v >= 0 && (any || pv);
  if (work && !own_loaded) own = F::load(f.cur, v, G, sub);
  if (work) {
    acc = F::max(acc, own);
    if (sub == 0) cnt.read++;
  }
  const bool diff = work && F::differ(acc, own);
  const uint64_t bal = __ballot(diff);
  const int first_lane = lane & ~(G - 1);
  const uint64_t gmask = (G == 64) ? ~0ull : ((1ull << G) - 1ull);
  const uint64_t rowbits = (bal >> first_lane) & gmask;  // lanes of this row that changed
  const bool changed = rowbits != 0ull;
  if (work && (changed || pv)) {
    F::store(f.nxt, v, G, sub, acc);
    if (sub == 0) cnt.written++;
  }
  if (changed) {  // uniform over the row's lanes
    const int gs = a.gs;
    const uint64_t smask = (gs == 64) ? ~0ull : ((1ull << gs) - 1ull);
    if constexpr (F::kEstimateInUnion) {
      const double E = slot_estimate<F>(acc, a.lc, a.K, gs);
      const int j = sub / gs;  // counter of this lane
      if (sub % gs == 0 && ((rowbits >> (j * gs)) & smask)) a.est[((size_t)v << f.sl) + j] = E;
    }
    if (sub == 0) {
      uint32_t mask = 0u;
      for (int k = 0; k < (G / gs); ++k)
        if ((rowbits >> (k * gs)) & smask) mask |= 1u << k;
      atomicOr(&f.cur_bits[(uint32_t)v >> (5 - f.sl)], mask << (((uint32_t)v << f.sl) & 31u));
    }
  }
}

// One round of a light tile: each slot handles one node v (-1: none), whose arcs are
// [beg, end). Per step the slot's G lanes load G*U consecutive successor ids (lane `sub`
// takes ids p + k*G + sub), keep those to maximise in (all of them, or those modified by
// the previous pass), compact the kept ids into the slot's queue in LDS and gather the
// queued counters U at a time.
template <class F, int G, int U, bool ST>
__device__ __forceinline__ void light_round(const PassArgs &a, const Flags &f, int32_t v, int32_t beg, int32_t end,
                                            int lane, int32_t *queue, Counters &cnt, bool count_scan,
                                            const uint8_t *stage, bool staged, int32_t lo) {
  using Lane = typename F::Lane;
  const int sub = lane % G;
  const int first = lane & ~(G - 1);
  const uint64_t smask = ((G == 64) ? ~0ull : ((1ull << G) - 1ull)) << first;
  const uint64_t below = (1ull << lane) - 1ull;
  int32_t *q = queue + first * U;  // G*U entries per slot
  // every node handed to a light round produces a new counter (all nodes in a pass over
  // all successors; otherwise nodes with a modified successor or a stale update row), so
  // its own counter is loaded up front, in parallel with the scan
  Lane own = F::zero();
  typename F::Acc acc = F::acc_zero();
  bool own_loaded = false;
  if (end > beg) {
    // (two one-sided branches, not an if-else: the compiler would merge the two loads into
    // one flat load through a selected pointer)
    if (!staged) own = F::load(f.cur, v, G, sub);
    if constexpr (ST) {
      if (staged) own = stage_row(stage, v - lo, G, sub);
    }
    if (f.gather_all) acc = F::acc_from(own);
    own_loaded = true;
  }
  const uint8_t *lane_base = f.cur + sub * F::kBytes;
  int32_t gathered = 0, local = 0, near = 0;
  // successor ids: the node's arcs, or in a systolic pass its signalled successors (every
  // one of them maximised in, no flag to test)
  const int32_t *succ = f.systolic ? a.sig_list : a.col_idx;
  for (int32_t p = beg; p < end; p += G * U) {
    int32_t w[U];
    bool ok[U];
#pragma unroll
    for (int k = 0; k < U; ++k) {
      const int32_t idx = p + k * G + sub;
      ok[k] = idx < end;
      w[k] = ok[k] ? succ[idx] : 0;
    }
    if (!f.gather_all && !f.systolic) {
      uint32_t fw[U];
      load_flag_words<U>(a, f, w, fw);  // (w = 0 where !ok)
#pragma unroll
      for (int k = 0; k < U; ++k) ok[k] = ok[k] && mod_in_word(fw[k], w[k], f.sl);
    }
    int32_t total = 0;
#pragma unroll
    for (int k = 0; k < U; ++k) {
      const uint64_t bk = __ballot(ok[k]) & smask;
      if (ok[k]) q[total + __popcll(bk & below)] = w[k];
      total += __popcll(bk);
      if constexpr (ST)
        near += (ok[k] && (uint32_t)(w[k] - v + a.near_window - 1) < 2u * (uint32_t)a.near_window - 1u) ? 1 : 0;
    }
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
    // Queue entries past the slot's last are read as its last one: a counter maximised in
    // twice changes nothing, and every load is then unconditional.
    for (int32_t j = 0; j < total; j += U) {
      Lane x[U];
      if constexpr (ST) {
        if (staged) {  // successors in the tile's id range come from its rows in LDS
          int32_t w[U];
          bool in[U];
#pragma unroll
          for (int i = 0; i < U; ++i) {
            w[i] = j + i < total ? q[j + i] : lo - 1;
            in[i] = (uint32_t)(w[i] - lo) < (uint32_t)a.tile_nodes;
            x[i] = F::zero();
          }
#pragma unroll
          for (int i = 0; i < U; ++i)
            if (j + i < total && !in[i]) x[i] = F::load(f.cur, w[i], G, sub);
#pragma unroll
          for (int i = 0; i < U; ++i) {
            if (in[i]) {
              x[i] = stage_row(stage, w[i] - lo, G, sub);
              ++local;
            }
          }
        } else {
#pragma unroll
          for (int i = 0; i < U; ++i) x[i] = F::load_at(lane_base, (uint32_t)q[min(j + i, total - 1)], G);
        }
      } else {
#pragma unroll
        for (int i = 0; i < U; ++i) x[i] = F::load_at(lane_base, (uint32_t)q[min(j + i, total - 1)], G);
      }
#pragma unroll
      for (int i = 0; i < U; ++i) F::acc_add(acc, x[i]);
    }
    gathered += total;
    if (count_scan && sub == 0) cnt.scanned += min(G * U, end - p);
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
  }
  if (sub == 0) {
    cnt.gathered += gathered;
    cnt.local += local;
  }
  if constexpr (ST) cnt.near += near;
  finalize_slot<F, G>(a, f, v, lane, F::acc_value(acc), gathered > 0, own_loaded, own, cnt);
}

// Max across the W slots of a wavefront (all lanes active).
template <class F, int G>
__device__ __forceinline__ void combine_slots(typename F::Lane &acc, bool &any) {
  int anyi = any ? 1 : 0;
#pragma unroll
  for (int off = G; off < kWave; off <<= 1) {
    acc = F::max(acc, F::shfl_xor(acc, off));
    anyi |= __shfl_xor(anyi, off);
  }
  any = anyi != 0;
}

// First phase of a frontier pass over a light tile: find the nodes that must produce a new
// counter (a successor modified by the previous pass, or their own counter modified by it,
// which leaves their update-buffer row stale). The tile covers consecutive ids, so the arcs
// of each 64-node sub-round form one contiguous CSR range: the wavefront streams it 64 ids
// per load (skipping the arcs of nodes with more than light_max arcs, which chunks handle),
// tests each successor's modified flag, and only a lane that hits one looks up its source
// node (binary search over the sub-round's 65 row pointers in LDS). The active nodes are
// then compacted into `act` in the tile's degree order. Returns their number
// (wavefront-uniform). `rps` holds 65 ints of LDS per wavefront. In a systolic pass the
// nodes with a modified successor are already marked in `todo`, and no arc is read here.
template <int U>
__device__ __forceinline__ int32_t find_active(const PassArgs &a, const Flags &f, const int32_t *tl, int32_t tile,
                                               int32_t light_max, int lane, int32_t *rps, int32_t *act,
                                               Counters &cnt) {
  const uint64_t below = (1ull << lane) - 1ull;
  const int32_t lo = tile * a.tile_nodes;
  const int32_t hi = min(a.n, lo + a.tile_nodes);
  uint64_t marks[kMaxTile / kWave];
#pragma unroll
  for (int k = 0; k < kMaxTile / kWave; ++k) marks[k] = 0ull;
  for (int32_t s0 = lo; s0 < hi; s0 += kWave) {
    const int32_t cnt_nodes = min(kWave, hi - s0);
    const int32_t v = s0 + lane;
    const bool valid = lane < cnt_nodes;
    const int32_t r0 = valid ? a.row_ptr[v] : 0;
    const int32_t r1 = valid ? a.row_ptr[v + 1] : 0;
    if (valid) rps[lane] = r0;
    if (lane == cnt_nodes - 1) rps[cnt_nodes] = r1;
    const int32_t deg = r1 - r0;
    const bool heavy = valid && deg > light_max;
    bool act = valid && deg > 0 && !heavy &&
               (node_mod(f.prev_bits, v, f.sl) || (f.systolic && f.todo[v] != 0));
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
    const uint64_t hmask = __ballot(heavy);
    uint64_t hit = 0ull;  // nodes (lanes) with a modified successor; the same value in every lane
    int32_t j0 = f.systolic ? cnt_nodes : 0;  // systolic: `todo` already names them
    while (j0 < cnt_nodes) {
      const uint64_t rest = hmask >> j0;
      const int32_t j1 = rest ? j0 + __ffsll((long long)rest) - 1 : cnt_nodes;  // light run [j0, j1)
      if (j1 > j0) {
        const int32_t A = rps[j0], B = rps[j1];
        if (lane == 0) cnt.scanned += B - A;
        // successor ids of the next step are loaded while the flags of this step are
        // tested, and the U flag words of a step are all requested before any is used
        int32_t wn[U];
#pragma unroll
        for (int k = 0; k < U; ++k) {
          const int32_t p = A + k * kWave + lane;
          wn[k] = p < B ? a.col_idx[p] : 0;
        }
        for (int32_t base = A; base < B; base += kWave * U) {
          int32_t w[U];
          bool ok[U];
#pragma unroll
          for (int k = 0; k < U; ++k) {
            ok[k] = base + k * kWave + lane < B;
            w[k] = wn[k];
          }
          const int32_t nb = base + kWave * U;
          if (nb < B) {
#pragma unroll
            for (int k = 0; k < U; ++k) {
              const int32_t p = nb + k * kWave + lane;
              wn[k] = p < B ? a.col_idx[p] : 0;
            }
          }
          bool hk[U];
          uint32_t fw[U];
          load_flag_words<U>(a, f, w, fw);  // (w = 0 where !ok)
#pragma unroll
          for (int k = 0; k < U; ++k) hk[k] = ok[k] && mod_in_word(fw[k], w[k], f.sl);
#pragma unroll
          for (int k = 0; k < U; ++k) {
            const bool h = hk[k];
            if (__any(h)) {
              int32_t src = -1;
              if (h) {  // source node: the last j in [j0, j1) with rps[j] <= arc
                const int32_t arc = base + k * kWave + lane;
                int32_t l = j0, r = j1;
                while (r - l > 1) {
                  const int32_t mid = (l + r) >> 1;
                  if (rps[mid] <= arc) l = mid; else r = mid;
                }
                src = l;
              }
              // OR the source lanes into `hit`, one distinct source per step
              uint64_t pending = __ballot(src >= 0);
              while (pending) {
                const int leader = __ffsll((long long)pending) - 1;
                const int32_t sv = __shfl(src, leader);
                hit |= 1ull << sv;
                pending &= ~__ballot(src == sv);
              }
            }
          }
        }
      }
      j0 = j1 + 1;
    }
    act = act || (valid && ((hit >> lane) & 1ull));
    const uint64_t am = __ballot(act);
#pragma unroll
    for (int k = 0; k < kMaxTile / kWave; ++k)
      if ((s0 - lo) / kWave == k) marks[k] = am;
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
  }
  // compact the active nodes in the tile's (degree) order
  int32_t n_act = 0;
  for (int32_t i = 0; i < a.tile_nodes; i += kWave) {
    const int32_t v = i + lane < a.tile_nodes ? tl[i + lane] : -1;
    if (!__any(v >= 0)) break;  // empty entries sort last
    bool keep = false;
    if (v >= 0) {
      const int32_t lv = v - lo;
#pragma unroll
      for (int k = 0; k < kMaxTile / kWave; ++k)
        if ((lv >> 6) == k) keep = (marks[k] >> (lv & 63)) & 1ull;
    }
    const uint64_t bal = __ballot(keep);
    if (keep) act[n_act + __popcll(bal & below)] = v;
    n_act += __popcll(bal);
  }
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
  return n_act;
}

// A chunk of one node's arcs handled by a whole wavefront: every lane examines its own
// successor id (64 per load), the ids to maximise in are compacted into the wavefront's
// queue in LDS, and the W slots gather the queued counters.
template <class F, int G, int U, bool ST>
__device__ __forceinline__ void chunk_wave(const PassArgs &a, const Flags &f, int32_t c, int lane,
                                           int32_t *q, Counters &cnt) {
  using Lane = typename F::Lane;
  constexpr int W = kWave / G;
  const int slot = lane / G, sub = lane % G;
  const uint64_t below = (1ull << lane) - 1ull;
  const Chunk ch = a.chunks[c];
  // systolic pass: the chunk reads the part of its node's signalled successors that falls
  // in its arc range (none for a node no modified successor signalled, which keeps its
  // counter; the copy rule below still applies)
  const int32_t *succ = f.systolic ? a.sig_list : a.col_idx;
  const int32_t a1 = f.systolic ? max(ch.a0, min(ch.a1, a.row_ptr[ch.v] + a.sig_cnt[ch.v])) : ch.a1;
  typename F::Acc acc_s = F::acc_zero();
  const uint8_t *lane_base = f.cur + sub * F::kBytes;
  // a node in a single chunk is finalised here: its own counter is loaded up front, in
  // parallel with the scan (it is needed unless no successor was modified and its update
  // row is current, which is rare where chunks are read)
  Lane own = F::zero();
  const bool own_loaded = ch.part < 0 && slot == 0 && a1 > ch.a0;
  if (own_loaded) own = F::load(f.cur, ch.v, G, sub);
  int32_t gathered = 0, near = 0;  // (wavefront-uniform)
  for (int32_t base = ch.a0; base < a1; base += kWave * U) {
    int32_t w[U];
    bool ok[U];
#pragma unroll
    for (int k = 0; k < U; ++k) {
      const int32_t p = base + k * kWave + lane;
      ok[k] = p < a1;
      w[k] = ok[k] ? succ[p] : 0;
    }
    if (!f.gather_all && !f.systolic) {
      uint32_t fw[U];
      load_flag_words<U>(a, f, w, fw);  // (w = 0 where !ok)
#pragma unroll
      for (int k = 0; k < U; ++k) ok[k] = ok[k] && mod_in_word(fw[k], w[k], f.sl);
    }
    int32_t total = 0;
#pragma unroll
    for (int k = 0; k < U; ++k) {
      const uint64_t bk = __ballot(ok[k]);
      if (ok[k]) q[total + __popcll(bk & below)] = w[k];
      total += __popcll(bk);
      if constexpr (ST)
        near += __popcll(__ballot(ok[k] && (uint32_t)(w[k] - ch.v + a.near_window - 1) < 2u * (uint32_t)a.near_window - 1u));
    }
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
    for (int32_t j = slot; j < total; j += W * U) {  // (entries past the last read as the last)
      Lane x[U];
#pragma unroll
      for (int i = 0; i < U; ++i) x[i] = F::load_at(lane_base, (uint32_t)q[min(j + i * W, total - 1)], G);
#pragma unroll
      for (int i = 0; i < U; ++i) F::acc_add(acc_s, x[i]);
    }
    gathered += total;
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
  }
  if (lane == 0) {
    cnt.scanned += a1 - ch.a0;
    cnt.gathered += gathered;
    if constexpr (ST) cnt.near += near;
  }
  Lane acc = F::acc_value(acc_s);
  bool any = gathered > 0;  // wavefront-uniform
  if (any) combine_slots<F, G>(acc, any);
  if (ch.part < 0) {
    finalize_slot<F, G>(a, f, slot == 0 ? ch.v : -1, lane, acc, any, own_loaded, own, cnt);
  } else if (slot == 0) {
    if (any) F::store(a.partial, ch.part, G, sub, acc);  // rows of empty chunks are never read
    if (sub == 0) a.partial_any[ch.part] = any ? 1 : 0;
  }
}

// Logical index of light workgroup j when workgroups are dealt to the 8 XCDs round-robin:
// each XCD receives a contiguous run of tiles.
__device__ __forceinline__ int32_t xcd_remap(int32_t j, int32_t total) {
  const int32_t x = j % kXcds, pos = j / kXcds;
  const int32_t base = total / kXcds, extra = total % kXcds;
  return x * base + min(x, extra) + pos;
}

template <typename T>
__device__ __forceinline__ T wave_sum(T x) {
#pragma unroll
  for (int off = kWave / 2; off > 0; off >>= 1) x += __shfl_xor(x, off);
  return x;
}

// Adds the wavefront's work counters to one of kStatSlots slot rows (spread to avoid
// contention; lane k adds field k); k_reduce_top sums and clears the slots. Per wavefront
// and without a workgroup barrier, so that a wavefront that finishes its unit leaves at
// once instead of holding its slot until the workgroup's slowest wavefront is done.
__device__ __forceinline__ void add_wave_counters(const Counters &c, int64_t *slots) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int32_t s0 = wave_sum(c.scanned), s1 = wave_sum(c.gathered), s2 = wave_sum(c.written),
                s3 = wave_sum(c.read), s4 = wave_sum(c.local), s5 = wave_sum(c.near);
  static_assert(kStatFields == 6, "one lane per counter field");
  const int32_t mine = lane == 0 ? s0 : lane == 1 ? s1 : lane == 2 ? s2 : lane == 3 ? s3 : lane == 4 ? s4 : s5;
  const int64_t row = ((int64_t)blockIdx.x * (kBlockThreads / kWave) + wave) % kStatSlots;
  if (lane < kStatFields && mine != 0)
    atomicAdd(reinterpret_cast<unsigned long long *>(slots + row * kStatFields + lane), (unsigned long long)(int64_t)mine);
}

// ------------------------------------------------------------------ kernels: one pass

// One light tile handled by one wavefront: every node when the pass maximises with all
// successors, else the active nodes found by find_active, W nodes per round.
// In a pass over every successor with a.stage set, the wavefront first copies the rows of c_t
// of the tile's id range [lo, hi) into `lds` (the wavefront's share of the dynamic LDS;
// 16 bytes per lane and load, four loads in flight): the tile's own counters, and the
// successor counters of arcs that stay inside the range (most arcs of a graph whose ids
// follow its locality, such as the hosts of a web graph), are then read from LDS. In other
// passes `lds` holds the list of active nodes.
template <class F, int G, int U, bool ST>
__device__ __forceinline__ void process_tile(const PassArgs &a, const Flags &f, int32_t tile, int lane, int32_t *qw,
                                             uint8_t *lds, int32_t *rps, int32_t *ent, Counters &cnt) {
  constexpr int W = kWave / G;
  const int32_t *tl = a.light + (size_t)tile * a.tile_nodes;
  const int32_t lo = tile * a.tile_nodes;
  const int slot = lane / G;
  int32_t *act = reinterpret_cast<int32_t *>(lds);
  int32_t count = a.tile_nodes;
  bool staged = false;  // `lds` holds the tile's rows (never a null pointer: its address space stays known)
  if (!f.gather_all) {
    count = find_active<U>(a, f, tl, tile, a.light_max, lane, rps, act, cnt);
  } else if constexpr (ST) {
    if (a.stage) {
      const int32_t hi = min(a.n, lo + a.tile_nodes);
      const int32_t n16 = (int32_t)(((int64_t)(hi - lo) * G * F::kBytes) >> 4);
      const uint4 *src = reinterpret_cast<const uint4 *>(f.cur + (size_t)lo * G * F::kBytes);
      uint4 *dst = reinterpret_cast<uint4 *>(lds);
      for (int32_t b = 0; b < n16; b += 4 * kWave) {
        uint4 t[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          const int32_t i = b + k * kWave + lane;
          t[k] = i < n16 ? src[i] : zero4();
        }
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          const int32_t i = b + k * kWave + lane;
          if (i < n16) dst[i] = t[k];
        }
      }
      __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
      __builtin_amdgcn_wave_barrier();
      staged = true;
    }
  }
  // arcs read here are counted unless find_active already scanned them
  const bool count_scan = f.gather_all || f.systolic;
  // The node ids of 64 entries of the list at a time, and their arc ranges, one entry per
  // lane, are loaded together (one coalesced load each) and handed to the rounds through
  // `ent` (3 x 64 ints of LDS per wavefront): a round then waits for no device load before it
  // reads its successor ids. The list is
  // the tile's (device memory) or the active nodes (LDS), read with two one-sided loads so
  // that neither becomes a flat load through a selected pointer.
  int32_t held = -1;
  for (int32_t r = 0; r < count; r += W) {
    const int32_t c64 = r & ~(kWave - 1);
    if (c64 != held) {  // (wavefront-uniform)
      held = c64;
      const bool in = c64 + lane < count;
      int32_t hv = -1;
      if (in && f.gather_all) hv = tl[c64 + lane];
      if (in && !f.gather_all) hv = act[c64 + lane];
      const int32_t hb = hv >= 0 ? a.row_ptr[hv] : 0;
      // (a systolic pass reads the node's signalled successors, which start where its arcs do)
      const int32_t he = hv < 0 ? 0 : f.systolic ? hb + a.sig_cnt[hv] : a.row_ptr[hv + 1];
      __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
      __builtin_amdgcn_wave_barrier();
      ent[lane] = hv;
      ent[kWave + lane] = hb;
      ent[2 * kWave + lane] = he;
      __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
      __builtin_amdgcn_wave_barrier();
    }
    const int src = (r & (kWave - 1)) + slot;  // (r is a multiple of W, and W divides 64)
    const int32_t v = ent[src], beg = ent[kWave + src], end = ent[2 * kWave + src];
    if (!__any(v >= 0)) break;  // empty tile entries sort last
    light_round<F, G, U, ST>(a, f, v, beg, end, lane, qw, cnt, count_scan, lds, staged, lo);
  }
}

// A systolic pass that signals at least arcs / 128 arcs has work in most units: one
// wavefront per unit (k_union) runs it faster than the persistent kernel, which is faster
// when few units have work (rmat22sym: 0.375 against 0.41 ms for a pass that signalled
// 1.2M of 67M arcs, 0.09 against 0.04 ms for one that signalled 7K). Both kernels read the
// count the signal kernels left, so exactly one of them takes the pass.
__device__ __forceinline__ bool wide_systolic(const PassArgs &a, const DevState *st) {
  return (int64_t)(st->sys_acc & 0xffffffffull) * 128 >= a.arcs;
}

// The union step of one pass (Algorithm 2), one work unit per wavefront: workgroups below
// n_chunk_wgs take 4 chunks each, the others 4 light tiles (XCD-aware order). With
// `list_too` set, k_union_list runs the systolic passes that signal few arcs and this
// kernel leaves them at once.
template <class F, int G, int U, bool ST>
__global__ __launch_bounds__(kBlockThreads) void k_union(PassArgs a, int32_t list_too) {
  const DevState *st = a.st;
  if (st->halted) return;
  const Flags f = make_flags(a, st);
  if (list_too && f.systolic && !wide_systolic(a, st)) return;
  Counters cnt;
  __shared__ int32_t queue[kBlockThreads * U];
  __shared__ int32_t rp_buf[(kBlockThreads / kWave) * (kWave + 1)];
  __shared__ int32_t ent_buf[(kBlockThreads / kWave) * 3 * kWave];
  extern __shared__ uint4 wave_lds[];  // a.lds_wave_bytes per wavefront
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // (scalar: per-wavefront LDS bases in SGPRs)
  int32_t *qw = queue + wave * kWave * U;
  if ((int32_t)blockIdx.x < a.n_chunk_wgs) {
    const int32_t c = (int32_t)blockIdx.x * 4 + wave;
    if (c < a.n_chunks) chunk_wave<F, G, U, ST>(a, f, c, lane, qw, cnt);
  } else {
    const int32_t L = xcd_remap((int32_t)blockIdx.x - a.n_chunk_wgs, a.n_light_wgs);
    const int32_t tile = L * 4 + wave;
    if (tile < a.n_tiles)
      process_tile<F, G, U, ST>(a, f, tile, lane, qw, reinterpret_cast<uint8_t *>(wave_lds) + wave * a.lds_wave_bytes,
                                rp_buf + wave * (kWave + 1), ent_buf + wave * 3 * kWave, cnt);
  }
  add_wave_counters(cnt, a.stat_slots);
}

// The union step from a persistent grid (kListWgs workgroups): in a systolic pass over the
// work units k_sys_units listed, else over every unit (chunks, then light tiles), one unit
// per wavefront at a time. With `full_too` set, k_union runs the other passes (and the
// systolic ones that signal many arcs) and this kernel leaves at once. Its grid is far smaller than one wavefront per unit, so a pass in
// which few nodes are active costs few launches.
template <class F, int G, int U, bool ST>
__global__ __launch_bounds__(kBlockThreads) void k_union_list(PassArgs a, int32_t full_too) {
  const DevState *st = a.st;
  if (st->halted) return;
  const Flags f = make_flags(a, st);
  if (full_too && !(f.systolic && !wide_systolic(a, st))) return;
  Counters cnt;
  __shared__ int32_t queue[kBlockThreads * U];
  __shared__ int32_t rp_buf[(kBlockThreads / kWave) * (kWave + 1)];
  __shared__ int32_t ent_buf[(kBlockThreads / kWave) * 3 * kWave];
  extern __shared__ uint4 wave_lds[];  // a.lds_wave_bytes per wavefront
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // (scalar: per-wavefront LDS bases in SGPRs)
  int32_t *qw = queue + wave * kWave * U;
  const int64_t total = f.systolic ? (int64_t)st->sys_units : (int64_t)a.n_chunks + a.n_tiles;
  const int64_t stride = (int64_t)gridDim.x * (kBlockThreads / kWave);
  for (int64_t i = (int64_t)blockIdx.x * (kBlockThreads / kWave) + wave; i < total; i += stride) {
    const int32_t u = f.systolic ? a.unit_list[i] : (int32_t)i;
    if (u < a.n_chunks)
      chunk_wave<F, G, U, ST>(a, f, u, lane, qw, cnt);
    else
      process_tile<F, G, U, ST>(a, f, u - a.n_chunks, lane, qw,
                                reinterpret_cast<uint8_t *>(wave_lds) + wave * a.lds_wave_bytes,
                                rp_buf + wave * (kWave + 1), ent_buf + wave * 3 * kWave, cnt);
  }
  add_wave_counters(cnt, a.stat_slots);
}

// Combines the partial maxima of nodes split over several chunks (one wavefront per node).
template <class F, int G>
__global__ __launch_bounds__(kBlockThreads) void k_finalize(PassArgs a) {
  using Lane = typename F::Lane;
  const DevState *st = a.st;
  if (st->halted) return;
  const Flags f = make_flags(a, st);
  Counters cnt;
  constexpr int W = kWave / G;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int slot = lane / G, sub = lane % G;
  const int32_t h = (int32_t)blockIdx.x * 4 + wave;
  if (h < a.n_heavy) {
    const Heavy hv = a.heavy[h];
    Lane acc = F::zero();
    bool any = false;
    // systolic pass: the chunks of an unsignalled node gathered nothing (they may have been
    // skipped without clearing their flags)
    const int32_t count = (f.systolic && f.todo[hv.v] == 0) ? 0 : hv.count;
    for (int32_t j0 = slot; j0 < count; j0 += 4 * W) {  // 4 partial rows in flight per slot
      bool ok[4];
      Lane x[4];
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const int32_t j = j0 + k * W;
        ok[k] = j < count && a.partial_any[hv.first + j];
      }
#pragma unroll
      for (int k = 0; k < 4; ++k) x[k] = ok[k] ? F::load(a.partial, hv.first + j0 + k * W, G, sub) : F::zero();
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        acc = F::max(acc, x[k]);
        any = any || ok[k];
      }
    }
    combine_slots<F, G>(acc, any);
    finalize_slot<F, G>(a, f, slot == 0 ? hv.v : -1, lane, acc, any, false, F::zero(), cnt);
  }
  add_wave_counters(cnt, a.stat_slots);
}

// Estimates of the counters this pass changed, for formats whose union step leaves them out.
// G lanes per node row; counter j of the row is lanes j*gs .. j*gs+gs-1, which take the
// same branch (their flag bit), so the estimate's shuffles stay inside active groups.
template <class F, int G>
__device__ __forceinline__ void estimate_changed_lane(const PassArgs &a, const Flags &f, int64_t gid) {
  const int64_t v64 = gid / G;
  if (v64 >= a.n) return;  // whole nodes leave together (G | 64)
  const int32_t v = (int32_t)v64;
  const int sub = (int)(gid % G), gs = a.gs, j = sub / gs;
  const uint64_t bit = ((uint64_t)v << f.sl) + j;
  if (((f.cur_bits[bit >> 5] >> (bit & 31)) & 1u) == 0u) return;
  const double E = slot_estimate<F>(F::load(f.nxt, v, G, sub), a.lc, a.K, gs);
  if (sub % gs == 0) a.est[((size_t)v << f.sl) + j] = E;
}

// (a sweep over n * G row lanes, as k_init's)
template <class F, int G>
__global__ __launch_bounds__(kBlockThreads) void k_estimate_changed(PassArgs a, int64_t lanes) {
  const DevState *st = a.st;
  if (st->halted) return;
  const Flags f = make_flags(a, st);
  const int64_t stride = (int64_t)gridDim.x * kBlockThreads;
  for (int64_t base = (int64_t)blockIdx.x * kBlockThreads; base < lanes; base += stride)
    estimate_changed_lane<F, G>(a, f, base + threadIdx.x);
}

// Per 64-node block, one lane each: re-sum the estimates where a counter changed (else
// reuse the cached sums, Section 3.3), count changed counters, clear the flags of the
// previous pass (and the signals of a systolic pass). A workgroup covers kReduceBlocks
// consecutive blocks, a quarter per wavefront; sums are taken in a fixed order. With S
// counters per node a block has 2S flag words (kept in registers) and S sums.
template <int S>
__global__ __launch_bounds__(kBlockThreads) void k_reduce_blocks(PassArgs a, int32_t force) {
  const DevState *st = a.st;
  if (st->halted) return;
  __shared__ double s_sum[kBlockThreads / kWave];
  __shared__ int32_t s_cnt[kBlockThreads / kWave], s_mark[kBlockThreads / kWave];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int32_t t = st->t;
  const uint32_t *cb = (t & 1) ? a.bits0 : a.bits1;
  uint32_t *pb = (t & 1) ? a.bits1 : a.bits0;
  const bool sys = st->systolic != 0;  // this pass's signals are cleared with its flags
  constexpr int sl = S == 1 ? 0 : S == 2 ? 1 : S == 4 ? 2 : S == 8 ? 3 : S == 16 ? 4 : 5;
  constexpr int WB = 2 * S;  // flag words per block
  constexpr int kPerWave = kReduceBlocks / (kBlockThreads / kWave);  // blocks per wavefront
  const int64_t b0 = (int64_t)blockIdx.x * kReduceBlocks + wave * kPerWave;  // the wavefront's first block
  const int64_t b = b0 + lane;
  const bool valid = lane < kPerWave && b < a.n_blocks;
  uint32_t wv[WB];
  uint32_t any = 0u;
  int32_t bc = 0;
#pragma unroll
  for (int k = 0; k < WB; ++k) {
    wv[k] = (valid && !force) ? cb[b * WB + k] : 0u;
    any |= wv[k];
    bc += __popc(wv[k]);
  }
  const bool dirty = valid && (force || any != 0u);
  // the summary byte of the wavefront's 2^kSumShift nodes (after init or resume every
  // group counts as marked)
  static_assert(kPerWave << 6 == 1 << kSumShift, "one summary byte per reduction wavefront");
  const bool marked = __ballot(dirty) != 0ull;
  if (lane == 0 && b0 < a.n_blocks) a.mod_sum[b0 / kPerWave] = marked ? 1 : 0;
  double bs = (S == 1 && valid && !dirty) ? a.blocksum[b] : 0.0;
  // the dirty blocks of the wavefront, 4 at a time: each block's 64 S estimates are read 64
  // per step; lane l always holds row seed l mod S, so a butterfly over the offsets S..32
  // leaves seed j's block sum in lane j
  uint64_t pend = __ballot(dirty);
  while (pend) {
    int32_t jb[4];
    double e[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      jb[k] = pend ? __ffsll((long long)pend) - 1 : -1;
      if (pend) pend &= pend - 1;
      e[k] = 0.0;
    }
#pragma unroll
    for (int r = 0; r < S; ++r) {
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const int64_t ei = ((b0 + jb[k]) * kNodesPerBlock << sl) + (int64_t)r * kWave + lane;
        if (jb[k] >= 0 && (ei >> sl) < a.n) e[k] += a.est[ei];
      }
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      if (jb[k] >= 0) {  // wavefront-uniform
        double sum = e[k];
#pragma unroll
        for (int off = S; off < kWave; off <<= 1) sum += __shfl_xor(sum, off);
        if (lane < S) a.blocksum[((b0 + jb[k]) << sl) + lane] = sum;
        if (S == 1 && lane == jb[k]) bs = sum;
      }
    }
  }
  if (valid && a.batch.active) {
    // changed counters of every row seed j: its flag bits are j, j+S, ... in every word
    constexpr uint32_t pattern = S == 32 ? 1u : 0xffffffffu / ((S == 32 ? 0u : (1u << S)) - 1u);
#pragma unroll
    for (int jj = 0; jj < S; ++jj) {
      int32_t cj = 0;
#pragma unroll
      for (int k = 0; k < WB; ++k) cj += __popc(wv[k] & (pattern << jj));
      a.batch.blkcnt[(b << sl) + jj] = cj;
    }
  }
  if (valid && !force)
#pragma unroll
    for (int k = 0; k < WB; ++k) pb[b * WB + k] = 0u;
  if (valid && sys) {
    uint4 *tq = reinterpret_cast<uint4 *>(a.todo + b * kNodesPerBlock);
#pragma unroll
    for (int k = 0; k < kNodesPerBlock / 16; ++k) tq[k] = make_uint4(0u, 0u, 0u, 0u);
    uint4 *tc = reinterpret_cast<uint4 *>(a.sig_cnt + b * kNodesPerBlock);
#pragma unroll
    for (int k = 0; k < kNodesPerBlock / 4; ++k) tc[k] = make_uint4(0u, 0u, 0u, 0u);
  }
  const double ws = wave_sum(bs);  // the total estimate; meaningful for one counter per node
  const int32_t wc = wave_sum(bc);
  if (lane == 0) {
    s_sum[wave] = ws;
    s_cnt[wave] = wc;
    s_mark[wave] = marked && b0 < a.n_blocks ? 1 : 0;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    a.wgsum[blockIdx.x] = (s_sum[0] + s_sum[1]) + (s_sum[2] + s_sum[3]);
    // changed counters (below 2^36) and, from bit kMarkedShift, the marked summary bytes
    a.wgcnt[blockIdx.x] = (int64_t)s_cnt[0] + s_cnt[1] + s_cnt[2] + s_cnt[3] +
                          ((int64_t)(s_mark[0] + s_mark[1] + s_mark[2] + s_mark[3]) << kMarkedShift);
  }
}

// Batched runs, first step: the sums of every chunk of a result component (at most
// kCompChunkBlocks blocks of its layout component, its row seed's block sums and change
// counts), one workgroup per chunk, in a fixed order.
__global__ __launch_bounds__(kBlockThreads) void k_reduce_comp_chunks(PassArgs a, int32_t mode) {
  const DevState *st = a.st;
  if (st->halted) return;
  __shared__ double s_sum[kBlockThreads];
  __shared__ int64_t s_cnt[kBlockThreads];
  const int32_t k = blockIdx.x;
  const int tid = threadIdx.x;
  const int sl = a.seed_log2;
  const int32_t c = a.batch.cchunk_comp[k];
  const int32_t row = a.batch.comp_row[c];
  const int32_t L = row >> sl, jj = row & ((1 << sl) - 1);
  const int32_t end = a.batch.comp_node_off[L + 1] / kNodesPerBlock;
  const int32_t b0 = a.batch.cchunk_b0[k], b1 = min(end, b0 + kCompChunkBlocks);
  double sum = 0.0;
  int64_t cnt = 0;
  for (int32_t b = b0 + tid; b < b1; b += kBlockThreads) {
    sum += a.blocksum[((size_t)b << sl) + jj];
    if (mode == kReducePass) cnt += a.batch.blkcnt[((size_t)b << sl) + jj];
  }
  s_sum[tid] = sum;
  s_cnt[tid] = cnt;
  __syncthreads();
  for (int off = kBlockThreads / 2; off > 0; off >>= 1) {
    if (tid < off) {
      s_sum[tid] += s_sum[tid + off];
      s_cnt[tid] += s_cnt[tid + off];
    }
    __syncthreads();
  }
  if (tid == 0) {
    a.batch.cchunk_sum[k] = s_sum[0];
    a.batch.cchunk_cnt[k] = s_cnt[0];
  }
}

// Second step, one thread per result component: N_hat and the changed count from its
// chunks in order. Marks the component's fixpoint T the first time a pass leaves it
// unchanged; until then appends N_hat(t+1) to its history.
__global__ __launch_bounds__(kBlockThreads) void k_reduce_components(PassArgs a, int32_t mode) {
  const DevState *st = a.st;
  if (st->halted) return;
  const int32_t c = (int32_t)blockIdx.x * kBlockThreads + threadIdx.x;
  if (c >= a.batch.n_comp) return;
  double sum = 0.0;
  int64_t cnt = 0;
  for (int32_t k = a.batch.comp_chunk0[c]; k < a.batch.comp_chunk0[c + 1]; ++k) {
    sum += a.batch.cchunk_sum[k];
    cnt += a.batch.cchunk_cnt[k];
  }
  const int32_t t = st->t;
  double *hist = a.batch.comp_nt + (size_t)c * a.nt_cap;
  if (mode == kReduceInit) {
    a.batch.comp_T[c] = -1;
    if (t < a.nt_cap) hist[t] = sum;
  } else if (a.batch.comp_T[c] < 0) {
    if (cnt == 0)
      a.batch.comp_T[c] = t;
    else if (t + 1 < a.nt_cap)
      hist[t + 1] = sum;
  }
}

// Batched ingest: component c = g * n_seeds + s is a copy of input graph g placed at node
// comp_node_off[c] (rows past the graph's own nodes are empty padding) and arc
// comp_arc_off[c]. Arcs leaving their graph set error bit 32.
__global__ void k_expand(const int32_t *graph_off, const int32_t *rp_in, const int32_t *ci_in,
                         int32_t n_seeds, PassArgs a, const int32_t *comp_arc_off, int32_t *rp_exp,
                         int32_t *ci_exp, int64_t n_exp, int64_t e_exp, DevState *st) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  for (int64_t i = gid; i <= n_exp; i += stride) {
    if (i == n_exp) {
      rp_exp[i] = (int32_t)e_exp;
      continue;
    }
    const int32_t c = a.batch.blk_comp[i / kNodesPerBlock];
    const int32_t g = c / n_seeds;
    const int32_t local = (int32_t)(i - a.batch.comp_node_off[c]);
    const int32_t ng = graph_off[g + 1] - graph_off[g];
    const int32_t row = graph_off[g] + (local < ng ? local : ng);
    rp_exp[i] = comp_arc_off[c] + (rp_in[row] - rp_in[graph_off[g]]);
  }
  int32_t err = 0;
  for (int64_t j = gid; j < e_exp; j += stride) {
    int32_t lo = 0, hi = a.batch.n_lay;  // component with comp_arc_off[c] <= j < comp_arc_off[c+1]
    while (hi - lo > 1) {
      const int32_t mid = (lo + hi) >> 1;
      if (comp_arc_off[mid] <= j) lo = mid; else hi = mid;
    }
    const int32_t c = lo, g = c / n_seeds;
    const int32_t w = ci_in[rp_in[graph_off[g]] + (int32_t)(j - comp_arc_off[c])];
    if (w < graph_off[g] || w >= graph_off[g + 1]) {
      err |= 32;
      ci_exp[j] = a.batch.comp_node_off[c];
    } else {
      ci_exp[j] = a.batch.comp_node_off[c] + (w - graph_off[g]);
    }
  }
  if (err) atomicOr(&st->err, err);
}

// Batched ingest from graphs given separately with their own ids: graph g's row_ptr
// (n_g + 1 entries, from 0) is at rp_in[graph_off[g] + g], its col_idx (ids 0..n_g-1) at
// ci_in[arc_off[g]]. Builds the expanded CSR as k_expand does and checks every graph's CSR
// (error bits: 1 row_ptr[0] != 0, 2 decreasing, 4 row_ptr[n] != arcs, 8 id out of range).
__global__ void k_expand_local(const int32_t *graph_off, const int32_t *arc_off, const int32_t *rp_in,
                               const int32_t *ci_in, int32_t n_graphs, int32_t n_seeds, PassArgs a,
                               const int32_t *comp_arc_off, int32_t *rp_exp, int32_t *ci_exp, int64_t n_exp,
                               int64_t e_exp, DevState *st) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int32_t err = 0;
  for (int64_t i = gid; i <= n_exp; i += stride) {
    if (i == n_exp) {
      rp_exp[i] = (int32_t)e_exp;
      continue;
    }
    const int32_t c = a.batch.blk_comp[i / kNodesPerBlock];
    const int32_t g = c / n_seeds;
    const int32_t local = (int32_t)(i - a.batch.comp_node_off[c]);
    const int32_t ng = graph_off[g + 1] - graph_off[g];
    const int32_t *rp = rp_in + graph_off[g] + g;
    const int32_t row = local < ng ? local : ng;
    const int32_t r0 = rp[row];
    rp_exp[i] = comp_arc_off[c] + r0;
    if (c % n_seeds == 0 && local < ng) {  // checks, once per graph
      if (local == 0 && r0 != 0) err |= 1;
      if (rp[local + 1] < r0) err |= 2;
      if (local == ng - 1 && rp[ng] != arc_off[g + 1] - arc_off[g]) err |= 4;
    }
  }
  for (int64_t j = gid; j < e_exp; j += stride) {
    int32_t lo = 0, hi = a.batch.n_lay;
    while (hi - lo > 1) {
      const int32_t mid = (lo + hi) >> 1;
      if (comp_arc_off[mid] <= j) lo = mid; else hi = mid;
    }
    const int32_t c = lo, g = c / n_seeds;
    const int32_t w = ci_in[arc_off[g] + (int32_t)(j - comp_arc_off[c])];
    const int32_t ng = graph_off[g + 1] - graph_off[g];
    if (w < 0 || w >= ng) {
      err |= 8;
      ci_exp[j] = a.batch.comp_node_off[c];
    } else {
      ci_exp[j] = a.batch.comp_node_off[c] + w;
    }
  }
  if (err) atomicOr(&st->err, err);
}

// row_ptr at every graph boundary must equal the graph's arc offset (error bit 64).
__global__ void k_check_offsets(const int32_t *rp, const int32_t *goff, const int32_t *aoff, int32_t n_graphs,
                                DevState *st) {
  const int32_t g = blockIdx.x * blockDim.x + threadIdx.x;
  if (g <= n_graphs && rp[goff[g]] != aoff[g]) atomicOr(&st->err, 64);
}

// Totals of a pass (one workgroup, fixed summation order): N_hat(t+1), changed count and
// work counters; advances t or marks the fixpoint.
constexpr int kTopThreads = 1024;

__global__ __launch_bounds__(kTopThreads) void k_reduce_top(PassArgs a, int32_t mode) {
  DevState *st = a.st;
  if (st->halted) return;
  __shared__ double s_sum[kTopThreads];
  __shared__ int64_t s_i[8][kTopThreads];
  const int tid = threadIdx.x;
  double s = 0.0;
  int64_t c = 0, sc = 0, ga = 0, wr = 0, rd = 0, lo = 0, ne = 0;
  int64_t mk = 0;
  for (int32_t i = tid; i < a.n_reduce_wgs; i += kTopThreads) {
    s += a.wgsum[i];
    const int64_t x = a.wgcnt[i];
    c += x & ((1ll << kMarkedShift) - 1);
    mk += x >> kMarkedShift;
  }
  if (tid < kStatSlots) {
    int64_t *sl = a.stat_slots + tid * kStatFields;
    if (mode == kReducePass) {
      sc = sl[0];
      ga = sl[1];
      wr = sl[2];
      rd = sl[3];
      lo = sl[4];
      ne = sl[5];
    }
    sl[0] = sl[1] = sl[2] = sl[3] = sl[4] = sl[5] = 0;
  }
  s_sum[tid] = s;
  s_i[0][tid] = c;
  s_i[1][tid] = sc;
  s_i[2][tid] = ga;
  s_i[3][tid] = wr;
  s_i[4][tid] = rd;
  s_i[5][tid] = lo;
  s_i[6][tid] = ne;
  s_i[7][tid] = mk;
  __syncthreads();
  for (int off = kTopThreads / 2; off > 0; off >>= 1) {
    if (tid < off) {
      s_sum[tid] += s_sum[tid + off];
      for (int k = 0; k < 8; ++k) s_i[k][tid] += s_i[k][tid + off];
    }
    __syncthreads();
  }
  if (tid == 0) {
    const double total = s_sum[0];
    const int32_t t = st->t;
    // whether this pass read the flag summary (as make_flags decided), and whether the next
    // one will: when at most 1 / kSumDiv of its bytes are set
    const bool dense = st->first_pass || !st->frontier || st->dense_next;
    const int64_t used_sum = (st->use_sum && !dense && !st->systolic) ? 1 : 0;
    st->use_sum = (mode != kReduceInit && s_i[7][0] * kSumDiv <= a.n_sum) ? 1 : 0;
    if (mode == kReduceInit) {
      if (t < a.nt_cap) a.nt[t] = total;
    } else {
      const int32_t p = st->passes;
      PassLog rec;
      rec.gather_all = dense ? 1 : 0;
      rec.summary = used_sum;
      rec.changed = s_i[0][0];
      rec.scanned = s_i[1][0];
      rec.gathered = s_i[2][0];
      rec.written = s_i[3][0];
      rec.read = s_i[4][0];
      rec.local = s_i[5][0];
      rec.near = s_i[6][0];
      rec.systolic = st->systolic ? (a.trow_ptr ? 1 : 2) : 0;  // 2: marks from a forward scan
      rec.signalled = rec.systolic ? (int64_t)(st->sys_acc & 0xffffffffull) : 0;
      if (p < a.log_cap) a.log[p] = rec;
      st->passes = p + 1;
      st->changed_last = rec.changed;
      st->first_pass = 0;
      st->dense_next = (st->dense_threshold > 0 && rec.changed >= st->dense_threshold) ? 1 : 0;
      // Section 3.3, systolic computation: once fewer than n S / sys_div counters changed,
      // the next pass recomputes only the nodes their changes signal
      st->systolic = (!st->dense_next && st->frontier && st->sys_div > 0 &&
                      rec.changed * (int64_t)st->sys_div < ((int64_t)a.n << a.seed_log2)) ? 1 : 0;
      st->sys_acc = 0ull;
      st->sys_units = 0;
      if (rec.changed == 0) {
        st->done = 1;
        st->halted = 1;
      } else {
        st->t = t + 1;
        if (t + 1 < a.nt_cap) a.nt[t + 1] = total;
        if (p + 1 >= st->max_passes) {
          st->capped = 1;
          st->halted = 1;
        }
      }
    }
  }
}

// ------------------------------------------------------------------ kernels: systolic signals

// Section 3.3, systolic computation. A counter modified by pass t-1 signals its predecessors
// (its arcs in the transposed graph) that they may change in pass t; pass t then recomputes
// only signalled nodes. Three kernels run before the union step of a systolic pass:
// k_sys_list lists the modified nodes that have predecessors, each with the offset of its
// predecessor arcs in one virtual array of all of them (each workgroup reserves its list
// entries and arc offsets together with one 64-bit atomic, so offsets increase along the
// list); k_sys_mark walks that virtual array in fixed tiles of kMarkTile arcs, whatever the
// in-degrees, and marks every predecessor; k_sys_units lists the work units (chunks, light
// tiles) that hold a marked or modified node.
constexpr int kMarkTile = 1024;
static_assert(kMarkTile % kBlockThreads == 0, "whole arcs per thread in k_sys_mark");
constexpr int kListWgs = 2048;  // persistent union grid: 8 workgroups per compute unit
constexpr int kSigRounds = 4;   // items per thread in the signal compaction kernels
constexpr int kSysArcDiv = 16;  // a systolic pass that would signal more than arcs/16 arcs falls
                                // back to testing every arc's flag (cheaper at that density)

// Inclusive scan across the wavefront of a 64-bit value (two 32-bit shuffles per step).
__device__ __forceinline__ unsigned long long wave_scan_u64(unsigned long long x, int lane) {
#pragma unroll
  for (int off = 1; off < kWave; off <<= 1) {
    const uint32_t lo = __shfl_up((uint32_t)(x & 0xffffffffull), off);
    const uint32_t hi = __shfl_up((uint32_t)(x >> 32), off);
    if (lane >= off) x += ((unsigned long long)hi << 32) | lo;
  }
  return x;
}

// Each workgroup takes kSigRounds * 256 consecutive items, one per thread and round, and
// reserves room for all its results with one atomic (positions in the list follow the
// item order inside the workgroup).
__global__ __launch_bounds__(kBlockThreads) void k_sys_list(PassArgs a) {
  DevState *st = a.st;
  if (st->halted || !st->systolic) return;
  const int32_t t = st->t;
  const uint32_t *pb = (t & 1) ? a.bits1 : a.bits0;  // counters modified by pass t-1
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  constexpr int NW = kBlockThreads / kWave;
  __shared__ unsigned long long s_tot[kSigRounds * NW];
  __shared__ unsigned long long s_base;
  const int sl = a.seed_log2, S = 1 << sl;
  const uint32_t field = sl == 5 ? 0xffffffffu : ((1u << S) - 1u);  // one node's flag bits
  const int64_t nwords = 2 * ((int64_t)a.n_blocks << sl);
  const int64_t base = (int64_t)blockIdx.x * (kBlockThreads * kSigRounds);
  uint32_t word[kSigRounds];
  unsigned long long own[kSigRounds], incl[kSigRounds];
#pragma unroll
  for (int r = 0; r < kSigRounds; ++r) {
    const int64_t wi = base + r * kBlockThreads + threadIdx.x;  // one flag word per thread and round
    word[r] = wi < nwords ? pb[wi] : 0u;
    uint32_t cnt = 0, deg = 0;
    for (uint32_t x = word[r]; x;) {  // each modified node once, whatever counters of it changed
      const int64_t i = wi * 32 + __ffs(x) - 1;
      x &= ~(field << (i & 31 & ~(S - 1)));
      const int64_t v = i >> sl;
      const int32_t d = v < a.n ? a.trow_ptr[v + 1] - a.trow_ptr[v] : 0;
      if (d > 0) {
        cnt++;
        deg += (uint32_t)d;
      }
    }
    own[r] = ((unsigned long long)cnt << 32) | deg;  // arcs < 2^31: the low half never carries
    incl[r] = wave_scan_u64(own[r], lane);
    if (lane == kWave - 1) s_tot[r * NW + wave] = incl[r];
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned long long acc = 0ull;
    for (int i = 0; i < kSigRounds * NW; ++i) {
      const unsigned long long x = s_tot[i];
      s_tot[i] = acc;
      acc += x;
    }
    s_base = acc ? atomicAdd(reinterpret_cast<unsigned long long *>(&st->sys_acc), acc) : 0ull;
  }
  __syncthreads();
#pragma unroll
  for (int r = 0; r < kSigRounds; ++r) {
    const int64_t wi = base + r * kBlockThreads + threadIdx.x;
    const unsigned long long off = s_base + s_tot[r * NW + wave] + incl[r] - own[r];
    int32_t idx = (int32_t)(off >> 32);
    int32_t pos = (int32_t)(off & 0xffffffffull);
    for (uint32_t x = word[r]; x;) {
      const int64_t i = wi * 32 + __ffs(x) - 1;
      x &= ~(field << (i & 31 & ~(S - 1)));
      const int64_t v = i >> sl;
      const int32_t d = v < a.n ? a.trow_ptr[v + 1] - a.trow_ptr[v] : 0;
      if (d > 0) {
        a.sys_node[idx] = (int32_t)v;
        a.sys_pos[idx] = pos;
        idx++;
        pos += d;
      }
    }
  }
}

__global__ __launch_bounds__(kBlockThreads) void k_sys_mark(PassArgs a) {
  DevState *st = a.st;
  if (st->halted || !st->systolic) return;
  const uint64_t acc = st->sys_acc;
  const int32_t K = (int32_t)(acc >> 32);             // listed nodes
  const int64_t P = (int64_t)(acc & 0xffffffffull);   // their predecessor arcs
  if (P * kSysArcDiv > a.arcs) {  // every workgroup sees the same P and leaves
    if (blockIdx.x == 0 && threadIdx.x == 0) st->systolic = 0;
    return;
  }
  __shared__ int32_t s_pos[kMarkTile], s_base[kMarkTile], s_node[kMarkTile];
  __shared__ int32_t s_red[kBlockThreads / kWave];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int64_t t0 = (int64_t)blockIdx.x * kMarkTile; t0 < P; t0 += (int64_t)gridDim.x * kMarkTile) {
    // first list entry of the tile: the last with sys_pos <= t0, by a 256-way search
    // (offsets strictly increase along the list, and entry 0 starts at 0)
    int32_t lo = 0, hi = K;
    while (hi - lo > 1) {
      const int32_t step = (hi - lo + kBlockThreads - 1) / kBlockThreads;
      const int64_t j = (int64_t)lo + (int64_t)threadIdx.x * step;
      const bool ok = j < hi && a.sys_pos[j] <= t0;  // true on a prefix of the threads
      const int c = __popcll(__ballot(ok));
      if (lane == 0) s_red[wave] = c;
      __syncthreads();
      const int total = s_red[0] + s_red[1] + s_red[2] + s_red[3];  // >= 1: thread 0 holds lo
      __syncthreads();
      lo += (total - 1) * step;
      hi = min(hi, lo + step);
    }
    // the entries that can own arcs of this tile (at most one per arc), to LDS
    const int32_t cnt = min(kMarkTile, K - lo);
    for (int j = threadIdx.x; j < kMarkTile; j += kBlockThreads) {
      if (j < cnt) {
        const int32_t p = a.sys_pos[lo + j];
        const int32_t w = a.sys_node[lo + j];
        s_pos[j] = p;
        s_base[j] = a.trow_ptr[w] - p;
        s_node[j] = w;
      }
    }
    __syncthreads();
    // each thread's kMarkTile / kBlockThreads arcs go through every step together, so their
    // loads and atomics are in flight at the same time
    constexpr int kPer = kMarkTile / kBlockThreads;
    int32_t u[kPer], wl[kPer], r0[kPer], r1[kPer], k[kPer];
#pragma unroll
    for (int q = 0; q < kPer; ++q) {
      const int64_t i = t0 + threadIdx.x + q * kBlockThreads;
      u[q] = -1;
      wl[q] = 0;
      if (i < P) {
        int32_t l = 0, r = cnt;  // last entry with s_pos <= i
        while (r - l > 1) {
          const int32_t mid = (l + r) >> 1;
          if (s_pos[mid] <= i) l = mid; else r = mid;
        }
        u[q] = a.tcol_idx[s_base[l] + (int32_t)i];
        wl[q] = s_node[l];
      }
    }
#pragma unroll
    for (int q = 0; q < kPer; ++q) {
      if (u[q] >= 0) {
        a.todo[u[q]] = 1;  // same value from every writer: no atomic needed at byte granularity
        a.tile_todo[u[q] / a.tile_nodes] = 1;
        r0[q] = a.row_ptr[u[q]];
        r1[q] = a.row_ptr[u[q] + 1];
        // the arc (u -> w) into the modified counter w goes to u's list of signalled
        // successors: at most one entry per arc of u, so the list fits u's own arc range
        k[q] = atomicAdd(&a.sig_cnt[u[q]], 1);
      }
    }
    // An entry beyond u's arc range (possible only with a transposed graph that does not
    // match the graph) is dropped and its add taken back: the count then ends at u's
    // degree, never above, so the union step reads only entries written here. (Once the
    // count has passed the degree it never falls below it, so later adds cannot reuse a
    // slot inside the range.)
#pragma unroll
    for (int q = 0; q < kPer; ++q) {
      if (u[q] < 0) continue;
      if (k[q] < r1[q] - r0[q]) a.sig_list[r0[q] + k[q]] = wl[q];
      else atomicSub(&a.sig_cnt[u[q]], 1);
    }
    __syncthreads();
  }
}

// Systolic passes without a transposed graph (Section 3.3: only a node with a successor whose
// counter the previous pass modified can change). With no predecessor lists to follow from the
// modified counters, the successor lists are scanned forward: a node is marked (todo, and its
// light tile's flag) when some successor's modified flag is set. One wavefront per work unit
// of the union step: a chunk of a heavy node's arcs, or a light tile, whose light nodes' arcs
// form one contiguous CSR range per 64 consecutive ids (heavy nodes' arcs are skipped: their
// chunks cover them). Arc ids are streamed 64 per load, kFwdLoads loads in flight per lane, and
// the flag words of all of them are loaded before any is tested; a lane that hits looks up its
// source node by binary search over the 65 row pointers of its 64 ids, kept in LDS, and marks
// it in a per-wavefront byte array there. The counts (marked light nodes and chunks with a hit, arcs into modified counters) go to the run
// state's signal counter, as k_sys_list's do. The union step then runs on the marks.
constexpr int kFwdLoads = 8;

__global__ __launch_bounds__(kBlockThreads) void k_fwd_mark(PassArgs a) {
  DevState *st = a.st;
  if (st->halted || !st->systolic) return;
  const int32_t t = st->t;
  const uint32_t *pb = (t & 1) ? a.bits1 : a.bits0;  // counters modified by pass t-1
  const int sl = a.seed_log2;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  __shared__ int32_t s_rp[kBlockThreads / kWave][kWave + 1];
  __shared__ uint8_t s_mark[kBlockThreads / kWave][kWave];
  __shared__ int32_t s_nsig[kBlockThreads / kWave][kWave];
  int32_t *rps = s_rp[wave];
  uint8_t *mark = s_mark[wave];
  int32_t *nsig = s_nsig[wave];  // signalled successors of the sub-round's nodes so far
  const int64_t u = (int64_t)blockIdx.x * (kBlockThreads / kWave) + wave;
  uint32_t marked = 0, arcs_hit = 0;  // wavefront-uniform
  if (u < a.n_chunks) {
    const Chunk ch = a.chunks[u];
    const uint64_t below = (1ull << lane) - 1ull;
    const int32_t r0 = a.row_ptr[ch.v];  // the node's list of signalled successors
    for (int32_t base = ch.a0; base < ch.a1; base += kWave * kFwdLoads) {
      int32_t w[kFwdLoads];
      uint32_t fw[kFwdLoads];
#pragma unroll
      for (int k = 0; k < kFwdLoads; ++k) w[k] = a.col_idx[min(base + k * kWave + lane, ch.a1 - 1)];
#pragma unroll
      for (int k = 0; k < kFwdLoads; ++k) fw[k] = mod_word(pb, w[k], sl);
#pragma unroll
      for (int k = 0; k < kFwdLoads; ++k) {
        const bool h = base + k * kWave + lane < ch.a1 && mod_in_word(fw[k], w[k], sl);
        const uint64_t hits = __ballot(h);
        if (hits) {  // one atomic per load for the node's other chunks, then one entry per hit
          int32_t at = 0;
          if (lane == 0) at = atomicAdd(&a.sig_cnt[ch.v], __popcll(hits));
          at = __shfl(at, 0);
          if (h) a.sig_list[r0 + at + __popcll(hits & below)] = w[k];
          arcs_hit += __popcll(hits);
        }
      }
    }
    if (arcs_hit) {
      marked = 1;
      if (lane == 0) a.todo[ch.v] = 1;
    }
  } else if (u < (int64_t)a.n_chunks + a.n_tiles) {
    const int32_t tile = (int32_t)(u - a.n_chunks);
    const int32_t lo = tile * a.tile_nodes;
    const int32_t hi = min(a.n, lo + a.tile_nodes);
    for (int32_t s0 = lo; s0 < hi; s0 += kWave) {
      const int32_t cnt = min(kWave, hi - s0);
      const int32_t v = s0 + lane;
      const bool valid = lane < cnt;
      const int32_t r0 = valid ? a.row_ptr[v] : 0;
      const int32_t r1 = valid ? a.row_ptr[v + 1] : 0;
      if (valid) rps[lane] = r0;
      if (lane == cnt - 1) rps[cnt] = r1;
      mark[lane] = 0;
      nsig[lane] = 0;
      const uint64_t heavy = __ballot(valid && r1 - r0 > a.light_max);
      __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
      __builtin_amdgcn_wave_barrier();
      int32_t j0 = 0;
      while (j0 < cnt) {
        const uint64_t rest = heavy >> j0;
        const int32_t j1 = rest ? j0 + __ffsll((long long)rest) - 1 : cnt;  // light run [j0, j1)
        if (j1 > j0) {
          const int32_t A = rps[j0], B = rps[j1];
          for (int32_t base = A; base < B; base += kWave * kFwdLoads) {
            int32_t w[kFwdLoads];
            uint32_t fw[kFwdLoads];
#pragma unroll
            for (int k = 0; k < kFwdLoads; ++k) w[k] = a.col_idx[min(base + k * kWave + lane, B - 1)];
#pragma unroll
            for (int k = 0; k < kFwdLoads; ++k) fw[k] = mod_word(pb, w[k], sl);
#pragma unroll
            for (int k = 0; k < kFwdLoads; ++k) {
              const int32_t arc = base + k * kWave + lane;
              const bool h = arc < B && mod_in_word(fw[k], w[k], sl);
              arcs_hit += __popcll(__ballot(h));
              if (h) {  // the source node: the last j in [j0, j1) with rps[j] <= arc
                int32_t l = j0, r = j1;
                while (r - l > 1) {
                  const int32_t mid = (l + r) >> 1;
                  if (rps[mid] <= arc) l = mid; else r = mid;
                }
                mark[l] = 1;  // the same value from every lane that hits this node
                a.sig_list[rps[l] + atomicAdd(&nsig[l], 1)] = w[k];  // (a light node's arcs are all here)
              }
            }
          }
        }
        j0 = j1 + 1;
      }
      __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
      __builtin_amdgcn_wave_barrier();
      const bool hit = mark[lane] != 0;
      if (hit) {
        a.todo[v] = 1;
        a.sig_cnt[v] = nsig[lane];
      }
      marked += (uint32_t)__popcll(__ballot(hit));
      __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
      __builtin_amdgcn_wave_barrier();
    }
    if (marked && lane == 0) a.tile_todo[tile] = 1;
  }
  if (lane == 0 && (marked || arcs_hit))
    atomicAdd(reinterpret_cast<unsigned long long *>(&st->sys_acc),
              ((unsigned long long)marked << 32) | (unsigned long long)arcs_hit);
}

// Third signal kernel: the work units of the systolic pass (appended per workgroup, as in
// k_sys_list): a chunk whose node was signalled or modified by the previous pass (the copy
// rule), a light tile whose flag k_sys_mark set (the flag is consumed here) or that holds a
// modified node.
__global__ __launch_bounds__(kBlockThreads) void k_sys_units(PassArgs a) {
  DevState *st = a.st;
  if (st->halted || !st->systolic) return;
  const int32_t t = st->t;
  const uint32_t *pb = (t & 1) ? a.bits1 : a.bits0;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  constexpr int NW = kBlockThreads / kWave;
  __shared__ int32_t s_tot[kSigRounds * NW];
  __shared__ int32_t s_base;
  const uint64_t below = (1ull << lane) - 1ull;
  const int64_t units = (int64_t)a.n_chunks + a.n_tiles;
  const int64_t base = (int64_t)blockIdx.x * (kBlockThreads * kSigRounds);
  uint64_t bal[kSigRounds];
#pragma unroll
  for (int r = 0; r < kSigRounds; ++r) {
    const int64_t u = base + r * kBlockThreads + threadIdx.x;
    bool need = false;
    if (u < a.n_chunks) {
      const int32_t v = a.chunks[u].v;
      need = a.todo[v] != 0 || node_mod(pb, v, a.seed_log2);
    } else if (u < units) {
      const int32_t tile = (int32_t)(u - a.n_chunks);
      need = a.tile_todo[tile] != 0;
      if (need) {
        a.tile_todo[tile] = 0;  // consumed
      } else {  // the flag words of the tile's nodes
        const int64_t lo = (int64_t)tile * a.tile_nodes;
        const int64_t hi = min((int64_t)a.n, lo + a.tile_nodes);
        for (int64_t w = (lo << a.seed_log2) >> 5; w <= ((hi << a.seed_log2) - 1) >> 5 && !need; ++w)
          need = pb[w] != 0u;
      }
    }
    bal[r] = __ballot(need);
    if (lane == 0) s_tot[r * NW + wave] = __popcll(bal[r]);
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    int32_t acc = 0;
    for (int i = 0; i < kSigRounds * NW; ++i) {
      const int32_t x = s_tot[i];
      s_tot[i] = acc;
      acc += x;
    }
    s_base = acc ? atomicAdd(&st->sys_units, acc) : 0;
  }
  __syncthreads();
#pragma unroll
  for (int r = 0; r < kSigRounds; ++r) {
    if ((bal[r] >> lane) & 1ull) {
      const int64_t u = base + r * kBlockThreads + threadIdx.x;
      a.unit_list[s_base + s_tot[r * NW + wave] + __popcll(bal[r] & below)] = (int32_t)u;
    }
  }
}

// ------------------------------------------------------------------ kernels: transposed graph

__global__ void k_fill_u64(uint64_t *p, int64_t count, uint64_t value) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += stride) p[i] = value;
}

__global__ void k_transpose_count(const int32_t *ci, int64_t arcs, uint64_t *keys) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < arcs; e += stride)
    atomicAdd(reinterpret_cast<unsigned long long *>(keys + ci[e]), 1ull);
}

__global__ void k_transpose_rows(const uint64_t *keys, int32_t n, int32_t *trp) {
  const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (v <= n) trp[v] = (int32_t)keys[v];
}

// One wavefront per 64 consecutive nodes: their arcs form one CSR range, read 64 at a time;
// each lane finds its arc's source by binary search over the 65 row pointers (LDS) and
// appends the source to its target's predecessor list. The order inside a list is
// arbitrary (it only feeds the signal marks, a set).
__global__ __launch_bounds__(kBlockThreads) void k_transpose_fill(const int32_t *rp, const int32_t *ci, int32_t n,
                                                                  uint64_t *cursor, int32_t *tci) {
  __shared__ int32_t rps[kBlockThreads / kWave][kWave + 1];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t groups = ((int64_t)n + kWave - 1) / kWave;
  const int64_t stride = (int64_t)gridDim.x * (kBlockThreads / kWave);
  for (int64_t g = (int64_t)blockIdx.x * (kBlockThreads / kWave) + wave; g < groups; g += stride) {
    const int32_t v0 = (int32_t)(g * kWave);
    const int32_t cn = min(kWave, n - v0);
    if (lane < cn) rps[wave][lane] = rp[v0 + lane];
    if (lane == cn - 1) rps[wave][cn] = rp[v0 + cn];
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
    const int64_t A = rps[wave][0], B = rps[wave][cn];
    for (int64_t base = A; base < B; base += kWave) {
      const int32_t p = (int32_t)min(base + lane, B);
      if (p < B) {
        int32_t l = 0, r = cn;  // last node j with rps[j] <= p: the arc's source
        while (r - l > 1) {
          const int32_t mid = (l + r) >> 1;
          if (rps[wave][mid] <= p) l = mid; else r = mid;
        }
        const int32_t w = ci[p];
        const uint64_t at = atomicAdd(reinterpret_cast<unsigned long long *>(cursor + w), 1ull);
        tci[at] = v0 + l;
      }
    }
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
  }
}

// ------------------------------------------------------------------ kernels: init

// Clears the modified-counter flags, the systolic signals and the tile flags (every kernel
// that starts a run does this first; the grid covers init_lanes() threads).
__device__ __forceinline__ void clear_run_flags(const PassArgs &a, int64_t gid) {
  if (gid < 2 * ((int64_t)a.n_blocks << a.seed_log2)) {
    a.bits0[gid] = 0u;
    a.bits1[gid] = 0u;
  }
  if (a.todo && gid < (int64_t)(kNodesPerBlock / 4) * a.n_blocks) reinterpret_cast<uint32_t *>(a.todo)[gid] = 0u;
  if (gid < ((int64_t)a.n_tiles + 3) / 4) reinterpret_cast<uint32_t *>(a.tile_todo)[gid] = 0u;
}

// Algorithm 2's initialisation (add v to c[v]) into both register buffers, the estimates,
// and cleared flags. G lanes per node row, F::kRegs registers each; counter j of the row is
// lanes j*gs .. j*gs+gs-1 and is hashed with its own seed.
template <class F, int G>
__device__ __forceinline__ void init_lane(const PassArgs &a, uint64_t seed, int64_t gid) {
  clear_run_flags(a, gid);
  const int64_t v64 = gid / G;
  const int sub = (int)(gid % G);
  if (v64 >= a.n) return;  // whole slots leave together (n * G lanes, G | 256)
  const int32_t v = (int32_t)v64;
  const int gs = a.gs;
  const int j = sub / gs;
  // the item hashed is the node's id in its own graph (the caller's id when the library
  // chose its own node order); batched runs have a seed per component
  uint64_t key = a.node_id ? (uint64_t)a.node_id[v] : (uint64_t)v, sd = seed;
  bool real = true;
  if (a.batch.active) {
    const int32_t L = a.batch.blk_comp[v / kNodesPerBlock];
    const int32_t local = v - a.batch.comp_node_off[L];
    const int32_t c = a.batch.slot_comp[((size_t)L << a.seed_log2) + j];
    real = local < a.batch.comp_n[L] && c >= 0;
    key = (uint64_t)local;
    sd = c >= 0 ? a.batch.comp_seed[c] : 0ull;
  }
  const uint64_t h = splitmix64_output(sd, key + 1);
  const int b = a.log2m;
  const uint32_t idx = (uint32_t)(h >> (64 - b));
  const uint64_t rest = h << b;
  int r = rest ? __clzll((long long)rest) + 1 : 64 - b + 1;
  r = r > 31 ? 31 : r;
  // the lane holding register idx sets it; every other register is 0
  const bool mine = real && (int)(idx / F::kRegs) == sub % gs;
  const typename F::Lane c = F::single(idx % F::kRegs, mine ? (uint32_t)r : 0u);
  F::store(a.regs0, v, G, sub, c);
  F::store(a.regs1, v, G, sub, c);
  const double E = slot_estimate<F>(c, a.lc, a.K, gs);
  if (sub % gs == 0) a.est[((size_t)v << a.seed_log2) + j] = E;
}

// The kernels over row lanes sweep `lanes` threads with a grid of at most 2^28 (a launch
// holds fewer than 2^32 threads; n * G reaches that at 2^28 nodes of 256 registers). The
// sweep advances a whole workgroup at a time, so slots stay whole in every step.
template <class F, int G>
__global__ __launch_bounds__(kBlockThreads) void k_init(PassArgs a, uint64_t seed, int64_t lanes) {
  const int64_t stride = (int64_t)gridDim.x * kBlockThreads;
  for (int64_t base = (int64_t)blockIdx.x * kBlockThreads; base < lanes; base += stride)
    init_lane<F, G>(a, seed, base + threadIdx.x);
}

// Estimates of every counter of `regs` (resume from a checkpoint) and cleared flags.
template <class F, int G>
__device__ __forceinline__ void estimate_all_lane(const PassArgs &a, const uint8_t *regs, int64_t gid) {
  clear_run_flags(a, gid);
  const int64_t v64 = gid / G;
  const int sub = (int)(gid % G);
  if (v64 >= a.n) return;
  const int32_t v = (int32_t)v64;
  const int gs = a.gs;
  const double E = slot_estimate<F>(F::load(regs, v, G, sub), a.lc, a.K, gs);
  if (sub % gs == 0) a.est[((size_t)v << a.seed_log2) + sub / gs] = E;
}

template <class F, int G>
__global__ __launch_bounds__(kBlockThreads) void k_estimate_all(PassArgs a, const uint8_t *regs, int64_t lanes) {
  const int64_t stride = (int64_t)gridDim.x * kBlockThreads;
  for (int64_t base = (int64_t)blockIdx.x * kBlockThreads; base < lanes; base += stride)
    estimate_all_lane<F, G>(a, regs, base + threadIdx.x);
}

// ------------------------------------------------------------------ kernels: graph ingest

// CSR checks: row_ptr starts at 0, never decreases and ends at `arcs`; every successor id
// is in [0, n). Successor ids are read 16 bytes per lane when col_idx is 16-byte aligned.
__global__ void k_validate(const int32_t *rp, const int32_t *ci, int32_t n, int64_t arcs,
                           DevState *st) {
  int32_t err = 0;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  for (int64_t i = tid; i <= n; i += stride) {
    if (i == 0 && rp[0] != 0) err |= 1;
    if (i < n && rp[i] > rp[i + 1]) err |= 2;
    if (i == n && (int64_t)rp[n] != arcs) err |= 4;
  }
  const uint32_t un = (uint32_t)n;  // w < 0 becomes >= 2^31 > n
  const int64_t quads = (reinterpret_cast<uintptr_t>(ci) & 15u) == 0 ? arcs / 4 : 0;
  const int4 *ci4 = reinterpret_cast<const int4 *>(ci);
  for (int64_t q = tid; q < quads; q += stride) {
    const int4 w = ci4[q];
    if ((uint32_t)w.x >= un || (uint32_t)w.y >= un || (uint32_t)w.z >= un || (uint32_t)w.w >= un) err |= 8;
  }
  for (int64_t i = 4 * quads + tid; i < arcs; i += stride)
    if ((uint32_t)ci[i] >= un) err |= 8;
  if (err) atomicOr(&st->err, err);
}

__global__ void k_check_registers(const uint32_t *words, int64_t nwords, DevState *st) {
  int32_t err = 0;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nwords; i += stride)
    if (words[i] & 0xe0e0e0e0u) err = 16;  // a register above 31
  if (err) atomicOr(&st->err, err);
}

__global__ void k_state_reset(DevState *st, int32_t t, int32_t frontier, int32_t max_passes,
                              int64_t dense_threshold, int32_t sys_div) {
  st->t = t;
  st->halted = 0;
  st->done = 0;
  st->capped = 0;
  st->first_pass = 1;
  st->frontier = frontier;
  st->max_passes = max_passes;
  st->passes = 0;
  st->err = 0;
  st->changed_last = -1;
  st->dense_next = 0;
  st->dense_threshold = dense_threshold;
  st->systolic = 0;
  st->sys_div = sys_div;
  st->sys_acc = 0ull;
  st->sys_units = 0;
  st->use_sum = 0;
}

// keys[v] = (chunks of v) << 32 | (v needs a combine step); keys[n] = 0.
__global__ void k_classify(const int32_t *rp, int32_t n, int32_t light_max, int32_t chunk_arcs,
                           uint64_t *keys) {
  const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (v > n) return;
  if (v == n) {
    keys[n] = 0;
    return;
  }
  const int32_t deg = rp[v + 1] - rp[v];
  uint64_t nch = 0;
  if (deg > light_max) nch = ((uint64_t)deg + chunk_arcs - 1) / chunk_arcs;
  keys[v] = (nch << 32) | (nch > 1 ? 1ull : 0ull);
}

__global__ void k_fill_chunks(const int32_t *rp, int32_t n, const uint64_t *offs, int32_t chunk_arcs,
                              Chunk *chunks, Heavy *heavy) {
  const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= n) return;
  const uint64_t o0 = offs[v], o1 = offs[v + 1];
  const int32_t c0 = (int32_t)(o0 >> 32), nch = (int32_t)((o1 >> 32) - (o0 >> 32));
  if (nch == 0) return;
  const bool multi = nch > 1;
  const int32_t beg = rp[v], end = rp[v + 1];
  for (int32_t j = 0; j < nch; ++j) {
    Chunk c;
    c.v = (int32_t)v;
    const int64_t a0 = (int64_t)beg + (int64_t)j * chunk_arcs;
    c.a0 = (int32_t)a0;
    c.a1 = (int32_t)min((int64_t)end, a0 + chunk_arcs);
    c.part = multi ? c0 + j : -1;
    chunks[c0 + j] = c;
  }
  if (multi) {
    Heavy h;
    h.v = (int32_t)v;
    h.first = c0;
    h.count = nch;
    h.pad_ = 0;
    heavy[(int32_t)(o0 & 0xffffffffull)] = h;
  }
}

// One workgroup per tile of consecutive ids: light nodes sorted by decreasing degree (ties
// by id), the rest of the tile filled with -1. The workgroup is as wide as the bitonic sort:
// the power of two >= tile_nodes (at least one wavefront).
__global__ __launch_bounds__(kMaxTile) void k_build_tiles(const int32_t *rp, int32_t n, int32_t light_max,
                                                          int32_t tile_nodes, int32_t *light) {
  __shared__ uint64_t keys[kMaxTile];
  const int i = threadIdx.x;
  const int width = (int)blockDim.x;
  const int64_t base = (int64_t)blockIdx.x * tile_nodes;
  const int64_t v = base + i;
  uint64_t key = ~0ull;
  if (i < tile_nodes && v < n) {
    const int32_t deg = rp[v + 1] - rp[v];
    // nodes without successors never change: their counter stays c_0 in both buffers
    if (deg > 0 && deg <= light_max) key = ((uint64_t)(0x7fffffff - deg) << 32) | (uint32_t)i;
  }
  keys[i] = key;
  __syncthreads();
  for (int k = 2; k <= width; k <<= 1) {
    for (int j = k >> 1; j > 0; j >>= 1) {
      const int p = i ^ j;
      if (p > i) {
        const uint64_t x = keys[i], y = keys[p];
        const bool up = (i & k) == 0;
        if ((x > y) == up) {
          keys[i] = y;
          keys[p] = x;
        }
      }
      __syncthreads();
    }
  }
  if (i < tile_nodes) {
    const uint64_t s = keys[i];
    light[base + i] = (s == ~0ull) ? -1 : (int32_t)(base + (int64_t)(s & 0xffffffffull));
  }
}

// ------------------------------------------------------------------ exclusive scan (uint64)

constexpr int kScanThreads = 256;
constexpr int kScanPer = 4;
constexpr int kScanBlock = kScanThreads * kScanPer;

__device__ uint64_t block_exclusive_scan(uint64_t x, uint64_t *total) {
  __shared__ uint64_t buf[kScanThreads];
  const int i = threadIdx.x;
  buf[i] = x;
  __syncthreads();
  for (int off = 1; off < kScanThreads; off <<= 1) {
    const uint64_t y = i >= off ? buf[i - off] : 0;
    __syncthreads();
    buf[i] += y;
    __syncthreads();
  }
  const uint64_t incl = buf[i];
  *total = buf[kScanThreads - 1];
  __syncthreads();
  return incl - x;
}

__global__ __launch_bounds__(kScanThreads) void k_scan_sums(const uint64_t *d, int64_t n, uint64_t *sums) {
  const int64_t base = (int64_t)blockIdx.x * kScanBlock + (int64_t)threadIdx.x * kScanPer;
  uint64_t s = 0;
  for (int k = 0; k < kScanPer; ++k)
    if (base + k < n) s += d[base + k];
  uint64_t total;
  block_exclusive_scan(s, &total);
  if (threadIdx.x == 0) sums[blockIdx.x] = total;
}

__global__ __launch_bounds__(kScanThreads) void k_scan_top(uint64_t *sums, int64_t nb) {
  const int64_t per = (nb + kScanThreads - 1) / kScanThreads;
  const int64_t lo = (int64_t)threadIdx.x * per, hi = min(nb, lo + per);
  uint64_t s = 0;
  for (int64_t i = lo; i < hi; ++i) s += sums[i];
  uint64_t total;
  uint64_t run = block_exclusive_scan(s, &total);
  for (int64_t i = lo; i < hi; ++i) {
    const uint64_t x = sums[i];
    sums[i] = run;
    run += x;
  }
}

__global__ __launch_bounds__(kScanThreads) void k_scan_apply(uint64_t *d, int64_t n, const uint64_t *sums) {
  const int64_t base = (int64_t)blockIdx.x * kScanBlock + (int64_t)threadIdx.x * kScanPer;
  uint64_t v[kScanPer];
  uint64_t s = 0;
  for (int k = 0; k < kScanPer; ++k) {
    v[k] = base + k < n ? d[base + k] : 0;
    s += v[k];
  }
  uint64_t total;
  uint64_t run = block_exclusive_scan(s, &total) + sums[blockIdx.x];
  for (int k = 0; k < kScanPer; ++k) {
    if (base + k < n) d[base + k] = run;
    run += v[k];
  }
}

// ------------------------------------------------------------------ kernels: transpose by buckets

// The transposed graph by a two-level counting sort, with no global atomic per arc. Arcs
// are first grouped by target into buckets of 2^bs consecutive ids (at most kTpBuckets
// buckets; node ranges of `range` nodes count and place their arcs with LDS counters),
// then each bucket is sorted by target in LDS: in one workgroup, or in chunks for the
// buckets of hubs. The order inside a predecessor list is arbitrary.
constexpr int kTpBuckets = kTpNumBuckets;  // first-level buckets (LDS counters)
constexpr int kTpMaxBucket = 8192;  // ids per bucket (LDS counters of the second level)
constexpr int kTpThreads = 256;     // = kScanThreads (block_exclusive_scan)

// Per node range r: arcs into every bucket b, stored bucket-major at hist[b * n_ranges + r]
// so that one exclusive scan gives every (bucket, range) its place.
__global__ __launch_bounds__(kTpThreads) void k_tp_hist(const int32_t *rp, const int32_t *ci, int32_t n, int32_t range,
                                                       int32_t bs, int32_t nb, int32_t n_ranges, uint64_t *hist) {
  __shared__ uint32_t cnt[kTpBuckets];
  for (int i = threadIdx.x; i < nb; i += kTpThreads) cnt[i] = 0u;
  __syncthreads();
  const int32_t r = blockIdx.x;
  const int64_t v0 = (int64_t)r * range, v1 = min((int64_t)n, v0 + range);
  const int64_t a0 = rp[v0], a1 = rp[v1];
  for (int64_t a = a0 + threadIdx.x; a < a1; a += kTpThreads) atomicAdd(&cnt[ci[a] >> bs], 1u);
  __syncthreads();
  for (int i = threadIdx.x; i < nb; i += kTpThreads) hist[(int64_t)i * n_ranges + r] = cnt[i];
}

// Places the arcs of node range r as (target - bucket start) << 32 | source at the
// positions of the scanned histogram (one LDS cursor per bucket). Each wavefront takes 64
// consecutive nodes at a time and finds an arc's source by binary search over their row
// pointers in LDS.
__global__ __launch_bounds__(kTpThreads) void k_tp_scatter(const int32_t *rp, const int32_t *ci, int32_t n, int32_t range,
                                                          int32_t bs, int32_t nb, int32_t n_ranges, const uint64_t *pos,
                                                          uint64_t *pairs) {
  __shared__ uint32_t cur[kTpBuckets];
  __shared__ int32_t rps[kTpThreads / kWave][kWave + 1];
  const int32_t r = blockIdx.x;
  for (int i = threadIdx.x; i < nb; i += kTpThreads) cur[i] = (uint32_t)pos[(int64_t)i * n_ranges + r];
  __syncthreads();
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const uint32_t low = (1u << bs) - 1u;
  const int64_t v0 = (int64_t)r * range, v1 = min((int64_t)n, v0 + range);
  for (int64_t g0 = v0 + (int64_t)wave * kWave; g0 < v1; g0 += kTpThreads) {
    const int32_t cn = (int32_t)min((int64_t)kWave, v1 - g0);
    if (lane < cn) rps[wave][lane] = rp[g0 + lane];
    if (lane == cn - 1) rps[wave][cn] = rp[g0 + cn];
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
    const int64_t A = rps[wave][0], B = rps[wave][cn];
    for (int64_t base = A; base < B; base += kWave) {
      const int64_t p = base + lane;
      if (p < B) {
        int32_t l = 0, h = cn;  // the arc's source: the last node j with rps[j] <= p
        while (h - l > 1) {
          const int32_t mid = (l + h) >> 1;
          if (rps[wave][mid] <= p) l = mid; else h = mid;
        }
        const uint32_t w = (uint32_t)ci[p];
        const uint32_t at = atomicAdd(&cur[w >> bs], 1u);
        pairs[at] = ((uint64_t)(w & low) << 32) | (uint64_t)(uint32_t)(g0 + l);
      }
    }
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
  }
}

// Start of every bucket's pairs (and the total at bstart[nb]).
__global__ void k_tp_bounds(const uint64_t *pos, int32_t nb, int32_t n_ranges, uint64_t *bstart) {
  const int32_t b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b <= nb) bstart[b] = pos[(int64_t)b * n_ranges];
}

// Counts per target of a run of a bucket's pairs, into LDS.
__device__ __forceinline__ void tp_count(const uint64_t *pairs, int64_t lo, int64_t hi, uint32_t *cnt) {
  for (int64_t p = lo + threadIdx.x; p < hi; p += kTpThreads) atomicAdd(&cnt[(uint32_t)(pairs[p] >> 32)], 1u);
}

// A whole bucket in one workgroup: counts per target, their exclusive scan (the bucket's
// rows of the transposed graph), then every source placed with LDS cursors.
__global__ __launch_bounds__(kTpThreads) void k_tp_bucket(const uint64_t *pairs, const uint64_t *bstart,
                                                         const int32_t *blist, int32_t bs, int32_t n, int32_t *trp,
                                                         int32_t *tci) {
  __shared__ uint32_t cnt[kTpMaxBucket];
  const int32_t b = blist[blockIdx.x];
  const int32_t B = 1 << bs;
  const int64_t s = (int64_t)bstart[b], e = (int64_t)bstart[b + 1];
  for (int i = threadIdx.x; i < B; i += kTpThreads) cnt[i] = 0u;
  __syncthreads();
  tp_count(pairs, s, e, cnt);
  __syncthreads();
  const int per = B / kTpThreads, i0 = threadIdx.x * per;  // B is a multiple of 256
  uint64_t sum = 0;
  for (int k = 0; k < per; ++k) sum += cnt[i0 + k];
  uint64_t total;
  uint64_t run = block_exclusive_scan(sum, &total);
  for (int k = 0; k < per; ++k) {
    const uint32_t c = cnt[i0 + k];
    const int64_t v = ((int64_t)b << bs) + i0 + k;
    if (v < n) trp[v] = (int32_t)(s + (int64_t)run);
    cnt[i0 + k] = (uint32_t)run;  // cursor, relative to s
    run += c;
  }
  __syncthreads();
  for (int64_t p = s + threadIdx.x; p < e; p += kTpThreads) {
    const uint64_t x = pairs[p];
    const uint32_t at = atomicAdd(&cnt[(uint32_t)(x >> 32)], 1u);
    tci[s + at] = (int32_t)(uint32_t)x;
  }
}

// Buckets of hubs, in chunks: counts per target of every chunk (h2[chunk][target]).
__global__ __launch_bounds__(kTpThreads) void k_tp_chunk_hist(const uint64_t *pairs, const int64_t *chunk_lo,
                                                             const int64_t *chunk_hi, int32_t bs, uint32_t *h2) {
  __shared__ uint32_t cnt[kTpMaxBucket];
  const int32_t B = 1 << bs;
  const int32_t k = blockIdx.x;
  for (int i = threadIdx.x; i < B; i += kTpThreads) cnt[i] = 0u;
  __syncthreads();
  tp_count(pairs, chunk_lo[k], chunk_hi[k], cnt);
  __syncthreads();
  for (int i = threadIdx.x; i < B; i += kTpThreads) h2[(int64_t)k * B + i] = cnt[i];
}

// Per hub bucket: rows of the transposed graph from the chunk counts, and every chunk's
// place in every row (h2 rewritten with positions relative to the bucket start).
__global__ __launch_bounds__(kTpThreads) void k_tp_heavy_scan(const uint64_t *bstart, const int32_t *hlist,
                                                             const int32_t *hchunk0, int32_t bs, int32_t n,
                                                             uint32_t *h2, int32_t *trp) {
  const int32_t b = hlist[blockIdx.x];
  const int32_t k0 = hchunk0[blockIdx.x], k1 = hchunk0[blockIdx.x + 1];
  const int32_t B = 1 << bs;
  const int64_t s = (int64_t)bstart[b];
  const int per = B / kTpThreads, i0 = threadIdx.x * per;
  uint64_t sum = 0;
  for (int i = i0; i < i0 + per; ++i)
    for (int32_t k = k0; k < k1; ++k) sum += h2[(int64_t)k * B + i];
  uint64_t total;
  uint64_t run = block_exclusive_scan(sum, &total);
  for (int i = i0; i < i0 + per; ++i) {
    const int64_t v = ((int64_t)b << bs) + i;
    if (v < n) trp[v] = (int32_t)(s + (int64_t)run);
    for (int32_t k = k0; k < k1; ++k) {
      const uint32_t c = h2[(int64_t)k * B + i];
      h2[(int64_t)k * B + i] = (uint32_t)run;
      run += c;
    }
  }
}

// Places the sources of one chunk of a hub bucket with LDS cursors from h2.
__global__ __launch_bounds__(kTpThreads) void k_tp_chunk_scatter(const uint64_t *pairs, const int64_t *chunk_lo,
                                                                const int64_t *chunk_hi, const int64_t *chunk_s,
                                                                int32_t bs, const uint32_t *h2, int32_t *tci) {
  __shared__ uint32_t cur[kTpMaxBucket];
  const int32_t B = 1 << bs;
  const int32_t k = blockIdx.x;
  for (int i = threadIdx.x; i < B; i += kTpThreads) cur[i] = h2[(int64_t)k * B + i];
  __syncthreads();
  const int64_t s = chunk_s[k];
  for (int64_t p = chunk_lo[k] + threadIdx.x; p < chunk_hi[k]; p += kTpThreads) {
    const uint64_t x = pairs[p];
    const uint32_t at = atomicAdd(&cur[(uint32_t)(x >> 32)], 1u);
    tci[s + at] = (int32_t)(uint32_t)x;
  }
}

// ------------------------------------------------------------------ statistics (Sections 4-5)


__global__ void k_stats(const double *nt, const int32_t *T_or_null, const DevState *st, double alpha,
                        double eps, int32_t distinct, double *out) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  const int32_t T = (T_or_null && *T_or_null >= 0) ? *T_or_null : st->t;
  stats_of(nt, T, alpha, eps, distinct, out);
}

// Statistics of every component of a batch, one thread each: record out[c] (every field
// written, so `out` needs no clearing).
__global__ void k_stats_all(PassArgs a, double alpha, double eps, int32_t distinct, StatsRec *out) {
  const int32_t c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= a.batch.n_comp) return;
  const int32_t Tc = a.batch.comp_T[c];
  double b[9];
  stats_of(a.batch.comp_nt + (size_t)c * a.nt_cap, Tc >= 0 ? Tc : a.st->t, alpha, eps, distinct, b);
  StatsRec r;
#pragma unroll
  for (int k = 0; k < 8; ++k) r.v[k] = b[k];
  r.T = (int32_t)b[8];
  r.distinct = distinct;
  out[c] = r;
}

// The paper's a-posteriori figures over many runs of one graph (Section 6): for graph g
// (components g * n_seeds .. g * n_seeds + n_seeds - 1, one thread per graph), the mean of
// ed, ied, the average distance and spid over its runs, then their sample standard deviation
// (n_seeds - 1 in the denominator, two passes over the runs; NaN with one run).
__global__ void k_seed_summary(PassArgs a, int32_t n_graphs, int32_t n_seeds, double alpha, int32_t distinct,
                               SummaryRec *out) {
  const int32_t g = blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= n_graphs) return;
  constexpr int kPick[4] = {0, 1, 2, 4};  // ed, ied, avg_dist, spid in stats_of's output
  double mean[4] = {0.0, 0.0, 0.0, 0.0}, ss[4] = {0.0, 0.0, 0.0, 0.0};
  for (int pass = 0; pass < 2; ++pass) {
    for (int32_t s = 0; s < n_seeds; ++s) {
      const int32_t c = g * n_seeds + s;
      const int32_t Tc = a.batch.comp_T[c];
      double b[9];
      stats_of(a.batch.comp_nt + (size_t)c * a.nt_cap, Tc >= 0 ? Tc : a.st->t, alpha, 0.0, distinct, b);
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const double x = b[kPick[k]];
        if (pass == 0) {
          mean[k] += x;
        } else {
          const double d = x - mean[k];
          ss[k] += d * d;
        }
      }
    }
    if (pass == 0)
#pragma unroll
      for (int k = 0; k < 4; ++k) mean[k] /= (double)n_seeds;
  }
  SummaryRec r;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    r.v[k] = mean[k];
    r.v[4 + k] = n_seeds > 1 ? sqrt(ss[k] / (double)(n_seeds - 1)) : __builtin_nan("");
  }
  r.runs = n_seeds;
  r.distinct = distinct;
  out[g] = r;
}

__global__ void k_bytemax_words(const uint32_t *x, const uint32_t *y, uint32_t *out, int64_t count) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += stride)
    out[i] = bytemax(x[i], y[i]);
}

// The union step's gather accumulator on its own: out[i] = the register-wise max of the k
// lanes x[i*k .. i*k+k), accumulated from empty (from_first 0) or from the first lane.
__global__ void k_gathermax_lanes(const uint4 *x, int32_t k, int32_t from_first, uint4 *out, int64_t count) {
  using F = ByteRegs;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += stride) {
    const uint4 *g = x + i * k;
    F::Acc a = from_first ? F::acc_from(g[0]) : F::acc_zero();
    for (int32_t j = from_first ? 1 : 0; j < k; ++j) F::acc_add(a, g[j]);
    out[i] = F::acc_value(a);
  }
}

// The packed max on its own: groups of 64 5-bit registers (five 64-bit words each).
__global__ void k_max5_groups(const uint8_t *x, const uint8_t *y, uint8_t *out, int64_t groups) {
  using F = Packed5Regs;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g < groups; g += stride)
    F::store(out, g, 1, 0, F::max(F::load(x, g, 1, 0), F::load(y, g, 1, 0)));
}

// One counter of every row of a packed layout to one register per byte: `rows` rows of
// `row_stride` bytes from `src` (the counter's first byte in the first row), `gpr` groups of
// 64 registers per counter; group q of row r goes to out + (r * gpr + q) * 64.
__global__ void k_unpack5_rows(const uint8_t *src, int64_t row_stride, int32_t gpr, int64_t rows, uint8_t *out) {
  using F = Packed5Regs;
  const int64_t groups = rows * gpr;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g < groups; g += stride) {
    const int64_t r = g / gpr, q = g % gpr;
    const F::Lane x = F::load(src + r * row_stride + q * F::kBytes, 0, 1, 0);
    uint32_t w[16];
#pragma unroll
    for (int i = 0; i < 16; ++i) w[i] = 0u;
#pragma unroll
    for (int j = 0; j < 64; ++j) w[j >> 2] |= F::field(x, j) << (8 * (j & 3));
    uint4 *o = reinterpret_cast<uint4 *>(out + g * 64);
#pragma unroll
    for (int i = 0; i < 4; ++i) o[i] = make_uint4(w[4 * i], w[4 * i + 1], w[4 * i + 2], w[4 * i + 3]);
  }
}

// Packed counters (5 bits per register) to one register per byte and back, 64 registers
// per thread: group g is bytes 40g .. 40g+39 packed and 64g .. 64g+63 unpacked.
__global__ void k_unpack5(const uint8_t *packed, uint8_t *out, int64_t groups) {
  using F = Packed5Regs;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g < groups; g += stride) {
    const F::Lane x = F::load(packed, g, 1, 0);
    uint32_t w[16];
#pragma unroll
    for (int i = 0; i < 16; ++i) w[i] = 0u;
#pragma unroll
    for (int j = 0; j < 64; ++j) w[j >> 2] |= F::field(x, j) << (8 * (j & 3));
    uint4 *q = reinterpret_cast<uint4 *>(out + g * 64);
#pragma unroll
    for (int i = 0; i < 4; ++i) q[i] = make_uint4(w[4 * i], w[4 * i + 1], w[4 * i + 2], w[4 * i + 3]);
  }
}

// Registers must be <= 31 (checked by the caller).
__global__ void k_pack5(const uint8_t *in, uint8_t *packed, int64_t groups) {
  using F = Packed5Regs;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g < groups; g += stride) {
    const uint4 *q = reinterpret_cast<const uint4 *>(in + g * 64);
    uint32_t w[16];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const uint4 t = q[i];
      w[4 * i] = t.x;
      w[4 * i + 1] = t.y;
      w[4 * i + 2] = t.z;
      w[4 * i + 3] = t.w;
    }
    F::Lane x = F::zero();
#pragma unroll
    for (int j = 0; j < 64; ++j) {
      const int p = 5 * j, i = p >> 5, o = p & 31;
      const uint32_t r = (w[j >> 2] >> (8 * (j & 3))) & 31u;
      x.w[i] |= r << o;
      if (o > 27) x.w[i + 1 < 10 ? i + 1 : 9] |= r >> (32 - o);
    }
    F::store(packed, g, 1, 0, x);
  }
}

// Workgroups of a sweep over row lanes: 2^28 threads per step of the sweep.
constexpr int64_t kLaneSweepWgs = (int64_t)1 << 20;

int grid_for(int64_t items, int threads, int64_t cap = 1 << 20) {
  int64_t g = (items + threads - 1) / threads;
  if (g < 1) g = 1;
  if (g > cap) g = cap;
  return (int)g;
}

}  // namespace

// ------------------------------------------------------------------ launchers

hipError_t launch_validate(const int32_t *row_ptr, const int32_t *col_idx, int32_t n, int64_t arcs,
                           DevState *st, hipStream_t s) {
  const int64_t top = arcs > (int64_t)n + 1 ? arcs : (int64_t)n + 1;
  hipLaunchKernelGGL(k_validate, dim3(grid_for(top, 256, 8192)), dim3(256), 0, s, row_ptr, col_idx, n,
                     arcs, st);
  return hipGetLastError();
}

hipError_t launch_state_reset(DevState *st, int32_t t, int32_t frontier, int32_t max_passes,
                              int64_t dense_threshold, int32_t sys_div, hipStream_t s) {
  hipLaunchKernelGGL(k_state_reset, dim3(1), dim3(1), 0, s, st, t, frontier, max_passes, dense_threshold,
                     sys_div);
  return hipGetLastError();
}

hipError_t launch_classify(const int32_t *row_ptr, int32_t n, int32_t light_max, int32_t chunk_arcs,
                           uint64_t *keys, hipStream_t s) {
  hipLaunchKernelGGL(k_classify, dim3(grid_for((int64_t)n + 1, 256, 1 << 30)), dim3(256), 0, s, row_ptr,
                     n, light_max, chunk_arcs, keys);
  return hipGetLastError();
}

int64_t scan_tmp_elems(int64_t n) { return (n + kScanBlock - 1) / kScanBlock + 1; }

hipError_t launch_exclusive_scan_u64(uint64_t *data, int64_t n, uint64_t *tmp, hipStream_t s) {
  const int64_t nb = (n + kScanBlock - 1) / kScanBlock;
  hipLaunchKernelGGL(k_scan_sums, dim3((unsigned)nb), dim3(kScanThreads), 0, s, data, n, tmp);
  hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(kScanThreads), 0, s, tmp, nb);
  hipLaunchKernelGGL(k_scan_apply, dim3((unsigned)nb), dim3(kScanThreads), 0, s, data, n, tmp);
  return hipGetLastError();
}

hipError_t launch_fill_chunks(const int32_t *row_ptr, int32_t n, const uint64_t *offs,
                              int32_t chunk_arcs, Chunk *chunks, Heavy *heavy, hipStream_t s) {
  hipLaunchKernelGGL(k_fill_chunks, dim3(grid_for(n, 256, 1 << 30)), dim3(256), 0, s, row_ptr, n, offs,
                     chunk_arcs, chunks, heavy);
  return hipGetLastError();
}

hipError_t launch_build_tiles(const int32_t *row_ptr, int32_t n, int32_t light_max, int32_t tile_nodes,
                              int32_t n_tiles, int32_t *light, hipStream_t s) {
  if (tile_nodes < 1 || tile_nodes > kMaxTile) return hipErrorInvalidValue;
  int width = kWave;
  while (width < tile_nodes) width <<= 1;
  hipLaunchKernelGGL(k_build_tiles, dim3((unsigned)n_tiles), dim3(width), 0, s, row_ptr, n, light_max,
                     tile_nodes, light);
  return hipGetLastError();
}

// Instantiations: byte registers with 1..64 lanes per node row (rows up to 1024 bytes),
// 5-bit registers with 1..16 (rows up to 1024 registers, 640 bytes).
#define HANF_DISPATCH_FG(P_, G_, EXPR)                          \
  if (P_) {                                                     \
    using F = Packed5Regs;                                      \
    switch (G_) {                                               \
      case 1: { constexpr int G = 1; EXPR; } break;             \
      case 2: { constexpr int G = 2; EXPR; } break;             \
      case 4: { constexpr int G = 4; EXPR; } break;             \
      case 8: { constexpr int G = 8; EXPR; } break;             \
      case 16: { constexpr int G = 16; EXPR; } break;           \
      default: return hipErrorInvalidValue;                     \
    }                                                           \
  } else {                                                      \
    using F = ByteRegs;                                         \
    switch (G_) {                                               \
      case 1: { constexpr int G = 1; EXPR; } break;             \
      case 2: { constexpr int G = 2; EXPR; } break;             \
      case 4: { constexpr int G = 4; EXPR; } break;             \
      case 8: { constexpr int G = 8; EXPR; } break;             \
      case 16: { constexpr int G = 16; EXPR; } break;           \
      case 32: { constexpr int G = 32; EXPR; } break;           \
      case 64: { constexpr int G = 64; EXPR; } break;           \
      default: return hipErrorInvalidValue;                     \
    }                                                           \
  }

// A launch whose start and end record `e0` and `e1` (either may be NULL): the events are
// taken from the kernel's own dispatch, so timing a pass adds no marker between its kernels.
template <typename... KArgs, typename... Args>
void launch_k(void (*kernel)(KArgs...), dim3 grid, dim3 block, hipStream_t s, hipEvent_t e0, hipEvent_t e1,
              Args... args) {
  if (e0 || e1)
    hipExtLaunchKernelGGL(kernel, grid, block, 0, s, e0, e1, 0, args...);
  else
    hipLaunchKernelGGL(kernel, grid, block, 0, s, args...);
}

// The same with `lds` bytes of dynamic LDS per workgroup.
template <typename... KArgs, typename... Args>
void launch_k_lds(void (*kernel)(KArgs...), dim3 grid, dim3 block, size_t lds, hipStream_t s, hipEvent_t e0,
                  hipEvent_t e1, Args... args) {
  if (e0 || e1)
    hipExtLaunchKernelGGL(kernel, grid, block, lds, s, e0, e1, 0, args...);
  else
    hipLaunchKernelGGL(kernel, grid, block, lds, s, args...);
}

// Events of a group that launched no kernel: recorded on the stream instead.
hipError_t record_empty(hipEvent_t e0, hipEvent_t e1, hipStream_t s) {
  if (e0) (void)hipEventRecord(e0, s);
  if (e1) (void)hipEventRecord(e1, s);
  return hipGetLastError();
}

// Lanes per node row: S counters of m/16 lanes each (bytes), or of m/64 lanes (5-bit).
int row_lanes(const PassArgs &a) {
  return (a.packed ? 1 << (a.log2m - 6) : 1 << (a.log2m - 4)) << a.seed_log2;
}

// Threads of the kernels that start a run: one per row lane, and enough to clear the flag
// words, signal bytes and tile flags.
int64_t init_lanes(const PassArgs &a) {
  int64_t lanes = (int64_t)a.n * row_lanes(a);
  lanes = std::max<int64_t>(lanes, 2 * ((int64_t)a.n_blocks << a.seed_log2));
  lanes = std::max<int64_t>(lanes, (int64_t)(kNodesPerBlock / 4) * a.n_blocks);
  lanes = std::max<int64_t>(lanes, ((int64_t)a.n_tiles + 3) / 4);
  return lanes;
}

hipError_t launch_init(const PassArgs &a, uint64_t seed, hipStream_t s) {
  const int G = row_lanes(a);
  const int64_t lanes = init_lanes(a);
  const int grid = grid_for(lanes, kBlockThreads, kLaneSweepWgs);
  HANF_DISPATCH_FG(a.packed, G,
                   hipLaunchKernelGGL((k_init<F, G>), dim3(grid), dim3(kBlockThreads), 0, s, a, seed, lanes));
  return hipGetLastError();
}

hipError_t launch_estimate_all(const PassArgs &a, const uint8_t *regs, hipStream_t s) {
  const int G = row_lanes(a);
  const int64_t lanes = init_lanes(a);
  const int grid = grid_for(lanes, kBlockThreads, kLaneSweepWgs);
  HANF_DISPATCH_FG(a.packed, G,
                   hipLaunchKernelGGL((k_estimate_all<F, G>), dim3(grid), dim3(kBlockThreads), 0, s, a, regs, lanes));
  return hipGetLastError();
}

hipError_t launch_signal(const PassArgs &a, int64_t arcs, hipStream_t s, hipEvent_t e0, hipEvent_t e1) {
  if (!a.trow_ptr) {
    if (!a.todo) return record_empty(e0, e1, s);
    // no transposed graph: the marks come from a forward scan of the successor lists
    const int64_t units = (int64_t)a.n_chunks + a.n_tiles;
    launch_k(k_fwd_mark, dim3(grid_for(units, kBlockThreads / kWave, 1 << 30)), dim3(kBlockThreads), s, e0, nullptr, a);
    launch_k(k_sys_units, dim3(grid_for(units, kBlockThreads * kSigRounds, 1 << 30)), dim3(kBlockThreads), s, nullptr,
             e1, a);
    return hipGetLastError();
  }
  launch_k(k_sys_list, dim3(grid_for(2 * ((int64_t)a.n_blocks << a.seed_log2), kBlockThreads * kSigRounds, 1 << 30)),
           dim3(kBlockThreads), s, e0, nullptr, a);
  hipLaunchKernelGGL(k_sys_mark, dim3(grid_for(arcs, kMarkTile, 2048)), dim3(kBlockThreads), 0, s, a);
  launch_k(k_sys_units, dim3(grid_for((int64_t)a.n_chunks + a.n_tiles, kBlockThreads * kSigRounds, 1 << 30)),
           dim3(kBlockThreads), s, nullptr, e1, a);
  return hipGetLastError();
}

hipError_t launch_fill_u64(uint64_t *p, int64_t count, uint64_t value, hipStream_t s) {
  hipLaunchKernelGGL(k_fill_u64, dim3(grid_for(count, 256, 8192)), dim3(256), 0, s, p, count, value);
  return hipGetLastError();
}

hipError_t launch_tp_first(const int32_t *row_ptr, const int32_t *col_idx, int32_t n, int32_t range, int32_t bs,
                           int32_t nb, int32_t n_ranges, uint64_t *hist, uint64_t *scan_tmp, uint64_t *pairs,
                           uint64_t *bstart, hipStream_t s) {
  hipLaunchKernelGGL(k_tp_hist, dim3((unsigned)n_ranges), dim3(kTpThreads), 0, s, row_ptr, col_idx, n, range, bs, nb,
                     n_ranges, hist);
  hipError_t e = launch_fill_u64(hist + (int64_t)nb * n_ranges, 1, 0ull, s);  // the total's slot
  if (e != hipSuccess) return e;
  e = launch_exclusive_scan_u64(hist, (int64_t)nb * n_ranges + 1, scan_tmp, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_tp_scatter, dim3((unsigned)n_ranges), dim3(kTpThreads), 0, s, row_ptr, col_idx, n, range, bs, nb,
                     n_ranges, hist, pairs);
  hipLaunchKernelGGL(k_tp_bounds, dim3(grid_for((int64_t)nb + 1, 256, 1 << 30)), dim3(256), 0, s, hist, nb, n_ranges,
                     bstart);
  return hipGetLastError();
}

hipError_t launch_tp_second(const uint64_t *pairs, const uint64_t *bstart, const int32_t *blist, int32_t n_light,
                            const int32_t *hlist, const int32_t *hchunk0, int32_t n_heavy, const int64_t *chunk_lo,
                            const int64_t *chunk_hi, const int64_t *chunk_s, int32_t n_hchunks, uint32_t *h2, int32_t bs,
                            int32_t n, int32_t *trow_ptr, int32_t *tcol_idx, hipStream_t s) {
  if (n_light > 0)
    hipLaunchKernelGGL(k_tp_bucket, dim3((unsigned)n_light), dim3(kTpThreads), 0, s, pairs, bstart, blist, bs, n,
                       trow_ptr, tcol_idx);
  if (n_heavy > 0) {
    hipLaunchKernelGGL(k_tp_chunk_hist, dim3((unsigned)n_hchunks), dim3(kTpThreads), 0, s, pairs, chunk_lo, chunk_hi, bs,
                       h2);
    hipLaunchKernelGGL(k_tp_heavy_scan, dim3((unsigned)n_heavy), dim3(kTpThreads), 0, s, bstart, hlist, hchunk0, bs, n,
                       h2, trow_ptr);
    hipLaunchKernelGGL(k_tp_chunk_scatter, dim3((unsigned)n_hchunks), dim3(kTpThreads), 0, s, pairs, chunk_lo, chunk_hi,
                       chunk_s, bs, h2, tcol_idx);
  }
  return hipGetLastError();
}

hipError_t launch_transpose_count(const int32_t *col_idx, int64_t arcs, uint64_t *keys, hipStream_t s) {
  if (arcs == 0) return hipSuccess;
  hipLaunchKernelGGL(k_transpose_count, dim3(grid_for(arcs, 256, 16384)), dim3(256), 0, s, col_idx, arcs, keys);
  return hipGetLastError();
}

hipError_t launch_transpose_fill(const int32_t *row_ptr, const int32_t *col_idx, int32_t n, uint64_t *keys,
                                 int32_t *trow_ptr, int32_t *tcol_idx, hipStream_t s) {
  hipLaunchKernelGGL(k_transpose_rows, dim3(grid_for((int64_t)n + 1, 256, 1 << 30)), dim3(256), 0, s, keys, n,
                     trow_ptr);
  const int64_t groups = ((int64_t)n + kWave - 1) / kWave;
  hipLaunchKernelGGL(k_transpose_fill, dim3(grid_for(groups, kBlockThreads / kWave, 1 << 16)), dim3(kBlockThreads), 0,
                     s, row_ptr, col_idx, n, keys, tcol_idx);
  return hipGetLastError();
}

// The instantiation that stages light tiles in LDS (a.stage) and counts near successors
// (a.count_near; always counted when staging): byte registers, rows of at most 16 lanes
// (256 bytes), 4 loads in flight (the schedule allows either only there).
#define HANF_DISPATCH_STAGED(G_, EXPR)                          \
  {                                                             \
    using F = ByteRegs;                                         \
    switch (G_) {                                               \
      case 1: { constexpr int G = 1; EXPR; } break;             \
      case 2: { constexpr int G = 2; EXPR; } break;             \
      case 4: { constexpr int G = 4; EXPR; } break;             \
      case 8: { constexpr int G = 8; EXPR; } break;             \
      case 16: { constexpr int G = 16; EXPR; } break;           \
      default: return hipErrorInvalidValue;                     \
    }                                                           \
  }

hipError_t launch_union(const PassArgs &a, int u, int full, int list, hipStream_t s, hipEvent_t e0, hipEvent_t e1) {
  const int G = row_lanes(a);
  const dim3 block(kBlockThreads);
  const size_t lds = (size_t)a.lds_wave_bytes * (kBlockThreads / kWave);
  if (a.n_chunk_wgs + a.n_light_wgs == 0 || (!full && !list)) return record_empty(e0, e1, s);
  const bool st = a.stage || a.count_near;  // the instantiation that stages and counts near successors
  if (st && (a.packed || u != 4)) return hipErrorInvalidValue;
  if (full) {
    const dim3 grid((unsigned)(a.n_chunk_wgs + a.n_light_wgs));
    const int32_t list_too = list ? 1 : 0;
    hipEvent_t end = list ? nullptr : e1;
    if (st) {
      HANF_DISPATCH_STAGED(G, launch_k_lds(k_union<F, G, 4, true>, grid, block, lds, s, e0, end, a, list_too));
    } else {
      switch (u) {
        case 2:
          HANF_DISPATCH_FG(a.packed, G, launch_k_lds(k_union<F, G, 2, false>, grid, block, lds, s, e0, end, a, list_too));
          break;
        case 8:
          HANF_DISPATCH_FG(a.packed, G, launch_k_lds(k_union<F, G, 8, false>, grid, block, lds, s, e0, end, a, list_too));
          break;
        default:
          HANF_DISPATCH_FG(a.packed, G, launch_k_lds(k_union<F, G, 4, false>, grid, block, lds, s, e0, end, a, list_too));
          break;
      }
    }
  }
  if (list) {
    const int64_t units = (int64_t)a.n_chunks + a.n_tiles;
    const dim3 grid((unsigned)grid_for(units, kBlockThreads / kWave, kListWgs));
    const int32_t full_too = full ? 1 : 0;
    hipEvent_t start = full ? nullptr : e0;
    if (st) {
      HANF_DISPATCH_STAGED(G, launch_k_lds(k_union_list<F, G, 4, true>, grid, block, lds, s, start, e1, a, full_too));
    } else {
      switch (u) {
        case 2:
          HANF_DISPATCH_FG(a.packed, G,
                           launch_k_lds(k_union_list<F, G, 2, false>, grid, block, lds, s, start, e1, a, full_too));
          break;
        case 8:
          HANF_DISPATCH_FG(a.packed, G,
                           launch_k_lds(k_union_list<F, G, 8, false>, grid, block, lds, s, start, e1, a, full_too));
          break;
        default:
          HANF_DISPATCH_FG(a.packed, G,
                           launch_k_lds(k_union_list<F, G, 4, false>, grid, block, lds, s, start, e1, a, full_too));
          break;
      }
    }
  }
  return hipGetLastError();
}

hipError_t launch_finalize(const PassArgs &a, hipStream_t s, hipEvent_t e0, hipEvent_t e1) {
  if (a.n_fin_wgs == 0) return record_empty(e0, e1, s);
  const int G = row_lanes(a);
  HANF_DISPATCH_FG(a.packed, G, launch_k(k_finalize<F, G>, dim3((unsigned)a.n_fin_wgs), dim3(kBlockThreads), s, e0, e1, a));
  return hipGetLastError();
}

hipError_t launch_estimate_changed(const PassArgs &a, hipStream_t s, hipEvent_t e0, hipEvent_t e1) {
  if (!a.packed) return record_empty(e0, e1, s);  // byte rows: the union step wrote them
  const int G = row_lanes(a);
  const int64_t lanes = (int64_t)a.n * G;
  const int grid = grid_for(lanes, kBlockThreads, kLaneSweepWgs);
  HANF_DISPATCH_FG(a.packed, G, launch_k(k_estimate_changed<F, G>, dim3(grid), dim3(kBlockThreads), s, e0, e1, a, lanes));
  return hipGetLastError();
}

hipError_t launch_reduce(const PassArgs &a, int32_t mode, int32_t force, hipStream_t s, hipEvent_t e0,
                         hipEvent_t e1) {
  const dim3 grid((unsigned)a.n_reduce_wgs), block(kBlockThreads);
  switch (a.seed_log2) {
    case 0: launch_k(k_reduce_blocks<1>, grid, block, s, e0, nullptr, a, force); break;
    case 1: launch_k(k_reduce_blocks<2>, grid, block, s, e0, nullptr, a, force); break;
    case 2: launch_k(k_reduce_blocks<4>, grid, block, s, e0, nullptr, a, force); break;
    case 3: launch_k(k_reduce_blocks<8>, grid, block, s, e0, nullptr, a, force); break;
    case 4: launch_k(k_reduce_blocks<16>, grid, block, s, e0, nullptr, a, force); break;
    case 5: launch_k(k_reduce_blocks<32>, grid, block, s, e0, nullptr, a, force); break;
    default: return hipErrorInvalidValue;
  }
  if (a.batch.active && a.batch.n_comp > 0) {
    hipLaunchKernelGGL(k_reduce_comp_chunks, dim3((unsigned)a.batch.n_cchunks), dim3(kBlockThreads), 0, s, a, mode);
    hipLaunchKernelGGL(k_reduce_components, dim3(grid_for(a.batch.n_comp, kBlockThreads, 1 << 30)),
                       dim3(kBlockThreads), 0, s, a, mode);
  }
  launch_k(k_reduce_top, dim3(1), dim3(kTopThreads), s, nullptr, e1, a, mode);
  return hipGetLastError();
}

hipError_t launch_stats(const double *nt, const int32_t *T_or_null, const DevState *st, double alpha,
                        double eps, int32_t distinct, double *out, hipStream_t s) {
  hipLaunchKernelGGL(k_stats, dim3(1), dim3(64), 0, s, nt, T_or_null, st, alpha, eps, distinct, out);
  return hipGetLastError();
}

hipError_t launch_seed_summary(const PassArgs &a, int32_t n_graphs, int32_t n_seeds, double alpha, int32_t distinct,
                               SummaryRec *out, hipStream_t s) {
  hipLaunchKernelGGL(k_seed_summary, dim3(grid_for(n_graphs, 64, 1 << 30)), dim3(64), 0, s, a, n_graphs, n_seeds,
                     alpha, distinct, out);
  return hipGetLastError();
}

hipError_t launch_stats_all(const PassArgs &a, double alpha, double eps, int32_t distinct, StatsRec *out,
                            hipStream_t s) {
  hipLaunchKernelGGL(k_stats_all, dim3(grid_for(a.batch.n_comp, 64, 1 << 30)), dim3(64), 0, s, a, alpha, eps, distinct,
                     out);
  return hipGetLastError();
}

hipError_t launch_expand_local(const int32_t *graph_off, const int32_t *arc_off, const int32_t *rp_in,
                               const int32_t *ci_in, int32_t n_graphs, int32_t n_seeds, const PassArgs &a,
                               const int32_t *comp_arc_off, int32_t *rp_exp, int32_t *ci_exp, int64_t n_exp,
                               int64_t e_exp, DevState *st, hipStream_t s) {
  const int64_t top = e_exp > n_exp + 1 ? e_exp : n_exp + 1;
  hipLaunchKernelGGL(k_expand_local, dim3(grid_for(top, 256, 16384)), dim3(256), 0, s, graph_off, arc_off, rp_in, ci_in,
                     n_graphs, n_seeds, a, comp_arc_off, rp_exp, ci_exp, n_exp, e_exp, st);
  return hipGetLastError();
}

hipError_t launch_check_offsets(const int32_t *rp, const int32_t *goff, const int32_t *aoff, int32_t n_graphs,
                                DevState *st, hipStream_t s) {
  hipLaunchKernelGGL(k_check_offsets, dim3(grid_for((int64_t)n_graphs + 1, 256, 1 << 30)), dim3(256), 0, s, rp, goff,
                     aoff, n_graphs, st);
  return hipGetLastError();
}

hipError_t launch_expand(const int32_t *graph_off, const int32_t *rp_in, const int32_t *ci_in,
                         int32_t n_seeds, const PassArgs &a, const int32_t *comp_arc_off, int32_t *rp_exp,
                         int32_t *ci_exp, int64_t n_exp, int64_t e_exp, DevState *st, hipStream_t s) {
  const int64_t top = e_exp > n_exp + 1 ? e_exp : n_exp + 1;
  hipLaunchKernelGGL(k_expand, dim3(grid_for(top, 256, 16384)), dim3(256), 0, s, graph_off, rp_in, ci_in, n_seeds,
                     a, comp_arc_off, rp_exp, ci_exp, n_exp, e_exp, st);
  return hipGetLastError();
}

hipError_t launch_check_registers(const uint8_t *regs, int64_t bytes, DevState *st, hipStream_t s) {
  const int64_t nw = bytes / 4;
  hipLaunchKernelGGL(k_check_registers, dim3(grid_for(nw, 256, 8192)), dim3(256), 0, s,
                     reinterpret_cast<const uint32_t *>(regs), nw, st);
  return hipGetLastError();
}

hipError_t launch_bytemax_words(const uint32_t *x, const uint32_t *y, uint32_t *out, int64_t count,
                                hipStream_t s) {
  hipLaunchKernelGGL(k_bytemax_words, dim3(grid_for(count, 256, 8192)), dim3(256), 0, s, x, y, out, count);
  return hipGetLastError();
}

hipError_t launch_gathermax_lanes(const uint4 *x, int32_t k, int32_t from_first, uint4 *out, int64_t count,
                                 hipStream_t s) {
  hipLaunchKernelGGL(k_gathermax_lanes, dim3(grid_for(count, 256, 8192)), dim3(256), 0, s, x, k, from_first, out, count);
  return hipGetLastError();
}

hipError_t launch_max5_groups(const uint8_t *x, const uint8_t *y, uint8_t *out, int64_t groups, hipStream_t s) {
  hipLaunchKernelGGL(k_max5_groups, dim3(grid_for(groups, 256, 8192)), dim3(256), 0, s, x, y, out, groups);
  return hipGetLastError();
}

hipError_t launch_unpack5(const uint8_t *packed, uint8_t *out, int64_t groups, hipStream_t s) {
  if (groups == 0) return hipSuccess;
  hipLaunchKernelGGL(k_unpack5, dim3(grid_for(groups, 256, 8192)), dim3(256), 0, s, packed, out, groups);
  return hipGetLastError();
}

hipError_t launch_unpack5_rows(const uint8_t *src, int64_t row_stride, int32_t gpr, int64_t rows, uint8_t *out,
                               hipStream_t s) {
  if (rows == 0) return hipSuccess;
  hipLaunchKernelGGL(k_unpack5_rows, dim3(grid_for(rows * gpr, 256, 8192)), dim3(256), 0, s, src, row_stride, gpr,
                     rows, out);
  return hipGetLastError();
}

hipError_t launch_pack5(const uint8_t *in, uint8_t *packed, int64_t groups, hipStream_t s) {
  if (groups == 0) return hipSuccess;
  hipLaunchKernelGGL(k_pack5, dim3(grid_for(groups, 256, 8192)), dim3(256), 0, s, in, packed, groups);
  return hipGetLastError();
}

}  // namespace hanf
