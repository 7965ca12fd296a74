// Device-side building blocks for the gfx950 graph builder: key arithmetic on
// 2-bit-packed DNA, canonical forms, edge decoding, digit extraction and the
// wave64 / workgroup scan primitives the kernels share.
//
// Key encoding (Sec. 2 order A < C < G < T): a string of L bases is the integer
// sum c_j 4^(L-1-j) with A=0 C=1 G=2 T=3, so integer order is string order.
// Keys of up to 32 bases are uint64_t; up to 64 bases unsigned __int128.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

typedef unsigned __int128 u128;

namespace dbg {

template <typename K> struct KeyTraits;
template <> struct KeyTraits<uint64_t> { static constexpr int bits = 64; };
template <> struct KeyTraits<u128> { static constexpr int bits = 128; };

template <typename K> __device__ __forceinline__ K all_ones() { return ~K(0); }

// x >> s for 0 <= s <= bits (s == bits gives 0).
template <typename K> __device__ __forceinline__ K shr(K x, int s) {
  return s >= KeyTraits<K>::bits ? K(0) : (x >> s);
}
template <typename K> __device__ __forceinline__ K shl(K x, int s) {
  return s >= KeyTraits<K>::bits ? K(0) : (x << s);
}
// mask of the low n bits, 0 <= n <= bits.
template <typename K> __device__ __forceinline__ K low_mask(int n) {
  return n >= KeyTraits<K>::bits ? all_ones<K>() : ((K(1) << n) - K(1));
}

// Reverse the order of the 2-bit groups of a 64-bit word.
__device__ __forceinline__ uint64_t reverse_pairs64(uint64_t x) {
  const uint64_t r = __builtin_bitreverse64(x);
  return ((r >> 1) & 0x5555555555555555ull) | ((r & 0x5555555555555555ull) << 1);
}

// Reverse complement of a key of len bases (Sec. 2): complement every base
// (c -> 3 - c, i.e. bitwise not of the 2-bit code) and reverse their order.
__device__ __forceinline__ uint64_t revcomp(uint64_t x, int len) {
  return reverse_pairs64(~x) >> (64 - 2 * len);
}
__device__ __forceinline__ u128 revcomp(u128 x, int len) {
  const uint64_t lo = (uint64_t)x, hi = (uint64_t)(x >> 64);
  const u128 r = ((u128)reverse_pairs64(~lo) << 64) | (u128)reverse_pairs64(~hi);
  return shr<u128>(r, 128 - 2 * len);
}

// Canonical k-mer (Sec. 2): the smaller of the key and its reverse complement.
template <typename K> __device__ __forceinline__ K canonical(K x, int len) {
  const K r = revcomp(x, len);
  return r < x ? r : x;
}

// Radix digit `level` counted from the most significant end of a key with `b`
// significant bits: bits [max(0, b - 8(level+1)), b - 8 level).  Only valid while
// b - 8 level > 0.
template <typename K> __device__ __forceinline__ uint32_t msd_digit(K x, int b, int level) {
  const int hi = b - 8 * level;
  const int lo = hi - 8;
  if (lo >= 0) return (uint32_t)(shr<K>(x, lo)) & 0xffu;
  return (uint32_t)x & ((1u << hi) - 1u);
}

// Extract `len` bases starting at stream position p from the MSB-first packed
// stream (base q sits in bits [63 - 2(q mod 32), 62 - 2(q mod 32)] of word q/32).
__device__ __forceinline__ uint64_t load_word(const uint64_t *__restrict__ w, uint64_t i,
                                              uint64_t n_words) {
  return i < n_words ? w[i] : 0ull;
}
__device__ __forceinline__ uint64_t extract_bases(const uint64_t *__restrict__ w, uint64_t n_words,
                                                  uint64_t p, int len, uint64_t) {
  const uint64_t wi = p >> 5;
  const int o = (int)(p & 31) * 2;
  const uint64_t w0 = load_word(w, wi, n_words);
  const uint64_t w1 = o ? load_word(w, wi + 1, n_words) : 0ull;
  const uint64_t v = o ? ((w0 << o) | (w1 >> (64 - o))) : w0;
  return len == 32 ? v : (v >> (64 - 2 * len));
}
__device__ __forceinline__ u128 extract_bases(const uint64_t *__restrict__ w, uint64_t n_words,
                                              uint64_t p, int len, u128) {
  const uint64_t wi = p >> 5;
  const int o = (int)(p & 31) * 2;
  const uint64_t w0 = load_word(w, wi, n_words);
  const uint64_t w1 = load_word(w, wi + 1, n_words);
  const uint64_t w2 = o ? load_word(w, wi + 2, n_words) : 0ull;
  const uint64_t hi = o ? ((w0 << o) | (w1 >> (64 - o))) : w0;
  const uint64_t lo = o ? ((w1 << o) | (w2 >> (64 - o))) : w1;
  const u128 v = ((u128)hi << 64) | (u128)lo;
  return shr<u128>(v, 128 - 2 * len);
}
__device__ __forceinline__ uint32_t base_at(const uint64_t *__restrict__ w, uint64_t q) {
  return (uint32_t)(w[q >> 5] >> (62 - 2 * (int)(q & 31))) & 3u;
}

// Edge record of a canonical (k+1)-mer z (STEP-1 of Sec. 3 in closed form):
// x = first k bases, y = last k bases; strand s = 0 when the k-mer is its
// canonical form ('+'), 1 otherwise.  If x^ < y^ the record is (x^, y^, s_x, s_y);
// if x^ > y^ it is (y^, x^, not s_y, not s_x); if x^ = y^ the record and its
// reversal name one edge and the smaller orientation pair is kept.
template <typename K>
__device__ __forceinline__ void decode_edge(K z, int k, K *u, K *v, uint32_t *orient) {
  const K x = z >> 2;
  const K y = z & low_mask<K>(2 * k);
  const K rx = revcomp(x, k), ry = revcomp(y, k);
  const uint32_t sx = rx < x ? 1u : 0u, sy = ry < y ? 1u : 0u;
  const K cx = sx ? rx : x, cy = sy ? ry : y;
  uint32_t o1, o2;
  if (cx < cy) {
    *u = cx; *v = cy; o1 = sx; o2 = sy;
  } else if (cy < cx) {
    *u = cy; *v = cx; o1 = 1u - sy; o2 = 1u - sx;
  } else {
    *u = cx; *v = cy;
    const uint32_t a = (sx << 1) | sy, b = ((1u - sy) << 1) | (1u - sx);
    const uint32_t m = a < b ? a : b;
    o1 = m >> 1; o2 = m & 1u;
  }
  *orient = (o1 << 1) | o2;
}

// ---------------------------------------------------------------------------
// wave64 and workgroup primitives.

__device__ __forceinline__ uint32_t lane_id() { return __lane_id(); }
__device__ __forceinline__ uint64_t lanemask_lt() {
  const uint32_t l = lane_id();
  return l ? (~0ull >> (64 - l)) : 0ull;
}

// Lanes of the (fully active) wave holding the same 8-bit digit as this lane:
// one ballot per digit bit, keeping the lanes that agree on that bit.
__device__ __forceinline__ uint64_t match_digit8(uint32_t d) {
  uint64_t m = ~0ull;
#pragma unroll
  for (int b = 0; b < 8; ++b) {
    const bool bit = (d >> b) & 1u;
    const uint64_t bal = __ballot(bit);
    m &= bit ? bal : ~bal;
  }
  return m;
}

// Wave64 scans and reductions through DPP lane moves inside rows of 16 lanes
// (row_shr), then the three row totals read out to scalars; no LDS crossbar
// traffic.  Every lane of the wave must be active.  `old` fills the lanes a
// shift leaves without a source: the identity of the operation.
template <int CTRL, uint32_t OLD> __device__ __forceinline__ uint32_t dpp_u32(uint32_t v) {
  return (uint32_t)__builtin_amdgcn_update_dpp((int)OLD, (int)v, CTRL, 0xf, 0xf, false);
}
template <int CTRL, uint32_t OLD, typename T> __device__ __forceinline__ T dpp_move(T v) {
  static_assert(sizeof(T) == 4 || sizeof(T) == 8, "32- or 64-bit lanes");
  if constexpr (sizeof(T) == 4) {
    return (T)dpp_u32<CTRL, OLD>((uint32_t)v);
  } else {
    const uint32_t lo = dpp_u32<CTRL, OLD>((uint32_t)v);
    const uint32_t hi = dpp_u32<CTRL, OLD>((uint32_t)((uint64_t)v >> 32));
    return (T)(((uint64_t)hi << 32) | lo);
  }
}
template <typename T> __device__ __forceinline__ T read_lane(T v, int l) {
  if constexpr (sizeof(T) == 4) {
    return (T)__builtin_amdgcn_readlane((uint32_t)v, l);
  } else {
    const uint32_t lo = __builtin_amdgcn_readlane((uint32_t)v, l);
    const uint32_t hi = __builtin_amdgcn_readlane((uint32_t)((uint64_t)v >> 32), l);
    return (T)(((uint64_t)hi << 32) | lo);
  }
}
constexpr int DPP_ROW_SHR1 = 0x111, DPP_ROW_SHR2 = 0x112, DPP_ROW_SHR4 = 0x114,
              DPP_ROW_SHR8 = 0x118;

// Inclusive scan across a wave64.
template <typename T> __device__ __forceinline__ T wave_inclusive_scan(T v) {
  v += dpp_move<DPP_ROW_SHR1, 0u>(v);
  v += dpp_move<DPP_ROW_SHR2, 0u>(v);
  v += dpp_move<DPP_ROW_SHR4, 0u>(v);
  v += dpp_move<DPP_ROW_SHR8, 0u>(v);
  const T r0 = read_lane(v, 15), r1 = read_lane(v, 31), r2 = read_lane(v, 47);
  const uint32_t l = lane_id();
  const T add = (l >= 16 ? r0 : T(0)) + (l >= 32 ? r1 : T(0)) + (l >= 48 ? r2 : T(0));
  return v + add;
}
// Reductions whose result every lane receives.
template <typename T> __device__ __forceinline__ T wave_sum(T v) {
  v += dpp_move<DPP_ROW_SHR1, 0u>(v);
  v += dpp_move<DPP_ROW_SHR2, 0u>(v);
  v += dpp_move<DPP_ROW_SHR4, 0u>(v);
  v += dpp_move<DPP_ROW_SHR8, 0u>(v);
  return read_lane(v, 15) + read_lane(v, 31) + read_lane(v, 47) + read_lane(v, 63);
}
template <typename T> __device__ __forceinline__ T wave_or(T v) {
  v |= dpp_move<DPP_ROW_SHR1, 0u>(v);
  v |= dpp_move<DPP_ROW_SHR2, 0u>(v);
  v |= dpp_move<DPP_ROW_SHR4, 0u>(v);
  v |= dpp_move<DPP_ROW_SHR8, 0u>(v);
  return read_lane(v, 15) | read_lane(v, 31) | read_lane(v, 47) | read_lane(v, 63);
}
template <typename T> __device__ __forceinline__ T wave_and(T v) {
  v &= dpp_move<DPP_ROW_SHR1, 0xffffffffu>(v);
  v &= dpp_move<DPP_ROW_SHR2, 0xffffffffu>(v);
  v &= dpp_move<DPP_ROW_SHR4, 0xffffffffu>(v);
  v &= dpp_move<DPP_ROW_SHR8, 0xffffffffu>(v);
  return read_lane(v, 15) & read_lane(v, 31) & read_lane(v, 47) & read_lane(v, 63);
}

// Exclusive scan of one value per thread over a workgroup of NT threads
// (NT a multiple of 64, at most 1024).  `wsum` is LDS scratch of NT/64 entries.
// Returns the exclusive prefix; *total receives the sum.  Contains barriers:
// every thread of the workgroup must call it.
template <int NT, typename T>
__device__ __forceinline__ T block_exclusive_scan(T v, T *wsum, T *total) {
  constexpr int NW = NT / 64;
  const uint32_t w = threadIdx.x >> 6, l = lane_id();
  const T inc = wave_inclusive_scan(v);
  if (l == 63) wsum[w] = inc;
  __syncthreads();
  if (w == 0) {
    T s = l < (uint32_t)NW ? wsum[l] : T(0);
    const T si = wave_inclusive_scan(s);
    if (l < (uint32_t)NW) wsum[l] = si - s;
    if (l == NW - 1) wsum[NW] = si;
  }
  __syncthreads();
  const T r = wsum[w] + inc - v;
  *total = wsum[NW];
  __syncthreads();
  return r;
}

}  // namespace dbg
