// Device helpers shared by the counting kernels: pair/triple existence
// tests (fill-in, Section 4.3 Fig. 3b), bit-row masks, wavefront scans and
// reductions, LDS class-counter helpers and the Philox4x64-10 generator.
#pragma once

#include "hm_internal.h"

namespace hm {

constexpr int kThreads = 256;
constexpr int kWavesPerBlock = kThreads / kWave;
// pattern bits of the pairs among 4 local nodes: masks 3,5,6,9,10,12 -> bits 0,1,2,4,5,7
constexpr uint32_t kPairBits4 = (1u << 0) | (1u << 1) | (1u << 2) | (1u << 4) | (1u << 5) | (1u << 7);
constexpr uint32_t kPairBits3 = 0x7u;

__device__ inline bool has2(const Set64& s, uint32_t u, uint32_t v) {
  return set64_has(s, u < v ? key2(u, v) : key2(v, u));
}
__device__ inline void sort3(uint32_t& a, uint32_t& b, uint32_t& c) {
  uint32_t t;
  if (a > b) { t = a; a = b; b = t; }
  if (b > c) { t = b; b = c; c = t; }
  if (a > b) { t = a; a = b; b = t; }
}
__device__ inline bool has3(const Set128& s, uint32_t a, uint32_t b, uint32_t c) {
  sort3(a, b, c);
  return set128_has(s, key3(a, b, c));
}
// Membership tests split in two, so that the first probes of several keys
// are loaded together: *_start loads the key's home slot, *_end finishes the
// probe (further loads only after a collision).
struct Probe64 {
  unsigned long long key, pos, v;
};
struct Probe128 {
  Key128 key;
  unsigned long long pos;
  ulonglong2 v;
};
__device__ inline Probe64 probe2_start(const Set64& s, uint32_t u, uint32_t w) {
  Probe64 p;
  p.key = u < w ? key2(u, w) : key2(w, u);
  p.pos = mix64(p.key) & s.mask;
  p.v = s.slot[p.pos];
  return p;
}
__device__ inline bool probe64_end(const Set64& s, Probe64 p) {
  while (true) {
    if (p.v == p.key) return true;
    if (p.v == kEmpty64) return false;
    p.pos = (p.pos + 1) & s.mask;
    p.v = s.slot[p.pos];
  }
}
__device__ inline Probe128 probe128_start(const Set128& s, Key128 key) {
  Probe128 p;
  p.key = key;
  p.pos = hash128(key) & s.mask;
  p.v = *reinterpret_cast<const ulonglong2*>(s.slot + 2 * p.pos);
  return p;
}
__device__ inline Probe128 probe3_start(const Set128& s, uint32_t a, uint32_t b, uint32_t c) {
  sort3(a, b, c);
  return probe128_start(s, key3(a, b, c));
}
__device__ inline bool probe128_end(const Set128& s, Probe128 p) {
  while (true) {
    if (p.v.x == p.key.hi && p.v.y == p.key.lo) return true;
    if (p.v.x == kEmpty64) return false;
    p.pos = (p.pos + 1) & s.mask;
    p.v = *reinterpret_cast<const ulonglong2*>(s.slot + 2 * p.pos);
  }
}
// lexicographic comparison of ascending triples
__device__ inline bool tri_less(uint32_t a0, uint32_t a1, uint32_t a2, uint32_t b0, uint32_t b1, uint32_t b2) {
  if (a0 != b0) return a0 < b0;
  if (a1 != b1) return a1 < b1;
  return a2 < b2;
}
// The members of a sorted 3- or 4-node hyperedge m other than m[j], 16 bits
// each in ascending order (node ids below 2^16: graphs with bit rows), kept
// beside incidence entries so that a walk over a node's list needs no second
// load for the members.
static_assert(kBitsetMaxNodes <= 65536, "packed members need node ids below 2^16");
__device__ inline uint32_t others3(const uint32_t* m, int j) {
  const uint32_t x = m[j == 0 ? 1 : 0], y = m[j == 2 ? 1 : 2];
  return x | (y << 16);
}
__device__ inline unsigned long long others4(const uint32_t* m, int j) {
  unsigned long long o = 0;
  int s = 0;
  for (int q = 0; q < 4; ++q)
    if (q != j) {
      o |= (unsigned long long)m[q] << s;
      s += 16;
    }
  return o;
}

__device__ inline bool bit_of(const uint32_t* bits, uint32_t words, uint32_t u, uint32_t v) {
  return (bits[uint64_t(u) * words + (v >> 5)] >> (v & 31)) & 1u;
}
// bits of word w whose node index is greater than y
__device__ inline uint32_t mask_gt(uint32_t y, uint32_t w) {
  const uint32_t lo = w << 5;
  if (y < lo) return ~0u;
  const uint32_t d = y - lo;
  if (d >= 31) return 0u;
  return ~0u << (d + 1);
}
// bits of word w whose node index is below n
__device__ inline uint32_t mask_below(uint32_t n, uint32_t w) {
  const uint32_t lo = w << 5;
  if (lo + 32 <= n) return ~0u;
  if (lo >= n) return 0u;
  return (1u << (n - lo)) - 1u;
}
// first position in the ascending row [p, e) whose value is greater than x
__device__ inline uint32_t upper_bound(const uint32_t* adj, uint32_t p, uint32_t e, uint32_t x) {
  while (p < e) {
    uint32_t m = p + ((e - p) >> 1);
    if (adj[m] <= x) p = m + 1; else e = m;
  }
  return p;
}
// A value every active lane holds alike, moved to a scalar register.
__device__ __forceinline__ uint32_t uniform_u32(uint32_t x) { return uint32_t(__builtin_amdgcn_readfirstlane(int(x))); }
__device__ __forceinline__ uint64_t uniform_u64(uint64_t x) {
  return (uint64_t(uniform_u32(uint32_t(x >> 32))) << 32) | uniform_u32(uint32_t(x));
}

// Wavefront sums with data-parallel-primitive moves (no LDS round trips):
// shifts right by 1, 2, 4 and 8 lanes within each row of 16 leave a row's
// total in its last lane; the broadcasts of lane 15 into rows 1 and 3 and of
// lane 31 into rows 2 and 3 then leave the wavefront's total in lane 63,
// which is read into a scalar.  Lanes shifted in from outside a row read 0.
// Every lane of the wavefront must be active.
namespace dpp {
constexpr int kRowShr1 = 0x111, kRowShr2 = 0x112, kRowShr4 = 0x114, kRowShr8 = 0x118;
constexpr int kRowBcast15 = 0x142, kRowBcast31 = 0x143;
template <int CTRL, int ROWS>
__device__ __forceinline__ uint32_t mov(uint32_t x) {
  return uint32_t(__builtin_amdgcn_update_dpp(0, int(x), CTRL, ROWS, 0xF, true));
}
}  // namespace dpp

__device__ inline uint32_t wave_sum_u32(uint32_t x) {
  x += dpp::mov<dpp::kRowShr1, 0xF>(x);
  x += dpp::mov<dpp::kRowShr2, 0xF>(x);
  x += dpp::mov<dpp::kRowShr4, 0xF>(x);
  x += dpp::mov<dpp::kRowShr8, 0xF>(x);
  x += dpp::mov<dpp::kRowBcast15, 0xA>(x);
  x += dpp::mov<dpp::kRowBcast31, 0xC>(x);
  return uint32_t(__builtin_amdgcn_readlane(int(x), kWave - 1));
}

template <int CTRL, int ROWS>
__device__ __forceinline__ unsigned long long dpp_add64(unsigned long long v) {
  const uint32_t lo = dpp::mov<CTRL, ROWS>(uint32_t(v)), hi = dpp::mov<CTRL, ROWS>(uint32_t(v >> 32));
  return v + ((unsigned long long)hi << 32 | lo);
}

__device__ inline unsigned long long wave_sum(unsigned long long v) {
  v = dpp_add64<dpp::kRowShr1, 0xF>(v);
  v = dpp_add64<dpp::kRowShr2, 0xF>(v);
  v = dpp_add64<dpp::kRowShr4, 0xF>(v);
  v = dpp_add64<dpp::kRowShr8, 0xF>(v);
  v = dpp_add64<dpp::kRowBcast15, 0xA>(v);
  v = dpp_add64<dpp::kRowBcast31, 0xC>(v);
  const uint32_t lo = uint32_t(__builtin_amdgcn_readlane(int(uint32_t(v)), kWave - 1));
  const uint32_t hi = uint32_t(__builtin_amdgcn_readlane(int(uint32_t(v >> 32)), kWave - 1));
  return (unsigned long long)hi << 32 | lo;
}

__device__ inline void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
}

// Inclusive prefix sums over the wavefront by the same moves as the sums:
// after the shifts within rows each lane holds its row's prefix, the
// broadcasts then add the totals of the rows before it.  Every lane of the
// wavefront must be active.
__device__ inline uint32_t wave_inclusive_scan(uint32_t x) {
  x += dpp::mov<dpp::kRowShr1, 0xF>(x);
  x += dpp::mov<dpp::kRowShr2, 0xF>(x);
  x += dpp::mov<dpp::kRowShr4, 0xF>(x);
  x += dpp::mov<dpp::kRowShr8, 0xF>(x);
  x += dpp::mov<dpp::kRowBcast15, 0xA>(x);
  x += dpp::mov<dpp::kRowBcast31, 0xC>(x);
  return x;
}
__device__ inline unsigned long long wave_inclusive_scan(unsigned long long v) {
  v = dpp_add64<dpp::kRowShr1, 0xF>(v);
  v = dpp_add64<dpp::kRowShr2, 0xF>(v);
  v = dpp_add64<dpp::kRowShr4, 0xF>(v);
  v = dpp_add64<dpp::kRowShr8, 0xF>(v);
  v = dpp_add64<dpp::kRowBcast15, 0xA>(v);
  v = dpp_add64<dpp::kRowBcast31, 0xC>(v);
  return v;
}

__device__ inline uint32_t wave_exclusive_scan(uint32_t v, uint32_t* total) {
  const uint32_t x = wave_inclusive_scan(v);
  *total = uint32_t(__builtin_amdgcn_readlane(int(x), kWave - 1));
  return x - v;
}

__device__ inline void load_lut(uint8_t* lut, const uint8_t* g, int n) {
  for (int i = threadIdx.x; i < n; i += blockDim.x) lut[i] = g[i];
}

// This workgroup's copy of a histogram kept in kHistCopies copies.
__device__ inline unsigned long long* hist_copy(unsigned long long* hist, uint32_t stride) {
  return hist + uint64_t(blockIdx.x & (kHistCopies - 1)) * stride;
}

__device__ inline void flush(unsigned long long* lds, unsigned long long* out, int n) {
  for (int i = threadIdx.x; i < n; i += blockDim.x)
    if (lds[i]) atomicAdd(out + i, lds[i]);
}

__device__ inline uint32_t pair_bit(const Set64& hs2, const uint32_t* bits, uint32_t W, uint32_t u, uint32_t v) {
  return bits ? ((bits[uint64_t(u) * W + (v >> 5)] >> (v & 31)) & 1u) : uint32_t(has2(hs2, u, v));
}


// Philox4x64-10 (Salmon et al., SC'11): ten rounds of two 64x64->128-bit
// multiplications with the round keys bumped by the Weyl constants.
struct Philox4 {
  unsigned long long v[4];
};
__device__ inline Philox4 philox4x64_10(unsigned long long c0, unsigned long long c1, unsigned long long c2,
                                        unsigned long long c3, unsigned long long k0, unsigned long long k1) {
  const unsigned long long M0 = 0xD2E7470EE14C6C93ull, M1 = 0xCA5A826395121157ull;
  const unsigned long long W0 = 0x9E3779B97F4A7C15ull, W1 = 0xBB67AE8584CAA73Bull;
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const unsigned long long hi0 = __umul64hi(M0, c0), lo0 = M0 * c0;
    const unsigned long long hi1 = __umul64hi(M1, c2), lo1 = M1 * c2;
    const unsigned long long n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
    c0 = n0;
    c1 = lo1;
    c2 = n2;
    c3 = lo0;
    k0 += W0;
    k1 += W1;
  }
  return Philox4{{c0, c1, c2, c3}};
}
// a value in [0, n) from a uniform 64-bit word: the high word of word * n
__device__ inline unsigned long long bounded64(unsigned long long word, unsigned long long n) {
  return __umul64hi(word, n);
}
constexpr unsigned long long kDomainSample = 1ull;
constexpr unsigned long long kDomainNull = 2ull;
constexpr unsigned long long kDomainProposal = 3ull;

}  // namespace hm
