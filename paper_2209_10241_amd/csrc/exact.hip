// Exact counting of order-3 and order-4 higher-order motifs (Algorithms 2
// and 3, Section 4.2) on gfx950.
//
// Algorithm 3 finds every connected 4-node set once by three generators and a
// global "visited" set of node sets.  Here the visited set is replaced by
// ownership rules that decide, from the set alone, which generator counts it,
// so that every generator instance runs independently:
//   (a) a 4-node hyperedge counts its own node set;
//   (b) a set that is not a 4-node hyperedge but holds a 3-node hyperedge is
//       counted by its smallest 3-node hyperedge e (lexicographic order of the
//       ascending tuples), from the single generator instance (e, v) whose
//       witness -- the hyperedge that joins v to e -- comes first among
//       {a,v}, {b,v}, {c,v}, {a,b,v}, {a,c,v}, {b,c,v} for e = {a<b<c};
//   (c) a set whose sub-hypergraph holds only pairs is a connected 4-node set
//       of the pairwise graph G2 that none of (a), (b) counted.  The pairwise
//       graph's connected 4-node sets are counted per induced graph shape by
//       bit-parallel neighbour intersection (each set from its smallest node),
//       and the shapes of the G2-connected sets already counted in (a) and (b)
//       are subtracted.
// Order 3 is the same with (a) = each 3-node hyperedge and (c) = wedges and
// triangles of G2.  Every counted set is classified by fill-in (existence of
// each sub-hyperedge, Section 4.3 Fig. 3b) and one read of the pattern->class
// table (Section 4.3 Fig. 3a) held in LDS; per-class counters live in LDS and
// are flushed to device memory with one atomic per class per workgroup.
#include <vector>

#include "hm_b4.h"

namespace hm {
namespace {

// histogram regions (256 counters each) in hm_graph::hist
constexpr int kMain = 0;    // classes counted by (a) and (b)
constexpr int kSub = 256;   // G2 shape of G2-connected sets counted by (a) and (b)
constexpr int kG2 = 512;    // G2 shape counts of all connected 4-node (3-node) sets of G2

// ---------------------------------------------------------------- order 4
// (a): one thread per 4-node hyperedge; local positions a,b,c,d = 0..3.
__global__ void __launch_bounds__(kThreads) k_case_a4(const uint32_t* __restrict__ e4, uint64_t n4, Set64 hs2,
                                                      Set128 hs3, const uint32_t* __restrict__ bits, uint32_t W,
                                                      const uint8_t* __restrict__ lut_g,
                                                      unsigned long long* __restrict__ hist) {
  __shared__ uint8_t lut[2048];
  __shared__ unsigned long long h_main[256], h_sub[256];
  load_lut(lut, lut_g, 2048);
  h_main[threadIdx.x] = 0;
  h_sub[threadIdx.x] = 0;
  __syncthreads();
  for (uint64_t i = uint64_t(blockIdx.x) * kThreads + threadIdx.x; i < n4; i += uint64_t(gridDim.x) * kThreads) {
    const uint32_t a = e4[4 * i], b = e4[4 * i + 1], c = e4[4 * i + 2], d = e4[4 * i + 3];
    uint32_t p = 1u << 10;
    p |= pair_bit(hs2, bits, W, a, b) << 0;
    p |= pair_bit(hs2, bits, W, a, c) << 1;
    p |= pair_bit(hs2, bits, W, b, c) << 2;
    p |= uint32_t(set128_has(hs3, key3(a, b, c))) << 3;
    p |= pair_bit(hs2, bits, W, a, d) << 4;
    p |= pair_bit(hs2, bits, W, b, d) << 5;
    p |= uint32_t(set128_has(hs3, key3(a, b, d))) << 6;
    p |= pair_bit(hs2, bits, W, c, d) << 7;
    p |= uint32_t(set128_has(hs3, key3(a, c, d))) << 8;
    p |= uint32_t(set128_has(hs3, key3(b, c, d))) << 9;
    atomicAdd(&h_main[lut[p]], 1ull);
    const uint8_t g = lut[p & kPairBits4];
    if (g != 0xFF) atomicAdd(&h_sub[g], 1ull);
  }
  __syncthreads();
  flush(h_main, hist + kMain, 256);
  flush(h_sub, hist + kSub, 256);
}

// (b): one wavefront per 3-node hyperedge; see b4_edge_hash / b4_edge_bits.
__global__ void __launch_bounds__(kThreads) k_case_b4(
    const uint32_t* __restrict__ e3, uint64_t n3, const uint32_t* __restrict__ g2_off,
    const uint32_t* __restrict__ g2_adj, const uint32_t* __restrict__ i3_off, const uint32_t* __restrict__ i3_idx,
    Set64 hs2, Set128 hs3, Set128 hs4, const uint8_t* __restrict__ lut_g, unsigned long long* __restrict__ hist) {
  __shared__ uint8_t lut[2048];
  __shared__ unsigned long long h_main[256], h_sub[256];
  load_lut(lut, lut_g, 2048);
  h_main[threadIdx.x] = 0;
  h_sub[threadIdx.x] = 0;
  __syncthreads();
  const uint64_t wave = uint64_t(blockIdx.x) * kWavesPerBlock + threadIdx.x / kWave;
  const uint64_t n_waves = uint64_t(gridDim.x) * kWavesPerBlock;
  for (uint64_t i = wave; i < n3; i += n_waves)
    b4_edge_hash<true>(e3[3 * i], e3[3 * i + 1], e3[3 * i + 2], e3, g2_off, g2_adj, i3_off, i3_idx, hs2, hs3, hs4,
                       lut, h_main, h_sub);
  __syncthreads();
  flush(h_main, hist + kMain, 256);
  flush(h_sub, hist + kSub, 256);
}

__global__ void __launch_bounds__(kThreads) k_case_b4_bits(
    const uint32_t* __restrict__ e3, uint64_t n3, const uint32_t* __restrict__ e4,
    const uint32_t* __restrict__ i3_off, const uint32_t* __restrict__ i3_idx, const uint32_t* __restrict__ i4_off,
    const uint32_t* __restrict__ i4_idx, const uint32_t* __restrict__ bits, uint32_t W,
    const uint8_t* __restrict__ lut_g, unsigned long long* __restrict__ hist) {
  __shared__ uint8_t lut[2048];
  __shared__ unsigned long long h_main[256], h_sub[256];
  __shared__ B4Scratch scratch[kWavesPerBlock];
  load_lut(lut, lut_g, 2048);
  h_main[threadIdx.x] = 0;
  h_sub[threadIdx.x] = 0;
  __syncthreads();
  const int wv = threadIdx.x / kWave;
  const uint64_t wave = uint64_t(blockIdx.x) * kWavesPerBlock + wv;
  const uint64_t n_waves = uint64_t(gridDim.x) * kWavesPerBlock;
  for (uint64_t i = wave; i < n3; i += n_waves)
    b4_edge_bits<true>(e3[3 * i], e3[3 * i + 1], e3[3 * i + 2], e3, e4, i3_off, i3_idx, i4_off, i4_idx, bits, W,
                       scratch[wv], lut, h_main, h_sub);
  __syncthreads();
  flush(h_main, hist + kMain, 256);
  flush(h_sub, hist + kSub, 256);
}

// (c) with adjacency bit rows: one wavefront per pair {r<x} of G2, r the
// smallest node of the counted sets.  Shapes, with A = N(r) n V':
//   |A| = 3: {r,x,y,z}, x<y<z all neighbours of r
//   |A| = 2: x<y neighbours of r, z > r not a neighbour of r, adjacent to x or y
//   |A| = 1: x the only neighbour of r; y,z > r non-neighbours of r with
//            {x,y,z} connected: y<z both adjacent to x, or y~x, z~y, z!~x.
// A row has W words.  With W <= 64 the wavefront is split into 64/W groups of
// W lanes, lane (g, w) owning word w of every y that group g takes, so the
// words of r and x and the masks that depend only on r are loaded once per
// pair; wider rows loop over words.  Each word contributes popcounts of the
// candidate z it holds, split by the adjacency of z to x and y.
__device__ inline void c4_word(uint32_t Nr, uint32_t Nx, uint32_t Ny, uint32_t gy, uint32_t wr, bool xy,
                               unsigned long long (&t3_0)[4], unsigned long long (&t3_1)[4],
                               unsigned long long (&t2_0)[3], unsigned long long (&t2_1)[3]) {
  const uint32_t z3 = Nr & gy;
  const uint32_t z3x = z3 & Nx, z3n = z3 & ~Nx;
  const uint32_t c11 = __popc(z3x & Ny), c10 = __popc(z3x & ~Ny), c01 = __popc(z3n & Ny), c00 = __popc(z3n & ~Ny);
  const uint32_t z2 = wr & (Nx | Ny);
  const uint32_t b2 = __popc(z2 & Nx & Ny), bx = __popc(z2 & Nx & ~Ny), by = __popc(z2 & ~Nx & Ny);
  if (xy) {
    t3_1[3] += c11; t3_1[2] += c10; t3_1[1] += c01; t3_1[0] += c00;
    t2_1[0] += b2; t2_1[1] += bx; t2_1[2] += by;
  } else {
    t3_0[3] += c11; t3_0[2] += c10; t3_0[1] += c01; t3_0[0] += c00;
    t2_0[0] += b2; t2_0[1] += bx; t2_0[2] += by;
  }
}

__global__ void __launch_bounds__(kThreads) k_case_c4_bits(
    const uint32_t* __restrict__ e2, uint64_t n2, const uint32_t* __restrict__ g2_off,
    const uint32_t* __restrict__ g2_adj, const uint32_t* __restrict__ bits, uint32_t W, uint32_t N,
    const uint8_t* __restrict__ lut_g, unsigned long long* __restrict__ hist) {
  __shared__ uint8_t lut[2048];
  __shared__ unsigned long long h_g2[256];
  __shared__ uint32_t ylist[kWavesPerBlock][kWave];
  load_lut(lut, lut_g, 2048);
  h_g2[threadIdx.x] = 0;
  __syncthreads();
  unsigned long long t3_0[4] = {0, 0, 0, 0}, t3_1[4] = {0, 0, 0, 0};
  unsigned long long t2_0[3] = {0, 0, 0}, t2_1[3] = {0, 0, 0};
  unsigned long long paw = 0, star = 0, path = 0;
  const int lane = threadIdx.x & (kWave - 1);
  const int wv = threadIdx.x / kWave;
  uint32_t* ys = ylist[wv];
  const uint64_t wave = uint64_t(blockIdx.x) * kWavesPerBlock + wv;
  const uint64_t n_waves = uint64_t(gridDim.x) * kWavesPerBlock;
  const bool grouped = W <= uint32_t(kWave);
  const uint32_t G = grouped ? uint32_t(kWave) / W : 1u;     // y's in flight per wavefront
  const uint32_t g = grouped ? uint32_t(lane) / W : 0u;
  const uint32_t w0 = grouped ? uint32_t(lane) % W : uint32_t(lane);
  const uint32_t wstep = grouped ? W : uint32_t(kWave);
  const bool lane_on = grouped ? (g < G) : true;
  for (uint64_t i = wave; i < n2; i += n_waves) {
    const uint32_t r = e2[2 * i], x = e2[2 * i + 1];
    const uint32_t* Rr = bits + uint64_t(r) * W;
    const uint32_t* Rx = bits + uint64_t(x) * W;
    const uint32_t re = g2_off[r + 1];
    const uint32_t p = upper_bound(g2_adj, g2_off[r], re, x);
    const uint32_t xe = g2_off[x + 1];
    const uint32_t q = upper_bound(g2_adj, g2_off[x], xe, r);
    // |A| = 3 and |A| = 2: y over the neighbours of r above x, 64 at a time
    for (uint32_t base = p; base < re; base += kWave) {
      const uint32_t cnt = min(uint32_t(kWave), re - base);
      if (uint32_t(lane) < cnt) ys[lane] = g2_adj[base + lane];
      wave_sync();
      if (lane_on)
        for (uint32_t w = w0; w < W; w += wstep) {
          const uint32_t Nr = Rr[w], Nx = Rx[w];
          const uint32_t wr = ~Nr & mask_gt(r, w) & mask_below(N, w);
          for (uint32_t j = g; j < cnt; j += G) {
            const uint32_t y = ys[j];
            const uint32_t Ny = bits[uint64_t(y) * W + w];
            const bool xy = (Rx[y >> 5] >> (y & 31)) & 1u;
            c4_word(Nr, Nx, Ny, mask_gt(y, w), wr, xy, t3_0, t3_1, t2_0, t2_1);
          }
        }
      wave_sync();
    }
    // |A| = 1: y over the neighbours of x above r that are not neighbours of r
    for (uint32_t base = q; base < xe; base += kWave) {
      const bool in = base + lane < xe;
      const uint32_t y0 = in ? g2_adj[base + lane] : 0u;
      const bool keep = in && !((Rr[y0 >> 5] >> (y0 & 31)) & 1u);
      const unsigned long long mk = __ballot(keep);
      const uint32_t cnt = uint32_t(__popcll(mk));
      if (keep) ys[__popcll(mk & ((1ull << lane) - 1ull))] = y0;
      wave_sync();
      if (lane_on)
        for (uint32_t w = w0; w < W; w += wstep) {
          const uint32_t Nr = Rr[w], Nx = Rx[w];
          const uint32_t wr = ~Nr & mask_gt(r, w) & mask_below(N, w);
          const uint32_t nxw = Nx & wr;
          for (uint32_t j = g; j < cnt; j += G) {
            const uint32_t y = ys[j];
            const uint32_t Ny = bits[uint64_t(y) * W + w];
            const uint32_t zz = nxw & mask_gt(y, w);
            paw += __popc(zz & Ny);
            star += __popc(zz & ~Ny);
            path += __popc(Ny & wr & ~Nx);
          }
        }
      wave_sync();
    }
  }
  // local positions r=0, x=1, y=2, z=3; pair bits: rx 0, ry 1, xy 2, rz 4, xz 5, yz 7
  unsigned long long v[17];
  uint32_t pat[17];
  for (int xz = 0; xz < 2; ++xz)
    for (int yz = 0; yz < 2; ++yz) {
      const int j = xz * 2 + yz;
      v[j] = t3_0[j];
      pat[j] = (1u << 0) | (1u << 1) | (1u << 4) | (uint32_t(xz) << 5) | (uint32_t(yz) << 7);
      v[4 + j] = t3_1[j];
      pat[4 + j] = pat[j] | (1u << 2);
    }
  const uint32_t k2[3] = {(1u << 5) | (1u << 7), 1u << 5, 1u << 7};
  for (int j = 0; j < 3; ++j) {
    v[8 + j] = t2_0[j];
    pat[8 + j] = (1u << 0) | (1u << 1) | k2[j];
    v[11 + j] = t2_1[j];
    pat[11 + j] = pat[8 + j] | (1u << 2);
  }
  v[14] = paw;  pat[14] = (1u << 0) | (1u << 2) | (1u << 5) | (1u << 7);
  v[15] = star; pat[15] = (1u << 0) | (1u << 2) | (1u << 5);
  v[16] = path; pat[16] = (1u << 0) | (1u << 2) | (1u << 7);
  for (int j = 0; j < 17; ++j) {
    const unsigned long long sum = wave_sum(v[j]);
    if (lane == 0 && sum) atomicAdd(&h_g2[lut[pat[j]]], sum);
  }
  __syncthreads();
  flush(h_g2, hist + kG2, 256);
}

// (c) without bit rows: the same shapes enumerated one set at a time with
// pair lookups in the hash set (used when the node count is large).
__global__ void __launch_bounds__(kThreads) k_case_c4_hash(
    const uint32_t* __restrict__ e2, uint64_t n2, const uint32_t* __restrict__ g2_off,
    const uint32_t* __restrict__ g2_adj, Set64 hs2, const uint8_t* __restrict__ lut_g,
    unsigned long long* __restrict__ hist) {
  __shared__ uint8_t lut[2048];
  __shared__ unsigned long long h_g2[256];
  load_lut(lut, lut_g, 2048);
  h_g2[threadIdx.x] = 0;
  __syncthreads();
  const int lane = threadIdx.x & (kWave - 1);
  const uint64_t wave = uint64_t(blockIdx.x) * kWavesPerBlock + threadIdx.x / kWave;
  const uint64_t n_waves = uint64_t(gridDim.x) * kWavesPerBlock;
  for (uint64_t i = wave; i < n2; i += n_waves) {
    const uint32_t r = e2[2 * i], x = e2[2 * i + 1];
    const uint32_t rb = g2_off[r], re = g2_off[r + 1];
    const uint32_t xb = g2_off[x], xe = g2_off[x + 1];
    const uint32_t p = upper_bound(g2_adj, rb, re, x);
    // |A| = 3 and |A| = 2, lanes over y
    for (uint32_t yi = p + lane; yi < re; yi += kWave) {
      const uint32_t y = g2_adj[yi];
      const uint32_t xy = has2(hs2, x, y);
      for (uint32_t zi = yi + 1; zi < re; ++zi) {   // z > y, z ~ r
        const uint32_t z = g2_adj[zi];
        const uint32_t pz = (1u << 0) | (1u << 1) | (xy << 2) | (1u << 4) | (uint32_t(has2(hs2, x, z)) << 5) |
                            (uint32_t(has2(hs2, y, z)) << 7);
        atomicAdd(&h_g2[lut[pz]], 1ull);
      }
      for (uint32_t zi = xb; zi < xe; ++zi) {       // z ~ x
        const uint32_t z = g2_adj[zi];
        if (z <= r || z == y || has2(hs2, r, z)) continue;
        const uint32_t pz = (1u << 0) | (1u << 1) | (xy << 2) | (1u << 5) | (uint32_t(has2(hs2, y, z)) << 7);
        atomicAdd(&h_g2[lut[pz]], 1ull);
      }
      const uint32_t yb = g2_off[y], ye = g2_off[y + 1];
      for (uint32_t zi = yb; zi < ye; ++zi) {       // z ~ y, z !~ x
        const uint32_t z = g2_adj[zi];
        if (z <= r || z == x || has2(hs2, r, z) || has2(hs2, x, z)) continue;
        const uint32_t pz = (1u << 0) | (1u << 1) | (xy << 2) | (1u << 7);
        atomicAdd(&h_g2[lut[pz]], 1ull);
      }
    }
    // |A| = 1, lanes over y
    const uint32_t q = upper_bound(g2_adj, xb, xe, r);
    for (uint32_t yi = q + lane; yi < xe; yi += kWave) {
      const uint32_t y = g2_adj[yi];
      if (has2(hs2, r, y)) continue;
      for (uint32_t zi = yi + 1; zi < xe; ++zi) {   // z > y, z ~ x
        const uint32_t z = g2_adj[zi];
        if (has2(hs2, r, z)) continue;
        const uint32_t pz = (1u << 0) | (1u << 2) | (1u << 5) | (uint32_t(has2(hs2, y, z)) << 7);
        atomicAdd(&h_g2[lut[pz]], 1ull);
      }
      const uint32_t yb = g2_off[y], ye = g2_off[y + 1];
      for (uint32_t zi = yb; zi < ye; ++zi) {       // z ~ y, z !~ x, z !~ r, z > r
        const uint32_t z = g2_adj[zi];
        if (z <= r || z == x || has2(hs2, r, z) || has2(hs2, x, z)) continue;
        atomicAdd(&h_g2[lut[(1u << 0) | (1u << 2) | (1u << 7)]], 1ull);
      }
    }
  }
  __syncthreads();
  flush(h_g2, hist + kG2, 256);
}

// ---------------------------------------------------------------- order 3
// (a): one thread per 3-node hyperedge; local positions a,b,c = 0,1,2.
__global__ void __launch_bounds__(kThreads) k_case_a3(const uint32_t* __restrict__ e3, uint64_t n3, Set64 hs2,
                                                      const uint32_t* __restrict__ bits, uint32_t W,
                                                      const uint8_t* __restrict__ lut_g,
                                                      unsigned long long* __restrict__ hist) {
  __shared__ uint8_t lut[16];
  __shared__ unsigned long long h_main[256], h_sub[256];
  load_lut(lut, lut_g, 16);
  h_main[threadIdx.x] = 0;
  h_sub[threadIdx.x] = 0;
  __syncthreads();
  for (uint64_t i = uint64_t(blockIdx.x) * kThreads + threadIdx.x; i < n3; i += uint64_t(gridDim.x) * kThreads) {
    const uint32_t a = e3[3 * i], b = e3[3 * i + 1], c = e3[3 * i + 2];
    const uint32_t p = (1u << 3) | pair_bit(hs2, bits, W, a, b) | (pair_bit(hs2, bits, W, a, c) << 1) |
                       (pair_bit(hs2, bits, W, b, c) << 2);
    atomicAdd(&h_main[lut[p]], 1ull);
    const uint8_t g = lut[p & kPairBits3];
    if (g != 0xFF) atomicAdd(&h_sub[g], 1ull);
  }
  __syncthreads();
  flush(h_main, hist + kMain, 256);
  flush(h_sub, hist + kSub, 256);
}

// (c) for order 3: connected triples of G2 from their smallest node r; one
// thread per (pair {r<y}, word): z > y both neighbours of r (triangle or
// wedge centred at r), or z > r a neighbour of y only (wedge centred at y).
__global__ void __launch_bounds__(kThreads) k_case_c3_bits(const uint32_t* __restrict__ e2, uint64_t n2,
                                                           const uint32_t* __restrict__ bits, uint32_t W, uint32_t N,
                                                           const uint8_t* __restrict__ lut_g,
                                                           unsigned long long* __restrict__ hist) {
  __shared__ uint8_t lut[16];
  __shared__ unsigned long long h_g2[256];
  load_lut(lut, lut_g, 16);
  h_g2[threadIdx.x] = 0;
  __syncthreads();
  unsigned long long tri = 0, wedge_r = 0, wedge_y = 0;
  const uint64_t tasks = n2 * W;
  for (uint64_t t = uint64_t(blockIdx.x) * kThreads + threadIdx.x; t < tasks; t += uint64_t(gridDim.x) * kThreads) {
    const uint64_t i = t / W;
    const uint32_t w = uint32_t(t % W);
    const uint32_t r = e2[2 * i], y = e2[2 * i + 1];
    const uint32_t Nr = bits[uint64_t(r) * W + w], Ny = bits[uint64_t(y) * W + w];
    const uint32_t z = Nr & mask_gt(y, w);
    tri += __popc(z & Ny);
    wedge_r += __popc(z & ~Ny);
    wedge_y += __popc(Ny & ~Nr & mask_gt(r, w) & mask_below(N, w));
  }
  // local positions r=0, y=1, z=2: pair bits ry 0, rz 1, yz 2
  const unsigned long long s_tri = wave_sum(tri), s_wr = wave_sum(wedge_r), s_wy = wave_sum(wedge_y);
  if ((threadIdx.x & (kWave - 1)) == 0) {
    if (s_tri) atomicAdd(&h_g2[lut[7]], s_tri);
    if (s_wr) atomicAdd(&h_g2[lut[3]], s_wr);
    if (s_wy) atomicAdd(&h_g2[lut[5]], s_wy);
  }
  __syncthreads();
  flush(h_g2, hist + kG2, 256);
}

__global__ void __launch_bounds__(kThreads) k_case_c3_hash(const uint32_t* __restrict__ e2, uint64_t n2,
                                                           const uint32_t* __restrict__ g2_off,
                                                           const uint32_t* __restrict__ g2_adj, Set64 hs2,
                                                           const uint8_t* __restrict__ lut_g,
                                                           unsigned long long* __restrict__ hist) {
  __shared__ uint8_t lut[16];
  __shared__ unsigned long long h_g2[256];
  load_lut(lut, lut_g, 16);
  h_g2[threadIdx.x] = 0;
  __syncthreads();
  unsigned long long tri = 0, wedge_r = 0, wedge_y = 0;
  for (uint64_t i = uint64_t(blockIdx.x) * kThreads + threadIdx.x; i < n2; i += uint64_t(gridDim.x) * kThreads) {
    const uint32_t r = e2[2 * i], y = e2[2 * i + 1];
    const uint32_t re = g2_off[r + 1];
    for (uint32_t zi = upper_bound(g2_adj, g2_off[r], re, y); zi < re; ++zi) {
      if (has2(hs2, y, g2_adj[zi])) ++tri; else ++wedge_r;
    }
    for (uint32_t zi = g2_off[y]; zi < g2_off[y + 1]; ++zi) {
      const uint32_t z = g2_adj[zi];
      if (z > r && !has2(hs2, r, z)) ++wedge_y;
    }
  }
  const unsigned long long s_tri = wave_sum(tri), s_wr = wave_sum(wedge_r), s_wy = wave_sum(wedge_y);
  if ((threadIdx.x & (kWave - 1)) == 0) {
    if (s_tri) atomicAdd(&h_g2[lut[7]], s_tri);
    if (s_wr) atomicAdd(&h_g2[lut[3]], s_wr);
    if (s_wy) atomicAdd(&h_g2[lut[5]], s_wy);
  }
  __syncthreads();
  flush(h_g2, hist + kG2, 256);
}

// counts[c] = main[c] + (c pairs-only ? g2[c] - sub[c] : 0), as int64
struct ClassMask {
  unsigned long long w[4];
};

__global__ void k_combine(const unsigned long long* __restrict__ hist, int n_classes, ClassMask pairs_only,
                          int64_t* __restrict__ counts) {
  const int c = threadIdx.x;
  if (c >= n_classes) return;
  unsigned long long v = hist[kMain + c];
  if ((pairs_only.w[c >> 6] >> (c & 63)) & 1ull) v += hist[kG2 + c] - hist[kSub + c];
  counts[c] = int64_t(v);
}

// Counting kernels keep per-class counters in LDS and flush them once per
// workgroup; a grid of a few workgroups per CU that strides over the work
// keeps those flushes (global atomics on a few hundred addresses) rare.
constexpr unsigned kCountGrid = 512;

unsigned grid_waves(uint64_t items, unsigned cap = kCountGrid) {
  uint64_t g = (items + kWavesPerBlock - 1) / kWavesPerBlock;
  if (g < 1) g = 1;
  if (g > cap) g = cap;
  return unsigned(g);
}
unsigned grid_threads(uint64_t items, unsigned cap = kCountGrid, unsigned per_block = kThreads) {
  uint64_t g = (items + per_block - 1) / per_block;
  if (g < 1) g = 1;
  if (g > cap) g = cap;
  return unsigned(g);
}

}  // namespace

int count_exact_impl(const hm_graph* H, int k, int64_t* counts, hipStream_t st) {
  const uint8_t *lut4 = nullptr, *lut3 = nullptr;
  HM_TRY(device_luts(H->device, &lut4, &lut3));
  const ClassTables& t = class_tables();
  ClassMask pairs_only{{0, 0, 0, 0}};
  for (int c = 0; c < t.n_classes[k]; ++c)
    if (t.maxcard[k][c] == 2) pairs_only.w[c >> 6] |= 1ull << (c & 63);
  HM_TRY(fill_u64(H->hist, 0, 4 * 256, st));
  const uint64_t n2 = H->n_by_size[2], n3 = H->n_by_size[3], n4 = H->n_by_size[4];
  if (k == 4) {
    if (n4) {
      ProfileScope ps("k_case_a4", st);
      k_case_a4<<<grid_threads(n4), kThreads, 0, st>>>(H->e4, n4, H->hs2, H->hs3, H->bits, H->words, lut4,
                                                       H->hist);
    }
    if (n3) {
      if (H->bits) {
        ProfileScope ps("k_case_b4_bits", st);
        k_case_b4_bits<<<grid_waves(n3), kThreads, 0, st>>>(H->e3, n3, H->e4, H->i3_off, H->i3_idx, H->i4_off,
                                                            H->i4_idx, H->bits, H->words, lut4, H->hist);
      } else {
        ProfileScope ps("k_case_b4", st);
        k_case_b4<<<grid_waves(n3), kThreads, 0, st>>>(H->e3, n3, H->g2_off, H->g2_adj, H->i3_off, H->i3_idx,
                                                       H->hs2, H->hs3, H->hs4, lut4, H->hist);
      }
    }
    if (n2) {
      if (H->bits) {
        ProfileScope ps("k_case_c4_bits", st);
        k_case_c4_bits<<<grid_waves(n2), kThreads, 0, st>>>(H->e2, n2, H->g2_off, H->g2_adj, H->bits, H->words,
                                                            H->n_nodes, lut4, H->hist);
      } else {
        ProfileScope ps("k_case_c4_hash", st);
        k_case_c4_hash<<<grid_waves(n2), kThreads, 0, st>>>(H->e2, n2, H->g2_off, H->g2_adj, H->hs2, lut4, H->hist);
      }
    }
  } else {
    if (n3) {
      ProfileScope ps("k_case_a3", st);
      k_case_a3<<<grid_threads(n3), kThreads, 0, st>>>(H->e3, n3, H->hs2, H->bits, H->words, lut3, H->hist);
    }
    if (n2) {
      if (H->bits) {
        ProfileScope ps("k_case_c3_bits", st);
        k_case_c3_bits<<<grid_threads(n2 * H->words), kThreads, 0, st>>>(H->e2, n2, H->bits, H->words, H->n_nodes,
                                                                         lut3, H->hist);
      } else {
        ProfileScope ps("k_case_c3_hash", st);
        k_case_c3_hash<<<grid_threads(n2), kThreads, 0, st>>>(H->e2, n2, H->g2_off, H->g2_adj, H->hs2, lut3,
                                                              H->hist);
      }
    }
  }
  HM_HIP(hipGetLastError());
  k_combine<<<1, 256, 0, st>>>(H->hist, t.n_classes[k], pairs_only, counts);
  HM_HIP(hipGetLastError());
  return HM_OK;
}

}  // namespace hm

extern "C" int count_exact(const hm_graph* H, int k, int64_t* counts, void* stream) {
  if (!H || !counts) {
    hm::set_error("NULL argument to count_exact");
    return HM_EINVAL;
  }
  if (k != 3 && k != 4) {
    hm::set_error("order %d is not supported (3 or 4)", k);
    return HM_EUNSUPPORTED;
  }
  return hm::count_exact_impl(H, k, counts, static_cast<hipStream_t>(stream));
}
