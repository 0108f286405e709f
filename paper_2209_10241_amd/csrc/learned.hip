// Learned sampling proposal for Algorithm 4 (Section 5).
//
// Algorithm 4 draws hyperedges of each stratum uniformly; any proposal p_e > 0
// keeps the estimate unbiased when every draw of stratum j is weighted by
// 1 / (S_j p_e) (Hansen-Hurwitz), which is Algorithm 4's correction factor
// when p_e = 1 / |E_j|.  The proposal here scores each hyperedge with an MLP
// (16 features -> 64 -> 64 -> 1, ReLU; bf16 weights and activations on MFMA,
// fp32 accumulation) trained to predict, per stratum, the standardised
// log(1 + y_e) of the hyperedge's exact contribution
//   y_e = sum over classes m of raw_e[m] / countmax_m,
// raw_e being Algorithm 4's count for the single sample e (sum over e of
// stratum j of y_e = the exact total of the classes whose maxcard is j).
// Contributions are computed by the method itself on a subsampled hypergraph.
// Draws: p_e = (1 - eps) q_e / sum_j q + eps / |E_j|, q_e = (1 + y_e)^gamma
// as predicted; draw i of stratum j takes the first e whose cumulative
// probability exceeds u * total, u = (word0 >> 11) * 2^-53 of Philox4x64-10 at
// counter (i, 0, 0, 0) under key (seed, (3 << 32) | j).
#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstring>
#include <vector>

#include "hm_items.h"

namespace hm {

int enumerate_samples(const hm_graph* H, int k, const uint32_t* const idx[5], const uint64_t S[5],
                      unsigned long long* ps, const uint64_t row0[5], hipStream_t st);
int sample_sizes(const hm_graph* H, int k, double fraction, int allocation, uint64_t* S);

namespace {

constexpr int kF = 16, kHid = 64;
constexpr int kOffW1 = 0, kOffB1 = 1024, kOffW2 = 1088, kOffB2 = 5184, kOffW3 = 5248, kOffB3 = 5312;
constexpr int kNParams = 5313;

typedef short v4s __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));

__device__ inline short bf16_bits(float f) {
  uint32_t u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return short(u >> 16);
}

// ---------------------------------------------------------------- features
// Rows: the hyperedges of size 2, then 3 (then 4 at order 4), stratum order.
// Per member v: d2 = pairwise degree, d3 / d4 = incident 3- / 4-node hyperedges.
__global__ void k_features(View v, uint64_t n2, uint64_t n3, uint64_t n4, float* __restrict__ X) {
  const uint64_t n = n2 + n3 + n4;
  for (uint64_t r = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x; r < n; r += uint64_t(gridDim.x) * blockDim.x) {
    uint32_t m[4];
    int s;
    if (r < n2) {
      s = 2;
      m[0] = v.e2[2 * r];
      m[1] = v.e2[2 * r + 1];
    } else if (r < n2 + n3) {
      s = 3;
      const uint64_t i = r - n2;
      for (int j = 0; j < 3; ++j) m[j] = v.e3[3 * i + j];
    } else {
      s = 4;
      const uint64_t i = r - n2 - n3;
      for (int j = 0; j < 4; ++j) m[j] = v.e4[4 * i + j];
    }
    float d2[4], d3[4], d4[4];
    for (int j = 0; j < s; ++j) {
      d2[j] = float(v.g2_off[m[j] + 1] - v.g2_off[m[j]]);
      d3[j] = float(v.i3_off[m[j] + 1] - v.i3_off[m[j]]);
      d4[j] = float(v.i4_off[m[j] + 1] - v.i4_off[m[j]]);
    }
    float s2 = 0, mx2 = 0, mn2 = 1e30f, s3 = 0, mx3 = 0, s4 = 0, mx4 = 0, wed = 0, star = 0, d23 = 0;
    for (int j = 0; j < s; ++j) {
      s2 += d2[j];
      mx2 = fmaxf(mx2, d2[j]);
      mn2 = fminf(mn2, d2[j]);
      s3 += d3[j];
      mx3 = fmaxf(mx3, d3[j]);
      s4 += d4[j];
      mx4 = fmaxf(mx4, d4[j]);
      wed += 0.5f * d2[j] * (d2[j] - 1.f);
      star += d2[j] * (d2[j] - 1.f) * (d2[j] - 2.f) / 6.f;
      d23 += d2[j] * d3[j];
    }
    int pairs = 0, inside = 0;
    float pd = 0;
    for (int a = 0; a < s; ++a)
      for (int b = a + 1; b < s; ++b) {
        ++pairs;
        inside += int(pair_bit(v.hs2, v.bits, v.W, m[a], m[b]));
        pd += d2[a] * d2[b];
      }
    float* f = X + r * kF;
    f[0] = s == 2;
    f[1] = s == 3;
    f[2] = s == 4;
    f[3] = log1pf(s2 / s);
    f[4] = log1pf(mx2);
    f[5] = log1pf(mn2);
    f[6] = log1pf(s3 / s);
    f[7] = log1pf(mx3);
    f[8] = log1pf(s4 / s);
    f[9] = log1pf(mx4);
    f[10] = float(inside) / float(pairs);
    f[11] = 0.5f * log1pf(wed);
    f[12] = 0.5f * log1pf(d23);
    f[13] = 0.5f * log1pf(pd);
    f[14] = log1pf(star) / 3.f;
    f[15] = 1.f;
  }
}

// Deterministic mean / inverse standard deviation of column f over rows
// [lo, hi) of a row-major matrix (stride columns); one workgroup per
// (stratum, column), fixed summation order.
__global__ void k_column_stats(const float* __restrict__ M, int stride, const uint64_t* __restrict__ bounds,
                               int n_cols, float* __restrict__ stats) {
  __shared__ double s1[256], s2[256];
  const int strat = blockIdx.x / n_cols, f = blockIdx.x % n_cols;
  const uint64_t lo = bounds[strat], hi = bounds[strat + 1];
  double a = 0, b = 0;
  for (uint64_t r = lo + threadIdx.x; r < hi; r += blockDim.x) {
    const double x = M[r * stride + f];
    a += x;
    b += x * x;
  }
  s1[threadIdx.x] = a;
  s2[threadIdx.x] = b;
  __syncthreads();
  for (int d = 128; d > 0; d >>= 1) {
    if (int(threadIdx.x) < d) {
      s1[threadIdx.x] += s1[threadIdx.x + d];
      s2[threadIdx.x] += s2[threadIdx.x + d];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const double n = double(hi - lo);
    const double mean = n > 0 ? s1[0] / n : 0.0;
    const double var = n > 1 ? fmax(s2[0] / n - mean * mean, 0.0) : 0.0;
    stats[2 * blockIdx.x] = float(mean);
    stats[2 * blockIdx.x + 1] = var > 1e-12 ? float(1.0 / sqrt(var)) : 0.f;
  }
}

// Standardise columns 3..14 of the features per stratum (one-hots and the
// constant stay as they are).
__global__ void k_standardise(float* __restrict__ X, const uint64_t* __restrict__ bounds, int n_strata,
                              const float* __restrict__ stats) {
  const uint64_t n = bounds[n_strata];
  for (uint64_t r = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x; r < n; r += uint64_t(gridDim.x) * blockDim.x) {
    int s = 0;
    while (s + 1 < n_strata && r >= bounds[s + 1]) ++s;
    for (int f = 3; f < 15; ++f) {
      const float* st = stats + 2 * (s * kF + f);
      X[r * kF + f] = (X[r * kF + f] - st[0]) * st[1];
    }
  }
}

__global__ void k_log1p_targets(const double* __restrict__ y, uint64_t n, float* __restrict__ t) {
  for (uint64_t r = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x; r < n; r += uint64_t(gridDim.x) * blockDim.x)
    t[r] = float(log1p(y[r]));
}

__global__ void k_standardise_targets(float* __restrict__ t, const uint64_t* __restrict__ bounds, int n_strata,
                                      const float* __restrict__ stats) {
  const uint64_t n = bounds[n_strata];
  for (uint64_t r = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x; r < n; r += uint64_t(gridDim.x) * blockDim.x) {
    int s = 0;
    while (s + 1 < n_strata && r >= bounds[s + 1]) ++s;
    t[r] = (t[r] - stats[2 * s]) * stats[2 * s + 1];
  }
}

// ---------------------------------------------------------------- MLP on MFMA
// v_mfma_f32_16x16x16bf16_1k on a 16-row tile per wavefront.  Lane l, with
// r = l % 16 and q = l / 16: A operand holds A[r][4q..4q+3], B operand holds
// B[4q..4q+3][r], the result holds D[4q..4q+3][r].
struct MlpLds {
  short W1[kHid * kF];
  short W2[kHid * kHid];
  float b1[kHid], b2[kHid], w3[kHid];
  float b3;
};

__device__ void load_mlp(MlpLds& w, const float* __restrict__ p) {
  for (int i = threadIdx.x; i < kHid * kF; i += blockDim.x) w.W1[i] = bf16_bits(p[kOffW1 + i]);
  for (int i = threadIdx.x; i < kHid * kHid; i += blockDim.x) w.W2[i] = bf16_bits(p[kOffW2 + i]);
  for (int i = threadIdx.x; i < kHid; i += blockDim.x) {
    w.b1[i] = p[kOffB1 + i];
    w.b2[i] = p[kOffB2 + i];
    w.w3[i] = p[kOffW3 + i];
  }
  if (threadIdx.x == 0) w.b3 = p[kOffB3];
}

struct Tile {
  v4f z1[4], z2[4];
  float out[4];      // rows 4q + i, in every lane of group q
};

// Forward of rows r0..r0+15 of X (rows >= n read as zero).  h1s: 16 x 64
// wavefront-private LDS.
__device__ void mlp_forward_tile(const MlpLds& w, const float* __restrict__ X, uint64_t n, uint64_t r0, short* h1s,
                                 Tile& T) {
  const int l = threadIdx.x & (kWave - 1), r = l & 15, q = l >> 4;
  v4s xa;
  {
    const uint64_t row = r0 + r;
    for (int i = 0; i < 4; ++i) xa[i] = row < n ? bf16_bits(X[row * kF + 4 * q + i]) : short(0);
  }
  for (int nb = 0; nb < 4; ++nb) {
    v4s b;
    for (int i = 0; i < 4; ++i) b[i] = w.W1[(16 * nb + r) * kF + 4 * q + i];
    const v4f zero = {0.f, 0.f, 0.f, 0.f};
    v4f acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(xa, b, zero, 0, 0, 0);
    const float bias = w.b1[16 * nb + r];
    for (int i = 0; i < 4; ++i) {
      acc[i] += bias;
      h1s[(4 * q + i) * kHid + 16 * nb + r] = bf16_bits(fmaxf(acc[i], 0.f));
    }
    T.z1[nb] = acc;
  }
  wave_sync();
  for (int nb = 0; nb < 4; ++nb) T.z2[nb] = v4f{0.f, 0.f, 0.f, 0.f};
  for (int ks = 0; ks < 4; ++ks) {
    v4s a;
    for (int i = 0; i < 4; ++i) a[i] = h1s[r * kHid + 16 * ks + 4 * q + i];
    for (int nb = 0; nb < 4; ++nb) {
      v4s b;
      for (int i = 0; i < 4; ++i) b[i] = w.W2[(16 * nb + r) * kHid + 16 * ks + 4 * q + i];
      T.z2[nb] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, T.z2[nb], 0, 0, 0);
    }
  }
  float part[4] = {0.f, 0.f, 0.f, 0.f};
  for (int nb = 0; nb < 4; ++nb) {
    const float bias = w.b2[16 * nb + r], w3v = w.w3[16 * nb + r];
    for (int i = 0; i < 4; ++i) {
      T.z2[nb][i] += bias;
      part[i] += fmaxf(T.z2[nb][i], 0.f) * w3v;
    }
  }
  for (int i = 0; i < 4; ++i) {
    float x = part[i];
    for (int d = 1; d < 16; d <<= 1) x += __shfl_xor(x, d, kWave);
    T.out[i] = x + w.b3;
  }
  wave_sync();
}

__global__ void __launch_bounds__(kThreads) k_mlp_forward(const float* __restrict__ params,
                                                          const float* __restrict__ X, uint64_t n,
                                                          float* __restrict__ out) {
  __shared__ MlpLds w;
  __shared__ short h1s[kWavesPerBlock][16 * kHid];
  load_mlp(w, params);
  __syncthreads();
  const int l = threadIdx.x & (kWave - 1), r = l & 15, q = l >> 4;
  const int wv = threadIdx.x / kWave;
  const uint64_t tiles = (n + 15) / 16;
  for (uint64_t t = uint64_t(blockIdx.x) * kWavesPerBlock + wv; t < tiles; t += uint64_t(gridDim.x) * kWavesPerBlock) {
    Tile T;
    mlp_forward_tile(w, X, n, 16 * t, h1s[wv], T);
    if (r == 0)
      for (int i = 0; i < 4; ++i) {
        const uint64_t row = 16 * t + 4 * q + i;
        if (row < n) out[row] = T.out[i];
      }
  }
}

// Forward and backward of the mean squared error over n rows; every
// wavefront writes its gradient (and loss) partial to its own row of
// `partial` (kNParams + 1 values), reduced later in a fixed order.
__global__ void __launch_bounds__(kThreads) k_mlp_train(const float* __restrict__ params,
                                                        const float* __restrict__ X, const float* __restrict__ tgt,
                                                        uint64_t n, float inv_n, float* __restrict__ partial) {
  __shared__ MlpLds w;
  __shared__ short h1s[kWavesPerBlock][16 * kHid];
  __shared__ short dzs[kWavesPerBlock][16 * kHid];
  load_mlp(w, params);
  __syncthreads();
  const int l = threadIdx.x & (kWave - 1), r = l & 15, q = l >> 4;
  const int wv = threadIdx.x / kWave;
  v4f gW1[4], gW2[16];
  for (int i = 0; i < 4; ++i) gW1[i] = v4f{0.f, 0.f, 0.f, 0.f};
  for (int i = 0; i < 16; ++i) gW2[i] = v4f{0.f, 0.f, 0.f, 0.f};
  float gb1[4] = {0, 0, 0, 0}, gb2[4] = {0, 0, 0, 0}, gw3[4] = {0, 0, 0, 0}, gb3 = 0.f, loss = 0.f;
  const uint64_t tiles = (n + 15) / 16;
  const uint64_t wave = uint64_t(blockIdx.x) * kWavesPerBlock + wv;
  for (uint64_t t = wave; t < tiles; t += uint64_t(gridDim.x) * kWavesPerBlock) {
    const uint64_t r0 = 16 * t;
    Tile T;
    mlp_forward_tile(w, X, n, r0, h1s[wv], T);
    float dout[4];
    for (int i = 0; i < 4; ++i) {
      const uint64_t row = r0 + 4 * q + i;
      const bool valid = row < n;
      const float diff = valid ? T.out[i] - tgt[row] : 0.f;
      dout[i] = 2.f * diff * inv_n;
      if (r == 0) loss += diff * diff * inv_n;
      if (r == 0) gb3 += dout[i];
    }
    v4s dz2b[4], h1b[4];
    for (int nb = 0; nb < 4; ++nb) {
      const float w3v = w.w3[16 * nb + r];
      for (int i = 0; i < 4; ++i) {
        const float h2 = fmaxf(T.z2[nb][i], 0.f);
        gw3[nb] += dout[i] * h2;
        const float dz = T.z2[nb][i] > 0.f ? dout[i] * w3v : 0.f;
        gb2[nb] += dz;
        dz2b[nb][i] = bf16_bits(dz);
        h1b[nb][i] = bf16_bits(fmaxf(T.z1[nb][i], 0.f));
        dzs[wv][(4 * q + i) * kHid + 16 * nb + r] = dz2b[nb][i];
      }
    }
    for (int ob = 0; ob < 4; ++ob)
      for (int kb = 0; kb < 4; ++kb)
        gW2[ob * 4 + kb] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(dz2b[ob], h1b[kb], gW2[ob * 4 + kb], 0, 0, 0);
    wave_sync();
    v4s xd;
    for (int i = 0; i < 4; ++i) {
      const uint64_t row = r0 + 4 * q + i;
      xd[i] = row < n ? bf16_bits(X[row * kF + r]) : short(0);
    }
    for (int nb = 0; nb < 4; ++nb) {
      v4f acc = {0.f, 0.f, 0.f, 0.f};
      for (int ks = 0; ks < 4; ++ks) {
        v4s a, b;
        for (int i = 0; i < 4; ++i) {
          a[i] = dzs[wv][r * kHid + 16 * ks + 4 * q + i];
          b[i] = w.W2[(16 * ks + 4 * q + i) * kHid + 16 * nb + r];
        }
        acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, acc, 0, 0, 0);
      }
      v4s dz1b;
      for (int i = 0; i < 4; ++i) {
        const float dz = T.z1[nb][i] > 0.f ? acc[i] : 0.f;
        gb1[nb] += dz;
        dz1b[i] = bf16_bits(dz);
      }
      gW1[nb] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(dz1b, xd, gW1[nb], 0, 0, 0);
    }
    wave_sync();
  }
  // reduce the column partials over the four row groups, then write this
  // wavefront's row of partials
  float* out = partial + wave * (kNParams + 1);
  for (int nb = 0; nb < 4; ++nb) {
    float a = gb1[nb], b = gb2[nb], c = gw3[nb];
    for (int d = 16; d < kWave; d <<= 1) {
      a += __shfl_xor(a, d, kWave);
      b += __shfl_xor(b, d, kWave);
      c += __shfl_xor(c, d, kWave);
    }
    if (q == 0) {
      out[kOffB1 + 16 * nb + r] = a;
      out[kOffB2 + 16 * nb + r] = b;
      out[kOffW3 + 16 * nb + r] = c;
    }
    for (int i = 0; i < 4; ++i) out[kOffW1 + (16 * nb + 4 * q + i) * kF + r] = gW1[nb][i];
    for (int kb = 0; kb < 4; ++kb)
      for (int i = 0; i < 4; ++i) out[kOffW2 + (16 * nb + 4 * q + i) * kHid + 16 * kb + r] = gW2[nb * 4 + kb][i];
  }
  for (int d = 1; d < kWave; d <<= 1) {
    gb3 += __shfl_xor(gb3, d, kWave);
    loss += __shfl_xor(loss, d, kWave);
  }
  if (l == 0) {
    out[kOffB3] = gb3;
    out[kNParams] = loss;
  }
}

// grad[p] = sum over wavefronts of partial[w][p]; p = kNParams is the loss.
// Workgroups of four wavefronts take 64 consecutive parameters: wavefront q
// sums rows w = q, q + 4, ... and the four sums are added in the order
// q = 0..3, so the order of every addition is fixed.
constexpr uint32_t kReduceParams = kWave;
__global__ void __launch_bounds__(kThreads) k_reduce_partials(const float* __restrict__ partial, uint32_t n_waves,
                                                              float* __restrict__ grad) {
  __shared__ float part[kWavesPerBlock][kReduceParams];
  const uint32_t lane = threadIdx.x & (kWave - 1), q = threadIdx.x / kWave;
  const uint32_t p = blockIdx.x * kReduceParams + lane;
  float s = 0.f;
  if (p <= uint32_t(kNParams))
    for (uint32_t w = q; w < n_waves; w += kWavesPerBlock) s += partial[uint64_t(w) * (kNParams + 1) + p];
  part[q][lane] = s;
  __syncthreads();
  if (q == 0 && p <= uint32_t(kNParams)) {
    float t = part[0][lane];
    for (uint32_t r = 1; r < kWavesPerBlock; ++r) t += part[r][lane];
    grad[p] = t;
  }
}

// One Adam step; thread 0 also keeps the step's loss (grad[kNParams]) at loss[0].
__global__ void k_adam(float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m, float* __restrict__ v,
                       float lr, float b1, float b2, float eps, float c1, float c2, float* __restrict__ loss) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i == 0) loss[0] = g[kNParams];
  if (i >= kNParams) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.f - b1) * gi;
  const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

__global__ void k_gather_rows(const float* __restrict__ X, const float* __restrict__ t, const uint32_t* __restrict__ perm,
                              uint64_t n, float* __restrict__ Xp, float* __restrict__ tp) {
  for (uint64_t r = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x; r < n; r += uint64_t(gridDim.x) * blockDim.x) {
    const uint64_t s = perm[r];
    for (int f = 0; f < kF; ++f) Xp[r * kF + f] = X[s * kF + f];
    tp[r] = t[s];
  }
}

__global__ void k_perm_keys(uint64_t n, unsigned long long seed, unsigned long long* keys, uint32_t* vals) {
  for (uint64_t r = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x; r < n; r += uint64_t(gridDim.x) * blockDim.x) {
    keys[r] = philox4x64_10(r, 0, 0, 0, seed, (4ull << 32)).v[0];
    vals[r] = uint32_t(r);
  }
}

// ---------------------------------------------------------------- contributions
// y_e = sum_m raw_e[m] / countmax_m from per-sample rows of raw counts
struct CountmaxArg {
  uint8_t cm[256];
};

__global__ void k_contrib_rows(const unsigned long long* __restrict__ ps, uint64_t rows, int n_classes, CountmaxArg cm,
                               double* __restrict__ y) {
  for (uint64_t s = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x; s < rows; s += uint64_t(gridDim.x) * blockDim.x) {
    double acc = 0.0;
    for (int m = 0; m < n_classes; ++m) acc += double(ps[s * 256 + m]) / double(cm.cm[m]);
    y[s] = acc;
  }
}

__global__ void k_iota(uint32_t* p, uint64_t n, uint32_t base) {
  for (uint64_t i = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += uint64_t(gridDim.x) * blockDim.x)
    p[i] = base + uint32_t(i);
}

// ---------------------------------------------------------------- proposal
__global__ void k_scores(const float* __restrict__ out, const uint64_t* __restrict__ bounds, int n_strata,
                         const float* __restrict__ tstd, float gamma, double* __restrict__ q) {
  const uint64_t n = bounds[n_strata];
  for (uint64_t r = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x; r < n; r += uint64_t(gridDim.x) * blockDim.x) {
    int s = 0;
    while (s + 1 < n_strata && r >= bounds[s + 1]) ++s;
    // out ~ (log(1 + y) - mean) / sd on the training data: q ~ (1 + y)^gamma
    double e = double(gamma) * double(out[r]) * double(tstd[s]);
    e = fmin(fmax(e, -60.0), 60.0);
    q[r] = exp(e);
  }
}

// One workgroup per stratum: p = (1 - eps) q / sum q + eps / n_j, and the
// inclusive prefix sums of p (fixed order: per-chunk Hillis-Steele scans).
__global__ void k_proposal_cdf(const double* __restrict__ q, const uint64_t* __restrict__ bounds, float eps,
                               double* __restrict__ p, double* __restrict__ cdf) {
  __shared__ double buf[2][1024];
  __shared__ double total_s;
  const uint64_t lo = bounds[blockIdx.x], hi = bounds[blockIdx.x + 1];
  const uint64_t n = hi - lo;
  if (n == 0) return;
  // fixed-order sum of q
  double part = 0.0;
  for (uint64_t r = lo + threadIdx.x; r < hi; r += blockDim.x) part += q[r];
  buf[0][threadIdx.x] = part;
  __syncthreads();
  for (int d = 512; d > 0; d >>= 1) {
    if (int(threadIdx.x) < d) buf[0][threadIdx.x] += buf[0][threadIdx.x + d];
    __syncthreads();
  }
  if (threadIdx.x == 0) total_s = buf[0][0];
  __syncthreads();
  const double total = total_s, unif = double(eps) / double(n);
  double carry = 0.0;
  for (uint64_t base = lo; base < hi; base += 1024) {
    const uint64_t r = base + threadIdx.x;
    const double pv = r < hi ? (1.0 - double(eps)) * q[r] / total + unif : 0.0;
    if (r < hi) p[r] = pv;
    int cur = 0;
    buf[0][threadIdx.x] = pv;
    __syncthreads();
    for (int d = 1; d < 1024; d <<= 1) {
      const double x = buf[cur][threadIdx.x] + (int(threadIdx.x) >= d ? buf[cur][threadIdx.x - d] : 0.0);
      buf[1 - cur][threadIdx.x] = x;
      cur = 1 - cur;
      __syncthreads();
    }
    if (r < hi) cdf[r] = carry + buf[cur][threadIdx.x];
    carry += buf[cur][1023];
    __syncthreads();
  }
}

// Draw i of stratum j: the first position whose cumulative probability
// exceeds u * total.
__global__ void k_pps_draw(const double* __restrict__ cdf, const double* __restrict__ p, uint64_t n_j, uint64_t S,
                           unsigned long long seed, uint32_t j, uint32_t* __restrict__ idx, double* __restrict__ w) {
  const unsigned long long k1 = (kDomainProposal << 32) | j;
  const double total = cdf[n_j - 1];
  for (uint64_t i = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < S; i += uint64_t(gridDim.x) * blockDim.x) {
    const double u = double(philox4x64_10(i, 0, 0, 0, seed, k1).v[0] >> 11) * (1.0 / 9007199254740992.0);
    const double target = u * total;
    uint64_t a = 0, b = n_j - 1;
    while (a < b) {
      const uint64_t mid = (a + b) >> 1;
      if (cdf[mid] > target) b = mid; else a = mid + 1;
    }
    idx[i] = uint32_t(a);
    w[i] = 1.0 / (double(S) * p[a]);
  }
}

__global__ void k_weights_from_p(const double* __restrict__ pdraw, uint64_t S, double* __restrict__ w) {
  for (uint64_t i = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < S; i += uint64_t(gridDim.x) * blockDim.x)
    w[i] = 1.0 / (double(S) * pdraw[i]);
}

struct HHArgs {
  uint64_t row0[5], S[5];
  uint8_t maxcard[256], countmax[256];
};

// est_m = sum over draws s of stratum maxcard(m) of raw[s][m] w_s / countmax_m;
// one workgroup per class, fixed summation order.
__global__ void k_hh_estimate(const unsigned long long* __restrict__ ps, const double* __restrict__ w, HHArgs a,
                              int n_classes, float* __restrict__ est, int64_t* __restrict__ raw) {
  __shared__ double se[256];
  __shared__ unsigned long long sr[256];
  const int m = blockIdx.x;
  if (m >= n_classes) return;
  const int j = a.maxcard[m];
  double e = 0.0;
  unsigned long long rr = 0;
  for (uint64_t s = threadIdx.x; s < a.S[j]; s += blockDim.x) {
    const uint64_t row = a.row0[j] + s;
    const unsigned long long c = ps[row * 256 + m];
    e += double(c) * w[row];
    rr += c;
  }
  se[threadIdx.x] = e;
  sr[threadIdx.x] = rr;
  __syncthreads();
  for (int d = 128; d > 0; d >>= 1) {
    if (int(threadIdx.x) < d) {
      se[threadIdx.x] += se[threadIdx.x + d];
      sr[threadIdx.x] += sr[threadIdx.x + d];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    est[m] = float(se[0] / double(a.countmax[m]));
    if (raw) raw[m] = int64_t(sr[0]);
  }
}

unsigned grid_for(uint64_t n, unsigned cap = 4096) {
  uint64_t g = (n + 255) / 256;
  if (g < 1) g = 1;
  if (g > cap) g = cap;
  return unsigned(g);
}

// workgroups for an MLP pass over n rows: 16 rows per wavefront
unsigned mlp_grid(uint64_t n) {
  const uint64_t tiles = (n + 15) / 16;
  uint64_t g = (tiles + kWavesPerBlock - 1) / kWavesPerBlock;
  if (g < 1) g = 1;
  if (g > 2048) g = 2048;
  return unsigned(g);
}

// Temporaries of one call, released in stream order: the caching allocator
// hands a block out again only after the work enqueued on st before the
// release has completed, also when the call returns early on an error.
struct Bufs {
  std::vector<void*> ptrs;
  hipStream_t st;
  explicit Bufs(hipStream_t s) : st(s) {}
  ~Bufs() { dfree_on(ptrs.data(), ptrs.size(), st); }
  template <typename T>
  int get(T** p, uint64_t n) {
    void* q = nullptr;
    HM_TRY(dalloc(&q, size_t(n ? n : 1) * sizeof(T)));
    ptrs.push_back(q);
    *p = static_cast<T*>(q);
    return HM_OK;
  }
};

int strata_bounds(const hm_graph* H, int k, uint64_t b[5]) {
  b[0] = 0;
  b[1] = H->n_by_size[2];
  b[2] = b[1] + H->n_by_size[3];
  b[3] = b[2] + (k == 4 ? H->n_by_size[4] : 0);
  b[4] = b[3];
  return k == 4 ? 3 : 2;
}

// standardised features of every hyperedge of size 2..k (device, n x 16)
int features(const hm_graph* H, int k, float* X, Bufs& tmp, hipStream_t st) {
  note_use(H, st);
  uint64_t b[5];
  const int ns = strata_bounds(H, k, b);
  const uint64_t n = b[ns];
  if (!n) return HM_OK;
  const View v = view_of(H);
  k_features<<<grid_for(n), 256, 0, st>>>(v, H->n_by_size[2], H->n_by_size[3], k == 4 ? H->n_by_size[4] : 0, X);
  HM_HIP(hipGetLastError());
  uint64_t* db = nullptr;
  float* stats = nullptr;
  HM_TRY(tmp.get(&db, 5));
  HM_TRY(tmp.get(&stats, 2ull * ns * kF));
  HM_HIP(hipMemcpyAsync(db, b, sizeof(uint64_t) * 5, hipMemcpyHostToDevice, st));
  k_column_stats<<<ns * kF, 256, 0, st>>>(X, kF, db, kF, stats);
  k_standardise<<<grid_for(n), 256, 0, st>>>(X, db, ns, stats);
  HM_HIP(hipGetLastError());
  HM_HIP(hipStreamSynchronize(st));
  return HM_OK;
}

}  // namespace

// Per-hyperedge contributions y (device, stratum rows), by enumerating each
// hyperedge as a single sample (chunks of rows).
int contributions(const hm_graph* H, int k, double* y, hipStream_t st) {
  note_use(H, st);
  const ClassTables& t = class_tables();
  CountmaxArg cm;
  for (int c = 0; c < 256; ++c) cm.cm[c] = c < t.n_classes[k] ? t.countmax[k][c] : 1;
  constexpr uint64_t kChunk = 16384;
  Bufs tmp(st);
  unsigned long long* ps = nullptr;
  uint32_t* idx = nullptr;
  HM_TRY(tmp.get(&ps, kChunk * 256));
  HM_TRY(tmp.get(&idx, kChunk));
  uint64_t row = 0;
  for (int j = 2; j <= k; ++j) {
    const uint64_t nj = H->n_by_size[j];
    for (uint64_t base = 0; base < nj; base += kChunk) {
      const uint64_t cnt = std::min<uint64_t>(kChunk, nj - base);
      k_iota<<<grid_for(cnt), 256, 0, st>>>(idx, cnt, uint32_t(base));
      HM_TRY(fill_u64(ps, 0, cnt * 256, st));
      const uint32_t* ix[5] = {nullptr, nullptr, nullptr, nullptr, nullptr};
      uint64_t S[5] = {0, 0, 0, 0, 0};
      const uint64_t row0[5] = {0, 0, 0, 0, 0};
      ix[j] = idx;
      S[j] = cnt;
      HM_TRY(enumerate_samples(H, k, ix, S, ps, row0, st));
      k_contrib_rows<<<grid_for(cnt), 256, 0, st>>>(ps, cnt, t.n_classes[k], cm, y + row + base);
      HM_HIP(hipGetLastError());
    }
    row += nj;
  }
  HM_HIP(hipStreamSynchronize(st));
  return HM_OK;
}

// Hansen-Hurwitz estimate from explicit draws (device indices) and weights.
int hh_from_draws(const hm_graph* H, int k, const uint32_t* const idx[5], const uint64_t S[5], const double* w,
                  float* est, int64_t* raw, hipStream_t st) {
  note_use(H, st);
  Bufs tmp(st);
  uint64_t total = 0, row0[5] = {0, 0, 0, 0, 0};
  for (int j = 2; j <= k; ++j) {
    row0[j] = total;
    total += S[j];
  }
  unsigned long long* ps = nullptr;
  HM_TRY(tmp.get(&ps, (total + 1) * 256));
  HM_TRY(fill_u64(ps, 0, (total + 1) * 256, st));
  HM_TRY(enumerate_samples(H, k, idx, S, ps, row0, st));
  const ClassTables& t = class_tables();
  HHArgs a;
  for (int j = 0; j < 5; ++j) {
    a.row0[j] = row0[j];
    a.S[j] = (j >= 2 && j <= k) ? S[j] : 0;
  }
  for (int c = 0; c < 256; ++c) {
    a.maxcard[c] = c < t.n_classes[k] ? t.maxcard[k][c] : 0;
    a.countmax[c] = c < t.n_classes[k] ? t.countmax[k][c] : 1;
  }
  k_hh_estimate<<<t.n_classes[k], 256, 0, st>>>(ps, w, a, t.n_classes[k], est, raw);
  HM_HIP(hipGetLastError());
  HM_HIP(hipStreamSynchronize(st));
  return HM_OK;
}

}  // namespace hm

// ---------------------------------------------------------------- model handle
struct hm_model {
  int k = 4;
  int device = 0;
  float* params = nullptr;      // device, kNParams
  float tstd[4] = {1, 1, 1, 1};  // per stratum: sd of log(1 + y) on the training data
  float gamma = 0.5f;
  float epsilon = 0.1f;
  std::vector<float> loss;      // mean training loss per epoch
  uint64_t id = 0;
};

namespace hm {
namespace {

std::atomic<uint64_t> g_model_ids{1};

// host-side deterministic initialisation: splitmix64 + Box-Muller
struct InitRng {
  uint64_t s;
  uint64_t next() {
    uint64_t z = (s += 0x9e3779b97f4a7c15ull);
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    return z ^ (z >> 31);
  }
  double uniform() { return (double(next() >> 11) + 0.5) * (1.0 / 9007199254740992.0); }
  double normal() { return std::sqrt(-2.0 * std::log(uniform())) * std::cos(6.283185307179586 * uniform()); }
};

}  // namespace

struct ProposalCache {
  uint64_t model_id = 0;
  int k = 0;
  double* p = nullptr;      // per stratum row
  double* cdf = nullptr;
  uint64_t bounds[5] = {0, 0, 0, 0, 0};
  std::vector<void*> ptrs;
  ~ProposalCache() {
    for (void* q : ptrs) dfree(q);
  }
};

void destroy_proposal_cache(ProposalCache* c) { delete c; }

int build_proposal(const hm_graph* Hc, const hm_model* M, int k, hipStream_t st) {
  note_use(Hc, st);
  hm_graph* H = const_cast<hm_graph*>(Hc);
  if (H->proposal && H->proposal->model_id == M->id && H->proposal->k == k) return HM_OK;
  if (H->proposal) {
    HM_HIP(hipStreamSynchronize(st));
    destroy_proposal_cache(H->proposal);
    H->proposal = nullptr;
  }
  ProposalCache* C = new (std::nothrow) ProposalCache();
  if (!C) {
    set_error("host allocation failed");
    return HM_ENOMEM;
  }
  C->model_id = M->id;
  C->k = k;
  const int ns = strata_bounds(H, k, C->bounds);
  const uint64_t n = C->bounds[ns];
  Bufs tmp(st);
  float *X = nullptr, *out = nullptr, *tstd = nullptr;
  double* q = nullptr;
  uint64_t* db = nullptr;
  auto owned = [&](double** ptr, uint64_t count) {
    void* v = nullptr;
    int rc = dalloc(&v, (count ? count : 1) * sizeof(double));
    if (rc == HM_OK) {
      C->ptrs.push_back(v);
      *ptr = static_cast<double*>(v);
    }
    return rc;
  };
  int rc = owned(&C->p, n);
  if (rc == HM_OK) rc = owned(&C->cdf, n);
  if (rc == HM_OK) rc = tmp.get(&X, n * kF);
  if (rc == HM_OK) rc = tmp.get(&out, n);
  if (rc == HM_OK) rc = tmp.get(&q, n);
  if (rc == HM_OK) rc = tmp.get(&tstd, 4);
  if (rc == HM_OK) rc = tmp.get(&db, 5);
  if (rc == HM_OK) rc = features(H, k, X, tmp, st);
  if (rc == HM_OK && n) {
    k_mlp_forward<<<mlp_grid(n), kThreads, 0, st>>>(M->params, X, n, out);
    if (hipMemcpyAsync(tstd, M->tstd, sizeof(float) * 4, hipMemcpyHostToDevice, st) != hipSuccess ||
        hipMemcpyAsync(db, C->bounds, sizeof(uint64_t) * 5, hipMemcpyHostToDevice, st) != hipSuccess)
      rc = HM_EDEVICE;
    if (rc == HM_OK) {
      k_scores<<<grid_for(n), 256, 0, st>>>(out, db, ns, tstd, M->gamma, q);
      k_proposal_cdf<<<ns, 1024, 0, st>>>(q, db, M->epsilon, C->p, C->cdf);
      if (hipGetLastError() != hipSuccess) rc = HM_EDEVICE;
    }
  }
  if (rc == HM_OK && hipStreamSynchronize(st) != hipSuccess) rc = HM_EDEVICE;
  if (rc != HM_OK) {
    delete C;
    return rc;
  }
  H->proposal = C;
  return HM_OK;
}

}  // namespace hm

extern "C" {

int hm_features(const hm_graph* H, int k, float* x, void* stream) {
  try {
    if (!H || !x) {
      hm::set_error("NULL argument to hm_features");
      return HM_EINVAL;
    }
    if (k != 3 && k != 4) {
      hm::set_error("order %d is not supported (3 or 4)", k);
      return HM_EUNSUPPORTED;
    }
    hm::Bufs tmp(static_cast<hipStream_t>(stream));
    return hm::features(H, k, x, tmp, static_cast<hipStream_t>(stream));
  } catch (...) {
    return hm::api_failure();
  }
}

int hm_contrib(const hm_graph* H, int k, double* y, void* stream) {
  try {
    if (!H || !y) {
      hm::set_error("NULL argument to hm_contrib");
      return HM_EINVAL;
    }
    if (k != 3 && k != 4) {
      hm::set_error("order %d is not supported (3 or 4)", k);
      return HM_EUNSUPPORTED;
    }
    return hm::contributions(H, k, y, static_cast<hipStream_t>(stream));
  } catch (...) {
    return hm::api_failure();
  }
}

int hm_mlp_forward(const float* params, const float* x, uint64_t n, float* out, void* stream) {
  try {
    if (!params || (!x && n) || (!out && n)) {
      hm::set_error("NULL argument to hm_mlp_forward");
      return HM_EINVAL;
    }
    if (!n) return HM_OK;
    hipStream_t st = static_cast<hipStream_t>(stream);
    hm::k_mlp_forward<<<hm::mlp_grid(n), hm::kThreads, 0, st>>>(params, x, n, out);
    HM_HIP(hipGetLastError());
    return HM_OK;
  } catch (...) {
    return hm::api_failure();
  }
}

int hm_mlp_grad(const float* params, const float* x, const float* t, uint64_t n, float* grad, void* stream) {
  try {
    if (!params || !grad || (n && (!x || !t))) {
      hm::set_error("NULL argument to hm_mlp_grad");
      return HM_EINVAL;
    }
    hipStream_t st = static_cast<hipStream_t>(stream);
    const uint32_t blocks = uint32_t(std::min<uint64_t>((n + 63) / 64 + 1, 256));
    const uint32_t waves = blocks * hm::kWavesPerBlock;
    hm::Bufs tmp(st);
    float* partial = nullptr;
    HM_TRY(tmp.get(&partial, uint64_t(waves) * (hm::kNParams + 1)));
    hm::k_mlp_train<<<blocks, hm::kThreads, 0, st>>>(params, x, t, n, n ? 1.f / float(n) : 0.f, partial);
    hm::k_reduce_partials<<<(hm::kNParams + hm::kReduceParams) / hm::kReduceParams, hm::kThreads, 0, st>>>(partial, waves,
                                                                                                       grad);
    HM_HIP(hipGetLastError());
    HM_HIP(hipStreamSynchronize(st));
    return HM_OK;
  } catch (...) {
    return hm::api_failure();
  }
}

int hm_model_train(const hm_graph* H, int k, const hm_train_opts* opts, hm_model** out) {
  try {
    if (!H || !opts || !out) {
      hm::set_error("NULL argument to hm_model_train");
      return HM_EINVAL;
    }
    if (k != 3 && k != 4) {
      hm::set_error("order %d is not supported (3 or 4)", k);
      return HM_EUNSUPPORTED;
    }
    if (opts->epochs < 0 || opts->batch < 16 || !(opts->lr > 0) || !(opts->epsilon > 0 && opts->epsilon <= 1) ||
        !(opts->gamma >= 0)) {
      hm::set_error("bad training options");
      return HM_EINVAL;
    }
    *out = nullptr;
    hipStream_t st = nullptr;
    hm_model* M = new (std::nothrow) hm_model();
    if (!M) {
      hm::set_error("host allocation failed");
      return HM_ENOMEM;
    }
    M->k = k;
    M->gamma = opts->gamma;
    M->epsilon = opts->epsilon;
    M->id = hm::g_model_ids.fetch_add(1);
    (void)hipGetDevice(&M->device);
    void* pp = nullptr;
    int rc = hm::dalloc(&pp, hm::kNParams * sizeof(float));
    if (rc != HM_OK) {
      delete M;
      return rc;
    }
    M->params = static_cast<float*>(pp);
    // initial weights: He for the ReLU layers, biases zero
    std::vector<float> init(hm::kNParams, 0.f);
    hm::InitRng rng{opts->seed ^ 0x6a09e667f3bcc908ull};
    for (int i = 0; i < 1024; ++i) init[hm::kOffW1 + i] = float(rng.normal() * std::sqrt(2.0 / 16.0));
    for (int i = 0; i < 4096; ++i) init[hm::kOffW2 + i] = float(rng.normal() * std::sqrt(2.0 / 64.0));
    for (int i = 0; i < 64; ++i) init[hm::kOffW3 + i] = float(rng.normal() * std::sqrt(1.0 / 64.0));
    rc = hipMemcpy(M->params, init.data(), sizeof(float) * hm::kNParams, hipMemcpyHostToDevice) == hipSuccess
             ? HM_OK
             : HM_EDEVICE;
    uint64_t b[5];
    const int ns = hm::strata_bounds(H, k, b);
    const uint64_t n = b[ns];
    hm::Bufs tmp(st);
    float *X = nullptr, *t = nullptr, *Xp = nullptr, *tp = nullptr, *stats = nullptr, *partial = nullptr, *grad = nullptr,
          *m = nullptr, *v = nullptr;
    double* y = nullptr;
    uint64_t* db = nullptr;
    unsigned long long *keys = nullptr, *keys_tmp = nullptr;
    uint32_t *vals = nullptr, *vals_tmp = nullptr;
    const uint32_t batch = uint32_t(opts->batch);
    const uint32_t blocks = std::min<uint32_t>((batch + 63) / 64, 256);
    const uint32_t waves = blocks * hm::kWavesPerBlock;
    if (rc == HM_OK) rc = tmp.get(&X, n * hm::kF);
    if (rc == HM_OK) rc = tmp.get(&t, n);
    if (rc == HM_OK) rc = tmp.get(&Xp, n * hm::kF);
    if (rc == HM_OK) rc = tmp.get(&tp, n);
    if (rc == HM_OK) rc = tmp.get(&y, n);
    if (rc == HM_OK) rc = tmp.get(&stats, 8);
    if (rc == HM_OK) rc = tmp.get(&db, 5);
    if (rc == HM_OK) rc = tmp.get(&partial, uint64_t(waves) * (hm::kNParams + 1));
    if (rc == HM_OK) rc = tmp.get(&grad, hm::kNParams + 1);
    if (rc == HM_OK) rc = tmp.get(&m, hm::kNParams);
    if (rc == HM_OK) rc = tmp.get(&v, hm::kNParams);
    if (rc == HM_OK) rc = tmp.get(&keys, n);
    if (rc == HM_OK) rc = tmp.get(&keys_tmp, n);
    if (rc == HM_OK) rc = tmp.get(&vals, n);
    if (rc == HM_OK) rc = tmp.get(&vals_tmp, n);
    // features and exact contributions of the training hypergraph
    if (rc == HM_OK) rc = hm::features(H, k, X, tmp, st);
    if (rc == HM_OK) rc = hm::contributions(H, k, y, st);
    if (rc == HM_OK && n) {
      hm::k_log1p_targets<<<hm::grid_for(n), 256, 0, st>>>(y, n, t);
      if (hipMemcpyAsync(db, b, sizeof(uint64_t) * 5, hipMemcpyHostToDevice, st) != hipSuccess) rc = HM_EDEVICE;
      hm::k_column_stats<<<ns, 256, 0, st>>>(t, 1, db, 1, stats);
      hm::k_standardise_targets<<<hm::grid_for(n), 256, 0, st>>>(t, db, ns, stats);
      // one fixed random order of the rows
      hm::k_perm_keys<<<hm::grid_for(n), 256, 0, st>>>(n, opts->seed, keys, vals);
      if (hipGetLastError() != hipSuccess) rc = HM_EDEVICE;
      if (rc == HM_OK) rc = hm::radix_sort_pairs(keys, vals, keys_tmp, vals_tmp, n, 64, st);
      if (rc == HM_OK) hm::k_gather_rows<<<hm::grid_for(n), 256, 0, st>>>(X, t, vals, n, Xp, tp);
      if (rc == HM_OK) rc = hm::fill_u32(reinterpret_cast<uint32_t*>(m), 0, hm::kNParams, st);
      if (rc == HM_OK) rc = hm::fill_u32(reinterpret_cast<uint32_t*>(v), 0, hm::kNParams, st);
      float host_stats[8] = {0, 1, 0, 1, 0, 1, 0, 1};
      if (rc == HM_OK && hipMemcpyAsync(host_stats, stats, sizeof(float) * 2 * ns, hipMemcpyDeviceToHost, st) != hipSuccess)
        rc = HM_EDEVICE;
      if (rc == HM_OK && hipStreamSynchronize(st) != hipSuccess) rc = HM_EDEVICE;
      for (int s = 0; s < ns; ++s) M->tstd[s] = host_stats[2 * s + 1] > 0.f ? 1.f / host_stats[2 * s + 1] : 1.f;
    }
    // Adam over mini-batches; every step's loss stays on the device and an
    // epoch's losses are read back once, at its end
    int step = 0;
    const float b1 = 0.9f, b2 = 0.999f;
    const uint64_t batches_per_epoch = n ? (n + batch - 1) / batch : 0;
    float* losses = nullptr;
    if (rc == HM_OK) rc = tmp.get(&losses, batches_per_epoch + 1);
    std::vector<float> host_losses(batches_per_epoch + 1);
    for (int ep = 0; ep < opts->epochs && rc == HM_OK && n; ++ep) {
      uint64_t n_batches = 0;
      for (uint64_t b0 = 0; b0 < n && rc == HM_OK; b0 += batch) {
        const uint64_t nb = std::min<uint64_t>(batch, n - b0);
        hm::k_mlp_train<<<blocks, hm::kThreads, 0, st>>>(M->params, Xp + b0 * hm::kF, tp + b0, nb, 1.f / float(nb),
                                                         partial);
        hm::k_reduce_partials<<<(hm::kNParams + hm::kReduceParams) / hm::kReduceParams, hm::kThreads, 0, st>>>(
            partial, waves, grad);
        ++step;
        const float c1 = 1.f - std::pow(b1, float(step)), c2 = 1.f - std::pow(b2, float(step));
        hm::k_adam<<<(hm::kNParams + 255) / 256, 256, 0, st>>>(M->params, grad, m, v, opts->lr, b1, b2, 1e-8f, c1, c2,
                                                                losses + n_batches);
        if (hipGetLastError() != hipSuccess) rc = HM_EDEVICE;
        ++n_batches;
      }
      if (rc == HM_OK && hipMemcpyAsync(host_losses.data(), losses, sizeof(float) * n_batches, hipMemcpyDeviceToHost,
                                        st) != hipSuccess)
        rc = HM_EDEVICE;
      if (rc == HM_OK && hipStreamSynchronize(st) != hipSuccess) rc = HM_EDEVICE;
      double ep_loss = 0.0;
      for (uint64_t i = 0; i < n_batches; ++i) ep_loss += host_losses[i];
      M->loss.push_back(float(ep_loss / double(std::max<uint64_t>(1, n_batches))));
    }
    if (rc != HM_OK) {
      hm::dfree(M->params);
      delete M;
      return rc;
    }
    *out = M;
    return HM_OK;
  } catch (...) {
    return hm::api_failure();
  }
}

int hm_model_destroy(hm_model* M) {
  try {
    if (!M) return HM_OK;
    (void)hipDeviceSynchronize();
    hm::dfree(M->params);
    delete M;
    return HM_OK;
  } catch (...) {
    return hm::api_failure();
  }
}

int hm_model_params(const hm_model* M, float* params_out) {
  try {
    if (!M || !params_out) {
      hm::set_error("NULL argument");
      return HM_EINVAL;
    }
    HM_HIP(hipMemcpy(params_out, M->params, sizeof(float) * hm::kNParams, hipMemcpyDeviceToHost));
    return HM_OK;
  } catch (...) {
    return hm::api_failure();
  }
}

int hm_model_loss(const hm_model* M, int max_epochs, float* loss_out) {
  try {
    if (!M) {
      hm::set_error("NULL argument");
      return HM_EINVAL;
    }
    const int n = int(M->loss.size());
    for (int i = 0; i < n && i < max_epochs && loss_out; ++i) loss_out[i] = M->loss[i];
    return n;
  } catch (...) {
    return hm::api_failure();
  }
}

int hm_proposal_probs(const hm_graph* H, const hm_model* M, int k, double* p, void* stream) {
  try {
    if (!H || !M || !p) {
      hm::set_error("NULL argument to hm_proposal_probs");
      return HM_EINVAL;
    }
    if (k != 3 && k != 4) {
      hm::set_error("order %d is not supported (3 or 4)", k);
      return HM_EUNSUPPORTED;
    }
    hipStream_t st = static_cast<hipStream_t>(stream);
    HM_TRY(hm::build_proposal(H, M, k, st));
    const hm::ProposalCache* C = H->proposal;
    const uint64_t n = C->bounds[k == 4 ? 3 : 2];
    if (n) HM_HIP(hipMemcpyAsync(p, C->p, n * sizeof(double), hipMemcpyDeviceToDevice, st));
    HM_HIP(hipStreamSynchronize(st));
    return HM_OK;
  } catch (...) {
    return hm::api_failure();
  }
}

int count_sampled_learned(const hm_graph* H, const hm_model* M, int k, double fraction, uint64_t seed, float* est,
                          int64_t* raw, void* stream) {
  try {
    if (!H || !M || !est) {
      hm::set_error("NULL argument to count_sampled_learned");
      return HM_EINVAL;
    }
    hipStream_t st = static_cast<hipStream_t>(stream);
    uint64_t S[5];
    HM_TRY(hm::sample_sizes(H, k, fraction, HM_ALLOC_PROPORTIONAL, S));
    HM_TRY(hm::build_proposal(H, M, k, st));
    const hm::ProposalCache* C = H->proposal;
    hm::Bufs tmp(st);
    uint64_t total = 0;
    for (int j = 2; j <= k; ++j) total += S[j];
    uint32_t* idx = nullptr;
    double* w = nullptr;
    HM_TRY(tmp.get(&idx, total + 1));
    HM_TRY(tmp.get(&w, total + 1));
    const uint32_t* ix[5] = {nullptr, nullptr, nullptr, nullptr, nullptr};
    uint64_t off = 0;
    for (int j = 2; j <= k; ++j) {
      ix[j] = idx + off;
      const uint64_t lo = C->bounds[j - 2];
      const uint64_t nj = H->n_by_size[j];
      if (S[j] && nj) {
        hm::k_pps_draw<<<hm::grid_for(S[j], 1024), 256, 0, st>>>(C->cdf + lo, C->p + lo, nj, S[j], seed, uint32_t(j),
                                                                idx + off, w + off);
        HM_HIP(hipGetLastError());
      }
      off += S[j];
    }
    return hm::hh_from_draws(H, k, ix, S, w, est, raw, st);
  } catch (...) {
    return hm::api_failure();
  }
}

int count_sampled_weighted_indices(const hm_graph* H, int k, const uint32_t* idx2, const double* p2, uint64_t s2,
                                   const uint32_t* idx3, const double* p3, uint64_t s3, const uint32_t* idx4,
                                   const double* p4, uint64_t s4, float* est, int64_t* raw, void* stream) {
  try {
    if (!H || !est) {
      hm::set_error("NULL argument to count_sampled_weighted_indices");
      return HM_EINVAL;
    }
    if (k != 3 && k != 4) {
      hm::set_error("order %d is not supported (3 or 4)", k);
      return HM_EUNSUPPORTED;
    }
    hipStream_t st = static_cast<hipStream_t>(stream);
    const uint32_t* ix[5] = {nullptr, nullptr, idx2, idx3, k == 4 ? idx4 : nullptr};
    const double* pp[5] = {nullptr, nullptr, p2, p3, k == 4 ? p4 : nullptr};
    uint64_t S[5] = {0, 0, s2, s3, k == 4 ? s4 : 0};
    hm::Bufs tmp(st);
    uint64_t total = S[2] + S[3] + S[4];
    double* w = nullptr;
    HM_TRY(tmp.get(&w, total + 1));
    uint64_t off = 0;
    for (int j = 2; j <= k; ++j) {
      if (S[j] && (!ix[j] || !pp[j])) {
        hm::set_error("index or probability array of stratum %d is NULL", j);
        return HM_EINVAL;
      }
      if (S[j]) {
        hm::k_weights_from_p<<<hm::grid_for(S[j], 1024), 256, 0, st>>>(pp[j], S[j], w + off);
        HM_HIP(hipGetLastError());
      }
      off += S[j];
    }
    // the index check of count_sampled_indices applies: reuse it through a raw call
    HM_TRY(count_sampled_indices(H, k, idx2, s2, idx3, s3, idx4, s4, est, raw, stream));
    return hm::hh_from_draws(H, k, ix, S, w, est, raw, st);
  } catch (...) {
    return hm::api_failure();
  }
}

}  // extern "C"
