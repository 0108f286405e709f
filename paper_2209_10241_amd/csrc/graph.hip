// Building the device-resident hypergraph (ingest).
//
// A hypergraph's hyperedges form a set (Definition of a hypergraph,
// Section 3): repeated hyperedges collapse onto their first occurrence;
// singletons are ignored (the fill-in of Section 4.3 skips them).  Every
// hyperedge of size 2..4 is hashed so that fill-in checks existence in
// constant time (Section 4.3, Fig. 3b).  The pairwise graph (hyperedges of
// size 2) is kept as ascending CSR rows, plus adjacency bit rows when the
// node count is small, and every node lists its incident 3- and 4-node
// hyperedges: the neighbourhoods Algorithms 3 and 4 explore.
#include <algorithm>
#include <vector>

#include "hm_internal.h"

namespace hm {
namespace {

enum : uint32_t {
  kErrEmpty = 1u,
  kErrBadId = 2u,
  kErrRepeat = 4u,
  kErrOffsets = 8u,
};

struct DevFlags {
  uint32_t err;
  uint32_t err_edge;
  unsigned long long singletons;
  unsigned long long duplicates;
  uint32_t max_deg2;
  uint32_t max_deg3;
};

constexpr int kRegSort = 16;

__device__ inline unsigned long long tuple_hash(const uint32_t* m, uint32_t s) {
  unsigned long long h = mix64(0x51ed270b27a3ffb1ull ^ s);
  for (uint32_t i = 0; i < s; ++i) h = mix64(h ^ (m[i] + 0x9e3779b97f4a7c15ull * (i + 1)));
  return h;
}

// One thread per input hyperedge: copy its members, sort them, check ids and
// repeats, record its size and hash.
__global__ void k_prepare(const uint32_t* __restrict__ members, const uint64_t* __restrict__ offsets,
                          uint64_t n_edges, uint64_t nnz, uint32_t n_nodes, uint32_t* __restrict__ sm,
                          uint32_t* __restrict__ size, unsigned long long* __restrict__ hash,
                          DevFlags* flags) {
  for (uint64_t i = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n_edges;
       i += uint64_t(gridDim.x) * blockDim.x) {
    const uint64_t b = offsets[i], e = offsets[i + 1];
    uint32_t err = 0;
    if (e < b || e > nnz) {
      err |= kErrOffsets;
      size[i] = 0;
      hash[i] = 0;
    } else {
      const uint64_t s64 = e - b;
      const uint32_t s = s64 > 0xFFFFFFFFull ? 0xFFFFFFFFu : uint32_t(s64);
      if (s == 0) err |= kErrEmpty;
      uint32_t* out = sm + b;
      if (s <= kRegSort) {
        uint32_t r[kRegSort];
        for (uint32_t j = 0; j < s; ++j) {
          uint32_t v = members[b + j];
          if (v >= n_nodes) err |= kErrBadId;
          uint32_t k = j;
          while (k > 0 && r[k - 1] > v) {
            r[k] = r[k - 1];
            --k;
          }
          r[k] = v;
        }
        for (uint32_t j = 0; j < s; ++j) out[j] = r[j];
      } else {
        for (uint32_t j = 0; j < s; ++j) {
          uint32_t v = members[b + j];
          if (v >= n_nodes) err |= kErrBadId;
          uint32_t k = j;
          while (k > 0 && out[k - 1] > v) {
            out[k] = out[k - 1];
            --k;
          }
          out[k] = v;
        }
      }
      for (uint32_t j = 1; j < s; ++j)
        if (out[j] == out[j - 1]) err |= kErrRepeat;
      size[i] = s;
      hash[i] = tuple_hash(out, s);
    }
    if (err) {
      atomicOr(&flags->err, err);
      atomicMin(&flags->err_edge, uint32_t(i < 0xFFFFFFFFull ? i : 0xFFFFFFFEull));
    }
  }
}

__device__ inline bool same_tuple(const uint32_t* sm, const uint64_t* off, const uint32_t* size,
                                  const unsigned long long* hash, uint64_t a, uint64_t b) {
  if (size[a] != size[b] || hash[a] != hash[b]) return false;
  const uint32_t* x = sm + off[a];
  const uint32_t* y = sm + off[b];
  for (uint32_t j = 0; j < size[a]; ++j)
    if (x[j] != y[j]) return false;
  return true;
}

// Insert every hyperedge of size >= 2 into a table of edge indices; equal
// tuples meet in one slot, which keeps the smallest index (first occurrence).
__global__ void k_dedup_insert(const uint32_t* __restrict__ sm, const uint64_t* __restrict__ off,
                               const uint32_t* __restrict__ size, const unsigned long long* __restrict__ hash,
                               uint64_t n_edges, uint32_t* slots, unsigned long long mask) {
  for (uint64_t i = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n_edges;
       i += uint64_t(gridDim.x) * blockDim.x) {
    if (size[i] < 2) continue;
    unsigned long long pos = hash[i] & mask;
    while (true) {
      uint32_t cur = slots[pos];
      if (cur == kEmpty32) {
        uint32_t prev = atomicCAS(&slots[pos], kEmpty32, uint32_t(i));
        if (prev == kEmpty32) break;
        cur = prev;
      }
      if (same_tuple(sm, off, size, hash, cur, i)) {
        atomicMin(&slots[pos], uint32_t(i));
        break;
      }
      pos = (pos + 1) & mask;
    }
  }
}

// Flags of first occurrences, per size class, and the member counts of the
// unique hyperedges (for the member offsets of the unique list).
__global__ void k_first_flags(const uint32_t* __restrict__ sm, const uint64_t* __restrict__ off,
                              const uint32_t* __restrict__ size, const unsigned long long* __restrict__ hash,
                              uint64_t n_edges, const uint32_t* __restrict__ slots, unsigned long long mask,
                              uint32_t* f_all, uint32_t* f2, uint32_t* f3, uint32_t* f4,
                              unsigned long long* msize, DevFlags* flags) {
  unsigned long long singles = 0, dups = 0;
  for (uint64_t i = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n_edges;
       i += uint64_t(gridDim.x) * blockDim.x) {
    const uint32_t s = size[i];
    bool first = false;
    if (s >= 2) {
      unsigned long long pos = hash[i] & mask;
      while (true) {
        uint32_t cur = slots[pos];
        if (cur == kEmpty32) break;  // cannot happen: i was inserted
        if (same_tuple(sm, off, size, hash, cur, i)) {
          first = (cur == uint32_t(i));
          break;
        }
        pos = (pos + 1) & mask;
      }
      if (!first) ++dups;
    } else if (s == 1) {
      ++singles;
    }
    f_all[i] = first;
    f2[i] = first && s == 2;
    f3[i] = first && s == 3;
    f4[i] = first && s == 4;
    msize[i] = first ? s : 0;
  }
  if (singles) atomicAdd(&flags->singletons, singles);
  if (dups) atomicAdd(&flags->duplicates, dups);
}

__global__ void k_gather(const uint32_t* __restrict__ sm, const uint64_t* __restrict__ off,
                         const uint32_t* __restrict__ size, uint64_t n_edges, const uint32_t* __restrict__ f_all,
                         const uint32_t* __restrict__ p_all, const uint32_t* __restrict__ p2,
                         const uint32_t* __restrict__ p3, const uint32_t* __restrict__ p4,
                         const unsigned long long* __restrict__ moff, uint32_t* e2, uint32_t* e3, uint32_t* e4,
                         uint32_t* all_members, unsigned long long* all_off) {
  for (uint64_t i = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n_edges;
       i += uint64_t(gridDim.x) * blockDim.x) {
    if (!f_all[i]) continue;
    const uint32_t s = size[i];
    const uint32_t* m = sm + off[i];
    if (s == 2) {
      e2[2ull * p2[i]] = m[0];
      e2[2ull * p2[i] + 1] = m[1];
    } else if (s == 3) {
      for (int j = 0; j < 3; ++j) e3[3ull * p3[i] + j] = m[j];
    } else if (s == 4) {
      for (int j = 0; j < 4; ++j) e4[4ull * p4[i] + j] = m[j];
    }
    const unsigned long long mo = moff[i];
    for (uint32_t j = 0; j < s; ++j) all_members[mo + j] = m[j];
    all_off[p_all[i]] = mo;
  }
}

__global__ void k_set64_insert(const uint32_t* __restrict__ e2, uint64_t n, Set64 set) {
  for (uint64_t i = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += uint64_t(gridDim.x) * blockDim.x) {
    const unsigned long long key = key2(e2[2 * i], e2[2 * i + 1]);
    unsigned long long pos = mix64(key) & set.mask;
    while (atomicCAS(set.slot + pos, kEmpty64, key) != kEmpty64) pos = (pos + 1) & set.mask;
  }
}

// Keys are unique, so a slot is claimed by its high word alone; the low word
// is written by the claimant.  No kernel reads the set while it is built.
template <int J>
__global__ void k_set128_insert(const uint32_t* __restrict__ e, uint64_t n, Set128 set) {
  for (uint64_t i = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += uint64_t(gridDim.x) * blockDim.x) {
    const uint32_t* t = e + J * i;
    const Key128 key = (J == 3) ? key3(t[0], t[1], t[2]) : key4(t[0], t[1], t[2], t[3]);
    unsigned long long pos = hash128(key) & set.mask;
    while (atomicCAS(set.slot + 2 * pos, kEmpty64, key.hi) != kEmpty64) pos = (pos + 1) & set.mask;
    set.slot[2 * pos + 1] = key.lo;
  }
}

__global__ void k_pair_keys(const uint32_t* __restrict__ e2, uint64_t n, int bits_per_node,
                            unsigned long long* keys, uint32_t* vals, uint32_t* deg) {
  for (uint64_t i = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += uint64_t(gridDim.x) * blockDim.x) {
    const uint32_t a = e2[2 * i], b = e2[2 * i + 1];
    keys[2 * i] = ((unsigned long long)a << bits_per_node) | b;
    keys[2 * i + 1] = ((unsigned long long)b << bits_per_node) | a;
    vals[2 * i] = uint32_t(i);
    vals[2 * i + 1] = uint32_t(i);
    atomicAdd(&deg[a], 1u);
    atomicAdd(&deg[b], 1u);
  }
}

__global__ void k_pair_adj(const unsigned long long* __restrict__ keys, uint64_t n, unsigned long long low_mask,
                           uint32_t* adj) {
  for (uint64_t i = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += uint64_t(gridDim.x) * blockDim.x)
    adj[i] = uint32_t(keys[i] & low_mask);
}

__global__ void k_max(const uint32_t* __restrict__ v, uint64_t n, uint32_t* out) {
  uint32_t m = 0;
  for (uint64_t i = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += uint64_t(gridDim.x) * blockDim.x)
    m = max(m, v[i]);
  for (int d = kWave / 2; d > 0; d >>= 1) m = max(m, uint32_t(__shfl_xor(int(m), d, kWave)));
  if ((threadIdx.x & (kWave - 1)) == 0) atomicMax(out, m);
}

template <int J>
__global__ void k_incidence_count(const uint32_t* __restrict__ e, uint64_t n, uint32_t* deg) {
  for (uint64_t i = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += uint64_t(gridDim.x) * blockDim.x)
    for (int j = 0; j < J; ++j) atomicAdd(&deg[e[J * i + j]], 1u);
}

template <int J>
__global__ void k_incidence_fill(const uint32_t* __restrict__ e, uint64_t n, uint32_t* cursor, uint32_t* idx) {
  for (uint64_t i = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += uint64_t(gridDim.x) * blockDim.x)
    for (int j = 0; j < J; ++j) idx[atomicAdd(&cursor[e[J * i + j]], 1u)] = uint32_t(i);
}

__global__ void k_bits(const uint32_t* __restrict__ e2, uint64_t n, uint32_t words, uint32_t* bits) {
  for (uint64_t i = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += uint64_t(gridDim.x) * blockDim.x) {
    const uint32_t a = e2[2 * i], b = e2[2 * i + 1];
    atomicOr(&bits[uint64_t(a) * words + (b >> 5)], 1u << (b & 31));
    atomicOr(&bits[uint64_t(b) * words + (a >> 5)], 1u << (a & 31));
  }
}

unsigned grid_for(uint64_t n, unsigned block = 256) {
  uint64_t g = (n + block - 1) / block;
  if (g < 1) g = 1;
  if (g > 16384) g = 16384;
  return unsigned(g);
}

// RAII holder for temporary device buffers of the build
struct Temps {
  std::vector<void*> ptrs;
  ~Temps() {
    for (void* p : ptrs) dfree(p);
  }
  template <typename T>
  int get(T** p, uint64_t count) {
    void* q = nullptr;
    HM_TRY(dalloc(&q, size_t(count ? count : 1) * sizeof(T)));
    ptrs.push_back(q);
    *p = static_cast<T*>(q);
    return HM_OK;
  }
};

template <typename T>
int owned(T** p, uint64_t count) {
  void* q = nullptr;
  HM_TRY(dalloc(&q, size_t(count ? count : 1) * sizeof(T)));
  *p = static_cast<T*>(q);
  return HM_OK;
}

int node_bits(uint32_t n_nodes) {
  int b = 1;
  while (b < 32 && (1ull << b) < n_nodes) ++b;
  return b;
}

int build_csr_from_incidence(hm_graph* H, const uint32_t* e, uint64_t n, int J, uint32_t** off_out,
                             uint32_t** idx_out, uint32_t* max_deg, hipStream_t st) {
  Temps tmp;
  uint32_t *deg = nullptr, *cursor = nullptr, *dmax = nullptr;
  HM_TRY(tmp.get(&deg, H->n_nodes));
  HM_TRY(tmp.get(&dmax, 1));
  HM_TRY(owned(off_out, uint64_t(H->n_nodes) + 1));
  HM_TRY(owned(idx_out, uint64_t(J) * n));
  HM_TRY(fill_u32(deg, 0, H->n_nodes, st));
  HM_TRY(fill_u32(dmax, 0, 1, st));
  if (n) {
    if (J == 3)
      k_incidence_count<3><<<grid_for(n), 256, 0, st>>>(e, n, deg);
    else
      k_incidence_count<4><<<grid_for(n), 256, 0, st>>>(e, n, deg);
    HM_HIP(hipGetLastError());
  }
  HM_TRY(scan_exclusive_u32(deg, *off_out, H->n_nodes, *off_out + H->n_nodes, st));
  k_max<<<grid_for(H->n_nodes), 256, 0, st>>>(deg, H->n_nodes, dmax);
  HM_HIP(hipGetLastError());
  HM_TRY(tmp.get(&cursor, H->n_nodes));
  HM_HIP(hipMemcpyAsync(cursor, *off_out, sizeof(uint32_t) * H->n_nodes, hipMemcpyDeviceToDevice, st));
  if (n) {
    if (J == 3)
      k_incidence_fill<3><<<grid_for(n), 256, 0, st>>>(e, n, cursor, *idx_out);
    else
      k_incidence_fill<4><<<grid_for(n), 256, 0, st>>>(e, n, cursor, *idx_out);
    HM_HIP(hipGetLastError());
  }
  HM_HIP(hipMemcpyAsync(max_deg, dmax, sizeof(uint32_t), hipMemcpyDeviceToHost, st));
  return HM_OK;
}

int build(hm_graph* H, const uint32_t* members_in, const uint64_t* offsets_in, uint64_t n_edges, int mem_kind,
          hipStream_t st) {
  Temps tmp;
  uint64_t nnz = 0;
  const uint32_t* members = members_in;
  const uint64_t* offsets = offsets_in;
  if (mem_kind == HM_MEM_HOST) {
    nnz = offsets_in[n_edges];
    uint32_t* dm = nullptr;
    uint64_t* doff = nullptr;
    HM_TRY(tmp.get(&dm, nnz));
    HM_TRY(tmp.get(&doff, n_edges + 1));
    if (nnz) HM_HIP(hipMemcpyAsync(dm, members_in, nnz * sizeof(uint32_t), hipMemcpyHostToDevice, st));
    HM_HIP(hipMemcpyAsync(doff, offsets_in, (n_edges + 1) * sizeof(uint64_t), hipMemcpyHostToDevice, st));
    members = dm;
    offsets = doff;
  } else {
    uint64_t first = 0;
    HM_HIP(hipMemcpyAsync(&first, offsets_in, sizeof(uint64_t), hipMemcpyDeviceToHost, st));
    HM_HIP(hipMemcpyAsync(&nnz, offsets_in + n_edges, sizeof(uint64_t), hipMemcpyDeviceToHost, st));
    HM_HIP(hipStreamSynchronize(st));
    if (first != 0) {
      set_error("offsets[0] must be 0");
      return HM_EINVAL;
    }
  }
  if (mem_kind == HM_MEM_HOST && offsets_in[0] != 0) {
    set_error("offsets[0] must be 0");
    return HM_EINVAL;
  }
  if (nnz > 0xFFFFFFFFull) {
    set_error("more than 2^32-1 incidences are not supported");
    return HM_EUNSUPPORTED;
  }
  const uint64_t E = n_edges;
  DevFlags* flags = nullptr;
  uint32_t *sm = nullptr, *size = nullptr;
  unsigned long long* hash = nullptr;
  HM_TRY(tmp.get(&flags, 1));
  HM_TRY(tmp.get(&sm, nnz));
  HM_TRY(tmp.get(&size, E));
  HM_TRY(tmp.get(&hash, E));
  DevFlags init{0, 0xFFFFFFFFu, 0, 0, 0, 0};
  HM_HIP(hipMemcpyAsync(flags, &init, sizeof(init), hipMemcpyHostToDevice, st));
  if (E) {
    k_prepare<<<grid_for(E), 256, 0, st>>>(members, offsets, E, nnz, H->n_nodes, sm, size, hash, flags);
    HM_HIP(hipGetLastError());
  }
  DevFlags got;
  HM_HIP(hipMemcpyAsync(&got, flags, sizeof(got), hipMemcpyDeviceToHost, st));
  HM_HIP(hipStreamSynchronize(st));
  if (got.err) {
    const char* what = (got.err & kErrOffsets) ? "offsets decrease or exceed offsets[n_edges]"
                       : (got.err & kErrEmpty) ? "an empty hyperedge"
                       : (got.err & kErrBadId) ? "a node id >= n_nodes"
                                               : "a node repeated inside a hyperedge";
    set_error("invalid hypergraph: %s (first offending hyperedge index %u)", what, got.err_edge);
    return HM_EINVAL;
  }

  // collapse repeated hyperedges onto first occurrences
  const unsigned long long cap = pow2_capacity(E);
  uint32_t* slots = nullptr;
  HM_TRY(tmp.get(&slots, cap));
  HM_TRY(fill_u32(slots, kEmpty32, cap, st));
  uint32_t *f_all, *f2, *f3, *f4, *p_all, *p2, *p3, *p4, *tot;
  unsigned long long *msize, *moff;
  HM_TRY(tmp.get(&f_all, E));
  HM_TRY(tmp.get(&f2, E));
  HM_TRY(tmp.get(&f3, E));
  HM_TRY(tmp.get(&f4, E));
  HM_TRY(tmp.get(&p_all, E));
  HM_TRY(tmp.get(&p2, E));
  HM_TRY(tmp.get(&p3, E));
  HM_TRY(tmp.get(&p4, E));
  HM_TRY(tmp.get(&tot, 4));
  HM_TRY(tmp.get(&msize, E + 1));
  HM_TRY(tmp.get(&moff, E + 1));
  HM_TRY(fill_u32(tot, 0, 4, st));
  if (E) {
    k_dedup_insert<<<grid_for(E), 256, 0, st>>>(sm, offsets, size, hash, E, slots, cap - 1);
    HM_HIP(hipGetLastError());
    k_first_flags<<<grid_for(E), 256, 0, st>>>(sm, offsets, size, hash, E, slots, cap - 1, f_all, f2, f3, f4,
                                               msize, flags);
    HM_HIP(hipGetLastError());
    HM_TRY(scan_exclusive_u32(f_all, p_all, E, tot + 0, st));
    HM_TRY(scan_exclusive_u32(f2, p2, E, tot + 1, st));
    HM_TRY(scan_exclusive_u32(f3, p3, E, tot + 2, st));
    HM_TRY(scan_exclusive_u32(f4, p4, E, tot + 3, st));
    HM_TRY(fill_u64(msize + E, 0, 1, st));
    HM_TRY(scan_exclusive_u64(msize, moff, E + 1, st));
  }
  uint32_t totals[4] = {0, 0, 0, 0};
  unsigned long long n_members = 0;
  HM_HIP(hipMemcpyAsync(totals, tot, sizeof(totals), hipMemcpyDeviceToHost, st));
  if (E) HM_HIP(hipMemcpyAsync(&n_members, moff + E, sizeof(n_members), hipMemcpyDeviceToHost, st));
  HM_HIP(hipMemcpyAsync(&got, flags, sizeof(got), hipMemcpyDeviceToHost, st));
  HM_HIP(hipStreamSynchronize(st));
  H->n_unique = totals[0];
  H->n_by_size[2] = totals[1];
  H->n_by_size[3] = totals[2];
  H->n_by_size[4] = totals[3];
  H->n_by_size[5] = totals[0] - totals[1] - totals[2] - totals[3];
  H->n_singletons = got.singletons;
  H->n_duplicates = got.duplicates;
  H->n_unique_members = n_members;
  const uint64_t n2 = H->n_by_size[2], n3 = H->n_by_size[3], n4 = H->n_by_size[4];

  HM_TRY(owned(&H->e2, 2 * n2));
  HM_TRY(owned(&H->e3, 3 * n3));
  HM_TRY(owned(&H->e4, 4 * n4));
  HM_TRY(owned(&H->all_members, n_members));
  HM_TRY(owned(&H->all_off, H->n_unique + 1));
  if (E) {
    k_gather<<<grid_for(E), 256, 0, st>>>(sm, offsets, size, E, f_all, p_all, p2, p3, p4, moff, H->e2, H->e3, H->e4,
                                          H->all_members, H->all_off);
    HM_HIP(hipGetLastError());
  }
  HM_HIP(hipMemcpyAsync(H->all_off + H->n_unique, &n_members, sizeof(n_members), hipMemcpyHostToDevice, st));
  HM_HIP(hipStreamSynchronize(st));

  // hash sets of hyperedges of size 2, 3, 4
  const unsigned long long c2 = pow2_capacity(n2), c3 = pow2_capacity(n3), c4 = pow2_capacity(n4);
  HM_TRY(owned(&H->hs2.slot, c2));
  HM_TRY(owned(&H->hs3.slot, 2 * c3));
  HM_TRY(owned(&H->hs4.slot, 2 * c4));
  H->hs2.mask = c2 - 1;
  H->hs3.mask = c3 - 1;
  H->hs4.mask = c4 - 1;
  HM_TRY(fill_u64(H->hs2.slot, kEmpty64, c2, st));
  HM_TRY(fill_u64(H->hs3.slot, kEmpty64, 2 * c3, st));
  HM_TRY(fill_u64(H->hs4.slot, kEmpty64, 2 * c4, st));
  if (n2) k_set64_insert<<<grid_for(n2), 256, 0, st>>>(H->e2, n2, H->hs2);
  if (n3) k_set128_insert<3><<<grid_for(n3), 256, 0, st>>>(H->e3, n3, H->hs3);
  if (n4) k_set128_insert<4><<<grid_for(n4), 256, 0, st>>>(H->e4, n4, H->hs4);
  HM_HIP(hipGetLastError());

  // pairwise graph: ascending CSR rows from a radix sort of directed pairs
  {
    const int B = node_bits(H->n_nodes);
    const uint64_t m = 2 * n2;
    unsigned long long *keys, *keys_tmp;
    uint32_t *vals, *vals_tmp, *deg, *dmax;
    HM_TRY(tmp.get(&keys, m));
    HM_TRY(tmp.get(&keys_tmp, m));
    HM_TRY(owned(&H->g2_eid, m));
    vals = H->g2_eid;
    HM_TRY(tmp.get(&vals_tmp, m));
    HM_TRY(tmp.get(&deg, H->n_nodes));
    HM_TRY(tmp.get(&dmax, 1));
    HM_TRY(fill_u32(deg, 0, H->n_nodes, st));
    HM_TRY(fill_u32(dmax, 0, 1, st));
    HM_TRY(owned(&H->g2_off, uint64_t(H->n_nodes) + 1));
    HM_TRY(owned(&H->g2_adj, m));
    if (n2) {
      k_pair_keys<<<grid_for(n2), 256, 0, st>>>(H->e2, n2, B, keys, vals, deg);
      HM_HIP(hipGetLastError());
      HM_TRY(radix_sort_pairs(keys, vals, keys_tmp, vals_tmp, m, 2 * B, st));
      k_pair_adj<<<grid_for(m), 256, 0, st>>>(keys, m, (1ull << B) - 1, H->g2_adj);
      HM_HIP(hipGetLastError());
    }
    HM_TRY(scan_exclusive_u32(deg, H->g2_off, H->n_nodes, H->g2_off + H->n_nodes, st));
    k_max<<<grid_for(H->n_nodes), 256, 0, st>>>(deg, H->n_nodes, dmax);
    HM_HIP(hipGetLastError());
    HM_HIP(hipMemcpyAsync(&H->max_deg2, dmax, sizeof(uint32_t), hipMemcpyDeviceToHost, st));
    HM_HIP(hipStreamSynchronize(st));
  }
  HM_TRY(build_csr_from_incidence(H, H->e3, n3, 3, &H->i3_off, &H->i3_idx, &H->max_deg3, st));
  uint32_t max_deg4 = 0;
  HM_TRY(build_csr_from_incidence(H, H->e4, n4, 4, &H->i4_off, &H->i4_idx, &max_deg4, st));

  if (H->n_nodes <= bitset_max_nodes()) {
    H->words = (H->n_nodes + 31) / 32;
    const uint64_t nw = uint64_t(H->n_nodes) * H->words;
    HM_TRY(owned(&H->bits, nw));
    HM_TRY(fill_u32(H->bits, 0, nw, st));
    if (n2) {
      k_bits<<<grid_for(n2), 256, 0, st>>>(H->e2, n2, H->words, H->bits);
      HM_HIP(hipGetLastError());
    }
  }
  HM_TRY(owned(&H->hist, 4 * 256));
  HM_TRY(owned(&H->sample_hist, 256 + 8));
  HM_TRY(fill_u64(H->sample_hist, 0, 256 + 8, st));
  HM_HIP(hipStreamSynchronize(st));
  return HM_OK;
}

void release(hm_graph* H) {
  dfree(H->e2);
  dfree(H->e3);
  dfree(H->e4);
  dfree(H->all_members);
  dfree(H->all_off);
  dfree(H->hs2.slot);
  dfree(H->hs3.slot);
  dfree(H->hs4.slot);
  dfree(H->g2_off);
  dfree(H->g2_adj);
  dfree(H->g2_eid);
  dfree(H->i3_off);
  dfree(H->i3_idx);
  dfree(H->i4_off);
  dfree(H->i4_idx);
  dfree(H->bits);
  dfree(H->hist);
  dfree(H->sample_hist);
  dfree(H->pl_keys);
  dfree(H->pl_edge);
  dfree(H->ns_tri);
  dfree(H->ns_nbr);
  dfree(H->ns_h3);
  dfree(H->es);
  if (H->null_plan) destroy_null_plan(H->null_plan);
  H->null_plan = nullptr;
  if (H->proposal) destroy_proposal_cache(H->proposal);
  H->proposal = nullptr;
}

}  // namespace
}  // namespace hm

extern "C" {

int hm_graph_create(const uint32_t* members, const uint64_t* offsets, uint64_t n_edges, uint32_t n_nodes,
                    int mem_kind, void* stream, hm_graph** out) {
  if (!out) {
    hm::set_error("out is NULL");
    return HM_EINVAL;
  }
  *out = nullptr;
  if (!offsets || (!members && n_edges > 0)) {
    hm::set_error("members/offsets must not be NULL");
    return HM_EINVAL;
  }
  if (n_nodes == 0 || n_nodes == 0xFFFFFFFFu) {
    hm::set_error("n_nodes must be in [1, 2^32-2]");
    return HM_EINVAL;
  }
  if (mem_kind != HM_MEM_HOST && mem_kind != HM_MEM_DEVICE) {
    hm::set_error("mem_kind must be HM_MEM_HOST or HM_MEM_DEVICE");
    return HM_EINVAL;
  }
  if (n_edges >= 0xFFFFFFFFull) {
    hm::set_error("at most 2^32-2 hyperedges are supported");
    return HM_EUNSUPPORTED;
  }
  hipStream_t st = static_cast<hipStream_t>(stream);
  hm_graph* H = new (std::nothrow) hm_graph();
  if (!H) {
    hm::set_error("host allocation failed");
    return HM_ENOMEM;
  }
  if (hipGetDevice(&H->device) != hipSuccess) {
    delete H;
    hm::set_error("no HIP device");
    return HM_EDEVICE;
  }
  H->n_nodes = n_nodes;
  H->n_input = n_edges;
  int rc = hm::build(H, members, offsets, n_edges, mem_kind, st);
  if (rc != HM_OK) {
    (void)hipStreamSynchronize(st);
    hm::release(H);
    delete H;
    return rc;
  }
  *out = H;
  return HM_OK;
}

int hm_graph_destroy(hm_graph* H) {
  if (!H) return HM_OK;
  (void)hipDeviceSynchronize();
  hm::release(H);
  delete H;
  return HM_OK;
}

int hm_graph_stats(const hm_graph* H, uint64_t* out10) {
  uint64_t* out8 = out10;
  if (!H || !out8) {
    hm::set_error("NULL argument");
    return HM_EINVAL;
  }
  out8[0] = H->n_nodes;
  out8[1] = H->n_by_size[2];
  out8[2] = H->n_by_size[3];
  out8[3] = H->n_by_size[4];
  out8[4] = H->n_by_size[5];
  out8[5] = H->n_input;
  out8[6] = H->n_singletons;
  out8[7] = H->n_duplicates;
  out8[8] = H->n_unique;
  out8[9] = H->n_unique_members;
  return HM_OK;
}

int hm_graph_export(const hm_graph* H, int j, uint32_t* out) {
  if (!H || !out || j < 2 || j > 4) {
    hm::set_error("bad arguments to hm_graph_export");
    return HM_EINVAL;
  }
  const uint32_t* src = j == 2 ? H->e2 : j == 3 ? H->e3 : H->e4;
  const uint64_t n = H->n_by_size[j] * uint64_t(j);
  if (n) HM_HIP(hipMemcpy(out, src, n * sizeof(uint32_t), hipMemcpyDeviceToHost));
  return HM_OK;
}

}  // extern "C"
