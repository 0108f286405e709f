// Isomorphism classes of k-node patterns and the pattern -> class lookup
// table (Section 4.3, Fig. 3a): every labelled pattern of interactions among
// k nodes is mapped to its class, so classifying an observed sub-hypergraph
// is one table read.  Built once per process on the host, copied per device.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cstdarg>
#include <cstring>
#include <map>
#include <unordered_map>
#include <atomic>
#include <mutex>
#include <new>
#include <numeric>
#include <vector>

#include "hm_internal.h"

namespace hm {

namespace {

thread_local char g_err[512] = "";

struct Subsets {
  std::vector<int> masks;  // subsets of {0..k-1} with >= 2 members, ascending mask
};

Subsets subsets_of(int k) {
  Subsets s;
  for (int m = 0; m < (1 << k); ++m)
    if (__builtin_popcount(m) >= 2) s.masks.push_back(m);
  return s;
}

bool connected(uint32_t pattern, int k, const Subsets& s) {
  // grow the component of node 0 until it stops changing
  unsigned covered = 0;
  for (size_t b = 0; b < s.masks.size(); ++b)
    if (pattern >> b & 1u) covered |= unsigned(s.masks[b]);
  if (covered != (1u << k) - 1) return false;
  unsigned comp = 1u;
  bool grew = true;
  while (grew) {
    grew = false;
    for (size_t b = 0; b < s.masks.size(); ++b) {
      unsigned m = unsigned(s.masks[b]);
      if ((pattern >> b & 1u) && (m & comp) && (m & ~comp)) {
        comp |= m;
        grew = true;
      }
    }
  }
  return comp == (1u << k) - 1;
}

uint32_t relabel(uint32_t pattern, const std::array<int, 4>& perm, int k, const Subsets& s,
                 const std::vector<int>& index_of_mask) {
  uint32_t out = 0;
  for (size_t b = 0; b < s.masks.size(); ++b) {
    if (!(pattern >> b & 1u)) continue;
    int img = 0;
    for (int i = 0; i < k; ++i)
      if (s.masks[b] >> i & 1) img |= 1 << perm[i];
    out |= 1u << index_of_mask[img];
  }
  return out;
}

ClassTables build() {
  ClassTables t;
  std::memset(&t, 0, sizeof(t));
  for (int k = 3; k <= 4; ++k) {
    const Subsets s = subsets_of(k);
    std::vector<int> index_of_mask(1 << k, -1);
    for (size_t b = 0; b < s.masks.size(); ++b) index_of_mask[s.masks[b]] = int(b);
    const uint32_t n_patterns = 1u << s.masks.size();
    std::vector<std::array<int, 4>> perms;
    std::array<int, 4> p{0, 1, 2, 3};
    do {
      perms.push_back(p);
    } while (std::next_permutation(p.begin(), p.begin() + k));
    std::vector<uint32_t> canon(n_patterns, 0xFFFFFFFFu);
    std::vector<uint32_t> classes;
    for (uint32_t q = 0; q < n_patterns; ++q) {
      if (!connected(q, k, s)) continue;
      uint32_t best = 0xFFFFFFFFu;
      for (const auto& pm : perms) best = std::min(best, relabel(q, pm, k, s, index_of_mask));
      canon[q] = best;
      classes.push_back(best);
    }
    std::sort(classes.begin(), classes.end());
    classes.erase(std::unique(classes.begin(), classes.end()), classes.end());
    t.n_classes[k] = int(classes.size());
    uint8_t* lut = (k == 3) ? t.lut3 : t.lut4;
    for (uint32_t q = 0; q < n_patterns; ++q) {
      if (canon[q] == 0xFFFFFFFFu) {
        lut[q] = 0xFF;
        continue;
      }
      lut[q] = uint8_t(std::lower_bound(classes.begin(), classes.end(), canon[q]) - classes.begin());
    }
    for (size_t c = 0; c < classes.size(); ++c) {
      t.canon[k][c] = classes[c];
      int mc = 0, cm = 0;
      for (size_t b = 0; b < s.masks.size(); ++b) {
        if (!(classes[c] >> b & 1u)) continue;
        int sz = __builtin_popcount(s.masks[b]);
        if (sz > mc) {
          mc = sz;
          cm = 1;
        } else if (sz == mc) {
          ++cm;
        }
      }
      t.maxcard[k][c] = uint8_t(mc);
      t.countmax[k][c] = uint8_t(cm);
    }
  }
  return t;
}

std::mutex g_lut_mutex;
std::atomic<uint32_t> g_bitset_max_nodes{kBitsetMaxNodes};
std::vector<uint8_t*> g_device_luts;  // per device: lut4 (2048) + lut3 (16)

}  // namespace

void set_error(const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof(g_err), fmt, ap);
  va_end(ap);
}

const char* last_error() { return g_err; }

int api_failure() {
  try {
    throw;
  } catch (const std::bad_alloc&) {
    set_error("host allocation failed");
    return HM_ENOMEM;
  } catch (...) {
    set_error("internal error: an exception reached the C ABI");
    return HM_EINTERNAL;
  }
}

uint32_t bitset_max_nodes() { return g_bitset_max_nodes.load(); }
std::atomic<uint32_t> g_sample_chunk_scale{1};
uint32_t sample_chunk_scale() { return g_sample_chunk_scale.load(); }
std::atomic<uint64_t> g_one_pass_max_edges{kOnePassMaxEdges};
uint64_t one_pass_max_edges() { return g_one_pass_max_edges.load(); }
std::atomic<uint32_t> g_hub_min_degree{kHubMinDegree};
uint32_t hub_min_degree() { return g_hub_min_degree.load(); }
std::atomic<int> g_dedup_tag_bits{32};
int dedup_tag_bits() { return g_dedup_tag_bits.load(); }

const ClassTables& class_tables() {
  static const ClassTables t = build();
  return t;
}

int device_luts(int device, const uint8_t** lut4, const uint8_t** lut3) {
  std::lock_guard<std::mutex> lock(g_lut_mutex);
  if (device < 0) {
    set_error("bad device %d", device);
    return HM_EINVAL;
  }
  if (size_t(device) >= g_device_luts.size()) g_device_luts.resize(size_t(device) + 1, nullptr);
  if (!g_device_luts[size_t(device)]) {
    const ClassTables& t = class_tables();
    uint8_t host[2048 + 16];
    std::memcpy(host, t.lut4, 2048);
    std::memcpy(host + 2048, t.lut3, 16);
    void* p = nullptr;
    HM_TRY(dalloc(&p, sizeof(host)));
    HM_HIP(hipMemcpy(p, host, sizeof(host), hipMemcpyHostToDevice));
    g_device_luts[size_t(device)] = static_cast<uint8_t*>(p);
  }
  *lut4 = g_device_luts[size_t(device)];
  *lut3 = g_device_luts[size_t(device)] + 2048;
  return HM_OK;
}

// Device memory cache: blocks are rounded up to a power of two and, when
// released, kept on a free list of their (device, size class) for the next
// allocation of that class instead of being returned to the runtime.  A
// block released with dfree is assumed idle (its users were synchronised);
// one released with dfree_on stays pending until an event recorded on the
// given stream after its last use has completed, so it is never handed out
// while work enqueued before the release may still touch it.
namespace {
struct BlockInfo {
  int device;
  size_t bytes;
  bool filled = false;   // every byte 0xFF once its release has completed
};
// the blocks of one dfree_on call, free once its event has completed
struct Pending {
  hipEvent_t ev;
  int device;
  std::vector<std::pair<void*, BlockInfo>> blocks;
};
std::mutex g_pool_mu;
std::map<std::pair<int, size_t>, std::vector<void*>> g_free;
std::map<std::pair<int, size_t>, std::vector<void*>> g_free_filled;   // idle blocks of all-0xFF bytes
std::unordered_map<void*, BlockInfo> g_live;
std::vector<Pending> g_pending;
std::map<int, std::vector<hipEvent_t>> g_events;   // idle events per device
size_t g_cached_bytes = 0;
constexpr size_t kMaxCachedBytes = size_t(8) << 30;

size_t size_class(size_t bytes) {
  size_t c = 256;
  while (c < bytes) c <<= 1;
  return c;
}

// caller holds g_pool_mu
void cache_block(void* p, const BlockInfo& info) {
  if (g_cached_bytes + info.bytes > kMaxCachedBytes) {
    (void)hipFree(p);
    return;
  }
  (info.filled ? g_free_filled : g_free)[{info.device, info.bytes}].push_back(p);
  g_cached_bytes += info.bytes;
}

// caller holds g_pool_mu: pending blocks whose event has completed become
// free (one query per release batch)
void reap_pending() {
  for (size_t i = 0; i < g_pending.size();) {
    Pending& q = g_pending[i];
    if (hipEventQuery(q.ev) == hipSuccess) {
      for (auto& b : q.blocks) cache_block(b.first, b.second);
      g_events[q.device].push_back(q.ev);
      q = std::move(g_pending.back());
      g_pending.pop_back();
    } else {
      ++i;
    }
  }
  (void)hipGetLastError();
}

// caller holds g_pool_mu: a cached block of (dev, cls) (of all-0xFF bytes
// when filled), or null
void* take_cached(int dev, size_t cls, bool filled = false) {
  auto& free = filled ? g_free_filled : g_free;
  auto it = free.find({dev, cls});
  if (it == free.end() || it->second.empty()) return nullptr;
  void* p = it->second.back();
  it->second.pop_back();
  g_cached_bytes -= cls;
  g_live[p] = BlockInfo{dev, cls};
  return p;
}
}  // namespace

int dalloc(void** p, size_t bytes) {
  *p = nullptr;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) {
    set_error("hipGetDevice failed");
    return HM_EDEVICE;
  }
  const size_t cls = size_class(bytes ? bytes : 1);
  {
    // a cached block, else one whose release has completed since
    std::lock_guard<std::mutex> lock(g_pool_mu);
    *p = take_cached(dev, cls);
    if (!*p && !g_pending.empty()) {
      reap_pending();
      *p = take_cached(dev, cls);
    }
    if (*p) return HM_OK;
  }
  hipError_t e = hipMalloc(p, cls);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    *p = nullptr;
    set_error("hipMalloc(%zu) failed: %s", cls, hipGetErrorString(e));
    return e == hipErrorOutOfMemory ? HM_ENOMEM : HM_EDEVICE;
  }
  std::lock_guard<std::mutex> lock(g_pool_mu);
  g_live[*p] = BlockInfo{dev, cls};
  return HM_OK;
}

int dalloc_filled(void** p, size_t bytes, bool* filled) {
  *p = nullptr;
  *filled = false;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) {
    set_error("hipGetDevice failed");
    return HM_EDEVICE;
  }
  const size_t cls = size_class(bytes ? bytes : 1);
  {
    std::lock_guard<std::mutex> lock(g_pool_mu);
    *p = take_cached(dev, cls, true);
    if (!*p && !g_pending.empty()) {
      reap_pending();
      *p = take_cached(dev, cls, true);
    }
    if (*p) {
      *filled = true;
      return HM_OK;
    }
  }
  return dalloc(p, bytes);
}

void mark_filled(void* p) {
  std::lock_guard<std::mutex> lock(g_pool_mu);
  auto it = g_live.find(p);
  if (it != g_live.end()) it->second.filled = true;
}

void dfree(void* p) {
  if (!p) return;
  std::lock_guard<std::mutex> lock(g_pool_mu);
  auto it = g_live.find(p);
  if (it == g_live.end()) return;
  const BlockInfo info = it->second;
  g_live.erase(it);
  cache_block(p, info);
}

void dfree_on(void* const* ps, size_t n, hipStream_t st) {
  std::lock_guard<std::mutex> lock(g_pool_mu);
  std::vector<std::pair<void*, BlockInfo>> blocks;
  for (size_t i = 0; i < n; ++i) {
    if (!ps[i]) continue;
    auto it = g_live.find(ps[i]);
    if (it == g_live.end()) continue;
    blocks.emplace_back(ps[i], it->second);
    g_live.erase(it);
  }
  if (blocks.empty()) return;
  // one event for the batch, shared by its blocks
  const int dev = blocks.front().second.device;
  hipEvent_t ev = nullptr;
  auto& pool = g_events[dev];
  if (!pool.empty()) {
    ev = pool.back();
    pool.pop_back();
  } else if (hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess) {
    (void)hipGetLastError();
    ev = nullptr;
  }
  if (!ev || hipEventRecord(ev, st) != hipSuccess) {
    // no event: wait for the stream instead
    (void)hipGetLastError();
    (void)hipStreamSynchronize(st);
    if (ev) pool.push_back(ev);
    for (auto& b : blocks) cache_block(b.first, b.second);
    return;
  }
  g_pending.push_back(Pending{ev, dev, std::move(blocks)});
}

void dfree_on(void* p, hipStream_t st) { dfree_on(&p, 1, st); }

}  // namespace hm

extern "C" {

const char* hm_last_error(void) { return hm::last_error(); }

const char* hm_version(void) { return "homotif 0.1 (gfx950)"; }

int hm_set_option(int option, int64_t value) {
  try {
    if (option == HM_OPT_BITSET_MAX_NODES) {
      if (value < 0 || value > int64_t(hm::kBitsetMaxNodes)) {
        hm::set_error("HM_OPT_BITSET_MAX_NODES must be in [0, %u]", hm::kBitsetMaxNodes);
        return HM_EINVAL;
      }
      hm::g_bitset_max_nodes.store(uint32_t(value));
      return HM_OK;
    }
    if (option == HM_OPT_SAMPLE_CHUNK_SCALE) {
      if (value < 1 || value > 1024) {
        hm::set_error("HM_OPT_SAMPLE_CHUNK_SCALE must be in [1, 1024]");
        return HM_EINVAL;
      }
      hm::g_sample_chunk_scale.store(uint32_t(value));
      return HM_OK;
    }
    if (option == HM_OPT_ONE_PASS_MAX_EDGES) {
      if (value < 0 || value > int64_t(hm::kOnePassMaxEdges)) {
        hm::set_error("HM_OPT_ONE_PASS_MAX_EDGES must be in [0, %llu]", (unsigned long long)hm::kOnePassMaxEdges);
        return HM_EINVAL;
      }
      hm::g_one_pass_max_edges.store(uint64_t(value));
      return HM_OK;
    }
    if (option == HM_OPT_HUB_MIN_DEGREE) {
      if (value < 0 || value > int64_t(0xFFFFFFFFu)) {
        hm::set_error("HM_OPT_HUB_MIN_DEGREE must be in [0, 2^32 - 1]");
        return HM_EINVAL;
      }
      hm::g_hub_min_degree.store(uint32_t(value));
      return HM_OK;
    }
    if (option == HM_OPT_DEDUP_TAG_BITS) {
      if (value < -1 || value > 32) {
        hm::set_error("HM_OPT_DEDUP_TAG_BITS must be in [-1, 32]");
        return HM_EINVAL;
      }
      hm::g_dedup_tag_bits.store(int(value));
      return HM_OK;
    }
    hm::set_error("unknown option %d", option);
    return HM_EINVAL;
  } catch (...) {
    return hm::api_failure();
  }
}

int hm_get_option(int option, int64_t* value) {
  try {
    if (!value) {
      hm::set_error("value is NULL");
      return HM_EINVAL;
    }
    if (option == HM_OPT_BITSET_MAX_NODES) {
      *value = hm::g_bitset_max_nodes.load();
      return HM_OK;
    }
    if (option == HM_OPT_SAMPLE_CHUNK_SCALE) {
      *value = hm::g_sample_chunk_scale.load();
      return HM_OK;
    }
    if (option == HM_OPT_ONE_PASS_MAX_EDGES) {
      *value = int64_t(hm::g_one_pass_max_edges.load());
      return HM_OK;
    }
    if (option == HM_OPT_HUB_MIN_DEGREE) {
      *value = int64_t(hm::g_hub_min_degree.load());
      return HM_OK;
    }
    if (option == HM_OPT_DEDUP_TAG_BITS) {
      *value = hm::g_dedup_tag_bits.load();
      return HM_OK;
    }
    hm::set_error("unknown option %d", option);
    return HM_EINVAL;
  } catch (...) {
    return hm::api_failure();
  }
}

int hm_num_classes(int k) {
  try {
    if (k != 3 && k != 4) {
      hm::set_error("order %d is not supported (3 or 4)", k);
      return HM_EUNSUPPORTED;
    }
    return hm::class_tables().n_classes[k];
  } catch (...) {
    return hm::api_failure();
  }
}

int hm_class_info(int k, int cls, uint32_t* canon_pattern, int* maxcard, int* countmax) {
  try {
    int n = hm_num_classes(k);
    if (n < 0) return n;
    if (cls < 0 || cls >= n) {
      hm::set_error("class %d out of range [0, %d)", cls, n);
      return HM_EINVAL;
    }
    const hm::ClassTables& t = hm::class_tables();
    if (canon_pattern) *canon_pattern = t.canon[k][cls];
    if (maxcard) *maxcard = t.maxcard[k][cls];
    if (countmax) *countmax = t.countmax[k][cls];
    return HM_OK;
  } catch (...) {
    return hm::api_failure();
  }
}

int hm_pattern_class(int k, uint32_t pattern, int* cls) {
  try {
    int n = hm_num_classes(k);
    if (n < 0) return n;
    if (!cls) {
      hm::set_error("cls is NULL");
      return HM_EINVAL;
    }
    const hm::ClassTables& t = hm::class_tables();
    if (pattern >= (k == 3 ? 16u : 2048u)) {
      hm::set_error("pattern %u out of range for order %d", pattern, k);
      return HM_EINVAL;
    }
    uint8_t c = (k == 3) ? t.lut3[pattern] : t.lut4[pattern];
    *cls = c == 0xFF ? -1 : int(c);
    return HM_OK;
  } catch (...) {
    return hm::api_failure();
  }
}

}  // extern "C"
