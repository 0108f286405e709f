// Exact counts of many hypergraphs in one call (the counts of Algorithms 2
// and 3, as count_exact gives them for one).  The hypergraphs are shared
// among host worker threads, each building, counting and releasing its
// graphs on a stream of its own.  A build ends with the host waiting for the
// graph's validation report, so one thread alone leaves the GPU idle while
// it waits and while it issues the next launches; with several, one graph's
// build runs on the CUs beside another's count.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cstdio>
#include <mutex>
#include <thread>
#include <vector>

#include "hm_internal.h"

namespace hm {
namespace {

constexpr int kMaxWorkers = 16;

// Worker streams per device (default priority, not synchronising with the
// null stream), created on first use and kept for the process.
std::mutex g_worker_mu;
std::vector<std::vector<hipStream_t>> g_worker_streams;

int worker_streams(int device, int n, hipStream_t* out) {
  std::lock_guard<std::mutex> lock(g_worker_mu);
  try {
    if (size_t(device) >= g_worker_streams.size()) g_worker_streams.resize(size_t(device) + 1);
    auto& v = g_worker_streams[size_t(device)];
    v.reserve(kMaxWorkers);
    while (int(v.size()) < n) {
      hipStream_t s = nullptr;
      HM_HIP(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
      v.push_back(s);
    }
    for (int t = 0; t < n; ++t) out[t] = v[size_t(t)];
  } catch (...) {
    set_error("host allocation failed");
    return HM_ENOMEM;
  }
  return HM_OK;
}

// `waiter` waits for everything enqueued so far on each of the n streams.
int join_streams(const hipStream_t* from, int n, hipStream_t waiter) {
  for (int t = 0; t < n; ++t) {
    hipEvent_t ev = nullptr;
    HM_HIP(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
    const hipError_t e1 = hipEventRecord(ev, from[t]);
    const hipError_t e2 = e1 == hipSuccess ? hipStreamWaitEvent(waiter, ev, 0) : e1;
    (void)hipEventDestroy(ev);   // (released once the wait is satisfied)
    HM_HIP(e2);
  }
  return HM_OK;
}

}  // namespace
}  // namespace hm

extern "C" int count_exact_many(int n_graphs, const uint32_t* const* members, const uint64_t* const* offsets,
                                const uint64_t* n_edges, const uint64_t* n_members, const uint32_t* n_nodes,
                                int mem_kind, int k, int64_t* counts, int workers, void* stream) {
  try {
    if (n_graphs < 0) {
      hm::set_error("n_graphs must not be negative");
      return HM_EINVAL;
    }
    if (workers < 1 || workers > hm::kMaxWorkers) {
      hm::set_error("workers must be in [1, %d]", hm::kMaxWorkers);
      return HM_EINVAL;
    }
    const int C = hm_num_classes(k);
    if (C < 0) return C;
    if (n_graphs == 0) return HM_OK;
    if (!members || !offsets || !n_edges || !n_members || !n_nodes || !counts) {
      hm::set_error("count_exact_many: a NULL array");
      return HM_EINVAL;
    }
    int device = 0;
    HM_HIP(hipGetDevice(&device));
    const int T = std::min(workers, n_graphs);
    hipStream_t ws[hm::kMaxWorkers];
    HM_TRY(hm::worker_streams(device, T, ws));
    hipStream_t caller = static_cast<hipStream_t>(stream);
    // the workers start after what the caller enqueued on `stream`
    for (int t = 0; t < T; ++t) HM_TRY(hm::join_streams(&caller, 1, ws[t]));

    std::atomic<int> next{0};
    std::atomic<bool> stop{false};
    int rc[hm::kMaxWorkers], failed[hm::kMaxWorkers];
    char msg[hm::kMaxWorkers][512];
    for (int t = 0; t < T; ++t) {
      rc[t] = HM_OK;
      failed[t] = -1;
      msg[t][0] = 0;
    }
    auto work = [&](int t) {
      if (hipSetDevice(device) != hipSuccess) {
        rc[t] = HM_EDEVICE;
        failed[t] = -1;
        std::snprintf(msg[t], sizeof(msg[t]), "hipSetDevice failed in a worker thread");
        stop = true;
        return;
      }
      while (!stop.load()) {
        const int g = next.fetch_add(1);
        if (g >= n_graphs) break;
        hm_graph* H = nullptr;
        int r = hm_graph_create(members[g], offsets[g], n_edges[g], n_members[g], n_nodes[g], mem_kind, ws[t], &H);
        if (r == HM_OK) r = count_exact(H, k, counts + int64_t(g) * C, ws[t]);
        if (r != HM_OK) std::snprintf(msg[t], sizeof(msg[t]), "%s", hm_last_error());
        if (H) (void)hm_graph_destroy(H);
        if (r != HM_OK) {
          rc[t] = r;
          failed[t] = g;
          stop = true;
          return;
        }
      }
    };
    // the calling thread is worker 0; a worker thread that cannot be started
    // leaves its share to the others (the graphs are taken from one counter)
    std::vector<std::thread> threads;
    try {
      threads.reserve(size_t(T));
      for (int t = 1; t < T; ++t) threads.emplace_back(work, t);
    } catch (...) {
    }
    work(0);
    for (auto& th : threads) th.join();

    // the lowest failing graph among those attempted
    int worst = -1;
    for (int t = 0; t < T; ++t)
      if (rc[t] != HM_OK && (worst < 0 || failed[t] < failed[worst])) worst = t;
    // `stream` waits for every worker's work, also after a failure (the
    // caller's buffers stay in use until then)
    const int jr = hm::join_streams(ws, T, caller);
    if (worst >= 0) {
      if (failed[worst] >= 0)
        hm::set_error("hypergraph %d: %s", failed[worst], msg[worst]);
      else
        hm::set_error("%s", msg[worst]);
      return rc[worst];
    }
    return jr;
  } catch (...) {
    return hm::api_failure();
  }
}
