// Handle internals shared by the host translation units of the C ABI.
//
// Workspace rules (bsi.h, "Workspace, streams and graph capture"):
//   - Every call computes all of its workspace needs on the host and grows
//     the handle's buffers before it enqueues anything (prepare()).  Growth
//     allocates new buffers and retires the old ones; retired buffers stay
//     allocated (work already enqueued by earlier calls may still use them)
//     until bsi_reserve or bsi_destroy frees them after a device
//     synchronisation.  No call synchronises the device.
//   - A call made while its stream is being captured never allocates: if
//     the workspace is too small it fails with BSI_EINVAL before enqueueing
//     anything (bsi_reserve sizes the workspace beforehand).
//   - Host inputs that the device needs (batch plans, shear points) are
//     packed into one pinned, device-mapped staging buffer and copied by a
//     kernel, so a captured call records only kernel nodes.
//   - Calls outside capture record an event at their end; the next call on a
//     different stream waits for it before touching the shared workspace.
#pragma once

#include "bsi.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

struct DevBuf {
  void* p = nullptr;
  size_t n = 0;
};

constexpr int kAuxStreams = 4;
// streams of a forked launch: the caller's and up to kAuxStreams auxiliary
constexpr int kForkStreams = 4;

// An instantiated graph whose replays were enqueued; destroyed once `done`
// (recorded after the last replay) has completed.
struct PendingGraph {
  hipGraphExec_t exec = nullptr;
  hipGraph_t graph = nullptr;
  hipEvent_t done = nullptr;
};

struct bsi_ctx {
  int device = 0;
  int num_cu = 0;
  std::string err;
  hipStream_t own = nullptr;
  hipStream_t aux[kAuxStreams] = {};   // per-class branches of a forked launch
  hipEvent_t ev_fork = nullptr;
  hipEvent_t ev_join[kAuxStreams] = {};
  DevBuf gidx, ggidx, off, bin_off, dh, sqw, chi2, model, state, partial, pts, shear_state, bias_part,
      bias_mc;
  int plan_P[129] = {};   // slot plan per stamp side (0: the default, fewest slots)
  int transform[129] = {};   // render transform per stamp side (BSI_TRANSFORM_*, 0: default)
  // call ordering across streams
  hipEvent_t ev_done = nullptr;
  hipStream_t last_stream = nullptr;
  bool pending = false;
  // pinned, device-mapped staging of host inputs
  void* stage = nullptr;        // host pointer
  void* stage_dev = nullptr;    // its device address
  size_t stage_n = 0;
  hipEvent_t ev_stage = nullptr;
  bool stage_pending = false;
  std::vector<void*> retired;         // replaced device buffers
  std::vector<void*> retired_host;    // replaced staging buffers
  std::vector<PendingGraph> graphs;   // graphs whose replays may still run
  void* scratch = nullptr;   // this device's allocation-free scratch (device address)
  std::string arch;          // device architecture name (tuning cache key)
  std::string tune_cache;    // tuning cache path (empty: none)
};

namespace bsi_host {

// Render transform of stamp side N on handle h: the handle's choice, else
// the default (the FP32 DFT-as-GEMM on the matrix cores, the faster of the
// two at every workload size when measured).
inline int transform_of(const bsi_ctx* h, int N) {
  return h->transform[N] ? h->transform[N] : BSI_TRANSFORM_MFMA;
}

inline int fail(bsi_handle h, int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  if (h) h->err = buf;
  return code;
}

inline int hip_fail(bsi_handle h, hipError_t e, const char* where) {
  return fail(h, BSI_EHIP, "%s: %s", where, hipGetErrorString(e));
}

// True while `s` is being captured into a graph.
inline bool capturing(hipStream_t s) {
  hipStreamCaptureStatus st = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(s, &st) != hipSuccess) {
    (void)hipGetLastError();
    return false;
  }
  return st == hipStreamCaptureStatusActive;
}

// One workspace requirement of a call.
struct Need {
  DevBuf* buf;
  size_t bytes;
};

// Destroy the graphs whose replays have completed.
inline void reap_graphs(bsi_handle h) {
  auto& g = h->graphs;
  for (size_t i = 0; i < g.size();) {
    if (hipEventQuery(g[i].done) == hipSuccess) {
      (void)hipGraphExecDestroy(g[i].exec);
      (void)hipGraphDestroy(g[i].graph);
      (void)hipEventDestroy(g[i].done);
      g[i] = g.back();
      g.pop_back();
    } else {
      ++i;
    }
  }
  (void)hipGetLastError();
}

// Keep an instantiated graph whose replays were just enqueued on s until
// they have run (destroying it while they are in flight is not safe).
inline int keep_graph(bsi_handle h, hipGraphExec_t exec, hipGraph_t graph, hipStream_t s) {
  PendingGraph pg{exec, graph, nullptr};
  hipError_t e = hipEventCreateWithFlags(&pg.done, hipEventDisableTiming);
  if (e == hipSuccess) e = hipEventRecord(pg.done, s);
  if (e != hipSuccess) {
    // cannot track it: wait for the replays, then destroy
    (void)hipStreamSynchronize(s);
    (void)hipGraphExecDestroy(exec);
    (void)hipGraphDestroy(graph);
    if (pg.done) (void)hipEventDestroy(pg.done);
    return hip_fail(h, e, "graph tracking");
  }
  h->graphs.push_back(pg);
  return BSI_OK;
}

// Grow `b` to at least `bytes` (contents are not kept).  The old buffer is
// retired, not freed: earlier calls' work may still read it.
inline int grow(bsi_handle h, DevBuf& b, size_t bytes) {
  if (bytes <= b.n) return BSI_OK;
  const size_t n = std::max<size_t>({bytes, b.n + b.n / 2, 256});
  void* p = nullptr;
  hipError_t e = hipMalloc(&p, n);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return fail(h, BSI_ENOMEM, "workspace allocation of %zu bytes failed", n);
  }
  if (b.p) h->retired.push_back(b.p);
  b.p = p;
  b.n = n;
  return BSI_OK;
}

// Grow the pinned staging buffer to at least `bytes`.
inline int grow_stage(bsi_handle h, size_t bytes) {
  if (bytes <= h->stage_n) return BSI_OK;
  const size_t n = std::max<size_t>({bytes, h->stage_n + h->stage_n / 2, 4096});
  void* p = nullptr;
  hipError_t e = hipHostMalloc(&p, n, hipHostMallocMapped);
  void* d = nullptr;
  if (e == hipSuccess) e = hipHostGetDevicePointer(&d, p, 0);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    if (p) (void)hipHostFree(p);
    return fail(h, BSI_ENOMEM, "staging allocation of %zu bytes failed", n);
  }
  if (h->stage) h->retired_host.push_back(h->stage);
  h->stage = p;
  h->stage_dev = d;
  h->stage_n = n;
  h->stage_pending = false;   // the new buffer has no reader yet
  return BSI_OK;
}

// Start of a call on stream s, after validation and before anything is
// enqueued: size the workspace (and staging) for `needs`, and order the call
// after the handle's previous call when that ran on another stream.
inline int prepare(bsi_handle h, hipStream_t s, bool cap, std::initializer_list<Need> needs,
                   size_t stage_bytes = 0) {
  reap_graphs(h);
  for (const Need& nd : needs) {
    if (nd.bytes <= nd.buf->n) continue;
    if (cap)
      return fail(h, BSI_EINVAL,
                  "workspace of %zu bytes needed under graph capture (reserved %zu): call "
                  "bsi_reserve with larger limits before capturing", nd.bytes, nd.buf->n);
  }
  if (stage_bytes > h->stage_n && cap)
    return fail(h, BSI_EINVAL,
                "staging of %zu bytes needed under graph capture (reserved %zu): call bsi_reserve "
                "with larger limits before capturing", stage_bytes, h->stage_n);
  int rc;
  for (const Need& nd : needs)
    if ((rc = grow(h, *nd.buf, nd.bytes))) return rc;
  if ((rc = grow_stage(h, stage_bytes))) return rc;
  if (!cap && h->pending && h->last_stream != s) {
    hipError_t e = hipStreamWaitEvent(s, h->ev_done, 0);
    if (e != hipSuccess) return hip_fail(h, e, "ordering after the previous call");
  }
  return BSI_OK;
}

// End of a call: remember where it ran (calls under capture are ordered by
// the caller's graph instead).
inline int finish(bsi_handle h, hipStream_t s, bool cap) {
  if (cap) return BSI_OK;
  hipError_t e = hipEventRecord(h->ev_done, s);
  if (e != hipSuccess) return hip_fail(h, e, "end-of-call event");
  h->last_stream = s;
  h->pending = true;
  return BSI_OK;
}

// Host data destined for device workspace.
struct Piece {
  void* dst;          // device
  const void* src;    // host
  size_t bytes;
};

inline size_t stage_size(std::initializer_list<size_t> sizes) {
  size_t t = 0;
  for (size_t b : sizes) t += (b + 15) & ~size_t(15);
  return t;
}

// Tuning cache (autotune.cpp): apply the choices stored at h->tune_cache if
// the file exists and was written by this library version for this device
// (BSI_EINVAL with a message in err for a malformed file); write the
// handle's current choices there.
int load_tune_cache(bsi_ctx* h, std::string& err);
int save_tune_cache(bsi_handle h);

}  // namespace bsi_host

namespace bsi {
// stage.hip: copy n 16-byte words from mapped host memory to device memory.
hipError_t launch_stage_copy(const void* src_dev, void* dst, size_t bytes, hipStream_t s);
}  // namespace bsi

namespace bsi_host {

// Copy host pieces to device workspace through the staging buffer: wait for
// the previous reader of the staging buffer, pack, and enqueue one copy
// kernel per piece (kernel nodes only, so the call can be captured; a
// captured graph reads the staging buffer at each replay).
inline int stage_upload(bsi_handle h, hipStream_t s, bool cap, std::initializer_list<Piece> pieces) {
  size_t total = 0;
  for (const Piece& p : pieces) total += (p.bytes + 15) & ~size_t(15);
  if (total > h->stage_n) return fail(h, BSI_EINVAL, "staging buffer too small (internal)");
  if (h->stage_pending) {
    hipError_t e = hipEventSynchronize(h->ev_stage);
    if (e != hipSuccess) return hip_fail(h, e, "staging reuse");
    h->stage_pending = false;
  }
  size_t o = 0;
  for (const Piece& p : pieces) {
    if (p.bytes) std::memcpy(static_cast<char*>(h->stage) + o, p.src, p.bytes);
    hipError_t e = bsi::launch_stage_copy(static_cast<const char*>(h->stage_dev) + o, p.dst, p.bytes, s);
    if (e != hipSuccess) return hip_fail(h, e, "staging copy");
    o += (p.bytes + 15) & ~size_t(15);
  }
  if (!cap) {
    hipError_t e = hipEventRecord(h->ev_stage, s);
    if (e != hipSuccess) return hip_fail(h, e, "staging event");
    h->stage_pending = true;
  }
  return BSI_OK;
}

// Enqueue fn(i, stream) for i = 0..n-1 on s and the handle's auxiliary
// streams (at most kForkStreams streams in all), forked from and joined back
// into s by events, so that the launches of different size classes run
// concurrently.  cost(i) estimates item i's duration: the items are enqueued
// in descending cost, each on the stream with the least estimated cost so
// far, so the longest runs on s and the shortest share a stream.  Used
// outside stream capture only: a capture of the fork (with the executable
// kept alive until its replays had run) still ended in a host segmentation
// fault inside the call, so every capture records the launches in sequence
// on one stream instead.
template <typename F, typename Cost>
hipError_t fork_join(bsi_handle h, hipStream_t s, int n, F&& fn, Cost&& cost) {
  if (n <= 1) return n == 1 ? fn(0, s) : hipSuccess;
  const int ns = std::min(n, kForkStreams);
  std::vector<int> order(n);
  for (int i = 0; i < n; ++i) order[i] = i;
  std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return cost(x) > cost(y); });
  std::vector<double> load(ns, 0.0);
  std::vector<int> where(n, 0);
  for (int c : order) {
    int b = 0;
    for (int j = 1; j < ns; ++j)
      if (load[j] < load[b]) b = j;
    where[c] = b;
    load[b] += cost(c);
  }
  hipError_t e = hipEventRecord(h->ev_fork, s);
  for (int i = 0; e == hipSuccess && i < ns - 1; ++i) e = hipStreamWaitEvent(h->aux[i], h->ev_fork, 0);
  for (int c : order) {
    if (e != hipSuccess) break;
    e = fn(c, where[c] == 0 ? s : h->aux[where[c] - 1]);
  }
  for (int i = 0; e == hipSuccess && i < ns - 1; ++i) {
    e = hipEventRecord(h->ev_join[i], h->aux[i]);
    if (e == hipSuccess) e = hipStreamWaitEvent(s, h->ev_join[i], 0);
  }
  return e;
}

}  // namespace bsi_host
