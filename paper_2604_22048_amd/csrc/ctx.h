// Handle internals shared by the host translation units of the C ABI.
#pragma once

#include "bsi.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdarg>
#include <cstdio>
#include <string>

struct DevBuf {
  void* p = nullptr;
  size_t n = 0;
};

constexpr int kAuxStreams = 4;

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

// Grow a handle-owned device buffer to at least `bytes` (contents are not kept).
inline int ensure(bsi_handle h, DevBuf& b, size_t bytes) {
  if (bytes <= b.n) return BSI_OK;
  if (b.p) {
    hipError_t e = hipDeviceSynchronize();
    if (e != hipSuccess) return hip_fail(h, e, "workspace sync");
    (void)hipFree(b.p);
    b.p = nullptr;
    b.n = 0;
  }
  const size_t n = std::max<size_t>(bytes, 256);
  hipError_t e = hipMalloc(&b.p, n);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return fail(h, BSI_ENOMEM, "workspace allocation of %zu bytes failed", n);
  }
  b.n = n;
  return BSI_OK;
}

// Enqueue fn(i, stream) for i = 0..n-1 with item 0 on s and the others on
// the handle's auxiliary streams, forked from and joined back into s by
// events, so that the launches of different size classes can run
// concurrently (also inside a captured graph, as parallel branches).
template <typename F>
hipError_t fork_join(bsi_handle h, hipStream_t s, int n, F&& fn) {
  if (n <= 1) return n == 1 ? fn(0, s) : hipSuccess;
  const int n_aux = std::min(n - 1, kAuxStreams);
  hipError_t e = hipEventRecord(h->ev_fork, s);
  for (int i = 0; e == hipSuccess && i < n_aux; ++i) e = hipStreamWaitEvent(h->aux[i], h->ev_fork, 0);
  for (int c = 0; e == hipSuccess && c < n; ++c) e = fn(c, c == 0 ? s : h->aux[(c - 1) % kAuxStreams]);
  for (int i = 0; e == hipSuccess && i < n_aux; ++i) {
    e = hipEventRecord(h->ev_join[i], h->aux[i]);
    if (e == hipSuccess) e = hipStreamWaitEvent(s, h->ev_join[i], 0);
  }
  return e;
}

}  // namespace bsi_host
