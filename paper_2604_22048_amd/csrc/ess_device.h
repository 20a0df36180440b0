// Multi-chain effective sample size and R-hat of one parameter, computed by
// one whole workgroup of 256 threads (Section 4.1 diagnostics):
// autocorrelations combined across chains, Geyer's initial monotone
// sequence of pair sums, no rank normalisation, tau floored at
// 1 / log10(M n) (so ESS <= M n log10(M n)); classic R-hat.  The M x n draws
// are staged in LDS as float64.  Chain means and variances are block
// reductions; lags are computed 64 at a time (each lag's sum split over the
// four waves by draw index mod 4, partials added in wave order) until the
// pair sums turn non-positive.  Every reduction has a fixed order.
#pragma once

#include "bsi_device.h"

namespace bsi {

struct EssShared {
  double mean_c[16], var_c[16];
  double part[4][64];   // per-wave partials (block sums, lag sums)
  double rho[64];
  double W, vp;
  int done;
};

// Block sum of one value per thread, in a fixed order (waves in order);
// valid in every thread on return.
__device__ inline double ess_block_sum(double x, EssShared& es) {
  x = wave_sum(x);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) es.part[threadIdx.x >> 6][0] = x;
  __syncthreads();
  return ((es.part[0][0] + es.part[1][0]) + es.part[2][0]) + es.part[3][0];
}

// Draw s of chain c: src[(c * stride + s) * P + par], c < C <= 16, s < n,
// n >= 2.  xs: LDS double[C n]; es: LDS scratch.  Every thread of the
// workgroup must call; the results are valid in thread 0.
__device__ inline void ess_one_param(const float* __restrict__ src, int C, int n, int stride, int P,
                                     int par, double* xs, EssShared& es, float& ess_out,
                                     float& rhat_out) {
  const int tid = threadIdx.x;
  for (int t = tid; t < C * n; t += blockDim.x) {
    const int c = t / n, s = t - c * n;
    xs[t] = (double)src[((int64_t)c * stride + s) * P + par];
  }
  __syncthreads();
  for (int c = 0; c < C; ++c) {
    const double* xc = xs + c * n;
    double a = 0.0;
    for (int s = tid; s < n; s += blockDim.x) a += xc[s];
    const double m = ess_block_sum(a, es) / n;
    double v = 0.0;
    for (int s = tid; s < n; s += blockDim.x) {
      const double d = xc[s] - m;
      v += d * d;
    }
    v = ess_block_sum(v, es);
    if (tid == 0) {
      es.mean_c[c] = m;
      es.var_c[c] = v / (n - 1);
    }
  }
  __syncthreads();
  if (tid == 0) {
    double W = 0.0, mm = 0.0;
    for (int c = 0; c < C; ++c) {
      W += es.var_c[c];
      mm += es.mean_c[c];
    }
    W /= C;
    mm /= C;
    double B = 0.0;
    for (int c = 0; c < C; ++c) B += (es.mean_c[c] - mm) * (es.mean_c[c] - mm);
    double vp = W * (n - 1.0) / n;
    if (C > 1) vp += B / (C - 1.0);
    es.W = W;
    es.vp = vp;
    es.done = !(vp > 0.0);
  }
  __syncthreads();
  for (int t = tid; t < C * n; t += blockDim.x) xs[t] -= es.mean_c[t / n];
  __syncthreads();
  const double W = es.W, vp = es.vp;
  const int wv = tid >> 6, ln = tid & 63;
  double prev = 1e300, tau_sum = 0.0;   // thread 0 state
  for (int lag0 = 0; lag0 < n && !es.done; lag0 += 64) {
    const int t = lag0 + ln;
    double a = 0.0;
    if (t < n) {
      for (int c = 0; c < C; ++c) {
        const double* xc = xs + c * n;
        for (int s = wv; s + t < n; s += 4) a += xc[s] * xc[s + t];
      }
    }
    es.part[wv][ln] = a;
    __syncthreads();
    if (tid < 64) {
      const double tot = ((es.part[0][tid] + es.part[1][tid]) + es.part[2][tid]) + es.part[3][tid];
      es.rho[tid] = (lag0 + tid == 0) ? 1.0 : 1.0 - (W - tot / ((double)n * C)) / vp;
    }
    __syncthreads();
    if (tid == 0) {
      for (int k = 0; k < 32; ++k) {
        const int t0 = lag0 + 2 * k;
        if (t0 + 1 >= n) { es.done = 1; break; }
        double Pk = es.rho[2 * k] + es.rho[2 * k + 1];
        if (Pk <= 0.0) { es.done = 1; break; }
        if (Pk > prev) Pk = prev;
        prev = Pk;
        tau_sum += Pk;
      }
    }
    __syncthreads();
  }
  if (tid == 0) {
    const double m = (double)C * n;
    double tau = (vp > 0.0 && tau_sum > 0.0) ? -1.0 + 2.0 * tau_sum : 1.0;
    tau = fmax(tau, 1.0 / log10(m));
    ess_out = (vp > 0.0) ? (float)(m / tau) : (float)m;
    rhat_out = (float)sqrt(vp / W);
  }
  __syncthreads();   // xs and es may be reused by the caller
}

}  // namespace bsi
