// Multi-chain effective sample size and R-hat of one parameter, computed by
// one whole workgroup of 256 threads (Section 4.1 diagnostics):
// autocorrelations combined across chains, Geyer's initial monotone
// sequence of pair sums, no rank normalisation, tau floored at
// 1 / log10(M n) (so ESS <= M n log10(M n)); classic R-hat; optionally the
// split R-hat (each chain cut into its first and last floor(n/2) draws, the
// classic statistic over the 2M halves).  The M x n draws
// are staged in LDS as float64.  Chain means and variances are block
// reductions; lags are computed 64 at a time (each lag's sum split over the
// four waves by draw index mod 4, partials added in wave order) until the
// pair sums turn non-positive.  Every reduction has a fixed order.
#pragma once

#include "bsi_device.h"

namespace bsi {

struct EssShared {
  double mean_c[32], var_c[32];
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

// Mean and (n - 1)-normalised variance of the len draws xs[0..len), block-wide
// in a fixed order; valid in every thread.
__device__ inline void ess_block_moments(const double* xs, int len, EssShared& es, double& m,
                                         double& v) {
  double a = 0.0;
  for (int s = threadIdx.x; s < len; s += blockDim.x) a += xs[s];
  m = ess_block_sum(a, es) / len;
  double q = 0.0;
  for (int s = threadIdx.x; s < len; s += blockDim.x) {
    const double d = xs[s] - m;
    q += d * d;
  }
  v = ess_block_sum(q, es) / (len - 1);
}

// Classic R-hat from C chain means and variances of chains of length n.
__device__ inline double rhat_from_moments(const double* mean, const double* var, int C, int n) {
  double W = 0.0, mm = 0.0;
  for (int c = 0; c < C; ++c) {
    W += var[c];
    mm += mean[c];
  }
  W /= C;
  mm /= C;
  double B = 0.0;
  for (int c = 0; c < C; ++c) B += (mean[c] - mm) * (mean[c] - mm);
  double vp = W * (n - 1.0) / n;
  if (C > 1) vp += B / (C - 1.0);
  return sqrt(vp / W);
}

// Draw s of chain c: src[(c * stride + s) * P + par], c < C <= 16, s < n,
// n >= 2.  xs: LDS double[C n]; es: LDS scratch.  Every thread of the
// workgroup must call; the results are valid in thread 0.
// With rsplit non-NULL (and n >= 4) the split R-hat is also computed (thread 0).
__device__ inline void ess_one_param(const float* __restrict__ src, int C, int n, int stride, int P,
                                     int par, double* xs, EssShared& es, float& ess_out,
                                     float& rhat_out, float* rsplit = nullptr) {
  const int tid = threadIdx.x;
  for (int t = tid; t < C * n; t += blockDim.x) {
    const int c = t / n, s = t - c * n;
    xs[t] = (double)src[((int64_t)c * stride + s) * P + par];
  }
  __syncthreads();
  if (rsplit && n >= 4) {
    // halves: draws [0, h) and [n - h, n) of each chain (the middle one of an odd n dropped)
    const int h = n / 2;
    for (int c = 0; c < C; ++c)
      for (int k = 0; k < 2; ++k) {
        double m, v;
        ess_block_moments(xs + c * n + k * (n - h), h, es, m, v);
        if (tid == 0) {
          es.mean_c[2 * c + k] = m;
          es.var_c[2 * c + k] = v;
        }
      }
    __syncthreads();
    if (tid == 0) *rsplit = (float)rhat_from_moments(es.mean_c, es.var_c, 2 * C, h);
    __syncthreads();
  }
  for (int c = 0; c < C; ++c) {
    double m, v;
    ess_block_moments(xs + c * n, n, es, m, v);
    if (tid == 0) {
      es.mean_c[c] = m;
      es.var_c[c] = v;
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
