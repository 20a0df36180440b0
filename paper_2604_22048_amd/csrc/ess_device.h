// Multi-chain effective sample size and R-hat of one parameter, computed by
// one whole workgroup (Section 4.1 diagnostics): autocorrelations combined
// across chains, Geyer's initial monotone sequence of pair sums, no rank
// normalisation, tau floored at 1 / log10(M n) (so ESS <= M n log10(M n));
// classic R-hat.  The M x n draws are staged in LDS as float64 and the lags
// are computed 256 at a time until the pair sums turn non-positive.
#pragma once

#include "bsi_device.h"

namespace bsi {

struct EssShared {
  double mean_c[16], var_c[16];
  double W, vp;
  int done;
};

// Draw s of chain c: src[(c * stride + s) * P + par], c < C <= 16, s < n.
// xs: LDS double[C n]; rho: LDS double[256]; es: LDS scratch.  Every thread
// of the (256-thread) workgroup must call; the results are valid in thread 0.
__device__ inline void ess_one_param(const float* __restrict__ src, int C, int n, int stride, int P,
                                     int par, double* xs, double* rho, EssShared& es, float& ess_out,
                                     float& rhat_out) {
  for (int t = threadIdx.x; t < C * n; t += blockDim.x) {
    const int c = t / n, s = t - c * n;
    xs[t] = (double)src[((int64_t)c * stride + s) * P + par];
  }
  __syncthreads();
  if ((int)threadIdx.x < C) {
    const int c = threadIdx.x;
    double m = 0.0;
    for (int s = 0; s < n; ++s) m += xs[c * n + s];
    m /= n;
    double v = 0.0;
    for (int s = 0; s < n; ++s) {
      const double d = xs[c * n + s] - m;
      v += d * d;
    }
    es.mean_c[c] = m;
    es.var_c[c] = v / (n - 1);
  }
  __syncthreads();
  if (threadIdx.x == 0) {
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
  for (int t = threadIdx.x; t < C * n; t += blockDim.x) xs[t] -= es.mean_c[t / n];
  __syncthreads();
  const double W = es.W, vp = es.vp;
  double prev = 1e300, tau_sum = 0.0;   // thread 0 state
  for (int lag0 = 0; lag0 < n && !es.done; lag0 += 256) {
    const int t = lag0 + threadIdx.x;
    if (t < n) {
      double a = 0.0;
      for (int c = 0; c < C; ++c) {
        const double* xc = xs + c * n;
        double sc = 0.0;
        for (int s = 0; s + t < n; ++s) sc += xc[s] * xc[s + t];
        a += sc / n;
      }
      rho[threadIdx.x] = (t == 0) ? 1.0 : 1.0 - (W - a / C) / vp;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      for (int k = 0; k < 128; ++k) {
        const int t0 = lag0 + 2 * k;
        if (t0 + 1 >= n) { es.done = 1; break; }
        double Pk = rho[2 * k] + rho[2 * k + 1];
        if (Pk <= 0.0) { es.done = 1; break; }
        if (Pk > prev) Pk = prev;
        prev = Pk;
        tau_sum += Pk;
      }
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const double m = (double)C * n;
    double tau = (vp > 0.0 && tau_sum > 0.0) ? -1.0 + 2.0 * tau_sum : 1.0;
    tau = fmax(tau, 1.0 / log10(m));
    ess_out = (vp > 0.0) ? (float)(m / tau) : (float)m;
    rhat_out = (float)sqrt(vp / W);
  }
  __syncthreads();   // xs, rho and es may be reused by the caller
}

}  // namespace bsi
