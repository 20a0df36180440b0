// Chain diagnostics of Section 4.1: multi-chain effective sample size per
// parameter (autocorrelations combined across chains, Geyer's initial
// monotone sequence of pair sums, no rank normalisation; capped at
// M n log10(M n)) and the classic potential scale reduction R-hat.
// One workgroup per (galaxy, parameter); the M x n draws sit in LDS, lags are
// computed 256 at a time in float64 until the pair sums turn non-positive.
#include "bsi_kernels.h"

namespace bsi {

namespace {

__global__ void __launch_bounds__(256) ess_kernel(int C, int S, int P, const float* __restrict__ x,
                                                  float* __restrict__ ess, float* __restrict__ rhat) {
  extern __shared__ double sm[];
  double* xs = sm;                       // [C][S] centred per chain
  double* rho = xs + (size_t)C * S;      // [256]
  __shared__ double mean_c[16], var_c[16];
  __shared__ double s_W, s_vp, s_tau;
  __shared__ int s_done;
  const int gal = blockIdx.x / P, par = blockIdx.x - gal * P;
  const float* src = x + (int64_t)gal * C * S * P;
  for (int t = threadIdx.x; t < C * S; t += blockDim.x) xs[t] = (double)src[(int64_t)t * P + par];
  __syncthreads();
  if (threadIdx.x < C) {
    const int c = threadIdx.x;
    double m = 0.0;
    for (int s = 0; s < S; ++s) m += xs[c * S + s];
    m /= S;
    double v = 0.0;
    for (int s = 0; s < S; ++s) {
      const double d = xs[c * S + s] - m;
      v += d * d;
    }
    mean_c[c] = m;
    var_c[c] = v / (S - 1);
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double W = 0.0, mm = 0.0;
    for (int c = 0; c < C; ++c) {
      W += var_c[c];
      mm += mean_c[c];
    }
    W /= C;
    mm /= C;
    double B = 0.0;
    for (int c = 0; c < C; ++c) B += (mean_c[c] - mm) * (mean_c[c] - mm);
    double vp = W * (S - 1.0) / S;
    if (C > 1) vp += B / (C - 1.0);
    s_W = W;
    s_vp = vp;
    s_tau = -1.0;
    s_done = !(vp > 0.0);
  }
  __syncthreads();
  for (int t = threadIdx.x; t < C * S; t += blockDim.x) xs[t] -= mean_c[t / S];
  __syncthreads();
  const double W = s_W, vp = s_vp;
  double prev = 1e300, tau_sum = 0.0;   // thread 0 state
  for (int lag0 = 0; lag0 < S && !s_done; lag0 += 256) {
    const int t = lag0 + threadIdx.x;
    if (t < S) {
      double a = 0.0;
      for (int c = 0; c < C; ++c) {
        const double* xc = xs + c * S;
        double sc = 0.0;
        for (int s = 0; s + t < S; ++s) sc += xc[s] * xc[s + t];
        a += sc / S;
      }
      rho[threadIdx.x] = (t == 0) ? 1.0 : 1.0 - (W - a / C) / vp;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      for (int k = 0; k < 128; ++k) {
        const int t0 = lag0 + 2 * k;
        if (t0 + 1 >= S) { s_done = 1; break; }
        double Pk = rho[2 * k] + rho[2 * k + 1];
        if (Pk <= 0.0) { s_done = 1; break; }
        if (Pk > prev) Pk = prev;
        prev = Pk;
        tau_sum += Pk;
      }
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const double n = (double)C * S;
    double tau = (vp > 0.0 && tau_sum > 0.0) ? -1.0 + 2.0 * tau_sum : 1.0;
    tau = fmax(tau, 1.0 / log10(n));
    if (ess) ess[(int64_t)gal * P + par] = (vp > 0.0) ? (float)(n / tau) : (float)n;
    if (rhat) rhat[(int64_t)gal * P + par] = (float)sqrt(vp / W);
  }
}

}  // namespace

hipError_t launch_ess(int n_gal, int C, int S, int P, const float* samples, float* ess,
                      float* rhat, hipStream_t s) {
  if (n_gal <= 0) return hipSuccess;
  const size_t lds = sizeof(double) * ((size_t)C * S + 256);
  (void)hipFuncSetAttribute((const void*)ess_kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  hipLaunchKernelGGL(ess_kernel, dim3(n_gal * P), dim3(256), lds, s, C, S, P, samples, ess, rhat);
  return hipGetLastError();
}

}  // namespace bsi
