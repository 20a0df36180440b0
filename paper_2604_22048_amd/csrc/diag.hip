// Chain diagnostics of Section 4.1 over stored samples [gal][C][S][P]: one
// workgroup per (galaxy, parameter) runs ess_one_param.
#include "bsi_kernels.h"
#include "ess_device.h"

namespace bsi {

namespace {

__global__ void __launch_bounds__(256) ess_kernel(int C, int S, int P, const float* __restrict__ x,
                                                  float* __restrict__ ess, float* __restrict__ rhat,
                                                  float* __restrict__ rsplit) {
  extern __shared__ double xs[];         // [C][S] centred per chain
  __shared__ EssShared es;
  const int gal = blockIdx.x / P, par = blockIdx.x - gal * P;
  float e = 0.f, r = 0.f, rs = 0.f;
  ess_one_param(x + (int64_t)gal * C * S * P, C, S, S, P, par, xs, es, e, r, rsplit ? &rs : nullptr);
  if (threadIdx.x == 0) {
    if (ess) ess[(int64_t)gal * P + par] = e;
    if (rhat) rhat[(int64_t)gal * P + par] = r;
    if (rsplit) rsplit[(int64_t)gal * P + par] = rs;
  }
}

}  // namespace

hipError_t launch_ess(int n_gal, int C, int S, int P, const float* samples, float* ess,
                      float* rhat, float* rsplit, hipStream_t s) {
  if (n_gal <= 0) return hipSuccess;
  const size_t lds = sizeof(double) * (size_t)C * S;
  (void)hipFuncSetAttribute((const void*)ess_kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  hipLaunchKernelGGL(ess_kernel, dim3(n_gal * P), dim3(256), lds, s, C, S, P, samples, ess, rhat, rsplit);
  return hipGetLastError();
}

}  // namespace bsi
