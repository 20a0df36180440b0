// Device side of the request server: admission scatters each admitted
// request's scalars, start positions and stamp into its slot; harvest gathers
// finished requests' samples and chain statistics into caller buffers.
#include "bsi_kernels.h"

namespace bsi {

namespace {

__global__ void __launch_bounds__(256)
slots_scatter_kernel(const SlotRecord* __restrict__ rec, const float* __restrict__ init_src, int C,
                     SlotArrays sa, float* __restrict__ arena) {
  const SlotRecord r = rec[blockIdx.x];
  if (threadIdx.x == 0) {
    sa.off[r.slot] = r.off;
    sa.bin_off[r.slot] = r.bin_off;
    sa.psf[r.slot] = r.psf;
    sa.sigma[r.slot] = r.sigma;
    sa.ref_xy[2 * (int64_t)r.slot] = r.refx;
    sa.ref_xy[2 * (int64_t)r.slot + 1] = r.refy;
    sa.uid[r.slot] = r.uid;
  }
  const int nin = C * 6;
  for (int i = threadIdx.x; i < nin; i += blockDim.x)
    sa.init[(int64_t)r.slot * nin + i] = init_src[(int64_t)blockIdx.x * nin + i];
  const float* __restrict__ src = reinterpret_cast<const float*>(r.src);
  float* __restrict__ dst = arena + r.off;
  const int np = r.N * r.N;
  for (int i = threadIdx.x; i < np; i += blockDim.x) dst[i] = src[i];
}

__global__ void __launch_bounds__(256)
slots_gather_kernel(const int32_t* __restrict__ list, int C, int S, const ChainState* __restrict__ st,
                    const float* __restrict__ samples, float* __restrict__ out,
                    float* __restrict__ stats, uint32_t* __restrict__ status) {
  const int j = blockIdx.x;
  const int slot = list[j];
  if (out) {
    const int64_t n = (int64_t)C * S * 6;
    const float4* __restrict__ src = reinterpret_cast<const float4*>(samples + (int64_t)slot * n);
    float4* __restrict__ dst = reinterpret_cast<float4*>(out + (int64_t)j * n);
    for (int64_t i = threadIdx.x; i < n / 4; i += blockDim.x) dst[i] = src[i];
    for (int64_t i = (n / 4) * 4 + threadIdx.x; i < n; i += blockDim.x)
      out[(int64_t)j * n + i] = samples[(int64_t)slot * n + i];
  }
  if (threadIdx.x == 0 && status) {
    uint32_t s = 0;
    for (int c = 0; c < C; ++c) s |= st[(int64_t)slot * C + c].status;
    status[j] = s;
  }
  if (stats && (int)threadIdx.x < C) {
    const ChainState& x = st[(int64_t)slot * C + threadIdx.x];
    float* o = stats + ((int64_t)j * C + threadIdx.x) * 4;
    o[0] = S > 0 ? (float)x.n_acc / (float)S : 0.f;
    o[1] = x.eps;
    o[2] = (float)x.n_div;
    o[3] = (float)x.U;
  }
}

}  // namespace

hipError_t launch_slots_scatter(const SlotRecord* rec, const float* init_src, int n, int C,
                                const SlotArrays& sa, float* arena, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(slots_scatter_kernel, dim3(n), dim3(256), 0, s, rec, init_src, C, sa, arena);
  return hipGetLastError();
}

hipError_t launch_slots_gather(const int32_t* list, int n, int C, int S, const ChainState* st,
                               const float* samples, float* out, float* stats, uint32_t* status,
                               hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(slots_gather_kernel, dim3(n), dim3(256), 0, s, list, C, S, st, samples, out,
                     stats, status);
  return hipGetLastError();
}

}  // namespace bsi
