// Device side of the request server: admission scatters each admitted
// request's scalars, start positions and stamp into its slot; the ESS check
// decides at each of a request's checkpoints whether it has finished; harvest
// gathers finished requests' samples and chain statistics into caller buffers.
#include "bsi_kernels.h"
#include "ess_device.h"

namespace bsi {

namespace {

__global__ void __launch_bounds__(256)
slots_scatter_kernel(const SlotRecord* __restrict__ rec, const float* __restrict__ init_src, int C,
                     int stop0, SlotArrays sa, float* __restrict__ arena) {
  const SlotRecord r = rec[blockIdx.x];
  if (threadIdx.x == 0) {
    sa.off[r.slot] = r.off;
    sa.bin_off[r.slot] = r.bin_off;
    sa.psf[r.slot] = r.psf;
    sa.sigma[r.slot] = r.sigma;
    sa.ref_xy[2 * (int64_t)r.slot] = r.refx;
    sa.ref_xy[2 * (int64_t)r.slot + 1] = r.refy;
    sa.uid[r.slot] = r.uid;
    sa.stop[r.slot] = stop0;
    sa.ndraw[r.slot] = 0;
    sa.ess_cnt[r.slot] = 0;
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
                    const float* __restrict__ samples, const int32_t* __restrict__ ndraw,
                    float* __restrict__ out, float* __restrict__ stats, uint32_t* __restrict__ status,
                    int32_t* __restrict__ out_ndraw) {
  const int j = blockIdx.x;
  const int slot = list[j];
  const int nd = ndraw ? ndraw[slot] : S;
  if (out) {
    // draws past nd are NaN (a request finished at a check)
    const int64_t n = (int64_t)C * S * 6, valid = (int64_t)nd * 6;
    const float* __restrict__ src = samples + (int64_t)slot * n;
    float* __restrict__ dst = out + (int64_t)j * n;
    for (int64_t i = threadIdx.x; i < n; i += blockDim.x)
      dst[i] = (i % (S * 6) < valid) ? src[i] : __builtin_nanf("");
  }
  if (threadIdx.x == 0 && out_ndraw) out_ndraw[j] = nd;
  if (threadIdx.x == 0 && status) {
    uint32_t s = 0;
    for (int c = 0; c < C; ++c) s |= st[(int64_t)slot * C + c].status;
    status[j] = s;
  }
  if (stats && (int)threadIdx.x < C) {
    const ChainState& x = st[(int64_t)slot * C + threadIdx.x];
    float* o = stats + ((int64_t)j * C + threadIdx.x) * 4;
    o[0] = nd > 0 ? (float)x.n_acc / (float)nd : 0.f;
    o[1] = x.eps;
    o[2] = (float)x.n_div;
    o[3] = (float)x.U;
  }
}

// One workgroup per listed request and parameter.  A request whose chains
// have reached its stop W + n is checked there: it finishes with n draws when
// n = S or when the mean over the six parameters of its ESS over draws
// [0, n) reaches the target; otherwise its stop moves to W + min(n + every,
// S).  Requests still running towards their stop, and finished ones, are
// left alone.  The six parameters' ESS are computed by six workgroups; the
// last of them to finish (a per-request counter) adds them in parameter order
// and decides.  The decision depends on the request's own draws only.
__global__ void __launch_bounds__(256)
slots_check_kernel(const int32_t* __restrict__ list, int C, int W, int S, int every, float target,
                   const ChainState* __restrict__ st, const float* __restrict__ samples, SlotArrays sa) {
  extern __shared__ double xs[];
  __shared__ EssShared es;
  const int slot = list[blockIdx.x];
  const int par = blockIdx.y;
  // stop, t and ndraw are not changed by this launch before every workgroup
  // of the request has read them, so the six take the same branch
  const int stop = sa.stop[slot];
  if (st[(int64_t)slot * C].t < stop || sa.ndraw[slot] != 0) return;   // uniform in the block
  const int n = stop - W;
  if (n >= S) {
    // the draw cap: finished without an ESS
    if (par == 0 && threadIdx.x == 0) {
      sa.ndraw[slot] = n;
      sa.done_q[atomicAdd(sa.done_n, 1)] = slot;
    }
    return;
  }
  float e = 0.f, r = 0.f;
  ess_one_param(samples + (int64_t)slot * C * S * 6, C, n, S, 6, par, xs, es, e, r);
  if (threadIdx.x == 0) {
    sa.ess6[(int64_t)slot * 6 + par] = e;
    __threadfence();
    if (atomicAdd(&sa.ess_cnt[slot], 1) == 5) {
      __threadfence();
      double sum = 0.0;
      for (int q = 0; q < 6; ++q)
        sum += (double)__hip_atomic_load(&sa.ess6[(int64_t)slot * 6 + q], __ATOMIC_RELAXED,
                                         __HIP_MEMORY_SCOPE_AGENT);
      sa.ess_cnt[slot] = 0;
      if (sum / 6.0 >= (double)target) {
        sa.ndraw[slot] = n;
        sa.done_q[atomicAdd(sa.done_n, 1)] = slot;
      } else {
        sa.stop[slot] = W + min(n + every, S);
      }
    }
  }
}

}  // namespace

hipError_t launch_slots_scatter(const SlotRecord* rec, const float* init_src, int n, int C, int stop0,
                                const SlotArrays& sa, float* arena, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(slots_scatter_kernel, dim3(n), dim3(256), 0, s, rec, init_src, C, stop0, sa, arena);
  return hipGetLastError();
}

hipError_t launch_slots_gather(const int32_t* list, int n, int C, int S, const ChainState* st,
                               const float* samples, const int32_t* ndraw, float* out, float* stats,
                               uint32_t* status, int32_t* out_ndraw, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(slots_gather_kernel, dim3(n), dim3(256), 0, s, list, C, S, st, samples, ndraw,
                     out, stats, status, out_ndraw);
  return hipGetLastError();
}

size_t slots_check_lds_bytes(int C, int S) { return sizeof(double) * (size_t)C * S; }

hipError_t launch_slots_check(const int32_t* list, int n, int C, int W, int S, int every, float target,
                              const ChainState* st, const float* samples, const SlotArrays& sa,
                              hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const size_t lds = slots_check_lds_bytes(C, S);
  (void)hipFuncSetAttribute((const void*)slots_check_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)lds);
  hipLaunchKernelGGL(slots_check_kernel, dim3(n, 6), dim3(256), lds, s, list, C, W, S, every, target, st,
                     samples, sa);
  return hipGetLastError();
}

}  // namespace bsi
