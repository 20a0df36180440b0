// Batched log-likelihood and gradient (eq. likelihood-pixels), one wave per
// galaxy.  The DFT of the data (or, for the pixel method, of the pixel
// residual) at the half-plane bins is staged in LDS and contracted with the
// analytic spectrum by kspace_sums (the same routine the sampler uses).
#include <type_traits>

#include "bsi_kernels.h"
#include "kspace.h"

namespace bsi {

// MX: the sum over the galaxy's n_exp exposures (stamps gal n_exp + j, each
// staged in turn) with per-bin noise weights sqw_all beside the spectrum
// (Appendix C).
template <int PROF, bool RESID, int P, bool MX = false>
__global__ void __launch_bounds__(64) loglik_kernel(
    const float2* __restrict__ dh_all, const int64_t* __restrict__ bin_off, const int32_t* __restrict__ gidx,
    const float* __restrict__ params, const float* __restrict__ psf, const float* __restrict__ sigma,
    int N, float rscale, float pscale_inv, float nu, const double* __restrict__ chi2_pix,
    double* __restrict__ loglik, float* __restrict__ grad, uint32_t* __restrict__ status, int n_exp,
    const float* __restrict__ sqw_all) {
  static_assert(!(MX && RESID), "exposures: k-space form only");
  extern __shared__ float4 smem4[];
  const Geom g = make_geom(N);
  const SlotPlan sp = make_slot_plan_p(N, P);
  const int gal = gidx[blockIdx.x];
  const int nbp = (sp.nbins + 1) & ~1;
  float2* dh = reinterpret_cast<float2*>(smem4);
  float* sqw = reinterpret_cast<float*>(dh + nbp);
  float* atab = sqw + (MX ? (nbp + 3) & ~3 : 0);
  float4* cols = reinterpret_cast<float4*>(atab + ((g.ntab + 3) & ~3));
  float4* Ym = cols + sp.P * 64;
  float2* X = reinterpret_cast<float2*>(Ym + sp.ymax);
  float2* Yf = X + g.ntab + 2;
  float* red = reinterpret_cast<float*>(Yf + g.ntab + 1);
  red = reinterpret_cast<float*>((reinterpret_cast<uintptr_t>(red) + 15) & ~uintptr_t(15));
  build_col_table(g, sp, cols);
  const float* p = params + 6 * (int64_t)gal;
  const float F = p[0], s = p[1], e1 = p[2], e2 = p[3], dx = p[4], dy = p[5];
  const float E = e1 * e1 + e2 * e2;
  uint32_t st = 0;
  if (!(E < 1.0f) || !(s > 0.0f) || !(F > 0.0f)) st |= 1u;
  const Shape sh = make_shape<PROF>(s * rscale, e1, e2, nu);
  const LaneCols<P> lc = lane_cols<P>(cols);
  const int ne = MX ? n_exp : 1;
  KResult r{0.0, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
  float sig = 1.0f;
  for (int x = 0; x < ne; ++x) {
    const int64_t stp = MX ? (int64_t)gal * ne + x : gal;    // this exposure's stamp
    __syncthreads();
    const float2* src = dh_all + bin_off[stp];
    for (int b = threadIdx.x; b < sp.nbins; b += blockDim.x) dh[b] = src[b];
    if constexpr (MX)
      for (int b = threadIdx.x; b < sp.nbins; b += blockDim.x) sqw[b] = sqw_all[bin_off[stp] + b];
    const float spsf = psf[stp] * 0.42466090014400953f * pscale_inv;
    for (int t = threadIdx.x; t < g.ntab; t += blockDim.x) {
      const int u = t - g.h;
      const double k = 2.0 * 3.14159265358979323846 * u / N;
      const double sn = (u == 0) ? 1.0 : sinpi((double)u / N) / (3.14159265358979323846 * u / N);
      atab[t] = (float)(exp(-0.5 * (double)spsf * spsf * k * k) * sn);
    }
    __syncthreads();
    sig = sigma[stp];
    const float norm = 1.0f / ((float)N * (float)N * sig * sig);
    fill_tables(g, sp, atab, X, Ym, Yf, F, dx, dy);
    const KSums S = kspace_sums<PROF, P, RESID, true, 0, 1, 1, MX>(g, sp, lc, dh, X, Ym, Yf, sh, red, 0,
                                                                   nullptr, sqw);
    const KResult q = kspace_finish<PROF>(S, sh, F, s, e1, e2, norm);
    r.loglik += q.loglik;
    r.dF += q.dF;
    r.ds += q.ds;
    r.de1 += q.de1;
    r.de2 += q.de2;
    r.ddx += q.ddx;
    r.ddy += q.ddy;
  }
  if (RESID) r.loglik = -0.5 * chi2_pix[gal] / ((double)sig * (double)sig);
  if (!isfinite(r.loglik)) st |= 2u;
  if (threadIdx.x == 0) {
    if (loglik) loglik[gal] = r.loglik;
    if (status) status[gal] = st;
  }
  if (grad && threadIdx.x < 6) {
    const float v[6] = {r.dF, r.ds, r.de1, r.de2, r.ddx, r.ddy};
    float o = v[0];
#pragma unroll
    for (int j = 1; j < 6; ++j) o = (threadIdx.x == j) ? v[j] : o;
    grad[6 * (int64_t)gal + threadIdx.x] = o;
  }
}

static size_t loglik_lds_bytes(int N, int P, bool mx) {
  const Geom g = make_geom(N);
  const SlotPlan sp = make_slot_plan_p(N, P);
  const int nbp = (sp.nbins + 1) & ~1;
  return sizeof(float2) * nbp + sizeof(float) * (mx ? (nbp + 3) & ~3 : 0) +
         sizeof(float) * ((g.ntab + 3) & ~3) +
         sizeof(float4) * sp.P * 64 + sizeof(float4) * sp.ymax + sizeof(float2) * (2 * g.ntab + 3) +
         16 + sizeof(float) * 64 * 8;
}

template <int PROF, bool RESID, bool MX>
static void launch_loglik_p(int P, dim3 grid, size_t lds, hipStream_t s, const float2* dh,
                            const int64_t* bin_off, const int32_t* gidx, const float* params,
                            const float* psf, const float* sigma, int N, float rscale,
                            float pscale_inv, float nu, const double* chi2_pix, double* loglik,
                            float* grad, uint32_t* status, int n_exp, const float* sqw) {
  auto go = [&](auto kern) {
    (void)hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    hipLaunchKernelGGL(kern, grid, dim3(64), lds, s, dh, bin_off, gidx, params, psf, sigma, N,
                       rscale, pscale_inv, nu, chi2_pix, loglik, grad, status, n_exp, sqw);
  };
  switch (P) {
    case 1: go(loglik_kernel<PROF, RESID, 1, MX>); break;
    case 2: go(loglik_kernel<PROF, RESID, 2, MX>); break;
    case 3: go(loglik_kernel<PROF, RESID, 3, MX>); break;
    case 4: go(loglik_kernel<PROF, RESID, 4, MX>); break;
    case 5: go(loglik_kernel<PROF, RESID, 5, MX>); break;
    case 6: go(loglik_kernel<PROF, RESID, 6, MX>); break;
    default: go(loglik_kernel<PROF, RESID, 8, MX>); break;
  }
}

hipError_t launch_loglik(const float2* dh, const int64_t* bin_off, const int32_t* gidx, int n,
                         const float* params, const float* psf, const float* sigma, int N, int P,
                         float rscale, float pscale_inv, int prof, float nu, int resid_mode,
                         const double* chi2_pix, double* loglik, float* grad, uint32_t* status,
                         hipStream_t s, int n_exp, const float* sqw) {
  if (n <= 0) return hipSuccess;
  if (!plan_valid(N, P)) return hipErrorInvalidValue;
  const bool mx = sqw != nullptr;
  if (mx && (resid_mode || n_exp < 1)) return hipErrorInvalidValue;
  const size_t lds = loglik_lds_bytes(N, P, mx);
  const dim3 grid(n);
  auto run = [&](auto prof_tag) {
    constexpr int PR = decltype(prof_tag)::value;
    if (mx)
      launch_loglik_p<PR, false, true>(P, grid, lds, s, dh, bin_off, gidx, params, psf, sigma, N,
                                       rscale, pscale_inv, nu, chi2_pix, loglik, grad, status, n_exp,
                                       sqw);
    else if (resid_mode)
      launch_loglik_p<PR, true, false>(P, grid, lds, s, dh, bin_off, gidx, params, psf, sigma, N,
                                       rscale, pscale_inv, nu, chi2_pix, loglik, grad, status, 1,
                                       nullptr);
    else
      launch_loglik_p<PR, false, false>(P, grid, lds, s, dh, bin_off, gidx, params, psf, sigma, N,
                                        rscale, pscale_inv, nu, chi2_pix, loglik, grad, status, 1,
                                        nullptr);
  };
  if (prof == kProfExp)
    run(std::integral_constant<int, kProfExp>());
  else if (prof == kProfSpergel)
    run(std::integral_constant<int, kProfSpergel>());
  else
    run(std::integral_constant<int, kProfGauss>());
  return hipGetLastError();
}

}  // namespace bsi
