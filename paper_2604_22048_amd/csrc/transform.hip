// Stamp transforms for one size class (all galaxies of side N):
//   * dft_bins_kernel:  forward DFT of a real stamp (optionally minus a model
//     stamp) at the half-plane bins used by the k-space likelihood;
//   * render_kernel:    the model stamp as the truncated Fourier series of
//     the analytic spectrum (inverse transform, Hermitian in v).
// Both run one workgroup per galaxy with the stamp and the intermediate
// half-transform resident in LDS; twiddles come from a 2N-entry table of
// exp(-i pi m / N) built in double precision, indexed by the exactly reduced
// phase u (2 i - N + 1) mod 2N, since pixel centres sit at i - (N-1)/2.
#include <cmath>

#include "bsi_kernels.h"
#include "kspace.h"

namespace bsi {

__device__ __forceinline__ void build_twiddles(float2* tw, int N) {
  for (int m = threadIdx.x; m < 2 * N; m += blockDim.x) {
    double s, c;
    sincospi((double)m / (double)N, &s, &c);
    tw[m] = make_float2((float)c, (float)(-s));
  }
}

// One workgroup per galaxy of the class.  Writes nbins complex values at
// out + bin_off[g].
// With a model (float64 stamps), transforms the residual data - model and
// writes chi2[g] = sum over pixels of (data - model)^2 (float64 throughout).
__global__ void __launch_bounds__(256) dft_bins_kernel(
    const float* __restrict__ data, const double* __restrict__ model, const int32_t* __restrict__ gidx,
    const int64_t* __restrict__ off, const int64_t* __restrict__ bin_off, int N, int P,
    float2* __restrict__ out, double* __restrict__ chi2) {
  __shared__ double red[4];
  extern __shared__ float4 smem4[];
  const Geom g = make_geom(N);
  const int gal = gidx[blockIdx.x];
  float* d = reinterpret_cast<float*>(smem4);
  float2* tw = reinterpret_cast<float2*>(d + ((N * N + 3) & ~3));
  float2* Q = tw + 2 * N;
  const int64_t o = off[gal];
  double sq = 0.0;
  for (int t = threadIdx.x; t < N * N; t += blockDim.x) {
    double x = (double)data[o + t];
    if (model) x -= model[o + t];
    d[t] = (float)x;
    sq += x * x;
  }
  build_twiddles(tw, N);
  if (chi2) {
    sq = wave_sum(sq);
    if (lane_id() == 0) red[threadIdx.x / kWave] = sq;
  }
  __syncthreads();
  if (chi2 && threadIdx.x == 0) {
    double tot = 0.0;
    for (int w = 0; w < (int)(blockDim.x / kWave); ++w) tot += red[w];
    chi2[gal] = tot;
  }
  // pass 1 (along y), rows r = 0..h: v_r = r, except the Nyquist row -h of even N
  const int nrow = g.h + 1;
  const bool even = (N & 1) == 0;
  for (int t = threadIdx.x; t < nrow * N; t += blockDim.x) {
    const int r = t / N, i = t - r * N;
    const int v = (even && r == g.h) ? -g.h : r;
    float ar = 0.f, ai = 0.f;
    int m = tw_index(v, 0, N);
    const int step = (2 * v) % (2 * N) + (v < 0 ? 2 * N : 0);
    for (int j = 0; j < N; ++j) {
      const float x = d[j * N + i];
      const float2 w = tw[m];
      ar = fmaf(x, w.x, ar);
      ai = fmaf(x, w.y, ai);
      m += step;
      if (m >= 2 * N) m -= 2 * N;
    }
    Q[r * N + i] = make_float2(ar, ai);
  }
  __syncthreads();
  // pass 2 (along x) at every stored value: the pair-slot layout of the
  // k-space loop (slot_value_uv's scales, padding zero), then the Nyquist
  // bins, then zero up to the even length
  const SlotPlan sp = make_slot_plan_p(N, P);
  float2* dst = out + bin_off[gal];
  for (int b = threadIdx.x; b < sp.nbins; b += blockDim.x) {
    int u, v;
    float scale = 1.0f;
    if (b < 2 * sp.nslots) {
      if (!slot_value_uv(N, sp, b, u, v, scale)) {
        dst[b] = make_float2(0.f, 0.f);
        continue;
      }
    } else if (b < 2 * sp.nslots + sp.nspec) {
      int c;
      nyq_bin_uv(N, b - 2 * sp.nslots, u, v, c);
    } else {
      dst[b] = make_float2(0.f, 0.f);
      continue;
    }
    const int r = (v < 0) ? g.h : v;
    const float2* q = Q + r * N;
    float ar = 0.f, ai = 0.f;
    int m = tw_index(u, 0, N);
    const int step = (2 * u) % (2 * N) + (u < 0 ? 2 * N : 0);
    for (int i = 0; i < N; ++i) {
      const float2 a = q[i];
      const float2 w = tw[m];
      ar = fmaf(a.x, w.x, fmaf(-a.y, w.y, ar));
      ai = fmaf(a.x, w.y, fmaf(a.y, w.x, ai));
      m += step;
      if (m >= 2 * N) m -= 2 * N;
    }
    dst[b] = make_float2(scale * ar, scale * ai);
  }
}

size_t dft_bins_lds_bytes(int N) {
  const Geom g = make_geom(N);
  return sizeof(float) * (size_t)((N * N + 3) & ~3) + sizeof(float2) * (2 * N + (g.h + 1) * N);
}

// Analytic spectrum at frequency point (u, v) for render, in float64.
__device__ __forceinline__ double2 spectrum_point(int u, int v, int N, double F, double rpx,
                                                  double e1, double e2, double dx, double dy,
                                                  double sp, int prof, double nu) {
  const double ks = 2.0 * 3.14159265358979323846 / (double)N;
  const double kx = u * ks, ky = v * ks;
  const double E = e1 * e1 + e2 * e2;
  const double q = ((1.0 + E) * (kx * kx + ky * ky) + 2.0 * e1 * (kx * kx - ky * ky) +
                    4.0 * e2 * kx * ky) / (1.0 - E);
  double G;
  if (prof == kProfExp) {
    const double a = 1.0 + rpx * rpx * q;
    G = 1.0 / (a * sqrt(a));
  } else if (prof == kProfSpergel) {
    G = pow(1.0 + rpx * rpx * q, -(1.0 + nu));
  } else {
    G = exp(-0.5 * rpx * rpx * q);
  }
  const double psf = exp(-0.5 * sp * sp * (kx * kx + ky * ky));
  const double su = (u == 0) ? 1.0 : sinpi((double)u / N) / (3.14159265358979323846 * u / N);
  const double sv = (v == 0) ? 1.0 : sinpi((double)v / N) / (3.14159265358979323846 * v / N);
  double s, c;
  sincospi(2.0 * ((double)u * dx + (double)v * dy) / (double)N, &s, &c);
  const double amp = F * G * psf * su * sv;
  return make_double2(amp * c, -amp * s);
}

__device__ __forceinline__ void build_twiddles_f64(double2* tw, int N) {
  for (int m = threadIdx.x; m < 2 * N; m += blockDim.x) {
    double s, c;
    sincospi((double)m / (double)N, &s, &c);
    tw[m] = make_double2(c, -s);
  }
}

// The whole render runs in float64 (it is off the sampling path): the
// spectrum row of one v is built in LDS, transformed along x into the
// half-transform B[v][x], and B is then summed along y.
// OutT = double keeps the stamp unrounded for the pixel-space likelihood.
template <typename OutT>
__global__ void __launch_bounds__(256) render_kernel(
    const float* __restrict__ params, const float* __restrict__ psf_fwhm, const int32_t* __restrict__ gidx,
    const int64_t* __restrict__ off, int N, float rscale, float pscale_inv, int prof, float nu,
    int n_exp, OutT* __restrict__ out) {
  extern __shared__ double2 smemd[];
  const int gal = gidx[blockIdx.x];
  const int h = N / 2, ntab = 2 * h + 1, nrow = h + 1;
  const bool even = (N & 1) == 0;
  double2* tw = smemd;              // [2N]
  double2* B = tw + 2 * N;          // [nrow][N]
  double2* T = B + nrow * N;        // [ntab], one row at a time
  const float* p = params + 6 * (int64_t)(gal / n_exp);     // stamps gal n_exp + j share a galaxy
  const double F = p[0], s = p[1], e1 = p[2], e2 = p[3], dx = p[4], dy = p[5];
  const double rpx = s * (double)rscale;
  const double sp = (double)psf_fwhm[gal] * 0.42466090014400953 * (double)pscale_inv;
  build_twiddles_f64(tw, N);
  for (int r = 0; r < nrow; ++r) {
    const int v = r;
    __syncthreads();
    for (int c = threadIdx.x; c < ntab; c += blockDim.x) {
      const int u = c - h;
      double w = (even && (u == h || u == -h)) ? 0.5 : 1.0;      // Nyquist point weight
      w *= (v == 0 || (even && v == h)) ? 1.0 : 2.0;             // Hermitian mirror in v
      const double2 z = spectrum_point(u, v, N, F, rpx, e1, e2, dx, dy, sp, prof, (double)nu);
      T[c] = make_double2(w * z.x, w * z.y);
    }
    __syncthreads();
    // B[r][i] = sum_u T[u] exp(+i k_u x_i)
    for (int i = threadIdx.x; i < N; i += blockDim.x) {
      double ar = 0.0, ai = 0.0;
      for (int c = 0; c < ntab; ++c) {
        const double2 a = T[c];
        const double2 w = tw[tw_index(c - h, i, N)];   // exp(-i k x); use its conjugate
        ar += a.x * w.x + a.y * w.y;
        ai += a.y * w.x - a.x * w.y;
      }
      B[r * N + i] = make_double2(ar, ai);
    }
  }
  __syncthreads();
  // m[j][i] = N^-2 sum_v Re(B[v][i] exp(+i k_v y_j))
  const double inv = 1.0 / ((double)N * (double)N);
  const int64_t o = off[gal];
  for (int t = threadIdx.x; t < N * N; t += blockDim.x) {
    const int j = t / N, i = t - j * N;
    double acc = 0.0;
    for (int r = 0; r < nrow; ++r) {
      const double2 b = B[r * N + i];
      const double2 w = tw[tw_index(r, j, N)];
      acc += b.x * w.x + b.y * w.y;                    // Re(b * conj(w))
    }
    out[o + t] = (OutT)(acc * inv);
  }
}

size_t render_lds_bytes(int N) {
  const int h = N / 2, ntab = 2 * h + 1, nrow = h + 1;
  return sizeof(double2) * (size_t)(2 * N + nrow * N + ntab);
}

hipError_t launch_dft_bins(const float* data, const double* model, const int32_t* gidx, int n,
                           const int64_t* off, const int64_t* bin_off, int N, int P, float2* out,
                           double* chi2, const float* sigma, hipStream_t s) {
  (void)sigma;
  if (n <= 0) return hipSuccess;
  const size_t lds = dft_bins_lds_bytes(N);
  (void)hipFuncSetAttribute((const void*)dft_bins_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                      (int)lds);
  hipLaunchKernelGGL(dft_bins_kernel, dim3(n), dim3(256), lds, s, data, model, gidx, off, bin_off,
                     N, P, out, chi2);
  return hipGetLastError();
}

template <typename OutT>
static hipError_t render_impl(const float* params, const float* psf, const int32_t* gidx, int n,
                              const int64_t* off, int N, float rscale, float pscale_inv, int prof, float nu,
                              int n_exp, OutT* out, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const size_t lds = render_lds_bytes(N);
  (void)hipFuncSetAttribute((const void*)render_kernel<OutT>, hipFuncAttributeMaxDynamicSharedMemorySize,
                      (int)lds);
  hipLaunchKernelGGL(render_kernel<OutT>, dim3(n), dim3(256), lds, s, params, psf, gidx, off, N,
                     rscale, pscale_inv, prof, nu, n_exp, out);
  return hipGetLastError();
}

hipError_t launch_render(const float* params, const float* psf, const int32_t* gidx, int n,
                         const int64_t* off, int N, float rscale, float pscale_inv, int prof, float nu,
                         float* out, hipStream_t s, int n_exp) {
  return render_impl(params, psf, gidx, n, off, N, rscale, pscale_inv, prof, nu, n_exp, out, s);
}

hipError_t launch_render_f64(const float* params, const float* psf, const int32_t* gidx, int n,
                             const int64_t* off, int N, float rscale, float pscale_inv, int prof, float nu,
                             double* out, hipStream_t s, int n_exp) {
  return render_impl(params, psf, gidx, n, off, N, rscale, pscale_inv, prof, nu, n_exp, out, s);
}

// Noise weights of stationary correlated noise (Appendix C): every bin of
// stamp gidx[block] (pair-slot order, then the Nyquist bins) is multiplied by
// sqrt w = lambda^-1/2, lambda the noise power of its DFT mode (u, v) read
// from noise_ps at off[stamp] in FFT order; sqw receives sqrt w per bin (0 in
// padding bins).  noise_ps NULL: w = 1 (the spectrum is unchanged).
__global__ void __launch_bounds__(256) whiten_bins_kernel(
    const float* __restrict__ noise_ps, const int32_t* __restrict__ gidx, const int64_t* __restrict__ off,
    const int64_t* __restrict__ bin_off, int N, int P, float2* __restrict__ dh, float* __restrict__ sqw) {
  const int st = gidx[blockIdx.x];
  const SlotPlan sp = make_slot_plan_p(N, P);
  float2* d = dh + bin_off[st];
  float* w = sqw + bin_off[st];
  const float* ps = noise_ps ? noise_ps + off[st] : nullptr;
  for (int b = threadIdx.x; b < sp.nbins; b += blockDim.x) {
    int u = 0, v = 0;
    bool used = true;
    if (b < 2 * sp.nslots) {
      float sc;
      used = slot_value_uv(N, sp, b, u, v, sc);
    } else if (b < 2 * sp.nslots + sp.nspec) {
      int cm;
      nyq_bin_uv(N, b - 2 * sp.nslots, u, v, cm);
    } else {
      used = false;
    }
    float r = 0.0f;
    if (used) {
      const double lam = ps ? (double)ps[((v + N) % N) * N + (u + N) % N] : 1.0;
      r = (float)(1.0 / sqrt(lam));
    }
    w[b] = r;
    const float2 z = d[b];
    d[b] = make_float2(z.x * r, z.y * r);
  }
}

hipError_t launch_whiten(const float* noise_ps, const int32_t* gidx, int n, const int64_t* off,
                         const int64_t* bin_off, int N, int P, float2* dh, float* sqw, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(whiten_bins_kernel, dim3(n), dim3(256), 0, s, noise_ps, gidx, off, bin_off, N, P,
                     dh, sqw);
  return hipGetLastError();
}

double exponential_hlr_factor() {
  double x = 1.7;
  for (int i = 0; i < 60; ++i) {
    const double f = (1.0 + x) * exp(-x) - 0.5;
    x -= f / (-x * exp(-x));
  }
  return x;
}

double spergel_hlr_factor(double nu) {
  // x^(nu+1) K_(nu+1)(x) falls from 2^nu Gamma(nu+1) at 0 to 0; bisect for half of that
  const double target = std::tgamma(nu + 1.0) * std::pow(2.0, nu - 1.0);
  auto f = [&](double x) { return std::pow(x, nu + 1.0) * std::cyl_bessel_k(nu + 1.0, x) - target; };
  double lo = 1e-6, hi = 1.0;
  while (f(hi) > 0.0) hi *= 2.0;
  for (int i = 0; i < 80; ++i) {
    const double mid = 0.5 * (lo + hi);
    (f(mid) > 0.0 ? lo : hi) = mid;
  }
  return 0.5 * (lo + hi);
}

}  // namespace bsi
