// The stamp transforms as dense DFT products on the FP32 matrix cores
// (v_mfma_f32_16x16x4_f32, tiles of 16 x 16 accumulated over K steps of 4,
// sizes padded with zeros), one workgroup of 4 waves per galaxy, operands in
// LDS, DFT factors from a 2N-entry twiddle table indexed by the exactly
// reduced phase (pixel centres at x' = x - (N-1)/2).
//
// render_mfma_kernel -- the model stamp (Section 3.2's forward model) from
// the half-plane spectrum T (Hermitian mirror weight 2 on v > 0, the even-N
// Nyquist points weighted as in the float64 renderer):
//   pass 1  B[v][x] = sum_u T[v][u] e^{+i k_u x'}      (rows v = 0..h)
//   pass 2  m[y][x] = N^-2 sum_v Re(B[v][x] e^{+i k_v y'})
// The spectrum's separable factors (PSF, pixel sinc, centroid phase, flux,
// weights) are formed in float64 and rounded; G(q) and the products are
// float32.
//
// dft_bins_mfma_kernel -- the forward DFT of a stamp (or of data - model)
// at the half-plane bins of the k-space likelihood, written in slot order:
//   pass A  Q[v][x] = sum_y d[y][x] e^{-i k_v y'}      (rows v = 0..h; -h for
//                                                       the last row of even N)
//   pass B  D[v][u] = sum_x Q[v][x] e^{-i k_u x'}      (the N DFT columns u)
#include "bsi_kernels.h"
#include "kspace.h"

#include <algorithm>

namespace bsi {

namespace {

typedef float f32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ f32x4 mfma16x16x4(float a, float b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

struct RenderDims {
  int h, ntab, nrow;   // frequency points per row (u = -h..h), rows (v = 0..h)
  int ldT;             // row stride of T: ntab rounded up to 4
  int nrow4;           // rows of B: nrow rounded up to 4
  int Np;              // N rounded up to 16
};

__host__ __device__ inline RenderDims render_dims(int N) {
  RenderDims d;
  d.h = N / 2;
  d.ntab = 2 * d.h + 1;
  d.nrow = d.h + 1;
  d.ldT = (d.ntab + 3) & ~3;
  d.nrow4 = (d.nrow + 3) & ~3;
  d.Np = (N + 15) & ~15;
  return d;
}

// LDS: twiddles [2N], X [ntab], Y [nrow], T [nrow][ldT], B [nrow4][Np] (float2).
__host__ __device__ inline size_t render_mfma_lds(int N) {
  const RenderDims d = render_dims(N);
  return sizeof(float2) * ((size_t)2 * N + d.ntab + d.nrow + (size_t)d.nrow * d.ldT +
                           (size_t)d.nrow4 * d.Np);
}

__global__ void __launch_bounds__(256) render_mfma_kernel(
    const float* __restrict__ params, const float* __restrict__ psf_fwhm, const int32_t* __restrict__ gidx,
    const int64_t* __restrict__ off, int N, float rscale, float pscale_inv, int prof, float nu,
    int n_exp, float* __restrict__ out) {
  extern __shared__ float2 smr[];
  const RenderDims d = render_dims(N);
  const int h = d.h, ntab = d.ntab, nrow = d.nrow, ldT = d.ldT, nrow4 = d.nrow4, Np = d.Np;
  float2* tw = smr;                 // exp(-i pi m / N)
  float2* X = tw + 2 * N;           // u-factor incl. flux and Nyquist weight
  float2* Y = X + ntab;             // v-factor incl. mirror weight
  float2* T = Y + nrow;             // spectrum [nrow][ldT]
  float2* B = T + nrow * ldT;       // half-transform [nrow4][Np]
  const int gal = gidx[blockIdx.x];
  const float* p = params + 6 * (int64_t)(gal / n_exp);     // stamps gal n_exp + j share a galaxy
  const double F = p[0], rpx = (double)p[1] * (double)rscale;
  const float e1 = p[2], e2 = p[3];
  const double dx = p[4], dy = p[5];
  const double sp = (double)psf_fwhm[gal] * 0.42466090014400953 * (double)pscale_inv;
  const bool even = (N & 1) == 0;
  const double kst = 2.0 * 3.14159265358979323846 / (double)N;
  for (int m = threadIdx.x; m < 2 * N; m += blockDim.x) {
    double s, c;
    sincospi((double)m / (double)N, &s, &c);
    tw[m] = make_float2((float)c, (float)(-s));
  }
  for (int t = threadIdx.x; t < ntab + nrow; t += blockDim.x) {
    const bool isx = t < ntab;
    const int f = isx ? t - h : t - ntab;                // u or v
    const double k = f * kst;
    double a = exp(-0.5 * sp * sp * k * k);
    if (f != 0) a *= sinpi((double)f / N) / (3.14159265358979323846 * f / N);
    double s, c;
    sincospi(2.0 * (double)f * (isx ? dx : dy) / (double)N, &s, &c);
    if (isx) {
      a *= F * ((even && (f == h || f == -h)) ? 0.5 : 1.0);
      X[t] = make_float2((float)(a * c), (float)(-a * s));
    } else {
      a *= (f == 0 || (even && f == h)) ? 1.0 : 2.0;
      Y[f] = make_float2((float)(a * c), (float)(-a * s));
    }
  }
  __syncthreads();
  // spectrum T[v][u] = G(q) X(u) Y(v), zero in the padding columns
  {
    const float E = e1 * e1 + e2 * e2;
    const float inv1mE = 1.0f / (1.0f - E);
    const float ca = (1.0f + E + 2.0f * e1) * inv1mE, cb = (1.0f + E - 2.0f * e1) * inv1mE;
    const float cc = 4.0f * e2 * inv1mE;
    const float r2 = (float)(rpx * rpx), ks = (float)kst;
    for (int t = threadIdx.x; t < nrow * ldT; t += blockDim.x) {
      const int v = t / ldT, c = t - v * ldT;
      float2 z = make_float2(0.f, 0.f);
      if (c < ntab) {
        const float kx = (float)(c - h) * ks, ky = (float)v * ks;
        const float q = fmaf(ca, kx * kx, fmaf(cb, ky * ky, cc * kx * ky));
        float G;
        if (prof == kProfExp) {
          const float rs = rsqrtf(fmaf(r2, q, 1.0f));
          G = rs * rs * rs;
        } else if (prof == kProfSpergel) {
          G = exp2f(-(1.0f + nu) * log2f(fmaf(r2, q, 1.0f)));
        } else {
          G = expf(-0.5f * r2 * q);
        }
        const float2 x = X[c], y = Y[v];
        z = make_float2(G * fmaf(x.x, y.x, -x.y * y.y), G * fmaf(x.x, y.y, x.y * y.x));
      }
      T[t] = z;
    }
  }
  __syncthreads();
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int li = lane & 15, lk = lane >> 4;      // operand row/column, K index within a step
  // pass 1: tiles of B (16 rows v x 16 columns x), Re and Im accumulated together
  const int nrb = (nrow + 15) >> 4, ncb = Np >> 4;
  for (int ti = wave; ti < nrb * ncb; ti += 4) {
    const int rb = ti / ncb, cb = ti - rb * ncb;
    const int v = rb * 16 + li, x = cb * 16 + li;
    // twiddle index of (u = k - h, x), advanced by 4 in u per step
    int m = tw_index(lk - h, x, N);
    const int st4 = tw_index(4, x, N);
    f32x4 br = {0.f, 0.f, 0.f, 0.f}, bi = {0.f, 0.f, 0.f, 0.f};
    for (int k0 = 0; k0 < ldT; k0 += 4) {
      const int k = k0 + lk;
      const float2 a = (v < nrow) ? T[v * ldT + k] : make_float2(0.f, 0.f);
      float C = 0.f, S = 0.f;
      if (k < ntab && x < N) {
        const float2 w = tw[m];                        // exp(-i k_u x'); e^{+i..} = conj
        C = w.x;
        S = -w.y;
      }
      m += st4;
      if (m >= 2 * N) m -= 2 * N;
      br = mfma16x16x4(a.x, C, br);
      br = mfma16x16x4(-a.y, S, br);
      bi = mfma16x16x4(a.x, S, bi);
      bi = mfma16x16x4(a.y, C, bi);
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int row = rb * 16 + 4 * lk + r;
      if (row < nrow4) B[row * Np + x] = make_float2(br[r], bi[r]);
    }
  }
  __syncthreads();
  // pass 2: tiles of m (16 rows y x 16 columns x), K = v
  const float inv = (float)(1.0 / ((double)N * (double)N));
  const int64_t o = off[gal];
  const int nb = Np >> 4;
  for (int ti = wave; ti < nb * nb; ti += 4) {
    const int yb = ti / nb, xb = ti - yb * nb;
    const int y = yb * 16 + li, x = xb * 16 + li;
    int m = tw_index(lk, y, N);                        // (v, y), advanced by 4 in v per step
    const int st4 = tw_index(4, y, N);
    f32x4 acc = {0.f, 0.f, 0.f, 0.f};
    for (int k0 = 0; k0 < nrow4; k0 += 4) {
      const int v = k0 + lk;
      float cy = 0.f, sy = 0.f;
      float2 b = make_float2(0.f, 0.f);
      if (v < nrow) {
        if (y < N) {
          const float2 w = tw[m];                      // Re(b e^{+i k_v y'}) = b.x w.x + b.y w.y
          cy = w.x;
          sy = w.y;
        }
        b = B[v * Np + x];
      }
      m += st4;
      if (m >= 2 * N) m -= 2 * N;
      acc = mfma16x16x4(cy, b.x, acc);
      acc = mfma16x16x4(sy, b.y, acc);
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int yy = yb * 16 + 4 * lk + r;
      if (yy < N && x < N) out[o + (int64_t)yy * N + x] = acc[r] * inv;
    }
  }
}

// LDS of the forward transform: region 1 holds the stamp (float, N x N) and
// then D (float2, nrow x N); region 2 holds Q (float2, nrow x ldK), ldK = N
// rounded up to 4; twiddles after them.
__host__ __device__ inline size_t dft_mfma_lds(int N) {
  const int nrow = N / 2 + 1, ldK = (N + 3) & ~3;
  const size_t r1 = std::max<size_t>((size_t)N * N * sizeof(float), (size_t)nrow * N * sizeof(float2));
  return ((r1 + 15) & ~(size_t)15) + sizeof(float2) * ((size_t)nrow * ldK + 2 * N);
}

__global__ void __launch_bounds__(256) dft_bins_mfma_kernel(
    const float* __restrict__ data, const double* __restrict__ model, const int32_t* __restrict__ gidx,
    const int64_t* __restrict__ off, const int64_t* __restrict__ bin_off, int N, int P,
    float2* __restrict__ out, double* __restrict__ chi2) {
  extern __shared__ float4 smd4[];
  __shared__ double red[4];
  const int h = N / 2, nrow = h + 1, ldK = (N + 3) & ~3, Np = (N + 15) & ~15;
  const bool even = (N & 1) == 0;
  const size_t r1 = std::max<size_t>((size_t)N * N * sizeof(float), (size_t)nrow * N * sizeof(float2));
  char* base = reinterpret_cast<char*>(smd4);
  float* d = reinterpret_cast<float*>(base);                           // region 1: stamp
  float2* D = reinterpret_cast<float2*>(base);                         // region 1: spectrum
  float2* Q = reinterpret_cast<float2*>(base + ((r1 + 15) & ~(size_t)15));
  float2* tw = Q + nrow * ldK;
  const int gal = gidx[blockIdx.x];
  const int64_t o = off[gal];
  double sq = 0.0;
  for (int t = threadIdx.x; t < N * N; t += blockDim.x) {
    double x = (double)data[o + t];
    if (model) x -= model[o + t];
    d[t] = (float)x;
    sq += x * x;
  }
  for (int m = threadIdx.x; m < 2 * N; m += blockDim.x) {
    double s, c;
    sincospi((double)m / (double)N, &s, &c);
    tw[m] = make_float2((float)c, (float)(-s));
  }
  if (chi2) {
    sq = wave_sum(sq);
    if (lane_id() == 0) red[threadIdx.x / kWave] = sq;
  }
  __syncthreads();
  if (chi2 && threadIdx.x == 0) chi2[gal] = red[0] + red[1] + red[2] + red[3];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int li = lane & 15, lk = lane >> 4;
  const int nrb = (nrow + 15) >> 4, ncb = Np >> 4;
  // pass A: tiles of Q (16 rows v x 16 columns x), K = y
  for (int ti = wave; ti < nrb * ncb; ti += 4) {
    const int rb = ti / ncb, cb = ti - rb * ncb;
    const int r = rb * 16 + li, x = cb * 16 + li;
    const int v = (even && r == h) ? -h : r;
    int m = tw_index(v, lk, N);                  // (v, y = lk), advanced by 4 in y per step
    const int st4 = ((8 * v) % (2 * N) + 2 * N) % (2 * N);
    f32x4 qr = {0.f, 0.f, 0.f, 0.f}, qi = {0.f, 0.f, 0.f, 0.f};
    for (int k0 = 0; k0 < ldK; k0 += 4) {
      const int y = k0 + lk;
      float a_r = 0.f, a_i = 0.f, b = 0.f;
      if (r < nrow && y < N) {
        const float2 w = tw[m];                  // exp(-i k_v y')
        a_r = w.x;
        a_i = w.y;
      }
      if (y < N && x < N) b = d[y * N + x];
      m += st4;
      if (m >= 2 * N) m -= 2 * N;
      qr = mfma16x16x4(a_r, b, qr);
      qi = mfma16x16x4(a_i, b, qi);
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int row = rb * 16 + 4 * lk + j;
      if (row < nrow && x < ldK) Q[row * ldK + x] = make_float2(qr[j], qi[j]);
    }
  }
  __syncthreads();
  // pass B: tiles of D (16 rows v x 16 columns u = c - h), K = x
  for (int ti = wave; ti < nrb * ncb; ti += 4) {
    const int rb = ti / ncb, cb = ti - rb * ncb;
    const int r = rb * 16 + li, c = cb * 16 + li;
    int m = tw_index(c - h, lk, N);              // (u, x = lk), advanced by 4 in x per step
    const int st4 = ((8 * (c - h)) % (2 * N) + 2 * N) % (2 * N);
    f32x4 dr = {0.f, 0.f, 0.f, 0.f}, di = {0.f, 0.f, 0.f, 0.f};
    for (int k0 = 0; k0 < ldK; k0 += 4) {
      const int x = k0 + lk;
      const float2 q = (r < nrow) ? Q[r * ldK + x] : make_float2(0.f, 0.f);
      float wr = 0.f, wi = 0.f;
      if (x < N && c < N) {
        const float2 w = tw[m];                  // exp(-i k_u x')
        wr = w.x;
        wi = w.y;
      }
      m += st4;
      if (m >= 2 * N) m -= 2 * N;
      dr = mfma16x16x4(q.x, wr, dr);
      dr = mfma16x16x4(-q.y, wi, dr);
      di = mfma16x16x4(q.x, wi, di);
      di = mfma16x16x4(q.y, wr, di);
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int row = rb * 16 + 4 * lk + j;
      if (row < nrow && c < N) D[row * N + c] = make_float2(dr[j], di[j]);
    }
  }
  __syncthreads();
  // pair-slot order (slot_value_uv's scales, padding zero), then the
  // Nyquist bins, then zero up to the even length
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
      int cm;
      nyq_bin_uv(N, b - 2 * sp.nslots, u, v, cm);
    } else {
      dst[b] = make_float2(0.f, 0.f);
      continue;
    }
    const float2 z = D[((v < 0) ? h : v) * N + (u + h)];
    dst[b] = make_float2(scale * z.x, scale * z.y);
  }
}

}  // namespace

size_t render_mfma_lds_bytes(int N) { return render_mfma_lds(N); }
size_t dft_bins_mfma_lds_bytes(int N) { return dft_mfma_lds(N); }

hipError_t launch_dft_bins_mfma(const float* data, const double* model, const int32_t* gidx, int n,
                                const int64_t* off, const int64_t* bin_off, int N, int P, float2* out,
                                double* chi2, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const size_t lds = dft_mfma_lds(N);
  if (lds > 160 * 1024) return hipErrorInvalidValue;
  (void)hipFuncSetAttribute((const void*)dft_bins_mfma_kernel,
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  hipLaunchKernelGGL(dft_bins_mfma_kernel, dim3(n), dim3(256), lds, s, data, model, gidx, off, bin_off, N,
                     P, out, chi2);
  return hipGetLastError();
}

hipError_t launch_render_mfma(const float* params, const float* psf, const int32_t* gidx, int n,
                              const int64_t* off, int N, float rscale, float pscale_inv, int prof, float nu,
                              float* out, hipStream_t s, int n_exp) {
  if (n <= 0) return hipSuccess;
  const size_t lds = render_mfma_lds(N);
  if (lds > 160 * 1024) return hipErrorInvalidValue;
  (void)hipFuncSetAttribute((const void*)render_mfma_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)lds);
  hipLaunchKernelGGL(render_mfma_kernel, dim3(n), dim3(256), lds, s, params, psf, gidx, off, N, rscale,
                     pscale_inv, prof, nu, n_exp, out);
  return hipGetLastError();
}

}  // namespace bsi
