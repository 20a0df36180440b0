// Multiplicative and additive shear bias by shape-noise cancellation with
// bootstrap errors (Section 3.5).  With the population parameters fixed the
// shear posterior of a galaxy resample that draws galaxy n c_n times is
//   ln P_b(g_p) = sum_n c_bn ell_n(g_p),
// so every resample of both datasets (+g and -g) is one dense product of the
// count matrix C [R x G] (row 0 all ones: every galaxy once; rows 1..B the
// resamples) with the per-galaxy log-marginal tables E+ and E- [P x G]:
//   Lp[r][p] = sum_n C[r][n] E[p][n],  p < 2P over [E+; E-].
// The product runs on the FP64 matrix cores (v_mfma_f64_16x16x4f64): a
// workgroup of 4 waves owns a 64 x 64 output tile (each wave 32 x 32, i.e.
// 2 x 2 MFMA tiles) of one K split, stages 32 galaxies of C (converted to
// float64) and of E per step in LDS, and writes its partial tile; a second
// kernel adds the splits in order, forms each row's posterior mean of g on
// the grid, and m_r, c_r; a third takes the standard deviations over the
// resamples.  ell = -inf (a galaxy with no supported sample at that point)
// is carried as -1e300 so that a galaxy not drawn (c = 0) adds exactly 0.
#include <algorithm>

#include "bsi_kernels.h"

namespace bsi {

namespace {

typedef double f64x4 __attribute__((ext_vector_type(4)));

constexpr int kTile = 64;     // output tile (rows r and columns p) per workgroup
constexpr int kKc = 32;       // galaxies per LDS step
constexpr int kLd = kKc + 1;  // padded LDS row (doubles)
constexpr double kNegBig = -1e300;

__device__ __forceinline__ f64x4 mfma_f64(double a, double b, f64x4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// Partial products of one K split.  Grid: x = column tiles, y = row tiles,
// z = K splits.  out[z][r][p] for r < R, p < 2P.
__global__ void __launch_bounds__(256) bias_gemm_kernel(const int32_t* __restrict__ counts,
                                                        const double* __restrict__ ep,
                                                        const double* __restrict__ em, int G, int P,
                                                        int R, int k_per_split,
                                                        double* __restrict__ out) {
  __shared__ double As[kTile][kLd];   // C tile: rows r, galaxies k
  __shared__ double Bs[kTile][kLd];   // E tile: columns p, galaxies k
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int r0 = blockIdx.y * kTile, p0 = blockIdx.x * kTile;
  const int k_begin = blockIdx.z * k_per_split;
  const int k_end = min(G, k_begin + k_per_split);
  const int P2 = 2 * P;
  const int wr = (wave >> 1) * 32, wc = (wave & 1) * 32;   // the wave's 32 x 32 sub-tile
  const int li = lane & 15, lk = lane >> 4;
  f64x4 acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = f64x4{0.0, 0.0, 0.0, 0.0};
  for (int kc = k_begin; kc < k_end; kc += kKc) {
    __syncthreads();
    // stage 64 x 32 of C and of E (k fastest; zero outside the matrices)
    for (int t = tid; t < kTile * kKc; t += 256) {
      const int row = t / kKc, k = t - row * kKc;
      const int n = kc + k;
      double cv = 0.0, evv = 0.0;
      if (n < k_end) {
        const int r = r0 + row;
        if (r < R) cv = (r == 0) ? 1.0 : (double)counts[(int64_t)(r - 1) * G + n];
        const int p = p0 + row;
        if (p < P2) {
          const double v = (p < P) ? ep[(int64_t)p * G + n] : em[(int64_t)(p - P) * G + n];
          evv = (v > kNegBig) ? v : kNegBig;   // -inf (and anything below) -> -1e300
        }
      }
      As[row][k] = cv;
      Bs[row][k] = evv;
    }
    __syncthreads();
#pragma unroll
    for (int k0 = 0; k0 < kKc; k0 += 4) {
      const int k = k0 + lk;
      double a[2], b[2];
#pragma unroll
      for (int i = 0; i < 2; ++i) a[i] = As[wr + 16 * i + li][k];   // A[i = li][k = lk]
#pragma unroll
      for (int j = 0; j < 2; ++j) b[j] = Bs[wc + 16 * j + li][k];   // B[k = lk][j = li]
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = mfma_f64(a[i], b[j], acc[i][j]);
    }
  }
  // D[i][j] of a 16 x 16 float64 tile sits in lane j + 16 (i % 4), element
  // i / 4 (rows interleaved across the lane groups, unlike the float32 form)
  double* o = out + (int64_t)blockIdx.z * R * P2;
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int r = r0 + wr + 16 * i + lk + 4 * e;
        const int p = p0 + wc + 16 * j + li;
        if (r < R && p < P2) o[(int64_t)r * P2 + p] = acc[i][j][e];
      }
}

constexpr int kMeanThreads = 256;

// Fixed-order block sum of one value per thread (valid in thread 0).
__device__ __forceinline__ double block_sum(double v, double* red) {
  red[threadIdx.x] = v;
  __syncthreads();
  for (int w = kMeanThreads / 2; w >= 1; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  const double t = red[0];
  __syncthreads();
  return t;
}

__device__ __forceinline__ double block_max(double v, double* red) {
  red[threadIdx.x] = v;
  __syncthreads();
  for (int w = kMeanThreads / 2; w >= 1; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + w]);
    __syncthreads();
  }
  const double t = red[0];
  __syncthreads();
  return t;
}

// One workgroup per row r: the K splits added in order, then for each of
// the two datasets the posterior mean of g on its grid (gpts, then gpts +
// 2 P; weights exp(ln P - max)),
// then m_r = (g+_1 - g-_1) / (2 |g|) - 1 and c_r = (g+_2 + g-_2) / 2.
__global__ void __launch_bounds__(kMeanThreads) bias_mean_kernel(const double* __restrict__ part,
                                                                 int n_split, int R, int P,
                                                                 const double* __restrict__ gpts,
                                                                 double g_abs, double* __restrict__ gmean,
                                                                 double* __restrict__ mc) {
  extern __shared__ double lp[];      // [2P]
  __shared__ double red[kMeanThreads];
  const int r = blockIdx.x, P2 = 2 * P;
  for (int p = threadIdx.x; p < P2; p += kMeanThreads) {
    double v = 0.0;
    for (int s = 0; s < n_split; ++s) v += part[((int64_t)s * R + r) * P2 + p];
    lp[p] = v;
  }
  __syncthreads();
  double mean[2][2];
  for (int d = 0; d < 2; ++d) {
    const double* l = lp + d * P;
    const double* gd = gpts + 2 * (int64_t)d * P;
    double mx = -INFINITY;
    for (int p = threadIdx.x; p < P; p += kMeanThreads) mx = fmax(mx, l[p]);
    mx = block_max(mx, red);
    double w0 = 0.0, w1 = 0.0, w2 = 0.0;
    for (int p = threadIdx.x; p < P; p += kMeanThreads) {
      const double w = exp(l[p] - mx);
      w0 += w;
      w1 += w * gd[2 * p];
      w2 += w * gd[2 * p + 1];
    }
    w0 = block_sum(w0, red);
    w1 = block_sum(w1, red);
    w2 = block_sum(w2, red);
    mean[d][0] = w1 / w0;
    mean[d][1] = w2 / w0;
  }
  if (threadIdx.x == 0) {
    if (gmean) {
      gmean[2 * (int64_t)r] = mean[0][0];
      gmean[2 * (int64_t)r + 1] = mean[0][1];
      gmean[2 * ((int64_t)R + r)] = mean[1][0];
      gmean[2 * ((int64_t)R + r) + 1] = mean[1][1];
    }
    mc[2 * (int64_t)r] = (mean[0][0] - mean[1][0]) / (2.0 * g_abs) - 1.0;
    mc[2 * (int64_t)r + 1] = 0.5 * (mean[0][1] + mean[1][1]);
  }
}

// stats = {m_0, c_0, std(m_1..m_B), std(c_1..c_B)} (population standard
// deviations, two passes, fixed order); std 0 when B = 0.
__global__ void __launch_bounds__(kMeanThreads) bias_stats_kernel(const double* __restrict__ mc, int R,
                                                                  double* __restrict__ stats) {
  __shared__ double red[kMeanThreads];
  const int B = R - 1;
  double sd[2] = {0.0, 0.0};
  for (int q = 0; q < 2; ++q) {
    double s = 0.0;
    for (int b = 1 + threadIdx.x; b <= B; b += kMeanThreads) s += mc[2 * b + q];
    s = block_sum(s, red);
    const double mean = (B > 0) ? s / B : 0.0;
    double v = 0.0;
    for (int b = 1 + threadIdx.x; b <= B; b += kMeanThreads) {
      const double d = mc[2 * b + q] - mean;
      v += d * d;
    }
    v = block_sum(v, red);
    sd[q] = (B > 0) ? sqrt(v / B) : 0.0;
  }
  if (threadIdx.x == 0) {
    stats[0] = mc[0];
    stats[1] = mc[1];
    stats[2] = sd[0];
    stats[3] = sd[1];
  }
}

}  // namespace

BiasPlan bias_plan(int G, int P, int n_boot) {
  BiasPlan b;
  b.R = n_boot + 1;
  const int tiles = ((2 * P + kTile - 1) / kTile) * ((b.R + kTile - 1) / kTile);
  // enough K splits for about two workgroups per compute unit, each at least 4 LDS steps
  int splits = std::max(1, (512 + tiles - 1) / tiles);
  splits = std::min(splits, std::max(1, G / (4 * kKc)));
  b.k_per_split = ((G + splits - 1) / splits + kKc - 1) / kKc * kKc;
  b.n_split = std::max(1, (G + b.k_per_split - 1) / b.k_per_split);
  b.partial_doubles = (size_t)b.n_split * b.R * 2 * P;
  return b;
}

size_t bias_mean_lds_bytes(int P) { return sizeof(double) * 2 * (size_t)P; }

hipError_t launch_bias(const BiasPlan& b, const int32_t* counts, const double* ep, const double* em,
                       int G, int P, const double* gpts, double g_abs, double* partial, double* gmean,
                       double* mc, double* stats, hipStream_t s) {
  const dim3 grid((2 * P + kTile - 1) / kTile, (b.R + kTile - 1) / kTile, b.n_split);
  hipLaunchKernelGGL(bias_gemm_kernel, grid, dim3(256), 0, s, counts, ep, em, G, P, b.R,
                     b.k_per_split, partial);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const size_t lds = bias_mean_lds_bytes(P);
  (void)hipFuncSetAttribute((const void*)bias_mean_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)lds);
  hipLaunchKernelGGL(bias_mean_kernel, dim3(b.R), dim3(kMeanThreads), lds, s, partial, b.n_split, b.R,
                     P, gpts, g_abs, gmean, mc);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(bias_stats_kernel, dim3(1), dim3(kMeanThreads), 0, s, mc, b.R, stats);
  return hipGetLastError();
}

}  // namespace bsi
