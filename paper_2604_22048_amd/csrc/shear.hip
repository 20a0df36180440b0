// Phase 2: Monte-Carlo shear likelihood (eq. likelihood-shear) from fixed
// interim samples, with the true prior of the intrinsic properties and the
// Jacobian of the inverse shear map (eq. true-prior-jacobian-shear):
//   eps = (eps' - g) / (1 - conj(g) eps'),
//   ln |d eps / d eps'| = 2 ln(1 - |g|^2) - 2 ln |1 - conj(g) eps'|^2.
// Layout: structure of arrays, float[n_gal][K] per field.  Grid: y = chunk of
// up to 64 points, x = block of galaxies.  A wave keeps one galaxy's samples
// in registers (K <= 64 * kMaxPerLane) and loops over the chunk's points; lane
// j accumulates point j of the chunk.  Log-weights are float; max, exp and the
// sums over samples and galaxies are float64.  Per-block partials are reduced
// in a fixed order by shear_reduce_kernel (bitwise reproducible).
#include "bsi_kernels.h"

namespace bsi {

namespace {

constexpr int kMaxPerLane = 16;    // K <= 1024
constexpr int kPtsPerChunk = 64;
constexpr double kPi = 3.14159265358979323846;

__device__ __forceinline__ double log_z_e(int kind, double sig, double emax) {
  if (kind == 0) {
    const double c = 1.0 / (2.0 * sig * sig), s2 = sig * sig;
    return log(kPi * (2.0 * s2 - 8.0 * s2 * s2 + 16.0 * s2 * s2 * s2 * (1.0 - exp(-c))));
  }
  return log(2.0 * kPi * sig * sig * (1.0 - exp(-emax * emax / (2.0 * sig * sig))));
}

__device__ __forceinline__ double dlog_z_e(int kind, double sig, double emax) {
  if (kind == 0) {
    const double c = 1.0 / (2.0 * sig * sig), ex = exp(-c);
    const double f = 2 * sig * sig - 8 * pow(sig, 4) + 16 * pow(sig, 6) * (1.0 - ex);
    const double fp = 4 * sig - 32 * pow(sig, 3) + 96 * pow(sig, 5) * (1.0 - ex) - 16 * pow(sig, 3) * ex;
    return fp / f;
  }
  const double c = emax * emax / (2.0 * sig * sig), ex = exp(-c);
  return 2.0 / sig - 2.0 * c * ex / (sig * (1.0 - ex));
}

struct Point {
  float g1, g2, mu, sig_s, inv2se2, inv_sig_s;
  float lnZ, dlnZ, sig_e, ln1mgg, gg;
  float size_c;    // ln(ln 10) - ln sig_s - ln(2 pi)/2 + ln(span_s)
};

__device__ __forceinline__ Point make_point(const double* p, const ShearArgs& a) {
  Point q;
  q.g1 = (float)p[0];
  q.g2 = (float)p[1];
  q.mu = (float)p[2];
  q.sig_s = (float)p[3];
  q.sig_e = (float)p[4];
  q.inv2se2 = (float)(1.0 / (2.0 * p[4] * p[4]));
  q.inv_sig_s = (float)(1.0 / p[3]);
  q.lnZ = (float)log_z_e(a.e_kind, p[4], a.e_max);
  q.dlnZ = (float)dlog_z_e(a.e_kind, p[4], a.e_max);
  const double gg = p[0] * p[0] + p[1] * p[1];
  q.gg = (float)gg;
  q.ln1mgg = (float)log(1.0 - gg);
  q.size_c = (float)(log(kLn10) - log(p[3]) - 0.5 * log(2.0 * kPi) + a.log_span_s);
  return q;
}

// ln w of one sample at one point, excluding the point-independent part c0
// (the interim ellipticity and flux terms, added by the caller).
__device__ __forceinline__ float logw_point(const Point& P, const ShearArgs& a, float e1, float e2,
                                           float ls, float& E_out, float& B_out, float& br_out,
                                           float& bi_out) {
  const float ar = e1 - P.g1, ai = e2 - P.g2;
  const float br = 1.0f - (P.g1 * e1 + P.g2 * e2);
  const float bi = P.g2 * e1 - P.g1 * e2;
  const float B = br * br + bi * bi;
  const float E = (ar * ar + ai * ai) / B;
  E_out = E;
  B_out = B;
  br_out = br;
  bi_out = bi;
  float lp;
  if (a.e_kind == 0) {
    lp = (E < 1.0f) ? 2.0f * __logf(1.0f - E) - E * P.inv2se2 - P.lnZ : -INFINITY;
  } else {
    lp = (E < a.e_max * a.e_max) ? -E * P.inv2se2 - P.lnZ : -INFINITY;
  }
  float lw = lp + 2.0f * P.ln1mgg - 2.0f * __logf(B);
  if (a.size_term) {
    const float z = (ls * kLn10F - P.mu) * P.inv_sig_s;
    lw += P.size_c - 0.5f * z * z;
  }
  return lw;
}

__global__ void __launch_bounds__(256) shear_kernel(ShearArgs a) {
  __shared__ double red[4][kPtsPerChunk][6];
  const int lane = lane_id(), wave = threadIdx.x / kWave;
  const int chunk0 = blockIdx.y * kPtsPerChunk;
  const int npc = min(kPtsPerChunk, a.n_pts - chunk0);
  double acc[6] = {0, 0, 0, 0, 0, 0};      // lane j: point chunk0 + j
  const int KL = (a.K + kWave - 1) / kWave;
  const int waves_total = gridDim.x * 4;
  const float lnZ0 = (float)log_z_e(0, a.sigma_e_interim, 1.0);
  const float inv2s0 = (float)(1.0 / (2.0 * a.sigma_e_interim * a.sigma_e_interim));
  for (int gal = blockIdx.x * 4 + wave; gal < a.n_gal; gal += waves_total) {
    float e1[kMaxPerLane], e2[kMaxPerLane], ls[kMaxPerLane], c0[kMaxPerLane];
    const int64_t base = (int64_t)gal * a.K;
#pragma unroll
    for (int i = 0; i < kMaxPerLane; ++i) {
      const int k = lane + i * kWave;
      e1[i] = e2[i] = ls[i] = 0.f;
      c0[i] = -INFINITY;
      if (i < KL && k < a.K) {
        e1[i] = a.e1p[base + k];
        e2[i] = a.e2p[base + k];
        ls[i] = a.l10s[base + k];
        const float Ep = e1[i] * e1[i] + e2[i] * e2[i];
        // minus the interim ellipticity density (eq. interim-prior, sigma_e = 0.3)
        float c = -(2.0f * __logf(1.0f - Ep) - Ep * inv2s0 - lnZ0);
        if (a.flux_term) {
          const float lf = a.l10f[base + k];
          const double z = ((double)lf * kLn10 - a.mu_lnf) / a.sig_lnf;
          c += (float)(log(kLn10) - log(a.sig_lnf) - 0.5 * log(2.0 * kPi) - 0.5 * z * z +
                       a.log_span_f);
        }
        c0[i] = c;
      }
    }
    for (int pj = 0; pj < npc; ++pj) {
      const Point P = make_point(a.pts + 5 * (int64_t)(chunk0 + pj), a);
      float lw[kMaxPerLane];
      float m = -INFINITY;
#pragma unroll
      for (int i = 0; i < kMaxPerLane; ++i) {
        lw[i] = -INFINITY;
        if (i < KL && c0[i] > -INFINITY) {
          float E, B, br, bi;
          lw[i] = logw_point(P, a, e1[i], e2[i], ls[i], E, B, br, bi) + c0[i];
          m = fmaxf(m, lw[i]);
        }
      }
      m = wave_max(m);
      double S = 0.0, Sd[5] = {0, 0, 0, 0, 0};
      if (m > -INFINITY) {
#pragma unroll
        for (int i = 0; i < kMaxPerLane; ++i) {
          if (i < KL && lw[i] > -INFINITY) {
            const double ex = exp((double)lw[i] - (double)m);
            S += ex;
            if (a.want_grad) {
              float E, B, br, bi;
              (void)logw_point(P, a, e1[i], e2[i], ls[i], E, B, br, bi);
              const float ar = e1[i] - P.g1, ai = e2[i] - P.g2;
              const float dB1 = 2.0f * (-br * e1[i] - bi * e2[i]);
              const float dB2 = 2.0f * (-br * e2[i] + bi * e1[i]);
              const float iB = 1.0f / B;
              const float dE1 = (-2.0f * ar - E * dB1) * iB;
              const float dE2 = (-2.0f * ai - E * dB2) * iB;
              const float dlp = (a.e_kind == 0) ? -2.0f / (1.0f - E) - P.inv2se2 : -P.inv2se2;
              const float omg = 1.0f - P.gg;
              const float d0 = dlp * dE1 - 4.0f * P.g1 / omg - 2.0f * dB1 * iB;
              const float d1 = dlp * dE2 - 4.0f * P.g2 / omg - 2.0f * dB2 * iB;
              float d2 = 0.f, d3 = 0.f;
              if (a.size_term) {
                const float z = (ls[i] * kLn10F - P.mu) * P.inv_sig_s;
                d2 = z * P.inv_sig_s;
                d3 = (z * z - 1.0f) * P.inv_sig_s;
              }
              const float d4 = E / (P.sig_e * P.sig_e * P.sig_e) - P.dlnZ;
              Sd[0] += ex * d0;
              Sd[1] += ex * d1;
              Sd[2] += ex * d2;
              Sd[3] += ex * d3;
              Sd[4] += ex * d4;
            }
          }
        }
      }
      S = wave_sum(S);
      double ell = (m > -INFINITY) ? (double)m + log(S) - log((double)a.K) : -INFINITY;
      if (lane == pj) acc[0] += ell;
      if (a.want_grad) {
#pragma unroll
        for (int j = 0; j < 5; ++j) {
          const double v = wave_sum(Sd[j]) / S;
          if (lane == pj) acc[1 + j] += v;
        }
      }
    }
  }
#pragma unroll
  for (int j = 0; j < 6; ++j) red[wave][lane][j] = acc[j];
  __syncthreads();
  for (int t = threadIdx.x; t < npc * 6; t += blockDim.x) {
    const int pj = t / 6, j = t - pj * 6;
    const double v = red[0][pj][j] + red[1][pj][j] + red[2][pj][j] + red[3][pj][j];
    a.partial[((int64_t)blockIdx.x * a.n_pts + chunk0 + pj) * 6 + j] = v;
  }
}

__global__ void shear_reduce_kernel(const double* __restrict__ partial, int n_blocks, int n_pts,
                                    const double* __restrict__ pts, double* __restrict__ logpost,
                                    double* __restrict__ grad) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n_pts) return;
  double v[6] = {0, 0, 0, 0, 0, 0};
  for (int b = 0; b < n_blocks; ++b)
#pragma unroll
    for (int j = 0; j < 6; ++j) v[j] += partial[((int64_t)b * n_pts + p) * 6 + j];
  const double* q = pts + 5 * (int64_t)p;
  const double gg = q[0] * q[0] + q[1] * q[1];
  const bool inside = gg < 1.0 && q[4] > 1e-4 && q[4] < 1.0 && fabs(q[2]) < 2.0 * kLn10 &&
                      q[3] > 0.0 && q[3] < 0.5 * kLn10;
  logpost[p] = inside ? v[0] : -INFINITY;
  if (grad)
#pragma unroll
    for (int j = 0; j < 5; ++j) grad[5 * (int64_t)p + j] = v[1 + j];
}

}  // namespace

hipError_t launch_shear(const ShearArgs& a, int n_blocks, hipStream_t s) {
  if (a.n_pts <= 0) return hipSuccess;
  const int chunks = (a.n_pts + kPtsPerChunk - 1) / kPtsPerChunk;
  hipLaunchKernelGGL(shear_kernel, dim3(n_blocks, chunks), dim3(256), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_shear_reduce(const double* partial, int n_blocks, int n_pts, const double* pts,
                               double* logpost, double* grad, hipStream_t s) {
  if (n_pts <= 0) return hipSuccess;
  hipLaunchKernelGGL(shear_reduce_kernel, dim3((n_pts + 127) / 128), dim3(128), 0, s, partial,
                     n_blocks, n_pts, pts, logpost, grad);
  return hipGetLastError();
}

}  // namespace bsi
