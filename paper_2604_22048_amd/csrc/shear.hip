// Phase 2: Monte-Carlo shear likelihood (eq. likelihood-shear) from fixed
// interim samples, with the true prior of the intrinsic properties and the
// Jacobian of the inverse shear map (eq. true-prior-jacobian-shear):
//   eps = (eps' - g) / (1 - conj(g) eps'),
//   ln |d eps / d eps'| = 2 ln(1 - |g|^2) - 2 ln |1 - conj(g) eps'|^2.
// Layout: structure of arrays, float[n_gal][K] per field.  Grid: y = chunk of
// up to 64 points, x = block of galaxies.  A wave keeps one galaxy's samples
// in registers (K <= 64 * kMaxPerLane) and loops over the chunk's points; lane
// j accumulates point j of the chunk.  Log-weights and the per-lane sums of
// their exponentials (at most 16 terms in (0, 1]) are float; the wave maximum,
// the sums across lanes and galaxies, the logarithm and the gradient assembly
// are float64.  Per-block partials are reduced in a fixed order (bitwise
// reproducible).
#include "bsi.h"
#include "bsi_kernels.h"

#include <mutex>

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

// Per-point constants, computed once per block (float64, rounded to float).
struct Point {
  float g1, g2, mu, inv2se2, inv_sig_s;
  float lnZ, dlnZ, inv_se3;
  float lw0;       // 2 ln(1 - |g|^2) (+ size normaliser ln(ln 10) - ln sig_s - ln(2 pi)/2 + ln span_s)
  float c1, c2;    // 4 g / (1 - |g|^2): the Jacobian's |g| derivative
  float pad;
};

__device__ Point make_point(const double* p, const ShearArgs& a) {
  Point q;
  q.g1 = (float)p[0];
  q.g2 = (float)p[1];
  q.mu = (float)p[2];
  q.inv2se2 = (float)(1.0 / (2.0 * p[4] * p[4]));
  q.inv_sig_s = (float)(1.0 / p[3]);
  q.inv_se3 = (float)(1.0 / (p[4] * p[4] * p[4]));
  q.lnZ = (float)log_z_e(a.e_kind, p[4], a.e_max);
  q.dlnZ = (float)dlog_z_e(a.e_kind, p[4], a.e_max);
  const double gg = p[0] * p[0] + p[1] * p[1];
  double lw0 = 2.0 * log(1.0 - gg);
  if (a.size_term) lw0 += log(kLn10) - log(p[3]) - 0.5 * log(2.0 * kPi) + a.log_span_s;
  q.lw0 = (float)lw0;
  q.c1 = (float)(4.0 * p[0] / (1.0 - gg));
  q.c2 = (float)(4.0 * p[1] / (1.0 - gg));
  q.pad = 0.f;
  return q;
}

// Inverse shear of one sample at one point: eps = (eps' - g) / (1 - conj(g) eps')
// as numerator a = eps' - g, denominator b = 1 - conj(g) eps', B = |b|^2 and
// E = |eps|^2 = |a|^2 / B.
struct Geo {
  float ar, ai, br, bi, iB, E;
};

__device__ __forceinline__ Geo geo(const Point& P, float e1, float e2) {
  Geo q;
  q.ar = e1 - P.g1;
  q.ai = e2 - P.g2;
  q.br = 1.0f - (P.g1 * e1 + P.g2 * e2);
  q.bi = P.g2 * e1 - P.g1 * e2;
  const float B = q.br * q.br + q.bi * q.bi;
  q.iB = __builtin_amdgcn_rcpf(B);
  q.E = (q.ar * q.ar + q.ai * q.ai) * q.iB;
  return q;
}

// ln w of one sample at one point without the point-independent part c0
// (interim ellipticity and flux terms): true ellipticity density, shear
// Jacobian 2 ln(1 - |g|^2) - 2 ln B, and the size term.
template <int EK, bool SZ>
__device__ __forceinline__ float logw(const Point& P, const ShearArgs& a, const Geo& q, float ls) {
  float lp;
  if (EK == 0)
    lp = (q.E < 1.0f) ? 2.0f * __logf(1.0f - q.E) - q.E * P.inv2se2 - P.lnZ : -INFINITY;
  else
    lp = (q.E < a.e_max * a.e_max) ? -q.E * P.inv2se2 - P.lnZ : -INFINITY;
  float lw = lp + P.lw0 + 2.0f * __logf(q.iB);
  if (SZ) {
    const float z = (ls * kLn10F - P.mu) * P.inv_sig_s;
    lw -= 0.5f * z * z;
  }
  return lw;
}

// Float64 totals over the wave of six per-lane float values, in one
// transposed reduction through the wave's LDS scratch (64 x 8 floats): lane
// l adds value l / 8 of lanes 8 (l % 8) .. 8 (l % 8) + 7 in float64, a
// three-step DPP prefix sum inside each group of eight lanes finishes it on
// lane 8 j + 7, and the six totals are read back as wave-uniform values.
// Fixed order: the totals are bitwise reproducible.
__device__ __forceinline__ void wave_total6_f64(const float* v, float* scratch, double* T) {
  const int lane = lane_id();
  float4* s4 = reinterpret_cast<float4*>(scratch);
  s4[2 * lane] = make_float4(v[0], v[1], v[2], v[3]);
  s4[2 * lane + 1] = make_float4(v[4], v[5], 0.f, 0.f);
  wave_lds_sync();
  const int val = lane >> 3, grp = lane & 7;
  double acc = 0.0;
#pragma unroll
  for (int k = 0; k < 8; ++k) acc += (double)scratch[(8 * grp + k) * 8 + val];
  acc = dpp_shift_add<0x111, 0xf>(acc);   // row_shr:1
  acc = dpp_shift_add<0x112, 0xf>(acc);   // row_shr:2
  acc = dpp_shift_add<0x114, 0xf>(acc);   // row_shr:4
#pragma unroll
  for (int j = 0; j < 6; ++j) T[j] = bcast(acc, 8 * j + 7);
  wave_lds_sync();
}

// A wave holds one galaxy's K samples in registers (lane l: samples
// l, l + 64, ...) and evaluates, for each point, the lane's log weights
// (first pass, kept in registers with their lane maximum m_l), then the
// lane's sums of e^(lw - m_l) times 1, the two g-derivative terms, z, z^2
// and E (second pass, float: at most 16 terms, each in (0, 1]).  The lane
// sums are combined across the wave in float64 after rescaling by
// e^(m_l - M), M the wave maximum, and the log-sum-exp and the gradient are
// assembled in float64.
// Minimum resident waves per SIMD requested from the register allocator.
#ifndef BSI_SHEAR_WAVES_PER_EU
#define BSI_SHEAR_WAVES_PER_EU 2
#endif

// Template flags: GRAD = a.want_grad, SZ = a.size_term, EK = a.e_kind.
template <bool GRAD, bool SZ, int EK>
__global__ void __launch_bounds__(256, BSI_SHEAR_WAVES_PER_EU) shear_kernel(ShearArgs a) {
  __shared__ double red[4][kPtsPerChunk][6];
  __shared__ Point pts_s[kPtsPerChunk];
  __shared__ __align__(16) float wred[4][64 * 8];     // per-wave transposed-reduction scratch
  const int lane = lane_id(), wave = threadIdx.x / kWave;
  const int chunk0 = blockIdx.y * kPtsPerChunk;
  const int npc = min(kPtsPerChunk, a.n_pts - chunk0);
  if ((int)threadIdx.x < npc) pts_s[threadIdx.x] = make_point(a.pts + 5 * (int64_t)(chunk0 + threadIdx.x), a);
  __syncthreads();
  double acc[6] = {0, 0, 0, 0, 0, 0};      // lane j: point chunk0 + j
  const int KL = (a.K + kWave - 1) / kWave;
  const int waves_total = gridDim.x * 4;
  const float lnZ0 = (float)log_z_e(0, a.sigma_e_interim, 1.0);
  const float inv2s0 = (float)(1.0 / (2.0 * a.sigma_e_interim * a.sigma_e_interim));
  const double logK = log((double)a.K);
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
        // minus the interim ellipticity density (eq. interim-prior)
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
      const Point P = pts_s[pj];
      // pass 1: log weights (padding and out-of-support samples -inf), lane maximum
      float lw[kMaxPerLane];
      float m = -INFINITY;
#pragma unroll
      for (int i = 0; i < kMaxPerLane; ++i) {
        lw[i] = (i < KL) ? logw<EK, SZ>(P, a, geo(P, e1[i], e2[i]), ls[i]) + c0[i] : -INFINITY;
        m = fmaxf(m, lw[i]);
      }
      // pass 2: the lane's sums of e^(lw - m) times 1 and the derivative terms;
      // every term is finite (E is clamped below 1 in the ellipticity-density
      // derivative) and carries the factor e^(lw - m), zero for -inf weights
      const float ms = (m > -INFINITY) ? m : 0.0f;
      float v[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};   // s0, u0, u1, t1, t2, tE
#pragma unroll
      for (int i = 0; i < kMaxPerLane; ++i) {
        if (i >= KL) continue;
        const float ex = __expf(lw[i] - ms);
        v[0] += ex;
        if (GRAD) {
          const Geo q = geo(P, e1[i], e2[i]);
          const float dB1 = 2.0f * (-q.br * e1[i] - q.bi * e2[i]);
          const float dB2 = 2.0f * (-q.br * e2[i] + q.bi * e1[i]);
          const float dE1 = (-2.0f * q.ar - q.E * dB1) * q.iB;
          const float dE2 = (-2.0f * q.ai - q.E * dB2) * q.iB;
          const float dlp = (EK == 0)
                                ? -2.0f * __builtin_amdgcn_rcpf(1.0f - fminf(q.E, 0.999999f)) - P.inv2se2
                                : -P.inv2se2;
          v[1] = fmaf(ex, dlp * dE1 - 2.0f * dB1 * q.iB, v[1]);
          v[2] = fmaf(ex, dlp * dE2 - 2.0f * dB2 * q.iB, v[2]);
          if (SZ) {
            const float z = (ls[i] * kLn10F - P.mu) * P.inv_sig_s;
            v[3] = fmaf(ex, z, v[3]);
            v[4] = fmaf(ex * z, z, v[4]);
          }
          v[5] = fmaf(ex, q.E, v[5]);
        }
      }
      // the wave maximum M, the lanes' sums rescaled by e^(m - M), and their
      // float64 totals over the wave in one transposed reduction
      const float M = wave_max(m);
      double ell = -INFINITY, g[5] = {0, 0, 0, 0, 0};
      if (M > -INFINITY) {
        const float f = (m > -INFINITY) ? __expf(m - M) : 0.0f;
#pragma unroll
        for (int j = 0; j < 6; ++j) v[j] *= f;
        double T[6];
        wave_total6_f64(v, wred[wave], T);
        const double S = T[0];
        ell = (double)M + log(S) - logK;
        if (GRAD) {
          const double iS = 1.0 / S;
          const double inv_ss = (double)P.inv_sig_s;
          g[0] = T[1] * iS - (double)P.c1;
          g[1] = T[2] * iS - (double)P.c2;
          if (SZ) {
            g[2] = inv_ss * T[3] * iS;
            g[3] = inv_ss * (T[4] * iS - 1.0);
          }
          g[4] = (double)P.inv_se3 * T[5] * iS - (double)P.dlnZ;
        }
      }
      if (lane == pj) {
        if (a.per_gal) a.per_gal[(int64_t)(chunk0 + pj) * a.n_gal + gal] = ell;
        acc[0] += ell;
#pragma unroll
        for (int j = 0; j < 5; ++j) acc[1 + j] += g[j];
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

constexpr int kRedThreads = 256;

// Sum of the per-block partials of point p, in a fixed order: thread i adds
// blocks i, i + 256, ..., then a pairwise tree over the threads.  The total
// is returned on thread 0 (bitwise reproducible for a given n_blocks).
__device__ __forceinline__ void reduce_point(const double* __restrict__ partial, int n_blocks,
                                             int n_pts, int p, double (*red)[6], double* v) {
  double acc[6] = {0, 0, 0, 0, 0, 0};
  for (int b = threadIdx.x; b < n_blocks; b += kRedThreads)
#pragma unroll
    for (int j = 0; j < 6; ++j) acc[j] += partial[((int64_t)b * n_pts + p) * 6 + j];
#pragma unroll
  for (int j = 0; j < 6; ++j) red[threadIdx.x][j] = acc[j];
  __syncthreads();
  for (int w = kRedThreads / 2; w >= 1; w >>= 1) {
    if ((int)threadIdx.x < w)
#pragma unroll
      for (int j = 0; j < 6; ++j) red[threadIdx.x][j] += red[threadIdx.x + w][j];
    __syncthreads();
  }
#pragma unroll
  for (int j = 0; j < 6; ++j) v[j] = red[0][j];
}

// Support of the uniform hyper-priors (|g| < 1, 1e-4 < sigma_e < 1,
// |mu_ln_s| < 2 ln 10, 0 < sigma_ln_s < ln 10 / 2).
__device__ __forceinline__ bool hyper_inside(const double* q) {
  const double gg = q[0] * q[0] + q[1] * q[1];
  return gg < 1.0 && q[4] > 1e-4 && q[4] < 1.0 && fabs(q[2]) < 2.0 * kLn10 && q[3] > 0.0 &&
         q[3] < 0.5 * kLn10;
}

// One block per point.
__global__ void __launch_bounds__(kRedThreads)
shear_reduce_kernel(const double* __restrict__ partial, int n_blocks, int n_pts,
                    const double* __restrict__ pts, double* __restrict__ logpost,
                    double* __restrict__ grad) {
  __shared__ double red[kRedThreads][6];
  const int p = blockIdx.x;
  double v[6];
  reduce_point(partial, n_blocks, n_pts, p, red, v);
  if (threadIdx.x != 0) return;
  logpost[p] = hyper_inside(pts + 5 * (int64_t)p) ? v[0] : -INFINITY;
  if (grad)
#pragma unroll
    for (int j = 0; j < 5; ++j) grad[5 * (int64_t)p + j] = v[1 + j];
}

// ---- shear-level HMC -----------------------------------------------------
// The sampler of the per-galaxy phase (fixed-length HMC, Philox momenta,
// float64 energies, dual-averaging warmup) run on x = (g1, g2, mu_ln_s,
// sigma_ln_s, sigma_e) with U = -ln P(g, alpha | d).  Each evaluation of U is
// one pass of shear_kernel over all interim samples at the n_chains current
// points; shear_hmc_update_kernel (one block per chain) reduces that pass and
// moves its chain to the next point, so one leapfrog step is two launches and
// no state leaves the device.  Box-Muller, the energy and the adaptation run
// in float64 on one thread per chain.

constexpr double kDaGamma = 0.05, kDaT0 = 10.0, kDaKappa = 0.75;
constexpr double kDivergence = 1000.0;

__device__ void shear_begin_iteration(const ShearHmcArgs& a, ShearChain& c, uint32_t uid,
                                      double* pt) {
  const uint32_t t = (uint32_t)c.t;
  const uint4 w0 = philox4x32_10(make_uint4(uid, t, kTagMomentum, 0), a.k0, a.k1);
  const uint4 w1 = philox4x32_10(make_uint4(uid, t, kTagMomentum, 1), a.k0, a.k1);
  const uint4 wa = philox4x32_10(make_uint4(uid, t, kTagAccept, 0), a.k0, a.k1);
  const uint32_t wu[6] = {w0.x, w0.y, w0.z, w0.w, w1.x, w1.y};
  double z[6];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const double r = sqrt(-2.0 * log((double)u01(wu[2 * k])));
    const double ang = 2.0 * 3.14159265358979323846 * (double)u01(wu[2 * k + 1]);
    z[2 * k] = r * cos(ang);
    z[2 * k + 1] = r * sin(ang);
  }
  c.u_acc = (double)u01(wa.x);
  float eps_t = c.eps;
  if (a.jitter > 0.0f) {
    const uint4 wj = philox4x32_10(make_uint4(uid, t, kTagJitter, 0), a.k0, a.k1);
    eps_t = (float)((double)c.eps * (1.0 + (double)a.jitter * (2.0 * (double)u01(wj.x) - 1.0)));
  }
  c.eps_t = eps_t;
  double ke = 0.0;
#pragma unroll
  for (int j = 0; j < 5; ++j) {
    c.p[j] = z[j] / sqrt(a.im[j]);
    ke += a.im[j] * c.p[j] * c.p[j];
  }
  c.H0 = c.U0 + 0.5 * ke;
  c.ok = 1;
  c.l = 0;
#pragma unroll
  for (int j = 0; j < 5; ++j) {
    c.p[j] -= 0.5 * (double)eps_t * c.g0[j];
    c.x[j] = c.x0[j] + (double)eps_t * a.im[j] * c.p[j];
    pt[j] = c.x[j];
  }
}

__global__ void __launch_bounds__(kRedThreads) shear_hmc_update_kernel(ShearHmcArgs a, int init) {
  __shared__ double red[kRedThreads][6];
  const int chain = blockIdx.x;
  double v[6];
  reduce_point(a.partial, a.n_blocks, a.C, chain, red, v);
  if (threadIdx.x != 0) return;
  ShearChain c = a.state[chain];
  double* pt = a.pts + 5 * (int64_t)chain;
  const uint32_t uid = (uint32_t)(a.uid_base + (uint64_t)chain);
  const double U = hyper_inside(pt) ? -v[0] : INFINITY;
  double gU[5];
#pragma unroll
  for (int j = 0; j < 5; ++j) gU[j] = -v[1 + j];
  if (init) {
#pragma unroll
    for (int j = 0; j < 5; ++j) {
      c.x0[j] = pt[j];
      c.g0[j] = gU[j];
    }
    c.U0 = U;
    c.eps = a.eps0;
    c.hbar = 0.0;
    c.lbar = 0.0;
    c.t = 0;
    c.n_acc = 0;
    c.n_div = 0;
    c.status = isfinite(U) ? 0u : 1u;
    c.sum_alpha = 0.0;
    if (a.t_stop > 0) shear_begin_iteration(a, c, uid, pt);
    a.state[chain] = c;
    return;
  }
  if (c.t >= a.t_stop) return;
  c.l += 1;
  if (!isfinite(U)) c.ok = 0;
  const double e = (double)c.eps_t;
  if (c.l < a.L) {
#pragma unroll
    for (int j = 0; j < 5; ++j) {
      c.p[j] -= e * gU[j];
      c.x[j] += e * a.im[j] * c.p[j];
      pt[j] = c.x[j];
    }
    a.state[chain] = c;
    return;
  }
  double ke = 0.0;
#pragma unroll
  for (int j = 0; j < 5; ++j) {
    c.p[j] -= 0.5 * e * gU[j];
    ke += a.im[j] * c.p[j] * c.p[j];
  }
  const double dH = U + 0.5 * ke - c.H0;
  const bool finite = isfinite(dH);
  const bool accept = c.ok && finite && log(c.u_acc) < -dH;
  const double alpha = (c.ok && finite) ? fmin(1.0, exp(-dH)) : 0.0;
  if (!finite || fabs(dH) > kDivergence) {
    c.n_div += 1;
    c.status |= finite ? 4u : 2u;
  }
  if (!c.ok) c.status |= 1u;
  if (a.trace) {
    float* tr = a.trace + ((int64_t)chain * a.t_stop + c.t) * 4;
    tr[0] = c.eps;
    tr[1] = (float)dH;
    tr[2] = (float)alpha;
    tr[3] = accept ? 1.0f : 0.0f;
  }
  if (accept) {
#pragma unroll
    for (int j = 0; j < 5; ++j) {
      c.x0[j] = c.x[j];
      c.g0[j] = gU[j];
    }
    c.U0 = U;
  }
  if (c.t < a.W) {
    if (a.adapt) {
      const double m = (double)(c.t + 1);
      const double eta = 1.0 / (m + kDaT0);
      c.hbar = (1.0 - eta) * c.hbar + eta * ((double)a.delta - alpha);
      const double le = a.mu - sqrt(m) / kDaGamma * c.hbar;
      const double xw = pow(m, -kDaKappa);
      c.lbar = xw * le + (1.0 - xw) * c.lbar;
      c.eps = (c.t == a.W - 1) ? (float)exp(c.lbar) : (float)exp(le);
    }
  } else {
    c.n_acc += accept ? 1 : 0;
    c.sum_alpha += alpha;
    if (a.samples) {
      double* o = a.samples + ((int64_t)chain * a.S + (c.t - a.W)) * 5;
#pragma unroll
      for (int j = 0; j < 5; ++j) o[j] = c.x0[j];
    }
  }
  c.t += 1;
  c.l = 0;
  if (c.t < a.t_stop) shear_begin_iteration(a, c, uid, pt);
  a.state[chain] = c;
}

__global__ void shear_hmc_stats_kernel(const ShearChain* __restrict__ st, int C, int S,
                                       double* __restrict__ stats) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= C) return;
  const ShearChain& x = st[c];
  stats[4 * c + 0] = S > 0 ? (double)x.n_acc / (double)S : 0.0;
  stats[4 * c + 1] = (double)x.eps;
  stats[4 * c + 2] = (double)x.n_div;
  stats[4 * c + 3] = -x.U0;
}

}  // namespace

hipError_t launch_shear(const ShearArgs& a, int n_blocks, hipStream_t s) {
  if (a.n_pts <= 0) return hipSuccess;
  const int chunks = (a.n_pts + kPtsPerChunk - 1) / kPtsPerChunk;
  const dim3 grid(n_blocks, chunks), blk(256);
  const int key = (a.want_grad ? 4 : 0) | (a.size_term ? 2 : 0) | (a.e_kind == 0 ? 0 : 1);
  switch (key) {
    case 0: hipLaunchKernelGGL((shear_kernel<false, false, 0>), grid, blk, 0, s, a); break;
    case 1: hipLaunchKernelGGL((shear_kernel<false, false, 1>), grid, blk, 0, s, a); break;
    case 2: hipLaunchKernelGGL((shear_kernel<false, true, 0>), grid, blk, 0, s, a); break;
    case 3: hipLaunchKernelGGL((shear_kernel<false, true, 1>), grid, blk, 0, s, a); break;
    case 4: hipLaunchKernelGGL((shear_kernel<true, false, 0>), grid, blk, 0, s, a); break;
    case 5: hipLaunchKernelGGL((shear_kernel<true, false, 1>), grid, blk, 0, s, a); break;
    case 6: hipLaunchKernelGGL((shear_kernel<true, true, 0>), grid, blk, 0, s, a); break;
    default: hipLaunchKernelGGL((shear_kernel<true, true, 1>), grid, blk, 0, s, a); break;
  }
  return hipGetLastError();
}

hipError_t launch_shear_reduce(const double* partial, int n_blocks, int n_pts, const double* pts,
                               double* logpost, double* grad, hipStream_t s) {
  if (n_pts <= 0) return hipSuccess;
  hipLaunchKernelGGL(shear_reduce_kernel, dim3(n_pts), dim3(kRedThreads), 0, s, partial, n_blocks,
                     n_pts, pts, logpost, grad);
  return hipGetLastError();
}

// ---- allocation-free evaluation pass ---------------------------------------
// Scratch of bsi_shear_posterior_noalloc: the per-block partial sums of one
// pass (blocks x points x 6 doubles), in a file-scope device array that every
// device holds, at its own address, while the library is loaded.  Host code
// never uses the array's name as an address: noalloc_scratch reads each
// device's address once, with that device current, through
// hipGetSymbolAddress, and the entry point passes that pointer to the kernels
// as the ordinary entry point passes its workspace.  shear_kernel writes every
// (block, point) entry before shear_reduce_kernel reads it, so nothing needs
// clearing between calls.
static __device__ __align__(256) unsigned char scratch[BSI_NOALLOC_SCRATCH_BYTES];
static std::mutex g_scratch_mutex;
static void* g_scratch_ptr[kMaxDevices] = {};

hipError_t noalloc_scratch(int device, void** ptr) {
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mutex);
  if (!g_scratch_ptr[device]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_ptr[device] = p;
  }
  *ptr = g_scratch_ptr[device];
  return hipSuccess;
}

hipError_t launch_shear_hmc_update(const ShearHmcArgs& a, int init, hipStream_t s) {
  if (a.C <= 0) return hipSuccess;
  hipLaunchKernelGGL(shear_hmc_update_kernel, dim3(a.C), dim3(kRedThreads), 0, s, a, init);
  return hipGetLastError();
}

hipError_t launch_shear_hmc_stats(const ShearChain* st, int C, int S, double* stats, hipStream_t s) {
  if (C <= 0 || !stats) return hipSuccess;
  hipLaunchKernelGGL(shear_hmc_stats_kernel, dim3(1), dim3(64), 0, s, st, C, S, stats);
  return hipGetLastError();
}

}  // namespace bsi
