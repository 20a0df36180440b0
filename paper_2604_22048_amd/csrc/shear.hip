// Phase 2: Monte-Carlo shear likelihood (eq. likelihood-shear) from fixed
// interim samples, with the true prior of the intrinsic properties and the
// Jacobian of the inverse shear map (eq. true-prior-jacobian-shear):
//   eps = (eps' - g) / (1 - conj(g) eps'),
//   ln |d eps / d eps'| = 2 ln(1 - |g|^2) - 2 ln |1 - conj(g) eps'|^2.
// Layout: structure of arrays, float[n_gal][K] per field.  Grid: y = chunk of
// up to 64 points, x = block of galaxies.  A wave keeps one galaxy's samples
// in registers (K <= 64 * kMaxPerLane; larger K in chunks of 512 samples) and
// loops over the chunk's points; lane j accumulates point j of the chunk.  Log-weights and the per-lane sums of
// their exponentials (at most 16 terms in (0, 1]) are float; the wave maximum,
// the sums across lanes and galaxies, the logarithm and the gradient assembly
// are float64.  Per-block partials are reduced in a fixed order (bitwise
// reproducible).
#include "bsi.h"
#include "bsi_kernels.h"

#include <algorithm>
#include <mutex>

namespace bsi {

namespace {

constexpr int kMaxPerLane = 16;    // samples per lane held at once (K <= 1024 in one chunk)
constexpr int kSampleGroup = 16;   // samples per scheduling group of the weight sums
constexpr int kPairPoints = 2;     // points evaluated together in the main pass
constexpr int kFewPoints = 16;     // at most this many points: the chunked form for K > 512
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
    const double s2 = sig * sig, s3 = s2 * sig, s4 = s2 * s2, s5 = s4 * sig, s6 = s4 * s2;
    const double f = 2 * s2 - 8 * s4 + 16 * s6 * (1.0 - ex);
    const double fp = 4 * sig - 32 * s3 + 96 * s5 * (1.0 - ex) - 16 * s3 * ex;
    return fp / f;
  }
  const double c = emax * emax / (2.0 * sig * sig), ex = exp(-c);
  return 2.0 / sig - 2.0 * c * ex / (sig * (1.0 - ex));
}

// Per-point constants, computed once per block.  The log weights are carried
// in log2 units (lw2 = ln w / ln 2) so that their exponentials are bare
// exp2; the point-independent part of ln w is folded into each sample's c0,
// the sample-independent part (k0) is added after the log-sum-exp.
struct Point {
  float g1, g2, gg;       // shear and |g|^2
  float a1;               // E coefficient of lw2: log2(e) / (2 sigma_e^2)
  float dlp;              // natural-unit E coefficient -1 / (2 sigma_e^2) (gradient)
  float w0;               // 2 - dlp: w = c - dlp = dlp E + w0
  float kz, kz0;          // zq = kz log10 s + kz0 = sqrt(log2(e) / 2) z, z = (ln s - mu) / sigma
  float du;               // -4 log2(1 - |g|): bound of -2 log2 B on the unit disk
  double g1d, g2d;        // shear in float64 (gradient assembly)
  double k0;              // 2 ln(1 - |g|^2) - ln Z (+ size normaliser): natural units
  double c1, c2;          // 4 g / (1 - |g|^2): the Jacobian's |g| derivative
  double inv_sig_s, inv_se3, dlnZ;
};

// Dynamic LDS of shear_kernel for npa points: the point records (twice for
// the chunked form) and the points' constants.
inline size_t shear_dyn_lds(int npa, bool multi) {
  return sizeof(double) * (multi ? 64 : 32) * npa + sizeof(Point) * npa;
}

constexpr double kLog2e = 1.44269504088896340736;
constexpr double kLn2 = 0.69314718055994530942;
// zq^2 = log2(e) z^2 / 2, so z = zq / kZq and z^2 = zq^2 / kZq^2
constexpr double kZq = 0.84932180028801904272;   // sqrt(log2(e) / 2)

__device__ Point make_point(const double* p, const ShearArgs& a) {
  Point q;
  q.g1 = (float)p[0];
  q.g2 = (float)p[1];
  const double gg = p[0] * p[0] + p[1] * p[1];
  q.gg = (float)gg;
  const double i2s = 1.0 / (2.0 * p[4] * p[4]);
  q.a1 = (float)(kLog2e * i2s);
  q.dlp = (float)(-i2s);
  q.w0 = (float)(2.0 + i2s);
  q.kz = (float)(kZq * kLn10 / p[3]);
  q.kz0 = (float)(-kZq * p[2] / p[3]);
  // rounded up, so that the weight bound stays a bound
  q.du = (float)(-4.0 * log2(1.0 - sqrt(gg)) * (1.0 + 1e-6) + 1e-6);
  q.g1d = p[0];
  q.g2d = p[1];
  double k0 = 2.0 * log(1.0 - gg) - log_z_e(a.e_kind, p[4], a.e_max);
  if (a.size_term) k0 += log(kLn10) - log(p[3]) - 0.5 * log(2.0 * kPi) + a.log_span_s;
  q.k0 = k0;
  q.c1 = 4.0 * p[0] / (1.0 - gg);
  q.c2 = 4.0 * p[1] / (1.0 - gg);
  q.inv_sig_s = 1.0 / p[3];
  q.inv_se3 = 1.0 / (p[4] * p[4] * p[4]);
  q.dlnZ = dlog_z_e(a.e_kind, p[4], a.e_max);
  return q;
}

// Wave maximum with DPP row shifts and row broadcasts (lanes without a
// source keep their own value); the total is read from lane 63.
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ float dpp_max_step(float x) {
  const int v = __float_as_int(x);
  return fmaxf(x, __int_as_float(__builtin_amdgcn_update_dpp(v, v, CTRL, ROW_MASK, 0xf, false)));
}

__device__ __forceinline__ float wave_max_dpp(float x) {
  x = dpp_max_step<0x111, 0xf>(x);   // row_shr:1
  x = dpp_max_step<0x112, 0xf>(x);   // row_shr:2
  x = dpp_max_step<0x114, 0xf>(x);   // row_shr:4
  x = dpp_max_step<0x118, 0xf>(x);   // row_shr:8
  x = dpp_max_step<0x142, 0xa>(x);   // row_bcast:15 into rows 1 and 3
  x = dpp_max_step<0x143, 0xc>(x);   // row_bcast:31 into rows 2 and 3
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x), 63));
}

// Float64 totals over the wave of seven per-lane float values, in one
// transposed reduction through the wave's LDS scratch (64 x 8 floats): lane
// l adds value l / 8 of lanes 8 (l % 8) .. 8 (l % 8) + 7 in float64, and a
// three-step DPP prefix sum inside each group of eight lanes finishes total j
// on lane 8 j + 7 (returned there; value 7 is zero).  Fixed order: the totals
// are bitwise reproducible.
__device__ __forceinline__ double wave_group8_f64(const float* v, float* scratch) {
  const int lane = lane_id();
  float4* s4 = reinterpret_cast<float4*>(scratch);
  s4[2 * lane] = make_float4(v[0], v[1], v[2], v[3]);
  s4[2 * lane + 1] = make_float4(v[4], v[5], v[6], 0.f);
  wave_lds_sync();
  const int val = lane >> 3, grp = lane & 7;
  double acc = 0.0;
#pragma unroll
  for (int k = 0; k < 8; ++k) acc += (double)scratch[(8 * grp + k) * 8 + val];
  acc = dpp_shift_add<0x111, 0xf>(acc);   // row_shr:1
  acc = dpp_shift_add<0x112, 0xf>(acc);   // row_shr:2
  acc = dpp_shift_add<0x114, 0xf>(acc);   // row_shr:4
  wave_lds_sync();
  return acc;
}

// One sample's log weight at a point, in log2 units, and the quantities the
// gradient needs: B = |1 - conj(g) e'|^2 = 1 - 2 Re(conj(g) e') + |g|^2 |e'|^2,
// E = |e' - g|^2 / B with |e' - g|^2 = |e'|^2 - 2 Re(conj(g) e') + |g|^2,
// lw2 = c0 - a1 E - 2 log2 B - zq^2 (+ 2 log2(1 - E) for the unit-disk density),
// -inf outside the density's support.
template <bool SZ, int EK>
__device__ __forceinline__ float sample_lw(const Point& P, float emax2, float e1, float e2, float ep2,
                                           float ls, float c0, float& E, float& iB, float& zq) {
  const float dot = fmaf(P.g2, e2, P.g1 * e1);
  const float B = fmaf(P.gg, ep2, fmaf(-2.0f, dot, 1.0f));
  iB = __builtin_amdgcn_rcpf(B);
  E = fmaf(-2.0f, dot, ep2 + P.gg) * iB;
  float l = fmaf(-E, P.a1, c0);
  l = fmaf(-2.0f, __builtin_amdgcn_logf(B), l);
  if (EK == 0) {
    l = fmaf(2.0f, __builtin_amdgcn_logf(1.0f - E), l);
    l = (E < 1.0f) ? l : -INFINITY;
  } else {
    l = (E < emax2) ? l : -INFINITY;
  }
  if (SZ) {
    zq = fmaf(ls, P.kz, P.kz0);
    l = fmaf(-zq, zq, l);
  }
  return l;
}

// One sample's weight against a reference U, x = 2^(lw2 - U), formed as
// 2^(c0 - U - a1 E - zq^2) / B^2 (times (1 - E)^2 for the unit-disk density):
// the same value as exp2 of sample_lw's sum, with the logarithms of B and
// 1 - E replaced by products (one transcendental instead of three), and 0
// outside the density's support.  ep2 = |e'|^2 of the sample.
template <bool SZ, int EK>
__device__ __forceinline__ float sample_x(const Point& P, float emax2, float e1, float e2, float ep2,
                                          float ls, float c0U, float& E, float& iB, float& zq) {
  const float dot = fmaf(P.g2, e2, P.g1 * e1);
  const float B = fmaf(P.gg, ep2, fmaf(-2.0f, dot, 1.0f));
  iB = __builtin_amdgcn_rcpf(B);
  E = fmaf(-2.0f, dot, ep2 + P.gg) * iB;
  float l = fmaf(-E, P.a1, c0U);
  if (SZ) {
    zq = fmaf(ls, P.kz, P.kz0);
    l = fmaf(-zq, zq, l);
  }
  float x = __builtin_amdgcn_exp2f(l) * (iB * iB);
  if (EK == 0) {
    const float om = 1.0f - E;
    x = (E < 1.0f) ? x * (om * om) : 0.0f;
  } else {
    x = (E < emax2) ? x : 0.0f;
  }
  return x;
}

// The lane's sums over its samples at NP points at once (independent work
// for the scheduler to interleave), each weight taken as x = 2^(lw2 - U) for
// a wave-uniform reference U of its point: x and, with the gradient,
// x/B (dlp - c |e'|^2), x/B (c - dlp) e1', x/B (c - dlp) e2', x zq, x zq^2,
// x E, where c = dlp E + 2 and dlp = d ln p_e / dE (natural units): the
// g-derivative of ln w is 2/B [g (dlp - c |e'|^2) + (c - dlp) e'] - 4 g /
// (1 - |g|^2), so g enters only after the sums.
template <bool GRAD, bool SZ, int EK, int NS, int NP = 1>
__device__ __forceinline__ void lane_sums(const Point* const* Ps, float emax2, const float* e1,
                                          const float* e2, const float* ep2, const float* ls,
                                          const float* c0, const float* U, float (*v)[7]) {
#pragma unroll
  for (int p = 0; p < NP; ++p)
#pragma unroll
    for (int j = 0; j < 7; ++j) v[p][j] = 0.f;
#pragma unroll
  for (int i = 0; i < NS; ++i) {
#pragma unroll
    for (int p = 0; p < NP; ++p) {
      const Point& P = *Ps[p];
      float E, iB, zq = 0.f;
      const float x = sample_x<SZ, EK>(P, emax2, e1[i], e2[i], ep2[i], ls[i], c0[i] - U[p], E, iB, zq);
      v[p][0] += x;
      if (GRAD) {
        float c, w, dl;
        if (EK == 0) {
          dl = fmaf(-2.0f, __builtin_amdgcn_rcpf(1.0f - fminf(E, 0.999999f)), P.dlp);
          c = fmaf(dl, E, 2.0f);
          w = c - dl;
        } else {
          dl = P.dlp;
          c = fmaf(dl, E, 2.0f);
          w = fmaf(dl, E, P.w0);
        }
        const float u = fmaf(-c, ep2[i], dl);
        const float q = x * iB;
        v[p][1] = fmaf(q, u, v[p][1]);
        const float r = q * w;
        v[p][2] = fmaf(r, e1[i], v[p][2]);
        v[p][3] = fmaf(r, e2[i], v[p][3]);
        if (SZ) {
          const float xz = x * zq;
          v[p][4] += xz;
          v[p][5] = fmaf(xz, zq, v[p][5]);
        }
        v[p][6] = fmaf(x, E, v[p][6]);
      }
    }
    // groups of kSampleGroup samples: the scheduler interleaves within a
    // group only, which bounds the live temporaries (and so the registers)
    if ((i % kSampleGroup) == kSampleGroup - 1) __builtin_amdgcn_sched_barrier(0);
  }
}

// The wave maximum of the log weights at one point.
template <bool SZ, int EK, int NS>
__device__ __forceinline__ float wave_lw_max(const Point& P, float emax2, const float* e1, const float* e2,
                                             const float* ep2, const float* ls, const float* c0) {
  float m = -INFINITY;
#pragma unroll
  for (int i = 0; i < NS; ++i) {
    float E, iB, zq;
    m = fmaxf(m, sample_lw<SZ, EK>(P, emax2, e1[i], e2[i], ep2[i], ls[i], c0[i], E, iB, zq));
  }
  return wave_max_dpp(m);
}

// Wait counters (gfx9 encoding): all vector memory operations done; all LDS
// operations done.
constexpr int kWaitVmcnt0 = 0x0F70;
constexpr int kWaitLgkmcnt0 = 0xC07F;
// A point whose total weight against the bound falls below this is evaluated
// again against its exact maximum (weights below 2^-126 of the bound would
// have underflowed).
constexpr double kLooseTotal = 0x1p-60;

// A wave holds one galaxy's K samples in registers (lane l: samples l,
// l + 64, ...; NS slots per lane, padding slots with weight zero) with the
// point-independent part of each log weight (c0: minus the interim
// ellipticity density, plus the flux term) in log2 units; the next galaxy's
// samples stream into LDS meanwhile.  Per point one pass over the samples
// forms the lane's sums with weights 2^(lw2 - U) against the wave-uniform
// bound U = max c0 - 4 log2(1 - |g|) >= lw2 (the other terms are <= 0, and
// B >= (1 - |g|)^2 on the unit disk), so nothing is stored per sample and no
// lane needs rescaling; the sums are totalled over the wave in float64 into
// the wave's LDS record of the point.  A point whose total weight comes out
// below 2^-60 (extreme population parameters: tiny sigma_e or sigma_s) is
// evaluated again against the exact wave maximum of its log weights, so no
// weight that matters underflows.  When every point of the chunk is done,
// lane j finishes point j from its record -- the float64 logarithm of the
// log-sum-exp and the gradient assembly -- so those run once per point, in
// parallel across the lanes.
//
// MULTI (K > 64 NS): a galaxy's samples are taken in chunks of 64 NS; each
// chunk's totals (against the chunk's own bound, with the same fallback) are
// added in float64 into a running record per point, rescaled to the larger
// of the two references, and the finish runs after the galaxy's last chunk.
//
// LDS: the sample buffers and the reduction scratch are static; the point
// records (and the running records, MULTI) and the points' constants are
// dynamic, sized for npa = min(64, n_pts) points (shear_dyn_lds), so that a
// pass over few points (the shear-level sampler's chains) leaves LDS room for
// more resident blocks.  NS <= 8 kernels are built for three waves per SIMD.
template <bool GRAD, bool SZ, int EK, int NS, bool MULTI = false>
__global__ void __launch_bounds__(256, (NS <= 8 ? 3 : 2)) shear_kernel(ShearArgs a) {
  constexpr int CH = NS * kWave;   // samples per chunk
  // per wave: the next chunk's e1', e2', log10 s, loaded straight into LDS
  // while the current one is evaluated (sample k of the chunk at index k)
  __shared__ float pre[4][3][CH];
  __shared__ __align__(16) float wred[4][64 * 8];       // per-wave transposed-reduction scratch
  // dynamic: per-wave point records [4][npa][8] (7 totals, reference U) of the
  // current chunk, which also hold the block's per-point sums at the end;
  // per-wave running records [4][npa][8] of the galaxy over its chunks
  // (MULTI only); the points' constants [npa]
  extern __shared__ double dyn_s[];
  const int npa = min(kPtsPerChunk, a.n_pts);
  double* fin = dyn_s;
  Point* pts_s = reinterpret_cast<Point*>(dyn_s + (MULTI ? 64 : 32) * npa);
  const int lane = lane_id(), wave = threadIdx.x / kWave;
  const int chunk0 = blockIdx.y * kPtsPerChunk;
  const int npc = min(kPtsPerChunk, a.n_pts - chunk0);
  const int waves_total = gridDim.x * 4;
  const int nch = MULTI ? (a.K + CH - 1) / CH : 1;   // sample chunks per galaxy
  // LDS DMA of chunk c of galaxy g into this wave's buffer (lanes past K load
  // the chunk's first sample, masked when read)
  auto prefetch = [&](int g, int c) {
    const int64_t base = (int64_t)g * a.K + (int64_t)c * CH;
#pragma unroll
    for (int i = 0; i < NS; ++i) {
      const int k = lane + i * kWave;
      const int64_t o = base + (c * CH + k < a.K ? k : 0);
      __builtin_amdgcn_global_load_lds(a.e1p + o, &pre[wave][0][i * kWave], 4, 0, 0);
      __builtin_amdgcn_global_load_lds(a.e2p + o, &pre[wave][1][i * kWave], 4, 0, 0);
      if (SZ) __builtin_amdgcn_global_load_lds(a.l10s + o, &pre[wave][2][i * kWave], 4, 0, 0);
    }
  };
  int gal = blockIdx.x * 4 + wave, ch = 0;
  if (gal < a.n_gal) prefetch(gal, 0);
  // the points' constants, while the first galaxy's samples are in flight
  if ((int)threadIdx.x < npc) pts_s[threadIdx.x] = make_point(a.pts + 5 * (int64_t)(chunk0 + threadIdx.x), a);
  __syncthreads();
  double acc[6] = {0, 0, 0, 0, 0, 0};      // lane j: point chunk0 + j
  // minus the interim ellipticity density (eq. interim-prior) in log2 units:
  // -2 log2(1 - E') + E' b0 + lz0, b0 = log2(e) / (2 sigma0^2), lz0 = log2 Z0
  const float b0 = a.b0, lz0 = a.lz0;
  const double logK = a.logK;
  const float emax2 = a.e_max * a.e_max;
  double* rec = fin + wave * npa * 8;
  double* run = dyn_s + 32 * npa + wave * npa * 8;   // MULTI only
  while (gal < a.n_gal) {
    float e1[NS], e2[NS], ep2[NS], ls[NS], c0[NS];
    // this chunk's samples have landed: move them to registers, then start
    // the next chunk's transfer (of this galaxy or the next) into the freed buffer
    __builtin_amdgcn_s_waitcnt(kWaitVmcnt0);
    wave_lds_sync();
#pragma unroll
    for (int i = 0; i < NS; ++i) {
      e1[i] = pre[wave][0][i * kWave + lane];
      e2[i] = pre[wave][1][i * kWave + lane];
      ls[i] = SZ ? pre[wave][2][i * kWave + lane] : 0.f;
    }
    __builtin_amdgcn_s_waitcnt(kWaitLgkmcnt0);
    wave_lds_sync();
    int next_gal = gal, next_ch = ch + 1;
    if (next_ch == nch) {
      next_gal = gal + waves_total;
      next_ch = 0;
    }
    if (next_gal < a.n_gal) prefetch(next_gal, next_ch);
    float cmax = -INFINITY;
#pragma unroll
    for (int i = 0; i < NS; ++i) {
      const int k = ch * CH + lane + i * kWave;   // the sample's index in the galaxy
      c0[i] = -INFINITY;
      if (k >= a.K) {
        e1[i] = e2[i] = ls[i] = 0.f;
      }
      ep2[i] = fmaf(e1[i], e1[i], e2[i] * e2[i]);
      if (k < a.K) {
        const float Ep = ep2[i];
        float c = fmaf(-2.0f, __builtin_amdgcn_logf(1.0f - Ep), fmaf(Ep, b0, lz0));
        if (a.flux_term) {
          const float lf = a.l10f[(int64_t)gal * a.K + k];
          const double z = ((double)lf * kLn10 - a.mu_lnf) / a.sig_lnf;
          c += (float)(kLog2e * (log(kLn10) - log(a.sig_lnf) - 0.5 * log(2.0 * kPi) - 0.5 * z * z +
                                 a.log_span_f));
        }
        c0[i] = c;
        cmax = fmaxf(cmax, c);
      }
    }
    const float cwave = wave_max_dpp(cmax);
    // kPairPoints points per pass over the samples, then the remaining ones
    // singly; each point's sums are totalled over the wave in float64 (lane
    // 8 j + 7 holds total j) into the point's record, with U in slot 7
    int pj = 0;
    for (; pj + kPairPoints <= npc; pj += kPairPoints) {
      const Point* Ps[kPairPoints];
      float U[kPairPoints], v[kPairPoints][7];
#pragma unroll
      for (int p = 0; p < kPairPoints; ++p) {
        Ps[p] = &pts_s[pj + p];
        U[p] = (cwave > -INFINITY) ? cwave + Ps[p]->du : 0.0f;
      }
      lane_sums<GRAD, SZ, EK, NS, kPairPoints>(Ps, emax2, e1, e2, ep2, ls, c0, U, v);
#pragma unroll
      for (int p = 0; p < kPairPoints; ++p) {
        const double t = wave_group8_f64(v[p], wred[wave]);
        if ((lane & 7) == 7) rec[(pj + p) * 8 + (lane >> 3)] = (lane == 63) ? (double)U[p] : t;
      }
    }
    for (; pj < npc; ++pj) {
      const Point* Ps[1] = {&pts_s[pj]};
      float U[1] = {(cwave > -INFINITY) ? cwave + Ps[0]->du : 0.0f}, v[1][7];
      lane_sums<GRAD, SZ, EK, NS>(Ps, emax2, e1, e2, ep2, ls, c0, U, v);
      const double t = wave_group8_f64(v[0], wred[wave]);
      if ((lane & 7) == 7) rec[pj * 8 + (lane >> 3)] = (lane == 63) ? (double)U[0] : t;
    }
    wave_lds_sync();
    // points whose total weight against the bound is tiny (or zero): again
    // against the exact maximum of their log weights
    {
      const bool loose = lane < npc && rec[lane * 8] < kLooseTotal;
      uint64_t todo = __builtin_amdgcn_ballot_w64(loose);
      while (todo) {
        const int pj = __builtin_ctzll(todo);
        todo &= todo - 1;
        const Point* Ps[1] = {&pts_s[pj]};
        const float M = wave_lw_max<SZ, EK, NS>(*Ps[0], emax2, e1, e2, ep2, ls, c0);
        float v[1][7] = {{0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f}};
        if (M > -INFINITY) lane_sums<GRAD, SZ, EK, NS>(Ps, emax2, e1, e2, ep2, ls, c0, &M, v);
        const double t = wave_group8_f64(v[0], wred[wave]);
        if ((lane & 7) == 7) rec[pj * 8 + (lane >> 3)] = (lane == 63) ? (double)M : t;
      }
      wave_lds_sync();
    }
    if constexpr (MULTI) {
      // lane j adds the chunk's record of point j into the galaxy's running
      // record, both scaled to the larger reference (float64)
      if (lane < npc) {
        double* Rr = run + lane * 8;
        const double* T = rec + lane * 8;
        if (ch == 0 || !(Rr[0] > 0.0)) {
#pragma unroll
          for (int j = 0; j < 8; ++j) Rr[j] = T[j];
        } else if (T[0] > 0.0) {
          const double Un = fmax(Rr[7], T[7]);
          const double fo = exp2(Rr[7] - Un), fn = exp2(T[7] - Un);
#pragma unroll
          for (int j = 0; j < 7; ++j) Rr[j] = Rr[j] * fo + T[j] * fn;
          Rr[7] = Un;
        }
      }
      wave_lds_sync();
    }
    const int cur = gal;
    const bool last = ch + 1 == nch;
    gal = next_gal;
    ch = next_ch;
    if (!last) continue;
    // lane j finishes point j: log-sum-exp and gradient in float64
    if (lane < npc) {
      const Point& P = pts_s[lane];
      const double* T = (MULTI ? run : rec) + lane * 8;
      const double S = T[0];
      double ell = -INFINITY, g[5] = {0, 0, 0, 0, 0};
      if (S > 0.0) {
        ell = T[7] * kLn2 + log(S) + P.k0 - logK;
        if (GRAD) {
          const double iS = 1.0 / S;
          g[0] = 2.0 * (P.g1d * T[1] + T[2]) * iS - P.c1;
          g[1] = 2.0 * (P.g2d * T[1] + T[3]) * iS - P.c2;
          if (SZ) {
            g[2] = P.inv_sig_s * T[4] * iS * (1.0 / kZq);
            g[3] = P.inv_sig_s * (T[5] * iS * (1.0 / (kZq * kZq)) - 1.0);
          }
          g[4] = P.inv_se3 * T[6] * iS - P.dlnZ;
        }
      }
      if (a.per_gal) a.per_gal[(int64_t)(chunk0 + lane) * a.n_gal + cur] = ell;
      acc[0] += ell;
#pragma unroll
      for (int j = 0; j < 5; ++j) acc[1 + j] += g[j];
    }
    wave_lds_sync();
  }
  __syncthreads();    // every wave is done with its records
  double* red = fin;   // [4][npa][6]: each wave's per-point sums
  if (lane < npc)
#pragma unroll
    for (int j = 0; j < 6; ++j) red[(wave * npa + lane) * 6 + j] = acc[j];
  __syncthreads();
  for (int t = threadIdx.x; t < npc * 6; t += blockDim.x) {
    const int pj = t / 6, j = t - pj * 6;
    const double v = red[pj * 6 + j] + red[(npa + pj) * 6 + j] + red[(2 * npa + pj) * 6 + j] +
                     red[(3 * npa + pj) * 6 + j];
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

// One chain's move after an evaluation pass (v: the pass's totals at the
// chain's current point): the leapfrog, the Metropolis test at a trajectory's
// end, dual averaging, the next trajectory's start; pt then holds the chain's
// next evaluation point.
__device__ void shear_hmc_move(const ShearHmcArgs& a, int init, int chain, const double* v) {
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

__global__ void __launch_bounds__(kRedThreads) shear_hmc_update_kernel(ShearHmcArgs a, int init) {
  __shared__ double red[kRedThreads][6];
  const int chain = blockIdx.x;
  double v[6];
  reduce_point(a.partial, a.n_blocks, a.C, chain, red, v);
  if (threadIdx.x != 0) return;
  shear_hmc_move(a, init, chain, v);
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
  const int KL = (a.K + kWave - 1) / kWave;
  const int npa = std::min(kPtsPerChunk, a.n_pts);
  // 4, 8 or 16 sample slots per lane; beyond 16 x 64 samples, or beyond 8 x 64
  // with few points (whose records leave LDS room for a third wave per SIMD),
  // chunks of 8 x 64
  const int ns = KL <= 4 ? 0 : KL <= 8 ? 1 : (KL <= kMaxPerLane && npa > kFewPoints) ? 2 : 3;
  const size_t lds = shear_dyn_lds(npa, ns == 3);
  const int key = (a.want_grad ? 4 : 0) | (a.size_term ? 2 : 0) | (a.e_kind == 0 ? 0 : 1);
  switch (key * 4 + ns) {
#define BSI_SHEAR_CASE(G, S, E)                                                                     \
    case ((G) * 4 + (S) * 2 + (E)) * 4 + 0:                                                         \
      hipLaunchKernelGGL((shear_kernel<G, S, E, 4>), grid, blk, lds, s, a); break;                  \
    case ((G) * 4 + (S) * 2 + (E)) * 4 + 1:                                                         \
      hipLaunchKernelGGL((shear_kernel<G, S, E, 8>), grid, blk, lds, s, a); break;                  \
    case ((G) * 4 + (S) * 2 + (E)) * 4 + 2:                                                         \
      hipLaunchKernelGGL((shear_kernel<G, S, E, 16>), grid, blk, lds, s, a); break;                 \
    case ((G) * 4 + (S) * 2 + (E)) * 4 + 3:                                                         \
      hipLaunchKernelGGL((shear_kernel<G, S, E, 8, true>), grid, blk, lds, s, a); break;
    BSI_SHEAR_CASE(false, false, 0) BSI_SHEAR_CASE(false, false, 1)
    BSI_SHEAR_CASE(false, true, 0) BSI_SHEAR_CASE(false, true, 1)
    BSI_SHEAR_CASE(true, false, 0) BSI_SHEAR_CASE(true, false, 1)
    BSI_SHEAR_CASE(true, true, 0) BSI_SHEAR_CASE(true, true, 1)
#undef BSI_SHEAR_CASE
    default: return hipErrorInvalidValue;
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
