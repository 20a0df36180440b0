// Batched Hamiltonian Monte Carlo over the per-galaxy interim posteriors
// (eq. interim-post: pixel likelihood eq. likelihood-pixels times the interim
// prior eq. interim-prior), one wave per chain, the chains of one galaxy in
// one workgroup sharing that galaxy's data spectrum in LDS.
//
// A launch advances every chain of its galaxies by n_steps leapfrog steps,
// crossing trajectory boundaries as needed (a chain's state, including a
// trajectory in progress, lives in a 256-byte ChainState between launches).
// The batched form launches all galaxies with n_steps = L * iterations; the
// plain form launches one galaxy with n_steps = 1.  Both run the same code.
//
// Iteration t of a chain (Neal 2011, with the paper's dual-averaging warmup):
//   momentum p = z / sqrt(inv_mass), z from Philox (uid, t, 0, 0..1) by
//   Box-Muller; step eps_t = eps (1 + j (2u - 1)), u from Philox (uid, t, 3, 0);
//   L leapfrog steps; dH = H_end - H_start in float64; accept iff
//   ln u < -dH with u from Philox (uid, t, 1, 0); a trajectory that leaves the
//   support or has a non-finite dH is rejected; during warmup the step is
//   adapted by dual averaging (Hoffman & Gelman 2014, Algorithm 5) on
//   alpha = min(1, exp(-dH)).
#include <algorithm>

#include "bsi_kernels.h"
#include "kspace.h"

namespace bsi {

namespace {

constexpr double kDaGamma = 0.05, kDaT0 = 10.0, kDaKappa = 0.75;
constexpr double kDivergence = 1000.0;
constexpr float kEClamp = 1.0f - 1e-6f;

struct GalCtx {
  Geom g;
  SlotPlan sp;
  const float2* dh;
  const float* atab;
  float2* X;       // per-wave tables (see fill_tables); the Fisher metric reuses
  float4* Ym;      // X and Yf as full x and y tables
  float2* Yf;
  float* red;      // per-wave reduction scratch (2 KiB)
  const float4* cols;   // the workgroup's pair-slot column table
  int part;        // this wave's index among the W waves of its chain
  float* xch;      // the chain's partial-sum exchange area (2 x W x 12 floats)
  float norm;      // 1 / (N^2 sigma^2)
  float rscale;
  float nu;        // Spergel index (Spergel profile only)
  float refx, refy;
  // several exposures / correlated noise (MX kernels): exposure j's spectrum
  // at dh + j dstride, its sqrt-weights at sqw + j wstride, its PSF-sinc
  // table at atab + j astride, its noise sigma sig[j] and DFT-mode noise
  // powers nps + off[s0 + j] (NULL: white)
  int E, dstride, wstride, astride;
  const float* sqw;
  const float* sig;
  const float* nps;
  const int64_t* off;
  int64_t s0;
  int t_stop;      // iteration at which this galaxy's chains stop in this launch
};

// Plain separable tables over the full frequency range (Fisher metric only):
// X[u+h] = a(u) exp(-i k_u dx), Y[v+h] = a(v) exp(-i k_v dy).
__device__ __forceinline__ void fill_xy_full(const Geom& g, const float* __restrict__ atab, float2* X,
                                             float2* Y, float dx, float dy) {
  const int lane = lane_id();
  const float rx = dx / (float)g.N, ry = dy / (float)g.N;
  for (int t = lane; t < g.ntab; t += kWave) {
    const float a = atab[t];
    const float2 wx = cis_neg_rev((float)(t - g.h) * rx);
    const float2 wy = cis_neg_rev((float)(t - g.h) * ry);
    X[t] = make_float2(a * wx.x, a * wx.y);
    Y[t] = make_float2(a * wy.x, a * wy.y);
  }
  wave_lds_sync();
}

// 10^x for arguments bounded by the prior support (|x| < 30): 2^(x log2 10)
// with the rounding errors of the product and of the constant carried by a
// first-order correction (relative error a few 1e-7).
__device__ __forceinline__ float exp10_bounded(float x) {
  const float c = 3.32192802429199219f;           // log2(10) rounded to float
  const float c_lo = 7.05953713e-8f;              // log2(10) - c
  const float y = x * c;
  const float e = fmaf(x, c, -y) + x * c_lo;
  return __builtin_amdgcn_exp2f(y) * fmaf(e, 0.693147180559945309f, 1.0f);
}

struct Prior {
  float lf_lo, lf_hi, ls_lo, ls_hi, sd, se;
  float isd2, ise2;     // 1 / sd^2, 1 / se^2
};

__device__ __forceinline__ bool in_support(const float* th, const Prior& pr) {
  const float E = th[2] * th[2] + th[3] * th[3];
  return th[0] > pr.lf_lo && th[0] < pr.lf_hi && th[1] > pr.ls_lo && th[1] < pr.ls_hi && E < 1.0f;
}

// Potential U = -(log L + log P0) and its gradient in sampling coordinates.
// Outside the support U = +inf and the gradient is evaluated at the nearest
// admissible position (bounds clamped, |e|^2 <= 1 - 1e-6) so that a
// trajectory can continue (it is rejected anyway).
__device__ __forceinline__ void add_result(KResult& r, const KResult& q) {
  r.loglik += q.loglik;
  r.dF += q.dF;
  r.ds += q.ds;
  r.de1 += q.de1;
  r.de2 += q.de2;
  r.ddx += q.ddx;
  r.ddy += q.ddy;
}

template <int PROF, int P, bool CHI2 = true, int NFIX = 0, int W = 1, int H = 1, bool MX = false>
__device__ __forceinline__ double potential(const GalCtx& c, const LaneCols<P * H>& lc, const Prior& pr,
                                            const float* th, float* gU, uint32_t& status,
                                            float* xbuf = nullptr) {
  const bool inside = in_support(th, pr);
  float t0 = fminf(fmaxf(th[0], pr.lf_lo), pr.lf_hi);
  float t1 = fminf(fmaxf(th[1], pr.ls_lo), pr.ls_hi);
  float e1 = th[2], e2 = th[3];
  float E = e1 * e1 + e2 * e2;
  if (E > kEClamp) {
    const float f = sqrtf(kEClamp / E);
    e1 *= f;
    e2 *= f;
    E = e1 * e1 + e2 * e2;
  }
  // F = 10^t0 and s = 10^t1 in one lane-parallel evaluation
  const float e10 = exp10_bounded(chain_lane<H>() == 0 ? t0 : t1);
  const float F = hbcast<H>(e10, 0), s = hbcast<H>(e10, 1);
  const float dx = c.refx + th[4], dy = c.refy + th[5];
  const Shape sh = make_shape<PROF>(s * c.rscale, e1, e2, c.nu);
  KResult r;
  if constexpr (MX) {
    // log L and its gradient summed over the exposures (Appendix C)
    r = KResult{0.0, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    const float n2 = (float)c.g.N * (float)c.g.N;
    for (int j = 0; j < c.E; ++j) {
      fill_tables<H>(c.g, c.sp, c.atab + j * c.astride, c.X, c.Ym, c.Yf, F, dx, dy);
      const KSums S = kspace_sums<PROF, P, false, CHI2, NFIX, W, H, true>(
          c.g, c.sp, lc, c.dh + j * c.dstride, c.X, c.Ym, c.Yf, sh, c.red, c.part, xbuf,
          c.sqw + j * c.wstride);
      const float sj = c.sig[j];
      add_result(r, kspace_finish<PROF>(S, sh, F, s, e1, e2, 1.0f / (n2 * sj * sj)));
    }
  } else {
    fill_tables<H>(c.g, c.sp, c.atab, c.X, c.Ym, c.Yf, F, dx, dy);
    KSums S;
    if constexpr (H == 4) {
      // four chains per wave: the lane's 4 P columns are read from the column
      // table block by block at each evaluation rather than held in registers
      // for the whole trajectory
      constexpr int CB = (P * H) < 6 ? P * H : 6;
      S = kspace_sums_blocked<PROF, P, CHI2, NFIX, CB>(c.cols, c.dh, c.X, c.Ym, sh, c.red);
    } else {
      S = kspace_sums<PROF, P, false, CHI2, NFIX, W, H>(c.g, c.sp, lc, c.dh, c.X, c.Ym, c.Yf, sh,
                                                        c.red, c.part, xbuf);
    }
    r = kspace_finish<PROF>(S, sh, F, s, e1, e2, c.norm);
  }
  const float isd2 = pr.isd2, ise2 = pr.ise2;
  const float cpri = -4.0f * sh.inv1mE - ise2;
  gU[0] = -r.dF * F * kLn10F;
  gU[1] = -r.ds * s * kLn10F;
  gU[2] = -(r.de1 + cpri * e1);
  gU[3] = -(r.de2 + cpri * e2);
  gU[4] = -(r.ddx - th[4] * isd2);
  gU[5] = -(r.ddy - th[5] * isd2);
  double U = 0.0;        // only the gradient is needed inside a trajectory
  if (CHI2) {
    const double lp = -0.5 * ((double)th[4] * th[4] + (double)th[5] * th[5]) * (double)pr.isd2 +
                      (double)(2.0f * __logf(1.0f - E)) - 0.5 * (double)E * (double)pr.ise2;
    U = -(r.loglik + lp);
    if (!isfinite(U)) status |= 2u;
  }
  if (!inside) {
    status |= 1u;
    U = INFINITY;
  }
  return U;
}

// Diagonal Fisher information of the likelihood plus the prior curvature, at
// theta, in sampling coordinates; returns the inverse as the metric.
template <int PROF, bool MX = false>
__device__ void fisher_inv_mass(const GalCtx& c, const Prior& pr, const float* th, float* im) {
  const Geom& g = c.g;
  const int lane = lane_id();
  float t0 = fminf(fmaxf(th[0], pr.lf_lo), pr.lf_hi);
  float t1 = fminf(fmaxf(th[1], pr.ls_lo), pr.ls_hi);
  float e1 = th[2], e2 = th[3];
  float E = e1 * e1 + e2 * e2;
  if (E > kEClamp) {
    const float f = sqrtf(kEClamp / E);
    e1 *= f;
    e2 *= f;
    E = e1 * e1 + e2 * e2;
  }
  const float F = exp10f(t0), s = exp10f(t1);
  float2* Y = c.Yf;   // full x and y tables (ntab entries each)
  const Shape sh = make_shape<PROF>(s * c.rscale, e1, e2, c.nu);
  const float cg = sh.cg;
  float fi[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
  const int n_exp = MX ? c.E : 1;
  for (int x = 0; x < n_exp; ++x) {
  fill_xy_full(g, MX ? c.atab + x * c.astride : c.atab, c.X, Y, c.refx + th[4], c.refy + th[5]);
  // noise weights 1 / lambda of the exposure's DFT modes (correlated noise), else 1
  const float* nps = (MX && c.nps) ? c.nps + c.off[c.s0 + x] : nullptr;
  // accumulate sum_c |dM/dp|^2 over every bin, frequency points combined per bin
  float acc[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
  const bool even = (g.N & 1) == 0;
  for (int b = lane; b < g.nbins; b += kWave) {
    int ub, vb, cmul;
    if (b < g.nmain) {
      main_bin_uv(g, b, ub, vb);
      cmul = 2;
    } else {
      spec_bin_uv(g.N, b - g.nmain, ub, vb, cmul);
    }
    const float wgt = nps ? 1.0f / nps[((vb + g.N) % g.N) * g.N + (ub + g.N) % g.N] : 1.0f;
    const int nu = (even && ub == -g.h) ? 2 : 1;
    const int nv = (even && vb == -g.h) ? 2 : 1;
    float dr[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f}, di[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    for (int au = 0; au < nu; ++au) {
      const int u = (nu == 2) ? (au == 0 ? -g.h : g.h) : ub;
      const float cu = (nu == 2) ? (au == 0 ? 0.5f : -0.5f) : 1.0f;
      for (int av = 0; av < nv; ++av) {
        const int v = (nv == 2) ? (av == 0 ? -g.h : g.h) : vb;
        const float cv = (nv == 2) ? (av == 0 ? 0.5f : -0.5f) : 1.0f;
        const float kx = u * g.kstep, ky = v * g.kstep;
        const float2 xu = c.X[u + g.h], yv = Y[v + g.h];
        const float kx2 = kx * kx, ky2 = ky * ky, kxy = kx * ky;
        const float q = fmaf(sh.ca, kx2, fmaf(sh.cb, ky2, sh.cc * kxy));
        float G, ia;
        profile_factor<PROF>(sh, q, G, ia);
        const float amp = F * G * cu * cv;
        const float Tr = amp * fmaf(xu.x, yv.x, -xu.y * yv.y);
        const float Ti = amp * fmaf(xu.x, yv.y, xu.y * yv.x);
        const float dq1 = sh.inv1mE * ((2.f * e1 + 2.f) * kx2 + (2.f * e1 - 2.f) * ky2 + 2.f * e1 * q);
        const float dq2 = sh.inv1mE * (2.f * e2 * (kx2 + ky2) + 4.f * kxy + 2.f * e2 * q);
        const float f[4] = {1.0f / F, 2.0f * cg / s * q * ia, cg * dq1 * ia, cg * dq2 * ia};
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          dr[j] += f[j] * Tr;
          di[j] += f[j] * Ti;
        }
        // -i k T
        dr[4] += kx * Ti; di[4] -= kx * Tr;
        dr[5] += ky * Ti; di[5] -= ky * Tr;
      }
    }
#pragma unroll
    for (int j = 0; j < 6; ++j) acc[j] += (float)cmul * wgt * (dr[j] * dr[j] + di[j] * di[j]);
  }
  const float nx = MX ? 1.0f / ((float)g.N * (float)g.N * c.sig[x] * c.sig[x]) : c.norm;
#pragma unroll
  for (int j = 0; j < 6; ++j) fi[j] += wave_total(acc[j]) * nx;
  }
  fi[0] *= F * F * kLn10F * kLn10F;
  fi[1] *= s * s * kLn10F * kLn10F;
  const float ise2 = 1.0f / (pr.se * pr.se), omE = 1.0f - E;
  fi[2] += 4.0f / omE + 8.0f * e1 * e1 / (omE * omE) + ise2;
  fi[3] += 4.0f / omE + 8.0f * e2 * e2 / (omE * omE) + ise2;
  fi[4] += 1.0f / (pr.sd * pr.sd);
  fi[5] += 1.0f / (pr.sd * pr.sd);
#pragma unroll
  for (int j = 0; j < 6; ++j) im[j] = 1.0f / fi[j];
}

// LDS strides of one exposure (MX kernels): spectrum (float2), sqrt-weights
// and PSF-sinc table (floats), each a multiple of 16 bytes.
__host__ __device__ inline int dh_stride(const SlotPlan& sp) { return (sp.nbins + 1) & ~1; }
__host__ __device__ inline int sw_stride(const SlotPlan& sp) { return (dh_stride(sp) + 3) & ~3; }
__host__ __device__ inline int atab_stride(const Geom& g) { return (g.ntab + 3) & ~3; }

// Stage one galaxy's data spectrum and PSF-sinc table in LDS; MX: those of
// each of its E exposures (stamps gal E + j), and the sqrt-weights.
template <bool MX = false>
__device__ void stage_galaxy(const HmcArgs& a, int gal, const Geom& g, const SlotPlan& sp,
                             float2* dh, float* sqw, float* atab) {
  const int E = MX ? a.n_exp : 1;
  for (int x = 0; x < E; ++x) {
    const int64_t st = MX ? (int64_t)gal * E + x : gal;
    const int64_t bo = a.bin_off[st];
    float2* dx = dh + x * dh_stride(sp);
    const float4* src = reinterpret_cast<const float4*>(a.dh + bo);
    float4* d4 = reinterpret_cast<float4*>(dx);
    for (int b = threadIdx.x; b < sp.nbins / 2; b += blockDim.x) d4[b] = src[b];
    if ((sp.nbins & 1) && threadIdx.x == 0) dx[sp.nbins - 1] = a.dh[bo + sp.nbins - 1];
    if constexpr (MX) {
      float* wx = sqw + x * sw_stride(sp);
      for (int b = threadIdx.x; b < sp.nbins; b += blockDim.x) wx[b] = a.sqw[bo + b];
    }
    float* ax = atab + x * atab_stride(g);
    const float spsf = a.psf[st] * 0.42466090014400953f * a.pscale_inv;
    for (int t = threadIdx.x; t < g.ntab; t += blockDim.x) {
      const int u = t - g.h;
      const double k = 2.0 * 3.14159265358979323846 * u / g.N;
      const double sn = (u == 0) ? 1.0 : sinpi((double)u / g.N) / (3.14159265358979323846 * u / g.N);
      ax[t] = (float)(exp(-0.5 * (double)spsf * spsf * k * k) * sn);
    }
  }
}

struct NutsTree;

struct Lds {
  float2* dh;
  NutsTree* nuts;     // per-wave NUTS scratch (NUTS launches)
  float* sqw;         // sqrt-weights (MX kernels)
  float* atab;
  float4* cols;       // per-slot column table (shared)
  ChainState* cs;     // this wave's chain record
  float* red;         // this wave's reduction scratch (64 x 8 floats)
  float2* X;
  float4* Ym;
  float2* Yf;
  float* xch0;        // exchange areas of split chains (2 x W x 12 floats per chain)
};

// Per-wave tables, in float2 units: Ym (ymax float4, first so that it is
// 16-byte aligned), X (ntab + 1, padded to ntab + 2), Yf (ntab); the length
// is even.
__host__ __device__ inline int wave_table_len(const Geom& g, const SlotPlan& sp) {
  return 2 * sp.ymax + 2 * g.ntab + 2;
}

// Four chains per wave (odd N only): Ym and X (padded to an even length),
// no Nyquist table.
__host__ __device__ inline int quad_table_len(const Geom& g, const SlotPlan& sp) {
  return (2 * sp.ymax + g.ntab + 3) & ~1;
}

// LDS: [data spectrum | sqrt-weights | atab | column table | NW chain
// records | NWV reduction scratches | NW table sets | exchange areas] for NW
// chain records (one per wave, or per chain with two chains per wave) and NWV
// waves per block; E exposures of the first three (sqrt-weights only for MX).
// idx: this lane's chain record and table set (its wave, or its chain with
// two chains per wave); wave: its reduction scratch.
//
// Four chains per wave (quad; odd N, one wave per workgroup, one exposure):
// [data spectrum | atab | column table | C chain records | C table sets
// without the Nyquist table], the wave's reduction scratch laid over the
// table sets (a chain's reduction runs after its pair loop, when the tables
// of the evaluation are no longer read), no exchange areas: about 20 KiB per
// wave at N = 53, so that 8 waves fit a CU's LDS.
__device__ __forceinline__ Lds carve(const Geom& g, const SlotPlan& sp, int idx, int wave, int C,
                                     int NWV, int E = 1, bool mx = false, bool quad = false) {
  extern __shared__ float4 smem4[];
  Lds l;
  l.dh = reinterpret_cast<float2*>(smem4);
  l.sqw = reinterpret_cast<float*>(l.dh + E * dh_stride(sp));
  l.atab = l.sqw + (mx ? E * sw_stride(sp) : 0);
  l.cols = reinterpret_cast<float4*>(l.atab + E * atab_stride(g));
  ChainState* cs0 = reinterpret_cast<ChainState*>(l.cols + sp.P * 64);
  l.cs = cs0 + idx;
  if (quad) {
    float2* wt = reinterpret_cast<float2*>(cs0 + C);
    float2* w0 = wt + quad_table_len(g, sp) * idx;
    l.Ym = reinterpret_cast<float4*>(w0);
    l.X = w0 + 2 * sp.ymax;
    l.Yf = nullptr;
    l.red = reinterpret_cast<float*>(wt);
    l.xch0 = l.red;    // unused (one wave per chain group, no split evaluation)
    l.nuts = nullptr;
    return l;
  }
  float* red0 = reinterpret_cast<float*>(cs0 + C);
  l.red = red0 + 512 * wave;
  float2* wt = reinterpret_cast<float2*>(red0 + 512 * NWV);
  float2* w0 = wt + wave_table_len(g, sp) * idx;
  l.Ym = reinterpret_cast<float4*>(w0);
  l.X = w0 + 2 * sp.ymax;
  l.Yf = l.X + g.ntab + 2;
  l.xch0 = reinterpret_cast<float*>(wt + wave_table_len(g, sp) * C);
  l.nuts = reinterpret_cast<NutsTree*>(l.xch0 + 2 * 12 * C);
  return l;
}

// Lane-uniform copy of a chain's state (word w of the 64-word record on lane w).
struct Regs {
  float theta[6], grad[6], th[6], p[6], g[6], im[6];
  double U, H0, hbar, lbar, Uth;
  float eps, eps_t, sum_alpha, u_acc;
  int l, ok, t, n_acc, n_div;
  uint32_t status, uid;
};

__device__ __forceinline__ Regs load_state(const ChainState* st) {
  const uint32_t w = reinterpret_cast<const uint32_t*>(st)[lane_id()];
  Regs r;
  auto f = [&](int i) { return __uint_as_float(bcast(w, i)); };
  auto d = [&](int i) {
    const uint64_t lo = bcast(w, i), hi = bcast(w, i + 1);
    return __longlong_as_double((long long)((hi << 32) | lo));
  };
#pragma unroll
  for (int j = 0; j < 6; ++j) {
    r.theta[j] = f(j);
    r.grad[j] = f(6 + j);
    r.th[j] = f(12 + j);
    r.p[j] = f(18 + j);
    r.g[j] = f(24 + j);
    r.im[j] = f(30 + j);
  }
  r.U = d(36);
  r.H0 = d(38);
  r.hbar = d(40);
  r.lbar = d(42);
  r.Uth = d(44);
  r.eps = f(46);
  r.eps_t = f(47);
  r.l = (int)bcast(w, 48);
  r.ok = (int)bcast(w, 49);
  r.t = (int)bcast(w, 50);
  r.n_acc = (int)bcast(w, 51);
  r.n_div = (int)bcast(w, 52);
  r.status = bcast(w, 53);
  r.sum_alpha = f(54);
  r.u_acc = f(55);
  r.uid = bcast(w, 56);
  return r;
}

__device__ __forceinline__ void store_state(ChainState* st, const Regs& r) {
  const int lane = lane_id();
  uint32_t w = 0;
  auto put_f = [&](int i, float x) { if (lane == i) w = __float_as_uint(x); };
  auto put_u = [&](int i, uint32_t x) { if (lane == i) w = x; };
  auto put_d = [&](int i, double x) {
    const uint64_t b = (uint64_t)__double_as_longlong(x);
    if (lane == i) w = (uint32_t)(b & 0xffffffffu);
    if (lane == i + 1) w = (uint32_t)(b >> 32);
  };
#pragma unroll
  for (int j = 0; j < 6; ++j) {
    put_f(j, r.theta[j]);
    put_f(6 + j, r.grad[j]);
    put_f(12 + j, r.th[j]);
    put_f(18 + j, r.p[j]);
    put_f(24 + j, r.g[j]);
    put_f(30 + j, r.im[j]);
  }
  put_d(36, r.U);
  put_d(38, r.H0);
  put_d(40, r.hbar);
  put_d(42, r.lbar);
  put_d(44, r.Uth);
  put_f(46, r.eps);
  put_f(47, r.eps_t);
  put_u(48, (uint32_t)r.l);
  put_u(49, (uint32_t)r.ok);
  put_u(50, (uint32_t)r.t);
  put_u(51, (uint32_t)r.n_acc);
  put_u(52, (uint32_t)r.n_div);
  put_u(53, r.status);
  put_f(54, r.sum_alpha);
  put_f(55, r.u_acc);
  put_u(56, r.uid);
  reinterpret_cast<uint32_t*>(st)[lane] = w;
}

// Random numbers of iteration t: 6 normals (Box-Muller on lanes 0 and 1,
// float hardware log/sqrt/sin/cos: relative error ~1e-7), the Metropolis
// uniform and the step-jitter uniform.
template <int H = 1>
__device__ __forceinline__ void draw_iteration(uint32_t uid, uint32_t t, uint32_t k0, uint32_t k1,
                                               float* z, float& u_acc, float& u_jit) {
  const int lane = chain_lane<H>();
  uint32_t tag = kTagMomentum, blk = 0;
  if (lane == 1) blk = 1;
  if (lane == 2) tag = kTagAccept;
  if (lane == 3) tag = kTagJitter;
  const uint4 w = philox4x32_10(make_uint4(uid, t, tag, blk), k0, k1);
  // two Box-Muller pairs per lane from (w.x, w.y) and (w.z, w.w)
  const float r1 = sqrtf(-2.0f * kLn2F * __builtin_amdgcn_logf(u01(w.x)));
  const float r2 = sqrtf(-2.0f * kLn2F * __builtin_amdgcn_logf(u01(w.z)));
  const float a1 = u01(w.y), a2 = u01(w.w);       // angles in revolutions
  const float za = r1 * __builtin_amdgcn_cosf(a1), zb = r1 * __builtin_amdgcn_sinf(a1);
  const float zc = r2 * __builtin_amdgcn_cosf(a2), zd = r2 * __builtin_amdgcn_sinf(a2);
  z[0] = hbcast<H>(za, 0);
  z[1] = hbcast<H>(zb, 0);
  z[2] = hbcast<H>(zc, 0);
  z[3] = hbcast<H>(zd, 0);
  z[4] = hbcast<H>(za, 1);
  z[5] = hbcast<H>(zb, 1);
  u_acc = u01(hbcast<H>(w.x, 2));
  u_jit = u01(hbcast<H>(w.x, 3));
}

// Values the leapfrog touches every step stay in registers; the rest of the
// chain state lives in the wave's LDS record and is read and written (by
// lane 0) only at trajectory boundaries.
struct Hot {
  float th[6], p[6], g[6];
  float eim[6];        // eps_t * inverse mass: the drift coefficients of this trajectory
  double Uth;
  float eps_t;
  int l, ok, t;
  uint32_t status;
};

__device__ __forceinline__ void lane0_sync() { wave_lds_sync(); }

// H = 2 or 4: several chains per wave, each group of 64 / H lanes running its
// own chain (its own record cs, tables and outputs); lane below is the lane
// within the group.
template <int PROF, int P, int NFIX, int W, int H = 1, bool MX = false>
__device__ void advance_chain(const HmcArgs& a, const GalCtx& c, const LaneCols<P * H>& lc,
                              const Prior& pr, ChainState* cs, float* samples_chain,
                              float* trace_chain) {
  const int lane = chain_lane<H>();
  const uint32_t uid = cs->uid;
  int nev = 0;           // evaluations so far (alternates the exchange buffers)
  Hot h;
#pragma unroll
  for (int j = 0; j < 6; ++j) {
    h.th[j] = cs->th[j];
    h.p[j] = cs->p[j];
    h.g[j] = cs->g[j];
  }
  h.Uth = cs->Uth;
  h.eps_t = cs->eps_t;
#pragma unroll
  for (int j = 0; j < 6; ++j) h.eim[j] = h.eps_t * cs->inv_mass[j];
  h.l = cs->l;
  h.ok = cs->ok;
  h.t = cs->t;
  h.status = cs->status;
  for (int step = 0; step < a.n_steps; ++step) {
    if (h.t >= c.t_stop) break;
    if (h.l == 0) {
      float z[6], u_acc, u_jit;
      draw_iteration<H>(uid, (uint32_t)h.t, a.k0, a.k1, z, u_acc, u_jit);
      const float eps = cs->eps;
      h.eps_t = eps;
      if (a.jitter > 0.0f)
        h.eps_t = (float)((double)eps * (1.0 + (double)a.jitter * (2.0 * (double)u_jit - 1.0)));
      double ke = 0.0;
#pragma unroll
      for (int j = 0; j < 6; ++j) {
        const float im = cs->inv_mass[j];
        h.p[j] = z[j] * __builtin_amdgcn_rsqf(im);
        ke += (double)(im * h.p[j] * h.p[j]);
        h.th[j] = cs->theta[j];
        h.g[j] = cs->grad[j];
        h.eim[j] = h.eps_t * im;
      }
      const double H0 = cs->U + 0.5 * ke;
      lane0_sync();
      if (lane == 0) {
        cs->H0 = H0;
        cs->u_acc = u_acc;
      }
      lane0_sync();
      h.ok = 1;
#pragma unroll
      for (int j = 0; j < 6; ++j) h.p[j] -= 0.5f * h.eps_t * h.g[j];
    }
#pragma unroll
    for (int j = 0; j < 6; ++j) h.th[j] += h.eim[j] * h.p[j];
    uint32_t st = 0;
    // the potential itself is needed only at the end of the trajectory
    float* xbuf = W > 1 ? c.xch + (nev & 1) * (12 * W) : nullptr;
    ++nev;
    if (h.l + 1 == a.L)
      h.Uth = potential<PROF, P, true, NFIX, W, H, MX>(c, lc, pr, h.th, h.g, st, xbuf);
    else
      h.Uth = potential<PROF, P, false, NFIX, W, H, MX>(c, lc, pr, h.th, h.g, st, xbuf);
    if (h.t >= a.W) h.status |= st;     // warmup probes are not reported
    if (!in_support(h.th, pr)) h.ok = 0;
    h.l += 1;
    if (h.l < a.L) {
#pragma unroll
      for (int j = 0; j < 6; ++j) h.p[j] -= h.eps_t * h.g[j];
      continue;
    }
    // end of trajectory: Metropolis test, adaptation, output
#pragma unroll
    for (int j = 0; j < 6; ++j) h.p[j] -= 0.5f * h.eps_t * h.g[j];
    double ke = 0.0;
#pragma unroll
    for (int j = 0; j < 6; ++j) ke += (double)(cs->inv_mass[j] * h.p[j] * h.p[j]);
    const double dH = h.Uth + 0.5 * ke - cs->H0;
    const bool finite = isfinite(dH);
    const bool accept = h.ok && finite && log((double)cs->u_acc) < -dH;
    const double alpha = (h.ok && finite) ? fmin(1.0, exp(-dH)) : 0.0;
    if ((!finite || fabs(dH) > kDivergence) && h.t >= a.W) h.status |= finite ? 4u : 2u;
    const float eps_used = cs->eps;
    if (trace_chain && lane < 4) {
      const float v = lane == 0 ? eps_used : lane == 1 ? (float)dH : lane == 2 ? (float)alpha
                                                                    : (accept ? 1.0f : 0.0f);
      trace_chain[(int64_t)h.t * 4 + lane] = v;
    }
    lane0_sync();
    if (lane == 0) {
      if ((!finite || fabs(dH) > kDivergence) && h.t >= a.W) cs->n_div += 1;
      if (accept) {
#pragma unroll
        for (int j = 0; j < 6; ++j) {
          cs->theta[j] = h.th[j];
          cs->grad[j] = h.g[j];
        }
        cs->U = h.Uth;
      }
      if (h.t < a.W) {
        if (a.adapt) {
          const double m = (double)(h.t + 1);
          const double eta = 1.0 / (m + kDaT0);
          const double hbar = (1.0 - eta) * cs->hbar + eta * ((double)a.delta - alpha);
          const double le = (double)a.mu - sqrt(m) / kDaGamma * hbar;
          const double x = (double)exp2f(-(float)kDaKappa * log2f((float)m));   // m^-kappa
          const double lbar = x * le + (1.0 - x) * cs->log_eps_bar;
          cs->hbar = hbar;
          cs->log_eps_bar = lbar;
          cs->eps = (h.t == a.W - 1) ? (float)exp(lbar) : (float)exp(le);
        }
      } else {
        cs->n_acc += accept ? 1 : 0;
        cs->sum_alpha += (float)alpha;
      }
    }
    lane0_sync();
    if (h.t >= a.W && samples_chain && lane < 6) {
      float v = cs->theta[0];
#pragma unroll
      for (int j = 1; j < 6; ++j) v = (lane == j) ? cs->theta[j] : v;
      samples_chain[(int64_t)(h.t - a.W) * 6 + lane] = v;
    }
    h.t += 1;
    h.l = 0;
  }
  lane0_sync();
  if (lane == 0) {
#pragma unroll
    for (int j = 0; j < 6; ++j) {
      cs->th[j] = h.th[j];
      cs->p[j] = h.p[j];
      cs->g[j] = h.g[j];
    }
    cs->Uth = h.Uth;
    cs->eps_t = h.eps_t;
    cs->l = h.l;
    cs->ok = h.ok;
    cs->t = h.t;
    cs->status = h.status;
  }
  lane0_sync();
}

// ---- No-U-Turn transitions (Section 3.3's sampler) -------------------------
//
// One transition per call, run by the chain's wave to the end: draw p0, then
// double the trajectory up to max_depth times in Philox-chosen directions;
// within a new subtree each point replaces the subtree's candidate with
// probability w / (sum of the subtree's weights so far), w = exp(H0 - H); the
// subtree is abandoned (and the transition ends) at a divergence (H - H0 >
// 1000 or not finite) or when any complete aligned block of 2^k of its points
// (k >= 1) makes a U-turn; otherwise its candidate replaces the proposal with
// probability min(1, W_sub / W_old) and the transition ends if the whole
// trajectory makes a U-turn.  A span makes a U-turn when rho = the sum of its
// momenta has (M^-1 p_end) . rho <= 0 at either end.  The open block of each
// level k keeps its first momentum and the running momentum sum at its start
// (checkpoints), so each check costs one difference and two dot products.
// Philox NUTS stream: counter (uid, t, tag 4, d) words 0, 1 = direction and
// merge uniform of doubling d; (uid, t, 4, 64 + n / 4) word n % 4 = the
// uniform of the transition's n-th point.
constexpr uint32_t kTagNuts = 4;

struct NutsTree {                  // per-wave LDS scratch, written by lane 0
  float eth[2][6], ep[2][6], eg[2][6];   // trajectory ends: 0 backward, 1 forward
  double eU[2];
  float pth[6], pg[6];             // proposal
  double pU;
  float sth[6], sg[6];             // candidate of the subtree being built
  double sU;
  float rho[6];                    // momentum sum of the trajectory
  float ckp[kNutsMaxDepth][6];     // first momentum of the open block of level k + 1
  float ckr[kNutsMaxDepth][6];     // subtree momentum sum at that block's start
};

// log(e^a + e^b) in float for the trajectory weights (hardware exp2/log2).
__device__ __forceinline__ float log_add_expf(float a, float b) {
  if (a == -INFINITY) return b;
  if (b == -INFINITY) return a;
  const float m = fmaxf(a, b);
  return m + __logf(1.0f + __expf(-fabsf(a - b)));
}

// A 6-vector held in registers (the same in every lane of the chain) stored
// by one lane as three 8-byte writes (the LDS records' vectors are 8-aligned).
__device__ __forceinline__ void store6(float* dst, const float* v) {
  float2* d = reinterpret_cast<float2*>(dst);
  d[0] = make_float2(v[0], v[1]);
  d[1] = make_float2(v[2], v[3]);
  d[2] = make_float2(v[4], v[5]);
}

__device__ __forceinline__ bool u_turn(const float* pa, const float* pb, const float* rho,
                                       const float* im) {
  float da = 0.f, db = 0.f;
#pragma unroll
  for (int j = 0; j < 6; ++j) {
    da = fmaf(im[j] * pa[j], rho[j], da);
    db = fmaf(im[j] * pb[j], rho[j], db);
  }
  return da <= 0.f || db <= 0.f;
}

// Advance the chain by up to a.n_steps NUTS transitions (iterations).
template <int PROF, int P, int NFIX, bool MX>
__device__ void advance_chain_nuts(const HmcArgs& a, const GalCtx& c, const LaneCols<P>& lc,
                                   const Prior& pr, ChainState* cs, NutsTree* tr,
                                   float* samples_chain, float* trace_chain) {
  const int lane = lane_id();
  const uint32_t uid = cs->uid;
  float im[6];
#pragma unroll
  for (int j = 0; j < 6; ++j) im[j] = cs->inv_mass[j];
  int t = cs->t;
  uint32_t status = cs->status;
  for (int it = 0; it < a.n_steps && t < c.t_stop; ++it, ++t) {
    const float eps = cs->eps;
    float z[6], u_acc, u_jit;
    draw_iteration<1>(uid, (uint32_t)t, a.k0, a.k1, z, u_acc, u_jit);
    float p0[6];
    double ke0 = 0.0;
#pragma unroll
    for (int j = 0; j < 6; ++j) {
      p0[j] = z[j] * __builtin_amdgcn_rsqf(im[j]);
      ke0 += (double)(im[j] * p0[j] * p0[j]);
    }
    const double H0 = cs->U + 0.5 * ke0;
    lane0_sync();
    if (lane == 0) {
      for (int e = 0; e < 2; ++e) {
#pragma unroll
        for (int j = 0; j < 6; ++j) {
          tr->eth[e][j] = cs->theta[j];
          tr->ep[e][j] = p0[j];
          tr->eg[e][j] = cs->grad[j];
        }
        tr->eU[e] = cs->U;
      }
#pragma unroll
      for (int j = 0; j < 6; ++j) {
        tr->pth[j] = cs->theta[j];
        tr->pg[j] = cs->grad[j];
        tr->rho[j] = p0[j];
      }
      tr->pU = cs->U;
    }
    lane0_sync();
    float log_w = 0.0f, sum_alpha = 0.0f;
    int n_lf = 0, n_leaf = 0, depth = 0;
    uint4 wl = make_uint4(0u, 0u, 0u, 0u);   // leaf uniforms, four per Philox block
    bool diverged = false, turned = false, moved = false;
    for (int d = 0; d < a.max_depth; ++d) {
      const uint4 wd = philox4x32_10(make_uint4(uid, (uint32_t)t, kTagNuts, (uint32_t)d), a.k0, a.k1);
      const int side = (u01(wd.x) < 0.5f) ? 0 : 1;
      const float ve = side ? eps : -eps;
      const float u_merge = u01(wd.y);
      float th[6], p[6], g[6], srho[6];
      double U = tr->eU[side];
#pragma unroll
      for (int j = 0; j < 6; ++j) {
        th[j] = tr->eth[side][j];
        p[j] = tr->ep[side][j];
        g[j] = tr->eg[side][j];
        srho[j] = 0.f;
      }
      float sub_logw = -INFINITY;
      bool sub_turn = false;
      const int n_sub = 1 << d;
      for (int jl = 0; jl < n_sub; ++jl) {
#pragma unroll
        for (int j = 0; j < 6; ++j) {
          p[j] -= 0.5f * ve * g[j];
          th[j] += ve * im[j] * p[j];
        }
        uint32_t st = 0;
        U = potential<PROF, P, true, NFIX, 1, 1, MX>(c, lc, pr, th, g, st);
        if (t >= a.W) status |= st;     // warmup probes are not reported
        double ke = 0.0;
#pragma unroll
        for (int j = 0; j < 6; ++j) {
          p[j] -= 0.5f * ve * g[j];
          ke += (double)(im[j] * p[j] * p[j]);
        }
        const double dH = U + 0.5 * ke - H0;     // float64: U and H0 are O(N^2)
        ++n_lf;
        const bool fin = isfinite(dH);
        const float lw = -(float)dH;               // the weights' arithmetic in float
        sum_alpha += fin ? fminf(1.0f, __expf(lw)) : 0.0f;
        if (!(fin && dH <= kDivergence)) {
          diverged = true;
          if (t >= a.W) status |= fin ? 4u : 2u;
          break;
        }
        const float nl = log_add_expf(sub_logw, lw);
        if ((n_leaf & 3) == 0)
          wl = philox4x32_10(make_uint4(uid, (uint32_t)t, kTagNuts, 64u + (uint32_t)(n_leaf >> 2)), a.k0,
                             a.k1);
        const uint32_t wsel = (n_leaf & 3) == 0 ? wl.x : (n_leaf & 3) == 1 ? wl.y : (n_leaf & 3) == 2 ? wl.z : wl.w;
        const bool take = __logf(u01(wsel)) < lw - nl;
        sub_logw = nl;
        ++n_leaf;
        // the subtree candidate and the checkpoints of the blocks opening at this
        // point, one component per lane (lanes 0..11)
        if (lane == 0) {
          if (take) {
            store6(tr->sth, th);
            store6(tr->sg, g);
            tr->sU = U;
          }
          for (int k = 1; k <= d; ++k) {
            if ((jl & ((1 << k) - 1)) == 0) {
              store6(tr->ckp[k - 1], p);
              store6(tr->ckr[k - 1], srho);
            }
          }
        }
        lane0_sync();
#pragma unroll
        for (int j = 0; j < 6; ++j) srho[j] += p[j];
        // every complete aligned block ending here
        for (int k = 1; k <= d && !sub_turn; ++k) {
          if (((jl + 1) & ((1 << k) - 1)) == 0) {
            float rb[6], pf[6];
#pragma unroll
            for (int j = 0; j < 6; ++j) {
              rb[j] = srho[j] - tr->ckr[k - 1][j];
              pf[j] = tr->ckp[k - 1][j];
            }
            sub_turn = u_turn(pf, p, rb, im);
          }
        }
        if (sub_turn) break;
      }
      if (diverged || sub_turn) {
        turned = sub_turn;
        break;
      }
      const bool merge = __logf(u_merge) < sub_logw - log_w;
      log_w = log_add_expf(log_w, sub_logw);
      lane0_sync();
      if (lane == 0) {
        if (merge) {
#pragma unroll
          for (int j = 0; j < 6; ++j) {
            tr->pth[j] = tr->sth[j];
            tr->pg[j] = tr->sg[j];
          }
          tr->pU = tr->sU;
        }
#pragma unroll
        for (int j = 0; j < 6; ++j) {
          tr->rho[j] += srho[j];
          tr->eth[side][j] = th[j];
          tr->ep[side][j] = p[j];
          tr->eg[side][j] = g[j];
        }
        tr->eU[side] = U;
      }
      lane0_sync();
      moved |= merge;
      depth = d + 1;
      float pl[6], pr6[6], rh[6];
#pragma unroll
      for (int j = 0; j < 6; ++j) {
        pl[j] = tr->ep[0][j];
        pr6[j] = tr->ep[1][j];
        rh[j] = tr->rho[j];
      }
      if (u_turn(pl, pr6, rh, im)) {
        turned = true;
        break;
      }
    }
    (void)turned;
    const double alpha = (double)(sum_alpha / (float)max(n_lf, 1));
    if (trace_chain && lane < 4) {
      const float v = lane == 0 ? eps : lane == 1 ? (float)n_lf : lane == 2 ? (float)alpha : (float)depth;
      trace_chain[(int64_t)t * 4 + lane] = v;
    }
    lane0_sync();
    if (lane == 0) {
      if (diverged && t >= a.W) cs->n_div += 1;
#pragma unroll
      for (int j = 0; j < 6; ++j) {
        cs->theta[j] = tr->pth[j];
        cs->grad[j] = tr->pg[j];
      }
      cs->U = tr->pU;
      if (t < a.W) {
        if (a.adapt) {
          const double m = (double)(t + 1);
          const double eta = 1.0 / (m + kDaT0);
          const double hbar = (1.0 - eta) * cs->hbar + eta * ((double)a.delta - alpha);
          const double le = (double)a.mu - sqrt(m) / kDaGamma * hbar;
          const double x = (double)exp2f(-(float)kDaKappa * log2f((float)m));   // m^-kappa
          const double lbar = x * le + (1.0 - x) * cs->log_eps_bar;
          cs->hbar = hbar;
          cs->log_eps_bar = lbar;
          cs->eps = (t == a.W - 1) ? (float)exp(lbar) : (float)exp(le);
        }
      } else {
        cs->n_acc += moved ? 1 : 0;
        cs->sum_alpha += (float)alpha;
      }
    }
    lane0_sync();
    if (t >= a.W && samples_chain && lane < 6) {
      float v = cs->theta[0];
#pragma unroll
      for (int j = 1; j < 6; ++j) v = (lane == j) ? cs->theta[j] : v;
      samples_chain[(int64_t)(t - a.W) * 6 + lane] = v;
    }
  }
  lane0_sync();
  if (lane == 0) {
    cs->t = t;
    cs->status = status;
  }
  lane0_sync();
}

// Two chains per wave (H = 2): the same transitions, each 32-lane half running
// its own chain's tree as a step machine.  Every pass of the loop evaluates the
// potential once for both halves (the evaluation is a whole-wave function);
// before it each half starts a transition or a doubling as its own state
// requires and takes the first half of a leapfrog step, after it the half does
// its point's bookkeeping and ends its subtree or transition when due.  A half
// whose transitions are done evaluates at its last position and discards the
// result until the other half is done too.  The trees and the random streams
// are those of advance_chain_nuts, so both forms give the same chains.
template <int PROF, int P, int NFIX>
__device__ void advance_chain_nuts2(const HmcArgs& a, const GalCtx& c, const LaneCols<2 * P>& lc,
                                    const Prior& pr, ChainState* cs, NutsTree* tr,
                                    float* samples_chain, float* trace_chain) {
  constexpr int H = 2;
  const int hl = chain_lane<H>();
  const uint32_t uid = cs->uid;
  float im[6], th[6], p[6], g[6], srho[6];
#pragma unroll
  for (int j = 0; j < 6; ++j) {
    im[j] = cs->inv_mass[j];
    th[j] = cs->theta[j];
    p[j] = 0.f;
    g[j] = cs->grad[j];
    srho[j] = 0.f;
  }
  int t = cs->t;
  uint32_t status = cs->status;
  int it = 0, phase = 0, d = 0, jl = 0, side = 0, depth = 0, n_lf = 0, n_leaf = 0;
  bool active = (a.n_steps > 0 && t < c.t_stop);
  bool diverged = false, moved = false;
  double H0 = 0.0, U = 0.0;
  float eps = 0.f, ve = 0.f, u_merge = 0.f, log_w = 0.f, sub_logw = 0.f, sum_alpha = 0.f;
  uint4 wl = make_uint4(0u, 0u, 0u, 0u);
  // evaluations needed at most: every transition builds fewer than 2^max_depth points
  const int cap = a.n_steps * (1 << a.max_depth) + 2;
  for (int pass = 0; pass < cap; ++pass) {
    if (__ballot(active) == 0) break;
    if (active && phase == 0) {            // start a transition
      eps = cs->eps;
      float z[6], u_acc, u_jit;
      draw_iteration<H>(uid, (uint32_t)t, a.k0, a.k1, z, u_acc, u_jit);
      double ke0 = 0.0;
#pragma unroll
      for (int j = 0; j < 6; ++j) {
        p[j] = z[j] * __builtin_amdgcn_rsqf(im[j]);
        ke0 += (double)(im[j] * p[j] * p[j]);
      }
      H0 = cs->U + 0.5 * ke0;
      wave_lds_sync();
      if (hl == 0) {
        store6(tr->ep[0], p);
        store6(tr->ep[1], p);
        store6(tr->rho, p);
      }
      if (hl >= 6 && hl < 12) {
        const float v = cs->theta[hl - 6];
        tr->eth[0][hl - 6] = v;
        tr->eth[1][hl - 6] = v;
        tr->pth[hl - 6] = v;
      } else if (hl >= 12 && hl < 18) {
        const float v = cs->grad[hl - 12];
        tr->eg[0][hl - 12] = v;
        tr->eg[1][hl - 12] = v;
        tr->pg[hl - 12] = v;
      } else if (hl == 18) {
        tr->eU[0] = cs->U;
        tr->eU[1] = cs->U;
        tr->pU = cs->U;
      }
      wave_lds_sync();
      log_w = 0.f;
      sum_alpha = 0.f;
      n_lf = n_leaf = depth = 0;
      d = 0;
      diverged = moved = false;
      phase = 1;
    }
    if (active && phase == 1) {            // start doubling d
      const uint4 wd = philox4x32_10(make_uint4(uid, (uint32_t)t, kTagNuts, (uint32_t)d), a.k0, a.k1);
      side = (u01(wd.x) < 0.5f) ? 0 : 1;
      ve = side ? eps : -eps;
      u_merge = u01(wd.y);
      U = tr->eU[side];
#pragma unroll
      for (int j = 0; j < 6; ++j) {
        th[j] = tr->eth[side][j];
        p[j] = tr->ep[side][j];
        g[j] = tr->eg[side][j];
        srho[j] = 0.f;
      }
      sub_logw = -INFINITY;
      jl = 0;
      phase = 2;
    }
    if (active) {
#pragma unroll
      for (int j = 0; j < 6; ++j) {
        p[j] -= 0.5f * ve * g[j];
        th[j] += ve * im[j] * p[j];
      }
    }
    uint32_t st = 0;
    const double Un = potential<PROF, P, true, NFIX, 1, H>(c, lc, pr, th, g, st);
    if (!active) continue;
    U = Un;
    if (t >= a.W) status |= st;
    double ke = 0.0;
#pragma unroll
    for (int j = 0; j < 6; ++j) {
      p[j] -= 0.5f * ve * g[j];
      ke += (double)(im[j] * p[j] * p[j]);
    }
    const double dH = U + 0.5 * ke - H0;
    ++n_lf;
    const bool fin = isfinite(dH);
    const float lw = -(float)dH;
    sum_alpha += fin ? fminf(1.0f, __expf(lw)) : 0.0f;
    bool end_sub = false, end_tr = false;
    if (!(fin && dH <= kDivergence)) {
      diverged = true;
      if (t >= a.W) status |= fin ? 4u : 2u;
      end_tr = true;
    } else {
      const float nl = log_add_expf(sub_logw, lw);
      if ((n_leaf & 3) == 0)
        wl = philox4x32_10(make_uint4(uid, (uint32_t)t, kTagNuts, 64u + (uint32_t)(n_leaf >> 2)), a.k0,
                           a.k1);
      const uint32_t wsel = (n_leaf & 3) == 0 ? wl.x : (n_leaf & 3) == 1 ? wl.y : (n_leaf & 3) == 2 ? wl.z : wl.w;
      const bool take = __logf(u01(wsel)) < lw - nl;
      sub_logw = nl;
      ++n_leaf;
      if (hl == 0) {
        if (take) {
          store6(tr->sth, th);
          store6(tr->sg, g);
          tr->sU = U;
        }
        for (int k = 1; k <= d; ++k) {
          if ((jl & ((1 << k) - 1)) == 0) {
            store6(tr->ckp[k - 1], p);
            store6(tr->ckr[k - 1], srho);
          }
        }
      }
      wave_lds_sync();
#pragma unroll
      for (int j = 0; j < 6; ++j) srho[j] += p[j];
      bool sub_turn = false;
      for (int k = 1; k <= d && !sub_turn; ++k) {
        if (((jl + 1) & ((1 << k) - 1)) == 0) {
          float rb[6], pf[6];
#pragma unroll
          for (int j = 0; j < 6; ++j) {
            rb[j] = srho[j] - tr->ckr[k - 1][j];
            pf[j] = tr->ckp[k - 1][j];
          }
          sub_turn = u_turn(pf, p, rb, im);
        }
      }
      ++jl;
      if (sub_turn) end_tr = true;
      else if (jl == (1 << d)) end_sub = true;
    }
    if (end_sub) {                          // merge the finished subtree
      const bool merge = __logf(u_merge) < sub_logw - log_w;
      log_w = log_add_expf(log_w, sub_logw);
      wave_lds_sync();
      if (merge && hl < 12) (&tr->pth[0])[hl] = (&tr->sth[0])[hl];   // pth, pg and sth, sg are adjacent
      if (hl == 0) {
        float r6[6];
#pragma unroll
        for (int j = 0; j < 6; ++j) r6[j] = tr->rho[j] + srho[j];
        store6(tr->rho, r6);
        store6(tr->ep[side], p);
        store6(tr->eth[side], th);
        store6(tr->eg[side], g);
        if (merge) tr->pU = tr->sU;
        tr->eU[side] = U;
      }
      wave_lds_sync();
      moved |= merge;
      depth = d + 1;
      float pl[6], pr6[6], rh[6];
#pragma unroll
      for (int j = 0; j < 6; ++j) {
        pl[j] = tr->ep[0][j];
        pr6[j] = tr->ep[1][j];
        rh[j] = tr->rho[j];
      }
      if (u_turn(pl, pr6, rh, im) || d + 1 == a.max_depth) {
        end_tr = true;
      } else {
        d += 1;
        phase = 1;
      }
    }
    if (end_tr) {                           // the transition's outputs
      const double alpha = (double)(sum_alpha / (float)max(n_lf, 1));
      if (trace_chain && hl < 4) {
        const float v = hl == 0 ? eps : hl == 1 ? (float)n_lf : hl == 2 ? (float)alpha : (float)depth;
        trace_chain[(int64_t)t * 4 + hl] = v;
      }
      wave_lds_sync();
      if (hl == 0) {
        if (diverged && t >= a.W) cs->n_div += 1;
#pragma unroll
        for (int j = 0; j < 6; ++j) {
          cs->theta[j] = tr->pth[j];
          cs->grad[j] = tr->pg[j];
        }
        cs->U = tr->pU;
        if (t < a.W) {
          if (a.adapt) {
            const double m = (double)(t + 1);
            const double eta = 1.0 / (m + kDaT0);
            const double hbar = (1.0 - eta) * cs->hbar + eta * ((double)a.delta - alpha);
            const double le = (double)a.mu - sqrt(m) / kDaGamma * hbar;
            const double x = (double)exp2f(-(float)kDaKappa * log2f((float)m));   // m^-kappa
            const double lbar = x * le + (1.0 - x) * cs->log_eps_bar;
            cs->hbar = hbar;
            cs->log_eps_bar = lbar;
            cs->eps = (t == a.W - 1) ? (float)exp(lbar) : (float)exp(le);
          }
        } else {
          cs->n_acc += moved ? 1 : 0;
          cs->sum_alpha += (float)alpha;
        }
      }
      wave_lds_sync();
      if (t >= a.W && samples_chain && hl < 6)
        samples_chain[(int64_t)(t - a.W) * 6 + hl] = cs->theta[hl];
      t += 1;
      it += 1;
      phase = 0;
      active = (it < a.n_steps && t < c.t_stop);
    }
  }
  wave_lds_sync();
  if (hl == 0) {
    cs->t = t;
    cs->status = status;
  }
  wave_lds_sync();
}

// Minimum resident waves per SIMD requested from the register allocator for
// the trajectory kernel (occupancy against instruction-level parallelism;
// in a sweep on an earlier form of the kernel one wave per SIMD ran 1.7x
// slower than two, and three or four were slower as well).
constexpr int kHmcWavesPerEu = 2;

// NFIX > 0: a kernel specialised for stamp side NFIX (a.N == NFIX).
// W > 1: each chain is evaluated by W waves (split evaluation; advance only).
// H = 2 or 4: two chains per wave (lanes 0..31 and 32..63) or four (16 lanes
// each); advance only, C a multiple of H.
// MX: several exposures per galaxy and/or per-bin noise weights (advance
// kernels of either form with one wave per chain or two chains per wave; the
// chain start runs on the general kernels).
// NUTS: No-U-Turn transitions instead of fixed-length trajectories (advance
// only; one wave per chain, or two chains per wave on the specialised kernels
// of the paired plans without MX).
template <int PROF, bool INIT, int P, int MAXT, int NFIX, int W = 1, int H = 1, bool MX = false,
          bool NUTS = false>
__global__ void __launch_bounds__(MAXT, (MAXT > 256 ? 1 : kHmcWavesPerEu)) hmc_kernel(HmcArgs a) {
  static_assert(W == 1 || !INIT, "chain start is evaluated by one wave");
  static_assert(!NUTS || (!INIT && W == 1 && (H == 1 || NFIX > 0)), "NUTS: advance kernels, W = 1");
  static_assert(!MX || (W == 1 && (NFIX == 0 || !INIT)), "exposures and noise weights: no split evaluation");
  static_assert(H == 1 || (!INIT && W == 1 && NFIX > 0), "several chains per wave: advance kernels only");
  static_assert(H <= 2 || (!MX && !NUTS), "four chains per wave: fixed-length trajectories, one exposure");
  const int N = NFIX > 0 ? NFIX : a.N;
  const Geom g = make_geom(N);
  const SlotPlan sp = make_slot_plan_p(N, P);
  const int wave = threadIdx.x / kWave;
  // chain of the galaxy, part of the chain
  const int cw = (H == 1) ? wave / W : H * wave + (int)((threadIdx.x % kWave) / (kWave / H));
  const int part = (H == 1) ? wave % W : 0;
  const int E = MX ? a.n_exp : 1;
  const Lds l = carve(g, sp, H == 1 ? wave : cw, wave, a.C * W, a.C * W / H, E, MX, H == 4);
  build_col_table(g, sp, l.cols);
  const Prior pr{a.lf_lo, a.lf_hi, a.ls_lo, a.ls_hi, a.sigma_d, a.sigma_e,
                 1.0f / (a.sigma_d * a.sigma_d), 1.0f / (a.sigma_e * a.sigma_e)};
  for (int gi = blockIdx.x; gi < a.n_gal; gi += gridDim.x) {
    const int gal = a.gidx[gi];
    __syncthreads();
    stage_galaxy<MX>(a, gal, g, sp, l.dh, l.sqw, l.atab);
    __syncthreads();
    if (cw >= a.C) continue;
    const LaneCols<P * H> lc = lane_cols<P * H, H>(l.cols);
    const int64_t s0 = (int64_t)gal * E;     // the galaxy's first stamp
    const float sig = a.sigma[s0];
    GalCtx c;
    c.g = g;
    c.sp = sp;
    c.dh = l.dh;
    c.atab = l.atab;
    c.X = l.X;
    c.Ym = l.Ym;
    c.Yf = l.Yf;
    c.red = l.red;
    c.cols = l.cols;
    c.part = part;
    c.xch = l.xch0 + cw * (2 * 12 * W);
    c.norm = 1.0f / ((float)g.N * (float)g.N * sig * sig);
    c.rscale = a.rscale;
    c.nu = a.nu;
    c.refx = a.ref_xy[2 * (int64_t)gal];
    c.refy = a.ref_xy[2 * (int64_t)gal + 1];
    c.t_stop = a.t_stop_gal ? min(a.t_stop, a.t_stop_gal[gal]) : a.t_stop;
    if constexpr (MX) {
      c.E = E;
      c.dstride = dh_stride(sp);
      c.wstride = sw_stride(sp);
      c.astride = atab_stride(g);
      c.sqw = l.sqw;
      c.sig = a.sigma + s0;
      c.nps = a.noise_ps;
      c.off = a.off;
      c.s0 = s0;
    }
    const int64_t chain = (int64_t)gal * a.C + cw;
    ChainState* st = a.state + chain;
    if constexpr (INIT) {
      Regs r;
      const float* ini = a.init + chain * 6;
#pragma unroll
      for (int j = 0; j < 6; ++j) r.theta[j] = ini[j];
      if (a.metric == 1) {
        fisher_inv_mass<PROF, MX>(c, pr, r.theta, r.im);
      } else {
#pragma unroll
        for (int j = 0; j < 6; ++j) r.im[j] = a.inv_mass ? a.inv_mass[(int64_t)gal * 6 + j] : 1.0f;
      }
      uint32_t stt = 0;
      r.U = potential<PROF, P, true, 0, 1, 1, MX>(c, lc, pr, r.theta, r.grad, stt);
      r.status = stt;
#pragma unroll
      for (int j = 0; j < 6; ++j) {
        r.th[j] = r.theta[j];
        r.p[j] = 0.f;
        r.g[j] = r.grad[j];
      }
      r.H0 = 0.0;
      r.hbar = 0.0;
      r.lbar = 0.0;
      r.Uth = r.U;
      r.eps = a.eps0;
      r.eps_t = a.eps0;
      r.sum_alpha = 0.f;
      r.u_acc = 0.5f;
      r.l = 0;
      r.ok = 1;
      r.t = 0;
      r.n_acc = 0;
      r.n_div = 0;
      r.uid = (uint32_t)((a.uid_gal ? a.uid_gal[gal] : a.uid_base + (uint64_t)gal * a.C) +
                         (uint64_t)cw);
      store_state(st, r);
    } else {
      // the 64-word record of this lane's chain, copied by the chain's lanes
      uint32_t* csw = reinterpret_cast<uint32_t*>(l.cs);
      const uint32_t* src = reinterpret_cast<const uint32_t*>(st);
      const int cl = chain_lane<H>();
#pragma unroll
      for (int k = 0; k < H; ++k) csw[cl + (kWave / H) * k] = src[cl + (kWave / H) * k];
      wave_lds_sync();
      // the W waves of a split chain hold identical copies of its state; the
      // first writes the outputs
      float* sc = (a.samples && part == 0) ? a.samples + chain * (int64_t)a.S * 6 : nullptr;
      float* tc = (a.trace && part == 0) ? a.trace + chain * (int64_t)a.t_stop * 4 : nullptr;
      if constexpr (NUTS && H == 2)
        advance_chain_nuts2<PROF, P, NFIX>(a, c, lc, pr, l.cs, l.nuts + cw, sc, tc);
      else if constexpr (NUTS)
        advance_chain_nuts<PROF, P, NFIX, MX>(a, c, lc, pr, l.cs, l.nuts + wave, sc, tc);
      else
        advance_chain<PROF, P, NFIX, W, H, MX>(a, c, lc, pr, l.cs, sc, tc);
      if (part == 0) {
        uint32_t* dst = reinterpret_cast<uint32_t*>(st);
#pragma unroll
        for (int k = 0; k < H; ++k) dst[cl + (kWave / H) * k] = csw[cl + (kWave / H) * k];
      }
    }
  }
}

__global__ void hmc_finalize_kernel(const ChainState* __restrict__ st, int n_gal, int C, int S,
                                    float* __restrict__ stats, uint32_t* __restrict__ status) {
  const int gal = blockIdx.x * blockDim.x + threadIdx.x;
  if (gal >= n_gal) return;
  uint32_t s = 0;
  for (int c = 0; c < C; ++c) {
    const ChainState& x = st[(int64_t)gal * C + c];
    s |= x.status;
    if (stats) {
      float* o = stats + ((int64_t)gal * C + c) * 4;
      o[0] = S > 0 ? (float)x.n_acc / (float)S : 0.f;
      o[1] = x.eps;
      o[2] = (float)x.n_div;
      o[3] = (float)x.U;
    }
  }
  if (status) status[gal] = s;
}

}  // namespace

size_t hmc_lds_bytes(int N, int C, int P, int W, int H, int E, bool mx, bool nuts) {
  const Geom g = make_geom(N);
  const SlotPlan sp = make_slot_plan_p(N, P);
  const int NW = C * W;
  if (H == 4)   // the quad layout of carve
    return sizeof(float2) * dh_stride(sp) + sizeof(float) * atab_stride(g) + sizeof(float4) * sp.P * 64 +
           sizeof(ChainState) * NW +
           std::max<size_t>(sizeof(float2) * quad_table_len(g, sp) * NW, sizeof(float) * 512);
  return sizeof(float2) * E * dh_stride(sp) + sizeof(float) * (mx ? E * sw_stride(sp) : 0) +
         sizeof(float) * E * atab_stride(g) +
         sizeof(float4) * sp.P * 64 + sizeof(ChainState) * NW + sizeof(float) * 512 * (NW / H) +
         sizeof(float2) * wave_table_len(g, sp) * NW + sizeof(float) * 2 * 12 * NW +
         (nuts ? sizeof(NutsTree) * NW : 0);
}

template <int PROF, bool INIT, int P, int NFIX = 0, int W = 1, int H = 1, bool MX = false>
static void launch_p(const HmcArgs& a, int grid, size_t lds, hipStream_t s) {
  const dim3 blk(kWave * a.C * W / H);
  if constexpr (!INIT && NFIX == 0 && W == 1 && H == 1) {
    if (a.nuts) {
      if (MX || a.C <= 4) {
        auto k = hmc_kernel<PROF, false, P, 256, 0, 1, 1, MX, true>;
        (void)hipFuncSetAttribute((const void*)k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        hipLaunchKernelGGL(k, dim3(grid), blk, lds, s, a);
      } else {
        auto k = hmc_kernel<PROF, false, P, 1024, 0, 1, 1, false, true>;
        (void)hipFuncSetAttribute((const void*)k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        hipLaunchKernelGGL(k, dim3(grid), blk, lds, s, a);
      }
      return;
    }
  }
  if constexpr (MX) {
    auto k = hmc_kernel<PROF, INIT, P, 256, NFIX, 1, H, true>;   // C <= 4 (checked by the caller)
    (void)hipFuncSetAttribute((const void*)k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    hipLaunchKernelGGL(k, dim3(grid), blk, lds, s, a);
  } else if (a.C * W <= 4) {
    auto k = hmc_kernel<PROF, INIT, P, 256, NFIX, W, H>;
    (void)hipFuncSetAttribute((const void*)k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    hipLaunchKernelGGL(k, dim3(grid), blk, lds, s, a);
  } else {
    auto k = hmc_kernel<PROF, INIT, P, 1024, 0, 1>;
    (void)hipFuncSetAttribute((const void*)k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    hipLaunchKernelGGL(k, dim3(grid), blk, lds, s, a);
  }
}

// Trajectory kernels specialised for the stamp sizes of the workloads
// (compile-time geometry, fully unrolled pair loop), one per candidate plan
// (the plans within 10 % of the fewest pair-slots, at most three; for 41 also
// P = 4 beside the single best), and for the default plan also split over 2
// and 4 waves per chain; other sizes and plans use the generic kernel of
// their P.
#define BSI_FIXED_PLANS(X) \
  X(25, 3) X(32, 1) X(32, 2) X(32, 4) X(41, 1) X(41, 4) \
  X(53, 3) X(53, 4) X(53, 6) X(73, 3) X(73, 6) X(73, 8) X(101, 4) X(101, 5)

// Plans whose two-chains-per-wave kernel is faster than the one-chain kernel
// (measured per size and plan; at 73 and 101 the two-chain kernels either
// spill or run slower, and the larger P spill everywhere).
constexpr bool paired_chains_plan(int N, int P) {
  return (N == 25 && P == 3) || (N == 41 && P == 1) || (N == 53 && P == 3);
}

// Plans with a four-chains-per-wave kernel (16 lanes per chain; fixed-length
// trajectories of four chains, one exposure, odd N): the work outside the
// pair loop (tables, reductions, leapfrog update, random numbers) is per wave
// and so shared by four chains instead of two.  A wave then holds a whole
// galaxy, so each wave needs its own data spectrum in LDS (the quad layout of
// carve keeps 53 px at about 20 KiB, 8 waves per CU), and the pair loop runs
// in column blocks (kspace_sums_blocked) so that it stays in registers.
constexpr bool quad_chains_plan(int N, int P) {
  return (N == 25 && P == 3) || (N == 41 && P == 1) || (N == 53 && P == 3);
}

// Chains per wave of an advance launch, the one rule that launch_fixed_w,
// launch_fixed_nuts, launch_fixed_mx and the LDS size follow.  Several chains
// per wave only on the specialised kernels of the paired plans, one wave per
// galaxy at most (C <= 4) and no split evaluation; four for fixed-length
// trajectories of exactly four chains on the quad plans.  With noise weights
// two only for a single exposure on the default plan: with several, the
// two-chain kernels keep too much live across the exposure loop (they spill).
static int launch_chains_per_wave(const HmcArgs& a, bool init) {
  if (init || a.prof == kProfGauss || a.wpc != 1 || a.C > 4 || (a.C & 1)) return 1;
  if (!paired_chains_plan(a.N, a.P)) return 1;
  if (a.mx && (a.nuts || a.n_exp != 1 || !hmc_mx_fixed(a.N, a.P, a.prof, a.wpc))) return 1;
  if (!a.mx && !a.nuts && a.C == 4 && quad_chains_plan(a.N, a.P)) return 4;
  return 2;
}

template <int PROF, int NFIX, int PP>
static bool launch_fixed_w(const HmcArgs& a, int grid, size_t lds, hipStream_t s) {
  if (a.wpc == 1) {
    if constexpr (paired_chains_plan(NFIX, PP)) {
      const int H = launch_chains_per_wave(a, false);
      if constexpr (quad_chains_plan(NFIX, PP)) {
        if (H == 4) {
          launch_p<PROF, false, PP, NFIX, 1, 4>(a, grid, lds, s);
          return true;
        }
      }
      if (H == 2) {
        launch_p<PROF, false, PP, NFIX, 1, 2>(a, grid, lds, s);
        return true;
      }
    }
    launch_p<PROF, false, PP, NFIX, 1>(a, grid, lds, s);
    return true;
  }
  if constexpr (make_slot_plan(NFIX).P == PP) {
    if (a.wpc == 2) {
      launch_p<PROF, false, PP, NFIX, 2>(a, grid, lds, s);
      return true;
    }
    if (a.wpc == 4) {
      launch_p<PROF, false, PP, NFIX, 4>(a, grid, lds, s);
      return true;
    }
  }
  return false;
}

// Several exposures / noise weights on the specialised kernels of the
// default plan of each size.
template <int PROF>
static bool launch_fixed_mx(const HmcArgs& a, int grid, size_t lds, hipStream_t s) {
#define BSI_CASE(NN, PP)                                                         \
  if (a.N == NN && a.P == PP) {                                                  \
    if constexpr (make_slot_plan(NN).P == PP) {                                  \
      if constexpr (paired_chains_plan(NN, PP)) {                                \
        if (launch_chains_per_wave(a, false) == 2) {                             \
          launch_p<PROF, false, PP, NN, 1, 2, true>(a, grid, lds, s);            \
          return true;                                                           \
        }                                                                        \
      }                                                                          \
      launch_p<PROF, false, PP, NN, 1, 1, true>(a, grid, lds, s);                \
      return true;                                                               \
    }                                                                            \
  }
  BSI_FIXED_PLANS(BSI_CASE)
#undef BSI_CASE
  return false;
}

template <int PROF>
static bool launch_fixed(const HmcArgs& a, int grid, size_t lds, hipStream_t s) {
#define BSI_CASE(NN, PP) \
  if (a.N == NN && a.P == PP) return launch_fixed_w<PROF, NN, PP>(a, grid, lds, s);
  BSI_FIXED_PLANS(BSI_CASE)
#undef BSI_CASE
  return false;
}

int hmc_split_waves(int N, int C, int P, int prof, int max_w) {
  if (max_w <= 1 || prof == kProfGauss || P != make_slot_plan(N).P) return 1;
  bool fixed = false;
  for (const int* p = hmc_fixed_plans(N); *p; ++p) fixed |= (*p == P);
  if (!fixed) return 1;
  const int nsr = make_slot_plan_p(N, P).nsr;
  int W = 1;
  while (W * 2 <= max_w && W * 2 <= nsr && C * W * 2 <= 4) W *= 2;
  return W;
}

bool hmc_mx_fixed(int N, int P, int prof, int wpc) {
  if (wpc != 1 || prof == kProfGauss || P != make_slot_plan(N).P) return false;
  for (const int* p = hmc_fixed_plans(N); *p; ++p)
    if (*p == P) return true;
  return false;
}

const int* hmc_fixed_plans(int N) {
  static const int none[] = {0};
  switch (N) {
    case 25: { static const int p[] = {3, 0}; return p; }
    case 32: { static const int p[] = {1, 2, 4, 0}; return p; }
    case 41: { static const int p[] = {1, 4, 0}; return p; }
    case 53: { static const int p[] = {3, 4, 6, 0}; return p; }
    case 73: { static const int p[] = {3, 6, 8, 0}; return p; }
    case 101: { static const int p[] = {4, 5, 0}; return p; }
    default: return none;
  }
}

// NUTS on the kernels specialised per stamp size (one wave per chain, or two
// on the paired plans; with exposures / noise weights one wave per chain on
// the default plans).
template <int PROF>
static bool launch_fixed_nuts(const HmcArgs& a, int grid, size_t lds, hipStream_t s) {
#define BSI_CASE(NN, PP)                                                                        \
  if (a.N == NN && a.P == PP) {                                                                 \
    if (a.mx) {                                                                                 \
      if constexpr (make_slot_plan(NN).P == PP) {                                               \
        auto km = hmc_kernel<PROF, false, PP, 256, NN, 1, 1, true, true>;                       \
        (void)hipFuncSetAttribute((const void*)km, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds); \
        hipLaunchKernelGGL(km, dim3(grid), dim3(kWave * a.C), lds, s, a);                       \
        return true;                                                                            \
      }                                                                                         \
      return false;                                                                             \
    }                                                                                           \
    if constexpr (paired_chains_plan(NN, PP)) {                                                 \
      if (launch_chains_per_wave(a, false) == 2) {                                              \
        auto k2 = hmc_kernel<PROF, false, PP, 256, NN, 1, 2, false, true>;                      \
        (void)hipFuncSetAttribute((const void*)k2, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds); \
        hipLaunchKernelGGL(k2, dim3(grid), dim3(kWave * a.C / 2), lds, s, a);                   \
        return true;                                                                            \
      }                                                                                         \
    }                                                                                           \
    auto k = hmc_kernel<PROF, false, PP, 256, NN, 1, 1, false, true>;                           \
    (void)hipFuncSetAttribute((const void*)k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds); \
    hipLaunchKernelGGL(k, dim3(grid), dim3(kWave * a.C), lds, s, a);                            \
    return true;                                                                                \
  }
  BSI_FIXED_PLANS(BSI_CASE)
#undef BSI_CASE
  return false;
}

template <int PROF, bool INIT>
static void launch_prof(const HmcArgs& a, int grid, size_t lds, hipStream_t s) {
  if constexpr (!INIT && PROF != kProfGauss)
    if (a.nuts && a.C <= 4 && (!a.mx || hmc_mx_fixed(a.N, a.P, a.prof, a.wpc)) &&
        launch_fixed_nuts<PROF>(a, grid, lds, s))
      return;
  if (a.nuts && !a.mx) {
    switch (a.P) {
      case 1: launch_p<PROF, INIT, 1>(a, grid, lds, s); break;
      case 2: launch_p<PROF, INIT, 2>(a, grid, lds, s); break;
      case 3: launch_p<PROF, INIT, 3>(a, grid, lds, s); break;
      case 4: launch_p<PROF, INIT, 4>(a, grid, lds, s); break;
      case 5: launch_p<PROF, INIT, 5>(a, grid, lds, s); break;
      case 6: launch_p<PROF, INIT, 6>(a, grid, lds, s); break;
      default: launch_p<PROF, INIT, 8>(a, grid, lds, s); break;
    }
    return;
  }
  if (a.mx) {
    if constexpr (!INIT && PROF != kProfGauss)
      if (!a.nuts && hmc_mx_fixed(a.N, a.P, a.prof, a.wpc) && launch_fixed_mx<PROF>(a, grid, lds, s))
        return;
    switch (a.P) {
      case 1: launch_p<PROF, INIT, 1, 0, 1, 1, true>(a, grid, lds, s); break;
      case 2: launch_p<PROF, INIT, 2, 0, 1, 1, true>(a, grid, lds, s); break;
      case 3: launch_p<PROF, INIT, 3, 0, 1, 1, true>(a, grid, lds, s); break;
      case 4: launch_p<PROF, INIT, 4, 0, 1, 1, true>(a, grid, lds, s); break;
      case 5: launch_p<PROF, INIT, 5, 0, 1, 1, true>(a, grid, lds, s); break;
      case 6: launch_p<PROF, INIT, 6, 0, 1, 1, true>(a, grid, lds, s); break;
      default: launch_p<PROF, INIT, 8, 0, 1, 1, true>(a, grid, lds, s); break;
    }
    return;
  }
  if constexpr (!INIT && PROF != kProfGauss)
    if (a.C * a.wpc <= 4 && launch_fixed<PROF>(a, grid, lds, s)) return;
  switch (a.P) {
    case 1: launch_p<PROF, INIT, 1>(a, grid, lds, s); break;
    case 2: launch_p<PROF, INIT, 2>(a, grid, lds, s); break;
    case 3: launch_p<PROF, INIT, 3>(a, grid, lds, s); break;
    case 4: launch_p<PROF, INIT, 4>(a, grid, lds, s); break;
    case 5: launch_p<PROF, INIT, 5>(a, grid, lds, s); break;
    case 6: launch_p<PROF, INIT, 6>(a, grid, lds, s); break;
    default: launch_p<PROF, INIT, 8>(a, grid, lds, s); break;
  }
}

template <bool INIT>
static hipError_t launch_impl(const HmcArgs& a, int grid, hipStream_t s) {
  if (a.n_gal <= 0) return hipSuccess;
  if (!plan_valid(a.N, a.P)) return hipErrorInvalidValue;
  // split chains only where a specialised kernel exists (hmc_split_waves)
  if (a.wpc != 1 && (INIT || a.wpc != hmc_split_waves(a.N, a.C, a.P, a.prof, a.wpc)))
    return hipErrorInvalidValue;
  // exposures / noise weights: no split evaluation, C <= 4
  if (a.mx && (a.wpc != 1 || a.C > 4 || a.n_exp < 1 || !a.sqw)) return hipErrorInvalidValue;
  // NUTS: no split evaluation
  if (a.nuts && (a.wpc != 1 || a.max_depth < 1 || a.max_depth > kNutsMaxDepth))
    return hipErrorInvalidValue;
  // several chains per wave exactly where launch_fixed_w, launch_fixed_nuts
  // and launch_fixed_mx launch them
  const int H = launch_chains_per_wave(a, INIT);
  const size_t lds = a.mx ? hmc_lds_bytes(a.N, a.C, a.P, 1, H, a.n_exp, true, a.nuts)
                          : hmc_lds_bytes(a.N, a.C, a.P, INIT ? 1 : a.wpc, H, 1, false, a.nuts);
  if (a.prof == kProfExp)
    launch_prof<kProfExp, INIT>(a, grid, lds, s);
  else if (a.prof == kProfSpergel)
    launch_prof<kProfSpergel, INIT>(a, grid, lds, s);
  else
    launch_prof<kProfGauss, INIT>(a, grid, lds, s);
  return hipGetLastError();
}

hipError_t launch_hmc_init(const HmcArgs& a, int grid, hipStream_t s) { return launch_impl<true>(a, grid, s); }
hipError_t launch_hmc_advance(const HmcArgs& a, int grid, hipStream_t s) { return launch_impl<false>(a, grid, s); }

hipError_t launch_hmc_finalize(const ChainState* st, int n_gal, int C, int S, float* chain_stats,
                               uint32_t* status, hipStream_t s) {
  if (n_gal <= 0) return hipSuccess;
  hipLaunchKernelGGL(hmc_finalize_kernel, dim3((n_gal + 255) / 256), dim3(256), 0, s, st, n_gal, C,
                     S, chain_stats, status);
  return hipGetLastError();
}

}  // namespace bsi
