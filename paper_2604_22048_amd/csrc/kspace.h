// Exact k-space evaluation of the pixel log-likelihood and its gradient.
//
// The model stamp is a finite Fourier series on the stamp's own frequency
// grid, so its N x N DFT equals the spectrum T at the interior bins (and a
// fixed +-1/2 combination of the two Nyquist frequency points at the Nyquist
// bins of an even N).  By Parseval, with D the DFT of the data,
//   sum_p (d_p - m_p)^2 = N^-2 sum_bins |D - M|^2,
// so log L (eq. likelihood-pixels) and its gradient need no inverse
// transform per evaluation: one forward DFT of the data per galaxy, then
// O(N^2) pointwise work per evaluation.  With R = D - M,
//   log L        = -(1/2) sigma^-2 N^-2 sum |R|^2,
//   dlog L / dp  =  sigma^-2 N^-2 sum Re[conj(R) dM/dp].
// The spectrum derivatives are closed forms: dT/dF = T/F,
// dT/ds = -3 r0^2 q / (s (1 + r0^2 q)) T, dT/de = -3/2 r0^2 (dq/de) /
// (1 + r0^2 q) T (exponential profile), dT/d(dx, dy) = -i (k_x, k_y) T, so
// every gradient component is a weighted sum of Re or Im of conj(R) T.
//
// Work layout ("slot plan"): the odd core of the grid, |u|, |v| <= hc, is
// walked as rows v = 0..hc.  Row 0 is taken whole with weight 1 (it holds
// each mirror pair once and the DC bin), rows v > 0 with weight 2 (their
// mirrors, v < 0, are not stored).  R consecutive rows form a super-row of
// R * nc slots, spread over P iterations of the 64 lanes: lane l in iteration
// i owns slot s = l + 64 i, i.e. row offset s / nc and column s % nc, the
// same for every super-row.  Column quantities (k_x, the x factor of the
// spectrum) are therefore lane constants, and the data spectrum is stored in
// slot order so that each bin is one LDS read at a fixed offset.  Slots past
// R * nc and rows past hc carry zero data and a zero spectrum factor, and
// row 0 carries a 1/sqrt(2) factor in both, so the loop is branch-free and
// every sum is doubled at the end.  (R, P) is chosen per N to minimise the
// number of slots (lane utilisation 85-97 % for the stamp sizes in use).
// The Nyquist bins of an even N follow the slots as "special" bins.
#pragma once

#include "bsi_device.h"

namespace bsi {

enum { kProfExp = 0, kProfGauss = 1, kProfSpergel = 2 };

// Supported iterations per super-row (template instances of the bin loop).
constexpr int kPlanP[] = {1, 2, 3, 4, 5, 6, 8};

// Half-plane bins of the odd core (nc = N, or N - 1 for even N, columns u =
// -hc..hc, rows v = 0..hc) in pair-slots: pair-slot (j, v) holds the bins
// (+j, v) and (-j, v) for j = 1..hc, and for j = 0 the bin (0, v) split into
// two half-weight copies, so each row has npc = hc + 1 pair-slots.  A
// super-row holds R rows in P * 64 pair-slots: lane l of iteration i takes
// pair-slot l + 64 i, row offset (l + 64 i) / npc, column (l + 64 i) mod npc.
struct SlotPlan {
  int R, P, nsr;      // rows per super-row, iterations per super-row, super-rows
  int nslots;         // pair-slots: nsr * P * 64
  int ymax;           // nsr * R rows covered (>= hc + 1)
  int nspec;          // special (Nyquist) bins after the pair-slots: N + 1 for even N, else 0
  int nbins;          // stored spectrum length in complex values: 2 nslots + nspec, made even
};

__host__ __device__ constexpr int pair_cols(int N) { return (((N & 1) ? N : N - 1) - 1) / 2 + 1; }

// The slot plan of stamp side N with P iterations per super-row: R rows
// per super-row (as many as P * 64 pair-slots hold, at most all rows), nsr
// super-rows.  P must give R >= 1 (plan_valid).
__host__ __device__ constexpr SlotPlan make_slot_plan_p(int N, int P) {
  const int npc = pair_cols(N);
  const int rows = npc;
  const int R = (64 * P) / npc;
  const int Rr = R < rows ? R : rows;
  const int nsr = Rr > 0 ? (rows + Rr - 1) / Rr : 0;
  SlotPlan sp{Rr, P, nsr, nsr * P * 64, nsr * Rr, 0, 0};
  sp.nspec = (N & 1) ? 0 : N + 1;
  sp.nbins = (2 * sp.nslots + sp.nspec + 1) & ~1;
  return sp;
}

__host__ __device__ constexpr bool plan_valid(int N, int P) { return (64 * P) / pair_cols(N) >= 1; }

// Whether pair-iteration j of super-row k holds a bin for any of the LS
// lanes of a chain (lane l takes the super-row's pair-slots l, l + LS, ...):
// the last super-row can cover fewer rows, and a super-row's last pair-slots
// are padding.  A dead iteration would add exact zeros, so kernels that know
// N at compile time skip it.
__host__ __device__ constexpr bool pair_iter_live(int N, const SlotPlan& sp, int LS, int k, int j) {
  const int rows = pair_cols(N) - k * sp.R;
  return j * LS < (rows < sp.R ? rows : sp.R) * pair_cols(N);
}

// Default plan: the supported P with the fewest slots (ties: smaller P).
__host__ __device__ constexpr SlotPlan make_slot_plan(int N) {
  SlotPlan best{0, 0, 0, 1 << 30, 0, 0, 0};
  for (int k = 0; k < 7; ++k) {
    const int P = kPlanP[k];
    if (!plan_valid(N, P)) continue;
    const SlotPlan sp = make_slot_plan_p(N, P);
    if (sp.nslots < best.nslots) best = sp;
  }
  return best;
}

// Stored complex value b < 2 nslots -> its bin (u, v) and the scale of the
// stored data, or invalid (padding, stored as zero).  Value 2 s holds (+j, v)
// and 2 s + 1 holds (-j, v) of pair-slot s; the data are scaled by 1/sqrt(2)
// in row 0 (whose bins all appear with their mirrors) and in column 0 (split
// into two copies).
__host__ __device__ inline bool slot_value_uv(int N, const SlotPlan& sp, int b, int& u, int& v,
                                              float& scale) {
  const int npc = pair_cols(N);
  const int slot = b >> 1;
  const int per = sp.P * 64;
  const int sr = slot / per, s = slot - sr * per;
  if (s >= sp.R * npc) return false;
  const int ro = s / npc;
  const int j = s - ro * npc;
  v = sr * sp.R + ro;
  u = (b & 1) ? -j : j;
  scale = (v == 0 ? 0.70710678118654752f : 1.0f) * (j == 0 ? 0.70710678118654752f : 1.0f);
  return v < npc;
}

// Special (Nyquist) bin i of an even N -> DFT bin (u_b, v_b), Nyquist bins
// at frequency -N/2, and its multiplicity c in a full-grid sum.
__host__ __device__ inline void nyq_bin_uv(int N, int i, int& u, int& v, int& c) {
  const int h = N / 2;
  if (i == 0) { u = -h; v = 0; c = 1; return; }
  if (i == 1) { u = 0; v = -h; c = 1; return; }
  if (i < h + 1) { u = i - 1; v = -h; c = 2; return; }        // u = 1..h-1
  if (i == h + 1) { u = -h; v = -h; c = 1; return; }
  u = -h; v = i - (h + 1); c = 2;                               // v = 1..h-1
}

// Half of the full-grid sums (the stored half plane counts once; the factor
// 2 is applied by kspace_finish).
struct KSums {
  double chi2;                                    // half the full-grid sum of |D - M|^2
  float sF, sxx, syy, sxy, sq, sdx, sdy;          // weighted Re/Im sums (halved likewise)
};

struct KResult {
  double loglik;
  float dF, ds, de1, de2, ddx, ddy;               // d log L / d params
};

// 1/x to within an ulp: the hardware reciprocal refined by one Newton step.
__device__ __forceinline__ float rcp_nr(float x) {
  const float r = __builtin_amdgcn_rcpf(x);
  return fmaf(fmaf(-x, r, 1.0f), r, r);
}

// Per-evaluation constants of the quadratic form q = ca kx^2 + cb ky^2 + cc kx ky
// and of the profile exponent t = ta kx^2 + tb ky^2 + tc kx ky + t0 in which
// the profile factor is evaluated: G = t^(-3/2) with t = 1 + r0^2 q for the
// exponential, G = t^(-(1+nu)) with the same t for the Spergel profile of
// index nu, G = 2^t with t = -r^2 q log2(e) / 2 for the Gaussian.  cg is
// (d ln G / dq) times a = 1 + r0^2 q (times 1 for the Gaussian), gw the
// Spergel exponent -(2 + nu) of G / t.
struct Shape {
  float ca, cb, cc, r2, inv1mE;
  float ta, tb, tc, t0;
  float cg, gw;
};

template <int PROF>
__device__ __forceinline__ Shape make_shape(float rpx, float e1, float e2, float nu = 0.5f) {
  Shape s;
  const float E = e1 * e1 + e2 * e2;
  s.inv1mE = rcp_nr(1.0f - E);
  s.ca = (1.0f + E + 2.0f * e1) * s.inv1mE;
  s.cb = (1.0f + E - 2.0f * e1) * s.inv1mE;
  s.cc = 4.0f * e2 * s.inv1mE;
  s.r2 = rpx * rpx;
  const float f = (PROF != kProfGauss) ? s.r2 : -0.72134752044448170368f * s.r2;   // -log2(e) / 2
  s.ta = f * s.ca;
  s.tb = f * s.cb;
  s.tc = f * s.cc;
  s.t0 = (PROF != kProfGauss) ? 1.0f : 0.0f;
  s.cg = (PROF == kProfExp) ? -1.5f * s.r2 : (PROF == kProfGauss) ? -0.5f * s.r2 : -(1.0f + nu) * s.r2;
  s.gw = -(2.0f + nu);
  return s;
}

// The flux sum sum G z' from the shape sums: w0 = sum G a^-1 z' and
// sq = sum G a^-1 z' q, with a = 1 + r0^2 q for the exponential and Spergel
// profiles and G a^-1 = G for the Gaussian.
template <int PROF>
__device__ __forceinline__ float flux_sum(float w0, float sq, const Shape& sh) {
  return PROF == kProfGauss ? w0 : fmaf(sh.r2, sq, w0);
}

// Spergel factors from a = 1 + r0^2 q >= 1: G / a = a^gw = 2^(gw log2 a)
// and G = a (G / a).
__device__ __forceinline__ void spergel_factor(float gw, float a, float& G, float& Gw) {
  Gw = __builtin_amdgcn_exp2f(gw * __builtin_amdgcn_logf(a));
  G = Gw * a;
}

// Profile factor G(q) and the factor ia multiplying z in the shape sums
// (1/(1 + r0^2 q) for the exponential and Spergel profiles, 1 for the Gaussian).
template <int PROF>
__device__ __forceinline__ void profile_factor(const Shape& sh, float q, float& G, float& ia) {
  if (PROF == kProfExp) {
    const float a = fmaf(sh.r2, q, 1.0f);
    const float rs = __builtin_amdgcn_rsqf(a);
    ia = rs * rs;
    G = ia * rs;
  } else if (PROF == kProfSpergel) {
    const float a = fmaf(sh.r2, q, 1.0f);
    float Gw;
    spergel_factor(sh.gw, a, G, Gw);
    ia = rcp_nr(a);
  } else {
    G = __expf(-0.5f * sh.r2 * q);
    ia = 1.0f;
  }
}

// This lane's pair-columns: iteration i holds column j (bins +-j).
template <int P>
struct LaneCols {
  float kx[P];       // k_x = j kstep of the lane's column in iteration i (0 if unused)
  float kx2[P];      // k_x^2
  int xi[P];         // index into the X table: j + h; ntab + 1 (X(0) / sqrt 2, the two
                     // half-weight copies of column 0) for j = 0; ntab (zero entry) if unused
  int yo[P];         // row offset within the super-row
};

// Per-pair-slot column table shared by the workgroup: entry (i, lane) =
// {k_x, k_x^2, X index, row offset}.
__device__ __forceinline__ void build_col_table(const Geom& g, const SlotPlan& sp, float4* tab) {
  const int npc = g.hc + 1;
  for (int t = threadIdx.x; t < sp.P * 64; t += blockDim.x) {
    float4 e = make_float4(0.f, 0.f, __int_as_float(g.ntab), __int_as_float(0));
    if (t < sp.R * npc) {
      const int ro = t / npc;
      const int j = t - ro * npc;
      const float kx = (float)j * g.kstep;
      e = make_float4(kx, kx * kx, __int_as_float(j == 0 ? g.ntab + 1 : j + g.h), __int_as_float(ro));
    }
    tab[t] = e;
  }
}

// PI pair-iterations per super-row for this lane: with H chains per wave the
// 64 / H lanes of a chain take pair-slots l, l + 64 / H, ... (PI = H P).
template <int PI, int H = 1>
__device__ __forceinline__ LaneCols<PI> lane_cols(const float4* tab) {
  LaneCols<PI> c;
  const int lane = chain_lane<H>();
#pragma unroll
  for (int i = 0; i < PI; ++i) {
    const float4 e = tab[lane + (64 / H) * i];
    c.kx[i] = e.x;
    c.kx2[i] = e.y;
    c.xi[i] = __float_as_int(e.z);
    c.yo[i] = __float_as_int(e.w);
  }
  return c;
}

// Per-wave LDS tables of one evaluation.
//   X [ntab+1]: F a(u) exp(-i k_u dx),   u = -h..h  (k_u dx = 2 pi u dx / N), then 0
//               (u >= 0 only for odd N: entries u < 0 are left unwritten)
//   Ym[ymax]  : {a(v) exp(-i k_v dy), k_v, k_v^2} for rows v = 0..ymax-1 (row 0
//               scaled by 1/sqrt 2, rows > hc zero)
//   Yf[ntab]  : a(v) exp(-i k_v dy),     v = -h..h (even N only, for the Nyquist bins)
// with a(u) = PSF(k_u) sinc(u/N) from atab.
// exp(-2 pi i r) for r in revolutions with the hardware sin/cos (input in
// revolutions; measured max abs error 1.3e-7 for |r| <= 3).
__device__ __forceinline__ float2 cis_neg_rev(float r) {
  return make_float2(__builtin_amdgcn_cosf(r), -__builtin_amdgcn_sinf(r));
}

// H chains per wave: the 64 / H lanes of each chain fill that chain's tables.
template <int H = 1>
__device__ __forceinline__ void fill_tables(const Geom& g, const SlotPlan& sp,
                                            const float* __restrict__ atab, float2* X, float4* Ym,
                                            float2* Yf, float F, float dx, float dy) {
  constexpr int LS = kWave / H;
  const int lane = chain_lane<H>();
  const float invN = rcp_nr((float)g.N);
  const float rx = dx * invN, ry = dy * invN;   // revolutions per unit frequency
  // the pair loop reads X(u) for u >= 0 only (X(-u) = conj X(u) is formed
  // there); the even-N Nyquist bins also read u = -N/2, so odd N fill half
  for (int t = ((g.N & 1) ? g.h : 0) + lane; t < g.ntab; t += LS) {
    const float a = F * atab[t];
    const float2 w = cis_neg_rev((float)(t - g.h) * rx);
    X[t] = make_float2(a * w.x, a * w.y);
    // column 0 of the pair loop: two half-weight copies of X(0)
    if (t == g.h) X[g.ntab + 1] = make_float2(0.70710678118654752f * a * w.x, 0.70710678118654752f * a * w.y);
  }
  if (lane == 0) X[g.ntab] = make_float2(0.f, 0.f);
  const bool even = (g.N & 1) == 0;
  for (int v = lane; v < sp.ymax; v += LS) {
    float4 y = make_float4(0.f, 0.f, 0.f, 0.f);
    if (v <= g.hc) {
      const float a = atab[v + g.h] * (v == 0 ? 0.70710678118654752f : 1.0f);
      const float2 w = cis_neg_rev((float)v * ry);
      const float ky = (float)v * g.kstep;
      y = make_float4(a * w.x, a * w.y, ky, ky * ky);
    }
    Ym[v] = y;
  }
  if (even) {
    for (int t = lane; t < g.ntab; t += LS) {
      const float a = atab[t];
      const float2 w = cis_neg_rev((float)(t - g.h) * ry);
      Yf[t] = make_float2(a * w.x, a * w.y);
    }
  }
  wave_lds_sync();
}

// Accumulate the k-space sums of one wave (red: this wave's 2 KiB reduction
// scratch in LDS).  dh: the data spectrum (or, with RESID, the spectrum of the
// pixel residual d - m) in pair-slot order followed by the Nyquist bins.  The
// X table already contains the flux.  CHI2 = false skips sum |R|^2 (the
// gradient alone).  NFIX > 0: the stamp side is the compile-time constant
// NFIX (fully unrolled super-row loop).  Result is lane-uniform.
//
// Per bin, with p = X Y the separable factor and T = G p the model spectrum,
// R = D - T, and z' = conj(R) p: the sums are sum G z' (flux), sum G a^-1 z'
// times 1, kx^2, ky^2, kx ky (shape) and sum G Im z' times kx, ky (centroid).
// The flux sum is not accumulated: a = 1 + r0^2 q (exponential and Spergel
// profiles; for the Gaussian G a^-1 = G), so sum G z' = sum G a^-1 z' +
// r0^2 sum G a^-1 z' q, and q is linear in kx^2, ky^2, kx ky (flux_sum).
//
// One pair-slot holds the bins (+kx, ky) and (-kx, ky).  They share ky, the
// row factor Y, kx^2 and |X|, and X(-kx) = conj X(kx) (the PSF-sinc factor is
// even in kx), so the two profile arguments are t = base +- tc kx ky and the
// two separable factors X Y and conj(X) Y share their four products.  The
// kx-odd sums (kx ky and kx terms) take the difference of the pair's terms,
// the even ones their sum; the kx and kx^2 factors are applied per column
// after the loop.
//
// Stationary correlated noise (CORR): each bin carries the weight w = 1 /
// lambda (lambda the noise power of its DFT mode relative to sigma^2).  The
// data spectrum is stored whitened (D sqrt w) and sw = (sqrt w(+kx), sqrt
// w(-kx)) scales the model of each bin, so every sum above becomes its
// w-weighted form (Appendix C, eq. covar-pixel-likelihood).
template <int PROF, bool RESID, bool CORR = false>
__device__ __forceinline__ void pair_step(const Shape& sh, float4 D, float4 y, float xr, float xi,
                                          float TA, float Tc, float& c2, float& swq,
                                          float& syy, float& wky, float& sdx, float& sdy, bool chi2,
                                          float2 sw = float2{1.f, 1.f}) {
  const float base = fmaf(sh.tb, y.w, TA);
  const float tp = fmaf(Tc, y.z, base), tm = fmaf(-Tc, y.z, base);
  float Gp, Gm, Gwp, Gwm;
  if (PROF == kProfExp) {
    const float rp = __builtin_amdgcn_rsqf(tp), rm = __builtin_amdgcn_rsqf(tm);
    const float rp2 = rp * rp, rm2 = rm * rm;
    Gp = rp2 * rp;
    Gm = rm2 * rm;
    Gwp = Gp * rp2;
    Gwm = Gm * rm2;
  } else if (PROF == kProfSpergel) {
    spergel_factor(sh.gw, tp, Gp, Gwp);
    spergel_factor(sh.gw, tm, Gm, Gwm);
  } else {
    Gp = __builtin_amdgcn_exp2f(tp);
    Gm = __builtin_amdgcn_exp2f(tm);
    Gwp = Gp;
    Gwm = Gm;
  }
  if constexpr (CORR) {
    Gp *= sw.x;
    Gwp *= sw.x;
    Gm *= sw.y;
    Gwm *= sw.y;
  }
  const float a = xi * y.y, b = xi * y.x;
  const float ppr = fmaf(xr, y.x, -a), pmr = fmaf(xr, y.x, a);     // X Y, conj(X) Y
  const float ppi = fmaf(xr, y.y, b), pmi = fmaf(xr, y.y, -b);
  const float Rpr = RESID ? D.x : fmaf(-Gp, ppr, D.x);
  const float Rpi = RESID ? D.y : fmaf(-Gp, ppi, D.y);
  const float Rmr = RESID ? D.z : fmaf(-Gm, pmr, D.z);
  const float Rmi = RESID ? D.w : fmaf(-Gm, pmi, D.w);
  if (chi2) c2 = fmaf(Rpr, Rpr, fmaf(Rpi, Rpi, fmaf(Rmr, Rmr, fmaf(Rmi, Rmi, c2))));
  const float zrp = fmaf(Rpr, ppr, Rpi * ppi), zip = fmaf(Rpr, ppi, -Rpi * ppr);
  const float zrm = fmaf(Rmr, pmr, Rmi * pmi), zim = fmaf(Rmr, pmi, -Rmi * pmr);
  const float wqp = Gwp * zrp;
  const float ws = fmaf(Gwm, zrm, wqp), wd = fmaf(-Gwm, zrm, wqp);
  swq += ws;
  syy = fmaf(y.w, ws, syy);
  wky = fmaf(y.z, wd, wky);
  const float gzp = Gp * zip;
  sdx = fmaf(-Gm, zim, sdx + gzp);
  sdy = fmaf(y.z, fmaf(Gm, zim, gzp), sdy);
}

// Split evaluation (W > 1 waves per chain, NFIX kernels only): wave `part`
// of the chain sums the super-rows part, part + W, ... and the Nyquist bins
// lane + 64 part, ...; the W partial sums are then exchanged through `xch`
// (W x 12 floats of LDS per chain, alternating between two buffers across
// evaluations) and added in the order 0..W-1 by every wave, so that all W
// waves hold the same totals.  The block must reach this function with all
// its waves (the exchange uses a workgroup barrier).
//
// Several chains per wave (H = 2 or 4, NFIX kernels only): the 64 / H lanes
// of each chain run the loop for their own chain (its own X, Ym, Yf tables
// and shape constants) over pair-slots l, l + 64 / H, ..., i.e. H P
// pair-iterations per super-row, and the sums are reduced per chain.
//
// CORR (one wave per chain or two chains per wave; not with a split
// evaluation): sqw holds sqrt w per bin in the data spectrum's order
// (pair-slot order, then the Nyquist bins).
template <int PROF, int P, bool RESID = false, bool CHI2 = true, int NFIX = 0, int W = 1, int H = 1,
          bool CORR = false>
__device__ KSums kspace_sums(const Geom& g, const SlotPlan& sp, const LaneCols<P * H>& lc,
                             const float2* __restrict__ dh, const float2* X, const float4* Ym,
                             const float2* Yf, const Shape& sh, float* red, int part = 0,
                             float* xch = nullptr, const float* __restrict__ sqw = nullptr) {
  static_assert(W == 1 || NFIX > 0, "split evaluation needs a specialised kernel");
  static_assert(!CORR || W == 1, "noise weights: not with a split evaluation");
  static_assert(H == 1 || (NFIX > 0 && W == 1), "several chains per wave need a specialised kernel");
  constexpr int PI = P * H;           // pair-iterations per super-row of this lane
  constexpr int LS = kWave / H;       // lanes per chain
  const int lane = chain_lane<H>();
  float xr[PI], xi[PI], TA[PI], Tc[PI];
  const float4* yp[PI];
#pragma unroll
  for (int i = 0; i < PI; ++i) {
    const float2 x = X[lc.xi[i]];
    xr[i] = x.x;
    xi[i] = x.y;
    TA[i] = fmaf(sh.ta, lc.kx2[i], sh.t0);
    Tc[i] = sh.tc * lc.kx[i];
    yp[i] = Ym + lc.yo[i];
  }
  double chi2 = 0.0;
  float syy = 0.f, sdy = 0.f;
  float swq[PI], wky[PI], sdc[PI];    // per column: times kx^2, kx, kx after the loop
#pragma unroll
  for (int i = 0; i < PI; ++i) {
    swq[i] = 0.f;
    wky[i] = 0.f;
    sdc[i] = 0.f;
  }
  const float4* dp = reinterpret_cast<const float4*>(dh) + lane;
  if constexpr (NFIX > 0) {
    constexpr SlotPlan spc = make_slot_plan_p(NFIX, P);
    static_assert(spc.R >= 1, "P too small for NFIX");
    constexpr int K = (spc.nsr + W - 1) / W;   // super-rows of this wave (at most)
    // this wave's super-rows are part + k W, k = 0..K-1 (the last may not exist)
    const float4* dq = dp + part * P * 64;
    const float2* wq = CORR ? reinterpret_cast<const float2*>(sqw) + lane : nullptr;
    const float4* yq[PI];
#pragma unroll
    for (int i = 0; i < PI; ++i) yq[i] = yp[i] + part * spc.R;
    if constexpr (W == 1) {
      // software pipeline: the LDS reads of the next pair are issued before the
      // arithmetic of the current one
      float4 Dn = dq[0];
      float4 yn = yq[0][0];
      float2 wn = CORR ? wq[0] : float2{1.f, 1.f};
#pragma unroll
      for (int k = 0; k < K; ++k) {
        float c2 = 0.f;
#pragma unroll
        for (int i = 0; i < PI; ++i) {
          const float4 D = Dn;
          const float4 y = yn;
          const float2 w = wn;
          const int b = k * PI + i + 1;         // next pair-slot of this lane
          if (b < K * PI) {
            Dn = dq[b * LS];
            yn = yq[b % PI][(b / PI) * spc.R];
            if constexpr (CORR) wn = wq[b * LS];
          }
          __builtin_amdgcn_sched_barrier(0);   // keep the reads ahead of this pair's arithmetic
          if (pair_iter_live(NFIX, spc, LS, k, i))
            pair_step<PROF, RESID, CORR>(sh, D, y, xr[i], xi[i], TA[i], Tc[i], c2, swq[i], syy,
                                         wky[i], sdc[i], sdy, CHI2, w);
        }
        if (CHI2) chi2 += (double)c2;
      }
    } else {
      const int nown = (spc.nsr - part + W - 1) / W;
      for (int k = 0; k < nown; ++k) {
        float c2 = 0.f;
#pragma unroll
        for (int i = 0; i < P; ++i)
          pair_step<PROF, RESID>(sh, dq[i * 64], yq[i][0], xr[i], xi[i], TA[i], Tc[i], c2, swq[i],
                                 syy, wky[i], sdc[i], sdy, CHI2);
        if (CHI2) chi2 += (double)c2;
        dq += W * P * 64;
#pragma unroll
        for (int i = 0; i < P; ++i) yq[i] += W * spc.R;
      }
    }
  } else {
    const float2* wp = CORR ? reinterpret_cast<const float2*>(sqw) + lane : nullptr;
    for (int sr = 0; sr < sp.nsr; ++sr) {
      float c2 = 0.f;
      const float4* yr = Ym + sr * sp.R;
#pragma unroll
      for (int i = 0; i < P; ++i)
        pair_step<PROF, RESID, CORR>(sh, dp[i * 64], yr[lc.yo[i]], xr[i], xi[i], TA[i], Tc[i], c2,
                                     swq[i], syy, wky[i], sdc[i], sdy, CHI2,
                                     CORR ? wp[i * 64] : float2{1.f, 1.f});
      if (CHI2) chi2 += (double)c2;
      dp += P * 64;
      if constexpr (CORR) wp += P * 64;
    }
  }
  float w0 = 0.f, sxx = 0.f, sxy = 0.f, sdx = 0.f;
#pragma unroll
  for (int i = 0; i < PI; ++i) {
    w0 += swq[i];
    sxx = fmaf(lc.kx2[i], swq[i], sxx);
    sxy = fmaf(lc.kx[i], wky[i], sxy);
    sdx = fmaf(lc.kx[i], sdc[i], sdx);
  }

  // Nyquist bins of an even N: each combines the frequency points +-N/2
  // (weights 1/2, sign -1 on +N/2) on its Nyquist axis or axes.
  const int h = g.h;
  const float ks = g.kstep;
  for (int i = lane + LS * part; i < sp.nspec; i += LS * W) {
    int ub, vb, c;
    nyq_bin_uv(g.N, i, ub, vb, c);
    const float2 D = dh[2 * sp.nslots + i];
    const float sw = CORR ? sqw[2 * sp.nslots + i] : 1.0f;
    const int nu = (ub == -h) ? 2 : 1;
    const int nv = (vb == -h) ? 2 : 1;
    float Mr = 0.f, Mi = 0.f;
    for (int au = 0; au < nu; ++au) {
      const int u = (nu == 2) ? (au == 0 ? -h : h) : ub;
      const float cu = (nu == 2) ? (au == 0 ? 0.5f : -0.5f) : 1.0f;
      for (int av = 0; av < nv; ++av) {
        const int v = (nv == 2) ? (av == 0 ? -h : h) : vb;
        const float cv = (nv == 2) ? (av == 0 ? 0.5f : -0.5f) : 1.0f;
        const float kx = (float)u * ks, ky = (float)v * ks;
        const float2 xu = X[u + h], yv = Yf[v + h];
        const float q = fmaf(sh.ca, kx * kx, fmaf(sh.cb, ky * ky, sh.cc * kx * ky));
        float G, ia;
        profile_factor<PROF>(sh, q, G, ia);
        const float amp = sw * G * cu * cv;
        Mr += amp * fmaf(xu.x, yv.x, -xu.y * yv.y);
        Mi += amp * fmaf(xu.x, yv.y, xu.y * yv.x);
      }
    }
    const float Rr = RESID ? D.x : D.x - Mr, Ri = RESID ? D.y : D.y - Mi;
    const float cf = 0.5f * (float)c;         // the sums are kept halved
    if (CHI2) chi2 += (double)(cf * fmaf(Rr, Rr, Ri * Ri));
    for (int au = 0; au < nu; ++au) {
      const int u = (nu == 2) ? (au == 0 ? -h : h) : ub;
      const float cu = (nu == 2) ? (au == 0 ? 0.5f : -0.5f) : 1.0f;
      for (int av = 0; av < nv; ++av) {
        const int v = (nv == 2) ? (av == 0 ? -h : h) : vb;
        const float cv = (nv == 2) ? (av == 0 ? 0.5f : -0.5f) : 1.0f;
        const float kx = (float)u * ks, ky = (float)v * ks;
        const float2 xu = X[u + h], yv = Yf[v + h];
        const float kx2b = kx * kx, ky2b = ky * ky, kxy = kx * ky;
        const float q = fmaf(sh.ca, kx2b, fmaf(sh.cb, ky2b, sh.cc * kxy));
        float G, ia;
        profile_factor<PROF>(sh, q, G, ia);
        const float Tr = sw * G * fmaf(xu.x, yv.x, -xu.y * yv.y);
        const float Ti = sw * G * fmaf(xu.x, yv.y, xu.y * yv.x);
        const float w = cf * cu * cv;
        const float zr = w * fmaf(Rr, Tr, Ri * Ti);
        const float zi = w * fmaf(Rr, Ti, -Ri * Tr);
        const float wq = zr * ia;
        w0 += wq;
        sxx = fmaf(kx2b, wq, sxx);
        syy = fmaf(ky2b, wq, syy);
        sxy = fmaf(kxy, wq, sxy);
        sdx = fmaf(kx, zi, sdx);
        sdy = fmaf(ky, zi, sdy);
      }
    }
  }

  KSums s;
  float v[7] = {w0, sxx, syy, sxy, sdx, sdy, 0.f};
  if constexpr (H == 1) {
    s.chi2 = CHI2 ? wave_total(chi2) : 0.0;
    wave_total7(v, red);
  } else {
    s.chi2 = CHI2 ? group_total<H>(chi2) : 0.0;
    group_total7<H>(v, red);
  }
  s.sF = v[0];
  s.sxx = v[1];
  s.syy = v[2];
  s.sxy = v[3];
  s.sdx = v[4];
  s.sdy = v[5];
  if constexpr (W > 1) {
    float* mine = xch + 12 * part;
    if (lane == 0) {
#pragma unroll
      for (int j = 0; j < 6; ++j) mine[j] = v[j];
      reinterpret_cast<double*>(mine)[4] = s.chi2;
    }
    __syncthreads();
    double c2 = 0.0;
    float t[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int w = 0; w < W; ++w) {
      const float* o = xch + 12 * w;
#pragma unroll
      for (int j = 0; j < 6; ++j) t[j] += o[j];
      c2 += reinterpret_cast<const double*>(o)[4];
    }
    s.chi2 = c2;
    s.sF = t[0];
    s.sxx = t[1];
    s.syy = t[2];
    s.sxy = t[3];
    s.sdx = t[4];
    s.sdy = t[5];
  }
  // q is linear in (kx^2, ky^2, kx ky), so sum q w = ca Sxx + cb Syy + cc Sxy
  s.sq = sh.ca * s.sxx + sh.cb * s.syy + sh.cc * s.sxy;
  s.sF = flux_sum<PROF>(s.sF, s.sq, sh);
  return s;
}

// Four chains per wave on an odd stamp side (NFIX kernels, one wave per
// galaxy, no noise weights): the same sums as kspace_sums with H = 4, with the
// lane's 4 P pair-slot columns taken in blocks of CB.  Each block reads its
// columns from the column table, runs over every super-row (the next pair's
// LDS reads issued ahead of the current pair's arithmetic), and folds its
// per-column sums into the totals before the next block, so only one block's
// column constants and accumulators are live at a time.
template <int PROF, int P, bool CHI2, int NFIX, int CB>
__device__ KSums kspace_sums_blocked(const float4* cols, const float2* __restrict__ dh, const float2* X,
                                     const float4* Ym, const Shape& sh, float* red) {
  constexpr int H = 4;
  constexpr int LS = kWave / H;      // lanes per chain
  constexpr int PI = P * H;          // pair-slot columns of a lane per super-row
  constexpr SlotPlan spc = make_slot_plan_p(NFIX, P);
  constexpr int K = spc.nsr;
  static_assert((NFIX & 1) && PI % CB == 0, "odd stamp sides, whole column blocks");
  const int lane = chain_lane<H>();
  const float4* dp = reinterpret_cast<const float4*>(dh) + lane;
  double chi2 = 0.0;
  float w0 = 0.f, syy = 0.f, sdy = 0.f, sxx = 0.f, sxy = 0.f, sdx = 0.f;
#pragma unroll
  for (int cb = 0; cb < PI; cb += CB) {
    float kx[CB], kx2[CB], xr[CB], xi[CB], TA[CB], Tc[CB];
    const float4* yq[CB];
#pragma unroll
    for (int i = 0; i < CB; ++i) {
      const float4 e = cols[lane + LS * (cb + i)];
      kx[i] = e.x;
      kx2[i] = e.y;
      const float2 x = X[__float_as_int(e.z)];
      xr[i] = x.x;
      xi[i] = x.y;
      TA[i] = fmaf(sh.ta, kx2[i], sh.t0);
      Tc[i] = sh.tc * kx[i];
      yq[i] = Ym + __float_as_int(e.w);
    }
    float swq[CB], wky[CB], sdc[CB];
#pragma unroll
    for (int i = 0; i < CB; ++i) {
      swq[i] = 0.f;
      wky[i] = 0.f;
      sdc[i] = 0.f;
    }
    float4 Dn = dp[cb * LS];
    float4 yn = yq[0][0];
#pragma unroll
    for (int k = 0; k < K; ++k) {
      float c2 = 0.f;
#pragma unroll
      for (int i = 0; i < CB; ++i) {
        const float4 D = Dn;
        const float4 y = yn;
        const int b = k * CB + i + 1;          // next pair of this block
        if (b < K * CB) {
          Dn = dp[((b / CB) * PI + cb + b % CB) * LS];
          yn = yq[b % CB][(b / CB) * spc.R];
        }
        __builtin_amdgcn_sched_barrier(0);   // keep the reads ahead of this pair's arithmetic
        if (pair_iter_live(NFIX, spc, LS, k, cb + i))
          pair_step<PROF, false>(sh, D, y, xr[i], xi[i], TA[i], Tc[i], c2, swq[i], syy, wky[i],
                                 sdc[i], sdy, CHI2);
      }
      if (CHI2) chi2 += (double)c2;
    }
#pragma unroll
    for (int i = 0; i < CB; ++i) {
      w0 += swq[i];
      sxx = fmaf(kx2[i], swq[i], sxx);
      sxy = fmaf(kx[i], wky[i], sxy);
      sdx = fmaf(kx[i], sdc[i], sdx);
    }
  }
  KSums s;
  float v[7] = {w0, sxx, syy, sxy, sdx, sdy, 0.f};
  s.chi2 = CHI2 ? group_total<H>(chi2) : 0.0;
  group_total7<H>(v, red);
  s.sF = v[0];
  s.sxx = v[1];
  s.syy = v[2];
  s.sxy = v[3];
  s.sdx = v[4];
  s.sdy = v[5];
  s.sq = sh.ca * s.sxx + sh.cb * s.syy + sh.cc * s.sxy;
  s.sF = flux_sum<PROF>(s.sF, s.sq, sh);
  return s;
}

// Turn the sums into log L and d log L / d(F, s, e1, e2, dx, dy).
// norm = 1 / (N^2 sigma^2); s_arcsec is the half-light radius.  The X table
// carried the flux, so sF = sum Re(conj R T) and dT/dF = T / F.
template <int PROF>
__device__ __forceinline__ KResult kspace_finish(const KSums& S, const Shape& sh, float F,
                                                 float s_arcsec, float e1, float e2, float norm) {
  KResult r;
  r.loglik = -(double)norm * S.chi2;            // -1/2 norm (2 S.chi2)
  const float c = sh.cg;                          // d ln G / dq * a
  const float n2 = 2.0f * norm;                  // the halved sums doubled
  r.dF = n2 * S.sF * rcp_nr(F);
  r.ds = n2 * (2.0f * c * rcp_nr(s_arcsec)) * S.sq;
  r.de1 = n2 * c * sh.inv1mE *
          ((2.0f * e1 + 2.0f) * S.sxx + (2.0f * e1 - 2.0f) * S.syy + 2.0f * e1 * S.sq);
  r.de2 = n2 * c * sh.inv1mE * (2.0f * e2 * (S.sxx + S.syy) + 4.0f * S.sxy + 2.0f * e2 * S.sq);
  r.ddx = n2 * S.sdx;
  r.ddy = n2 * S.sdy;
  return r;
}

}  // namespace bsi
