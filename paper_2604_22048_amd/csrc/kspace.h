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
#pragma once

#include "bsi_device.h"

namespace bsi {

enum { kProfExp = 0, kProfGauss = 1 };

struct KSums {
  double chi2;                                    // sum over the full grid of |D - M|^2
  float sF, sxx, syy, sxy, sq, sdx, sdy;          // weighted Re/Im sums (see below)
};

struct KResult {
  double loglik;
  float dF, ds, de1, de2, ddx, ddy;               // d log L / d params
};

// Per-evaluation constants of the quadratic form q = ca kx^2 + cb ky^2 + cc kx ky.
struct Shape {
  float ca, cb, cc, r2, inv1mE;
};

__device__ __forceinline__ Shape make_shape(float rpx, float e1, float e2) {
  Shape s;
  const float E = e1 * e1 + e2 * e2;
  s.inv1mE = 1.0f / (1.0f - E);
  s.ca = (1.0f + E + 2.0f * e1) * s.inv1mE;
  s.cb = (1.0f + E - 2.0f * e1) * s.inv1mE;
  s.cc = 4.0f * e2 * s.inv1mE;
  s.r2 = rpx * rpx;
  return s;
}

// Profile factor G(q) and the factor ia multiplying z in the shape sums
// (1/(1 + r0^2 q) for the exponential, 1 for the Gaussian).
template <int PROF>
__device__ __forceinline__ void profile_factor(const Shape& sh, float q, float& G, float& ia) {
  if (PROF == kProfExp) {
    const float a = fmaf(sh.r2, q, 1.0f);
    const float rs = __builtin_amdgcn_rsqf(a);
    ia = rs * rs;
    G = ia * rs;
  } else {
    G = __expf(-0.5f * sh.r2 * q);
    ia = 1.0f;
  }
}

// Fill this wave's separable factor tables: X[u+h] = a(u) exp(-i k_u dx),
// Y[v+h] = a(v) exp(-i k_v dy), a(u) = PSF(k_u) sinc(u/N).
__device__ __forceinline__ void fill_xy(const Geom& g, const float* __restrict__ atab, float2* X,
                                        float2* Y, float dx, float dy) {
  const int lane = lane_id();
  const float two_over_n = 2.0f / (float)g.N;
  for (int t = lane; t < g.ntab; t += kWave) {
    const float u = (float)(t - g.h);
    const float a = atab[t];
    float s, c;
    sincospif(u * dx * two_over_n, &s, &c);
    X[t] = make_float2(a * c, -a * s);
    sincospif(u * dy * two_over_n, &s, &c);
    Y[t] = make_float2(a * c, -a * s);
  }
  wave_lds_sync();
}

// Accumulate the k-space sums of one wave.  dh: DFT of the data at the bins
// (main bins then special bins), or with RESID the DFT of the pixel
// residual d - m itself.  F: flux.  Result is lane-uniform.
template <int PROF, bool RESID = false>
__device__ KSums kspace_sums(const Geom& g, const float2* __restrict__ dh, const float2* X,
                             const float2* Y, float F, const Shape& sh) {
  const int lane = lane_id();
  double chi2 = 0.0;
  float sF = 0.f, sxx = 0.f, syy = 0.f, sxy = 0.f, sq = 0.f, sdx = 0.f, sdy = 0.f;
  const float ks = g.kstep;
  const int h = g.h;

  // Main bins: one frequency point each, multiplicity 2.
  for (int b = lane; b < g.nmain; b += kWave) {
    int u, v;
    main_bin_uv(g, b, u, v);
    const float kx = (float)u * ks, ky = (float)v * ks;
    const float2 D = dh[b];
    const float2 xu = X[u + h], yv = Y[v + h];
    const float pr = fmaf(xu.x, yv.x, -xu.y * yv.y);
    const float pi = fmaf(xu.x, yv.y, xu.y * yv.x);
    const float kx2 = kx * kx, ky2 = ky * ky, kxy = kx * ky;
    const float q = fmaf(sh.ca, kx2, fmaf(sh.cb, ky2, sh.cc * kxy));
    float G, ia;
    profile_factor<PROF>(sh, q, G, ia);
    const float amp = F * G;
    const float Tr = amp * pr, Ti = amp * pi;
    const float Rr = RESID ? D.x : D.x - Tr, Ri = RESID ? D.y : D.y - Ti;
    chi2 += (double)fmaf(Rr, Rr, Ri * Ri);
    const float zr = fmaf(Rr, Tr, Ri * Ti);
    const float zi = fmaf(Rr, Ti, -Ri * Tr);
    sF += zr;
    const float wq = zr * ia;
    sxx = fmaf(kx2, wq, sxx);
    syy = fmaf(ky2, wq, syy);
    sxy = fmaf(kxy, wq, sxy);
    sq = fmaf(q, wq, sq);
    sdx = fmaf(kx, zi, sdx);
    sdy = fmaf(ky, zi, sdy);
  }
  chi2 *= 2.0;
  sF *= 2.f; sxx *= 2.f; syy *= 2.f; sxy *= 2.f; sq *= 2.f; sdx *= 2.f; sdy *= 2.f;

  // Special bins: DC (all N) and the Nyquist bins of an even N.
  const bool even = (g.N & 1) == 0;
  for (int i = lane; i < g.nspec; i += kWave) {
    int ub, vb, c;
    spec_bin_uv(g.N, i, ub, vb, c);
    const float2 D = dh[g.nmain + i];
    const int nu = (even && ub == -h) ? 2 : 1;
    const int nv = (even && vb == -h) ? 2 : 1;
    float Mr = 0.f, Mi = 0.f;
    for (int au = 0; au < nu; ++au) {
      const int u = (nu == 2) ? (au == 0 ? -h : h) : ub;
      const float cu = (nu == 2) ? (au == 0 ? 0.5f : -0.5f) : 1.0f;
      for (int av = 0; av < nv; ++av) {
        const int v = (nv == 2) ? (av == 0 ? -h : h) : vb;
        const float cv = (nv == 2) ? (av == 0 ? 0.5f : -0.5f) : 1.0f;
        const float kx = (float)u * ks, ky = (float)v * ks;
        const float2 xu = X[u + h], yv = Y[v + h];
        const float q = fmaf(sh.ca, kx * kx, fmaf(sh.cb, ky * ky, sh.cc * kx * ky));
        float G, ia;
        profile_factor<PROF>(sh, q, G, ia);
        const float amp = F * G * cu * cv;
        Mr += amp * fmaf(xu.x, yv.x, -xu.y * yv.y);
        Mi += amp * fmaf(xu.x, yv.y, xu.y * yv.x);
      }
    }
    const float Rr = RESID ? D.x : D.x - Mr, Ri = RESID ? D.y : D.y - Mi;
    const float cf = (float)c;
    chi2 += (double)(cf * fmaf(Rr, Rr, Ri * Ri));
    for (int au = 0; au < nu; ++au) {
      const int u = (nu == 2) ? (au == 0 ? -h : h) : ub;
      const float cu = (nu == 2) ? (au == 0 ? 0.5f : -0.5f) : 1.0f;
      for (int av = 0; av < nv; ++av) {
        const int v = (nv == 2) ? (av == 0 ? -h : h) : vb;
        const float cv = (nv == 2) ? (av == 0 ? 0.5f : -0.5f) : 1.0f;
        const float kx = (float)u * ks, ky = (float)v * ks;
        const float2 xu = X[u + h], yv = Y[v + h];
        const float kx2 = kx * kx, ky2 = ky * ky, kxy = kx * ky;
        const float q = fmaf(sh.ca, kx2, fmaf(sh.cb, ky2, sh.cc * kxy));
        float G, ia;
        profile_factor<PROF>(sh, q, G, ia);
        const float amp = F * G;
        const float Tr = amp * fmaf(xu.x, yv.x, -xu.y * yv.y);
        const float Ti = amp * fmaf(xu.x, yv.y, xu.y * yv.x);
        const float w = cf * cu * cv;
        const float zr = w * fmaf(Rr, Tr, Ri * Ti);
        const float zi = w * fmaf(Rr, Ti, -Ri * Tr);
        sF += zr;
        const float wq = zr * ia;
        sxx = fmaf(kx2, wq, sxx);
        syy = fmaf(ky2, wq, syy);
        sxy = fmaf(kxy, wq, sxy);
        sq = fmaf(q, wq, sq);
        sdx = fmaf(kx, zi, sdx);
        sdy = fmaf(ky, zi, sdy);
      }
    }
  }

  KSums s;
  s.chi2 = wave_sum(chi2);
  s.sF = wave_sum(sF);
  s.sxx = wave_sum(sxx);
  s.syy = wave_sum(syy);
  s.sxy = wave_sum(sxy);
  s.sq = wave_sum(sq);
  s.sdx = wave_sum(sdx);
  s.sdy = wave_sum(sdy);
  return s;
}

// Turn the sums into log L and d log L / d(F, s, e1, e2, dx, dy).
// norm = 1 / (N^2 sigma^2); s_arcsec is the half-light radius.
template <int PROF>
__device__ __forceinline__ KResult kspace_finish(const KSums& S, const Shape& sh, float F,
                                                 float s_arcsec, float e1, float e2, float norm) {
  KResult r;
  r.loglik = -0.5 * (double)norm * S.chi2;
  const float c = (PROF == kProfExp) ? -1.5f * sh.r2 : -0.5f * sh.r2;   // d ln G / dq * a
  r.dF = norm * S.sF / F;
  r.ds = norm * (2.0f * c / s_arcsec) * S.sq;
  r.de1 = norm * c * sh.inv1mE *
          ((2.0f * e1 + 2.0f) * S.sxx + (2.0f * e1 - 2.0f) * S.syy + 2.0f * e1 * S.sq);
  r.de2 = norm * c * sh.inv1mE * (2.0f * e2 * (S.sxx + S.syy) + 4.0f * S.sxy + 2.0f * e2 * S.sq);
  r.ddx = norm * S.sdx;
  r.ddy = norm * S.sdy;
  return r;
}

}  // namespace bsi
