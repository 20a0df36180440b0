// Kernel launchers shared by the host API (one translation unit per .hip).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "bsi_device.h"

namespace bsi {

enum { kProfExpHost = 0, kProfGaussHost = 1, kProfSpergelHost = 2 };

// Half-light radius of exp(-r) in scale radii: root of (1 + x) exp(-x) = 1/2.
double exponential_hlr_factor();
// Half-light radius of the Spergel profile of index nu in scale radii r0: the
// root of x^(nu+1) K_(nu+1)(x) = 2^(nu-1) Gamma(nu+1) (enclosed flux 1/2).
double spergel_hlr_factor(double nu);

// Scale from half-light radius [arcsec] to the profile radius in pixels.
inline float profile_rscale(int prof, float pixel_scale, float nu = 0.5f) {
  if (prof == kProfExpHost) return (float)(1.0 / (exponential_hlr_factor() * (double)pixel_scale));
  if (prof == kProfSpergelHost)
    return (float)(1.0 / (spergel_hlr_factor((double)nu) * (double)pixel_scale));
  return (float)(1.0 / (1.1774100225154747 * (double)pixel_scale));   // sqrt(2 ln 2)
}

// ---- transform.hip ----
size_t dft_bins_lds_bytes(int N);
size_t render_lds_bytes(int N);
size_t render_mfma_lds_bytes(int N);
size_t dft_bins_mfma_lds_bytes(int N);
// The transforms as FP32 DFT products on the matrix cores (dft_mfma.hip)
hipError_t launch_render_mfma(const float* params, const float* psf, const int32_t* gidx, int n,
                              const int64_t* off, int N, float rscale, float pscale_inv, int prof, float nu,
                              float* out, hipStream_t s, int n_exp = 1);
hipError_t launch_dft_bins_mfma(const float* data, const double* model, const int32_t* gidx, int n,
                                const int64_t* off, const int64_t* bin_off, int N, int P, float2* out,
                                double* chi2, hipStream_t s);
// Forward DFT at the half-plane bins by either transform (mfma: the matrix-
// core form where its LDS fits, else the direct sums).
inline hipError_t launch_stamp_dft(bool mfma, const float* data, const double* model,
                                   const int32_t* gidx, int n, const int64_t* off,
                                   const int64_t* bin_off, int N, int P, float2* out, double* chi2,
                                   hipStream_t s);
// The data spectrum is written in the slot order of plan (N, P).
hipError_t launch_dft_bins(const float* data, const double* model, const int32_t* gidx, int n,
                           const int64_t* off, const int64_t* bin_off, int N, int P, float2* out,
                           double* chi2, const float* sigma, hipStream_t s);
hipError_t launch_render(const float* params, const float* psf, const int32_t* gidx, int n,
                         const int64_t* off, int N, float rscale, float pscale_inv, int prof, float nu,
                         float* out, hipStream_t s, int n_exp = 1);
hipError_t launch_render_f64(const float* params, const float* psf, const int32_t* gidx, int n,
                             const int64_t* off, int N, float rscale, float pscale_inv, int prof, float nu,
                             double* out, hipStream_t s, int n_exp = 1);

// Whitened spectrum and per-bin sqrt-weights for stationary correlated noise.
hipError_t launch_whiten(const float* noise_ps, const int32_t* gidx, int n, const int64_t* off,
                         const int64_t* bin_off, int N, int P, float2* dh, float* sqw, hipStream_t s);

// ---- likelihood.hip ----
hipError_t launch_loglik(const float2* dh, const int64_t* bin_off, const int32_t* gidx, int n,
                         const float* params, const float* psf, const float* sigma, int N, int P,
                         float rscale, float pscale_inv, int prof, float nu, int resid_mode,
                         const double* chi2_pix, double* loglik, float* grad, uint32_t* status,
                         hipStream_t s, int n_exp = 1, const float* sqw = nullptr);

// ---- hmc.hip ----
// Per-chain device state: 64 words, loaded and stored one word per lane.
struct ChainState {
  float theta[6];      // accepted position (sampling coordinates)
  float grad[6];       // grad U at theta
  float th[6];         // trajectory position
  float p[6];          // trajectory momentum
  float g[6];          // grad U at th
  float inv_mass[6];   // diagonal inverse metric
  double U;            // potential at theta
  double H0;           // Hamiltonian at the trajectory start
  double hbar;         // dual averaging: running mean of (delta - alpha)
  double log_eps_bar;  // dual averaging: averaged log step
  double Uth;          // potential at th
  float eps;           // current base step size
  float eps_t;         // this trajectory's (jittered) step
  int32_t l;           // leapfrog steps done in the current trajectory
  int32_t ok;          // trajectory stayed inside the support
  int32_t t;           // iteration index
  int32_t n_acc;       // accepted stored iterations
  int32_t n_div;       // divergent or non-finite trajectories
  uint32_t status;     // BSI_STATUS_* bits
  float sum_alpha;     // sum of acceptance statistics over stored iterations
  float u_acc;         // Metropolis uniform of the current trajectory
  uint32_t uid;        // Philox counter word 0 of this chain
  float pad[7];
};
static_assert(sizeof(ChainState) == 256, "ChainState must be 64 words");

struct HmcArgs {
  const float2* dh;
  const int64_t* bin_off;
  const int32_t* gidx;
  int n_gal;              // galaxies in this launch (entries of gidx)
  const float* psf;
  const float* sigma;
  const float* ref_xy;
  const float* init;      // [gal][C][6] (init kernel only)
  const float* inv_mass;  // [gal][6] or NULL (init kernel only)
  const uint64_t* uid_gal;  // [gal] chain-uid base or NULL: uid_base + gal * C (init kernel only)
  ChainState* state;      // [gal][C]
  float* samples;         // [gal][C][S][6] or NULL
  float* trace;           // [gal][C][W+S][4] or NULL
  int N;
  int P;                  // slot plan of N (iterations per super-row)
  int wpc;                // waves per chain of the trajectory kernel (hmc_split_waves)
  float rscale, pscale_inv;
  int prof;
  float nu;               // Spergel index (prof == kProfSpergelHost)
  int C, L, W, S, adapt, metric;
  float eps0, delta, jitter, mu;
  uint32_t k0, k1;
  uint64_t uid_base;
  float lf_lo, lf_hi, ls_lo, ls_hi, sigma_d, sigma_e;
  int n_steps;            // leapfrog steps to advance in this launch
  int t_stop;             // iteration at which a chain stops (W + S)
  const int32_t* t_stop_gal;  // [gal] per-galaxy stop (<= t_stop) or NULL (advance kernel only)
  // several exposures / correlated noise (mx = 1): galaxy
  // gal's exposures are the stamps gal * n_exp + j (psf, sigma and bin_off
  // are indexed by stamp), sqw holds sqrt w per bin beside dh, noise_ps the
  // DFT-mode noise powers at off[stamp] (NULL: white; Fisher metric only)
  int mx, n_exp;
  const float* sqw;
  const float* noise_ps;
  const int64_t* off;
  // NUTS (one wave or half-wave per chain): n_steps counts transitions
  int nuts, max_depth;
};

// Deepest NUTS tree (doublings per transition).
constexpr int kNutsMaxDepth = 10;

// LDS bytes of the trajectory kernel: C chains, W waves per chain, H chains per
// wave; E exposures and sqrt-weights (mx) for the kernels' MX form.
size_t hmc_lds_bytes(int N, int C, int P, int W, int H = 1, int E = 1, bool mx = false,
                     bool nuts = false);
// Waves per chain for stamp side N, C chains and plan P when up to max_w are
// requested: a power of two <= max_w, <= the plan's super-rows, C W <= 4, and
// 1 unless the profile is exponential or Spergel and P is N's default plan with a
// specialised kernel.
int hmc_split_waves(int N, int C, int P, int prof, int max_w);
// Whether the advance kernel with exposures / noise weights (mx) runs on the
// kernels specialised for stamp side N: one wave per chain, the exponential or
// Spergel profile and P N's default plan with a specialised kernel.
bool hmc_mx_fixed(int N, int P, int prof, int wpc);
// Slot plans with a trajectory kernel specialised for stamp side N (0-terminated list of P).
const int* hmc_fixed_plans(int N);
hipError_t launch_hmc_init(const HmcArgs& a, int grid, hipStream_t s);
hipError_t launch_hmc_advance(const HmcArgs& a, int grid, hipStream_t s);
hipError_t launch_hmc_finalize(const ChainState* st, int n_gal, int C, int S, float* chain_stats,
                               uint32_t* status, hipStream_t s);

// ---- shear.hip ----
struct ShearArgs {
  int n_gal, K;
  const float *e1p, *e2p, *l10s, *l10f;
  int e_kind;
  float e_max;
  int size_term, flux_term;
  double mu_lnf, sig_lnf;
  double log_span_s, log_span_f;   // ln of the interim uniform widths (log10 units)
  double sigma_e_interim;
  int n_pts;
  const double* pts;               // device [n_pts][5]
  double* partial;                 // device [n_blocks][n_pts][6]
  int want_grad;
  double* per_gal;                 // device [n_pts][n_gal] per-galaxy log-marginals, or NULL
  float b0, lz0;                   // interim ellipticity density in log2 units: E' coefficient,
                                   // log2 of its normaliser
  double logK;                     // ln K
};

hipError_t launch_shear(const ShearArgs& a, int n_blocks, hipStream_t s);

// ---- bootstrap.hip ----
// Shape of the m/c bootstrap product: R = n_boot + 1 rows, the galaxies
// split into n_split ranges of k_per_split for the partial products.
struct BiasPlan {
  int R, n_split, k_per_split;
  size_t partial_doubles;   // n_split x R x 2 P
};
BiasPlan bias_plan(int G, int P, int n_boot);
size_t bias_mean_lds_bytes(int P);
hipError_t launch_bias(const BiasPlan& b, const int32_t* counts, const double* ep, const double* em,
                       int G, int P, const double* gpts, double g_abs, double* partial, double* gmean,
                       double* mc, double* stats, hipStream_t s);
hipError_t launch_shear_reduce(const double* partial, int n_blocks, int n_pts, const double* pts,
                               double* logpost, double* grad, hipStream_t s);

// Shear-level sampler state per chain (float64 except the step sizes, which
// are carried in float like the per-galaxy sampler's).
struct ShearChain {
  double x[5];     // trajectory position (g1, g2, mu_ln_s, sigma_ln_s, sigma_e)
  double p[5];     // trajectory momentum
  double x0[5];    // accepted position
  double g0[5];    // grad U at x0
  double U0;       // U at x0
  double H0;       // Hamiltonian at the trajectory start
  double hbar, lbar;
  double u_acc;
  double sum_alpha;
  float eps, eps_t;
  int32_t l, t, ok, n_acc, n_div;
  uint32_t status;
};

struct ShearHmcArgs {
  ShearChain* state;   // [C]
  double* pts;         // [C][5] points of the next evaluation (read by shear_kernel)
  const double* partial;
  int n_blocks;        // blocks of the evaluation pass
  int C, L, W, S, t_stop, adapt;
  double im[5];        // diagonal inverse metric
  float eps0, delta, jitter;
  double mu;
  uint32_t k0, k1;
  uint64_t uid_base;
  double* samples;     // [C][S][5] or NULL
  float* trace;        // [C][W+S][4] or NULL
};
hipError_t launch_shear_hmc_update(const ShearHmcArgs& a, int init, hipStream_t s);
// Device address of the allocation-free pass's scratch array on `device`
// (which must be current); looked up once per device.
constexpr int kMaxDevices = 64;
hipError_t noalloc_scratch(int device, void** ptr);
hipError_t launch_shear_hmc_stats(const ShearChain* st, int C, int S, double* stats, hipStream_t s);

// ---- slots.hip ----
// One admitted request: where its slot's scalars go and where its stamp is
// copied from and to (arena offsets are in floats for the stamp and in
// complex bins for the data spectrum).
struct SlotRecord {
  int32_t slot, N;
  float psf, sigma, refx, refy;
  uint64_t uid;       // chain uid base of the request
  uint64_t src;       // device address of the caller's stamp
  int64_t off;        // stamp copy, floats from the arena start
  int64_t bin_off;    // data spectrum, complex bins from the arena start
};

// Per-slot device arrays of the request server.
struct SlotArrays {
  int64_t* off;
  int64_t* bin_off;
  float* psf;
  float* sigma;
  float* ref_xy;      // [slot][2]
  uint64_t* uid;
  float* init;        // [slot][C][6]
  int32_t* stop;      // [slot] iteration at which the request's chains wait (its next check)
  int32_t* ndraw;     // [slot] draws returned once finished, 0 while running
  int32_t* done_q;    // [slot] requests finished at checks since the last poll
  int32_t* done_n;    // entries of done_q
  float* ess6;        // [slot][6] each parameter's ESS at the request's current check
  int32_t* ess_cnt;   // [slot] parameters whose ESS is in ess6 (reset to 0 by the last)
};
// stop0: the first stop of an admitted request (its first check, or W + S).
hipError_t launch_slots_scatter(const SlotRecord* rec, const float* init_src, int n, int C, int stop0,
                                const SlotArrays& sa, float* arena, hipStream_t s);
// ndraw: per-slot draws returned (NULL: all S); out_ndraw: [n] or NULL.
hipError_t launch_slots_gather(const int32_t* list, int n, int C, int S, const ChainState* st,
                               const float* samples, const int32_t* ndraw, float* out, float* stats,
                               uint32_t* status, int32_t* out_ndraw, hipStream_t s);
// ESS checks of the listed requests whose chains wait at their stop: finish
// (ndraw, done queue) when the ESS reaches target or S draws are done, else
// move the stop `every` draws on.
hipError_t launch_slots_check(const int32_t* list, int n, int C, int W, int S, int every, float target,
                              const ChainState* st, const float* samples, const SlotArrays& sa,
                              hipStream_t s);
size_t slots_check_lds_bytes(int C, int S);

inline hipError_t launch_stamp_dft(bool mfma, const float* data, const double* model,
                                   const int32_t* gidx, int n, const int64_t* off,
                                   const int64_t* bin_off, int N, int P, float2* out, double* chi2,
                                   hipStream_t s) {
  if (mfma && dft_bins_mfma_lds_bytes(N) <= 160 * 1024)
    return launch_dft_bins_mfma(data, model, gidx, n, off, bin_off, N, P, out, chi2, s);
  return launch_dft_bins(data, model, gidx, n, off, bin_off, N, P, out, chi2, nullptr, s);
}

// ---- diag.hip ----
hipError_t launch_ess(int n_gal, int C, int S, int P, const float* samples, float* ess,
                      float* rhat, float* rsplit, hipStream_t s);

}  // namespace bsi
