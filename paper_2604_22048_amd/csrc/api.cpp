// Host implementation of the C ABI declared in include/bsi.h.
#include "bsi.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <string>
#include <vector>

#include "bsi_kernels.h"
#include "ctx.h"
#include "kspace.h"

using namespace bsi;

using namespace bsi_host;

namespace {

thread_local std::string g_create_error;

// A batch holds n_gal galaxies of E exposures each: stamp i E + j is exposure
// j of galaxy i (E = 1: one stamp per galaxy, stamp = galaxy).
struct ClassRange {
  int N;
  int P;       // slot plan
  int begin;   // position in the sorted stamp list
  int count;   // stamps
  int gbegin;  // position in the sorted galaxy list
  int gcount;  // galaxies
};

struct Plan {
  int E = 1;                      // exposures per galaxy
  std::vector<int32_t> gidx;      // stamps grouped by stamp side (a galaxy's exposures in order)
  std::vector<int32_t> ggidx;     // galaxies grouped by stamp side
  std::vector<int64_t> bin_off;   // per stamp, offset into the bin buffer (complex units)
  std::vector<ClassRange> classes;
  int64_t total_bins = 0;
  int64_t max_pixel = 0;          // one past the largest pixel index
};

inline int exposures(const bsi_batch* b) { return b->n_exp > 1 ? b->n_exp : 1; }

int check_batch(bsi_handle h, const bsi_batch* b) {
  if (!b) return fail(h, BSI_EINVAL, "batch is NULL");
  if (b->n_gal < 0) return fail(h, BSI_EINVAL, "n_gal < 0");
  if (b->n_gal == 0) return BSI_OK;
  if (!b->n || !b->off) return fail(h, BSI_EINVAL, "batch n/off host arrays are NULL");
  if (!b->psf_fwhm || !b->sigma) return fail(h, BSI_EINVAL, "batch psf_fwhm/sigma are NULL");
  if (!(b->pixel_scale > 0.0f) || !std::isfinite(b->pixel_scale))
    return fail(h, BSI_EINVAL, "pixel_scale must be positive");
  if (b->profile != BSI_PROFILE_EXPONENTIAL && b->profile != BSI_PROFILE_GAUSSIAN &&
      b->profile != BSI_PROFILE_SPERGEL)
    return fail(h, BSI_EINVAL, "unknown profile %d", b->profile);
  if (b->profile == BSI_PROFILE_SPERGEL &&
      !(b->spergel_nu >= BSI_SPERGEL_NU_MIN && b->spergel_nu <= BSI_SPERGEL_NU_MAX))
    return fail(h, BSI_EINVAL, "Spergel index %g outside [%g, %g]", (double)b->spergel_nu,
                (double)BSI_SPERGEL_NU_MIN, (double)BSI_SPERGEL_NU_MAX);
  if (b->n_exp < 0 || b->n_exp > BSI_MAX_EXPOSURES)
    return fail(h, BSI_EINVAL, "n_exp %d outside [0, %d]", b->n_exp, BSI_MAX_EXPOSURES);
  const int E = exposures(b);
  for (int64_t i = 0; i < (int64_t)b->n_gal * E; ++i) {
    if (b->n[i] < 8 || b->n[i] > kMaxN)
      return fail(h, BSI_EUNSUPPORTED, "stamp side %d of stamp %lld outside [8, %d]", b->n[i],
                  (long long)i, kMaxN);
    if (b->n[i] != b->n[i - i % E])
      return fail(h, BSI_EINVAL, "exposures of galaxy %lld differ in stamp side", (long long)(i / E));
    if (b->off[i] < 0) return fail(h, BSI_EINVAL, "negative offset for stamp %lld", (long long)i);
  }
  return BSI_OK;
}

// Slot plan of stamp side N on this handle.
int plan_of(bsi_handle h, int N) {
  const int P = (N >= 0 && N <= kMaxN) ? h->plan_P[N] : 0;
  return P > 0 ? P : make_slot_plan(N).P;
}

Plan make_plan(bsi_handle h, const bsi_batch* b) {
  Plan p;
  p.E = exposures(b);
  const int E = p.E;
  std::map<int, std::vector<int32_t>> by;
  for (int i = 0; i < b->n_gal; ++i) by[b->n[(int64_t)i * E]].push_back(i);
  p.bin_off.assign((size_t)b->n_gal * E, 0);
  int64_t bins = 0;
  for (auto& kv : by) {
    ClassRange c{kv.first, plan_of(h, kv.first), (int)p.gidx.size(), (int)kv.second.size() * E,
                 (int)p.ggidx.size(), (int)kv.second.size()};
    const SlotPlan sp = make_slot_plan_p(c.N, c.P);
    for (int32_t i : kv.second) {
      p.ggidx.push_back(i);
      for (int j = 0; j < E; ++j) {
        const int32_t st = i * E + j;
        p.gidx.push_back(st);
        p.bin_off[st] = bins;
        bins += sp.nbins;
        p.max_pixel = std::max<int64_t>(p.max_pixel, b->off[st] + (int64_t)kv.first * kv.first);
      }
    }
    p.classes.push_back(c);
  }
  p.total_bins = bins;
  return p;
}

// Workspace of a batch's plan: stamp and galaxy index lists, pixel and bin
// offsets (device), and their staging.
struct PlanBytes {
  size_t gidx, off, bin_off, ggidx;
  size_t stage() const { return bsi_host::stage_size({gidx, off, bin_off, ggidx}); }
};

PlanBytes plan_bytes(const bsi_batch* b, const Plan& p) {
  const size_t n = (size_t)b->n_gal * p.E;     // stamps
  return {n * sizeof(int32_t), n * sizeof(int64_t), n * sizeof(int64_t),
          p.E > 1 ? (size_t)b->n_gal * sizeof(int32_t) : 0};
}

// Upload the plan's index arrays into the handle workspace (sized by prepare).
int upload_plan(bsi_handle h, const bsi_batch* b, const Plan& p, hipStream_t s, bool cap) {
  const PlanBytes pb = plan_bytes(b, p);
  return stage_upload(h, s, cap, {{h->gidx.p, p.gidx.data(), pb.gidx},
                                   {h->off.p, b->off, pb.off},
                                   {h->bin_off.p, p.bin_off.data(), pb.bin_off},
                                   {h->ggidx.p, p.ggidx.data(), pb.ggidx}});
}

// The class's stamps, and its galaxies (the same list when E = 1).
const int32_t* gidx_ptr(bsi_handle h, const ClassRange& c) {
  return static_cast<const int32_t*>(h->gidx.p) + c.begin;
}

const int32_t* ggidx_ptr(bsi_handle h, const Plan& p, const ClassRange& c) {
  return static_cast<const int32_t*>(p.E > 1 ? h->ggidx.p : h->gidx.p) + c.gbegin;
}

// Per-bin noise weights (sqrt w beside the spectrum, which is whitened) for
// batches with several exposures or correlated noise.
int noise_weights(bsi_handle h, const bsi_batch* b, const Plan& p, hipStream_t s) {
  for (const ClassRange& c : p.classes) {
    hipError_t e = launch_whiten(b->noise_ps, gidx_ptr(h, c), c.count,
                                 static_cast<const int64_t*>(h->off.p),
                                 static_cast<const int64_t*>(h->bin_off.p), c.N, c.P,
                                 static_cast<float2*>(h->dh.p), static_cast<float*>(h->sqw.p), s);
    if (e != hipSuccess) return hip_fail(h, e, "noise weights launch");
  }
  return BSI_OK;
}

inline bool weighted(const bsi_batch* b) { return b->n_exp > 1 || b->noise_ps != nullptr; }

int data_spectrum(bsi_handle h, const bsi_batch* b, const Plan& p, const float* data,
                  const double* model, double* chi2, hipStream_t s) {
  for (const ClassRange& c : p.classes) {
    hipError_t e = launch_stamp_dft(transform_of(h, c.N) == BSI_TRANSFORM_MFMA, data, model,
                                    gidx_ptr(h, c), c.count, static_cast<const int64_t*>(h->off.p),
                                    static_cast<const int64_t*>(h->bin_off.p), c.N, c.P,
                                    static_cast<float2*>(h->dh.p), chi2, s);
    if (e != hipSuccess) return hip_fail(h, e, "dft_bins launch");
  }
  return BSI_OK;
}

// Every workspace buffer of a handle (an array: an initializer_list returned
// from a function would refer to a temporary that dies with the return).
std::array<DevBuf*, 14> all_buffers(bsi_handle h) {
  return {&h->gidx, &h->ggidx, &h->off, &h->bin_off, &h->dh, &h->sqw, &h->chi2, &h->model, &h->state,
          &h->partial, &h->pts, &h->shear_state, &h->bias_part, &h->bias_mc};
}

// Free replaced buffers and finished graphs; the caller has synchronised the
// device, so nothing enqueued by the library can still use them.
void release_retired(bsi_handle h) {
  for (void* p : h->retired) (void)hipFree(p);
  h->retired.clear();
  for (void* p : h->retired_host) (void)hipHostFree(p);
  h->retired_host.clear();
  bsi_host::reap_graphs(h);
  h->stage_pending = false;
}

// Largest stored spectrum (complex values) of one stamp of side <= max_n
// under any slot plan a handle can choose.
size_t max_bins_per_stamp(int max_n) {
  size_t m = 0;
  for (int N = 8; N <= max_n; ++N)
    for (int P : kPlanP)
      if (plan_valid(N, P)) m = std::max<size_t>(m, (size_t)make_slot_plan_p(N, P).nbins);
  return m;
}

}  // namespace

extern "C" {

int bsi_version(void) { return BSI_VERSION; }

int bsi_device_count(int32_t* n) {
  if (!n) return BSI_EINVAL;
  int c = 0;
  hipError_t e = hipGetDeviceCount(&c);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    *n = 0;
    return BSI_OK;
  }
  *n = c;
  return BSI_OK;
}

int bsi_create(bsi_handle* out, int32_t device, const char* tune_cache) {
  if (!out) {
    g_create_error = "out is NULL";
    return BSI_EINVAL;
  }
  *out = nullptr;
  int count = 0;
  if (hipGetDeviceCount(&count) != hipSuccess || count == 0) {
    (void)hipGetLastError();
    g_create_error = "no HIP device";
    return BSI_ENODEV;
  }
  if (device < 0 || device >= count) {
    g_create_error = "device ordinal out of range";
    return BSI_EINVAL;
  }
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, device) != hipSuccess) {
    g_create_error = "hipGetDeviceProperties failed";
    return BSI_EHIP;
  }
  if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0) {
    g_create_error = std::string("unsupported device architecture ") + prop.gcnArchName;
    return BSI_EUNSUPPORTED;
  }
  if (hipSetDevice(device) != hipSuccess) {
    g_create_error = "hipSetDevice failed";
    return BSI_EHIP;
  }
  // the allocation-free entry point's scratch: this device's address of the
  // library's device array, looked up once per device with the device current
  void* scratch = nullptr;
  if (device >= kMaxDevices || noalloc_scratch(device, &scratch) != hipSuccess) {
    (void)hipGetLastError();
    g_create_error = "device scratch lookup failed";
    return BSI_EHIP;
  }
  bsi_ctx* h = new bsi_ctx();
  h->device = device;
  h->num_cu = prop.multiProcessorCount;
  h->scratch = scratch;
  h->arch = std::string(prop.gcnArchName).substr(0, std::string(prop.gcnArchName).find(':'));
  if (tune_cache && *tune_cache) {
    h->tune_cache = tune_cache;
    std::string err;
    if (load_tune_cache(h, err) != BSI_OK) {
      delete h;
      g_create_error = err;
      return BSI_EINVAL;
    }
  }
  bool ok = hipStreamCreate(&h->own) == hipSuccess &&
            hipEventCreateWithFlags(&h->ev_fork, hipEventDisableTiming) == hipSuccess &&
            hipEventCreateWithFlags(&h->ev_done, hipEventDisableTiming) == hipSuccess &&
            hipEventCreateWithFlags(&h->ev_stage, hipEventDisableTiming) == hipSuccess;
  // the auxiliary streams do not synchronise implicitly with the null stream:
  // a forked launch's branches are ordered by its events alone, so a branch
  // left on a caller's null stream runs beside the others instead of
  // holding them back until it ends
  for (int i = 0; ok && i < kAuxStreams; ++i)
    ok = hipStreamCreateWithFlags(&h->aux[i], hipStreamNonBlocking) == hipSuccess &&
         hipEventCreateWithFlags(&h->ev_join[i], hipEventDisableTiming) == hipSuccess;
  if (!ok) {
    (void)hipGetLastError();
    bsi_destroy(h);
    g_create_error = "stream or event creation failed";
    return BSI_EHIP;
  }
  *out = h;
  return BSI_OK;
}

void bsi_destroy(bsi_handle h) {
  if (!h) return;
  (void)hipSetDevice(h->device);
  (void)hipDeviceSynchronize();
  release_retired(h);
  for (DevBuf* b : all_buffers(h))
    if (b->p) (void)hipFree(b->p);
  if (h->stage) (void)hipHostFree(h->stage);
  if (h->ev_done) (void)hipEventDestroy(h->ev_done);
  if (h->ev_stage) (void)hipEventDestroy(h->ev_stage);
  if (h->own) (void)hipStreamDestroy(h->own);
  for (int i = 0; i < kAuxStreams; ++i) {
    if (h->aux[i]) (void)hipStreamDestroy(h->aux[i]);
    if (h->ev_join[i]) (void)hipEventDestroy(h->ev_join[i]);
  }
  if (h->ev_fork) (void)hipEventDestroy(h->ev_fork);
  delete h;
}

const char* bsi_last_error(bsi_handle h) {
  if (!h) return g_create_error.c_str();
  return h->err.c_str();
}

int bsi_render_stamps(bsi_handle h, const bsi_batch* batch, const float* params, float* out,
                      bsi_stream stream) {
  if (!h) return BSI_EINVAL;
  h->err.clear();
  int rc = check_batch(h, batch);
  if (rc) return rc;
  if (batch->n_gal == 0) return BSI_OK;
  if (!params || !out) return fail(h, BSI_EINVAL, "params/out is NULL");
  (void)hipSetDevice(h->device);
  hipStream_t s = static_cast<hipStream_t>(stream);
  const bool cap = capturing(s);
  const Plan p = make_plan(h, batch);
  const PlanBytes pb = plan_bytes(batch, p);
  if ((rc = prepare(h, s, cap, {{&h->gidx, pb.gidx}, {&h->off, pb.off}, {&h->bin_off, pb.bin_off},
                                {&h->ggidx, pb.ggidx}}, pb.stage())))
    return rc;
  if ((rc = upload_plan(h, batch, p, s, cap))) return rc;
  const float rs = profile_rscale(batch->profile, batch->pixel_scale, batch->spergel_nu);
  for (const ClassRange& c : p.classes) {
    const int32_t* gi = gidx_ptr(h, c);
    const int64_t* off = static_cast<const int64_t*>(h->off.p);
    hipError_t e = transform_of(h, c.N) == BSI_TRANSFORM_MFMA
        ? launch_render_mfma(params, batch->psf_fwhm, gi, c.count, off, c.N, rs,
                             1.0f / batch->pixel_scale, batch->profile, batch->spergel_nu, out, s,
                             p.E)
        : launch_render(params, batch->psf_fwhm, gi, c.count, off, c.N, rs,
                        1.0f / batch->pixel_scale, batch->profile, batch->spergel_nu, out, s, p.E);
    if (e != hipSuccess) return hip_fail(h, e, "render launch");
  }
  return finish(h, s, cap);
}

int bsi_loglik_grad(bsi_handle h, const bsi_batch* batch, const float* data, const float* params,
                    double* loglik, float* grad, uint32_t* status, int32_t method,
                    bsi_stream stream) {
  if (!h) return BSI_EINVAL;
  h->err.clear();
  int rc = check_batch(h, batch);
  if (rc) return rc;
  if (batch->n_gal == 0) return BSI_OK;
  if (!data || !params) return fail(h, BSI_EINVAL, "data/params is NULL");
  if (method != BSI_LIK_KSPACE && method != BSI_LIK_PIXEL)
    return fail(h, BSI_EINVAL, "unknown likelihood method %d", method);
  if (method == BSI_LIK_PIXEL && weighted(batch))
    return fail(h, BSI_EUNSUPPORTED, "several exposures / noise_ps need the k-space method");
  (void)hipSetDevice(h->device);
  hipStream_t s = static_cast<hipStream_t>(stream);
  const bool cap = capturing(s);
  const Plan p = make_plan(h, batch);
  const PlanBytes pb = plan_bytes(batch, p);
  const bool pixel = method == BSI_LIK_PIXEL;
  const bool mx = weighted(batch);
  if ((rc = prepare(h, s, cap,
                    {{&h->gidx, pb.gidx}, {&h->off, pb.off}, {&h->bin_off, pb.bin_off},
                     {&h->ggidx, pb.ggidx}, {&h->dh, (size_t)p.total_bins * sizeof(float2)},
                     {&h->sqw, mx ? (size_t)p.total_bins * sizeof(float) : 0},
                     {&h->model, pixel ? (size_t)p.max_pixel * sizeof(double) : 0},
                     {&h->chi2, pixel ? (size_t)batch->n_gal * sizeof(double) : 0}},
                    pb.stage())))
    return rc;
  if ((rc = upload_plan(h, batch, p, s, cap))) return rc;
  const float rs = profile_rscale(batch->profile, batch->pixel_scale, batch->spergel_nu);
  const int64_t* off = static_cast<const int64_t*>(h->off.p);
  double* chi2 = nullptr;
  const double* model = nullptr;
  if (pixel) {
    for (const ClassRange& c : p.classes) {
      hipError_t e = launch_render_f64(params, batch->psf_fwhm, gidx_ptr(h, c), c.count, off, c.N,
                                       rs, 1.0f / batch->pixel_scale, batch->profile, batch->spergel_nu,
                                       static_cast<double*>(h->model.p), s);
      if (e != hipSuccess) return hip_fail(h, e, "render launch");
    }
    model = static_cast<const double*>(h->model.p);
    chi2 = static_cast<double*>(h->chi2.p);
  }
  if ((rc = data_spectrum(h, batch, p, data, model, chi2, s))) return rc;
  if (mx && (rc = noise_weights(h, batch, p, s))) return rc;
  for (const ClassRange& c : p.classes) {
    hipError_t e = launch_loglik(static_cast<const float2*>(h->dh.p),
                                 static_cast<const int64_t*>(h->bin_off.p), ggidx_ptr(h, p, c),
                                 c.gcount, params, batch->psf_fwhm, batch->sigma, c.N, c.P, rs,
                                 1.0f / batch->pixel_scale, batch->profile, batch->spergel_nu,
                                 method == BSI_LIK_PIXEL, chi2, loglik, grad, status, s, p.E,
                                 mx ? static_cast<const float*>(h->sqw.p) : nullptr);
    if (e != hipSuccess) return hip_fail(h, e, "loglik launch");
  }
  return finish(h, s, cap);
}

int bsi_hmc_sample(bsi_handle h, const bsi_batch* batch, const float* data, const float* ref_xy,
                   const float* inv_mass, const float* init, const bsi_interim* ip,
                   const bsi_hmc_cfg* cfg, float* samples, float* chain_stats, uint32_t* status,
                   bsi_stream stream) {
  if (!h) return BSI_EINVAL;
  h->err.clear();
  int rc = check_batch(h, batch);
  if (rc) return rc;
  if (!cfg || !ip) return fail(h, BSI_EINVAL, "cfg/interim is NULL");
  if (cfg->n_chains < 1 || cfg->n_chains > 16) return fail(h, BSI_EINVAL, "n_chains must be 1..16");
  if (cfg->n_leapfrog < 1) return fail(h, BSI_EINVAL, "n_leapfrog must be >= 1");
  if (cfg->n_warmup < 0 || cfg->n_samples < 0) return fail(h, BSI_EINVAL, "negative iteration count");
  if (!(cfg->step_size > 0.0f) || !std::isfinite(cfg->step_size))
    return fail(h, BSI_EINVAL, "step_size must be positive");
  if (cfg->adapt && !(cfg->target_accept > 0.0f && cfg->target_accept < 1.0f))
    return fail(h, BSI_EINVAL, "target_accept must be in (0, 1)");
  if (!(cfg->jitter >= 0.0f && cfg->jitter < 1.0f)) return fail(h, BSI_EINVAL, "jitter must be in [0, 1)");
  if (cfg->metric != BSI_METRIC_GIVEN && cfg->metric != BSI_METRIC_FISHER)
    return fail(h, BSI_EINVAL, "unknown metric %d", cfg->metric);
  if (cfg->form != BSI_FORM_BATCHED && cfg->form != BSI_FORM_PLAIN)
    return fail(h, BSI_EINVAL, "unknown form %d", cfg->form);
  if (cfg->form == BSI_FORM_BATCHED && cfg->iters_per_launch < 1)
    return fail(h, BSI_EINVAL, "iters_per_launch must be >= 1");
  if (cfg->waves_per_chain < 0 || cfg->waves_per_chain > 4)
    return fail(h, BSI_EINVAL, "waves_per_chain must be 0..4");
  if (cfg->sampler != BSI_SAMPLER_HMC && cfg->sampler != BSI_SAMPLER_NUTS)
    return fail(h, BSI_EINVAL, "unknown sampler %d", cfg->sampler);
  const bool nuts = cfg->sampler == BSI_SAMPLER_NUTS;
  if (nuts && (cfg->max_tree_depth < 1 || cfg->max_tree_depth > BSI_NUTS_MAX_DEPTH))
    return fail(h, BSI_EINVAL, "max_tree_depth must be 1..%d", BSI_NUTS_MAX_DEPTH);
  if (!(ip->log10f_lo < ip->log10f_hi) || !(ip->log10s_lo < ip->log10s_hi) || !(ip->sigma_d > 0) ||
      !(ip->sigma_e > 0))
    return fail(h, BSI_EINVAL, "invalid interim prior");
  if (batch->n_gal == 0) return BSI_OK;
  if (!data || !ref_xy || !init) return fail(h, BSI_EINVAL, "data/ref_xy/init is NULL");
  if (cfg->n_samples > 0 && !samples && !chain_stats && !status)
    return fail(h, BSI_EINVAL, "no output requested");
  (void)hipSetDevice(h->device);
  hipStream_t s = stream ? static_cast<hipStream_t>(stream) : h->own;
  const bool cap = capturing(s);
  const Plan p = make_plan(h, batch);
  const int C = cfg->n_chains;
  const bool mx = weighted(batch);
  // every check before anything is enqueued
  if (mx && C > 4) return fail(h, BSI_EUNSUPPORTED, "several exposures / noise_ps: n_chains <= 4");
  for (const ClassRange& c : p.classes) {
    const size_t lds = mx ? hmc_lds_bytes(c.N, C, c.P, 1, 1, p.E, true, nuts)
                     : nuts ? hmc_lds_bytes(c.N, C, c.P, 1, 1, 1, false, true)
                          : hmc_lds_bytes(c.N, C, c.P,
                                          hmc_split_waves(c.N, C, c.P, batch->profile, cfg->waves_per_chain));
    if (lds > 160 * 1024)
      return fail(h, BSI_EUNSUPPORTED, "N = %d with %d chains (and %d exposures) exceeds LDS", c.N, C, p.E);
  }
  const PlanBytes pb = plan_bytes(batch, p);
  if ((rc = prepare(h, s, cap,
                    {{&h->gidx, pb.gidx}, {&h->off, pb.off}, {&h->bin_off, pb.bin_off},
                     {&h->ggidx, pb.ggidx}, {&h->dh, (size_t)p.total_bins * sizeof(float2)},
                     {&h->sqw, mx ? (size_t)p.total_bins * sizeof(float) : 0},
                     {&h->state, (size_t)batch->n_gal * C * sizeof(ChainState)}},
                    pb.stage())))
    return rc;
  if ((rc = upload_plan(h, batch, p, s, cap))) return rc;
  if ((rc = data_spectrum(h, batch, p, data, nullptr, nullptr, s))) return rc;
  if (mx && (rc = noise_weights(h, batch, p, s))) return rc;

  HmcArgs a{};
  a.dh = static_cast<const float2*>(h->dh.p);
  a.bin_off = static_cast<const int64_t*>(h->bin_off.p);
  a.psf = batch->psf_fwhm;
  a.sigma = batch->sigma;
  a.ref_xy = ref_xy;
  a.init = init;
  a.inv_mass = inv_mass;
  a.state = static_cast<ChainState*>(h->state.p);
  a.samples = samples;
  a.trace = cfg->trace;
  a.rscale = profile_rscale(batch->profile, batch->pixel_scale, batch->spergel_nu);
  a.pscale_inv = 1.0f / batch->pixel_scale;
  a.prof = batch->profile;
  a.nu = batch->spergel_nu;
  a.C = C;
  a.L = cfg->n_leapfrog;
  a.W = cfg->n_warmup;
  a.S = cfg->n_samples;
  a.adapt = cfg->adapt;
  a.metric = cfg->metric;
  a.eps0 = cfg->step_size;
  a.delta = cfg->target_accept;
  a.jitter = cfg->jitter;
  a.mu = (float)std::log(10.0 * (double)cfg->step_size);
  a.k0 = (uint32_t)(cfg->seed & 0xffffffffu);
  a.k1 = (uint32_t)(cfg->seed >> 32);
  a.uid_base = cfg->uid_base;
  a.lf_lo = ip->log10f_lo;
  a.lf_hi = ip->log10f_hi;
  a.ls_lo = ip->log10s_lo;
  a.ls_hi = ip->log10s_hi;
  a.sigma_d = ip->sigma_d;
  a.sigma_e = ip->sigma_e;
  a.t_stop = cfg->n_warmup + cfg->n_samples;
  a.wpc = 1;
  a.mx = mx ? 1 : 0;
  a.n_exp = p.E;
  a.sqw = mx ? static_cast<const float*>(h->sqw.p) : nullptr;
  a.noise_ps = batch->noise_ps;
  a.off = static_cast<const int64_t*>(h->off.p);
  a.nuts = nuts ? 1 : 0;
  a.max_depth = cfg->max_tree_depth;

  for (const ClassRange& c : p.classes) {
    HmcArgs ac = a;
    ac.N = c.N;
    ac.P = c.P;
    ac.gidx = ggidx_ptr(h, p, c);
    ac.n_gal = c.gcount;
    ac.n_steps = 0;
    hipError_t e = launch_hmc_init(ac, c.gcount, s);
    if (e != hipSuccess) return hip_fail(h, e, "hmc init launch");
  }
  const int T = a.t_stop;
  if (cfg->form == BSI_FORM_PLAIN) {
    // one galaxy, one leapfrog step per launch
    for (const ClassRange& c : p.classes) {
      for (int i = 0; i < c.gcount; ++i) {
        HmcArgs ac = a;
        ac.N = c.N;
        ac.P = c.P;
        ac.gidx = ggidx_ptr(h, p, c) + i;
        ac.n_gal = 1;
        ac.n_steps = 1;
        for (int64_t k = 0; k < (int64_t)T * (nuts ? 1 : a.L); ++k) {
          hipError_t e = launch_hmc_advance(ac, 1, s);
          if (e != hipSuccess) return hip_fail(h, e, "hmc advance launch");
        }
      }
    }
  } else {
    const int ipl = std::min(cfg->iters_per_launch, std::max(T, 1));
    const int n_launch = (T + ipl - 1) / ipl;
    auto advance_class = [&](int i, hipStream_t sc) -> hipError_t {
      const ClassRange& c = p.classes[i];
      HmcArgs ac = a;
      ac.N = c.N;
      ac.P = c.P;
      ac.wpc = (mx || nuts) ? 1 : hmc_split_waves(c.N, C, c.P, batch->profile, cfg->waves_per_chain);
      ac.gidx = ggidx_ptr(h, p, c);
      ac.n_gal = c.gcount;
      ac.n_steps = nuts ? ipl : ipl * a.L;
      return launch_hmc_advance(ac, c.gcount, sc);
    };
    // direct launches: the sizes run concurrently on forked streams
    auto enqueue = [&](hipStream_t st) -> hipError_t {
      return fork_join(h, st, (int)p.classes.size(), advance_class, [&](int i) {
        const ClassRange& c = p.classes[i];
        return (double)c.N * c.N * c.gcount;    // the class's share of the work
      });
    };
    // any capture (the library's own graph or the caller's): one stream, the
    // sizes' launches in sequence.  Capturing the fork/join has ended in a
    // host segmentation fault inside the call (cause not identified), so it
    // is never captured.
    auto enqueue_serial = [&](hipStream_t st) -> hipError_t {
      for (int i = 0; i < (int)p.classes.size(); ++i) {
        hipError_t e = advance_class(i, st);
        if (e != hipSuccess) return e;
      }
      return hipSuccess;
    };
    if (cap) {
      // the caller's graph replays this call: its launches go in as they are,
      // the sizes in sequence on the capturing stream
      for (int k = 0; k < n_launch; ++k) {
        hipError_t e = enqueue_serial(s);
        if (e != hipSuccess) return hip_fail(h, e, "hmc advance launch");
      }
    } else if (cfg->use_graph && n_launch > 1) {
      hipGraph_t graph = nullptr;
      hipGraphExec_t exec = nullptr;
      hipError_t e = hipStreamBeginCapture(s, hipStreamCaptureModeRelaxed);
      if (e == hipSuccess) e = enqueue_serial(s);
      hipError_t e2 = hipStreamEndCapture(s, &graph);
      if (e == hipSuccess) e = e2;
      if (e == hipSuccess) e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
      for (int k = 0; e == hipSuccess && k < n_launch; ++k) e = hipGraphLaunch(exec, s);
      if (e != hipSuccess) {
        // nothing of the graph may still run unless a launch succeeded: wait, then destroy
        (void)hipStreamSynchronize(s);
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
        return hip_fail(h, e, "hmc graph");
      }
      // the replays are in flight: the graph is destroyed once they have run
      if ((rc = keep_graph(h, exec, graph, s))) return rc;
    } else {
      for (int k = 0; k < n_launch; ++k) {
        hipError_t e = enqueue(s);
        if (e != hipSuccess) return hip_fail(h, e, "hmc advance launch");
      }
    }
  }
  hipError_t e = launch_hmc_finalize(static_cast<const ChainState*>(h->state.p), batch->n_gal, C,
                                     cfg->n_samples, chain_stats, status, s);
  if (e != hipSuccess) return hip_fail(h, e, "hmc finalize launch");
  if ((rc = finish(h, s, cap))) return rc;
  if (!stream) {
    e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_fail(h, e, "hmc sync");
  }
  return BSI_OK;
}

}  // extern "C"

namespace {

int check_shear_inputs(bsi_handle h, int32_t n_gal, int32_t K, const float* e1p, const float* e2p,
                       const float* log10s, const float* log10f, const bsi_true_prior* tp,
                       const bsi_interim* ip) {
  if (n_gal < 1) return fail(h, BSI_EINVAL, "n_gal must be >= 1");
  if (K < 1) return fail(h, BSI_EINVAL, "K must be >= 1");
  if (!tp || !ip) return fail(h, BSI_EINVAL, "true prior / interim is NULL");
  if (tp->e_kind != BSI_E_BA14 && tp->e_kind != BSI_E_TRUNC_GAUSS)
    return fail(h, BSI_EINVAL, "unknown e_kind");
  if (tp->e_kind == BSI_E_TRUNC_GAUSS && !(tp->e_max > 0.0f && tp->e_max <= 1.0f))
    return fail(h, BSI_EINVAL, "e_max must be in (0, 1]");
  if (tp->flux_term && !(tp->sigma_ln_f > 0.0)) return fail(h, BSI_EINVAL, "sigma_ln_f must be > 0");
  if (!(ip->log10f_lo < ip->log10f_hi) || !(ip->log10s_lo < ip->log10s_hi) || !(ip->sigma_e > 0))
    return fail(h, BSI_EINVAL, "invalid interim prior");
  if (!e1p || !e2p || (tp->size_term && !log10s) || (tp->flux_term && !log10f))
    return fail(h, BSI_EINVAL, "sample arrays are NULL");
  return BSI_OK;
}

// Blocks of one evaluation pass over n_gal galaxies at n_pts points (four
// waves per block, one galaxy per wave at a time): about one round of
// resident workgroups over all point chunks, so that each wave runs through
// several galaxies and prefetches the next one's samples while it evaluates
// the current one.  At most 16 points the kernel forms hold 8 samples per
// lane and fit three blocks on each of the 256 compute units; otherwise two.
int shear_blocks(int n_gal, int n_pts) {
  const int chunks = (n_pts + 63) / 64;
  const int resident = n_pts <= 16 ? 768 : 512;
  return std::max(1, std::min((n_gal + 3) / 4, std::max(16, resident / chunks)));
}

ShearArgs shear_args(int32_t n_gal, int32_t K, const float* e1p, const float* e2p,
                     const float* log10s, const float* log10f, const bsi_true_prior* tp,
                     const bsi_interim* ip, int n_pts, const double* dpts, double* partial,
                     int want_grad) {
  ShearArgs a{};
  a.n_gal = n_gal;
  a.K = K;
  a.e1p = e1p;
  a.e2p = e2p;
  a.l10s = log10s ? log10s : e1p;
  a.l10f = log10f ? log10f : e1p;
  a.e_kind = tp->e_kind;
  a.e_max = tp->e_kind == BSI_E_BA14 ? 1.0f : tp->e_max;
  a.size_term = tp->size_term;
  a.flux_term = tp->flux_term;
  a.mu_lnf = tp->mu_ln_f;
  a.sig_lnf = tp->flux_term ? tp->sigma_ln_f : 1.0;
  a.log_span_s = std::log((double)ip->log10s_hi - (double)ip->log10s_lo);
  a.log_span_f = std::log((double)ip->log10f_hi - (double)ip->log10f_lo);
  a.sigma_e_interim = ip->sigma_e;
  a.n_pts = n_pts;
  a.pts = dpts;
  a.partial = partial;
  a.want_grad = want_grad;
  a.per_gal = nullptr;
  // the interim ellipticity density (eq. interim-prior, the unit-disk form) in
  // log2 units: E' coefficient log2(e) / (2 sigma0^2) and log2 of its normaliser
  // Z0 = pi (2 s^2 - 8 s^4 + 16 s^6 (1 - exp(-1 / (2 s^2))))
  const double s0 = ip->sigma_e, s2 = s0 * s0;
  const double z0 = M_PI * (2.0 * s2 - 8.0 * s2 * s2 + 16.0 * s2 * s2 * s2 * (1.0 - std::exp(-1.0 / (2.0 * s2))));
  a.b0 = (float)(1.0 / (2.0 * s2) / M_LN2);
  a.lz0 = (float)std::log2(z0);
  a.logK = std::log((double)K);
  return a;
}

}  // namespace

extern "C" {

int bsi_shear_posterior(bsi_handle h, int32_t n_gal, int32_t K, const float* e1p,
                        const float* e2p, const float* log10s, const float* log10f,
                        const bsi_true_prior* tp, const bsi_interim* ip, int32_t n_pts,
                        const double* pts, int32_t pts_on_device, double* logpost, double* grad,
                        bsi_stream stream) {
  if (!h) return BSI_EINVAL;
  h->err.clear();
  int rc = check_shear_inputs(h, n_gal, K, e1p, e2p, log10s, log10f, tp, ip);
  if (rc) return rc;
  if (n_pts < 0) return fail(h, BSI_EINVAL, "n_pts < 0");
  if (n_pts == 0) return BSI_OK;
  if (!pts || !logpost) return fail(h, BSI_EINVAL, "pts/logpost is NULL");
  (void)hipSetDevice(h->device);
  hipStream_t s = static_cast<hipStream_t>(stream);
  const bool cap = capturing(s);
  const int n_blocks = shear_blocks(n_gal, n_pts);
  const size_t pts_bytes = pts_on_device ? 0 : (size_t)n_pts * 5 * sizeof(double);
  if ((rc = prepare(h, s, cap, {{&h->pts, pts_bytes},
                                {&h->partial, (size_t)n_blocks * n_pts * 6 * sizeof(double)}},
                    stage_size({pts_bytes}))))
    return rc;
  const double* dpts = pts;
  if (!pts_on_device) {
    if ((rc = stage_upload(h, s, cap, {{h->pts.p, pts, pts_bytes}}))) return rc;
    dpts = static_cast<const double*>(h->pts.p);
  }
  const ShearArgs a = shear_args(n_gal, K, e1p, e2p, log10s, log10f, tp, ip, n_pts, dpts,
                                 static_cast<double*>(h->partial.p), grad != nullptr);
  hipError_t e = launch_shear(a, n_blocks, s);
  if (e != hipSuccess) return hip_fail(h, e, "shear launch");
  e = launch_shear_reduce(a.partial, n_blocks, n_pts, dpts, logpost, grad, s);
  if (e != hipSuccess) return hip_fail(h, e, "shear reduce launch");
  return finish(h, s, cap);
}

int bsi_shear_posterior_noalloc(bsi_handle h, int32_t n_gal, int32_t K, const float* e1p,
                                const float* e2p, const float* log10s, const float* log10f,
                                const bsi_true_prior* tp, const bsi_interim* ip, int32_t n_pts,
                                const double* pts, double* logpost, double* grad, bsi_stream stream) {
  if (!h) return BSI_EINVAL;
  h->err.clear();
  int rc = check_shear_inputs(h, n_gal, K, e1p, e2p, log10s, log10f, tp, ip);
  if (rc) return rc;
  if (n_pts < 0) return fail(h, BSI_EINVAL, "n_pts < 0");
  if (n_pts == 0) return BSI_OK;
  if (!pts || !logpost) return fail(h, BSI_EINVAL, "pts/logpost is NULL");
  const int n_blocks = shear_blocks(n_gal, n_pts);
  const size_t need = (size_t)n_blocks * n_pts * 6 * sizeof(double);
  if (need > (size_t)BSI_NOALLOC_SCRATCH_BYTES)
    return fail(h, BSI_EINVAL, "%d galaxies at %d points need %zu bytes of scratch, more than %d",
                n_gal, n_pts, need, BSI_NOALLOC_SCRATCH_BYTES);
  if (!h->scratch) return fail(h, BSI_EHIP, "device scratch unavailable");
  (void)hipSetDevice(h->device);
  hipStream_t s = static_cast<hipStream_t>(stream);
  const ShearArgs a = shear_args(n_gal, K, e1p, e2p, log10s, log10f, tp, ip, n_pts, pts,
                                 static_cast<double*>(h->scratch), grad != nullptr);
  hipError_t e = launch_shear(a, n_blocks, s);
  if (e != hipSuccess) return hip_fail(h, e, "shear launch");
  e = launch_shear_reduce(a.partial, n_blocks, n_pts, pts, logpost, grad, s);
  if (e != hipSuccess) return hip_fail(h, e, "shear reduce launch");
  return BSI_OK;
}

int bsi_shear_galaxy_loglik(bsi_handle h, int32_t n_gal, int32_t K, const float* e1p,
                            const float* e2p, const float* log10s, const float* log10f,
                            const bsi_true_prior* tp, const bsi_interim* ip, int32_t n_pts,
                            const double* pts, int32_t pts_on_device, double* ell,
                            bsi_stream stream) {
  if (!h) return BSI_EINVAL;
  h->err.clear();
  int rc = check_shear_inputs(h, n_gal, K, e1p, e2p, log10s, log10f, tp, ip);
  if (rc) return rc;
  if (n_pts < 0) return fail(h, BSI_EINVAL, "n_pts < 0");
  if (n_pts == 0 || n_gal == 0) return BSI_OK;
  if (!pts || !ell) return fail(h, BSI_EINVAL, "pts/ell is NULL");
  (void)hipSetDevice(h->device);
  hipStream_t s = static_cast<hipStream_t>(stream);
  const bool cap = capturing(s);
  const int n_blocks = shear_blocks(n_gal, n_pts);
  const size_t pts_bytes = pts_on_device ? 0 : (size_t)n_pts * 5 * sizeof(double);
  if ((rc = prepare(h, s, cap, {{&h->pts, pts_bytes},
                                {&h->partial, (size_t)n_blocks * n_pts * 6 * sizeof(double)}},
                    stage_size({pts_bytes}))))
    return rc;
  const double* dpts = pts;
  if (!pts_on_device) {
    if ((rc = stage_upload(h, s, cap, {{h->pts.p, pts, pts_bytes}}))) return rc;
    dpts = static_cast<const double*>(h->pts.p);
  }
  ShearArgs a = shear_args(n_gal, K, e1p, e2p, log10s, log10f, tp, ip, n_pts, dpts,
                           static_cast<double*>(h->partial.p), 0);
  a.per_gal = ell;
  hipError_t e = launch_shear(a, n_blocks, s);
  if (e != hipSuccess) return hip_fail(h, e, "shear launch");
  return finish(h, s, cap);
}

int bsi_shear_bias(bsi_handle h, int32_t n_gal, int32_t n_pts, const double* ell_plus,
                   const double* ell_minus, const double* gpts, double g_abs, int32_t n_boot,
                   const int32_t* counts, double* gmean, double* mc, double* stats,
                   bsi_stream stream) {
  if (!h) return BSI_EINVAL;
  h->err.clear();
  if (n_gal < 1) return fail(h, BSI_EINVAL, "n_gal must be >= 1");
  if (n_pts < 1 || n_pts > 8192) return fail(h, BSI_EINVAL, "n_pts must be 1..8192");
  if (n_boot < 0) return fail(h, BSI_EINVAL, "n_boot < 0");
  if (!(g_abs > 0.0) || !std::isfinite(g_abs)) return fail(h, BSI_EINVAL, "g_abs must be positive");
  if (!ell_plus || !ell_minus || !gpts || !stats) return fail(h, BSI_EINVAL, "ell/gpts/stats is NULL");
  if (n_boot > 0 && !counts) return fail(h, BSI_EINVAL, "counts is NULL");
  (void)hipSetDevice(h->device);
  hipStream_t s = static_cast<hipStream_t>(stream);
  const bool cap = capturing(s);
  const BiasPlan b = bias_plan(n_gal, n_pts, n_boot);
  int rc;
  if ((rc = prepare(h, s, cap, {{&h->bias_part, b.partial_doubles * sizeof(double)},
                                {&h->bias_mc, mc ? 0 : (size_t)b.R * 2 * sizeof(double)}})))
    return rc;
  double* mcp = mc ? mc : static_cast<double*>(h->bias_mc.p);
  hipError_t e = launch_bias(b, counts, ell_plus, ell_minus, n_gal, n_pts, gpts, g_abs,
                             static_cast<double*>(h->bias_part.p), gmean, mcp, stats, s);
  if (e != hipSuccess) return hip_fail(h, e, "bias launch");
  return finish(h, s, cap);
}

int bsi_shear_hmc(bsi_handle h, int32_t n_gal, int32_t K, const float* e1p, const float* e2p,
                  const float* log10s, const float* log10f, const bsi_true_prior* tp,
                  const bsi_interim* ip, const bsi_shear_hmc_cfg* cfg, const double* init,
                  double* samples, double* chain_stats, bsi_stream stream) {
  if (!h) return BSI_EINVAL;
  h->err.clear();
  int rc = check_shear_inputs(h, n_gal, K, e1p, e2p, log10s, log10f, tp, ip);
  if (rc) return rc;
  if (!cfg || !init) return fail(h, BSI_EINVAL, "cfg/init is NULL");
  const int C = cfg->n_chains;
  if (C < 1 || C > 64) return fail(h, BSI_EINVAL, "n_chains must be 1..64");
  if (cfg->n_leapfrog < 1) return fail(h, BSI_EINVAL, "n_leapfrog must be >= 1");
  if (cfg->n_warmup < 0 || cfg->n_samples < 0) return fail(h, BSI_EINVAL, "negative iteration count");
  if (!(cfg->step_size > 0.0f) || !std::isfinite(cfg->step_size))
    return fail(h, BSI_EINVAL, "step_size must be positive");
  if (cfg->adapt && !(cfg->target_accept > 0.0f && cfg->target_accept < 1.0f))
    return fail(h, BSI_EINVAL, "target_accept must be in (0, 1)");
  if (!(cfg->jitter >= 0.0f && cfg->jitter < 1.0f)) return fail(h, BSI_EINVAL, "jitter must be in [0, 1)");
  for (int j = 0; j < 5; ++j)
    if (!(cfg->inv_mass[j] > 0.0) || !std::isfinite(cfg->inv_mass[j]))
      return fail(h, BSI_EINVAL, "inv_mass entries must be positive");
  (void)hipSetDevice(h->device);
  hipStream_t s = stream ? static_cast<hipStream_t>(stream) : h->own;
  const bool cap = capturing(s);
  const int n_blocks = shear_blocks(n_gal, C);
  const size_t pts_bytes = (size_t)C * 5 * sizeof(double);
  if ((rc = prepare(h, s, cap, {{&h->pts, pts_bytes},
                                {&h->partial, (size_t)n_blocks * C * 6 * sizeof(double)},
                                {&h->shear_state, (size_t)C * sizeof(ShearChain)}},
                    stage_size({pts_bytes}))))
    return rc;
  if ((rc = stage_upload(h, s, cap, {{h->pts.p, init, pts_bytes}}))) return rc;
  hipError_t e;

  double* dpts = static_cast<double*>(h->pts.p);
  const ShearArgs sa = shear_args(n_gal, K, e1p, e2p, log10s, log10f, tp, ip, C, dpts,
                                  static_cast<double*>(h->partial.p), 1);
  ShearHmcArgs a{};
  a.state = static_cast<ShearChain*>(h->shear_state.p);
  a.pts = dpts;
  a.partial = sa.partial;
  a.n_blocks = n_blocks;
  a.C = C;
  a.L = cfg->n_leapfrog;
  a.W = cfg->n_warmup;
  a.S = cfg->n_samples;
  a.t_stop = cfg->n_warmup + cfg->n_samples;
  a.adapt = cfg->adapt;
  for (int j = 0; j < 5; ++j) a.im[j] = cfg->inv_mass[j];
  a.eps0 = cfg->step_size;
  a.delta = cfg->target_accept;
  a.jitter = cfg->jitter;
  a.mu = std::log(10.0 * (double)cfg->step_size);
  a.k0 = (uint32_t)(cfg->seed & 0xffffffffu);
  a.k1 = (uint32_t)(cfg->seed >> 32);
  a.uid_base = cfg->uid_base;
  a.samples = samples;
  a.trace = cfg->trace;

  // the potential at the start points, then one trajectory per iteration
  e = launch_shear(sa, n_blocks, s);
  if (e == hipSuccess) e = launch_shear_hmc_update(a, 1, s);
  if (e != hipSuccess) return hip_fail(h, e, "shear hmc init");
  auto trajectory = [&](hipStream_t st) -> hipError_t {
    for (int l = 0; l < a.L; ++l) {
      hipError_t x = launch_shear(sa, n_blocks, st);
      if (x == hipSuccess) x = launch_shear_hmc_update(a, 0, st);
      if (x != hipSuccess) return x;
    }
    return hipSuccess;
  };
  const int T = a.t_stop;
  if (!cap && cfg->use_graph && T > 1) {
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    e = hipStreamBeginCapture(s, hipStreamCaptureModeRelaxed);
    if (e == hipSuccess) e = trajectory(s);
    hipError_t e2 = hipStreamEndCapture(s, &graph);
    if (e == hipSuccess) e = e2;
    if (e == hipSuccess) e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    for (int k = 0; e == hipSuccess && k < T; ++k) e = hipGraphLaunch(exec, s);
    if (e != hipSuccess) {
      (void)hipStreamSynchronize(s);
      if (exec) (void)hipGraphExecDestroy(exec);
      if (graph) (void)hipGraphDestroy(graph);
      return hip_fail(h, e, "shear hmc graph");
    }
    if ((rc = keep_graph(h, exec, graph, s))) return rc;
  } else {
    for (int k = 0; k < T; ++k) {
      e = trajectory(s);
      if (e != hipSuccess) return hip_fail(h, e, "shear hmc launch");
    }
  }
  e = launch_shear_hmc_stats(a.state, C, a.S, chain_stats, s);
  if (e != hipSuccess) return hip_fail(h, e, "shear hmc stats");
  if ((rc = finish(h, s, cap))) return rc;
  if (!stream) {
    e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_fail(h, e, "shear hmc sync");
  }
  return BSI_OK;
}

int bsi_reserve(bsi_handle h, const bsi_reserve_cfg* r) {
  if (!h) return BSI_EINVAL;
  h->err.clear();
  if (!r) return fail(h, BSI_EINVAL, "cfg is NULL");
  if (r->max_stamps < 0 || r->max_shear_gal < 0 || r->max_points < 0 || r->max_chains < 0 ||
      r->max_boot < 0)
    return fail(h, BSI_EINVAL, "negative limit");
  if (r->max_stamps > 0 && (r->max_n < 8 || r->max_n > kMaxN))
    return fail(h, BSI_EUNSUPPORTED, "max_n %d outside [8, %d]", r->max_n, kMaxN);
  if (r->max_chains > 16) return fail(h, BSI_EINVAL, "max_chains must be 0..16");
  if (r->bias && (r->max_points < 1 || r->max_points > 8192))
    return fail(h, BSI_EINVAL, "bias workspace needs max_points in 1..8192");
  (void)hipSetDevice(h->device);
  hipError_t e = hipDeviceSynchronize();
  if (e != hipSuccess) return hip_fail(h, e, "reserve: device synchronisation");
  release_retired(h);
  const size_t S = (size_t)r->max_stamps;
  const size_t bins = S ? max_bins_per_stamp(r->max_n) : 0;
  const size_t N2 = (size_t)r->max_n * r->max_n;
  // shear partial sums: the largest blocks x points over every point count
  size_t partial = 0;
  const int64_t sg = std::max<int64_t>(r->max_shear_gal, 1);
  const int sgi = (int)std::min<int64_t>(sg, 1 << 30);
  for (int np = 1; np <= r->max_points; ++np)
    partial = std::max(partial, (size_t)shear_blocks(sgi, np) * np * 6 * sizeof(double));
  size_t bias_part = 0, bias_mc = 0;
  if (r->bias) {
    bias_part = std::max(bias_plan(std::max(sgi, 1), r->max_points, r->max_boot).partial_doubles,
                         bias_plan(1 << 30, r->max_points, r->max_boot).partial_doubles) * sizeof(double);
    bias_mc = (size_t)(r->max_boot + 1) * 2 * sizeof(double);
  }
  const size_t stage = std::max(bsi_host::stage_size({S * 4, S * 8, S * 8, r->weighted ? S * 4 : 0}),
                                bsi_host::stage_size({(size_t)r->max_points * 5 * sizeof(double)}));
  struct { DevBuf* b; size_t n; } want[] = {
      {&h->gidx, S * 4}, {&h->ggidx, r->weighted ? S * 4 : 0}, {&h->off, S * 8}, {&h->bin_off, S * 8},
      {&h->dh, S * bins * sizeof(float2)}, {&h->sqw, r->weighted ? S * bins * sizeof(float) : 0},
      {&h->state, S * (size_t)r->max_chains * sizeof(ChainState)},
      {&h->model, r->pixel_method ? S * N2 * sizeof(double) : 0},
      {&h->chi2, r->pixel_method ? S * sizeof(double) : 0},
      {&h->pts, (size_t)r->max_points * 5 * sizeof(double)}, {&h->partial, partial},
      {&h->shear_state, (size_t)r->max_points * sizeof(ShearChain)},
      {&h->bias_part, bias_part}, {&h->bias_mc, bias_mc}};
  int rc;
  for (auto& w : want)
    if ((rc = bsi_host::grow(h, *w.b, w.n))) return rc;
  if ((rc = bsi_host::grow_stage(h, stage))) return rc;
  release_retired(h);   // the buffers just replaced were idle
  h->pending = false;
  return BSI_OK;
}

int bsi_ess(bsi_handle h, int32_t n_gal, int32_t n_chains, int32_t n_samples, int32_t n_par,
            const float* samples, float* ess, float* rhat, float* rhat_split, bsi_stream stream) {
  if (!h) return BSI_EINVAL;
  h->err.clear();
  if (n_gal < 0 || n_chains < 1 || n_chains > 16 || n_samples < 4 || n_par < 1)
    return fail(h, BSI_EINVAL, "invalid ESS shape");
  if ((size_t)n_chains * n_samples * sizeof(double) + 256 * sizeof(double) > 150 * 1024)
    return fail(h, BSI_EUNSUPPORTED, "n_chains * n_samples too large for LDS");
  if (n_gal == 0) return BSI_OK;
  if (!samples || (!ess && !rhat && !rhat_split)) return fail(h, BSI_EINVAL, "NULL samples or outputs");
  (void)hipSetDevice(h->device);
  hipError_t e = launch_ess(n_gal, n_chains, n_samples, n_par, samples, ess, rhat, rhat_split,
                            static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return hip_fail(h, e, "ess launch");
  return BSI_OK;   // uses no handle workspace
}

}  // extern "C"
