// Host side of the request server (slot-based continuous batching of the
// per-galaxy sampler).  Device memory is one allocation of the HBM budget:
// per-slot arrays (scalars, start positions, chain states, stored samples)
// for max_slots requests, and an arena from which each admitted request
// takes its stamp copy and data spectrum (first fit, coalescing free list).
// Scheduling is host-side and deterministic: a request admitted before
// advance k runs iterations from advance k on and is finished once
// n_warmup + n_samples iterations have been enqueued for it.  With an ESS
// target the device decides instead: each request's chains stop at its next
// checkpoint, a check kernel enqueued after every advance finishes it there
// or moves the checkpoint on, and a poll reads the finished requests back.
#include "bsi.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <deque>
#include <map>
#include <vector>

#include "bsi_kernels.h"
#include "ctx.h"
#include "kspace.h"

using namespace bsi;
using namespace bsi_host;

namespace {

constexpr int64_t kAlign = 256;
constexpr int kMaxSizes = 16;

int64_t align_up(int64_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

// First-fit allocator over [0, n) with coalescing of freed extents.
class Arena {
 public:
  void reset(int64_t n) {
    free_.clear();
    if (n > 0) free_[0] = n;
    size_ = n;
  }
  int64_t alloc(int64_t n) {
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second < n) continue;
      const int64_t off = it->first, rest = it->second - n;
      free_.erase(it);
      if (rest > 0) free_[off + n] = rest;
      return off;
    }
    return -1;
  }
  void release(int64_t off, int64_t n) {
    auto next = free_.lower_bound(off);
    if (next != free_.end() && off + n == next->first) {
      n += next->second;
      next = free_.erase(next);
    }
    if (next != free_.begin()) {
      auto prev = std::prev(next);
      if (prev->first + prev->second == off) {
        prev->second += n;
        return;
      }
    }
    free_[off] = n;
  }
  int64_t free_bytes() const {
    int64_t s = 0;
    for (const auto& kv : free_) s += kv.second;
    return s;
  }
  int64_t largest() const {
    int64_t m = 0;
    for (const auto& kv : free_) m = std::max(m, kv.second);
    return m;
  }
  int64_t size() const { return size_; }

 private:
  std::map<int64_t, int64_t> free_;
  int64_t size_ = 0;
};

struct Slot {
  bool used = false;
  bool done = false;
  uint64_t id = 0;
  uint64_t seq = 0;       // admission order
  int cls = -1;
  int t = 0;              // iterations enqueued so far
  int64_t arena_off = 0;  // bytes
  int64_t arena_len = 0;
};

struct SizeClass {
  int N;
  int P;                           // slot plan (the handle's at creation)
  int W;                           // waves per chain of the trajectory kernel
  bool mfma;                       // data transform on the matrix cores (the handle's choice)
  int64_t stamp_bytes, bin_bytes;
  hipEvent_t ev_beg = nullptr, ev_end = nullptr;   // this size's last advance launch
  double tau = -1.0;               // measured milliseconds per iteration (-1: unknown)
  int last_k = 0;                  // iterations of the last timed launch (0: none pending)
  std::vector<int32_t> fresh;      // slots admitted since the last advance
  std::vector<int32_t> resident;   // running slots
};

}  // namespace

struct bsi_slots_s {
  bsi_handle h = nullptr;
  hipStream_t s = nullptr;
  bsi_slots_cfg cfg{};
  int C = 1, L = 1, T = 0, S = 0;
  bool ess = false;               // ESS-targeted requests (device-side completion)
  uint64_t n_admitted = 0;
  std::vector<SizeClass> cls;
  int max_slots = 0;
  int64_t fixed_bytes = 0;
  // device
  void* block = nullptr;
  int64_t block_bytes = 0;
  SlotArrays arr{};
  ChainState* state = nullptr;
  float* samples = nullptr;
  char* arena = nullptr;
  Arena alloc;
  // uploads: admission records, start positions and per-class slot lists
  char* pinned = nullptr;
  char* dev_up = nullptr;
  int64_t up_bytes = 0;
  hipEvent_t ev_up = nullptr;
  bool up_pending = false;
  int32_t* rd = nullptr;          // pinned readback of the done queue: count, then entries
  // bookkeeping
  std::vector<Slot> slots;
  std::vector<int32_t> free_ids;
  std::vector<SlotRecord> rec;
  std::vector<float> rec_init;
  std::deque<int32_t> finished;
};

namespace {

int class_of(const bsi_slots_s* sv, int N) {
  for (size_t i = 0; i < sv->cls.size(); ++i)
    if (sv->cls[i].N == N) return (int)i;
  return -1;
}

HmcArgs base_args(const bsi_slots_s* sv) {
  const bsi_hmc_cfg& c = sv->cfg.hmc;
  const bsi_interim& ip = sv->cfg.interim;
  HmcArgs a{};
  a.dh = reinterpret_cast<const float2*>(sv->arena);
  a.bin_off = sv->arr.bin_off;
  a.psf = sv->arr.psf;
  a.sigma = sv->arr.sigma;
  a.ref_xy = sv->arr.ref_xy;
  a.init = sv->arr.init;
  a.inv_mass = nullptr;
  a.uid_gal = sv->arr.uid;
  a.state = sv->state;
  a.samples = sv->samples;
  a.trace = nullptr;
  a.rscale = profile_rscale(sv->cfg.profile, sv->cfg.pixel_scale, sv->cfg.spergel_nu);
  a.pscale_inv = 1.0f / sv->cfg.pixel_scale;
  a.prof = sv->cfg.profile;
  a.nu = sv->cfg.spergel_nu;
  a.C = sv->C;
  a.L = sv->L;
  a.W = c.n_warmup;
  a.S = c.n_samples;
  a.adapt = c.adapt;
  a.metric = c.metric;
  a.eps0 = c.step_size;
  a.delta = c.target_accept;
  a.jitter = c.jitter;
  a.mu = (float)std::log(10.0 * (double)c.step_size);
  a.k0 = (uint32_t)(c.seed & 0xffffffffu);
  a.k1 = (uint32_t)(c.seed >> 32);
  a.uid_base = 0;
  a.lf_lo = ip.log10f_lo;
  a.lf_hi = ip.log10f_hi;
  a.ls_lo = ip.log10s_lo;
  a.ls_hi = ip.log10s_hi;
  a.sigma_d = ip.sigma_d;
  a.sigma_e = ip.sigma_e;
  a.t_stop = sv->T;
  a.t_stop_gal = sv->ess ? sv->arr.stop : nullptr;
  a.wpc = 1;
  return a;
}

}  // namespace

extern "C" {

int bsi_slots_create(bsi_handle h, const bsi_slots_cfg* cfg, bsi_stream stream, bsi_slots* out) {
  if (!h) return BSI_EINVAL;
  h->err.clear();
  if (!out || !cfg) return fail(h, BSI_EINVAL, "cfg/out is NULL");
  *out = nullptr;
  if (cfg->n_sizes < 1 || cfg->n_sizes > kMaxSizes || !cfg->sizes)
    return fail(h, BSI_EINVAL, "n_sizes must be 1..%d with sizes given", kMaxSizes);
  const bsi_hmc_cfg& hc = cfg->hmc;
  if (hc.n_chains < 1 || hc.n_chains > 16) return fail(h, BSI_EINVAL, "n_chains must be 1..16");
  if (hc.n_leapfrog < 1 || hc.n_warmup < 0 || hc.n_samples < 1)
    return fail(h, BSI_EINVAL, "need n_leapfrog >= 1, n_warmup >= 0, n_samples >= 1");
  if (!(hc.step_size > 0.0f) || !std::isfinite(hc.step_size))
    return fail(h, BSI_EINVAL, "step_size must be positive");
  if (hc.adapt && !(hc.target_accept > 0.0f && hc.target_accept < 1.0f))
    return fail(h, BSI_EINVAL, "target_accept must be in (0, 1)");
  if (!(hc.jitter >= 0.0f && hc.jitter < 1.0f)) return fail(h, BSI_EINVAL, "jitter must be in [0, 1)");
  if (hc.metric != BSI_METRIC_GIVEN && hc.metric != BSI_METRIC_FISHER)
    return fail(h, BSI_EINVAL, "unknown metric %d", hc.metric);
  if (hc.waves_per_chain < 0 || hc.waves_per_chain > 4)
    return fail(h, BSI_EINVAL, "waves_per_chain must be 0..4");
  const bsi_interim& ip = cfg->interim;
  if (!(ip.log10f_lo < ip.log10f_hi) || !(ip.log10s_lo < ip.log10s_hi) || !(ip.sigma_d > 0) ||
      !(ip.sigma_e > 0))
    return fail(h, BSI_EINVAL, "invalid interim prior");
  if (!(cfg->pixel_scale > 0.0f)) return fail(h, BSI_EINVAL, "pixel_scale must be positive");
  if (cfg->hmc.sampler != BSI_SAMPLER_HMC)
    return fail(h, BSI_EUNSUPPORTED, "the request server runs fixed-length HMC only");
  if (cfg->profile != BSI_PROFILE_EXPONENTIAL && cfg->profile != BSI_PROFILE_GAUSSIAN &&
      cfg->profile != BSI_PROFILE_SPERGEL)
    return fail(h, BSI_EINVAL, "unknown profile %d", cfg->profile);
  if (cfg->profile == BSI_PROFILE_SPERGEL &&
      !(cfg->spergel_nu >= BSI_SPERGEL_NU_MIN && cfg->spergel_nu <= BSI_SPERGEL_NU_MAX))
    return fail(h, BSI_EINVAL, "Spergel index %g outside [%g, %g]", (double)cfg->spergel_nu,
                (double)BSI_SPERGEL_NU_MIN, (double)BSI_SPERGEL_NU_MAX);
  if (cfg->hbm_budget <= 0 || cfg->max_slots < 0) return fail(h, BSI_EINVAL, "invalid budget/max_slots");
  if (!(cfg->ess_target >= 0.0f) || !std::isfinite(cfg->ess_target))
    return fail(h, BSI_EINVAL, "ess_target must be finite and >= 0");
  if (cfg->ess_target > 0.0f && cfg->ess_every < 4) return fail(h, BSI_EINVAL, "ess_every must be >= 4");
  if (cfg->ess_target > 0.0f && slots_check_lds_bytes(hc.n_chains, hc.n_samples) > 150 * 1024)
    return fail(h, BSI_EUNSUPPORTED, "n_chains * n_samples too large for the on-device ESS check");

  bsi_slots_s* sv = new bsi_slots_s();
  sv->h = h;
  sv->s = static_cast<hipStream_t>(stream);
  sv->cfg = *cfg;
  sv->cfg.sizes = nullptr;
  sv->C = hc.n_chains;
  sv->L = hc.n_leapfrog;
  sv->S = hc.n_samples;
  sv->T = hc.n_warmup + hc.n_samples;
  sv->ess = cfg->ess_target > 0.0f;
  int64_t min_var = INT64_MAX, max_var = 0;
  for (int i = 0; i < cfg->n_sizes; ++i) {
    const int N = cfg->sizes[i];
    if (N < 8 || N > kMaxN || class_of(sv, N) >= 0) {
      delete sv;
      return fail(h, BSI_EINVAL, "sizes must be distinct and in 8..%d", kMaxN);
    }
    SizeClass c;
    c.N = N;
    c.P = h->plan_P[N] > 0 ? h->plan_P[N] : make_slot_plan(N).P;
    c.W = hmc_split_waves(N, sv->C, c.P, cfg->profile, hc.waves_per_chain);
    c.mfma = transform_of(h, N) == BSI_TRANSFORM_MFMA;
    if (hmc_lds_bytes(N, sv->C, c.P, c.W) > 160 * 1024) {
      delete sv;
      return fail(h, BSI_EUNSUPPORTED, "N = %d with %d chains exceeds LDS", N, hc.n_chains);
    }
    c.stamp_bytes = align_up((int64_t)N * N * 4);
    c.bin_bytes = align_up((int64_t)make_slot_plan_p(N, c.P).nbins * 8);
    min_var = std::min(min_var, c.stamp_bytes + c.bin_bytes);
    max_var = std::max(max_var, c.stamp_bytes + c.bin_bytes);
    sv->cls.push_back(c);
  }
  const int64_t C = sv->C;
  // per slot: off, bin_off, psf, sigma, ref_xy, uid, init, states, samples,
  // stop, ndraw, done queue entry
  sv->fixed_bytes = 8 + 8 + 4 + 4 + 8 + 8 + C * 24 + C * (int64_t)sizeof(ChainState) +
                    C * sv->S * 24 + 12;
  const int64_t budget = cfg->hbm_budget;
  int64_t ms = cfg->max_slots > 0 ? cfg->max_slots : budget / (sv->fixed_bytes + min_var);
  ms = std::min<int64_t>(ms, 1 << 22);
  // array section, each array 256-byte aligned
  auto arrays_bytes = [&](int64_t n) {
    return align_up(n * 8) * 3 + align_up(n * 4) * 2 + align_up(n * 8) + align_up(n * C * 24) +
           align_up(n * C * (int64_t)sizeof(ChainState)) + align_up(n * C * sv->S * 24) +
           align_up(n * 4) * 3 + align_up(4) + align_up(n * 24) + align_up(n * 4);
  };
  if (ms < 1 || arrays_bytes(ms) + max_var > budget) {
    delete sv;
    return fail(h, BSI_EINVAL, "hbm_budget %lld cannot hold one request of every size with "
                "max_slots %lld", (long long)budget, (long long)ms);
  }
  sv->max_slots = (int)ms;
  const int64_t arena_bytes = (budget - arrays_bytes(ms)) / kAlign * kAlign;
  sv->block_bytes = arrays_bytes(ms) + arena_bytes;
  hipSetDevice(h->device);
  hipError_t e = hipMalloc(&sv->block, (size_t)sv->block_bytes);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    delete sv;
    return fail(h, BSI_ENOMEM, "server allocation of %lld bytes failed", (long long)budget);
  }
  char* p = static_cast<char*>(sv->block);
  auto take = [&](int64_t bytes) {
    char* q = p;
    p += align_up(bytes);
    return q;
  };
  sv->arr.off = reinterpret_cast<int64_t*>(take(ms * 8));
  sv->arr.bin_off = reinterpret_cast<int64_t*>(take(ms * 8));
  sv->arr.uid = reinterpret_cast<uint64_t*>(take(ms * 8));
  sv->arr.psf = reinterpret_cast<float*>(take(ms * 4));
  sv->arr.sigma = reinterpret_cast<float*>(take(ms * 4));
  sv->arr.ref_xy = reinterpret_cast<float*>(take(ms * 8));
  sv->arr.init = reinterpret_cast<float*>(take(ms * C * 24));
  sv->state = reinterpret_cast<ChainState*>(take(ms * C * (int64_t)sizeof(ChainState)));
  sv->samples = reinterpret_cast<float*>(take(ms * C * sv->S * 24));
  sv->arr.stop = reinterpret_cast<int32_t*>(take(ms * 4));
  sv->arr.ndraw = reinterpret_cast<int32_t*>(take(ms * 4));
  sv->arr.done_q = reinterpret_cast<int32_t*>(take(ms * 4));
  sv->arr.done_n = reinterpret_cast<int32_t*>(take(4));
  sv->arr.ess6 = reinterpret_cast<float*>(take(ms * 24));
  sv->arr.ess_cnt = reinterpret_cast<int32_t*>(take(ms * 4));
  sv->arena = p;
  sv->alloc.reset(arena_bytes);
  // upload staging: records, start positions, two slot lists per class, and
  // the list of all resident slots (ESS checks)
  sv->up_bytes = align_up(ms * (int64_t)sizeof(SlotRecord)) + align_up(ms * C * 24) +
                 align_up(ms * 4) * (2 * (int64_t)sv->cls.size() + 1);
  e = hipHostMalloc(reinterpret_cast<void**>(&sv->pinned), (size_t)sv->up_bytes, hipHostMallocDefault);
  if (e == hipSuccess)
    e = hipHostMalloc(reinterpret_cast<void**>(&sv->rd), (size_t)(ms + 1) * 4, hipHostMallocDefault);
  if (e == hipSuccess) e = hipMemsetAsync(sv->arr.done_n, 0, 4, sv->s);
  if (e == hipSuccess) e = hipMalloc(reinterpret_cast<void**>(&sv->dev_up), (size_t)sv->up_bytes);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&sv->ev_up, hipEventDisableTiming);
  for (SizeClass& k : sv->cls) {
    if (e == hipSuccess) e = hipEventCreate(&k.ev_beg);
    if (e == hipSuccess) e = hipEventCreate(&k.ev_end);
  }
  if (e != hipSuccess) {
    (void)hipGetLastError();
    bsi_slots_destroy(sv);
    return fail(h, BSI_ENOMEM, "server staging allocation failed");
  }
  sv->slots.assign((size_t)ms, Slot{});
  sv->free_ids.reserve((size_t)ms);
  for (int64_t i = ms - 1; i >= 0; --i) sv->free_ids.push_back((int32_t)i);
  *out = sv;
  return BSI_OK;
}

void bsi_slots_destroy(bsi_slots sv) {
  if (!sv) return;
  (void)hipSetDevice(sv->h->device);
  if (sv->s) (void)hipStreamSynchronize(sv->s);
  else (void)hipDeviceSynchronize();
  if (sv->ev_up) (void)hipEventDestroy(sv->ev_up);
  for (SizeClass& k : sv->cls) {
    if (k.ev_beg) (void)hipEventDestroy(k.ev_beg);
    if (k.ev_end) (void)hipEventDestroy(k.ev_end);
  }
  if (sv->dev_up) (void)hipFree(sv->dev_up);
  if (sv->pinned) (void)hipHostFree(sv->pinned);
  if (sv->rd) (void)hipHostFree(sv->rd);
  if (sv->block) (void)hipFree(sv->block);
  delete sv;
}

int bsi_slots_footprint(bsi_slots sv, int32_t n, int64_t* bytes) {
  if (!sv || !bytes) return BSI_EINVAL;
  const int c = class_of(sv, n);
  if (c < 0) return fail(sv->h, BSI_EINVAL, "stamp side %d is not served", n);
  *bytes = sv->fixed_bytes + sv->cls[c].stamp_bytes + sv->cls[c].bin_bytes;
  return BSI_OK;
}

int bsi_slots_admit(bsi_slots sv, const bsi_request* r, int32_t* admitted) {
  if (!sv) return BSI_EINVAL;
  bsi_handle h = sv->h;
  h->err.clear();
  if (!r || !admitted) return fail(h, BSI_EINVAL, "request/admitted is NULL");
  *admitted = 0;
  const int c = class_of(sv, r->n);
  if (c < 0) return fail(h, BSI_EINVAL, "stamp side %d is not served", r->n);
  if (!r->stamp || !r->init) return fail(h, BSI_EINVAL, "stamp/init is NULL");
  if (!(r->psf_fwhm > 0.0f) || !(r->sigma > 0.0f) || !std::isfinite(r->ref_x) ||
      !std::isfinite(r->ref_y))
    return fail(h, BSI_EINVAL, "psf_fwhm and sigma must be positive, ref finite");
  if (sv->free_ids.empty()) return BSI_OK;
  const SizeClass& k = sv->cls[c];
  const int64_t len = k.stamp_bytes + k.bin_bytes;
  const int64_t off = sv->alloc.alloc(len);
  if (off < 0) return BSI_OK;
  const int32_t slot = sv->free_ids.back();
  sv->free_ids.pop_back();
  Slot& s = sv->slots[slot];
  s = Slot{};
  s.used = true;
  s.id = r->id;
  s.seq = sv->n_admitted++;
  s.cls = c;
  s.arena_off = off;
  s.arena_len = len;
  SlotRecord rec{};
  rec.slot = slot;
  rec.N = r->n;
  rec.psf = r->psf_fwhm;
  rec.sigma = r->sigma;
  rec.refx = r->ref_x;
  rec.refy = r->ref_y;
  rec.uid = r->id * (uint64_t)sv->C;
  rec.src = (uint64_t)reinterpret_cast<uintptr_t>(r->stamp);
  rec.off = off / 4;
  rec.bin_off = (off + k.stamp_bytes) / 8;
  sv->rec.push_back(rec);
  sv->rec_init.insert(sv->rec_init.end(), r->init, r->init + sv->C * 6);
  sv->cls[c].fresh.push_back(slot);
  *admitted = 1;
  return BSI_OK;
}

int bsi_slots_admit_many(bsi_slots sv, int32_t n, const bsi_request* reqs, int32_t* n_admitted) {
  if (!sv) return BSI_EINVAL;
  if (!n_admitted || n < 0 || (n > 0 && !reqs)) return fail(sv->h, BSI_EINVAL, "bad admit_many arguments");
  *n_admitted = 0;
  for (int32_t i = 0; i < n; ++i) {
    int32_t ok = 0;
    const int rc = bsi_slots_admit(sv, reqs + i, &ok);
    if (rc) return rc;
    if (!ok) break;
    *n_admitted = i + 1;
  }
  return BSI_OK;
}

int bsi_slots_advance(bsi_slots sv, int32_t n_iter) {
  if (!sv) return BSI_EINVAL;
  bsi_handle h = sv->h;
  h->err.clear();
  if (n_iter < 1) return fail(h, BSI_EINVAL, "n_iter must be >= 1");
  hipSetDevice(h->device);
  hipError_t e = hipSuccess;
  // the staging buffer is reused: the previous upload must have been copied
  if (sv->up_pending) {
    e = hipEventSynchronize(sv->ev_up);
    if (e != hipSuccess) return hip_fail(h, e, "staging wait");
    sv->up_pending = false;
  }
  const int n_new = (int)sv->rec.size();
  const int C = sv->C;
  char* hp = sv->pinned;
  int64_t pos = 0;
  auto place = [&](const void* src, int64_t bytes) {
    const int64_t at = pos;
    if (bytes > 0) std::memcpy(hp + at, src, (size_t)bytes);
    pos += align_up(bytes);
    return at;
  };
  const int64_t rec_at = place(sv->rec.data(), (int64_t)n_new * (int64_t)sizeof(SlotRecord));
  const int64_t init_at = place(sv->rec_init.data(), (int64_t)n_new * C * 24);
  std::vector<int64_t> fresh_at(sv->cls.size()), res_at(sv->cls.size());
  std::vector<int32_t> all_res;
  for (size_t i = 0; i < sv->cls.size(); ++i) {
    SizeClass& k = sv->cls[i];
    k.resident.insert(k.resident.end(), k.fresh.begin(), k.fresh.end());
    fresh_at[i] = place(k.fresh.data(), (int64_t)k.fresh.size() * 4);
    res_at[i] = place(k.resident.data(), (int64_t)k.resident.size() * 4);
    if (sv->ess) all_res.insert(all_res.end(), k.resident.begin(), k.resident.end());
  }
  const int64_t all_at = place(all_res.data(), (int64_t)all_res.size() * 4);
  if (pos > 0) {
    e = hipMemcpyAsync(sv->dev_up, hp, (size_t)pos, hipMemcpyHostToDevice, sv->s);
    if (e == hipSuccess) e = hipEventRecord(sv->ev_up, sv->s);
    if (e != hipSuccess) return hip_fail(h, e, "staging upload");
    sv->up_pending = true;
  }
  const int every = sv->cfg.ess_every;
  const int stop0 = sv->cfg.hmc.n_warmup + (sv->ess ? std::min(every, sv->S) : sv->S);
  e = launch_slots_scatter(reinterpret_cast<const SlotRecord*>(sv->dev_up + rec_at),
                           reinterpret_cast<const float*>(sv->dev_up + init_at), n_new, C, stop0,
                           sv->arr, reinterpret_cast<float*>(sv->arena), sv->s);
  if (e != hipSuccess) return hip_fail(h, e, "admission scatter");
  std::vector<int> active;
  for (size_t i = 0; i < sv->cls.size(); ++i)
    if (!sv->cls[i].resident.empty()) active.push_back((int)i);
  // iterations per size: n_iter, or balanced by the measured per-iteration times
  std::vector<int> iters(sv->cls.size(), n_iter);
  if (sv->cfg.pace) {
    double tmax = 0.0;
    for (int i : active) tmax = std::max(tmax, sv->cls[i].tau);
    for (int i : active) {
      const double tau = sv->cls[i].tau;
      if (tau > 0.0 && tmax > 0.0)
        iters[i] = (int)std::min<double>(64.0 * n_iter, std::max(1.0, std::round(n_iter * tmax / tau)));
    }
  }
  const HmcArgs base = base_args(sv);
  e = fork_join(h, sv->s, (int)active.size(), [&](int j, hipStream_t st) -> hipError_t {
    const int i = active[j];
    const SizeClass& k = sv->cls[i];
    const int32_t* fresh = reinterpret_cast<const int32_t*>(sv->dev_up + fresh_at[i]);
    const int32_t* res = reinterpret_cast<const int32_t*>(sv->dev_up + res_at[i]);
    hipError_t x = hipSuccess;
    if (!k.fresh.empty()) {
      x = launch_stamp_dft(k.mfma, reinterpret_cast<const float*>(sv->arena), nullptr, fresh,
                           (int)k.fresh.size(), sv->arr.off, sv->arr.bin_off, k.N, k.P,
                           reinterpret_cast<float2*>(sv->arena), nullptr, st);
      if (x != hipSuccess) return x;
      HmcArgs a = base;
      a.N = k.N;
      a.P = k.P;
      a.gidx = fresh;
      a.n_gal = (int)k.fresh.size();
      a.n_steps = 0;
      x = launch_hmc_init(a, a.n_gal, st);
      if (x != hipSuccess) return x;
    }
    HmcArgs a = base;
    a.N = k.N;
    a.P = k.P;
    a.wpc = k.W;
    a.gidx = res;
    a.n_gal = (int)k.resident.size();
    a.n_steps = iters[i] * sv->L;
    if (sv->cfg.pace && (x = hipEventRecord(k.ev_beg, st)) != hipSuccess) return x;
    x = launch_hmc_advance(a, a.n_gal, st);
    if (x == hipSuccess && sv->cfg.pace) x = hipEventRecord(k.ev_end, st);
    return x;
  }, [&](int j) {
    // a launch's duration follows one request's chain (the requests of a
    // size run side by side): its bins per wave, times its iterations
    const SizeClass& k = sv->cls[active[j]];
    return (double)k.N * k.N / k.W * iters[active[j]];
  });
  if (e != hipSuccess) return hip_fail(h, e, "advance launch");
  if (sv->ess) {
    // checks at the requests' stops (one launch over every resident request);
    // finished requests are read back by a poll
    e = launch_slots_check(reinterpret_cast<const int32_t*>(sv->dev_up + all_at), (int)all_res.size(), C,
                           sv->cfg.hmc.n_warmup, sv->S, every, sv->cfg.ess_target, sv->state,
                           sv->samples, sv->arr, sv->s);
    if (e != hipSuccess) return hip_fail(h, e, "ESS check launch");
    for (SizeClass& k : sv->cls) {
      k.fresh.clear();
      if (sv->cfg.pace && !k.resident.empty()) k.last_k = iters[&k - sv->cls.data()];
    }
    sv->rec.clear();
    sv->rec_init.clear();
    return BSI_OK;
  }
  // bookkeeping: every resident request got its size's iterations (or what it had left)
  for (size_t i = 0; i < sv->cls.size(); ++i) {
    SizeClass& k = sv->cls[i];
    k.fresh.clear();
    if (sv->cfg.pace && !k.resident.empty()) k.last_k = iters[i];
    std::vector<int32_t> keep;
    keep.reserve(k.resident.size());
    for (int32_t slot : k.resident) {
      Slot& s = sv->slots[slot];
      s.t = std::min(sv->T, s.t + iters[i]);
      if (s.t >= sv->T) {
        s.done = true;
        sv->finished.push_back(slot);
      } else {
        keep.push_back(slot);
      }
    }
    k.resident.swap(keep);
  }
  sv->rec.clear();
  sv->rec_init.clear();
  return BSI_OK;
}

int bsi_slots_poll(bsi_slots sv, int32_t* n_finished) {
  if (!sv) return BSI_EINVAL;
  bsi_handle h = sv->h;
  h->err.clear();
  hipSetDevice(h->device);
  hipError_t e = sv->s ? hipStreamSynchronize(sv->s) : hipDeviceSynchronize();
  if (e != hipSuccess) return hip_fail(h, e, "server sync");
  sv->up_pending = false;
  // pacing: per-iteration time of each size's last launch
  for (SizeClass& k : sv->cls) {
    if (k.last_k <= 0) continue;
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, k.ev_beg, k.ev_end) == hipSuccess && ms > 0.f) {
      const double t = (double)ms / (double)k.last_k;
      k.tau = k.tau < 0.0 ? t : 0.5 * (k.tau + t);
    } else {
      (void)hipGetLastError();
    }
    k.last_k = 0;
  }
  if (sv->ess) {
    e = hipMemcpy(sv->rd, sv->arr.done_n, 4, hipMemcpyDeviceToHost);
    const int n = e == hipSuccess ? sv->rd[0] : 0;
    if (e == hipSuccess && n > 0)
      e = hipMemcpy(sv->rd + 1, sv->arr.done_q, (size_t)n * 4, hipMemcpyDeviceToHost);
    if (e == hipSuccess && n > 0) e = hipMemsetAsync(sv->arr.done_n, 0, 4, sv->s);
    if (e != hipSuccess) return hip_fail(h, e, "finished-request readback");
    if (n > 0) {
      // the queue's order comes from atomics: hand out in admission order
      std::vector<int32_t> got(sv->rd + 1, sv->rd + 1 + n);
      std::sort(got.begin(), got.end(),
                [&](int32_t a, int32_t b) { return sv->slots[a].seq < sv->slots[b].seq; });
      for (int32_t slot : got) {
        sv->slots[slot].done = true;
        sv->finished.push_back(slot);
      }
      for (SizeClass& k : sv->cls) {
        std::vector<int32_t> keep;
        keep.reserve(k.resident.size());
        for (int32_t slot : k.resident)
          if (!sv->slots[slot].done) keep.push_back(slot);
        k.resident.swap(keep);
      }
    }
  }
  if (n_finished) *n_finished = (int32_t)sv->finished.size();
  return BSI_OK;
}

int bsi_slots_harvest(bsi_slots sv, int32_t max, uint64_t* ids, float* samples,
                      float* chain_stats, uint32_t* status, int32_t* n_draws, int32_t* n_out) {
  if (!sv) return BSI_EINVAL;
  bsi_handle h = sv->h;
  h->err.clear();
  if (!n_out || max < 0 || (max > 0 && !ids)) return fail(h, BSI_EINVAL, "bad harvest arguments");
  *n_out = 0;
  int rc = bsi_slots_poll(sv, nullptr);
  if (rc) return rc;
  hipError_t e = hipSuccess;
  const int n = (int)std::min<size_t>((size_t)max, sv->finished.size());
  if (n == 0) return BSI_OK;
  std::vector<int32_t> list(sv->finished.begin(), sv->finished.begin() + n);
  if (samples || chain_stats || status || n_draws) {
    std::memcpy(sv->pinned, list.data(), (size_t)n * 4);
    e = hipMemcpyAsync(sv->dev_up, sv->pinned, (size_t)n * 4, hipMemcpyHostToDevice, sv->s);
    if (e == hipSuccess)
      e = launch_slots_gather(reinterpret_cast<const int32_t*>(sv->dev_up), n, sv->C, sv->S,
                              sv->state, sv->samples, sv->ess ? sv->arr.ndraw : nullptr, samples,
                              chain_stats, status, n_draws, sv->s);
    if (e == hipSuccess) e = sv->s ? hipStreamSynchronize(sv->s) : hipDeviceSynchronize();
    if (e != hipSuccess) return hip_fail(h, e, "harvest gather");
  }
  for (int j = 0; j < n; ++j) {
    Slot& s = sv->slots[list[j]];
    ids[j] = s.id;
    sv->alloc.release(s.arena_off, s.arena_len);
    s = Slot{};
    sv->free_ids.push_back(list[j]);
  }
  sv->finished.erase(sv->finished.begin(), sv->finished.begin() + n);
  *n_out = n;
  return BSI_OK;
}

int bsi_slots_get_info(bsi_slots sv, bsi_slots_info* info) {
  if (!sv || !info) return BSI_EINVAL;
  bsi_slots_info o{};
  o.max_slots = sv->max_slots;
  o.resident = sv->max_slots - (int)sv->free_ids.size();
  o.finished = (int)sv->finished.size();
  o.pending = (int)sv->rec.size();
  o.budget = sv->block_bytes;
  o.slot_fixed_bytes = sv->fixed_bytes;
  o.arena_bytes = sv->alloc.size();
  o.arena_free = sv->alloc.free_bytes();
  o.arena_largest_free = sv->alloc.largest();
  *info = o;
  return BSI_OK;
}

}  // extern "C"
