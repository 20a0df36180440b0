// Per-stamp-side choices held by a handle, explicit or measured on the
// device: the trajectory kernel's slot plan (bsi_set_plan, bsi_autotune) and
// the render transform (bsi_set_transform, bsi_autotune_transform).
#include "bsi.h"

#include <hip/hip_runtime.h>

#include <unistd.h>

#include <algorithm>
#include <cerrno>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <sstream>
#include <string>
#include <vector>

#include "bsi_kernels.h"
#include "ctx.h"
#include "kspace.h"

using namespace bsi;
using namespace bsi_host;

namespace {

bool supported_p(int P) {
  for (int k : kPlanP)
    if (k == P) return true;
  return false;
}

// Candidate plans of side N, the default first: the specialised ones if
// any, else the supported P within 10 % of the fewest slots (at most three,
// fewest slots first).
std::vector<int> candidates(int N) {
  std::vector<int> out{make_slot_plan(N).P};
  for (const int* p = hmc_fixed_plans(N); *p; ++p)
    if (*p != out[0]) out.push_back(*p);
  if (out.size() > 1) return out;
  const int best = make_slot_plan(N).nslots;
  std::vector<std::pair<int, int>> c;
  for (int P : kPlanP)
    if (plan_valid(N, P) && make_slot_plan_p(N, P).nslots * 10 <= best * 11)
      c.push_back({make_slot_plan_p(N, P).nslots, P});
  std::sort(c.begin(), c.end());
  for (size_t i = 0; i < c.size() && out.size() < 3; ++i)
    if (c[i].second != out[0]) out.push_back(c[i].second);
  return out;
}

struct Scratch {
  std::vector<void*> bufs;
  hipError_t err = hipSuccess;
  template <typename T>
  T* get(size_t n) {
    void* p = nullptr;
    if (err == hipSuccess) err = hipMalloc(&p, std::max<size_t>(n * sizeof(T), 256));
    if (p) bufs.push_back(p);
    return static_cast<T*>(p);
  }
  ~Scratch() {
    for (void* p : bufs) (void)hipFree(p);
  }
};

}  // namespace

// Tuning cache file: a text file of lines
//   bsi-tune-cache 1
//   library <BSI_VERSION>
//   device <architecture name> <compute units>
//   plan <N> <P>              one per stamp side with a chosen slot plan
//   transform <N> <method>    one per stamp side with a chosen transform
// The choices were measured on one device with one library build: a file of
// another library version or device is ignored, and a missing file is an
// empty cache.  Anything else that does not parse is an error.
namespace bsi_host {

int load_tune_cache(bsi_ctx* h, std::string& err) {
  FILE* fp = std::fopen(h->tune_cache.c_str(), "r");
  if (!fp) {
    if (errno == ENOENT) return BSI_OK;
    err = "tune cache " + h->tune_cache + ": cannot read (" + std::strerror(errno) + ")";
    return BSI_EINVAL;
  }
  std::string text;
  char buf[4096];
  for (size_t k; (k = std::fread(buf, 1, sizeof(buf), fp)) > 0;) text.append(buf, k);
  const bool read_ok = !std::ferror(fp);
  std::fclose(fp);
  if (!read_ok) {
    err = "tune cache " + h->tune_cache + ": read error";
    return BSI_EINVAL;
  }
  std::istringstream f(text);
  int plan[kMaxN + 1] = {}, tr[kMaxN + 1] = {};
  bool matches = true, seen_lib = false, seen_dev = false;
  std::string line;
  int no = 0;
  auto bad = [&](const char* why) {
    err = "tune cache " + h->tune_cache + ", line " + std::to_string(no) + ": " + why;
    return BSI_EINVAL;
  };
  while (std::getline(f, line)) {
    ++no;
    std::istringstream in(line);
    std::string key;
    if (!(in >> key)) continue;   // blank line
    std::string extra;
    if (no == 1) {
      int fmt = 0;
      if (key != "bsi-tune-cache" || !(in >> fmt) || fmt != 1 || (in >> extra))
        return bad("not a tuning cache of format 1");
      continue;
    }
    if (key == "library") {
      int v = 0;
      if (!(in >> v) || (in >> extra)) return bad("expected 'library <version>'");
      matches &= (v == BSI_VERSION);
      seen_lib = true;
    } else if (key == "device") {
      std::string arch;
      int cus = 0;
      if (!(in >> arch >> cus) || (in >> extra)) return bad("expected 'device <arch> <compute units>'");
      matches &= (arch == h->arch && cus == h->num_cu);
      seen_dev = true;
    } else if (key == "plan" || key == "transform") {
      int n = 0, v = 0;
      if (!(in >> n >> v) || (in >> extra)) return bad("expected '<key> <stamp side> <value>'");
      if (n < 8 || n > kMaxN) return bad("stamp side outside [8, 128]");
      if (key == "plan") {
        if (!supported_p(v) || !plan_valid(n, v)) return bad("slot plan not available for this side");
        plan[n] = v;
      } else {
        if (v != BSI_TRANSFORM_DIRECT && v != BSI_TRANSFORM_MFMA) return bad("unknown transform");
        tr[n] = v;
      }
    } else {
      return bad("unknown key");
    }
  }
  if (no == 0) return BSI_OK;        // empty file: empty cache
  if (!seen_lib || !seen_dev) {
    err = "tune cache " + h->tune_cache + ": no 'library' or 'device' line";
    return BSI_EINVAL;
  }
  if (!matches) return BSI_OK;       // measured by another build or on another device
  for (int n = 8; n <= kMaxN; ++n) {
    if (plan[n]) h->plan_P[n] = plan[n];
    if (tr[n]) h->transform[n] = tr[n];
  }
  return BSI_OK;
}

int save_tune_cache(bsi_handle h) {
  if (h->tune_cache.empty()) return BSI_OK;
  // written whole to a private file, then renamed over the cache
  const std::string tmp = h->tune_cache + ".tmp." + std::to_string((long)getpid());
  FILE* f = std::fopen(tmp.c_str(), "w");
  if (!f) return fail(h, BSI_EINVAL, "tune cache %s: cannot write (%s)", tmp.c_str(), std::strerror(errno));
  std::fprintf(f, "bsi-tune-cache 1\nlibrary %d\ndevice %s %d\n", BSI_VERSION, h->arch.c_str(), h->num_cu);
  for (int n = 8; n <= kMaxN; ++n)
    if (h->plan_P[n] > 0) std::fprintf(f, "plan %d %d\n", n, h->plan_P[n]);
  for (int n = 8; n <= kMaxN; ++n)
    if (h->transform[n] != 0) std::fprintf(f, "transform %d %d\n", n, h->transform[n]);
  const bool ok = !std::ferror(f);
  if (std::fclose(f) != 0 || !ok || std::rename(tmp.c_str(), h->tune_cache.c_str()) != 0) {
    const int e = errno;
    std::remove(tmp.c_str());
    return fail(h, BSI_EINVAL, "tune cache %s: write failed (%s)", h->tune_cache.c_str(), std::strerror(e));
  }
  return BSI_OK;
}

}  // namespace bsi_host

extern "C" {

int bsi_set_plan(bsi_handle h, int32_t n, int32_t P) {
  if (!h) return BSI_EINVAL;
  h->err.clear();
  if (n < 8 || n > kMaxN) return fail(h, BSI_EINVAL, "stamp side %d outside [8, %d]", n, kMaxN);
  if (P != 0 && (!supported_p(P) || !plan_valid(n, P)))
    return fail(h, BSI_EINVAL, "plan P = %d is not available for N = %d", P, n);
  h->plan_P[n] = P;
  return BSI_OK;
}

int bsi_get_plan(bsi_handle h, int32_t n, int32_t* P, int32_t* slots) {
  if (!h || !P) return BSI_EINVAL;
  if (n < 8 || n > kMaxN) return fail(h, BSI_EINVAL, "stamp side %d outside [8, %d]", n, kMaxN);
  *P = h->plan_P[n] > 0 ? h->plan_P[n] : make_slot_plan(n).P;
  if (slots) *slots = 2 * make_slot_plan_p(n, *P).nslots;
  return BSI_OK;
}

int bsi_autotune(bsi_handle h, int32_t n_sizes, const int32_t* sizes, int32_t n_chains,
                 int32_t* chosen, float* ms_out) {
  if (!h) return BSI_EINVAL;
  h->err.clear();
  if (n_sizes < 0 || (n_sizes > 0 && !sizes)) return fail(h, BSI_EINVAL, "sizes is NULL");
  if (n_chains < 1 || n_chains > 16) return fail(h, BSI_EINVAL, "n_chains must be 1..16");
  for (int i = 0; i < n_sizes; ++i)
    if (sizes[i] < 8 || sizes[i] > kMaxN)
      return fail(h, BSI_EUNSUPPORTED, "stamp side %d outside [8, %d]", sizes[i], kMaxN);
  hipSetDevice(h->device);
  hipStream_t s = h->own;
  const int C = n_chains;
  const int G = std::max(64, 16384 / C);
  const float pixel_scale = 0.2f;
  const float rs = profile_rscale(kProfExpHost, pixel_scale);
  for (int i = 0; i < n_sizes; ++i) {
    const int N = sizes[i];
    const std::vector<int> cand = candidates(N);
    int best_P = make_slot_plan(N).P;
    float best_ms = -1.0f;
    if (cand.size() > 1) {
      Scratch sc;
      const int64_t npx = (int64_t)N * N;
      int max_bins = 0;
      for (int P : cand) max_bins = std::max(max_bins, make_slot_plan_p(N, P).nbins);
      float* data = sc.get<float>((size_t)G * npx);
      float* psf = sc.get<float>(G);
      float* sig = sc.get<float>(G);
      float* ref = sc.get<float>((size_t)G * 2);
      float* prm = sc.get<float>((size_t)G * 6);
      float* init = sc.get<float>((size_t)G * C * 6);
      int32_t* gidx = sc.get<int32_t>(G);
      int64_t* off = sc.get<int64_t>(G);
      int64_t* boff = sc.get<int64_t>(G);
      float2* dh = sc.get<float2>((size_t)G * max_bins);
      ChainState* st = sc.get<ChainState>((size_t)G * C);
      hipEvent_t e0 = nullptr, e1 = nullptr;
      if (sc.err == hipSuccess) sc.err = hipEventCreate(&e0);
      if (sc.err == hipSuccess) sc.err = hipEventCreate(&e1);
      if (sc.err != hipSuccess) {
        (void)hipGetLastError();
        if (e0) (void)hipEventDestroy(e0);
        return fail(h, BSI_ENOMEM, "autotune buffers for N = %d", N);
      }
      // one synthetic galaxy repeated: F = 1000, hlr 0.5", e = (0.1, -0.05), centred
      std::vector<float> hp((size_t)G * 6), hi((size_t)G * C * 6), hpsf(G, 0.7f), hsig(G, 1.0f),
          href((size_t)G * 2, 0.0f);
      std::vector<int32_t> hg(G);
      std::vector<int64_t> ho(G), hb(G);
      for (int g = 0; g < G; ++g) {
        const float p6[6] = {1000.0f, 0.5f, 0.1f, -0.05f, 0.0f, 0.0f};
        std::copy(p6, p6 + 6, hp.begin() + 6 * g);
        for (int c = 0; c < C; ++c) {
          const float t6[6] = {3.0f, std::log10(0.5f), 0.1f, -0.05f, 0.0f, 0.0f};
          std::copy(t6, t6 + 6, hi.begin() + ((size_t)g * C + c) * 6);
        }
        hg[g] = g;
        ho[g] = g * npx;
        hb[g] = (int64_t)g * max_bins;
      }
      hipError_t e = hipMemcpy(prm, hp.data(), hp.size() * 4, hipMemcpyHostToDevice);
      if (e == hipSuccess) e = hipMemcpy(init, hi.data(), hi.size() * 4, hipMemcpyHostToDevice);
      if (e == hipSuccess) e = hipMemcpy(psf, hpsf.data(), G * 4, hipMemcpyHostToDevice);
      if (e == hipSuccess) e = hipMemcpy(sig, hsig.data(), G * 4, hipMemcpyHostToDevice);
      if (e == hipSuccess) e = hipMemcpy(ref, href.data(), href.size() * 4, hipMemcpyHostToDevice);
      if (e == hipSuccess) e = hipMemcpy(gidx, hg.data(), G * 4, hipMemcpyHostToDevice);
      if (e == hipSuccess) e = hipMemcpy(off, ho.data(), G * 8, hipMemcpyHostToDevice);
      if (e == hipSuccess) e = hipMemcpy(boff, hb.data(), G * 8, hipMemcpyHostToDevice);
      if (e == hipSuccess) e = launch_render(prm, psf, gidx, G, off, N, rs, 1.0f / pixel_scale,
                                            kProfExpHost, 0.5f, data, s);
      HmcArgs a{};
      a.dh = dh;
      a.bin_off = boff;
      a.gidx = gidx;
      a.n_gal = G;
      a.psf = psf;
      a.sigma = sig;
      a.ref_xy = ref;
      a.init = init;
      a.state = st;
      a.N = N;
      a.rscale = rs;
      a.pscale_inv = 1.0f / pixel_scale;
      a.prof = kProfExpHost;
      a.C = C;
      a.L = 20;
      a.W = 1 << 20;
      a.S = 0;
      a.eps0 = 1e-3f;
      a.delta = 0.8f;
      a.mu = std::log(1e-2f);
      a.lf_lo = -1.0f;
      a.lf_hi = 9.0f;
      a.ls_lo = -2.0f;
      a.ls_hi = 1.0f;
      a.sigma_d = 0.5f;
      a.sigma_e = 0.3f;
      a.t_stop = 1 << 20;
      a.wpc = 1;
      for (int P : cand) {
        if (e != hipSuccess) break;
        if (hmc_lds_bytes(N, C, P, 1) > 160 * 1024) continue;
        a.P = P;
        e = launch_stamp_dft(transform_of(h, N) == BSI_TRANSFORM_MFMA, data, nullptr, gidx, G, off,
                             boff, N, P, dh, nullptr, s);
        if (e == hipSuccess) {
          a.n_steps = 0;
          e = launch_hmc_init(a, G, s);
        }
        a.n_steps = a.L;
        if (e == hipSuccess) e = launch_hmc_advance(a, G, s);     // warm
        float best = -1.0f;
        for (int r = 0; r < 5 && e == hipSuccess; ++r) {
          e = hipEventRecord(e0, s);
          if (e == hipSuccess) e = launch_hmc_advance(a, G, s);
          if (e == hipSuccess) e = hipEventRecord(e1, s);
          if (e == hipSuccess) e = hipEventSynchronize(e1);
          float t = 0.0f;
          if (e == hipSuccess) e = hipEventElapsedTime(&t, e0, e1);
          if (e == hipSuccess && (best < 0.0f || t < best)) best = t;
        }
        // the default plan (the first candidate) is kept unless another is
        // at least 2 % faster
        if (e == hipSuccess && (best_ms < 0.0f || best < 0.98f * best_ms)) {
          best_ms = best;
          best_P = P;
        }
      }
      (void)hipEventDestroy(e0);
      (void)hipEventDestroy(e1);
      if (e != hipSuccess) return hip_fail(h, e, "autotune");
    }
    h->plan_P[N] = best_P;
    if (chosen) chosen[i] = best_P;
    if (ms_out) ms_out[i] = best_ms;
  }
  return save_tune_cache(h);
}

int bsi_set_transform(bsi_handle h, int32_t n, int32_t method) {
  if (!h) return BSI_EINVAL;
  h->err.clear();
  if (n < 8 || n > kMaxN) return fail(h, BSI_EINVAL, "stamp side %d outside [8, %d]", n, kMaxN);
  if (method != BSI_TRANSFORM_DEFAULT && method != BSI_TRANSFORM_DIRECT && method != BSI_TRANSFORM_MFMA)
    return fail(h, BSI_EINVAL, "unknown transform %d", method);
  h->transform[n] = method;
  return BSI_OK;
}

int bsi_get_transform(bsi_handle h, int32_t n, int32_t* method) {
  if (!h || !method) return BSI_EINVAL;
  if (n < 8 || n > kMaxN) return fail(h, BSI_EINVAL, "stamp side %d outside [8, %d]", n, kMaxN);
  *method = transform_of(h, n);
  return BSI_OK;
}

int bsi_autotune_transform(bsi_handle h, int32_t n_sizes, const int32_t* sizes, int32_t n_gal,
                           int32_t* chosen, float* ms_out) {
  if (!h) return BSI_EINVAL;
  h->err.clear();
  if (n_sizes < 0 || (n_sizes > 0 && !sizes)) return fail(h, BSI_EINVAL, "sizes is NULL");
  if (n_gal < 1 || n_gal > (1 << 20)) return fail(h, BSI_EINVAL, "n_gal must be 1..2^20");
  for (int i = 0; i < n_sizes; ++i)
    if (sizes[i] < 8 || sizes[i] > kMaxN)
      return fail(h, BSI_EUNSUPPORTED, "stamp side %d outside [8, %d]", sizes[i], kMaxN);
  hipSetDevice(h->device);
  hipStream_t s = h->own;
  const int G = n_gal;
  const float pixel_scale = 0.2f;
  const float rs = profile_rscale(kProfExpHost, pixel_scale);
  for (int i = 0; i < n_sizes; ++i) {
    const int N = sizes[i];
    Scratch sc;
    const int64_t npx = (int64_t)N * N;
    const int P = make_slot_plan(N).P;
    const int nb = make_slot_plan_p(N, P).nbins;
    float* out = sc.get<float>((size_t)G * npx);
    float* psf = sc.get<float>(G);
    float* prm = sc.get<float>((size_t)G * 6);
    int32_t* gidx = sc.get<int32_t>(G);
    int64_t* off = sc.get<int64_t>(G);
    int64_t* boff = sc.get<int64_t>(G);
    float2* dh = sc.get<float2>((size_t)G * nb);
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (sc.err == hipSuccess) sc.err = hipEventCreate(&e0);
    if (sc.err == hipSuccess) sc.err = hipEventCreate(&e1);
    if (sc.err != hipSuccess) {
      (void)hipGetLastError();
      if (e0) (void)hipEventDestroy(e0);
      return fail(h, BSI_ENOMEM, "transform autotune buffers for N = %d", N);
    }
    // galaxies with varied shapes and centroids (F = 1000, hlr 0.3-0.9")
    std::vector<float> hp((size_t)G * 6), hpsf(G);
    std::vector<int32_t> hg(G);
    std::vector<int64_t> ho(G), hb(G);
    for (int g = 0; g < G; ++g) {
      const float f = (float)(g % 97) / 97.0f;
      const float p6[6] = {1000.0f, 0.3f + 0.6f * f, 0.3f * f - 0.15f, 0.1f - 0.2f * f, f - 0.5f,
                           0.5f - f};
      std::copy(p6, p6 + 6, hp.begin() + 6 * g);
      hpsf[g] = 0.6f + 0.3f * f;
      hg[g] = g;
      ho[g] = g * npx;
      hb[g] = (int64_t)g * nb;
    }
    hipError_t e = hipMemcpy(prm, hp.data(), hp.size() * 4, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(boff, hb.data(), G * 8, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(psf, hpsf.data(), G * 4, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(gidx, hg.data(), G * 4, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(off, ho.data(), G * 8, hipMemcpyHostToDevice);
    // 0, 1: render direct / MFMA; 2, 3: forward DFT of the rendered stamps direct / MFMA
    float best[4] = {-1.0f, -1.0f, -1.0f, -1.0f};
    for (int m = 0; m < 4 && e == hipSuccess; ++m) {
      auto run = [&]() {
        switch (m) {
          case 0: return launch_render(prm, psf, gidx, G, off, N, rs, 1.0f / pixel_scale, kProfExpHost,
                                       0.5f, out, s);
          case 1: return launch_render_mfma(prm, psf, gidx, G, off, N, rs, 1.0f / pixel_scale,
                                            kProfExpHost, 0.5f, out, s);
          default: return launch_stamp_dft(m == 3, out, nullptr, gidx, G, off, boff, N, P, dh, nullptr, s);
        }
      };
      e = run();     // warm
      for (int r = 0; r < 5 && e == hipSuccess; ++r) {
        e = hipEventRecord(e0, s);
        if (e == hipSuccess) e = run();
        if (e == hipSuccess) e = hipEventRecord(e1, s);
        if (e == hipSuccess) e = hipEventSynchronize(e1);
        float t = 0.0f;
        if (e == hipSuccess) e = hipEventElapsedTime(&t, e0, e1);
        if (e == hipSuccess && (best[m] < 0.0f || t < best[m])) best[m] = t;
      }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (e != hipSuccess) return hip_fail(h, e, "transform autotune");
    const int pick = best[1] + best[3] <= best[0] + best[2] ? BSI_TRANSFORM_MFMA : BSI_TRANSFORM_DIRECT;
    h->transform[N] = pick;
    if (chosen) chosen[i] = pick;
    if (ms_out)
      for (int m = 0; m < 4; ++m) ms_out[4 * i + m] = best[m];
  }
  return save_tune_cache(h);
}

}  // extern "C"
