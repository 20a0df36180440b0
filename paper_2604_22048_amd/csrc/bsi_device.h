// Device-side building blocks of the shear-inference kernels (gfx950, wave64).
//
// Frequency grid of an N x N stamp.  Frequencies u, v run over
// -h..h with h = floor(N/2) ("frequency points"; 2h+1 of them per axis, the
// ends carrying weight 1/2 when N is even).  The DFT of a real stamp is
// Hermitian, so only a half plane of DFT bins is kept:
//   * main bins: the odd core |u|, |v| <= hc (hc = h for odd N, h-1 for even
//     N) with v > 0, or v = 0 and u > 0.  Each stands for itself and its
//     mirror bin, so it counts twice in every sum over the full grid.
//   * special bins: the DC bin, and for even N the Nyquist row/column bins
//     (frequency -N/2 on either axis).  For even N a Nyquist bin of the
//     model's DFT collects two frequency points per Nyquist axis, +-N/2, each
//     with weight 1/2 and the sign (-1)^(N-1) = -1 on the +N/2 point, because
//     pixel centres sit at half-integer offsets from the stamp centre.
// Bins are stored main bins first (row-major over v, u), then special bins.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace bsi {

constexpr int kWave = 64;
constexpr int kMaxN = 128;
constexpr float kPiF = 3.14159265358979323846f;
constexpr double kLn10 = 2.30258509299404568402;
constexpr float kLn10F = 2.30258509299404568402f;
constexpr float kLn2F = 0.69314718055994530942f;

struct Geom {
  int N, h, nc, hc;
  int nmain, nspec, nbins, ntab;
  float kstep;      // 2 pi / N
  float inv_nc;
};

__host__ __device__ constexpr Geom make_geom(int N) {
  Geom g{};
  g.N = N;
  g.h = N / 2;
  g.nc = (N & 1) ? N : N - 1;
  g.hc = (g.nc - 1) / 2;
  g.nmain = (g.nc * g.nc - 1) / 2;
  g.nspec = (N & 1) ? 1 : N + 2;
  g.nbins = g.nmain + g.nspec;
  g.ntab = 2 * g.h + 1;
  g.kstep = 2.0f * kPiF / (float)N;
  g.inv_nc = 1.0f / (float)g.nc;
  return g;
}

// Main bin index -> (u, v) frequencies.
__device__ __forceinline__ void main_bin_uv(const Geom& g, int b, int& u, int& v) {
  int bp = b + g.hc + 1;                       // skip u <= 0 of row v = 0
  v = (int)(((float)bp + 0.5f) * g.inv_nc);    // exact: bp < 2^14
  u = bp - v * g.nc - g.hc;
}

// Special bin index -> (u_b, v_b) DFT bin (Nyquist bins use frequency -N/2)
// and the multiplicity c of the bin in a full-grid sum (1 = self-mirror).
__host__ __device__ inline void spec_bin_uv(int N, int i, int& u, int& v, int& c) {
  int h = N / 2;
  if (i == 0) { u = 0; v = 0; c = 1; return; }
  // even N only below
  if (i == 1) { u = -h; v = 0; c = 1; return; }
  if (i == 2) { u = 0; v = -h; c = 1; return; }
  if (i < h + 2) { u = i - 2; v = -h; c = 2; return; }        // u = 1..h-1
  if (i == h + 2) { u = -h; v = -h; c = 1; return; }
  u = -h; v = i - (h + 2); c = 2;                               // v = 1..h-1
}

// Twiddle index: k_u x_i = pi * u * (2 i - N + 1) / N, reduced mod 2N.
__device__ __forceinline__ int tw_index(int u, int i, int N) {
  int m = (u * (2 * i - N + 1)) % (2 * N);
  return m < 0 ? m + 2 * N : m;
}

// ---- Philox4x32-10 (Salmon et al., SC'11) -----------------------------------
__device__ __forceinline__ uint4 philox4x32_10(uint4 c, uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r) {
      k0 += 0x9E3779B9u;
      k1 += 0xBB67AE85u;
    }
    const uint32_t hi0 = __umulhi(0xD2511F53u, c.x), lo0 = 0xD2511F53u * c.x;
    const uint32_t hi1 = __umulhi(0xCD9E8D57u, c.z), lo1 = 0xCD9E8D57u * c.z;
    c = make_uint4(hi1 ^ c.y ^ k0, lo1, hi0 ^ c.w ^ k1, lo0);
  }
  return c;
}

// Top 23 bits to an odd multiple of 2^-24 in (0, 1): exact in float.
__device__ __forceinline__ float u01(uint32_t w) {
  return ((float)(w >> 9) + 0.5f) * 1.1920928955078125e-07f;   // 2^-23
}

enum { kTagMomentum = 0, kTagAccept = 1, kTagInit = 2, kTagJitter = 3 };

// ---- wave helpers --------------------------------------------------------------
__device__ __forceinline__ int lane_id() { return (int)(threadIdx.x & (kWave - 1)); }

// Order this wave's LDS writes before its subsequent LDS reads by other lanes.
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ float wave_sum(float x) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) x += __shfl_xor(x, o, kWave);
  return x;
}

__device__ __forceinline__ double wave_sum(double x) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) x += __shfl_xor(x, o, kWave);
  return x;
}

// Wave-wide sums with DPP row shifts and row broadcasts (no LDS traffic): an
// inclusive prefix sum within each row of 16 lanes, then rows combined by
// broadcasting lanes 15 and 31; lane 63 ends with the total, which is read
// back as a wave-uniform value.
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ float dpp_shift_add(float x) {
  return x + __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), CTRL, ROW_MASK, 0xf, false));
}

template <int CTRL, int ROW_MASK>
__device__ __forceinline__ double dpp_shift_add(double x) {
  const long long v = __double_as_longlong(x);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)(v & 0xffffffffll), CTRL, ROW_MASK, 0xf, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(v >> 32), CTRL, ROW_MASK, 0xf, false);
  return x + __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

template <typename T>
__device__ __forceinline__ T wave_sum_dpp(T x) {
  x = dpp_shift_add<0x111, 0xf>(x);   // row_shr:1
  x = dpp_shift_add<0x112, 0xf>(x);   // row_shr:2
  x = dpp_shift_add<0x114, 0xf>(x);   // row_shr:4
  x = dpp_shift_add<0x118, 0xf>(x);   // row_shr:8
  x = dpp_shift_add<0x142, 0xa>(x);   // row_bcast:15 into rows 1 and 3
  x = dpp_shift_add<0x143, 0xc>(x);   // row_bcast:31 into rows 2 and 3
  return x;                           // total on lane 63
}

__device__ __forceinline__ float wave_total(float x) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(wave_sum_dpp(x)), 63));
}

__device__ __forceinline__ double wave_total(double x) {
  const long long v = __double_as_longlong(wave_sum_dpp(x));
  const int lo = __builtin_amdgcn_readlane((int)(v & 0xffffffffll), 63);
  const int hi = __builtin_amdgcn_readlane((int)(v >> 32), 63);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// Seven wave-wide float sums at once through a per-wave LDS scratch of
// 64 x 8 words: each lane writes its eight partials (slot 7 unused), lane l
// then adds the partials of value l / 8 held by lanes 8 (l % 8) .. 8 (l % 8) + 7,
// and a three-step DPP prefix sum inside each group of eight lanes finishes
// the sum on lane 8 v + 7.  scratch must be 16-byte aligned, 2 KiB per wave.
__device__ __forceinline__ void wave_total7(float* v, float* scratch) {
  const int lane = lane_id();
  float4* s4 = reinterpret_cast<float4*>(scratch);
  s4[2 * lane] = make_float4(v[0], v[1], v[2], v[3]);
  s4[2 * lane + 1] = make_float4(v[4], v[5], v[6], 0.f);
  wave_lds_sync();
  const int val = lane >> 3, grp = lane & 7;
  float acc = 0.f;
#pragma unroll
  for (int k = 0; k < 8; ++k) acc += scratch[(8 * grp + k) * 8 + val];
  acc = dpp_shift_add<0x111, 0xf>(acc);   // row_shr:1
  acc = dpp_shift_add<0x112, 0xf>(acc);   // row_shr:2
  acc = dpp_shift_add<0x114, 0xf>(acc);   // row_shr:4
#pragma unroll
  for (int j = 0; j < 7; ++j) v[j] = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(acc), 8 * j + 7));
  wave_lds_sync();
}

// ---- Several chains per wave: H = 2 (lanes 0..31 and 32..63) or H = 4 -----
// (lanes 16 c .. 16 c + 15 serve chain c of the wave)

// Lane index within the lanes serving this lane's chain (H chains per wave).
template <int H>
__device__ __forceinline__ int chain_lane() {
  static_assert(H == 1 || H == 2 || H == 4, "1, 2 or 4 chains per wave");
  return lane_id() & (kWave / H - 1);
}

// Value of lane k of this lane's chain (lane k of the wave for H = 1; for
// H = 2 two lane reads and a select; for H = 4 one ds_bpermute, which uses
// no LDS storage).
template <int H>
__device__ __forceinline__ uint32_t hbcast(uint32_t x, int k) {
  if constexpr (H == 1) {
    return (uint32_t)__builtin_amdgcn_readlane((int)x, k);
  } else if constexpr (H == 2) {
    const uint32_t a = (uint32_t)__builtin_amdgcn_readlane((int)x, k);
    const uint32_t b = (uint32_t)__builtin_amdgcn_readlane((int)x, 32 + k);
    return (lane_id() & 32) ? b : a;
  } else {
    const int src = (lane_id() & ~(kWave / H - 1)) + k;
    return (uint32_t)__builtin_amdgcn_ds_bpermute(src << 2, (int)x);
  }
}
template <int H>
__device__ __forceinline__ float hbcast(float x, int k) {
  return __uint_as_float(hbcast<H>(__float_as_uint(x), k));
}

// Sum over the 64 / H lanes of each chain by a butterfly: every lane of a
// chain ends with the same bits (each stage adds the same two operands on
// both partners).
template <int H>
__device__ __forceinline__ double group_total(double x) {
#pragma unroll
  for (int o = kWave / H / 2; o >= 1; o >>= 1) x += __shfl_xor(x, o, kWave);
  return x;
}

// Seven sums over the LS = 64 / H lanes of each chain (H = 2 or 4) through
// the wave's 2 KiB LDS scratch: each lane writes its eight partials; with
// LV = LS / 8 lanes per value, lane r of a chain adds value r / LV of lanes
// 8 (r % LV) .. 8 (r % LV) + 7 of its chain, a DPP prefix sum inside each
// group of LV lanes finishes the sum on its last lane, and the sums go back
// through LDS to every lane of their chain.
template <int H>
__device__ __forceinline__ void group_total7(float* v, float* scratch) {
  static_assert(H == 2 || H == 4, "several chains per wave");
  constexpr int LS = kWave / H, LV = LS / 8;
  const int lane = lane_id();
  float4* s4 = reinterpret_cast<float4*>(scratch);
  s4[2 * lane] = make_float4(v[0], v[1], v[2], v[3]);
  s4[2 * lane + 1] = make_float4(v[4], v[5], v[6], 0.f);
  wave_lds_sync();
  const int base = lane & ~(LS - 1), r = lane & (LS - 1);
  const int val = r / LV, grp = r % LV;
  float acc = 0.f;
#pragma unroll
  for (int k = 0; k < 8; ++k) acc += scratch[(base + 8 * grp + k) * 8 + val];
  acc = dpp_shift_add<0x111, 0xf>(acc);                        // row_shr:1
  if constexpr (LV == 4) acc = dpp_shift_add<0x112, 0xf>(acc);  // row_shr:2
  wave_lds_sync();
  if (grp == LV - 1) scratch[base / LV + val] = acc;
  wave_lds_sync();
  const float* res = scratch + base / LV;
#pragma unroll
  for (int j = 0; j < 7; ++j) v[j] = res[j];
  wave_lds_sync();
}

__device__ __forceinline__ float wave_max(float x) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) x = fmaxf(x, __shfl_xor(x, o, kWave));
  return x;
}

__device__ __forceinline__ float bcast(float x, int l) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x), l));
}
__device__ __forceinline__ int bcast(int x, int l) { return __builtin_amdgcn_readlane(x, l); }
__device__ __forceinline__ uint32_t bcast(uint32_t x, int l) {
  return (uint32_t)__builtin_amdgcn_readlane((int)x, l);
}
__device__ __forceinline__ double bcast(double x, int l) {
  long long v = __double_as_longlong(x);
  int lo = __builtin_amdgcn_readlane((int)(v & 0xffffffffll), l);
  int hi = __builtin_amdgcn_readlane((int)(v >> 32), l);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

}  // namespace bsi
