// HIP kernels of libmpg (gfx950 / CDNA4, wave64).
//
// Paper: Prusa, Holighaus, Balazs, "Fast Matching Pursuit with Multi-Gabor
// Dictionaries", ACM TOMS 47(3), 2021.  Notation: system w has window g_w
// of length gl_w, hop a_w, M_w channels, N_w = L / a_w frames and M_w/2 + 1
// reduced bins (Sec. 5).  A selected atom is (v, k, j); a target coefficient
// is (w, m, n).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <mutex>
#include <type_traits>

#include "mpg_internal.h"

namespace mpg {

template <typename R>
struct Cx {
  R re, im;
};

// --------------------------------------------------------------------------
// integer helpers

__device__ __forceinline__ int64_t floor_div(int64_t a, int64_t b) {
  return a >= 0 ? a / b : -((-a + b - 1) / b);
}
__device__ __forceinline__ int64_t ceil_div(int64_t a, int64_t b) { return -floor_div(-a, b); }
__device__ __forceinline__ int floor_div32(int a, int b) { return a >= 0 ? a / b : -((-a + b - 1) / b); }
__device__ __forceinline__ int ceil_div32(int a, int b) { return -floor_div32(-a, b); }
__device__ __forceinline__ int32_t mod_pos(int32_t v, int32_t n) {
  int32_t r = v % n;
  return r < 0 ? r + n : r;
}
// representative of v modulo n in (-n/2, n/2]
__device__ __forceinline__ int32_t cmod(int32_t v, int32_t n) {
  int32_t r = mod_pos(v, n);
  return r > n / 2 ? r - n : r;
}

__device__ __forceinline__ int uni(int v) { return __builtin_amdgcn_readfirstlane(v); }

// --------------------------------------------------------------------------
// max-tree keys.  A key orders coefficients by |rho|^2 and, among equal
// values, by the lower coefficient index (ties go to the lowest index).

template <typename R>
struct KeyOps;

template <>
struct KeyOps<float> {
  // high word: bits of |rho|^2 (>= 0, so integer order = float order),
  // low word: ~index.
  using Key = uint64_t;
  static __device__ __forceinline__ Key make(float v, uint32_t idx) {
    return ((uint64_t)__float_as_uint(v) << 32) | (uint64_t)(~idx);
  }
  static __device__ __forceinline__ Key empty() { return 0ull; }
  static __device__ __forceinline__ bool gt(Key a, Key b) { return a > b; }
  static __device__ __forceinline__ bool eq(Key a, Key b) { return a == b; }
  static __device__ __forceinline__ uint32_t index(Key a) { return ~(uint32_t)a; }
  static __device__ __forceinline__ float value(Key a) { return __uint_as_float((uint32_t)(a >> 32)); }
  static __device__ __forceinline__ Key shfl_xor(Key a, int m) { return __shfl_xor(a, m); }
};

struct Key96 {
  uint64_t v;   // bits of |rho|^2 as double
  uint32_t n;   // ~index
};

template <>
struct KeyOps<double> {
  using Key = Key96;
  static __device__ __forceinline__ Key make(double v, uint32_t idx) {
    return Key96{(uint64_t)__double_as_longlong(v), ~idx};
  }
  static __device__ __forceinline__ Key empty() { return Key96{0ull, 0u}; }
  static __device__ __forceinline__ bool gt(Key a, Key b) {
    return a.v > b.v || (a.v == b.v && a.n > b.n);
  }
  static __device__ __forceinline__ bool eq(Key a, Key b) { return a.v == b.v && a.n == b.n; }
  static __device__ __forceinline__ uint32_t index(Key a) { return ~a.n; }
  static __device__ __forceinline__ double value(Key a) { return __longlong_as_double((long long)a.v); }
  static __device__ __forceinline__ Key shfl_xor(Key a, int m) {
    return Key96{__shfl_xor(a.v, m), (uint32_t)__shfl_xor((int)a.n, m)};
  }
};

// A leaf of the max tree.  FP32: the key alone.  FP64: the key and the
// complex value there.
template <typename R>
struct Leaf;
template <>
struct __align__(8) Leaf<float> {
  uint64_t key;
};
template <>
struct __align__(16) Leaf<double> {
  uint64_t v;
  uint32_t n, pad;
  double re, im;
};

__device__ __forceinline__ uint64_t leaf_key(const Leaf<float>& l) { return l.key; }
__device__ __forceinline__ Key96 leaf_key(const Leaf<double>& l) { return Key96{l.v, l.n}; }
__device__ __forceinline__ Leaf<float> make_leaf(uint64_t k, float, float) {
  Leaf<float> l;
  l.key = k;
  return l;
}
__device__ __forceinline__ Leaf<double> make_leaf(Key96 k, double re, double im) {
  Leaf<double> l;
  l.v = k.v;
  l.n = k.n;
  l.pad = 0;
  l.re = re;
  l.im = im;
  return l;
}

template <typename R>
__device__ __forceinline__ void sincospi_(R x, R* s, R* c);
template <>
__device__ __forceinline__ void sincospi_<float>(float x, float* s, float* c) {
  sincospif(x, s, c);
}
template <>
__device__ __forceinline__ void sincospi_<double>(double x, double* s, double* c) {
  sincospi(x, s, c);
}

// --------------------------------------------------------------------------
// Cross-lane primitives on DPP (no LDS round trips).  Every call site runs
// with all 64 lanes active.

template <int CTRL>
__device__ __forceinline__ uint32_t dpp32(uint32_t v) {
  return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, CTRL, 0xF, 0xF, false);
}
template <int CTRL>
__device__ __forceinline__ uint64_t dpp64(uint64_t v) {
  const uint32_t lo = dpp32<CTRL>((uint32_t)v), hi = dpp32<CTRL>((uint32_t)(v >> 32));
  return ((uint64_t)hi << 32) | lo;
}
__device__ __forceinline__ uint32_t rdlane32(uint32_t v, int l) {
  return (uint32_t)__builtin_amdgcn_readlane((int)v, l);
}
__device__ __forceinline__ uint64_t rdlane64(uint64_t v, int l) {
  return ((uint64_t)rdlane32((uint32_t)(v >> 32), l) << 32) | rdlane32((uint32_t)v, l);
}
__device__ __forceinline__ int uni_i(int v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ int64_t uni_l(int64_t v) {
  return (int64_t)(((uint64_t)(uint32_t)uni_i((int)(v >> 32)) << 32) | (uint32_t)uni_i((int)v));
}
__device__ __forceinline__ double uni_d(double v) {
  return __builtin_bit_cast(double, uni_l(__builtin_bit_cast(int64_t, v)));
}

// DPP controls: quad_perm [1,0,3,2], quad_perm [2,3,0,1], row_ror:4, row_ror:8.
// Applied in sequence with a max they leave every lane holding its row maximum.
template <typename R>
struct KeyDpp;

template <>
struct KeyDpp<float> {
  using Key = uint64_t;
  static __device__ __forceinline__ Key kmax(Key a, Key b) { return a > b ? a : b; }
  static __device__ __forceinline__ Key row_max(Key k) {
    k = kmax(k, dpp64<0xB1>(k));
    k = kmax(k, dpp64<0x4E>(k));
    k = kmax(k, dpp64<0x124>(k));
    k = kmax(k, dpp64<0x128>(k));
    return k;
  }
  static __device__ __forceinline__ Key lane(Key k, int l) { return rdlane64(k, l); }
  static __device__ __forceinline__ Key sentinel() { return ~0ull; }
  static __device__ __forceinline__ bool is_sentinel(Key k) { return k == ~0ull; }
};

template <>
struct KeyDpp<double> {
  using Key = Key96;
  static __device__ __forceinline__ Key kmax(Key a, Key b) {
    return (a.v > b.v || (a.v == b.v && a.n > b.n)) ? a : b;
  }
  template <int C>
  static __device__ __forceinline__ Key mv(Key k) {
    return Key96{dpp64<C>(k.v), dpp32<C>(k.n)};
  }
  static __device__ __forceinline__ Key row_max(Key k) {
    k = kmax(k, mv<0xB1>(k));
    k = kmax(k, mv<0x4E>(k));
    k = kmax(k, mv<0x124>(k));
    k = kmax(k, mv<0x128>(k));
    return k;
  }
  static __device__ __forceinline__ Key lane(Key k, int l) { return Key96{rdlane64(k.v, l), rdlane32(k.n, l)}; }
  static __device__ __forceinline__ Key sentinel() { return Key96{~0ull, ~0u}; }
  static __device__ __forceinline__ bool is_sentinel(Key k) { return k.v == ~0ull; }
};

// Wave maximum, returned uniformly (scalar) to every lane.
template <typename R>
__device__ __forceinline__ typename KeyDpp<R>::Key wave_max_key(typename KeyDpp<R>::Key k) {
  using KD = KeyDpp<R>;
  k = KD::row_max(k);
  return KD::kmax(KD::kmax(KD::lane(k, 0), KD::lane(k, 16)), KD::kmax(KD::lane(k, 32), KD::lane(k, 48)));
}

__device__ __forceinline__ bool key_eq(uint64_t a, uint64_t b) { return a == b; }
__device__ __forceinline__ bool key_eq(Key96 a, Key96 b) { return a.v == b.v && a.n == b.n; }

// q / d for 0 <= q < 2^31 with the divisor's magic pair (m, s).
__device__ __forceinline__ int magic_div(int q, uint32_t m, int s) {
  return (int)((__umulhi((uint32_t)q, m) + (uint32_t)q) >> s);
}

// Row (16-lane) maximum of non-negative |rho|^2 bit patterns; every lane of
// a row receives the row's maximum.  FP32 values use 32-bit DPP max steps.
__device__ __forceinline__ uint64_t val_bits(float v) { return (uint64_t)__float_as_uint(v); }
__device__ __forceinline__ uint64_t val_bits(double v) { return (uint64_t)__double_as_longlong(v); }
template <int CTRL>
__device__ __forceinline__ uint32_t max_dpp32(uint32_t v) {
  const uint32_t o = dpp32<CTRL>(v);
  return v > o ? v : o;
}
template <int CTRL>
__device__ __forceinline__ uint64_t max_dpp64(uint64_t v) {
  const uint64_t o = dpp64<CTRL>(v);
  return v > o ? v : o;
}
template <typename R>
__device__ __forceinline__ uint64_t row_max_bits(uint64_t b);
template <>
__device__ __forceinline__ uint64_t row_max_bits<float>(uint64_t b) {
  uint32_t v = (uint32_t)b;
  v = max_dpp32<0xB1>(v);
  v = max_dpp32<0x4E>(v);
  v = max_dpp32<0x124>(v);
  v = max_dpp32<0x128>(v);
  return v;
}
template <>
__device__ __forceinline__ uint64_t row_max_bits<double>(uint64_t b) {
  b = max_dpp64<0xB1>(b);
  b = max_dpp64<0x4E>(b);
  b = max_dpp64<0x124>(b);
  b = max_dpp64<0x128>(b);
  return b;
}
// Selection score of a coefficient: |rho|^2, or with pedantic selection
// (Sec. 5) the energy removed by projecting onto its real atom pair,
// Eq. (projenfaster) with the adjusted coefficient of Eq. (dualatprod) and
// gamma = <d, conj d> of its bin; DC and Nyquist bins (no partner) keep
// |rho|^2.  Never negative, so the bits order like the values.
template <typename R>
__device__ __forceinline__ R sel_score(R re, R im, Cx<R> g, bool pedantic_pair) {
  if (!pedantic_pair) return re * re + im * im;
  const R nr = re - (g.re * re - g.im * im), ni = im - (-g.re * im - g.im * re);
  const R den = (R)1 - (g.re * g.re + g.im * g.im);
  const R cr = nr / den, ci = ni / den;
  const R e = (R)2 * (cr * cr + ci * ci + g.re * (cr * cr - ci * ci) - (R)2 * g.im * cr * ci);
  return e > (R)0 ? e : (R)0;
}

// Wave maximum of keys, returned uniformly.  FP32 keys: maximum of the value
// word, then of the inverted index among lanes holding that value.
template <typename R>
__device__ __forceinline__ typename KeyOps<R>::Key wave_max_key2(typename KeyOps<R>::Key k);
template <>
__device__ __forceinline__ uint64_t wave_max_key2<float>(uint64_t k) {
  uint32_t hi = (uint32_t)(k >> 32);
  uint32_t h = max_dpp32<0xB1>(hi);
  h = max_dpp32<0x4E>(h);
  h = max_dpp32<0x124>(h);
  h = max_dpp32<0x128>(h);
  uint32_t hm = max(max(rdlane32(h, 0), rdlane32(h, 16)), max(rdlane32(h, 32), rdlane32(h, 48)));
  // one lane holds the maximum value word (the common case): its index word
  const uint64_t eq = __ballot(hi == hm);
  if (__popcll(eq) == 1) return ((uint64_t)hm << 32) | rdlane32((uint32_t)k, (int)__ffsll((unsigned long long)eq) - 1);
  uint32_t lo = hi == hm ? (uint32_t)k : 0u;
  uint32_t l = max_dpp32<0xB1>(lo);
  l = max_dpp32<0x4E>(l);
  l = max_dpp32<0x124>(l);
  l = max_dpp32<0x128>(l);
  const uint32_t lm = max(max(rdlane32(l, 0), rdlane32(l, 16)), max(rdlane32(l, 32), rdlane32(l, 48)));
  return ((uint64_t)hm << 32) | lm;
}
template <>
__device__ __forceinline__ Key96 wave_max_key2<double>(Key96 k) {
  return wave_max_key<double>(k);
}

// --------------------------------------------------------------------------
// Gram-kernel precompute, FP64 (Sec. 4.1, 4.2).  For the pair (target w,
// source v) on the common grid (a_min, M_max):
//   h(mu, Delta) = sum_s g_v(s + Delta) g_w(s) exp(-2 pi i mu s / M_max),
// Delta = (c - D) a_min for column c.  One thread per (c, mu).

__global__ void k_gram_full(const double* __restrict__ gw, int glw, const double* __restrict__ gv,
                            int glv, int amin, int D, int Mmax,
                            const double2* __restrict__ roots, double2* __restrict__ out) {
  const int c = blockIdx.x;
  const int mu = blockIdx.y * blockDim.x + threadIdx.x;
  if (mu >= Mmax) return;
  const int Delta = (c - D) * amin;
  // s in [-glw/2, glw/2) and s + Delta in [-glv/2, glv/2)
  int s0 = -glw / 2, s1 = glw / 2;
  if (-glv / 2 - Delta > s0) s0 = -glv / 2 - Delta;
  if (glv / 2 - Delta < s1) s1 = glv / 2 - Delta;
  double sr = 0.0, si = 0.0;
  for (int s = s0; s < s1; ++s) {
    const double p = gv[s + Delta + glv / 2] * gw[s + glw / 2];
    const int64_t idx = ((int64_t)mu * s) % Mmax;
    const double2 r = roots[idx < 0 ? idx + Mmax : idx];
    sr += p * r.x;
    si += p * r.y;
  }
  out[(int64_t)c * Mmax + mu] = make_double2(sr, si);
}

// Maximum |h| over a full table (for the relative threshold).
__global__ void k_gram_absmax(const double2* __restrict__ t, int64_t n,
                              unsigned long long* __restrict__ out) {
  double m = 0.0;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const double2 v = t[i];
    const double a = sqrt(v.x * v.x + v.y * v.y);
    if (a > m) m = a;
  }
  atomicMax(out, (unsigned long long)__double_as_longlong(m));
}

// Bounding box of the surviving entries |h| > thr.
// box[0] = max |delta|, box[1] = min mu, box[2] = max mu, box[3] = count.
__global__ void k_gram_box(const double2* __restrict__ t, int D, int Mmax, double thr,
                           int* __restrict__ box) {
  const int c = blockIdx.x;
  int bd = -1, lo = Mmax, hi = -Mmax, cnt = 0;
  for (int mu = threadIdx.x; mu < Mmax; mu += blockDim.x) {
    const double2 v = t[(int64_t)c * Mmax + mu];
    if (sqrt(v.x * v.x + v.y * v.y) > thr) {
      const int d = c - D < 0 ? D - c : c - D;
      const int mc = mu > Mmax / 2 ? mu - Mmax : mu;
      bd = d > bd ? d : bd;
      lo = mc < lo ? mc : lo;
      hi = mc > hi ? mc : hi;
      ++cnt;
    }
  }
  if (cnt) {
    atomicMax(&box[0], bd);
    atomicMin(&box[1], lo);
    atomicMax(&box[2], hi);
    atomicAdd(&box[3], cnt);
  }
}

// Extract the box, zeroing entries at or below the threshold; FP64 and FP32.
__global__ void k_gram_extract(const double2* __restrict__ t, int D, int Mmax, double thr,
                               int dbox, int mu_lo, int width, double2* __restrict__ o64,
                               float2* __restrict__ o32) {
  const int row = blockIdx.x;  // delta + dbox
  const int c = row - dbox + D;
  for (int i = threadIdx.x; i < width; i += blockDim.x) {
    const int mc = mu_lo + i;
    const int mu = mc < 0 ? mc + Mmax : mc;
    double2 v = t[(int64_t)c * Mmax + mu];
    if (!(sqrt(v.x * v.x + v.y * v.y) > thr)) v = make_double2(0.0, 0.0);
    o64[(int64_t)row * width + i] = v;
    o32[(int64_t)row * width + i] = make_float2((float)v.x, (float)v.y);
  }
}

// Stage-major copy of the DFT twiddles tw[j] = exp(-2 pi i j / M), j < M/2,
// stored behind them: entry h - 1 + pos = exp(-2 pi i pos / 2h) =
// tw[pos M / 2h] for h = 1, 2, 4, ..., M/4 and pos < h, so that the FFT
// stage with half-length h reads adjacent entries for adjacent pos.
template <typename T>
__global__ void k_stage_tw(int M, T* __restrict__ tw) {
  const int H = M >> 1;
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= H - 1) return;
  const int h = 1 << (31 - __clz(idx + 1));
  const int pos = idx + 1 - h;
  tw[H + idx] = tw[pos * (M / (2 * h))];
}

hipError_t launch_stage_tw(int M, double2* t64, float2* t32, hipStream_t st) {
  const int n = M / 2 - 1;
  if (n <= 0) return hipSuccess;
  k_stage_tw<double2><<<(n + 255) / 256, 256, 0, st>>>(M, t64);
  k_stage_tw<float2><<<(n + 255) / 256, 256, 0, st>>>(M, t32);
  return hipGetLastError();
}

// Table of M-th roots of unity exp(sign 2 pi i j / M), j = 0..n-1, FP64 and FP32.
__global__ void k_roots(int M, int n, int sign, double2* __restrict__ o64, float2* __restrict__ o32) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n) return;
  double s, c;
  sincospi((double)sign * 2.0 * (double)j / (double)M, &s, &c);
  if (o64) o64[j] = make_double2(c, s);
  if (o32) o32[j] = make_float2((float)c, (float)s);
}

// --------------------------------------------------------------------------
// ||x||^2 per signal in FP64 (Alg. 1 initialisation) and state reset.  Two
// passes with a fixed summation order: ENERGY_PARTS workgroups per signal
// each reduce one contiguous chunk, then one wave per signal adds the parts.

template <typename XT>
__global__ void __launch_bounds__(256) k_energy_part(const XT* __restrict__ x, const SigDev* __restrict__ sigs,
                                                     double* __restrict__ part) {
  __shared__ double red[4];
  const int s = blockIdx.x, b = blockIdx.y;
  const int64_t L = sigs[s].L, off = sigs[s].x_off;
  const int64_t chunk = (L + ENERGY_PARTS - 1) / ENERGY_PARTS;
  const int64_t i0 = b * chunk, i1 = i0 + chunk < L ? i0 + chunk : L;
  double acc = 0.0;
  for (int64_t i = i0 + threadIdx.x; i < i1; i += 256) {
    const double v = (double)x[off + i];
    acc += v * v;
  }
  for (int o = 32; o; o >>= 1) acc += __shfl_xor(acc, o);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) part[(int64_t)s * ENERGY_PARTS + b] = (red[0] + red[1]) + (red[2] + red[3]);
}

__global__ void __launch_bounds__(64) k_energy_fin(const double* __restrict__ part, SigState* __restrict__ st) {
  const int s = blockIdx.x;
  double acc = threadIdx.x < ENERGY_PARTS ? part[(int64_t)s * ENERGY_PARTS + threadIdx.x] : 0.0;
  for (int o = 32; o; o >>= 1) acc += __shfl_xor(acc, o);
  if (threadIdx.x == 0) {
    SigState z;
    z.E0 = acc;
    z.E = acc;
    z.k = 0;
    z.stop = 0;
    z.pad = 0;
    z.updated = z.blocks = z.groups = 0;
    z.Eout = acc;
    z.kout = 0;
    z.done = 0;
    z.resets = 0;
    st[s] = z;
  }
}

// --------------------------------------------------------------------------
// DGT analysis (Sec. 5): for frame n of system w,
//   rho(m, n) = sum_{t=-gl/2}^{gl/2-1} x(n a + t) g(t) exp(-2 pi i m t / M),
// the length-M DFT of the windowed frame u laid out circularly (t mod M,
// samples that share a slot summed when the window is longer than M).
// u is real, so one complex FFT of length H = M/2 suffices: with
// z(q) = u(2q) + i u(2q+1) and Z = FFT_H(z),
//   rho(m) = (Z(m) + conj Z(H-m)) / 2 + e^{-2 pi i m / M} (Z(m) - conj Z(H-m)) / (2i),
// indices of Z mod H, m = 0..M/2.  One workgroup per frame: bit-reversed load
// into LDS (H complex entries), in-place decimation-in-time stages taken two
// at a time (a radix-2 pair per thread: 4 entries, 3 twiddles, one barrier;
// one plain radix-2 stage first when log2 H is odd), then the unpacking fused
// with the plane write and the max-tree leaves (16 bins per leaf).  LDS entry
// i lives at slot dgt_sw(i) = i + i/32 (one pad entry per 32), which spreads
// the bit-reversed scatter and most butterfly strides over the banks at two
// VALU operations per address (the kernel is bound by VALU issue).  The
// signal is zero beyond L and circular over L_padded.
//
// M = 3 2^k (mode 1): H = 3 P with P a power of two.  The pairs z(3q + r),
// r = 0, 1, 2, are stored as three bit-reversed sub-arrays of length P and
// transformed by the same radix-2 stages (no butterfly group crosses a
// sub-array); the unpacking then combines them, Z(k) = sum_r W_H^{r k}
// Z_r(k mod P) (decimation in time by 3, W_H = e^{-2 pi i / H}).
// Other M (mode 2): the frame is stored in natural order and each bin is the
// defining sum of the DFT, rho(m) = sum_t u(t) e^{-2 pi i m t / M},
// accumulated in FP64 with the phase index m t mod M stepped exactly in
// integers (roots64 = e^{+2 pi i j / M}, j < M); O(M^2) per frame.

// Frame of workgroup blockIdx.x: the hardware deals workgroups to the 8 XCDs
// in turn (workgroup i to XCD i mod 8), so XCD x gets one contiguous run of
// frames; neighbouring frames share samples (a < gl) and output cache lines
// in that XCD's L2.  A bijection on [0, gridDim.x).
__device__ __forceinline__ int64_t xcd_frame() {
  const int64_t i = blockIdx.x, nb = gridDim.x;
  const int64_t q = nb >> 3, r = nb & 7, x = i & 7;
  return x * q + (x < r ? x : r) + (i >> 3);
}

__device__ __forceinline__ int dgt_sw(int i) { return i + (i >> 5); }

// R: arithmetic of the window products and the FFT; O: the plan's
// coefficient type (planes, leaves, selection scores), O = R except for an
// FP32 plan with the FP64 DFT.
template <typename R, typename XT, typename O>
__global__ void __launch_bounds__(256) k_dgt(const XT* __restrict__ x, const SigDev* __restrict__ sigs,
                                             int w, int gl, int a, int M, int mode, int logP, int MR,
                                             const int64_t* __restrict__ frame_prefix, int batch,
                                             const R* __restrict__ win, const Cx<R>* __restrict__ tw,
                                             Cx<O>* __restrict__ planes, Leaf<O>* __restrict__ leaves,
                                             const Cx<O>* __restrict__ gam, int pedantic,
                                             const double2* __restrict__ roots64) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  Cx<R>* buf = reinterpret_cast<Cx<R>*>(smem_raw);
  const bool direct = mode == 2, radix3 = mode == 1;
  const int H = M >> 1, P = radix3 ? H / 3 : H;
  const int logH = direct ? 0 : logP;  // radix-2 stages (of each sub-array)
  // first window position >= -gl/2 of the slot at t: t - floor((t + gl/2) / M) M
  auto first_pos = [&](int t) {
    return t - (mode == 0 ? (t + gl / 2) >> (logP + 1) : floor_div32(t + gl / 2, M)) * M;
  };
  // LDS slot of pair z(q): bit-reversed within its sub-array
  auto slot_of = [&](int q) -> int {
    if (direct) return q;
    const int r = radix3 ? q % 3 : 0, q1 = radix3 ? q / 3 : q;
    return r * P + (logP > 0 ? (int)(__brev((unsigned)q1) >> (32 - logP)) : 0);
  };
  const int64_t f = xcd_frame();
  // signal owning global frame f: last s with frame_prefix[s] <= f
  int lo = 0, hi = batch - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (frame_prefix[mid] <= f) lo = mid;
    else hi = mid - 1;
  }
  const int s = lo;
  const SigDev& S = sigs[s];
  const int64_t n = f - frame_prefix[s];
  // 32-bit sample indices (the plan keeps Lp < 2^30)
  const int L = (int)S.L, Lp = (int)S.Lp;
  const XT* xs = x + S.x_off;
  // sample of window position tt: (n a + tt) mod Lp = base + tt + gl/2, less
  // Lp at most once (n a < Lp, and the plan keeps gl <= Lp / 2)
  int base = (int)n * a - gl / 2;
  if (base < 0) base += Lp;
  const int bd = (int)blockDim.x;
  if (gl <= M) {
    // at most one window position per slot: two slot pairs per thread in
    // flight at a time (H / bd = 2 for M <= 1024)
    for (int q0 = threadIdx.x; q0 < H; q0 += 2 * bd) {
      R v[2][2];
#pragma unroll
      for (int u = 0; u < 2; ++u) {
#pragma unroll
        for (int e = 0; e < 2; ++e) {
          const int i = 2 * (q0 + u * bd) + e;
          const int t = i < H ? i : i - M;
          const int tt = first_pos(t);
          int l = base + (tt + gl / 2);
          if (l >= Lp) l -= Lp;
          // unconditional loads (stand-in sample 0 and window entry 0 where
          // the slot is empty), so that all of them are in flight at once
          const bool ok = q0 + u * bd < H && tt < gl / 2 && l < L;
          const R xv = (R)xs[ok ? (uint32_t)l : 0u], wv = win[ok ? (uint32_t)(tt + gl / 2) : 0u];
          v[u][e] = ok ? xv * wv : (R)0;
        }
      }
#pragma unroll
      for (int u = 0; u < 2; ++u) {
        const int q = q0 + u * bd;
        if (q < H) buf[dgt_sw(slot_of(q))] = Cx<R>{v[u][0], v[u][1]};
      }
    }
  } else {
    for (int q = threadIdx.x; q < H; q += bd) {
      R v2[2];
#pragma unroll
      for (int e = 0; e < 2; ++e) {
        const int i = 2 * q + e;
        const int t = i < H ? i : i - M;
        // window positions t, t + M, ... in [-gl/2, gl/2) fold onto slot i;
        // the first is t - floor((t + gl/2) / M) M
        R v = (R)0;
        for (int tt = first_pos(t); tt < gl / 2; tt += M) {
          int l = base + (tt + gl / 2);
          if (l >= Lp) l -= Lp;
          if (l < L) v += (R)xs[l] * win[tt + gl / 2];
        }
        v2[e] = v;
      }
      buf[dgt_sw(slot_of(q))] = Cx<R>{v2[0], v2[1]};
    }
  }
  __syncthreads();
  const Cx<R>* stw = tw + H;  // stage-major twiddles
  int ls = 1;
  if (logH & 1) {  // stage 1 alone: twiddle 1
    for (int b = threadIdx.x; b < H / 2; b += bd) {
      const int j0 = dgt_sw(2 * b), j1 = dgt_sw(2 * b + 1);
      const Cx<R> u = buf[j0], q = buf[j1];
      buf[j0] = Cx<R>{u.re + q.re, u.im + q.im};
      buf[j1] = Cx<R>{u.re - q.re, u.im - q.im};
    }
    __syncthreads();
    ls = 2;
  }
  for (; ls < logH; ls += 2) {
    // stages ls and ls + 1: sub-transforms of length 2h and 4h, h = 2^(ls-1);
    // e^{-2 pi i pos / 2h} = stw[h - 1 + pos] (lanes read adjacent entries)
    const int h = 1 << (ls - 1);
    for (int b = threadIdx.x; b < H / 4; b += bd) {
      const int pos = b & (h - 1);
      const int i0 = ((b >> (ls - 1)) << (ls + 1)) + pos;
      const int j0 = dgt_sw(i0), j1 = dgt_sw(i0 + h), j2 = dgt_sw(i0 + 2 * h), j3 = dgt_sw(i0 + 3 * h);
      const Cx<R> wa = stw[(uint32_t)(h - 1 + pos)], wb = stw[(uint32_t)(2 * h - 1 + pos)],
                  wc = stw[(uint32_t)(3 * h - 1 + pos)];
      const Cx<R> x0 = buf[j0], x1 = buf[j1], x2 = buf[j2], x3 = buf[j3];
      const R ar = x1.re * wa.re - x1.im * wa.im, ai = x1.re * wa.im + x1.im * wa.re;
      const R cr = x3.re * wa.re - x3.im * wa.im, ci = x3.re * wa.im + x3.im * wa.re;
      const Cx<R> y0{x0.re + ar, x0.im + ai}, y1{x0.re - ar, x0.im - ai};
      const Cx<R> y2{x2.re + cr, x2.im + ci}, y3{x2.re - cr, x2.im - ci};
      const R br = y2.re * wb.re - y2.im * wb.im, bi = y2.re * wb.im + y2.im * wb.re;
      const R dr = y3.re * wc.re - y3.im * wc.im, di = y3.re * wc.im + y3.im * wc.re;
      buf[j0] = Cx<R>{y0.re + br, y0.im + bi};
      buf[j2] = Cx<R>{y0.re - br, y0.im - bi};
      buf[j1] = Cx<R>{y1.re + dr, y1.im + di};
      buf[j3] = Cx<R>{y1.re - dr, y1.im - di};
    }
    __syncthreads();
  }
  // unpack, write the plane row and the leaves: leaf i = maximum of |rho|^2
  // over bins 16 i .. 16 i + 15 (ties to the lowest bin), one DPP row per leaf
  Cx<O>* out = planes + S.coef_base + S.off[w] + n * MR;
  const int lpf = (MR + ROW - 1) >> LOG_ROW;
  Leaf<O>* lf = leaves + S.leaf_base + S.lbase[w] + n * lpf;
  const uint32_t p0 = (uint32_t)(S.off[w] + n * MR);
  const int lane = threadIdx.x & 63;
  // twiddle of bin m (e^{-2 pi i m / M}; -1 at m = H), fetched one pass ahead
  auto twid = [&](int m) -> Cx<R> {
    const Cx<R> t = tw[m < H ? (uint32_t)m : 0u];  // unconditional load
    return m < H ? t : Cx<R>{(R)-1, (R)0};
  };
  Cx<R> tnext = twid((int)threadIdx.x);
  for (int m0 = 0; m0 < lpf * ROW; m0 += blockDim.x) {
    const int m = m0 + threadIdx.x;
    const bool valid = m < MR;
    const Cx<R> t = tnext;
    if (m0 + (int)blockDim.x < lpf * ROW) tnext = twid(m + (int)blockDim.x);
    Cx<O> v = {(O)0, (O)0};
    if (valid && direct) {
      // u(2q) = buf[q].re, u(2q+1) = buf[q].im; phase indices 2 m q and
      // m (2q + 1) mod M, both stepped by 2 m mod M
      const int st2 = (2 * m) % M;
      int ie = 0, io = m;
      double sr = 0.0, si = 0.0;
      for (int q = 0; q < H; ++q) {
        const Cx<R> z = buf[dgt_sw(q)];
        const double2 re = roots64[ie], ro = roots64[io];
        sr += (double)z.re * re.x + (double)z.im * ro.x;
        si -= (double)z.re * re.y + (double)z.im * ro.y;
        ie += st2;
        ie -= ie >= M ? M : 0;
        io += st2;
        io -= io >= M ? M : 0;
      }
      v.re = (O)sr;
      v.im = (O)si;
      out[(uint32_t)m] = v;
    } else if (valid) {
      Cx<R> zk, zr;
      if (radix3) {
        // Z(k) = Z_0(k mod P) + W^k Z_1(k mod P) + W^{2k} Z_2(k mod P),
        // W^j = e^{-2 pi i 2 j / M}: tw[j'] for j' < H, -tw[j' - H] above
        auto twm = [&](int jm) -> Cx<R> {
          const Cx<R> t0 = tw[(uint32_t)(jm < H ? jm : jm - H)];
          return jm < H ? t0 : Cx<R>{-t0.re, -t0.im};
        };
        auto zcomb = [&](int k) -> Cx<R> {
          const int kp = k & (P - 1);
          const Cx<R> a0 = buf[dgt_sw(kp)], a1 = buf[dgt_sw(P + kp)], a2 = buf[dgt_sw(2 * P + kp)];
          int j1 = 2 * k;
          j1 -= j1 >= M ? M : 0;
          int j2 = 2 * j1;
          j2 -= j2 >= M ? M : 0;
          const Cx<R> w1 = twm(j1), w2 = twm(j2);
          return Cx<R>{a0.re + (w1.re * a1.re - w1.im * a1.im) + (w2.re * a2.re - w2.im * a2.im),
                       a0.im + (w1.re * a1.im + w1.im * a1.re) + (w2.re * a2.im + w2.im * a2.re)};
        };
        const int k1 = m < H ? m : m - H, k2 = m == 0 ? 0 : H - m;
        zk = zcomb(k1);
        zr = zcomb(k2 < H ? k2 : k2 - H);
      } else {
        zk = buf[dgt_sw(m & (H - 1))];
        zr = buf[dgt_sw((H - m) & (H - 1))];
      }
      // even part (zk + conj zr) / 2, odd part (zk - conj zr) / (2i)
      const R er = (R)0.5 * (zk.re + zr.re), ei = (R)0.5 * (zk.im - zr.im);
      const R or_ = (R)0.5 * (zk.im + zr.im), oi = (R)0.5 * (zr.re - zk.re);
      v.re = (O)(er + (t.re * or_ - t.im * oi));
      v.im = (O)(ei + (t.re * oi + t.im * or_));
      out[(uint32_t)m] = v;
    }
    const bool ped = pedantic && valid && m != 0 && m != H;
    const O val = sel_score<O>(v.re, v.im, ped ? gam[m] : Cx<O>{(O)0, (O)0}, ped);
    const uint64_t bits = valid ? val_bits(val) : 0ull;
    const uint64_t rm = row_max_bits<O>(bits);
    const uint64_t bal = __ballot(valid && bits == rm);
    const uint32_t rowbits = (uint32_t)(bal >> (lane & ~(ROW - 1))) & 0xFFFFu;
    if (rowbits && lane == (lane & ~(ROW - 1)) + __ffs(rowbits) - 1)
      lf[(uint32_t)m >> LOG_ROW] = make_leaf(KeyOps<O>::make(val, p0 + (uint32_t)m), v.re, v.im);
  }
}

// --------------------------------------------------------------------------
// DGT with the DFT on matrix cores, in split half precision (FP16 or BF16
// pairs hi + lo, products hi*hi + hi*lo + lo*hi, FP32 accumulation).  Same
// result as k_dgt up to the split rounding.  The length-H complex FFT of the
// real-input packing is done as a four-step DFT, H = N1 N2, n = n1 + N1 n2,
// k = N2 k1 + k2:
//   B(n1, k2) = sum_n2 z(n1 + N1 n2) w_N2^{n2 k2}   (GEMM, 16x16x16 MFMA tiles)
//   B(n1, k2) *= w_H^{n1 k2}                           (FP32)
//   Z(N2 k1 + k2) = sum_n1 w_N1^{k1 n1} B(n1, k2)       (GEMM)
// with w_N = exp(-2 pi i / N).  The DFT matrices come split and already laid
// out per MFMA operand (k_dft_tables); N1, N2 <= 128, padded with zeros to
// multiples of 16.  The frame is scaled by a power of two to max |z| <= 1
// before the split, so FP16 does not overflow.  This form (one workgroup per
// frame, unscaled lo halves) serves the sizes the frame-group kernel below
// does not: M <= 128 and M >= 8192, and signals whose sample byte offsets
// need more than 31 bits.

typedef short mf_s4 __attribute__((ext_vector_type(4)));
typedef _Float16 mf_h4 __attribute__((ext_vector_type(4)));
typedef float mf_f4 __attribute__((ext_vector_type(4)));

template <int FMT>  // 0: FP16, 1: BF16
__device__ __forceinline__ uint16_t to_half_bits(float x) {
  if (FMT == 0) return __builtin_bit_cast(uint16_t, (_Float16)x);
  uint32_t u = __float_as_uint(x);
  u += 0x7FFFu + ((u >> 16) & 1u);  // round to nearest even (finite x)
  return (uint16_t)(u >> 16);
}
template <int FMT>
__device__ __forceinline__ float from_half_bits(uint16_t b) {
  if (FMT == 0) return (float)__builtin_bit_cast(_Float16, b);
  return __uint_as_float((uint32_t)b << 16);
}
// x = hi + lo in the half format
template <int FMT>
__device__ __forceinline__ void split_half(float x, uint16_t& hi, uint16_t& lo) {
  hi = to_half_bits<FMT>(x);
  lo = to_half_bits<FMT>(x - from_half_bits<FMT>(hi));
}
template <int FMT>
__device__ __forceinline__ mf_f4 mfma16(mf_s4 a, mf_s4 b, mf_f4 c) {
  if constexpr (FMT == 0)
    return __builtin_amdgcn_mfma_f32_16x16x16f16(__builtin_bit_cast(mf_h4, a), __builtin_bit_cast(mf_h4, b), c, 0,
                                                0, 0);
  else
    return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0);
}
// c += (ah + al)(bh + bl) without al*bl
template <int FMT>
__device__ __forceinline__ mf_f4 mfma_split(mf_s4 ah, mf_s4 al, mf_s4 bh, mf_s4 bl, mf_f4 c) {
  c = mfma16<FMT>(ah, bh, c);
  c = mfma16<FMT>(ah, bl, c);
  return mfma16<FMT>(al, bh, c);
}

// Operand tile (a, b) of the DFT matrix F(r, c) = w_N^{r c} (zero outside N):
// lane l holds F(16 a + 4 (l >> 4) + j, 16 b + (l & 15)), j = 0..3; planes
// re_hi, re_lo, im_hi, im_lo, re_lo 2^11, im_lo 2^11, each T*T*256 halves
// (T = Np/16).  The last two hold the remainders scaled by 2^11 (MFW_LO_SCALE),
// which keeps them out of FP16's subnormal range.
// F is symmetric, so the same tile serves as the B operand of the first GEMM
// (rows n2, columns k2) and, with (a, b) swapped, as the A operand of the
// second (rows k1, columns n1).
template <int FMT>
__global__ void k_dft_tables(int N, int Np, uint16_t* __restrict__ out) {
  const int a = blockIdx.y * blockDim.y + threadIdx.y, b = blockIdx.x * blockDim.x + threadIdx.x;
  if (a >= Np || b >= Np) return;
  double re = 0.0, im = 0.0;
  if (a < N && b < N) {
    const int64_t q = ((int64_t)a * b) % N;
    sincospi(-2.0 * (double)q / (double)N, &im, &re);
  }
  const int T = Np >> 4;
  const int A = a >> 4, qa = a & 15, B = b >> 4;
  const int l = ((qa >> 2) << 4) | (b & 15), j = qa & 3;
  const size_t idx = (((size_t)A * T + B) * 64 + l) * 4 + j;
  const size_t plane = (size_t)Np * Np;
  uint16_t h, lo;
  split_half<FMT>((float)re, h, lo);
  out[0 * plane + idx] = h;
  out[1 * plane + idx] = lo;
  split_half<FMT>((float)im, h, lo);
  out[2 * plane + idx] = h;
  out[3 * plane + idx] = lo;
  const float fr = (float)re, fi = (float)im;
  out[4 * plane + idx] = to_half_bits<FMT>((fr - from_half_bits<FMT>(to_half_bits<FMT>(fr))) * 2048.0f);
  out[5 * plane + idx] = to_half_bits<FMT>((fi - from_half_bits<FMT>(to_half_bits<FMT>(fi))) * 2048.0f);
}

struct TileOp {
  mf_s4 rh, rl, ih, il, nh, nl;  // re, im, -im (hi, lo)
};
__device__ __forceinline__ TileOp load_tile(const uint16_t* __restrict__ tab, int Np, int a, int b, int lane) {
  const int T = Np >> 4;
  const size_t plane = (size_t)Np * Np;
  const size_t idx = (((size_t)a * T + b) * 64 + lane) * 4;
  TileOp t;
  t.rh = *reinterpret_cast<const mf_s4*>(tab + 0 * plane + idx);
  t.rl = *reinterpret_cast<const mf_s4*>(tab + 1 * plane + idx);
  t.ih = *reinterpret_cast<const mf_s4*>(tab + 2 * plane + idx);
  t.il = *reinterpret_cast<const mf_s4*>(tab + 3 * plane + idx);
  typedef uint32_t u2 __attribute__((ext_vector_type(2)));
  t.nh = __builtin_bit_cast(mf_s4, __builtin_bit_cast(u2, t.ih) ^ u2{0x80008000u, 0x80008000u});
  t.nl = __builtin_bit_cast(mf_s4, __builtin_bit_cast(u2, t.il) ^ u2{0x80008000u, 0x80008000u});
  return t;
}

template <int FMT, typename XT>
__global__ void __launch_bounds__(256) k_dgt_mfma(const XT* __restrict__ x, const SigDev* __restrict__ sigs, int w,
                                                  int gl, int a, int M, int MR,
                                                  const int64_t* __restrict__ frame_prefix, int batch,
                                                  const float* __restrict__ win, const Cx<float>* __restrict__ tw,
                                                  int N1, int N2, const uint16_t* __restrict__ F1,
                                                  const uint16_t* __restrict__ F2, Cx<float>* __restrict__ planes,
                                                  Leaf<float>* __restrict__ leaves,
                                                  const Cx<float>* __restrict__ gam, int pedantic) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int H = M >> 1;
  Cx<float>* buf = reinterpret_cast<Cx<float>*>(smem_raw);  // z, then B
  Cx<float>* ybuf = buf + H;                                  // Z
  __shared__ float s_red[4];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = (int)blockDim.x >> 6;
  const int N1p = N1 < 16 ? 16 : N1, N2p = N2 < 16 ? 16 : N2;
  const int64_t f = xcd_frame();
  int lo = 0, hi = batch - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (frame_prefix[mid] <= f) lo = mid;
    else hi = mid - 1;
  }
  const int s = lo;
  const SigDev& S = sigs[s];
  const int64_t n = f - frame_prefix[s];
  const int64_t L = S.L, Lp = S.Lp;
  const XT* xs = x + S.x_off;
  float amax = 0.0f;
  // (n a + tt) mod Lp = base + tt + gl/2, less Lp at most once (gl <= Lp / 2)
  int64_t base = (n * a - gl / 2) % Lp;
  if (base < 0) base += Lp;
  const int logM = __ffs(M) - 1;
  for (int q = threadIdx.x; q < H; q += blockDim.x) {
    float v2[2];
#pragma unroll
    for (int e = 0; e < 2; ++e) {
      const int i = 2 * q + e;
      const int t = i < H ? i : i - M;
      // window positions t, t + M, ... in [-gl/2, gl/2) fold onto slot i
      float v = 0.0f;
      if (gl <= M) {  // at most one position: unconditional loads (stand-ins where none)
        const int tt = t - ((t + gl / 2) >> logM) * M;
        int64_t l = base + (tt + gl / 2);
        if (l >= Lp) l -= Lp;
        const bool ok = tt < gl / 2 && l < L;
        const float xv = (float)xs[ok ? l : 0], wv = win[ok ? tt + gl / 2 : 0];
        v = ok ? xv * wv : 0.0f;
      } else {
        for (int tt = t - ((t + gl / 2) >> logM) * M; tt < gl / 2; tt += M) {
          int64_t l = base + (tt + gl / 2);
          if (l >= Lp) l -= Lp;
          if (l < L) v += (float)xs[l] * win[tt + gl / 2];
        }
      }
      v2[e] = v;
    }
    buf[q].re = v2[0];
    buf[q].im = v2[1];
    amax = fmaxf(amax, fmaxf(fabsf(v2[0]), fabsf(v2[1])));
  }
  // block maximum -> power-of-two scale with max |z| * scale <= 1
  for (int o = 32; o; o >>= 1) amax = fmaxf(amax, __shfl_xor(amax, o));
  if (lane == 0) s_red[wave] = amax;
  __syncthreads();
  amax = s_red[0];
  for (int v = 1; v < nw; ++v) amax = fmaxf(amax, s_red[v]);
  int ex = 0;
  if (amax > 0.0f) frexpf(amax, &ex);
  const float scale = ldexpf(1.0f, -ex), unscale = ldexpf(1.0f, ex);

  // ---- step 1: B = X F_N2 (row blocks of 16 n1), twiddle, in place ----
  const int r16 = lane & 15, k4 = (lane >> 4) * 4;
  for (int rb = wave; rb < (N1p >> 4); rb += nw) {
    const int n1a = 16 * rb + r16;  // A-operand row of this lane
    mf_s4 xr_h[8], xr_l[8], xi_h[8], xi_l[8];
#pragma unroll
    for (int ks = 0; ks < 8; ++ks) {
      if (ks < (N2p >> 4)) {
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const int n2 = 16 * ks + k4 + j;
          Cx<float> v = {0.0f, 0.0f};
          if (n1a < N1 && n2 < N2) v = buf[n1a + N1 * n2];
          uint16_t h0, l0, h1, l1;
          split_half<FMT>(v.re * scale, h0, l0);
          split_half<FMT>(v.im * scale, h1, l1);
          xr_h[ks][j] = (short)h0;
          xr_l[ks][j] = (short)l0;
          xi_h[ks][j] = (short)h1;
          xi_l[ks][j] = (short)l1;
        }
      }
    }
    for (int ct = 0; ct < (N2p >> 4); ++ct) {
      mf_f4 cr = {0.0f, 0.0f, 0.0f, 0.0f}, ci = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
      for (int ks = 0; ks < 8; ++ks) {
        if (ks < (N2p >> 4)) {
          const TileOp F = load_tile(F2, N2p, ks, ct, lane);
          // (xr + i xi)(fr + i fi): re = xr fr + xi (-fi), im = xr fi + xi fr
          cr = mfma_split<FMT>(xr_h[ks], xr_l[ks], F.rh, F.rl, cr);
          cr = mfma_split<FMT>(xi_h[ks], xi_l[ks], F.nh, F.nl, cr);
          ci = mfma_split<FMT>(xr_h[ks], xr_l[ks], F.ih, F.il, ci);
          ci = mfma_split<FMT>(xi_h[ks], xi_l[ks], F.rh, F.rl, ci);
        }
      }
      // lane holds rows n1 = 16 rb + k4 + j of column k2 = 16 ct + r16
      const int k2 = 16 * ct + r16;
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int n1 = 16 * rb + k4 + j;
        if (n1 < N1 && k2 < N2) {
          const int jj = 2 * ((n1 * k2) & (H - 1));  // w_H^{n1 k2} = e^{-2 pi i jj / M}
          Cx<float> t = tw[jj < H ? jj : jj - H];
          if (jj >= H) {
            t.re = -t.re;
            t.im = -t.im;
          }
          Cx<float> o;
          o.re = cr[j] * t.re - ci[j] * t.im;
          o.im = cr[j] * t.im + ci[j] * t.re;
          buf[n1 + N1 * k2] = o;
        }
      }
    }
  }
  __syncthreads();

  // ---- step 2: Z = F_N1 B (column blocks of 16 k2) ----
  for (int ct = wave; ct < (N2p >> 4); ct += nw) {
    const int k2b = 16 * ct + r16;  // B-operand column of this lane
    mf_s4 br_h[8], br_l[8], bi_h[8], bi_l[8];
#pragma unroll
    for (int ks = 0; ks < 8; ++ks) {
      if (ks < (N1p >> 4)) {
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const int n1 = 16 * ks + k4 + j;
          Cx<float> v = {0.0f, 0.0f};
          if (n1 < N1 && k2b < N2) v = buf[n1 + N1 * k2b];
          uint16_t h0, l0, h1, l1;
          split_half<FMT>(v.re, h0, l0);
          split_half<FMT>(v.im, h1, l1);
          br_h[ks][j] = (short)h0;
          br_l[ks][j] = (short)l0;
          bi_h[ks][j] = (short)h1;
          bi_l[ks][j] = (short)l1;
        }
      }
    }
    for (int rt = 0; rt < (N1p >> 4); ++rt) {
      mf_f4 cr = {0.0f, 0.0f, 0.0f, 0.0f}, ci = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
      for (int ks = 0; ks < 8; ++ks) {
        if (ks < (N1p >> 4)) {
          const TileOp F = load_tile(F1, N1p, ks, rt, lane);  // F(k1, n1) tile (rt, ks), F symmetric
          // (fr + i fi)(br + i bi): re = fr br + (-fi) bi, im = fr bi + fi br
          cr = mfma_split<FMT>(F.rh, F.rl, br_h[ks], br_l[ks], cr);
          cr = mfma_split<FMT>(F.nh, F.nl, bi_h[ks], bi_l[ks], cr);
          ci = mfma_split<FMT>(F.rh, F.rl, bi_h[ks], bi_l[ks], ci);
          ci = mfma_split<FMT>(F.ih, F.il, br_h[ks], br_l[ks], ci);
        }
      }
      const int k2 = 16 * ct + r16;
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int k1 = 16 * rt + k4 + j;
        if (k1 < N1 && k2 < N2) ybuf[N2 * k1 + k2] = Cx<float>{cr[j] * unscale, ci[j] * unscale};
      }
    }
  }
  __syncthreads();

  // ---- unpack the real-input packing, plane row, leaves ----
  Cx<float>* out = planes + S.coef_base + S.off[w] + n * MR;
  const int lpf = (MR + ROW - 1) >> LOG_ROW;
  Leaf<float>* lf = leaves + S.leaf_base + S.lbase[w] + n * lpf;
  const uint32_t p0 = (uint32_t)(S.off[w] + n * MR);
  for (int m0 = 0; m0 < lpf * ROW; m0 += blockDim.x) {
    const int m = m0 + threadIdx.x;
    const bool valid = m < MR;
    Cx<float> v = {0.0f, 0.0f};
    if (valid) {
      const Cx<float> zk = ybuf[m & (H - 1)], zr = ybuf[(H - m) & (H - 1)];
      const float er = 0.5f * (zk.re + zr.re), ei = 0.5f * (zk.im - zr.im);
      const float or_ = 0.5f * (zk.im + zr.im), oi = 0.5f * (zr.re - zk.re);
      Cx<float> t = {-1.0f, 0.0f};
      if (m < H) t = tw[m];
      v.re = er + (t.re * or_ - t.im * oi);
      v.im = ei + (t.re * oi + t.im * or_);
      out[m] = v;
    }
    const bool ped = pedantic && valid && m != 0 && m != H;
    const float val = sel_score<float>(v.re, v.im, ped ? gam[m] : Cx<float>{0.0f, 0.0f}, ped);
    const uint64_t bits = valid ? val_bits(val) : 0ull;
    const uint64_t rm = row_max_bits<float>(bits);
    const uint64_t bal = __ballot(valid && bits == rm);
    const uint32_t rowbits = (uint32_t)(bal >> (lane & ~(ROW - 1))) & 0xFFFFu;
    if (rowbits && lane == (lane & ~(ROW - 1)) + __ffs(rowbits) - 1)
      lf[m >> LOG_ROW] = make_leaf(KeyOps<float>::make(val, p0 + (uint32_t)m), v.re, v.im);
  }
}

// --------------------------------------------------------------------------
// The same split-precision DGT for H = M/2 = 128 .. 2048, one wave per group
// of frames, each wave looping over many groups.  A wave stacks FPW = 64 / N1
// frames into the 64 rows (frame, n1) of the first GEMM; the DFT matrices
// (hi planes and 2^11-scaled lo planes of re and im, in MFMA operand order),
// the twiddles w_H^{n1 k2} of every (n1, k2) tile, the unpacking twiddles and
// the window are staged in LDS once per workgroup.  A 16x16 MFMA result tile (lane: column, four consecutive rows)
// has the lane layout of a 16x16x16 B operand (lane: column, four
// consecutive k), so B(n1, k2) passes from the first GEMM to the second in
// registers, after its twiddle and split.  Z goes through a per-wave LDS
// buffer for the real-input unpacking, which pairs bins m and H - m.  Waves
// do not synchronise after the staging.

typedef uint32_t mfw_u2 __attribute__((ext_vector_type(2)));
typedef float mfw_f2 __attribute__((ext_vector_type(2)));

// The lo half of a split operand carries the remainder scaled by 2^11, so
// that it stays in FP16's normal range (a remainder below 2^-14 would be
// quantised to 2^-24 absolute, the dominant error of unscaled pairs); the
// products with a lo factor are summed apart and scaled back by 2^-11.
constexpr float MFW_LO_SCALE = 2048.0f, MFW_LO_UNSCALE = 1.0f / 2048.0f;

// (a, b) -> hi: both rounded to the half format (nearest even, packed);
// lo: the remainders a - hi_a, b - hi_b (exact in FP32) times 2^11, rounded
// likewise.
template <int FMT>
__device__ __forceinline__ void split_pair(float a, float b, uint32_t& hi, uint32_t& lo) {
  if constexpr (FMT == 0) {
    typedef _Float16 h2 __attribute__((ext_vector_type(2)));
    const h2 h = __builtin_convertvector(mfw_f2{a, b}, h2);
    const mfw_f2 hb = __builtin_convertvector(h, mfw_f2);
    hi = __builtin_bit_cast(uint32_t, h);
    lo = __builtin_bit_cast(uint32_t, __builtin_convertvector(
                                          mfw_f2{(a - hb.x) * MFW_LO_SCALE, (b - hb.y) * MFW_LO_SCALE}, h2));
  } else {
    typedef __bf16 b2 __attribute__((ext_vector_type(2)));
    hi = __builtin_bit_cast(uint32_t, __builtin_convertvector(mfw_f2{a, b}, b2));
    const float ha = __uint_as_float(hi << 16), hb = __uint_as_float(hi & 0xFFFF0000u);
    lo = __builtin_bit_cast(uint32_t, __builtin_convertvector(
                                          mfw_f2{(a - ha) * MFW_LO_SCALE, (b - hb) * MFW_LO_SCALE}, b2));
  }
}

// A complex 16x16x16 operand split into hi and lo halves: four consecutive
// k (A) or rows (B) per lane, two per 32-bit word.
struct SplitOp {
  mf_s4 rh, rl, ih, il;
};
__device__ __forceinline__ mf_s4 mfw_pack(uint32_t p0, uint32_t p1) {
  return __builtin_bit_cast(mf_s4, mfw_u2{p0, p1});
}
__device__ __forceinline__ mf_s4 mfw_neg(mf_s4 v) {  // both halves of both words
  return __builtin_bit_cast(mf_s4, __builtin_bit_cast(mfw_u2, v) ^ mfw_u2{0x80008000u, 0x80008000u});
}
template <int FMT>
__device__ __forceinline__ SplitOp split_op(const float (&re)[4], const float (&im)[4]) {
  uint32_t h0, l0, h1, l1;
  SplitOp o;
  split_pair<FMT>(re[0], re[1], h0, l0);
  split_pair<FMT>(re[2], re[3], h1, l1);
  o.rh = mfw_pack(h0, h1);
  o.rl = mfw_pack(l0, l1);
  split_pair<FMT>(im[0], im[1], h0, l0);
  split_pair<FMT>(im[2], im[3], h1, l1);
  o.ih = mfw_pack(h0, h1);
  o.il = mfw_pack(l0, l1);
  return o;
}
// Table tile (4 planes, 64 lanes each) from LDS
__device__ __forceinline__ SplitOp lds_op(const mfw_u2* t, int lane) {
  SplitOp o;
  o.rh = __builtin_bit_cast(mf_s4, t[lane]);
  o.rl = __builtin_bit_cast(mf_s4, t[64 + lane]);
  o.ih = __builtin_bit_cast(mf_s4, t[128 + lane]);
  o.il = __builtin_bit_cast(mf_s4, t[192 + lane]);
  return o;
}
// Two consecutive K = 16 operands as one K = 32 operand of the double-rate
// 16x16x32 MFMA: lane group g holds k-slots 8 g .. 8 g + 7 of A and B alike,
// here the four k of the first step, then the four of the second, so the
// product sums the same terms as the two K = 16 products.
typedef short mf_s8 __attribute__((ext_vector_type(8)));
struct SplitOp8 {
  mf_s8 rh, rl, ih, il;
};
__device__ __forceinline__ mf_s8 mf_cat(mf_s4 a, mf_s4 b) { return __builtin_shufflevector(a, b, 0, 1, 2, 3, 4, 5, 6, 7); }
__device__ __forceinline__ SplitOp8 mf_cat(const SplitOp& a, const SplitOp& b) {
  return SplitOp8{mf_cat(a.rh, b.rh), mf_cat(a.rl, b.rl), mf_cat(a.ih, b.ih), mf_cat(a.il, b.il)};
}
__device__ __forceinline__ mf_s8 mfw_neg(mf_s8 v) {
  typedef uint32_t u4 __attribute__((ext_vector_type(4)));
  return __builtin_bit_cast(mf_s8, __builtin_bit_cast(u4, v) ^ u4{0x80008000u, 0x80008000u, 0x80008000u, 0x80008000u});
}
template <int FMT>
__device__ __forceinline__ mf_f4 mfma32(mf_s8 a, mf_s8 b, mf_f4 c) {
  if constexpr (FMT == 0) {
    typedef _Float16 h8 __attribute__((ext_vector_type(8)));
    return __builtin_amdgcn_mfma_f32_16x16x32_f16(__builtin_bit_cast(h8, a), __builtin_bit_cast(h8, b), c, 0, 0, 0);
  } else {
    typedef __bf16 b8 __attribute__((ext_vector_type(8)));
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(b8, a), __builtin_bit_cast(b8, b), c, 0, 0, 0);
  }
}
// Accumulators of one complex output tile: hi*hi products, and products
// with one lo factor (scaled by 2^11); value = h + 2^-11 l.
struct CAcc {
  mf_f4 rh, rl, ih, il;
};
__device__ __forceinline__ void cacc_zero(CAcc& a) {
  a.rh = a.rl = a.ih = a.il = mf_f4{0.0f, 0.0f, 0.0f, 0.0f};
}
__device__ __forceinline__ float cacc_re(const CAcc& a, int j) { return fmaf(a.rl[j], MFW_LO_UNSCALE, a.rh[j]); }
__device__ __forceinline__ float cacc_im(const CAcc& a, int j) { return fmaf(a.il[j], MFW_LO_UNSCALE, a.ih[j]); }
template <int FMT, typename V>
__device__ __forceinline__ mf_f4 mfw_mma(V a, V b, mf_f4 c) {
  if constexpr (sizeof(V) == 16) return mfma32<FMT>(a, b, c);
  else return mfma16<FMT>(a, b, c);
}
// (a + i b)(c + i d) for split complex operands P (A side) and Q (B side),
// re = ac - bd, im = ad + bc, each real product hi hi + (hi lo + lo hi)
template <int FMT, typename Op>
__device__ __forceinline__ void cmac(const Op& P, const Op& Q, CAcc& a) {
  const auto qnh = mfw_neg(Q.ih), qnl = mfw_neg(Q.il);
  a.rh = mfw_mma<FMT>(P.rh, Q.rh, a.rh);
  a.rh = mfw_mma<FMT>(P.ih, qnh, a.rh);
  a.rl = mfw_mma<FMT>(P.rh, Q.rl, a.rl);
  a.rl = mfw_mma<FMT>(P.rl, Q.rh, a.rl);
  a.rl = mfw_mma<FMT>(P.ih, qnl, a.rl);
  a.rl = mfw_mma<FMT>(P.il, qnh, a.rl);
  a.ih = mfw_mma<FMT>(P.rh, Q.ih, a.ih);
  a.ih = mfw_mma<FMT>(P.ih, Q.rh, a.ih);
  a.il = mfw_mma<FMT>(P.rh, Q.il, a.il);
  a.il = mfw_mma<FMT>(P.rl, Q.ih, a.il);
  a.il = mfw_mma<FMT>(P.ih, Q.rl, a.il);
  a.il = mfw_mma<FMT>(P.il, Q.rh, a.il);
}
// Orders this wave's LDS accesses before and after (a compiler barrier; one
// wave's LDS operations complete in order).
__device__ __forceinline__ void wave_lds_fence() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <int LN1, int LN2>
struct MfwShape {
  static constexpr int N1 = 1 << LN1, N2 = 1 << LN2, H = N1 * N2, M = 2 * H;
  static constexpr int T1 = N1 / 16;             // 16-row tiles per frame
  static constexpr int FPW = 4 / T1;             // frames per wave (64 rows)
  static constexpr int N2P = N2 < 16 ? 16 : N2;  // K and columns of the first GEMM, padded
  static constexpr int T2 = N2P / 16;
  static constexpr int ZP = N2 + 4;              // Z row pitch: 4 mod 8 complex, conflict-free stores
  static constexpr int ZW = FPW * N1 * ZP;       // Z entries per wave
  static constexpr int IT = (H + ROW + 63) / 64;  // unpacking passes per frame (H + 1 bins, whole rows)
  // DFT tiles, step-1 twiddles, Z of the 4 waves, unpacking twiddles, window
  static constexpr size_t lds_bytes() {
    return (size_t)(T1 * T1 + T2 * T2) * 4 * 64 * 8 + (size_t)T1 * T2 * 2 * 64 * 16 + (size_t)4 * ZW * 8 +
           (size_t)H * 8 + (size_t)M * 4;
  }
  // waves per SIMD that the LDS admits (four 256-thread workgroups at most),
  // asked of the register allocator
  static constexpr int WPE = lds_bytes() <= 40 * 1024 ? 4 : (lds_bytes() <= 53 * 1024 ? 3 : (lds_bytes() <= 80 * 1024 ? 2 : 1));
  static_assert(N1 >= 16 && N1 <= 64 && N2 >= 8 && N2 <= N1, "frame-group DGT shape");
};

// Frame of a frame group: signal, index within the signal, present.
struct MfwFrame {
  int s, n;
  bool ok;
};

__device__ __forceinline__ __amdgpu_buffer_rsrc_t mfw_rsrc(const void* p, uint32_t bytes) {
  // raw (unstrided) buffer: accesses at or past `bytes` read 0 and write nothing
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), (short)0, (int)bytes, 0x00020000);
}

template <int FMT, typename XT, int LN1, int LN2>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(MfwShape<LN1, LN2>::WPE)))
k_dgt_mfw(const XT* __restrict__ x, const SigDev* __restrict__ sigs, int w,
                                                 int gl, int a, int MR, const int64_t* __restrict__ frame_prefix,
                                                 int batch, int64_t frames, const float* __restrict__ win,
                                                 const Cx<float>* __restrict__ tw, const uint16_t* __restrict__ F1g,
                                                 const uint16_t* __restrict__ F2g, Cx<float>* __restrict__ planes,
                                                 Leaf<float>* __restrict__ leaves, const Cx<float>* __restrict__ gam,
                                                 int pedantic) {
  using Sh = MfwShape<LN1, LN2>;
  constexpr int N1 = Sh::N1, N2 = Sh::N2, H = Sh::H, M = Sh::M, T1 = Sh::T1, FPW = Sh::FPW, N2P = Sh::N2P,
                T2 = Sh::T2, ZP = Sh::ZP;
  constexpr uint32_t XB = sizeof(XT);
  constexpr bool PF = XB == 4;  // FP32 samples: the next group's loads fly during this group's GEMMs
  extern __shared__ __align__(16) unsigned char smem_raw[];
  mfw_u2* sF1 = reinterpret_cast<mfw_u2*>(smem_raw);  // T1 x T1 tiles, 4 planes of 64 lanes
  mfw_u2* sF2 = sF1 + T1 * T1 * 256;                   // T2 x T2 tiles
  float4* sTw = reinterpret_cast<float4*>(sF2 + T2 * T2 * 256);  // T1 x T2 tiles, 2 x 64 lanes
  Cx<float>* sZ = reinterpret_cast<Cx<float>*>(sTw + T1 * T2 * 128);  // 4 waves x ZW
  Cx<float>* sU = sZ + 4 * Sh::ZW;                                     // e^{-2 pi i m / M}, m < H
  float* sW = reinterpret_cast<float*>(sU + H);                        // window entries < M (0 past gl)
  // the wave index as a uniform value, so that everything derived from the
  // frame group (signal, buffer descriptors) stays in scalar registers
  const int lane = threadIdx.x & 63, wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  const int c = lane & 15, g = lane >> 4;

  // ---- staging (global tables: plane p at p Np^2 halves, tile t at 256 t) ----
  {
    const mfw_u2* g1 = reinterpret_cast<const mfw_u2*>(F1g);
    const mfw_u2* g2 = reinterpret_cast<const mfw_u2*>(F2g);
    // LDS planes re_hi, re_lo 2^11, im_hi, im_lo 2^11 = global planes 0, 4, 2, 5
    auto gplane = [](int p) { return (p & 1) ? 4 + (p >> 1) : p; };
    for (int i = threadIdx.x; i < T1 * T1 * 256; i += 256)
      sF1[i] = g1[gplane(i >> 6 & 3) * (N1 * N1 / 4) + (i >> 8) * 64 + (i & 63)];
    for (int i = threadIdx.x; i < T2 * T2 * 256; i += 256)
      sF2[i] = g2[gplane(i >> 6 & 3) * (N2P * N2P / 4) + (i >> 8) * 64 + (i & 63)];
    // tile (r, cb), half p: lane l holds w_H^{n1 k2} for n1 = 16 r + 4 (l >> 4)
    // + 2 p + {0, 1}, k2 = 16 cb + (l & 15) (0 for padding columns)
    for (int i = threadIdx.x; i < T1 * T2 * 128; i += 256) {
      const int l = i & 63, p = i >> 6 & 1, t = i >> 7;
      const int r = t / T2, cb = t - r * T2, k2 = 16 * cb + (l & 15);
      float v[4];
#pragma unroll
      for (int u = 0; u < 2; ++u) {
        const int n1 = 16 * r + 4 * (l >> 4) + 2 * p + u;
        Cx<float> z = {0.0f, 0.0f};
        if (k2 < N2) {
          const int e = 2 * ((n1 * k2) & (H - 1));  // e^{-2 pi i e / M}
          z = tw[e < H ? e : e - H];
          if (e >= H) z = Cx<float>{-z.re, -z.im};
        }
        v[2 * u] = z.re;
        v[2 * u + 1] = z.im;
      }
      sTw[i] = make_float4(v[0], v[1], v[2], v[3]);
    }
    for (int i = threadIdx.x; i < H; i += 256) sU[i] = tw[i];
    for (int i = threadIdx.x; i < M; i += 256) sW[i] = i < gl ? win[i] : 0.0f;
  }
  __syncthreads();

  // ---- frame groups: XCD x (workgroups x, x + 8, ...) takes a contiguous
  // run of groups in proportion to its workgroups; its waves interleave ----
  const int64_t NG = (frames + FPW - 1) / FPW;
  const int nb = (int)gridDim.x, xcd = (int)(blockIdx.x & 7);
  const int nbx = (nb >> 3) + (xcd < (nb & 7) ? 1 : 0);
  const int before = xcd * (nb >> 3) + (xcd < (nb & 7) ? xcd : (nb & 7));
  const int64_t grp_hi = NG * (before + nbx) / nb;
  const int nwx = nbx * 4;
  int64_t grp = NG * before / nb + (int64_t)(blockIdx.x >> 3) * 4 + wave;
  Cx<float>* zw = sZ + wave * Sh::ZW;
  const int lpf = (MR + ROW - 1) >> LOG_ROW;
  const int KW = (gl + M - 1) / M;  // window entries per slot (more than one: folded window)
  const __amdgpu_buffer_rsrc_t wrs = mfw_rsrc(win, (uint32_t)gl * 4u);

  // signal of frame f (frames of a wave only increase): last s with
  // frame_prefix[s] <= f, found once by bisection, then by stepping forward
  int scur = 0;
  if (grp < grp_hi) {
    const int64_t f = grp * FPW;
    int lo = 0, hi = batch - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (frame_prefix[mid] <= f) lo = mid;
      else hi = mid - 1;
    }
    scur = lo;
  }
  auto locate = [&](int64_t gq, MfwFrame (&fi)[FPW]) {
#pragma unroll
    for (int fr = 0; fr < FPW; ++fr) {
      const int64_t f = gq * FPW + fr;
      fi[fr].ok = f < frames;
      if (fi[fr].ok)
        while (scur + 1 < batch && frame_prefix[scur + 1] <= f) ++scur;
      fi[fr].s = scur;
      fi[fr].n = fi[fr].ok ? (int)(f - frame_prefix[scur]) : 0;
    }
  };
  // Slot i = 2 (n1 + N1 n2) + e of a frame (A operand row n1 = 16 r + c, k =
  // n2 = 16 ks + 4 g + j, z(n1 + N1 n2) = u(2q) + i u(2q + 1)) holds window
  // entries wi + k M < gl, wi = (i + gl/2) mod M, times the samples
  // (n a - gl/2 + wi + k M) mod Lp.  Range-checked buffer loads read 0 past the
  // signal's L samples (all of them for an absent frame), so the samples load
  // without tests; only entries inside the window need the wrap, and they lie
  // below Lp + Lp/2, so one conditional subtraction suffices.
  // per-lane parts of the slot and bin indices; passed through an empty asm
  // at the top of each group so that the compiler recomputes the indices
  // derived from them instead of keeping dozens of them live across groups
  int lbase = 2 * (c + N1 * 4 * g) + gl / 2, lnv = lane;
  auto wslot = [&](int r, int ks, int j, int e) -> uint32_t {
    return (uint32_t)(lbase + 2 * (16 * r + N1 * (16 * ks + j)) + e) & (uint32_t)(M - 1);
  };
  struct Src {
    __amdgpu_buffer_rsrc_t rs;
    uint32_t bb, lpb;
  };
  auto source = [&](const MfwFrame& F) -> Src {
    const SigDev& S = sigs[F.s];
    const int Lp = (int)S.Lp;
    int base = F.n * a - gl / 2;
    if (base < 0) base += Lp;
    return Src{mfw_rsrc(x + S.x_off, F.ok ? (uint32_t)S.L * XB : 0u), (uint32_t)base * XB, (uint32_t)Lp * XB};
  };
  auto sample = [&](const Src& q, uint32_t wi) -> float {
    uint32_t lb = q.bb + wi * XB;
    lb = min(lb, lb - q.lpb);
    if constexpr (XB == 4)
      return __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(q.rs, (int)lb, 0, 0));
    else
      return (float)__builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(q.rs, (int)lb, 0, 0));
  };
  auto issue = [&](const MfwFrame (&fi)[FPW], float (&xr)[4][T2][4][2]) {
#pragma unroll
    for (int rt = 0; rt < 4; ++rt) {
      const Src q = source(fi[rt / T1]);
#pragma unroll
      for (int ks = 0; ks < T2; ++ks)
#pragma unroll
        for (int j = 0; j < 4; ++j)
#pragma unroll
          for (int e = 0; e < 2; ++e) xr[rt][ks][j][e] = sample(q, wslot(rt % T1, ks, j, e));
    }
  };

  MfwFrame cur[FPW];
  float xr[4][T2][4][2];
  if (grp < grp_hi) {
    locate(grp, cur);
    if (PF) issue(cur, xr);
  }
  for (; grp < grp_hi; grp += nwx) {
    asm volatile("" : "+v"(lbase), "+v"(lnv));
    if (!PF) issue(cur, xr);
    // ---- window products (first entry from LDS, folded entries from global) ----
#pragma unroll
    for (int rt = 0; rt < 4; ++rt)
#pragma unroll
      for (int ks = 0; ks < T2; ++ks)
#pragma unroll
        for (int j = 0; j < 4; ++j)
#pragma unroll
          for (int e = 0; e < 2; ++e) xr[rt][ks][j][e] *= sW[wslot(rt % T1, ks, j, e)];
    if (KW > 1) {
#pragma unroll
      for (int rt = 0; rt < 4; ++rt) {
        const Src q = source(cur[rt / T1]);
#pragma unroll 1
        for (int k = 1; k < KW; ++k)
#pragma unroll
          for (int ks = 0; ks < T2; ++ks)
#pragma unroll
            for (int j = 0; j < 4; ++j)
#pragma unroll
              for (int e = 0; e < 2; ++e) {
                const uint32_t wk = wslot(rt % T1, ks, j, e) + (uint32_t)(k * M);
                const float wq = __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(wrs, (int)(wk * 4u), 0, 0));
                xr[rt][ks][j][e] += sample(q, wk) * wq;
              }
      }
    }
    // ---- per-frame power-of-two scale (max |z| * scale in [1/2, 1)), split.
    // Slots n2 >= N2 (N2 = 8: lanes g >= 2) hold other samples of the frame;
    // the zero rows n2 >= N2 of the padded F_N2 cancel them, and they are
    // left out of the maximum. ----
    float sc[FPW], usc[FPW];
#pragma unroll
    for (int fr = 0; fr < FPW; ++fr) {
      float m_ = 0.0f;
#pragma unroll
      for (int r = 0; r < T1; ++r)
#pragma unroll
        for (int ks = 0; ks < T2; ++ks)
#pragma unroll
          for (int j = 0; j < 4; ++j) {
            const float v = fmaxf(fabsf(xr[fr * T1 + r][ks][j][0]), fabsf(xr[fr * T1 + r][ks][j][1]));
            m_ = fmaxf(m_, (N2 >= 16 || 16 * ks + 4 * g + j < N2) ? v : 0.0f);
          }
      for (int o = 32; o; o >>= 1) m_ = fmaxf(m_, __shfl_xor(m_, o));
      int ex = 0;
      if (m_ > 0.0f) frexpf(m_, &ex);
      sc[fr] = ldexpf(1.0f, -ex);
      usc[fr] = ldexpf(1.0f, ex);
    }
    SplitOp xa[4][T2];
#pragma unroll
    for (int rt = 0; rt < 4; ++rt)
#pragma unroll
      for (int ks = 0; ks < T2; ++ks) {
        const float s_ = sc[rt / T1];
        float re[4], im[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          re[j] = xr[rt][ks][j][0] * s_;
          im[j] = xr[rt][ks][j][1] * s_;
        }
        xa[rt][ks] = split_op<FMT>(re, im);
      }

    // ---- step 1: B = X F_N2, all 64 rows, columns k2 = 16 cb + c; twiddle
    // w_H^{n1 k2} and split: lane holds rows n1 = 16 r + 4 g + j of column
    // k2, the B operand layout of step 2 ----
    SplitOp bq[T2][4];
#pragma unroll
    for (int cb = 0; cb < T2; ++cb)
#pragma unroll
      for (int rt = 0; rt < 4; ++rt) {
        // one output tile at a time (its accumulators alone live); the table
        // tiles are LDS reads, repeated per row block
        CAcc acc;
        cacc_zero(acc);
        if constexpr (T2 % 2 == 0) {  // K = 32 steps: pairs of 16-row blocks of n2
#pragma unroll
          for (int ks = 0; ks < T2; ks += 2)
            cmac<FMT>(mf_cat(xa[rt][ks], xa[rt][ks + 1]),
                      mf_cat(lds_op(sF2 + (ks * T2 + cb) * 256, lane), lds_op(sF2 + ((ks + 1) * T2 + cb) * 256, lane)),
                      acc);  // F(n2, k2)
        } else {
#pragma unroll
          for (int ks = 0; ks < T2; ++ks) cmac<FMT>(xa[rt][ks], lds_op(sF2 + (ks * T2 + cb) * 256, lane), acc);
        }
        const int r = rt % T1;
        const float4 w01 = sTw[((r * T2 + cb) * 2) * 64 + lane], w23 = sTw[((r * T2 + cb) * 2 + 1) * 64 + lane];
        const float tr[4] = {w01.x, w01.z, w23.x, w23.z}, ti[4] = {w01.y, w01.w, w23.y, w23.w};
        float re[4], im[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const float cr = cacc_re(acc, j), ci = cacc_im(acc, j);
          re[j] = cr * tr[j] - ci * ti[j];
          im[j] = cr * ti[j] + ci * tr[j];
        }
        bq[cb][rt] = split_op<FMT>(re, im);
      }

    // ---- the next group's samples load during step 2 and the unpacking ----
    MfwFrame nxt[FPW];
    if (grp + nwx < grp_hi) {
      locate(grp + nwx, nxt);
      if (PF) issue(nxt, xr);
    }

    // ---- step 2: Z = F_N1 B, one 16-row block k1 = 16 r2 + 4 g + j and one
    // frame at a time ----
#pragma unroll 1
    for (int r2 = 0; r2 < T1; ++r2)
#pragma unroll
      for (int fr = 0; fr < FPW; ++fr) {
        CAcc za[T2];
#pragma unroll
        for (int cb = 0; cb < T2; ++cb) cacc_zero(za[cb]);
        if constexpr (T1 % 2 == 0) {  // K = 32 steps: pairs of 16-row blocks of n1
#pragma unroll
          for (int ks2 = 0; ks2 < T1; ks2 += 2) {
            const SplitOp8 F = mf_cat(lds_op(sF1 + (ks2 * T1 + r2) * 256, lane),
                                      lds_op(sF1 + ((ks2 + 1) * T1 + r2) * 256, lane));  // F(n1, k1)
#pragma unroll
            for (int cb = 0; cb < T2; ++cb)
              cmac<FMT>(F, mf_cat(bq[cb][fr * T1 + ks2], bq[cb][fr * T1 + ks2 + 1]), za[cb]);
          }
        } else {
#pragma unroll
          for (int ks2 = 0; ks2 < T1; ++ks2) {
            const SplitOp F = lds_op(sF1 + (ks2 * T1 + r2) * 256, lane);  // F(n1, k1) = F(k1, n1)
#pragma unroll
            for (int cb = 0; cb < T2; ++cb) cmac<FMT>(F, bq[cb][fr * T1 + ks2], za[cb]);
          }
        }
#pragma unroll
        for (int cb = 0; cb < T2; ++cb) {
          const int k2 = 16 * cb + c;
          if (N2 >= 16 || k2 < N2) {
#pragma unroll
            for (int j = 0; j < 4; ++j)
              zw[(fr * N1 + 16 * r2 + 4 * g + j) * ZP + k2] =
                  Cx<float>{cacc_re(za[cb], j) * usc[fr], cacc_im(za[cb], j) * usc[fr]};
          }
        }
      }
    wave_lds_fence();

    // ---- unpack the real-input packing, plane rows, leaves: range-checked
    // buffer stores drop the lanes past bin H and the non-maximal lanes of a
    // row, so the passes run without branches.  Without pedantic selection
    // the passes load nothing from global memory, so they never wait for the
    // next group's samples. ----
    auto unpack = [&](auto ped_c) {
      constexpr bool PED = decltype(ped_c)::value;
#pragma unroll
      for (int fr = 0; fr < FPW; ++fr) {
        if (!cur[fr].ok) continue;  // wave-uniform
        const SigDev& S = sigs[cur[fr].s];
        const int64_t n = cur[fr].n;
        const __amdgpu_buffer_rsrc_t ors = mfw_rsrc(planes + S.coef_base + S.off[w] + n * MR, (uint32_t)MR * 8u);
        const __amdgpu_buffer_rsrc_t lrs =
            mfw_rsrc(leaves + S.leaf_base + S.lbase[w] + n * lpf, (uint32_t)lpf * (uint32_t)sizeof(Leaf<float>));
        const uint32_t p0 = (uint32_t)(S.off[w] + n * MR);
        const Cx<float>* zf = zw + fr * N1 * ZP;
        auto zat = [&](int k) { return zf[k + 4 * (k >> LN2)]; };  // row pitch ZP = N2 + 4
#pragma unroll
        for (int it = 0; it < Sh::IT; ++it) {
          const int m = 64 * it + lnv;
          const bool valid = m <= H;
          // e^{-2 pi i m / M}; bin H takes -1 = -e^0 (a sign, not a branch, so
          // that the passes form one block the scheduler can interleave)
          const Cx<float> tu = sU[m & (H - 1)];
          const float sg = m == H ? -1.0f : 1.0f;
          const Cx<float> t = {tu.re * sg, tu.im * sg};
          const Cx<float> zk = zat(m & (H - 1)), zr_ = zat((H - m) & (H - 1));
          // even part (zk + conj zr) / 2, odd part (zk - conj zr) / (2i)
          const float er = 0.5f * (zk.re + zr_.re), ei = 0.5f * (zk.im - zr_.im);
          const float or_ = 0.5f * (zk.im + zr_.im), oi = 0.5f * (zr_.re - zk.re);
          Cx<float> v;
          v.re = er + (t.re * or_ - t.im * oi);
          v.im = ei + (t.re * oi + t.im * or_);
          __builtin_amdgcn_raw_buffer_store_b64(mfw_u2{__float_as_uint(v.re), __float_as_uint(v.im)}, ors, m * 8,
                                                0, 0);
          float val;
          if constexpr (PED) {
            const mfw_u2 gb = __builtin_amdgcn_raw_buffer_load_b64(mfw_rsrc(gam, (uint32_t)MR * 8u), m * 8, 0, 0);
            val = sel_score<float>(v.re, v.im, Cx<float>{__uint_as_float(gb.x), __uint_as_float(gb.y)},
                                   m != 0 && m != H);
          } else {
            val = v.re * v.re + v.im * v.im;
          }
          const uint64_t bits = valid ? val_bits(val) : 0ull;
          const uint64_t rm = row_max_bits<float>(bits);
          const uint64_t bal = __ballot(valid && bits == rm);
          const uint32_t rowbits = (uint32_t)(bal >> (lnv & ~(ROW - 1))) & 0xFFFFu;
          const bool wr = rowbits && lnv == (lnv & ~(ROW - 1)) + __ffs(rowbits) - 1;
          const uint64_t key = KeyOps<float>::make(val, p0 + (uint32_t)m);
          __builtin_amdgcn_raw_buffer_store_b64(mfw_u2{(uint32_t)key, (uint32_t)(key >> 32)}, lrs,
                                                wr ? (m >> LOG_ROW) * 8 : 0x7FFFFFF8, 0, 0);
        }
      }
    };
    if (pedantic) unpack(std::true_type{});
    else unpack(std::false_type{});
    wave_lds_fence();  // the next group's Z stores follow this group's reads
#pragma unroll
    for (int fr = 0; fr < FPW; ++fr) cur[fr] = nxt[fr];
  }
}

// --------------------------------------------------------------------------
// The MP loop (Alg. 1 with Eq. approxResDef, the real-atom pairs of Sec. 5
// and the residual update of Alg. 3).  One persistent workgroup per signal;
// signals come from a queue, longest first.
//
// Tree: leaves (16 bins of one frame, global memory) -> groups of G leaves
// (LDS) -> root (reduced from the group keys).
//
// Per selection:
//   1. wave 0: root from the group keys; rho(p) sits beside its group key;
//      decode p -> (v, k, j); for every target system w the kernel box covers
//      frames n with |n a_w - j a_v| <= dbox a_min and the bin hull where
//      mu = m r_w -/+ k r_v lies in [mu_lo, mu_hi]; the covered leaves form a
//      (frame x 16-bin block) grid per target; the touched groups get slots;
//   2. barrier; every wave takes rows of the grid (four per slot, one DPP row
//      each), owners of touched groups preload the group's old leaves, and all
//      loads (rho, h for the atom and for its conjugate partner, the phase
//      exp(2 pi i k Delta / M_v) of Eqs. GramKern/hkj) are issued before the
//      coefficient adjustment (Eq. dualatprod) is computed;
//   3. rho -= c h1 phi + conj(c) h2 conj(phi); each row's maximum (DPP) becomes
//      the new leaf, also written to an LDS scratch for the group owner;
//   4. barrier; owners merge old and new leaves into the group maximum;
//      barrier.
// E_k is tracked in FP64 (Eq. projenfaster) by every wave identically, so the
// stop decision needs no communication.

// Constants of the pair (target w, source v) for the current signal (LDS).
struct __align__(16) PairC {
  int32_t MR, N, off, lbase;
  int32_t lpf, Mmax, rw, rv;
  int32_t dbox, mulo, muhi, width;
  int32_t sw, sv, Lpa, amin;
  int32_t M, sw_sh, rw_sh, pad;
  int64_t tab;
  int32_t pad2[2];
};

// Constants of system w for the current signal (LDS).
struct __align__(16) DictC {
  int32_t off, MR, M, mr_sh;
  uint32_t mr_mul;
  int32_t lbase, lpf, pad;
  int64_t gamma_off, root_off;
};

// Geometry of one target system for the current selection (LDS, written by wave 0).
struct __align__(16) Tgt {
  int32_t MR, N, off, lbase;
  int32_t lpf, Mmax, rw, kr;
  int32_t mulo, muhi, width, sw;
  int32_t nlo, nF, dlo, ilo;
  int32_t bpf, item_base, cph, dbox;
  int32_t gA_lo, gA_n, gB_lo, slot_base;
  int64_t tab;
  int32_t pad[2];
};

// Per-selection values shared by all waves (written by wave 0).
template <typename R>
struct __align__(16) IterS {
  Cx<R> rp;       // rho(p)
  int64_t gamma_off, root_off;
  int32_t v, kk, j, pair;
  int32_t T_items, TG, stop, M;
};

template <typename R>
struct MPShape;
template <>
struct MPShape<float> {
  static constexpr int MAXTG = 16;  // groups merged through the LDS scratch
};
template <>
struct MPShape<double> {
  static constexpr int MAXTG = 8;
};

constexpr int SLOTMAX = 256;  // touched-group slots listed per selection

template <typename R, int NT, int SLOTS>
__host__ __device__ constexpr size_t mp_lds_bytes(int n_groups_max, bool preload) {
  return (size_t)n_groups_max * (sizeof(typename KeyOps<R>::Key) + sizeof(Cx<R>)) +
         (preload ? (size_t)MPShape<R>::MAXTG * GLEAVES * sizeof(Leaf<R>) : 0) + (size_t)MAXW * sizeof(Tgt) +
         (size_t)MAXW * MAXW * sizeof(PairC) + (size_t)MAXW * sizeof(DictC) + (size_t)SLOTMAX * sizeof(int) +
         sizeof(IterS<R>) + 64;
}

__device__ __forceinline__ int fdiv_p(int x, int d, int sh) { return sh >= 0 ? (x >> sh) : floor_div32(x, d); }
__device__ __forceinline__ int cdiv_p(int x, int d, int sh) { return sh >= 0 ? -((-x) >> sh) : ceil_div32(x, d); }

// Group of touched-group slot gs, from the targets' runs in the shared table.
__device__ __forceinline__ int slot_to_group(const Tgt* tg, int W, int gs) {
  int g = -1;
  for (int u = 0; u < W; ++u) {
    const int sbu = tg[u].slot_base, an = tg[u].gA_n;
    const int end = u + 1 < W ? tg[u + 1].slot_base : (1 << 30);
    if (gs >= sbu && gs < sbu + an) g = tg[u].gA_lo + gs - sbu;
    else if (gs >= sbu + an && gs < end) g = tg[u].gB_lo + gs - sbu - an;
  }
  return g;
}

template <typename R, int NT, int SLOTS>
__device__ void mp_signal(const MPArgs& A, int s, unsigned char* smem, int lane, int wave) {
  if (A.reset_it > 0 && A.state[s].done) return;  // finished in an earlier round of the reset procedure
  using KO = KeyOps<R>;
  using KD = KeyDpp<R>;
  using Key = typename KO::Key;
  constexpr int NW = NT / 64;
  constexpr int MAXTG = MPShape<R>::MAXTG;
  constexpr int RPR = NW * 4 * SLOTS;  // rows per round
  const SigDev& S = A.sigs[s];
  const int W = A.W;
  const int G = A.G, logG = A.logG;
  const bool preload = (G == GLEAVES);
  const int n_leaves = S.n_leaves, n_groups = S.n_groups;
  Cx<R>* rho = reinterpret_cast<Cx<R>*>(A.planes) + S.coef_base;
  Leaf<R>* leaves = reinterpret_cast<Leaf<R>*>(A.leaves) + S.leaf_base;
  const Cx<R>* tabs = reinterpret_cast<const Cx<R>*>(A.tabs);
  const Cx<R>* gams = reinterpret_cast<const Cx<R>*>(A.gammas);
  const Cx<R>* roots = reinterpret_cast<const Cx<R>*>(A.roots);
  const int Lp = (int)S.Lp;
  const int rid = lane >> LOG_ROW, rl = lane & (ROW - 1);

  // LDS carve-up (must match mp_lds_bytes)
  Key* gkey = reinterpret_cast<Key*>(smem);
  Cx<R>* gval = reinterpret_cast<Cx<R>*>(gkey + A.n_groups_max);
  Leaf<R>* lscr = reinterpret_cast<Leaf<R>*>(gval + A.n_groups_max);
  Tgt* tg = reinterpret_cast<Tgt*>(
      reinterpret_cast<unsigned char*>(lscr) + (preload ? (size_t)MAXTG * GLEAVES * sizeof(Leaf<R>) : 0));
  PairC* pc = reinterpret_cast<PairC*>(tg + MAXW);
  DictC* dc = reinterpret_cast<DictC*>(pc + MAXW * MAXW);
  int* slotg = reinterpret_cast<int*>(dc + MAXW);
  IterS<R>* is = reinterpret_cast<IterS<R>*>(slotg + SLOTMAX);

  // ---- per-signal constants, group maxima, scratch reset ----
  for (int t = threadIdx.x; t < W * W; t += NT) {
    const int w = t / W;
    const PairDev P = A.pairs[t];
    const DictDev Dw = A.dicts[w];
    PairC c;
    c.MR = Dw.MR; c.N = S.N[w]; c.off = (int)S.off[w]; c.lbase = (int)S.lbase[w];
    c.lpf = Dw.lpf; c.Mmax = P.Mmax; c.rw = P.rw; c.rv = P.rv;
    c.dbox = P.dbox; c.mulo = P.mu_lo; c.muhi = P.mu_hi; c.width = P.width;
    c.sw = P.sw; c.sv = P.sv; c.Lpa = Lp / P.amin; c.amin = P.amin;
    c.M = Dw.M;
    c.sw_sh = (P.sw & (P.sw - 1)) ? -1 : (31 - __clz(P.sw));
    c.rw_sh = (P.rw & (P.rw - 1)) ? -1 : (31 - __clz(P.rw));
    c.pad = 0;
    c.tab = P.tab_off;
    c.pad2[0] = c.pad2[1] = 0;
    pc[t] = c;
  }
  if (threadIdx.x < W) {
    const int w = threadIdx.x;
    const DictDev Dw = A.dicts[w];
    DictC d;
    d.off = (int)S.off[w]; d.MR = Dw.MR; d.M = Dw.M; d.mr_sh = Dw.mr_sh; d.mr_mul = Dw.mr_mul;
    d.lbase = (int)S.lbase[w]; d.lpf = Dw.lpf; d.pad = 0;
    d.gamma_off = Dw.gamma_off; d.root_off = Dw.root_off;
    dc[w] = d;
  }
  for (int g = wave; g < n_groups; g += NW) {
    Key best = KO::empty();
    Cx<R> bv = {(R)0, (R)0};
    for (int i = lane; i < G; i += 64) {
      const int b = (g << logG) + i;
      if (b < n_leaves) {
        const Leaf<R> c = leaves[b];
        if (KO::gt(leaf_key(c), best)) {
          best = leaf_key(c);
          bv = Cx<R>{c.re, c.im};
        }
      }
    }
    const Key wm = wave_max_key2<R>(best);
    const uint64_t own = __ballot(key_eq(best, wm));
    if (lane == __ffsll((unsigned long long)own) - 1) {
      gkey[g] = wm;
      gval[g] = bv;
    }
  }
  if (preload)
    for (int i = threadIdx.x; i < MAXTG * GLEAVES; i += NT) lscr[i] = make_leaf(KD::sentinel(), (R)0, (R)0);
  __syncthreads();

  SigState st = A.state[s];
  double E = st.E;
  int64_t k = st.k;
  const double E0 = st.E0;
  int64_t K = A.K > 0 ? A.K : S.Lp / 5;
  if (K > S.cap) K = S.cap;
  double Etarget = A.snr_db > 0.0 ? E0 * exp10(-A.snr_db / 10.0) : -__builtin_huge_val();
  if (A.reset_it > 0) {
    // inner loop of the reset procedure (Alg. 2)
    K = min(K, st.kout + A.reset_it);
    if (A.reset_db < 0.0) Etarget = fmax(Etarget, st.Eout * exp10(A.reset_db / 10.0));
  }
  int stop = 0;
  int64_t c_upd = 0, c_blk = 0, c_grp = 0;

  for (;;) {
    if (k >= K) { stop = 1; break; }
    if (E <= Etarget) { stop = 2; break; }
    if (E < 0.0) { stop = 3; break; }

    // ---- wave 0: root, decode, target grids, touched-group slots ----
    if (wave == 0) {
      Key best = KO::empty();
      for (int i0 = 0; i0 < n_groups; i0 += 256) {
        Key c[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int i = i0 + lane + 64 * u;
          c[u] = i < n_groups ? gkey[i] : KO::empty();
        }
#pragma unroll
        for (int u = 0; u < 4; ++u)
          if (KO::gt(c[u], best)) best = c[u];
      }
      const Key bk = wave_max_key2<R>(best);
      if (!(KO::value(bk) > (R)0)) {
        if (lane == 0) is->stop = 1;
      } else {
        const int p = uni_i((int)KO::index(bk));
        int v = 0;
        for (int u = 1; u < W; ++u)
          if (p >= dc[u].off) v = u;
        v = uni_i(v);
        const DictC Dv = dc[v];
        const int q0 = p - Dv.off;
        const int j = magic_div(q0, Dv.mr_mul, Dv.mr_sh);
        const int kk = q0 - j * Dv.MR;
        const bool pair = kk != 0 && 2 * kk != Dv.M;
        const int vmask = Dv.M - 1;
        int t_items = 0, t_groups = 0;
        Tgt T;
        if (lane < W) {
          const PairC P = pc[lane * W + v];
          T.MR = P.MR; T.N = P.N; T.off = P.off; T.lbase = P.lbase;
          T.lpf = P.lpf; T.Mmax = P.Mmax; T.rw = P.rw; T.kr = kk * P.rv;
          T.mulo = P.mulo; T.muhi = P.muhi; T.width = P.width; T.sw = P.sw;
          T.dbox = P.dbox; T.tab = P.tab; T.pad[0] = (int32_t)dc[lane].gamma_off;
          T.pad[1] = (P.Mmax & (P.Mmax - 1)) == 0;  // M_max a power of two: indices mod M_max by masks
          T.cph = (vmask & Dv.M) == 0 ? (kk * P.amin) & vmask : (int)(((int64_t)kk * P.amin) % Dv.M);
          T.nlo = 0; T.nF = 0; T.dlo = 0; T.ilo = 0; T.bpf = 1;
          T.gA_lo = T.gA_n = T.gB_lo = 0;
          if (P.dbox >= 0) {
            const int jsv = j * P.sv;
            const int nlo = cdiv_p(jsv - P.dbox, P.sw, P.sw_sh), nhi = fdiv_p(jsv + P.dbox, P.sw, P.sw_sh);
            const int half = P.M >> 1;
            int mlo = 1 << 30, mhi = -1;
            for (int term = 0; term < (pair ? 2 : 1); ++term) {
              const int base = term == 0 ? T.kr : -T.kr;  // m r_w in base + [mu_lo, mu_hi]
              const int A1 = cdiv_p(base + P.mulo, P.rw, P.rw_sh), B1 = fdiv_p(base + P.muhi, P.rw, P.rw_sh);
              if (B1 - A1 + 1 >= P.M) {
                mlo = 0;
                mhi = half;
              } else {
                for (int c = -1; c <= 1; ++c) {
                  const int lo = max(A1 + c * P.M, 0), hi = min(B1 + c * P.M, half);
                  if (lo <= hi) {
                    mlo = min(mlo, lo);
                    mhi = max(mhi, hi);
                  }
                }
              }
            }
            if (mhi >= 0 && nhi >= nlo) {
              int nl = nlo % P.N;
              if (nl < 0) nl += P.N;
              T.nlo = nl;
              T.nF = nhi - nlo + 1;
              T.dlo = nlo * P.sw - jsv;  // delta of the first frame, in [-dbox, dbox]
              T.ilo = mlo >> LOG_ROW;
              T.bpf = (mhi >> LOG_ROW) - T.ilo + 1;
              t_items = ((T.nF * T.bpf) + 3) & ~3;
              // touched groups: run A = frames nlo.., run B = wrapped frames 0..
              const int ihi = mhi >> LOG_ROW;
              const int nAe = min(T.nlo + T.nF - 1, T.N - 1);
              T.gA_lo = (T.lbase + T.nlo * T.lpf + T.ilo) >> logG;
              T.gA_n = ((T.lbase + nAe * T.lpf + ihi) >> logG) - T.gA_lo + 1;
              t_groups = T.gA_n;
              if (T.nlo + T.nF - 1 >= T.N) {
                const int nBe = T.nlo + T.nF - 1 - T.N;
                T.gB_lo = (T.lbase + T.ilo) >> logG;
                const int gBhi = min((T.lbase + nBe * T.lpf + ihi) >> logG, T.gA_lo - 1);
                t_groups += max(0, gBhi - T.gB_lo + 1);
              }
            }
          }
        }
        int ib = 0, sb = 0;
        for (int u = 0; u < W; ++u) {
          const int iu = (int)rdlane32((uint32_t)t_items, u), gu = (int)rdlane32((uint32_t)t_groups, u);
          if (u < lane) {
            ib += iu;
            sb += gu;
          }
        }
        if (lane < W) {
          T.item_base = ib;
          T.slot_base = sb;
          tg[lane] = T;
        }
        const int T_items = (int)rdlane32((uint32_t)(ib + t_items), W - 1);
        const int TG = (int)rdlane32((uint32_t)(sb + t_groups), W - 1);
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        for (int gs = lane; gs < min(TG, SLOTMAX); gs += 64) slotg[gs] = slot_to_group(tg, W, gs);
        if (lane == 0) {
          IterS<R> I;
          I.rp = gval[(Dv.lbase + j * Dv.lpf + (kk >> LOG_ROW)) >> logG];
          I.gamma_off = Dv.gamma_off;
          I.root_off = Dv.root_off;
          I.v = v;
          I.kk = kk;
          I.j = j;
          I.pair = pair;
          I.T_items = T_items;
          I.TG = TG;
          I.stop = 0;
          I.M = Dv.M;
          *is = I;
        }
      }
    }
    __syncthreads();
    const IterS<R> I = *is;
    if (I.stop) { stop = 4; break; }
    const int v = uni_i(I.v), kk = uni_i(I.kk), j = uni_i(I.j), T_items = uni_i(I.T_items), TG = uni_i(I.TG);
    const bool pair = uni_i(I.pair) != 0;
    Cx<R> gam = {(R)0, (R)0};
    if (pair) gam = gams[I.gamma_off + kk];  // consumed after the row loads are issued
    const Cx<R>* vroots = roots + I.root_off;
    const int vmask = uni_i(I.M) - 1;

    const int my_gs = wave;
    const bool own_pre = preload && my_gs < TG && my_gs < MAXTG;
    const int my_g = my_gs < TG ? uni_i(my_gs < SLOTMAX ? slotg[my_gs] : slot_to_group(tg, W, my_gs)) : -1;
    Leaf<R> old[4];
    if (own_pre) {
#pragma unroll
      for (int i = 0; i < 4; ++i) old[i] = leaves[(my_g << logG) + lane + 64 * i];
    }

    // ---- rows of the target grids: loads, adjustment, update, rescan ----
    Cx<R> cc = {(R)0, (R)0};
    bool partner = false;
    for (int round = 0;; ++round) {
      Cx<R> r[SLOTS], h1[SLOTS], h2[SLOTS], ph[SLOTS], gg[SLOTS];
      int ee[SLOTS], lfi[SLOTS], gsl[SLOTS];
      bool act[SLOTS], rowok[SLOTS], vld[SLOTS], chg[SLOTS], pp[SLOTS];
      int cw = -1;
      Tgt T;
#pragma unroll
      for (int sl = 0; sl < SLOTS; ++sl) {
        r[sl] = h1[sl] = h2[sl] = gg[sl] = Cx<R>{(R)0, (R)0};
        ph[sl] = Cx<R>{(R)1, (R)0};
        ee[sl] = lfi[sl] = gsl[sl] = 0;
        act[sl] = rowok[sl] = vld[sl] = chg[sl] = pp[sl] = false;
        const int base4 = ((round * SLOTS + sl) * NW + wave) * 4;
        if (base4 >= T_items) continue;  // wave-uniform
        act[sl] = true;
        int w = 0;
        for (int u = 1; u < W; ++u)
          if (base4 >= tg[u].item_base) w = u;
        w = uni_i(w);
        if (w != cw) {
          T = tg[w];
          cw = w;
        }
        // row t of target w's grid: frame f, 16-bin block i
        const int t = base4 - T.item_base + rid;
        const int bpf = T.bpf;
        int f = (int)((float)t * __frcp_rn((float)bpf));
        if (f * bpf > t) --f;
        if ((f + 1) * bpf <= t) ++f;
        const int i = T.ilo + t - f * bpf;
        const bool ok = f < T.nF;
        rowok[sl] = ok;
        int n = T.nlo + f;
        if (n >= T.N) n -= T.N;
        const int li = T.lbase + n * T.lpf + i;
        lfi[sl] = li;
        {
          const int g = li >> logG;
          gsl[sl] = (g >= T.gA_lo && g < T.gA_lo + T.gA_n) ? T.slot_base + g - T.gA_lo
                                                           : T.slot_base + T.gA_n + g - T.gB_lo;
        }
        const int m = (i << LOG_ROW) + rl;
        const int e = T.off + n * T.MR + m;
        ee[sl] = e;
        if (!ok || m >= T.MR) continue;
        vld[sl] = true;
        r[sl] = rho[e];
        pp[sl] = A.pedantic && m != 0 && m != T.MR - 1;
        if (pp[sl]) gg[sl] = gams[T.pad[0] + m];
        const int d = T.dlo + f * T.sw;  // delta = Delta / a_min, in [-dbox, dbox]
        const int mm = T.Mmax - 1;
        // mu = m r_w -/+ k r_v taken mod M_max into (-M_max/2, M_max/2]; the
        // unreduced values lie in [-M_max/2, M_max + r_w]
        auto wrapmu = [&](int x) {
          if (T.pad[1]) {
            x &= mm;
          } else {
            x += x < 0 ? T.Mmax : 0;
            x -= x >= T.Mmax ? T.Mmax : 0;
          }
          return x > (T.Mmax >> 1) ? x - T.Mmax : x;
        };
        const int mu1 = wrapmu(m * T.rw - T.kr);
        const int64_t rowoff = T.tab + (int64_t)(d + T.dbox) * T.width - T.mulo;
        bool any = false;
        if (mu1 >= T.mulo && mu1 <= T.muhi) {
          h1[sl] = tabs[rowoff + mu1];
          any = true;
        }
        if (pair) {
          const int mu2 = wrapmu(m * T.rw + T.kr);
          if (mu2 >= T.mulo && mu2 <= T.muhi) {
            h2[sl] = tabs[rowoff + mu2];
            any = true;
          }
        }
        if (any) {
          // phase index (k Delta) mod M_v = ((delta mod M_v) cph) mod M_v
          const int Mv = vmask + 1;
          const int pi = (Mv & vmask) == 0 ? ((d & vmask) * T.cph) & vmask
                                           : (int)(((int64_t)mod_pos(d, Mv) * T.cph) % Mv);
          ph[sl] = vroots[pi];
        }
        chg[sl] = any;
      }
      if (round == 0) {
        // coefficient adjustment for the pair, Eq. (dualatprod), and energy
        // decrease, Eq. (projenfaster); after the loads so that gamma's load
        // overlaps with them
        const R rr = I.rp.re, ri = I.rp.im;
        double Et;
        if (pair) {
          const R gr = gam.re, gi = gam.im;
          const R nr = rr - (gr * rr - gi * ri);
          const R ni = ri - (-gr * ri - gi * rr);
          const R den = (R)1 - (gr * gr + gi * gi);
          cc.re = nr / den;
          cc.im = ni / den;
          const double cr = cc.re, ci = cc.im, dgr = gr, dgi = gi;
          Et = 2.0 * (cr * cr + ci * ci + dgr * (cr * cr - ci * ci) - 2.0 * dgi * cr * ci);
          partner = A.partner_gate ? (gr != (R)0 || gi != (R)0) : true;
        } else {
          cc.re = rr;
          cc.im = ri;
          const double cr = cc.re, ci = cc.im;
          Et = cr * cr + ci * ci;
        }
        E -= Et;
        if (wave == 0 && lane == 0) {
          AtomRec ar;
          ar.w = v;
          ar.m = kk;
          ar.n = j;
          ar.pad = 0;
          ar.re = (double)cc.re;
          ar.im = (double)cc.im;
          ar.E_after = E;
          A.atoms[S.atom_base + k] = ar;
        }
        ++k;
      }
#pragma unroll
      for (int sl = 0; sl < SLOTS; ++sl) {
        if (!act[sl]) continue;  // wave-uniform
        bool nz = false;
        if (chg[sl]) {
          const Cx<R> b2 = partner ? h2[sl] : Cx<R>{(R)0, (R)0};
          nz = (h1[sl].re != (R)0) | (h1[sl].im != (R)0) | (b2.re != (R)0) | (b2.im != (R)0);
          if (nz) {
            const R cs = ph[sl].re, sn = ph[sl].im;
            // c (h1 phi) + conj(c) (h2 conj(phi))
            const R ar = h1[sl].re * cs - h1[sl].im * sn, ai = h1[sl].re * sn + h1[sl].im * cs;
            R ur = cc.re * ar - cc.im * ai, ui = cc.re * ai + cc.im * ar;
            const R br = b2.re * cs + b2.im * sn, bi = b2.im * cs - b2.re * sn;
            ur += cc.re * br + cc.im * bi;
            ui += cc.re * bi - cc.im * br;
            r[sl].re -= ur;
            r[sl].im -= ui;
            rho[ee[sl]] = r[sl];
          }
        }
        const R val = sel_score<R>(r[sl].re, r[sl].im, gg[sl], pp[sl]);
        const uint64_t bits = vld[sl] ? val_bits(val) : 0ull;
        const uint64_t rm = row_max_bits<R>(bits);
        const uint64_t bal = __ballot(vld[sl] && bits == rm);
        const uint32_t rowbits = (uint32_t)(bal >> (rid * ROW)) & 0xFFFFu;
        const bool leader = rowok[sl] && rowbits && lane == rid * ROW + __ffs(rowbits) - 1;
        c_upd += __popcll(__ballot(nz));
        c_blk += __popcll(__ballot(leader));
        if (leader) {
          const Leaf<R> nl = make_leaf(KO::make(val, (uint32_t)ee[sl]), r[sl].re, r[sl].im);
          const int b = lfi[sl];
          leaves[b] = nl;
          if (preload && gsl[sl] < MAXTG) lscr[gsl[sl] * GLEAVES + (b & (GLEAVES - 1))] = nl;
        }
      }
      if ((round + 1) * RPR >= T_items) break;
    }
    __syncthreads();

    // ---- group maxima of the touched groups ----
    for (int gs = wave; gs < TG; gs += NW) {
      const int g = gs == my_gs ? my_g : uni_i(gs < SLOTMAX ? slotg[gs] : slot_to_group(tg, W, gs));
      Key bkey = KO::empty();
      Cx<R> bval = {(R)0, (R)0};
      if (preload && gs < MAXTG) {
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          Leaf<R>& sc = lscr[gs * GLEAVES + lane + 64 * i];
          Leaf<R> c = (gs == my_gs && own_pre) ? old[i] : leaves[(g << logG) + lane + 64 * i];
          const Leaf<R> scv = sc;
          if (!KD::is_sentinel(leaf_key(scv))) {
            c = scv;
            sc = make_leaf(KD::sentinel(), (R)0, (R)0);
          }
          if (KO::gt(leaf_key(c), bkey)) {
            bkey = leaf_key(c);
            bval = Cx<R>{c.re, c.im};
          }
        }
      } else {
        for (int i = lane; i < G; i += 64) {
          const int b = (g << logG) + i;
          if (b < n_leaves) {
            const Leaf<R> c = leaves[b];
            if (KO::gt(leaf_key(c), bkey)) {
              bkey = leaf_key(c);
              bval = Cx<R>{c.re, c.im};
            }
          }
        }
      }
      const Key wm = wave_max_key2<R>(bkey);
      const uint64_t own = __ballot(key_eq(bkey, wm));
      if (lane == __ffsll((unsigned long long)own) - 1) {
        gkey[g] = wm;
        gval[g] = bval;
      }
      ++c_grp;
    }
    __syncthreads();
  }

  if (lane == 0) {
    atomicAdd((unsigned long long*)&A.state[s].updated, (unsigned long long)c_upd);
    atomicAdd((unsigned long long*)&A.state[s].blocks, (unsigned long long)c_blk);
    atomicAdd((unsigned long long*)&A.state[s].groups, (unsigned long long)c_grp);
  }
  if (wave == 0 && lane == 0) {
    A.state[s].E = E;
    A.state[s].k = k;
    A.state[s].stop = stop;
  }
}

template <typename R, int NT, int SLOTS>
__global__ void __launch_bounds__(NT) k_mp(MPArgs A) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  __shared__ int s_next;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (;;) {
    if (threadIdx.x == 0) s_next = atomicAdd(A.queue, 1);
    __syncthreads();
    const int qi = s_next;
    __syncthreads();
    if (qi >= A.batch) break;
    mp_signal<R, NT, SLOTS>(A, A.order[qi], smem_raw, lane, wave);
  }
}

// --------------------------------------------------------------------------
// FP32 MP loop.  Same selection / adjustment / update as above; the tree is
// kept differently:
//   leaves (16 bins of one frame, 8-byte keys, global memory)
//     -> groups of GL leaves (keys in LDS) -> root (reduced per selection).
// Every group touched by the update is re-reduced after it: its old leaves
// are preloaded into registers while the rows are processed, the rewritten
// ones go through an LDS scratch, and the owner wave merges the two.
//
// Selection is pipelined.  The keys of the groups an update does not touch
// cannot change in it, so while the other waves update the rows of atom k,
// wave 0 takes the maximum over those groups as the candidate atom k+1 and
// lays out its target grids and adjusted coefficient in a second buffer.
// After the merge one key comparison decides: the candidate is atom k+1
// unless a touched group now holds a larger key, in which case wave 0 decodes
// that key (the maximum over the touched groups, gathered by the merge) before
// the next update.  The selections are the same as with a serial root scan.
//
// Per selection: all waves (rows; wave 0 first builds the candidate) |
// barrier | owners merge touched groups | barrier | [refuted candidate:
// wave 0 selects | barrier].

constexpr uint64_t KEY_SENT = ~0ull;     // scratch entry not written

// Row geometry of one target system for the current selection (LDS).  Term t
// (1: the atom, 2: its conjugate partner) reaches bin m of the target iff
// d_t = (m - c_t) mod M_w <= span_t; its FP32 kernel entry is then entry d_t
// of the term's part of the table row (see select_into).
struct __align__(16) RowT {
  int32_t MR, N, off, lbase;
  int32_t lpf, nlo, nF, ilo;
  int32_t bpf, item_base, Mw, span1;
  int32_t c1, c2, span2, hrow0;
  int32_t hstep, slot_base;          // table row of frame f: hrow0 + f hstep; first touched-group slot
  uint32_t ph0, phs;                 // phase index of frame f: (ph0 + f phs) mod M_v
  int32_t gA_lo, gA_n, gB_lo, gB_n;  // touched groups (run A: frames from nlo, run B: wrapped)
  float rbpf;                        // 1 / bpf
  int32_t pad[3];
};

// Per-selection values shared by all waves (written by wave 0).
struct __align__(16) It32 {
  int32_t p, v, kk, j;
  int32_t pair, T_items, TG, stop;
  int32_t root_off, vmask, partner, pad;
  int32_t Mv, mv_sh;                 // M_v, and q / M_v == (umulhi(q, mv_mul) + q) >> mv_sh
  uint32_t mv_mul;
  int32_t pad2;
  Cx<float> cc;                      // adjusted coefficient c~ of the selected atom (pair)
  double Et;                         // energy decrease of the selection
  int32_t ibase[MAXW];               // first row item of each target
  int32_t sbase[MAXW];               // first touched-group slot of each target
  int32_t glist[64];                 // group of touched-group slot gs < 64
};

__host__ __device__ constexpr int mp32_groups_padded(int n_groups) { return (n_groups + 511) & ~511; }

template <int NT, int GL>
__host__ __device__ constexpr size_t mp32_lds_bytes(int n_groups_max) {
  return (size_t)mp32_groups_padded(n_groups_max) * 8 + (size_t)(2 * (NT / 64)) * GL * 8 +
         (size_t)(2 * MAXW) * sizeof(RowT) + (size_t)MAXW * MAXW * sizeof(PairC) + 2 * sizeof(It32) + 4 * 8 + 64;
}

__device__ __forceinline__ uint64_t umax64(uint64_t a, uint64_t b) { return a > b ? a : b; }

// Two adjacent complex FP32 values (16 bytes, 8-byte aligned).
struct __align__(8) C4f {
  float x, y, z, w;
};
__device__ __forceinline__ C4f ld_c4(const Cx<float>* q) {
  C4f v;
  __builtin_memcpy(&v, q, sizeof(C4f));
  return v;
}
__device__ __forceinline__ void st_c4(Cx<float>* q, const C4f& v) { __builtin_memcpy(q, &v, sizeof(C4f)); }

// P2: every M of the plan is a power of two (indices mod M by masks).
// XP: touched groups beyond the preloaded ones are loaded before the preloaded
// merges (plans whose selections can touch more groups than are preloaded).
template <int NT, int SLOTS, int GL, bool P2, bool XP>
__device__ void mp_signal32(const MPArgs& A, int s, unsigned char* smem, int lane, int wave) {
  if (A.reset_it > 0 && A.state[s].done) return;  // finished in an earlier round of the reset procedure
  constexpr int NW = NT / 64;
  constexpr int LPL = GL / 64;                 // leaves of a group per lane
  constexpr int LOG_GL = GL == 128 ? 7 : 8;
  constexpr int NPRE = 2 * NW;                 // touched groups merged from registers + LDS scratch
  static_assert(GL == 128 || GL == 256, "group size");
  const SigDev& S = A.sigs[s];
  const int W = A.W;
  const int n_groups = S.n_groups;
  const int ngp = mp32_groups_padded(n_groups);
  const int ngp_max = mp32_groups_padded(A.n_groups_max);
  Cx<float>* rho = reinterpret_cast<Cx<float>*>(A.planes) + S.coef_base;
  uint64_t* leaves = reinterpret_cast<uint64_t*>(A.leaves) + S.leaf_base;
  const Cx<float>* tabs = reinterpret_cast<const Cx<float>*>(A.tabs);
  const Cx<float>* gams = reinterpret_cast<const Cx<float>*>(A.gammas);
  const Cx<float>* roots = reinterpret_cast<const Cx<float>*>(A.roots);
  AtomRec* const atoms = A.atoms + S.atom_base;  // read once: the loop stores to global memory
  const int rid8 = lane >> 3, rl8 = lane & 7;
  const bool pedantic = A.pedantic != 0;

  // LDS carve-up (must match mp32_lds_bytes)
  uint64_t* gkey = reinterpret_cast<uint64_t*>(smem);
  uint64_t* lscr = gkey + ngp_max;
  RowT* tg2 = reinterpret_cast<RowT*>(lscr + NPRE * GL);     // two buffers of MAXW
  PairC* pc = reinterpret_cast<PairC*>(tg2 + 2 * MAXW);
  It32* it2 = reinterpret_cast<It32*>(pc + MAXW * MAXW);        // two buffers
  uint64_t* ckey = reinterpret_cast<uint64_t*>(it2 + 2);        // [b]: candidate key of buffer b
  uint64_t* tmax = ckey + 2;                                     // [b]: maximum over the touched groups
  int* rowq = reinterpret_cast<int*>(tmax + 2);                  // row-batch counter

  // ---- per-signal constants, group maxima, scratch reset ----
  for (int t = threadIdx.x; t < W * W; t += NT) {
    const int w = t / W;
    const PairDev P = A.pairs[t];
    const DictDev Dw = A.dicts[w];
    PairC c;
    c.MR = Dw.MR; c.N = S.N[w]; c.off = (int)S.off[w]; c.lbase = (int)S.lbase[w];
    c.lpf = Dw.lpf; c.Mmax = P.Mmax; c.rw = P.rw; c.rv = P.rv;
    c.dbox = P.dbox; c.mulo = P.mu_lo; c.muhi = P.mu_hi; c.width = P.width;
    c.sw = P.sw; c.sv = P.sv; c.Lpa = 0; c.amin = P.amin;
    c.M = Dw.M;
    c.sw_sh = (P.sw & (P.sw - 1)) ? -1 : (31 - __clz(P.sw));  // -1: a_w / gcd not a power of two
    c.rw_sh = (P.rw & (P.rw - 1)) ? -1 : (31 - __clz(P.rw));  // -1: M_max / M_w not a power of two
    c.pad = P.cw;          // FP32 table: phase-major rows
    c.width = P.width32;
    c.tab = P.tab_off32;
    c.pad2[0] = c.pad2[1] = 0;
    pc[t] = c;
  }
  // every pair's a_w / gcd a power of two (nested hops): frame ranges by shifts
  const bool pow2hops =
      __ballot(lane < W * W && (A.pairs[lane < W * W ? lane : 0].sw & (A.pairs[lane < W * W ? lane : 0].sw - 1)) != 0) == 0ull;
  // dictionary constants, lane u < W holds system u
  int d_off = 0x7fffffff, d_MR = 1, d_M = 2, d_sh = 0, d_gam = 0, d_root = 0, d_msh = 0;
  uint32_t d_mul = 0, d_mmul = 0;
  if (lane < W) {
    const DictDev D = A.dicts[lane];
    d_off = (int)S.off[lane];
    d_MR = D.MR;
    d_M = D.M;
    d_sh = D.mr_sh;
    d_mul = D.mr_mul;
    d_gam = (int)D.gamma_off;
    d_root = (int)D.root_off;
    d_mmul = D.m_mul;
    d_msh = D.m_sh;
  }
  for (int g = wave; g < ngp; g += NW) {
    uint64_t best = 0ull;
    if (g < n_groups) {
#pragma unroll
      for (int x = 0; x < LPL; ++x) best = umax64(best, leaves[g * GL + lane + 64 * x]);
    }
    const uint64_t wm = wave_max_key2<float>(best);
    if (lane == 0) gkey[g] = wm;
  }
  for (int i = threadIdx.x; i < NPRE * GL; i += NT) lscr[i] = KEY_SENT;
  if (threadIdx.x < 4) ckey[threadIdx.x] = 0ull;  // ckey[0..1], tmax[0..1]
  if (threadIdx.x == 0) *rowq = 0;
  static_assert(2 * NW <= 64, "owner slots are listed in It32::glist");
  __syncthreads();

  SigState st = A.state[s];
  double E = uni_d(st.E);  // the loop state is uniform: its stop tests branch on scalars
  int64_t k = uni_l(st.k);
  const double E0 = uni_d(st.E0);
  int64_t K = A.K > 0 ? A.K : S.Lp / 5;
  if (K > S.cap) K = S.cap;
  double Etarget = A.snr_db > 0.0 ? E0 * exp10(-A.snr_db / 10.0) : -__builtin_huge_val();
  if (A.reset_it > 0) {
    // inner loop of the reset procedure (Alg. 2)
    K = min(K, st.kout + A.reset_it);
    if (A.reset_db < 0.0) Etarget = fmax(Etarget, st.Eout * exp10(A.reset_db / 10.0));
  }
  int stop = 0;
  int64_t c_upd = 0, c_blk = 0, c_grp = 0;

  // Wave 0: maximum group key.
  auto scan_root = [&]() -> uint64_t {
    uint64_t best = 0ull;
    for (int i0 = 0; i0 < ngp; i0 += 512) {
      const ulonglong2* g2 = reinterpret_cast<const ulonglong2*>(gkey + i0);
      const ulonglong2 a = g2[lane], b = g2[lane + 64], c = g2[lane + 128], d = g2[lane + 192];
      best = umax64(best, umax64(umax64(umax64(a.x, a.y), umax64(b.x, b.y)),
                                 umax64(umax64(c.x, c.y), umax64(d.x, d.y))));
    }
    return wave_max_key2<float>(best);
  };

  // Wave 0: decode key bk (the selected atom), lay out its target grids and
  // compute its adjusted coefficient into buffer b.  Reads rho(p): the caller
  // guarantees that no row being updated covers p.
  auto select_into = [&](uint64_t bk, int b) {
    It32* itb = it2 + b;
    RowT* tgb = tg2 + b * MAXW;
    if ((uint32_t)(bk >> 32) == 0u) {  // max score is zero
      if (lane == 0) itb->stop = 1;
      return;
    }
    const int p = uni_i((int)~(uint32_t)bk);
    const int v = uni_i(__popcll(__ballot(lane < W && p >= d_off)) - 1);
    const int off_v = (int)rdlane32((uint32_t)d_off, v), MR_v = (int)rdlane32((uint32_t)d_MR, v);
    const int M_v = (int)rdlane32((uint32_t)d_M, v), sh_v = (int)rdlane32((uint32_t)d_sh, v);
    const uint32_t mul_v = rdlane32(d_mul, v);
    const int q0 = p - off_v;
    const int j = magic_div(q0, mul_v, sh_v);
    const int kk = q0 - j * MR_v;
    const bool pair = kk != 0 && 2 * kk != M_v;
    const int vmask = M_v - 1;
    const Cx<float> rp = rho[p];
    const Cx<float> gam = gams[(int)rdlane32((uint32_t)d_gam, v) + (pair ? kk : 0)];

    // geometry of target u = lane (all lanes compute; lanes >= W are discarded)
    const int u = lane < W ? lane : 0;
    const PairC P = pc[u * W + v];
    RowT T;
    T.MR = P.MR; T.N = P.N; T.off = P.off; T.lbase = P.lbase; T.lpf = P.lpf;
    const int kr = (int)__umul24((uint32_t)kk, (uint32_t)P.rv);
    // Term t's entries (t = 1: the atom, 2: its partner) for bin m of target
    // u sit at mu' = (m r_w - k_t) mod M_max of the box row (mu' = mu - mu_lo;
    // k_1 = k r_v + mu_lo, k_2 = mu_lo - k r_v).  With ph_t = (-k_t) mod r_w
    // and c_t = ((k_t + ph_t) / r_w) mod M_w, mu' = r_w ((m - c_t) mod M_w) +
    // ph_t (M_max = r_w M_w): the term reaches bin m iff d_t = (m - c_t) mod
    // M_w <= span_t = floor((mu_hi - mu_lo - ph_t) / r_w), and the phase-major
    // FP32 row keeps that entry at d_t of phase ph_t's part.
    const int k1 = kr + P.mulo, k2 = P.mulo - kr, mspan = P.muhi - P.mulo;
    int ph1, ph2, c1, c2;
    if (P2 || P.rw_sh >= 0) {  // every M a power of two: so is r_w = M_max / M_w
      ph1 = (-k1) & (P.rw - 1);
      ph2 = (-k2) & (P.rw - 1);
      c1 = (k1 + ph1) >> P.rw_sh;  // exact multiples of r_w
      c2 = (k2 + ph2) >> P.rw_sh;
      T.span1 = (mspan - ph1) >> P.rw_sh;
      T.span2 = (mspan - ph2) >> P.rw_sh;
    } else {
      ph1 = mod_pos(-k1, P.rw);
      ph2 = mod_pos(-k2, P.rw);
      c1 = (k1 + ph1) / P.rw;
      c2 = (k2 + ph2) / P.rw;
      T.span1 = floor_div32(mspan - ph1, P.rw);
      T.span2 = floor_div32(mspan - ph2, P.rw);
    }
    T.Mw = P.M;
    T.c1 = P2 ? c1 & (P.M - 1) : mod_pos(c1, P.M);
    T.c2 = P2 ? c2 & (P.M - 1) : mod_pos(c2, P.M);
    T.pad[0] = d_gam;  // gamma(m) of target u's bins (lane u holds system u's offset)
    const int jsv = (int)__umul24((uint32_t)j, (uint32_t)P.sv);
    int nlo, nhi;
    if (pow2hops) {  // uniform
      nlo = -((P.dbox - jsv) >> P.sw_sh);
      nhi = (jsv + P.dbox) >> P.sw_sh;
    } else {
      nlo = ceil_div32(jsv - P.dbox, P.sw);
      nhi = floor_div32(jsv + P.dbox, P.sw);
    }
    const int half = P.M >> 1;
    // bins m in [0, M/2] with m r_w in +-k r_v + [mu_lo, mu_hi] (mod M_max):
    // the bins [A1, B1] of one term, taken mod M, meet [0, M/2] in at most
    // two pieces, [A1 mod M, .] and the wrapped [0, .]
    int mlo = 1 << 30, mhi = -1;
    bool t2 = false;  // term 2 (the conjugate partner) reaches a bin of target u
#pragma unroll
    for (int term = 0; term < 2; ++term) {
      const int base = term == 0 ? kr : -kr;
      const int A1 = P2 ? -((-(base + P.mulo)) >> P.rw_sh) : cdiv_p(base + P.mulo, P.rw, P.rw_sh);
      const int B1 = P2 ? (base + P.muhi) >> P.rw_sh : fdiv_p(base + P.muhi, P.rw, P.rw_sh);
      const bool use = term == 0 || pair;
      const bool full = B1 - A1 + 1 >= P.M;
      const int A1m = P2 ? A1 & (P.M - 1) : mod_pos(A1, P.M), B1m = B1 + (A1m - A1);
      const int lo0 = full ? 0 : A1m, hi0 = full ? half : min(B1m, half);
      const bool ok0 = use && lo0 <= hi0;
      const bool ok1 = use && !full && B1m >= P.M;  // piece [0, B1m - M]
      const int hi1 = min(B1m - P.M, half);
      mlo = ok0 ? min(mlo, lo0) : mlo;
      mhi = ok0 ? max(mhi, hi0) : mhi;
      mlo = ok1 ? 0 : mlo;
      mhi = ok1 ? max(mhi, hi1) : mhi;
      if (term == 1) t2 = ok0 || ok1;
    }
    const bool valid = lane < W && P.dbox >= 0 && mhi >= 0 && nhi >= nlo;
    const bool any2 = __ballot(valid && t2) != 0ull;
    const int nl = nlo < 0 ? nlo + P.N : (nlo >= P.N ? nlo - P.N : nlo);
    T.nlo = nl;
    T.nF = valid ? nhi - nlo + 1 : 0;
    const int dlo = nlo * P.sw - jsv;  // delta of the first frame, in [-dbox, dbox]
    T.ilo = valid ? mlo >> LOG_ROW : 0;
    T.bpf = valid ? (mhi >> LOG_ROW) - T.ilo + 1 : 1;
    T.rbpf = __builtin_amdgcn_rcpf((float)T.bpf);  // within 1 ulp of 1 / bpf
    T.pad[1] = __float_as_int(0.5f * T.rbpf);
    // table rows are phase-major: term t's part starts at ph_t ceil(width / r_w)
    T.hrow0 = (int)P.tab + (int)__umul24((uint32_t)(dlo + P.dbox), (uint32_t)P.width) +
              (int)__umul24((uint32_t)ph1, (uint32_t)P.pad);
    T.pad[2] = __mul24(ph2 - ph1, P.pad);
    T.hstep = (int)__umul24((uint32_t)P.width, (uint32_t)P.sw);
    // phase index of frame f: (k Delta / a_min ... ) = (ph0 + f phs) mod M_v
    if (P2) {
      const uint32_t cph = __umul24((uint32_t)kk, (uint32_t)P.amin) & (uint32_t)vmask;
      T.ph0 = (uint32_t)__mul24(dlo, (int)cph);                         // taken mod M_v
      T.phs = __umul24(cph, (uint32_t)P.sw) & (uint32_t)vmask;        // phases are taken mod M_v
    } else {
      const int64_t cph = ((int64_t)kk * P.amin) % M_v;
      const int64_t q = ((int64_t)dlo * cph) % M_v;
      T.ph0 = (uint32_t)(q < 0 ? q + M_v : q);
      T.phs = (uint32_t)((cph * P.sw) % M_v);
    }
    const int t_items = valid ? ((int)__umul24((uint32_t)T.nF, (uint32_t)T.bpf) + 7) & ~7 : 0;  // whole 8-row slots per target
    const int ihi = mhi >> LOG_ROW;
    const int nend = T.nlo + T.nF - 1;
    const int nAe = min(nend, T.N - 1);
    T.gA_lo = (T.lbase + T.nlo * T.lpf + T.ilo) >> LOG_GL;
    T.gA_n = valid ? ((T.lbase + nAe * T.lpf + ihi) >> LOG_GL) - T.gA_lo + 1 : 0;
    T.gB_lo = (T.lbase + T.ilo) >> LOG_GL;
    const int gBhi = min((T.lbase + (nend - T.N) * T.lpf + ihi) >> LOG_GL, T.gA_lo - 1);
    T.gB_n = (valid && nend >= T.N) ? max(0, gBhi - T.gB_lo + 1) : 0;
    const int t_groups = T.gA_n + T.gB_n;
    int ib = 0, sb = 0;
    for (int w = 0; w + 1 < W; ++w) {
      const int iw = (int)rdlane32((uint32_t)t_items, w), gw = (int)rdlane32((uint32_t)t_groups, w);
      ib += w < lane ? iw : 0;
      sb += w < lane ? gw : 0;
    }
    T.item_base = ib;
    T.slot_base = sb;
    // cross-lane reads with the whole wave active
    const int T_items = (int)rdlane32((uint32_t)(ib + t_items), W - 1);
    const int TG = (int)rdlane32((uint32_t)(sb + t_groups), W - 1);
    const int root_v = (int)rdlane32((uint32_t)d_root, v);
    const int msh_v = (int)rdlane32((uint32_t)d_msh, v);
    const uint32_t mmul_v = rdlane32(d_mmul, v);
    if (lane < W) {
      tgb[lane] = T;
      itb->ibase[lane] = ib;
      itb->sbase[lane] = sb;
    }
    // group of touched-group slot gs = lane: target ws is the last one whose
    // first slot is at or before gs (its geometry read back from LDS)
    {
      int ws = 0;
      for (int w = 1; w < W; ++w) ws += (int)rdlane32((uint32_t)sb, w) <= lane ? 1 : 0;
      // target ws's runs from its lane's registers (cross-lane moves, no LDS read-back)
      const int gal = __shfl(T.gA_lo, ws), gan = __shfl(T.gA_n, ws), gbl = __shfl(T.gB_lo, ws);
      const int c = lane - __shfl(sb, ws);
      const int g = c < gan ? gal + c : gbl + (c - gan);
      itb->glist[lane] = lane < TG ? g : 0;
    }
    // coefficient adjustment for the pair, Eq. (dualatprod), and energy
    // decrease, Eq. (projenfaster)
    Cx<float> cc;
    double Et;
    bool partner = false;
    {
      const float rr = rp.re, ri = rp.im;
      if (pair) {
        const float gr = gam.re, gi = gam.im;
        const float nr = rr - (gr * rr - gi * ri);
        const float ni = ri - (-gr * ri - gi * rr);
        const float den = 1.0f - (gr * gr + gi * gi);
        cc.re = nr / den;
        cc.im = ni / den;
        const double cr = cc.re, ci = cc.im, dgr = gr, dgi = gi;
        Et = 2.0 * (cr * cr + ci * ci + dgr * (cr * cr - ci * ci) - 2.0 * dgi * cr * ci);
        partner = A.partner_gate ? (gr != 0.0f || gi != 0.0f) : true;
      } else {
        cc.re = rr;
        cc.im = ri;
        const double cr = cc.re, ci = cc.im;
        Et = cr * cr + ci * ci;
      }
    }
    if (lane == 0) {
      int4* I = reinterpret_cast<int4*>(&itb->p);
      I[0] = make_int4(p, v, kk, j);
      I[1] = make_int4(pair, T_items, TG, 0);
      I[2] = make_int4(root_v, vmask, partner, (partner && any2) ? 1 : 0);
      I[3] = make_int4(M_v, msh_v, (int)mmul_v, 0);
      itb->cc = cc;
      itb->Et = Et;
    }
  };

  // per-selection values every wave reads from buffer b (one batch of LDS reads)
  struct ItR {
    int4 I0, I1, I2, I3;
    Cx<float> cc;
    double Et;
    int ibase, sbase, g0, g1;
    int gl;  // touched-group list entry `lane` (used by wave 0)
  };
  auto read_it = [&](int b) -> ItR {
    const It32* itb = it2 + b;
    ItR r;
    r.I0 = *reinterpret_cast<const int4*>(&itb->p);
    r.I1 = *reinterpret_cast<const int4*>(&itb->pair);
    r.I2 = *reinterpret_cast<const int4*>(&itb->root_off);
    r.I3 = P2 ? make_int4(0, 0, 0, 0) : *reinterpret_cast<const int4*>(&itb->Mv);
    r.cc = itb->cc;
    r.Et = itb->Et;
    r.ibase = lane < W ? itb->ibase[lane] : 0x7fffffff;
    r.sbase = lane < W ? itb->sbase[lane] : 0x7fffffff;
    r.g0 = itb->glist[wave];
    r.g1 = itb->glist[wave + NW];
    r.gl = wave == 0 ? itb->glist[lane] : 0;
    return r;
  };

  // ---- rows of one batch: loads, update, new leaves ----
  // A slot is 8 rows; 8 lanes per row, each with 2 adjacent bins m0 = 16 i +
  // 2 rl8 and m0 + 1.  fl bit 0: row in grid, 1/2: bin 0/1 valid, 3/4: term 1
  // of bin 0/1 in the box, 5/6: term 2 of bin 0/1, 7: pedantic score.
  // phase index (ph0 + f phs) mod M_v: a mask when M_v is a power of two,
  // else a division by M_v (x < 2^31, bounded at plan creation)
  struct PhaseMod {
    uint32_t mask, mul;
    int Mv, sh;
  };
  auto do_batch = [&](auto has2, uint64_t* o0, uint64_t* o1, const RowT* tg, int qb, int nact, int ibase,
                      int p, bool pair, uint32_t root_off, PhaseMod pm, Cx<float> cc) {
    constexpr bool H2 = decltype(has2)::value;  // some bin of this selection sees term 2
    C4f r[SLOTS], gg[SLOTS];
    Cx<float> h1a[SLOTS], h1b[SLOTS], h2a[SLOTS], h2b[SLOTS], ph[SLOTS];
    uint32_t ee[SLOTS], lfi[SLOTS], fl[SLOTS];
    int gsl[SLOTS];
    {
      int cw = -1;
      RowT T;
#pragma unroll
      for (int sl = 0; sl < SLOTS; ++sl) {
        if (sl >= nact) break;  // wave-uniform
        const int base8 = (qb + sl) * 8;
        const int w = uni_i(__popcll(__ballot(ibase <= base8)) - 1);
        if (w != cw) {
          T = tg[w];
          cw = w;
        }
        // row t of target w's grid: frame f = floor(t / bpf), 16-bin block i.
        // (t + 1/2) / bpf lies at least 1/(2 bpf) from an integer; its FP32
        // value (reciprocal within 1 ulp, one fma) is within
        // 1.5 2^-23 (t + 1/2) / bpf of it, so truncation is exact while
        // t < 2^21 (rows per selection are bounded so at plan creation).
        // All products below are of non-negative operands under 2^24
        // (24-bit multiplies).
        const int t = base8 - T.item_base + rid8;
        const int f = (int)fmaf((float)t, T.rbpf, __int_as_float(T.pad[1]));
        const int i = T.ilo + t - (int)__umul24((uint32_t)f, (uint32_t)T.bpf);
        const bool ok = f < T.nF;
        int n = T.nlo + f;
        n -= n >= T.N ? T.N : 0;
        const int li = T.lbase + (int)__umul24((uint32_t)n, (uint32_t)T.lpf) + i;
        const int m0 = (i << LOG_ROW) + 2 * rl8;
        const bool v0 = ok && m0 < T.MR, v1 = ok && m0 + 1 < T.MR;
        const uint32_t e = (uint32_t)T.off + __umul24((uint32_t)n, (uint32_t)T.MR) + (uint32_t)m0;
        const uint32_t hrow = (uint32_t)T.hrow0 + __umul24((uint32_t)f, (uint32_t)T.hstep);
        // d_t = (m - c_t) mod M_w for the two bins (valid bins: m <= M_w / 2,
        // 0 <= c_t < M_w, so one correction suffices)
        const int Mw = T.Mw;
        int d1 = m0 - T.c1, d2 = m0 - T.c2;
        int d1b, d2b;
        if constexpr (P2) {
          d1 &= Mw - 1;
          d2 &= Mw - 1;
          d1b = (d1 + 1) & (Mw - 1);
          d2b = (d2 + 1) & (Mw - 1);
        } else {
          d1 += d1 < 0 ? Mw : 0;
          d2 += d2 < 0 ? Mw : 0;
          d1b = d1 + 1 == Mw ? 0 : d1 + 1;
          d2b = d2 + 1 == Mw ? 0 : d2 + 1;
        }
        const bool i1a = v0 && d1 <= T.span1, i1b = v1 && d1b <= T.span1;
        const bool i2a = v0 && pair && d2 <= T.span2, i2b = v1 && pair && d2b <= T.span2;
        // every lane loads (out-of-grid lanes from valid stand-in addresses;
        // the second bin of a pair may lie one element past its frame)
        r[sl] = ld_c4(rho + (v0 ? e : (uint32_t)p));
        h1a[sl] = tabs[i1a ? hrow + (uint32_t)d1 : 0u];
        h1b[sl] = tabs[i1b ? hrow + (uint32_t)d1b : 0u];
        if constexpr (H2) {
          const uint32_t hrow2 = hrow + (uint32_t)T.pad[2];
          h2a[sl] = tabs[i2a ? hrow2 + (uint32_t)d2 : 0u];
          h2b[sl] = tabs[i2b ? hrow2 + (uint32_t)d2b : 0u];
        }
        {
          const uint32_t x = T.ph0 + __umul24((uint32_t)f, T.phs);
          uint32_t pix;
          if constexpr (P2)
            pix = x & pm.mask;
          else
            pix = x - (uint32_t)magic_div((int)x, pm.mul, pm.sh) * (uint32_t)pm.Mv;
          ph[sl] = roots[root_off + pix];
        }
        ee[sl] = e;
        lfi[sl] = (uint32_t)li;
        gg[sl] = C4f{0.0f, 0.0f, 0.0f, 0.0f};
        if (pedantic) gg[sl] = ld_c4(gams + (v0 ? (uint32_t)(T.pad[0] + m0) : 0u));
        // the pedantic score applies to bins with a partner (not DC, not Nyquist)
        const bool pe0 = pedantic && m0 != 0 && m0 != T.MR - 1, pe1 = pedantic && m0 + 1 != T.MR - 1;
        fl[sl] = (ok ? 1u : 0u) | (v0 ? 2u : 0u) | (v1 ? 4u : 0u) | (i1a ? 8u : 0u) | (i1b ? 16u : 0u) |
                 (i2a ? 32u : 0u) | (i2b ? 64u : 0u) | (pe0 ? 128u : 0u) | (pe1 ? 256u : 0u);
        // touched-group slot of the row's group (wrapped frames, run B, lie
        // below run A)
        const int g = li >> LOG_GL;
        gsl[sl] = T.slot_base + (g >= T.gA_lo ? g - T.gA_lo : T.gA_n + g - T.gB_lo);
      }
    }
    __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0): the batch's loads (and the old leaves before them)
    // the row flags live in VGPRs across the two phases (not as scalar
    // masks); the old leaves count as arrived from here on
#pragma unroll
    for (int sl = 0; sl < SLOTS; ++sl) asm volatile("" : "+v"(fl[sl]));
#pragma unroll
    for (int x = 0; x < LPL; ++x) asm volatile("" : "+v"(o0[x]), "+v"(o1[x]));
    uint32_t n_upd = 0, n_blk = 0;
#pragma unroll
    for (int sl = 0; sl < SLOTS; ++sl) {
      if (sl >= nact) break;  // wave-uniform
      const uint32_t fs = fl[sl];
      const float cs = ph[sl].re, sn = ph[sl].im;
      // c (h1 phi) + conj(c) (h2 conj(phi)) for one bin
      auto upd = [&](Cx<float> a1, Cx<float> b2, float& re, float& im) {
        const float ar = a1.re * cs - a1.im * sn, ai = a1.re * sn + a1.im * cs;
        float ur = cc.re * ar - cc.im * ai, ui = cc.re * ai + cc.im * ar;
        if constexpr (H2) {
          const float br = b2.re * cs + b2.im * sn, bi = b2.im * cs - b2.re * sn;
          ur += cc.re * br + cc.im * bi;
          ui += cc.re * bi - cc.im * br;
        }
        re -= ur;
        im -= ui;
      };
      const Cx<float> z{0.0f, 0.0f};
      const Cx<float> a1 = (fs & 8u) ? h1a[sl] : z, a2 = (fs & 16u) ? h1b[sl] : z;
      Cx<float> b1 = z, b2 = z;
      if constexpr (H2) {
        b1 = (fs & 32u) ? h2a[sl] : z;
        b2 = (fs & 64u) ? h2b[sl] : z;
      }
      const bool nz0 = (a1.re != 0.0f) | (a1.im != 0.0f) | (b1.re != 0.0f) | (b1.im != 0.0f);
      const bool nz1 = (a2.re != 0.0f) | (a2.im != 0.0f) | (b2.re != 0.0f) | (b2.im != 0.0f);
      C4f rv = r[sl];
      upd(a1, b1, rv.x, rv.y);
      upd(a2, b2, rv.z, rv.w);
      if (nz0 | nz1) {
        if (fs & 4u)
          st_c4(rho + ee[sl], rv);
        else
          rho[ee[sl]] = Cx<float>{rv.x, rv.y};
      }
      float s0, s1;
      if (pedantic) {  // uniform
        s0 = sel_score<float>(rv.x, rv.y, Cx<float>{gg[sl].x, gg[sl].y}, (fs & 128u) != 0);
        s1 = sel_score<float>(rv.z, rv.w, Cx<float>{gg[sl].z, gg[sl].w}, (fs & 256u) != 0);
      } else {
        s0 = rv.x * rv.x + rv.y * rv.y;
        s1 = rv.z * rv.z + rv.w * rv.w;
      }
      const uint32_t bits0 = (fs & 2u) ? __float_as_uint(s0) : 0u;
      const uint32_t bits1 = (fs & 4u) ? __float_as_uint(s1) : 0u;
      uint32_t rm = bits0 > bits1 ? bits0 : bits1;
      rm = max_dpp32<0xB1>(rm);
      rm = max_dpp32<0x4E>(rm);
      rm = max_dpp32<0x141>(rm);  // half-row mirror: the two quads of an 8-lane row
      const bool hit0 = (fs & 2u) && bits0 == rm, hit1 = (fs & 4u) && bits1 == rm;
      const uint64_t bal = __ballot(hit0 | hit1);
      const uint32_t rowbits = (uint32_t)(bal >> (rid8 * 8)) & 0xFFu;
      const bool leader = (fs & 1u) && rowbits && lane == rid8 * 8 + __ffs(rowbits) - 1;
      n_upd += (uint32_t)(__popcll(__ballot(nz0)) + __popcll(__ballot(nz1)));
      n_blk += (uint32_t)__popcll(__ballot(leader));
      if (leader) {
        const uint32_t eb = ee[sl] + (hit0 ? 0u : 1u);  // lowest bin holding the row maximum
        const uint64_t key = ((uint64_t)rm << 32) | (uint64_t)(~eb);
        const uint32_t b = lfi[sl];
        leaves[b] = key;
        if (gsl[sl] < NPRE) lscr[gsl[sl] * GL + (b & (GL - 1))] = key;
      }
    }
    c_upd += n_upd;
    c_blk += n_blk;
  };
  // wave: next batch index from the shared counter
  auto grab = [&]() -> int {
    int qi = 0;
    if (lane == 0) qi = atomicAdd(rowq, 1);
    return uni_i(qi);
  };

  // first selection: full scan
  int cur = 0;
  if (wave == 0) select_into(scan_root(), 0);
  __syncthreads();
  ItR cr = read_it(0);

  for (;;) {
    if (k >= K) { stop = 1; break; }
    if (E <= Etarget) { stop = 2; break; }
    if (E < 0.0) { stop = 3; break; }
    if (uni_i(cr.I1.w)) {  // max score is zero
      stop = 4;
      break;
    }
    const RowT* tg = tg2 + cur * MAXW;
    const int p = uni_i(cr.I0.x);
    const bool pair = uni_i(cr.I1.x) != 0;
    const int T_items = uni_i(cr.I1.y), TG = uni_i(cr.I1.z);
    const uint32_t root_off = (uint32_t)uni_i(cr.I2.x);
    const PhaseMod pm{(uint32_t)uni_i(cr.I2.y), (uint32_t)uni_i(cr.I3.z), uni_i(cr.I3.x), uni_i(cr.I3.y)};
    const bool has2 = uni_i(cr.I2.w) != 0;
    const int ibase = cr.ibase, sbase = cr.sbase;
    const Cx<float> cc = cr.cc;
    const double Et = uni_d(cr.Et);
    if (wave == NW - 1 && lane == 0) {  // wave 0 is busy with the next candidate
      AtomRec ar;
      ar.w = cr.I0.y;
      ar.m = cr.I0.z;
      ar.n = cr.I0.w;
      ar.pad = 0;
      ar.re = (double)cc.re;
      ar.im = (double)cc.im;
      ar.E_after = E - Et;
      atoms[k] = ar;
    }
    E -= Et;
    ++k;

    // touched-group slots this wave merges: gs = wave and wave + NW; their
    // old leaves are loaded now and consumed after the update
    const int gs0 = wave, gs1 = wave + NW;
    const int g0 = uni_i(cr.g0), g1 = uni_i(cr.g1);
    uint64_t old0[LPL] = {}, old1[LPL] = {};
    if (gs0 < TG) {
#pragma unroll
      for (int x = 0; x < LPL; ++x) old0[x] = leaves[(uint32_t)(g0 * GL + lane + 64 * x)];
    }
    if (gs1 < TG) {
#pragma unroll
      for (int x = 0; x < LPL; ++x) old1[x] = leaves[(uint32_t)(g1 * GL + lane + 64 * x)];
    }

    // ---- wave 0: candidate for the next selection ----
    // The touched groups' keys are cleared (the merge below rewrites them);
    // the maximum over the others cannot change in this update, so it is the
    // next selection unless a touched group ends above it.
    if (wave == 0) {
      if (TG <= 64) {
        if (lane < TG) gkey[cr.gl] = 0ull;
      } else {
        for (int w = 0; w < W; ++w) {
          const int4 a = *reinterpret_cast<const int4*>(&tg[w].gA_lo);
          const int alo = uni_i(a.x), an = uni_i(a.y), blo = uni_i(a.z), bn = uni_i(a.w);
          for (int i = lane; i < an; i += 64) gkey[alo + i] = 0ull;
          for (int i = lane; i < bn; i += 64) gkey[blo + i] = 0ull;
        }
      }
      const uint64_t bk = scan_root();
      select_into(bk, cur ^ 1);
      if (lane == 0) ckey[cur ^ 1] = bk;
      __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0): no load of this block stays in flight into the rows
    }

    // ---- rows: batches of bs slots (8 rows each) from a shared counter,
    // sized so that waves 1..NW-1 take one batch each; wave 0 takes what is
    // left once its candidate is built.  Each batch waits for all its loads at once, which
    // also completes the old-leaf loads above, so the merge does not wait on
    // this wave's row stores.
    {
      const int nslots = T_items >> 3;
      const int bs = min(min(SLOTS, A.slot_cap), max(1, (nslots + NW - 2) / (NW - 1)));
      int qb = grab() * bs;
      if (qb < nslots) {
        do {
          if (has2)
            do_batch(std::true_type{}, old0, old1, tg, qb, min(bs, nslots - qb), ibase, p, pair, root_off, pm,
                     cc);
          else
            do_batch(std::false_type{}, old0, old1, tg, qb, min(bs, nslots - qb), ibase, p, pair, root_off, pm,
                     cc);
          qb = grab() * bs;
        } while (qb < nslots);
      } else {
        __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0)
#pragma unroll
        for (int x = 0; x < LPL; ++x) asm volatile("" : "+v"(old0[x]), "+v"(old1[x]));
      }
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      *rowq = 0;
      tmax[cur ^ 1] = 0ull;  // read by every wave after the previous merge, before this barrier
    }

    // ---- touched groups: merge old and rewritten leaves ----
    auto merge_slot = [&](int gs, int g, const uint64_t* old) {
      uint64_t scv[LPL];
#pragma unroll
      for (int x = 0; x < LPL; ++x) scv[x] = lscr[gs * GL + lane + 64 * x];
      uint64_t cand[LPL];
#pragma unroll
      for (int x = 0; x < LPL; ++x) {
        lscr[gs * GL + lane + 64 * x] = KEY_SENT;
        cand[x] = scv[x] != KEY_SENT ? scv[x] : old[x];
      }
      // pairwise tree: depth log2(LPL)
#pragma unroll
      for (int w2 = LPL / 2; w2 >= 1; w2 /= 2)
#pragma unroll
        for (int x = 0; x < w2; ++x) cand[x] = umax64(cand[x], cand[x + w2]);
      const uint64_t best = cand[0];
      const uint64_t wm = wave_max_key2<float>(best);
      if (lane == 0) {
        gkey[g] = wm;
        atomicMax((unsigned long long*)&tmax[cur], (unsigned long long)wm);
      }
      ++c_grp;
    };
    if constexpr (XP) {
      // slots beyond the preloaded ones: the leaves in global memory are
      // current.  The loads of a wave's first two such slots are issued before
      // its preloaded merges, so that their latency overlaps them.
      auto slot_group = [&](int gs) -> int {
        if (gs < 64) return uni_i(it2[cur].glist[gs]);
        const int w = uni_i(__popcll(__ballot(sbase <= gs)) - 1);
        const int4 a = *reinterpret_cast<const int4*>(&tg[w].gA_lo);
        const int c = gs - tg[w].slot_base;
        return uni_i(c < a.y ? a.x + c : a.z + (c - a.y));
      };
      auto fold_group = [&](int g, const uint64_t* v) {
        uint64_t best = 0ull;
#pragma unroll
        for (int x = 0; x < LPL; ++x) best = umax64(best, v[x]);
        const uint64_t wm = wave_max_key2<float>(best);
        if (lane == 0) {
          gkey[g] = wm;
          atomicMax((unsigned long long*)&tmax[cur], (unsigned long long)wm);
        }
        ++c_grp;
      };
      const int gx0 = NPRE + wave, gx1 = NPRE + NW + wave;
      int ga0 = 0, ga1 = 0;
      uint64_t ex0[LPL], ex1[LPL];
      if (gx0 < TG) {
        ga0 = slot_group(gx0);
#pragma unroll
        for (int x = 0; x < LPL; ++x) ex0[x] = leaves[(uint32_t)(ga0 * GL + lane + 64 * x)];
      }
      if (gx1 < TG) {
        ga1 = slot_group(gx1);
#pragma unroll
        for (int x = 0; x < LPL; ++x) ex1[x] = leaves[(uint32_t)(ga1 * GL + lane + 64 * x)];
      }
      if (gs0 < TG) merge_slot(gs0, g0, old0);
      if (gs1 < TG) merge_slot(gs1, g1, old1);
      if (gx0 < TG) fold_group(ga0, ex0);
      if (gx1 < TG) fold_group(ga1, ex1);
      for (int gs = NPRE + 2 * NW + wave; gs < TG; gs += NW) {
        const int g = slot_group(gs);
        uint64_t v[LPL];
#pragma unroll
        for (int x = 0; x < LPL; ++x) v[x] = leaves[(uint32_t)(g * GL + lane + 64 * x)];
        fold_group(g, v);
      }
    } else {
      if (gs0 < TG) merge_slot(gs0, g0, old0);
      if (gs1 < TG) merge_slot(gs1, g1, old1);
      // slots beyond the preloaded ones: the leaves in global memory are current
      for (int gs = NPRE + wave; gs < TG; gs += NW) {
        int g;
        if (gs < 64) {
          g = uni_i(it2[cur].glist[gs]);
        } else {
          const int w = uni_i(__popcll(__ballot(sbase <= gs)) - 1);
          const int4 a = *reinterpret_cast<const int4*>(&tg[w].gA_lo);
          const int c = gs - tg[w].slot_base;
          g = uni_i(c < a.y ? a.x + c : a.z + (c - a.y));
        }
        uint64_t best = 0ull;
#pragma unroll
        for (int x = 0; x < LPL; ++x) best = umax64(best, leaves[(uint32_t)(g * GL + lane + 64 * x)]);
        const uint64_t wm = wave_max_key2<float>(best);
        if (lane == 0) {
          gkey[g] = wm;
          atomicMax((unsigned long long*)&tmax[cur], (unsigned long long)wm);
        }
        ++c_grp;
      }
    }
    __syncthreads();

    // the candidate stands unless a touched group now holds a larger key
    const uint64_t kc = ckey[cur ^ 1], kt = tmax[cur];
    cur ^= 1;
    cr = read_it(cur);
    if (kc < kt) {
      if (wave == 0) select_into(kt, cur);
      __syncthreads();
      cr = read_it(cur);
    }
  }

  if (lane == 0) {
    atomicAdd((unsigned long long*)&A.state[s].updated, (unsigned long long)c_upd);
    atomicAdd((unsigned long long*)&A.state[s].blocks, (unsigned long long)c_blk);
    atomicAdd((unsigned long long*)&A.state[s].groups, (unsigned long long)c_grp);
  }
  if (wave == 0 && lane == 0) {
    A.state[s].E = E;
    A.state[s].k = k;
    A.state[s].stop = stop;
  }
}

template <int NT, int SLOTS, int GL, bool P2, bool XP>
__global__ void __launch_bounds__(NT) k_mp32(MPArgs A) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  __shared__ int s_next;
  const int lane = threadIdx.x & 63, wave = uni_i(threadIdx.x >> 6);
  for (;;) {
    if (threadIdx.x == 0) s_next = atomicAdd(A.queue, 1);
    __syncthreads();
    const int qi = uni_i(s_next);
    __syncthreads();
    if (qi >= A.batch) break;
    mp_signal32<NT, SLOTS, GL, P2, XP>(A, uni_i(A.order[qi]), smem_raw, lane, wave);
  }
}

__global__ void k_fill_i32(int32_t* p, int n, int v) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

// --------------------------------------------------------------------------
// Synthesis of real atoms (Eq. idgtreal), accumulated in FP64.  The padded
// signal is cut into segments of RS_SEG samples, one workgroup each.  A
// workgroup walks the atoms in selection order and adds the part of each atom
// that falls into its segment; thread t owns the samples lo + t + T r of the
// segment, so every sample receives its contributions in selection order
// without atomics (the result does not depend on the number of workgroups).
// The last step rounds the segment to the output type.

constexpr int RS_SEG = 8192;
constexpr int RS_NT = 256;

template <typename YT>
__global__ void __launch_bounds__(RS_NT) k_resynth(const AtomRec* __restrict__ atoms,
                                                   const SigState* __restrict__ st,
                                                   const DictDev* __restrict__ dicts,
                                                   const double* __restrict__ win64, int64_t Lp,
                                                   double* __restrict__ acc, YT* __restrict__ y) {
  const int64_t T = blockDim.x, tid = threadIdx.x;
  const int64_t lo = (int64_t)blockIdx.x * RS_SEG, hi = lo + RS_SEG < Lp ? lo + RS_SEG : Lp;
  const int64_t n_atoms = st->k;
  for (int64_t l = lo + tid; l < hi; l += T) acc[l] = 0.0;
  // adds samples l in [a, b) of the atom, whose window sample tp is l + sh
  auto add = [&](const AtomRec& at, const DictDev& D, const double* g, double mult, int64_t a, int64_t b,
                 int64_t sh) {
    int64_t l = a + ((tid - (a - lo)) % T + T) % T;  // first owned sample at or after a
    for (; l < b; l += T) {
      const int64_t tp = l + sh;
      const int64_t t = tp - D.gl / 2;
      int64_t pi = ((int64_t)at.m * t) % D.M;
      if (pi < 0) pi += D.M;
      double sn, cs;
      sincospi(2.0 * (double)pi / (double)D.M, &sn, &cs);
      acc[l] += mult * g[tp] * (at.re * cs - at.im * sn);
    }
  };
  for (int64_t i = 0; i < n_atoms; ++i) {
    const AtomRec at = atoms[i];
    const DictDev D = dicts[at.w];
    // window sample tp = 0 (t = -gl/2) sits at s0, wrapped into [0, Lp):
    // samples s0 .. s0 + split - 1, then 0 .. gl - split - 1
    int64_t s0 = ((int64_t)at.n * D.a - D.gl / 2) % Lp;
    if (s0 < 0) s0 += Lp;
    const int64_t split = D.gl < Lp - s0 ? D.gl : Lp - s0;
    const int64_t a1 = s0 > lo ? s0 : lo, b1 = s0 + split < hi ? s0 + split : hi;
    const int64_t b2 = D.gl - split < hi ? D.gl - split : hi;
    if (a1 >= b1 && lo >= b2) continue;  // uniform: the atom misses the segment
    const double mult = (at.m != 0 && 2 * at.m != D.M) ? 2.0 : 1.0;
    const double* g = win64 + D.win_off;
    if (a1 < b1) add(at, D, g, mult, a1, b1, -s0);
    if (lo < b2) add(at, D, g, mult, lo, b2, Lp - s0);
  }
  for (int64_t l = lo + tid; l < hi; l += T) y[l] = (YT)acc[l];
}

// Solution vector (Alg. 1 solution update): c(m, n) = sum of c~ of the atoms
// selected at (w, m, n), added in selection order.  Entries are cut into
// ranges of CF_SEG, one workgroup each; thread t owns the entries
// lo + t + T r of its range.
constexpr int CF_SEG = 16384;

__global__ void __launch_bounds__(1024) k_coefs(const AtomRec* __restrict__ atoms, const SigState* __restrict__ st,
                                                int w, int MR, int64_t n_entries, double2* __restrict__ c) {
  const int64_t T = blockDim.x, tid = threadIdx.x;
  const int64_t lo = (int64_t)blockIdx.x * CF_SEG, hi = lo + CF_SEG < n_entries ? lo + CF_SEG : n_entries;
  const int64_t n_atoms = st->k;
  for (int64_t i = lo + tid; i < hi; i += T) c[i] = make_double2(0.0, 0.0);
  for (int64_t i = 0; i < n_atoms; ++i) {
    const AtomRec at = atoms[i];
    if (at.w != w) continue;
    const int64_t idx = (int64_t)at.n * MR + at.m;
    if (idx < lo || idx >= hi || (idx - lo) % T != tid) continue;
    double2 v = c[idx];
    v.x += at.re;
    v.y += at.im;
    c[idx] = v;
  }
}

// --------------------------------------------------------------------------
// Reset procedure (Alg. 2).  The true residual r = x - D c over the padded
// length is kept in FP64, signal s at roff[s] (stride L_padded).  After each
// inner loop the new selections are synthesized and subtracted in selection
// order (one workgroup per signal; thread t owns the samples l = t mod T, so
// no atomics), the residual's energy becomes the new error, and the signal is
// finished when that true error reaches the target, the selection cap is
// reached, the coefficients vanished, or the inner loop made no selection.

template <typename XT>
__global__ void __launch_bounds__(256) k_reset_init(const XT* __restrict__ x, const SigDev* __restrict__ sigs,
                                                    const int64_t* __restrict__ roff, double* __restrict__ r) {
  const int s = blockIdx.y;
  const SigDev& S = sigs[s];
  for (int64_t l = (int64_t)blockIdx.x * 256 + threadIdx.x; l < S.Lp; l += (int64_t)gridDim.x * 256)
    r[roff[s] + l] = l < S.L ? (double)x[S.x_off + l] : 0.0;
}

__global__ void __launch_bounds__(1024) k_reset_update(const AtomRec* __restrict__ atoms,
                                                       const SigDev* __restrict__ sigs, SigState* __restrict__ st,
                                                       const DictDev* __restrict__ dicts,
                                                       const double* __restrict__ win64,
                                                       const int64_t* __restrict__ roff, double* __restrict__ r,
                                                       double snr_db, int64_t K_total, int* __restrict__ active) {
  __shared__ double part[1024];
  const int s = blockIdx.x;
  const SigState S0 = st[s];
  if (S0.done) return;
  const SigDev& S = sigs[s];
  const int64_t T = blockDim.x, tid = threadIdx.x;
  const int64_t Lp = S.Lp;
  double* rs = r + roff[s];
  const AtomRec* as = atoms + S.atom_base;
  for (int64_t i = S0.kout; i < S0.k; ++i) {
    const AtomRec at = as[i];
    const DictDev D = dicts[at.w];
    const double mult = (at.m != 0 && 2 * at.m != D.M) ? 2.0 : 1.0;
    const double* g = win64 + D.win_off;
    int64_t s0 = ((int64_t)at.n * D.a - D.gl / 2) % Lp;
    if (s0 < 0) s0 += Lp;
    // samples of the support by owner thread (l mod T); tp < split: l = s0 + tp, else l = s0 + tp - Lp
    const int64_t split = D.gl < Lp - s0 ? D.gl : Lp - s0;
    int64_t t0 = (tid - s0) % T;
    if (t0 < 0) t0 += T;
    for (int64_t tp = t0; tp < split; tp += T) {
      const int64_t t = tp - D.gl / 2;
      int64_t pi = ((int64_t)at.m * t) % D.M;
      if (pi < 0) pi += D.M;
      double sn, cs;
      sincospi(2.0 * (double)pi / (double)D.M, &sn, &cs);
      rs[s0 + tp] -= mult * g[tp] * (at.re * cs - at.im * sn);
    }
    for (int64_t l = tid; l < D.gl - split; l += T) {
      const int64_t tp = l + Lp - s0;
      const int64_t t = tp - D.gl / 2;
      int64_t pi = ((int64_t)at.m * t) % D.M;
      if (pi < 0) pi += D.M;
      double sn, cs;
      sincospi(2.0 * (double)pi / (double)D.M, &sn, &cs);
      rs[l] -= mult * g[tp] * (at.re * cs - at.im * sn);
    }
  }
  double acc = 0.0;
  for (int64_t l = tid; l < Lp; l += T) acc += rs[l] * rs[l];
  part[tid] = acc;
  __syncthreads();
  for (int h = (int)T / 2; h > 0; h >>= 1) {
    if (tid < h) part[tid] += part[tid + h];
    __syncthreads();
  }
  if (tid == 0) {
    const double Eout = part[0];
    const double Etg = snr_db > 0.0 ? S0.E0 * exp10(-snr_db / 10.0) : -__builtin_huge_val();
    int64_t K = K_total > 0 ? K_total : Lp / 5;
    if (K > S.cap) K = S.cap;
    int stop = 0;
    if (Eout <= Etg) stop = 2;
    else if (S0.k >= K) stop = 1;
    else if (S0.stop == 4) stop = 4;
    else if (S0.k == S0.kout) stop = S0.stop ? S0.stop : 1;
    SigState n = S0;
    n.Eout = Eout;
    n.E = Eout;
    n.kout = S0.k;
    n.resets = S0.resets + 1;
    n.stop = stop;
    n.done = stop != 0;
    st[s] = n;
    if (!stop) atomicAdd(active, 1);
  }
}

// --------------------------------------------------------------------------
// host-side launchers (called from mpg_api.cpp)

#define CHK(x)                         \
  do {                                 \
    hipError_t e_ = (x);               \
    if (e_ != hipSuccess) return e_;   \
  } while (0)

hipError_t launch_roots(int M, int n, int sign, double2* o64, float2* o32, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  k_roots<<<(n + 255) / 256, 256, 0, st>>>(M, n, sign, o64, o32);
  return hipGetLastError();
}

hipError_t launch_gram_full(const double* gw, int glw, const double* gv, int glv, int amin, int D,
                            int Mmax, const double2* roots, double2* out, hipStream_t st) {
  dim3 grid(2 * D + 1, (Mmax + 255) / 256);
  k_gram_full<<<grid, 256, 0, st>>>(gw, glw, gv, glv, amin, D, Mmax, roots, out);
  return hipGetLastError();
}

hipError_t launch_gram_absmax(const double2* t, int64_t n, unsigned long long* out, hipStream_t st) {
  k_gram_absmax<<<256, 256, 0, st>>>(t, n, out);
  return hipGetLastError();
}

hipError_t launch_gram_box(const double2* t, int D, int Mmax, double thr, int* box, hipStream_t st) {
  k_gram_box<<<2 * D + 1, 256, 0, st>>>(t, D, Mmax, thr, box);
  return hipGetLastError();
}

hipError_t launch_gram_extract(const double2* t, int D, int Mmax, double thr, int dbox, int mu_lo,
                               int width, double2* o64, float2* o32, hipStream_t st) {
  if (dbox < 0 || width <= 0) return hipSuccess;
  k_gram_extract<<<2 * dbox + 1, 256, 0, st>>>(t, D, Mmax, thr, dbox, mu_lo, width, o64, o32);
  return hipGetLastError();
}

hipError_t launch_energy(const void* x, int dtype, const SigDev* sigs, int batch, double* part, SigState* st_,
                         hipStream_t st) {
  if (batch <= 0) return hipSuccess;
  const dim3 grid((unsigned)batch, ENERGY_PARTS);
  if (dtype == 0)
    k_energy_part<float><<<grid, 256, 0, st>>>((const float*)x, sigs, part);
  else
    k_energy_part<double><<<grid, 256, 0, st>>>((const double*)x, sigs, part);
  CHK(hipGetLastError());
  k_energy_fin<<<batch, 64, 0, st>>>(part, st_);
  return hipGetLastError();
}

hipError_t launch_dgt(bool f64, bool dft64, const void* x, int dtype, const SigDev* sigs, int w, int gl, int a,
                      int M, int MR, const int64_t* frame_prefix, int batch, int64_t frames,
                      const void* win, const void* tw, void* planes, void* leaves, const void* gam, int pedantic,
                      const double2* roots64, hipStream_t st) {
  if (frames <= 0) return hipSuccess;
  // mode 0: M a power of two (H = 2^logP), 1: M = 3 2^k (H = 3 2^logP),
  // 2: any other M (defining sum)
  int mode = 2, logP = 0;
  for (int c = 0; c < 2; ++c) {
    const int Pc = c == 0 ? M / 2 : M / 6;
    if (Pc >= 1 && (Pc & (Pc - 1)) == 0 && Pc * (c == 0 ? 2 : 6) == M) {
      mode = c;
      while ((1 << logP) < Pc) ++logP;
      break;
    }
  }
  const bool r64 = f64 || dft64;  // FFT arithmetic in FP64
  const size_t sh = (size_t)(M / 2 + M / 64) * (r64 ? 16 : 8);  // H entries + one pad per 32
  if (sh > 160 * 1024) return hipErrorInvalidValue;
  const dim3 grid((unsigned)frames);
  // threads per frame: H / 2 (one radix-2 pair per thread, two samples per
  // thread in the load), clamped to 64 .. 256
  const int nt = M / 4 < 64 ? 64 : (M / 4 > 256 ? 256 : M / 4);
#define MPG_DGT(RT, XTT, OT)                                                                                \
  do {                                                                                                      \
    if (sh > 64 * 1024)                                                                                     \
      CHK(hipFuncSetAttribute((const void*)k_dgt<RT, XTT, OT>, hipFuncAttributeMaxDynamicSharedMemorySize, \
                              (int)sh));                                                                    \
    k_dgt<RT, XTT, OT><<<grid, nt, sh, st>>>((const XTT*)x, sigs, w, gl, a, M, mode, logP, MR, frame_prefix, \
                                             batch, (const RT*)win, (const Cx<RT>*)tw, (Cx<OT>*)planes,     \
                                             (Leaf<OT>*)leaves, (const Cx<OT>*)gam, pedantic, roots64);     \
  } while (0)
  if (f64) {
    if (dtype == 0) MPG_DGT(double, float, double);
    else MPG_DGT(double, double, double);
  } else if (dft64) {
    if (dtype == 0) MPG_DGT(double, float, float);
    else MPG_DGT(double, double, float);
  } else {
    if (dtype == 0) MPG_DGT(float, float, float);
    else MPG_DGT(float, double, float);
  }
#undef MPG_DGT
  return hipGetLastError();
}

hipError_t launch_dft_tables(int fmt, int N, int Np, uint16_t* out, hipStream_t st) {
  const dim3 blk(16, 16), grid((unsigned)(Np / 16), (unsigned)(Np / 16));
  if (fmt == 0)
    k_dft_tables<0><<<grid, blk, 0, st>>>(N, Np, out);
  else
    k_dft_tables<1><<<grid, blk, 0, st>>>(N, Np, out);
  return hipGetLastError();
}

template <int FMT, typename XT, int LN1, int LN2>
static hipError_t launch_dgt_mfw_t(const void* x, const SigDev* sigs, int w, int gl, int a, int MR,
                                   const int64_t* frame_prefix, int batch, int64_t frames, const float* win,
                                   const void* tw, const uint16_t* F1, const uint16_t* F2, void* planes,
                                   void* leaves, const void* gam, int pedantic, hipStream_t st) {
  using Sh = MfwShape<LN1, LN2>;
  const auto kern = k_dgt_mfw<FMT, XT, LN1, LN2>;
  const size_t sh = Sh::lds_bytes();
  if (sh > 64 * 1024)
    CHK(hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)sh));
  // as many workgroups as are resident at once, at most one wave per frame group
  int dev = 0, ncu = 0, occ = 0;
  CHK(hipGetDevice(&dev));
  CHK(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
  CHK(hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, (const void*)kern, 256, sh));
  const int64_t groups = (frames + Sh::FPW - 1) / Sh::FPW;
  const int64_t want = (groups + 3) / 4, cap = (int64_t)(ncu > 0 ? ncu : 1) * (occ > 0 ? occ : 1);
  const unsigned grid = (unsigned)(want < cap ? want : cap);
  kern<<<grid, 256, sh, st>>>((const XT*)x, sigs, w, gl, a, MR, frame_prefix, batch, frames, win,
                              (const Cx<float>*)tw, F1, F2, (Cx<float>*)planes, (Leaf<float>*)leaves,
                              (const Cx<float>*)gam, pedantic);
  return hipGetLastError();
}

hipError_t launch_dgt_mfma(int fmt, const void* x, int dtype, const SigDev* sigs, int w, int gl, int a, int M,
                           int MR, const int64_t* frame_prefix, int batch, int64_t frames, const float* win,
                           const void* tw, int N1, int N2, const uint16_t* F1, const uint16_t* F2, void* planes,
                           void* leaves, const void* gam, int pedantic, int64_t max_Lp, hipStream_t st) {
  if (frames <= 0) return hipSuccess;
  // H = 128 .. 2048: frame groups per wave (the factorisations the plan
  // makes), while the sample byte offsets of every signal fit in 31 bits
  const int H = M / 2;
  if (max_Lp * 8 < ((int64_t)1 << 31) && (H == 128 && N1 == 16 && N2 == 8) || (H == 256 && N1 == 16 && N2 == 16) ||
      (H == 512 && N1 == 32 && N2 == 16) || (H == 1024 && N1 == 32 && N2 == 32) ||
      (H == 2048 && N1 == 64 && N2 == 32)) {
    if (MR != H + 1) return hipErrorInvalidValue;
#define DGT_MFW(L1, L2)                                                                                        \
  do {                                                                                                         \
    if (fmt == 0) {                                                                                            \
      if (dtype == 0) return launch_dgt_mfw_t<0, float, L1, L2>(x, sigs, w, gl, a, MR, frame_prefix, batch,   \
                                                                 frames, win, tw, F1, F2, planes, leaves, gam, \
                                                                 pedantic, st);                               \
      return launch_dgt_mfw_t<0, double, L1, L2>(x, sigs, w, gl, a, MR, frame_prefix, batch, frames, win, tw,  \
                                                  F1, F2, planes, leaves, gam, pedantic, st);                  \
    }                                                                                                          \
    if (dtype == 0) return launch_dgt_mfw_t<1, float, L1, L2>(x, sigs, w, gl, a, MR, frame_prefix, batch,     \
                                                               frames, win, tw, F1, F2, planes, leaves, gam,   \
                                                               pedantic, st);                                 \
    return launch_dgt_mfw_t<1, double, L1, L2>(x, sigs, w, gl, a, MR, frame_prefix, batch, frames, win, tw, F1, \
                                                F2, planes, leaves, gam, pedantic, st);                        \
  } while (0)
    switch (H) {
      case 128: DGT_MFW(4, 3);
      case 256: DGT_MFW(4, 4);
      case 512: DGT_MFW(5, 4);
      case 1024: DGT_MFW(5, 5);
      default: DGT_MFW(6, 5);
    }
#undef DGT_MFW
  }
  const size_t sh = (size_t)M * 8;  // z / B and Z, H complex FP32 each
  if (sh > 160 * 1024) return hipErrorInvalidValue;
  const dim3 grid((unsigned)frames);
  // one wave per 16-row block of the larger GEMM dimension (1 to 4 waves)
  const int tiles = (N1 > N2 ? N1 : N2) / 16;
  const int nt = 64 * (tiles < 1 ? 1 : (tiles > 4 ? 4 : tiles));
  const Cx<float>* twc = (const Cx<float>*)tw;
  Cx<float>* pl = (Cx<float>*)planes;
  Leaf<float>* lv = (Leaf<float>*)leaves;
#define DGT_MFMA(F, XT)                                                                                     \
  do {                                                                                                      \
    if (sh > 64 * 1024)                                                                                     \
      CHK(hipFuncSetAttribute((const void*)k_dgt_mfma<F, XT>, hipFuncAttributeMaxDynamicSharedMemorySize,  \
                              (int)sh));                                                                    \
    k_dgt_mfma<F, XT><<<grid, nt, sh, st>>>((const XT*)x, sigs, w, gl, a, M, MR, frame_prefix, batch, win,   \
                                             twc, N1, N2, F1, F2, pl, lv, (const Cx<float>*)gam, pedantic); \
  } while (0)
  if (fmt == 0) {
    if (dtype == 0) DGT_MFMA(0, float);
    else DGT_MFMA(0, double);
  } else {
    if (dtype == 0) DGT_MFMA(1, float);
    else DGT_MFMA(1, double);
  }
#undef DGT_MFMA
  return hipGetLastError();
}

hipError_t launch_reset_init(const void* x, int dtype, const SigDev* sigs, int batch, int64_t max_Lp,
                             const int64_t* roff, double* r, hipStream_t st) {
  const int64_t nb = (max_Lp + 255) / 256;
  const dim3 grid((unsigned)(nb < 4096 ? nb : 4096), (unsigned)batch);
  if (dtype == 0)
    k_reset_init<float><<<grid, 256, 0, st>>>((const float*)x, sigs, roff, r);
  else
    k_reset_init<double><<<grid, 256, 0, st>>>((const double*)x, sigs, roff, r);
  return hipGetLastError();
}

hipError_t launch_reset_update(const AtomRec* atoms, const SigDev* sigs, SigState* st_, const DictDev* dicts,
                               const double* win64, const int64_t* roff, double* r, int batch, double snr_db,
                               int64_t K_total, int* active, hipStream_t st) {
  k_reset_update<<<batch, 1024, 0, st>>>(atoms, sigs, st_, dicts, win64, roff, r, snr_db, K_total, active);
  return hipGetLastError();
}

size_t leaf_bytes(bool f64) { return f64 ? sizeof(Leaf<double>) : sizeof(Leaf<float>); }

template <typename R, int NT, int SLOTS>
static hipError_t launch_mp_t(const MPArgs& a, int grid, bool preload, hipStream_t st) {
  const size_t sh = mp_lds_bytes<R, NT, SLOTS>(a.n_groups_max, preload);
  if (sh > 160 * 1024) return hipErrorInvalidValue;
  CHK(hipFuncSetAttribute((const void*)k_mp<R, NT, SLOTS>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)sh));
  k_mp<R, NT, SLOTS><<<grid, NT, sh, st>>>(a);
  return hipGetLastError();
}

template <int NT, int SLOTS, int GL, bool P2, bool XP>
static hipError_t launch_mp32_t(const MPArgs& a, int grid, hipStream_t st) {
  const size_t sh = mp32_lds_bytes<NT, GL>(a.n_groups_max);
  if (sh > 160 * 1024) return hipErrorInvalidValue;
  CHK(hipFuncSetAttribute((const void*)k_mp32<NT, SLOTS, GL, P2, XP>, hipFuncAttributeMaxDynamicSharedMemorySize,
                          (int)sh));
  k_mp32<NT, SLOTS, GL, P2, XP><<<grid, NT, sh, st>>>(a);
  return hipGetLastError();
}

// The early loads of the groups beyond the preloaded ones have their own
// 768-thread kernels (kept apart: their registers change the allocation of
// the whole loop); 512-thread plans merge those groups as the other kernels do.
template <int NT, int SLOTS, int GL>
static hipError_t launch_mp32_p(const MPArgs& a, int grid, hipStream_t st) {
  if constexpr (NT == 768) {
    if (a.xpre)
      return a.p2 ? launch_mp32_t<NT, SLOTS, GL, true, true>(a, grid, st)
                  : launch_mp32_t<NT, SLOTS, GL, false, true>(a, grid, st);
  }
  return a.p2 ? launch_mp32_t<NT, SLOTS, GL, true, false>(a, grid, st)
              : launch_mp32_t<NT, SLOTS, GL, false, false>(a, grid, st);
}

// LDS bytes of the MP kernel for the launch shape (0: unsupported shape).
size_t mp_shmem_bytes(bool f64, int nt, int G, int n_groups_max) {
  if (f64) {
    const bool preload = G == GLEAVES;
    return nt == 512 ? mp_lds_bytes<double, 512, 4>(n_groups_max, preload) : 0;
  }
  if (nt != 512 && nt != 768) return 0;
  if (G == 128) return nt == 768 ? mp32_lds_bytes<768, 128>(n_groups_max) : mp32_lds_bytes<512, 128>(n_groups_max);
  if (G == 256) return nt == 768 ? mp32_lds_bytes<768, 256>(n_groups_max) : mp32_lds_bytes<512, 256>(n_groups_max);
  return 0;
}

hipError_t launch_mp(bool f64, int nt, const MPArgs& a, int grid, hipStream_t st) {
  k_fill_i32<<<1, 64, 0, st>>>(a.queue, 1, 0);
  CHK(hipGetLastError());
  if (f64) {
    const bool preload = a.G == GLEAVES;
    if (nt != 512) return hipErrorInvalidValue;
    return launch_mp_t<double, 512, 4>(a, grid, preload, st);
  }
  // tiles of 1 or 2 slots run the two-slot kernel with a cap; 4 slots (512
  // threads only) have their own
  if (a.slot_cap == 4 && nt != 512) return hipErrorInvalidValue;
  if (a.G == 128) {
    if (nt == 768) return launch_mp32_p<768, 2, 128>(a, grid, st);
    if (a.slot_cap == 4) return launch_mp32_p<512, 4, 128>(a, grid, st);
    return launch_mp32_p<512, 2, 128>(a, grid, st);
  }
  if (a.G == 256) {
    if (nt == 768) return launch_mp32_p<768, 2, 256>(a, grid, st);
    if (a.slot_cap == 4) return launch_mp32_p<512, 4, 256>(a, grid, st);
    return launch_mp32_p<512, 2, 256>(a, grid, st);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_resynth(const AtomRec* atoms, const SigState* st_, const DictDev* dicts, const double* win64,
                          int64_t Lp, double* acc, void* y, int dtype, hipStream_t st) {
  if (Lp <= 0) return hipSuccess;
  const unsigned g = (unsigned)((Lp + RS_SEG - 1) / RS_SEG);
  if (dtype == 0)
    k_resynth<float><<<g, RS_NT, 0, st>>>(atoms, st_, dicts, win64, Lp, acc, (float*)y);
  else
    k_resynth<double><<<g, RS_NT, 0, st>>>(atoms, st_, dicts, win64, Lp, acc, (double*)y);
  return hipGetLastError();
}

// ---- scratch of the allocation-free synthesis (mp_resynth_static) ----
// The FP64 accumulator of one signal lives in this module-scope array instead
// of a plan buffer.  Each device that loads the library holds its own copy
// until the process ends.  In host code the name `scratch` is a host-side
// stand-in and not a device address: host code uses only the address that
// hipGetSymbolAddress returns for the current device (kept per device below).
static __device__ __align__(256) double scratch[STATIC_RESYNTH_MAX];

namespace {
std::mutex g_scratch_mu;
void* g_scratch_ptr[MAX_DEVICES] = {};
}  // namespace

hipError_t static_scratch(double** out, int64_t* n_out) {
  int dev = -1;
  CHK(hipGetDevice(&dev));
  if (dev < 0 || dev >= MAX_DEVICES) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    CHK(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));  // device `dev` is current
    if (!ptr) return hipErrorInvalidSymbol;
    g_scratch_ptr[dev] = ptr;
  }
  *out = static_cast<double*>(g_scratch_ptr[dev]);
  *n_out = STATIC_RESYNTH_MAX;
  return hipSuccess;
}

hipError_t launch_coefs(const AtomRec* atoms, const SigState* st_, int w, int MR, int64_t n_entries, void* c,
                        hipStream_t st) {
  if (n_entries <= 0) return hipSuccess;
  const unsigned g = (unsigned)((n_entries + CF_SEG - 1) / CF_SEG);
  k_coefs<<<g, 1024, 0, st>>>(atoms, st_, w, MR, n_entries, (double2*)c);
  return hipGetLastError();
}

}  // namespace mpg
