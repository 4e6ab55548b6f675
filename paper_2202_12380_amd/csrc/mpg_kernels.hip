// HIP kernels of libmpg (gfx950 / CDNA4, wave64).
//
// Paper: Prusa, Holighaus, Balazs, "Fast Matching Pursuit with Multi-Gabor
// Dictionaries", ACM TOMS 47(3), 2021.  Notation: system w has window g_w
// of length gl_w, hop a_w, M_w channels, N_w = L / a_w frames and M_w/2 + 1
// reduced bins (Sec. 5).  A selected atom is (v, k, j); a target coefficient
// is (w, m, n).
#include <hip/hip_runtime.h>
#include <stdint.h>

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

// A leaf / tree node: key of the block maximum and the complex value there.
template <typename R>
struct Leaf;
template <>
struct __align__(16) Leaf<float> {
  uint64_t key;
  float re, im;
};
template <>
struct __align__(16) Leaf<double> {
  uint64_t v;
  uint32_t n, pad;
  double re, im;
};

__device__ __forceinline__ uint64_t leaf_key(const Leaf<float>& l) { return l.key; }
__device__ __forceinline__ Key96 leaf_key(const Leaf<double>& l) { return Key96{l.v, l.n}; }
__device__ __forceinline__ Leaf<float> make_leaf(uint64_t k, float re, float im) {
  Leaf<float> l;
  l.key = k;
  l.re = re;
  l.im = im;
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

// Wave-wide maximum of (key, value): every lane returns the winner.
template <typename R>
__device__ __forceinline__ Leaf<R> wave_max_leaf(const Leaf<R>& mine) {
  using KO = KeyOps<R>;
  typename KO::Key k = leaf_key(mine);
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) {
    typename KO::Key o = KO::shfl_xor(k, off);
    if (KO::gt(o, k)) k = o;
  }
  const uint64_t own = __ballot(KO::eq(k, leaf_key(mine)));
  const int src = __ffsll((unsigned long long)own) - 1;
  const R re = __shfl(mine.re, src);
  const R im = __shfl(mine.im, src);
  return make_leaf(k, re, im);
}

// Inclusive prefix sum over the wave.
__device__ __forceinline__ int wave_incl_scan(int v, int lane) {
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    int o = __shfl_up(v, off);
    if (lane >= off) v += o;
  }
  return v;
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
// ||x||^2 per signal in FP64 (Alg. 1 initialisation) and state reset.

template <typename XT>
__global__ void __launch_bounds__(256) k_energy(const XT* __restrict__ x, const SigDev* __restrict__ sigs,
                                                SigState* __restrict__ st) {
  __shared__ double part[256];
  const int s = blockIdx.x;
  const int64_t L = sigs[s].L, off = sigs[s].x_off;
  double acc = 0.0;
  for (int64_t i = threadIdx.x; i < L; i += 256) {
    const double v = (double)x[off + i];
    acc += v * v;
  }
  part[threadIdx.x] = acc;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if (threadIdx.x < h) part[threadIdx.x] += part[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    SigState z;
    z.E0 = part[0];
    z.E = part[0];
    z.k = 0;
    z.stop = 0;
    z.pad = 0;
    z.updated = z.blocks = z.groups = 0;
    st[s] = z;
  }
}

// --------------------------------------------------------------------------
// DGT analysis (Sec. 5): for frame n of system w,
//   rho(m, n) = sum_{t=-gl/2}^{gl/2-1} x(n a + t) g(t) exp(-2 pi i m t / M),
// the length-M DFT of the windowed frame laid out circularly (t mod M).
// One workgroup per frame: bit-reversed load into LDS, radix-2 DIT stages,
// bins 0..M/2 written contiguously (m fastest).  The signal is zero beyond L
// and circular over L_padded.

template <typename R, typename XT>
__global__ void __launch_bounds__(256) k_dgt(const XT* __restrict__ x, const SigDev* __restrict__ sigs,
                                             int w, int gl, int a, int M, int logM, int MR,
                                             const int64_t* __restrict__ frame_prefix, int batch,
                                             const R* __restrict__ win, const Cx<R>* __restrict__ tw,
                                             Cx<R>* __restrict__ planes) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  Cx<R>* buf = reinterpret_cast<Cx<R>*>(smem_raw);
  const int64_t f = blockIdx.x;
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
  const int64_t L = S.L, Lp = S.Lp;
  const XT* xs = x + S.x_off;
  for (int i = threadIdx.x; i < M; i += blockDim.x) {
    const int t = i < M / 2 ? i : i - M;
    R v = (R)0;
    if (t >= -gl / 2 && t < gl / 2) {
      int64_t l = (n * a + t) % Lp;
      if (l < 0) l += Lp;
      if (l < L) v = (R)xs[l] * win[t + gl / 2];
    }
    const int r = (int)(__brev((unsigned)i) >> (32 - logM));
    buf[r].re = v;
    buf[r].im = (R)0;
  }
  __syncthreads();
  for (int ls = 1; ls <= logM; ++ls) {
    const int half = 1 << (ls - 1);
    const int tstride = M >> ls;  // twiddle index step
    for (int b = threadIdx.x; b < M / 2; b += blockDim.x) {
      const int grp = b >> (ls - 1);
      const int pos = b & (half - 1);
      const int i0 = (grp << ls) + pos, i1 = i0 + half;
      const Cx<R> wv = tw[pos * tstride];
      const Cx<R> u = buf[i0], q = buf[i1];
      const R tr = q.re * wv.re - q.im * wv.im, ti = q.re * wv.im + q.im * wv.re;
      buf[i0].re = u.re + tr;
      buf[i0].im = u.im + ti;
      buf[i1].re = u.re - tr;
      buf[i1].im = u.im - ti;
    }
    __syncthreads();
  }
  Cx<R>* out = planes + S.coef_base + S.off[w] + n * MR;
  for (int m = threadIdx.x; m < MR; m += blockDim.x) out[m] = buf[m];
}

// --------------------------------------------------------------------------
// Max-tree leaves (Sec. 5.1): one wave per block of BLK coefficients.

template <typename R>
__global__ void __launch_bounds__(256) k_leaves(const Cx<R>* __restrict__ planes, Leaf<R>* __restrict__ leaves,
                                                const SigDev* __restrict__ sigs, int batch, int W,
                                                const DictDev* __restrict__ dicts, int64_t total_blocks) {
  using KO = KeyOps<R>;
  const int lane = threadIdx.x & 63;
  const int64_t b = blockIdx.x * (int64_t)(blockDim.x / 64) + (threadIdx.x >> 6);
  if (b >= total_blocks) return;
  const int64_t e = b * BLK;
  int lo = 0, hi = batch - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (sigs[mid].coef_base <= e) lo = mid;
    else hi = mid - 1;
  }
  const SigDev& S = sigs[lo];
  const int64_t le = e - S.coef_base + lane;  // signal-local index
  int w = 0;
  for (int u = 1; u < W; ++u)
    if (le >= S.off[u]) w = u;
  const int64_t q = le - S.off[w];
  const bool valid = le < S.n_coef_padded && q < (int64_t)S.N[w] * dicts[w].MR;
  Cx<R> v = {(R)0, (R)0};
  typename KO::Key k = KO::empty();
  if (valid) {
    v = planes[e + lane];
    k = KO::make(v.re * v.re + v.im * v.im, (uint32_t)le);
  }
  const Leaf<R> best = wave_max_leaf<R>(make_leaf(k, v.re, v.im));
  if (lane == 0) leaves[b] = best;
}

// --------------------------------------------------------------------------
// The MP loop (Alg. 1 with Eq. approxResDef, the real-atom pairs of Sec. 5
// and the update of Alg. 3).  One persistent workgroup per signal, signals
// taken from a queue (longest first).  Per selection:
//   1. every wave reduces the group maxima kept in LDS -> the global maximum
//      (key, rho(p)) without touching global memory;
//   2. decode p -> (v, k, j); load gamma = <d, conj d>; per target system w
//      the kernel box covers frames n with |n a_w - j a_v| <= dbox a_min and
//      bins m whose mu = m r_w -/+ k r_v falls in the box;
//   3. the covered 64-entry blocks are split over the waves; all their loads
//      (rho, h for the atom, h for its conjugate partner) are issued before
//      the coefficient adjustment (Eq. dualatprod) is computed;
//   4. rho -= c h1 phi + conj(c) h2 conj(phi), phi = exp(2 pi i k Delta / M_v)
//      (Eqs. GramKern, hkj); the block maximum is recomputed in the same
//      pass and written as the new leaf;
//   5. barrier; the touched groups are recomputed from their leaves into LDS;
//      barrier.
// E_k is tracked in FP64 (Eq. projenfaster); every wave keeps an identical
// copy so that the stop decision needs no communication.



template <typename R, int NT, int SLOTS, int GSLOTS>
__device__ void mp_signal(const MPArgs& A, int s, Leaf<R>* l1, int lane, int wave) {
  using KO = KeyOps<R>;
  using Key = typename KO::Key;
  constexpr int NW = NT / 64;
  const SigDev& S = A.sigs[s];
  const int W = A.W;
  const int G = A.G, logG = A.logG;
  const int n_leaves = S.n_leaves, n_groups = S.n_groups;
  Cx<R>* rho = reinterpret_cast<Cx<R>*>(A.planes) + S.coef_base;
  Leaf<R>* leaves = reinterpret_cast<Leaf<R>*>(A.leaves) + S.coef_base / BLK;
  const Cx<R>* tabs = reinterpret_cast<const Cx<R>*>(A.tabs);
  const Cx<R>* gams = reinterpret_cast<const Cx<R>*>(A.gammas);
  const int32_t Lp = (int32_t)S.Lp;

  // ---- group maxima from the leaves ----
  for (int g = wave; g < n_groups; g += NW) {
    Leaf<R> best = make_leaf(KO::empty(), (R)0, (R)0);
    for (int i = lane; i < G; i += 64) {
      const int b = (g << logG) + i;
      if (b < n_leaves) {
        const Leaf<R> c = leaves[b];
        if (KO::gt(leaf_key(c), leaf_key(best))) best = c;
      }
    }
    best = wave_max_leaf<R>(best);
    if (lane == 0) l1[g] = best;
  }
  __syncthreads();

  // per-lane copy of target system `lane` (lanes >= W unused)
  int d_a = 1, d_M = 2, d_MR = 1, d_N = 1;
  int64_t d_off = 0, d_gamoff = 0;
  if (lane < W) {
    const DictDev D = A.dicts[lane];
    d_a = D.a;
    d_M = D.M;
    d_MR = D.MR;
    d_gamoff = D.gamma_off;
    d_N = S.N[lane];
    d_off = S.off[lane];
  }

  SigState st = A.state[s];
  double E = st.E;
  int64_t k = st.k;
  const double E0 = st.E0;
  int64_t K = A.K > 0 ? A.K : S.Lp / 5;
  if (K > S.cap) K = S.cap;
  const double Etarget = A.snr_db > 0.0 ? E0 * exp10(-A.snr_db / 10.0) : -__builtin_huge_val();
  int stop = 0;
  int64_t c_upd = 0, c_blk = 0, c_grp = 0;

  for (;;) {
    if (k >= K) { stop = 1; break; }
    if (E <= Etarget) { stop = 2; break; }
    if (E < 0.0) { stop = 3; break; }

    // 1. global maximum from the group maxima
    Leaf<R> best = make_leaf(KO::empty(), (R)0, (R)0);
    for (int i = lane; i < n_groups; i += 64) {
      const Leaf<R> c = l1[i];
      if (KO::gt(leaf_key(c), leaf_key(best))) best = c;
    }
    best = wave_max_leaf<R>(best);
    const Key bk = leaf_key(best);
    if (!(KO::value(bk) > (R)0)) { stop = 4; break; }
    const int p = uni((int)KO::index(bk));

    // 2. decode p -> (v, kk, j)
    int v = 0;
    for (int u = 1; u < W; ++u)
      if (p >= uni((int)__shfl(d_off, u))) v = u;
    const int v_a = uni(__shfl(d_a, v)), v_M = uni(__shfl(d_M, v)), v_MR = uni(__shfl(d_MR, v));
    const int q = p - uni((int)__shfl(d_off, v));
    const int j = q / v_MR;
    const int kk = q - j * v_MR;
    const bool pair = kk != 0 && 2 * kk != v_M;
    Cx<R> gam = {(R)0, (R)0};
    if (pair) gam = gams[__shfl(d_gamoff, v) + kk];  // overlaps with the block loads below

    // per-target geometry, lane t < W handles target t
    int t_nlo = 0, t_nF = 0, t_mlo = 0, t_mhi = -1;
    int t_amin = 1, t_Mmax = 2, t_rw = 1, t_rv = 1, t_dbox = -1, t_mulo = 0, t_muhi = -1, t_width = 0;
    int64_t t_tab = 0;
    if (lane < W) {
      const PairDev P = A.pairs[lane * W + v];
      t_amin = P.amin; t_Mmax = P.Mmax; t_rw = P.rw; t_rv = P.rv;
      t_dbox = P.dbox; t_mulo = P.mu_lo; t_muhi = P.mu_hi; t_width = P.width; t_tab = P.tab_off;
      if (P.dbox >= 0) {
        const int64_t jav = (int64_t)j * v_a, span = (int64_t)P.dbox * P.amin;
        const int64_t nlo = ceil_div(jav - span, d_a), nhi = floor_div(jav + span, d_a);
        // bins whose mu = m rw -/+ k rv lies in [mu_lo, mu_hi] modulo M_max
        const int kr = kk * P.rv;
        const int half = d_M / 2;
        int mlo = 1 << 30, mhi = -1;
        for (int term = 0; term < 2; ++term) {
          if (term == 1 && !pair) break;
          const int base = term == 0 ? kr : -kr;  // m rw in base + [mu_lo, mu_hi]
          const int A1 = (int)ceil_div(base + P.mu_lo, P.rw), B1 = (int)floor_div(base + P.mu_hi, P.rw);
          if (B1 - A1 + 1 >= d_M) {
            mlo = 0;
            mhi = half;
          } else {
            for (int c = -1; c <= 1; ++c) {
              const int lo = max(A1 + c * d_M, 0), hi = min(B1 + c * d_M, half);
              if (lo <= hi) {
                mlo = min(mlo, lo);
                mhi = max(mhi, hi);
              }
            }
          }
        }
        if (mhi >= 0 && nhi >= nlo) {
          t_nlo = (int)(((nlo % d_N) + d_N) % d_N);
          t_nF = (int)(nhi - nlo + 1);
          t_mlo = mlo;
          t_mhi = mhi;
        }
      }
    }
    // exclusive prefix of frame counts over targets
    const int t_cum = wave_incl_scan(lane < W ? t_nF : 0, lane) - (lane < W ? t_nF : 0);
    const int S_tot = uni(__shfl(t_cum, W - 1) + __shfl(t_nF, W - 1));

    // 3. resolve this wave's blocks (slots) and groups from the segment list:
    //    segment = (target w, frame n) with bins [mlo, mhi]; blocks of
    //    consecutive frames are de-duplicated, the wrapped run is clipped
    //    below the first run.
    int blk[SLOTS], bw[SLOTS], grp[GSLOTS];
#pragma unroll
    for (int i = 0; i < SLOTS; ++i) blk[i] = -1, bw[i] = 0;
#pragma unroll
    for (int i = 0; i < GSLOTS; ++i) grp[i] = -1;
    int totB = 0, totG = 0;
    auto resolve = [&](int roundB, int roundG) {
      int baseB = 0, baseG = 0;
      for (int c0 = 0; c0 < S_tot; c0 += 64) {
        // every lane takes part in the shuffles below; lanes past the end
        // compute a dummy segment and contribute no blocks
        const int sg = min(c0 + lane, S_tot - 1);
        int cnt = 0, cntg = 0, bl = 0, gl = 0, ws = 0;
        {
          for (int u = 1; u < W; ++u) {
            const int cu = __shfl(t_cum, u), nu = __shfl(t_nF, u);
            if (sg >= cu && nu > 0) ws = u;
          }
          // fields of target ws
          const int s_nlo = __shfl(t_nlo, ws), s_cum = __shfl(t_cum, ws);
          const int s_N = __shfl(d_N, ws), s_MR = __shfl(d_MR, ws);
          const int s_mlo = __shfl(t_mlo, ws), s_mhi = __shfl(t_mhi, ws);
          const int64_t s_off = __shfl(d_off, ws);
          const int f = sg - s_cum;
          int n = s_nlo + f;
          if (n >= s_N) n -= s_N;
          if (n >= s_N) n %= s_N;
          const int64_t rowb = s_off + (int64_t)n * s_MR;
          bl = (int)((rowb + s_mlo) >> 6);
          int bh = (int)((rowb + s_mhi) >> 6);
          gl = bl >> logG;
          if (f > 0 && n > 0 && n != s_nlo) {
            // predecessor frame n-1 is adjacent in memory
            const int pbh = (int)((s_off + (int64_t)(n - 1) * s_MR + s_mhi) >> 6);
            if (bl <= pbh) bl = pbh + 1;
            gl = bl >> logG;
            if (gl == (pbh >> logG)) ++gl;
          }
          if (f > 0 && n < s_nlo) {
            const int fbl = (int)((s_off + (int64_t)s_nlo * s_MR + s_mlo) >> 6);
            if (bh >= fbl) bh = fbl - 1;
          }
          cnt = bh >= bl ? bh - bl + 1 : 0;
          const int gh = bh >> logG;
          cntg = (cnt > 0 && gh >= gl) ? gh - gl + 1 : 0;
          if (c0 + lane >= S_tot) cnt = cntg = 0;
        }
        const int incB = wave_incl_scan(cnt, lane);
        const int incG = wave_incl_scan(cntg, lane);
        const int chB = __shfl(incB, 63), chG = __shfl(incG, 63);
#pragma unroll
        for (int i = 0; i < SLOTS; ++i) {
          const int it = wave + NW * (i + SLOTS * roundB) - baseB;
          if (it >= 0 && it < chB) {
            const uint64_t bal = __ballot(incB > it);
            const int src = __ffsll((unsigned long long)bal) - 1;
            blk[i] = uni(__shfl(bl, src) + it - (__shfl(incB, src) - __shfl(cnt, src)));
            bw[i] = uni(__shfl(ws, src));
          }
        }
#pragma unroll
        for (int i = 0; i < GSLOTS; ++i) {
          const int it = wave + NW * (i + GSLOTS * roundG) - baseG;
          if (it >= 0 && it < chG) {
            const uint64_t bal = __ballot(incG > it);
            const int src = __ffsll((unsigned long long)bal) - 1;
            grp[i] = uni(__shfl(gl, src) + it - (__shfl(incG, src) - __shfl(cntg, src)));
          }
        }
        baseB += chB;
        baseG += chG;
      }
      totB = baseB;
      totG = baseG;
    };
    resolve(0, 0);

    // 4. update the covered blocks, rescan them, write the leaves
    Cx<R> cc = {(R)0, (R)0};
    bool partner = false;
    for (int roundB = 0;; ++roundB) {
      if (roundB > 0) {
        if (wave + NW * SLOTS * roundB >= totB) break;
#pragma unroll
        for (int i = 0; i < SLOTS; ++i) blk[i] = -1;
        resolve(roundB, 1 << 20);
      }
      Cx<R> r[SLOTS], h1[SLOTS], h2[SLOTS];
      int ph[SLOTS], le[SLOTS];
      bool valid[SLOTS];
#pragma unroll
      for (int i = 0; i < SLOTS; ++i) {
        r[i] = h1[i] = h2[i] = Cx<R>{(R)0, (R)0};
        ph[i] = 0;
        valid[i] = false;
        le[i] = 0;
        if (blk[i] < 0) continue;
        const int w = bw[i];
        const int w_a = uni(__shfl(d_a, w)), w_MR = uni(__shfl(d_MR, w)), w_N = uni(__shfl(d_N, w));
        const int w_off = uni((int)__shfl(d_off, w));
        const int amin = uni(__shfl(t_amin, w)), Mmax = uni(__shfl(t_Mmax, w));
        const int rw = uni(__shfl(t_rw, w)), rv = uni(__shfl(t_rv, w));
        const int dbox = uni(__shfl(t_dbox, w)), mulo = uni(__shfl(t_mulo, w)), muhi = uni(__shfl(t_muhi, w));
        const int width = uni(__shfl(t_width, w));
        const int64_t tab = __shfl(t_tab, w);
        const int e = blk[i] * BLK + lane;
        le[i] = e;
        const int qq = e - w_off;
        valid[i] = qq < w_N * w_MR;
        if (!valid[i]) continue;
        r[i] = rho[e];
        const int n = qq / w_MR, m = qq - n * w_MR;
        const int Delta = cmod(n * w_a - j * v_a, Lp);
        const int span = dbox * amin;
        if (Delta > span || Delta < -span) continue;
        const int row = Delta / amin + dbox;
        const int mu1 = cmod(m * rw - kk * rv, Mmax);
        if (mu1 >= mulo && mu1 <= muhi) h1[i] = tabs[tab + (int64_t)row * width + (mu1 - mulo)];
        if (pair) {
          const int mu2 = cmod(m * rw + kk * rv, Mmax);
          if (mu2 >= mulo && mu2 <= muhi) h2[i] = tabs[tab + (int64_t)row * width + (mu2 - mulo)];
        }
        ph[i] = (int)(((int64_t)kk * mod_pos(Delta, v_M)) % v_M);
      }
      if (roundB == 0) {
        // coefficient adjustment for the pair, Eq. (dualatprod), and energy
        // decrease, Eq. (projenfaster); placed after the loads above so that
        // the gamma load overlaps with them.
        const R rr = best.re, ri = best.im;
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
      for (int i = 0; i < SLOTS; ++i) {
        if (blk[i] < 0) continue;
        if (!partner) h2[i] = Cx<R>{(R)0, (R)0};
        const bool ch = (h1[i].re != (R)0) | (h1[i].im != (R)0) | (h2[i].re != (R)0) | (h2[i].im != (R)0);
        if (ch) {
          R sn, cs;
          sincospi_<R>((R)2 * (R)ph[i] / (R)v_M, &sn, &cs);
          // c * (h1 phi) + conj(c) * (h2 conj(phi))
          const R ar = h1[i].re * cs - h1[i].im * sn, ai = h1[i].re * sn + h1[i].im * cs;
          R ur = cc.re * ar - cc.im * ai, ui = cc.re * ai + cc.im * ar;
          const R br = h2[i].re * cs + h2[i].im * sn, bi = h2[i].im * cs - h2[i].re * sn;
          ur += cc.re * br + cc.im * bi;
          ui += cc.re * bi - cc.im * br;
          r[i].re -= ur;
          r[i].im -= ui;
          rho[le[i]] = r[i];
        }
        Key key = valid[i] ? KO::make(r[i].re * r[i].re + r[i].im * r[i].im, (uint32_t)le[i]) : KO::empty();
        const Leaf<R> bl = wave_max_leaf<R>(make_leaf(key, r[i].re, r[i].im));
        const int nch = __popcll(__ballot(ch));
        if (lane == 0) {
          leaves[blk[i]] = bl;
          c_upd += nch;
          ++c_blk;
        }
      }
      if (wave + NW * SLOTS * (roundB + 1) >= totB) break;
    }
    __syncthreads();

    // 5. recompute the touched groups
    for (int roundG = 0;; ++roundG) {
      if (roundG > 0) {
        if (wave + NW * GSLOTS * roundG >= totG) break;
#pragma unroll
        for (int i = 0; i < GSLOTS; ++i) grp[i] = -1;
        resolve(1 << 20, roundG);
      }
#pragma unroll
      for (int i = 0; i < GSLOTS; ++i) {
        if (grp[i] < 0) continue;
        const int g = grp[i];
        Leaf<R> gb = make_leaf(KO::empty(), (R)0, (R)0);
        for (int t = lane; t < G; t += 64) {
          const int b = (g << logG) + t;
          if (b < n_leaves) {
            const Leaf<R> c = leaves[b];
            if (KO::gt(leaf_key(c), leaf_key(gb))) gb = c;
          }
        }
        gb = wave_max_leaf<R>(gb);
        if (lane == 0) {
          l1[g] = gb;
          ++c_grp;
        }
      }
      if (wave + NW * GSLOTS * (roundG + 1) >= totG) break;
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

template <typename R, int NT, int SLOTS, int GSLOTS>
__global__ void __launch_bounds__(NT) k_mp(MPArgs A) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  Leaf<R>* l1 = reinterpret_cast<Leaf<R>*>(smem_raw);
  __shared__ int s_next;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (;;) {
    if (threadIdx.x == 0) s_next = atomicAdd(A.queue, 1);
    __syncthreads();
    const int qi = s_next;
    __syncthreads();
    if (qi >= A.batch) break;
    mp_signal<R, NT, SLOTS, GSLOTS>(A, A.order[qi], l1, lane, wave);
  }
}

__global__ void k_fill_i32(int32_t* p, int n, int v) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

// --------------------------------------------------------------------------
// Synthesis of real atoms (Eq. idgtreal).  One workgroup; thread t owns the
// samples l with l mod blockDim.x == t, so atoms are added in selection order
// without atomics.  Accumulation in FP64.

__global__ void __launch_bounds__(1024) k_resynth(const AtomRec* __restrict__ atoms, const SigState* __restrict__ st,
                                                  const DictDev* __restrict__ dicts,
                                                  const double* __restrict__ win64, int64_t Lp,
                                                  double* __restrict__ acc) {
  const int64_t T = blockDim.x, tid = threadIdx.x;
  const int64_t n_atoms = st->k;
  for (int64_t l = tid; l < Lp; l += T) acc[l] = 0.0;
  for (int64_t i = 0; i < n_atoms; ++i) {
    const AtomRec at = atoms[i];
    const DictDev D = dicts[at.w];
    const double mult = (at.m != 0 && 2 * at.m != D.M) ? 2.0 : 1.0;
    const double* g = win64 + D.win_off;
    // sample of t = -gl/2 (tp = 0), wrapped into [0, Lp)
    int64_t s0 = ((int64_t)at.n * D.a - D.gl / 2) % Lp;
    if (s0 < 0) s0 += Lp;
    const int64_t split = D.gl < Lp - s0 ? D.gl : Lp - s0;
    int64_t t0 = (tid - s0) % T;
    if (t0 < 0) t0 += T;
    // tp < split: l = s0 + tp; tp >= split: l = s0 + tp - Lp
    for (int64_t tp = t0; tp < split; tp += T) {
      const int64_t t = tp - D.gl / 2;
      int64_t pi = ((int64_t)at.m * t) % D.M;
      if (pi < 0) pi += D.M;
      double sn, cs;
      sincospi(2.0 * (double)pi / (double)D.M, &sn, &cs);
      acc[s0 + tp] += mult * g[tp] * (at.re * cs - at.im * sn);
    }
    for (int64_t l = tid; l < D.gl - split; l += T) {
      const int64_t tp = l + Lp - s0;
      const int64_t t = tp - D.gl / 2;
      int64_t pi = ((int64_t)at.m * t) % D.M;
      if (pi < 0) pi += D.M;
      double sn, cs;
      sincospi(2.0 * (double)pi / (double)D.M, &sn, &cs);
      acc[l] += mult * g[tp] * (at.re * cs - at.im * sn);
    }
  }
}

template <typename YT>
__global__ void k_store_y(const double* __restrict__ acc, int64_t n, YT* __restrict__ y) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n) y[i] = (YT)acc[i];
}

// Solution vector (Alg. 1 solution update): c(m, n) = sum of c~ of the atoms
// selected at (w, m, n).  One workgroup; thread t owns entries idx mod T.
__global__ void __launch_bounds__(1024) k_coefs(const AtomRec* __restrict__ atoms, const SigState* __restrict__ st,
                                                int w, int MR, int64_t n_entries, double2* __restrict__ c) {
  const int T = blockDim.x, tid = threadIdx.x;
  const int64_t n_atoms = st->k;
  for (int64_t i = tid; i < n_entries; i += T) c[i] = make_double2(0.0, 0.0);
  for (int64_t i = 0; i < n_atoms; ++i) {
    const AtomRec at = atoms[i];
    if (at.w != w) continue;
    const int64_t idx = (int64_t)at.n * MR + at.m;
    if (idx % T != tid) continue;
    double2 v = c[idx];
    v.x += at.re;
    v.y += at.im;
    c[idx] = v;
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

hipError_t launch_energy(const void* x, int dtype, const SigDev* sigs, int batch, SigState* st_,
                         hipStream_t st) {
  if (dtype == 0)
    k_energy<float><<<batch, 256, 0, st>>>((const float*)x, sigs, st_);
  else
    k_energy<double><<<batch, 256, 0, st>>>((const double*)x, sigs, st_);
  return hipGetLastError();
}

hipError_t launch_dgt(bool f64, const void* x, int dtype, const SigDev* sigs, int w, int gl, int a,
                      int M, int MR, const int64_t* frame_prefix, int batch, int64_t frames,
                      const void* win, const void* tw, void* planes, hipStream_t st) {
  if (frames <= 0) return hipSuccess;
  int logM = 0;
  while ((1 << logM) < M) ++logM;
  const size_t sh = (size_t)M * (f64 ? 16 : 8);
  const dim3 grid((unsigned)frames);
  if (f64) {
    if (dtype == 0)
      k_dgt<double, float><<<grid, 256, sh, st>>>((const float*)x, sigs, w, gl, a, M, logM, MR, frame_prefix,
                                                  batch, (const double*)win, (const Cx<double>*)tw,
                                                  (Cx<double>*)planes);
    else
      k_dgt<double, double><<<grid, 256, sh, st>>>((const double*)x, sigs, w, gl, a, M, logM, MR, frame_prefix,
                                                   batch, (const double*)win, (const Cx<double>*)tw,
                                                   (Cx<double>*)planes);
  } else {
    if (dtype == 0)
      k_dgt<float, float><<<grid, 256, sh, st>>>((const float*)x, sigs, w, gl, a, M, logM, MR, frame_prefix,
                                                 batch, (const float*)win, (const Cx<float>*)tw,
                                                 (Cx<float>*)planes);
    else
      k_dgt<float, double><<<grid, 256, sh, st>>>((const double*)x, sigs, w, gl, a, M, logM, MR, frame_prefix,
                                                  batch, (const float*)win, (const Cx<float>*)tw,
                                                  (Cx<float>*)planes);
  }
  return hipGetLastError();
}

hipError_t launch_leaves(bool f64, const void* planes, void* leaves, const SigDev* sigs, int batch, int W,
                         const DictDev* dicts, int64_t total_blocks, hipStream_t st) {
  if (total_blocks <= 0) return hipSuccess;
  const unsigned grid = (unsigned)((total_blocks + 3) / 4);
  if (f64)
    k_leaves<double><<<grid, 256, 0, st>>>((const Cx<double>*)planes, (Leaf<double>*)leaves, sigs, batch, W,
                                           dicts, total_blocks);
  else
    k_leaves<float><<<grid, 256, 0, st>>>((const Cx<float>*)planes, (Leaf<float>*)leaves, sigs, batch, W,
                                          dicts, total_blocks);
  return hipGetLastError();
}

size_t leaf_bytes(bool f64) { return f64 ? sizeof(Leaf<double>) : sizeof(Leaf<float>); }

hipError_t launch_mp(bool f64, int nt, const MPArgs& a, int grid, size_t shmem, hipStream_t st) {
  k_fill_i32<<<1, 64, 0, st>>>(a.queue, 1, 0);
  CHK(hipGetLastError());
  if (f64) {
    if (nt == 256) {
      (void)hipFuncSetAttribute((const void*)k_mp<double, 256, 4, 2>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)shmem);
      k_mp<double, 256, 4, 2><<<grid, 256, shmem, st>>>(a);
    } else {
      (void)hipFuncSetAttribute((const void*)k_mp<double, 512, 4, 1>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)shmem);
      k_mp<double, 512, 4, 1><<<grid, 512, shmem, st>>>(a);
    }
  } else {
    if (nt == 256) {
      (void)hipFuncSetAttribute((const void*)k_mp<float, 256, 4, 2>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)shmem);
      k_mp<float, 256, 4, 2><<<grid, 256, shmem, st>>>(a);
    } else if (nt == 512) {
      (void)hipFuncSetAttribute((const void*)k_mp<float, 512, 4, 1>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)shmem);
      k_mp<float, 512, 4, 1><<<grid, 512, shmem, st>>>(a);
    } else {
      (void)hipFuncSetAttribute((const void*)k_mp<float, 1024, 2, 1>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)shmem);
      k_mp<float, 1024, 2, 1><<<grid, 1024, shmem, st>>>(a);
    }
  }
  return hipGetLastError();
}

hipError_t launch_resynth(const AtomRec* atoms, const SigState* st_, const DictDev* dicts, const double* win64,
                          int64_t Lp, double* acc, void* y, int dtype, hipStream_t st) {
  k_resynth<<<1, 1024, 0, st>>>(atoms, st_, dicts, win64, Lp, acc);
  CHK(hipGetLastError());
  const unsigned g = (unsigned)((Lp + 255) / 256);
  if (dtype == 0)
    k_store_y<float><<<g, 256, 0, st>>>(acc, Lp, (float*)y);
  else
    k_store_y<double><<<g, 256, 0, st>>>(acc, Lp, (double*)y);
  return hipGetLastError();
}

hipError_t launch_coefs(const AtomRec* atoms, const SigState* st_, int w, int MR, int64_t n_entries, void* c,
                        hipStream_t st) {
  k_coefs<<<1, 1024, 0, st>>>(atoms, st_, w, MR, n_entries, (double2*)c);
  return hipGetLastError();
}

}  // namespace mpg
