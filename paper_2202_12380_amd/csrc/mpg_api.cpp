// Host side of libmpg: plan validation and layout, FP64 kernel precompute
// driver, and the C-ABI entry points declared in include/mpg.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <new>
#include <numeric>
#include <vector>

#include "mpg.h"
#include "mpg_internal.h"

namespace mpg {

hipError_t launch_roots(int M, int n, int sign, double2* o64, float2* o32, hipStream_t st);
hipError_t launch_stage_tw(int M, double2* t64, float2* t32, hipStream_t st);
hipError_t launch_gram_full(const double* gw, int glw, const double* gv, int glv, int amin, int D,
                            int Mmax, const double2* roots, double2* out, hipStream_t st);
hipError_t launch_gram_absmax(const double2* t, int64_t n, unsigned long long* out, hipStream_t st);
hipError_t launch_gram_box(const double2* t, int D, int Mmax, double thr, int* box, hipStream_t st);
hipError_t launch_gram_extract(const double2* t, int D, int Mmax, double thr, int dbox, int mu_lo,
                               int width, double2* o64, float2* o32, hipStream_t st);
hipError_t launch_energy(const void* x, int dtype, const SigDev* sigs, int batch, double* part, SigState* st_,
                         hipStream_t st);
hipError_t launch_reset_init(const void* x, int dtype, const SigDev* sigs, int batch, int64_t max_Lp,
                             const int64_t* roff, double* r, hipStream_t st);
hipError_t launch_reset_update(const AtomRec* atoms, const SigDev* sigs, SigState* st_, const DictDev* dicts,
                               const double* win64, const int64_t* roff, double* r, int batch, double snr_db,
                               int64_t K_total, int* active, hipStream_t st);
hipError_t launch_dft_tables(int fmt, int N, int Np, uint16_t* out, hipStream_t st);
hipError_t launch_dgt_mfma(int fmt, const void* x, int dtype, const SigDev* sigs, int w, int gl, int a, int M,
                           int MR, const int64_t* frame_prefix, int batch, int64_t frames, const float* win,
                           const void* tw, int N1, int N2, const uint16_t* F1, const uint16_t* F2, void* planes,
                           void* leaves, const void* gam, int pedantic, int64_t max_Lp, hipStream_t st);
hipError_t launch_dgt(bool f64, bool dft64, const void* x, int dtype, const SigDev* sigs, int w, int gl, int a,
                      int M, int MR, const int64_t* frame_prefix, int batch, int64_t frames,
                      const void* win, const void* tw, void* planes, void* leaves, const void* gam, int pedantic,
                      const double2* roots64, hipStream_t st);
size_t leaf_bytes(bool f64);
size_t mp_shmem_bytes(bool f64, int nt, int G, int n_groups_max);
hipError_t launch_mp(bool f64, int nt, const MPArgs& a, int grid, hipStream_t st);
hipError_t launch_resynth(const AtomRec* atoms, const SigState* st_, const DictDev* dicts,
                          const double* win64, int64_t Lp, double* acc, void* y, int dtype,
                          hipStream_t st);
hipError_t launch_coefs(const AtomRec* atoms, const SigState* st_, int w, int MR, int64_t n_entries,
                        void* c, hipStream_t st);
hipError_t static_scratch(double** out, int64_t* n_out);
}  // namespace mpg

using namespace mpg;

struct mp_plan {
  int device = 0;
  int W = 0, batch = 0;
  uint32_t flags = 0;
  double eps = 0.0;
  bool f64 = false;
  int dft_fmt = -1;  // -1: FP32/FP64 FFT, 0: FP16 pairs on MFMA, 1: BF16 pairs
  std::vector<int> dft_n1, dft_n2;
  std::vector<uint16_t*> d_dft1, d_dft2;
  // reset procedure: FP64 residuals (stride L_padded), their offsets and a
  // copy of the signal table that reads them over the padded length
  double* d_res = nullptr;
  int64_t* d_roff = nullptr;
  SigDev* d_sigs_res = nullptr;
  int* d_active = nullptr;
  std::vector<mp_dict> dicts;
  std::vector<DictDev> hd;
  std::vector<PairDev> hp;
  std::vector<SigDev> hs;
  std::vector<mp_kernel_info> kinfo;
  std::vector<std::vector<double>> kre, kim;
  std::vector<int32_t> order;
  std::vector<int64_t> frames_total;  // per system, over the batch
  int G = 64, logG = 6, n_groups_max = 0;
  int64_t tg_bound = 0;  // bound on the tree groups one selection touches
  int nt = 512, grid = 1;
  size_t shmem = 0;
  int64_t total_coef = 0, total_leaves = 0, total_cap = 0, max_Lp = 0;
  bool analyzed = false;
  hipStream_t last_stream = nullptr;
  int64_t last_K = 0;

  // device memory
  DictDev* d_dicts = nullptr;
  PairDev* d_pairs = nullptr;
  SigDev* d_sigs = nullptr;
  SigState* d_state = nullptr;
  double* d_epart = nullptr;  // ENERGY_PARTS partial sums of ||x||^2 per signal
  double* d_win64 = nullptr;
  float* d_win32 = nullptr;
  double2* d_tw64 = nullptr;
  float2* d_tw32 = nullptr;
  double2* d_tab64 = nullptr;
  float2* d_tab32 = nullptr;
  double2* d_gam64 = nullptr;
  float2* d_gam32 = nullptr;
  double2* d_root64 = nullptr;
  float2* d_root32 = nullptr;
  void* d_planes = nullptr;
  void* d_leaves = nullptr;
  AtomRec* d_atoms = nullptr;
  int32_t* d_order = nullptr;
  int32_t* d_queue = nullptr;
  int64_t* d_fprefix[MAXW] = {};
  double* d_acc = nullptr;
  hipEvent_t ev[6] = {};
  bool ev_valid = false;
  bool ran = false;
};

namespace {

bool is_pow2(int64_t v) { return v > 0 && (v & (v - 1)) == 0; }

// The stream is being captured into a HIP graph: mp_analyze and mp_run then
// enqueue kernels only (no timing events), and nothing may allocate.
bool capturing(hipStream_t s) {
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  return hipStreamIsCapturing(s, &cs) == hipSuccess && cs != hipStreamCaptureStatusNone;
}

int64_t gcd64(int64_t a, int64_t b) {
  while (b) {
    int64_t t = a % b;
    a = b;
    b = t;
  }
  return a;
}

// Magic pair for q / d with 0 <= q < 2^31: q / d == (umulhi(q, m) + q) >> s.
void magic_u32(uint32_t d, uint32_t* m, int32_t* s) {
  int sh = 0;
  while ((1ull << sh) < d) ++sh;
  *m = (uint32_t)((((uint64_t)1 << 32) * (((uint64_t)1 << sh) - d)) / d + 1);
  *s = sh;
}

template <typename T>
hipError_t dalloc(T** p, size_t n) {
  *p = nullptr;
  if (n == 0) n = 1;
  return hipMalloc((void**)p, n * sizeof(T));
}

// Centred periodic window on t = -gl/2 .. gl/2-1, unit 2-norm (Sec. 2.1).
// Gaussian (the width is a reading; the paper's kernel figure names the window
// only): exp(-pi t^2 / (a M)), time and frequency spreads matched to the lattice.
void make_window(int type, int gl, int a, int M, std::vector<double>& g) {
  g.resize(gl);
  const double pi = 3.14159265358979323846;
  double e = 0.0;
  for (int i = 0; i < gl; ++i) {
    const double t = (double)(i - gl / 2);
    double v;
    if (type == MP_WIN_BLACKMAN)
      v = 0.42 + 0.5 * std::cos(2.0 * pi * t / gl) + 0.08 * std::cos(4.0 * pi * t / gl);
    else if (type == MP_WIN_HANN)
      v = 0.5 + 0.5 * std::cos(2.0 * pi * t / gl);
    else
      v = std::exp(-pi * t * t / ((double)a * (double)M));
    g[i] = v;
    e += v * v;
  }
  const double s = 1.0 / std::sqrt(e);
  for (auto& v : g) v *= s;
}

void dfree(void* q) { (void)hipFree(q); }

void free_plan(mp_plan* p) {
  if (!p) return;
  dfree(p->d_dicts);
  dfree(p->d_pairs);
  dfree(p->d_sigs);
  dfree(p->d_state);
  dfree(p->d_epart);
  dfree(p->d_win64);
  dfree(p->d_win32);
  dfree(p->d_tw64);
  dfree(p->d_tw32);
  dfree(p->d_tab64);
  dfree(p->d_tab32);
  dfree(p->d_gam64);
  dfree(p->d_gam32);
  dfree(p->d_root64);
  dfree(p->d_root32);
  dfree(p->d_planes);
  dfree(p->d_leaves);
  dfree(p->d_atoms);
  dfree(p->d_order);
  dfree(p->d_queue);
  for (auto& f : p->d_fprefix) dfree(f);
  dfree(p->d_acc);
  dfree(p->d_res);
  dfree(p->d_roff);
  dfree(p->d_sigs_res);
  dfree(p->d_active);
  for (auto t : p->d_dft1) dfree(t);
  for (auto t : p->d_dft2) dfree(t);
  if (p->ev_valid)
    for (auto& e : p->ev) (void)hipEventDestroy(e);
  delete p;
}

int check_dicts(const mp_dict* d, int W) {
  for (int w = 0; w < W; ++w) {
    if (d[w].window != MP_WIN_BLACKMAN && d[w].window != MP_WIN_HANN && d[w].window != MP_WIN_GAUSS)
      return MP_E_ARG;
    if (d[w].gl <= 0 || d[w].a <= 0 || d[w].M <= 0) return MP_E_ARG;
    if (d[w].M < 2 || (d[w].M & 1)) return MP_E_GRID;  // even M: bins 0 .. M/2, Nyquist included
    if ((d[w].gl & 1) || (int64_t)d[w].gl > 8 * (int64_t)d[w].M) return MP_E_GRID;  // longer than M: folded
    // a periodic Blackman or Hann window of length 2 has one nonzero sample:
    // every atom is real, so a pair's d and conj d coincide and the pair
    // adjustment (Eq. dualatprod) divides by 1 - |gamma|^2 = 0
    if (d[w].gl == 2 && d[w].window != MP_WIN_GAUSS && d[w].M >= 4) return MP_E_ARG;
  }
  // neither the hops nor the numbers of channels need divide each other:
  // each pair lives on the common grid gcd(a_w, a_v) x lcm(M_w, M_v) (Sec. 4.2)
  return MP_OK;
}

#define HCHK(x)                 \
  do {                          \
    if ((x) != hipSuccess) {    \
      rc = MP_E_HIP;            \
      goto fail;                \
    }                           \
  } while (0)

#define ACHK(x)                                            \
  do {                                                     \
    hipError_t e_ = (x);                                   \
    if (e_ != hipSuccess) {                                \
      rc = e_ == hipErrorOutOfMemory ? MP_E_NOMEM : MP_E_HIP; \
      goto fail;                                           \
    }                                                      \
  } while (0)

// Grows the atom logs so that every signal can hold `need` atoms, keeping
// what is already logged.
int ensure_cap(mp_plan* p, int64_t K, hipStream_t st) {
  std::vector<int64_t> caps(p->batch);
  bool grow = false;
  for (int s = 0; s < p->batch; ++s) {
    const int64_t want = K > 0 ? K : std::max<int64_t>(p->hs[s].Lp / 5, 1);
    caps[s] = std::max(p->hs[s].cap, want);
    if (caps[s] != p->hs[s].cap) grow = true;
  }
  if (!grow) return MP_OK;
  int64_t total = 0;
  for (auto c : caps) total += c;
  AtomRec* na = nullptr;
  if (hipMalloc((void**)&na, sizeof(AtomRec) * (size_t)total) != hipSuccess) return MP_E_NOMEM;
  if (hipStreamSynchronize(st) != hipSuccess) {
    dfree(na);
    return MP_E_HIP;
  }
  int64_t base = 0;
  std::vector<SigDev> ns = p->hs;
  for (int s = 0; s < p->batch; ++s) {
    if (p->hs[s].cap > 0 &&
        hipMemcpy(na + base, p->d_atoms + p->hs[s].atom_base, sizeof(AtomRec) * (size_t)p->hs[s].cap,
                  hipMemcpyDeviceToDevice) != hipSuccess) {
      dfree(na);
      return MP_E_HIP;
    }
    ns[s].atom_base = base;
    ns[s].cap = caps[s];
    base += caps[s];
  }
  if (hipMemcpy(p->d_sigs, ns.data(), sizeof(SigDev) * ns.size(), hipMemcpyHostToDevice) != hipSuccess) {
    dfree(na);
    return MP_E_HIP;
  }
  dfree(p->d_atoms);
  p->d_atoms = na;
  p->hs = ns;
  p->total_cap = total;
  return MP_OK;
}

}  // namespace

extern "C" {

const char* mp_strerror(int code) {
  switch (code) {
    case MP_OK: return "ok";
    case MP_E_ARG: return "invalid argument";
    case MP_E_GRID: return "unsupported Gabor system (M odd, gl odd or gl > 8 M; split DFT with M not a power of two)";
    case MP_E_LEN: return "signal length too short for the kernels (padded L < gl_v + gl_w)";
    case MP_E_NOMEM: return "out of memory";
    case MP_E_HIP: return "HIP runtime error";
    case MP_E_STATE: return "call out of order";
    case MP_E_LIMIT: return "size exceeds an implementation limit";
    default: return "unknown error";
  }
}

int mp_plan_create(const mp_dict* dicts, int32_t W, const int64_t* L, int32_t batch, double kernel_tol,
                   uint32_t flags, mp_plan** out) {
  if (!out) return MP_E_ARG;
  *out = nullptr;
  if (!dicts || !L || W < 1 || W > MAXW || batch < 1 || batch > (1 << 20)) return MP_E_ARG;
  if (!(kernel_tol >= 0.0 && kernel_tol < 1.0)) return MP_E_ARG;
  constexpr uint32_t SCHED = MP_SCHED_NT512 | MP_SCHED_G128 | MP_SCHED_TILE8 | MP_SCHED_TILE32;
  if (flags & ~(MP_PREC_F64 | MP_THR_REL | MP_CONJ_GATE_GAMMA | MP_DFT_F16SPLIT | MP_DFT_BF16SPLIT | MP_DFT_F64 |
                MP_PEDANTIC | SCHED))
    return MP_E_ARG;
  if ((flags & MP_SCHED_TILE8) && (flags & MP_SCHED_TILE32)) return MP_E_ARG;
  if ((flags & MP_SCHED_TILE32) && !(flags & MP_SCHED_NT512)) return MP_E_ARG;  // 4 slots fit 512 threads only
  const uint32_t dftf = flags & (MP_DFT_F16SPLIT | MP_DFT_BF16SPLIT);
  const uint32_t dfts = flags & (MP_DFT_F16SPLIT | MP_DFT_BF16SPLIT | MP_DFT_F64);
  if ((dfts & (dfts - 1)) || (dfts && (flags & MP_PREC_F64))) return MP_E_ARG;  // at most one, FP32 plans only
  if ((flags & MP_PREC_F64) && (flags & SCHED)) return MP_E_ARG;
  int rc = check_dicts(dicts, W);
  if (rc) return rc;
  // the split DFT is a four-step transform over powers of two
  for (int w = 0; w < W; ++w)
    if (dftf && !is_pow2(dicts[w].M)) return MP_E_GRID;
  for (int s = 0; s < batch; ++s)
    if (L[s] <= 0) return MP_E_ARG;
  // the DGT keeps one frame's half-length FFT in LDS
  for (int w = 0; w < W; ++w)
    if ((size_t)(dicts[w].M / 2 + (dftf ? dicts[w].M / 2 : dicts[w].M / 64)) *
            ((flags & (MP_PREC_F64 | MP_DFT_F64)) ? 16 : 8) >
        160 * 1024)
      return MP_E_LIMIT;
  {
    // padded lengths must fit every pair's kernel (checked before any HIP call)
    int64_t q = 1, need = 0;
    for (int w = 0; w < W; ++w) {
      q = q / gcd64(q, dicts[w].a) * dicts[w].a;
      q = q / gcd64(q, dicts[w].M) * dicts[w].M;
      for (int v = 0; v < W; ++v) need = std::max<int64_t>(need, dicts[w].gl + dicts[v].gl);
    }
    for (int s = 0; s < batch; ++s) {
      const int64_t Lp = (L[s] + q - 1) / q * q;
      if (Lp < need) return MP_E_LEN;
      if (Lp >= (int64_t)1 << 30) return MP_E_LIMIT;
    }
  }

  mp_plan* p = new (std::nothrow) mp_plan;
  if (!p) return MP_E_NOMEM;
  p->W = W;
  p->batch = batch;
  p->flags = flags;
  p->eps = kernel_tol;
  p->f64 = (flags & MP_PREC_F64) != 0;
  p->dft_fmt = (flags & MP_DFT_F16SPLIT) ? 0 : ((flags & MP_DFT_BF16SPLIT) ? 1 : -1);
  p->dicts.assign(dicts, dicts + W);
  hipStream_t st = nullptr;
  double2* d_roots = nullptr;
  double2* d_full = nullptr;
  int* d_box = nullptr;
  unsigned long long* d_max = nullptr;
  std::vector<double2*> ptab64;
  std::vector<float2*> ptab32;
  {
    int dev_count = 0;
    if (hipGetDeviceCount(&dev_count) != hipSuccess || dev_count < 1) {
      delete p;
      return MP_E_HIP;
    }
    HCHK(hipGetDevice(&p->device));
    hipDeviceProp_t prop;
    HCHK(hipGetDeviceProperties(&prop, p->device));

    // ---- lengths (Sec. 2.1: a_w, M_w divide L; zero padding) ----
    int64_t q = 1, need = 0;
    for (int w = 0; w < W; ++w) {
      q = q / gcd64(q, dicts[w].a) * dicts[w].a;
      q = q / gcd64(q, dicts[w].M) * dicts[w].M;
      for (int v = 0; v < W; ++v) need = std::max<int64_t>(need, dicts[w].gl + dicts[v].gl);
    }
    // tree group size.  FP64: keep the group nodes within 32 KiB of LDS.
    // FP32: 256 leaves (128 with MP_SCHED_G128) if the group keys fit the LDS.
    {
      auto groups_max = [&](int G) {
        int64_t m = 0;
        for (int s = 0; s < batch; ++s) {
          const int64_t Lp = (L[s] + q - 1) / q * q;
          int64_t c = 0;
          for (int w = 0; w < W; ++w)
            c += ((Lp / dicts[w].a) * ((dicts[w].M / 2 + 1 + ROW - 1) / ROW) + G - 1) / G;
          m = std::max(m, c);
        }
        return m;
      };
      if (p->f64) {
        const size_t node = 32;
        int64_t maxl = 0;
        for (int s = 0; s < batch; ++s) {
          const int64_t Lp = (L[s] + q - 1) / q * q;
          int64_t c = 0;
          for (int w = 0; w < W; ++w) c += (Lp / dicts[w].a) * ((dicts[w].M / 2 + 1 + ROW - 1) / ROW);
          maxl = std::max(maxl, c);
        }
        p->G = GLEAVES;
        p->logG = 8;
        while ((size_t)((maxl + p->G - 1) / p->G + W) * node > 32 * 1024) {
          p->G *= 2;
          p->logG += 1;
        }
      } else {
        // 768 threads (12 waves) unless the group keys and the owners'
        // scratch only fit the LDS with 512 (or MP_SCHED_NT512 asks for it)
        p->G = 0;
        const int gpref = (flags & MP_SCHED_G128) ? 128 : 256, ntpref = (flags & MP_SCHED_NT512) ? 512 : 768;
        for (int nt : {768, 512}) {
          if (nt > ntpref) continue;
          for (int G : {128, 256}) {
            if (G < gpref) continue;
            const int64_t ng = groups_max(G);
            if (ng < (1 << 24) && mp_shmem_bytes(false, nt, G, (int)ng) <= 160 * 1024) {
              p->G = G;
              p->logG = G == 128 ? 7 : 8;
              p->nt = nt;
              break;
            }
          }
          if (p->G) break;
        }
        if (!p->G) {
          rc = MP_E_LIMIT;
          goto fail;
        }
      }
    }
    p->hs.resize(batch);
    int64_t xoff = 0, cbase = 0, lbase_all = 0;
    for (int s = 0; s < batch; ++s) {
      SigDev& S = p->hs[s];
      memset(&S, 0, sizeof(S));
      S.L = L[s];
      S.Lp = (L[s] + q - 1) / q * q;
      S.x_off = xoff;
      xoff += S.L;
      int64_t off = 0, lb = 0;
      for (int w = 0; w < W; ++w) {
        const int MR = dicts[w].M / 2 + 1, lpf = (MR + ROW - 1) / ROW;
        S.N[w] = (int32_t)(S.Lp / dicts[w].a);
        if (S.N[w] >= (1 << 24)) {  // frame indices enter 24-bit multiplies
          rc = MP_E_LIMIT;
          goto fail;
        }
        S.off[w] = off;
        off += (int64_t)S.N[w] * MR;
        S.lbase[w] = lb;
        lb += ((int64_t)S.N[w] * lpf + p->G - 1) / p->G * p->G;
      }
      for (int w = W; w <= MAXW; ++w) {
        S.off[w] = off;
        S.lbase[w] = lb;
      }
      if (off >= ((int64_t)1 << 31) - ROW || lb >= ((int64_t)1 << 31)) {
        rc = MP_E_LIMIT;
        goto fail;
      }
      S.n_coef_padded = (off + ROW - 1) / ROW * ROW;
      S.coef_base = cbase;
      cbase += S.n_coef_padded;
      S.leaf_base = lbase_all;
      lbase_all += lb;
      S.n_leaves = (int32_t)lb;
      S.n_groups = (int32_t)(lb / p->G);
      p->max_Lp = std::max(p->max_Lp, S.Lp);
    }
    p->total_coef = cbase;
    p->total_leaves = lbase_all;
    p->n_groups_max = 0;
    for (auto& S : p->hs) p->n_groups_max = std::max(p->n_groups_max, S.n_groups);
    // atom logs (default capacity L_padded / 5)
    {
      int64_t base = 0;
      for (auto& S : p->hs) {
        S.atom_base = base;
        S.cap = std::max<int64_t>(S.Lp / 5, 1);
        base += S.cap;
      }
      p->total_cap = base;
    }

    HCHK(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));

    // ---- windows and DFT twiddles ----
    p->hd.resize(W);
    {
      std::vector<double> w64;
      std::vector<float> w32;
      int64_t twoff = 0, gamoff = 0, rootoff = 0;
      for (int w = 0; w < W; ++w) {
        std::vector<double> g;
        make_window(dicts[w].window, dicts[w].gl, dicts[w].a, dicts[w].M, g);
        DictDev& D = p->hd[w];
        D.gl = dicts[w].gl;
        D.a = dicts[w].a;
        D.M = dicts[w].M;
        D.MR = dicts[w].M / 2 + 1;
        D.win_off = (int64_t)w64.size();
        D.tw_off = twoff;
        D.gamma_off = gamoff;
        D.root_off = rootoff;
        magic_u32((uint32_t)D.MR, &D.mr_mul, &D.mr_sh);
        magic_u32((uint32_t)D.M, &D.m_mul, &D.m_sh);
        D.lpf = (D.MR + ROW - 1) / ROW;
        D.pad = 0;
        D.pad2[0] = D.pad2[1] = 0;
        twoff += std::max(D.M, 2);  // M/2 twiddles, then their stage-major copy
        gamoff += D.MR;
        rootoff += D.M;
        for (double v : g) {
          w64.push_back(v);
          w32.push_back((float)v);
        }
      }
      ACHK(dalloc(&p->d_win64, w64.size()));
      ACHK(dalloc(&p->d_win32, w32.size()));
      HCHK(hipMemcpy(p->d_win64, w64.data(), w64.size() * sizeof(double), hipMemcpyHostToDevice));
      HCHK(hipMemcpy(p->d_win32, w32.data(), w32.size() * sizeof(float), hipMemcpyHostToDevice));
      ACHK(dalloc(&p->d_tw64, (size_t)twoff));
      ACHK(dalloc(&p->d_tw32, (size_t)twoff));
      for (int w = 0; w < W; ++w) {
        HCHK(launch_roots(p->hd[w].M, p->hd[w].M / 2, -1, p->d_tw64 + p->hd[w].tw_off,
                          p->d_tw32 + p->hd[w].tw_off, st));
        // the radix-2 stages' twiddle copy (M a power of two, or 3 times one)
        if (is_pow2(p->hd[w].M) || (p->hd[w].M % 3 == 0 && is_pow2(p->hd[w].M / 3)))
          HCHK(launch_stage_tw(p->hd[w].M, p->d_tw64 + p->hd[w].tw_off, p->d_tw32 + p->hd[w].tw_off, st));
      }
      // one entry past the end: the FP32 loop reads gamma of two adjacent bins
      ACHK(dalloc(&p->d_gam64, (size_t)gamoff + 1));
      ACHK(dalloc(&p->d_gam32, (size_t)gamoff + 1));
      // exp(+2 pi i j / M), j < M: the phases exp(2 pi i k Delta / M_v) of Eq. (hkj)
      ACHK(dalloc(&p->d_root64, (size_t)rootoff));
      ACHK(dalloc(&p->d_root32, (size_t)rootoff));
      for (int w = 0; w < W; ++w)
        HCHK(launch_roots(p->hd[w].M, p->hd[w].M, +1, p->d_root64 + p->hd[w].root_off,
                          p->d_root32 + p->hd[w].root_off, st));
    }

    // ---- split half-precision DFT matrices for the four-step DFT ----
    if (p->dft_fmt >= 0) {
      p->dft_n1.assign(W, 0);
      p->dft_n2.assign(W, 0);
      p->d_dft1.assign(W, nullptr);
      p->d_dft2.assign(W, nullptr);
      for (int w = 0; w < W; ++w) {
        const int H = dicts[w].M / 2;
        int lh = 0;
        while ((1 << lh) < H) ++lh;
        const int n1 = 1 << ((lh + 1) / 2), n2 = H / n1;
        p->dft_n1[w] = n1;
        p->dft_n2[w] = n2;
        const int n1p = std::max(n1, 16), n2p = std::max(n2, 16);
        ACHK(dalloc(&p->d_dft1[w], (size_t)6 * n1p * n1p));
        ACHK(dalloc(&p->d_dft2[w], (size_t)6 * n2p * n2p));
        HCHK(launch_dft_tables(p->dft_fmt, n1, n1p, p->d_dft1[w], st));
        HCHK(launch_dft_tables(p->dft_fmt, n2, n2p, p->d_dft2[w], st));
      }
    }

    // ---- truncated cross-kernels, FP64 on the device (Sec. 4.1, 4.2) ----
    p->hp.resize((size_t)W * W);
    p->kinfo.resize((size_t)W * W);
    p->kre.resize((size_t)W * W);
    p->kim.resize((size_t)W * W);
    {
      size_t full_max = 0;
      int Mmax_all = 0;
      for (int w = 0; w < W; ++w)
        for (int v = 0; v < W; ++v) {
          const int amin = (int)gcd64(dicts[w].a, dicts[v].a);
          const int Mmax = (int)(dicts[w].M / gcd64(dicts[w].M, dicts[v].M) * dicts[v].M);  // lcm
          const int half = (dicts[w].gl + dicts[v].gl) / 2;
          const int D = (half + amin - 1) / amin - 1;
          full_max = std::max(full_max, (size_t)(2 * D + 1) * (size_t)Mmax);
          Mmax_all = std::max(Mmax_all, Mmax);
        }
      ACHK(dalloc(&d_full, full_max));
      ACHK(dalloc(&d_roots, (size_t)Mmax_all));
      ACHK(dalloc(&d_box, 4));
      ACHK(dalloc(&d_max, 1));
      int64_t tab_total = 0, tab_total32 = 0;
      ptab64.assign((size_t)W * W, nullptr);
      ptab32.assign((size_t)W * W, nullptr);
      for (int w = 0; w < W; ++w)
        for (int v = 0; v < W; ++v) {
          const int idx = w * W + v;
          const int amin = (int)gcd64(dicts[w].a, dicts[v].a);
          const int Mmax = (int)(dicts[w].M / gcd64(dicts[w].M, dicts[v].M) * dicts[v].M);  // lcm
          const int half = (dicts[w].gl + dicts[v].gl) / 2;
          const int D = (half + amin - 1) / amin - 1;
          HCHK(launch_roots(Mmax, Mmax, -1, d_roots, nullptr, st));
          HCHK(launch_gram_full(p->d_win64 + p->hd[w].win_off, dicts[w].gl, p->d_win64 + p->hd[v].win_off,
                                dicts[v].gl, amin, D, Mmax, d_roots, d_full, st));
          double thr = kernel_tol;
          if (flags & MP_THR_REL) {
            unsigned long long zero = 0, mx = 0;
            HCHK(hipMemcpyAsync(d_max, &zero, sizeof(zero), hipMemcpyHostToDevice, st));
            HCHK(launch_gram_absmax(d_full, (int64_t)(2 * D + 1) * Mmax, d_max, st));
            HCHK(hipMemcpyAsync(&mx, d_max, sizeof(mx), hipMemcpyDeviceToHost, st));
            HCHK(hipStreamSynchronize(st));
            double m;
            memcpy(&m, &mx, sizeof(m));
            thr = kernel_tol * m;
          }
          int box[4] = {-1, Mmax, -Mmax, 0};
          HCHK(hipMemcpyAsync(d_box, box, sizeof(box), hipMemcpyHostToDevice, st));
          HCHK(launch_gram_box(d_full, D, Mmax, thr, d_box, st));
          HCHK(hipMemcpyAsync(box, d_box, sizeof(box), hipMemcpyDeviceToHost, st));
          HCHK(hipStreamSynchronize(st));
          PairDev& P = p->hp[idx];
          P.amin = amin;
          P.Mmax = Mmax;
          P.rw = Mmax / dicts[w].M;
          P.rv = Mmax / dicts[v].M;
          P.sw = dicts[w].a / amin;
          P.sv = dicts[v].a / amin;
          if (box[3] > 0) {
            P.dbox = box[0];
            P.mu_lo = box[1];
            P.mu_hi = box[2];
          } else {
            P.dbox = -1;
            P.mu_lo = 0;
            P.mu_hi = -1;
          }
          P.width = P.mu_hi - P.mu_lo + 1;
          P.cw = (P.width + P.rw - 1) / P.rw;
          P.width32 = P.cw * P.rw;
          // the FP32 loop steps table rows with 24-bit multiplies
          if ((int64_t)P.width32 * P.sw >= ((int64_t)1 << 24)) {
            rc = MP_E_LIMIT;
            goto fail;
          }
          const size_t n = P.dbox >= 0 ? (size_t)(2 * P.dbox + 1) * (size_t)P.width : 0;
          P.tab_off = tab_total;
          tab_total += (int64_t)n;
          P.tab_off32 = tab_total32;
          tab_total32 += P.dbox >= 0 ? (int64_t)(2 * P.dbox + 1) * P.width32 : 0;
          mp_kernel_info& KI = p->kinfo[idx];
          KI.amin = amin;
          KI.Mmax = Mmax;
          KI.D = D;
          KI.delta_box = P.dbox;
          KI.mu_lo = P.mu_lo;
          KI.mu_hi = P.mu_hi;
          KI.n_nonzero = box[3];
          if (n) {
            ACHK(dalloc(&ptab64[idx], n));
            ACHK(dalloc(&ptab32[idx], n));
            HCHK(launch_gram_extract(d_full, D, Mmax, thr, P.dbox, P.mu_lo, P.width, ptab64[idx],
                                     ptab32[idx], st));
            std::vector<double2> host(n);
            HCHK(hipMemcpyAsync(host.data(), ptab64[idx], n * sizeof(double2), hipMemcpyDeviceToHost, st));
            HCHK(hipStreamSynchronize(st));
            p->kre[idx].resize(n);
            p->kim[idx].resize(n);
            for (size_t i = 0; i < n; ++i) {
              p->kre[idx][i] = host[i].x;
              p->kim[idx][i] = host[i].y;
            }
          }
        }
      // rows updated per selection: the FP32 loop maps row -> frame with an
      // FP32 reciprocal, exact while the row index stays below 2^21
      for (int v = 0; v < W; ++v) {
        int64_t rows = 0, tg = 0;
        for (int w = 0; w < W; ++w) {
          const PairDev& P = p->hp[w * W + v];
          if (P.dbox < 0) continue;
          rows += ((int64_t)2 * P.dbox / P.sw + 10) * (((int64_t)dicts[w].M / 2 + ROW) / ROW);
          // the touched leaves of target w span at most (frames) x (leaves per
          // frame); each of the two runs (the second one past the wrap) may
          // straddle one more group boundary
          tg += ((int64_t)2 * P.dbox / P.sw + 2) * (((int64_t)dicts[w].M / 2 + ROW) / ROW) / p->G + 3;
        }
        p->tg_bound = std::max(p->tg_bound, tg);
        if (rows >= ((int64_t)1 << 21)) {
          rc = MP_E_LIMIT;
          goto fail;
        }
        // the FP32 loop takes the phase index (ph0 + f phs) mod M_v of frame
        // f < frames per selection by a 31-bit division
        for (int w = 0; w < W; ++w) {
          const PairDev& P = p->hp[w * W + v];
          if (P.dbox >= 0 && (int64_t)dicts[v].M * ((int64_t)2 * P.dbox / P.sw + 3) >= ((int64_t)1 << 31)) {
            rc = MP_E_LIMIT;
            goto fail;
          }
        }
      }
      ACHK(dalloc(&p->d_tab64, (size_t)tab_total));
      if (tab_total32 >= ((int64_t)1 << 31)) {  // FP32 table rows are addressed with 32-bit indices
        rc = MP_E_LIMIT;
        goto fail;
      }
      ACHK(dalloc(&p->d_tab32, (size_t)tab_total32));
      for (int i = 0; i < W * W; ++i) {
        const PairDev& P = p->hp[i];
        const size_t n = P.dbox >= 0 ? (size_t)(2 * P.dbox + 1) * (size_t)P.width : 0;
        if (!n) continue;
        HCHK(hipMemcpyAsync(p->d_tab64 + P.tab_off, ptab64[i], n * sizeof(double2), hipMemcpyDeviceToDevice, st));
        // FP32 copy in phase-major rows (padding entries are zero)
        std::vector<float2> nat(n), perm((size_t)(2 * P.dbox + 1) * P.width32, make_float2(0.0f, 0.0f));
        HCHK(hipMemcpyAsync(nat.data(), ptab32[i], n * sizeof(float2), hipMemcpyDeviceToHost, st));
        HCHK(hipStreamSynchronize(st));
        for (int r = 0; r < 2 * P.dbox + 1; ++r)
          for (int u = 0; u < P.width; ++u)
            perm[(size_t)r * P.width32 + (size_t)(u % P.rw) * P.cw + (size_t)(u / P.rw)] = nat[(size_t)r * P.width + u];
        HCHK(hipMemcpyAsync(p->d_tab32 + P.tab_off32, perm.data(), perm.size() * sizeof(float2),
                            hipMemcpyHostToDevice, st));
        HCHK(hipStreamSynchronize(st));
      }
      // gamma(k) = <d, conj d> = h_{v,v}(-2k mod M_v, 0) of the truncated auto kernel (Sec. 5.2)
      std::vector<double2> g64;
      std::vector<float2> g32;
      for (int v = 0; v < W; ++v) {
        const PairDev& P = p->hp[v * W + v];
        const int M = dicts[v].M;
        for (int k = 0; k <= M / 2; ++k) {
          int mu = (-2 * k) % M;
          if (mu < 0) mu += M;
          if (mu > M / 2) mu -= M;
          double re = 0.0, im = 0.0;
          if (P.dbox >= 0 && mu >= P.mu_lo && mu <= P.mu_hi) {
            const size_t i = (size_t)P.dbox * P.width + (size_t)(mu - P.mu_lo);
            re = p->kre[v * W + v][i];
            im = p->kim[v * W + v][i];
          }
          g64.push_back(make_double2(re, im));
          g32.push_back(make_float2((float)re, (float)im));
        }
      }
      g64.push_back(make_double2(0.0, 0.0));
      g32.push_back(make_float2(0.0f, 0.0f));
      HCHK(hipMemcpy(p->d_gam64, g64.data(), g64.size() * sizeof(double2), hipMemcpyHostToDevice));
      HCHK(hipMemcpy(p->d_gam32, g32.data(), g32.size() * sizeof(float2), hipMemcpyHostToDevice));
    }

    // ---- per-signal buffers ----
    ACHK(dalloc(&p->d_dicts, (size_t)W));
    HCHK(hipMemcpy(p->d_dicts, p->hd.data(), sizeof(DictDev) * W, hipMemcpyHostToDevice));
    ACHK(dalloc(&p->d_pairs, (size_t)W * W));
    HCHK(hipMemcpy(p->d_pairs, p->hp.data(), sizeof(PairDev) * W * W, hipMemcpyHostToDevice));
    ACHK(dalloc(&p->d_sigs, (size_t)batch));
    HCHK(hipMemcpy(p->d_sigs, p->hs.data(), sizeof(SigDev) * batch, hipMemcpyHostToDevice));
    ACHK(dalloc(&p->d_state, (size_t)batch));
    HCHK(hipMemset(p->d_state, 0, sizeof(SigState) * batch));
    ACHK(dalloc(&p->d_epart, (size_t)batch * ENERGY_PARTS));
    const size_t cb = p->f64 ? 16 : 8;
    // one coefficient past the end: the FP32 loop reads two adjacent bins
    HCHK(hipMalloc(&p->d_planes, (size_t)(p->total_coef + 1) * cb));
    HCHK(hipMemset(p->d_planes, 0, (size_t)(p->total_coef + 1) * cb));
    HCHK(hipMalloc(&p->d_leaves, (size_t)std::max<int64_t>(p->total_leaves, 1) * leaf_bytes(p->f64)));
    // padding leaves (systems rounded up to whole groups) are never written by
    // the analysis and must read as empty keys
    HCHK(hipMemset(p->d_leaves, 0, (size_t)std::max<int64_t>(p->total_leaves, 1) * leaf_bytes(p->f64)));
    ACHK(dalloc(&p->d_atoms, (size_t)p->total_cap));
    ACHK(dalloc(&p->d_acc, (size_t)p->max_Lp));
    // longest signals first
    p->order.resize(batch);
    std::iota(p->order.begin(), p->order.end(), 0);
    std::stable_sort(p->order.begin(), p->order.end(),
                     [&](int a, int b) { return p->hs[a].Lp > p->hs[b].Lp; });
    ACHK(dalloc(&p->d_order, (size_t)batch));
    HCHK(hipMemcpy(p->d_order, p->order.data(), sizeof(int32_t) * batch, hipMemcpyHostToDevice));
    ACHK(dalloc(&p->d_queue, 1));
    p->frames_total.assign(W, 0);
    for (int w = 0; w < W; ++w) {
      std::vector<int64_t> pre(batch);
      int64_t acc = 0;
      for (int s = 0; s < batch; ++s) {
        pre[s] = acc;
        acc += p->hs[s].N[w];
      }
      p->frames_total[w] = acc;
      ACHK(dalloc(&p->d_fprefix[w], (size_t)batch));
      HCHK(hipMemcpy(p->d_fprefix[w], pre.data(), sizeof(int64_t) * batch, hipMemcpyHostToDevice));
    }
    for (auto& e : p->ev) HCHK(hipEventCreate(&e));
    p->ev_valid = true;

    // launch shape of the MP loop (FP32: chosen with the group size above)
    if (p->f64) p->nt = 512;
    p->shmem = mp_shmem_bytes(p->f64, p->nt, p->G, p->n_groups_max);
    if (p->shmem == 0 || p->shmem > 160 * 1024) {
      rc = MP_E_LIMIT;
      goto fail;
    }
    p->grid = std::min(batch, 2 * prop.multiProcessorCount);
    HCHK(hipStreamSynchronize(st));
  }
  for (auto t : ptab64) dfree(t);
  for (auto t : ptab32) dfree(t);
  dfree(d_full);
  dfree(d_roots);
  dfree(d_box);
  dfree(d_max);
  (void)hipStreamDestroy(st);
  *out = p;
  return MP_OK;

fail:
  if (st) {
    (void)hipStreamSynchronize(st);
    (void)hipStreamDestroy(st);
  }
  for (auto t : ptab64) dfree(t);
  for (auto t : ptab32) dfree(t);
  dfree(d_full);
  dfree(d_roots);
  dfree(d_box);
  dfree(d_max);
  free_plan(p);
  return rc;
}

int mp_autotune(const mp_dict* dicts, int32_t W, const int64_t* L, int32_t batch, double kernel_tol, uint32_t flags,
                const void* x_dev, int32_t dtype, int64_t probe_atoms, hipStream_t stream, mp_plan** out,
                mp_tune_report* rep) {
  constexpr uint32_t NT = MP_SCHED_NT512, G1 = MP_SCHED_G128, T8 = MP_SCHED_TILE8, T32 = MP_SCHED_TILE32;
  if (!out || !x_dev || probe_atoms <= 0 || (flags & (NT | G1 | T8 | T32))) return MP_E_ARG;
  *out = nullptr;
  const uint32_t cands[MP_TUNE_MAX] = {0u, G1, NT, NT | G1, T8, G1 | T8, NT | T8, NT | G1 | T8, NT | T32, NT | G1 | T32};
  const int ncand = (flags & MP_PREC_F64) ? 1 : MP_TUNE_MAX;
  mp_tune_report r;
  memset(&r, 0, sizeof(r));
  r.chosen = -1;
  mp_plan* best = nullptr;
  double best_ms = 0.0;
  for (int c = 0; c < ncand; ++c) {
    mp_plan* p = nullptr;
    int rc = mp_plan_create(dicts, W, L, batch, kernel_tol, flags | cands[c], &p);
    if (rc == MP_E_LIMIT) continue;  // this schedule does not fit
    if (rc != MP_OK) {
      mp_plan_destroy(best);
      return rc;
    }
    mp_stats s0;
    (void)mp_get_stats(p, &s0);  // launch shape and tile of the plan (no device work before analysis)
    bool dup = false;  // a preference that fell back to an earlier schedule
    for (int i = 0; i < r.n_cand; ++i)
      if (r.threads[i] == p->nt && r.group_leaves[i] == p->G && r.tile_rows[i] == s0.tile_rows) dup = true;
    if (dup) {
      mp_plan_destroy(p);
      continue;
    }
    rc = mp_analyze(p, x_dev, dtype, stream);
    if (rc == MP_OK) rc = mp_run(p, probe_atoms, 0.0, stream);
    if (rc == MP_OK && hipStreamSynchronize(stream) != hipSuccess) rc = MP_E_HIP;
    mp_stats st;
    if (rc == MP_OK) rc = mp_get_stats(p, &st);
    if (rc != MP_OK) {
      mp_plan_destroy(p);
      mp_plan_destroy(best);
      return rc;
    }
    const int i = r.n_cand++;
    r.flags[i] = cands[c];
    r.threads[i] = p->nt;
    r.group_leaves[i] = p->G;
    r.tile_rows[i] = st.tile_rows;
    r.probe_ms[i] = st.loop_ms;
    r.probe_bytes[i] = (p->f64 ? 32.0 : 16.0) * (double)st.updated + 8.0 * (double)(st.blocks + st.l1_groups);
    if (!best || st.loop_ms < 0.99 * best_ms) {  // more than 1 % faster: noise does not flip the choice
      mp_plan_destroy(best);
      best = p;
      best_ms = st.loop_ms;
      r.chosen = i;
    } else {
      mp_plan_destroy(p);
    }
  }
  if (!best) return MP_E_LIMIT;
  *out = best;
  if (rep) *rep = r;
  return MP_OK;
}

int mp_analyze(mp_plan* p, const void* x_dev, int32_t dtype, hipStream_t stream) {
  if (!p || !x_dev || (dtype != MP_DTYPE_F32 && dtype != MP_DTYPE_F64)) return MP_E_ARG;
  int rc = MP_OK;
  const bool dft64 = !p->f64 && (p->flags & MP_DFT_F64);  // FP64 DFT for an FP32 plan
  const bool r64 = p->f64 || dft64;
  const void* win = r64 ? (const void*)p->d_win64 : (const void*)p->d_win32;
  const bool cap = capturing(stream);
  if (!cap) HCHK(hipEventRecord(p->ev[0], stream));
  HCHK(launch_energy(x_dev, dtype, p->d_sigs, p->batch, p->d_epart, p->d_state, stream));
  if (!cap) HCHK(hipEventRecord(p->ev[5], stream));  // the DGT kernels alone: ev[5] -> ev[1]
  for (int w = 0; w < p->W; ++w) {
    const DictDev& D = p->hd[w];
    const void* tw = p->dft_fmt >= 0 ? (const void*)(p->d_tw32 + D.tw_off)
                     : (r64 ? (const void*)(p->d_tw64 + D.tw_off) : (const void*)(p->d_tw32 + D.tw_off));
    if (p->dft_fmt >= 0)
      HCHK(launch_dgt_mfma(p->dft_fmt, x_dev, dtype, p->d_sigs, w, D.gl, D.a, D.M, D.MR, p->d_fprefix[w],
                           p->batch, p->frames_total[w], p->d_win32 + D.win_off, tw, p->dft_n1[w],
                           p->dft_n2[w], p->d_dft1[w], p->d_dft2[w], p->d_planes, p->d_leaves, (p->f64 ? (const void*)(p->d_gam64 + D.gamma_off) : (const void*)(p->d_gam32 + D.gamma_off)), (p->flags & MP_PEDANTIC) ? 1 : 0, p->max_Lp, stream));
    else
      HCHK(launch_dgt(p->f64, dft64, x_dev, dtype, p->d_sigs, w, D.gl, D.a, D.M, D.MR, p->d_fprefix[w], p->batch,
                      p->frames_total[w], (const char*)win + D.win_off * (r64 ? 8 : 4), tw, p->d_planes,
                      p->d_leaves, (p->f64 ? (const void*)(p->d_gam64 + D.gamma_off) : (const void*)(p->d_gam32 + D.gamma_off)), (p->flags & MP_PEDANTIC) ? 1 : 0,
                      p->d_root64 + D.root_off, stream));
  }
  if (!cap) {
    HCHK(hipEventRecord(p->ev[1], stream));
    HCHK(hipEventRecord(p->ev[2], stream));
  }
  p->analyzed = true;
  p->ran = false;
  p->last_stream = stream;
  return MP_OK;
fail:
  return rc;
}

static MPArgs mp_args(const mp_plan* p, int64_t max_atoms, double target_snr_db) {
  MPArgs a;
  a.dicts = p->d_dicts;
  a.pairs = p->d_pairs;
  a.sigs = p->d_sigs;
  a.state = p->d_state;
  a.planes = p->d_planes;
  a.leaves = p->d_leaves;
  a.atoms = p->d_atoms;
  a.tabs = p->f64 ? (const void*)p->d_tab64 : (const void*)p->d_tab32;
  a.gammas = p->f64 ? (const void*)p->d_gam64 : (const void*)p->d_gam32;
  a.roots = p->f64 ? (const void*)p->d_root64 : (const void*)p->d_root32;
  a.n_groups_max = p->n_groups_max;
  a.slot_cap = (p->flags & MP_SCHED_TILE8) ? 1 : ((p->flags & MP_SCHED_TILE32) ? 4 : 2);
  // selections that may touch more groups than the loop preloads (two per
  // wave) get the kernel that loads the rest early
  a.xpre = p->tg_bound > 2 * (p->nt / 64) ? 1 : 0;
  a.p2 = 1;
  for (int w = 0; w < p->W; ++w)
    if (!is_pow2(p->hd[w].M)) a.p2 = 0;
  a.order = p->d_order;
  a.queue = p->d_queue;
  a.W = p->W;
  a.batch = p->batch;
  a.G = p->G;
  a.logG = p->logG;
  a.K = max_atoms;
  a.snr_db = target_snr_db;
  a.partner_gate = (p->flags & MP_CONJ_GATE_GAMMA) ? 1u : 0u;
  a.pedantic = (p->flags & MP_PEDANTIC) ? 1u : 0u;
  a.reset_it = 0;
  a.reset_db = 0.0;
  return a;
}

int mp_run(mp_plan* p, int64_t max_atoms, double target_snr_db, hipStream_t stream) {
  if (!p) return MP_E_ARG;
  if (!p->analyzed) return MP_E_STATE;
  const bool cap = capturing(stream);
  if (cap) {  // the atom logs must already hold max_atoms: no allocation under capture
    for (int s = 0; s < p->batch; ++s)
      if (p->hs[s].cap < (max_atoms > 0 ? max_atoms : std::max<int64_t>(p->hs[s].Lp / 5, 1))) return MP_E_STATE;
  }
  int rc = ensure_cap(p, max_atoms, stream);
  if (rc) return rc;
  const MPArgs a = mp_args(p, max_atoms, target_snr_db);
  if (!cap) HCHK(hipEventRecord(p->ev[3], stream));
  HCHK(launch_mp(p->f64, p->nt, a, p->grid, stream));
  if (!cap) HCHK(hipEventRecord(p->ev[4], stream));
  p->last_stream = stream;
  p->last_K = max_atoms;
  p->ran = true;
  return MP_OK;
fail:
  return rc;
}

int mp_signal_info_get(const mp_plan* p, int32_t sig, mp_signal_info* out) {
  if (!p || !out || sig < 0 || sig >= p->batch) return MP_E_ARG;
  if (hipStreamSynchronize(p->last_stream) != hipSuccess) return MP_E_HIP;
  SigState st;
  if (hipMemcpy(&st, p->d_state + sig, sizeof(st), hipMemcpyDeviceToHost) != hipSuccess) return MP_E_HIP;
  const SigDev& S = p->hs[sig];
  out->L = S.L;
  out->L_padded = S.Lp;
  out->x_offset = S.x_off;
  int64_t nc = 0;
  for (int w = 0; w < p->W; ++w) nc += (int64_t)S.N[w] * p->hd[w].MR;
  out->n_coefs = nc;
  out->n_atoms = p->analyzed ? st.k : 0;
  out->stop_reason = p->analyzed ? st.stop : 0;
  out->pad = 0;
  out->E0 = st.E0;
  out->E = st.E;
  return MP_OK;
}

int mp_run_resets(mp_plan* p, const void* x_dev, int32_t dtype, int64_t max_atoms, double target_snr_db,
                  int64_t reset_it, double reset_db, hipStream_t stream) {
  if (!p || !x_dev || (dtype != MP_DTYPE_F32 && dtype != MP_DTYPE_F64) || !(reset_db <= 0.0)) return MP_E_ARG;
  if (!p->analyzed || p->ran) return MP_E_STATE;
  if (reset_it <= 0) {
    // default reset criterion derived from the kernel threshold (Sec. 7, the
    // 'reset' flag; the paper does not print its formula): at most
    // ceil(32 / eps) selections per round (the schedule of Sec. 6.1's second
    // experiment at eps = 1e-4 and 1e-3), and a reset once the estimate has
    // fallen by the factor eps below the error at the last reset
    reset_it = p->eps > 0.0 ? (int64_t)std::ceil(32.0 / p->eps) : ((int64_t)1 << 62);
    if (reset_db == 0.0 && p->eps > 0.0) reset_db = 10.0 * std::log10(p->eps);
  }
  int rc = ensure_cap(p, max_atoms, stream);
  if (rc) return rc;
  if (!p->d_res) {
    std::vector<int64_t> roff((size_t)p->batch);
    std::vector<SigDev> sr = p->hs;
    int64_t tot = 0;
    for (int s = 0; s < p->batch; ++s) {
      roff[s] = tot;
      sr[s].x_off = tot;
      sr[s].L = sr[s].Lp;
      tot += p->hs[s].Lp;
    }
    ACHK(dalloc(&p->d_res, (size_t)tot));
    ACHK(dalloc(&p->d_roff, (size_t)p->batch));
    ACHK(dalloc(&p->d_sigs_res, (size_t)p->batch));
    ACHK(dalloc(&p->d_active, 1));
    HCHK(hipMemcpy(p->d_roff, roff.data(), sizeof(int64_t) * p->batch, hipMemcpyHostToDevice));
    HCHK(hipMemcpy(p->d_sigs_res, sr.data(), sizeof(SigDev) * p->batch, hipMemcpyHostToDevice));
  }
  {
    MPArgs a = mp_args(p, max_atoms, target_snr_db);
    a.reset_it = reset_it;
    a.reset_db = reset_db;
    HCHK(hipEventRecord(p->ev[3], stream));
    HCHK(launch_reset_init(x_dev, dtype, p->d_sigs, p->batch, p->max_Lp, p->d_roff, p->d_res, stream));
    const bool dft64 = !p->f64 && (p->flags & MP_DFT_F64);
    const bool r64 = p->f64 || dft64;
    const void* win = r64 ? (const void*)p->d_win64 : (const void*)p->d_win32;
    for (;;) {
      // inner loop: approximate MP on the current residual's coefficients
      HCHK(launch_mp(p->f64, p->nt, a, p->grid, stream));
      // solution and true residual, error, finished signals
      HCHK(hipMemsetAsync(p->d_active, 0, sizeof(int), stream));
      HCHK(launch_reset_update(p->d_atoms, p->d_sigs, p->d_state, p->d_dicts, p->d_win64, p->d_roff, p->d_res,
                               p->batch, target_snr_db, max_atoms, p->d_active, stream));
      int active = 0;
      HCHK(hipMemcpyAsync(&active, p->d_active, sizeof(int), hipMemcpyDeviceToHost, stream));
      // re-analysis of the residual: rho = D* r (also for the signals that just
      // finished, so that their planes hold the analysis of the final residual)
      for (int w = 0; w < p->W; ++w) {
        const DictDev& D = p->hd[w];
        const void* tw = p->dft_fmt >= 0 ? (const void*)(p->d_tw32 + D.tw_off)
                         : (r64 ? (const void*)(p->d_tw64 + D.tw_off) : (const void*)(p->d_tw32 + D.tw_off));
        if (p->dft_fmt >= 0)
          HCHK(launch_dgt_mfma(p->dft_fmt, p->d_res, MP_DTYPE_F64, p->d_sigs_res, w, D.gl, D.a, D.M, D.MR,
                               p->d_fprefix[w], p->batch, p->frames_total[w], p->d_win32 + D.win_off, tw,
                               p->dft_n1[w], p->dft_n2[w], p->d_dft1[w], p->d_dft2[w], p->d_planes, p->d_leaves,
                               (p->f64 ? (const void*)(p->d_gam64 + D.gamma_off) : (const void*)(p->d_gam32 + D.gamma_off)), (p->flags & MP_PEDANTIC) ? 1 : 0, p->max_Lp, stream));
        else
          HCHK(launch_dgt(p->f64, dft64, p->d_res, MP_DTYPE_F64, p->d_sigs_res, w, D.gl, D.a, D.M, D.MR,
                          p->d_fprefix[w], p->batch, p->frames_total[w],
                          (const char*)win + D.win_off * (r64 ? 8 : 4), tw,
                          p->d_planes, p->d_leaves, (p->f64 ? (const void*)(p->d_gam64 + D.gamma_off) : (const void*)(p->d_gam32 + D.gamma_off)), (p->flags & MP_PEDANTIC) ? 1 : 0,
                          p->d_root64 + D.root_off, stream));
      }
      HCHK(hipStreamSynchronize(stream));
      if (!active) break;
    }
    HCHK(hipEventRecord(p->ev[4], stream));
  }
  p->last_stream = stream;
  p->last_K = max_atoms;
  p->ran = true;
  return MP_OK;
fail:
  return rc;
}

int mp_get_atoms(const mp_plan* p, int32_t sig, mp_atom* out_host, int64_t cap, int64_t* n_out) {
  if (!p || sig < 0 || sig >= p->batch || cap < 0 || (cap > 0 && !out_host)) return MP_E_ARG;
  mp_signal_info inf;
  int rc = mp_signal_info_get(p, sig, &inf);
  if (rc) return rc;
  if (n_out) *n_out = inf.n_atoms;
  const int64_t n = std::min(cap, inf.n_atoms);
  if (n > 0 && hipMemcpy(out_host, p->d_atoms + p->hs[sig].atom_base, sizeof(AtomRec) * (size_t)n,
                         hipMemcpyDeviceToHost) != hipSuccess)
    return MP_E_HIP;
  return MP_OK;
}

int mp_get_energy(const mp_plan* p, int32_t sig, double* E_host, int64_t cap, int64_t* n_out) {
  if (!p || sig < 0 || sig >= p->batch || cap < 0 || (cap > 0 && !E_host)) return MP_E_ARG;
  mp_signal_info inf;
  int rc = mp_signal_info_get(p, sig, &inf);
  if (rc) return rc;
  if (n_out) *n_out = inf.n_atoms + 1;
  if (cap == 0) return MP_OK;
  E_host[0] = inf.E0;
  const int64_t n = std::min(cap - 1, inf.n_atoms);
  if (n > 0) {
    std::vector<AtomRec> a((size_t)n);
    if (hipMemcpy(a.data(), p->d_atoms + p->hs[sig].atom_base, sizeof(AtomRec) * (size_t)n,
                  hipMemcpyDeviceToHost) != hipSuccess)
      return MP_E_HIP;
    for (int64_t i = 0; i < n; ++i) E_host[i + 1] = a[(size_t)i].E_after;
  }
  return MP_OK;
}

int mp_get_coefs(const mp_plan* p, int32_t sig, int32_t w, void* c_dev, hipStream_t stream) {
  if (!p || !c_dev || sig < 0 || sig >= p->batch || w < 0 || w >= p->W) return MP_E_ARG;
  if (!p->analyzed) return MP_E_STATE;
  const SigDev& S = p->hs[sig];
  const int64_t n = (int64_t)S.N[w] * p->hd[w].MR;
  if (launch_coefs(p->d_atoms + S.atom_base, p->d_state + sig, w, p->hd[w].MR, n, c_dev, stream) != hipSuccess)
    return MP_E_HIP;
  return MP_OK;
}

int mp_get_residual(const mp_plan* p, int32_t sig, int32_t w, void* dst_dev, hipStream_t stream) {
  if (!p || !dst_dev || sig < 0 || sig >= p->batch || w < 0 || w >= p->W) return MP_E_ARG;
  if (!p->analyzed) return MP_E_STATE;
  const SigDev& S = p->hs[sig];
  const size_t cb = p->f64 ? 16 : 8;
  const int64_t n = (int64_t)S.N[w] * p->hd[w].MR;
  const char* src = (const char*)p->d_planes + (size_t)(S.coef_base + S.off[w]) * cb;
  if (hipMemcpyAsync(dst_dev, src, (size_t)n * cb, hipMemcpyDeviceToDevice, stream) != hipSuccess)
    return MP_E_HIP;
  return MP_OK;
}

int mp_resynth(const mp_plan* p, int32_t sig, void* y_dev, int32_t dtype, hipStream_t stream) {
  if (!p || !y_dev || sig < 0 || sig >= p->batch || (dtype != MP_DTYPE_F32 && dtype != MP_DTYPE_F64))
    return MP_E_ARG;
  if (!p->analyzed) return MP_E_STATE;
  const SigDev& S = p->hs[sig];
  if (launch_resynth(p->d_atoms + S.atom_base, p->d_state + sig, p->d_dicts, p->d_win64, S.Lp, p->d_acc, y_dev,
                     dtype, stream) != hipSuccess)
    return MP_E_HIP;
  return MP_OK;
}

int mp_resynth_static(const mp_plan* p, int32_t sig, void* y_dev, int32_t dtype, hipStream_t stream) {
  if (!p || !y_dev || sig < 0 || sig >= p->batch || (dtype != MP_DTYPE_F32 && dtype != MP_DTYPE_F64))
    return MP_E_ARG;
  if (!p->analyzed) return MP_E_STATE;
  const SigDev& S = p->hs[sig];
  if (S.Lp > MP_STATIC_RESYNTH_MAX) return MP_E_LIMIT;
  static_assert(MP_STATIC_RESYNTH_MAX == STATIC_RESYNTH_MAX, "limit in the header and the array agree");
  int cur = -1;
  if (hipGetDevice(&cur) != hipSuccess) return MP_E_HIP;
  if (cur != p->device && hipSetDevice(p->device) != hipSuccess) return MP_E_HIP;
  double* acc = nullptr;
  int64_t cap = 0;
  int rc = MP_OK;
  if (static_scratch(&acc, &cap) != hipSuccess || cap < S.Lp)
    rc = MP_E_HIP;
  else if (launch_resynth(p->d_atoms + S.atom_base, p->d_state + sig, p->d_dicts, p->d_win64, S.Lp, acc, y_dev,
                          dtype, stream) != hipSuccess)
    rc = MP_E_HIP;
  if (cur != p->device && hipSetDevice(cur) != hipSuccess && rc == MP_OK) rc = MP_E_HIP;
  return rc;
}

int mp_kernel_info_get(const mp_plan* p, int32_t w, int32_t v, mp_kernel_info* out) {
  if (!p || !out || w < 0 || v < 0 || w >= p->W || v >= p->W) return MP_E_ARG;
  *out = p->kinfo[(size_t)w * p->W + v];
  return MP_OK;
}

int mp_get_kernel(const mp_plan* p, int32_t w, int32_t v, double* re, double* im, int64_t cap) {
  if (!p || w < 0 || v < 0 || w >= p->W || v >= p->W || cap < 0) return MP_E_ARG;
  const size_t i = (size_t)w * p->W + v;
  const int64_t n = (int64_t)p->kre[i].size();
  if (cap < n || (n > 0 && (!re || !im))) return MP_E_ARG;
  if (n) {
    memcpy(re, p->kre[i].data(), sizeof(double) * (size_t)n);
    memcpy(im, p->kim[i].data(), sizeof(double) * (size_t)n);
  }
  return MP_OK;
}

int mp_get_stats(const mp_plan* p, mp_stats* out) {
  if (!p || !out) return MP_E_ARG;
  memset(out, 0, sizeof(*out));
  out->group_leaves = p->G;
  out->threads = p->nt;
  out->tile_rows = p->f64 ? 0 : ((p->flags & MP_SCHED_TILE8) ? 8 : ((p->flags & MP_SCHED_TILE32) ? 32 : 16));
  out->early_groups = (!p->f64 && p->nt == 768 && p->tg_bound > 2 * (p->nt / 64)) ? 1 : 0;
  if (!p->analyzed) return MP_OK;
  if (hipStreamSynchronize(p->last_stream) != hipSuccess) return MP_E_HIP;
  std::vector<SigState> st((size_t)p->batch);
  if (hipMemcpy(st.data(), p->d_state, sizeof(SigState) * (size_t)p->batch, hipMemcpyDeviceToHost) != hipSuccess)
    return MP_E_HIP;
  for (auto& s : st) {
    out->atoms += s.k;
    out->updated += s.updated;
    out->blocks += s.blocks;
    out->l1_groups += s.groups;
  }
  float ms = 0.f;
  if (hipEventElapsedTime(&ms, p->ev[0], p->ev[2]) == hipSuccess) out->analyze_ms = ms;
  if (hipEventElapsedTime(&ms, p->ev[5], p->ev[1]) == hipSuccess) out->dgt_ms = ms;
  if (p->ran && hipEventElapsedTime(&ms, p->ev[3], p->ev[4]) == hipSuccess) out->loop_ms = ms;
  return MP_OK;
}

int mp_plan_destroy(mp_plan* p) {
  if (!p) return MP_E_ARG;
  if (p->last_stream) (void)hipStreamSynchronize(p->last_stream);
  (void)hipDeviceSynchronize();
  free_plan(p);
  return MP_OK;
}

}  // extern "C"
