/*
 * Plain FP64 CPU oracle for approximate coefficient-domain MP on multi-Gabor
 * dictionaries.  TEST INFRASTRUCTURE ONLY: used by the test suite, the smoke
 * check and the benchmark's CPU baseline; never by the GPU library.
 *
 * Notation follows the paper: a Gabor system (g, a, M) has atoms
 *   d_{m,n}(l) = g(l - n a) exp(2 pi i m (l - n a) / M)          (Sec. 2.1)
 * with circular indexing modulo the signal length L, N = L / a frames and, for
 * real signals, the reduced set of bins m = 0 .. M/2 (Sec. 5).
 */
#include "mp_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

#ifndef M_PI
#define M_PI 3.14159265358979323846
#endif

/* ------------------------------------------------------------------------ */
/* small integer helpers                                                    */

static int is_pow2(int64_t n) { return n > 0 && (n & (n - 1)) == 0; }

static int64_t gcd64(int64_t a, int64_t b) {
  while (b) {
    int64_t t = a % b;
    a = b;
    b = t;
  }
  return a;
}

static int64_t lcm64(int64_t a, int64_t b) { return a / gcd64(a, b) * b; }

/* representative of v modulo n in [0, n) */
static int64_t mod64(int64_t v, int64_t n) {
  int64_t r = v % n;
  return r < 0 ? r + n : r;
}

/* representative of v modulo n in (-n/2, n/2] */
static int64_t cmod64(int64_t v, int64_t n) {
  int64_t r = mod64(v, n);
  return r > n / 2 ? r - n : r;
}

/* ------------------------------------------------------------------------ */
/* windows.  The paper fixes only that the window is real with unit 2-norm
 * (Sec. 2.1) and uses Blackman (or Hann) windows of length gl (Sec. 6); its
 * kernel figure (Sec. 4.1) also shows a Gaussian window without giving its
 * width.  We sample the window centred at t = 0 on t = -gl/2 .. gl/2-1.
 * Gaussian (a reading): exp(-pi t^2 / (a M)), the Gaussian whose time and
 * frequency spreads match the lattice (a, M); truncated to gl samples.     */

int orc_window_ga(int32_t type, int32_t gl, int32_t a, int32_t M, double *g) {
  if (gl <= 0 || (gl & 1) || !g) return ORC_E_ARG;
  if (type == ORC_WIN_GAUSS && ((int64_t)a * M <= 0)) return ORC_E_ARG;
  double nrm = 0.0;
  for (int32_t i = 0; i < gl; ++i) {
    double t = (double)(i - gl / 2);
    double v;
    if (type == ORC_WIN_BLACKMAN)
      v = 0.42 + 0.5 * cos(2.0 * M_PI * t / gl) + 0.08 * cos(4.0 * M_PI * t / gl);
    else if (type == ORC_WIN_HANN)
      v = 0.5 + 0.5 * cos(2.0 * M_PI * t / gl);
    else if (type == ORC_WIN_GAUSS)
      v = exp(-M_PI * t * t / ((double)a * (double)M));
    else
      return ORC_E_ARG;
    g[i] = v;
    nrm += v * v;
  }
  nrm = sqrt(nrm);
  for (int32_t i = 0; i < gl; ++i) g[i] /= nrm;
  return ORC_OK;
}

int orc_window(int32_t type, int32_t gl, double *g) { return orc_window_ga(type, gl, 0, 0, g); }

/* g(t) for any integer t: zero outside [-gl/2, gl/2) */
static double win_at(const double *g, int32_t gl, int64_t t) {
  if (t < -gl / 2 || t >= gl / 2) return 0.0;
  return g[t + gl / 2];
}

/* ------------------------------------------------------------------------ */
/* grid rules.  Sec. 2.1 asks only for L to be a multiple of every a (and of
 * every M); Sec. 4.2 puts a pair of systems on the common grid with time
 * step gcd(a_w, a_v) and lcm(M_w, M_v) bins.  Readings of this
 * implementation: M is even (bins 0 .. M/2 with a Nyquist bin), gl is even
 * and gl <= 8 M (a window longer than M is folded modulo M).  Neither the
 * hops nor the numbers of channels need divide each other.                 */

int orc_check_dicts(const orc_dict *d, int32_t W) {
  if (!d || W <= 0) return ORC_E_ARG;
  for (int32_t w = 0; w < W; ++w) {
    if (d[w].window != ORC_WIN_BLACKMAN && d[w].window != ORC_WIN_HANN &&
        d[w].window != ORC_WIN_GAUSS)
      return ORC_E_ARG;
    if (d[w].a <= 0 || d[w].M <= 0 || d[w].gl <= 0) return ORC_E_ARG;
    if (d[w].M < 2 || (d[w].M & 1)) return ORC_E_GRID;
    if ((d[w].gl & 1) || d[w].gl > 8 * d[w].M) return ORC_E_GRID;
    /* Blackman or Hann of length 2: a single nonzero sample makes every atom
       real, and Eq. (dualatprod) for a pair would divide by 1 - |gamma|^2 = 0 */
    if (d[w].gl == 2 && d[w].window != ORC_WIN_GAUSS && d[w].M >= 4) return ORC_E_ARG;
  }
  return ORC_OK;
}

/* Zero-pad L to a multiple of lcm(a_w, M_w); reject lengths too short for
 * the kernels to be independent of L (shorter than gl_v + gl_w). */
int64_t orc_padded_length(const orc_dict *d, int32_t W, int64_t L) {
  int rc = orc_check_dicts(d, W);
  if (rc) return rc;
  if (L <= 0) return ORC_E_ARG;
  int64_t q = 1;
  int64_t need = 0;
  for (int32_t w = 0; w < W; ++w) {
    q = lcm64(q, d[w].a);
    q = lcm64(q, d[w].M);
    for (int32_t v = 0; v < W; ++v)
      if (d[w].gl + d[v].gl > need) need = d[w].gl + d[v].gl;
  }
  int64_t Lp = (L + q - 1) / q * q;
  if (Lp < need) return ORC_E_LEN;
  return Lp;
}

/* ------------------------------------------------------------------------ */
/* radix-2 DFT (decimation in time, bit-reversed input order)               */

int orc_fft(int32_t n, double *re, double *im, int32_t sign) {
  if (!is_pow2(n)) return ORC_E_ARG;
  for (int32_t i = 1, j = 0; i < n; ++i) {
    int32_t bit = n >> 1;
    for (; j & bit; bit >>= 1) j ^= bit;
    j ^= bit;
    if (i < j) {
      double t = re[i];
      re[i] = re[j];
      re[j] = t;
      t = im[i];
      im[i] = im[j];
      im[j] = t;
    }
  }
  for (int32_t len = 2; len <= n; len <<= 1) {
    int32_t half = len / 2;
    for (int32_t k = 0; k < half; ++k) {
      double ang = (double)sign * 2.0 * M_PI * (double)k / (double)len;
      double wr = cos(ang), wi = sin(ang);
      for (int32_t s = 0; s < n; s += len) {
        double ur = re[s + k], ui = im[s + k];
        double xr = re[s + k + half], xi = im[s + k + half];
        double vr = xr * wr - xi * wi, vi = xr * wi + xi * wr;
        re[s + k] = ur + vr;
        im[s + k] = ui + vi;
        re[s + k + half] = ur - vr;
        im[s + k + half] = ui - vi;
      }
    }
  }
  return ORC_OK;
}

/* DFT of any length: the radix-2 FFT above for powers of two, the defining
 * sum otherwise (phase index k t mod n taken exactly in integers). */
static int dft_any(int32_t n, double *re, double *im, int32_t sign) {
  if (is_pow2(n)) return orc_fft(n, re, im, sign);
  double *xr = malloc(sizeof(double) * n), *xi = malloc(sizeof(double) * n);
  if (!xr || !xi) {
    free(xr), free(xi);
    return ORC_E_NOMEM;
  }
  memcpy(xr, re, sizeof(double) * n);
  memcpy(xi, im, sizeof(double) * n);
  for (int64_t k = 0; k < n; ++k) {
    double sr = 0.0, si = 0.0;
    for (int64_t t = 0; t < n; ++t) {
      double ang = (double)sign * 2.0 * M_PI * (double)mod64(k * t, n) / (double)n;
      double c = cos(ang), sn = sin(ang);
      sr += xr[t] * c - xi[t] * sn;
      si += xr[t] * sn + xi[t] * c;
    }
    re[k] = sr;
    im[k] = si;
  }
  free(xr), free(xi);
  return ORC_OK;
}

int orc_dft(int32_t n, double *re, double *im, int32_t sign) {
  if (n < 1 || !re || !im) return ORC_E_ARG;
  return dft_any(n, re, im, sign);
}

/* ------------------------------------------------------------------------ */
/* DGT analysis rho_0 = D* x (Sec. 5): for frame n,
 *   rho(m, n) = sum_{t=-gl/2}^{gl/2-1} x(n a + t) g(t) exp(-2 pi i m t / M),
 * which is the length-M DFT of the windowed frame laid out circularly.     */

int orc_dgt(const orc_dict *d, const double *x, int64_t L, double *re,
            double *im) {
  if (orc_check_dicts(d, 1)) return ORC_E_GRID;
  if (L % d->a || L < d->gl) return ORC_E_LEN;
  const int32_t M = d->M, gl = d->gl, MR = M / 2 + 1;
  const int64_t N = L / d->a;
  double *g = malloc(sizeof(double) * gl);
  double *br = malloc(sizeof(double) * M), *bi = malloc(sizeof(double) * M);
  if (!g || !br || !bi) {
    free(g), free(br), free(bi);
    return ORC_E_NOMEM;
  }
  orc_window_ga(d->window, gl, d->a, d->M, g);
  for (int64_t n = 0; n < N; ++n) {
    memset(br, 0, sizeof(double) * M);
    memset(bi, 0, sizeof(double) * M);
    /* the windowed frame laid out circularly: t mod M (folded when gl > M) */
    for (int32_t t = -gl / 2; t < gl / 2; ++t)
      br[mod64(t, M)] += x[mod64(n * d->a + t, L)] * g[t + gl / 2];
    dft_any(M, br, bi, -1);
    for (int32_t m = 0; m < MR; ++m) {
      re[n * MR + m] = br[m];
      im[n * MR + m] = bi[m];
    }
  }
  free(g), free(br), free(bi);
  return ORC_OK;
}

int orc_dgt_direct(const orc_dict *d, const double *x, int64_t L, double *re,
                   double *im) {
  if (orc_check_dicts(d, 1)) return ORC_E_GRID;
  if (L % d->a || L < d->gl) return ORC_E_LEN;
  const int32_t M = d->M, gl = d->gl, MR = M / 2 + 1;
  const int64_t N = L / d->a;
  double *g = malloc(sizeof(double) * gl);
  if (!g) return ORC_E_NOMEM;
  orc_window_ga(d->window, gl, d->a, d->M, g);
  for (int64_t n = 0; n < N; ++n)
    for (int32_t m = 0; m < MR; ++m) {
      double sr = 0.0, si = 0.0;
      for (int32_t t = -gl / 2; t < gl / 2; ++t) {
        double v = x[mod64(n * d->a + t, L)] * g[t + gl / 2];
        double ang = -2.0 * M_PI * (double)mod64((int64_t)m * t, M) / M;
        sr += v * cos(ang);
        si += v * sin(ang);
      }
      re[n * MR + m] = sr;
      im[n * MR + m] = si;
    }
  free(g);
  return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Cross-kernels (Sec. 4.2).  For a selected atom (v, k, j) and a target atom
 * (w, m, n) put Delta = n a_w - j a_v and mu = m r_w - k r_v with
 * r = M_max / M.  Then
 *   <d^v_{k,j}, d^w_{m,n}> = h_{w,v}(mu, Delta) exp(2 pi i k Delta / M_v),
 *   h_{w,v}(mu, Delta) = sum_t g_v(t) g_w(t - Delta) exp(-2 pi i mu (t - Delta) / M_max),
 * the twisted-convolution form of Eq. (GramKern)/(hkj) on the common grid
 * (a_min, M_max), M_max = lcm(M_w, M_v).                                   */

int orc_kernel_direct(const orc_dict *dw, const orc_dict *dv, int64_t mu,
                      int64_t Delta, double *re, double *im) {
  const int32_t Mmax = (int32_t)lcm64(dw->M, dv->M);
  double *gw = malloc(sizeof(double) * dw->gl);
  double *gv = malloc(sizeof(double) * dv->gl);
  if (!gw || !gv) {
    free(gw), free(gv);
    return ORC_E_NOMEM;
  }
  orc_window_ga(dw->window, dw->gl, dw->a, dw->M, gw);
  orc_window_ga(dv->window, dv->gl, dv->a, dv->M, gv);
  double sr = 0.0, si = 0.0;
  for (int64_t t = -dv->gl / 2; t < dv->gl / 2; ++t) {
    double p = win_at(gv, dv->gl, t) * win_at(gw, dw->gl, t - Delta);
    if (p == 0.0) continue;
    double ang = -2.0 * M_PI * (double)mod64(mu * (t - Delta), Mmax) / Mmax;
    sr += p * cos(ang);
    si += p * sin(ang);
  }
  *re = sr;
  *im = si;
  free(gw), free(gv);
  return ORC_OK;
}

/* Table of h_{w,v} for every Delta = delta * a_min whose window supports can
 * overlap (|Delta| < (gl_v + gl_w)/2) and every mu in 0..M_max-1, computed
 * column by column as the length-M_max DFT of s -> g_v(s + Delta) g_w(s),
 * then hard thresholded entry by entry as in Eq. (truncgram).              */
int orc_kernel_table(const orc_dict *dw, const orc_dict *dv, double eps,
                     uint32_t flags, int32_t *D_out, double *re, double *im,
                     int32_t *box_mu, int32_t *box_delta) {
  /* common grid (Sec. 4.2): time step gcd(a_w, a_v), lcm(M_w, M_v) bins */
  const int32_t amin = (int32_t)gcd64(dw->a, dv->a);
  const int32_t Mmax = (int32_t)lcm64(dw->M, dv->M);
  const int32_t halfsum = (dw->gl + dv->gl) / 2;
  /* largest delta with |delta * amin| < halfsum */
  const int32_t D = (halfsum + amin - 1) / amin - 1;
  if (D_out) *D_out = D;
  if (!re || !im) return ORC_OK;
  double *gw = malloc(sizeof(double) * dw->gl);
  double *gv = malloc(sizeof(double) * dv->gl);
  if (!gw || !gv) {
    free(gw), free(gv);
    return ORC_E_NOMEM;
  }
  orc_window_ga(dw->window, dw->gl, dw->a, dw->M, gw);
  orc_window_ga(dv->window, dv->gl, dv->a, dv->M, gv);
  const int64_t ncol = 2 * (int64_t)D + 1;
  for (int64_t c = 0; c < ncol; ++c) {
    int64_t Delta = (c - D) * amin;
    double *cr = re + c * Mmax, *ci = im + c * Mmax;
    memset(cr, 0, sizeof(double) * Mmax);
    memset(ci, 0, sizeof(double) * Mmax);
    for (int64_t s = -dw->gl / 2; s < dw->gl / 2; ++s)
      cr[mod64(s, Mmax)] += win_at(gv, dv->gl, s + Delta) * win_at(gw, dw->gl, s);
    dft_any(Mmax, cr, ci, -1);
  }
  double thr = eps;
  if (flags & ORC_THR_REL) {
    double pk = 0.0;
    for (int64_t i = 0; i < ncol * Mmax; ++i) {
      double a = sqrt(re[i] * re[i] + im[i] * im[i]);
      if (a > pk) pk = a;
    }
    thr = eps * pk;
  }
  int32_t bm = -1, bd = -1;
  for (int64_t c = 0; c < ncol; ++c)
    for (int64_t mu = 0; mu < Mmax; ++mu) {
      int64_t i = c * Mmax + mu;
      double a = sqrt(re[i] * re[i] + im[i] * im[i]);
      if (a > thr) {
        int32_t amu = (int32_t)llabs(cmod64(mu, Mmax));
        int32_t ad = (int32_t)llabs(c - D);
        if (amu > bm) bm = amu;
        if (ad > bd) bd = ad;
      } else {
        re[i] = 0.0;
        im[i] = 0.0;
      }
    }
  if (flags & ORC_KEEP_BOX) {
    /* reading of the kernel figure's "fixed size and shape": keep every entry
     * of the survivors' bounding box, sub-threshold ones included */
    for (int64_t c = 0; c < ncol; ++c) {
      if (llabs(c - D) > bd) continue;
      int64_t Delta = (c - D) * amin;
      double *cr = re + c * Mmax, *ci = im + c * Mmax;
      memset(cr, 0, sizeof(double) * Mmax);
      memset(ci, 0, sizeof(double) * Mmax);
      for (int64_t s = -dw->gl / 2; s < dw->gl / 2; ++s)
        cr[mod64(s, Mmax)] += win_at(gv, dv->gl, s + Delta) * win_at(gw, dw->gl, s);
      dft_any(Mmax, cr, ci, -1);
      for (int64_t mu = 0; mu < Mmax; ++mu)
        if (llabs(cmod64(mu, Mmax)) > bm) cr[mu] = ci[mu] = 0.0;
    }
  }
  if (box_mu) *box_mu = bm;
  if (box_delta) *box_delta = bd;
  free(gw), free(gv);
  return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* approximate coefficient-domain MP (Eq. (approxResDef) with the real-atom
 * pairs of Sec. 5 and the cross-kernel update of Alg. 3)                   */

typedef struct {
  int32_t D, Mmax, amin;
  double *re, *im;
} pair_table;

typedef struct {
  int64_t N;
  int32_t MR;
  int64_t off; /* global index of (m = 0, n = 0) */
  double *re, *im;
  double *fbest, *fsecond; /* per-frame top-2 of the selection score */
  int32_t *farg;           /* bin of the per-frame maximum */
  /* pedantic selection: gamma(m) = <d, conj d> of bin m (0 at DC and Nyquist) */
  const double *gre, *gim;
} plane;

/* Energy removed by projecting onto the real atom pair of coefficient rho
 * with gamma = <d, conj d>, Eq. (projenfaster) with the adjusted coefficient
 * of Eq. (dualatprod). */
static double pair_energy(double rr, double ri, double gr, double gi) {
  double nr = rr - (gr * rr - gi * ri);
  double ni = ri - (-gr * ri - gi * rr);
  double den = 1.0 - (gr * gr + gi * gi);
  double cr = nr / den, ci = ni / den;
  return 2.0 * (cr * cr + ci * ci + gr * (cr * cr - ci * ci) - 2.0 * gi * cr * ci);
}

/* Selection score of bin m: |rho|^2, or with pedantic selection the energy
 * of the projection onto the pair (|rho|^2 at DC and Nyquist, which have no
 * partner). */
static double score(const plane *P, int32_t m, double r, double i) {
  if (!P->gre || m == 0 || m == P->MR - 1) return r * r + i * i;
  return pair_energy(r, i, P->gre[m], P->gim[m]);
}

static void frame_top2(plane *P, int64_t n) {
  double b = -1.0, s = -1.0;
  int32_t arg = 0;
  for (int32_t m = 0; m < P->MR; ++m) {
    double r = P->re[n * P->MR + m], i = P->im[n * P->MR + m];
    double v = score(P, m, r, i);
    if (v > b) {
      s = b;
      b = v;
      arg = m;
    } else if (v > s) {
      s = v;
    }
  }
  P->fbest[n] = b;
  P->fsecond[n] = s;
  P->farg[n] = arg;
}

/* The loop of orc_mp.  With n_forced >= 0 the selections are not taken
 * from the maximum but from fw / fm / fn (replay of another run): K =
 * n_forced, no other stop rule, and best / chosen receive the largest score
 * and the score of the replayed atom at each step. */
static int mp_core(const orc_dict *d, int32_t W, const double *x, int64_t L,
                   double eps, uint32_t flags, int64_t K, double target_db,
                   int64_t cap, int32_t *aw, int32_t *am, int32_t *an,
                   double *cre, double *cim, double *E_after, double *gap,
                   double *best_sel, double *final_re, double *final_im,
                   orc_stats *st, int64_t n_forced, const int32_t *fw,
                   const int32_t *fm, const int32_t *fn, double *best_out,
                   double *chosen_out) {
  int rc = ORC_OK;
  if (!st || !x || eps < 0.0) return ORC_E_ARG;
  memset(st, 0, sizeof(*st));
  int64_t Lp = orc_padded_length(d, W, L);
  if (Lp < 0) return (int)Lp;
  st->L_padded = Lp;
  if (K <= 0) K = Lp / 5;
  if (n_forced >= 0) {
    K = n_forced;
    target_db = 0.0;
  }
  if (K > cap) K = cap;

  double *xp = calloc((size_t)Lp, sizeof(double));
  plane *P = calloc((size_t)W, sizeof(plane));
  pair_table *T = calloc((size_t)W * W, sizeof(pair_table));
  if (!xp || !P || !T) {
    rc = ORC_E_NOMEM;
    goto done;
  }
  memcpy(xp, x, sizeof(double) * (size_t)L);

  /* E_0 = ||x||^2 (Alg. 1 initialisation) */
  double E0 = 0.0;
  for (int64_t l = 0; l < Lp; ++l) E0 += xp[l] * xp[l];
  st->E0 = E0;

  /* kernels for every ordered pair (target w, source v) */
  for (int32_t w = 0; w < W; ++w)
    for (int32_t v = 0; v < W; ++v) {
      pair_table *t = &T[w * W + v];
      t->amin = (int32_t)gcd64(d[w].a, d[v].a);
      t->Mmax = (int32_t)lcm64(d[w].M, d[v].M);
      orc_kernel_table(&d[w], &d[v], eps, flags, &t->D, NULL, NULL, NULL, NULL);
      size_t n = (size_t)(2 * t->D + 1) * (size_t)t->Mmax;
      t->re = malloc(sizeof(double) * n);
      t->im = malloc(sizeof(double) * n);
      if (!t->re || !t->im) {
        rc = ORC_E_NOMEM;
        goto done;
      }
      orc_kernel_table(&d[w], &d[v], eps, flags, &t->D, t->re, t->im, NULL,
                       NULL);
    }

  /* rho_0 = D* x for every system, and per-frame maxima (Sec. 5.1) */
  int64_t off = 0;
  for (int32_t w = 0; w < W; ++w) {
    plane *p = &P[w];
    p->N = Lp / d[w].a;
    p->MR = d[w].M / 2 + 1;
    p->off = off;
    off += p->N * p->MR;
    p->re = malloc(sizeof(double) * (size_t)(p->N * p->MR));
    p->im = malloc(sizeof(double) * (size_t)(p->N * p->MR));
    p->fbest = malloc(sizeof(double) * (size_t)p->N);
    p->fsecond = malloc(sizeof(double) * (size_t)p->N);
    p->farg = malloc(sizeof(int32_t) * (size_t)p->N);
    if (!p->re || !p->im || !p->fbest || !p->fsecond || !p->farg) {
      rc = ORC_E_NOMEM;
      goto done;
    }
    orc_dgt(&d[w], xp, Lp, p->re, p->im);
    p->gre = p->gim = NULL;
    if (flags & ORC_PEDANTIC) {
      /* gamma(m) = h_{w,w}(-2m mod M_w, 0) of the truncated auto kernel */
      double *gr = calloc((size_t)p->MR, sizeof(double)), *gi = calloc((size_t)p->MR, sizeof(double));
      if (!gr || !gi) {
        free(gr), free(gi);
        rc = ORC_E_NOMEM;
        goto done;
      }
      pair_table *tw = &T[w * W + w];
      for (int32_t m = 1; m + 1 < p->MR; ++m) {
        int64_t mu = mod64(-2 * (int64_t)m, tw->Mmax);
        gr[m] = tw->re[(int64_t)tw->D * tw->Mmax + mu];
        gi[m] = tw->im[(int64_t)tw->D * tw->Mmax + mu];
      }
      p->gre = gr;
      p->gim = gi;
    }
    for (int64_t n = 0; n < p->N; ++n) frame_top2(p, n);
  }

  const double Etarget = target_db > 0.0 ? E0 * pow(10.0, -target_db / 10.0)
                                         : -INFINITY;
  double E = E0;
  int64_t k = 0;
  int32_t reason = 0;
  for (;;) {
    /* stopping criteria (Alg. 1; the error-estimate rule of Sec. 6.1) */
    if (k >= K) {
      reason = ORC_STOP_K;
      break;
    }
    if (E <= Etarget) {
      reason = ORC_STOP_SNR;
      break;
    }
    if (E < 0.0 && n_forced < 0) {
      reason = ORC_STOP_ENEG;
      break;
    }
    /* selection: global maximum of the score (|rho|^2, or the pair
     * projection energy with pedantic selection), lowest global index on ties.
     * Frames are visited in increasing global index, so a strict '>' keeps
     * the first (lowest-index) maximum. */
    double best = -1.0, second = -1.0;
    int32_t v = -1, kk = 0;
    int64_t j = 0;
    for (int32_t w = 0; w < W; ++w)
      for (int64_t n = 0; n < P[w].N; ++n) {
        double fb = P[w].fbest[n], fs = P[w].fsecond[n];
        if (fb > best) {
          second = best > fs ? best : fs;
          best = fb;
          v = w;
          j = n;
          kk = P[w].farg[n];
        } else if (fb > second) {
          second = fb;
        }
      }
    if (n_forced >= 0) {
      /* replay: the k-th selection of the other run */
      v = fw[k];
      if (v < 0 || v >= W || fm[k] < 0 || fm[k] >= P[v].MR || fn[k] < 0 || fn[k] >= P[v].N) {
        rc = ORC_E_ARG;
        goto done;
      }
      kk = fm[k];
      j = fn[k];
      best_out[k] = best;
      chosen_out[k] = score(&P[v], kk, P[v].re[j * P[v].MR + kk], P[v].im[j * P[v].MR + kk]);
    } else if (!(best > 0.0)) {
      reason = ORC_STOP_ZERO;
      break;
    }
    plane *Pv = &P[v];
    const int32_t Mv = d[v].M;
    const double rr = Pv->re[j * Pv->MR + kk], ri = Pv->im[j * Pv->MR + kk];

    /* coefficient adjustment for the real atom pair, Eq. (dualatprod), and
     * energy decrease, Eq. (projenfaster).  gamma = <d, conj d> is the
     * auto-kernel entry at mu = -2k, Delta = 0.  DC and Nyquist atoms are
     * real and have no partner. */
    const int pair = (kk != 0 && 2 * kk != Mv);
    double cr, ci, Et, gr = 0.0, gi = 0.0;
    if (pair) {
      pair_table *tv = &T[v * W + v];
      int64_t mu = mod64(-2 * (int64_t)kk, tv->Mmax);
      gr = tv->re[(int64_t)tv->D * tv->Mmax + mu];
      gi = tv->im[(int64_t)tv->D * tv->Mmax + mu];
      /* c = (rho - conj(gamma) conj(rho)) / (1 - |gamma|^2) */
      double nr = rr - (gr * rr - gi * ri);  /* Re(conj(g) conj(r)) = gr rr - gi ri */
      double ni = ri - (-gr * ri - gi * rr); /* Im(conj(g) conj(r)) = -gr ri - gi rr */
      double den = 1.0 - (gr * gr + gi * gi);
      cr = nr / den;
      ci = ni / den;
      Et = 2.0 * (cr * cr + ci * ci + gr * (cr * cr - ci * ci) - 2.0 * gi * cr * ci);
    } else {
      cr = rr;
      ci = ri;
      Et = cr * cr + ci * ci;
    }
    E -= Et;
    aw[k] = v;
    am[k] = kk;
    an[k] = (int32_t)j;
    cre[k] = cr;
    cim[k] = ci;
    E_after[k] = E;
    gap[k] = best > 0.0 ? (best - (second > 0.0 ? second : 0.0)) / best : 0.0;
    if (best_sel) best_sel[k] = best;
    ++k;

    /* residual update (Alg. 3): for every target system w and every target
     * coefficient whose frame lies within the kernel's time extent,
     *   rho -= c G_eps(., (v,k,j)) + [pair] conj(c) G_eps(., (v, M_v - k, j)),
     * with G_eps(., (v,k,j)) = h_{w,v}(mu, Delta) exp(2 pi i k Delta / M_v). */
    const int apply_partner = pair && (!(flags & ORC_CONJ_GATE_GAMMA) ||
                                       (gr != 0.0 || gi != 0.0));
    for (int32_t w = 0; w < W; ++w) {
      pair_table *t = &T[w * W + v];
      plane *Pw = &P[w];
      const int64_t rw = t->Mmax / d[w].M, rv = t->Mmax / Mv;
      for (int64_t n = 0; n < Pw->N; ++n) {
        int64_t Delta = cmod64(n * d[w].a - j * d[v].a, Lp);
        if (Delta > (int64_t)t->D * t->amin || Delta < -(int64_t)t->D * t->amin)
          continue;
        int64_t col = Delta / t->amin + t->D;
        double ang = 2.0 * M_PI * (double)mod64((int64_t)kk * Delta, Mv) / Mv;
        double pr = cos(ang), pi = sin(ang);
        const double *hr = t->re + col * t->Mmax, *hi = t->im + col * t->Mmax;
        for (int32_t m = 0; m < Pw->MR; ++m) {
          int64_t mu1 = mod64(m * rw - kk * rv, t->Mmax);
          /* c * h1 * phase */
          double ar = hr[mu1] * pr - hi[mu1] * pi, ai = hr[mu1] * pi + hi[mu1] * pr;
          double ur = cr * ar - ci * ai, ui = cr * ai + ci * ar;
          if (apply_partner) {
            int64_t mu2 = mod64(m * rw + kk * rv, t->Mmax);
            /* conj(c) * h2 * conj(phase) */
            double br = hr[mu2] * pr + hi[mu2] * pi, bi = hi[mu2] * pr - hr[mu2] * pi;
            ur += cr * br + ci * bi;
            ui += cr * bi - ci * br;
          }
          Pw->re[n * Pw->MR + m] -= ur;
          Pw->im[n * Pw->MR + m] -= ui;
        }
        frame_top2(Pw, n);
      }
    }
  }
  st->n_atoms = k;
  st->stop_reason = reason;
  st->E_final = E;

  if (final_re && final_im)
    for (int32_t w = 0; w < W; ++w) {
      memcpy(final_re + P[w].off, P[w].re, sizeof(double) * (size_t)(P[w].N * P[w].MR));
      memcpy(final_im + P[w].off, P[w].im, sizeof(double) * (size_t)(P[w].N * P[w].MR));
    }

done:
  if (P)
    for (int32_t w = 0; w < W; ++w) {
      free(P[w].re), free(P[w].im), free(P[w].fbest), free(P[w].fsecond);
      free(P[w].farg);
      free((void *)P[w].gre), free((void *)P[w].gim);
    }
  if (T)
    for (int32_t i = 0; i < W * W; ++i) free(T[i].re), free(T[i].im);
  free(P), free(T), free(xp);
  return rc;
}

int orc_mp(const orc_dict *d, int32_t W, const double *x, int64_t L,
           double eps, uint32_t flags, int64_t K, double target_db,
           int64_t cap, int32_t *aw, int32_t *am, int32_t *an, double *cre,
           double *cim, double *E_after, double *gap, double *best,
           double *final_re, double *final_im, orc_stats *st) {
  return mp_core(d, W, x, L, eps, flags, K, target_db, cap, aw, am, an, cre, cim,
                 E_after, gap, best, final_re, final_im, st, -1, NULL, NULL, NULL,
                 NULL, NULL);
}

int orc_mp_replay(const orc_dict *d, int32_t W, const double *x, int64_t L,
                  double eps, uint32_t flags, int64_t n, const int32_t *fw,
                  const int32_t *fm, const int32_t *fn, double *cre,
                  double *cim, double *E_after, double *gap, double *best,
                  double *chosen, double *final_re, double *final_im,
                  orc_stats *st) {
  if (n < 0 || (n > 0 && (!fw || !fm || !fn || !cre || !cim || !E_after || !gap ||
                          !best || !chosen)))
    return ORC_E_ARG;
  int32_t *aw = malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
  int32_t *am = malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
  int32_t *an = malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
  int rc = ORC_E_NOMEM;
  if (aw && am && an)
    rc = mp_core(d, W, x, L, eps, flags, n, 0.0, n > 0 ? n : 1, aw, am, an, cre, cim,
                 E_after, gap, NULL, final_re, final_im, st, n, fw, fm, fn, best, chosen);
  free(aw), free(am), free(an);
  return rc;
}

/* ------------------------------------------------------------------------ */
/* synthesis of real atoms, Eq. (idgtreal): each pair contributes
 * c d + conj(c) conj(d) = 2 Re(c d); a DC or Nyquist atom contributes Re(c d). */

int orc_resynth(const orc_dict *d, int32_t W, int64_t Lp, int64_t n_atoms,
                const int32_t *aw, const int32_t *am, const int32_t *an,
                const double *cre, const double *cim, double *y) {
  if (orc_check_dicts(d, W)) return ORC_E_GRID;
  double **g = calloc((size_t)W, sizeof(double *));
  if (!g) return ORC_E_NOMEM;
  for (int32_t w = 0; w < W; ++w) {
    g[w] = malloc(sizeof(double) * d[w].gl);
    if (!g[w]) {
      for (int32_t u = 0; u < w; ++u) free(g[u]);
      free(g);
      return ORC_E_NOMEM;
    }
    orc_window_ga(d[w].window, d[w].gl, d[w].a, d[w].M, g[w]);
  }
  memset(y, 0, sizeof(double) * (size_t)Lp);
  for (int64_t i = 0; i < n_atoms; ++i) {
    const orc_dict *dv = &d[aw[i]];
    const int32_t gl = dv->gl, M = dv->M, k = am[i];
    const double mult = (k != 0 && 2 * k != M) ? 2.0 : 1.0;
    for (int32_t t = -gl / 2; t < gl / 2; ++t) {
      double ang = 2.0 * M_PI * (double)mod64((int64_t)k * t, M) / M;
      double re = g[aw[i]][t + gl / 2] * (cre[i] * cos(ang) - cim[i] * sin(ang));
      y[mod64((int64_t)an[i] * dv->a + t, Lp)] += mult * re;
    }
  }
  for (int32_t w = 0; w < W; ++w) free(g[w]);
  free(g);
  return ORC_OK;
}
