/*
 * Plain FP64 CPU oracle for approximate coefficient-domain matching pursuit
 * (MP) on multi-Gabor dictionaries (Prusa, Holighaus, Balazs, "Fast Matching
 * Pursuit with Multi-Gabor Dictionaries", ACM TOMS 47(3), 2021).
 *
 * TEST INFRASTRUCTURE ONLY.  This code exists to check the GPU library.  Only
 * the test suite, the smoke check and the benchmark's CPU-baseline leg may
 * load it.  It shares no code, header, table or helper with the GPU path.
 *
 * Everything is double precision, single threaded, written for readability
 * rather than speed.  Each function names the passage of the paper it follows.
 */
#ifndef MP_ORACLE_H
#define MP_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* window shapes */
#define ORC_WIN_BLACKMAN 0
#define ORC_WIN_HANN 1
#define ORC_WIN_GAUSS 2 /* exp(-pi t^2 / (a M)), a reading: see orc_window_ga */

/* flags for orc_mp */
#define ORC_THR_REL 1u         /* threshold relative to each kernel's peak   */
#define ORC_CONJ_GATE_GAMMA 2u /* conjugate-partner update only if gamma!=0  */
#define ORC_PEDANTIC 4u        /* select by the pair projection energy       */
#define ORC_KEEP_BOX 8u        /* keep the survivors' whole bounding box     */

/* return codes */
#define ORC_OK 0
#define ORC_E_ARG (-1)
#define ORC_E_GRID (-2)
#define ORC_E_LEN (-3)
#define ORC_E_NOMEM (-4)

/* stop reasons */
#define ORC_STOP_K 1
#define ORC_STOP_SNR 2
#define ORC_STOP_ENEG 3
#define ORC_STOP_ZERO 4

typedef struct {
  int32_t window, gl, a, M;
} orc_dict;

typedef struct {
  int64_t n_atoms;
  int32_t stop_reason;
  int32_t pad_;
  int64_t L_padded;
  double E0;
  double E_final;
} orc_stats;

/* Unit-norm window sampled at t = -gl/2 .. gl/2-1; g[i] holds t = i - gl/2. */
int orc_window(int32_t type, int32_t gl, double *g);
/* as orc_window; the Gaussian's width depends on the lattice (a, M) */
int orc_window_ga(int32_t type, int32_t gl, int32_t a, int32_t M, double *g);

/* Grid validation (M even, gl even and gl <= 8 M) and padded length. */
int orc_check_dicts(const orc_dict *d, int32_t W);
int64_t orc_padded_length(const orc_dict *d, int32_t W, int64_t L);

/* In-place radix-2 DFT, X(k) = sum_t x(t) exp(-2 pi i k t / n)
 * (sign = -1) or the unnormalised inverse (sign = +1). n a power of two. */
int orc_fft(int32_t n, double *re, double *im, int32_t sign);
/* The same transform for any n >= 1: orc_fft for powers of two, the defining
 * sum otherwise. */
int orc_dft(int32_t n, double *re, double *im, int32_t sign);

/* DGT of a real signal in one Gabor system, reduced to m = 0..M/2.
 * Output planes are N x (M/2+1), m fastest.  L must be a multiple of a. */
int orc_dgt(const orc_dict *d, const double *x, int64_t L, double *re,
            double *im);
/* Same quantity by direct summation (for pinning orc_dgt). */
int orc_dgt_direct(const orc_dict *d, const double *x, int64_t L, double *re,
                   double *im);

/* Cross-kernel entry by direct summation:
 * h_{w,v}(mu, Delta) = sum_t g_v(t) g_w(t - Delta) exp(-2 pi i mu (t-Delta)/Mmax)
 * with Mmax = lcm(M_w, M_v).  dw = target system, dv = source system. */
int orc_kernel_direct(const orc_dict *dw, const orc_dict *dv, int64_t mu,
                      int64_t Delta, double *re, double *im);

/* Truncated cross-kernel table for the pair (target w, source v), on the
 * common grid (a_min, M_max): entries for delta = -D..D (Delta = delta*a_min)
 * and mu = 0..M_max-1, stored [(delta + D) * M_max + mu].  Entries with
 * |h| <= thr are set to zero (thr = eps, or eps * max|h| with ORC_THR_REL).
 * *D_out receives D; pass re = im = NULL to query D only.  box_mu / box_delta
 * (may be NULL) receive the half extents of the bounding box of survivors. */
int orc_kernel_table(const orc_dict *dw, const orc_dict *dv, double eps,
                     uint32_t flags, int32_t *D_out, double *re, double *im,
                     int32_t *box_mu, int32_t *box_delta);

/* Approximate coefficient-domain MP with real-atom pairs.
 * x has L samples; it is zero-padded to orc_padded_length.
 * K <= 0 selects the default L/5; target_db <= 0 disables the SNR stop.
 * Per selected atom: dictionary, bin, frame, adjusted coefficient c~,
 * error estimate after the step, the relative top-2 gap of the selection
 * score at selection and (best, may be NULL) the selected score itself.
 * final_re / final_im (may be NULL) receive the residual planes
 * concatenated over the dictionaries. */
int orc_mp(const orc_dict *d, int32_t W, const double *x, int64_t L,
           double eps, uint32_t flags, int64_t K, double target_db,
           int64_t cap, int32_t *aw, int32_t *am, int32_t *an, double *cre,
           double *cim, double *E_after, double *gap, double *best,
           double *final_re, double *final_im, orc_stats *st);

/* Replay: the loop of orc_mp with the selections taken from fw / fm / fn
 * (n of them, e.g. another implementation's run) instead of the maximum.
 * Every other step is orc_mp's, in its order, on the oracle's own
 * coefficients.  Per step: adjusted coefficient c~ of the replayed atom,
 * error estimate after it, top-2 gap, best = largest selection score and
 * chosen = score of the replayed atom before the step.  No stop rule other
 * than n.  ORC_E_ARG if a replayed atom lies outside its system's grid. */
int orc_mp_replay(const orc_dict *d, int32_t W, const double *x, int64_t L,
                  double eps, uint32_t flags, int64_t n, const int32_t *fw,
                  const int32_t *fm, const int32_t *fn, double *cre,
                  double *cim, double *E_after, double *gap, double *best,
                  double *chosen, double *final_re, double *final_im,
                  orc_stats *st);

/* Signal-domain synthesis of a list of real atoms into y (length Lp). */
int orc_resynth(const orc_dict *d, int32_t W, int64_t Lp, int64_t n_atoms,
                const int32_t *aw, const int32_t *am, const int32_t *an,
                const double *cre, const double *cim, double *y);

#ifdef __cplusplus
}
#endif
#endif
