/*
 * mpg.h - C-ABI of the MI355X matching-pursuit library (libmpg.so).
 *
 * The library computes approximate coefficient-domain matching pursuit (MP)
 * on multi-Gabor dictionaries for batches of real signals, after
 * Prusa, Holighaus, Balazs, "Fast Matching Pursuit with Multi-Gabor
 * Dictionaries", ACM TOMS 47(3), 2021:
 *   - DGT analysis rho_0 = D* x in every Gabor system (Sec. 5);
 *   - per iteration: the global maximum of |rho|^2 (or, with MP_PEDANTIC,
 *     of the real-atom pair projection energy, Sec. 5) taken from a max tree
 *     (Sec. 5.1), the real-atom pair adjustment (Sec. 5, Eqs. dualatprod and
 *     projenfaster), and the residual update by truncated, modulated
 *     cross-kernels (Sec. 4, Eqs. GramKern, hkj, fastkernupdate; Alg. 3);
 *   - the reset procedure (Alg. 2): approximate MP in rounds, each started
 *     from the analysis of the true residual (mp_run_resets);
 *   - synthesis of the selected atoms (Sec. 5, Eq. idgtreal).
 * Systems may use Blackman, Hann or Gaussian windows (windows longer than M
 * are folded), any even M (the analysis of an M that is not a power of two
 * runs the defining sum of the DFT), and hops that neither nest nor divide M:
 * each pair of systems lives on the common grid gcd(a_w, a_v) x
 * lcm(M_w, M_v) (Sec. 4.2).
 *
 * Conventions.
 *   - Every function returns 0 (MP_OK) or a negative MP_E_* code and never
 *     throws.  On error the plan is left unchanged.
 *   - "_dev" pointers are device pointers owned by the caller; "_host"
 *     pointers are host memory owned by the caller.  The plan owns every
 *     buffer it allocates and frees them in mp_plan_destroy.
 *   - Calls taking a hipStream_t only enqueue work on that stream (they may
 *     block only in mp_plan_create).  mp_get_atoms, mp_get_energy and
 *     mp_get_stats wait for the stream of the last mp_run on the plan.
 *   - Calls on one plan must not overlap; different plans are independent.
 *   - Signal s of a batch is identified by its index 0 .. batch-1.
 *   - Coefficient planes are laid out N_w x (M_w/2 + 1), bin m fastest
 *     (c(m, n) = c[n * (M_w/2 + 1) + m]), interleaved complex.
 */
#ifndef MPG_H
#define MPG_H

#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- return codes ---- */
#define MP_OK 0
#define MP_E_ARG (-1)   /* invalid argument (null pointer, bad size, bad index) */
#define MP_E_GRID (-2)  /* unsupported Gabor system: M odd, gl odd or gl > 8 M, or a
                           split DFT (MP_DFT_*SPLIT) with M not a power of two.
                           Neither the hops nor the M need divide each other:
                           every pair lives on its common grid gcd(a_w, a_v) x
                           lcm(M_w, M_v) (Sec. 2.1, Sec. 4.2)                      */
#define MP_E_LEN (-3)   /* a padded length is shorter than gl_v + gl_w of some pair  */
#define MP_E_NOMEM (-4) /* device or host allocation failed                         */
#define MP_E_HIP (-5)   /* a HIP runtime call failed                                */
#define MP_E_STATE (-6) /* call out of order (e.g. mp_run before mp_analyze)        */
#define MP_E_LIMIT (-7) /* a size exceeds a limit of this implementation            */

/* ---- windows ---- */
#define MP_WIN_BLACKMAN 0
#define MP_WIN_HANN 1
#define MP_WIN_GAUSS 2 /* exp(-pi t^2 / (a M)): spreads matched to the lattice (a, M) */

/* ---- plan flags ---- */
#define MP_PREC_F32 0x0u         /* FP32 planes, kernels and updates (default)      */
#define MP_PREC_F64 0x1u         /* FP64 planes, kernels and updates               */
#define MP_THR_REL 0x10u         /* threshold relative to each kernel's peak |h|   */
#define MP_CONJ_GATE_GAMMA 0x20u /* conjugate-partner update only when gamma != 0  */
/* DFT inside the analysis (FP32 plans only; at most one; default MP_DFT_F32,
 * the FFT in FP32).  MP_DFT_F64 runs the window products and the FFT in FP64
 * and rounds the coefficients to the plan's FP32 (systems need M <= 16384).
 * The split variants run the DFT on matrix cores as a four-step transform
 * with each operand a pair of half-precision numbers (hi + lo; products
 * hi*hi + hi*lo + lo*hi accumulated in FP32; for M = 256 .. 4096 the lo half
 * holds the remainder scaled by 2^11, which keeps FP16 pairs as accurate as
 * the FP32 FFT); systems need M a power of two, M <= 16384. */
#define MP_DFT_F32 0x0u          /* FFT in FP32 (default)                           */
#define MP_DFT_F64 0x200u        /* FFT in FP64, coefficients rounded to FP32        */
#define MP_DFT_F16SPLIT 0x40u    /* FP16 pairs                                      */
#define MP_DFT_BF16SPLIT 0x80u   /* BF16 pairs                                      */
/* Pedantic selection (Sec. 5): choose the atom whose real-pair projection
 * removes the most energy (Eq. projenfaster with the adjusted coefficient of
 * Eq. dualatprod) instead of the largest |rho|^2; DC and Nyquist atoms, which
 * have no partner, score |rho|^2. */
#define MP_PEDANTIC 0x100u
/* Schedule of the FP32 MP kernel (FP32 plans only).  Default: 768 threads
 * (12 waves) per signal, 256-leaf tree groups, 16-row tiles, each falling
 * back when the tree groups would not fit the LDS.  The tile is the unit of
 * the neighbourhood split: the 16-bin rows an update touches (its kernel
 * neighbourhood in every target system) go to the waves from a counter, a
 * tile per grab.  The results do not depend on the schedule; mp_autotune
 * picks one by timing. */
#define MP_SCHED_NT512 0x1000u   /* 512 threads (8 waves) per signal            */
#define MP_SCHED_G128 0x2000u    /* 128-leaf tree groups                        */
#define MP_SCHED_TILE8 0x4000u   /* 8-row tiles                                 */
#define MP_SCHED_TILE32 0x8000u  /* 32-row tiles (with MP_SCHED_NT512 only)     */

/* ---- input sample types for mp_analyze / output types for mp_resynth ---- */
#define MP_DTYPE_F32 0
#define MP_DTYPE_F64 1

/* ---- stop reasons (mp_signal_info.stop_reason) ---- */
#define MP_STOP_NONE 0 /* not run yet                                  */
#define MP_STOP_K 1    /* selection cap reached                        */
#define MP_STOP_SNR 2  /* error estimate reached the target            */
#define MP_STOP_ENEG 3 /* error estimate became negative (Sec. 6.1)    */
#define MP_STOP_ZERO 4 /* all coefficients are zero                    */

typedef struct mp_plan mp_plan;

/* One Gabor system (g, a, M): window shape, window length gl, hop a and
 * number of channels M (Sec. 2.1, Eq. gabdict).  gl is even; a window longer
 * than M (up to 8 M) is folded modulo M in the analysis. */
typedef struct {
  int32_t window, gl, a, M;
} mp_dict;

/* One selected real atom: system w, bin m (0..M_w/2), frame n, the adjusted
 * coefficient c~ of Eq. (dualatprod), and the error estimate E_k after the
 * selection (Alg. 1, error update, with Eq. projenfaster). */
typedef struct {
  int32_t w, m, n, pad;
  double re, im;
  double E_after;
} mp_atom;

typedef struct {
  int64_t L;           /* length given at plan creation                       */
  int64_t L_padded;    /* zero-padded length (multiple of lcm(a_w, M_w))       */
  int64_t x_offset;    /* element offset of this signal in the packed input   */
  int64_t n_coefs;     /* sum_w N_w (M_w/2 + 1)                                */
  int64_t n_atoms;     /* selections made so far                              */
  int32_t stop_reason; /* MP_STOP_*                                           */
  int32_t pad;
  double E0;           /* ||x||^2                                             */
  double E;            /* current error estimate                              */
} mp_signal_info;

typedef struct {
  int32_t amin, Mmax;     /* common grid of the pair (Sec. 4.2)              */
  int32_t D;              /* largest |delta| whose supports overlap         */
  int32_t delta_box;      /* half extent in delta of the surviving entries  */
  int32_t mu_lo, mu_hi;   /* extent in mu of the surviving entries          */
  int64_t n_nonzero;      /* surviving entries |h| > threshold              */
} mp_kernel_info;

typedef struct {
  int64_t atoms;          /* selections in the last mp_run, over the batch  */
  int64_t updated;        /* coefficient updates with a nonzero kernel entry */
  int64_t blocks;         /* max-tree leaves (16 bins of a frame) rewritten  */
  int64_t l1_groups;      /* tree groups recomputed                          */
  double loop_ms;         /* device time of the last mp_run's MP kernel     */
  double analyze_ms;      /* device time of the last mp_analyze             */
  double dgt_ms;          /* device time of the DGT kernels in it           */
  int32_t group_leaves;   /* leaves per tree group of the plan              */
  int32_t threads;        /* threads per workgroup of the MP kernel         */
  int32_t tile_rows;      /* rows per tile of the neighbourhood split       */
  int32_t early_groups;   /* 1: the FP32 loop loads the touched tree groups
                           * beyond the preloaded ones (two per wave) before
                           * merging, for plans whose selections can touch
                           * more of them; 0 otherwise (and for FP64 plans) */
} mp_stats;

/* Creates a plan for `batch` signals of lengths L[0..batch-1] and the W
 * Gabor systems dicts[0..W-1].  Validates the grids (Sec. 2.1), pads each
 * length to a multiple of lcm(a_w, M_w), and precomputes on the device, in
 * FP64, every truncated cross-kernel h_{w,v} on its common grid (Sec. 4.1,
 * 4.2; threshold Eq. truncgram, absolute unless MP_THR_REL) plus FP32 copies.
 * kernel_tol is the threshold epsilon, 0 <= epsilon < 1 (0 keeps every
 * entry whose overlap is nonzero; MP_E_ARG otherwise).  flags: MP_PREC_*, MP_THR_REL,
 * MP_CONJ_GATE_GAMMA, MP_PEDANTIC, at most one MP_DFT_* (not with
 * MP_PREC_F64), MP_SCHED_* (not with MP_PREC_F64; at most one MP_SCHED_TILE*,
 * MP_SCHED_TILE32 only with MP_SCHED_NT512).  Uses the
 * current HIP device; blocks until the kernels are built.  *out receives the
 * plan.  MP_E_LIMIT: a frame's FFT exceeds the LDS of one workgroup (M/2
 * complex entries of the DFT's precision; twice that for the split
 * MP_DFT_*), or the signal's tree groups do not fit it. */
int mp_plan_create(const mp_dict *dicts, int32_t W, const int64_t *L,
                   int32_t batch, double kernel_tol, uint32_t flags,
                   mp_plan **out);

/* Timings of mp_autotune: one entry per schedule tried. */
#define MP_TUNE_MAX 10
typedef struct {
  int32_t n_cand;                    /* schedules tried (distinct ones)       */
  int32_t chosen;                    /* index of the returned one             */
  uint32_t flags[MP_TUNE_MAX];       /* MP_SCHED_* bits of each               */
  int32_t threads[MP_TUNE_MAX];      /* threads per workgroup of each         */
  int32_t group_leaves[MP_TUNE_MAX]; /* leaves per tree group of each         */
  int32_t tile_rows[MP_TUNE_MAX];    /* rows per neighbourhood tile of each   */
  double probe_ms[MP_TUNE_MAX];      /* device time of each probe run         */
  double probe_bytes[MP_TUNE_MAX];   /* algorithmic bytes of each probe: 16 B per
                                        coefficient update with a nonzero kernel
                                        entry + 8 B per tree leaf and group
                                        rewritten (FP32 plans; FP64: 32 B)  */
} mp_tune_report;

/* Schedule autotuner (no counterpart in the paper: the launch shape of the
 * batched loop is a property of this GPU implementation).  Creates a plan as
 * mp_plan_create(dicts, W, L, batch, kernel_tol, flags | s) for each
 * schedule s among the MP_SCHED_* combinations (one schedule for FP64
 * plans): the four launch shapes (threads x group leaves) with 16- and 8-row
 * tiles, and the two 512-thread shapes with 32-row tiles.  It skips schedules
 * whose plan would duplicate an earlier one or does not fit (MP_E_LIMIT),
 * analyses x_dev (as mp_analyze) and times an mp_run of probe_atoms
 * selections per signal without SNR rule on `stream` (device events;
 * synchronizes).  The schedules are tried in the order default, MP_SCHED_G128,
 * MP_SCHED_NT512, both, then the same with MP_SCHED_TILE8, then the two
 * MP_SCHED_TILE32 ones; a later one replaces the current choice only when
 * its probe is more than 1 % faster, so that timing noise does not flip the
 * choice.  *out receives the chosen plan, the others are
 * destroyed; the returned plan holds the probe's state, so call mp_analyze
 * before using it.  rep (may be null) receives the timings.  Errors:
 * MP_E_ARG for null pointers, probe_atoms <= 0 or MP_SCHED_* bits in flags,
 * else those of mp_plan_create, mp_analyze and mp_run (no plan is returned
 * then). */
int mp_autotune(const mp_dict *dicts, int32_t W, const int64_t *L,
                int32_t batch, double kernel_tol, uint32_t flags,
                const void *x_dev, int32_t dtype, int64_t probe_atoms,
                hipStream_t stream, mp_plan **out, mp_tune_report *rep);

/* Analysis: E0 = ||x||^2 (FP64), rho_0 = D_w* x for every system (Sec. 5)
 * and the max tree over |rho_0|^2 (Sec. 5.1).  x_dev holds the batch packed
 * back to back in the order given at creation (signal s starts at element
 * sum_{r<s} L[r]); dtype is MP_DTYPE_F32 or MP_DTYPE_F64.  Resets the atom
 * logs.  May be captured into a HIP graph (it then enqueues kernels only and
 * records no timing events for mp_get_stats). */
int mp_analyze(mp_plan *plan, const void *x_dev, int32_t dtype,
               hipStream_t stream);

/* Runs the MP loop of every signal until a stop rule holds: n_atoms >=
 * max_atoms (<= 0: L_padded/5 per signal), E <= 10^(-target_snr_db/10) E0
 * (target_snr_db <= 0: no SNR rule), E < 0, or max |rho| = 0 (Alg. 1 with
 * the stopping conditions of Sec. 6.1 and Sec. 7).  Continues from the
 * current state when called again without mp_analyze.  Grows the atom logs
 * when max_atoms exceeds their capacity (the only allocation it makes).  May
 * be captured into a HIP graph once the logs hold max_atoms (an earlier
 * mp_run with the same max_atoms); under capture it records no timing
 * events, and a run that would have to grow the logs returns MP_E_STATE. */
int mp_run(mp_plan *plan, int64_t max_atoms, double target_snr_db,
           hipStream_t stream);

/* Approximate MP with resets (Alg. 2), from a fresh mp_analyze of the same
 * x_dev (same layout and dtype).  The inner loop (Alg. 1 on the current
 * residual's coefficients) runs until reset_it selections (> 0) or, when
 * reset_db < 0, until its error estimate falls below 10^(reset_db/10) times
 * the error at the last reset, or until any stop rule of mp_run.  Then the
 * selections are added to the solution, synthesized, and subtracted from the
 * true residual r = x - D c (FP64, over the padded length); ||r||^2 becomes
 * the error and rho = D* r the new coefficients.  A signal finishes when its
 * true error reaches target_snr_db (> 0), when max_atoms selections were made
 * (<= 0: L_padded/5), when all coefficients are zero, or when an inner loop
 * made no selection.  The atom log holds every selection; E_after is the
 * inner estimate, reset to the true error at each reset.  reset_it <= 0
 * selects the default criterion derived from the kernel threshold eps (Sec.
 * 7): reset_it = ceil(32 / eps) and, unless reset_db < 0 is given,
 * reset_db = 10 log10(eps).  Synchronizes with the stream once per reset
 * round.  MP_E_STATE unless called right after mp_analyze; MP_E_ARG for
 * reset_db > 0. */
int mp_run_resets(mp_plan *plan, const void *x_dev, int32_t dtype,
                  int64_t max_atoms, double target_snr_db, int64_t reset_it,
                  double reset_db, hipStream_t stream);

/* The solution of Alg. 1 as a list: copies up to `cap` selected atoms of
 * signal `sig` (system, bin, frame, the adjusted coefficient c~ of Eq.
 * dualatprod that the solution update adds, and the error estimate after the
 * selection) to out_host, in selection order; *n_out (may be null) receives
 * the number of atoms selected.  Waits for the stream of the last mp_run.
 * MP_E_ARG for a bad plan, signal, cap < 0 or out_host null with cap > 0;
 * MP_E_HIP if the copy fails. */
int mp_get_atoms(const mp_plan *plan, int32_t sig, mp_atom *out_host,
                 int64_t cap, int64_t *n_out);

/* Error-estimate curve of signal `sig` (Alg. 1, error update E_k = E_{k-1} -
 * E~_k with E~_k of Eq. projenfaster): E_0 = ||x||^2 followed by E_k after
 * each selection, up to `cap` values into E_curve_host; *n_out (may be null)
 * receives n_atoms + 1.  Waits for the stream of the last mp_run.  Errors as
 * mp_get_atoms. */
int mp_get_energy(const mp_plan *plan, int32_t sig, double *E_curve_host,
                  int64_t cap, int64_t *n_out);

/* Solution vector of signal `sig` in system w: the sum of c~ of the
 * selected atoms at each (m, n) (Alg. 1, solution update), as FP64 complex
 * N_w x (M_w/2 + 1) into c_dev. */
int mp_get_coefs(const mp_plan *plan, int32_t sig, int32_t w, void *c_dev,
                 hipStream_t stream);

/* Current residual coefficient plane of signal `sig` in system w
 * (coefficient-domain residual rho), N_w x (M_w/2 + 1) complex in the plan's
 * precision (FP32 pairs or FP64 pairs) into dst_dev. */
int mp_get_residual(const mp_plan *plan, int32_t sig, int32_t w,
                    void *dst_dev, hipStream_t stream);

/* Synthesis of the selected atoms of signal `sig` (Eq. idgtreal): pairs add
 * 2 Re(c d), DC and Nyquist atoms add Re(c d).  y_dev receives L_padded
 * samples of type dtype (MP_DTYPE_F32 or MP_DTYPE_F64: the output type is an
 * argument so that FP32 plans can return an FP64 synthesis); accumulation is
 * FP64.  MP_E_ARG for a bad plan, signal, dtype or null y_dev; MP_E_STATE
 * before mp_analyze. */
int mp_resynth(const mp_plan *plan, int32_t sig, void *y_dev, int32_t dtype,
               hipStream_t stream);

/* Allocation-free synthesis, for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc).  Same arguments, output and errors as mp_resynth, and the same
 * kernels; the FP64 accumulator is not a plan buffer but a static device
 * array of MP_STATIC_RESYNTH_MAX samples that the library holds on every
 * device it runs on until the process ends (its address is looked up once
 * per device, on the first call there).  The call allocates nothing (no
 * hipMalloc, hipFree or allocating library routine).  L_padded of the signal
 * above MP_STATIC_RESYNTH_MAX: MP_E_LIMIT.  The call runs on the plan's
 * device.  All calls on one device share the array (each call clears the
 * part it uses before accumulating), so calls that overlap in time on one
 * device, on any streams or plans, race and must be serialised by the
 * caller. */
#define MP_STATIC_RESYNTH_MAX ((int64_t)1 << 22)
int mp_resynth_static(const mp_plan *plan, int32_t sig, void *y_dev, int32_t dtype,
                      hipStream_t stream);

int mp_signal_info_get(const mp_plan *plan, int32_t sig, mp_signal_info *out);

/* Pair (target w, source v) kernel geometry, and the FP64 box table
 * h_{w,v}(mu, delta) for delta = -delta_box..delta_box (rows) and
 * mu = mu_lo..mu_hi (columns, fastest): (2 delta_box + 1)(mu_hi - mu_lo + 1)
 * complex values as separate re / im host arrays, entries at or below the
 * threshold set to zero. */
int mp_kernel_info_get(const mp_plan *plan, int32_t w, int32_t v,
                       mp_kernel_info *out);
int mp_get_kernel(const mp_plan *plan, int32_t w, int32_t v, double *re_host,
                  double *im_host, int64_t cap);

/* Counters and device timings of the last mp_analyze / mp_run. */
int mp_get_stats(const mp_plan *plan, mp_stats *out);

/* Releases the plan and every buffer it owns (the C module's final call,
 * Sec. 7); waits for the plan's last stream and the device first.  MP_E_ARG
 * for a null plan. */
int mp_plan_destroy(mp_plan *plan);

/* Text of a return code (the C module's functions return integer error
 * codes, Sec. 7); a static string, never null. */
const char *mp_strerror(int code);

#ifdef __cplusplus
}
#endif
#endif
