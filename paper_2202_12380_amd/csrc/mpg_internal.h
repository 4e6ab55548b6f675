// Internal layout shared by the host plan code and the HIP kernels of libmpg.
// Not part of the C-ABI.
#pragma once
#include <stdint.h>

namespace mpg {

constexpr int MAXW = 8;        // Gabor systems per plan
constexpr int ROW = 16;        // coefficients per max-tree leaf (one DPP row)
constexpr int ENERGY_PARTS = 32;  // partial sums per signal in the energy kernel
constexpr int LOG_ROW = 4;
constexpr int GLEAVES = 256;   // leaves per group when the group preload path is used (FP64)
// Samples of the static FP64 accumulator used by mp_resynth_static (32 MiB
// per device), and the devices it tracks.
constexpr int64_t STATIC_RESYNTH_MAX = (int64_t)1 << 22;
constexpr int MAX_DEVICES = 64;

// One Gabor system.  M is even; it need not be a power of two (then the
// analysis runs the defining sum of the DFT and the loops take indices mod M
// by division instead of masks).
struct DictDev {
  int32_t gl, a, M, MR;        // MR = M/2 + 1 reduced bins
  int64_t win_off;             // offset of its window in the window arrays
  int64_t tw_off;              // offset of its DFT twiddles exp(-2 pi i j / M), j < M/2, then their
                               // stage-major copy (M entries in all)
  int64_t gamma_off;           // offset of gamma(k), k = 0..M/2
  int64_t root_off;            // offset of exp(+2 pi i j / M), j < M (update phases)
  uint32_t mr_mul;             // q / MR == (umulhi(q, mr_mul) + q) >> mr_sh, q < 2^31
  int32_t mr_sh;
  int32_t lpf;                 // max-tree leaves per frame, ceil(MR / ROW)
  int32_t pad;
  uint32_t m_mul;              // q / M the same way (phase indices mod M when M is not a power of two)
  int32_t m_sh;
  int32_t pad2[2];
};

// Kernel of the ordered pair (target w, source v) on the common grid
// (a_min, M_max).  The stored box is delta = -dbox..dbox (rows) by
// mu = mu_lo..mu_hi (columns, fastest); mu_hi - mu_lo + 1 <= M_max.
struct PairDev {
  int32_t amin, Mmax, rw, rv;  // r = M_max / M
  int32_t dbox, mu_lo, mu_hi, width;
  int32_t sw, sv;              // a_w / a_min, a_v / a_min
  int64_t tab_off;             // entry offset of the box table
  // FP32 copy of the table, phase-major rows: entry mu' = mu - mu_lo of row
  // Delta sits at (mu' mod rw) cw + mu' div rw, so the bins of a target
  // frame (mu' stepping by rw) read consecutive entries
  int32_t cw, width32;         // ceil(width / rw), row stride rw cw
  int64_t tab_off32;           // entry offset in the FP32 table
};

// One signal of the batch.  Plane of system w: coef_base + off[w], N_w x MR_w
// complex entries, bin m fastest; off[w] is also the global coefficient index
// of (w, m = 0, n = 0).  Max-tree leaves cover 16 bins of one frame: leaf
// (w, n, i) is leaf_base + lbase[w] + n * lpf_w + i; each system's leaves are
// padded to whole groups of G leaves.
struct SigDev {
  int64_t L, Lp, x_off;
  int64_t coef_base;           // first coefficient of the signal
  int64_t n_coef_padded;       // sum_w N_w MR_w, rounded up to a multiple of ROW
  int64_t atom_base, cap;      // atom log slice
  int64_t leaf_base;           // first leaf of the signal
  int32_t n_leaves, n_groups;  // leaves (padded) and groups of G leaves
  int32_t N[MAXW];             // frames per system
  int64_t off[MAXW + 1];       // plane offsets within the signal, off[W] = total
  int64_t lbase[MAXW + 1];     // leaf offsets within the signal, lbase[W] = n_leaves
};

// Mutable per-signal state (device).
struct SigState {
  double E0, E;
  int64_t k;
  int32_t stop, pad;
  int64_t updated, blocks, groups;
  // reset procedure (Alg. 2): true error and selections at the last reset
  double Eout;
  int64_t kout;
  int32_t done, resets;
};

// Atom record, same layout as mp_atom.
struct AtomRec {
  int32_t w, m, n, pad;
  double re, im;
  double E_after;
};

// Arguments of the persistent MP kernel.
struct MPArgs {
  const DictDev* dicts;
  const PairDev* pairs;
  const SigDev* sigs;
  SigState* state;
  void* planes;
  void* leaves;
  AtomRec* atoms;
  const void* tabs;
  const void* gammas;
  const void* roots;
  const int32_t* order;
  int32_t* queue;
  int32_t W, batch, G, logG;
  int32_t n_groups_max, p2;    // p2: every M of the plan is a power of two
  int32_t slot_cap;            // 8-row slots per tile of the neighbourhood split (1, 2 or 4)
  int32_t xpre;                // 1: touched groups beyond the preloaded ones are loaded before the merges
  int64_t K;
  double snr_db;
  uint32_t partner_gate, pedantic;  // pedantic: select by the pair projection energy (Sec. 5)
  int64_t reset_it;            // > 0: inner loop of the reset procedure, at most reset_it selections
  double reset_db;             // < 0: inner loop also ends when E <= Eout 10^(reset_db / 10)
};

}  // namespace mpg
