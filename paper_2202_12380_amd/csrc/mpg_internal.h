// Internal layout shared by the host plan code and the HIP kernels of libmpg.
// Not part of the C-ABI.
#pragma once
#include <stdint.h>

namespace mpg {

constexpr int MAXW = 8;        // Gabor systems per plan
constexpr int BLK = 64;        // coefficients per max-tree leaf (one wavefront)
constexpr int MAXB = 256;      // signals per plan (queue/order arrays are sized at plan time)

// One Gabor system.
struct DictDev {
  int32_t gl, a, M, MR;        // MR = M/2 + 1 reduced bins
  int64_t win_off;             // offset of its window in the window arrays
  int64_t tw_off;              // offset of its twiddle table (M/2 entries)
  int64_t gamma_off;           // offset of gamma(k), k = 0..M/2
};

// Kernel of the ordered pair (target w, source v) on the common grid
// (a_min, M_max).  The stored box is delta = -dbox..dbox (rows) by
// mu = mu_lo..mu_hi (columns, fastest); mu_hi - mu_lo + 1 <= M_max.
struct PairDev {
  int32_t amin, Mmax, rw, rv;  // r = M_max / M
  int32_t dbox, mu_lo, mu_hi, width;
  int64_t tab_off;             // entry offset of the box table
};

// One signal of the batch.  Planes of system w start at coef_base + off[w]
// (complex entries); each plane is padded to a multiple of BLK entries so
// that no leaf straddles two systems.
struct SigDev {
  int64_t L, Lp, x_off;
  int64_t coef_base;           // first coefficient of the signal (multiple of BLK)
  int64_t n_coef_padded;       // sum of padded plane sizes
  int64_t atom_base, cap;      // atom log slice
  int32_t n_leaves, n_groups;  // leaves = n_coef_padded / BLK, groups of G leaves
  int32_t N[MAXW];             // frames per system
  int64_t off[MAXW + 1];       // plane offsets within the signal (padded), off[W] = total
};

// Mutable per-signal state (device).
struct SigState {
  double E0, E;
  int64_t k;
  int32_t stop, pad;
  int64_t updated, blocks, groups;
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
  const int32_t* order;
  int32_t* queue;
  int32_t W, batch, G, logG;
  int64_t K;
  double snr_db;
  uint32_t partner_gate;
};

}  // namespace mpg
