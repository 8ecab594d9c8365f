// Intrinsic pre-selection (Sec. IV D; App. B eqs. dh_itop, x_ML,
// single_det_ML): for every bank row, each detector's maximum likelihood
// over a phase x time grid with the detector response and distance
// replaced by one free real amplitude per polarisation, summed over the
// detectors (the incoherent maximum); the rows within delta of the best are
// kept.  Shared by the host runtime and the translation unit with the
// kernels (preselect.hip).
//
// Per row i (inclination iota_i, a property of the row here), detector k,
// time t_kj = t0_k + j dt and phase phi_o:
//     Y_ikc(t) = sum_b conj(h_icb) w_kb d_kb exp(2 pi i f_b t)     (complex GEMM,
//                over the bank operand the evidence pass uses)
//     b_p      = Re sum_c conj(K_cp(iota_i)) exp(i m_c phi_o) Y_ikc
//     H_pp'    = Re sum_cc' K_cp conj(K_c'p') exp(-i (m_c - m_c') phi_o) G_ikcc',
//     G_ikcc'  = sum_b w_kb h_icb conj(h_ic'b)
//     lnL^ML   = b^T H^+ b / 2  (H^+: pseudo-inverse of the 2x2 matrix)
// with K_c+ = (Y_l,-m + (-1)^l Y_lm)/2 real and K_cx = i (Y_l,-m - (-1)^l Y_lm)/2.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "common.h"

namespace dotpe {

constexpr int kPreMaxT = 128;      // time-grid points per detector (a multiple of 32)
constexpr int64_t kPreChunk = int64_t(1) << 18;   // rows per (h|h) Gram block

struct PreArgs {
  // bank operand (split precisions): conj(h) 2^-e_i in op_index layout
  const void* A0;
  const void* A1;
  const void* R0;            // the same hi and lo parts row by row ([n_wf][K2])
  const void* R1;
  const double* row_scale;
  int64_t K2;
  int n_c, n_b, n_bp;
  int l[kMaxC], m[kMaxC];    // (l, m) of each channel, bank (group) order
  int cg[kMaxC];             // group of each channel
  int gm[kMaxG];             // m of each group
  int G;
  // rows: bank rows row0 .. row0 + n_rows - 1; this launch's block of them
  int64_t row0, n_rows, chunk0, n_chunk;
  const double* cos_iota;    // [n_rows]
  // data side
  int n_det, n_t, n_phi;
  const double* f;           // [n_b]
  const double2* d;          // [n_det][n_b]
  const double* w;           // [n_det][n_b]
  const double* t0;          // [n_det]
  double dt;
  const void* B0;            // [n_det * n_t][K2p] hi, lo (op_index)
  const void* B1;
  double* col_scale;         // [n_det * n_t]
  int64_t K2p;               // 2 n_bp
  // work and outputs
  double2* gram;             // [n_chunk][n_det][NP], c <= c'
  double* ml_det;            // [n_rows][n_det]: max over (t, o) per detector
  double* lnl;               // [n_rows]: sum over detectors
  uint64_t* state;           // [0] largest lnl (ordered bits), [1] rows selected
  double delta;              // selection width
  int* counts;               // [n_blocks] rows selected per block of 1024
  int64_t* offsets;          // [n_blocks]
  int64_t* selected;         // [n_rows] bank rows kept, ascending
  double* ml_t;              // optional [n_rows][n_det][n_t]: max over phases per grid time
};

__host__ __device__ inline int pre_pairs(int n_c) { return n_c * (n_c + 1) / 2; }

// The whole pass on stream s: data operand, then per block of kPreChunk
// rows the Gram matrices and the grid maximum, then the incoherent sums and
// the selection.  prec: kFP16X2 or kBF16X2.  Returns the first launch error.
hipError_t preselect_launch(int prec, PreArgs a, hipStream_t s);

}  // namespace dotpe
