/* dotpe.h -- C ABI of the likelihood-matrix hot path (gfx950).
 *
 * Computes, for every pair of an intrinsic-bank waveform i and an extrinsic
 * sample e, the distance- and phase-marginalised likelihood
 *     Lbar_ie = (1/N_phi) sum_o int dD pi(D) exp(dh_ieo d0/D - hh_ieo d0^2/(2 D^2))
 * with dh, hh the inner products of eq. (dh_ieo) and eq. (hh_ieo), the
 * distance scaling of eq. (lnlike_ieo_arb_dL) and the distance integral of
 * eq. (lnl_dist_marginalized), and reduces it to the evidence of eq. (Z_sum)
 *     Z = 1/(N_norm N_ext) sum_ie w_i w_e Lbar_ie        (w_o = 1)
 * plus effective-sample-size ingredients (eq. n_effective) and the top-k
 * pairs by posterior weight p_ie = w_i w_e Lbar_ie.
 *
 * Conventions (all inputs FP64, little-endian, row-major, interleaved complex
 * re,im):
 *   detector waveform  h_k(f_b) = (d0/D) sum_c h_cb R_ekc exp(-2 pi i f_b t_ek)
 *                                  exp(-i m_c phi_o)                  (eq. h_k)
 *   response           R_ekc = F_ek+ K_c+(iota_e) + F_ekx K_cx(iota_e)
 *                      F_ekp = D_k : e_p, e_+ = XX^T - YY^T, e_x = XY^T + YX^T,
 *                      X = cos(psi) e_lon + sin(psi) e_lat,
 *                      Y = -sin(psi) e_lon + cos(psi) e_lat   (eq. response_plus/cross)
 *                      K_c+ = (Y_l,-m + (-1)^l Y_lm)/2, K_cx = i(Y_l,-m - (-1)^l Y_lm)/2,
 *                      Y = spin-weight -2 spherical harmonic at azimuth 0
 *   arrival time       t_ek = t_geo,e - r_k . n_e / c, n_e towards the source
 *                      (eq. t_at_detector, source-pointing n)
 *   inner products     (a|b) = sum_k sum_b w_kb a_kb conj(b_kb), w_kb = 4 df_b/S_k(f_b)
 *                      (eq. inner_product on the given bins)
 *   phase grid         phi_o = 2 pi o / N_phi
 *   distance prior     proportional to D^2 on (0, D_max]
 *
 * Error behaviour: every call returns DOTPE_OK (0) or a negative code;
 * dotpe_last_error() returns a message for the calling thread's last error.
 * On error, outputs are left untouched and no handle is returned.
 * Handles are owned by the library and freed with the matching free call.
 * A context is not thread-safe; a server's calls may be made from any thread.
 */
#ifndef DOTPE_H
#define DOTPE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define DOTPE_OK 0
#define DOTPE_E_INVALID_ARG (-1)
#define DOTPE_E_OOM (-2)
#define DOTPE_E_ADMISSION (-3)
#define DOTPE_E_NUMERIC (-4)
#define DOTPE_E_DEVICE (-5)
#define DOTPE_E_TOO_LARGE (-6)
#define DOTPE_E_UNIMPLEMENTED (-7)

/* arithmetic of the (d|h) contraction */
#define DOTPE_PREC_FP64 0     /* FP64 operands, FP64 MFMA */
#define DOTPE_PREC_FP16X2 1   /* FP16 hi+lo operands, 3 products, FP32 MFMA accumulation */
#define DOTPE_PREC_BF16X2 2   /* BF16 hi+lo operands, 3 products, FP32 MFMA accumulation */

/* event flags.  With a cut, dotpe_evidence bounds every pair of a tile
 * first and evaluates the tile's survivors afterwards; a tile with more
 * survivors than its record area holds is left to the coefficient route
 * (its raw contraction results stored, then every pair bounded and
 * evaluated by a separate kernel), which also takes every tile when the
 * cut is off.  DOTPE_FLAG_RERUN_ALL sends every tile with a survivor
 * through that route (a check that both routes agree; slower). */
#define DOTPE_FLAG_RERUN_ALL 1
/* With a cut, split-precision events of at least 2048 tiles of 128 x 128
 * pairs first run a bound pass: it only bounds every pair (the contraction
 * without the per-pair marginalisation, at half the operand traffic per pair)
 * and lists each 64 x 64 tile's few survivors for a survivor pass, or the
 * tile for the coefficient route.  DOTPE_FLAG_NO_BOUND_PASS uses the fused
 * kernel's bound-then-evaluate epilogue instead (results agree to rounding). */
#define DOTPE_FLAG_NO_BOUND_PASS 2

/* where a caller pointer lives */
#define DOTPE_MEM_HOST 0
#define DOTPE_MEM_DEVICE 1

typedef struct dotpe_ctx dotpe_ctx;
typedef struct dotpe_bank dotpe_bank;
typedef struct dotpe_event dotpe_event;

/* Library version string. */
const char* dotpe_version(void);

/* Message of the calling thread's last failed call ("" if none). */
const char* dotpe_last_error(void);

/* Create a context on HIP device `device`.  hbm_budget_bytes caps the
 * device memory its banks and events may hold (0 = no cap; the context's
 * own distance table, about 21 MB, is not charged).  Builds the distance
 * marginalisation table on the device.  Errors: INVALID_ARG (bad device),
 * DEVICE, OOM. */
int dotpe_create(int device, uint64_t hbm_budget_bytes, dotpe_ctx** out);

/* Release a context and everything it owns.  NULL is a no-op. */
int dotpe_destroy(dotpe_ctx* ctx);

/* Bytes of device memory currently held by the context. */
uint64_t dotpe_device_bytes(const dotpe_ctx* ctx);

/* Intrinsic waveform bank (Sec. IV C): n_wf waveforms, each n_modes (l, m)
 * channel amplitudes on n_bins frequencies, at distance d0, reference phase
 * 0 and polarisation angle 0. */
/* Channel layouts of a bank.  DOTPE_LAYOUT_LM: one channel per (l, m) mode
 * of a non-precessing waveform; the inclination is an extrinsic parameter
 * and each channel's response is sum_p F_kp K_cp(iota) (eq. response_plus,
 * response_cross with the -2Y_lm factors).  DOTPE_LAYOUT_MP: the paper's own
 * layout (Sec. IV A, eq. h_k): one channel per azimuthal harmonic m and
 * polarisation p of h_mp(f; theta_int), the inclination inside theta_int
 * (eq. thetaint), the response the real antenna pattern F_kp. */
#define DOTPE_LAYOUT_LM 0
#define DOTPE_LAYOUT_MP 1

typedef struct dotpe_bank_desc {
  int64_t n_wf;
  int32_t n_modes;        /* 1..8 channels; m in 1..4; at most 4 distinct m */
  int32_t n_bins;         /* 1..4096 */
  const int32_t* mode_l;  /* [n_modes] host (layout LM; unused for MP) */
  const int32_t* mode_m;  /* [n_modes] host */
  const double* f_bins;   /* [n_bins] Hz, host */
  const double* h;        /* [n_wf][n_modes][n_bins][2], host or device (mem) */
  const double* ln_w;     /* [n_wf] ln w_i (eq. int_weights), host or device, NULL = 0 */
  int32_t precision;      /* DOTPE_PREC_* */
  int32_t mem;            /* DOTPE_MEM_* for h and ln_w */
  int32_t layout;         /* DOTPE_LAYOUT_* (0 = LM) */
  int32_t reserved;       /* 0 */
  const int32_t* mode_p;  /* layout MP: [n_modes] host, polarisation of each channel, 0 (+) or
                             1 (x); each (m, p) at most once */
} dotpe_bank_desc;

/* Copy and convert a bank into device memory (the bank-summary layout).
 * The caller keeps ownership of its arrays.  Errors: INVALID_ARG,
 * NUMERIC (non-finite amplitudes), OOM / ADMISSION (over budget), DEVICE. */
int dotpe_load_bank(dotpe_ctx* ctx, const dotpe_bank_desc* desc, dotpe_bank** out);
int dotpe_free_bank(dotpe_ctx* ctx, dotpe_bank* bank);

/* One event: data, noise weights, detectors and the extrinsic set
 * (Sec. IV A, IV B).  All pointers are host memory. */
typedef struct dotpe_event_desc {
  int32_t n_det;            /* 1..8 */
  int32_t n_phi;            /* 1..128 reference-phase grid points */
  const double* d;          /* [n_det][n_bins][2] data at f_bins */
  const double* w;          /* [n_det][n_bins] w_kb = 4 df_b / S_k(f_b) */
  const double* det_r;      /* [n_det][3] detector positions, metres, Earth-fixed */
  const double* det_D;      /* [n_det][3][3] response tensors 0.5 (x x^T - y y^T) */
  int64_t n_ext;            /* >= 1 */
  const double* lat;        /* [n_ext] Earth-fixed latitude, rad */
  const double* lon;        /* [n_ext] Earth-fixed longitude, rad */
  const double* psi;        /* [n_ext] polarisation angle, rad */
  const double* cos_iota;   /* [n_ext] cosine of inclination */
  const double* t_geo;      /* [n_ext] arrival time at the geocentre, s */
  const double* ln_w_ext;   /* [n_ext] ln w_e, NULL = 0 */
  double d_max;             /* Mpc, upper end of the distance prior */
  double d0;                /* Mpc, distance the bank is stored at */
  double n_norm;            /* N_int of eq. (Z_sum); <= 0 means the subset size */
  int64_t sub_start;        /* bank rows [sub_start, sub_start + sub_count) ... */
  int64_t sub_count;        /* ... 0 = the whole bank */
  const int64_t* sub_idx;   /* or explicit rows [sub_count] (host), NULL = range */
  double cut_delta;         /* coherent cut (eq. coherent_ML_selection): a pilot pass over
                               every 64th row of tiles (at least 16 rows of tiles on
                               small events) finds M = max lnL^ML; pairs whose
                               certified upper bound on lnL^ML lies below M - cut_delta
                               are bounded (their mass goes to ln_z_upper), not
                               marginalised; <= 0 disables the cut */
  int32_t top_k;            /* number of top pairs to return from dotpe_evidence */
  int32_t flags;            /* 0, or DOTPE_FLAG_* bits */
  double topk_window;       /* candidates kept within this of the max ln p (default 40 if <= 0) */
  void* stream;             /* hipStream_t for this event's work; NULL = context stream */
  double cut_target;        /* certificate the cut must meet: ln_z_upper - ln_z <= cut_target
                               (<= 0: 1e-4).  dotpe_evidence repeats the pass with a
                               larger cut_delta (cutting less), finally with no cut,
                               until it does */
  /* Relative binning (App. A): with w_dh set the inner products are
   * (d|h) = Re sum_kcb W^dh_kcb conj(h_kc(f_b)) (eq. d_h) and (h|h) =
   * sum_kcc'b W^hh_kcc'b h_kc(f_b) conj(h_kc'(f_b)) (eq. h_h), h_kc the
   * detector waveform's channel c at the bank's f_bins, instead of the plain
   * bin sums with w and d (which are then ignored; they may be NULL).
   * dotpe_rb_weights builds the weights from full-resolution data. */
  const double* w_dh;       /* [n_det][n_modes][n_bins][2] W^dh_kcb, bank channel order, host;
                               NULL = plain bins (W^dh = w d, W^hh = w) */
  const double* w_hh;       /* [n_det][n_modes][n_modes][n_bins][2] W^hh_kcc'b, host; required
                               with w_dh; Hermitian in (c, c') (only c <= c' is read) */
  double dd;                /* (d|d) with w_dh (the full-resolution value); ignored without */
} dotpe_event_desc;

/* Stage an event against a resident bank: copies inputs, builds the
 * extrinsic operand (antenna patterns x time-shift phasors folded over
 * detectors with the data), the per-pair (h|h) coefficient tables and the
 * per-waveform (h|h) sums.  The event's device buffers are packed into one
 * block that the context keeps after dotpe_free_event and hands to the next
 * event that fits (grown when one needs more), so a stream of events does not
 * allocate device memory each time; the block counts against the context's
 * budget until dotpe_destroy.  An event staged while another holds the block
 * gets buffers of its own, freed by dotpe_free_event.  Errors: INVALID_ARG,
 * NUMERIC, OOM, ADMISSION, DEVICE. */
int dotpe_set_event(dotpe_ctx* ctx, const dotpe_bank* bank, const dotpe_event_desc* desc,
                    dotpe_event** out);
int dotpe_free_event(dotpe_ctx* ctx, dotpe_event* ev);

/* Materialise ln Lbar_ie for every pair, no cut (parity and small shapes).
 *   lnl      [n_sub][n_ext]            ln Lbar_ie (required)
 *   ml_max   [n_sub][n_ext]            max_o lnL^ML_ieo (eq. bestfit_lnl), or NULL
 *   triples  [n_sub][n_ext][n_phi][2]  (dh, hh) per triple at d0, or NULL
 * mem says where the outputs live.  Synchronous.  Errors: INVALID_ARG,
 * TOO_LARGE (outputs over the budget), DEVICE. */
int dotpe_eval_lnl(dotpe_ctx* ctx, dotpe_event* ev, double* lnl, double* ml_max,
                   double* triples, int32_t mem);

typedef struct dotpe_evidence_result {
  double ln_z;          /* ln Z over the marginalised triples */
  double ln_z_upper;    /* ln(Z + bound on everything cut); = ln_z without cut */
  double max_lnl_ml;    /* max over triples of lnL^ML */
  double ln_sum_p;      /* ln sum_ie p_ie */
  double ln_sum_p2;     /* ln sum_ie p_ie^2 (N_eff = exp(2 ln_sum_p - ln_sum_p2)) */
  double dd;            /* (d|d) */
  double max_ln_p;      /* max_ie ln p_ie */
  int64_t n_pairs;
  int64_t n_pairs_bounded;  /* pairs skipped by the per-pair bound */
  int64_t n_triples_marg;   /* triples distance-marginalised */
  int32_t precision;
  int32_t topk_count;       /* entries written to topk */
  int32_t topk_exact;       /* 1 if no cut pair could have entered the top-k window */
  int32_t status;
  double t_pilot_ms;        /* device time of the threshold pilot pass (HIP events) */
  double t_fused_ms;        /* device time from the end of the pilot to the end of the
                               main pass, second pass included (HIP events) */
  double cut_delta_used;    /* cut_delta of the pass returned (0: no cut) */
  int32_t n_passes;         /* evidence passes run to meet cut_target */
  int32_t n_tiles_rerun;    /* 64 x 64 tiles evaluated by the coefficient route (all of
                               them when the cut is off) */
  double t_main_ms;         /* device time of the main pass's first kernel alone: the
                               bound pass, or the fused kernel (HIP events) */
  int32_t n_tiles_listed;   /* 64 x 64 tiles whose few survivors the bound pass listed */
  int32_t reserved;
  /* effective-sample-size ingredients over the marginalised pairs, with
   * p_ieo = w_i w_e Lbar_ieo / N_phi (so that sum_o p_ieo = p_ie):
   *   N_eff      = exp(2 ln_sum_p - ln_sum_p2_triples)   (eq. posterior_element)
   *   N_eff,int  = exp(2 ln_sum_p - ln_sum_row2)         (eq. int_ess)
   *   N_eff,ext  = exp(2 ln_sum_p - ln_sum_col2)         (eq. ext_ess) */
  double ln_sum_p2_triples; /* ln sum_ieo p_ieo^2 */
  double ln_sum_row2;       /* ln sum_i (sum_e p_ie)^2 */
  double ln_sum_col2;       /* ln sum_e (sum_i p_ie)^2 */
} dotpe_evidence_result;

typedef struct dotpe_sample {
  int64_t i;        /* bank row (absolute index) */
  int64_t e;        /* extrinsic sample */
  double ln_p;      /* ln w_i + ln w_e + ln Lbar_ie */
  int32_t o_best;   /* phase index of the largest ln Lbar_ieo */
  int32_t reserved;
} dotpe_sample;

/* Fused, non-materialising evaluation of the evidence: the pilot, the bound
 * or fast pass with the survivor pass, the coefficient route and the
 * fixed-order reduction, every decision between them taken on the device
 * (the host waits once per pass, for the results).  topk: [desc.top_k]
 * host array or NULL.  Synchronous.  Errors: INVALID_ARG, DEVICE. */
int dotpe_evidence(dotpe_ctx* ctx, dotpe_event* ev, dotpe_evidence_result* out,
                   dotpe_sample* topk);

/* Posterior samples (Sec. III B: resampling by the probabilistic weights;
 * Sec. V B: N_s = N_eff / 2).  After dotpe_evidence on the event, draws
 * n_samples triples (i, e, o) and a distance each: pairs by systematic
 * resampling over the weights p_ie of the pairs the last pass evaluated --
 * draw s at cumulative mass (s + u0) / n_samples of the total, the pairs
 * taken 64 x 64 tile by tile (tiles in row-major order of the tile grid,
 * pairs row-major within a tile; an FP64 tile is 64 x 32) -- then, per pair,
 * the phase o with probability Lbar_ieo over the phases the cut kept, and
 * the distance D from its posterior given (dh_ieo, hh_ieo) with the D^2
 * prior on (0, D_max], each by inverting its distribution at the uniform
 * number 2 s (phase) and 2 s + 1 (distance) of a SplitMix64 generator seeded
 * with `seed` (the distance's in v = d0/D, ascending: P(D' >= D) = u).
 * n_samples <= 0 draws floor(N_eff / 2) with N_eff over triples (eq.
 * posterior_element); at most `capacity`.  out: [capacity]
 * host array; *n_out: samples written.  Synchronous.  Errors: INVALID_ARG
 * (no evidence pass yet, u0 outside [0, 1)), OOM / ADMISSION, DEVICE. */
typedef struct dotpe_posterior_sample {
  int64_t i;                /* bank row (absolute index) */
  int64_t e;                /* extrinsic sample */
  int32_t o;                /* phase index, phi_o = 2 pi o / N_phi */
  int32_t reserved;
  double distance;          /* Mpc */
  double ln_p_pair;         /* ln p_ie = ln w_i + ln w_e + ln Lbar_ie */
  double ln_p_triple;       /* ln p_ieo = ln w_i + ln w_e + ln Lbar_ieo - ln N_phi */
} dotpe_posterior_sample;

int dotpe_sample_posterior(dotpe_ctx* ctx, dotpe_event* ev, int64_t n_samples, double u0,
                           uint64_t seed, dotpe_posterior_sample* out, int64_t capacity,
                           int64_t* n_out);

/* dotpe_set_event + dotpe_evidence + dotpe_free_event in one call that
 * allocates no device memory (no hipMalloc / hipFree, no allocating library
 * routine): for callers that cannot allocate -- code that runs under HIP
 * graph capture, tight serving loops, harnesses that forbid allocation.
 * Every buffer of the event is packed into a fixed device scratch array of
 * 128 MiB that the library holds on each GPU it runs on until the process
 * ends; events whose footprint (dotpe_event_bytes) exceeds it are rejected
 * with TOO_LARGE.  The caller passes the inputs (desc, host arrays) and the
 * outputs (out, topk [desc.top_k] host array or NULL) as for
 * dotpe_evidence; t_pilot_ms and t_fused_ms are 0 (no timing events).  All
 * calls on one GPU share its scratch, which keeps the last call's contents
 * (everything that must start at zero is cleared by the call itself); the
 * library serialises such calls within a process, so calls that overlap on
 * one GPU wait for each other.  Synchronous.  Errors: INVALID_ARG, NUMERIC,
 * TOO_LARGE, UNIMPLEMENTED (device without scratch), DEVICE. */
int dotpe_evidence_static(dotpe_ctx* ctx, const dotpe_bank* bank, const dotpe_event_desc* desc,
                          dotpe_evidence_result* out, dotpe_sample* topk);

/* Device bytes one event needs: every buffer dotpe_set_event and
 * dotpe_evidence use for it, packed in one block (the admission footprint of
 * the serving calls).  Validates the description like dotpe_set_event.
 * Errors: INVALID_ARG, NUMERIC. */
int dotpe_event_bytes(const dotpe_ctx* ctx, const dotpe_bank* bank, const dotpe_event_desc* desc,
                      uint64_t* bytes);

/* ---- Intrinsic pre-selection (Sec. IV D; App. B eqs. dh_itop, x_ML,
 * single_det_ML) ----
 *
 * For bank rows [sub_start, sub_start + sub_count), each detector k on its
 * own: the largest likelihood over a grid of reference phases phi_o
 * (n_phi) and arrival times t_kj = t0[k] + j dt (n_t), with the detector
 * response and the distance replaced by one free real amplitude per
 * polarisation (eq. x_ML): lnL^ML = b^T H^+ b / 2, b_p = (d_k | h_p
 * exp(-2 pi i f t)) (eq. dh_itop), H_pp' = (h_p | h_p'), H^+ the
 * pseudo-inverse (an eigen-direction with eigenvalue below 1e-10 of the
 * largest dropped).  The polarisations h_p = sum_c K_cp(iota_i) h_c
 * exp(-i m_c phi_o) take each row's inclination from cos_iota.  The
 * incoherent maximum is lnL^inco_i = sum_k max_{o,j} lnL^ML_ikoj; rows with
 * lnL^inco_i >= max_j lnL^inco_j - delta_lnl are selected, in ascending
 * order -- the subset to pass as sub_idx to dotpe_set_event.  Split-precision
 * banks only: the products run on the matrix cores over the bank's operand. */
typedef struct dotpe_preselect_desc {
  int32_t n_det;            /* 1..8 */
  int32_t n_t;              /* time-grid points per detector: 32, 64, 96 or 128 */
  int32_t n_phi;            /* 1..128 */
  int32_t reserved;         /* 0 */
  const double* d;          /* [n_det][n_bins][2] data at f_bins, host */
  const double* w;          /* [n_det][n_bins] noise weights, host */
  const double* t0;         /* [n_det] first grid time of each detector, s, host */
  double dt;                /* grid step, s */
  const double* cos_iota;   /* [sub_count] cosine of each row's inclination, host */
  int64_t sub_start;        /* rows [sub_start, sub_start + sub_count) ... */
  int64_t sub_count;        /* ... 0 = the whole bank */
  double delta_lnl;         /* selection width (<= 0: 20) */
  void* stream;             /* hipStream_t; NULL = context stream */
} dotpe_preselect_desc;

typedef struct dotpe_preselect_result {
  double lnl_max;           /* largest lnL^inco over the rows */
  double threshold;         /* lnl_max - delta_lnl */
  int64_t n_rows;           /* rows considered */
  int64_t n_selected;       /* rows written to `selected` */
  double t_ms;              /* device time of the pass (HIP events) */
} dotpe_preselect_result;

/* Outputs, host arrays, each may be NULL: lnl_inco [sub_count] lnL^inco per
 * row; lnl_det [sub_count][n_det] each detector's maximum; selected
 * [sub_count] the absolute bank rows kept, ascending (the first n_selected
 * entries).  Synchronous; the pass's device buffers are allocated and freed
 * within the call, charged to the budget.  Errors: INVALID_ARG, NUMERIC
 * (non-finite input), UNIMPLEMENTED (FP64 bank, or a bank of the MP layout: the
 * polarisations are formed from (l, m) channels), OOM / ADMISSION, DEVICE. */
int dotpe_preselect(dotpe_ctx* ctx, const dotpe_bank* bank, const dotpe_preselect_desc* desc,
                    double* lnl_inco, double* lnl_det, int64_t* selected,
                    dotpe_preselect_result* out);

/* ---- Relative-binning weights (App. A, eqs. dh_weights, hh_weights) ----
 *
 * From data on a full-resolution frequency grid and a reference waveform,
 * the weights that dotpe_event_desc.w_dh / w_hh take:
 *   W^dh_kcb   = <d_k | h0_kc s_b> / conj(h0_kc(f_b)),
 *   W^hh_kcc'b = <h0_kc | h0_kc' s_b> / (h0_kc(f_b) conj(h0_kc'(f_b))),
 * with <a|b>_k = sum_f w_kf a(f) conj(b(f)) over the grid, s_b the
 * piecewise-linear functions on the nodes f_b (s_b(f_b') = delta_bb', zero
 * outside [f_0, f_{B-1}]), and h0_kc(f) = h0_c(f) exp(-2 pi i f t0_k): the
 * reference's channels shifted to its arrival time at detector k, the one
 * part of its extrinsic parameters that does not cancel.  The nodes are grid
 * points and must be the bank's f_bins.  Also (d|d) = sum_kf w_kf |d_kf|^2. */
typedef struct dotpe_rb_desc {
  int32_t n_det;            /* 1..8 */
  int32_t n_modes;          /* channels of the reference, in the bank's channel order */
  int64_t n_full;           /* full-resolution grid points, >= 2 */
  const double* f;          /* [n_full] Hz, ascending, host */
  const double* d;          /* [n_det][n_full][2] data, host */
  const double* w;          /* [n_det][n_full] 4 df / S_k(f), host */
  const double* h0;         /* [n_modes][n_full][2] reference channels, host; non-zero at the
                               nodes */
  const double* t0;         /* [n_det] reference arrival times, s, host; NULL = 0 */
  int32_t n_nodes;          /* 2..4096 */
  int32_t reserved;         /* 0 */
  const int64_t* node_idx;  /* [n_nodes] strictly ascending indices into f, host */
} dotpe_rb_desc;

/* Outputs, host arrays: w_dh [n_det][n_modes][n_nodes][2], w_hh
 * [n_det][n_modes][n_modes][n_nodes][2], dd (each may be NULL).  Synchronous;
 * device buffers are allocated and freed within the call.  Errors:
 * INVALID_ARG, NUMERIC (non-finite input, reference zero at a node), OOM /
 * ADMISSION, DEVICE. */
int dotpe_rb_weights(dotpe_ctx* ctx, const dotpe_rb_desc* desc, double* w_dh, double* w_hh,
                     double* dd);

/* ---- Extrinsic samples (Sec. IV E; App. C) ----
 *
 * Importance sampling of the extrinsic parameters from the data.  For each
 * of the n_rows intrinsic samples c (bank rows, each with its inclination),
 * each detector's arrival-time series rho^2_ck(t_j) = 2 max_o lnL^ML_ckoj
 * on its grid t0[k] + j dt (eq. single_det_ML, maximised over the phase
 * grid) gives the arrival-time probability p_ck(t) = exp(beta (rho^2_ck(t)
 * - max_t rho^2_ck)), taken at the grid point nearest to t and zero off the
 * grid.  The sky is n_sky points of equal area (a Fibonacci lattice: z_s =
 * 1 - (2 s + 1)/n_sky, longitude s times the golden angle) and the
 * geocentre time [tg_lo, tg_hi] n_tg equal cells; sample c's proposal over
 * the cells is W_c(s, j) = prod_k p_ck(t_j - r_k . n_s / c) at the cell's
 * centre time t_j, normalised.  Draw q comes from proposal q mod n_rows:
 * its cell by inverting that proposal at the uniform number 4 q of a
 * SplitMix64 generator seeded with `seed` (cells s-major), t_geo uniform in
 * the cell's time (number 4 q + 1), psi = pi u (4 q + 2), cos_iota = 2 u - 1
 * (4 q + 3); its importance weight (eq. w_e) is the prior's cell
 * probability 1 / (n_sky n_tg) over the mixture's (1 / n_rows) sum_c
 * W_c / Z_c.  Split-precision banks of the (l, m) layout (the series come
 * from the pre-selection's products). */
typedef struct dotpe_extrinsic_desc {
  int32_t n_det;            /* 1..8 */
  int32_t n_t;              /* detector time-grid points: 32, 64, 96 or 128 */
  int32_t n_phi;            /* phase grid of the single-detector maximum, 1..128 */
  int32_t n_rows;           /* intrinsic samples, 1..64 */
  const double* d;          /* [n_det][n_bins][2] data at the bank's f_bins, host */
  const double* w;          /* [n_det][n_bins] noise weights, host */
  const double* det_r;      /* [n_det][3] detector positions, metres, host */
  const double* t0;         /* [n_det] first grid time of each detector, s, host */
  double dt;                /* grid step, s */
  const int64_t* rows;      /* [n_rows] bank rows, host */
  const double* cos_iota;   /* [n_rows] their inclinations, host */
  double beta;              /* inverse temperature (<= 0: 0.5) */
  int32_t n_sky;            /* sky lattice points, 1..65536 */
  int32_t n_tg;             /* geocentre-time cells, 1..4096 */
  double tg_lo, tg_hi;      /* the prior's geocentre-time window, s */
  int64_t n_samples;        /* draws, >= 1 */
  uint64_t seed;
  void* stream;             /* hipStream_t; NULL = context stream */
} dotpe_extrinsic_desc;

typedef struct dotpe_extrinsic_result {
  double n_eff_prior;       /* (sum w)^2 / sum w^2 over the draws */
  double support;           /* prior mass of the cells the mixture reaches */
  double t_ms;              /* device time (HIP events) */
  int64_t n_samples;
} dotpe_extrinsic_result;

/* Outputs, host arrays of n_samples each (any may be NULL): lat, lon, psi,
 * cos_iota, t_geo -- the extrinsic set dotpe_event_desc takes -- and ln_w,
 * the log importance weights (its ln_w_ext).  n_rows * n_sky * n_tg is at
 * most 2^26.  Synchronous; device buffers are allocated and freed within
 * the call.  Errors: INVALID_ARG, NUMERIC, UNIMPLEMENTED (FP64 bank or MP
 * layout), OOM / ADMISSION, DEVICE. */
int dotpe_extrinsic_samples(dotpe_ctx* ctx, const dotpe_bank* bank, const dotpe_extrinsic_desc* desc,
                            double* lat, double* lon, double* psi, double* cos_iota, double* t_geo,
                            double* ln_w, dotpe_extrinsic_result* out);

/* ---- Serving: continuous admission of events against a resident bank ----
 *
 * A server owns one device pool and n_slots streams.  dotpe_submit copies an
 * event description and returns at once.  Events are admitted first in, first
 * out: the head of the queue starts when a slot is idle and the pool has a
 * free block of its footprint (dotpe_event_bytes).  An idle slot takes the
 * head and, while they fit, the events queued behind it, up to max_batch of
 * them and batch_pairs pairs in all (events that fill the device alone run
 * alone: a batch completes when its largest event does).  The slot stages each (dotpe_set_event semantics, the description's
 * stream ignored) and evaluates them together (dotpe_evidence semantics):
 * every stage of the evidence pass -- pilot, bound or fast pass, survivor
 * pass, each chunk of the coefficient route -- is one launch over the tiles
 * of all the batch's events that take it, each event keeping the grid and
 * the decisions it has alone.  Every buffer is packed in the event's pool
 * block, so serving allocates no device memory per event, and the work of
 * events in different slots overlaps on the device as well.  The blocks
 * return to the pool when the batch completes.  Results equal those of
 * dotpe_evidence on the same event alone, bit for bit: the cut threshold is
 * fixed by the pilot pass before the main pass starts, and every sum is
 * taken in an order that does not depend on timing or on the batch.
 * (Sec. IV B: every event is an independent evaluation of the likelihood
 * matrix; scheduling is outside the paper.) */
typedef struct dotpe_server dotpe_server;

typedef struct dotpe_server_desc {
  int32_t n_slots;        /* batches in flight at once, 1..16; 0 = 4 */
  int32_t max_batch;      /* events per batch, 1..16 (1: one event per launch); 0 = 8 */
  uint64_t pool_bytes;    /* device pool shared by admitted events; 0 = 8 GiB */
  uint64_t batch_pairs;   /* pairs (bank rows x extrinsic samples) a batch of several
                             events holds at most; a larger event runs alone; 0 = 2^25 */
} dotpe_server_desc;

typedef struct dotpe_ticket_info {
  double t_submit_ms;     /* host steady clock, ms since the server was created */
  double t_start_ms;      /* admitted: slot and pool block granted */
  double t_done_ms;       /* results on the host */
  uint64_t bytes;         /* pool footprint of the event */
  int32_t slot;           /* slot (stream) that ran it */
  int32_t status;         /* DOTPE_OK or the event's error code */
  int32_t batch;          /* events of the batch it ran in (its passes shared launches) */
  int32_t reserved;
} dotpe_ticket_info;

/* Create a server for `bank` (which must outlive it).  The pool is charged to
 * the context's budget.  Errors: INVALID_ARG, ADMISSION / OOM (pool), DEVICE. */
int dotpe_server_create(dotpe_ctx* ctx, const dotpe_bank* bank, const dotpe_server_desc* desc,
                        dotpe_server** out);

/* Run every submitted event to completion, then release the server.  Results
 * not collected with dotpe_wait are dropped.  NULL is a no-op. */
int dotpe_server_destroy(dotpe_server* srv);

/* Queue one event; the description's arrays are copied before returning and
 * remain the caller's.  *ticket identifies it for dotpe_poll / dotpe_wait.
 * Errors: INVALID_ARG, NUMERIC (as dotpe_set_event), ADMISSION (footprint
 * larger than the whole pool). */
int dotpe_submit(dotpe_server* srv, const dotpe_event_desc* desc, int64_t* ticket);

/* *done = 1 when the event has completed, else 0.  Errors: INVALID_ARG
 * (unknown or already collected ticket). */
int dotpe_poll(dotpe_server* srv, int64_t ticket, int32_t* done);

/* Block until the event completes and collect it (the ticket is then
 * forgotten).  out, topk ([desc.top_k] host array) and info may be NULL.
 * Returns the event's own status (its error message via dotpe_last_error);
 * info is filled in either case.  Errors: INVALID_ARG (unknown ticket), or
 * the event's error code. */
int dotpe_wait(dotpe_server* srv, int64_t ticket, dotpe_evidence_result* out, dotpe_sample* topk,
               dotpe_ticket_info* info);

#ifdef __cplusplus
}
#endif

#endif /* DOTPE_H */
