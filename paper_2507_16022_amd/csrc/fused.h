// The fused likelihood kernel: complex MFMA contraction of (d|h) and the
// (h|h) phase coefficients, then the per-pair marginalisation epilogue.
// Included by the host runtime (argument and tile shapes) and by the
// translation units that instantiate the kernel.
#pragma once

#include "common.h"
#include "pack.h"

namespace dotpe {

// ---------------------------------------------------------------------------
// fused kernel: complex MFMA contraction (d|h) + (h|h) phase coefficients,
// then the per-pair marginalisation epilogue
// ---------------------------------------------------------------------------
struct FusedArgs {
  // operands are laid out by op_index
  // bank operand (n_wf rows of K2)
  const void* A0;
  const void* A1;
  // split precisions: the bank's hi and lo parts row by row ([n_wf][K2])
  const void* R0;
  const void* R1;
  const double* row_scale;
  const double* ln_w_bank;
  // subset
  const int64_t* sub_idx;
  int64_t sub0, n_sub;
  // extrinsic operand (n_ext_p rows of K2)
  const void* B0;
  const void* B1;
  const void* B2;
  const void* B3;
  const double* col_scale;
  const double* ln_w_ext;
  int64_t n_ext, n_ext_p;
  int64_t K2;
  int n_chunks;
  // (h|h) operands (n_sub and n_ext_p rows of KH)
  const void* Ah0;
  const void* Ah1;
  const double* ah_scale;
  const void* Bh0;
  const void* Bh1;
  const double* bh_scale;
  int KH;
  int n_det;
  ModeTables mt;
  // phases
  int n_phi;
  const double* phase_cs;   // [kMaxM][n_phi][2] cos, sin of m phi_o, m = 1..kMaxM
  double ln_nphi;
  // distance rule
  DistArgs dist;
  double r0;                 // d0 / D_max
  // eval outputs
  double* lnl_out;
  double* ml_out;
  double* trip_out;
  // evidence
  double cut_delta;          // <= 0: no cut
  double topk_window;
  uint64_t* state;           // [0] max lnL^ML bits, [1] ordered max ln p, [2] candidate count
  double* partials;          // [n_tiles][kNPart]
  double* cand;              // [cap][4]: ln p, i, e, o
  int64_t cand_cap;
  int64_t n_tiles_m, n_tiles_n, n_tiles;
  int64_t pilot_stride;      // pilot pass: every pilot_stride-th row of tiles
  int* rerun;                // fast or bound pass: tiles left to the coefficient route
  int rec_cap;               // fast pass: survivors a tile may have (<= the record area)
  // bound pass: survivors of tiles with at most kSurvCap of them, as
  // (row << 8 | column) within the tile, [n_tiles][kSurvCap]; and the list
  // of such tiles, (tile id, count) pairs, its length in state[5]
  uint16_t* surv;
  int* surv_list;
  // bound pass margin: per row of each split operand the 2-norms of its hi
  // part and of what a product of hi parts leaves out, per m group (bank
  // rows [n_wf][G], extrinsic rows [n_ext_p][G]) and per output ((h|h) row
  // and column operands, [n_sub][NRT] and [n_ext_p][NRT]); the accumulation
  // factors sqrt2 K_g 2^-23 (K_g: positions of group g) and 32 2^-23
  const float2* a_nrm;
  const float2* b_nrm;
  const float2* ah_nrm;
  const float2* bh_nrm;
  float gam_dh[kMaxG];
  float gam_hh;
  // test hook: when set, the bound pass writes every pair's bounds on
  // lnL^ML here instead of cutting: [0][n_sub][n_ext] from the margin of
  // whole rows, [1][n_sub][n_ext] from the margin per group and output
  // (+inf where the (h|h) lower bound is not positive)
  float* bound_out;
  // coefficient route: work items work0 .. work0 + coef_tiles - 1 (tiles: all
  // of them when the cut is off, else the rerun list), the raw accumulators
  // of each stored at coef + (item - work0) * NCO * TM * TN, component-major
  // (X_g re, im per group, then the (h|h) outputs), pairs row-major
  void* coef;
  int64_t work0, coef_tiles;
  // per tile, the evaluated pairs' p_ie summed over each of its rows (64
  // slots) and columns (64 slots, from slot 64), relative to the tile's
  // largest ln p (partial [9]): the intrinsic and extrinsic marginals of
  // eqs. int_ess and ext_ess are their sums over tiles
  double* rowcol;
  // posterior sampling: the tiles to evaluate again (ascending), and per
  // tile the range of samples that fall in it
  const int* work_list;
  int64_t n_work_list;
  const int64_t* sample_first;   // [n_work_list + 1]
  const double* sample_res;      // [n_samples] residual mass within the tile (relative to e^M)
  double* samples;               // [n_samples][6]: i, e, o, D, ln p_ie, ln p_ieo
  uint64_t seed;                 // counter-based uniforms for the phase and distance draws
  const double* final_out;       // the reduced results (the global max of ln p at [9])
  double d0;                     // distance the bank is stored at
};

// the arguments of the event in slot q of packed launch p: its sizes and
// tables from device memory, every pointer from the kernel arguments
__device__ __forceinline__ FusedArgs pack_args(const PackLaunch& p, int e, int q) {
  FusedArgs a = p.args[e];
  const PackPtrs& r = p.ptr[q];
  a.A0 = p.A0;
  a.A1 = p.A1;
  a.R0 = p.R0;
  a.R1 = p.R1;
  a.row_scale = p.row_scale;
  a.ln_w_bank = p.ln_w_bank;
  a.a_nrm = p.a_nrm;
  a.dist.tab = p.dist_tab;
  a.dist.prm = p.dist_prm;
  a.sub_idx = r.sub_idx;
  a.B0 = r.B0;
  a.B1 = r.B1;
  a.B2 = r.B2;
  a.B3 = r.B3;
  a.col_scale = r.col_scale;
  a.ln_w_ext = r.ln_w_ext;
  a.Ah0 = r.Ah0;
  a.Ah1 = r.Ah1;
  a.ah_scale = r.ah_scale;
  a.Bh0 = r.Bh0;
  a.Bh1 = r.Bh1;
  a.bh_scale = r.bh_scale;
  a.phase_cs = r.phase_cs;
  a.state = r.state;
  a.partials = r.partials;
  a.cand = r.cand;
  a.rerun = r.rerun;
  a.surv = r.surv;
  a.surv_list = r.surv_list;
  a.b_nrm = r.b_nrm;
  a.ah_nrm = r.ah_nrm;
  a.bh_nrm = r.bh_nrm;
  a.coef = r.coef;
  a.rowcol = r.rowcol;
  // outputs of other entry points: none in a packed pass
  a.lnl_out = nullptr;
  a.ml_out = nullptr;
  a.trip_out = nullptr;
  a.bound_out = nullptr;
  a.work_list = nullptr;
  a.sample_first = nullptr;
  a.sample_res = nullptr;
  a.samples = nullptr;
  a.final_out = nullptr;
  return a;
}

template <int PREC>
struct Pol;
// BS x BS: the output block of one matrix-core product, NE of whose
// elements each lane holds.
// FP64: 4 waves (2 x 2), each 32 x 16 pairs (16x16x4 products); 64 x 32 tile
template <>
struct Pol<kFP64> {
  typedef double T;
  typedef f64x4 Acc;
  static constexpr int NA = 1, NB = 2, PITCH = 33, BM = 2, BN = 1, WM = 2, WN = 2;
  static constexpr int BS = 16, NE = 4;
};
// split precisions: 4 waves (2 x 2), one per SIMD, each 32 x 32 pairs
// (32x32x16 products); 64 x 64 tile.  A wave's accumulators (4 m groups x
// re/im plus 7 (h|h) outputs, 240 registers) sit in the accumulation
// registers; single-wave issue keeps the matrix core at its full rate.
template <>
struct Pol<kFP16X2> {
  typedef uint16_t T;
  typedef f32x16 Acc;
  static constexpr int NA = 2, NB = 2, PITCH = 32, BM = 1, BN = 1, WM = 2, WN = 2;
  static constexpr int BS = 32, NE = 16;
};
template <>
struct Pol<kBF16X2> : Pol<kFP16X2> {};

template <int PREC>
struct Tile {
  typedef Pol<PREC> P;
  static constexpr int NW = P::WM * P::WN;           // waves per workgroup
  static constexpr int NT = 64 * NW;                 // threads per workgroup
  static constexpr int TM = P::WM * P::BS * P::BM;   // rows per workgroup tile
  static constexpr int TN = P::WN * P::BS * P::BN;   // columns per workgroup tile
  static constexpr int STAGE_ELEMS = (P::NA * TM + P::NB * TN) * P::PITCH;
  static constexpr int STAGE_BYTES = STAGE_ELEMS * (int)sizeof(typename P::T);
  static constexpr int ACC_T_BYTES = (PREC == kFP64) ? 8 : 4;
  // epilogue batches: each lane offers EPB of its pairs at a time (split
  // precisions: half of them, so that half of the accumulators are free
  // while the first half is evaluated), a batch holding at most EPB per
  // lane; survivors' records (X_g re/im, the (h|h) outputs) have an odd
  // stride to spread LDS banks
  static constexpr int REC = 2 * kMaxG + kMaxNR;       // 15
  static constexpr int EPB = (PREC == kFP64) ? 2 : P::BM * P::BN * P::NE / 2;
  static constexpr int BATCH = EPB * NT;
  static constexpr int EPI_BYTES = BATCH * REC * ACC_T_BYTES;
  // LDS stage buffers: FP64 stages chunks j..j+2 through registers; the
  // split precisions load chunks straight into LDS, up to NS - 1 ahead
  static constexpr int NSB = (PREC == kFP64) ? 3 : 8;
  static constexpr int UNION_BYTES = (NSB * STAGE_BYTES > EPI_BYTES) ? NSB * STAGE_BYTES : EPI_BYTES;
  static constexpr int ROWD_OFF = (UNION_BYTES + 15) / 16 * 16;    // double [TM][4]
  static constexpr int COLD_OFF = ROWD_OFF + TM * 4 * 8;           // double [TN][3]
  static constexpr int LIST_OFF = COLD_OFF + TN * 3 * 8;           // uint16 [BATCH]
  static constexpr int RED_OFF = (LIST_OFF + BATCH * 2 + 15) / 16 * 16;   // double [NW][kNPart]
  static constexpr int CNT_OFF = RED_OFF + NW * kNPart * 8;        // (spare), u64 tile max of ln p
  static constexpr int ROWQ_OFF = CNT_OFF + 16;                    // double [TM][2]
  static constexpr int MAIN_BYTES = ROWQ_OFF + TM * 2 * 8;
  // then the distance-rule parameters and the phase table
  static constexpr int DP_OFF = (MAIN_BYTES + 15) / 16 * 16;
  static constexpr int CS_OFF = DP_OFF + ((int)sizeof(DistParams) + 15) / 16 * 16;
  static constexpr int PIECE_ELEMS = 16 / (int)sizeof(typename P::T);   // 16-byte pieces
  static constexpr int PIECES_PER_ROW = 32 / PIECE_ELEMS;
  static constexpr int PIECES = (P::NA * TM + P::NB * TN) * PIECES_PER_ROW;
  static constexpr int PIECES_PER_THREAD = PIECES / NT;
  static_assert(PIECES % NT == 0, "pieces must split evenly over the threads");
};

// wait until at most N vector-memory operations of this wave are in flight
// (expcnt and lgkmcnt left unconstrained)
// s_waitcnt immediate: vmcnt N (6 bits, split over [3:0] and [15:14]),
// expcnt unconstrained, lgkmcnt L
template <int N, int L>
constexpr int waitcnt_imm() {
  static_assert(N >= 0 && N < 64 && L >= 0 && L < 16, "waitcnt immediate");
  return (N & 0xF) | ((N >> 4) << 14) | (0x7 << 4) | (L << 8);
}
template <int N>
__device__ __forceinline__ void wait_vmcnt() {
  __builtin_amdgcn_s_waitcnt(waitcnt_imm<N, 0xF>());
}

// workgroup barrier for the LDS-load pipeline: this wave's LDS reads are
// complete and at most N of its loads into LDS are in flight; the compiler
// may not move memory operations across it.  (A full __syncthreads() would
// also wait for every load still streaming into LDS.)
template <int N>
__device__ __forceinline__ void pipeline_barrier() {
  __builtin_amdgcn_s_waitcnt(waitcnt_imm<N, 0>());
  __asm__ __volatile__("" ::: "memory");
  __builtin_amdgcn_s_barrier();
  __asm__ __volatile__("" ::: "memory");
}

// acc += a b over 16 positions (32 x 32 block): lane 32 h + r holds
// positions 8 h .. 8 h + 7 of row r of a and of column r of b
template <int PREC>
__device__ __forceinline__ void mma(typename Pol<PREC>::Acc& acc, const uint4& a, const uint4& b) {
  if constexpr (PREC == kFP16X2) {
    half8 av, bv;
    __builtin_memcpy(&av, &a, 16);
    __builtin_memcpy(&bv, &b, 16);
    acc = __builtin_amdgcn_mfma_f32_32x32x16_f16(av, bv, acc, 0, 0, 0);
  } else if constexpr (PREC == kBF16X2) {
    bf16x8 av, bv;
    __builtin_memcpy(&av, &a, 16);
    __builtin_memcpy(&bv, &b, 16);
    acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(av, bv, acc, 0, 0, 0);
  }
}

enum Mode { kEval = 0, kEvidence = 1, kPilot = 2, kBound = 3, kSurvivors = 4, kCoef = 5, kE2 = 6,
            kSample = 7 };

// The cut of an evidence pass is on when the threshold frozen after the
// pilot (state[3], the pilot's largest lnL^ML) less cut_delta is above
// zero.  Then the fast or bound pass bounds every pair and lists the tiles
// it leaves to the coefficient route; otherwise that route takes every
// tile.  Every kernel of the pass takes this decision from device memory.
// Append (ln p, i, e, best phase) to the top-k candidate buffer for the
// lanes with `want` set: one atomic per wave for all of them (the order of
// the buffer is irrelevant; it is sorted).  Called by the active lanes of
// a wave; those without a candidate pass want = false.
__device__ __forceinline__ void append_candidate(const FusedArgs& a, bool want, double lnp,
                                                 double i, double e, int ob) {
  const unsigned long long m = __ballot(want);
  if (!want) return;
  const unsigned lane = __builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0u));
  const int leader = __builtin_ctzll(m);
  unsigned long long base = 0;
  if ((int)lane == leader)
    base = atomicAdd((unsigned long long*)&a.state[2], (unsigned long long)__popcll(m));
  base = __shfl(base, leader, 64);
  const unsigned long long slot =
      base + __builtin_amdgcn_mbcnt_hi((unsigned)(m >> 32), __builtin_amdgcn_mbcnt_lo((unsigned)m, 0u));
  if ((int64_t)slot < a.cand_cap) {
    double* cd = a.cand + 4 * slot;
    cd[0] = lnp;
    cd[1] = i;
    cd[2] = e;
    cd[3] = (double)ob;
  }
}

__device__ __forceinline__ bool cut_on(const FusedArgs& a) {
  return a.cut_delta > 0.0 && __longlong_as_double(a.state[3]) - a.cut_delta > 0.0;
}
// (a sampling pass names its tiles in work_list instead)
__device__ __forceinline__ int64_t coef_work_count(const FusedArgs& a) {
  if (a.work_list) return a.n_work_list;
  return cut_on(a) ? (int64_t)a.state[4] : a.n_tiles;
}
__device__ __forceinline__ int64_t coef_tile(const FusedArgs& a, int64_t q) {
  if (a.work_list) return a.work_list[q];
  return cut_on(a) ? (int64_t)a.rerun[q] : q;
}

// Wave-wide reductions through DPP lane moves (no LDS round trips): pairs
// of lanes, quads, half rows and rows of 16 are combined within rows, then
// rows 0+1 and 2+3 by the row-15 broadcast and all four by the lane-31
// broadcast; lane 63 ends with the result, which is then read by every lane.
template <int CTRL, int ROWMASK>
__device__ __forceinline__ unsigned dpp_mov(unsigned ident, unsigned v) {
  return __builtin_amdgcn_update_dpp(ident, v, CTRL, ROWMASK, 0xF, false);
}
template <int CTRL, int ROWMASK>
__device__ __forceinline__ double dpp_mov(double ident, double v) {
  const unsigned long long bi = (unsigned long long)__double_as_longlong(ident);
  const unsigned long long bv = (unsigned long long)__double_as_longlong(v);
  const unsigned lo = dpp_mov<CTRL, ROWMASK>((unsigned)bi, (unsigned)bv);
  const unsigned hi = dpp_mov<CTRL, ROWMASK>((unsigned)(bi >> 32), (unsigned)(bv >> 32));
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}
template <int CTRL, int ROWMASK>
__device__ __forceinline__ float dpp_mov(float ident, float v) {
  return __uint_as_float(dpp_mov<CTRL, ROWMASK>(__float_as_uint(ident), __float_as_uint(v)));
}
template <int CTRL, int ROWMASK>
__device__ __forceinline__ int dpp_mov(int ident, int v) {
  return (int)dpp_mov<CTRL, ROWMASK>((unsigned)ident, (unsigned)v);
}
template <typename T, typename Op>
__device__ __forceinline__ T wave_reduce(T v, T ident, Op op) {
  v = op(v, dpp_mov<0xB1, 0xF>(ident, v));    // quad_perm 1,0,3,2
  v = op(v, dpp_mov<0x4E, 0xF>(ident, v));    // quad_perm 2,3,0,1
  v = op(v, dpp_mov<0x141, 0xF>(ident, v));   // row_half_mirror
  v = op(v, dpp_mov<0x140, 0xF>(ident, v));   // row_mirror
  v = op(v, dpp_mov<0x142, 0xA>(ident, v));   // row_bcast:15
  v = op(v, dpp_mov<0x143, 0xC>(ident, v));   // row_bcast:31
  return v;                                   // complete in lane 63
}
__device__ __forceinline__ double wave_max(double v) {
  return read_lane(wave_reduce(v, (double)-INFINITY, [](double x, double y) { return fmax(x, y); }), 63);
}

// float online log-sum-exp (for upper bounds of cut contributions)
struct LseF {
  float m, s;
  __device__ void init() { m = -INFINITY; s = 0.f; }
  // x = -inf leaves it unchanged; branch-free (one exponential)
  __device__ void add(float x) {
    const float d = x - m;
    const float t = __expf(-fabsf(d));
    const bool up = d > 0.f;
    const float ns = up ? fmaf(s, t, 1.f) : s + t;
    const float nm = up ? x : m;
    const bool skip = !(x > -INFINITY);
    s = skip ? s : ns;
    m = skip ? m : nm;
  }
  __device__ void merge(float mb, float sb) {
    const float mm = fmaxf(m, mb);
    const float sa = m == -INFINITY ? 0.f : s * __expf(m - mm);
    const float sc = mb == -INFINITY ? 0.f : sb * __expf(mb - mm);
    s = sa + sc;
    m = mm;
  }
};

// per-thread accumulators of the evidence reduction
struct EvAcc {
  Lse p;              // ln p_ie of evaluated pairs
  LseF drop;          // upper bounds of everything cut (ln)
  double ml_max;      // max lnL^ML over evaluated triples
  float max_bound;    // max over bounded pairs of ln w + bound
  int n_marg;         // kept phases evaluated
  double n_bounded, n_pairs;
  __device__ void init() {
    p.init(); drop.init();
    ml_max = 0.0; max_bound = -INFINITY;
    n_marg = 0; n_bounded = 0.0; n_pairs = 0.0;
  }
};

// phases o = o0, o0 + os, ... of one pair given X_g and the (h|h)
// coefficients: cut, distance marginalisation.  The kept phases' ln L go to
// lse, the best one to best / o_best (first of equal values), the largest
// lnL^ML to mlmax; cut phases' upper bounds go to ev.drop.  The caller
// combines the parts of one pair.  INL: the distance rule inlined (for a
// kernel whose lanes each evaluate many pairs).
// dh and hh of phase o of one pair from X_g and the (h|h) phase
// coefficients (hh clamped at zero)
template <int G>
__device__ __forceinline__ void phase_dh_hh(const FusedArgs& a, const double* lds_cs,
                                            const double2 (&X)[G], double S0,
                                            const double (&Sr)[kMaxND], const double (&Si)[kMaxND],
                                            int o, double& dh_out, double& hh_out) {
  const ModeTables& mt = a.mt;
  double dh = 0.0;
#pragma unroll
  for (int g = 0; g < G; ++g) {
    const double* cs = lds_cs + ((mt.gm[g] - 1) * a.n_phi + o) * 2;
    dh += X[g].x * cs[0] - X[g].y * cs[1];
  }
  double hh = S0;
#pragma unroll
  for (int d = 1; d < kMaxND; ++d) {
    if (d < mt.ND) {
      const double* cs = lds_cs + ((d - 1) * a.n_phi + o) * 2;
      hh += 2.0 * (Sr[d] * cs[0] + Si[d] * cs[1]);
    }
  }
  dh_out = dh;
  hh_out = fmax(hh, 0.0);
}

template <int MODE, int G, bool INL = false>
__device__ void pair_phases(const FusedArgs& a, const double* lds_cs, const DistParams& dp,
                            int64_t ie, int64_t e,
                            const double2 (&X)[G], double S0, const double (&Sr)[kMaxND],
                            const double (&Si)[kMaxND], double lnw, double thr_ml, int o0, int os,
                            EvAcc& ev, LsePh& lse, double& best, int& o_best, double& mlmax) {
  constexpr bool EVAL = MODE == kEval;
  const double thr2 = 2.0 * thr_ml;
  // the largest lnL^ML = dh^2 / (2 hh), kept as a fraction (mn / md) and
  // divided once at the end
  double mn = 0.0, md = 1.0;
  for (int o = o0; o < a.n_phi; o += os) {
    double dh, hh;
    phase_dh_hh<G>(a, lds_cs, X, S0, Sr, Si, o, dh, hh);
    if (EVAL && a.trip_out) {
      size_t t = (((size_t)ie * a.n_ext + e) * a.n_phi + o) * 2;
      a.trip_out[t] = dh;
      a.trip_out[t + 1] = hh;
    }
    const bool pos = dh > 0.0 && hh > 0.0;
    const double dh2 = dh * dh;
    if (pos && dh2 * md > mn * hh) { mn = dh2; md = hh; }
    if (MODE == kPilot) continue;
    // lnL^ML >= thr  <=>  dh > 0 and dh^2 >= 2 thr hh (no division)
    const bool keep = EVAL || thr_ml <= 0.0 || (dh > 0.0 && dh2 >= thr2 * hh);
    if (!keep) {
      const double ml = pos ? dh2 / (2.0 * hh) : 0.0;
      float x = (float)(lnw + ml - a.ln_nphi);
      ev.drop.add(x + fabsf(x) * 1e-6f + 1e-5f);   // rounding margin keeps it a bound
      continue;
    }
    double v;
    if constexpr (INL) v = dr_ln_marg_inl(dh, hh, a.r0, a.dist.tab, dp.ghx, dp.ghw);
    else v = dr_ln_marg(dh, hh, a.r0, a.dist.tab, dp.ghx, dp.ghw);
    if (v > best) { best = v; o_best = o; }
    lse.add(v);
    if (!EVAL) ev.n_marg += 1;
  }
  mlmax = fmax(mlmax, mn / (2.0 * md));
}

// The tile's partial from the per-thread accumulators: counts and maxima
// by wave reductions, evaluated and dropped mass merged lane by lane, then
// the waves' parts merged in wave order by thread 0 (a fixed order); red is
// LDS [NW][kNPart], tile_lnp_max the tile's largest ln p (ordered bits).
template <int NW>
__device__ __forceinline__ void tile_partial(const FusedArgs& a, const EvAcc& ev, int n_pairs_i,
                                             int n_bounded_i, double* red,
                                             const unsigned long long* tile_lnp_max,
                                             int64_t tile_id) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  {
    // counts and maxima: wave reductions, then one lane per wave
    auto add_i = [](int x, int y) { return x + y; };
    const int w_np = wave_reduce(n_pairs_i, 0, add_i);
    const int w_nb = wave_reduce(n_bounded_i, 0, add_i);
    const int w_nm = wave_reduce(ev.n_marg, 0, add_i);
    const double w_ml = wave_reduce(ev.ml_max, 0.0, [](double x, double y) { return fmax(x, y); });
    const float w_mb = wave_reduce(ev.max_bound, (float)-INFINITY, [](float x, float y) { return fmaxf(x, y); });
    // dropped mass: (m, s) pairs merged the same way
    float dm = ev.drop.m, ds = ev.drop.s;
    auto dmerge = [&](auto ctrl, auto rowmask) {
      constexpr int C = decltype(ctrl)::value, RM = decltype(rowmask)::value;
      LseF t{dm, ds};
      t.merge(dpp_mov<C, RM>(-INFINITY, dm), dpp_mov<C, RM>(0.f, ds));
      dm = t.m;
      ds = t.s;
    };
    dmerge(std::integral_constant<int, 0xB1>{}, std::integral_constant<int, 0xF>{});
    dmerge(std::integral_constant<int, 0x4E>{}, std::integral_constant<int, 0xF>{});
    dmerge(std::integral_constant<int, 0x141>{}, std::integral_constant<int, 0xF>{});
    dmerge(std::integral_constant<int, 0x140>{}, std::integral_constant<int, 0xF>{});
    dmerge(std::integral_constant<int, 0x142>{}, std::integral_constant<int, 0xA>{});
    dmerge(std::integral_constant<int, 0x143>{}, std::integral_constant<int, 0xC>{});
    // evaluated pairs: a few lanes of the wave at most, merged in lane order
    Lse p;
    p.init();
    unsigned long long pl = __ballot(ev.p.m != -INFINITY);
    while (pl) {
      const int src = __ffsll((long long)pl) - 1;
      p.merge(read_lane(ev.p.m, src), read_lane(ev.p.s, src), read_lane(ev.p.s2, src),
              read_lane(ev.p.s3, src));
      pl &= pl - 1;
    }
    if (lane == 63) {
      double* r = red + wave * kNPart;
      r[0] = p.m; r[1] = p.s; r[2] = p.s2;
      r[3] = dm == -INFINITY ? -INFINITY : (double)dm;
      r[4] = ds; r[5] = w_ml; r[6] = (double)w_nm; r[7] = (double)w_nb; r[8] = (double)w_mb;
      r[10] = (double)w_np; r[11] = p.s3;
    }
  }
  __syncthreads();
  if (tid == 0) {
    Lse p, d;
    p.init(); d.init();
    double mlm = 0.0, mb = -INFINITY, nm = 0, nb = 0, np_ = 0;
    for (int w = 0; w < NW; ++w) {
      const double* r = red + w * kNPart;
      p.merge(r[0], r[1], r[2], r[11]);
      d.merge(r[3], r[4], 0.0);
      mlm = fmax(mlm, r[5]);
      nm += r[6]; nb += r[7]; mb = fmax(mb, r[8]); np_ += r[10];
    }
    // every wave's E2 has finished (barrier above): the tile maximum is final
    const double mxp = order_value(*tile_lnp_max == 0ull ? 0x000fffffffffffffull : *tile_lnp_max);
    double* out = a.partials + tile_id * kNPart;
    out[0] = p.m; out[1] = p.s; out[2] = p.s2; out[3] = d.m; out[4] = d.s; out[5] = mlm;
    out[6] = nm; out[7] = nb; out[8] = mb; out[9] = mxp; out[10] = np_; out[11] = p.s3;
    // running maxima (the results are not waited for)
    if (mlm > 0.0) atomicMax((unsigned long long*)&a.state[0], (unsigned long long)__double_as_longlong(mlm));
    if (mxp > -INFINITY) atomicMax((unsigned long long*)&a.state[1], (unsigned long long)order_bits(mxp));
  }
}

// One tile (tm, tn) of the fused kernel; `slot` is the work item's place
// in the coefficient buffer (kCoef only).
template <int PREC, int G, int MODE, bool FAST>
__device__ __forceinline__ void fused_tile(const FusedArgs& a, unsigned char* smem, int64_t tm,
                                           int64_t tn, int64_t slot) {
  constexpr bool EVAL = MODE == kEval;
  // (h|h) outputs: a single m group has S0 only; otherwise up to 7, padded
  // to an even number of K blocks
  constexpr int NRT = (G == 1) ? 1 : kMaxNR;
  // (h|h) blocks after the (d|h) chunks: enough that every (d|h) step of
  // either K loop keeps its pipeline full
  constexpr int NHB = kMaxNR + 1;
  typedef Pol<PREC> P;
  typedef Tile<PREC> TL;
  typedef typename P::T T;
  typedef typename P::Acc Acc;
  constexpr int TM = TL::TM, TN = TL::TN, PITCH = P::PITCH, NT = TL::NT, NW = TL::NW;
  T* stage = (T*)smem;
  double* lds_cs = (double*)(smem + TL::CS_OFF);
  DistParams* lds_dp = (DistParams*)(smem + TL::DP_OFF);

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave / P::WN, wn = wave % P::WN;

  // partials and rerun lists are indexed by the row-major tile id
  const int64_t tile_id = tm * a.n_tiles_n + tn;
  const int64_t row0 = tm * TM, col0 = tn * TN;

  // phase table and distance-rule parameters to LDS (the rule's segment
  // search and nodes are read per triple)
  for (int t = tid; t < kMaxM * a.n_phi * 2; t += NT) lds_cs[t] = a.phase_cs[t];
  static_assert(sizeof(DistParams) % 4 == 0, "DistParams words");
  for (int t = tid; t < (int)(sizeof(DistParams) / 4); t += NT)
    ((unsigned*)lds_dp)[t] = ((const unsigned*)a.dist.prm)[t];

  // per-row / per-column scalars: issued first, stored after the first
  // chunk's loads are in flight
  double* rowd = (double*)(smem + TL::ROWD_OFF);
  double* cold = (double*)(smem + TL::COLD_OFF);
  uint16_t* list = (uint16_t*)(smem + TL::LIST_OFF);

  // per row for the E1 bound: row_scale^2 / ah_scale and ln w
  double* rowq = (double*)(smem + TL::ROWQ_OFF);
  unsigned long long* tile_lnp_max = (unsigned long long*)(smem + TL::CNT_OFF + 8);
  double rv0 = 0.0, rv1 = 1.0, rv2 = 1.0, rv3 = -1.0;
  if (tid < TM) {
    int64_t ie = row0 + tid;
    if (ie < a.n_sub) {
      int64_t i = a.sub_idx ? a.sub_idx[ie] : a.sub0 + ie;
      rv0 = a.ln_w_bank ? a.ln_w_bank[i] : 0.0;
      rv1 = PREC == kFP64 ? 1.0 : a.row_scale[i];
      rv2 = PREC == kFP64 ? 1.0 : a.ah_scale[ie];
      rv3 = (double)i;
    }
  } else if (tid < TM + TN) {
    int64_t e = col0 + (tid - TM);
    if (e < a.n_ext) {
      rv0 = a.ln_w_ext ? a.ln_w_ext[e] : 0.0;
      rv1 = PREC == kFP64 ? 1.0 : a.col_scale[e];
      rv2 = PREC == kFP64 ? 1.0 : a.bh_scale[e];
    }
  }

  // ---- K loop ----
  Acc acc[G][P::BM][P::BN][2];     // (d|h): per m group, re and im
  Acc acch[NRT][P::BM][P::BN];     // (h|h) phase coefficients
#pragma unroll
  for (int g = 0; g < G; ++g)
#pragma unroll
    for (int bm = 0; bm < P::BM; ++bm)
#pragma unroll
      for (int bn = 0; bn < P::BN; ++bn)
#pragma unroll
        for (int ri = 0; ri < 2; ++ri) acc[g][bm][bn][ri] = Acc{};

  if constexpr (PREC != kFP64) {
    // ---- split precisions: loads straight into LDS, NS buffers ----
    // A stage buffer (16 KB) holds one chunk of A hi, A lo, B hi, B lo: 4 KB
    // each, 2 row blocks x 2 slices of 1 KB, each slice copied as it sits in
    // HBM (op_index order), which is the order a fragment read wants.  Wave w
    // loads array w: its load q brings row block q / 2, slice q % 2.  Rows
    // past the subset re-read the last row (their pairs are never used).
    typedef __attribute__((address_space(1))) const unsigned char gbyte;
    typedef __attribute__((address_space(3))) void lvoid;
    constexpr int ES = (int)sizeof(T);
    constexpr int NS = TL::NSB;
    constexpr int LPC = 4;               // loads per thread per chunk
    static_assert(TL::PIECES_PER_THREAD == LPC && TL::STAGE_BYTES == 16384 && NW == 4 &&
                      P::BM == 1 && P::BN == 1 && TM == 64 && TN == 64,
                  "split staging layout");
    gbyte* srcp[LPC];
    gbyte* srch[LPC];
#pragma unroll
    for (int q = 0; q < LPC; ++q) {
      // row r of the tile; element offset of its piece lane / 32 in slice q % 2
      // of chunk 0 (a chunk adds 1024 elements)
      const int r = 32 * (q >> 1) + (lane & 31);
      const int64_t in_chunk = (q & 1) * 512 + (lane >> 5) * 256;
      auto blk = [](int64_t i, int64_t K) { return (i >> 5) * (K >> 5) * 1024 + (i & 31) * 8; };
      if (wave < 2) {
        const int64_t ie = min(row0 + r, a.n_sub - 1);
        const int64_t i = a.sub_idx ? a.sub_idx[ie] : a.sub0 + ie;
        srcp[q] = (gbyte*)(wave == 0 ? a.A0 : a.A1) + (blk(i, a.K2) + in_chunk) * ES;
        srch[q] = (gbyte*)(wave == 0 ? a.Ah0 : a.Ah1) + (blk(ie, a.KH) + in_chunk) * ES;
      } else {
        const int64_t e = col0 + r;
        srcp[q] = (gbyte*)(wave == 2 ? a.B0 : a.B1) + (blk(e, a.K2) + in_chunk) * ES;
        srch[q] = (gbyte*)(wave == 2 ? a.Bh0 : a.Bh1) + (blk(e, a.KH) + in_chunk) * ES;
      }
    }
    const int ndh = a.n_chunks;        // (d|h) chunks (a multiple of 4), then NHB (h|h) blocks
    // next chunk to load: per-thread source of each of its loads, and the
    // wave's LDS destination base (wave-uniform); chunk c goes to buffer
    // c mod NS.  The loads of chunk c follow those of c - 1, so the sources
    // advance by one chunk (2 KB) at a time and switch to the (h|h) operands
    // after the last (d|h) chunk.
    gbyte* gp[LPC];
#pragma unroll
    for (int q = 0; q < LPC; ++q) gp[q] = (ndh == 0) ? srch[q] : srcp[q];
    const unsigned lds_wave =
        __builtin_amdgcn_readfirstlane((unsigned)(uintptr_t)(lvoid*)(smem + wave * 4096));
    auto advance = [&](int c) {       // after chunk c has been issued
#pragma unroll
      for (int q = 0; q < LPC; ++q) gp[q] = (c + 1 == ndh) ? srch[q] : gp[q] + 1024 * ES;
    };
    // the loads of chunk c, issued as asm so that the compiler does not treat
    // them as pending LDS stores that every later LDS read must wait for; the
    // pipeline's own vmcnt waits order them (they have no register result).
    // M0 carries the LDS destination and the immediate offset applies to both
    // addresses, so one M0 write serves the 4 loads; the asm saves and
    // restores M0 (the compiler keeps lane indices in it elsewhere) and waits
    // the one state an M0 write needs before a load reads it.
    auto issue4 = [&](int c) {
      const unsigned m0v = lds_wave + (unsigned)((c & (NS - 1)) * TL::STAGE_BYTES);
      gbyte* p0 = gp[0];
      gbyte* p1 = gp[1] - 1024;
      gbyte* p2 = gp[2] - 2048;
      gbyte* p3 = gp[3] - 3072;
      unsigned m0_saved;
      __asm__ __volatile__(
          "s_mov_b32 %0, m0\n\ts_mov_b32 m0, %1\n\ts_nop 0\n\t"
          "global_load_lds_dwordx4 %2, off\n\t"
          "global_load_lds_dwordx4 %3, off offset:1024\n\t"
          "global_load_lds_dwordx4 %4, off offset:2048\n\t"
          "global_load_lds_dwordx4 %5, off offset:3072\n\ts_mov_b32 m0, %0"
          : "=&s"(m0_saved)
          : "s"(__builtin_amdgcn_readfirstlane(m0v)), "v"(p0), "v"(p1), "v"(p2), "v"(p3)
          : "memory");
    };
    auto issue = [&](int c) {
      issue4(c);
      advance(c);
    };
    // fragments of one chunk: A hi/lo and B_re hi/lo of both slices
    struct Frag {
      uint4 ah[2], al[2], bh[2], bl[2];
    };
    Frag fr0, fr1;
    auto frag = [&](auto fi) -> Frag& {
      if constexpr (decltype(fi)::value % 2 == 0) return fr0;
      else return fr1;
    };
    // fragment read k (0..7) of chunk c
    auto read_k = [&](Frag& f, int c, int k) {
      const unsigned char* buf = smem + (c & (NS - 1)) * TL::STAGE_BYTES + lane * 16;
      const int sl = k & 1;
      switch (k >> 1) {
        case 0: f.ah[sl] = *(const uint4*)(buf + 0 * 4096 + (2 * wm + sl) * 1024); break;
        case 1: f.al[sl] = *(const uint4*)(buf + 1 * 4096 + (2 * wm + sl) * 1024); break;
        case 2: f.bh[sl] = *(const uint4*)(buf + 2 * 4096 + (2 * wn + sl) * 1024); break;
        default: f.bl[sl] = *(const uint4*)(buf + 3 * 4096 + (2 * wn + sl) * 1024); break;
      }
    };
    auto read_frag = [&](Frag& f, int c) {
#pragma unroll
      for (int k = 0; k < 8; ++k) read_k(f, c, k);
    };
    // The matrix products of one chunk in issue order.  (d|h): with A =
    // [hr | hi] and B_re = [Br | -Bi] by slice, re += A B_re and im += A B_im,
    // B_im = [Bi | Br] = [-(B_re slice 1) | B_re slice 0]; 3 split products
    // per real product, the smaller ones first, re and im alternating.
    // (h|h) block r: the real product of the row and column (h|h) operands.
    auto mfma_dh = [&](const Frag& f, const uint4& nbh, const uint4& nbl, int g, int k) {
      Acc& re = acc[g][0][0][0];
      Acc& im = acc[g][0][0][1];
      switch (k) {
        case 0: mma<PREC>(re, f.al[0], f.bh[0]); break;
        case 1: mma<PREC>(im, f.al[0], nbh); break;
        case 2: mma<PREC>(re, f.ah[0], f.bl[0]); break;
        case 3: mma<PREC>(im, f.ah[0], nbl); break;
        case 4: mma<PREC>(re, f.ah[0], f.bh[0]); break;
        case 5: mma<PREC>(im, f.ah[0], nbh); break;
        case 6: mma<PREC>(re, f.al[1], f.bh[1]); break;
        case 7: mma<PREC>(im, f.al[1], f.bh[0]); break;
        case 8: mma<PREC>(re, f.ah[1], f.bl[1]); break;
        case 9: mma<PREC>(im, f.ah[1], f.bl[0]); break;
        case 10: mma<PREC>(re, f.ah[1], f.bh[1]); break;
        default: mma<PREC>(im, f.ah[1], f.bh[0]); break;
      }
    };
    auto mfma_hh = [&](const Frag& f, int r, int k) {
      Acc& h = acch[r][0][0];
      const int sl = k / 3;
      switch (k % 3) {
        case 0: mma<PREC>(h, f.al[sl], f.bh[sl]); break;
        case 1: mma<PREC>(h, f.ah[sl], f.bl[sl]); break;
        default: mma<PREC>(h, f.ah[sl], f.bh[sl]); break;
      }
    };
    // Pipeline: NS buffers; the loads of chunk c are issued at step c + 1 -
    // NS (the first NS - 1 chunks before step 0), into the buffer of chunk
    // c - NS, whose fragments were read at step c - NS - 1 (before the last
    // barrier).  Step j multiplies chunk j and reads the fragments of chunk
    // j + 1 between its products (one wave per SIMD issues everything, so
    // LDS reads and loads go where a product is running).  A barrier after
    // every second step (j odd) makes chunks up to j + 3 visible to all
    // waves and frees the buffers read so far.
    auto fence = [] { __builtin_amdgcn_sched_barrier(0); };
    // FL: 1 read ahead, 2 issue, 4 barrier after; W: loads allowed in flight
    // at that barrier; NMF: products; O: the slot after which the loads go
    auto step = [&](int j, auto slot, auto fl, auto w, auto nmf, auto off, auto&& mfma_k) {
      constexpr int sl = decltype(slot)::value;
      constexpr int FL = decltype(fl)::value;
      constexpr int NMF = decltype(nmf)::value;
      constexpr int O = decltype(off)::value;
      Frag& cur = frag(slot);
      Frag& nxt = frag(std::integral_constant<int, sl + 1>{});
      const int ci = j - 1 + NS;      // chunk issued in this step
      // slot t (0 .. max(NMF, 8) - 1): product t, then read t; the chunk's
      // loads go after slot O
      constexpr int NSLOT = NMF > 8 ? NMF : 8;
      static_for<NSLOT>([&](auto ti) {
        constexpr int t = decltype(ti)::value;
        if constexpr (t < NMF) mfma_k(cur, t);
        if constexpr ((FL & 1) && t < 8) read_k(nxt, j + 1, t);
        if constexpr ((FL & 2) && t == O) {   // the chunk's loads after product O
          fence();
          issue4(ci);
          fence();
        }
      });
      if constexpr (FL & 2) advance(ci);
      if constexpr (FL & 4) pipeline_barrier<decltype(w)::value>();
    };
    // prologue: chunks 0 .. NS-2 in flight; wait for 0, 1, 2; read chunk 0
    static_for<NS - 1>([&](auto q) { issue(decltype(q)::value); });
    if (tid < TM) {
      rowd[tid * 4] = rv0; rowd[tid * 4 + 1] = rv1; rowd[tid * 4 + 2] = rv2; rowd[tid * 4 + 3] = rv3;
      rowq[tid * 2] = rv1 * rv1 / rv2; rowq[tid * 2 + 1] = rv0;
    } else if (tid < TM + TN) {
      cold[(tid - TM) * 3] = rv0; cold[(tid - TM) * 3 + 1] = rv1; cold[(tid - TM) * 3 + 2] = rv2;
    }
    if (tid == 0) *tile_lnp_max = 0ull;
    __syncthreads();                              // rowd, cold, counters
    pipeline_barrier<LPC * (NS - 4)>();           // chunks 0, 1, 2 have landed
    read_frag(fr0, 0);
    pipeline_barrier<LPC * (NS - 4)>();           // chunk 0 read everywhere (step 1 refills it)
    // every group spans a multiple of 4 chunks (bins padded to 64), so the
    // fragment set and the barrier of each step are static; with at least
    // NS (h|h) blocks after them every (d|h) step reads ahead and issues
    static_assert(NHB >= NS && NS >= 4, "pipeline needs NS trailing blocks");
    int ch = 0;
    static_for<G>([&](auto gi) {
      constexpr int g = decltype(gi)::value;
      const int gend = a.mt.gk0[g + 1];
      auto run = [&](auto off) {
        for (; ch < gend; ch += 4) {
          // B_im slice 0 is minus B_re slice 1: the sign flips are formed per step
          static_for<4>([&](auto slot) {
            constexpr int s4 = decltype(slot)::value;
            const Frag& f = frag(slot);
            const uint4 nbh = make_uint4(f.bh[1].x ^ 0x80008000u, f.bh[1].y ^ 0x80008000u,
                                         f.bh[1].z ^ 0x80008000u, f.bh[1].w ^ 0x80008000u);
            const uint4 nbl = make_uint4(f.bl[1].x ^ 0x80008000u, f.bl[1].y ^ 0x80008000u,
                                         f.bl[1].z ^ 0x80008000u, f.bl[1].w ^ 0x80008000u);
            step(ch + s4, slot, std::integral_constant<int, 3 | (s4 & 1 ? 4 : 0)>{},
                 std::integral_constant<int, LPC * (NS - 4)>{}, std::integral_constant<int, 12>{},
                 off, [&](const Frag& fc, int k) { mfma_dh(fc, nbh, nbl, g, k); });
          });
        }
      };
      run(std::integral_constant<int, 2>{});
    });
#pragma unroll
    for (int r = 0; r < NRT; ++r) acch[r][0][0] = Acc{};
    static_for<NHB>([&](auto ri) {
      constexpr int r = decltype(ri)::value;
      // reads ahead while a block follows; issues while one is left to load;
      // barrier after odd steps (ndh is even) with blocks r+4 .. last in flight
      constexpr int fl = (r + 1 < NHB ? 1 : 0) | (r + NS - 1 < NHB ? 2 : 0) | (r % 2 ? 4 : 0);
      constexpr int last = (r + NS - 1 < NHB - 1) ? r + NS - 1 : NHB - 1;
      constexpr int wc = LPC * (last > r + 3 ? last - r - 3 : 0);
      step(ndh + r, std::integral_constant<int, r % 4>{}, std::integral_constant<int, fl>{},
           std::integral_constant<int, wc>{}, std::integral_constant<int, (r < NRT ? 6 : 0)>{},
           std::integral_constant<int, 2>{}, [&](const Frag& fc, int k) { mfma_hh(fc, r, k); });
    });
  } else {
  // per-thread source addresses of its 16-byte pieces for chunk 0 of the
  // (d|h) operands (srcp) and block 0 of the (h|h) operands (srch), in the
  // global address space so that the loads wait on the vector-memory counter
  // only.  Rows past the subset re-read the last row (their pairs are never
  // used) and the FP64 B_im slot of an (h|h) block re-reads B_re (the block
  // does not use it), so no load is predicated.
  typedef __attribute__((address_space(1))) const unsigned char gbyte;
  typedef unsigned u32x4 __attribute__((ext_vector_type(4)));
  typedef __attribute__((address_space(1))) const u32x4 gu4;
  gbyte* srcp[TL::PIECES_PER_THREAD];
  gbyte* srch[TL::PIECES_PER_THREAD];
  {
    constexpr int ES = (int)sizeof(T);
#pragma unroll
    for (int q = 0; q < TL::PIECES_PER_THREAD; ++q) {
      int p = tid + NT * q;
      int rowsel = p / TL::PIECES_PER_ROW, piece = p % TL::PIECES_PER_ROW;
      if (rowsel < P::NA * TM) {
        int arr = rowsel / TM, r = rowsel % TM;
        int64_t ie = min(row0 + r, a.n_sub - 1);
        int64_t i = a.sub_idx ? a.sub_idx[ie] : a.sub0 + ie;
        srcp[q] = (gbyte*)(arr == 0 ? a.A0 : a.A1) + (i * a.K2 + piece * TL::PIECE_ELEMS) * ES;
        srch[q] = (gbyte*)(arr == 0 ? a.Ah0 : a.Ah1) + (ie * a.KH + piece * TL::PIECE_ELEMS) * ES;
      } else {
        int rs = rowsel - P::NA * TM;
        int arr = rs / TN, c = rs % TN;
        srcp[q] = (gbyte*)(arr == 0 ? a.B0 : a.B1) + ((col0 + c) * a.K2 + piece * TL::PIECE_ELEMS) * ES;
        srch[q] = (gbyte*)a.Bh0 + ((col0 + c) * a.KH + piece * TL::PIECE_ELEMS) * ES;
      }
    }
  }
  const int ndh = a.n_chunks;        // (d|h) chunks (a multiple of 4)
  const int nch = ndh + NHB;         // then the (h|h) blocks
  constexpr int ES = (int)sizeof(T);
  // R = 2 register stage sets (set c mod 2 holds chunk c): loads run two
  // chunks ahead, as many as the register file holds at this tile size.
  // Separate arrays picked at compile time keep them in registers.
  constexpr int R = 2;
  u32x4 st0[TL::PIECES_PER_THREAD], st1[TL::PIECES_PER_THREAD];
  auto set = [&](auto slot) -> u32x4* {
    if constexpr (decltype(slot)::value % R == 0) return st0;
    else return st1;
  };
  // chunk c into a stage set: a (d|h) chunk for c < ndh, else (h|h) block c - ndh
  auto load = [&](u32x4* stq, int c) {
    const bool hh = c >= ndh;
    const int64_t od = (int64_t)c * 32 * ES, oh = (int64_t)(c - ndh) * 32 * ES;
#pragma unroll
    for (int q = 0; q < TL::PIECES_PER_THREAD; ++q) {
      gbyte* pq = hh ? srch[q] + oh : srcp[q] + od;
      stq[q] = *(gu4*)pq;
    }
  };
  auto store_from = [&](const u32x4* st, T* base) {
#pragma unroll
    for (int q = 0; q < TL::PIECES_PER_THREAD; ++q) {
      int p = tid + NT * q;
      int rowsel = p / TL::PIECES_PER_ROW, piece = p % TL::PIECES_PER_ROW;
      // the odd pitch keeps doubles 8-byte aligned only
      typedef unsigned u32x2 __attribute__((ext_vector_type(2)));
      u32x2* d2 = (u32x2*)(base + rowsel * PITCH + piece * TL::PIECE_ELEMS);
      d2[0] = st[q].xy;
      d2[1] = st[q].zw;
    }
  };
  // (d|h) chunk: complex product from the LDS buffer, one FP64 product per
  // real product
  auto compute_dh = [&](const T* base, auto gi) {
    constexpr int g = decltype(gi)::value;
    const double* Ad = (const double*)base;
    const double* Bd = (const double*)(base + P::NA * TM * PITCH);
#pragma unroll
    for (int s8 = 0; s8 < 8; ++s8) {
      double av[P::BM], brv[P::BN], biv[P::BN];
#pragma unroll
      for (int bm = 0; bm < P::BM; ++bm)
        av[bm] = Ad[(wm * 16 * P::BM + bm * 16 + (lane & 15)) * PITCH + 4 * s8 + (lane >> 4)];
#pragma unroll
      for (int bn = 0; bn < P::BN; ++bn) {
        int cc = wn * 16 * P::BN + bn * 16 + (lane & 15);
        brv[bn] = Bd[cc * PITCH + 4 * s8 + (lane >> 4)];
        biv[bn] = Bd[(TN + cc) * PITCH + 4 * s8 + (lane >> 4)];
      }
#pragma unroll
      for (int bm = 0; bm < P::BM; ++bm)
#pragma unroll
        for (int bn = 0; bn < P::BN; ++bn) {
          acc[g][bm][bn][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[bm], brv[bn], acc[g][bm][bn][0], 0, 0, 0);
          acc[g][bm][bn][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[bm], biv[bn], acc[g][bm][bn][1], 0, 0, 0);
        }
    }
  };
  // (h|h) block r: real product of the row and column (h|h) operands
  auto compute_hh = [&](const T* base, auto ri) {
    constexpr int r = decltype(ri)::value;
    if constexpr (r < NRT) {
      const double* Ad = (const double*)base;
      const double* Bd = (const double*)(base + P::NA * TM * PITCH);
#pragma unroll
      for (int s8 = 0; s8 < 8; ++s8) {
        double av[P::BM], bv[P::BN];
#pragma unroll
        for (int bm = 0; bm < P::BM; ++bm)
          av[bm] = Ad[(wm * 16 * P::BM + bm * 16 + (lane & 15)) * PITCH + 4 * s8 + (lane >> 4)];
#pragma unroll
        for (int bn = 0; bn < P::BN; ++bn)
          bv[bn] = Bd[(wn * 16 * P::BN + bn * 16 + (lane & 15)) * PITCH + 4 * s8 + (lane >> 4)];
#pragma unroll
        for (int bm = 0; bm < P::BM; ++bm)
#pragma unroll
          for (int bn = 0; bn < P::BN; ++bn)
            acch[r][bm][bn] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[bm], bv[bn], acch[r][bm][bn], 0, 0, 0);
      }
    }
  };

  // Pipeline over chunks, LDS buffers rotating with the chunk index (chunk c
  // sits in buffer c mod 3 from step c-2 to step c).  Step j: multiply chunk
  // j, write chunk j+2 from its stage set and refill that set with chunk
  // j+2+R, then one barrier.  The global loads of chunk j+2+R are in flight
  // over the products of R steps.
  T* buf_c = stage;                          // chunk j
  T* buf_r = stage + TL::STAGE_ELEMS;        // chunk j+1
  T* buf_w = stage + 2 * TL::STAGE_ELEMS;    // chunk j+2
  static_for<R>([&](auto q) { load(set(q), decltype(q)::value); });
  if (tid < TM) {
    rowd[tid * 4] = rv0; rowd[tid * 4 + 1] = rv1; rowd[tid * 4 + 2] = rv2; rowd[tid * 4 + 3] = rv3;
    rowq[tid * 2] = rv1 * rv1 / rv2; rowq[tid * 2 + 1] = rv0;
  } else if (tid < TM + TN) {
    cold[(tid - TM) * 3] = rv0; cold[(tid - TM) * 3 + 1] = rv1; cold[(tid - TM) * 3 + 2] = rv2;
  }
  if (tid == 0) *tile_lnp_max = 0ull;
  store_from(set(std::integral_constant<int, 0>{}), buf_c);
  store_from(set(std::integral_constant<int, 1>{}), buf_r);
  if (R < nch) load(set(std::integral_constant<int, 0>{}), R);
  if (R + 1 < nch) load(set(std::integral_constant<int, 1>{}), R + 1);
  __syncthreads();
  // flags: 2 write chunk j+2, 4 refill its stage set
  auto step = [&](int j, auto slot, auto flags, auto&& compute_fn) {
    constexpr int sl = decltype(slot)::value;
    constexpr int FL = decltype(flags)::value;
    compute_fn((const T*)buf_c);
    if constexpr (FL & 2) {
      u32x4* sw = set(std::integral_constant<int, sl + 2>{});
      store_from(sw, buf_w);
      if constexpr (FL & 4) load(sw, j + 2 + R);
    }
    __syncthreads();
    T* t = buf_c;
    buf_c = buf_r;
    buf_r = buf_w;
    buf_w = t;
  };
  // every group spans a multiple of 4 chunks (bins padded to 64), so the
  // stage set (j mod R) of each step is static; with NHB >= R + 2 (h|h)
  // blocks after them, every (d|h) step writes and refills
  int ch = 0;
  static_for<G>([&](auto gi) {
    constexpr int g = decltype(gi)::value;
    const int gend = a.mt.gk0[g + 1];
    for (; ch < gend; ch += 4) {
      static_for<4>([&](auto slot) {
        step(ch + decltype(slot)::value, slot, std::integral_constant<int, 6>{},
             [&](const T* base) { compute_dh(base, gi); });
      });
    }
  });
  // the (h|h) accumulators only live from here on
#pragma unroll
  for (int r = 0; r < NRT; ++r)
#pragma unroll
    for (int bm = 0; bm < P::BM; ++bm)
#pragma unroll
      for (int bn = 0; bn < P::BN; ++bn) acch[r][bm][bn] = Acc{0, 0, 0, 0};
  static_for<NHB>([&](auto ri) {
    constexpr int r = decltype(ri)::value;
    constexpr int fl = (r + 2 < NHB ? 2 : 0) | (r + 2 + R < NHB ? 4 : 0);
    step(ndh + r, std::integral_constant<int, r % 4>{}, std::integral_constant<int, fl>{},
         [&](const T* base) { compute_hh(base, ri); });
  });
  }

  // ---- epilogue ----
  typedef typename std::conditional<PREC == kFP64, double, float>::type AT;
  // output element r of a lane's accumulator block sits in row rowmap(r),
  // column lane mod BS (16x16x4 FP64 and 32x32x16 split-precision layouts)
  auto rowmap = [&](int r) {
    return (PREC == kFP64) ? ((lane >> 4) + 4 * r) : (8 * (r >> 2) + 4 * (lane >> 5) + (r & 3));
  };
  constexpr int BS = P::BS, NE = P::NE;
  if constexpr (MODE == kCoef) {
    // the raw accumulators to the coefficient buffer, as the accumulator
    // type: component-major, pairs row-major (a row of a block is BS
    // consecutive elements)
    constexpr int NCO = 2 * G + NRT, NPT = TM * TN;
    AT* cf = (AT*)a.coef + slot * (int64_t)(NCO * NPT);
#pragma unroll
    for (int bm = 0; bm < P::BM; ++bm)
#pragma unroll
      for (int bn = 0; bn < P::BN; ++bn) {
        const int tc = wn * BS * P::BN + bn * BS + (lane & (BS - 1));
#pragma unroll
        for (int r = 0; r < NE; ++r) {
          const int tr = wm * BS * P::BM + bm * BS + rowmap(r);
          AT* o = cf + tr * TN + tc;
#pragma unroll
          for (int g = 0; g < G; ++g) {
            o[(2 * g) * NPT] = (AT)acc[g][bm][bn][0][r];
            o[(2 * g + 1) * NPT] = (AT)acc[g][bm][bn][1][r];
          }
#pragma unroll
          for (int q = 0; q < NRT; ++q) o[(2 * G + q) * NPT] = (AT)acch[q][bm][bn][r];
        }
      }
    return;
  }
  double thr_ml = -INFINITY, thr_topk_glob = -INFINITY;
  if (MODE == kEvidence) {
    // the cut threshold is the one frozen after the pilot pass, so which
    // triples are cut does not depend on the order in which tiles finish
    if (a.cut_delta > 0.0) thr_ml = __longlong_as_double(a.state[3]) - a.cut_delta;
    thr_topk_glob = order_value(a.state[1]) - a.topk_window;
  }
  // the pilot only needs pairs that can raise the running maximum
  if (MODE == kPilot) thr_ml = __longlong_as_double(a.state[0]);
  const bool use_bound = MODE != kEval && thr_ml > 0.0;
  const float thr_f = (float)thr_ml;
  EvAcc ev;
  ev.init();
  int n_pairs_i = 0, n_bounded_i = 0;
  AT* recs = (AT*)smem;                  // [BATCH][REC] survivors' records
  constexpr int XO = 0, SO = 2 * G;      // offsets of X and S in a record
  // per column of this lane for the E1 bound: col_scale^2 / bh_scale and ln w
  double colq[P::BN], colw[P::BN];
#pragma unroll
  for (int bn = 0; bn < P::BN; ++bn) {
    const int tc = wn * BS * P::BN + bn * BS + (lane & (BS - 1));
    colq[bn] = cold[tc * 3 + 1] * cold[tc * 3 + 1] / cold[tc * 3 + 2];
    colw[bn] = cold[tc * 3];
  }

  // E1 for the pair in element r of block (bm, bn) of this lane, straight
  // from the accumulators: the certified bound on lnL^ML, bounded pairs into
  // the dropped mass; true for a survivor (no shared-memory writes, so that
  // the elements' loads and arithmetic overlap)
  // rows and columns of the tile inside the subset and the sample set
  const int rows_in = (int)min((int64_t)TM, a.n_sub - row0);
  const int cols_in = (int)min((int64_t)TN, a.n_ext - col0);
  // UB: use_bound, known at compile time where the caller knows it
  auto e1_bound = [&](auto bmi, auto bni, auto ri, auto ub) -> bool {
    constexpr int bm = decltype(bmi)::value, bn = decltype(bni)::value, r = decltype(ri)::value;
    constexpr bool UB = decltype(ub)::value;
    const int tc = wn * BS * P::BN + bn * BS + (lane & (BS - 1));
    const int tr = wm * BS * P::BM + bm * BS + rowmap(r);
    const bool in = tc < cols_in && tr < rows_in;
    n_pairs_i += in ? 1 : 0;
    if constexpr (!UB) return in;
    // bound = (sx^2 / sh) U0^2 / (2 lo0) from the raw accumulators:
    // U0 = sum_g |X_g|, and hh_o >= S0 - 2 sum_d |S_d| for every phase (the
    // margin, relative to the magnitudes involved, covers FP32 accumulation
    // and sqrt rounding even when the difference cancels); lnL^ML_o <=
    // U^2 / (2 lo) for every phase.  sx^2 / sh is a power of two.
    float U0 = 0.f;
#pragma unroll
    for (int g = 0; g < G; ++g) {
      const float xr = (float)acc[g][bm][bn][0][r], xi = (float)acc[g][bm][bn][1][r];
      U0 += __builtin_amdgcn_sqrtf(xr * xr + xi * xi);
    }
    const float s0 = (float)acch[0][bm][bn][r];
    float sabs = 0.f;
#pragma unroll
    for (int d = 1; d < (NRT + 1) / 2; ++d) {   // outputs past ND are zero
      const float sr = (float)acch[2 * d - 1][bm][bn][r], si = (float)acch[2 * d][bm][bn][r];
      sabs += 2.f * __builtin_amdgcn_sqrtf(sr * sr + si * si);
    }
    const float lo0 = (s0 - sabs) - 2e-5f * (fabsf(s0) + sabs);
    const float q = (float)(rowq[tr * 2] * colq[bn]);
    // rcp is within an ulp; the 1.001 factor covers it
    const float bound = q * (U0 * U0) * __builtin_amdgcn_rcpf(2.f * lo0) * 1.001f + 1e-3f;
    const bool bounded = in && lo0 > 0.f && bound < thr_f;
    if (MODE == kEvidence) {
      const float lw = (float)(rowq[tr * 2 + 1] + colw[bn]);
      ev.drop.add(bounded ? lw + bound : -INFINITY);
      ev.max_bound = bounded ? fmaxf(ev.max_bound, lw + bound) : ev.max_bound;
      n_bounded_i += bounded ? 1 : 0;
    }
    return in && !bounded;
  };
  // a survivor's record into LDS slot `slot` (slots past BATCH are counted
  // but not written)
  auto e1_record = [&](auto bmi, auto bni, auto ri, int slot) {
    constexpr int bm = decltype(bmi)::value, bn = decltype(bni)::value, r = decltype(ri)::value;
    const int tc = wn * BS * P::BN + bn * BS + (lane & (BS - 1));
    const int tr = wm * BS * P::BM + bm * BS + rowmap(r);
    if (slot < TL::BATCH) {
      AT* rec = recs + slot * TL::REC;
#pragma unroll
      for (int g = 0; g < G; ++g) {
        rec[XO + 2 * g] = (AT)acc[g][bm][bn][0][r];
        rec[XO + 2 * g + 1] = (AT)acc[g][bm][bn][1][r];
      }
#pragma unroll
      for (int q = 0; q < NRT; ++q) rec[SO + q] = (AT)acch[q][bm][bn][r];
      list[slot] = (uint16_t)((tr << 8) | tc);
    }
  };
  // Survivor slots in a fixed order -- wave by wave, within a wave by
  // element (bit of `mask`) then lane -- so that which lane evaluates which
  // survivor, and with it the order of every floating-point sum, does not
  // depend on timing.  slot_base returns this wave's first slot and the
  // tile's total (one barrier; the per-wave counts use the tile-reduction
  // area, which is free until the end); record_all then hands bit k of each
  // lane its slot.
  int* wcnt = (int*)(smem + TL::RED_OFF);
  auto slot_base = [&](unsigned mask, auto nbits, int& total) -> int {
    constexpr int NB = decltype(nbits)::value;
    int cnt = 0;
    static_for<NB>([&](auto ki) {
      cnt += (int)__popcll(__ballot((mask >> decltype(ki)::value) & 1u));
    });
    if (lane == 0) wcnt[wave] = cnt;
    __syncthreads();
    int base = 0;
    total = 0;
#pragma unroll
    for (int w = 0; w < NW; ++w) {
      const int c = wcnt[w];
      base += w < wave ? c : 0;
      total += c;
    }
    return base;
  };
  auto record_all = [&](unsigned mask, int base, auto nbits, auto&& rec_k) {
    constexpr int NB = decltype(nbits)::value;
    int run = base;
    static_for<NB>([&](auto ki) {
      constexpr int k = decltype(ki)::value;
      const unsigned long long b = __ballot((mask >> k) & 1u);
      if ((mask >> k) & 1u)
        rec_k(ki, run + (int)__builtin_amdgcn_mbcnt_hi((unsigned)(b >> 32),
                                                       __builtin_amdgcn_mbcnt_lo((unsigned)b, 0u)));
      run += (int)__popcll(b);
    });
  };
  // E2: the survivors' full evaluation.  With few survivors the phases of
  // one survivor are spread over a group of 32 lanes (phase o on lane o mod
  // 32) and combined by shuffles within the group, the groups taking
  // survivors in turn; with many, each lane takes whole survivors.
  auto e2_run = [&](int nsurv, auto lps) {
    constexpr int LPS = decltype(lps)::value;      // lanes per survivor
    constexpr int NGRP = NT / LPS;
    const int grp = tid / LPS, gl = tid % LPS;
    for (int j = grp; j < nsurv; j += NGRP) {
      const int tr = list[j] >> 8, tcs = list[j] & 255;
      const int64_t ie = row0 + tr, e = col0 + tcs;
      const AT* xq = recs + j * TL::REC;
      double sx = rowd[tr * 4 + 1] * cold[tcs * 3 + 1];
      double sh = rowd[tr * 4 + 2] * cold[tcs * 3 + 2];
      double2 X[G];
#pragma unroll
      for (int g = 0; g < G; ++g)
        X[g] = make_double2(sx * (double)xq[XO + 2 * g], sx * (double)xq[XO + 2 * g + 1]);
      double S0 = sh * (double)xq[SO], Sr[kMaxND], Si[kMaxND];
#pragma unroll
      for (int d = 0; d < kMaxND; ++d) { Sr[d] = 0.0; Si[d] = 0.0; }
#pragma unroll
      for (int d = 1; d < (NRT + 1) / 2; ++d) {
        Sr[d] = sh * (double)xq[SO + 2 * d - 1];
        Si[d] = sh * (double)xq[SO + 2 * d];
      }
      double lnw = rowd[tr * 4] + cold[tcs * 3];
      LsePh lse;
      lse.init();
      double best = -INFINITY, mlmax = 0.0;
      int ob = 0;
      pair_phases<MODE, G>(a, lds_cs, *lds_dp, ie, e, X, S0, Sr, Si, lnw, thr_ml, gl, LPS, ev, lse,
                           best, ob, mlmax);
#pragma unroll
      for (int off = LPS / 2; off > 0; off >>= 1) {
        const double lm = __shfl_xor(lse.m, off, LPS), ls = __shfl_xor(lse.s, off, LPS);
        const double ls2 = __shfl_xor(lse.s2, off, LPS);
        lse.merge(lm, ls, ls2);
        const double bv = __shfl_xor(best, off, LPS);
        const int bo = __shfl_xor(ob, off, LPS);
        if (bv > best || (bv == best && bo < ob)) { best = bv; ob = bo; }
        mlmax = fmax(mlmax, __shfl_xor(mlmax, off, LPS));
      }
      if (gl != 0) continue;
      const double lnl = (lse.m == -INFINITY) ? -INFINITY : lse.m + log(lse.s) - a.ln_nphi;
      if (EVAL) {
        const size_t t = (size_t)ie * a.n_ext + e;
        a.lnl_out[t] = lnl;
        if (a.ml_out) a.ml_out[t] = mlmax;
        continue;
      }
      ev.ml_max = fmax(ev.ml_max, mlmax);
      if (MODE == kPilot || lnl == -INFINITY) continue;
      const double lnp = lnw + lnl;
      ev.p.add(lnp, lse.sq_ratio());
      if (MODE == kEvidence) {
        unsigned long long ob_bits = order_bits(lnp);
        unsigned long long prev = atomicMax(tile_lnp_max, ob_bits);
        double tmax = order_value(prev > ob_bits ? prev : ob_bits);
        double thr_k = fmax(thr_topk_glob, tmax - a.topk_window);
        append_candidate(a, lnp >= thr_k, lnp, rowd[tr * 4 + 3], (double)e, ob);
      }
    }
  };
  auto e2_list = [&](int nsurv) {
    if (nsurv >= NT / 2) e2_run(nsurv, std::integral_constant<int, 1>{});
    else e2_run(nsurv, std::integral_constant<int, 32>{});
  };

  if constexpr (FAST) {
    // every pair of the tile through E1 first, then one E2 once the
    // accumulators are dead.  A tile with more survivors than the record
    // area holds is left to the coefficient route: it is listed and
    // contributes nothing here.
    static_assert(P::BM * P::BN * NE <= 32, "survivor mask");
    unsigned sm = 0;
    static_for<P::BM>([&](auto bmi) {
      static_for<P::BN>([&](auto bni) {
        static_for<NE>([&](auto ri) {
          constexpr int k = (decltype(bmi)::value * P::BN + decltype(bni)::value) * NE + decltype(ri)::value;
          // the fast pass always cuts (threshold frozen above zero)
          if (e1_bound(bmi, bni, ri, std::true_type{})) sm |= 1u << k;
        });
      });
    });
    constexpr int NK = P::BM * P::BN * NE;
    int nsurv = 0;
    const int base = slot_base(sm, std::integral_constant<int, NK>{}, nsurv);
    record_all(sm, base, std::integral_constant<int, NK>{}, [&](auto ki, int slot) {
      constexpr int k = decltype(ki)::value;
      e1_record(std::integral_constant<int, k / NE / P::BN>{},
                std::integral_constant<int, k / NE % P::BN>{}, std::integral_constant<int, k % NE>{},
                slot);
    });
    __syncthreads();
    if (nsurv > min(a.rec_cap, TL::BATCH)) {
      if (tid == 0) {
        unsigned long long k = atomicAdd((unsigned long long*)&a.state[4], 1ull);
        a.rerun[k] = (int)tile_id;
      }
      return;
    }
    e2_list(nsurv);
  } else {
    // batches of EPB pairs per lane (at most BATCH survivors each)
    constexpr int EPB = TL::EPB;
    static_assert(NE % EPB == 0 || EPB % NE == 0, "batch split");
    static_assert(EPB <= 32, "survivor mask");
    static_for<P::BM * P::BN * NE / EPB>([&](auto bi) {
      constexpr int k0 = decltype(bi)::value * EPB;
      // element k0 + q of this lane in (block, element) order
      unsigned sm = 0;
      static_for<EPB>([&](auto qi) {
        constexpr int k = k0 + decltype(qi)::value;
        const auto bmi = std::integral_constant<int, k / NE / P::BN>{};
        const auto bni = std::integral_constant<int, k / NE % P::BN>{};
        const auto rr = std::integral_constant<int, k % NE>{};
        const bool surv = use_bound ? e1_bound(bmi, bni, rr, std::true_type{})
                                    : e1_bound(bmi, bni, rr, std::false_type{});
        if (surv) sm |= 1u << decltype(qi)::value;
      });
      int nsurv = 0;
      const int base = slot_base(sm, std::integral_constant<int, EPB>{}, nsurv);
      record_all(sm, base, std::integral_constant<int, EPB>{}, [&](auto qi, int slot) {
        constexpr int k = k0 + decltype(qi)::value;
        e1_record(std::integral_constant<int, k / NE / P::BN>{},
                  std::integral_constant<int, k / NE % P::BN>{},
                  std::integral_constant<int, k % NE>{}, slot);
      });
      __syncthreads();
      e2_list(min(nsurv, TL::BATCH));
      __syncthreads();
    });
  }
  if (EVAL) return;
  if (MODE == kPilot) {
    double mlm = wave_max(ev.ml_max);
    if (lane == 0)
      atomicMax((unsigned long long*)&a.state[0], (unsigned long long)__double_as_longlong(mlm));
    return;
  }
  ev.n_pairs = (double)n_pairs_i;
  ev.n_bounded = (double)n_bounded_i;

  // ---- tile reduction ----
  tile_partial<NW>(a, ev, n_pairs_i, n_bounded_i, (double*)(smem + TL::RED_OFF), tile_lnp_max,
                   tile_id);
}

// workgroup blk of a grid of nblk (a multiple of 8 outside the coefficient
// route) -> its tile or tiles
template <int PREC, int G, int MODE, bool FAST>
__device__ __forceinline__ void fused_grid_tile(const FusedArgs& a, unsigned char* smem,
                                                int64_t wg_id, int64_t wg_count) {
  if constexpr (MODE == kCoef) {
    // coefficient route: the workgroups take the chunk's work items in turn
    const int64_t end = min(a.work0 + a.coef_tiles, coef_work_count(a));
    for (int64_t q = a.work0 + wg_id; q < end; q += wg_count) {
      const int64_t t = coef_tile(a, q);
      fused_tile<PREC, G, MODE, FAST>(a, smem, t / a.n_tiles_n, t % a.n_tiles_n, q - a.work0);
      __syncthreads();
    }
  } else {
    // the fast pass only runs when the cut is on
    if (MODE == kEvidence && FAST && !cut_on(a)) return;
    // workgroup -> tile: spread consecutive ids over the XCDs so that each
    // XCD walks a contiguous band of tiles, then raster in bands of 4 tile
    // rows (the ~32 tiles an XCD runs at once then share 4 row blocks and 8
    // column blocks of operands in its L2)
    int64_t wg = wg_id;
    int64_t tm, tn;
    const int64_t nwg = wg_count;                   // multiple of 8
    wg = (wg % 8) * (nwg / 8) + wg / 8;
    if (MODE == kPilot) {
      // every pilot_stride-th row of tiles, all columns
      const int64_t npr = (a.n_tiles_m + a.pilot_stride - 1) / a.pilot_stride;
      if (wg >= npr * a.n_tiles_n) return;
      tm = (wg / a.n_tiles_n) * a.pilot_stride;
      tn = wg % a.n_tiles_n;
    } else {
      if (wg >= a.n_tiles) return;
      const int64_t GM = 4;
      const int64_t band = wg / (GM * a.n_tiles_n);
      const int64_t rows_in_band = min(GM, a.n_tiles_m - band * GM);
      const int64_t in = wg - band * GM * a.n_tiles_n;
      tm = band * GM + in % rows_in_band;
      tn = in / rows_in_band;
    }
    fused_tile<PREC, G, MODE, FAST>(a, smem, tm, tn, 0);
  }
}

template <int PREC, int G, int MODE, bool FAST>
__global__ __launch_bounds__(Tile<PREC>::NT) void k_lnl_fused(FusedArgs a) {
  extern __shared__ __align__(16) unsigned char smem[];
  fused_grid_tile<PREC, G, MODE, FAST>(a, smem, blockIdx.x, gridDim.x);
}

// the pilot, the fast pass or one chunk of the coefficient route of several
// events in one launch
template <int PREC, int G, int MODE, bool FAST>
__global__ __launch_bounds__(Tile<PREC>::NT) void k_lnl_fused_packed(PackLaunch p) {
  extern __shared__ __align__(16) unsigned char smem[];
  int64_t blk, nblk;
  int q;
  const int e = pack_locate(p, blockIdx.x, &blk, &nblk, &q);
  FusedArgs a = pack_args(p, e, q);
  if (MODE == kCoef) a.work0 = p.chunk * a.coef_tiles;
  fused_grid_tile<PREC, G, MODE, FAST>(a, smem, blk, nblk);
}

}  // namespace dotpe
