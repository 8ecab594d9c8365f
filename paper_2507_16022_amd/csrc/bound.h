// Bound pass of the evidence with the coherent cut (split precisions).
//
// Every pair's certified upper bound on lnL^ML (eq. bestfit_lnl) is
//     bound = (sx^2 / sh) U^2 / (2 lo),   U >= sum_g |X_g|,
//     lo <= S0 - 2 sum_{delta > 0} |S_delta|   (<= hh_o for every phase o).
// This kernel forms it from products of the hi parts of the split operands
// alone -- one matrix-core product per real product, where the value itself
// takes three -- and bounds what that leaves out by Cauchy-Schwarz: with
// a = ah + al and b = bh + bl (complex vectors over a row's positions),
//     |sum a b - fl(sum ah bh)| <= |ah| |bl| + |al| |bh| + |al| |bl|
//                                  + sqrt2 gamma_K |ah| |bh|,
// |.| the 2-norm and gamma_K = K 2^-23 for the FP32 accumulation of K real
// products.  k_operand_norms gives these norms per operand row and per m
// group ((d|h)) or output ((h|h)), so with c_0 = 1, c_r = 2 for the outputs
// r > 0 (Re, Im of S_delta):
//     U  = sum_g |X~_g| + sum_g [ah_g (bl_g + sqrt2 gamma_g bh_g) + al_g (bh_g + bl_g)],
//     lo = S~0 - 2 sum |S~_delta|
//          - sum_r c_r [nh_r (ql_r + gamma_32 qh_r) + nl_r (qh_r + ql_r)]
// (a, b: bank and extrinsic operand rows; n, q: the (h|h) operand rows).
// Each sum is a dot product of a row vector with a column vector, which
// Cauchy-Schwarz bounds by the product of their norms; that looser margin
// (four multiply-adds per pair) decides almost every pair, and only pairs
// it leaves near the threshold take the per-group one.  The (h|h) phase
// coefficients come first,
// folded into lo as each output completes, then the (d|h) contraction one m
// group at a time, each group's |X_g| added into U as the group completes.
// So a wave keeps lo, U and one group's accumulators: 64 x 64 pairs per
// wave, a 128 x 128 tile per workgroup.
//
// Each wave's 64 x 64 quadrant is one tile of the fused kernel's grid.  A
// quadrant all of whose pairs are bounded writes that tile's partial (the
// bounded mass and counts); one with a few survivors lists them for the
// survivor pass, which adds their evaluation to the partial; one with more
// is listed whole for the coefficient route, which bounds and evaluates the
// tile again.
#pragma once

#include "fused.h"

namespace dotpe {

struct BoundTile {
  static constexpr int NT = 256;           // 4 waves, one per SIMD
  static constexpr int TS = 128;           // rows and columns per tile
  static constexpr int NS = 7;             // LDS stages
  static constexpr int LPC = 4;            // 1 KB loads per wave per chunk
  static constexpr int ARR = 8192;         // bytes of one operand's hi part per stage
  static constexpr int STAGE = 2 * ARR;    // A hi, B hi
  static constexpr int NV = 24;            // margin factors per row or column
  static constexpr int ROWQ_OFF = NS * STAGE;            // double2 [128]: q factor, ln w
  static constexpr int COLQ_OFF = ROWQ_OFF + TS * 16;    // double2 [128]
  static constexpr int ROWN_OFF = COLQ_OFF + TS * 16;    // float4 [128]: the norms of whole rows
  static constexpr int COLN_OFF = ROWN_OFF + TS * 16;    // float4 [128]
  static constexpr int ROWT_OFF = COLN_OFF + TS * 16;    // float [128][NV]: per group and output
  static constexpr int COLT_OFF = ROWT_OFF + TS * NV * 4;
  static constexpr int LDS_BYTES = COLT_OFF + TS * NV * 4;
};

// Keep a value computed here: without it the compiler may defer the
// arithmetic that folds accumulators into lo0 and U0 to the end of the
// kernel, keeping every accumulator alive (and spilled) until then.
template <typename T>
__device__ __forceinline__ void pin(T& x) {
  __asm__ __volatile__("" : "+v"(x));
}

// pipeline_barrier with at most n (0..M, uniform over the workgroup) chunks
// of LPC loads each still in flight
template <int M, int LPC>
__device__ __forceinline__ void barrier_in_flight(int n) {
  static_for<M + 1>([&](auto qi) {
    constexpr int q = decltype(qi)::value;
    if (n == q) pipeline_barrier<q * LPC>();
  });
}

template <int PREC, int G>
__device__ __forceinline__ void bound_pass_tile(const FusedArgs& a, int64_t wg_id, int64_t wg_count) {
  static_assert(PREC != kFP64, "split precisions only");
  typedef BoundTile BT;
  typedef typename Pol<PREC>::Acc Acc;
  typedef __attribute__((address_space(1))) const unsigned char gbyte;
  typedef __attribute__((address_space(3))) void lvoid;
  constexpr int ES = 2;                         // bytes per operand element
  constexpr int NRT = (G == 1) ? 1 : kMaxNR;    // (h|h) outputs: S0, Re/Im S_1..3
  constexpr int NS = BT::NS, LPC = BT::LPC;
  static_assert(NS >= 5, "two chunks issued per barrier, two more in flight");
  extern __shared__ __align__(16) unsigned char smem[];
  // with the cut off the coefficient route takes every tile
  if (!a.bound_out && !cut_on(a)) return;

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;

  // workgroup -> 128 x 128 tile: consecutive ids spread over the XCDs, each
  // XCD walking a contiguous band of tiles in bands of 4 tile rows
  const int64_t nst_m = (a.n_tiles_m + 1) / 2, nst_n = (a.n_tiles_n + 1) / 2;
  int64_t wg = wg_id;
  {
    const int64_t nwg = wg_count;   // multiple of 8
    wg = (wg % 8) * (nwg / 8) + wg / 8;
  }
  if (wg >= nst_m * nst_n) return;
  int64_t sm_, sn_;
  {
    const int64_t GM = 4;
    const int64_t band = wg / (GM * nst_n);
    const int64_t rows_in_band = min(GM, nst_m - band * GM);
    const int64_t in = wg - band * GM * nst_n;
    sm_ = band * GM + in % rows_in_band;
    sn_ = in / rows_in_band;
  }
  const int64_t row0 = sm_ * BT::TS, col0 = sn_ * BT::TS;

  // per row and column: the factors of the bound (q = row_scale^2 /
  // ah_scale x the column's: powers of two, each possibly outside float
  // range, so multiplied in double; ln w) and of its margin, per group and
  // output (row: ah_g, al_g, nh_r, nl_r at 0, 4, 8, 16; column: bl_g +
  // sqrt2 gamma_g bh_g, bh_g + bl_g, c_r (ql_r + gamma_32 qh_r), c_r (qh_r +
  // ql_r) at the same places) and the norms of those four vectors (rounded
  // up) for the margin of whole rows
  double2* rowq = (double2*)(smem + BT::ROWQ_OFF);
  double2* colq = (double2*)(smem + BT::COLQ_OFF);
  float4* rown = (float4*)(smem + BT::ROWN_OFF);
  float4* coln = (float4*)(smem + BT::COLN_OFF);
  float* rowt = (float*)(smem + BT::ROWT_OFF);
  float* colt = (float*)(smem + BT::COLT_OFF);
  {
    const bool is_row = tid < BT::TS;
    const int t = is_row ? tid : tid - BT::TS;
    double2 v = make_double2(1.0, 0.0);
    float f[BT::NV];
#pragma unroll
    for (int k = 0; k < BT::NV; ++k) f[k] = 0.f;
    if (is_row) {
      const int64_t ie = row0 + t;
      if (ie < a.n_sub) {
        const int64_t i = a.sub_idx ? a.sub_idx[ie] : a.sub0 + ie;
        const double rs = a.row_scale[i];
        v = make_double2(rs * rs / a.ah_scale[ie], a.ln_w_bank ? a.ln_w_bank[i] : 0.0);
#pragma unroll
        for (int g = 0; g < G; ++g) {
          const float2 x = a.a_nrm[i * G + g];
          f[g] = x.x;
          f[4 + g] = x.y;
        }
#pragma unroll
        for (int r = 0; r < NRT; ++r) {
          const float2 x = a.ah_nrm[ie * NRT + r];
          f[8 + r] = x.x;
          f[16 + r] = x.y;
        }
      }
    } else {
      const int64_t e = col0 + t;
      if (e < a.n_ext) {
        const double cs = a.col_scale[e];
        v = make_double2(cs * cs / a.bh_scale[e], a.ln_w_ext ? a.ln_w_ext[e] : 0.0);
#pragma unroll
        for (int g = 0; g < G; ++g) {
          const float2 x = a.b_nrm[e * G + g];
          f[g] = x.y + a.gam_dh[g] * x.x;
          f[4 + g] = x.x + x.y;
        }
#pragma unroll
        for (int r = 0; r < NRT; ++r) {
          const float2 x = a.bh_nrm[e * NRT + r];
          const float c = r == 0 ? 1.f : 2.f;
          f[8 + r] = c * (x.y + a.gam_hh * x.x);
          f[16 + r] = c * (x.x + x.y);
        }
      }
    }
    float nv[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int k0 = q < 2 ? 4 * q : 8 * q - 8, nk = q < 2 ? 4 : 8;
      float s = 0.f;
      for (int k = 0; k < nk; ++k) s += f[k0 + k] * f[k0 + k];
      nv[q] = __builtin_sqrtf(s) * (1.f + 0x1p-18f);
    }
    float* dst = (is_row ? rowt : colt) + t * BT::NV;
#pragma unroll
    for (int k = 0; k < BT::NV; k += 4) *(float4*)(dst + k) = make_float4(f[k], f[k + 1], f[k + 2], f[k + 3]);
    (is_row ? rowq : colq)[t] = v;
    (is_row ? rown : coln)[t] = make_float4(nv[0], nv[1], nv[2], nv[3]);
  }

  // ---- operand streams: waves 0, 1 load the A hi rows of 32-row blocks
  // 2 w, 2 w + 1, waves 2, 3 the B hi rows of blocks 2 (w - 2), 2 (w - 2) + 1:
  // of every chunk, slices 0 and 1 of both blocks, 1 KB each copied as it
  // sits in HBM (fragment order).  A lane's address of block q, slice 0;
  // slice 1 is 1 KB further.  Rows past the subset re-read the last row;
  // columns run to the padded sample count (a multiple of 128, zero rows
  // past n_ext). ----
  gbyte* src_dh[2];
  gbyte* src_hh[2];
  auto blk = [](int64_t i, int64_t K) { return (i >> 5) * (K >> 5) * 1024 + (i & 31) * 8; };
#pragma unroll
  for (int q = 0; q < 2; ++q) {
    const int r = 32 * (2 * (wave & 1) + q) + (lane & 31);
    const int64_t in_chunk = (lane >> 5) * 256;
    if (wave < 2) {
      const int64_t ie = min(row0 + r, a.n_sub - 1);
      const int64_t i = a.sub_idx ? a.sub_idx[ie] : a.sub0 + ie;
      src_dh[q] = (gbyte*)a.A0 + (blk(i, a.K2) + in_chunk) * ES;
      src_hh[q] = (gbyte*)a.Ah0 + (blk(ie, a.KH) + in_chunk) * ES;
    } else {
      const int64_t e = col0 + r;
      src_dh[q] = (gbyte*)a.B0 + (blk(e, a.K2) + in_chunk) * ES;
      src_hh[q] = (gbyte*)a.Bh0 + (blk(e, a.KH) + in_chunk) * ES;
    }
  }
  // chunks: NRT (h|h) blocks first, then the (d|h) chunks; chunk c sits in
  // stage c mod NS, where this wave's part starts 4 KB x wave in
  const int ndh = a.n_chunks;
  const int nk = NRT + ndh;
  const unsigned lds_wave =
      __builtin_amdgcn_readfirstlane((unsigned)(uintptr_t)(lvoid*)(smem + wave * 4096));
  // the 4 loads of chunk c (block q, slice s to stage offset (2 q + s) KB)
  // sharing one M0 value: the immediate offset applies to the global and
  // the LDS address alike.  The asm saves and restores M0 and waits the
  // state an M0 write needs.
  auto issue = [&](int c) {
    gbyte* p0 = c < NRT ? src_hh[0] + (int64_t)c * 1024 * ES
                        : src_dh[0] + (int64_t)(c - NRT) * 1024 * ES;
    gbyte* p1 = c < NRT ? src_hh[1] + (int64_t)c * 1024 * ES
                        : src_dh[1] + (int64_t)(c - NRT) * 1024 * ES;
    const unsigned base = lds_wave + (unsigned)((c % NS) * BT::STAGE);
    unsigned m0_saved;
    __asm__ __volatile__(
        "s_mov_b32 %0, m0\n\ts_mov_b32 m0, %1\n\ts_nop 0\n\t"
        "global_load_lds_dwordx4 %2, off\n\t"
        "global_load_lds_dwordx4 %2, off offset:1024\n\t"
        "global_load_lds_dwordx4 %3, off offset:2048\n\t"
        "global_load_lds_dwordx4 %3, off offset:3072\n\ts_mov_b32 m0, %0"
        : "=&s"(m0_saved)
        : "s"(__builtin_amdgcn_readfirstlane(base)), "v"(p0), "v"(p1 - 2048)
        : "memory");
  };

  // Fragments of one chunk for this wave: A rows 64 wm + 32 bm (FA: [bm]
  // [slice]) and B rows 64 wn + 32 bn (FB: [slice], one per bn).  The
  // products of a chunk run in two halves, bn = 0 then bn = 1.  During the
  // first half the bn = 1 fragments of the same chunk are read, and the A
  // and bn = 0 fragments of the next chunk.
  struct FA {
    uint4 v[2][2];
  };
  struct FB {
    uint4 v[2];
  };
  FA fa0, fa1;
  FB fb0_0, fb0_1, fb1;
  auto fa = [&](auto pi) -> FA& {
    if constexpr (decltype(pi)::value % 2 == 0) return fa0;
    else return fa1;
  };
  auto fb0 = [&](auto pi) -> FB& {
    if constexpr (decltype(pi)::value % 2 == 0) return fb0_0;
    else return fb0_1;
  };
  auto stage_lane = [&](int c) { return smem + (c % NS) * BT::STAGE + lane * 16; };
  auto read_a = [&](FA& f, int c, int k) {    // k: block (k >> 1), slice
    const int bm = k >> 1, sl = k & 1;
    f.v[bm][sl] = *(const uint4*)(stage_lane(c) + (2 * (2 * wm + bm) + sl) * 1024);
  };
  auto read_b = [&](FB& f, int c, int bn, int sl) {
    f.v[sl] = *(const uint4*)(stage_lane(c) + BT::ARR + (2 * (2 * wn + bn) + sl) * 1024);
  };
  auto fence = [] { __builtin_amdgcn_sched_barrier(0); };

  // Step j (fragment parity P = j mod 2): on even steps, wait until chunks
  // j + 1 and j + 2 have landed (every wave's loads) and every wave is done
  // with chunks j - 2 and j - 1, and issue chunks j + NS - 2, j + NS - 1 into
  // the stages those used (a barrier every second chunk); then the products
  // of chunk j (NH per half; mf(fa, fb, bm, bn, k) issues product k of block
  // (bm, bn)) with the fragment reads between them.  After the last chunk
  // the reads fetch a stale stage, unused, so no branch sits between the
  // products.
  auto step = [&](int j, auto pi, auto nh, auto&& mf) {
    constexpr int P = decltype(pi)::value % 2;
    constexpr int NH = decltype(nh)::value;
    FA& acur = fa(std::integral_constant<int, P>{});
    FA& anxt = fa(std::integral_constant<int, P + 1>{});
    FB& bcur = fb0(std::integral_constant<int, P>{});
    FB& bnxt = fb0(std::integral_constant<int, P + 1>{});
    if constexpr (P == 0) {
      // chunks j + 3 .. min(j + NS - 3, nk - 1) may stay in flight
      barrier_in_flight<NS - 3, LPC>(max(0, min(NS - 5, nk - 3 - j)));
      fence();
      if (j + NS - 2 < nk) issue(j + NS - 2);
      if (j + NS - 1 < nk) issue(j + NS - 1);
      fence();
    }
    // half 0: blocks (0, 0), (1, 0), a read after each of its products
    static_for<2 * NH>([&](auto ti) {
      constexpr int t = decltype(ti)::value;
      mf(acur, bcur, t & 1, 0, t >> 1);
      if constexpr (t < 2) read_b(fb1, j, 1, t);
      else if constexpr (t < 6) read_a(anxt, j + 1, t - 2);
      else if constexpr (t < 8) read_b(bnxt, j + 1, 0, t - 6);
    });
    static_for<8>([&](auto ki) {     // reads not placed between products
      constexpr int k = decltype(ki)::value;
      if constexpr (k >= 2 * NH) {
        if constexpr (k < 2) read_b(fb1, j, 1, k);
        else if constexpr (k < 6) read_a(anxt, j + 1, k - 2);
        else read_b(bnxt, j + 1, 0, k - 6);
      }
    });
    // half 1: blocks (0, 1), (1, 1)
    static_for<2 * NH>([&](auto ti) {
      constexpr int t = decltype(ti)::value;
      mf(acur, fb1, t & 1, 1, t >> 1);
    });
  };

  // prologue: chunks 0 .. NS - 3 in flight; once chunk 0 has landed, its A
  // and bn = 0 fragments are read
#pragma unroll
  for (int c = 0; c < NS - 2; ++c)
    if (c < nk) issue(c);
  barrier_in_flight<NS - 3, LPC>(min(NS - 3, nk - 1));   // (also makes rowq .. colt visible)
  static_for<4>([&](auto ki) { read_a(fa0, 0, decltype(ki)::value); });
  static_for<2>([&](auto ki) { read_b(fb0_0, 0, 0, decltype(ki)::value); });

  // ---- (h|h): lo0 = S0 - 2 sum |S_delta| per pair, output by output ----
  Acc s0[2][2], sabs[2][2], sre[2][2], hacc[2][2];
  auto mf_hh = [&](const FA& A, const FB& B, int bm, int bn, int k) {   // k: slice
    mma<PREC>(hacc[bm][bn], A.v[bm][k], B.v[k]);
  };
  static_for<NRT>([&](auto ri) {
    constexpr int r = decltype(ri)::value;
#pragma unroll
    for (int bm = 0; bm < 2; ++bm)
#pragma unroll
      for (int bn = 0; bn < 2; ++bn) hacc[bm][bn] = Acc{};
    step(r, std::integral_constant<int, r>{}, std::integral_constant<int, 2>{}, mf_hh);
#pragma unroll
    for (int bm = 0; bm < 2; ++bm)
#pragma unroll
      for (int bn = 0; bn < 2; ++bn) {
        if constexpr (r == 0) {
          s0[bm][bn] = hacc[bm][bn];
          sabs[bm][bn] = Acc{};
        } else if constexpr (r % 2 == 1) {
          sre[bm][bn] = hacc[bm][bn];
        } else {
#pragma unroll
          for (int e = 0; e < 16; ++e) {
            const float x = sre[bm][bn][e], y = hacc[bm][bn][e];
            sabs[bm][bn][e] += 2.f * __builtin_amdgcn_sqrtf(x * x + y * y);
          }
          pin(sabs[bm][bn]);
        }
      }
  });
  // lo0 with a margin for the rounding of the fold itself
  Acc lo0[2][2];
#pragma unroll
  for (int bm = 0; bm < 2; ++bm)
#pragma unroll
    for (int bn = 0; bn < 2; ++bn)
#pragma unroll
      for (int e = 0; e < 16; ++e) {
        const float x = s0[bm][bn][e], sa = sabs[bm][bn][e];
        lo0[bm][bn][e] = (x - sa) - 2e-5f * (fabsf(x) + sa);
      }
#pragma unroll
  for (int bm = 0; bm < 2; ++bm)
#pragma unroll
    for (int bn = 0; bn < 2; ++bn) pin(lo0[bm][bn]);

  // ---- (d|h): one m group at a time, |X_g| into U0 ----
  Acc u0[2][2], acc[2][2][2];
#pragma unroll
  for (int bm = 0; bm < 2; ++bm)
#pragma unroll
    for (int bn = 0; bn < 2; ++bn) u0[bm][bn] = Acc{};
  // product k (0..3) of block (bm, bn): with A = [hr | hi] and B_re =
  // [Br | -Bi] by slice, B_im = [Bi | Br] = [-(B_re slice 1) | B_re slice 0]
  auto neg = [](const uint4& x) {
    return make_uint4(x.x ^ 0x80008000u, x.y ^ 0x80008000u, x.z ^ 0x80008000u, x.w ^ 0x80008000u);
  };
  auto mf_dh = [&](const FA& A, const FB& B, int bm, int bn, int k) {
    Acc& re = acc[bm][bn][0];
    Acc& im = acc[bm][bn][1];
    switch (k) {
      case 0: mma<PREC>(re, A.v[bm][0], B.v[0]); break;
      case 1: mma<PREC>(im, A.v[bm][0], neg(B.v[1])); break;
      case 2: mma<PREC>(re, A.v[bm][1], B.v[1]); break;
      default: mma<PREC>(im, A.v[bm][1], B.v[0]); break;
    }
  };
  int ch = 0;
  static_for<G>([&](auto gi) {
    constexpr int g = decltype(gi)::value;
#pragma unroll
    for (int bm = 0; bm < 2; ++bm)
#pragma unroll
      for (int bn = 0; bn < 2; ++bn) {
        acc[bm][bn][0] = Acc{};
        acc[bm][bn][1] = Acc{};
      }
    // each group spans a multiple of 4 chunks, so the fragment parity of
    // every step is static
    const int gend = a.mt.gk0[g + 1];
    for (; ch < gend; ch += 2) {
      step(NRT + ch, std::integral_constant<int, NRT>{}, std::integral_constant<int, 4>{}, mf_dh);
      step(NRT + ch + 1, std::integral_constant<int, NRT + 1>{}, std::integral_constant<int, 4>{},
           mf_dh);
    }
#pragma unroll
    for (int bm = 0; bm < 2; ++bm)
#pragma unroll
      for (int bn = 0; bn < 2; ++bn)
#pragma unroll
        for (int e = 0; e < 16; ++e) {
          const float xr = acc[bm][bn][0][e], xi = acc[bm][bn][1][e];
          u0[bm][bn][e] += __builtin_amdgcn_sqrtf(xr * xr + xi * xi);
        }
#pragma unroll
    for (int bm = 0; bm < 2; ++bm)
#pragma unroll
      for (int bn = 0; bn < 2; ++bn) pin(u0[bm][bn]);
  });

  // ---- bound every pair of this wave's tile ----
  const int64_t tm = 2 * sm_ + wm, tn = 2 * sn_ + wn;
  if (tm >= a.n_tiles_m || tn >= a.n_tiles_n) return;
  const int64_t tile_id = tm * a.n_tiles_n + tn;
  const int rows_in = (int)min((int64_t)64, a.n_sub - tm * 64);
  const int cols_in = (int)min((int64_t)64, a.n_ext - tn * 64);
  // bound from the accumulators and a margin (q, ln w of the pair's row and
  // column in rq, cq)
  auto bound_of = [](double2 rq, double2 cq, float U0, float lo) {
    // rcp is within an ulp; the 1.001 factor covers it
    return (float)(rq.x * cq.x) * (U0 * U0) * __builtin_amdgcn_rcpf(2.f * lo) * 1.001f + 1e-3f;
  };
  // margin per group and output: row factors r, column factors c
  auto tight = [](const float* r, const float* c, float& du, float& dl) {
    du = 0.f;
    dl = 0.f;
#pragma unroll
    for (int g = 0; g < G; ++g) du += r[g] * c[g] + r[4 + g] * c[4 + g];
#pragma unroll
    for (int q = 0; q < NRT; ++q) dl += r[8 + q] * c[8 + q] + r[16 + q] * c[16 + q];
  };
  auto load_nv = [](const float* p, float* f) {
#pragma unroll
    for (int k = 0; k < BoundTile::NV; k += 4) {
      const float4 v = *(const float4*)(p + k);
      f[k] = v.x; f[k + 1] = v.y; f[k + 2] = v.z; f[k + 3] = v.w;
    }
  };
  if (a.bound_out) {
    const int64_t plane = a.n_sub * a.n_ext;
#pragma unroll
    for (int bm = 0; bm < 2; ++bm)
#pragma unroll
      for (int e = 0; e < 16; ++e) {
        const int tr = 32 * bm + 8 * (e >> 2) + 4 * (lane >> 5) + (e & 3);
        const double2 rq = rowq[64 * wm + tr];
        const float4 rn = rown[64 * wm + tr];
        float rt[BT::NV];
        load_nv(rowt + (64 * wm + tr) * BT::NV, rt);
#pragma unroll
        for (int bn = 0; bn < 2; ++bn) {
          const int tc = 32 * bn + (lane & 31);
          if (tr >= rows_in || tc >= cols_in) continue;
          const double2 cq = colq[64 * wn + tc];
          const float4 cn = coln[64 * wn + tc];
          float ct[BT::NV];
          load_nv(colt + (64 * wn + tc) * BT::NV, ct);
          float du, dl;
          tight(rt, ct, du, dl);
          const float U0 = u0[bm][bn][e], lo = lo0[bm][bn][e];
          const float Ul = U0 + (rn.x * cn.x + rn.y * cn.y), ll = lo - (rn.z * cn.z + rn.w * cn.w);
          const float Ut = U0 + du, lt = lo - dl;
          const int64_t o = (tm * 64 + tr) * a.n_ext + tn * 64 + tc;
          a.bound_out[o] = ll > 0.f ? bound_of(rq, cq, Ul, ll) : INFINITY;
          a.bound_out[plane + o] = lt > 0.f ? bound_of(rq, cq, Ut, lt) : INFINITY;
        }
      }
    return;
  }
  const float thr_f = (float)(__longlong_as_double(a.state[3]) - a.cut_delta);
  // The bounded mass is summed against a fixed reference: every bounded
  // pair has bound < thr_f and ln w no larger than the tile's largest row
  // weight plus its largest column weight, so each term exp(lw + bound -
  // m_ref) is at most 1 and a plain float sum holds them (its rounding, at
  // most ~1e-5 relative here, is far inside the bound's e^0.001 margin).
  const float lw_max = wave_max((double)rowq[64 * wm + lane].y) + wave_max((double)colq[64 * wn + lane].y);
  const float m_ref = thr_f + lw_max;
  float dsum = 0.f, max_bound = -INFINITY;
  // first with the margin of whole rows; pairs it leaves (bit 16 bm + e of
  // tmask[bn]) with the margin per group and output; survivors of both in
  // smask
  unsigned tmask[2] = {0u, 0u}, smask[2] = {0u, 0u};
  double2 cq[2];
  float4 cn[2];
  bool col_in[2];
#pragma unroll
  for (int bn = 0; bn < 2; ++bn) {
    const int tc = 32 * bn + (lane & 31);
    cq[bn] = colq[64 * wn + tc];
    cn[bn] = coln[64 * wn + tc];
    col_in[bn] = tc < cols_in;
  }
#pragma unroll
  for (int bm = 0; bm < 2; ++bm)
#pragma unroll
    for (int e = 0; e < 16; ++e) {
      const int tr = 32 * bm + 8 * (e >> 2) + 4 * (lane >> 5) + (e & 3);
      const double2 rq = rowq[64 * wm + tr];
      const float4 rn = rown[64 * wm + tr];
#pragma unroll
      for (int bn = 0; bn < 2; ++bn) {
        const bool in = col_in[bn] && tr < rows_in;
        const float U0 = u0[bm][bn][e] + (rn.x * cn[bn].x + rn.y * cn[bn].y);
        const float lo = lo0[bm][bn][e] - (rn.z * cn[bn].z + rn.w * cn[bn].w);
        const float bound = bound_of(rq, cq[bn], U0, lo);
        const bool bounded = in && lo > 0.f && bound < thr_f;
        const float x = (float)(rq.y + cq[bn].y) + bound;
        dsum += bounded ? __expf(x - m_ref) : 0.f;
        max_bound = bounded ? fmaxf(max_bound, x) : max_bound;
        tmask[bn] |= (in && !bounded) ? 1u << (16 * bm + e) : 0u;
      }
    }
  if (__ballot((tmask[0] | tmask[1]) != 0u)) {
    float ct[2][BT::NV];
#pragma unroll
    for (int bn = 0; bn < 2; ++bn) load_nv(colt + (64 * wn + 32 * bn + (lane & 31)) * BT::NV, ct[bn]);
#pragma unroll
    for (int bm = 0; bm < 2; ++bm)
#pragma unroll
      for (int e = 0; e < 16; ++e) {
        const unsigned bit = 1u << (16 * bm + e);
        if (!__ballot(((tmask[0] | tmask[1]) & bit) != 0u)) continue;
        const int tr = 32 * bm + 8 * (e >> 2) + 4 * (lane >> 5) + (e & 3);
        const double2 rq = rowq[64 * wm + tr];
        float rt[BT::NV];
        load_nv(rowt + (64 * wm + tr) * BT::NV, rt);
#pragma unroll
        for (int bn = 0; bn < 2; ++bn) {
          if (!(tmask[bn] & bit)) continue;
          float du, dl;
          tight(rt, ct[bn], du, dl);
          const float lo = lo0[bm][bn][e] - dl;
          const float bound = bound_of(rq, cq[bn], u0[bm][bn][e] + du, lo);
          if (lo > 0.f && bound < thr_f) {
            const float x = (float)(rq.y + cq[bn].y) + bound;
            dsum += __expf(x - m_ref);
            max_bound = fmaxf(max_bound, x);
          } else {
            smask[bn] |= bit;
          }
        }
      }
  }
  // survivors in a fixed order (bn, bm, element, lane): only the (bn, bit)
  // columns in which some lane has one are visited
  int n_surv = 0;
  unsigned cols[2] = {0u, 0u};
  if (__ballot((smask[0] | smask[1]) != 0u)) {
    auto or_i = [](int x, int y) { return x | y; };
#pragma unroll
    for (int bn = 0; bn < 2; ++bn) {
      cols[bn] = (unsigned)__builtin_amdgcn_readlane(wave_reduce((int)smask[bn], 0, or_i), 63);
      for (unsigned m = cols[bn]; m; m &= m - 1u)
        n_surv += (int)__popcll(__ballot((smask[bn] >> __builtin_ctz(m)) & 1u));
    }
  }
  if (n_surv > kSurvCap) {
    // the whole tile goes to the coefficient route
    if (lane == 0) {
      const unsigned long long k = atomicAdd((unsigned long long*)&a.state[4], 1ull);
      a.rerun[k] = (int)tile_id;
    }
    return;
  }
  if (n_surv > 0) {
    // listed one by one for the survivor pass, which adds their evaluation
    // to the partial written below
    uint16_t* rec = a.surv + tile_id * kSurvCap;
    int run = 0;
#pragma unroll
    for (int bn = 0; bn < 2; ++bn)
      for (unsigned m = cols[bn]; m; m &= m - 1u) {
        const int q = __builtin_ctz(m);
        const unsigned long long bal = __ballot((smask[bn] >> q) & 1u);
        if ((smask[bn] >> q) & 1u) {
          const int slot = run + (int)__builtin_amdgcn_mbcnt_hi((unsigned)(bal >> 32),
                                                                __builtin_amdgcn_mbcnt_lo((unsigned)bal, 0u));
          const int bm = q >> 4, e = q & 15;
          const int tr = 32 * bm + 8 * (e >> 2) + 4 * (lane >> 5) + (e & 3);
          const int tc = 32 * bn + (lane & 31);
          rec[slot] = (uint16_t)((tr << 8) | tc);
        }
        run += (int)__popcll(bal);
      }
    if (lane == 0) {
      const unsigned long long k = atomicAdd((unsigned long long*)&a.state[5], 1ull);
      a.surv_list[2 * k] = (int)tile_id;
      a.surv_list[2 * k + 1] = n_surv;
    }
  }
  // the tile's partial: bounded mass (m_ref, sum), counts, largest bound
  const float w_mb = wave_reduce(max_bound, (float)-INFINITY, [](float x, float y) { return fmaxf(x, y); });
  const float w_ds = wave_reduce(dsum, 0.f, [](float x, float y) { return x + y; });
  if (lane == 63) {
    const int n_in = rows_in * cols_in;
    double* out = a.partials + tile_id * kNPart;
    out[0] = -INFINITY; out[1] = 0.0; out[2] = 0.0;          // no pair evaluated (yet)
    out[3] = w_ds > 0.f ? (double)m_ref : -INFINITY;
    out[4] = w_ds > 0.f ? (double)w_ds : 0.0;
    out[5] = 0.0; out[6] = 0.0; out[7] = (double)(n_in - n_surv);
    out[8] = (double)w_mb; out[9] = -INFINITY; out[10] = (double)n_in; out[11] = 0.0;
  }
}

template <int PREC, int G>
__global__ __launch_bounds__(BoundTile::NT) void k_lnl_bound(FusedArgs a) {
  bound_pass_tile<PREC, G>(a, blockIdx.x, gridDim.x);
}

// the bound pass of several events in one launch
template <int PREC, int G>
__global__ __launch_bounds__(BoundTile::NT) void k_lnl_bound_packed(PackLaunch p) {
  int64_t blk, nblk;
  int q;
  const int e = pack_locate(p, blockIdx.x, &blk, &nblk, &q);
  FusedArgs a = pack_args(p, e, q);
  bound_pass_tile<PREC, G>(a, blk, nblk);
}

// Survivor pass after the bound pass: a wave per listed tile evaluates its
// survivors one at a time.  For a survivor (i, e) the wave forms X_g and the
// (h|h) phase coefficients as FP64 sums of the products of the split
// operands (each value hi + lo is exact in double; lanes take chunks of the
// contraction, then a wave reduction), and then the per-phase
// marginalisation of the fused kernel (pair_phases), one phase per lane.
// The results are merged into the tile's partial, which the bound pass wrote
// with the tile's bounded mass.
template <int PREC, int G>
__device__ __forceinline__ void survivor_pass(const FusedArgs& a, int64_t wg_id, int64_t wg_count) {
  static_assert(PREC != kFP64, "split precisions only");
  constexpr int NRT = (G == 1) ? 1 : kMaxNR;
  typedef typename std::conditional<PREC == kFP16X2, _Float16, __bf16>::type H;
  __shared__ __align__(16) unsigned char sm[sizeof(DistParams) + 16 + kMaxM * kMaxPhi * 2 * 8];
  DistParams* dp = (DistParams*)sm;
  double* lds_cs = (double*)(sm + (sizeof(DistParams) + 15) / 16 * 16);
  const int tid = threadIdx.x, lane = tid & 63;
  for (int t = tid; t < kMaxM * a.n_phi * 2; t += 256) lds_cs[t] = a.phase_cs[t];
  for (int t = tid; t < (int)(sizeof(DistParams) / 4); t += 256)
    ((unsigned*)dp)[t] = ((const unsigned*)a.dist.prm)[t];
  __syncthreads();
  // the workgroups' waves take the listed tiles in turn (the list's length
  // is known on the device only; the grid is large enough that a wave
  // takes a few at most)
  const int64_t n_list = (int64_t)a.state[5];
  for (int64_t item = wg_id * 4 + (tid >> 6); item < n_list; item += wg_count * 4) {
    const int64_t tile_id = a.surv_list[2 * item];
    const int n_surv = a.surv_list[2 * item + 1];
    const int64_t tm = tile_id / a.n_tiles_n, tn = tile_id % a.n_tiles_n;
    const double thr_ml = __longlong_as_double(a.state[3]) - a.cut_delta;
    const double thr_topk_glob = order_value(a.state[1]) - a.topk_window;
    const int nch = (int)(a.K2 >> 5);
    auto val = [](const H* p, const H* q, int j) { return (double)(float)p[j] + (double)(float)q[j]; };
    EvAcc ev;
    ev.init();
    double tile_max = -INFINITY;
    double my_lnp = -INFINITY;     // lane s: ln p of survivor s (-inf if not evaluated)
    int my_ob = 0;                 //   and its best phase
    for (int sidx = 0; sidx < n_surv; ++sidx) {
      const unsigned rc = a.surv[tile_id * kSurvCap + sidx];
      const int64_t ie = tm * 64 + (rc >> 8), e = tn * 64 + (rc & 255);
      const int64_t i = a.sub_idx ? a.sub_idx[ie] : a.sub0 + ie;
      // X_g: lane l takes half l % 2 (8 positions of each slice) of chunks
      // l / 2, l / 2 + 32, ...  The bank row comes from the row-major copy
      // (64 contiguous bytes per chunk and array: a wave reads whole lines),
      // the extrinsic row from the fragment layout (16 bytes per chunk,
      // slice and half; its 2^14 rows stay in the caches)
      double xr[G], xi[G];
#pragma unroll
      for (int g = 0; g < G; ++g) { xr[g] = 0.0; xi[g] = 0.0; }
      const int h = lane & 1;
      const int64_t arow = i * a.K2 + h * 8;
      const int64_t brow = ((e >> 5) * (a.K2 >> 5)) * 1024 + (e & 31) * 8 + h * 256;
      for (int c = lane >> 1; c < nch; c += 32) {
        const H* a0h = (const H*)a.R0 + arow + (int64_t)c * 32;
        const H* a0l = (const H*)a.R1 + arow + (int64_t)c * 32;
        const H* b0h = (const H*)a.B0 + brow + (int64_t)c * 1024;
        const H* b0l = (const H*)a.B1 + brow + (int64_t)c * 1024;
        double re = 0.0, im = 0.0;
#pragma unroll
        for (int j = 0; j < 8; ++j) {
          const double x0 = val(a0h, a0l, j), x1 = val(a0h + 16, a0l + 16, j);
          const double y0 = val(b0h, b0l, j), y1 = val(b0h + 512, b0l + 512, j);
          re += x0 * y0 + x1 * y1;      // A [hr | hi'] . B_re [Br | -Bi]
          im += x1 * y0 - x0 * y1;      // A . B_im, B_im = [-(B_re slice 1) | B_re slice 0]
        }
#pragma unroll
        for (int g = 0; g < G; ++g) {
          const bool in_g = c >= a.mt.gk0[g] && c < a.mt.gk0[g + 1];
          xr[g] += in_g ? re : 0.0;
          xi[g] += in_g ? im : 0.0;
        }
      }
      // (h|h) outputs: lanes 4 r .. 4 r + 3 take block r (slice, half)
      double sv = 0.0;
      if (lane < 4 * NRT) {
        const int r = lane >> 2, s2 = (lane >> 1) & 1, h2 = lane & 1;
        const int64_t ho = ((ie >> 5) * (a.KH >> 5) + r) * 1024 + s2 * 512 + h2 * 256 + (ie & 31) * 8;
        const int64_t bo = ((e >> 5) * (a.KH >> 5) + r) * 1024 + s2 * 512 + h2 * 256 + (e & 31) * 8;
#pragma unroll
        for (int j = 0; j < 8; ++j)
          sv += val((const H*)a.Ah0 + ho, (const H*)a.Ah1 + ho, j) *
                val((const H*)a.Bh0 + bo, (const H*)a.Bh1 + bo, j);
      }
      // quad sums, then every lane reads the totals
      sv += dpp_mov<0xB1, 0xF>(0.0, sv);
      sv += dpp_mov<0x4E, 0xF>(0.0, sv);
      auto add_d = [](double x, double y) { return x + y; };
      const double sx = a.row_scale[i] * a.col_scale[e];
      const double shh = a.ah_scale[ie] * a.bh_scale[e];
      double2 X[G];
#pragma unroll
      for (int g = 0; g < G; ++g) {
        X[g].x = sx * read_lane(wave_reduce(xr[g], 0.0, add_d), 63);
        X[g].y = sx * read_lane(wave_reduce(xi[g], 0.0, add_d), 63);
      }
      double S0 = shh * read_lane(sv, 0), Sr[kMaxND], Si[kMaxND];
#pragma unroll
      for (int d = 0; d < kMaxND; ++d) { Sr[d] = 0.0; Si[d] = 0.0; }
#pragma unroll
      for (int d = 1; d < (NRT + 1) / 2; ++d) {
        Sr[d] = shh * read_lane(sv, 4 * (2 * d - 1));
        Si[d] = shh * read_lane(sv, 4 * (2 * d));
      }
      const double lnw = (a.ln_w_bank ? a.ln_w_bank[i] : 0.0) + (a.ln_w_ext ? a.ln_w_ext[e] : 0.0);
      LsePh lse;
      lse.init();
      double best = -INFINITY, mlmax = 0.0;
      int ob = 0;
      pair_phases<kEvidence, G, true>(a, lds_cs, *dp, ie, e, X, S0, Sr, Si, lnw, thr_ml, lane, 64, ev, lse,
                                best, ob, mlmax);
#pragma unroll
      for (int off = 32; off > 0; off >>= 1) {
        const double lm = __shfl_xor(lse.m, off, 64), ls = __shfl_xor(lse.s, off, 64);
        const double ls2 = __shfl_xor(lse.s2, off, 64);
        lse.merge(lm, ls, ls2);
        const double bv = __shfl_xor(best, off, 64);
        const int bo = __shfl_xor(ob, off, 64);
        if (bv > best || (bv == best && bo < ob)) { best = bv; ob = bo; }
        mlmax = fmax(mlmax, __shfl_xor(mlmax, off, 64));
      }
      ev.ml_max = fmax(ev.ml_max, mlmax);
      if (lse.m == -INFINITY) continue;
      const double lnp = lnw + lse.m + log(lse.s) - a.ln_nphi;
      if (lane == sidx) {
        my_lnp = lnp;
        my_ob = ob;
      }
      if (lane != 0) continue;
      ev.p.add(lnp, lse.sq_ratio());
      tile_max = fmax(tile_max, lnp);
    }
    // top-k candidates among the survivors (within the window of the tile's
    // and the running global maximum), appended with one atomic per tile in
    // survivor order: lane s holds survivor s
    {
      const double thr_c = fmax(thr_topk_glob, read_lane(tile_max, 0) - a.topk_window);
      const bool cand = lane < n_surv && my_lnp > -INFINITY && my_lnp >= thr_c;
      const unsigned long long bal = __ballot(cand);
      if (bal) {
        unsigned long long base = 0;
        if (lane == 0) base = atomicAdd((unsigned long long*)&a.state[2], (unsigned long long)__popcll(bal));
        base = (unsigned long long)__shfl((long long)base, 0, 64);
        if (cand) {
          const unsigned long long slot =
              base + __builtin_amdgcn_mbcnt_hi((unsigned)(bal >> 32), __builtin_amdgcn_mbcnt_lo((unsigned)bal, 0u));
          if ((int64_t)slot < a.cand_cap) {
            const unsigned rc = a.surv[tile_id * kSurvCap + lane];
            const int64_t ie = tm * 64 + (rc >> 8), e = tn * 64 + (rc & 255);
            double* cd = a.cand + 4 * slot;
            cd[0] = my_lnp;
            cd[1] = (double)(a.sub_idx ? a.sub_idx[ie] : a.sub0 + ie);
            cd[2] = (double)e;
            cd[3] = (double)my_ob;
          }
        }
      }
    }
    // merge into the tile's partial: the cut phases' bounds (every lane), the
    // evaluated pairs (lane 0), the phases marginalised
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
    const int n_marg = wave_reduce(ev.n_marg, 0, [](int x, int y) { return x + y; });
    const double dmd = read_lane(dm == -INFINITY ? -INFINITY : (double)dm, 63);
    const double dsd = read_lane((double)ds, 63);
    const int n_marg_all = __builtin_amdgcn_readlane(n_marg, 63);
    // the survivors' p in the tile's row and column sums, relative to the
    // tile maximum, in survivor order (the bound pass left the sums zero)
    const double tmax = read_lane(tile_max, 0);
    for (int sidx = 0; sidx < n_surv; ++sidx) {
      const double v = read_lane(my_lnp, sidx);
      if (lane == 0 && v > -INFINITY) {
        const unsigned rc = a.surv[tile_id * kSurvCap + sidx];
        double* rs = a.rowcol + tile_id * 128;
        const double x = exp(v - tmax);
        rs[rc >> 8] += x;
        rs[64 + (rc & 255)] += x;
      }
    }
    if (lane == 0) {
      double* out = a.partials + tile_id * kNPart;
      Lse d;
      d.m = out[3];
      d.s = out[4];
      d.s2 = 0.0;
      d.s3 = 0.0;
      d.merge(dmd, dsd, 0.0);
      out[0] = ev.p.m; out[1] = ev.p.s; out[2] = ev.p.s2; out[11] = ev.p.s3;
      out[3] = d.m; out[4] = d.s;
      out[5] = ev.ml_max; out[6] = (double)n_marg_all; out[9] = tile_max;
      // running maxima: most tiles cannot raise them, so they read before
      // they update (a stale read costs only an unneeded atomic)
      if (ev.ml_max > 0.0 && __double_as_longlong(ev.ml_max) > (long long)a.state[0])
        atomicMax((unsigned long long*)&a.state[0], (unsigned long long)__double_as_longlong(ev.ml_max));
      if (tile_max > -INFINITY && order_bits(tile_max) > a.state[1])
        atomicMax((unsigned long long*)&a.state[1], (unsigned long long)order_bits(tile_max));
    }
  }
}

template <int PREC, int G>
__global__ __launch_bounds__(256, 2) void k_survivors(FusedArgs a) {
  survivor_pass<PREC, G>(a, blockIdx.x, gridDim.x);
}

// the survivor pass of several events in one launch
template <int PREC, int G>
__global__ __launch_bounds__(256, 2) void k_survivors_packed(PackLaunch p) {
  int64_t blk, nblk;
  int q;
  const int e = pack_locate(p, blockIdx.x, &blk, &nblk, &q);
  FusedArgs a = pack_args(p, e, q);
  survivor_pass<PREC, G>(a, blk, nblk);
}

}  // namespace dotpe
