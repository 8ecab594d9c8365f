// Second half of the coefficient route of an evidence pass.  The fused
// kernel (mode kCoef) has stored the raw accumulators of every pair of the
// chunk's tiles; this kernel bounds (E1) and evaluates (E2: per-phase
// distance marginalisation, eq. lnl_dist_marginalized, and the phase
// average) every pair, one lane per pair with the phases in a loop, and
// writes each tile's partial.  Apart from the accumulators it holds a
// handful of doubles per lane, so several waves share every SIMD and hide
// the latency of the distance rule's table reads, which the fused kernel,
// one wave per SIMD, cannot.
#pragma once

#include "fused.h"

namespace dotpe {

template <int PREC, int G>
__global__ __launch_bounds__(256) void k_e2_tiles(FusedArgs a) {
  typedef Tile<PREC> TL;
  typedef typename std::conditional<PREC == kFP64, double, float>::type AT;
  constexpr int NRT = (G == 1) ? 1 : kMaxNR;
  constexpr int NCO = 2 * G + NRT;
  constexpr int TM = TL::TM, TN = TL::TN, NPT = TM * TN, NT = 256, NW = NT / 64;
  static_assert(NPT % NT == 0, "whole pairs per thread");
  __shared__ DistParams dp;
  __shared__ double lds_cs[kMaxM * kMaxPhi * 2];
  __shared__ double rowd[TM * 4], cold[TN * 3], rowq[TM * 2], red[NW * kNPart];
  __shared__ double lnp_pair[NPT];       // ln p of each evaluated pair, -inf otherwise
  __shared__ unsigned long long tile_lnp_max;

  const int tid = threadIdx.x;
  for (int t = tid; t < kMaxM * a.n_phi * 2; t += NT) lds_cs[t] = a.phase_cs[t];
  static_assert(sizeof(DistParams) % 4 == 0, "DistParams words");
  for (int t = tid; t < (int)(sizeof(DistParams) / 4); t += NT)
    ((unsigned*)&dp)[t] = ((const unsigned*)a.dist.prm)[t];
  // the cut as the fused kernel's epilogue applies it
  const bool on = cut_on(a);
  const double thr_ml = on ? __longlong_as_double(a.state[3]) - a.cut_delta : -INFINITY;
  const float thr_f = (float)thr_ml;
  const int64_t end = min(a.work0 + a.coef_tiles, coef_work_count(a));

  for (int64_t q = a.work0 + blockIdx.x; q < end; q += gridDim.x) {
    const int64_t t = coef_tile(a, q);
    const int64_t tm = t / a.n_tiles_n, tn = t % a.n_tiles_n;
    const int64_t row0 = tm * TM, col0 = tn * TN;
    // per-row and per-column scalars, as the fused kernel forms them
    if (tid < TM) {
      double rv0 = 0.0, rv1 = 1.0, rv2 = 1.0, rv3 = -1.0;
      const int64_t ie = row0 + tid;
      if (ie < a.n_sub) {
        const int64_t i = a.sub_idx ? a.sub_idx[ie] : a.sub0 + ie;
        rv0 = a.ln_w_bank ? a.ln_w_bank[i] : 0.0;
        rv1 = PREC == kFP64 ? 1.0 : a.row_scale[i];
        rv2 = PREC == kFP64 ? 1.0 : a.ah_scale[ie];
        rv3 = (double)i;
      }
      rowd[tid * 4] = rv0; rowd[tid * 4 + 1] = rv1; rowd[tid * 4 + 2] = rv2; rowd[tid * 4 + 3] = rv3;
      rowq[tid * 2] = rv1 * rv1 / rv2;
      rowq[tid * 2 + 1] = rv0;
    } else if (tid < TM + TN) {
      double cv0 = 0.0, cv1 = 1.0, cv2 = 1.0;
      const int64_t e = col0 + (tid - TM);
      if (e < a.n_ext) {
        cv0 = a.ln_w_ext ? a.ln_w_ext[e] : 0.0;
        cv1 = PREC == kFP64 ? 1.0 : a.col_scale[e];
        cv2 = PREC == kFP64 ? 1.0 : a.bh_scale[e];
      }
      cold[(tid - TM) * 3] = cv0; cold[(tid - TM) * 3 + 1] = cv1; cold[(tid - TM) * 3 + 2] = cv2;
    }
    if (tid == 0) tile_lnp_max = 0ull;
    __syncthreads();
    const double thr_topk_glob = order_value(a.state[1]) - a.topk_window;
    const int rows_in = (int)min((int64_t)TM, a.n_sub - row0);
    const int cols_in = (int)min((int64_t)TN, a.n_ext - col0);
    const AT* cf = (const AT*)a.coef + (q - a.work0) * (int64_t)(NCO * NPT);
    EvAcc ev;
    ev.init();
    int n_pairs_i = 0, n_bounded_i = 0;
#pragma unroll 1
    for (int k = 0; k < NPT / NT; ++k) {
      // a wave takes consecutive pairs of a row: coalesced component reads
      const int p = k * NT + tid, tr = p / TN, tc = p % TN;
      lnp_pair[p] = -INFINITY;
      if (!(tr < rows_in && tc < cols_in)) continue;
      ++n_pairs_i;
      AT x[2 * G], sv[NRT];
#pragma unroll
      for (int c = 0; c < 2 * G; ++c) x[c] = cf[c * NPT + p];
#pragma unroll
      for (int c = 0; c < NRT; ++c) sv[c] = cf[(2 * G + c) * NPT + p];
      if (on) {
        // E1: the certified bound on lnL^ML, the same arithmetic as the
        // fused kernel's epilogue on the same accumulators
        float U0 = 0.f;
#pragma unroll
        for (int g = 0; g < G; ++g) {
          const float xr = (float)x[2 * g], xi = (float)x[2 * g + 1];
          U0 += __builtin_amdgcn_sqrtf(xr * xr + xi * xi);
        }
        const float s0 = (float)sv[0];
        float sabs = 0.f;
#pragma unroll
        for (int d = 1; d < (NRT + 1) / 2; ++d) {
          const float sr = (float)sv[2 * d - 1], si = (float)sv[2 * d];
          sabs += 2.f * __builtin_amdgcn_sqrtf(sr * sr + si * si);
        }
        const float lo0 = (s0 - sabs) - 2e-5f * (fabsf(s0) + sabs);
        const double colq = cold[tc * 3 + 1] * cold[tc * 3 + 1] / cold[tc * 3 + 2];
        const float qf = (float)(rowq[tr * 2] * colq);
        const float bound = qf * (U0 * U0) * __builtin_amdgcn_rcpf(2.f * lo0) * 1.001f + 1e-3f;
        if (lo0 > 0.f && bound < thr_f) {
          const float lw = (float)(rowq[tr * 2 + 1] + cold[tc * 3]);
          ev.drop.add(lw + bound);
          ev.max_bound = fmaxf(ev.max_bound, lw + bound);
          ++n_bounded_i;
          continue;
        }
      }
      // E2
      const double sx = rowd[tr * 4 + 1] * cold[tc * 3 + 1];
      const double sh = rowd[tr * 4 + 2] * cold[tc * 3 + 2];
      double2 X[G];
#pragma unroll
      for (int g = 0; g < G; ++g)
        X[g] = make_double2(sx * (double)x[2 * g], sx * (double)x[2 * g + 1]);
      double S0 = sh * (double)sv[0], Sr[kMaxND], Si[kMaxND];
#pragma unroll
      for (int d = 0; d < kMaxND; ++d) { Sr[d] = 0.0; Si[d] = 0.0; }
#pragma unroll
      for (int d = 1; d < (NRT + 1) / 2; ++d) {
        Sr[d] = sh * (double)sv[2 * d - 1];
        Si[d] = sh * (double)sv[2 * d];
      }
      const double lnw = rowd[tr * 4] + cold[tc * 3];
      const int64_t e = col0 + tc;
      LsePh lse;
      lse.init();
      double best = -INFINITY, mlmax = 0.0;
      int ob = 0;
      pair_phases<kEvidence, G, false>(a, lds_cs, dp, row0 + tr, e, X, S0, Sr, Si, lnw, thr_ml, 0, 1,
                                      ev, lse, best, ob, mlmax);
      ev.ml_max = fmax(ev.ml_max, mlmax);
      if (lse.m == -INFINITY) continue;
      const double lnp = lnw + (lse.m + log(lse.s) - a.ln_nphi);
      ev.p.add(lnp, lse.sq_ratio());
      lnp_pair[p] = lnp;
      // top-k candidates within the window of the running maxima
      const unsigned long long ob_bits = order_bits(lnp);
      const unsigned long long prev = atomicMax(&tile_lnp_max, ob_bits);
      const double tmax = order_value(prev > ob_bits ? prev : ob_bits);
      if (lnp >= fmax(thr_topk_glob, tmax - a.topk_window)) {
        const unsigned long long slot = atomicAdd((unsigned long long*)&a.state[2], 1ull);
        if ((int64_t)slot < a.cand_cap) {
          double* cd = a.cand + 4 * slot;
          cd[0] = lnp;
          cd[1] = rowd[tr * 4 + 3];
          cd[2] = (double)e;
          cd[3] = (double)ob;
        }
      }
    }
    tile_partial<NW>(a, ev, n_pairs_i, n_bounded_i, red, &tile_lnp_max, t);
    // (every pair's ln p and the tile maximum are final: tile_partial has a
    // barrier) the row and column sums relative to the tile maximum, each
    // summed in index order
    {
      const unsigned long long mb = tile_lnp_max;
      const double mxp = mb == 0ull ? -INFINITY : order_value(mb);
      double* rc = a.rowcol + t * 128;
      if (tid < TM) {
        double sum = 0.0;
        for (int c = 0; c < TN; ++c) {
          const double v = lnp_pair[tid * TN + c];
          sum += v == -INFINITY ? 0.0 : exp(v - mxp);
        }
        rc[tid] = sum;
      } else if (tid < TM + TN) {
        const int c = tid - TM;
        double sum = 0.0;
        for (int r = 0; r < TM; ++r) {
          const double v = lnp_pair[r * TN + c];
          sum += v == -INFINITY ? 0.0 : exp(v - mxp);
        }
        rc[64 + c] = sum;
      }
    }
    __syncthreads();   // the tile's scalars and reduction area are reused
  }
}

}  // namespace dotpe
