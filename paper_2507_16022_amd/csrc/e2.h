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

// Per-row and per-column scalars of a tile into LDS, as the fused kernel
// forms them: rowd [TM][4] (ln w_i, row scale, (h|h) row scale, bank row),
// cold [TN][3] (ln w_e, column scale, (h|h) column scale), rowq [TM][2]
// (row scale^2 / (h|h) row scale, ln w_i).  Threads 0 .. TM + TN - 1 write.
template <int PREC, int TM, int TN>
__device__ __forceinline__ void e2_scalars(const FusedArgs& a, int64_t row0, int64_t col0,
                                           double* rowd, double* cold, double* rowq) {
  const int tid = threadIdx.x;
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
}

// The stored accumulators of one pair and the quantities E1 and E2 take
// from them.
template <typename AT, int G, int NRT>
struct PairCoef {
  AT x[2 * G], sv[NRT];
  template <int NPT>
  __device__ __forceinline__ void load(const AT* cf, int p) {
#pragma unroll
    for (int c = 0; c < 2 * G; ++c) x[c] = cf[c * NPT + p];
#pragma unroll
    for (int c = 0; c < NRT; ++c) sv[c] = cf[(2 * G + c) * NPT + p];
  }
  // E1: the certified bound on lnL^ML, the same arithmetic as the fused
  // kernel's epilogue on the same accumulators; true when the pair is
  // bounded (below thr_f), with the bound and ln w_ie in FP32
  __device__ __forceinline__ bool bounded(const double* rowq, const double* cold, int tr, int tc,
                                          float thr_f, float& bound, float& lw) const {
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
    bound = qf * (U0 * U0) * __builtin_amdgcn_rcpf(2.f * lo0) * 1.001f + 1e-3f;
    lw = (float)(rowq[tr * 2 + 1] + cold[tc * 3]);
    return lo0 > 0.f && bound < thr_f;
  }
  // E2 inputs: X_g and the (h|h) phase coefficients at d0, ln w_ie
  __device__ __forceinline__ void unscale(const double* rowd, const double* cold, int tr, int tc,
                                          double2 (&X)[G], double& S0, double (&Sr)[kMaxND],
                                          double (&Si)[kMaxND], double& lnw) const {
    const double sx = rowd[tr * 4 + 1] * cold[tc * 3 + 1];
    const double sh = rowd[tr * 4 + 2] * cold[tc * 3 + 2];
#pragma unroll
    for (int g = 0; g < G; ++g) X[g] = make_double2(sx * (double)x[2 * g], sx * (double)x[2 * g + 1]);
    S0 = sh * (double)sv[0];
#pragma unroll
    for (int d = 0; d < kMaxND; ++d) { Sr[d] = 0.0; Si[d] = 0.0; }
#pragma unroll
    for (int d = 1; d < (NRT + 1) / 2; ++d) {
      Sr[d] = sh * (double)sv[2 * d - 1];
      Si[d] = sh * (double)sv[2 * d];
    }
    lnw = rowd[tr * 4] + cold[tc * 3];
  }
};

template <int PREC, int G>
__device__ __forceinline__ void e2_pass(const FusedArgs& a, int64_t wg_id, int64_t wg_count) {
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

  for (int64_t q = a.work0 + wg_id; q < end; q += wg_count) {
    const int64_t t = coef_tile(a, q);
    const int64_t tm = t / a.n_tiles_n, tn = t % a.n_tiles_n;
    const int64_t row0 = tm * TM, col0 = tn * TN;
    e2_scalars<PREC, TM, TN>(a, row0, col0, rowd, cold, rowq);
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
      PairCoef<AT, G, NRT> pc;
      pc.template load<NPT>(cf, p);
      if (on) {
        float bound, lw;
        if (pc.bounded(rowq, cold, tr, tc, thr_f, bound, lw)) {
          ev.drop.add(lw + bound);
          ev.max_bound = fmaxf(ev.max_bound, lw + bound);
          ++n_bounded_i;
          continue;
        }
      }
      // E2
      double2 X[G];
      double S0, Sr[kMaxND], Si[kMaxND], lnw;
      pc.unscale(rowd, cold, tr, tc, X, S0, Sr, Si, lnw);
      const int64_t e = col0 + tc;
      LsePh lse;
      lse.init();
      double best = -INFINITY, mlmax = 0.0;
      int ob = 0;
      pair_phases<kEvidence, G, true>(a, lds_cs, dp, row0 + tr, e, X, S0, Sr, Si, lnw, thr_ml, 0, 1,
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
      append_candidate(a, lnp >= fmax(thr_topk_glob, tmax - a.topk_window), lnp, rowd[tr * 4 + 3],
                       (double)e, ob);
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

template <int PREC, int G>
__global__ __launch_bounds__(256, 3) void k_e2_tiles(FusedArgs a) {
  e2_pass<PREC, G>(a, blockIdx.x, gridDim.x);
}

// one chunk of the coefficient route's second half for several events
template <int PREC, int G>
__global__ __launch_bounds__(256, 3) void k_e2_tiles_packed(PackLaunch p) {
  int64_t blk, nblk;
  int q;
  const int e = pack_locate(p, blockIdx.x, &blk, &nblk, &q);
  FusedArgs a = pack_args(p, e, q);
  a.work0 = p.chunk * a.coef_tiles;
  e2_pass<PREC, G>(a, blk, nblk);
}

// ---------------------------------------------------------------------------
// Posterior sampling (Sec. III B: resampling by the probabilistic weights;
// Sec. V B).  A systematic draw over the pairs' weights p_ie has been placed
// in tiles (by the tiles' masses from the evidence pass); here each listed
// tile is evaluated again and its draws resolved: the pair by the running
// sum of its weights in index order, then the phase o with probability
// proportional to Lbar_ieo, then the distance from its posterior given that
// triple.
// ---------------------------------------------------------------------------

// D drawn from its posterior given (dh, hh) at d0 with the prior
// proportional to D^2 on (0, D_max] (the integrand of eq.
// lnl_dist_marginalized): in x = ln u, u = d0 / D >= u0 = d0 / D_max, the
// density is proportional to u^-3 exp(dh u - hh u^2 / 2).  Its CDF on NG
// points uniform in x over [ln u0, ln u_hi] (u_hi past the peak by 12
// widths and at least 100 u0) by the trapezoid rule, inverted at `uni` by
// linear interpolation within the cell.  Every lane of the wave takes part
// and gets the result.
__device__ inline double draw_distance(double dh, double hh, double u0, double d0, double uni,
                                       int lane) {
  constexpr int NG = 4096, PER = NG / 64;
  const double us = hh > 0.0 ? fmax(u0, dh / hh) : u0;
  const double sg = hh > 0.0 ? 1.0 / sqrt(hh) : 0.0;
  const double uhi = fmax(100.0 * u0, us + 12.0 * sg);
  const double x0 = log(u0), hx = (log(uhi) - x0) / (NG - 1);
  auto lg = [&](int j) {
    const double x = x0 + hx * j, u = exp(x);
    return -3.0 * x + dh * u - 0.5 * hh * u * u;
  };
  double mx = -INFINITY;
  for (int q = 0; q < PER; ++q) mx = fmax(mx, lg(lane * PER + q));
  mx = wave_max(mx);
  // this lane's cells j = lane * PER .. lane * PER + PER - 1 (the last one
  // stops at NG - 2)
  double part = 0.0, fprev = exp(lg(lane * PER) - mx);
  for (int q = 0; q < PER; ++q) {
    const int j = lane * PER + q;
    if (j + 1 >= NG) break;
    const double fn = exp(lg(j + 1) - mx);
    part += 0.5 * hx * (fprev + fn);
    fprev = fn;
  }
  double pre = part;      // inclusive prefix over lanes
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const double v = __shfl_up(pre, off, 64);
    if (lane >= off) pre += v;
  }
  const double total = __shfl(pre, 63, 64);
  const double target = uni * total;
  const unsigned long long hit = __ballot(pre > target && part > 0.0);
  const int src = hit ? __ffsll((long long)hit) - 1 : 63;
  double x = x0 + hx * (NG - 1);
  if (lane == src && hit) {
    double run = pre - part, fa = exp(lg(lane * PER) - mx);
    for (int q = 0; q < PER; ++q) {
      const int j = lane * PER + q;
      if (j + 1 >= NG) break;
      const double fb = exp(lg(j + 1) - mx), cell = 0.5 * hx * (fa + fb);
      if (run + cell > target) {
        x = x0 + hx * (j + (target - run) / cell);
        break;
      }
      run += cell;
      fa = fb;
    }
  }
  x = __shfl(x, src, 64);
  return d0 / exp(x);
}

template <int PREC, int G>
__global__ __launch_bounds__(256) void k_sample_tiles(FusedArgs a) {
  typedef Tile<PREC> TL;
  typedef typename std::conditional<PREC == kFP64, double, float>::type AT;
  constexpr int NRT = (G == 1) ? 1 : kMaxNR;
  constexpr int NCO = 2 * G + NRT;
  constexpr int TM = TL::TM, TN = TL::TN, NPT = TM * TN, NT = 256, NW = NT / 64;
  __shared__ DistParams dp;
  __shared__ double lds_cs[kMaxM * kMaxPhi * 2];
  __shared__ double rowd[TM * 4], cold[TN * 3], rowq[TM * 2];
  __shared__ double lnp_pair[NPT];

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  for (int t = tid; t < kMaxM * a.n_phi * 2; t += NT) lds_cs[t] = a.phase_cs[t];
  for (int t = tid; t < (int)(sizeof(DistParams) / 4); t += NT)
    ((unsigned*)&dp)[t] = ((const unsigned*)a.dist.prm)[t];
  const bool on = cut_on(a);
  const double thr_ml = on ? __longlong_as_double(a.state[3]) - a.cut_delta : -INFINITY;
  const float thr_f = (float)thr_ml;
  const double M = a.final_out[9];
  const int64_t end = min(a.work0 + a.coef_tiles, coef_work_count(a));

  for (int64_t q = a.work0 + blockIdx.x; q < end; q += gridDim.x) {
    const int64_t t = coef_tile(a, q);
    const int64_t tm = t / a.n_tiles_n, tn = t % a.n_tiles_n;
    const int64_t row0 = tm * TM, col0 = tn * TN;
    e2_scalars<PREC, TM, TN>(a, row0, col0, rowd, cold, rowq);
    __syncthreads();
    const int rows_in = (int)min((int64_t)TM, a.n_sub - row0);
    const int cols_in = (int)min((int64_t)TN, a.n_ext - col0);
    const AT* cf = (const AT*)a.coef + (q - a.work0) * (int64_t)(NCO * NPT);
    // every pair's ln p, as the evidence pass evaluated it
#pragma unroll 1
    for (int k = 0; k < NPT / NT; ++k) {
      const int p = k * NT + tid, tr = p / TN, tc = p % TN;
      lnp_pair[p] = -INFINITY;
      if (!(tr < rows_in && tc < cols_in)) continue;
      PairCoef<AT, G, NRT> pc;
      pc.template load<NPT>(cf, p);
      float bound, lw;
      if (on && pc.bounded(rowq, cold, tr, tc, thr_f, bound, lw)) continue;
      double2 X[G];
      double S0, Sr[kMaxND], Si[kMaxND], lnw;
      pc.unscale(rowd, cold, tr, tc, X, S0, Sr, Si, lnw);
      EvAcc ev;
      ev.init();
      LsePh lse;
      lse.init();
      double best = -INFINITY, mlmax = 0.0;
      int ob = 0;
      pair_phases<kEvidence, G, false>(a, lds_cs, dp, row0 + tr, col0 + tc, X, S0, Sr, Si, lnw,
                                      thr_ml, 0, 1, ev, lse, best, ob, mlmax);
      if (lse.m == -INFINITY) continue;
      lnp_pair[p] = lnw + (lse.m + log(lse.s) - a.ln_nphi);
    }
    __syncthreads();
    // the tile's reference: its largest ln p in the evidence pass
    const double pm = a.partials[t * kNPart];
    for (int64_t s = a.sample_first[q] + wave; s < a.sample_first[q + 1]; s += NW) {
      // the pair: the draw's residual mass within the tile, against the
      // running sum of the pairs' weights in index order
      const double r = a.sample_res[s] * exp(M - pm);
      double run = 0.0;
      int sel = -1, last = -1;
      for (int c0 = 0; c0 < NPT; c0 += 64) {
        const double v = lnp_pair[c0 + lane];
        const double x = v == -INFINITY ? 0.0 : exp(v - pm);
        const unsigned long long live = __ballot(v > -INFINITY);
        if (live) last = c0 + 63 - __clzll((long long)live);
        double pre = x;
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) {
          const double y = __shfl_up(pre, off, 64);
          if (lane >= off) pre += y;
        }
        if (sel < 0) {
          const unsigned long long hit = __ballot(x > 0.0 && run + pre > r);
          if (hit) sel = c0 + __ffsll((long long)hit) - 1;
        }
        run += __shfl(pre, 63, 64);
      }
      if (sel < 0) sel = last;       // rounding past the tile's total
      if (sel < 0) continue;         // (a tile with mass always has a pair)
      const int tr = sel / TN, tc = sel % TN;
      PairCoef<AT, G, NRT> pc;
      pc.template load<NPT>(cf, sel);
      double2 X[G];
      double S0, Sr[kMaxND], Si[kMaxND], lnw;
      pc.unscale(rowd, cold, tr, tc, X, S0, Sr, Si, lnw);
      // the phase: probability Lbar_ieo over the phases kept by the cut
      double v_o[2], dh_o[2], hh_o[2];
      for (int h = 0; h < 2; ++h) {
        const int o = lane + 64 * h;
        v_o[h] = -INFINITY;
        dh_o[h] = 0.0;
        hh_o[h] = 0.0;
        if (o < a.n_phi) {
          phase_dh_hh<G>(a, lds_cs, X, S0, Sr, Si, o, dh_o[h], hh_o[h]);
          const bool keep = thr_ml <= 0.0 || (dh_o[h] > 0.0 && dh_o[h] * dh_o[h] >= 2.0 * thr_ml * hh_o[h]);
          if (keep) v_o[h] = dr_ln_marg(dh_o[h], hh_o[h], a.r0, a.dist.tab, dp.ghx, dp.ghw);
        }
      }
      const double vmax = wave_max(fmax(v_o[0], v_o[1]));
      const double w0 = v_o[0] == -INFINITY ? 0.0 : exp(v_o[0] - vmax);
      const double w1 = v_o[1] == -INFINITY ? 0.0 : exp(v_o[1] - vmax);
      double pre0 = w0, pre1 = w1;
#pragma unroll
      for (int off = 1; off < 64; off <<= 1) {
        const double y0 = __shfl_up(pre0, off, 64), y1 = __shfl_up(pre1, off, 64);
        if (lane >= off) { pre0 += y0; pre1 += y1; }
      }
      const double tot0 = __shfl(pre0, 63, 64);
      const double tot = tot0 + __shfl(pre1, 63, 64);
      const double target = sm64_uniform(a.seed, 2 * (uint64_t)s) * tot;
      const unsigned long long h0 = __ballot(w0 > 0.0 && pre0 > target);
      const unsigned long long h1 = __ballot(w1 > 0.0 && tot0 + pre1 > target);
      int osel;
      if (h0) osel = __ffsll((long long)h0) - 1;
      else if (h1) osel = 64 + __ffsll((long long)h1) - 1;
      else {   // rounding past the total: the last kept phase
        const unsigned long long k0 = __ballot(w0 > 0.0), k1 = __ballot(w1 > 0.0);
        osel = k1 ? 64 + 63 - __clzll((long long)k1) : 63 - __clzll((long long)k0);
      }
      const int src = osel & 63, hs = osel >> 6;
      const double dh = __shfl(hs ? dh_o[1] : dh_o[0], src, 64);
      const double hh = __shfl(hs ? hh_o[1] : hh_o[0], src, 64);
      const double v = __shfl(hs ? v_o[1] : v_o[0], src, 64);
      const double D = draw_distance(dh, hh, a.r0, a.d0,
                                     sm64_uniform(a.seed, 2 * (uint64_t)s + 1), lane);
      if (lane == 0) {
        double* out = a.samples + 6 * s;
        out[0] = rowd[tr * 4 + 3];
        out[1] = (double)(col0 + tc);
        out[2] = (double)osel;
        out[3] = D;
        out[4] = lnp_pair[sel];
        out[5] = lnw + v - a.ln_nphi;
      }
    }
    __syncthreads();   // the tile's scalars and pair values are reused
  }
}

}  // namespace dotpe
