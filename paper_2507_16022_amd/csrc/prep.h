// Per-bank and per-event preparation kernels (bank-summary layout,
// extrinsic response and operand, (h|h) tables, (d|d)), the evidence
// finalisation and the top-k sort.  Included by the host runtime only.
#pragma once

#include "common.h"

namespace dotpe {

// ---------------------------------------------------------------------------
// distance-marginalisation table
// ---------------------------------------------------------------------------
__global__ void k_build_dist_table(double* tab, DistTableGeom g) {
  int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (int64_t)g.ncol * g.nrow) return;
  const int col = (int)(idx % g.ncol), row = (int)(idx / g.ncol);
  int k = 0;
  while (k + 1 < kDrRowSeg && row >= g.roff[k + 1]) ++k;
  const double w = g.wlo[k] + (row - g.roff[k] - 2) / g.ihw[k];   // two guard rows below the edge
  tab[idx] = dr_ln_exact(dr_col_z(g, col), g.wlog[k] ? exp(w) : 1.0 + w);
}

__global__ void k_debug_distmarg(int64_t n, const double* dh, const double* hh, double r0,
                                 DistArgs da, double* out) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  out[i] = dr_ln_marg(dh[i], hh[i], r0, da.tab, da.prm->ghx, da.prm->ghw);
}

// Element offset of (row i, position k) in an operand with K positions per
// row (K a multiple of 32).  FP64: row-major.  Split precisions: fragment
// order -- 32-row blocks; within a block each chunk of 32 positions is 2 KB
// ---------------------------------------------------------------------------
// bank-summary layout: FP64 amplitudes -> MFMA operand rows
// row layout (K2 = n_c * n_bp * 2 per row): for channel c (group order) and
// chunk j of 16 bins, 32 consecutive values: Re A (16 bins) then Im A,
// A = conj(h) (scaled by 2^-e_i in the split precisions).
// ---------------------------------------------------------------------------
template <int PREC>
__global__ void k_bank_convert(const double* __restrict__ h, int64_t n_wf, int n_c_in, int n_b,
                               int n_bp, ModeTables mt, void* __restrict__ A0,
                               void* __restrict__ A1, double* __restrict__ row_scale,
                               int* __restrict__ err, void* __restrict__ R0,
                               void* __restrict__ R1) {
  const int64_t row = blockIdx.x;
  if (row >= n_wf) return;
  const double* hr = h + (size_t)row * n_c_in * n_b * 2;
  __shared__ double red[256];
  double mx = 0.0;
  bool bad = false;
  for (int t = threadIdx.x; t < n_c_in * n_b; t += blockDim.x) {
    double re = hr[2 * t], im = hr[2 * t + 1];
    if (!isfinite(re) || !isfinite(im)) bad = true;
    mx = fmax(mx, fmax(fabs(re), fabs(im)));
  }
  if (bad) atomicOr(err, 1);
  red[threadIdx.x] = mx;
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + s]);
    __syncthreads();
  }
  mx = red[0];
  int ex = 0;
  if (PREC != kFP64 && mx > 0.0 && isfinite(mx)) ex = ilogb(mx) - 13;   // max in [2^13, 2^14)
  if (threadIdx.x == 0 && row_scale) row_scale[row] = ldexp(1.0, ex);
  const int64_t K2 = (int64_t)mt.n_c * n_bp * 2;
  for (int t = threadIdx.x; t < mt.n_c * n_bp; t += blockDim.x) {
    int c = t / n_bp, b = t % n_bp;
    double re = 0.0, im = 0.0;
    if (b < n_b) {
      const double* src = hr + ((size_t)mt.orig[c] * n_b + b) * 2;
      re = ldexp(src[0], -ex);
      im = -ldexp(src[1], -ex);                 // conj(h)
    }
    const int64_t base = ((int64_t)c * (n_bp / kChunk) + b / kChunk) * 32 + (b % kChunk);
    const int64_t o = op_index<PREC>(row, base, K2), o16 = op_index<PREC>(row, base + 16, K2);
    if (PREC == kFP64) {
      double* A = (double*)A0;
      A[o] = re;
      A[o16] = im;
    } else if (PREC == kFP16X2) {
      _Float16* Ah = (_Float16*)A0;
      _Float16* Al = (_Float16*)A1;
      _Float16 hr_ = (_Float16)re, hi_ = (_Float16)im;
      const _Float16 lr_ = (_Float16)(re - (double)hr_), li_ = (_Float16)(im - (double)hi_);
      Ah[o] = hr_; Ah[o16] = hi_;
      Al[o] = lr_; Al[o16] = li_;
      if (R0) {
        _Float16* Rh = (_Float16*)R0 + row * K2;
        _Float16* Rl = (_Float16*)R1 + row * K2;
        Rh[base] = hr_; Rh[base + 16] = hi_;
        Rl[base] = lr_; Rl[base + 16] = li_;
      }
    } else {
      __bf16* Ah = (__bf16*)A0;
      __bf16* Al = (__bf16*)A1;
      __bf16 hr_ = (__bf16)(float)re, hi_ = (__bf16)(float)im;
      const __bf16 lr_ = (__bf16)(float)(re - (double)(float)hr_);
      const __bf16 li_ = (__bf16)(float)(im - (double)(float)hi_);
      Ah[o] = hr_; Ah[o16] = hi_;
      Al[o] = lr_; Al[o16] = li_;
      if (R0) {
        __bf16* Rh = (__bf16*)R0 + row * K2;
        __bf16* Rl = (__bf16*)R1 + row * K2;
        Rh[base] = hr_; Rh[base + 16] = hi_;
        Rl[base] = lr_; Rl[base + 16] = li_;
      }
    }
  }
}

// reconstructed conj(h) value (A) of row i, channel c (group order), bin b
template <int PREC>
__device__ __forceinline__ double2 bank_value(const void* A0, const void* A1, int64_t i, int64_t K2,
                                              int c, int b, int n_bp) {
  const int64_t base = ((int64_t)c * (n_bp / kChunk) + b / kChunk) * 32 + (b % kChunk);
  const int64_t o = op_index<PREC>(i, base, K2), o16 = op_index<PREC>(i, base + 16, K2);
  if (PREC == kFP64) {
    const double* A = (const double*)A0;
    return make_double2(A[o], A[o16]);
  } else if (PREC == kFP16X2) {
    const _Float16* Ah = (const _Float16*)A0;
    const _Float16* Al = (const _Float16*)A1;
    return make_double2((double)Ah[o] + (double)Al[o], (double)Ah[o16] + (double)Al[o16]);
  } else {
    const __bf16* Ah = (const __bf16*)A0;
    const __bf16* Al = (const __bf16*)A1;
    return make_double2((double)(float)Ah[o] + (double)(float)Al[o],
                        (double)(float)Ah[o16] + (double)(float)Al[o16]);
  }
}

// ---------------------------------------------------------------------------
// extrinsic response (Sec. IV A): antenna patterns, arrival times, mode
// factors, R_ekc, |R_ekc|^2 and Q_ekcc'
// ---------------------------------------------------------------------------
__global__ void k_ext_response(int64_t n_ext, int n_det, const double* __restrict__ det_r,
                               const double* __restrict__ det_D, const double* __restrict__ lat,
                               const double* __restrict__ lon, const double* __restrict__ psi,
                               const double* __restrict__ cosi, const double* __restrict__ tgeo,
                               ModeTables mt, double2* __restrict__ R, double* __restrict__ T,
                               double2* __restrict__ Q, double* __restrict__ R2) {
  int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n_ext) return;
  const double C = 299792458.0;
  double la = lat[e], lo = lon[e], ps = psi[e];
  double sla = sin(la), cla = cos(la), slo = sin(lo), clo = cos(lo), sps = sin(ps), cps = cos(ps);
  double n[3] = {cla * clo, cla * slo, sla};
  double elon[3] = {-slo, clo, 0.0};
  double elat[3] = {-sla * clo, -sla * slo, cla};
  double X[3], Y[3];
  for (int a = 0; a < 3; ++a) {
    X[a] = cps * elon[a] + sps * elat[a];
    Y[a] = -sps * elon[a] + cps * elat[a];
  }
  // per channel and polarisation the factor of F_kp in R_ekc: the -2Y_lm
  // combinations (layout (l, m)), or 1 for the channel's own polarisation
  // (layout (m, p), the inclination inside the bank)
  double2 K[kMaxC][2];
  for (int c = 0; c < mt.n_c; ++c) {
    if (mt.layout == 1) {
      K[c][0] = make_double2(mt.pol[c] == 0 ? 1.0 : 0.0, 0.0);
      K[c][1] = make_double2(mt.pol[c] == 1 ? 1.0 : 0.0, 0.0);
      continue;
    }
    int l = mt.l[c], m = mt.m[c];
    double yn = swsh_m2(l, -m, cosi[e]), yp = swsh_m2(l, m, cosi[e]);
    double sg = (l & 1) ? -1.0 : 1.0;
    K[c][0] = make_double2(0.5 * (yn + sg * yp), 0.0);
    K[c][1] = make_double2(0.0, 0.5 * (yn - sg * yp));
  }
  for (int k = 0; k < n_det; ++k) {
    const double* Dk = det_D + 9 * k;
    double fp = 0.0, fx = 0.0, rn = 0.0;
    for (int a = 0; a < 3; ++a) {
      rn += det_r[3 * k + a] * n[a];
      for (int b = 0; b < 3; ++b) {
        fp += Dk[3 * a + b] * (X[a] * X[b] - Y[a] * Y[b]);
        fx += Dk[3 * a + b] * (X[a] * Y[b] + Y[a] * X[b]);
      }
    }
    T[e * n_det + k] = tgeo[e] - rn / C;
    double2 Rk[kMaxC];
    for (int c = 0; c < mt.n_c; ++c) {
      Rk[c] = make_double2(fp * K[c][0].x + fx * K[c][1].x, fp * K[c][0].y + fx * K[c][1].y);
      R[(e * n_det + k) * mt.n_c + c] = Rk[c];
      R2[(e * n_det + k) * mt.n_c + c] = Rk[c].x * Rk[c].x + Rk[c].y * Rk[c].y;
    }
    for (int p = 0; p < mt.NP; ++p)
      Q[(e * n_det + k) * mt.NP + p] = cmul(Rk[mt.pc[p]], cconj(Rk[mt.pc2[p]]));
  }
}

// B_cb(e) = sum_k w_kb d_kb conj(R_ekc) exp(+2 pi i f_b t_ek), bins padded
// B_ecb = sum_k W_kcb conj(R_ekc) exp(2 pi i f_b t_ek) with W_kcb = w_kb d_kb
// (plain bins) or the relative-binning weights wdh [n_det][n_c][n_b] (group
// order) when given
__global__ void k_build_B(int64_t n_ext, int n_det, int n_c, int n_b, int n_bp,
                          const double* __restrict__ f, const double2* __restrict__ d,
                          const double* __restrict__ w, const double2* __restrict__ wdh,
                          const double2* __restrict__ R, const double* __restrict__ T,
                          double2* __restrict__ Btmp) {
  int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int64_t total = n_ext * n_c * n_bp;
  if (idx >= total) return;
  int b = (int)(idx % n_bp);
  int c = (int)((idx / n_bp) % n_c);
  int64_t e = idx / ((int64_t)n_bp * n_c);
  double2 acc = make_double2(0.0, 0.0);
  if (b < n_b) {
    for (int k = 0; k < n_det; ++k) {
      double x = f[b] * T[e * n_det + k];     // cycles
      double fr = x - rint(x);
      double sn, cs;
      sincos(2.0 * M_PI * fr, &sn, &cs);
      double2 r = cconj(R[(e * n_det + k) * n_c + c]);
      double2 wd;
      if (wdh) {
        wd = wdh[((int64_t)k * n_c + c) * n_b + b];
      } else {
        const double2 dk = d[k * n_b + b];
        const double wk = w[k * n_b + b];
        wd = make_double2(wk * dk.x, wk * dk.y);
      }
      double2 v = cmul(cmul(wd, r), make_double2(cs, sn));
      acc.x += v.x;
      acc.y += v.y;
    }
  }
  Btmp[idx] = acc;
}

template <int PREC>
__device__ __forceinline__ void store_split(void* A0, void* A1, int64_t o, double v) {
  if (PREC == kFP64) {
    ((double*)A0)[o] = v;
  } else if (PREC == kFP16X2) {
    _Float16 h = (_Float16)v;
    ((_Float16*)A0)[o] = h;
    ((_Float16*)A1)[o] = (_Float16)(v - (double)h);
  } else {
    __bf16 h = (__bf16)(float)v;
    ((__bf16*)A0)[o] = h;
    ((__bf16*)A1)[o] = (__bf16)(float)(v - (double)(float)h);
  }
}

// extrinsic operand rows: Bre = [Br | -Bi], Bim = [Bi | Br] per chunk,
// scaled by 2^-g_e in the split precisions; rows e >= n_ext are zero
template <int PREC>
__global__ void k_convert_B(int64_t n_ext, int64_t n_ext_p, int n_c, int n_bp,
                            const double2* __restrict__ Btmp, void* __restrict__ B0,
                            void* __restrict__ B1, void* __restrict__ B2, void* __restrict__ B3,
                            double* __restrict__ col_scale, int* __restrict__ err) {
  const int64_t e = blockIdx.x;
  if (e >= n_ext_p) return;
  __shared__ double red[256];
  const int n = n_c * n_bp;
  double mx = 0.0;
  bool bad = false;
  if (e < n_ext) {
    for (int t = threadIdx.x; t < n; t += blockDim.x) {
      double2 v = Btmp[e * n + t];
      if (!isfinite(v.x) || !isfinite(v.y)) bad = true;
      mx = fmax(mx, fmax(fabs(v.x), fabs(v.y)));
    }
  }
  if (bad) atomicOr(err, 2);
  red[threadIdx.x] = mx;
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + s]);
    __syncthreads();
  }
  mx = red[0];
  int ex = 0;
  if (PREC != kFP64 && mx > 0.0 && isfinite(mx)) ex = ilogb(mx) - 13;
  if (threadIdx.x == 0 && col_scale && e < n_ext) col_scale[e] = ldexp(1.0, ex);
  const int64_t K2 = (int64_t)n * 2;
  for (int t = threadIdx.x; t < n; t += blockDim.x) {
    int c = t / n_bp, b = t % n_bp;
    double br = 0.0, bi = 0.0;
    if (e < n_ext) {
      double2 v = Btmp[e * n + t];
      br = ldexp(v.x, -ex);
      bi = ldexp(v.y, -ex);
    }
    const int64_t base = ((int64_t)c * (n_bp / kChunk) + b / kChunk) * 32 + (b % kChunk);
    const int64_t o = op_index<PREC>(e, base, K2), o16 = op_index<PREC>(e, base + 16, K2);
    if (PREC == kFP64) {
      double* Bre = (double*)B0;
      double* Bim = (double*)B1;
      Bre[o] = br; Bre[o16] = -bi;     // B_re = [Br | -Bi]
      Bim[o] = bi; Bim[o16] = br;      // B_im = [Bi | Br]
    } else {
      // split precisions: B_re only (B_im is the other slice of B_re)
      store_split<PREC>(B0, B1, o, br);
      store_split<PREC>(B0, B1, o16, -bi);
    }
  }
}

// Chunk ranges [c0[r], c0[r + 1]), r < n, of an operand row (chunks of 32
// positions): the m groups of a (d|h) operand, the outputs of a (h|h) one.
struct NormRanges {
  int n;
  int c0[kMaxNR + 2];
};

// Per row of a split operand (op_index layout, K positions per row) and
// per chunk range: the 2-norm of its hi parts and the 2-norm of what a
// product of the hi parts alone leaves out -- the lo parts, plus any hi part
// below the format's normal range in case the matrix cores flush it -- each
// rounded up to float: out[row * n + r] = (hi, left out).  The bound pass
// builds its margin from them.  A thread per row: the lanes of a wave read
// 16 contiguous bytes each, 512 contiguous bytes per 32-row block.
template <int PREC>
__global__ void k_operand_norms(const void* __restrict__ P0, const void* __restrict__ P1,
                                int64_t n_rows, int64_t K, NormRanges rg, float2* __restrict__ out) {
  typedef typename std::conditional<PREC == kFP16X2, _Float16, __bf16>::type H;
  const int64_t row = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (row >= n_rows) return;
  const int64_t base = (row >> 5) * (K >> 5) * 1024 + (row & 31) * 8;
  const double tiny = PREC == kFP16X2 ? 0x1p-14 : 0x1p-126;
  for (int r = 0; r < rg.n; ++r) {
    double sh = 0.0, sl = 0.0;
    for (int64_t c = rg.c0[r]; c < rg.c0[r + 1]; ++c)
#pragma unroll
      for (int q = 0; q < 4; ++q) {     // (slice, piece) of the chunk
        const int64_t o = base + c * 1024 + q * 256;
        const uint4 vh = *(const uint4*)((const H*)P0 + o);
        const uint4 vl = *(const uint4*)((const H*)P1 + o);
        H xh[8], xl[8];
        __builtin_memcpy(xh, &vh, 16);
        __builtin_memcpy(xl, &vl, 16);
#pragma unroll
        for (int j = 0; j < 8; ++j) {
          const double h = (double)(float)xh[j], l = (double)(float)xl[j];
          const double t = fabs(h) < tiny ? l + h : l;
          sh += h * h;
          sl += t * t;
        }
      }
    out[row * rg.n + r] = make_float2((float)(sqrt(sh) * (1.0 + 0x1p-20)),
                                      (float)(sqrt(sl) * (1.0 + 0x1p-20)));
  }
}

// ---------------------------------------------------------------------------
// relative-binning weights (App. A, eqs. dh_weights, hh_weights): a thread
// per (k, c, b) of W^dh and per (k, c, c', b) of W^hh, each a sum over the
// full-resolution points of the hat function s_b's support (from the node
// before to the node after).  Reference of detector k: h0_c(f) exp(-2 pi i
// f t0_k), so W^dh carries exp(2 pi i (f - f_b) t0_k), reduced in cycles,
// and W^hh none.
// ---------------------------------------------------------------------------
__global__ void k_rb_weights(int n_det, int n_c, int64_t n_full, int n_nodes,
                             const double* __restrict__ f, const double2* __restrict__ d,
                             const double* __restrict__ w, const double2* __restrict__ h0,
                             const double* __restrict__ t0, const int64_t* __restrict__ node_idx,
                             double2* __restrict__ wdh, double2* __restrict__ whh) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t n_dh = (int64_t)n_det * n_c * n_nodes;
  const int64_t n_hh = (int64_t)n_det * n_c * n_c * n_nodes;
  if (idx >= n_dh + n_hh) return;
  const bool is_dh = idx < n_dh;
  const int64_t j = is_dh ? idx : idx - n_dh;
  const int b = (int)(j % n_nodes);
  int c, c2 = 0, k;
  if (is_dh) {
    c = (int)((j / n_nodes) % n_c);
    k = (int)(j / ((int64_t)n_nodes * n_c));
  } else {
    c2 = (int)((j / n_nodes) % n_c);
    c = (int)((j / ((int64_t)n_nodes * n_c)) % n_c);
    k = (int)(j / ((int64_t)n_nodes * n_c * n_c));
  }
  const int64_t qb = node_idx[b];
  const int64_t lo = b > 0 ? node_idx[b - 1] : qb, hi = b + 1 < n_nodes ? node_idx[b + 1] : qb;
  const double fb = f[qb], flo = f[lo], fhi = f[hi];
  const double tk = t0 ? t0[k] : 0.0;
  double2 acc = make_double2(0.0, 0.0);
  for (int64_t q = lo; q <= hi; ++q) {
    const double fq = f[q];
    const double s = q < qb ? (fq - flo) / (fb - flo) : q > qb ? (fhi - fq) / (fhi - fb) : 1.0;
    const double ws = w[(int64_t)k * n_full + q] * s;
    double2 v;
    if (is_dh) {
      const double x = (fq - fb) * tk;
      double sn, cs;
      sincospi(2.0 * (x - rint(x)), &sn, &cs);
      v = cmul(cmul(d[(int64_t)k * n_full + q], cconj(h0[(int64_t)c * n_full + q])), make_double2(cs, sn));
    } else {
      v = cmul(h0[(int64_t)c * n_full + q], cconj(h0[(int64_t)c2 * n_full + q]));
    }
    acc.x += ws * v.x;
    acc.y += ws * v.y;
  }
  // divide by conj(h0_c(f_b)), or by h0_c(f_b) conj(h0_c'(f_b))
  double2 den = cconj(h0[(int64_t)c * n_full + qb]);
  if (!is_dh) den = cmul(h0[(int64_t)c * n_full + qb], cconj(h0[(int64_t)c2 * n_full + qb]));
  const double dn = den.x * den.x + den.y * den.y;
  const double2 r = cmul(acc, cconj(den));
  (is_dh ? wdh : whh)[j] = make_double2(r.x / dn, r.y / dn);
}

// ---------------------------------------------------------------------------
// extrinsic-sample proposals (Sec. IV E; App. C): per intrinsic sample c a
// distribution over the cells (sky lattice point s, geocentre-time cell j)
// from the detectors' arrival-time probabilities, their mixture, draws and
// importance weights
// ---------------------------------------------------------------------------
struct PropGeom {
  int C, S, J, K, n_t;
  double t0[kMaxDet], dt, r[kMaxDet][3];
  double tg_lo, dtg, beta;
};

__device__ __forceinline__ void fib_sky(int s, int S, double* lat, double* lon) {
  const double z = 1.0 - (2.0 * s + 1.0) / S;
  const double ga = M_PI * (3.0 - sqrt(5.0));
  *lat = asin(z);
  *lon = fmod((double)s * ga, 2.0 * M_PI);
}

// rmax[c][k] = max_j of the per-time maxima ml[c][k][j]
__global__ void k_prop_max(const double* __restrict__ ml, PropGeom g, double* __restrict__ rmax) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= g.C * g.K) return;
  double m = -INFINITY;
  for (int j = 0; j < g.n_t; ++j) m = fmax(m, ml[(int64_t)t * g.n_t + j]);
  rmax[t] = m;
}

// ln W_c(s, j) = sum_k beta (rho^2_ck(t_i) - max rho^2_ck), i the grid point
// nearest to t_j - r_k . n_s / c (-inf off the grid); rho^2 = 2 ml
__global__ void k_prop_table(const double* __restrict__ ml, const double* __restrict__ rmax,
                             PropGeom g, double* __restrict__ lnW) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t SJ = (int64_t)g.S * g.J;
  if (idx >= (int64_t)g.C * SJ) return;
  const int c = (int)(idx / SJ);
  const int s = (int)((idx % SJ) / g.J), j = (int)(idx % g.J);
  double lat, lon;
  fib_sky(s, g.S, &lat, &lon);
  const double n0 = cos(lat) * cos(lon), n1 = cos(lat) * sin(lon), n2 = sin(lat);
  const double tj = g.tg_lo + (j + 0.5) * g.dtg;
  double acc = 0.0;
  for (int k = 0; k < g.K; ++k) {
    const double tk = tj - (g.r[k][0] * n0 + g.r[k][1] * n1 + g.r[k][2] * n2) / 299792458.0;
    const double x = rint((tk - g.t0[k]) / g.dt);
    if (!(x >= 0.0 && x < g.n_t)) {
      acc = -INFINITY;
      break;
    }
    const int64_t ck = (int64_t)c * g.K + k;
    acc += g.beta * 2.0 * (ml[ck * g.n_t + (int)x] - rmax[ck]);
  }
  lnW[idx] = acc;
}

// ln Z_c = LSE over the cells of ln W_c, in two steps: blocks (part, c) each
// reduce one of kPropParts contiguous ranges of component c's cells to (max,
// sum of exp(x - max)), lanes then threads in a fixed tree order; then a
// block per c merges its parts the same way.
constexpr int kPropParts = 256;

__device__ __forceinline__ void lse_merge(double& m, double& s, double m2, double s2) {
  if (m2 == -INFINITY) return;
  if (m2 > m) {
    s = s * exp(m - m2) + s2;
    m = m2;
  } else {
    s += s2 * exp(m2 - m);
  }
}

// (m, s) of the 256 threads' (m, s) in LDS, tree order; thread 0 gets them
__device__ __forceinline__ void lse_block_256(double* sm, double* ss, double& m, double& s) {
  sm[threadIdx.x] = m;
  ss[threadIdx.x] = s;
  __syncthreads();
  for (int k = 128; k > 0; k >>= 1) {
    if ((int)threadIdx.x < k) {
      double a = sm[threadIdx.x], b = ss[threadIdx.x];
      lse_merge(a, b, sm[threadIdx.x + k], ss[threadIdx.x + k]);
      sm[threadIdx.x] = a;
      ss[threadIdx.x] = b;
    }
    __syncthreads();
  }
  m = sm[0];
  s = ss[0];
}

__global__ __launch_bounds__(256) void k_prop_lse_part(const double* __restrict__ lnW, PropGeom g,
                                                        double* __restrict__ part) {
  __shared__ double sm[256], ss[256];
  const int c = blockIdx.y, p = blockIdx.x;
  const int64_t SJ = (int64_t)g.S * g.J, per = (SJ + kPropParts - 1) / kPropParts;
  const int64_t lo = p * per, hi = min(SJ, lo + per);
  const double* x = lnW + (int64_t)c * SJ;
  double m = -INFINITY, s = 0.0;
  for (int64_t t = lo + threadIdx.x; t < hi; t += 256) lse_merge(m, s, x[t], 1.0);
  lse_block_256(sm, ss, m, s);
  if (threadIdx.x == 0) {
    part[2 * ((int64_t)c * kPropParts + p)] = m;
    part[2 * ((int64_t)c * kPropParts + p) + 1] = s;
  }
}

__global__ __launch_bounds__(256) void k_prop_lse(const double* __restrict__ part,
                                                   double* __restrict__ lnZ) {
  static_assert(kPropParts == 256, "one part per thread");
  __shared__ double sm[256], ss[256];
  const int c = blockIdx.x;
  double m = part[2 * ((int64_t)c * kPropParts + threadIdx.x)];
  double s = part[2 * ((int64_t)c * kPropParts + threadIdx.x) + 1];
  lse_block_256(sm, ss, m, s);
  if (threadIdx.x == 0) lnZ[c] = m == -INFINITY ? -INFINITY : m + log(s);
}

// P_c(cell) = W_c / Z_c (in place over ln W), and the mixture (1/C) sum_c P_c
__global__ void k_prop_prob(double* __restrict__ x, const double* __restrict__ lnZ, PropGeom g,
                            double* __restrict__ mix) {
  const int64_t cell = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t SJ = (int64_t)g.S * g.J;
  if (cell >= SJ) return;
  double m = 0.0;
  for (int c = 0; c < g.C; ++c) {
    const double v = x[(int64_t)c * SJ + cell];
    const double p = (v == -INFINITY || lnZ[c] == -INFINITY) ? 0.0 : exp(v - lnZ[c]);
    x[(int64_t)c * SJ + cell] = p;
    m += p;
  }
  mix[cell] = m / g.C;
}

// draws: q from component q mod C, its cell the first whose running sum
// (cum: inclusive running sums over the components back to back) exceeds
// u times the component's total
__global__ void k_prop_draw(const double* __restrict__ cum, const double* __restrict__ mix,
                            PropGeom g, int64_t n_s, uint64_t seed, double* __restrict__ out) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= n_s) return;
  const int64_t SJ = (int64_t)g.S * g.J;
  const int c = (int)(q % g.C);
  const int64_t lo0 = (int64_t)c * SJ;
  const double base = c > 0 ? cum[lo0 - 1] : 0.0;
  const double tot = cum[lo0 + SJ - 1] - base;
  const double target = sm64_uniform(seed, 4 * (uint64_t)q) * tot;
  int64_t lo = 0, hi = SJ - 1;          // first x with cum[lo0 + x] - base > target (the last if none)
  while (lo < hi) {
    const int64_t mid = (lo + hi) / 2;
    if (cum[lo0 + mid] - base > target) hi = mid;
    else lo = mid + 1;
  }
  const int s = (int)(lo / g.J), j = (int)(lo % g.J);
  double lat, lon;
  fib_sky(s, g.S, &lat, &lon);
  double* o = out + 7 * q;
  o[0] = lat;
  o[1] = lon;
  o[2] = M_PI * sm64_uniform(seed, 4 * (uint64_t)q + 2);
  o[3] = 2.0 * sm64_uniform(seed, 4 * (uint64_t)q + 3) - 1.0;
  o[4] = g.tg_lo + (j + sm64_uniform(seed, 4 * (uint64_t)q + 1)) * g.dtg;
  o[5] = -log((double)SJ) - log(mix[lo]);
  o[6] = (double)lo;
}

// cells of the mixture's support (mix > 0), counted into *n (zeroed before)
__global__ __launch_bounds__(256) void k_count_support(const double* __restrict__ mix, int64_t SJ,
                                                       unsigned long long* __restrict__ n) {
  const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const unsigned long long v = __ballot(t < SJ && mix[t] > 0.0);
  if ((threadIdx.x & 63) == 0 && v) atomicAdd(n, (unsigned long long)__popcll(v));
}

// N_eff over the draws' weights and the prior mass of the mixture's support:
// one block; st[0] = (sum w)^2 / sum w^2, st[1] = support (from the count)
__global__ void k_prop_stats(const double* __restrict__ out, int64_t n_s,
                             const unsigned long long* __restrict__ n_support, int64_t SJ,
                             double* __restrict__ st) {
  __shared__ double a[256], b[256], m[256];
  double mx = -INFINITY;
  for (int64_t q = threadIdx.x; q < n_s; q += 256) mx = fmax(mx, out[7 * q + 5]);
  m[threadIdx.x] = mx;
  __syncthreads();
  if (threadIdx.x == 0) {
    double M = -INFINITY;
    for (int t = 0; t < 256; ++t) M = fmax(M, m[t]);
    m[0] = M;
  }
  __syncthreads();
  const double M = m[0];
  double s1 = 0.0, s2 = 0.0;
  for (int64_t q = threadIdx.x; q < n_s; q += 256) {
    const double v = exp(out[7 * q + 5] - M);
    s1 += v;
    s2 += v * v;
  }
  a[threadIdx.x] = s1;
  b[threadIdx.x] = s2;
  __syncthreads();
  if (threadIdx.x == 0) {
    double A = 0.0, B = 0.0;
    for (int t = 0; t < 256; ++t) {
      A += a[t];
      B += b[t];
    }
    st[0] = A * A / B;
    st[1] = (double)*n_support / (double)SJ;
  }
}

// (d|d)
__global__ void k_data_norm(int n, const double2* __restrict__ d, const double* __restrict__ w,
                            double* __restrict__ out) {
  __shared__ double red[256];
  double s = 0.0;
  for (int t = threadIdx.x; t < n; t += blockDim.x) s += w[t] * (d[t].x * d[t].x + d[t].y * d[t].y);
  red[threadIdx.x] = s;
  __syncthreads();
  for (int k = blockDim.x / 2; k > 0; k >>= 1) {
    if (threadIdx.x < k) red[threadIdx.x] += red[threadIdx.x + k];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = red[0];
}

// ---------------------------------------------------------------------------
// (h|h) operands.  For one pair, the phase coefficients of (h|h)
//     S0 (real), Re S_d, Im S_d (d = 1 .. ND-1)      -- NR = 2 ND - 1 outputs
// are each a dot product of at most 32 terms a * b with a taken from the
// waveform's H_ikcc' and b from the sample's Q_ekcc'; they are computed by
// the same matrix cores as (d|h), as extra K blocks of 32.  A term (output r,
// slot j) is encoded in 17 bits: k (0-3), p (4-9), a from Im H (10), b from
// Im Q (11), coefficient index (12-14: 0, 1, -1, 2, -2), valid (15), and
// folded (16): p is then an entry of the (m, p) layout's folded sums, whose
// row value sums its member pairs and whose column value is its first
// member's (every member has the same F_kp F_kp').
// ---------------------------------------------------------------------------

__device__ __forceinline__ double term_value(int code, const double2* X, const ModeTables& mt,
                                             bool row_side) {
  if (!(code & 0x8000)) return 0.0;
  const int NP = mt.NP;
  int k = code & 15, p = (code >> 4) & 63;
  int part = row_side ? (code >> 10) & 1 : (code >> 11) & 1;
  double2 v;
  if (code & 0x10000) {
    v = make_double2(0.0, 0.0);
    const int n = row_side ? mt.fcnt[p] : 1;
    for (int j = 0; j < n; ++j) {
      double2 u = X[k * NP + mt.fpair[p][j]];
      if (mt.fconj[p][j]) u.y = -u.y;
      v.x += u.x;
      v.y += u.y;
    }
  } else {
    v = X[k * NP + p];
  }
  double x = part ? v.y : v.x;
  if (row_side) {
    int ci = (code >> 12) & 7;
    x *= ci == 1 ? 1.0 : ci == 2 ? -1.0 : ci == 3 ? 2.0 : ci == 4 ? -2.0 : 0.0;
  }
  return x;
}

__device__ __forceinline__ double2 to_d2(double2 v) { return v; }
__device__ __forceinline__ double2 to_d2(float2 v) { return make_double2(v.x, v.y); }

// per-waveform (h|h) sums H_ikcc' = sum_b w_kb h_icb conj(h_ic'b) (relative
// binning: sum_b W_kcc'b h_icb conj(h_ic'b), whh [n_det][NP][n_b]) for the
// event's bank subset, from the same operand values the contraction uses,
// written as the row-side (h|h) operand (n_sub rows of KH, op_index layout)
// with a power-of-two
// row scale in the split precisions
template <int PREC>
__global__ void k_hh_precompute(int64_t n_sub, const int64_t* __restrict__ sub_idx, int64_t sub0,
                                const void* __restrict__ A0, const void* __restrict__ A1,
                                const double* __restrict__ row_scale, int n_bp, int n_b,
                                int n_det, const double* __restrict__ w,
                                const double2* __restrict__ whh, ModeTables mt,
                                const int* __restrict__ terms, int KH, void* __restrict__ H0,
                                void* __restrict__ H1, double* __restrict__ hscale,
                                const void* __restrict__ R0, const void* __restrict__ R1) {
  // the row [n_c][n_bp] then w [n_det][n_b], when they fit.  A split value
  // hi + lo spans at most 23 significant bits, so float holds it exactly.
  typedef typename std::conditional<PREC == kFP64, double2, float2>::type RB;
  extern __shared__ __align__(16) unsigned char hh_smem[];
  RB* rowbuf = (RB*)hh_smem;
  // the block's waves split the bins: wave q sums bins [q n_b / nq, (q + 1) n_b / nq)
  // of every (detector, channel pair), and the nq partial sums are added in order;
  // their area follows the staged row in the dynamic LDS
  __shared__ double vals[256];
  __shared__ double red[256];
  const int nq = (int)blockDim.x / 64, wq = (int)threadIdx.x / 64, u = (int)threadIdx.x % 64;
  const int64_t ie = blockIdx.x;
  if (ie >= n_sub) return;
  const int64_t i = sub_idx ? sub_idx[ie] : sub0 + ie;
  const int64_t K2 = (int64_t)mt.n_c * n_bp * 2;
  // channel rows and detector rows one entry longer than the data, so that
  // the lanes reading one bin of different channels or detectors fall on
  // different LDS banks
  const int rs = n_bp + 1, ws = n_b + 1;
  const size_t stage_bytes = (size_t)mt.n_c * rs * sizeof(RB) + (size_t)n_det * ws * sizeof(double);
  const bool staged = stage_bytes <= 65536;
  double* wl = (double*)(rowbuf + mt.n_c * rs);
  const int nhp = n_det * mt.NP;   // (detector, channel pair) sums
  double2* Hq_base = (double2*)(hh_smem + (staged ? (stage_bytes + 15) / 16 * 16 : 0));
  auto Hq = [&](int q, int t) -> double2& { return Hq_base[q * nhp + t]; };
  if (staged) {
    // the row in pieces of 8 consecutive positions (16 bytes per operand
    // array in the split layouts): 8 bins of the real or the imaginary part;
    // from the row-major copy of the split bank when there is one (whole
    // lines), else from the fragment layout (16 bytes of each line)
    const bool rm = PREC != kFP64 && R0 != nullptr;
    const void* S0 = rm ? R0 : A0;
    const void* S1 = rm ? R1 : A1;
    for (int pc = threadIdx.x; pc < (int)(K2 / 8); pc += blockDim.x) {
      const int64_t o = rm ? i * K2 + (int64_t)pc * 8 : op_index<PREC>(i, (int64_t)pc * 8, K2);
      double v[8];
      if (PREC == kFP64) {
#pragma unroll
        for (int j = 0; j < 8; ++j) v[j] = ((const double*)A0)[o + j];
      } else {
        const uint4 hq = *(const uint4*)((const uint16_t*)S0 + o);
        const uint4 lq = *(const uint4*)((const uint16_t*)S1 + o);
        const unsigned hw[4] = {hq.x, hq.y, hq.z, hq.w}, lw[4] = {lq.x, lq.y, lq.z, lq.w};
#pragma unroll
        for (int j = 0; j < 8; ++j) {
          const uint16_t hb = (uint16_t)(hw[j >> 1] >> (16 * (j & 1)));
          const uint16_t lb = (uint16_t)(lw[j >> 1] >> (16 * (j & 1)));
          if (PREC == kFP16X2)
            v[j] = (double)__builtin_bit_cast(_Float16, hb) + (double)__builtin_bit_cast(_Float16, lb);
          else
            v[j] = (double)(float)__builtin_bit_cast(__bf16, hb) + (double)(float)__builtin_bit_cast(__bf16, lb);
        }
      }
      const int kk = pc * 8, chunk = kk >> 5, within = kk & 31;
      const int c = chunk / (n_bp / kChunk), b0 = (chunk % (n_bp / kChunk)) * kChunk + (within & 15);
      typedef typename std::conditional<PREC == kFP64, double, float>::type RV;
      RV* dst = (RV*)(rowbuf + c * rs + b0) + (within >= 16 ? 1 : 0);
#pragma unroll
      for (int j = 0; j < 8; ++j) dst[2 * j] = (RV)v[j];
    }
    if (!whh)
      for (int t = threadIdx.x; t < n_det * n_b; t += blockDim.x) wl[(t / n_b) * ws + t % n_b] = w[t];
    __syncthreads();
  }
  double sc = row_scale ? row_scale[i] : 1.0;
  sc = sc * sc;
  const int b_lo = wq * n_b / nq, b_hi = (wq + 1) * n_b / nq;
  for (int t = u; t < n_det * mt.NP; t += 64) {
    int k = t / mt.NP, p = t % mt.NP;
    int c = mt.pc[p], c2 = mt.pc2[p];
    double2 acc = make_double2(0.0, 0.0);
    if (whh) {
      // relative binning: a complex weight per channel pair and bin
      const double2* Wp = whh + ((int64_t)k * mt.NP + p) * n_b;
      for (int b = b_lo; b < b_hi; ++b) {
        const double2 a = staged ? to_d2(rowbuf[c * rs + b]) : bank_value<PREC>(A0, A1, i, K2, c, b, n_bp);
        const double2 a2 = staged ? to_d2(rowbuf[c2 * rs + b]) : bank_value<PREC>(A0, A1, i, K2, c2, b, n_bp);
        const double2 u = cmul(Wp[b], cmul(cconj(a), a2));
        acc.x += u.x;
        acc.y += u.y;
      }
    } else if (staged) {
      // two partial sums, so that consecutive bins do not wait on each other
      double2 acc2 = make_double2(0.0, 0.0);
      int b = b_lo;
      for (; b + 1 < b_hi; b += 2) {
        const double2 v0 = cmul(cconj(to_d2(rowbuf[c * rs + b])), to_d2(rowbuf[c2 * rs + b]));
        const double2 v1 = cmul(cconj(to_d2(rowbuf[c * rs + b + 1])), to_d2(rowbuf[c2 * rs + b + 1]));
        const double w0 = wl[k * ws + b], w1 = wl[k * ws + b + 1];
        acc.x += w0 * v0.x;
        acc.y += w0 * v0.y;
        acc2.x += w1 * v1.x;
        acc2.y += w1 * v1.y;
      }
      if (b < b_hi) {
        const double2 v0 = cmul(cconj(to_d2(rowbuf[c * rs + b])), to_d2(rowbuf[c2 * rs + b]));
        acc.x += wl[k * ws + b] * v0.x;
        acc.y += wl[k * ws + b] * v0.y;
      }
      acc.x += acc2.x;
      acc.y += acc2.y;
    } else {
      for (int b = b_lo; b < b_hi; ++b) {
        double2 a = bank_value<PREC>(A0, A1, i, K2, c, b, n_bp);
        double2 a2 = bank_value<PREC>(A0, A1, i, K2, c2, b, n_bp);
        double2 v = cmul(cconj(a), a2);      // h_c conj(h_c') = conj(A_c) A_c'
        double ww = w[k * n_b + b];
        acc.x += ww * v.x;
        acc.y += ww * v.y;
      }
    }
    Hq(wq, t) = acc;
  }
  __syncthreads();
  for (int t = threadIdx.x; t < nhp; t += blockDim.x) {
    double2 h = Hq(0, t);
    for (int q = 1; q < nq; ++q) {
      h.x += Hq(q, t).x;
      h.y += Hq(q, t).y;
    }
    Hq(0, t) = make_double2(h.x * sc, h.y * sc);
  }
  __syncthreads();
  const double2* Hs = Hq_base;
  double mx = 0.0;
  for (int j = threadIdx.x; j < KH; j += blockDim.x) {
    double v = term_value(terms[j], Hs, mt, true);
    vals[j] = v;
    mx = fmax(mx, fabs(v));
  }
  red[threadIdx.x] = mx;
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + s]);
    __syncthreads();
  }
  int ex = 0;
  if (PREC != kFP64 && red[0] > 0.0 && isfinite(red[0])) ex = ilogb(red[0]) - 13;
  if (threadIdx.x == 0 && hscale) hscale[ie] = ldexp(1.0, ex);
  for (int j = threadIdx.x; j < KH; j += blockDim.x)
    store_split<PREC>(H0, H1, op_index<PREC>(ie, j, KH), ldexp(vals[j], -ex));
}

// column-side (h|h) operand (n_ext_p rows of KH, op_index layout) from
// Q_ekcc' = R_ekc conj(R_ekc')
template <int PREC>
__global__ void k_build_Bhh(int64_t n_ext, int64_t n_ext_p, int n_det, const double2* __restrict__ Q,
                            ModeTables mt, const int* __restrict__ terms, int KH,
                            void* __restrict__ B0, void* __restrict__ B1,
                            double* __restrict__ bscale) {
  __shared__ double vals[256];
  __shared__ double red[64];
  const int64_t e = blockIdx.x;
  if (e >= n_ext_p) return;
  double mx = 0.0;
  for (int j = threadIdx.x; j < KH; j += blockDim.x) {
    double v = e < n_ext ? term_value(terms[j], Q + e * n_det * mt.NP, mt, false) : 0.0;
    vals[j] = v;
    mx = fmax(mx, fabs(v));
  }
  red[threadIdx.x] = mx;
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + s]);
    __syncthreads();
  }
  int ex = 0;
  if (PREC != kFP64 && red[0] > 0.0 && isfinite(red[0])) ex = ilogb(red[0]) - 13;
  if (threadIdx.x == 0 && bscale && e < n_ext) bscale[e] = ldexp(1.0, ex);
  for (int j = threadIdx.x; j < KH; j += blockDim.x)
    store_split<PREC>(B0, B1, op_index<PREC>(e, j, KH), ldexp(vals[j], -ex));
}

// fixed-order reduction of tile partials: block b combines tiles
// [b * per, (b + 1) * per) into out[b][kNPart]; a second launch with one
// block combines the block results
__global__ void k_finalize(const double* __restrict__ partials, int64_t n_tiles, int64_t per,
                           double* __restrict__ out) {
  __shared__ double sh[256 * kNPart];
  const int64_t t0 = blockIdx.x * per, t1 = min(n_tiles, t0 + per);
  Lse p, d;
  p.init(); d.init();
  double mlm = 0.0, mb = -INFINITY, mxp = -INFINITY, nm = 0, nb = 0, np_ = 0;
  for (int64_t t = t0 + threadIdx.x; t < t1; t += blockDim.x) {
    const double* r = partials + t * kNPart;
    p.merge(r[0], r[1], r[2], r[11]);
    d.merge(r[3], r[4], 0.0);
    mlm = fmax(mlm, r[5]);
    nm += r[6]; nb += r[7]; mb = fmax(mb, r[8]); mxp = fmax(mxp, r[9]); np_ += r[10];
  }
  double* m = sh + threadIdx.x * kNPart;
  m[0] = p.m; m[1] = p.s; m[2] = p.s2; m[3] = d.m; m[4] = d.s; m[5] = mlm;
  m[6] = nm; m[7] = nb; m[8] = mb; m[9] = mxp; m[10] = np_; m[11] = p.s3;
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) {
      double* x = sh + threadIdx.x * kNPart;
      double* y = sh + (threadIdx.x + s) * kNPart;
      Lse pp, dd;
      pp.m = x[0]; pp.s = x[1]; pp.s2 = x[2]; pp.s3 = x[11];
      dd.m = x[3]; dd.s = x[4]; dd.s2 = 0.0; dd.s3 = 0.0;
      pp.merge(y[0], y[1], y[2], y[11]);
      dd.merge(y[3], y[4], 0.0);
      x[0] = pp.m; x[1] = pp.s; x[2] = pp.s2; x[3] = dd.m; x[4] = dd.s; x[11] = pp.s3;
      x[5] = fmax(x[5], y[5]); x[6] += y[6]; x[7] += y[7]; x[8] = fmax(x[8], y[8]);
      x[9] = fmax(x[9], y[9]); x[10] += y[10];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0)
    for (int q = 0; q < kNPart; ++q) out[blockIdx.x * kNPart + q] = sh[q];
}

// one bitonic merge step over candidate records [n][4] (ln p, i, e, o):
// order = ln p descending, then i, then e ascending
__device__ __forceinline__ bool cand_before(const double* x, const double* y) {
  if (x[0] != y[0]) return x[0] > y[0];
  if (x[1] != y[1]) return x[1] < y[1];
  return x[2] < y[2];
}
__global__ void k_bitonic_step(double* __restrict__ c, int64_t n, int64_t j, int64_t k) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  int64_t l = i ^ j;
  if (l <= i) return;
  double* x = c + 4 * i;
  double* y = c + 4 * l;
  bool up = (i & k) == 0;
  bool swap = up ? cand_before(y, x) : cand_before(x, y);
  if (swap) {
    for (int q = 0; q < 4; ++q) {
      double t = x[q];
      x[q] = y[q];
      y[q] = t;
    }
  }
}
// Top-k by sorted chunks and pairwise merges: k_topk_chunks sorts each chunk
// of C records (a power of two, <= kTopkChunk) in LDS; k_topk_merge then
// replaces chunk a = 2 p s by the best C records of chunks a and a + s (both
// sorted), which are max(A[t], B[C - 1 - t]) over t -- the upper half of the
// half-cleaner applied to the bitonic sequence A, reversed B -- and sorts
// that bitonic half with the merge network.  After log2(n / C) merge rounds
// (s = 1, 2, 4, ...) the first chunk holds the best C records of all n in
// order: the first C records of a full sort.
constexpr int kTopkChunk = 4096;

__device__ __forceinline__ bool cand_before_lds(const double* x, const double* y) {
  if (x[0] != y[0]) return x[0] > y[0];
  if (x[1] != y[1]) return x[1] < y[1];
  return x[2] < y[2];
}

// compare-exchange steps (j) of the bitonic network of stage k over C records
// in LDS, by all threads of the block (k = C: one sorted run)
__device__ __forceinline__ void lds_bitonic_steps(double* r, int C, int k, int j_first) {
  for (int j = j_first; j > 0; j >>= 1) {
    for (int t = threadIdx.x; t < C / 2; t += blockDim.x) {
      const int i = ((t & ~(j - 1)) << 1) | (t & (j - 1));
      const int l = i | j;
      double* x = r + 4 * i;
      double* y = r + 4 * l;
      const bool up = (i & k) == 0;
      if (up ? cand_before_lds(y, x) : cand_before_lds(x, y)) {
        const double4 tx = make_double4(x[0], x[1], x[2], x[3]);
        x[0] = y[0]; x[1] = y[1]; x[2] = y[2]; x[3] = y[3];
        y[0] = tx.x; y[1] = tx.y; y[2] = tx.z; y[3] = tx.w;
      }
    }
    __syncthreads();
  }
}

__global__ __launch_bounds__(256) void k_topk_chunks(double* __restrict__ c, int C) {
  extern __shared__ __align__(16) double rec[];
  double* g = c + (int64_t)blockIdx.x * C * 4;
  for (int t = threadIdx.x; t < C * 4; t += blockDim.x) rec[t] = g[t];
  __syncthreads();
  for (int k = 2; k <= C; k <<= 1) lds_bitonic_steps(rec, C, k, k >> 1);
  for (int t = threadIdx.x; t < C * 4; t += blockDim.x) g[t] = rec[t];
}

__global__ __launch_bounds__(256) void k_topk_merge(double* __restrict__ c, int C, int64_t s) {
  extern __shared__ __align__(16) double rec[];
  const int64_t a = 2 * (int64_t)blockIdx.x * s;
  double* A = c + a * C * 4;
  const double* B = c + (a + s) * C * 4;
  for (int t = threadIdx.x; t < C; t += blockDim.x) {
    const double* x = A + 4 * t;
    const double* y = B + 4 * (C - 1 - t);
    const double* w = cand_before_lds(y, x) ? y : x;
    rec[4 * t] = w[0];
    rec[4 * t + 1] = w[1];
    rec[4 * t + 2] = w[2];
    rec[4 * t + 3] = w[3];
  }
  __syncthreads();
  lds_bitonic_steps(rec, C, C, C >> 1);
  for (int t = threadIdx.x; t < C * 4; t += blockDim.x) A[t] = rec[t];
}

__global__ void k_zero(double* __restrict__ x, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    x[i] = 0.0;
}

// Marginals for eqs. int_ess and ext_ess: the sum of p_ie over one row i
// (rows = 1) or one column e (rows = 0) of the pair matrix, from the tiles'
// row and column sums scaled from each tile's maximum to the global maximum
// M = final_out[9].  Block (x, c) sums the tiles c * q_per .. (c + 1) *
// q_per - 1 along the row or column: part[c][x].
__global__ void k_marginal_part(const double* __restrict__ partials, const double* __restrict__ rowcol,
                                const double* __restrict__ final_out, int64_t n_tiles_m,
                                int64_t n_tiles_n, int tm_rows, int tn_cols, int64_t n_idx, int rows,
                                int64_t q_per, double* __restrict__ part) {
  const double M = final_out[9];
  const int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (x >= n_idx) return;
  const int64_t outer = rows ? x / tm_rows : x / tn_cols;
  const int slot = rows ? (int)(x % tm_rows) : 64 + (int)(x % tn_cols);
  const int64_t n_other = rows ? n_tiles_n : n_tiles_m;
  const int64_t q0 = (int64_t)blockIdx.y * q_per, q1 = min(n_other, q0 + q_per);
  double P = 0.0;
  if (M > -INFINITY)
    for (int64_t q = q0; q < q1; ++q) {
      const int64_t t = rows ? outer * n_tiles_n + q : q * n_tiles_n + outer;
      const double mx = partials[t * kNPart + 9];
      if (mx > -INFINITY) P += rowcol[t * 128 + slot] * exp(mx - M);
    }
  part[blockIdx.y * n_idx + x] = P;
}

// each index's marginal (the sum of its parts, in part order), squared;
// block sums of the squares (tree order) to blk
__global__ void k_marginal_sq(const double* __restrict__ part, int64_t n_parts, int64_t n_idx,
                              double* __restrict__ blk) {
  __shared__ double sh[256];
  const int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  double v = 0.0;
  if (x < n_idx) {
    double P = 0.0;
    for (int64_t c = 0; c < n_parts; ++c) P += part[c * n_idx + x];
    v = P * P;
  }
  sh[threadIdx.x] = v;
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) blk[blockIdx.x] = sh[0];
}

// out[0] = sum of blk[0 .. n) in a fixed order
__global__ void k_sum_blocks(const double* __restrict__ blk, int64_t n, double* __restrict__ out) {
  __shared__ double sh[256];
  double v = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += blockDim.x) v += blk[i];
  sh[threadIdx.x] = v;
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = sh[0];
}

// ---------------------------------------------------------------------------
// posterior sampling: the tiles' masses, their running sum, the systematic
// draws placed in tiles
// ---------------------------------------------------------------------------
// mass of tile t relative to e^M (M = final_out[9]): e^(p.m - M) p.s
__global__ void k_tile_mass(const double* __restrict__ partials, const double* __restrict__ final_out,
                            int64_t n_tiles, double* __restrict__ mass) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n_tiles) return;
  const double M = final_out[9], m = partials[t * kNPart], s = partials[t * kNPart + 1];
  mass[t] = (m > -INFINITY && M > -INFINITY) ? exp(m - M) * s : 0.0;
}

// Inclusive running sum in place over blocks of 1024 (scan_inclusive on the
// host drives it): each block's own running sum, in LDS, its total to blk;
// the blocks' totals are summed the same way, one level up, and each block
// then adds the running total before it.
__global__ void k_scan_block(double* __restrict__ x, int64_t n, double* __restrict__ blk) {
  __shared__ double sh[1024];
  const int64_t i = (int64_t)blockIdx.x * 1024 + threadIdx.x;
  sh[threadIdx.x] = i < n ? x[i] : 0.0;
  __syncthreads();
  for (int s = 1; s < 1024; s <<= 1) {
    const double v = threadIdx.x >= (unsigned)s ? sh[threadIdx.x - s] : 0.0;
    __syncthreads();
    sh[threadIdx.x] += v;
    __syncthreads();
  }
  if (i < n) x[i] = sh[threadIdx.x];
  if (threadIdx.x == 1023) blk[blockIdx.x] = sh[1023];
}
// blk: the blocks' inclusive running totals
__global__ void k_scan_add(double* __restrict__ x, int64_t n, const double* __restrict__ blk) {
  const int64_t i = (int64_t)blockIdx.x * 1024 + threadIdx.x;
  if (blockIdx.x > 0 && i < n) x[i] += blk[blockIdx.x - 1];
}

// systematic draws t_s = (s + u0) W / n_s (W = the total mass, cum[n - 1])
// placed in tiles: the first tile whose running sum exceeds t_s, and the
// residual t_s minus the mass before that tile
__global__ void k_place_draws(const double* __restrict__ cum, int64_t n_tiles, int64_t n_s, double u0,
                              int* __restrict__ tile, double* __restrict__ res) {
  const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= n_s) return;
  const double W = cum[n_tiles - 1];
  const double ts = ((double)s + u0) * W / (double)n_s;
  int64_t lo = 0, hi = n_tiles - 1;     // first index with cum > ts (the last if none)
  while (lo < hi) {
    const int64_t mid = (lo + hi) / 2;
    if (cum[mid] > ts) hi = mid;
    else lo = mid + 1;
  }
  tile[s] = (int)lo;
  res[s] = ts - (lo > 0 ? cum[lo - 1] : 0.0);
}

// the distinct tiles of the (ascending) draws and, per distinct tile, its
// first draw; n_out[0] = number of distinct tiles (one thread, in order)
__global__ void k_group_draws(const int* __restrict__ tile, int64_t n_s, int* __restrict__ list,
                              int64_t* __restrict__ first, int64_t* __restrict__ n_out) {
  if (threadIdx.x != 0) return;
  int64_t u = 0;
  for (int64_t s = 0; s < n_s; ++s)
    if (s == 0 || tile[s] != tile[s - 1]) {
      list[u] = tile[s];
      first[u] = s;
      ++u;
    }
  first[u] = n_s;
  n_out[0] = u;
}

__global__ void k_fill_cand(double* __restrict__ c, int64_t from, int64_t to) {
  int64_t i = from + (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= to) return;
  c[4 * i] = -INFINITY;
  c[4 * i + 1] = 1e300;
  c[4 * i + 2] = 1e300;
  c[4 * i + 3] = 0;
}

}  // namespace dotpe
