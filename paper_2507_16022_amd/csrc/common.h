// Shared definitions of the device code of the likelihood-matrix hot path
// (gfx950, wave64, MFMA): types, constants, mode tables, small helpers and
// the split-operand layout.  Included by every translation unit with kernels.
//
// Notation: i bank row (subset index ie), e extrinsic sample, k detector,
// c mode channel (channels reordered so that equal m are contiguous; g the
// group of channels sharing m), b frequency bin, o phase grid index.
//
// (d|h) for a triple (eq. dh_ieo) is rearranged as
//     dh_ieo = Re sum_g exp(i m_g phi_o) X_ieg,
//     X_ieg  = sum_{c in g} sum_b conj(h_icb) B_cb(e),
//     B_cb(e) = sum_k w_kb d_kb conj(R_ekc) exp(+2 pi i f_b t_ek),
// i.e. a complex GEMM over K = (c, b) with the detector sum folded into the
// extrinsic operand; (h|h) (eq. hh_ieo) as
//     hh_ieo = S0 + 2 Re sum_{delta > 0} S_delta exp(-i delta phi_o),
//     S_delta = sum_k sum_{c,c': m_c - m_c' = delta} H_ikcc' Q_ekcc',
//     H_ikcc' = sum_b w_kb h_icb conj(h_ic'b),  Q_ekcc' = R_ekc conj(R_ekc').
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

#include "dist_rule.h"

namespace dotpe {

typedef _Float16 half8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x4 __attribute__((ext_vector_type(4)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

constexpr int kMaxC = 8;        // channels
constexpr int kMaxG = 4;        // distinct m
constexpr int kMaxDet = 8;
constexpr int kMaxPhi = 128;
constexpr int kMaxNP = kMaxC * (kMaxC + 1) / 2;
constexpr int kMaxND = 4;       // delta = 0..3
constexpr int kMaxM = 4;
constexpr int kChunk = 16;      // bins per K chunk (32 real K)
constexpr int kNPart = 12;      // doubles per tile partial
constexpr int kSurvCap = 16;    // survivors of a 64 x 64 tile the bound pass lists one by one
constexpr int kMaxNF = 16;      // (m, p) layout: (h|h) sums folded over m

enum Prec { kFP64 = 0, kFP16X2 = 1, kBF16X2 = 2 };

struct ModeTables {
  int n_c, G, ND, NP;
  int l[kMaxC], m[kMaxC];          // per channel (group order)
  int orig[kMaxC];                 // input channel index of each
  int gm[kMaxG];                   // m of each group
  int gk0[kMaxG + 1];              // chunk index where each group starts
  // channel pairs (c, c') with c <= c', sorted by |m_c - m_c'|: pairs with
  // |delta| = d occupy [pstart[d], pstart[d + 1])
  int pc[kMaxNP], pc2[kMaxNP], pdel[kMaxNP];   // m_c - m_c' (signed)
  int pstart[kMaxND + 1];
  float pf[kMaxNP];                // delta = 0: 1 (c = c') or 2 (c != c')
  float ps[kMaxNP];                // sign of the imaginary part (conjugate when delta < 0)
  int pdiag[kMaxC];                // pair index of (c, c)
  // channel layout: 0 (l, m) modes; 1 (m, p): pol[c] is the channel's
  // polarisation and its response the real antenna pattern F_{k,pol[c]}
  int layout;
  int pol[kMaxC];
  // (m, p) layout: (h|h) sums folded over m.  Entry f sums the channel
  // pairs fpair[f][0 .. fcnt[f]) -- conjugated where fconj -- which share
  // (delta, p, p') and so the column factor F_kp F_kp'
  int nf;
  int fcnt[kMaxNF], fpair[kMaxNF][kMaxG], fconj[kMaxNF][kMaxG];
};

// distance-rule parameters (the tail formula's Gauss-Hermite nodes), kept in
// device memory next to the table (the table's geometry is a compile-time
// constant)
struct DistParams {
  double ghx[kGH], ghw[kGH];
};
struct DistArgs {
  const double* tab;
  const DistParams* prm;
};

// ---------------------------------------------------------------------------
// small helpers
// ---------------------------------------------------------------------------
__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ double2 cconj(double2 a) { return make_double2(a.x, -a.y); }

// compile-time loop: f(std::integral_constant<int, i>) for i = 0 .. N-1
template <int I, int N, typename F>
__device__ __forceinline__ void static_for_impl(F&& f) {
  if constexpr (I < N) {
    f(std::integral_constant<int, I>{});
    static_for_impl<I + 1, N>(f);
  }
}
template <int N, typename F>
__device__ __forceinline__ void static_for(F&& f) {
  static_for_impl<0, N>(f);
}


// online log-sum-exp accumulator of terms e^x: s = sum e^(x - m), s2 = sum
// e^(2 (x - m)), and s3 = sum r e^(2 (x - m)) with a weight r per term (for
// a pair, r = sum_o p_ieo^2 / p_ie^2: the triples' squares of eq.
// posterior_element)
struct Lse {
  double m, s, s2, s3;
  __device__ void init() { m = -INFINITY; s = 0.0; s2 = 0.0; s3 = 0.0; }
  __device__ void add(double x, double r = 1.0) {
    if (x == -INFINITY) return;
    if (x > m) {
      double f = exp(m - x);
      s = s * f + 1.0;
      s2 = s2 * f * f + 1.0;
      s3 = s3 * f * f + r;
      m = x;
    } else {
      double f = exp(x - m);
      s += f;
      s2 += f * f;
      s3 += f * f * r;
    }
  }
  __device__ void merge(double mb, double sb, double s2b, double s3b = 0.0) {
    if (mb == -INFINITY) return;
    if (m == -INFINITY) { m = mb; s = sb; s2 = s2b; s3 = s3b; return; }
    double mm = fmax(m, mb);
    double fa = exp(m - mm), fb = exp(mb - mm);
    s = s * fa + sb * fb;
    s2 = s2 * fa * fa + s2b * fb * fb;
    s3 = s3 * fa * fa + s3b * fb * fb;
    m = mm;
  }
};

// online log-sum-exp over the phases of one pair: FP64 running maximum and
// sum, each term's exponential taken in FP32 (a relative error ~1e-7, far
// inside the tolerance on ln Lbar; a term more than ~87 below the running
// maximum, under 1e-37 of the sum, counts as zero); one exponential and no
// branch per term
struct LsePh {
  double m, s, s2;     // s2: sum of the squared terms (the triples' squares)
  __device__ void init() { m = -INFINITY; s = 0.0; s2 = 0.0; }
  __device__ void add(double x) {
    const double d = x - m;                       // +inf while empty
    const double t = (double)__expf(-fabsf((float)d));
    const bool up = d > 0.0;
    const double ns = up ? fma(s, t, 1.0) : s + t;
    const double ns2 = up ? fma(s2, t * t, 1.0) : fma(t, t, s2);
    const bool skip = !(x > -INFINITY);
    s = skip ? s : ns;
    s2 = skip ? s2 : ns2;
    m = (up && !skip) ? x : m;
  }
  __device__ void merge(double mb, double sb, double s2b) {
    if (mb == -INFINITY) return;
    if (m == -INFINITY) { m = mb; s = sb; s2 = s2b; return; }
    const double mm = fmax(m, mb);
    const double fa = exp(m - mm), fb = exp(mb - mm);
    s = s * fa + sb * fb;
    s2 = s2 * fa * fa + s2b * fb * fb;
    m = mm;
  }
  // sum_o p_o^2 / (sum_o p_o)^2 of the terms added
  __device__ double sq_ratio() const { return s > 0.0 ? s2 / (s * s) : 1.0; }
};

__device__ __forceinline__ uint64_t order_bits(double x) {
  uint64_t u = __double_as_longlong(x);
  return (u & 0x8000000000000000ull) ? ~u : (u | 0x8000000000000000ull);
}
__device__ __forceinline__ double order_value(uint64_t u) {
  u = (u & 0x8000000000000000ull) ? (u & 0x7fffffffffffffffull) : ~u;
  return __longlong_as_double(u);
}
// value of lane src (wave-uniform) of a double
__device__ __forceinline__ double read_lane(double v, int src) {
  const unsigned long long b = (unsigned long long)__double_as_longlong(v);
  const unsigned lo = __builtin_amdgcn_readlane((unsigned)b, src);
  const unsigned hi = __builtin_amdgcn_readlane((unsigned)(b >> 32), src);
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// made of 2 slices (positions 16 s .. 16 s + 15) of 1 KB, and in a slice the
// 8 positions of piece h (8 h .. 8 h + 7) of row r sit at elements
// 8 (32 h + r) .. +7.  One 32-row slice is then exactly the 1 KB that a
// 32x32x16 matrix-core operand read takes (lane 32 h + r holds row r, piece
// h), so loads and LDS reads are contiguous.
template <int PREC>
__host__ __device__ __forceinline__ int64_t op_index(int64_t i, int64_t k, int64_t K) {
  if (PREC == kFP64) return i * K + k;
  return ((i >> 5) * (K >> 5) + (k >> 5)) * 1024 + ((k >> 4) & 1) * 512 + ((k >> 3) & 1) * 256 +
         (i & 31) * 8 + (k & 7);
}


constexpr int kMaxNR = 2 * kMaxND - 1;   // (h|h) phase-coefficient outputs

// SplitMix64 (Steele, Lea and Flood, 2014): output n (from 0) of the
// generator seeded with `seed`, as a uniform double in [0, 1) from its top
// 53 bits.  A counter-based source of the draws that the posterior sampling
// needs: any draw is computed from (seed, n) alone.
__host__ __device__ inline double sm64_uniform(uint64_t seed, uint64_t n) {
  uint64_t z = seed + (n + 1) * 0x9e3779b97f4a7c15ull;
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
  z ^= z >> 31;
  return (double)(z >> 11) * 0x1.0p-53;
}

__device__ inline double swsh_m2(int l, int m, double cos_t) {
  // spin-weight -2 harmonic at azimuth 0: sqrt((2l+1)/4pi) d^l_{m,2}(theta)
  const double fact[13] = {1, 1, 2, 6, 24, 120, 720, 5040, 40320, 362880, 3628800, 39916800,
                           479001600};
  double ct = fmin(1.0, fmax(-1.0, cos_t));
  double cb = sqrt(0.5 * (1.0 + ct)), sb = sqrt(0.5 * (1.0 - ct));   // cos, sin of theta/2
  const int s = 2;
  double sum = 0.0;
  for (int k = 0; k <= 2 * l; ++k) {
    int a = l + s - k, b = k, c = l - k - m, d = k - s + m;
    if (a < 0 || c < 0 || d < 0) continue;
    double coef = sqrt(fact[l + s] * fact[l - s] * fact[l + m] * fact[l - m]) /
                  (fact[a] * fact[b] * fact[c] * fact[d]);
    if ((k - s + m) & 1) coef = -coef;
    int pc = 2 * l - 2 * k + s - m, ps = 2 * k - s + m;
    double v = coef;
    for (int q = 0; q < pc; ++q) v *= cb;
    for (int q = 0; q < ps; ++q) v *= sb;
    sum += v;
  }
  return sqrt((2.0 * l + 1.0) / (4.0 * M_PI)) * sum;
}

}  // namespace dotpe
