// Kernels of the intrinsic pre-selection (Sec. IV D; App. B eqs. dh_itop,
// x_ML, single_det_ML); the arithmetic is laid out in preselect.h.
//
// The per-channel inner products Y_ikc(t) are one complex matrix product
// per channel on the matrix cores: the bank rows (the split operand the
// evidence pass reads) against one data operand whose rows are the
// (detector, time) grid points, the same for every channel.  A workgroup
// takes 32 bank rows and one detector, a wave 32 grid times; its epilogue
// forms the polarisation projections for every phase, applies the 2x2
// pseudo-inverse and keeps the maximum, and the workgroup writes the
// per-row maximum for its detector.
#include <hip/hip_runtime.h>

#include <type_traits>

#include "fused.h"
#include "preselect.h"

namespace dotpe {
namespace {

template <int PREC>
__device__ __forceinline__ void store_split(void* p0, void* p1, int64_t o, double x) {
  if constexpr (PREC == kFP16X2) {
    const _Float16 hi = (_Float16)x;
    ((_Float16*)p0)[o] = hi;
    ((_Float16*)p1)[o] = (_Float16)(x - (double)hi);
  } else {
    const __bf16 hi = (__bf16)(float)x;
    ((__bf16*)p0)[o] = hi;
    ((__bf16*)p1)[o] = (__bf16)(float)(x - (double)(float)hi);
  }
}

template <int PREC>
__device__ __forceinline__ double load_split(const void* p0, const void* p1, int64_t o) {
  if constexpr (PREC == kFP16X2) return (double)((const _Float16*)p0)[o] + (double)((const _Float16*)p1)[o];
  else return (double)(float)((const __bf16*)p0)[o] + (double)(float)((const __bf16*)p1)[o];
}

// w_kb d_kb exp(2 pi i f_b t) with f_b t reduced to a fraction of a cycle in FP64
__device__ __forceinline__ double2 pre_data(const PreArgs& a, int k, int b, double t) {
  const double x = a.f[b] * t;
  double sn, cn;
  sincospi(2.0 * (x - floor(x)), &sn, &cn);
  const double2 d = a.d[(int64_t)k * a.n_b + b];
  const double w = a.w[(int64_t)k * a.n_b + b];
  return make_double2(w * (d.x * cn - d.y * sn), w * (d.x * sn + d.y * cn));
}

// Data operand: row r = k n_t + j holds w_kb d_kb exp(2 pi i f_b t_kj) (bins
// past n_b zero), scaled by 2^-e_r so that its largest component lies in
// [2^13, 2^14) (col_scale[r] = 2^e_r), stored [Re | -Im] by slice in hi + lo.
template <int PREC>
__global__ __launch_bounds__(256) void k_pre_build_B(PreArgs a) {
  const int64_t r = blockIdx.x;
  const int k = (int)(r / a.n_t), j = (int)(r % a.n_t);
  const double t = a.t0[k] + j * a.dt;
  __shared__ double red[256];
  double mx = 0.0;
  for (int b = threadIdx.x; b < a.n_b; b += blockDim.x) {
    const double2 v = pre_data(a, k, b, t);
    mx = fmax(mx, fmax(fabs(v.x), fabs(v.y)));
  }
  red[threadIdx.x] = mx;
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + s]);
    __syncthreads();
  }
  mx = red[0];
  const int ex = (mx > 0.0 && isfinite(mx)) ? ilogb(mx) - 13 : 0;
  if (threadIdx.x == 0) a.col_scale[r] = ldexp(1.0, ex);
  for (int b = threadIdx.x; b < a.n_bp; b += blockDim.x) {
    double br = 0.0, bi = 0.0;
    if (b < a.n_b) {
      const double2 v = pre_data(a, k, b, t);
      br = ldexp(v.x, -ex);
      bi = ldexp(v.y, -ex);
    }
    const int64_t base = (int64_t)(b / kChunk) * 32 + (b % kChunk);
    store_split<PREC>((void*)a.B0, (void*)a.B1, op_index<PREC>(r, base, a.K2p), br);
    store_split<PREC>((void*)a.B0, (void*)a.B1, op_index<PREC>(r, base + 16, a.K2p), -bi);
  }
}

// G_ikcc' = sum_b w_kb h_icb conj(h_ic'b) (c <= c') from the split bank
// values (h = conj(A) 2^e_i), in FP64: a wave per row, its lanes over the
// bins, one wave sum per output.  The row is read from the row-major copy
// of the split parts: in the fragment layout a single row's 16-byte pieces
// lie 512 bytes apart, one per cache line.
template <int PREC, int NC>
__global__ __launch_bounds__(256) void k_pre_gram(PreArgs a) {
  constexpr int NP = NC * (NC + 1) / 2;
  const int lane = threadIdx.x & 63;
  const int64_t q = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (q >= a.n_chunk) return;
  const int64_t i = a.row0 + a.chunk0 + q;
  const double s2 = a.row_scale[i] * a.row_scale[i];
  auto add = [](double x, double y) { return x + y; };
  for (int k = 0; k < a.n_det; ++k) {
    double gr[NP], gi[NP];
#pragma unroll
    for (int p = 0; p < NP; ++p) { gr[p] = 0.0; gi[p] = 0.0; }
    for (int b = lane; b < a.n_b; b += 64) {
      double hr[NC], hi[NC];
#pragma unroll
      for (int c = 0; c < NC; ++c) {
        const int64_t base = ((int64_t)c * (a.n_bp / kChunk) + b / kChunk) * 32 + (b % kChunk);
        hr[c] = load_split<PREC>(a.R0, a.R1, i * a.K2 + base);
        hi[c] = -load_split<PREC>(a.R0, a.R1, i * a.K2 + base + 16);
      }
      const double w = a.w[(int64_t)k * a.n_b + b];
      int p = 0;
#pragma unroll
      for (int c = 0; c < NC; ++c)
#pragma unroll
        for (int c2 = c; c2 < NC; ++c2, ++p) {
          gr[p] += w * (hr[c] * hr[c2] + hi[c] * hi[c2]);
          gi[p] += w * (hi[c] * hr[c2] - hr[c] * hi[c2]);
        }
    }
    double2* out = a.gram + (q * a.n_det + k) * NP;
#pragma unroll
    for (int p = 0; p < NP; ++p) {
      const double r = wave_reduce(gr[p], 0.0, add), m = wave_reduce(gi[p], 0.0, add);
      if (lane == 63) out[p] = make_double2(s2 * r, s2 * m);
    }
  }
}

__device__ __forceinline__ uint4 ld16(const void* base, int64_t elem) {
  return *(const uint4*)((const uint16_t*)base + elem);
}
__device__ __forceinline__ uint4 neg16(const uint4& x) {
  return make_uint4(x.x ^ 0x80008000u, x.y ^ 0x80008000u, x.z ^ 0x80008000u, x.w ^ 0x80008000u);
}

template <int PREC, int NC>
__global__ __launch_bounds__(64 * kPreMaxT / 32) void k_preselect(PreArgs a) {
  typedef typename Pol<PREC>::Acc Acc;
  extern __shared__ __align__(16) double pls[];
  const int n_phi = a.n_phi;
  double* cs = pls;                          // [kMaxM][n_phi][2] cos, sin of m phi_o
  double* kp = cs + kMaxM * n_phi * 2;       // [32][NC] K_c+
  double* kx = kp + 32 * NC;                 // [32][NC] K_cx / i
  float* qf = (float*)(kx + 32 * NC);        // [32][n_phi][4] H^+ / 2 as (cos, sin, a1, a2)
  double* red = (double*)(qf + 32 * n_phi * 4);   // [NW][32]
  float* csf = (float*)(red + 32 * (kPreMaxT / 32));   // [kMaxM][n_phi][2] in FP32
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, nt = blockDim.x;
  const int k = blockIdx.y;
  const int64_t rb0 = a.chunk0 + (int64_t)blockIdx.x * 32;   // first row of the block
  const int rows_in = (int)min((int64_t)32, a.chunk0 + a.n_chunk - rb0);

  for (int t = tid; t < kMaxM * n_phi; t += nt) {
    const int mm = t / n_phi + 1, o = t % n_phi;
    double sn, cn;
    sincospi(2.0 * (double)((mm * o) % n_phi) / n_phi, &sn, &cn);
    cs[2 * t] = cn;
    cs[2 * t + 1] = sn;
    csf[2 * t] = (float)cn;
    csf[2 * t + 1] = (float)sn;
  }
  for (int t = tid; t < 32 * NC; t += nt) {
    const int rr = t / NC, c = t % NC;
    const double ci = rr < rows_in ? a.cos_iota[rb0 + rr] : 0.0;
    const double yn = swsh_m2(a.l[c], -a.m[c], ci), yp = swsh_m2(a.l[c], a.m[c], ci);
    const double sg = (a.l[c] & 1) ? -1.0 : 1.0;
    kp[t] = 0.5 * (yn + sg * yp);
    kx[t] = 0.5 * (yn - sg * yp);
  }
  __syncthreads();
  // H_pp'(row, o) from the Gram matrix, then its pseudo-inverse / 2 (an
  // eigen-direction with eigenvalue below 1e-10 of the largest dropped) in
  // eigen-form: b^T H^+ b / 2 = a1 (c b+ + s bx)^2 + a2 (-s b+ + c bx)^2, a
  // sum of non-negative terms, so the epilogue may evaluate it in FP32
  constexpr int NP = NC * (NC + 1) / 2;
  for (int t = tid; t < 32 * n_phi; t += nt) {
    const int rr = t / n_phi, o = t % n_phi;
    double h00 = 0.0, h01 = 0.0, h11 = 0.0;
    if (rr < rows_in) {
      const double2* g = a.gram + ((rb0 + rr - a.chunk0) * a.n_det + k) * NP;
      int p = 0;
#pragma unroll
      for (int c = 0; c < NC; ++c)
#pragma unroll
        for (int c2 = c; c2 < NC; ++c2, ++p) {
          const double2 G = g[p];
          const int dm = a.m[c] - a.m[c2];
          double cd = 1.0, sd = 0.0;
          if (dm != 0) {
            const int ad = dm < 0 ? -dm : dm;
            cd = cs[((ad - 1) * n_phi + o) * 2];
            sd = dm < 0 ? -cs[((ad - 1) * n_phi + o) * 2 + 1] : cs[((ad - 1) * n_phi + o) * 2 + 1];
          }
          // exp(-i dm phi) G_cc'; the (c', c) term is its conjugate
          const double re = cd * G.x + sd * G.y, im = cd * G.y - sd * G.x;
          const double pa = kp[rr * NC + c], pb = kp[rr * NC + c2];
          const double xa = kx[rr * NC + c], xb = kx[rr * NC + c2];
          const double f = (c == c2) ? 1.0 : 2.0;
          h00 += f * pa * pb * re;
          h11 += f * xa * xb * re;
          h01 += (c == c2) ? pa * xb * im : (pa * xb - pb * xa) * im;
        }
    }
    double ec = 1.0, es = 0.0, a1 = 0.0, a2 = 0.0;
    const double df = 0.5 * (h00 - h11);
    const double lp = 0.5 * (h00 + h11) + sqrt(df * df + h01 * h01);
    if (lp > 0.0) {
      // eigenvector of the larger eigenvalue, then the smaller one as det / lp
      const double vx = df >= 0.0 ? lp - h11 : h01, vy = df >= 0.0 ? h01 : lp - h00;
      const double nn = sqrt(vx * vx + vy * vy);
      if (nn > 0.0) {
        ec = vx / nn;
        es = vy / nn;
      }
      a1 = 0.5 / lp;
      const double lm = (h00 * h11 - h01 * h01) / lp;
      a2 = lm > 1e-10 * lp ? 0.5 / lm : 0.0;
    }
    qf[4 * t] = (float)ec;
    qf[4 * t + 1] = (float)es;
    qf[4 * t + 2] = (float)a1;
    qf[4 * t + 3] = (float)a2;
  }

  // ---- Y_ikc for this wave's 32 grid times, every channel ----
  const int h = lane >> 5;
  const int64_t ia = a.row0 + min(rb0 + (lane & 31), a.n_rows - 1);   // (rows past the end re-read the last)
  const int64_t abase = ((ia >> 5) * (a.K2 >> 5)) * 1024 + h * 256 + (ia & 31) * 8;
  const int64_t rbB = (int64_t)k * a.n_t + 32 * wave + (lane & 31);
  const int64_t bbase = ((rbB >> 5) * (a.K2p >> 5)) * 1024 + h * 256 + (rbB & 31) * 8;
  Acc acc[NC][2];
#pragma unroll
  for (int c = 0; c < NC; ++c) {
    acc[c][0] = Acc{};
    acc[c][1] = Acc{};
  }
  // fragments of one bin chunk: B hi/lo of both slices, A hi/lo of both
  // slices for every channel; the next chunk's are loaded while this one's
  // products run (one wave per SIMD: the loads' latency is hidden by the
  // wave's own work)
  struct Frag {
    uint4 b[4];          // bh0, bh1, bl0, bl1
    uint4 a[NC][4];      // ah0, ah1, al0, al1
  };
  const int nj = a.n_bp / kChunk;    // a multiple of 4 (bins padded to 64)
  auto load = [&](Frag& f, int j) {
    const int64_t bo = bbase + (int64_t)j * 1024;
    f.b[0] = ld16(a.B0, bo);
    f.b[1] = ld16(a.B0, bo + 512);
    f.b[2] = ld16(a.B1, bo);
    f.b[3] = ld16(a.B1, bo + 512);
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      const int64_t ao = abase + (int64_t)(c * nj + j) * 1024;
      f.a[c][0] = ld16(a.A0, ao);
      f.a[c][1] = ld16(a.A0, ao + 512);
      f.a[c][2] = ld16(a.A1, ao);
      f.a[c][3] = ld16(a.A1, ao + 512);
    }
  };
  auto compute = [&](const Frag& f) {
    const uint4 &bh0 = f.b[0], &bh1 = f.b[1], &bl0 = f.b[2], &bl1 = f.b[3];
    const uint4 nbh1 = neg16(bh1), nbl1 = neg16(bl1);
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      const uint4 &ah0 = f.a[c][0], &ah1 = f.a[c][1], &al0 = f.a[c][2], &al1 = f.a[c][3];
      // A = [Re conj h | Im conj h], B_re = [Br | -Bi], B_im = [Bi | Br]:
      // 3 split products per real product
      Acc& re = acc[c][0];
      Acc& im = acc[c][1];
      mma<PREC>(re, al0, bh0);  mma<PREC>(im, al0, nbh1);
      mma<PREC>(re, ah0, bl0);  mma<PREC>(im, ah0, nbl1);
      mma<PREC>(re, ah0, bh0);  mma<PREC>(im, ah0, nbh1);
      mma<PREC>(re, al1, bh1);  mma<PREC>(im, al1, bh0);
      mma<PREC>(re, ah1, bl1);  mma<PREC>(im, ah1, bl0);
      mma<PREC>(re, ah1, bh1);  mma<PREC>(im, ah1, bh0);
    }
  };
  Frag f0, f1;
  load(f0, 0);
  for (int j = 0; j < nj; j += 2) {
    load(f1, j + 1);
    compute(f0);
    if (j + 2 < nj) load(f0, j + 2);
    compute(f1);
  }
  __syncthreads();   // (the forms in qf are complete)

  // ---- epilogue: polarisation projections, 2x2 form, maximum ----
  // (in FP32: the accumulators are FP32 and the form is a sum of squares)
  const double csc = a.col_scale[rbB];
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    const int rr = 8 * (r >> 2) + 4 * h + (r & 3);
    const float sc = (float)((rr < rows_in ? a.row_scale[a.row0 + rb0 + rr] : 0.0) * csc);
    float wpr[NC], wpi[NC], wxr[NC], wxi[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      const float yr = sc * acc[c][0][r], yi = sc * acc[c][1][r];
      const float pk = (float)kp[rr * NC + c], xk = (float)kx[rr * NC + c];
      wpr[c] = pk * yr;     // conj(K_c+) Y
      wpi[c] = pk * yi;
      wxr[c] = xk * yi;     // conj(K_cx) Y = -i (K_cx / i) Y
      wxi[c] = -xk * yr;
    }
    float bestf = 0.f;
    for (int o = 0; o < n_phi; ++o) {
      float bp = 0.f, bx = 0.f;
#pragma unroll
      for (int c = 0; c < NC; ++c) {
        const float cn = csf[((a.m[c] - 1) * n_phi + o) * 2], sn = csf[((a.m[c] - 1) * n_phi + o) * 2 + 1];
        bp += cn * wpr[c] - sn * wpi[c];
        bx += cn * wxr[c] - sn * wxi[c];
      }
      const float4 q = *(const float4*)(qf + 4 * (rr * n_phi + o));
      const float u = q.x * bp + q.y * bx, v = q.x * bx - q.y * bp;
      bestf = fmaxf(bestf, q.z * u * u + q.w * v * v);
    }
    if (a.ml_t && rr < rows_in)
      a.ml_t[((rb0 + rr) * a.n_det + k) * a.n_t + 32 * wave + (lane & 31)] = (double)bestf;
    double best = (double)bestf;
#pragma unroll
    for (int off = 16; off > 0; off >>= 1) best = fmax(best, __shfl_xor(best, off, 32));
    if ((lane & 31) == 0) red[wave * 32 + rr] = best;
  }
  __syncthreads();
  if (tid < rows_in) {
    double m = red[tid];
    for (int w = 1; w < nt / 64; ++w) m = fmax(m, red[w * 32 + tid]);
    a.ml_det[(rb0 + tid) * a.n_det + k] = m;
  }
}

// incoherent sums over detectors (fixed order), and their maximum
__global__ __launch_bounds__(256) void k_pre_final(PreArgs a) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  double v = -INFINITY;
  if (i < a.n_rows) {
    v = 0.0;
    for (int k = 0; k < a.n_det; ++k) v += a.ml_det[i * a.n_det + k];
    a.lnl[i] = v;
  }
  const double m = wave_max(v);
  if ((threadIdx.x & 63) == 0 && m > -INFINITY)
    atomicMax((unsigned long long*)&a.state[0], (unsigned long long)order_bits(m));
}

// selection: rows with lnl >= max - delta, in row order (blocks of 1024
// rows, 4 consecutive per thread)
__device__ __forceinline__ unsigned pre_flags(const PreArgs& a, int64_t r0) {
  const double thr = order_value(a.state[0]) - a.delta;
  unsigned f = 0;
  for (int q = 0; q < 4; ++q) {
    const int64_t i = r0 + q;
    if (i < a.n_rows && a.lnl[i] >= thr) f |= 1u << q;
  }
  return f;
}

__global__ __launch_bounds__(256) void k_pre_count(PreArgs a) {
  __shared__ int sc[256];
  const unsigned f = pre_flags(a, (int64_t)blockIdx.x * 1024 + 4 * threadIdx.x);
  sc[threadIdx.x] = __popc(f);
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s) sc[threadIdx.x] += sc[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) a.counts[blockIdx.x] = sc[0];
}

__global__ __launch_bounds__(256) void k_pre_scan(PreArgs a, int64_t nb) {
  if (threadIdx.x != 0) return;
  int64_t run = 0;
  for (int64_t b = 0; b < nb; ++b) {
    a.offsets[b] = run;
    run += a.counts[b];
  }
  a.state[1] = (uint64_t)run;
}

__global__ __launch_bounds__(256) void k_pre_write(PreArgs a) {
  __shared__ int sc[256];
  const int64_t r0 = (int64_t)blockIdx.x * 1024 + 4 * threadIdx.x;
  const unsigned f = pre_flags(a, r0);
  sc[threadIdx.x] = __popc(f);
  __syncthreads();
  // inclusive scan (Hillis-Steele)
  for (int s = 1; s < 256; s <<= 1) {
    const int v = threadIdx.x >= s ? sc[threadIdx.x - s] : 0;
    __syncthreads();
    sc[threadIdx.x] += v;
    __syncthreads();
  }
  int64_t pos = a.offsets[blockIdx.x] + sc[threadIdx.x] - __popc(f);
  for (int q = 0; q < 4; ++q)
    if (f & (1u << q)) a.selected[pos++] = a.row0 + r0 + q;
}

template <int PREC, int NC>
hipError_t launch_pre_main(const PreArgs& a, hipStream_t s) {
  const size_t lds = sizeof(double) * ((size_t)kMaxM * a.n_phi * 2 + 64 * NC + 32 * (size_t)a.n_phi * 2 +
                                       (kPreMaxT / 32) * 32 + (size_t)kMaxM * a.n_phi);
  static bool attr_done = false;
  if (!attr_done) {
    const size_t most = sizeof(double) * ((size_t)kMaxM * kMaxPhi * 2 + 64 * NC + 32 * (size_t)kMaxPhi * 2 +
                                          (kPreMaxT / 32) * 32 + (size_t)kMaxM * kMaxPhi);
    if (hipFuncSetAttribute((const void*)k_preselect<PREC, NC>, hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)most) != hipSuccess)
      (void)hipGetLastError();
    attr_done = true;
  }
  hipLaunchKernelGGL((k_pre_gram<PREC, NC>), dim3((unsigned)((a.n_chunk + 3) / 4)), dim3(256), 0, s, a);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  dim3 grid((unsigned)((a.n_chunk + 31) / 32), (unsigned)a.n_det);
  hipLaunchKernelGGL((k_preselect<PREC, NC>), grid, dim3(64 * (a.n_t / 32)), lds, s, a);
  return hipGetLastError();
}

template <int PREC>
hipError_t launch_pre_nc(const PreArgs& a, hipStream_t s) {
  switch (a.n_c) {
    case 1: return launch_pre_main<PREC, 1>(a, s);
    case 2: return launch_pre_main<PREC, 2>(a, s);
    case 3: return launch_pre_main<PREC, 3>(a, s);
    case 4: return launch_pre_main<PREC, 4>(a, s);
    case 5: return launch_pre_main<PREC, 5>(a, s);
    case 6: return launch_pre_main<PREC, 6>(a, s);
    case 7: return launch_pre_main<PREC, 7>(a, s);
    case 8: return launch_pre_main<PREC, 8>(a, s);
  }
  return hipErrorInvalidValue;
}

template <int PREC>
hipError_t run_all(PreArgs a, hipStream_t s) {
  hipLaunchKernelGGL(k_pre_build_B<PREC>, dim3((unsigned)(a.n_det * a.n_t)), dim3(256), 0, s, a);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  for (int64_t c0 = 0; c0 < a.n_rows; c0 += kPreChunk) {
    a.chunk0 = c0;
    a.n_chunk = std::min<int64_t>(kPreChunk, a.n_rows - c0);
    if ((e = launch_pre_nc<PREC>(a, s)) != hipSuccess) return e;
  }
  hipLaunchKernelGGL(k_pre_final, dim3((unsigned)((a.n_rows + 255) / 256)), dim3(256), 0, s, a);
  const int64_t nb = (a.n_rows + 1023) / 1024;
  hipLaunchKernelGGL(k_pre_count, dim3((unsigned)nb), dim3(256), 0, s, a);
  hipLaunchKernelGGL(k_pre_scan, dim3(1), dim3(256), 0, s, a, nb);
  hipLaunchKernelGGL(k_pre_write, dim3((unsigned)nb), dim3(256), 0, s, a);
  return hipGetLastError();
}

}  // namespace

hipError_t preselect_launch(int prec, PreArgs a, hipStream_t s) {
  if (prec == kFP16X2) return run_all<kFP16X2>(a, s);
  if (prec == kBF16X2) return run_all<kBF16X2>(a, s);
  return hipErrorInvalidValue;
}

}  // namespace dotpe
