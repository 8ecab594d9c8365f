// Host runtime of the C ABI in include/dotpe.h: context, bank-summary
// layout, event staging, launches of the fused likelihood kernel, evidence
// finalisation and top-k selection.  All compute runs in the kernels of
// kernels.h; host code validates, allocates, copies and launches.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/dotpe.h"
#include "../../include/dotpe_test.h"
#include "launch.h"
#include "prep.h"
#include "preselect.h"
#include "serving.h"

using namespace dotpe;

namespace {

thread_local std::string g_err;

int fail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

#define HIP_OK(expr)                                                                    \
  do {                                                                                  \
    hipError_t e_ = (expr);                                                             \
    if (e_ != hipSuccess)                                                               \
      return fail(DOTPE_E_DEVICE, "%s: %s (%s:%d)", #expr, hipGetErrorString(e_), __FILE__, \
                  __LINE__);                                                            \
  } while (0)

int64_t round_up(int64_t x, int64_t m) { return (x + m - 1) / m * m; }

// 128 x 128 tiles an event needs before the bound pass replaces the fused
// kernel's fast epilogue (fewer would leave the device partly idle)
constexpr int64_t kBoundMinTiles = 2048;
constexpr int64_t kMargPer = 256;     // tiles summed by one thread of the marginal pass

}  // namespace

// Device scratch of dotpe_evidence_static: every buffer of one event packed
// into one file-scope array, so that the call allocates no device memory.
// Each GPU holds its own copy until the process ends.  In host code the
// array's name is only a handle: the device address of each GPU's copy is
// taken once per device (scratch_setup, from dotpe_create) and used instead.
constexpr uint64_t kScratchBytes = uint64_t(128) << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {

constexpr int kScratchDevices = 64;
struct ScratchSlot {
  std::mutex mu;            // held for a whole dotpe_evidence_static call
  void* ptr = nullptr;      // device address of this GPU's copy of `scratch`
};
ScratchSlot g_scratch[kScratchDevices];
std::mutex g_scratch_setup;

// with `device` current: record the device address of its copy of scratch
int scratch_setup(int device) {
  if (device >= kScratchDevices) return DOTPE_OK;   // static entry point unavailable there
  std::lock_guard<std::mutex> lk(g_scratch_setup);
  if (g_scratch[device].ptr) return DOTPE_OK;
  void* p = nullptr;
  hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess || !p) {
    (void)hipGetLastError();
    return fail(DOTPE_E_DEVICE, "hipGetSymbolAddress(scratch) on device %d: %s", device,
                hipGetErrorString(e));
  }
  g_scratch[device].ptr = p;
  return DOTPE_OK;
}

}  // namespace

struct dotpe_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  uint64_t budget = 0;
  std::atomic<uint64_t> bytes{0};   // serving slot threads also release through it
  // one device block that dotpe_set_event packs an event's buffers into and
  // keeps after dotpe_free_event for the next event that fits, so that a
  // stream of events does not allocate and free device memory each time
  std::mutex ev_mu;
  char* ev_block = nullptr;
  uint64_t ev_block_len = 0;
  bool ev_block_busy = false;
  uint64_t own_bytes = 0;    // the context's own tables (not charged to the budget)
  double* dist_tab = nullptr;
  DistParams* dist_prm = nullptr;   // device copy of the Gauss-Hermite nodes
  double ghx[kGH], ghw[kGH];
};

struct dotpe_bank {
  int64_t n_wf = 0;
  int n_c = 0, n_b = 0, n_bp = 0;
  int64_t K2 = 0;
  int prec = 0;
  ModeTables mt{};
  double* f = nullptr;          // device [n_b]
  std::vector<double> f_host;
  void* A0 = nullptr;
  void* A1 = nullptr;
  void* R0 = nullptr;           // split precisions: the same hi and lo parts row by row
  void* R1 = nullptr;           //   ([n_wf][K2]), read by the survivor pass one row at a time
  double* row_scale = nullptr;
  float2* nrm = nullptr;        // split precisions: per row, norms of the hi and left-out parts
  double* ln_w = nullptr;
  uint64_t bytes = 0;
};

struct dotpe_event {
  const dotpe_bank* bank = nullptr;
  hipStream_t stream = nullptr;
  int n_det = 0, n_phi = 0;
  int64_t n_ext = 0, n_ext_p = 0, n_sub = 0, sub0 = 0;
  int64_t* sub_idx = nullptr;
  double d0 = 1.0, d_max = 1.0, n_norm = 0.0, cut_delta = 0.0, topk_window = 40.0;
  double cut_target = 1e-4;
  int top_k = 0;
  int flags = 0;
  double dd = 0.0;
  // device arrays
  void* B[4] = {nullptr, nullptr, nullptr, nullptr};
  double* col_scale = nullptr;
  double* ln_w_ext = nullptr;
  int* hh_terms = nullptr;     // (h|h) term codes [KH]
  int KH = 0;                  // (h|h) operand row length
  void* Ah[2] = {nullptr, nullptr};   // row-side (h|h) operand [n_sub][KH]
  double* ah_scale = nullptr;
  void* Bh[2] = {nullptr, nullptr};   // column-side (h|h) operand [n_ext_p][KH]
  double* bh_scale = nullptr;
  float2* b_nrm = nullptr;     // split precisions: per row of B, Ah, Bh, norms of the hi
  float2* ah_nrm = nullptr;    //   and left-out parts (the bound pass's margin)
  float2* bh_nrm = nullptr;
  bool norms_done = false;     // b_nrm, ah_nrm, bh_nrm computed (before the first bound pass)
  bool ctx_block = false;      // its buffers sit in the context's event block
  double2* Q = nullptr;
  double* R2 = nullptr;
  double2* R = nullptr;
  double* T = nullptr;
  double* phase_cs = nullptr;
  // evidence scratch
  double* partials = nullptr;
  uint64_t* state = nullptr;
  double* cand = nullptr;
  int64_t cand_cap = 0;
  double* final_out = nullptr;
  double* final_blk = nullptr;
  int* rerun = nullptr;          // tiles the fast or bound pass leaves to the coefficient route
  uint16_t* surv = nullptr;      // bound pass: listed survivors [n_tiles][kSurvCap]
  int* surv_list = nullptr;      // bound pass: (tile, count) of tiles with listed survivors
  void* coef = nullptr;          // coefficient route: raw accumulators of coef_tiles tiles
  int64_t coef_tiles = 0;
  double* rowcol = nullptr;      // per tile: row and column sums of the evaluated p [n_tiles][128]
  bool evaluated = false;        // the last evidence pass's partials, state and results are
  double last_cut = 0.0;         //   on the device: its cut_delta and N_eff over triples
  double last_n_eff = 0.0;
  double* marg_part = nullptr;   // marginals in parts along rows / columns of tiles
  double* marg_blk = nullptr;    // block sums of the squared marginals
  hipEvent_t ev_t[4] = {nullptr, nullptr, nullptr, nullptr};
  std::vector<void*> allocs;
  uint64_t bytes = 0;
};

namespace {

int dev_alloc(dotpe_ctx* ctx, void** p, size_t n, std::vector<void*>* owner, uint64_t* acct) {
  if (n == 0) n = 16;
  if (ctx->budget && ctx->bytes - ctx->own_bytes + n > ctx->budget)
    return fail(DOTPE_E_ADMISSION, "device budget exceeded: %llu + %zu > %llu bytes",
                (unsigned long long)(ctx->bytes - ctx->own_bytes), n,
                (unsigned long long)ctx->budget);
  hipError_t e = hipMalloc(p, n);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return fail(DOTPE_E_OOM, "hipMalloc(%zu): %s", n, hipGetErrorString(e));
  }
  ctx->bytes += n;
  if (acct) *acct += n;
  if (owner) owner->push_back(*p);
  return DOTPE_OK;
}

// probabilists' Gauss-Hermite nodes/weights (weight exp(-x^2/2)/sqrt(2 pi)):
// roots of He_n bracketed on a grid and polished by Newton steps
void gauss_hermite(int n, double* x, double* w) {
  auto he = [n](double t, double* dn) {
    double p0 = 1.0, p1 = t;
    for (int k = 1; k < n; ++k) {
      double p2 = t * p1 - k * p0;
      p0 = p1;
      p1 = p2;
    }
    *dn = n * p0;   // He_n' = n He_{n-1}
    return p1;
  };
  int found = 0;
  double prev_t = -12.0, d;
  double prev_v = he(prev_t, &d);
  for (int s = 1; s <= 240000 && found < n; ++s) {
    double t = -12.0 + s * 1e-4;
    double v = he(t, &d);
    if ((v < 0) != (prev_v < 0)) {
      double r = 0.5 * (t + prev_t);
      for (int it = 0; it < 50; ++it) {
        double val = he(r, &d);
        double step = val / d;
        r -= step;
        if (std::fabs(step) < 1e-16) break;
      }
      x[found++] = r;
    }
    prev_t = t;
    prev_v = v;
  }
  double sum = 0.0;
  for (int k = 0; k < n; ++k) {
    double hn1 = 0.0;
    he(x[k], &hn1);
    hn1 /= n;      // He_{n-1}(x_k)
    w[k] = 1.0 / (n * hn1 * hn1);   // up to the n! normalisation, fixed below
    sum += w[k];
  }
  for (int k = 0; k < n; ++k) w[k] /= sum;
}

int build_modes(const dotpe_bank_desc* d, ModeTables* mt, int n_bp) {
  const int nc = d->n_modes;
  const bool mp = d->layout == DOTPE_LAYOUT_MP;
  std::vector<int> ms;
  for (int c = 0; c < nc; ++c) {
    int m = d->mode_m[c];
    if (mp) {
      const int p = d->mode_p[c];
      if (m < 1 || m > kMaxM || (p != 0 && p != 1))
        return fail(DOTPE_E_INVALID_ARG, "channel (m=%d, p=%d) unsupported (need 1<=m<=4, p 0 or 1)",
                    m, p);
      for (int c2 = 0; c2 < c; ++c2)
        if (d->mode_m[c2] == m && d->mode_p[c2] == p)
          return fail(DOTPE_E_INVALID_ARG, "channel (m=%d, p=%d) given twice", m, p);
    } else {
      int l = d->mode_l[c];
      if (m < 1 || m > kMaxM || l < 2 || l > 8 || m > l)
        return fail(DOTPE_E_INVALID_ARG, "mode (%d,%d) unsupported (need 2<=l<=8, 1<=m<=min(l,4))",
                    l, m);
    }
    if (std::find(ms.begin(), ms.end(), m) == ms.end()) ms.push_back(m);
  }
  std::sort(ms.begin(), ms.end());
  if ((int)ms.size() > kMaxG) return fail(DOTPE_E_INVALID_ARG, "too many distinct m");
  std::memset(mt, 0, sizeof(*mt));
  mt->n_c = nc;
  mt->G = (int)ms.size();
  mt->layout = mp ? 1 : 0;
  int c2 = 0;
  const int cpc = n_bp / kChunk;
  for (int g = 0; g < mt->G; ++g) {
    mt->gm[g] = ms[g];
    mt->gk0[g] = c2 * cpc;
    // (m, p) layout: + before x within a group
    for (int pp = 0; pp < (mp ? 2 : 1); ++pp)
      for (int c = 0; c < nc; ++c)
        if (d->mode_m[c] == ms[g] && (!mp || d->mode_p[c] == pp)) {
          mt->l[c2] = mp ? 0 : d->mode_l[c];
          mt->m[c2] = d->mode_m[c];
          mt->pol[c2] = mp ? pp : 0;
          mt->orig[c2] = c;
          ++c2;
        }
  }
  mt->gk0[mt->G] = c2 * cpc;
  mt->ND = ms.back() - ms.front() + 1;
  // channel pairs c <= c', sorted by |m_c - m_c'|
  int p = 0;
  for (int d = 0; d <= mt->ND - 1 && d < kMaxND; ++d) {
    mt->pstart[d] = p;
    for (int a = 0; a < nc; ++a)
      for (int b = a; b < nc; ++b) {
        int del = mt->m[a] - mt->m[b];
        if (std::abs(del) != d) continue;
        mt->pc[p] = a;
        mt->pc2[p] = b;
        mt->pdel[p] = del;
        mt->pf[p] = (d == 0) ? (a == b ? 1.0f : 2.0f) : 1.0f;
        mt->ps[p] = del < 0 ? -1.0f : 1.0f;
        if (a == b) mt->pdiag[a] = p;
        ++p;
      }
  }
  for (int d = std::min(mt->ND, kMaxND); d <= kMaxND; ++d) mt->pstart[d] = p;
  mt->NP = p;
  if (mp) {
    // folded (h|h) sums: per delta and polarisation pair, the channel pairs
    // (c, c') with m_c - m_c' = delta, pol p_c, p_c' -- conjugated where the
    // stored pair runs the other way.  delta = 0: (+,+), (x,x), (+,x).
    auto chan = [&](int m, int pol) {
      for (int c = 0; c < nc; ++c)
        if (mt->m[c] == m && mt->pol[c] == pol) return c;
      return -1;
    };
    auto pair_of = [&](int a, int b) {
      for (int q = 0; q < mt->NP; ++q)
        if (mt->pc[q] == std::min(a, b) && mt->pc2[q] == std::max(a, b)) return q;
      return -1;
    };
    for (int dd = 0; dd < std::min(mt->ND, kMaxND); ++dd) {
      const int np_ = dd == 0 ? 3 : 4;
      for (int q = 0; q < np_; ++q) {
        const int pa = dd == 0 ? (q == 1 ? 1 : 0) : q >> 1, pb = dd == 0 ? (q == 0 ? 0 : 1) : q & 1;
        const int f = mt->nf;
        if (f >= kMaxNF) return fail(DOTPE_E_INVALID_ARG, "too many folded (h|h) sums");
        for (int g = 0; g < mt->G; ++g) {
          const int a = chan(mt->gm[g], pa), b = chan(mt->gm[g] - dd, pb);
          if (a < 0 || b < 0) continue;
          mt->fpair[f][mt->fcnt[f]] = pair_of(a, b);
          mt->fconj[f][mt->fcnt[f]] = a > b ? 1 : 0;
          ++mt->fcnt[f];
        }
        if (mt->fcnt[f] > 0) ++mt->nf;
      }
    }
  }
  return DOTPE_OK;
}

// (h|h) term codes: output r < NR owns K block r (32 slots); see kernels.h
int build_hh_terms(const ModeTables& mt, int n_det, std::vector<int>* terms, int* KH) {
  const int nhb = kMaxNR + 1;
  *KH = nhb * 32;
  terms->assign(*KH, 0);
  const int NR = 2 * mt.ND - 1;
  auto code = [](int k, int p, int apart, int bpart, int coef_idx) {
    return (k & 15) | ((p & 63) << 4) | (apart << 10) | (bpart << 11) | (coef_idx << 12) | 0x8000;
  };
  for (int r = 0; r < NR; ++r) {
    std::vector<int> t;
    for (int k = 0; k < n_det && mt.layout == 1; ++k) {
      // (m, p) layout: one term per folded sum (its column factor F_kp F_kp'
      // is real): S0 from the delta = 0 sums (x2 for (+, x)), Re / Im S_d
      // from the real / imaginary parts of the delta = d sums
      for (int f = 0; f < mt.nf; ++f) {
        const int q0 = mt.fpair[f][0];
        const int del = std::abs(mt.pdel[q0]);
        if (r == 0) {
          if (del == 0)
            t.push_back(code(k, f, 0, 0, mt.pc[q0] == mt.pc2[q0] ? 1 : 3) | 0x10000);
        } else if (del == (r + 1) / 2) {
          t.push_back(code(k, f, (r % 2) == 0 ? 1 : 0, 0, 1) | 0x10000);
        }
      }
    }
    for (int k = 0; k < n_det && mt.layout == 0; ++k) {
      if (r == 0) {
        for (int p = mt.pstart[0]; p < mt.pstart[1]; ++p) {
          if (mt.pc[p] == mt.pc2[p]) {
            t.push_back(code(k, p, 0, 0, 1));
          } else {
            t.push_back(code(k, p, 0, 0, 3));     // 2 Re(H Q) = 2 (Hr Qr - Hi Qi)
            t.push_back(code(k, p, 1, 1, 4));
          }
        }
      } else {
        const int d = (r + 1) / 2;
        const bool im = (r % 2) == 0;
        for (int p = mt.pstart[d]; p < mt.pstart[d + 1]; ++p) {
          if (!im) {                               // Re(H Q) = Hr Qr - Hi Qi
            t.push_back(code(k, p, 0, 0, 1));
            t.push_back(code(k, p, 1, 1, 2));
          } else {                                 // ps Im(H Q) = ps (Hr Qi + Hi Qr)
            int ci = mt.ps[p] > 0 ? 1 : 2;
            t.push_back(code(k, p, 0, 1, ci));
            t.push_back(code(k, p, 1, 0, ci));
          }
        }
      }
    }
    if (t.size() > 32)
      return fail(DOTPE_E_INVALID_ARG,
                  "(h|h) output %d needs %zu terms (> 32): too many modes x detectors", r,
                  t.size());
    for (size_t j = 0; j < t.size(); ++j) (*terms)[r * 32 + j] = t[j];
  }
  return DOTPE_OK;
}

template <int PREC>
void launch_bank_convert(const double* h, dotpe_bank* bk, int* err, hipStream_t s) {
  hipLaunchKernelGGL(k_bank_convert<PREC>, dim3((unsigned)bk->n_wf), dim3(256), 0, s, h, bk->n_wf,
                     bk->n_c, bk->n_b, bk->n_bp, bk->mt, bk->A0, bk->A1, bk->row_scale, err, bk->R0,
                     bk->R1);
}

template <int PREC>
void launch_convert_B(dotpe_event* ev, const double2* Btmp, int* err) {
  const dotpe_bank* bk = ev->bank;
  hipLaunchKernelGGL(k_convert_B<PREC>, dim3((unsigned)ev->n_ext_p), dim3(256), 0, ev->stream,
                     ev->n_ext, ev->n_ext_p, bk->n_c, bk->n_bp, Btmp, ev->B[0], ev->B[1], ev->B[2],
                     ev->B[3], ev->col_scale, err);
}

template <int PREC>
void launch_hh(dotpe_event* ev, const double* w, const double2* whh) {
  const dotpe_bank* bk = ev->bank;
  // the row's amplitudes and the noise weights in LDS when they fit (the
  // kernel applies the same test)
  const size_t rb = PREC == kFP64 ? sizeof(double2) : sizeof(float2);   // staged row value
  size_t sh = (size_t)bk->n_c * (bk->n_bp + 1) * rb + (size_t)ev->n_det * (bk->n_b + 1) * sizeof(double);
  sh = sh > 65536 ? 0 : (sh + 15) / 16 * 16;
  // four waves per row, each summing a quarter of the bins (their partial
  // sums after the staged row)
  sh += (size_t)4 * ev->n_det * bk->mt.NP * sizeof(double2);
  // more than 64 KB of dynamic LDS needs the attribute (FP64 banks with many
  // channels and detectors); set once, up to what a CU holds
  static std::once_flag attr_once;
  std::call_once(attr_once, [] {
    if (hipFuncSetAttribute((const void*)k_hh_precompute<PREC>,
                            hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024 - 8192) !=
        hipSuccess)
      (void)hipGetLastError();
  });
  hipLaunchKernelGGL(k_hh_precompute<PREC>, dim3((unsigned)ev->n_sub), dim3(256), sh, ev->stream,
                     ev->n_sub, ev->sub_idx, ev->sub0, bk->A0, bk->A1, bk->row_scale, bk->n_bp,
                     bk->n_b, ev->n_det, w, whh, bk->mt, ev->hh_terms, ev->KH, ev->Ah[0],
                     ev->Ah[1], ev->ah_scale, bk->R0, bk->R1);
  hipLaunchKernelGGL(k_build_Bhh<PREC>, dim3((unsigned)ev->n_ext_p), dim3(64), 0, ev->stream,
                     ev->n_ext, ev->n_ext_p, ev->n_det, ev->Q, bk->mt, ev->hh_terms, ev->KH,
                     ev->Bh[0], ev->Bh[1], ev->bh_scale);
}

// chunk ranges of the m groups of a (d|h) operand row
NormRanges group_ranges(const ModeTables& mt) {
  NormRanges r{};
  r.n = mt.G;
  for (int g = 0; g <= mt.G; ++g) r.c0[g] = mt.gk0[g];
  return r;
}

// (h|h) phase-coefficient outputs the kernels use: S0, and Re, Im of
// S_1..3 with more than one m group
int hh_outputs(int G) { return G == 1 ? 1 : kMaxNR; }

// chunk ranges of those outputs in a (h|h) operand row (one chunk each)
NormRanges output_ranges(int G) {
  NormRanges r{};
  r.n = hh_outputs(G);
  for (int q = 0; q <= r.n; ++q) r.c0[q] = q;
  return r;
}

// per-row, per-range norms of a split operand (no-op for FP64)
void launch_norms(int prec, const void* P0, const void* P1, int64_t n_rows, int64_t K,
                  const NormRanges& rg, float2* out, hipStream_t s) {
  if (prec == kFP64 || n_rows <= 0) return;
  const dim3 g((unsigned)((n_rows + 255) / 256));
  if (prec == kFP16X2)
    hipLaunchKernelGGL(k_operand_norms<kFP16X2>, g, dim3(256), 0, s, P0, P1, n_rows, K, rg, out);
  else
    hipLaunchKernelGGL(k_operand_norms<kBF16X2>, g, dim3(256), 0, s, P0, P1, n_rows, K, rg, out);
}

// the per-row norms of the event's split operands that the bound pass's
// margin takes, computed once, before the event's first bound pass
void event_norms(dotpe_event* ev, hipStream_t s) {
  if (ev->norms_done) return;
  const dotpe_bank* bk = ev->bank;
  const ModeTables& mt = bk->mt;
  launch_norms(bk->prec, ev->B[0], ev->B[1], ev->n_ext_p, bk->K2, group_ranges(mt), ev->b_nrm, s);
  launch_norms(bk->prec, ev->Ah[0], ev->Ah[1], ev->n_sub, ev->KH, output_ranges(mt.G), ev->ah_nrm, s);
  launch_norms(bk->prec, ev->Bh[0], ev->Bh[1], ev->n_ext_p, ev->KH, output_ranges(mt.G), ev->bh_nrm,
               s);
  ev->norms_done = true;
}

// FAST (evidence pass only): every pair through the bound first, one full
// evaluation pass after, tiles with too many survivors listed for a rerun
template <int MODE, bool FAST = false>
int launch_fused(int prec, const FusedArgs& a, int64_t grid, hipStream_t s) {
  FusedLaunchFn fn = fused_launcher(prec, a.mt.G);
  if (!fn) return fail(DOTPE_E_INVALID_ARG, "bad precision %d or group count %d", prec, a.mt.G);
  hipError_t e = fn(MODE, FAST, a, grid, s);
  if (e != hipSuccess)
    return fail(DOTPE_E_DEVICE, "fused kernel launch: %s", hipGetErrorString(e));
  return DOTPE_OK;
}

void tile_shape(int prec, int* tm, int* tn) {
  if (prec == kFP64) {
    *tm = Tile<kFP64>::TM;
    *tn = Tile<kFP64>::TN;
  } else {
    *tm = Tile<kFP16X2>::TM;
    *tn = Tile<kFP16X2>::TN;
  }
}

FusedArgs make_args(dotpe_ctx* ctx, dotpe_event* ev) {
  const dotpe_bank* bk = ev->bank;
  FusedArgs a;
  std::memset(&a, 0, sizeof(a));
  a.A0 = bk->A0;
  a.A1 = bk->A1;
  a.R0 = bk->R0;
  a.R1 = bk->R1;
  a.row_scale = bk->row_scale;
  a.ln_w_bank = bk->ln_w;
  a.sub_idx = ev->sub_idx;
  a.sub0 = ev->sub0;
  a.n_sub = ev->n_sub;
  a.B0 = ev->B[0];
  a.B1 = ev->B[1];
  a.B2 = ev->B[2];
  a.B3 = ev->B[3];
  a.col_scale = ev->col_scale;
  a.ln_w_ext = ev->ln_w_ext;
  a.n_ext = ev->n_ext;
  a.n_ext_p = ev->n_ext_p;
  a.K2 = bk->K2;
  a.n_chunks = (int)(bk->K2 / 32);
  a.Ah0 = ev->Ah[0];
  a.Ah1 = ev->Ah[1];
  a.ah_scale = ev->ah_scale;
  a.Bh0 = ev->Bh[0];
  a.Bh1 = ev->Bh[1];
  a.bh_scale = ev->bh_scale;
  a.KH = ev->KH;
  a.a_nrm = bk->nrm;
  a.b_nrm = ev->b_nrm;
  a.ah_nrm = ev->ah_nrm;
  a.bh_nrm = ev->bh_nrm;
  for (int g = 0; g < bk->mt.G; ++g)
    a.gam_dh[g] = (float)(1.4143 * 32.0 * (bk->mt.gk0[g + 1] - bk->mt.gk0[g]) * 0x1p-23);
  a.gam_hh = (float)(32.0 * 0x1p-23);
  a.n_det = ev->n_det;
  a.mt = bk->mt;
  a.n_phi = ev->n_phi;
  a.phase_cs = ev->phase_cs;
  a.ln_nphi = std::log((double)ev->n_phi);
  a.dist.tab = ctx->dist_tab;
  a.dist.prm = ctx->dist_prm;
  a.r0 = ev->d0 / ev->d_max;
  a.cut_delta = ev->cut_delta;
  a.topk_window = ev->topk_window;
  int tm, tn;
  tile_shape(bk->prec, &tm, &tn);
  a.n_tiles_m = (ev->n_sub + tm - 1) / tm;
  a.n_tiles_n = (ev->n_ext + tn - 1) / tn;
  a.n_tiles = a.n_tiles_m * a.n_tiles_n;
  a.coef = ev->coef;
  a.coef_tiles = ev->coef_tiles;
  a.rowcol = ev->rowcol;
  return a;
}

bool finite_all(const double* p, size_t n) {
  for (size_t i = 0; i < n; ++i)
    if (!std::isfinite(p[i])) return false;
  return true;
}

// state words: [0] running max of lnL^ML (bits of a non-negative double),
// [1] running max of ln p (ordered encoding), [2] candidate count,
// [3] cut reference frozen after the pilot pass, [4] tiles listed for the
// coefficient route, [5] tiles whose survivors are listed
__global__ void k_reset_state(uint64_t* st) {
  if (threadIdx.x == 0) {
    st[0] = 0ull;                       // bits of +0.0
    st[1] = 0x000fffffffffffffull;      // ordered encoding below every finite value
    st[2] = 0ull;
    st[3] = 0ull;
    st[4] = 0ull;
    st[5] = 0ull;
  }
}

__global__ void k_freeze_threshold(uint64_t* st) {
  if (threadIdx.x == 0) st[3] = st[0];
}

}  // namespace

extern "C" {

const char* dotpe_version(void) { return "dotpe 0.1 (gfx950)"; }

const char* dotpe_last_error(void) { return g_err.c_str(); }

int dotpe_create(int device, uint64_t hbm_budget_bytes, dotpe_ctx** out) {
  if (!out) return fail(DOTPE_E_INVALID_ARG, "out is NULL");
  int n = 0;
  HIP_OK(hipGetDeviceCount(&n));
  if (device < 0 || device >= n) return fail(DOTPE_E_INVALID_ARG, "device %d of %d", device, n);
  HIP_OK(hipSetDevice(device));
  {
    int rc0 = scratch_setup(device);
    if (rc0) return rc0;
  }
  dotpe_ctx* ctx = new dotpe_ctx();
  ctx->device = device;
  ctx->budget = hbm_budget_bytes;
  hipError_t e = hipStreamCreate(&ctx->stream);
  if (e != hipSuccess) {
    delete ctx;
    return fail(DOTPE_E_DEVICE, "hipStreamCreate: %s", hipGetErrorString(e));
  }
  constexpr DistTableGeom g = kDrGeom;
  size_t ntab = (size_t)g.ncol * g.nrow;
  ctx->budget = 0;
  int rc = dev_alloc(ctx, (void**)&ctx->dist_tab, ntab * sizeof(double) + sizeof(DistParams),
                     nullptr, nullptr);
  ctx->dist_prm = (DistParams*)(ctx->dist_tab + ntab);
  ctx->budget = hbm_budget_bytes;
  ctx->own_bytes = ctx->bytes;
  if (rc) {
    (void)hipStreamDestroy(ctx->stream);
    delete ctx;
    return rc;
  }
  hipLaunchKernelGGL(k_build_dist_table, dim3((unsigned)((ntab + 255) / 256)), dim3(256), 0,
                     ctx->stream, ctx->dist_tab, g);
  gauss_hermite(kGH, ctx->ghx, ctx->ghw);
  DistParams prm;
  for (int k = 0; k < kGH; ++k) {
    prm.ghx[k] = ctx->ghx[k];
    prm.ghw[k] = ctx->ghw[k];
  }
  e = hipMemcpyAsync(ctx->dist_prm, &prm, sizeof(prm), hipMemcpyHostToDevice, ctx->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
  if (e != hipSuccess) {
    dotpe_destroy(ctx);
    return fail(DOTPE_E_DEVICE, "distance table build: %s", hipGetErrorString(e));
  }
  *out = ctx;
  return DOTPE_OK;
}

int dotpe_destroy(dotpe_ctx* ctx) {
  if (!ctx) return DOTPE_OK;
  (void)hipSetDevice(ctx->device);
  if (ctx->ev_block) (void)hipFree(ctx->ev_block);
  if (ctx->dist_tab) (void)hipFree(ctx->dist_tab);
  if (ctx->stream) (void)hipStreamDestroy(ctx->stream);
  delete ctx;
  return DOTPE_OK;
}

uint64_t dotpe_device_bytes(const dotpe_ctx* ctx) { return ctx ? ctx->bytes.load() : 0; }

int dotpe_load_bank(dotpe_ctx* ctx, const dotpe_bank_desc* d, dotpe_bank** out) {
  if (!ctx || !d || !out) return fail(DOTPE_E_INVALID_ARG, "NULL argument");
  if (d->n_wf < 1 || d->n_modes < 1 || d->n_modes > kMaxC || d->n_bins < 1 || d->n_bins > 4096)
    return fail(DOTPE_E_INVALID_ARG, "bank shape n_wf=%lld n_modes=%d n_bins=%d out of range",
                (long long)d->n_wf, d->n_modes, d->n_bins);
  if (d->layout != DOTPE_LAYOUT_LM && d->layout != DOTPE_LAYOUT_MP)
    return fail(DOTPE_E_INVALID_ARG, "bad layout %d", d->layout);
  if ((d->layout == DOTPE_LAYOUT_LM && !d->mode_l) || (d->layout == DOTPE_LAYOUT_MP && !d->mode_p) ||
      !d->mode_m || !d->f_bins || !d->h)
    return fail(DOTPE_E_INVALID_ARG, "bank arrays must not be NULL");
  if (d->precision < 0 || d->precision > 2) return fail(DOTPE_E_INVALID_ARG, "bad precision");
  if (d->mem != DOTPE_MEM_HOST && d->mem != DOTPE_MEM_DEVICE)
    return fail(DOTPE_E_INVALID_ARG, "bad mem");
  if (!finite_all(d->f_bins, d->n_bins)) return fail(DOTPE_E_NUMERIC, "non-finite f_bins");
  HIP_OK(hipSetDevice(ctx->device));
  dotpe_bank* bk = new dotpe_bank();
  bk->n_wf = d->n_wf;
  bk->n_c = d->n_modes;
  bk->n_b = d->n_bins;
  bk->n_bp = (int)round_up(d->n_bins, 4 * kChunk);   // chunk count per channel divisible by 4
  bk->K2 = (int64_t)bk->n_c * bk->n_bp * 2;
  bk->prec = d->precision;
  int rc = build_modes(d, &bk->mt, bk->n_bp);
  if (rc) {
    delete bk;
    return rc;
  }
  bk->f_host.assign(d->f_bins, d->f_bins + d->n_bins);
  std::vector<void*> owned;
  auto cleanup = [&](int code) {
    for (void* p : owned) (void)hipFree(p);
    ctx->bytes -= bk->bytes;
    delete bk;
    return code;
  };
  const size_t esz = bk->prec == kFP64 ? 8 : 2;
  // split precisions: whole 32-row blocks (op_index layout)
  const size_t nA = (size_t)(bk->prec == kFP64 ? bk->n_wf : round_up(bk->n_wf, 32)) * bk->K2;
  if ((rc = dev_alloc(ctx, &bk->A0, nA * esz, &owned, &bk->bytes))) return cleanup(rc);
  if (bk->prec != kFP64) {
    if ((rc = dev_alloc(ctx, &bk->A1, nA * esz, &owned, &bk->bytes))) return cleanup(rc);
    const size_t nR = (size_t)bk->n_wf * bk->K2;
    if ((rc = dev_alloc(ctx, &bk->R0, nR * esz, &owned, &bk->bytes))) return cleanup(rc);
    if ((rc = dev_alloc(ctx, &bk->R1, nR * esz, &owned, &bk->bytes))) return cleanup(rc);
    if ((rc = dev_alloc(ctx, (void**)&bk->row_scale, bk->n_wf * 8, &owned, &bk->bytes)))
      return cleanup(rc);
    if ((rc = dev_alloc(ctx, (void**)&bk->nrm, bk->n_wf * bk->mt.G * sizeof(float2), &owned,
                        &bk->bytes)))
      return cleanup(rc);
  }
  if ((rc = dev_alloc(ctx, (void**)&bk->f, bk->n_b * 8, &owned, &bk->bytes))) return cleanup(rc);
  if ((rc = dev_alloc(ctx, (void**)&bk->ln_w, bk->n_wf * 8, &owned, &bk->bytes)))
    return cleanup(rc);
  int* err = nullptr;
  if ((rc = dev_alloc(ctx, (void**)&err, 64, &owned, &bk->bytes))) return cleanup(rc);
  hipStream_t s = ctx->stream;
  auto hip_fail = [&](hipError_t e, const char* what) {
    (void)hipStreamSynchronize(s);
    int c = fail(DOTPE_E_DEVICE, "%s: %s", what, hipGetErrorString(e));
    return cleanup(c);
  };
  hipError_t e;
  if ((e = hipMemcpyAsync(bk->f, d->f_bins, bk->n_b * 8, hipMemcpyHostToDevice, s)))
    return hip_fail(e, "copy f");
  if ((e = hipMemsetAsync(err, 0, 64, s))) return hip_fail(e, "memset");
  if (d->ln_w) {
    if ((e = hipMemcpyAsync(bk->ln_w, d->ln_w, bk->n_wf * 8,
                            d->mem == DOTPE_MEM_HOST ? hipMemcpyHostToDevice
                                                     : hipMemcpyDeviceToDevice, s)))
      return hip_fail(e, "copy ln_w");
  } else if ((e = hipMemsetAsync(bk->ln_w, 0, bk->n_wf * 8, s))) {
    return hip_fail(e, "memset ln_w");
  }
  if (bk->prec == kFP64 && (e = hipMemsetAsync(bk->A0, 0, nA * esz, s)))
    return hip_fail(e, "memset A");
  // amplitudes: staged through a bounded device buffer when on the host
  const size_t row_bytes = (size_t)bk->n_c * bk->n_b * 16;
  if (d->mem == DOTPE_MEM_DEVICE) {
    switch (bk->prec) {
      case kFP64: launch_bank_convert<kFP64>(d->h, bk, err, s); break;
      case kFP16X2: launch_bank_convert<kFP16X2>(d->h, bk, err, s); break;
      default: launch_bank_convert<kBF16X2>(d->h, bk, err, s); break;
    }
    if ((e = hipGetLastError())) return hip_fail(e, "bank convert");
  } else {
    // whole 32-row blocks per stage, so that a stage starts a block
    int64_t rows_per = std::max<int64_t>(32, (int64_t)((256ull << 20) / row_bytes) / 32 * 32);
    rows_per = std::min(rows_per, round_up(bk->n_wf, 32));
    double* stagebuf = nullptr;
    if ((e = hipMalloc((void**)&stagebuf, rows_per * row_bytes))) return hip_fail(e, "stage alloc");
    for (int64_t r0 = 0; r0 < bk->n_wf; r0 += rows_per) {
      int64_t nr = std::min(rows_per, bk->n_wf - r0);
      e = hipMemcpyAsync(stagebuf, d->h + (size_t)r0 * bk->n_c * bk->n_b * 2, nr * row_bytes,
                         hipMemcpyHostToDevice, s);
      if (e) break;
      dotpe_bank view = *bk;
      view.n_wf = nr;
      view.A0 = (char*)bk->A0 + (size_t)r0 * bk->K2 * esz;
      view.A1 = bk->A1 ? (char*)bk->A1 + (size_t)r0 * bk->K2 * esz : nullptr;
      view.R0 = bk->R0 ? (char*)bk->R0 + (size_t)r0 * bk->K2 * esz : nullptr;
      view.R1 = bk->R1 ? (char*)bk->R1 + (size_t)r0 * bk->K2 * esz : nullptr;
      view.row_scale = bk->row_scale ? bk->row_scale + r0 : nullptr;
      switch (bk->prec) {
        case kFP64: launch_bank_convert<kFP64>(stagebuf, &view, err, s); break;
        case kFP16X2: launch_bank_convert<kFP16X2>(stagebuf, &view, err, s); break;
        default: launch_bank_convert<kBF16X2>(stagebuf, &view, err, s); break;
      }
      if ((e = hipGetLastError())) break;
      if ((e = hipStreamSynchronize(s))) break;
    }
    (void)hipStreamSynchronize(s);
    (void)hipFree(stagebuf);
    if (e) return hip_fail(e, "bank staging");
  }
  launch_norms(bk->prec, bk->A0, bk->A1, bk->n_wf, bk->K2, group_ranges(bk->mt), bk->nrm, s);
  if ((e = hipGetLastError())) return hip_fail(e, "bank norms");
  int herr = 0;
  if ((e = hipMemcpyAsync(&herr, err, sizeof(int), hipMemcpyDeviceToHost, s)))
    return hip_fail(e, "copy err");
  if ((e = hipStreamSynchronize(s))) return hip_fail(e, "bank sync");
  if (herr) return cleanup(fail(DOTPE_E_NUMERIC, "non-finite bank amplitudes"));
  (void)hipFree(err);
  owned.erase(std::find(owned.begin(), owned.end(), (void*)err));
  ctx->bytes -= 64;
  bk->bytes -= 64;
  *out = bk;
  return DOTPE_OK;
}

int dotpe_free_bank(dotpe_ctx* ctx, dotpe_bank* bk) {
  if (!ctx || !bk) return DOTPE_OK;
  (void)hipSetDevice(ctx->device);
  for (void* p : {bk->A0, bk->A1, bk->R0, bk->R1, (void*)bk->row_scale, (void*)bk->nrm, (void*)bk->f,
                  (void*)bk->ln_w})
    if (p) (void)hipFree(p);
  ctx->bytes -= bk->bytes;
  delete bk;
  return DOTPE_OK;
}

int dotpe_free_event(dotpe_ctx* ctx, dotpe_event* ev) {
  if (!ctx || !ev) return DOTPE_OK;
  (void)hipSetDevice(ctx->device);
  (void)hipStreamSynchronize(ev->stream);
  for (void* p : ev->allocs) (void)hipFree(p);
  for (hipEvent_t t : ev->ev_t)
    if (t) (void)hipEventDestroy(t);
  if (ev->ctx_block) {
    std::lock_guard<std::mutex> lk(ctx->ev_mu);
    ctx->ev_block_busy = false;    // kept for the next event
  }
  ctx->bytes -= ev->bytes;
  delete ev;
  return DOTPE_OK;
}

}  // extern "C"

namespace {

// validated description of one event and the shapes derived from it
struct EvDims {
  int nk = 0, nb = 0, nc = 0, n_bp = 0, n_phi = 0, KH = 0, NP = 0, prec = 0, G = 0;
  int64_t ne = 0, ne_p = 0, n_sub = 0, K2 = 0, n_tiles = 0, cand_cap = 0;
  int64_t coef_tiles = 0;          // tiles per chunk of the coefficient route
  uint64_t coef_tile_bytes = 0;    // their raw accumulators, bytes per tile
  bool ln_w_ext = false, sub_idx = false;
  bool rb = false;                 // relative-binning weights given
};

// input staging buffers of set_event (used only while the event is staged)
struct EvStage {
  double *d = nullptr, *w = nullptr, *r = nullptr, *D = nullptr, *lat = nullptr, *lon = nullptr,
         *psi = nullptr, *ci = nullptr, *tg = nullptr;
  double2* Btmp = nullptr;
  double2* wdh = nullptr;   // relative binning: [nk][nc][nb] (group order), [nk][NP][nb]
  double2* whh = nullptr;
  int* err = nullptr;
};

struct EvBuf {
  void** p;
  size_t n;
  bool stage;
};

// coef_cap: most bytes of the coefficient route's buffer (0: 8 GiB)
int event_dims(const dotpe_bank* bk, const dotpe_event_desc* d, EvDims* D, std::vector<int>* terms,
               uint64_t coef_cap = 0) {
  if (d->n_det < 1 || d->n_det > kMaxDet) return fail(DOTPE_E_INVALID_ARG, "n_det=%d", d->n_det);
  if (d->n_phi < 1 || d->n_phi > kMaxPhi) return fail(DOTPE_E_INVALID_ARG, "n_phi=%d", d->n_phi);
  if (d->n_ext < 1) return fail(DOTPE_E_INVALID_ARG, "n_ext=%lld", (long long)d->n_ext);
  const bool rb = d->w_dh != nullptr;
  if ((!rb && (!d->d || !d->w)) || !d->det_r || !d->det_D || !d->lat || !d->lon || !d->psi ||
      !d->cos_iota || !d->t_geo)
    return fail(DOTPE_E_INVALID_ARG, "event arrays must not be NULL");
  if (rb && !d->w_hh)
    return fail(DOTPE_E_INVALID_ARG, "relative binning needs both w_dh and w_hh");
  if (!(d->d_max > 0.0) || !(d->d0 > 0.0) || !std::isfinite(d->d_max) || !std::isfinite(d->d0))
    return fail(DOTPE_E_INVALID_ARG, "distances must be positive and finite");
  if (d->flags & ~(DOTPE_FLAG_RERUN_ALL | DOTPE_FLAG_NO_BOUND_PASS))
    return fail(DOTPE_E_INVALID_ARG, "unknown flags 0x%x", d->flags);
  int KH = 0;
  {
    int rc0 = build_hh_terms(bk->mt, d->n_det, terms, &KH);
    if (rc0) return rc0;
  }
  const int nb = bk->n_b, nk = d->n_det;
  const int64_t ne = d->n_ext;
  const size_t nc_ = (size_t)bk->n_c;
  if ((!rb && (!finite_all(d->d, (size_t)nk * nb * 2) || !finite_all(d->w, (size_t)nk * nb))) ||
      (rb && (!finite_all(d->w_dh, (size_t)nk * nc_ * nb * 2) ||
              !finite_all(d->w_hh, (size_t)nk * nc_ * nc_ * nb * 2) || !std::isfinite(d->dd))) ||
      !finite_all(d->det_r, nk * 3) || !finite_all(d->det_D, nk * 9) || !finite_all(d->lat, ne) ||
      !finite_all(d->lon, ne) || !finite_all(d->psi, ne) || !finite_all(d->cos_iota, ne) ||
      !finite_all(d->t_geo, ne) || (d->ln_w_ext && !finite_all(d->ln_w_ext, ne)))
    return fail(DOTPE_E_NUMERIC, "non-finite event input");
  for (int64_t e = 0; e < ne; ++e)
    if (std::fabs(d->cos_iota[e]) > 1.0) return fail(DOTPE_E_INVALID_ARG, "|cos_iota| > 1");
  for (size_t t = 0; t < (size_t)nk * nb && !rb; ++t)
    if (d->w[t] < 0.0) return fail(DOTPE_E_INVALID_ARG, "negative noise weight");
  int64_t n_sub = d->sub_count > 0 ? d->sub_count : bk->n_wf;
  if (d->sub_idx) {
    if (d->sub_count < 1) return fail(DOTPE_E_INVALID_ARG, "sub_idx needs sub_count >= 1");
    for (int64_t r = 0; r < n_sub; ++r)
      if (d->sub_idx[r] < 0 || d->sub_idx[r] >= bk->n_wf)
        return fail(DOTPE_E_INVALID_ARG, "sub_idx[%lld]=%lld out of range", (long long)r,
                    (long long)d->sub_idx[r]);
  } else if (d->sub_start < 0 || d->sub_start + n_sub > bk->n_wf) {
    return fail(DOTPE_E_INVALID_ARG, "bank range out of bounds");
  }
  D->nk = nk;
  D->nb = nb;
  D->nc = bk->n_c;
  D->n_bp = bk->n_bp;
  D->n_phi = d->n_phi;
  D->KH = KH;
  D->NP = bk->mt.NP;
  D->G = bk->mt.G;
  D->prec = bk->prec;
  D->ne = ne;
  D->ne_p = round_up(ne, 128);   // whole 128-sample tiles of the bound pass
  D->n_sub = n_sub;
  D->K2 = bk->K2;
  int tm, tn;
  tile_shape(bk->prec, &tm, &tn);
  D->n_tiles = ((n_sub + tm - 1) / tm) * ((ne + tn - 1) / tn);
  // top-k candidate buffer: a power of two (the bitonic sort runs in place),
  // never more than the number of pairs
  int64_t want = std::max<int64_t>(int64_t(1) << 20, 16 * (int64_t)std::max(0, d->top_k));
  want = std::max<int64_t>(1, std::min<int64_t>(want, n_sub * ne));
  int64_t cap = 1;
  while (cap < want) cap <<= 1;
  D->cand_cap = cap;
  // coefficient route: chunks of whole tiles, enough to fill the device and
  // few enough that a pass makes at most ~64 pairs of launches
  {
    const int G = bk->mt.G, nrt = G == 1 ? 1 : kMaxNR;
    D->coef_tile_bytes = (uint64_t)(2 * G + nrt) * tm * tn * (bk->prec == kFP64 ? 8 : 4);
    const uint64_t most = coef_cap ? coef_cap : (uint64_t(8) << 30);
    int64_t c = std::max<int64_t>(2048, (D->n_tiles + 63) / 64);
    c = std::min<int64_t>(c, (int64_t)(most / D->coef_tile_bytes));
    D->coef_tiles = std::max<int64_t>(1, std::min(c, D->n_tiles));
  }
  D->ln_w_ext = d->ln_w_ext != nullptr;
  D->rb = d->w_dh != nullptr;
  D->sub_idx = d->sub_idx != nullptr;
  return DOTPE_OK;
}

// the event's device buffers in allocation order: what it keeps, then the
// staging of its inputs
std::vector<EvBuf> event_buffers(const EvDims& D, dotpe_event* ev, EvStage* st) {
  std::vector<EvBuf> v;
  const size_t esz = D.prec == kFP64 ? 8 : 2;
  // FP64: B_re, B_im; split precisions: B_re hi, lo (B_im is the other slice of B_re)
  for (int q = 0; q < 2; ++q) v.push_back({&ev->B[q], (size_t)D.ne_p * D.K2 * esz, false});
  if (D.prec != kFP64) v.push_back({(void**)&ev->col_scale, (size_t)D.ne * 8, false});
  v.push_back({(void**)&ev->hh_terms, (size_t)D.KH * sizeof(int), false});
  for (int q = 0; q < (D.prec == kFP64 ? 1 : 2); ++q) {
    // split precisions: whole 32-row blocks (op_index layout)
    const int64_t ah_rows = D.prec == kFP64 ? D.n_sub : round_up(D.n_sub, 32);
    v.push_back({&ev->Ah[q], (size_t)ah_rows * D.KH * esz, false});
    v.push_back({&ev->Bh[q], (size_t)D.ne_p * D.KH * esz, false});
  }
  if (D.prec != kFP64) {
    v.push_back({(void**)&ev->ah_scale, (size_t)D.n_sub * 8, false});
    v.push_back({(void**)&ev->bh_scale, (size_t)D.ne * 8, false});
    v.push_back({(void**)&ev->b_nrm, (size_t)D.ne_p * D.G * sizeof(float2), false});
    v.push_back({(void**)&ev->ah_nrm, (size_t)D.n_sub * hh_outputs(D.G) * sizeof(float2), false});
    v.push_back({(void**)&ev->bh_nrm, (size_t)D.ne_p * hh_outputs(D.G) * sizeof(float2), false});
  }
  v.push_back({(void**)&ev->Q, (size_t)D.ne * D.nk * D.NP * 16, false});
  v.push_back({(void**)&ev->R2, (size_t)D.ne * D.nk * D.nc * 8, false});
  v.push_back({(void**)&ev->R, (size_t)D.ne * D.nk * D.nc * 16, false});
  v.push_back({(void**)&ev->T, (size_t)D.ne * D.nk * 8, false});
  v.push_back({(void**)&ev->phase_cs, (size_t)kMaxM * D.n_phi * 2 * 8, false});
  if (D.ln_w_ext) v.push_back({(void**)&ev->ln_w_ext, (size_t)D.ne * 8, false});
  if (D.sub_idx) v.push_back({(void**)&ev->sub_idx, (size_t)D.n_sub * 8, false});
  v.push_back({(void**)&ev->state, 64, false});
  v.push_back({(void**)&ev->final_out, kNPart * 8 + 64, false});
  v.push_back({(void**)&ev->partials, (size_t)D.n_tiles * kNPart * 8, false});
  v.push_back({(void**)&ev->final_blk, (size_t)((D.n_tiles + 4095) / 4096) * kNPart * 8, false});
  v.push_back({(void**)&ev->cand, (size_t)D.cand_cap * 32, false});
  v.push_back({(void**)&ev->rerun, (size_t)D.n_tiles * sizeof(int), false});
  v.push_back({&ev->coef, (size_t)D.coef_tiles * D.coef_tile_bytes, false});
  v.push_back({(void**)&ev->rowcol, (size_t)D.n_tiles * 128 * 8, false});
  {
    int tm, tn;
    tile_shape(D.prec, &tm, &tn);
    const int64_t ntm = (D.n_sub + tm - 1) / tm, ntn = (D.ne + tn - 1) / tn;
    const int64_t parts = std::max(D.n_sub * ((ntn + kMargPer - 1) / kMargPer),
                                   D.ne * ((ntm + kMargPer - 1) / kMargPer));
    v.push_back({(void**)&ev->marg_part, (size_t)parts * 8, false});
  }
  v.push_back({(void**)&ev->marg_blk, (size_t)((std::max(D.n_sub, D.ne) + 255) / 256) * 8, false});
  if (D.prec != kFP64) {
    v.push_back({(void**)&ev->surv, (size_t)D.n_tiles * kSurvCap * sizeof(uint16_t), false});
    v.push_back({(void**)&ev->surv_list, (size_t)D.n_tiles * 2 * sizeof(int), false});
  }
  v.push_back({(void**)&st->d, (size_t)D.nk * D.nb * 16, true});
  v.push_back({(void**)&st->w, (size_t)D.nk * D.nb * 8, true});
  v.push_back({(void**)&st->r, (size_t)D.nk * 24, true});
  v.push_back({(void**)&st->D, (size_t)D.nk * 72, true});
  v.push_back({(void**)&st->lat, (size_t)D.ne * 8, true});
  v.push_back({(void**)&st->lon, (size_t)D.ne * 8, true});
  v.push_back({(void**)&st->psi, (size_t)D.ne * 8, true});
  v.push_back({(void**)&st->ci, (size_t)D.ne * 8, true});
  v.push_back({(void**)&st->tg, (size_t)D.ne * 8, true});
  v.push_back({(void**)&st->Btmp, (size_t)D.ne * D.nc * D.n_bp * 16, true});
  if (D.rb) {
    v.push_back({(void**)&st->wdh, (size_t)D.nk * D.nc * D.nb * 16, true});
    v.push_back({(void**)&st->whh, (size_t)D.nk * D.NP * D.nb * 16, true});
  }
  v.push_back({(void**)&st->err, 64, true});
  return v;
}

constexpr uint64_t kBlockAlign = 256;

// bytes of one block holding every buffer of the list, packed as set_event packs them
uint64_t block_bytes(const std::vector<EvBuf>& v) {
  uint64_t off = 0;
  for (const EvBuf& b : v) off = round_up(off, kBlockAlign) + b.n;
  return round_up(off, kBlockAlign);
}

// Stage one event.  With block == nullptr every buffer is its own device
// allocation (staging buffers are freed before returning); otherwise all of
// them are packed into the caller's device block of block_len bytes and
// nothing is allocated.
int set_event_impl(dotpe_ctx* ctx, const dotpe_bank* bk, const dotpe_event_desc* d, char* block,
                   uint64_t block_len, hipStream_t s, dotpe_event** out, uint64_t coef_cap = 0) {
  EvDims D;
  std::vector<int> terms;
  int rc = event_dims(bk, d, &D, &terms, coef_cap);
  if (rc) return rc;
  HIP_OK(hipSetDevice(ctx->device));
  dotpe_event* ev = new dotpe_event();
  ev->bank = bk;
  ev->stream = s;
  ev->n_det = D.nk;
  ev->n_phi = D.n_phi;
  ev->n_ext = D.ne;
  ev->n_ext_p = D.ne_p;
  ev->n_sub = D.n_sub;
  ev->sub0 = d->sub_idx ? 0 : d->sub_start;
  ev->d0 = d->d0;
  ev->d_max = d->d_max;
  ev->n_norm = d->n_norm > 0 ? d->n_norm : (double)D.n_sub;
  ev->cut_delta = d->cut_delta;
  ev->topk_window = d->topk_window > 0 ? d->topk_window : 40.0;
  ev->cut_target = d->cut_target > 0 ? d->cut_target : 1e-4;
  ev->top_k = std::max(0, d->top_k);
  ev->flags = d->flags;
  ev->KH = D.KH;
  ev->cand_cap = D.cand_cap;
  ev->coef_tiles = D.coef_tiles;
  const ModeTables& mt = bk->mt;
  const int nb = D.nb, nk = D.nk, nc = D.nc;
  const int64_t ne = D.ne, n_sub = D.n_sub;
  EvStage st;
  std::vector<EvBuf> bufs = event_buffers(D, ev, &st);
  std::vector<void*> tmp;
  uint64_t tmp_bytes = 0;
  auto release_tmp = [&]() {
    (void)hipStreamSynchronize(s);
    for (void* p : tmp) (void)hipFree(p);
    ctx->bytes -= tmp_bytes;
    tmp.clear();
    tmp_bytes = 0;
  };
  auto cleanup = [&](int code) {
    release_tmp();
    for (void* p : ev->allocs) (void)hipFree(p);
    ctx->bytes -= ev->bytes;
    delete ev;
    return code;
  };
  uint64_t off = 0;
  for (const EvBuf& b : bufs) {
    if (block) {
      off = round_up(off, kBlockAlign);
      if (off + b.n > block_len)
        return cleanup(fail(DOTPE_E_ADMISSION, "event does not fit its %llu-byte block",
                            (unsigned long long)block_len));
      *b.p = block + off;
      off += b.n;
    } else {
      rc = b.stage ? dev_alloc(ctx, b.p, b.n, &tmp, &tmp_bytes)
                   : dev_alloc(ctx, b.p, b.n, &ev->allocs, &ev->bytes);
      if (rc) return cleanup(rc);
    }
  }
  hipError_t e = hipSuccess;
  auto H2D = [&](void* dst, const void* src, size_t n) {
    if (e == hipSuccess) e = hipMemcpyAsync(dst, src, n, hipMemcpyHostToDevice, s);
  };
  if (D.rb) {
    // relative-binning weights: W^dh to group order, W^hh to the stored
    // channel pairs (c <= c' in group order), read from c <= c' in the
    // caller's order and conjugated where the two orders differ
    std::vector<double2> wdh((size_t)nk * nc * nb), whh((size_t)nk * D.NP * nb);
    const double2* Wd = (const double2*)d->w_dh;
    const double2* Wh = (const double2*)d->w_hh;
    for (int k = 0; k < nk; ++k) {
      for (int c = 0; c < nc; ++c)
        for (int b = 0; b < nb; ++b)
          wdh[((size_t)k * nc + c) * nb + b] = Wd[((size_t)k * nc + mt.orig[c]) * nb + b];
      for (int p = 0; p < D.NP; ++p) {
        const int a = mt.orig[mt.pc[p]], a2 = mt.orig[mt.pc2[p]];
        const int lo = std::min(a, a2), hi = std::max(a, a2);
        for (int b = 0; b < nb; ++b) {
          double2 v = Wh[(((size_t)k * nc + lo) * nc + hi) * nb + b];
          if (a > a2) v.y = -v.y;
          whh[((size_t)k * D.NP + p) * nb + b] = v;
        }
      }
    }
    H2D(st.wdh, wdh.data(), wdh.size() * 16);
    H2D(st.whh, whh.data(), whh.size() * 16);
    if (e == hipSuccess) e = hipStreamSynchronize(s);   // the host vectors end with this scope
  } else {
    H2D(st.d, d->d, (size_t)nk * nb * 16);
    H2D(st.w, d->w, (size_t)nk * nb * 8);
  }
  H2D(st.r, d->det_r, (size_t)nk * 24);
  H2D(st.D, d->det_D, (size_t)nk * 72);
  H2D(st.lat, d->lat, ne * 8);
  H2D(st.lon, d->lon, ne * 8);
  H2D(st.psi, d->psi, ne * 8);
  H2D(st.ci, d->cos_iota, ne * 8);
  H2D(st.tg, d->t_geo, ne * 8);
  if (d->ln_w_ext) H2D(ev->ln_w_ext, d->ln_w_ext, ne * 8);
  if (d->sub_idx) H2D(ev->sub_idx, d->sub_idx, n_sub * 8);
  H2D(ev->hh_terms, terms.data(), terms.size() * sizeof(int));
  if (e == hipSuccess) e = hipMemsetAsync(st.err, 0, 64, s);
  // phase table cos, sin (m phi_o), m = 1..4 (a twiddle table of the grid)
  std::vector<double> cs((size_t)kMaxM * d->n_phi * 2);
  for (int m = 1; m <= kMaxM; ++m)
    for (int o = 0; o < d->n_phi; ++o) {
      double ph = 2.0 * M_PI * (double)((m * o) % d->n_phi) / d->n_phi;
      cs[((m - 1) * d->n_phi + o) * 2] = std::cos(ph);
      cs[((m - 1) * d->n_phi + o) * 2 + 1] = std::sin(ph);
    }
  H2D(ev->phase_cs, cs.data(), cs.size() * 8);
  if (e != hipSuccess)
    return cleanup(fail(DOTPE_E_DEVICE, "event upload: %s", hipGetErrorString(e)));
  // extrinsic response, B operand, (h|h) tables, (d|d)
  hipLaunchKernelGGL(k_ext_response, dim3((unsigned)((ne + 127) / 128)), dim3(128), 0, s, ne, nk,
                     st.r, st.D, st.lat, st.lon, st.psi, st.ci, st.tg, mt, ev->R, ev->T, ev->Q,
                     ev->R2);
  int64_t nbt = ne * nc * bk->n_bp;
  hipLaunchKernelGGL(k_build_B, dim3((unsigned)((nbt + 255) / 256)), dim3(256), 0, s, ne, nk, nc,
                     nb, bk->n_bp, bk->f, (const double2*)st.d, st.w, (const double2*)st.wdh, ev->R,
                     ev->T, st.Btmp);
  switch (bk->prec) {
    case kFP64: launch_convert_B<kFP64>(ev, st.Btmp, st.err); break;
    case kFP16X2: launch_convert_B<kFP16X2>(ev, st.Btmp, st.err); break;
    default: launch_convert_B<kBF16X2>(ev, st.Btmp, st.err); break;
  }
  switch (bk->prec) {
    case kFP64: launch_hh<kFP64>(ev, st.w, st.whh); break;
    case kFP16X2: launch_hh<kFP16X2>(ev, st.w, st.whh); break;
    default: launch_hh<kBF16X2>(ev, st.w, st.whh); break;
  }
  hipError_t e_dd = hipSuccess;
  if (D.rb) {
    // (d|d) as given (full resolution)
    e_dd = hipMemcpyAsync(ev->final_out + kNPart, &d->dd, 8, hipMemcpyHostToDevice, s);
  } else {
    hipLaunchKernelGGL(k_data_norm, dim3(1), dim3(256), 0, s, nk * nb, (const double2*)st.d, st.w,
                       ev->final_out + kNPart);
  }
  e = hipGetLastError();
  if (e == hipSuccess) e = e_dd;
  int herr = 0;
  if (e == hipSuccess) e = hipMemcpyAsync(&herr, st.err, sizeof(int), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess)
    e = hipMemcpyAsync(&ev->dd, ev->final_out + kNPart, 8, hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  release_tmp();
  if (e != hipSuccess) return cleanup(fail(DOTPE_E_DEVICE, "event staging: %s", hipGetErrorString(e)));
  if (herr) return cleanup(fail(DOTPE_E_NUMERIC, "non-finite extrinsic operand"));
  *out = ev;
  return DOTPE_OK;
}

}  // namespace

extern "C" {

int dotpe_set_event(dotpe_ctx* ctx, const dotpe_bank* bk, const dotpe_event_desc* d,
                    dotpe_event** out) {
  if (!ctx || !bk || !d || !out) return fail(DOTPE_E_INVALID_ARG, "NULL argument");
  hipStream_t s = d->stream ? (hipStream_t)d->stream : ctx->stream;
  uint64_t need = 0;
  {
    EvDims D;
    std::vector<int> terms;
    int rc = event_dims(bk, d, &D, &terms);
    if (rc) return rc;
    dotpe_event probe;
    EvStage st;
    need = block_bytes(event_buffers(D, &probe, &st));
  }
  // the context's event block when it is free: grown (freed and allocated
  // again) when the event needs more; an event set while another holds the
  // block gets buffers of its own
  char* block = nullptr;
  uint64_t len = 0;
  {
    std::lock_guard<std::mutex> lk(ctx->ev_mu);
    if (!ctx->ev_block_busy) {
      HIP_OK(hipSetDevice(ctx->device));
      if (ctx->ev_block_len < need) {
        if (ctx->ev_block) {
          (void)hipFree(ctx->ev_block);
          ctx->bytes -= ctx->ev_block_len;
          ctx->ev_block = nullptr;
          ctx->ev_block_len = 0;
        }
        if (dev_alloc(ctx, (void**)&ctx->ev_block, need, nullptr, nullptr) == DOTPE_OK)
          ctx->ev_block_len = need;
      }
      if (ctx->ev_block) {
        ctx->ev_block_busy = true;
        block = ctx->ev_block;
        len = ctx->ev_block_len;
      }
    }
  }
  if (!block) return set_event_impl(ctx, bk, d, nullptr, 0, s, out);
  int rc = set_event_impl(ctx, bk, d, block, len, s, out);
  if (rc) {
    std::lock_guard<std::mutex> lk(ctx->ev_mu);
    ctx->ev_block_busy = false;
    return rc;
  }
  (*out)->ctx_block = true;
  return DOTPE_OK;
}

int dotpe_event_bytes(const dotpe_ctx* ctx, const dotpe_bank* bk, const dotpe_event_desc* d,
                      uint64_t* bytes) {
  if (!ctx || !bk || !d || !bytes) return fail(DOTPE_E_INVALID_ARG, "NULL argument");
  EvDims D;
  std::vector<int> terms;
  int rc = event_dims(bk, d, &D, &terms);
  if (rc) return rc;
  dotpe_event probe;
  EvStage st;
  *bytes = block_bytes(event_buffers(D, &probe, &st));
  return DOTPE_OK;
}

int dotpe_eval_lnl(dotpe_ctx* ctx, dotpe_event* ev, double* lnl, double* ml_max, double* triples,
                   int32_t mem) {
  if (!ctx || !ev || !lnl) return fail(DOTPE_E_INVALID_ARG, "NULL argument");
  if (mem != DOTPE_MEM_HOST && mem != DOTPE_MEM_DEVICE) return fail(DOTPE_E_INVALID_ARG, "bad mem");
  HIP_OK(hipSetDevice(ctx->device));
  const size_t npair = (size_t)ev->n_sub * ev->n_ext;
  const size_t ntrip = triples ? npair * ev->n_phi * 2 : 0;
  hipStream_t s = ev->stream;
  double *o1 = lnl, *o2 = ml_max, *o3 = triples;
  std::vector<void*> tmp;
  uint64_t tb = 0;
  auto release = [&]() {
    (void)hipStreamSynchronize(s);
    for (void* p : tmp) (void)hipFree(p);
    ctx->bytes -= tb;
  };
  int rc;
  if (mem == DOTPE_MEM_HOST) {
    if ((rc = dev_alloc(ctx, (void**)&o1, npair * 8, &tmp, &tb))) { release(); return rc == DOTPE_E_ADMISSION ? fail(DOTPE_E_TOO_LARGE, "%s", g_err.c_str()) : rc; }
    if (ml_max && (rc = dev_alloc(ctx, (void**)&o2, npair * 8, &tmp, &tb))) { release(); return rc == DOTPE_E_ADMISSION ? fail(DOTPE_E_TOO_LARGE, "%s", g_err.c_str()) : rc; }
    if (triples && (rc = dev_alloc(ctx, (void**)&o3, ntrip * 8, &tmp, &tb))) { release(); return rc == DOTPE_E_ADMISSION ? fail(DOTPE_E_TOO_LARGE, "%s", g_err.c_str()) : rc; }
  }
  FusedArgs a = make_args(ctx, ev);
  a.lnl_out = o1;
  a.ml_out = ml_max ? o2 : nullptr;
  a.trip_out = triples ? o3 : nullptr;
  int64_t grid = round_up(a.n_tiles, 8);
  rc = launch_fused<kEval>(ev->bank->prec, a, grid, s);
  if (rc) { release(); return rc; }
  hipError_t e = hipSuccess;
  if (mem == DOTPE_MEM_HOST) {
    e = hipMemcpyAsync(lnl, o1, npair * 8, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess && ml_max) e = hipMemcpyAsync(ml_max, o2, npair * 8, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess && triples) e = hipMemcpyAsync(triples, o3, ntrip * 8, hipMemcpyDeviceToHost, s);
  }
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  release();
  if (e != hipSuccess) return fail(DOTPE_E_DEVICE, "eval_lnl: %s", hipGetErrorString(e));
  return DOTPE_OK;
}

// Persistent grids of the passes whose work is known on the device only
constexpr int64_t kSurvGrid = 65536;  // workgroups of 4 waves, a listed tile per wave
constexpr int64_t kCoefGrid = 1024;   // fused kernel, a tile per workgroup at a time
constexpr int64_t kE2Grid = 4096;

// Arguments of one evidence pass of ev with cut `cut_delta` (<= 0: none).
// The fast pass only bounds: a tile with any survivor takes the coefficient
// route (where every evaluated pair also enters its tile's row and column
// sums).  The pilot takes every pilot_stride-th row of tiles: 1 in 64 rows
// on large events, and at least 16 rows of tiles on small ones (a sparse
// pilot there may miss the rows that set the maximum, and then nothing is
// cut).
static FusedArgs pass_args(dotpe_ctx* ctx, dotpe_event* ev, double cut_delta) {
  FusedArgs a = make_args(ctx, ev);
  a.cut_delta = cut_delta;
  a.state = ev->state;
  a.partials = ev->partials;
  a.cand = ev->cand;
  a.cand_cap = ev->cand_cap;
  a.rerun = ev->rerun;
  a.surv = ev->surv;
  a.surv_list = ev->surv_list;
  a.rec_cap = 0;
  a.pilot_stride = std::max<int64_t>(1, std::min<int64_t>(64, a.n_tiles_m / 16));
  return a;
}

// The pass's decisions that the host takes from sizes alone.  The cut needs
// a pilot over other rows of tiles than the ones it cuts; without one the
// frozen threshold stays at zero and the cut is off.  The bound pass (128 x
// 128 tiles, split precisions) runs when the event has enough of them to
// fill the device, else the fused kernel's fast pass; both return at once
// when the frozen threshold does not cut.
struct PassPlan {
  bool may_cut = false, bound_pass = false;
  int64_t pilot_grid = 0, cut_grid = 0, surv_grid = 0, n_chunks = 0, coef_grid = 0, e2_grid = 0;
};

static PassPlan pass_plan(const dotpe_event* ev, const FusedArgs& a) {
  PassPlan p;
  const int prec = ev->bank->prec;
  p.may_cut = a.cut_delta > 0.0 && a.n_tiles_m > 1;
  if (p.may_cut) {
    const int64_t npr = (a.n_tiles_m + a.pilot_stride - 1) / a.pilot_stride;
    p.pilot_grid = round_up(npr * a.n_tiles_n, 8);
    const int64_t n_big = ((a.n_tiles_m + 1) / 2) * ((a.n_tiles_n + 1) / 2);
    p.bound_pass = prec != kFP64 && n_big >= kBoundMinTiles &&
                   !(ev->flags & (DOTPE_FLAG_NO_BOUND_PASS | DOTPE_FLAG_RERUN_ALL));
    p.cut_grid = round_up(p.bound_pass ? n_big : a.n_tiles, 8);
    if (p.bound_pass) p.surv_grid = std::min<int64_t>(kSurvGrid, (a.n_tiles + 3) / 4);
  }
  // coefficient route: chunks of coef_tiles work items, as many chunks as
  // every tile would need; the kernels of a chunk past the device's count
  // return at once
  const int64_t C = ev->coef_tiles;
  p.n_chunks = (a.n_tiles + C - 1) / C;
  p.coef_grid = std::min(C, kCoefGrid);
  p.e2_grid = std::min(C, kE2Grid);
  return p;
}

// the pass's first kernels: its state and the tiles' row and column sums
static int pass_head(dotpe_event* ev, const FusedArgs& a, hipStream_t s) {
  hipLaunchKernelGGL(k_reset_state, dim3(1), dim3(64), 0, s, ev->state);
  hipLaunchKernelGGL(k_zero, dim3((unsigned)std::min<int64_t>(4096, (a.n_tiles * 128 + 255) / 256)),
                     dim3(256), 0, s, ev->rowcol, a.n_tiles * 128);
  HIP_OK(hipGetLastError());
  return DOTPE_OK;
}

// fixed-order two-level reduction of the tile partials, then the sums of
// the squared intrinsic and extrinsic marginals (final_out[kNPart + 1, + 2]);
// the results and the state are copied to fo and st (host memory, read
// after the stream has been synchronised)
static int pass_tail(dotpe_event* ev, const FusedArgs& a, hipStream_t s, double* fo,
                     uint64_t* st) {
  const int prec = ev->bank->prec;
  const int64_t per = 4096;
  const int64_t nblk = (a.n_tiles + per - 1) / per;
  hipLaunchKernelGGL(k_finalize, dim3((unsigned)nblk), dim3(256), 0, s, ev->partials, a.n_tiles,
                     per, ev->final_blk);
  hipLaunchKernelGGL(k_finalize, dim3(1), dim3(256), 0, s, ev->final_blk, nblk, nblk,
                     ev->final_out);
  int tm, tn;
  tile_shape(prec, &tm, &tn);
  for (int rows = 1; rows >= 0; --rows) {
    const int64_t n_idx = rows ? ev->n_sub : ev->n_ext;
    const int64_t nb = (n_idx + 255) / 256;
    const int64_t n_other = rows ? a.n_tiles_n : a.n_tiles_m;
    const int64_t n_parts = (n_other + kMargPer - 1) / kMargPer;
    hipLaunchKernelGGL(k_marginal_part, dim3((unsigned)nb, (unsigned)n_parts), dim3(256), 0, s,
                       ev->partials, ev->rowcol, ev->final_out, a.n_tiles_m, a.n_tiles_n, tm, tn,
                       n_idx, rows, kMargPer, ev->marg_part);
    hipLaunchKernelGGL(k_marginal_sq, dim3((unsigned)nb), dim3(256), 0, s, ev->marg_part, n_parts,
                       n_idx, ev->marg_blk);
    hipLaunchKernelGGL(k_sum_blocks, dim3(1), dim3(256), 0, s, ev->marg_blk, nb,
                       ev->final_out + kNPart + (rows ? 1 : 2));
  }
  HIP_OK(hipGetLastError());
  HIP_OK(hipMemcpyAsync(fo, ev->final_out, sizeof(double) * (kNPart + 3), hipMemcpyDeviceToHost, s));
  HIP_OK(hipMemcpyAsync(st, ev->state, sizeof(uint64_t) * 6, hipMemcpyDeviceToHost, s));
  return DOTPE_OK;
}

// the pass's results from the reduced partials fo and the state st: fills
// *out except the top-k fields and the timings, and returns the raw
// candidate count in *n_cand
static void pass_results(const dotpe_event* ev, const FusedArgs& a, const double* fo,
                         const uint64_t* st, dotpe_evidence_result* out, uint64_t* n_cand) {
  const double cut_delta = a.cut_delta;
  double thr_frozen;
  std::memcpy(&thr_frozen, &st[3], 8);
  const bool cut = cut_delta > 0.0 && thr_frozen - cut_delta > 0.0;
  const double ln_norm = std::log(ev->n_norm) + std::log((double)ev->n_ext);
  dotpe_evidence_result r;
  std::memset(&r, 0, sizeof(r));
  r.ln_sum_p = fo[0] + std::log(fo[1]);
  r.ln_sum_p2 = 2.0 * fo[0] + std::log(fo[2]);
  r.ln_sum_p2_triples = 2.0 * fo[0] + std::log(fo[11]);
  r.ln_sum_row2 = 2.0 * fo[9] + std::log(fo[kNPart + 1]);
  r.ln_sum_col2 = 2.0 * fo[9] + std::log(fo[kNPart + 2]);
  r.ln_z = r.ln_sum_p - ln_norm;
  double ln_drop = (fo[3] == -INFINITY) ? -INFINITY : fo[3] + std::log(fo[4]);
  double mx = std::max(r.ln_sum_p, ln_drop);
  r.ln_z_upper = (mx == -INFINITY) ? -INFINITY
                                   : mx + std::log(std::exp(r.ln_sum_p - mx) + std::exp(ln_drop - mx)) - ln_norm;
  r.max_lnl_ml = fo[5];
  r.n_triples_marg = (int64_t)fo[6];
  r.n_pairs_bounded = (int64_t)fo[7];
  r.max_ln_p = fo[9];
  r.n_pairs = (int64_t)fo[10];
  r.dd = ev->dd;
  r.precision = ev->bank->prec;
  r.cut_delta_used = cut ? cut_delta : 0.0;
  // tiles of the coefficient route (all of them with the cut off), tiles
  // whose survivors the survivor pass evaluated
  r.n_tiles_rerun = (int32_t)(cut ? (int64_t)st[4] : a.n_tiles);
  r.n_tiles_listed = (int32_t)st[5];
  // no cut pair could have entered the top-k window
  const double thr = r.max_ln_p - ev->topk_window;
  r.topk_exact = ((int64_t)st[2] <= ev->cand_cap && !(fo[8] >= thr)) ? 1 : 0;
  *n_cand = st[2];
  *out = r;
}

// One evidence pass with cut `cut_delta` (<= 0: none), every decision taken
// on the device: pilot, then, if the threshold it freezes cuts, the bound
// pass (or the fused kernel's fast pass on small events) with the survivor
// pass; then the coefficient route over the tiles those leave (every tile
// when the cut is off), chunk by chunk; then the fixed-order finalisation.
// The host waits once, for the results.  Fills *out except the top-k
// fields and returns the raw candidate count in *n_cand.
static int evidence_pass(dotpe_ctx* ctx, dotpe_event* ev, double cut_delta,
                         dotpe_evidence_result* out, uint64_t* n_cand) {
  hipStream_t s = ev->stream;
  const int prec = ev->bank->prec;
  FusedArgs a = pass_args(ctx, ev, cut_delta);
  const PassPlan pl = pass_plan(ev, a);
  const bool timed = ev->ev_t[0] != nullptr;
  int rc;
  if ((rc = pass_head(ev, a, s))) return rc;
  if (timed) HIP_OK(hipEventRecord(ev->ev_t[0], s));
  // pilot: max lnL^ML over the pilot rows sets the cut threshold, frozen
  // before the main pass (so the cut does not depend on tile order)
  if (pl.may_cut && (rc = launch_fused<kPilot>(prec, a, pl.pilot_grid, s))) return rc;
  hipLaunchKernelGGL(k_freeze_threshold, dim3(1), dim3(64), 0, s, ev->state);
  if (timed) HIP_OK(hipEventRecord(ev->ev_t[1], s));
  if (pl.may_cut) {
    if (pl.bound_pass) {
      event_norms(ev, s);
      if ((rc = launch_fused<kBound>(prec, a, pl.cut_grid, s))) return rc;
      if (timed) HIP_OK(hipEventRecord(ev->ev_t[3], s));
      if ((rc = launch_fused<kSurvivors>(prec, a, pl.surv_grid, s))) return rc;
    } else {
      if ((rc = launch_fused<kEvidence, true>(prec, a, pl.cut_grid, s))) return rc;
      if (timed) HIP_OK(hipEventRecord(ev->ev_t[3], s));
    }
  } else if (timed) {
    HIP_OK(hipEventRecord(ev->ev_t[3], s));
  }
  for (int64_t c = 0; c < pl.n_chunks; ++c) {
    a.work0 = c * ev->coef_tiles;
    if ((rc = launch_fused<kCoef>(prec, a, pl.coef_grid, s))) return rc;
    if ((rc = launch_fused<kE2>(prec, a, pl.e2_grid, s))) return rc;
  }
  if (timed) HIP_OK(hipEventRecord(ev->ev_t[2], s));
  double fo[kNPart + 3];
  uint64_t st[6];
  if ((rc = pass_tail(ev, a, s, fo, st))) return rc;
  HIP_OK(hipStreamSynchronize(s));
  pass_results(ev, a, fo, st, out, n_cand);
  if (timed) {
    float t_pilot = 0.f, t_all = 0.f, t_first = 0.f;
    HIP_OK(hipEventElapsedTime(&t_pilot, ev->ev_t[0], ev->ev_t[1]));
    HIP_OK(hipEventElapsedTime(&t_all, ev->ev_t[1], ev->ev_t[2]));
    HIP_OK(hipEventElapsedTime(&t_first, ev->ev_t[1], ev->ev_t[3]));
    out->t_pilot_ms = t_pilot;
    out->t_fused_ms = t_all;
    out->t_main_ms = t_first;
  }
  return DOTPE_OK;
}

// Host and device buffers of packed passes (one set per serving slot): the
// events' arguments and, per event, its reduced results and state.
struct PackBufs {
  FusedArgs* h_args = nullptr;   // pinned host
  FusedArgs* d_args = nullptr;   // device
  double* h_fo = nullptr;        // pinned host [kMaxPack][kNPart + 3]
  uint64_t* h_st = nullptr;      // pinned host [kMaxPack][6]
};

// Packed launches of one pass for the events whose per-event grid (grids[k])
// is positive, kMaxPack events per launch at most: each event keeps its own
// grid, laid end to end at multiples of 8.  h_args: the events' arguments
// on the host (their pointers go into the launch's kernel arguments), d_args
// their device copy.
static int launch_packed_pass(int prec, int G, int mode, int n, const int64_t* grids, int64_t chunk,
                              const FusedArgs* h_args, const FusedArgs* d_args, int n_phi,
                              hipStream_t s) {
  PackedLaunchFn fn = packed_launcher(prec, G);
  if (!fn) return fail(DOTPE_E_INVALID_ARG, "bad precision %d or group count %d", prec, G);
  PackLaunch p;
  std::memset(&p, 0, sizeof(p));
  p.args = d_args;
  p.chunk = chunk;
  p.A0 = h_args[0].A0;
  p.A1 = h_args[0].A1;
  p.R0 = h_args[0].R0;
  p.R1 = h_args[0].R1;
  p.row_scale = h_args[0].row_scale;
  p.ln_w_bank = h_args[0].ln_w_bank;
  p.a_nrm = h_args[0].a_nrm;
  p.dist_tab = h_args[0].dist.tab;
  p.dist_prm = h_args[0].dist.prm;
  auto flush = [&]() -> int {
    if (p.n == 0) return DOTPE_OK;
    hipError_t e = fn(mode, p, n_phi, s);
    if (e != hipSuccess) return fail(DOTPE_E_DEVICE, "packed launch: %s", hipGetErrorString(e));
    p.n = 0;
    p.off[0] = 0;
    return DOTPE_OK;
  };
  for (int k = 0; k < n; ++k) {
    if (grids[k] <= 0) continue;
    if (p.off[p.n] + round_up(grids[k], 8) > (int64_t)INT32_MAX) {
      int rc = flush();
      if (rc) return rc;
    }
    const FusedArgs& a = h_args[k];
    PackPtrs& r = p.ptr[p.n];
    r.sub_idx = a.sub_idx;
    r.B0 = a.B0;
    r.B1 = a.B1;
    r.B2 = a.B2;
    r.B3 = a.B3;
    r.col_scale = a.col_scale;
    r.ln_w_ext = a.ln_w_ext;
    r.Ah0 = a.Ah0;
    r.Ah1 = a.Ah1;
    r.ah_scale = a.ah_scale;
    r.Bh0 = a.Bh0;
    r.Bh1 = a.Bh1;
    r.bh_scale = a.bh_scale;
    r.phase_cs = a.phase_cs;
    r.state = a.state;
    r.partials = a.partials;
    r.cand = a.cand;
    r.rerun = a.rerun;
    r.surv = a.surv;
    r.surv_list = a.surv_list;
    r.b_nrm = a.b_nrm;
    r.ah_nrm = a.ah_nrm;
    r.bh_nrm = a.bh_nrm;
    r.coef = a.coef;
    r.rowcol = a.rowcol;
    p.ev[p.n] = k;
    p.off[p.n + 1] = p.off[p.n] + round_up(grids[k], 8);
    if (++p.n == kMaxPack) {
      int rc = flush();
      if (rc) return rc;
    }
  }
  return flush();
}

// One evidence pass for n events at once (all on stream s, the same bank):
// the same kernels and per-event decisions as evidence_pass, each stage one
// packed launch over the events that take it, so the tiles of several events
// share the device; the host waits once for all of them.
static int evidence_pass_packed(dotpe_ctx* ctx, dotpe_event* const* evs, int n,
                                const double* deltas, PackBufs* pb, hipStream_t s,
                                dotpe_evidence_result* outs, uint64_t* n_cands) {
  if (n < 1 || n > kMaxPack) return fail(DOTPE_E_INVALID_ARG, "packed pass of %d events", n);
  const dotpe_bank* bk = evs[0]->bank;
  const int prec = bk->prec, G = bk->mt.G;
  std::vector<PassPlan> pl(n);
  int n_phi = 1;
  int64_t max_chunks = 0;
  for (int k = 0; k < n; ++k) {
    if (evs[k]->bank != bk) return fail(DOTPE_E_INVALID_ARG, "packed events of different banks");
    pb->h_args[k] = pass_args(ctx, evs[k], deltas[k]);
    pl[k] = pass_plan(evs[k], pb->h_args[k]);
    n_phi = std::max(n_phi, evs[k]->n_phi);
    max_chunks = std::max(max_chunks, pl[k].n_chunks);
  }
  HIP_OK(hipMemcpyAsync(pb->d_args, pb->h_args, sizeof(FusedArgs) * n, hipMemcpyHostToDevice, s));
  int rc;
  for (int k = 0; k < n; ++k) {
    if ((rc = pass_head(evs[k], pb->h_args[k], s))) return rc;
    if (pl[k].bound_pass) event_norms(evs[k], s);
  }
  std::vector<int64_t> g(n);
  auto stage = [&](int mode, int64_t chunk, auto grid_of) -> int {
    for (int k = 0; k < n; ++k) g[k] = grid_of(k);
    return launch_packed_pass(prec, G, mode, n, g.data(), chunk, pb->h_args, pb->d_args, n_phi, s);
  };
  if ((rc = stage(kPilot, 0, [&](int k) { return pl[k].pilot_grid; }))) return rc;
  for (int k = 0; k < n; ++k)
    hipLaunchKernelGGL(k_freeze_threshold, dim3(1), dim3(64), 0, s, evs[k]->state);
  if ((rc = stage(kBound, 0, [&](int k) { return pl[k].bound_pass ? pl[k].cut_grid : 0; })))
    return rc;
  if ((rc = stage(kSurvivors, 0, [&](int k) { return pl[k].surv_grid; }))) return rc;
  if ((rc = stage(kEvidence, 0,
                  [&](int k) { return pl[k].may_cut && !pl[k].bound_pass ? pl[k].cut_grid : 0; })))
    return rc;
  for (int64_t c = 0; c < max_chunks; ++c) {
    if ((rc = stage(kCoef, c, [&](int k) { return c < pl[k].n_chunks ? pl[k].coef_grid : 0; })))
      return rc;
    if ((rc = stage(kE2, c, [&](int k) { return c < pl[k].n_chunks ? pl[k].e2_grid : 0; })))
      return rc;
  }
  for (int k = 0; k < n; ++k)
    if ((rc = pass_tail(evs[k], pb->h_args[k], s, pb->h_fo + k * (kNPart + 3), pb->h_st + k * 6)))
      return rc;
  HIP_OK(hipStreamSynchronize(s));
  for (int k = 0; k < n; ++k)
    pass_results(evs[k], pb->h_args[k], pb->h_fo + k * (kNPart + 3), pb->h_st + k * 6, &outs[k],
                 &n_cands[k]);
  return DOTPE_OK;
}

// top-k among the candidates of the last pass within the window of the
// final maximum: bitonic sort of the candidate buffer on the device
static int evidence_topk(dotpe_event* ev, uint64_t n_cand_raw, dotpe_evidence_result* r,
                         dotpe_sample* topk) {
  hipStream_t s = ev->stream;
  const int64_t ncand = std::min<int64_t>((int64_t)n_cand_raw, ev->cand_cap);
  const double thr = r->max_ln_p - ev->topk_window;
  r->topk_count = 0;
  if (ev->top_k <= 0 || !topk || ncand <= 0) return DOTPE_OK;
  int64_t n2 = 1;
  while (n2 < ncand) n2 <<= 1;
  // the candidate buffer is a power of two at least as long as ncand
  if (n2 > ev->cand_cap) return fail(DOTPE_E_DEVICE, "top-k buffer too small");
  double* buf = ev->cand;
  if (n2 > ncand)
    hipLaunchKernelGGL(k_fill_cand, dim3((unsigned)((n2 - ncand + 255) / 256)), dim3(256), 0, s,
                       buf, ncand, n2);
  const int64_t take = std::min<int64_t>(ev->top_k, ncand);
  if (take <= kTopkChunk) {
    // sorted chunks, then pairwise merges keeping the best chunk of each pair
    const int C = (int)std::min<int64_t>(kTopkChunk, n2);
    const size_t lds = (size_t)C * 4 * sizeof(double);
    static std::once_flag attr_once;
    std::call_once(attr_once, [] {
      const int most = kTopkChunk * 4 * (int)sizeof(double);
      if (hipFuncSetAttribute((const void*)k_topk_chunks, hipFuncAttributeMaxDynamicSharedMemorySize,
                              most) != hipSuccess ||
          hipFuncSetAttribute((const void*)k_topk_merge, hipFuncAttributeMaxDynamicSharedMemorySize,
                              most) != hipSuccess)
        (void)hipGetLastError();
    });
    const int64_t n_chunks = n2 / C;
    hipLaunchKernelGGL(k_topk_chunks, dim3((unsigned)n_chunks), dim3(256), lds, s, buf, C);
    for (int64_t st = 1; st < n_chunks; st <<= 1)
      hipLaunchKernelGGL(k_topk_merge, dim3((unsigned)(n_chunks / (2 * st))), dim3(256), lds, s, buf,
                         C, st);
  } else {
    // a longer top-k: the whole buffer through the bitonic network
    for (int64_t k = 2; k <= n2; k <<= 1)
      for (int64_t j = k >> 1; j > 0; j >>= 1)
        hipLaunchKernelGGL(k_bitonic_step, dim3((unsigned)((n2 + 255) / 256)), dim3(256), 0, s,
                           buf, n2, j, k);
  }
  HIP_OK(hipGetLastError());
  std::vector<double> h(take * 4);
  HIP_OK(hipMemcpyAsync(h.data(), buf, take * 32, hipMemcpyDeviceToHost, s));
  HIP_OK(hipStreamSynchronize(s));
  int cnt = 0;
  for (int64_t q = 0; q < take; ++q) {
    if (!(h[4 * q] >= thr)) break;
    topk[cnt].ln_p = h[4 * q];
    topk[cnt].i = (int64_t)h[4 * q + 1];
    topk[cnt].e = (int64_t)h[4 * q + 2];
    topk[cnt].o_best = (int32_t)h[4 * q + 3];
    topk[cnt].reserved = 0;
    ++cnt;
  }
  r->topk_count = cnt;
  return DOTPE_OK;
}

// passes with a growing cut_delta until the certificate meets the target
static int evidence_run(dotpe_ctx* ctx, dotpe_event* ev, dotpe_evidence_result* out,
                        dotpe_sample* topk) {
  double delta = ev->cut_delta;
  dotpe_evidence_result r;
  uint64_t n_cand = 0;
  int passes = 0;
  for (;;) {
    int rc = evidence_pass(ctx, ev, delta, &r, &n_cand);
    if (rc) return rc;
    ++passes;
    if (!(delta > 0.0) || r.ln_z_upper - r.ln_z <= ev->cut_target) break;
    delta = passes < 3 ? delta + 20.0 : 0.0;    // cut less, finally not at all
  }
  r.n_passes = passes;
  int rc = evidence_topk(ev, n_cand, &r, topk);
  if (rc) return rc;
  ev->evaluated = true;
  ev->last_cut = r.cut_delta_used;
  ev->last_n_eff = std::exp(2.0 * r.ln_sum_p - r.ln_sum_p2_triples);
  r.status = DOTPE_OK;
  *out = r;
  return DOTPE_OK;
}

// evidence_run for n events of one bank on stream s, their passes packed:
// every event takes the passes it would take alone (a growing cut_delta
// until its certificate meets its target), the events still short of their
// target sharing each further pass; then each event's top-k.  rcs[k] is
// event k's status; the return value is nonzero only when the batch as a
// whole failed (then every event has that status).
static int evidence_run_packed(dotpe_ctx* ctx, dotpe_event* const* evs, int n, PackBufs* pb,
                               hipStream_t s, dotpe_evidence_result* outs,
                               dotpe_sample* const* topks, int* rcs) {
  std::vector<double> delta(n);
  std::vector<int> passes(n, 0);
  std::vector<uint64_t> n_cand(n, 0);
  std::vector<int> active(n);
  for (int k = 0; k < n; ++k) {
    delta[k] = evs[k]->cut_delta;
    active[k] = k;
    rcs[k] = DOTPE_OK;
  }
  std::vector<dotpe_event*> sub;
  std::vector<double> sub_delta;
  std::vector<dotpe_evidence_result> sub_out;
  std::vector<uint64_t> sub_cand;
  while (!active.empty()) {
    const int m = (int)active.size();
    sub.resize(m);
    sub_delta.resize(m);
    sub_out.resize(m);
    sub_cand.resize(m);
    for (int q = 0; q < m; ++q) {
      sub[q] = evs[active[q]];
      sub_delta[q] = delta[active[q]];
    }
    int rc = evidence_pass_packed(ctx, sub.data(), m, sub_delta.data(), pb, s, sub_out.data(),
                                  sub_cand.data());
    if (rc) {
      for (int k = 0; k < n; ++k) rcs[k] = rc;
      return rc;
    }
    std::vector<int> next;
    for (int q = 0; q < m; ++q) {
      const int k = active[q];
      outs[k] = sub_out[q];
      n_cand[k] = sub_cand[q];
      ++passes[k];
      const dotpe_evidence_result& r = sub_out[q];
      if (!(delta[k] > 0.0) || r.ln_z_upper - r.ln_z <= evs[k]->cut_target) continue;
      delta[k] = passes[k] < 3 ? delta[k] + 20.0 : 0.0;    // cut less, finally not at all
      next.push_back(k);
    }
    active.swap(next);
  }
  for (int k = 0; k < n; ++k) {
    dotpe_evidence_result& r = outs[k];
    r.n_passes = passes[k];
    int rc = evidence_topk(evs[k], n_cand[k], &r, topks[k]);
    if (rc) {
      rcs[k] = rc;
      continue;
    }
    evs[k]->evaluated = true;
    evs[k]->last_cut = r.cut_delta_used;
    evs[k]->last_n_eff = std::exp(2.0 * r.ln_sum_p - r.ln_sum_p2_triples);
    r.status = DOTPE_OK;
  }
  return DOTPE_OK;
}

int dotpe_evidence(dotpe_ctx* ctx, dotpe_event* ev, dotpe_evidence_result* out, dotpe_sample* topk) {
  if (!ctx || !ev || !out) return fail(DOTPE_E_INVALID_ARG, "NULL argument");
  HIP_OK(hipSetDevice(ctx->device));
  if (!ev->ev_t[0]) {
    HIP_OK(hipEventCreate(&ev->ev_t[0]));
    HIP_OK(hipEventCreate(&ev->ev_t[1]));
    HIP_OK(hipEventCreate(&ev->ev_t[2]));
    HIP_OK(hipEventCreate(&ev->ev_t[3]));
  }
  return evidence_run(ctx, ev, out, topk);
}

int dotpe_evidence_static(dotpe_ctx* ctx, const dotpe_bank* bk, const dotpe_event_desc* d,
                          dotpe_evidence_result* out, dotpe_sample* topk) {
  if (!ctx || !bk || !d || !out) return fail(DOTPE_E_INVALID_ARG, "NULL argument");
  if (ctx->device >= kScratchDevices || !g_scratch[ctx->device].ptr)
    return fail(DOTPE_E_UNIMPLEMENTED, "no device scratch on device %d", ctx->device);
  EvDims D;
  std::vector<int> terms;
  int rc = event_dims(bk, d, &D, &terms);
  if (rc) return rc;
  // the coefficient route's buffer takes what the rest leaves (at least
  // one tile; its size per tile is a multiple of the block alignment)
  uint64_t need;
  {
    dotpe_event probe;
    EvStage st;
    EvDims E = D;
    E.coef_tiles = 1;
    need = block_bytes(event_buffers(E, &probe, &st));
  }
  if (need > kScratchBytes)
    return fail(DOTPE_E_TOO_LARGE,
                "event needs %llu bytes of device scratch; dotpe_evidence_static holds %llu",
                (unsigned long long)need, (unsigned long long)kScratchBytes);
  const uint64_t coef_cap = (kScratchBytes - need) / D.coef_tile_bytes * D.coef_tile_bytes +
                            D.coef_tile_bytes;
  HIP_OK(hipSetDevice(ctx->device));
  ScratchSlot& slot = g_scratch[ctx->device];
  std::lock_guard<std::mutex> lk(slot.mu);
  dotpe_event* ev = nullptr;
  rc = set_event_impl(ctx, bk, d, (char*)slot.ptr, kScratchBytes,
                      d->stream ? (hipStream_t)d->stream : ctx->stream, &ev, coef_cap);
  if (rc) return rc;
  dotpe_evidence_result r;
  rc = evidence_run(ctx, ev, &r, topk);     // untimed: the event has no HIP events
  dotpe_free_event(ctx, ev);                // frees nothing: every buffer is in the scratch
  if (rc) return rc;
  *out = r;
  return DOTPE_OK;
}

int dotpe_preselect(dotpe_ctx* ctx, const dotpe_bank* bk, const dotpe_preselect_desc* d,
                    double* lnl_inco, double* lnl_det, int64_t* selected,
                    dotpe_preselect_result* out) {
  if (!ctx || !bk || !d || !out) return fail(DOTPE_E_INVALID_ARG, "NULL argument");
  if (bk->prec == kFP64)
    return fail(DOTPE_E_UNIMPLEMENTED, "pre-selection runs on split-precision banks only");
  if (bk->mt.layout != 0)
    return fail(DOTPE_E_UNIMPLEMENTED, "pre-selection forms polarisations from (l, m) channels");
  if (d->n_det < 1 || d->n_det > kMaxDet) return fail(DOTPE_E_INVALID_ARG, "n_det=%d", d->n_det);
  if (d->n_t < 32 || d->n_t > kPreMaxT || d->n_t % 32)
    return fail(DOTPE_E_INVALID_ARG, "n_t=%d (32, 64, 96 or 128)", d->n_t);
  if (d->n_phi < 1 || d->n_phi > kMaxPhi) return fail(DOTPE_E_INVALID_ARG, "n_phi=%d", d->n_phi);
  if (!d->d || !d->w || !d->t0 || !d->cos_iota)
    return fail(DOTPE_E_INVALID_ARG, "pre-selection arrays must not be NULL");
  const int64_t n_rows = d->sub_count > 0 ? d->sub_count : bk->n_wf;
  if (d->sub_start < 0 || d->sub_start + n_rows > bk->n_wf)
    return fail(DOTPE_E_INVALID_ARG, "bank range out of bounds");
  const int nk = d->n_det, nb = bk->n_b;
  if (!finite_all(d->d, (size_t)nk * nb * 2) || !finite_all(d->w, (size_t)nk * nb) ||
      !finite_all(d->t0, nk) || !std::isfinite(d->dt) || !finite_all(d->cos_iota, n_rows))
    return fail(DOTPE_E_NUMERIC, "non-finite pre-selection input");
  for (int64_t r = 0; r < n_rows; ++r)
    if (std::fabs(d->cos_iota[r]) > 1.0) return fail(DOTPE_E_INVALID_ARG, "|cos_iota| > 1");
  for (size_t t = 0; t < (size_t)nk * nb; ++t)
    if (d->w[t] < 0.0) return fail(DOTPE_E_INVALID_ARG, "negative noise weight");
  HIP_OK(hipSetDevice(ctx->device));
  hipStream_t s = d->stream ? (hipStream_t)d->stream : ctx->stream;
  const ModeTables& mt = bk->mt;
  PreArgs a;
  std::memset(&a, 0, sizeof(a));
  a.A0 = bk->A0;
  a.A1 = bk->A1;
  a.R0 = bk->R0;
  a.R1 = bk->R1;
  a.row_scale = bk->row_scale;
  a.K2 = bk->K2;
  a.n_c = mt.n_c;
  a.n_b = nb;
  a.n_bp = bk->n_bp;
  for (int c = 0; c < mt.n_c; ++c) {
    a.l[c] = mt.l[c];
    a.m[c] = mt.m[c];
    for (int g = 0; g < mt.G; ++g)
      if (mt.gm[g] == mt.m[c]) a.cg[c] = g;
  }
  for (int g = 0; g < mt.G; ++g) a.gm[g] = mt.gm[g];
  a.G = mt.G;
  a.row0 = d->sub_start;
  a.n_rows = n_rows;
  a.n_det = nk;
  a.n_t = d->n_t;
  a.n_phi = d->n_phi;
  a.f = bk->f;
  a.dt = d->dt;
  a.K2p = 2 * (int64_t)bk->n_bp;
  a.delta = d->delta_lnl > 0.0 ? d->delta_lnl : 20.0;
  const int64_t n_grid = (int64_t)nk * d->n_t;
  const int64_t nblk = (n_rows + 1023) / 1024;
  const int64_t n_chunk = std::min<int64_t>(n_rows, kPreChunk);
  // the pass's buffers, freed on every return below
  std::vector<void*> bufs;
  uint64_t held = 0;
  struct Release {
    dotpe_ctx* ctx;
    std::vector<void*>* bufs;
    uint64_t* held;
    hipStream_t s;
    ~Release() {
      (void)hipStreamSynchronize(s);
      for (void* p : *bufs) (void)hipFree(p);
      ctx->bytes -= *held;
    }
  } release{ctx, &bufs, &held, s};
  int rc;
  auto alloc = [&](void** p, size_t n) { return dev_alloc(ctx, p, n, &bufs, &held); };
  void *dd = nullptr, *ww = nullptr, *tt = nullptr, *ci = nullptr, *st = nullptr;
  if ((rc = alloc(&dd, (size_t)nk * nb * 16)) || (rc = alloc(&ww, (size_t)nk * nb * 8)) ||
      (rc = alloc(&tt, (size_t)nk * 8)) || (rc = alloc(&ci, (size_t)n_rows * 8)) ||
      (rc = alloc((void**)&a.B0, (size_t)n_grid * a.K2p * 2)) ||
      (rc = alloc((void**)&a.B1, (size_t)n_grid * a.K2p * 2)) ||
      (rc = alloc((void**)&a.col_scale, (size_t)n_grid * 8)) ||
      (rc = alloc((void**)&a.gram, (size_t)n_chunk * nk * pre_pairs(mt.n_c) * 16)) ||
      (rc = alloc((void**)&a.ml_det, (size_t)n_rows * nk * 8)) ||
      (rc = alloc((void**)&a.lnl, (size_t)n_rows * 8)) || (rc = alloc(&st, 64)) ||
      (rc = alloc((void**)&a.counts, (size_t)nblk * 4)) ||
      (rc = alloc((void**)&a.offsets, (size_t)nblk * 8)) ||
      (rc = alloc((void**)&a.selected, (size_t)n_rows * 8)))
    return rc;
  a.d = (const double2*)dd;
  a.w = (const double*)ww;
  a.t0 = (const double*)tt;
  a.cos_iota = (const double*)ci;
  a.state = (uint64_t*)st;
  const uint64_t st0[2] = {0x000fffffffffffffull, 0ull};   // below every ordered value; count
  HIP_OK(hipMemcpyAsync(dd, d->d, (size_t)nk * nb * 16, hipMemcpyHostToDevice, s));
  HIP_OK(hipMemcpyAsync(ww, d->w, (size_t)nk * nb * 8, hipMemcpyHostToDevice, s));
  HIP_OK(hipMemcpyAsync(tt, d->t0, (size_t)nk * 8, hipMemcpyHostToDevice, s));
  HIP_OK(hipMemcpyAsync(ci, d->cos_iota, (size_t)n_rows * 8, hipMemcpyHostToDevice, s));
  HIP_OK(hipMemcpyAsync(st, st0, sizeof(st0), hipMemcpyHostToDevice, s));
  hipEvent_t e0, e1;
  HIP_OK(hipEventCreate(&e0));
  HIP_OK(hipEventCreate(&e1));
  struct Events {
    hipEvent_t a, b;
    ~Events() {
      (void)hipEventDestroy(a);
      (void)hipEventDestroy(b);
    }
  } evs{e0, e1};
  HIP_OK(hipEventRecord(e0, s));
  hipError_t e = preselect_launch(bk->prec, a, s);
  if (e != hipSuccess) return fail(DOTPE_E_DEVICE, "pre-selection launch: %s", hipGetErrorString(e));
  HIP_OK(hipEventRecord(e1, s));
  uint64_t sth[2];
  HIP_OK(hipMemcpyAsync(sth, st, sizeof(sth), hipMemcpyDeviceToHost, s));
  HIP_OK(hipStreamSynchronize(s));
  const int64_t n_sel = (int64_t)sth[1];
  if (lnl_inco) HIP_OK(hipMemcpyAsync(lnl_inco, a.lnl, (size_t)n_rows * 8, hipMemcpyDeviceToHost, s));
  if (lnl_det) HIP_OK(hipMemcpyAsync(lnl_det, a.ml_det, (size_t)n_rows * nk * 8, hipMemcpyDeviceToHost, s));
  if (selected && n_sel > 0)
    HIP_OK(hipMemcpyAsync(selected, a.selected, (size_t)n_sel * 8, hipMemcpyDeviceToHost, s));
  HIP_OK(hipStreamSynchronize(s));
  float ms = 0.f;
  HIP_OK(hipEventElapsedTime(&ms, e0, e1));
  uint64_t u = sth[0];
  u = (u & 0x8000000000000000ull) ? (u & 0x7fffffffffffffffull) : ~u;
  double mx;
  std::memcpy(&mx, &u, 8);
  dotpe_preselect_result r;
  std::memset(&r, 0, sizeof(r));
  r.lnl_max = mx;
  r.threshold = mx - a.delta;
  r.n_rows = n_rows;
  r.n_selected = n_sel;
  r.t_ms = ms;
  *out = r;
  return DOTPE_OK;
}

// Doubles of workspace scan_inclusive needs for n values: the block totals
// of every level.
static int64_t scan_tmp_size(int64_t n) {
  int64_t t = 0;
  for (int64_t nb = (n + 1023) / 1024; nb > 1; nb = (nb + 1023) / 1024) t += nb;
  return t + 1;
}

// Inclusive running sum of x[0, n) in place on stream s (tmp: scan_tmp_size(n)
// doubles): blocks of 1024 scanned, their totals scanned the same way one
// level up, the totals before each block added.
static void scan_inclusive(double* x, int64_t n, double* tmp, hipStream_t s) {
  const int64_t nb = (n + 1023) / 1024;
  hipLaunchKernelGGL(k_scan_block, dim3((unsigned)nb), dim3(1024), 0, s, x, n, tmp);
  if (nb > 1) {
    scan_inclusive(tmp, nb, tmp + nb, s);
    hipLaunchKernelGGL(k_scan_add, dim3((unsigned)nb), dim3(1024), 0, s, x, n, (const double*)tmp);
  }
}

int dotpe_sample_posterior(dotpe_ctx* ctx, dotpe_event* ev, int64_t n_samples, double u0,
                           uint64_t seed, dotpe_posterior_sample* out, int64_t capacity,
                           int64_t* n_out) {
  if (!ctx || !ev || !out || !n_out) return fail(DOTPE_E_INVALID_ARG, "NULL argument");
  if (!ev->evaluated) return fail(DOTPE_E_INVALID_ARG, "call dotpe_evidence on the event first");
  if (!(u0 >= 0.0 && u0 < 1.0)) return fail(DOTPE_E_INVALID_ARG, "u0 must lie in [0, 1)");
  if (capacity < 1) return fail(DOTPE_E_INVALID_ARG, "capacity must be positive");
  int64_t ns = n_samples > 0 ? n_samples : (int64_t)std::floor(0.5 * ev->last_n_eff);
  ns = std::max<int64_t>(1, std::min(ns, capacity));
  HIP_OK(hipSetDevice(ctx->device));
  hipStream_t s = ev->stream;
  const int prec = ev->bank->prec;
  FusedArgs a = make_args(ctx, ev);
  a.cut_delta = ev->last_cut;
  a.state = ev->state;
  a.partials = ev->partials;
  a.final_out = ev->final_out;
  a.d0 = ev->d0;
  a.seed = seed;
  std::vector<void*> bufs;
  uint64_t held = 0;
  struct Release {
    dotpe_ctx* ctx;
    std::vector<void*>* bufs;
    uint64_t* held;
    hipStream_t s;
    ~Release() {
      (void)hipStreamSynchronize(s);
      for (void* p : *bufs) (void)hipFree(p);
      ctx->bytes -= *held;
    }
  } release{ctx, &bufs, &held, s};
  auto alloc = [&](void** p, size_t n) { return dev_alloc(ctx, p, n, &bufs, &held); };
  const int64_t nt = a.n_tiles, nb = scan_tmp_size(nt);
  double *cum = nullptr, *blk = nullptr, *res = nullptr, *smp = nullptr;
  int *tile = nullptr, *list = nullptr;
  int64_t *first = nullptr, *n_u_dev = nullptr;
  int rc;
  if ((rc = alloc((void**)&cum, (size_t)nt * 8)) || (rc = alloc((void**)&blk, (size_t)nb * 8)) ||
      (rc = alloc((void**)&tile, (size_t)ns * 4)) || (rc = alloc((void**)&res, (size_t)ns * 8)) ||
      (rc = alloc((void**)&list, (size_t)ns * 4)) || (rc = alloc((void**)&first, (size_t)(ns + 1) * 8)) ||
      (rc = alloc((void**)&n_u_dev, 8)) || (rc = alloc((void**)&smp, (size_t)ns * 6 * 8)))
    return rc;
  hipLaunchKernelGGL(k_tile_mass, dim3((unsigned)((nt + 255) / 256)), dim3(256), 0, s, ev->partials,
                     ev->final_out, nt, cum);
  scan_inclusive(cum, nt, blk, s);
  hipLaunchKernelGGL(k_place_draws, dim3((unsigned)((ns + 255) / 256)), dim3(256), 0, s, cum, nt, ns,
                     u0, tile, res);
  hipLaunchKernelGGL(k_group_draws, dim3(1), dim3(64), 0, s, tile, ns, list, first, n_u_dev);
  HIP_OK(hipGetLastError());
  int64_t n_u = 0;
  HIP_OK(hipMemcpyAsync(&n_u, n_u_dev, 8, hipMemcpyDeviceToHost, s));
  HIP_OK(hipStreamSynchronize(s));
  a.work_list = list;
  a.n_work_list = n_u;
  a.sample_first = first;
  a.sample_res = res;
  a.samples = smp;
  const int64_t C = ev->coef_tiles;
  for (int64_t c = 0; c * C < n_u; ++c) {
    a.work0 = c * C;
    if ((rc = launch_fused<kCoef>(prec, a, std::min(C, kCoefGrid), s))) return rc;
    if ((rc = launch_fused<kSample>(prec, a, std::min(C, kE2Grid), s))) return rc;
  }
  std::vector<double> h((size_t)ns * 6);
  HIP_OK(hipMemcpyAsync(h.data(), smp, (size_t)ns * 6 * 8, hipMemcpyDeviceToHost, s));
  HIP_OK(hipStreamSynchronize(s));
  for (int64_t q = 0; q < ns; ++q) {
    dotpe_posterior_sample& o = out[q];
    o.i = (int64_t)h[6 * q];
    o.e = (int64_t)h[6 * q + 1];
    o.o = (int32_t)h[6 * q + 2];
    o.reserved = 0;
    o.distance = h[6 * q + 3];
    o.ln_p_pair = h[6 * q + 4];
    o.ln_p_triple = h[6 * q + 5];
  }
  *n_out = ns;
  return DOTPE_OK;
}

int dotpe_debug_distmarg(dotpe_ctx* ctx, int64_t n, const double* dh, const double* hh,
                         double r0, double* out) {
  if (!ctx || n < 0 || (n > 0 && (!dh || !hh || !out))) return fail(DOTPE_E_INVALID_ARG, "bad args");
  if (n == 0) return DOTPE_OK;
  HIP_OK(hipSetDevice(ctx->device));
  double* buf = nullptr;
  std::vector<void*> tmp;
  uint64_t tb = 0;
  int rc;
  if ((rc = dev_alloc(ctx, (void**)&buf, (size_t)n * 24, &tmp, &tb))) return rc;
  hipStream_t s = ctx->stream;
  DistArgs da;
  da.tab = ctx->dist_tab;
  da.prm = ctx->dist_prm;
  hipError_t e = hipMemcpyAsync(buf, dh, n * 8, hipMemcpyHostToDevice, s);
  if (!e) e = hipMemcpyAsync(buf + n, hh, n * 8, hipMemcpyHostToDevice, s);
  if (!e) {
    hipLaunchKernelGGL(k_debug_distmarg, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, n, buf,
                       buf + n, r0, da, buf + 2 * n);
    e = hipGetLastError();
  }
  if (!e) e = hipMemcpyAsync(out, buf + 2 * n, n * 8, hipMemcpyDeviceToHost, s);
  if (!e) e = hipStreamSynchronize(s);
  (void)hipFree(buf);
  ctx->bytes -= tb;
  if (e) return fail(DOTPE_E_DEVICE, "debug_distmarg: %s", hipGetErrorString(e));
  return DOTPE_OK;
}

int dotpe_extrinsic_samples(dotpe_ctx* ctx, const dotpe_bank* bk, const dotpe_extrinsic_desc* d,
                            double* lat, double* lon, double* psi, double* cos_iota, double* t_geo,
                            double* ln_w, dotpe_extrinsic_result* out) {
  if (!ctx || !bk || !d || !out) return fail(DOTPE_E_INVALID_ARG, "NULL argument");
  if (bk->prec == kFP64 || bk->mt.layout != 0)
    return fail(DOTPE_E_UNIMPLEMENTED,
                "arrival-time series come from the pre-selection: split-precision (l, m) banks only");
  if (d->n_det < 1 || d->n_det > kMaxDet) return fail(DOTPE_E_INVALID_ARG, "n_det=%d", d->n_det);
  if (d->n_t < 32 || d->n_t > kPreMaxT || d->n_t % 32)
    return fail(DOTPE_E_INVALID_ARG, "n_t=%d (32, 64, 96 or 128)", d->n_t);
  if (d->n_phi < 1 || d->n_phi > kMaxPhi) return fail(DOTPE_E_INVALID_ARG, "n_phi=%d", d->n_phi);
  if (d->n_rows < 1 || d->n_rows > 64) return fail(DOTPE_E_INVALID_ARG, "n_rows=%d", d->n_rows);
  if (d->n_sky < 1 || d->n_sky > 65536 || d->n_tg < 1 || d->n_tg > 4096 || d->n_samples < 1)
    return fail(DOTPE_E_INVALID_ARG, "n_sky=%d n_tg=%d n_samples=%lld", d->n_sky, d->n_tg,
                (long long)d->n_samples);
  const int64_t SJ = (int64_t)d->n_sky * d->n_tg, CSJ = SJ * d->n_rows;
  if (CSJ > (int64_t(1) << 26)) return fail(DOTPE_E_INVALID_ARG, "n_rows x n_sky x n_tg > 2^26");
  if (!d->d || !d->w || !d->det_r || !d->t0 || !d->rows || !d->cos_iota)
    return fail(DOTPE_E_INVALID_ARG, "extrinsic-sample arrays must not be NULL");
  const int nk = d->n_det, nb = bk->n_b, C = d->n_rows;
  if (!finite_all(d->d, (size_t)nk * nb * 2) || !finite_all(d->w, (size_t)nk * nb) ||
      !finite_all(d->det_r, (size_t)nk * 3) || !finite_all(d->t0, nk) || !std::isfinite(d->dt) ||
      !finite_all(d->cos_iota, C) || !std::isfinite(d->tg_lo) || !std::isfinite(d->tg_hi) ||
      !std::isfinite(d->beta))
    return fail(DOTPE_E_NUMERIC, "non-finite extrinsic-sample input");
  if (!(d->dt > 0.0) || !(d->tg_hi > d->tg_lo))
    return fail(DOTPE_E_INVALID_ARG, "dt and the geocentre-time window must be positive");
  for (int c = 0; c < C; ++c) {
    if (d->rows[c] < 0 || d->rows[c] >= bk->n_wf) return fail(DOTPE_E_INVALID_ARG, "row out of range");
    if (std::fabs(d->cos_iota[c]) > 1.0) return fail(DOTPE_E_INVALID_ARG, "|cos_iota| > 1");
  }
  for (size_t t = 0; t < (size_t)nk * nb; ++t)
    if (d->w[t] < 0.0) return fail(DOTPE_E_INVALID_ARG, "negative noise weight");
  HIP_OK(hipSetDevice(ctx->device));
  hipStream_t s = d->stream ? (hipStream_t)d->stream : ctx->stream;
  const ModeTables& mt = bk->mt;
  // the pre-selection's products, one intrinsic sample at a time, keeping
  // each detector's per-time maxima
  PreArgs a;
  std::memset(&a, 0, sizeof(a));
  a.A0 = bk->A0;
  a.A1 = bk->A1;
  a.R0 = bk->R0;
  a.R1 = bk->R1;
  a.row_scale = bk->row_scale;
  a.K2 = bk->K2;
  a.n_c = mt.n_c;
  a.n_b = nb;
  a.n_bp = bk->n_bp;
  for (int c = 0; c < mt.n_c; ++c) {
    a.l[c] = mt.l[c];
    a.m[c] = mt.m[c];
    for (int g = 0; g < mt.G; ++g)
      if (mt.gm[g] == mt.m[c]) a.cg[c] = g;
  }
  for (int g = 0; g < mt.G; ++g) a.gm[g] = mt.gm[g];
  a.G = mt.G;
  a.n_rows = 1;
  a.n_det = nk;
  a.n_t = d->n_t;
  a.n_phi = d->n_phi;
  a.f = bk->f;
  a.dt = d->dt;
  a.K2p = 2 * (int64_t)bk->n_bp;
  a.delta = 20.0;
  const int64_t n_grid = (int64_t)nk * d->n_t;
  std::vector<void*> bufs;
  uint64_t held = 0;
  struct Release {
    dotpe_ctx* ctx;
    std::vector<void*>* bufs;
    uint64_t* held;
    hipStream_t s;
    ~Release() {
      (void)hipStreamSynchronize(s);
      for (void* p : *bufs) (void)hipFree(p);
      ctx->bytes -= *held;
    }
  } release{ctx, &bufs, &held, s};
  int rc;
  auto alloc = [&](void** p, size_t n) { return dev_alloc(ctx, p, n, &bufs, &held); };
  void *dd = nullptr, *ww = nullptr, *tt = nullptr, *ci = nullptr, *st = nullptr;
  double *ml = nullptr, *rmax = nullptr, *tab = nullptr, *lnZ = nullptr, *mix = nullptr,
         *blk = nullptr, *draws = nullptr, *stats = nullptr, *lse_part = nullptr;
  unsigned long long* n_supp = nullptr;
  const int64_t nblk = scan_tmp_size(CSJ);
  if ((rc = alloc(&dd, (size_t)nk * nb * 16)) || (rc = alloc(&ww, (size_t)nk * nb * 8)) ||
      (rc = alloc(&tt, (size_t)nk * 8)) || (rc = alloc(&ci, (size_t)C * 8)) ||
      (rc = alloc((void**)&a.B0, (size_t)n_grid * a.K2p * 2)) ||
      (rc = alloc((void**)&a.B1, (size_t)n_grid * a.K2p * 2)) ||
      (rc = alloc((void**)&a.col_scale, (size_t)n_grid * 8)) ||
      (rc = alloc((void**)&a.gram, (size_t)nk * pre_pairs(mt.n_c) * 16)) ||
      (rc = alloc((void**)&a.ml_det, (size_t)nk * 8)) || (rc = alloc((void**)&a.lnl, 8)) ||
      (rc = alloc(&st, 64)) || (rc = alloc((void**)&a.counts, 4)) ||
      (rc = alloc((void**)&a.offsets, 8)) || (rc = alloc((void**)&a.selected, 8)) ||
      (rc = alloc((void**)&ml, (size_t)C * n_grid * 8)) ||
      (rc = alloc((void**)&rmax, (size_t)C * nk * 8)) ||
      (rc = alloc((void**)&tab, (size_t)CSJ * 8)) || (rc = alloc((void**)&lnZ, (size_t)C * 8)) ||
      (rc = alloc((void**)&mix, (size_t)SJ * 8)) || (rc = alloc((void**)&blk, (size_t)nblk * 8)) ||
      (rc = alloc((void**)&draws, (size_t)d->n_samples * 7 * 8)) ||
      (rc = alloc((void**)&stats, 16)) ||
      (rc = alloc((void**)&lse_part, (size_t)C * kPropParts * 16)) ||
      (rc = alloc((void**)&n_supp, 8)))
    return rc;
  a.d = (const double2*)dd;
  a.w = (const double*)ww;
  a.t0 = (const double*)tt;
  a.state = (uint64_t*)st;
  HIP_OK(hipMemcpyAsync(dd, d->d, (size_t)nk * nb * 16, hipMemcpyHostToDevice, s));
  HIP_OK(hipMemcpyAsync(ww, d->w, (size_t)nk * nb * 8, hipMemcpyHostToDevice, s));
  HIP_OK(hipMemcpyAsync(tt, d->t0, (size_t)nk * 8, hipMemcpyHostToDevice, s));
  HIP_OK(hipMemcpyAsync(ci, d->cos_iota, (size_t)C * 8, hipMemcpyHostToDevice, s));
  hipEvent_t e0, e1;
  HIP_OK(hipEventCreate(&e0));
  HIP_OK(hipEventCreate(&e1));
  struct Events {
    hipEvent_t a, b;
    ~Events() {
      (void)hipEventDestroy(a);
      (void)hipEventDestroy(b);
    }
  } evs{e0, e1};
  HIP_OK(hipEventRecord(e0, s));
  const uint64_t st0[2] = {0x000fffffffffffffull, 0ull};
  for (int c = 0; c < C; ++c) {
    HIP_OK(hipMemcpyAsync(st, st0, sizeof(st0), hipMemcpyHostToDevice, s));
    a.row0 = d->rows[c];
    a.cos_iota = (const double*)ci + c;
    a.ml_t = ml + (size_t)c * n_grid;
    hipError_t e = preselect_launch(bk->prec, a, s);
    if (e != hipSuccess) return fail(DOTPE_E_DEVICE, "arrival-time series: %s", hipGetErrorString(e));
  }
  // the proposals over (sky, geocentre-time) cells, their mixture, the draws
  PropGeom g;
  std::memset(&g, 0, sizeof(g));
  g.C = C;
  g.S = d->n_sky;
  g.J = d->n_tg;
  g.K = nk;
  g.n_t = d->n_t;
  for (int k = 0; k < nk; ++k) {
    g.t0[k] = d->t0[k];
    for (int q = 0; q < 3; ++q) g.r[k][q] = d->det_r[3 * k + q];
  }
  g.dt = d->dt;
  g.tg_lo = d->tg_lo;
  g.dtg = (d->tg_hi - d->tg_lo) / d->n_tg;
  g.beta = d->beta > 0.0 ? d->beta : 0.5;
  hipLaunchKernelGGL(k_prop_max, dim3((unsigned)((C * nk + 63) / 64)), dim3(64), 0, s, ml, g, rmax);
  hipLaunchKernelGGL(k_prop_table, dim3((unsigned)((CSJ + 255) / 256)), dim3(256), 0, s, ml, rmax, g,
                     tab);
  hipLaunchKernelGGL(k_prop_lse_part, dim3((unsigned)kPropParts, (unsigned)C), dim3(256), 0, s, tab,
                     g, lse_part);
  hipLaunchKernelGGL(k_prop_lse, dim3((unsigned)C), dim3(256), 0, s, (const double*)lse_part, lnZ);
  hipLaunchKernelGGL(k_prop_prob, dim3((unsigned)((SJ + 255) / 256)), dim3(256), 0, s, tab, lnZ, g,
                     mix);
  scan_inclusive(tab, CSJ, blk, s);
  hipLaunchKernelGGL(k_prop_draw, dim3((unsigned)((d->n_samples + 255) / 256)), dim3(256), 0, s,
                     (const double*)tab, (const double*)mix, g, d->n_samples, d->seed, draws);
  HIP_OK(hipMemsetAsync(n_supp, 0, 8, s));
  hipLaunchKernelGGL(k_count_support, dim3((unsigned)((SJ + 255) / 256)), dim3(256), 0, s,
                     (const double*)mix, SJ, n_supp);
  hipLaunchKernelGGL(k_prop_stats, dim3(1), dim3(256), 0, s, (const double*)draws, d->n_samples,
                     (const unsigned long long*)n_supp, SJ, stats);
  HIP_OK(hipGetLastError());
  HIP_OK(hipEventRecord(e1, s));
  std::vector<double> h((size_t)d->n_samples * 7);
  double sth[2];
  HIP_OK(hipMemcpyAsync(h.data(), draws, h.size() * 8, hipMemcpyDeviceToHost, s));
  HIP_OK(hipMemcpyAsync(sth, stats, 16, hipMemcpyDeviceToHost, s));
  HIP_OK(hipStreamSynchronize(s));
  double* outs[6] = {lat, lon, psi, cos_iota, t_geo, ln_w};
  for (int f = 0; f < 6; ++f)
    if (outs[f])
      for (int64_t q = 0; q < d->n_samples; ++q) outs[f][q] = h[(size_t)q * 7 + f];
  float ms = 0.f;
  HIP_OK(hipEventElapsedTime(&ms, e0, e1));
  dotpe_extrinsic_result r;
  std::memset(&r, 0, sizeof(r));
  r.n_eff_prior = sth[0];
  r.support = sth[1];
  r.t_ms = ms;
  r.n_samples = d->n_samples;
  *out = r;
  return DOTPE_OK;
}

int dotpe_rb_weights(dotpe_ctx* ctx, const dotpe_rb_desc* d, double* w_dh, double* w_hh,
                     double* dd) {
  if (!ctx || !d) return fail(DOTPE_E_INVALID_ARG, "NULL argument");
  if (d->n_det < 1 || d->n_det > kMaxDet) return fail(DOTPE_E_INVALID_ARG, "n_det=%d", d->n_det);
  if (d->n_modes < 1 || d->n_modes > kMaxC) return fail(DOTPE_E_INVALID_ARG, "n_modes=%d", d->n_modes);
  if (d->n_full < 2 || d->n_full > (int64_t(1) << 26) || d->n_nodes < 2 || d->n_nodes > 4096 ||
      d->reserved)
    return fail(DOTPE_E_INVALID_ARG, "n_full=%lld n_nodes=%d", (long long)d->n_full, d->n_nodes);
  if (!d->f || !d->d || !d->w || !d->h0 || !d->node_idx)
    return fail(DOTPE_E_INVALID_ARG, "relative-binning arrays must not be NULL");
  const int nk = d->n_det, nc = d->n_modes, nn = d->n_nodes;
  const int64_t nf = d->n_full;
  for (int b = 0; b < nn; ++b)
    if (d->node_idx[b] < 0 || d->node_idx[b] >= nf || (b > 0 && d->node_idx[b] <= d->node_idx[b - 1]))
      return fail(DOTPE_E_INVALID_ARG, "node_idx must rise strictly within the grid");
  for (int64_t q = 1; q < nf; ++q)
    if (!(d->f[q] > d->f[q - 1])) return fail(DOTPE_E_INVALID_ARG, "f must rise strictly");
  if (!finite_all(d->f, nf) || !finite_all(d->d, (size_t)nk * nf * 2) ||
      !finite_all(d->w, (size_t)nk * nf) || !finite_all(d->h0, (size_t)nc * nf * 2) ||
      (d->t0 && !finite_all(d->t0, nk)))
    return fail(DOTPE_E_NUMERIC, "non-finite relative-binning input");
  for (int c = 0; c < nc; ++c)
    for (int b = 0; b < nn; ++b) {
      const double* v = d->h0 + ((size_t)c * nf + d->node_idx[b]) * 2;
      if (v[0] == 0.0 && v[1] == 0.0)
        return fail(DOTPE_E_NUMERIC, "reference channel %d is zero at node %d", c, b);
    }
  HIP_OK(hipSetDevice(ctx->device));
  hipStream_t s = ctx->stream;
  std::vector<void*> owned;
  uint64_t acct = 0;
  double *f = nullptr, *w = nullptr, *t0 = nullptr;
  double2 *dv = nullptr, *h0 = nullptr, *wdh = nullptr, *whh = nullptr;
  int64_t* idx = nullptr;
  double* ddv = nullptr;
  const size_t n_dh = (size_t)nk * nc * nn, n_hh = (size_t)nk * nc * nc * nn;
  auto release = [&](int code) {
    (void)hipStreamSynchronize(s);
    for (void* p : owned) (void)hipFree(p);
    ctx->bytes -= acct;
    return code;
  };
  int rc;
  if ((rc = dev_alloc(ctx, (void**)&f, nf * 8, &owned, &acct)) ||
      (rc = dev_alloc(ctx, (void**)&w, (size_t)nk * nf * 8, &owned, &acct)) ||
      (rc = dev_alloc(ctx, (void**)&t0, (size_t)nk * 8, &owned, &acct)) ||
      (rc = dev_alloc(ctx, (void**)&dv, (size_t)nk * nf * 16, &owned, &acct)) ||
      (rc = dev_alloc(ctx, (void**)&h0, (size_t)nc * nf * 16, &owned, &acct)) ||
      (rc = dev_alloc(ctx, (void**)&idx, (size_t)nn * 8, &owned, &acct)) ||
      (rc = dev_alloc(ctx, (void**)&wdh, n_dh * 16, &owned, &acct)) ||
      (rc = dev_alloc(ctx, (void**)&whh, n_hh * 16, &owned, &acct)) ||
      (rc = dev_alloc(ctx, (void**)&ddv, 8, &owned, &acct)))
    return release(rc);
  std::vector<double> t0h(nk, 0.0);
  if (d->t0) t0h.assign(d->t0, d->t0 + nk);
  hipError_t e = hipSuccess;
  auto H2D = [&](void* dst, const void* src, size_t n) {
    if (e == hipSuccess) e = hipMemcpyAsync(dst, src, n, hipMemcpyHostToDevice, s);
  };
  H2D(f, d->f, nf * 8);
  H2D(w, d->w, (size_t)nk * nf * 8);
  H2D(t0, t0h.data(), (size_t)nk * 8);
  H2D(dv, d->d, (size_t)nk * nf * 16);
  H2D(h0, d->h0, (size_t)nc * nf * 16);
  H2D(idx, d->node_idx, (size_t)nn * 8);
  if (e == hipSuccess) {
    const int64_t n = (int64_t)(n_dh + n_hh);
    hipLaunchKernelGGL(k_rb_weights, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, nk, nc, nf,
                       nn, f, dv, w, h0, t0, idx, wdh, whh);
    hipLaunchKernelGGL(k_data_norm, dim3(1), dim3(256), 0, s, (int)(nk * nf), dv, w, ddv);
    e = hipGetLastError();
  }
  if (e == hipSuccess && w_dh) e = hipMemcpyAsync(w_dh, wdh, n_dh * 16, hipMemcpyDeviceToHost, s);
  if (e == hipSuccess && w_hh) e = hipMemcpyAsync(w_hh, whh, n_hh * 16, hipMemcpyDeviceToHost, s);
  if (e == hipSuccess && dd) e = hipMemcpyAsync(dd, ddv, 8, hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return release(fail(DOTPE_E_DEVICE, "relative-binning weights: %s",
                                           hipGetErrorString(e)));
  return release(DOTPE_OK);
}

int dotpe_debug_bound(dotpe_ctx* ctx, dotpe_event* ev, float* out) {
  if (!ctx || !ev || !out) return fail(DOTPE_E_INVALID_ARG, "NULL argument");
  const int prec = ev->bank->prec;
  if (prec == kFP64) return fail(DOTPE_E_INVALID_ARG, "the bound pass runs on split precisions only");
  HIP_OK(hipSetDevice(ctx->device));
  FusedArgs a = make_args(ctx, ev);
  const size_t n = 2 * (size_t)ev->n_sub * ev->n_ext * sizeof(float);
  float* buf = nullptr;
  std::vector<void*> owned;
  uint64_t acct = 0;
  int rc = dev_alloc(ctx, (void**)&buf, n, &owned, &acct);
  if (rc) return rc;
  a.bound_out = buf;
  event_norms(ev, ev->stream);
  const int64_t n_big = ((a.n_tiles_m + 1) / 2) * ((a.n_tiles_n + 1) / 2);
  rc = launch_fused<kBound>(prec, a, round_up(n_big, 8), ev->stream);
  hipError_t e = rc ? hipSuccess : hipMemcpyAsync(out, buf, n, hipMemcpyDeviceToHost, ev->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(ev->stream);
  (void)hipFree(buf);
  ctx->bytes -= acct;
  if (rc) return rc;
  if (e != hipSuccess) return fail(DOTPE_E_DEVICE, "bound hook: %s", hipGetErrorString(e));
  return DOTPE_OK;
}

int dotpe_debug_response(dotpe_ctx* ctx, const dotpe_event* ev, double* R, double* t) {
  if (!ctx || !ev || !R || !t) return fail(DOTPE_E_INVALID_ARG, "NULL argument");
  HIP_OK(hipSetDevice(ctx->device));
  const dotpe_bank* bk = ev->bank;
  const int nc = bk->n_c;
  std::vector<double> Rg((size_t)ev->n_ext * ev->n_det * nc * 2);
  HIP_OK(hipMemcpyAsync(Rg.data(), ev->R, Rg.size() * 8, hipMemcpyDeviceToHost, ev->stream));
  HIP_OK(hipMemcpyAsync(t, ev->T, (size_t)ev->n_ext * ev->n_det * 8, hipMemcpyDeviceToHost,
                        ev->stream));
  HIP_OK(hipStreamSynchronize(ev->stream));
  for (int64_t e = 0; e < ev->n_ext; ++e)
    for (int k = 0; k < ev->n_det; ++k)
      for (int c = 0; c < nc; ++c) {
        size_t src = ((e * ev->n_det + k) * nc + c) * 2;
        size_t dst = ((e * ev->n_det + k) * nc + bk->mt.orig[c]) * 2;
        R[dst] = Rg[src];
        R[dst + 1] = Rg[src + 1];
      }
  return DOTPE_OK;
}


}  // extern "C"

// ---------------------------------------------------------------------------
// Serving: events submitted while others run are admitted FIFO as a slot and
// blocks of the device pool free up; each slot takes a batch of queued events,
// stages them and runs their evidence passes packed into shared launches on
// its own stream, so the device work of concurrent batches overlaps too.
// ---------------------------------------------------------------------------
namespace {

struct ServeJob {
  dotpe_event_desc desc{};
  std::vector<double> d, w, r, D, lat, lon, psi, ci, tg, lnwe;
  std::vector<int64_t> sub_idx;
  uint64_t bytes = 0;
  dotpe_evidence_result res{};
  std::vector<dotpe_sample> topk;
  std::string err;
};

template <class T>
const T* copy_in(std::vector<T>* v, const T* src, size_t n) {
  if (!src) return nullptr;
  v->assign(src, src + n);
  return v->data();
}

}  // namespace

struct dotpe_server;
static void serve_batch(dotpe_server* s, int slot, std::vector<Scheduler::BatchItem>& items);
static void free_server_buffers(dotpe_server* s);

struct dotpe_server {
  dotpe_ctx* ctx = nullptr;
  const dotpe_bank* bank = nullptr;
  char* pool = nullptr;
  uint64_t pool_len = 0;
  std::vector<hipStream_t> streams;
  std::vector<PackBufs> packs;   // per slot
  std::unique_ptr<Scheduler> sched;
  std::mutex mu;
  std::map<int64_t, std::shared_ptr<ServeJob>> jobs;
};

// Stage the batch's events in their pool blocks, run their evidence passes
// packed (evidence_run_packed) and release the events; each item's status is
// its event's.
static void serve_batch(dotpe_server* s, int slot, std::vector<Scheduler::BatchItem>& items) {
  const int n = (int)items.size();
  hipStream_t st = s->streams[slot];
  std::vector<dotpe_event*> evs(n, nullptr);
  std::vector<ServeJob*> jobs(n);
  std::vector<dotpe_event*> run;
  std::vector<int> run_idx;
  for (int k = 0; k < n; ++k) {
    jobs[k] = (ServeJob*)items[k].payload;
    items[k].rc = set_event_impl(s->ctx, s->bank, &jobs[k]->desc, s->pool + items[k].off,
                                 jobs[k]->bytes, st, &evs[k]);
    if (items[k].rc != DOTPE_OK) {
      jobs[k]->err = g_err;
      continue;
    }
    run.push_back(evs[k]);
    run_idx.push_back(k);
  }
  if (!run.empty()) {
    const int m = (int)run.size();
    std::vector<dotpe_evidence_result> res(m);
    std::vector<dotpe_sample*> topk(m);
    std::vector<int> rcs(m, DOTPE_OK);
    for (int q = 0; q < m; ++q) {
      ServeJob* j = jobs[run_idx[q]];
      topk[q] = j->topk.empty() ? nullptr : j->topk.data();
    }
    if (m == 1)   // alone: the event's own launches
      rcs[0] = dotpe_evidence(s->ctx, run[0], &res[0], topk[0]);
    else
      (void)evidence_run_packed(s->ctx, run.data(), m, &s->packs[slot], st, res.data(),
                                topk.data(), rcs.data());
    // after a failure, work may still be queued: the blocks return to the
    // pool only once the stream has drained
    if (std::any_of(rcs.begin(), rcs.end(), [](int r) { return r != DOTPE_OK; }))
      (void)hipStreamSynchronize(st);
    for (int q = 0; q < m; ++q) {
      const int k = run_idx[q];
      items[k].rc = rcs[q];
      if (rcs[q] == DOTPE_OK)
        jobs[k]->res = res[q];
      else
        jobs[k]->err = g_err;
    }
  }
  for (int k = 0; k < n; ++k)
    if (evs[k]) dotpe_free_event(s->ctx, evs[k]);
}

static void free_server_buffers(dotpe_server* s) {
  for (PackBufs& pb : s->packs) {
    if (pb.h_args) (void)hipHostFree(pb.h_args);
    if (pb.h_fo) (void)hipHostFree(pb.h_fo);
    if (pb.h_st) (void)hipHostFree(pb.h_st);
    if (pb.d_args) (void)hipFree(pb.d_args);
  }
  s->packs.clear();
  for (hipStream_t t : s->streams) (void)hipStreamDestroy(t);
  s->streams.clear();
  if (s->pool) {
    (void)hipFree(s->pool);
    s->ctx->bytes -= s->pool_len;
    s->pool = nullptr;
  }
}

extern "C" {

int dotpe_server_create(dotpe_ctx* ctx, const dotpe_bank* bank, const dotpe_server_desc* desc,
                        dotpe_server** out) {
  if (!ctx || !bank || !out) return fail(DOTPE_E_INVALID_ARG, "NULL argument");
  int n_slots = (desc && desc->n_slots > 0) ? desc->n_slots : 4;
  int max_batch = (desc && desc->max_batch > 0) ? desc->max_batch : 8;
  const double batch_pairs =
      (desc && desc->batch_pairs) ? (double)desc->batch_pairs : (double)(uint64_t(1) << 25);
  uint64_t pool = (desc && desc->pool_bytes) ? desc->pool_bytes : (uint64_t(8) << 30);
  if (n_slots > 16) return fail(DOTPE_E_INVALID_ARG, "n_slots=%d (at most 16)", n_slots);
  if (max_batch > kMaxPack)
    return fail(DOTPE_E_INVALID_ARG, "max_batch=%d (at most %d)", max_batch, kMaxPack);
  pool = pool / kBlockAlign * kBlockAlign;
  if (pool < kBlockAlign) return fail(DOTPE_E_INVALID_ARG, "pool_bytes too small");
  HIP_OK(hipSetDevice(ctx->device));
  dotpe_server* srv = new dotpe_server();
  srv->ctx = ctx;
  srv->bank = bank;
  int rc = dev_alloc(ctx, (void**)&srv->pool, pool, nullptr, nullptr);
  if (rc) {
    delete srv;
    return rc;
  }
  srv->pool_len = pool;
  for (int q = 0; q < n_slots; ++q) {
    hipStream_t st = nullptr;
    PackBufs pb;
    hipError_t e = hipStreamCreateWithFlags(&st, hipStreamNonBlocking);
    if (e == hipSuccess) {
      srv->streams.push_back(st);
      e = hipHostMalloc((void**)&pb.h_args, sizeof(FusedArgs) * kMaxPack, hipHostMallocDefault);
      if (e == hipSuccess)
        e = hipHostMalloc((void**)&pb.h_fo, sizeof(double) * kMaxPack * (kNPart + 3),
                          hipHostMallocDefault);
      if (e == hipSuccess)
        e = hipHostMalloc((void**)&pb.h_st, sizeof(uint64_t) * kMaxPack * 6, hipHostMallocDefault);
      if (e == hipSuccess) e = hipMalloc((void**)&pb.d_args, sizeof(FusedArgs) * kMaxPack);
      srv->packs.push_back(pb);
    }
    if (e != hipSuccess) {
      free_server_buffers(srv);
      delete srv;
      return fail(DOTPE_E_DEVICE, "server set-up: %s", hipGetErrorString(e));
    }
  }
  const int dev = ctx->device;
  dotpe_server* sv = srv;
  Scheduler::BatchFn batch = [sv](int slot, std::vector<Scheduler::BatchItem>& items) {
    serve_batch(sv, slot, items);
  };
  srv->sched.reset(new Scheduler(n_slots, pool, [dev](int) { (void)hipSetDevice(dev); }, max_batch,
                                 batch, batch_pairs));
  *out = srv;
  return DOTPE_OK;
}

int dotpe_server_destroy(dotpe_server* srv) {
  if (!srv) return DOTPE_OK;
  srv->sched.reset();   // runs every submitted event to completion
  free_server_buffers(srv);
  delete srv;
  return DOTPE_OK;
}

int dotpe_submit(dotpe_server* srv, const dotpe_event_desc* d, int64_t* ticket) {
  if (!srv || !d || !ticket) return fail(DOTPE_E_INVALID_ARG, "NULL argument");
  EvDims D;
  std::vector<int> terms;
  int rc = event_dims(srv->bank, d, &D, &terms);
  if (rc) return rc;
  auto job = std::make_shared<ServeJob>();
  {
    dotpe_event probe;
    EvStage st;
    job->bytes = block_bytes(event_buffers(D, &probe, &st));
  }
  if (!srv->sched->admissible(job->bytes))
    return fail(DOTPE_E_ADMISSION, "event needs %llu bytes; the serving pool holds %llu",
                (unsigned long long)job->bytes, (unsigned long long)srv->pool_len);
  const size_t nk = (size_t)d->n_det, nb = (size_t)srv->bank->n_b, ne = (size_t)d->n_ext;
  job->desc = *d;
  job->desc.d = copy_in(&job->d, d->d, nk * nb * 2);
  job->desc.w = copy_in(&job->w, d->w, nk * nb);
  job->desc.det_r = copy_in(&job->r, d->det_r, nk * 3);
  job->desc.det_D = copy_in(&job->D, d->det_D, nk * 9);
  job->desc.lat = copy_in(&job->lat, d->lat, ne);
  job->desc.lon = copy_in(&job->lon, d->lon, ne);
  job->desc.psi = copy_in(&job->psi, d->psi, ne);
  job->desc.cos_iota = copy_in(&job->ci, d->cos_iota, ne);
  job->desc.t_geo = copy_in(&job->tg, d->t_geo, ne);
  job->desc.ln_w_ext = copy_in(&job->lnwe, d->ln_w_ext, ne);
  job->desc.sub_idx = copy_in(&job->sub_idx, d->sub_idx, d->sub_idx ? (size_t)D.n_sub : 0);
  job->desc.stream = nullptr;
  job->topk.resize((size_t)std::max(0, d->top_k));
  dotpe_server* s = srv;
  int64_t t = srv->sched->submit(
      job->bytes,
      [s, job](int slot, uint64_t off) -> int {
        std::vector<Scheduler::BatchItem> one{Scheduler::BatchItem{job.get(), off, 0}};
        serve_batch(s, slot, one);
        return one[0].rc;
      },
      job, (double)D.n_sub * (double)D.ne);
  {
    std::lock_guard<std::mutex> lk(srv->mu);
    srv->jobs[t] = job;
  }
  *ticket = t;
  return DOTPE_OK;
}

int dotpe_poll(dotpe_server* srv, int64_t ticket, int32_t* done) {
  if (!srv || !done) return fail(DOTPE_E_INVALID_ARG, "NULL argument");
  int r = srv->sched->poll(ticket);
  if (r < 0) return fail(DOTPE_E_INVALID_ARG, "unknown ticket %lld", (long long)ticket);
  *done = r;
  return DOTPE_OK;
}

int dotpe_wait(dotpe_server* srv, int64_t ticket, dotpe_evidence_result* out, dotpe_sample* topk,
               dotpe_ticket_info* info) {
  if (!srv) return fail(DOTPE_E_INVALID_ARG, "NULL argument");
  std::shared_ptr<ServeJob> job;
  {
    std::lock_guard<std::mutex> lk(srv->mu);
    auto it = srv->jobs.find(ticket);
    if (it == srv->jobs.end())
      return fail(DOTPE_E_INVALID_ARG, "unknown ticket %lld", (long long)ticket);
    job = it->second;
  }
  JobTimes tm;
  int rc = srv->sched->wait(ticket, &tm);
  {
    std::lock_guard<std::mutex> lk(srv->mu);
    srv->jobs.erase(ticket);
  }
  if (rc == Scheduler::kUnknown)
    return fail(DOTPE_E_INVALID_ARG, "unknown ticket %lld", (long long)ticket);
  if (info) {
    info->t_submit_ms = tm.t_submit_ms;
    info->t_start_ms = tm.t_start_ms;
    info->t_done_ms = tm.t_done_ms;
    info->bytes = tm.bytes;
    info->slot = tm.slot;
    info->status = rc;
    info->batch = tm.batch;
    info->reserved = 0;
  }
  if (rc != DOTPE_OK) return fail(rc, "%s", job->err.c_str());
  if (out) *out = job->res;
  if (topk)
    for (int q = 0; q < job->res.topk_count; ++q) topk[q] = job->topk[q];
  return DOTPE_OK;
}

}  // extern "C"
