// hd_api.cpp -- C ABI of libhdconv: plans, device tables, workspace and the
// launch sequence of one convolution.
#include <hip/hip_runtime.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <tuple>
#include <vector>

#include "hdconv.h"
#include "hd_engine.hpp"
#include "hd_plan.hpp"

using namespace hd;

// ---------------------------------------------------------------------------
// thread-local last error
namespace {
thread_local int g_err_code = HDCONV_OK;
thread_local char g_err_msg[512] = {0};

int set_err(int code, const char* fmt, ...) {
  g_err_code = code;
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err_msg, sizeof(g_err_msg), fmt, ap);
  va_end(ap);
  return code;
}
void clear_err() {
  g_err_code = HDCONV_OK;
  g_err_msg[0] = 0;
}
int hip_err(hipError_t e, const char* what) {
  return set_err(HDCONV_EDEVICE, "%s: %s", what, hipGetErrorString(e));
}

int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }

// Device copy of the per-dimension tables.
struct DimDev {
  void* fft_m = nullptr;  // stage twiddles of the m-point transform
  void* fft_p = nullptr;  // stage twiddles of the p-point transform
  void* zq = nullptr;     // zeta_q^k, k < q (inner form)
  void* zlo = nullptr;    // two-level table of zeta_{qm}
  void* zhi = nullptr;
  int kbits = 0;
};

}  // namespace

// One row-pass launch's share of an output: up to three of the plan's
// inputs and the weights of their pairs (pair_slot order); the output is the
// sum of its shares.
struct Share {
  int n = 0;                 // inputs of the launch (2 or 3)
  int idx[kMaxA] = {0, 0, 0};  // the plan's input of each
  double c[6] = {};
};

struct Plan {
  int dims = 0, A = 0, B = 0, dtype = 0, method = 0, flags = 0;
  int64_t L[3] = {1, 1, 1}, M[3] = {1, 1, 1};
  int64_t Lio[3] = {1, 1, 1};  // stored extents (Hermitian: ceil(L/2))
  int64_t npad[3] = {0, 0, 0};
  DimPlan dp[3];
  int device = -1;
  int cus = 1;  // compute units of the device (sizes persistent grids)
  bool host_only = false;
  // device memory
  char* table_mem = nullptr;
  size_t table_bytes = 0;
  DimDev dd[3];
  char* work_mem = nullptr;
  size_t work_bytes = 0;
  void* pad_in[kMaxIn] = {};                          // explicit method
  void* lvl[2][kMaxIn] = {{nullptr}};                 // outer-level buffers W_d
  void* rowwork[kMaxIn] = {};                         // inner-form work rows
  double* acc64 = nullptr;                            // multi-block accumulator
  int64_t batch_rows = 1;                             // rows of a batched group
  int64_t copies = 1, dist = 0;                       // copies per execute, words between them
  int64_t stride[2] = {0, 0};                         // element strides of dims 0, 1 (0: dense)
  int quad = 0;                                       // quadratic multiplication operator, B outputs
  bool conj_pairs = true;                             // inner form: residues v and n - v together
  // the launches of the row pass per output: shares of at most three inputs
  // (one share with every input for products and A <= 3)
  std::vector<Share> shares[kMaxB];
  void* rowout = nullptr;                             // quadratic: result rows of the row pass
  void* outbuf = nullptr;                             // quadratic 2D/3D: the innermost level's result
  void* padout = nullptr;                             // quadratic explicit method: padded result
  int64_t span = 0;                                   // words one copy of an array spans
  int tuner = 0, tuned_candidates = 0, timed_candidates = 0;
  double tuned_ms = 0;
  int launches = 0;
  // per-launch event timing (hdconv_profile_begin / hdconv_profile_end)
  struct Prof {
    bool on = false;
    int max_exec = 0, used = 0, slot = 0, nslots = 0;
    std::vector<hipEvent_t> ev;  // [exec][slot][start, end]
    std::vector<std::string> names;
    std::vector<double> bytes;
  } prof;
};

// Records an event pair around one kernel launch when profiling is on.
struct ProfScope {
  Plan* P;
  hipStream_t s;
  int idx = -1;
  ProfScope(Plan* P_, hipStream_t s_, const char* name, double bytes) : P(P_), s(s_) {
    Plan::Prof& f = P->prof;
    if (!f.on || f.used >= f.max_exec || f.slot >= f.nslots) return;
    if ((int)f.names.size() <= f.slot) {
      f.names.resize(f.slot + 1);
      f.bytes.resize(f.slot + 1);
    }
    f.names[f.slot] = name;
    f.bytes[f.slot] = bytes;
    idx = (f.used * f.nslots + f.slot) * 2;
    (void)hipEventRecord(f.ev[idx], s);
  }
  ~ProfScope() {
    if (idx >= 0) {
      (void)hipEventRecord(P->prof.ev[idx + 1], s);
      P->prof.slot++;
    }
  }
};

// ---------------------------------------------------------------------------
// planning

static int tbytes_of(int dtype) { return dtype == HDCONV_C64 ? 4 : 8; }

// Hermitian arrays of nominal length L store ceil(L/2) entries and stand for
// the centered array of length 2 ceil(L/2) - 1 the engine transforms.
static int64_t herm_stored(int64_t L) { return (L + 1) / 2; }
static int64_t herm_full(int64_t L) { return 2 * herm_stored(L) - 1; }
// An outer dimension in the inner form (column passes of p points, then the
// m-point pass; all q residues in one block).
static bool outer_inner(const DimPlan& dp) { return dp.variant == VAR_OUTER && dp.p > 2; }

static int tune_shapes(const int64_t* L, const int64_t* M, int A, int B, int dims, int dtype,
                       const hdconv_options* opt, hdconv_dim_info_t* shp, int* ncand, int* ntimed, double* best_ms);
static hdconv_options opts_from_shape(const hdconv_dim_info_t* shp, int dims);

// Independent lines one launch of dimension d processes: the product of the
// other dimensions' lengths (outer ones padded to about twice their length
// by the residues), so 1 only for a single 1D convolution.
static int64_t lines_of_shape(const int64_t* L, int dims, int d) {
  int64_t n = 1;
  for (int e = 0; e < dims; ++e)
    if (e != d) n *= (e < d ? 2 : 1) * L[e];
  return n;
}
static int64_t lines_of(const Plan* P, int d) {
  return P->batch_rows > 1 ? P->batch_rows : P->copies * lines_of_shape(P->L, P->dims, d);
}

// Inputs one kernel launch combines (quadratic operators with more inputs
// run shares of at most three).
static int kernel_inputs(const Plan* P) { return std::min(P->A, kMaxA); }

static int build_dims(Plan* P, const hdconv_options* opt) {
  const int tb = tbytes_of(P->dtype);
  // centered hybrid plans run centered transforms; the explicit method pads
  // the arrays as they are and reads the centered window out of the result
  const int herm = (P->flags & HDCONV_PLAN_HERMITIAN) && P->method != HDCONV_METHOD_EXPLICIT ? 1 : 0;
  const int ctr = ((P->flags & (HDCONV_PLAN_CENTERED | HDCONV_PLAN_HERMITIAN)) &&
                   P->method != HDCONV_METHOD_EXPLICIT) ? 1 : 0;
  for (int d = 0; d < P->dims; ++d) {
    const bool contiguous = (d == P->dims - 1);
    // a Hermitian plan's last dimension runs at the full centered length
    const int hd = herm && contiguous;
    int64_t Le = hd ? herm_full(P->L[d]) : P->L[d], Me = P->M[d];
    if (P->method == HDCONV_METHOD_EXPLICIT) Le = Me = P->npad[d];
    DimPlan& dp = P->dp[d];
    std::string why;
    const int64_t fm = opt ? opt->m[d] : 0;
    const int64_t fp = opt ? opt->p[d] : 0;
    int fv = opt ? opt->variant[d] : 0;
    if (P->method == HDCONV_METHOD_EXPLICIT || (fm == 0 && fp == 0 && fv == 0)) {
      if (P->method == HDCONV_METHOD_EXPLICIT) {
        // one full-length transform per dimension: p = q = 1 (or inner form
        // with n = 1); options.m, when set, picks the split N' = p m
        dp = DimPlan{};
        dp.L = Le;
        dp.M = Me;
        if (fm > 0 && contiguous) {
          if (Le % fm != 0 || !fft_size_ok(fm) || (Le / fm > 1 && !col_size_ok(Le / fm)))
            return set_err(HDCONV_EINVAL, "explicit padding, dim %d: m=%lld does not split N'=%lld", d,
                           (long long)fm, (long long)Le);
          dp.m = fm;
          dp.p = Le / fm;
          dp.n = dp.D = 1;
          dp.q = dp.p;
          dp.variant = dp.p == 1 ? VAR_FUSED : VAR_MULTI;
          if (opt) {
            dp.E_m = opt->E_m[d];
            dp.E_p = opt->E_p[d];
          }
        } else if (!contiguous || (Le <= kMaxFusedM && [&] {
                     // one whole-row transform, if it fits the row kernel (LDS)
                     DimPlan t = dp;
                     t.m = Le;
                     t.p = t.q = t.n = t.D = 1;
                     t.variant = VAR_FUSED;
                     std::string w;
                     return finish_dim(&t, kernel_inputs(P), tb, &w);
                   }())) {
          dp.m = Le;
          dp.p = dp.q = dp.n = dp.D = 1;
          dp.variant = contiguous ? VAR_FUSED : VAR_OUTER;
        } else {
          // largest m up to 8192 (c64) / 4096 (c128), then any m, with p = N'/m valid
          int64_t m = 0;
          for (int pass = 0; pass < 2 && m == 0; ++pass) {
            const int64_t mmax = pass == 0 ? (tb == 4 ? 8192 : 4096) : kMaxRowM;
            for (int64_t c = mmax; c >= 8 && m == 0; --c)
              if (fft_size_ok(c) && Le % c == 0 && col_size_ok(Le / c) && Le / c <= kMaxColP) m = c;
          }
          if (m == 0) return set_err(HDCONV_EUNSUPPORTED, "explicit padding, dim %d: no split of N'=%lld", d, (long long)Le);
          dp.m = m;
          dp.p = Le / m;
          dp.n = dp.D = 1;
          dp.q = dp.p;
          dp.variant = VAR_MULTI;
        }
        if (!finish_dim(&dp, kernel_inputs(P), tb, &why))
          return set_err(HDCONV_EUNSUPPORTED, "explicit padding, dim %d (N'=%lld): %s", d, (long long)Le, why.c_str());
      } else if (!choose_dim(Le, Me, kernel_inputs(P), tb, contiguous, lines_of(P, d), &dp, &why, ctr, P->dims)) {
        return set_err(HDCONV_EUNSUPPORTED, "dim %d: %s", d, why.c_str());
      }
      if (opt && opt->D[d] > 0 && dp.variant == VAR_OUTER) dp.D = std::min<int64_t>(opt->D[d], dp.n);
      if (opt && (opt->E_m[d] || opt->E_p[d] || opt->S[d] || opt->rows_per_block[d] || opt->twiddles[d])) {
        // the chosen geometry with the caller's launch shape
        if (opt->E_m[d]) dp.E_m = opt->E_m[d];
        if (opt->E_p[d]) dp.E_p = opt->E_p[d];
        if (opt->S[d] || opt->E_m[d] || opt->E_p[d]) dp.S = opt->S[d];
        if (opt->rows_per_block[d] || opt->E_m[d]) dp.rows_per_block = opt->rows_per_block[d];
        if (opt->twiddles[d]) dp.tw_pref = opt->twiddles[d];
        if (!finish_dim(&dp, kernel_inputs(P), tb, &why))
          return set_err(HDCONV_EUNSUPPORTED, "dim %d (m=%lld, p=%lld, q=%lld): %s", d, (long long)dp.m,
                         (long long)dp.p, (long long)dp.q, why.c_str());
      }
      dp.herm = hd;
    } else {
      if (fv == HDCONV_VARIANT_AUTO) {
        Geometry g = geometry_c(Le, Me, fm ? fm : next_fft_size(Le), fp, false, ctr);
        fv = contiguous ? (g.inner ? VAR_MULTI : VAR_FUSED) : VAR_OUTER;
      }
      if (contiguous && fv == VAR_OUTER) return set_err(HDCONV_EINVAL, "dim %d: outer variant on the innermost dimension", d);
      if (!contiguous && fv != VAR_OUTER) return set_err(HDCONV_EUNSUPPORTED, "dim %d: outer dimensions use the outer variant", d);
      int64_t m = fm ? fm : next_fft_size(fv == VAR_MULTI ? cdiv(Le, std::max<int64_t>(fp, 4)) : Le);
      // a forced inner form without a forced m: rows of at most 4096 points
      // (the row pass's best size), the column count then follows from L
      if (!fm && fv == VAR_MULTI && m > 4096) m = 4096;
      // an outer dimension takes the inner form when p > 2 (forced, or L > 2m)
      const bool oin = fv == VAR_OUTER && (fp > 2 || cdiv(Le, m) > 2);
      Geometry g = geometry_c(Le, Me, m, fp, fv == VAR_MULTI || oin, ctr);
      if (g.inner && fv != VAR_MULTI && !oin)
        return set_err(HDCONV_EINVAL, "dim %d: m=%lld gives p=%lld > 2, which needs the multipass variant", d,
                       (long long)m, (long long)g.p);
      if (fv == VAR_MULTI && !col_size_ok(g.p)) {
        g = geometry_c(Le, Me, m, next_col_size(g.p), true, ctr);
      }
      if (oin) {  // the least compiled column size: 2^k, or 3 * 2^k from 12 (complex64)
        int64_t p2 = 4;
        while (p2 < g.p) p2 *= 2;
        int64_t pc = p2;
        for (int64_t p3 = 12; p3 <= 96 && tb == 4; p3 *= 2)
          if (p3 >= g.p && p3 < pc) pc = p3;
        if (pc != g.p) g = geometry_c(Le, Me, m, pc, true, ctr);
      }
      dp = DimPlan{};
      dp.L = Le;
      dp.M = Me;
      dp.m = g.m;
      dp.p = g.p;
      dp.n = g.n;
      dp.q = g.q;
      dp.D = (opt && opt->D[d] > 0) ? std::min<int64_t>(opt->D[d], g.n) : g.n;
      dp.variant = fv;
      dp.ctr = ctr;
      dp.herm = hd;
      if (opt) {
        dp.E_m = opt->E_m[d];
        dp.E_p = opt->E_p[d];
        dp.S = opt->S[d];
        dp.rows_per_block = opt->rows_per_block[d];
        dp.tw_pref = opt->twiddles[d];
      }
      if (!finish_dim(&dp, kernel_inputs(P), tb, &why))
        return set_err(HDCONV_EUNSUPPORTED, "dim %d (m=%lld, p=%lld, q=%lld): %s", d, (long long)dp.m,
                       (long long)dp.p, (long long)dp.q, why.c_str());
    }
  }
  // residue blocks (D < q) on the first outer dimension only
  for (int d = 1; d + 1 < P->dims; ++d)
    if (P->dp[d].D < P->dp[d].n)
      return set_err(HDCONV_EUNSUPPORTED, "dim %d: residue blocks (D < q) apply to the first dimension only", d);
  // the inner form of an outer dimension reads dense planes
  if (P->dims > 1 && outer_inner(P->dp[0]) && (P->stride[0] || P->stride[1]))
    return set_err(HDCONV_EUNSUPPORTED, "dim 0: the inner form of an outer dimension takes dense arrays (no strides)");
  return HDCONV_OK;
}

template <typename T>
static QuadMult<T> quad_of(const Plan* P, const Share& sh) {
  QuadMult<T> q{};
  q.on = P->quad;
  for (int k = 0; k < 6; ++k) q.c[k] = P->quad ? (T)sh.c[k] : T(0);
  return q;
}

// Splits output b of a quadratic operator (coefficients c[i][j], i <= j,
// row-major A x A) into shares of at most three inputs: each term F_i F_j
// joins the first share that stays within three inputs with i and j.  A
// lone input is paired with another one at zero weight (the kernels combine
// two or three transforms).
static std::vector<Share> make_shares(int A, const double* c) {
  std::vector<Share> out;
  if (A <= kMaxA) {
    Share sh;
    sh.n = A;
    for (int i = 0; i < A; ++i) sh.idx[i] = i;
    for (int i = 0; i < A; ++i)
      for (int j = i; j < A; ++j) sh.c[pair_slot(i, j)] = c[i * A + j];
    out.push_back(sh);
    return out;
  }
  auto local = [](Share& sh, int x) {
    for (int k = 0; k < sh.n; ++k)
      if (sh.idx[k] == x) return k;
    sh.idx[sh.n] = x;
    return sh.n++;
  };
  auto has = [](const Share& sh, int x) {
    for (int k = 0; k < sh.n; ++k)
      if (sh.idx[k] == x) return true;
    return false;
  };
  for (int i = 0; i < A; ++i)
    for (int j = i; j < A; ++j) {
      const double w = c[i * A + j];
      if (w == 0.0) continue;
      Share* tgt = nullptr;
      for (Share& sh : out) {
        const int need = (has(sh, i) ? 0 : 1) + (i != j && !has(sh, j) ? 1 : 0);
        if (sh.n + need <= kMaxA) {
          tgt = &sh;
          break;
        }
      }
      if (!tgt) {
        out.emplace_back();
        tgt = &out.back();
      }
      int li = local(*tgt, i), lj = local(*tgt, j);
      if (li > lj) std::swap(li, lj);
      tgt->c[pair_slot(li, lj)] += w;
    }
  if (out.empty()) {  // the zero operator
    out.emplace_back();
    out.back().n = 1;
  }
  for (Share& sh : out)
    if (sh.n == 1) sh.idx[sh.n++] = sh.idx[0] == 0 ? 1 : 0;
  return out;
}

// Largest number of shares of any output.
static int max_shares(const Plan* P) {
  size_t n = 1;
  for (int b = 0; b < P->B; ++b) n = std::max(n, P->shares[b].size());
  return (int)n;
}

// Extent of dimension d as stored between passes: the engine length, or the
// stored half of a Hermitian last dimension.
static int64_t stored_extent(const DimPlan& dp) { return dp.herm ? herm_stored(dp.L) : dp.L; }

// bytes moved by the kernels of one execute, by design (reads + writes)
static double plan_traffic(const Plan* P, int* launches) {
  const double w = 2.0 * tbytes_of(P->dtype);
  const int A = P->A;
  const int nout = P->quad ? P->B : 1;  // outputs, each through the row pass and the inverse passes
  const int groups = (int)cdiv(A, kMaxA);  // forward launches per pass (three inputs each)
  // row-pass launches per output and the inputs they read
  int shares = 0;
  double share_in = 0;
  for (int b = 0; b < nout; ++b)
    for (const Share& sh : P->shares[b]) {
      shares += 1;
      share_in += sh.n;
    }
  double bytes = 0;
  int nl = 0;
  int64_t Le[3];
  for (int d = 0; d < P->dims; ++d) Le[d] = P->dp[d].L;
  double ltot = 1, etot = 1;
  for (int d = 0; d < P->dims; ++d) {
    ltot *= (double)P->Lio[d];
    etot *= (double)Le[d];
  }
  if (P->method == HDCONV_METHOD_EXPLICIT) {
    bytes += A * (ltot + etot) * w;     // padding copies
    bytes += nout * (etot + ltot) * w;  // truncating copies
    nl += A + nout;
  }
  double nb = 1;  // planes entering the current level
  // residue blocks of the first outer dimension: the pipeline runs once per
  // block; each block reads the inputs, later blocks also read the output
  const int64_t blocks0 = P->dims > 1 ? cdiv(P->dp[0].q, P->dp[0].D) : 1;
  for (int d = 0; d + 1 < P->dims; ++d) {
    const DimPlan& dp = P->dp[d];
    double rest = 1;
    for (int e = d + 1; e < P->dims; ++e) rest *= (double)stored_extent(P->dp[e]);
    const double in_el = nb * Le[d] * rest, out_el = nb * dp.q * dp.m * rest;
    const double nbk = d == 0 ? (double)blocks0 : 1.0;
    bytes += A * (nbk * in_el + out_el) * w + nout * (out_el + (2.0 * nbk - 1.0) * in_el) * w;  // forward + backward
    nl += (int)blocks0 * (groups + nout);
    if (outer_inner(dp)) {  // the m-point passes read and write the level in place
      bytes += 2.0 * (A + nout) * out_el * w;
      nl += A + nout;
    }
    nb *= (double)(dp.q * dp.m);
  }
  const DimPlan& dl = P->dp[P->dims - 1];
  // words each row reads per input and writes (Hermitian rows: the stored half)
  const double rows = nb, Lr = (double)(dl.herm ? P->Lio[P->dims - 1] : Le[P->dims - 1]);
  if (dl.variant == VAR_FUSED) {
    // every share reads its inputs and writes; later shares also read the output
    bytes += rows * (share_in + shares + (shares - nout)) * Lr * w;
    nl += (int)blocks0 * shares;
  } else {
    const int64_t blocks = cdiv(dl.n, dl.D);
    const double wk = rows * (double)dl.q * dl.m;  // all residues' rows
    // K1 (read inputs per block, write work) once, or per output with blocks
    const int k1_runs = blocks > 1 ? nout : 1;
    bytes += k1_runs * (blocks * rows * A * Lr * w + A * wk * w);
    bytes += (share_in + shares) * wk * w;      // K2
    bytes += shares * wk * w + nout * rows * Lr * w;  // K3
    // FP64 accumulator round trips over the blocks and shares of each output
    for (int b = 0; b < nout; ++b) {
      const double contrib = (double)blocks * (double)P->shares[b].size();
      if (contrib > 1) bytes += (2.0 * contrib - 2) * rows * Lr * 16.0;
    }
    nl += (int)blocks0 * (k1_runs * (int)blocks * groups + 2 * (int)blocks * shares);
  }
  if (launches) *launches = P->method == HDCONV_METHOD_EXPLICIT ? nl * (int)P->copies : nl;
  return bytes * (double)P->copies;
}

template <typename T>
static void to_dtype(const std::vector<double>& v, std::vector<char>* out) {
  out->resize(v.size() * sizeof(T));
  T* p = reinterpret_cast<T*>(out->data());
  for (size_t i = 0; i < v.size(); ++i) p[i] = (T)v[i];
}

static int alloc_tables(Plan* P) {
  // host images of every table, concatenated with 256-byte alignment
  std::vector<std::vector<double>> parts;
  struct Ref { int dim, kind; };
  std::vector<Ref> refs;
  for (int d = 0; d < P->dims; ++d) {
    DimPlan& dp = P->dp[d];
    parts.push_back(fft_table(dp.fd_m));
    refs.push_back({d, 0});
    if (dp.variant == VAR_MULTI || (dp.variant == VAR_OUTER && dp.p > 2)) {
      parts.push_back(fft_table(dp.fd_p));
      refs.push_back({d, 1});
      std::vector<double> zq(2 * dp.q);
      for (int64_t k = 0; k < dp.q; ++k) root(dp.q, k, &zq[2 * k], &zq[2 * k + 1]);
      parts.push_back(zq);
      refs.push_back({d, 2});
    }
    const int64_t qm = dp.q * dp.m;
    int kb = 0;
    while ((int64_t(1) << (2 * kb)) < qm) ++kb;  // K ~ sqrt(qm)
    P->dd[d].kbits = kb;
    const int64_t K = int64_t(1) << kb;
    std::vector<double> lo(2 * K), hi(2 * cdiv(qm, K));
    for (int64_t e = 0; e < K; ++e) root(qm, e, &lo[2 * e], &lo[2 * e + 1]);
    for (int64_t h = 0; h < cdiv(qm, K); ++h) root(qm, h * K, &hi[2 * h], &hi[2 * h + 1]);
    parts.push_back(lo);
    refs.push_back({d, 3});
    parts.push_back(hi);
    refs.push_back({d, 4});
  }
  const int tb = tbytes_of(P->dtype);
  std::vector<size_t> off;
  size_t total = 0;
  for (auto& v : parts) {
    off.push_back(total);
    total += ((v.size() * tb + 255) / 256) * 256 + 256;
  }
  P->table_bytes = total;
  if (P->host_only) return HDCONV_OK;
  hipError_t e = hipMalloc((void**)&P->table_mem, total);
  if (e != hipSuccess) return set_err(HDCONV_ENOMEM, "hipMalloc(tables, %zu): %s", total, hipGetErrorString(e));
  std::vector<char> host(total, 0);
  for (size_t i = 0; i < parts.size(); ++i) {
    std::vector<char> img;
    if (tb == 4) to_dtype<float>(parts[i], &img);
    else to_dtype<double>(parts[i], &img);
    if (!img.empty()) memcpy(host.data() + off[i], img.data(), img.size());
    void* ptr = P->table_mem + off[i];
    DimDev& dd = P->dd[refs[i].dim];
    switch (refs[i].kind) {
      case 0: dd.fft_m = ptr; break;
      case 1: dd.fft_p = ptr; break;
      case 2: dd.zq = ptr; break;
      case 3: dd.zlo = ptr; break;
      case 4: dd.zhi = ptr; break;
    }
  }
  e = hipMemcpy(P->table_mem, host.data(), total, hipMemcpyHostToDevice);
  if (e != hipSuccess) return hip_err(e, "hipMemcpy(tables)");
  return HDCONV_OK;
}

static size_t align256(size_t x) { return (x + 255) / 256 * 256; }

// The workspace of a plan as parts (where each part's pointer goes, its
// bytes); each part starts on a 256-byte boundary.
static std::vector<std::pair<void**, size_t>> workspace_parts(Plan* P) {
  const size_t w = 2 * (size_t)tbytes_of(P->dtype);
  int64_t Le[3];
  for (int d = 0; d < P->dims; ++d) Le[d] = P->dp[d].L;
  std::vector<std::pair<void**, size_t>> want;
  if (P->method == HDCONV_METHOD_EXPLICIT) {
    size_t n = 1;
    for (int d = 0; d < P->dims; ++d) n *= (size_t)P->npad[d];
    for (int a = 0; a < P->A; ++a) want.push_back({&P->pad_in[a], n * w});
  }
  // independent rows (batched groups) or copies, else 1 (the explicit method
  // runs copies one at a time)
  size_t nb = (size_t)(P->method == HDCONV_METHOD_EXPLICIT ? 1 : P->batch_rows * P->copies);
  for (int d = 0; d + 1 < P->dims; ++d) {
    size_t rest = 1;
    for (int e = d + 1; e < P->dims; ++e) rest *= (size_t)stored_extent(P->dp[e]);
    // the first outer dimension holds one block of D residues at a time
    // (the inner form: all of them)
    nb *= (size_t)((d == 0 && !outer_inner(P->dp[d]) ? P->dp[d].D : P->dp[d].q) * P->dp[d].m);
    for (int a = 0; a < P->A; ++a) want.push_back({&P->lvl[d][a], nb * rest * w});
  }
  const DimPlan& dl = P->dp[P->dims - 1];
  if (P->quad && P->method == HDCONV_METHOD_EXPLICIT) {  // padded result of one output
    size_t n = 1;
    for (int d = 0; d < P->dims; ++d) n *= (size_t)P->npad[d];
    want.push_back({&P->padout, n * w});
  }
  if (P->quad && P->dims > 1) {  // the innermost level's result of one output
    size_t last = nb;
    want.push_back({&P->outbuf, last * (size_t)stored_extent(P->dp[P->dims - 1]) * w});
  }
  if (dl.variant == VAR_MULTI) {
    const size_t rowsz = nb * (size_t)(dl.D * dl.p * dl.m);
    for (int a = 0; a < P->A; ++a) want.push_back({&P->rowwork[a], rowsz * w});
    if (P->quad) want.push_back({&P->rowout, rowsz * w});
    // the FP64 accumulator is laid out like the rows' output (1D copies: dist apart)
    size_t acc_rows = nb, acc_len = (size_t)Le[P->dims - 1];
    if (P->dims == 1 && P->copies > 1 && P->method != HDCONV_METHOD_EXPLICIT) {
      acc_rows = (size_t)P->copies;
      acc_len = (size_t)P->dist;
    }
    // (also for outputs summed over several row-pass shares)
    // (not with HDCONV_PLAN_ACCUMULATE_OUTPUT: the output array accumulates)
    if ((dl.D < dl.n || max_shares(P) > 1) && !(P->flags & HDCONV_PLAN_ACCUMULATE_OUTPUT))
      want.push_back({(void**)&P->acc64, acc_rows * acc_len * 16});
  }
  return want;
}

// Point the workspace parts into `base` (nullptr: clear them).
static void carve_workspace(Plan* P, char* base) {
  size_t o = 0;
  for (auto& x : workspace_parts(P)) {
    *x.first = base ? base + o : nullptr;
    o += align256(x.second);
  }
}

// Workspace bytes, checked against the HDCONV_WORKSPACE_CAP environment
// variable (a byte count; HDCONV_ENOMEM above it).  Host only.
static int size_workspace(Plan* P) {
  size_t total = 0;
  for (auto& x : workspace_parts(P)) total += align256(x.second);
  P->work_bytes = total;
  const char* cap = getenv("HDCONV_WORKSPACE_CAP");
  if (cap && total > 0 && (size_t)atoll(cap) < total)
    return set_err(HDCONV_ENOMEM, "workspace of %zu bytes exceeds HDCONV_WORKSPACE_CAP=%s", total, cap);
  return HDCONV_OK;
}

// With HDCONV_POISON_WORKSPACE set in the environment every new workspace is
// filled with all-ones bytes (a NaN in FP32 and FP64), so a kernel that reads
// a workspace word no earlier kernel of the execute wrote shows up as NaN
// outputs.  A debugging aid; off by default.
static int alloc_workspace(Plan* P) {
  const size_t total = P->work_bytes;
  if (P->host_only || total == 0 || (P->flags & HDCONV_PLAN_NO_WORKSPACE)) return HDCONV_OK;
  hipError_t e = hipMalloc((void**)&P->work_mem, total);
  if (e != hipSuccess) return set_err(HDCONV_ENOMEM, "hipMalloc(workspace, %zu): %s", total, hipGetErrorString(e));
  carve_workspace(P, P->work_mem);
  const char* poison = getenv("HDCONV_POISON_WORKSPACE");
  if (poison && poison[0] && poison[0] != '0') {
    e = hipMemset(P->work_mem, 0xff, total);
    if (e == hipSuccess) e = hipDeviceSynchronize();
    if (e != hipSuccess) return hip_err(e, "hipMemset(workspace poison)");
  }
  return HDCONV_OK;
}

// ---------------------------------------------------------------------------
// Static device scratch of hdconv_execute_noalloc.  In host code the array's
// name only stands for the variable; its device address (one per GPU) comes
// from hipGetSymbolAddress, called once per device with that device current.
static __device__ __align__(256) char hd_scratch[HDCONV_SCRATCH_BYTES];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
char* g_scratch_ptr[kMaxDevices] = {};

// Device address of the scratch area on the current device `dev`.
int scratch_of(int dev, char** out) {
  if (dev < 0 || dev >= kMaxDevices)
    return set_err(HDCONV_EUNSUPPORTED, "device %d beyond the %d supported", dev, kMaxDevices);
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(hd_scratch));
    if (e != hipSuccess) return hip_err(e, "hipGetSymbolAddress(scratch)");
    if (!ptr) return set_err(HDCONV_EDEVICE, "hipGetSymbolAddress(scratch) returned NULL");
    g_scratch_ptr[dev] = (char*)ptr;
  }
  *out = g_scratch_ptr[dev];
  return HDCONV_OK;
}
}  // namespace

static void free_plan(Plan* P) {
  if (!P) return;
  if (P->table_mem || P->work_mem) (void)hipDeviceSynchronize();
  if (P->table_mem) (void)hipFree(P->table_mem);
  if (P->work_mem) (void)hipFree(P->work_mem);
  delete P;
}

// ---------------------------------------------------------------------------
// execution

template <typename T>
static RootTable<T> rtab(const Plan* P, int d) {
  RootTable<T> r;
  r.lo = (const cpx<T>*)P->dd[d].zlo;
  r.hi = (const cpx<T>*)P->dd[d].zhi;
  r.N = P->dp[d].q * P->dp[d].m;
  r.kbits = P->dd[d].kbits;
  return r;
}

// rows of the innermost dimension: nrows rows of length dp.L, row stride dp.L,
// or (tasks != NULL) nrows independent rows described by a device task table
// `b` selects the output of a quadratic multiplication operator, whose
// shares run one after another into the same output; `skip_fwd` reuses the
// column pass of the previous output (one residue block only).
template <typename T>
static int run_rows(Plan* P, const cpx<T>* const* in, cpx<T>* out, int64_t nrows, hipStream_t s,
                    const RowTask<T>* tasks = nullptr, int64_t row_stride = 0, int b = 0, bool skip_fwd = false) {
  const int d = P->dims - 1;
  const DimPlan& dp = P->dp[d];
  const int A = P->A;
  const std::vector<Share>& shares = P->shares[b];
  const int nsh = (int)shares.size();
  // words between consecutive rows of the inputs and the output (default: dense)
  const int64_t rs = row_stride ? row_stride : stored_extent(dp);
  hipError_t e;
  if (dp.variant == VAR_FUSED && !tasks && nsh == 1 && !P->quad && dp.p <= 2 && !dp.ctr && !dp.herm && in &&
      rows_lean_supported((int)dp.m, dp.E_m, shares[0].n, (int)dp.q, (int)sizeof(T))) {
    // many rows of one or two blocks: the lean row kernel (the same arithmetic)
    const Share& sh = shares[0];
    LeanRowArgs<T> a{};
    for (int i = 0; i < sh.n; ++i) a.in[i] = in[sh.idx[i]];
    a.out = out;
    a.in_stride = a.out_stride = rs;
    a.nrows = nrows;
    a.L = (uint32_t)dp.L;
    a.q = (int)dp.q;
    a.scale = (T)(1.0 / ((double)dp.q * (double)dp.m));
    a.fd = dp.fd_m;
    a.fft_tw = (const cpx<T>*)P->dd[d].fft_m;
    a.zqm = rtab<T>(P, d);
    ProfScope ps(P, s, "rows_lean", (double)nrows * (sh.n + 1) * (double)dp.L * 2.0 * sizeof(T));
    e = launch_rows_lean<T>(a, dp.E_m, sh.n, P->cus, s);
    if (e != hipSuccess) return hip_err(e, "rows_lean launch");
    return HDCONV_OK;
  }
  if (dp.variant == VAR_FUSED) {
    for (int k = 0; k < nsh; ++k) {
      const Share& sh = shares[k];
      FusedArgs<T> a{};
      a.tasks = tasks;
      for (int i = 0; i < sh.n; ++i) a.in[i] = in ? in[sh.idx[i]] : nullptr;
      a.out = out;
      a.in_stride = a.out_stride = rs;
      a.nrows = nrows;
      a.L = dp.L;
      a.m = (int)dp.m;
      a.q = (int)dp.q;
      a.rows_per_block = dp.rows_per_block;
      a.ctr = dp.ctr;
      a.herm = dp.herm;
      // paired real residue transforms (measured: 2047 x 2048 FP32 inner rows
      // 160 -> 134 us, L = 4096 42 -> 34 us)
      a.pair = dp.herm;
      a.quad = quad_of<T>(P, sh);
      a.out_add = k > 0;
      a.scale = (T)(1.0 / ((double)dp.q * (double)dp.m));
      a.fd = dp.fd_m;
      a.fft_tw = (const cpx<T>*)P->dd[d].fft_m;
      a.zqm = rtab<T>(P, d);
      const double wb = 2.0 * sizeof(T);
      ProfScope ps(P, s, "fused1d", (double)nrows * (sh.n + 1 + (k > 0)) * (double)stored_extent(dp) * wb);
      e = launch_fused1d<T>(a, dp.E_m, (int)dp.p, sh.n, s);
      if (e != hipSuccess) return hip_err(e, "fused1d launch");
    }
    return HDCONV_OK;
  }
  // inner form, blocks of D residues; every block adds each share of the
  // output to the FP64 accumulator unless one contribution is all there is
  const int64_t nblk = cdiv(dp.n, dp.D);
  const int64_t ncontrib = nblk * nsh;
  for (int64_t blk = 0; blk < nblk; ++blk) {
    const int v0 = (int)(blk * dp.D);
    const int D = (int)std::min<int64_t>(dp.D, dp.n - v0);
    const double wb = 2.0 * sizeof(T);
    // forward column pass, three inputs per launch
    for (int g0 = 0; g0 < A && !skip_fwd; g0 += kMaxA) {
      const int na = std::min(kMaxA, A - g0);
      ColFwdArgs<T> k1{};
      k1.tasks = tasks;
      for (int i = 0; i < na; ++i) {
        k1.in[i] = in ? in[g0 + i] : nullptr;
        k1.work[i] = (cpx<T>*)P->rowwork[g0 + i];
      }
      k1.in_stride = rs;
      k1.nrows = nrows;
      k1.L = dp.L;
      k1.m = (int)dp.m;
      k1.p = (int)dp.p;
      k1.q = (int)dp.q;
      k1.v0 = v0;
      k1.D = D;
      k1.S = dp.S;
      k1.ctr = dp.ctr;
      k1.fold = centered_folds(dp) ? 1 : 0;
      k1.herm = dp.herm;
      k1.pair = (P->conj_pairs && !dp.ctr && !k1.fold && !dp.herm && v0 == 0 && D == dp.n && dp.n >= 3) ? 1 : 0;
      k1.fd = dp.fd_p;
      k1.fft_tw = (const cpx<T>*)P->dd[d].fft_p;
      k1.zq = (const cpx<T>*)P->dd[d].zq;
      ProfScope ps(P, s, "cols_fwd", (double)nrows * na * ((double)stored_extent(dp) + (double)D * dp.p * dp.m) * wb);
      e = launch_cols_fwd<T>(k1, dp.E_p, na, s);
      if (e != hipSuccess) return hip_err(e, "cols_fwd launch");
    }
    for (int k = 0; k < nsh; ++k) {
      const Share& sh = shares[k];
      RowConvArgs<T> k2{};
      for (int i = 0; i < sh.n; ++i) k2.work[i] = (cpx<T>*)P->rowwork[sh.idx[i]];
      // quadratic operators keep the transformed inputs for the other outputs
      k2.out = P->quad ? (cpx<T>*)P->rowout : nullptr;
      k2.quad = quad_of<T>(P, sh);
      k2.nrows = nrows * D * dp.p;
      k2.m = (int)dp.m;
      k2.p = (int)dp.p;
      k2.n = (int)dp.n;
      k2.v0 = v0;
      k2.D = D;
      k2.rows_per_block = dp.rows_per_block;
      // two real-output rows per transform: FP64 (transform-bound), or FP32
      // when the rows are plenty (pairing halves the slots; with few rows that
      // leaves CUs idle, measured slower at 384 rows)
      k2.herm = dp.herm && (sizeof(T) == 8 || k2.nrows >= 2048);
      k2.qm = dp.q * dp.m;
      k2.fd = dp.fd_m;
      k2.fft_tw = (const cpx<T>*)P->dd[d].fft_m;
      k2.zqm = rtab<T>(P, d);
      {
        ProfScope ps(P, s, "rows_conv", (double)nrows * D * dp.p * dp.m * (sh.n + 1) * wb);
        e = launch_rows_conv<T>(k2, dp.E_m, sh.n, s);
      }
      if (e != hipSuccess) return hip_err(e, "rows_conv launch");

      const int64_t ci = blk * nsh + k;  // this contribution's place in the sum
      ColBwdArgs<T> k3{};
      k3.tasks = tasks;
      k3.work = (const cpx<T>*)(P->quad ? P->rowout : P->rowwork[0]);
      k3.out = out;
      k3.acc = P->acc64;
      if (P->flags & HDCONV_PLAN_ACCUMULATE_OUTPUT)  // the first contribution writes, later ones add
        k3.acc_mode = ci == 0 ? ACC_WRITE : ACC_OUT_ADD;
      else
        k3.acc_mode = ncontrib == 1 ? ACC_WRITE : (ci == 0 ? ACC_FIRST : (ci == ncontrib - 1 ? ACC_LAST : ACC_ADD));
      k3.out_stride = rs;
      k3.nrows = nrows;
      k3.L = dp.L;
      k3.m = (int)dp.m;
      k3.p = (int)dp.p;
      k3.q = (int)dp.q;
      k3.v0 = v0;
      k3.D = D;
      k3.S = dp.S;
      k3.ctr = dp.ctr;
      k3.fold = centered_folds(dp) ? 1 : 0;
      k3.herm = dp.herm;
      k3.scale = (T)(1.0 / ((double)dp.q * (double)dp.m));
      k3.fd = dp.fd_pb;
      k3.fft_tw = (const cpx<T>*)P->dd[d].fft_p;
      k3.zq = (const cpx<T>*)P->dd[d].zq;
      {
        const double Lw = (double)stored_extent(dp);
        const double accb = k3.acc_mode == ACC_WRITE ? Lw * wb
                            : (k3.acc_mode == ACC_FIRST ? 16.0 * Lw
                                                        : (k3.acc_mode == ACC_ADD ? 32.0 * Lw : 16.0 * Lw + Lw * wb));
        ProfScope ps(P, s, "cols_bwd", (double)nrows * ((double)D * dp.p * dp.m * wb + accb));
        e = launch_cols_bwd<T>(k3, dp.E_pb, s);
      }
      if (e != hipSuccess) return hip_err(e, "cols_bwd launch");
    }
  }
  return HDCONV_OK;
}

// One execute.  Hybrid plans take all copies in the same launches (the
// copies are the first level's planes, or the rows of a 1D plan); `nc` is
// the number of copies this call covers (the explicit method calls it once
// per copy with nc = 1).
template <typename T>
static int run_copies(Plan* P, const void* const* inputs, void* const* outputs, hipStream_t s, int64_t nc) {
  const int A = P->A;
  // outputs computed one after another (quadratic operators), each through
  // the row pass and the outer inverse passes; the forward passes run once
  const int nout = P->quad ? P->B : 1;
  const int Aeff = P->quad ? 2 : A;  // factors per product (window offsets)
  hipError_t e;
  int64_t Le[3];
  for (int d = 0; d < P->dims; ++d) Le[d] = P->dp[d].L;
  // words between copies in the user's arrays (default: one copy's extent)
  const int64_t dist = nc > 1 ? P->dist : (P->span ? P->span : 1);
  // the user's layout in the first outer pass (strided 2D/3D arrays; the
  // explicit method reads and writes the user's arrays in its copies only)
  ColLayout user{};
  if (P->dims >= 2 && (P->stride[0] || P->stride[1]) && P->method != HDCONV_METHOD_EXPLICIT) {
    const int64_t s1 = P->dims == 3 ? (P->stride[1] ? P->stride[1] : P->Lio[2]) : 1;
    user.jstride = P->stride[0] ? P->stride[0] : P->Lio[1] * s1;
    if (P->dims == 3) {
      user.cgrp = P->Lio[2];
      user.cgstride = s1;
    }
  }
  const cpx<T>* cur[kMaxIn];
  // where the engine leaves output b: the user's array, or for the explicit
  // method its padded buffer (in place over the first input for products)
  auto engine_out = [&](int b) -> cpx<T>* {
    if (P->method != HDCONV_METHOD_EXPLICIT) return (cpx<T>*)outputs[b];
    return (cpx<T>*)(P->quad ? P->padout : P->pad_in[0]);
  };
  if (P->method == HDCONV_METHOD_EXPLICIT) {
    for (int a = 0; a < A; ++a) {
      BoxCopyArgs<T> b{};
      b.src = (const cpx<T>*)inputs[a];
      b.dst = (cpx<T>*)P->pad_in[a];
      for (int k = 0; k < 3; ++k) b.L[k] = b.N[k] = 1;
      for (int d = 0; d < P->dims; ++d) {
        b.L[3 - P->dims + d] = P->Lio[d];
        b.N[3 - P->dims + d] = P->npad[d];
      }
      b.pad = 1;
      if (P->dims >= 2) {  // the user's strides (0: dense)
        b.ls[3 - P->dims] = P->stride[0];
        if (P->dims == 3) b.ls[1] = P->stride[1];
      }
      if (P->flags & HDCONV_PLAN_HERMITIAN) {  // the expanded centered array
        b.herm = 1;
        b.hH = P->Lio[P->dims - 1] - 1;
      }
      {
        double lt = 1, nt = 1;
        for (int d = 0; d < P->dims; ++d) {
          lt *= (double)P->Lio[d];
          nt *= (double)P->npad[d];
        }
        ProfScope ps(P, s, "pad", (lt + nt) * 2.0 * sizeof(T));
        e = launch_box_copy<T>(b, s);
      }
      if (e != hipSuccess) return hip_err(e, "pad launch");
      cur[a] = (const cpx<T>*)P->pad_in[a];
    }
  } else {
    for (int a = 0; a < A; ++a) cur[a] = (const cpx<T>*)inputs[a];
  }
  // Residue blocks of the first outer dimension (Sec. 5: one block of D
  // residues at a time through the inner dimensions, buffers reused): every
  // block runs the whole pipeline, its inverse adds to the output.
  const cpx<T>* cur0[kMaxIn];
  for (int a = 0; a < A; ++a) cur0[a] = cur[a];
  const int64_t q0 = P->dims > 1 ? P->dp[0].q : 1;
  const int64_t D0 = P->dims > 1 ? (outer_inner(P->dp[0]) ? q0 : P->dp[0].D) : 1;
  for (int64_t r0 = 0; r0 < q0; r0 += D0) {
  const int Db = (int)std::min<int64_t>(D0, q0 - r0);
  for (int a = 0; a < A; ++a) cur[a] = cur0[a];
  // outer dimensions, forward
  int64_t nb = nc;
  for (int d = 0; d + 1 < P->dims; ++d) {
    // residues of this launch: the block's on the first dimension, all on the others
    const int rr0 = d == 0 ? (int)r0 : 0;
    const int nres = d == 0 ? Db : (int)P->dp[d].q;
    const DimPlan& dp = P->dp[d];
    int64_t rest = 1;
    for (int k = d + 1; k < P->dims; ++k) rest *= stored_extent(P->dp[k]);
    // the lean outer kernel for ordinary dimensions of one block over dense planes
    const bool dense = d > 0 || (user.jstride == 0 && user.cgrp == 0);
    if (outer_inner(dp)) {
      // the inner form: column passes into the level, then the m-point pass in place
      if (!dense) return set_err(HDCONV_EUNSUPPORTED, "the inner form of an outer dimension takes dense arrays");
      for (int g0 = 0; g0 < A; g0 += kMaxA) {
        const int na = std::min(kMaxA, A - g0);
        OuterColArgs<T> o{};
        OuterLeanArgs<T> r{};
        for (int a = 0; a < na; ++a) {
          o.in[a] = cur[g0 + a];
          o.out[a] = r.out[a] = (cpx<T>*)P->lvl[d][g0 + a];
          r.in[a] = o.out[a];
        }
        o.na = r.na = na;
        o.nb = nb;
        o.in_bstride = d == 0 ? dist : Le[d] * rest;
        o.R = r.R = rest;
        o.L = Le[d];
        o.m = (int)dp.m;
        o.n = (int)dp.n;
        o.fd = dp.fd_p;
        o.fft_tw = (const cpx<T>*)P->dd[d].fft_p;
        o.zq = (const cpx<T>*)P->dd[d].zq;
        const double lvl_el = (double)nb * dp.q * dp.m * rest;
        {
          ProfScope ps(P, s, "outer_cols_fwd", ((double)nb * Le[d] * rest + lvl_el) * na * 2.0 * sizeof(T));
          e = launch_outer_cols<T>(o, (int)dp.p, true, P->cus, s);
        }
        if (e != hipSuccess) return hip_err(e, "outer_cols_fwd launch");
        r.nb = nb * dp.q;
        r.in_bstride = dp.m * rest;
        r.L = (uint32_t)dp.m;
        r.q = (int)dp.q;
        r.D = 1;
        r.inner_n = (int)dp.n;
        r.fd = dp.fd_m;
        r.fft_tw = (const cpx<T>*)P->dd[d].fft_m;
        r.zqm = rtab<T>(P, d);
        {
          ProfScope ps(P, s, "outer_rows_fwd", 2.0 * lvl_el * na * 2.0 * sizeof(T));
          e = launch_outer_lean<T>(r, dp.E_m, dp.S, true, P->cus, s);
        }
        if (e != hipSuccess) return hip_err(e, "outer_rows_fwd launch");
      }
      for (int a = 0; a < A; ++a) cur[a] = (const cpx<T>*)P->lvl[d][a];
      nb *= dp.q * dp.m;
      continue;
    }
    const bool lean = dense && !dp.ctr && dp.p <= 2 && outer_lean_supported((int)dp.m, dp.E_m, dp.S, (int)dp.q, (int)sizeof(T));
    for (int g0 = 0; g0 < A && lean; g0 += kMaxA) {
      const int na = std::min(kMaxA, A - g0);
      OuterLeanArgs<T> o{};
      for (int a = 0; a < na; ++a) {
        o.in[a] = cur[g0 + a];
        o.out[a] = (cpx<T>*)P->lvl[d][g0 + a];
      }
      o.na = na;
      o.nb = nb;
      o.in_bstride = d == 0 ? dist : Le[d] * rest;
      o.R = rest;
      o.L = (uint32_t)Le[d];
      o.q = (int)dp.q;
      o.r0 = rr0;
      o.D = nres;
      o.fd = dp.fd_m;
      o.fft_tw = (const cpx<T>*)P->dd[d].fft_m;
      o.zqm = rtab<T>(P, d);
      {
        ProfScope ps(P, s, "outer_lean_fwd",
                     (double)nb * na * ((double)Le[d] + (double)nres * dp.m) * rest * 2.0 * sizeof(T));
        e = launch_outer_lean<T>(o, dp.E_m, dp.S, true, P->cus, s);
      }
      if (e != hipSuccess) return hip_err(e, "outer_lean_fwd launch");
    }
    for (int g0 = 0; g0 < A && !lean; g0 += kMaxA) {  // three inputs per launch
      const int na = std::min(kMaxA, A - g0);
      OuterFwdArgs<T> o{};
      for (int a = 0; a < na; ++a) {
        o.in[a] = cur[g0 + a];
        o.out[a] = (cpx<T>*)P->lvl[d][g0 + a];
      }
      o.nb = nb;
      o.in_bstride = d == 0 ? dist : Le[d] * rest;  // the user's copies are dist apart
      if (d == 0) o.lay = user;
      o.R = rest;
      o.L = Le[d];
      o.m = (int)dp.m;
      o.q = (int)dp.q;
      o.r0 = rr0;
      o.D = nres;
      o.S = dp.S;
      o.ctr = dp.ctr;
      o.fd = dp.fd_m;
      o.fft_tw = (const cpx<T>*)P->dd[d].fft_m;
      o.zqm = rtab<T>(P, d);
      {
        ProfScope ps(P, s, "outer_fwd", (double)nb * na * ((double)Le[d] + (double)nres * dp.m) * rest * 2.0 * sizeof(T));
        e = launch_outer_fwd<T>(o, dp.E_m, (int)dp.p, na, s);
      }
      if (e != hipSuccess) return hip_err(e, "outer_fwd launch");
    }
    for (int a = 0; a < A; ++a) cur[a] = (const cpx<T>*)P->lvl[d][a];
    nb *= nres * dp.m;
  }
  const int64_t nb_rows = nb;
  for (int ob = 0; ob < nout; ++ob) {
    nb = nb_rows;
    cpx<T>* final_out = engine_out(ob);
    // innermost rows (products: in place over the first input's level)
    cpx<T>* rows_out = P->dims == 1 ? final_out
                                    : (cpx<T>*)(P->quad ? P->outbuf : P->lvl[P->dims - 2][0]);
    {
      const bool one_block = P->dp[P->dims - 1].variant != VAR_MULTI ||
                             P->dp[P->dims - 1].D >= P->dp[P->dims - 1].n;
      int rc = run_rows<T>(P, cur, rows_out, nb, s, nullptr, P->dims == 1 ? dist : 0, ob, ob > 0 && one_block);
      if (rc != HDCONV_OK) return rc;
    }
    // outer dimensions, backward (the first level's transformed inputs are
    // free by now and carry the intermediate levels of every output)
    const cpx<T>* yl = rows_out;
    for (int d = P->dims - 2; d >= 0; --d) {
      const DimPlan& dp = P->dp[d];
      const int rr0 = d == 0 ? (int)r0 : 0;
      const int nres = d == 0 ? Db : (int)dp.q;
      const bool add = d == 0 && r0 > 0;  // later blocks add to the output
      nb /= nres * dp.m;
      int64_t rest = 1;
      for (int k = d + 1; k < P->dims; ++k) rest *= stored_extent(P->dp[k]);
      const bool dense = d > 0 || (user.jstride == 0 && user.cgrp == 0);
      if (outer_inner(dp)) {
        // the m-point pass in place over the level, then the column pass into the output
        OuterLeanArgs<T> r{};
        r.in[0] = yl;
        r.out[0] = (cpx<T>*)yl;
        r.nb = nb * dp.q;
        r.out_bstride = dp.m * rest;
        r.R = rest;
        r.L = (uint32_t)dp.m;
        r.q = (int)dp.q;
        r.D = 1;
        r.inner_n = (int)dp.n;
        r.scale = (T)1;
        r.fd = dp.fd_m;
        r.fft_tw = (const cpx<T>*)P->dd[d].fft_m;
        r.zqm = rtab<T>(P, d);
        const double lvl_el = (double)nb * dp.q * dp.m * rest;
        {
          ProfScope ps(P, s, "outer_rows_bwd", 2.0 * lvl_el * 2.0 * sizeof(T));
          e = launch_outer_lean<T>(r, dp.E_m, dp.S, false, P->cus, s);
        }
        if (e != hipSuccess) return hip_err(e, "outer_rows_bwd launch");
        OuterColArgs<T> o{};
        o.in[0] = yl;
        o.out[0] = d == 0 ? final_out : (cpx<T>*)P->lvl[d - 1][0];
        o.nb = nb;
        o.out_bstride = d == 0 ? dist : Le[d] * rest;
        o.R = rest;
        o.L = Le[d];
        o.m = (int)dp.m;
        o.n = (int)dp.n;
        o.add = add ? 1 : 0;
        o.scale = (T)(1.0 / ((double)dp.q * (double)dp.m));
        o.fd = dp.fd_p;
        o.fft_tw = (const cpx<T>*)P->dd[d].fft_p;
        o.zq = (const cpx<T>*)P->dd[d].zq;
        {
          ProfScope ps(P, s, "outer_cols_bwd", (lvl_el + (add ? 2.0 : 1.0) * (double)nb * Le[d] * rest) * 2.0 * sizeof(T));
          e = launch_outer_cols<T>(o, (int)dp.p, false, P->cus, s);
        }
        if (e != hipSuccess) return hip_err(e, "outer_cols_bwd launch");
        yl = o.out[0];
        continue;
      }
      if (dense && !dp.ctr && dp.p <= 2 && outer_lean_supported((int)dp.m, dp.E_m, dp.S, (int)dp.q, (int)sizeof(T))) {
        OuterLeanArgs<T> o{};
        o.in[0] = yl;
        o.out[0] = d == 0 ? final_out : (cpx<T>*)P->lvl[d - 1][0];
        o.nb = nb;
        o.out_bstride = d == 0 ? dist : Le[d] * rest;
        o.R = rest;
        o.L = (uint32_t)Le[d];
        o.q = (int)dp.q;
        o.r0 = rr0;
        o.D = nres;
        o.add = add ? 1 : 0;
        o.scale = (T)(1.0 / ((double)dp.q * (double)dp.m));
        o.fd = dp.fd_m;
        o.fft_tw = (const cpx<T>*)P->dd[d].fft_m;
        o.zqm = rtab<T>(P, d);
        {
          ProfScope ps(P, s, "outer_lean_bwd",
                       (double)nb * ((add ? 2.0 : 1.0) * (double)Le[d] + (double)nres * dp.m) * rest * 2.0 * sizeof(T));
          e = launch_outer_lean<T>(o, dp.E_m, dp.S, false, P->cus, s);
        }
        if (e != hipSuccess) return hip_err(e, "outer_lean_bwd launch");
        yl = o.out[0];
        continue;
      }
      OuterBwdArgs<T> o{};
      o.y = yl;
      o.out = d == 0 ? final_out : (cpx<T>*)P->lvl[d - 1][0];
      o.acc = nullptr;
      o.acc_mode = add ? ACC_OUT_ADD : ACC_WRITE;
      o.nb = nb;
      o.out_bstride = d == 0 ? dist : Le[d] * rest;
      if (d == 0) o.lay = user;
      o.R = rest;
      o.L = Le[d];
      o.m = (int)dp.m;
      o.q = (int)dp.q;
      o.r0 = rr0;
      o.D = nres;
      o.S = dp.S;
      o.ctr = dp.ctr;
      o.scale = (T)(1.0 / ((double)dp.q * (double)dp.m));
      o.fd = dp.fd_m;
      o.fft_tw = (const cpx<T>*)P->dd[d].fft_m;
      o.zqm = rtab<T>(P, d);
      {
        ProfScope ps(P, s, "outer_bwd",
                     (double)nb * ((add ? 2.0 : 1.0) * (double)Le[d] + (double)nres * dp.m) * rest * 2.0 * sizeof(T));
        e = launch_outer_bwd<T>(o, dp.E_m, (int)dp.p, s);
      }
      if (e != hipSuccess) return hip_err(e, "outer_bwd launch");
      yl = o.out;
    }
    if (P->method == HDCONV_METHOD_EXPLICIT) {
      BoxCopyArgs<T> b{};
      b.src = final_out;
      b.dst = (cpx<T>*)outputs[ob];
      for (int k = 0; k < 3; ++k) b.L[k] = b.N[k] = 1;
      for (int d = 0; d < P->dims; ++d) {
        b.L[3 - P->dims + d] = P->Lio[d];
        b.N[3 - P->dims + d] = P->npad[d];
        // centered: entries (F-1)H .. (F-1)H+L-1 of the padded product of F
        // factors are the outputs -H .. L-1-H (the arrays were padded as they
        // are, index c at position c + H, so a product of F of them sits F H
        // further on); Hermitian: the outputs c >= 0 start at F H (H = Lh - 1)
        if ((P->flags & HDCONV_PLAN_HERMITIAN) && d == P->dims - 1)
          b.off[3 - P->dims + d] = (int64_t)Aeff * (P->Lio[d] - 1);
        else if (P->flags & (HDCONV_PLAN_CENTERED | HDCONV_PLAN_HERMITIAN))
          b.off[3 - P->dims + d] = (int64_t)(Aeff - 1) * (P->L[d] / 2);
      }
      b.pad = 0;
      if (P->dims >= 2) {
        b.ls[3 - P->dims] = P->stride[0];
        if (P->dims == 3) b.ls[1] = P->stride[1];
      }
      {
        double lt = 1;
        for (int d = 0; d < P->dims; ++d) lt *= (double)P->Lio[d];
        ProfScope ps(P, s, "truncate", 2.0 * lt * 2.0 * sizeof(T));
        e = launch_box_copy<T>(b, s);
      }
      if (e != hipSuccess) return hip_err(e, "truncate launch");
    }
  }
  }  // residue blocks of the first outer dimension
  return HDCONV_OK;
}

template <typename T>
static int run_plan(Plan* P, const void* const* inputs, void* const* outputs, hipStream_t s) {
  if (P->method != HDCONV_METHOD_EXPLICIT || P->copies == 1) return run_copies<T>(P, inputs, outputs, s, P->copies);
  // the explicit baseline pads one copy at a time into its work buffers
  for (int64_t c = 0; c < P->copies; ++c) {
    const void* in_c[kMaxIn];
    void* out_c[kMaxB];
    for (int a = 0; a < P->A; ++a) in_c[a] = (const cpx<T>*)inputs[a] + c * P->dist;
    for (int b = 0; b < P->B; ++b) out_c[b] = (cpx<T>*)outputs[b] + c * P->dist;
    int rc = run_copies<T>(P, in_c, out_c, s, 1);
    if (rc != HDCONV_OK) return rc;
  }
  return HDCONV_OK;
}

// ---------------------------------------------------------------------------
// C ABI

extern "C" {

void hdconv_options_init(hdconv_options* opt) {
  if (opt) memset(opt, 0, sizeof(*opt));
}

const char* hdconv_version(void) { return "hdconv 0.1 (gfx950)"; }

int hdconv_last_error(char* msg, size_t cap) {
  if (msg && cap) {
    strncpy(msg, g_err_msg, cap - 1);
    msg[cap - 1] = 0;
  }
  return g_err_code;
}

int hdconv_geometry(int64_t L, int64_t M, int64_t m, int64_t p_min, int force_inner, hdconv_dim_info_t* out) {
  clear_err();
  if (!out) return set_err(HDCONV_EINVAL, "out is NULL");
  if (L < 1 || M < 1 || m < 1 || p_min < 0) return set_err(HDCONV_EINVAL, "need L, M, m >= 1 and p_min >= 0");
  Geometry g = geometry(L, M, m, p_min, force_inner != 0);
  memset(out, 0, sizeof(*out));
  out->L = L;
  out->M = M;
  out->m = g.m;
  out->p = g.p;
  out->n = g.n;
  out->q = g.q;
  out->D = g.n;
  out->variant = g.inner ? HDCONV_VARIANT_MULTIPASS : HDCONV_VARIANT_FUSED;
  return HDCONV_OK;
}

int hdconv_geometry_ex(int64_t L, int64_t M, int64_t m, int64_t p_min, int force_inner, int flags,
                       hdconv_dim_info_t* out) {
  clear_err();
  if (!out) return set_err(HDCONV_EINVAL, "out is NULL");
  if (L < 1 || M < 1 || m < 1 || p_min < 0) return set_err(HDCONV_EINVAL, "need L, M, m >= 1 and p_min >= 0");
  if (flags & ~(HDCONV_PLAN_CENTERED | HDCONV_PLAN_HERMITIAN))
    return set_err(HDCONV_EINVAL, "flags may hold HDCONV_PLAN_CENTERED and HDCONV_PLAN_HERMITIAN only");
  const bool herm = (flags & HDCONV_PLAN_HERMITIAN) != 0;
  const int ctr = (flags & (HDCONV_PLAN_CENTERED | HDCONV_PLAN_HERMITIAN)) ? 1 : 0;
  const int64_t Le = herm ? herm_full(L) : L;  // the centered length a Hermitian half stands for
  Geometry g = geometry_c(Le, M, m, p_min, force_inner != 0, ctr);
  memset(out, 0, sizeof(*out));
  out->L = Le;
  out->M = M;
  out->m = g.m;
  out->p = g.p;
  out->n = g.n;
  out->q = g.q;
  out->D = g.n;
  out->variant = g.inner ? HDCONV_VARIANT_MULTIPASS : HDCONV_VARIANT_FUSED;
  out->centered = herm ? 2 : ctr;
  return HDCONV_OK;
}

int64_t hdconv_centered_span(int64_t L, int64_t m) {
  if (L < 1 || m < 1) return 0;
  return centered_blocks(L, m);
}

int hdconv_min_padding(int64_t L, int A, int flags, int64_t* M) {
  clear_err();
  if (!M) return set_err(HDCONV_EINVAL, "M is NULL");
  if (L < 1 || A < 2 || A > kMaxA) return set_err(HDCONV_EINVAL, "need L >= 1 and A in 2 .. %d", kMaxA);
  if (flags & ~(HDCONV_PLAN_CENTERED | HDCONV_PLAN_HERMITIAN))
    return set_err(HDCONV_EINVAL, "flags may hold HDCONV_PLAN_CENTERED and HDCONV_PLAN_HERMITIAN only");
  if (flags & HDCONV_PLAN_HERMITIAN)
    *M = centered_min_padding(herm_full(L), A);
  else if (flags & HDCONV_PLAN_CENTERED)
    *M = centered_min_padding(L, A);
  else
    *M = (int64_t)A * (L - 1) + 1;
  return HDCONV_OK;
}

hdconv_plan_t hdconv_plan_ex(const int64_t* L, const int64_t* M, int A, int B, int dims, int dtype,
                     const hdconv_options* opt) {
  clear_err();
  if (!L || !M) {
    set_err(HDCONV_EINVAL, "L and M must not be NULL");
    return nullptr;
  }
  if (dims < 1 || dims > 3) {
    set_err(HDCONV_EINVAL, "dims must be 1, 2 or 3 (got %d)", dims);
    return nullptr;
  }
  const bool quad = opt && opt->mult == HDCONV_MULT_QUADRATIC;
  // products multiply two or three transforms; quadratic operators take up to
  // six inputs (their outputs sum pairs)
  if (A < 2 || A > (quad ? kMaxIn : kMaxA)) {
    set_err(HDCONV_EUNSUPPORTED, "A must be 2 or 3 (quadratic operators: 2 ... %d; got %d)", kMaxIn, A);
    return nullptr;
  }
  if (opt && opt->mult != HDCONV_MULT_PRODUCT && !quad) {
    set_err(HDCONV_EINVAL, "unknown multiplication operator %d", opt->mult);
    return nullptr;
  }
  if (!quad && B != 1) {
    set_err(HDCONV_EUNSUPPORTED, "the product operator has B = 1 output (got %d); use HDCONV_MULT_QUADRATIC", B);
    return nullptr;
  }
  if (quad && (B < 1 || B > kMaxB || !opt->mult_coef)) {
    set_err(HDCONV_EINVAL, "a quadratic operator needs 1 <= B <= %d and its coefficients (got B = %d)", kMaxB, B);
    return nullptr;
  }
  if (quad && opt->tuner != HDCONV_TUNER_HEURISTIC) {
    set_err(HDCONV_EUNSUPPORTED, "quadratic operators use the heuristic planner");
    return nullptr;
  }
  if (dtype != HDCONV_C64 && dtype != HDCONV_C128) {
    set_err(HDCONV_EINVAL, "dtype must be HDCONV_C64 or HDCONV_C128 (got %d)", dtype);
    return nullptr;
  }
  const bool herm = opt && (opt->flags & HDCONV_PLAN_HERMITIAN);
  // 2D/3D Hermitian: the outer dimensions are centered with a symmetric index
  // range, so their extents are odd
  for (int d = 0; herm && d + 1 < dims; ++d)
    if (L[d] % 2 == 0) {
      set_err(HDCONV_EINVAL, "Hermitian plans need odd outer extents (L[%d] = %lld)", d, (long long)L[d]);
      return nullptr;
    }
  for (int d = 0; d < dims; ++d) {
    if (L[d] < 1 || L[d] > (int64_t(1) << 31)) {
      set_err(HDCONV_EINVAL, "L[%d] = %lld out of range", d, (long long)L[d]);
      return nullptr;
    }
    const bool ctr = opt && (opt->flags & (HDCONV_PLAN_CENTERED | HDCONV_PLAN_HERMITIAN));
    const bool hd = herm && d == dims - 1;
    const int F = quad ? 2 : A;  // factors per product
    const int64_t Mmin = hd ? centered_min_padding(herm_full(L[d]), F)
                            : (ctr ? centered_min_padding(L[d], F) : (int64_t)F * (L[d] - 1) + 1);
    if (M[d] < Mmin) {
      set_err(HDCONV_EINVAL, "M[%d] = %lld is below %s = %lld, so the product would alias", d, (long long)M[d],
              hd ? "the Hermitian minimum (F+1)(ceil(L/2)-1)+1 (F factors per product)"
                 : (ctr ? "the centered minimum max(F(L-1-H)+H, L-1-H+FH)+1 (F factors per product)"
                        : "F(L-1)+1 (F factors per product)"),
              (long long)Mmin);
      return nullptr;
    }
  }
  if (opt && opt->tuner != HDCONV_TUNER_HEURISTIC && opt->method != HDCONV_METHOD_EXPLICIT &&
      !(opt->flags & HDCONV_PLAN_HOST_ONLY)) {
    // tuned plan: choose every dimension's shape, then build it like a forced plan
    hdconv_dim_info_t shp[3];
    int nc = 0, nt = 0;
    double ms = 0;
    if (tune_shapes(L, M, A, B, dims, dtype, opt, shp, &nc, &nt, &ms) != HDCONV_OK) return nullptr;
    hdconv_options o = opts_from_shape(shp, dims);
    o.flags = opt->flags;
    o.copies = opt->copies;
    o.dist = opt->dist;
    o.stride[0] = opt->stride[0];
    o.stride[1] = opt->stride[1];
    o.conj_pairs = opt->conj_pairs;
    Plan* T = (Plan*)hdconv_plan_ex(L, M, A, B, dims, dtype, &o);
    if (T) {
      T->tuner = opt->tuner;
      T->tuned_candidates = nc;
      T->timed_candidates = nt;
      T->tuned_ms = ms;
    }
    return (hdconv_plan_t)T;
  }
  Plan* P = new (std::nothrow) Plan();
  if (!P) {
    set_err(HDCONV_ENOMEM, "host allocation failed");
    return nullptr;
  }
  P->dims = dims;
  P->A = A;
  P->B = B;
  P->dtype = dtype;
  P->method = (opt && opt->method == HDCONV_METHOD_EXPLICIT) ? HDCONV_METHOD_EXPLICIT : HDCONV_METHOD_HYBRID;
  P->flags = opt ? opt->flags : 0;
  P->host_only = (P->flags & HDCONV_PLAN_HOST_ONLY) != 0;
  P->conj_pairs = !(opt && opt->conj_pairs < 0);
  // coef is B x A x A (row-major); the pair (i, j), i <= j, weighs F_i F_j
  P->quad = quad ? 1 : 0;
  for (int b = 0; b < B; ++b) {
    double c[kMaxIn * kMaxIn] = {};
    for (int i = 0; quad && i < A; ++i)
      for (int j = i; j < A; ++j) c[i * A + j] = opt->mult_coef[(b * A + i) * A + j];
    P->shares[b] = make_shares(A, c);
  }
  {
    int64_t ext[3];
    for (int d = 0; d < dims; ++d) ext[d] = (herm && d == dims - 1) ? (L[d] + 1) / 2 : L[d];
    // element strides of the outer dimensions (dense unless given)
    int64_t st[3] = {0, 0, 1};
    st[dims - 1] = 1;
    for (int d = dims - 2; d >= 0; --d) {
      const int64_t dense = ext[d + 1] * st[d + 1];
      const int64_t want = (opt && opt->stride[d] > 0) ? opt->stride[d] : dense;
      if (want < dense) {
        set_err(HDCONV_EINVAL, "stride[%d] = %lld is below %lld (rows would overlap)", d, (long long)want,
                (long long)dense);
        free_plan(P);
        return nullptr;
      }
      st[d] = want;
      if (want != dense || (opt && opt->stride[d] > 0)) P->stride[d] = want;
    }
    if (opt && dims == 1 && (opt->stride[0] > 0 || opt->stride[1] > 0)) {
      set_err(HDCONV_EINVAL, "strides apply to the outer dimensions of 2D/3D plans");
      free_plan(P);
      return nullptr;
    }
    const int64_t one = ext[0] * st[0];  // one copy's extent (its last row padded too)
    P->span = one;
    P->copies = (opt && opt->copies > 0) ? opt->copies : 1;
    P->dist = (opt && opt->dist > 0) ? opt->dist : one;
    if (P->dist < one || P->copies > (int64_t(1) << 31)) {
      set_err(HDCONV_EINVAL, "copies must be dist >= %lld words apart (got dist = %lld, copies = %lld)",
              (long long)one, (long long)P->dist, (long long)P->copies);
      free_plan(P);
      return nullptr;
    }
  }
  for (int d = 0; d < dims; ++d) {
    P->L[d] = L[d];
    P->Lio[d] = (herm && d == dims - 1) ? herm_stored(L[d]) : L[d];
    P->M[d] = M[d];
    if (P->method == HDCONV_METHOD_EXPLICIT) P->npad[d] = std::max<int64_t>(8, next_fft_size(M[d]));
  }
  int rc = build_dims(P, opt);
  if (rc == HDCONV_OK) rc = size_workspace(P);
  // over the workspace cap: fewer residues per block of the first outer
  // dimension (Sec. 5's buffer reuse), unless the caller fixed D there
  while (rc == HDCONV_ENOMEM && P->dims > 1 && P->dp[0].variant == VAR_OUTER && P->dp[0].p <= 2 &&
         P->dp[0].D > 1 && !(opt && opt->D[0] > 0)) {
    P->dp[0].D = (P->dp[0].D + 1) / 2;
    clear_err();
    rc = size_workspace(P);
  }
  if (rc != HDCONV_OK) {
    free_plan(P);
    return nullptr;
  }
  if (!P->host_only) {
    int ndev = 0;
    hipError_t e = hipGetDeviceCount(&ndev);
    if (e != hipSuccess || ndev < 1) {
      set_err(HDCONV_ENODEV, "no HIP device available (%s)", hipGetErrorString(e));
      free_plan(P);
      return nullptr;
    }
    e = hipGetDevice(&P->device);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&P->cus, hipDeviceAttributeMultiprocessorCount, P->device);
    if (e != hipSuccess) {
      hip_err(e, "hipGetDevice");
      free_plan(P);
      return nullptr;
    }
    if (P->cus < 1) P->cus = 1;
  }
  if ((rc = alloc_tables(P)) != HDCONV_OK || (rc = alloc_workspace(P)) != HDCONV_OK) {
    free_plan(P);
    return nullptr;
  }
  plan_traffic(P, &P->launches);
  return (hdconv_plan_t)P;
}

hdconv_plan_t hdconv_plan(const int64_t* L, const int64_t* M, int A, int B, int dims, int dtype) {
  return hdconv_plan_ex(L, M, A, B, dims, dtype, nullptr);
}

int hdconv_plan_info(hdconv_plan_t plan, hdconv_plan_info_t* out) {
  clear_err();
  if (!plan || !out) return set_err(HDCONV_EINVAL, "plan and out must not be NULL");
  const Plan* P = (const Plan*)plan;
  memset(out, 0, sizeof(*out));
  out->dims = P->dims;
  out->A = P->A;
  out->B = P->B;
  out->dtype = P->dtype;
  out->method = P->method;
  double ltot = 1;
  for (int d = 0; d < 3; ++d) {
    out->L[d] = d < P->dims ? P->L[d] : 0;
    out->M[d] = d < P->dims ? P->M[d] : 0;
    out->npad[d] = P->npad[d];
    if (d >= P->dims) continue;
    ltot *= (double)P->Lio[d];
    const DimPlan& dp = P->dp[d];
    hdconv_dim_info_t& di = out->dim[d];
    di.L = dp.L;
    di.M = dp.M;
    di.m = dp.m;
    di.p = dp.p;
    di.n = dp.n;
    di.q = dp.q;
    di.D = dp.D;
    di.variant = dp.variant;
    di.E_m = dp.E_m;
    di.E_p = dp.E_p;
    di.S = dp.S;
    di.rows_per_block = dp.rows_per_block;
    di.tw_m = dp.fd_m.N ? dp.fd_m.twmode + 1 : 0;
    di.tw_p = dp.fd_p.N ? dp.fd_p.twmode + 1 : 0;
    di.centered = ((P->flags & HDCONV_PLAN_HERMITIAN) && d == P->dims - 1)
                      ? 2
                      : ((P->flags & (HDCONV_PLAN_CENTERED | HDCONV_PLAN_HERMITIAN)) ? 1 : 0);
  }
  out->workspace_bytes = P->work_bytes;
  out->table_bytes = P->table_bytes;
  out->compulsory_bytes = (double)(P->A + P->B) * ltot * (double)P->copies * 2.0 * tbytes_of(P->dtype);
  out->traffic_bytes = plan_traffic(P, &out->launches);
  out->tuner = P->tuner;
  out->tuned_candidates = P->tuned_candidates;
  out->timed_candidates = P->timed_candidates;
  out->tuned_ms = P->tuned_ms;
  return HDCONV_OK;
}

// Argument checks and the launches of one execute, with the workspace parts
// pointing wherever the caller carved them.
static int execute_plan(Plan* P, const void* const* inputs, void* const* outputs, void* stream) {
  // span of one array: (C-1) dist + one copy's extent
  const size_t bytes =
      2 * (size_t)tbytes_of(P->dtype) * ((size_t)(P->copies - 1) * (size_t)P->dist + (size_t)P->span);
  for (int a = 0; a < P->A; ++a)
    if (!inputs[a]) return set_err(HDCONV_EINVAL, "inputs[%d] is NULL", a);
  for (int b = 0; b < P->B; ++b)
    if (!outputs[b]) return set_err(HDCONV_EINVAL, "outputs[%d] is NULL", b);
  auto overlap = [&](const char* x, const char* y) { return x < y + bytes && y < x + bytes; };
  const char* o = (const char*)outputs[0];
  // several outputs, or one summed over several row-pass launches, are
  // written while inputs are still read: then no output may touch an input
  // (also: residue blocks of the first outer dimension read the inputs again
  // after earlier blocks wrote the output)
  const bool out_of_place = P->B > 1 || max_shares(P) > 1 || (P->dims > 1 && P->dp[0].D < P->dp[0].q) ||
                            (P->flags & HDCONV_PLAN_ACCUMULATE_OUTPUT);
  for (int a = 0; a < P->A; ++a) {
    const char* i = (const char*)inputs[a];
    if (!out_of_place && i != o && overlap(i, o))
      return set_err(HDCONV_EINVAL, "outputs[0] partially overlaps inputs[%d]", a);
    for (int b = 0; out_of_place && b < P->B; ++b)
      if (overlap(i, (const char*)outputs[b]))
        return set_err(HDCONV_EINVAL, "outputs[%d] overlaps inputs[%d] (this operator runs out of place)", b, a);
  }
  for (int b = 0; b < P->B; ++b)
    for (int c = b + 1; c < P->B; ++c)
      if (overlap((const char*)outputs[b], (const char*)outputs[c]))
        return set_err(HDCONV_EINVAL, "outputs[%d] and outputs[%d] overlap", b, c);
  int cur = -1;
  (void)hipGetDevice(&cur);
  if (cur != P->device) return set_err(HDCONV_EINVAL, "plan belongs to device %d, current device is %d", P->device, cur);
  hipStream_t s = (hipStream_t)stream;
  P->prof.slot = 0;
  int rc = P->dtype == HDCONV_C64 ? run_plan<float>(P, inputs, outputs, s)
                                  : run_plan<double>(P, inputs, outputs, s);
  if (P->prof.on && P->prof.used < P->prof.max_exec) P->prof.used++;
  return rc;
}

int hdconv_execute(hdconv_plan_t plan, const void* const* inputs, void* const* outputs, void* stream) {
  clear_err();
  if (!plan || !inputs || !outputs) return set_err(HDCONV_EINVAL, "plan, inputs and outputs must not be NULL");
  Plan* P = (Plan*)plan;
  if (P->host_only) return set_err(HDCONV_EINVAL, "plan was created with HDCONV_PLAN_HOST_ONLY");
  if (P->work_bytes && !P->work_mem)
    return set_err(HDCONV_EINVAL, "plan has no workspace (HDCONV_PLAN_NO_WORKSPACE): run it with hdconv_execute_noalloc");
  return execute_plan(P, inputs, outputs, stream);
}

int hdconv_execute_noalloc(hdconv_plan_t plan, const void* const* inputs, void* const* outputs, void* stream) {
  clear_err();
  if (!plan || !inputs || !outputs) return set_err(HDCONV_EINVAL, "plan, inputs and outputs must not be NULL");
  Plan* P = (Plan*)plan;
  if (P->host_only) return set_err(HDCONV_EINVAL, "plan was created with HDCONV_PLAN_HOST_ONLY");
  if (P->work_bytes > HDCONV_SCRATCH_BYTES)
    return set_err(HDCONV_EUNSUPPORTED, "workspace of %zu bytes exceeds the %zu-byte scratch of hdconv_execute_noalloc",
                   P->work_bytes, (size_t)HDCONV_SCRATCH_BYTES);
  int cur = -1;
  hipError_t e = hipGetDevice(&cur);
  if (e != hipSuccess) return hip_err(e, "hipGetDevice");
  if (cur != P->device) return set_err(HDCONV_EINVAL, "plan belongs to device %d, current device is %d", P->device, cur);
  char* base = nullptr;
  if (P->work_bytes) {
    int rc = scratch_of(cur, &base);
    if (rc != HDCONV_OK) return rc;
  }
  // the same launches with the workspace parts carved from the scratch, then
  // the plan's own workspace (or none) again
  carve_workspace(P, base);
  const int rc = execute_plan(P, inputs, outputs, stream);
  carve_workspace(P, P->work_mem);
  return rc;
}

static void prof_release(Plan* P) {
  for (hipEvent_t e : P->prof.ev) (void)hipEventDestroy(e);
  P->prof = Plan::Prof{};
}

int hdconv_profile_begin(hdconv_plan_t plan, int max_executes) {
  clear_err();
  if (!plan || max_executes < 1) return set_err(HDCONV_EINVAL, "need a plan and max_executes >= 1");
  Plan* P = (Plan*)plan;
  if (P->host_only) return set_err(HDCONV_EINVAL, "host-only plan");
  prof_release(P);
  Plan::Prof& f = P->prof;
  f.nslots = P->launches;
  f.max_exec = max_executes;
  f.ev.resize((size_t)max_executes * f.nslots * 2);
  for (auto& e : f.ev) {
    hipError_t r = hipEventCreate(&e);
    if (r != hipSuccess) {
      e = nullptr;
      prof_release(P);
      return hip_err(r, "hipEventCreate");
    }
  }
  f.on = true;
  return HDCONV_OK;
}

int hdconv_profile_end(hdconv_plan_t plan, hdconv_kernel_stat_t* out, int cap, int* count) {
  clear_err();
  if (!plan) return set_err(HDCONV_EINVAL, "plan is NULL");
  Plan* P = (Plan*)plan;
  Plan::Prof& f = P->prof;
  if (!f.on) return set_err(HDCONV_EINVAL, "profiling was not started");
  const int ns = (int)f.names.size();
  std::vector<double> tot(ns, 0.0);
  std::vector<int64_t> cnt(ns, 0);
  for (int x = 0; x < f.used; ++x)
    for (int k = 0; k < ns; ++k) {
      const int idx = (x * f.nslots + k) * 2;
      float ms = 0;
      if (hipEventSynchronize(f.ev[idx + 1]) != hipSuccess) continue;
      if (hipEventElapsedTime(&ms, f.ev[idx], f.ev[idx + 1]) == hipSuccess) {
        tot[k] += ms;
        cnt[k] += 1;
      }
    }
  if (count) *count = ns;
  for (int k = 0; k < ns && k < cap && out; ++k) {
    memset(&out[k], 0, sizeof(out[k]));
    snprintf(out[k].name, sizeof(out[k].name), "%s", f.names[k].c_str());
    out[k].launches = cnt[k];
    out[k].total_ms = tot[k];
    out[k].bytes_per_launch = f.bytes[k];
  }
  prof_release(P);
  return HDCONV_OK;
}

void hdconv_destroy(hdconv_plan_t plan) {
  if (plan) prof_release((Plan*)plan);
  free_plan((Plan*)plan);
}

}  // extern "C"

// ---------------------------------------------------------------------------
// autotuning: candidates, timing, cost-model features

static void fill_dim_info(const DimPlan& dp, hdconv_dim_info_t* di) {
  memset(di, 0, sizeof(*di));
  di->L = dp.L;
  di->M = dp.M;
  di->m = dp.m;
  di->p = dp.p;
  di->n = dp.n;
  di->q = dp.q;
  di->D = dp.D;
  di->variant = dp.variant;
  di->E_m = dp.E_m;
  di->E_p = dp.E_p;
  di->S = dp.S;
  di->rows_per_block = dp.rows_per_block;
  di->tw_m = dp.fd_m.N ? dp.fd_m.twmode + 1 : 0;
  di->tw_p = dp.fd_p.N ? dp.fd_p.twmode + 1 : 0;
  di->centered = dp.herm ? 2 : dp.ctr;
}

// options that reproduce the per-dimension shapes exactly
static hdconv_options opts_from_shape(const hdconv_dim_info_t* shp, int dims) {
  hdconv_options o;
  memset(&o, 0, sizeof(o));
  o.method = HDCONV_METHOD_HYBRID;
  if (shp[dims - 1].centered == 2) o.flags |= HDCONV_PLAN_HERMITIAN;
  else if (shp[0].centered == 1) o.flags |= HDCONV_PLAN_CENTERED;
  for (int d = 0; d < dims; ++d) {
    o.m[d] = shp[d].m;
    o.p[d] = shp[d].p;
    o.D[d] = shp[d].D;
    o.variant[d] = shp[d].variant;
    o.E_m[d] = shp[d].E_m;
    o.E_p[d] = shp[d].E_p;
    o.S[d] = shp[d].S;
    o.rows_per_block[d] = shp[d].rows_per_block;
    o.twiddles[d] = shp[d].tw_m == 2 ? 2 : 0;
  }
  return o;
}

// default plan plus, per dimension, that plan with the dimension replaced by
// each of its candidates (Sec. 7: dimensions are tuned independently)
static int list_candidates(const int64_t* L, const int64_t* M, int A, int dims, int dtype, int ctr,
                           std::vector<hdconv_dim_info_t>* out, std::vector<int>* varied) {
  const int tb = tbytes_of(dtype);
  std::vector<DimPlan> base(dims);
  for (int d = 0; d < dims; ++d) {
    std::string why;
    if (!choose_dim(L[d], M[d], A, tb, d == dims - 1, lines_of_shape(L, dims, d), &base[d], &why, ctr, dims))
      return set_err(HDCONV_EUNSUPPORTED, "dim %d: %s", d, why.c_str());
  }
  auto push = [&](const std::vector<DimPlan>& s, int v) {
    for (int d = 0; d < dims; ++d) {
      hdconv_dim_info_t di;
      fill_dim_info(s[d], &di);
      out->push_back(di);
    }
    varied->push_back(v);
  };
  push(base, -1);
  for (int d = 0; d < dims; ++d) {
    for (const DimPlan& c : dim_candidates(L[d], M[d], A, tb, d == dims - 1, ctr)) {
      const DimPlan& b = base[d];
      if (c.variant == b.variant && c.m == b.m && c.p == b.p && c.E_m == b.E_m && c.E_p == b.E_p && c.S == b.S &&
          c.rows_per_block == b.rows_per_block)
        continue;
      std::vector<DimPlan> s = base;
      s[d] = c;
      push(s, d);
    }
  }
  return HDCONV_OK;
}

static int time_plan_ms(hdconv_plan_t plan, int A, size_t bytes, int reps, double* ms) {
  void* buf[kMaxA + 1] = {nullptr, nullptr, nullptr, nullptr};
  hipStream_t s = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  int rc = HDCONV_OK;
  std::vector<float> t;
  hipError_t e = hipStreamCreateWithFlags(&s, hipStreamNonBlocking);
  for (int a = 0; a <= A && e == hipSuccess; ++a) {
    e = hipMalloc(&buf[a], bytes);
    if (e == hipSuccess) e = hipMemsetAsync(buf[a], 0, bytes, s);
  }
  if (e == hipSuccess) e = hipEventCreate(&e0);
  if (e == hipSuccess) e = hipEventCreate(&e1);
  if (e != hipSuccess) {
    rc = set_err(HDCONV_ENOMEM, "tuning buffers: %s", hipGetErrorString(e));
  } else {
    const void* ins[kMaxA] = {buf[0], buf[1], buf[2]};
    void* outs[1] = {buf[A]};
    rc = hdconv_execute(plan, ins, outs, s);  // warm-up
    // Three blocks of `reps` executes back to back, each timed as a whole:
    // the steady state a caller running many steps sees (a lone execute
    // between host synchronisations measured up to 30 % slower at 256^3,
    // with the chip's clocks down between them, and ranked shapes
    // differently).  The candidate's time is the median block average.
    for (int b = 0; b < 3 && rc == HDCONV_OK; ++b) {
      (void)hipEventRecord(e0, s);
      for (int r = 0; r < reps && rc == HDCONV_OK; ++r) rc = hdconv_execute(plan, ins, outs, s);
      (void)hipEventRecord(e1, s);
      float x = 0;
      if (rc == HDCONV_OK && (e = hipEventSynchronize(e1)) == hipSuccess &&
          (e = hipEventElapsedTime(&x, e0, e1)) == hipSuccess)
        t.push_back(x / (float)reps);
      else if (rc == HDCONV_OK)
        rc = hip_err(e, "tuning timing");
    }
  }
  if (s) (void)hipStreamSynchronize(s);
  for (void* b : buf)
    if (b) (void)hipFree(b);
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  if (s) (void)hipStreamDestroy(s);
  if (rc == HDCONV_OK) {
    std::sort(t.begin(), t.end());
    *ms = t.empty() ? 0.0 : t[t.size() / 2];
  }
  return rc;
}

extern "C" int hdconv_time_shape(const int64_t* L, const int64_t* M, int A, int B, int dims, int dtype,
                                 const hdconv_dim_info_t* shape, int reps, double* ms);

static void db_append(const char* path, const int64_t* L, const int64_t* M, int A, int dims, int dtype,
                      const hdconv_dim_info_t* shp, int varied, double ms) {
  FILE* f = fopen(path, "a");
  if (!f) return;
  fprintf(f, "%d,%d,%d", dims, A, dtype);
  for (int d = 0; d < 3; ++d) fprintf(f, ",%lld,%lld", (long long)(d < dims ? L[d] : 0), (long long)(d < dims ? M[d] : 0));
  fprintf(f, ",%d", varied);
  for (int d = 0; d < 3; ++d) {
    if (d < dims)
      fprintf(f, ",%d,%lld,%lld,%lld,%d,%d,%d,%d", shp[d].variant, (long long)shp[d].m, (long long)shp[d].p,
              (long long)shp[d].q, shp[d].E_m, shp[d].E_p, shp[d].S, shp[d].rows_per_block);
    else
      fprintf(f, ",0,0,0,0,0,0,0,0");
  }
  fprintf(f, ",%.6f\n", ms);
  fclose(f);
}

namespace hd {
int mlp_predict_host(void* model, const float* X, int64_t n, float* out);
}

// Choose shapes with the requested tuner; fills shp[0..dims).
static int tune_shapes(const int64_t* L, const int64_t* M, int A, int B, int dims, int dtype,
                       const hdconv_options* opt, hdconv_dim_info_t* shp, int* ncand, int* ntimed, double* best_ms) {
  std::vector<hdconv_dim_info_t> cand;
  std::vector<int> varied;
  // candidates are shapes of the engine's lengths (Hermitian: the full centered length)
  const bool herm = (opt->flags & HDCONV_PLAN_HERMITIAN) != 0;
  int64_t Lc[3];
  for (int d = 0; d < dims; ++d) Lc[d] = (herm && d == dims - 1) ? herm_full(L[d]) : L[d];
  int rc = list_candidates(Lc, M, A, dims, dtype,
                           (opt->flags & (HDCONV_PLAN_CENTERED | HDCONV_PLAN_HERMITIAN)) ? 1 : 0, &cand, &varied);
  if (rc != HDCONV_OK) return rc;
  if (herm)  // the last dimension of every candidate is the Hermitian one
    for (size_t k = 0; k < cand.size(); k += dims) cand[k + dims - 1].centered = 2;
  const int nc = (int)varied.size();
  *ncand = nc;
  *ntimed = 0;
  const int reps = opt->tune_reps > 0 ? opt->tune_reps : 5;
  // measured ms (timed candidates) and, for the model tuner, predicted log ms
  std::vector<double> meas(nc, 1e300), pred(nc, 0.0);
  std::vector<char> timed(nc, 0);
  auto time_one = [&](int k) -> int {
    double ms = 0;
    int r = hdconv_time_shape(L, M, A, B, dims, dtype, &cand[(size_t)k * dims], reps, &ms);
    timed[k] = 1;  // a candidate that cannot run keeps meas = 1e300
    if (r != HDCONV_OK) return r;
    meas[k] = ms;
    (*ntimed)++;
    if (opt->db_path) db_append(opt->db_path, L, M, A, dims, dtype, &cand[(size_t)k * dims], varied[k], ms);
    return HDCONV_OK;
  };
  const bool model = opt->tuner == HDCONV_TUNER_MODEL;
  if (!model) {
    for (int k = 0; k < nc; ++k) (void)time_one(k);
  } else {
    if (!opt->model) return set_err(HDCONV_EINVAL, "the model tuner needs options.model");
    std::vector<float> X((size_t)nc * HDCONV_NFEATURES), pf(nc);
    for (int k = 0; k < nc; ++k)
      if ((rc = hdconv_features(L, M, A, B, dims, dtype, &cand[(size_t)k * dims], &X[(size_t)k * HDCONV_NFEATURES])) != HDCONV_OK)
        return rc;
    if ((rc = hd::mlp_predict_host(opt->model, X.data(), nc, pf.data())) != HDCONV_OK) return rc;
    for (int k = 0; k < nc; ++k) pred[k] = pf[k];
  }
  // per dimension, the best candidate varying that dimension (or the default)
  const double margin = opt->margin > 0 ? opt->margin : 0.05;
  for (int d = 0; d < dims; ++d) {
    std::vector<int> ks;
    for (int k = 0; k < nc; ++k)
      if (varied[k] == -1 || varied[k] == d) ks.push_back(k);
    const std::vector<double>& key = model ? pred : meas;
    std::stable_sort(ks.begin(), ks.end(), [&](int a, int b) { return key[a] < key[b]; });
    int best = ks[0];
    if (model && ks.size() > 1) {
      // The model's pick is timed against the default plan, which it must
      // beat to be taken (a guard against shapes the network ranks wrongly:
      // timings taken under another runtime, or shapes it was never trained
      // on); on a close call the predicted top three are timed as well.
      // The fastest that runs is kept.
      const bool close = pred[ks[1]] - pred[ks[0]] < margin;
      std::vector<int> tk(ks.begin(), ks.begin() + (close ? std::min<size_t>(3, ks.size()) : 1));
      for (int k : ks)
        if (varied[k] == -1 && std::find(tk.begin(), tk.end(), k) == tk.end()) tk.push_back(k);
      double bm = 1e300;
      for (int k : tk) {
        if (!timed[k]) (void)time_one(k);
        if (meas[k] < bm) {
          bm = meas[k];
          best = k;
        }
      }
    }
    shp[d] = cand[(size_t)best * dims + d];
  }
  *best_ms = 0;
  for (int k = 0; k < nc; ++k) {
    bool same = true;
    for (int d = 0; d < dims; ++d) {
      const hdconv_dim_info_t &a = cand[(size_t)k * dims + d], &b = shp[d];
      same = same && a.variant == b.variant && a.m == b.m && a.p == b.p && a.E_m == b.E_m && a.E_p == b.E_p &&
             a.S == b.S && a.rows_per_block == b.rows_per_block;
    }
    if (same && timed[k] && meas[k] < 1e300) *best_ms = meas[k];
  }
  return HDCONV_OK;
}

extern "C" {

int hdconv_candidates(const int64_t* L, const int64_t* M, int A, int B, int dims, int dtype, int flags,
                      hdconv_dim_info_t* out, int* varied, int cap, int* count) {
  clear_err();
  if (!L || !M || dims < 1 || dims > 3 || A < 2 || A > 3 || B != 1 || (dtype != HDCONV_C64 && dtype != HDCONV_C128))
    return set_err(HDCONV_EINVAL, "invalid problem");
  if (flags & ~(HDCONV_PLAN_CENTERED | HDCONV_PLAN_HERMITIAN))
    return set_err(HDCONV_EINVAL, "flags: HDCONV_PLAN_CENTERED or HDCONV_PLAN_HERMITIAN only");
  // candidates are shapes of the engine's lengths (Hermitian: the full
  // centered length of the last dimension), as the plan tuner lists them
  const bool herm = (flags & HDCONV_PLAN_HERMITIAN) != 0;
  int64_t Lc[3];
  for (int d = 0; d < dims; ++d) Lc[d] = (herm && d == dims - 1) ? herm_full(L[d]) : L[d];
  std::vector<hdconv_dim_info_t> cand;
  std::vector<int> var;
  int rc = list_candidates(Lc, M, A, dims, dtype, flags ? 1 : 0, &cand, &var);
  if (rc != HDCONV_OK) return rc;
  if (herm)
    for (size_t k = 0; k < cand.size(); k += dims) cand[k + dims - 1].centered = 2;
  if (count) *count = (int)var.size();
  for (int k = 0; k < (int)var.size() && k < cap; ++k) {
    if (out)
      for (int d = 0; d < dims; ++d) out[(size_t)k * dims + d] = cand[(size_t)k * dims + d];
    if (varied) varied[k] = var[k];
  }
  return HDCONV_OK;
}

int hdconv_time_shape(const int64_t* L, const int64_t* M, int A, int B, int dims, int dtype,
                      const hdconv_dim_info_t* shape, int reps, double* ms) {
  clear_err();
  if (!shape || !ms || reps < 1) return set_err(HDCONV_EINVAL, "need a shape, ms and reps >= 1");
  hdconv_options o = opts_from_shape(shape, dims);
  hdconv_plan_t plan = hdconv_plan_ex(L, M, A, B, dims, dtype, &o);
  if (!plan) return g_err_code;
  size_t bytes = 2 * (size_t)tbytes_of(dtype);
  for (int d = 0; d < dims; ++d) bytes *= (size_t)L[d];
  int rc = time_plan_ms(plan, A, bytes, reps, ms);
  hdconv_destroy(plan);
  return rc;
}

int hdconv_features(const int64_t* L, const int64_t* M, int A, int B, int dims, int dtype,
                    const hdconv_dim_info_t* shape, float* out) {
  clear_err();
  if (!shape || !out) return set_err(HDCONV_EINVAL, "need a shape and out");
  hdconv_options o = opts_from_shape(shape, dims);
  o.flags |= HDCONV_PLAN_HOST_ONLY;
  Plan* P = (Plan*)hdconv_plan_ex(L, M, A, B, dims, dtype, &o);
  if (!P) return g_err_code;
  auto lg = [](double x) { return (float)std::log2(std::max(x, 1.0)); };
  for (int i = 0; i < HDCONV_NFEATURES; ++i) out[i] = 0.f;
  int launches = 0;
  const double traffic = plan_traffic(P, &launches);
  double tot = 1, work = 0, nb = 1;
  for (int d = 0; d < dims; ++d) tot *= (double)L[d];
  for (int d = 0; d < dims; ++d) {
    const DimPlan& dp = P->dp[d];
    double rest = 1;
    for (int e = d + 1; e < dims; ++e) rest *= (double)L[e];
    // transform work of this level: (A+B) transforms of q m points per line
    work += (A + B) * nb * rest * (double)(dp.q * dp.m) * std::log2(std::max<double>(2.0, (double)(dp.m * dp.p)));
    nb *= (double)(dp.q * dp.m);
    float* f = out + 13 + 10 * d;
    f[0] = lg((double)dp.m);
    f[1] = lg((double)dp.p);
    f[2] = lg((double)dp.q);
    f[3] = dp.variant == VAR_FUSED;
    f[4] = dp.variant == VAR_MULTI;
    f[5] = dp.variant == VAR_OUTER;
    f[6] = lg((double)dp.E_m);
    f[7] = lg((double)dp.E_p);
    f[8] = lg((double)dp.S);
    f[9] = lg((double)dp.rows_per_block);
  }
  out[0] = (float)dims;
  out[1] = (float)A;
  out[2] = (float)dtype;
  for (int d = 0; d < dims; ++d) {
    out[3 + d] = lg((double)L[d]);
    out[6 + d] = lg((double)M[d]);
  }
  out[9] = lg(tot);
  out[10] = lg(traffic);
  out[11] = lg((double)launches);
  out[12] = lg(work);
  out[43] = lg((double)P->work_bytes + 1.0);
  // centered / Hermitian problem, dimensions on the lean kernels (one
  // block, ordinary dimension, compiled size and width), largest q
  out[44] = (P->flags & (HDCONV_PLAN_CENTERED | HDCONV_PLAN_HERMITIAN)) ? 1.f : 0.f;
  out[45] = (P->flags & HDCONV_PLAN_HERMITIAN) ? 1.f : 0.f;
  {
    int nlean = 0;
    double qmax = 1;
    const int tb = tbytes_of(P->dtype);
    for (int d = 0; d < dims; ++d) {
      const DimPlan& dp = P->dp[d];
      qmax = std::max(qmax, (double)dp.q);
      if (dp.ctr || dp.herm || dp.p > 2) continue;
      if (dp.variant == VAR_OUTER && outer_lean_supported((int)dp.m, dp.E_m, dp.S, (int)dp.q, tb)) ++nlean;
      if (dp.variant == VAR_FUSED && rows_lean_supported((int)dp.m, dp.E_m, A, (int)dp.q, tb)) ++nlean;
    }
    out[46] = (float)nlean;
    out[47] = lg(qmax);
  }
  hdconv_destroy((hdconv_plan_t)P);
  return HDCONV_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// batched plans: many independent 1D convolutions of uneven length

namespace {
constexpr int kSideStreams = 4;

struct GroupKey {
  int variant;
  int64_t m, p, n, q;
  int E_m, E_p, S, rpb;
  bool operator<(const GroupKey& o) const {
    return std::tie(variant, m, p, n, q, E_m, E_p, S, rpb) <
           std::tie(o.variant, o.m, o.p, o.n, o.q, o.E_m, o.E_p, o.S, o.rpb);
  }
};
}  // namespace

struct Batch {
  int A = 0, B = 0, dtype = 0, flags = 0, device = -1;
  int64_t count = 0;
  std::vector<int64_t> L, M;
  std::vector<Plan*> groups;                  // one plan per shape, rows = its members
  std::vector<std::vector<int64_t>> members;  // convolution indices per group
  std::vector<size_t> task_off;               // byte offset of each group's task table
  char* task_dev = nullptr;
  char* task_host = nullptr;  // pinned staging of the task tables
  size_t task_bytes = 0;
  hipEvent_t copied = nullptr;
  bool copy_pending = false;
  hipStream_t side[kSideStreams] = {};
  hipStream_t capture = nullptr;  // stream the graph is captured on
  hipEvent_t fork = nullptr;
  std::vector<hipEvent_t> joins;
  hipGraphExec_t exec = nullptr;
  int executes = 0;
  int tuner = 0, tuned_candidates = 0, timed_candidates = 0;
  std::vector<char> shadow, uploaded;  // task tables of this execute and of the last upload
  // persistent form: launches of k_batch over device task tables, one per
  // pass of the inner form
  bool persist = false;
  char* pmem = nullptr;  // buckets, then the task tables
  void* pbuckets = nullptr;
  BatchTask* ptasks[3] = {};
  int ntasks[3] = {};
  int pgrid = 0, xwords = 0;
  size_t plds = 0;
};

// A one-dimensional plan for `rows` independent rows sharing the shape dp.
static Plan* make_group_plan(int A, int B, int dtype, const DimPlan& dp, int64_t rows, int device) {
  Plan* P = new (std::nothrow) Plan();
  if (!P) {
    set_err(HDCONV_ENOMEM, "host allocation failed");
    return nullptr;
  }
  P->dims = 1;
  P->A = A;
  P->B = B;
  P->dtype = dtype;
  P->method = HDCONV_METHOD_HYBRID;
  {
    const double none[kMaxA * kMaxA] = {};
    P->shares[0] = make_shares(A, none);  // the product of the A inputs
  }
  P->L[0] = dp.L;
  P->Lio[0] = dp.herm ? herm_stored(dp.L) : dp.L;
  P->M[0] = dp.M;
  P->dp[0] = dp;
  P->batch_rows = rows;
  P->device = device;
  if (size_workspace(P) != HDCONV_OK || alloc_tables(P) != HDCONV_OK || alloc_workspace(P) != HDCONV_OK) {
    free_plan(P);
    return nullptr;
  }
  plan_traffic(P, &P->launches);
  return P;
}

static void free_batch(Batch* Bt) {
  if (!Bt) return;
  (void)hipDeviceSynchronize();
  for (Plan* P : Bt->groups) free_plan(P);
  if (Bt->exec) (void)hipGraphExecDestroy(Bt->exec);
  for (hipEvent_t e : Bt->joins) (void)hipEventDestroy(e);
  if (Bt->fork) (void)hipEventDestroy(Bt->fork);
  if (Bt->copied) (void)hipEventDestroy(Bt->copied);
  for (hipStream_t s : Bt->side)
    if (s) (void)hipStreamDestroy(s);
  if (Bt->capture) (void)hipStreamDestroy(Bt->capture);
  if (Bt->task_dev) (void)hipFree(Bt->task_dev);
  if (Bt->task_host) (void)hipHostFree(Bt->task_host);
  if (Bt->pmem) (void)hipFree(Bt->pmem);
  delete Bt;
}

// Launch every group: fork from `s` onto the side streams, join back (the
// persistent form: its one launch).
template <typename T>
static int issue_batch(Batch* Bt, hipStream_t s) {
  hipError_t e;
  if (Bt->persist) {
    for (int ph = 0; ph < 3; ++ph) {
      if (Bt->ntasks[ph] == 0) continue;
      BatchArgs<T> a{};
      a.buckets = (const BatchBucket<T>*)Bt->pbuckets;
      a.tasks = Bt->ptasks[ph];
      a.ntasks = Bt->ntasks[ph];
      a.xwords = Bt->xwords;
      const int grid = std::min(Bt->pgrid, Bt->ntasks[ph]);
      if ((e = launch_batch<T>(a, Bt->A, grid, Bt->plds, s)) != hipSuccess) return hip_err(e, "k_batch launch");
    }
    return HDCONV_OK;
  }
  e = hipEventRecord(Bt->fork, s);
  if (e != hipSuccess) return hip_err(e, "hipEventRecord(fork)");
  for (size_t g = 0; g < Bt->groups.size(); ++g) {
    hipStream_t hs = Bt->side[g % kSideStreams];
    if ((e = hipStreamWaitEvent(hs, Bt->fork, 0)) != hipSuccess) return hip_err(e, "hipStreamWaitEvent");
    const RowTask<T>* tasks = (const RowTask<T>*)(Bt->task_dev + Bt->task_off[g]);
    int rc = run_rows<T>(Bt->groups[g], nullptr, nullptr, (int64_t)Bt->members[g].size(), hs, tasks);
    if (rc != HDCONV_OK) return rc;
    if ((e = hipEventRecord(Bt->joins[g], hs)) != hipSuccess) return hip_err(e, "hipEventRecord(join)");
  }
  for (size_t g = 0; g < Bt->groups.size(); ++g)
    if ((e = hipStreamWaitEvent(s, Bt->joins[g], 0)) != hipSuccess) return hip_err(e, "hipStreamWaitEvent");
  return HDCONV_OK;
}

template <typename T>
static void fill_tasks(Batch* Bt, const void* const* inputs, void* const* outputs) {
  Bt->shadow.assign(Bt->task_bytes, 0);
  for (size_t g = 0; g < Bt->groups.size(); ++g) {
    RowTask<T>* t = (RowTask<T>*)(Bt->shadow.data() + Bt->task_off[g]);
    for (size_t k = 0; k < Bt->members[g].size(); ++k) {
      const int64_t i = Bt->members[g][k];
      RowTask<T> r{};
      for (int a = 0; a < Bt->A; ++a) r.in[a] = (const cpx<T>*)inputs[i * Bt->A + a];
      r.out = (cpx<T>*)outputs[i * Bt->B];
      r.L = Bt->L[i];
      t[k] = r;
    }
  }
}

template <typename T>
static int run_batched(Batch* Bt, const void* const* inputs, void* const* outputs, hipStream_t s) {
  hipError_t e;
  fill_tasks<T>(Bt, inputs, outputs);
  // the same pointers as the table on the device: no upload (and no wait)
  if (Bt->shadow != Bt->uploaded) {
    if (Bt->copy_pending) {  // the staging buffer is reused: wait for the previous upload
      if ((e = hipEventSynchronize(Bt->copied)) != hipSuccess) return hip_err(e, "hipEventSynchronize");
      Bt->copy_pending = false;
    }
    memcpy(Bt->task_host, Bt->shadow.data(), Bt->task_bytes);
    if ((e = hipMemcpyAsync(Bt->task_dev, Bt->task_host, Bt->task_bytes, hipMemcpyHostToDevice, s)) != hipSuccess)
      return hip_err(e, "hipMemcpyAsync(tasks)");
    if ((e = hipEventRecord(Bt->copied, s)) != hipSuccess) return hip_err(e, "hipEventRecord");
    Bt->copy_pending = true;
    Bt->uploaded = Bt->shadow;
  }
  const bool graph = !(Bt->flags & HDCONV_BATCH_NO_GRAPH);
  // the first execute runs eagerly (kernels loaded, LDS limits granted);
  // the second captures the launches into a graph that later executes replay
  if (!graph || Bt->executes == 0) {
    Bt->executes++;
    return issue_batch<T>(Bt, s);
  }
  if (!Bt->exec) {
    // capture on the plan's own stream (the caller's may be the legacy null
    // stream, which cannot be captured); the graph then runs on the caller's
    hipGraph_t g = nullptr;
    hipStream_t cs = Bt->capture;
    if ((e = hipStreamBeginCapture(cs, hipStreamCaptureModeRelaxed)) != hipSuccess)
      return hip_err(e, "hipStreamBeginCapture");
    int rc = issue_batch<T>(Bt, cs);
    hipError_t e2 = hipStreamEndCapture(cs, &g);
    if (rc != HDCONV_OK) {
      if (g) (void)hipGraphDestroy(g);
      return rc;
    }
    if (e2 != hipSuccess) return hip_err(e2, "hipStreamEndCapture");
    e = hipGraphInstantiate(&Bt->exec, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) {
      Bt->exec = nullptr;
      return hip_err(e, "hipGraphInstantiate");
    }
  }
  Bt->executes++;
  if ((e = hipGraphLaunch(Bt->exec, s)) != hipSuccess) return hip_err(e, "hipGraphLaunch");
  return HDCONV_OK;
}

// Median ms of one group's launches with shape dp over rows of the given
// lengths (each row in its own zeroed slot of Lmax words), as the batch runs
// them.  Returns a non-OK code if the shape cannot be planned or launched.
template <typename T>
static int time_group_ms(int A, int B, int dtype, const DimPlan& dp, const std::vector<int64_t>& Ls, int device,
                         int reps, double* ms) {
  const int64_t rows = (int64_t)Ls.size();
  int64_t Lmax = 1;
  for (int64_t v : Ls) Lmax = std::max(Lmax, v);
  Plan* P = make_group_plan(A, B, dtype, dp, rows, device);
  if (!P) return g_err_code;
  const size_t bytes = (size_t)rows * (size_t)Lmax * sizeof(cpx<T>);
  cpx<T>* buf[kMaxA + 1] = {nullptr, nullptr, nullptr, nullptr};
  RowTask<T>* tdev = nullptr;
  hipStream_t s = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  std::vector<float> t;
  int rc = HDCONV_OK;
  hipError_t e = hipStreamCreateWithFlags(&s, hipStreamNonBlocking);
  for (int a = 0; a <= A && e == hipSuccess; ++a) {
    e = hipMalloc((void**)&buf[a], bytes);
    if (e == hipSuccess) e = hipMemsetAsync(buf[a], 0, bytes, s);
  }
  std::vector<RowTask<T>> th((size_t)rows);
  for (int64_t i = 0; i < rows; ++i) {
    RowTask<T> r{};
    for (int a = 0; a < A; ++a) r.in[a] = buf[a] ? buf[a] + i * Lmax : nullptr;
    r.out = buf[A] ? buf[A] + i * Lmax : nullptr;
    r.L = Ls[(size_t)i];
    th[(size_t)i] = r;
  }
  if (e == hipSuccess) e = hipMalloc((void**)&tdev, th.size() * sizeof(RowTask<T>));
  if (e == hipSuccess) e = hipMemcpyAsync(tdev, th.data(), th.size() * sizeof(RowTask<T>), hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipEventCreate(&e0);
  if (e == hipSuccess) e = hipEventCreate(&e1);
  if (e != hipSuccess) {
    rc = set_err(HDCONV_ENOMEM, "batch tuning buffers: %s", hipGetErrorString(e));
  } else {
    rc = run_rows<T>(P, nullptr, nullptr, rows, s, tdev);  // warm-up
    for (int r = 0; r < reps && rc == HDCONV_OK; ++r) {
      (void)hipEventRecord(e0, s);
      rc = run_rows<T>(P, nullptr, nullptr, rows, s, tdev);
      (void)hipEventRecord(e1, s);
      float x = 0;
      if (rc == HDCONV_OK && (e = hipEventSynchronize(e1)) == hipSuccess &&
          (e = hipEventElapsedTime(&x, e0, e1)) == hipSuccess)
        t.push_back(x);
      else if (rc == HDCONV_OK)
        rc = hip_err(e, "batch tuning timing");
    }
  }
  if (s) (void)hipStreamSynchronize(s);
  for (cpx<T>* b : buf)
    if (b) (void)hipFree(b);
  if (tdev) (void)hipFree(tdev);
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  if (s) (void)hipStreamDestroy(s);
  free_plan(P);
  if (rc == HDCONV_OK) {
    std::sort(t.begin(), t.end());
    *ms = t.empty() ? 0.0 : t[t.size() / 2];
  }
  return rc;
}

// Per-group tuning of a batched plan (the size buckets are the heuristic
// groups).  Candidates are the one-dimensional candidates of the group's
// longest member (so every member fits every candidate), plus row-packing
// variants of the whole-row kernel; the exhaustive tuner times all of them
// over the group's own lengths, the model tuner ranks them by predicted time
// and times the top three when the best two are within the margin.  Groups
// whose tuned shapes coincide are merged.  Returns candidates and timings
// counted into *ncand / *ntimed.
static int tune_batch_groups(int A, int B, int dtype, int device, const hdconv_options* opt,
                             const std::vector<int64_t>& Lall, std::map<GroupKey, std::vector<int64_t>>* byk,
                             std::map<GroupKey, DimPlan>* shape, int* ncand, int* ntimed) {
  const int tb = tbytes_of(dtype);
  const int reps = opt->tune_reps > 0 ? opt->tune_reps : 5;
  const double margin = opt->margin > 0 ? opt->margin : 0.05;
  const bool model = opt->tuner == HDCONV_TUNER_MODEL;
  if (model && !opt->model) return set_err(HDCONV_EINVAL, "the model tuner needs options.model");
  std::map<GroupKey, std::vector<int64_t>> nbyk;
  std::map<GroupKey, DimPlan> nshape;
  for (auto& kv : *byk) {
    const DimPlan& base = (*shape)[kv.first];
    std::vector<int64_t> Ls;
    for (int64_t i : kv.second) Ls.push_back(Lall[(size_t)i]);
    std::vector<DimPlan> cands = {base};
    auto same = [](const DimPlan& a, const DimPlan& b) {
      return a.variant == b.variant && a.m == b.m && a.p == b.p && a.q == b.q && a.E_m == b.E_m &&
             a.E_p == b.E_p && a.S == b.S && a.rows_per_block == b.rows_per_block;
    };
    auto add = [&](const DimPlan& c) {
      for (const DimPlan& u : cands)
        if (same(u, c)) return;
      cands.push_back(c);
    };
    for (DimPlan c : dim_candidates(base.L, base.M, A, tb, true, base.ctr)) {
      c.herm = base.herm;
      add(c);
      if (c.variant == VAR_FUSED)
        for (int f : {2, 4}) {
          for (int dir = 0; dir < 2; ++dir) {
            DimPlan v = c;
            v.rows_per_block = dir ? c.rows_per_block * f : c.rows_per_block / f;
            std::string w;
            if (v.rows_per_block >= 1 && finish_dim(&v, A, tb, &w)) add(v);
          }
        }
    }
    const int nc = (int)cands.size();
    *ncand += nc;
    std::vector<double> meas(nc, 1e300), pred(nc, 0.0);
    auto time_one = [&](int k) {
      double ms = 0;
      const int r = tb == 4 ? time_group_ms<float>(A, B, dtype, cands[k], Ls, device, reps, &ms)
                            : time_group_ms<double>(A, B, dtype, cands[k], Ls, device, reps, &ms);
      if (r == HDCONV_OK && ms > 0) {
        meas[k] = ms;
        (*ntimed)++;
      }
    };
    int best = 0;
    if (!model) {
      for (int k = 0; k < nc; ++k) time_one(k);
      for (int k = 1; k < nc; ++k)
        if (meas[k] < meas[best]) best = k;
    } else {
      std::vector<float> X((size_t)nc * HDCONV_NFEATURES), pf(nc);
      for (int k = 0; k < nc; ++k) {
        hdconv_dim_info_t di;
        fill_dim_info(cands[k], &di);
        const int r = hdconv_features(&base.L, &base.M, A, B, 1, dtype, &di, &X[(size_t)k * HDCONV_NFEATURES]);
        if (r != HDCONV_OK) return r;
      }
      int r = hd::mlp_predict_host(opt->model, X.data(), nc, pf.data());
      if (r != HDCONV_OK) return r;
      std::vector<int> ks(nc);
      for (int k = 0; k < nc; ++k) ks[k] = k;
      std::stable_sort(ks.begin(), ks.end(), [&](int a, int b) { return pf[a] < pf[b]; });
      best = ks[0];
      if (nc > 1 && pf[ks[1]] - pf[ks[0]] < margin) {
        double bm = 1e300;
        for (int i = 0; i < nc && i < 3; ++i) {
          time_one(ks[i]);
          if (meas[ks[i]] < bm) {
            bm = meas[ks[i]];
            best = ks[i];
          }
        }
      }
    }
    DimPlan dp = cands[best];
    GroupKey k{dp.variant, dp.m, dp.p, dp.n, dp.q, dp.E_m, dp.E_p, dp.S, dp.rows_per_block};
    auto it = nshape.find(k);
    if (it == nshape.end()) nshape[k] = dp;
    else {
      it->second.L = std::max(it->second.L, dp.L);
      it->second.M = std::max(it->second.M, dp.M);
    }
    auto& mem = nbyk[k];
    mem.insert(mem.end(), kv.second.begin(), kv.second.end());
  }
  for (auto& kv : nbyk) std::sort(kv.second.begin(), kv.second.end());
  *byk = std::move(nbyk);
  *shape = std::move(nshape);
  return HDCONV_OK;
}

// Shape of one convolution in the persistent form (false: no compiled
// body, or its LDS exceeds 64 KiB): whole rows of N = max(64, 2^ceil(log2 L))
// points up to 2048 (FP64 1024) with q = ceil(M/N) <= 8 residues, else the
// inner form with rows of 2048 (FP64 1024) points and the least compiled p
// at or above ceil(L/m) (powers of two, and in FP32 3 * 2^k from 12 to 96).
static bool persist_dim(int64_t L, int64_t M, int A, int tb, DimPlan* dp) {
  const int64_t nmax = tb == 4 ? 2048 : 1024;
  int64_t N = 64;
  while (N < L) N *= 2;
  DimPlan c;
  int body = 0, Em = 0, Ep = 0, S = 0;
  c.L = L;
  c.M = M;
  if (N <= nmax) {
    const Geometry g = geometry(L, M, N, 0, false);
    if (g.inner || g.p != 1 || g.q > kLeanMaxQ || !batch_shape(0, N, 1, tb, &body, &Em, &Ep, &S)) return false;
    c.m = N;
    c.p = 1;
    c.n = c.q = c.D = g.q;
    c.variant = VAR_FUSED;
    c.E_m = Em;
    c.rows_per_block = kBatchThreads / (int)(N / Em);
  } else {
    // the least compiled p with p m >= L: a power of two or 3 * 2^k (12 .. 96)
    const int64_t m = nmax;
    int64_t p = 2;
    while (p * m < L) p *= 2;
    for (int64_t p3 = 12; p3 <= 96 && tb == 4; p3 *= 2)
      if (p3 * m >= L && p3 < p) p = p3;
    const Geometry g = geometry(L, M, m, p, true);
    if (g.p != p || !batch_shape(1, m, p, tb, &body, &Em, &Ep, &S)) return false;
    c.m = m;
    c.p = p;
    c.n = c.D = g.n;
    c.q = g.q;
    c.variant = VAR_MULTI;
    c.E_m = Em;
    c.E_p = Ep;
    c.S = S;
    c.rows_per_block = 1;
  }
  std::string why;
  if (!finish_dim(&c, A, tb, &why)) return false;
  int xw = 0, tw = 0;
  batch_lds_words(body, (int)c.m, (int)c.p, (int)c.q, c.fd_m.ntw_stage, c.variant == VAR_MULTI ? c.fd_p.ntw_stage : 0,
                  tb, &xw, &tw);
  if ((size_t)(xw + tw) * 2 * tb > 64 * 1024) return false;
  *dp = c;
  return true;
}

// Bytes of traffic one task aims at (a few tens of microseconds of one
// workgroup's share of the bandwidth).
constexpr double kTaskBytes = 256.0 * 1024;

// Buckets and the three task tables of the persistent form (device memory):
// the column passes, the row passes, then the back passes followed by the
// whole rows; the widest convolutions first in each.
template <typename T>
static int build_persist(Batch* Bt) {
  const int tb = (int)sizeof(T), A = Bt->A;
  const double w = 2.0 * tb;
  const size_t ng = Bt->groups.size();
  std::vector<BatchBucket<T>> bk(ng);
  int xw = 0, tw = 0;
  for (size_t g = 0; g < ng; ++g) {
    Plan* P = Bt->groups[g];
    const DimPlan& dp = P->dp[0];
    BatchBucket<T>& b = bk[g];
    b.inner = dp.variant == VAR_MULTI;
    int body = 0, Em = 0, Ep = 0, S = 0;
    if (!batch_shape(b.inner, dp.m, dp.p, tb, &body, &Em, &Ep, &S) || Em != dp.E_m ||
        (b.inner && (Ep != dp.E_p || S != dp.S)))
      return set_err(HDCONV_EUNSUPPORTED, "group %zu (m=%lld, p=%lld) has no persistent body", g, (long long)dp.m,
                     (long long)dp.p);
    b.body = body;
    b.m = (int)dp.m;
    b.p = (int)dp.p;
    b.n = (int)dp.n;
    b.q = (int)dp.q;
    b.S = S;
    b.scale = (T)(1.0 / (double)(dp.q * dp.m));
    b.tw_m = (const cpx<T>*)P->dd[0].fft_m + dp.fd_m.ntw;
    b.ntw_m = dp.fd_m.ntw_stage;
    if (b.inner) {
      b.tw_p = (const cpx<T>*)P->dd[0].fft_p + dp.fd_p.ntw;
      b.ntw_p = dp.fd_p.ntw_stage;
      b.zq = (const cpx<T>*)P->dd[0].zq;
    }
    b.zqm = rtab<T>(P, 0);
    b.rows = (const RowTask<T>*)(Bt->task_dev + Bt->task_off[g]);
    for (int a = 0; a < A; ++a) b.work[a] = (cpx<T>*)P->rowwork[a];
    int x = 0, t = 0;
    batch_lds_words(body, b.m, b.p, b.q, b.ntw_m, b.ntw_p, tb, &x, &t);
    xw = std::max(xw, x);
    tw = std::max(tw, t);
  }
  // inner-form convolutions, the widest buckets first
  std::vector<std::pair<int, int64_t>> inner;
  {
    std::vector<size_t> gi;
    for (size_t g = 0; g < ng; ++g)
      if (bk[g].inner) gi.push_back(g);
    std::stable_sort(gi.begin(), gi.end(), [&](size_t a, size_t b) { return bk[a].p * bk[a].m > bk[b].p * bk[b].m; });
    for (size_t g : gi)
      for (int64_t c = 0; c < (int64_t)Bt->members[g].size(); ++c) inner.push_back({(int)g, c});
  }
  std::vector<BatchTask> tl[3];
  for (auto& ic : inner) {
    const BatchBucket<T>& b = bk[ic.first];
    const int tiles = b.m / b.S;
    auto per = [](double bytes_per_unit, int units) {
      return std::max(1, std::min(units, (int)(kTaskBytes / bytes_per_unit)));
    };
    const int c = (int)ic.second;
    const int u1 = A * tiles, p1 = per((1.0 + b.n) * b.p * b.S * w, u1);
    const int u2 = b.q, p2 = per((A + 1.0) * b.m * w, u2);
    const int u3 = tiles, p3 = per((double)(b.n + 1) * b.p * b.S * w, u3);
    for (int u = 0; u < u1; u += p1) tl[0].push_back({ic.first, BK_COLF, c, u, std::min(p1, u1 - u)});
    for (int u = 0; u < u2; u += p2) tl[1].push_back({ic.first, BK_ROWP, c, u, std::min(p2, u2 - u)});
    for (int u = 0; u < u3; u += p3) tl[2].push_back({ic.first, BK_COLB, c, u, std::min(p3, u3 - u)});
  }
  {
    std::vector<size_t> gr;
    for (size_t g = 0; g < ng; ++g)
      if (!bk[g].inner) gr.push_back(g);
    std::stable_sort(gr.begin(), gr.end(), [&](size_t a, size_t b) { return bk[a].m > bk[b].m; });
    for (size_t g : gr) {
      const int rpb = kBatchThreads / (bk[g].m / Bt->groups[g]->dp[0].E_m);
      const int cnt = (int)Bt->members[g].size();
      for (int c = 0; c < cnt; c += rpb) tl[2].push_back({(int)g, BK_ROWS, c, 0, std::min(rpb, cnt - c)});
    }
  }
  for (auto& v : tl)
    if (v.size() > (size_t)INT32_MAX) return set_err(HDCONV_EUNSUPPORTED, "too many tasks for one launch");
  const size_t bbytes = align256(ng * sizeof(BatchBucket<T>));
  size_t tbytes[3], total = bbytes;
  for (int ph = 0; ph < 3; ++ph) total += (tbytes[ph] = align256(std::max<size_t>(1, tl[ph].size()) * sizeof(BatchTask)));
  hipError_t e = hipMalloc((void**)&Bt->pmem, total);
  if (e != hipSuccess) return set_err(HDCONV_ENOMEM, "persistent batch tables: %s", hipGetErrorString(e));
  Bt->pbuckets = Bt->pmem;
  if ((e = hipMemcpy(Bt->pbuckets, bk.data(), ng * sizeof(BatchBucket<T>), hipMemcpyHostToDevice)) != hipSuccess)
    return hip_err(e, "persistent batch tables");
  size_t off = bbytes;
  for (int ph = 0; ph < 3; ++ph) {
    Bt->ptasks[ph] = (BatchTask*)(Bt->pmem + off);
    Bt->ntasks[ph] = (int)tl[ph].size();
    if (!tl[ph].empty() &&
        (e = hipMemcpy(Bt->ptasks[ph], tl[ph].data(), tl[ph].size() * sizeof(BatchTask), hipMemcpyHostToDevice)) !=
            hipSuccess)
      return hip_err(e, "persistent batch tables");
    off += tbytes[ph];
  }
  Bt->xwords = xw;
  Bt->plds = (size_t)(xw + tw) * sizeof(cpx<T>);
  int cus = 1;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, Bt->device) != hipSuccess || cus < 1) cus = 1;
  Bt->pgrid = batch_grid_t<T>(A, Bt->plds, cus);
  Bt->persist = true;
  return HDCONV_OK;
}

extern "C" {

hdconv_batch_t hdconv_plan_batched(const int64_t* L, const int64_t* M, int64_t count, int A, int B, int dims, int dtype,
                          const hdconv_options* opt) {
  clear_err();
  if (!L || !M || count < 1) {
    set_err(HDCONV_EINVAL, "need L, M and count >= 1");
    return nullptr;
  }
  if (dims != 1) {
    set_err(HDCONV_EUNSUPPORTED, "batched plans are one-dimensional (got dims = %d)", dims);
    return nullptr;
  }
  if (A < 2 || A > 3 || B != 1) {
    set_err(HDCONV_EUNSUPPORTED, "batched plans need A in {2,3} and B = 1");
    return nullptr;
  }
  if (opt && opt->mult != HDCONV_MULT_PRODUCT) {
    set_err(HDCONV_EUNSUPPORTED, "batched plans take the product operator only");
    return nullptr;
  }
  if (dtype != HDCONV_C64 && dtype != HDCONV_C128) {
    set_err(HDCONV_EINVAL, "dtype must be HDCONV_C64 or HDCONV_C128");
    return nullptr;
  }
  const int herm = (opt && (opt->flags & HDCONV_PLAN_HERMITIAN)) ? 1 : 0;
  const int ctr = (opt && (opt->flags & (HDCONV_PLAN_CENTERED | HDCONV_PLAN_HERMITIAN))) ? 1 : 0;
  for (int64_t i = 0; i < count; ++i)
    if (L[i] < 1 || L[i] > (int64_t(1) << 31) ||
        M[i] < (herm ? centered_min_padding(herm_full(L[i]), A)
                     : (ctr ? centered_min_padding(L[i], A) : (int64_t)A * (L[i] - 1) + 1))) {
      set_err(HDCONV_EINVAL, "convolution %lld: need L >= 1 and M >= %s (L=%lld, M=%lld)", (long long)i,
              herm ? "the Hermitian minimum (A+1)(ceil(L/2)-1)+1"
                   : (ctr ? "the centered minimum max(A(L-1-H)+H, L-1-H+AH)+1" : "A(L-1)+1"),
              (long long)L[i], (long long)M[i]);
      return nullptr;
    }
  int ndev = 0;
  hipError_t e = hipGetDeviceCount(&ndev);
  if (e != hipSuccess || ndev < 1) {
    set_err(HDCONV_ENODEV, "no HIP device available");
    return nullptr;
  }
  Batch* Bt = new (std::nothrow) Batch();
  if (!Bt) {
    set_err(HDCONV_ENOMEM, "host allocation failed");
    return nullptr;
  }
  (void)hipGetDevice(&Bt->device);
  Bt->A = A;
  Bt->B = B;
  Bt->dtype = dtype;
  Bt->flags = opt ? opt->flags : 0;
  Bt->count = count;
  Bt->L.assign(L, L + count);  // engine lengths (Hermitian: the full centered length)
  if (herm)
    for (auto& v : Bt->L) v = herm_full(v);
  Bt->M.assign(M, M + count);
  const int tb = tbytes_of(dtype);
  // the persistent form when every convolution has a compiled shape
  bool persist = !(Bt->flags & HDCONV_BATCH_GROUPED) && !ctr && (!opt || opt->tuner == HDCONV_TUNER_HEURISTIC);
  std::vector<DimPlan> pdims;
  if (persist) {
    pdims.resize((size_t)count);
    for (int64_t i = 0; i < count && persist; ++i) persist = persist_dim(Bt->L[i], M[i], A, tb, &pdims[(size_t)i]);
  }
  std::map<GroupKey, std::vector<int64_t>> byk;
  std::map<GroupKey, DimPlan> shape;
  for (int64_t i = 0; i < count; ++i) {
    DimPlan dp;
    std::string why;
    if (persist) {
      dp = pdims[(size_t)i];
    } else if (!choose_dim(Bt->L[i], M[i], A, tb, true, count, &dp, &why, ctr)) {
      set_err(HDCONV_EUNSUPPORTED, "convolution %lld (L=%lld): %s", (long long)i, (long long)L[i], why.c_str());
      free_batch(Bt);
      return nullptr;
    }
    dp.herm = herm;
    GroupKey k{dp.variant, dp.m, dp.p, dp.n, dp.q, dp.E_m, dp.E_p, dp.S, dp.rows_per_block};
    auto it = shape.find(k);
    if (it == shape.end()) shape[k] = dp;
    else {
      it->second.L = std::max(it->second.L, dp.L);
      it->second.M = std::max(it->second.M, dp.M);
    }
    byk[k].push_back(i);
  }
  if (opt && opt->tuner != HDCONV_TUNER_HEURISTIC) {
    int nc = 0, nt = 0;
    if (tune_batch_groups(A, B, dtype, Bt->device, opt, Bt->L, &byk, &shape, &nc, &nt) != HDCONV_OK) {
      free_batch(Bt);
      return nullptr;
    }
    Bt->tuner = opt->tuner;
    Bt->tuned_candidates = nc;
    Bt->timed_candidates = nt;
  }
  // largest rows first, so long groups start early on their side stream
  std::vector<GroupKey> order;
  for (auto& kv : byk) order.push_back(kv.first);
  std::sort(order.begin(), order.end(), [&](const GroupKey& a, const GroupKey& b) {
    return shape[a].m * shape[a].p * (int64_t)byk[a].size() > shape[b].m * shape[b].p * (int64_t)byk[b].size();
  });
  size_t off = 0;
  for (const GroupKey& k : order) {
    Plan* P = make_group_plan(A, B, dtype, shape[k], (int64_t)byk[k].size(), Bt->device);
    if (!P) {
      free_batch(Bt);
      return nullptr;
    }
    Bt->groups.push_back(P);
    Bt->members.push_back(byk[k]);
    Bt->task_off.push_back(off);
    off += align256(byk[k].size() * (tb == 4 ? sizeof(RowTask<float>) : sizeof(RowTask<double>)));
  }
  Bt->task_bytes = off;
  if ((e = hipMalloc((void**)&Bt->task_dev, off)) != hipSuccess ||
      (e = hipHostMalloc((void**)&Bt->task_host, off, hipHostMallocDefault)) != hipSuccess) {
    set_err(HDCONV_ENOMEM, "task tables: %s", hipGetErrorString(e));
    free_batch(Bt);
    return nullptr;
  }
  for (int i = 0; i <= kSideStreams; ++i) {
    hipStream_t* ps = i < kSideStreams ? &Bt->side[i] : &Bt->capture;
    if ((e = hipStreamCreateWithFlags(ps, hipStreamNonBlocking)) != hipSuccess) {
      hip_err(e, "hipStreamCreateWithFlags");
      free_batch(Bt);
      return nullptr;
    }
  }
  Bt->joins.resize(Bt->groups.size(), nullptr);
  bool ok = hipEventCreateWithFlags(&Bt->fork, hipEventDisableTiming) == hipSuccess &&
            hipEventCreateWithFlags(&Bt->copied, hipEventDisableTiming) == hipSuccess;
  for (auto& j : Bt->joins) ok = ok && hipEventCreateWithFlags(&j, hipEventDisableTiming) == hipSuccess;
  if (!ok) {
    set_err(HDCONV_EDEVICE, "event creation failed");
    free_batch(Bt);
    return nullptr;
  }
  if (persist && (tb == 4 ? build_persist<float>(Bt) : build_persist<double>(Bt)) != HDCONV_OK) {
    free_batch(Bt);
    return nullptr;
  }
  return (hdconv_batch_t)Bt;
}

int hdconv_execute_batched(hdconv_batch_t batch, const void* const* inputs, void* const* outputs, void* stream) {
  clear_err();
  if (!batch || !inputs || !outputs) return set_err(HDCONV_EINVAL, "batch, inputs and outputs must not be NULL");
  Batch* Bt = (Batch*)batch;
  for (int64_t i = 0; i < Bt->count; ++i) {
    for (int a = 0; a < Bt->A; ++a)
      if (!inputs[i * Bt->A + a]) return set_err(HDCONV_EINVAL, "inputs[%lld] is NULL", (long long)(i * Bt->A + a));
    if (!outputs[i * Bt->B]) return set_err(HDCONV_EINVAL, "outputs[%lld] is NULL", (long long)(i * Bt->B));
  }
  int cur = -1;
  (void)hipGetDevice(&cur);
  if (cur != Bt->device) return set_err(HDCONV_EINVAL, "batch belongs to device %d, current is %d", Bt->device, cur);
  hipStream_t s = (hipStream_t)stream;
  return Bt->dtype == HDCONV_C64 ? run_batched<float>(Bt, inputs, outputs, s)
                                 : run_batched<double>(Bt, inputs, outputs, s);
}

int hdconv_batch_info(hdconv_batch_t batch, hdconv_dim_info_t* groups, int64_t* counts, int cap, int* ngroups) {
  clear_err();
  if (!batch) return set_err(HDCONV_EINVAL, "batch is NULL");
  const Batch* Bt = (const Batch*)batch;
  if (ngroups) *ngroups = (int)Bt->groups.size();
  for (int g = 0; g < (int)Bt->groups.size() && g < cap; ++g) {
    const DimPlan& dp = Bt->groups[g]->dp[0];
    if (groups) {
      hdconv_dim_info_t& di = groups[g];
      memset(&di, 0, sizeof(di));
      di.L = dp.L;
      di.M = dp.M;
      di.m = dp.m;
      di.p = dp.p;
      di.n = dp.n;
      di.q = dp.q;
      di.D = dp.D;
      di.variant = dp.variant;
      di.E_m = dp.E_m;
      di.E_p = dp.E_p;
      di.S = dp.S;
      di.rows_per_block = dp.rows_per_block;
      di.tw_m = dp.fd_m.N ? dp.fd_m.twmode + 1 : 0;
      di.tw_p = dp.fd_p.N ? dp.fd_p.twmode + 1 : 0;
      di.centered = dp.herm ? 2 : dp.ctr;
    }
    if (counts) counts[g] = (int64_t)Bt->members[g].size();
  }
  return HDCONV_OK;
}

int hdconv_batch_stats(hdconv_batch_t batch, hdconv_batch_stats_t* out) {
  clear_err();
  if (!batch || !out) return set_err(HDCONV_EINVAL, "batch and out must not be NULL");
  const Batch* Bt = (const Batch*)batch;
  memset(out, 0, sizeof(*out));
  out->persistent = Bt->persist ? 1 : 0;
  out->grid = Bt->pgrid;
  out->tasks = (int64_t)Bt->ntasks[0] + Bt->ntasks[1] + Bt->ntasks[2];
  out->lds_bytes = (int64_t)Bt->plds;
  for (const Plan* P : Bt->groups) out->work_bytes += (int64_t)P->work_bytes;
  return HDCONV_OK;
}

void hdconv_batch_destroy(hdconv_batch_t batch) { free_batch((Batch*)batch); }

}  // extern "C"
