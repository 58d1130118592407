// hd_k_batch.hip -- many independent 1D convolutions of uneven length in
// persistent launches over device task tables.
//
// The batch is split into size buckets; each bucket's convolutions share a
// shape (m, p, n, q):
//  * whole rows (p = 1): the direct form of Sec. 2 (Algorithms 3-6), one row
//    per G = N/E lanes, the lean row body (hd_lean.hpp);
//  * inner form (Sec. 6.1, q = n p, all n residues at once): per convolution
//      column pass  W_a[v p + u][s] = sum_t zeta_p^{u t} zeta_q^{v t} f_a[t m + s]
//      row pass     Y[j] = zeta_{qm}^{-r s} ifft_m(prod_a fft_m(zeta_{qm}^{r s} W_a[j])),
//                   row j = v p + u, residue r = u n + v (in place over W_0)
//      back pass    h[t m + s] = sum_v zeta_q^{-v t} sum_u zeta_p^{-u t} Y[v p + u][s] / (q m).
// A batch runs as three launches of one kernel, one per pass of the inner
// form (the whole rows join the last), each over its own task table: a task
// is a range of units of one pass of one convolution, or up to RPB whole
// rows, and each of the launch's resident workgroups takes every gridDim-th
// task.  The passes meet at kernel boundaries, which make one pass's stores
// visible to the next on every XCD: a dependency inside one launch would
// need an L2 write-back and invalidation per task (measured on the 4096-
// convolution workload: 5.8 ms with per-task counters and device-scope
// fences against 1.7 ms without them).
#include "hd_lean.hpp"

namespace hd {

// ---------------------------------------------------------------------------
// compiled bodies

// Whole rows: N points (64 .. 2048 in FP32 with 8 points per lane, 64 .. 1024
// in FP64 with 4), one block (L <= N).  Inner form: rows of 2048 points (FP32,
// 8 per lane) or 1024 (FP64, 4 per lane), columns of p = 2 .. 64 points, and
// in FP32 also 3 * 2^k = 12 .. 96 points (12 per lane: the padding p m / L
// drops from 1.44 to about 1.2 on average; in FP64 those bodies spill).
// (Whole rows of two blocks are left to the inner form with p = 2: their
// body needs more registers than the persistent kernel's budget.)
template <typename T>
constexpr int bw_rows_e() {
  return sizeof(T) == 4 ? 8 : 4;
}
template <typename T>
constexpr int bw_inner_m() {
  return sizeof(T) == 4 ? 2048 : 1024;
}
// points per lane of a p-point column transform
__host__ __device__ constexpr int bw_col_e(int p, int tbytes) {
  return p % 3 == 0 ? 12 : (p <= 4 ? p : (tbytes == 4 ? 8 : 4));
}
constexpr int kBodyInner = 100;   // inner-form bodies: kBodyInner + log2(p) - 1
constexpr int kBodyInner3 = 110;  // and kBodyInner3 + log2(p / 3) for p = 3 * 2^k

__host__ __device__ constexpr int ilog2c(int x) {
  int r = 0;
  while ((1 << r) < x) ++r;
  return r;
}

// ---------------------------------------------------------------------------
// inner-form pass bodies (one unit each)

// Column pass: input ai, columns s = ct S + c (c < S); lane g of a column
// holds points t = g + G e.  The p-point transforms of S columns share one
// exchange area (point i of column c at xc[i S]).
template <typename T, int P, int E, int S>
__device__ __forceinline__ void batch_colf(const BatchBucket<T>& b, const RowTask<T>& rt, int ai, int ct,
                                           cpx<T>* xc, const cpx<T>* twp, const cpx<T>* zq, cpx<T>* w, int tid) {
  constexpr int G = P / E;
  const int c = tid % S, g = tid / S;
  const int m = b.m, n = b.n;
  const int s = ct * S + c;
  const uint32_t L = (uint32_t)rt.L;
  const cpx<T>* src = rt.in[ai];
  cpx<T> x[E];
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const uint32_t i = (uint32_t)(g + G * e) * (uint32_t)m + (uint32_t)s;
    const cpx<T> v = src[i < L ? i : L - 1];  // no branch: a point beyond L reads point L-1
    x[e] = i < L ? v : czero<T>();
  }
  for (int v = 0; v < n; ++v) {
    cpx<T> y[E];
#pragma unroll
    for (int e = 0; e < E; ++e) y[e] = cmul(x[e], zq[v * (g + G * e)]);  // v t < n p = q
    lean_fft<T, P, E, +1, S, false>(y, g, xc + c, twp);
    cpx<T>* dst = w + (int64_t)(v * P + g) * m + s;
#pragma unroll
    for (int e = 0; e < E; ++e) dst[(int64_t)G * e * m] = y[e];
  }
}

// Back pass: columns s = ct S + c of the row-pass result y (rows v p + u).
template <typename T, int P, int E, int S>
__device__ __forceinline__ void batch_colb(const BatchBucket<T>& b, const RowTask<T>& rt, int ct, cpx<T>* xc,
                                           const cpx<T>* twp, const cpx<T>* zq, const cpx<T>* w, int tid) {
  constexpr int G = P / E;
  const int c = tid % S, g = tid / S;
  const int m = b.m, n = b.n;
  const int s = ct * S + c;
  cpx<T> acc[E];
  for (int v = 0; v < n; ++v) {
    const cpx<T>* src = w + (int64_t)(v * P + g) * m + s;
    cpx<T> y[E];
#pragma unroll
    for (int e = 0; e < E; ++e) y[e] = src[(int64_t)G * e * m];
    lean_fft<T, P, E, -1, S, false>(y, g, xc + c, twp);
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const cpx<T> z = cmulc(y[e], zq[v * (g + G * e)]);
      acc[e] = v == 0 ? z : acc[e] + z;
    }
  }
  const uint32_t L = (uint32_t)rt.L;
  cpx<T>* dst = rt.out;
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const uint32_t i = (uint32_t)(g + G * e) * (uint32_t)m + (uint32_t)s;
    if (i < L) dst[i] = cscale(acc[e], b.scale);
  }
}

// Row pass: rows j0 .. j0+nj-1 of one convolution, one row at a time (G =
// N / E = kBatchThreads lanes).  The A inputs of a row are loaded together,
// and the next row's are loaded while the current row's inverse transform
// and stores run.
template <typename T, int N, int E, int A>
__device__ __forceinline__ void batch_rowp(const BatchBucket<T>& b, int64_t cq, int j0, int nj, cpx<T>* xr,
                                           const cpx<T>* twm, int tid) {
  constexpr int G = N / E;
  const int g = tid;
  cpx<T> x[A][E];
  auto load = [&](int j) {
    const int64_t off = (cq + j) * (int64_t)N + g;
#pragma unroll
    for (int ai = 0; ai < A; ++ai)
#pragma unroll
      for (int e = 0; e < E; ++e) x[ai][e] = b.work[ai][off + G * e];
  };
  load(j0);
  for (int k = 0; k < nj; ++k) {
    const int j = j0 + k;
    const int u = j % b.p, v = j / b.p;
    const uint32_t r = (uint32_t)(u * b.n + v);
    b.zqm.template run<E>(r * (uint32_t)g, r * (uint32_t)G, [&](int e, cpx<T> z) {
#pragma unroll
      for (int ai = 0; ai < A; ++ai) x[ai][e] = cmul(x[ai][e], z);
    });
    cpx<T> pr[E];
#pragma unroll
    for (int ai = 0; ai < A; ++ai) {
      cpx<T> w[E];
#pragma unroll
      for (int e = 0; e < E; ++e) w[e] = x[ai][e];
      lean_fft<T, N, E, +1>(w, g, xr, twm);
#pragma unroll
      for (int e = 0; e < E; ++e) pr[e] = ai == 0 ? w[e] : cmul(pr[e], w[e]);
    }
    if (k + 1 < nj) load(j + 1);
    lean_fft<T, N, E, -1>(pr, g, xr, twm);
    cpx<T>* dst = b.work[0] + (cq + j) * (int64_t)N + g;
    b.zqm.template run<E>(r * (uint32_t)g, r * (uint32_t)G, [&](int e, cpx<T> z) { dst[G * e] = cmulc(pr[e], z); });
  }
}

// ---------------------------------------------------------------------------
// dispatch of one task to the compiled body of its bucket

constexpr int kBatchKeep = 8;  // input words per lane held across the residues

template <typename T, int A, int N, int P>
__device__ __forceinline__ void run_rows_task(const BatchBucket<T>& b, const BatchTask& tk, cpx<T>* lds,
                                              const cpx<T>* tab, int tid) {
  constexpr int E = bw_rows_e<T>();
  constexpr int G = N / E;
  constexpr int XW = lean_xwords<N, E>();
  const int slot = tid / G, g = tid % G;
  const bool valid = slot < tk.nu;
  const RowTask<T>& rt = b.rows[tk.conv + (valid ? slot : 0)];
  const cpx<T>* src[A];
#pragma unroll
  for (int ai = 0; ai < A; ++ai) src[ai] = rt.in[ai] + g;
  const cpx<T>* zA = tab + b.ntw_m;
  const cpx<T>* zB = zA + b.q * G;
  const cpx<T>* zC = zB + b.q * E;
  lean_row<T, N, E, A, P, false, kBatchKeep>(src, rt.out + g, valid, (uint32_t)rt.L, b.q, b.scale, g, lds + slot * XW,
                                             tab, zA, zB, zC);
}

template <typename T, int A, int P>
__device__ __forceinline__ void run_inner_task(const BatchBucket<T>& b, const BatchTask& tk, cpx<T>* lds,
                                               const cpx<T>* tab, int tid) {
  constexpr int EP = bw_col_e(P, sizeof(T));
  constexpr int S = kBatchThreads / (P / EP);
  constexpr int N = bw_inner_m<T>();
  const RowTask<T>& rt = b.rows[tk.conv];
  const int64_t cq = (int64_t)tk.conv * b.q;  // first work row of the convolution
  const int tiles = b.m / S;
  if (tk.kind == BK_ROWP) {
    batch_rowp<T, N, bw_rows_e<T>(), A>(b, cq, tk.u0, tk.nu, lds, tab, tid);
    return;
  }
  for (int k = 0; k < tk.nu; ++k) {
    const int unit = tk.u0 + k;
    if (tk.kind == BK_COLF) {
      const int ai = unit / tiles, ct = unit % tiles;
      batch_colf<T, P, EP, S>(b, rt, ai, ct, lds, tab, tab + b.ntw_p, b.work[ai] + cq * b.m, tid);
    } else {
      batch_colb<T, P, EP, S>(b, rt, unit, lds, tab, tab + b.ntw_p, b.work[0] + cq * b.m, tid);
    }
  }
}

template <typename T, int A>
__device__ __forceinline__ void run_task(const BatchBucket<T>& b, const BatchTask& tk, cpx<T>* lds,
                                         const cpx<T>* tab, int tid) {
  switch (b.body) {
#define HD_ROWS_BODY(NN, PP)                                                        \
  case (ilog2c(NN) - 6) * 2 + (PP - 1):                                             \
    if constexpr (NN / bw_rows_e<T>() <= kBatchThreads) run_rows_task<T, A, NN, PP>(b, tk, lds, tab, tid); \
    break;
    HD_ROWS_BODY(64, 1) HD_ROWS_BODY(128, 1) HD_ROWS_BODY(256, 1) HD_ROWS_BODY(512, 1)
    HD_ROWS_BODY(1024, 1) HD_ROWS_BODY(2048, 1)
#undef HD_ROWS_BODY
#define HD_INNER_BODY(PP)                                                           \
  case kBodyInner + ilog2c(PP) - 1:                                                 \
    run_inner_task<T, A, PP>(b, tk, lds, tab, tid);                                      \
    break;
    HD_INNER_BODY(2) HD_INNER_BODY(4) HD_INNER_BODY(8) HD_INNER_BODY(16) HD_INNER_BODY(32) HD_INNER_BODY(64)
#undef HD_INNER_BODY
#define HD_INNER_BODY3(PP)                                                          \
  case kBodyInner3 + ilog2c(PP / 3):                                                \
    if constexpr (sizeof(T) == 4) run_inner_task<T, A, PP>(b, tk, lds, tab, tid);   \
    break;
    HD_INNER_BODY3(12) HD_INNER_BODY3(24) HD_INNER_BODY3(48) HD_INNER_BODY3(96)
#undef HD_INNER_BODY3
    default:
      break;
  }
}

// Tables of a task's kind in LDS (tab): whole rows: the m-point per-stage
// twiddles and the residue tables of lean_row_tables; column passes: the
// p-point per-stage twiddles then zeta_q^k (k < q); row pass: the m-point
// per-stage twiddles.
template <typename T>
__device__ __forceinline__ void stage_tables(const BatchBucket<T>& b, int kind, cpx<T>* tab, int tid) {
  if (kind == BK_ROWS) {
    switch (b.body) {
#define HD_TAB(NN, PP)                                                                                      \
  case (ilog2c(NN) - 6) * 2 + (PP - 1): {                                                                   \
    constexpr int E = bw_rows_e<T>();                                                                       \
    cpx<T>* zA = tab + b.ntw_m;                                                                             \
    cpx<T>* zB = zA + b.q * (NN / E);                                                                       \
    lean_row_tables<T, NN, E, PP>(b.tw_m, b.ntw_m, b.zqm, b.q, tid, kBatchThreads, tab, zA, zB, zB + b.q * E); \
    break;                                                                                                  \
  }
      HD_TAB(64, 1) HD_TAB(128, 1) HD_TAB(256, 1) HD_TAB(512, 1) HD_TAB(1024, 1) HD_TAB(2048, 1)
#undef HD_TAB
      default:
        break;
    }
  } else if (kind == BK_ROWP) {
    for (int i = tid; i < b.ntw_m; i += kBatchThreads) tab[i] = b.tw_m[i];
  } else {
    for (int i = tid; i < b.ntw_p; i += kBatchThreads) tab[i] = b.tw_p[i];
    for (int i = tid; i < b.q; i += kBatchThreads) tab[b.ntw_p + i] = b.zq[i];
  }
}

// Waves per SIMD the register allocation aims at.
template <typename T>
constexpr int batch_waves() {
  return 3;
}

template <typename T, int A>
__global__ void __launch_bounds__(kBatchThreads, batch_waves<T>()) k_batch(BatchArgs<T> a) {
  cpx<T>* lds = smem_as<T>();
  cpx<T>* tab = lds + a.xwords;
  int staged = -1;  // bucket * 4 + table kind held in LDS
  for (int t = blockIdx.x; t < a.ntasks; t += gridDim.x) {
    // The lane index is made opaque per task, so that no body's lane
    // arithmetic is hoisted out of the task loop (each would hold registers
    // for the whole launch).
    int tid = (int)threadIdx.x;
    asm volatile("" : "+v"(tid));
    const BatchTask tk = a.tasks[t];
    const BatchBucket<T>& b = a.buckets[tk.bucket];
    const int tkind = tk.kind == BK_COLB ? BK_COLF : tk.kind;  // both column passes use one table set
    const int key = tk.bucket * 4 + tkind;
    if (key != staged) {
      __syncthreads();  // the previous task's reads of the tables are done
      stage_tables<T>(b, tkind, tab, tid);
      staged = key;
      __syncthreads();
    }
    run_task<T, A>(b, tk, lds, tab, tid);
    __syncthreads();  // the exchange area is free again
  }
}

// ---------------------------------------------------------------------------
// host side

#if !defined(HD_PART) || HD_PART == 1  // host helpers, in one object only
bool batch_shape(int inner, int64_t m, int64_t p, int tbytes, int* body, int* E_m, int* E_p, int* S) {
  const int e_rows = tbytes == 4 ? 8 : 4;
  auto pow2 = [](int64_t x) { return x > 0 && (x & (x - 1)) == 0; };
  if (!inner) {
    const int64_t nmax = kBatchThreads * (int64_t)e_rows;  // one row per workgroup at most
    if (!pow2(m) || m < 64 || m > nmax || p != 1) return false;
    *body = (ilog2c((int)m) - 6) * 2;
    *E_m = e_rows;
    *E_p = 0;
    *S = 0;
    return true;
  }
  if (m != (tbytes == 4 ? 2048 : 1024)) return false;
  if (tbytes == 4 && p % 3 == 0 && pow2(p / 3) && p >= 12 && p <= 96) {
    *body = kBodyInner3 + ilog2c((int)p / 3);
  } else if (pow2(p) && p >= 2 && p <= 64) {
    *body = kBodyInner + ilog2c((int)p) - 1;
  } else {
    return false;
  }
  *E_m = e_rows;
  *E_p = bw_col_e((int)p, tbytes);
  *S = kBatchThreads / ((int)p / *E_p);
  return true;
}

void batch_lds_words(int body, int m, int p, int q, int ntw_m, int ntw_p, int tbytes, int* xwords, int* twords) {
  const int e_rows = tbytes == 4 ? 8 : 4;
  if (body < kBodyInner) {
    const int N = m, G = N / e_rows;
    const int ps = ilog2c(ct_radix(N, e_rows));
    *xwords = (kBatchThreads / G) * (N + (N >> ps));
    *twords = ntw_m + q * (G + e_rows + 1);
    return;
  }
  const int ep = bw_col_e(p, tbytes), S = kBatchThreads / (p / ep);
  const int ps = ilog2c(ct_radix(m, e_rows));
  *xwords = std::max(p * S, m + (m >> ps));
  *twords = std::max(ntw_p + q, ntw_m);
}
#endif

template <typename T, int A>
static int batch_resident(size_t lds) {
  static std::mutex mu;
  static std::unordered_map<size_t, int> seen;
  std::lock_guard<std::mutex> lk(mu);
  auto it = seen.find(lds);
  if (it != seen.end()) return it->second;
  int n = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, reinterpret_cast<const void*>(k_batch<T, A>), kBatchThreads,
                                                   lds) != hipSuccess || n < 1)
    n = 1;
  seen[lds] = n;
  return n;
}

template <typename T>
int batch_grid_t(int A, size_t lds, int cus) {
  const int r = A == 2 ? batch_resident<T, 2>(lds) : batch_resident<T, 3>(lds);
  return std::max(1, r * cus);
}

template <typename T>
hipError_t launch_batch(const BatchArgs<T>& a, int A, int grid, size_t lds, hipStream_t s) {
  if (grid < 1 || a.ntasks < 0) return HD_BAD;
  if (A == 2) return go(k_batch<T, 2>, dim3(grid), dim3(kBatchThreads), lds, s, a);
  if (A == 3) return go(k_batch<T, 3>, dim3(grid), dim3(kBatchThreads), lds, s, a);
  return HD_BAD;
}

#define HD_INST(T)                                                                             \
  template hipError_t launch_batch<T>(const BatchArgs<T>&, int, int, size_t, hipStream_t); \
  template int batch_grid_t<T>(int, size_t, int);
#if !defined(HD_PART) || HD_PART == 1
HD_INST(float)
#endif
#if !defined(HD_PART) || HD_PART == 2
HD_INST(double)
#endif
#undef HD_INST

}  // namespace hd
