// hd_k_lean.hip -- whole rows of one block (p = 1) with the product
// operator, for launches over many rows: the innermost dimension of 2D/3D
// plans and the rows of 1D copies.
//
// It computes what k_fused1d computes for P = 1 (the direct form of Sec. 2,
// Algorithms 3-6): for each residue r < q,
//   W_s = zeta_{qm}^{r s} f_s        (zero for s >= L)
//   F_a = fft_m(W) for each input a;  H = prod_a F_a
//   h_s += zeta_{qm}^{-r s} ifft_m(H)_s,
// and out_s = h_s / (q m) for s < L.  It is laid out for throughput:
//  * the transform size and points per lane are template parameters: the
//    stage plan is unrolled, and every LDS address of an exchange is one
//    per-lane base plus a constant (the instruction's offset field);
//  * the inputs are transformed one after another through one exchange
//    area per row;
//  * the residue twiddles come from two small LDS tables,
//    zeta_{qm}^{r(g + G e)} = zeta_{qm}^{r g} zeta_{qm}^{r G e}, made once
//    per workgroup;
//  * a workgroup loops over rows (the grid is sized to the resident
//    workgroups), so its tables are staged into LDS once.
#include <map>
#include <utility>

#include "hd_lean.hpp"
#include "hd_plan.hpp"

namespace hd {

// The q = 2 twiddle table (N words) is kept in LDS only where it costs at
// most 4 KB.
template <typename T, int N>
constexpr bool lean_zf() {
  return N * (int)sizeof(cpx<T>) <= 4096;
}

template <typename T, int N, int E, int A, int RPB, int WAVES, bool FULL, int P, bool ZF = false>
__global__ void __launch_bounds__(RPB*(N / E), WAVES) k_rows_lean(LeanRowArgs<T> a) {
  constexpr int G = N / E;
  constexpr int NT = RPB * G;
  constexpr int XW = lean_xwords<N, E>();
  const int slot = threadIdx.x / G;
  const int g = threadIdx.x % G;
  const int q = a.q;
  cpx<T>* lds = smem_as<T>();
  cpx<T>* xr = lds + slot * XW;
  cpx<T>* twl = lds + RPB * XW;        // per-stage FFT twiddles
  cpx<T>* zA = twl + a.fd.ntw_stage;   // zeta_{qm}^{r g}, [r][g]
  cpx<T>* zB = zA + q * G;             // zeta_{qm}^{r G e}, [r][e]
  cpx<T>* zC = zB + q * E;             // zeta_q^r = zeta_{qm}^{r m} (second block, P = 2)
  cpx<T>* zF = zC + q;                 // zeta_{qm}^s, s < N (q = 2, ZF)
  // the per-stage tables follow the two-level one
  lean_row_tables<T, N, E, P>(a.fft_tw + a.fd.ntw, a.fd.ntw_stage, a.zqm, q, (int)threadIdx.x, NT, twl, zA, zB, zC);
  if constexpr (ZF)
    if (q == 2) lean_row_q2_table<T, N>(a.zqm, (int)threadIdx.x, NT, zF);
  __syncthreads();
  const int64_t step = (int64_t)gridDim.x * RPB;
  for (int64_t row0 = (int64_t)blockIdx.x * RPB; row0 < a.nrows; row0 += step) {
    const int64_t row = row0 + slot;
    const bool valid = row < a.nrows;
    const int64_t rowc = valid ? row : a.nrows - 1;
    const cpx<T>* src[A];
#pragma unroll
    for (int ai = 0; ai < A; ++ai) src[ai] = a.in[ai] + rowc * a.in_stride + g;
    lean_row<T, N, E, A, P, FULL, 8, ZF>(src, a.out + rowc * a.out_stride + g, valid, a.L, q, a.scale, g, xr, twl,
                                         zA, zB, zC, zF + g);
  }
}

// Outer dimension of a 2D/3D convolution (Sec. 5), direct form with one or
// two blocks (p <= 2), dense planes [nb][L][R]: what k_outer_fwd /
// k_outer_bwd compute for an ordinary (not centered) dimension, laid out like
// the lean row kernel.  A workgroup takes S adjacent columns (lanes of one
// column are S apart, so every global access of a wave covers S consecutive
// words per row) and loops over (input, plane, column tile) units.
//   forward:  out[a][((b D + dr) m + k) R + col] = fft_m(W)_k for r = r0 + dr,
//             W_s = zeta_{qm}^{r s} (x_s + zeta_q^r x_{m+s})
//   backward: out[b][t m + s][col] (+)= sum_r zeta_q^{-r t} zeta_{qm}^{-r s} ifft_m(y_r)_s / (q m)
// (a launch takes the residues r0 .. r0+D-1; the backward adds to the output
// for later residue blocks)
template <typename T, int N, int E, int S, bool FWD, int WAVES, bool FULL, int P>
__global__ void __launch_bounds__(S*(N / E), WAVES) k_outer_lean(OuterLeanArgs<T> a) {
  constexpr int G = N / E;
  constexpr int NT = S * G;
  const int c = threadIdx.x % S;
  const int g = threadIdx.x / S;
  const int q = a.q;
  const int64_t R = a.R;
  cpx<T>* lds = smem_as<T>();
  cpx<T>* xr = lds + c;                // point i of this column at xr[i S]
  cpx<T>* twl = lds + N * S;           // per-stage FFT twiddles
  cpx<T>* zA = twl + a.fd.ntw_stage;   // zeta_{qm}^{r g}, [r][g]
  cpx<T>* zB = zA + q * G;             // zeta_{qm}^{r G e}, [r][e]
  cpx<T>* zC = zB + q * E;             // zeta_q^r (second block, P = 2)
  {
    const cpx<T>* st = a.fft_tw + a.fd.ntw;
    for (int i = threadIdx.x; i < a.fd.ntw_stage; i += NT) twl[i] = st[i];
    for (int i = threadIdx.x; i < q * G; i += NT) zA[i] = a.zqm.get((uint32_t)((i / G) * (i % G)));
    for (int i = threadIdx.x; i < q * E; i += NT) zB[i] = a.zqm.get((uint32_t)((i / E) * G * (i % E)));
    if constexpr (P == 2)
      for (int i = threadIdx.x; i < q; i += NT) zC[i] = a.zqm.get((uint32_t)(i * N));
  }
  __syncthreads();
  constexpr bool full = FULL;  // one block and L = m: no point beyond L
  const int64_t tiles = (R + S - 1) / S;
  const int64_t units = tiles * a.nb * (FWD ? a.na : 1);
  const int64_t GR = (int64_t)G * R;  // words between a lane's points
  const int64_t NR = (int64_t)N * R;  // words between the blocks
  for (int64_t u = blockIdx.x; u < units; u += gridDim.x) {
    const int64_t ct = u % tiles;
    const int64_t rest = u / tiles;
    const int64_t b = rest % a.nb;
    const int ai = FWD ? (int)(rest / a.nb) : 0;
    const int64_t col = ct * S + c;
    const bool valid = col < R;
    const int64_t colc = valid ? col : R - 1;
    if constexpr (FWD) {
      const cpx<T>* src = a.in[ai] + b * a.in_bstride + colc + (int64_t)g * R;
      cpx<T> x[P][E];
#pragma unroll
      for (int t = 0; t < P; ++t)
#pragma unroll
        for (int e = 0; e < E; ++e) {
          if constexpr (full) {
            x[t][e] = src[e * GR];
          } else {
            const uint32_t i = (uint32_t)(t * N + g + G * e);
            const cpx<T> v = src[((int64_t)(i < a.L ? i : a.L - 1) - g) * R];
            x[t][e] = i < a.L ? v : czero<T>();
          }
        }
      for (int dr = 0; dr < a.D; ++dr) {
        const int r = a.r0 + dr;
        const cpx<T> za = zA[r * G + g];
        const cpx<T> zc = P == 2 ? zC[r] : mk(T(1), T(0));
        cpx<T> w[E];
#pragma unroll
        for (int e = 0; e < E; ++e) {
          cpx<T> xv = x[0][e];
          if constexpr (P == 2) xv = xv + cmul(x[P - 1][e], zc);
          w[e] = cmul(xv, cmul(za, zB[r * E + e]));
        }
        lean_fft<T, N, E, +1, S, false>(w, g, xr, twl);
        if (valid) {
          cpx<T>* dst = a.out[ai] + ((b * a.D + dr) * N + g) * R + col;
#pragma unroll
          for (int e = 0; e < E; ++e) dst[e * GR] = w[e];
        }
      }
    } else {
      cpx<T> acc[P][E];
      for (int dr = 0; dr < a.D; ++dr) {
        const int r = a.r0 + dr;
        const cpx<T>* src = a.in[0] + ((b * a.D + dr) * N + g) * R + colc;
        cpx<T> y[E];
#pragma unroll
        for (int e = 0; e < E; ++e) y[e] = src[e * GR];
        lean_fft<T, N, E, -1, S, false>(y, g, xr, twl);
        const cpx<T> za = zA[r * G + g];
        const cpx<T> zc = P == 2 ? zC[r] : mk(T(1), T(0));
#pragma unroll
        for (int e = 0; e < E; ++e) {
          const cpx<T> v = cmulc(y[e], cmul(za, zB[r * E + e]));
          acc[0][e] = dr == 0 ? v : acc[0][e] + v;
          if constexpr (P == 2) {
            const cpx<T> v1 = cmulc(v, zc);
            acc[P - 1][e] = dr == 0 ? v1 : acc[P - 1][e] + v1;
          }
        }
      }
      if (valid) {
        cpx<T>* dst = a.out[0] + b * a.out_bstride + col + (int64_t)g * R;
#pragma unroll
        for (int t = 0; t < P; ++t)
#pragma unroll
          for (int e = 0; e < E; ++e)
            if (full || (uint32_t)(t * N + g + G * e) < a.L) {
              cpx<T> v = cscale(acc[t][e], a.scale);
              if (a.add) v = v + dst[t * NR + e * GR];
              dst[t * NR + e * GR] = v;
            }
      }
    }
  }
}

// Outer dimension in the inner form, the m-point pass over dense planes of
// m rows (plane b is row j = b mod q of its transform, residue
// r = (j mod p) n + j div p): forward W = fft_m(zeta_{qm}^{r s} y_s), backward
// y_s = zeta_{qm}^{-r s} ifft_m(W)_s, in place.  Layout and lanes as in
// k_outer_lean; the residue twiddles come from the two-level table (one
// residue per plane).
template <typename T, int N, int E, int S, bool FWD, int WAVES>
__global__ void __launch_bounds__(S*(N / E), WAVES) k_outer_inner_rows(OuterLeanArgs<T> a) {
  constexpr int G = N / E;
  constexpr int NT = S * G;
  const int c = threadIdx.x % S;
  const int g = threadIdx.x / S;
  const int q = a.q, n = a.inner_n, p = q / n;
  const int64_t R = a.R;
  cpx<T>* lds = smem_as<T>();
  cpx<T>* xr = lds + c;       // point i of this column at xr[i S]
  cpx<T>* twl = lds + N * S;  // per-stage FFT twiddles
  {
    const cpx<T>* st = a.fft_tw + a.fd.ntw;
    for (int i = threadIdx.x; i < a.fd.ntw_stage; i += NT) twl[i] = st[i];
  }
  __syncthreads();
  const int64_t tiles = (R + S - 1) / S;
  const int64_t units = tiles * a.nb * (FWD ? a.na : 1);
  const int64_t GR = (int64_t)G * R;
  for (int64_t u = blockIdx.x; u < units; u += gridDim.x) {
    const int64_t ct = u % tiles;
    const int64_t rest = u / tiles;
    const int64_t b = rest % a.nb;
    const int ai = FWD ? (int)(rest / a.nb) : 0;
    const int64_t col = ct * S + c;
    const bool valid = col < R;
    const int64_t colc = valid ? col : R - 1;
    const int j = (int)(b % q);
    const uint32_t r = (uint32_t)((j % p) * n + j / p);
    const int64_t base = b * (int64_t)N * R + (int64_t)g * R;
    const cpx<T>* src = a.in[ai] + base + colc;
    cpx<T> y[E];
#pragma unroll
    for (int e = 0; e < E; ++e) y[e] = src[e * GR];
    if constexpr (FWD) {
      a.zqm.template run<E>(r * (uint32_t)g, r * (uint32_t)G, [&](int e, cpx<T> z) { y[e] = cmul(y[e], z); });
      lean_fft<T, N, E, +1, S, false>(y, g, xr, twl);
    } else {
      lean_fft<T, N, E, -1, S, false>(y, g, xr, twl);
      a.zqm.template run<E>(r * (uint32_t)g, r * (uint32_t)G, [&](int e, cpx<T> z) { y[e] = cmulc(y[e], z); });
    }
    if (valid) {
      cpx<T>* dst = a.out[ai] + base + col;
#pragma unroll
      for (int e = 0; e < E; ++e) dst[e * GR] = y[e];
    }
  }
}

// Outer dimension in the inner form, the column passes (see OuterColArgs):
// S adjacent columns of one block offset s per unit, lanes of a column S
// apart, the p-point transforms interleaved in LDS.  Units are (input,
// plane, s, column tile), column tiles fastest.
template <typename T, int P, int E, int S, bool FWD, int WAVES>
__global__ void __launch_bounds__(S*(P / E), WAVES) k_outer_cols(OuterColArgs<T> a) {
  constexpr int G = P / E;
  constexpr int NT = S * G;
  const int c = threadIdx.x % S;
  const int g = threadIdx.x / S;
  const int m = a.m, n = a.n, q = n * P;
  const int64_t R = a.R;
  cpx<T>* lds = smem_as<T>();
  cpx<T>* xc = lds + c;       // point t of this column at xc[t S]
  cpx<T>* twl = lds + P * S;  // per-stage twiddles of the p-point transform
  cpx<T>* zq = twl + a.fd.ntw_stage;
  {
    const cpx<T>* st = a.fft_tw + a.fd.ntw;
    for (int i = threadIdx.x; i < a.fd.ntw_stage; i += NT) twl[i] = st[i];
    for (int i = threadIdx.x; i < q; i += NT) zq[i] = a.zq[i];
  }
  __syncthreads();
  const int64_t tiles = (R + S - 1) / S;
  const int64_t units = tiles * m * a.nb * (FWD ? a.na : 1);
  for (int64_t u = blockIdx.x; u < units; u += gridDim.x) {
    const int64_t ct = u % tiles;
    int64_t rest = u / tiles;
    const int s = (int)(rest % m);
    rest /= m;
    const int64_t b = rest % a.nb;
    const int ai = FWD ? (int)(rest / a.nb) : 0;
    const int64_t col = ct * S + c;
    const bool valid = col < R;
    const int64_t colc = valid ? col : R - 1;
    if constexpr (FWD) {
      const cpx<T>* src = a.in[ai] + b * a.in_bstride + colc;
      cpx<T> x[E];
#pragma unroll
      for (int e = 0; e < E; ++e) {
        const int64_t i = (int64_t)(g + G * e) * m + s;
        const cpx<T> v = src[(i < a.L ? i : a.L - 1) * R];  // no branch: beyond L reads the last point
        x[e] = i < a.L ? v : czero<T>();
      }
      for (int v = 0; v < n; ++v) {
        cpx<T> y[E];
#pragma unroll
        for (int e = 0; e < E; ++e) y[e] = cmul(x[e], zq[v * (g + G * e)]);  // v t < n p = q
        lean_fft<T, P, E, +1, S, false>(y, g, xc, twl);
        if (valid) {
          cpx<T>* dst = a.out[ai] + ((b * q + v * P + g) * (int64_t)m + s) * R + col;
#pragma unroll
          for (int e = 0; e < E; ++e) dst[(int64_t)G * e * m * R] = y[e];
        }
      }
    } else {
      cpx<T> acc[E];
      for (int v = 0; v < n; ++v) {
        const cpx<T>* src = a.in[0] + ((b * q + v * P + g) * (int64_t)m + s) * R + colc;
        cpx<T> y[E];
#pragma unroll
        for (int e = 0; e < E; ++e) y[e] = src[(int64_t)G * e * m * R];
        lean_fft<T, P, E, -1, S, false>(y, g, xc, twl);
#pragma unroll
        for (int e = 0; e < E; ++e) {
          const cpx<T> z = cmulc(y[e], zq[v * (g + G * e)]);
          acc[e] = v == 0 ? z : acc[e] + z;
        }
      }
      if (valid) {
        cpx<T>* dst = a.out[0] + b * a.out_bstride + col;
#pragma unroll
        for (int e = 0; e < E; ++e) {
          const int64_t i = (int64_t)(g + G * e) * m + s;
          if (i < a.L) {
            cpx<T> v = cscale(acc[e], a.scale);
            if (a.add) v = v + dst[i * R];
            dst[i * R] = v;
          }
        }
      }
    }
  }
}

#if !defined(HD_PART) || HD_PART == 1  // host helpers, in one object only
// Points per lane built for each precision: 8 and 16 in FP32, 4 and 8 in
// FP64 (the same register footprint).
static bool lean_e_ok(int E, int tbytes) { return tbytes == 4 ? (E == 8 || E == 16) : (E == 4 || E == 8); }

bool outer_lean_supported(int m, int E, int S, int q, int tbytes, bool inner) {
  if (q < 1 || (!inner && q > kLeanMaxQ) || !lean_e_ok(E, tbytes) || (S != 8 && S != 16 && !(S == 32 && !inner)))
    return false;
  if (m != 64 && m != 128 && m != 256 && m != 512 && m != 1024) return false;
  return S * (m / E) <= 1024 && (size_t)S * m * 16 <= 128 * 1024;  // threads; exchange area (FP64 words)
}

bool outer_cols_supported(int p, int E, int tbytes) {
  const bool p2 = p >= 4 && p <= 64 && (p & (p - 1)) == 0;
  const bool p3 = tbytes == 4 && p % 3 == 0 && p >= 12 && p <= 96 && ((p / 3) & (p / 3 - 1)) == 0;
  return (p2 || p3) && E == outer_col_e(p, tbytes);
}

bool rows_lean_supported(int m, int E, int A, int q, int tbytes) {
  if ((A != 2 && A != 3) || q < 1 || q > kLeanMaxQ || !lean_e_ok(E, tbytes)) return false;
  return m >= 64 && m <= 2048 && (m & (m - 1)) == 0;
}
#endif

// Resident workgroups per CU of one kernel instance with one LDS size,
// asked once.
template <typename K>
static int lean_resident(K kernel, int threads, size_t lds) {
  static std::mutex mu;
  static std::map<std::pair<const void*, size_t>, int> seen;
  const void* fn = reinterpret_cast<const void*>(kernel);
  const auto key = std::make_pair(fn, lds);
  std::lock_guard<std::mutex> lk(mu);
  auto it = seen.find(key);
  if (it != seen.end()) return it->second;
  int n = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, fn, threads, lds) != hipSuccess || n < 1) n = 1;
  seen[key] = n;
  return n;
}

// Rows per workgroup: one wavefront, or one row of more lanes.
template <int N, int E>
constexpr int lean_rpb() {
  return 64 / (N / E) > 0 ? 64 / (N / E) : 1;
}
// Occupancy the register allocation aims at (waves per SIMD): 4, or 3 for
// 16 FP32 (8 FP64) points per lane and for rows of three inputs (which spill
// at 128 registers).
template <typename T, int E, int A = 2>
constexpr int lean_waves() {
  return (E * (int)sizeof(T) >= 64 || A >= 3) ? 3 : 4;
}

template <typename T, int N, int E, int A, bool FULL, int P, bool ZF>
static hipError_t go_lean_z(const LeanRowArgs<T>& a, int cus, hipStream_t s) {
  constexpr int RPB = lean_rpb<N, E>();
  constexpr int nt = RPB * (N / E);
  const size_t zf = ZF ? N : 0;
  const size_t lds =
      ((size_t)RPB * lean_xwords<N, E>() + a.fd.ntw_stage + (size_t)a.q * (N / E + E + 1) + zf) * sizeof(cpx<T>);
  auto k = k_rows_lean<T, N, E, A, RPB, lean_waves<T, E, A>(), FULL, P, ZF>;
  hipError_t e = allow_lds(k, lds);
  if (e != hipSuccess) return e;
  const int64_t need = (a.nrows + RPB - 1) / RPB;
  const int64_t cap = (int64_t)cus * lean_resident(k, nt, lds);
  const unsigned grid = (unsigned)std::max<int64_t>(1, std::min(need, cap));
  hipLaunchKernelGGL(k, dim3(grid), dim3(nt), lds, s, a);
  return hipGetLastError();
}

// The q = 2 twiddle table trades a complex product per point and use for an
// LDS read.  Measured row passes on gfx950 (256^3 and 128^3 plans, with
// against without): FP64 256 points at 8 per lane 0.83 against 1.05 ms,
// FP32 128 points at 16 per lane 0.048 against 0.051 ms; elsewhere it was
// neutral or slower (FP32 256 points at 16 per lane 0.49 against 0.38 ms,
// FP64 256 points at 4 per lane 1.40 against 1.04 ms), so only those two
// shapes take it.
template <typename T, int N, int E>
constexpr bool lean_use_zf() {
  return lean_zf<T, N>() && ((sizeof(T) == 8 && N == 256 && E == 8) || (sizeof(T) == 4 && N == 128 && E == 16));
}

template <typename T, int N, int E, int A, bool FULL, int P>
static hipError_t go_lean(const LeanRowArgs<T>& a, int cus, hipStream_t s) {
  if constexpr (A == 2 && lean_use_zf<T, N, E>())
    if (a.q == 2) return go_lean_z<T, N, E, A, FULL, P, true>(a, cus, s);
  return go_lean_z<T, N, E, A, FULL, P, false>(a, cus, s);
}

template <typename T, int N, int E, int S, bool FWD, bool FULL, int P>
static hipError_t go_outer_lean(const OuterLeanArgs<T>& a, int cus, hipStream_t s) {
  constexpr int nt = S * (N / E);
  const size_t lds = ((size_t)N * S + a.fd.ntw_stage + (size_t)a.q * (N / E + E + 1)) * sizeof(cpx<T>);
  auto k = k_outer_lean<T, N, E, S, FWD, lean_waves<T, E>(), FULL, P>;
  hipError_t e = allow_lds(k, lds);
  if (e != hipSuccess) return e;
  const int64_t units = ((a.R + S - 1) / S) * a.nb * (FWD ? a.na : 1);
  const int64_t cap = (int64_t)cus * lean_resident(k, nt, lds);
  const unsigned grid = (unsigned)std::max<int64_t>(1, std::min(units, cap));
  hipLaunchKernelGGL(k, dim3(grid), dim3(nt), lds, s, a);
  return hipGetLastError();
}

template <typename T, int N, int E, int S, bool FWD>
static hipError_t go_outer_inner_rows(const OuterLeanArgs<T>& a, int cus, hipStream_t s) {
  constexpr int nt = S * (N / E);
  const size_t lds = ((size_t)N * S + a.fd.ntw_stage) * sizeof(cpx<T>);
  auto k = k_outer_inner_rows<T, N, E, S, FWD, lean_waves<T, E>()>;
  hipError_t e = allow_lds(k, lds);
  if (e != hipSuccess) return e;
  const int64_t units = ((a.R + S - 1) / S) * a.nb * (FWD ? a.na : 1);
  const int64_t cap = (int64_t)cus * lean_resident(k, nt, lds);
  const unsigned grid = (unsigned)std::max<int64_t>(1, std::min(units, cap));
  hipLaunchKernelGGL(k, dim3(grid), dim3(nt), lds, s, a);
  return hipGetLastError();
}

// Points per lane of the column transforms, at compile time.
template <typename T, int P>
constexpr int ocol_e() {
  return P % 3 == 0 ? 12 : (P <= 4 ? P : (sizeof(T) == 4 ? 8 : 4));
}

template <typename T, int P, bool FWD>
static hipError_t go_outer_cols(const OuterColArgs<T>& a, int cus, hipStream_t s) {
  constexpr int E = ocol_e<T, P>();
  constexpr int S = 256 / (P / E);
  constexpr int nt = S * (P / E);
  const int q = a.n * P;
  const size_t lds = ((size_t)P * S + a.fd.ntw_stage + q) * sizeof(cpx<T>);
  auto k = k_outer_cols<T, P, E, S, FWD, 3>;
  hipError_t e = allow_lds(k, lds);
  if (e != hipSuccess) return e;
  const int64_t units = ((a.R + S - 1) / S) * a.m * a.nb * (FWD ? a.na : 1);
  const int64_t cap = (int64_t)cus * lean_resident(k, nt, lds);
  const unsigned grid = (unsigned)std::max<int64_t>(1, std::min(units, cap));
  hipLaunchKernelGGL(k, dim3(grid), dim3(nt), lds, s, a);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_outer_cols(const OuterColArgs<T>& a, int p, bool fwd, int cus, hipStream_t s) {
  if (!outer_cols_supported(p, a.fd.G ? p / a.fd.G : 0, (int)sizeof(T)) || a.fd.N != p || a.m < 1 || a.n < 1 ||
      a.R < 1 || a.nb < 1 || a.L < 1 || a.L > (int64_t)p * a.m || (fwd && (a.na < 1 || a.na > kMaxA)))
    return HD_BAD;
#define OC(PP)                                                                                   \
  if (p == PP) {                                                                                 \
    if constexpr (PP % 3 != 0 || sizeof(T) == 4)                                                 \
      return fwd ? go_outer_cols<T, PP, true>(a, cus, s) : go_outer_cols<T, PP, false>(a, cus, s); \
  }
  OC(4) OC(8) OC(16) OC(32) OC(64) OC(12) OC(24) OC(48) OC(96)
#undef OC
  return HD_BAD;
}

// The same at compile time.
template <typename T>
constexpr bool lean_e_built(int E) {
  return sizeof(T) == 4 ? (E == 8 || E == 16) : (E == 4 || E == 8);
}

// One block (L <= m) or two (m < L <= 2m; the second block is then partial).
template <typename T>
hipError_t launch_outer_lean(const OuterLeanArgs<T>& a, int E, int S, bool fwd, int cus, hipStream_t s) {
  const int N = a.fd.N;
  if (a.inner_n) {
    // the inner form's m-point pass: full planes of N rows, one residue each
    if (!outer_lean_supported(N, E, S, a.q, (int)sizeof(T), true) || a.fd.G * E != N || a.L != (uint32_t)N ||
        a.R < 1 || a.nb < 1 || (fwd && (a.na < 1 || a.na > kMaxA)) || a.q % a.inner_n != 0)
      return HD_BAD;
#define IQ(NN, EE, SS)                                                                                 \
  if (N == NN && E == EE && S == SS) {                                                                 \
    if constexpr (lean_e_built<T>(EE) && SS * (NN / EE) <= 1024 && SS * NN * 16 <= 128 * 1024)        \
      return fwd ? go_outer_inner_rows<T, NN, EE, SS, true>(a, cus, s)                                 \
                 : go_outer_inner_rows<T, NN, EE, SS, false>(a, cus, s);                               \
  }
#define IN(NN) IQ(NN, 4, 8) IQ(NN, 4, 16) IQ(NN, 8, 8) IQ(NN, 8, 16) IQ(NN, 16, 8) IQ(NN, 16, 16)
    IN(64) IN(128) IN(256) IN(512) IN(1024)
#undef IN
#undef IQ
    return HD_BAD;
  }
  if (!outer_lean_supported(N, E, S, a.q, (int)sizeof(T)) || a.fd.G * E != N || a.L > 2u * (uint32_t)N ||
      a.L < 1 || a.R < 1 || a.nb < 1 || (fwd && (a.na < 1 || a.na > kMaxA)) || a.D < 1 || a.r0 < 0 ||
      a.r0 + a.D > a.q)
    return HD_BAD;
  const int P = a.L > (uint32_t)N ? 2 : 1;
  if (P == 2 && a.q < 2) return HD_BAD;  // two blocks need q >= p
  const bool full = a.L == (uint32_t)N;
#define OQ(NN, EE, SS)                                                                                 \
  if (N == NN && E == EE && S == SS) {                                                                 \
    if constexpr (lean_e_built<T>(EE) && SS * (NN / EE) <= 1024 && SS * NN * 16 <= 128 * 1024) {      \
      if (P == 2)                                                                                      \
        return fwd ? go_outer_lean<T, NN, EE, SS, true, false, 2>(a, cus, s)                           \
                   : go_outer_lean<T, NN, EE, SS, false, false, 2>(a, cus, s);                         \
      if (fwd) return full ? go_outer_lean<T, NN, EE, SS, true, true, 1>(a, cus, s)                    \
                           : go_outer_lean<T, NN, EE, SS, true, false, 1>(a, cus, s);                  \
      return full ? go_outer_lean<T, NN, EE, SS, false, true, 1>(a, cus, s)                            \
                  : go_outer_lean<T, NN, EE, SS, false, false, 1>(a, cus, s);                          \
    }                                                                                                  \
  }
#define ON(NN) OQ(NN, 4, 8) OQ(NN, 4, 16) OQ(NN, 8, 8) OQ(NN, 8, 16) OQ(NN, 16, 8) OQ(NN, 16, 16) \
  OQ(NN, 8, 32) OQ(NN, 16, 32)
  ON(64) ON(128) ON(256) ON(512) ON(1024)
#undef ON
#undef OQ
  return HD_BAD;
}

template <typename T>
hipError_t launch_rows_lean(const LeanRowArgs<T>& a, int E, int A, int cus, hipStream_t s) {
  const int N = a.fd.N;
  if (!rows_lean_supported(N, E, A, a.q, (int)sizeof(T)) || a.fd.G * E != N || a.L > 2u * (uint32_t)N)
    return HD_BAD;
  const int P = a.L > (uint32_t)N ? 2 : 1;
  if (P == 2 && a.q < 2) return HD_BAD;
  const bool full = a.L == (uint32_t)N;
#define LQ(NN, EE, AA)                                                                                 \
  if (N == NN && E == EE && A == AA) {                                                                 \
    if constexpr (lean_e_built<T>(EE)) {                                                               \
      if (P == 2) return go_lean<T, NN, EE, AA, false, 2>(a, cus, s);                                  \
      return full ? go_lean<T, NN, EE, AA, true, 1>(a, cus, s) : go_lean<T, NN, EE, AA, false, 1>(a, cus, s); \
    }                                                                                                  \
  }
#define LN(NN) LQ(NN, 4, 2) LQ(NN, 8, 2) LQ(NN, 16, 2) LQ(NN, 4, 3) LQ(NN, 8, 3) LQ(NN, 16, 3)
  LN(64) LN(128) LN(256) LN(512) LN(1024) LN(2048)
#undef LN
#undef LQ
  return HD_BAD;
}

#define HD_INST(T)                                                                                 \
  template hipError_t launch_rows_lean<T>(const LeanRowArgs<T>&, int, int, int, hipStream_t);    \
  template hipError_t launch_outer_lean<T>(const OuterLeanArgs<T>&, int, int, bool, int, hipStream_t); \
  template hipError_t launch_outer_cols<T>(const OuterColArgs<T>&, int, bool, int, hipStream_t);
#if !defined(HD_PART) || HD_PART == 1
HD_INST(float)
#endif
#if !defined(HD_PART) || HD_PART == 2
HD_INST(double)
#endif
#undef HD_INST

}  // namespace hd
