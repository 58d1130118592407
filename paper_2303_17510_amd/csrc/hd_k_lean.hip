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
#include "hd_kcommon.hpp"

namespace hd {

// log2 of the first stage's radix: the exchange pads one slot every 2^PS
// points, so the first stage's writes (R apart) spread over the banks.
template <int N, int E>
__host__ __device__ constexpr int lean_ps() {
  int ps = 0;
  while ((1 << ps) < ct_radix(N, E)) ++ps;
  return ps;
}
template <int N, int E>
__host__ __device__ constexpr int lean_xwords() {
  return N + (N >> lean_ps<N, E>());
}
__host__ __device__ constexpr int pad_pos(int pos, int ps) { return pos + (pos >> ps); }

// Stages Ns.. of an N-point Stockham transform held as E points per lane
// (lane g, register e: point g + G e), twiddle offset TO into the per-stage
// table twl (w_{Ns R}^{k i} at TO + k (R-1) + i - 1).  Output c of butterfly
// j (k = j mod Ns) goes to position (j - k) R + k + c Ns; the last stage
// leaves the natural-order result in the strided layout.  Exchange position
// i lives at xr[pad(i) XS]: XS = 1 with PAD (one slot every 2^PS points) for
// a transform of its own, XS = S without padding for S interleaved column
// transforms (consecutive lanes then touch consecutive words).
template <typename T, int N, int E, int S, int XS = 1, bool PAD = true, int Ns = 1, int TO = 0>
__device__ __forceinline__ void lean_fft(cpx<T> (&v)[E], const int g, cpx<T>* __restrict__ xr,
                                         const cpx<T>* __restrict__ twl) {
  if constexpr (Ns < N) {
    constexpr int R = ct_radix(N / Ns, E);
    static_assert(R > 1 && (N / Ns) % R == 0 && E % R == 0, "no stage plan");
    constexpr int G = N / E, NB = E / R, PS = PAD ? lean_ps<N, E>() : 30;
    constexpr bool last = Ns * R == N;
    // with G a multiple of Ns every butterfly of a lane has k = g mod Ns
    constexpr bool kconst = G % Ns == 0;
    // write positions split as P(g) + C(b, c); with C a multiple of 2^PS
    // (or no padding) the padded position is pad(P) + pad(C)
    constexpr bool wlin = kconst && (!PAD || ((Ns == 1 || Ns % (1 << PS) == 0) && (G * R) % (1 << PS) == 0));
#pragma unroll
    for (int b = 0; b < NB; ++b) {
      const int j = g + G * b;
      const int k = kconst ? (g & (Ns - 1)) : (j & (Ns - 1));
      cpx<T> x[R];
#pragma unroll
      for (int i = 0; i < R; ++i) x[i] = v[b + i * NB];
      if constexpr (Ns > 1) {
        const cpx<T>* t = twl + (TO - 1) + k * (R - 1);
#pragma unroll
        for (int i = 1; i < R; ++i) x[i] = cmul_s<S>(x[i], t[i]);
      }
      dftr<R, S>(x);
      if constexpr (last) {
#pragma unroll
        for (int c = 0; c < R; ++c) v[b + c * NB] = x[c];
      } else if constexpr (wlin) {
        // padded, Ns = 1: position j R + c lands at j (R + 1) + c
        const int P = (PAD && Ns == 1) ? g * (R + 1) : pad_pos((g - k) * R + k, PS);
#pragma unroll
        for (int c = 0; c < R; ++c) {
          const int C = (PAD && Ns == 1) ? G * b * (R + 1) + c : pad_pos(G * b * R + c * Ns, PS);
          xr[(P + C) * XS] = x[c];
        }
      } else {
#pragma unroll
        for (int c = 0; c < R; ++c) xr[pad_pos((j - k) * R + k + c * Ns, PS) * XS] = x[c];
      }
    }
    if constexpr (!last) {
      __syncthreads();
      if constexpr (!PAD || G % (1 << PS) == 0) {
        const int P = pad_pos(g, PS);
#pragma unroll
        for (int e = 0; e < E; ++e) v[e] = xr[(P + pad_pos(G * e, PS)) * XS];
      } else {
#pragma unroll
        for (int e = 0; e < E; ++e) v[e] = xr[pad_pos(g + G * e, PS) * XS];
      }
      __syncthreads();
      lean_fft<T, N, E, S, XS, PAD, Ns * R, TO + (Ns > 1 ? Ns * (R - 1) : 0)>(v, g, xr, twl);
    }
  }
}

template <typename T, int N, int E, int A, int RPB, int WAVES, bool FULL, int P>
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
  {
    const cpx<T>* st = a.fft_tw + a.fd.ntw;  // the per-stage tables follow the two-level one
    for (int i = threadIdx.x; i < a.fd.ntw_stage; i += NT) twl[i] = st[i];
    // exponents r g < q G, r G e < q G E = q m and r m < q m: no reduction
    for (int i = threadIdx.x; i < q * G; i += NT) zA[i] = a.zqm.get((uint32_t)((i / G) * (i % G)));
    for (int i = threadIdx.x; i < q * E; i += NT) zB[i] = a.zqm.get((uint32_t)((i / E) * G * (i % E)));
    if constexpr (P == 2)
      for (int i = threadIdx.x; i < q; i += NT) zC[i] = a.zqm.get((uint32_t)(i * N));
  }
  __syncthreads();

  // Inputs of A P E <= 8 words per lane stay in registers across the
  // residues; larger ones are read again (from cache) for each residue.
  // With 16 points per lane the residue twiddles are formed again at each
  // use rather than held across the transforms.
  constexpr bool kKeep = A * P * E <= 8;
  constexpr bool kHoldZ = E <= 8;
  // Loads never branch: a row beyond the last reads the last row (and
  // stores nothing); a point beyond L reads point L-1 and is replaced by 0.
  // Full rows (FULL: one block and L = m, the usual case) read at constant
  // offsets from one per-lane address.
  constexpr bool full = FULL;
  const int64_t step = (int64_t)gridDim.x * RPB;
  for (int64_t row0 = (int64_t)blockIdx.x * RPB; row0 < a.nrows; row0 += step) {
    const int64_t row = row0 + slot;
    const bool valid = row < a.nrows;
    const int64_t rowc = valid ? row : a.nrows - 1;
    const cpx<T>* src[A];
#pragma unroll
    for (int ai = 0; ai < A; ++ai) src[ai] = a.in[ai] + rowc * a.in_stride + g;
    // point t m + g + G e of input ai
    auto load = [&](int ai, int t, int e) -> cpx<T> {
      if constexpr (full) return src[ai][G * e];
      const uint32_t i = (uint32_t)(t * N + g + G * e);
      const cpx<T> v = src[ai][(int)(i < a.L ? i : a.L - 1) - g];
      return i < a.L ? v : czero<T>();
    };
    cpx<T> x[kKeep ? A : 1][kKeep ? P : 1][kKeep ? E : 1];
    if constexpr (kKeep) {
#pragma unroll
      for (int ai = 0; ai < A; ++ai)
#pragma unroll
        for (int t = 0; t < P; ++t)
#pragma unroll
          for (int e = 0; e < E; ++e) x[ai][t][e] = load(ai, t, e);
    }
    cpx<T> acc[P][E];
    constexpr bool kTwo = A == 2;  // the two-residue path below (products of two inputs)
    if (kTwo && q == 2) {
      // Two residues (the usual M = 2L): each input is read once and
      // transformed for both residues, the two partial products are held
      // (residue 0 has unit twiddles).
      const cpx<T> za = zA[G + g];
      const cpx<T> zc = P == 2 ? zC[1] : mk(T(1), T(0));
      cpx<T> p0[E], p1[E];
#pragma unroll
      for (int ai = 0; ai < A; ++ai) {
        cpx<T> xa[P][E];
#pragma unroll
        for (int t = 0; t < P; ++t)
#pragma unroll
          for (int e = 0; e < E; ++e) {
            if constexpr (kKeep) xa[t][e] = x[ai][t][e];
            else xa[t][e] = load(ai, t, e);
          }
        cpx<T> w[E];
#pragma unroll
        for (int e = 0; e < E; ++e) w[e] = P == 2 ? xa[0][e] + xa[P - 1][e] : xa[0][e];
        lean_fft<T, N, E, +1>(w, g, xr, twl);
#pragma unroll
        for (int e = 0; e < E; ++e) p0[e] = ai == 0 ? w[e] : cmul(p0[e], w[e]);
#pragma unroll
        for (int e = 0; e < E; ++e) {
          const cpx<T> xv = P == 2 ? xa[0][e] + cmul(xa[P - 1][e], zc) : xa[0][e];
          w[e] = cmul(xv, cmul(za, zB[E + e]));
        }
        lean_fft<T, N, E, +1>(w, g, xr, twl);
#pragma unroll
        for (int e = 0; e < E; ++e) p1[e] = ai == 0 ? w[e] : cmul(p1[e], w[e]);
      }
      lean_fft<T, N, E, -1>(p0, g, xr, twl);
#pragma unroll
      for (int e = 0; e < E; ++e) acc[0][e] = acc[P - 1][e] = p0[e];
      lean_fft<T, N, E, -1>(p1, g, xr, twl);
#pragma unroll
      for (int e = 0; e < E; ++e) {
        const cpx<T> y = cmulc(p1[e], cmul(za, zB[E + e]));
        acc[0][e] = acc[0][e] + y;
        if constexpr (P == 2) acc[P - 1][e] = acc[P - 1][e] + cmulc(y, zc);
      }
    }
    for (int r = 0; r < q && !(kTwo && q == 2); ++r) {
      // this lane's residue twiddles zeta_{qm}^{r (g + G e)} (r = 0: ones)
      const cpx<T>* zb = zB + r * E;
      const int zai = r * G + g;
      cpx<T> zh[kHoldZ ? E : 1];
      if constexpr (kHoldZ) {
        const cpx<T> za = zA[zai];
#pragma unroll
        for (int e = 0; e < E; ++e) zh[e] = cmul(za, zb[e]);
      }
      auto zat = [&](int e) -> cpx<T> {
        if constexpr (kHoldZ) return zh[e];
        else return cmul(zA[zai], zb[e]);
      };
      // the second block's points carry zeta_{qm}^{r (m + s)} = zeta_q^r zeta_{qm}^{r s}
      const cpx<T> zc = P == 2 ? zC[r] : mk(T(1), T(0));
      cpx<T> pr[E];
#pragma unroll
      for (int ai = 0; ai < A; ++ai) {
        cpx<T> w[E];
#pragma unroll
        for (int e = 0; e < E; ++e) {
          cpx<T> xv;
          if constexpr (kKeep) xv = x[ai][0][e];
          else xv = load(ai, 0, e);
          if constexpr (P == 2) {
            cpx<T> x1;
            if constexpr (kKeep) x1 = x[ai][P - 1][e];
            else x1 = load(ai, P - 1, e);
            xv = xv + cmul(x1, zc);
          }
          w[e] = cmul(xv, zat(e));
        }
        lean_fft<T, N, E, +1>(w, g, xr, twl);
#pragma unroll
        for (int e = 0; e < E; ++e) pr[e] = ai == 0 ? w[e] : cmul(pr[e], w[e]);
      }
      lean_fft<T, N, E, -1>(pr, g, xr, twl);
#pragma unroll
      for (int e = 0; e < E; ++e) {
        const cpx<T> y = cmulc(pr[e], zat(e));
        acc[0][e] = r == 0 ? y : acc[0][e] + y;
        if constexpr (P == 2) {
          const cpx<T> y1 = cmulc(y, zc);
          acc[P - 1][e] = r == 0 ? y1 : acc[P - 1][e] + y1;
        }
      }
    }
    if (valid) {
      cpx<T>* dst = a.out + row * a.out_stride + g;
#pragma unroll
      for (int t = 0; t < P; ++t)
#pragma unroll
        for (int e = 0; e < E; ++e)
          if (full || (uint32_t)(t * N + g + G * e) < a.L) dst[t * N + G * e] = cscale(acc[t][e], a.scale);
    }
  }
}

// Outer dimension of a 2D/3D convolution (Sec. 5), direct form with one or
// two blocks (p <= 2), dense planes [nb][L][R]: what k_outer_fwd /
// k_outer_bwd compute for an ordinary (not centered) dimension, laid out like
// the lean row kernel.  A workgroup takes S adjacent columns (lanes of one
// column are S apart, so every global access of a wave covers S consecutive
// words per row) and loops over (input, plane, column tile) units.
//   forward:  out[a][((b q + r) m + k) R + col] = fft_m(W)_k,
//             W_s = zeta_{qm}^{r s} (x_s + zeta_q^r x_{m+s})
//   backward: out[b][t m + s][col] = zeta_q^{-r t} sum_r zeta_{qm}^{-r s} ifft_m(y_r)_s / (q m)
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
      for (int r = 0; r < q; ++r) {
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
          cpx<T>* dst = a.out[ai] + ((b * q + r) * N + g) * R + col;
#pragma unroll
          for (int e = 0; e < E; ++e) dst[e * GR] = w[e];
        }
      }
    } else {
      cpx<T> acc[P][E];
      for (int r = 0; r < q; ++r) {
        const cpx<T>* src = a.in[0] + ((b * q + r) * N + g) * R + colc;
        cpx<T> y[E];
#pragma unroll
        for (int e = 0; e < E; ++e) y[e] = src[e * GR];
        lean_fft<T, N, E, -1, S, false>(y, g, xr, twl);
        const cpx<T> za = zA[r * G + g];
        const cpx<T> zc = P == 2 ? zC[r] : mk(T(1), T(0));
#pragma unroll
        for (int e = 0; e < E; ++e) {
          const cpx<T> v = cmulc(y[e], cmul(za, zB[r * E + e]));
          acc[0][e] = r == 0 ? v : acc[0][e] + v;
          if constexpr (P == 2) {
            const cpx<T> v1 = cmulc(v, zc);
            acc[P - 1][e] = r == 0 ? v1 : acc[P - 1][e] + v1;
          }
        }
      }
      if (valid) {
        cpx<T>* dst = a.out[0] + b * a.out_bstride + col + (int64_t)g * R;
#pragma unroll
        for (int t = 0; t < P; ++t)
#pragma unroll
          for (int e = 0; e < E; ++e)
            if (full || (uint32_t)(t * N + g + G * e) < a.L) dst[t * NR + e * GR] = cscale(acc[t][e], a.scale);
      }
    }
  }
}

#if !defined(HD_PART) || HD_PART == 1  // host helpers, in one object only
// Points per lane built for each precision: 8 and 16 in FP32, 4 and 8 in
// FP64 (the same register footprint).
static bool lean_e_ok(int E, int tbytes) { return tbytes == 4 ? (E == 8 || E == 16) : (E == 4 || E == 8); }

bool outer_lean_supported(int m, int E, int S, int q, int tbytes) {
  if (q < 1 || q > kLeanMaxQ || !lean_e_ok(E, tbytes) || (S != 8 && S != 16)) return false;
  if (m != 64 && m != 128 && m != 256 && m != 512 && m != 1024) return false;
  return S * (m / E) <= 1024 && (size_t)S * m * 16 <= 128 * 1024;  // threads; exchange area (FP64 words)
}

bool rows_lean_supported(int m, int E, int A, int q, int tbytes) {
  if ((A != 2 && A != 3) || q < 1 || q > kLeanMaxQ || !lean_e_ok(E, tbytes)) return false;
  return m >= 64 && m <= 2048 && (m & (m - 1)) == 0;
}
#endif

// Resident workgroups per CU of one kernel instance, asked once.
template <typename K>
static int lean_resident(K kernel, int threads, size_t lds) {
  static std::mutex mu;
  static std::unordered_map<const void*, int> seen;
  const void* key = reinterpret_cast<const void*>(kernel);
  std::lock_guard<std::mutex> lk(mu);
  auto it = seen.find(key);
  if (it != seen.end()) return it->second;
  int n = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, key, threads, lds) != hipSuccess || n < 1) n = 1;
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

template <typename T, int N, int E, int A, bool FULL, int P>
static hipError_t go_lean(const LeanRowArgs<T>& a, int cus, hipStream_t s) {
  constexpr int RPB = lean_rpb<N, E>();
  constexpr int nt = RPB * (N / E);
  const size_t lds =
      ((size_t)RPB * lean_xwords<N, E>() + a.fd.ntw_stage + (size_t)a.q * (N / E + E + 1)) * sizeof(cpx<T>);
  auto k = k_rows_lean<T, N, E, A, RPB, lean_waves<T, E, A>(), FULL, P>;
  hipError_t e = allow_lds(k, lds);
  if (e != hipSuccess) return e;
  const int64_t need = (a.nrows + RPB - 1) / RPB;
  const int64_t cap = (int64_t)cus * lean_resident(k, nt, lds);
  const unsigned grid = (unsigned)std::max<int64_t>(1, std::min(need, cap));
  hipLaunchKernelGGL(k, dim3(grid), dim3(nt), lds, s, a);
  return hipGetLastError();
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

// The same at compile time.
template <typename T>
constexpr bool lean_e_built(int E) {
  return sizeof(T) == 4 ? (E == 8 || E == 16) : (E == 4 || E == 8);
}

// One block (L <= m) or two (m < L <= 2m; the second block is then partial).
template <typename T>
hipError_t launch_outer_lean(const OuterLeanArgs<T>& a, int E, int S, bool fwd, int cus, hipStream_t s) {
  const int N = a.fd.N;
  if (!outer_lean_supported(N, E, S, a.q, (int)sizeof(T)) || a.fd.G * E != N || a.L > 2u * (uint32_t)N ||
      a.L < 1 || a.R < 1 || a.nb < 1 || (fwd && (a.na < 1 || a.na > kMaxA)))
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
#define ON(NN) OQ(NN, 4, 8) OQ(NN, 4, 16) OQ(NN, 8, 8) OQ(NN, 8, 16) OQ(NN, 16, 8) OQ(NN, 16, 16)
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

#define HD_INST(T)                                                                              \
  template hipError_t launch_rows_lean<T>(const LeanRowArgs<T>&, int, int, int, hipStream_t); \
  template hipError_t launch_outer_lean<T>(const OuterLeanArgs<T>&, int, int, bool, int, hipStream_t);
#if !defined(HD_PART) || HD_PART == 1
HD_INST(float)
#endif
#if !defined(HD_PART) || HD_PART == 2
HD_INST(double)
#endif
#undef HD_INST

}  // namespace hd
