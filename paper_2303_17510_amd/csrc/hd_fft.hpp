// hd_fft.hpp -- FFT building blocks for gfx950 (wave64, LDS exchange).
//
// An N-point transform is done by a group of G threads, each holding E = N/G
// points in registers in the "strided" layout: lane g, register e holds point
// g + G*e.  A Stockham autosort pass of radix R (R divides E) has each lane
// run E/R radix-R butterflies on points it already holds; the outputs are
// exchanged through LDS so that the next pass again finds its inputs in the
// strided layout.  The last pass needs no exchange: its outputs land in the
// strided layout of the natural-order result.  So an S-stage transform costs
// S-1 LDS round trips, and input/output stay coalesced (consecutive lanes
// touch consecutive points).
//
// Sign convention: S = +1 computes X_k = sum_j x_j exp(+2 pi i jk/N), the
// paper's forward transform (zeta_N = exp(2 pi i/N), Sec. 2); S = -1 the
// unnormalised inverse.
#pragma once
#include "hd_common.hpp"

namespace hd {

// cos(2 pi k / 64) for k = 0..16 (quarter wave), rounded from exact values.
__device__ __host__ constexpr double qcos64(int k) {
  constexpr double t[17] = {
      1.00000000000000000000e+00, 9.95184726672196886245e-01, 9.80785280403230449126e-01,
      9.56940335732208864936e-01, 9.23879532511286756128e-01, 8.81921264348355029713e-01,
      8.31469612302545237079e-01, 7.73010453362736960810e-01, 7.07106781186547524401e-01,
      6.34393284163645498215e-01, 5.55570233019602224743e-01, 4.71396736825997648556e-01,
      3.82683432365089771728e-01, 2.90284677254462367636e-01, 1.95090322016128267848e-01,
      9.80171403295606019942e-02, 0.0};
  return t[k];
}

// exp(S 2 pi i e / 64) for 0 <= e < 32, as (cos, sin) rounded to T
template <typename T, int S>
__device__ __forceinline__ cpx<T> w64(int e) {
  double c = e <= 16 ? qcos64(e) : -qcos64(32 - e);
  double s = e <= 16 ? qcos64(16 - e) : qcos64(e - 16);
  return mk(T(c), T(S * s));
}

// o * exp(S 2 pi i e / 64) for a compile-time-foldable e in [0, 32)
template <int S, typename T>
__device__ __forceinline__ cpx<T> rot64(cpx<T> o, int e) {
  if (e == 0) return o;
  if (e == 16) return mul_si<S>(o);
  if (e == 8) {
    const T h = T(7.07106781186547524401e-01);
    return mk(h * (o.x - S * o.y), h * (o.y + S * o.x));
  }
  if (e == 24) {
    const T h = T(7.07106781186547524401e-01);
    return mk(-h * (o.x + S * o.y), h * (S * o.x - o.y));
  }
  return cmul(o, w64<T, S>(e));
}

// In-place radix-R DFT in registers, natural order in and out:
//   Y_c = sum_i x_i exp(S 2 pi i i c / R).
template <int R, int S, typename T>
__device__ __forceinline__ void dftr(cpx<T>* x) {
  if constexpr (R == 1) {
    return;
  } else if constexpr (R == 2) {
    cpx<T> a = x[0] + x[1], b = x[0] - x[1];
    x[0] = a;
    x[1] = b;
  } else if constexpr (R == 3) {
    // exp(S 2 pi i/3) = -1/2 + S i sqrt(3)/2
    const T h = T(8.66025403784438646764e-01);
    cpx<T> t = x[1] + x[2];
    cpx<T> d = x[1] - x[2];
    cpx<T> m0 = mk(x[0].x - T(0.5) * t.x, x[0].y - T(0.5) * t.y);
    cpx<T> sd = mk(-S * h * d.y, S * h * d.x);  // d * (S i sqrt(3)/2)
    x[0] = x[0] + t;
    x[1] = m0 + sd;
    x[2] = m0 - sd;
  } else if constexpr (R == 4) {
    cpx<T> a = x[0] + x[2], b = x[0] - x[2];
    cpx<T> c = x[1] + x[3], d = mul_si<S>(x[1] - x[3]);
    x[0] = a + c;
    x[2] = a - c;
    x[1] = b + d;
    x[3] = b - d;
  } else {
    static_assert(R == 8 || R == 16 || R == 32, "unsupported radix");
    // decimation in time: even and odd halves, then R/2 butterflies
    cpx<T> ev[R / 2], od[R / 2];
#pragma unroll
    for (int i = 0; i < R / 2; ++i) {
      ev[i] = x[2 * i];
      od[i] = x[2 * i + 1];
    }
    dftr<R / 2, S>(ev);
    dftr<R / 2, S>(od);
#pragma unroll
    for (int k = 0; k < R / 2; ++k) {
      cpx<T> t = rot64<S>(od[k], k * (64 / R));
      x[k] = ev[k] + t;
      x[k + R / 2] = ev[k] - t;
    }
  }
}

// Stage plan of one transform size, passed to kernels by value.
struct FftDesc {
  int N;          // points
  int G;          // lanes per transform; N = G * E
  int nst;        // stages
  int radix[12];  // radix of each stage (each divides E)
  int kb;         // twiddle table split: K = 2^kb
  int ntw;        // entries of the two-level table: K + ceil(N / K)
  int twmode;     // 1: per-stage tables staged in LDS; 0: two-level table in LDS
  int twoff[12];  // per-stage table: offset of each stage (entries k (R-1) + i - 1)
  int ntw_stage;  // entries of all per-stage tables
  int ps;         // row exchanges pad one slot every 2^ps points (first-stage writes
                  // land R apart, so ps = log2 R spreads them over the banks)
};

// LDS words (complex) a transform's twiddles occupy.
__host__ __device__ inline int tw_words(const FftDesc& d) { return d.twmode ? d.ntw_stage : d.ntw; }

// Twiddles of a transform, held in LDS.  Mode 0: powers of zeta_N from a
// two-level table, zeta_N^e = lo[e & (K-1)] * hi[e >> kb] (within about two
// ulps of the exact root).  Mode 1: for each stage the exact values
// w_{Ns R}^{k i} (k < Ns, 1 <= i < R), each rounded once from FP64.
template <typename T>
struct TwLds {
  const cpx<T>* lo;
  const cpx<T>* hi;
  int kb;
  int mode;
  __device__ __forceinline__ cpx<T> get(int e) const {
    const cpx<T> a = lo[e & ((1 << kb) - 1)];
    const int h = e >> kb;
    return h ? cmul(a, hi[h]) : a;
  }
};

// Copy a transform's twiddles (the global table holds the two-level table,
// ntw entries, followed by the per-stage tables) into LDS; all lanes of the
// workgroup take part.  The caller puts a barrier between this and the first
// use.
template <typename T>
__device__ __forceinline__ TwLds<T> stage_table(const FftDesc& d, const cpx<T>* __restrict__ g,
                                                cpx<T>* lds) {
  const int n = tw_words(d);
  const cpx<T>* src = d.twmode ? g + d.ntw : g;
  for (int i = threadIdx.x; i < n; i += blockDim.x) lds[i] = src[i];
  TwLds<T> t;
  t.lo = lds;
  t.hi = lds + (1 << d.kb);
  t.kb = d.kb;
  t.mode = d.twmode;
  return t;
}

// LDS exchange addressing: point i of transform n lives at
// base[n * ns + i * xs + (i >> ps)] -- xs > 1 interleaves the transforms of
// adjacent columns; ps < 31 pads one slot every 2^ps points to spread banks.
template <typename T>
struct Xchg {
  cpx<T>* base;
  int xs;
  int ps;
  int ns;
  __device__ __forceinline__ cpx<T>& at(int n, int i) const { return base[n * ns + i * xs + (i >> ps)]; }
};

// Twiddles w^i, i = 1 .. R-1, of one butterfly, with w = zeta_N^{e1}: the
// base-4 digits of i select products of w^{d 4^k} (d = 1..3), so a radix-R
// butterfly needs ceil(log4 R) table lookups and every twiddle is a product
// of at most ceil(log4 R) + 2 rounded factors.
template <typename T, int R>
__device__ __forceinline__ void butterfly_twiddles(const TwLds<T>& tw, int e1, cpx<T> (&w)[R]) {
  constexpr int ND = R <= 4 ? 1 : (R <= 16 ? 2 : 3);
  cpx<T> P[ND][4];
  int e = e1;
#pragma unroll
  for (int d = 0; d < ND; ++d) {
    P[d][0] = mk(T(1), T(0));
    P[d][1] = tw.get(e);
    P[d][2] = cmul(P[d][1], P[d][1]);
    P[d][3] = cmul(P[d][2], P[d][1]);
    e <<= 2;
  }
  w[0] = mk(T(1), T(0));
#pragma unroll
  for (int i = 1; i < R; ++i) {
    cpx<T> t = P[0][i & 3];
    if (ND > 1 && (i >> 2) > 0) t = (i & 3) ? cmul(t, P[ND > 1 ? 1 : 0][(i >> 2) & 3]) : P[ND > 1 ? 1 : 0][(i >> 2) & 3];
    if (ND > 2 && (i >> 4) > 0) t = cmul(t, P[ND > 2 ? 2 : 0][(i >> 4) & 3]);
    w[i] = t;
  }
}

// One Stockham pass of radix R over span Ns, applied to NT transforms that
// share twiddles and barriers.  Butterfly j = g + G*b reads points
// j + i*N/R (registers b + i*E/R), multiplies point i by w_{Ns R}^{S k i}
// (k = j mod Ns), runs the radix-R DFT and stores output c at
// (j - k) R + k + c Ns.  The last pass keeps its outputs in registers: they
// are already in the strided layout of the natural-order result.  tws =
// N / (Ns R): w_{Ns R} = zeta_N^{tws}.
template <typename T, int E, int R, int S, int NT>
__device__ __forceinline__ void fft_stage(cpx<T> (&v)[NT][E], int g, int G, int tws, int Ns, int twoff,
                                          const TwLds<T>& tw, const Xchg<T>& xb, bool last) {
  constexpr int NB = E / R;
  const bool pow2 = (Ns & (Ns - 1)) == 0;
#pragma unroll
  for (int b = 0; b < NB; ++b) {
    const int j = g + G * b;
    const int k = pow2 ? (j & (Ns - 1)) : j % Ns;
    cpx<T> w[R];
    if (Ns > 1) {
      if (tw.mode) {
        const cpx<T>* t = tw.lo + twoff + k * (R - 1) - 1;
#pragma unroll
        for (int i = 1; i < R; ++i) w[i] = t[i];
      } else {
        butterfly_twiddles<T, R>(tw, k * tws, w);
      }
    }
#pragma unroll
    for (int n = 0; n < NT; ++n) {
      cpx<T> x[R];
#pragma unroll
      for (int i = 0; i < R; ++i) x[i] = v[n][b + i * NB];
      if (Ns > 1) {
#pragma unroll
        for (int i = 1; i < R; ++i) x[i] = cmul_s<S>(x[i], w[i]);
      }
      dftr<R, S>(x);
      if (last) {
#pragma unroll
        for (int c = 0; c < R; ++c) v[n][b + c * NB] = x[c];
      } else {
        const int base = (j - k) * R + k;
#pragma unroll
        for (int c = 0; c < R; ++c) xb.at(n, base + c * Ns) = x[c];
      }
    }
  }
  if (!last) {
    __syncthreads();
#pragma unroll
    for (int n = 0; n < NT; ++n)
#pragma unroll
      for (int e = 0; e < E; ++e) v[n][e] = xb.at(n, g + G * e);
    __syncthreads();
  }
}

// Stage radix for `rem` points left, the same rule make_fft_desc applies on
// the host: factors 3 first, then the largest power of two up to 16 that
// divides both E and rem.
__host__ __device__ constexpr int ct_radix(int rem, int E) {
  if (rem % 3 == 0) return 3;
  int r = 1;
  while (r < 16 && E % (2 * r) == 0) r *= 2;
  while (r > 1 && rem % r != 0) r /= 2;
  return r;
}

// NT transforms of one size at once.  Every lane of the workgroup must call
// this with the same descriptor (the stage count decides the barriers).  The
// stage radices are recomputed from (N, E) by the planner's rule rather than
// read from d.radix[], and the per-stage table offsets accumulate as in
// make_fft_desc: indexing the descriptor's arrays with a run-time stage
// number would make the compiler copy the whole kernel argument block to
// scratch memory.
template <typename T, int E, int S, int NT>
__device__ __forceinline__ void gfft(cpx<T> (&v)[NT][E], int g, const FftDesc& d, const TwLds<T>& tw,
                                     const Xchg<T>& xb) {
  const int N = d.N, G = d.G;
  int Ns = 1, rem = N, to = 0;
  while (rem > 1) {
    const int R = ct_radix(rem, E);
    const bool last = (R == rem);
    switch (R) {
      case 2:
        if constexpr (E % 2 == 0) fft_stage<T, E, 2, S, NT>(v, g, G, rem / 2, Ns, to, tw, xb, last);
        break;
      case 3:
        if constexpr (E % 3 == 0) fft_stage<T, E, 3, S, NT>(v, g, G, rem / 3, Ns, to, tw, xb, last);
        break;
      case 4:
        if constexpr (E % 4 == 0) fft_stage<T, E, 4, S, NT>(v, g, G, rem / 4, Ns, to, tw, xb, last);
        break;
      case 8:
        if constexpr (E % 8 == 0) fft_stage<T, E, 8, S, NT>(v, g, G, rem / 8, Ns, to, tw, xb, last);
        break;
      case 16:
        if constexpr (E % 16 == 0) fft_stage<T, E, 16, S, NT>(v, g, G, rem / 16, Ns, to, tw, xb, last);
        break;
      default:
        return;  // no such plan (the host never builds one)
    }
    if (Ns > 1) to += Ns * (R - 1);
    Ns *= R;
    rem /= R;
  }
}

// The same transform with N and E known at compile time: the stage plan is
// unrolled and every span, mask and twiddle stride is a constant.
template <typename T, int N, int E, int S, int NT, int Ns = 1, int ST = 0>
__device__ __forceinline__ void gfft_ct(cpx<T> (&v)[NT][E], int g, const FftDesc& d, const TwLds<T>& tw,
                                        const Xchg<T>& xb) {
  if constexpr (Ns < N) {
    constexpr int R = ct_radix(N / Ns, E);
    static_assert(R > 1 && (N / Ns) % R == 0 && E % R == 0, "no stage plan");
    fft_stage<T, E, R, S, NT>(v, g, N / E, N / (Ns * R), Ns, d.twoff[ST], tw, xb, Ns * R == N);
    gfft_ct<T, N, E, S, NT, Ns * R, ST + 1>(v, g, d, tw, xb);
  }
}

// Sizes compiled with a fixed stage plan for each points-per-lane E.
template <int E, int N>
__host__ __device__ constexpr bool ct_size() {
  if (E == 8) return N == 128 || N == 256 || N == 512 || N == 1024 || N == 2048 || N == 4096;
  if (E == 16) return N == 256 || N == 512 || N == 1024 || N == 2048 || N == 4096 || N == 8192;
  return false;
}

// Sizes each kernel kind specialises (bit k: N = 2^k); the others take the
// general path.
constexpr unsigned kCtFused = 0;
constexpr unsigned kCtRows = (1u << 11) | (1u << 12) | (1u << 13);
constexpr unsigned kCtCols = (1u << 7) | (1u << 8) | (1u << 9) | (1u << 10);
constexpr unsigned kCtOuter = 0;

// Transform with the specialised plan when one exists for (N, E) and the
// kernel kind's MASK selects N, else the general one.  d.N is the same on
// every lane, so the branch is uniform.
template <typename T, int E, int S, int NT, unsigned MASK>
__device__ __forceinline__ void gfft_any(cpx<T> (&v)[NT][E], int g_in, const FftDesc& d, const TwLds<T>& tw,
                                         const Xchg<T>& xb) {
  // The butterfly twiddles depend only on the lane, so a caller that
  // transforms in a loop (residues) would have them hoisted out of the loop
  // and kept live across it, which costs more registers than recomputing
  // them; an opaque copy of the lane index keeps them inside.
  int g = g_in;
  asm volatile("" : "+v"(g));
#define HD_CT(NN)                                              \
  if constexpr (ct_size<E, NN>() && (MASK & (NN)) != 0) {      \
    if (d.N == NN) {                                           \
      gfft_ct<T, NN, E, S, NT>(v, g, d, tw, xb);               \
      return;                                                  \
    }                                                          \
  }
  HD_CT(128) HD_CT(256) HD_CT(512) HD_CT(1024) HD_CT(2048) HD_CT(4096) HD_CT(8192)
#undef HD_CT
  gfft<T, E, S, NT>(v, g, d, tw, xb);
}

}  // namespace hd
