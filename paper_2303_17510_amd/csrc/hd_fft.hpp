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
  int twoff[12];  // offset of the stage's twiddle table in the size's table
};

// LDS exchange addressing: point i of a transform lives at
// base[i * xs + (i >> ps)] -- xs > 1 interleaves the transforms of adjacent
// columns; ps < 31 pads one slot every 2^ps points to spread LDS banks.
template <typename T>
struct Xchg {
  cpx<T>* base;
  int xs;
  int ps;
  __device__ __forceinline__ cpx<T>& at(int i) const { return base[i * xs + (i >> ps)]; }
};

// One Stockham pass of radix R over span Ns.  Butterfly j = g + G*b reads
// points j + i*N/R (registers b + i*E/R), multiplies point i by
// w_{Ns R}^{S k i} (k = j mod Ns, table entries tw[k (R-1) + i - 1]), runs
// the radix-R DFT and stores output c at (j - k) R + k + c Ns.
template <typename T, int E, int R, int S>
__device__ __forceinline__ void fft_stage(cpx<T> (&v)[E], int g, int G, int Ns,
                                          const cpx<T>* __restrict__ tw, const Xchg<T>& xb,
                                          bool last) {
  constexpr int NB = E / R;
#pragma unroll
  for (int b = 0; b < NB; ++b) {
    const int j = g + G * b;
    const int k = j % Ns;
    cpx<T> x[R];
#pragma unroll
    for (int i = 0; i < R; ++i) x[i] = v[b + i * NB];
    if (Ns > 1) {
      const cpx<T>* w = tw + k * (R - 1) - 1;
#pragma unroll
      for (int i = 1; i < R; ++i) x[i] = cmul_s<S>(x[i], w[i]);
    }
    dftr<R, S>(x);
    if (last) {
#pragma unroll
      for (int c = 0; c < R; ++c) v[b + c * NB] = x[c];
    } else {
      const int base = (j - k) * R + k;
#pragma unroll
      for (int c = 0; c < R; ++c) xb.at(base + c * Ns) = x[c];
    }
  }
  if (!last) {
    __syncthreads();
#pragma unroll
    for (int e = 0; e < E; ++e) v[e] = xb.at(g + G * e);
    __syncthreads();
  }
}

// Whole transform.  Every lane of the workgroup must call this with the same
// descriptor (the stage count decides the number of barriers).
template <typename T, int E, int S>
__device__ __forceinline__ void gfft(cpx<T> (&v)[E], int g, const FftDesc& d,
                                     const cpx<T>* __restrict__ tw, const Xchg<T>& xb) {
  int Ns = 1;
  for (int st = 0; st < d.nst; ++st) {
    const int R = d.radix[st];
    const bool last = (st == d.nst - 1);
    const cpx<T>* t = tw + d.twoff[st];
    switch (R) {
      case 2:
        if constexpr (E % 2 == 0) fft_stage<T, E, 2, S>(v, g, d.G, Ns, t, xb, last);
        break;
      case 3:
        if constexpr (E % 3 == 0) fft_stage<T, E, 3, S>(v, g, d.G, Ns, t, xb, last);
        break;
      case 4:
        if constexpr (E % 4 == 0) fft_stage<T, E, 4, S>(v, g, d.G, Ns, t, xb, last);
        break;
      case 8:
        if constexpr (E % 8 == 0) fft_stage<T, E, 8, S>(v, g, d.G, Ns, t, xb, last);
        break;
      case 16:
        if constexpr (E % 16 == 0) fft_stage<T, E, 16, S>(v, g, d.G, Ns, t, xb, last);
        break;
      case 32:
        if constexpr (E % 32 == 0) fft_stage<T, E, 32, S>(v, g, d.G, Ns, t, xb, last);
        break;
      default:
        break;
    }
    Ns *= R;
  }
}

}  // namespace hd
