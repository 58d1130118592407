// hd_lean.hpp -- the compile-time-planned Stockham transform and the whole-row
// direct-form body shared by the lean kernels (hd_k_lean.hip) and the
// persistent batched kernel (hd_k_batch.hip).
#pragma once
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
// Pad period of the exchange after the stage of span Ns.  Stages of span
// 32 or more (transforms of at most 8 points per lane, 32 or more lanes)
// write butterfly outputs Ns points apart, where one slot every 32 points
// keeps every group of 16 or 32 lanes on distinct LDS banks (one every 2^PS
// leaves 2-way conflicts); the addresses stay one per-lane base plus
// constants, and a longer period needs no more room.
template <int N, int E, int Ns>
__host__ __device__ constexpr int lean_ps_at() {
  return (Ns >= 32 && E <= 8 && (N / E) % 32 == 0 && lean_ps<N, E>() < 5) ? 5 : lean_ps<N, E>();
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
    constexpr int G = N / E, NB = E / R, PS = PAD ? lean_ps_at<N, E, Ns>() : 30;
    constexpr bool last = Ns * R == N;
    // with G a multiple of Ns every butterfly of a lane has k = g mod Ns
    // (Ns is a power of two, or 3 times one after a first radix-3 stage)
    constexpr bool kconst = G % Ns == 0;
    constexpr bool ns2 = (Ns & (Ns - 1)) == 0;
    // write positions split as P(g) + C(b, c); with C a multiple of 2^PS
    // (or no padding) the padded position is pad(P) + pad(C)
    constexpr bool wlin = kconst && (!PAD || ((Ns == 1 || Ns % (1 << PS) == 0) && (G * R) % (1 << PS) == 0));
#pragma unroll
    for (int b = 0; b < NB; ++b) {
      const int j = g + G * b;
      const int k = ns2 ? (kconst ? (g & (Ns - 1)) : (j & (Ns - 1))) : (kconst ? g % Ns : j % Ns);
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


// Tables of the whole-row body in LDS, written by the NT threads of the
// workgroup (the caller synchronises before use): the per-stage FFT
// twiddles (ntw words from st), and for residues r < q
//   zA[r G + g] = zeta_{qm}^{r g},  zB[r E + e] = zeta_{qm}^{r G e},
//   zC[r] = zeta_{qm}^{r m} = zeta_q^r (second block, P = 2).
// Exponents r g < q G, r G e < q m and r m < q m need no reduction.
template <typename T, int N, int E, int P>
__device__ __forceinline__ void lean_row_tables(const cpx<T>* st, int ntw, const RootTable<T>& zqm, int q, int tid,
                                                int NT, cpx<T>* twl, cpx<T>* zA, cpx<T>* zB, cpx<T>* zC) {
  constexpr int G = N / E;
  for (int i = tid; i < ntw; i += NT) twl[i] = st[i];
  for (int i = tid; i < q * G; i += NT) zA[i] = zqm.get((uint32_t)((i / G) * (i % G)));
  for (int i = tid; i < q * E; i += NT) zB[i] = zqm.get((uint32_t)((i / E) * G * (i % E)));
  if constexpr (P == 2)
    for (int i = tid; i < q; i += NT) zC[i] = zqm.get((uint32_t)(i * N));
}

// A complex word read as one aligned pair (entries of the LDS tables are
// aligned to their size, which the element type alone does not state).
template <typename T>
__device__ __forceinline__ cpx<T> ld_pair(const cpx<T>* p) {
  typedef T pair_t __attribute__((ext_vector_type(2)));
  const pair_t v = *reinterpret_cast<const pair_t*>(p);
  return mk(v.x, v.y);
}

// Whole-point table of the second residue when q = 2 (the usual M = 2L):
// zF[s] = zeta_{qm}^{s}, s < N, so that a lane's twiddle at point
// s = g + G e is one LDS read at a constant offset rather than a complex
// product per use.
template <typename T, int N>
__device__ __forceinline__ void lean_row_q2_table(const RootTable<T>& zqm, int tid, int NT, cpx<T>* zF) {
  for (int i = tid; i < N; i += NT) zF[i] = zqm.get((uint32_t)i);
}

// One row of the direct form (Sec. 2, Algorithms 3-6) with p = P <= 2
// blocks of N points: for each residue r < q
//   W_s = zeta_{qm}^{r s} (f_s + zeta_q^r f_{N+s}),  F_a = fft_N(W) per input,
//   h_{tN+s} += zeta_q^{-r t} zeta_{qm}^{-r s} ifft_N(prod_a F_a)_s,
// and out = h / (q N) for the first L points.  Lane g of the row's G = N/E
// lanes holds points g + G e; src[a] and dst point at the row's point g.
// Every lane of the row calls this (the transforms synchronise the
// workgroup); `valid` is false for a row beyond the last (it reads its
// clamped source and stores nothing).  FULL: one block and L = N.  Inputs of
// at most KEEP words per lane are held in registers across the residues.
// ZF: zF points at this lane's entry of the q = 2 table of lean_row_q2_table.
template <typename T, int N, int E, int A, int P, bool FULL, int KEEP = 8, bool ZF = false>
__device__ __forceinline__ void lean_row(const cpx<T>* const (&src)[A], cpx<T>* dst, bool valid, uint32_t L, int q,
                                         T scale, int g, cpx<T>* xr, const cpx<T>* twl, const cpx<T>* zA,
                                         const cpx<T>* zB, const cpx<T>* zC, const cpx<T>* zF = nullptr) {
  constexpr int G = N / E;
  // Inputs of A P E <= KEEP words per lane stay in registers across the
  // residues; larger ones are read again (from cache) for each residue.
  // With 16 points per lane the residue twiddles are formed again at each
  // use rather than held across the transforms.
  constexpr bool kKeep = A * P * E <= KEEP;
  constexpr bool kHoldZ = E <= 8;
  // Loads never branch: a point beyond L reads point L-1 and is replaced by
  // 0.  Full rows read at constant offsets from one per-lane address.
  auto load = [&](int ai, int t, int e) -> cpx<T> {
    if constexpr (FULL) return src[ai][G * e];
    const uint32_t i = (uint32_t)(t * N + g + G * e);
    const cpx<T> v = src[ai][(int)(i < L ? i : L - 1) - g];
    return i < L ? v : czero<T>();
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
  // this lane's second-residue twiddle at point g + G e.  Without the
  // whole-point table the products zeta^{g} zeta^{G e} are formed again at
  // each of their three uses: the LDS entries are read through an opaque
  // offset, so the compiler cannot keep the E products live across the
  // transforms (with 16 points per lane they spilled to scratch memory,
  // 0.5 GB of extra HBM traffic per 256^3 row pass).
  auto z1_base = [&]() -> const cpx<T>* {
    int off = E;
    asm volatile("" : "+v"(off));
    return zB + off;
  };
  auto z1 = [&](cpx<T> za, const cpx<T>* zb1, int e) -> cpx<T> {
    if constexpr (ZF) return ld_pair(zF + G * e);
    else return cmul(za, zb1[e]);
  };
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
      const cpx<T>* zb1 = z1_base();
#pragma unroll
      for (int e = 0; e < E; ++e) {
        const cpx<T> xv = P == 2 ? xa[0][e] + cmul(xa[P - 1][e], zc) : xa[0][e];
        w[e] = cmul(xv, z1(za, zb1, e));
      }
      lean_fft<T, N, E, +1>(w, g, xr, twl);
#pragma unroll
      for (int e = 0; e < E; ++e) p1[e] = ai == 0 ? w[e] : cmul(p1[e], w[e]);
    }
    lean_fft<T, N, E, -1>(p0, g, xr, twl);
#pragma unroll
    for (int e = 0; e < E; ++e) acc[0][e] = acc[P - 1][e] = p0[e];
    lean_fft<T, N, E, -1>(p1, g, xr, twl);
    const cpx<T>* zb1 = z1_base();
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const cpx<T> y = cmulc(p1[e], z1(za, zb1, e));
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
#pragma unroll
    for (int t = 0; t < P; ++t)
#pragma unroll
      for (int e = 0; e < E; ++e)
        if (FULL || (uint32_t)(t * N + g + G * e) < L) dst[t * N + G * e] = cscale(acc[t][e], scale);
  }
}

}  // namespace hd
