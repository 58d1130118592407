// hd_k_multi.hip -- the three passes of the inner-loop form (Sec. 6.1), with
// the centered (signed block, folded) and Hermitian (mirrored half, paired
// real rows) variants.
#include "hd_kcommon.hpp"

namespace hd {

// ---------------------------------------------------------------------------
// Block index of column position tau (0 <= tau < p): tau itself, or for a
// centered row with tneg blocks left of index 0 the signed block tau - p once
// tau >= p - tneg (the p-point DFT is periodic in the block index).
__device__ __forceinline__ int signed_block(int tau, int p, int tneg) { return tau < p - tneg ? tau : tau - p; }

// Calls f(e, zeta_q^{v (g + G e)}) for e = 0 .. E-1 (v < n, so v (g + G e) <
// q): the powers are composed from three table lookups, zeta_q^{v g},
// w = zeta_q^{v G} and w^4, as z = base w^{e mod 4} (w^4)^{e div 4}, instead
// of one lookup per point.
template <int E, typename T, typename F>
__device__ __forceinline__ void zq_run(const cpx<T>* zq, int v, int g, int G, int q, F&& f) {
  static_assert(E <= 16, "at most 16 powers per run");
  const cpx<T> base = zq[v * g];
  cpx<T> p0[4], p1[4];
  p0[0] = p1[0] = mk(T(1), T(0));
  if constexpr (E > 1) {
    const int st = v * G;  // < q
    p0[1] = zq[st];
    p0[2] = cmul(p0[1], p0[1]);
    p0[3] = cmul(p0[2], p0[1]);
    if constexpr (E > 4) {
      int s4 = 4 * st;
      while (s4 >= q) s4 -= q;
      p1[1] = zq[s4];
      p1[2] = cmul(p1[1], p1[1]);
      p1[3] = cmul(p1[2], p1[1]);
    }
  }
#pragma unroll
  for (int e = 0; e < E; ++e) {
    cpx<T> z = base;
    if (e & 3) z = cmul(z, p0[e & 3]);
    if (e >> 2) z = cmul(z, p1[e >> 2]);
    f(e, z);
  }
}

// Inner form, pass 1 (Sec. 6.1, forward): columns s of the p x m view.  For
// each residue v the column is scaled by zeta_q^{vt} and p-point transformed;
// residues are taken two at a time (shared twiddles and barriers).  Centered
// rows (the paper's centered inner form) use the signed block index t; with
// FOLD, position tau carries block tau (x) and the negative block tau - p
// (x1), each with its own twiddle.
template <typename T, int E, int NT, bool FOLD>
__device__ __forceinline__ void cols_fwd_residues(const ColFwdArgs<T>& a, const cpx<T> (&x)[E],
                                                  const cpx<T> (&x1)[FOLD ? E : 1], int dv0, int g, int s,
                                                  int64_t row, int ai, int tneg, const TwLds<T>& tw,
                                                  const Xchg<T>& xb) {
  const int G = a.fd.G, m = a.m, p = a.p, q = a.q;
  cpx<T> y[NT][E];
#pragma unroll
  for (int n = 0; n < NT; ++n) {
    const int v = a.v0 + dv0 + n;
    // the negative block t - p carries zeta_q^{v (t - p)} = zeta_q^{v t} c
    const cpx<T> zc = a.zq[v * p ? q - v * p : 0];
    if constexpr (FOLD) {
      zq_run<E>(a.zq, v, g, G, q, [&](int e, cpx<T> z) { y[n][e] = cmul(z, x[e] + cmul(zc, x1[FOLD ? e : 0])); });
    } else if (tneg == 0) {
      zq_run<E>(a.zq, v, g, G, q, [&](int e, cpx<T> z) { y[n][e] = cmul(x[e], z); });
    } else {
      zq_run<E>(a.zq, v, g, G, q, [&](int e, cpx<T> z) {
        const cpx<T> xe = g + G * e >= p - tneg ? cmul(x[e], zc) : x[e];
        y[n][e] = cmul(xe, z);
      });
    }
  }
  gfft_any<T, E, +1, NT, (sizeof(T) == 4 ? kCtCols : 0u)>(y, g, a.fd, tw, xb);
#pragma unroll
  for (int n = 0; n < NT; ++n) {
    cpx<T>* dst = a.work[ai] + ((row * a.D + dv0 + n) * p) * (int64_t)m + s;
#pragma unroll
    for (int e = 0; e < E; ++e) dst[(int64_t)(g + G * e) * m] = y[n][e];
  }
}

// Conjugate-symmetry pairing (the paper's conjugate symmetry optimization,
// complex case): residue n - v needs the p-point DFT of
// zeta_q^{(n-v)t} f_t = zeta_p^t conj(zeta_q^{vt}) f_t, i.e. at frequency u
// the DFT of conj(zeta_q^{vt}) f_t at u + 1.  So the twiddles of residue v
// serve both: W'_t = conj(z_t) x_t is transformed and its frequency u is
// stored as frequency u - 1 (mod p) of residue n - v.  For v = n - v (v = 0
// or n/2) the pair is the residue alone.  Ordinary rows only (no centered
// shift, no folding), a block of all n residues.
template <typename T, int E>
__device__ __forceinline__ void cols_fwd_pair(const ColFwdArgs<T>& a, const cpx<T> (&x)[E], int v, int g, int s,
                                              int64_t row, int ai, const TwLds<T>& tw, const Xchg<T>& xb) {
  const int G = a.fd.G, m = a.m, p = a.p, n = a.q / a.p;
  const int v2 = v == 0 ? 0 : n - v;
  cpx<T> y[1][E], y2[1][E];
  zq_run<E>(a.zq, v, g, G, a.q, [&](int e, cpx<T> z) {
    y[0][e] = cmul(x[e], z);
    y2[0][e] = cmulc(x[e], z);
  });
  gfft_any<T, E, +1, 1, (sizeof(T) == 4 ? kCtCols : 0u)>(y, g, a.fd, tw, xb);
  {
    cpx<T>* dst = a.work[ai] + ((row * a.D + (v - a.v0)) * p) * (int64_t)m + s;
#pragma unroll
    for (int e = 0; e < E; ++e) dst[(int64_t)(g + G * e) * m] = y[0][e];
  }
  if (v2 == v) return;
  gfft_any<T, E, +1, 1, (sizeof(T) == 4 ? kCtCols : 0u)>(y2, g, a.fd, tw, xb);
  cpx<T>* dst = a.work[ai] + ((row * a.D + (v2 - a.v0)) * p) * (int64_t)m + s;
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const int u = g + G * e;
    dst[(int64_t)(u ? u - 1 : p - 1) * m] = y2[0][e];
  }
}

// Grid x enumerates (row, column tile) pairs, column tiles fastest, so the
// row count is not bound by the grid's y limit.
template <typename T, int E, bool FOLD>
__global__ void __launch_bounds__(512) k_cols_fwd(ColFwdArgs<T> a) {
  const int S = a.S, G = a.fd.G, m = a.m;
  const int c = threadIdx.x % S;
  const int g = threadIdx.x / S;
  const uint32_t tiles = (uint32_t)(m / S);
  const int s = (int)(blockIdx.x % tiles) * S + c;
  const int64_t row = blockIdx.x / tiles;
  const int ai = blockIdx.z;
  const cpx<T>* src = a.tasks ? a.tasks[row].in[ai] : a.in[ai] + row * a.in_stride;
  const int64_t L = a.tasks ? a.tasks[row].L : a.L;
  const int64_t H = a.ctr ? L / 2 : 0;  // array position of index 0
  const int tneg = (int)((H + m - 1) / m);
  cpx<T>* lds = smem_as<T>();
  Xchg<T> xb{lds + c, S, 30, a.p * S};
  const TwLds<T> tw = stage_table(a.fd, a.fft_tw, lds + xwords_cols(a.p, S, 2));

  cpx<T> x[E], x1[FOLD ? E : 1];
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const int tau = g + G * e;
    // position i of the row (Hermitian rows: the signed index i - H of the
    // stored half, mirrored)
    auto ld = [&](int64_t i) -> cpx<T> {
      if (i < 0 || i >= L) return czero<T>();
      return a.herm ? herm_value(src, i - H) : src[i];
    };
    if constexpr (FOLD) {
      x[e] = ld((int64_t)tau * m + s + H);
      x1[FOLD ? e : 0] = ld((int64_t)(tau - a.p) * m + s + H);
    } else {
      x[e] = ld((int64_t)signed_block(tau, a.p, tneg) * m + s + H);
    }
  }
  __syncthreads();
  if constexpr (!FOLD) {
    if (a.pair) {
      // residues v and n - v together (v <= n/2; the block holds all n)
      const int n = a.q / a.p;
      for (int v = 0; 2 * v <= n; ++v) cols_fwd_pair<T, E>(a, x, v, g, s, row, ai, tw, xb);
      return;
    }
  }
  // FP32 transforms one residue at a time (fewer registers, twice the
  // resident workgroups: measured faster); FP64 two at a time.
  constexpr int NT = sizeof(T) == 4 ? 1 : 2;
  int dv = 0;
  if constexpr (NT == 2)
    for (; dv + 2 <= a.D; dv += 2) cols_fwd_residues<T, E, 2, FOLD>(a, x, x1, dv, g, s, row, ai, tneg, tw, xb);
  for (; dv < a.D; ++dv) cols_fwd_residues<T, E, 1, FOLD>(a, x, x1, dv, g, s, row, ai, tneg, tw, xb);
}

// Inner form, pass 2: m-point convolution rows.  The A rows are loaded
// together and transformed together.  The twiddles zeta_{qm}^{r s} are looked
// up again for the post-multiplication rather than kept in registers across
// the transforms.  Hermitian plans (HERM): every row's transform is real, so
// a slot takes two rows a, b and packs them as x_a + i x_b into one
// transform per input (F_a = Re, F_b = Im), the products go back packed as
// P_a + i P_b, and the inverse Y splits by conjugate symmetry:
// y_a(s) = (Y(s) + conj Y(-s)) / 2, y_b(s) = (Y(s) - conj Y(-s)) / (2i).
template <typename T, int E, int A, bool HERM, bool QUAD>
__global__ void __launch_bounds__(512) k_rows_conv(RowConvArgs<T> a) {
  const int G = a.fd.G, m = a.m, p = a.p;
  const int slot = threadIdx.x / G;
  const int g = threadIdx.x - slot * G;
  const int64_t R2 = HERM ? 2 * ((int64_t)blockIdx.x * a.rows_per_block + slot)
                          : (int64_t)blockIdx.x * a.rows_per_block + slot;
  const bool valid = R2 < a.nrows;
  const bool valid_b = HERM && R2 + 1 < a.nrows;
  // twiddle exponent r s for s = g + G e: start and step; r < q and g, G < m,
  // so both stay below q m without reduction
  auto residue = [&](int64_t row) -> uint32_t {
    const int u = (int)(row % p);
    const int dv = (int)((row / p) % a.D);
    return (uint32_t)u * (uint32_t)a.n + (uint32_t)(a.v0 + dv);
  };
  const uint32_t r = residue(R2);
  const uint32_t rb = HERM ? residue(R2 + 1) : 0u;
  cpx<T>* lds = smem_as<T>();
  Xchg<T> xb{lds + (size_t)slot * A * row_pad(m, a.fd.ps), 1, a.fd.ps, row_pad(m, a.fd.ps)};

  cpx<T> x[A][E];
#pragma unroll
  for (int ai = 0; ai < A; ++ai) {
    const cpx<T>* src = a.work[ai] + R2 * m;
#pragma unroll
    for (int e = 0; e < E; ++e) x[ai][e] = valid ? ld_at(src, (uint32_t)(g + G * e)) : czero<T>();
  }
  const TwLds<T> tw = stage_table(a.fd, a.fft_tw, lds + xwords_rows(m, a.fd.ps, a.rows_per_block, A));
  a.zqm.template run<E>(r * (uint32_t)g, r * (uint32_t)G, [&](int e, cpx<T> z) {
#pragma unroll
    for (int ai = 0; ai < A; ++ai) x[ai][e] = cmul(x[ai][e], z);
  });
  if constexpr (HERM) {
    // the second row enters as i times its twiddled values
    a.zqm.template run<E>(rb * (uint32_t)g, rb * (uint32_t)G, [&](int e, cpx<T> z) {
#pragma unroll
      for (int ai = 0; ai < A; ++ai) {
        const cpx<T> v = valid_b ? cmul(ld_at(a.work[ai] + (R2 + 1) * m, (uint32_t)(g + G * e)), z) : czero<T>();
        x[ai][e] = x[ai][e] + mk(-v.y, v.x);
      }
    });
  }
  __syncthreads();
  gfft_any<T, E, +1, A, (A == 2 ? kCtRows : 0u)>(x, g, a.fd, tw, xb);
  cpx<T> prod[1][E];
  mult_all<QUAD>(x, prod, a.quad, HERM);
  gfft_any<T, E, -1, 1, (A == 2 ? kCtRows : 0u)>(prod, g, a.fd, tw, xb);
  if constexpr (HERM) {
    // Y(-s) from the lane that holds it, through LDS
    __syncthreads();
#pragma unroll
    for (int e = 0; e < E; ++e) xb.at(0, g + G * e) = prod[0][e];
    __syncthreads();
    cpx<T> ym[E];
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const int sidx = g + G * e;
      ym[e] = xb.at(0, sidx ? m - sidx : 0);
    }
    if (valid_b) {
      cpx<T>* dstb = (a.out ? a.out : a.work[0]) + (R2 + 1) * m;
      a.zqm.template run<E>(rb * (uint32_t)g, rb * (uint32_t)G, [&](int e, cpx<T> z) {
        const cpx<T> yv = prod[0][e];  // y_b = -i (Y - conj Ym) / 2
        st_at(dstb, (uint32_t)(g + G * e), cmulc(mk(T(0.5) * (yv.y + ym[e].y), T(0.5) * (ym[e].x - yv.x)), z));
      });
    }
#pragma unroll
    for (int e = 0; e < E; ++e)  // y_a = (Y + conj Ym) / 2
      prod[0][e] = mk(T(0.5) * (prod[0][e].x + ym[e].x), T(0.5) * (prod[0][e].y - ym[e].y));
  }
  if (valid) {
    cpx<T>* dst = (a.out ? a.out : a.work[0]) + R2 * m;
    a.zqm.template run<E>(r * (uint32_t)g, r * (uint32_t)G, [&](int e, cpx<T> z) {
      st_at(dst, (uint32_t)(g + G * e), cmulc(prod[0][e], z));
    });
  }
}

// Inner form, pass 3 (eq. invInner): columns back to the p x m view.  With
// FOLD the value at position tau also feeds the negative block tau - p (acc1).
template <typename T, int E, int NT, bool FOLD>
__device__ __forceinline__ void cols_bwd_residues(const ColBwdArgs<T>& a, cpx<T> (&acc)[E],
                                                  cpx<T> (&acc1)[FOLD ? E : 1], int dv0, int g, int s,
                                                  int64_t row, int tneg, const TwLds<T>& tw, const Xchg<T>& xb) {
  const int G = a.fd.G, m = a.m, p = a.p, q = a.q;
  cpx<T> y[NT][E];
#pragma unroll
  for (int n = 0; n < NT; ++n) {
    const cpx<T>* src = a.work + ((row * a.D + dv0 + n) * p) * (int64_t)m + s;
#pragma unroll
    for (int e = 0; e < E; ++e) y[n][e] = src[(int64_t)(g + G * e) * m];
  }
  gfft_any<T, E, -1, NT, (sizeof(T) == 4 ? kCtCols : 0u)>(y, g, a.fd, tw, xb);
#pragma unroll
  for (int n = 0; n < NT; ++n) {
    const int v = a.v0 + dv0 + n;
    // the negative block t - p takes conj(zeta_q^{v (t - p)}) = conj(zeta_q^{v t} c)
    const cpx<T> zc = a.zq[v * p ? q - v * p : 0];
    if constexpr (FOLD) {
      zq_run<E>(a.zq, v, g, G, q, [&](int e, cpx<T> z) {
        const cpx<T> t = cmulc(y[n][e], z);
        acc[e] = acc[e] + t;
        acc1[FOLD ? e : 0] = acc1[FOLD ? e : 0] + cmulc(t, zc);
      });
    } else if (tneg == 0) {
      zq_run<E>(a.zq, v, g, G, q, [&](int e, cpx<T> z) { acc[e] = acc[e] + cmulc(y[n][e], z); });
    } else {
      zq_run<E>(a.zq, v, g, G, q, [&](int e, cpx<T> z) {
        const cpx<T> t = cmulc(y[n][e], z);
        acc[e] = acc[e] + (g + G * e >= p - tneg ? cmulc(t, zc) : t);
      });
    }
  }
}

template <typename T, int E, bool FOLD>
__global__ void __launch_bounds__(512) k_cols_bwd(ColBwdArgs<T> a) {
  const int S = a.S, G = a.fd.G, m = a.m;
  const int c = threadIdx.x % S;
  const int g = threadIdx.x / S;
  const uint32_t tiles = (uint32_t)(m / S);
  const int s = (int)(blockIdx.x % tiles) * S + c;
  const int64_t row = blockIdx.x / tiles;
  cpx<T>* lds = smem_as<T>();
  Xchg<T> xb{lds + c, S, 30, a.p * S};
  const TwLds<T> tw = stage_table(a.fd, a.fft_tw, lds + xwords_cols(a.p, S, 2));
  __syncthreads();

  const int64_t L = a.tasks ? a.tasks[row].L : a.L;
  const int64_t H = a.ctr ? L / 2 : 0;  // array position of index 0
  const int tneg = (int)((H + m - 1) / m);
  cpx<T> acc[E], acc1[FOLD ? E : 1];
#pragma unroll
  for (int e = 0; e < E; ++e) acc[e] = czero<T>();
  if constexpr (FOLD)
#pragma unroll
    for (int e = 0; e < E; ++e) acc1[FOLD ? e : 0] = czero<T>();
  int dv = 0;
  for (; dv + 2 <= a.D; dv += 2) cols_bwd_residues<T, E, 2, FOLD>(a, acc, acc1, dv, g, s, row, tneg, tw, xb);
  if (dv < a.D) cols_bwd_residues<T, E, 1, FOLD>(a, acc, acc1, dv, g, s, row, tneg, tw, xb);
  cpx<T>* dst = a.tasks ? a.tasks[row].out : a.out + row * a.out_stride;
  double* acc64 = a.acc ? a.acc + 2 * row * a.out_stride : nullptr;
  // Hermitian rows keep the outputs c = i - H >= 0, at c
  const int64_t lo = a.herm ? H : 0, osh = a.herm ? H : 0;
  auto put = [&](int64_t i, cpx<T> v) {
    if (i >= lo && i < L) acc_store(dst, acc64, a.acc_mode, i - osh, v, a.scale);
  };
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const int tau = g + G * e;
    if constexpr (FOLD) {
      put((int64_t)tau * m + s + H, acc[e]);
      put((int64_t)(tau - a.p) * m + s + H, acc1[FOLD ? e : 0]);
    } else {
      put((int64_t)signed_block(tau, a.p, tneg) * m + s + H, acc[e]);
    }
  }
}

template <typename T>
hipError_t launch_cols_fwd(const ColFwdArgs<T>& a, int E, int A, hipStream_t s) {
  const int nt = a.S * a.fd.G;
  if (nt > 512 || !fft_fits(a.fd, E) || a.p != a.fd.N || a.m % a.S != 0 ||
      (int64_t)(a.m / a.S) * a.nrows > 0x7fffffff)
    return HD_BAD;
  dim3 grid((unsigned)((a.m / a.S) * a.nrows), 1, A), block(nt);
  const size_t lds = lds_cols(a.p, a.S, tw_words(a.fd), sizeof(T));
#define C1(EE)                                                                   \
  if (E == EE)                                                                   \
    return a.fold ? go(k_cols_fwd<T, EE, true>, grid, block, lds, s, a)         \
                  : go(k_cols_fwd<T, EE, false>, grid, block, lds, s, a);
  C1(1) C1(2) C1(4) C1(8) C1(12) C1(16)
#undef C1
  return HD_BAD;
}

template <typename T>
hipError_t launch_rows_conv(const RowConvArgs<T>& a, int E, int A, hipStream_t s) {
  const int nt = a.fd.G * a.rows_per_block;
  if (nt > 512 || !fft_fits(a.fd, E) || a.m != a.fd.N) return HD_BAD;
  // Hermitian plans: a slot takes two rows
  const int64_t slots = a.herm ? (a.nrows + 1) / 2 : a.nrows;
  dim3 grid((unsigned)((slots + a.rows_per_block - 1) / a.rows_per_block)), block(nt);
  const size_t lds = lds_rows(a.m, a.fd.ps, a.rows_per_block, A, tw_words(a.fd), sizeof(T));
#define R2(EE, AA, QQ)                                                            \
  return a.herm ? go(k_rows_conv<T, EE, AA, true, QQ>, grid, block, lds, s, a)    \
                : go(k_rows_conv<T, EE, AA, false, QQ>, grid, block, lds, s, a);
#define R1(EE, AA)                     \
  if (E == EE && A == AA) {            \
    if (a.quad.on) R2(EE, AA, true)    \
    R2(EE, AA, false)                  \
  }
  R1(4, 2) R1(4, 3) R1(8, 2) R1(8, 3) R1(12, 2) R1(12, 3) R1(16, 2) R1(16, 3)
#undef R1
#undef R2
  return HD_BAD;
}

template <typename T>
hipError_t launch_cols_bwd(const ColBwdArgs<T>& a, int E, hipStream_t s) {
  const int nt = a.S * a.fd.G;
  if (nt > 512 || !fft_fits(a.fd, E) || a.p != a.fd.N || a.m % a.S != 0 ||
      (int64_t)(a.m / a.S) * a.nrows > 0x7fffffff)
    return HD_BAD;
  dim3 grid((unsigned)((a.m / a.S) * a.nrows)), block(nt);
  const size_t lds = lds_cols(a.p, a.S, tw_words(a.fd), sizeof(T));
#define C1(EE)                                                                   \
  if (E == EE)                                                                   \
    return a.fold ? go(k_cols_bwd<T, EE, true>, grid, block, lds, s, a)         \
                  : go(k_cols_bwd<T, EE, false>, grid, block, lds, s, a);
  C1(1) C1(2) C1(4) C1(8) C1(12) C1(16)
#undef C1
  return HD_BAD;
}

#define HD_INST(T) \
  template hipError_t launch_cols_fwd<T>(const ColFwdArgs<T>&, int, int, hipStream_t); \
  template hipError_t launch_rows_conv<T>(const RowConvArgs<T>&, int, int, hipStream_t); \
  template hipError_t launch_cols_bwd<T>(const ColBwdArgs<T>&, int, hipStream_t);
// both precisions, or one per object when the build splits this file
// (HD_PART 1: FP32, 2: FP64)
#if !defined(HD_PART) || HD_PART == 1
HD_INST(float)
#endif
#if !defined(HD_PART) || HD_PART == 2
HD_INST(double)
#endif
#undef HD_INST

}  // namespace hd
