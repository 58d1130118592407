/*
 * oracle/conv.c -- plain, slow, FP64 CPU reference for the linear convolutions
 * that hybrid dealiasing computes (Murasko & Bowman, "Hybrid Dealiasing of
 * Complex Convolutions", arXiv 2303.17510).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library includes, links or
 * calls this file; only tests/, the smoke check and the benchmark's CPU
 * baseline leg use it.  It shares no code, table or header with the GPU path.
 *
 * What it computes (all in FP64, interleaved (re, im) doubles):
 *
 *  O1  direct sums of the definition (Sec. 2): for A = 2 inputs
 *          c_j = sum_{i=0}^{j} f_i g_{j-i},           j = 0 .. L-1,
 *      i.e. the first L outputs of the linear convolution, which are the
 *      outputs Algorithm 1 returns (its accumulators have length L).  The
 *      d-dimensional version (Sec. 5) sums over the box i_k <= j_k.  For
 *      A = 3 the product operator gives the triple convolution; because every
 *      index is non-negative it equals ((f*g) truncated to L) * h truncated
 *      to L, which is how it is evaluated.  Each real and imaginary partial
 *      sum uses Neumaier compensated summation.
 *
 *  O2  an explicitly zero-padded FFT convolution (the conventional method
 *      that Sec. 1 describes): every input is padded to N' = a power of two
 *      >= A(L-1)+1 per dimension (the minimal padding of Sec. 2), transformed
 *      with this file's own iterative radix-2 FFT, multiplied pointwise,
 *      inverse transformed, divided by N', and truncated to the first L
 *      entries per dimension.  N' is this file's own choice.
 *
 *  OC  centered convolutions (the paper's section on centered convolutions
 *      in one dimension, eq. centDFT; Sec. 5 per dimension): an array of L
 *      entries holds f_c for the centered indices c = -H .. L-1-H,
 *      H = floor(L/2), at position c + H, and the convolution is
 *          h_c = sum_{c1} f_{c1} g_{c-c1},   c = -H .. L-1-H,
 *      over every c1 with both c1 and c - c1 in range (A = 3: the triple
 *      sum, formed from the full pairwise convolution).  Evaluated as direct
 *      compensated sums, and as O2 on the full linear convolution whose
 *      entries (A-1)H .. (A-1)H+L-1 per dimension are the centered outputs.
 *
 *  OH  Hermitian convolutions (the paper's section on Hermitian symmetric
 *      convolutions): an array of Lh entries holds f_0 .. f_{Lh-1}, and the
 *      array it stands for is the centered f_{-(Lh-1)} .. f_{Lh-1} with
 *      f_{-j} = conj(f_j) (f_0 taken real).  The result is the centered
 *      convolution of the expanded arrays at c = 0 .. Lh-1.  The expansion is
 *      here (oracle_hermitian_expand, and oracle_hermitian_expand_nd for 2D/3D
 *      arrays whose last axis is the Hermitian one); the sums are OC's.
 *
 *  PD  the padded DFT of Sec. 2, F_k = sum_{j<L} zeta_N^{kj} f_j with
 *      zeta_N = exp(+2 pi i / N), evaluated term by term at requested k with
 *      the phase k*j reduced modulo N in exact integer arithmetic.  Used to
 *      check a single residue block of the forward transform (eq. forStan).
 *
 *  FFT the unnormalised transform X_k = sum_j x_j exp(sign 2 pi i jk/N) for a
 *      power-of-two N (sign +1 is the paper's forward transform, Sec. 2).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define TWO_PI 6.283185307179586476925286766559

/* Planted mistakes, compiled in only by the pin-strength test
 * (tests/test_oracle_mutants.py) with -DORACLE_MUTANT=k; the default build
 * has ORACLE_MUTANT == 0 and none of them. */
#ifndef ORACLE_MUTANT
#define ORACLE_MUTANT 0
#endif

/* ---- Neumaier compensated sum ---------------------------------------- */
typedef struct { double s, c; } nsum_t;

static inline void nsum_add(nsum_t* a, double x) {
  double t = a->s + x;
  if (fabs(a->s) >= fabs(x)) a->c += (a->s - t) + x;
  else a->c += (x - t) + a->s;
  a->s = t;
}
static inline double nsum_get(const nsum_t* a) { return a->s + a->c; }

/* accumulate the complex product (ar + i ai)(br + i bi) into (re, im) */
static inline void cmac(nsum_t* re, nsum_t* im, double ar, double ai, double br, double bi) {
#if ORACLE_MUTANT == 1 /* conjugated second operand */
  bi = -bi;
#endif
  nsum_add(re, ar * br);
  nsum_add(re, -(ai * bi));
  nsum_add(im, ar * bi);
  nsum_add(im, ai * br);
}

/* ---- O1: direct sums ---------------------------------------------------
 * shape: dims (1..3) extents L[0..dims-1], row-major, last index fastest.
 * f, g: complex arrays of prod(L) entries.  idx: flat output indices to
 * evaluate (nidx of them); out: 2*nidx doubles.
 */
int oracle_direct2(const double* f, const double* g, int dims, const int64_t* L,
                   const int64_t* idx, int64_t nidx, double* out) {
  if (dims < 1 || dims > 3) return -1;
  int64_t e[3] = {1, 1, 1};
  for (int d = 0; d < dims; ++d) e[3 - dims + d] = L[d];
  const int64_t n0 = e[0], n1 = e[1], n2 = e[2];
  int64_t total = n0 * n1 * n2;
  for (int64_t k = 0; k < nidx; ++k)
    if (idx[k] < 0 || idx[k] >= total) return -2;
#pragma omp parallel for schedule(dynamic, 1)
  for (int64_t k = 0; k < nidx; ++k) {
    int64_t j = idx[k];
    int64_t j2 = j % n2, j1 = (j / n2) % n1, j0 = j / (n1 * n2);
    nsum_t re = {0, 0}, im = {0, 0};
    for (int64_t i0 = 0; i0 <= j0; ++i0)
      for (int64_t i1 = 0; i1 <= j1; ++i1)
        for (int64_t i2 = 0; i2 <= j2; ++i2) {
#if ORACLE_MUTANT == 2 /* dropped last term of every sum */
          if (i2 == j2 && j2 > 0) continue;
#endif
          int64_t a = (i0 * n1 + i1) * n2 + i2;
#if ORACLE_MUTANT == 3 /* second operand read transposed (square last two axes) */
          int64_t b = (n1 == n2) ? ((j0 - i0) * n1 + (j2 - i2)) * n2 + (j1 - i1)
                                 : ((j0 - i0) * n1 + (j1 - i1)) * n2 + (j2 - i2);
#else
          int64_t b = ((j0 - i0) * n1 + (j1 - i1)) * n2 + (j2 - i2);
#endif
          cmac(&re, &im, f[2 * a], f[2 * a + 1], g[2 * b], g[2 * b + 1]);
        }
    out[2 * k] = nsum_get(&re);
    out[2 * k + 1] = nsum_get(&im);
  }
  return 0;
}

/* ---- FFT: iterative radix-2, unnormalised, exp(sign*2*pi*i*jk/N) -------- */
static int is_pow2(int64_t n) { return n > 0 && (n & (n - 1)) == 0; }

/* in-place transform of n complex values spaced `stride` complex apart */
static void fft_strided(double* x, int64_t n, int64_t stride, int sign, double* tmp) {
  /* gather into contiguous scratch */
  for (int64_t i = 0; i < n; ++i) {
    tmp[2 * i] = x[2 * i * stride];
    tmp[2 * i + 1] = x[2 * i * stride + 1];
  }
  /* bit-reversal permutation */
  for (int64_t i = 1, j = 0; i < n; ++i) {
    int64_t bit = n >> 1;
    for (; j & bit; bit >>= 1) j ^= bit;
    j ^= bit;
    if (i < j) {
      double tr = tmp[2 * i], ti = tmp[2 * i + 1];
      tmp[2 * i] = tmp[2 * j];
      tmp[2 * i + 1] = tmp[2 * j + 1];
      tmp[2 * j] = tr;
      tmp[2 * j + 1] = ti;
    }
  }
  /* butterflies; each twiddle is evaluated directly from its exact phase */
  for (int64_t len = 2; len <= n; len <<= 1) {
    int64_t half = len >> 1;
    for (int64_t k = 0; k < half; ++k) {
#if ORACLE_MUTANT == 4 /* twiddle sign flipped */
      double ang = -sign * TWO_PI * (double)k / (double)len;
#else
      double ang = sign * TWO_PI * (double)k / (double)len;
#endif
      double wr = cos(ang), wi = sin(ang);
      for (int64_t s = 0; s < n; s += len) {
        double* a = tmp + 2 * (s + k);
        double* b = tmp + 2 * (s + k + half);
        double br = b[0] * wr - b[1] * wi;
        double bi = b[0] * wi + b[1] * wr;
        b[0] = a[0] - br;
        b[1] = a[1] - bi;
        a[0] += br;
        a[1] += bi;
      }
    }
  }
  for (int64_t i = 0; i < n; ++i) {
    x[2 * i * stride] = tmp[2 * i];
    x[2 * i * stride + 1] = tmp[2 * i + 1];
  }
}

int oracle_fft(double* x, int64_t n, int sign) {
  if (!is_pow2(n) || (sign != 1 && sign != -1)) return -1;
  double* tmp = (double*)malloc(sizeof(double) * 2 * (size_t)n);
  if (!tmp) return -3;
  fft_strided(x, n, 1, sign, tmp);
  free(tmp);
  return 0;
}

/* n-dimensional transform of a row-major array with extents N[0..dims-1] */
static int fft_nd(double* x, int dims, const int64_t* N, int sign) {
  int64_t total = 1, nmax = 1;
  for (int d = 0; d < dims; ++d) {
    if (!is_pow2(N[d])) return -1;
    total *= N[d];
    if (N[d] > nmax) nmax = N[d];
  }
  for (int d = 0; d < dims; ++d) {
    int64_t n = N[d], inner = 1;
    for (int e = d + 1; e < dims; ++e) inner *= N[e];
    int64_t outer = total / (n * inner);
    int64_t lines = outer * inner;
    int err = 0;
#pragma omp parallel reduction(| : err)
    {
      double* tmp = (double*)malloc(sizeof(double) * 2 * (size_t)nmax);
      if (!tmp) err = 1;
      else {
#pragma omp for schedule(static)
        for (int64_t l = 0; l < lines; ++l) {
          int64_t o = l / inner, i = l % inner;
          fft_strided(x + 2 * (o * n * inner + i), n, inner, sign, tmp);
        }
        free(tmp);
      }
    }
    if (err) return -3;
  }
  return 0;
}

int oracle_fft_nd(double* x, int dims, const int64_t* N, int sign) {
  if (dims < 1 || dims > 3 || (sign != 1 && sign != -1)) return -1;
  return fft_nd(x, dims, N, sign);
}

/* ---- O2: explicitly padded FFT convolution ------------------------------
 * inputs: A pointers to complex arrays of prod(L) entries; out: prod(L)
 * complex.  A in {2, 3}; mult = product of the A transforms.
 */
/* O2 with the output box starting at position off[d] of the full linear
 * convolution (0 for O1's first L outputs, (A-1)H for the centered ones). */
static int explicit_window(const double* const* inputs, int A, int dims, const int64_t* L, const int64_t* off,
                           double* out) {
  if (A < 2 || A > 3 || dims < 1 || dims > 3) return -1;
  for (int d = 0; d < dims; ++d)
    if (off[d] < 0 || off[d] + L[d] > (int64_t)A * (L[d] - 1) + 1) return -1;
  int64_t N[3], total = 1, ltotal = 1;
  for (int d = 0; d < dims; ++d) {
#if ORACLE_MUTANT == 5 /* padding one short of the minimal A(L-1)+1 */
    int64_t need = (int64_t)A * (L[d] - 1), n = 1;
    if (need < 1) need = 1;
#else
    int64_t need = (int64_t)A * (L[d] - 1) + 1, n = 1;
#endif
    while (n < need) n <<= 1;
    N[d] = n;
    total *= n;
    ltotal *= L[d];
  }
  double* buf[3] = {0, 0, 0};
  int rc = 0;
  for (int a = 0; a < A; ++a) {
    buf[a] = (double*)calloc(2 * (size_t)total, sizeof(double));
    if (!buf[a]) { rc = -3; goto done; }
  }
  /* zero padding: copy each input into the corner of its padded box */
  for (int a = 0; a < A; ++a) {
    for (int64_t j = 0; j < ltotal; ++j) {
      int64_t rem = j, dst = 0, mul = 1;
      for (int d = dims - 1; d >= 0; --d) {
        int64_t c = rem % L[d];
        rem /= L[d];
        dst += c * mul;
        mul *= N[d];
      }
      buf[a][2 * dst] = inputs[a][2 * j];
      buf[a][2 * dst + 1] = inputs[a][2 * j + 1];
    }
    if ((rc = fft_nd(buf[a], dims, N, +1)) != 0) goto done;
  }
  /* pointwise product into buf[0] */
#pragma omp parallel for schedule(static)
  for (int64_t k = 0; k < total; ++k) {
    double pr = buf[0][2 * k], pi = buf[0][2 * k + 1];
    for (int a = 1; a < A; ++a) {
      double br = buf[a][2 * k], bi = buf[a][2 * k + 1];
      double r = pr * br - pi * bi;
      pi = pr * bi + pi * br;
      pr = r;
    }
    buf[0][2 * k] = pr;
    buf[0][2 * k + 1] = pi;
  }
  if ((rc = fft_nd(buf[0], dims, N, -1)) != 0) goto done;
  {
#if ORACLE_MUTANT == 6 /* normalised by the first extent only */
    double scale = 1.0 / (double)N[0];
#else
    double scale = 1.0 / (double)total;
#endif
    for (int64_t j = 0; j < ltotal; ++j) {
      int64_t rem = j, src = 0, mul = 1;
      for (int d = dims - 1; d >= 0; --d) {
        int64_t c = rem % L[d] + off[d];
        rem /= L[d];
        src += c * mul;
        mul *= N[d];
      }
      out[2 * j] = buf[0][2 * src] * scale;
      out[2 * j + 1] = buf[0][2 * src + 1] * scale;
    }
  }
done:
  for (int a = 0; a < A; ++a) free(buf[a]);
  return rc;
}

int oracle_explicit(const double* const* inputs, int A, int dims, const int64_t* L, double* out) {
  const int64_t off[3] = {0, 0, 0};
  return explicit_window(inputs, A, dims, L, off, out);
}

/* OC by O2: the centered outputs are entries (A-1)H .. (A-1)H+L-1 of the
 * full linear convolution of the arrays (every centered index shifted by H). */
int oracle_explicit_centered(const double* const* inputs, int A, int dims, const int64_t* L, double* out) {
  if (A < 2 || A > 3 || dims < 1 || dims > 3) return -1;
  int64_t off[3] = {0, 0, 0};
#if ORACLE_MUTANT == 9 /* centre rounded up instead of down */
  for (int d = 0; d < dims; ++d) off[d] = (int64_t)(A - 1) * ((L[d] + 1) / 2);
#else
  for (int d = 0; d < dims; ++d) off[d] = (int64_t)(A - 1) * (L[d] / 2);
#endif
  return explicit_window(inputs, A, dims, L, off, out);
}

/* ---- OC: centered direct sums ------------------------------------------
 * Operand a has extents La and centre offsets Ha (entry at position k holds
 * centered index k - Ha), operand b likewise (Lb, Hb); output position i
 * holds centered index i - Ho (extents Lo).  For every requested flat output
 * position: out = sum over positions k of a with
 *     c1 = k - Ha,  c2 = (i - Ho) - c1  and  0 <= c2 + Hb < Lb
 * of a[k] * b[c2 + Hb], per dimension.
 */
int oracle_direct_centered(const double* fa, const int64_t* La, const int64_t* Ha, const double* fb,
                           const int64_t* Lb, const int64_t* Hb, int dims, const int64_t* Lo, const int64_t* Ho,
                           const int64_t* idx, int64_t nidx, double* out) {
  if (dims < 1 || dims > 3) return -1;
  int64_t ea[3] = {1, 1, 1}, ha[3] = {0, 0, 0}, eb[3] = {1, 1, 1}, hb[3] = {0, 0, 0};
  int64_t eo[3] = {1, 1, 1}, ho[3] = {0, 0, 0};
  for (int d = 0; d < dims; ++d) {
    const int k = 3 - dims + d;
    ea[k] = La[d];
    ha[k] = Ha[d];
    eb[k] = Lb[d];
    hb[k] = Hb[d];
    eo[k] = Lo[d];
    ho[k] = Ho[d];
  }
  const int64_t total = eo[0] * eo[1] * eo[2];
  for (int64_t n = 0; n < nidx; ++n)
    if (idx[n] < 0 || idx[n] >= total) return -2;
#pragma omp parallel for schedule(dynamic, 1)
  for (int64_t n = 0; n < nidx; ++n) {
    const int64_t j = idx[n];
    const int64_t o[3] = {j / (eo[1] * eo[2]), (j / eo[2]) % eo[1], j % eo[2]};
    nsum_t re = {0, 0}, im = {0, 0};
    for (int64_t k0 = 0; k0 < ea[0]; ++k0) {
      const int64_t b0 = (o[0] - ho[0]) - (k0 - ha[0]) + hb[0];
      if (b0 < 0 || b0 >= eb[0]) continue;
      for (int64_t k1 = 0; k1 < ea[1]; ++k1) {
        const int64_t b1 = (o[1] - ho[1]) - (k1 - ha[1]) + hb[1];
        if (b1 < 0 || b1 >= eb[1]) continue;
        for (int64_t k2 = 0; k2 < ea[2]; ++k2) {
#if ORACLE_MUTANT == 8 /* centre of the second operand off by one (last axis) */
          const int64_t b2 = (o[2] - ho[2]) - (k2 - ha[2]) + hb[2] + 1;
#else
          const int64_t b2 = (o[2] - ho[2]) - (k2 - ha[2]) + hb[2];
#endif
          if (b2 < 0 || b2 >= eb[2]) continue;
          const int64_t a = (k0 * ea[1] + k1) * ea[2] + k2;
          const int64_t b = (b0 * eb[1] + b1) * eb[2] + b2;
          cmac(&re, &im, fa[2 * a], fa[2 * a + 1], fb[2 * b], fb[2 * b + 1]);
        }
      }
    }
    out[2 * n] = nsum_get(&re);
    out[2 * n + 1] = nsum_get(&im);
  }
  return 0;
}

/* ---- OH: Hermitian expansion --------------------------------------------
 * f holds f_0 .. f_{Lh-1}; out (2 Lh - 1 entries) receives the centered array
 * f_{-(Lh-1)} .. f_{Lh-1} at positions c + Lh - 1, with f_{-j} = conj(f_j)
 * and f_0 replaced by its real part (a Hermitian array has a real centre). */
int oracle_hermitian_expand(const double* f, int64_t Lh, double* out) {
  if (Lh < 1) return -1;
  const int64_t H = Lh - 1;
  for (int64_t c = -H; c <= H; ++c) {
    const int64_t j = c < 0 ? -c : c;
    double re = f[2 * j], im = f[2 * j + 1];
#if ORACLE_MUTANT == 10 /* mirror without the conjugate */
    if (c == 0) im = 0.0;
#else
    if (c < 0) im = -im;
    if (c == 0) im = 0.0;
#endif
    out[2 * (c + H)] = re;
    out[2 * (c + H) + 1] = im;
  }
  return 0;
}

/* OH in 2D/3D: f holds the stored box n[0] x n[1] x Lh (leading extents 1
 * below 3D; outer extents odd) of the array F(k, c), k the signed outer
 * indices (centre (n-1)/2 per outer axis), c = 0 .. Lh-1 on the last axis;
 * out (n[0] x n[1] x (2 Lh - 1)) receives F for c = -(Lh-1) .. Lh-1 with
 *     F(k, -c) = conj F(-k, c)              (c > 0),
 *     F(k, 0)  = (F(k, 0) + conj F(-k, 0)) / 2,
 * the Hermitian symmetry F(-k, -c) = conj F(k, c) of a real function's
 * coefficients (the c = 0 plane is replaced by its Hermitian part). */
int oracle_hermitian_expand_nd(const double* f, const int64_t* n, int64_t Lh, double* out) {
  if (Lh < 1 || n[0] < 1 || n[1] < 1 || n[0] % 2 == 0 || n[1] % 2 == 0) return -1;
  const int64_t H = Lh - 1, W = 2 * Lh - 1;
  for (int64_t i0 = 0; i0 < n[0]; ++i0)
    for (int64_t i1 = 0; i1 < n[1]; ++i1) {
      const int64_t r0 = n[0] - 1 - i0, r1 = n[1] - 1 - i1;  /* the reflected outer index -k */
      for (int64_t c = -H; c <= H; ++c) {
        const int64_t j = c < 0 ? -c : c;
        const double* a = f + 2 * ((i0 * n[1] + i1) * Lh + j);
        const double* b = f + 2 * ((r0 * n[1] + r1) * Lh + j);
        double re, im;
        if (c > 0) {
          re = a[0];
          im = a[1];
        } else if (c < 0) {
#if ORACLE_MUTANT == 10
          re = b[0];
          im = b[1];
#else
          re = b[0];
          im = -b[1];
#endif
        } else {
          re = 0.5 * (a[0] + b[0]);
          im = 0.5 * (a[1] - b[1]);
        }
        double* o = out + 2 * ((i0 * n[1] + i1) * W + (c + H));
        o[0] = re;
        o[1] = im;
      }
    }
  return 0;
}

/* ---- PD: padded DFT at requested frequencies ------------------------------
 * F_k = sum_{j<L} exp(+2 pi i (k j mod N) / N) f_j, for k in ks[0..nk-1].
 */
int oracle_padded_dft(const double* f, int64_t L, int64_t N, const int64_t* ks, int64_t nk, double* out) {
  if (L < 1 || N < 1) return -1;
#pragma omp parallel for schedule(dynamic, 4)
  for (int64_t i = 0; i < nk; ++i) {
    int64_t k = ((ks[i] % N) + N) % N;
    nsum_t re = {0, 0}, im = {0, 0};
    for (int64_t j = 0; j < L; ++j) {
      int64_t e = (int64_t)(((__int128)k * j) % N);
#if ORACLE_MUTANT == 7 /* exp(-2 pi i/N) instead of exp(+2 pi i/N) */
      double ang = -TWO_PI * (double)e / (double)N;
#else
      double ang = TWO_PI * (double)e / (double)N;
#endif
      cmac(&re, &im, cos(ang), sin(ang), f[2 * j], f[2 * j + 1]);
    }
    out[2 * i] = nsum_get(&re);
    out[2 * i + 1] = nsum_get(&im);
  }
  return 0;
}

int oracle_num_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

/* Threads for the parallel loops that follow (timing runs); returns the count. */
int oracle_set_num_threads(int n) {
#ifdef _OPENMP
  if (n > 0) omp_set_num_threads(n);
  return omp_get_max_threads();
#else
  (void)n;
  return 1;
#endif
}
