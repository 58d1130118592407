// hd_kernels.hip -- HIP kernels of the hybrid-dealiasing engine (gfx950).
//
// The convolution is bandwidth-bound, so no kernel uses matrix cores: every
// kernel streams its operands through registers once, runs its transforms
// with LDS exchanges (hd_fft.hpp) and writes its result once.  Global loads
// and stores are coalesced: consecutive lanes touch consecutive complex words.
#include "hd_engine.hpp"

namespace hd {

extern __shared__ __align__(16) char hd_smem[];

template <typename T>
__device__ __forceinline__ cpx<T>* smem_as() {
  return reinterpret_cast<cpx<T>*>(hd_smem);
}

__host__ __device__ constexpr int row_pad(int m) { return m + (m >> 4); }

// LDS words (complex) of each kernel's exchange area; the transform's twiddle
// table follows it.
__host__ __device__ constexpr int xwords_rows(int m, int rows_per_block, int nt) {
  return rows_per_block * nt * row_pad(m);
}
__host__ __device__ constexpr int xwords_cols(int p, int S, int nt) { return nt * p * S; }

// ---------------------------------------------------------------------------
// Whole 1D convolution of one contiguous row per lane group, direct form
// (Algorithms 1, 3-6): for each residue r < q,
//   W_s   = sum_{t<P} zeta_{qm}^{r(tm+s)} f_{tm+s}      (zero where tm+s >= L)
//   F     = fft_m(W) per input;  H = prod_a F_a         (mult, B = 1)
//   h_j  += zeta_{qm}^{-rj} ifft_m(H)_{j mod m}          (j = tm+s < L)
// and finally out_j = h_j / (qm).  With P = 2 the backward step is the
// corrected form of Algorithm 6 (the second half carries zeta_{qm}^{-rj},
// j = m+s, as eq. invStan requires).  The A forward transforms of a residue
// run together (shared twiddles and barriers).
template <typename T, int E, int P, int A>
__global__ void __launch_bounds__(512) k_fused1d(FusedArgs<T> a) {
  const int G = a.fd.G;
  const int m = a.m;
  const int slot = threadIdx.x / G;
  const int g = threadIdx.x - slot * G;
  const int64_t row = (int64_t)blockIdx.x * a.rows_per_block + slot;
  const bool valid = row < a.nrows;
  const int64_t L = a.L;
  const int64_t qm = (int64_t)a.q * m;
  cpx<T>* lds = smem_as<T>();
  Xchg<T> xb{lds + (size_t)slot * A * row_pad(m), 1, 4, row_pad(m)};
  const TwLds<T> tw = stage_table(a.fd, a.fft_tw, lds + xwords_rows(m, a.rows_per_block, A));
  __syncthreads();

  cpx<T> acc[P][E];
#pragma unroll
  for (int t = 0; t < P; ++t)
#pragma unroll
    for (int e = 0; e < E; ++e) acc[t][e] = czero<T>();

  for (int r = 0; r < a.q; ++r) {
    // exponents of zeta_{qm}^{r j} for j = t m + g + G e advance by r G per e
    const int64_t st = ((int64_t)r * G) % qm;
    cpx<T> w[A][E];
#pragma unroll
    for (int ai = 0; ai < A; ++ai)
#pragma unroll
      for (int e = 0; e < E; ++e) w[ai][e] = czero<T>();
#pragma unroll
    for (int t = 0; t < P; ++t) {
      int64_t ex = ((int64_t)r * (t * m + g)) % qm;
#pragma unroll
      for (int e = 0; e < E; ++e) {
        const int64_t j = (int64_t)t * m + g + G * e;
        if (valid && j < L) {
          const cpx<T> z = a.zqm.get(ex);
#pragma unroll
          for (int ai = 0; ai < A; ++ai) w[ai][e] = w[ai][e] + cmul(a.in[ai][row * a.in_stride + j], z);
        }
        ex += st;
        if (ex >= qm) ex -= qm;
      }
    }
    gfft<T, E, +1, A>(w, g, a.fd, tw, xb);
    cpx<T> prod[1][E];
#pragma unroll
    for (int e = 0; e < E; ++e) {
      cpx<T> pr = w[0][e];
#pragma unroll
      for (int ai = 1; ai < A; ++ai) pr = cmul(pr, w[ai][e]);
      prod[0][e] = pr;
    }
    gfft<T, E, -1, 1>(prod, g, a.fd, tw, xb);
#pragma unroll
    for (int t = 0; t < P; ++t) {
      int64_t ex = ((int64_t)r * (t * m + g)) % qm;
#pragma unroll
      for (int e = 0; e < E; ++e) {
        acc[t][e] = acc[t][e] + cmulc(prod[0][e], a.zqm.get(ex));
        ex += st;
        if (ex >= qm) ex -= qm;
      }
    }
  }
  if (valid) {
    cpx<T>* dst = a.out + row * a.out_stride;
#pragma unroll
    for (int t = 0; t < P; ++t)
#pragma unroll
      for (int e = 0; e < E; ++e) {
        const int64_t j = (int64_t)t * m + g + G * e;
        if (j < L) dst[j] = cscale(acc[t][e], a.scale);
      }
  }
}

// ---------------------------------------------------------------------------
// Inner form, pass 1 (Sec. 6.1, forward): columns s of the p x m view.  For
// each residue v the column is scaled by zeta_q^{vt} and p-point transformed;
// residues are taken two at a time (shared twiddles and barriers).
template <typename T, int E, int NT>
__device__ __forceinline__ void cols_fwd_residues(const ColFwdArgs<T>& a, const cpx<T> (&x)[E], int dv0, int g,
                                                  int s, int64_t row, int ai, const TwLds<T>& tw,
                                                  const Xchg<T>& xb) {
  const int G = a.fd.G, m = a.m, p = a.p, q = a.q;
  cpx<T> y[NT][E];
#pragma unroll
  for (int n = 0; n < NT; ++n) {
    const int v = a.v0 + dv0 + n;
#pragma unroll
    for (int e = 0; e < E; ++e) y[n][e] = cmul(x[e], a.zq[(v * (g + G * e)) % q]);
  }
  gfft<T, E, +1, NT>(y, g, a.fd, tw, xb);
#pragma unroll
  for (int n = 0; n < NT; ++n) {
    cpx<T>* dst = a.work[ai] + ((row * a.D + dv0 + n) * p) * (int64_t)m + s;
#pragma unroll
    for (int e = 0; e < E; ++e) dst[(int64_t)(g + G * e) * m] = y[n][e];
  }
}

template <typename T, int E>
__global__ void __launch_bounds__(512) k_cols_fwd(ColFwdArgs<T> a) {
  const int S = a.S, G = a.fd.G, m = a.m;
  const int c = threadIdx.x % S;
  const int g = threadIdx.x / S;
  const int s = blockIdx.x * S + c;
  const int64_t row = blockIdx.y;
  const int ai = blockIdx.z;
  const cpx<T>* src = a.in[ai] + row * a.in_stride;
  cpx<T>* lds = smem_as<T>();
  Xchg<T> xb{lds + c, S, 30, a.p * S};
  const TwLds<T> tw = stage_table(a.fd, a.fft_tw, lds + xwords_cols(a.p, S, 2));

  cpx<T> x[E];
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const int64_t j = (int64_t)(g + G * e) * m + s;
    x[e] = (j < a.L) ? src[j] : czero<T>();
  }
  __syncthreads();
  int dv = 0;
  for (; dv + 2 <= a.D; dv += 2) cols_fwd_residues<T, E, 2>(a, x, dv, g, s, row, ai, tw, xb);
  if (dv < a.D) cols_fwd_residues<T, E, 1>(a, x, dv, g, s, row, ai, tw, xb);
}

// Inner form, pass 2: m-point convolution rows.  The A rows are loaded
// together and transformed together.
template <typename T, int E, int A>
__global__ void __launch_bounds__(512) k_rows_conv(RowConvArgs<T> a) {
  const int G = a.fd.G, m = a.m, p = a.p;
  const int slot = threadIdx.x / G;
  const int g = threadIdx.x - slot * G;
  const int64_t R2 = (int64_t)blockIdx.x * a.rows_per_block + slot;
  const bool valid = R2 < a.nrows;
  const int u = (int)(R2 % p);
  const int dv = (int)((R2 / p) % a.D);
  const int64_t r = (int64_t)u * a.n + a.v0 + dv;
  const int64_t qm = a.qm;
  cpx<T>* lds = smem_as<T>();
  Xchg<T> xb{lds + (size_t)slot * A * row_pad(m), 1, 4, row_pad(m)};

  cpx<T> x[A][E];
#pragma unroll
  for (int ai = 0; ai < A; ++ai) {
    const cpx<T>* src = a.work[ai] + R2 * m;
#pragma unroll
    for (int e = 0; e < E; ++e) x[ai][e] = valid ? src[g + G * e] : czero<T>();
  }
  const TwLds<T> tw = stage_table(a.fd, a.fft_tw, lds + xwords_rows(m, a.rows_per_block, A));
  cpx<T> z[E];
  {
    int64_t ex = (r * g) % qm;
    const int64_t st = (r * G) % qm;
#pragma unroll
    for (int e = 0; e < E; ++e) {
      z[e] = a.zqm.get(ex);
      ex += st;
      if (ex >= qm) ex -= qm;
    }
  }
#pragma unroll
  for (int ai = 0; ai < A; ++ai)
#pragma unroll
    for (int e = 0; e < E; ++e) x[ai][e] = cmul(x[ai][e], z[e]);
  __syncthreads();
  gfft<T, E, +1, A>(x, g, a.fd, tw, xb);
  cpx<T> prod[1][E];
#pragma unroll
  for (int e = 0; e < E; ++e) {
    cpx<T> pr = x[0][e];
#pragma unroll
    for (int ai = 1; ai < A; ++ai) pr = cmul(pr, x[ai][e]);
    prod[0][e] = pr;
  }
  gfft<T, E, -1, 1>(prod, g, a.fd, tw, xb);
  if (valid) {
    cpx<T>* dst = a.work[0] + R2 * m;
#pragma unroll
    for (int e = 0; e < E; ++e) dst[g + G * e] = cmulc(prod[0][e], z[e]);
  }
}

template <typename T>
__device__ __forceinline__ void acc_store(cpx<T>* out, double* acc, int mode, int64_t i, cpx<T> v, T scale) {
  if (mode == ACC_WRITE) {
    out[i] = cscale(v, scale);
  } else if (mode == ACC_FIRST) {
    acc[2 * i] = (double)v.x;
    acc[2 * i + 1] = (double)v.y;
  } else if (mode == ACC_ADD) {
    acc[2 * i] += (double)v.x;
    acc[2 * i + 1] += (double)v.y;
  } else {
    const double sx = acc[2 * i] + (double)v.x, sy = acc[2 * i + 1] + (double)v.y;
    out[i] = mk(T(sx * (double)scale), T(sy * (double)scale));
  }
}

// Inner form, pass 3 (eq. invInner): columns back to the p x m view.
template <typename T, int E, int NT>
__device__ __forceinline__ void cols_bwd_residues(const ColBwdArgs<T>& a, cpx<T> (&acc)[E], int dv0, int g, int s,
                                                  int64_t row, const TwLds<T>& tw, const Xchg<T>& xb) {
  const int G = a.fd.G, m = a.m, p = a.p, q = a.q;
  cpx<T> y[NT][E];
#pragma unroll
  for (int n = 0; n < NT; ++n) {
    const cpx<T>* src = a.work + ((row * a.D + dv0 + n) * p) * (int64_t)m + s;
#pragma unroll
    for (int e = 0; e < E; ++e) y[n][e] = src[(int64_t)(g + G * e) * m];
  }
  gfft<T, E, -1, NT>(y, g, a.fd, tw, xb);
#pragma unroll
  for (int n = 0; n < NT; ++n) {
    const int v = a.v0 + dv0 + n;
#pragma unroll
    for (int e = 0; e < E; ++e) acc[e] = acc[e] + cmulc(y[n][e], a.zq[(v * (g + G * e)) % q]);
  }
}

template <typename T, int E>
__global__ void __launch_bounds__(512) k_cols_bwd(ColBwdArgs<T> a) {
  const int S = a.S, G = a.fd.G, m = a.m;
  const int c = threadIdx.x % S;
  const int g = threadIdx.x / S;
  const int s = blockIdx.x * S + c;
  const int64_t row = blockIdx.y;
  cpx<T>* lds = smem_as<T>();
  Xchg<T> xb{lds + c, S, 30, a.p * S};
  const TwLds<T> tw = stage_table(a.fd, a.fft_tw, lds + xwords_cols(a.p, S, 2));
  __syncthreads();

  cpx<T> acc[E];
#pragma unroll
  for (int e = 0; e < E; ++e) acc[e] = czero<T>();
  int dv = 0;
  for (; dv + 2 <= a.D; dv += 2) cols_bwd_residues<T, E, 2>(a, acc, dv, g, s, row, tw, xb);
  if (dv < a.D) cols_bwd_residues<T, E, 1>(a, acc, dv, g, s, row, tw, xb);
  cpx<T>* dst = a.out + row * a.out_stride;
  double* acc64 = a.acc ? a.acc + 2 * row * a.out_stride : nullptr;
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const int64_t j = (int64_t)(g + G * e) * m + s;
    if (j < a.L) acc_store(dst, acc64, a.acc_mode, j, acc[e], a.scale);
  }
}

// ---------------------------------------------------------------------------
// Outer dimension, direct form, forward: S adjacent columns per workgroup.
template <typename T, int E, int P>
__global__ void __launch_bounds__(512) k_outer_fwd(OuterFwdArgs<T> a) {
  const int S = a.S, G = a.fd.G, m = a.m;
  const int c = threadIdx.x % S;
  const int g = threadIdx.x / S;
  const int64_t col = (int64_t)blockIdx.x * S + c;
  const bool valid = col < a.R;
  const int64_t b = blockIdx.y;
  const int ai = blockIdx.z;
  const int64_t R = a.R;
  const int64_t qm = (int64_t)a.q * m;
  const cpx<T>* src = a.in[ai] + b * a.in_bstride + col;
  cpx<T>* lds = smem_as<T>();
  Xchg<T> xb{lds + c, S, 30, m * S};
  const TwLds<T> tw = stage_table(a.fd, a.fft_tw, lds + xwords_cols(m, S, 1));

  cpx<T> x[P][E];
#pragma unroll
  for (int t = 0; t < P; ++t)
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const int64_t j = (int64_t)t * m + g + G * e;
      x[t][e] = (valid && j < a.L) ? src[j * R] : czero<T>();
    }
  __syncthreads();
  for (int dr = 0; dr < a.D; ++dr) {
    const int64_t r = a.r0 + dr;
    cpx<T> w[1][E];
#pragma unroll
    for (int e = 0; e < E; ++e) w[0][e] = czero<T>();
#pragma unroll
    for (int t = 0; t < P; ++t) {
      int64_t ex = (r * (t * m + g)) % qm;
      const int64_t st = (r * G) % qm;
#pragma unroll
      for (int e = 0; e < E; ++e) {
        w[0][e] = w[0][e] + cmul(x[t][e], a.zqm.get(ex));
        ex += st;
        if (ex >= qm) ex -= qm;
      }
    }
    gfft<T, E, +1, 1>(w, g, a.fd, tw, xb);
    if (valid) {
      cpx<T>* dst = a.out[ai] + ((b * a.D + dr) * m) * R + col;
#pragma unroll
      for (int e = 0; e < E; ++e) dst[(int64_t)(g + G * e) * R] = w[0][e];
    }
  }
}

// Outer dimension, direct form, backward and accumulation over residues.
template <typename T, int E, int P>
__global__ void __launch_bounds__(512) k_outer_bwd(OuterBwdArgs<T> a) {
  const int S = a.S, G = a.fd.G, m = a.m;
  const int c = threadIdx.x % S;
  const int g = threadIdx.x / S;
  const int64_t col = (int64_t)blockIdx.x * S + c;
  const bool valid = col < a.R;
  const int64_t b = blockIdx.y;
  const int64_t R = a.R;
  const int64_t qm = (int64_t)a.q * m;
  cpx<T>* lds = smem_as<T>();
  Xchg<T> xb{lds + c, S, 30, m * S};
  const TwLds<T> tw = stage_table(a.fd, a.fft_tw, lds + xwords_cols(m, S, 1));
  __syncthreads();

  cpx<T> acc[P][E];
#pragma unroll
  for (int t = 0; t < P; ++t)
#pragma unroll
    for (int e = 0; e < E; ++e) acc[t][e] = czero<T>();
  for (int dr = 0; dr < a.D; ++dr) {
    const int64_t r = a.r0 + dr;
    const cpx<T>* src = a.y + ((b * a.D + dr) * m) * R + col;
    cpx<T> y[1][E];
#pragma unroll
    for (int e = 0; e < E; ++e) y[0][e] = valid ? src[(int64_t)(g + G * e) * R] : czero<T>();
    gfft<T, E, -1, 1>(y, g, a.fd, tw, xb);
#pragma unroll
    for (int t = 0; t < P; ++t) {
      int64_t ex = (r * (t * m + g)) % qm;
      const int64_t st = (r * G) % qm;
#pragma unroll
      for (int e = 0; e < E; ++e) {
        acc[t][e] = acc[t][e] + cmulc(y[0][e], a.zqm.get(ex));
        ex += st;
        if (ex >= qm) ex -= qm;
      }
    }
  }
  if (!valid) return;
  cpx<T>* dst = a.out + b * a.out_bstride + col;
  double* acc64 = a.acc ? a.acc + 2 * (b * a.out_bstride + col) : nullptr;
#pragma unroll
  for (int t = 0; t < P; ++t)
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const int64_t j = (int64_t)t * m + g + G * e;
      if (j < a.L) acc_store(dst, acc64, a.acc_mode, j * R, acc[t][e], a.scale);
    }
}

// ---------------------------------------------------------------------------
template <typename T>
__global__ void __launch_bounds__(256) k_box_copy(BoxCopyArgs<T> a) {
  // one destination row (i0, i1) per blockIdx.y step; lanes run along i2
  const int64_t* D = a.pad ? a.N : a.L;
  const int64_t* Sx = a.pad ? a.L : a.N;
  const int64_t rows = D[0] * D[1];
  for (int64_t row = blockIdx.y; row < rows; row += gridDim.y) {
    const int64_t i1 = row % D[1], i0 = row / D[1];
    const bool in_src = i0 < Sx[0] && i1 < Sx[1];
    const cpx<T>* src = a.src + (i0 * Sx[1] + i1) * Sx[2];
    cpx<T>* dst = a.dst + row * D[2];
    for (int64_t i2 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i2 < D[2];
         i2 += (int64_t)gridDim.x * blockDim.x)
      dst[i2] = (in_src && i2 < Sx[2]) ? src[i2] : czero<T>();
  }
}

// ---------------------------------------------------------------------------
// Host-side launchers.

size_t lds_fused1d(int m, int rows_per_block, int A, int ntw, int tbytes) {
  return ((size_t)xwords_rows(m, rows_per_block, A) + ntw) * 2 * tbytes;
}
size_t lds_rows(int m, int rows_per_block, int A, int ntw, int tbytes) {
  return ((size_t)xwords_rows(m, rows_per_block, A) + ntw) * 2 * tbytes;
}
size_t lds_cols(int p, int S, int ntw, int tbytes) { return ((size_t)xwords_cols(p, S, 2) + ntw) * 2 * tbytes; }
size_t lds_outer(int m, int S, int ntw, int tbytes) { return ((size_t)xwords_cols(m, S, 1) + ntw) * 2 * tbytes; }

bool fft_fits(const FftDesc& d, int E) {
  if ((int64_t)d.G * E != d.N) return false;
  for (int i = 0; i < d.nst; ++i)
    if (E % d.radix[i] != 0) return false;
  return true;
}

template <typename K>
static hipError_t allow_lds(K kernel, size_t lds) {
  if (lds <= 65536) return hipSuccess;
  return hipFuncSetAttribute(reinterpret_cast<const void*>(kernel),
                             hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
}

template <typename K, typename Args>
static hipError_t go(K kernel, dim3 grid, dim3 block, size_t lds, hipStream_t s, const Args& a) {
  hipError_t e = allow_lds(kernel, lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(kernel, grid, block, lds, s, a);
  return hipGetLastError();
}

#define HD_BAD hipErrorInvalidConfiguration

template <typename T>
hipError_t launch_fused1d(const FusedArgs<T>& a, int E, int P, int A, hipStream_t s) {
  const int nt = a.fd.G * a.rows_per_block;
  if (nt > 512 || !fft_fits(a.fd, E) || a.m != a.fd.N) return HD_BAD;
  dim3 grid((unsigned)((a.nrows + a.rows_per_block - 1) / a.rows_per_block)), block(nt);
  const size_t lds = lds_fused1d(a.m, a.rows_per_block, A, a.fd.ntw, sizeof(T));
#define F1(EE, PP, AA) \
  if (E == EE && P == PP && A == AA) return go(k_fused1d<T, EE, PP, AA>, grid, block, lds, s, a);
  F1(8, 1, 2) F1(8, 2, 2) F1(8, 1, 3) F1(8, 2, 3)
  F1(16, 1, 2) F1(16, 2, 2) F1(16, 1, 3) F1(16, 2, 3)
  F1(24, 1, 2) F1(24, 2, 2) F1(24, 1, 3) F1(24, 2, 3)
  F1(32, 1, 2) F1(32, 2, 2) F1(32, 1, 3) F1(32, 2, 3)
#undef F1
  return HD_BAD;
}

template <typename T>
hipError_t launch_cols_fwd(const ColFwdArgs<T>& a, int E, int A, hipStream_t s) {
  const int nt = a.S * a.fd.G;
  if (nt > 512 || !fft_fits(a.fd, E) || a.p != a.fd.N || a.m % a.S != 0 || a.nrows > 65535) return HD_BAD;
  dim3 grid(a.m / a.S, (unsigned)a.nrows, A), block(nt);
  const size_t lds = lds_cols(a.p, a.S, a.fd.ntw, sizeof(T));
#define C1(EE) \
  if (E == EE) return go(k_cols_fwd<T, EE>, grid, block, lds, s, a);
  C1(1) C1(2) C1(4) C1(8) C1(16) C1(24)
#undef C1
  return HD_BAD;
}

template <typename T>
hipError_t launch_rows_conv(const RowConvArgs<T>& a, int E, int A, hipStream_t s) {
  const int nt = a.fd.G * a.rows_per_block;
  if (nt > 512 || !fft_fits(a.fd, E) || a.m != a.fd.N) return HD_BAD;
  dim3 grid((unsigned)((a.nrows + a.rows_per_block - 1) / a.rows_per_block)), block(nt);
  const size_t lds = lds_rows(a.m, a.rows_per_block, A, a.fd.ntw, sizeof(T));
#define R1(EE, AA) \
  if (E == EE && A == AA) return go(k_rows_conv<T, EE, AA>, grid, block, lds, s, a);
  R1(8, 2) R1(8, 3) R1(16, 2) R1(16, 3) R1(24, 2) R1(24, 3) R1(32, 2) R1(32, 3)
#undef R1
  return HD_BAD;
}

template <typename T>
hipError_t launch_cols_bwd(const ColBwdArgs<T>& a, int E, hipStream_t s) {
  const int nt = a.S * a.fd.G;
  if (nt > 512 || !fft_fits(a.fd, E) || a.p != a.fd.N || a.m % a.S != 0 || a.nrows > 65535) return HD_BAD;
  dim3 grid(a.m / a.S, (unsigned)a.nrows), block(nt);
  const size_t lds = lds_cols(a.p, a.S, a.fd.ntw, sizeof(T));
#define C1(EE) \
  if (E == EE) return go(k_cols_bwd<T, EE>, grid, block, lds, s, a);
  C1(1) C1(2) C1(4) C1(8) C1(16) C1(24)
#undef C1
  return HD_BAD;
}

template <typename T>
hipError_t launch_outer_fwd(const OuterFwdArgs<T>& a, int E, int P, int A, hipStream_t s) {
  const int nt = a.S * a.fd.G;
  if (nt > 512 || !fft_fits(a.fd, E) || a.m != a.fd.N || a.nb > 65535) return HD_BAD;
  dim3 grid((unsigned)((a.R + a.S - 1) / a.S), (unsigned)a.nb, A), block(nt);
  const size_t lds = lds_outer(a.m, a.S, a.fd.ntw, sizeof(T));
#define O1(EE, PP) \
  if (E == EE && P == PP) return go(k_outer_fwd<T, EE, PP>, grid, block, lds, s, a);
  O1(8, 1) O1(8, 2) O1(16, 1) O1(16, 2) O1(24, 1) O1(24, 2) O1(32, 1) O1(32, 2)
#undef O1
  return HD_BAD;
}

template <typename T>
hipError_t launch_outer_bwd(const OuterBwdArgs<T>& a, int E, int P, hipStream_t s) {
  const int nt = a.S * a.fd.G;
  if (nt > 512 || !fft_fits(a.fd, E) || a.m != a.fd.N || a.nb > 65535) return HD_BAD;
  dim3 grid((unsigned)((a.R + a.S - 1) / a.S), (unsigned)a.nb), block(nt);
  const size_t lds = lds_outer(a.m, a.S, a.fd.ntw, sizeof(T));
#define O1(EE, PP) \
  if (E == EE && P == PP) return go(k_outer_bwd<T, EE, PP>, grid, block, lds, s, a);
  O1(8, 1) O1(8, 2) O1(16, 1) O1(16, 2) O1(24, 1) O1(24, 2) O1(32, 1) O1(32, 2)
#undef O1
  return HD_BAD;
}

template <typename T>
hipError_t launch_box_copy(const BoxCopyArgs<T>& a, hipStream_t s) {
  const int64_t* D = a.pad ? a.N : a.L;
  const int64_t rows = D[0] * D[1];
  int64_t bx = (D[2] + 255) / 256;
  if (bx > 4096) bx = 4096;
  int64_t by = rows < 65535 ? rows : 65535;
  hipLaunchKernelGGL(k_box_copy<T>, dim3((unsigned)bx, (unsigned)by), dim3(256), 0, s, a);
  return hipGetLastError();
}

#define HD_INST(T)                                                                      \
  template hipError_t launch_fused1d<T>(const FusedArgs<T>&, int, int, int, hipStream_t); \
  template hipError_t launch_cols_fwd<T>(const ColFwdArgs<T>&, int, int, hipStream_t);    \
  template hipError_t launch_rows_conv<T>(const RowConvArgs<T>&, int, int, hipStream_t);  \
  template hipError_t launch_cols_bwd<T>(const ColBwdArgs<T>&, int, hipStream_t);         \
  template hipError_t launch_outer_fwd<T>(const OuterFwdArgs<T>&, int, int, int, hipStream_t); \
  template hipError_t launch_outer_bwd<T>(const OuterBwdArgs<T>&, int, int, hipStream_t); \
  template hipError_t launch_box_copy<T>(const BoxCopyArgs<T>&, hipStream_t);
HD_INST(float)
HD_INST(double)
#undef HD_INST

}  // namespace hd
