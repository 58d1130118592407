// hd_k_outer.hip -- outer dimensions of 2D/3D convolutions (Sec. 5) and the
// explicit method's padding copies.
#include "hd_kcommon.hpp"

namespace hd {

// ---------------------------------------------------------------------------
// Position of index 0 and block shift of a centered outer dimension (the
// transform then runs over the signed indices c = (t - tneg) m + s, stored at
// array position t m + s - sh); all zero for an ordinary dimension.
struct CtrShift {
  int64_t tneg, sh;
};
template <int P>
__device__ __forceinline__ CtrShift ctr_shift(int ctr, int64_t L, int m) {
  // a centered dimension spans two blocks unless L = 1, so P = 1 never shifts
  const int64_t H = (P == 2 && ctr) ? L / 2 : 0;
  const int64_t tneg = H ? (H + m - 1) / m : 0;
  return CtrShift{tneg, tneg * m - H};
}

// Residue twiddle exponents of the direct form without division: for r < q
// and g < G <= m, r g and r G stay below qm; block t starts at the signed
// index (t - tneg) m + g, whose exponent is r g + m ((r (t - tneg)) mod q)
// with t - tneg in {-1, 0, 1} (P <= 2).
__device__ __forceinline__ uint32_t block_exp(uint32_t r, int t, int64_t tneg, uint32_t g, uint32_t m,
                                              uint32_t qm) {
  const int64_t d = t - tneg;
  const uint32_t rm = r * m;
  const uint32_t add = d == 0 ? 0u : (d > 0 ? rm : (rm ? qm - rm : 0u));
  const uint32_t e = r * g + add;
  return e >= qm ? e - qm : e;
}

// Offset of column col and the stride between rows j, for a layout (dense
// when all fields are zero).
__device__ __forceinline__ int64_t col_offset(const ColLayout& l, int64_t col) {
  return l.cgrp ? (col / l.cgrp) * l.cgstride + col % l.cgrp : col;
}

// Outer dimension, direct form, forward: S adjacent columns per workgroup.
template <typename T, int E, int P>
__global__ void __launch_bounds__(512) k_outer_fwd(OuterFwdArgs<T> a) {
  const int S = a.S, G = a.fd.G, m = a.m;
  const int c = threadIdx.x % S;
  const int g = threadIdx.x / S;
  const int64_t col = (int64_t)blockIdx.x * S + c;
  const bool valid = col < a.R;
  const int ai = blockIdx.z;
  const int64_t R = a.R;
  const int64_t qm = (int64_t)a.q * m;
  const int64_t js = a.lay.jstride ? a.lay.jstride : R;
  const CtrShift cs = ctr_shift<P>(a.ctr, a.L, m);
  cpx<T>* lds = smem_as<T>();
  Xchg<T> xb{lds + c, S, 30, m * S};
  const TwLds<T> tw = stage_table(a.fd, a.fft_tw, lds + xwords_cols(m, S, 1));

  // planes (copies, outer levels) beyond the grid's y extent loop; every
  // transform ends with a barrier after its last LDS read, so the next
  // plane's exchanges cannot overtake it
  for (int64_t b = blockIdx.y; b < a.nb; b += gridDim.y) {
    const cpx<T>* src = a.in[ai] + b * a.in_bstride + (valid ? col_offset(a.lay, col) : 0);
    cpx<T> x[P][E];
#pragma unroll
    for (int t = 0; t < P; ++t)
#pragma unroll
      for (int e = 0; e < E; ++e) {
        const int64_t i = (int64_t)t * m + g + G * e - cs.sh;
        x[t][e] = (valid && i >= 0 && i < a.L) ? src[i * js] : czero<T>();
      }
    __syncthreads();
    for (int dr = 0; dr < a.D; ++dr) {
      const int64_t r = a.r0 + dr;  // r < q
      const uint32_t st = (uint32_t)r * (uint32_t)G;
      cpx<T> w[1][E];
#pragma unroll
      for (int e = 0; e < E; ++e) w[0][e] = czero<T>();
#pragma unroll
      for (int t = 0; t < P; ++t)
        a.zqm.template run<E>(block_exp((uint32_t)r, t, cs.tneg, g, m, (uint32_t)qm), st,
                              [&](int e, cpx<T> z) { w[0][e] = w[0][e] + cmul(x[t][e], z); });
      gfft_any<T, E, +1, 1, kCtOuter>(w, g, a.fd, tw, xb);
      if (valid) {
        cpx<T>* dst = a.out[ai] + ((b * a.D + dr) * m) * R + col;
#pragma unroll
        for (int e = 0; e < E; ++e) dst[(int64_t)(g + G * e) * R] = w[0][e];
      }
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
  const int64_t R = a.R;
  const int64_t qm = (int64_t)a.q * m;
  const CtrShift cs = ctr_shift<P>(a.ctr, a.L, m);
  cpx<T>* lds = smem_as<T>();
  Xchg<T> xb{lds + c, S, 30, m * S};
  const TwLds<T> tw = stage_table(a.fd, a.fft_tw, lds + xwords_cols(m, S, 1));
  __syncthreads();

  // planes beyond the grid's y extent loop (see k_outer_fwd)
  for (int64_t b = blockIdx.y; b < a.nb; b += gridDim.y) {
    cpx<T> acc[P][E];
#pragma unroll
    for (int t = 0; t < P; ++t)
#pragma unroll
      for (int e = 0; e < E; ++e) acc[t][e] = czero<T>();
    for (int dr = 0; dr < a.D; ++dr) {
      const int64_t r = a.r0 + dr;  // r < q
      const uint32_t st = (uint32_t)r * (uint32_t)G;
      const cpx<T>* src = a.y + ((b * a.D + dr) * m) * R + col;
      cpx<T> y[1][E];
#pragma unroll
      for (int e = 0; e < E; ++e) y[0][e] = valid ? src[(int64_t)(g + G * e) * R] : czero<T>();
      gfft_any<T, E, -1, 1, kCtOuter>(y, g, a.fd, tw, xb);
#pragma unroll
      for (int t = 0; t < P; ++t)
        a.zqm.template run<E>(block_exp((uint32_t)r, t, cs.tneg, g, m, (uint32_t)qm), st,
                              [&](int e, cpx<T> z) { acc[t][e] = acc[t][e] + cmulc(y[0][e], z); });
    }
    if (!valid) continue;
    const int64_t coff = col_offset(a.lay, col), js = a.lay.jstride ? a.lay.jstride : R;
    cpx<T>* dst = a.out + b * a.out_bstride + coff;
    double* acc64 = a.acc ? a.acc + 2 * (b * a.out_bstride + coff) : nullptr;
#pragma unroll
    for (int t = 0; t < P; ++t)
#pragma unroll
      for (int e = 0; e < E; ++e) {
        const int64_t i = (int64_t)t * m + g + G * e - cs.sh;
        if (i >= 0 && i < a.L) acc_store(dst, acc64, a.acc_mode, i * js, acc[t][e], a.scale);
      }
  }
}

// ---------------------------------------------------------------------------
template <typename T>
__global__ void __launch_bounds__(256) k_box_copy(BoxCopyArgs<T> a) {
  // one destination row (i0, i1) per blockIdx.y step; lanes run along i2
  const int64_t* D = a.pad ? a.N : a.L;
  const int64_t* Sx = a.pad ? a.L : a.N;
  // source offsets (truncation only: the window of the padded result)
  const int64_t o0 = a.pad ? 0 : a.off[0], o1 = a.pad ? 0 : a.off[1], o2 = a.pad ? 0 : a.off[2];
  // element strides of the L box (the user's array, possibly strided) and of
  // the N box (dense)
  const int64_t l1 = a.ls[1] ? a.ls[1] : a.L[2], l0 = a.ls[0] ? a.ls[0] : a.L[1] * l1;
  const int64_t s1 = a.pad ? l1 : Sx[2], s0 = a.pad ? l0 : Sx[1] * Sx[2];
  const int64_t d1 = a.pad ? D[2] : l1, d0 = a.pad ? D[1] * D[2] : l0;
  const int64_t rows = D[0] * D[1];
  for (int64_t row = blockIdx.y; row < rows; row += gridDim.y) {
    const int64_t i1 = row % D[1], i0 = row / D[1];
    const bool in_src = i0 + o0 < Sx[0] && i1 + o1 < Sx[1];
    const cpx<T>* src = a.src + (i0 + o0) * s0 + (i1 + o1) * s1 + o2;
    cpx<T>* dst = a.dst + i0 * d0 + i1 * d1;
    for (int64_t i2 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i2 < D[2];
         i2 += (int64_t)gridDim.x * blockDim.x) {
      if (a.herm && a.pad) {
        // Hermitian padding: the expanded centered box, last-axis index
        // c = i2 - hH; c < 0 reads the conjugate at the reflected outer
        // position, c = 0 the Hermitian part of the stored plane
        cpx<T> v = czero<T>();
        if (i0 < a.L[0] && i1 < a.L[1] && i2 <= 2 * a.hH) {
          const int64_t c = i2 - a.hH, j = c < 0 ? -c : c;
          const cpx<T> f = a.src[i0 * l0 + i1 * l1 + j];
          const cpx<T> g = a.src[(a.L[0] - 1 - i0) * l0 + (a.L[1] - 1 - i1) * l1 + j];
          v = c > 0 ? f : (c < 0 ? mk(g.x, -g.y) : mk(T(0.5) * (f.x + g.x), T(0.5) * (f.y - g.y)));
        }
        dst[i2] = v;
      } else
        dst[i2] = (in_src && i2 + o2 < Sx[2]) ? src[i2] : czero<T>();
    }
  }
}

template <typename T>
hipError_t launch_outer_fwd(const OuterFwdArgs<T>& a, int E, int P, int A, hipStream_t s) {
  const int nt = a.S * a.fd.G;
  if (nt > 512 || !fft_fits(a.fd, E) || a.m != a.fd.N || a.nb < 1) return HD_BAD;
  dim3 grid((unsigned)((a.R + a.S - 1) / a.S), (unsigned)std::min<int64_t>(a.nb, 65535), A), block(nt);
  const size_t lds = lds_outer(a.m, a.S, tw_words(a.fd), sizeof(T));
#define O1(EE, PP) \
  if (E == EE && P == PP) return go(k_outer_fwd<T, EE, PP>, grid, block, lds, s, a);
  O1(4, 1) O1(4, 2) O1(8, 1) O1(8, 2) O1(12, 1) O1(12, 2) O1(16, 1) O1(16, 2)
#undef O1
  return HD_BAD;
}

template <typename T>
hipError_t launch_outer_bwd(const OuterBwdArgs<T>& a, int E, int P, hipStream_t s) {
  const int nt = a.S * a.fd.G;
  if (nt > 512 || !fft_fits(a.fd, E) || a.m != a.fd.N || a.nb < 1) return HD_BAD;
  dim3 grid((unsigned)((a.R + a.S - 1) / a.S), (unsigned)std::min<int64_t>(a.nb, 65535)), block(nt);
  const size_t lds = lds_outer(a.m, a.S, tw_words(a.fd), sizeof(T));
#define O1(EE, PP) \
  if (E == EE && P == PP) return go(k_outer_bwd<T, EE, PP>, grid, block, lds, s, a);
  O1(4, 1) O1(4, 2) O1(8, 1) O1(8, 2) O1(12, 1) O1(12, 2) O1(16, 1) O1(16, 2)
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

#define HD_INST(T) \
  template hipError_t launch_outer_fwd<T>(const OuterFwdArgs<T>&, int, int, int, hipStream_t); \
  template hipError_t launch_outer_bwd<T>(const OuterBwdArgs<T>&, int, int, hipStream_t); \
  template hipError_t launch_box_copy<T>(const BoxCopyArgs<T>&, hipStream_t);
HD_INST(float)
HD_INST(double)
#undef HD_INST

}  // namespace hd
