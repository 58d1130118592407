// hd_kcommon.hpp -- helpers shared by the kernel translation units.
#pragma once
#include <mutex>
#include <unordered_map>

#include "hd_engine.hpp"

namespace hd {

// Largest dynamic LDS size already granted to each kernel on this device, so
// the attribute call happens once per kernel (not inside captured graphs).
inline std::unordered_map<const void*, size_t>& lds_granted() {
  static std::unordered_map<const void*, size_t> m;
  return m;
}
inline std::mutex& lds_mutex() {
  static std::mutex mu;
  return mu;
}

extern __shared__ __align__(16) char hd_smem[];

template <typename T>
__device__ __forceinline__ cpx<T>* smem_as() {
  return reinterpret_cast<cpx<T>*>(hd_smem);
}

// Row exchange area: one pad slot every 2^ps points.
__host__ __device__ constexpr int row_pad(int m, int ps) { return m + (m >> ps); }

// LDS words (complex) of each kernel's exchange area; the transform's twiddle
// table follows it.
__host__ __device__ constexpr int xwords_rows(int m, int ps, int rows_per_block, int nt) {
  return rows_per_block * nt * row_pad(m, ps);
}
__host__ __device__ constexpr int xwords_cols(int p, int S, int nt) { return nt * p * S; }

// Hermitian rows store f_0 .. f_{Lh-1} of a centered array with
// f_{-c} = conj(f_c): the value at the signed index c (|c| < Lh), with the
// centre taken real.
template <typename T>
__device__ __forceinline__ cpx<T> herm_value(const cpx<T>* src, int64_t c) {
  cpx<T> v = src[c < 0 ? -c : c];
  if (c < 0) v.y = -v.y;
  if (c == 0) v.y = T(0);
  return v;
}

// The pointwise multiplication operator at point e: the product of the A
// transforms, or the quadratic form sum_{i <= j} c_ij F_i F_j.
template <typename T, int A, int E>
__device__ __forceinline__ cpx<T> mult_at(const cpx<T> (&w)[A][E], int e, const QuadMult<T>& q) {
  cpx<T> pr = w[0][e];
  if (!q.on) {
#pragma unroll
    for (int ai = 1; ai < A; ++ai) pr = cmul(pr, w[ai][e]);
    return pr;
  }
  pr = czero<T>();
#pragma unroll
  for (int i = 0; i < A; ++i)
#pragma unroll
    for (int j = i; j < A; ++j) pr = pr + cscale(cmul(w[i][e], w[j][e]), q.c[pair_slot(i, j)]);
  return pr;
}
// The same for two packed real transforms (Hermitian pairs): x parts and y
// parts separately.
template <typename T, int A, int E>
__device__ __forceinline__ cpx<T> mult_at_real_pair(const cpx<T> (&w)[A][E], int e, const QuadMult<T>& q) {
  T pa = w[0][e].x, pb = w[0][e].y;
  if (!q.on) {
#pragma unroll
    for (int ai = 1; ai < A; ++ai) {
      pa *= w[ai][e].x;
      pb *= w[ai][e].y;
    }
    return mk(pa, pb);
  }
  pa = T(0);
  pb = T(0);
#pragma unroll
  for (int i = 0; i < A; ++i)
#pragma unroll
    for (int j = i; j < A; ++j) {
      const T c = q.c[pair_slot(i, j)];
      pa += c * w[i][e].x * w[j][e].x;
      pb += c * w[i][e].y * w[j][e].y;
    }
  return mk(pa, pb);
}

// The operator at every point of a lane.  QUAD is a template parameter so
// that product kernels carry no code of the quadratic form.
template <bool QUAD, typename T, int A, int E>
__device__ __forceinline__ void mult_all(const cpx<T> (&w)[A][E], cpx<T> (&out)[1][E], const QuadMult<T>& q,
                                         bool real_pair) {
  if constexpr (!QUAD) {
    constexpr QuadMult<T> none{};
    if (real_pair) {
#pragma unroll
      for (int e = 0; e < E; ++e) out[0][e] = mult_at_real_pair(w, e, none);
    } else {
#pragma unroll
      for (int e = 0; e < E; ++e) out[0][e] = mult_at(w, e, none);
    }
  } else {
    if (real_pair) {
#pragma unroll
      for (int e = 0; e < E; ++e) out[0][e] = mult_at_real_pair(w, e, q);
    } else {
#pragma unroll
      for (int e = 0; e < E; ++e) out[0][e] = mult_at(w, e, q);
    }
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
  } else if (mode == ACC_OUT_ADD) {
    out[i] = out[i] + cscale(v, scale);
  } else {
    const double sx = acc[2 * i] + (double)v.x, sy = acc[2 * i + 1] + (double)v.y;
    out[i] = mk(T(sx * (double)scale), T(sy * (double)scale));
  }
}

template <typename K>
static hipError_t allow_lds(K kernel, size_t lds) {
  if (lds <= 65536) return hipSuccess;
  const void* key = reinterpret_cast<const void*>(kernel);
  std::lock_guard<std::mutex> lk(lds_mutex());
  auto it = lds_granted().find(key);
  if (it != lds_granted().end() && it->second >= lds) return hipSuccess;
  hipError_t e = hipFuncSetAttribute(key, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e == hipSuccess) lds_granted()[key] = lds;
  return e;
}

template <typename K, typename Args>
static hipError_t go(K kernel, dim3 grid, dim3 block, size_t lds, hipStream_t s, const Args& a) {
  hipError_t e = allow_lds(kernel, lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(kernel, grid, block, lds, s, a);
  return hipGetLastError();
}

#define HD_BAD hipErrorInvalidConfiguration

}  // namespace hd
