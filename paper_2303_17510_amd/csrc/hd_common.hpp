// hd_common.hpp -- complex arithmetic and small helpers shared by the HIP
// kernels of the hybrid-dealiasing engine (device and host).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace hd {

template <typename T>
struct cpx {
  T x, y;
};

template <typename T>
__device__ __host__ __forceinline__ cpx<T> mk(T a, T b) {
  cpx<T> r;
  r.x = a;
  r.y = b;
  return r;
}
template <typename T>
__device__ __host__ __forceinline__ cpx<T> operator+(cpx<T> a, cpx<T> b) {
  return mk(a.x + b.x, a.y + b.y);
}
template <typename T>
__device__ __host__ __forceinline__ cpx<T> operator-(cpx<T> a, cpx<T> b) {
  return mk(a.x - b.x, a.y - b.y);
}
// a * b
template <typename T>
__device__ __host__ __forceinline__ cpx<T> cmul(cpx<T> a, cpx<T> b) {
  return mk(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
// a * conj(b)
template <typename T>
__device__ __host__ __forceinline__ cpx<T> cmulc(cpx<T> a, cpx<T> b) {
  return mk(a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y);
}
template <typename T>
__device__ __host__ __forceinline__ cpx<T> cscale(cpx<T> a, T s) {
  return mk(a.x * s, a.y * s);
}
// a * (S i), S = +1 or -1
template <int S, typename T>
__device__ __forceinline__ cpx<T> mul_si(cpx<T> a) {
  return S > 0 ? mk(-a.y, a.x) : mk(a.y, -a.x);
}
// a * w when S = +1, a * conj(w) when S = -1
template <int S, typename T>
__device__ __forceinline__ cpx<T> cmul_s(cpx<T> a, cpx<T> w) {
  return S > 0 ? cmul(a, w) : cmulc(a, w);
}
template <typename T>
__device__ __forceinline__ cpx<T> czero() {
  return mk(T(0), T(0));
}

// Two-level table of the powers of one root of unity:
//   zeta_N^e = lo[e & (K-1)] * hi[e >> kbits],  0 <= e < N,  K = 2^kbits.
// Both halves are rounded from FP64 values, so an entry is within about two
// ulps of the exact root.
// Loads and stores at a 32-bit byte offset from a base pointer: with a
// wave-uniform base the address is one scalar pair plus one vector register,
// instead of a 64-bit vector address per access.
template <typename T>
__device__ __forceinline__ cpx<T> ld_at(const cpx<T>* base, uint32_t idx) {
  return *(const cpx<T>*)((const char*)base + idx * (uint32_t)sizeof(cpx<T>));
}
template <typename T>
__device__ __forceinline__ void st_at(cpx<T>* base, uint32_t idx, cpx<T> v) {
  *(cpx<T>*)((char*)base + idx * (uint32_t)sizeof(cpx<T>)) = v;
}

// Offsets passed to ld_at/st_at are positions within one row of at most
// 2 * 8192 points (or a table of at most ~2^16 entries), so their byte
// offsets stay far below 2^32; the planner keeps q m below 2^31, so
// twiddle exponents reduced mod q m fit 32 bits.
template <typename T>
struct RootTable {
  const cpx<T>* lo;
  const cpx<T>* hi;
  int64_t N;
  int kbits;
  __device__ __forceinline__ cpx<T> get(int64_t e64) const {
    const uint32_t e = (uint32_t)e64;
    return cmul(ld_at(lo, e & ((1u << kbits) - 1)), ld_at(hi, e >> kbits));
  }
  // zeta_N^{(a*b) mod N} for non-negative a, b with a*b < 2^63
  __device__ __forceinline__ cpx<T> pow_prod(int64_t a, int64_t b) const {
    return get((int64_t)((uint64_t)(a * b) % (uint64_t)N));
  }
  // Calls f(e, zeta_N^{ex0 + e st}) for e = 0 .. E-1 (ex0, st < N).  The
  // powers are composed from three lookups: base = zeta^{ex0}, w = zeta^{st}
  // and w4 = zeta^{4 st}, with zeta^{e st} = w^{e mod 4} w4^{e div 4}
  // (E <= 16), so each value is a product of at most five rounded factors
  // instead of two table loads per point.
  template <int E, typename F>
  __device__ __forceinline__ void run(uint32_t ex0, uint32_t st, F&& f) const {
    static_assert(E <= 16, "at most 16 powers per run");
    const cpx<T> base = get(ex0);
    cpx<T> p0[4], p1[4];
    p0[0] = p1[0] = mk(T(1), T(0));
    p0[1] = get(st);
    p0[2] = cmul(p0[1], p0[1]);
    p0[3] = cmul(p0[2], p0[1]);
    if constexpr (E > 4) {
      p1[1] = get((uint32_t)((4ull * st) % (uint64_t)N));
      p1[2] = cmul(p1[1], p1[1]);
      p1[3] = cmul(p1[2], p1[1]);
    }
#pragma unroll
    for (int e = 0; e < E; ++e) {
      cpx<T> z = base;
      if (e & 3) z = cmul(z, p0[e & 3]);
      if (e >> 2) z = cmul(z, p1[e >> 2]);
      f(e, z);
    }
  }
};

}  // namespace hd
