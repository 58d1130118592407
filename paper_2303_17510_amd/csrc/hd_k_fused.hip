// hd_k_fused.hip -- whole 1D convolutions per row, direct form (p <= 2).
// The convolution is bandwidth-bound, so no kernel uses matrix cores: every
// kernel streams its operands through registers once, runs its transforms
// with LDS exchanges (hd_fft.hpp) and writes its result once.  Global loads
// and stores are coalesced: consecutive lanes touch consecutive complex words.
#include "hd_kcommon.hpp"

namespace hd {

// ---------------------------------------------------------------------------
// Whole 1D convolution of one contiguous row per lane group, direct form
// (Algorithms 1, 3-6): for each residue r < q,
//   W_s   = sum_{t<P} zeta_{qm}^{r(tm+s)} f_{tm+s}      (zero where tm+s >= L)
//   F     = fft_m(W) per input;  H = prod_a F_a         (mult, B = 1)
//   h_j  += zeta_{qm}^{-rj} ifft_m(H)_{j mod m}          (j = tm+s < L)
// and finally out_j = h_j / (qm).  With P = 2 the backward step is the
// corrected form of Algorithm 6 (the second half carries zeta_{qm}^{-rj},
// j = m+s, as eq. invStan requires).  The A forward transforms of a residue
// run together (shared twiddles and barriers).  Centered rows (a.ctr, the
// paper's centered case with p = 2, eq. forCent/wDef): block t holds the
// signed indices c = (t - tneg) m + s at array position t m + s - sh, and the
// twiddles are zeta_{qm}^{r c}; the output c goes back to position c + H.
template <typename T, int E, int P, int A, bool HERM, bool QUAD>
__global__ void __launch_bounds__(512) k_fused1d(FusedArgs<T> a) {
  // Inputs small enough stay in registers across the residues; larger ones
  // are read again for each residue (from cache) to keep registers free.
  constexpr bool kKeep = P * A * E <= 8;
  const int G = a.fd.G;
  const int m = a.m;
  const int slot = threadIdx.x / G;
  const int g = threadIdx.x - slot * G;
  const int64_t row = (int64_t)blockIdx.x * a.rows_per_block + slot;
  const bool valid = row < a.nrows;
  // per-row pointers and length: from the task table (batched plans) or strided rows
  const RowTask<T>* tk = (a.tasks && valid) ? a.tasks + row : nullptr;
  const uint32_t L = valid ? (uint32_t)(tk ? tk->L : a.L) : 0u;
  const uint32_t qm = (uint32_t)a.q * (uint32_t)m;
  // centered rows: tneg blocks left of index 0, block position j holds array
  // position j - sh (both 0 for an ordinary row; a centered row spans two
  // blocks unless L = 1, so P = 1 never shifts)
  const uint32_t H = (P == 2 && a.ctr) ? (L >> 1) : 0u;
  const uint32_t tneg = H ? (H + (uint32_t)m - 1) / (uint32_t)m : 0u;
  const uint32_t sh = tneg * (uint32_t)m - H;
  const cpx<T>* src[A];
#pragma unroll
  for (int ai = 0; ai < A; ++ai) src[ai] = tk ? tk->in[ai] : a.in[ai] + row * a.in_stride;
  cpx<T>* lds = smem_as<T>();
  Xchg<T> xb{lds + (size_t)slot * A * row_pad(m, a.fd.ps), 1, a.fd.ps, row_pad(m, a.fd.ps)};
  const TwLds<T> tw = stage_table(a.fd, a.fft_tw, lds + xwords_rows(m, a.fd.ps, a.rows_per_block, A));

  // the row's inputs (zero beyond L; Hermitian rows mirror the stored half,
  // and a one-block Hermitian row is the lone real centre, L = 1).  HERM is a
  // template parameter: the mirror sits in the residue loop when the inputs
  // are re-read there, and ordinary rows must not pay its registers.
  constexpr bool herm = HERM;
  auto load = [&](int ai, int t, int e) -> cpx<T> {
    const uint32_t i = (uint32_t)(t * m + g + G * e) - sh;  // wraps above L when j < sh
    if (!(i < L)) return czero<T>();
    return herm ? herm_value(src[ai], (int64_t)i - (int64_t)H) : ld_at(src[ai], i);
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
  __syncthreads();

  cpx<T> acc[P][E];
#pragma unroll
  for (int t = 0; t < P; ++t)
#pragma unroll
    for (int e = 0; e < E; ++e) acc[t][e] = czero<T>();

  // Residue twiddle exponents without division: r g and r G stay below qm
  // (r < q, g < G <= m).  Block t starts at the signed index
  // c = (t - tneg) m + g, whose exponent is r g + m ((r (t - tneg)) mod q),
  // with t - tneg in {-1, 0, 1} (P <= 2).
  auto ex_of = [&](int r, int t) -> uint32_t {
    const int d = t - (int)tneg;
    const uint32_t rm = (uint32_t)r * (uint32_t)m;
    const uint32_t add = d == 0 ? 0u : (d > 0 ? rm : (r ? qm - rm : 0u));
    const uint32_t e = (uint32_t)r * (uint32_t)g + add;
    return e >= qm ? e - qm : e;
  };
  // Hermitian rows: every residue transform is real (the paper's
  // complex-to-real residue DFTs), so two residues r, r+1 share one complex
  // transform per input: z = W_r + i W_{r+1} gives F_r = Re Z and
  // F_{r+1} = Im Z; the products go back packed as P_r + i P_{r+1}, whose
  // inverse Y splits by conjugate symmetry, y_r(s) = (Y(s) + conj Y(-s)) / 2
  // and y_{r+1}(s) = (Y(s) - conj Y(-s)) / (2i).  Half the transforms.
  for (int r = 0; r < a.q;) {
    const bool pair = HERM && a.pair && r + 1 < a.q;  // uniform
    cpx<T> w[A][E];
#pragma unroll
    for (int ai = 0; ai < A; ++ai)
#pragma unroll
      for (int e = 0; e < E; ++e) w[ai][e] = czero<T>();
    auto gather = [&](int rr, bool times_i) {
#pragma unroll
      for (int t = 0; t < P; ++t) {
        a.zqm.template run<E>(ex_of(rr, t), (uint32_t)rr * (uint32_t)G, [&](int e, cpx<T> z) {
#pragma unroll
          for (int ai = 0; ai < A; ++ai) {
            cpx<T> xv;
            if constexpr (kKeep) xv = x[ai][t][e];
            else xv = load(ai, t, e);
            const cpx<T> v = cmul(xv, z);
            w[ai][e] = w[ai][e] + (times_i ? mk(-v.y, v.x) : v);
          }
        });
      }
    };
    gather(r, false);
    if constexpr (HERM)
      if (pair) gather(r + 1, true);
    gfft_any<T, E, +1, A, (A == 2 ? kCtFused : 0u)>(w, g, a.fd, tw, xb);
    cpx<T> prod[1][E];
    mult_all<QUAD>(w, prod, a.quad, HERM && pair);
    gfft_any<T, E, -1, 1, (A == 2 ? kCtFused : 0u)>(prod, g, a.fd, tw, xb);
    if constexpr (HERM) {
      if (pair) {
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
        __syncthreads();
        cpx<T> y1[E];
#pragma unroll
        for (int e = 0; e < E; ++e) {
          const cpx<T> yv = prod[0][e];
          // y_r = (Y + conj Ym) / 2,  y_{r+1} = -i (Y - conj Ym) / 2
          prod[0][e] = mk(T(0.5) * (yv.x + ym[e].x), T(0.5) * (yv.y - ym[e].y));
          y1[e] = mk(T(0.5) * (yv.y + ym[e].y), T(0.5) * (ym[e].x - yv.x));
        }
#pragma unroll
        for (int t = 0; t < P; ++t)
          a.zqm.template run<E>(ex_of(r + 1, t), (uint32_t)(r + 1) * (uint32_t)G,
                                [&](int e, cpx<T> z) { acc[t][e] = acc[t][e] + cmulc(y1[e], z); });
      }
    }
#pragma unroll
    for (int t = 0; t < P; ++t)
      a.zqm.template run<E>(ex_of(r, t), (uint32_t)r * (uint32_t)G,
                            [&](int e, cpx<T> z) { acc[t][e] = acc[t][e] + cmulc(prod[0][e], z); });
    r += pair ? 2 : 1;
  }
  if (valid) {
    cpx<T>* dst = tk ? tk->out : a.out + row * a.out_stride;
#pragma unroll
    for (int t = 0; t < P; ++t)
#pragma unroll
      for (int e = 0; e < E; ++e) {
        const uint32_t i = (uint32_t)(t * m + g + G * e) - sh;
        // Hermitian rows keep the outputs c = i - H >= 0, at c
        const uint32_t o = herm ? i - H : i;
        if (i < L && (!herm || i >= H)) {
          cpx<T> v = cscale(acc[t][e], a.scale);
          if constexpr (QUAD)
            if (a.out_add) v = v + ld_at(dst, o);
          st_at(dst, o, v);
        }
      }
  }
}


#if !defined(HD_PART) || HD_PART == 1  // host helpers, in one object only
size_t lds_fused1d(int m, int ps, int rows_per_block, int A, int ntw, int tbytes) {
  return ((size_t)xwords_rows(m, ps, rows_per_block, A) + ntw) * 2 * tbytes;
}
size_t lds_rows(int m, int ps, int rows_per_block, int A, int ntw, int tbytes) {
  return ((size_t)xwords_rows(m, ps, rows_per_block, A) + ntw) * 2 * tbytes;
}
size_t lds_cols(int p, int S, int ntw, int tbytes) { return ((size_t)xwords_cols(p, S, 2) + ntw) * 2 * tbytes; }
size_t lds_outer(int m, int S, int ntw, int tbytes) { return ((size_t)xwords_cols(m, S, 1) + ntw) * 2 * tbytes; }

bool fft_fits(const FftDesc& d, int E) {
  if ((int64_t)d.G * E != d.N) return false;
  for (int i = 0; i < d.nst; ++i)
    if (E % d.radix[i] != 0) return false;
  return true;
}
#endif

template <typename T>
hipError_t launch_fused1d(const FusedArgs<T>& a, int E, int P, int A, hipStream_t s) {
  const int nt = a.fd.G * a.rows_per_block;
  if (nt > 512 || !fft_fits(a.fd, E) || a.m != a.fd.N) return HD_BAD;
  dim3 grid((unsigned)((a.nrows + a.rows_per_block - 1) / a.rows_per_block)), block(nt);
  const size_t lds = lds_fused1d(a.m, a.fd.ps, a.rows_per_block, A, tw_words(a.fd), sizeof(T));
#define F2(EE, PP, AA, QQ)                                                                 \
  return a.herm ? go(k_fused1d<T, EE, PP, AA, true, QQ>, grid, block, lds, s, a)           \
                : go(k_fused1d<T, EE, PP, AA, false, QQ>, grid, block, lds, s, a);
#define F1(EE, PP, AA)                  \
  if (E == EE && P == PP && A == AA) {  \
    if (a.quad.on) F2(EE, PP, AA, true) \
    F2(EE, PP, AA, false)               \
  }
  F1(4, 1, 2) F1(4, 2, 2) F1(4, 1, 3) F1(4, 2, 3)
  F1(8, 1, 2) F1(8, 2, 2) F1(8, 1, 3) F1(8, 2, 3)
  F1(12, 1, 2) F1(12, 2, 2) F1(12, 1, 3) F1(12, 2, 3)
  F1(16, 1, 2) F1(16, 2, 2) F1(16, 1, 3) F1(16, 2, 3)
#undef F1
#undef F2
  return HD_BAD;
}

#define HD_INST(T) \
  template hipError_t launch_fused1d<T>(const FusedArgs<T>&, int, int, int, hipStream_t);
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
