// hd_engine.hpp -- argument blocks and launchers of the hybrid-dealiasing
// HIP kernels.  Host code fills these structs from a plan; the kernels live in
// hd_k_fused.hip, hd_k_multi.hip and hd_k_outer.hip.
//
// Notation (Murasko & Bowman, arXiv 2303.17510): a dimension of length L is
// padded to at least M; m is the subtransform size, the input is explicitly
// padded to p*m and implicitly to q*m; zeta_N = exp(2 pi i/N).
//  * direct form (Algorithms 3-6, p <= 2): q residues r, each an m-point
//    FFT of W_s = sum_t zeta_{qm}^{r(tm+s)} f_{tm+s};
//  * inner form (Sec. 6.1, q = n p): n residues v of size p*m; the sum over t
//    becomes p-point DFTs of zeta_q^{vt} f_{tm+s}, then zeta_{qm}^{(un+v)s}
//    and an m-point FFT per u.
//  * centered dimensions (ctr = 1; the paper's centered case, eq. centDFT,
//    and its inner form): the array of L entries holds the signed indices
//    c = -H .. L-1-H (H = floor(L/2)) at positions c + H, and the transform
//    runs over c itself.  The p blocks then cover c in
//    [-tneg m, (p - tneg) m) with tneg = ceil(H/m); block t (0-based) holds
//    c = (t - tneg) m + s at array position t m + s - sh, sh = tneg m - H,
//    and the twiddle exponents use the signed c (r c mod q m).  In the inner
//    form the p-point column DFT takes block t = c div m at position t mod p,
//    with twiddle zeta_q^{v t}; when p is below the span (fold = 1) the
//    negative block t - p shares position t with block t (the paper's
//    p/2-term sum of the centered inner form), and the inverse hands the
//    value at position t to both output blocks, each with its own twiddle.
//    The inverse stores output c at position c + H, so the result is the
//    centered convolution.
//  * Hermitian rows (herm = 1; the paper's Hermitian symmetric case): L is the
//    full centered length 2 Lh - 1 and the arrays hold only f_0 .. f_{Lh-1};
//    a load of a negative index c reads conj(f_{-c}) (f_0 real), and only the
//    outputs c >= 0 are stored, at position c.
#pragma once
#include "hd_common.hpp"
#include "hd_fft.hpp"

namespace hd {

constexpr int kMaxA = 3;   // inputs one kernel launch combines
constexpr int kMaxIn = 6;  // inputs of a plan (quadratic operators; products take kMaxA)
constexpr int kMaxB = 8;   // outputs of a quadratic multiplication operator

// Quadratic multiplication operator (Sec. 2: mult maps the A transforms to B
// outputs pointwise): one launch's share of an output, H = sum_{i <= j}
// c_ij F_i F_j over the launch's (at most three) inputs, the pairs (0,0),
// (0,1), (0,2), (1,1), (1,2), (2,2) in slots 0 .. 5 (unused: 0).
template <typename T>
struct QuadMult {
  int on;     // 0: the product of the A transforms (B = 1)
  T c[6];
};
__host__ __device__ constexpr int pair_slot(int i, int j) { return i == 0 ? j : (i == 1 ? 2 + j : 5); }

// Accumulation of one residue block into the output (blocks of D residues):
//   ACC_WRITE : out  = sum * scale              (single block)
//   ACC_FIRST : acc  = sum                      (first of several blocks)
//   ACC_ADD   : acc += sum
//   ACC_LAST  : out  = (acc + sum) * scale      (last block)
//   ACC_OUT_ADD: out += sum * scale             (later residue blocks of the
//                first outer dimension, accumulated in the output itself)
// acc is an FP64 buffer laid out like out.
enum AccMode { ACC_WRITE = 0, ACC_FIRST = 1, ACC_ADD = 2, ACC_LAST = 3, ACC_OUT_ADD = 4 };

// One independent 1D convolution of a batched plan: its own inputs, output
// and length (all rows of a launch share m, p, q).
template <typename T>
struct RowTask {
  const cpx<T>* in[kMaxA];
  cpx<T>* out;
  int64_t L;
};

// Whole 1D convolutions along contiguous rows, direct form with p <= 2.
// One group of G lanes per row; rows_per_block rows per workgroup.  When
// `tasks` is set, row i takes its pointers and length from tasks[i] instead
// of in/out/L and the strides.
template <typename T>
struct FusedArgs {
  const RowTask<T>* tasks;
  const cpx<T>* in[kMaxA];
  cpx<T>* out;
  int64_t in_stride, out_stride;  // elements between consecutive rows
  int64_t nrows;
  int64_t L;
  int m, q;
  int rows_per_block;
  int ctr;   // 1: centered rows (H = floor(L/2) of each row's own L)
  int herm;  // 1: Hermitian rows (half storage, see above)
  int pair;  // 1: Hermitian rows transform two residues per complex transform
  QuadMult<T> quad;  // multiplication operator of the output this launch computes
  int out_add;       // quadratic operators: add to the output (later shares of one output)
  T scale;  // 1/(q m)
  FftDesc fd;
  const cpx<T>* fft_tw;  // two-level table of zeta for fd.N (lo then hi)
  RootTable<T> zqm;  // powers of zeta_{qm}
};

// Whole rows of one block (p = 1), product operator, dense rows: the lean
// row kernel for launches over many rows (hd_k_lean.hip).
template <typename T>
struct LeanRowArgs {
  const cpx<T>* in[kMaxA];
  cpx<T>* out;
  int64_t in_stride, out_stride;  // elements between consecutive rows
  int64_t nrows;
  uint32_t L;  // row length (<= m)
  int q;       // residues
  T scale;     // 1/(q m)
  FftDesc fd;  // m points (the kernel reads its per-stage twiddle tables)
  const cpx<T>* fft_tw;
  RootTable<T> zqm;  // powers of zeta_{qm}
};

// Inner form, pass 1: for a tile of S consecutive columns s of the p x m
// view f_{tm+s} of each row, the p-point DFT over t of zeta_q^{vt} f_{tm+s}
// for residues v0 .. v0+D-1.  Output work[a][(row D + dv) p + u][s].
template <typename T>
struct ColFwdArgs {
  const RowTask<T>* tasks;  // batched plans: per-row inputs and length
  const cpx<T>* in[kMaxA];
  cpx<T>* work[kMaxA];
  int64_t in_stride;
  int64_t nrows;
  int64_t L;
  int m, p, q, v0, D, S;
  int ctr;   // 1: centered rows
  int fold;  // 1: two blocks per column position (centered, p below the span)
  int herm;  // 1: Hermitian rows
  int pair;  // 1: residues v and n - v taken together (conjugate symmetry; block of all n residues)
  FftDesc fd;  // p points
  const cpx<T>* fft_tw;  // two-level table of zeta for fd.N (lo then hi)
  const cpx<T>* zq;  // zeta_q^k, k < q
};

// Inner form, pass 2: per row (v,u): pre-twiddle zeta_{qm}^{(un+v)s}, m-point
// FFT of each input, pointwise product, inverse FFT, post-twiddle; the result
// replaces work[0]'s row.
template <typename T>
struct RowConvArgs {
  cpx<T>* work[kMaxA];
  cpx<T>* out;  // result rows (nullptr: in place, over work[0])
  QuadMult<T> quad;
  int64_t nrows;  // rows of the work buffer (= batch * D * p)
  int m, p, n, v0, D;
  int rows_per_block;
  int herm;  // 1: Hermitian plan transforming two (real-output) rows per slot
  int64_t qm;
  FftDesc fd;  // m points
  const cpx<T>* fft_tw;  // two-level table of zeta for fd.N (lo then hi)
  RootTable<T> zqm;
};

// Inner form, pass 3: p-point inverse DFT over u of each column, times
// zeta_q^{-vt}, accumulated over the block's residues, scaled by 1/(qm) and
// truncated to L.
template <typename T>
struct ColBwdArgs {
  const RowTask<T>* tasks;  // batched plans: per-row output and length
  const cpx<T>* work;
  cpx<T>* out;
  double* acc;  // FP64 accumulator (interleaved), for multi-block plans
  int acc_mode;
  int64_t out_stride;
  int64_t nrows;
  int64_t L;
  int m, p, q, v0, D, S;
  int ctr;   // 1: centered rows
  int fold;  // 1: two blocks per column position (centered, p below the span)
  int herm;  // 1: Hermitian rows
  T scale;
  FftDesc fd;  // p points
  const cpx<T>* fft_tw;  // two-level table of zeta for fd.N (lo then hi)
  const cpx<T>* zq;
};

// Outer dimension of a multidimensional convolution (Sec. 5), direct form:
// data viewed as [nb][L][R] (R contiguous columns).  Forward writes, for
// residues r0 .. r0+D-1, out[a][((b D + dr) m + l) R + c].
// Layout of the user's array in the first outer pass: element (j, col) of a
// plane is at j jstride + (col / cgrp) cgstride + col % cgrp (all zero: dense,
// j R + col).  Strided 2D/3D layouts set it; the level buffers are dense.
struct ColLayout {
  int64_t jstride, cgrp, cgstride;
};

template <typename T>
struct OuterFwdArgs {
  const cpx<T>* in[kMaxA];
  cpx<T>* out[kMaxA];
  ColLayout lay;  // of in
  int64_t nb, in_bstride, R;
  int64_t L;
  int m, q, r0, D, S;
  int ctr;  // 1: centered dimension
  FftDesc fd;
  const cpx<T>* fft_tw;  // two-level table of zeta for fd.N (lo then hi)
  RootTable<T> zqm;
};

template <typename T>
struct OuterBwdArgs {
  const cpx<T>* y;  // [nb][D][m][R]
  cpx<T>* out;      // out[b * out_bstride + x R + c], x < L (or as lay says)
  ColLayout lay;    // of out
  double* acc;
  int acc_mode;
  int64_t nb, out_bstride, R;
  int64_t L;
  int m, q, r0, D, S;
  int ctr;  // 1: centered dimension
  T scale;
  FftDesc fd;
  const cpx<T>* fft_tw;  // two-level table of zeta for fd.N (lo then hi)
  RootTable<T> zqm;
};

// Outer dimension, direct form with one block, dense planes: the lean outer
// kernel (hd_k_lean.hip).  Forward: in[a] -> out[a] (level buffers) for the
// na inputs of the launch; backward: in[0] (the level buffer) -> out[0].
template <typename T>
struct OuterLeanArgs {
  const cpx<T>* in[kMaxA];
  cpx<T>* out[kMaxA];
  int na;                           // forward: inputs of this launch
  int64_t nb;                       // planes
  int64_t in_bstride, out_bstride;  // words between planes of the user-side array (fwd: in, bwd: out)
  int64_t R;                        // columns per plane (contiguous)
  uint32_t L;                       // length of the transformed dimension (<= m)
  int q;                            // residues
  int r0, D;                        // residues r0 .. r0+D-1 of this launch (level planes b D + dr)
  int add;                          // backward: add to the output (later residue blocks)
  T scale;                          // backward: 1/(q m)
  FftDesc fd;                       // m points (the kernel reads its per-stage twiddle tables)
  const cpx<T>* fft_tw;
  RootTable<T> zqm;
  int inner_n;  // 0: direct form; n: the inner form's m-point pass (plane b is row j = b mod q of its
                // convolution, residue (j mod p) n + j div p, p = q / n; D = 1, in place)
};

// Outer dimension in the inner form (Sec. 6.1 with Sec. 5), column passes,
// dense planes [nb][L][R]:
//   forward:  out[a][((b q + v p + u) m + s) R + c] = sum_t zeta_p^{ut} zeta_q^{vt} in[a][b][t m + s][c]
//   backward: out[b][t m + s][c] (+)= scale sum_v zeta_q^{-vt} sum_u zeta_p^{-ut} in[0][((b q + v p + u) m + s) R + c]
// (the m-point transforms between them run on the lean outer kernel).
template <typename T>
struct OuterColArgs {
  const cpx<T>* in[kMaxA];
  cpx<T>* out[kMaxA];
  int na;                           // forward: inputs of this launch
  int64_t nb;                       // planes
  int64_t in_bstride, out_bstride;  // words between planes of the user-side array (fwd: in, bwd: out)
  int64_t R;                        // columns per plane (contiguous)
  int64_t L;                        // length of the dimension (<= p m)
  int m, n;                         // block length, residue blocks (q = n p)
  int add;                          // backward: add to the output
  T scale;                          // backward: 1/(q m)
  FftDesc fd;                       // p points (per-stage twiddle tables follow the two-level one)
  const cpx<T>* fft_tw;
  const cpx<T>* zq;                 // zeta_q^k, k < q
};

// Zero padding / truncation copies between a dense box L[0..2] and a dense
// box N[0..2] (the explicit method's materialised padding).
template <typename T>
struct BoxCopyArgs {
  const cpx<T>* src;
  cpx<T>* dst;
  int64_t L[3], N[3];  // leading unused extents are 1
  int64_t ls[2];       // element strides of the L box's first two axes (0: dense)
  int64_t off[3];      // truncation: dst[i] = src[i + off] (0, or the centered window start)
  int pad;             // 1: dst (N box) <- src (L box) with zeros; 0: dst (L box) <- src (N box)
  int herm;            // padding of a Hermitian array (stored box L, last axis c = 0 .. hH):
  int64_t hH;          // the expanded centered box, F(k, -c) = conj F(-k, c)
};

// Persistent batched execution (hd_k_batch.hip): launches of resident
// workgroups over device task tables.  Convolutions of one size bucket share
// a shape: whole rows (direct form, p = 1, the lean row body) or the inner
// form (Sec. 6.1: column pass, row pass, back pass, each task a range of
// units of one convolution); one launch per pass.
constexpr int kBatchThreads = 256;  // threads of the persistent workgroup
enum BatchKind { BK_ROWS = 0, BK_COLF = 1, BK_ROWP = 2, BK_COLB = 3 };

template <typename T>
struct BatchBucket {
  int inner;        // 0: whole rows; 1: inner form
  int body;         // compiled body of the bucket's shape (hd_k_batch.hip)
  int m, p, n, q;   // shape shared by the bucket's convolutions (D = n)
  int S;            // inner form: columns per column-pass unit
  T scale;          // 1/(q m)
  const cpx<T>* tw_m;  // per-stage twiddles of the m-point transform
  const cpx<T>* tw_p;  // per-stage twiddles of the p-point transform (inner form)
  int ntw_m, ntw_p;    // their words
  const cpx<T>* zq;    // zeta_q^k, k < q (inner form)
  RootTable<T> zqm;    // powers of zeta_{qm}
  const RowTask<T>* rows;  // per convolution: inputs, output, length
  cpx<T>* work[kMaxA];     // inner form: input a of convolution c, row j = v p + u, at work[a][(c q + j) m]
};

struct BatchTask {
  int bucket, kind;  // BatchKind
  int conv;          // whole rows: first convolution of the task; else the convolution
  int u0, nu;        // units [u0, u0 + nu): rows (whole rows, row pass), (input, column tile) or column tiles
};

template <typename T>
struct BatchArgs {
  const BatchBucket<T>* buckets;
  const BatchTask* tasks;  // this launch's table
  int ntasks;
  int xwords;  // LDS words of the largest exchange area (the tables follow)
};

// Launchers (return the launch status).  E, P and A select the template
// instance; the host checks that the plan's geometry fits before calling.
template <typename T>
hipError_t launch_fused1d(const FusedArgs<T>& a, int E, int P, int A, hipStream_t s);
template <typename T>
hipError_t launch_rows_lean(const LeanRowArgs<T>& a, int E, int A, int cus, hipStream_t s);
template <typename T>
hipError_t launch_outer_lean(const OuterLeanArgs<T>& a, int E, int S, bool fwd, int cus, hipStream_t s);
// Sizes, points per lane and columns per workgroup the lean outer kernel is
// built for (tbytes: bytes of a real word); inner: the inner form's m-point
// pass (any q).
bool outer_lean_supported(int m, int E, int S, int q, int tbytes, bool inner = false);
// The column passes of an outer dimension in the inner form.
template <typename T>
hipError_t launch_outer_cols(const OuterColArgs<T>& a, int p, bool fwd, int cus, hipStream_t s);
bool outer_cols_supported(int p, int E, int tbytes);
// Sizes, points per lane, input and residue counts the lean row kernel is
// built for.
constexpr int kLeanMaxQ = 8;
bool rows_lean_supported(int m, int E, int A, int q, int tbytes);
template <typename T>
hipError_t launch_cols_fwd(const ColFwdArgs<T>& a, int E, int A, hipStream_t s);
template <typename T>
hipError_t launch_rows_conv(const RowConvArgs<T>& a, int E, int A, hipStream_t s);
template <typename T>
hipError_t launch_cols_bwd(const ColBwdArgs<T>& a, int E, hipStream_t s);
template <typename T>
hipError_t launch_outer_fwd(const OuterFwdArgs<T>& a, int E, int P, int A, hipStream_t s);
template <typename T>
hipError_t launch_outer_bwd(const OuterBwdArgs<T>& a, int E, int P, hipStream_t s);
template <typename T>
hipError_t launch_box_copy(const BoxCopyArgs<T>& a, hipStream_t s);
// The persistent batched kernel for A inputs with `grid` workgroups and
// `lds` bytes of LDS.  batch_shape() names the compiled body of a bucket
// shape (false: none) and the points per lane and columns it uses;
// batch_lds_words() its LDS words (exchange area, tables of its largest
// kind); batch_grid_t() the resident workgroups of the instance on `cus`
// compute units.
template <typename T>
hipError_t launch_batch(const BatchArgs<T>& a, int A, int grid, size_t lds, hipStream_t s);
bool batch_shape(int inner, int64_t m, int64_t p, int tbytes, int* body, int* E_m, int* E_p, int* S);
void batch_lds_words(int body, int m, int p, int q, int ntw_m, int ntw_p, int tbytes, int* xwords, int* twords);
template <typename T>
int batch_grid_t(int A, size_t lds, int cus);

// LDS bytes each launcher requests (host-side sizing and validation).
size_t lds_fused1d(int m, int ps, int rows_per_block, int A, int ntw, int tbytes);
size_t lds_cols(int p, int S, int ntw, int tbytes);
size_t lds_rows(int m, int ps, int rows_per_block, int A, int ntw, int tbytes);
size_t lds_outer(int m, int S, int ntw, int tbytes);

// True when the radix set of d fits the template instance E.
bool fft_fits(const FftDesc& d, int E);

}  // namespace hd
