// hd_plan.hpp -- host-side planning of a hybrid-dealiased convolution.
// Integer logic only; no device calls (usable without a GPU).
#pragma once
#include <stdint.h>

#include <string>
#include <vector>

#include "hd_fft.hpp"

namespace hd {

enum Variant {
  VAR_AUTO = 0,
  VAR_FUSED = 1,  // whole 1D convolution per row, direct form (p <= 2)
  VAR_MULTI = 2,  // inner-loop form, three passes over HBM
  VAR_OUTER = 3   // outer dimension of a multidimensional convolution: direct form (p <= 2)
                  // or the inner form (p > 2)
};

// Limits of the kernels (hd_k_fused.hip, hd_k_multi.hip, hd_k_outer.hip).
constexpr int kMaxThreads = 512;
constexpr int64_t kMaxFusedM = 8192;   // m of the fused and outer kernels
constexpr int64_t kMaxRowM = 8192;     // m of the row-convolution pass
constexpr int64_t kMaxColP = 4096;     // p of the column passes
constexpr size_t kLdsBudget = 160 * 1024;

struct DimPlan {
  int64_t L = 0, M = 0;       // lengths the engine sees in this dimension
  int64_t m = 0, p = 0, n = 0, q = 0, D = 0;
  int variant = VAR_AUTO;
  FftDesc fd_m{};             // m-point transform
  int E_m = 0;
  FftDesc fd_p{};             // p-point transform of the forward column pass (inner form)
  int E_p = 0;
  FftDesc fd_pb{};            // the same transform as the backward column pass runs it
  int E_pb = 0;               // (FP32: at most 8 points per lane there, see finish_dim)
  int S = 0;                  // columns per workgroup (column / outer kernels)
  int rows_per_block = 0;     // rows per workgroup (fused / row kernels)
  int tw_pref = 0;            // twiddles: 0 choose, 1 two-level table, 2 per-stage tables
  int ctr = 0;                // 1: centered convolution (indices -H .. L-1-H, H = floor(L/2))
  int herm = 0;               // 1: Hermitian rows: L = 2 Lh - 1 is the full centered length, the
                              // arrays hold f_0 .. f_{Lh-1} (f_{-c} = conj f_c); implies ctr
};

// Blocks of m points a centered dimension spans (the centered transform of
// the paper's one-dimensional centered case): the signed indices -H .. L-1-H
// lie in blocks -ceil(H/m) .. ceil((L-H)/m)-1, so p is at least
// ceil(H/m) + ceil((L-H)/m) (2 whenever m >= L/2 and L >= 2).
int64_t centered_blocks(int64_t L, int64_t m);
// Blocks of the non-negative indices 0 .. L-1-H: ceil((L-H)/m).
int64_t centered_pos_blocks(int64_t L, int64_t m);
// True when an inner-form centered dimension folds two blocks onto one
// column position (p below the full span centered_blocks(L, m)).
bool centered_folds(const struct DimPlan& dp);

// Least M for which a centered product of A inputs is not aliased: the
// index sums of A inputs span -A H .. A(L-1-H), and an output index c in
// -H .. L-1-H must not meet another sum congruent to it modulo q m.
int64_t centered_min_padding(int64_t L, int A);

// Paper's geometry rules for a given m (Algorithm 1, Sec. 2.1, Sec. 6.1):
//   p = ceil(L/m) (or the caller's larger p_min), then
//   p <= 2 (direct):  q = n = ceil(M/m), residues of size m;
//   p  > 2 (inner):   n = ceil(M/(p m)), q = n p, residues of size p m.
struct Geometry {
  int64_t m, p, n, q;
  bool inner;
};
Geometry geometry(int64_t L, int64_t M, int64_t m, int64_t p_min, bool force_inner);

// The same rules for a centered dimension (ctr = 1; the paper's centered case
// and its inner form): the direct form spans p = ceil(H/m) + ceil((L-H)/m)
// blocks (p <= 2, q = n = ceil(M/m)); the inner form folds the blocks of
// negative indices onto the column positions of the positive ones (the
// paper's padded DFT of p/2 terms in the centered inner form), so p only has
// to reach ceil((L-H)/m), and n = ceil(M/(p m)), q = n p.  ctr = 0 is
// geometry().
Geometry geometry_c(int64_t L, int64_t M, int64_t m, int64_t p_min, bool force_inner, int ctr);

bool fft_size_ok(int64_t N);            // 2^a, or 3 * 2^a with a >= 3
int64_t next_fft_size(int64_t n);       // smallest size >= n accepted by fft_size_ok
bool col_size_ok(int64_t p);            // 2^a, or 3 * 2^a with a >= 2
int64_t next_col_size(int64_t n);       // smallest p >= n the column passes accept

// Factor N into stage radices that divide E (largest first; a factor 3 first).
// Returns false when impossible.
bool make_fft_desc(int64_t N, int E, FftDesc* d);

// Points per lane of an outer dimension's column transforms in the inner form.
int outer_col_e(int p, int tbytes);

// Choose template widths, tiles and rows per block for a dimension whose
// (m, p, n, q, variant) are set.  tbytes = sizeof(real).  On failure returns
// false with a reason.
bool finish_dim(DimPlan* dp, int A, int tbytes, std::string* why);

// Default (heuristic) choice for one dimension.  `contiguous` marks the
// innermost dimension (rows), others are outer dimensions; `lines` is the
// number of independent lines one launch of this dimension processes (1 for
// a single 1D convolution: latency first; many: throughput first).
// `ctr` selects the centered convolution; `dims` is the plan's dimension
// count (the outer-dimension rules differ between 2D and 3D).
bool choose_dim(int64_t L, int64_t M, int A, int tbytes, bool contiguous, int64_t lines, DimPlan* dp,
                std::string* why, int ctr = 0, int dims = 1);

// Candidates for the autotuner: every supported (m, variant) of a dimension.
std::vector<DimPlan> dim_candidates(int64_t L, int64_t M, int A, int tbytes, bool contiguous, int ctr = 0);

// FP64 two-level table of zeta_N for a descriptor (interleaved re, im):
// lo[j] = zeta_N^j for j < 2^kb, then hi[h] = zeta_N^{h 2^kb} for h < ceil(N / 2^kb).
std::vector<double> fft_table(const FftDesc& d);

// Roots of unity in FP64 (long double internally), zeta_N^e for e in [0, N).
void root(int64_t N, int64_t e, double* re, double* im);

}  // namespace hd
