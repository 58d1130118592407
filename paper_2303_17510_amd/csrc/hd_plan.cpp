// hd_plan.cpp -- geometry rules and kernel-shape choices (host only).
#include "hd_plan.hpp"

#include <cmath>

#include <math.h>

#include <algorithm>

namespace hd {

static int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }

Geometry geometry(int64_t L, int64_t M, int64_t m, int64_t p_min, bool force_inner) {
  Geometry g{};
  g.m = m;
  g.p = std::max(cdiv(L, m), p_min);
  if (g.p <= 2 && !force_inner) {
    // Algorithm 1, p = 1 or 2: q = n = ceil(M/m) residues of size m
    g.n = g.q = cdiv(M, m);
    g.inner = false;
  } else {
    // Sec. 6.1: q is the smallest multiple of p with q m >= M
    g.n = cdiv(M, g.p * m);
    g.q = g.n * g.p;
    g.inner = true;
  }
  return g;
}

int64_t centered_blocks(int64_t L, int64_t m) {
  const int64_t H = L / 2;
  return cdiv(H, m) + cdiv(L - H, m);
}

int64_t centered_pos_blocks(int64_t L, int64_t m) { return cdiv(L - L / 2, m); }

bool centered_folds(const DimPlan& dp) {
  return dp.ctr && dp.variant == VAR_MULTI && dp.p < centered_blocks(dp.L, dp.m);
}

Geometry geometry_c(int64_t L, int64_t M, int64_t m, int64_t p_min, bool force_inner, int ctr) {
  if (!ctr) return geometry(L, M, m, p_min, force_inner);
  Geometry g{};
  g.m = m;
  const int64_t pd = std::max(p_min, centered_blocks(L, m));
  if (pd <= 2 && !force_inner) {
    g.p = pd;
    g.n = g.q = cdiv(M, m);
    g.inner = false;
  } else {
    g.p = std::max(p_min, centered_pos_blocks(L, m));
    g.n = cdiv(M, g.p * m);
    g.q = g.n * g.p;
    g.inner = true;
  }
  return g;
}

int64_t centered_min_padding(int64_t L, int A) {
  const int64_t H = L / 2, P = L - 1 - H;  // most negative and most positive index
  return std::max<int64_t>((int64_t)A * P + H, P + (int64_t)A * H) + 1;
}

bool fft_size_ok(int64_t N) {
  if (N < 1) return false;
  if ((N & (N - 1)) == 0) return true;
  if (N % 3 == 0) {
    int64_t t = N / 3;
    return (t & (t - 1)) == 0 && t >= 8;
  }
  return false;
}

int64_t next_fft_size(int64_t n) {
  int64_t best = 1;
  while (best < n) best <<= 1;
  for (int64_t t = 8; 3 * t < best; t <<= 1)
    if (3 * t >= n) return 3 * t;
  return best;
}

// Column transform sizes: powers of two and 3 * 2^a with a >= 2 (12, 24, ...).
bool col_size_ok(int64_t p) {
  if (p < 1) return false;
  if ((p & (p - 1)) == 0) return true;
  if (p % 3 != 0) return false;
  const int64_t t = p / 3;
  return (t & (t - 1)) == 0 && t >= 4;
}

int64_t next_col_size(int64_t n) {
  int64_t best = 1;
  while (best < n) best <<= 1;
  for (int64_t t = 4; 3 * t < best; t <<= 1)
    if (3 * t >= n) return 3 * t;
  return best;
}

bool make_fft_desc(int64_t N, int E, FftDesc* d) {
  *d = FftDesc{};
  if (N < 1 || E < 1 || N % E != 0 || N / E > kMaxThreads) return false;
  d->N = (int)N;
  d->G = (int)(N / E);
  int64_t rem = N;
  int st = 0;
  while (rem % 3 == 0) {
    if (E % 3 != 0 || st >= 12) return false;
    d->radix[st++] = 3;
    rem /= 3;
  }
  int rmax = 1;
  while (rmax < 16 && E % (rmax * 2) == 0) rmax *= 2;
  while (rem > 1) {
    if (rem & 1) return false;
    int r = rmax;
    while (rem % r != 0) r /= 2;
    if (r < 2 || st >= 12) return false;
    d->radix[st++] = r;
    rem /= r;
  }
  d->nst = st;
  d->kb = 0;
  while ((int64_t(1) << (2 * d->kb)) < N) ++d->kb;
  d->ntw = (1 << d->kb) + (int)((N + (int64_t(1) << d->kb) - 1) >> d->kb);
  int64_t Ns = 1, off = 0;
  for (int s = 0; s < st; ++s) {
    d->twoff[s] = (int)off;
    if (Ns > 1) off += Ns * (d->radix[s] - 1);
    Ns *= d->radix[s];
  }
  d->ntw_stage = (int)std::max<int64_t>(off, 1);
  d->twmode = 0;
  d->ps = 3;
  if (st > 0 && d->radix[0] == 16) d->ps = 4;
  if (st > 0 && d->radix[0] == 32) d->ps = 5;
  return true;
}

static int pow2_floor(int64_t x) {
  int r = 1;
  while ((int64_t)r * 2 <= x) r *= 2;
  return r;
}

// Points per lane of a row transform (fused and row kernels): enough that m
// points need at most kMaxThreads lanes, few enough that the kernel keeps
// its values in registers.  Sizes with a factor 3 take 12 (radices 3 and 4).
// Powers of two: measured on gfx950, the row pass is fastest with fewer,
// wider passes (16 points per lane in FP32 from m = 2048, 8 in FP64), the
// whole-row kernel with 8 (FP32, m >= 1024) or 4 points per lane.
static bool pow2_in(int64_t m, int64_t lo, int64_t hi) { return m >= lo && m <= hi && (m & (m - 1)) == 0; }

static bool pick_e_row(int64_t m, int64_t p, int64_t q, int A, bool fused, bool ctr, int tbytes, int* E) {
  // whole rows of one or two blocks (not centered) run the lean row kernel
  // (hd_k_lean.hip; 256 points, 256^2 rows: 0.46 ms against 0.90 ms for the
  // general whole-row kernel).  Measured row passes on gfx950: FP32 takes 8
  // points per lane, except 16 for products of two inputs on single-block
  // rows of 128 and 256 points with 2 .. 8 residues (256^3: 0.38 against 0.43 ms,
  // 128^3: 0.048 against 0.066 ms; half the LDS exchanges); FP64 takes 8
  // (256^3: 0.83 against 1.40 ms with 4), except 4 for single-residue rows
  // of 1024 points.
  // (FP64 rows of 2048 points: the general kernel with 8 points per lane,
  // 0.29 against 0.32-0.34 ms for the 2048^2 row pass)
  if (fused && p <= 2 && !ctr && pow2_in(m, 64, tbytes == 4 ? 2048 : 1024)) {
    if (tbytes == 4) *E = (A == 2 && p == 1 && q >= 2 && q <= 8 && (m == 128 || m == 256)) ? 16 : 8;
    else *E = (m == 1024 && q < 2) ? 4 : 8;
    return true;
  }
  if (m % 3 == 0) {
    *E = 12;
    return m % 12 == 0 && m / 12 <= kMaxThreads;
  }
  int e;
  // (whole rows of two 1024-point blocks: 4, measured 7 % faster in the 2D
  // centered and Hermitian plans, slower at 2048)
  if (tbytes == 4) e = fused ? ((m >= 1024 && !(p == 2 && m == 1024)) ? 8 : 4) : (m >= 2048 ? 16 : 8);
  else e = m >= 2048 ? 8 : 4;
  while (m / e > kMaxThreads && e < 16) e *= 2;
  if (m < e) e = (int)m;
  *E = e;
  return m % e == 0 && m / e <= kMaxThreads;
}

// Points per lane of a column transform (p points per column).
static bool pick_e_col(int64_t p, int tbytes, int* E) {
  if (p % 3 == 0) {
    *E = 12;
    return p % 12 == 0 && p / 12 <= kMaxThreads;
  }
  if (p <= 8) {
    *E = (int)p;
    return p == 1 || p == 2 || p == 4 || p == 8;
  }
  // FP32: 16 points per lane from p = 256 (measured faster for the forward
  // pass, which transforms one residue at a time), else 8; FP64: 4.
  const int e0 = tbytes == 4 ? (p >= 256 ? 16 : 8) : 4;
  *E = p / e0 <= kMaxThreads ? e0 : (p / 8 <= kMaxThreads ? 8 : 16);
  return p / *E <= kMaxThreads;
}

// Points per lane of an outer-dimension transform: the workgroup holds S
// adjacent columns, so fewer lanes per column give wider coalesced rows, but
// short transforms run best with few points per lane (measured: 4 up to 256
// points, 8 up to 1024, 16 beyond in FP32 and for the p = 2 form except at
// 512 points).
static bool pick_e_outer(int64_t m, int64_t p, bool ctr, int tbytes, int* E) {
  // one or two blocks of 64 .. 1024 points (not centered) run the lean
  // outer kernel: 8 points per lane up to 256 points, else 16 (FP64: 4,
  // else 8)
  // (also the m-point pass of the inner form, p > 2, which runs on the same
  // kernel's layout)
  if (!ctr && pow2_in(m, 64, 1024)) {
    *E = (tbytes == 4 ? 8 : 4) * (m <= 256 ? 1 : 2);
    return true;
  }
  if (m % 3 == 0) {
    *E = 12;
    return m % 12 == 0 && m / 12 <= kMaxThreads;
  }
  // (the p = 2 form of 512 points: 8, recorded 2D timings 1.12-1.29x over 16)
  if (tbytes == 4) *E = ((p >= 2 && m != 512) || m > 1024) ? 16 : (m <= 256 ? 4 : 8);
  else *E = m <= 256 ? 4 : 8;
  if (m < *E) *E = (int)m;
  while (m / *E > kMaxThreads && *E < 16) *E *= 2;
  return m % *E == 0 && m / *E <= kMaxThreads;
}

// Points per lane of the column transforms of an outer dimension in the
// inner form (p points; the workgroup holds 256 / (p / E) columns).
int outer_col_e(int p, int tbytes) { return p % 3 == 0 ? 12 : (p <= 4 ? p : (tbytes == 4 ? 8 : 4)); }

bool finish_dim(DimPlan* dp, int A, int tbytes, std::string* why) {
  const int cb = 2 * tbytes;  // bytes per complex word
  auto fail = [&](const char* s) {
    if (why) *why = s;
    return false;
  };
  if (dp->m < 1 || dp->p < 1 || dp->q * dp->m < dp->M) return fail("invalid geometry: need q m >= M");
  // (a centered dimension may have q < p: p = 2 whenever m >= L/2)
  if (!dp->ctr && dp->q < dp->p) return fail("invalid geometry: need q >= p");
  if (!dp->ctr && dp->p * dp->m < dp->L) return fail("invalid geometry: need p m >= L");
  if (dp->ctr && dp->variant != VAR_MULTI && dp->p < centered_blocks(dp->L, dp->m))
    return fail("invalid geometry: a centered direct form needs p >= ceil(H/m) + ceil((L-H)/m)");
  if (dp->ctr && dp->variant == VAR_MULTI && dp->p < centered_pos_blocks(dp->L, dp->m))
    return fail("invalid geometry: a centered inner form needs p >= ceil((L-H)/m)");
  // residue twiddle exponents are reduced mod q m in 32-bit arithmetic
  if (dp->q * dp->m >= (int64_t(1) << 31)) return fail("q m must stay below 2^31");
  if (!fft_size_ok(dp->m)) return fail("m must be 2^a or 3*2^a (a >= 3)");
  if (dp->D < 1) dp->D = dp->n;
  if (dp->D > dp->n) return fail("D exceeds the number of residues");
  // Preset shape fields (nonzero on entry) are kept and validated; zero ones
  // are chosen here.
  auto in_set = [](int v, std::initializer_list<int> s) {
    for (int x : s)
      if (x == v) return true;
    return false;
  };
  switch (dp->variant) {
    case VAR_FUSED:
    case VAR_MULTI: {
      const bool fused = dp->variant == VAR_FUSED;
      if (fused) {
        if (dp->p > 2) return fail("fused variant needs p <= 2");
        if (dp->m > kMaxFusedM) return fail("fused variant needs m <= 8192");
        if (dp->D != dp->n) return fail("fused variant processes all residues");
      } else {
        if (dp->q != dp->n * dp->p) return fail("inner form needs q = n p");
        if (dp->m < 8 || dp->m > kMaxRowM) return fail("multipass variant needs 8 <= m <= 8192");
        if (dp->p > kMaxColP || !col_size_ok(dp->p)) return fail("unsupported p for the column passes");
      }
      if (dp->E_m == 0 && !pick_e_row(dp->m, dp->p, dp->q, A, fused, dp->ctr != 0, tbytes, &dp->E_m)) return fail("unsupported m for the row kernel");
      if (!in_set(dp->E_m, {4, 8, 12, 16})) return fail("row points per lane must be 4, 8, 12 or 16");
      if (!make_fft_desc(dp->m, dp->E_m, &dp->fd_m)) return fail("no stage plan for m with these points per lane");
      auto need = [&](int r) {
        return ((size_t)r * A * (dp->m + (dp->m >> dp->fd_m.ps)) + tw_words(dp->fd_m)) * cb;
      };
      dp->fd_m.twmode = dp->tw_pref == 2;
      if (dp->tw_pref == 0 && need(1) > 81920) dp->fd_m.twmode = 0;
      if (dp->rows_per_block == 0) {
        int rpb = std::max(1, 256 / dp->fd_m.G);
        while (rpb > 1 && need(rpb) > 65536) rpb /= 2;
        dp->rows_per_block = rpb;
      }
      if (dp->rows_per_block < 1 || dp->rows_per_block * dp->fd_m.G > kMaxThreads)
        return fail("rows per block exceed the thread limit");
      if (need(dp->rows_per_block) > kLdsBudget) return fail("row does not fit in LDS");
      if (fused) return true;
      if (dp->E_p == 0 && !pick_e_col(dp->p, tbytes, &dp->E_p)) return fail("unsupported p for the column passes");
      if (!in_set(dp->E_p, {1, 2, 4, 8, 12, 16})) return fail("column points per lane must be 1, 2, 4, 8, 12 or 16");
      if (!make_fft_desc(dp->p, dp->E_p, &dp->fd_p)) return fail("no stage plan for p with these points per lane");
      // The backward column pass transforms two residues at once and keeps an
      // accumulator, so in FP32 it runs with at most 8 points per lane
      // (measured: 16 there costs registers and time); the forward pass uses
      // the requested width.
      dp->E_pb = (tbytes == 4 && dp->E_p > 8 && dp->E_p % 8 == 0) ? 8 : dp->E_p;
      if (!make_fft_desc(dp->p, dp->E_pb, &dp->fd_pb)) return fail("no stage plan for the backward column pass");
      auto cneed = [&](int S) { return ((size_t)2 * dp->p * S + tw_words(dp->fd_p)) * cb; };
      dp->fd_p.twmode = dp->tw_pref == 2;
      if (dp->tw_pref == 0 && cneed(std::min(16, (int)dp->m)) > 81920) dp->fd_p.twmode = 0;
      if (dp->S == 0) {
        int S = 64;
        while (S > 1 && (dp->m % S != 0 || S * std::max(dp->fd_p.G, dp->fd_pb.G) > kMaxThreads || cneed(S) > 81920))
          S /= 2;
        dp->S = S;
      }
      if (dp->m % dp->S != 0 || dp->S * std::max(dp->fd_p.G, dp->fd_pb.G) > kMaxThreads || cneed(dp->S) > kLdsBudget)
        return fail("column tile does not fit");
      return true;
    }
    case VAR_OUTER: {
      if (dp->p > 2) {
        // the inner form on an outer dimension (Sec. 6.1 with Sec. 5): column
        // transforms of p points over the blocks of m, then m-point
        // transforms, both on the lean outer kernels; ordinary dimensions,
        // all residues in one block
        if (dp->ctr) return fail("the inner form of an outer dimension takes ordinary (not centered) dimensions");
        if (dp->q != dp->n * dp->p) return fail("inner form needs q = n p");
        if (dp->D != dp->n) return fail("the inner form of an outer dimension keeps all residues in one block");
        if (!pow2_in(dp->m, 64, 1024)) return fail("the inner form of an outer dimension needs m = 2^k, 64 <= m <= 1024");
        const bool p3 = tbytes == 4 && dp->p % 3 == 0 && pow2_in(dp->p / 3, 4, 32);
        if (!pow2_in(dp->p, 4, 64) && !p3)
          return fail("the inner form of an outer dimension needs p = 4 .. 64 (a power of two) or 12 .. 96 (3 * 2^k, complex64)");
        if (dp->E_p == 0) dp->E_p = outer_col_e((int)dp->p, tbytes);
        if (dp->E_p != outer_col_e((int)dp->p, tbytes)) return fail("outer column points per lane do not match p");
        if (!make_fft_desc(dp->p, dp->E_p, &dp->fd_p)) return fail("no stage plan for p with these points per lane");
        dp->fd_p.twmode = 1;
        dp->E_pb = dp->E_p;
        dp->fd_pb = dp->fd_p;
      }
      if (dp->m > kMaxFusedM) return fail("outer variant needs m <= 8192");
      if (dp->D < 1 || dp->D > dp->n) return fail("outer variant needs 1 <= D <= q residues per block");
      if (dp->m < 8) return fail("outer variant needs m >= 8");
      if (dp->E_m == 0 && !pick_e_outer(dp->m, dp->p, dp->ctr != 0, tbytes, &dp->E_m)) return fail("unsupported m for the outer kernel");
      if (!in_set(dp->E_m, {4, 8, 12, 16})) return fail("outer points per lane must be 4, 8, 12 or 16");
      if (!make_fft_desc(dp->m, dp->E_m, &dp->fd_m)) return fail("no stage plan for m with these points per lane");
      auto oneed = [&](int S) { return ((size_t)dp->m * S + tw_words(dp->fd_m)) * cb; };
      dp->fd_m.twmode = dp->tw_pref == 2;
      if (dp->tw_pref == 0 && oneed(8) > 128 * 1024) dp->fd_m.twmode = 0;
      if (dp->S == 0) {
        // the lean outer kernel: 16 columns (measured at 256 points: 16
        // columns 1.30 ms against 8 columns 1.59 ms for the whole 256^3 plan)
        const bool lean = !dp->ctr && pow2_in(dp->m, 64, 1024);
        int S = std::min(pow2_floor(std::max(1, kMaxThreads / dp->fd_m.G)), lean ? 16 : 64);
        while (S > 1 && oneed(S) > 128 * 1024) S /= 2;
        dp->S = S;
      }
      // (the lean outer kernel takes workgroups of up to 1024 lanes)
      const bool lean_e = tbytes == 4 ? (dp->E_m == 8 || dp->E_m == 16) : (dp->E_m == 4 || dp->E_m == 8);
      const bool lean_tile = !dp->ctr && pow2_in(dp->m, 64, 1024) && dp->p <= 2 && dp->q <= 8 && lean_e &&
                             (size_t)dp->S * dp->m * 16 <= 128 * 1024;
      if (dp->S * dp->fd_m.G > (lean_tile ? 2 * kMaxThreads : kMaxThreads) || oneed(dp->S) > kLdsBudget)
        return fail("outer column tile does not fit");
      return true;
    }
    default:
      return fail("unknown variant");
  }
}

static bool set_geom(DimPlan* dp, int64_t L, int64_t M, int64_t m, int64_t p_min, int variant, int ctr = 0,
                     bool outer_inner = false) {
  Geometry g = geometry_c(L, M, m, p_min, variant == VAR_MULTI || outer_inner, ctr);
  if (variant == VAR_FUSED && g.inner) return false;
  if (variant == VAR_OUTER && g.inner != outer_inner) return false;
  dp->L = L;
  dp->M = M;
  dp->m = g.m;
  dp->p = g.p;
  dp->n = g.n;
  dp->q = g.q;
  dp->D = g.n;
  dp->variant = variant;
  dp->ctr = ctr;
  dp->E_m = dp->E_p = dp->S = dp->rows_per_block = 0;
  return true;
}

static int64_t pow2_ceil(int64_t x) {
  int64_t r = 1;
  while (r < x) r <<= 1;
  return r;
}

// Centered dimensions: the least padding q m over the supported shapes.
// Whole rows (p = 2 once m >= L/2): a single convolution takes one transform
// of m >= M (q = 1) up to 4096 points; many rows the least q m with m up to
// 4096, powers of two first, then the smallest such m (the transform work
// q m log m falls with m at equal q m).  Beyond, the inner form with the
// least q m over every column size p (a factor 3 in p reaches p m = 3L/2,
// the centered padding, with one residue block), then m nearest 4096.  Outer dimensions: the least q m over m up to 8192
// with p <= 2, powers of two first, then the larger m.
static bool choose_dim_centered(int64_t L, int64_t M, int A, int tbytes, bool contiguous, int64_t lines,
                                DimPlan* dp, std::string* why) {
  std::string w;
  std::vector<int64_t> sizes;
  for (int64_t s = 8; s <= kMaxRowM; s <<= 1) {
    sizes.push_back(s);
    if (3 * s <= kMaxRowM) sizes.push_back(3 * s);
  }
  std::sort(sizes.begin(), sizes.end());
  auto pow2 = [](int64_t m) { return (m & (m - 1)) == 0; };
  // better(a, b): less padding, then a power of two, then the preferred size
  auto pick = [&](int variant, int64_t mmax, bool prefer_large) {
    DimPlan best;
    bool found = false;
    for (int64_t m : sizes) {
      if (m > mmax) break;
      DimPlan c;
      if (!set_geom(&c, L, M, m, 0, variant, 1) || !finish_dim(&c, A, tbytes, &w)) continue;
      bool take = !found;
      if (found) {
        const int64_t a = c.q * c.m, b = best.q * best.m;
        if (a != b) take = a < b;
        else if (pow2(c.m) != pow2(best.m)) take = pow2(c.m);
        else take = prefer_large ? c.m > best.m : c.m < best.m;
      }
      if (take) {
        best = c;
        found = true;
      }
    }
    if (found) *dp = best;
    return found;
  };
  if (contiguous) {
    if (lines <= 1) {
      // a power of two (a lone row of 3 * 2^k points measured ~2x slower),
      // else 3 * 2^k when only that stays within 4096 points
      int64_t m = std::max<int64_t>(8, pow2_ceil(M));
      if (m > 4096) m = std::max<int64_t>(8, next_fft_size(M));
      if (m <= 4096 && set_geom(dp, L, M, m, 0, VAR_FUSED, 1) && finish_dim(dp, A, tbytes, &w)) return true;
    }
    if (pick(VAR_FUSED, 4096, false)) return true;
    DimPlan best;
    bool found = false;
    double best_key = 0;
    for (int64_t mm : {1024, 2048, 4096, 8192}) {
      if (mm > kMaxRowM) continue;
      // every column size from the folded span (negative blocks on the
      // positive ones) up to the full span or one residue block (n = 1,
      // p m >= M): q m = ceil(M/(p m)) p m is not monotone in p
      const int64_t pmin = centered_pos_blocks(L, mm);
      const int64_t pmax = std::max(next_col_size(centered_blocks(L, mm)), next_col_size(cdiv(M, mm)));
      for (int64_t p = next_col_size(pmin); p <= pmax; p = next_col_size(p + 1)) {
        if (p > kMaxColP) break;
        DimPlan c;
        if (!set_geom(&c, L, M, mm, p, VAR_MULTI, 1)) continue;
        // FP32 rows of 4096 points and more: 16 points per lane (measured
        // faster from 384 rows on, the fewest a centered 2^20 plan has)
        if (tbytes == 4) c.E_m = (mm >= 8192 || (mm >= 4096 && c.n * c.p * lines >= 256)) ? 16 : 8;
        if (!finish_dim(&c, A, tbytes, &w)) continue;
        if (centered_folds(c)) {
          // folded column passes: narrower column tiles (16 columns FP32, 8
          // FP64: more workgroups, measured 3-7 % faster at 2^20)
          DimPlan t = c;
          t.S = tbytes == 4 ? 16 : 8;
          if (t.S < c.S && finish_dim(&t, A, tbytes, &w)) c = t;
        }
        const double key = (double)(c.q * c.m) * 1e3 + std::fabs(std::log2((double)mm / 4096.0));
        if (!found || key < best_key) {
          best = c;
          best_key = key;
          found = true;
        }
      }
    }
    if (found) {
      *dp = best;
      return true;
    }
    if (why) *why = "no supported plan for this centered length" + (w.empty() ? std::string() : ": " + w);
    return false;
  }
  if (pick(VAR_OUTER, kMaxFusedM, true)) return true;
  if (why) *why = "no supported plan for this centered outer length: " + w;
  return false;
}

bool choose_dim(int64_t L, int64_t M, int A, int tbytes, bool contiguous, int64_t lines, DimPlan* dp,
                std::string* why, int ctr, int dims) {
  if (ctr) return choose_dim_centered(L, M, A, tbytes, contiguous, lines, dp, why);
  std::string w;
  if (contiguous) {
    // Whole rows in one workgroup.  A single convolution is latency-bound:
    // one transform of m >= M (q = 1, no residue loop in the lone workgroup)
    // up to 4096 points.  Many rows are throughput-bound: m >= L with the
    // residues looped (q = 2 for M = 2L), half the transform work.  Powers
    // of two only: sizes with a factor 3 measured slower at equal padding.
    // The rows of 2D plans up to 1024 points and of 3D plans up to 64 points
    // also take one transform of m >= M: the recorded 2D timings give
    // 1.12-1.32x per size class (1.0x at 2048), the 3D ones 1.09-1.16x up to
    // 64 points and 0.87-0.95x beyond.
    const int64_t mM = std::max<int64_t>(8, pow2_ceil(M));
    const int64_t q1max = dims == 2 ? 1024 : (dims == 3 ? 64 : 0);
    const int64_t m = (lines <= 1 || mM <= q1max) ? mM : std::max<int64_t>(8, pow2_ceil(L));
    // (sizes 3 * 2^k, even with 25 % less padding, measured slower here:
    // 1D single rows 1.9-2.1x, 2D rows 1.2-1.6x, 3D rows 1.1x)
    if (m <= 4096) {
      const DimPlan base_try = [&] {
        DimPlan t;
        std::string w2;
        if (!set_geom(&t, L, M, m, 0, VAR_FUSED)) {
          t.m = 0;
          return t;
        }
        // a lone FP32 row of up to 1024 points: 4 points per lane, one row
        // per workgroup (the most lanes for one latency-bound workgroup;
        // recorded timings 1.22x at 1024 points, 0.98x at 2048)
        if (lines <= 1 && tbytes == 4 && m >= 16 && m <= 1024) {
          t.E_m = 4;
          t.rows_per_block = 1;
        }
        if (!finish_dim(&t, A, tbytes, &w2)) t.m = 0;
        return t;
      }();
      // rows just above a power of two: two blocks of half the length (p = 2)
      // when that pads at least 20 % less, for halves of 2048 points and more
      // in 2D plans and of 64 and more in 3D (recorded timings 1.06-1.21x per
      // size class there, 0.95x for shorter halves)
      const int64_t half_min = dims == 2 ? 2048 : (dims == 3 ? 64 : 0);
      if (base_try.m && lines > 1 && half_min && m == std::max<int64_t>(8, pow2_ceil(L)) && m / 2 >= half_min) {
        DimPlan t;
        std::string w2;
        if (set_geom(&t, L, M, m / 2, 0, VAR_FUSED) && t.p == 2 && 5 * t.q * t.m <= 4 * base_try.q * base_try.m &&
            finish_dim(&t, A, tbytes, &w2)) {
          *dp = t;
          return true;
        }
      }
      if (base_try.m) {
        *dp = base_try;
        return true;
      }
    }
    // Inner form: the least padding q m over m = 1024 .. 8192 and p a power
    // of two, or for FP32 beyond L = 2^21 also 3 * 2^k from 96 up (column
    // transforms with a factor 3 measured slower even at 25 % less padding
    // below that: L = 7e5 62 -> 44 us, 1.5e6 95 -> 88 us with powers of two;
    // FP64 ones spill, so powers of two there).  Among equal
    // padding the m nearest the measured best for that size: for a single
    // convolution 2048 up to q m = 2^20, 4096 for 2^21, 8192 beyond; for many
    // rows (throughput) 4096.  Rows of 4096 points or more take 16 points per
    // lane when there are enough of them (n p lines >= 512) to fill the
    // chip and the rows combine two inputs, else 8 (with three inputs the
    // 16-point row kernel spills: recorded timings 1.15-1.33x for 8, whole
    // plans L = 7.5e5 117 -> 96 us, 3.2e6 568 -> 482 us).
    DimPlan best;
    bool found = false;
    double best_key = 0;
    for (int64_t mm : {1024, 2048, 4096, 8192}) {
      if (mm > kMaxRowM) continue;
      const int64_t pmin = cdiv(L, mm);
      std::vector<int64_t> ps = {pow2_ceil(pmin)};
      const int64_t p3 = next_col_size(pmin);
      if (tbytes == 4 && p3 % 3 == 0 && p3 >= 96 && L > (int64_t(1) << 21)) ps.push_back(p3);
      for (int64_t p : ps) {
        if (p > kMaxColP) continue;
        DimPlan c;
        if (!set_geom(&c, L, M, mm, p, VAR_MULTI)) continue;
        if (tbytes == 4) c.E_m = (mm >= 8192 || (mm >= 4096 && A == 2 && c.n * c.p * lines >= 512)) ? 16 : 8;
        if (!finish_dim(&c, A, tbytes, &w)) continue;
        const double qm = (double)(c.q * c.m);
        const double mt = lines > 1 ? 4096.0
                                    : (qm <= (double)(1 << 20) ? 2048.0 : (qm <= (double)(1 << 21) ? 4096.0 : 8192.0));
        const double key = qm * 1e3 + std::fabs(std::log2((double)mm / mt));
        if (!found || key < best_key) {
          best = c;
          best_key = key;
          found = true;
        }
      }
    }
    if (found) {
      *dp = best;
      return true;
    }
    if (why)
      *why = "no supported plan for this length (the inner form reaches L = 8192 x 4096)" +
             (w.empty() ? std::string() : ": " + w);
    return false;
  }
  // Outer dimensions (every residue multiplies the inner work, measured on
  // the autotuner's 2D/3D timings): powers of two only; up to 1024 points one
  // transform of m >= M (q = 1); beyond, the direct form with p = 1 or p = 2
  // (half the length: twice the columns per workgroup) and the least padding,
  // ties to p = 2 once the p = 1 transform would exceed 1024 points.  3D
  // plans beyond 64 points: see below.
  {
    const int64_t m1 = std::max<int64_t>(8, pow2_ceil(M));
    // 3D plans beyond 64 points: the power of two m >= L (p = 1) or its half
    // (p = 2), the least padding q m, ties to p = 1.  Both run the lean outer
    // kernel; measured for whole 3D cubes against the earlier choices (3 * 2^k
    // transforms, two residues of half the power of two): 96^3 0.170 ->
    // 0.084 ms, 150^3 1.02 -> 0.61, 192^3 1.21 -> 0.63, 320^3 8.4 -> 3.8,
    // 384^3 10.5 -> 4.7; at 229^3 the tie goes to p = 1 (1.72 against 1.89).
    // With 2^16 or more columns (FP32, from 256^3 on) the lean outer kernel
    // takes 32 columns per workgroup where the tile fits (at most 1024 lanes
    // and 128 KB of exchange), and ties then go to p = 2: measured at 256^3,
    // forward outer passes 0.266 -> 0.256 ms (p = 1) and 0.246 ms (p = 2,
    // m = 128), whole step 1.215 -> 1.202 -> 1.169 ms; at 128^3 (2^14 and
    // 2^15 columns) 32 columns were 6 % slower.
    const int64_t mA = std::max<int64_t>(8, pow2_ceil(L));
    if (dims == 3 && mA >= 128 && mA <= 2048) {
      DimPlan a, b;
      std::string w2;
      const bool oka = mA <= 1024 && set_geom(&a, L, M, mA, 0, VAR_OUTER) && finish_dim(&a, A, tbytes, &w2);
      const bool okb = set_geom(&b, L, M, mA / 2, 0, VAR_OUTER) && b.p == 2 && finish_dim(&b, A, tbytes, &w2);
      const bool wide = tbytes == 4 && lines >= 65536;
      auto widen = [&](DimPlan* c) {
        DimPlan t = *c;
        t.S = 32;
        std::string w3;
        if (pow2_in(t.m, 64, 256) && finish_dim(&t, A, tbytes, &w3)) *c = t;
      };
      if (wide) {
        if (oka) widen(&a);
        if (okb) widen(&b);
      }
      if (oka && (!okb || a.q * a.m < b.q * b.m || (a.q * a.m == b.q * b.m && !(wide && b.S == 32)))) {
        *dp = a;
        return true;
      }
      if (okb) {
        *dp = b;
        return true;
      }
    }
    if (m1 <= 1024 && set_geom(dp, L, M, m1, 0, VAR_OUTER) && finish_dim(dp, A, tbytes, &w)) return true;
    DimPlan a, b;
    const int64_t ma = std::max<int64_t>(8, pow2_ceil(L)), mb = std::max<int64_t>(8, pow2_ceil(cdiv(L, 2)));
    const bool oka = ma <= kMaxFusedM && set_geom(&a, L, M, ma, 0, VAR_OUTER) && finish_dim(&a, A, tbytes, &w);
    const bool okb = set_geom(&b, L, M, mb, 0, VAR_OUTER) && finish_dim(&b, A, tbytes, &w);
    // (in 2D plans halves of 256 points or fewer lose to the whole transform
    // even with more padding: recorded timings 1.33x for p = 1 at L ~ 350,
    // A = 3; in 3D the halves stay ahead)
    if (oka && (!okb || (dims == 2 && mb <= 256) || a.q * a.m < b.q * b.m || (a.q * a.m == b.q * b.m && ma <= 1024))) {
      *dp = a;
      return true;
    }
    if (okb) {
      *dp = b;
      return true;
    }
  }
  if (why) *why = "no supported plan for this outer length: " + w;
  return false;
}

std::vector<DimPlan> dim_candidates(int64_t L, int64_t M, int A, int tbytes, bool contiguous, int ctr) {
  std::vector<DimPlan> out;
  std::vector<int64_t> sizes;
  for (int64_t s = 8; s <= kMaxRowM; s <<= 1) {
    sizes.push_back(s);
    if (s >= 8 && 3 * s <= kMaxRowM) sizes.push_back(3 * s);
  }
  std::sort(sizes.begin(), sizes.end());
  auto add = [&](int64_t m, int64_t pmin, int variant, int E_m) {
    DimPlan dp;
    std::string w;
    if (!set_geom(&dp, L, M, m, pmin, variant, ctr)) return;
    dp.E_m = E_m;
    if (finish_dim(&dp, A, tbytes, &w)) out.push_back(dp);
  };
  const int64_t mlim = std::max<int64_t>(8, pow2_ceil(M));  // up to one transform of m >= M
  for (int64_t m : sizes) {
    if (m > mlim) break;
    // widths of the m-point transform: 12 for sizes with a factor 3, else
    // 4, 8 and 16 points per lane
    std::vector<int> Es;
    if (m % 3 == 0) Es = {12};
    else Es = {4, 8, 16};
    // blocks of m points the inputs span
    const int64_t pneed = ctr ? centered_blocks(L, m) : cdiv(L, m);
    if (contiguous) {
      // whole rows in one workgroup (p <= 2)
      if (pneed <= 2)
        for (int E : Es) add(m, 0, VAR_FUSED, E);
      // inner form: p rounded up to a supported size, and to a power of two
      // (centered: from the folded span up to the full span or n = 1)
      const int64_t pin = ctr ? centered_pos_blocks(L, m) : pneed;
      if (m >= 16 && pin <= kMaxColP) {
        const int64_t p0 = pin;
        int64_t p2 = 1;
        while (p2 < p0) p2 <<= 1;
        std::vector<int64_t> ps = {next_col_size(p0)};
        if (p2 != ps[0]) ps.push_back(p2);
        if (ctr)
          for (int64_t p = next_col_size(p0 + 1);
               p <= std::max(next_col_size(pneed), next_col_size(cdiv(M, m))) && p <= kMaxColP;
               p = next_col_size(p + 1))
            if (std::find(ps.begin(), ps.end(), p) == ps.end()) ps.push_back(p);
        for (int64_t p : ps) {
          if (p > kMaxColP) continue;
          for (int E : Es) add(m, p, VAR_MULTI, E);
        }
      }
    } else {
      if (pneed <= 2)
        for (int E : Es) add(m, 0, VAR_OUTER, E);
      // the inner form of an ordinary outer dimension: the least compiled
      // column size at or above the span (m = 64 .. 1024)
      if (!ctr && pneed > 2 && pow2_in(m, 64, 1024)) {
        int64_t p = 4;
        while (p < pneed) p *= 2;
        for (int64_t p3 = 12; p3 <= 96 && tbytes == 4; p3 *= 2)
          if (p3 >= pneed && p3 < p) p = p3;
        if (p <= 96) {
          DimPlan dp;
          std::string w;
          if (set_geom(&dp, L, M, m, p, VAR_OUTER, 0, true) && finish_dim(&dp, A, tbytes, &w)) out.push_back(dp);
        }
      }
    }
  }
  // drop exact duplicates (same shape reached twice)
  std::vector<DimPlan> uniq;
  for (const DimPlan& d : out) {
    bool dup = false;
    for (const DimPlan& u : uniq)
      dup = dup || (u.variant == d.variant && u.m == d.m && u.p == d.p && u.q == d.q && u.E_m == d.E_m &&
                    u.E_p == d.E_p && u.S == d.S && u.rows_per_block == d.rows_per_block);
    if (!dup) uniq.push_back(d);
  }
  return uniq;
}

void root(int64_t N, int64_t e, double* re, double* im) {
  e %= N;
  if (e < 0) e += N;
  // exact octant symmetries first, then one long-double evaluation
  const long double pi = 3.141592653589793238462643383279502884L;
  long double a = 2.0L * pi * (long double)e / (long double)N;
  *re = (double)cosl(a);
  *im = (double)sinl(a);
  if (4 * e == N) { *re = 0.0; *im = 1.0; }
  if (2 * e == N) { *re = -1.0; *im = 0.0; }
  if (4 * e == 3 * N) { *re = 0.0; *im = -1.0; }
  if (e == 0) { *re = 1.0; *im = 0.0; }
}

std::vector<double> fft_table(const FftDesc& d) {
  std::vector<double> v;
  const int64_t K = int64_t(1) << d.kb;
  for (int64_t j = 0; j < K; ++j) {
    double re, im;
    root(d.N, j, &re, &im);
    v.push_back(re);
    v.push_back(im);
  }
  for (int64_t h = 0; h * K < d.N; ++h) {
    double re, im;
    root(d.N, h * K, &re, &im);
    v.push_back(re);
    v.push_back(im);
  }
  // per-stage tables: w_{Ns R}^{k i}, k < Ns, 1 <= i < R
  int64_t Ns = 1;
  size_t base = v.size();
  for (int s = 0; s < d.nst; ++s) {
    const int R = d.radix[s];
    if (Ns > 1)
      for (int64_t k = 0; k < Ns; ++k)
        for (int i = 1; i < R; ++i) {
          double re, im;
          root(Ns * R, (k * i) % (Ns * R), &re, &im);
          v.push_back(re);
          v.push_back(im);
        }
    Ns *= R;
  }
  if (v.size() == base) {  // no twiddled stage: one placeholder entry
    v.push_back(1.0);
    v.push_back(0.0);
  }
  return v;
}

}  // namespace hd
