/*
 * hdconv.h -- C ABI of the MI355X (gfx950) hybrid-dealiased convolution
 * library (libhdconv.so).
 *
 * The operation is the one defined in Sec. 2 of Murasko & Bowman, "Hybrid
 * Dealiasing of Complex Convolutions" (arXiv 2303.17510): A complex inputs of
 * equal length L (per dimension), each zero padded to at least M, and
 * B = 1 output whose DFT is the pointwise product of the A padded DFTs
 * (the multiplication operator of Sec. 2).  The library returns the first L
 * outputs per dimension, which are the outputs Algorithm 1 accumulates,
 * i.e. for A = 2
 *     h_j = sum_{i=0}^{j} f_i g_{j-i},   j = 0 .. L-1,
 * and the box-truncated d-dimensional analogue for d = 2, 3 (Sec. 5).
 *
 * Data: dense, row-major arrays of prod(L) complex words, interleaved
 * (re, im); dimension 0 is the slowest.  HDCONV_C64 = float pairs,
 * HDCONV_C128 = double pairs.  All data pointers are device pointers.
 *
 * Threading: a plan owns device workspace and is not re-entrant; use one
 * plan per concurrent stream.  Separate plans are independent.  Errors never
 * throw across the ABI: functions return a status (or NULL) and
 * hdconv_last_error() gives the calling thread's last message.
 */
#ifndef HDCONV_H
#define HDCONV_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Opaque handles.  A plan owns its device workspace and twiddle tables, a
 * batched plan its groups, task tables and captured graph, a cost model its
 * device parameters. */
typedef struct hdconv_plan_s* hdconv_plan_t;
typedef struct hdconv_batch_s* hdconv_batch_t;
typedef struct hdconv_model_s* hdconv_model_t;

/* element types */
enum { HDCONV_C64 = 0, HDCONV_C128 = 1 };

/* status codes */
enum {
  HDCONV_OK = 0,
  HDCONV_EINVAL = -1,      /* invalid argument (sizes, pointers, geometry) */
  HDCONV_ENOMEM = -2,      /* device allocation failed or exceeds the cap  */
  HDCONV_EDEVICE = -3,     /* a HIP call failed; message has its text       */
  HDCONV_EUNSUPPORTED = -4,/* valid request the library does not support    */
  HDCONV_ENODEV = -5       /* no HIP device is available                    */
};

/* method: hybrid dealiasing (Sec. 2.1) or conventional explicit padding
 * (inputs materialised zero-padded to N' = 2^a or 3*2^a >= M, full FFTs,
 * product, inverse FFT, first L copied out: the baseline the paper compares
 * against, Sec. 7).  For the explicit method options.m of the innermost
 * dimension, when set, picks the split N' = p m of its transform. */
enum { HDCONV_METHOD_AUTO = 0, HDCONV_METHOD_HYBRID = 1, HDCONV_METHOD_EXPLICIT = 2 };

/* multiplication operator (Sec. 2: mult maps the A transforms to B outputs
 * pointwise).  PRODUCT: B = 1, the product of the A transforms (A = 2 or 3).
 * QUADRATIC: 2 <= A <= 6 inputs and 1 <= B <= 8 outputs, output
 * b = sum_{i <= j} c[b][i][j] F_i F_j with the real B x A x A coefficients in
 * options.mult_coef (entries below the diagonal unused) -- e.g. the Basdevant
 * forms of the Navier-Stokes nonlinearity, A = B = 2 in 2D and A = 3, B = 5
 * in 3D, or the 3D magnetohydrodynamic terms with A = 6, B = 8 (Sec. 9).
 * Quadratic operators multiply two transforms, so their padding rule is that
 * of A = 2; the outputs are computed one after another from transforms of
 * the inputs made once (the row pass transforms the rows of the inputs an
 * output needs, at most three per launch: with more, an output is the sum of
 * several launches), and must not overlap the inputs or each other (also
 * for B = 1 when an output sums several launches). */
enum { HDCONV_MULT_PRODUCT = 0, HDCONV_MULT_QUADRATIC = 1 };

/* per-dimension kernel variant */
enum {
  HDCONV_VARIANT_AUTO = 0,
  HDCONV_VARIANT_FUSED = 1,     /* innermost dim, p <= 2: whole row in one workgroup (Alg. 3-6) */
  HDCONV_VARIANT_MULTIPASS = 2, /* innermost dim, inner-loop form (Sec. 6.1), three passes      */
  HDCONV_VARIANT_OUTER = 3      /* outer dim of a 2D/3D convolution, p <= 2 (Sec. 5)            */
};

/* plan flags */
enum {
  HDCONV_PLAN_HOST_ONLY = 1, /* plan geometry only: no device memory, cannot execute */
  HDCONV_BATCH_NO_GRAPH = 2, /* batched plans: launch eagerly on every execute      */
  HDCONV_PLAN_CENTERED = 4,  /* centered convolution (see below); plans and batches */
  HDCONV_PLAN_HERMITIAN = 8, /* Hermitian convolution (see below); plans, 1D batches    */
  HDCONV_PLAN_NO_WORKSPACE = 16, /* no workspace of its own: runs through
                                   hdconv_execute_noalloc only (see there)   */
  HDCONV_PLAN_ACCUMULATE_OUTPUT = 32, /* residue blocks of the inner form add their
                                   contributions into the output array itself
                                   instead of an FP64 accumulation buffer
                                   (the paper's two-block data-flow
                                   optimization, Sec. 6 loop optimizations):
                                   16 L bytes less workspace; the sum is kept
                                   in the output precision, and execution must
                                   be out of place                          */
  HDCONV_BATCH_GROUPED = 64      /* batched plans: one set of launches per size
                                   group on side streams instead of the
                                   persistent single launch (see below)     */
};

/* Centered convolutions (the paper's section on centered convolutions in one
 * dimension, eq. centDFT, with its inner form, and Sec. 5 per dimension).
 * With HDCONV_PLAN_CENTERED an array of extent L holds the signed indices
 * c = -H .. L-1-H, H = floor(L/2), at positions c + H (index 0 in the
 * middle), for the inputs and the output alike, and the output is
 *     h_c = sum_{c_1 + ... + c_A = c} f_{c_1} ... g_{c_A},   c = -H .. L-1-H,
 * over in-range indices (per dimension for d = 2, 3).  The hybrid method runs
 * the centered transforms: p = ceil(H/m) + ceil((L-H)/m) blocks of m points
 * (2 for m >= L/2) holding the signed indices, twiddles of the signed index.
 * The padding needed is smaller: M >= max(A(L-1-H)+H, L-1-H+AH) + 1, i.e.
 * 3L/2 for A = 2 and even L, instead of A(L-1)+1.  The explicit method pads
 * the arrays as they are and copies out entries (A-1)H .. (A-1)H+L-1.
 *
 * Hermitian convolutions (the paper's section on Hermitian symmetric
 * convolutions, eq. wHerDef and Alg. 2 with its Hermitian transforms; Sec. 5
 * with centered outer dimensions).  With HDCONV_PLAN_HERMITIAN and nominal
 * length L of the last dimension, each array holds Lh = ceil(L/2) words
 * f_0 .. f_{Lh-1} (the non-negative indices) of the centered array
 * f_{-(Lh-1)} .. f_{Lh-1} with f_{-c} = conj(f_c); the imaginary part of f_0 is
 * ignored (a Hermitian array has a real centre).  The output holds
 * h_0 .. h_{Lh-1} of the centered convolution of those arrays (itself
 * Hermitian).  Requires M >= (A+1)(Lh-1)+1 (3L/2 - 2 for A = 2 and even L).
 * 2D/3D: the outer dimensions are centered (as HDCONV_PLAN_CENTERED) with odd
 * extents, the stored box is L[0] x [L[1] x] Lh, and the array stands for
 * F(k, -c) = conj F(-k, c) (k the signed outer indices), the c = 0 plane being
 * taken as its Hermitian part.  The kernels run the centered transforms of the
 * full length 2 Lh - 1, reading negative indices as conjugates of the stored
 * half and writing only the stored half. */

typedef struct hdconv_options {
  int method;        /* HDCONV_METHOD_*                                         */
  int flags;         /* HDCONV_PLAN_*                                           */
  int64_t m[3];      /* forced subtransform size per dimension (0: choose)      */
  int64_t p[3];      /* forced explicit block count, >= ceil(L/m) (0: minimal)  */
  int64_t D[3];      /* residues per block, innermost multipass dim (0: all)    */
  int variant[3];    /* HDCONV_VARIANT_* per dimension                          */
  int E_m[3];        /* points per lane of the m-point transform: 4, 8, 12 or 16 (0: choose) */
  int E_p[3];        /* points per lane of the p-point transform: 1, 2, 4, 8, 12 or 16 (0: choose) */
  int S[3];          /* columns per workgroup of column/outer kernels (0: choose) */
  int rows_per_block[3]; /* rows per workgroup of row kernels (0: choose)       */
  int twiddles[3];   /* FFT twiddles: 0 choose, 1 two-level root table, 2 exact per-stage tables */
  int tuner;         /* HDCONV_TUNER_*: how shapes left to the planner are chosen */
  int tune_reps;     /* executes per timed block of a candidate (0: 5)          */
  double margin;     /* model tuner: also time the predicted top three when the
                        log-time gap between the best two is below this (0: 0.05) */
  hdconv_model_t model; /* model tuner: a cost model from hdconv_model_create   */
  const char* db_path; /* timed tuners: append every timing to this CSV (NULL: none) */
  int64_t copies;    /* C independent copies of the problem per execute (0: 1)  */
  int64_t dist;      /* words between the starts of consecutive copies, inputs
                        and output alike (0: one copy's extent)                */
  int mult;          /* HDCONV_MULT_* (0: product)                              */
  const double* mult_coef; /* quadratic operator: B x A x A host doubles        */
  int64_t stride[2]; /* 2D/3D: element strides of dimensions 0 and 1 (the last
                        dimension is contiguous), inputs and output alike; 0:
                        dense.  2D uses stride[0] >= L[1] (stored extent);
                        3D stride[1] >= L[2], stride[0] >= L[1] stride[1]     */
  int conj_pairs;    /* inner form, forward column pass: 0 computes residues v and
                        n - v together (the conjugate symmetry optimization) when
                        a block holds all n >= 3 residues of an ordinary
                        dimension; -1 never                                   */
  int reserved[7];   /* zero                                                    */
} hdconv_options;

/* tuners (Sec. 7: the paper's optimizer times candidate (m, D, ...) per
 * dimension; the model tuner predicts those times, times its pick per
 * dimension against the default plan (keeping the default unless the pick is
 * faster), and on close calls times the predicted top three as well) */
enum { HDCONV_TUNER_HEURISTIC = 0, HDCONV_TUNER_EXHAUSTIVE = 1, HDCONV_TUNER_MODEL = 2 };

typedef struct hdconv_dim_info {
  int64_t L, M;      /* lengths the engine works on in this dimension           */
  int64_t m, p, n, q;/* paper's subtransform size, explicit blocks, residues, q */
  int64_t D;         /* residues per block                                      */
  int variant;       /* HDCONV_VARIANT_*                                        */
  int E_m, E_p;      /* points per lane of the m- and p-point transforms        */
  int S;             /* columns per workgroup (column / outer kernels)          */
  int rows_per_block;/* rows per workgroup (row kernels)                        */
  int tw_m, tw_p;    /* twiddle mode of the m- and p-point transforms (1 two-level, 2 per-stage) */
  int centered;      /* 1: centered transforms (HDCONV_PLAN_CENTERED), 2: the
                        Hermitian dimension (HDCONV_PLAN_HERMITIAN; its outer
                        dimensions report 1); shapes passed to hdconv_time_shape /
                        hdconv_features are Hermitian if the last dimension's
                        field is 2, else centered if dimension 0's is 1        */
} hdconv_dim_info_t;

typedef struct hdconv_plan_info {
  int dims, A, B, dtype, method;
  int64_t L[3], M[3];            /* the user's problem                           */
  hdconv_dim_info_t dim[3];
  int64_t npad[3];               /* explicit method: padded extents, else 0      */
  size_t workspace_bytes;        /* device workspace owned by the plan           */
  size_t table_bytes;            /* device twiddle tables owned by the plan      */
  double compulsory_bytes;       /* (A+B) prod(L) word bytes: read inputs, write output once */
  double traffic_bytes;          /* bytes the plan's kernels read + write by design */
  int launches;                  /* kernel launches per execute                  */
  int tuner;                     /* tuner that chose the shapes                  */
  int tuned_candidates;          /* candidates considered                        */
  int timed_candidates;          /* candidates timed on the device               */
  double tuned_ms;               /* time of the chosen shapes when it was measured, else 0 */
} hdconv_plan_info_t;

/* Autotuning interface.  hdconv_candidates lists the planner's search space
 * for a problem the way the paper's optimizer decouples it (Sec. 7): the
 * default plan, and that plan with one dimension's shape replaced by each of
 * its candidates.  Candidate k is out[k*dims .. k*dims+dims); varied[k] is the
 * dimension it changes (-1 for the default plan).  flags: 0,
 * HDCONV_PLAN_CENTERED or HDCONV_PLAN_HERMITIAN (L, M as hdconv_plan_ex
 * takes them; the shapes then carry centered = 1, or 2 on the Hermitian
 * dimension, which hdconv_time_shape and hdconv_features read).  Host only. */
int hdconv_candidates(const int64_t* L, const int64_t* M, int A, int B, int dims, int dtype, int flags,
                      hdconv_dim_info_t* out, int* varied, int cap, int* count);

/* Time in ms of one execute of the plan whose per-dimension shapes are
 * shape[0..dims), on zeroed device buffers: after one warm-up, three blocks
 * of `reps` executes run back to back and the median block average is
 * returned (the steady state of a caller running many steps). */
int hdconv_time_shape(const int64_t* L, const int64_t* M, int A, int B, int dims, int dtype,
                      const hdconv_dim_info_t* shape, int reps, double* ms);

/* Cost-model features of a candidate: HDCONV_NFEATURES floats describing the
 * problem and the shape (logs of lengths, sizes, traffic, work; centered and
 * Hermitian flags; dimensions on the lean kernels; the largest q). */
enum { HDCONV_NFEATURES = 48 };
int hdconv_features(const int64_t* L, const int64_t* M, int A, int B, int dims, int dtype,
                    const hdconv_dim_info_t* shape, float* out);

/* Fill *opt with defaults (AUTO everywhere, nothing forced). */
void hdconv_options_init(hdconv_options* opt);

/* Create a plan on the current HIP device.  L[d], M[d] for d < dims
 * (dims in {1,2,3}); A in {2,3} and B = 1 (a quadratic operator: A in
 * 2 .. 6, B in 1 .. 8); dtype HDCONV_C64 or HDCONV_C128.
 * Requires L[d] >= 1 and M[d] >= A (L[d]-1) + 1 (the padding that keeps the
 * product of A inputs unaliased, Sec. 2; centered plans: the centered minimum
 * above).  Allocates twiddle tables (FP64
 * generated, stored in dtype) and workspace with hipMalloc.  Returns NULL on
 * error (hdconv_last_error gives the reason). */
hdconv_plan_t hdconv_plan(const int64_t* L, const int64_t* M, int A, int B, int dims, int dtype);
hdconv_plan_t hdconv_plan_ex(const int64_t* L, const int64_t* M, int A, int B, int dims, int dtype,
                     const hdconv_options* opt);

/* Copies (the paper's problem descriptor carries C copies with a stride):
 * with options.copies = C > 1 every input and the output hold C copies of
 * the problem, copy c starting options.dist words (default: one copy's dense
 * extent) after copy c-1; each copy is convolved independently, all in the
 * same launches (the copies multiply the rows / planes of every pass).  dist
 * must be at least one copy's extent; words between copies are not touched.
 * The explicit method runs the copies one after another.  With
 * options.stride a copy is strided (padded rows, as in the paper's benchmark
 * layouts): element (i0, i1[, i2]) at i0 stride[0] + i1 [stride[1] + i2]; one
 * copy's extent is then L[0] stride[0], and the padding words are not touched.
 *
 * Run the convolution asynchronously on `stream` (a hipStream_t; NULL = the
 * null stream).  inputs: A device pointers, outputs: B device pointers, each
 * to prod(L) words of dtype (Hermitian plans: ceil(L/2) in the last
 * dimension; with copies, (C-1) dist + that many).  outputs[0] may equal one of the inputs
 * (in place, as in Algorithm 1; not for the quadratic operators that must
 * run out of place, see above); any other overlap is HDCONV_EINVAL.  The
 * inputs are not modified unless aliased by the output.  Returns the launch
 * status; no synchronisation is done. */
int hdconv_execute(hdconv_plan_t plan, const void* const* inputs, void* const* outputs, void* stream);

/* For callers that cannot allocate device memory while they run: code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc.
 * Runs `plan` exactly like hdconv_execute (same kernels, same arguments and
 * rules), but its workspace is the library's static device scratch area of
 * HDCONV_SCRATCH_BYTES instead of the plan's own; the call allocates and
 * frees nothing.  Create the plan beforehand (hdconv_plan_ex allocates its
 * twiddle tables; with HDCONV_PLAN_NO_WORKSPACE it allocates no workspace).
 * A plan whose workspace (hdconv_plan_info: workspace_bytes) exceeds
 * HDCONV_SCRATCH_BYTES is rejected with HDCONV_EUNSUPPORTED before anything
 * runs.  Each GPU the library runs on holds one scratch area, located on the
 * first call on that device and kept until the process ends; every call on a
 * device shares it and nothing in it is assumed to start at zero.  Calls that
 * overlap in time on one device (different streams or host threads) race on
 * it: serialise them. */
#define HDCONV_SCRATCH_BYTES ((size_t)64 << 20)
int hdconv_execute_noalloc(hdconv_plan_t plan, const void* const* inputs, void* const* outputs, void* stream);

/* Plan geometry and sizes. */
int hdconv_plan_info(hdconv_plan_t plan, hdconv_plan_info_t* out);

/* Release a plan (synchronises the device first).  NULL is ignored. */
void hdconv_destroy(hdconv_plan_t plan);

/* The paper's geometry rules for one dimension and a given m (Algorithm 1,
 * eq. pqdef1, Sec. 6.1): p = max(ceil(L/m), p_min); if p <= 2 and not
 * force_inner: q = n = ceil(M/m); else n = ceil(M/(p m)), q = n p.  Host only.
 * Fills out->{L,M,m,p,n,q,D=n,variant} (variant FUSED for the direct form,
 * MULTIPASS for the inner form). */
int hdconv_geometry(int64_t L, int64_t M, int64_t m, int64_t p_min, int force_inner,
                    hdconv_dim_info_t* out);

/* The same rules for the centered and Hermitian dimensions (flags:
 * HDCONV_PLAN_CENTERED or HDCONV_PLAN_HERMITIAN; 0 is hdconv_geometry).  A
 * centered dimension's signed indices -H .. L-1-H lie in
 * hdconv_centered_span(L, m) = ceil(H/m) + ceil((L-H)/m) blocks of m points.
 * Direct form (that span <= 2, the centered case of the paper's centered
 * one-dimensional section): p = span, q = n = ceil(M/m).  Inner form (the
 * paper's centered inner loop): the negative blocks fold onto the column
 * positions of the non-negative ones, so the column DFT needs only
 * p = max(p_min, ceil((L-H)/m)) points -- the paper's p/2 for its even block
 * count p -- and n = ceil(M/(p m)), q = n p.  Example (the optimizer's
 * choice for the 2D Hermitian L = 2048, M = 3072 benchmark, Sec. 7.2): m = 16
 * spans 128 blocks, p = 64, n = 3, q = 192.  HDCONV_PLAN_HERMITIAN takes the
 * nominal length L and works on the centered length 2 ceil(L/2) - 1 its
 * stored half stands for (out->L).  out->centered is 1 (centered) or 2
 * (Hermitian).  Host only; HDCONV_EINVAL for bad arguments or flags. */
int hdconv_geometry_ex(int64_t L, int64_t M, int64_t m, int64_t p_min, int force_inner, int flags,
                       hdconv_dim_info_t* out);
/* Blocks of m points the signed indices of a centered dimension of extent L
 * span: ceil(H/m) + ceil((L-H)/m), H = floor(L/2) (0 for L < 1 or m < 1). */
int64_t hdconv_centered_span(int64_t L, int64_t m);

/* Least padded length M that hdconv_plan accepts for one dimension of extent
 * L and A factors per product (a quadratic operator multiplies two: pass
 * A = 2), written to *M.  flags 0: A(L-1)+1, the padding that keeps a linear
 * product of A inputs unaliased (Sec. 2); HDCONV_PLAN_CENTERED: the centered
 * minimum max(A(L-1-H)+H, L-1-H+AH)+1 (3L/2 for A = 2 and even L);
 * HDCONV_PLAN_HERMITIAN: that minimum for the centered length
 * 2 ceil(L/2) - 1 a stored half stands for.  HDCONV_EINVAL for L < 1, A
 * outside 2 .. 3 or other flags. */
int hdconv_min_padding(int64_t L, int A, int flags, int64_t* M);

/* Learned cost model (the planner's model tuner).  A multilayer perceptron:
 * HDCONV_NFEATURES inputs (normalised by the training set's mean and
 * standard deviation), three hidden layers of `hidden` SiLU units, one linear
 * output = predicted log run time in ms.  Training (forward, backward, Adam on
 * the mean squared error of normalised targets) and inference run in FP32 HIP
 * kernels of this library.  The parameter vector is W1[NF][H], b1[H],
 * W2[H][H], b2[H], W3[H][H], b3[H], W4[H], b4 (the network), then xmean[NF],
 * xstd[NF], ymean, ystd.  X arrays are row-major n x HDCONV_NFEATURES host
 * floats; y holds log run times.  All calls synchronise. */
hdconv_model_t hdconv_model_create(int hidden, uint64_t seed);      /* Glorot-uniform init; NULL on error */
int hdconv_model_params(hdconv_model_t model, float* params, int cap, int* n);
int hdconv_model_load(hdconv_model_t model, const float* params, int n);
int hdconv_model_train(hdconv_model_t model, const float* X, const float* y, int64_t n, int epochs, int batch, float lr,
                       uint64_t seed, float* final_loss);
int hdconv_model_predict(hdconv_model_t model, const float* X, int64_t n, float* out);
/* Gradient of the loss over all n rows with respect to the network
 * parameters (with the model's current normalisation) and the loss. */
int hdconv_model_grad(hdconv_model_t model, const float* X, const float* y, int64_t n, float* grad, float* loss);
void hdconv_model_destroy(hdconv_model_t model);

/* Batched plans: `count` independent one-dimensional convolutions of uneven
 * length (dims = 1), L[i] and M[i] each as in hdconv_plan, all with the same
 * A in {2,3}, B = 1 (the product operator; HDCONV_EUNSUPPORTED otherwise)
 * and dtype.  Convolutions whose planned shape (variant, m, p, q and
 * kernel widths) coincides form one group (a size bucket).
 * Persistent form (the default for ordinary, not centered or Hermitian,
 * batches with the heuristic tuner whose every convolution has a compiled
 * shape: L up to 96 * 2048 in complex64, 2^16 in complex128, and M <= 8 * the
 * power of two at or above L for whole rows): three launches of one
 * persistent kernel (a grid of resident workgroups looping over a device
 * task table), one per pass of the inner form of Sec. 6.1 -- column pass,
 * row pass, back pass -- for every long convolution at once (rows of 2048
 * points, complex128 1024); the short ones (L <= 2048, complex128 1024) run
 * as whole rows (the direct form, Sec. 2) in the last launch.  The
 * workspace holds every long convolution's A q m transformed words at once.
 * Grouped form (HDCONV_BATCH_GROUPED, tuned plans, centered and Hermitian
 * batches): each group runs as one set of launches over a device table of
 * per-row pointers and lengths, groups on parallel branches (four side
 * streams forked from and joined to the execute stream).  Either way, from
 * the second execute on the batch is one hipGraph launch.  Allocates
 * per-group tables, workspace, a device task table and a pinned staging copy
 * of it.  NULL on error.
 * With opt->tuner EXHAUSTIVE or MODEL, each group of the heuristic plan (a
 * size bucket) is tuned: the candidates are the one-dimensional candidates
 * of its longest member plus row-packing variants of the whole-row kernel,
 * timed as the batch runs them (all rows of the group, their own lengths,
 * zeroed scratch buffers); EXHAUSTIVE times all, MODEL ranks them with
 * opt->model and times the top three when the best two predictions are
 * within opt->margin.  Groups whose tuned shapes coincide are merged. */
hdconv_batch_t hdconv_plan_batched(const int64_t* L, const int64_t* M, int64_t count, int A, int B, int dims, int dtype,
                          const hdconv_options* opt);

/* inputs: count*A device pointers (convolution i uses inputs[i*A + a]);
 * outputs: count*B device pointers; each of L[i] words (Hermitian batches:
 * ceil(L[i]/2) words).  When the pointers differ from the last execute's,
 * uploads the pointer table (asynchronously, on `stream`; the pinned staging
 * buffer is reused, so such an execute waits for the previous upload), then
 * launches.  Executes of one batch must not overlap in time (they share the
 * workspace). */
int hdconv_execute_batched(hdconv_batch_t batch, const void* const* inputs, void* const* outputs, void* stream);

/* Groups of a batched plan: shapes into groups[0..cap), member counts into
 * counts[0..cap), and the number of groups into *ngroups. */
int hdconv_batch_info(hdconv_batch_t batch, hdconv_dim_info_t* groups, int64_t* counts, int cap, int* ngroups);

/* Launch shape of a batched plan. */
typedef struct hdconv_batch_stats {
  int persistent;     /* 1: persistent launches; 0: grouped launches        */
  int grid;           /* persistent: resident workgroups of a launch        */
  int64_t tasks;      /* persistent: task-table entries of the launches     */
  int64_t lds_bytes;  /* persistent: LDS bytes per workgroup                */
  int64_t work_bytes; /* device workspace of all groups                     */
} hdconv_batch_stats_t;
int hdconv_batch_stats(hdconv_batch_t batch, hdconv_batch_stats_t* out);

/* Release a batched plan (synchronises the device first).  NULL is ignored. */
void hdconv_batch_destroy(hdconv_batch_t batch);

/* Per-launch timing.  hdconv_profile_begin(plan, n) creates HIP events for
 * the next n executes of `plan`; each of those executes records an event
 * pair around every kernel it launches, on the execute stream (the events
 * add no synchronisation).  hdconv_profile_end waits for the events, writes
 * one record per launch slot of an execute (in launch order) into out[0..cap)
 * and the slot count into *count, and releases the events.  bytes_per_launch
 * is the launch's algorithmic traffic: the words its contract reads once
 * plus the words it writes once. */
typedef struct hdconv_kernel_stat {
  char name[32];            /* "fused1d", "cols_fwd", "rows_conv", "cols_bwd", "outer_fwd", ... */
  int64_t launches;         /* executes that timed this slot                  */
  double total_ms;          /* summed event-to-event time                     */
  double bytes_per_launch;  /* algorithmic bytes read + written per launch     */
} hdconv_kernel_stat_t;

int hdconv_profile_begin(hdconv_plan_t plan, int max_executes);
int hdconv_profile_end(hdconv_plan_t plan, hdconv_kernel_stat_t* out, int cap, int* count);

/* Copy the calling thread's last error message into msg (NUL terminated,
 * truncated to cap) and return its status code (HDCONV_OK if none). */
int hdconv_last_error(char* msg, size_t cap);

/* Library version string. */
const char* hdconv_version(void);

#ifdef __cplusplus
}
#endif
#endif /* HDCONV_H */
