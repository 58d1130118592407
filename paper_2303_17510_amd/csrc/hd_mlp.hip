// hd_mlp.hip -- learned cost model of the planner: a multilayer perceptron
// that maps a candidate's features (problem geometry and shape) to its
// predicted log run time.  Training (forward, backward, Adam) and inference
// run in FP32 HIP kernels written here; the host only orchestrates.
//
// Network: x (HDCONV_NFEATURES, normalised by training-set mean and std) ->
// three hidden layers of H SiLU units -> one linear output (normalised log
// time).  Loss: mean squared error on normalised targets.
//
// Parameter vector (hdconv_model_params / hdconv_model_load), in order:
//   W1[NF][H], b1[H], W2[H][H], b2[H], W3[H][H], b3[H], W4[H], b4[1]
//   (the network; gradients cover exactly these), then
//   xmean[NF], xstd[NF], ymean, ystd (normalisation).
#include <hip/hip_runtime.h>
#include <math.h>
#include <string.h>

#include <algorithm>
#include <new>
#include <random>
#include <vector>

#include "hdconv.h"

namespace hd {

constexpr int NF = HDCONV_NFEATURES;

struct Mlp {
  int H = 64;
  int nnet = 0;              // network parameters
  std::vector<float> norm;   // xmean[NF], xstd[NF], ymean, ystd
  float* d_p = nullptr;      // network parameters (device)
  float* d_g = nullptr;      // gradient
  float* d_m = nullptr;      // Adam first moment
  float* d_v = nullptr;      // Adam second moment
  int64_t adam_t = 0;
  int off[8];                // offsets of W1 b1 W2 b2 W3 b3 W4 b4
};

static int layer_in(const Mlp& M, int l) { return l == 0 ? NF : M.H; }
static int layer_out(const Mlp& M, int l) { return l == 3 ? 1 : M.H; }

// ---------------------------------------------------------------------------
// kernels (one thread per output element; sizes are small)

__device__ __forceinline__ float sigm(float z) { return 1.f / (1.f + __expf(-z)); }

__global__ void k_normalize(const float* __restrict__ X, int64_t n, const float* __restrict__ mean,
                            const float* __restrict__ stdv, float* __restrict__ Xn) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n * NF) return;
  const int k = (int)(i % NF);
  Xn[i] = (X[i] - mean[k]) / stdv[k];
}

// Z = X W + b; Y = silu(Z) when act, else Z.  X: n x I, W: I x O.
__global__ void k_dense(const float* __restrict__ X, const float* __restrict__ W, const float* __restrict__ b,
                        float* __restrict__ Z, float* __restrict__ Y, int64_t n, int I, int O, int act) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n * O) return;
  const int64_t r = t / O;
  const int o = (int)(t % O);
  float z = b[o];
  for (int k = 0; k < I; ++k) z = fmaf(X[r * I + k], W[(int64_t)k * O + o], z);
  Z[t] = z;
  Y[t] = act ? z * sigm(z) : z;
}

// dZ = dY * silu'(Z) (act) or dY
__global__ void k_act_bwd(const float* __restrict__ dY, const float* __restrict__ Z, float* __restrict__ dZ,
                          int64_t cnt, int act) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= cnt) return;
  if (!act) {
    dZ[t] = dY[t];
    return;
  }
  const float s = sigm(Z[t]);
  dZ[t] = dY[t] * s * (1.f + Z[t] * (1.f - s));
}

// dW[k][o] = sum_r X[r][k] dZ[r][o];  db[o] = sum_r dZ[r][o]
__global__ void k_wgrad(const float* __restrict__ X, const float* __restrict__ dZ, float* __restrict__ dW,
                        float* __restrict__ db, int64_t n, int I, int O) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t < I * O) {
    const int k = t / O, o = t % O;
    float s = 0.f;
    for (int64_t r = 0; r < n; ++r) s = fmaf(X[r * I + k], dZ[r * O + o], s);
    dW[t] = s;
  } else if (t < I * O + O) {
    const int o = t - I * O;
    float s = 0.f;
    for (int64_t r = 0; r < n; ++r) s += dZ[r * O + o];
    db[o] = s;
  }
}

// dX[r][k] = sum_o dZ[r][o] W[k][o]
__global__ void k_dgrad(const float* __restrict__ dZ, const float* __restrict__ W, float* __restrict__ dX,
                        int64_t n, int I, int O) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n * I) return;
  const int64_t r = t / I;
  const int k = (int)(t % I);
  float s = 0.f;
  for (int o = 0; o < O; ++o) s = fmaf(dZ[r * O + o], W[(int64_t)k * O + o], s);
  dX[t] = s;
}

// dY = 2 (yhat - y) / n
__global__ void k_mse_grad(const float* __restrict__ yhat, const float* __restrict__ y, float* __restrict__ dY,
                           int64_t n) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n) return;
  dY[t] = 2.f * (yhat[t] - y[t]) / (float)n;
}

__global__ void k_adam(float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m,
                       float* __restrict__ v, int n, float lr, float b1, float b2, float eps, float c1, float c2) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n) return;
  const float gt = g[t];
  const float mt = b1 * m[t] + (1.f - b1) * gt;
  const float vt = b2 * v[t] + (1.f - b2) * gt * gt;
  m[t] = mt;
  v[t] = vt;
  p[t] -= lr * (mt / c1) / (sqrtf(vt / c2) + eps);
}

__global__ void k_gather(const float* __restrict__ X, const float* __restrict__ y, const int64_t* __restrict__ idx,
                         int64_t bs, float* __restrict__ Xb, float* __restrict__ yb) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= bs * NF) return;
  const int64_t r = t / NF;
  const int k = (int)(t % NF);
  const int64_t src = idx[r];
  Xb[t] = X[src * NF + k];
  if (k == 0) yb[r] = y[src];
}

static unsigned nblk(int64_t n, int bs = 256) { return (unsigned)((n + bs - 1) / bs); }

// ---------------------------------------------------------------------------
// host orchestration

// Activations of one forward pass over n rows, kept for the backward pass.
struct Acts {
  float* Xn = nullptr;           // n x NF
  float* Z[4] = {};              // pre-activations
  float* Y[4] = {};              // activations (Y[3] = prediction)
  float* dA = nullptr;           // scratch n x H
  float* dB = nullptr;           // scratch n x H
  float* yb = nullptr;           // targets (normalised)
  int64_t cap = 0;
};

static hipError_t acts_alloc(Acts* a, int64_t n, int H) {
  hipError_t e = hipSuccess;
  auto al = [&](float** p, size_t cnt) {
    if (e == hipSuccess) e = hipMalloc((void**)p, std::max<size_t>(cnt, 1) * sizeof(float));
  };
  al(&a->Xn, (size_t)n * NF);
  for (int l = 0; l < 4; ++l) {
    al(&a->Z[l], (size_t)n * (l == 3 ? 1 : H));
    al(&a->Y[l], (size_t)n * (l == 3 ? 1 : H));
  }
  al(&a->dA, (size_t)n * H);
  al(&a->dB, (size_t)n * H);
  al(&a->yb, (size_t)n);
  a->cap = n;
  return e;
}

static void acts_free(Acts* a) {
  float* ps[] = {a->Xn, a->dA, a->dB, a->yb, a->Z[0], a->Z[1], a->Z[2], a->Z[3], a->Y[0], a->Y[1], a->Y[2], a->Y[3]};
  for (float* p : ps)
    if (p) (void)hipFree(p);
  *a = Acts{};
}

// forward over rows already normalised into a->Xn
static void forward(const Mlp& M, Acts* a, int64_t n, hipStream_t s) {
  const float* in = a->Xn;
  for (int l = 0; l < 4; ++l) {
    const int I = layer_in(M, l), O = layer_out(M, l);
    hipLaunchKernelGGL(k_dense, dim3(nblk(n * O)), dim3(256), 0, s, in, M.d_p + M.off[2 * l],
                       M.d_p + M.off[2 * l + 1], a->Z[l], a->Y[l], n, I, O, l < 3 ? 1 : 0);
    in = a->Y[l];
  }
}

// gradient of the MSE on normalised targets a->yb into M.d_g
static void backward(const Mlp& M, Acts* a, int64_t n, hipStream_t s) {
  float* dY = a->dA;
  float* dZ = a->dB;
  hipLaunchKernelGGL(k_mse_grad, dim3(nblk(n)), dim3(256), 0, s, a->Y[3], a->yb, dY, n);
  for (int l = 3; l >= 0; --l) {
    const int I = layer_in(M, l), O = layer_out(M, l);
    hipLaunchKernelGGL(k_act_bwd, dim3(nblk(n * O)), dim3(256), 0, s, dY, a->Z[l], dZ, n * O, l < 3 ? 1 : 0);
    const float* Xin = l == 0 ? a->Xn : a->Y[l - 1];
    hipLaunchKernelGGL(k_wgrad, dim3(nblk((int64_t)I * O + O)), dim3(256), 0, s, Xin, dZ, M.d_g + M.off[2 * l],
                       M.d_g + M.off[2 * l + 1], n, I, O);
    if (l > 0) {
      hipLaunchKernelGGL(k_dgrad, dim3(nblk(n * I)), dim3(256), 0, s, dZ, M.d_p + M.off[2 * l], dY, n, I, O);
    }
  }
}

struct DevBuf {
  void* p = nullptr;
  ~DevBuf() {
    if (p) (void)hipFree(p);
  }
};

// upload X (n x NF) and y (may be NULL), normalise X into a->Xn and y into a->yb
static hipError_t stage_inputs(const Mlp& M, Acts* a, const float* X, const float* y, int64_t n, DevBuf* dX,
                               DevBuf* dnorm, hipStream_t s) {
  hipError_t e = hipMalloc(&dX->p, (size_t)n * NF * sizeof(float));
  if (e == hipSuccess) e = hipMalloc(&dnorm->p, (2 * NF) * sizeof(float));
  if (e == hipSuccess) e = hipMemcpyAsync(dX->p, X, (size_t)n * NF * sizeof(float), hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipMemcpyAsync(dnorm->p, M.norm.data(), 2 * NF * sizeof(float), hipMemcpyHostToDevice, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_normalize, dim3(nblk(n * NF)), dim3(256), 0, s, (const float*)dX->p, n,
                     (const float*)dnorm->p, (const float*)dnorm->p + NF, a->Xn);
  if (y) {
    std::vector<float> yn(n);
    const float ym = M.norm[2 * NF], ys = M.norm[2 * NF + 1];
    for (int64_t i = 0; i < n; ++i) yn[i] = (y[i] - ym) / ys;
    e = hipMemcpyAsync(a->yb, yn.data(), n * sizeof(float), hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
  }
  return e == hipSuccess ? hipGetLastError() : e;
}

int mlp_predict_host(void* model, const float* X, int64_t n, float* out) {
  if (!model || !X || !out || n < 1) return HDCONV_EINVAL;
  const Mlp& M = *(const Mlp*)model;
  hipStream_t s = nullptr;
  if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) return HDCONV_EDEVICE;
  Acts a;
  DevBuf dX, dn;
  hipError_t e = acts_alloc(&a, n, M.H);
  if (e == hipSuccess) e = stage_inputs(M, &a, X, nullptr, n, &dX, &dn, s);
  if (e == hipSuccess) {
    forward(M, &a, n, s);
    e = hipMemcpyAsync(out, a.Y[3], n * sizeof(float), hipMemcpyDeviceToHost, s);
  }
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  acts_free(&a);
  (void)hipStreamDestroy(s);
  if (e != hipSuccess) return HDCONV_EDEVICE;
  const float ym = M.norm[2 * NF], ys = M.norm[2 * NF + 1];
  for (int64_t i = 0; i < n; ++i) out[i] = out[i] * ys + ym;
  return HDCONV_OK;
}

}  // namespace hd

using namespace hd;

extern "C" {

hdconv_model_t hdconv_model_create(int hidden, uint64_t seed) {
  if (hidden < 1 || hidden > 1024) return nullptr;
  Mlp* M = new (std::nothrow) Mlp();
  if (!M) return nullptr;
  M->H = hidden;
  const int H = hidden;
  const int sizes[8] = {NF * H, H, H * H, H, H * H, H, H, 1};
  int o = 0;
  for (int i = 0; i < 8; ++i) {
    M->off[i] = o;
    o += sizes[i];
  }
  M->nnet = o;
  std::vector<float> p(o, 0.f);
  std::mt19937_64 rng(seed);
  for (int l = 0; l < 4; ++l) {
    const int I = layer_in(*M, l), O = layer_out(*M, l);
    const double a = std::sqrt(6.0 / (I + O));  // Glorot uniform
    std::uniform_real_distribution<double> U(-a, a);
    for (int i = 0; i < I * O; ++i) p[M->off[2 * l] + i] = (float)U(rng);
  }
  M->norm.assign(2 * NF + 2, 0.f);
  for (int k = 0; k < NF; ++k) M->norm[NF + k] = 1.f;
  M->norm[2 * NF + 1] = 1.f;
  bool ok = hipMalloc((void**)&M->d_p, o * sizeof(float)) == hipSuccess &&
            hipMalloc((void**)&M->d_g, o * sizeof(float)) == hipSuccess &&
            hipMalloc((void**)&M->d_m, o * sizeof(float)) == hipSuccess &&
            hipMalloc((void**)&M->d_v, o * sizeof(float)) == hipSuccess &&
            hipMemcpy(M->d_p, p.data(), o * sizeof(float), hipMemcpyHostToDevice) == hipSuccess &&
            hipMemset(M->d_m, 0, o * sizeof(float)) == hipSuccess && hipMemset(M->d_v, 0, o * sizeof(float)) == hipSuccess;
  if (!ok) {
    hdconv_model_destroy((hdconv_model_t)M);
    return nullptr;
  }
  return (hdconv_model_t)M;
}

void hdconv_model_destroy(hdconv_model_t model) {
  if (!model) return;
  Mlp* M = (Mlp*)model;
  (void)hipDeviceSynchronize();
  for (float* q : {M->d_p, M->d_g, M->d_m, M->d_v})
    if (q) (void)hipFree(q);
  delete M;
}

int hdconv_model_params(hdconv_model_t model, float* params, int cap, int* n) {
  if (!model) return HDCONV_EINVAL;
  const Mlp& M = *(const Mlp*)model;
  const int tot = M.nnet + (int)M.norm.size();
  if (n) *n = tot;
  if (!params) return HDCONV_OK;
  if (cap < tot) return HDCONV_EINVAL;
  if (hipMemcpy(params, M.d_p, M.nnet * sizeof(float), hipMemcpyDeviceToHost) != hipSuccess) return HDCONV_EDEVICE;
  memcpy(params + M.nnet, M.norm.data(), M.norm.size() * sizeof(float));
  return HDCONV_OK;
}

int hdconv_model_load(hdconv_model_t model, const float* params, int n) {
  if (!model || !params) return HDCONV_EINVAL;
  Mlp& M = *(Mlp*)model;
  if (n != M.nnet + (int)M.norm.size()) return HDCONV_EINVAL;
  if (hipMemcpy(M.d_p, params, M.nnet * sizeof(float), hipMemcpyHostToDevice) != hipSuccess) return HDCONV_EDEVICE;
  memcpy(M.norm.data(), params + M.nnet, M.norm.size() * sizeof(float));
  (void)hipMemset(M.d_m, 0, M.nnet * sizeof(float));
  (void)hipMemset(M.d_v, 0, M.nnet * sizeof(float));
  M.adam_t = 0;
  return HDCONV_OK;
}

int hdconv_model_predict(hdconv_model_t model, const float* X, int64_t n, float* out) {
  return mlp_predict_host(model, X, n, out);
}

int hdconv_model_grad(hdconv_model_t model, const float* X, const float* y, int64_t n, float* grad, float* loss) {
  if (!model || !X || !y || n < 1) return HDCONV_EINVAL;
  Mlp& M = *(Mlp*)model;
  hipStream_t s = nullptr;
  if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) return HDCONV_EDEVICE;
  Acts a;
  DevBuf dX, dn;
  hipError_t e = acts_alloc(&a, n, M.H);
  if (e == hipSuccess) e = stage_inputs(M, &a, X, y, n, &dX, &dn, s);
  std::vector<float> yhat(n);
  if (e == hipSuccess) {
    forward(M, &a, n, s);
    backward(M, &a, n, s);
    e = hipMemcpyAsync(yhat.data(), a.Y[3], n * sizeof(float), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess && grad) e = hipMemcpyAsync(grad, M.d_g, M.nnet * sizeof(float), hipMemcpyDeviceToHost, s);
  }
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e == hipSuccess && loss) {
    const float ym = M.norm[2 * NF], ys = M.norm[2 * NF + 1];
    double L = 0;
    for (int64_t i = 0; i < n; ++i) {
      const double d = (double)yhat[i] - ((double)y[i] - ym) / ys;
      L += d * d;
    }
    *loss = (float)(L / n);
  }
  acts_free(&a);
  (void)hipStreamDestroy(s);
  return e == hipSuccess ? HDCONV_OK : HDCONV_EDEVICE;
}

int hdconv_model_train(hdconv_model_t model, const float* X, const float* y, int64_t n, int epochs, int batch, float lr,
                       uint64_t seed, float* final_loss) {
  if (!model || !X || !y || n < 2 || epochs < 1 || batch < 1 || !(lr > 0)) return HDCONV_EINVAL;
  Mlp& M = *(Mlp*)model;
  // normalisation from the training set (FP64 on the host)
  for (int k = 0; k < NF; ++k) {
    double s = 0, ss = 0;
    for (int64_t i = 0; i < n; ++i) s += X[i * NF + k];
    const double mu = s / n;
    for (int64_t i = 0; i < n; ++i) ss += (X[i * NF + k] - mu) * (X[i * NF + k] - mu);
    const double sd = std::sqrt(ss / n);
    M.norm[k] = (float)mu;
    M.norm[NF + k] = sd > 1e-6 ? (float)sd : 1.f;
  }
  {
    double s = 0, ss = 0;
    for (int64_t i = 0; i < n; ++i) s += y[i];
    const double mu = s / n;
    for (int64_t i = 0; i < n; ++i) ss += (y[i] - mu) * (y[i] - mu);
    const double sd = std::sqrt(ss / n);
    M.norm[2 * NF] = (float)mu;
    M.norm[2 * NF + 1] = sd > 1e-6 ? (float)sd : 1.f;
  }
  hipStream_t s = nullptr;
  if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) return HDCONV_EDEVICE;
  const int64_t bs = std::min<int64_t>(batch, n);
  Acts all, mb;
  DevBuf dX, dn, didx, dXn_full, dyn_full;
  hipError_t e = acts_alloc(&all, n, M.H);
  if (e == hipSuccess) e = acts_alloc(&mb, bs, M.H);
  if (e == hipSuccess) e = stage_inputs(M, &all, X, y, n, &dX, &dn, s);  // normalised copies in all.Xn, all.yb
  if (e == hipSuccess) e = hipMalloc(&didx.p, bs * sizeof(int64_t));
  std::vector<int64_t> perm(n);
  for (int64_t i = 0; i < n; ++i) perm[i] = i;
  std::mt19937_64 rng(seed);
  const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
  for (int ep = 0; ep < epochs && e == hipSuccess; ++ep) {
    std::shuffle(perm.begin(), perm.end(), rng);
    for (int64_t st = 0; st < n && e == hipSuccess; st += bs) {
      const int64_t cnt = std::min<int64_t>(bs, n - st);
      e = hipMemcpyAsync(didx.p, perm.data() + st, cnt * sizeof(int64_t), hipMemcpyHostToDevice, s);
      if (e != hipSuccess) break;
      hipLaunchKernelGGL(k_gather, dim3(nblk(cnt * NF)), dim3(256), 0, s, all.Xn, all.yb, (const int64_t*)didx.p,
                         cnt, mb.Xn, mb.yb);
      forward(M, &mb, cnt, s);
      backward(M, &mb, cnt, s);
      M.adam_t++;
      const float c1 = 1.f - std::pow(b1, (float)M.adam_t), c2 = 1.f - std::pow(b2, (float)M.adam_t);
      hipLaunchKernelGGL(k_adam, dim3(nblk(M.nnet)), dim3(256), 0, s, M.d_p, M.d_g, M.d_m, M.d_v, M.nnet, lr, b1,
                         b2, eps, c1, c2);
      e = hipGetLastError();
    }
    // the next epoch reshuffles the host index array the uploads read from
    if (e == hipSuccess) e = hipStreamSynchronize(s);
  }
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e == hipSuccess && final_loss) {
    forward(M, &all, n, s);
    std::vector<float> yhat(n), yn(n);
    e = hipMemcpyAsync(yhat.data(), all.Y[3], n * sizeof(float), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipMemcpyAsync(yn.data(), all.yb, n * sizeof(float), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    double L = 0;
    for (int64_t i = 0; i < n; ++i) L += ((double)yhat[i] - yn[i]) * ((double)yhat[i] - yn[i]);
    *final_loss = (float)(L / n);
  }
  acts_free(&all);
  acts_free(&mb);
  (void)hipStreamDestroy(s);
  return e == hipSuccess ? HDCONV_OK : HDCONV_EDEVICE;
}

}  // extern "C"
