// Learned cost model: a small fully connected network trained on the GPU.
//
// widths[0] -> widths[1] -> ... -> widths[n-1], ReLU after every layer but the
// last, fp32.  Forward keeps every layer's pre-activation for the backward
// pass; backward computes dL/dW, dL/db and dL/dx layer by layer; Adam updates
// the packed parameters.  Every reduction runs in a fixed order in one
// thread (no atomics), so results are reproducible run to run.
#include <cmath>
#include <cstring>

#include "../../include/ficgcn.h"
#include "internal.h"

struct ficgcn_mlp {
  ckks_ctx* ctx = nullptr;
  std::vector<uint32_t> w;        // widths
  std::vector<size_t> w_off, b_off;
  size_t n_params = 0;
  float* p = nullptr;             // parameters
  float* g = nullptr;             // gradient
  float* m = nullptr;             // Adam moments
  float* v = nullptr;
  int step = 0;
  // per-layer activations of the last forward: act[0] = x (copied), z[j] = pre-activation of layer j
  std::vector<float*> act, z, dz;
  size_t cap_rows = 0;
  float* loss_dev = nullptr;
  ~ficgcn_mlp();
};

namespace ficgcn {

constexpr int MT = 256;

// Z[r][o] = b[o] + sum_i X[r][i] W[o][i];  A = relu(Z) (or Z on the last layer)
__global__ void k_lin_fwd(const float* __restrict__ X, const float* __restrict__ W, const float* __restrict__ b,
                          float* __restrict__ Z, float* __restrict__ A, int rows, int n_in, int n_out, int relu) {
  const int idx = blockIdx.x * MT + threadIdx.x;
  if (idx >= rows * n_out) return;
  const int r = idx / n_out, o = idx - r * n_out;
  const float* x = X + (size_t)r * n_in;
  const float* w = W + (size_t)o * n_in;
  float s = b[o];
  for (int i = 0; i < n_in; ++i) s = fmaf(x[i], w[i], s);
  Z[idx] = s;
  A[idx] = relu ? fmaxf(s, 0.0f) : s;
}

// squared error: dA = 2 (yhat - y) / n_total; loss = mean over all entries (one block, fixed order)
__global__ void k_mse(const float* __restrict__ yhat, const float* __restrict__ y, float* __restrict__ dA, int total,
                      float* __restrict__ loss) {
  __shared__ float part[MT];
  float s = 0.0f;
  for (int i = threadIdx.x; i < total; i += MT) {
    const float d = yhat[i] - y[i];
    dA[i] = 2.0f * d / (float)total;
    s = fmaf(d, d, s);
  }
  part[threadIdx.x] = s;
  __syncthreads();
  for (int h = MT / 2; h > 0; h >>= 1) {
    if (threadIdx.x < h) part[threadIdx.x] += part[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) *loss = part[0] / (float)total;
}

// dZ = dA * relu'(Z) (in place on dA when relu)
__global__ void k_relu_bwd(float* __restrict__ dA, const float* __restrict__ Z, int total) {
  const int i = blockIdx.x * MT + threadIdx.x;
  if (i < total && Z[i] <= 0.0f) dA[i] = 0.0f;
}

// dW[o][i] = sum_r dZ[r][o] X[r][i];  db[o] = sum_r dZ[r][o]
__global__ void k_lin_bwd_w(const float* __restrict__ dZ, const float* __restrict__ X, float* __restrict__ dW,
                            float* __restrict__ db, int rows, int n_in, int n_out) {
  const int idx = blockIdx.x * MT + threadIdx.x;
  if (idx >= n_out * (n_in + 1)) return;
  const int o = idx / (n_in + 1), i = idx - o * (n_in + 1);
  float s = 0.0f;
  if (i < n_in) {
    for (int r = 0; r < rows; ++r) s = fmaf(dZ[(size_t)r * n_out + o], X[(size_t)r * n_in + i], s);
    dW[(size_t)o * n_in + i] = s;
  } else {
    for (int r = 0; r < rows; ++r) s += dZ[(size_t)r * n_out + o];
    db[o] = s;
  }
}

// dX[r][i] = sum_o dZ[r][o] W[o][i]
__global__ void k_lin_bwd_x(const float* __restrict__ dZ, const float* __restrict__ W, float* __restrict__ dX, int rows,
                            int n_in, int n_out) {
  const int idx = blockIdx.x * MT + threadIdx.x;
  if (idx >= rows * n_in) return;
  const int r = idx / n_in, i = idx - r * n_in;
  float s = 0.0f;
  for (int o = 0; o < n_out; ++o) s = fmaf(dZ[(size_t)r * n_out + o], W[(size_t)o * n_in + i], s);
  dX[idx] = s;
}

__global__ void k_adam(float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m, float* __restrict__ v,
                       int n, float lr, float b1, float b2, float eps, float c1, float c2) {
  const int i = blockIdx.x * MT + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.0f - b1) * gi;
  const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

static unsigned blocks(size_t n) { return (unsigned)((n + MT - 1) / MT); }

static void ensure_rows(ficgcn_mlp* a, size_t rows) {
  if (rows <= a->cap_rows) return;
  for (float* q : a->act) (void)hipFree(q);
  for (float* q : a->z) (void)hipFree(q);
  for (float* q : a->dz) (void)hipFree(q);
  const size_t nl = a->w.size();
  a->act.assign(nl, nullptr);
  a->z.assign(nl, nullptr);
  a->dz.assign(nl, nullptr);
  for (size_t j = 0; j < nl; ++j) {
    HIPCHECK(hipMalloc(&a->act[j], rows * a->w[j] * 4));
    HIPCHECK(hipMalloc(&a->z[j], rows * a->w[j] * 4));
    HIPCHECK(hipMalloc(&a->dz[j], rows * a->w[j] * 4));
  }
  a->cap_rows = rows;
}

static void forward(ficgcn_mlp* a, const float* x, size_t rows) {
  ensure_rows(a, rows);
  hipStream_t st = a->ctx->stream;
  HIPCHECK(hipMemcpyAsync(a->act[0], x, rows * a->w[0] * 4, hipMemcpyDeviceToDevice, st));
  const size_t nl = a->w.size();
  for (size_t j = 0; j + 1 < nl; ++j) {
    const int ni = (int)a->w[j], no = (int)a->w[j + 1];
    hipLaunchKernelGGL(k_lin_fwd, dim3(blocks(rows * no)), dim3(MT), 0, st, a->act[j], a->p + a->w_off[j],
                       a->p + a->b_off[j], a->z[j + 1], a->act[j + 1], (int)rows, ni, no, j + 2 < nl ? 1 : 0);
    HIPCHECK(hipGetLastError());
  }
}

// loss and gradient into a->g (device), loss into a->loss_dev
static void backward(ficgcn_mlp* a, const float* y, size_t rows) {
  hipStream_t st = a->ctx->stream;
  const size_t nl = a->w.size();
  const int total = (int)(rows * a->w[nl - 1]);
  hipLaunchKernelGGL(k_mse, dim3(1), dim3(MT), 0, st, a->act[nl - 1], y, a->dz[nl - 1], total, a->loss_dev);
  HIPCHECK(hipGetLastError());
  for (size_t j = nl - 1; j >= 1; --j) {
    const int ni = (int)a->w[j - 1], no = (int)a->w[j];
    if (j + 1 < nl) {
      hipLaunchKernelGGL(k_relu_bwd, dim3(blocks(rows * no)), dim3(MT), 0, st, a->dz[j], a->z[j], (int)(rows * no));
      HIPCHECK(hipGetLastError());
    }
    hipLaunchKernelGGL(k_lin_bwd_w, dim3(blocks((size_t)no * (ni + 1))), dim3(MT), 0, st, a->dz[j], a->act[j - 1],
                       a->g + a->w_off[j - 1], a->g + a->b_off[j - 1], (int)rows, ni, no);
    HIPCHECK(hipGetLastError());
    if (j >= 2) {
      hipLaunchKernelGGL(k_lin_bwd_x, dim3(blocks(rows * ni)), dim3(MT), 0, st, a->dz[j], a->p + a->w_off[j - 1],
                         a->dz[j - 1], (int)rows, ni, no);
      HIPCHECK(hipGetLastError());
    }
  }
}

void mlp_predict(ficgcn_mlp* a, const float* x_dev, size_t rows, float* y_dev) {
  forward(a, x_dev, rows);
  const size_t nl = a->w.size();
  HIPCHECK(hipMemcpyAsync(y_dev, a->act[nl - 1], rows * a->w[nl - 1] * 4, hipMemcpyDeviceToDevice,
                          a->ctx->stream));
}

}  // namespace ficgcn

ficgcn_mlp::~ficgcn_mlp() {
  if (ctx && ctx->stream) (void)hipStreamSynchronize(ctx->stream);
  for (float* q : {p, g, m, v, loss_dev})
    if (q) (void)hipFree(q);
  for (float* q : act) (void)hipFree(q);
  for (float* q : z) (void)hipFree(q);
  for (float* q : dz) (void)hipFree(q);
}

using namespace ficgcn;

static ficgcn_status mlp_status(const Error& e) {
  set_error(e.msg);
  return (ficgcn_status)e.code;
}

#define MLP_TRY try {
#define MLP_END                                       \
  return FICGCN_OK;                                   \
  }                                                   \
  catch (const Error& e) { return mlp_status(e); }    \
  catch (const std::exception& e) {                   \
    set_error(e.what());                              \
    return FICGCN_EINVAL;                             \
  }

extern "C" {

ficgcn_status ficgcn_mlp_create(ckks_ctx* ctx, const uint32_t* widths, uint32_t n_widths, const float* params,
                                ficgcn_mlp** out) {
  MLP_TRY
  if (!ctx || !widths || !params || !out || n_widths < 2) FICGCN_THROW(EINVAL_, "bad argument");
  for (uint32_t j = 0; j < n_widths; ++j)
    if (widths[j] == 0 || widths[j] > 4096) FICGCN_THROW(EINVAL_, "layer width must be in 1..4096");
  ensure_device(ctx);
  std::unique_ptr<ficgcn_mlp> a(new ficgcn_mlp());
  a->ctx = ctx;
  a->w.assign(widths, widths + n_widths);
  size_t off = 0;
  for (uint32_t j = 0; j + 1 < n_widths; ++j) {
    a->w_off.push_back(off);
    off += (size_t)widths[j] * widths[j + 1];
    a->b_off.push_back(off);
    off += widths[j + 1];
  }
  a->n_params = off;
  for (float** q : {&a->p, &a->g, &a->m, &a->v}) {
    HIPCHECK(hipMalloc(q, off * 4));
  }
  HIPCHECK(hipMalloc(&a->loss_dev, 4));
  HIPCHECK(hipMemcpy(a->p, params, off * 4, hipMemcpyHostToDevice));
  HIPCHECK(hipMemset(a->m, 0, off * 4));
  HIPCHECK(hipMemset(a->v, 0, off * 4));
  *out = a.release();
  MLP_END
}

void ficgcn_mlp_destroy(ficgcn_mlp* mlp) { delete mlp; }

ficgcn_status ficgcn_mlp_param_count(const ficgcn_mlp* mlp, size_t* n_out) {
  MLP_TRY
  if (!mlp || !n_out) FICGCN_THROW(EINVAL_, "null argument");
  *n_out = mlp->n_params;
  MLP_END
}

ficgcn_status ficgcn_mlp_get_params(const ficgcn_mlp* mlp, float* params_out) {
  MLP_TRY
  if (!mlp || !params_out) FICGCN_THROW(EINVAL_, "null argument");
  HIPCHECK(hipStreamSynchronize(mlp->ctx->stream));
  HIPCHECK(hipMemcpy(params_out, mlp->p, mlp->n_params * 4, hipMemcpyDeviceToHost));
  MLP_END
}

ficgcn_status ficgcn_mlp_forward(ficgcn_mlp* mlp, const float* x_dev, uint32_t n, float* y_dev) {
  MLP_TRY
  if (!mlp || !x_dev || !y_dev || n == 0) FICGCN_THROW(EINVAL_, "bad argument");
  mlp_predict(mlp, x_dev, n, y_dev);
  MLP_END
}

ficgcn_status ficgcn_mlp_gradient(ficgcn_mlp* mlp, const float* x_dev, const float* y_dev, uint32_t n,
                                  float* loss_out, float* grad_out) {
  MLP_TRY
  if (!mlp || !x_dev || !y_dev || !loss_out || !grad_out || n == 0) FICGCN_THROW(EINVAL_, "bad argument");
  forward(mlp, x_dev, n);
  backward(mlp, y_dev, n);
  HIPCHECK(hipStreamSynchronize(mlp->ctx->stream));
  HIPCHECK(hipMemcpy(loss_out, mlp->loss_dev, 4, hipMemcpyDeviceToHost));
  HIPCHECK(hipMemcpy(grad_out, mlp->g, mlp->n_params * 4, hipMemcpyDeviceToHost));
  MLP_END
}

ficgcn_status ficgcn_mlp_train_step(ficgcn_mlp* mlp, const float* x_dev, const float* y_dev, uint32_t n, float lr,
                                    float* loss_out) {
  MLP_TRY
  if (!mlp || !x_dev || !y_dev || n == 0 || !(lr > 0.0f)) FICGCN_THROW(EINVAL_, "bad argument");
  forward(mlp, x_dev, n);
  backward(mlp, y_dev, n);
  mlp->step += 1;
  const float b1 = 0.9f, b2 = 0.999f;
  const float c1 = 1.0f - std::pow(b1, (float)mlp->step), c2 = 1.0f - std::pow(b2, (float)mlp->step);
  hipLaunchKernelGGL(k_adam, dim3(blocks(mlp->n_params)), dim3(MT), 0, mlp->ctx->stream, mlp->p, mlp->g, mlp->m,
                     mlp->v, (int)mlp->n_params, lr, b1, b2, 1e-8f, c1, c2);
  HIPCHECK(hipGetLastError());
  if (loss_out) {
    HIPCHECK(hipStreamSynchronize(mlp->ctx->stream));
    HIPCHECK(hipMemcpy(loss_out, mlp->loss_dev, 4, hipMemcpyDeviceToHost));
  }
  MLP_END
}

}  // extern "C"
