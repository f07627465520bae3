// Small multilayer perceptron trained and evaluated on the GPU (FP32): the
// learned parameter proposer predicts log10 errors of ESP results from the
// method parameters and a few system features.
//
// Layers: x -> tanh(W1 x + b1) -> tanh(W2 h1 + b2) -> ... -> W_L h + b_L.
// Parameters are one flat device array, layer by layer (W as nout x nin
// row-major, then b).  Training minimises the masked mean squared error
// sum_b sum_o mask[b,o] (y - t)^2 / sum mask with Adam.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstring>
#include <new>
#include <vector>

#include "../../include/esp.h"

namespace {

constexpr int kMaxLayers = 8;

struct Mlp {
  int nlayer = 0;                   // number of weight layers
  int dims[kMaxLayers + 1] = {};    // dims[0] = nin, dims[nlayer] = nout
  int64_t woff[kMaxLayers] = {}, boff[kMaxLayers] = {};
  int64_t nparam = 0;
  float* w = nullptr;               // parameters
  float* g = nullptr;               // gradient
  float* m = nullptr;               // Adam first moment
  float* v = nullptr;               // Adam second moment
  float* act = nullptr;             // activations of every layer for the current batch
  float* dact = nullptr;            // their gradients
  float* loss = nullptr;            // [0]: loss of the last step
  int64_t cap = 0;                  // batch capacity of act / dact
  int64_t step = 0;
  hipStream_t stream = nullptr;
  int64_t act_off[kMaxLayers + 1] = {};
  int64_t act_per_row = 0;
};

// ---------------------------------------------------------------- kernels
__global__ void k_dense_fwd(const float* __restrict__ x, const float* __restrict__ W,
                            const float* __restrict__ b, float* __restrict__ y, int64_t B, int nin,
                            int nout, int tanh_act) {
  const int64_t t = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= B * nout) return;
  const int64_t r = t / nout;
  const int o = static_cast<int>(t - r * nout);
  const float* xr = x + r * nin;
  const float* wo = W + static_cast<int64_t>(o) * nin;
  float s = b[o];
  for (int i = 0; i < nin; ++i) s += wo[i] * xr[i];
  y[t] = tanh_act ? tanhf(s) : s;
}

// dy = 2 mask (y - t) / sum(mask); partial loss sums per block
__global__ void k_mse_grad(const float* __restrict__ y, const float* __restrict__ t,
                           const float* __restrict__ mask, float* __restrict__ dy, int64_t n,
                           float inv_count, float* __restrict__ loss) {
  __shared__ float red[256];
  float acc = 0.f;
  for (int64_t k = threadIdx.x; k < n; k += blockDim.x) {
    const float mk = mask ? mask[k] : 1.f;
    const float e = y[k] - t[k];
    dy[k] = 2.f * mk * e * inv_count;
    acc += mk * e * e;
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int off = blockDim.x / 2; off > 0; off >>= 1) {
    if (static_cast<int>(threadIdx.x) < off) red[threadIdx.x] += red[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) loss[0] = red[0] * inv_count;
}

// turn dy into the gradient at the pre-activation: dz = dy (1 - y^2) for tanh
__global__ void k_tanh_back(const float* __restrict__ y, float* __restrict__ dy, int64_t n) {
  const int64_t k = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (k < n) dy[k] *= 1.f - y[k] * y[k];
}

// dx[b, i] = sum_o dz[b, o] W[o, i]
__global__ void k_dense_bwd_x(const float* __restrict__ dz, const float* __restrict__ W,
                              float* __restrict__ dx, int64_t B, int nin, int nout) {
  const int64_t t = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= B * nin) return;
  const int64_t r = t / nin;
  const int i = static_cast<int>(t - r * nin);
  const float* dr = dz + r * nout;
  float s = 0.f;
  for (int o = 0; o < nout; ++o) s += dr[o] * W[static_cast<int64_t>(o) * nin + i];
  dx[t] = s;
}

// dW[o, i] = sum_b dz[b, o] x[b, i]; db[o] = sum_b dz[b, o]  (one thread per weight,
// fixed summation order)
__global__ void k_dense_bwd_w(const float* __restrict__ dz, const float* __restrict__ x,
                              float* __restrict__ dW, float* __restrict__ db, int64_t B, int nin,
                              int nout) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nout * (nin + 1)) return;
  const int o = t / (nin + 1), i = t - o * (nin + 1);
  float s = 0.f;
  if (i < nin)
    for (int64_t r = 0; r < B; ++r) s += dz[r * nout + o] * x[r * nin + i];
  else
    for (int64_t r = 0; r < B; ++r) s += dz[r * nout + o];
  if (i < nin) dW[static_cast<int64_t>(o) * nin + i] = s; else db[o] = s;
}

__global__ void k_adam(float* __restrict__ w, const float* __restrict__ g, float* __restrict__ m,
                       float* __restrict__ v, int64_t n, float lr, float b1, float b2, float eps,
                       float c1, float c2) {
  const int64_t k = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (k >= n) return;
  const float gk = g[k];
  const float mk = b1 * m[k] + (1.f - b1) * gk;
  const float vk = b2 * v[k] + (1.f - b2) * gk * gk;
  m[k] = mk;
  v[k] = vk;
  w[k] -= lr * (mk / c1) / (sqrtf(vk / c2) + eps);
}

inline int nblk(int64_t n, int t = 256) { return static_cast<int>((n + t - 1) / t); }

esp_status ensure_cap(Mlp* p, int64_t B) {
  if (B <= p->cap) return ESP_OK;
  if (p->act) (void)hipFree(p->act);
  if (p->dact) (void)hipFree(p->dact);
  p->act = p->dact = nullptr;
  p->cap = 0;
  if (hipMalloc(&p->act, B * p->act_per_row * sizeof(float)) != hipSuccess) return ESP_ENOMEM;
  if (hipMalloc(&p->dact, B * p->act_per_row * sizeof(float)) != hipSuccess) return ESP_ENOMEM;
  p->cap = B;
  return ESP_OK;
}

// forward of a batch; activations of layer l at act + B * act_off[l]
hipError_t forward(Mlp* p, const float* x, int64_t B, float* y_out) {
  const float* in = x;
  for (int l = 0; l < p->nlayer; ++l) {
    const int nin = p->dims[l], nout = p->dims[l + 1];
    const bool last = l == p->nlayer - 1;
    float* out = (last && y_out) ? y_out : p->act + B * p->act_off[l + 1];
    hipLaunchKernelGGL(k_dense_fwd, dim3(nblk(B * nout)), dim3(256), 0, p->stream, in, p->w + p->woff[l],
                       p->w + p->boff[l], out, B, nin, nout, last ? 0 : 1);
    in = out;
  }
  return hipGetLastError();
}

hipError_t backward(Mlp* p, const float* x, const float* t, const float* mask, int64_t B) {
  const int L = p->nlayer;
  const int nout = p->dims[L];
  float* y = p->act + B * p->act_off[L];
  float* dy = p->dact + B * p->act_off[L];
  float cnt = static_cast<float>(B * nout);
  if (mask) {
    std::vector<float> h(B * nout);
    if (hipMemcpyAsync(h.data(), mask, B * nout * sizeof(float), hipMemcpyDeviceToHost, p->stream) != hipSuccess)
      return hipErrorUnknown;
    if (hipStreamSynchronize(p->stream) != hipSuccess) return hipErrorUnknown;
    cnt = 0.f;
    for (float v : h) cnt += v;
    if (cnt <= 0.f) cnt = 1.f;
  }
  hipLaunchKernelGGL(k_mse_grad, dim3(1), dim3(256), 0, p->stream, y, t, mask, dy, B * nout, 1.f / cnt,
                     p->loss);
  for (int l = L - 1; l >= 0; --l) {
    const int nin = p->dims[l], no = p->dims[l + 1];
    float* dz = p->dact + B * p->act_off[l + 1];
    const float* yl = p->act + B * p->act_off[l + 1];
    if (l != L - 1) hipLaunchKernelGGL(k_tanh_back, dim3(nblk(B * no)), dim3(256), 0, p->stream, yl, dz, B * no);
    const float* xin = l == 0 ? x : p->act + B * p->act_off[l];
    hipLaunchKernelGGL(k_dense_bwd_w, dim3(nblk(no * (nin + 1))), dim3(256), 0, p->stream, dz, xin,
                       p->g + p->woff[l], p->g + p->boff[l], B, nin, no);
    if (l > 0)
      hipLaunchKernelGGL(k_dense_bwd_x, dim3(nblk(B * nin)), dim3(256), 0, p->stream, dz, p->w + p->woff[l],
                         p->dact + B * p->act_off[l], B, nin, no);
  }
  return hipGetLastError();
}

// xorshift64* for deterministic initialisation
double urand(uint64_t& s) {
  s ^= s >> 12;
  s ^= s << 25;
  s ^= s >> 27;
  return static_cast<double>((s * 2685821657736338717ULL) >> 11) * (1.0 / 9007199254740992.0);
}

}  // namespace

struct esp_mlp_s : Mlp {};

extern "C" {

esp_status esp_mlp_create(int nlayer, const int* dims, uint64_t seed, esp_mlp_t** out) {
  if (!out || !dims || nlayer < 1 || nlayer > kMaxLayers) return ESP_EINVAL;
  *out = nullptr;
  esp_mlp_s* p = new (std::nothrow) esp_mlp_s();
  if (!p) return ESP_ENOMEM;
  p->nlayer = nlayer;
  int64_t off = 0, aoff = 0;
  for (int l = 0; l <= nlayer; ++l) {
    if (dims[l] < 1 || dims[l] > 4096) {
      delete p;
      return ESP_EINVAL;
    }
    p->dims[l] = dims[l];
    p->act_off[l] = aoff;
    aoff += dims[l];
  }
  p->act_per_row = aoff;
  for (int l = 0; l < nlayer; ++l) {
    p->woff[l] = off;
    off += static_cast<int64_t>(dims[l]) * dims[l + 1];
    p->boff[l] = off;
    off += dims[l + 1];
  }
  p->nparam = off;
  std::vector<float> w(off, 0.f);
  uint64_t s = seed ? seed : 0x9e3779b97f4a7c15ULL;
  for (int l = 0; l < nlayer; ++l) {
    const double a = std::sqrt(6.0 / (dims[l] + dims[l + 1]));   // Glorot uniform
    for (int64_t k = 0; k < static_cast<int64_t>(dims[l]) * dims[l + 1]; ++k)
      w[p->woff[l] + k] = static_cast<float>((2.0 * urand(s) - 1.0) * a);
  }
  bool ok = hipMalloc(&p->w, off * sizeof(float)) == hipSuccess &&
            hipMalloc(&p->g, off * sizeof(float)) == hipSuccess &&
            hipMalloc(&p->m, off * sizeof(float)) == hipSuccess &&
            hipMalloc(&p->v, off * sizeof(float)) == hipSuccess &&
            hipMalloc(&p->loss, 4 * sizeof(float)) == hipSuccess;
  ok = ok && hipMemcpy(p->w, w.data(), off * sizeof(float), hipMemcpyHostToDevice) == hipSuccess &&
       hipMemset(p->m, 0, off * sizeof(float)) == hipSuccess && hipMemset(p->v, 0, off * sizeof(float)) == hipSuccess &&
       hipMemset(p->g, 0, off * sizeof(float)) == hipSuccess;
  if (!ok) {
    esp_mlp_destroy(p);
    return ESP_ENOMEM;
  }
  *out = p;
  return ESP_OK;
}

int64_t esp_mlp_num_params(const esp_mlp_t* p) { return p ? p->nparam : -1; }

esp_status esp_mlp_set_params(esp_mlp_t* p, const float* host, int64_t n) {
  if (!p || !host || n != p->nparam) return ESP_EINVAL;
  return hipMemcpy(p->w, host, n * sizeof(float), hipMemcpyHostToDevice) == hipSuccess ? ESP_OK : ESP_EDEVICE;
}

esp_status esp_mlp_get_params(const esp_mlp_t* p, float* host, int64_t n) {
  if (!p || !host || n != p->nparam) return ESP_EINVAL;
  if (hipStreamSynchronize(p->stream) != hipSuccess) return ESP_EDEVICE;
  return hipMemcpy(host, p->w, n * sizeof(float), hipMemcpyDeviceToHost) == hipSuccess ? ESP_OK : ESP_EDEVICE;
}

esp_status esp_mlp_set_stream(esp_mlp_t* p, void* stream) {
  if (!p) return ESP_EINVAL;
  p->stream = static_cast<hipStream_t>(stream);
  return ESP_OK;
}

esp_status esp_mlp_forward(esp_mlp_t* p, const float* x, int64_t B, float* y) {
  if (!p || !x || !y || B < 1) return ESP_EINVAL;
  if (ensure_cap(p, B) != ESP_OK) return ESP_ENOMEM;
  return forward(p, x, B, y) == hipSuccess ? ESP_OK : ESP_EDEVICE;
}

esp_status esp_mlp_gradient(esp_mlp_t* p, const float* x, const float* t, const float* mask, int64_t B,
                            float* grad_out, float* loss_out) {
  if (!p || !x || !t || B < 1) return ESP_EINVAL;
  if (ensure_cap(p, B) != ESP_OK) return ESP_ENOMEM;
  hipError_t e = forward(p, x, B, nullptr);
  if (e == hipSuccess) e = backward(p, x, t, mask, B);
  if (e == hipSuccess && grad_out)
    e = hipMemcpyAsync(grad_out, p->g, p->nparam * sizeof(float), hipMemcpyDeviceToDevice, p->stream);
  if (e == hipSuccess && loss_out)
    e = hipMemcpyAsync(loss_out, p->loss, sizeof(float), hipMemcpyDeviceToDevice, p->stream);
  return e == hipSuccess ? ESP_OK : ESP_EDEVICE;
}

esp_status esp_mlp_train_step(esp_mlp_t* p, const float* x, const float* t, const float* mask, int64_t B,
                              float lr, float* loss_out) {
  esp_status st = esp_mlp_gradient(p, x, t, mask, B, nullptr, loss_out);
  if (st != ESP_OK) return st;
  ++p->step;
  const float b1 = 0.9f, b2 = 0.999f;
  const float c1 = 1.f - std::pow(b1, static_cast<float>(p->step));
  const float c2 = 1.f - std::pow(b2, static_cast<float>(p->step));
  hipLaunchKernelGGL(k_adam, dim3(nblk(p->nparam)), dim3(256), 0, p->stream, p->w, p->g, p->m, p->v, p->nparam,
                     lr, b1, b2, 1e-8f, c1, c2);
  return hipGetLastError() == hipSuccess ? ESP_OK : ESP_EDEVICE;
}

void esp_mlp_destroy(esp_mlp_t* p) {
  if (!p) return;
  (void)hipStreamSynchronize(p->stream);
  for (float* q : {p->w, p->g, p->m, p->v, p->act, p->dact, p->loss})
    if (q) (void)hipFree(q);
  delete p;
}

}  // extern "C"

namespace espx {

// Host-to-host batch evaluation on the network's own stream (plan time only).
esp_status mlp_predict_host(esp_mlp_t* p, const float* xh, int64_t B, float* yh) {
  if (!p || !xh || !yh || B < 1) return ESP_EINVAL;
  const int nin = p->dims[0], nout = p->dims[p->nlayer];
  float *dx = nullptr, *dy = nullptr;
  esp_status st = ESP_EDEVICE;
  if (hipMalloc(&dx, B * nin * sizeof(float)) == hipSuccess && hipMalloc(&dy, B * nout * sizeof(float)) == hipSuccess &&
      hipMemcpyAsync(dx, xh, B * nin * sizeof(float), hipMemcpyHostToDevice, p->stream) == hipSuccess) {
    st = esp_mlp_forward(p, dx, B, dy);
    if (st == ESP_OK &&
        (hipMemcpyAsync(yh, dy, B * nout * sizeof(float), hipMemcpyDeviceToHost, p->stream) != hipSuccess ||
         hipStreamSynchronize(p->stream) != hipSuccess))
      st = ESP_EDEVICE;
  }
  (void)hipStreamSynchronize(p->stream);
  if (dx) (void)hipFree(dx);
  if (dy) (void)hipFree(dy);
  return st;
}

int mlp_dim(const esp_mlp_t* p, int which) { return which == 0 ? p->dims[0] : p->dims[p->nlayer]; }

}  // namespace espx
