// The temperature-step network: a small FP32 multilayer perceptron that
// proposes log(dbeta) for the next annealing step from energy-histogram
// summaries of a population.  Training (forward, backward, Adam) and
// inference run in the hand-written kernels below; the exact bisection on the
// energy-distribution overlap stays the check and the fallback, and the
// reweighting stays exact, so a poor proposal costs time, never bias.
//
//   u   = (x - mu) / sigma
//   h_l = tanh(W_l h_{l-1} + b_l),  l = 1..depth
//   z   = w . h_depth + b            (standardised output)
//   log dbeta = mu_y + sigma_y z
// Parameters: one flat FP32 vector, per layer W (out x in, row-major) then b.
//
// Every kernel is a plain per-element map: one thread per (sample, unit) in
// the forward and delta passes, one thread per weight in the gradient pass
// (a loop over the samples in order, so gradients are deterministic).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstring>
#include <exception>
#include <mutex>
#include <new>
#include <vector>

#include "pa.h"
#include "pa_internal.h"

namespace pa {

__global__ void k_mlp_standardize(const float* X, const int32_t* idx,
                                  const float* T, const float* norm, float* U,
                                  float* Tb, int B, int n_in) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= B * n_in) return;
  const int s = t / n_in, i = t - s * n_in;
  const int src = idx ? idx[s] : s;
  U[t] = (X[(size_t)src * n_in + i] - norm[i]) / norm[n_in + i];
  if (T && i == 0) Tb[s] = (T[src] - norm[2 * n_in]) / norm[2 * n_in + 1];
}

__global__ void k_mlp_fwd(const float* W, const float* b, const float* Hin,
                          float* Hout, int B, int n_in, int n_out, int act) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= B * n_out) return;
  const int s = t / n_out, o = t - s * n_out;
  const float* w = W + (size_t)o * n_in;
  const float* h = Hin + (size_t)s * n_in;
  float z = b[o];
  for (int i = 0; i < n_in; ++i) z = fmaf(w[i], h[i], z);
  Hout[t] = act ? tanhf(z) : z;
}

// d loss / d z for the mean squared error on standardised targets, and the
// per-sample squared residuals (summed on the host).
__global__ void k_mlp_out_delta(const float* z, const float* t, float* dz,
                                float* r2, int B) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= B) return;
  const float r = z[s] - t[s];
  dz[s] = (2.0f / (float)B) * r;
  r2[s] = r * r;
}

// dW[o][i] = sum_s dA[s][o] Hin[s][i]; db[o] = sum_s dA[s][o]  (i == n_in)
__global__ void k_mlp_wgrad(const float* dA, const float* Hin, float* dW,
                            float* db, int B, int n_in, int n_out) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n_out * (n_in + 1)) return;
  const int o = t / (n_in + 1), i = t - o * (n_in + 1);
  float acc = 0.0f;
  if (i < n_in) {
    for (int s = 0; s < B; ++s)
      acc = fmaf(dA[(size_t)s * n_out + o], Hin[(size_t)s * n_in + i], acc);
    dW[(size_t)o * n_in + i] = acc;
  } else {
    for (int s = 0; s < B; ++s) acc += dA[(size_t)s * n_out + o];
    db[o] = acc;
  }
}

// dAprev[s][i] = (sum_o W[o][i] dA[s][o]) (1 - Hprev[s][i]^2)   (through tanh)
__global__ void k_mlp_back(const float* W, const float* dA, const float* Hprev,
                           float* dAprev, int B, int n_in, int n_out) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= B * n_in) return;
  const int s = t / n_in, i = t - s * n_in;
  float acc = 0.0f;
  for (int o = 0; o < n_out; ++o)
    acc = fmaf(W[(size_t)o * n_in + i], dA[(size_t)s * n_out + o], acc);
  const float h = Hprev[t];
  dAprev[t] = acc * (1.0f - h * h);
}

// Adam (Kingma and Ba) with bias-corrected moments; c1 = 1/(1-beta1^t),
// c2 = 1/(1-beta2^t) come from the host.
__global__ void k_mlp_adam(float* p, const float* g, float* m, float* v, int n,
                           float lr, float b1, float b2, float eps, float c1,
                           float c2) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  const float gk = g[k];
  const float mk = b1 * m[k] + (1.0f - b1) * gk;
  const float vk = b2 * v[k] + (1.0f - b2) * gk * gk;
  m[k] = mk;
  v[k] = vk;
  p[k] -= lr * (mk * c1) / (sqrtf(vk * c2) + eps);
}

// y[s] = mu_y + sigma_y z[s] in place, each operation rounded on its own (no
// fused multiply-add), as the host does it for pa_mlp_forward.
__global__ void k_mlp_out_affine(float* y, int B, float mu_y, float sigma_y) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= B) return;
  y[s] = __fadd_rn(mu_y, __fmul_rn(sigma_y, y[s]));
}

static unsigned blocks_for(int64_t n) { return (unsigned)((n + 255) / 256); }

}  // namespace pa

// Activations of pa_mlp_forward_noalloc: two ping-pong slots of
// PA_MLP_NOALLOC_MAX_ELEMS floats (2 MiB in all), one copy on every device
// the library runs on, held until the process ends.  Host code never uses
// this name as an address: the device address comes from
// hipGetSymbolAddress, once per device, and is kept in g_scratch_dev.
static __device__ __align__(256) float scratch[2 * PA_MLP_NOALLOC_MAX_ELEMS];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
float* g_scratch_dev[kMaxDevices] = {};

// Device address of `scratch` on `device`, which must be the current device;
// looked up on the first call for that device.  nullptr on failure.
float* scratch_on(int device) {
  if (device < 0 || device >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_dev[device]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
      (void)hipGetLastError();
      ::pa::set_last_error("hipGetSymbolAddress", e, __LINE__);
      return nullptr;
    }
    g_scratch_dev[device] = static_cast<float*>(p);
  }
  return g_scratch_dev[device];
}

// The address looked up before for `device`, or nullptr.
float* scratch_known(int device) {
  if (device < 0 || device >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  return g_scratch_dev[device];
}

}  // namespace

using namespace pa;

struct pa_mlp {
  int device = 0;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  int n_in = 0, width = 0, depth = 0;
  int64_t n_params = 0;
  std::vector<int64_t> w_off, b_off, fan_in, fan_out;
  float* d_params = nullptr;
  float* d_grad = nullptr;
  float* d_m = nullptr;
  float* d_v = nullptr;
  float* d_norm = nullptr;  // mu[n_in], sigma[n_in], mu_y, sigma_y
  float h_norm[2 * 64 + 2] = {0};
  int64_t adam_t = 0;
  // per-batch scratch (grown on demand)
  int cap_B = 0;
  float *d_X = nullptr, *d_T = nullptr, *d_Tb = nullptr, *d_act = nullptr,
        *d_delta = nullptr, *d_r2 = nullptr;
  int32_t* d_idx = nullptr;
  int64_t act_stride = 0;  // floats per activation slot (B * max width)
  // changes whenever a captured inference would go stale: new scratch
  // addresses or new output scale
  uint64_t gen = 0;
};

namespace {

#define MK(x) PA_HIP(x)

std::atomic<uint64_t> g_generation{0};
void bump(pa_mlp* m) { m->gen = ++g_generation; }

void mlp_free_scratch(pa_mlp* m) {
  void* p[] = {m->d_X, m->d_T, m->d_Tb, m->d_act, m->d_delta, m->d_r2,
               m->d_idx};
  for (void* q : p)
    if (q) (void)hipFree(q);
  m->d_X = m->d_T = m->d_Tb = m->d_act = m->d_delta = m->d_r2 = nullptr;
  m->d_idx = nullptr;
  m->cap_B = 0;
}

int ensure_batch(pa_mlp* m, int B) {
  if (B <= m->cap_B) return PA_OK;
  mlp_free_scratch(m);
  const int wmax = std::max(m->width, m->n_in);
  m->act_stride = (int64_t)B * wmax;
  bool ok = true;
  ok = ok && hipMalloc(&m->d_X, (size_t)B * m->n_in * 4) == hipSuccess;
  ok = ok && hipMalloc(&m->d_T, (size_t)B * 4) == hipSuccess;
  ok = ok && hipMalloc(&m->d_Tb, (size_t)B * 4) == hipSuccess;
  ok = ok && hipMalloc(&m->d_act, (size_t)(m->depth + 2) * m->act_stride * 4) == hipSuccess;
  ok = ok && hipMalloc(&m->d_delta, (size_t)2 * m->act_stride * 4) == hipSuccess;
  ok = ok && hipMalloc(&m->d_r2, (size_t)B * 4) == hipSuccess;
  ok = ok && hipMalloc(&m->d_idx, (size_t)B * 4) == hipSuccess;
  if (!ok) {
    (void)hipGetLastError();  // a failed allocation is no later launch's error
    mlp_free_scratch(m);
    return PA_ENOMEM;
  }
  m->cap_B = B;
  bump(m);
  return PA_OK;
}

float* act_slot(pa_mlp* m, int l) { return m->d_act + (size_t)l * m->act_stride; }

}  // namespace

namespace pa {

// Forward pass of B standardised samples already in activation slot 0; the
// output z lands in slot depth+1.
int mlp_forward_on(pa_mlp* m, int B, hipStream_t st) {
  for (int l = 0; l <= m->depth; ++l) {
    const int n_out = (int)m->fan_out[l], n_in = (int)m->fan_in[l];
    hipLaunchKernelGGL(k_mlp_fwd, dim3(blocks_for((int64_t)B * n_out)),
                       dim3(256), 0, st, m->d_params + m->w_off[l],
                       m->d_params + m->b_off[l], act_slot(m, l),
                       act_slot(m, l + 1), B, n_in, n_out,
                       l < m->depth ? 1 : 0);
    MK(hipGetLastError());
  }
  return PA_OK;
}

int mlp_forward_dev(pa_mlp* m, int B) { return mlp_forward_on(m, B, m->stream); }

// Scratch for batches of up to B samples (allocates; not during a capture).
int mlp_prepare(pa_mlp* m, int B) { return ensure_batch(m, B); }

// Standardise B raw feature rows (device pointer) into slot 0 and run the
// forward pass on stream st; z (standardised) in slot depth+1.  Needs
// mlp_prepare(m, B) first; allocates nothing, so a graph may capture it.
int mlp_infer_on(pa_mlp* m, const float* X, int B, hipStream_t st) {
  if (B > m->cap_B) return PA_EINVAL;
  hipLaunchKernelGGL(k_mlp_standardize, dim3(blocks_for((int64_t)B * m->n_in)),
                     dim3(256), 0, st, X, nullptr, nullptr, m->d_norm,
                     act_slot(m, 0), nullptr, B, m->n_in);
  MK(hipGetLastError());
  return mlp_forward_on(m, B, st);
}

int mlp_infer_dev(pa_mlp* m, const float* X, int B) {
  int rc = ensure_batch(m, B);
  if (rc) return rc;
  return mlp_infer_on(m, X, B, m->stream);
}

const float* mlp_output_dev(pa_mlp* m) { return act_slot(m, m->depth + 1); }
void mlp_out_scale(const pa_mlp* m, float* mu_y, float* sigma_y) {
  *mu_y = m->h_norm[2 * m->n_in];
  *sigma_y = m->h_norm[2 * m->n_in + 1];
}
int mlp_n_in(const pa_mlp* m) { return m->n_in; }
uint64_t mlp_generation(const pa_mlp* m) { return m ? m->gen : 0; }

// Backward pass for B samples whose forward activations are in the slots and
// whose standardised targets are in d_Tb: gradient into d_grad.
int mlp_backward_dev(pa_mlp* m, int B) {
  float* dz = m->d_delta;                      // [B][1]
  float* bufA = m->d_delta;
  float* bufB = m->d_delta + m->act_stride;
  hipLaunchKernelGGL(k_mlp_out_delta, dim3(blocks_for(B)), dim3(256), 0,
                     m->stream, act_slot(m, m->depth + 1), m->d_Tb, dz,
                     m->d_r2, B);
  MK(hipGetLastError());
  float* dA = bufA;
  for (int l = m->depth; l >= 0; --l) {
    const int n_out = (int)m->fan_out[l], n_in = (int)m->fan_in[l];
    hipLaunchKernelGGL(k_mlp_wgrad, dim3(blocks_for((int64_t)n_out * (n_in + 1))),
                       dim3(256), 0, m->stream, dA, act_slot(m, l),
                       m->d_grad + m->w_off[l], m->d_grad + m->b_off[l], B,
                       n_in, n_out);
    MK(hipGetLastError());
    if (l == 0) break;
    float* dPrev = (dA == bufA) ? bufB : bufA;
    hipLaunchKernelGGL(k_mlp_back, dim3(blocks_for((int64_t)B * n_in)),
                       dim3(256), 0, m->stream, m->d_params + m->w_off[l], dA,
                       act_slot(m, l), dPrev, B, n_in, n_out);
    MK(hipGetLastError());
    dA = dPrev;
  }
  return PA_OK;
}

}  // namespace pa

namespace {

// splitmix64, for the initial weights and the minibatch order
uint64_t sm64(uint64_t* s) {
  uint64_t z = (*s += 0x9E3779B97F4A7C15ull);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

}  // namespace

extern "C" {

int pa_mlp_create(int32_t n_in, int32_t width, int32_t depth, uint64_t seed,
                  void* stream, pa_mlp** out) try {
  if (!out) return PA_EINVAL;
  *out = nullptr;
  if (n_in < 1 || n_in > 64 || width < 1 || width > 1024 || depth < 1 ||
      depth > 8)
    return PA_EINVAL;
  pa_mlp* m = new (std::nothrow) pa_mlp();
  if (!m) return PA_ENOMEM;
  if (hipGetDevice(&m->device) != hipSuccess) {
    delete m;
    return PA_EDEVICE;
  }
  // the no-allocation forward pass's scratch address on this device (a
  // failed lookup only disables pa_mlp_forward_noalloc)
  (void)scratch_on(m->device);
  m->stream = reinterpret_cast<hipStream_t>(stream);
  m->n_in = n_in;
  m->width = width;
  m->depth = depth;
  int64_t k = 0;
  int prev = n_in;
  for (int l = 0; l <= depth; ++l) {
    const int o = (l < depth) ? width : 1;
    m->fan_in.push_back(prev);
    m->fan_out.push_back(o);
    m->w_off.push_back(k);
    k += (int64_t)o * prev;
    m->b_off.push_back(k);
    k += o;
    prev = o;
  }
  m->n_params = k;
  // Glorot-uniform weights, zero biases, identity standardisation
  std::vector<float> p((size_t)k, 0.0f);
  uint64_t st = seed ^ 0x5A17ull;
  for (int l = 0; l <= depth; ++l) {
    const double a = std::sqrt(6.0 / (double)(m->fan_in[l] + m->fan_out[l]));
    for (int64_t i = 0; i < m->fan_in[l] * m->fan_out[l]; ++i) {
      const double u = (double)(sm64(&st) >> 11) * (1.0 / 9007199254740992.0);
      p[(size_t)(m->w_off[l] + i)] = (float)((2.0 * u - 1.0) * a);
    }
  }
  for (int i = 0; i < n_in; ++i) {
    m->h_norm[i] = 0.0f;
    m->h_norm[n_in + i] = 1.0f;
  }
  m->h_norm[2 * n_in] = 0.0f;
  m->h_norm[2 * n_in + 1] = 1.0f;
  bool ok = true;
  ok = ok && hipMalloc(&m->d_params, (size_t)k * 4) == hipSuccess;
  ok = ok && hipMalloc(&m->d_grad, (size_t)k * 4) == hipSuccess;
  ok = ok && hipMalloc(&m->d_m, (size_t)k * 4) == hipSuccess;
  ok = ok && hipMalloc(&m->d_v, (size_t)k * 4) == hipSuccess;
  ok = ok && hipMalloc(&m->d_norm, (size_t)(2 * n_in + 2) * 4) == hipSuccess;
  if (ok) {
    std::vector<float> z((size_t)k, 0.0f);
    ok = hipMemcpy(m->d_params, p.data(), (size_t)k * 4, hipMemcpyHostToDevice) == hipSuccess &&
         hipMemcpy(m->d_m, z.data(), (size_t)k * 4, hipMemcpyHostToDevice) == hipSuccess &&
         hipMemcpy(m->d_v, z.data(), (size_t)k * 4, hipMemcpyHostToDevice) == hipSuccess &&
         hipMemcpy(m->d_norm, m->h_norm, (size_t)(2 * n_in + 2) * 4,
                   hipMemcpyHostToDevice) == hipSuccess;
  }
  if (!ok) {
    (void)hipGetLastError();  // a failed allocation is no later launch's error
    pa_mlp_destroy(m);
    return PA_ENOMEM;
  }
  *out = m;
  return PA_OK;
} catch (const std::bad_alloc&) {
  return PA_ENOMEM;
} catch (const std::exception& e) {
  ::pa::note_exception(e.what());
  return PA_EDEVICE;
} catch (...) {
  ::pa::note_exception("unknown exception");
  return PA_EDEVICE;
}

void pa_mlp_destroy(pa_mlp* m) try {
  if (!m) return;
  (void)hipStreamSynchronize(m->stream);
  mlp_free_scratch(m);
  void* p[] = {m->d_params, m->d_grad, m->d_m, m->d_v, m->d_norm};
  for (void* q : p)
    if (q) (void)hipFree(q);
  delete m;
} catch (...) {
}

int pa_mlp_n_params(pa_mlp* m, int64_t* n) try {
  if (!m || !n) return PA_EINVAL;
  *n = m->n_params;
  return PA_OK;
} catch (const std::bad_alloc&) {
  return PA_ENOMEM;
} catch (const std::exception& e) {
  ::pa::note_exception(e.what());
  return PA_EDEVICE;
} catch (...) {
  ::pa::note_exception("unknown exception");
  return PA_EDEVICE;
}

int pa_mlp_set_params(pa_mlp* m, const float* p, int64_t n) try {
  if (!m || !p || n != m->n_params) return PA_EINVAL;
  MK(hipMemcpyAsync(m->d_params, p, (size_t)n * 4, hipMemcpyHostToDevice,
                    m->stream));
  MK(hipStreamSynchronize(m->stream));
  m->adam_t = 0;
  return PA_OK;
} catch (const std::bad_alloc&) {
  return PA_ENOMEM;
} catch (const std::exception& e) {
  ::pa::note_exception(e.what());
  return PA_EDEVICE;
} catch (...) {
  ::pa::note_exception("unknown exception");
  return PA_EDEVICE;
}

int pa_mlp_get_params(pa_mlp* m, float* p, int64_t n) try {
  if (!m || !p || n != m->n_params) return PA_EINVAL;
  MK(hipMemcpyAsync(p, m->d_params, (size_t)n * 4, hipMemcpyDeviceToHost,
                    m->stream));
  MK(hipStreamSynchronize(m->stream));
  return PA_OK;
} catch (const std::bad_alloc&) {
  return PA_ENOMEM;
} catch (const std::exception& e) {
  ::pa::note_exception(e.what());
  return PA_EDEVICE;
} catch (...) {
  ::pa::note_exception("unknown exception");
  return PA_EDEVICE;
}

int pa_mlp_set_norm(pa_mlp* m, const float* mu, const float* sigma,
                    float mu_y, float sigma_y) try {
  if (!m || !mu || !sigma || !(sigma_y > 0.0f)) return PA_EINVAL;
  for (int i = 0; i < m->n_in; ++i) {
    if (!(sigma[i] > 0.0f)) return PA_EINVAL;
    m->h_norm[i] = mu[i];
    m->h_norm[m->n_in + i] = sigma[i];
  }
  m->h_norm[2 * m->n_in] = mu_y;
  m->h_norm[2 * m->n_in + 1] = sigma_y;
  MK(hipMemcpyAsync(m->d_norm, m->h_norm, (size_t)(2 * m->n_in + 2) * 4,
                    hipMemcpyHostToDevice, m->stream));
  MK(hipStreamSynchronize(m->stream));
  bump(m);
  return PA_OK;
} catch (const std::bad_alloc&) {
  return PA_ENOMEM;
} catch (const std::exception& e) {
  ::pa::note_exception(e.what());
  return PA_EDEVICE;
} catch (...) {
  ::pa::note_exception("unknown exception");
  return PA_EDEVICE;
}

int pa_mlp_forward(pa_mlp* m, const float* X, int32_t B, float* y) try {
  if (!m || !X || !y || B < 1) return PA_EINVAL;
  int rc = ensure_batch(m, B);
  if (rc) return rc;
  MK(hipMemcpyAsync(m->d_X, X, (size_t)B * m->n_in * 4, hipMemcpyHostToDevice,
                    m->stream));
  rc = mlp_infer_dev(m, m->d_X, B);
  if (rc) return rc;
  std::vector<float> z((size_t)B);
  MK(hipMemcpyAsync(z.data(), act_slot(m, m->depth + 1), (size_t)B * 4,
                    hipMemcpyDeviceToHost, m->stream));
  MK(hipStreamSynchronize(m->stream));
  const float mu_y = m->h_norm[2 * m->n_in], sy = m->h_norm[2 * m->n_in + 1];
  for (int s = 0; s < B; ++s) y[s] = mu_y + sy * z[(size_t)s];
  return PA_OK;
} catch (const std::bad_alloc&) {
  return PA_ENOMEM;
} catch (const std::exception& e) {
  ::pa::note_exception(e.what());
  return PA_EDEVICE;
} catch (...) {
  ::pa::note_exception("unknown exception");
  return PA_EDEVICE;
}

int pa_mlp_forward_noalloc(pa_mlp* m, const float* X, int32_t B,
                           float* y) try {
  if (!m || !X || !y || B < 1) return PA_EINVAL;
  const int64_t wmax = std::max(m->width, m->n_in);
  if ((int64_t)B * wmax > PA_MLP_NOALLOC_MAX_ELEMS) {
    note_error("pa_mlp_forward_noalloc: batch x max(width, n_in) exceeds "
               "PA_MLP_NOALLOC_MAX_ELEMS");
    return PA_EINVAL;
  }
  float* base = scratch_known(m->device);  // looked up by pa_mlp_create
  if (!base) {
    note_error("pa_mlp_forward_noalloc: no scratch address for the device");
    return PA_EDEVICE;
  }
  float* slot[2] = {base, base + PA_MLP_NOALLOC_MAX_ELEMS};
  hipLaunchKernelGGL(k_mlp_standardize, dim3(blocks_for((int64_t)B * m->n_in)),
                     dim3(256), 0, m->stream, X, nullptr, nullptr, m->d_norm,
                     slot[0], nullptr, B, m->n_in);
  MK(hipGetLastError());
  for (int l = 0; l <= m->depth; ++l) {
    const int n_out = (int)m->fan_out[l], n_in = (int)m->fan_in[l];
    float* out = (l == m->depth) ? y : slot[(l + 1) & 1];
    hipLaunchKernelGGL(k_mlp_fwd, dim3(blocks_for((int64_t)B * n_out)),
                       dim3(256), 0, m->stream, m->d_params + m->w_off[l],
                       m->d_params + m->b_off[l], slot[l & 1], out, B, n_in,
                       n_out, l < m->depth ? 1 : 0);
    MK(hipGetLastError());
  }
  hipLaunchKernelGGL(k_mlp_out_affine, dim3(blocks_for(B)), dim3(256), 0,
                     m->stream, y, B, m->h_norm[2 * m->n_in],
                     m->h_norm[2 * m->n_in + 1]);
  MK(hipGetLastError());
  return PA_OK;
} catch (const std::bad_alloc&) {
  return PA_ENOMEM;
} catch (const std::exception& e) {
  ::pa::note_exception(e.what());
  return PA_EDEVICE;
} catch (...) {
  ::pa::note_exception("unknown exception");
  return PA_EDEVICE;
}

int pa_mlp_loss_grad(pa_mlp* m, const float* X, const float* T, int32_t B,
                     float* loss, float* grad) try {
  if (!m || !X || !T || B < 1) return PA_EINVAL;
  int rc = ensure_batch(m, B);
  if (rc) return rc;
  MK(hipMemcpyAsync(m->d_X, X, (size_t)B * m->n_in * 4, hipMemcpyHostToDevice,
                    m->stream));
  MK(hipMemcpyAsync(m->d_T, T, (size_t)B * 4, hipMemcpyHostToDevice,
                    m->stream));
  hipLaunchKernelGGL(k_mlp_standardize, dim3(blocks_for((int64_t)B * m->n_in)),
                     dim3(256), 0, m->stream, m->d_X, nullptr, m->d_T,
                     m->d_norm, act_slot(m, 0), m->d_Tb, B, m->n_in);
  MK(hipGetLastError());
  rc = mlp_forward_dev(m, B);
  if (!rc) rc = mlp_backward_dev(m, B);
  if (rc) return rc;
  std::vector<float> r2((size_t)B);
  MK(hipMemcpyAsync(r2.data(), m->d_r2, (size_t)B * 4, hipMemcpyDeviceToHost,
                    m->stream));
  if (grad)
    MK(hipMemcpyAsync(grad, m->d_grad, (size_t)m->n_params * 4,
                      hipMemcpyDeviceToHost, m->stream));
  MK(hipStreamSynchronize(m->stream));
  if (loss) {
    double acc = 0.0;
    for (int s = 0; s < B; ++s) acc += r2[(size_t)s];
    *loss = (float)(acc / B);
  }
  return PA_OK;
} catch (const std::bad_alloc&) {
  return PA_ENOMEM;
} catch (const std::exception& e) {
  ::pa::note_exception(e.what());
  return PA_EDEVICE;
} catch (...) {
  ::pa::note_exception("unknown exception");
  return PA_EDEVICE;
}

int pa_mlp_train(pa_mlp* m, const float* X, const float* T, int64_t n,
                 int32_t batch, int32_t iters, float lr, uint64_t seed,
                 float* loss_out) try {
  if (!m || !X || !T || n < 1 || batch < 1 || iters < 1 || !(lr > 0.0f))
    return PA_EINVAL;
  const int B = (int)std::min<int64_t>(batch, n);
  int rc = ensure_batch(m, B);
  if (rc) return rc;
  float *dXall = nullptr, *dTall = nullptr;
  int32_t* dIdx = nullptr;
  MK(hipMalloc(&dXall, (size_t)n * m->n_in * 4));
  if (hipMalloc(&dTall, (size_t)n * 4) != hipSuccess ||
      hipMalloc(&dIdx, (size_t)iters * B * 4) != hipSuccess) {
    (void)hipFree(dXall);
    if (dTall) (void)hipFree(dTall);
    return PA_ENOMEM;
  }
  // minibatch order: successive shuffled passes over the data
  std::vector<int32_t> order((size_t)n), idx((size_t)iters * B);
  uint64_t st = seed;
  size_t pos = (size_t)n;
  for (size_t k = 0; k < idx.size(); ++k) {
    if (pos == (size_t)n) {
      for (int64_t i = 0; i < n; ++i) order[(size_t)i] = (int32_t)i;
      for (int64_t i = n - 1; i > 0; --i) {
        const int64_t j = (int64_t)(sm64(&st) % (uint64_t)(i + 1));
        std::swap(order[(size_t)i], order[(size_t)j]);
      }
      pos = 0;
    }
    idx[k] = order[pos++];
  }
  rc = PA_OK;
  auto run = [&]() -> int {
    MK(hipMemcpyAsync(dXall, X, (size_t)n * m->n_in * 4, hipMemcpyHostToDevice,
                      m->stream));
    MK(hipMemcpyAsync(dTall, T, (size_t)n * 4, hipMemcpyHostToDevice,
                      m->stream));
    MK(hipMemcpyAsync(dIdx, idx.data(), idx.size() * 4, hipMemcpyHostToDevice,
                      m->stream));
    const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
    for (int it = 0; it < iters; ++it) {
      hipLaunchKernelGGL(k_mlp_standardize,
                         dim3(blocks_for((int64_t)B * m->n_in)), dim3(256), 0,
                         m->stream, dXall, dIdx + (size_t)it * B, dTall,
                         m->d_norm, act_slot(m, 0), m->d_Tb, B, m->n_in);
      MK(hipGetLastError());
      int r = mlp_forward_dev(m, B);
      if (!r) r = mlp_backward_dev(m, B);
      if (r) return r;
      m->adam_t += 1;
      const float c1 = (float)(1.0 / (1.0 - std::pow((double)b1, (double)m->adam_t)));
      const float c2 = (float)(1.0 / (1.0 - std::pow((double)b2, (double)m->adam_t)));
      hipLaunchKernelGGL(k_mlp_adam, dim3(blocks_for(m->n_params)), dim3(256),
                         0, m->stream, m->d_params, m->d_grad, m->d_m, m->d_v,
                         (int)m->n_params, lr, b1, b2, eps, c1, c2);
      MK(hipGetLastError());
    }
    if (loss_out) {
      std::vector<float> r2((size_t)B);
      MK(hipMemcpyAsync(r2.data(), m->d_r2, (size_t)B * 4,
                        hipMemcpyDeviceToHost, m->stream));
      MK(hipStreamSynchronize(m->stream));
      double acc = 0.0;
      for (int s = 0; s < B; ++s) acc += r2[(size_t)s];
      *loss_out = (float)(acc / B);
    }
    MK(hipStreamSynchronize(m->stream));
    return PA_OK;
  };
  rc = run();
  (void)hipStreamSynchronize(m->stream);
  (void)hipFree(dXall);
  (void)hipFree(dTall);
  (void)hipFree(dIdx);
  return rc;
} catch (const std::bad_alloc&) {
  return PA_ENOMEM;
} catch (const std::exception& e) {
  ::pa::note_exception(e.what());
  return PA_EDEVICE;
} catch (...) {
  ::pa::note_exception("unknown exception");
  return PA_EDEVICE;
}

}  // extern "C"
