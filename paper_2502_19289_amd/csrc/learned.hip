// Host side of the kept-rank network: creation, parameters, inference,
// gradients and Adam training on the device (C ABI, see cluster_tebd.h).
#include <algorithm>
#include <cmath>
#include <cstring>
#include <random>
#include <vector>

#include "engine.hpp"

using namespace ctebd;

namespace {

struct MFail {
  mps_status st;
};

#define MHIP(expr)                                                   \
  do {                                                               \
    hipError_t e_ = (expr);                                          \
    if (e_ != hipSuccess) {                                          \
      if (h) h->err = std::string(#expr) + ": " + hipGetErrorString(e_); \
      throw MFail{e_ == hipErrorOutOfMemory ? MPS_ENOMEM : MPS_EDEVICE}; \
    }                                                                \
  } while (0)

template <typename F>
mps_status mguard(mlp_ctx* h, F&& f) {
  try {
    return f();
  } catch (const MFail& e) {
    return e.st;
  } catch (const std::bad_alloc&) {
    return MPS_ENOMEM;
  }
}

// device scratch for one call (freed before returning)
struct Scratch {
  std::vector<void*> ptrs;
  ~Scratch() {
    for (void* p : ptrs) (void)hipFree(p);
  }
  template <typename T>
  T* get(size_t n) {
    void* p = nullptr;
    if (hipMalloc(&p, std::max<size_t>(n, 1) * sizeof(T)) != hipSuccess) throw MFail{MPS_ENOMEM};
    ptrs.push_back(p);
    return (T*)p;
  }
};

}  // namespace

extern "C" {

int mlp_num_params(void) { return mlp_param_count(); }

mps_status mlp_create(int seed, mlp_handle* out) {
  if (!out) return MPS_EINVAL;
  *out = nullptr;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) {
    (void)hipGetLastError();
    return MPS_EDEVICE;
  }
  mlp_ctx* h = new (std::nothrow) mlp_ctx();
  if (!h) return MPS_ENOMEM;
  mps_status st = mguard(h, [&]() -> mps_status {
    const int np = mlp_param_count();
    MHIP(hipStreamCreateWithFlags(&h->stream, hipStreamNonBlocking));
    MHIP(hipMalloc(&h->P, np * sizeof(float)));
    MHIP(hipMalloc(&h->m, np * sizeof(float)));
    MHIP(hipMalloc(&h->v, np * sizeof(float)));
    MHIP(hipMalloc(&h->g, np * sizeof(float)));
    MHIP(hipMemset(h->m, 0, np * sizeof(float)));
    MHIP(hipMemset(h->v, 0, np * sizeof(float)));
    // He initialisation of the weights, zero biases (layout W1, b1, W2, b2, w3, b3)
    std::mt19937_64 rng((uint64_t)seed * 0x9E3779B97F4A7C15ull + 1);
    std::normal_distribution<float> nd(0.f, 1.f);
    std::vector<float> p(np, 0.f);
    const int NI = N_FEAT, NH = 64;
    for (int i = 0; i < NH * NI; ++i) p[i] = nd(rng) * std::sqrt(2.f / NI);
    const int ow2 = NH * NI + NH;
    for (int i = 0; i < NH * NH; ++i) p[ow2 + i] = nd(rng) * std::sqrt(2.f / NH);
    const int ow3 = ow2 + NH * NH + NH;
    for (int i = 0; i < NH; ++i) p[ow3 + i] = nd(rng) * std::sqrt(1.f / NH);
    MHIP(hipMemcpy(h->P, p.data(), np * sizeof(float), hipMemcpyHostToDevice));
    return MPS_OK;
  });
  if (st != MPS_OK) {
    mlp_destroy(h);
    return st;
  }
  *out = h;
  return MPS_OK;
}

mps_status mlp_destroy(mlp_handle h) {
  if (!h) return MPS_OK;
  if (h->stream) (void)hipStreamSynchronize(h->stream);
  for (float* p : {h->P, h->m, h->v, h->g})
    if (p) (void)hipFree(p);
  if (h->stream) (void)hipStreamDestroy(h->stream);
  delete h;
  return MPS_OK;
}

mps_status mlp_get_params(mlp_handle h, float* p) {
  if (!h || !p) return MPS_EINVAL;
  return mguard(h, [&]() -> mps_status {
    MHIP(hipStreamSynchronize(h->stream));
    MHIP(hipMemcpy(p, h->P, mlp_param_count() * sizeof(float), hipMemcpyDeviceToHost));
    return MPS_OK;
  });
}

mps_status mlp_set_params(mlp_handle h, const float* p) {
  if (!h || !p) return MPS_EINVAL;
  return mguard(h, [&]() -> mps_status {
    MHIP(hipStreamSynchronize(h->stream));
    MHIP(hipMemcpy(h->P, p, mlp_param_count() * sizeof(float), hipMemcpyHostToDevice));
    return MPS_OK;
  });
}

mps_status mlp_forward(mlp_handle h, const float* X, int n, float* y) {
  if (!h || n < 0 || (n > 0 && (!X || !y))) return MPS_EINVAL;
  if (n == 0) return MPS_OK;
  return mguard(h, [&]() -> mps_status {
    Scratch S;
    float* dX = S.get<float>((size_t)n * N_FEAT);
    float* dy = S.get<float>(n);
    MHIP(hipMemcpyAsync(dX, X, (size_t)n * N_FEAT * sizeof(float), hipMemcpyHostToDevice, h->stream));
    MHIP(launch_mlp_forward(h->P, dX, dy, n, h->stream));
    MHIP(hipMemcpyAsync(y, dy, n * sizeof(float), hipMemcpyDeviceToHost, h->stream));
    MHIP(hipStreamSynchronize(h->stream));
    return MPS_OK;
  });
}

mps_status mlp_grad(mlp_handle h, const float* X, const float* t, int n, float tau, float* grad, float* loss) {
  if (!h || n <= 0 || !X || !t || !(tau > 0.f && tau < 1.f)) return MPS_EINVAL;
  return mguard(h, [&]() -> mps_status {
    Scratch S;
    const int np = mlp_param_count();
    const int nparts = (n + mlp_chunk() - 1) / mlp_chunk();
    float* dX = S.get<float>((size_t)n * N_FEAT);
    float* dt = S.get<float>(n);
    float* part = S.get<float>((size_t)nparts * np);
    float* lpart = S.get<float>(nparts);
    float* dl = S.get<float>(1);
    MHIP(hipMemcpyAsync(dX, X, (size_t)n * N_FEAT * sizeof(float), hipMemcpyHostToDevice, h->stream));
    MHIP(hipMemcpyAsync(dt, t, n * sizeof(float), hipMemcpyHostToDevice, h->stream));
    MHIP(launch_mlp_grad(h->P, dX, dt, nullptr, n, tau, part, lpart, h->g, dl, h->stream));
    if (grad) MHIP(hipMemcpyAsync(grad, h->g, np * sizeof(float), hipMemcpyDeviceToHost, h->stream));
    float l = 0.f;
    MHIP(hipMemcpyAsync(&l, dl, sizeof(float), hipMemcpyDeviceToHost, h->stream));
    MHIP(hipStreamSynchronize(h->stream));
    if (loss) *loss = l;
    return MPS_OK;
  });
}

mps_status mlp_train(mlp_handle h, const float* X, const float* t, int n, int epochs, int batch, float lr,
                     float tau, uint64_t seed, float* final_loss) {
  if (!h || n <= 0 || !X || !t || epochs < 0 || batch <= 0 || !(lr > 0.f) || !(tau > 0.f && tau < 1.f))
    return MPS_EINVAL;
  return mguard(h, [&]() -> mps_status {
    Scratch S;
    const int np = mlp_param_count();
    const int b = std::min(batch, n);
    const int nparts_max = (std::max(b, n) + mlp_chunk() - 1) / mlp_chunk();
    float* dX = S.get<float>((size_t)n * N_FEAT);
    float* dt = S.get<float>(n);
    int* didx = S.get<int>(n);
    float* part = S.get<float>((size_t)nparts_max * np);
    float* lpart = S.get<float>(nparts_max);
    float* dl = S.get<float>(1);
    MHIP(hipMemcpyAsync(dX, X, (size_t)n * N_FEAT * sizeof(float), hipMemcpyHostToDevice, h->stream));
    MHIP(hipMemcpyAsync(dt, t, n * sizeof(float), hipMemcpyHostToDevice, h->stream));
    std::vector<int> perm(n);
    for (int i = 0; i < n; ++i) perm[i] = i;
    std::mt19937_64 rng(seed);
    for (int ep = 0; ep < epochs; ++ep) {
      std::shuffle(perm.begin(), perm.end(), rng);
      MHIP(hipMemcpyAsync(didx, perm.data(), n * sizeof(int), hipMemcpyHostToDevice, h->stream));
      for (int s0 = 0; s0 + b <= n; s0 += b) {
        MHIP(launch_mlp_grad(h->P, dX, dt, didx + s0, b, tau, part, lpart, h->g, nullptr, h->stream));
        h->t += 1;
        MHIP(launch_adam(h->P, h->g, h->m, h->v, lr, h->t, h->stream));
      }
      MHIP(hipStreamSynchronize(h->stream));  // perm is rewritten next epoch
    }
    MHIP(launch_mlp_grad(h->P, dX, dt, nullptr, n, tau, part, lpart, h->g, dl, h->stream));
    float l = 0.f;
    MHIP(hipMemcpyAsync(&l, dl, sizeof(float), hipMemcpyDeviceToHost, h->stream));
    MHIP(hipStreamSynchronize(h->stream));
    if (final_loss) *final_loss = l;
    return MPS_OK;
  });
}

mps_status mps_set_sketch_model(mps_handle ctx, mlp_handle model) {
  if (!ctx) return MPS_EINVAL;
  if (model) (void)hipStreamSynchronize(model->stream);
  ctx->mlp_params = model ? model->P : nullptr;
  return MPS_OK;
}

mps_status mps_svd_log(mps_handle ctx, float* X, float* t, int cap, int* count) {
  if (!ctx || !count) return MPS_EINVAL;
  const int total = (int)ctx->log_t.size();
  *count = total;
  if (!X || !t || cap <= 0) return MPS_OK;
  const int n = std::min(cap, total);
  std::memcpy(X, ctx->log_x.data(), (size_t)n * N_FEAT * sizeof(float));
  std::memcpy(t, ctx->log_t.data(), (size_t)n * sizeof(float));
  ctx->log_x.erase(ctx->log_x.begin(), ctx->log_x.begin() + (size_t)n * N_FEAT);
  ctx->log_t.erase(ctx->log_t.begin(), ctx->log_t.begin() + n);
  return MPS_OK;
}

}  // extern "C"
