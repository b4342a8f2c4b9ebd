// C ABI of the stand-alone warm-start network (training and inference on
// caller-owned device buffers).
#include <cmath>
#include <cstring>
#include <string>

#include "ek_internal.h"
#include "unet.h"

using namespace ek;

struct ek_unet {
  UNet net;
  char* ws = nullptr;
  bool own_ws = false;
  void* pinned = nullptr;
  std::string err;
  ek_status fail(ek_status st, const std::string& m) {
    err = m;
    return st;
  }
  ek_status sync() {
    hipError_t e = hipStreamSynchronize(net.stream);
    if (e != hipSuccess) return fail(EK_EHIP, std::string("hipStreamSynchronize: ") + hipGetErrorString(e));
    return EK_OK;
  }
};

namespace {
thread_local std::string g_unet_error;

#define UN_HIP(call)                                                                    \
  do {                                                                                  \
    hipError_t e_ = (call);                                                             \
    if (e_ != hipSuccess) return u->fail(EK_EHIP, std::string(#call) + ": " + hipGetErrorString(e_)); \
  } while (0)
}  // namespace

extern "C" {

ek_status ek_unet_workspace_bytes(int32_t nx, int32_t ny, int32_t nz, int32_t training,
                                  size_t* bytes) {
  if (!bytes || !UNet::shape_ok(nx, ny, nz)) {
    g_unet_error = "nx, ny, nz must be positive multiples of 4";
    return EK_EINVAL;
  }
  *bytes = UNet::bytes(nx, ny, nz, training != 0);
  return EK_OK;
}

ek_status ek_unet_create(int32_t nx, int32_t ny, int32_t nz, int32_t training, void* dev_ws,
                         size_t ws_bytes, void* hip_stream, ek_unet** out) {
  if (!out) { g_unet_error = "out is NULL"; return EK_EINVAL; }
  *out = nullptr;
  if (!UNet::shape_ok(nx, ny, nz)) { g_unet_error = "nx, ny, nz must be positive multiples of 4"; return EK_EINVAL; }
  const size_t need = UNet::bytes(nx, ny, nz, training != 0);
  char* ws = (char*)dev_ws;
  bool own = false;
  if (ws) {
    if (ws_bytes < need) { g_unet_error = "workspace too small"; return EK_ENOMEM; }
    if (((uintptr_t)ws & 255) != 0) { g_unet_error = "workspace must be 256-byte aligned"; return EK_EINVAL; }
  } else {
    if (hipMalloc((void**)&ws, need) != hipSuccess) { g_unet_error = "hipMalloc of the workspace failed"; return EK_ENOMEM; }
    own = true;
  }
  ek_unet* u = new ek_unet();
  u->ws = ws;
  u->own_ws = own;
  u->net.stream = (hipStream_t)hip_stream;
  u->net.carve(ws, nx, ny, nz, training != 0);
  if (hipHostMalloc(&u->pinned, 256, hipHostMallocDefault) != hipSuccess) {
    if (own) (void)hipFree(ws);
    delete u;
    g_unet_error = "hipHostMalloc failed";
    return EK_EHIP;
  }
  if (u->net.init_state() != hipSuccess) u->err = "initialising the network state failed";
  if (!u->err.empty() || u->sync()) {
    g_unet_error = u->err;
    (void)hipHostFree(u->pinned);
    if (own) (void)hipFree(ws);
    delete u;
    return EK_EHIP;
  }
  *out = u;
  return EK_OK;
}

void ek_unet_destroy(ek_unet* u) {
  if (!u) return;
  (void)hipStreamSynchronize(u->net.stream);
  if (u->pinned) (void)hipHostFree(u->pinned);
  if (u->own_ws) (void)hipFree(u->ws);
  delete u;
}

const char* ek_unet_last_error(const ek_unet* u) { return u ? u->err.c_str() : g_unet_error.c_str(); }

ek_status ek_unet_set_params(ek_unet* u, const float* params, int32_t n, float out_scale) {
  if (!u) return EK_EINVAL;
  if (!params || n != UNET_PARAMS) return u->fail(EK_EINVAL, "expected EK_UNET_PARAMS parameters");
  if (!(out_scale > 0.0f) || !std::isfinite(out_scale)) return u->fail(EK_EINVAL, "out_scale must be positive");
  UN_HIP(hipMemcpyAsync(u->net.params, params, size_t(n) * 4, hipMemcpyHostToDevice, u->net.stream));
  u->net.out_scale = out_scale;
  u->net.pack();
  UN_HIP(u->net.init_state());
  u->net.have_params = true;
  return u->sync();
}

ek_status ek_unet_get_params(ek_unet* u, float* params, int32_t n, float* out_scale) {
  if (!u) return EK_EINVAL;
  if (!u->net.have_params) return u->fail(EK_ESTATE, "no parameters set");
  if (!params || n != UNET_PARAMS) return u->fail(EK_EINVAL, "expected EK_UNET_PARAMS parameters");
  UN_HIP(hipMemcpyAsync(params, u->net.params, size_t(n) * 4, hipMemcpyDeviceToHost, u->net.stream));
  if (out_scale) *out_scale = u->net.out_scale;
  return u->sync();
}

ek_status ek_unet_forward(ek_unet* u, const double* dev_b, const uint8_t* dev_solid,
                          double* dev_guess) {
  if (!u) return EK_EINVAL;
  if (!u->net.have_params) return u->fail(EK_ESTATE, "no parameters set");
  if (!dev_b || !dev_solid || !dev_guess) return u->fail(EK_EINVAL, "NULL device buffer");
  u->net.forward(dev_b, dev_solid, false, dev_guess);
  return u->sync();
}

ek_status ek_unet_accumulate(ek_unet* u, const double* dev_b, const uint8_t* dev_solid,
                             const double* dev_target) {
  if (!u) return EK_EINVAL;
  if (!u->net.training) return u->fail(EK_ESTATE, "network was created without training buffers");
  if (!u->net.have_params) return u->fail(EK_ESTATE, "no parameters set");
  if (!dev_b || !dev_solid || !dev_target) return u->fail(EK_EINVAL, "NULL device buffer");
  u->net.accumulate(dev_b, dev_solid, dev_target);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return u->fail(EK_EHIP, std::string("kernel launch: ") + hipGetErrorString(e));
  return EK_OK;
}

ek_status ek_unet_get_gradient(ek_unet* u, float* grad, int32_t n) {
  if (!u) return EK_EINVAL;
  if (!u->net.training) return u->fail(EK_ESTATE, "network was created without training buffers");
  if (!grad || n != UNET_PARAMS) return u->fail(EK_EINVAL, "expected EK_UNET_PARAMS values");
  UN_HIP(hipMemcpyAsync(grad, u->net.grad, size_t(n) * 4, hipMemcpyDeviceToHost, u->net.stream));
  return u->sync();
}

ek_status ek_unet_zero_gradient(ek_unet* u) {
  if (!u) return EK_EINVAL;
  if (!u->net.training) return u->fail(EK_ESTATE, "network was created without training buffers");
  UN_HIP(hipMemsetAsync(u->net.grad, 0, UNET_PARAMS * 4, u->net.stream));
  return EK_OK;
}

ek_status ek_unet_adam_step(ek_unet* u, float lr, float beta1, float beta2, float eps,
                            float grad_scale) {
  if (!u) return EK_EINVAL;
  if (!u->net.training) return u->fail(EK_ESTATE, "network was created without training buffers");
  if (!u->net.have_params) return u->fail(EK_ESTATE, "no parameters set");
  if (!(lr > 0.f) || !(beta1 >= 0.f && beta1 < 1.f) || !(beta2 >= 0.f && beta2 < 1.f) ||
      !(eps > 0.f) || !std::isfinite(grad_scale))
    return u->fail(EK_EINVAL, "bad Adam hyper-parameters");
  u->net.adam(lr, beta1, beta2, eps, grad_scale);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return u->fail(EK_EHIP, std::string("kernel launch: ") + hipGetErrorString(e));
  return EK_OK;
}

ek_status ek_unet_read_loss(ek_unet* u, double* mean_loss, int64_t* count) {
  if (!u) return EK_EINVAL;
  UN_HIP(hipMemcpyAsync(u->pinned, u->net.sc, sizeof(UNetScalars), hipMemcpyDeviceToHost,
                        u->net.stream));
  ek_status st = u->sync();
  if (st) return st;
  UNetScalars h;
  std::memcpy(&h, u->pinned, sizeof h);
  if (mean_loss) *mean_loss = h.loss_count ? h.loss_sum / double(h.loss_count) : 0.0;
  if (count) *count = h.loss_count;
  UN_HIP(hipMemsetAsync(&u->net.sc->loss_sum, 0, 16, u->net.stream));
  return u->sync();
}

}  // extern "C"
