// The correction network of the learned preconditioner (bem_mlp.hip): a 3-layer
// perceptron trained and evaluated by the library's own kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace bem {

constexpr int kMlpSlots = 64;  // block size of the correction (slots of a tile)
constexpr int kMlpRank = 8;    // rank of the correction U V^T

constexpr size_t kMlpScratchBytes = (size_t)32 << 20;  // fixed forward-pass scratch per device
constexpr int kMlpMaxDevices = 64;
constexpr int kMlpMaxBatch = 1 << 20;  // rows per product launch stay within the grid's y extent

int64_t mlp_nparams(int in, int hid, int out);
size_t mlp_ws_bytes(int hid, int out, int batch);
hipError_t mlp_init(int in, int hid, int out, uint64_t seed, float* params, hipStream_t st);
// Y [batch][out] = net(X [batch][in]); precision 0 FP32, 1 BF16 operands / FP32 accumulation
hipError_t mlp_forward(int in, int hid, int out, int batch, const float* params, const float* X, float* Y,
                       int precision, void* ws, hipStream_t st);
// the device address of this device's fixed scratch array (looked up once per device)
hipError_t mlp_scratch(void** ptr);
// bytes of scratch the forward pass needs (hidden activations H1, H2)
size_t mlp_forward_scratch_bytes(int hid, int batch);
// mlp_forward with H1, H2 at scratch_ptr (from mlp_scratch) instead of a workspace
hipError_t mlp_forward_noalloc(int in, int hid, int out, int batch, const float* params, const float* X, float* Y,
                               int precision, void* scratch_ptr, hipStream_t st);
// mean over the batch of ||T_b - U_b V_b^T||_F^2 / ||T_b||_F^2 (out = 2 or 4 x 64 x 8) into
// loss[0] (device) and its gradient with respect to every parameter into grad
hipError_t mlp_loss_grad(int in, int hid, int out, int batch, int cplx, const float* params, const float* X,
                         const float* T, float* grad, float* loss, int precision, void* ws, hipStream_t st);
hipError_t mlp_adam(int64_t n, float* params, const float* grad, float* m, float* v, int step, float lr, float b1,
                    float b2, float eps, hipStream_t st);

}  // namespace bem
