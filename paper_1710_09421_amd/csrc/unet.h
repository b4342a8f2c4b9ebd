// Small 3-D convolutional network that guesses the Poisson solution from the
// charge density and the solid mask (the learned warm start).  Activations
// are bfloat16 in channels-last order [z][y][x][c]; convolutions run on MFMA
// with float32 accumulation; parameters, their gradient and the Adam moments
// are float32.
//
// Network (channels-first in the description, periodic convolutions):
//   A 3x3x3 conv 2->16 + ReLU -> a1; 2x2x2 average pool -> p1
//   B 3x3x3 conv 16->32 + ReLU -> a2; pool -> p2
//   C 3x3x3 conv 32->64 + ReLU -> a3
//   D 1x1x1 conv 64->32 -> u3; c2 = ReLU(upsample(u3) + a2)
//   E 1x1x1 conv 32->16 -> u2; c1 = ReLU(upsample(u2) + a1)
//   F 3x3x3 conv 16->1 -> output
// Input channels: (b - mean(b)) / s and the solid flag, s the RMS of
// b - mean(b); the guess is s * out_scale * output, which uses the linearity
// of the Poisson equation so one network covers every charge scale.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace ek {

constexpr int UNET_LAYERS = 6;
constexpr int UNET_PARAMS = 73137;

struct UNetLayer {
  int taps, cin, cout;      // real sizes
  int cinp, coutp;          // padded to multiples of 16 for the matrix cores
  int woff, boff;           // offsets of weights [taps][cin][cout] and bias in the flat vector
  int pw, pb;               // offsets in the packed weight and padded bias arrays
};

// Layer table in parameter order A..F.
constexpr UNetLayer UNET[UNET_LAYERS] = {
    {27, 2, 16, 16, 16, 0, 864, 0, 0},
    {27, 16, 32, 16, 32, 880, 14704, 6912, 16},
    {27, 32, 64, 32, 64, 14736, 70032, 20736, 48},
    {1, 64, 32, 64, 32, 70096, 72144, 76032, 112},
    {1, 32, 16, 32, 16, 72176, 72688, 78080, 144},
    {27, 16, 1, 16, 16, 72704, 73136, 78592, 160}};
constexpr int UNET_PACKED = 85504;       // bfloat16 elements of one packed weight set
constexpr int UNET_BIAS_PADDED = 176;

struct Grid3 {
  int nx, ny, nz, n;
};

// Device scalars of one forward pass.
struct UNetScalars {
  double mean, s, inv_s;    // input normalisation
  double scale, inv_scale;  // s * out_scale and its inverse
  double loss_sum;          // sum of per-call mean squared errors since the last read
  long long loss_count;
  long long pad;
};

struct UNet {
  Grid3 g[3]{};              // full, half and quarter resolution
  bool training = false;
  float out_scale = 1.0f;
  bool have_params = false;
  long long adam_t = 0;
  hipStream_t stream = nullptr;

  // forward activations
  uint16_t *x0 = nullptr, *a1 = nullptr, *p1 = nullptr, *a2 = nullptr, *p2 = nullptr;
  uint16_t *a3 = nullptr, *u3 = nullptr, *c2 = nullptr, *u2 = nullptr, *c1 = nullptr;
  float* out = nullptr;
  // backward
  uint16_t *d0 = nullptr, *g1 = nullptr, *du2 = nullptr, *g2 = nullptr, *du3 = nullptr;
  uint16_t *g3 = nullptr, *dp2 = nullptr, *gb = nullptr, *dp1 = nullptr, *ga = nullptr;
  float* wpart = nullptr;
  // parameters
  float *params = nullptr, *grad = nullptr, *adam_m = nullptr, *adam_v = nullptr;
  uint16_t *wf = nullptr, *wb = nullptr;
  float* bias = nullptr;
  UNetScalars* sc = nullptr;
  double* red = nullptr;     // block partial sums

  static bool shape_ok(int nx, int ny, int nz);
  static size_t bytes(int nx, int ny, int nz, bool training);
  void carve(char* base, int nx, int ny, int nz, bool training);
  hipError_t init_state();                             // zero moments, gradient, loss
  void pack();                                         // params -> packed bf16 + bias
  // guess = s * out_scale * N(b, solid); solid is a byte mask (nonzero = solid)
  // or, with link = true, link words whose top bit marks solid sites.
  void forward(const double* b, const void* solid, bool link, double* guess);
  // forward + mean squared error against target / (s * out_scale) + backward;
  // the gradient is added to grad.
  void accumulate(const double* b, const void* solid, const double* target);
  void adam(float lr, float beta1, float beta2, float eps, float grad_scale);
};

}  // namespace ek
