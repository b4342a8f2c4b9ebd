// Kernels of the warm-start network: MFMA implicit-GEMM convolutions (forward
// and, with flipped taps and transposed weights, backward-data), MFMA weight
// gradients with a fixed-order reduction, pooling / upsampling / skip
// kernels, the loss, parameter packing and Adam.
//
// Convolution as a matrix product per 16 output sites:
//   D[co][site] = sum_k W[co][k] X[k][site],  k = (tap, input channel).
// The A operand (weights) is read as 8 or 4 consecutive input channels of one
// output channel, the B operand (activations) as 8 or 4 consecutive channels
// of one site; both are single vector loads in channels-last order.  The
// result lane holds 4 consecutive output channels of one site, stored as one
// 8-byte vector.
#include <hip/hip_runtime.h>

#include <cmath>

#include "ek_internal.h"
#include "reduce.h"
#include "unet.h"

namespace ek {

typedef float f4 __attribute__((ext_vector_type(4)));
typedef short s4 __attribute__((ext_vector_type(4)));
typedef __bf16 b8 __attribute__((ext_vector_type(8)));

constexpr uint16_t BF_ONE = 0x3F80;

__device__ __forceinline__ uint16_t f2bf(float v) {
  return __builtin_bit_cast(uint16_t, (__bf16)v);
}
__device__ __forceinline__ float bf2f(uint16_t u) {
  return __builtin_bit_cast(float, uint32_t(u) << 16);
}

// Periodic neighbour r + (dx, dy, dz) of site (x, y, z).
__device__ __forceinline__ int nbr_site(const Grid3& g, int x, int y, int z, int dx, int dy,
                                        int dz) {
  int xx = x + dx, yy = y + dy, zz = z + dz;
  xx = xx < 0 ? xx + g.nx : (xx >= g.nx ? xx - g.nx : xx);
  yy = yy < 0 ? yy + g.ny : (yy >= g.ny ? yy - g.ny : yy);
  zz = zz < 0 ? zz + g.nz : (zz >= g.nz ? zz - g.nz : zz);
  return (zz * g.ny + yy) * g.nx + xx;
}

__device__ __forceinline__ void decode(const Grid3& g, int r, int& x, int& y, int& z) {
  const unsigned q = unsigned(r) / unsigned(g.nx);
  x = r - int(q) * g.nx;
  z = int(q / unsigned(g.ny));
  y = int(q) - z * g.ny;
}

// ---------------------------------------------------------------------------
// Convolution (forward, or backward-data with the flipped weight set)
// ---------------------------------------------------------------------------
enum Epi { EPI_RELU = 0, EPI_LINEAR = 1, EPI_MASK = 2, EPI_PLAIN = 3, EPI_OUT = 4 };

struct ConvIO {
  const uint16_t* in;       // [n][CIN]
  const uint16_t* w;        // [T][COUT][CIN]
  const float* bias;        // [COUT] (EPI_RELU, EPI_LINEAR, EPI_OUT)
  const uint16_t* act;      // [n][COUT]: ReLU gate (EPI_MASK)
  uint16_t* out;            // [n][COUT]
  float* out32;             // [n]: channel 0 (EPI_OUT)
  double* guess;            // [n]: channel 0 times the output scale (EPI_OUT, optional)
  const UNetScalars* sc;
};

template <int CIN, int COUT, int T, int EPI, int NS>
__global__ __launch_bounds__(256) void k_conv(ConvIO io, Grid3 g) {
  constexpr int NC = COUT / 16;
  constexpr int KB = CIN == 16 ? 1 : CIN / 32;
  const int lane = threadIdx.x & 63;
  const int col = lane & 15, grp = lane >> 4;
  const int wave = blockIdx.x * 4 + (threadIdx.x >> 6);
  int xs[NS], ys[NS], zs[NS];
  int site[NS];
#pragma unroll
  for (int j = 0; j < NS; ++j) {
    site[j] = (wave * NS + j) * 16 + col;
    const int r = site[j] < g.n ? site[j] : g.n - 1;
    decode(g, r, xs[j], ys[j], zs[j]);
  }
  f4 acc[NC][NS];
#pragma unroll
  for (int c = 0; c < NC; ++c)
#pragma unroll
    for (int j = 0; j < NS; ++j) acc[c][j] = f4{0.f, 0.f, 0.f, 0.f};

  for (int t = 0; t < T; ++t) {
    const int dz = T == 1 ? 0 : t / 9 - 1;
    const int dy = T == 1 ? 0 : (t / 3) % 3 - 1;
    const int dx = T == 1 ? 0 : t % 3 - 1;
    if constexpr (CIN == 16) {
      s4 bf[NS];
#pragma unroll
      for (int j = 0; j < NS; ++j) {
        const int nb = nbr_site(g, xs[j], ys[j], zs[j], dx, dy, dz);
        bf[j] = *(const s4*)(io.in + (size_t)nb * CIN + grp * 4);
      }
#pragma unroll
      for (int c = 0; c < NC; ++c) {
        const s4 af = *(const s4*)(io.w + ((size_t)(t * COUT + c * 16 + col)) * CIN + grp * 4);
#pragma unroll
        for (int j = 0; j < NS; ++j)
          acc[c][j] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(af, bf[j], acc[c][j], 0, 0, 0);
      }
    } else {
      b8 bf[NS][KB];
#pragma unroll
      for (int j = 0; j < NS; ++j) {
        const int nb = nbr_site(g, xs[j], ys[j], zs[j], dx, dy, dz);
#pragma unroll
        for (int kb = 0; kb < KB; ++kb)
          bf[j][kb] = *(const b8*)(io.in + (size_t)nb * CIN + kb * 32 + grp * 8);
      }
#pragma unroll
      for (int c = 0; c < NC; ++c)
#pragma unroll
        for (int kb = 0; kb < KB; ++kb) {
          const b8 af =
              *(const b8*)(io.w + ((size_t)(t * COUT + c * 16 + col)) * CIN + kb * 32 + grp * 8);
#pragma unroll
          for (int j = 0; j < NS; ++j)
            acc[c][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af, bf[j][kb], acc[c][j], 0, 0, 0);
        }
    }
  }

#pragma unroll
  for (int j = 0; j < NS; ++j) {
    if (site[j] >= g.n) continue;
    const size_t r = (size_t)site[j];
    if constexpr (EPI == EPI_OUT) {
      if (grp == 0) {
        const float v = acc[0][j][0] + io.bias[0];
        io.out32[r] = v;
        if (io.guess) io.guess[r] = double(v) * io.sc->scale;
      }
    } else {
#pragma unroll
      for (int c = 0; c < NC; ++c) {
        const int co = c * 16 + grp * 4;
        float v[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          v[i] = acc[c][j][i];
          if constexpr (EPI == EPI_RELU || EPI == EPI_LINEAR) v[i] += io.bias[co + i];
          if constexpr (EPI == EPI_RELU) v[i] = fmaxf(v[i], 0.f);
        }
        if constexpr (EPI == EPI_MASK) {
          const uint2 a = *(const uint2*)(io.act + r * COUT + co);
          if ((a.x & 0xFFFFu) == 0 || (a.x & 0x8000u)) v[0] = 0.f;
          if ((a.x >> 16) == 0 || (a.x & 0x80000000u)) v[1] = 0.f;
          if ((a.y & 0xFFFFu) == 0 || (a.y & 0x8000u)) v[2] = 0.f;
          if ((a.y >> 16) == 0 || (a.y & 0x80000000u)) v[3] = 0.f;
        }
        uint2 o;
        o.x = uint32_t(f2bf(v[0])) | (uint32_t(f2bf(v[1])) << 16);
        o.y = uint32_t(f2bf(v[2])) | (uint32_t(f2bf(v[3])) << 16);
        *(uint2*)(io.out + r * COUT + co) = o;
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Weight gradient: dW[t][ci][co] = sum_r in(r + d_t)[ci] dy(r)[co] and, as an
// extra tap T, the bias gradient sum_r dy(r)[co] in row ci = 0.  A block owns
// `subs` consecutive chunks of 256 sites; per tap it stages the shifted input
// and dy of a chunk transposed in LDS ([channel][site]) so both MFMA operands
// are 16-byte LDS reads, sums over its chunks in registers, then over its 4
// waves in LDS, and writes one partial per tap: part[block][t][ci][co].
// ---------------------------------------------------------------------------
constexpr int WG_LD = 264;     // LDS row length (256 sites + 8 padding)

template <int CIN, int COUT, int T>
__global__ __launch_bounds__(256) void k_wgrad(const uint16_t* __restrict__ in,
                                               const uint16_t* __restrict__ dy,
                                               float* __restrict__ part, Grid3 g, int subs) {
  constexpr int NI = CIN / 16, NO = COUT / 16;
  static_assert(4 * CIN * COUT * 4 <= (CIN + COUT) * WG_LD * 2, "reduction buffer");
  __shared__ __align__(16) uint16_t lds[(CIN + COUT) * WG_LD];
  uint16_t* a_l = lds;
  uint16_t* d_l = lds + CIN * WG_LD;
  float* red = (float*)lds;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int col = lane & 15, grp = lane >> 4;

  for (int t = 0; t <= T; ++t) {
    const int dz = T == 1 ? 0 : t / 9 - 1;
    const int dyy = T == 1 ? 0 : (t / 3) % 3 - 1;
    const int dx = T == 1 ? 0 : t % 3 - 1;
    f4 acc[NI][NO];
#pragma unroll
    for (int i = 0; i < NI; ++i)
#pragma unroll
      for (int o = 0; o < NO; ++o) acc[i][o] = f4{0.f, 0.f, 0.f, 0.f};
    for (int sc = 0; sc < subs; ++sc) {
      const long long site = ((long long)blockIdx.x * subs + sc) * 256 + tid;
      __syncthreads();
      if (site < g.n) {
        if (t < T) {
          int x, y, z;
          decode(g, int(site), x, y, z);
          const int nb = nbr_site(g, x, y, z, dx, dyy, dz);
#pragma unroll
          for (int v = 0; v < CIN / 8; ++v) {
            const uint4 q = *(const uint4*)(in + (size_t)nb * CIN + v * 8);
            const uint32_t w4[4] = {q.x, q.y, q.z, q.w};
#pragma unroll
            for (int e = 0; e < 8; ++e)
              a_l[(v * 8 + e) * WG_LD + tid] = uint16_t(w4[e >> 1] >> (16 * (e & 1)));
          }
        } else {
#pragma unroll
          for (int c = 0; c < CIN; ++c) a_l[c * WG_LD + tid] = c == 0 ? BF_ONE : 0;
        }
#pragma unroll
        for (int v = 0; v < COUT / 8; ++v) {
          const uint4 q = *(const uint4*)(dy + (size_t)site * COUT + v * 8);
          const uint32_t w4[4] = {q.x, q.y, q.z, q.w};
#pragma unroll
          for (int e = 0; e < 8; ++e)
            d_l[(v * 8 + e) * WG_LD + tid] = uint16_t(w4[e >> 1] >> (16 * (e & 1)));
        }
      } else {
#pragma unroll
        for (int c = 0; c < CIN; ++c) a_l[c * WG_LD + tid] = 0;
#pragma unroll
        for (int c = 0; c < COUT; ++c) d_l[c * WG_LD + tid] = 0;
      }
      __syncthreads();
#pragma unroll
      for (int kb = 0; kb < 2; ++kb) {
        const int k0 = wv * 64 + kb * 32 + grp * 8;
        b8 af[NI], bf[NO];
#pragma unroll
        for (int i = 0; i < NI; ++i) af[i] = *(const b8*)(a_l + (i * 16 + col) * WG_LD + k0);
#pragma unroll
        for (int o = 0; o < NO; ++o) bf[o] = *(const b8*)(d_l + (o * 16 + col) * WG_LD + k0);
#pragma unroll
        for (int i = 0; i < NI; ++i)
#pragma unroll
          for (int o = 0; o < NO; ++o)
            acc[i][o] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[i], bf[o], acc[i][o], 0, 0, 0);
      }
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < NI; ++i)
#pragma unroll
      for (int o = 0; o < NO; ++o)
#pragma unroll
        for (int q = 0; q < 4; ++q)
          red[(wv * CIN + i * 16 + grp * 4 + q) * COUT + o * 16 + col] = acc[i][o][q];
    __syncthreads();
    float* dst = part + ((size_t)blockIdx.x * (T + 1) + t) * CIN * COUT;
    for (int e = tid; e < CIN * COUT; e += 256)
      dst[e] = (red[e] + red[CIN * COUT + e]) + (red[2 * CIN * COUT + e] + red[3 * CIN * COUT + e]);
  }
}

// Sum of the per-block partials added to the flat gradient at the real
// (unpadded) positions of one layer.  A block of 1024 threads owns 64
// consecutive elements; its 16 waves take every 16th partial block and the 16
// sums are added in a fixed order, so the result does not depend on timing.
__global__ __launch_bounds__(1024) void k_wreduce(const float* __restrict__ part, int nblk,
                                                  UNetLayer L, float* __restrict__ grad) {
  __shared__ float sh[16][64];
  const int per = (L.taps + 1) * L.cinp * L.coutp;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int e = blockIdx.x * 64 + lane;
  float s = 0.f;
  if (e < per) {
#pragma unroll 8
    for (int b = wv; b < nblk; b += 16) s += part[(size_t)b * per + e];
  }
  sh[wv][lane] = s;
  __syncthreads();
  if (wv != 0 || e >= per) return;
  float t = 0.f;
#pragma unroll
  for (int w = 0; w < 16; ++w) t += sh[w][lane];
  const int co = e % L.coutp;
  const int ci = (e / L.coutp) % L.cinp;
  const int tap = e / (L.coutp * L.cinp);
  if (co >= L.cout) return;
  if (tap < L.taps) {
    if (ci < L.cin) grad[L.woff + (tap * L.cin + ci) * L.cout + co] += t;
  } else if (ci == 0) {
    grad[L.boff + co] += t;
  }
}

// ---------------------------------------------------------------------------
// Elementwise kernels on channels-last bfloat16 tensors, 8 channels a thread
// ---------------------------------------------------------------------------
__device__ __forceinline__ void unpack8(const uint4 q, float (&f)[8]) {
  const uint32_t w[4] = {q.x, q.y, q.z, q.w};
#pragma unroll
  for (int e = 0; e < 8; ++e) f[e] = bf2f(uint16_t(w[e >> 1] >> (16 * (e & 1))));
}
__device__ __forceinline__ uint4 pack8(const float (&f)[8]) {
  uint32_t w[4];
#pragma unroll
  for (int e = 0; e < 4; ++e) w[e] = uint32_t(f2bf(f[2 * e])) | (uint32_t(f2bf(f[2 * e + 1])) << 16);
  return uint4{w[0], w[1], w[2], w[3]};
}

// Site index of child (cx, cy, cz) in {0,1}^3 of coarse site rc.
__device__ __forceinline__ size_t child(const Grid3& fine, const Grid3& coarse, int rc, int k) {
  int x, y, z;
  decode(coarse, rc, x, y, z);
  return ((size_t)(2 * z + (k >> 2)) * fine.ny + 2 * y + ((k >> 1) & 1)) * fine.nx + 2 * x + (k & 1);
}
__device__ __forceinline__ int parent(const Grid3& fine, const Grid3& coarse, int rf) {
  int x, y, z;
  decode(fine, rf, x, y, z);
  return ((z >> 1) * coarse.ny + (y >> 1)) * coarse.nx + (x >> 1);
}

// mode 0: average of the 8 children (pooling); mode 1: sum (upsample backward)
__global__ __launch_bounds__(256) void k_down(const uint16_t* __restrict__ in,
                                              uint16_t* __restrict__ out, int C, Grid3 fine,
                                              Grid3 coarse, int mode) {
  const int groups = C / 8;
  const long long id = (long long)blockIdx.x * 256 + threadIdx.x;
  if (id >= (long long)coarse.n * groups) return;
  const int rc = int(id / groups), v = int(id % groups);
  float s[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  for (int k = 0; k < 8; ++k) {
    float f[8];
    unpack8(*(const uint4*)(in + child(fine, coarse, rc, k) * C + v * 8), f);
#pragma unroll
    for (int e = 0; e < 8; ++e) s[e] += f[e];
  }
  if (mode == 0)
#pragma unroll
    for (int e = 0; e < 8; ++e) s[e] *= 0.125f;
  *(uint4*)(out + (size_t)rc * C + v * 8) = pack8(s);
}

// out = ReLU(upsample(u) + skip)
__global__ __launch_bounds__(256) void k_up_add_relu(const uint16_t* __restrict__ u,
                                                     const uint16_t* __restrict__ skip,
                                                     uint16_t* __restrict__ out, int C, Grid3 fine,
                                                     Grid3 coarse) {
  const int groups = C / 8;
  const long long id = (long long)blockIdx.x * 256 + threadIdx.x;
  if (id >= (long long)fine.n * groups) return;
  const int rf = int(id / groups), v = int(id % groups);
  float a[8], b[8];
  unpack8(*(const uint4*)(u + (size_t)parent(fine, coarse, rf) * C + v * 8), a);
  unpack8(*(const uint4*)(skip + (size_t)rf * C + v * 8), b);
#pragma unroll
  for (int e = 0; e < 8; ++e) a[e] = fmaxf(a[e] + b[e], 0.f);
  *(uint4*)(out + (size_t)rf * C + v * 8) = pack8(a);
}

// Gradient at a pooled-and-skipped activation: (g + dp(parent) / 8) * [act > 0]
__global__ __launch_bounds__(256) void k_skip_grad(const uint16_t* __restrict__ gsk,
                                                   const uint16_t* __restrict__ dp,
                                                   const uint16_t* __restrict__ act,
                                                   uint16_t* __restrict__ out, int C, Grid3 fine,
                                                   Grid3 coarse) {
  const int groups = C / 8;
  const long long id = (long long)blockIdx.x * 256 + threadIdx.x;
  if (id >= (long long)fine.n * groups) return;
  const int rf = int(id / groups), v = int(id % groups);
  float a[8], b[8], m[8];
  unpack8(*(const uint4*)(gsk + (size_t)rf * C + v * 8), a);
  unpack8(*(const uint4*)(dp + (size_t)parent(fine, coarse, rf) * C + v * 8), b);
  unpack8(*(const uint4*)(act + (size_t)rf * C + v * 8), m);
#pragma unroll
  for (int e = 0; e < 8; ++e) a[e] = m[e] > 0.f ? a[e] + 0.125f * b[e] : 0.f;
  *(uint4*)(out + (size_t)rf * C + v * 8) = pack8(a);
}

// ---------------------------------------------------------------------------
// Input normalisation, loss
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_in_stats(const double* __restrict__ b,
                                                  double* __restrict__ partials, int n) {
  const int r = blockIdx.x * 256 + threadIdx.x;
  double v[2] = {0.0, 0.0};
  if (r < n) {
    v[0] = b[r];
    v[1] = b[r] * b[r];
  }
  block_partials<2>(v, partials, blockIdx.x, gridDim.x);
}

__global__ __launch_bounds__(1024) void k_in_final(const double* __restrict__ partials,
                                                   int nblocks, int n, double out_scale,
                                                   UNetScalars* __restrict__ sc) {
  double t[2];
  block_sums_1024<2>(partials, nblocks, t);
  if (threadIdx.x == 0) {
    const double mean = t[0] / n;
    const double var = t[1] / n - mean * mean;
    const double s = var > 0.0 ? sqrt(var) : 1.0;
    sc->mean = mean;
    sc->s = s;
    sc->inv_s = 1.0 / s;
    sc->scale = s * out_scale;
    sc->inv_scale = 1.0 / (s * out_scale);
  }
}

// x0[r] = ((b - mean) / s, solid, 0 ...); solid from a byte mask or link words
template <bool LINK>
__global__ __launch_bounds__(256) void k_input(const double* __restrict__ b,
                                               const void* __restrict__ solid,
                                               const UNetScalars* __restrict__ sc,
                                               uint16_t* __restrict__ x0, int n) {
  const int r = blockIdx.x * 256 + threadIdx.x;
  if (r >= n) return;
  const float v = float((b[r] - sc->mean) * sc->inv_s);
  bool s;
  if constexpr (LINK) s = (((const uint32_t*)solid)[r] & MASK_SOLID) != 0;
  else s = ((const uint8_t*)solid)[r] != 0;
  uint4 q0{uint32_t(f2bf(v)) | (uint32_t(s ? BF_ONE : 0) << 16), 0u, 0u, 0u};
  *(uint4*)(x0 + (size_t)r * 16) = q0;
  *(uint4*)(x0 + (size_t)r * 16 + 8) = uint4{0u, 0u, 0u, 0u};
}

// d0[r] = (2 (out - target / scale) / n, 0, ...); partial sums of the squared error
__global__ __launch_bounds__(256) void k_loss(const float* __restrict__ out,
                                              const double* __restrict__ target,
                                              const UNetScalars* __restrict__ sc,
                                              uint16_t* __restrict__ d0,
                                              double* __restrict__ partials, int n) {
  const int r = blockIdx.x * 256 + threadIdx.x;
  double v[1] = {0.0};
  if (r < n) {
    const double diff = double(out[r]) - target[r] * sc->inv_scale;
    v[0] = diff * diff;
    const float gval = float(2.0 * diff / n);
    *(uint4*)(d0 + (size_t)r * 16) = uint4{uint32_t(f2bf(gval)), 0u, 0u, 0u};
    *(uint4*)(d0 + (size_t)r * 16 + 8) = uint4{0u, 0u, 0u, 0u};
  }
  block_partials<1>(v, partials, blockIdx.x, gridDim.x);
}

__global__ __launch_bounds__(1024) void k_loss_final(const double* __restrict__ partials,
                                                     int nblocks, int n,
                                                     UNetScalars* __restrict__ sc) {
  double t[1];
  block_sums_1024<1>(partials, nblocks, t);
  if (threadIdx.x == 0) {
    sc->loss_sum += t[0] / n;
    sc->loss_count += 1;
  }
}

// ---------------------------------------------------------------------------
// Parameters
// ---------------------------------------------------------------------------
// Packed forward weights wf[t][co][ci], backward-data weights wb[t][ci][co] =
// w[taps-1-t][ci][co] (the flipped kernel), padded bias; padding is zero.
__global__ __launch_bounds__(256) void k_pack(const float* __restrict__ p, uint16_t* __restrict__ wf,
                                              uint16_t* __restrict__ wb, float* __restrict__ bias) {
  const int e = blockIdx.x * 256 + threadIdx.x;
  if (e < UNET_BIAS_PADDED) {
    int l = 0;
    while (l + 1 < UNET_LAYERS && UNET[l + 1].pb <= e) ++l;
    const int co = e - UNET[l].pb;
    bias[e] = co < UNET[l].cout ? p[UNET[l].boff + co] : 0.f;
  }
  if (e >= UNET_PACKED) return;
  int l = 0;
  while (l + 1 < UNET_LAYERS && UNET[l + 1].pw <= e) ++l;
  const UNetLayer L = UNET[l];
  const int k = e - L.pw;
  {   // forward: k = (t * coutp + co) * cinp + ci
    const int ci = k % L.cinp, co = (k / L.cinp) % L.coutp, t = k / (L.cinp * L.coutp);
    const bool real = ci < L.cin && co < L.cout;
    wf[e] = real ? f2bf(p[L.woff + (t * L.cin + ci) * L.cout + co]) : 0;
  }
  if (wb) {   // backward-data: k = (t * cinp + ci) * coutp + co
    const int co = k % L.coutp, ci = (k / L.coutp) % L.cinp, t = k / (L.cinp * L.coutp);
    const int tf = L.taps - 1 - t;
    const bool real = ci < L.cin && co < L.cout;
    wb[e] = real ? f2bf(p[L.woff + (tf * L.cin + ci) * L.cout + co]) : 0;
  }
}

__global__ __launch_bounds__(256) void k_adam(float* __restrict__ p, float* __restrict__ g,
                                              float* __restrict__ m, float* __restrict__ v,
                                              float lr, float b1, float b2, float eps, float c1,
                                              float c2, float gscale) {
  const int e = blockIdx.x * 256 + threadIdx.x;
  if (e >= UNET_PARAMS) return;
  const float gr = g[e] * gscale;
  const float mm = b1 * m[e] + (1.f - b1) * gr;
  const float vv = b2 * v[e] + (1.f - b2) * gr * gr;
  m[e] = mm;
  v[e] = vv;
  p[e] -= lr * (mm / c1) / (sqrtf(vv / c2) + eps);
  g[e] = 0.f;
}

// ---------------------------------------------------------------------------
// Host side
// ---------------------------------------------------------------------------
namespace {

inline int blocks_for(long long n) { return int((n + 255) / 256); }

constexpr int WG_MAX_BLOCKS = 1024;

inline int wgrad_subs(int n) {
  const int chunks = (n + 255) / 256;
  return (chunks + WG_MAX_BLOCKS - 1) / WG_MAX_BLOCKS;
}
inline int wgrad_blocks(int n) {
  const int chunks = (n + 255) / 256;
  const int subs = wgrad_subs(n);
  return (chunks + subs - 1) / subs;
}

template <int CIN, int COUT, int T, int EPI>
void conv(const ConvIO& io, const Grid3& g, hipStream_t s) {
  const int tiles = (g.n + 15) / 16;
  if (tiles >= 16384) {
    const int waves = (tiles + 1) / 2;
    hipLaunchKernelGGL((k_conv<CIN, COUT, T, EPI, 2>), dim3((waves + 3) / 4), dim3(256), 0, s, io,
                       g);
  } else {
    hipLaunchKernelGGL((k_conv<CIN, COUT, T, EPI, 1>), dim3((tiles + 3) / 4), dim3(256), 0, s, io,
                       g);
  }
}

template <int CIN, int COUT, int T>
void wgrad(const uint16_t* in, const uint16_t* dy, float* part, float* grad, const UNetLayer& L,
           const Grid3& g, hipStream_t s) {
  const int nblk = wgrad_blocks(g.n);
  hipLaunchKernelGGL((k_wgrad<CIN, COUT, T>), dim3(nblk), dim3(256), 0, s, in, dy, part, g,
                     wgrad_subs(g.n));
  const int per = (T + 1) * CIN * COUT;
  hipLaunchKernelGGL(k_wreduce, dim3((per + 63) / 64), dim3(1024), 0, s, part, nblk, L, grad);
}

size_t align256(size_t b) { return (b + 255) & ~size_t(255); }

}  // namespace

bool UNet::shape_ok(int nx, int ny, int nz) {
  return nx >= 4 && ny >= 4 && nz >= 4 && nx % 4 == 0 && ny % 4 == 0 && nz % 4 == 0 &&
         (long long)nx * ny * nz < (1ll << 31);
}

namespace {
struct UNetCarve {
  char* base;
  size_t off = 0;
  template <typename T>
  T* take(size_t count) {
    T* p = base ? (T*)(base + off) : nullptr;
    off += align256(count * sizeof(T));
    return p;
  }
};

void carve_all(UNet& u, UNetCarve& c, int nx, int ny, int nz, bool training) {
  const size_t n0 = (size_t)nx * ny * nz, n1 = n0 / 8, n2 = n0 / 64;
  u.x0 = c.take<uint16_t>(n0 * 16);
  u.a1 = c.take<uint16_t>(n0 * 16);
  u.p1 = c.take<uint16_t>(n1 * 16);
  u.a2 = c.take<uint16_t>(n1 * 32);
  u.p2 = c.take<uint16_t>(n2 * 32);
  u.a3 = c.take<uint16_t>(n2 * 64);
  u.u3 = c.take<uint16_t>(n2 * 32);
  u.c2 = c.take<uint16_t>(n1 * 32);
  u.u2 = c.take<uint16_t>(n1 * 16);
  u.c1 = c.take<uint16_t>(n0 * 16);
  u.out = c.take<float>(n0);
  u.params = c.take<float>(UNET_PARAMS);
  u.wf = c.take<uint16_t>(UNET_PACKED);
  u.bias = c.take<float>(UNET_BIAS_PADDED);
  u.sc = c.take<UNetScalars>(1);
  u.red = c.take<double>(2 * ((n0 + 255) / 256));
  if (training) {
    u.wb = c.take<uint16_t>(UNET_PACKED);
    u.grad = c.take<float>(UNET_PARAMS);
    u.adam_m = c.take<float>(UNET_PARAMS);
    u.adam_v = c.take<float>(UNET_PARAMS);
    u.d0 = c.take<uint16_t>(n0 * 16);
    u.g1 = c.take<uint16_t>(n0 * 16);
    u.du2 = c.take<uint16_t>(n1 * 16);
    u.g2 = c.take<uint16_t>(n1 * 32);
    u.du3 = c.take<uint16_t>(n2 * 32);
    u.g3 = c.take<uint16_t>(n2 * 64);
    u.dp2 = c.take<uint16_t>(n2 * 32);
    u.gb = c.take<uint16_t>(n1 * 32);
    u.dp1 = c.take<uint16_t>(n1 * 16);
    u.ga = c.take<uint16_t>(n0 * 16);
    size_t part = 0;
    const int ns[3] = {int(n0), int(n1), int(n2)};
    for (int l = 0; l < UNET_LAYERS; ++l) {
      const int lev = l == 0 || l == 5 ? 0 : (l == 1 || l == 4 ? 1 : 2);
      const UNetLayer& L = UNET[l];
      part = std::max(part, (size_t)wgrad_blocks(ns[lev]) * (L.taps + 1) * L.cinp * L.coutp);
    }
    u.wpart = c.take<float>(part);
  }
}
}  // namespace

size_t UNet::bytes(int nx, int ny, int nz, bool training) {
  UNet u;
  UNetCarve c{nullptr};
  carve_all(u, c, nx, ny, nz, training);
  return c.off;
}

void UNet::carve(char* base, int nx, int ny, int nz, bool train) {
  UNetCarve c{base};
  carve_all(*this, c, nx, ny, nz, train);
  training = train;
  for (int l = 0; l < 3; ++l) g[l] = Grid3{nx >> l, ny >> l, nz >> l, (nx >> l) * (ny >> l) * (nz >> l)};
}

hipError_t UNet::init_state() {
  adam_t = 0;
  hipError_t e = hipMemsetAsync(sc, 0, sizeof(UNetScalars), stream);
  if (e == hipSuccess && training) {
    e = hipMemsetAsync(grad, 0, UNET_PARAMS * 4, stream);
    if (e == hipSuccess) e = hipMemsetAsync(adam_m, 0, UNET_PARAMS * 4, stream);
    if (e == hipSuccess) e = hipMemsetAsync(adam_v, 0, UNET_PARAMS * 4, stream);
  }
  return e;
}

void UNet::pack() {
  hipLaunchKernelGGL(k_pack, dim3(blocks_for(UNET_PACKED)), dim3(256), 0, stream, params, wf,
                     training ? wb : nullptr, bias);
}

void UNet::forward(const double* b, const void* solid, bool link, double* guess) {
  hipStream_t s = stream;
  const Grid3 G0 = g[0], G1 = g[1], G2 = g[2];
  const int nb = blocks_for(G0.n);
  hipLaunchKernelGGL(k_in_stats, dim3(nb), dim3(256), 0, s, b, red, G0.n);
  hipLaunchKernelGGL(k_in_final, dim3(1), dim3(1024), 0, s, red, nb, G0.n, double(out_scale), sc);
  if (link)
    hipLaunchKernelGGL(k_input<true>, dim3(nb), dim3(256), 0, s, b, solid, sc, x0, G0.n);
  else
    hipLaunchKernelGGL(k_input<false>, dim3(nb), dim3(256), 0, s, b, solid, sc, x0, G0.n);
  ConvIO io{};
  io.sc = sc;
  // A
  io.in = x0; io.w = wf + UNET[0].pw; io.bias = bias + UNET[0].pb; io.out = a1;
  conv<16, 16, 27, EPI_RELU>(io, G0, s);
  hipLaunchKernelGGL(k_down, dim3(blocks_for((long long)G1.n * 2)), dim3(256), 0, s, a1, p1, 16, G0, G1, 0);
  // B
  io.in = p1; io.w = wf + UNET[1].pw; io.bias = bias + UNET[1].pb; io.out = a2;
  conv<16, 32, 27, EPI_RELU>(io, G1, s);
  hipLaunchKernelGGL(k_down, dim3(blocks_for((long long)G2.n * 4)), dim3(256), 0, s, a2, p2, 32, G1, G2, 0);
  // C
  io.in = p2; io.w = wf + UNET[2].pw; io.bias = bias + UNET[2].pb; io.out = a3;
  conv<32, 64, 27, EPI_RELU>(io, G2, s);
  // D
  io.in = a3; io.w = wf + UNET[3].pw; io.bias = bias + UNET[3].pb; io.out = u3;
  conv<64, 32, 1, EPI_LINEAR>(io, G2, s);
  hipLaunchKernelGGL(k_up_add_relu, dim3(blocks_for((long long)G1.n * 4)), dim3(256), 0, s, u3, a2, c2, 32, G1, G2);
  // E
  io.in = c2; io.w = wf + UNET[4].pw; io.bias = bias + UNET[4].pb; io.out = u2;
  conv<32, 16, 1, EPI_LINEAR>(io, G1, s);
  hipLaunchKernelGGL(k_up_add_relu, dim3(blocks_for((long long)G0.n * 2)), dim3(256), 0, s, u2, a1, c1, 16, G0, G1);
  // F
  io.in = c1; io.w = wf + UNET[5].pw; io.bias = bias + UNET[5].pb; io.out = nullptr;
  io.out32 = out; io.guess = guess;
  conv<16, 16, 27, EPI_OUT>(io, G0, s);
}

void UNet::accumulate(const double* b, const void* solid, const double* target) {
  hipStream_t s = stream;
  forward(b, solid, false, nullptr);
  const Grid3 G0 = g[0], G1 = g[1], G2 = g[2];
  const int nb = blocks_for(G0.n);
  hipLaunchKernelGGL(k_loss, dim3(nb), dim3(256), 0, s, out, target, sc, d0, red, G0.n);
  hipLaunchKernelGGL(k_loss_final, dim3(1), dim3(1024), 0, s, red, nb, G0.n, sc);
  ConvIO io{};
  io.sc = sc;
  // F: weight gradient from (c1, d0); data gradient through the ReLU of c1
  wgrad<16, 16, 27>(c1, d0, wpart, grad, UNET[5], G0, s);
  io.in = d0; io.w = wb + UNET[5].pw; io.act = c1; io.out = g1;
  conv<16, 16, 27, EPI_MASK>(io, G0, s);
  // E: input c2, output gradient = sum of g1 over the 8 children
  hipLaunchKernelGGL(k_down, dim3(blocks_for((long long)G1.n * 2)), dim3(256), 0, s, g1, du2, 16, G0, G1, 1);
  wgrad<32, 16, 1>(c2, du2, wpart, grad, UNET[4], G1, s);
  io.in = du2; io.w = wb + UNET[4].pw; io.act = c2; io.out = g2;
  conv<16, 32, 1, EPI_MASK>(io, G1, s);
  // D: input a3, output gradient = sum of g2 over the children
  hipLaunchKernelGGL(k_down, dim3(blocks_for((long long)G2.n * 4)), dim3(256), 0, s, g2, du3, 32, G1, G2, 1);
  wgrad<64, 32, 1>(a3, du3, wpart, grad, UNET[3], G2, s);
  io.in = du3; io.w = wb + UNET[3].pw; io.act = a3; io.out = g3;
  conv<32, 64, 1, EPI_MASK>(io, G2, s);
  // C: input p2
  wgrad<32, 64, 27>(p2, g3, wpart, grad, UNET[2], G2, s);
  io.in = g3; io.w = wb + UNET[2].pw; io.act = nullptr; io.out = dp2;
  conv<64, 32, 27, EPI_PLAIN>(io, G2, s);
  // a2 gets the skip gradient g2 and the pooled gradient dp2 / 8, then its ReLU
  hipLaunchKernelGGL(k_skip_grad, dim3(blocks_for((long long)G1.n * 4)), dim3(256), 0, s, g2, dp2, a2, gb, 32, G1, G2);
  // B: input p1
  wgrad<16, 32, 27>(p1, gb, wpart, grad, UNET[1], G1, s);
  io.in = gb; io.w = wb + UNET[1].pw; io.out = dp1;
  conv<32, 16, 27, EPI_PLAIN>(io, G1, s);
  hipLaunchKernelGGL(k_skip_grad, dim3(blocks_for((long long)G0.n * 2)), dim3(256), 0, s, g1, dp1, a1, ga, 16, G0, G1);
  // A: input x0
  wgrad<16, 16, 27>(x0, ga, wpart, grad, UNET[0], G0, s);
}

void UNet::adam(float lr, float beta1, float beta2, float eps, float grad_scale) {
  ++adam_t;
  const float c1 = float(1.0 - std::pow(double(beta1), double(adam_t)));
  const float c2 = float(1.0 - std::pow(double(beta2), double(adam_t)));
  hipLaunchKernelGGL(k_adam, dim3(blocks_for(UNET_PARAMS)), dim3(256), 0, stream, params, grad,
                     adam_m, adam_v, lr, beta1, beta2, eps, c1, c2, grad_scale);
  pack();
}

}  // namespace ek
