// Counter-based random numbers for the thermal noise (Sec. II.B and II.C):
// Philox4x32-10 (Salmon, Moraes, Dror and Shaw, SC 2011), uniforms
// (x + 1/2) 2^-32 in (0, 1), and standard normals by the Box-Muller
// transform on word pairs (0, 1) and (2, 3).  Also the D3Q19 mode
// polynomials whose normalised forms carry the lattice noise.
//
// Streams (key = the 64-bit seed split into its low and high words):
//   lattice noise of species a at site r in step t: counters (r, t, 4 a + j, 0)
//     for j = 0..3, normals 4 j .. 4 j + 3, the first 15 driving modes 4..18;
//   bead noise of bead i in step t, substep s: counter (i, t, s, 1), normals
//     0..2 the x, y, z components.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "ek_internal.h"

namespace ek {

struct Philox4 {
  uint32_t v[4];
};

__host__ __device__ inline uint32_t mulhi32(uint32_t a, uint32_t b) {
  return uint32_t((uint64_t(a) * uint64_t(b)) >> 32);
}

// Ten rounds of Philox4x32 on counter c with key (k0, k1).
__host__ __device__ inline Philox4 philox4x32_10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                                 uint32_t k0, uint32_t k1) {
  constexpr uint32_t MA = 0xD2511F53u, MB = 0xCD9E8D57u;   // round multipliers
  constexpr uint32_t WA = 0x9E3779B9u, WB = 0xBB67AE85u;   // key increments
#pragma unroll
  for (int round = 0; round < 10; ++round) {
    const uint32_t hiA = mulhi32(MA, c0), loA = MA * c0;
    const uint32_t hiB = mulhi32(MB, c2), loB = MB * c2;
    const uint32_t n0 = hiB ^ c1 ^ k0, n2 = hiA ^ c3 ^ k1;
    c0 = n0;
    c1 = loB;
    c2 = n2;
    c3 = loA;
    k0 += WA;
    k1 += WB;
  }
  return Philox4{{c0, c1, c2, c3}};
}

// Uniform in (0, 1) of a 32-bit word, in T.
template <typename T>
__device__ inline T word_uniform(uint32_t x) {
  return T((double(x) + 0.5) * 2.3283064365386962890625e-10);
}

// Four standard normals from one Philox output: Box-Muller in T.
template <typename T>
__device__ inline void box_muller4(const Philox4& w, T (&z)[4]) {
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const T u1 = word_uniform<T>(w.v[2 * h]);
    const T u2 = word_uniform<T>(w.v[2 * h + 1]);
    T s, c;
    if constexpr (sizeof(T) == 4) {
      const float r = sqrtf(-2.0f * logf(u1));
      sincospif(2.0f * u2, &s, &c);
      z[2 * h] = r * c;
      z[2 * h + 1] = r * s;
    } else {
      const double r = sqrt(-2.0 * log(u1));
      sincospi(2.0 * u2, &s, &c);
      z[2 * h] = r * c;
      z[2 * h + 1] = r * s;
    }
  }
}

// Unnormalised D3Q19 mode polynomial k (0..18) at population p: integers.
// 0: 1; 1-3: c; 4: c^2 - 1; 5: 3 cx^2 - c^2; 6: cy^2 - cz^2; 7-9: cx cy,
// cy cz, cx cz; 10-12: (3 c^2 - 5) c; 13-15: (cy^2 - cz^2) cx,
// (cz^2 - cx^2) cy, (cx^2 - cy^2) cz; 16: 3 c^4 - 6 c^2 + 1;
// 17: (2 c^2 - 3)(3 cx^2 - c^2); 18: (2 c^2 - 3)(cy^2 - cz^2).
__host__ __device__ constexpr int mode_poly(int k, int p) {
  const int x = CX[p], y = CY[p], z = CZ[p];
  const int x2 = x * x, y2 = y * y, z2 = z * z, c2 = x2 + y2 + z2;
  switch (k) {
    case 0: return 1;
    case 1: return x;
    case 2: return y;
    case 3: return z;
    case 4: return c2 - 1;
    case 5: return 3 * x2 - c2;
    case 6: return y2 - z2;
    case 7: return x * y;
    case 8: return y * z;
    case 9: return x * z;
    case 10: return (3 * c2 - 5) * x;
    case 11: return (3 * c2 - 5) * y;
    case 12: return (3 * c2 - 5) * z;
    case 13: return (y2 - z2) * x;
    case 14: return (z2 - x2) * y;
    case 15: return (x2 - y2) * z;
    case 16: return 3 * c2 * c2 - 6 * c2 + 1;
    case 17: return (2 * c2 - 3) * (3 * x2 - c2);
    default: return (2 * c2 - 3) * (y2 - z2);
  }
}

// Noise parameters of the fused lattice step.
struct NoiseParams {
  uint32_t key0 = 0, key1 = 0;   // the seed's low and high words
  uint32_t step = 0;             // steps completed before this one
  double amp2[3] = {0, 0, 0};    // m omega (2 - omega) per species, m = k_B T / v_T^2
  double inv_norm[15] = {};      // 1 / sqrt(sum_p w_p mode_poly(k, p)^2), k = 4..18
};

// Stochastic term of one species at site r: g[p] += Delta_p with
// Delta_p = sqrt(amp2 n) w_p sum_{k=4}^{18} chi_kp N_k (density n clamped
// at zero).
template <typename T>
__device__ inline void add_lattice_noise(T (&g)[Q], const NoiseParams& np, int species, uint32_t r,
                                         T n) {
  T s[16];
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const Philox4 w = philox4x32_10(r, np.step, uint32_t(4 * species + j), 0u, np.key0, np.key1);
    T z[4];
    box_muller4<T>(w, z);
#pragma unroll
    for (int c = 0; c < 4; ++c) s[4 * j + c] = z[c];
  }
  const T amp = sqrt(T(np.amp2[species]) * (n > T(0) ? n : T(0)));
#pragma unroll
  for (int k = 0; k < 15; ++k) s[k] *= T(np.inv_norm[k]) * amp;
#pragma unroll
  for (int p = 0; p < Q; ++p) {
    T d = T(0);
#pragma unroll
    for (int k = 0; k < 15; ++k) {
      const int e = mode_poly(k + 4, p);
      if (e) d += T(e) * s[k];
    }
    g[p] += T(weight(p)) * d;
  }
}

}  // namespace ek
