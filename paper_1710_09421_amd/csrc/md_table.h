// Table of the lattice nodes touched by the beads in the current step.
//
// Beads deposit their charge and spread their friction onto the 8 trilinear
// corner nodes.  Those few nodes are kept in an open-addressing hash table
// (key = site index) holding fixed-point sums, so that contributions from
// different beads and substeps add up in any order to the same bits.  The
// site's link word carries MASK_BEAD so that the lattice kernels probe the
// table only where a bead is near.
#pragma once

#include <hip/hip_runtime.h>

#include "ek_internal.h"

namespace ek {

__host__ __device__ inline int hash_slot(long long r, int bits) {
  return int(((unsigned long long)r * 0x9E3779B97F4A7C15ull) >> (64 - bits));
}

// Slot layout: charge, then K[species][xyz] (9 values), all int64 fixed point.
constexpr int SLOT_VALUES = 10;

struct BeadTableView {
  const int* keys = nullptr;               // 2^bits keys, -1 = empty
  const long long* vals = nullptr;         // [2^bits][SLOT_VALUES]
  int bits = HASH_BITS;

  __device__ int find(long long r) const {
    const int slots = 1 << bits;
    int h = hash_slot(r, bits);
    for (int k = 0; k < slots; ++k) {
      const int key = keys[h];
      if (key == int(r)) return h;
      if (key < 0) return -1;
      h = (h + 1) & (slots - 1);
    }
    return -1;
  }
  __device__ double charge_at(long long r) const {
    const int h = find(r);
    return h < 0 ? 0.0 : double(vals[(size_t)h * SLOT_VALUES]) * (1.0 / FIX_CHARGE);
  }
  __device__ void force_at(long long r, double (&k)[3][3]) const {
    const int h = find(r);
#pragma unroll
    for (int s = 0; s < 3; ++s)
#pragma unroll
      for (int c = 0; c < 3; ++c)
        k[s][c] = h < 0 ? 0.0 : double(vals[(size_t)h * SLOT_VALUES + 1 + 3 * s + c]) * (1.0 / FIX_FORCE);
  }
};

}  // namespace ek
