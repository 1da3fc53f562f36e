// Shared definitions of libmlc's device code and host orchestration.
#pragma once
#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

#include "fft.h"

namespace mlc {

constexpr int NREF = 4;     // fine/coarse refinement ratio
constexpr int KMAX = 20;    // Legendre moments for P <= 4
constexpr int SMAX = 33;    // patch nodes per axis, n <= 32
constexpr int SMAXN = SMAX;

// Mehrstellen coefficients b_0..b_3 (19- and 27-point operators).
struct Stencil { double b[4]; };
inline Stencil stencil_of(int Q) {
  if (Q == 4) return {{-4.0, 1.0 / 3.0, 1.0 / 6.0, 0.0}};
  return {{-64.0 / 15.0, 7.0 / 15.0, 1.0 / 10.0, 1.0 / 30.0}};
}

__host__ __device__ inline int64_t cube(int64_t a) { return a * a * a; }

// Output-coordinate list of the local fields along one axis: b coarse nodes
// below Omega_alpha, every node of Omega_alpha, b coarse nodes above.
__host__ __device__ inline int out_coord(int i, int b, int Wa, int e, int da, int n) {
  if (i < b) return -e + NREF * i;
  if (i < b + Wa) return -da + (i - b);
  return n + da + NREF * (i - b - Wa + 1);
}

}  // namespace mlc
