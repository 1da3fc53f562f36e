// Shared definitions of libmlc's device code and host orchestration.
#pragma once
#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

#include "fft.h"

namespace mlc {

constexpr int NREF = 4;     // fine/coarse refinement ratio
constexpr int PMAX = 9;     // Legendre truncation order built (modes of total degree < P)
constexpr int KMAX = PMAX * (PMAX + 1) * (PMAX + 2) / 6;   // 165 moments at P = 9
constexpr int SMAX = 33;    // patch nodes per axis, n <= 32
constexpr int SMAXN = SMAX;

// Mehrstellen coefficients b_0..b_3 (19- and 27-point operators).
struct Stencil { double b[4]; };
inline Stencil stencil_of(int Q) {
  if (Q == 4) return {{-4.0, 1.0 / 3.0, 1.0 / 6.0, 0.0}};
  return {{-64.0 / 15.0, 7.0 / 15.0, 1.0 / 10.0, 1.0 / 30.0}};
}

__host__ __device__ inline int64_t cube(int64_t a) { return a * a * a; }

// Orthonormal Legendre polynomial sqrt((2a+1)/2) P_a(t) (sec. 3): closed
// forms up to degree 3, Bonnet's recurrence (k+1) P_{k+1} = (2k+1) t P_k -
// k P_{k-1} above.
__host__ __device__ inline double qhat(int a, double t) {
  switch (a) {
    case 0: return 0.70710678118654752440;
    case 1: return 1.22474487139158904910 * t;
    case 2: return 1.58113883008418966600 * 0.5 * (3.0 * t * t - 1.0);
    case 3: return 1.87082869338697069280 * 0.5 * (5.0 * t * t * t - 3.0 * t);
    default: {
      double pm = 1.0, pk = t;
      for (int k = 1; k < a; ++k) {
        const double pn = ((2 * k + 1) * t * pk - k * pm) / (k + 1);
        pm = pk;
        pk = pn;
      }
      return sqrt((2 * a + 1) * 0.5) * pk;
    }
  }
}

// Composite Boole weight of node j of [0, n] mapped to [-1, 1] (n % 4 == 0),
// the quadrature of the moments (sec. 4.1, step 1).
__host__ __device__ inline double boole_w(int j, int n) {
  double base = 4.0 / (45.0 * n);   // (2 delta / 45), delta = 2/n
  if (j == 0 || j == n) return 7.0 * base;
  int r = j & 3;
  return (r == 0 ? 14.0 : (r == 2 ? 12.0 : 32.0)) * base;
}

// A pointer taken from a descriptor as a global-memory pointer, so that its
// accesses compile to global (not flat) instructions.
template <typename T>
__device__ __forceinline__ __attribute__((address_space(1))) T* gbl(T* p) {
  return (__attribute__((address_space(1))) T*)p;
}

// Partial moment sums per patch z-plane: one per (a1, a2), a1, a2 < P, at
// index a1 P + a2.

// Output-coordinate list of the local fields along one axis: b coarse nodes
// below Omega_alpha, every node of Omega_alpha, b coarse nodes above.
__host__ __device__ inline int out_coord(int i, int b, int Wa, int e, int da, int n) {
  if (i < b) return -e + NREF * i;
  if (i < b + Wa) return -da + (i - b);
  return n + da + NREF * (i - b - Wa + 1);
}

// One problem of a batch as the patch-level kernels see it.  Patches of all
// problems are numbered consecutively: problem k owns the global patch slots
// [patch0, patch0 + ppa^3).
struct ProbDesc {
  const double* f;
  double* phi;
  double* phiB;
  int N, ppa, patch0;
  int skip;     // 1: patches whose node charge is all zero skip their local convolutions
  double h2;    // h^2
  double R15;   // (n h / 2)^{3/2}, the Legendre basis scale
  double c2h2;  // C2 h^2 of the final correction, 0 for a coarser level of the multilevel method
};

// Index of the problem owning global patch slot g (descriptors sorted by
// patch0, patch0 of the first is 0).
__device__ __forceinline__ int find_problem(const ProbDesc* __restrict__ pd, int nprob, int g) {
  int lo = 0, hi = nprob - 1;
  while (lo < hi) {
    int mid = (lo + hi + 1) >> 1;
    if (pd[mid].patch0 <= g) lo = mid; else hi = mid - 1;
  }
  return lo;
}

// Descriptors travel to the device as kernel arguments, DESC_PACK at a time.
constexpr int DESC_PACK = 8;
struct DescPack { ProbDesc d[DESC_PACK]; int count; };
__global__ void desc_upload_kernel(ProbDesc* __restrict__ dst, DescPack pk) {
  if (int(threadIdx.x) < pk.count) dst[threadIdx.x] = pk.d[threadIdx.x];
}

}  // namespace mlc
