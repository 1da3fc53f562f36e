// Register-resident DFTs and the two-pass line FFT used by the local
// convolution kernels.
//
// A length-M transform is split as M = R1 * R2.  Pass 1 (R2 threads per
// line): thread t takes x[t + R2 j1], j1 < R1, does an R1-point DFT in
// registers and multiplies by w_M^(t k1).  After one exchange through LDS,
// pass 2 (R1 threads per line): thread s takes the R2 values of column s and
// does an R2-point DFT, giving X[s + R1 k2], k2 < R2.  The inverse runs the
// same steps backwards, so the forward transform, a pointwise product and
// the first inverse pass all happen in the same registers, with one LDS
// exchange per direction.
#pragma once
#include "fft.h"

namespace mlc {

constexpr int first_factor(int R) {
  return (R % 4 == 0 && R != 4) ? 4 : (R % 5 == 0 ? 5 : (R % 3 == 0 ? 3 : 2));
}

// In-place DFT of R values in registers, natural order in and out.
// tw[m * step] must be w_R^m = exp(-2 pi i m / R) (forward convention).
template <typename T, int R, int DIR>
__device__ __forceinline__ void dft_reg(cplx<T>* v, const cplx<T>* tw, int step) {
  if constexpr (R == 1) {
    return;
  } else if constexpr (R == 2 || R == 3 || R == 4 || R == 5) {
    dft_small<T, R, DIR>(v);
  } else {
    constexpr int A = first_factor(R), B = R / A;
    cplx<T> tmp[R];
#pragma unroll
    for (int j2 = 0; j2 < B; ++j2) {
      cplx<T> a[A];
#pragma unroll
      for (int j1 = 0; j1 < A; ++j1) a[j1] = v[j2 + B * j1];
      dft_small<T, A, DIR>(a);
#pragma unroll
      for (int k1 = 0; k1 < A; ++k1) {
        if (j2 * k1 == 0) {
          tmp[j2 * A + k1] = a[k1];
        } else {
          cplx<T> w = tw[((j2 * k1) % R) * step];
          if constexpr (DIR < 0) w.y = -w.y;
          tmp[j2 * A + k1] = cmul(a[k1], w);
        }
      }
    }
#pragma unroll
    for (int k1 = 0; k1 < A; ++k1) {
      cplx<T> bb[B];
#pragma unroll
      for (int j2 = 0; j2 < B; ++j2) bb[j2] = tmp[j2 * A + k1];
      dft_reg<T, B, DIR>(bb, tw, step * A);
#pragma unroll
      for (int k2 = 0; k2 < B; ++k2) v[k1 + A * k2] = bb[k2];
    }
  }
}

// The same DFT when only the first NZ inputs can be nonzero (zero-padded
// source lines): with R = A * B and NZ <= B, the first-stage DFTs over
// v[j2 + B j1] each see one input (j1 = 0), so they reduce to the twiddle
// products, and the second-stage DFTs again have NZ leading inputs.
template <typename T, int R, int DIR, int NZ>
__device__ __forceinline__ void dft_reg_nz(cplx<T>* v, const cplx<T>* tw, int step) {
  constexpr int A = first_factor(R), B = R / A;
  if constexpr (NZ >= R || R <= 5 || NZ > B) {
    dft_reg<T, R, DIR>(v, tw, step);
  } else {
    cplx<T> tmp[R];
#pragma unroll
    for (int j2 = 0; j2 < B; ++j2)
#pragma unroll
      for (int k1 = 0; k1 < A; ++k1) {
        if (j2 >= NZ) {
          tmp[j2 * A + k1] = {T(0), T(0)};
        } else if (j2 * k1 == 0) {
          tmp[j2 * A + k1] = v[j2];
        } else {
          cplx<T> w = tw[((j2 * k1) % R) * step];
          if constexpr (DIR < 0) w.y = -w.y;
          tmp[j2 * A + k1] = cmul(v[j2], w);
        }
      }
#pragma unroll
    for (int k1 = 0; k1 < A; ++k1) {
      cplx<T> bb[B];
#pragma unroll
      for (int j2 = 0; j2 < B; ++j2) bb[j2] = tmp[j2 * A + k1];
      dft_reg_nz<T, B, DIR, NZ>(bb, tw, step * A);
#pragma unroll
      for (int k2 = 0; k2 < B; ++k2) v[k1 + A * k2] = bb[k2];
    }
  }
}

// Split M = R1 * R2 with R1 (pass-2 threads per line, the heavier pass in the
// convolution) >= R2, both at most 16.
template <int M> struct Split;
template <> struct Split<50> { static constexpr int R1 = 10, R2 = 5; };
template <> struct Split<64> { static constexpr int R1 = 8, R2 = 8; };
template <> struct Split<72> { static constexpr int R1 = 9, R2 = 8; };
template <> struct Split<90> { static constexpr int R1 = 10, R2 = 9; };
template <> struct Split<96> { static constexpr int R1 = 12, R2 = 8; };
template <> struct Split<120> { static constexpr int R1 = 12, R2 = 10; };
template <> struct Split<128> { static constexpr int R1 = 16, R2 = 8; };
template <> struct Split<150> { static constexpr int R1 = 15, R2 = 10; };
template <> struct Split<160> { static constexpr int R1 = 16, R2 = 10; };
template <> struct Split<180> { static constexpr int R1 = 15, R2 = 12; };
template <> struct Split<192> { static constexpr int R1 = 16, R2 = 12; };

// Exchange buffer layouts (padded rows against bank conflicts), per line:
//   forward  F[t][k1]: offset t * (R1 + 1) + k1
//   inverse  B[s][t]:  offset s * (R2 + 1) + t
template <int M> struct XLayout {
  static constexpr int R1 = Split<M>::R1, R2 = Split<M>::R2;
  static constexpr int FWD = R2 * (R1 + 1), INV = R1 * (R2 + 1);
  static constexpr int LINE = FWD > INV ? FWD : INV;
};

}  // namespace mlc
