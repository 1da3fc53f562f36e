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
#include <utility>

#include "fft.h"

namespace mlc {

constexpr int first_factor(int R) {
  return (R % 4 == 0 && R != 4) ? 4 : (R % 5 == 0 ? 5 : (R % 3 == 0 ? 3 : 2));
}

// Compile-time twiddles w_R^m = exp(-2 pi i m / R): the angle is reduced to
// a quadrant k and a remainder psi in [0, pi/2) with integer arithmetic, and
// cos / sin of psi (or of pi/2 - psi, whichever is <= pi/4) are summed from
// their Taylor series, which converge to double precision well within 12
// terms there.
constexpr double ce_pi = 3.141592653589793;
// nested (Horner) form, innermost term first
constexpr double ce_sin_series(double x) {
  const double x2 = x * x;
  double s = 1.0;
  for (int k = 12; k >= 1; --k) s = 1.0 - x2 / double((2 * k) * (2 * k + 1)) * s;
  return x * s;
}
constexpr double ce_cos_series(double x) {
  const double x2 = x * x;
  double s = 1.0;
  for (int k = 12; k >= 1; --k) s = 1.0 - x2 / double((2 * k - 1) * (2 * k)) * s;
  return s;
}
struct CosSin { double c, s; };
constexpr CosSin ce_cossin_2pi(int m, int R) {   // cos, sin of 2 pi m / R
  const int q = (4 * (m % R) + 4 * R) % (4 * R);  // angle in quarter turns, times R
  const int k = q / R, rem = q % R;               // angle = (k + rem / R) pi / 2
  double c0, s0;
  if (2 * rem <= R) {
    const double psi = (ce_pi / 2) * double(rem) / double(R);
    c0 = ce_cos_series(psi);
    s0 = ce_sin_series(psi);
  } else {
    const double phi = (ce_pi / 2) * double(R - rem) / double(R);
    c0 = ce_sin_series(phi);
    s0 = ce_cos_series(phi);
  }
  switch (k) {
    case 0: return {c0, s0};
    case 1: return {-s0, c0};
    case 2: return {-c0, -s0};
    default: return {s0, -c0};
  }
}
template <int R> struct TwiddleTable {
  double c[R], s[R];   // w_R^m = c[m] - i s[m]
  constexpr TwiddleTable() : c(), s() {
    for (int m = 0; m < R; ++m) {
      const CosSin cs = ce_cossin_2pi(m, R);
      c[m] = cs.c;
      s[m] = cs.s;
    }
  }
};
template <int R> inline constexpr TwiddleTable<R> kTwiddle{};

// w_R^m (forward, DIR > 0) or its conjugate (inverse), as constants
template <typename T, int R, int DIR, int MM>
__device__ __forceinline__ cplx<T> twc() {
  constexpr int m = MM % R;
  constexpr double c = kTwiddle<R>.c[m], sn = kTwiddle<R>.s[m];
  return {T(c), T(DIR > 0 ? -sn : sn)};
}

// v * w_R^m with the trivial angles (multiples of a quarter turn) exact
template <typename T, int R, int DIR, int MM>
__device__ __forceinline__ cplx<T> twmul(cplx<T> a) {
  constexpr int m = MM % R;
  if constexpr (m == 0) {
    return a;
  } else if constexpr (4 * m == R) {
    return rot90<T, DIR>(a);
  } else if constexpr (2 * m == R) {
    return {-a.x, -a.y};
  } else if constexpr (4 * m == 3 * R) {
    return rot90<T, -DIR>(a);
  } else {
    return cmul(a, twc<T, R, DIR, m>());
  }
}

namespace detail {
template <typename T, int R, int DIR, int A, int B, int J2, int K1>
__device__ __forceinline__ void first_stage_entry(const cplx<T>* a, cplx<T>* tmp) {
  tmp[J2 * A + K1] = twmul<T, R, DIR, J2 * K1>(a[K1]);
}
template <typename T, int R, int DIR, int A, int B, int J2, int... K1s>
__device__ __forceinline__ void first_stage_row(const cplx<T>* a, cplx<T>* tmp, std::integer_sequence<int, K1s...>) {
  (first_stage_entry<T, R, DIR, A, B, J2, K1s>(a, tmp), ...);
}
}  // namespace detail

// In-place DFT of R values in registers, natural order in and out.
template <typename T, int R, int DIR>
__device__ __forceinline__ void dft_reg(cplx<T>* v);

namespace detail {
template <typename T, int R, int DIR, int A, int B, int J2>
__device__ __forceinline__ void dft_first(cplx<T>* v, cplx<T>* tmp) {
  cplx<T> a[A];
#pragma unroll
  for (int j1 = 0; j1 < A; ++j1) a[j1] = v[J2 + B * j1];
  dft_small<T, A, DIR>(a);
  first_stage_row<T, R, DIR, A, B, J2>(a, tmp, std::make_integer_sequence<int, A>{});
}
template <typename T, int R, int DIR, int A, int B, int... J2s>
__device__ __forceinline__ void dft_first_all(cplx<T>* v, cplx<T>* tmp, std::integer_sequence<int, J2s...>) {
  (dft_first<T, R, DIR, A, B, J2s>(v, tmp), ...);
}
// pruned first stage: only v[J2] (J2 < NZ) nonzero, one input per first-stage DFT
template <typename T, int R, int DIR, int A, int B, int NZ, int J2, int... K1s>
__device__ __forceinline__ void first_nz_row(const cplx<T>* v, cplx<T>* tmp, std::integer_sequence<int, K1s...>) {
  if constexpr (J2 < NZ) {
    ((tmp[J2 * A + K1s] = twmul<T, R, DIR, J2 * K1s>(v[J2])), ...);
  } else {
    ((tmp[J2 * A + K1s] = cplx<T>{T(0), T(0)}), ...);
  }
}
template <typename T, int R, int DIR, int A, int B, int NZ, int... J2s>
__device__ __forceinline__ void first_nz_all(const cplx<T>* v, cplx<T>* tmp, std::integer_sequence<int, J2s...>) {
  (first_nz_row<T, R, DIR, A, B, NZ, J2s>(v, tmp, std::make_integer_sequence<int, A>{}), ...);
}
}  // namespace detail

template <typename T, int R, int DIR>
__device__ __forceinline__ void dft_reg(cplx<T>* v) {
  if constexpr (R == 1) {
    return;
  } else if constexpr (R == 2 || R == 3 || R == 4 || R == 5) {
    dft_small<T, R, DIR>(v);
  } else {
    constexpr int A = first_factor(R), B = R / A;
    cplx<T> tmp[R];
    detail::dft_first_all<T, R, DIR, A, B>(v, tmp, std::make_integer_sequence<int, B>{});
#pragma unroll
    for (int k1 = 0; k1 < A; ++k1) {
      cplx<T> bb[B];
#pragma unroll
      for (int j2 = 0; j2 < B; ++j2) bb[j2] = tmp[j2 * A + k1];
      dft_reg<T, B, DIR>(bb);
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
__device__ __forceinline__ void dft_reg_nz(cplx<T>* v) {
  constexpr int A = first_factor(R), B = R / A;
  if constexpr (NZ >= R || R <= 5 || NZ > B) {
    dft_reg<T, R, DIR>(v);
  } else {
    cplx<T> tmp[R];
    detail::first_nz_all<T, R, DIR, A, B, NZ>(v, tmp, std::make_integer_sequence<int, B>{});
#pragma unroll
    for (int k1 = 0; k1 < A; ++k1) {
      cplx<T> bb[B];
#pragma unroll
      for (int j2 = 0; j2 < B; ++j2) bb[j2] = tmp[j2 * A + k1];
      dft_reg_nz<T, B, DIR, NZ>(bb);
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
