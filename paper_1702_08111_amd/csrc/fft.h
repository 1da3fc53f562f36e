// In-LDS batched complex FFTs for gfx950 (wave64), radices 2, 3, 4, 5.
//
// A batch of NL lines of length M lives in LDS; element e of line l sits at
// buf[l * LS + e * ES].  The transform is Stockham autosort, in place: each
// stage reads every butterfly's R inputs into registers, synchronises, and
// writes the R outputs, so one buffer suffices.  Sizes are compile-time so
// that the per-thread register arrays are fixed.
//
// Forward: X[k] = sum_j x[j] exp(-2 pi i j k / M); inverse: the conjugate
// kernel, unnormalised.
#pragma once
#include <hip/hip_runtime.h>

namespace mlc {

template <typename T> struct cplx { T x, y; };

template <typename T> __device__ __forceinline__ cplx<T> cadd(cplx<T> a, cplx<T> b) { return {a.x + b.x, a.y + b.y}; }
template <typename T> __device__ __forceinline__ cplx<T> csub(cplx<T> a, cplx<T> b) { return {a.x - b.x, a.y - b.y}; }
template <typename T> __device__ __forceinline__ cplx<T> cmul(cplx<T> a, cplx<T> b) {
  return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
template <typename T> __device__ __forceinline__ cplx<T> cscale(cplx<T> a, T s) { return {a.x * s, a.y * s}; }
// multiply by -i (DIR = +1, forward) or +i (DIR = -1, inverse)
template <typename T, int DIR> __device__ __forceinline__ cplx<T> rot90(cplx<T> a) {
  if constexpr (DIR > 0) return {a.y, -a.x};
  else return {-a.y, a.x};
}

// ---- radix plans -------------------------------------------------------
// Factor M into radices, 4 first, then 5, 3, 2.  Stored as a small constexpr
// array so the stage loop unrolls.
struct RadixPlan { int n; int r[12]; };

constexpr RadixPlan make_plan(int M) {
  RadixPlan p{0, {0}};
  int m = M;
  while (m % 4 == 0 && m > 4) { p.r[p.n++] = 4; m /= 4; }
  while (m % 5 == 0) { p.r[p.n++] = 5; m /= 5; }
  while (m % 3 == 0) { p.r[p.n++] = 3; m /= 3; }
  while (m % 4 == 0) { p.r[p.n++] = 4; m /= 4; }
  while (m % 2 == 0) { p.r[p.n++] = 2; m /= 2; }
  if (m != 1) p.n = -1;  // unsupported prime factor
  return p;
}

constexpr bool fft_size_ok(int M) { return M >= 2 && make_plan(M).n > 0; }

// ---- butterflies ---------------------------------------------------------
template <typename T, int R, int DIR>
__device__ __forceinline__ void dft_small(cplx<T>* v) {
  if constexpr (R == 2) {
    cplx<T> a = v[0], b = v[1];
    v[0] = cadd(a, b);
    v[1] = csub(a, b);
  } else if constexpr (R == 4) {
    cplx<T> a = cadd(v[0], v[2]), b = csub(v[0], v[2]);
    cplx<T> c = cadd(v[1], v[3]), d = rot90<T, DIR>(csub(v[1], v[3]));
    v[0] = cadd(a, c);
    v[2] = csub(a, c);
    v[1] = cadd(b, d);
    v[3] = csub(b, d);
  } else if constexpr (R == 3) {
    // exp(-2 pi i / 3) = -1/2 - i sqrt(3)/2
    const T c1 = T(-0.5);
    const T s1 = T(DIR > 0 ? -0.86602540378443864676 : 0.86602540378443864676);
    cplx<T> a = v[0], b = v[1], c = v[2];
    cplx<T> t = cadd(b, c);
    cplx<T> u = csub(b, c);
    cplx<T> m = {a.x + c1 * t.x, a.y + c1 * t.y};
    // i * s1 * u
    cplx<T> r = {-s1 * u.y, s1 * u.x};
    v[0] = cadd(a, t);
    v[1] = cadd(m, r);
    v[2] = csub(m, r);
  } else if constexpr (R == 5) {
    // cos/sin of 2 pi / 5 and 4 pi / 5
    const T c1 = T(0.30901699437494742410), c2 = T(-0.80901699437494742410);
    const T sg = T(DIR > 0 ? -1 : 1);
    const T s1 = sg * T(0.95105651629515357212), s2 = sg * T(0.58778525229247312917);
    cplx<T> a = v[0];
    cplx<T> t1 = cadd(v[1], v[4]), u1 = csub(v[1], v[4]);
    cplx<T> t2 = cadd(v[2], v[3]), u2 = csub(v[2], v[3]);
    cplx<T> m1 = {a.x + c1 * t1.x + c2 * t2.x, a.y + c1 * t1.y + c2 * t2.y};
    cplx<T> m2 = {a.x + c2 * t1.x + c1 * t2.x, a.y + c2 * t1.y + c1 * t2.y};
    // X1 = m1 + i(s1 u1 + s2 u2), X4 = m1 - i(...), X2 = m2 + i(s2 u1 - s1 u2), X3 = m2 - i(...)
    cplx<T> n1 = {s1 * u1.x + s2 * u2.x, s1 * u1.y + s2 * u2.y};
    cplx<T> n2 = {s2 * u1.x - s1 * u2.x, s2 * u1.y - s1 * u2.y};
    cplx<T> in1 = {-n1.y, n1.x}, in2 = {-n2.y, n2.x};
    v[0] = {a.x + t1.x + t2.x, a.y + t1.y + t2.y};
    v[1] = cadd(m1, in1);
    v[4] = csub(m1, in1);
    v[2] = cadd(m2, in2);
    v[3] = csub(m2, in2);
  }
}

// ---- twiddle table -------------------------------------------------------
// tw[j] = exp(-2 pi i j / M), j in [0, M), computed in float64 with an
// exact integer argument and rounded to T.
template <typename T>
__device__ void fill_twiddles(cplx<T>* tw, int M) {
  for (int j = threadIdx.x; j < M; j += blockDim.x) {
    double s, c;
    sincospi(-2.0 * double(j) / double(M), &s, &c);
    tw[j] = {T(c), T(s)};
  }
}

// ---- one Stockham stage ----------------------------------------------------
// LINE_FAST: consecutive threads take consecutive lines (good when lines are
// adjacent columns, ES > 1, LS == 1); otherwise consecutive elements of one
// line (good for contiguous rows).
template <typename T, int M, int R, int NS, int NL, int NT, int DIR, bool LINE_FAST>
__device__ __forceinline__ void fft_stage(cplx<T>* buf, int LS, int ES, const cplx<T>* tw, int tid) {
  constexpr int NB1 = M / R;          // butterflies per line
  constexpr int NB = NB1 * NL;
  constexpr int PER = (NB + NT - 1) / NT;
  cplx<T> v[PER][R];
#pragma unroll
  for (int p = 0; p < PER; ++p) {
    int b = tid + p * NT;
    if (NB % NT == 0 || b < NB) {
      int line = LINE_FAST ? (b % NL) : (b / NB1);
      int j = LINE_FAST ? (b / NL) : (b % NB1);
      cplx<T>* base = buf + line * LS;
#pragma unroll
      for (int m = 0; m < R; ++m) v[p][m] = base[(j + m * NB1) * ES];
    }
  }
  __syncthreads();
#pragma unroll
  for (int p = 0; p < PER; ++p) {
    int b = tid + p * NT;
    if (NB % NT == 0 || b < NB) {
      int line = LINE_FAST ? (b % NL) : (b / NB1);
      int j = LINE_FAST ? (b / NL) : (b % NB1);
      int k = j % NS;
      if constexpr (NS > 1) {
#pragma unroll
        for (int m = 1; m < R; ++m) {
          cplx<T> w = tw[(m * k) * (M / (NS * R))];
          if constexpr (DIR < 0) w.y = -w.y;
          v[p][m] = cmul(v[p][m], w);
        }
      }
      dft_small<T, R, DIR>(v[p]);
      int outb = (j / NS) * NS * R + k;
      cplx<T>* base = buf + line * LS;
#pragma unroll
      for (int m = 0; m < R; ++m) base[(outb + m * NS) * ES] = v[p][m];
    }
  }
  __syncthreads();
}

template <typename T, int M, int STAGE, int NS, int NL, int NT, int DIR, bool LINE_FAST>
__device__ __forceinline__ void fft_stages(cplx<T>* buf, int LS, int ES, const cplx<T>* tw, int tid) {
  constexpr RadixPlan plan = make_plan(M);
  if constexpr (STAGE < plan.n) {
    constexpr int R = plan.r[STAGE];
    fft_stage<T, M, R, NS, NL, NT, DIR, LINE_FAST>(buf, LS, ES, tw, tid);
    fft_stages<T, M, STAGE + 1, NS * R, NL, NT, DIR, LINE_FAST>(buf, LS, ES, tw, tid);
  }
}

// Transform NL lines of length M in place (all NT threads of the block
// participate; the call begins and ends with the buffer consistent).
template <typename T, int M, int NL, int NT, int DIR, bool LINE_FAST>
__device__ __forceinline__ void fft_lines(cplx<T>* buf, int LS, int ES, const cplx<T>* tw) {
  static_assert(fft_size_ok(M), "FFT length must factor into 2, 3, 5");
  fft_stages<T, M, 0, 1, NL, NT, DIR, LINE_FAST>(buf, LS, ES, tw, threadIdx.x);
}

}  // namespace mlc
