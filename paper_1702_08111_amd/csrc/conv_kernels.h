// Local discrete convolutions phi_i = G^h * (chi_i f) of every patch by
// Hockney's method (sec. 4.1 step 1; appendix A.2), batched over patches.
//
// Torus M^3 per patch; the source chi_i f occupies slots [0, n]^3, output
// node x (patch-relative, x in [-e, n+e]) sits at slot x mod M, and the
// kernel is the DGF "symmetric fill" (real, even), so its spectrum is real
// and even and is stored as the octant spec[kx][kz'][ky'] (kx = wavenumber of
// the fastest array axis) with 1/M^3 folded in.  M >= 2(n+e)+1 makes the
// periodic convolution equal the free-space one on every output node.
//
// Three kernels, arithmetic in T (float or double):
//   xdft  block (sz, patch): X[p][kx][sz][sy] = sum_sx q[sz][sy][sx] w^(kx sx),
//         kx in [0, M/2]  (real input: half spectrum on the fastest axis)
//   yz    block (kx, patch): FFT along y of the n+1 source rows, then per
//         column ky: FFT along z, multiply by the spectrum, inverse FFT along
//         z, keep the Wp output z's -> Zb[p][zi][kx][ky]
//   out   block (zi, patch): inverse FFT along y for every kx (keep the Wp
//         output y's), then the Hermitian inverse along x (two real lines per
//         complex FFT) -> coarse samples and skeleton planes, times h^2.
#pragma once
#include "common.h"

namespace mlc {

template <typename T, int M>
__global__ void __launch_bounds__(256) conv_xdft_kernel(const double* __restrict__ f, int N, int n, int ppa,
                                                        cplx<T>* __restrict__ X) {
  constexpr int Mh = M / 2 + 1;
  __shared__ T q[SMAX * SMAX];
  __shared__ cplx<T> tw[M];
  const int S = n + 1;
  const int p = blockIdx.y, sz = blockIdx.x;
  const int i0 = p / (ppa * ppa), i1 = (p / ppa) % ppa, i2 = p % ppa;
  const int64_t Np = N + 1;
  const double cz = (sz == 0 || sz == n) ? 0.5 : 1.0;
  const double* fp = f + (int64_t(n) * i0 + sz) * Np * Np + int64_t(n) * i1 * Np + int64_t(n) * i2;
  for (int t = threadIdx.x; t < S * S; t += blockDim.x) {
    int sy = t / S, sx = t % S;
    double c = cz * ((sy == 0 || sy == n) ? 0.5 : 1.0) * ((sx == 0 || sx == n) ? 0.5 : 1.0);
    q[t] = T(c * fp[sy * Np + sx]);
  }
  fill_twiddles(tw, M);
  __syncthreads();
  cplx<T>* out = X + (int64_t(p) * Mh * S + sz) * S;
  for (int o = threadIdx.x; o < Mh * S; o += blockDim.x) {
    int kx = o / S, sy = o % S;
    T ar = 0, ai = 0;
    const T* row = q + sy * S;
    int idx = 0;
    for (int sx = 0; sx < S; ++sx) {
      cplx<T> w = tw[idx];
      ar += row[sx] * w.x;
      ai += row[sx] * w.y;
      idx += kx;
      if (idx >= M) idx -= M;
    }
    out[int64_t(kx) * S * S + sy] = {ar, ai};
  }
}

template <typename T> struct ConvCfg;
template <> struct ConvCfg<float> { static constexpr int CB = 16, NLB = 4, CK = 8; };
template <> struct ConvCfg<double> { static constexpr int CB = 8, NLB = 4, CK = 4; };

template <int n, int NLB> struct SRows { static constexpr int v = ((n + 1 + NLB - 1) / NLB) * NLB; };

template <typename T, int n, int M>
__global__ void __launch_bounds__(256) conv_yz_kernel(const cplx<T>* __restrict__ X, const T* __restrict__ spec,
                                                      cplx<T>* __restrict__ Zb, int Wp, int b, int Wa, int e, int da) {
  constexpr int Mh = M / 2 + 1;
  constexpr int S = n + 1;
  constexpr int CB = ConvCfg<T>::CB, NLB = ConvCfg<T>::NLB;
  constexpr int SR = SRows<n, NLB>::v;
  __shared__ cplx<T> Y[SR * M];
  __shared__ cplx<T> Cb[CB * M];
  __shared__ cplx<T> tw[M];
  const int kx = blockIdx.x, p = blockIdx.y;
  const cplx<T>* xin = X + (int64_t(p) * Mh + kx) * S * S;
  for (int t = threadIdx.x; t < SR * M; t += blockDim.x) {
    int r = t / M, c = t % M;
    Y[t] = (r < S && c < S) ? xin[r * S + c] : cplx<T>{T(0), T(0)};
  }
  fill_twiddles(tw, M);
  __syncthreads();
  // FFT along y of every source row sz
#pragma unroll 1
  for (int rb = 0; rb < SR; rb += NLB) fft_lines<T, M, NLB, 256, 1, false>(Y + rb * M, M, 1, tw);
  const T* sp = spec + int64_t(kx) * Mh * Mh;
  cplx<T>* zout = Zb + (int64_t(p) * Wp * Mh + kx) * M;
#pragma unroll 1
  for (int cb = 0; cb < M; cb += CB) {
    for (int t = threadIdx.x; t < CB * M; t += blockDim.x) {
      int c = t % CB, z = t / CB;
      Cb[c * M + z] = (z < S && cb + c < M) ? Y[z * M + cb + c] : cplx<T>{T(0), T(0)};
    }
    __syncthreads();
    fft_lines<T, M, CB, 256, 1, false>(Cb, M, 1, tw);
    for (int t = threadIdx.x; t < CB * M; t += blockDim.x) {
      int c = t / M, kz = t % M;
      int ky = cb + c;
      if (ky >= M) continue;
      int az = kz <= M / 2 ? kz : M - kz, ay = ky <= M / 2 ? ky : M - ky;
      T g = sp[az * Mh + ay];
      Cb[t] = {Cb[t].x * g, Cb[t].y * g};
    }
    __syncthreads();
    fft_lines<T, M, CB, 256, -1, false>(Cb, M, 1, tw);
    for (int t = threadIdx.x; t < CB * Wp; t += blockDim.x) {
      int c = t % CB, zi = t / CB;
      if (cb + c >= M) continue;
      int z = out_coord(zi, b, Wa, e, da, n);
      int slot = z < 0 ? z + M : z;
      zout[int64_t(zi) * Mh * M + cb + c] = Cb[c * M + slot];
    }
    __syncthreads();
  }
}

struct OutGeom {
  int n, e, da, b, Wa, Wp, Wc, P0, npl;
  double h2;
};

__device__ __forceinline__ int mod_pos(int a, int m) { int r = a % m; return r < 0 ? r + m : r; }

template <typename T, int n, int M>
__global__ void __launch_bounds__(256) conv_out_kernel(const cplx<T>* __restrict__ Zb, T* __restrict__ coarse,
                                                       T* __restrict__ planes, OutGeom g) {
  constexpr int Mh = M / 2 + 1;
  constexpr int CK = ConvCfg<T>::CK;
  constexpr int WPMAX = n + 2 * n + 1 + 2 * 4;  // Wa + 2b with d_alpha <= n, b <= 4
  __shared__ cplx<T> A[Mh * WPMAX];
  __shared__ cplx<T> Cb[CK * M];
  __shared__ cplx<T> tw[M];
  const int zi = blockIdx.x, p = blockIdx.y;
  const int Wp = g.Wp;
  fill_twiddles(tw, M);
  const cplx<T>* zin = Zb + (int64_t(p) * Wp + zi) * Mh * M;
  // inverse FFT along y for every kx; keep the Wp output y's
#pragma unroll 1
  for (int kb = 0; kb < Mh; kb += CK) {
    __syncthreads();
    for (int t = threadIdx.x; t < CK * M; t += blockDim.x) {
      int r = t / M, ky = t % M;
      Cb[t] = (kb + r < Mh) ? zin[int64_t(kb + r) * M + ky] : cplx<T>{T(0), T(0)};
    }
    __syncthreads();
    fft_lines<T, M, CK, 256, -1, false>(Cb, M, 1, tw);
    for (int t = threadIdx.x; t < CK * Wp; t += blockDim.x) {
      int r = t / Wp, yi = t % Wp;
      if (kb + r < Mh) {
        int y = out_coord(yi, g.b, g.Wa, g.e, g.da, n);
        A[(kb + r) * Wp + yi] = Cb[r * M + (y < 0 ? y + M : y)];
      }
    }
  }
  const int z = out_coord(zi, g.b, g.Wa, g.e, g.da, n);
  const bool zin_a = z >= -g.da && z <= n + g.da;
  const bool zc = mod_pos(z, NREF) == 0;
  const bool zpl = zin_a && mod_pos(z, n) == 0;
  const int npl = g.npl, Wa = g.Wa, Wc = g.Wc;
  T* cbase = coarse + int64_t(p) * Wc * Wc * Wc;
  T* pbase = planes + int64_t(p) * 3 * npl * Wa * Wa;
  // Hermitian inverse along x: two real lines (y_j, y_j+1) per complex line
#pragma unroll 1
  for (int yb = 0; yb < Wp; yb += 2 * CK) {
    __syncthreads();
    for (int t = threadIdx.x; t < CK * M; t += blockDim.x) {
      int c = t / M, k = t % M;
      int y1 = yb + 2 * c, y2 = y1 + 1;
      cplx<T> h1 = {T(0), T(0)}, h2 = {T(0), T(0)};
      if (k < Mh) {
        if (y1 < Wp) h1 = A[k * Wp + y1];
        if (y2 < Wp) h2 = A[k * Wp + y2];
      } else {
        if (y1 < Wp) { h1 = A[(M - k) * Wp + y1]; h1.y = -h1.y; }
        if (y2 < Wp) { h2 = A[(M - k) * Wp + y2]; h2.y = -h2.y; }
      }
      if (k == 0 || k == M / 2) { h1.y = T(0); h2.y = T(0); }   // real DC / Nyquist
      Cb[t] = {h1.x - h2.y, h1.y + h2.x};   // h1 + i h2
    }
    __syncthreads();
    fft_lines<T, M, CK, 256, -1, false>(Cb, M, 1, tw);
    for (int t = threadIdx.x; t < 2 * CK * Wp; t += blockDim.x) {
      int yl = t / Wp, xi = t % Wp;
      int yi = yb + yl;
      if (yi >= Wp) continue;
      int y = out_coord(yi, g.b, g.Wa, g.e, g.da, n);
      int x = out_coord(xi, g.b, g.Wa, g.e, g.da, n);
      cplx<T> zv = Cb[(yl >> 1) * M + (x < 0 ? x + M : x)];
      T val = T(((yl & 1) ? zv.y : zv.x) * g.h2);
      const bool yin_a = y >= -g.da && y <= n + g.da;
      const bool xin_a = x >= -g.da && x <= n + g.da;
      if (zc && mod_pos(y, NREF) == 0 && mod_pos(x, NREF) == 0)
        cbase[(int64_t((z + g.e) / NREF) * Wc + (y + g.e) / NREF) * Wc + (x + g.e) / NREF] = val;
      if (zpl && yin_a && xin_a)
        pbase[((int64_t(0) * npl + (z - g.P0) / n) * Wa + (y + g.da)) * Wa + (x + g.da)] = val;
      if (zin_a && yin_a && xin_a) {
        if (mod_pos(y, n) == 0)
          pbase[((int64_t(1) * npl + (y - g.P0) / n) * Wa + (z + g.da)) * Wa + (x + g.da)] = val;
        if (mod_pos(x, n) == 0)
          pbase[((int64_t(2) * npl + (x - g.P0) / n) * Wa + (z + g.da)) * Wa + (y + g.da)] = val;
      }
    }
  }
}

}  // namespace mlc
