// Setup kernels: the DGF table (appendix A.1), batched axis FFTs of cubic
// arrays, DGF spectra for Hockney's method (appendix A.2) and the far-field
// tables of the Legendre modes (sec. 4.1: built once, kept for every solve).
#pragma once
#include "common.h"

namespace mlc {

// ---------------------------------------------------------------- DGF ----
// Right-hand side of the residual-correction Dirichlet problem on the
// interior [-L+1, L-1]^3 of [-L, L]^3: delta_0 - (L w), w = -1/(4 pi |g|) on
// the layer |g|_inf = L.  Array rhs[m0][m1][m2], m = g + L - 1, Nd = 2L-1.
__global__ void dgf_rhs_kernel(double* rhs, int L, Stencil st) {
  const int Nd = 2 * L - 1;
  int64_t idx = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (idx >= cube(Nd)) return;
  int g2 = int(idx % Nd) - (L - 1);
  int g1 = int((idx / Nd) % Nd) - (L - 1);
  int g0 = int(idx / (int64_t(Nd) * Nd)) - (L - 1);
  double v = (g0 == 0 && g1 == 0 && g2 == 0) ? 1.0 : 0.0;
  int amax = max(abs(g0), max(abs(g1), abs(g2)));
  if (amax == L - 1) {
    double s = 0.0;
    for (int s0 = -1; s0 <= 1; ++s0)
      for (int s1 = -1; s1 <= 1; ++s1)
        for (int s2 = -1; s2 <= 1; ++s2) {
          int h0 = g0 + s0, h1 = g1 + s1, h2 = g2 + s2;
          if (max(abs(h0), max(abs(h1), abs(h2))) != L) continue;
          double r = sqrt(double(h0) * h0 + double(h1) * h1 + double(h2) * h2);
          int nz = (s0 != 0) + (s1 != 0) + (s2 != 0);
          s += st.b[nz] * (-1.0 / (4.0 * M_PI * r));
        }
    v -= s;
  }
  rhs[idx] = v;
}

// Unnormalised DST-I along one axis of the Nd^3 real array (in place):
//   S_k = sum_{m=1..Nd} x_m sin(pi k m / (Nd+1)),  k = 1..Nd.
// Two real lines share one complex FFT of length MF = 2(Nd+1) of their odd
// extensions y = [0, x, 0, -reverse(x)]: with z = y1 + i y2, Z[k] =
// 2 S2_k - 2i S1_k.
template <int MF, int NLC>
__global__ void __launch_bounds__(256) dst1_axis_kernel(double* data, int axis) {
  constexpr int Nd = MF / 2 - 1;
  __shared__ cplx<double> buf[NLC * MF];
  __shared__ cplx<double> tw[MF];
  fill_twiddles(tw, MF);
  const int64_t es = axis == 2 ? 1 : (axis == 1 ? Nd : int64_t(Nd) * Nd);
  // lines are indexed by (u, v) over the other two axes, v the faster one
  const int64_t vs = axis == 2 ? Nd : 1;
  const int64_t us = axis == 0 ? Nd : int64_t(Nd) * Nd;
  const int nreal = 2 * NLC;
  const int v0 = blockIdx.x * nreal;
  const int u = blockIdx.y;
  // zero + load: real line r goes to complex line r/2, component r%2
  for (int t = threadIdx.x; t < NLC * MF; t += blockDim.x) buf[t] = {0.0, 0.0};
  __syncthreads();
  for (int t = threadIdx.x; t < nreal * Nd; t += blockDim.x) {
    int r, m;
    if (axis == 2) { r = t / Nd; m = t % Nd; } else { r = t % nreal; m = t / nreal; }
    int v = v0 + r;
    if (v >= Nd) continue;
    double x = data[u * us + v * vs + m * es];
    cplx<double>* line = buf + (r / 2) * MF;
    if (r % 2 == 0) { line[m + 1].x = x; line[MF - 1 - m].x = -x; }
    else { line[m + 1].y = x; line[MF - 1 - m].y = -x; }
  }
  __syncthreads();
  fft_lines<double, MF, NLC, 256, 1, false>(buf, MF, 1, tw);
  for (int t = threadIdx.x; t < nreal * Nd; t += blockDim.x) {
    int r, m;
    if (axis == 2) { r = t / Nd; m = t % Nd; } else { r = t % nreal; m = t / nreal; }
    int v = v0 + r;
    if (v >= Nd) continue;
    cplx<double> z = buf[(r / 2) * MF + m + 1];
    data[u * us + v * vs + m * es] = (r % 2 == 0) ? -0.5 * z.y : 0.5 * z.x;
  }
}

// Divide by the stencil symbol on the DST-I modes (and fold the inverse
// normalisation 1/L^3 of the second transform).
__global__ void dgf_divide_kernel(double* data, int L, Stencil st) {
  const int Nd = 2 * L - 1;
  int64_t idx = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (idx >= cube(Nd)) return;
  int k2 = int(idx % Nd) + 1, k1 = int((idx / Nd) % Nd) + 1, k0 = int(idx / (int64_t(Nd) * Nd)) + 1;
  double c0 = cospi(double(k0) / (2.0 * L)), c1 = cospi(double(k1) / (2.0 * L)), c2 = cospi(double(k2) / (2.0 * L));
  double lam = st.b[0] + 2.0 * st.b[1] * (c0 + c1 + c2) + 4.0 * st.b[2] * (c0 * c1 + c0 * c2 + c1 * c2) +
               8.0 * st.b[3] * c0 * c1 * c2;
  double inv = 1.0 / (double(L) * L * L);
  data[idx] = data[idx] / lam * inv;
}

// Restrict the interior solution to [-Z, Z]^3.
__global__ void dgf_restrict_kernel(const double* u, double* table, int L, int Z) {
  const int Nd = 2 * L - 1, W = 2 * Z + 1;
  int64_t idx = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (idx >= cube(W)) return;
  int a2 = int(idx % W), a1 = int((idx / W) % W), a0 = int(idx / (int64_t(W) * W));
  int off = L - 1 - Z;
  table[idx] = u[(int64_t(a0 + off) * Nd + (a1 + off)) * Nd + (a2 + off)];
}

// ------------------------------------------------- generic axis FFT ----
// Complex M^3 array, transform along `axis`.  NL lines per block; lines
// adjacent along the fastest other axis; blockIdx.z: array of a batch of
// consecutive M^3 arrays.  Only the lines (u, v) with u = uoff + blockIdx.y
// and v = voff + j, j < vcount (both taken mod M) are transformed: callers
// skip lines known to be zero on input or not needed on output.
template <typename T, int M, int NL, int DIR>
__global__ void __launch_bounds__(256) fft_axis_kernel(cplx<T>* data, int axis, int uoff, int voff, int vcount) {
  __shared__ cplx<T> buf[NL * M];
  __shared__ cplx<T> tw[M];
  fill_twiddles(tw, M);
  data += int64_t(blockIdx.z) * M * M * M;
  const int64_t es = axis == 2 ? 1 : (axis == 1 ? M : int64_t(M) * M);
  const int64_t vs = axis == 2 ? M : 1;
  const int64_t us = axis == 0 ? M : int64_t(M) * M;
  const int j0 = blockIdx.x * NL;
  const int u = (uoff + int(blockIdx.y)) % M;
  for (int t = threadIdx.x; t < NL * M; t += blockDim.x) {
    int r, m;
    if (axis == 2) { r = t / M; m = t % M; } else { r = t % NL; m = t / NL; }
    const int v = (voff + j0 + r) % M;
    buf[r * M + m] = j0 + r < vcount ? data[u * us + v * vs + m * es] : cplx<T>{T(0), T(0)};
  }
  __syncthreads();
  fft_lines<T, M, NL, 256, DIR, false>(buf, M, 1, tw);
  for (int t = threadIdx.x; t < NL * M; t += blockDim.x) {
    int r, m;
    if (axis == 2) { r = t / M; m = t % M; } else { r = t % NL; m = t / NL; }
    const int v = (voff + j0 + r) % M;
    if (j0 + r < vcount) data[u * us + v * vs + m * es] = buf[r * M + m];
  }
}

// One sweep along axis 0 of a batch of complex M^3 arrays: forward
// transform, times a real-even spectrum stored as its octant [Mh]^3 (layout
// k0, k1, k2), inverse transform.  The last forward pass, the product and the
// first inverse pass of a torus convolution, with the same arithmetic as
// fft_axis_kernel, mul_real_even_kernel, fft_axis_kernel in turn.  Block:
// NL lines (k1 = blockIdx.y, consecutive k2); blockIdx.z: array.
template <typename T, int M, int NL>
__global__ void __launch_bounds__(256) fft_axis0_conv_kernel(cplx<T>* data, const double* oct) {
  __shared__ cplx<T> buf[NL * M];
  __shared__ cplx<T> tw[M];
  constexpr int Mh = M / 2 + 1;
  fill_twiddles(tw, M);
  data += int64_t(blockIdx.z) * M * M * M;
  const int64_t es = int64_t(M) * M;
  const int j0 = blockIdx.x * NL, u = blockIdx.y;
  for (int t = threadIdx.x; t < NL * M; t += blockDim.x) {
    const int r = t % NL, m = t / NL, v = j0 + r;
    buf[r * M + m] = v < M ? data[int64_t(u) * M + v + m * es] : cplx<T>{T(0), T(0)};
  }
  __syncthreads();
  fft_lines<T, M, NL, 256, 1, false>(buf, M, 1, tw);
  const int a1 = min(u, M - u);
  for (int t = threadIdx.x; t < NL * M; t += blockDim.x) {
    const int r = t % NL, m = t / NL, v = j0 + r;
    if (v >= M) continue;
    const double g = oct[(int64_t(min(m, M - m)) * Mh + a1) * Mh + min(v, M - v)];
    buf[r * M + m] = {buf[r * M + m].x * g, buf[r * M + m].y * g};
  }
  __syncthreads();
  fft_lines<T, M, NL, 256, -1, false>(buf, M, 1, tw);
  for (int t = threadIdx.x; t < NL * M; t += blockDim.x) {
    const int r = t % NL, m = t / NL, v = j0 + r;
    if (v < M) data[int64_t(u) * M + v + m * es] = buf[r * M + m];
  }
}

// Periodised DGF on an M^3 torus, "symmetric fill": slot k holds G1 at the
// signed offset k~ in (-M/2, M/2] (zero where the table ends).  The kernel
// is real and even, so its DFT is real and even.
__global__ void fill_periodic_dgf_kernel(cplx<double>* out, const double* G1, int Z, int M) {
  int64_t idx = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (idx >= cube(M)) return;
  int k2 = int(idx % M), k1 = int((idx / M) % M), k0 = int(idx / (int64_t(M) * M));
  auto sgn = [M](int k) { return k <= M / 2 ? k : k - M; };
  int s0 = sgn(k0), s1 = sgn(k1), s2 = sgn(k2);
  double v = 0.0;
  if (abs(s0) <= Z && abs(s1) <= Z && abs(s2) <= Z) {
    const int W = 2 * Z + 1;
    v = G1[(int64_t(s0 + Z) * W + (s1 + Z)) * W + (s2 + Z)];
  }
  out[idx] = {v, 0.0};
}

// Real octant [0, M/2]^3 of a real-even spectrum, times `scale`, in layout
// order (a, b, c) -> spec[(a * Mh + b) * Mh + c] with (a, b, c) a
// permutation of the wavenumber axes given by p0 p1 p2.
template <typename T>
__global__ void spectrum_octant_kernel(const cplx<double>* full, T* spec, int M, double scale, int p0, int p1,
                                       int p2) {
  const int Mh = M / 2 + 1;
  int64_t idx = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (idx >= cube(Mh)) return;
  int c = int(idx % Mh), b = int((idx / Mh) % Mh), a = int(idx / (int64_t(Mh) * Mh));
  int k[3];
  k[p0] = a; k[p1] = b; k[p2] = c;
  spec[idx] = T(full[(int64_t(k[0]) * M + k[1]) * M + k[2]].x * scale);
}

// ------------------------------------------------ far-field tables ----
struct ModeList { int K; int p[KMAX][3]; };

// chi_0 Q_p on the patch nodes [0, n]^3 placed at slots [0, n]^3 of a zeroed
// M^3 torus.  Q_p = R^{-3/2} prod_d qhat(p_d, (s_d - n/2)/(n/2)).
__global__ void fill_mode_source_kernel(cplx<double>* out, int M, int n, int p0, int p1, int p2, double rscale) {
  int64_t idx = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  int S = n + 1;
  if (idx >= cube(S)) return;
  int s2 = int(idx % S), s1 = int((idx / S) % S), s0 = int(idx / (int64_t(S) * S));
  auto chi = [n](int s) { return (s == 0 || s == n) ? 0.5 : 1.0; };
  double h = n * 0.5;
  double v = rscale * chi(s0) * chi(s1) * chi(s2) * qhat(p0, (s0 - h) / h) * qhat(p1, (s1 - h) / h) *
             qhat(p2, (s2 - h) / h);
  out[(int64_t(s0) * M + s1) * M + s2] = {v, 0.0};
}

// Multiply a complex M^3 array by a real-even spectrum stored as its octant
// [Mh]^3 (layout k0, k1, k2).
// blockIdx.y: array of a batch of consecutive M^3 arrays.
__global__ void mul_real_even_kernel(cplx<double>* data, const double* oct, int M) {
  int64_t idx = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (idx >= cube(M)) return;
  data += int64_t(blockIdx.y) * cube(M);
  const int Mh = M / 2 + 1;
  int k2 = int(idx % M), k1 = int((idx / M) % M), k0 = int(idx / (int64_t(M) * M));
  k0 = min(k0, M - k0); k1 = min(k1, M - k1); k2 = min(k2, M - k2);
  double g = oct[(int64_t(k0) * Mh + k1) * Mh + k2];
  data[idx] = {data[idx].x * g, data[idx].y * g};
}

// Extract Phi_p = scale * Re(torus[x mod M]) at (a) the coarse nodes of the
// table box [-eb, n+eb]^3 and (b) the skeleton planes of Omega_beta(0)
// (normal d, planes P0 + j n, in-plane [-db, n+db]).
__global__ void extract_mode_kernel(const cplx<double>* torus, int M, double scale, int n, int eb, int db,
                                    int P0b, int nplb, double* coarse, double* planes) {
  const int Wtc = (n + 2 * eb) / NREF + 1, Wb = n + 2 * db + 1;
  int64_t nc = cube(Wtc), npl = int64_t(3) * nplb * Wb * Wb;
  int64_t idx = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  auto at = [&](int x0, int x1, int x2) {
    int m0 = ((x0 % M) + M) % M, m1 = ((x1 % M) + M) % M, m2 = ((x2 % M) + M) % M;
    return scale * torus[(int64_t(m0) * M + m1) * M + m2].x;
  };
  if (idx < nc) {
    int c2 = int(idx % Wtc), c1 = int((idx / Wtc) % Wtc), c0 = int(idx / (int64_t(Wtc) * Wtc));
    coarse[idx] = at(-eb + NREF * c0, -eb + NREF * c1, -eb + NREF * c2);
  } else if (idx < nc + npl) {
    int64_t r = idx - nc;
    int v = int(r % Wb), u = int((r / Wb) % Wb), j = int((r / (int64_t(Wb) * Wb)) % nplb);
    int d = int(r / (int64_t(Wb) * Wb * nplb));
    int x[3];
    x[d] = P0b + j * n;
    int a0 = d == 0 ? 1 : 0, a1 = d == 2 ? 1 : 2;
    x[a0] = -db + u;
    x[a1] = -db + v;
    planes[r] = at(x[0], x[1], x[2]);
  }
}

// T_p = Delta^H Phi_p on C(Omega_beta(0)) = [-db/4, (n+db)/4]^3 from the
// coarse samples, set to zero on C(Omega_alpha(0)) (that part of a patch's
// coarse charge comes from its full local field).
__global__ void annulus_coarse_table_kernel(const double* coarse, double* T, int n, int eb, int db, int da,
                                            Stencil st, double invH2, int K, int k) {
  const int Wtc = (n + 2 * eb) / NREF + 1, Wbc = (n + 2 * db) / NREF + 1;
  int64_t idx = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (idx >= cube(Wbc)) return;
  int c2 = int(idx % Wbc), c1 = int((idx / Wbc) % Wbc), c0 = int(idx / (int64_t(Wbc) * Wbc));
  int g0 = -db / NREF + c0, g1 = -db / NREF + c1, g2 = -db / NREF + c2;   // coarse coords rel. patch
  int alo = -da / NREF, ahi = (n + da) / NREF;
  bool inner = g0 >= alo && g0 <= ahi && g1 >= alo && g1 <= ahi && g2 >= alo && g2 <= ahi;
  double s = 0.0;
  if (!inner) {
    int o = eb / NREF;   // coarse index of coord 0 in the sample array
    for (int s0 = -1; s0 <= 1; ++s0)
      for (int s1 = -1; s1 <= 1; ++s1)
        for (int s2 = -1; s2 <= 1; ++s2) {
          int nz = (s0 != 0) + (s1 != 0) + (s2 != 0);
          s += st.b[nz] * coarse[(int64_t(g0 + s0 + o) * Wtc + (g1 + s1 + o)) * Wtc + (g2 + s2 + o)];
        }
    s *= invH2;
  }
  T[idx * K + k] = s;
}

// 1-D Lagrange weights on the 2b+2 nodes -b..b+1 at theta (b <= 4).
__host__ __device__ inline void lagrange_weights(int b, double th, double* w) {
  for (int k = -b; k <= b + 1; ++k) {
    double v = 1.0;
    for (int m = -b; m <= b + 1; ++m)
      if (m != k) v *= (th - m) / double(k - m);
    w[k + b] = v;
  }
}

// Coplanar interpolation of coarse samples c (2-D, in-plane coarse index
// origin cofs: coarse coordinate U sits at index U + cofs, row length Wc)
// to the fine in-plane point (u, v).  theta = 0 on an axis takes the single
// node (exactly, no arithmetic on that axis).
__device__ inline double interp2(const double* c, int Wc, int cofs, int u, int v, int b) {
  int U0 = u >= 0 ? u / NREF : -((-u + NREF - 1) / NREF);
  int V0 = v >= 0 ? v / NREF : -((-v + NREF - 1) / NREF);
  int tu = u - NREF * U0, tv = v - NREF * V0;
  double wu[10], wv[10];
  int ku0 = 0, ku1 = 0, kv0 = 0, kv1 = 0;
  if (tu) { lagrange_weights(b, tu / double(NREF), wu); ku0 = -b; ku1 = b + 1; } else { wu[b] = 1.0; }
  if (tv) { lagrange_weights(b, tv / double(NREF), wv); kv0 = -b; kv1 = b + 1; } else { wv[b] = 1.0; }
  double s = 0.0;
  for (int ku = ku0; ku <= ku1; ++ku) {
    double r = 0.0;
    const double* row = c + int64_t(U0 + ku + cofs) * Wc;
    for (int kv = kv0; kv <= kv1; ++kv) r += wv[kv + b] * row[V0 + kv + cofs];
    s += wu[ku + b] * r;
  }
  return s;
}

// D_p = Phi_p - I(Phi_p) on the skeleton planes of Omega_beta(0), zero
// where the node lies in Omega_alpha(0).
__global__ void annulus_plane_table_kernel(const double* planes, const double* coarse, double* D, int n, int eb,
                                           int db, int da, int P0b, int nplb, int b, int K, int k) {
  const int Wtc = (n + 2 * eb) / NREF + 1, Wb = n + 2 * db + 1;
  int64_t per = int64_t(3) * nplb * Wb * Wb;
  int64_t idx = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (idx >= per) return;
  int v = int(idx % Wb), u = int((idx / Wb) % Wb), j = int((idx / (int64_t(Wb) * Wb)) % nplb);
  int d = int(idx / (int64_t(Wb) * Wb * nplb));
  int P = P0b + j * n;
  int xu = -db + u, xv = -db + v;
  bool inner = P >= -da && P <= n + da && xu >= -da && xu <= n + da && xv >= -da && xv <= n + da;
  double out = 0.0;
  if (!inner) {
    // coarse samples of the plane x_d = P: index along d is (P + eb)/4
    int cd = (P + eb) / NREF;
    // gather the 2-D coarse plane on the fly through a strided view
    const int a0 = d == 0 ? 1 : 0, a1 = d == 2 ? 1 : 2;
    (void)a0; (void)a1;
    int U0 = xu >= 0 ? xu / NREF : -((-xu + NREF - 1) / NREF);
    int V0 = xv >= 0 ? xv / NREF : -((-xv + NREF - 1) / NREF);
    int tu = xu - NREF * U0, tv = xv - NREF * V0;
    double wu[10], wv[10];
    int ku0 = 0, ku1 = 0, kv0 = 0, kv1 = 0;
    if (tu) { lagrange_weights(b, tu / double(NREF), wu); ku0 = -b; ku1 = b + 1; } else { wu[b] = 1.0; }
    if (tv) { lagrange_weights(b, tv / double(NREF), wv); kv0 = -b; kv1 = b + 1; } else { wv[b] = 1.0; }
    int o = eb / NREF;
    double s = 0.0;
    for (int ku = ku0; ku <= ku1; ++ku)
      for (int kv = kv0; kv <= kv1; ++kv) {
        int c[3];
        c[d] = cd;
        c[d == 0 ? 1 : 0] = U0 + ku + o;
        c[d == 2 ? 1 : 2] = V0 + kv + o;
        s += wu[ku + b] * wv[kv + b] * coarse[(int64_t(c[0]) * Wtc + c[1]) * Wtc + c[2]];
      }
    out = planes[idx] - s;
  }
  D[idx * K + k] = out;
}

}  // namespace mlc
