// Per-solve kernels of the two-level MLC other than the local convolutions,
// all in float64: Legendre moments, the coarse right-hand side, the coarse
// Hockney solve's torus fill/extract, the boundary values on the patch
// skeleton, and the patch Dirichlet solves with the final correction.
#pragma once
#include "common.h"
#include "setup_kernels.h"

namespace mlc {

// ------------------------------------------------------------ moments ----
// c_{i,p} = R^{3/2} sum_j W_j f[j] qhat_p(t_j) / mu_p over the (n+1)^3 nodes of
// the closed patch, W = tensor composite Boole weights on [-1, 1], and mu_p
// the diagonal of the Boole Gram matrix (sec. 3 projection; sec. 4.1 step 1
// quadrature).  For P <= 4 the Gram matrix is diagonal.
__device__ inline double boole_w(int j, int n) {
  double base = 4.0 / (45.0 * n);   // (2 delta / 45), delta = 2/n
  if (j == 0 || j == n) return 7.0 * base;
  int r = j & 3;
  return (r == 0 ? 14.0 : (r == 2 ? 12.0 : 32.0)) * base;
}

__global__ void __launch_bounds__(256) moments_kernel(const double* __restrict__ f, int N, int n, int ppa,
                                                      ModeList modes, double R15, double* __restrict__ out) {
  __shared__ double B[4][SMAXN];
  __shared__ double mu1[4];
  __shared__ double red[256];
  const int S = n + 1;
  const int p = blockIdx.x;
  const int i0 = p / (ppa * ppa), i1 = (p / ppa) % ppa, i2 = p % ppa;
  for (int t = threadIdx.x; t < 4 * S; t += blockDim.x) {
    int a = t / S, j = t % S;
    double tt = (j - 0.5 * n) / (0.5 * n);
    B[a][j] = boole_w(j, n) * qhat(a, tt);
  }
  __syncthreads();
  if (threadIdx.x < 4) {
    int a = threadIdx.x;
    double s = 0.0;
    for (int j = 0; j < S; ++j) {
      double tt = (j - 0.5 * n) / (0.5 * n);
      s += B[a][j] * qhat(a, tt);
    }
    mu1[a] = s;
  }
  const int64_t Np = N + 1;
  const double* fp = f + (int64_t(n) * i0) * Np * Np + int64_t(n) * i1 * Np + int64_t(n) * i2;
  double acc[KMAX];
  for (int k = 0; k < KMAX; ++k) acc[k] = 0.0;
  for (int t = threadIdx.x; t < S * S * S; t += blockDim.x) {
    int j2 = t % S, j1 = (t / S) % S, j0 = t / (S * S);
    double v = fp[(j0 * Np + j1) * Np + j2];
#pragma unroll
    for (int k = 0; k < KMAX; ++k)
      if (k < modes.K) acc[k] += v * B[modes.p[k][0]][j0] * B[modes.p[k][1]][j1] * B[modes.p[k][2]][j2];
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < KMAX; ++k) {
    if (k >= modes.K) break;
    red[threadIdx.x] = acc[k];
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
      if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
      __syncthreads();
    }
    if (threadIdx.x == 0) {
      double mu = mu1[modes.p[k][0]] * mu1[modes.p[k][1]] * mu1[modes.p[k][2]];
      out[int64_t(p) * modes.K + k] = R15 * red[0] / mu;
    }
    __syncthreads();
  }
}

// ------------------------------------------------------- coarse rhs ----
struct CoarseGeom {
  int n, ppa, K, da, db, e, Wc, S_lo, Ns, Wbc;
  double invH2;
};

// Inner part of F^H: F[c] = sum over patches i with c in C(Omega_alpha(i)) of
// Delta^H of phi_i's coarse samples (sec. 4.1 eq. FDLD, first case), patches
// visited in a fixed order.
template <typename T>
__global__ void __launch_bounds__(256) coarse_rhs_kernel(const T* __restrict__ cs, Stencil st, CoarseGeom g,
                                                         double* __restrict__ F) {
  int64_t idx = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (idx >= cube(g.Ns)) return;
  int c[3];
  c[2] = g.S_lo + int(idx % g.Ns);
  c[1] = g.S_lo + int((idx / g.Ns) % g.Ns);
  c[0] = g.S_lo + int(idx / (int64_t(g.Ns) * g.Ns));
  const int n = g.n, q = n / NREF;
  // patches whose C(Omega_alpha) contains c: n i - da <= 4c <= n i + n + da
  int lo[3], hi[3];
  for (int d = 0; d < 3; ++d) {
    int a = NREF * c[d] - n - g.da;
    lo[d] = max(a >= 0 ? (a + n - 1) / n : -((-a) / n), 0);
    int bnd = NREF * c[d] + g.da;
    hi[d] = min(bnd >= 0 ? bnd / n : -((-bnd + n - 1) / n), g.ppa - 1);
  }
  const int Wc = g.Wc, o = g.e / NREF;
  double s = 0.0;
  for (int a0 = lo[0]; a0 <= hi[0]; ++a0)
    for (int a1 = lo[1]; a1 <= hi[1]; ++a1)
      for (int a2 = lo[2]; a2 <= hi[2]; ++a2) {
        int r0 = c[0] - q * a0 + o, r1 = c[1] - q * a1 + o, r2 = c[2] - q * a2 + o;
        int pidx = (a0 * g.ppa + a1) * g.ppa + a2;
        const T* base = cs + int64_t(pidx) * Wc * Wc * Wc;
        double l = 0.0;
        for (int s0 = -1; s0 <= 1; ++s0)
          for (int s1 = -1; s1 <= 1; ++s1)
            for (int s2 = -1; s2 <= 1; ++s2) {
              int nz = (s0 != 0) + (s1 != 0) + (s2 != 0);
              l += st.b[nz] * double(base[(int64_t(r0 + s0) * Wc + (r1 + s1)) * Wc + (r2 + s2)]);
            }
        s += l * g.invH2;
      }
  F[idx] = s;
}

constexpr int MAXPATCH = 512;   // patches whose moments fit the LDS of one block

// Annulus part of F^H (sec. 4.1 eq. FDLD, second case), added to F:
//   F[c] += sum_i sum_p c_{i,p} T_p[c - n i / 4],  T zero on C(Omega_alpha(0)).
// Write c = q k + rho (q = n/4, rho in [0, q)^3); then c - n i/4 =
// q (k - i) + rho, so for one rho the sum is a convolution over the patch
// lattice.  Block = one rho; the block's threads take the lattice points k;
// all moments sit in LDS; the table values of one lattice offset are read
// once and reused by every k.
__global__ void __launch_bounds__(256) coarse_annulus_kernel(const double* __restrict__ mom,
                                                             const double* __restrict__ Tt, CoarseGeom g,
                                                             double* __restrict__ F) {
  __shared__ double cm[MAXPATCH * KMAX];
  const int n = g.n, q = n / NREF, K = g.K, ppa = g.ppa;
  const int npatch = ppa * ppa * ppa;
  const bool in_lds = npatch <= MAXPATCH;
  if (in_lds)
    for (int t = threadIdx.x; t < npatch * K; t += blockDim.x) cm[t] = mom[t];
  const double* cmp = in_lds ? cm : mom;
  const int rb = blockIdx.x;
  const int rho[3] = {rb / (q * q), (rb / q) % q, rb % q};
  // lattice points k with c = q k + rho inside the support box
  int klo[3], kn[3], dlo[3], dhi[3];
  const int S_hi = g.S_lo + g.Ns - 1;
  const int blo = -g.db / NREF, bhi = (n + g.db) / NREF;   // C(Omega_beta(0))
  for (int d = 0; d < 3; ++d) {
    int a = g.S_lo - rho[d];
    klo[d] = a >= 0 ? (a + q - 1) / q : -((-a) / q);
    int bnd = S_hi - rho[d];
    int khi = bnd >= 0 ? bnd / q : -((-bnd + q - 1) / q);
    kn[d] = khi - klo[d] + 1;
    // lattice offsets D = k - i with q D + rho inside C(Omega_beta(0))
    int x = blo - rho[d];
    dlo[d] = x >= 0 ? (x + q - 1) / q : -((-x) / q);
    int y = bhi - rho[d];
    dhi[d] = y >= 0 ? y / q : -((-y + q - 1) / q);
  }
  __syncthreads();
  constexpr int PER = 16;
  const int nk = kn[0] * kn[1] * kn[2];
  const int ob = g.db / NREF, Wbc = g.Wbc;
  for (int kbase = 0; kbase < nk; kbase += PER * 256) {
  double acc[PER];
#pragma unroll
  for (int t = 0; t < PER; ++t) acc[t] = 0.0;
  for (int D0 = dlo[0]; D0 <= dhi[0]; ++D0)
    for (int D1 = dlo[1]; D1 <= dhi[1]; ++D1)
      for (int D2 = dlo[2]; D2 <= dhi[2]; ++D2) {
        const double* tv = Tt + ((int64_t(q * D0 + rho[0] + ob) * Wbc + (q * D1 + rho[1] + ob)) * Wbc +
                                 (q * D2 + rho[2] + ob)) * K;
        double tr[KMAX];
#pragma unroll
        for (int p = 0; p < KMAX; ++p) tr[p] = p < K ? tv[p] : 0.0;
#pragma unroll
        for (int t = 0; t < PER; ++t) {
          int kk = kbase + threadIdx.x + t * 256;
          if (kk >= nk) break;
          int i0 = klo[0] + kk / (kn[1] * kn[2]) - D0;
          int i1 = klo[1] + (kk / kn[2]) % kn[1] - D1;
          int i2 = klo[2] + kk % kn[2] - D2;
          if (i0 < 0 || i0 >= ppa || i1 < 0 || i1 >= ppa || i2 < 0 || i2 >= ppa) continue;
          const double* mv = cmp + ((i0 * ppa + i1) * ppa + i2) * K;
          double l = 0.0;
#pragma unroll
          for (int p = 0; p < KMAX; ++p)
            if (p < K) l += tr[p] * mv[p];
          acc[t] += l;
        }
      }
#pragma unroll
  for (int t = 0; t < PER; ++t) {
    int kk = kbase + threadIdx.x + t * 256;
    if (kk >= nk) break;
    int c0 = q * (klo[0] + kk / (kn[1] * kn[2])) + rho[0];
    int c1 = q * (klo[1] + (kk / kn[2]) % kn[1]) + rho[1];
    int c2 = q * (klo[2] + kk % kn[2]) + rho[2];
    F[(int64_t(c0 - g.S_lo) * g.Ns + (c1 - g.S_lo)) * g.Ns + (c2 - g.S_lo)] += acc[t];
  }
  }
}

// Coarse Hockney solve: F^H on slots [0, Ns)^3 of a zeroed Mc^3 torus.
__global__ void coarse_fill_kernel(const double* __restrict__ F, cplx<double>* __restrict__ tor, int Ns, int Mc) {
  int64_t idx = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (idx >= cube(Mc)) return;
  int k2 = int(idx % Mc), k1 = int((idx / Mc) % Mc), k0 = int(idx / (int64_t(Mc) * Mc));
  double v = (k0 < Ns && k1 < Ns && k2 < Ns) ? F[(int64_t(k0) * Ns + k1) * Ns + k2] : 0.0;
  tor[idx] = {v, 0.0};
}

// phi^H[c] = scale * Re(torus[(c - S_lo) mod Mc]) for c in [O_lo, O_lo+No)^3.
__global__ void coarse_extract_kernel(const cplx<double>* __restrict__ tor, double* __restrict__ phiH, int Mc,
                                      int S_lo, int O_lo, int No, double scale) {
  int64_t idx = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (idx >= cube(No)) return;
  int c2 = int(idx % No), c1 = int((idx / No) % No), c0 = int(idx / (int64_t(No) * No));
  auto slot = [&](int c) { int s = (O_lo + c - S_lo) % Mc; return s < 0 ? s + Mc : s; };
  phiH[idx] = scale * tor[(int64_t(slot(c0)) * Mc + slot(c1)) * Mc + slot(c2)].x;
}

// ---------------------------------------------- local plane corrections ----
// Lagrange weights of the coplanar interpolation for the four fine offsets
// t = x - 4 floor(x/4) within a coarse cell: w[t][k+b], k = -b..b+1
// (t = 0: the single weight 1 at k = 0).
struct LagW { double w[4][10]; };

inline LagW make_lagw(int b) {
  LagW L{};
  for (int t = 0; t < 4; ++t) {
    if (t == 0) { L.w[0][b] = 1.0; continue; }
    lagrange_weights(b, t / double(NREF), L.w[t]);
  }
  return L;
}

__device__ __forceinline__ int floor4(int x) { return x >= 0 ? x / NREF : -((-x + NREF - 1) / NREF); }

constexpr int WCMAX = 40, WAMAX = 97;

struct PlaneGeom { int n, e, da, Wa, Wc, P0, npl, b; };

// delta_i = phi_i - I(phi_i) on phi_i's skeleton planes inside Omega_alpha,
// in place.  Block (plane, patch): the plane's coarse samples go to LDS, are
// interpolated along the faster in-plane axis row by row, then along the
// slower one.
template <typename T>
__global__ void __launch_bounds__(256) plane_delta_kernel(T* __restrict__ planes, const T* __restrict__ cs,
                                                          PlaneGeom g, LagW lw) {
  __shared__ double C[WCMAX * WCMAX];
  __shared__ double R[WCMAX * WAMAX];
  const int pl = blockIdx.x, p = blockIdx.y;
  const int d = pl / g.npl, j = pl % g.npl;
  const int n = g.n, Wc = g.Wc, Wa = g.Wa, b = g.b, o = g.e / NREF;
  const int cd = (g.P0 + j * n + g.e) / NREF;
  const T* cb = cs + int64_t(p) * Wc * Wc * Wc;
  for (int t = threadIdx.x; t < Wc * Wc; t += blockDim.x) {
    int cu = t / Wc, cv = t % Wc;
    int c[3];
    c[d] = cd;
    c[d == 0 ? 1 : 0] = cu;
    c[d == 2 ? 1 : 2] = cv;
    C[t] = double(cb[(int64_t(c[0]) * Wc + c[1]) * Wc + c[2]]);
  }
  __syncthreads();
  for (int t = threadIdx.x; t < Wc * Wa; t += blockDim.x) {
    int cu = t / Wa, v = t % Wa;
    int xv = -g.da + v, V0 = floor4(xv), tv = xv - NREF * V0;
    const double* row = C + cu * Wc + V0 + o;
    double s;
    if (tv == 0) {
      s = row[0];
    } else {
      s = 0.0;
      for (int k = -b; k <= b + 1; ++k) s += lw.w[tv][k + b] * row[k];
    }
    R[cu * Wa + v] = s;
  }
  __syncthreads();
  T* out = planes + ((int64_t(p) * 3 + d) * g.npl + j) * Wa * Wa;
  for (int t = threadIdx.x; t < Wa * Wa; t += blockDim.x) {
    int u = t / Wa, v = t % Wa;
    int xu = -g.da + u, U0 = floor4(xu), tu = xu - NREF * U0;
    const double* col = R + (U0 + o) * Wa + v;
    double s;
    if (tu == 0) {
      s = col[0];
    } else {
      s = 0.0;
      for (int k = -b; k <= b + 1; ++k) s += lw.w[tu][k + b] * col[k * Wa];
    }
    out[t] = T(double(out[t]) - s);
  }
}

// ------------------------------------------------------------ skeleton ----
struct SkelGeom {
  int N, n, ppa, K, da, db, b, Wa, P0, npl, Wb, P0b, nplb, O_lo, No;
  double c2h2;   // C2 h^2
};

// Legendre far field of the annulus patches at every skeleton node
// (sec. 4.1 eq. philocmlcII, second sum, after the regrouping by linearity):
//   A[g] = sum_{i in S_beta(g)} sum_p c_{i,p} D_p[g - n i],
// D_p = Phi_p - I(Phi_p) on the skeleton planes of Omega_beta(0), zero on
// Omega_alpha(0).  With g = n k + r (r in [0, n)^2 in the face plane of
// normal d, r_d = 0), g - n i = n (k - i) + r: for one (d, r) the sum is a
// convolution over the patch lattice.  Block = one (r, d); threads take the
// lattice points k; moments in LDS; the table values of one lattice offset
// are read once per block.  Writes A into phiB (every canonical node).
__global__ void __launch_bounds__(256) skeleton_annulus_kernel(const double* __restrict__ mom,
                                                               const double* __restrict__ D, SkelGeom g,
                                                               double* __restrict__ phiB) {
  __shared__ double cm[MAXPATCH * KMAX];
  const int n = g.n, K = g.K, ppa = g.ppa, N = g.N, Np = N + 1;
  const int npatch = ppa * ppa * ppa;
  const int ra = blockIdx.x / n, rb = blockIdx.x % n, d = blockIdx.y;
  const int a0 = d == 0 ? 1 : 0, a1 = d == 2 ? 1 : 2;
  // canonical plane: no in-plane axis below d on a patch face
  if ((a0 < d && ra == 0) || (a1 < d && rb == 0)) return;
  const bool in_lds = npatch <= MAXPATCH;
  if (in_lds)
    for (int t = threadIdx.x; t < npatch * K; t += blockDim.x) cm[t] = mom[t];
  const double* cmp = in_lds ? cm : mom;
  __syncthreads();
  // offsets k - i = Dl with n Dl + r inside Omega_beta(0) on each axis
  auto drange = [&](int r, int& lo, int& hi) {
    int x = -g.db - r;
    lo = x >= 0 ? (x + n - 1) / n : -((-x) / n);
    int y = n + g.db - r;
    hi = y >= 0 ? y / n : -((-y + n - 1) / n);
  };
  int dlo[3], dhi[3];
  drange(0, dlo[0], dhi[0]);
  drange(ra, dlo[1], dhi[1]);
  drange(rb, dlo[2], dhi[2]);
  // lattice points: kd in [0, ppa], ka, kb in [0, ppa] with n k + r <= N
  const int nka = (ra == 0) ? ppa + 1 : ppa, nkb = (rb == 0) ? ppa + 1 : ppa;
  const int nk = (ppa + 1) * nka * nkb;
  constexpr int PER = 8;
  for (int kbase = 0; kbase < nk; kbase += PER * 256) {
    double acc[PER];
#pragma unroll
    for (int t = 0; t < PER; ++t) acc[t] = 0.0;
    for (int E0 = dlo[0]; E0 <= dhi[0]; ++E0)
      for (int E1 = dlo[1]; E1 <= dhi[1]; ++E1)
        for (int E2 = dlo[2]; E2 <= dhi[2]; ++E2) {
          int jb = (n * E0 - g.P0b) / n;
          const double* dv = D + ((((int64_t(d) * g.nplb + jb) * g.Wb + (ra + n * E1 + g.db)) * g.Wb) +
                                  (rb + n * E2 + g.db)) * K;
          double tr[KMAX];
#pragma unroll
          for (int p = 0; p < KMAX; ++p) tr[p] = p < K ? dv[p] : 0.0;
#pragma unroll
          for (int t = 0; t < PER; ++t) {
            int kk = kbase + threadIdx.x + t * 256;
            if (kk >= nk) break;
            int kd = kk / (nka * nkb), ka = (kk / nkb) % nka, kb = kk % nkb;
            int i[3];
            i[d] = kd - E0;
            i[a0] = ka - E1;
            i[a1] = kb - E2;
            if (i[0] < 0 || i[0] >= ppa || i[1] < 0 || i[1] >= ppa || i[2] < 0 || i[2] >= ppa) continue;
            const double* mv = cmp + ((i[0] * ppa + i[1]) * ppa + i[2]) * K;
            double l = 0.0;
#pragma unroll
            for (int p = 0; p < KMAX; ++p)
              if (p < K) l += tr[p] * mv[p];
            acc[t] += l;
          }
        }
#pragma unroll
    for (int t = 0; t < PER; ++t) {
      int kk = kbase + threadIdx.x + t * 256;
      if (kk >= nk) break;
      int kd = kk / (nka * nkb), ka = (kk / nkb) % nka, kb = kk % nkb;
      int gg[3];
      gg[d] = n * kd;
      gg[a0] = n * ka + ra;
      gg[a1] = n * kb + rb;
      phiB[(int64_t(gg[0]) * Np + gg[1]) * Np + gg[2]] = acc[t];
    }
  }
}

// phi^B[g] = I(phi^H)(g) + sum_{i in S_alpha(g)} delta_i[g] (+ the annulus
// far field already in phiB when `annulus`) for every skeleton node g (taken
// once, on its lowest face-normal axis); also writes
// phi[g] = phi^B[g] + C2 h^2 f[g] (sec. 4.1 eqs. mlcfulldiscr,
// mcapplicationfulldiscr).
template <typename T>
__global__ void __launch_bounds__(256) skeleton_kernel(const double* __restrict__ phiH, const T* __restrict__ delta,
                                                       const double* __restrict__ f, SkelGeom g, LagW lw,
                                                       int annulus, double* __restrict__ phiB,
                                                       double* __restrict__ phi) {
  const int N = g.N, n = g.n, Np = N + 1;
  const int planes = N / n + 1;
  int64_t idx = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (idx >= int64_t(3) * planes * Np * Np) return;
  int v = int(idx % Np), u = int((idx / Np) % Np), j = int((idx / (int64_t(Np) * Np)) % planes);
  int d = int(idx / (int64_t(Np) * Np * planes));
  int a0 = d == 0 ? 1 : 0, a1 = d == 2 ? 1 : 2;
  // canonical plane: no lower axis divisible by n
  if (a0 < d && u % n == 0) return;
  if (a1 < d && v % n == 0) return;
  int gg[3];
  gg[d] = j * n;
  gg[a0] = u;
  gg[a1] = v;
  // coarse interpolation of phi^H in the plane x_d = g_d
  double val;
  {
    int U0 = u / NREF, V0 = v / NREF, tu = u - NREF * U0, tv = v - NREF * V0;
    const double* wu = lw.w[tu];
    const double* wv = lw.w[tv];
    int ku0 = tu ? -g.b : 0, ku1 = tu ? g.b + 1 : 0, kv0 = tv ? -g.b : 0, kv1 = tv ? g.b + 1 : 0;
    int cd = gg[d] / NREF - g.O_lo;
    double s = 0.0;
    for (int ku = ku0; ku <= ku1; ++ku) {
      double rs = 0.0;
      for (int kv = kv0; kv <= kv1; ++kv) {
        int c[3];
        c[d] = cd;
        c[a0] = U0 + ku - g.O_lo;
        c[a1] = V0 + kv - g.O_lo;
        rs += wv[kv + g.b] * phiH[(int64_t(c[0]) * g.No + c[1]) * g.No + c[2]];
      }
      s += wu[ku + g.b] * rs;
    }
    val = s;
  }
  // patches with g in Omega_alpha(i): n i - da <= g <= n i + n + da
  int lo[3], hi[3];
  for (int a = 0; a < 3; ++a) {
    int x = gg[a] - n - g.da;
    lo[a] = max(x >= 0 ? (x + n - 1) / n : -((-x) / n), 0);
    hi[a] = min((gg[a] + g.da) / n, g.ppa - 1);
  }
  const int Wa = g.Wa;
  for (int i0 = lo[0]; i0 <= hi[0]; ++i0)
    for (int i1 = lo[1]; i1 <= hi[1]; ++i1)
      for (int i2 = lo[2]; i2 <= hi[2]; ++i2) {
        int r[3] = {gg[0] - n * i0, gg[1] - n * i1, gg[2] - n * i2};
        int pidx = (i0 * g.ppa + i1) * g.ppa + i2;
        int jj = (r[d] - g.P0) / n;
        val += double(delta[((((int64_t(pidx) * 3 + d) * g.npl + jj) * Wa + (r[a0] + g.da)) * Wa) + (r[a1] + g.da)]);
      }
  int64_t node = (int64_t(gg[0]) * Np + gg[1]) * Np + gg[2];
  if (annulus) val += phiB[node];
  phiB[node] = val;
  phi[node] = val + g.c2h2 * f[node];
}

// ----------------------------------------------------------- Dirichlet ----
// rhs[p][m0][m1][m2] over the (n-1)^3 interior nodes of patch p:
//   h^2 f[g] - sum_{s : g+s on the patch boundary} b_|s| phi^B[g+s].
__global__ void dirichlet_rhs_kernel(const double* __restrict__ f, const double* __restrict__ phiB, int N, int n,
                                     int ppa, Stencil st, double h2, double* __restrict__ rhs) {
  const int m = n - 1;
  const int p = blockIdx.y;
  int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= cube(m)) return;
  int m2 = int(t % m), m1 = int((t / m) % m), m0 = int(t / (int64_t(m) * m));
  const int i0 = p / (ppa * ppa), i1 = (p / ppa) % ppa, i2 = p % ppa;
  const int64_t Np = N + 1;
  int l0 = m0 + 1, l1 = m1 + 1, l2 = m2 + 1;   // patch-local node
  int64_t base = (int64_t(n) * i0) * Np * Np + int64_t(n) * i1 * Np + int64_t(n) * i2;
  double s = h2 * f[base + (l0 * Np + l1) * Np + l2];
  if (l0 == 1 || l0 == n - 1 || l1 == 1 || l1 == n - 1 || l2 == 1 || l2 == n - 1) {
    for (int s0 = -1; s0 <= 1; ++s0)
      for (int s1 = -1; s1 <= 1; ++s1)
        for (int s2 = -1; s2 <= 1; ++s2) {
          int k0 = l0 + s0, k1 = l1 + s1, k2 = l2 + s2;
          bool bnd = k0 == 0 || k0 == n || k1 == 0 || k1 == n || k2 == 0 || k2 == n;
          if (!bnd) continue;
          int nz = (s0 != 0) + (s1 != 0) + (s2 != 0);
          s -= st.b[nz] * phiB[base + (k0 * Np + k1) * Np + k2];
        }
  }
  rhs[int64_t(p) * cube(m) + t] = s;
}

// Dense DST-I of length m = n-1 along one axis of each patch's m^3 block:
//   out[k] = scale * sum_j sin(pi (k+1)(j+1) / n) in[j].
// Block (slab u, patch): the slab is the m x m plane of the two axes other
// than `axis`... processed as m lines of length m.
__global__ void __launch_bounds__(256) dst_small_axis_kernel(const double* __restrict__ in, double* __restrict__ out,
                                                             int n, int axis, double scale) {
  const int m = n - 1;
  __shared__ double sn[SMAXN * SMAXN];
  __shared__ double slab[SMAXN * SMAXN];
  const int u = blockIdx.x, p = blockIdx.y;
  for (int t = threadIdx.x; t < m * m; t += blockDim.x) {
    int k = t / m, j = t % m;
    // sin(pi (k+1)(j+1)/n) with an exact integer argument reduced mod 2n
    int a = ((k + 1) * (j + 1)) % (2 * n);
    sn[t] = sinpi(double(a) / double(n));
  }
  // slab: lines along `axis`; the other two axes are (u, w) with u the slower
  const int64_t M3 = cube(m);
  const int64_t sa = axis == 0 ? int64_t(m) * m : (axis == 1 ? m : 1);
  const int64_t su = axis == 0 ? m : int64_t(m) * m;   // slower other axis
  const int64_t sw = axis == 2 ? m : 1;                 // faster other axis
  const double* ib = in + int64_t(p) * M3 + u * su;
  for (int t = threadIdx.x; t < m * m; t += blockDim.x) {
    int j = t / m, w = t % m;   // element j of line w
    slab[j * m + w] = ib[j * sa + w * sw];
  }
  __syncthreads();
  double* ob = out + int64_t(p) * M3 + u * su;
  for (int t = threadIdx.x; t < m * m; t += blockDim.x) {
    int k = t / m, w = t % m;
    double s = 0.0;
    for (int j = 0; j < m; ++j) s += sn[k * m + j] * slab[j * m + w];
    ob[k * sa + w * sw] = scale * s;
  }
}

__global__ void dirichlet_divide_kernel(double* __restrict__ data, int n, Stencil st) {
  const int m = n - 1;
  const int p = blockIdx.y;
  int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= cube(m)) return;
  int k2 = int(t % m) + 1, k1 = int((t / m) % m) + 1, k0 = int(t / (int64_t(m) * m)) + 1;
  double c0 = cospi(double(k0) / n), c1 = cospi(double(k1) / n), c2 = cospi(double(k2) / n);
  double lam = st.b[0] + 2.0 * st.b[1] * (c0 + c1 + c2) + 4.0 * st.b[2] * (c0 * c1 + c0 * c2 + c1 * c2) +
               8.0 * st.b[3] * c0 * c1 * c2;
  data[int64_t(p) * cube(m) + t] /= lam;
}

// phi = u + C2 h^2 f on the interior nodes of every patch.
__global__ void dirichlet_final_kernel(const double* __restrict__ u, const double* __restrict__ f, int N, int n,
                                       int ppa, double c2h2, double* __restrict__ phi) {
  const int m = n - 1;
  const int p = blockIdx.y;
  int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= cube(m)) return;
  int m2 = int(t % m), m1 = int((t / m) % m), m0 = int(t / (int64_t(m) * m));
  const int i0 = p / (ppa * ppa), i1 = (p / ppa) % ppa, i2 = p % ppa;
  const int64_t Np = N + 1;
  int64_t node = (int64_t(n) * i0 + m0 + 1) * Np * Np + (int64_t(n) * i1 + m1 + 1) * Np + int64_t(n) * i2 + m2 + 1;
  phi[node] = u[int64_t(p) * cube(m) + t] + c2h2 * f[node];
}

}  // namespace mlc
