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

// F^H[c] = sum_i F_i[c]: Delta^H of phi_i's coarse samples on C(Omega_alpha(i)),
// the Legendre far field sum_p c_{i,p} T_p[c - n i / 4] on
// C(Omega_beta(i)) \ C(Omega_alpha(i)) (T is zero on the inner box), patches
// visited in a fixed order.
template <typename T>
__global__ void __launch_bounds__(256) coarse_rhs_kernel(const T* __restrict__ cs, const double* __restrict__ mom,
                                                         const double* __restrict__ Tt, Stencil st, CoarseGeom g,
                                                         double* __restrict__ F) {
  int64_t idx = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (idx >= cube(g.Ns)) return;
  int c[3];
  c[2] = g.S_lo + int(idx % g.Ns);
  c[1] = g.S_lo + int((idx / g.Ns) % g.Ns);
  c[0] = g.S_lo + int(idx / (int64_t(g.Ns) * g.Ns));
  const int n = g.n, q = n / NREF;
  // patches whose C(Omega_beta) contains c: n i - db <= 4c <= n i + n + db
  int lo[3], hi[3];
  for (int d = 0; d < 3; ++d) {
    int a = NREF * c[d] - n - g.db;   // n i >= a
    lo[d] = a >= 0 ? (a + n - 1) / n : -((-a) / n);
    int bnd = NREF * c[d] + g.db;     // n i <= bnd
    hi[d] = bnd >= 0 ? bnd / n : -((-bnd + n - 1) / n);
    lo[d] = max(lo[d], 0);
    hi[d] = min(hi[d], g.ppa - 1);
  }
  const int Wc = g.Wc, Wbc = g.Wbc, K = g.K;
  double s = 0.0;
  for (int a0 = lo[0]; a0 <= hi[0]; ++a0)
    for (int a1 = lo[1]; a1 <= hi[1]; ++a1)
      for (int a2 = lo[2]; a2 <= hi[2]; ++a2) {
        int r0 = c[0] - q * a0, r1 = c[1] - q * a1, r2 = c[2] - q * a2;   // coarse coords rel. patch
        int alo = -g.da / NREF, ahi = (n + g.da) / NREF;
        int pidx = (a0 * g.ppa + a1) * g.ppa + a2;
        if (r0 >= alo && r0 <= ahi && r1 >= alo && r1 <= ahi && r2 >= alo && r2 <= ahi) {
          const T* base = cs + int64_t(pidx) * Wc * Wc * Wc;
          int o = g.e / NREF;
          double l = 0.0;
          for (int s0 = -1; s0 <= 1; ++s0)
            for (int s1 = -1; s1 <= 1; ++s1)
              for (int s2 = -1; s2 <= 1; ++s2) {
                int nz = (s0 != 0) + (s1 != 0) + (s2 != 0);
                l += st.b[nz] * double(base[(int64_t(r0 + s0 + o) * Wc + (r1 + s1 + o)) * Wc + (r2 + s2 + o)]);
              }
          s += l * g.invH2;
        } else if (K > 0) {
          int ob = g.db / NREF;
          const double* tv = Tt + ((int64_t(r0 + ob) * Wbc + (r1 + ob)) * Wbc + (r2 + ob)) * K;
          const double* mv = mom + int64_t(pidx) * K;
          double l = 0.0;
          for (int k = 0; k < K; ++k) l += mv[k] * tv[k];
          s += l;
        }
      }
  F[idx] = s;
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
// delta_i = phi_i - I(phi_i) on phi_i's skeleton planes inside Omega_alpha,
// in place; I interpolates phi_i's coarse samples in the plane.
template <typename T>
__global__ void plane_delta_kernel(T* __restrict__ planes, const T* __restrict__ cs, int n, int e, int da, int Wa,
                                   int Wc, int P0, int npl, int b) {
  const int p = blockIdx.y;
  const int64_t per = int64_t(3) * npl * Wa * Wa;
  int64_t r = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (r >= per) return;
  int v = int(r % Wa), u = int((r / Wa) % Wa), j = int((r / (int64_t(Wa) * Wa)) % npl);
  int d = int(r / (int64_t(Wa) * Wa * npl));
  int P = P0 + j * n;
  int xu = -da + u, xv = -da + v;
  int U0 = xu >= 0 ? xu / NREF : -((-xu + NREF - 1) / NREF);
  int V0 = xv >= 0 ? xv / NREF : -((-xv + NREF - 1) / NREF);
  int tu = xu - NREF * U0, tv = xv - NREF * V0;
  double wu[10], wv[10];
  int ku0 = 0, ku1 = 0, kv0 = 0, kv1 = 0;
  if (tu) { lagrange_weights(b, tu / double(NREF), wu); ku0 = -b; ku1 = b + 1; } else { wu[b] = 1.0; }
  if (tv) { lagrange_weights(b, tv / double(NREF), wv); kv0 = -b; kv1 = b + 1; } else { wv[b] = 1.0; }
  const T* cb = cs + int64_t(p) * Wc * Wc * Wc;
  int o = e / NREF, cd = (P + e) / NREF;
  double s = 0.0;
  for (int ku = ku0; ku <= ku1; ++ku) {
    double rs = 0.0;
    for (int kv = kv0; kv <= kv1; ++kv) {
      int c[3];
      c[d] = cd;
      c[d == 0 ? 1 : 0] = U0 + ku + o;
      c[d == 2 ? 1 : 2] = V0 + kv + o;
      rs += wv[kv + b] * double(cb[(int64_t(c[0]) * Wc + c[1]) * Wc + c[2]]);
    }
    s += wu[ku + b] * rs;
  }
  T* pl = planes + int64_t(p) * per + r;
  *pl = T(double(*pl) - s);
}

// ------------------------------------------------------------ skeleton ----
struct SkelGeom {
  int N, n, ppa, K, da, db, b, Wa, P0, npl, Wb, P0b, nplb, O_lo, No;
  double c2h2;   // C2 h^2
};

// phi^B[g] = I(phi^H)(g) + sum_{i in S_alpha(g)} delta_i[g]
//          + sum_{i in S_beta(g)} sum_p c_{i,p} D_p[g - n i]
// for every skeleton node g (taken once, on its lowest face-normal axis);
// also writes phi[g] = phi^B[g] + C2 h^2 f[g] (sec. 4.1 eqs. mlcfulldiscr,
// mcapplicationfulldiscr).
template <typename T>
__global__ void __launch_bounds__(256) skeleton_kernel(const double* __restrict__ phiH, const T* __restrict__ delta,
                                                       const double* __restrict__ mom, const double* __restrict__ D,
                                                       const double* __restrict__ f, SkelGeom g,
                                                       double* __restrict__ phiB, double* __restrict__ phi) {
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
    double wu[10], wv[10];
    int ku0 = 0, ku1 = 0, kv0 = 0, kv1 = 0;
    if (tu) { lagrange_weights(g.b, tu / double(NREF), wu); ku0 = -g.b; ku1 = g.b + 1; } else { wu[g.b] = 1.0; }
    if (tv) { lagrange_weights(g.b, tv / double(NREF), wv); kv0 = -g.b; kv1 = g.b + 1; } else { wv[g.b] = 1.0; }
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
  // patches with g in Omega_beta(i): n i - db <= g <= n i + n + db
  int lo[3], hi[3];
  for (int a = 0; a < 3; ++a) {
    int x = gg[a] - n - g.db;
    lo[a] = max(x >= 0 ? (x + n - 1) / n : -((-x) / n), 0);
    int y = gg[a] + g.db;
    hi[a] = min(y / n, g.ppa - 1);
  }
  const int Wa = g.Wa, Wb = g.Wb, K = g.K;
  for (int i0 = lo[0]; i0 <= hi[0]; ++i0)
    for (int i1 = lo[1]; i1 <= hi[1]; ++i1)
      for (int i2 = lo[2]; i2 <= hi[2]; ++i2) {
        int r[3] = {gg[0] - n * i0, gg[1] - n * i1, gg[2] - n * i2};
        int pidx = (i0 * g.ppa + i1) * g.ppa + i2;
        bool inner = r[0] >= -g.da && r[0] <= n + g.da && r[1] >= -g.da && r[1] <= n + g.da && r[2] >= -g.da &&
                     r[2] <= n + g.da;
        if (inner) {
          int jj = (r[d] - g.P0) / n;
          val += double(delta[((((int64_t(pidx) * 3 + d) * g.npl + jj) * Wa + (r[a0] + g.da)) * Wa) + (r[a1] + g.da)]);
        } else if (K > 0) {
          int jb = (r[d] - g.P0b) / n;
          const double* dv = D + ((((int64_t(d) * g.nplb + jb) * Wb + (r[a0] + g.db)) * Wb) + (r[a1] + g.db)) * K;
          const double* mv = mom + int64_t(pidx) * K;
          double l = 0.0;
          for (int k = 0; k < K; ++k) l += mv[k] * dv[k];
          val += l;
        }
      }
  int64_t node = (int64_t(gg[0]) * Np + gg[1]) * Np + gg[2];
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
