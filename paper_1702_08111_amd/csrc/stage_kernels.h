// Per-solve kernels of the two-level MLC other than the local convolutions,
// all in float64: Legendre moments, the coarse right-hand side, the coarse
// Hockney solve's torus fill/extract, the boundary values on the patch
// skeleton, and the patch Dirichlet solves with the final correction.
#pragma once
#include "common.h"
#include "setup_kernels.h"

namespace mlc {

// ------------------------------------------------------------ moments ----
// c_{i,p}: the raw moments m_p = R^{3/2} sum_j W_j f[j] qhat_p(t_j) over the
// (n+1)^3 nodes of the closed patch, W = tensor composite Boole weights on
// [-1, 1] (sec. 4.1 step 1 quadrature), projected with the Boole Gram matrix
// of the modes, c = Gram^{-1} m (sec. 3 projection).  For P <= 4 the Gram
// matrix is diagonal, mu_p = prod_d sum_j w_j qhat_{p_d}(t_j)^2, and the
// kernel divides (diag = 1); for P >= 5 it writes m and
// moments_gram_kernel applies the inverse.  The sums over the two fastest
// axes are taken per z-plane by the x-DFT kernel of the local convolutions
// (which loads every plane anyway): part[p][j0][a1 P + a2] =
// sum_{j1,j2} w_j1 qhat_a1 w_j2 qhat_a2 f.  This kernel contracts j0, one
// thread per (patch, mode).
__global__ void __launch_bounds__(256) moments_finish_kernel(const ProbDesc* __restrict__ pd, int nprob, int n,
                                                             int P, ModeList modes, const double* __restrict__ part,
                                                             double* __restrict__ out, int total, int diag,
                                                             const int* __restrict__ patch_of) {
  const int64_t idx = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (idx >= int64_t(total) * modes.K) return;
  // one thread per (slot, mode); the slot's patch owns the output row
  const int slot = int(idx / modes.K), k = int(idx % modes.K);
  const int p = patch_of ? patch_of[slot] : slot;
  const ProbDesc& D = pd[find_problem(pd, nprob, p)];
  const int a0 = modes.p[k][0], a1 = modes.p[k][1], a2 = modes.p[k][2];
  const int S = n + 1, PP = P * P;
  const double* pp = part + int64_t(slot) * S * PP + P * a1 + a2;
  double s = 0.0, mu0 = 0.0, mu1 = 0.0, mu2 = 0.0;
  for (int j = 0; j < S; ++j) {
    const double t = (j - 0.5 * n) / (0.5 * n), w = boole_w(j, n);
    const double q0 = qhat(a0, t), q1 = qhat(a1, t), q2 = qhat(a2, t);
    s += w * q0 * pp[j * PP];
    mu0 += w * q0 * q0;
    mu1 += w * q1 * q1;
    mu2 += w * q2 * q2;
  }
  out[int64_t(p) * modes.K + k] = diag ? D.R15 * s / (mu0 * mu1 * mu2) : D.R15 * s;
}

// c = Gram^{-1} m per patch (P >= 5, where the Boole Gram matrix of the modes
// is no longer diagonal): one thread per (patch, mode), the row of the
// inverse (K x K, row-major, built on the host) against the patch's raw
// moments, summed in mode order.
__global__ void __launch_bounds__(256) moments_gram_kernel(const double* __restrict__ raw,
                                                           const double* __restrict__ ginv, int K,
                                                           double* __restrict__ out, int total) {
  const int64_t idx = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (idx >= int64_t(total) * K) return;
  const int p = int(idx / K), k = int(idx % K);
  const double* m = raw + int64_t(p) * K;
  const double* g = ginv + int64_t(k) * K;
  double s = 0.0;
  for (int q = 0; q < K; ++q) s += g[q] * m[q];
  out[idx] = s;
}

// dst[d + i] = src[s + i] for i in [0, w)^3 (cubic node arrays of edges sn,
// dn; s and d per-axis offsets): the coarse charge into the next level's
// box, and that level's solution back onto the coarse output box.
__global__ void box_copy_kernel(const double* __restrict__ src, int sn, int soff, double* __restrict__ dst, int dn,
                                int doff, int w) {
  const int64_t idx = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (idx >= int64_t(w) * w * w) return;
  const int i2 = int(idx % w), i1 = int((idx / w) % w), i0 = int(idx / (int64_t(w) * w));
  dst[(int64_t(doff + i0) * dn + (doff + i1)) * dn + (doff + i2)] =
      src[(int64_t(soff + i0) * sn + (soff + i1)) * sn + (soff + i2)];
}

// ------------------------------------------------------- coarse rhs ----
struct CoarseGeom {
  int n, ppa, K, da, db, e, Wc, S_lo, Ns, Wbc;
  double invH2;
};

// Per-problem data of the kernels that run over all problems of a batch in
// one flat launch: problem k owns the thread indices [start_k, start_{k+1}).
template <typename D>
__device__ __forceinline__ const D& flat_problem(const D* __restrict__ pr, int np, int64_t idx) {
  int lo = 0, hi = np - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (pr[mid].start <= idx) lo = mid; else hi = mid - 1;
  }
  return pr[lo];
}
constexpr int FLAT_PACK = 8;
template <typename D> struct FlatPack { D d[FLAT_PACK]; int count; };
template <typename D>
__global__ void flat_upload_kernel(D* __restrict__ dst, FlatPack<D> pk) {
  if (int(threadIdx.x) < pk.count) dst[threadIdx.x] = pk.d[threadIdx.x];
}

template <typename T> struct CoarseRhsProb {
  const double* lap;   // coarse Laplacians of the problem's patches' coarse samples
  double* F;           // its F^H
  CoarseGeom g;
  int64_t start;
  const int* slot_of;  // patch -> its slot in lap (-1: an empty patch, no slot), or null (slot = patch)
};

// Delta^H of each patch's coarse samples at the points r in [b, Wc - b)^3 of
// its coarse box (those of C(Omega_alpha), the only ones the right-hand side
// reads; their 27-point neighbourhoods stay inside the box since b >= 1), in
// float64: lap[patch][r - b].  Block (output plane r0 - b, patch): the three
// sample planes r0 - 1 .. r0 + 1 go to dynamic LDS (3 Wc^2 values), then one
// thread per output point.
template <typename T>
__global__ void __launch_bounds__(256) coarse_lap_kernel(const T* __restrict__ cs, double* __restrict__ lap, int Wc,
                                                         int b, Stencil st, const int* __restrict__ live, int p0) {
  extern __shared__ unsigned char lap_lds[];
  T* sm = reinterpret_cast<T*>(lap_lds);
  const int Li = Wc - 2 * b, i0 = blockIdx.x, W2 = Wc * Wc;
  const int64_t p = p0 + int64_t(blockIdx.y);
  if (live && !live[p]) {
    // an empty patch: the Laplacian of its zero samples
    double* dst = lap + (p * Li + i0) * Li * Li;
    for (int t = threadIdx.x; t < Li * Li; t += blockDim.x) dst[t] = 0.0;
    return;
  }
  const T* src = cs + (p * Wc + (b + i0 - 1)) * W2;   // planes r0 - 1 .. r0 + 1 are consecutive
  for (int t = threadIdx.x; t < 3 * W2; t += blockDim.x) sm[t] = src[t];
  __syncthreads();
  double* dst = lap + (p * Li + i0) * Li * Li;
  for (int t = threadIdx.x; t < Li * Li; t += blockDim.x) {
    const int r1 = b + t / Li, r2 = b + t % Li;
    double l = 0.0;
#pragma unroll
    for (int s0 = -1; s0 <= 1; ++s0)
#pragma unroll
      for (int s1 = -1; s1 <= 1; ++s1)
#pragma unroll
        for (int s2 = -1; s2 <= 1; ++s2) {
          const int nz = (s0 != 0) + (s1 != 0) + (s2 != 0);
          l += st.b[nz] * double(sm[((1 + s0) * Wc + (r1 + s1)) * Wc + (r2 + s2)]);
        }
    dst[t] = l;
  }
}

// Inner part of F^H: F[c] += sum over patches i with c in C(Omega_alpha(i)) of
// Delta^H of phi_i's coarse samples (sec. 4.1 eq. FDLD, first case), patches
// visited in a fixed order.  One thread per coarse point of every problem.
template <typename T>
__global__ void __launch_bounds__(256) coarse_rhs_kernel(const CoarseRhsProb<T>* __restrict__ pr, int np,
                                                         int64_t total, int b) {
  const int64_t gidx = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (gidx >= total) return;
  const CoarseRhsProb<T>& pb = flat_problem(pr, np, gidx);
  const CoarseGeom g = pb.g;
  const double* __restrict__ lap = pb.lap;
  double* __restrict__ F = pb.F;
  const int64_t idx = gidx - pb.start;
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
  const int Li = g.Wc - 2 * b, o = g.e / NREF - b;
  // at most 4 covering patches per axis (their C(Omega_alpha) spans n + 2 da
  // <= 3n fine cells); the 16 values of one a0 are loaded together, then
  // added in (a0, a1, a2) order
  constexpr int PA = 4;
  double s = 0.0;
  for (int a0 = lo[0]; a0 <= hi[0]; ++a0) {
    double v[PA][PA];
#pragma unroll
    for (int j1 = 0; j1 < PA; ++j1)
#pragma unroll
      for (int j2 = 0; j2 < PA; ++j2) {
        const int a1 = lo[1] + j1, a2 = lo[2] + j2;
        v[j1][j2] = 0.0;
        if (a1 <= hi[1] && a2 <= hi[2]) {
          const int i0 = c[0] - q * a0 + o, i1 = c[1] - q * a1 + o, i2 = c[2] - q * a2 + o;
          int pidx = (a0 * g.ppa + a1) * g.ppa + a2;
          if (pb.slot_of) pidx = pb.slot_of[pidx];
          if (pidx >= 0) v[j1][j2] = lap[(int64_t(pidx) * Li + i0) * Li * Li + int64_t(i1) * Li + i2];
        }
      }
#pragma unroll
    for (int j1 = 0; j1 < PA; ++j1)
#pragma unroll
      for (int j2 = 0; j2 < PA; ++j2)
        if (lo[1] + j1 <= hi[1] && lo[2] + j2 <= hi[2]) s += v[j1][j2] * g.invH2;
  }
  F[idx] += s;   // F starts at zero; the far-field sums may add first
}

// The optional input check: flag = 1 if f is nonzero at any node within
// `layers` node layers of the six outer faces of its (B0+1)(B1+1)(B2+1) node
// box.  Threads cover (face, layer, a, b) with a, b up to the largest edge;
// those past a face's own extent do nothing.
__global__ void set_flag_kernel(int* __restrict__ flag, int v) { *flag = v; }
__global__ void boundary_check_kernel(const double* __restrict__ f, int B0, int B1, int B2, int layers,
                                      int* __restrict__ flag) {
  const int64_t Bm = max(B0, max(B1, B2)) + 1;
  const int64_t idx = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (idx >= 6 * layers * Bm * Bm) return;
  const int face = int(idx / (layers * Bm * Bm));
  const int layer = int((idx / (Bm * Bm)) % layers);
  const int64_t a = (idx / Bm) % Bm, b = idx % Bm;
  const int B[3] = {B0, B1, B2};
  const int d = face / 2;                            // the face's normal axis
  const int u = d == 0 ? 1 : 0, v = d == 2 ? 1 : 2;   // its in-plane axes
  if (a > B[u] || b > B[v] || layer > B[d]) return;
  int64_t g[3];
  g[d] = (face & 1) ? B[d] - layer : layer;
  g[u] = a;
  g[v] = b;
  if (f[(g[0] * (B1 + 1) + g[1]) * (B2 + 1) + g[2]] != 0.0) *flag = 1;
}

// dst[i] = src[i] for i in [0, w0) x [0, w1) x [0, w2) of node arrays of
// extents (s0, s1, s2) and (d0, d1, d2): a box domain into its enclosing cube
// and the cube's phi back onto the box.
__global__ void box3_copy_kernel(const double* __restrict__ src, int s0, int s1, int s2, double* __restrict__ dst,
                                 int d0, int d1, int d2, int w0, int w1, int w2) {
  (void)s0;
  (void)d0;
  // grid-stride: node arrays can exceed 2^32 entries, more than one launch's threads
  for (int64_t idx = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; idx < int64_t(w0) * w1 * w2;
       idx += int64_t(gridDim.x) * blockDim.x) {
    const int i2 = int(idx % w2), i1 = int((idx / w2) % w1), i0 = int(idx / (int64_t(w1) * w2));
    dst[(int64_t(i0) * d1 + i1) * d2 + i2] = src[(int64_t(i0) * s1 + i1) * s2 + i2];
  }
}

// The modified right-hand side of the sixth-order variant for the 27-point
// operator (sec. 2 eq. msCorr; the h^4 operator is the one in that
// operator's truncation error, appendix A.1):
//   f~ = f + (1/12) sum_d (-f[+-2 e_d] + 16 f[+-1 e_d] - 30 f) / 12
//          + (1/360) (sum_d (f[+-2 e_d] - 4 f[+-1 e_d] + 6 f) + 4 sum_{d<e} dd_d dd_e f),
// dd the second difference (h = 1 units; the result does not depend on h).
// Collected per offset class: centre 1 - 90/144 + (18 + 48)/360 = 67/120;
// axis +-1: 16/144 + (-4 - 2 * 2 * 4)/360 = 1/18; axis +-2: -1/144 + 1/360 =
// -1/240; in-plane diagonals (+-1, +-1, 0): 4/360 = 1/90; the sum is 1.
// f is taken as zero past the node box.  One thread per node.
__global__ void sixth_rhs_kernel(const double* __restrict__ f, int N, double* __restrict__ ft) {
  const int64_t Np = N + 1;
  // grid-stride over the nodes
  for (int64_t idx = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; idx < Np * Np * Np;
       idx += int64_t(gridDim.x) * blockDim.x) {
    const int g2 = int(idx % Np), g1 = int((idx / Np) % Np), g0 = int(idx / (Np * Np));
    auto at = [&](int a, int b, int c) -> double {
      if (a < 0 || a > N || b < 0 || b > N || c < 0 || c > N) return 0.0;
      return f[(int64_t(a) * Np + b) * Np + c];
    };
    const double ax1 = at(g0 - 1, g1, g2) + at(g0 + 1, g1, g2) + at(g0, g1 - 1, g2) + at(g0, g1 + 1, g2) +
                       at(g0, g1, g2 - 1) + at(g0, g1, g2 + 1);
    const double ax2 = at(g0 - 2, g1, g2) + at(g0 + 2, g1, g2) + at(g0, g1 - 2, g2) + at(g0, g1 + 2, g2) +
                       at(g0, g1, g2 - 2) + at(g0, g1, g2 + 2);
    double dg = 0.0;
    for (int s = -1; s <= 1; s += 2)
      for (int t = -1; t <= 1; t += 2)
        dg += at(g0 + s, g1 + t, g2) + at(g0 + s, g1, g2 + t) + at(g0, g1 + s, g2 + t);
    ft[idx] = (67.0 / 120.0) * at(g0, g1, g2) + (1.0 / 18.0) * ax1 - (1.0 / 240.0) * ax2 + (1.0 / 90.0) * dg;
  }
}

// live[p] = 1 when patch p's node charge (the (n+1)^3 nodes of its closed
// box) has a nonzero value or its problem does not skip empty patches; an
// empty patch has a zero local field and zero moments.  Block per patch.
__global__ void __launch_bounds__(256) patch_live_kernel(const ProbDesc* __restrict__ pd, int nprob, int n,
                                                         int* __restrict__ live, int p0) {
  __shared__ int any;
  const int p = p0 + blockIdx.x;
  const ProbDesc& D = pd[find_problem(pd, nprob, p)];
  if (!D.skip) {
    if (threadIdx.x == 0) live[p] = 1;
    return;
  }
  if (threadIdx.x == 0) any = 0;
  __syncthreads();
  const int pl = p - D.patch0, ppa = D.ppa, S = n + 1;
  const int i0 = pl / (ppa * ppa), i1 = (pl / ppa) % ppa, i2 = pl % ppa;
  const int64_t Np = D.N + 1;
  const double* f = D.f + (int64_t(n) * i0 * Np + int64_t(n) * i1) * Np + int64_t(n) * i2;
  int mine = 0;
  for (int t = threadIdx.x; t < S * S * S; t += blockDim.x) {
    const int a = t / (S * S), b = (t / S) % S, c = t % S;
    mine |= f[(a * Np + b) * Np + c] != 0.0;
  }
  if (mine) any = 1;   // benign race: every writer stores 1
  __syncthreads();
  if (threadIdx.x == 0) live[p] = any;
}

template <typename T>
__global__ void fill_zero_t_kernel(T* __restrict__ p, int64_t count) {
  for (int64_t idx = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; idx < count; idx += int64_t(gridDim.x) * blockDim.x)
    p[idx] = T(0);
}

__global__ void fill_zero_kernel(double* __restrict__ p, int64_t count) {
  for (int64_t idx = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; idx < count; idx += int64_t(gridDim.x) * blockDim.x)
    p[idx] = 0.0;
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


struct PlaneGeom { int n, e, da, Wa, Wc, P0, npl, b; };

// delta_i = phi_i - I(phi_i) on phi_i's skeleton planes inside Omega_alpha,
// in place.  Block (plane, patch): the plane's coarse samples go to LDS, are
// interpolated along the faster in-plane axis row by row, then along the
// slower one.
template <typename T>
__global__ void __launch_bounds__(256) plane_delta_kernel(T* __restrict__ planes, const T* __restrict__ cs,
                                                          PlaneGeom g, LagW lw, const int* __restrict__ live,
                                                          int p0) {
  // dynamic LDS of (Wc^2 + Wc Wa) doubles: the coarse samples C, then the
  // rows interpolated along the faster axis R
  extern __shared__ double plane_lds[];
  double* C = plane_lds;
  double* R = plane_lds + g.Wc * g.Wc;
  __shared__ double W[4][10];
  const int pl = blockIdx.x, p = p0 + blockIdx.y;
  if (live && !live[p]) return;   // an empty patch: its planes hold zeros, and so do their corrections
  if (threadIdx.x < 40) W[threadIdx.x / 10][threadIdx.x % 10] = lw.w[threadIdx.x / 10][threadIdx.x % 10];
  const int d = pl / g.npl, j = pl % g.npl;
  const int n = g.n, Wc = g.Wc, Wa = g.Wa, b = g.b, o = g.e / NREF;
  const int cd = (g.P0 + j * n + g.e) / NREF;
  const T* cb = cs + int64_t(p) * Wc * Wc * Wc;
  // the plane's coarse samples, four loads in flight per thread
  constexpr int UC = 4;
  for (int t0 = threadIdx.x; t0 < Wc * Wc; t0 += UC * blockDim.x) {
    T cv4[UC];
#pragma unroll
    for (int u = 0; u < UC; ++u) {
      const int t = t0 + u * int(blockDim.x);
      cv4[u] = T(0);
      if (t < Wc * Wc) {
        int c[3];
        c[d] = cd;
        c[d == 0 ? 1 : 0] = t / Wc;
        c[d == 2 ? 1 : 2] = t % Wc;
        cv4[u] = cb[(int64_t(c[0]) * Wc + c[1]) * Wc + c[2]];
      }
    }
#pragma unroll
    for (int u = 0; u < UC; ++u) {
      const int t = t0 + u * int(blockDim.x);
      if (t < Wc * Wc) C[t] = double(cv4[u]);
    }
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
      for (int k = -b; k <= b + 1; ++k) s += W[tv][k + b] * row[k];
    }
    R[cu * Wa + v] = s;
  }
  __syncthreads();
  T* out = planes + ((int64_t(p) * 3 + d) * g.npl + j) * Wa * Wa;
  // eight of the thread's points at a time: their old values in flight
  // during the interpolation
  constexpr int UO = 8;
  const int WW = Wa * Wa;
  for (int t0 = threadIdx.x; t0 < WW; t0 += UO * blockDim.x) {
    T old[UO];
#pragma unroll
    for (int q = 0; q < UO; ++q) {
      const int t = t0 + q * int(blockDim.x);
      old[q] = T(0);
      if (t < WW) old[q] = out[t];
    }
#pragma unroll
    for (int q = 0; q < UO; ++q) {
      const int t = t0 + q * int(blockDim.x);
      if (t >= WW) continue;
      int u = t / Wa, v = t % Wa;
      int xu = -g.da + u, U0 = floor4(xu), tu = xu - NREF * U0;
      const double* col = R + (U0 + o) * Wa + v;
      double s;
      if (tu == 0) {
        s = col[0];
      } else {
        s = 0.0;
        for (int k = -b; k <= b + 1; ++k) s += W[tu][k + b] * col[k * Wa];
      }
      out[t] = T(double(old[q]) - s);
    }
  }
}

// ------------------------------------------------------------ skeleton ----
struct SkelGeom {
  int N, n, ppa, K, da, db, b, Wa, P0, npl, Wb, P0b, nplb, O_lo, No;
  double c2h2;   // C2 h^2
};
template <typename T> struct SkelProb {
  const double* phiH;
  const T* delta;   // the problem's patches' plane corrections
  const double* f;
  double* phiB;
  double* phi;
  SkelGeom g;
  int64_t start;
  const int* slot_of;  // patch -> its slot in delta (-1: an empty patch), or null (slot = patch)
  int64_t bstart;      // the problem's first block in skeleton_finish_kernel
  const int* live;     // per patch of the problem: 1 unless known empty, or null (read f everywhere)
};

// ---------------------------------------------- annulus sums on MFMA ----
// Both Legendre far-field sums are dense contractions over (lattice offset E,
// mode p) once the intra-patch position is fixed:
//   out[r][k] = sum_{E, p} A[E][p][r] * c[k - E][p]
// with A a re-laid-out, zero-padded far-field table and c the moments
// (zero outside the patch lattice).  They run on v_mfma_f64_16x16x4f64:
// A fragment lane l = row (r) l%16, column p = l/16; B fragment lane l =
// column (k) l%16, row p = l/16; accumulator lane l, register j holds
// out[4 j + l/16][l%16].
//
// The moments are first copied into a zero-padded lattice (patch i at slot
// i + padlo per axis), so that c[k - E] is one address shifted by a uniform
// per-offset amount: no bounds tests in the inner loop.  Two layouts, each
// faster for one of the contractions: slot-major Cpad[L^3][KP] and
// mode-major Cpad[KP][L^3] (a tile's 16 consecutive columns of one mode are
// one contiguous run).
typedef double f64x4 __attribute__((ext_vector_type(4)));

struct MfmaGeom {
  int ppa, K, KP;            // patches per axis, moments, moments padded to 4
  int nr, nrp;               // rows (intra-patch positions) of one orientation; padded to 64
  int e0lo, ne0, elo, ne;    // offset box: first axis [e0lo, e0lo+ne0), others [elo, elo+ne)
  int nk0, nk1, nk2;         // lattice box sizes (k0 slowest)
  int k0lo, k1lo, k2lo;      // lattice box origins
  int L, padlo;              // padded moment lattice
};

// Cs[slot][p] and Cp[p][slot], slot = ((i0 + padlo) L + i1 + padlo) L + i2 + padlo.
__global__ void pad_moments_kernel(const double* __restrict__ mom, double* __restrict__ Cs, double* __restrict__ Cp,
                                   int ppa, int K, int KP, int L, int padlo) {
  int64_t idx = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (idx >= cube(L) * KP) return;
  const int p = int(idx / cube(L));
  const int64_t slot = idx % cube(L);
  const int a2 = int(slot % L) - padlo, a1 = int((slot / L) % L) - padlo, a0 = int(slot / (int64_t(L) * L)) - padlo;
  double v = 0.0;
  if (p < K && a0 >= 0 && a0 < ppa && a1 >= 0 && a1 < ppa && a2 >= 0 && a2 < ppa)
    v = mom[(int64_t(a0 * ppa + a1) * ppa + a2) * K + p];
  Cp[idx] = v;
  Cs[slot * KP + p] = v;
}

// nz[slot] = 1 when the patch at that slot of the padded lattice has a
// nonzero moment (0 for the padding): the far-field sums of a plan that
// skips empty patches pass over offsets whose source patches are all zero
// (an exact skip: those products add zero).
__global__ void pad_flags_kernel(const double* __restrict__ mom, int* __restrict__ nz, int ppa, int K, int L,
                                 int padlo) {
  const int64_t slot = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (slot >= cube(L)) return;
  const int a2 = int(slot % L) - padlo, a1 = int((slot / L) % L) - padlo, a0 = int(slot / (int64_t(L) * L)) - padlo;
  int any = 0;
  if (a0 >= 0 && a0 < ppa && a1 >= 0 && a1 < ppa && a2 >= 0 && a2 < ppa) {
    const double* m = mom + (int64_t(a0 * ppa + a1) * ppa + a2) * K;
    for (int p = 0; p < K; ++p) any |= m[p] != 0.0;
  }
  nz[slot] = any;
}

// A rows for the skeleton: r = ra * n + rb over the face plane of normal d;
// table Am[d][E][pc][r][4] (E = (E0, E1, E2) over the offset box, r < nrp),
// value D[d][E0 plane][ra + n E1][rb + n E2][p] when inside the table, else 0.
__global__ void skel_mfma_table_kernel(const double* __restrict__ D, double* __restrict__ Am, int n, int db,
                                       int P0b, int nplb, int Wb, int K, MfmaGeom mg) {
  const int npc = mg.KP / 4;
  const int64_t per_d = int64_t(mg.ne0) * mg.ne * mg.ne * npc * mg.nrp * 4;
  int64_t idx = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (idx >= 3 * per_d) return;
  int j = int(idx % 4);
  int64_t t = idx / 4;
  int r = int(t % mg.nrp); t /= mg.nrp;
  int pc = int(t % npc); t /= npc;
  int e2 = int(t % mg.ne); t /= mg.ne;
  int e1 = int(t % mg.ne); t /= mg.ne;
  int e0 = int(t % mg.ne0);
  int d = int(t / mg.ne0);
  int p = 4 * pc + j;
  int E0 = mg.e0lo + e0, E1 = mg.elo + e1, E2 = mg.elo + e2;
  int ra = r / n, rb = r % n;
  int jb = (n * E0 - P0b) / n;
  int ub = ra + n * E1 + db, vb = rb + n * E2 + db;
  double v = 0.0;
  if (r < mg.nr && p < K && jb >= 0 && jb < nplb && ub >= 0 && ub < Wb && vb >= 0 && vb < Wb)
    v = D[((((int64_t(d) * nplb + jb) * Wb + ub) * Wb) + vb) * K + p];
  Am[idx] = v;
}

// A rows for the coarse grid: rho = (r0, r1, r2) in [0, q)^3 (r < nrp); table
// Tm[E][pc][rho][4] = T[q E + rho][p] inside C(Omega_beta(0)), else 0.
__global__ void coarse_mfma_table_kernel(const double* __restrict__ Tt, double* __restrict__ Tm, int q, int db,
                                         int Wbc, int K, MfmaGeom mg) {
  const int npc = mg.KP / 4;
  const int64_t total = int64_t(mg.ne) * mg.ne * mg.ne * npc * mg.nrp * 4;
  int64_t idx = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (idx >= total) return;
  int j = int(idx % 4);
  int64_t t = idx / 4;
  int r = int(t % mg.nrp); t /= mg.nrp;
  int pc = int(t % npc); t /= npc;
  int e2 = int(t % mg.ne); t /= mg.ne;
  int e1 = int(t % mg.ne);
  int e0 = int(t / mg.ne);
  int p = 4 * pc + j;
  int rr[3] = {r / (q * q), (r / q) % q, r % q};
  int E[3] = {mg.elo + e0, mg.elo + e1, mg.elo + e2};
  int ob = db / NREF;
  int c[3];
  bool ok = r < mg.nr && p < K;
  for (int a = 0; a < 3; ++a) {
    c[a] = q * E[a] + rr[a] + ob;
    ok = ok && c[a] >= 0 && c[a] < Wbc;
  }
  Tm[idx] = ok ? Tt[((int64_t(c[0]) * Wbc + c[1]) * Wbc + c[2]) * K + p] : 0.0;
}

// A wave computes RT tiles of 16 rows x TILES column tiles (16 lattice
// points each); a
// block's WAVES waves form ROWW tiles of 16 rows by WAVES / ROWW column
// groups (waves on the same rows share the streamed table fragments through
// the CU's L1, waves on the same columns share the moments).  Chosen per
// contraction by measurement:
//   skeleton: 4 waves on 4 consecutive 64-row strips of the same 32
//     points, each wave 4 x 2 tiles (a table fragment serves two MFMAs, a
//     moments fragment four); faces of fewer than 256 rows (n = 8) take
//     16-row strips instead;
//   coarse grid: 8 waves on the same 32 rows, 16 points each (2 x 1 tiles);
//     at q = 2 (8 rows) 16 rows, which keeps more blocks in flight.
struct SkelTiling { static constexpr int TILES = 2, WAVES = 4, ROWW = 4, RT = 4; };
struct SkelTilingSmall { static constexpr int TILES = 2, WAVES = 4, ROWW = 4, RT = 1; };
struct CoarseTiling { static constexpr int TILES = 1, WAVES = 8, ROWW = 1, RT = 2; };
struct CoarseTilingSmall { static constexpr int TILES = 1, WAVES = 8, ROWW = 1, RT = 1; };
// lattice points and rows covered by one block (a wave: 16 RT rows)
template <class TL> constexpr int ann_block_cols() { return 16 * TL::TILES * (TL::WAVES / TL::ROWW); }
template <class TL> constexpr int ann_block_rows() { return 16 * TL::RT * TL::ROWW; }
// first row and first lattice point of wave `wave` in column block `cb`
template <class TL> __device__ __forceinline__ int ann_rowbase(int bx, int wave) {
  return bx * ann_block_rows<TL>() + (wave % TL::ROWW) * 16 * TL::RT;
}
template <class TL> __device__ __forceinline__ int ann_kbase(int cb, int wave) {
  return cb * ann_block_cols<TL>() + (wave / TL::ROWW) * 16 * TL::TILES;
}

// One wave: 16 rows x 16*ANN_TILES lattice points.  `d` selects the skeleton orientation, or is -1 for the
// coarse grid.  Offsets whose patches all fall outside the lattice for the
// wave's box of columns are skipped (a uniform test).
template <int ANN_TILES, bool PMAJOR, int RT>
__device__ __forceinline__ void annulus_mfma_tiles(const double* __restrict__ Am, const double* __restrict__ Cpad,
                                                   const int* __restrict__ nzf, const MfmaGeom& mg, int d,
                                                   int rowbase, int kbase, int e0b, int e0e,
                                                   f64x4 (&acc)[RT][ANN_TILES]) {
  const int lane = threadIdx.x & 63;
  const int rl = lane & 15, pj = lane >> 4;
  const int npc = mg.KP / 4;
  const int n12 = mg.nk1 * mg.nk2, nk = mg.nk0 * n12;
  const int L = mg.L, pad = mg.padlo;
  // strides of the lattice axes (normal or first, lower, upper) in the padded array
  int st0, st1, st2;
  if (d <= 0) { st0 = L * L; st1 = L; st2 = 1; }
  else if (d == 1) { st0 = L; st1 = L * L; st2 = 1; }
  else { st0 = 1; st1 = L * L; st2 = L; }
  int64_t boff[ANN_TILES], sl[ANN_TILES];
#pragma unroll
  for (int t = 0; t < ANN_TILES; ++t) {
    const int k = min(kbase + 16 * t + rl, nk - 1);
    const int a = mg.k0lo + k / n12, b = mg.k1lo + (k / mg.nk2) % mg.nk1, c = mg.k2lo + k % mg.nk2;
    const int64_t slot = (a + pad) * st0 + (b + pad) * st1 + (c + pad) * st2;
    sl[t] = slot;
    boff[t] = PMAJOR ? slot + int64_t(pj) * L * L * L : slot * mg.KP + pj;
#pragma unroll
    for (int rt = 0; rt < RT; ++rt) acc[rt][t] = f64x4{0.0, 0.0, 0.0, 0.0};
  }
  // lattice box of the wave's columns
  const int klast = min(kbase + 16 * ANN_TILES, nk) - 1;
  int a_lo = kbase / n12, a_hi = klast / n12;
  int b_lo = 0, b_hi = mg.nk1 - 1, c_lo = 0, c_hi = mg.nk2 - 1;
  if (a_lo == a_hi) {
    b_lo = (kbase / mg.nk2) % mg.nk1;
    b_hi = (klast / mg.nk2) % mg.nk1;
    if (b_lo == b_hi) { c_lo = kbase % mg.nk2; c_hi = klast % mg.nk2; }
  }
  a_lo += mg.k0lo; a_hi += mg.k0lo;
  b_lo += mg.k1lo; b_hi += mg.k1lo;
  c_lo += mg.k2lo; c_hi += mg.k2lo;
  const int ppa = mg.ppa;
  const int64_t per_d = int64_t(mg.ne0) * mg.ne * mg.ne * npc * mg.nrp * 4;
  const double* Ad = Am + (d > 0 ? d : 0) * per_d + (rowbase + rl) * 4 + pj;
  for (int e0 = e0b; e0 < e0e; ++e0) {
    const int E0 = mg.e0lo + e0;
    if (a_hi - E0 < 0 || a_lo - E0 > ppa - 1) continue;
    for (int e1 = 0; e1 < mg.ne; ++e1) {
      const int E1 = mg.elo + e1;
      if (b_hi - E1 < 0 || b_lo - E1 > ppa - 1) continue;
      for (int e2 = 0; e2 < mg.ne; ++e2) {
        const int E2 = mg.elo + e2;
        if (c_hi - E2 < 0 || c_lo - E2 > ppa - 1) continue;
        const int eoff = E0 * st0 + E1 * st1 + E2 * st2;
        if (nzf) {
          // skip the offset when every source patch of the wave's columns is zero
          int any = 0;
#pragma unroll
          for (int t = 0; t < ANN_TILES; ++t) any |= nzf[sl[t] - eoff];
          if (!__any(any)) continue;
        }
        const int64_t off = int64_t(eoff) * (PMAJOR ? 1 : mg.KP);
        const double* Ae = Ad + ((int64_t(e0) * mg.ne + e1) * mg.ne + e2) * npc * mg.nrp * 4;
        for (int pc = 0; pc < npc; ++pc) {
          // the RT row tiles' table fragments (16 rows apart) and the
          // moments fragments, each used RT or ANN_TILES times
          double a[RT];
#pragma unroll
          for (int rt = 0; rt < RT; ++rt) a[rt] = Ae[int64_t(pc) * mg.nrp * 4 + 64 * rt];
          const double* Cp = Cpad + (PMAJOR ? int64_t(4 * pc) * L * L * L : int64_t(4 * pc)) - off;
#pragma unroll
          for (int t = 0; t < ANN_TILES; ++t) {
            const double b = Cp[boff[t]];
#pragma unroll
            for (int rt = 0; rt < RT; ++rt)
              acc[rt][t] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[rt], b, acc[rt][t], 0, 0, 0);
          }
        }
      }
    }
  }
}

// One problem of a batched far-field launch: its far-field table (same
// layout across a class, values scaled by the problem's h), the lattice
// geometry that differs between the problems of a class, its padded moments
// and output, and its first column block (problems' column blocks are
// consecutive).
struct AnnProb {
  const double* tab;    // Am (skeleton) or Tm (coarse)
  const double* cpad;   // slot-major (skeleton) or mode-major (coarse) moments
  double* out;          // phi^B (skeleton) or F^H (coarse)
  int ppa, nk0, nk1, nk2, k0lo, k1lo, k2lo, L, padlo;
  int N, S_lo, Ns;
  int blk0;       // first block (along the launch's column-block axis)
  int ncb;        // column blocks of one offset chunk
  int esplit;     // offset chunks: blocks blk0 + c ncb + j take chunk c
  double* part;   // esplit > 1: partial sums [chunk][(d)][row][column]
  int64_t start;  // first thread of the problem in the reduction launch
  const int* nzf; // per lattice slot: nonzero moments (skips zero sources), or null (no skipping)
};
constexpr int ANN_PACK = 8;
struct AnnPack { AnnProb d[ANN_PACK]; int count; };
__global__ void ann_upload_kernel(AnnProb* __restrict__ dst, AnnPack pk) {
  if (int(threadIdx.x) < pk.count) dst[threadIdx.x] = pk.d[threadIdx.x];
}
// The problem owning column block b, and the class geometry completed with it.
__device__ __forceinline__ const AnnProb& ann_problem(const AnnProb* __restrict__ ap, int np, int b, MfmaGeom& mg) {
  int lo = 0, hi = np - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (ap[mid].blk0 <= b) lo = mid; else hi = mid - 1;
  }
  const AnnProb& A = ap[lo];
  mg.ppa = A.ppa;
  mg.nk0 = A.nk0; mg.nk1 = A.nk1; mg.nk2 = A.nk2;
  mg.k0lo = A.k0lo; mg.k1lo = A.k1lo; mg.k2lo = A.k2lo;
  mg.L = A.L; mg.padlo = A.padlo;
  return A;
}
// The e0 range [e0b, e0e) of offset chunk c of esplit over ne0 planes.
__device__ __forceinline__ void ann_chunk(int c, int esplit, int ne0, int* e0b, int* e0e) {
  *e0b = c * ne0 / esplit;
  *e0e = (c + 1) * ne0 / esplit;
}

// Skeleton: rows r = ra * n + rb of the face plane of normal d = blockIdx.z,
// columns k = (kd, ka, kb) in [0, ppa]^3 of the problem owning column block
// blockIdx.y; writes the far field into its phiB at every canonical
// skeleton node.
template <class TL>
__global__ void __launch_bounds__(64 * TL::WAVES) skeleton_annulus_mfma_kernel(const AnnProb* __restrict__ ap, int np,
                                                                             MfmaGeom mg, int n) {
  constexpr int ANN_TILES = TL::TILES, RT = TL::RT;
  const int d = blockIdx.z;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const AnnProb& A = ann_problem(ap, np, blockIdx.y, mg);
  const int N = A.N;
  double* __restrict__ phiB = A.out;
  const int local = int(blockIdx.y) - A.blk0, chunk = local / A.ncb;
  const int rowbase = ann_rowbase<TL>(blockIdx.x, wave);
  const int kbase = ann_kbase<TL>(local % A.ncb, wave);
  int e0b, e0e;
  ann_chunk(chunk, A.esplit, mg.ne0, &e0b, &e0e);
  f64x4 acc[RT][ANN_TILES];
  annulus_mfma_tiles<ANN_TILES, false, RT>(A.tab, A.cpad, A.nzf, mg, d, rowbase, kbase, e0b, e0e, acc);
  const int a0 = d == 0 ? 1 : 0, a1 = d == 2 ? 1 : 2, Np = N + 1;
  const int nk = mg.nk0 * mg.nk1 * mg.nk2;
  if (A.esplit > 1) {
    // partial sums of this offset chunk; skeleton_reduce_kernel adds them
    double* part = A.part + (int64_t(chunk) * 3 + d) * mg.nrp * nk;
#pragma unroll
    for (int rt = 0; rt < RT; ++rt)
#pragma unroll
      for (int t = 0; t < ANN_TILES; ++t) {
        const int k = kbase + 16 * t + (lane & 15);
        if (k >= nk) continue;
#pragma unroll
        for (int j = 0; j < 4; ++j)
          part[int64_t(rowbase + 16 * rt + 4 * j + (lane >> 4)) * nk + k] = acc[rt][t][j];
      }
    return;
  }
#pragma unroll
  for (int rt = 0; rt < RT; ++rt)
#pragma unroll
  for (int t = 0; t < ANN_TILES; ++t) {
    int k = kbase + 16 * t + (lane & 15);
    if (k >= nk) continue;
    int kd = k / (mg.nk1 * mg.nk2), ka = (k / mg.nk2) % mg.nk1, kb = k % mg.nk2;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      int r = rowbase + 16 * rt + 4 * j + (lane >> 4);
      if (r >= mg.nr) continue;
      int ra = r / n, rb = r % n;
      if ((a0 < d && ra == 0) || (a1 < d && rb == 0)) continue;     // not canonical
      int gg[3];
      gg[d] = n * kd;
      gg[a0] = n * ka + ra;
      gg[a1] = n * kb + rb;
      if (gg[a0] > N || gg[a1] > N) continue;
      phiB[(int64_t(gg[0]) * Np + gg[1]) * Np + gg[2]] = acc[rt][t][j];
    }
  }
}

// Coarse grid: rows rho in [0, q)^3, columns k over the lattice box of the
// problem owning column block blockIdx.y; adds the far field to its
// F[c = q k + rho] inside the support box.
template <class TL>
__global__ void __launch_bounds__(64 * TL::WAVES) coarse_annulus_mfma_kernel(const AnnProb* __restrict__ ap,
                                                                                      int np, MfmaGeom mg, int q) {
  constexpr int ANN_TILES = TL::TILES, RT = TL::RT;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const AnnProb& A = ann_problem(ap, np, blockIdx.y, mg);
  const int S_lo = A.S_lo, Ns = A.Ns;
  double* __restrict__ F = A.out;
  const int local = int(blockIdx.y) - A.blk0, chunk = local / A.ncb;
  const int rowbase = ann_rowbase<TL>(blockIdx.x, wave);
  const int kbase = ann_kbase<TL>(local % A.ncb, wave);
  int e0b, e0e;
  ann_chunk(chunk, A.esplit, mg.ne0, &e0b, &e0e);
  f64x4 acc[RT][ANN_TILES];
  annulus_mfma_tiles<ANN_TILES, true, RT>(A.tab, A.cpad, A.nzf, mg, -1, rowbase, kbase, e0b, e0e, acc);
  const int nk = mg.nk0 * mg.nk1 * mg.nk2;
  if (A.esplit > 1) {
    // partial sums of this offset chunk; coarse_reduce_kernel adds them
    double* part = A.part + int64_t(chunk) * mg.nrp * nk;
#pragma unroll
    for (int rt = 0; rt < RT; ++rt)
#pragma unroll
      for (int t = 0; t < ANN_TILES; ++t) {
        const int k = kbase + 16 * t + (lane & 15);
        if (k >= nk) continue;
#pragma unroll
        for (int j = 0; j < 4; ++j)
          part[int64_t(rowbase + 16 * rt + 4 * j + (lane >> 4)) * nk + k] = acc[rt][t][j];
      }
    return;
  }
#pragma unroll
  for (int rt = 0; rt < RT; ++rt)
#pragma unroll
  for (int t = 0; t < ANN_TILES; ++t) {
    int k = kbase + 16 * t + (lane & 15);
    if (k >= nk) continue;
    int k0 = mg.k0lo + k / (mg.nk1 * mg.nk2), k1 = mg.k1lo + (k / mg.nk2) % mg.nk1, k2 = mg.k2lo + k % mg.nk2;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      int r = rowbase + 16 * rt + 4 * j + (lane >> 4);
      if (r >= mg.nr) continue;
      int c0 = q * k0 + r / (q * q), c1 = q * k1 + (r / q) % q, c2 = q * k2 + r % q;
      if (c0 < S_lo || c0 >= S_lo + Ns || c1 < S_lo || c1 >= S_lo + Ns || c2 < S_lo || c2 >= S_lo + Ns) continue;
      F[(int64_t(c0 - S_lo) * Ns + (c1 - S_lo)) * Ns + (c2 - S_lo)] += acc[rt][t][j];
    }
  }
}

// Sums of the offset chunks of problems whose far-field sums were split
// (AnnProb::esplit > 1), chunk by chunk in order; one thread per (d, row,
// column) of every such problem.  Same outputs as the unsplit kernels.
__global__ void __launch_bounds__(256) skeleton_reduce_kernel(const AnnProb* __restrict__ ap, int np, int64_t total,
                                                              MfmaGeom mg, int n) {
  const int64_t gidx = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (gidx >= total) return;
  const AnnProb& A = flat_problem(ap, np, gidx);
  mg.nk0 = A.nk0; mg.nk1 = A.nk1; mg.nk2 = A.nk2;
  const int nk = mg.nk0 * mg.nk1 * mg.nk2;
  const int64_t idx = gidx - A.start;
  const int k = int(idx % nk), r = int((idx / nk) % mg.nr), d = int(idx / (int64_t(nk) * mg.nr));
  const int a0 = d == 0 ? 1 : 0, a1 = d == 2 ? 1 : 2, N = A.N, Np = N + 1;
  const int kd = k / (mg.nk1 * mg.nk2), ka = (k / mg.nk2) % mg.nk1, kb = k % mg.nk2;
  const int ra = r / n, rb = r % n;
  if ((a0 < d && ra == 0) || (a1 < d && rb == 0)) return;     // not canonical
  int gg[3];
  gg[d] = n * kd;
  gg[a0] = n * ka + ra;
  gg[a1] = n * kb + rb;
  if (gg[a0] > N || gg[a1] > N) return;
  double s = 0.0;
  for (int c = 0; c < A.esplit; ++c) s += A.part[((int64_t(c) * 3 + d) * mg.nrp + r) * nk + k];
  A.out[(int64_t(gg[0]) * Np + gg[1]) * Np + gg[2]] = s;
}

__global__ void __launch_bounds__(256) coarse_reduce_kernel(const AnnProb* __restrict__ ap, int np, int64_t total,
                                                            MfmaGeom mg, int q) {
  const int64_t gidx = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (gidx >= total) return;
  const AnnProb& A = flat_problem(ap, np, gidx);
  const int nk1 = A.nk1, nk2 = A.nk2, nk = A.nk0 * nk1 * nk2;
  const int64_t idx = gidx - A.start;
  const int k = int(idx % nk), r = int(idx / nk);
  const int S_lo = A.S_lo, Ns = A.Ns;
  const int k0 = A.k0lo + k / (nk1 * nk2), k1 = A.k1lo + (k / nk2) % nk1, k2 = A.k2lo + k % nk2;
  const int c0 = q * k0 + r / (q * q), c1 = q * k1 + (r / q) % q, c2 = q * k2 + r % q;
  if (c0 < S_lo || c0 >= S_lo + Ns || c1 < S_lo || c1 >= S_lo + Ns || c2 < S_lo || c2 >= S_lo + Ns) return;
  double s = 0.0;
  for (int c = 0; c < A.esplit; ++c) s += A.part[(int64_t(c) * mg.nrp + r) * nk + k];
  A.out[(int64_t(c0 - S_lo) * Ns + (c1 - S_lo)) * Ns + (c2 - S_lo)] += s;
}

// phi^B[g] = I(phi^H)(g) + sum_{i in S_alpha(g)} delta_i[g] (+ the annulus
// far field already in phiB when `annulus`) for every skeleton node g (taken
// once, on its lowest face-normal axis); also writes
// phi[g] = phi^B[g] + C2 h^2 f[g] (sec. 4.1 eqs. mlcfulldiscr,
// mcapplicationfulldiscr).  In two launches: skeleton_deltas_kernel (needs
// only the plane corrections, one thread per skeleton node slot) writes the
// sum of the delta_i to dsum[slot]; skeleton_finish_kernel (needs phi^H)
// adds the interpolation and the far field, so the first can run while the
// coarse solve is still going.  A slot is ((d planes + j) (N+1) + u) (N+1) + v:
// plane x_d = j n, in-plane coordinates u (axis a0) and v (axis a1).
template <typename T>
__global__ void __launch_bounds__(256) skeleton_deltas_kernel(const SkelProb<T>* __restrict__ pr, int np,
                                                              int64_t total, double* __restrict__ dsum) {
  const int64_t gidx = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (gidx >= total) return;
  const SkelProb<T>& pb = flat_problem(pr, np, gidx);
  const SkelGeom g = pb.g;
  const T* __restrict__ delta = pb.delta;
  const int N = g.N, n = g.n, Np = N + 1;
  const int planes = N / n + 1;
  const int64_t idx = gidx - pb.start;
  const int v = int(idx % Np), u = int((idx / Np) % Np), j = int((idx / (int64_t(Np) * Np)) % planes);
  const int d = int(idx / (int64_t(Np) * Np * planes));
  const int a0 = d == 0 ? 1 : 0, a1 = d == 2 ? 1 : 2;
  // canonical plane: no lower axis divisible by n
  if (a0 < d && u % n == 0) return;
  if (a1 < d && v % n == 0) return;
  int gg[3];
  gg[d] = j * n;
  gg[a0] = u;
  gg[a1] = v;
  // patches with g in Omega_alpha(i): n i - da <= g <= n i + n + da
  int lo[3], hi[3];
  for (int a = 0; a < 3; ++a) {
    int x = gg[a] - n - g.da;
    lo[a] = max(x >= 0 ? (x + n - 1) / n : -((-x) / n), 0);
    hi[a] = min((gg[a] + g.da) / n, g.ppa - 1);
  }
  const int Wa = g.Wa;
  double sd = 0.0;
  for (int i0 = lo[0]; i0 <= hi[0]; ++i0)
    for (int i1 = lo[1]; i1 <= hi[1]; ++i1)
      // four patches of the last axis at a time (loads issued together); a
      // slot past hi[2] repeats that patch and adds an exact zero
      for (int i2b = lo[2]; i2b <= hi[2]; i2b += 4) {
#pragma unroll
        for (int t2 = 0; t2 < 4; ++t2) {
          const bool valid = i2b + t2 <= hi[2];
          const int i2 = valid ? i2b + t2 : hi[2];
          const int r[3] = {gg[0] - n * i0, gg[1] - n * i1, gg[2] - n * i2};
          int pidx = (i0 * g.ppa + i1) * g.ppa + i2;
          if (pb.slot_of) pidx = pb.slot_of[pidx];
          const int jj = (r[d] - g.P0) / n;
          const double x = pidx < 0 ? 0.0 :
              double(delta[((((int64_t(pidx) * 3 + d) * g.npl + jj) * Wa + (r[a0] + g.da)) * Wa) + (r[a1] + g.da)]);
          sd += valid ? x : 0.0;
        }
      }
  dsum[gidx] = sd;
}

// The interpolation part, one block per tile of 4 rows u (one coarse row
// interval, u = 4 U0 .. 4 U0 + 3) by 64 columns v of one skeleton plane.  The
// tile's coarse samples (at most 2b + 2 rows by 16 + 2b + 2 columns) are
// loaded once into LDS, interpolated along v for each coarse row, then along
// u: the sum of each node is the same as tap by tap (along v first, then u).
constexpr int SKF_COLS = 64;
template <typename T>
__global__ void __launch_bounds__(256) skeleton_finish_kernel(const SkelProb<T>* __restrict__ pr, int np, LagW lw,
                                                              int annulus, const double* __restrict__ dsum) {
  __shared__ double C[10][SKF_COLS / NREF + 12];   // 2b + 2 <= 10 rows, 16 + 2b + 2 <= 26 columns
  __shared__ double R[10][SKF_COLS];
  const int64_t bid = blockIdx.x;
  // the problem owning this block: problem k owns blocks [bstart_k, bstart_{k+1})
  int lo = 0, hi = np - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (pr[mid].bstart <= bid) lo = mid; else hi = mid - 1;
  }
  const SkelProb<T>& pb = pr[lo];
  const SkelGeom g = pb.g;
  const int N = g.N, n = g.n, Np = N + 1, b = g.b;
  const int planes = N / n + 1, UT = N / NREF + 1, VT = (Np + SKF_COLS - 1) / SKF_COLS;
  int64_t t = bid - pb.bstart;
  const int vt = int(t % VT);
  t /= VT;
  const int U0 = int(t % UT);
  t /= UT;
  const int j = int(t % planes), d = int(t / planes);
  const int a0 = d == 0 ? 1 : 0, a1 = d == 2 ? 1 : 2;
  const int v0 = SKF_COLS * vt, vm = min(v0 + SKF_COLS - 1, N);
  // coarse rows: U0 - b .. U0 + b + 1 when a row u = 4 U0 + tu, tu > 0 is in
  // the grid, else U0 alone (u = N)
  const bool rows_i = NREF * U0 + 1 <= N;
  const int r_lo = rows_i ? U0 - b : U0, nr = rows_i ? 2 * b + 2 : 1;
  // coarse columns: the union over v0 .. vm of V0 (tv = 0) or V0 - b .. V0 + b + 1
  const int c_lo = (vm > v0 || v0 % NREF) ? v0 / NREF - b : v0 / NREF;
  const int c_hi = (vm % NREF) ? vm / NREF + b + 1 : (vm > v0 ? vm / NREF + b : vm / NREF);
  const int nc = c_hi - c_lo + 1;
  const int cd = j * n / NREF - g.O_lo;
  const double* __restrict__ phiH = pb.phiH;
  for (int q = threadIdx.x; q < nr * nc; q += blockDim.x) {
    const int rr = q / nc, cc = q % nc;
    int c[3];
    c[d] = cd;
    c[a0] = r_lo + rr - g.O_lo;
    c[a1] = c_lo + cc - g.O_lo;
    C[rr][cc] = phiH[(int64_t(c[0]) * g.No + c[1]) * g.No + c[2]];
  }
  __syncthreads();
  for (int q = threadIdx.x; q < nr * SKF_COLS; q += blockDim.x) {
    const int rr = q / SKF_COLS, x = q % SKF_COLS, v = v0 + x;
    double s = 0.0;
    if (v <= vm) {
      const int V0 = v / NREF, tv = v - NREF * V0;
      if (tv == 0) {
        s = C[rr][V0 - c_lo];
      } else {
        const double* wv = lw.w[tv];
        for (int kv = -b; kv <= b + 1; ++kv) s = fma(wv[kv + b], C[rr][V0 + kv - c_lo], s);
      }
    }
    R[rr][x] = s;
  }
  __syncthreads();
  const int x = threadIdx.x % SKF_COLS, u = NREF * U0 + int(threadIdx.x) / SKF_COLS, v = v0 + x;
  if (u > N || v > vm) return;
  // canonical plane: no lower axis divisible by n
  if (a0 < d && u % n == 0) return;
  if (a1 < d && v % n == 0) return;
  const int tu = u - NREF * U0;
  double val;
  if (tu == 0) {
    val = R[U0 - r_lo][x];
  } else {
    const double* wu = lw.w[tu];
    val = 0.0;
    for (int ku = -b; ku <= b + 1; ++ku) val = fma(wu[ku + b], R[U0 + ku - r_lo][x], val);
  }
  const int64_t slot = pb.start + ((int64_t(d) * planes + j) * Np + u) * Np + v;
  val += dsum[slot];
  int gg[3];
  gg[d] = j * n;
  gg[a0] = u;
  gg[a1] = v;
  const int64_t node = (int64_t(gg[0]) * Np + gg[1]) * Np + gg[2];
  double* __restrict__ phiB = pb.phiB;
  if (annulus) val += phiB[node];
  phiB[node] = val;
  // f at the node is zero when every patch whose closed box holds it is empty
  bool has_f = true;
  if (pb.live) {
    int lo[3], hi[3];
    for (int a = 0; a < 3; ++a) {
      hi[a] = min(gg[a] / n, g.ppa - 1);
      lo[a] = (gg[a] % n == 0 && gg[a] > 0) ? gg[a] / n - 1 : hi[a];
    }
    has_f = false;
    for (int i0 = lo[0]; i0 <= hi[0]; ++i0)
      for (int i1 = lo[1]; i1 <= hi[1]; ++i1)
        for (int i2 = lo[2]; i2 <= hi[2]; ++i2) has_f = has_f || pb.live[(i0 * g.ppa + i1) * g.ppa + i2] != 0;
  }
  pb.phi[node] = val + g.c2h2 * (has_f ? pb.f[node] : 0.0);
}

// --------------------------------------------- Dirichlet solves on MFMA ----
// The patch solve (sec. 4.1 eq. last_step_fulldiscr) diagonalises in the
// DST-I basis of length m = n - 1: u = S^-1 (S rhs / lambda) with
// S[k][j] = sin(pi (k+1)(j+1) / n) along each axis, S symmetric and
// S^-1 = (2/n) S.  A slab (m x m padded to 32 x 32) is transformed along
// both of its axes as S X S, along one as S X, each product on
// v_mfma_f64_16x16x4f64 (dirichlet_fused_kernel for 32^3-cell patches,
// dirichlet_mfma_kernel for smaller ones).
struct DirGeom {
  int n, npatch;   // patches of this launch: p0 .. p0 + npatch - 1 (one block each)
  double scale;    // 2/n
  Stencil st;
  int p0;
};

// Orders one wave's LDS writes before its later LDS reads by other lanes
// (the wave's LDS operations execute in order; this fences the compiler).
__device__ __forceinline__ void wave_sync_lds() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// D = A B for 32 x 32 row-major LDS matrices of stride 33 (one wave).  D may
// be A or B: every input is read before the first output is written.
__device__ __forceinline__ void mm32(const double* A, const double* B, double* D, int lane) {
  f64x4 acc[2][2];
#pragma unroll
  for (int it = 0; it < 2; ++it)
#pragma unroll
    for (int kt = 0; kt < 2; ++kt) acc[it][kt] = f64x4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int jj = 0; jj < 8; ++jj) {
    const int jrow = 4 * jj + (lane >> 4);
#pragma unroll
    for (int it = 0; it < 2; ++it) {
      const double a = A[(16 * it + (lane & 15)) * 33 + jrow];
#pragma unroll
      for (int kt = 0; kt < 2; ++kt) {
        const double b = B[jrow * 33 + 16 * kt + (lane & 15)];
        acc[it][kt] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[it][kt], 0, 0, 0);
      }
    }
  }
#pragma unroll
  for (int it = 0; it < 2; ++it)
#pragma unroll
    for (int kt = 0; kt < 2; ++kt)
#pragma unroll
      for (int r = 0; r < 4; ++r) D[(16 * it + 4 * r + (lane >> 4)) * 33 + 16 * kt + (lane & 15)] = acc[it][kt][r];
}

// For 32^3-cell patches (m = 31) the transform matrix pairs its rows k and
// 30 - k: S[30 - k][j] = (-1)^j S[k][j] (and S is symmetric).  A product
// S X then takes the even and the odd j apart over the 16 rows k < 16,
// E = sum over even j of S[k][j] X[j], O = the same over odd j (half the
// MFMAs of mm32), and gives row k = E + O and row 30 - k = E - O (row 15
// pairs with itself, its O being zero; row 31, padding, is zero).  X S
// likewise along the columns.  D may be the matrix that is not S.
__device__ __forceinline__ void mm32_sl(const double* S, const double* B, double* D, int lane) {
  f64x4 e[2], o[2];
#pragma unroll
  for (int kt = 0; kt < 2; ++kt) e[kt] = o[kt] = f64x4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int kk = 0; kk < 4; ++kk) {
    const int jj = 4 * kk + (lane >> 4);
    const double ae = S[(lane & 15) * 33 + 2 * jj], ao = S[(lane & 15) * 33 + 2 * jj + 1];
#pragma unroll
    for (int kt = 0; kt < 2; ++kt) {
      const double be = B[(2 * jj) * 33 + 16 * kt + (lane & 15)];
      const double bo = B[(2 * jj + 1) * 33 + 16 * kt + (lane & 15)];
      e[kt] = __builtin_amdgcn_mfma_f64_16x16x4f64(ae, be, e[kt], 0, 0, 0);
      o[kt] = __builtin_amdgcn_mfma_f64_16x16x4f64(ao, bo, o[kt], 0, 0, 0);
    }
  }
#pragma unroll
  for (int kt = 0; kt < 2; ++kt)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int k = 4 * r + (lane >> 4), col = 16 * kt + (lane & 15);
      const double ev = e[kt][r], ov = o[kt][r];
      D[k * 33 + col] = ev + ov;
      D[(k < 15 ? 30 - k : 31) * 33 + col] = k < 15 ? ev - ov : 0.0;
    }
}
__device__ __forceinline__ void mm32_sr(const double* B, const double* S, double* D, int lane) {
  f64x4 e[2], o[2];
#pragma unroll
  for (int it = 0; it < 2; ++it) e[it] = o[it] = f64x4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int kk = 0; kk < 4; ++kk) {
    const int jj = 4 * kk + (lane >> 4);
    const double se = S[(2 * jj) * 33 + (lane & 15)], so = S[(2 * jj + 1) * 33 + (lane & 15)];
#pragma unroll
    for (int it = 0; it < 2; ++it) {
      const double ae = B[(16 * it + (lane & 15)) * 33 + 2 * jj];
      const double ao = B[(16 * it + (lane & 15)) * 33 + 2 * jj + 1];
      e[it] = __builtin_amdgcn_mfma_f64_16x16x4f64(ae, se, e[it], 0, 0, 0);
      o[it] = __builtin_amdgcn_mfma_f64_16x16x4f64(ao, so, o[it], 0, 0, 0);
    }
  }
#pragma unroll
  for (int it = 0; it < 2; ++it)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int i = 16 * it + 4 * r + (lane >> 4), c = lane & 15;
      const double ev = e[it][r], ov = o[it][r];
      D[i * 33 + c] = ev + ov;
      D[i * 33 + (c < 15 ? 30 - c : 31)] = c < 15 ? ev - ov : 0.0;
    }
}

// D = A B for TW x TW row-major LDS matrices of stride TW + 1 (one wave):
// mm32, or for TW = 16 a single 16 x 16 MFMA tile over four k-steps.
__device__ __forceinline__ void mm16(const double* A, const double* B, double* D, int lane) {
  f64x4 acc = f64x4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int kk = 0; kk < 4; ++kk) {
    const int krow = 4 * kk + (lane >> 4);
    acc = __builtin_amdgcn_mfma_f64_16x16x4f64(A[(lane & 15) * 17 + krow], B[krow * 17 + (lane & 15)], acc, 0, 0, 0);
  }
#pragma unroll
  for (int r = 0; r < 4; ++r) D[(4 * r + (lane >> 4)) * 17 + (lane & 15)] = acc[r];
}
template <int TW> __device__ __forceinline__ void mm_tile(const double* A, const double* B, double* D, int lane) {
  if constexpr (TW == 32) mm32(A, B, D, lane);
  else mm16(A, B, D, lane);
}

// Smaller patches (n < 32: at most 15 slabs, half the fused kernel's waves
// idle) take three passes over an (n-1)^3 work array per patch instead:
//   0: slabs of fixed index 0: right-hand side h^2 f - (boundary terms), S X S
//   1: slabs of fixed index 1: S X along index 0, divide by the symbol,
//      S X again (times 2/n)
//   2: slabs of fixed index 0: S X S (times (2/n)^2), then
//      phi = u + C2 h^2 f on the patch interior
// Slabs (waves) per block of the Dirichlet passes.
constexpr int DIR_WAVES = 8;

// TW: the slab tile, 32 (n - 1 <= 31) or 16 (n - 1 <= 15: a quarter of the
// LDS and an eighth of the MFMAs of a padded 32 x 32 slab)
template <int PASS, int TW>
__global__ void __launch_bounds__(64 * DIR_WAVES) dirichlet_mfma_kernel(const ProbDesc* __restrict__ pd, int nprob,
                                                                        double* __restrict__ work, DirGeom g) {
  constexpr int LD = TW + 1, RG = 64 / TW, NR = TW * TW / 64;   // row stride, row groups, rows per lane
  __shared__ double Sm[TW * LD];
  __shared__ double Ls[DIR_WAVES][TW * LD];
  __shared__ double sn[2 * 32], cs[32];
  const int m = g.n - 1;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  // sin(pi a / n) for a < 2n and cos(pi (k+1) / n): every entry of the
  // transform matrix and of the symbol is one of these
  if (threadIdx.x < 2 * g.n) sn[threadIdx.x] = sinpi(double(threadIdx.x) / double(g.n));
  if (threadIdx.x < m) cs[threadIdx.x] = cospi(double(threadIdx.x + 1) / double(g.n));
  __syncthreads();
  for (int t = threadIdx.x; t < TW * TW; t += blockDim.x) {
    int k = t / TW, j = t % TW;
    Sm[k * LD + j] = (k < m && j < m) ? sn[((k + 1) * (j + 1)) % (2 * g.n)] : 0.0;
  }
  const int slab = blockIdx.x * DIR_WAVES + wave;     // over patches x m
  const int pw = slab / m, u = slab % m;               // pw: the patch's slot in the work array
  const int p = g.p0 + pw;
  const bool live = pw < g.npatch;
  const ProbDesc& D = pd[find_problem(pd, nprob, live ? p : 0)];
  const auto* f = gbl(D.f);
  const auto* phiB = gbl(D.phiB);
  auto* phi = gbl(D.phi);
  const int ppa = D.ppa, pl = p - D.patch0;
  const double h2 = D.h2;
  // slab element (row i, column j):
  //   passes 0, 2: node index (u, i, j); pass 1: node index (i, u, j)
  const int64_t M3 = int64_t(m) * m * m;
  auto off = [&](int i, int j) -> int64_t {
    if (PASS == 1) return int64_t(i) * m * m + int64_t(u) * m + j;
    return int64_t(u) * m * m + int64_t(i) * m + j;
  };
  double* wp = work + int64_t(pw) * M3;
  const int i0 = pl / (ppa * ppa), i1 = (pl / ppa) % ppa, i2 = pl % ppa;
  const int64_t Np = D.N + 1;
  const int64_t pbase = (int64_t(g.n) * i0) * Np * Np + int64_t(g.n) * i1 * Np + int64_t(g.n) * i2;
  double* L = Ls[wave];
  // lanes 0..TW-1 walk a row's columns, the RG lane groups take every RG-th
  // row; all NR rows of a lane are loaded before the first LDS write, so
  // the loads overlap
  const int jc = lane % TW, ih = lane / TW;
  double rows[NR];
#pragma unroll
  for (int r = 0; r < NR; ++r) {
    const int i = ih + RG * r;
    double v = 0.0;
    if (live && i < m && jc < m) {
      if constexpr (PASS == 0) {
        v = h2 * f[pbase + (int64_t(u + 1) * Np + (i + 1)) * Np + (jc + 1)];
      } else {
        v = wp[off(i, jc)];
      }
    }
    rows[r] = v;
  }
#pragma unroll
  for (int r = 0; r < NR; ++r) L[(ih + RG * r) * LD + jc] = rows[r];
  if constexpr (PASS == 0) {
    // boundary terms, only at nodes next to the patch boundary: the whole
    // slab if it is the first or last of its patch, else its ring of
    // 4(m-1) nodes.  The block's threads share the node lists of all its
    // slabs (a first or last slab has eight times the nodes of the others).
    __shared__ const double* sl_phiB[DIR_WAVES];
    __shared__ int64_t sl_base[DIR_WAVES], sl_Np[DIR_WAVES];
    __shared__ int sl_u[DIR_WAVES], sl_cnt[DIR_WAVES];
    if (lane == 0) {
      const bool end_slab = u == 0 || u == m - 1;
      sl_phiB[wave] = D.phiB;
      sl_base[wave] = pbase;
      sl_Np[wave] = Np;
      sl_u[wave] = u;
      sl_cnt[wave] = live ? (end_slab ? m * m : 4 * (m - 1)) : 0;
    }
    __syncthreads();   // every slab's L and the node lists
    int total = 0;
#pragma unroll
    for (int w = 0; w < DIR_WAVES; ++w) total += sl_cnt[w];
    for (int q0 = threadIdx.x; q0 < total; q0 += blockDim.x) {
      int w = 0, q = q0;
      while (q >= sl_cnt[w]) q -= sl_cnt[w++];
      const int uw = sl_u[w];
      int i, j;
      if (uw == 0 || uw == m - 1) {
        i = q / m;
        j = q % m;
      } else if (q < 2 * m) {
        i = q < m ? 0 : m - 1;
        j = q % m;
      } else {
        const int r = q - 2 * m;
        i = 1 + r / 2;
        j = (r & 1) ? m - 1 : 0;
      }
      const auto* phiBw = gbl(sl_phiB[w]);
      const int64_t base = sl_base[w], Npw = sl_Np[w];
      const int l0 = uw + 1, l1 = i + 1, l2 = j + 1;
      // every neighbour is a node of the patch box, so all 27 loads are
      // issued together; those off the boundary (whose phi^B is not
      // defined) are selected away, the boundary ones summed in order
      double corr = 0.0;
#pragma unroll
      for (int s0 = -1; s0 <= 1; ++s0)
#pragma unroll
        for (int s1 = -1; s1 <= 1; ++s1)
#pragma unroll
          for (int s2 = -1; s2 <= 1; ++s2) {
            const int k0 = l0 + s0, k1 = l1 + s1, k2 = l2 + s2;
            const bool bnd = k0 == 0 || k0 == g.n || k1 == 0 || k1 == g.n || k2 == 0 || k2 == g.n;
            const int nz = (s0 != 0) + (s1 != 0) + (s2 != 0);
            const double x = phiBw[base + (int64_t(k0) * Npw + k1) * Npw + k2];
            corr = fma(bnd ? g.st.b[nz] : 0.0, bnd ? x : 0.0, corr);
          }
      Ls[w][i * LD + j] -= corr;
    }
  }
  __syncthreads();   // Sm; from here on each wave touches only its own slab
  if constexpr (PASS == 1) {
    mm_tile<TW>(Sm, L, L, lane);          // forward along index 0
    wave_sync_lds();
    for (int i = ih; i < TW; i += RG) {   // divide by the symbol at (k0, k1, k2) = (i, u, jc)
      double v = 0.0;
      if (i < m && jc < m) {
        const double c0 = cs[i], c1 = cs[u], c2 = cs[jc];
        const double lam = g.st.b[0] + 2.0 * g.st.b[1] * (c0 + c1 + c2) +
                           4.0 * g.st.b[2] * (c0 * c1 + c0 * c2 + c1 * c2) + 8.0 * g.st.b[3] * c0 * c1 * c2;
        v = L[i * LD + jc] / lam;
      }
      L[i * LD + jc] = v;
    }
    wave_sync_lds();
    mm_tile<TW>(Sm, L, L, lane);          // inverse along index 0
  } else {
    mm_tile<TW>(Sm, L, L, lane);          // along index 1 (rows)
    wave_sync_lds();
    mm_tile<TW>(L, Sm, L, lane);          // along index 2 (columns)
  }
  wave_sync_lds();
  if (!live) return;
  const double sc = PASS == 0 ? 1.0 : (PASS == 1 ? g.scale : g.scale * g.scale);
  for (int i = ih; i < m; i += RG) {
    if (jc >= m) continue;
    const double v = sc * L[i * LD + jc];
    if constexpr (PASS == 2) {
      const int64_t node = pbase + (int64_t(u + 1) * Np + (i + 1)) * Np + (jc + 1);
      phi[node] = v + D.c2h2 * f[node];
    } else {
      wp[off(i, jc)] = v;
    }
  }
}


// One block of 16 waves per patch: the patch's (n-1)^3 values stay on the
// chip (wave w holds the slabs of index 0 equal to w and w + 16 in
// registers), so no work array goes through HBM.
//   A: per slab u: right-hand side h^2 f - (boundary terms), S X S
//   B: along index 0, in four chunks of 8 rows of index 1: the slabs' rows
//      are staged in LDS as a 32 x 256 matrix (index 0 by (index 1, index 2)),
//      each wave takes 16 columns: S X, divide by the symbol, S X (times 2/n)
//   C: per slab u: S X S (times (2/n)^2), phi = u + C2 h^2 f
constexpr int DIRF_WAVES = 16;
constexpr int DIRF_TS = 260;   // row stride of the staging matrix (256 columns + 4)
static_assert(32 * DIRF_TS <= DIRF_WAVES * 32 * 33, "staging matrix must fit in the slab buffers");
__global__ void __launch_bounds__(64 * DIRF_WAVES) dirichlet_fused_kernel(const ProbDesc* __restrict__ pd, int nprob,
                                                                         DirGeom g,
                                                                         const int* __restrict__ patch_live) {
  __shared__ double Sm[32 * 33];
  __shared__ double Ls[DIRF_WAVES][32 * 33];
  __shared__ double sn[2 * 32], cs[32];
  __shared__ const double* sl_phiB[DIRF_WAVES];
  __shared__ int64_t sl_base[DIRF_WAVES], sl_Np[DIRF_WAVES];
  __shared__ int sl_u[DIRF_WAVES], sl_cnt[DIRF_WAVES];
  const int m = g.n - 1;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  if (threadIdx.x < 2 * g.n) sn[threadIdx.x] = sinpi(double(threadIdx.x) / double(g.n));
  if (threadIdx.x < m) cs[threadIdx.x] = cospi(double(threadIdx.x + 1) / double(g.n));
  __syncthreads();
  for (int t = threadIdx.x; t < 32 * 32; t += blockDim.x) {
    const int k = t / 32, j = t % 32;
    Sm[k * 33 + j] = (k < m && j < m) ? sn[((k + 1) * (j + 1)) % (2 * g.n)] : 0.0;
  }
  const int p = g.p0 + int(blockIdx.x);
  const ProbDesc& D = pd[find_problem(pd, nprob, p)];
  const auto* f = gbl(D.f);
  auto* phi = gbl(D.phi);
  const int ppa = D.ppa, pl = p - D.patch0;
  const double h2 = D.h2;
  // a patch known to be empty (every node of its closed box zero) reads no f
  const bool has_f = !patch_live || patch_live[p];
  const int i0 = pl / (ppa * ppa), i1 = (pl / ppa) % ppa, i2 = pl % ppa;
  const int64_t Np = D.N + 1;
  const int64_t pbase = (int64_t(g.n) * i0) * Np * Np + int64_t(g.n) * i1 * Np + int64_t(g.n) * i2;
  double* L = Ls[wave];
  // lanes 0..31 walk a row's columns, the two half-waves take alternate rows
  const int jc = lane & 31, ih = lane >> 5;
  double xs[2][16];
  // ---- A: right-hand side and the transforms along indices 1 and 2
#pragma unroll
  for (int sl = 0; sl < 2; ++sl) {
    const int u = wave + DIRF_WAVES * sl;
    const bool live = u < m;
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int i = ih + 2 * r;
      double v = 0.0;
      if (has_f && live && i < m && jc < m) v = h2 * f[pbase + (int64_t(u + 1) * Np + (i + 1)) * Np + (jc + 1)];
      xs[sl][r] = v;
    }
#pragma unroll
    for (int r = 0; r < 16; ++r) L[(ih + 2 * r) * 33 + jc] = xs[sl][r];
    // boundary terms at the nodes next to the patch boundary (the whole slab
    // for the first and last slab, else its ring), shared by the block's threads
    if (lane == 0) {
      const bool end_slab = u == 0 || u == m - 1;
      sl_phiB[wave] = D.phiB;
      sl_base[wave] = pbase;
      sl_Np[wave] = Np;
      sl_u[wave] = u;
      sl_cnt[wave] = live ? (end_slab ? m * m : 4 * (m - 1)) : 0;
    }
    __syncthreads();   // every slab's L and the node lists (and Sm)
    int total = 0;
#pragma unroll
    for (int w = 0; w < DIRF_WAVES; ++w) total += sl_cnt[w];
    for (int q0 = threadIdx.x; q0 < total; q0 += blockDim.x) {
      int w = 0, q = q0;
      while (q >= sl_cnt[w]) q -= sl_cnt[w++];
      const int uw = sl_u[w];
      int i, j;
      if (uw == 0 || uw == m - 1) {
        i = q / m;
        j = q % m;
      } else if (q < 2 * m) {
        i = q < m ? 0 : m - 1;
        j = q % m;
      } else {
        const int r = q - 2 * m;
        i = 1 + r / 2;
        j = (r & 1) ? m - 1 : 0;
      }
      const auto* phiBw = gbl(sl_phiB[w]);
      const int64_t base = sl_base[w], Npw = sl_Np[w];
      const int l0 = uw + 1, l1 = i + 1, l2 = j + 1;
      // all 27 neighbours are nodes of the patch box: the loads of one
      // plane of neighbours are issued together, those off the boundary
      // selected away, the boundary ones summed in order
      double corr = 0.0;
#pragma unroll 1
      for (int s0 = -1; s0 <= 1; ++s0)
#pragma unroll
        for (int s1 = -1; s1 <= 1; ++s1)
#pragma unroll
          for (int s2 = -1; s2 <= 1; ++s2) {
            const int k0 = l0 + s0, k1 = l1 + s1, k2 = l2 + s2;
            const bool bnd = k0 == 0 || k0 == g.n || k1 == 0 || k1 == g.n || k2 == 0 || k2 == g.n;
            const int nz = (s0 != 0) + (s1 != 0) + (s2 != 0);
            const double x = phiBw[base + (int64_t(k0) * Npw + k1) * Npw + k2];
            corr = fma(bnd ? g.st.b[nz] : 0.0, bnd ? x : 0.0, corr);
          }
      Ls[w][i * 33 + j] -= corr;
    }
    __syncthreads();   // from here on each wave touches only its own slab
    mm32_sl(Sm, L, L, lane);              // along index 1 (rows)
    wave_sync_lds();
    mm32_sr(L, Sm, L, lane);              // along index 2 (columns)
    wave_sync_lds();
#pragma unroll
    for (int r = 0; r < 16; ++r) xs[sl][r] = L[(ih + 2 * r) * 33 + jc];
  }
  // ---- B: along index 0, 8 rows of index 1 at a time
  double* T = &Ls[0][0];
#pragma unroll 1
  for (int c = 0; c < 4; ++c) {
    __syncthreads();   // the slab buffers are free (A done, or the previous chunk read back)
#pragma unroll
    for (int sl = 0; sl < 2; ++sl) {
      const int u = wave + DIRF_WAVES * sl;   // 0 .. 31: every row of T
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int i = ih + 2 * r;
        if ((i >> 3) == c) T[u * DIRF_TS + (i & 7) * 32 + jc] = xs[sl][r];
      }
    }
    __syncthreads();
    // this wave's 16 columns: (index 1, index 2) = (8 c + col / 32, col % 32)
    const int col = 16 * wave + (lane & 15);
    const int ii = 8 * c + col / 32, j2 = col % 32;
#pragma unroll
    for (int pass = 0; pass < 2; ++pass) {
      // S times the wave's columns, rows k < 16 from the even and odd u apart
      f64x4 e = f64x4{0.0, 0.0, 0.0, 0.0}, o = e;
#pragma unroll
      for (int kk = 0; kk < 4; ++kk) {
        const int jj = 4 * kk + (lane >> 4);
        const double ae = Sm[(lane & 15) * 33 + 2 * jj], ao = Sm[(lane & 15) * 33 + 2 * jj + 1];
        const double be = T[(2 * jj) * DIRF_TS + col], bo = T[(2 * jj + 1) * DIRF_TS + col];
        e = __builtin_amdgcn_mfma_f64_16x16x4f64(ae, be, e, 0, 0, 0);
        o = __builtin_amdgcn_mfma_f64_16x16x4f64(ao, bo, o, 0, 0, 0);
      }
      wave_sync_lds();   // every lane's reads of its columns before they are overwritten
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int k0 = 4 * r + (lane >> 4);
        const double y[2] = {e[r] + o[r], e[r] - o[r]};
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          // row k0 (E + O) and its pair 30 - k0 (E - O); row 15's pair is row 31, zero
          const int k = h == 0 ? k0 : (k0 < 15 ? 30 - k0 : 31);
          double v = 0.0;
          if (pass == 0) {
            // divide by the symbol at (k0, k1, k2) = (k, ii, j2)
            if (k < m && ii < m && j2 < m) {
              const double c0 = cs[k], c1 = cs[ii], c2 = cs[j2];
              const double lam = g.st.b[0] + 2.0 * g.st.b[1] * (c0 + c1 + c2) +
                                 4.0 * g.st.b[2] * (c0 * c1 + c0 * c2 + c1 * c2) + 8.0 * g.st.b[3] * c0 * c1 * c2;
              v = y[h] / lam;
            }
          } else if (k < m) {
            v = g.scale * y[h];
          }
          T[k * DIRF_TS + col] = v;
        }
      }
      wave_sync_lds();
    }
    __syncthreads();
#pragma unroll
    for (int sl = 0; sl < 2; ++sl) {
      const int u = wave + DIRF_WAVES * sl;
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int i = ih + 2 * r;
        if ((i >> 3) == c) xs[sl][r] = T[u * DIRF_TS + (i & 7) * 32 + jc];
      }
    }
  }
  __syncthreads();   // the staging matrix is read back before the slab buffers are reused
  // ---- C: the inverse transforms along indices 1 and 2, and phi
  const double sc = g.scale * g.scale;
#pragma unroll
  for (int sl = 0; sl < 2; ++sl) {
    const int u = wave + DIRF_WAVES * sl;
#pragma unroll
    for (int r = 0; r < 16; ++r) L[(ih + 2 * r) * 33 + jc] = xs[sl][r];
    wave_sync_lds();
    mm32_sl(Sm, L, L, lane);
    wave_sync_lds();
    mm32_sr(L, Sm, L, lane);
    wave_sync_lds();
    if (u < m) {
      for (int i = ih; i < m; i += 2) {
        if (jc >= m) continue;
        const double v = sc * L[i * 33 + jc];
        const int64_t node = pbase + (int64_t(u + 1) * Np + (i + 1)) * Np + (jc + 1);
        phi[node] = v + D.c2h2 * (has_f ? f[node] : 0.0);
      }
    }
    wave_sync_lds();   // the slab's reads before the next slab overwrites L
  }
}

}  // namespace mlc
