// Charges given analytically as sums of radial terms (mlc_solve_analytic):
// their samples on the grid nodes, and the Legendre coefficients of every
// patch by composite Gauss-Legendre integration (sec. 4.1 step 1: Gauss
// integration when f is specified analytically, Boole's rule when it is known
// only on the nodes).
#pragma once
#include "../../include/mlc.h"
#include "common.h"
#include "setup_kernels.h"

namespace mlc {

struct RadialTerm {
  double c[3], R, w, param;
  int profile, pad;
};
struct RadialCharge {
  RadialTerm t[MLC_MAX_RADIAL_TERMS];
  int count;
};

// weight-free profile of one term at r = |x - c| / R (zero for r >= 1)
__device__ __forceinline__ double radial_profile(int kind, double r, double param) {
  if (r >= 1.0) return 0.0;
  if (kind == MLC_PROFILE_BUMP) {
    const double u = 1.0 - r * r, u2 = u * u;
    return u2 * u2;
  }
  const double u = r - r * r;
  if (kind == MLC_PROFILE_SMOOTH) {
    const double u2 = u * u;
    return u2 * u2;
  }
  const double s = sin(0.5 * param * r);
  return u * u * s * s;
}

__device__ __forceinline__ double term_value(const RadialTerm& t, double x0, double x1, double x2) {
  const double d0 = x0 - t.c[0], d1 = x1 - t.c[1], d2 = x2 - t.c[2];
  return t.w * radial_profile(t.profile, sqrt(d0 * d0 + d1 * d1 + d2 * d2) / t.R, t.param);
}

// f at the (N+1)^3 nodes g h (C order, axis 2 fastest)
__global__ void analytic_fill_kernel(RadialCharge q, int N, double h, double* __restrict__ f) {
  const int64_t Np = N + 1;
  // grid-stride: (N+1)^3 can exceed the threads of one launch
  for (int64_t idx = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; idx < Np * Np * Np;
       idx += int64_t(gridDim.x) * blockDim.x) {
    const int g2 = int(idx % Np), g1 = int((idx / Np) % Np), g0 = int(idx / (Np * Np));
    double v = 0.0;
    for (int k = 0; k < q.count; ++k) v += term_value(q.t[k], g0 * h, g1 * h, g2 * h);
    f[idx] = v;
  }
}

// Composite Gauss-Legendre rule: gp points per cell, nodes xi and weights
// om on [-1, 1].
struct GaussRule {
  int gp;
  double xi[4], om[4];
};

constexpr int GAUSS_THREADS = 128;   // one thread per point column: n gp <= 32 * 4

// c_p = R^{3/2} sum over the patch's Gauss points of W f qhat_p(t), one block
// per patch.  Thread j holds the points' column along the fastest axis (axis
// 2 index j) and accumulates S[a0][a1] = sum_{j0, j1} W_j0 qhat_a0(t_j0)
// W_j1 qhat_a1(t_j1) f over the two slower axes; mode (a0, a1, a2) then takes
// S[a0][a1] W_j qhat_a2(t_j) summed over the threads (wave shuffles, then the
// block's waves in order).  Terms whose support misses the patch are skipped.
template <int P>
__global__ void __launch_bounds__(GAUSS_THREADS) gauss_moments_kernel(const ProbDesc* __restrict__ pd, int nprob,
                                                                      int n, RadialCharge q, GaussRule rule,
                                                                      ModeList modes, double* __restrict__ mom,
                                                                      int p0) {
  constexpr int NW = GAUSS_THREADS / 64;
  __shared__ double Bw[P][GAUSS_THREADS];   // W_j qhat_a(t_j) at the patch's Gauss coordinates
  __shared__ double off[GAUSS_THREADS];     // their offsets from the patch corner, in units of h
  __shared__ int live[MLC_MAX_RADIAL_TERMS];
  __shared__ int nlive;
  __shared__ double red[NW][KMAX];
  const int p = p0 + blockIdx.x;
  const ProbDesc& D = pd[find_problem(pd, nprob, p)];
  const int ppa = D.ppa, pl = p - D.patch0;
  const int i0 = pl / (ppa * ppa), i1 = (pl / ppa) % ppa, i2 = pl % ppa;
  const double h = sqrt(D.h2);
  const int npt = n * rule.gp, tid = threadIdx.x;
  for (int j = tid; j < npt; j += blockDim.x) {
    const int c = j / rule.gp, k = j % rule.gp;
    const double u = c + 0.5 * (1.0 + rule.xi[k]);         // offset in cells
    const double t = (u - 0.5 * n) / (0.5 * n);
    const double w = rule.om[k] / n;                      // weight on [-1, 1]: om (2/n) / 2
    off[j] = u;
#pragma unroll
    for (int a = 0; a < P; ++a) Bw[a][j] = w * qhat(a, t);
  }
  if (tid == 0) {
    // terms whose ball meets the patch box
    const double lo[3] = {double(n) * i0 * h, double(n) * i1 * h, double(n) * i2 * h};
    int cnt = 0;
    for (int k = 0; k < q.count; ++k) {
      double d2 = 0.0;
      for (int d = 0; d < 3; ++d) {
        const double a = lo[d], b = lo[d] + n * h, x = q.t[k].c[d];
        const double e = x < a ? a - x : (x > b ? x - b : 0.0);
        d2 += e * e;
      }
      if (d2 < q.t[k].R * q.t[k].R) live[cnt++] = k;
    }
    nlive = cnt;
  }
  __syncthreads();
  double S[P][P];
#pragma unroll
  for (int a = 0; a < P; ++a)
#pragma unroll
    for (int b = 0; b < P; ++b) S[a][b] = 0.0;
  const int nl = nlive;
  const double x2 = (double(n) * i2 + (tid < npt ? off[tid] : 0.0)) * h;
  if (tid < npt && nl > 0) {
    for (int j0 = 0; j0 < npt; ++j0) {
      const double x0 = (double(n) * i0 + off[j0]) * h;
      double T[P];
#pragma unroll
      for (int b = 0; b < P; ++b) T[b] = 0.0;
      for (int j1 = 0; j1 < npt; ++j1) {
        const double x1 = (double(n) * i1 + off[j1]) * h;
        double v = 0.0;
        for (int k = 0; k < nl; ++k) v += term_value(q.t[live[k]], x0, x1, x2);
#pragma unroll
        for (int b = 0; b < P; ++b) T[b] += Bw[b][j1] * v;
      }
#pragma unroll
      for (int a = 0; a < P; ++a)
#pragma unroll
        for (int b = 0; b < P; ++b) S[a][b] += Bw[a][j0] * T[b];
    }
  }
  const int wave = tid >> 6, lane = tid & 63;
  for (int k = 0; k < modes.K; ++k) {
    const int a0 = modes.p[k][0], a1 = modes.p[k][1], a2 = modes.p[k][2];
    double s = 0.0;
#pragma unroll
    for (int a = 0; a < P; ++a)
#pragma unroll
      for (int b = 0; b < P; ++b)
        if (a == a0 && b == a1) s = S[a][b];
    double v = tid < npt ? s * Bw[a2][tid] : 0.0;
    for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
    if (lane == 0) red[wave][k] = v;
  }
  __syncthreads();
  for (int k = tid; k < modes.K; k += blockDim.x) {
    double v = 0.0;
    for (int w = 0; w < NW; ++w) v += red[w][k];
    mom[int64_t(p) * modes.K + k] = D.R15 * v;
  }
}

}  // namespace mlc
