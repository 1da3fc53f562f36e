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
#include "fft_reg.h"

namespace mlc {

template <typename T, int M>
__global__ void __launch_bounds__(256) conv_xdft_kernel(const ProbDesc* __restrict__ pd, int nprob, int n, int P,
                                                        cplx<T>* __restrict__ X, double* __restrict__ mpart,
                                                        const int* __restrict__ live,
                                                        const int* __restrict__ patch_of, int p0) {
  constexpr int Mh = M / 2 + 1;
  __shared__ T q[SMAX * SMAX];
  __shared__ cplx<T> tw[M];
  __shared__ double fd[SMAX * SMAX];   // the plane of f as given (moment sums)
  __shared__ double Bw[PMAX][SMAX];    // Boole weight x qhat_a at each node, a < P
  __shared__ double gx[PMAX][SMAX];    // x-contracted moment sums per row
  const int S = n + 1;
  // slot: this patch's place in the per-patch buffers (its own index unless
  // the plan keeps only its live patches, listed in patch_of)
  const int slot = p0 + blockIdx.y, sz = blockIdx.x;
  const int p = patch_of ? patch_of[slot] : slot;
  if (live && !live[p]) {
    // an empty patch: zero moment sums; its x-DFT is never read
    if (int(threadIdx.x) < P * P) mpart[(int64_t(slot) * (n + 1) + sz) * (P * P) + threadIdx.x] = 0.0;
    return;
  }
  const ProbDesc& D = pd[find_problem(pd, nprob, p)];
  const auto* f = gbl(D.f);
  const int ppa = D.ppa, pl = p - D.patch0;
  const int i0 = pl / (ppa * ppa), i1 = (pl / ppa) % ppa, i2 = pl % ppa;
  const int64_t Np = D.N + 1;
  const double cz = (sz == 0 || sz == n) ? 0.5 : 1.0;
  const auto* fp = f + (int64_t(n) * i0 + sz) * Np * Np + int64_t(n) * i1 * Np + int64_t(n) * i2;
  for (int t = threadIdx.x; t < S * S; t += blockDim.x) {
    int sy = t / S, sx = t % S;
    double c = cz * ((sy == 0 || sy == n) ? 0.5 : 1.0) * ((sx == 0 || sx == n) ? 0.5 : 1.0);
    const double v = fp[sy * Np + sx];
    fd[t] = v;
    q[t] = T(c * v);
  }
  for (int t = threadIdx.x; t < P * S; t += blockDim.x) {
    int a = t / S, j = t % S;
    Bw[a][j] = boole_w(j, n) * qhat(a, (j - 0.5 * n) / (0.5 * n));
  }
  fill_twiddles(tw, M);
  __syncthreads();
  // Legendre moment sums of this plane (sec. 4.1, step 1), x axis first
  for (int t = threadIdx.x; t < P * S; t += blockDim.x) {
    const int a = t / S, sy = t % S;
    double acc = 0.0;
    for (int sx = 0; sx < S; ++sx) acc += Bw[a][sx] * fd[sy * S + sx];
    gx[a][sy] = acc;
  }
  // X[kx][sy] = sum_sx q[sy][sx] w^(kx sx): each thread a 3 x 4 register
  // tile (kx = kg + NK a, sy = sg + NY b), so one twiddle read from LDS serves
  // four products and one sample three (3 x 4 leaves fewer threads idle than
  // 4 x 4: 243 of 256 at M = 160, n = 32)
  constexpr int TK = 3, TY = 4;
  constexpr int NK = (Mh + TK - 1) / TK;
  const int NY = (S + TY - 1) / TY;
  cplx<T>* out = X + (int64_t(slot) * Mh * S + sz) * S;
  for (int o = threadIdx.x; o < NK * NY; o += blockDim.x) {
    const int kg = o / NY, sg = o % NY;
    int kx[TK], idx[TK], sy[TY];
#pragma unroll
    for (int a = 0; a < TK; ++a) {
      kx[a] = min(kg + NK * a, Mh - 1);   // clamped lanes compute a duplicate, not stored
      idx[a] = 0;
    }
#pragma unroll
    for (int b = 0; b < TY; ++b) sy[b] = min(sg + NY * b, S - 1);
    T ar[TK][TY], ai[TK][TY];
#pragma unroll
    for (int a = 0; a < TK; ++a)
#pragma unroll
      for (int b = 0; b < TY; ++b) ar[a][b] = ai[a][b] = T(0);
    for (int sx = 0; sx < S; ++sx) {
      cplx<T> w[TK];
      T r[TY];
#pragma unroll
      for (int a = 0; a < TK; ++a) w[a] = tw[idx[a]];
#pragma unroll
      for (int b = 0; b < TY; ++b) r[b] = q[sy[b] * S + sx];
#pragma unroll
      for (int a = 0; a < TK; ++a)
#pragma unroll
        for (int b = 0; b < TY; ++b) {
          ar[a][b] += r[b] * w[a].x;
          ai[a][b] += r[b] * w[a].y;
        }
#pragma unroll
      for (int a = 0; a < TK; ++a) {
        idx[a] += kx[a];
        if (idx[a] >= M) idx[a] -= M;
      }
    }
#pragma unroll
    for (int a = 0; a < TK; ++a)
#pragma unroll
      for (int b = 0; b < TY; ++b)
        if (kg + NK * a < Mh && sg + NY * b < S) out[int64_t(kx[a]) * S * S + sy[b]] = {ar[a][b], ai[a][b]};
  }
  __syncthreads();
  if (int(threadIdx.x) < P * P) {
    const int a1 = threadIdx.x / P, a2 = threadIdx.x % P;
    double acc = 0.0;
    for (int sy = 0; sy < S; ++sy) acc += Bw[a1][sy] * gx[a2][sy];
    mpart[(int64_t(slot) * S + sz) * (P * P) + threadIdx.x] = acc;
  }
}

// Lines transformed together per batch (one thread per (line, pass index)).
template <typename T, int M> struct Batch {
  static constexpr int R1 = Split<M>::R1, R2 = Split<M>::R2;
  static constexpr int RMAX = R1 > R2 ? R1 : R2;
  static constexpr int CB = 256 / RMAX;
  static constexpr int LC = 64 / RMAX;   // columns per wave step (conv_yz column phase)
  // odd padded line stride of the exchange buffer
  static constexpr int XL = (XLayout<M>::LINE % 2) ? XLayout<M>::LINE : XLayout<M>::LINE + 1;
  // conv_yz: line stride = 8 (mod 32) complex elements, so that the four
  // columns of a wave step land on disjoint LDS bank sets in its widest
  // exchange (the forward pass writes)
  static constexpr int XLYZ = XLayout<M>::LINE + ((8 - XLayout<M>::LINE % 32) + 32) % 32;
};
// conv_out holds the (kx, y) plane in LDS, so one block fills a CU.  Each
// wave transforms its own lines (LW per step) through a private slice of
// the exchange buffer, with no block barriers between FFT passes.
template <typename T, int M, bool MULTI = true> struct OutBatch {
  static constexpr bool F32 = sizeof(T) == 4;
  // (12-wave single-plane blocks, which fit three waves per SIMD, measured
  // slower: 128^3 output pass 0.58 -> 0.94 ms; 6-wave fp64 blocks too:
  // 256^3 fp64 output pass 6.0 -> 12.9 ms per solve)
  static constexpr int NT = F32 ? 512 : 256;
  static constexpr int LW = 64 / Split<M>::R1;
  static constexpr int CB = (NT / 64) * LW;   // exchange lines of the block
  // fp64: a plane's (kx, y) half-spectrum does not fit in LDS beside the
  // exchange slices, so its wavenumbers split over two blocks, each keeping
  // its kx rows: every block reads its part of the plane's spectra once and
  // transforms the x lines with the other part taken as zero, and the two
  // partial outputs are added into zeroed buffers with float64 atomics (two
  // terms added onto zero give the same sum in either order)
  static constexpr int KSPL = F32 ? 1 : 2;
};

// z planes per output block when no tuned value is given: the next plane's
// first lines load during the current plane's x pass, and the set-up is
// shared (measured at 256^3: 5 at M >= 150, against 2, 3, 4 and 6 for fp32
// and 2 to 4 for fp64; one for the smaller tori).  The count only decides
// which block computes a plane, never the arithmetic of a plane.
__host__ __device__ constexpr int default_out_planes(int M) { return M >= 150 ? 5 : 1; }

// LDS ordering among the lanes of one wave (the wave's LDS operations are
// executed in order; this keeps the compiler from moving them across).
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <typename T>
__device__ __forceinline__ cplx<T> conjw(cplx<T> w) { return {w.x, -w.y}; }

template <typename T, int n, int M>
__global__ void __launch_bounds__(256) conv_yz_kernel(const cplx<T>* __restrict__ X, const T* __restrict__ spec,
                                                      cplx<T>* __restrict__ Zb, int Wp, int b, int Wa, int e, int da,
                                                      const int* __restrict__ live, int p0) {
  constexpr int Mh = M / 2 + 1;
  constexpr int S = n + 1;
  constexpr int R1 = Split<M>::R1, R2 = Split<M>::R2;
  constexpr int CB = Batch<T, M>::CB, XL = Batch<T, M>::XLYZ;
  // source rows after the y FFT; row stride M + 4 keeps the column reads of
  // one wave on distinct LDS banks
  constexpr int YS = M + 4;
  __shared__ cplx<T> Y[S * YS];
  __shared__ cplx<T> Ex[CB * XL];
  __shared__ cplx<T> tw[M];
  __shared__ short zmap[M];
  // p: patch; pc: its slot in the chunk-local Zb (patches p0 .. p0 + gridDim.y - 1)
  // (a grid padded to 88 wavenumbers, so that each XCD sees only kx = x
  // (mod 8) and holds fewer spectrum slices in its L2, measured slower:
  // 2.20 -> 2.38 ms at 256^3)
  const int kx = blockIdx.x, pc = blockIdx.y, p = p0 + pc;
  if (live && !live[p]) return;   // an empty patch: its spectra are never read
  const int tid = threadIdx.x;
  fill_twiddles(tw, M);
  for (int m = tid; m < M; m += blockDim.x) zmap[m] = -1;
  __syncthreads();
  for (int zi = tid; zi < Wp; zi += blockDim.x) {
    int z = out_coord(zi, b, Wa, e, da, n);
    zmap[z < 0 ? z + M : z] = short(zi);
  }
  const cplx<T>* xin = X + (int64_t(p) * Mh + kx) * S * S;
  const cplx<T> zero = {T(0), T(0)};
  // the block's source rows, loaded up front (R1 >= ceil(S / R2) values each)
  constexpr int NBR = (S + CB - 1) / CB;
  constexpr int NJ = (S + R2 - 1) / R2;   // nonzero inputs of one pass-1 line
  cplx<T> xr[NBR][NJ];
  {
    const int t = tid % R2, r = tid / R2;
#pragma unroll
    for (int j = 0; j < NBR; ++j)
#pragma unroll
      for (int j1 = 0; j1 < NJ; ++j1) {
        int sz = j * CB + r, sy = t + R2 * j1;
        // (a loaded-or-zero value: a select between the load's address and
        // a local zero would turn the load into a flat one)
        cplx<T> x = zero;
        if (tid < CB * R2 && sz < S && sy < S) x = xin[sz * S + sy];
        xr[j][j1] = x;
      }
  }
  // ---- FFT along y of the S source rows (CB rows per batch) ----
  // the thread's twiddles w^(t k1) of every batch, held in registers
  cplx<T> twY[R1];
#pragma unroll
  for (int k1 = 0; k1 < R1; ++k1) twY[k1] = tw[(tid % R2) * k1];
#pragma unroll 1
  for (int rb = 0, jr = 0; rb < S; rb += CB, ++jr) {
    if (tid < CB * R2) {
      const int t = tid % R2, r = tid / R2;
      cplx<T> v[R1];
#pragma unroll
      for (int j1 = 0; j1 < R1; ++j1) v[j1] = zero;
#pragma unroll
      for (int j = 0; j < NBR; ++j)
        if (j == jr) {
#pragma unroll
          for (int j1 = 0; j1 < NJ; ++j1) v[j1] = xr[j][j1];
        }
      dft_reg_nz<T, R1, 1, NJ>(v);
      cplx<T>* ex = Ex + r * XL + t * (R1 + 1);
#pragma unroll
      for (int k1 = 0; k1 < R1; ++k1) ex[k1] = k1 == 0 ? v[k1] : cmul(v[k1], twY[k1]);
    }
    __syncthreads();
    if (tid < CB * R1) {
      const int s = tid % R1, r = tid / R1, sz = rb + r;
      cplx<T> u[R2];
#pragma unroll
      for (int t = 0; t < R2; ++t) u[t] = Ex[r * XL + t * (R1 + 1) + s];
      dft_reg<T, R2, 1>(u);
      if (sz < S) {
#pragma unroll
        for (int k2 = 0; k2 < R2; ++k2) Y[sz * YS + s + R1 * k2] = u[k2];
      }
    }
    __syncthreads();
  }
  // ---- per column ky: FFT along z, times the spectrum, inverse along z ----
  // Each wave takes LC columns per step through its own slice of Ex, with
  // no block barriers (wave_sync orders the wave's own LDS traffic).
  const T* sp = spec + int64_t(kx) * Mh * Mh;
  cplx<T>* zout = Zb + (int64_t(pc) * Wp * Mh + kx) * M;
  constexpr int LC = Batch<T, M>::LC;
  const int wave = tid >> 6, lane = tid & 63;
  cplx<T>* ex = Ex + wave * LC * XL;
  const int ca = lane % LC, ta = lane / LC;     // R1-point passes: R2 lanes per column (columns fastest)
  const int sb = lane % R1, cb2 = lane / R1;    // R2-point passes: R1 lanes per column
  const bool actA = lane < LC * R2, actB = lane < LC * R1;
  __syncthreads();   // zmap
  int zoff[R1];      // the lane's output rows: zi * Mh * M, or -1
#pragma unroll
  for (int j1 = 0; j1 < R1; ++j1) {
    const int zi = zmap[ta + R2 * j1];
    zoff[j1] = zi >= 0 ? zi * Mh * M : -1;
  }
  // the lane's twiddles, the same at every column step, held in registers:
  // w^(ta k1) after the R1-point pass, w^(-t sb) after the R2-point pass
  cplx<T> twA[R1], twB[R2];
#pragma unroll
  for (int k1 = 0; k1 < R1; ++k1) twA[k1] = ta < R2 ? tw[ta * k1] : cplx<T>{T(1), T(0)};
#pragma unroll
  for (int t = 0; t < R2; ++t) twB[t] = conjw(tw[t * sb]);
#pragma unroll 1
  for (int c0 = wave * LC; c0 < M; c0 += (blockDim.x / 64) * LC) {
    if (actA) {
      const int ky = c0 + ca;
      cplx<T> v[R1];
#pragma unroll
      for (int j1 = 0; j1 < R1; ++j1) {
        int sz = ta + R2 * j1;
        cplx<T> y = zero;
        if (j1 < NJ && sz < S && ky < M) y = Y[sz * YS + ky];
        v[j1] = y;
      }
      dft_reg_nz<T, R1, 1, NJ>(v);
      cplx<T>* e = ex + ca * XL + ta * (R1 + 1);
#pragma unroll
      for (int k1 = 0; k1 < R1; ++k1) e[k1] = k1 == 0 ? v[k1] : cmul(v[k1], twA[k1]);
    }
    wave_sync();
    cplx<T> u[R2];
    if (actB) {
      const int ky = c0 + cb2;
#pragma unroll
      for (int t = 0; t < R2; ++t) u[t] = ex[cb2 * XL + t * (R1 + 1) + sb];
      dft_reg<T, R2, 1>(u);
      const int ay = ky < M ? (ky <= M / 2 ? ky : M - ky) : 0;
      const T* srow = sp + ay * Mh;
#pragma unroll
      for (int k2 = 0; k2 < R2; ++k2) {
        int kz = sb + R1 * k2;
        T gk = srow[kz <= M / 2 ? kz : M - kz];
        u[k2] = {u[k2].x * gk, u[k2].y * gk};
      }
      dft_reg<T, R2, -1>(u);
#pragma unroll
      for (int t = 1; t < R2; ++t)
        u[t] = cmul(u[t], twB[t]);
    }
    wave_sync();
    if (actB) {
#pragma unroll
      for (int t = 0; t < R2; ++t) ex[cb2 * XL + sb * (R2 + 1) + t] = u[t];
    }
    wave_sync();
    if (actA) {
      const int ky = c0 + ca;
      cplx<T> v[R1];
#pragma unroll
      for (int s1 = 0; s1 < R1; ++s1) v[s1] = ex[ca * XL + s1 * (R2 + 1) + ta];
      dft_reg<T, R1, -1>(v);
      if (ky < M) {
        cplx<T>* col = zout + ky;
#pragma unroll
        for (int j1 = 0; j1 < R1; ++j1)
          if (zoff[j1] >= 0) col[zoff[j1]] = v[j1];
      }
    }
    wave_sync();
  }
}


struct OutGeom {
  int n, e, da, b, Wa, Wp, Wc, P0, npl;
};

__device__ __forceinline__ int mod_pos(int a, int m) { int r = a % m; return r < 0 ? r + m : r; }

// MULTI = false: one z plane per block, a compile-time count (the plane
// loop and the next plane's prefetch compile away); MULTI = true: zpb >= 2
// planes per block.
template <typename T, int n, int M, bool MULTI>
__global__ void __launch_bounds__((OutBatch<T, M, MULTI>::NT)) conv_out_kernel(const cplx<T>* __restrict__ Zb,
                                                                      T* __restrict__ coarse,
                                                                      T* __restrict__ planes, OutGeom g,
                                                                      const ProbDesc* __restrict__ pd, int nprob,
                                                                      const int* __restrict__ live,
                                                                      const int* __restrict__ patch_of, int p0,
                                                                      int zpb_arg) {
  constexpr int Mh = M / 2 + 1;
  constexpr int R1 = Split<M>::R1, R2 = Split<M>::R2;
  constexpr int CB = OutBatch<T, M, MULTI>::CB, XL = Batch<T, M>::XLYZ;
  constexpr int WPMAX = n + 2 * n + 1 + 2 * 4;  // Wa + 2b with d_alpha <= n, b <= 4
  // fp32: A rows padded to a stride of 11 (mod 32) elements, so the lines
  // of one wave step start on spread-out LDS banks (fp64: no room to pad)
  constexpr bool PADA = sizeof(T) == 4;
  constexpr int KSPL = OutBatch<T, M>::KSPL;
  constexpr int KXH = (Mh + KSPL - 1) / KSPL;   // wavenumbers per block
  constexpr int WQMAX = PADA ? WPMAX + ((11 - WPMAX % 32) + 32) % 32 : WPMAX;
  __shared__ cplx<T> A[KXH * WQMAX];
  __shared__ cplx<T> Ex[CB * XL];
  __shared__ cplx<T> tw[M];
  __shared__ short omap[M];
  // per output index i (same list on the y and x axes): coordinate and flags
  // bit 0: inside Omega_alpha, bit 1: coarse node, bit 2: skeleton plane
  __shared__ short ocrd[WPMAX];
  __shared__ unsigned char oflg[WPMAX];
  // rows (output y) whose whole x line is needed, and rows that only need
  // the x coordinates of skeleton planes
  __shared__ short frow[WPMAX], crow[WPMAX];
  __shared__ int nfull, ncols;
  // inverse twiddles of the skeleton-plane x coordinates: Wx[j][k] = w^(k x_j)
  constexpr int NPLMAX = 4;
  // torus slots of the x outputs (or -1): of x + d_alpha over Omega_alpha, of
  // the coarse nodes (x + e)/4, of the skeleton planes
  __shared__ short xs_a[WPMAX], xs_c[WPMAX], xs_p[NPLMAX];
  constexpr int WXS = M / 2 + 1;   // row stride: the four rows on distinct LDS banks
  __shared__ cplx<T> Wx[NPLMAX * WXS];
  const int zpb = MULTI ? zpb_arg : 1;
  const int zi0 = (blockIdx.x / KSPL) * zpb, pc = blockIdx.y, p = p0 + pc;
  const int Wp = g.Wp;
  if (live && !live[p]) {
    // an empty patch: its local field is zero (the first block writes the
    // zeros; split blocks add into buffers already zeroed)
    if (KSPL == 1 && blockIdx.x == 0) {
      T* cz = coarse + int64_t(p) * g.Wc * g.Wc * g.Wc;
      T* pz = planes + int64_t(p) * 3 * g.npl * g.Wa * g.Wa;
      for (int i = threadIdx.x; i < g.Wc * g.Wc * g.Wc; i += blockDim.x) cz[i] = T(0);
      for (int i = threadIdx.x; i < 3 * g.npl * g.Wa * g.Wa; i += blockDim.x) pz[i] = T(0);
    }
    return;
  }
  // this block's wavenumbers [kx_lo, kx_hi) (all of them in fp32)
  const int kx_lo = int(blockIdx.x % KSPL) * KXH, kx_hi = min(Mh, kx_lo + KXH);
  const int Wq = PADA ? Wp + ((11 - Wp % 32) + 32) % 32 : Wp;   // row stride of A
  const int tid = threadIdx.x;
  // h^2 in the kernel's precision (for the fp32 kernel: one rounding of h^2,
  // none when h is a power of two)
  const T hsq = T(pd[find_problem(pd, nprob, patch_of ? patch_of[p] : p)].h2);
  const cplx<T>* zin = Zb + (int64_t(pc) * Wp + zi0) * Mh * M;   // the current plane
  constexpr int LW = OutBatch<T, M, MULTI>::LW, NW = OutBatch<T, M, MULTI>::NT / 64;
  const int wave = tid >> 6, lane = tid & 63;
  const int s1 = lane % R1, r1 = lane / R1, t2 = lane % R2, r2 = lane / R2;
  const bool act1 = lane < LW * R1, act2 = lane < LW * R2;
  cplx<T>* ex = Ex + wave * LW * XL;   // this wave's exchange slice
  // the first step's lines, issued before the set-up below
  cplx<T> u0[R2];
  auto load_lines = [&](cplx<T>* dst, int kb) {
    const int kx = kb + r1;
#pragma unroll
    for (int k2 = 0; k2 < R2; ++k2)
      dst[k2] = (act1 && kx < kx_hi) ? zin[int64_t(kx) * M + s1 + R1 * k2] : cplx<T>{T(0), T(0)};
  };
  // an output value: stored, or (wavenumbers split) added to the zeroed buffer
  auto put = [&](T* dst, T v) {
    if constexpr (KSPL > 1) unsafeAtomicAdd(dst, v);
    else *dst = v;
  };
  load_lines(u0, kx_lo + wave * LW);
  fill_twiddles(tw, M);
  for (int m = tid; m < M; m += blockDim.x) omap[m] = -1;
  for (int i = tid; i < WPMAX; i += blockDim.x) xs_a[i] = xs_c[i] = -1;
  if (tid < NPLMAX) xs_p[tid] = -1;
  __syncthreads();
  for (int k = tid; k < Wp; k += blockDim.x) {
    int y = out_coord(k, g.b, g.Wa, g.e, g.da, n);
    omap[y < 0 ? y + M : y] = short(k);
    ocrd[k] = short(y);
    bool ina = y >= -g.da && y <= n + g.da;
    oflg[k] = (ina ? 1 : 0) | (mod_pos(y, NREF) == 0 ? 2 : 0) | ((ina && mod_pos(y, n) == 0) ? 4 : 0);
  }
  __syncthreads();
  for (int m = tid; m < M; m += blockDim.x) {
    const int xi = omap[m];
    if (xi >= 0) {
      const int x = ocrd[xi], xf = oflg[xi];
      const int xda = x + g.da, xcc = (x + g.e) / NREF, xpl = (x - g.P0) / n;
      if ((xf & 1) && xda < WPMAX) xs_a[xda] = short(m);
      if ((xf & 2) && xcc < WPMAX) xs_c[xcc] = short(m);
      if ((xf & 4) && xpl < NPLMAX) xs_p[xpl] = short(m);
    }
  }
  for (int t = tid; t < g.npl * (M / 2); t += blockDim.x) {
    const int j = t / (M / 2), k = t % (M / 2);
    const int x = g.P0 + j * n, xs = x < 0 ? x + M : x;
    Wx[j * WXS + k] = tw[(k * xs) % M];
  }
#pragma unroll 1
  for (int q = 0; q < zpb; ++q) {
    const int zi = zi0 + q;
    if (zi >= Wp) break;   // uniform over the block
    if (tid < 64) {
      // compact the two row lists in ascending order with wave ballots
      const int zf = oflg[zi];
      int a = 0, c = 0;
      const uint64_t below = (uint64_t(1) << tid) - 1;
      for (int base = 0; base < Wp; base += 64) {
        const int yi = base + tid;
        const int yf = yi < Wp ? oflg[yi] : 0;
        // z-plane rows in Omega_alpha, coarse rows of a coarse z, y-plane rows
        const bool full = ((zf & 4) && (yf & 1)) || ((zf & 2) && (yf & 2)) || ((zf & 1) && (yf & 4));
        const bool col = !full && (zf & 1) && (yf & 1);   // x-plane columns only
        const uint64_t mf = __ballot(full), mc = __ballot(col);
        if (full) frow[a + __popcll(mf & below)] = short(yi);
        if (col) crow[c + __popcll(mc & below)] = short(yi);
        a += __popcll(mf);
        c += __popcll(mc);
      }
      if (tid == 0) {
        nfull = a;
        ncols = c;
      }
    }
    // y pass, second half: one line's R1-point DFT in R2 lanes (lanes (t, r)),
    // kept outputs into A
    // (ymap[j1] = omap[t + R2 j1], the lane's output slots, held in registers)
    auto y_pass2 = [&](const cplx<T>* ex, int t, int r, int kx, const short* ymap) {
      cplx<T> v[R1];
#pragma unroll
      for (int s = 0; s < R1; ++s) v[s] = ex[r * XL + s * (R2 + 1) + t];
      dft_reg<T, R1, -1>(v);
      if (kx < kx_hi) {
        cplx<T>* arow = A + (kx - kx_lo) * Wq;
#pragma unroll
        for (int j1 = 0; j1 < R1; ++j1)
          if (ymap[j1] >= 0) arow[ymap[j1]] = v[j1];
      }
    };
    // the lane's inverse twiddles w^(-t s1) of both first-half passes, held in
    // registers
    cplx<T> tws[R2];
#pragma unroll
    for (int t = 0; t < R2; ++t) tws[t] = conjw(tw[t * s1]);
    // y pass, first half: R2-point DFT of one line's column s (= s1), twiddled, to ex
    auto y_pass1 = [&](cplx<T>* u, cplx<T>* ex, int s, int r) {
      dft_reg<T, R2, -1>(u);
#pragma unroll
      for (int t = 0; t < R2; ++t) {
        cplx<T> w = t ? cmul(u[t], tws[t]) : u[t];
        ex[r * XL + s * (R2 + 1) + t] = w;
      }
    };
    __syncthreads();
    // ---- inverse FFT along y for every kx ----
    {
      short ymap[R1];
#pragma unroll
      for (int j1 = 0; j1 < R1; ++j1) {
        ymap[j1] = omap[t2 + R2 * j1];
      }
#pragma unroll 1
      for (int kb = kx_lo + wave * LW; kb < kx_hi; kb += NW * LW) {
        cplx<T> un[R2];
        load_lines(un, kb + NW * LW);   // next step's lines in flight meanwhile
        if (act1) y_pass1(u0, ex, s1, r1);
        wave_sync();
        if (act2) y_pass2(ex, t2, r2, kb + r2, ymap);
        wave_sync();
#pragma unroll
        for (int k2 = 0; k2 < R2; ++k2) u0[k2] = un[k2];
      }
    }
    // the next plane's first lines stay in flight through this plane's x pass
    if (q + 1 < zpb && zi + 1 < Wp) {
      zin += int64_t(Mh) * M;
      load_lines(u0, kx_lo + wave * LW);
    }
    __syncthreads();
    const int z = ocrd[zi];
    const bool zin_a = oflg[zi] & 1, zc = oflg[zi] & 2, zpl = oflg[zi] & 4;
    const int npl = g.npl, Wa = g.Wa, Wc = g.Wc;
    T* cbase = coarse + int64_t(p) * Wc * Wc * Wc;
    T* pbase = planes + int64_t(p) * 3 * npl * Wa * Wa;
    const int nf = nfull, ncl = ncols;
    // ---- Hermitian inverse along x of the full rows: two real lines per complex line ----
    // first half: pair-line c's column s (rows frow[2c], frow[2c+1])
    auto x_pass1 = [&](cplx<T>* ex, int s, int c, int pi) {
      const int i1 = 2 * pi;
      const int y1 = i1 < nf ? frow[i1] : Wp, y2 = i1 + 1 < nf ? frow[i1 + 1] : Wp;
      cplx<T> u[R2];
#pragma unroll
      for (int k2 = 0; k2 < R2; ++k2) {
        int k = s + R1 * k2;
        cplx<T> h1 = {T(0), T(0)}, h2 = {T(0), T(0)};
        // the line's half-spectrum entry (mirrored and conjugated above M/2),
        // zero for wavenumbers of the other block
        const bool lo = k < Mh;
        const int kk = lo ? k : M - k;
        if (kk >= kx_lo && kk < kx_hi) {
          const cplx<T>* ar = A + (kk - kx_lo) * Wq;
          if (y1 < Wp) h1 = lo ? ar[y1] : conjw(ar[y1]);
          if (y2 < Wp) h2 = lo ? ar[y2] : conjw(ar[y2]);
        }
        if (k == 0 || k == M / 2) { h1.y = T(0); h2.y = T(0); }   // real DC / Nyquist
        u[k2] = {h1.x - h2.y, h1.y + h2.x};                        // h1 + i h2
      }
      dft_reg<T, R2, -1>(u);
#pragma unroll
      for (int t = 0; t < R2; ++t) {
        cplx<T> w = t ? cmul(u[t], tws[t]) : u[t];
        ex[c * XL + s * (R2 + 1) + t] = w;
      }
    };
    // second half: pair-line c's R1-point DFT in R2 lanes (lanes (t, c));
    // the line's two real output rows (real and imaginary parts) then go back
    // to the slice in torus order
    auto x_pass2 = [&](const cplx<T>* ex, int t, int c, cplx<T>* v) {
#pragma unroll
      for (int s = 0; s < R1; ++s) v[s] = ex[c * XL + s * (R2 + 1) + t];
      dft_reg<T, R1, -1>(v);
    };
    // torus slots of the lane's x outputs (the same lists for every row)
    constexpr int NXC = (WPMAX + 63) / 64;
    int mA[NXC], mC[NXC];
#pragma unroll
    for (int a = 0; a < NXC; ++a) {
      const int i = lane + 64 * a;
      mA[a] = i < WPMAX ? xs_a[i] : -1;
      mC[a] = i < WPMAX ? xs_c[i] : -1;
    }
    const int mP = lane < NPLMAX ? xs_p[lane] : -1;
    const int Wa2 = Wa * Wa;
    const int npair = (nf + 1) / 2;
    // pair lines from the last wave down, the direct sums below from the
    // first thread up: on most planes the two go to different waves
#pragma unroll 1
    for (int pb = (NW - 1 - wave) * LW; pb < npair; pb += NW * LW) {
      // lane rr < 2 LW: destination bases of row 2 pb + rr (or -1), read by
      // every lane below with readlane
      int rZ = -1, rY = -1, rC = -1, rX = -1;
      if (lane < 2 * LW && 2 * pb + lane < nf) {
        const int yi = frow[2 * pb + lane];
        const int y = ocrd[yi], yf = oflg[yi];
        if (zpl && (yf & 1)) rZ = ((z - g.P0) / n * Wa + (y + g.da)) * Wa;
        if (zin_a && (yf & 1) && (yf & 4)) rY = ((npl + (y - g.P0) / n) * Wa + (z + g.da)) * Wa;
        if (zc && (yf & 2)) rC = (((z + g.e) / NREF) * Wc + (y + g.e) / NREF) * Wc;
        if (zin_a && (yf & 1)) rX = (2 * npl * Wa + (z + g.da)) * Wa + (y + g.da);
      }
      if (act1) x_pass1(ex, s1, r1, pb + r1);
      wave_sync();
      cplx<T> v[R1];
      if (act2) x_pass2(ex, t2, r2, v);
      wave_sync();
      if (act2) {
#pragma unroll
        for (int j1 = 0; j1 < R1; ++j1) ex[r2 * XL + t2 + R2 * j1] = v[j1];
      }
      wave_sync();
      // outputs, one row at a time, the lanes along its destinations
#pragma unroll
      for (int rr = 0; rr < 2 * LW; ++rr) {
        const int rowZ = __builtin_amdgcn_readlane(rZ, rr), rowY = __builtin_amdgcn_readlane(rY, rr);
        const int rowC = __builtin_amdgcn_readlane(rC, rr), rowX = __builtin_amdgcn_readlane(rX, rr);
        const T* line = reinterpret_cast<const T*>(ex + (rr >> 1) * XL) + (rr & 1);
        if (rowZ >= 0 || rowY >= 0) {
#pragma unroll
          for (int a = 0; a < NXC; ++a) {
            if (mA[a] < 0) continue;
            const T val = line[2 * mA[a]] * hsq;
            if (rowZ >= 0) put(pbase + rowZ + lane + 64 * a, val);
            if (rowY >= 0) put(pbase + rowY + lane + 64 * a, val);
          }
        }
        if (rowC >= 0) {
#pragma unroll
          for (int a = 0; a < NXC; ++a)
            if (mC[a] >= 0) put(cbase + rowC + lane + 64 * a, line[2 * mC[a]] * hsq);
        }
        if (rowX >= 0 && mP >= 0) put(pbase + rowX + lane * Wa2, line[2 * mP] * hsq);
      }
      wave_sync();
    }
    // ---- x-plane columns of the other rows: direct Hermitian sums ----
    //   f(x) = F_0 + (-1)^x F_{M/2} + 2 sum_{0<k<M/2} Re(F_k e^{2 pi i k x / M})
    for (int q = tid; q < ncl * npl; q += blockDim.x) {
      const int yi = crow[q / npl], j = q % npl;
      const int x = g.P0 + j * n, xs = x < 0 ? x + M : x;
      const cplx<T>* wj = Wx + j * WXS;
      // four interleaved partial sums over the block's k in 1 .. M/2 - 1
      const int k_first = max(1, kx_lo), k_last = min(M / 2 - 1, kx_hi - 1);
      auto ay = [&](int k) { return A[(k - kx_lo) * Wq + yi]; };   // the entry of wavenumber k
      T acc[4] = {T(0), T(0), T(0), T(0)};
      int k0 = k_first;
#pragma unroll 2
      for (; k0 + 3 <= k_last; k0 += 4) {
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const cplx<T> a = ay(k0 + u);
          const cplx<T> w = wj[k0 + u];
          acc[u] += a.x * w.x + a.y * w.y;
        }
      }
#pragma unroll
      for (int u = 0; u < 3; ++u) {
        if (k0 + u <= k_last) {
          const cplx<T> a = ay(k0 + u);
          const cplx<T> w = wj[k0 + u];
          acc[u] += a.x * w.x + a.y * w.y;
        }
      }
      const T dc = kx_lo == 0 ? ay(0).x : T(0);
      const T ny = (M / 2 >= kx_lo && M / 2 < kx_hi) ? ay(M / 2).x : T(0);
      const T val = dc + ((xs & 1) ? -ny : ny) + T(2) * ((acc[0] + acc[1]) + (acc[2] + acc[3]));
      const int y = ocrd[yi];
      put(pbase + ((int64_t(2) * npl + j) * Wa + (z + g.da)) * Wa + (y + g.da), val * hsq);
    }
    __syncthreads();   // A, Ex and the row lists are rewritten for the next plane
  }
}

}  // namespace mlc
