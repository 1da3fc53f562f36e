// libmlc: host side of the C ABI declared in include/mlc.h.  Validation and
// sizing, the context (resident DGF tables), plan set-up (DGF spectra and
// far-field tables) and the enqueueing of every stage of a solve.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <functional>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <utility>
#include <vector>

#include "../../include/mlc.h"
#include "common.h"
#include "conv_kernels.h"
#include "setup_kernels.h"
#include "stage_kernels.h"
#include "analytic_kernels.h"

using namespace mlc;

// ------------------------------------------------------------------ state
struct mlc_context {
  int device = 0;
  size_t budget = 0;                  // cap on resident device memory (0: none)
  std::atomic<size_t> resident{0};    // DGF tables, plan tables, server arenas
  std::mutex err_mu;    // guards last_error
  std::string last_error;
  std::mutex build_mu;  // serialises plan and DGF builds (a server thread may build too)
  std::map<std::pair<int, int>, double*> dgf;   // (Q, Z) -> (2Z+1)^3 table
  // autotuned (local torus, output planes per block) per patch-work class
  std::map<std::vector<int>, std::pair<int, int>> tuned;
  // per caller stream: a second stream (default priority) for the stages
  // that do not depend on the local convolutions, and the fork/join events
  // and the MLC_CHECK flag of that caller stream (set by the device when f
  // is nonzero on the outer boundary)
  struct Side {
    hipStream_t stream = nullptr;
    hipEvent_t ev[3] = {nullptr, nullptr, nullptr};
    int* check_flag = nullptr;
  };
  std::mutex side_mu;
  std::map<hipStream_t, Side> side;
};

// Resident-memory accounting against the context's budget (hbm_budget_bytes
// of mlc_context_create): DGF tables, the tables of every live plan and the
// server arenas.  Transient build buffers and caller workspaces are not
// counted.
bool mlc_budget_take(mlc_context* ctx, size_t bytes) {
  size_t cur = ctx->resident.load();
  for (;;) {
    if (ctx->budget && cur + bytes > ctx->budget) return false;
    if (ctx->resident.compare_exchange_weak(cur, cur + bytes)) return true;
  }
}
void mlc_budget_give(mlc_context* ctx, size_t bytes) { ctx->resident -= bytes; }

struct mlc_plan {
  mlc_context* ctx = nullptr;
  mlc_problem prob{};
  mlc_plan_info info{};
  int S = 0, Mh = 0, Wp = 0, P0 = 0, eb = 0, Wtc = 0, Wb = 0, Wbc = 0, P0b = 0, nplb = 0, Kann = 0;
  ModeList modes{};
  LagW lagw{};
  void* conv_spec = nullptr;
  double* coarse_spec = nullptr;
  double* T = nullptr;
  double* D = nullptr;
  double* Am = nullptr;   // skeleton far-field table laid out for MFMA
  double* Tm = nullptr;   // coarse far-field table laid out for MFMA
  double* gram_inv = nullptr;   // P >= 5: inverse Boole Gram matrix of the modes, K x K
  mlc_plan* child = nullptr;    // multilevel: the plan of the next coarser level
  bool correct = true;          // add the final Mehrstellen correction (false at coarser levels)
  size_t o_lf = 0, o_lphi = 0, o_lws = 0;   // multilevel: the next level's charge, solution, workspace
  size_t o_ft = 0;                          // sixth-order right-hand side
  MfmaGeom mg_skel{}, mg_coarse{};
  // workspace offsets of the plan's own (batch-of-one) layout
  size_t o_mom = 0, o_cs = 0, o_pl = 0, o_F = 0, o_phiH = 0, o_phiB = 0;
  size_t ws_total = 0;
  size_t table_bytes = 0;   // device bytes of the buffers above (the plan's resident tables)
  bool charged = false;     // table_bytes counted against the context's budget
  // per-kernel timing (instrumentation)
  struct Pending { const char* name; hipEvent_t a, b; };
  mutable bool timing_on = false;
  mutable std::vector<Pending> pending;
  mutable std::vector<hipEvent_t> event_pool;
  mutable std::vector<std::pair<std::string, std::pair<int, double>>> acc;
};

static hipEvent_t pool_event(const mlc_plan* P) {
  if (!P->event_pool.empty()) {
    hipEvent_t e = P->event_pool.back();
    P->event_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  hipEventCreate(&e);
  return e;
}

// Brackets one launch (or a fixed group of launches) with timing events when
// timing is enabled on the plan.
struct TimedScope {
  const mlc_plan* P;
  hipStream_t s;
  const char* name;
  hipEvent_t a = nullptr;
  TimedScope(const mlc_plan* p, hipStream_t st, const char* nm) : P(p), s(st), name(nm) {
    if (P->timing_on) { a = pool_event(P); hipEventRecord(a, s); }
  }
  ~TimedScope() {
    if (P->timing_on && a) {
      hipEvent_t b = pool_event(P);
      hipEventRecord(b, s);
      P->pending.push_back({name, a, b});
    }
  }
};

static thread_local std::string g_error;   // errors before a context exists

// ------------------------------------------------- allocation-free solves
// The workspace of mlc_solve_static: one file-scope device array, of which
// every GPU the library runs on holds its own copy until the process ends.
// In host code `scratch` names a host-side stand-in, not a device address;
// its device address on each GPU comes from hipGetSymbolAddress, taken once
// per device (with that device current) when a context is created there,
// and only that address is ever passed to kernels.
constexpr size_t kStaticScratchBytes = MLC_STATIC_SCRATCH_BYTES;
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];
static std::mutex g_scratch_mu;
static std::map<int, void*> g_scratch_ptr;   // device -> its copy of scratch

// With `device` current: record the address of its copy of scratch.
static hipError_t scratch_init(int device) {
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (g_scratch_ptr.count(device)) return hipSuccess;
  void* ptr = nullptr;
  const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  if (e == hipSuccess && ptr) g_scratch_ptr[device] = ptr;
  return e == hipSuccess && !ptr ? hipErrorInvalidSymbol : e;
}

static void* scratch_of(int device) {
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  auto it = g_scratch_ptr.find(device);
  return it == g_scratch_ptr.end() ? nullptr : it->second;
}

static mlc_status fail(mlc_context* ctx, mlc_status s, const std::string& msg) {
  if (ctx) {
    std::lock_guard<std::mutex> lk(ctx->err_mu);
    ctx->last_error = msg;
  }
  g_error = msg;
  return s;
}

// for the serving loop (server.hip)
void mlc_set_error(mlc_context* ctx, const std::string& msg) { fail(ctx, MLC_OK, msg); }
int mlc_context_device(const mlc_context* ctx) { return ctx->device; }

#define HIP_TRY(ctx, expr)                                                                       \
  do {                                                                                          \
    hipError_t e_ = (expr);                                                                     \
    if (e_ != hipSuccess)                                                                       \
      return fail((ctx), MLC_ERR_DEVICE, std::string(#expr) + ": " + hipGetErrorString(e_));   \
  } while (0)

// ------------------------------------------------------- supported sizes
// Local-convolution tori (n, M) with compiled kernels, per precision.
#define MLC_CONV_SIZES_F32(X) X(8, 50) X(8, 64) X(8, 72) X(16, 90) X(16, 96) X(16, 120) X(16, 128) \
  X(32, 150) X(32, 160) X(32, 180) X(32, 192)
#define MLC_CONV_SIZES_F64(X) X(8, 50) X(8, 64) X(8, 72) X(16, 90) X(16, 96) X(16, 120) X(16, 128) \
  X(32, 150) X(32, 160)
// Generic FFT lengths (DGF spectra, far-field tables, coarse solve).
#define MLC_FFT_SIZES(X) X(50) X(64) X(72) X(80) X(90) X(96) X(100) X(120) X(128) X(144) X(150) X(160) \
  X(180) X(192) X(200) X(216) X(240) X(250) X(256)

static bool conv_size_ok(int prec, int n, int M) {
#define CHK(nn, MM) if (n == nn && M == MM) return true;
  if (prec == MLC_CONV_FP32) { MLC_CONV_SIZES_F32(CHK) }
  else { MLC_CONV_SIZES_F64(CHK) }
#undef CHK
  return false;
}
static const int kFftSizes[] = {
#define LST(MM) MM,
    MLC_FFT_SIZES(LST)
#undef LST
};
static int pick_fft(int minimum, int maximum) {
  for (int m : kFftSizes)
    if (m >= minimum && m <= maximum) return m;
  return -1;
}
static int pick_conv(int prec, int n, int minimum) {
  for (int m : kFftSizes)
    if (m >= minimum && conv_size_ok(prec, n, m)) return m;
  return -1;
}

static int margin_of(double r, int n) {
  // ceil((r - 1) n / 2) with a tolerance for decimal radii such as 3.25
  double v = (r - 1.0) * n / 2.0;
  double c = std::ceil(v - 1e-9);
  return int(c);
}

static ModeList mode_list(int P) {
  ModeList m{};
  m.K = 0;
  for (int deg = 0; deg < P; ++deg) {
    // descending lexicographic order within a degree
    for (int a = deg; a >= 0; --a)
      for (int b = deg - a; b >= 0; --b) {
        int c = deg - a - b;
        m.p[m.K][0] = a; m.p[m.K][1] = b; m.p[m.K][2] = c;
        ++m.K;
      }
  }
  return m;
}

// ------------------------------------------------------------ validation
extern "C" const char* mlc_status_string(mlc_status s) {
  switch (s) {
    case MLC_OK: return "MLC_OK";
    case MLC_ERR_INVALID_ARG: return "MLC_ERR_INVALID_ARG";
    case MLC_ERR_UNSUPPORTED: return "MLC_ERR_UNSUPPORTED";
    case MLC_ERR_OUT_OF_MEMORY: return "MLC_ERR_OUT_OF_MEMORY";
    case MLC_ERR_DEVICE: return "MLC_ERR_DEVICE";
    case MLC_ERR_BUSY: return "MLC_ERR_BUSY";
    case MLC_ERR_NOT_READY: return "MLC_ERR_NOT_READY";
  }
  return "MLC_ERR_UNKNOWN";
}

// The next coarser level of a multilevel problem (sec. 5): its box
// [-m, N/4 + m] in coarse cells, m the smallest multiple of n with m >=
// d_beta/4 + b + 1 (F^H, supported on the coarsened Omega_beta regions,
// vanishes on the box's outer nodes, and its b-grown support lies inside: the
// proper nesting condition) -- and, when that level has a coarser level of
// its own, with (N/4 + 2m)/4 a multiple of n -- at spacing Nref h, everything
// else the same.
static void set_level_box(mlc_plan_info* I) {
  const int need = I->d_beta / NREF + I->b + 1;
  int m = (need + I->n - 1) / I->n * I->n;
  // a box that is itself multilevel must be 4-aligned in patches too
  if (I->levels > 3)
    while (((I->N / NREF + 2 * m) / NREF) % I->n || (I->N / NREF + 2 * m) % NREF) m += I->n;
  I->level_margin = m;
  I->level_N = I->N / NREF + 2 * m;
  I->M_coarse = 0;   // no coarse convolution at a level with a coarser level below
}

static mlc_status derive(const mlc_problem* p, mlc_plan_info* o, std::string* why);

// The problem the next coarser level solves: the level box at spacing Nref h,
// its own inner radius (level_alpha[0]), the coarser radii shifted down, and
// this level's local torus when it is large enough for that radius (so an
// autotuned torus is not tuned again), else the smallest built one.
static mlc_problem child_problem(const mlc_plan_info& I) {
  mlc_problem c{};
  c.n_cells = I.level_N;
  c.h = NREF * I.h;
  c.patch = I.n;
  c.alpha = I.level_alpha[0];
  c.beta = I.beta;
  c.P = I.P;
  c.Q = I.Q;
  c.interp_b = I.b;
  c.conv_precision = I.conv_precision;
  c.dgf_half_width = I.Z;
  c.levels = I.levels - 1;
  c.level_alpha[0] = I.level_alpha[1];
  c.level_alpha[1] = I.level_alpha[2];
  c.level_alpha[2] = 0.0;
  c.rhs_order = 0;   // the coarser levels solve their node charge as it is
  c.skip_empty = I.skip_empty;   // box_cells stay zero: the level box is a cube; max_live 0 (dense)
  const int e = margin_of(c.alpha, I.n) + NREF * I.b;
  c.fft_size = (I.M >= 2 * (I.n + e) + 1 && conv_size_ok(I.conv_precision, I.n, I.M)) ? I.M : 0;
  return c;
}

// Sizes of the next coarser level (derive of child_problem, which the caller
// has validated).
static mlc_plan_info level_info(const mlc_plan_info& I) {
  const mlc_problem c = child_problem(I);
  mlc_plan_info C{};
  std::string why;
  derive(&c, &C, &why);
  return C;
}

static mlc_status derive(const mlc_problem* p, mlc_plan_info* o, std::string* why) {
  if (!p || !o) { *why = "null argument"; return MLC_ERR_INVALID_ARG; }
  mlc_plan_info I{};
  I.N = p->n_cells; I.n = p->patch; I.P = p->P; I.Q = p->Q;
  I.b = p->interp_b ? p->interp_b : p->Q / 2;
  I.conv_precision = p->conv_precision;
  I.h = p->h;
  I.H = NREF * p->h;
  I.Z = p->dgf_half_width ? p->dgf_half_width : 128;
  I.levels = p->levels ? p->levels : 2;
  if (I.levels < 2 || I.levels > 4) { *why = "levels must be 2, 3 or 4"; return MLC_ERR_UNSUPPORTED; }
  if (p->box_cells[0] || p->box_cells[1] || p->box_cells[2]) {
    // a box domain, solved in the smallest cube the plan can run
    if (p->n_cells != 0) { *why = "give n_cells or box_cells, not both"; return MLC_ERR_INVALID_ARG; }
    if (I.n <= 0) { *why = "N, n and h must be positive"; return MLC_ERR_INVALID_ARG; }
    int bmax = 0;
    for (int d = 0; d < 3; ++d) {
      if (p->box_cells[d] <= 0 || p->box_cells[d] % I.n) { *why = "box_cells must be positive multiples of the patch size"; return MLC_ERR_INVALID_ARG; }
      I.box[d] = p->box_cells[d];
      bmax = std::max(bmax, p->box_cells[d]);
    }
    const int unit = I.levels > 2 ? NREF * I.n : I.n;
    I.N = (bmax + unit - 1) / unit * unit;
  } else {
    I.box[0] = I.box[1] = I.box[2] = I.N;
  }
  for (int d = 0; d < 3; ++d) I.origin[d] = p->origin[d];
  if (I.N <= 0 || I.n <= 0 || !(p->h > 0) || !std::isfinite(p->h)) { *why = "N, n and h must be positive"; return MLC_ERR_INVALID_ARG; }
  if (I.N % I.n) { *why = "N must be a multiple of the patch size"; return MLC_ERR_INVALID_ARG; }
  if (I.n % NREF || I.n < 8) { *why = "patch size must be a multiple of 4 and >= 8"; return MLC_ERR_INVALID_ARG; }
  if (!(p->alpha >= 1.0) || !(p->beta >= p->alpha) || !std::isfinite(p->beta)) { *why = "need 1 <= alpha <= beta"; return MLC_ERR_INVALID_ARG; }
  if (I.P < 1) { *why = "P must be >= 1"; return MLC_ERR_INVALID_ARG; }
  if (I.Q != 4 && I.Q != 6) { *why = "Q must be 4 (L19) or 6 (L27)"; return MLC_ERR_UNSUPPORTED; }
  if (p->conv_precision != MLC_CONV_FP32 && p->conv_precision != MLC_CONV_FP64) { *why = "bad conv_precision"; return MLC_ERR_INVALID_ARG; }
  if (I.b < 1 || I.b > 4) { *why = "interpolation radius must be in [1, 4]"; return MLC_ERR_UNSUPPORTED; }
  if (I.P > PMAX) { *why = "P above 9 is not built"; return MLC_ERR_UNSUPPORTED; }
  if (I.n > 32) { *why = "patch size above 32 is not built"; return MLC_ERR_UNSUPPORTED; }
  if (I.Z != 32 && I.Z != 64 && I.Z != 128) { *why = "DGF half-width must be 32, 64 or 128"; return MLC_ERR_UNSUPPORTED; }
  if (p->rhs_order != 0 && p->rhs_order != 4 && p->rhs_order != 6) { *why = "rhs_order must be 0, 4 or 6"; return MLC_ERR_INVALID_ARG; }
  if (p->rhs_order == 6 && I.Q != 6) { *why = "rhs_order 6 is the 27-point operator's (Q = 6)"; return MLC_ERR_UNSUPPORTED; }
  I.rhs_order = p->rhs_order == 6 ? 6 : 4;
  if (p->skip_empty != 0 && p->skip_empty != 1) { *why = "skip_empty must be 0 or 1"; return MLC_ERR_INVALID_ARG; }
  I.skip_empty = p->skip_empty;
  I.K = I.P * (I.P + 1) * (I.P + 2) / 6;
  I.alpha = p->alpha;
  I.beta = p->beta;
  for (int k = 0; k < 3; ++k) {
    const double a = p->level_alpha[k];
    if (a != 0.0 && !(a >= 1.0 && a <= p->beta)) { *why = "level_alpha entries must be 0 or in [1, beta]"; return MLC_ERR_INVALID_ARG; }
    I.level_alpha[k] = a != 0.0 ? a : (k ? I.level_alpha[k - 1] : p->alpha);
  }
  I.d_alpha = margin_of(p->alpha, I.n);
  I.d_beta = margin_of(p->beta, I.n);
  if (I.d_alpha % NREF || I.d_beta % NREF) { *why = "localisation margins must be multiples of 4"; return MLC_ERR_UNSUPPORTED; }
  if (I.d_alpha > I.n) { *why = "alpha > 3 is not built"; return MLC_ERR_UNSUPPORTED; }
  // the skeleton kernels take one thread per skeleton node in one launch
  if (int64_t(3) * (I.N / I.n + 1) * (I.N + 1) * (I.N + 1) >= (int64_t(1) << 31)) {
    *why = "grid too large: the skeleton exceeds one launch";
    return MLC_ERR_UNSUPPORTED;
  }
  I.e = I.d_alpha + NREF * I.b;
  I.patches_per_axis = I.N / I.n;
  I.npatch = I.patches_per_axis * I.patches_per_axis * I.patches_per_axis;
  if (p->max_live < 0) { *why = "max_live must be >= 0"; return MLC_ERR_INVALID_ARG; }
  I.slots = p->max_live > 0 ? std::min(p->max_live, I.npatch) : I.npatch;
  if (p->max_live > 0) I.skip_empty = 1;   // the live patches are the ones with charge
  int Mmin = 2 * (I.n + I.e) + 1;
  if (p->fft_size < -1) { *why = "fft_size must be > 0, 0 (smallest) or -1 (autotune)"; return MLC_ERR_INVALID_ARG; }
  if (p->fft_size > 0) {
    if (p->fft_size < Mmin) { *why = "fft_size below the Hockney minimum 2(n+e)+1"; return MLC_ERR_INVALID_ARG; }
    if (!conv_size_ok(p->conv_precision, I.n, p->fft_size)) { *why = "fft_size not built for this patch size"; return MLC_ERR_UNSUPPORTED; }
    I.M = p->fft_size;
  } else {
    I.M = pick_conv(p->conv_precision, I.n, Mmin);
    if (I.M < 0) { *why = "no built local FFT size fits this problem"; return MLC_ERR_UNSUPPORTED; }
  }
  if (I.M / 2 > I.Z) { *why = "DGF table too small for the local torus"; return MLC_ERR_UNSUPPORTED; }
  I.out_planes = default_out_planes(I.M);
  I.Wc = (I.n + 2 * I.e) / NREF + 1;
  I.Wa = I.n + 2 * I.d_alpha + 1;
  {
    int P0 = -((I.d_alpha / I.n) * I.n);
    I.nplanes_a = (I.n + I.d_alpha - P0) / I.n + 1;
  }
  I.S_lo = -I.d_beta / NREF;
  I.Ns = (I.N + 2 * I.d_beta) / NREF + 1;
  I.O_lo = -I.b;
  I.No = I.N / NREF + 2 * I.b + 1;
  if (I.levels > 2) {
    if ((I.N / NREF) % I.n) { *why = "multilevel: N/4 must be a multiple of the patch size"; return MLC_ERR_UNSUPPORTED; }
    set_level_box(&I);
    // every coarser level must be built too (derive recurses through them)
    const mlc_problem c = child_problem(I);
    mlc_plan_info C{};
    std::string cwhy;
    const mlc_status cs = derive(&c, &C, &cwhy);
    if (cs != MLC_OK) {
      *why = "multilevel, level " + std::to_string(I.levels - 2) + ": " + cwhy;
      return cs;
    }
  } else {
    I.M_coarse = pick_fft(I.Ns + I.No - 1, 2 * I.Z);
    if (I.M_coarse < 0) { *why = "coarse grid too large for the built FFT sizes / DGF table (more levels lift this)"; return MLC_ERR_UNSUPPORTED; }
  }
  const int eb = I.d_beta + NREF * I.b;
  if (I.d_beta > I.d_alpha) {
    int Wt = I.n + 2 * eb + 1;
    I.M_table = pick_fft(Wt + I.n, 2 * I.Z);
    if (I.M_table < 0) { *why = "far-field table box too large for the built FFT sizes / DGF table"; return MLC_ERR_UNSUPPORTED; }
  } else {
    I.M_table = 0;
  }
  *o = I;
  return MLC_OK;
}

extern "C" mlc_status mlc_problem_info(const mlc_problem* prob, mlc_plan_info* out) {
  std::string why;
  mlc_status s = derive(prob, out, &why);
  if (s != MLC_OK) return fail(nullptr, s, why);
  return MLC_OK;
}

extern "C" mlc_status mlc_last_error(mlc_context* ctx, char* buf, size_t len) {
  if (!buf || len == 0) return MLC_ERR_INVALID_ARG;
  if (ctx) {
    std::lock_guard<std::mutex> lk(ctx->err_mu);
    std::snprintf(buf, len, "%s", ctx->last_error.c_str());
  } else {
    std::snprintf(buf, len, "%s", g_error.c_str());
  }
  return MLC_OK;
}

// ------------------------------------------------------------- context
extern "C" mlc_status mlc_context_create(int device, size_t hbm_budget_bytes, mlc_context** out) {
  if (!out) return fail(nullptr, MLC_ERR_INVALID_ARG, "null output pointer");
  int count = 0;
  hipError_t e = hipGetDeviceCount(&count);
  if (e != hipSuccess || count <= 0) return fail(nullptr, MLC_ERR_DEVICE, "no HIP device available");
  if (device < 0 || device >= count) return fail(nullptr, MLC_ERR_INVALID_ARG, "device index out of range");
  e = hipSetDevice(device);
  if (e != hipSuccess) return fail(nullptr, MLC_ERR_DEVICE, hipGetErrorString(e));
  e = scratch_init(device);
  if (e != hipSuccess)
    return fail(nullptr, MLC_ERR_DEVICE, std::string("static scratch address: ") + hipGetErrorString(e));
  auto* c = new (std::nothrow) mlc_context;
  if (!c) return fail(nullptr, MLC_ERR_OUT_OF_MEMORY, "host allocation failed");
  c->device = device;
  c->budget = hbm_budget_bytes;
  *out = c;
  return MLC_OK;
}

extern "C" mlc_status mlc_context_destroy(mlc_context* ctx) {
  if (!ctx) return MLC_ERR_INVALID_ARG;
  hipSetDevice(ctx->device);
  for (auto& kv : ctx->side) {
    hipStreamSynchronize(kv.second.stream);
    hipStreamDestroy(kv.second.stream);
    for (hipEvent_t e : kv.second.ev) hipEventDestroy(e);
    hipFree(kv.second.check_flag);
  }
  for (auto& kv : ctx->dgf) hipFree(kv.second);
  delete ctx;
  return MLC_OK;
}

static inline unsigned blocks_for(int64_t n, int t = 256) { return unsigned((n + t - 1) / t); }
// Blocks of 256 for the grid-stride kernels over node arrays: at most 2^20
// (one launch holds fewer than 2^32 threads; (N+1)^3 reaches 8.6e9 at 2048^3)
static inline unsigned flat_blocks(int64_t n) {
  return unsigned(std::max<int64_t>(1, std::min<int64_t>((n + 255) / 256, int64_t(1) << 20)));
}

// ----------------------------------------------------- generic 3-D FFT
template <int M>
static void fft3_impl(cplx<double>* data, int dir, hipStream_t s) {
  constexpr int NL = (M % 4 == 0) ? 4 : 2;
  dim3 grid(M / NL, M);
  for (int axis = 0; axis < 3; ++axis) {
    if (dir > 0) hipLaunchKernelGGL((fft_axis_kernel<double, M, NL, 1>), grid, dim3(256), 0, s, data, axis, 0, 0, M);
    else hipLaunchKernelGGL((fft_axis_kernel<double, M, NL, -1>), grid, dim3(256), 0, s, data, axis, 0, 0, M);
  }
}
static bool fft3(cplx<double>* data, int M, int dir, hipStream_t s) {
  switch (M) {
#define CASE(MM) case MM: fft3_impl<MM>(data, dir, s); return true;
    MLC_FFT_SIZES(CASE)
#undef CASE
  }
  return false;
}

// --------------------------------------------------------- DGF table
template <int MF, int NLC>
static void dst3(double* data, int Nd, hipStream_t s) {
  dim3 grid((Nd + 2 * NLC - 1) / (2 * NLC), Nd);
  for (int axis = 0; axis < 3; ++axis)
    hipLaunchKernelGGL((dst1_axis_kernel<MF, NLC>), grid, dim3(256), 0, s, data, axis);
}

static mlc_status get_dgf(mlc_context* ctx, int Q, int Z, double** table) {
  auto key = std::make_pair(Q, Z);
  auto it = ctx->dgf.find(key);
  if (it != ctx->dgf.end()) { *table = it->second; return MLC_OK; }
  HIP_TRY(ctx, hipSetDevice(ctx->device));
  const int L = 2 * Z, Nd = 2 * L - 1, W = 2 * Z + 1;
  double* rhs = nullptr;
  double* tab = nullptr;
  const size_t tab_bytes = sizeof(double) * cube(W);
  if (!mlc_budget_take(ctx, tab_bytes)) return fail(ctx, MLC_ERR_OUT_OF_MEMORY, "DGF table exceeds the context's budget");
  if (hipMalloc(&rhs, sizeof(double) * cube(Nd)) != hipSuccess) {
    mlc_budget_give(ctx, tab_bytes);
    return fail(ctx, MLC_ERR_OUT_OF_MEMORY, "DGF work array allocation failed");
  }
  if (hipMalloc(&tab, tab_bytes) != hipSuccess) {
    hipFree(rhs);
    mlc_budget_give(ctx, tab_bytes);
    return fail(ctx, MLC_ERR_OUT_OF_MEMORY, "DGF table allocation failed");
  }
  Stencil st = stencil_of(Q);
  hipStream_t s = nullptr;
  hipLaunchKernelGGL(dgf_rhs_kernel, dim3(blocks_for(cube(Nd))), dim3(256), 0, s, rhs, L, st);
  auto run = [&](void) {
    if (L * 4 == 1024) dst3<1024, 4>(rhs, Nd, s);
    else if (L * 4 == 512) dst3<512, 8>(rhs, Nd, s);
    else dst3<256, 8>(rhs, Nd, s);
  };
  run();
  hipLaunchKernelGGL(dgf_divide_kernel, dim3(blocks_for(cube(Nd))), dim3(256), 0, s, rhs, L, st);
  run();
  hipLaunchKernelGGL(dgf_restrict_kernel, dim3(blocks_for(cube(W))), dim3(256), 0, s, rhs, tab, L, Z);
  hipError_t e = hipDeviceSynchronize();
  hipFree(rhs);
  if (e != hipSuccess) {
    hipFree(tab);
    mlc_budget_give(ctx, tab_bytes);
    return fail(ctx, MLC_ERR_DEVICE, std::string("DGF build: ") + hipGetErrorString(e));
  }
  ctx->dgf[key] = tab;
  *table = tab;
  return MLC_OK;
}

extern "C" mlc_status mlc_dgf_table(mlc_context* ctx, int32_t Q, int32_t Z, const double** table) {
  if (!ctx || !table) return fail(ctx, MLC_ERR_INVALID_ARG, "null argument");
  if (Q != 4 && Q != 6) return fail(ctx, MLC_ERR_UNSUPPORTED, "Q must be 4 or 6");
  if (Z != 32 && Z != 64 && Z != 128) return fail(ctx, MLC_ERR_UNSUPPORTED, "Z must be 32, 64 or 128");
  double* t = nullptr;
  std::lock_guard<std::mutex> lk(ctx->build_mu);
  mlc_status s = get_dgf(ctx, Q, Z, &t);
  if (s != MLC_OK) return s;
  *table = t;
  return MLC_OK;
}

// ----------------------------------------------------------------- plan
static size_t align_up(size_t v) { return (v + 255) & ~size_t(255); }

// hipMalloc of one of a plan's resident buffers, counted in table_bytes
template <typename T>
static bool plan_alloc(mlc_plan* P, T** ptr, size_t bytes) {
  if (hipMalloc(reinterpret_cast<void**>(ptr), bytes) != hipSuccess) {
    *ptr = nullptr;
    return false;
  }
  P->table_bytes += bytes;
  return true;
}

static void plan_destroy_buffers(mlc_plan* p) {
  if (p->charged) mlc_budget_give(p->ctx, p->table_bytes);
  p->charged = false;
  p->table_bytes = 0;
  hipFree(p->conv_spec);
  hipFree(p->coarse_spec);
  hipFree(p->T);
  hipFree(p->D);
  hipFree(p->Am);
  hipFree(p->Tm);
  hipFree(p->gram_inv);
  p->conv_spec = nullptr; p->coarse_spec = nullptr; p->T = nullptr; p->D = nullptr; p->Am = nullptr; p->Tm = nullptr;
  p->gram_inv = nullptr;
}

// spectrum of the periodised DGF on an M^3 torus -> real octant (fp64 work)
static mlc_status build_spectrum(mlc_context* ctx, const double* G1, int Z, int M, cplx<double>* work,
                                 double* oct64, void* octT, int Tsize, double scale, int p0, int p1, int p2) {
  hipStream_t s = nullptr;
  hipLaunchKernelGGL(fill_periodic_dgf_kernel, dim3(blocks_for(cube(M))), dim3(256), 0, s, work, G1, Z, M);
  if (!fft3(work, M, 1, s)) return fail(ctx, MLC_ERR_UNSUPPORTED, "FFT size not built");
  const int Mh = M / 2 + 1;
  if (oct64)
    hipLaunchKernelGGL(spectrum_octant_kernel<double>, dim3(blocks_for(cube(Mh))), dim3(256), 0, s, work, oct64, M,
                       scale, p0, p1, p2);
  if (octT) {
    if (Tsize == 4)
      hipLaunchKernelGGL(spectrum_octant_kernel<float>, dim3(blocks_for(cube(Mh))), dim3(256), 0, s, work,
                         (float*)octT, M, scale, p0, p1, p2);
    else
      hipLaunchKernelGGL(spectrum_octant_kernel<double>, dim3(blocks_for(cube(Mh))), dim3(256), 0, s, work,
                         (double*)octT, M, scale, p0, p1, p2);
  }
  return MLC_OK;
}

// Rows of one block of the skeleton far-field tiling used for patches of n
// cells per side (the strips of SkelTiling unless the face has fewer rows
// than one block), and the lattice points of one block (the same for both
// tilings).
static int skel_block_rows(int n) {
  return n * n >= ann_block_rows<SkelTiling>() ? ann_block_rows<SkelTiling>() : ann_block_rows<SkelTilingSmall>();
}
constexpr int kSkelCols = ann_block_cols<SkelTiling>();
// The same for the coarse-grid contraction, by q = n / 4 (q^3 rows); its two
// tilings may differ in both rows and lattice points per block.
static bool coarse_big(int q) { return q * q * q >= ann_block_rows<CoarseTiling>() && q >= 4; }
static int coarse_block_rows(int q) {
  return coarse_big(q) ? ann_block_rows<CoarseTiling>() : ann_block_rows<CoarseTilingSmall>();
}
static int coarse_block_cols(int q) {
  return coarse_big(q) ? ann_block_cols<CoarseTiling>() : ann_block_cols<CoarseTilingSmall>();
}
static_assert(ann_block_cols<SkelTilingSmall>() == kSkelCols && SkelTilingSmall::WAVES == SkelTiling::WAVES,
              "both skeleton tilings cover the same lattice points with the same waves");

// Geometry of the two far-field contractions (skeleton planes, coarse grid)
// and of the zero-padded moment lattice they share.
static void annulus_geoms(const mlc_plan_info& I, MfmaGeom* skel, MfmaGeom* coarse) {
  auto cdiv_floor = [](int a, int b) { return a >= 0 ? a / b : -((-a + b - 1) / b); };
  auto cdiv_ceil = [](int a, int b) { return a >= 0 ? (a + b - 1) / b : -((-a) / b); };
  const int n = I.n, db = I.d_beta, ppa = I.patches_per_axis, K = I.K, KP = (K + 3) / 4 * 4;
  auto rows64 = [](int r) { return (r + 63) / 64 * 64; };
  MfmaGeom& gs = *skel;
  gs = MfmaGeom{};
  // skeleton rows padded to whole blocks of the skeleton tiling (zero rows)
  const int SKR = skel_block_rows(n);
  gs.ppa = ppa; gs.K = K; gs.KP = KP; gs.nr = n * n; gs.nrp = std::max(rows64(gs.nr), (gs.nr + SKR - 1) / SKR * SKR);
  gs.e0lo = cdiv_ceil(-db, n);
  gs.ne0 = cdiv_floor(n + db, n) - gs.e0lo + 1;
  gs.elo = cdiv_ceil(-db - (n - 1), n);
  gs.ne = cdiv_floor(n + db, n) - gs.elo + 1;
  gs.nk0 = gs.nk1 = gs.nk2 = ppa + 1;
  gs.k0lo = gs.k1lo = gs.k2lo = 0;
  MfmaGeom& gc = *coarse;
  gc = MfmaGeom{};
  const int q = n / NREF, cb = db / NREF;
  const int COR = coarse_block_rows(n / NREF);
  gc.ppa = ppa; gc.K = K; gc.KP = KP; gc.nr = q * q * q; gc.nrp = std::max(rows64(gc.nr), (gc.nr + COR - 1) / COR * COR);
  gc.elo = cdiv_ceil(-cb - (q - 1), q);
  gc.ne = cdiv_floor((n + db) / NREF, q) - gc.elo + 1;
  gc.e0lo = gc.elo; gc.ne0 = gc.ne;
  gc.k0lo = gc.k1lo = gc.k2lo = cdiv_floor(I.S_lo, q);
  gc.nk0 = gc.nk1 = gc.nk2 = cdiv_floor(I.S_lo + I.Ns - 1, q) - gc.k0lo + 1;
  // padded lattice: patch coordinate k - E over both contractions, every axis
  const int emax = std::max({gs.e0lo + gs.ne0 - 1, gs.elo + gs.ne - 1, gc.elo + gc.ne - 1});
  const int emin = std::min({gs.e0lo, gs.elo, gc.elo});
  const int kmin = std::min(0, gc.k0lo), kmax = std::max(ppa, gc.k0lo + gc.nk0 - 1);
  const int padlo = std::max(emax - kmin, 0);
  const int L = std::max(kmax - emin, ppa - 1) + padlo + 1;
  gs.L = gc.L = L;
  gs.padlo = gc.padlo = padlo;
}

// Offset chunks of a problem's far-field sums: a problem whose sums cover
// too few waves to fill the chip splits its offset planes over up to ne0
// chunks, each written as partial sums and added in order by a reduction.
// The count depends on the problem alone, so a problem gives the same result
// solved alone or in a batch.
struct AnnSplit {
  int es_s = 1, es_c = 1;   // chunks: skeleton, coarse grid
  int ncb_s = 0, ncb_c = 0; // column blocks of one chunk
  size_t part = 0;          // doubles of partial sums (shared by both sums)
};
static AnnSplit ann_split(const mlc_plan_info& I) {
  AnnSplit a;
  MfmaGeom gs, gc;
  annulus_geoms(I, &gs, &gc);
  const int SK_COLS = kSkelCols, SK_ROWS = skel_block_rows(I.n);
  const int CO_COLS = coarse_block_cols(I.n / NREF), CO_ROWS = coarse_block_rows(I.n / NREF);
  // waves to aim for: with float32 convolutions the far-field sums span most
  // of the output pass beside them, so they take more of the chip (measured
  // at 256^3: 7.00 -> 6.89 ms); with float64 ones the output pass outlasts
  // them anyway and a larger share only slows it
  const int TARGET_WAVES = I.conv_precision == MLC_CONV_FP32 ? 8192 : 4096;
  const int64_t nks = int64_t(gs.nk0) * gs.nk1 * gs.nk2, nkc = int64_t(gc.nk0) * gc.nk1 * gc.nk2;
  a.ncb_s = int((nks + SK_COLS - 1) / SK_COLS);
  a.ncb_c = int((nkc + CO_COLS - 1) / CO_COLS);
  const int64_t ws = int64_t(gs.nrp / SK_ROWS) * a.ncb_s * 3 * SkelTiling::WAVES;
  static_assert(CoarseTiling::WAVES == CoarseTilingSmall::WAVES, "both coarse tilings launch the same waves");
  const int64_t wc = int64_t(gc.nrp / CO_ROWS) * a.ncb_c * CoarseTiling::WAVES;
  a.es_s = int(std::min<int64_t>(gs.ne0, std::max<int64_t>(1, (TARGET_WAVES + ws - 1) / ws)));
  a.es_c = int(std::min<int64_t>(gc.ne0, std::max<int64_t>(1, (TARGET_WAVES + wc - 1) / wc)));
  const size_t ps = a.es_s > 1 ? size_t(a.es_s) * 3 * gs.nrp * nks : 0;
  const size_t pc = a.es_c > 1 ? size_t(a.es_c) * gc.nrp * nkc : 0;
  a.part = std::max(ps, pc);
  return a;
}

static mlc_status build_tables(mlc_plan* P, const double* G1) {
  mlc_context* ctx = P->ctx;
  const mlc_plan_info& I = P->info;
  const int Mt = I.M_table, Mth = Mt / 2 + 1, K = I.K;
  hipStream_t s = nullptr;
  cplx<double>* work = nullptr;
  double* oct = nullptr;
  double* coarse = nullptr;
  double* planes = nullptr;
  const int64_t nc = cube(P->Wtc), npl = int64_t(3) * P->nplb * P->Wb * P->Wb;
  bool ok = hipMalloc(&work, sizeof(cplx<double>) * cube(Mt)) == hipSuccess &&
            hipMalloc(&oct, sizeof(double) * cube(Mth)) == hipSuccess &&
            hipMalloc(&coarse, sizeof(double) * nc) == hipSuccess &&
            hipMalloc(&planes, sizeof(double) * npl) == hipSuccess &&
            plan_alloc(P, &P->T, sizeof(double) * cube(P->Wbc) * K) &&
            plan_alloc(P, &P->D, sizeof(double) * npl * K);
  mlc_status st = MLC_OK;
  if (!ok) st = fail(ctx, MLC_ERR_OUT_OF_MEMORY, "far-field table allocation failed");
  if (st == MLC_OK) st = build_spectrum(ctx, G1, I.Z, Mt, work, oct, nullptr, 8, 1.0, 0, 1, 2);
  const double h = I.h, R = I.n * h / 2.0;
  const double scale = h * h / (double(Mt) * Mt * Mt);
  const Stencil stc = stencil_of(I.Q);
  for (int k = 0; st == MLC_OK && k < K; ++k) {
    hipMemsetAsync(work, 0, sizeof(cplx<double>) * cube(Mt), s);
    hipLaunchKernelGGL(fill_mode_source_kernel, dim3(blocks_for(cube(I.n + 1))), dim3(256), 0, s, work, Mt, I.n,
                       P->modes.p[k][0], P->modes.p[k][1], P->modes.p[k][2], std::pow(R, -1.5));
    fft3(work, Mt, 1, s);
    hipLaunchKernelGGL(mul_real_even_kernel, dim3(blocks_for(cube(Mt))), dim3(256), 0, s, work, oct, Mt);
    fft3(work, Mt, -1, s);
    hipLaunchKernelGGL(extract_mode_kernel, dim3(blocks_for(nc + npl)), dim3(256), 0, s, work, Mt, scale, I.n, P->eb,
                       I.d_beta, P->P0b, P->nplb, coarse, planes);
    hipLaunchKernelGGL(annulus_coarse_table_kernel, dim3(blocks_for(cube(P->Wbc))), dim3(256), 0, s, coarse, P->T,
                       I.n, P->eb, I.d_beta, I.d_alpha, stc, 1.0 / (I.H * I.H), K, k);
    hipLaunchKernelGGL(annulus_plane_table_kernel, dim3(blocks_for(npl)), dim3(256), 0, s, planes, coarse, P->D, I.n,
                       P->eb, I.d_beta, I.d_alpha, P->P0b, P->nplb, I.b, K, k);
  }
  if (st == MLC_OK) {
    hipError_t e = hipDeviceSynchronize();
    if (e != hipSuccess) st = fail(ctx, MLC_ERR_DEVICE, std::string("table build: ") + hipGetErrorString(e));
  }
  hipFree(work); hipFree(oct); hipFree(coarse); hipFree(planes);
  if (st != MLC_OK) return st;
  // MFMA layouts of both tables
  annulus_geoms(I, &P->mg_skel, &P->mg_coarse);
  const int n = I.n, db = I.d_beta;
  {
    const MfmaGeom& g = P->mg_skel;
    int64_t total = int64_t(3) * g.ne0 * g.ne * g.ne * (g.KP / 4) * g.nrp * 4;
    if (!plan_alloc(P, &P->Am, sizeof(double) * total))
      return fail(ctx, MLC_ERR_OUT_OF_MEMORY, "far-field MFMA table allocation failed");
    hipLaunchKernelGGL(skel_mfma_table_kernel, dim3(blocks_for(total)), dim3(256), 0, s, P->D, P->Am, n, db, P->P0b,
                       P->nplb, P->Wb, K, g);
  }
  {
    const MfmaGeom& g = P->mg_coarse;
    const int q = n / NREF;
    int64_t total = int64_t(g.ne) * g.ne * g.ne * (g.KP / 4) * g.nrp * 4;
    if (!plan_alloc(P, &P->Tm, sizeof(double) * total))
      return fail(ctx, MLC_ERR_OUT_OF_MEMORY, "far-field MFMA table allocation failed");
    hipLaunchKernelGGL(coarse_mfma_table_kernel, dim3(blocks_for(total)), dim3(256), 0, s, P->T, P->Tm, q, db,
                       P->Wbc, K, g);
  }
  hipError_t e = hipDeviceSynchronize();
  if (e != hipSuccess) return fail(ctx, MLC_ERR_DEVICE, std::string("table layout: ") + hipGetErrorString(e));
  return MLC_OK;
}

// --------------------------------------------------------- batch layout
// Plans whose patch-level work is identical (patch size, margins, P, Q, b,
// convolution precision, local torus, DGF table) form one class: the patch
// kernels of all their problems run as single launches over the
// concatenated patch list, with per-problem data reached through ProbDesc.
static bool same_class(const mlc_plan* a, const mlc_plan* b) {
  const mlc_plan_info &A = a->info, &B = b->info;
  return A.n == B.n && A.d_alpha == B.d_alpha && A.d_beta == B.d_beta && A.P == B.P && A.Q == B.Q &&
         A.b == B.b && A.conv_precision == B.conv_precision && A.M == B.M && A.Z == B.Z;
}

// Workspace of one class group, relative to the group's base:
//   descriptors (per-patch stages, far fields) | per patch (all problems):
//   moments, per-plane moment sums,
//   x-DFTs, one chunk of
//   z-transformed spectra, coarse samples, skeleton planes, Dirichlet work |
//   per problem: F^H, coarse torus (consecutive within equal M_coarse),
//   phi^H, phi^B.
struct Layout {
  size_t o_desc = 0, o_ann = 0, o_flat = 0, o_mom = 0, o_mpart = 0, o_mraw = 0, o_X = 0, o_Z = 0, o_cs = 0, o_pl = 0,
         o_dir = 0;
  size_t o_dsum = 0;   // per skeleton thread: the sum of the plane corrections
  std::vector<size_t> o_F, o_tor, o_phiH, o_phiB, o_cpad;
  std::vector<size_t> o_lf, o_lphi, o_lws;   // multilevel problems: the next level's charge, solution, workspace
  std::vector<size_t> o_ft;                  // sixth-order problems: the modified right-hand side
  std::vector<size_t> o_fbox, o_pbox;        // box problems: f and phi in the enclosing cube
  int slots = 0;                             // per-patch buffer rows (= total unless a plan keeps live patches only)
  bool compact = false;                      // the group's one plan keeps its live patches only
  size_t o_patch_of = 0, o_slot_of = 0;      // compact: slot -> patch, patch -> slot (-1: empty)
  int dir_chunk = 0;                         // n < 32: patches per three-pass Dirichlet launch
  size_t o_live = 0;                         // per patch: 1 unless skipped as empty (int)
  bool any_skip = false;                     // some problem skips empty patches
  std::vector<int> patch0;
  int total = 0, chunk = 0;
  size_t bytes = 0;
};

static const int kMaxGridY = 65535;

// MLC_CONV_CHUNK (largest patch chunk of the local convolutions), read once
// per process so that every layout of a plan agrees with its workspace size.
static int conv_chunk_override() {
  static const int v = [] {
    const char* e = std::getenv("MLC_CONV_CHUNK");
    return e ? std::max(1, std::atoi(e)) : 0;
  }();
  return v;
}

static bool is_boxed(const mlc_plan_info& I) { return I.box[0] != I.N || I.box[1] != I.N || I.box[2] != I.N; }

static Layout layout_of(const std::vector<const mlc_plan_info*>& g) {
  Layout L;
  const mlc_plan_info& I = *g[0];
  const int np = int(g.size());
  const size_t tsz = I.conv_precision == MLC_CONV_FP32 ? 4 : 8, csz = 2 * tsz;
  const int S = I.n + 1, Mh = I.M / 2 + 1, Wp = I.Wa + 2 * I.b;
  for (int k = 0; k < np; ++k) {
    L.patch0.push_back(L.total);
    L.total += g[k]->npatch;
  }
  const size_t T = size_t(L.total);
  for (int k = 0; k < np; ++k) L.slots += g[k]->slots;
  L.compact = L.slots < L.total;
  const size_t Ts = size_t(L.slots);
  size_t o = 0;
  auto take = [&](size_t bytes) { size_t at = o; o = align_up(o + bytes); return at; };
  L.o_desc = take(sizeof(ProbDesc) * np);
  L.o_ann = take(2 * sizeof(AnnProb) * np);   // far-field descriptors: skeleton, coarse
  // coarse right-hand side and skeleton descriptors
  L.o_flat = take((sizeof(CoarseRhsProb<double>) + sizeof(SkelProb<double>)) * np);
  L.o_live = take(sizeof(int) * T);
  for (int k = 0; k < np; ++k) L.any_skip = L.any_skip || g[k]->skip_empty;
  L.o_mom = take(sizeof(double) * T * I.K);
  L.o_mpart = take(sizeof(double) * Ts * S * I.P * I.P);
  if (L.compact) {
    L.o_patch_of = take(sizeof(int) * Ts);
    L.o_slot_of = take(sizeof(int) * T);
  }
  L.o_mraw = take(I.P >= 5 ? sizeof(double) * T * I.K : 0);
  // the x-DFT spectra; once the last y/z pass has read them, the same bytes
  // hold the coarse Laplacians of the patches' coarse samples (at most as
  // many bytes, since alpha <= 3)
  L.o_X = take(std::max(csz * Ts * Mh * S * S, sizeof(double) * Ts * size_t(cube(I.Wc - 2 * I.b))));
  // patch chunks of equal size whose z-transformed spectra stay within
  // 6 GB (MLC_CONV_CHUNK overrides the largest chunk): at 256^3 with 32^3
  // patches one chunk holds every patch, measured faster than two or three
  const size_t per_patch = csz * size_t(Wp) * Mh * I.M;
  int chunk = int(std::max<size_t>(1, (size_t(6) << 30) / per_patch));
  if (const int c = conv_chunk_override()) chunk = c;
  chunk = std::min(std::min(chunk, std::max(L.slots, 1)), kMaxGridY);
  const int nchunks = (std::max(L.slots, 1) + chunk - 1) / chunk;
  L.chunk = (std::max(L.slots, 1) + nchunks - 1) / nchunks;
  L.o_Z = take(per_patch * L.chunk);
  L.o_cs = take(tsz * Ts * cube(I.Wc));
  L.o_pl = take(tsz * Ts * 3 * I.nplanes_a * I.Wa * I.Wa);
  // smaller patches: the three-pass Dirichlet work array, every patch at
  // once up to 4 GB, else chunks (32^3-cell patches need none)
  if (I.n < 32) {
    const size_t per = sizeof(double) * size_t(cube(I.n - 1));
    L.dir_chunk = int(std::min<size_t>(T, std::max<size_t>(1, (size_t(4) << 30) / per)));
    L.o_dir = take(per * size_t(L.dir_chunk));
  }
  {
    size_t nsk = 0;
    for (int k = 0; k < np; ++k) nsk += size_t(3) * (g[k]->N / g[k]->n + 1) * size_t(g[k]->N + 1) * (g[k]->N + 1);
    L.o_dsum = take(sizeof(double) * nsk);
  }
  L.o_F.resize(np); L.o_tor.resize(np); L.o_phiH.resize(np); L.o_phiB.resize(np);
  for (int k = 0; k < np; ++k) L.o_F[k] = take(sizeof(double) * cube(g[k]->Ns));
  std::vector<int> done(np, 0);
  for (int k = 0; k < np; ++k) {
    if (done[k]) continue;
    const int Mc = g[k]->M_coarse;
    for (int j = k; j < np; ++j)
      if (!done[j] && g[j]->M_coarse == Mc) { L.o_tor[j] = o; o += sizeof(cplx<double>) * cube(Mc); done[j] = 1; }
    o = align_up(o);
  }
  for (int k = 0; k < np; ++k) L.o_phiH[k] = take(sizeof(double) * cube(g[k]->No));
  for (int k = 0; k < np; ++k) L.o_phiB[k] = take(sizeof(double) * cube(g[k]->N + 1));
  L.o_cpad.resize(np);
  for (int k = 0; k < np; ++k) {
    size_t bytes = 0;
    if (g[k]->d_beta > g[k]->d_alpha) {
      MfmaGeom gs, gc;
      annulus_geoms(*g[k], &gs, &gc);
      // slot-major and mode-major moment copies, the partial sums of split
      // far-field sums, then the nonzero-moment flags of the lattice slots
      bytes = 2 * sizeof(double) * cube(gs.L) * gs.KP + sizeof(double) * ann_split(*g[k]).part +
              sizeof(int) * cube(gs.L);
    }
    L.o_cpad[k] = take(bytes);
  }
  L.o_ft.assign(np, 0);
  for (int k = 0; k < np; ++k)
    if (g[k]->rhs_order == 6) L.o_ft[k] = take(sizeof(double) * cube(g[k]->N + 1));
  L.o_fbox.assign(np, 0);
  L.o_pbox.assign(np, 0);
  for (int k = 0; k < np; ++k)
    if (is_boxed(*g[k])) {
      L.o_fbox[k] = take(sizeof(double) * cube(g[k]->N + 1));
      L.o_pbox[k] = take(sizeof(double) * cube(g[k]->N + 1));
    }
  L.o_lf.assign(np, 0); L.o_lphi.assign(np, 0); L.o_lws.assign(np, 0);
  for (int k = 0; k < np; ++k) {
    if (g[k]->levels <= 2) continue;
    const mlc_plan_info C = level_info(*g[k]);
    L.o_lf[k] = take(sizeof(double) * cube(C.N + 1));
    L.o_lphi[k] = take(sizeof(double) * cube(C.N + 1));
    L.o_lws[k] = take(layout_of({&C}).bytes);
  }
  L.bytes = o;
  return L;
}

static std::vector<const mlc_plan_info*> infos_of(const std::vector<mlc_plan*>& g) {
  std::vector<const mlc_plan_info*> v;
  for (const mlc_plan* p : g) v.push_back(&p->info);
  return v;
}

extern "C" mlc_status mlc_problem_workspace_bytes(const mlc_problem* prob, size_t* bytes) {
  if (!prob || !bytes) return fail(nullptr, MLC_ERR_INVALID_ARG, "null argument");
  mlc_plan_info I{};
  std::string why;
  mlc_status s = derive(prob, &I, &why);
  if (s != MLC_OK) return fail(nullptr, s, why);
  *bytes = layout_of({&I}).bytes;
  if (prob->fft_size == -1) {
    // the autotuner may pick any built torus the problem admits: the figure
    // is the largest of their layouts, so that it bounds the plan's own
    const int Mmin = 2 * (I.n + I.e) + 1;
    for (int M : kFftSizes) {
      if (M < Mmin || M / 2 > I.Z || !conv_size_ok(I.conv_precision, I.n, M)) continue;
      mlc_plan_info J = I;
      J.M = M;
      *bytes = std::max(*bytes, layout_of({&J}).bytes);
    }
  }
  return MLC_OK;
}

// Inverse of the Boole Gram matrix of the modes (sec. 3 projection in the
// discrete inner product of the composite Boole rule): G[r][s] =
// prod_d g1(p_r,d, p_s,d), g1(a, b) = sum_j w_j qhat_a(t_j) qhat_b(t_j); Gauss-Jordan
// elimination with partial pivoting (G is symmetric positive definite and
// close to the identity).  Row-major K x K.
static bool gram_inverse(int n, int P, const ModeList& m, std::vector<double>* out) {
  std::vector<double> g1(size_t(P) * P, 0.0);
  for (int a = 0; a < P; ++a)
    for (int b = 0; b < P; ++b) {
      double acc = 0.0;
      for (int j = 0; j <= n; ++j) {
        const double t = (j - 0.5 * n) / (0.5 * n);
        acc += boole_w(j, n) * qhat(a, t) * qhat(b, t);
      }
      g1[size_t(a) * P + b] = acc;
    }
  const int K = m.K;
  std::vector<double> A(size_t(K) * 2 * K, 0.0);   // [G | I]
  for (int r = 0; r < K; ++r) {
    for (int c = 0; c < K; ++c)
      A[size_t(r) * 2 * K + c] = g1[size_t(m.p[r][0]) * P + m.p[c][0]] * g1[size_t(m.p[r][1]) * P + m.p[c][1]] *
                                 g1[size_t(m.p[r][2]) * P + m.p[c][2]];
    A[size_t(r) * 2 * K + K + r] = 1.0;
  }
  for (int c = 0; c < K; ++c) {
    int piv = c;
    for (int r = c + 1; r < K; ++r)
      if (std::fabs(A[size_t(r) * 2 * K + c]) > std::fabs(A[size_t(piv) * 2 * K + c])) piv = r;
    if (!(std::fabs(A[size_t(piv) * 2 * K + c]) > 0.0)) return false;
    if (piv != c)
      for (int j = 0; j < 2 * K; ++j) std::swap(A[size_t(c) * 2 * K + j], A[size_t(piv) * 2 * K + j]);
    const double d = A[size_t(c) * 2 * K + c];
    for (int j = 0; j < 2 * K; ++j) A[size_t(c) * 2 * K + j] /= d;
    for (int r = 0; r < K; ++r) {
      if (r == c) continue;
      const double f = A[size_t(r) * 2 * K + c];
      if (f == 0.0) continue;
      for (int j = 0; j < 2 * K; ++j) A[size_t(r) * 2 * K + j] -= f * A[size_t(c) * 2 * K + j];
    }
  }
  out->assign(size_t(K) * K, 0.0);
  for (int r = 0; r < K; ++r)
    for (int c = 0; c < K; ++c) (*out)[size_t(r) * K + c] = A[size_t(r) * 2 * K + K + c];
  return true;
}

static std::pair<int, int> autotune_conv(mlc_context* ctx, const mlc_plan_info& I, const double* G1);

static void plan_free(mlc_plan* plan);

// Builds a plan (the context's build lock held); `correct` = false for the
// coarser levels of a multilevel plan, which return the uncorrected
// solution.
static mlc_status plan_create_impl(mlc_context* ctx, const mlc_problem* prob, bool correct, mlc_plan** out) {
  std::string why;
  mlc_plan_info I{};
  mlc_status s = derive(prob, &I, &why);
  if (s != MLC_OK) return fail(ctx, s, why);
  auto* P = new (std::nothrow) mlc_plan;
  if (!P) return fail(ctx, MLC_ERR_OUT_OF_MEMORY, "host allocation failed");
  P->ctx = ctx;
  P->prob = *prob;
  P->info = I;
  P->correct = correct;
  P->S = I.n + 1;
  P->Mh = I.M / 2 + 1;
  P->Wp = I.Wa + 2 * I.b;
  P->P0 = -((I.d_alpha / I.n) * I.n);
  P->eb = I.d_beta + NREF * I.b;
  P->Wtc = (I.n + 2 * P->eb) / NREF + 1;
  P->Wb = I.n + 2 * I.d_beta + 1;
  P->Wbc = (I.n + 2 * I.d_beta) / NREF + 1;
  P->P0b = -((I.d_beta / I.n) * I.n);
  P->nplb = (I.n + I.d_beta - P->P0b) / I.n + 1;
  P->Kann = I.d_beta > I.d_alpha ? I.K : 0;
  P->modes = mode_list(I.P);
  P->lagw = make_lagw(I.b);
  double* G1 = nullptr;
  s = get_dgf(ctx, I.Q, I.Z, &G1);
  if (s != MLC_OK) { delete P; return s; }
  if (prob->fft_size == -1) {
    const std::pair<int, int> t = autotune_conv(ctx, I, G1);
    if (t.first < 0) { delete P; return fail(ctx, MLC_ERR_DEVICE, "local FFT autotune failed"); }
    I.M = t.first;
    I.out_planes = t.second;
    P->info = I;
    P->Mh = I.M / 2 + 1;
  }
  const int tsz = I.conv_precision == MLC_CONV_FP32 ? 4 : 8;
  // local-convolution spectrum: layout [kx][ky'][kz'] (kx: fastest array axis)
  {
    cplx<double>* work = nullptr;
    const int M = I.M, Mh = P->Mh;
    if (hipMalloc(&work, sizeof(cplx<double>) * cube(M)) != hipSuccess ||
        !plan_alloc(P, &P->conv_spec, size_t(tsz) * cube(Mh))) {
      hipFree(work);
      plan_destroy_buffers(P);
      delete P;
      return fail(ctx, MLC_ERR_OUT_OF_MEMORY, "spectrum allocation failed");
    }
    s = build_spectrum(ctx, G1, I.Z, M, work, nullptr, P->conv_spec, tsz, 1.0 / (double(M) * M * M), 2, 1, 0);
    if (s == MLC_OK && I.M_coarse > 0) {
      // coarse spectrum (fp64 octant, layout k0 k1 k2)
      const int Mc = I.M_coarse, Mch = Mc / 2 + 1;
      cplx<double>* cw = nullptr;
      if (hipMalloc(&cw, sizeof(cplx<double>) * cube(Mc)) != hipSuccess ||
          !plan_alloc(P, &P->coarse_spec, sizeof(double) * cube(Mch))) {
        s = fail(ctx, MLC_ERR_OUT_OF_MEMORY, "coarse spectrum allocation failed");
      } else {
        s = build_spectrum(ctx, G1, I.Z, Mc, cw, P->coarse_spec, nullptr, 8, 1.0, 0, 1, 2);
      }
      hipError_t e = hipDeviceSynchronize();
      hipFree(cw);
      if (s == MLC_OK && e != hipSuccess) s = fail(ctx, MLC_ERR_DEVICE, hipGetErrorString(e));
    }
    hipFree(work);
    if (s != MLC_OK) { plan_destroy_buffers(P); delete P; return s; }
  }
  if (P->Kann > 0) {
    s = build_tables(P, G1);
    if (s != MLC_OK) { plan_destroy_buffers(P); delete P; return s; }
  }
  if (I.P >= 5) {
    std::vector<double> gi;
    if (!gram_inverse(I.n, I.P, P->modes, &gi)) {
      plan_destroy_buffers(P);
      delete P;
      return fail(ctx, MLC_ERR_UNSUPPORTED, "singular Boole Gram matrix of the Legendre modes");
    }
    if (!plan_alloc(P, &P->gram_inv, sizeof(double) * gi.size()) ||
        hipMemcpy(P->gram_inv, gi.data(), sizeof(double) * gi.size(), hipMemcpyHostToDevice) != hipSuccess) {
      plan_destroy_buffers(P);
      delete P;
      return fail(ctx, MLC_ERR_OUT_OF_MEMORY, "Gram matrix upload failed");
    }
  }
  // workspace layout (a batch of one)
  {
    Layout L = layout_of({&P->info});
    P->o_mom = L.o_mom;
    P->o_cs = L.o_cs;
    P->o_pl = L.o_pl;
    P->o_F = L.o_F[0];
    P->o_phiH = L.o_phiH[0];
    P->o_phiB = L.o_phiB[0];
    P->o_lf = L.o_lf[0];
    P->o_lphi = L.o_lphi[0];
    P->o_lws = L.o_lws[0];
    P->o_ft = L.o_ft[0];
    P->ws_total = L.bytes;
  }
  if (!mlc_budget_take(ctx, P->table_bytes)) {
    plan_destroy_buffers(P);
    delete P;
    return fail(ctx, MLC_ERR_OUT_OF_MEMORY, "plan tables exceed the context's budget");
  }
  P->charged = true;
  if (I.levels > 2) {
    // the next coarser level: the same method on the level box at spacing
    // Nref h with that level's inner radius
    const mlc_problem c = child_problem(I);
    s = plan_create_impl(ctx, &c, false, &P->child);
    if (s != MLC_OK) {
      plan_free(P);
      return s;
    }
  }
  *out = P;
  return MLC_OK;
}

extern "C" mlc_status mlc_plan_create(mlc_context* ctx, const mlc_problem* prob, mlc_plan** out) {
  if (!ctx || !prob || !out) return fail(ctx, MLC_ERR_INVALID_ARG, "null argument");
  HIP_TRY(ctx, hipSetDevice(ctx->device));
  std::lock_guard<std::mutex> lk(ctx->build_mu);
  return plan_create_impl(ctx, prob, true, out);
}

static void drain_timing(const mlc_plan* P) {
  for (auto& pe : P->pending) {
    hipEventSynchronize(pe.b);
    float ms = 0.f;
    hipEventElapsedTime(&ms, pe.a, pe.b);
    bool found = false;
    for (auto& kv : P->acc)
      if (kv.first == pe.name) { kv.second.first += 1; kv.second.second += ms; found = true; break; }
    if (!found) P->acc.push_back({pe.name, {1, double(ms)}});
    P->event_pool.push_back(pe.a);
    P->event_pool.push_back(pe.b);
  }
  P->pending.clear();
}

extern "C" mlc_status mlc_plan_set_timing(mlc_plan* plan, int32_t enable) {
  if (!plan) return fail(nullptr, MLC_ERR_INVALID_ARG, "null plan");
  drain_timing(plan);
  plan->acc.clear();
  plan->timing_on = enable != 0;
  return MLC_OK;
}

extern "C" mlc_status mlc_plan_timing(mlc_plan* plan, mlc_kernel_time* out, int32_t max, int32_t* count) {
  if (!plan || !count || (max > 0 && !out)) return fail(plan ? plan->ctx : nullptr, MLC_ERR_INVALID_ARG, "bad argument");
  drain_timing(plan);
  int k = 0;
  for (auto& kv : plan->acc) {
    if (k < max) {
      std::snprintf(out[k].name, sizeof(out[k].name), "%s", kv.first.c_str());
      out[k].launches = kv.second.first;
      out[k].total_ms = kv.second.second;
    }
    ++k;
  }
  *count = k;
  return MLC_OK;
}

static void plan_free(mlc_plan* plan) {
  if (plan->child) plan_free(plan->child);
  drain_timing(plan);
  for (hipEvent_t e : plan->event_pool) hipEventDestroy(e);
  plan_destroy_buffers(plan);
  delete plan;
}

extern "C" mlc_status mlc_plan_destroy(mlc_plan* plan) {
  if (!plan) return MLC_ERR_INVALID_ARG;
  hipSetDevice(plan->ctx->device);
  plan_free(plan);
  return MLC_OK;
}

extern "C" mlc_status mlc_plan_coarse_level(const mlc_plan* plan, const mlc_plan** level) {
  if (!plan || !level) return fail(nullptr, MLC_ERR_INVALID_ARG, "null argument");
  if (!plan->child) return fail(plan->ctx, MLC_ERR_INVALID_ARG, "a two-level plan has no coarser level");
  *level = plan->child;
  return MLC_OK;
}

extern "C" mlc_status mlc_plan_get_info(const mlc_plan* plan, mlc_plan_info* out) {
  if (!plan || !out) return MLC_ERR_INVALID_ARG;
  *out = plan->info;
  return MLC_OK;
}

extern "C" mlc_status mlc_plan_workspace_bytes(const mlc_plan* plan, size_t* bytes) {
  if (!plan || !bytes) return MLC_ERR_INVALID_ARG;
  *bytes = plan->ws_total;
  return MLC_OK;
}

extern "C" mlc_status mlc_workspace_view(const mlc_plan* plan, void* ws, int32_t which, void** ptr,
                                         size_t* bytes) {
  if (!plan || !ws || !ptr) return MLC_ERR_INVALID_ARG;
  const mlc_plan_info& I = plan->info;
  const size_t tsz = I.conv_precision == MLC_CONV_FP32 ? 4 : 8;
  char* b = static_cast<char*>(ws);
  size_t at = 0, len = 0;
  switch (which) {
    case MLC_VIEW_MOMENTS: at = plan->o_mom; len = sizeof(double) * I.npatch * I.K; break;
    case MLC_VIEW_COARSE_RHS: at = plan->o_F; len = sizeof(double) * cube(I.Ns); break;
    case MLC_VIEW_COARSE_PHI: at = plan->o_phiH; len = sizeof(double) * cube(I.No); break;
    case MLC_VIEW_BOUNDARY: at = plan->o_phiB; len = sizeof(double) * cube(I.N + 1); break;
    case MLC_VIEW_LOCAL_COARSE: at = plan->o_cs; len = tsz * I.slots * cube(I.Wc); break;
    case MLC_VIEW_LOCAL_PLANES: at = plan->o_pl; len = tsz * I.slots * 3 * I.nplanes_a * I.Wa * I.Wa; break;
    case MLC_VIEW_LEVEL_CHARGE:
    case MLC_VIEW_LEVEL_PHI:
    case MLC_VIEW_LEVEL_WORKSPACE:
      if (!plan->child) return fail(plan->ctx, MLC_ERR_INVALID_ARG, "a two-level plan has no coarser level");
      at = which == MLC_VIEW_LEVEL_CHARGE ? plan->o_lf : (which == MLC_VIEW_LEVEL_PHI ? plan->o_lphi : plan->o_lws);
      len = which == MLC_VIEW_LEVEL_WORKSPACE ? plan->child->ws_total : sizeof(double) * cube(I.level_N + 1);
      break;
    case MLC_VIEW_CHARGE:
      if (I.rhs_order != 6) return fail(plan->ctx, MLC_ERR_INVALID_ARG, "only a sixth-order plan keeps its charge");
      at = plan->o_ft;
      len = sizeof(double) * cube(I.N + 1);
      break;
    default: return fail(plan->ctx, MLC_ERR_INVALID_ARG, "unknown workspace view");
  }
  *ptr = b + at;
  if (bytes) *bytes = len;
  return MLC_OK;
}

// ---------------------------------------------------------------- solve
// One class group of a batch, enqueued on one stream.
struct Group {
  std::vector<mlc_plan*> plans;
  std::vector<int> pos;   // positions of the problems in the caller's batch
  std::vector<const double*> f;
  std::vector<double*> phi;
  Layout L;
  size_t off = 0;         // the group's region of the workspace
  char* ws = nullptr;
  ProbDesc* desc = nullptr;
  bool one_stream = false;   // every stage on the caller's stream (no side stream)
  mutable int nslots = -1;   // slots in use this solve (the live patches when compact)
};

// Coarse Hockney convolution of a batch of nb tori with the real-even
// spectrum `oct` (octant layout): forward along axes 2 and 1, one sweep along
// axis 0 (forward, product, inverse), inverse along axes 1 and 2.  Forward:
// the source occupies slots [0, ns)^3, so the axis-2 pass skips lines outside
// [0, ns)^2 and the axis-1 pass slabs k0 >= ns (all zero).  Inverse: only
// slots (o0 + [0, no)) mod M of each axis are read afterwards, so the axis-1
// pass is limited to those k0 and the axis-2 pass to those (k0, k1).
template <int M>
static void conv3_coarse_impl(cplx<double>* data, const double* oct, int nb, int ns, int o0, int no,
                              hipStream_t s) {
  constexpr int NL = (M % 4 == 0) ? 4 : 2;
  auto blocks = [](int cnt) { return unsigned((cnt + NL - 1) / NL); };
  hipLaunchKernelGGL((fft_axis_kernel<double, M, NL, 1>), dim3(blocks(ns), ns, nb), dim3(256), 0, s, data, 2, 0, 0, ns);
  hipLaunchKernelGGL((fft_axis_kernel<double, M, NL, 1>), dim3(blocks(M), ns, nb), dim3(256), 0, s, data, 1, 0, 0, M);
  hipLaunchKernelGGL((fft_axis0_conv_kernel<double, M, NL>), dim3(blocks(M), M, nb), dim3(256), 0, s, data, oct);
  hipLaunchKernelGGL((fft_axis_kernel<double, M, NL, -1>), dim3(blocks(M), no, nb), dim3(256), 0, s, data, 1, o0, 0, M);
  hipLaunchKernelGGL((fft_axis_kernel<double, M, NL, -1>), dim3(blocks(no), no, nb), dim3(256), 0, s, data, 2, o0, o0,
                     no);
}
static bool conv3_coarse(cplx<double>* data, const double* oct, int M, int nb, int ns, int o0, int no, hipStream_t s) {
  // the passes index lines o0 .. o0 + no - 1 and 0 .. ns - 1 of each torus
  if (o0 < 0 || no < 1 || o0 + no > M || ns < 1 || ns > M) return false;
  switch (M) {
#define CASE(MM) case MM: conv3_coarse_impl<MM>(data, oct, nb, ns, o0, no, s); return true;
    MLC_FFT_SIZES(CASE)
#undef CASE
  }
  return false;
}

// Descriptor tables travel as kernel arguments, FLAT_PACK at a time.
template <typename D>
static void upload_flat(D* dst, const std::vector<D>& v, hipStream_t s) {
  for (size_t k0 = 0; k0 < v.size(); k0 += FLAT_PACK) {
    FlatPack<D> pk{};
    pk.count = int(std::min<size_t>(FLAT_PACK, v.size() - k0));
    for (int j = 0; j < pk.count; ++j) pk.d[j] = v[k0 + j];
    hipLaunchKernelGGL(flat_upload_kernel<D>, dim3(1), dim3(FLAT_PACK), 0, s, dst + k0, pk);
  }
}

// The charge the method solves for member k: f, or for a sixth-order problem
// the modified right-hand side in the workspace (written by launch_sixth_rhs).
static const double* input_of(const Group& G, int k) {
  if (is_boxed(G.plans[k]->info)) return reinterpret_cast<const double*>(G.ws + G.L.o_fbox[k]);
  return G.f[k];
}
static const double* charge_of(const Group& G, int k) {
  if (G.plans[k]->info.rhs_order == 6) return reinterpret_cast<const double*>(G.ws + G.L.o_ft[k]);
  return input_of(G, k);
}
// where the solve writes phi: the caller's array, or for a box problem the
// enclosing cube's (copied out by launch_box_out)
static double* phi_of(const Group& G, int k) {
  if (is_boxed(G.plans[k]->info)) return reinterpret_cast<double*>(G.ws + G.L.o_pbox[k]);
  return G.phi[k];
}
// box problems: f into the zeroed enclosing cube, and phi back out of it
static void launch_box_in(const Group& G, hipStream_t s) {
  for (size_t k = 0; k < G.plans.size(); ++k) {
    const mlc_plan_info& I = G.plans[k]->info;
    if (!is_boxed(I)) continue;
    double* fc = const_cast<double*>(input_of(G, int(k)));
    const int64_t nc = cube(I.N + 1);
    hipLaunchKernelGGL(fill_zero_kernel, dim3(flat_blocks(nc)), dim3(256), 0, s, fc, nc);
    const int64_t nb = int64_t(I.box[0] + 1) * (I.box[1] + 1) * (I.box[2] + 1);
    hipLaunchKernelGGL(box3_copy_kernel, dim3(flat_blocks(nb)), dim3(256), 0, s, G.f[k], I.box[0] + 1, I.box[1] + 1,
                       I.box[2] + 1, fc, I.N + 1, I.N + 1, I.N + 1, I.box[0] + 1, I.box[1] + 1, I.box[2] + 1);
  }
}
static void launch_box_out(const Group& G, hipStream_t s) {
  for (size_t k = 0; k < G.plans.size(); ++k) {
    const mlc_plan_info& I = G.plans[k]->info;
    if (!is_boxed(I)) continue;
    const int64_t nb = int64_t(I.box[0] + 1) * (I.box[1] + 1) * (I.box[2] + 1);
    hipLaunchKernelGGL(box3_copy_kernel, dim3(flat_blocks(nb)), dim3(256), 0, s, phi_of(G, int(k)), I.N + 1, I.N + 1,
                       I.N + 1, G.phi[k], I.box[0] + 1, I.box[1] + 1, I.box[2] + 1, I.box[0] + 1, I.box[1] + 1,
                       I.box[2] + 1);
  }
}
// C2 h^2 of the final correction (sec. 4.1): none at the coarser levels of a
// multilevel solve, none for the sixth-order right-hand side
static double final_c2h2(const mlc_plan& P) {
  return (P.correct && P.info.rhs_order != 6) ? P.info.h * P.info.h / 12.0 : 0.0;
}
// per-patch live flags of the group (nullptr when no member skips empty patches)
// Per-patch flags of which patches carry charge, for kernels indexed by
// patch; none when no problem skips, or when the buffers hold the live
// patches only (every slot then is live).
static const int* live_of(const Group& G) {
  return G.L.any_skip && !G.L.compact ? reinterpret_cast<const int*>(G.ws + G.L.o_live) : nullptr;
}
// Rows of the per-patch buffers in use: every patch, or the live ones
static int slots_in_use(const Group& G) { return G.L.compact ? G.nslots : G.L.total; }
static const int* patch_of_slot(const Group& G) {
  return G.L.compact ? reinterpret_cast<const int*>(G.ws + G.L.o_patch_of) : nullptr;
}
static const int* slot_of_patch(const Group& G) {
  return G.L.compact ? reinterpret_cast<const int*>(G.ws + G.L.o_slot_of) : nullptr;
}
static void launch_sixth_rhs(const Group& G, hipStream_t s) {
  for (size_t k = 0; k < G.plans.size(); ++k) {
    const mlc_plan_info& I = G.plans[k]->info;
    if (I.rhs_order != 6) continue;
    hipLaunchKernelGGL(sixth_rhs_kernel, dim3(flat_blocks(cube(I.N + 1))), dim3(256), 0, s, input_of(G, int(k)), I.N,
                       const_cast<double*>(charge_of(G, int(k))));
  }
}

static void upload_descs(const Group& G, hipStream_t s) {
  const int np = int(G.plans.size());
  for (int k0 = 0; k0 < np; k0 += DESC_PACK) {
    DescPack pk{};
    pk.count = std::min(DESC_PACK, np - k0);
    for (int j = 0; j < pk.count; ++j) {
      const int k = k0 + j;
      const mlc_plan_info& I = G.plans[k]->info;
      ProbDesc& d = pk.d[j];
      d.f = charge_of(G, k);
      d.phi = phi_of(G, k);
      d.phiB = reinterpret_cast<double*>(G.ws + G.L.o_phiB[k]);
      d.N = I.N;
      d.ppa = I.patches_per_axis;
      d.patch0 = G.L.patch0[k];
      d.h2 = I.h * I.h;
      d.R15 = std::pow(I.n * I.h / 2.0, 1.5);
      d.c2h2 = final_c2h2(*G.plans[k]);
      d.skip = I.skip_empty;
    }
    hipLaunchKernelGGL(desc_upload_kernel, dim3(1), dim3(DESC_PACK), 0, s, G.desc + k0, pk);
  }
}

// phase 0: x-DFTs (and the per-plane moment sums); phase 1: the rest, in
// patch chunks, calling after_yz (if set) once the first chunk's y/z pass
// is enqueued
template <typename T, int n, int M>
static void launch_conv(const Group& G, hipStream_t s, int phase, const std::function<void()>* after_yz) {
  const mlc_plan* P = G.plans[0];
  const mlc_plan_info& I = P->info;
  const Layout& L = G.L;
  const int np = int(G.plans.size());
  cplx<T>* X = reinterpret_cast<cplx<T>*>(G.ws + L.o_X);
  cplx<T>* Zb = reinterpret_cast<cplx<T>*>(G.ws + L.o_Z);
  T* cs = reinterpret_cast<T*>(G.ws + L.o_cs);
  T* pl = reinterpret_cast<T*>(G.ws + L.o_pl);
  // which patches carry charge (only when some problem skips empty ones and
  // the buffers hold every patch; compact buffers were filled by compact_live)
  int* live = const_cast<int*>(live_of(G));
  const int* pof = patch_of_slot(G);
  const int ns = slots_in_use(G);
  if (phase == 0) {
    if (live) {
      TimedScope ts(P, s, "patch_live");
      hipLaunchKernelGGL(patch_live_kernel, dim3(L.total), dim3(256), 0, s, G.desc, np, I.n, live, 0);
    }
    TimedScope ts(P, s, "conv_xdft");
    for (int p0 = 0; p0 < ns; p0 += kMaxGridY)
      hipLaunchKernelGGL((conv_xdft_kernel<T, M>), dim3(P->S, std::min(kMaxGridY, ns - p0)), dim3(256), 0, s,
                         G.desc, np, I.n, I.P, X, reinterpret_cast<double*>(G.ws + L.o_mpart), live, pof, p0);
  }
  if (phase == 0) return;
  OutGeom g{I.n, I.e, I.d_alpha, I.b, I.Wa, P->Wp, I.Wc, P->P0, I.nplanes_a};
  // patches in chunks: the chunk's z-transformed spectra (Zb) stay small
  // enough to be re-read from the last-level cache
  if (ns == 0 && after_yz) (*after_yz)();   // no live patch: nothing to convolve
  for (int p0 = 0; p0 < ns; p0 += L.chunk) {
    const int cnt = std::min(L.chunk, ns - p0);
    {
      TimedScope ts(P, s, "conv_yz");
      hipLaunchKernelGGL((conv_yz_kernel<T, n, M>), dim3(P->Mh, cnt), dim3(256), 0, s, X,
                         static_cast<const T*>(P->conv_spec), Zb, P->Wp, I.b, I.Wa, I.e, I.d_alpha, live, p0);
    }
    if (p0 == 0 && after_yz) (*after_yz)();
    {
      TimedScope ts(P, s, "conv_out");
      const int zpb = I.out_planes;
      constexpr int kspl = OutBatch<T, M>::KSPL;
      if (kspl > 1) {
        // the blocks of a plane add their partial outputs: start from zero
        const int64_t nc = cube(I.Wc), npl = int64_t(3) * I.nplanes_a * I.Wa * I.Wa;
        hipLaunchKernelGGL(fill_zero_t_kernel<T>, dim3(flat_blocks(nc * cnt)), dim3(256), 0, s, cs + p0 * nc, nc * cnt);
        hipLaunchKernelGGL(fill_zero_t_kernel<T>, dim3(flat_blocks(npl * cnt)), dim3(256), 0, s, pl + p0 * npl,
                           npl * cnt);
      }
      const dim3 grid((P->Wp + zpb - 1) / zpb * kspl, cnt);
      if (zpb == 1)
        hipLaunchKernelGGL((conv_out_kernel<T, n, M, false>), grid, dim3(OutBatch<T, M, false>::NT), 0, s, Zb, cs, pl, g,
                           G.desc, np, live, pof, p0, 1);
      else
        hipLaunchKernelGGL((conv_out_kernel<T, n, M, true>), grid, dim3(OutBatch<T, M, true>::NT), 0, s, Zb, cs, pl, g,
                           G.desc, np, live, pof, p0, zpb);
    }
  }
}

template <typename T>
static bool dispatch_conv(const Group& G, hipStream_t s, int phase,
                          const std::function<void()>* after_yz = nullptr) {
  const int n = G.plans[0]->info.n, M = G.plans[0]->info.M;
#define CASE(nn, MM) if (n == nn && M == MM) { launch_conv<T, nn, MM>(G, s, phase, after_yz); return true; }
  if constexpr (sizeof(T) == 4) { MLC_CONV_SIZES_F32(CASE) }
  else { MLC_CONV_SIZES_F64(CASE) }
#undef CASE
  return false;
}

// Stages after the local convolutions' x-DFTs:
//   FAR:    far-field sums (moments only) -- overlaps the convolutions
//   COARSE: coarse right-hand side and coarse solve (coarse samples)
//   PLANES: plane corrections delta_i (local fields on the planes)
//   FINISH: skeleton boundary values, Dirichlet solves and correction
enum Stage { FAR, COARSE, PLANES, FINISH };

struct AnalyticInput;
static mlc_status enqueue_group(const Group& G, hipStream_t s, const AnalyticInput* an = nullptr);

template <typename T>
static mlc_status launch_rest(const Group& G, hipStream_t s, Stage stage) {
  const mlc_plan* P0 = G.plans[0];
  const mlc_plan_info& I0 = P0->info;
  const Layout& L = G.L;
  const int np = int(G.plans.size());
  const Stencil st = stencil_of(I0.Q);
  const T* cs = reinterpret_cast<const T*>(G.ws + L.o_cs);
  T* pl = reinterpret_cast<T*>(G.ws + L.o_pl);
  const double* mom = reinterpret_cast<const double*>(G.ws + L.o_mom);
  auto F_of = [&](int k) { return reinterpret_cast<double*>(G.ws + L.o_F[k]); };
  auto tor_of = [&](int k) { return reinterpret_cast<cplx<double>*>(G.ws + L.o_tor[k]); };
  auto phiH_of = [&](int k) { return reinterpret_cast<double*>(G.ws + L.o_phiH[k]); };
  auto phiB_of = [&](int k) { return reinterpret_cast<double*>(G.ws + L.o_phiB[k]); };
  const int64_t csz = cube(I0.Wc), plsz = int64_t(3) * I0.nplanes_a * I0.Wa * I0.Wa;
  if (stage == FAR) {
    // F^H starts at zero: the coarse far-field sums and the inner part add
    for (int k = 0; k < np; ++k)
      hipLaunchKernelGGL(fill_zero_kernel, dim3(flat_blocks(cube(G.plans[k]->info.Ns))), dim3(256), 0, s, F_of(k),
                         cube(G.plans[k]->info.Ns));
  }
  // coarse right-hand side, every problem in one launch
  if (stage == COARSE) {
    auto* pr = reinterpret_cast<CoarseRhsProb<T>*>(G.ws + L.o_flat);
    // coarse Laplacians of every patch's coarse samples, in the x-DFT region
    // (free once the convolutions are done)
    double* lap = reinterpret_cast<double*>(G.ws + L.o_X);
    const int Li = I0.Wc - 2 * I0.b;
    const int64_t lsz = cube(Li);
    std::vector<CoarseRhsProb<T>> v(np);
    int64_t total = 0;
    for (int k = 0; k < np; ++k) {
      const mlc_plan* P = G.plans[k];
      const mlc_plan_info& I = P->info;
      CoarseGeom cg{I.n, I.patches_per_axis, P->Kann, I.d_alpha, I.d_beta, I.e, I.Wc, I.S_lo, I.Ns, P->Wbc,
                    1.0 / (I.H * I.H)};
      v[k] = CoarseRhsProb<T>{lap + L.patch0[k] * lsz, F_of(k), cg, total, slot_of_patch(G)};
      total += cube(I.Ns);
    }
    upload_flat(pr, v, s);
    {
      TimedScope ts(P0, s, "coarse_lap");
      const size_t lds = 3 * sizeof(T) * size_t(I0.Wc) * I0.Wc;   // <= 26 KB (Wc <= 33)
      const int ns = slots_in_use(G);
      for (int p0 = 0; p0 < ns; p0 += kMaxGridY)
        hipLaunchKernelGGL(coarse_lap_kernel<T>, dim3(Li, std::min(kMaxGridY, ns - p0)), dim3(256), lds, s, cs, lap,
                           I0.Wc, I0.b, st, live_of(G), p0);
    }
    TimedScope ts(P0, s, "coarse_rhs");
    hipLaunchKernelGGL(coarse_rhs_kernel<T>, dim3(blocks_for(total)), dim3(256), 0, s, pr, np, total, I0.b);
  }
  // padded moment lattices: slot-major (skeleton sums), then mode-major (coarse sums)
  auto cpad_s = [&](int k) { return reinterpret_cast<double*>(G.ws + L.o_cpad[k]); };
  auto cpad_p = [&](int k) {
    const MfmaGeom& g = G.plans[k]->mg_coarse;
    return reinterpret_cast<double*>(G.ws + L.o_cpad[k]) + cube(g.L) * g.KP;
  };
  const int SK_COLS = kSkelCols, SK_ROWS = skel_block_rows(I0.n);
  const int CO_COLS = coarse_block_cols(I0.n / NREF), CO_ROWS = coarse_block_rows(I0.n / NREF);
  // far-field sums of every problem in one launch per contraction
  if (stage == FAR && P0->Kann > 0) {
    AnnProb* ap_s = reinterpret_cast<AnnProb*>(G.ws + L.o_ann);
    AnnProb* ap_c = ap_s + np;
    std::vector<AnnProb> vs(np), vc(np);
    int bs = 0, bc = 0;
    int64_t rs = 0, rc = 0;   // threads of the reductions
    for (int k = 0; k < np; ++k) {
      const mlc_plan* P = G.plans[k];
      const mlc_plan_info& I = P->info;
      const MfmaGeom& gs = P->mg_skel;
      const MfmaGeom& gc = P->mg_coarse;
      const AnnSplit sp = ann_split(I);
      double* part = cpad_s(k) + 2 * cube(gs.L) * gs.KP;
      // plans that skip empty patches also skip zero source patches here
      const int* nzf = I.skip_empty ? reinterpret_cast<const int*>(part + sp.part) : nullptr;
      vs[k] = AnnProb{P->Am, cpad_s(k), phiB_of(k), gs.ppa, gs.nk0, gs.nk1, gs.nk2, gs.k0lo, gs.k1lo, gs.k2lo, gs.L,
                      gs.padlo, I.N, I.S_lo, I.Ns, bs, sp.ncb_s, sp.es_s, part, rs, nzf};
      bs += sp.ncb_s * sp.es_s;
      if (sp.es_s > 1) rs += int64_t(3) * gs.nr * gs.nk0 * gs.nk1 * gs.nk2;
      vc[k] = AnnProb{P->Tm, cpad_p(k), F_of(k), gc.ppa, gc.nk0, gc.nk1, gc.nk2, gc.k0lo, gc.k1lo, gc.k2lo, gc.L,
                      gc.padlo, I.N, I.S_lo, I.Ns, bc, sp.ncb_c, sp.es_c, part, rc, nzf};
      bc += sp.ncb_c * sp.es_c;
      if (sp.es_c > 1) rc += int64_t(gc.nr) * gc.nk0 * gc.nk1 * gc.nk2;
    }
    for (int k0 = 0; k0 < np; k0 += ANN_PACK) {
      AnnPack ps{}, pcq{};
      ps.count = pcq.count = std::min(ANN_PACK, np - k0);
      for (int j = 0; j < ps.count; ++j) {
        ps.d[j] = vs[k0 + j];
        pcq.d[j] = vc[k0 + j];
      }
      hipLaunchKernelGGL(ann_upload_kernel, dim3(1), dim3(ANN_PACK), 0, s, ap_s + k0, ps);
      hipLaunchKernelGGL(ann_upload_kernel, dim3(1), dim3(ANN_PACK), 0, s, ap_c + k0, pcq);
    }
    {
      TimedScope ts(P0, s, "coarse_annulus");
      // moments into the zero-padded lattices both far-field sums read
      for (int k = 0; k < np; ++k) {
        const mlc_plan_info& I = G.plans[k]->info;
        const MfmaGeom& g = G.plans[k]->mg_coarse;
        hipLaunchKernelGGL(pad_moments_kernel, dim3(blocks_for(cube(g.L) * g.KP)), dim3(256), 0, s,
                           mom + int64_t(L.patch0[k]) * I.K, cpad_s(k), cpad_p(k), g.ppa, g.K, g.KP, g.L, g.padlo);
        if (I.skip_empty)
          hipLaunchKernelGGL(pad_flags_kernel, dim3(blocks_for(cube(g.L))), dim3(256), 0, s,
                             mom + int64_t(L.patch0[k]) * I.K,
                             reinterpret_cast<int*>(cpad_s(k) + 2 * cube(g.L) * g.KP + ann_split(I).part), g.ppa,
                             g.K, g.L, g.padlo);
      }
      const MfmaGeom& g = P0->mg_coarse;
      if (coarse_big(I0.n / NREF))
        hipLaunchKernelGGL(coarse_annulus_mfma_kernel<CoarseTiling>, dim3(g.nrp / CO_ROWS, bc),
                           dim3(64 * CoarseTiling::WAVES), 0, s, ap_c, np, g, I0.n / NREF);
      else
        hipLaunchKernelGGL(coarse_annulus_mfma_kernel<CoarseTilingSmall>, dim3(g.nrp / CO_ROWS, bc),
                           dim3(64 * CoarseTilingSmall::WAVES), 0, s, ap_c, np, g, I0.n / NREF);
      if (rc > 0)
        hipLaunchKernelGGL(coarse_reduce_kernel, dim3(blocks_for(rc)), dim3(256), 0, s, ap_c, np, rc, g, I0.n / NREF);
    }
    {
      TimedScope ts(P0, s, "skeleton_annulus");
      const MfmaGeom& g = P0->mg_skel;
      if (SK_ROWS == ann_block_rows<SkelTiling>())
        hipLaunchKernelGGL(skeleton_annulus_mfma_kernel<SkelTiling>, dim3(g.nrp / SK_ROWS, bs, 3),
                           dim3(64 * SkelTiling::WAVES), 0, s, ap_s, np, g, I0.n);
      else
        hipLaunchKernelGGL(skeleton_annulus_mfma_kernel<SkelTilingSmall>, dim3(g.nrp / SK_ROWS, bs, 3),
                           dim3(64 * SkelTilingSmall::WAVES), 0, s, ap_s, np, g, I0.n);
      if (rs > 0)
        hipLaunchKernelGGL(skeleton_reduce_kernel, dim3(blocks_for(rs)), dim3(256), 0, s, ap_s, np, rs, g, I0.n);
    }
  }
  // coarse solves, the FFTs batched over problems of equal coarse torus
  if (stage == COARSE) {
    TimedScope ts(P0, s, "coarse_solve");
    for (int k = 0; k < np; ++k) {
      const mlc_plan_info& I = G.plans[k]->info;
      if (I.levels > 2) continue;
      hipLaunchKernelGGL(coarse_fill_kernel, dim3(blocks_for(cube(I.M_coarse))), dim3(256), 0, s, F_of(k), tor_of(k),
                         I.Ns, I.M_coarse);
    }
    std::vector<int> done(np, 0);
    for (int k = 0; k < np; ++k)
      if (G.plans[k]->info.levels > 2) done[k] = 1;
    for (int k = 0; k < np; ++k) {
      if (done[k]) continue;
      const int Mc = G.plans[k]->info.M_coarse;
      int nb = 0;
      for (int j = k; j < np; ++j)
        if (!done[j] && G.plans[j]->info.M_coarse == Mc) { done[j] = 1; ++nb; }
      // every torus of the bucket has M_coarse = Mc; their source and output
      // boxes differ with N, so the pruning uses the bucket's largest
      int ns = 0, no = 0, o0 = 0;
      for (int j = k; j < np; ++j) {
        const mlc_plan_info& Ij = G.plans[j]->info;
        if (Ij.M_coarse != Mc) continue;
        ns = std::max(ns, Ij.Ns);
      }
      {
        // output slots (O_lo - S_lo + [0, No)) mod Mc; O_lo - S_lo and No grow with N
        int lo = Mc, hi = 0;
        for (int j = k; j < np; ++j) {
          const mlc_plan_info& Ij = G.plans[j]->info;
          if (Ij.M_coarse != Mc) continue;
          lo = std::min(lo, Ij.O_lo - Ij.S_lo);
          hi = std::max(hi, Ij.O_lo - Ij.S_lo + Ij.No);
        }
        // with d_beta / 4 < b the output box starts below the source box
        // (O_lo < S_lo): its slots wrap around the torus end, so the inverse
        // passes cover every slot
        if (lo < 0 || hi > Mc) {
          o0 = 0;
          no = Mc;
        } else {
          o0 = lo;
          no = hi - lo;
        }
      }
      if (!conv3_coarse(tor_of(k), G.plans[k]->coarse_spec, Mc, nb, ns, o0, no, s))
        return fail(P0->ctx, MLC_ERR_UNSUPPORTED, "coarse torus size or output range not built");
    }
    for (int k = 0; k < np; ++k) {
      const mlc_plan_info& I = G.plans[k]->info;
      if (I.levels > 2) continue;
      const int Mc = I.M_coarse;
      hipLaunchKernelGGL(coarse_extract_kernel, dim3(blocks_for(cube(I.No))), dim3(256), 0, s, tor_of(k), phiH_of(k),
                         Mc, I.S_lo, I.O_lo, I.No, I.H * I.H / (double(Mc) * Mc * Mc));
    }
      // multilevel problems (sec. 5): the coarse charge is solved by the method
    // one level up, on that level's box, and its uncorrected solution read
    // back onto the coarse output box
    for (int k = 0; k < np; ++k) {
      const mlc_plan* P = G.plans[k];
      const mlc_plan_info& I = P->info;
      if (I.levels <= 2) continue;
      const mlc_plan* C = P->child;
      const int m = I.level_margin, E = I.level_N + 1;
      double* f1 = reinterpret_cast<double*>(G.ws + L.o_lf[k]);
      double* phi1 = reinterpret_cast<double*>(G.ws + L.o_lphi[k]);
      hipLaunchKernelGGL(fill_zero_kernel, dim3(flat_blocks(cube(E))), dim3(256), 0, s, f1, cube(E));
      hipLaunchKernelGGL(box_copy_kernel, dim3(blocks_for(cube(I.Ns))), dim3(256), 0, s, F_of(k), I.Ns, 0, f1, E,
                         I.S_lo + m, I.Ns);
      Group G1;
      G1.plans = {const_cast<mlc_plan*>(C)};
      G1.f = {f1};
      G1.phi = {phi1};
      G1.L = layout_of({&C->info});
      G1.ws = G.ws + L.o_lws[k];
      G1.desc = reinterpret_cast<ProbDesc*>(G1.ws + G1.L.o_desc);
      // the coarser level's stages in order on this stream, with no side
      // stream of its own: a solve never creates a stream or an event after
      // its first call on a caller stream (graph capture forbids it)
      G1.one_stream = true;
      const mlc_status st1 = enqueue_group(G1, s);
      if (st1 != MLC_OK) return st1;
      hipLaunchKernelGGL(box_copy_kernel, dim3(blocks_for(cube(I.No))), dim3(256), 0, s, phi1, E, I.O_lo + m,
                         phiH_of(k), I.No, 0, I.No);
    }
}
  // local plane corrections delta_i = phi_i - I(phi_i), all patches
  if (stage == PLANES) {
    TimedScope ts(P0, s, "plane_delta");
    PlaneGeom pg{I0.n, I0.e, I0.d_alpha, I0.Wa, I0.Wc, P0->P0, I0.nplanes_a, I0.b};
    const size_t lds = sizeof(double) * (size_t(I0.Wc) * I0.Wc + size_t(I0.Wc) * I0.Wa);   // <= 35 KB (Wc <= 33, Wa <= 97)
    const int ns = slots_in_use(G);
    for (int p0 = 0; p0 < ns; p0 += kMaxGridY)
      hipLaunchKernelGGL(plane_delta_kernel<T>, dim3(3 * I0.nplanes_a, std::min(kMaxGridY, ns - p0)), dim3(256),
                         lds, s, pl, cs, pg, P0->lagw, live_of(G), p0);
  }
  // skeleton boundary values (+ phi there), every problem in one launch each
  // part: the plane-correction sums right after plane_delta (they need no
  // coarse solution), the interpolated coarse solution after the join
  if (stage == PLANES || stage == FINISH) {
    auto* pr = reinterpret_cast<SkelProb<T>*>(G.ws + L.o_flat + sizeof(CoarseRhsProb<double>) * np);
    double* dsum = reinterpret_cast<double*>(G.ws + L.o_dsum);
    int64_t total = 0, blocks = 0;
    std::vector<SkelProb<T>> v(np);
    for (int k = 0; k < np; ++k) {
      const mlc_plan* P = G.plans[k];
      const mlc_plan_info& I = P->info;
      SkelGeom sg{I.N, I.n, I.patches_per_axis, P->Kann, I.d_alpha, I.d_beta, I.b, I.Wa, P->P0, I.nplanes_a, P->Wb,
                  P->P0b, P->nplb, I.O_lo, I.No, final_c2h2(*P)};
      const int* plive = L.any_skip ? reinterpret_cast<const int*>(G.ws + L.o_live) + L.patch0[k] : nullptr;
      v[k] = SkelProb<T>{phiH_of(k), pl + L.patch0[k] * plsz, charge_of(G, k), phiB_of(k), phi_of(G, k), sg, total,
                         slot_of_patch(G), blocks, plive};
      total += int64_t(3) * (I.N / I.n + 1) * (I.N + 1) * (I.N + 1);
      // finishing tiles: planes x (N/4 + 1 coarse row intervals) x column chunks
      blocks += int64_t(3) * (I.N / I.n + 1) * (I.N / NREF + 1) * ((I.N + SKF_COLS) / SKF_COLS);
    }
    if (stage == PLANES) {
      upload_flat(pr, v, s);   // read by both parts
      TimedScope ts(P0, s, "skeleton_deltas");
      hipLaunchKernelGGL(skeleton_deltas_kernel<T>, dim3(blocks_for(total)), dim3(256), 0, s, pr, np, total, dsum);
    } else {
      TimedScope ts(P0, s, "skeleton");
      hipLaunchKernelGGL(skeleton_finish_kernel<T>, dim3(unsigned(blocks)), dim3(256), 0, s, pr, np, P0->lagw,
                         P0->Kann > 0 ? 1 : 0, dsum);
    }
  }
  // Dirichlet solves + Mehrstellen correction on the patch interiors, all patches
  if (stage == FINISH) {
    TimedScope ts(P0, s, "dirichlet");
    if (I0.n == 32) {
      // one block per patch, every patch in one launch (no work array: each
      // patch's values stay on the chip)
      DirGeom dg{I0.n, L.total, 2.0 / I0.n, st, 0};
      // the per-patch flags of which patches carry charge, when the solve has them
      const int* plive = L.any_skip ? reinterpret_cast<const int*>(G.ws + L.o_live) : nullptr;
      hipLaunchKernelGGL(dirichlet_fused_kernel, dim3(unsigned(L.total)), dim3(64 * DIRF_WAVES), 0, s, G.desc, np,
                         dg, plive);
    } else {
      // three passes over the work array, in chunks of patches when it cannot hold them all
      double* dir = reinterpret_cast<double*>(G.ws + L.o_dir);
      const int m = I0.n - 1;
      for (int p0 = 0; p0 < L.total; p0 += L.dir_chunk) {
        const int cnt = std::min(L.dir_chunk, L.total - p0);
        DirGeom dg{I0.n, cnt, 2.0 / I0.n, st, p0};
        dim3 gd(unsigned((int64_t(cnt) * m + DIR_WAVES - 1) / DIR_WAVES));
        if (I0.n <= 16) {   // 16 x 16 slab tiles
          hipLaunchKernelGGL((dirichlet_mfma_kernel<0, 16>), gd, dim3(64 * DIR_WAVES), 0, s, G.desc, np, dir, dg);
          hipLaunchKernelGGL((dirichlet_mfma_kernel<1, 16>), gd, dim3(64 * DIR_WAVES), 0, s, G.desc, np, dir, dg);
          hipLaunchKernelGGL((dirichlet_mfma_kernel<2, 16>), gd, dim3(64 * DIR_WAVES), 0, s, G.desc, np, dir, dg);
        } else {
          hipLaunchKernelGGL((dirichlet_mfma_kernel<0, 32>), gd, dim3(64 * DIR_WAVES), 0, s, G.desc, np, dir, dg);
          hipLaunchKernelGGL((dirichlet_mfma_kernel<1, 32>), gd, dim3(64 * DIR_WAVES), 0, s, G.desc, np, dir, dg);
          hipLaunchKernelGGL((dirichlet_mfma_kernel<2, 32>), gd, dim3(64 * DIR_WAVES), 0, s, G.desc, np, dir, dg);
        }
      }
    }
  }
  return MLC_OK;
}

// The side stream of caller stream s (created on first use).
static mlc_context::Side* side_of(mlc_context* ctx, hipStream_t s) {
  std::lock_guard<std::mutex> lk(ctx->side_mu);
  auto it = ctx->side.find(s);
  if (it != ctx->side.end()) return &it->second;
  mlc_context::Side sd;
  if (hipStreamCreateWithFlags(&sd.stream, hipStreamNonBlocking) != hipSuccess) return nullptr;
  for (hipEvent_t& e : sd.ev) {
    if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) {
      for (hipEvent_t x : sd.ev)
        if (x) hipEventDestroy(x);
      hipStreamDestroy(sd.stream);
      return nullptr;
    }
  }
  return &(ctx->side[s] = sd);
}

// Launch order on the caller stream s and its side stream:
//   s:    descriptors, x-DFTs, moments, first chunk's y/z pass | fork |
//         the other convolution passes | fork | plane corrections and their
//         sums at the skeleton nodes | join | skeleton, Dirichlet
//   side: (after fork 1) far-field sums | (after fork 2) coarse rhs and solve
// Every launch of one call has ended before the caller stream passes the
// join, so consecutive calls on s may reuse the workspace.
// The Legendre moments of every patch of a group from the per-plane sums of
// the x-DFT pass: divided by the diagonal Boole Gram matrix (P <= 4), or
// raw and then multiplied by the plan's inverse Gram matrix (P >= 5).
static void launch_moments(const Group& G, hipStream_t s) {
  const mlc_plan* P0 = G.plans[0];
  const mlc_plan_info& I0 = P0->info;
  const int np = int(G.plans.size());
  TimedScope ts(P0, s, "moments");
  const int ns = slots_in_use(G);
  const int64_t work = int64_t(ns) * I0.K, all = int64_t(G.L.total) * I0.K;
  const bool diag = I0.P <= 4;
  double* mom = reinterpret_cast<double*>(G.ws + G.L.o_mom);
  double* raw = reinterpret_cast<double*>(G.ws + G.L.o_mraw);
  // compact buffers: the empty patches' moments are zero, the others are set below
  if (G.L.compact)
    hipLaunchKernelGGL(fill_zero_kernel, dim3(flat_blocks(all)), dim3(256), 0, s, diag ? mom : raw, all);
  if (work > 0)
    hipLaunchKernelGGL(moments_finish_kernel, dim3(unsigned((work + 255) / 256)), dim3(256), 0, s, G.desc, np, I0.n,
                       I0.P, P0->modes, reinterpret_cast<const double*>(G.ws + G.L.o_mpart), diag ? mom : raw, ns,
                       diag ? 1 : 0, patch_of_slot(G));
  if (!diag)
    hipLaunchKernelGGL(moments_gram_kernel, dim3(unsigned((all + 255) / 256)), dim3(256), 0, s, raw, P0->gram_inv,
                       I0.K, mom, G.L.total);
}

// A charge given analytically: sampled into f before the convolutions, and
// the moments by Gauss integration instead of Boole's rule.
struct AnalyticInput {
  RadialCharge q;
  GaussRule rule;
  double* f;   // the caller's node array the samples go to
};

static void launch_analytic_fill(const Group& G, hipStream_t s, const AnalyticInput& an) {
  const mlc_plan_info& I = G.plans[0]->info;
  const int64_t nodes = cube(I.N + 1);
  hipLaunchKernelGGL(analytic_fill_kernel, dim3(flat_blocks(nodes)), dim3(256), 0, s, an.q, I.N, I.h, an.f);
}

static void launch_gauss_moments(const Group& G, hipStream_t s, const AnalyticInput& an) {
  const mlc_plan* P0 = G.plans[0];
  const mlc_plan_info& I0 = P0->info;
  const int np = int(G.plans.size());
  TimedScope ts(P0, s, "moments_gauss");
  double* mom = reinterpret_cast<double*>(G.ws + G.L.o_mom);
  for (int p0 = 0; p0 < G.L.total; p0 += kMaxGridY) {
    const dim3 grid(unsigned(std::min(kMaxGridY, G.L.total - p0)));
    switch (I0.P) {
#define CASE(PP)                                                                                                  \
  case PP:                                                                                                        \
    hipLaunchKernelGGL(gauss_moments_kernel<PP>, grid, dim3(GAUSS_THREADS), 0, s, G.desc, np, I0.n, an.q, an.rule, \
                       P0->modes, mom, p0);                                                                      \
    break;
      CASE(1) CASE(2) CASE(3) CASE(4) CASE(5) CASE(6) CASE(7) CASE(8) CASE(9)
#undef CASE
    }
  }
}

// A plan that keeps its live patches only (max_live): flag the patches that
// carry charge, wait for the flags, and number the live patches in order as
// the slots of the per-patch buffers.  The one host synchronisation of such
// a solve; the lists go back to the device before any kernel reads them.
static mlc_status compact_live(const Group& G, hipStream_t s) {
  const mlc_plan* P0 = G.plans[0];
  const Layout& L = G.L;
  const int np = int(G.plans.size());
  int* live = reinterpret_cast<int*>(G.ws + L.o_live);
  {
    TimedScope ts(P0, s, "patch_live");
    hipLaunchKernelGGL(patch_live_kernel, dim3(L.total), dim3(256), 0, s, G.desc, np, P0->info.n, live, 0);
  }
  std::vector<int> flag(L.total), patch_of, slot_of(L.total, -1);
  hipError_t e = hipMemcpyAsync(flag.data(), live, sizeof(int) * L.total, hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return fail(P0->ctx, MLC_ERR_DEVICE, std::string("live patches: ") + hipGetErrorString(e));
  for (int p = 0; p < L.total; ++p)
    if (flag[p]) {
      slot_of[p] = int(patch_of.size());
      patch_of.push_back(p);
    }
  if (int(patch_of.size()) > L.slots)
    return fail(P0->ctx, MLC_ERR_OUT_OF_MEMORY,
                std::to_string(patch_of.size()) + " patches carry charge, more than max_live = " +
                    std::to_string(L.slots));
  if (!patch_of.empty())
    e = hipMemcpyAsync(G.ws + L.o_patch_of, patch_of.data(), sizeof(int) * patch_of.size(), hipMemcpyHostToDevice, s);
  if (e == hipSuccess)
    e = hipMemcpyAsync(G.ws + L.o_slot_of, slot_of.data(), sizeof(int) * L.total, hipMemcpyHostToDevice, s);
  // the host lists go out of scope on return
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return fail(P0->ctx, MLC_ERR_DEVICE, std::string("live patches: ") + hipGetErrorString(e));
  G.nslots = int(patch_of.size());
  return MLC_OK;
}

// With G.one_stream set, every stage runs on s in the same order (no side
// stream, no events): the same kernels on the same data, so the same result.
static mlc_status enqueue_group(const Group& G, hipStream_t s, const AnalyticInput* an) {
  const mlc_plan* P0 = G.plans[0];
  const mlc_plan_info& I0 = P0->info;
  const int np = int(G.plans.size());
  if (G.one_stream) {
    const bool f32 = I0.conv_precision == MLC_CONV_FP32;
    upload_descs(G, s);
    launch_box_in(G, s);
    if (an) launch_analytic_fill(G, s, *an);
    launch_sixth_rhs(G, s);
    if (const hipError_t e0 = hipGetLastError(); e0 != hipSuccess)
      return fail(P0->ctx, MLC_ERR_DEVICE, std::string("launch: ") + hipGetErrorString(e0));
    if (G.L.compact) {
      const mlc_status r = compact_live(G, s);
      if (r != MLC_OK) return r;
    }
    if (!(f32 ? dispatch_conv<float>(G, s, 0) : dispatch_conv<double>(G, s, 0)))
      return fail(P0->ctx, MLC_ERR_UNSUPPORTED, "local FFT size not built");
    if (an) launch_gauss_moments(G, s, *an);
    else launch_moments(G, s);
    if (f32) dispatch_conv<float>(G, s, 1);
    else dispatch_conv<double>(G, s, 1);
    for (Stage st : {FAR, COARSE, PLANES, FINISH}) {
      const mlc_status r = f32 ? launch_rest<float>(G, s, st) : launch_rest<double>(G, s, st);
      if (r != MLC_OK) return r;
    }
    launch_box_out(G, s);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(P0->ctx, MLC_ERR_DEVICE, std::string("launch: ") + hipGetErrorString(e));
    return MLC_OK;
  }
  mlc_context::Side* sd = side_of(P0->ctx, s);
  if (!sd) return fail(P0->ctx, MLC_ERR_DEVICE, "could not create the side stream");
  const bool fp32 = I0.conv_precision == MLC_CONV_FP32;
  upload_descs(G, s);
  launch_box_in(G, s);
  if (an) launch_analytic_fill(G, s, *an);
  launch_sixth_rhs(G, s);
  // the launches so far, checked before the API calls that follow
  if (const hipError_t e0 = hipGetLastError(); e0 != hipSuccess)
    return fail(P0->ctx, MLC_ERR_DEVICE, std::string("launch: ") + hipGetErrorString(e0));
  if (G.L.compact) {
    const mlc_status r = compact_live(G, s);
    if (r != MLC_OK) return r;
  }
  // the x-DFT pass of the local convolutions also leaves the per-plane
  // moment sums, finished here before the far-field sums read the moments
  const bool ok = fp32 ? dispatch_conv<float>(G, s, 0) : dispatch_conv<double>(G, s, 0);
  if (!ok) return fail(P0->ctx, MLC_ERR_UNSUPPORTED, "local FFT size not built");
  if (an) launch_gauss_moments(G, s, *an);
  else launch_moments(G, s);
  // fork 1 after the first chunk's y/z pass: the far-field sums then share
  // the chip with the output pass (one block per CU, LDS and registers to
  // spare) rather than with the y/z pass (whose blocks fill the LDS)
  hipError_t e = hipSuccess;
  const std::function<void()> fork_far = [&]() {
    e = hipEventRecord(sd->ev[0], s);
    if (e == hipSuccess) e = hipStreamWaitEvent(sd->stream, sd->ev[0], 0);
    if (e != hipSuccess) return;
    if (fp32) launch_rest<float>(G, sd->stream, FAR);
    else launch_rest<double>(G, sd->stream, FAR);
  };
  if (fp32) dispatch_conv<float>(G, s, 1, &fork_far);
  else dispatch_conv<double>(G, s, 1, &fork_far);
  if (e != hipSuccess) return fail(P0->ctx, MLC_ERR_DEVICE, std::string("fork: ") + hipGetErrorString(e));
  e = hipEventRecord(sd->ev[1], s);
  if (e == hipSuccess) e = hipStreamWaitEvent(sd->stream, sd->ev[1], 0);
  if (e != hipSuccess) return fail(P0->ctx, MLC_ERR_DEVICE, std::string("fork: ") + hipGetErrorString(e));
  const mlc_status rc = fp32 ? launch_rest<float>(G, sd->stream, COARSE) : launch_rest<double>(G, sd->stream, COARSE);
  if (rc != MLC_OK) return rc;
  e = hipEventRecord(sd->ev[2], sd->stream);
  if (fp32) launch_rest<float>(G, s, PLANES);
  else launch_rest<double>(G, s, PLANES);
  if (e == hipSuccess) e = hipStreamWaitEvent(s, sd->ev[2], 0);
  if (e != hipSuccess) return fail(P0->ctx, MLC_ERR_DEVICE, std::string("join: ") + hipGetErrorString(e));
  if (fp32) launch_rest<float>(G, s, FINISH);
  else launch_rest<double>(G, s, FINISH);
  launch_box_out(G, s);
  e = hipGetLastError();
  if (e != hipSuccess) return fail(P0->ctx, MLC_ERR_DEVICE, std::string("launch: ") + hipGetErrorString(e));
  return MLC_OK;
}

// With MLC_CHECK=1 in the environment, each f of a solve is checked on the
// device to vanish on the outer boundary nodes (the charge must be supported
// inside the domain, sec. 4); the check synchronises the stream.  Off by
// default.
static bool check_enabled() {
  const char* e = std::getenv("MLC_CHECK");
  return e && e[0] == '1';
}

// The flag lives with the caller stream's side-stream state, so callers on
// different streams (a server thread and the caller's own thread) never
// share one.
static mlc_status check_boundary(mlc_context* ctx, const double* f, const int* B, int layers, hipStream_t s) {
  mlc_context::Side* sd = side_of(ctx, s);
  if (!sd) return fail(ctx, MLC_ERR_DEVICE, "could not create the side stream");
  int* flag = nullptr;
  {
    std::lock_guard<std::mutex> lk(ctx->side_mu);
    if (!sd->check_flag && hipMalloc(&sd->check_flag, sizeof(int)) != hipSuccess) sd->check_flag = nullptr;
    flag = sd->check_flag;
  }
  if (!flag) return fail(ctx, MLC_ERR_OUT_OF_MEMORY, "check flag allocation failed");
  const int Bm = std::max(B[0], std::max(B[1], B[2]));
  const int64_t faces = int64_t(6) * layers * (Bm + 1) * (Bm + 1);
  hipLaunchKernelGGL(set_flag_kernel, dim3(1), dim3(1), 0, s, flag, 0);
  hipLaunchKernelGGL(boundary_check_kernel, dim3(blocks_for(faces)), dim3(256), 0, s, f, B[0], B[1], B[2], layers,
                     flag);
  int h = 0;
  hipError_t e = hipMemcpyAsync(&h, flag, sizeof(int), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return fail(ctx, MLC_ERR_DEVICE, std::string("boundary check: ") + hipGetErrorString(e));
  if (h)
    return fail(ctx, MLC_ERR_INVALID_ARG,
                layers > 1 ? "f is nonzero within two nodes of the outer boundary (MLC_CHECK, rhs_order 6)"
                           : "f is nonzero on the outer boundary (MLC_CHECK)");
  return MLC_OK;
}

// for the serving loop (server.hip): whether MLC_CHECK is on, and the check
// of one request's charge on the server's launch stream
bool mlc_check_enabled() { return check_enabled(); }
// layers of the outer faces a charge must vanish on: one, three for the
// sixth-order right-hand side
int mlc_check_layers(const mlc_plan_info& I) { return I.rhs_order == 6 ? 3 : 1; }
mlc_status mlc_check_charge(mlc_context* ctx, const double* f, const mlc_plan_info& I, void* stream) {
  HIP_TRY(ctx, hipSetDevice(ctx->device));
  return check_boundary(ctx, f, I.box, mlc_check_layers(I), static_cast<hipStream_t>(stream));
}

// ----------------------------------------------------------------- trace
// MLC_TRACE=<file>: every mlc_solve and mlc_solve_batched call appends one
// JSON line to the file: the problems, the call's status and wall time, and
// per stage timer its launches and device milliseconds, at every level of a
// multilevel plan ("L1." prefixes the next coarser level).  A traced call
// waits for its stream before it returns: tracing is for diagnosis, not for
// timing runs.
static const char* trace_path() {
  const char* e = std::getenv("MLC_TRACE");
  return (e && *e) ? e : nullptr;
}
struct Trace {
  struct Entry {
    mlc_plan* plan;
    int depth;
    bool was_on;
    std::vector<std::pair<std::string, std::pair<int, double>>> before;
  };
  std::vector<Entry> e;
  std::vector<const mlc_plan*> roots;
  std::chrono::steady_clock::time_point t0;
};
static std::mutex g_trace_mu;

static void trace_begin(Trace* T, mlc_plan* const* plans, int count) {
  T->t0 = std::chrono::steady_clock::now();
  for (int k = 0; k < count; ++k) {
    T->roots.push_back(plans[k]);
    int depth = 0;
    for (mlc_plan* q = plans[k]; q; q = q->child, ++depth) {
      bool seen = false;
      for (auto& x : T->e) seen = seen || x.plan == q;
      if (seen) continue;
      drain_timing(q);
      T->e.push_back({q, depth, q->timing_on, q->acc});
      q->timing_on = true;
    }
  }
}

static void trace_end(Trace* T, const char* entry, hipStream_t s, mlc_status st) {
  const hipError_t se = hipStreamSynchronize(s);
  const double wall = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - T->t0).count();
  std::map<std::string, std::pair<int, double>> stages;
  for (auto& x : T->e) {
    drain_timing(x.plan);
    const std::string pre = x.depth ? "L" + std::to_string(x.depth) + "." : "";
    for (auto& kv : x.plan->acc) {
      int l = kv.second.first;
      double ms = kv.second.second;
      for (auto& b : x.before)
        if (b.first == kv.first) { l -= b.second.first; ms -= b.second.second; }
      if (l > 0) {
        auto& d = stages[pre + kv.first];
        d.first += l;
        d.second += ms;
      }
    }
    if (!x.was_on) {
      x.plan->acc = x.before;
      x.plan->timing_on = false;
    }
  }
  std::string line = std::string("{\"entry\": \"") + entry + "\", \"status\": \"" + mlc_status_string(st) + "\"";
  if (se != hipSuccess) line += std::string(", \"stream_error\": \"") + hipGetErrorString(se) + "\"";
  char buf[256];
  std::snprintf(buf, sizeof(buf), ", \"wall_ms\": %.4f, \"problems\": [", wall);
  line += buf;
  for (size_t k = 0; k < T->roots.size(); ++k) {
    const mlc_plan_info& I = T->roots[k]->info;
    std::snprintf(buf, sizeof(buf),
                  "%s{\"N\": %d, \"n\": %d, \"alpha\": %g, \"beta\": %g, \"P\": %d, \"Q\": %d, \"levels\": %d, "
                  "\"conv\": \"%s\", \"rhs_order\": %d}",
                  k ? ", " : "", I.N, I.n, I.alpha, I.beta, I.P, I.Q, I.levels,
                  I.conv_precision == MLC_CONV_FP32 ? "fp32" : "fp64", I.rhs_order);
    line += buf;
  }
  line += "], \"stages\": {";
  bool first = true;
  for (auto& kv : stages) {
    std::snprintf(buf, sizeof(buf), "%s\"%s\": [%d, %.5f]", first ? "" : ", ", kv.first.c_str(), kv.second.first,
                  kv.second.second);
    line += buf;
    first = false;
  }
  line += "}}\n";
  std::lock_guard<std::mutex> lk(g_trace_mu);
  if (FILE* fp = std::fopen(trace_path(), "a")) {
    std::fputs(line.c_str(), fp);
    std::fclose(fp);
  }
}

extern "C" mlc_status mlc_solve(mlc_plan* plan, const double* f, double* phi, void* workspace, size_t ws_bytes,
                                void* stream) {
  if (!plan || !f || !phi || !workspace) return fail(plan ? plan->ctx : nullptr, MLC_ERR_INVALID_ARG, "null argument");
  if (ws_bytes < plan->ws_total) return fail(plan->ctx, MLC_ERR_INVALID_ARG, "workspace too small");
  if (reinterpret_cast<uintptr_t>(workspace) % 256)
    return fail(plan->ctx, MLC_ERR_INVALID_ARG, "workspace must be 256-byte aligned");
  HIP_TRY(plan->ctx, hipSetDevice(plan->ctx->device));
  Group G;
  G.plans = {plan};
  G.f = {f};
  G.phi = {phi};
  G.L = layout_of(infos_of(G.plans));
  if (ws_bytes < G.L.bytes) return fail(plan->ctx, MLC_ERR_INVALID_ARG, "workspace too small");
  if (check_enabled()) {
    const mlc_status cs =
        check_boundary(plan->ctx, f, plan->info.box, mlc_check_layers(plan->info), static_cast<hipStream_t>(stream));
    if (cs != MLC_OK) return cs;
  }
  G.ws = static_cast<char*>(workspace);
  G.desc = reinterpret_cast<ProbDesc*>(G.ws + G.L.o_desc);
  if (!trace_path()) return enqueue_group(G, static_cast<hipStream_t>(stream));
  Trace T;
  trace_begin(&T, &plan, 1);
  const mlc_status st = enqueue_group(G, static_cast<hipStream_t>(stream));
  trace_end(&T, "mlc_solve", static_cast<hipStream_t>(stream), st);
  return st;
}

// Gauss-Legendre nodes and weights on [-1, 1], gp = 1..4
static GaussRule gauss_rule(int gp) {
  GaussRule r{};
  r.gp = gp;
  switch (gp) {
    case 1: r.xi[0] = 0.0; r.om[0] = 2.0; break;
    case 2: r.xi[0] = -1.0 / std::sqrt(3.0); r.xi[1] = -r.xi[0]; r.om[0] = r.om[1] = 1.0; break;
    case 3:
      r.xi[0] = -std::sqrt(0.6); r.xi[1] = 0.0; r.xi[2] = std::sqrt(0.6);
      r.om[0] = r.om[2] = 5.0 / 9.0; r.om[1] = 8.0 / 9.0;
      break;
    default: {
      const double a = std::sqrt(3.0 / 7.0 - 2.0 / 7.0 * std::sqrt(1.2)), b = std::sqrt(3.0 / 7.0 + 2.0 / 7.0 * std::sqrt(1.2));
      const double wa = (18.0 + std::sqrt(30.0)) / 36.0, wb = (18.0 - std::sqrt(30.0)) / 36.0;
      r.xi[0] = -b; r.xi[1] = -a; r.xi[2] = a; r.xi[3] = b;
      r.om[0] = wb; r.om[1] = wa; r.om[2] = wa; r.om[3] = wb;
    }
  }
  return r;
}

extern "C" mlc_status mlc_solve_analytic(mlc_plan* plan, int32_t nterms, const mlc_radial_charge* terms,
                                         int32_t gauss_points, double* f, double* phi, void* workspace,
                                         size_t ws_bytes, void* stream) {
  mlc_context* ctx = plan ? plan->ctx : nullptr;
  if (!plan || !terms || !f || !phi || !workspace) return fail(ctx, MLC_ERR_INVALID_ARG, "null argument");
  if (nterms < 1 || nterms > MLC_MAX_RADIAL_TERMS)
    return fail(ctx, MLC_ERR_INVALID_ARG, "nterms must be in [1, MLC_MAX_RADIAL_TERMS]");
  if (gauss_points < 1 || gauss_points > 4) return fail(ctx, MLC_ERR_INVALID_ARG, "gauss_points must be in [1, 4]");
  if (plan->info.rhs_order == 6)
    return fail(ctx, MLC_ERR_UNSUPPORTED, "the Gauss moments are those of f, not of the sixth-order right-hand side");
  if (is_boxed(plan->info)) return fail(ctx, MLC_ERR_UNSUPPORTED, "analytic charges are sampled on cubes only");
  if (ws_bytes < plan->ws_total) return fail(ctx, MLC_ERR_INVALID_ARG, "workspace too small");
  if (reinterpret_cast<uintptr_t>(workspace) % 256)
    return fail(ctx, MLC_ERR_INVALID_ARG, "workspace must be 256-byte aligned");
  const mlc_plan_info& I = plan->info;
  const double L = I.N * I.h;
  AnalyticInput an{};
  an.q.count = nterms;
  for (int k = 0; k < nterms; ++k) {
    const mlc_radial_charge& t = terms[k];
    if (!(t.radius > 0.0) || !std::isfinite(t.radius) || !std::isfinite(t.weight) || !std::isfinite(t.param) ||
        t.profile < MLC_PROFILE_BUMP || t.profile > MLC_PROFILE_OSCILLATORY)
      return fail(ctx, MLC_ERR_INVALID_ARG, "radial term " + std::to_string(k) + " is malformed");
    for (int d = 0; d < 3; ++d)
      if (!(t.centre[d] - t.radius >= 0.0) || !(t.centre[d] + t.radius <= L))
        return fail(ctx, MLC_ERR_INVALID_ARG,
                    "radial term " + std::to_string(k) + " reaches the outer boundary (f must vanish there)");
    RadialTerm& r = an.q.t[k];
    for (int d = 0; d < 3; ++d) r.c[d] = t.centre[d];
    r.R = t.radius;
    r.w = t.weight;
    r.param = t.param;
    r.profile = t.profile;
  }
  an.rule = gauss_rule(gauss_points);
  an.f = f;
  HIP_TRY(ctx, hipSetDevice(ctx->device));
  Group G;
  G.plans = {plan};
  G.f = {f};
  G.phi = {phi};
  G.L = layout_of(infos_of(G.plans));
  G.ws = static_cast<char*>(workspace);
  G.desc = reinterpret_cast<ProbDesc*>(G.ws + G.L.o_desc);
  return enqueue_group(G, static_cast<hipStream_t>(stream), &an);
}

// mlc_solve on the device's static scratch instead of a caller workspace,
// every stage on the caller's stream: no device allocation, stream or event
// is created.  Calls that overlap on one device share the scratch and race.
extern "C" mlc_status mlc_solve_static(mlc_plan* plan, const double* f, double* phi, void* stream) {
  if (!plan || !f || !phi) return fail(plan ? plan->ctx : nullptr, MLC_ERR_INVALID_ARG, "null argument");
  if (plan->info.slots < plan->info.npatch)
    return fail(plan->ctx, MLC_ERR_UNSUPPORTED, "a plan with max_live waits for its live-patch count: use mlc_solve");
  if (plan->ws_total > kStaticScratchBytes)
    return fail(plan->ctx, MLC_ERR_UNSUPPORTED,
                "the plan's workspace (" + std::to_string(plan->ws_total) + " bytes) exceeds the static scratch (" +
                    std::to_string(kStaticScratchBytes) + " bytes); use mlc_solve with a workspace");
  char* ws = static_cast<char*>(scratch_of(plan->ctx->device));
  if (!ws) return fail(plan->ctx, MLC_ERR_DEVICE, "no static scratch address for the plan's device");
  HIP_TRY(plan->ctx, hipSetDevice(plan->ctx->device));
  Group G;
  G.plans = {plan};
  G.f = {f};
  G.phi = {phi};
  G.L = layout_of(infos_of(G.plans));
  G.ws = ws;
  G.desc = reinterpret_cast<ProbDesc*>(G.ws + G.L.o_desc);
  G.one_stream = true;
  return enqueue_group(G, static_cast<hipStream_t>(stream));
}

// Split a batch into class groups (first-appearance order) and lay them out
// one after another in the workspace.
static mlc_status make_groups(int32_t count, mlc_plan* const* plans, std::vector<Group>* out, size_t* bytes) {
  if (count <= 0 || !plans || !bytes) return fail(nullptr, MLC_ERR_INVALID_ARG, "bad batch arguments");
  for (int k = 0; k < count; ++k)
    if (!plans[k]) return fail(nullptr, MLC_ERR_INVALID_ARG, "null plan in batch");
  for (int k = 0; k < count; ++k)
    if (plans[k]->info.slots < plans[k]->info.npatch)
      return fail(plans[k]->ctx, MLC_ERR_UNSUPPORTED,
                  "a plan with max_live solves alone (mlc_solve, mlc_solve_analytic), not in batches or graphs");
  mlc_context* ctx = plans[0]->ctx;
  for (int k = 1; k < count; ++k)
    if (plans[k]->ctx != ctx) return fail(ctx, MLC_ERR_INVALID_ARG, "plans of one batch must share a context");
  std::vector<Group> groups;
  for (int k = 0; k < count; ++k) {
    size_t gi = 0;
    while (gi < groups.size() && !same_class(groups[gi].plans[0], plans[k])) ++gi;
    if (gi == groups.size()) groups.emplace_back();
    groups[gi].plans.push_back(plans[k]);
    groups[gi].pos.push_back(k);
  }
  size_t off = 0;
  for (auto& G : groups) {
    G.L = layout_of(infos_of(G.plans));
    G.off = off;
    off = align_up(off + G.L.bytes);
  }
  *bytes = off;
  if (out) *out = std::move(groups);
  return MLC_OK;
}

extern "C" mlc_status mlc_batch_workspace_bytes(int32_t count, mlc_plan* const* plans, size_t* bytes) {
  return make_groups(count, plans, nullptr, bytes);
}

extern "C" mlc_status mlc_solve_batched(int32_t count, mlc_plan* const* plans, const double* const* f,
                                        double* const* phi, void* workspace, size_t ws_bytes, void* stream) {
  size_t need = 0;
  std::vector<Group> groups;
  mlc_status st = make_groups(count, plans, &groups, &need);
  if (st != MLC_OK) return st;
  mlc_context* ctx = plans[0]->ctx;
  if (!f || !phi || !workspace) return fail(ctx, MLC_ERR_INVALID_ARG, "null argument");
  if (ws_bytes < need) return fail(ctx, MLC_ERR_INVALID_ARG, "workspace too small");
  if (reinterpret_cast<uintptr_t>(workspace) % 256)
    return fail(ctx, MLC_ERR_INVALID_ARG, "workspace must be 256-byte aligned");
  for (int k = 0; k < count; ++k)
    if (!f[k] || !phi[k]) return fail(ctx, MLC_ERR_INVALID_ARG, "null array in batch");
  HIP_TRY(ctx, hipSetDevice(ctx->device));
  if (check_enabled()) {
    for (int k = 0; k < count; ++k) {
      st = check_boundary(ctx, f[k], plans[k]->info.box, mlc_check_layers(plans[k]->info), static_cast<hipStream_t>(stream));
      if (st != MLC_OK) return st;
    }
  }
  char* base = static_cast<char*>(workspace);
  for (auto& G : groups) {
    for (int k : G.pos) {
      G.f.push_back(f[k]);
      G.phi.push_back(phi[k]);
    }
    G.ws = base + G.off;
    G.desc = reinterpret_cast<ProbDesc*>(G.ws + G.L.o_desc);
  }
  Trace T;
  const bool traced = trace_path() != nullptr;
  if (traced) trace_begin(&T, plans, count);
  for (auto& G : groups) {
    st = enqueue_group(G, static_cast<hipStream_t>(stream));
    if (st != MLC_OK) break;
  }
  if (traced) trace_end(&T, "mlc_solve_batched", static_cast<hipStream_t>(stream), st);
  return st;
}

// ---------------------------------------------------------- batch graphs
// One batched solve (fixed plans, arrays and workspace) captured once into a
// HIP graph: the launches of every class group, the side-stream fork and join
// included (they become parallel branches of the graph), so that a replay
// re-runs the whole batch with one launch call.  The solve path enqueues
// kernels only (no memsets, no host synchronisation), so it captures as is.
struct mlc_graph {
  mlc_context* ctx = nullptr;
  hipStream_t cap = nullptr;     // the stream the batch was captured on (kept for its side stream)
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

extern "C" mlc_status mlc_graph_create(int32_t count, mlc_plan* const* plans, const double* const* f,
                                       double* const* phi, void* workspace, size_t ws_bytes, mlc_graph** out) {
  if (!out) return fail(nullptr, MLC_ERR_INVALID_ARG, "null output pointer");
  size_t need = 0;
  std::vector<Group> groups;
  mlc_status st = make_groups(count, plans, &groups, &need);
  if (st != MLC_OK) return st;
  mlc_context* ctx = plans[0]->ctx;
  if (!f || !phi || !workspace) return fail(ctx, MLC_ERR_INVALID_ARG, "null argument");
  if (ws_bytes < need) return fail(ctx, MLC_ERR_INVALID_ARG, "workspace too small");
  if (reinterpret_cast<uintptr_t>(workspace) % 256)
    return fail(ctx, MLC_ERR_INVALID_ARG, "workspace must be 256-byte aligned");
  for (int k = 0; k < count; ++k) {
    if (!f[k] || !phi[k]) return fail(ctx, MLC_ERR_INVALID_ARG, "null array in batch");
    if (plans[k]->timing_on) return fail(ctx, MLC_ERR_INVALID_ARG, "per-kernel timing must be off while capturing");
  }
  HIP_TRY(ctx, hipSetDevice(ctx->device));
  auto* g = new (std::nothrow) mlc_graph;
  if (!g) return fail(ctx, MLC_ERR_OUT_OF_MEMORY, "host allocation failed");
  g->ctx = ctx;
  auto cleanup = [&](mlc_status s, const std::string& msg) {
    if (g->exec) hipGraphExecDestroy(g->exec);
    if (g->graph) hipGraphDestroy(g->graph);
    if (g->cap) hipStreamDestroy(g->cap);
    delete g;
    return fail(ctx, s, msg);
  };
  if (hipStreamCreateWithFlags(&g->cap, hipStreamNonBlocking) != hipSuccess) {
    g->cap = nullptr;
    return cleanup(MLC_ERR_DEVICE, "capture stream creation failed");
  }
  // the capture stream's side stream and events exist before the capture
  if (!side_of(ctx, g->cap)) return cleanup(MLC_ERR_DEVICE, "could not create the side stream");
  char* base = static_cast<char*>(workspace);
  for (auto& G : groups) {
    for (int k : G.pos) {
      G.f.push_back(f[k]);
      G.phi.push_back(phi[k]);
    }
    G.ws = base + G.off;
    G.desc = reinterpret_cast<ProbDesc*>(G.ws + G.L.o_desc);
  }
  hipError_t e = hipStreamBeginCapture(g->cap, hipStreamCaptureModeThreadLocal);
  if (e != hipSuccess) return cleanup(MLC_ERR_DEVICE, std::string("begin capture: ") + hipGetErrorString(e));
  for (auto& G : groups) {
    st = enqueue_group(G, g->cap);
    if (st != MLC_OK) break;
  }
  hipGraph_t graph = nullptr;
  e = hipStreamEndCapture(g->cap, &graph);
  g->graph = graph;
  if (st != MLC_OK) return cleanup(st, "capture: a stage could not be enqueued");
  if (e != hipSuccess) return cleanup(MLC_ERR_DEVICE, std::string("end capture: ") + hipGetErrorString(e));
  e = hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0);
  if (e != hipSuccess) {
    g->exec = nullptr;
    return cleanup(MLC_ERR_DEVICE, std::string("graph instantiation: ") + hipGetErrorString(e));
  }
  *out = g;
  return MLC_OK;
}

extern "C" mlc_status mlc_graph_launch(mlc_graph* g, void* stream) {
  if (!g) return fail(nullptr, MLC_ERR_INVALID_ARG, "null graph");
  HIP_TRY(g->ctx, hipSetDevice(g->ctx->device));
  HIP_TRY(g->ctx, hipGraphLaunch(g->exec, static_cast<hipStream_t>(stream)));
  return MLC_OK;
}

extern "C" mlc_status mlc_graph_destroy(mlc_graph* g) {
  if (!g) return MLC_ERR_INVALID_ARG;
  hipSetDevice(g->ctx->device);
  if (g->exec) hipGraphExecDestroy(g->exec);
  if (g->graph) hipGraphDestroy(g->graph);
  if (g->cap) {
    hipStreamSynchronize(g->cap);
    hipStreamDestroy(g->cap);
  }
  delete g;
  return MLC_OK;
}

// ------------------------------------------------------------- autotune
// Local torus edge M and output planes per block for fft_size = -1: every
// built size >= the Hockney minimum (and within the DGF table), with each
// planes-per-block count, is timed on an 8x8x8-patch probe grid (the three
// local-convolution kernels, zero charge), and the fastest pair is kept per
// patch-work class in the context.  The planes per block never change a
// result (each output plane is computed the same way by whichever block
// holds it).  Synchronises the device.
template <typename T>
static double time_conv(mlc_context* ctx, const mlc_plan_info& I0, const double* G1, int M, int zpb) {
  mlc_plan Pt;
  Pt.ctx = ctx;
  Pt.info = I0;
  Pt.info.M = M;
  Pt.info.out_planes = zpb;
  Pt.info.levels = 2;
  Pt.info.level_margin = Pt.info.level_N = 0;
  // an 8^3-patch probe: as many blocks per launch as a full-size problem, so
  // that the tiling's effect on how the chip fills is seen
  Pt.info.N = 8 * I0.n;
  Pt.info.patches_per_axis = 8;
  Pt.info.npatch = 512;
  Pt.S = I0.n + 1;
  Pt.Mh = M / 2 + 1;
  Pt.Wp = I0.Wa + 2 * I0.b;
  Pt.P0 = -((I0.d_alpha / I0.n) * I0.n);
  const mlc_plan_info& I = Pt.info;
  cplx<double>* work = nullptr;
  double* f = nullptr;
  char* ws = nullptr;
  hipEvent_t a = nullptr, b = nullptr;
  double ms = -1.0;
  const Layout L = layout_of({&I});
  const size_t fbytes = sizeof(double) * cube(I.N + 1);
  if (hipMalloc(&work, sizeof(cplx<double>) * cube(M)) == hipSuccess &&
      hipMalloc(&Pt.conv_spec, sizeof(T) * cube(Pt.Mh)) == hipSuccess &&
      hipMalloc(&f, fbytes) == hipSuccess && hipMalloc(&ws, L.bytes) == hipSuccess &&
      hipEventCreate(&a) == hipSuccess && hipEventCreate(&b) == hipSuccess &&
      build_spectrum(ctx, G1, I.Z, M, work, nullptr, Pt.conv_spec, int(sizeof(T)), 1.0 / (double(M) * M * M), 2, 1,
                     0) == MLC_OK &&
      hipMemset(f, 0, fbytes) == hipSuccess) {
    Group G;
    G.plans = {&Pt};
    G.f = {f};
    G.phi = {nullptr};
    G.L = L;
    G.ws = ws;
    G.desc = reinterpret_cast<ProbDesc*>(ws + L.o_desc);
    hipStream_t s = nullptr;
    upload_descs(G, s);
    bool ok = dispatch_conv<T>(G, s, 0) && dispatch_conv<T>(G, s, 1);
    // the best of three timings of two passes each
    for (int trial = 0; ok && trial < 3; ++trial) {
      hipEventRecord(a, s);
      for (int r = 0; r < 2; ++r) {
        dispatch_conv<T>(G, s, 0);
        dispatch_conv<T>(G, s, 1);
      }
      hipEventRecord(b, s);
      float t = 0.f;
      if (hipEventSynchronize(b) != hipSuccess || hipEventElapsedTime(&t, a, b) != hipSuccess) {
        ok = false;
        break;
      }
      if (ms < 0.0 || t / 2.0 < ms) ms = t / 2.0;
    }
    if (!ok) ms = -1.0;
  }
  hipDeviceSynchronize();
  if (a) hipEventDestroy(a);
  if (b) hipEventDestroy(b);
  hipFree(work);
  hipFree(Pt.conv_spec);
  Pt.conv_spec = nullptr;
  hipFree(f);
  hipFree(ws);
  return ms;
}

static std::pair<int, int> autotune_conv(mlc_context* ctx, const mlc_plan_info& I, const double* G1) {
  const std::vector<int> key{I.n, I.e, I.conv_precision, I.Q, I.Z};
  auto it = ctx->tuned.find(key);
  if (it != ctx->tuned.end()) return it->second;
  const int Mmin = 2 * (I.n + I.e) + 1, Wp = I.Wa + 2 * I.b;
  std::pair<int, int> best{-1, 1};
  double best_ms = 0.0;
  // every built torus, and for each the z planes per block of the output
  // pass (the tile of output planes a block walks through)
  for (int M : kFftSizes) {
    if (M < Mmin || M / 2 > I.Z || !conv_size_ok(I.conv_precision, I.n, M)) continue;
    for (int zpb : {1, 2, 3, 5, 8}) {
      if (zpb > Wp) continue;
      const double ms = I.conv_precision == MLC_CONV_FP32 ? time_conv<float>(ctx, I, G1, M, zpb)
                                                            : time_conv<double>(ctx, I, G1, M, zpb);
      if (ms > 0.0 && (best.first < 0 || ms < best_ms)) { best = {M, zpb}; best_ms = ms; }
    }
  }
  if (best.first > 0) ctx->tuned[key] = best;
  return best;
}
