/*
 * mlc.h -- C ABI of libmlc, a two-level Method of Local Corrections solver
 * for the free-space Poisson equation  Delta phi = f  on MI355X (gfx950).
 *
 * The operation is the fully discrete two-level algorithm of Kavouklis &
 * Colella, "Computation of Volume Potentials on Structured Grids via the
 * Method of Local Corrections" (sec. 4.1, steps 1-3 and the final
 * Mehrstellen correction), with the discrete Green's function built as in
 * appendix A.1 and local convolutions by Hockney's method (appendix A.2).
 *
 * Conventions shared by every call
 *  - Every call returns mlc_status; MLC_OK == 0, errors are negative.  No C++
 *    exception or abort crosses this boundary.
 *  - Grids are cubes of N cells per axis, (N+1)^3 nodes g h, g in [0, N]^3, or
 *    boxes of B0 x B1 x B2 cells (mlc_problem.box_cells), solved inside their
 *    enclosing cube.
 *    Node arrays are float64, C order [g0][g1][g2] (g2 fastest), length
 *    (N+1)^3.  f must vanish on the outer boundary nodes (the charge is
 *    supported inside the domain, sec. 4).
 *  - Pointers called "device" are HIP device addresses on the context's GPU;
 *    the caller owns them and keeps them alive until the work enqueued on
 *    the given stream has completed.  "stream" is a hipStream_t (NULL = the
 *    default stream).  Work is enqueued asynchronously; no call synchronises
 *    the device except where stated.  A solve also runs some stages on a
 *    second stream that the context creates for each caller stream (default
 *    priority, kept until mlc_context_destroy); it forks from and joins back
 *    into the caller stream with events, so when the caller stream passes a
 *    solve, all of that solve's work has ended.
 *  - Arguments are validated before anything is enqueued; on an error
 *    nothing is written to any output.  With MLC_CHECK=1 in the environment,
 *    mlc_solve and mlc_solve_batched also check on the device that each f
 *    vanishes on the outer boundary nodes (MLC_ERR_INVALID_ARG otherwise);
 *    that check synchronises the caller's stream.
 *  - With MLC_TRACE=<file> in the environment, each mlc_solve and
 *    mlc_solve_batched call appends one JSON line to <file>: its status,
 *    wall time, problems, and per stage timer the launches and device
 *    milliseconds, at every level of a multilevel plan ("L1." prefixes the
 *    next coarser level).  A traced call synchronises the caller's stream.
 *  - A context is used from one host thread at a time; plans are immutable
 *    after creation and may be used by several solves in sequence.
 */
#ifndef MLC_H
#define MLC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  MLC_OK = 0,
  MLC_ERR_INVALID_ARG = -1,   /* malformed argument or inconsistent sizes            */
  MLC_ERR_UNSUPPORTED = -2,   /* well formed, but outside what this build implements */
  MLC_ERR_OUT_OF_MEMORY = -3, /* device allocation failed or budget exceeded          */
  MLC_ERR_DEVICE = -4,        /* a HIP runtime error; see mlc_last_error              */
  MLC_ERR_BUSY = -5,          /* server admission queue full                          */
  MLC_ERR_NOT_READY = -6      /* server ticket still in flight                        */
} mlc_status;

/* Arithmetic of the local convolutions (sec. 4.1 step 1).  Every other step
 * (DGF, moments, far fields, coarse solve, boundary values, Dirichlet
 * solves) is always float64. */
typedef enum { MLC_CONV_FP64 = 0, MLC_CONV_FP32 = 1 } mlc_conv_precision;

/* The problem, in the paper's notation (sec. 4, sec. 7.1). */
typedef struct {
  int32_t n_cells;        /* N: cells per axis; N % patch == 0                          */
  double h;               /* mesh spacing > 0 (unit cube: 1/N)                          */
  int32_t patch;          /* n: cells per patch edge; n % 4 == 0, n >= 8                */
  double alpha, beta;     /* localisation radii in units of R = n h / 2; 1 <= alpha <= beta;
                             the margins ceil((r-1) n / 2) must be multiples of 4 (Nref)  */
  int32_t P;              /* Legendre truncation: modes with |p|_1 < P; 1 <= P <= 9     */
  int32_t Q;              /* Mehrstellen operator: 4 -> L19, 6 -> L27                   */
  int32_t interp_b;       /* coplanar interpolation radius b (order 2b+2); 0 -> Q/2     */
  int32_t conv_precision; /* mlc_conv_precision                                        */
  int32_t fft_size;       /* Hockney torus edge M of the local convolutions: > 0 exact;
                             0 -> the smallest built size >= 2(n+e)+1; -1 -> autotuned:
                             plan creation times every built size, each with every
                             count of output planes per block in {1, 2, 3, 5, 8}, on a
                             probe grid and keeps the fastest pair (cached per
                             patch-work class in the context; mlc_problem_info
                             reports the smallest size and the default count)       */
  int32_t dgf_half_width; /* Z of the DGF table [-Z, Z]^3 (solved on [-2Z, 2Z]^3); 0 -> 128 */
  int32_t levels;         /* levels of the method (sec. 5): 0 or 2 -> the two-level method;
                             3 or 4 -> multilevel: the coarse convolution is replaced by
                             the method one level up (spacing 4h, the same n, radii, P,
                             Q, b, precision) on a patch box extending m = the smallest
                             multiple of n >= d_beta/4 + b + 1 cells past [0, N/4]
                             (proper nesting), recursively; needs (N/4) % n == 0     */
  double level_alpha[3];  /* multilevel: the inner radius alpha at the coarser levels that
                             are solved by the method (sec. 7.2 raises it there to bound
                             the error of the truncated Legendre expansions):
                             level_alpha[k] at k+1 levels above the finest; 0 -> the
                             radius of the next finer level; same rules as alpha;
                             entries past levels - 2 are ignored                     */
  int32_t rhs_order;      /* 0 or 4: the fourth-order method, phi = phi~ + C2 h^2 f (sec.
                             4.1, final step); 6 (Q = 6 only): the method applied to the
                             modified right-hand side of sec. 2 eq. msCorr, with the
                             27-point operator's h^4 term from its truncation error
                             (appendix A.1): f~ = f + (h^2/12) (Delta f)_4 + (h^4/360)
                             (Delta^2 + 2 (d_xxyy + d_yyzz + d_zzxx)) f by differences of
                             f (fourth order for Delta f, second for the h^4 term), and
                             no final correction: sixth order in h up to the method's
                             own errors.  f must vanish within two nodes of the faces
                             (MLC_CHECK then checks the three outer node layers); the
                             workspace holds f~, (N+1)^3 doubles more;
                             mlc_solve_analytic refuses it                           */
  int32_t skip_empty;     /* 1: patches whose node charge (all (n+1)^3 nodes of the closed
                             patch) is zero skip their local convolutions, found on the
                             device at every solve; their local fields and moments are
                             zero, so the result is the same as with 0 (the method only
                             needs patches over the support of f, sec. 1); the far-field
                             sums also pass over source patches with zero moments.  0:
                             every patch is convolved                                */
  int32_t box_cells[3];   /* a box domain [0, B0] x [0, B1] x [0, B2] (cells per axis, each
                             a multiple of n; n_cells must then be 0): f and phi are
                             (B0+1)(B1+1)(B2+1) node arrays, C order, axis 2 fastest.  The
                             box is solved inside the smallest cube of N >= max B_d cells
                             that the plan can run (N a multiple of n, of 4n with three
                             levels, 16n with four), f padded with zeros: the free-space
                             solution on the box does not depend on the padding (with
                             skip_empty the empty padding patches cost no convolutions).
                             All zero: the cube of n_cells.  mlc_solve_analytic refuses
                             box problems                                            */
  double origin[3];       /* physical coordinates of node (0,0,0); recorded, not used    */
  int32_t max_live;       /* > 0: keep per-patch convolution buffers for at most this many
                             patches with charge (implies skip_empty): each solve finds
                             them on the device, waits for its stream once to list them,
                             and returns MLC_ERR_OUT_OF_MEMORY if there are more.  For
                             large grids whose charge covers few patches (e.g. 2048^3).
                             mlc_solve and
                             mlc_solve_analytic only: batches, graphs, the static
                             scratch and the server refuse it (MLC_ERR_UNSUPPORTED).
                             The coarser levels of a multilevel plan keep every patch.
                             0: buffers for every patch                              */
} mlc_problem;

/* Sizes derived from an mlc_problem (all counts per axis unless noted). */
typedef struct {
  int32_t N, n, P, Q, b, K;          /* K = P(P+1)(P+2)/6 Legendre moments per patch     */
  int32_t d_alpha, d_beta;           /* margins of Omega_alpha, Omega_beta (fine cells)  */
  int32_t e;                         /* d_alpha + 4b: half-margin of the local field box */
  int32_t patches_per_axis, npatch;  /* N/n and (N/n)^3                                  */
  int32_t M, M_coarse, M_table;      /* Hockney torus edges: local, coarse, far-field    */
  int32_t Wc;                        /* coarse samples of a local field per axis         */
  int32_t Wa, nplanes_a;             /* skeleton planes of a local field: width, count   */
  int32_t S_lo, Ns;                  /* coarse right-hand side box [S_lo, S_lo+Ns-1]     */
  int32_t O_lo, No;                  /* coarse solution box [O_lo, O_lo+No-1]            */
  int32_t Z;                         /* DGF table half-width                             */
  int32_t conv_precision;
  double h, H;                       /* fine and coarse (4h) spacing                     */
  int32_t out_planes;                /* z planes per block of the local convolutions'
                                        output pass (tuned with fft_size = -1)           */
  int32_t levels;                    /* levels of the method (2: two-level)              */
  int32_t level_margin, level_N;     /* multilevel: the next level's box [-m, N/4 + m],
                                        m = level_margin, of level_N cells; else 0     */
  double alpha, beta;                /* localisation radii of this level                 */
  double level_alpha[3];             /* alpha at 1, 2, 3 levels above (resolved: no 0)  */
  int32_t rhs_order;                 /* 4 or 6 (mlc_problem.rhs_order, 0 -> 4)           */
  int32_t skip_empty;                /* mlc_problem.skip_empty                           */
  int32_t box[3];                    /* cells per axis of the problem's domain (N, N, N for
                                        a cube); N above is the cube it is solved in      */
  double origin[3];                  /* mlc_problem.origin                               */
  int32_t slots;                     /* patches the per-patch buffers hold (npatch, or
                                        min(max_live, npatch))                           */
} mlc_plan_info;

typedef struct mlc_context mlc_context;
typedef struct mlc_plan mlc_plan;

/* Human-readable name of a status code (static storage). */
const char* mlc_status_string(mlc_status s);

/* Validate a problem and fill its derived sizes, on the host only (no
 * device is touched).  Returns MLC_ERR_INVALID_ARG for malformed input,
 * MLC_ERR_UNSUPPORTED for valid problems this build cannot run. */
mlc_status mlc_problem_info(const mlc_problem* prob, mlc_plan_info* out);

/* Create a context on HIP device `device`.  hbm_budget_bytes caps the
 * resident device memory of the context (0 = no cap): its DGF tables, the
 * tables of every live plan and the arenas of its servers.  A DGF build,
 * mlc_plan_create or mlc_server_create that would exceed the cap returns
 * MLC_ERR_OUT_OF_MEMORY and keeps nothing; destroying a plan or server gives
 * its share back.  Caller-owned workspaces and the transient buffers of a
 * build are not counted.  Returns MLC_ERR_DEVICE if the device cannot be
 * opened. */
mlc_status mlc_context_create(int device, size_t hbm_budget_bytes, mlc_context** out);
mlc_status mlc_context_destroy(mlc_context* ctx);

/* Copy the last error message of the context (NUL-terminated, truncated to
 * len).  ctx may be NULL for errors raised before a context existed. */
mlc_status mlc_last_error(mlc_context* ctx, char* buf, size_t len);

/* Build a plan: validates the problem, then builds (or reuses, per Q and Z)
 * the resident DGF table (appendix A.1), the DGF spectra of the local and
 * coarse convolutions and the far-field tables of the Legendre modes
 * (sec. 4.1: built once, kept for every solve).  Synchronises the device. */
mlc_status mlc_plan_create(mlc_context* ctx, const mlc_problem* prob, mlc_plan** out);
mlc_status mlc_plan_destroy(mlc_plan* plan);
mlc_status mlc_plan_get_info(const mlc_plan* plan, mlc_plan_info* out);

/* Bytes of device workspace a solve with this plan needs.  It includes one
 * chunk of the local convolutions' z-transformed spectra (equal patch
 * chunks of at most 6 GB; the environment variable MLC_CONV_CHUNK, read once
 * per process, caps the patches per chunk instead). */
mlc_status mlc_plan_workspace_bytes(const mlc_plan* plan, size_t* bytes);

/* The same figure computed from the problem alone, on the host (no device
 * is touched): equal to mlc_plan_workspace_bytes of the problem's plan, and
 * for fft_size = -1 the largest figure over the tori the autotuner may pick,
 * so that it bounds the plan's own. */
mlc_status mlc_problem_workspace_bytes(const mlc_problem* prob, size_t* bytes);

/* One two-level MLC solve (sec. 4.1): f (device, (N+1)^3 float64, read
 * only) -> phi (device, (N+1)^3 float64, fully overwritten).  workspace is
 * device memory of at least mlc_plan_workspace_bytes bytes, owned by the
 * caller; its contents after the solve are the intermediates listed under
 * mlc_workspace_view.  Enqueued on `stream`. */
mlc_status mlc_solve(mlc_plan* plan, const double* f, double* phi,
                     void* workspace, size_t ws_bytes, void* stream);

/* The same solve for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * instead of a caller workspace it uses the library's static scratch, a
 * device array of MLC_STATIC_SCRATCH_BYTES of which each GPU the library runs
 * on holds one copy until the process ends, and it runs every stage on
 * `stream` (no side stream).  It calls no device allocator and creates no
 * stream or event; f, phi and the plan are as for mlc_solve (the plan, with
 * its resident tables, is built beforehand by mlc_plan_create).  Returns
 * MLC_ERR_UNSUPPORTED when mlc_plan_workspace_bytes of the plan exceeds the
 * scratch (for example every 32^3-cell-patch problem above 64^3 cells, or
 * 16^3-cell patches above 96^3 cells with float32 convolutions).  Every call
 * on one GPU shares that GPU's scratch, which keeps the last call's
 * contents (a solve writes every scratch value it reads): calls that overlap
 * on one GPU (on different streams, or from different threads) race, and
 * must be ordered by the caller.  The MLC_CHECK device check is not run. */
#define MLC_STATIC_SCRATCH_BYTES ((size_t)512 << 20)
mlc_status mlc_solve_static(mlc_plan* plan, const double* f, double* phi, void* stream);

/* Charges given analytically (sec. 4.1 step 1: the Legendre coefficients
 * are then computed by Gauss integration instead of Boole's rule): a sum of
 * radial terms f(x) = weight * profile(|x - centre| / radius), each zero for
 * |x - centre| >= radius, in the physical coordinates of the grid (node g at
 * g h).  Profiles, r = |x - centre| / radius < 1:
 *   MLC_PROFILE_BUMP         (1 - r^2)^4
 *   MLC_PROFILE_SMOOTH       (r - r^2)^4            (sec. 7.1's charge)
 *   MLC_PROFILE_OSCILLATORY  (r - r^2)^2 sin^2(param r / 2)   (sec. 7.2's, param = gamma) */
typedef enum { MLC_PROFILE_BUMP = 0, MLC_PROFILE_SMOOTH = 1, MLC_PROFILE_OSCILLATORY = 2 } mlc_profile;
typedef struct {
  double centre[3];
  double radius;          /* > 0 */
  double weight;
  double param;           /* oscillatory: gamma; ignored otherwise */
  int32_t profile;        /* mlc_profile */
} mlc_radial_charge;
#define MLC_MAX_RADIAL_TERMS 16

/* mlc_solve for a charge given as nterms (1..MLC_MAX_RADIAL_TERMS) radial
 * terms (host array, read during the call).  The library samples the charge
 * on the (N+1)^3 nodes into f (device, caller-owned, fully overwritten; it
 * must vanish on the outer boundary nodes: MLC_ERR_INVALID_ARG if a term's
 * support reaches them) and solves with it, except that each patch's Legendre
 * coefficients are the composite Gauss-Legendre integrals
 *   c_p = R^{3/2} sum_k W_k f(x_k) qhat_p(t_k)
 * over gauss_points (1..4) points per cell per axis of the patch's n cells
 * (the inner products <Q^p, f> of the L2 projection, sec. 3; for products of
 * modes up to degree 2 gauss_points - 1 per cell the rule is exact, so no
 * Gram correction is applied).  Workspace and stream as for mlc_solve. */
mlc_status mlc_solve_analytic(mlc_plan* plan, int32_t nterms, const mlc_radial_charge* terms, int32_t gauss_points,
                              double* f, double* phi, void* workspace, size_t ws_bytes, void* stream);

/* Several independent problems in one pass: the per-patch stages of all
 * problems run in shared launches (their plans must share n, alpha, b, Q,
 * the torus M and the conv precision); coarse solves run per problem.
 * f[k], phi[k] are device arrays of plan k's size; workspace must hold
 * mlc_batch_workspace_bytes(count, plans) bytes. */
mlc_status mlc_batch_workspace_bytes(int32_t count, mlc_plan* const* plans, size_t* bytes);
mlc_status mlc_solve_batched(int32_t count, mlc_plan* const* plans, const double* const* f,
                             double* const* phi, void* workspace, size_t ws_bytes, void* stream);

/* A batched solve captured once into a HIP graph and replayed: the arguments
 * are those of mlc_solve_batched and stay bound to the graph (the caller keeps
 * the plans, arrays and workspace alive and unmoved while the graph exists;
 * a replay reads the current contents of f).  mlc_graph_create captures the
 * launches of the batch (both streams' branches) on a stream of its own and
 * instantiates the graph, enqueueing no work; mlc_graph_launch enqueues one
 * replay on `stream`, equal bit for bit to mlc_solve_batched with the same
 * arguments; replays of one graph, or of graphs sharing a workspace, must be
 * ordered by the caller.  Per-kernel timing must be off for the captured
 * plans (MLC_ERR_INVALID_ARG otherwise) and the MLC_CHECK device check is not
 * part of a graph. */
typedef struct mlc_graph mlc_graph;
mlc_status mlc_graph_create(int32_t count, mlc_plan* const* plans, const double* const* f, double* const* phi,
                            void* workspace, size_t ws_bytes, mlc_graph** out);
mlc_status mlc_graph_launch(mlc_graph* graph, void* stream);
mlc_status mlc_graph_destroy(mlc_graph* graph);

/* Intermediates of the last solve held in a workspace (device pointers into
 * it; valid until the workspace is reused):
 *   MLC_VIEW_MOMENTS      float64 [npatch][K]: c_{i,p}, patches in C order of i,
 *                         modes by total degree then descending lexicographic p
 *   MLC_VIEW_COARSE_RHS   float64 [Ns]^3: F^H on [S_lo, S_lo+Ns-1]^3
 *   MLC_VIEW_COARSE_PHI   float64 [No]^3: phi^H on [O_lo, O_lo+No-1]^3
 *   MLC_VIEW_BOUNDARY     float64 [(N+1)^3]: phi^B on skeleton nodes (the other
 *                         entries are not written by a solve)
 *   MLC_VIEW_LOCAL_COARSE conv precision [npatch][Wc]^3: phi_i at the coarse
 *                         nodes of its box G(Omega_alpha, 4b), starting at -e
 *   MLC_VIEW_LOCAL_PLANES conv precision [npatch][3][nplanes_a][Wa][Wa]:
 *                         phi_i on its skeleton planes inside Omega_alpha,
 *                         plane normal d, planes at -d_alpha rounded up to a
 *                         multiple of n, in-plane axes ascending from -d_alpha
 *   (with max_live the two local views hold [slots] rows: the patches that
 *   carry charge, in increasing patch order; the other patches' fields are 0)
 *   multilevel plans only (levels > 2), the next coarser level:
 *   MLC_VIEW_LEVEL_CHARGE float64 [(level_N+1)^3]: its node charge (F^H placed
 *                         in its box; node 0 at coarse coordinate -level_margin)
 *   MLC_VIEW_LEVEL_PHI    float64 [(level_N+1)^3]: its uncorrected solution
 *   MLC_VIEW_LEVEL_WORKSPACE  the workspace of its own solve (for the views of
 *                         mlc_plan_coarse_level's plan, recursively)
 * (MLC_VIEW_COARSE_PHI of a multilevel plan is that solution on [O_lo,
 * O_lo+No-1]^3, the values the boundary interpolation reads.)
 *   sixth-order plans only (rhs_order 6):
 *   MLC_VIEW_CHARGE       float64 [(N+1)^3]: the modified right-hand side f~
 *                         the method solved */
enum {
  MLC_VIEW_MOMENTS = 0, MLC_VIEW_COARSE_RHS = 1, MLC_VIEW_COARSE_PHI = 2,
  MLC_VIEW_BOUNDARY = 3, MLC_VIEW_LOCAL_COARSE = 4, MLC_VIEW_LOCAL_PLANES = 5,
  MLC_VIEW_LEVEL_CHARGE = 6, MLC_VIEW_LEVEL_PHI = 7, MLC_VIEW_LEVEL_WORKSPACE = 8,
  MLC_VIEW_CHARGE = 9
};
/* The plan of the next coarser level of a multilevel plan (owned by it;
 * MLC_ERR_INVALID_ARG for a two-level plan). */
mlc_status mlc_plan_coarse_level(const mlc_plan* plan, const mlc_plan** level);
mlc_status mlc_workspace_view(const mlc_plan* plan, void* workspace, int32_t which,
                              void** ptr, size_t* bytes);

/* The resident DGF table G^{h=1} on [-Z, Z]^3 ((2Z+1)^3 float64, C order,
 * centre at index (Z, Z, Z)) of operator Q, building it if needed
 * (appendix A.1).  The pointer stays owned by the context.  Synchronises. */
mlc_status mlc_dgf_table(mlc_context* ctx, int32_t Q, int32_t Z, const double** table);

/* Per-kernel timing of solves (instrumentation, not part of the method).
 * While enabled, every kernel a solve with this plan enqueues is bracketed
 * by HIP events on the stream it runs on (the caller stream, or the side
 * stream for the stages that overlap the local convolutions, whose
 * durations then include the sharing of the chip).  mlc_plan_timing waits for the
 * recorded events, then reports, per kernel name, the number of launches
 * and their summed duration in milliseconds since timing was enabled; it
 * fills at most `max` entries and sets *count to the number of distinct
 * kernels.  Enabling resets the sums. */
typedef struct {
  char name[48];
  int32_t launches;
  double total_ms;
} mlc_kernel_time;
mlc_status mlc_plan_set_timing(mlc_plan* plan, int32_t enable);
mlc_status mlc_plan_timing(mlc_plan* plan, mlc_kernel_time* out, int32_t max, int32_t* count);

/* ------------------------------------------------------------- serving
 * A request loop over one context.  mlc_server_submit queues a solve
 * (problem, f, phi as for mlc_solve) and returns at once; the server's own
 * host thread builds plans on first use (kept resident: DGF tables, spectra
 * and far-field tables per distinct problem), admits queued requests in
 * arrival order as a stream slot and workspace memory free up, and launches
 * queued requests whose patch work is identical (same n, radii, P, Q, b,
 * torus, precision; any N) together through the batched solve.  Launches run
 * on several streams, so requests admitted while others run overlap with
 * them on the device.  Workspaces come from one device arena of
 * workspace_budget_bytes allocated at creation; a request whose workspace
 * alone exceeds it is refused at submit.
 *
 * f and phi are device arrays the caller owns and keeps alive (f unchanged)
 * until the ticket reports done.  A request's result does not depend on
 * which other requests share its launch (the per-problem arithmetic is the
 * same).  Server calls may come from one caller thread at a time; while a
 * server runs, its context may still be used from that thread (plan builds
 * are serialised inside the context). */
typedef struct {
  size_t workspace_budget_bytes; /* device arena for solve workspaces; 0 -> 16 GiB          */
  int32_t streams;               /* concurrent launches (HIP streams, default priority);
                                    0 -> 2, at most 8                                        */
  int32_t max_batch;             /* most requests per launch; 0 -> 16                         */
  int32_t max_queue;             /* unfinished requests allowed; 0 -> 4096                    */
} mlc_server_config;

typedef struct {
  int32_t status;      /* mlc_status of the request's solve                              */
  int32_t batch_size;  /* requests in the launch that ran it                             */
  double queue_ms;     /* submit -> launch enqueued (includes a first-use plan build)     */
  double device_ms;    /* the launch's device time, from HIP events around it            */
  double total_ms;     /* submit -> completion observed by the server thread             */
} mlc_timing;

typedef struct mlc_server mlc_server;

/* Start a server on ctx (allocates the arena and streams, starts its thread). */
mlc_status mlc_server_create(mlc_context* ctx, const mlc_server_config* cfg, mlc_server** out);
/* Build the problem's plan now (resident tables) instead of at first use.
 * Synchronises the device. */
mlc_status mlc_server_prepare(mlc_server* srv, const mlc_problem* prob);
/* Queue one solve.  MLC_ERR_INVALID_ARG / MLC_ERR_UNSUPPORTED for a bad
 * problem, MLC_ERR_OUT_OF_MEMORY if its workspace exceeds the arena,
 * MLC_ERR_BUSY if max_queue requests are unfinished.  *ticket is nonzero.
 * f must already hold its values on the device: the server's streams wait on
 * no caller stream, so a caller that fills f asynchronously synchronises
 * that work before submitting.  With MLC_CHECK=1 each request's f is checked
 * alone (a failing request ends with MLC_ERR_INVALID_ARG without affecting
 * the others). */
mlc_status mlc_server_submit(mlc_server* srv, const mlc_problem* prob, const double* f, double* phi,
                             uint64_t* ticket);
/* Status of a ticket: MLC_ERR_NOT_READY (*done = 0) while queued or
 * running; once finished, *done = 1, *t (if not NULL) is filled, the ticket
 * is released (polling it again is MLC_ERR_INVALID_ARG) and the return value
 * is the solve's own status. */
mlc_status mlc_server_poll(mlc_server* srv, uint64_t ticket, int32_t* done, mlc_timing* t);
/* Block until every submitted request has finished. */
mlc_status mlc_server_drain(mlc_server* srv);
/* Drain, stop the thread, free plans, arena and streams. */
mlc_status mlc_server_destroy(mlc_server* srv);

#ifdef __cplusplus
}
#endif
#endif /* MLC_H */
