/*
 * mistencil -- structured-grid 3D stencil sweeps for MI355X (gfx950).
 *
 * C ABI of the hot path of Brown et al., "Fortran performance optimisation
 * and auto-parallelisation by leveraging MLIR-based domain specific
 * abstractions in Flang" (SC-W 2023): the stencils its stencil-discovery
 * flow extracts from Fortran loop nests (Section 3) -- the 7-point Laplace
 * iteration and the fused Piacsek-Williams advection source term of the
 * evaluation (Section 4.1) -- plus the residual-norm reduction that decides
 * convergence, FP32-storage refinement, batched solves and a learned warm
 * start.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Fields. A field lives in caller-owned device memory. Its layout follows
 * the paper's Fortran column-major order (first index contiguous, Section
 * 2.2): element (i, j, k), i = x, sits at
 *     base[(k + 1) * sz + (j + 1) * sy + (i + 1)]
 * for halo-inclusive indices i in [-1, nx], j in [-1, ny], k in [-1, nz];
 * the base pointer addresses halo cell (-1, -1, -1). The interior is
 * [0, nx) x [0, ny) x [0, nz) and the halo is one cell wide, as the bounds
 * of stencil.apply's input and output temps in Listing 2 show. Strides are
 * in elements, x stride is 1, sy >= nx + 2 and sz >= sy * (ny + 2) (a padded
 * pitch is allowed). Outputs are written on the interior only; the halo of
 * an output is never touched.
 *
 * Streams. `stream` is a hipStream_t passed as void*; NULL is the default
 * stream. Entry points marked "async" only enqueue work. Host structs are
 * read before the call returns.
 *
 * Ownership. The library keeps no pointer after a call returns (except for
 * work still in flight on `stream`) and allocates no field-sized memory:
 * scratch comes from a caller-owned device workspace whose size the
 * matching *_workspace_bytes function returns.
 *
 * Errors. Every int-returning entry point returns one of the MS_* codes
 * below; no exception crosses the ABI. ms_last_error() returns a
 * thread-local message for the last non-OK return on the calling thread.
 */
#ifndef MISTENCIL_H
#define MISTENCIL_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ---------------------------------------------------- */
#define MS_OK 0
#define MS_NOT_CONVERGED 1  /* solve hit its sweep/outer cap; result filled */
#define MS_EINVAL (-1)      /* null pointer, bad extents/strides, aliasing, |offset| > 1 */
#define MS_EUNSUPPORTED (-2) /* dtype, tap count or option not supported */
#define MS_EHIP (-3)        /* HIP runtime error (message in ms_last_error) */
#define MS_EWORKSPACE (-4)  /* workspace missing or too small */
#define MS_ENONFINITE (-5)  /* a residual norm came out NaN or Inf */

/* ---- element types --------------------------------------------------- */
#define MS_F64 0
#define MS_F32 1

/* ---- grid descriptor ------------------------------------------------- */
typedef struct {
  int32_t nx, ny, nz; /* interior extents, each >= 1 */
  int32_t reserved;   /* must be 0 */
  int64_t sy, sz;     /* element strides of y and z (x stride is 1) */
} ms_grid;

/* Thread-local text of the last error on this thread ("" if none). */
const char* ms_last_error(void);

/* Library version string. */
const char* ms_version(void);

/* ---- general constant-offset stencil ----------------------------------
 * The paper's stencil.apply (Section 2.2, Listing 2): a region evaluated at
 * every interior cell p that reads the input at constant offsets:
 *   out[p] = scale * ((...((w0*in[p+o0]) + w1*in[p+o1]) + ...) + rhs_coef*rhs[p])
 * accumulated in tap order, in the arithmetic of `dtype` (weights and
 * coefficients are rounded to FP32 for MS_F32). The rhs term is present only
 * when rhs != NULL. 1 <= ntaps <= 27, each |dx|,|dy|,|dz| <= 1.
 * in, rhs and out share the grid `g`. out may not alias in or rhs (the
 * apply is out-of-place) -> MS_EINVAL. Async. */
typedef struct {
  int8_t dx, dy, dz;
  int8_t reserved[5];
  double w;
} ms_tap;

typedef struct {
  int32_t ntaps;
  int32_t reserved;
  const ms_tap* taps; /* host array of ntaps taps */
  double rhs_coef;
  double scale;
} ms_stencil;

int stencil_apply(const ms_stencil* st, const ms_grid* g, int dtype,
                  const void* in, const void* rhs, void* out, void* stream);

/* ---- residual norm ------------------------------------------------------
 * ||f - L(u)||_2 over the interior, L(u) = S(u) - 6u with S the six-neighbour
 * sum of the 7-point Laplace stencil (Section 4.1), evaluated per cell as
 * r = f - (S - u*6) and accumulated in FP64 (FP32 fields are widened
 * exactly first). f may be NULL (Laplace, f = 0). The reduction order is
 * fixed, so repeated calls give identical bits.
 * norm_out: device pointer if out_on_device != 0 (async), else host pointer
 * (the call then synchronises `stream`).
 * work: device workspace of at least residual_workspace_bytes(g) bytes. */
size_t residual_workspace_bytes(const ms_grid* g);
int residual_norm(const ms_grid* g, int dtype, const void* u, const void* f,
                  double* norm_out, int out_on_device, void* work,
                  size_t work_bytes, void* stream);

/* ---- runtime-compiled stencil programs ---------------------------------
 * stencil.apply with an arbitrary arithmetic body (Section 2.2 and
 * Listing 2: a region of arith operations on constant-offset accesses of
 * input temps, writing the interior out-of-place; Section 3: the flow
 * extracts such regions from Fortran loop nests). The region is given as
 * text, parsed and compiled to a device kernel with hipRTC (gfx950) by
 * ms_jit_compile, once; ms_jit_apply runs it on any grid.
 *
 * Language. Statements end with ';'; '#' starts a comment to end of line.
 *   field a, b, ...;     input fields (at most 8), in argument order
 *   param p, ...;        scalar parameters (at most 8), passed as double
 *   profile t, ...;      per-level coefficients (at most 4): one value per
 *                        interior level k (nz values), read as t at level k
 *   let x = expr;        a named per-cell value (at most 256)
 *   out o = expr;        an output field (1 to 4), in argument order
 * expr: + - (left-associative) over terms; term: * / (left-associative)
 * over unary; unary: '-' unary | primary; primary: a decimal number
 * (digits [. digits] [e|E [+|-] digits]), a field access a[dx,dy,dz]
 * with integer offsets in [-1, 1] (a bare field name is a[0,0,0]), a
 * param, a profile, a let name, or '(' expr ')'. Names are unique across
 * all declarations; outputs cannot be read.
 * Arithmetic: every operation is evaluated in the program's dtype exactly
 * in the order the text gives (no contraction, no reassociation, IEEE
 * division, round to nearest); constants are rounded to double, then to
 * the dtype; params are rounded from double to the dtype at launch.
 *
 * ms_jit_compile: program (host string, at most 64 KiB), dtype MS_F64 or
 * MS_F32; *out receives a handle owned by the caller (ms_jit_free). Parse
 * errors -> MS_EINVAL with "line L col C: ..." in ms_last_error; hipRTC
 * failures -> MS_EHIP. Needs no GPU. Synchronous.
 * ms_jit_apply: fields / profiles / outputs are arrays of device pointers
 * (fields and outputs on grid g, profiles of nz values), params a host
 * array; each count must equal the program's. Outputs are written on the
 * interior only and must not overlap any input or each other (MS_EINVAL).
 * Loads the code on the current device on first use. Async on `stream`.
 * ms_jit_signature / ms_jit_name: declared counts and names (kind
 * MS_JIT_FIELD, MS_JIT_PARAM, MS_JIT_PROFILE, MS_JIT_OUTPUT); ms_jit_name
 * returns NULL out of range. ms_jit_source: the generated HIP source, valid
 * until ms_jit_free. */
typedef struct ms_jit_stencil ms_jit_stencil;
#define MS_JIT_FIELD 0
#define MS_JIT_PARAM 1
#define MS_JIT_PROFILE 2
#define MS_JIT_OUTPUT 3
int ms_jit_compile(const char* program, int dtype, ms_jit_stencil** out);
int ms_jit_apply(ms_jit_stencil* st, const ms_grid* g, const void* const* fields,
                 int n_fields, const double* params, int n_params,
                 const void* const* profiles, int n_profiles,
                 void* const* outputs, int n_outputs, void* stream);
int ms_jit_signature(const ms_jit_stencil* st, int* n_fields, int* n_params,
                     int* n_profiles, int* n_outputs);
const char* ms_jit_name(const ms_jit_stencil* st, int kind, int index);
const char* ms_jit_source(const ms_jit_stencil* st);
void ms_jit_free(ms_jit_stencil* st);

/* ---- fixed number of Jacobi sweeps -------------------------------------
 * The 7-point Laplace/Poisson iteration of Section 4.1 as an out-of-place
 * (Jacobi) update, u'(p) = (S(p) - f(p)) * fl(1/6) (u'(p) = S(p) * fl(1/6)
 * when f is NULL), with ping-pong buffers u and u_tmp (same grid; u_tmp's
 * halo must hold the same Dirichlet values as u's). Exactly n >= 0 sweeps.
 * u_n lands in u if n is even, else in u_tmp.
 * res_dev (device, may be NULL): n + 1 doubles, res_dev[k] = ||r(u_k)||,
 * k = 0..n; entries 0..n-1 come from the residual fused into each sweep,
 * entry n from one trailing residual pass.
 * dtype MS_F64, or MS_F32 (FP32 storage and sweep arithmetic, FP64 norms).
 * work: jacobi_sweeps_workspace_bytes(g) bytes. Async. */
size_t jacobi_sweeps_workspace_bytes(const ms_grid* g);
int jacobi_sweeps(const ms_grid* g, int dtype, void* u, void* u_tmp,
                  const void* f, int64_t n, double* res_dev, void* work,
                  size_t work_bytes, void* stream);

/* As jacobi_sweeps, with temporal_block sweeps fused into each pass over
 * memory (1 or 2). With 2, each pass reads u_k and f once and writes
 * u_{k+2}; the intermediate iterate stays on chip; an odd n ends with one
 * single sweep. Per-cell arithmetic, results and res_dev are identical to
 * jacobi_sweeps. u_n lands in u if the number of passes (n for 1,
 * n/2 + n%2 for 2) is even, else in u_tmp. Same workspace. Async. */
int jacobi_sweeps_tb(const ms_grid* g, int dtype, void* u, void* u_tmp,
                     const void* f, int64_t n, int temporal_block,
                     double* res_dev, void* work, size_t work_bytes,
                     void* stream);

/* As jacobi_sweeps_tb, for callers that cannot allocate device memory (code
 * under stream capture, tight serving loops, harnesses that forbid it): no
 * workspace argument, and the call allocates nothing. The residual partials
 * live in a fixed device array of jacobi_sweeps_noalloc_scratch_bytes()
 * bytes (2 MiB) per GPU, held until the process ends; every grid that
 * jacobi_sweeps accepts fits it (a larger need returns MS_EWORKSPACE).
 * Calls on one GPU share that array: calls that overlap in time on one GPU
 * (different streams, or different host threads) race and must not be
 * issued; calls in sequence on one stream are safe. Nothing in the array
 * has to start at zero. Results are bit-identical to jacobi_sweeps_tb.
 * The first call on each device looks the array's address up (with that
 * device current). Async. */
size_t jacobi_sweeps_noalloc_scratch_bytes(void);
int jacobi_sweeps_noalloc(const ms_grid* g, int dtype, void* u, void* u_tmp,
                          const void* f, int64_t n, int temporal_block,
                          double* res_dev, void* stream);

/* ---- Jacobi sweeps on a field held in host memory -------------------------
 * Exactly n >= 0 sweeps of jacobi_sweeps on a field that stays in host
 * memory (Section 4.3's data management taken to fields larger than the
 * device holds): u, u_tmp and f (f may be NULL) are HOST pointers with the
 * layout of grid g (page-locked memory, as from hipHostMalloc, lets copies
 * overlap the sweeps); both u and u_tmp carry the Dirichlet halo. The field
 * is cut into z slabs of slab_planes interior planes; each pass uploads a
 * slab with sweeps_per_pass (T) extra planes on either side, runs T sweeps
 * on the device and downloads the slab's own planes, so every value is
 * bit-identical to jacobi_sweeps. Passes alternate between u and u_tmp: the
 * result lands in u if ceil(n / min(T, nz)) is even, else in u_tmp. Two internal
 * streams (default priority) overlap one slab's copies with another's
 * sweeps. No residual norms. work: device, at least
 * jacobi_sweeps_streamed_workspace_bytes(g, dtype, T, slab_planes) bytes
 * (two sets of three slab buffers of slab_planes + 2T + 2 planes). Blocks
 * until done (synchronises `stream` first). T in [1, 4096], slab_planes
 * >= 1. */
size_t jacobi_sweeps_streamed_workspace_bytes(const ms_grid* g, int dtype,
                                              int sweeps_per_pass, int slab_planes);
int jacobi_sweeps_streamed(const ms_grid* g, int dtype, void* u, void* u_tmp,
                           const void* f, int64_t n, int sweeps_per_pass,
                           int slab_planes, void* work, size_t work_bytes,
                           void* stream);

/* ---- fixed number of red-black Gauss-Seidel sweeps ----------------------
 * The Section 4.1 benchmark is a Gauss-Seidel iteration of the same 7-point
 * stencil; its in-place, lexicographic form is sequential, so this is the
 * red-black ordering, which keeps every half-sweep data parallel. Cells with
 * i + j + k even (interior coordinates, 0-based) are red. One sweep: every
 * red cell takes (S - f) * fl(1/6) of the current field, then every black
 * cell takes the same expression of the field with the red cells updated;
 * the six neighbours of a cell always have the other colour. Arguments, the
 * ping-pong buffers, res_dev (||r(u_k)||, k = 0..n, u_k the field after k
 * sweeps), dtype, workspace (jacobi_sweeps_workspace_bytes) and errors are
 * those of jacobi_sweeps; u_n lands in u if n is even, else in u_tmp. Each
 * sweep is one pass over memory. Async. */
int rbgs_sweeps(const ms_grid* g, int dtype, void* u, void* u_tmp,
                const void* f, int64_t n, double* res_dev, void* work,
                size_t work_bytes, void* stream);

/* ---- convergence-controlled solve ----------------------------------------
 * Relative-residual Jacobi (or red-black Gauss-Seidel, method) solve of
 * L(u) = f with Dirichlet halo.
 * res0 = ||r(u^0)||, u^0 = u with its interior zeroed (same halo, same f);
 * the answer is u_K with K the smallest k >= 0 such that
 * ||r(u_k)|| / res0 <= rel_tol (K = 0 if res0 = 0).
 *
 * precision MS_SOLVE_F64: plain FP64 sweeps, max_sweeps caps K.
 * precision MS_SOLVE_F32_REFINED: FP64 iterative refinement around FP32
 *   sweeps. Outer: r = f - L(x) in FP64; stop if rel = ||r||/res0 <= rel_tol;
 *   s = 2^floor(log2(||r|| / sqrt(N))); rhat = fl32(r / s); inner FP32 Jacobi
 *   on L(e) = rhat from e = 0 (zero halo) until its FP64 residual drops to
 *   max(inner_eta, rel_tol / (2 rel)) times its start, or stalls (no
 *   decrease over stall_window sweeps), or max_inner sweeps; then
 *   x += s * e in FP64. max_outer caps the outer steps, max_sweeps the total
 *   inner sweeps.
 * check_every: sweeps per device-side chunk between host checks (0 = auto).
 * temporal_block: sweeps fused per pass over memory: 0 or 1 = one,
 *   2 = two (as jacobi_sweeps_tb; same iterates, same K; the default).
 * use_graph: 1 = replay chunks as hipGraphs (default), 0 = plain launches.
 * method: MS_METHOD_JACOBI (default) or MS_METHOD_RBGS, red-black
 *   Gauss-Seidel sweeps as rbgs_sweeps (for the FP32 inner iteration too;
 *   temporal_block is then ignored). K counts Gauss-Seidel sweeps.
 *
 * u: device, in: initial guess + Dirichlet halo; out: the answer u_K.
 * f: device, may be NULL. hist_host: host, may be NULL; receives
 * ||r(u_k)|| for k = 0..K (MS_SOLVE_F64, needs max_sweeps + 1 doubles) or
 * ||r(x_o)|| / res0 per outer step o = 0..outer_iters (refined, needs
 * max_outer + 1 doubles). Blocks until done.
 * Returns MS_OK, MS_NOT_CONVERGED (result still filled), MS_ENONFINITE,
 * or an error. */
#define MS_SOLVE_F64 0
#define MS_SOLVE_F32_REFINED 1
#define MS_METHOD_JACOBI 0
#define MS_METHOD_RBGS 1

typedef struct {
  double rel_tol;
  int64_t max_sweeps;
  int32_t precision;
  int32_t check_every;
  double inner_eta;
  int32_t max_outer;
  int32_t max_inner;
  int32_t stall_window;
  int32_t temporal_block;
  int32_t use_graph;
  int32_t method;
} ms_solve_opts;

typedef struct {
  int64_t sweeps;      /* K (F64) or the total inner sweeps (refined) */
  int32_t outer_iters; /* refinement steps taken (0 for F64) */
  int32_t status;      /* same as the return value */
  double res0;         /* ||r(u^0)|| */
  double res_final;    /* ||r(u_K)|| (FP64, recomputed for refined) */
  double rel_final;    /* res_final / res0 */
  double seconds;      /* jacobi_solve: host wall time of the call; batched:
                          device real-time clock from the earliest team start
                          of the launch to this instance's team finish */
} ms_solve_result;

/* Fill `o` with the library defaults (rel_tol 1e-8, F64, auto chunks, two
 * sweeps per pass, graphs on, inner_eta 1e-5, max_outer 20, stall 256). */
void ms_solve_opts_default(ms_solve_opts* o);
size_t jacobi_workspace_bytes(const ms_grid* g, const ms_solve_opts* o);
int jacobi_solve(const ms_grid* g, const ms_solve_opts* o, double* u,
                 const double* f, void* work, size_t work_bytes,
                 double* hist_host, ms_solve_result* res, void* stream);

/* ---- autotuning of the sweep tile shape ------------------------------------
 * The sweeps of jacobi_sweeps / jacobi_solve run z-marching wave tiles whose
 * shape -- x cells per lane (vec), waves across x (wx), rows per lane
 * (rows) and the number of blocks the z split aims at -- changes the
 * bandwidth they reach. ms_autotune_sweeps times every candidate shape on
 * the caller's buffers (u and u_tmp are overwritten: pass scratch fields
 * laid out like the real ones), keeps the fastest in a process-wide table
 * keyed by (dtype, nx, ny, nz, vector alignment of the buffers) and returns
 * it; later sweeps on a matching grid use it. Every shape gives the same
 * bits. ms_tuning_get / ms_tuning_set export and import the table (for a
 * cache file); ms_tuning_clear empties it. */
typedef struct {
  int32_t dtype, nx, ny, nz, vec_ok;
  int32_t vec, wx, rows;
  int64_t target_blocks;
  double us_per_sweep; /* measured time of the chosen shape */
} ms_tuning;

int ms_autotune_sweeps(const ms_grid* g, int dtype, void* u, void* u_tmp, const void* f,
                       int sweeps_per_trial, void* work, size_t work_bytes,
                       ms_tuning* best, void* stream);
/* Copies up to cap entries into out; returns the number of entries. */
/* The sweep shape jacobi_sweeps / jacobi_solve would use for a grid of this
 * dtype whose buffers are `bufs` (host-side query, no device work): vec_ok
 * is the vector width the buffers' alignment allows, vec / wx / rows the
 * shape, target_blocks the block count of one sweep launch, us_per_sweep
 * the tuned time if the shape came from the tuning table, else 0. */
int ms_sweep_shape(const ms_grid* g, int dtype, const void* const* bufs, int nbufs,
                   ms_tuning* out);
int ms_tuning_get(ms_tuning* out, int cap);
int ms_tuning_set(const ms_tuning* in, int n);
void ms_tuning_clear(void);

/* ---- batched solves ---------------------------------------------------------
 * Many independent instances of jacobi_solve, each with its own grid,
 * solved in ONE persistent kernel launch (captured in a hipGraph). The
 * device's resident blocks are split into teams, and each team runs a
 * chain of instances one after the other (a large instance alone, small
 * ones several in turn), so that the longest estimated chain time is as
 * short as possible (an instance's estimate: cells x Jacobi sweeps to
 * rel_tol, from the spectral radius and the reference residual's component
 * along the slowest mode (one device pass before planning; see
 * jacobi_batched_plan), split over the team, plus a per-sweep barrier cost
 * for teams of more than one block); a team runs each instance's whole
 * solve with team barriers and never waits for another team. Any number of
 * instances (n >= 1). precision: MS_SOLVE_F64 or
 * MS_SOLVE_F32_REFINED with the refinement rules of jacobi_solve (same
 * per-cell arithmetic, same stopping rules; norms are summed per team, so an
 * iteration count may differ from jacobi_solve's by one only when a norm
 * sits within rounding of its threshold). method must be MS_METHOD_JACOBI
 * (else MS_EUNSUPPORTED). Options used: rel_tol,
 * max_sweeps, precision, inner_eta, max_outer, max_inner, stall_window
 * (<= 1024). Instances must not overlap.
 * res: host array of n results. Blocks until done. Returns MS_OK,
 * MS_NOT_CONVERGED or MS_ENONFINITE (worst over instances), or an error;
 * MS_EHIP if a team barrier exceeds its time limit (20 s). */
typedef struct {
  ms_grid grid;
  double* x;       /* device: initial guess + Dirichlet halo; the answer on return */
  const double* f; /* device right-hand side, may be NULL */
} ms_instance;

size_t jacobi_batched_workspace_bytes(int n, const ms_instance* inst,
                                      const ms_solve_opts* o);
int jacobi_solve_batched(int n, const ms_instance* inst, const ms_solve_opts* o,
                         void* work, size_t work_bytes, ms_solve_result* res,
                         void* stream);
/* The plan the batched solve would use; any output may be NULL. team_sizes
 * (n ints): the size of the team that runs each instance; groups (n ints):
 * the index of that team (instances of one team run one after the other,
 * in increasing order of their position in the team's chain, longest
 * estimate first); grid_blocks: the blocks of the launch (the sum of the
 * team sizes over distinct teams); est_sweeps (n doubles): the
 * per-instance sweep estimates.
 * The estimates come from one device pass over the instances (the same
 * probe the solve runs): ||r(u^0)|| and the component c1 of r(u^0) along
 * the slowest Jacobi mode give about ln(tol ||r(u^0)|| / c1) / ln(rho)
 * sweeps, kept within [1/10, 1] of ln(tol) / ln(rho). They depend on f and
 * the halo of x, not on its interior. work: device, at least
 * jacobi_batched_plan_workspace_bytes(n) bytes. Synchronises `stream`. */
size_t jacobi_batched_plan_workspace_bytes(int n);
int jacobi_batched_plan(int n, const ms_instance* inst, const ms_solve_opts* o,
                        int* team_sizes, int* groups, int* grid_blocks, double* est_sweeps,
                        void* work, size_t work_bytes, void* stream);

/* The planner alone, on the host (no device work): teams and chains for n
 * grids with the given sweep estimates (each finite, >= 1) on `blocks`
 * resident blocks, for `precision` (MS_SOLVE_F64 or MS_SOLVE_F32_REFINED),
 * with the outputs of jacobi_batched_plan. Estimated time of an instance of
 * extents nx x ny x nz and S sweeps on a team of t blocks: with one sweep
 * per team barrier (MS_SOLVE_F64, or MS_BATCH_TB=1), C S / t for C cells,
 * plus 8192 S when t > 1; with two sweeps per barrier (MS_SOLVE_F32_REFINED
 * by default), S / 2 x (R x (nz / p + 2) + 15 [t > 1]), where p in {1, 2, 4,
 * 8, 16} (at most nz; the fewest on a tie) minimises R x (nz / p + 2) and R
 * = ceil(ceil(nx / 60) ceil(ny / 4) p / (16 t)) is the number of rounds in
 * which the team's 16 t waves take the 60 x 4 x nz / p tiles. For a target
 * makespan M each instance takes the
 * smallest team (at most min(blocks, 8 x its 64 x 16 tiles)) whose time is
 * at most M; instances wanting the same team size go into chains of total
 * time at most M (longest first, first chain with room); the smallest M
 * that fits is found by bisection from the makespan of one team per
 * instance (or, with more instances than blocks, of one block running them
 * all), and left-over blocks then go to the longest chain that some of
 * them shorten, the fewest blocks that do, until none does. */
int jacobi_batched_plan_from_estimates(int n, const ms_grid* grids, const double* est_sweeps,
                                       int blocks, int precision, int* team_sizes,
                                       int* groups, int* grid_blocks);

/* ---- batched solves on concurrent streams -----------------------------------
 * The same batch as jacobi_solve_batched, run instead by `workers` (1..64)
 * host threads, each with its own HIP stream (created and destroyed by the
 * call, default priority) and its own slice of the workspace. The threads
 * take the instances in order of estimated work (cells x the planner's
 * sweep estimate, largest first) and solve each exactly as jacobi_solve
 * does with `o` (any precision, temporal_block and method), so instances
 * overlap on the device and every result equals jacobi_solve's (fields bit
 * for bit). res[i] as jacobi_solve's result. work: device, at least
 * jacobi_batched_streams_workspace_bytes(n, inst, o, workers) bytes (the
 * probe area plus workers x the largest single-instance workspace).
 * Synchronises `stream` before it starts (its one device pass runs there)
 * and blocks until every instance is done. Returns MS_OK, MS_NOT_CONVERGED
 * or MS_ENONFINITE (worst over instances), or the first other error with
 * its instance. Instances' x must not overlap. */
size_t jacobi_batched_streams_workspace_bytes(int n, const ms_instance* inst,
                                              const ms_solve_opts* o, int workers);
int jacobi_solve_batched_streams(int n, const ms_instance* inst, const ms_solve_opts* o,
                                 int workers, void* work, size_t work_bytes,
                                 ms_solve_result* res, void* stream);

/* ---- autotuning of the batched tile shapes ----------------------------------
 * A team walks its instance in tiles of tx x-cells (one row of tx lanes;
 * a 64-lane wave covers 64/tx rows, a block four times that) and splits
 * each tile column into zsplit chunks along z. Candidates: tx in {64, 32,
 * 16} x zsplit in {1, 2, 4, 8}. The shape moves work between lanes and
 * blocks only: fields are the same for every shape; the norms' summation
 * order changes with it (see the batched solve on iteration counts).
 *
 * jacobi_batched_autotune times every candidate on this batch: one launch
 * per candidate with the solve's team plan, each team running
 * sweeps_per_trial sweeps of its instance (precision o->precision, with the
 * per-sweep norm and team barrier) on workspace buffers, all teams at once.
 * Each instance's fastest shape goes into a process-wide table keyed by
 * (precision, nx, ny, nz, team size) that jacobi_solve_batched consults
 * (untuned default: tx 64 and the fewest z chunks that give every block of
 * the team a tile). The instances' x are not read or written; f
 * is read in FP64 trials. best: host array of n entries or NULL. Blocks
 * until done. Workspace from jacobi_batched_autotune_workspace_bytes.
 * ms_batch_tuning_get copies up to cap entries and returns the count;
 * ms_batch_tuning_set validates and inserts (MS_EINVAL on a bad entry, none
 * inserted); ms_batch_tuning_clear empties the table. */
typedef struct {
  int32_t precision, nx, ny, nz, team, tx, zsplit, reserved;
  double us_per_sweep; /* measured under the batch's contention */
} ms_batch_tuning;

size_t jacobi_batched_autotune_workspace_bytes(int n, const ms_instance* inst,
                                               const ms_solve_opts* o);
int jacobi_batched_autotune(int n, const ms_instance* inst, const ms_solve_opts* o,
                            int sweeps_per_trial, void* work, size_t work_bytes,
                            ms_batch_tuning* best, void* stream);
int ms_batch_tuning_get(ms_batch_tuning* out, int cap);
int ms_batch_tuning_set(const ms_batch_tuning* in, int n);
void ms_batch_tuning_clear(void);

/* ---- advection source term ------------------------------------------------
 * The fused three-field Piacsek-Williams advection source term of Section
 * 4.1 (three stencils over u, v, w fused into one pass, 63 flops per cell).
 * The paper prints no formula; this library's definition on a staggered
 * C-grid (u at i+1/2, v at j+1/2, w at k+1/2), for phi in (u, v, w):
 *   s_phi = (tcx*(Px- - Px+) + tcy*(Py- - Py+)) + (tzc1[k]*Pz- - tzc2[k]*Pz+)
 * where each P is phi at the neighbour on that side times the sum of the
 * two samples of the advecting velocity straddling that face, e.g. for su:
 *   Px- = u[i-1]*(u[i-1]+u[i])          Px+ = u[i+1]*(u[i]+u[i+1])
 *   Py- = u[j-1]*(v[j-1]+v[i+1,j-1])    Py+ = u[j+1]*(v[j]+v[i+1,j])
 *   Pz- = u[k-1]*(w[k-1]+w[i+1,k-1])    Pz+ = u[k+1]*(w[k]+w[i+1,k])
 * (sv, sw likewise with the roles of the axes exchanged). FP64, evaluation
 * order as written, no contraction.
 * u, v, w: device fields on grid g with a valid halo (edges and corners
 * included); tzc1, tzc2: device arrays of nz doubles; su, sv, sw: device
 * outputs on grid g (interior written). Outputs may not alias inputs.
 * Async. */
int advect_source(const ms_grid* g, const double* u, const double* v,
                  const double* w, const double* tzc1, const double* tzc2,
                  double tcx, double tcy, double* su, double* sv, double* sw,
                  void* stream);

/* ---- learned warm start: 3x3x3 convolutions on BF16 MFMA ----------------
 * Not in the paper: a small 3D CNN (8 -> 32 -> 32 -> 32 -> 1 channels,
 * ReLU after the first three layers) maps features of the right-hand side
 * f and the boundary lift g (scaled by s = max(max|f|, max|g|); see
 * cnn_features) to u / (s * lambda), an initial guess for jacobi_solve.
 * These entry points are its training and inference kernels.
 *
 * Activations: BF16, channels-last over an X x Y x Z volume with a
 * one-voxel zero halo (the "same" zero padding of the convolution): element
 * (x, y, z, c) at ((((z+1)*(Y+2) + (y+1))*(X+2) + (x+1))*C + c); C = cin
 * (8 or 32) for inputs, 32 for outputs (channels beyond the real count are
 * zero). The caller allocates them zero-filled; kernels write the interior.
 * Weights: BF16 [27][32][cin] (forward) and [27][cin][32] (input gradient),
 * tap t = (dx+1) + 3(dy+1) + 9(dz+1); FP32 master copies [27][32][cin] and
 * biases [32]. Products in BF16, sums in FP32. All pointers are device
 * pointers; all calls are async on `stream`. */

/* out[v][co] = act(bias[co] + sum_{t,ci} w[t][co][ci] in[v + d_t][ci]);
 * act = ReLU if relu, else identity. out (BF16, C = 32) and/or out32 (FP32
 * channel 0 in the field layout (X+2)(Y+2)(Z+2), sy = X+2) may be NULL. */
int conv3d_bf16_fwd(int X, int Y, int Z, int cin, const void* in, const void* w,
                    const float* bias, void* out, float* out32, int relu,
                    void* stream);
/* din[v][ci] = [mask[v][ci] > 0] * sum_{t,co} wd[t][ci][co] dout[v - d_t][co]
 * (mask = the layer input, i.e. the previous layer's ReLU output; NULL for
 * no mask). */
int conv3d_bf16_dgrad(int X, int Y, int Z, int cin, const void* dout, const void* wd,
                      const void* mask, void* din, void* stream);
/* dw[t][co][ci] = sum_v dpre[v][co] in[v + d_t][ci], db[co] = sum_v dpre[v][co]
 * over interior voxels v (FP32, deterministic two-pass reduction through
 * `work`). The halo of dpre is not read; that of `in` must be zero. */
size_t conv3d_bf16_wgrad_workspace_bytes(int cin);
int conv3d_bf16_wgrad(int X, int Y, int Z, int cin, const void* in, const void* dpre,
                      float* dw, float* db, void* work, size_t work_bytes, void* stream);
/* loss_part[b] = partial sums of (pred - target)^2 over interior voxels
 * (nparts blocks); dpre channel 0 = BF16(2 (pred - target) / N). pred and
 * target: FP32 in the field layout. dpre channels 1..31 are left as they are
 * (zero). */
int cnn_mse_grad(int X, int Y, int Z, const float* pred, const float* target, void* dpre,
                 double* loss_part, int nparts, void* stream);
/* One Adam step (beta 0.9, 0.999, eps 1e-8, step t >= 1) on FP32 master
 * weights w and biases b, then BF16 copies in both layouts. */
int cnn_adam(int cin, float* w, float* b, float* mw, float* vw, float* mb, float* vb,
             const float* gw, const float* gb, void* wf, void* wd, float lr, int t,
             void* stream);
/* BF16 copies of FP32 master weights in both layouts. */
int cnn_pack_weights(int cin, const float* w, void* wf, void* wd, void* stream);
/* Network input (BF16, C = 8) of the Poisson problem (u: halo = Dirichlet
 * values, f may be NULL) and *scale = s (device). Channels: 0 f/s, 1 g/s,
 * 2..5 the means of f/s over cubes of side 5, 11, 23, 47 around the cell
 * (zero outside the interior; sums along x, then y, then z, each over
 * increasing offsets, then one division by the cube's volume), 6 the
 * slowest Jacobi mode prod_a sin(pi (i_a+1)/(n_a+1)), 7 the mean over cubes
 * of side 95. work: cnn_features_workspace_bytes(g) bytes. */
size_t cnn_features_workspace_bytes(const ms_grid* g);
int cnn_features(const ms_grid* g, const double* u, const double* f, void* feat,
                 double* scale, void* work, size_t work_bytes, void* stream);
/* x interior = (*scale) * lambda * uhat (FP64); the halo is not touched. */
int cnn_guess(const ms_grid* g, const float* uhat, const double* scale, double lambda,
              double* x, void* stream);
/* out (FP32, field layout of the volume) = u / ((*scale) * lambda) on the
 * interior: training targets from solved fields. */
int cnn_target(const ms_grid* g, const double* u, const double* scale, double lambda,
               float* out, void* stream);

/* ---- learned warm start, whole path --------------------------------------
 * The network above behind two calls: an initial guess for jacobi_solve
 * (warmstart_forward) and one training step on a solved instance
 * (warmstart_train_step). Every arithmetic step runs on the device.
 *
 * Parameters: one caller-owned device buffer of warmstart_params_bytes()
 * bytes, three blocks of warmstart_params_floats() floats: the FP32 master
 * parameters, then Adam's first and second moments in the same layout
 * (zero before the first training step). Master layout: layer l = 0..3
 * starts at float warmstart_layer_offset(l) and holds its weights
 * [27][32][cin_l] (cin = 8, 32, 32, 32; tap t = (dx+1) + 3(dy+1) + 9(dz+1);
 * input channels beyond the real 2 of layer 0 and output channels beyond the
 * real 1 of layer 3 are zero) followed by its 32 biases.
 * The guess is x = s * out_scale * u_hat with s = max(max|f|, max|g|) of the
 * features; out_scale is a property of the trained parameters (the trainer
 * stores it beside them).
 *
 * work: device workspace of warmstart_workspace_bytes(g, train) bytes (train
 * = 0 for warmstart_forward, 1 for warmstart_train_step); activations in it
 * are rewritten on every call. */
#define MS_START_RESIDUAL 0   /* keep the guess iff ||r(x)|| < ||r(u0)|| */
#define MS_START_SLOW_MODES 1 /* keep it iff its slowest components are smaller */
#define MS_START_FORCE 2      /* always keep the guess */
size_t warmstart_params_floats(void);
size_t warmstart_params_bytes(void);
size_t warmstart_layer_offset(int layer);
size_t warmstart_workspace_bytes(const ms_grid* g, int train);

/* Initial guess for L(x) = f with the Dirichlet halo of u (u's interior is
 * not read). Writes the guess into x's interior (x: grid g, FP64; its halo
 * must hold the same Dirichlet values as u's; x may be u, must not overlap
 * f), applies `smooth` damped Jacobi sweeps to it (even, 0 .. 64:
 * x <- x + (2/3) (J(x) - x), J(x) = (S(x) - f) * fl(1/6) the plain sweep's
 * update, FP64, in this order), then chooses the start: with u0 = u with
 * its interior zeroed,
 *   MS_START_RESIDUAL:   keep the guess iff ||r(x)|| < ||r(u0)||;
 *   MS_START_SLOW_MODES: keep it iff the projection of r(x) on the two
 *     slowest-decaying eigenvectors of the Jacobi iteration (phi = the
 *     product of sin(pi (i+1)/(n+1)) over the axes, eigenvalue rho; psi =
 *     (-1)^(i+j+k) phi, eigenvalue -rho) is shorter than that of r(u0)
 *     (these two set the sweep count at tight tolerances);
 *   MS_START_FORCE:      always keep it;
 * and zeroes x's interior again when u0 wins (x is then u0 exactly). All
 * measures in FP64, r = f - (S - 6x). used (device int, may be NULL): 1 if
 * the guess was kept. measures (device, 4 doubles, may be NULL):
 * ||r(x)||, ||r(u0)||, slow(r(x)), slow(r(u0)). f may be NULL. Async. */
int warmstart_forward(const ms_grid* g, const double* u, const double* f,
                      const float* params, double out_scale, int smooth, int rule,
                      double* x, void* work, size_t work_bytes, int* used,
                      double* measures, void* stream);

/* One training step on a solved instance: forward pass on (u's halo, f),
 * target u_solved / (s * out_scale) in FP32 (u_solved: the solved field on
 * grid g), MSE loss mean over the interior voxels, gradients of every
 * layer, then one Adam step (beta 0.9 / 0.999, eps 1e-8, learning rate lr,
 * 1-based step count `step`) on params (master and moments updated in
 * place). loss (device double, may be NULL) receives the loss before the
 * update, reduced in a fixed order. Async. */
int warmstart_train_step(const ms_grid* g, const double* u, const double* f,
                         const double* u_solved, float* params, double out_scale,
                         float lr, int step, void* work, size_t work_bytes,
                         double* loss, void* stream);

/* ---- bandwidth probe ------------------------------------------------------
 * Not a stencil: out[i] = a[i] + b[i] (b non-NULL: two reads, one write) or
 * out[i] = a[i] (b NULL: one read, one write) over n doubles (n even; all
 * arrays 16-byte aligned device memory; out must not overlap a or b), in
 * 16-byte lanes with nontemporal stores, on `blocks` blocks of 256 threads,
 * form 0: grid-stride, one element per lane per stride; 1: four strides of
 * loads issued before their stores; 2: as 1 with nontemporal loads; 3: each
 * block streams its own contiguous share, two 4 KiB steps in flight.
 * Measures the achievable HBM bandwidth of the stencils' access patterns.
 * Async. */
int ms_stream_probe(const double* a, const double* b, double* out, int64_t n,
                    int blocks, int form, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* MISTENCIL_H */
