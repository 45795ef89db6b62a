/*
 * lem.h -- C ABI of the MI355X (gfx950) Local Exponential Method library.
 *
 * The Local Exponential Method (L. Bonaventura, "Local Exponential Methods: a
 * domain decomposition approach to exponential time integration of PDEs",
 * section 3) advances the semi-discrete linear system du/dt = A u (eq. (3)
 * with zero forcing, periodic boundaries) by one step dt as follows: the grid
 * is covered by regions M_i = D_i u B_i (disjoint cores D_i plus buffers B_i);
 * on each region the local problem (4) -- A restricted to M_i with the
 * couplings to outside nodes removed (homogeneous Dirichlet data) -- is
 * advanced by the exponential update (5), which for zero forcing is
 * v <- exp(dt A_{M_i}) v; the core rows of every local result overwrite the
 * global state (step 3).  The operator is the centered finite-difference
 * advection-diffusion operator of the paper's model problem (eq. (2); 1D as
 * in section 4.1, 2D conservative form as in section 4.3).
 *
 * Conventions shared by every call:
 *  - Status: every call returns a lem_status; on anything but LEM_OK a
 *    message is available from lem_last_error() (thread-local).
 *  - Streams: `stream` is a hipStream_t passed as void* (NULL = the legacy
 *    default stream).  Device work is enqueued asynchronously on it; argument
 *    validation happens synchronously before anything is enqueued.
 *  - State layout: a state array holds N = n^ndim grid values for each of
 *    n_states ensemble members, DOF-major with the ensemble index fastest:
 *    x[(j*n + i) * n_states + s] for grid point (i, j) (x fastest), float64,
 *    in DEVICE memory owned by the caller.
 *  - Ownership: a plan owns every buffer it allocates (index maps, local
 *    exponential blocks, coefficients, work space) and frees them in
 *    lem_plan_destroy.  Host arrays passed in are copied during the call.
 *  - Device-side failures (Krylov estimate above tolerance, non-finite
 *    values) are latched in the plan's status word; they are reported by
 *    lem_plan_query (field device_status: LEM_ERR_NOT_CONVERGED or
 *    LEM_ERR_NONFINITE, the latter taking precedence) after the stream has
 *    drained.  The word stays latched for the life of the plan.
 *  - A plan is not thread-safe: do not call lem_step on one plan from two
 *    threads at once, nor enqueue two steps of one plan on different streams.
 */
#ifndef LEM_H
#define LEM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  LEM_OK = 0,
  LEM_ERR_INVALID = 1,        /* bad argument (sizes, aliasing, NULL)         */
  LEM_ERR_NOMEM = 2,          /* device or host allocation failed            */
  LEM_ERR_HIP = 3,            /* a HIP runtime call failed                    */
  LEM_ERR_NOT_CONVERGED = 4,  /* Krylov estimate above tolerance              */
  LEM_ERR_BUDGET = 5,         /* request does not fit the memory budget       */
  LEM_ERR_UNSUPPORTED = 6,    /* valid but not implemented combination        */
  LEM_ERR_NOT_FOUND = 7,      /* unknown request id                           */
  LEM_ERR_NONFINITE = 8       /* a step produced non-finite values (NaN/Inf)  */
} lem_status;

/* Algorithm for the stored local exponentials (dense method, plan time). */
enum {
  LEM_EXPM_PADE = 0,   /* scaling and squaring with the Pade [13/13] approximant
                          (sections 3 and 4), denominator solved by pivoted LU */
  LEM_EXPM_TAYLOR = 1  /* scaling and squaring with the degree-18 Taylor
                          polynomial in Paterson-Stockmeyer form: GEMMs only
                          (faster plans for many distinct blocks)          */
};

/* Method used for the local exponential actions. */
enum {
  LEM_METHOD_KRYLOV = 0,  /* Arnoldi-Krylov action per block (section 4.3)     */
  LEM_METHOD_DENSE = 1,   /* stored local exponentials by Pade scaling and
                             squaring, applied as matrix products (sections 3
                             and 4: "computed only at the first time step")  */
  LEM_METHOD_GLOBAL = 2,  /* no decomposition (D = 1): global Krylov action  */
  LEM_METHOD_ROSENBROCK = 3, /* exponential Rosenbrock-Euler for Burgers; plans
                               come from lem_ere_plan only                    */
  LEM_METHOD_KRONECKER = 4  /* stored local exponentials of a 2D constant-
                               coefficient operator in Kronecker-factored form:
                               on a rectangular box the local matrix is the
                               Kronecker sum of two 1D tridiagonal matrices,
                               so exp(dt A_M) = exp(dt A_y) (x) exp(dt A_x)
                               exactly and a block's core is
                               E_y[core,:] X E_x[core,:]^T for the box values
                               X; the two 1D exponentials are computed once
                               (opt.expm) -- uniform core <= 64, box side
                               core + 2 halo <= 128, FP64, no forcing       */
};

/* Arithmetic used to apply stored local exponentials (dense method only). */
enum {
  LEM_FP64 = 0,     /* float64 throughout                                    */
  LEM_FP32 = 1,     /* float32 products, float32 accumulation                */
  LEM_BF16X2 = 2,   /* bf16 hi/lo split of both operands, 3 products,
                       float32 accumulation (one correction of the bf16
                       product)                                              */
  LEM_BF16X3 = 3    /* bf16 hi/mid/lo split, 6 products, float32 accumulation */
};

/* The semi-discrete operator: the periodic advection-diffusion operator of
 * eq. (2), centered finite differences on n (1D) or n x n (2D) points with
 * spacing dx.  With constant nu the 1D row of dt*A is
 *   (mu + C/2) u_{i-1} - 2 mu u_i + (mu - C/2) u_{i+1},
 * C = vel*dt/dx, mu = nu*dt/dx^2, and 2D adds the same along y.  When
 * nu_field is given (HOST pointer to N values, [j][i], copied by lem_plan)
 * the diffusion is in conservative flux form with arithmetic face means
 * mu_{i+1/2} = dt (nu_i + nu_{i+1}) / (2 dx^2). */
typedef struct {
  int32_t ndim;            /* 1 or 2                                          */
  int32_t n;               /* points per axis, >= 3                           */
  double dx;               /* grid spacing, > 0                               */
  double vel[2];           /* constant velocity (vel[1] ignored in 1D)        */
  double nu;               /* constant diffusivity >= 0 (if nu_field == NULL) */
  const double* nu_field;  /* optional per-node diffusivity, host, or NULL    */
  const double* forcing;   /* optional source g of du/dt = A u + g, constant in
                              time (rate units): host, N x n_states with the
                              state index fastest, copied at plan time; NULL
                              for g = 0.  A step is then the exponential-Euler
                              update (5) of section 3 with g_M, i.e.
                              exp(dt A_M) v + phi_1(dt A_M)(dt g_M), and the
                              global method takes exp(dt A) u + phi_1(dt A)(dt g).
                              Not accepted by the server (LEM_ERR_UNSUPPORTED). */
  const double* vel_faces; /* optional face velocities replacing vel (which must
                              then be zero): host, ndim x N doubles, a_x on the
                              east face (i+1/2, j) of node j*n + i, then (2D)
                              a_y on its north face (i, j+1/2); the advection
                              is taken in the conservative form -div(a c) of
                              eq. ibv2d (section 4.3) with centered face
                              fluxes.  Krylov and global methods only (the
                              dense method and the server reject it).       */
  double dy;               /* y spacing of an anisotropic 2D mesh (section
                              4.3); 0 means dy = dx                         */
} lem_operator;

typedef struct {
  int32_t method;        /* LEM_METHOD_*                                     */
  int32_t precision;     /* LEM_FP64 / LEM_FP32 / LEM_BF16X2 / LEM_BF16X3    */
  int32_t n_states;      /* ensemble members per state array, >= 1          */
  int32_t core;          /* core side c (must divide n); 0 = uneven cores
                            chosen per 64x64 tile (Krylov, 2D only)          */
  int32_t halo;          /* buffer width h per side; 0 = decay bound        */
  int32_t halo_min;      /* clamp range for the decay-bound halo            */
  int32_t halo_max;
  double halo_tol;       /* per-step relative bound the halo must meet      */
  int32_t krylov_m;      /* Krylov dimension; 0 = calibrate per block       */
  int32_t krylov_m_max;  /* largest dimension allowed: <= 40 for local
                            actions, <= 48 for LEM_METHOD_GLOBAL            */
  int32_t max_substeps;  /* largest number of equal sub-steps per step      */
  double krylov_tol;     /* relative tolerance of the Krylov estimate       */
  int32_t use_graph;     /* capture lem_step's launches in a HIP graph      */
  int32_t autotune;      /* time candidate launch shapes at plan time       */
  int32_t dry_run;       /* 1: build partition and maps on the host only;
                            no device memory is touched (lem_step fails)     */
  int32_t expm;          /* LEM_EXPM_PADE (default) or LEM_EXPM_TAYLOR      */
  int32_t columns;       /* 2D Krylov: column-wise decomposition (section
                            4.3): cores of core x n points spanning whole
                            columns, buffers of halo points across the
                            columns only, the periodic coupling along the
                            columns kept inside every box; exported boxes
                            then read (ox, 0, core, n, h)                   */
  int32_t core_max;      /* uneven cores (core = 0): largest core side tried
                            per 64x64 tile, 16, 32 or 64 (0 = 64).  With
                            autotune set, the planner builds the partitions
                            with core_max 32 and 64, each with the Krylov
                            dimension capped at 30 and at krylov_m_max,
                            times a step of each on a probe state and keeps
                            the fastest                                     */
  int32_t tile;          /* dense method, n_states % 64 == 0: launch shape of
                            the apply; -1 = the default shape (or the
                            fastest one when autotune is set), 0..7 = that
                            shape for FP64/FP32 (rows per wave, K chunk,
                            waves: 32,16,4 / 32,32,4 / 32,32,8 / 64,32,4 /
                            16,32,8 / 16,32,4 / 16,16,8 / 16,32,16), 0..4
                            for split bf16 (rows per wave, waves, states
                            per workgroup: 32,4,64 / 64,4,64 / 32,8,64 /
                            64,8,64 / 32,8,128, the last for n_states %
                            128 == 0); a shape
                            that does not fit the block is LEM_ERR_UNSUPPORTED
                            at plan time                                    */
} lem_options;

typedef struct {
  int32_t n_blocks;        /* number of regions M_i                           */
  int32_t n_unique;        /* distinct local operators (dense method)         */
  int64_t n_loc_total;     /* sum of local box sizes |M_i|                    */
  int32_t n_loc_max;
  int32_t halo_min, halo_max;  /* range of buffer widths used                */
  int32_t halo_clamped;    /* blocks whose decay-bound halo hit halo_max      */
  int32_t m_min, m_max;    /* Krylov dimensions used                          */
  int32_t substeps_max;
  int32_t squarings;       /* Pade squarings of the largest dense block; for
                              Rosenbrock boxes of <= 80 points, the most
                              phi_1 doublings at the last refresh           */
  int64_t bytes_blocks;    /* device bytes of stored local exponentials       */
  int64_t bytes_work;      /* device bytes of work space                      */
  int32_t device_status;   /* latched device-side lem_status (0 = fine)       */
  double max_estimate;     /* largest Krylov error estimate seen (relative)   */
  double plan_ms;          /* wall time of lem_plan                           */
  int32_t tile_config;     /* launch shape chosen (autotuner id)              */
  double krylov_bytes_step;     /* Krylov methods: algorithmic basis traffic of
                                   one step, sum over blocks and members of
                                   |M_i| * 8 * (m (m + 1) + 3 m) * sub-steps
                                   bytes (each basis row read twice per
                                   Arnoldi column, classical Gram-Schmidt) */
  double krylov_bytes_streamed; /* the part of it on blocks whose basis is
                                   streamed through device memory (the rest
                                   stays in LDS)                           */
  int32_t resident_steps;  /* 1: lem_step runs all steps of a call in one
                              launch (1D dense FP64 plans with one stored
                              block, cores tiling the grid, core of 4 to
                              128 and box <= 128 points, two states per
                              workgroup in LDS)                             */
} lem_plan_info;

typedef struct lem_plan_s* lem_plan_t;

/* Fill *opt with defaults: Krylov, FP64, one state, core 64 (1D) / 32 (2D),
 * decay-bound halo in [4, 64] at tol 1e-8, calibrated m <= 30 at tol 1e-13,
 * up to 64 sub-steps, no graph, no autotune, default apply shape (tile -1). */
void lem_options_default(lem_options* opt);

/* Build a plan for steps of size dt of the operator *op (section 3).
 * Partitions the grid into cores with buffers (uniform core side, uneven
 * cores with per-block buffer widths from the off-diagonal decay bound of
 * section 2, or column-wise cores), builds index maps, and for the dense
 * method computes every distinct local exponential exp(dt A_{M_i}) once in
 * float64 on the device (opt->expm: Pade [13/13] scaling and squaring by
 * default; the paper computes these once, at the first step).  A constant-
 * coefficient operator has one block shared by all regions; a variable one
 * (nu_field or vel_faces) one block per region, every box then taking the
 * partition's largest buffer width (uniform core, FP64 or FP32, no forcing).
 * For the Krylov methods, calibrates the Krylov dimension per block on a
 * pseudo-random probe.  Blocks until the plan is ready.
 * Errors: LEM_ERR_INVALID for a bad operator/options (c must divide n, a box
 * c + 2h must be < n unless it spans the whole axis), LEM_ERR_UNSUPPORTED for
 * combinations not built (column-wise dense, bf16 with variable coefficients,
 * Krylov boxes above 9216 points -- 9215 with a forcing --, ...),
 * LEM_ERR_NOMEM, LEM_ERR_HIP, LEM_ERR_NOT_CONVERGED when no (m, sub-step)
 * pair within the limits meets krylov_tol. */
lem_status lem_plan(const lem_operator* op, double dt, const lem_options* opt,
                    void* stream, lem_plan_t* out);

/* Advance x_in by n_steps >= 1 LEM steps (local problems (4), updates (5),
 * core overwrite) and leave the result in x_out.  x_in and x_out are device
 * arrays of N * n_states doubles and must not overlap (buffers read
 * neighbouring cores); x_in is not modified.  Intermediate steps ping-pong
 * through a plan-owned buffer.  Asynchronous on `stream`. */
lem_status lem_step(lem_plan_t plan, const double* x_in, double* x_out,
                    int32_t n_steps, void* stream);

/* Viscous Burgers u_t = -(u^2/2)_x + nu u_xx on a periodic 1D grid of n >= 3
 * points (section 4.2), centered differences. */
typedef struct {
  int32_t n;
  double dx;   /* > 0 */
  double nu;   /* >= 0 */
} lem_burgers;

/* Plan exponential Rosenbrock-Euler LEM steps (sections 3 and 4):
 *   u^{n+1} = u^n + dt phi_1(dt J_M) F(u^n)_M on every region, core rows,
 * J_M the principal submatrix on the box of the Jacobian of F, frozen at the
 * state of the last refresh and refreshed every `refresh` >= 1 steps (the
 * first lem_step refreshes).  Cores of `core` points (dividing n) with
 * buffers of `halo` points per side; core = n with halo = 0 is the global
 * method (D = 1, periodic coupling kept).  A refresh computes phi_1(dt J_M)
 * of every (block, member) in float64 on the device: for boxes of at most 80
 * points in one launch (Taylor polynomial of degree 30 on dt J_M / 2^s, then
 * s doublings, asynchronous); for larger boxes from the exponentials of the
 * augmented matrices [[dt J_M, I], [0, 0]] by the GEMM-only Taylor pipeline
 * of LEM_EXPM_TAYLOR (synchronizes the stream); a step is
 * F on the grid and one contraction per core row.  lem_step, lem_plan_query,
 * lem_plan_copy_maps and lem_plan_destroy apply; no graphs, no serving.
 * Errors: LEM_ERR_INVALID (bad sizes), LEM_ERR_NOMEM, LEM_ERR_HIP. */
lem_status lem_ere_plan(const lem_burgers* op, double dt, int32_t n_states, int32_t core,
                        int32_t halo, int32_t refresh, void* stream, lem_plan_t* out);

/* 1D Schroedinger equation with a harmonic potential (section 4.1):
 *   c_t = (i/2) c_xx - i (kappa/2) x^2 c on n >= 3 points x_j = -L/2 + j L/n,
 * periodic, centered differences. */
typedef struct {
  int32_t n;
  double L;      /* > 0 */
  double kappa;  /* >= 0 */
} lem_schrodinger;

/* Plan LEM steps of the Schroedinger problem with stored complex local
 * exponentials exp(-i dt H_M) (sections 3 and 4.1), cores of `core` nodes
 * (dividing n) and `halo` buffer nodes per side; core = n with halo = 0 is
 * the global method (D = 1, periodic coupling kept).  The complex state is
 * carried in real form, interleaved per node: x[(2 j + c) * n_states + s] is
 * the real (c = 0) or imaginary (c = 1) part of member s at node j, float64,
 * device memory owned by the caller (2 n n_states doubles).  Every region has
 * its own block (the potential varies); the blocks are the exponentials of
 * the real forms dt [[0, H_M], [-H_M, 0]] by Pade [13/13] on the device, and
 * a step is the dense method's MFMA application on a grid of 2n real
 * unknowns (lem_plan_query reports that doubled geometry).  autotune != 0
 * times the apply tile shapes when n_states % 64 == 0.  lem_step,
 * lem_plan_query and lem_plan_destroy apply.  Errors: LEM_ERR_INVALID
 * (sizes, dt, L, kappa), LEM_ERR_UNSUPPORTED (boxes above 2048 nodes),
 * LEM_ERR_NOMEM, LEM_ERR_HIP. */
lem_status lem_schrodinger_plan(const lem_schrodinger* op, double dt, int32_t n_states,
                                int32_t core, int32_t halo, int32_t autotune, void* stream,
                                lem_plan_t* out);

/* y = exp(t A) x on the whole grid (no decomposition) by the Krylov method
 * of section 4.3, for n_states ensemble members (with op->forcing set:
 * y = exp(t A) x + phi_1(t A)(t g)); device arrays, may not overlap.
 * Allocates and frees its own work space (a plan with LEM_METHOD_GLOBAL
 * avoids that for repeated use).  Synchronous.  Returns
 * LEM_ERR_NOT_CONVERGED when the Krylov estimate stayed above tol and
 * LEM_ERR_NONFINITE when the result holds NaN or Inf (y is written either
 * way). */
lem_status lem_global_expmv(const lem_operator* op, double t, const double* x,
                            double* y, int32_t n_states, double tol,
                            int32_t m_max, void* stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * action as lem_global_expmv -- same arguments, calibration, kernels and
 * result -- with all of its device work space taken from a static per-device
 * scratch array of 64 MiB instead of hipMalloc/hipFree.  The caller still
 * passes x and y.  A problem whose work space could exceed the scratch
 * (roughly (m_max + 3) x N x n_states doubles plus per-point coefficients) is
 * refused with LEM_ERR_BUDGET before any device work.  Synchronous.  Calls on
 * one device share the array: calls that overlap in time on one device race
 * (serialize them); calls on different devices are independent. */
lem_status lem_global_expmv_static(const lem_operator* op, double t, const double* x,
                                   double* y, int32_t n_states, double tol, int32_t m_max,
                                   void* stream);

/* Plan statistics; device_status requires the plan's stream to have drained
 * (this call synchronizes the plan's last stream). */
lem_status lem_plan_query(lem_plan_t plan, lem_plan_info* info);

/* Copy the partition to HOST arrays (any may be NULL):
 *   boxes  [n_blocks][5] int32: core origin x, origin y, core size x,
 *          core size y, halo h (1D: origin y = 0, size y = 1);
 *   gather [n_loc_total] int32: per block in order, the global DOF of every
 *          local point (row-major, x fastest, wrapped periodically);
 *   scatter[N] int32: per block in order, the global DOF of every core row. */
lem_status lem_plan_copy_maps(lem_plan_t plan, int32_t* boxes, int32_t* gather,
                              int32_t* scatter);

/* Copy the per-block Krylov dimensions and sub-step counts (host arrays of
 * n_blocks int32 each; either may be NULL). */
lem_status lem_plan_copy_krylov(lem_plan_t plan, int32_t* m, int32_t* substeps);

/* Copy the core rows of stored local exponential `unique` (dense method) to a
 * host array of (core rows) x (local size) doubles, row-major. */
lem_status lem_plan_copy_block(lem_plan_t plan, int32_t unique, double* out,
                               int32_t* rows, int32_t* cols);

/* Free a plan and everything it owns.  Waits for the plan's stream and the
 * side streams its Krylov steps fork onto; steps the caller enqueued on other
 * streams must have completed.  NULL is ok. */
lem_status lem_plan_destroy(lem_plan_t plan);

/* ------------------------------------------------------------------------
 * Serving: continuous batching of independent time-stepping requests.
 *
 * Each request is one periodic problem (its own operator, dt, step count and
 * initial state, one ensemble member).  On admission it is planned like
 * lem_plan (partition with decay-bound buffers, per-block Krylov
 * calibration) -- or, when no core side keeps the buffer overhead within
 * max_overhead, as a global Krylov stepper (D = 1) -- and all of its device
 * memory (state, coefficients, work space) is taken from one pool of
 * hbm_budget bytes reserved at creation.  Requests are admitted first come,
 * first served while the pool and max_active allow.  Every lem_server_tick
 * advances every active request by steps_per_tick steps of (5) (fewer when
 * it has fewer left); the local problems of all active LEM requests run in
 * shared launches, one set per step (one Kronecker-factored launch for the
 * constant-coefficient 2D requests, bucketed Krylov launches for the rest).
 * The buffer width of a request comes from the decay bound, capped at
 * halo_max; a request whose bound exceeds the cap, or whose boxes fit
 * neither kernel, runs the global method.  Every block's arithmetic
 * depends only on its own request, so a request's result is the same whether
 * it runs alone or in a mix.  A server is not thread-safe.
 * ------------------------------------------------------------------------ */
typedef struct lem_server_s* lem_server_t;

enum { LEM_REQ_QUEUED = 0, LEM_REQ_ACTIVE = 1, LEM_REQ_DONE = 2, LEM_REQ_FAILED = 3 };

typedef struct {
  size_t hbm_budget;     /* bytes of device memory for resident requests       */
  int32_t max_active;    /* requests advanced together, >= 1                  */
  double halo_tol;       /* decay-bound tolerance per step                     */
  int32_t halo_min, halo_max;
  double max_overhead;   /* largest (local points / core points) before a
                            request falls back to the global method, >= 1    */
  double krylov_tol;     /* relative Krylov tolerance per step                 */
  int32_t krylov_m_max;  /* <= 40                                              */
  int32_t max_substeps;
  int32_t dry_run;       /* host-only scheduling: no device memory or kernels;
                            a finished request returns its initial state     */
  int32_t steps_per_tick; /* steps per tick of every active request, >= 1;
                            requests are admitted and retired between ticks,
                            so larger values trade admission latency for
                            fewer host synchronizations                      */
} lem_server_options;

/* A request whose step latched a device-side failure (non-finite values or a
 * Krylov estimate above tolerance) is retired as LEM_REQ_FAILED with error
 * LEM_ERR_NONFINITE or LEM_ERR_NOT_CONVERGED at the end of that tick; every
 * request has its own status word, so the others are not affected. */
typedef struct {
  int32_t state;         /* LEM_REQ_*                                          */
  int32_t method;        /* LEM_METHOD_KRONECKER, _KRYLOV or _GLOBAL           */
  int32_t core, halo;    /* partition (0, 0 for the global method)             */
  int32_t n_blocks, m_max, substeps_max;
  int32_t n_steps, steps_done;
  int64_t bytes;         /* pool bytes held while active                       */
  double t_submit_ms, t_admit_ms, t_done_ms;  /* ms since server creation      */
  int32_t error;         /* lem_status of a failed request                     */
} lem_request_info;

typedef struct {
  int32_t n_queued, n_active, n_done, n_failed;
  int64_t ticks;
  int64_t bytes_in_use, bytes_budget;
  double dof_steps;      /* grid points x steps advanced so far                */
  int32_t device_status; /* latched device-side status (0 = fine)              */
} lem_server_info;

/* Defaults: 8 GiB pool, 256 active, halo tol 1e-8 in [4, 56] (56: the
 * widest buffer of a 16-point core in a Kronecker box of side 128; the
 * Krylov box limit of 9216 points binds earlier), overhead 4,
 * Krylov tol 1e-12, m <= 30, <= 64 sub-steps, one step per tick. */
void lem_server_options_default(lem_server_options* opt);

/* Reserve the pool and create a server working on `stream`.  Errors:
 * LEM_ERR_INVALID (options), LEM_ERR_NOMEM (pool). */
lem_status lem_server_create(const lem_server_options* opt, void* stream, lem_server_t* out);

/* Queue a request: operator *op (copied, including nu_field), step dt,
 * n_steps >= 1 steps from the HOST state x0_host (N doubles, copied).
 * Returns its id.  LEM_ERR_BUDGET if its state alone cannot fit the pool;
 * LEM_ERR_INVALID for a bad operator. */
lem_status lem_server_submit(lem_server_t s, const lem_operator* op, double dt,
                             int32_t n_steps, const double* x0_host, uint64_t* id);

/* Admit queued requests, advance every active request by steps_per_tick
 * steps (at most the steps it has left), retire the finished ones (their
 * results are copied to host memory) and the failed ones.  Blocks until
 * the tick's device work is done.  Optional outputs: active / queued counts. */
lem_status lem_server_tick(lem_server_t s, int32_t* n_active, int32_t* n_queued);

/* State of a request (LEM_REQ_*); LEM_ERR_NOT_FOUND for unknown ids. */
lem_status lem_server_poll(lem_server_t s, uint64_t id, int32_t* state);

lem_status lem_server_request_info(lem_server_t s, uint64_t id, lem_request_info* info);

/* Copy a finished request's final state (N doubles) to x_host and forget the
 * request.  LEM_ERR_INVALID while it is not finished; a failed request
 * returns its error and is forgotten. */
lem_status lem_server_fetch(lem_server_t s, uint64_t id, double* x_host);

lem_status lem_server_query(lem_server_t s, lem_server_info* info);

/* Wait for the server's stream and free everything it owns.  NULL is ok. */
lem_status lem_server_destroy(lem_server_t s);

/* Message for the last non-OK status on this thread ("" if none). */
const char* lem_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* LEM_H */
