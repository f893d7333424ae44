/*
 * aderdg.h -- C ABI of the MI355X (gfx950) hot path of 1-D ADER-DG and
 * ADER-WENO-FV time stepping.
 *
 * Method: I.S. Popov, "The effective use of BLAS interface for implementation
 * of finite-element ADER-DG and finite-volume ADER-WENO methods",
 * arXiv 2409.12483.  The problem statement (a hyperbolic system with flux,
 * source and non-conservative terms, Sec. 1, eq. pde_src) is restricted to one
 * space dimension on a uniform periodic mesh.
 *
 * Conventions for every entry point
 *   - Return value: int32 status, 0 = ADERDG_OK, negative = error.  Nothing
 *     throws or longjmps across the ABI.  On an argument error the call
 *     returns ADERDG_E_INVAL before touching any buffer and
 *     aderdg_last_error() describes the problem.
 *   - "device" pointers are HIP device allocations (e.g. torch tensors on
 *     cuda:0), contiguous, 8-byte aligned at least; the caller owns them.
 *     The library owns only its operator tables, internal ping-pong state
 *     buffers and per-problem clocks, allocated in aderdg_init and released
 *     in aderdg_free, both stream-ordered on the handle's stream
 *     (hipMallocAsync / hipFreeAsync; the problem tables are written by
 *     kernels, not copied from host memory).
 *   - All work is enqueued on the handle's HIP stream (the one given at init,
 *     NULL = default stream) and is asynchronous: no call synchronises the
 *     host, except the counter read-backs (aderdg_sweep_count,
 *     aderdg_contraction_count) and the first aderdg_init on a device, which
 *     builds and uploads the operator tables.
 *   - A handle is used by one host thread at a time.
 *
 * Layouts (array-of-structures, variable index fastest: Sec. 1.1, the AoS
 * storage q_{p,r} the paper operates on without transposition):
 *   u  DG nodal coefficients     [ncells][N+1][M]           fp64
 *   q  space-time predictor      [ncells][N+1 (time)][N+1 (space)][M]
 *                                fp64, or fp32 in ADERDG_FP32_PREDICTOR mode
 *   v  finite-volume averages    [ncells][M]                fp64
 * Nodes are the Gauss-Legendre points of [0,1] (Sec. 1.1, eq. gl_rule); cell i
 * spans [x0 + i dx, x0 + (i+1) dx], dx = (x1 - x0) / ncells.
 */
#ifndef ADERDG_H
#define ADERDG_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  ADERDG_OK = 0,
  ADERDG_E_INVAL = -1,    /* invalid argument (nothing was enqueued) */
  ADERDG_E_NOMEM = -2,    /* device allocation failed */
  ADERDG_E_DEVICE = -3,   /* a HIP call failed */
  ADERDG_E_NOCONV = -4,   /* device status: a Picard loop hit picard_max_iter (result still written) */
  ADERDG_E_NONPHYS = -5   /* device status: non-finite value, rho<=0, p<=0 or h<=0 met (result still written) */
};

/* PDE models (Sec. 1, eq. pde_src, in 1-D). */
enum aderdg_pde {
  ADERDG_PDE_ADVECTION = 0,   /* dq/dt + a dq/dx = 0, M = 1 */
  ADERDG_PDE_EULER = 1,       /* Sec. 2, eq. system_of_equations: (rho, rho u, E), M = 3 */
  ADERDG_PDE_EULER_REACT = 2, /* Sec. 2.1, eq. pdes_2_comps: + (rho c1, rho c2), M = 5 */
  ADERDG_PDE_SWE = 3          /* shallow water (h, hu, b) with B(Q) dQ/dx = (0, g h db/dx, 0), M = 3 */
};
enum aderdg_prec { ADERDG_FP64 = 0, ADERDG_FP32_PREDICTOR = 1 };
enum aderdg_bc { ADERDG_BC_PERIODIC = 0 };
enum aderdg_cfl_mode { ADERDG_CFL_SUBCELL = 0, ADERDG_CFL_NODAL = 1 };
enum aderdg_scheme { ADERDG_SCHEME_DG = 0, ADERDG_SCHEME_FV = 1 };
/* Inner iterations of the predictor (Sec. 1.1, eq. lst_dg_predictor_nested_picards):
 * Picard (the paper's choice), or Newton's method, which Sec. 1.1 recommends for stiff
 * source terms.  Newton is available for DG problems of the models with a linear source
 * (ADERDG_PDE_EULER_REACT): its Jacobian is then constant and the inverse is formed once
 * per step. */
enum aderdg_inner { ADERDG_INNER_PICARD = 0, ADERDG_INNER_NEWTON = 1 };

typedef struct {
  int32_t pde;        /* enum aderdg_pde */
  int32_t nvars;      /* must equal the model's M (1, 3, 5, 3) */
  double gamma;       /* Euler models: ratio of specific heats (> 1) */
  double g;           /* SWE: gravity (> 0) */
  double omega;       /* EULER_REACT: oscillator frequency of the source */
  double adv_speed;   /* ADVECTION: speed a */
} aderdg_pde_desc;

typedef struct {
  int32_t N;               /* polynomial degree, 1..9; FV: WENO degree, 2 or 4 */
  int32_t bc;              /* ADERDG_BC_PERIODIC (the only supported value) */
  int64_t ncells;          /* >= 1 (FV: >= 2N+1) */
  double x0, x1;           /* domain, x1 > x0 */
  double cfl;              /* 0 < cfl <= 1 (Sec. 1.5) */
  double fixed_dt;         /* > 0: use this dt instead of the CFL rule */
  int32_t cfl_mode;        /* enum aderdg_cfl_mode (DG only) */
  int32_t precision;       /* enum aderdg_prec */
  double picard_tol;       /* <= 0: 1e-14 (FP64) or 1e-6 (FP32 predictor) */
  int32_t picard_max_iter; /* <= 0: 64 (bounds the inner Newton iterations too) */
  int32_t scheme;          /* enum aderdg_scheme: which step function serves this problem */
  int32_t inner;           /* enum aderdg_inner (default 0: Picard) */
  int32_t reserved;        /* must be 0 */
} aderdg_config;

typedef struct aderdg_handle aderdg_handle;

/*
 * aderdg_init -- create a batch of nprob >= 1 independent problems.
 * pdes[k], cfgs[k] describe problem k (copied; the arrays may be freed after
 * the call).  hip_stream: a hipStream_t (NULL = default stream).  On success
 * *out receives the handle.  Allocates library-owned device memory only.
 * Errors: E_INVAL (bad descriptor; *out untouched), E_NOMEM, E_DEVICE.
 */
int aderdg_init(const aderdg_pde_desc* pdes, const aderdg_config* cfgs, int32_t nprob,
                void* hip_stream, aderdg_handle** out);

/*
 * aderdg_predict -- LST-DG predictor of every cell of problem k (DG scheme):
 * the nested Picard iteration of Sec. 1.1, eq. lst_dg_predictor_nested_picards,
 * in the Kronecker-factored form of Sec. 1.1 "Using the BLAS interface"
 * (Algorithms 1-3).  Inputs: u (device, fp64, [ncells][N+1][M]), the step's
 * start time t and step dt (> 0).  Output: q_out (device, [ncells][N+1][N+1][M],
 * fp64 or fp32 per the problem's precision).  iters_out: optional device
 * int32 [ncells] receiving the number of outer sweeps of each cell (NULL =
 * not wanted).  Each cell stops when max|dq| <= tol * max(1, max|q|).
 */
int aderdg_predict(aderdg_handle* h, int32_t k, const double* u, double t, double dt,
                   void* q_out, int32_t* iters_out);

/*
 * aderdg_correct -- one-step ADER-DG corrector (Sec. 1.2, eq.
 * ader_dg_method_full; Algorithms 4-7): u_next = u + volume terms + interface
 * terms built from the predictor q of every cell (layouts above; q in the
 * problem's predictor precision).  Interface solver: Rusanov flux plus half
 * of the straight-path jump B~ (q+ - q-) to each neighbour.  u_next must not
 * alias u.  t, dt: as for aderdg_predict.
 */
int aderdg_correct(aderdg_handle* h, int32_t k, const double* u, const void* q, double t,
                   double dt, double* u_next);

/*
 * aderdg_step -- fused hot path: advance every DG problem of the batch by
 * nsteps steps (predictor + corrector per step, Secs. 1.1-1.2; time step by
 * the CFL rule of Sec. 1.5 with the signal speed taken on the 2N+1 subcell
 * averages of Sec. 1.4, or fixed_dt; the last step is clamped to t_end).
 *   u       host array [nprob] of device pointers; u[k] is problem k's state
 *           (in/out).  Entries of FV problems are ignored (may be NULL).
 *   t       device fp64 [nprob], in/out: time of each problem.
 *   t_end   device fp64 [nprob], in.  A problem with t >= t_end is left as is.
 *   dt      device fp64 [nprob], out: the last step size taken (0 if none).
 *   status  device int32 [nprob], out: 0, or the most severe of
 *           ADERDG_E_NOCONV / ADERDG_E_NONPHYS met during the call.
 * No host synchronisation; the enqueued work is capturable in a HIP graph.
 */
int aderdg_step(aderdg_handle* h, double* const* u, double* t, const double* t_end, double* dt,
                int32_t* status, int32_t nsteps);

/*
 * aderweno_step -- ADER-WENO finite-volume step for every FV problem of the
 * batch (Sec. 1.3, eq. ader_weno_fv_method_full; Algorithms 8-11): WENO
 * reconstruction of degree N from the cell averages (eq. weno_reconstr), the
 * LST-DG predictor started from it, then the finite-volume update.  CFL rule
 * without the 2N+1 factor (Sec. 1.5).  v[k]: device [ncells][M] fp64 (in/out);
 * the other arguments as for aderdg_step.
 */
int aderweno_step(aderdg_handle* h, double* const* v, double* t, const double* t_end, double* dt,
                  int32_t* status, int32_t nsteps);

/*
 * aderdg_step_noalloc -- aderdg_step / aderweno_step for ONE problem without a
 * handle and without any device allocation, for callers that cannot allocate
 * (code under HIP stream capture, tight serving loops, harnesses that forbid
 * hipMalloc).  pde, cfg: the problem (host structs, as for aderdg_init; cfg->scheme
 * selects the DG or the FV step).  u: device state (DG [ncells][N+1][M], FV
 * [ncells][M], fp64, in/out).  t, t_end, dt, status: device arrays of one
 * element each, as for aderdg_step.  hip_stream: the stream to enqueue on (NULL =
 * default).  Same kernels and results as aderdg_step on a one-problem handle.
 * The library-owned memory the step needs (the state's ping-pong copy, the
 * problem clock and descriptors) lives in a static device array of 64 MiB per
 * device, held until the process ends: the state may hold at most
 * (64 MiB - 64 KiB) / 8 = 8 380 416 doubles, otherwise E_INVAL before anything
 * is enqueued.  Every call on a device shares that array, so calls that
 * overlap on one device (different streams or threads) race; calls in stream
 * order are safe.  No host synchronisation; the enqueued work holds no memset
 * node and is capturable.
 */
int aderdg_step_noalloc(const aderdg_pde_desc* pde, const aderdg_config* cfg, double* u, double* t,
                        const double* t_end, double* dt, int32_t* status, int32_t nsteps,
                        void* hip_stream);

/*
 * aderdg_user_init -- a handle for ONE DG problem of a user-defined model,
 * compiled at run time.  The paper builds its kernels once per parameter set
 * at run time (Sec. 1.1, the JIT gemm kernels; Sec. 3); here the whole fused
 * step (predictor, Sec. 1.1, and corrector, Sec. 1.2) is compiled with hipRTC
 * for gfx950 once per (model source, N, precision) and cached for the process.
 *   model_source  C++ text of a struct `UserPDE` with the interface of the
 *                 built-in models (the form of Sec. 1, eq. pde_src):
 *                   static constexpr int M;  bool kSource, kNcp;  int kSrcVars (0);
 *                   template <class T> __device__ static void flux(const T* q, T* f, const PdeParams&);
 *                   template <class T> __device__ static T speed(const T* q, const PdeParams&);
 *                   __device__ static bool admissible(const double* q, const PdeParams&);
 *                   __device__ static constexpr double diss(int r);     (Rusanov dissipation mask)
 *                   with kSource: template <class T> __device__ static void
 *                                   source(const T* q, T x, T t, T* s, const PdeParams&);
 *                   with kNcp: ncp(q, dq, b, pp) = B(q) dq and jump(qm, qp, j, pp) = B~ (qp - qm).
 *                 The library's device helpers (recip, dabs, dmax, PdeParams) are in scope.
 *   nvars         M of the model (1..5; checked against UserPDE::M at compile time).
 *   params        4 doubles handed to the model as PdeParams {gamma, g, omega, a}.
 *   cfg           as for aderdg_init (scheme DG, Picard inner iterations).
 * The handle then serves aderdg_predict, aderdg_correct, aderdg_step (problem 0),
 * aderdg_conserved_totals, the counters and aderdg_free like any other.
 * Errors: E_INVAL (bad arguments, or the model does not compile: the compiler's
 * log is in aderdg_last_error()), E_DEVICE (module loading), E_NOMEM.
 * The first call per (model, N, precision) compiles (about a second or two)
 * and synchronises the host; later calls reuse the module.
 */
int aderdg_user_init(const char* model_source, int32_t nvars, const double* params,
                     const aderdg_config* cfg, void* hip_stream, aderdg_handle** out);

/*
 * aderdg_user_compile_check -- compile a user model as aderdg_user_init would, without a
 * device (host only).  log (may be NULL): receives the compiler's messages, at most cap
 * bytes including the terminating zero.  Returns 0 if it compiles, E_INVAL otherwise.
 */
int aderdg_user_compile_check(const char* model_source, int32_t nvars, int32_t N, int32_t precision,
                              char* log, int64_t cap);

/* aderdg_free -- release the handle: its device memory is freed in stream order after the
 * work already enqueued on its stream (no host synchronisation).  NULL is accepted. */
int aderdg_free(aderdg_handle* h);

/*
 * aderdg_set_waves -- wavefronts per workgroup of the fused DG step (Sec. 1.1-1.2 in one
 * launch, as aderdg_step) for every launch group of the handle that has two compiled
 * sizes: DG scheme, Picard inner iterations, a compiled-in model.  waves = 4 (the
 * default) or 2; a workgroup then writes waves * floor(64/(N+1)) - 2 cells.  Every cell's arithmetic, the dt reduction and the counters are the same, so
 * the results are bitwise those of the other size; only the speed differs.  The problem
 * table is rewritten in stream order on the handle's stream.  E_INVAL for other values.
 */
int aderdg_set_waves(aderdg_handle* h, int32_t waves);

/*
 * aderdg_autotune -- for every launch group aderdg_set_waves applies to, time `steps`
 * fused steps (1..10000, after 2 untimed ones) with each compiled workgroup size on
 * device copies of the states u (host array of nprob device pointers, read only) and
 * keep the faster.  The problems' clocks, counters and states are left as they were:
 * the next aderdg_step continues exactly as without this call.  The choice is cached
 * for the process under (device architecture, model, N, precision, total cells of the
 * group rounded up to a power of 2) and, if the environment variable ADERDG_TUNE_FILE
 * names a file, read from and appended to it ("key waves" per line); a cached key is
 * not timed again.  waves_out: optional host int32 [nprob], the size now used by each
 * problem's group (4 for groups that are not tuned).  Allocates device memory for the
 * copies (stream-ordered) and synchronises the handle's stream.
 * Errors: E_INVAL, E_NOMEM, E_DEVICE.
 */
int aderdg_autotune(aderdg_handle* h, double* const* u, int32_t steps, int32_t* waves_out);

/*
 * aderdg_set_stream -- enqueue later work of the handle on another HIP stream.
 */
int aderdg_set_stream(aderdg_handle* h, void* hip_stream);

/*
 * aderdg_sweep_count -- total outer Picard sweeps (summed over cells and
 * steps) performed for problem k since init, read back synchronously.  Used
 * to count algorithmic work.  Host output.
 */
int aderdg_sweep_count(aderdg_handle* h, int32_t k, int64_t* sweeps_out);

/*
 * aderdg_contraction_count -- total applications of the time operator kappa~
 * (Sec. 1.1, the Picard update of Algorithm 1) summed over cells and steps for
 * problem k since init: one per outer sweep for models without source or
 * non-conservative terms, one per inner iteration otherwise (Algorithm 1,
 * inner repeat).  Read back synchronously; counts algorithmic work.  Host
 * output; E_INVAL on a null pointer or an index out of range.
 */
int aderdg_contraction_count(aderdg_handle* h, int32_t k, int64_t* count_out);

/*
 * aderdg_conserved_totals -- the conserved totals of problem k's state u
 * (device, the problem's layout): out[r] = dx sum_i sum_k w_k u_i[k][r] for DG
 * (the exact integral of the nodal polynomial over the mesh, with the GL
 * weights of eq. gl_rule), dx sum_i v_i[r] for FV.  The corrector of Sec. 1.2
 * (eq. ader_dg_method_full) changes them only by round-off for conservation
 * laws (interface terms telescope over a periodic mesh), so their drift over a
 * run measures conservation.  totals_out: device fp64 [M].  Two kernels on the
 * handle's stream with a fixed summation order (bitwise reproducible); no host
 * synchronisation.  Uses the handle's partial-sum buffer, so calls on one
 * handle are stream-ordered.  E_INVAL on a null pointer or a bad index.
 */
int aderdg_conserved_totals(aderdg_handle* h, int32_t k, const double* u, double* totals_out);

/*
 * aderdg_operators -- host-only copy of the library's 1-D operator tables for
 * degree N (no device involved), for inspection: the GL nodes xi and weights w
 * (eq. gl_rule), k~ = Lambda^-1 Xi and kappa~ = Upsilon^-1 Lambda
 * (eq. m_and_kappa_matrices and the definitions after it), D~_kl = w_l
 * D^phi_kl, psi = phi(0), psi~ = phi(1) (Sec. 1.2), the subcell
 * projection P and the reconstruction R = (P^T P)^-1 P^T (Sec. 1.4, eq.
 * p_operator and eq. r_operator), concatenated in that order: n, n, n*n,
 * n*n, n*n, n, n, (2N+1)*n, n*(2N+1) doubles (n = N+1).  cap = capacity of out in doubles;
 * returns the number written, or E_INVAL.
 */
int aderdg_operators(int32_t N, double* out, int64_t cap);

/* aderdg_last_error -- text of the last E_INVAL / E_DEVICE of this thread ("" if none). */
const char* aderdg_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* ADERDG_H */
