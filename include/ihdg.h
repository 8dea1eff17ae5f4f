/*
 * ihdg.h -- C ABI of the MI355X iHDG library.
 *
 * The library solves the upwind-HDG discretisation of a linear first-order
 * system (the paper's Section 2, eq. LPDE, discretised as in eqs. HDGlocal,
 * HDGeqn and RiemannFluxBoth) with the iterative HDG method (Algorithm 1):
 * every sweep solves each element's local problem independently, taking the
 * weighted trace of the previous iterate on its faces, so no global trace
 * system is ever formed.  Three PDE families are supported, as in the paper:
 *
 *   IHDG_TRANSPORT      div(beta u) + sigma u = f, u = g on the inflow
 *                       boundary (Section 3, eqs. transportLocalk1 and
 *                       transportLocale; sigma is an added reaction);
 *   IHDG_SHALLOW_WATER  one implicit step of the linearised shallow-water
 *                       system (Section 3, eq. linearizedShallow and the local
 *                       equations localSolverDD), walls on the boundary;
 *   IHDG_CONVDIFF       first-order convection-diffusion (Section 4,
 *                       eq. Convection-diffusion-eqn and the iterative scheme
 *                       that follows it), Dirichlet data on the boundary.
 *
 * Discretisation: uniform box of quads (dim 2) or hexes (dim 3); tensor Q^p
 * Lagrange basis on Gauss-Lobatto-Legendre nodes; Gauss-Legendre quadrature
 * with p+2 points per direction on volumes and faces.
 *
 * Memory ownership.  Every device buffer (coefficients, workspace, scratch,
 * solution copies) is allocated by the caller; the library never calls
 * hipMalloc or hipFree.  The library owns only the host-side context.
 * `workspace` must stay allocated until ihdg_destroy; `scratch` may be freed
 * as soon as ihdg_setup has returned.  Coefficient arrays are read during
 * ihdg_setup only.
 *
 * Streams.  All device work of a context is ordered on the stream given to
 * ihdg_setup (or ihdg_set_stream).  Calls that return host values
 * synchronise that stream; the others only enqueue work.
 *
 * Errors.  Every call returns an ihdg_status; no exception crosses the ABI.
 * On error, output arguments are left untouched and ihdg_last_error() gives a
 * message.  Asynchronous HIP faults surface as IHDG_ERR_HIP at the next
 * synchronising call.  IHDG_ERR_DIVERGED and IHDG_ERR_MAXITER leave the last
 * iterate in place (readable with ihdg_get_solution).
 *
 * Thread safety.  A context may be used by one host thread at a time;
 * distinct contexts are independent.
 */
#ifndef IHDG_H
#define IHDG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ihdg_ctx ihdg_ctx;

typedef enum {
  IHDG_OK = 0,
  IHDG_ERR_ARG = 1,            /* invalid argument (null pointer, bad size, bad enum)     */
  IHDG_ERR_UNSUPPORTED = 2,    /* valid but not supported (order, dim, mixed-sign face)   */
  IHDG_ERR_NOMEM = 3,          /* workspace or scratch smaller than ihdg_footprint says   */
  IHDG_ERR_HIP = 4,            /* a HIP runtime call or kernel failed                     */
  IHDG_ERR_SINGULAR_LOCAL = 5, /* a local HDG matrix could not be factored                */
  IHDG_ERR_DIVERGED = 6,       /* increment non-finite or grew 1e3x above its minimum    */
  IHDG_ERR_MAXITER = 7         /* tolerance not reached within max_iters sweeps           */
} ihdg_status;

typedef enum { IHDG_TRANSPORT = 0, IHDG_SHALLOW_WATER = 1, IHDG_CONVDIFF = 2 } ihdg_pde;

typedef enum {
  IHDG_FP64 = 0,  /* FP64 operators, FP64 state, FP64 sweeps                               */
  IHDG_MIXED = 1  /* FP32 operators and FP32 correction sweeps; FP64 defect sweeps, FP64
                     convergence test and FP64 solution update (defect correction)          */
} ihdg_precision;

/* Uniform box [lo, hi] split into n[0] x n[1] (x n[2]) elements.  Elements are
 * numbered lexicographically, x fastest.  Unused entries (dim 2: index 2) are
 * ignored. */
typedef struct {
  int32_t dim;     /* 2 or 3 (3 only for IHDG_TRANSPORT) */
  int32_t n[3];
  double lo[3];
  double hi[3];
} ihdg_mesh;

/* Sizes of the discretisation (filled by ihdg_sizes). */
typedef struct {
  int64_t n_el;      /* number of elements                                              */
  int64_t n_face;    /* number of unique faces of the skeleton                          */
  int32_t np;        /* nodes per element and field, (p+1)^dim                           */
  int32_t m;         /* fields: 1 transport, 3 shallow water, dim+1 convection-diffusion */
  int32_t n_loc;     /* local unknowns, m*np                                             */
  int32_t nq;        /* volume quadrature points per element, (p+2)^dim                  */
  int32_t nfq;       /* quadrature points per face, (p+2)^(dim-1)                        */
  int32_t nfp;       /* nodes per face, (p+1)^(dim-1)                                    */
  int32_t n_in;      /* face values feeding a local solve, 2*dim*nfp                     */
  int32_t m_f;       /* components of the forcing array: 1, or 3 for shallow water       */
} ihdg_sizes_t;

/*
 * Coefficients and data, all device pointers to FP64 arrays, all read only
 * during ihdg_setup.  Quadrature points are the ones ihdg_quadrature_points
 * returns.  Faces are numbered as ihdg_quadrature_points documents; every
 * face-point array is indexed by unique face, so both elements of a face see
 * the same values.
 *
 *   beta_q    [n_el][nq][dim]  advection field (transport, conv.-diff.), or NULL
 *                              to use beta_const everywhere
 *   divbeta_q [n_el][nq]       div beta at the volume points, or NULL for 0
 *   bn_fq     [n_face][nfq]    beta . e_axis at the face points (e_axis = the
 *                              face's coordinate axis, pointing to +axis), or
 *                              NULL to take it from beta_const
 *   sigma_el  [n_el]           transport reaction per element, or NULL for
 *                              sigma_const
 *   f_q       [n_el][nq][m_f]  forcing at the volume points, or NULL for 0
 *   g_fq      [n_face][nfq]    boundary data at the face points (transport:
 *                              inflow values; conv.-diff.: Dirichlet values),
 *                              entries of interior faces are ignored; NULL = 0
 *
 * The shared-operator path (one reference local operator for all elements)
 * is taken when the local matrices cannot differ between elements: transport
 * with beta_q, divbeta_q, bn_fq and sigma_el all NULL; shallow water always;
 * conv.-diff. with beta_q and bn_fq NULL.  Otherwise every element gets its
 * own pre-factored operator.
 */
typedef struct {
  const double* beta_q;
  const double* divbeta_q;
  const double* bn_fq;
  const double* sigma_el;
  const double* f_q;
  const double* g_fq;
  double beta_const[3];
  double sigma_const;
  double kappa;      /* conv.-diff.: diffusion coefficient (kappa > 0)                 */
  double nu;         /* conv.-diff.: reaction nu                                       */
  double Phi;        /* shallow water: mean geopotential Phi > 0                       */
  double f0;         /* shallow water: Coriolis parameter (constant)                   */
  double gamma;      /* shallow water: bottom friction                                 */
  double mass_coef;  /* shallow water: coefficient a/dt of the mass term (a = 2: CN)   */
  /* conv.-diff. stabilisation (the comment on elliptic PDEs closing Section 4).
   * 0: the upwind flux, tau = (alpha - beta.n)/2 with alpha = sqrt((beta.n)^2 + 4).
   * gamma > 0: the mesh-dependent tau* = gamma (p+1)(p+2)/h on every face, h the
   * smallest element edge, so the trace is
   *   uhat = (jump(s.n) + jump(beta.n u) + tau* (u- + u+)) / (2 tau*);
   * the paper's analysis asks for gamma > d/4, and convergence of the iteration
   * then holds only on meshes that are not too fine (solve with krylov_restart on
   * fine meshes).  Negative values, or a nonzero value for another PDE, are
   * IHDG_ERR_ARG.                                                                  */
  double tau_gamma;
} ihdg_coeffs;

typedef struct {
  ihdg_precision prec;
  int32_t check_every;     /* sweeps per convergence check (0 = library default, 16)           */
  int32_t max_iters;       /* sweep cap of ihdg_solve (0 = 100000)                            */
  int32_t krylov_restart;  /* 0: plain iHDG; 0 < m <= 256: GMRES(m) on (I - T)u = c, T the sweep.
                              With prec = IHDG_MIXED every restart forms the true residual with
                              one FP64 sweep, and the cycle runs with the FP32 operators and an
                              FP32 basis ((m+1) x 4 bytes per unknown instead of 8), updating u
                              in FP64; the tolerance is the same FP64 relative residual       */
  double inner_rtol;       /* mixed: inner FP32 loop stops when its increment <= this x the
                              correction; mixed GMRES: a cycle ends once its residual estimate
                              fell by this factor (0 = 1e-6)                                  */
  int32_t use_graph;       /* 1: replay sweep batches from a captured HIP graph               */
  int32_t force_per_element; /* 1: per-element operators even where one could be shared      */
  int32_t block_waves;     /* launch shape of the sweep kernel: 0 = autotuned at setup (cached per
                              shape), 1/2/4/8 = waves per 64-element block, 3 = vector-FMA shared
                              operator, 5 = transport (2-D, 3-D p <= 3) or convection-diffusion
                              (2-D p <= 4, the face projection folded into the operator) with a
                              shared operator on the matrix cores without LDS staging of the
                              traces.  Other values:
                              IHDG_ERR_ARG; 3 or 5 where they do not apply: IHDG_ERR_UNSUPPORTED */
  int32_t time_stepping;   /* 1: keep what ihdg_time_step needs (shared operators only)               */
  int32_t transport_flux;  /* transport only: 0 = upwind HDG flux (eq. RiemannFluxBoth with |A| = |beta.n|),
                              1 = the NPC flux analysed after Theorem 1 (eq. Ntaub): tau = 0 on outflow,
                              |beta.n| on inflow, so the iteration terminates after as many sweeps as the
                              mesh has flow layers (Theorem 2); same fixed point                        */
  int32_t krylov_method;   /* 0: GMRES(krylov_restart) as above.  1: BiCGStab (van der Vorst) on
                              (I - T)u = c, FP64, two sweeps per iteration and six vectors of
                              workspace, scalars kept on the device; krylov_restart must be > 0
                              to select a Krylov solve and is otherwise unused; the recursive
                              residual is confirmed by the true one before IHDG_OK, and the
                              iteration restarts from the current u when they disagree or when
                              the recursive residual has not improved for 256 iterations; four
                              restarts in a row without progress end with IHDG_ERR_MAXITER.  max_iters
                              caps the iterations; prec must be IHDG_FP64 (else IHDG_ERR_UNSUPPORTED).
                              The iHDG sweep as the Krylov operator is the use the paper suggests
                              for regimes where the plain iteration fails (end of Section 4)      */
  int32_t mixed_period;    /* IHDG_MIXED without krylov_restart: FP32 correction sweeps between
                              two FP64 defect sweeps (0 = 4 x check_every).  Every outer step
                              forms the FP64 defect d = psi(u) - u, starts the FP32 correction
                              at delta = d (the first sweep from zero), runs this many FP32
                              sweeps delta <- d + G32 x(delta) and adds delta to u in FP64, so
                              the solve advances the iteration by mixed_period + 1 sweeps per
                              outer step.  Once the last defect is within 1e3 x tol, a round of
                              check_every FP32 sweeps whose increment meets tol ends the
                              correction early (the FP64 defect then decides).  < 0: each
                              correction runs until its increment falls below inner_rtol or
                              stalls at the FP32 rounding floor                                */
} ihdg_options;

/* Discretisation sizes for (mesh, order, pde).  No device work. */
ihdg_status ihdg_sizes(const ihdg_mesh* mesh, int32_t order, ihdg_pde pde, ihdg_sizes_t* out);

/*
 * Quadrature points at which the caller evaluates its coefficients.
 *   xq_dev  [n_el][nq][dim]   volume points of every element (may be NULL)
 *   xfq_dev [n_face][nfq][dim] face points of every unique face (may be NULL)
 * Unique faces: first all faces normal to x, then normal to y, then z.  The
 * faces normal to axis a are indexed lexicographically (x fastest) by their
 * integer position j with j_a in [0, n_a] and j_b in [0, n_b) for b != a.
 * Points inside a volume or face are ordered lexicographically over the
 * Gauss points, lowest remaining axis fastest.  `stream` is a hipStream_t.
 */
ihdg_status ihdg_quadrature_points(const ihdg_mesh* mesh, int32_t order, double* xq_dev,
                                   double* xfq_dev, void* stream);

/*
 * Coordinates of the GLL nodes of every element, x_dev [n_el][np][dim]
 * (nodes lexicographic, x fastest): where a nodal initial state or warm start
 * for ihdg_set_solution is evaluated.  `stream` is a hipStream_t.
 */
ihdg_status ihdg_node_points(const ihdg_mesh* mesh, int32_t order, double* x_dev, void* stream);

/*
 * Device memory the caller must provide to ihdg_setup for these arguments:
 * `persistent_bytes` for the workspace (operators, state, maps) and
 * `scratch_bytes` for setup-only scratch.  `coeffs` decides shared versus
 * per-element operators (it may be NULL: per-element unless shallow water).
 */
ihdg_status ihdg_footprint(const ihdg_mesh* mesh, int32_t order, ihdg_pde pde,
                           const ihdg_coeffs* coeffs, const ihdg_options* opts,
                           size_t* persistent_bytes, size_t* scratch_bytes);

/*
 * Assemble every local HDG operator and reduce it by Gauss-Jordan elimination
 * with partial pivoting (FP64, on the GPU) to G_K = L_K^{-1} E_K and
 * c_K = L_K^{-1} F_K, so that a sweep is u_K^{k+1} = c_K + G_K x_K(u^k) (the
 * local solve of eq. iHDGlocal with the weighted trace of eq. iHDGtrace as its
 * input x_K).  The initial iterate is u^0 = 0.  `workspace` and `scratch` are
 * caller-owned device buffers of at least the ihdg_footprint sizes, 256-byte
 * aligned; the workspace must outlive the context, the scratch may be freed
 * once this returns.  *out is a library-owned host object, freed by
 * ihdg_destroy.  `stream` is a hipStream_t.  Synchronises the stream (it
 * checks for setup errors).  Errors (no context is returned):
 *   IHDG_ERR_ARG          NULL or misaligned pointers, an invalid mesh, order,
 *                         option or coefficient (e.g. kappa <= 0, Phi <= 0);
 *   IHDG_ERR_UNSUPPORTED  a valid request this library does not serve: an
 *                         interior transport face on which beta.n changes sign,
 *                         a launch shape that does not apply, BiCGStab with the
 *                         mixed precision, time stepping without a shared
 *                         operator;
 *   IHDG_ERR_NOMEM        workspace or scratch smaller than the footprint;
 *   IHDG_ERR_SINGULAR_LOCAL  a local matrix with a pivot of magnitude
 *                         <= 1e-300 or not finite (e.g. non-finite coefficients);
 *   IHDG_ERR_HIP          a HIP call or kernel failed.
 */
ihdg_status ihdg_setup(const ihdg_mesh* mesh, int32_t order, ihdg_pde pde, const ihdg_coeffs* coeffs,
                       const ihdg_options* opts, void* workspace, size_t workspace_bytes,
                       void* scratch, size_t scratch_bytes, void* stream, ihdg_ctx** out);

/*
 * ihdg_setup for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): the
 * same setup and the same context, without the `scratch` argument.  The setup
 * scratch is a 64 MiB device array inside the library (one per device, held
 * until the process ends); local problems are assembled and reduced in chunks
 * that fit it.  Calls no hipMalloc, hipFree or other allocating routine and
 * creates no HIP events: with opts.block_waves = 0 the launch shape is the one
 * the autotuner has cached for this problem shape, else 4 waves per block
 * (nothing is timed).  Calls in one process are serialised (the array is
 * shared) and each has finished its device work when it returns.  The caller
 * still provides the workspace (the footprint's persistent_bytes).  Errors as
 * ihdg_setup, and IHDG_ERR_NOMEM if one element's local problem does not fit
 * the 64 MiB (no supported order comes near it).
 */
ihdg_status ihdg_setup_noalloc(const ihdg_mesh* mesh, int32_t order, ihdg_pde pde, const ihdg_coeffs* coeffs,
                               const ihdg_options* opts, void* workspace, size_t workspace_bytes, void* stream,
                               ihdg_ctx** out);

/*
 * Run n_sweeps iHDG sweeps (Algorithm 1, the local solve and trace update) in
 * the context's working precision: FP64 for IHDG_FP64; for IHDG_MIXED the
 * sweeps are FP64 too (ihdg_solve is where the mixed path runs).  If
 * incr_norm is not NULL it receives, after synchronising, the h-norm of the
 * last increment ||u^k - u^{k-1}||_h and, in incr_norm[1], ||u^k||_h.
 * The h-norm is ||e||_h^2 = sum_K |J_K| sum_i W_i e_i^2 (GLL weights W_i).
 */
ihdg_status ihdg_sweep(ihdg_ctx* ctx, int32_t n_sweeps, double* incr_norm);

/*
 * Run n_sweeps of the mixed path's FP32 correction sweeps
 * delta <- d + G32 x(delta) (FP32 operators, FP32 state, the FP32 matrix
 * cores or FP32 FMAs) on the context's correction state: zero after setup,
 * the last correction after ihdg_solve.  incr_norm as in ihdg_sweep, of the
 * correction.  IHDG_ERR_UNSUPPORTED unless the context is IHDG_MIXED.  For
 * timing the FP32 sweep; the solution is not touched.
 */
ihdg_status ihdg_sweep32(ihdg_ctx* ctx, int32_t n_sweeps, double* incr_norm);

/*
 * Iterate from the current iterate until ||u^k - u^{k-1}||_h <= tol ||u^k||_h
 * (IHDG_FP64, plain iHDG), or until the FP64 defect ||psi(u) - u||_h <= tol
 * ||u||_h (IHDG_MIXED; and the Krylov path, on its residual).  iters receives
 * the number of sweeps (FP64 + FP32 for mixed), final_incr the last relative
 * increment, final_defect the relative FP64 defect of the returned iterate
 * (one extra FP64 sweep, not counted in iters).  Any output may be NULL.
 * Errors: IHDG_ERR_ARG (NULL ctx, tol <= 0); IHDG_ERR_DIVERGED (a non-finite
 * increment or residual, or an increment 1e3x above its smallest);
 * IHDG_ERR_MAXITER (max_iters reached; for BiCGStab also four restarts in a
 * row without progress); IHDG_ERR_HIP.  After DIVERGED or MAXITER the last
 * iterate stays readable; final_defect is filled in after IHDG_OK and
 * IHDG_ERR_MAXITER only.
 */
ihdg_status ihdg_solve(ihdg_ctx* ctx, double tol, int32_t* iters, double* final_incr,
                       double* final_defect);

/* Relative FP64 defect ||psi(u) - u||_h / ||u||_h of the current iterate, where
 * psi is one FP64 sweep; defect_norm[0] = relative, defect_norm[1] = absolute.
 * Does not change the iterate. */
ihdg_status ihdg_residual(ihdg_ctx* ctx, double* defect_norm);

/* Copy the current iterate to / from u_dev, FP64 [n_el][m][np] (element-major,
 * fields contiguous per element, GLL nodes lexicographic, x fastest).
 * Stream-ordered; no synchronisation. */
ihdg_status ihdg_get_solution(ihdg_ctx* ctx, double* u_dev);
ihdg_status ihdg_set_solution(ihdg_ctx* ctx, const double* u_dev);

/*
 * Time marching (the time-dependent remarks of Sections 3 and 4 and the
 * shallow-water experiment of Section 5): turn the current iterate u^n into the
 * right-hand side of the next implicit step, keeping u^n as the warm start of
 * the next ihdg_solve.  The context's operator is the implicit one,
 * A = mass_coef * M_Phi + S (M_Phi: the mass matrix, times Phi on the
 * shallow-water velocity fields; S: the spatial HDG operator), with forcing
 * part c_f = A^{-1} F set at setup.
 *   scheme 0, backward Euler:  c <- c_f + H u^n
 *   scheme 1, Crank-Nicolson written as (2/dt) M (u^{n+1} - u^n) + L u^{n+1} + L u^n = 2 f,
 *             i.e. mass_coef = 2/dt:  c <- c_f + 2 H u^n - u^n + G x(u^n)
 * with H = mass_coef A^{-1} M_Phi and G x(u^n) the trace part of one sweep of
 * u^n.  Requires opts.time_stepping = 1 and a shared operator
 * (IHDG_ERR_UNSUPPORTED otherwise).  Stream-ordered.
 */
ihdg_status ihdg_time_step(ihdg_ctx* ctx, int32_t scheme);

/* Change the stream all later work of ctx is ordered on (a hipStream_t). */
ihdg_status ihdg_set_stream(ihdg_ctx* ctx, void* stream);

/* Statistics of the last ihdg_solve: number of FP64 and FP32 sweeps, outer
 * defect-correction steps, Krylov iterations. */
typedef struct {
  int64_t fp64_sweeps;
  int64_t fp32_sweeps;
  int32_t outer_steps;
  int32_t krylov_iters;
  int32_t shared_operator;  /* 1 if one operator is shared by all elements */
  int32_t kernel_waves;     /* waves per workgroup used by the sweep kernel */
} ihdg_stats;
ihdg_status ihdg_get_stats(const ihdg_ctx* ctx, ihdg_stats* out);

/*
 * Batched solves (continuous batching).  A batch advances many contexts
 * together: every round, each member performs up to `sweeps` sweeps of its own
 * solve (the same FP64 iHDG or mixed defect-correction steps as ihdg_solve
 * with check_every = sweeps), and members of the same shape (PDE, dimension,
 * order, operator kind, precision) share one kernel launch per sweep whatever
 * their mesh sizes.  A member's arithmetic does not depend on the other
 * members, so its result is the same alone and in any mix.  Members may join
 * (ihdg_batch_add) between rounds and leave when they finish; finished members
 * are reported by ihdg_batch_poll and their contexts stay valid (the caller
 * reads the solution and destroys them).  All batch work runs on the batch's
 * stream; a member context must not be used elsewhere while it is in the batch.
 *
 * Device memory: ihdg_batch_footprint gives the bytes of `workspace` for at
 * most max_members members whose 64-element blocks total at most max_blocks.
 */
typedef struct ihdg_batch ihdg_batch;
typedef struct {
  int64_t tag;        /* the caller's tag from ihdg_batch_add                      */
  int32_t status;     /* IHDG_OK, IHDG_ERR_DIVERGED or IHDG_ERR_MAXITER            */
  int32_t iters;      /* sweeps done (FP64 + FP32)                                */
  double final_rel;   /* last relative increment (FP64) or FP64 defect (mixed)    */
} ihdg_batch_result;
/* IHDG_ERR_ARG if max_members < 1, max_blocks < 1 or bytes is NULL.  No device work. */
ihdg_status ihdg_batch_footprint(int32_t max_members, int64_t max_blocks, size_t* bytes);
/* workspace: caller-owned device memory, 256-byte aligned, at least the footprint
 * (`bytes`), kept until ihdg_batch_destroy.  stream: the HIP stream of all batch
 * work (NULL: the null stream, whose rounds are never graph-captured).  *out is a
 * library-owned host object.  IHDG_ERR_ARG: NULL or misaligned workspace, NULL
 * out, max_members or max_blocks < 1; IHDG_ERR_NOMEM: bytes below the footprint. */
ihdg_status ihdg_batch_create(int32_t max_members, int64_t max_blocks, void* workspace, size_t bytes, void* stream,
                              ihdg_batch** out);
/* Join the active set from the context's current iterate, to tolerance tol > 0;
 * tag is returned by ihdg_batch_poll.  Resets the context's statistics.
 * IHDG_ERR_ARG: NULL b or ctx, tol <= 0, ctx already a member; IHDG_ERR_NOMEM:
 * max_members members already, or the members' 64-element blocks would exceed
 * max_blocks; IHDG_ERR_UNSUPPORTED: a context set up for a Krylov solve
 * (krylov_restart > 0), which a batch does not advance.  No device work. */
ihdg_status ihdg_batch_add(ihdg_batch* b, ihdg_ctx* ctx, double tol, int64_t tag);
/* One round of `sweeps` >= 1 sweeps (else IHDG_ERR_ARG); n_active (nullable)
 * receives the number of members still active.  Synchronises the batch stream
 * (it reads every member's norms).  A failing HIP call gives IHDG_ERR_HIP, named
 * by ihdg_batch_last_error. */
ihdg_status ihdg_batch_round(ihdg_batch* b, int32_t sweeps, int32_t* n_active);
/* Results of members that finished since the last poll, at most max_out of them
 * into the caller's array out (NULL allowed when max_out is 0); *n_out receives
 * their number, and results beyond max_out stay for the next poll.
 * IHDG_ERR_ARG: NULL b or n_out, or NULL out with max_out > 0. */
ihdg_status ihdg_batch_poll(ihdg_batch* b, ihdg_batch_result* out, int32_t max_out, int32_t* n_out);
/* Rounds replay a HIP graph of their launches (all groups' sweeps and the norm
 * reduction), captured when the round's structure (groups, their block counts,
 * sweeps per round) differs from the previous round's and replayed while it is
 * the same; 1 by default on a non-null stream.  enable = 0: launch directly.
 * The results are the same either way. */
ihdg_status ihdg_batch_use_graphs(ihdg_batch* b, int32_t enable);
/* The HIP call that last failed in a batch call (its name and the runtime's
 * error name), for IHDG_ERR_HIP; "" if none.  Owned by the batch. */
const char* ihdg_batch_last_error(const ihdg_batch* b);
/* Frees the batch object and its captured graph (NULL allowed).  The caller
 * then frees the workspace, and destroys the member contexts itself. */
void ihdg_batch_destroy(ihdg_batch* b);

const char* ihdg_last_error(const ihdg_ctx* ctx);
const char* ihdg_status_string(ihdg_status s);
void ihdg_destroy(ihdg_ctx* ctx);

#ifdef __cplusplus
}
#endif
#endif /* IHDG_H */
