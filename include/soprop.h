/*
 * soprop.h -- C ABI of libsoprop, a gfx950 (MI355X) implementation of the
 * composed split-operator propagator for a separable diabatic Hamiltonian
 * H = T(p) + V(q) (Roulet, Choi, Vanicek, arXiv:1903.04946).
 *
 * One time step is the pruned splitting sequence
 *     U(dt) = U_B(b_N dt) U_A(a_N dt) ... U_B(b_1 dt) U_A(a_1 dt)
 * (Sec. "Compositions of split-operator algorithms") of a recursive
 * symmetric composition -- triple jump or Suzuki's fractal -- of the
 * second-order VTV or TVT algorithm (Eqs. so_VTV, so_TVT, second_order_so;
 * Sec. "Symmetric composition schemes"), after pruning zero coefficients and
 * merging neighbouring A actions (Eq. merging_splitting_coeff_b_zero), with
 * one stored evolution-operator table per unique coefficient and integer
 * index arrays into them (Eq. range_index_unq, Table II).  Each kinetic action
 * is forward FFT -> phase exp(-i tau T(p)/hbar) -> inverse FFT, each potential
 * action the S x S unitary exp(-i tau V(q)/hbar) at every grid point
 * (Sec. "Dynamic Fourier method", Eq. diab_mol_ham), obtained from a Jacobi
 * eigen-decomposition of V(q) (Sec. "Molecular Hamiltonian in the diabatic
 * basis").
 *
 * Conventions
 *   - Units: any consistent set; hbar is a plan parameter (1 in atomic units).
 *   - Grid: ndim in {1, 3}; periodic box [lo_d, hi_d), n_d points,
 *     dx_d = (hi_d - lo_d)/n_d.  Momenta p = hbar * 2 pi k'/(n_d dx_d) with
 *     k' = k for k < n_d/2 and k - n_d otherwise.
 *   - Wavefunction psi: caller-owned DEVICE memory, C-contiguous
 *     [nsurf][n_0]..[n_{ndim-1}] (last axis fastest), interleaved complex
 *     (complex128 for SOP_C128 plans, complex64 for SOP_C64 plans).
 *   - V-table: caller-owned HOST memory, double, the packed upper triangle of
 *     the real symmetric S x S potential per grid point in the order
 *     V00, V01, .., V0,S-1, V11, V12, .., VS-1,S-1; array
 *     [nsurf*(nsurf+1)/2][npts], points flattened like psi.  The library
 *     copies it; the caller may free it after sop_plan_create returns.
 *   - Kinetic energy T(p) = sum_d inv_mass[d] p_d^2 / 2.
 *
 * Streams and synchronisation
 *   All device work is enqueued on the HIP stream given at plan creation
 *   (NULL = the default stream).  sop_propagate and sop_interpolate are
 *   asynchronous.  sop_plan_create, sop_plan_update_v, sop_plan_set_params,
 *   sop_observables, sop_overlap, sop_distance, sop_apply_action,
 *   sop_propagate_driven, sop_propagate_trapezoid, the adjoint calls,
 *   sop_timing_read, sop_batch_create and sop_plan_destroy synchronise the
 *   stream before returning.
 *
 * Errors
 *   Every call returns a sop_status.  Arguments are validated before any
 *   device work: on SOP_ERR_INVALID or SOP_ERR_UNSUPPORTED nothing is
 *   touched.  On SOP_ERR_HIP the HIP error text is available from
 *   sop_last_error() and psi is undefined.  Out-parameters are written only
 *   on SOP_OK.  A plan is not thread-safe; distinct plans are.
 */
#ifndef SOPROP_H
#define SOPROP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SOP_ABI_VERSION 3

typedef enum {
  SOP_OK = 0,
  SOP_ERR_INVALID = 1,     /* malformed argument (null pointer, bad size, ...) */
  SOP_ERR_UNSUPPORTED = 2, /* valid but not implemented (e.g. a grid length)  */
  SOP_ERR_NOMEM = 3,       /* device allocation failed                        */
  SOP_ERR_HIP = 4,         /* a HIP runtime call failed                       */
  SOP_ERR_STATE = 5        /* call not allowed in the plan's current state    */
} sop_status;

/* Elementary splitting (Eqs. so_VT, so_TV, so_VTV, so_TVT).  A is the
 * operator applied first: VTV and TV apply V first, TVT and VT apply T
 * first.  VT/TV are first order and take no composition (order 1). */
typedef enum { SOP_SPLIT_VTV = 0, SOP_SPLIT_TVT = 1, SOP_SPLIT_VT = 2, SOP_SPLIT_TV = 3 } sop_split;

/* Composition scheme (Sec. "Symmetric composition schemes"): Strang (the
 * bare second-order method, order 2), recursive triple jump (M = 3^n Strang
 * stages for order 2(n+1)), Suzuki's fractal (M = 5^n), or a custom
 * symmetric composition whose M coefficients the caller gives (the
 * non-recursive "optimal" schemes the paper cites, whose coefficients it does
 * not print, are of this kind: Table II lists their sequence lengths). */
typedef enum {
  SOP_COMP_STRANG = 0,
  SOP_COMP_TRIPLE_JUMP = 1,
  SOP_COMP_SUZUKI = 2,
  SOP_COMP_CUSTOM = 3
} sop_comp;

typedef enum { SOP_C128 = 0, SOP_C64 = 1 } sop_dtype;

typedef struct {
  int ndim;        /* 1 or 3 */
  int n[3];        /* points per axis; supported lengths listed by sop_supported_length */
  double lo[3];
  double hi[3];
} sop_grid;

typedef struct {
  sop_grid grid;
  int nsurf;              /* S: 1..2 for ndim = 1, 1..3 for ndim = 3 */
  const double* inv_mass; /* [ndim] host, 1/m_d (Eq. diab_mol_ham, diagonal mass matrix) */
  const double* vtable;   /* host, packed upper triangle, see above */
  sop_split split;
  sop_comp comp;
  int order;              /* 1 for VT/TV; 2 (Strang) or 4, 6, 8, 10 */
  double dt;              /* time step, nonzero, finite */
  double hbar;            /* > 0 */
  sop_dtype dtype;
  /* Optional parameters theta_k of a potential linear in them,
   * V(theta) = vtable + sum_k theta_k dvtables[k] (vtable is V at theta = 0),
   * for sop_plan_set_params and the adjoint.  nparams = 0 and dvtables = NULL
   * when unused; at most 8.  dvtables: host, [nparams][S(S+1)/2][npts]. */
  int nparams;
  const double* dvtables;
  /* SOP_COMP_CUSTOM only (0 and NULL otherwise): gamma[ngamma] host, the
   * composition coefficients gamma_1..gamma_M of the Strang stages, applied
   * as U(dt) = S(gamma_M dt) ... S(gamma_1 dt).  They must be finite and
   * nonzero, sum to one (to 1e-12) and be symmetric, gamma_j = gamma_{M+1-j}
   * (to 1e-14 of the largest |gamma|; the mirrored half is taken from the
   * first), 1 <= M <= 625.  `order` then states the scheme's order (even,
   * >= 2); the library does not check it.  The plan copies gamma. */
  int ngamma;
  const double* gamma;
} sop_plan_desc;

/* Sizes of a plan (Table II quantities for its scheme and order). */
typedef struct {
  int M;          /* Strang stages per step = number of B actions N_B       */
  int n_a;        /* A actions per step after pruning (M+1; 1 for VT/TV)    */
  int n_b;        /* B actions per step                                     */
  int n_a_unq;    /* unique A coefficients                                  */
  int n_b_unq;    /* unique B coefficients                                  */
  int n_v_tables; /* stored potential tables (= n_a_unq if A = V; 1 for the eigen form) */
  int n_t_tables; /* stored kinetic factor sets                             */
  int64_t npts;
  size_t table_bytes;   /* device bytes of stored evolution operators      */
  size_t scratch_bytes; /* device bytes of observables scratch             */
} sop_plan_info;

typedef struct sop_plan sop_plan;

/* ABI version (SOP_ABI_VERSION of the built library). */
int sop_abi_version(void);

/* Static text for a status code. */
const char* sop_status_string(sop_status s);

/* Detail of the last failure on the calling thread ("" if none). */
const char* sop_last_error(void);

/* 1 if a grid length n is supported on a 1D (ndim = 1) or 3D axis. */
int sop_supported_length(int ndim, int n);

/* Composition coefficients and the pruned, deduplicated sequence, computed
 * on the host only (no device needed).  Sec. "Symmetric composition schemes",
 * Sec. "Pruning splitting coefficients", Eq. range_index_unq.
 *   a, b        : [cap] out, the pruned sequence (a_1..a_N, b_1..b_N; the
 *                 trailing b_N = 0 of a composed method is included)
 *   a_unq, b_unq: [cap] out, the unique nonzero values (first occurrence)
 *   ia, ib      : [cap] out, 0-based indices into a_unq/b_unq; ib = -1 where b = 0
 *   counts      : [4] out = {N, n_a_unq, n_b_unq, M}
 * Any array pointer may be NULL to skip it.  SOP_ERR_INVALID if cap < N. */
sop_status sop_scheme_sequence(sop_split split, sop_comp comp, int order, int cap, double* a,
                               double* b, double* a_unq, double* b_unq, int* ia, int* ib,
                               int* counts);

/* The same for a custom symmetric composition (SOP_COMP_CUSTOM): gamma[ngamma]
 * host, validated as for sop_plan_desc.gamma; split is VTV or TVT.
 * sop_scheme_sequence refuses comp = SOP_COMP_CUSTOM. */
sop_status sop_custom_sequence(sop_split split, int ngamma, const double* gamma, int cap,
                               double* a, double* b, double* a_unq, double* b_unq, int* ia,
                               int* ib, int* counts);

/* Builds a plan: validates, computes the sequence on the host, uploads the
 * V-table and forms the unique potential tables exp(-i c dt V/hbar) on the
 * device (FP64 formation, rounded once to complex64 for SOP_C64 plans), plus
 * per-axis kinetic factors and FFT twiddles.  3D FP64 plans of two or three
 * surfaces store instead one compact eigen form of V per point (the rotation
 * of its Jacobi diagonalisation and its eigenvalues, 32 or 64 bytes), from
 * which each potential action forms exp(-i tau lam) in FP64; they do so when
 * every phase |tau lam| (bounded by the Gershgorin row sums of the V-table)
 * stays within 1e6, and keep the per-coefficient tables otherwise.
 * SOP_C64 plans keep each twiddle and kinetic factor as its FP32 rounding
 * plus the rounding residue, which their products fold in: a fixed rounded
 * unit-modulus factor would otherwise bias the norm the same way at every
 * substep.
 * hip_stream: a hipStream_t or NULL.  Synchronises the stream.  *out
 * receives the plan. */
sop_status sop_plan_create(const sop_plan_desc* desc, void* hip_stream, sop_plan** out);

/* Device memory hooks for a plan: alloc(ctx, bytes, stream) returns device
 * memory usable on `stream` (NULL on failure), free(ctx, ptr, stream) takes
 * it back; `stream` is the hip_stream given at creation.  With hooks, every
 * device buffer the plan owns -- tables, factors, programs, reduction and
 * scratch space -- comes from alloc and goes back through free when the
 * plan is destroyed (after sop_plan_destroy has synchronised the plan's
 * stream), so that a framework's caching allocator (PyTorch's) owns the
 * memory.  Batches and HIP graph objects keep their own small allocations. */
typedef struct {
  void* ctx;
  void* (*alloc)(void* ctx, size_t bytes, void* stream);
  void (*free)(void* ctx, void* ptr, void* stream);
} sop_allocator;

/* sop_plan_create with device memory from `allocator` (NULL: hipMalloc, the
 * same as sop_plan_create).  SOP_ERR_INVALID if only one hook is set;
 * SOP_ERR_NOMEM if alloc returns NULL.  The hooks must stay callable until
 * sop_plan_destroy returns. */
sop_status sop_plan_create_with_allocator(const sop_plan_desc* desc, void* hip_stream,
                                          const sop_allocator* allocator, sop_plan** out);

/* Frees the plan's device memory.  NULL is accepted. */
sop_status sop_plan_destroy(sop_plan* plan);

sop_status sop_plan_info_get(const sop_plan* plan, sop_plan_info* out);

/* Rebinds the plan to another stream (NULL = default). */
sop_status sop_plan_set_stream(sop_plan* plan, void* hip_stream);

/* psi <- U(direction * dt)^nsteps psi, in place, on the plan's stream.
 * direction = -1 applies the same sequence with every table conjugated,
 * i.e. U(-dt) (time reversal; Sec. "Geometric properties of the exact
 * evolution operator").  nsteps = 0 is a no-op.  Asynchronous. */
sop_status sop_propagate(sop_plan* plan, void* psi_dev, int64_t nsteps, int direction);

/* Propagates count independent states of this plan stored contiguously,
 * psi_dev = [count][nsurf][n...], each as sop_propagate does (1D: one
 * launch, one persistent workgroup per state; 3D: the states in turn).
 * count in 1..65535.  Asynchronous. */
sop_status sop_propagate_many(sop_plan* plan, void* psi_dev, int count, int64_t nsteps,
                              int direction);

/* Observables of psi in FP64 (Sec. "Geometric properties of the exact
 * evolution operator"): out[0] = <psi|psi>, out[1] = <psi|H|psi>,
 * out[2+s] = population of surface s (s < nsurf), out[2+S] = <T>,
 * out[3+S] = <V>.  Inner products carry the volume element.  <T> is taken
 * in the momentum representation from an FFT of a scratch copy; psi is not
 * modified.  out must hold 4 + nsurf doubles (host).  Synchronises. */
sop_status sop_observables(sop_plan* plan, const void* psi_dev, double* out);

/* <psi|phi> with the volume element; out[0] = Re, out[1] = Im (host).
 * The symplectic two-form is -2 hbar Im<psi|phi>.  Synchronises. */
sop_status sop_overlap(sop_plan* plan, const void* psi_dev, const void* phi_dev, double* out);

/* L2 distance between two states of the plan's shape and dtype:
 * out[0] = ||psi - phi|| = sqrt(sum |psi - phi|^2 dV), out[1] = ||psi - phi|| /
 * ||phi|| (0 when phi = 0); host, [2].  The error norm of the convergence
 * studies (Sec. "Numerical examples"), formed from the difference in FP64
 * (the expansion through sop_overlap would cancel when the states agree
 * closely).  Fixed-order reduction; synchronises. */
sop_status sop_distance(sop_plan* plan, const void* psi_dev, const void* phi_dev, double* out);

/* Applies one action to psi (testing aid): op = 0 potential
 * exp(-i tau V/hbar) with tau = coef * dt, op = 1 kinetic exp(-i tau T/hbar).
 * The table for coef is formed on the fly into the plan's scratch (allocated
 * on first use).  Synchronises the stream before returning (its host staging
 * buffers must outlive the copies). */
sop_status sop_apply_action(sop_plan* plan, void* psi_dev, int op, double coef);

/* Times of the potential actions of one step, in units of dt from the
 * step's start (host, [count]): the kinetic actions advance time and the
 * potential actions act at an instant, so for VTV c_v = b_1 + .. + b_{v-1}
 * (Sec. "Compositions of split-operator algorithms": the sequence U_B(b_N dt)
 * U_A(a_N dt) .. U_A(a_1 dt)).  Sampling a drive s(t) at t0 + (n + c_v) dt
 * keeps the composition's order for a time-dependent potential.  c may be
 * NULL to query count; SOP_ERR_INVALID if cap < count. */
sop_status sop_action_times(const sop_plan* plan, double* c, int cap, int* count);

/* Driven propagation with V(x, t) = V(x) + s D(x), D the plan's one
 * parameter table (dvtables[0]) and V the table at theta = 0: the v-th
 * potential action of step n uses s = drive[n * count + v] (host,
 * [nsteps][count], count from sop_action_times).  A time-dependent operator
 * is formed on the fly (Sec. "Pruning splitting coefficients"): before
 * every potential action the library forms V + s D and its exponential
 * (the eigen form, or the one table that action reads) on the device, and
 * the actions run one at a time, eagerly.  Afterwards the plan's tables
 * are those of its current parameter again.  Synchronises.
 * SOP_ERR_STATE unless the plan has exactly one parameter table;
 * SOP_ERR_INVALID for a NULL or non-finite drive; SOP_ERR_UNSUPPORTED if
 * the plan holds the eigen form and the drive could take a phase beyond its
 * range (then nothing changes). */
sop_status sop_propagate_driven(sop_plan* plan, void* psi_dev, int64_t nsteps,
                                const double* drive);

/* Replaces the plan's V-table (host FP64, [S(S+1)/2][npts], the layout of
 * sop_plan_desc.vtable) and forms the potential tables again on the device,
 * in the same buffers, so captured graphs and batches that hold the plan stay
 * valid.  For a plan with parameters the new table is V at theta = 0 and the
 * current theta applies on top of it.  The unitaries exp(-i tau V) of the
 * sequence are tables of V (Sec. "Pruning splitting coefficients": formed
 * once, reused by every step); this forms them for another V of the same
 * grid and surfaces.  Synchronises.  SOP_ERR_INVALID for a NULL or
 * non-finite table; SOP_ERR_UNSUPPORTED if the plan holds the eigen form and
 * the new V could take a phase |tau lam| beyond its range (then nothing
 * changes). */
sop_status sop_plan_update_v(sop_plan* plan, const double* vtable);

/* Sets the parameters: V <- vtable + sum_k theta[k] dvtables[k], and forms the
 * potential tables again on the device (theta: host, [nparams]).
 * Synchronises.  SOP_ERR_STATE if the plan has no parameters;
 * SOP_ERR_UNSUPPORTED if the plan holds the eigen form and theta could take
 * a phase |tau lam| beyond its range (then nothing changes). */
sop_status sop_plan_set_params(sop_plan* plan, const double* theta);

/* Adjoint (reverse-mode) derivatives of the final surface populations
 * P_s(T) = ||psi_s(T)||^2 dV with respect to the plan's parameters, for
 * FP64 plans on 3D grids of 32, 64, 128 or 256 points per axis.
 *
 * The gradient of L = sum_s w_s P_s is 2 dV sum_j Re <lambda_j| dU_j/dtheta_k
 * |psi_{j-1}> over the potential actions j, with lambda_j = (U_N..U_{j+1})^dag
 * W psi_T (Sec. "Geometric properties of the exact evolution operator": the
 * propagator is unitary, so U^dag = U^{-1} = U(-dt), conjugated tables).
 * The backward sweep applies U_j^dag to lambda and to psi together, so psi
 * is recomputed by time reversibility (symmetric compositions are exactly
 * reversible, Appendix A) instead of stored; every K steps the stored
 * forward state replaces the recomputed one (checkpoints).  dU_j/dtheta_k
 * is the Frechet derivative of exp(-i tau V) in direction dvtables[k], in
 * the divided-difference (Daleckii-Krein) form in V's eigenbasis.
 *
 * Workspace: caller-owned device memory of sop_adjoint_workspace_bytes
 * bytes; it holds psi(T) (its first S*npts complex values), lambda, the
 * gradient accumulator and ceil(nsteps/K) checkpoints. */
sop_status sop_adjoint_workspace_bytes(const sop_plan* plan, int64_t nsteps, int K,
                                       size_t* bytes);
/* Forward sweep from psi0_dev (not modified): propagates nsteps steps in the
 * workspace, storing checkpoints, and writes P_s(T) to pops_out[S] (host).
 * Synchronises. */
sop_status sop_adjoint_forward(sop_plan* plan, const void* psi0_dev, int64_t nsteps, int K,
                               void* workspace_dev, double* pops_out);
/* Backward sweep after sop_adjoint_forward with the same nsteps and K:
 * grad_out[k] = sum_s weights[s] dP_s/dtheta_k (host arrays [S], [nparams]).
 * Synchronises.  The workspace's psi is consumed. */
sop_status sop_adjoint_backward(sop_plan* plan, int64_t nsteps, int K, const double* weights,
                                void* workspace_dev, double* grad_out);

/* Both sweeps in one call: pops_out [S] = P_s(T) from the forward sweep,
 * grad_out [nparams] = sum_s weights[s] dP_s/dtheta_k from the backward one
 * (host arrays; the workspace as for sop_adjoint_forward).  Synchronises;
 * out-parameters are written only on SOP_OK. */
sop_status sop_adjoint(sop_plan* plan, const void* psi0_dev, int64_t nsteps, int K,
                       const double* weights, void* workspace_dev, double* pops_out,
                       double* grad_out);

/* Plan options.  SOP_OPT_GRAPHS (default 1): on 3D grids, runs of 4 or more
 * steps launch the first step, the steady step (replayed) and the final
 * pass as HIP graphs captured once per state pointer, direction and count,
 * and the trapezoidal rule launches its iterations in captured blocks of
 * four (once per state pointer and stage coefficient); 0 launches every
 * pass eagerly.  SOP_OPT_PLANE_PASS: on 3D grids whose xy
 * plane fits in LDS (n <= 64 in FP64, n <= 128 in FP32) the y- and x-passes
 * of a kinetic action run as one plane pass; default 1 for n <= 64, 0 for
 * larger grids.  Every setting gives bitwise identical results.
 * SOP_OPT_QUEUE and SOP_OPT_QUEUE_SPIN are options of batches only
 * (sop_batch_set_option); a plan refuses them. */
enum { SOP_OPT_GRAPHS = 1, SOP_OPT_PLANE_PASS = 2, SOP_OPT_QUEUE = 3, SOP_OPT_QUEUE_SPIN = 4 };
sop_status sop_plan_set_option(sop_plan* plan, int option, int value);

/* Compositions of the trapezoidal rule (the implicit, unitary and
 * energy-conserving comparison integrator of the paper's figures; for a
 * linear equation the trapezoidal rule and the implicit midpoint rule are the
 * same map).  Each of the plan's composition stages g_j solves
 * (1 + i tau H) psi' = (1 - i tau H) psi, tau = g_j dt / (2 hbar), with
 * H = T + V of the plan (its current V-table) and T(k) = hbar^2 kappa^2
 * inv_mass / 2 on the grid's frequencies.  The solve is the conjugate
 * orthogonal conjugate gradient method for the complex symmetric matrix
 * 1 + i tau H, started from psi, stopped when the residual's norm falls to
 * tol times the right-hand side's (the error of psi' is then at most that
 * residual), at most max_iter iterations per stage.
 * SOP_C128 plans only (SOP_ERR_UNSUPPORTED otherwise): 1D of 512..8192
 * points, each state in one workgroup for the whole call; or 3D, one state
 * after another, the iterations enqueued from the host with H u = the
 * three one-axis kinetic terms F_d^-1 T_d F_d u (the propagator's pass
 * kernels) plus V u, every reduction in a fixed order, the method's scalars
 * kept on the device and read back every few iterations (the iterate stays
 * frozen from the iteration that meets tol, so the result does not depend
 * on when the host looks).  VT/TV plans have no composition
 * (SOP_ERR_INVALID).  psi:
 * device [count][S][grid], count (1..65535) independent states, advanced in
 * place by nsteps steps.  *iterations (may be NULL) receives the total
 * iteration count over all states.  Synchronises the plan's stream;
 * SOP_ERR_STATE if a stage did not reach tol (psi then holds the last
 * iterate).  Keeps a workspace (1D: count S N complex values; 3D: six
 * state-sized vectors) grown on demand in the plan. */
sop_status sop_propagate_trapezoid(sop_plan* plan, void* psi, int count, int64_t nsteps,
                                   double tol, int max_iter, int64_t* iterations);

/* For callers that cannot allocate device memory (tight serving loops,
 * harnesses that forbid hipMalloc): sop_propagate_trapezoid with the same
 * arguments, kernel and results (bitwise), whose workspace is a static
 * device array of SOP_TRAP_SCRATCH_BYTES (32 MiB) that every GPU the library
 * runs on holds until the process ends, instead of plan memory grown on
 * demand.  The call allocates nothing (no hipMalloc, hipFree or allocating
 * library routine); it needs (1D) count * nsurf * N * 16 bytes of residuals
 * plus 24 bytes of statistics per state (rounded up to 256) and 8 bytes per
 * composition stage, or (3D) six vectors of nsurf * npts * 16 bytes plus
 * about 33 KB, and returns SOP_ERR_INVALID, before any device work, if that
 * exceeds the array (e.g. at most 1023 states of 1024 points and two
 * surfaces; 3D grids up to 32^3 x 3).  Every call on one GPU shares that
 * GPU's array: calls that
 * overlap on one GPU (other streams, other host threads) race and must be
 * serialised by the caller.  Nothing in the array needs clearing between
 * calls.  Synchronises the plan's stream. */
#define SOP_TRAP_SCRATCH_BYTES ((size_t)32 << 20)
sop_status sop_propagate_trapezoid_noalloc(sop_plan* plan, void* psi, int count, int64_t nsteps,
                                           double tol, int max_iter, int64_t* iterations);

/* Trigonometric interpolation of a state onto another grid (Appendix B:
 * states on grids of different range and density are compared through the
 * trigonometric interpolant of the one on the sparser grid).  psi_dst
 * (dst's grid, layout [S][grid]) receives, on every surface and at every
 * point of dst's grid, the value of psi_src's interpolant: along each axis
 * sum over |k| < n/2 of c_k exp(2 pi i k xi), c_k the DFT coefficients of the
 * samples divided by n, xi = (x - lo)/(hi - lo) of src's grid, plus for even
 * n the Nyquist term c_{n/2} cos(pi n xi); points outside src's [lo, hi)
 * receive zero.  Equal grids give psi_dst = psi_src up to rounding.
 * Both plans need the same ndim and nsurf and SOP_C128 (SOP_ERR_UNSUPPORTED
 * otherwise); their lengths and boxes may differ freely (destination axes up
 * to 65535 points).  psi_src and psi_dst are device buffers and must differ.
 * Runs asynchronously on dst's stream (psi_src must be ready there); the
 * axis matrices and intermediate states live in a workspace that dst keeps
 * and grows on demand (16 bytes per matrix entry and per intermediate
 * element; growing it synchronises dst's stream), released with dst.  The
 * matrices are formed on the first call and again only when the source
 * grid (lengths and box) differs from the previous call's. */
sop_status sop_interpolate(const sop_plan* src, const void* psi_src, sop_plan* dst,
                           void* psi_dst);

/* Per-kernel timing (measurement aid).  While enabled, every kernel launch
 * of the plan is bracketed by HIP events on the plan's stream, and
 * consecutive launches within one call share their boundary event (so the
 * intervals of a propagate call tile its wall time).  Graph capture is off
 * while timing is on.  sop_timing_read synchronises the stream and returns, per kernel kind
 * (SOP_KIND_*), the summed event time in ms, the launch count and the summed
 * algorithmic bytes (state read + written, tables read; for SOP_KIND_INTERP,
 * the products of sop_interpolate, FP64 flops instead), then clears the
 * records.  ms, counts, bytes: host arrays of SOP_KIND_COUNT entries. */
enum { SOP_KIND_ZPASS = 0, SOP_KIND_YPASS = 1, SOP_KIND_XPASS = 2, SOP_KIND_1D = 3,
       SOP_KIND_OTHER = 4, SOP_KIND_PLANE = 5, SOP_KIND_INTERP = 6, SOP_KIND_COUNT = 7 };
sop_status sop_plan_set_timing(sop_plan* plan, int enable);
sop_status sop_timing_read(sop_plan* plan, double* ms, int64_t* counts, double* bytes);

/* ------------------------------------------------------------------ batches
 * A batch propagates many independent plans -- any mix of 1D and 3D grids,
 * surfaces, precisions, compositions, orders and dt -- with one HIP graph
 * launch per call.  Members are grouped by the kernel that runs them
 * together: 1D members of one (grid length, surfaces, precision) family run
 * in one persistent launch, one workgroup per member for its whole run;
 * 3D members on 32^3, 48^3 or 64^3 grids with a VTV program form one
 * (n, surfaces, precision) group each, run as lockstep pass launches (one
 * launch per pass and cycle over the members still running, each member
 * with its own tables, coefficients and step count; the members cut into
 * chains of similar cycle counts on separate branches) or, with
 * SOP_OPT_QUEUE, as one persistent work-queue launch per group: its
 * workgroups (four waves each, about occupancy x compute units of them)
 * take items of four z-, y- or x-pass tiles of one member in an order fixed
 * on the host (pass by pass, the longest-running members first), and an
 * item starts once its member's counter of finished items shows the
 * member's previous pass complete (Sec. "Dynamic Fourier method": each pass
 * transforms whole pencils of the state the previous pass wrote); any other
 * member runs its own plan's executor in a branch of the same graph.  The
 * per-member arithmetic is that of sop_propagate (3D members: bitwise the
 * same result; 1D members: the same DFTs, possibly in another radix order,
 * so equal up to rounding).
 *
 * sop_batch_create: plans[0..count) (1 <= count <= 65535; a plan may appear
 * more than once; the batch keeps pointers, so the plans must outlive it)
 * and the HIP stream that propagate calls run on.  It times the schedule
 * variants of each family (values per thread and radix order) and the tile
 * widths of each lockstep group's z, y and x passes on scratch states with
 * the members' own tables, and keeps the fastest.  Environment:
 * SOPROP_TUNE=0 keeps the default variants; SOPROP_TUNE_CACHE=<path> reads
 * the choices from, and records new ones in, a JSON file of "key": "variant"
 * pairs.  Synchronises the stream.
 *
 * sop_batch_propagate: psi_devs[i] is member i's state (device memory, the
 * layout and dtype of plans[i]; states must not overlap), nsteps[i] >= 0 its
 * step count, direction +1 or -1 for all members.  Asynchronous on the
 * batch's stream.  The graph is captured on the first call and replayed
 * while psi_devs, nsteps and direction stay the same; a call that changes
 * them synchronises the stream once to rewrite the member descriptors.
 * Runs longer than 200000 kernel launches are enqueued without a graph.
 *
 * sop_batch_set_option(SOP_OPT_GRAPHS, 0) enqueues the branches directly;
 * SOP_OPT_QUEUE 1 runs the 3D groups as work-queue launches (default 0:
 * lockstep launches, which measure faster on the ensembles tried: every
 * claim and completion of a queue item is an atomic on one address and
 * every item pays an L2 write-back and invalidation to make its stores
 * visible across the chip's L2 caches); SOP_OPT_PLANE_PASS 0 keeps separate
 * y- and x-passes in the lockstep launches (the queue always runs y- and
 * x-passes); SOP_OPT_QUEUE_SPIN (value >= 1, default 2^21) bounds the polls
 * of one wait in a queue launch.  Every setting gives the same results: 3D
 * members bitwise those of sop_propagate.
 *
 * sop_batch_check synchronises the batch's stream and returns
 * SOP_ERR_STATE if a queue launch since the last check ran a wait out of
 * polls (every workgroup then leaves and the members' states are left
 * part-propagated; a wait normally lasts microseconds, so only a fault
 * elsewhere or a tiny SOP_OPT_QUEUE_SPIN makes one run out), SOP_OK
 * otherwise.
 *
 * sop_batch_describe writes a NUL-terminated JSON description (families,
 * groups, chosen variants, tuning times in ms, branch count, whether the
 * last call used a graph) into buf[0..len) (truncated if short; buf may be
 * NULL) and the size it needs, NUL included, into *needed (may be NULL). */
typedef struct sop_batch sop_batch;
sop_status sop_batch_create(sop_plan* const* plans, int count, void* hip_stream,
                            sop_batch** out);
sop_status sop_batch_destroy(sop_batch* batch);
sop_status sop_batch_propagate(sop_batch* batch, void* const* psi_devs, const int64_t* nsteps,
                               int direction);
sop_status sop_batch_set_option(sop_batch* batch, int option, int value);
sop_status sop_batch_check(sop_batch* batch);
sop_status sop_batch_describe(const sop_batch* batch, char* buf, size_t len, size_t* needed);

#ifdef __cplusplus
}
#endif

#endif /* SOPROP_H */
