/*
 * helm.h -- C ABI of the MI355X (gfx950) Wave-ADR Helmholtz library (libhelm.so).
 *
 * Problem (paper Section 2, the damped equation and its 5-point discretisation):
 *     A u = -Delta_h u - kappa u = g,  kappa = k^2 n(x)^2 (1 + i sigma (delta(x) + s0)),
 * on a rectangle (the unit square by default; Section 4.3.2 runs the method on
 * non-square domains too) with zero Dirichlet values on the outer ring, where
 * n = 1/c is the slowness, k the angular frequency (the paper's omega) and
 * delta = damping_strength * rho^2 the sponge profile (rho ramps linearly from 0
 * to 1 over damping_cells fine cells towards the boundary, max over the axes).
 * sigma = +1 uses the carrier e^{+i k phi}; sigma = -1 is the paper's printed
 * sign convention (the complex conjugate of every operator).  s0 = 0 unless the
 * shifted equation of Section 4.3.2 is asked for (helm_desc.shift).
 *
 * Grid layout (every array argument): ny rows of n nodes (helm_desc.n columns and
 * helm_desc.ny rows; ny = n, the square, unless set), both powers of two, spacing
 * h = 1/max(n, ny) on both axes, row-major, element (i, j) at offset i*n + j,
 * i = y index, j = x index (x fastest).  Each level halves both sides.
 * Row 0 and column 0 are the Dirichlet ring and must be zero in g and u on
 * entry; the library keeps them zero.  Complex arrays are interleaved
 * (re, im) pairs of float (HELM_C64) or double (HELM_C128), i.e. the memory
 * layout of torch.complex64 / torch.complex128.
 *
 * Ownership: every array argument is caller-owned device memory unless marked
 * "host".  The context owns all workspaces; they are allocated by helm_setup
 * and freed by helm_destroy, except the Krylov bases of helm_solve (allocated by
 * the first solve in each mode) and the adjoint tape and checkpoints (allocated
 * by the first helm_cycle_backward).  helm_cycle allocates nothing.
 *
 * Streams: every call is asynchronous on the given stream (a hipStream_t passed
 * as void*, NULL = default stream), except helm_setup, helm_set_phase (which
 * synchronise once), and helm_solve (which reads one convergence scalar per
 * iteration back to the host).  A context may be used by one thread at a time.
 *
 * Errors: every call returns a helm_status and never aborts; no C++ exception
 * crosses the ABI.  Invalid arguments give HELM_EINVAL and leave outputs
 * untouched; helm_last_error() returns a thread-local description of the last
 * failure.
 */
#ifndef HELM_H_
#define HELM_H_

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct helm_ctx_s* helm_ctx;
typedef struct helm_batch_s* helm_batch;

typedef enum {
    HELM_OK = 0,
    HELM_EINVAL = 1,      /* invalid argument; nothing was done */
    HELM_ENOMEM = 2,      /* device allocation failed */
    HELM_EHIP = 3,        /* a HIP runtime call failed */
    HELM_ENOCONV = 4,     /* solve: tolerance not reached within maxit */
    HELM_EBREAKDOWN = 5,  /* solve: NaN/Inf or residual growth above 1e4 x initial */
    HELM_ESTATE = 6       /* call out of order (e.g. cycle before helm_set_phase) */
} helm_status;

typedef enum { HELM_C64 = 0, HELM_C128 = 1 } helm_prec;

/* Problem and cycle parameters.  Fill with helm_desc_default, then adjust. */
typedef struct {
    int32_t n;                /* nodes per row (x), power of two, 16..8192 */
    int32_t levels;           /* L, 2..log2(min(n, ny))-1; the ADR correction needs L >= 3 */
    double k;                 /* angular frequency, > 0 */
    int32_t damping_cells;    /* sponge width W in fine cells, >= 1 (default 16) */
    double damping_strength;  /* delta = strength * rho^2 (default 0.5) */
    int32_t sign;             /* sigma: +1 (default) or -1 */
    int32_t cycle_prec;       /* helm_prec of the cycle (the coarsest wave level is always FP64) */
    int32_t adr_steps;        /* ADR corrections after the level-2 post-smoother (default 8, 0 = off) */
    int32_t cheb_pre;         /* Chebyshev steps before the coarse correction (default 5) */
    int32_t cheb_post;        /* Chebyshev steps after it (default 5) */
    int32_t cheb_coarse;      /* Chebyshev steps on level L (default 10) */
    int32_t gmres_m;          /* GMRES(m) smoother on ADR levels (default 3) */
    int32_t gmres_coarse_m;   /* GMRES(m) on the coarsest ADR level (default 3) */
    int32_t level3_literal;   /* 0: no smoothing on level 3 (default); 1: Chebyshev post-smoother there */
    int32_t restart;          /* FGMRES restart length (default 20, at most 24) */
    int32_t gmres_arnoldi;    /* 0 (default): GMRES(m <= 4) smoother in s-step form (Krylov basis
                                 rebuilt on tiles, Gram least squares); 1: always Arnoldi */
    int32_t use_graphs;       /* 1 (default): each cycle is captured once per (g, u) pointer pair as a
                                 HIP graph and replayed; 0: kernels are launched one by one */
    int32_t adr_levels;       /* levels of the ADR V-cycle, from level 2 down (default 3; 0 = all, L - 1) */
    int32_t tail_n;           /* a coarsest ADR level with at most tail_n nodes on its longer side (and at most
                                 4096 nodes) runs its GMRES in one workgroup (default 64; 0 = never) */
    int32_t wave_tail_n;      /* the wave levels >= 3 with at most wave_tail_n nodes on the longer side run in
                                 one workgroup, all of them in a single launch (default 32; 0 = never) */
    double shift;             /* relative imaginary shift s0 >= 0 of the shifted equation (Section 4.3.2,
                                 gamma_0 = s0 k(x)^2 with k(x) = k n(x); the paper's test uses 0.01):
                                 kappa = k^2 n^2 (1 + i sigma (delta + s0)); default 0 */
    double cycle_shift;       /* relative imaginary shift >= 0 added to kappa inside the cycle only: the
                                 cycle is then a V-cycle for a complex-shifted operator while the
                                 system (helm_solve's operator, helm_residual, helm_loss) keeps kappa.
                                 With adr_steps = 0 and 0.5 this is the CSL preconditioner of the
                                 paper's comparison (Section 4.3.1); default 0 */
    int32_t ny;               /* rows of nodes (y), power of two, 16..8192, at most 16 times and at
                                 least 1/16 of n; 0 (default) means ny = n.  With ny != n the domain
                                 is the rectangle [0, n h] x [0, ny h], h = 1/max(n, ny) (the
                                 non-square domains of Section 4.3.2) */
} helm_desc;

/* Defaults of every field for an n x n grid at frequency k:
 * levels = min(7, log2 n - 3) (at least 2), W = 16, strength 0.5, sign +1, C128,
 * M = 8, Chebyshev 5/5/10, GMRES(3) on a 3-level ADR V-cycle (s-step form), restart 20,
 * graphs on. */
void helm_desc_default(helm_desc* d, int32_t n, double k);

/* Setup phase (paper Figure "cycle": the solver's setup/solve split).
 * velocity: device, ny*n doubles, c(x) > 0 (n^2 = 1/c^2 on the fine grid, injected
 * to coarse levels).  Computes per-level spectral bounds and the default
 * weights (helm_get_weights).  On success *out owns every workspace. */
helm_status helm_setup(const helm_desc* desc, const double* velocity, helm_ctx* out, void* stream);

/* Phase field of the ADR correction (the paper's tau, Section 3.2; eq. Rytov).
 * phi: device, ny*n, double (phi_is_f64 = 1) or float (0), fine grid.  Builds the
 * ADR coefficients (phase derivatives, reaction term) on levels 2..L and the
 * level-2 carrier.  Required before helm_cycle when adr_steps > 0. */
helm_status helm_set_phase(helm_ctx ctx, const void* phi, int32_t phi_is_f64, void* stream);

/* Wave-Ray phases instead of one phase (the ray functions of the Wave-Ray method, Section 3.2):
 * count plane waves phi_m = nbar (cos theta_m x + sin theta_m y), theta_m = 2 pi m / count,
 * m = 0..count-1, nbar^2 the mean of n^2 over the fine unknowns.  The m-th ADR correction of
 * a cycle (adr_steps of them, 8 for the paper's comparison) solves the ray equation of ray
 * m mod count, eq. ADR with phi_m, by the same ADR V-cycle.  count in 1..64; a later
 * helm_set_phase returns to one phase.  The adjoint supports one phase only. */
helm_status helm_set_rays(helm_ctx ctx, int32_t count, void* stream);

/* Travel-time phase of point sources computed on the device and installed as the
 * phase of the ADR correction (Section 3.2.1, the factored eikonal equation).
 * tau = tau0 tau1 with tau0 = |x - x0| (eq. eikonal_cons) and tau1 the solution
 * of |tau0 grad tau1 + tau1 grad tau0|^2 = s^2 (eq. eikeq), s = sqrt(n^2) from the
 * context's velocity, in the first-order upwind (Godunov) discretisation on the
 * fine nodes with grad tau0 exact; nodes within sqrt(2) h of the source are fixed
 * at tau1 = (s(node) + s(node nearest x0)) / 2.  Solved by fast sweeping: rounds of
 * four Gauss-Seidel passes ((i up, j up), (i up, j down), (i down, j up),
 * (i down, j down)), until the largest single decrease of tau1 in a round is
 * <= tol (tol < 0: exactly max_rounds rounds).  The result equals, bit for bit,
 * the sequential passes computed in IEEE double precision without contraction.
 * src_xy: host, nsrc (x, y) pairs in [0, (n-1) h]^2, 1 <= nsrc <= 64; several
 * sources give the first arrival, the smallest of their travel times.
 * The phase is then installed as by helm_set_phase, except that with one source the
 * ADR coefficients take the phase derivatives from the product rule of Section 3.2.1
 * (grad tau = tau0 grad tau1 + tau1 grad tau0, Lap tau = tau1 Lap tau0 +
 * 2 grad tau0 . grad tau1 + tau0 Lap tau1, the finite-difference rule of the phase
 * applied to tau1; at level nodes closer than one level spacing to the source, to
 * tau itself); that phase has no adjoint (helm_cycle_backward returns HELM_ESTATE).
 * tau1_out, phi_out (device, ny x n doubles, may be NULL): tau1 of the last source
 * and tau.  rounds, change (host, may be NULL): the most rounds run for a source and
 * the largest last-round decrease.  Returns HELM_ENOCONV, leaving the phase
 * unchanged, if a node is still unreached after max_rounds (1..100000).
 * Allocates and frees its own work arrays (about 3 n^2 doubles) and synchronises
 * the stream once per round. */
helm_status helm_eikonal(helm_ctx ctx, const double* src_xy, int32_t nsrc, int32_t max_rounds, double tol,
                         void* tau1_out, void* phi_out, int32_t* rounds, double* change, void* stream);

/* Per-level smoother weights (host, `levels` doubles): w[0] = damped-Jacobi weight
 * of level 1 (Section 3.1.1), w[l-1] = Chebyshev interval parameter alpha_l of
 * level l >= 2 (eq. cheb; interval [lambda_l/alpha_l, lambda_l]).  alpha_l >= 1. */
helm_status helm_set_weights(helm_ctx ctx, const double* w);
helm_status helm_get_weights(helm_ctx ctx, double* w);
/* Upper end lambda_l of the Chebyshev interval (eq. cheb), the Gershgorin bound of the
 * spectrum of A_l^* A_l, (max |4/h_l^2 - kappa_l| + 4/h_l^2)^2 (host out, `levels` doubles). */
helm_status helm_get_lambdas(helm_ctx ctx, double* lam);

/* One Wave-ADR cycle (paper Algorithm 1) on the fine grid: u <- C(u, g).
 * g, u: device, ny*n complex in cycle_prec; u is read and overwritten. */
helm_status helm_cycle(helm_ctx ctx, const void* g, void* u, void* stream);

/* Outer solve to ||g - A u|| / ||g|| < tol (paper Section 4.3.1).
 * g, u: device, ny*n complex128; u holds the initial guess and receives the result.
 * mode 0: FGMRES(restart) in FP64 right-preconditioned by one cycle (cycles in
 *         cycle_prec; cast around the cycle when cycle_prec = HELM_C64).
 * mode 1: FP64 iterative refinement around an FP32 FGMRES(restart) with FP32
 *         cycles (requires cycle_prec = HELM_C64): r = g - A u and u += d in FP64.
 * iters (host out): preconditioner applications; relres (host out): true FP64
 * relative residual at exit; history (host out, may be NULL): maxit+1 doubles,
 * the residual estimate after each iteration.  Returns HELM_ENOCONV if tol was
 * not reached within maxit (iters and relres still filled), HELM_EBREAKDOWN if g or
 * the initial u holds NaN or Inf (nothing is iterated; u is left as given, iters = 0)
 * or if the residual becomes non-finite or grows above 1e4 times its initial value. */
helm_status helm_solve(helm_ctx ctx, const void* g, void* u, double tol, int32_t maxit, int32_t mode,
                       int32_t* iters, double* relres, double* history, void* stream);

/* FP64 residual of the discrete damped equation (Section 2, the 5-point stencil with
 * the sponge term) on the fine grid: r = g - A u (device, complex128, r may be NULL)
 * and its 2-norm plus ||g|| (host out, may be NULL), the quantities of the stopping
 * test ||r|| / ||g|| (Section 4.3.1).  Synchronises the stream. */
helm_status helm_residual(helm_ctx ctx, const void* g, const void* u, void* r, double* rnorm,
                          double* gnorm, void* stream);

/* helm_residual without any allocation, for callers that cannot allocate device memory
 * (code under HIP graph capture, serving loops or harnesses that forbid hipMalloc): the
 * same results bit for bit, with the reduction scratch (per-block partial sums, at most
 * 2 * 2048 doubles, and the two totals) in one static device array per GPU that the
 * library holds until the process ends, instead of the context's workspace.  Calls that
 * overlap on one GPU share that array and race; a call on the same stream after another
 * is safe (every call rewrites the partials it reads).  Every grid the context accepts
 * (n <= 8192) fits; a larger reduction would give HELM_EINVAL.  Synchronises the stream. */
helm_status helm_residual_noalloc(helm_ctx ctx, const void* g, const void* u, void* r, double* rnorm,
                                  double* gnorm, void* stream);

/* Adjoint of K unrolled cycles (Section 3.3: the training loss after K cycles,
 * eq. loss, and its back-propagation; Algorithm 1 reversed).
 *   u_{k+1} = C(u_k, g), k = 0..K-1, from u_0 (device, cycle_prec, NULL = zero).
 *   grad_uK  (device, cycle_prec, ny*n complex): the cotangent of u_K in torch's
 *            convention for complex tensors, dL/dRe(u_K) + i dL/dIm(u_K).
 *   grad_phi (device, ny*n, overwritten): dL/dphi for the fine phase last passed to
 *            helm_set_phase; float for cycle_prec HELM_C64, double for HELM_C128.
 *            The phase enters only through its injection to the ADR levels, so the
 *            entries off the level-2 lattice (odd fine indices) are zero.
 *   grad_w   (device, `levels` doubles, overwritten): dL/dw for the weights of
 *            helm_set_weights (w[0] Jacobi, w[l-1] Chebyshev alpha of level l).
 *   ckpt_ws  device workspace of K*ny*n complex elements in cycle_prec for the
 *            per-cycle checkpoints, or NULL for a library-owned buffer.
 * The call re-runs the K cycles recording each cycle's intermediates on a library-owned
 * tape of its own (about 4 + 4*adr_steps fine-grid vectors per cycle, allocated by the
 * first call that needs them) and keeping u_0..u_{K-1} in the checkpoints, then reverses
 * them.  When the tapes still to be allocated would take more than a quarter of the
 * free device memory or 32 GiB (or the environment variable HELM_ADJ_TAPE_MB, in MiB,
 * when set), one tape is reused: the K cycles run first for the checkpoints and each
 * cycle is recorded again just before its reverse.
 * Requires gmres_m, gmres_coarse_m <= 6 (HELM_EINVAL otherwise) and the phase
 * (HELM_ESTATE otherwise).  Asynchronous on `stream`. */
helm_status helm_cycle_backward(helm_ctx ctx, int32_t K, const void* g, const void* u0,
                                const void* grad_uK, void* grad_phi, double* grad_w, void* ckpt_ws,
                                void* stream);

/* The same adjoint split at the loss (Section 3.3, eq. loss, and Algorithm 1 reversed), for
 * callers that run the K cycles anyway (training: the forward pass records, the backward
 * pass only reverses).
 * helm_cycle_record: u_{k+1} = C(u_k, g), k = 0..K-1, from u_0 (device, cycle_prec, NULL =
 *   zero), each cycle recorded on its own tape; u_K (device, ny*n complex in cycle_prec) to
 *   u_out, which must not overlap g (the reverse reads g again).  ckpt_ws as for
 *   helm_cycle_backward (it must stay untouched until the reverse).
 *   u_out equals the u_K of K helm_cycle calls up to rounding.  Returns HELM_ENOMEM (nothing
 *   run, no tape kept) when the K tapes would exceed the limit of helm_cycle_backward's
 *   one-tape-per-cycle mode; helm_cycle_backward still applies then.
 * helm_cycle_reverse: grad_phi, grad_w from grad_uK exactly as helm_cycle_backward would
 *   give them for the same K, g and u_0, using the tapes of the last helm_cycle_record.
 *   Returns HELM_ESTATE when there are none, when K or g differ from that call's, when the
 *   phase or the weights changed since, or when a helm_cycle_backward rewrote the tapes.
 *   Other calls (helm_cycle, helm_loss, helm_solve) may run in between.  The tapes stay
 *   valid, so one recording can be reversed for several cotangents.
 * Same requirements as helm_cycle_backward.  Both asynchronous on `stream`. */
helm_status helm_cycle_record(helm_ctx ctx, int32_t K, const void* g, const void* u0, void* u_out, void* ckpt_ws,
                              void* stream);
helm_status helm_cycle_reverse(helm_ctx ctx, int32_t K, const void* g, const void* grad_uK, void* grad_phi,
                               double* grad_w, void* stream);

/* Loss of the unrolled cycles (Section 3.3, eq. loss, without the normalisation by
 * ||g||^2): *loss = ||g - A u||^2 accumulated in FP64 from g, u (device, cycle_prec);
 * if grad_u (device, cycle_prec) is not NULL it receives the cotangent
 * -2 A^H (g - A u) in the convention of helm_cycle_backward.  Synchronises the
 * stream (the loss is returned on the host). */
helm_status helm_loss(helm_ctx ctx, const void* g, const void* u, double* loss, void* grad_u,
                      void* stream);

/* Batched solves: nprob independent problems of mixed sizes (the batch dimension of
 * Sections 1 and 4).  desc: host array of nprob descriptors; velocity, phi: host
 * arrays of nprob device pointers (phi may be NULL, or phi[p] NULL, to set the phase
 * later through helm_batch_get + helm_set_phase; phi_is_f64 as in helm_set_phase).
 * lanes: jobs in flight at once (0 = 4), each on its own stream and host thread; a job is
 * a lockstep class (see helm_batch_classes) or one problem.  Problems with equal
 * descriptors in FP32 cycles are grouped into classes of at most 64 and built in one
 * arena.  The contexts are built concurrently; the call returns when all are ready. */
helm_status helm_batch_setup(int32_t nprob, const helm_desc* desc, const double* const* velocity,
                             const void* const* phi, int32_t phi_is_f64, int32_t lanes,
                             helm_batch* out, void* stream);
/* The context of problem p (owned by the batch; valid until helm_batch_destroy). */
helm_status helm_batch_get(helm_batch b, int32_t p, helm_ctx* out);
/* helm_solve of every problem: g, u host arrays of nprob device pointers (complex128
 * n_p*n_p); iters, relres, status: host arrays of nprob outputs.  The lockstep classes
 * (mode 1, helm_batch_classes) and the remaining problems are taken largest first by the
 * lanes; every problem goes through exactly the operations of its single solve, so
 * results equal helm_solve on the same context bit for bit.  Work already queued on
 * `stream` is waited for; the call returns when every problem is done.  Returns
 * HELM_OK if all converged, otherwise the most severe per-problem status. */
helm_status helm_batch_solve(helm_batch b, const void* const* g, void* const* u, double tol,
                             int32_t maxit, int32_t mode, int32_t* iters, double* relres,
                             int32_t* status, void* stream);
/* Lockstep classes of the last helm_batch_solve (host out, nprob): class_of[p] = the class
 * problem p ran in, or -1 if it ran alone.  In mode 1, problems with equal descriptors
 * (FP32 cycles, at most 64 per class) are built region by region in one arena at setup and
 * solved in lockstep: every kernel is launched once for all problems of the class still
 * iterating (gridDim.z of them), each problem keeping its own Krylov scalars, Givens
 * rotations, stopping test and iteration count, so that its result equals its single
 * solve bit for bit.  A class runs in lockstep only while its contexts have one phase and
 * equal launch shapes; otherwise its problems run alone. */
helm_status helm_batch_classes(helm_batch b, int32_t* class_of);
helm_status helm_batch_destroy(helm_batch b); /* NULL-safe */

/* Autotuner of launch shapes (form of the s-step GMRES passes per ADR level: steps
 * per marching unit, or 1 / 2 for overlapped 16 x 16 / 32 x 32 tiles; block count of
 * the outer FGMRES passes), measured with HIP events on this context's own
 * hierarchy filled with hashed data.  The choice is applied to the context and
 * returned as JSON text in json (host, cap bytes; may be NULL):
 *   {"n": .., "levels": .., "prec": "c64"|"c128", "sstep_rows": {"<level>": form, ..},
 *    "fgmres_blocks": blocks, "timings_ms": {..}}
 * Only the split of FP64 partial sums changes, so results change at rounding level.
 * Synchronises the stream; overwrites the ADR work buffers (call it between cycles). */
helm_status helm_tune(helm_ctx ctx, char* json, int64_t cap, void* stream);
/* Applies a tuning JSON from helm_tune (a cached one); unknown keys are ignored,
 * invalid levels, forms (0 = default, 1, 2, or a multiple of 8 in 16..256) or block counts give
 * HELM_EINVAL and change nothing. */
helm_status helm_set_tuning(helm_ctx ctx, const char* json);
/* The tuning in effect (0 = built-in default) as JSON (host, cap bytes). */
helm_status helm_get_tuning(helm_ctx ctx, char* json, int64_t cap);

/* Internal operators, exposed for step-by-step parity tests.  op codes:
 *   1  out = A_l in              (level l, cycle_prec complex)
 *   2  out = R in                (in on level l, out on level l+1)
 *   3  out += P in               (in on level l+1, out on level l)
 *   4  out = Jacobi(in; g=in2)   (level 1)
 *   5  out = Chebyshev(in; g=in2, pre-step count)  (level l >= 2)
 *   6  out = M_l in              (ADR operator, level l >= 2)
 *   7  out = GMRES(M_l; b=in2, x0=in, m=gmres_m)   (level l >= 2)
 *   8  out = ADR V-cycle(b=in2, x0=0) (level l >= 2)
 *   9  out = ADR step(u=in, g=in2) (level 2)
 *  10  out = wave-ADR cycle on level l from (u=in, g=in2); in NULL means u = 0 (on
 *      level 1 this is the zero-start form used as the FGMRES preconditioner; coarser
 *      levels require NULL)
 *  11  out = R(in2 - A_l in)     (fused residual + restriction)
 *  12  out = in                  (plain copy of a level array: a probe of known
 *                                 size for hardware memory counters)
 * Arrays are device memory in cycle_prec (level L arrays are complex128). */
helm_status helm_debug_op(helm_ctx ctx, int32_t op, int32_t level, const void* in, const void* in2,
                          void* out, void* stream);

/* Per-launch kernel timing for measurement (not for use under graph capture).
 * helm_profile_begin starts recording a HIP event pair around every kernel launch
 * of the cycle and solve paths; helm_profile_end synchronises, stops recording and
 * writes a JSON summary into json (host, cap bytes):
 *   {"kernels": [{"name", "launches", "ms" (summed event time), "bytes"
 *                 (algorithmic bytes: each input read once, each output written once)}]}
 * sorted by time.  Returns HELM_EINVAL if cap is too small. */
helm_status helm_profile_begin(helm_ctx ctx);
helm_status helm_profile_end(helm_ctx ctx, char* json, int64_t cap);

/* Frees every workspace; NULL-safe; the context must not be used afterwards. */
helm_status helm_destroy(helm_ctx ctx);

const char* helm_status_string(helm_status s);
const char* helm_last_error(void);

/* Library version string. */
const char* helm_version(void);

#ifdef __cplusplus
}
#endif

#endif /* HELM_H_ */
