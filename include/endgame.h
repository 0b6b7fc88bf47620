/*
 * endgame.h — C ABI of the MI355X (gfx950) library that solves the Helmholtz
 * pressure-correction system  A x = b  of the ENDGame dynamical core.
 *
 * Paper: C. M. Maynard and D. N. Walters, "Precision of the ENDGame: Mixed-precision
 * arithmetic in the iterative solver of the Unified Model" (arXiv:1811.03852).
 *
 *   Sec. 1, Eq. 1        the linear system A x = b (x: pressure correction, b: forcing).
 *   Sec. 2, Eq. 4        A is the Schur-complement Helmholtz matrix: 7-band, non-symmetric,
 *                        variable coefficient, recomputed every time step.
 *   Sec. 2, Eq. 5        right ("post-") preconditioned BiCGStab on the diagonally scaled
 *                        system; the scaling is applied outside the solver (by the caller).
 *   Sec. 2, Eq. 6-7      T, the vertical tridiagonal part of A, inverted per column with no
 *                        vertical decomposition.
 *   Sec. 3, Eq. 8-9      halting on R = ||b - A x_i|| / ||b|| < R_c.
 *   Sec. 3, Eq. 10       32-bit arithmetic is adequate while R_c >> eps_32.
 *   Sec. 4               64-bit global sums, breakdown of near-zero scalar weights, and a
 *                        mandatory restart after a fixed number of iterations.
 *
 * General conventions
 *   - Every array argument is a DEVICE pointer (for example torch.Tensor.data_ptr() of a
 *     CUDA/HIP tensor) unless the comment says "host".  The caller owns every array it
 *     passes; the library never frees caller memory and keeps no pointer to it after a call
 *     returns.  The library owns the operator object and all its internal buffers.
 *   - Grid layout of every field: idx = i + nlon * (j + nlat * k), i = longitude (fastest,
 *     periodic), j = latitude (south to north), k = level (bottom to top).  n = nlon*nlat*nlev.
 *   - All device work is ordered on the operator's stream (eg_set_stream; default: the null
 *     stream).  Every call has completed on the device when it returns.
 *   - Return values: >= 0 is a numerical outcome (enum eg_status), < 0 an error.  On error
 *     eg_last_error() returns a message (thread-local).  No C++ exception crosses the ABI.
 *   - An operator object must not be used from two threads at once.
 */
#ifndef ENDGAME_H
#define ENDGAME_H

#ifdef __cplusplus
extern "C" {
#endif

typedef struct eg_operator eg_operator;

/* Solver modes (argument `mode` of eg_solve). */
enum eg_mode {
    EG_FP64 = 0,            /* BiCGStab in FP64, T^{-1} preconditioner (Sec. 2)                  */
    EG_FP32_IR = 1,         /* FP64 iterative refinement around an FP32 inner BiCGStab; FP64     */
                            /* true residual, solution update and dot-product accumulation       */
                            /* (Sec. 3-4: x kept in 64-bit, the rest 32-bit, 64-bit global sums) */
                            /* A refinement step that does not reduce the true residual is       */
                            /* undone, and so is the refinement when it stagnates: the solve     */
                            /* then continues from x with the EG_FP64 solver (info.fallbacks).   */
    EG_FP32_IR_BF16 = 2,    /* as EG_FP32_IR, inner off-diagonal couplings stored as BF16        */
                            /* remainders: coupling = offset + q * scale, one offset and one     */
                            /* power-of-two scale per direction, level and latitude row          */
    EG_FP32_IR_FP16 = 3,    /* as EG_FP32_IR_BF16 with FP16 remainders                           */
    EG_LEARNED_FP64 = 4,    /* flexible BiCGStab in FP64 with the learned preconditioner         */
    EG_LEARNED_FP32_IR = 5, /* FP64 refinement around flexible FP32 BiCGStab + learned precond.  */
    EG_FP32_MP = 6          /* the paper's mixed-precision BiCGStab (Sec. 3-4): FP32 vectors and
                               coefficients, FP64 solution updated every iteration, FP64 global
                               sums, restart from the FP64 true residual every restart_every
                               iterations (150 if 0) and when the recursive residual has met
                               tol but the true one has not; no refinement steps.  Where the
                               FP32 recurrence cannot carry the solve below tol it ends with
                               EG_STALLED after three such restarts                              */
};

/* Outcomes (>= 0) and errors (< 0). */
enum eg_status {
    EG_CONVERGED = 0,   /* true relative residual <= tol                                       */
    EG_MAXIT = 1,       /* iteration limit reached; x holds the last iterate                  */
    EG_BREAKDOWN = 2,   /* repeated breakdown without progress                                 */
    EG_STALLED = 3,     /* true residual could not be driven below tol (precision floor)       */
    EG_EINVAL = -1,     /* invalid argument or invalid operator                                */
    EG_ENOMEM = -2,     /* device allocation failed                                            */
    EG_EHIP = -3,       /* HIP runtime error                                                   */
    EG_ENONFINITE = -4, /* NaN or Inf in the right-hand side or the initial guess              */
    EG_ENOPC = -5       /* learned mode requested but no network is attached to the operator  */
};

/* Precision selector of the building-block calls (eg_apply, eg_apply_precond). */
enum eg_prec {
    EG_PREC_FP64 = 0,   /* double vectors, FP64 couplings                                      */
    EG_PREC_FP32 = 1,   /* float vectors, FP32 couplings                                       */
    EG_PREC_BF16 = 2,   /* float vectors, BF16 off-diagonal couplings                          */
    EG_PREC_FP16 = 3    /* float vectors, FP16 off-diagonal couplings                          */
};

typedef struct {
    int iterations;            /* Krylov iterations (summed over refinement steps)            */
    int outer_steps;           /* FP64 refinement steps (0 in EG_FP64 / EG_LEARNED_FP64)       */
    int restarts;              /* breakdown, periodic and residual-gap restarts               */
    int fallbacks;             /* learned modes: switches to the T^{-1} preconditioner;       */
                               /* refinement modes: +1 when the FP64 solver took over          */
    double true_rel_residual;  /* ||b - A x|| / ||b|| of the returned x, evaluated in FP64     */
    double seconds;            /* wall time of the solve                                       */
} eg_info;

/*
 * Build an operator from its seven coefficient arrays (Sec. 2, Eq. 4: A is the 7-band
 * Helmholtz matrix; the library solves the matrix it is given, scaling included).
 *   coeffs  device, double[7][nlev][nlat][nlon]; planes in the order W, E, S, N, D, U, C.
 *           W/E couple point (i,j,k) to (i-1,j,k) / (i+1,j,k) (periodic in i), S/N to
 *           (i,j-1,k) / (i,j+1,k), D/U to (i,j,k-1) / (i,j,k+1).  The six couplings are
 *           magnitudes >= 0: the matrix entries are their negatives.  C is the diagonal.
 *   Requirements (else EG_EINVAL, with the count of offending points in the message):
 *           nlon >= 3, nlat >= 1, nlev >= 1; all values finite; couplings >= 0;
 *           S = 0 on j = 0, N = 0 on j = nlat-1, D = 0 on k = 0, U = 0 on k = nlev-1;
 *           margin m = C - (W+E+S+N+D+U) > 0 at every point (row diagonal dominance).
 *   The library copies what it needs (the caller may free coeffs after return).  It keeps
 *   FP64 couplings, the margin m and the LU factors of the vertical tridiagonal; FP32 and
 *   16-bit copies are built on first use of a mode that needs them.
 *   *out receives the new operator (NULL on error).
 */
int eg_create_operator(const double *coeffs, int nlon, int nlat, int nlev, eg_operator **out);

/*
 * Solve A x = b to a true relative residual ||b - A x|| / ||b|| <= tol (Sec. 3, Eq. 8-9).
 *   b       device, double[n], read only.
 *   x       device, double[n]: initial guess in, solution out (untouched on error < 0).
 *   tol     > 0.
 *   maxit   > 0: limit on Krylov iterations (summed over refinement steps).
 *   mode    enum eg_mode.
 * Returns an eg_status; details of the solve via eg_get_info / eg_residual_history.
 * b = 0 gives x = 0 and EG_CONVERGED.  NaN/Inf in b or x gives EG_ENONFINITE.
 */
int eg_solve(eg_operator *op, const double *b, double *x, double tol, int maxit, int mode);

/* Statistics of the last eg_solve (host struct). */
int eg_get_info(const eg_operator *op, eg_info *info);

/*
 * Residual history of the last eg_solve: host double buffer of capacity cap receives the
 * recursive relative residual after each Krylov iteration (concatenated over refinement
 * steps).  Returns the number of entries available (may exceed cap; only cap are written).
 */
int eg_residual_history(const eg_operator *op, double *host_buf, int cap);

/* Order all later work of this operator on `hip_stream` (a hipStream_t; NULL = null stream). */
int eg_set_stream(eg_operator *op, void *hip_stream);

/*
 * Solver options (defaults in brackets):
 *   "eta"            inner relative tolerance of the FP32 refinement solves [1e-2]
 *                    (Sec. 3, Eq. 10: keep the 32-bit target well above eps_32)
 *   "restart_every"  mandatory restart period in iterations, 0 = off [0]
 *                    (Sec. 4 uses 150 operationally)
 *   "max_outer"      limit on refinement steps [30]
 *   "inner_maxit"    limit on the iterations of one inner FP32 solve [1000]; the correction of
 *                    a capped inner solve is kept only if it lowers the FP64 true residual
 *   "poll"           iterations enqueued between host checks of the device flags [8]
 *   "graph"          1 = the BiCGStab iterations between two host checks are captured once
 *                    (per precision, preconditioner and work buffers) as a HIP graph and
 *                    replayed: one launch call per batch instead of ten per iteration, for
 *                    grids small enough to be bound by launch overhead.  The graphs live on
 *                    a private stream created on first use and are freed by
 *                    eg_destroy_operator; 0 = launch every kernel (also whenever "profile"
 *                    is 1) [1]
 *   "eps_bd"         BiCGStab breakdown threshold, 0 <= eps_bd < 1 [2^-52]: the iteration
 *                    restarts (rhat = p = r) when |<rhat, r>| <= eps_bd ||rhat|| ||r|| or
 *                    |<rhat, v>| <= eps_bd ||rhat|| ||v|| (Sec. 4: near-zero scalar weights)
 *   "stall_window"   learned modes: iterations without a 2x gain that trigger fallback [20]
 *                    (FGMRES: at least one restart cycle, max(stall_window, gmres_m))
 *   "profile"        1 = time every streaming kernel launch (see eg_kernel_stats) [0]
 *   "precond"        preconditioner of the plain modes: 0 the vertical tridiagonal solve
 *                    T^{-1}, 1 red-black vertical-line SOR (the tri_sor of Sec. 2, Eq. 7, with
 *                    the columns in red-black order; needs an even nlon) [0].  The learned modes
 *                    and the harvests always build on T^{-1}.  The line SOR keeps the LU
 *                    factors and the W, E, S, N couplings a second time in colour-major order
 *                    (7n values in each precision used) and 5n/2 doubles of work space,
 *                    allocated on first use and held until eg_destroy_operator.
 *   "sor_sweeps"     sweeps of the line SOR, 1..16 [3]
 *   "sor_omega"      its relaxation factor, 0 < omega < 2 [1.5]
 *   "method"         Krylov method of the plain modes: 0 BiCGStab, 1 restarted FGMRES [0]
 *   "learned_method" Krylov method of the learned modes: 0 flexible BiCGStab, 1 FGMRES [1]
 *   "gmres_m"        FGMRES restart length, 1..64 [30]
 *   "mp_x32"         EG_FP32_MP only: 1 rounds the solution to FP32 after every update as well,
 *                    giving the all-32-bit BiCGStab of the paper's toy-model comparison (Sec. 4,
 *                    Fig. 1); with restart_every set beyond maxit it runs without restarts [0]
 *   "net_fused"      learned modes on grids with nlon a multiple of 64: 1 runs the network's
 *                    inference as one launch (input channels, all layers and q + rho delta,
 *                    activations kept on chip; a BF16 pair of static input channels per grid
 *                    point is built on first use and held until eg_destroy_operator), 0 as one
 *                    launch per layer with the activations in HBM [1]; the results are bitwise
 *                    the same
 * Returns EG_EINVAL for an unknown key or out-of-range value.
 */
int eg_set_option(eg_operator *op, const char *key, double value);

/* ---- building blocks (device pointers; used by the solver and exposed for tests) ---- */

/*
 * y = A x (Sec. 2, Eq. 4; 7-point stencil).  x, y: device arrays of n elements, double for
 * EG_PREC_FP64 and float otherwise; x and y must not overlap.  Computed in the difference
 * form y = m x + sum_d a_d (x - x_d), which equals the row definition C x - sum_d a_d x_d.
 */
int eg_apply(eg_operator *op, const void *x, void *y, int prec);

/*
 * z = M q with the operator's preconditioner.  Default: M = T^{-1}, T = tridiag(-D, C, -U) per
 * column (Sec. 2, Eq. 6-7: the vertical tridiagonal that replaces the diagonal; its LU factors
 * are precomputed per horizontal point when the operator is built).  With the option
 * "precond" = 1, M is the red-black vertical-line SOR from x = 0: each sweep updates the
 * columns with i + j even, then the others, by x_c <- (1 - omega) x_c + omega T_c^{-1}(q_c +
 * sum of the horizontal couplings times the neighbours' newest values).  q, z: device arrays
 * of n elements (double for EG_PREC_FP64, float otherwise); may not overlap.  FP64 uses the
 * FP64 factors and couplings; every other precision uses the FP32 rounding of the FP64 factors
 * and that precision's couplings.
 */
int eg_apply_precond(eg_operator *op, const void *q, void *z, int prec);

/*
 * r = b - A x in FP64 and *rel_host = ||r|| / ||b|| (host double; Sec. 3, Eq. 8-9).
 * b, x, r: device double[n]; r may be NULL (only the norm is returned).
 */
int eg_residual(eg_operator *op, const double *b, const double *x, double *r, double *rel_host);

/*
 * *out_host = sum_i a_i b_i with every product and the sum in FP64 (Sec. 4: 64-bit global
 * sums).  a, b: device arrays of n elements, double (prec = EG_PREC_FP64) or float (other).
 * Fixed-order two-pass reduction: bitwise reproducible for a given n.
 */
int eg_dot(eg_operator *op, const void *a, const void *b, long n, int prec, double *out_host);

/*
 * eg_dot for callers that cannot allocate device memory (code under stream capture, serving
 * loops that must not call hipMalloc): the same inner product with no operator and no
 * allocation of any kind.  Its partial sums and result live in a static device array of the
 * library, 8192 x 4 + 4 doubles (256 KiB + 32 B) per GPU, held from the first call on that GPU
 * until the process ends.
 *   a, b       device arrays of n elements, double (prec = EG_PREC_FP64) or float (other).
 *   n          0 .. 2^40 (EG_EINVAL beyond).
 *   hip_stream hipStream_t the work is ordered on (NULL = null stream); the call waits for it.
 *   out_host   host double.
 * Every call on one GPU uses that GPU's one array, which keeps the last call's contents: calls
 * that overlap on one GPU (from several threads or streams) race and must be serialised by the
 * caller.  Bitwise equal to eg_dot for the same n and inputs.
 */
int eg_dot_noalloc(const void *a, const void *b, long n, int prec, void *hip_stream, double *out_host);

/*
 * Kernel timing (tracing).  With the option "profile" set to 1, every streaming kernel launch
 * of eg_solve that does work is bracketed by HIP events on the operator's stream and its
 * device time is accumulated per (kernel, precision); the host then checks the device flags
 * after every iteration so no launch is wasted.
 *   kernel    enum eg_kernel;  prec  enum eg_prec of the vectors/couplings the launch used.
 *   launches  host long (may be NULL): number of timed launches.
 *   total_ms  host double (may be NULL): summed device time in milliseconds.
 * eg_reset_kernel_stats clears all counters.
 */
enum eg_kernel {
    EG_K_THOMAS_P = 0,   /* p = r + beta (p - omega v); phat = T^{-1} p                     */
    EG_K_SPMV_V = 1,     /* v = A phat with <rhat, v>, <v, v>                               */
    EG_K_THOMAS_S = 2,   /* s = r - alpha v; shat = T^{-1} s with <s, s>                    */
    EG_K_SPMV_T = 3,     /* t = A shat with <t, s>, <t, t>                                  */
    EG_K_UPDATE = 4,     /* x += alpha phat + omega shat; r = s - omega t with dots         */
    EG_K_RESIDUAL = 5,   /* FP64 true residual r = b - A x (refinement steps)               */
    EG_K_SOR_P = 6,      /* red-black line SOR half-sweeps on p (option "precond" = 1)      */
    EG_K_SOR_S = 7,      /* red-black line SOR half-sweeps on s                             */
    EG_K_COUNT = 8
};
int eg_kernel_stats(const eg_operator *op, int kernel, int prec, long *launches, double *total_ms);
int eg_reset_kernel_stats(eg_operator *op);

/* ---- learned right preconditioner ----
 *
 * The paper's preconditioner keeps the exact vertical tridiagonal solve (Sec. 2, Eq. 6-7).  The
 * learned form keeps it too and adds a correction from a small network in residual space:
 *     M(q) = T^{-1} (q + rho * delta(q)),   rho = rms(q),
 * delta from the input channels [q/rho, T^{-1}q / rms(T^{-1}q), D+U, W+E+S+N] through
 * conv1d over levels (4->32, 5 taps), ReLU, 3x3 horizontal mixing (32->32), ReLU, conv1d
 * (32->32, 5 taps), ReLU, conv1d (32->1, 5 taps).  15,233 parameters (flat FP32 vector,
 * order W1[5][32][4] b1[32] W2[9][32][32] b2[32] W3[5][32][32] b3[32] W4[5][32] b4; vertical
 * tap t couples level k+t-2, horizontal tap t couples (i + t%3 - 1, j + t/3 - 1), longitude
 * periodic, latitudes and levels zero-padded).  Inference and training run in BF16 on the
 * matrix cores with FP32 accumulation.  M is nonlinear, so the learned modes run flexible
 * BiCGStab (x is updated with exactly the preconditioned vectors that were multiplied by A),
 * and fall back to T^{-1} alone when the residual stalls (no halving of the best residual in
 * "stall_window" iterations, a residual 1e3 times the best, or a breakdown).
 */
typedef struct eg_net eg_net;

/* New network with He-normal weights from `seed` (splitmix64 + Box-Muller), zero biases and
 * a zero output layer, so that M = T^{-1} exactly until it is trained. */
int eg_net_create(unsigned long long seed, eg_net **out);
void eg_net_destroy(eg_net *net);                                   /* NULL-safe */
/* host float[count]; count must equal 15233.  Resets the optimiser state. */
int eg_net_set_weights(eg_net *net, const float *host, long count);
/* copies the weights to host float[cap] if cap >= 15233; returns 15233 */
int eg_net_get_weights(const eg_net *net, float *host, long cap);
/* Use `net` (not owned; must outlive its use; NULL detaches) in the EG_LEARNED_* modes. */
int eg_attach_learned_pc(eg_operator *op, eg_net *net);

/* z = M(q) in FP32 on the FP32 copy of the operator; q, z device float[n]; delta (may be
 * NULL) device float[n] receives the network output. */
int eg_net_apply(eg_operator *op, eg_net *net, const float *q, float *z, float *delta);

/* Training loss of a (residual, error) pair, A e = r:
 *   kind 1 (default)  ||A M(r) - r||^2 / ||r||^2   (residual space: what the Krylov method sees)
 *   kind 0            ||M(r) - e||^2 / ||e||^2     (error space)
 * Returns EG_EINVAL for another kind. */
int eg_net_set_loss(eg_net *net, int kind);

/* Loss of one (residual, error) pair (device float[n] each) and its gradient with respect to
 * the parameters (host double, host float[15233]; either may be NULL). */
int eg_net_loss_grad(eg_operator *op, eg_net *net, const float *r, const float *e, double *loss_host,
                     float *grad_host);

/* Harvest training pairs from the solver itself: solve A x* = b in FP64 as tightly as FP64
 * allows, then run FP64 BiCGStab from x0 = 0 and store r_i = b - A x_i and e_i = x* - x_i as
 * float for the iterates i = 0 .. nsnap-1 (i = 0 is x0 = 0: r_0 = b, e_0 = x*).
 * b: device double[n]; r_out, e_out: device float[nsnap][n].  Returns the number of pairs
 * stored (fewer if the solve converged first). */
int eg_harvest(eg_operator *op, const double *b, int nsnap, float *r_out, float *e_out);

/* Training pairs from the Krylov basis the preconditioner is applied to: one FGMRES(nvec) cycle
 * with M = T^{-1} from x0 = 0 on b (restarted flexible GMRES, Saad 1993; the paper's solver
 * family of Sec. 2 with its tridiagonal preconditioner of Eq. 7) stores its orthonormal basis
 * v_0 = b/||b||, v_1, ..., v_{nvec-1} in r_out (float), and, if e_out is not NULL, the errors
 * e_j = A^{-1} v_j from FP64 BiCGStab solves to a relative residual of 1e-10.
 * b: device double[n]; r_out, e_out: device float[nvec][n]; 1 <= nvec <= 64.  Returns the
 * number of pairs stored (fewer if the Krylov space became invariant first). */
int eg_harvest_krylov(eg_operator *op, const double *b, int nvec, float *r_out, float *e_out);

/* Train with Adam (lr; beta 0.9 / 0.999) on pairs r, e (device float[npairs][n]); pair i
 * belongs to operator ops[pair_op[i]] (host arrays; every operator must have the same grid).
 * Each epoch visits the pairs in a seeded random order in batches of `batch` (mean loss).
 * loss_hist (host double[epochs], may be NULL) receives each epoch's mean training loss.
 * All work is ordered on ops[0]'s stream. */
int eg_net_train(eg_net *net, eg_operator *const *ops, int nops, const float *r, const float *e, const int *pair_op,
                 int npairs, int epochs, int batch, double lr, unsigned long long seed, double *loss_hist);
/* Mean loss of the pairs (no training). */
int eg_net_eval(eg_net *net, eg_operator *const *ops, int nops, const float *r, const float *e, const int *pair_op,
                int npairs, double *mean_loss);

/* ---- the learned preconditioner as part of the operator ----
 *
 * The calls below give an operator a network of its own (created on first use, freed by
 * eg_destroy_operator) and make it the operator's learned preconditioner, as eg_attach_learned_pc
 * does with a caller-owned one.  Until one of them (or eg_attach_learned_pc) has run, the
 * EG_LEARNED_* modes return EG_ENOPC.
 *
 * Train it on (residual, error) pairs that the solver itself produces for this operator (the
 * iterates of FP64 BiCGStab, eg_harvest, or the Krylov basis of FGMRES, eg_harvest_krylov),
 * from seeded random right-hand sides b ~ N(0, 1) drawn in the library (splitmix64 + Box-Muller
 * from `seed`).  Sec. 2's solver is the source of the pairs; the network and its training are
 * this library's extension (the paper has no learned preconditioner).
 *   harvest_cfg  host string of comma-separated key=value settings (NULL or "" = defaults):
 *                  source=iterates|krylov   pairs r_i = b - A x_i, e_i = x* - x_i from the first
 *                                           iterates of an FP64 solve (eg_harvest), or the FGMRES
 *                                           basis v_j with e_j = A^{-1} v_j (eg_harvest_krylov)
 *                                           [iterates]
 *                  rhs=N         right-hand sides, 1..4096 [8]
 *                  pairs=K       pairs per right-hand side, 1..64 [20]
 *                  loss=error|residual      ||M(r) - e||^2/||e||^2 or ||A M(r) - r||^2/||r||^2 [error]
 *                  batch=B       pairs per Adam step [16]
 *                The pairs are held in device memory only during the call (2 K N n floats).
 *   epochs >= 0, lr > 0 (Adam, beta 0.9 / 0.999), seed: right-hand sides, shuffling and the
 *   network's initial weights when it is created here (a network that exists is trained on).
 * Returns 0, or EG_EINVAL for a bad setting (the message names it), EG_ENOMEM, EG_EHIP.
 */
int eg_train_learned_pc(eg_operator *op, const char *harvest_cfg, int epochs, double lr, unsigned seed);

/* The operator's learned preconditioner's weights as a byte image: a 16-byte header (the
 * characters "EGPC", format version 1, the parameter count 15233, 0, as int32) followed by the
 * 15233 FP32 weights in the order of eg_net_set_weights.
 *   weights  host buffer of cap bytes, or NULL to ask for the size.
 * Returns the image size in bytes (60948), whether or not it was written (it is written when
 * weights != NULL and cap is at least that size; a smaller cap gives EG_EINVAL), or EG_ENOPC
 * when the operator has no learned preconditioner. */
int eg_save_learned_pc(const eg_operator *op, void *weights, long cap);

/* Load an image written by eg_save_learned_pc (host buffer of nbytes bytes) into the
 * operator's own network (created if needed) and make it the learned preconditioner; the
 * optimiser state restarts.  EG_EINVAL when the header or the size does not match. */
int eg_load_learned_pc(eg_operator *op, const void *weights, long nbytes);

/* The network the operator's learned modes use (its own or an attached one), borrowed: valid
 * until the operator is destroyed or another network is attached.  *out = NULL and EG_ENOPC
 * when there is none. */
int eg_get_learned_pc(eg_operator *op, eg_net **out);

/* Grid sizes of an operator (host ints; any pointer may be NULL). */
int eg_get_shape(const eg_operator *op, int *nlon, int *nlat, int *nlev);

/* Release the operator and all its device memory.  NULL is accepted. */
void eg_destroy_operator(eg_operator *op);

/* Message describing the last error of the calling thread ("" if none). */
const char *eg_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* ENDGAME_H */
