/*
 * sem.h -- C ABI of the MI355X (gfx950) fast-diagonalisation solver for Q^k
 * spectral-element discretisations of  -Lap u + alpha u = f  on a 3D box.
 *
 * Method: Liu, Shen & Zhang, "A simple GPU implementation of spectral-element
 * methods for solving 3D Poisson type equations on rectangular domains and its
 * applications", arXiv 2310.00226.
 *   - discretisation: Sec. 2.1 (eq. fem): continuous Q^k Lagrange basis on the
 *     (k+1)-point Gauss-Lobatto nodes of each element, all integrals by that
 *     quadrature, hence a diagonal (lumped) mass matrix;
 *   - linear system: Sec. 2.4, eq. matvec3D,
 *       (K(x)M(x)M + M(x)K(x)M + M(x)M(x)K + alpha M(x)M(x)M) u = (M(x)M(x)M) f;
 *   - solver: Sec. 2.2-2.4, eq. 3D-Poisson with the robust eigen-solve of
 *     Sec. 2.3:  u = (S_x(x)S_y(x)S_z) diag(1/(lx_i+ly_j+lz_l+alpha)) (S_x(x)S_y(x)S_z)^T M_3 f,
 *     K S = M S Lambda, S^T M S = I per axis.
 *
 * Layout of every 3D array: row-major (n_x, n_y, n_z), z fastest, i.e. entry
 * u[(i*n_y + j)*n_z + l] is the value at node (x_i, y_j, z_l).  (The paper stores
 * the same array column-major; only the storage order differs.)  Values are
 * nodal; with Dirichlet conditions only interior nodes are unknowns
 * (n_a = ne_a*k - 1), with Neumann all nodes are (n_a = ne_a*k + 1), with
 * periodic conditions the node at the upper end of an axis is the node at its
 * lower end (n_a = ne_a*k; node 0 sits at box[2a]).
 *
 * Memory: array arguments named f, u, r, phi are DEVICE pointers owned by the
 * caller, float64, at least 8-byte aligned, on the device the plan was created
 * on.  Calls are asynchronous on the plan's stream (default: the null stream)
 * unless stated otherwise; a plan is not thread-safe (use one plan per stream).
 *
 * Errors: every call returns a sem_status and never aborts.  sem_last_error()
 * returns a description of the last failure on the calling thread.  A device
 * fault raised by earlier asynchronous work is reported as SEM_EDEVICE by the
 * next call that synchronises.
 */
#ifndef SEM_H_
#define SEM_H_

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct sem_plan sem_plan;

/* Boundary conditions on all six faces: homogeneous Dirichlet or Neumann (Sec. 2.1
 * remark), or periodic on every axis (Sec. 2.4 names periodic boundaries among
 * those of the same tensor form; Sec. 4 solves its Schroedinger problem with
 * them).  Periodic: the 1D stiffness and mass couple the last element to the
 * first, the factors stay dense n x n (for k > 1 they are not Fourier matrices). */
typedef enum { SEM_BC_DIRICHLET = 0, SEM_BC_NEUMANN = 1, SEM_BC_PERIODIC = 2 } sem_bc;

/* Arithmetic of the mode products.  The residual, the solution update and the
 * 1D eigen-decompositions are always FP64. */
typedef enum {
  SEM_F64 = 0,   /* FP64 MFMA, FP64 intermediates */
  SEM_F32 = 1,   /* FP32 MFMA, FP32 intermediates */
  SEM_BF16 = 2,  /* BF16 MFMA with FP32 accumulation, BF16 intermediates */
  SEM_BF16X3 = 3 /* split BF16 (hi + lo) operands, four BF16 MFMAs, FP32 accumulation */
} sem_prec;

typedef enum {
  SEM_OK = 0,
  SEM_EINVAL = 1,      /* invalid argument */
  SEM_ENOMEM = 2,      /* device or host allocation failed */
  SEM_EDEVICE = 3,     /* HIP runtime error or device fault */
  SEM_ESINGULAR = 4,   /* the operator has a zero eigenvalue (Neumann / periodic, alpha = 0) */
  SEM_ENOCONV = 5,     /* iterative refinement stopped without meeting the tolerance */
  SEM_ENONFINITE = 6   /* a residual or update became NaN / Inf */
} sem_status;

/* ---- plan ----------------------------------------------------------------- */

/* Build the 1D operators of each axis (Appendix SEGenerator1D: ne[a] uniform
 * elements on [box[2a], box[2a+1]], GLL rule of degree k), their generalised
 * eigen-decompositions in FP64 on the host (Sec. 2.3), and upload the factors to
 * the current HIP device.  k >= 1, ne[a] >= 1, box[2a] < box[2a+1], alpha >= 0.
 * Returns SEM_ESINGULAR when alpha + min eigenvalue sum is 0 (Neumann or periodic
 * with alpha = 0: the constants are in the kernel).
 * Synchronous.  The plan owns its factor storage (a few MB) until destroyed. */
sem_status sem_plan_create(int k, const int ne[3], const double box[6], double alpha, sem_bc bc, sem_plan **out);

/* As sem_plan_create with one boundary condition per axis (bc[a] on both faces of
 * axis a): the operators are Kronecker sums of per-axis 1D operators, so each
 * axis carries its own condition (Sec. 2.4 remark), e.g. periodic in x and z
 * with Dirichlet walls in y.  n_a follows bc[a]; SEM_ESINGULAR when no axis
 * removes the constants (no Dirichlet axis) and alpha = 0.  Every call that
 * takes a plan accepts such plans; sem_lift_boundary takes data on the faces of
 * the Dirichlet and Neumann axes. */
sem_status sem_plan_create_mixed(int k, const int ne[3], const double box[6], double alpha, const sem_bc bc[3],
                                 sem_plan **out);
void sem_plan_destroy(sem_plan *p);

/* n[a] = number of unknowns per axis. */
sem_status sem_plan_dims(const sem_plan *p, int n[3]);
/* Host copy of the n[axis] node coordinates / eigenvalues (ascending) of one axis. */
sem_status sem_plan_nodes(const sem_plan *p, int axis, double *x_host);
sem_status sem_plan_eigenvalues(const sem_plan *p, int axis, double *lam_host);
/* Run subsequent calls on this hipStream_t (NULL = the null stream). */
sem_status sem_plan_set_stream(sem_plan *p, void *hip_stream);

/* Scratch memory needed by sem_solve / sem_solve_refined at precision prec.
 * The caller may provide it (sem_plan_set_workspace, device memory that stays
 * valid while the plan uses it); otherwise the plan allocates it on first use. */
sem_status sem_plan_workspace_bytes(const sem_plan *p, sem_prec prec, size_t *bytes);
sem_status sem_plan_set_workspace(sem_plan *p, void *dev_ptr, size_t bytes);

/* ---- solve ---------------------------------------------------------------- */

/* FP64 fast-diagonalisation solve (eq. 3D-Poisson): u = A^{-1} M_3 f.
 * Forward mode products along z, y, x with F_a = S_a^T M_a, the divide by
 * lx_i + ly_j + lz_l + alpha fused into the x-axis product, backward products
 * with S_a.  On the uniform mesh the reflection of each axis commutes with its
 * 1D operators, so the eigenvectors are symmetric or antisymmetric: every
 * product runs as two half-size blocks on the folded vector (v_r + v_R(r),
 * v_r - v_R(r) over the orbit representatives r), half the flops of the dense
 * products; the forward blocks fold while they load, the backward blocks unfold
 * while they store.  Workspace: N doubles.  f and u are device arrays of
 * n_x n_y n_z doubles; u may alias f. */
sem_status sem_solve(sem_plan *p, const double *f, double *u);

/* For callers that cannot allocate device memory (code under HIP stream
 * capture, tight serving loops, allocation-free harnesses): the solve of
 * sem_solve, same kernels and same result bit for bit, with its intermediate
 * array of N doubles in a fixed device array inside this library instead of the
 * plan workspace.  Allocates nothing (no hipMalloc / hipFree, no library
 * allocation); the first call on a device looks up that device's copy of the
 * array, which the device holds until the process ends (SEM_NOALLOC_MAX_UNKNOWNS
 * doubles, 64 MiB).  Every call on one device shares that array: calls that
 * overlap on one device (concurrent streams or threads) race and must be
 * serialised by the caller; each call leaves its last intermediate in it.
 * f and u: device arrays of N doubles, u may alias f.  SEM_EINVAL: null
 * arguments, or N > SEM_NOALLOC_MAX_UNKNOWNS. */
#define SEM_NOALLOC_MAX_UNKNOWNS (8u * 1024u * 1024u)
sem_status sem_solve_noalloc(sem_plan *p, const double *f, double *u);

/* One FP64 mode product along `axis` (0 = x, 1 = y, 2 = z) with the forward
 * factor F_a (inverse = 0) or the backward factor S_a (inverse = 1):
 * out[.., l, ..] = sum_m A[l][m] in[.., m, ..].  in and out must not alias. */
sem_status sem_mode_product(sem_plan *p, int axis, int inverse, const double *in, double *out);

/* Nodal residual r = f - M_3^{-1} A u = f - alpha u - (H_x + H_y + H_z) u with
 * H = M^{-1} K (eq. matvec3D in H-form), FP64, matrix-free.  r must not alias u. */
sem_status sem_residual(sem_plan *p, const double *u, const double *f, double *r);

/* Non-homogeneous boundary data (Sec. 2.1 remark: boundary values and fluxes go
 * to the right-hand side, the matrix to invert stays the same).  Adds to the
 * nodal right-hand side f (device, plan layout, in place) the terms that carry
 * the data of the six faces; a following solve of the plan (sem_solve,
 * sem_solve_refined, a batch) then returns the solution with that data.
 * g[2a], g[2a+1]: device arrays with the data on the face x_a = box[2a] and
 * x_a = box[2a+1], row-major over the two other axes in their order (n_y x n_z,
 * n_x x n_z, n_x x n_y); a NULL face (or g == NULL) is homogeneous.
 *   Dirichlet axes: the values of u on the face at the nodes whose two other
 *     coordinates are unknowns (edge and corner values are not needed).  With u_b
 *     the data on the full grid of ne k + 1 nodes along the axis, f += -(H_x +
 *     H_y + H_z) u_b at the unknowns, which is -H_a(unknown, end node) g for the
 *     min(k, n_a) unknowns next to each face (H = M^{-1} K of the full-grid
 *     assembly).
 *   Neumann axes: the outward normal derivative at the face's nodes; by GLL
 *     quadrature of the boundary integral, f += g / M_a(end node) on the face
 *     (edges and corners sum the faces they lie on).
 *   Periodic axes: SEM_EINVAL for any non-NULL face of theirs.
 * Faces must not overlap f (SEM_EINVAL).  Asynchronous on the plan's stream;
 * the faces of one axis are one launch, the axes are applied in order. */
sem_status sem_lift_boundary(sem_plan *p, const double *const g[6], double *f);

/* Mixed-precision solve with FP64 iterative refinement:
 *   u = 0, r = f;  repeat  delta = FD_prec(r),  u += delta,  r = f - M_3^{-1} A u
 *   until ||delta||_inf <= tol * ||u||_inf, or until the updates contract fast
 *   enough that the remaining error is predicted below that: with
 *   r_k = ||delta_k|| / ||u_k|| and, from the third iteration on, q = the larger
 *   of r_k / r_{k-1} and r_{k-1} / r_{k-2}, stop when q < 1/2 and
 *   q r_k / (1 - q) <= tol / 10 (the next update and all later ones add up to
 *   q r_k / (1 - q) for a contraction that stays at q; q is an estimate, hence
 *   the factor of ten)  (iterations <= max_iter).
 * FD_prec is eq. 3D-Poisson with its six mode products in precision `prec`
 * (SEM_F32, SEM_BF16, SEM_BF16X3; SEM_F64 performs one FP64 solve); the update
 * of u and the residual are FP64.  tol = 0 runs exactly max_iter iterations.
 * f, u: device arrays of n_x n_y n_z doubles; u must not alias f.  Synchronises
 * the plan stream once per iteration (16-byte norm read-back).
 * Outputs: *iters = iterations run, *last_update_rel = ||delta||/||u|| of the last
 * one (either may be NULL).  Returns SEM_ENOCONV if tol > 0 was not met (u holds
 * the last iterate) or the updates grew for two consecutive iterations, and
 * SEM_ENONFINITE if an update became NaN / Inf. */
sem_status sem_solve_refined(sem_plan *p, sem_prec prec, double tol, int max_iter, const double *f, double *u,
                             int *iters, double *last_update_rel);

/* One fast-diagonalisation solve (eq. 3D-Poisson) with its six mode products in
 * precision prec (SEM_F32, SEM_BF16, SEM_BF16X3; SEM_F64 = sem_solve) and no
 * refinement: the single-precision solve of Sec. 3.7 (Table 10), accurate to
 * about the working precision times the conditioning.  u is FP64 (u = delta of
 * the first refinement iteration); u must not alias f.  Asynchronous. */
sem_status sem_solve_lowp(sem_plan *p, sem_prec prec, const double *f, double *u);

/* ---- launch-shape tuning ------------------------------------------------------
 * The low-precision mode products of a plan (sem_solve_refined, sem_solve_lowp,
 * the PCG preconditioner, the Cahn-Hilliard stepper, split-BF16 batch entries) run
 * with launch shapes chosen by timing on the first use of each precision: for
 * SEM_F32 the factor-tile rows (128, 96, 64 or 32) of each of the six passes; for
 * SEM_BF16 / SEM_BF16X3 the tile order, g = 1, 2 or 4 column strips of 256 that
 * consecutive workgroups share, and the launch: one workgroup per tile (value g)
 * or one workgroup per compute unit looping over the tiles (value 16 + g).  The
 * timed candidates are 1, 4, 17 and 20.  The shapes change no result bit.  Each candidate is launched
 * once untimed, then three times, on the plan's own workspace; the fastest is kept
 * in the plan and in a process-wide cache keyed by device architecture, kernel,
 * output layout and log2 size buckets of the pass, which later plans of similar
 * size read instead of timing.  With the environment variable SEM_TUNE_CACHE
 * naming a file, the cache is read from it on first use and rewritten after each
 * new entry (JSON: {"version": 1, "entries": {"<key>": <choice>, ...}}; an
 * unreadable file counts as empty).  Nothing is timed while the plan stream is
 * capturing a graph: the shapes then follow the fixed rule until a later call
 * outside capture tunes them. */
/* Tune prec now, consulting the cache (synchronous; uses the plan workspace).
 * SEM_EINVAL: prec is SEM_F64 (no tunable shape) or the plan stream is capturing. */
sem_status sem_plan_tune(sem_plan *p, sem_prec prec);
/* The shapes of prec's six passes in order of application (choice[s] = 0 and
 * *tuned = 0 before prec is tuned).  SEM_EINVAL: null pointers, SEM_F64. */
sem_status sem_plan_tuning(const sem_plan *p, sem_prec prec, int *tuned, int choice[6]);
/* Install shapes for prec without timing: 128, 96, 64 or 32 per pass for SEM_F32,
 * 1, 2, 4, 17, 18 or 20 for the BF16 modes.  SEM_EINVAL for anything else. */
sem_status sem_plan_set_tuning(sem_plan *p, sem_prec prec, const int choice[6]);
/* Process-wide cache counters: lookups answered, lookups missed, entries held. */
sem_status sem_tune_stats(int *hits, int *misses, int *entries);
/* Launch pass `pass` (0..5, order of application; for the BF16 modes the passes
 * of the reflection-split sequence) of prec's FD application `reps` times on the
 * plan stream, with the plan's tuned shapes, on whatever the plan workspace holds:
 * a way to time the mode-product kernels one by one (events around the call).
 * The result is not meaningful by itself; run a solve of prec first for
 * realistic data. Every access stays inside the workspace and the factors
 * whatever they hold. SEM_F32's last pass runs as an FP32 store of the same
 * shape instead of its accumulation into u. SEM_EINVAL: SEM_F64, pass outside
 * 0..5, reps < 1. */
sem_status sem_lowp_pass(sem_plan *p, sem_prec prec, int pass, int reps);

/* ---- other spectral multipliers --------------------------------------------- */

typedef enum { SEM_SPECTRAL_EXP = 1, SEM_SPECTRAL_POWER = 2 } sem_spectral;

/* u = g(H_3 + a I) f = S_3 g(Lambda3D + a) S_3^{-1} f on the transforms of the
 * solve (eq. 3D-Poisson with its divide replaced; the paper's introduction and
 * conclusion name exponential time differencing and spectral fractional
 * Laplacians as such multipliers), FP64:
 *  SEM_SPECTRAL_EXP:   g(x) = exp(-param x), param = t >= 0: the solution at time t
 *                      of u_t = Lap u - a u, u(0) = f;
 *  SEM_SPECTRAL_POWER: g(x) = x^(-param): the fractional operator (-Lap + a)^(-param)
 *                      (param = 1: the solve with alpha = a; param < 0: a positive
 *                      fractional power).
 * f, u: device FP64 arrays of N nodal values (u may alias f); uses the plan
 * workspace like sem_solve.  Asynchronous on the plan stream.  SEM_EINVAL: null
 * pointers, unknown kind, non-finite a or param, t < 0.  SEM_ESINGULAR: a
 * negative power with min(Lambda3D) + a <= 0. */
sem_status sem_apply_spectral(sem_plan *p, int kind, double a, double param, const double *f, double *u);

/* ---- variable coefficients (PCG) ---------------------------------------------- */

/* Bytes of the caller-provided workspace of sem_pcg_solve: four FP64 arrays of N
 * (r, z, p, q) and the partial sums of the inner products. */
sem_status sem_pcg_workspace_bytes(const sem_plan *p, size_t *bytes);

/* alpha u - Lap u + V u = f (the paper's Schrodinger-equation section, eq.
 * shrodinger; alpha = the plan's alpha, V >= 0 given at the nodes) by
 * preconditioned conjugate gradients with the fast-diagonalisation solve of
 * (shift I - Lap) as the preconditioner (eq. 3D-Poisson with alpha := shift).
 * The operator is the GLL-quadrature weak form divided by the lumped mass,
 * A u = alpha u + H_3 u + V u, applied matrix-free in FP64; the inner products are
 * M_3-weighted.  Starts from u = 0 and stops when ||f - A u||_M <= tol ||f||_M.
 *  v, f, u: device FP64 arrays of N nodal values (u must not alias f or v);
 *  shift: > 0 as given; <= 0 selects the paper's choice alpha + beta / 2 for
 *        0 <= V <= beta, with beta = max(V) reduced on the device;
 *  prec: precision of the preconditioner's mode products (SEM_F64, or SEM_F32 /
 *        SEM_BF16 / SEM_BF16X3, then with the flexible Polak-Ribiere update; the
 *        operator, the update and the inner products stay FP64);
 *  work: device buffer of sem_pcg_workspace_bytes bytes, 256-byte aligned.
 *        The preconditioner also uses the plan workspace.
 *  iters / relres / shift_used (may be NULL): iterations, final ||r||_M / ||f||_M
 *        and the shift the preconditioner used.
 * Synchronises with the plan stream once per inner product (three per iteration),
 * and once more for the default shift.
 * SEM_EINVAL: null pointers, aliasing, a non-finite shift, a default shift that is
 * not > 0, tol < 0, max_iter < 1, small or misaligned workspace.  SEM_ENOCONV: tol
 * not met within max_iter, or a non-positive curvature (V too negative: A not
 * positive definite).  SEM_ENONFINITE: NaN / Inf in V (default shift), in f or in
 * an iterate. */
sem_status sem_pcg_solve(sem_plan *p, const double *v, double shift, sem_prec prec, double tol, int max_iter,
                         const double *f, double *u, void *work, size_t work_bytes, int *iters, double *relres,
                         double *shift_used);

/* ---- batched solves ---------------------------------------------------------- */

typedef struct sem_batch sem_batch;

/* A batch of `count` independent problems, one plan each (any mix of k <= 8,
 * element counts, boxes, alpha and BC; all on one device).  A plan may appear
 * more than once: several right-hand sides of one operator, solved together; the
 * entries after its first occurrence get workspaces of their own (allocated by
 * the batch), the first uses the plan's.  The plans are not owned and must
 * outlive the batch.  Creation prepares the FP32 factors and workspaces of every
 * entry, then times the candidate tile shapes of the FP32 mode-product kernel on
 * the batch's own passes and keeps the fastest per contraction-length bucket
 * (through the tuning cache of sem_plan_tune: a bucket of the same length and
 * log2 work found there is not timed again).
 * Synchronous.  SEM_EINVAL: count < 1, a null plan, k > 8, plans on different
 * devices. */
sem_status sem_batch_create(int count, sem_plan *const *plans, sem_batch **out);
void sem_batch_destroy(sem_batch *b);
sem_status sem_batch_set_stream(sem_batch *b, void *hip_stream);
/* Block-tile rows chosen per contraction-length bucket n <= 16, 32, 64, 128, 256,
 * > 256 (0 = no such length in the batch). */
sem_status sem_batch_tile_rows(const sem_batch *b, int rows[6]);
/* Solve all problems: f[i], u[i] are device arrays of plan i's N_i doubles (host
 * arrays of count device pointers; u[i] must not alias f[i]).
 *  SEM_F32: the refinement of sem_solve_refined for every problem at once; each
 *           of the six mode products of an iteration is one persistent launch per
 *           tile shape over all still-unconverged problems, each residual one
 *           launch per k.  One synchronisation per iteration (norm read-back).
 *  SEM_BF16X3: as SEM_F32, except that every problem whose three dimensions are
 *           all >= 96 runs its iterations with the split-BF16 mode products of
 *           sem_solve_refined (one launch per pass, on three side streams that
 *           wait on and are joined back into the batch stream, concurrently with
 *           the persistent launches of the other problems); all problems refine
 *           in FP64 to the same tol.
 *  SEM_F64: one FP64 sem_solve per problem on the batch stream.
 * Every call (re)lays out each plan's low-precision workspace for the chosen
 * precision, so plans may be used by other calls between batch solves; the call
 * first waits for the batch stream.
 * iters (host array of count, may be NULL) receives the iterations per problem.
 * Returns SEM_ENONFINITE if a problem produced a non-finite update, else
 * SEM_ENOCONV if a problem stopped without meeting tol (diverging, or max_iter). */
sem_status sem_batch_solve(sem_batch *b, sem_prec prec, double tol, int max_iter, const double *const *f,
                           double *const *u, int *iters);

/* ---- Cahn-Hilliard IMEX time stepping (Sec. 3.6) ---------------------------- */

typedef struct sem_ch sem_ch;

/* Stepper of eq. chscheme-2 (BDF2 in time, nonlinear term extrapolated) for
 *   phi_t = m Lap w,  w = -eps Lap phi + (1/eps) F'(phi),  F'(phi) = phi^3 - phi,
 * Q^k SEM in space with homogeneous Neumann conditions on the box (all nodes are
 * unknowns, n_a = ne_a*k + 1).  One step solves
 *   (a I + m dt eps H_3^2) phi_{n+1} = phi_hat - (m dt / eps) H_3 F'(phi_bar),
 *   a = 3/2, phi_hat = 2 phi_n - phi_{n-1}/2, phi_bar = 2 phi_n - phi_{n-1},
 * H_3 = -Lap_h = M_3^{-1} K_3, by one fast-diagonalisation application with the
 * spectral multiplier 1 / (a + m dt eps Lambda3D^2) in precision `prec`, followed
 * by refine_sweeps (0..64) FP64 iterative-refinement sweeps against that operator
 * (matrix-free residual).  eps, mob (m), dt > 0.  Creates the plan, an internal
 * stream and all device buffers (5 arrays of N doubles plus the solve workspace)
 * up front.  Synchronous.  SEM_EINVAL on invalid arguments. */
sem_status sem_ch_create(int k, const int ne[3], const double box[6], double eps, double mob, double dt,
                         sem_prec prec, int refine_sweeps, sem_ch **out);
void sem_ch_destroy(sem_ch *c);
sem_status sem_ch_dims(const sem_ch *c, int n[3]);
/* Order the stepper's work after earlier work on this hipStream_t and before later
 * work on it (NULL = the null stream).  The steps themselves run on the stepper's
 * own stream. */
sem_status sem_ch_set_stream(sem_ch *c, void *hip_stream);
/* Launch shapes of the stepper's mode products, tuned at creation (see
 * sem_plan_tune; *tuned = 0 for SEM_F64). */
sem_status sem_ch_tuning(const sem_ch *c, int *tuned, int choice[6]);
/* enable = 1 (default): each step is a replay of a captured HIP graph (captured on
 * the first call, and again whenever phi_n / phi_nm1 change address); 0: the same
 * kernels launched one by one. */
sem_status sem_ch_set_graphs(sem_ch *c, int enable);
/* Optional source term (the accuracy test of the BDF2 scheme adds the source of a
 * manufactured solution): s = device array of N doubles read by every following
 * step as the nodal source at the new time level t_{n+1}, entering the step as
 * dt * s (BDF2 for phi_t = m Lap mu + s); NULL removes it.  The caller updates the
 * contents between steps (ordered on the stream of sem_ch_set_stream); a new
 * pointer re-captures the step graphs.  SEM_EINVAL: null handle. */
sem_status sem_ch_set_forcing(sem_ch *c, const double *s);
/* Advance nsteps >= 0 steps.  phi_n, phi_nm1: device arrays of N doubles (distinct),
 * holding phi_n and phi_{n-1} on entry (first step: pass phi_0 in both) and
 * phi_{n+nsteps}, phi_{n+nsteps-1} on return.  Asynchronous. */
sem_status sem_ch_step(sem_ch *c, double *phi_n, double *phi_nm1, int nsteps);

/* Host-only helper (no device needed): the 1D operators of one axis as built by
 * sem_plan_create.  Call with all output pointers NULL to get n; then pass
 * buffers of n (x, mass, lam) and n*n (S, F, row-major) doubles; any output may
 * be NULL.  S: backward factor (K S = M S Lambda, S^T M S = I); F = S^T M. */
sem_status sem_axis_host(int k, int ne, double a, double b, sem_bc bc, int *n, double *x, double *mass, double *lam,
                         double *S, double *F);

/* Host-only helper: the reflection-split form of the same axis that the BF16
 * passes use.  The uniform mesh is symmetric about the midpoint, node i maps to
 * R(i) = n - 1 - i (periodic: (n - i) mod n), and every eigenvector is symmetric
 * or antisymmetric.  nrep: orbit representatives 0..nrep-1 of {i, R(i)}; nodd =
 * n - nrep antisymmetric eigenvectors.  Folded mode order: nrep symmetric then
 * nodd antisymmetric, each ascending (lam_fold, n values).  With the folded vector
 * v+_r = v_r + v_R(r), v-_r = v_r - v_R(r) (r < nrep): F v = [ffold_sym v+;
 * ffold_anti v-] where ffold (n x nrep, row-major) holds both blocks in folded
 * mode order; and for folded coefficients c = [c_sym; c_anti] the backward
 * transform is u_r = e_r + o_r, u_R(r) = e_r - o_r with e = bfold_sym c_sym
 * (nrep x nrep) and o = bfold_anti c_anti (nrep x nodd).  Pass NULL for outputs not
 * wanted; nrep, nodd may be queried first with all arrays NULL. */
sem_status sem_axis_fold_host(int k, int ne, double a, double b, sem_bc bc, int *nrep, int *nodd, double *lam_fold,
                              double *ffold, double *bfold_sym, double *bfold_anti);

/* Text of the last error on the calling thread ("" if none). */
const char *sem_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* SEM_H_ */
