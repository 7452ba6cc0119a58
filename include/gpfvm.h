/*
 * gpfvm -- GP finite-volume PDE solver hot path for AMD Instinct MI355X (gfx950).
 *
 * A Gaussian-process prior with a separable squared-exponential kernel is
 * conditioned on
 *   - volume observations  L_V[u] = int_V D[u] dx = int_V f dx  over the cells
 *     of a factorised box grid (paper Sec. 3, eq. linop-def; Sec. 4.1,
 *     Definition of a factorised box FVM scheme), and
 *   - initial/boundary point observations d^beta u(x) = y (Sec. 2.2, L_IC,BC),
 * with Gram matrix G = L k L' + Sigma in observation order [points; volumes]
 * (Sec. 2.2; Sec. 2.1 eq. affine-posterior).  The volume block is applied
 * matrix-free as a sum of Kronecker products of closed-form 1-D cell-integral
 * factors (Sec. 3.2 eq. LkL; Sec. 4.1 eq. kronecker-structure); the point block
 * is conditioned exactly by Cholesky and the volume observations by IterGP
 * with CG actions (Sec. 4.1, Sec. 4.2).
 *
 * Conventions common to every call
 *   - Dimension 0 is time.  Volumes are flattened row-major (dimension 0
 *     slowest); a point group is a tensor grid flattened the same way.
 *   - "host" pointers are read during the call only and may be freed on return.
 *     "device" pointers are caller-owned HBM buffers (e.g. PyTorch tensors) that
 *     must stay valid until the work queued on `stream` has completed; the
 *     library never frees them.
 *   - `stream` is a hipStream_t passed as void* (NULL = the null stream).  All
 *     device work is queued on it; a call returns once its work is queued,
 *     except where a call states that it synchronises.
 *   - Every call returns GPFVM_OK (0) or a negative GPFVM_E_* code.  No C++
 *     exception crosses this boundary.  Arguments are validated before any HIP
 *     call, so invalid input never reaches the GPU.  gpfvm_last_error() gives
 *     a message.
 *   - A handle is not thread-safe; distinct handles are independent.
 */
#ifndef GPFVM_H
#define GPFVM_H

#ifdef __cplusplus
extern "C" {
#endif

#define GPFVM_OK             0
#define GPFVM_E_INVALID     -1   /* malformed argument or IBVP                      */
#define GPFVM_E_NOMEM       -2   /* device allocation failed / admission refused    */
#define GPFVM_E_HIP         -3   /* a HIP runtime call failed                       */
#define GPFVM_E_NOTPD       -4   /* Cholesky of the point block failed (not PD), or  */
                                 /* IterGP breakdown (eta <= 0)                      */
#define GPFVM_E_NOCONV      -5   /* iteration budget exhausted above the tolerance;  */
                                 /* the early-terminated state stays valid           */
#define GPFVM_E_STATE       -6   /* call out of order (e.g. posterior before solve)  */

#define GPFVM_MAX_DIM        3
#define GPFVM_MAX_TERMS     16
#define GPFVM_MAX_GROUPS    16
#define GPFVM_MAX_DERIV      4   /* highest derivative order per dim in any term    */
#define GPFVM_MAX_OUTPUTS    8   /* outputs of a multi-output prior (Sec. 3.3)      */
#define GPFVM_MAX_PTERMS     2   /* terms of one point observation (e.g. radiation) */

#define GPFVM_PREC_FP64      0   /* every step in float64                            */
#define GPFVM_PREC_MIXED     1   /* Gram matvec in low precision (tile format below)
                                    inside float64 iterative refinement; float64
                                    recurrences, directions and posterior            */

/* Tile formats of the low-precision volume Gram (chosen at assemble).  The
 * volume Gram is a sum of Kronecker terms that cancel to far below their
 * size: its small eigenvalues sit at the PDE noise level (about 1e-6 of the
 * mean diagonal), so the low-precision operator must keep float32 accuracy or
 * the volume system turns indefinite, as it does with a single bfloat16 or
 * float16 tile (relative error 2^-9 / 2^-11).  Both formats below keep float32
 * accuracy. */
#define GPFVM_TILE_FP32      0   /* float32 factor tiles and tensors on the float32
                                    matrix cores, float32 accumulation              */
#define GPFVM_TILE_BF16X3    1   /* float32 factor tiles and tensors, each value
                                    split into three bfloat16 slices on the way
                                    into the bfloat16 matrix cores; the six slice
                                    products of order <= 4 per block, float32
                                    accumulation (float32 accuracy)                 */

/* Solve methods (Sec. 4.1, "Iterative techniques"). */
#define GPFVM_METHOD_ITERGP  0   /* IterGP with CG actions: stores every direction;
                                    posterior mean and combined variance             */
#define GPFVM_METHOD_CG      1   /* plain conjugate gradients: O(N) state, no stored
                                    directions; posterior mean only (the variance
                                    needs the directions: GPFVM_E_STATE)             */

/* One-dimensional kernels of the tensor-product prior (Sec. 3.1-3.2).  The
 * half-integer Matern kernels k(r) = exp(-c r/l) p_q(c r/l), c = sqrt(2q+1),
 * nu = q + 1/2, admit derivative orders up to q in that dimension (PDE terms
 * and point observations alike); the squared exponential admits any order up
 * to GPFVM_MAX_DERIV. */
#define GPFVM_KERNEL_SE        0
#define GPFVM_KERNEL_MATERN12  1   /* q = 0 */
#define GPFVM_KERNEL_MATERN32  2   /* q = 1 */
#define GPFVM_KERNEL_MATERN52  3   /* q = 2 */
#define GPFVM_KERNEL_MATERN72  4   /* q = 3 */

typedef struct gpfvm_handle gpfvm_handle;

/* One term  coef * w(x) * d^deriv u_output(x)  of a point observation.  The
 * per-point weight is separable over the group's grid, w(x) = prod_i
 * weight[i][j_i] (NULL: 1 in that dim); e.g. the wave speed c = sqrt(g H)
 * along an edge in the radiation condition h_t = c dh/dn (appendix
 * "Tsunami propagation", boundary condition). */
typedef struct {
  int deriv[GPFVM_MAX_DIM];            /* derivative multi-index                     */
  double coef;                         /* finite                                     */
  int output;                          /* 0 .. nout-1                                */
  const double* weight[GPFVM_MAX_DIM]; /* host: n[i] values per dim, or NULL         */
} gpfvm_pointterm;

/* One tensor grid of point observations  d^deriv u(x) = y + eps,
 * eps ~ N(0, noise_var)  (Sec. 2.2: initial and boundary observations), or,
 * with nterm >= 1, of the sum of the point terms:  sum_c terms[c] = y + eps. */
typedef struct {
  int n[GPFVM_MAX_DIM];              /* points per dim (1 pins a dim, e.g. t = 0)    */
  const double* axis[GPFVM_MAX_DIM]; /* host: n[i] coordinates per dim               */
  int deriv[GPFVM_MAX_DIM];          /* derivative multi-index beta (nterm = 0)      */
  const double* y;                   /* host: prod(n) values, row-major              */
  double noise_var;                  /* > 0                                          */
  int output;                        /* observed output (nterm = 0)                  */
  int nterm;                         /* 0: the single term (deriv, output);          */
                                     /* 1..GPFVM_MAX_PTERMS: the sum of terms[]      */
  const gpfvm_pointterm* terms;      /* host                                         */
} gpfvm_pointgroup;

/* An initial-boundary value problem (Sec. 1 eq. def-lin-pde with the IBVP
 * stacking of Sec. 2.2).  The operator is D = sum_t coef[t] * (cell_coef if
 * cellwise[t]) * d^alpha_t; per-cell coefficients are constant inside a cell
 * (appendix on variable bathymetry).
 *
 * Systems (Sec. 3.3): with nout > 1 outputs the prior is
 * k = diag(s_0 k, ..., s_{nout-1} k) (eq. multioutput-cov-def; every output
 * the same tensor-product kernel k, outputscale s_i = out_scale[i]), and
 * with neq > 1 equations every cell carries neq volume observations,
 * equation e being sum over the terms t with term_eq[t] = e of
 * coef[t] (cell_coef) d^alpha_t u_{term_out[t]}.  Volume observations are
 * ordered equation-major (all cells of equation 0 first), so f_int then
 * holds neq * prod(ncell) values.  The linearised shallow-water equations
 * (appendix "Tsunami propagation", eq. sw1 to sw3) are such a system: three
 * outputs (h, u, v), three equations, cell_coef = H.  A system is solved in
 * float64 (IterGP or CG) and its posterior gives every output; the mixed
 * path, the coarse warm start, targeted reduction and the server take
 * single-output problems only (GPFVM_E_INVALID otherwise). */
typedef struct {
  int dim;                            /* 2 or 3 (time + 1 or 2 space dims)           */
  int ncell[GPFVM_MAX_DIM];           /* cells per dim, >= 1                          */
  const double* edges[GPFVM_MAX_DIM]; /* host: ncell[i]+1 strictly increasing edges  */
  double lengthscale[GPFVM_MAX_DIM];  /* lengthscale per dim, > 0                      */
  int kernel[GPFVM_MAX_DIM];          /* GPFVM_KERNEL_* per dim (0: squared exponential)*/
  double outputscale;                 /* sigma_f^2 > 0                                */
  int nterm;                          /* 1..GPFVM_MAX_TERMS                           */
  const int* alpha;                   /* host: nterm*dim derivative multi-indices     */
  const double* coef;                 /* host: nterm coefficients                     */
  const int* cellwise;                /* host: nterm flags, or NULL (all 0)           */
  const double* cell_coef;            /* host: N per-volume values, needed if any     */
                                      /* cellwise flag is set, else ignored           */
  const double* f_int;                /* host: neq*N values of int_V f, or NULL (= 0) */
  double noise_pde;                   /* PDE observation noise (see next field)       */
  int noise_pde_relative;             /* 1: variance = noise_pde * mean diagonal of   */
                                      /* L_V k L_V';  0: variance = noise_pde         */
  int ngroup;                         /* 0..GPFVM_MAX_GROUPS                          */
  const gpfvm_pointgroup* groups;     /* host                                         */
  int nout;                           /* outputs, 0 or 1: one                         */
  int neq;                            /* equations per cell, 0 or 1: one              */
  const int* term_out;                /* host: nterm output indices, or NULL (all 0)  */
  const int* term_eq;                 /* host: nterm equation indices, or NULL (0)    */
  const double* out_scale;            /* host: nout outputscales > 0, or NULL (all    */
                                      /* equal to outputscale)                        */
} gpfvm_ibvp;

typedef struct {
  int max_iter;        /* capacity for stored IterGP directions (>= 1)              */
  int tile;            /* GPFVM_TILE_* format of the low-precision volume Gram      */
  int reuse_memory;    /* 1 (default): device blocks come from and return to a      */
                       /* per-device cache of this process, so repeated             */
                       /* assemble/destroy cycles make no hipMalloc/hipFree calls;  */
                       /* gpfvm_release_cached_memory() hands the cached blocks     */
                       /* back.  0: the handle allocates and frees its own blocks.  */
} gpfvm_assemble_opts;

typedef struct {
  int prec;            /* GPFVM_PREC_FP64 or GPFVM_PREC_MIXED                       */
  double tol;          /* stop once ||r|| <= tol ||b|| on the volume system (0: none)*/
  int max_iter;        /* iterations (IterGP: <= assemble max_iter)                 */
  int resume;          /* 1: continue from the stored state of a previous solve     */
  int tile;            /* mixed path: must equal the handle's tile format           */
  int block;           /* mixed path: low-precision iterations per refinement block */
                       /* (1 .. GPFVM_MAX_BLOCK); each block is followed by the     */
                       /* float64 re-stabilisation of its directions               */
  int max_outer;       /* mixed path: refinement blocks at most                     */
  int check_every;     /* host convergence poll interval in iterations (>= 1)       */
  int reorth_passes;   /* 1: the published recurrence d = s - C z (one projection);  */
                       /* 2: the projection repeated on d (stored S D; default)      */
  int replace_every;   /* passes = 2: residual recomputed as b - S v every k iters   */
  int coarsen[GPFVM_MAX_DIM]; /* coarse warm start (appendix "Multigrid preconditioners"):*/
                       /* before CG, condition exactly on the nested coarse scheme   */
                       /* whose cells are coarsen[0] x ... x coarsen[d-1] blocks of  */
                       /* fine cells (factors divide the cell counts; all 1: off).   */
                       /* Needs a fresh FP64 solve with reorth_passes = 2; the       */
                       /* coarse cells (< assemble max_iter, <= GPFVM_MAX_COARSE)    */
                       /* become the first stored directions.                       */
  int method;          /* GPFVM_METHOD_ITERGP (default) or GPFVM_METHOD_CG; CG is    */
                       /* float64, fresh (no resume) and without the coarse start   */
} gpfvm_solve_opts;

#define GPFVM_MAX_COARSE 8192
#define GPFVM_MAX_BLOCK  64

typedef struct {
  int iters;           /* IterGP: directions stored (posterior rank); CG: iterations*/
  int outer;           /* refinement blocks taken (mixed path)                      */
  double rel_res;      /* ||b - S v|| / ||b|| on the volume (Schur) system          */
  double rel_res_full; /* ||y - G alpha|| / ||y|| on the whole IBVP system           */
  int status;          /* GPFVM_OK, GPFVM_E_NOCONV or GPFVM_E_NOTPD                 */
  int coarse;          /* directions of the coarse warm start (included in iters)   */
} gpfvm_solve_info;

typedef struct {
  int dim; long long n_pde; int n_b; long long n;
  double noise_pde_var;          /* absolute PDE noise variance actually used       */
  long long device_bytes;        /* HBM held by the handle                          */
  int volume_launches;           /* kernel launches of one gpfvm_volume_matvec       */
  double volume_flops;           /* flops those launches execute (all rhs)          */
} gpfvm_handle_info;

/* Default option values. */
void gpfvm_default_assemble_opts(gpfvm_assemble_opts* o);
void gpfvm_default_solve_opts(gpfvm_solve_opts* o);

/* Validate an IBVP without touching the GPU.  Returns GPFVM_OK or
 * GPFVM_E_INVALID (message via gpfvm_last_error(NULL)). */
int gpfvm_validate(const gpfvm_ibvp* p);

/* Build a handle: copy the IBVP to HBM, compute the closed-form 1-D factors
 * (Sec. 3.1 eq. linop-simplified reduces every cell integral of a derivative
 * to differences of antiderivatives/derivatives, evaluated with erf and exp),
 * form the point block G_bb (dense), factor it G_bb = L L^T (Sec. 4.2) and its
 * triangular inverse, and prepare the matrix-free plan of G_pp.  Synchronises
 * on `stream` before returning (so that a non-PD point block is reported).
 * Errors: INVALID, NOMEM, HIP, NOTPD.  On error *out is NULL. */
int gpfvm_assemble(const gpfvm_ibvp* p, const gpfvm_assemble_opts* opts,
                   void* stream, gpfvm_handle** out);

/* y = G x for the whole IBVP Gram (Sec. 2.2, G = L k L' + Sigma, observation
 * order [points; volumes], Sigma included), for nrhs right-hand sides.
 * x, y: device, n*nrhs values of type dtype (GPFVM_DTYPE_F64: double,
 * GPFVM_DTYPE_F32: float; float input is widened to float64 and the float64
 * result rounded to float), right-hand side r at offset r*n; x and y must not
 * overlap.  prec selects the float64 plan or the low-precision plan of the
 * volume block (GPFVM_PREC_MIXED, tile format given at assemble); the point
 * and cross blocks stay float64.  Errors: INVALID, NOMEM, HIP. */
#define GPFVM_DTYPE_F64 0
#define GPFVM_DTYPE_F32 1
int gpfvm_matvec(gpfvm_handle* h, int nrhs, const void* x, void* y, int dtype, int prec, void* stream);

/* y = S x with S = L_V k L_V' + Sigma_V - G_pb G_bb^{-1} G_bp, the Gram of the
 * volume observations under the prior already conditioned on the point
 * observations (Sec. 4.2): the operator the iterative solver applies.
 * x, y: device, N*nrhs doubles (N = volume observations, neq per cell), no overlap.  prec
 * GPFVM_PREC_MIXED evaluates the volume Kronecker block in the handle's
 * low-precision tile format and the point-block correction in float64.
 * Errors: INVALID, NOMEM, HIP. */
int gpfvm_schur_matvec(gpfvm_handle* h, int nrhs, const double* x, double* y, int prec, void* stream);

/* y = (L_V k L_V' + Sigma_V) x: the volume block of the Gram alone (Sec. 4.1
 * eq. kronecker-structure, with per-cell coefficients as diagonal scalings),
 * the Kronecker sum evaluated as MFMA mode products.  x, y: device,
 * N*nrhs doubles, no overlap.  For GPFVM_PREC_FP64 the plan is bound to x and
 * y on the first call with that (x, y, nrhs) and reused (the buffers must stay
 * allocated while the handle lives); GPFVM_PREC_MIXED runs the low-precision
 * plan (the handle's tile format) through internal buffers.  Errors: INVALID, NOMEM, HIP. */
int gpfvm_volume_matvec(gpfvm_handle* h, int nrhs, const double* x, double* y, int prec, void* stream);

/* The float64 volume-Gram matvec of gpfvm_volume_matvec (y = (L_V k L_V' +
 * Sigma_V) x, nrhs right-hand sides), for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc): the call makes no hipMalloc, hipFree or other device
 * allocation.  Its Kronecker-plan intermediates and GEMM descriptors live in
 * a static device scratch of GPFVM_NOALLOC_SCRATCH_BYTES that each GPU the
 * library runs on holds until the process ends; the plan is rebuilt in it on
 * every call (a host-side compile and one descriptor upload, which
 * synchronises `stream`), and nothing in it needs to start at zero.  Every
 * call on a GPU shares that GPU's scratch: calls that overlap on one GPU (from
 * several threads, or on several streams without ordering) race.  x, y:
 * device, N*nrhs doubles, no overlap.  Errors: INVALID (also when the plan
 * for this problem and nrhs does not fit the scratch), HIP. */
#define GPFVM_NOALLOC_SCRATCH_BYTES (32LL << 20)
int gpfvm_volume_matvec_noalloc(gpfvm_handle* h, int nrhs, const double* x, double* y, void* stream);

/* Representer weights alpha = G^{-1} y (Sec. 4, representer weights): exact
 * conditioning on the points, then IterGP with CG actions on the volume
 * observations (Sec. 4.1-4.2).  The state (weights, directions, eta) stays in
 * the handle for gpfvm_posterior and for resume.  Synchronises to fill info.
 * Returns GPFVM_OK, or NOCONV / NOTPD (info->status too), or INVALID / HIP.
 * A tolerance below the attainable accuracy: the float64 IterGP loop stops
 * once its residual has grown 1000-fold above the smallest value it reached,
 * rolls the weights and the stored directions back to that iterate, and
 * returns NOCONV (gpfvm_last_error says so) with that iterate's state, which
 * the posterior then uses. */
int gpfvm_solve(gpfvm_handle* h, const gpfvm_solve_opts* opts, gpfvm_solve_info* info,
                void* stream);

/* Posterior mean and variance on the tensor grid axis[0] x ... x axis[dim-1]
 * (Sec. 2.1 eq. lin-cond-mean and eq. lin-cond-cov).  The variance is the
 * IterGP combined variance: prior minus the exact point-block reduction minus
 * the reduction captured by the stored directions (it equals the mathematical
 * posterior variance once the directions span the volume system).
 * n: host, dim sizes; axis: host coordinate arrays; mean, var: device,
 * prod(n) doubles row-major (var may be NULL); for a system with nout > 1
 * outputs, nout * prod(n) doubles, output-major (output i at i * prod(n)),
 * each output's variance taken against its own prior s_i k.  Errors:
 * INVALID, STATE (no solve yet), NOMEM, HIP. */
int gpfvm_posterior(gpfvm_handle* h, int dim, const int* n, const double* const* axis,
                    double* mean, double* var, void* stream);

/* Targeted uncertainty reduction (appendix "Targeted uncertainty reduction"):
 * `iters` further IterGP iterations on the volume system after gpfvm_solve,
 * each taking as its action the residual b_i - S C b_i of the right-hand side
 * b_i = K_S(X~) beta_i, where K_S(X~) is the cross-covariance between the
 * volume observations and the target grid axis[0] x ... x axis[dim-1] under
 * the IC/BC-conditioned prior (Sec. 4.2) and C the inverse approximation of
 * the directions stored so far.  The new directions are appended, so the
 * combined variance of gpfvm_posterior drops first where the weights put
 * mass; the representer weights take the usual step with the data residual.
 * weights: host, iters x prod(n) doubles row-major (row i = beta_i, e.g. a
 * Dirichlet draw the caller makes).  n, axis: host, as for gpfvm_posterior.
 * Needs a preceding float64 solve with reorth_passes = 2 (its stored S D
 * images form the action without extra operator applications) and room for
 * the directions (iterations so far + iters <= assemble max_iter).
 * Synchronises to fill info (iters = directions now stored).  Errors: INVALID
 * (bad grid, weights or capacity), STATE (no suitable solve), NOMEM, HIP;
 * NOTPD when eta <= 0 (directions kept up to the last good one). */
int gpfvm_refine_variance(gpfvm_handle* h, int dim, const int* n, const double* const* axis,
                          int iters, const double* weights, gpfvm_solve_info* info,
                          void* stream);

/* Copy the current representer weights (n doubles, [points; volumes]) to the
 * device buffer `alpha`.  Errors: STATE, HIP. */
int gpfvm_weights(gpfvm_handle* h, double* alpha, void* stream);

/* Dense block of G (including Sigma): rows [r0, r0+nr), cols [c0, c0+nc) into
 * the device buffer out (row-major, leading dimension ld >= nc), built from the
 * factor tiles (Sec. 4.1 eq. kronecker-structure).  Errors: INVALID, HIP. */
int gpfvm_gram_block(gpfvm_handle* h, long long r0, long long nr, long long c0,
                     long long nc, double* out, long long ld, void* stream);

/* 1-D closed-form factor matrix (Sec. 3.1 eq. linop-simplified, Sec. 3.2
 * eq. LkL) for one lengthscale, evaluated by the factor kernel:
 *   kind 0  cell-cell   out[i*n2+j] = int_{I_i} int_{J_j} d^p_s d^q_s' k(s,s')
 *   kind 1  point-cell  out[i*n2+j] = int_{J_j} d^p_x d^q_s' k(x_i,s')
 *   kind 2  point-point out[i*n2+j] = d^p_x d^q_x' k(x_i,x'_j)
 * For cell arguments the host array holds n+1 edges, for points n coordinates.
 * kernel: GPFVM_KERNEL_*.  0 <= p, q and p+q <= 2*GPFVM_MAX_DERIV; for a Matern
 * kernel also p, q <= its q.  out: device, n1*n2 doubles. */
int gpfvm_factor(int kind, int kernel, int p, int q, int n1, const double* a1, int n2,
                 const double* a2, double lengthscale, double* out, void* stream);

int gpfvm_get_info(const gpfvm_handle* h, gpfvm_handle_info* info);

/* ---- continuous-batching server --------------------------------------------
 * Whole GP-PDE solves (assemble + solve + posterior) of different sizes and
 * data, submitted as they arrive.  Worker threads, one HIP stream each, admit
 * queued requests in arrival order whenever a worker is free and the
 * request's estimated HBM footprint fits in the budget left by the requests
 * in flight; the requests in flight run concurrently on the device.  Device
 * memory comes from a caching allocator owned by the server.  Results do not
 * depend on the other requests in flight (deterministic kernels). */
typedef struct gpfvm_server gpfvm_server;

typedef struct {
  int workers;              /* concurrent requests (1..16)                       */
  long long hbm_budget;     /* bytes of HBM the requests in flight may reserve    */
  int prec;                 /* GPFVM_PREC_* of every solve                        */
  double tol;               /* relative residual target of every solve            */
  int max_iter;             /* IterGP iteration cap (also sizes the directions)   */
  int check_every;          /* convergence poll interval                          */
  int coarse_cells;         /* coarse-scheme warm start of every solve (appendix  */
                            /* "Multigrid preconditioners"): the nested coarse    */
                            /* scheme with the most cells <= coarse_cells whose   */
                            /* factors divide the request's cell counts (0: off;  */
                            /* needs prec FP64, <= GPFVM_MAX_COARSE)              */
  int max_batch;            /* most requests solved together as one batch when    */
                            /* they share the operator (same grid, kernel, PDE and */
                            /* point layout; float64 path without the coarse       */
                            /* start), 1 .. GPFVM_MAX_SERVER_BATCH; 1: none        */
} gpfvm_server_opts;
#define GPFVM_MAX_SERVER_BATCH 64

typedef struct {
  int rc;                   /* GPFVM_OK / NOCONV / error code of the request      */
  gpfvm_solve_info info;
  double t_submit, t_start, t_done;   /* host steady-clock seconds                */
  long long est_bytes;      /* HBM reserved for it at admission                   */
  long long n_grid;         /* posterior grid points                              */
  int batch;                /* requests solved together with it (1: alone);      */
                            /* for batched requests info.rel_res_full is NaN      */
} gpfvm_request_result;

typedef struct {
  long long queued, completed;
  int in_flight, peak_in_flight;
  long long reserved_bytes, peak_reserved_bytes, cached_bytes, device_bytes;
} gpfvm_server_info;

void gpfvm_default_server_opts(gpfvm_server_opts* o);
/* Start the workers on the current device.  Errors: INVALID, HIP. */
int gpfvm_server_create(const gpfvm_server_opts* opts, gpfvm_server** out);
/* Queue one request: the IBVP (validated and deep-copied; the caller may free
 * its arrays on return) and its posterior grid (host axes).  *ticket
 * identifies it.  Errors: INVALID, STATE (server stopping). */
int gpfvm_server_submit(gpfvm_server* s, const gpfvm_ibvp* p, int dim, const int* n, const double* const* axis,
                        long long* ticket);
/* *done = 1 once the request has finished (wait = 1 blocks until then); then
 * fills res (if not NULL) and copies prod(n) posterior means / variances into
 * the host arrays mean / var (each may be NULL).  Errors: INVALID. */
int gpfvm_server_poll(gpfvm_server* s, long long ticket, int wait, int* done, gpfvm_request_result* res,
                      double* mean, double* var);
int gpfvm_server_stats(gpfvm_server* s, gpfvm_server_info* st);
/* Finish the queued requests, stop the workers and free all device memory. */
void gpfvm_server_destroy(gpfvm_server* s);

/* Free every device buffer of the handle (after synchronising its stream;
 * with reuse_memory, after synchronising the device, then the blocks go back
 * to the cache).  NULL is accepted. */
void gpfvm_destroy(gpfvm_handle* h);

/* Return the unused blocks of every per-device cache (reuse_memory) to the
 * runtime.  Blocks held by live handles stay.  Returns the bytes freed. */
long long gpfvm_release_cached_memory(void);

/* Message of the last error on h, or (h == NULL) of this thread's last
 * validation / assemble error.  Never NULL. */
const char* gpfvm_last_error(const gpfvm_handle* h);

#ifdef __cplusplus
}
#endif
#endif /* GPFVM_H */
