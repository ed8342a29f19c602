/*
 * bz.h - C ABI of the MI355X fast spectral Boltzmann collision library.
 *
 * The library evaluates, for every spatial cell handed to it, the fast
 * spectral approximation of the 3D-velocity Boltzmann collision operator
 * Q(f,f) (Sec. 4.4.1: truncated Carleman operator Q^R, decoupled kernel,
 * sum over A sphere directions of discrete convolutions evaluated by FFT),
 * and the moment-realizability regime mask that selects those cells
 * (Sec. 3.2-3.3 and 4.5, Algorithm 1).
 *
 * Conventions shared by every entry point
 *   - Return value: bz_status, 0 = BZ_OK, > 0 = BZ_AGAIN (not ready yet, or no
 *     room yet), < 0 = error.  No C++ exception crosses the ABI.  The text of
 *     the last error of the calling thread is returned by bz_last_error().
 *   - Device pointers are owned by the caller (e.g. torch tensors).  The
 *     library never allocates device memory: it reports the sizes it needs and
 *     the caller passes buffers.  Streams are hipStream_t passed as void*
 *     (NULL = the null stream).  Calls that take a stream only enqueue work;
 *     they return before the GPU finishes.
 *   - Velocity grid (Sec. 4.1): n points per axis on [-L, L)^3,
 *     v_j = (j - n/2) * 2L/n, a distribution is n^3 values in row-major
 *     order [i1][i2][i3] (i3 fastest).  A batch is [cells][n][n][n].
 */
#ifndef BZ_H
#define BZ_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define BZ_ABI_VERSION 5

typedef int32_t bz_status;

enum {
  BZ_OK = 0,
  BZ_AGAIN = 1,
  BZ_ERR_ARG = -1,         /* invalid argument (null pointer, bad size, bad enum) */
  BZ_ERR_UNSUPPORTED = -2, /* valid request the library does not implement */
  BZ_ERR_DEVICE = -3,      /* HIP runtime error (message in bz_last_error) */
  BZ_ERR_NOMEM = -4,       /* caller-supplied buffer or arena too small */
  BZ_ERR_STATE = -5,       /* call out of order (e.g. plan not bound) */
  BZ_ERR_NUMERIC = -6      /* invalid numeric input detected */
};

/* element types of distributions and outputs */
enum { BZ_FP64 = 0, BZ_FP32 = 1 };

/* direction rules for the angular quadrature over the half sphere
   (Sec. 4.4.1, 3D case); weights always sum to 2*pi */
enum {
  BZ_DIRS_EXPLICIT = 0, /* use desc.dirs / desc.weights */
  BZ_DIRS_ICOSA6 = 1,   /* six icosahedral axes, weight pi/3 (m must be 6) */
  BZ_DIRS_PRODUCT = 2,  /* theta_p=(p+1/2)pi/a1, phi_q=q pi/a2, weights ~ sin(theta) */
  BZ_DIRS_SPIRAL = 3,   /* equal-weight golden spiral, z_p=(p+1/2)/m */
  BZ_DIRS_CIRCLE = 4,   /* two velocity dimensions: theta_p = pi p/m, p = 1..m,
                           weight pi/m each (the only rule of dim = 2 plans) */
  BZ_DIRS_DESIGN = 5    /* equal-weight antipodal spherical design, 2 <= m <= 256:
                           the golden spiral moved by damped minimum-norm
                           Gauss-Newton steps until sum_p Y_lm(e_p) = 0 for every
                           real harmonic of even degree 2 <= l <= L, L the largest
                           even degree with L (L + 3) / 2 <= 2m - 3 equations
                           (lowered by 2 while the iteration stalls); the rule then
                           integrates polynomials of degree <= t = L + 1 exactly
                           (bz_plan_rule_degree; m = 32: t = 9, m = 64: t = 15) */
};

/* evaluation strategy */
enum {
  BZ_XF_AUTO = 0,  /* fused kernel where one exists for (n, precision), else plain */
  BZ_XF_FUSED = 1, /* fused per-direction kernel (FP32, n in {16, 24, 32}) */
  BZ_XF_PLAIN = 2, /* unfused pencil kernels through HBM (any precision, any n) */
  BZ_XF_DFT_GEMM = 3 /* the plain path with its last length-n inverse transforms
                        (along k1) done as dense DFT matrix products on the matrix
                        cores (FP32 MFMA, exact FP32 products; FP32 plans, n in
                        {16, 32, 48}): 8n flop per point against the FFT's
                        5 log2 n, kept only where the autotuner measures it faster */
};

/* bz_collide_batch flags */
enum {
  BZ_SCATTER = 1 /* write cell c of the output at row idx[c] instead of row c */
};

/*
 * Plan descriptor.  Defines the discrete operator: velocity grid (n, L),
 * truncation radius R of Q^R, decoupled kernel Btilde(x,y) = kernel_c *
 * |x|^(gamma-1) (gamma = 1, kernel_c = 4 is the hard-sphere kernel
 * B = |v - v*| of Sec. 2.1), and the direction rule.
 */
typedef struct {
  int32_t n;             /* points per velocity axis: 16, 24, 32 or 48 */
  double L;              /* half width of the velocity box */
  double R;              /* truncation radius; <= 0 selects (sqrt(2)-1) L; must be
                            <= 4L/(3+sqrt 2), the period-overlap bound of Sec. 4.4.1 */
  double gamma;          /* kernel exponent in [0, 1] */
  double kernel_c;       /* kernel constant; 4.0 gives B = |v - v*| at gamma = 1 */
  int32_t m;             /* number of half-sphere directions, 1..512 */
  int32_t dir_kind;      /* BZ_DIRS_* */
  const double* dirs;    /* host [m][3] unit vectors (BZ_DIRS_EXPLICIT), else ignored */
  const double* weights; /* host [m], sum 2*pi (BZ_DIRS_EXPLICIT), else ignored */
  int32_t a1, a2;        /* BZ_DIRS_PRODUCT grid sizes, a1*a2 == m */
  int32_t precision;     /* BZ_FP32: FP32 transforms, multipliers and products,
                            FP32 accumulation; BZ_FP64: everything in FP64 */
  int32_t transform;     /* BZ_XF_* */
  int32_t project;       /* 1: FP64 conservative projection, FP64 output;
                            0: raw Q in the plan precision */
  int32_t max_cells;     /* largest batch the bound workspace must hold; also sets
                            the plain path's directions per chunk at n = 48
                            (FP32: 8 up to 1024 cells, else 4; results do not
                            depend on it) */
  int32_t chunks;        /* plain path: directions per stage-A launch (1..17; 0 =
                            from max_cells, as described under max_cells);
                            fused path: direction chunks per cell, each a workgroup;
                            0 = from max_cells (n = 24, 32: 4 up to 64 cells, 2 up
                            to 128, else 1; n = 16: 4 up to 256, 2 up to 512), unless
                            a tune table has a line for the plan.  Results depend
                            on the chunk count at FP32 rounding level only */
  int32_t slices;        /* fused path: j3 slices of the LDS transposes, 1 or 2
                            (n = 16 either; n = 24 always uses 1, n = 32 2);
                            0 = auto */
  int32_t dealias;       /* 0: circular convolution (l + m = k mod n);
                            1: truncated convolution without wrap-around
                            (l + m = k over the series' own modes), evaluated
                            by the 3/2 rule on a padded 3n/2 grid; n = 16, 32 */
  int32_t dim;           /* velocity dimensions: 0 or 3 (the operator above), or 2:
                            Maxwell molecules in two velocity dimensions (Sec.
                            4.4.1, the 2d case): f is [n][n], gamma must be 0,
                            Btilde = kernel_c (the paper's normalisation is 1),
                            dir_kind BZ_DIRS_CIRCLE, n in {16, 32, 64} (FP64:
                            16, 32), one fused kernel (transform AUTO or FUSED),
                            dealias, chunks and slices 0 */
} bz_plan_desc;

typedef struct bz_plan bz_plan;

/* ABI version the library was built with (BZ_ABI_VERSION). */
int32_t bz_abi_version(void);

/* Text of the calling thread's last error ("" if none).  Valid until the
   thread's next failing call. */
const char* bz_last_error(void);

/*
 * Build a plan on the host: validates the descriptor (BZ_ERR_ARG on
 * unsupported n, R beyond the non-overlap bound, |sum w - 2 pi| > 1e-12,
 * non-unit directions), generates the direction rule and evaluates in FP64
 * the Fourier multipliers of the fast method for every direction p and wave
 * vector kappa_k (Sec. 4.4.1, 3D case, read as):
 *   alpha_p(k)  = phi_R(kappa_k . e_p),  phi_R(s) = 2 int_0^R r^gamma cos(r s) dr,
 *   alpha'_p(k) = psi_R(|kappa_k - (kappa_k . e_p) e_p|), psi_R(r) = 2 pi R J1(R r)/r,
 * the loss multiplier Bhat_M(k) = sum_p w_p alpha_p(k) alpha'_p(k), and the
 * inverse Gram matrix of the five collision invariants (hypothesis (H1)).
 * dim = 2 (Sec. 4.4.1, the 2d case): alpha_p(k) = phi(kappa_k . e_p),
 * alpha'_p(k) = phi(kappa_k . e_p'), phi(s) = 2R sinc(R s), e_p = (cos, sin)
 * theta_p, e_p' = e_p turned by pi/2, w_p = pi/m, and the four invariants
 * (1, v1, v2, |v|^2); bz_collide_batch then takes distributions of n^2 values
 * [i1][i2] (batches [cells][n][n]) and returns Q in the same layout.
 * *out receives a heap object owned by the caller (bz_plan_destroy).
 */
bz_status bz_plan_create(const bz_plan_desc* desc, bz_plan** out);

/* Device bytes the plan needs: multiplier tables (read-only, shared by all
   calls), and a workspace of ws_fixed + ws_per_cell * cells. */
bz_status bz_plan_device_bytes(const bz_plan* plan, size_t* tables, size_t* ws_fixed,
                               size_t* ws_per_cell);

/* Attach caller device memory and upload the tables (asynchronous copy on
   `stream`; the host tables stay alive inside the plan).  tables_dev must
   hold the `tables` bytes, ws_dev ws_bytes >= ws_fixed + ws_per_cell.  Both
   must be 256-byte aligned.  Calls that share a plan share its workspace:
   they must be ordered on one stream.  ws_dev NULL with ws_bytes 0 binds the
   tables only (capacity 0; for bz_collide_batch_noalloc). */
bz_status bz_plan_bind(bz_plan* plan, void* tables_dev, void* ws_dev, size_t ws_bytes,
                       void* stream);

/* Free the host plan (device buffers stay with the caller). */
bz_status bz_plan_destroy(bz_plan* plan);

/* Cells a bound plan can process per bz_collide_batch call. */
bz_status bz_plan_capacity(const bz_plan* plan, int32_t* cells);

/* Evaluation strategy the plan resolved to (BZ_XF_FUSED or BZ_XF_PLAIN). */
bz_status bz_plan_transform(const bz_plan* plan, int32_t* transform);

/* Strategy table written by the autotuner (paper_2505_03360_amd/autotune.py):
   one line per tuned case, "gfx950 n m precision max_cells transform chunks
   slices us_per_cell" (chunks: direction chunks per cell of the fused kernel,
   or directions per launch pair of the plain path).  bz_plan_create consults
   it when desc.transform is BZ_XF_AUTO and desc.chunks and desc.slices are 0:
   it takes the line with the same (n, m, precision) and the largest max_cells
   not above the plan's (else the smallest).  Which table: the one set here;
   with NULL (the default), the file named by the environment variable
   BZ_TUNE_TABLE, else tune_gfx950.txt in the directory of the library (the
   table measured on an MI355X and shipped with it); "" uses none (the size
   heuristics below). */
bz_status bz_set_tune_table(const char* path);

/* Strategy the plan resolved to: transform, chunks (fused: direction chunks
   per cell; plain: directions per stage-A launch), slices. */
bz_status bz_plan_strategy(const bz_plan* plan, int32_t* transform, int32_t* chunks, int32_t* slices);

/* Host copies of the plan's direction rule: dirs [m][3], weights [m]
   (dim = 2: (cos theta_p, sin theta_p, 0) and pi/m). */
bz_status bz_plan_get_rule(const bz_plan* plan, double* dirs, double* weights);

/* Antipodal spherical-design degree t of the plan's direction rule: the
   largest odd t such that the rule, extended to the whole sphere by e -> -e,
   integrates every polynomial of degree <= t exactly (checked through
   sum_{p,q} w_p w_q P_l(e_p . e_q) <= 1e-12 (sum w)^2 for every even l <= t - 1,
   up to l = 80).  ICOSA6 gives 5; the spiral and product rules give 1;
   BZ_ERR_UNSUPPORTED for dim = 2 plans. */
bz_status bz_plan_rule_degree(const bz_plan* plan, int32_t* t);

/* Host copy of the FP64 multipliers of pass p (0 <= p <= m; pass m is the
   loss pass (Bhat_M, 1)) as [k2][k3][k1][2] = (alpha_p, alpha'_p)
   (dim = 2: [k2][k1][2]). */
bz_status bz_plan_get_multipliers(const bz_plan* plan, int32_t p, double* out);

/*
 * Evaluate Q(f,f) for a batch of cells (Sec. 4.4.1):
 *   fhat = DFT(f)/n^3 with Nyquist modes zeroed;
 *   Q+   = sum_p w_p IDFT(alpha_p fhat) * IDFT(alpha'_p fhat);
 *   Q    = kernel_c * (Q+ - IDFT(fhat) * IDFT(Bhat_M fhat));
 *   if project: Q <- Q - C^T (C C^T)^-1 C Q (FP64; C = [1, v1, v2, v3, |v|^2]),
 *   which restores the invariants of (H1) that periodisation loses.
 * f:       device [*][n][n][n] of f_dtype (BZ_FP64 or BZ_FP32); cell c is row
 *          idx[c] (idx NULL: row c).
 * idx:     device int32 [ncells] or NULL.
 * ncells:  cells to process, <= capacity; with ncells_dev it is the upper bound.
 * ncells_dev: device int32 or NULL; when given, the number of cells processed
 *          is min(*ncells_dev, ncells), read on the GPU (no host sync; for
 *          graph capture and masks that choose the cells on the GPU).
 * q:       device output, FP64 if the plan projects, else the plan precision;
 *          row c (compact) or row idx[c] (flags & BZ_SCATTER).
 * stream:  hipStream_t.  Asynchronous.  The arithmetic of a cell does not
 *          depend on the other cells of the batch, so results are bitwise
 *          identical for any batch composition.
 */
bz_status bz_collide_batch(const bz_plan* plan, const void* f, int32_t f_dtype,
                           const int32_t* idx, int32_t ncells, const int32_t* ncells_dev,
                           void* q, int32_t flags, void* stream);

/*
 * bz_collide_batch for callers that cannot allocate device memory or take a
 * caller-owned workspace (code under HIP graph capture, tight serving loops,
 * harnesses that forbid allocation): the same evaluation, arguments and
 * results, with the workspace taken from a static 64 MiB device array that
 * the library holds on every device it runs on until the process ends.  It
 * allocates nothing.
 * plan:    bound to its tables; the workspace binding may be absent
 *          (bz_plan_bind with ws_dev NULL and ws_bytes 0) and is not used.
 * ncells:  at most what fits: ws_fixed + ws_per_cell * ncells <= 64 MiB
 *          (bz_plan_device_bytes; FP32 plans of more than 128 cells: 170
 *          cells at n = 32, 1360 at n = 16), else BZ_ERR_NOMEM with the limit
 *          in bz_last_error; with
 *          ncells_dev, ncells is the bound the array must hold.
 * Every call on a device shares that device's array, which keeps the last
 * call's contents: calls that overlap on one device (other streams, other
 * threads) race and must be serialised by the caller.  Non-finite outputs
 * are not reported (the array's status word is cleared by each call and
 * bz_plan_sync does not read it).
 */
bz_status bz_collide_batch_noalloc(const bz_plan* plan, const void* f, int32_t f_dtype,
                                   const int32_t* idx, int32_t ncells, const int32_t* ncells_dev,
                                   void* q, int32_t flags, void* stream);

/* Numeric status of the plan's evaluations: waits for `stream`, then returns
   BZ_ERR_NUMERIC (and clears the flag) if any bz_collide_batch /
   bz_imex_euler / bz_pr222_* output written through this plan's binding since
   the last sync (or bind) held a non-finite value (e.g. from a NaN in f),
   else BZ_OK.  Evaluations never stop on such values: they are reported. */
bz_status bz_plan_sync(bz_plan* plan, void* stream);

/* Per-stage GPU timing of bz_collide_batch, for measurement.  When enabled,
   each call records HIP events on its stream around the forward transform,
   the direction/loss kernel(s) and the projection (up to 512 calls are
   kept).  bz_plan_last_times waits for the recorded calls and returns the
   average milliseconds per call in ms[0..3] = {forward, directions,
   projection, total} (and, if n > 4, the number of calls in ms[4]); it then
   starts a new averaging window. */
bz_status bz_plan_set_timing(bz_plan* plan, int32_t enable);
bz_status bz_plan_last_times(bz_plan* plan, float* ms, int32_t n);

/*
 * Macroscopic fields of a batch of cells (Sec. 2: the density, velocity and
 * temperature that define the equilibria (H3)) and the L1 distance of the
 * kinetic-to-fluid criterion (Sec. 3.3), in FP64 over the velocity grid:
 *   rho = dv^3 sum_j f_j,  u = sum_j v_j f_j / sum_j f_j,
 *   T = (sum_j |v_j|^2 f_j / sum_j f_j - |u|^2) / 3,
 *   l1 = dv^3 sum_j |f_j - rho (2 pi T)^(-3/2) exp(-|v_j - u|^2 / (2T))|.
 * n: 16, 24, 32 or 48 (BZ_ERR_UNSUPPORTED otherwise); L > 0.
 * f, idx, ncells, ncells_dev: as for bz_collide_batch.
 * out: host struct of device FP64 arrays, each NULL (not computed / not
 *      written) or written at position c (compact) or idx[c] (BZ_SCATTER), so
 *      that rho, u1 (-> ux), u2 (-> uy), T and l1 can be written straight into
 *      the [ny][nx] inputs of bz_realizability_mask.  Cells with sum f <= 0
 *      give non-finite u, T and l1 (the mask then counts them as invalid).
 * Asynchronous on `stream`; per-cell results do not depend on the batch.
 */
typedef struct {
  double *rho, *u1, *u2, *u3, *T, *l1;
} bz_moments_out;

bz_status bz_cell_moments(int32_t n, double L, const void* f, int32_t f_dtype, const int32_t* idx,
                          int32_t ncells, const int32_t* ncells_dev, const bz_moments_out* out,
                          int32_t flags, void* stream);

/*
 * One step of the penalised first-order IMEX scheme of the Boltzmann layer
 * (Sec. 4.4, eq. (4.24), after Filbet and Jin), fused with the evaluation of
 * Q(f^n) by `plan`:
 *   g = f^n - dt tr,  U^{n+1} = int (1, v, |v|^2) g  (Q and P conserve them),
 *   beta = 2 pi rho^{n+1},  P(h) = beta (M[h] - h),
 *   f^{n+1} = (eps g + dt (Q(f^n) - P(f^n)) + beta dt M^{n+1}) / (eps + beta dt),
 * M^n the Maxwellian of f^n's moments, M^{n+1} that of U^{n+1}; Q is the
 * plan's operator (FP64 projected when the plan projects).
 * desc:   dt > 0; eps > 0 used when eps_cells is NULL, else eps_cells (device
 *         FP64, read at the rows of f) holds the Knudsen number per row.
 * f, tr:  device FP64 [*][n][n][n]: f^n and the transport term v . grad_x f^n,
 *         cell c at row idx[c] (idx NULL: row c).
 * f_out:  device FP64, row c or idx[c] (BZ_SCATTER); may equal f when the
 *         rows written are the rows read (BZ_SCATTER, or no idx).
 * ncells <= the plan's capacity; ncells_dev as for bz_collide_batch.
 * The plan must be bound; asynchronous on `stream`.
 */
typedef struct {
  double dt;
  double eps;
  const double* eps_cells;
} bz_imex_desc;

bz_status bz_imex_euler(const bz_plan* plan, const bz_imex_desc* desc, const double* f, const double* tr,
                        const int32_t* idx, int32_t ncells, const int32_t* ncells_dev, double* f_out,
                        int32_t flags, void* stream);

/*
 * The same penalised splitting integrated in time with the second-order
 * PR(2,2,2) IMEX Runge-Kutta scheme (tableaux of Sec. 4.3, C = 1/sqrt 2,
 * implicit diagonal gamma = 1 - 1/sqrt 2), explicit part
 * -v.grad_x y + (Q(y) - P(y))/eps, implicit part P(y)/eps, P(y) = beta (M[y] - y),
 * beta = 2 pi rho.  Each implicit stage Y = R + (h/eps) P(Y) is solved by
 * S(R, h) = (eps R + h beta M[R]) / (eps + h beta) (P conserves the invariants).
 * Since both tableaux share their weights, the step reduces to
 *   stage 1:  Y1 = S(y, gamma dt)
 *   [caller:  T1 = v . grad_x Y1]
 *   stage 2:  R2 = y - dt T1 + (dt/eps) Q(Y1) - (2 gamma dt/eps) P(Y1),
 *             Y2 = S(R2, gamma dt),  A = y - (dt/2) T1 + (dt/(2 eps)) Q(Y1)
 *   [caller:  T2 = v . grad_x Y2]
 *   finish:   y_out = A - (dt/2) T2 + (dt/(2 eps)) Q(Y2)
 * The transport terms need neighbouring cells, which is why the step is split
 * where the caller evaluates them.  Q is the plan's operator (FP64 projected
 * when the plan projects; an FP32 plan must project).
 * Every array is device FP64 [*][n][n][n] and cell c lives at row idx[c] (idx
 * NULL: row c) in all of them, inputs and outputs alike (the caller holds the
 * stage values on its grid).  desc: dt > 0; eps or eps_cells (per row) > 0.
 * Outputs must not alias the inputs of the same call (y_out may be y, which
 * finish does not read).  Asynchronous on `stream`.
 */
bz_status bz_pr222_stage1(const bz_plan* plan, const bz_imex_desc* desc, const double* y, const int32_t* idx,
                          int32_t ncells, const int32_t* ncells_dev, double* y1, void* stream);
bz_status bz_pr222_stage2(const bz_plan* plan, const bz_imex_desc* desc, const double* y, const double* y1,
                          const double* t1, const int32_t* idx, int32_t ncells, const int32_t* ncells_dev,
                          double* y2, double* a, void* stream);
bz_status bz_pr222_finish(const bz_plan* plan, const bz_imex_desc* desc, const double* a, const double* y2,
                          const double* t2, const int32_t* idx, int32_t ncells, const int32_t* ncells_dev,
                          double* y_out, void* stream);

/*
 * ES-BGK operator of the intermediate layer (Sec. 2.2) and its first-order
 * IMEX step (Sec. 4.3, after Filbet and Jin), FP64, one cell per workgroup:
 *   rho Theta = int (v-u)(x)(v-u) f,  T = tr(Theta)/3,
 *   Tau = (1 - beta) T I + beta Theta,
 *   G[f] = rho det(2 pi Tau)^(-1/2) exp(-(v-u) Tau^-1 (v-u) / 2),
 *   Q_ES(f) = nu (G[f] - f),  nu = rho sqrt(T) / (mu0 (1 - beta)) (the relaxation
 *   rate whose ES-BGK viscosity is the hard-sphere mu = mu0 sqrt(T); the paper
 *   names nu(rho, T) without a formula).
 * IMEX: g = f - dt tr; rho, u, T of g (the invariants of the step);
 *   Sigma = a int v(x)v g + (1 - a) rho (T I + u(x)u), a = eps/(eps + (1-beta) nu dt);
 *   Theta = Sigma/rho - u(x)u;  f_out = c g + (1 - c) G(rho, u, Tau), c = eps/(eps + nu dt).
 * desc: n in {16, 24, 32, 48}, L > 0, beta < 1 (-1/2: Prandtl 2/3), mu0 > 0.
 * f, tr: device FP64 [*][n][n][n], cell c at row idx[c] (idx NULL: row c).
 * q / f_out: device FP64, row c or idx[c] (BZ_SCATTER).  f_out may equal f
 * when the rows written are the rows read; q must not alias f.
 * Asynchronous on `stream`; per-cell results do not depend on the batch.
 */
typedef struct {
  int32_t n;
  double L;
  double beta;
  double mu0;
} bz_esbgk_desc;

bz_status bz_esbgk_collide(const bz_esbgk_desc* desc, const double* f, const int32_t* idx, int32_t ncells,
                           const int32_t* ncells_dev, double* q, int32_t flags, void* stream);
bz_status bz_esbgk_imex_euler(const bz_esbgk_desc* desc, const bz_imex_desc* imex, const double* f,
                              const double* tr, const int32_t* idx, int32_t ncells, const int32_t* ncells_dev,
                              double* f_out, int32_t flags, void* stream);

/*
 * The ES-BGK layer with the second-order PR(2,2,2) IMEX scheme (Sec. 4.3):
 * explicit part -v.grad_x y, implicit part Q_ES(y)/eps.  Each implicit stage
 * Y = R + (h/eps) Q_ES(Y) is solved explicitly like the first-order step
 * (no transport, dt -> h = gamma dt).  Split where the caller evaluates the
 * transport of the stage values:
 *   stage 1:  Y1 = S_ES(y, gamma dt)
 *   [caller:  T1 = v . grad_x Y1]
 *   stage 2:  R2 = y - dt T1 + (1 - 2 gamma) dt Q_ES(Y1)/eps,  Y2 = S_ES(R2, gamma dt),
 *             A = y - (dt/2) T1 + (dt/(2 eps)) Q_ES(Y1)
 *   [caller:  T2 = v . grad_x Y2]
 *   finish:   y_out = A - (dt/2) T2 + (dt/(2 eps)) Q_ES(Y2)
 * Arrays, rows and aliasing as for bz_pr222_*; in the finish y_out may also
 * be `a` itself.
 */
bz_status bz_esbgk_pr222_stage1(const bz_esbgk_desc* desc, const bz_imex_desc* imex, const double* y,
                                const int32_t* idx, int32_t ncells, const int32_t* ncells_dev, double* y1,
                                void* stream);
bz_status bz_esbgk_pr222_stage2(const bz_esbgk_desc* desc, const bz_imex_desc* imex, const double* y,
                                const double* y1, const double* t1, const int32_t* idx, int32_t ncells,
                                const int32_t* ncells_dev, double* y2, double* a, void* stream);
bz_status bz_esbgk_pr222_finish(const bz_esbgk_desc* desc, const bz_imex_desc* imex, const double* a,
                                const double* y2, const double* t2, const int32_t* idx, int32_t ncells,
                                const int32_t* ncells_dev, double* y_out, void* stream);


typedef struct {
  int32_t nx, ny;           /* spatial grid, arrays are row-major [iy][ix] */
  double dx, dy;            /* spacings */
  double mu0, kappa0;       /* mu = mu0 sqrt(T), kappa = kappa0 sqrt(T) (hard spheres) */
  double eta0, eta1, delta0; /* Euler<->kinetic, ES-BGK<->Boltzmann, L1 thresholds */
  int32_t laplacian_u_mode; /* 0: Lap u = Lap ux + Lap uy (as printed); 1: vector norm */
} bz_mask_desc;

enum { BZ_CELL_SOLID = 1, BZ_CELL_FORCE_BOLTZMANN = 2 };
#define BZ_REGIME_SOLID 255

/*
 * Regime update of Algorithm 1 for every cell, in FP64 with a fixed operation
 * order (no contraction):
 *   one-cell stencil clamped at the border (ghost cells copy the nearest
 *   cell), central first differences over 2 dx / 2 dy, 5-point Laplacians
 *   over dx*dy (Sec. 4.5);
 *   xi1 = eps mu/(rho T), xi2 = eps^2 2 kappa^2/(3 rho^2 T^3);
 *   eigenvalues lambda_a, lambda_b, lambda_c of V_eps1 (closed form, Sec. 4.5);
 *   lambda_B = eps^2 (|grad T|^2/T + |grad u|^2 + sqrt((|Lap u|^2 +
 *   |Lap rho/rho|^2)(1+T^2))) (Sec. 3.3);
 *   2 -> 2 iff |lambda_B| > eta1, else 1; 1 -> 2 iff |lambda_B| > eta1, else
 *   1 -> 0 iff all |lambda - 1| <= eta0 and l1dist <= delta0; 0 -> 1 iff some
 *   |lambda - 1| > eta0.  Cells flagged SOLID get 255 and regime_in 255 stays;
 *   FORCE_BOLTZMANN gets 2.
 * Inputs (device, [ny][nx]): rho, ux, uy, T, eps (FP64), regime_in (u8),
 *   l1dist (FP64, NULL: the 1 -> 0 switch never fires), cell_flags (u8, NULL
 *   allowed).
 * Outputs (device): regime_out [ny][nx] u8; boltz_idx int32 [nx*ny]: the
 *   regime-2 cells as ascending linear indices iy*nx+ix; counts int32[2]:
 *   counts[0] = number of regime-2 cells, counts[1] = number of cells whose
 *   inputs are invalid (rho <= 0, T <= 0, eps < 0 or non-finite: those cells
 *   keep regime_in); diag (NULL allowed) FP64 [nx*ny][4] = lambda_a,
 *   lambda_b, lambda_c, lambda_B.  Asynchronous on `stream`.
 */
bz_status bz_realizability_mask(const bz_mask_desc* desc, const double* rho, const double* ux,
                                const double* uy, const double* T, const double* eps,
                                const uint8_t* regime_in, const double* l1dist,
                                const uint8_t* cell_flags, uint8_t* regime_out,
                                int32_t* boltz_idx, int32_t* counts, double* diag, void* stream);

/* Numeric status of a mask evaluation: waits for `stream`, then returns
   BZ_ERR_NUMERIC if counts[1] (the mask's device status word, written by the
   bz_realizability_mask call that took `counts`) reports cells with invalid
   inputs, else BZ_OK.  Those cells kept their regime; the others are valid
   results either way. */
bz_status bz_mask_sync(const int32_t* counts, void* stream);

/*
 * Serving: continuous batching of collision evaluations from several
 * concurrent simulations on one GPU (each dynamic re-partition of a
 * simulation produces a request with its own grid size and cell count).
 *
 * The server carves plan tables and per-request workspaces out of one
 * caller-owned device arena; it never allocates device memory.  Queued
 * requests are admitted, the one with the least estimated work (cells x grid
 * points x passes) first, as soon as their workspace fits in the arena and an
 * in-flight slot is free; a request passed over by more than 8 later ones goes
 * first, and a workspace above a sixteenth of the arena is admitted ahead of
 * that turn only if an eighth of the arena stays free.  Admitted requests run
 * on n_streams streams, one slice per stream at a time, so their work overlaps
 * on the device; a request larger than the slice size runs as consecutive
 * slices, and a free stream takes the next slice of the admitted request with
 * the least work left, so long requests interleave with short ones.  With two
 * or more streams, stream 0 takes only short slices (at most 3 * 2^28 grid
 * points x passes), so a short request never waits for a long slice; a
 * request passed over by more than 32 slice launches goes first.
 * The strategy of a request's plan is that of its slice size.  Plans are cached by descriptor (max_cells is
 * ignored): the host plan is built on a builder thread the first time an
 * operator is requested (meanwhile its requests wait and the others go
 * ahead), its device tables are uploaded into the arena when a request needs
 * them and evicted least-recently-used when idle and memory is short.  A
 * request that does not fit while others run waits for them to finish.
 * Request buffers (f, idx, q) must stay valid and unmodified until
 * bz_serve_poll reports DONE or FAILED.  The server launches on its own
 * streams: work the caller has queued that writes f or idx must be complete,
 * or be covered by ready_event, before the request is admitted.  A request's
 * result does not depend on the other requests in flight.  A request whose
 * descriptor is invalid or whose workspace and tables can never fit in the
 * arena together ends FAILED (err set) without affecting the others; one
 * whose output holds a non-finite value ends FAILED with BZ_ERR_NUMERIC (its
 * output is written).
 */
typedef struct bz_server bz_server;

typedef struct {
  void* arena_dev;      /* device arena, 256-byte aligned, owned by the caller */
  size_t arena_bytes;
  int32_t max_inflight; /* requests on the GPU at once (>= 1) */
  int32_t n_streams;    /* launch streams (1..16), default priority */
  int32_t max_queue;    /* queued requests before bz_serve_submit returns BZ_AGAIN */
  int32_t slice_cells;  /* cells per launch; larger requests run slice by slice, one
                           slice in flight at a time on the least loaded stream, with
                           a workspace of one slice; 0 = by grid size (n = 16: 2048,
                           24: 1024, 32: 512, 48: 256; two dimensions: 4096) */
} bz_server_desc;

typedef struct {
  bz_plan_desc plan;    /* operator (dirs/weights copied at submission for explicit rules) */
  const void* f;        /* device [*][n][n][n], f_dtype */
  int32_t f_dtype;      /* BZ_FP64 | BZ_FP32 */
  const int32_t* idx;   /* device [ncells] or NULL (rows 0..ncells) */
  int32_t ncells;
  void* q;              /* device output as for bz_collide_batch */
  int32_t flags;        /* BZ_SCATTER */
  int32_t client_id;    /* caller's tag, unused by the server */
  void* ready_event;    /* hipEvent_t or NULL: the request's kernels wait for it
                           (hipStreamWaitEvent at admission), so a caller records
                           it on the stream that produced f; it must not be
                           re-recorded or destroyed before the request leaves
                           the QUEUED state */
} bz_request;

enum { BZ_REQ_QUEUED = 0, BZ_REQ_ADMITTED = 1, BZ_REQ_DONE = 2, BZ_REQ_FAILED = 3 };

typedef struct {
  int32_t state;        /* BZ_REQ_* */
  bz_status err;        /* BZ_OK, or the error of a FAILED request */
  uint64_t t_submit_ns, t_admit_ns, t_done_ns; /* steady-clock timestamps */
} bz_result;

typedef struct {
  uint64_t submitted, completed, failed;
  int32_t queued, inflight, plans_cached;
  size_t arena_used, arena_peak;  /* bytes (tables + workspaces) */
  double p50_ms, p99_ms;          /* submit-to-done latency of completed requests */
  double cells_per_s;             /* completed cells / (last done - first submit) */
} bz_server_stats_t;

/* Start a server (one scheduler thread) on the current device. */
bz_status bz_server_create(const bz_server_desc* desc, bz_server** out);
/* Queue a request; *ticket identifies it.  BZ_AGAIN if the queue is full. */
bz_status bz_serve_submit(bz_server* server, const bz_request* req, uint64_t* ticket);
/* BZ_OK with *out filled once the request is DONE or FAILED (the ticket is then
   released), BZ_AGAIN (with the current state) while it is queued or running,
   BZ_ERR_ARG for an unknown ticket. */
bz_status bz_serve_poll(bz_server* server, uint64_t ticket, bz_result* out);
/* Submit-to-done latency percentiles of the completed requests and the
   completed cells per second since the first submission (any pointer may be
   NULL). */
bz_status bz_server_stats(bz_server* server, double* p50_ms, double* p99_ms, double* cells_per_s);
/* The same figures with the request counters and arena use. */
bz_status bz_server_stats_ex(bz_server* server, bz_server_stats_t* out);
/* Run every queued and in-flight request to completion, then free the server. */
bz_status bz_server_destroy(bz_server* server);

/*
 * One time step of the hot path captured as a HIP graph (built once, replayed
 * every step): optionally the kinetic cells' moments from f (below), then
 * bz_realizability_mask on the macro fields, then
 * bz_collide_batch over the regime-2 cells it lists (count read on the GPU,
 * output scattered to rows boltz_idx of q, FP64 projected), then regime_out
 * copied over regime_in so that the next replay continues from the new
 * regimes.  The caller refreshes the contents of the buffers between replays;
 * the pointers are fixed at creation.  The plan must be bound with capacity
 * >= nx*ny and project = 1.  The graph holds the plan's tables and workspace
 * as bound at creation: the plan must not be rebound or destroyed while the
 * step exists, and replays must be ordered on one stream with every other use
 * of the plan (they share its workspace).
 */
typedef struct bz_step bz_step;
typedef struct {
  const double *rho, *ux, *uy, *T, *eps; /* [ny][nx] macro fields */
  uint8_t* regime_in;                    /* [ny][nx], overwritten by each replay */
  const double* l1dist;                  /* or NULL */
  const uint8_t* cell_flags;             /* or NULL */
  uint8_t* regime_out;                   /* [ny][nx] */
  int32_t* boltz_idx;                    /* [nx*ny] */
  int32_t* counts;                       /* [2] as for bz_realizability_mask */
  double* diag;                          /* or NULL */
  const void* f;                         /* [nx*ny][n][n][n], f_dtype */
  int32_t f_dtype;
  double* q;                             /* [nx*ny][n][n][n] FP64; only rows listed are written */
  /* Optional first stage (kinetic_moments != 0): the cells whose regime_in is
     1 or 2 (the kinetic layers, whose f is resident) are listed in kin_idx
     (ascending, count in kin_count[0]) and get rho, ux, uy, T and l1dist
     recomputed from f on the plan's velocity grid (bz_cell_moments), so the
     mask's 1 -> 0 switch sees each kinetic cell's own distance to
     equilibrium; those five arrays are then written by the replay (l1dist
     must be given).  Fluid cells keep the caller's fields. */
  int32_t kinetic_moments;
  int32_t* kin_idx;                      /* [nx*ny] */
  int32_t* kin_count;                    /* [1] */
} bz_step_buffers;

bz_status bz_step_create(const bz_plan* plan, const bz_mask_desc* mask, const bz_step_buffers* bufs,
                         bz_step** out);
bz_status bz_step_launch(bz_step* step, void* stream);
bz_status bz_step_destroy(bz_step* step);

#ifdef __cplusplus
}
#endif

#endif /* BZ_H */
