/*
 * nep.h -- C ABI of the MI355X (gfx950) contour-integral eigensolver.
 *
 * The library computes the eigenvalues of a holomorphic matrix function T(z)
 * (T(lambda) x = 0, eq (1.1) of Xi & Sun, "Parallel multi-step contour integral
 * methods for nonlinear eigenvalue problems") that lie in a rectangle Omega,
 * following pmCIMb (Section 3.2):
 *
 *   Step 1   cover Omega with equal cells, replace each cell by its circumscribed
 *            disk (Section 3), and at the N trapezoidal nodes of every circle solve
 *            T(z_j) X_j = [F | V] (eq (2.4)); form the N- and N/2-point rules of P f
 *            (eq (2.3)) and the ratio indicator (eq (3.1)); flag disks with
 *            I > tol_ind                                       -> nep_indicator
 *   Step 2   Beyn's extraction on flagged disks from the moments C0, C1
 *            (eqs (2.6)-(2.8), (3.2)-(3.3)) and the keep-inside-the-cell filter
 *            (Step 2.f)                                         -> nep_beyn
 *   Step 3   verification of each candidate by sigma_min(T(lambda)) < tol_ver
 *            (Step 3, with the smallest singular value in place of the smallest
 *            eigenvalue)                                        -> nep_verify
 *   (added)  candidates moved to the eigenvalue they approximate by the two-sided
 *            Rayleigh functional, then verified                 -> nep_refine
 *
 * Conventions for every entry point
 *   - Complex numbers are interleaved (re, im) pairs of IEEE doubles, the layout of
 *     C99 double _Complex, std::complex<double> and torch.complex128.
 *   - Matrices are dense and row-major: element (i, j) of an n x m block sits at
 *     offset i*m + j.
 *   - "_dev" pointers are device (HBM) addresses on the current HIP device;
 *     every other pointer is host memory.  Device pointers are borrowed: the caller
 *     keeps them valid for the lifetime stated on each call.  The library allocates
 *     its own device workspace in nep_plan and frees it in nep_destroy.
 *   - No exceptions cross the ABI.  Every call returns a nep_status; on a negative
 *     status, nep_last_error() holds a human-readable message.  Warnings
 *     (positive statuses) mean the outputs are complete but some node or disk was
 *     handled conservatively (see each status).
 *   - A plan is not thread-safe.  All work of a plan runs, in order, on the HIP
 *     stream given at nep_plan; calls return after that stream has produced the
 *     host outputs.  Use one plan per stream.
 */
#ifndef NEP_H
#define NEP_H

#include <stddef.h>
#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum nep_status {
  NEP_OK = 0,
  NEP_WARN_SINGULAR_NODE = 1,   /* a node matrix had an exactly zero pivot or a non-finite
                                   solution; its disk was flagged conservatively           */
  NEP_WARN_REFINE_FALLBACK = 2, /* mixed precision: some node did not converge within
                                   max_refine sweeps and was re-solved in complex128       */
  NEP_WARN_SATURATED = 3,       /* Beyn: some disk kept p = L singular values (the rank test
                                   may have been cut by the probe count)                   */
  NEP_ERR_ARG = -1,             /* invalid argument (null pointer, size, option)           */
  NEP_ERR_NOMEM = -2,           /* device or host allocation failed                        */
  NEP_ERR_HIP = -3,             /* a HIP runtime call failed                               */
  NEP_ERR_NONFINITE = -4,       /* non-finite data where the method cannot proceed         */
  NEP_ERR_CAPACITY = -5,        /* an output or workspace capacity would be exceeded       */
  NEP_ERR_STATE = -6            /* call order violated (e.g. nep_beyn before a sweep)      */
} nep_status;

/* Scalar functions phi_k of the split form T(z) = sum_k phi_k(z) A_k. */
enum {
  NEP_PHI_ONE = 0,            /* 1                                  */
  NEP_PHI_Z = 1,              /* z                                  */
  NEP_PHI_Z2 = 2,             /* z^2                                */
  NEP_PHI_NEG_Z = 3,          /* -z                                 */
  NEP_PHI_EXP_NEG_TAU_Z = 4   /* exp(-tau z), tau = phi_param[k]    */
};

/* Arithmetic of the node LU factorisations. */
enum {
  NEP_FP64 = 0,        /* complex128 LU                                                */
  NEP_FP32_REFINE = 1  /* complex64 LU, then complex128 residual iterative refinement    */
};

/* Pivot choice of the node LU factorisations (both give P T(z_j) = L U).
 *   NEP_PIVOT_PARTIAL     LAPACK-style partial pivoting (largest |Re|+|Im| in the
 *                         column, first row on ties), one workgroup per panel
 *   NEP_PIVOT_TOURNAMENT  each 64-column panel picks its pivot rows by a tournament:
 *                         128-row chunks run partial pivoting in parallel and their
 *                         winners are merged pairwise (communication-avoiding LU);
 *                         pays off when few matrices are factored at once        */
enum {
  NEP_PIVOT_PARTIAL = 0,
  NEP_PIVOT_TOURNAMENT = 1
};

/* The nonlinear eigenvalue problem T(lambda) x = 0 (eq (1.1)) in split form
 * T(z) = sum_{k < nterms} phi_{phi_kind[k]}(z) A_k, the structure of the paper's
 * appendix routine that generates T(z) (a quadratic T0 + z T1 + z^2 T2).
 *   n          matrix order, 1 <= n <= 4096
 *   nterms     1 .. 4 split terms, or 0 for a problem written by an assembler
 *              (nep_set_assembler, below)
 *   A_dev[k]   device pointer to A_k, complex128 row-major n x n; NULL means A_k = I
 *              (never materialised).  Borrowed until nep_destroy.
 *   phi_kind   host array of nterms NEP_PHI_* codes (copied at nep_plan)
 *   phi_param  host array of nterms parameters (tau), or NULL (copied)        */
typedef struct nep_problem {
  int n;
  int nterms;
  const void* const* A_dev;
  const int* phi_kind;
  const double* phi_param;
} nep_problem;

/* A problem with nterms = 0 has no split form: T(z) is written by a caller-supplied
 * assembler (the general matrix function of eq (1.1), as the paper's appendix routine
 * that generates T(z) leaves it), registered with nep_set_assembler before the first
 * sweep.  A_dev, phi_kind and phi_param are then ignored.  Such problems need
 * precision NEP_FP64 (the mixed path's complex128 residual uses the split
 * coefficients), and nep_refine takes them with iters = 0 only.
 *
 * nep_assemble_fn -- write T(z_b) for b < nb, complex128 row-major n x n, at
 * W_dev + b * mstride (complex elements), for the nodes z_dev[b] (device complex128).
 * The function must only enqueue device work on `stream` (no synchronisation, no
 * allocation, no host reads of device data): it is also recorded into HIP graphs.
 * It returns 0 on success; any other value aborts the call with NEP_ERR_ARG.      */
typedef int (*nep_assemble_fn)(void* ctx, int n, const void* z_dev, int nb, void* W_dev, long long mstride,
                               hipStream_t stream);

/* Omega = [x0, x1] x [y0, y1] split into nx x ny equal cells (Section 3).  Cell
 * (ix, iy) has centre (x0 + (2 ix + 1) hx, y0 + (2 iy + 1) hy), half-widths
 * hx = (x1 - x0) / (2 nx), hy = (y1 - y0) / (2 ny), and its disk has radius
 * sqrt(hx^2 + hy^2).  Disks are numbered ix * ny + iy within a problem, and
 * problems follow each other in the plan's global disk numbering.            */
typedef struct nep_region {
  double x0, x1, y0, y1;
  int nx, ny;
} nep_region;

/* Method parameters.
 *   N          trapezoidal nodes per circle (even, 4 <= N <= 256), eq (2.3)
 *   s          probe columns of F for the indicator (1 <= s <= 8)
 *   L          probe columns of V for Beyn's moments (0 <= L <= 32; 0 = no moments)
 *   tol_ind    flag a disk iff its indicator I > tol_ind (Step 1.c)
 *   tol_svd    keep singular values sigma > tol_svd (Step 2.d)
 *   tol_ver    accept lambda iff sigma_min(T(lambda)) < tol_ver (Step 3)
 *   precision  NEP_FP64 or NEP_FP32_REFINE
 *   max_refine maximum refinement sweeps for NEP_FP32_REFINE (0..8)
 *   batch      node matrices factored together (0 = chosen by the library: a workspace
 *              of 12% of the device memory per worker stream, at most 2048 matrices)
 *   streams    worker streams the batches alternate over (1 .. 3; 0 = 2), each with a
 *              workspace of its own: with two or more, one batch's panel steps
 *              overlap another batch's trailing updates
 *   pivot      NEP_PIVOT_PARTIAL (0) or NEP_PIVOT_TOURNAMENT (1)
 *   graph      1: nep_indicator captures its device work (every batch on both worker
 *              streams, the sums and the indicator) into a HIP graph on its first
 *              call and replays it while the probe pointers stay the same; the
 *              mixed-precision refinement then always runs max_refine masked sweeps
 *              and the complex128 re-solves it asks for run after the replay.
 *              Results equal the eager path's bit for bit; per-phase timings are
 *              not available (only ms_total).  0: eager launches.              */
typedef struct nep_options {
  int N;
  int s;
  int L;
  double tol_ind;
  double tol_svd;
  double tol_ver;
  int precision;
  int max_refine;
  int batch;
  int streams;
  int pivot;
  int graph;
} nep_options;

/* Counters and phase timings of the last call on a plan (device time measured with
 * HIP events on the plan's stream, milliseconds).                              */
typedef struct nep_stats {
  int64_t node_solves;       /* (problem, disk, node) units of the last sweep        */
  int64_t lu_count;          /* LU factorisations in the last sweep / verify          */
  double lu_flops;           /* sum of 8 n^3 / 3 over those LUs (real flops)          */
  int64_t refine_sweeps;     /* residual sweeps run (mixed precision)                 */
  int64_t refine_fallbacks;  /* nodes re-solved in complex128                         */
  int64_t singular_nodes;    /* nodes with a zero pivot or non-finite solution        */
  double ms_total;           /* the whole last call                                   */
  double ms_assemble;        /* T(z_j) assembly                                       */
  double ms_lu;              /* LU factorisations (panel + row exchange + update)      */
  double ms_solve;           /* triangular solves                                     */
  double ms_refine;          /* residuals + correction solves                         */
  double ms_sums;            /* quadrature sums, profiles, indicators                 */
  double ms_gemm;            /* the paired trailing update alone (timed launches)      */
  int64_t gemm_launches;     /* its timed launches (the first 2048 of the call)       */
  double gemm_flops;         /* its algorithmic flops over those launches             */
  double ms_gemm_busy;       /* the union of those launches' intervals: ms_gemm counts
                                twice the time two worker streams' launches overlap   */
} nep_stats;

typedef struct nep_plan nep_plan_t;

/* nep_plan -- validate the inputs, build the cover, nodes z_j = c + r e^{i theta_j}
 * (theta_j = 2 pi (j-1)/N, j = 1..N) and weights w_j = (r/N) e^{i theta_j} of every
 * disk (eq (2.3), Section 3), choose the batching and allocate the device workspace.
 *   probs, nprob  the problems (nprob >= 1); coefficient buffers are borrowed and
 *                 must stay valid and unchanged until nep_destroy
 *   regs          one region per problem
 *   opt           method parameters (copied)
 *   stream        the HIP stream all work of this plan runs on (0 = null stream)
 *   out           receives the plan; set to NULL on failure
 * Errors: NEP_ERR_ARG (bad sizes/options), NEP_ERR_NOMEM, NEP_ERR_HIP.            */
nep_status nep_plan(const nep_problem* probs, int nprob, const nep_region* regs,
                    const nep_options* opt, hipStream_t stream, nep_plan_t** out);

/* nep_indicator -- Step 1 over every disk of every problem, plus the Beyn moments
 * of Step 2.b when V is given (the same nodes serve both, so the moments come from
 * the same factorisations: eqs (3.2)-(3.3) with the garbled factor of eq (3.3) read
 * as the node z_j).
 *   F_dev[p]   device, complex128 n_p x s, the indicator probes (unit columns)
 *   V_dev      NULL, or V_dev[p] = device complex128 n_p x L (Beyn probes)
 *   ind        host double [total_disks * s]: I_q of eq (3.1) per probe column, read
 *              as || P f|_N ./ P f|_{N/2} ||_2 / sqrt(n) (elementwise ratio, each entry
 *              and the norm scaled so that no square overflows or underflows); a
 *              non-finite ratio is reported as +inf.  A column whose two sums are both
 *              at most 2^-30 times their summand sizes, S_N = sum_j |w_j| ||x_j[:, q]||
 *              and S_half = sum over the 1-based even nodes of 2 |w_j| ||x_j[:, q]||,
 *              is reported as 0: both sums are then rounding noise (a normwise error
 *              of n u kappa per node solution, with n <= 2^12 and kappa <= 2^10 far
 *              from every eigenvalue, is at most 2^-31 of S), and so is their ratio
 *   flags      host uint8 [total_disks]: 1 iff max_q I_q > tol_ind, or one of the
 *              disk's nodes had an exact zero pivot (complex128 LU) or a non-finite
 *              solution entry (the conservative flag of NEP_WARN_SINGULAR_NODE); in
 *              mixed precision the complex128 re-solve decides a zero pivot
 *   profiles   host double [total_disks * N * s] or NULL: ||x_j[:, q]||_2 per node
 * The half rule uses the 1-based even nodes x_2, x_4, ..., x_N with weights 2 w_j.
 * Returns NEP_OK, NEP_WARN_SINGULAR_NODE or NEP_WARN_REFINE_FALLBACK, or an error. */
nep_status nep_indicator(nep_plan_t* plan, const void* const* F_dev, const void* const* V_dev,
                         double* ind, uint8_t* flags, double* profiles);

/* nep_beyn -- Step 2.c-2.f on the listed disks: thin SVD C0 = U S W^H, p =
 * #{sigma > tol_svd}, D = U_0^H C1 W_0 S_0^{-1} (eq (2.8)), eig(D), and the
 * ownership filter of Step 2.f.
 *   disk_ids, ndisks   global disk indices (host)
 *   V_dev      NULL: reuse the moments of the last nep_indicator (which must have had
 *              V); otherwise per-problem device V blocks (n_p x L), and the listed disks
 *              are swept again with them
 *   eig        host complex128 [ndisks * L]: eigenvalues of D, first p[i] valid
 *   p          host int32 [ndisks]
 *   sv         host double [ndisks * L]: singular values of C0, descending
 *   keep       host uint8 [ndisks * L] or NULL: 1 iff eigenvalue k of disk i lies in the
 *              cell that owns it (strict inside test; a value within 1e-6 max(1,|l|) of
 *              an edge shared by two cells belongs to the neighbour with the smaller
 *              index, a value on the outer boundary of Omega to its only cell; the band
 *              exceeds the quadrature error of eigenvalues that lie on cell edges)
 *   eigvec_dev NULL or device complex128 [ndisks * n * L]: eigenvectors U_0 s_k (unit
 *              2-norm, column k of the n x L block of disk i; problems of one call must
 *              then share n)
 * Returns NEP_OK, NEP_WARN_SATURATED (some p == L), or an error.                  */
nep_status nep_beyn(nep_plan_t* plan, const int32_t* disk_ids, int ndisks,
                    const void* const* V_dev, void* eig, int32_t* p, double* sv,
                    uint8_t* keep, void* eigvec_dev);

/* nep_verify -- Step 3: sigma_min(T(lambda_i)) in complex128 for m candidates, from an
 * LU of T(lambda_i) and inverse iteration on T^H T (the estimate never undershoots
 * sigma_min); accepted[i] = sigma_min < tol_ver.
 *   prob_ids   host int32 [m]: problem of each candidate
 *   lam        host complex128 [m]
 *   sigma_min  host double [m]
 *   accepted   host uint8 [m]
 * Errors: NEP_ERR_ARG.                                                            */
nep_status nep_verify(nep_plan_t* plan, const int32_t* prob_ids, const void* lam, int m,
                      double* sigma_min, uint8_t* accepted);

/* nep_refine -- candidates moved onto the eigenvalues they approximate, then verified
 * as by nep_verify.  Not a step of the paper's method: Beyn's candidates carry the
 * quadrature error of their disk (largest for eigenvalues near the circle), and a cell
 * split by the saturation remedy (end of Section 3.2) can leave one there.  Each of
 * `iters` updates runs the inverse iteration of nep_verify at lambda, takes its left
 * and right singular-vector estimates u, v, forms a_k = u^H A_k v on the device and
 * moves lambda to the nearby root of the two-sided Rayleigh functional
 * u^H T(rho) v = sum_k phi_k(rho) a_k (Newton on the host); a final inverse iteration
 * gives sigma_min.  Each candidate returns the point of smallest sigma_min met, so
 * the result is never worse than the input; iters = 0 is nep_verify.
 *   prob_ids   host int32 [m]: problem of each candidate
 *   lam        host complex128 [m], in: candidates, out: refined values
 *   iters      0 .. NEP_REFINE_MAX_ITERS (2 takes a candidate within 1e-4 relative of
 *              a simple eigenvalue to rounding level)
 *   sigma_min  host double [m]: at the returned value
 *   accepted   host uint8 [m]: sigma_min < tol_ver
 *   vec        NULL, or host complex128 [m * ldv]: row i receives the right singular
 *              vector of sigma_min(T(lambda_i)) at the returned value (the eigenvector
 *              of pmCIMa's Step 2, Section 3.1): unit 2-norm, its largest-modulus
 *              entry real and positive; entries past the candidate's n are untouched;
 *              zeros where the LU of T(lambda_i) met an exact zero pivot (sigma 0)
 *   ldv        >= n of every listed candidate's problem when vec is given
 * Cost: (iters + 1) complex128 LUs per candidate.  Errors: NEP_ERR_ARG.           */
#define NEP_REFINE_MAX_ITERS 8
nep_status nep_refine(nep_plan_t* plan, const int32_t* prob_ids, void* lam, int m, int iters,
                      double* sigma_min, uint8_t* accepted, void* vec, int ldv);

/* nep_set_assembler -- register the assembler of problem `problem` (which must have
 * nterms = 0) and its context pointer (borrowed until nep_destroy or the next call).
 * A captured sweep graph of the plan is dropped (the next graph-mode sweep captures
 * again).  Errors: NEP_ERR_ARG.  Sweeps and verifications of a plan with an
 * unregistered assembler fail with NEP_ERR_STATE.                                */
nep_status nep_set_assembler(nep_plan_t* plan, int problem, nep_assemble_fn fn, void* ctx);

/* An assembler shipped with the library: the elementwise delay problem
 * T(z) = -z I + A0 + A1 .* exp(-tau .* z), each entry of A1 with a delay of its own
 * (n^2 distinct delays: no short split form).  Pass nep_assemble_elementwise_delay as
 * the function and a nep_elementwise_delay as the context.
 *   A0_dev, A1_dev  device complex128 row-major n x n;  tau_dev  device double n x n */
typedef struct nep_elementwise_delay {
  int n;
  const void* A0_dev;
  const void* A1_dev;
  const double* tau_dev;
} nep_elementwise_delay;
int nep_assemble_elementwise_delay(void* ctx, int n, const void* z_dev, int nb, void* W_dev, long long mstride,
                                   hipStream_t stream);

/* An assembler shipped with the library: the scattering poles of the sound-soft unit
 * disk (Section 4.2).  T(k) = (I + K_n(k)) / 2 with K the double-layer operator
 * (kernel 2 dPhi/dnu(y), Phi = (i/4) H0(k |x - y|)) on n equispaced points of the
 * unit circle (n even), discretised by Kress's Nystrom rule with the logarithmic
 * splitting; J1 and Y1 from their power series, used for |k| <= 10 (at |k| = 10 about
 * 1e-9 of the sums is lost to cancellation).  Nodes with |k| > 10 get a NaN matrix,
 * which nep_indicator reports as NEP_WARN_SINGULAR_NODE with the disk flagged.  The
 * context is unused (NULL).  Its singular points in the lower half-plane are the
 * zeros of the Hankel functions H_m, each double (modes m and -m).              */
int nep_assemble_circle_double_layer(void* ctx, int n, const void* z_dev, int nb, void* W_dev, long long mstride,
                                     hipStream_t stream);

/* nep_copy_sums -- copy the quadrature sums of disks [first, first + count) of the last
 * sweep to host buffers (any may be NULL): PfN, PfN2 as n x s, C0, C1 as n x L per disk,
 * complex128 row-major, disks back to back.  All listed disks must share n.        */
nep_status nep_copy_sums(nep_plan_t* plan, int first, int count, void* PfN, void* PfN2,
                         void* C0, void* C1);

/* nep_dedup -- merge candidates closer than rel * max(1, |lambda|): of a close pair the
 * one with the smaller sigma keeps its slot (the final list of Step 3 after values found
 * from two neighbouring disks).  Host only; keep[i] = 1 for survivors.             */
nep_status nep_dedup(const void* lam, const double* sigma, int m, double rel, uint8_t* keep);

/* nep_merge -- pmCIMa's merge of approximate eigenvalues (Section 3.1, the remark after
 * the algorithm: near an eigenvalue several small cells are flagged, and their centres
 * are merged).  The first centre not yet taken gathers every untaken centre closer than
 * tol_eps (absolute, strict), and the group's mean (summed in list order) is one merged
 * value; groups are formed in list order and each centre joins one group.
 *   centres  host complex128 [m];  merged  host complex128 [m] (the first *count valid)
 *   group    host int32 [m] or NULL: the merged value each centre joined
 * Host only.  Errors: NEP_ERR_ARG.                                                    */
nep_status nep_merge(const void* centres, int m, double tol_eps, void* merged, int* count, int32_t* group);

/* nep_own -- Step 2.f's keep-inside-the-cell rule across cells of different sizes (the
 * saturation remedy at the end of Section 3.2 splits saturated cells, so candidates come
 * from cells of several levels).  Candidate i was produced by the cell
 * cells[4i .. 4i+3] = (x0, x1, y0, y1).  The distinct producing cells are ordered by
 * (x0, y0); a candidate belongs to the first of them that contains it within
 * band * max(1, |lambda|) (closed), and owned[i] = 1 iff that cell produced it: a value
 * on an edge shared by two cells is kept once, by the cell with the smaller (x0, y0).
 *   cells  host double [4 m];  lam  host complex128 [m];  owned  host uint8 [m]
 * Host only.  Errors: NEP_ERR_ARG.                                                    */
nep_status nep_own(const double* cells, const void* lam, int m, double band, uint8_t* owned);

/* ---------------------------------------------------------------- learned screener/* ---------------------------------------------------------------- learned screener
 * A small network (not part of the paper's method) that orders the screening of the
 * four children of a flagged parent cell from the parent's node profile
 * ||T(z_j)^{-1} f||, j = 1..32.  It never decides a flag: every child is still swept.
 * Network: 32 -> 128 -> 128 -> 4, ReLU after the hidden layers, sigmoid outputs, fp32.
 * Parameters (nep_mlp_param_count() = 21252 floats, device): for each layer W
 * (in x out, row-major) then b (out).  Samples are rows of 32 features; targets are
 * rows of 4 values in {0, 1}.  idx (device int32, B entries) selects the rows of X (and
 * Y) that form the batch, or NULL for rows 0..B-1.  work is caller-allocated device
 * memory of nep_mlp_workspace_floats(B) floats.  All calls run on `stream`.          */
int nep_mlp_param_count(void);
size_t nep_mlp_workspace_floats(int B);
/* probs (device, B x 4) = sigmoid(network(X[idx]))                                    */
nep_status nep_mlp_forward(const float* params_dev, const float* X_dev, const int32_t* idx_dev, int B,
                           float* probs_dev, float* work_dev, hipStream_t stream);
/* nep_mlp_forward_noalloc -- nep_mlp_forward for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that forbid
 * allocation): the same kernels, with the activations in a library-owned device array
 * of NEP_MLP_NOALLOC_MAX_B x 260 floats (4.3 MB) per GPU, kept until the process ends.
 * No allocation happens in the call.  All calls on one GPU share that array: calls that
 * overlap in time on one GPU (other streams or threads) race and must be serialised by
 * the caller.  Errors: NEP_ERR_ARG, NEP_ERR_CAPACITY (B > NEP_MLP_NOALLOC_MAX_B),
 * NEP_ERR_HIP.                                                                       */
#define NEP_MLP_NOALLOC_MAX_B 4096
nep_status nep_mlp_forward_noalloc(const float* params_dev, const float* X_dev, const int32_t* idx_dev, int B,
                                   float* probs_dev, hipStream_t stream);
/* grad (device, 21252) = gradient of the mean binary cross-entropy over the batch and
 * the 4 outputs; *loss (host, or NULL) receives that mean (the call then synchronises) */
nep_status nep_mlp_grad(const float* params_dev, const float* X_dev, const float* Y_dev, const int32_t* idx_dev,
                        int B, float* grad_dev, float* loss, float* work_dev, hipStream_t stream);
/* one Adam step (bias-corrected, step counts from 1) on params with moments m, v      */
nep_status nep_mlp_adam(float* params_dev, const float* grad_dev, float* m_dev, float* v_dev, int step, float lr,
                        float beta1, float beta2, float eps, hipStream_t stream);
/* X (device, rows x ncol) = (log10(profiles) - mean) / sd per column; when stat_rows is
 * given, mean and sd are first computed over those rows (the training rows), otherwise
 * the given mean/sd (device, ncol) are used                                          */
nep_status nep_mlp_features(const double* profiles_dev, int rows, int ncol, const int32_t* stat_rows_dev,
                            int nstat, float* mean_dev, float* sd_dev, float* X_dev, hipStream_t stream);

/* nep_mfma_peak -- the device's matrix-core rate, measured (the check of the roofline
 * denominators): 1024 workgroups of four waves each issue independent chains of the
 * 16x16x4 MFMA of the LU's trailing update (precision NEP_FP64: f64; NEP_FP32_REFINE:
 * f32) for `iters` iterations on the null stream; *tflops receives the dense rate in
 * TFLOP/s (2 * 16 * 16 * 4 flops per instruction).  Allocates and frees 8 KB.
 * Errors: NEP_ERR_ARG, NEP_ERR_NOMEM, NEP_ERR_HIP.                                  */
nep_status nep_mfma_peak(int precision, int iters, double* tflops);

/* Sizes of a plan: total disks, and the first global disk of problem p.             */
int nep_total_disks(const nep_plan_t* plan);
int nep_disk_offset(const nep_plan_t* plan, int problem);

/* Counters and timings of the last call.                                            */
nep_status nep_get_stats(const nep_plan_t* plan, nep_stats* out);

/* Release the plan and its device workspace (NULL is ignored).                      */
void nep_destroy(nep_plan_t* plan);

/* Messages.                                                                         */
const char* nep_status_str(int status);
const char* nep_last_error(const nep_plan_t* plan);

#ifdef __cplusplus
}
#endif
#endif /* NEP_H */
