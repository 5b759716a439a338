/*
 * infft.h -- C ABI of the MI355X (gfx950) direct inverse NFFT library.
 *
 * Method: M. Kircheis, D. Potts, "Direct inversion of the nonequispaced fast Fourier
 * transform".  Notation follows the paper:
 *   M      number of Fourier coefficients per dimension (even), k = -M/2 .. M/2-1
 *   N      number of nodes x_j in [-1/2, 1/2)^d (nodes outside are wrapped onto the torus)
 *   sigma  oversampling factor, M_sigma = sigma M (must be an even integer)
 *   m      window cut-off: the truncated window reaches 2m+1 grid points per dimension
 *   A      nonequispaced Fourier matrix (1.3);  A ~ B F D  (Section 2.1, (2.4)-(2.6))
 *
 * Window: Kaiser-Bessel with shape b = pi (2 - 1/sigma); D = diag(1/I_0(m sqrt(b^2 -
 * (2 pi k / M_sigma)^2))) (the paper names the window family in Remark 2.1 without a formula).
 * d-dimensional problems (d = 1, 2) use the tensor product of the 1-D factors.
 *
 * Data layouts (all device pointers unless stated otherwise):
 *   x      float64 [N][d], caller order, row-major.
 *   fhat   coefficients, [nrhs][M_0]...[M_{d-1}], centred index k_t + M_t/2 ascending,
 *          last dimension fastest, right-hand sides outermost.
 *   f      samples, [nrhs][N] in the caller's node order.
 *   complex numbers are interleaved (re, im): complex64 for INFFT_F32 plans, complex128 for
 *          INFFT_F64 plans.
 *
 * Ownership: the caller owns every buffer it passes; pointers are only read/written during the
 * call's stream work.  A plan made by nfft_plan owns its device memory (allocated there, freed by
 * nfft_plan_destroy); a plan made by nfft_plan_ws lives in a workspace the caller owns and keeps
 * alive until nfft_plan_destroy, and no call on it allocates device memory.  Either keeps a copy
 * of the nodes, so `x` may be freed after nfft_plan / nfft_set_nodes return.
 *
 * Streams: every call enqueues work on the plan's stream (a hipStream_t passed as void*; NULL =
 * the default stream) and returns without synchronising, except nfft_plan_status,
 * nfft_plan_destroy and nfft_plan (which waits for its own set-up work).
 *
 * Errors: every call returns INFFT_OK (0) or a negative code; nothing throws across the ABI.
 * infft_last_error() returns a thread-local message for the last failing call.  Conditions found
 * on the device (non-finite nodes, failed local solves, empty I(l)) are counted in a device
 * status block read by nfft_plan_status.
 */
#ifndef INFFT_H
#define INFFT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define INFFT_OK 0
#define INFFT_EINVAL (-1)    /* invalid argument: M odd or <= 0, sigma M not an even integer,
                                m outside 2..8, 2m+2 > M_sigma, N <= 0, d not 1 or 2, null
                                pointer, nrhs < 1, unsupported FFT length */
#define INFFT_ENOMEM (-2)    /* device allocation failed */
#define INFFT_EDEVICE (-3)   /* HIP runtime error */
#define INFFT_ESINGULAR (-4) /* status: a local solve met a non-positive pivot */
#define INFFT_ESTATE (-5)    /* call out of order, e.g. infft_apply before infft_precompute_B */

#define INFFT_F32 0 /* complex64 data; FP32 spreading, FFT and accumulation */
#define INFFT_F64 1 /* complex128 data; FP64 throughout */

typedef struct infft_plan_s* infft_plan;

typedef struct {
    int precision;   /* INFFT_F32 or INFFT_F64 (default INFFT_F64) */
    int max_rhs;     /* right-hand sides processed per internal pass (default 1); larger nrhs
                        are processed in chunks */
    double rho;      /* ridge of the local least-squares problems (default 1e-8): the solve
                        minimises ||L_l b - e_l||^2 + lambda ||b||^2 with
                        lambda = rho * trace(L_l^* L_l) / |I(l)| */
    int tile[2];     /* spreading tile in grid cells per dimension (0 = automatic) */
    int inverse_kernel; /* kernel of the inverse (B optimisation, infft_apply, infft_apply_adjoint):
                           INFFT_KERNEL_WINDOW (default): D of the window, as in the NFFT;
                           INFFT_KERNEL_DIRICHLET: Remark 3.19, w_hat = 1 for |k| < M/2 and the
                           entry of k = -M/2 set to zero, so K is the Dirichlet kernel (3.23)
                           divided by M_sigma (the NFFT and its adjoint keep the window) */
    int work_slots;  /* sets of transform work buffers (oversampled grid, FFT scratch, spreading
                        halos), 1..8 (default 1; 0 means 1).  nfft_set_slot picks the set later
                        calls use, so calls on different slots and streams may run concurrently */
    int large_mib;   /* workspace plans (nfft_plan_ws) only: MiB of the workspace kept for the local
                        problems of Algorithm 3.17 beyond the register tiers (more than 64 members in
                        1-D, 32 in 2-D; a problem of n members needs 16 n^2 + 40 n bytes); 0 means
                        256.  Ordinary plans size that memory when needed (must be 0 there). */
    int ansatz1;     /* workspace plans only: 1 places the work arrays and inner plans of
                        infft_precompute_Bstar in the workspace (d = 1; must be 0 otherwise) */
    int reserved[2];
} infft_options;

#define INFFT_KERNEL_WINDOW 0
#define INFFT_KERNEL_DIRICHLET 1

typedef struct {
    int64_t nonfinite_nodes;  /* nodes with a NaN/Inf coordinate (counted; the coordinate is taken as 0) */
    int64_t failed_solves;    /* local problems whose Cholesky met a pivot <= 0 */
    int64_t empty_columns;    /* grid indices l with empty I(l): zero column of B_opt */
    int64_t oversized;        /* local problems not solved (zero columns): under graph capture,
                                 problems beyond the register tiers whose set differs from the one
                                 recorded by the last infft_precompute_B outside capture; for batch
                                 plans under capture, every problem beyond 64 members */
    int64_t min_members;      /* min |I(l)| over non-empty l of the last precompute */
    int64_t max_members;      /* max |I(l)| */
    int32_t bopt_ready;       /* 1 after a successful infft_precompute_B for the current nodes */
    int32_t max_supported;    /* largest |I(l)| the local solver handles (INT32_MAX: limited
                                 only by device memory, 16 |I(l)|^2 bytes for the largest) */
} infft_status;

/* Fills *o with the defaults listed above. */
void infft_default_options(infft_options* o);

/* Creates a plan for d-dimensional problems with M[0..d-1] coefficients, N nodes,
 * oversampling sigma and cut-off m, and runs the node preprocessing for x (N x d float64,
 * device).  Precomputes the deconvolution factors D (2.4), FFT twiddles and the kernel tables
 * used by infft_precompute_B.  stream: hipStream_t (void*), NULL for the default stream.
 * On success *out holds the plan; on failure *out is NULL. */
int nfft_plan(infft_plan* out, int d, const int64_t* M, int64_t N, double sigma, int m,
              const double* x, const infft_options* opts, void* stream);

/* Device bytes a plan made by nfft_plan_ws with these arguments occupies (host only: no device
 * work, no allocation).  The same validation as nfft_plan; *bytes = 0 on failure.  The size covers
 * the nodes and their sorted copies, the plan tables, work_slots sets of transform buffers for
 * max_rhs right-hand sides, B_opt, the solver lists, opts->large_mib MiB (256 if 0) for local
 * problems beyond the register tiers, and with opts->ansatz1 the work arrays and inner plans of
 * Algorithm 3.10. */
int nfft_plan_workspace_bytes(int d, const int64_t* M, int64_t N, double sigma, int m,
                              const infft_options* opts, size_t* bytes);

/* As nfft_plan, with every device buffer of the plan placed in `workspace` (device memory the
 * caller allocated, 256-byte aligned, at least nfft_plan_workspace_bytes long; INFFT_ENOMEM if
 * shorter).  Neither this call nor any later call on the plan allocates device memory: the local
 * problems of Algorithm 3.17 beyond the register tiers use the part sized by opts->large_mib
 * (INFFT_ENOMEM from infft_precompute_B if a problem does not fit), infft_autotune a buffer placed
 * here, and infft_precompute_Bstar the arrays placed when opts->ansatz1 is 1 (INFFT_ESTATE
 * otherwise).  The workspace must stay allocated until nfft_plan_destroy, which does not free it. */
int nfft_plan_ws(infft_plan* out, int d, const int64_t* M, int64_t N, double sigma, int m,
                 const double* x, const infft_options* opts, void* workspace, size_t workspace_bytes,
                 void* stream);

/* Replaces the node set (same N) and reruns the node preprocessing: wrap onto the torus,
 * stencil base l0 = ceil(M_sigma x - m) and offset per dimension, sort into grid tiles, and the
 * grid-index -> node lists I(l) of (3.29).  Invalidates B_opt. */
int nfft_set_nodes(infft_plan p, const double* x);

/* Changes the stream subsequent calls enqueue on. */
int nfft_set_stream(infft_plan p, void* stream);

/* Selects the set of work buffers (0 .. work_slots-1) that subsequent nfft_trafo, nfft_adjoint,
 * infft_apply, infft_apply_adjoint and nfft_grad_x calls use.  Those calls write nothing else of
 * the plan, so calls on different slots, enqueued on different streams, may overlap on the device
 * (the B optimisation and the node preprocessing use none of these buffers; the caller orders them
 * against the transforms that read their results).  Calls that share a slot must be ordered by the
 * caller.  INFFT_EINVAL for a slot out of range and for batch plans. */
int nfft_set_slot(infft_plan p, int slot);

/* NFFT: f = B F D fhat ~ A fhat (Section 2.1).  fhat [nrhs][M...], f [nrhs][N]. */
int nfft_trafo(infft_plan p, const void* fhat, void* f, int nrhs);

/* Adjoint NFFT: h~ = D^* F^* B^* f ~ A^* f ((2.8)).  f [nrhs][N], h [nrhs][M...]. */
int nfft_adjoint(infft_plan p, const void* f, void* h, int nrhs);

/* Algorithm 3.17: optimises the nonzero entries of B, one regularised least-squares problem
 * per oversampled grid index l over the nodes I(l) of (3.29), solved through its normal
 * equations in FP64 on the GPU (whatever the plan precision).  Stores B_opt in the plan: FP64
 * plans keep it in FP64; FP32 plans keep only its FP32 rounding, which infft_apply and
 * infft_apply_adjoint read (infft_get_B, infft_plan_export and infft_grad_x_bopt recompute the FP64
 * values first).  Problems with more than 64 members (1-D; 32 in 2-D) go to a blocked Cholesky pass.  Outside
 * graph capture the call records that pass: it reads the number and sizes of those problems back
 * (synchronising the stream), packs them into batches and uploads their task lists.  Under HIP
 * graph capture it replays the last record without touching the host: a kernel first checks that
 * the problems the tiers list are those recorded (same grid indices and sizes); if not (the nodes
 * changed since the record), their columns are zero and they are counted in
 * infft_status.oversized.  INFFT_ESTATE under capture when no record exists yet (call it once
 * outside capture first).  Workspace plans: INFFT_ENOMEM when a problem does not fit the memory
 * kept for large problems. */
int infft_precompute_B(infft_plan p);

/* Algorithm 3.10 (ansatz 1 of Section 3.2.1, the underdetermined inverse NFFT): optimises the
 * nonzero entries of B^* column by column, one regularised least-squares problem per node j over
 * the grid indices I(x_j) of (3.16), b~_j = M (K_j^* K_j + lambda_j I)^{-1} K_j^* e_j ((3.21)-(3.22))
 * with K = A D^* F^* (3.14) built on the inverse's D (window or Dirichlet, Remark 3.11) and
 * lambda_j = rho trace(K_j^* K_j) / |I(x_j)|.  The Gram matrices come from one banded table of
 * K^* K computed through the Toeplitz structure of A^* A (an adjoint NFFT of bandwidth 2M on the
 * plan's nodes and length-M_sigma FFTs, all FP64), the solves are FP64 whatever the plan precision.
 * Replaces the plan's B_opt: afterwards infft_apply computes the paper's estimate
 * f_check = (1/M) D^* F^* B_opt^* f and infft_apply_adjoint the inverse adjoint
 * f_tilde = (1/M) B_opt F D h of Remark 3.15; infft_get_B returns conj(b~_j) / M per node.
 * d = 1 single-problem plans only (INFFT_EINVAL otherwise); INFFT_ESTATE under graph capture.  The
 * first call creates two inner plans (allocates and synchronises); failed solves are counted in
 * infft_status.failed_solves and leave zero rows. */
int infft_precompute_Bstar(infft_plan p);

/* Modified adjoint NFFT (3.32): fcheck = D^* F^* B_opt^* f ~ fhat.  f [nrhs][N],
 * fcheck [nrhs][M...].  Returns INFFT_ESTATE before infft_precompute_B. */
int infft_apply(infft_plan p, const void* f, void* fcheck, int nrhs);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc): infft_apply with its work buffers -- two oversampled
 * grids and the spreading halos for as many of the plan's max_rhs right-hand sides per pass as
 * fit -- in a static device array of the library (64 MiB on each device it runs on, held until
 * the process ends) instead of the plan's.  Allocates nothing and leaves the plan's buffers alone
 * (the grid a preceding nfft_trafo left stays valid for nfft_grad_x_after_trafo).  Every call on a
 * device shares that array, keeping the last call's contents: calls that overlap on one device
 * (other streams, threads or plans) race, and the caller must order them.  The plan's device must
 * be current (INFFT_EINVAL otherwise).  INFFT_EINVAL when one right-hand side needs more work
 * memory than the array holds (about 2 x 8 M_sigma^d bytes for FP32 plans, 2 x 16 for FP64, plus
 * halos in 2-D) and for batch plans; INFFT_ESTATE before infft_precompute_B. */
int infft_apply_noalloc(infft_plan p, const void* f, void* fcheck, int nrhs);

/* Adjoint of infft_apply: f = B_opt F D h (the inverse adjoint NFFT of Remark 3.24).
 * h [nrhs][M...], f [nrhs][N].  Returns INFFT_ESTATE before infft_precompute_B. */
int infft_apply_adjoint(infft_plan p, const void* h, void* f, int nrhs);

/* Gradient of a real loss through the NFFT with respect to the nodes:
 * gradx[j][t] = sum_r Re( conj(gradf[r][j]) * d f_{r,j} / d x_{j,t} ), with f = B(x) F D fhat
 * and the derivative of the window inside its support.  fhat [nrhs][M...], gradf [nrhs][N]
 * (plan precision), gradx float64 [N][d]. */
int nfft_grad_x(infft_plan p, const void* fhat, const void* gradf, double* gradx, int nrhs);

/* The same node gradient from the oversampled grid F D fhat that the last nfft_trafo on the
 * current work slot left (the backward of an NFFT whose forward just ran: no second FFT of fhat).
 * gradf [nrhs][N] (plan precision), gradx float64 [N][d] overwritten; nrhs must equal that
 * nfft_trafo's, which must have fitted in one pass (nrhs <= max_rhs).  Every other call that
 * writes the slot's grid (nfft_adjoint, infft_apply, infft_apply_adjoint, nfft_grad_x,
 * infft_grad_x_bopt on that slot; nfft_set_nodes, infft_precompute_Bstar and infft_autotune on
 * any) ends the grid's validity: then INFFT_ESTATE.  INFFT_EINVAL for batch plans and a
 * different nrhs.  The validity is tracked on the host in call order, so under graph capture it
 * follows the captured order. */
int nfft_grad_x_after_trafo(infft_plan p, const void* gradf, double* gradx, int nrhs);

/* Gradient of a real loss through B_opt(x) with respect to the nodes, for fcheck = infft_apply(f)
 * with f held fixed: implicit differentiation of the ridge normal equations of Algorithm 3.17
 * ((3.30)-(3.31)); membership I(l) is piecewise constant in x and contributes nothing.  f [nrhs][N]
 * and gradfc [nrhs][M...] (the loss's gradient with respect to fcheck, PyTorch's convention) in the
 * plan precision; gradx float64 [N][d] is overwritten.  The total node gradient of a loss through
 * both the NFFT and the modified adjoint is the sum of nfft_grad_x and this.  Synchronises the
 * stream (it reads the sizes of local problems above 32 members back, like infft_precompute_B, and
 * solves those on the blocked Cholesky pass; an FP32 plan first recomputes its FP64 B_opt, as in
 * infft_get_B); returns INFFT_ESTATE before infft_precompute_B, for batch plans, and when B holds
 * the result of infft_precompute_Bstar. */
int infft_grad_x_bopt(infft_plan p, const void* f, const void* gradfc, double* gradx, int nrhs);

/* Copies B_opt to `rows` (device, complex128 [N][(2m+1)^d], caller node order, tap index
 * tau flattened with the first dimension slowest; entry (j, tau) multiplies grid index
 * (l0_j + tau) mod M_sigma).  Returns INFFT_ESTATE before infft_precompute_B.  For an FP32 plan
 * whose B_opt came from infft_precompute_B the FP64 values are first recomputed on the stream (the
 * same B optimisation, so the plan's FP32 copy is their rounding; it replays the plan's record of
 * the large-problem pass where one exists, so graphs captured on that record stay valid). */
int infft_get_B(infft_plan p, void* rows);

/* Serialises B_opt with what identifies it: plan parameters (d, M, N, sigma, m, rho, kernel of
 * the inverse, which algorithm made it), the wrapped nodes and the rows of B_opt in caller order
 * (the layout of infft_get_B), into host memory `host_buf` of *bytes bytes.  host_buf == NULL:
 * only sets *bytes to the size needed.  Synchronises the stream (an FP32 plan first recomputes
 * its FP64 B_opt, as in infft_get_B).  INFFT_ESTATE before a precompute, INFFT_EINVAL for a short
 * buffer or a batch plan. */
int infft_plan_export(infft_plan p, void* host_buf, size_t* bytes);

/* Loads what infft_plan_export wrote (host memory) into a plan made with the same d, M, N, sigma,
 * m, rho and kernel of the inverse (INFFT_EINVAL otherwise): the nodes go through the node
 * preprocessing, which is deterministic, so sorted order and lists I(l) match the exported B_opt;
 * then B_opt is loaded and the plan is ready for infft_apply without Algorithm 3.17.  The status
 * block's solve counts restart at zero.  Synchronises the stream; not under graph capture
 * (INFFT_ESTATE); not for batch plans. */
int infft_plan_import(infft_plan p, const void* host_buf, size_t bytes);

/* Synchronises the plan's stream and reports the device status block. */
int nfft_plan_status(infft_plan p, infft_status* out);

/* Bytes of device memory the plan holds. */
int64_t nfft_plan_device_bytes(infft_plan p);

/* Releases the plan (waits for the plan's stream first) and the device memory nfft_plan
 * allocated; a workspace passed to nfft_plan_ws stays the caller's. */
void nfft_plan_destroy(infft_plan p);

/* Autotuner: times each direction of the plan's FFT (coefficients -> grid and back, both passes)
 * with the default shapes and with every pair of 1, 2, 4, 8 and 16 sub-transforms per workgroup
 * (as far as LDS holds them): `reps` runs captured in a HIP graph on a stream of its own and
 * replayed, on the plan's buffers (and a buffer placed with the plan); keeps the fastest for
 * later calls.  With max_rhs > 1 it then times the spreading with each chunk of right-hand sides
 * per pass (infft_autotune_rhs_chunk) the same way.  Synchronous; not under graph capture (INFFT_ESTATE).  A no-op for
 * batch plans, whose launches pack workgroups as full as LDS allows; a workspace plan (which must
 * not allocate, and graph instantiation does) returns to the default shapes. */
int infft_autotune(infft_plan p, int reps);

/* Sub-transforms per workgroup the autotuner chose for step `step` (0 or 1) of direction `dir`
 * (0: coefficients -> grid, 1: grid -> coefficients); 0 when not tuned, -1 for bad arguments. */
int infft_autotune_rows(infft_plan p, int dir, int step);

/* Right-hand sides per pass of the plan's spreading (the adjoint (2.8) and the modified adjoint
 * (3.32)): in 1-D a cap on the kernel's chunk of 1, 2, 4 or 8 (default 8), in 2-D the chunk of
 * the LDS tile (default: as many as it holds).  infft_autotune sets it for plans with max_rhs > 1;
 * 0 for batch plans, -1 for a null plan. */
int infft_autotune_rhs_chunk(infft_plan p);

/* A batch of nprob independent one-dimensional problems of uneven sizes in one plan (the
 * setting of many small inverse NFFTs): problem i has M[i] coefficients (even) and N[i] nodes;
 * sigma, m and the options are shared.  M and N are host arrays; x (device, float64) holds the
 * nodes of all problems one after the other (sum N[i] values).  Every entry point above accepts
 * the batch plan and runs each stage for all problems in one kernel launch (per stage: FFT
 * passes grouped by pass type, spreading, interpolation, the local solves), so a whole step is
 * a handful of launches that a HIP graph can capture.  Caller arrays are problem-major:
 *   fhat, fcheck, h: [problem][nrhs][M_i]   f, gradf: [problem][nrhs][N_i]
 *   gradx: float64 [sum N_i]                 rows of infft_get_B: [sum N_i][2m+1]
 * with nrhs <= opts->max_rhs (INFFT_ESTATE otherwise).  nfft_set_nodes runs the node
 * preprocessing problem by problem; nfft_plan_status reports sums (and the extremes of
 * |I(l)|) over the problems.  On failure *out is NULL and the message names the problem. */
int nfft_plan_batched(infft_plan* out, int nprob, const int64_t* M, const int64_t* N, double sigma, int m,
                      const double* x, const infft_options* opts, void* stream);

/* Kernel classes for infft_profile_begin. */
#define INFFT_K_NODES 1    /* node preprocessing and sort */
#define INFFT_K_FFT 2      /* FFT passes (with the fused deconvolution and halo fold-in) */
#define INFFT_K_SPREAD 3   /* spreading with the window or with B_opt */
#define INFFT_K_INTERP 4   /* interpolation with the window or with B_opt, node gradient */
#define INFFT_K_SOLVE 5    /* local least-squares solves of the B optimisation */

/* Starts timing the launches of one kernel class: each launch of that class is bracketed by a
 * pair of HIP events recorded on the plan's stream (launch order is unchanged).  Not for use
 * while the stream is being captured into a graph. */
int infft_profile_begin(infft_plan p, int kernel_class);

/* Synchronises the stream, stops timing and returns the summed event time in milliseconds and
 * the number of timed launches. */
int infft_profile_end(infft_plan p, double* total_ms, int64_t* launches);

/* Thread-local description of the last error (empty string if none). */
const char* infft_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* INFFT_H */
