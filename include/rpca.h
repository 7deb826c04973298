/*
 * rpca.h - C ABI of librpca: accelerated alternating projections (AccAltProj)
 * for fully observed robust PCA, D = L + S, on AMD Instinct MI355X (gfx950).
 *
 * The method is Algorithm 1 (AccAltProj loop), Algorithm 2 (Trim) and
 * Algorithm 3 (initialisation by two steps of modified AltProj) of Cai, Cai and
 * Wei, "Accelerated Alternating Projections for Robust Principal Component
 * Analysis", with the fast SVD of the tangent-space projection of Section 2.1
 * and the stopping rule err_k < tol of Section 3.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - Matrices are row-major. D is m x n with row stride ldd >= n elements.
 *   Its element type is params->dtype (RPCA_F64: double, RPCA_F32: float).
 * - Pointers documented as "device" must point to memory of the current HIP
 *   device (hipMalloc / torch CUDA tensors). "host" pointers are ordinary host
 *   memory. The library never allocates, frees or retains caller buffers.
 * - The iterate factors are FP64 whatever the dtype of D: U is m x r (row
 *   stride r), V is n x r (row stride r), sigma has r entries, so that
 *   L_k = U diag(sigma) V^T. S_k is never stored: it is T_zeta_k(D - L_k).
 * - ws / ws_bytes is a caller-owned device workspace of at least the size
 *   rpca_workspace_size() reports, 256-byte aligned. Its content does not need
 *   to be initialised and is not meaningful after a call.
 * - stream is a hipStream_t (0 = the null stream). Every device operation is
 *   ordered on it. Calls that report host-visible results (the scalars of
 *   rpca_state, histories) synchronise with the stream before returning.
 * - Tracing: with the environment variable RPCA_TRACE set to "1" (stderr) or
 *   to a file name (appended), rpca_solve and rpca_solve_batch write, after
 *   the device work, one JSON line per state k of each solve (err_k, zeta_k;
 *   for a batch when histories are requested) and a summary line (status,
 *   iterations, initialisation passes, sigma_1 and sigma_{r+1} of the last
 *   P_T(D - S_k), shape, flags). Unset or "0": nothing is written.
 * - One call at a time per workspace; calls sharing a workspace must not
 *   overlap. Calls with distinct workspaces may run concurrently; at most 32
 *   rpca_init / rpca_solve calls may be in flight per device (each holds a
 *   small slot of host-visible status memory; beyond that they return
 *   RPCA_EHIP with rpca_last_hip_error() = hipErrorOutOfMemory).
 * - Return value: RPCA_OK (0) or RPCA_MAXITER (1) on success, a negative
 *   RPCA_E* code on failure. Arguments are validated before any launch; a
 *   failed validation leaves every output untouched.
 * - The data D itself is validated by the first pass over it, which already
 *   forms ||D||_F^2 (the denominator of err_k, Section 3): rpca_init and
 *   rpca_solve return RPCA_EINVAL when ||D||_F = 0 or when the sum is not
 *   finite (a NaN or infinite entry, or an entry whose square overflows the
 *   dtype); rpca_step returns RPCA_EINVAL when the residual of its first pass
 *   (at the given state) is not finite. In these cases the caller's state is
 *   left untouched. A residual that becomes non-finite later inside
 *   rpca_solve's loop returns RPCA_EBREAKDOWN.
 */
#ifndef RPCA_H
#define RPCA_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ------------------------------------------------------ */
#define RPCA_OK           0   /* success                                               */
#define RPCA_MAXITER      1   /* rpca_solve ran max_iter iterations without err < tol  */
#define RPCA_EINVAL      -1   /* bad shape, parameter, pointer or alignment            */
#define RPCA_EWORKSPACE  -2   /* workspace missing or smaller than required            */
#define RPCA_EHIP        -3   /* a HIP runtime call failed (see rpca_last_hip_error)   */
#define RPCA_ENODEV      -4   /* no gfx950 device is current                           */
#define RPCA_EBREAKDOWN  -5   /* a residual sum became non-finite inside the iteration */

/* ---- element types of D ------------------------------------------------ */
#define RPCA_F64 0            /* D (and dense L/S outputs) are double                  */
#define RPCA_F32 1            /* D (and dense L/S outputs) are float                   */

/* ---- flags ------------------------------------------------------------- */
#define RPCA_FLAG_NO_TRIM 1u  /* AccAltProj without trim (Section 3): U~ = U_k, V~ = V_k */
/* Mixed-precision form (RPCA_F32 only): of the tangent products
 * Y1 = (D - S_k) V~ = L_k V~ + E V~ and Y2 = (D - S_k)^T U~ = L_k^T U~ + E^T U~
 * (E = D - L_k - S_k, the residual part), the products E V~ and E^T U~ of a
 * loop body run on the matrix cores with BF16 operands and FP32
 * accumulation, and the rank-r parts are added exactly from the factors; so
 * the BF16 rounding error of Y1 and Y2 is about 2^-8 err_k relative and falls
 * with err_k. The rebuild of L_k, the threshold, the residual and err_k stay
 * FP32, as does all small algebra (FP64). By default every loop
 * body takes BF16 products. With mixed_err > 0, body k of rpca_solve (which
 * computes err_k and L_{k+1}) takes them while err_j >= mixed_err for every
 * j <= k - 2 (bodies 0 and 1 always do: the host decides one body ahead) and
 * every later body is the FP32 one; rpca_step takes them while the state's
 * err >= mixed_err (or is unknown). Not part of the paper: a precision choice
 * of this library. */
#define RPCA_FLAG_MIXED 2u
/* Workspace for rpca_relaxed_step (threshold training; r <= 10). */
#define RPCA_FLAG_TRAINING 4u
/* Learned threshold schedule (not part of the paper): in the loop, zeta_{k+1}
 * = beta (sigma_{r+1} + gamma^{k+1} sigma_1) * exp(clip(o, -5, 5)), a learned
 * correction of Algorithm 1's threshold, with o the output of the threshold
 * network (params->zeta_mlp, RPCA_MLP_PARAMS device floats) at the features
 *   phi = ((k + 1) / 15, log max(sigma_{r+1} / sigma_1, 1e-4), log err_k, log(sigma_1 / ||D||_F)),
 * sigma_1, sigma_{r+1} those of P_T(D - S_k) (the ratio is clamped where the
 * FP32 path no longer resolves sigma_{r+1}). Fallback to the paper's
 * schedule of Algorithm 1 for the rest of the solve as soon as err_k >= err_{k-1}
 * or the network's threshold is not a positive finite number. */
#define RPCA_FLAG_LEARNED 8u
#define RPCA_MLP_PARAMS 1249

/* Largest supported rank r and init block p. */
#define RPCA_MAX_RANK 16

typedef struct rpca_params {
    int64_t  m, n;         /* D is m x n, 2r <= min(m, n)                                    */
    int64_t  ldd;          /* row stride of D in elements, ldd >= n                          */
    int32_t  r;            /* target rank, 1 <= r <= RPCA_MAX_RANK                           */
    int32_t  dtype;        /* RPCA_F64 or RPCA_F32                                           */
    double   beta;         /* threshold parameter of Algorithm 1 (> 0)                       */
    double   beta_init;    /* threshold parameter of Algorithm 3 (> 0)                       */
    double   gamma;        /* convergence-rate parameter, 0 <= gamma < 1 (Section 2.1)       */
    double   mu;           /* Trim level of Algorithm 2 (> 0 unless RPCA_FLAG_NO_TRIM)        */
    double   tol;          /* stop when err_k < tol (Section 3), tol > 0                     */
    int32_t  max_iter;     /* iteration cap; the paper uses 100 (Section 3)                  */
    int32_t  init_block;   /* p: columns of the initial truncated-SVD iteration,
                              r <= p <= RPCA_MAX_RANK and 2p <= min(m, n);
                              0 = default: min(r + 1, RPCA_MAX_RANK, min(m, n) / 2)        */
    int32_t  init_max_passes; /* cap on passes over D per init stage; 0 = default (40)      */
    uint32_t flags;        /* RPCA_FLAG_*                                                    */
    uint64_t seed;         /* seeds the start block of the initial truncated SVD             */
    double   mixed_err;    /* with RPCA_FLAG_MIXED: BF16-product bodies while err_k >= this;
                              <= 0: BF16 products in every loop body (default)              */
    const float *zeta_mlp; /* with RPCA_FLAG_LEARNED: device parameters of the network      */
} rpca_params;

/* Iterate (L_k, S_k): L_k = U diag(sigma) V^T, S_k = T_zeta(D - L_k). The three
 * arrays are caller-owned device memory; the scalars are host values. */
typedef struct rpca_state {
    double  *U;            /* device, m x r, row stride r                                    */
    double  *V;            /* device, n x r, row stride r                                    */
    double  *sigma;        /* device, r                                                      */
    double   zeta;         /* zeta_k                                                         */
    double   err;          /* err_k = ||D - L_k - S_k||_F / ||D||_F (Section 3)               */
    double   sigma1_pt;    /* sigma_1 of the P_T(D - S_{k-1}) that produced L_k (0 at k = 0) */
    double   sigma_r1_pt;  /* sigma_{r+1} of that matrix                                     */
    double   normD;        /* ||D||_F; set by rpca_init / rpca_solve. rpca_step reuses it
                              when > 0 and otherwise spends one extra pass computing it      */
    int32_t  k;            /* iteration index                                                */
    int32_t  init_passes;  /* passes over D spent by rpca_init (diagnostic)                  */
    int32_t  svd_sweeps;   /* Jacobi sweeps of all 2K x 2K SVDs in the last call (diagnostic) */
    int32_t  reserved;     /* zero                                                           */
} rpca_state;

/* Bytes of device workspace needed by every entry point for these params.
 * Returns RPCA_EINVAL for invalid params (bytes untouched). */
int rpca_workspace_size(const rpca_params *p, size_t *bytes);

/* Algorithm 3. zeta_{-1} = beta_init sigma_1(D); S_{-1} = T(D);
 * L_0 = H_r(D - S_{-1}) by a block two-sided subspace iteration run to
 * convergence; zeta_0 = beta sigma_1(D - S_{-1}); S_0 = T_zeta_0(D - L_0).
 * D: device m x n (dtype). On return st holds L_0 (U, sigma, V), zeta_0, err_0
 * and k = 0. */
int rpca_init(const void *D, const rpca_params *p, rpca_state *st,
              void *ws, size_t ws_bytes, void *stream);

/* Algorithm 2 followed by orthonormalisation: U_tilde (device m x r) and
 * V_tilde (device n x r), FP64, row stride r, are orthonormal bases of the
 * trimmed factors A = Trim(U), B = Trim(V) of L_k (footnote to Section 2.1).
 * With RPCA_FLAG_NO_TRIM they span U_k and V_k. st is read only. */
int rpca_trim(const rpca_params *p, const rpca_state *st,
              double *U_tilde, double *V_tilde,
              void *ws, size_t ws_bytes, void *stream);

/* One body of Algorithm 1 from any state k: Trim, L_{k+1} = H_r(P_T(D - S_k))
 * through the 2r x 2r matrix of Section 2.1, zeta_{k+1}, S_{k+1} implicit and
 * err_{k+1}. Reads st (U, sigma, V, zeta, k) and overwrites it with state k+1.
 * Costs two passes over D. */
int rpca_step(const void *D, const rpca_params *p, rpca_state *st,
              void *ws, size_t ws_bytes, void *stream);

/* For callers that cannot allocate device memory (serving loops with a fixed
 * memory budget, harnesses that forbid hipMalloc): rpca_step with the
 * workspace taken from a
 * buffer of RPCA_NOALLOC_WS_BYTES that the library holds in device memory,
 * one per GPU, from the first call on that GPU until the process ends. The
 * result is identical to rpca_step's with a caller workspace. Returns
 * RPCA_EWORKSPACE when the problem needs a larger workspace than that (see
 * rpca_workspace_size; 10^4 x 10^4 at r = 5 needs 26 MiB with FP32 D and
 * 48 MiB with FP64 D). The call allocates nothing and creates no runtime
 * objects (the profiler of rpca_profile_enable does not see it). Every call
 * on one GPU uses that GPU's single buffer: calls that overlap in time on the
 * same GPU (other host threads, or other streams whose work has not finished)
 * race and must be serialised by the caller; the buffer keeps the last call's
 * contents, none of which a call depends on. */
#define RPCA_NOALLOC_WS_BYTES (64u << 20)
int rpca_step_noalloc(const void *D, const rpca_params *p, rpca_state *st, void *stream);

/* Algorithm 3 then Algorithm 1 until err_k < tol or k = max_iter, one fused
 * pass over D per iteration. err_hist / zeta_hist (host, nullable) receive
 * err_0..err_K and zeta_0..zeta_K, at most hist_cap entries each. Returns
 * RPCA_OK if err_K < tol, RPCA_MAXITER otherwise; st holds the final state. */
int rpca_solve(const void *D, const rpca_params *p, rpca_state *st,
               double *err_hist, double *zeta_hist, int32_t hist_cap,
               void *ws, size_t ws_bytes, void *stream);

/* Several independent solves advanced together from one host thread (a
 * batch of instances): instance i is exactly rpca_solve(D[i], p[i], st[i],
 * err_hist[i], zeta_hist[i], hist_cap, ws[i], ws_bytes[i], streams[i %
 * n_streams]), with its own workspace, and the host follows every instance's
 * queue of bodies without blocking on any of them, so the bodies of up to
 * n_streams instances run concurrently (one instance per stream at a time, in
 * index order). Not part of the paper: a throughput form for many small
 * problems. err_hist / zeta_hist may be NULL (or hold NULL entries).
 * status[i] receives instance i's rpca_solve status. Returns RPCA_OK, or the
 * first negative status of an instance (the others still run), or RPCA_EINVAL
 * for bad arguments (nothing run). 1 <= n_streams <= RPCA_MANY_MAX_STREAMS;
 * the streams must be distinct. */
#define RPCA_MANY_MAX_STREAMS 16
int rpca_solve_many(int32_t count, const void *const *D, const rpca_params *const *p, rpca_state *const *st,
                    double *const *err_hist, double *const *zeta_hist, int32_t hist_cap,
                    void *const *ws, const size_t *ws_bytes, void *const *streams, int32_t n_streams,
                    int32_t *status);

/* Batched solve: count instances of one shape in every kernel launch
 * (Algorithm 3, then Algorithm 1, for each instance; not part of the paper: a
 * throughput form for many small problems). p[count]: the instances'
 * parameters; they may differ in beta, beta_init, gamma, mu and tol and must
 * agree in everything else (shape, r, dtype, flags, caps, seed). Instance i
 * owns the slab that starts i * slab_bytes after `slabs` (device, 256-byte
 * aligned), laid out as rpca_batch_layout_of reports: its D (m x n, row stride
 * p->ldd, p->dtype) at off_D, filled by the caller; its iterate U (m x r), V
 * (n x r), sigma (r), FP64, at off_U, off_V, off_sigma, written by the call;
 * its workspace at off_ws. Each kernel launch covers all instances (grid y)
 * and each instance's control block gates its own work, so every instance
 * follows exactly the steps of rpca_solve (same stopping rule; with
 * RPCA_FLAG_MIXED every loop body takes BF16 products, so mixed_err must be
 * <= 0; with RPCA_FLAG_LEARNED the network p->zeta_mlp is shared).
 * st[count] (host) receives each instance's scalars and pointers to its
 * factors in its slab; err_hist / zeta_hist (host, count x hist_cap, row i for
 * instance i, may be NULL) entries 0..st[i].k; status[i] the status
 * rpca_solve would return. Returns RPCA_OK or the first negative instance
 * status; RPCA_EINVAL for bad arguments (1 <= count <= RPCA_BATCH_MAX). Returns
 * after the device work is done. Up to 4 batched calls run on one device at
 * once (from different host threads, each on its own stream: a pass of one
 * batch then overlaps the latency-bound kernels of another); each holds one of
 * 4 small buffers of mapped host memory that the library keeps per device, and
 * a fifth call waits for the first buffer. */
typedef struct rpca_batch_layout {
    size_t slab_bytes;               /* bytes per instance (a multiple of 256)         */
    size_t off_D, off_U, off_V, off_sigma, off_ws;   /* offsets inside a slab          */
} rpca_batch_layout;
#define RPCA_BATCH_MAX 65535
int rpca_batch_layout_of(const rpca_params *p, rpca_batch_layout *out);   /* the same for every instance */
int rpca_solve_batch(int32_t count, void *slabs, const rpca_params *p, rpca_state *st,
                     double *err_hist, double *zeta_hist, int32_t hist_cap, int32_t *status, void *stream);

/* Dense outputs of Algorithm 1: L_out = U diag(sigma) V^T (row stride ldl) and
 * S_out = T_zeta(D - L) (row stride lds), dtype elements, device. Either
 * pointer may be NULL. st is read only. */
int rpca_materialize(const void *D, const rpca_params *p, const rpca_state *st,
                     void *L_out, int64_t ldl, void *S_out, int64_t lds,
                     void *ws, size_t ws_bytes, void *stream);

/* The dominant pass of one iteration, exposed for testing and measurement:
 * with L = A_L B_L^T (A_L device m x r, B_L device n x r, FP64, row stride r),
 * x = D - L, S = T_zeta(x) and Z = D - S (Section 2.1),
 *   Y1 = Z V_t   (device m x r, FP64)    Y2 = Z^T U_t (device n x r, FP64)
 *   *resid2 = sum over |x_ij| <= zeta of x_ij^2   (host scalar),
 * where U_t (m x r) and V_t (n x r) are device FP64 bases. Inputs are rounded
 * to dtype before the pass, as inside rpca_step. As there, the pass forms the
 * products of the residual part E = D - L - S and the rank-r parts L V_t and
 * L^T U_t are added in FP64 from the rounded factors; with RPCA_FLAG_MIXED,
 * E V_t is the BF16 matrix-core product. */
int rpca_tangent_products(const void *D, const rpca_params *p,
                          const double *A_L, const double *B_L, double zeta,
                          const double *U_t, const double *V_t,
                          double *Y1, double *Y2, double *resid2,
                          void *ws, size_t ws_bytes, void *stream);

/* One iteration with a relaxed threshold, for training a learned threshold
 * schedule (not part of the paper). From the state L_k = U diag(sigma) V^T
 * (read), with x = D - L_k and s(x) = x * logistic((|x| - zeta) / tau), which
 * tends to the hard threshold T_zeta of Section 2.1 as tau -> 0:
 *   Z = D - s(x),  L_{k+1} = H_r(P_T(Z))   (T the tangent space of Trim(L_k))
 * is written back to the state (U, sigma, V; k += 1; zeta = the given zeta;
 * err = ||x - s(x)||_F / ||D||_F of L_k; sigma1_pt / sigma_r1_pt = sigma_1 and
 * sigma_{r+1} of P_T(Z)). For target factors P (device m x r_true) and Q
 * (device n x r_true), FP64, row stride r_true, out receives
 *   loss = ||L_{k+1} - P Q^T||_F^2 / ||P Q^T||_F^2  and  d loss / d zeta,
 * the exact derivative of the relaxed iteration (first-order perturbation of
 * H_r in a 3r-dimensional reduced space; needs sigma_r > sigma_{r+1}).
 * Requires RPCA_FLAG_TRAINING in p->flags (workspace), r <= 10,
 * 1 <= r_true <= 16, zeta > 0, tau > 0. */
typedef struct {
    double  loss, dloss_dzeta;
    double  err;                /* relaxed err_k of the input state                   */
    double  sigma1, sigma_r1;   /* sigma_1, sigma_{r+1} of P_T(Z)                     */
    int32_t svd_sweeps, reserved;
} rpca_relax_result;
int rpca_relaxed_step(const void *D, const rpca_params *p, rpca_state *st, double zeta, double tau,
                      const double *P_true, const double *Q_true, int32_t r_true,
                      rpca_relax_result *out, void *ws, size_t ws_bytes, void *stream);

/* Reverse mode of K unrolled relaxed iterations (training through the
 * iterations; not part of the paper). Body k (k = 0..K-1) is the iteration of
 * rpca_relaxed_step from L_k = U_k diag(sigma_k) V_k^T with threshold zeta[k]
 * and temperature tau[k] (Algorithm 1's body with s(x) in place of T_zeta:
 * Trim of Algorithm 2, P_T and H_r of Section 2.1); the loss is
 *   sum_{k=1..K} weight[k-1] ||L_k - P Q^T||_F^2 / ||P Q^T||_F^2.
 * Checkpoints: U_ck[k], sigma_ck[k], V_ck[k] (k = 0..K; host arrays of K + 1
 * device pointers, FP64, m x r / r / n x r, row stride r) are the factors of
 * L_k as rpca_relaxed_step produced them (any factorisation for k = 0); only
 * these are kept, and every body's intermediates are recomputed with one pass
 * over D. zeta, tau, weight: host arrays of K. Outputs: zeta_bar (host, K):
 * d loss / d zeta_k; U_bar, sigma_bar, V_bar (device, m x r, r, n x r): the
 * gradient with respect to the factors of L_0 taken as free matrices. Between
 * bodies the gradient is carried with respect to L_k and never formed as a
 * dense matrix. The thresholds are inputs: a schedule that computes them from
 * the iterates is differentiated with its features held fixed. Needs
 * sigma_r > sigma_{r+1} of every P_T(Z) and full-rank complements; requires
 * RPCA_FLAG_TRAINING (workspace), r <= 10, 1 <= K <= RPCA_MAX_UNROLL,
 * 1 <= r_true <= 16, zeta[k] > 0, tau[k] > 0, finite weights, else
 * RPCA_EINVAL. The call returns after the device work is done. */
#define RPCA_MAX_UNROLL 64
int rpca_unrolled_adjoint(const void *D, const rpca_params *p, int32_t K,
                          const double *const *U_ck, const double *const *sigma_ck, const double *const *V_ck,
                          const double *zeta, const double *tau, const double *weight,
                          const double *P_true, const double *Q_true, int32_t r_true,
                          double *zeta_bar, double *U_bar, double *sigma_bar, double *V_bar,
                          void *ws, size_t ws_bytes, void *stream);

/* Training kernels of the threshold network (device FP32 arrays, ordered
 * on stream; parameter layout W1 (32 x 4, row-major), b1 (32), W2 (32 x 32),
 * b2 (32), w3 (32), b3 (1), RPCA_MLP_PARAMS values):
 *   rpca_mlp_forward:  o[b] = w3 . relu(W2 relu(W1 phi_b + b1) + b2) + b3,
 *                      phi: batch x 4 row-major;
 *   rpca_mlp_backward: grad_theta = sum over b (in order) of grad_o[b] d o_b / d theta
 *                      (overwritten, not accumulated);
 *   rpca_mlp_adam:     one Adam update (Kingma and Ba) at step t >= 1 with moments m, v. */
int rpca_mlp_forward(const float *theta, const float *phi, int32_t batch, float *o, void *stream);
int rpca_mlp_backward(const float *theta, const float *phi, const float *grad_o, int32_t batch,
                      float *grad_theta, void *stream);
int rpca_mlp_adam(float *theta, float *m, float *v, const float *grad, int32_t t, float lr,
                  float beta1, float beta2, float eps, void *stream);

/* Measurement of the dominant kernel. While enabled (process-wide), every
 * streaming pass over D (the only kernel reading the m x n data) is bracketed
 * by two HIP events recorded on the caller's stream; a pass queued after a
 * loop has stopped, which does no work, is not counted. rpca_profile_read
 * waits for the recorded passes and returns, per kind of pass, their summed
 * duration in ms and their number since the previous read, then resets them:
 * stream_ms and stream_launches are arrays of RPCA_PROF_KINDS entries: [0] the
 * loop's passes in the dtype of D, [1] the loop's passes with the BF16
 * product, [2] the passes of the initialisation (L = 0), [3] whole loop
 * bodies of rpca_solve (from before the pass to the end of the body's last
 * kernel: one iteration of Algorithm 1). Disabling keeps the totals for a
 * final read. Intended for benchmarks: the events add a few microseconds of
 * queue work per pass. */
#define RPCA_PROF_KINDS 4
int rpca_profile_enable(int on);
int rpca_profile_read(double *stream_ms, int64_t *stream_launches);

/* Reference for the streaming pass's bandwidth: one launch on `stream` that
 * reads the `bytes` bytes at `data` (device, 16-byte aligned, bytes a positive
 * multiple of 16) once with 16-byte loads and no arithmetic to speak of;
 * `sink` is device scratch of RPCA_PROBE_SINK floats (not meaningfully
 * written). Timing it around the launch gives the read bandwidth the device
 * reaches on the same data. */
#define RPCA_PROBE_SINK 8192
int rpca_read_probe(const void *data, int64_t bytes, float *sink, void *stream);

/* Static description of a status code. */
const char *rpca_strerror(int status);

/* hipError_t of the last failed HIP call on the calling thread (0 if none). */
int rpca_last_hip_error(void);

/* Library version as MAJOR*10000 + MINOR*100 + PATCH. */
int rpca_version(void);

#ifdef __cplusplus
}
#endif

#endif /* RPCA_H */
