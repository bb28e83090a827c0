/* clamp.h — C ABI of the MI355X (gfx950) CLAMP forward-model library.
 *
 * CLAMP ("CLAMP: Majorized Plug-and-Play for Coherent 3D Lidar Imaging",
 * Allen, Rabb, Buzzard, Bouman) reconstructs a speckle-free reflectivity r
 * from L coherent looks y_l = A g_l + eta_l with A = D(a) F (Sec. II-B,
 * eq. A).  This library runs the data-parallel hot path of its MACE loop
 * (Alg. 2) on one GPU:
 *   - the aperture operator A, its adjoint A^H and A^H A (clamp_aperture_op);
 *   - the initialisation of Alg. 2 (clamp_fwd_init);
 *   - one application of every forward agent: covariance diagonal, one exact
 *     steepest-descent step on mu_l, quadratic-surrogate r-update of App. A
 *     (clamp_fwd_agent; with the Mann step fused in, clamp_fwd_agent_mace),
 *     and the residual refresh from the data (clamp_fwd_refresh);
 *   - a fixed Gaussian smoothing prior agent (clamp_prior_gauss);
 *   - the Mann consensus step of Alg. 1 with the convergence error
 *     (clamp_mace_step).
 *
 * Conventions shared by every call
 *   Grid.   A scene is nz range slices of ny x nx pixels, x fastest:
 *           element (z, y, x) of an image sits at (z*ny + y)*nx + x, which is
 *           the lexicographic order of Sec. II-B.  Look l of a stacked array
 *           starts at l*n with n = nx*ny*nz.
 *   F.      The orthonormal 2D DFT of each range slice, forward kernel
 *           exp(-2 pi i (u y/ny + v x/nx)) / sqrt(nx ny).  (With a range
 *           aperture that passes every range frequency this equals the
 *           paper's 3D operator up to a unitary change of data coordinates.)
 *   Pupil.  a[u][v] = 1 where su^2 + sv^2 <= R^2 in signed DFT indices
 *           (su = u for u < ny/2, else u - ny), or a caller-given binary mask.
 *   Compact pupil layout.  Pupil-plane vectors that the method only ever
 *           reads on the pupil are stored as P values per slice (P = ||a||_1
 *           per slice): the pupil samples column by column (v increasing),
 *           rows u increasing inside a column.  clamp_plan_pupil_index
 *           returns the u*nx + v position of each of the P entries.
 *   Types.  complex64 = interleaved float pairs (re, im).  Every array
 *           argument is a DEVICE pointer owned by the caller unless stated;
 *           the library never allocates or frees on the calls that take a
 *           stream, and it never synchronises the stream.  Work is enqueued
 *           on `hip_stream` (a hipStream_t; NULL = the default stream).
 *   Workspace.  `workspace` is caller-owned device memory of at least
 *           clamp_plan_workspace_size bytes, 256-byte aligned; its contents
 *           are scratch between calls.  Calls that overlap in time need
 *           separate workspaces.
 *   Errors.  Arguments are validated before anything is enqueued; an invalid
 *           argument returns a negative status and enqueues nothing.  A
 *           failed launch returns CLAMP_EDEVICE.  clamp_last_error gives a
 *           message for the calling thread's last non-OK status.
 *           Numerical trouble (non-finite values, r <= 0, gamma < 0) is not a
 *           status: kernels OR bits into the caller's device fault word.
 */
#ifndef CLAMP_H
#define CLAMP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t clamp_status;
#define CLAMP_OK 0
#define CLAMP_EINVAL (-1)       /* null pointer, bad scalar, bad index     */
#define CLAMP_ESHAPE (-2)       /* sizes inconsistent with the plan        */
#define CLAMP_EUNSUPPORTED (-3) /* FFT length not in the supported set     */
#define CLAMP_EDEVICE (-4)      /* HIP error (no device, launch failure)   */
#define CLAMP_ENOMEM (-5)       /* device allocation failed in plan_create */

/* clamp_aperture_op directions (Sec. II-B, eq. A). */
#define CLAMP_FWD 0     /* out = A x      = D(a) F x                         */
#define CLAMP_ADJ 1     /* out = A^H x    = F^H D(a) x                       */
#define CLAMP_NORMAL 2  /* out = A^H A x  (an orthogonal projector)          */

/* Fault bits written to the device fault word. */
#define CLAMP_FAULT_NONFINITE 1u  /* a non-finite mu, r or gamma            */
#define CLAMP_FAULT_RNONPOS 2u    /* an r-update returned r <= 0            */
#define CLAMP_FAULT_GAMMA 4u      /* a negative or non-finite step size     */

/* Supported FFT lengths for nx and ny: 32, 64, 128, 192, 256, 384, 512. */

typedef struct clamp_plan clamp_plan;

/* One scene.  pupil_mask, when not NULL, is a HOST array [ny][nx] (nonzero =
 * the aperture passes that DFT sample) and overrides pupil_radius; it is
 * copied by clamp_plan_create. */
typedef struct {
    int32_t nx, ny, nz;   /* pixels per row, rows per slice, range slices   */
    int32_t looks;        /* L, number of looks (>= 1)                      */
    float pupil_radius;   /* R of the circular pupil, in DFT samples (> 0)  */
    const uint8_t* pupil_mask;
    int32_t range_support; /* 0: per-slice 2D operator; K in [1, nz]: 3D     */
} clamp_scene;

/* Operator form (clamp_scene.range_support).
 * 0: A = D(a) F with F the orthonormal 2D DFT of each range slice and a the
 *    pupil on every slice (equal to the paper's operator whenever its range
 *    aperture passes every range frequency).
 * K >= 1: the paper's A = D(a) F with F the orthonormal 3D DFT (Sec. II-B,
 *    eq. A) and a the zero-padded aperture (Sec. II-A: only the K range
 *    frequencies nearest DC hold data): the pupil disk times the range
 *    frequencies of signed index -floor(K/2) .. ceil(K/2) - 1.  Looks,
 *    y_full and operator outputs are then 3D frequency grids (range
 *    frequency w, u, v).  The residual and every "compact" pupil array hold
 *    [K][P] per look: box index k (range frequency k for k < ceil(K/2), else
 *    nz - K + k) outer, pupil sample inner.  alpha = P K / (nx ny nz).
 *    nz must be 16, 32, 48, 64, 96, 128, 192 or 256 (CLAMP_EUNSUPPORTED
 *    otherwise); batches do not accept K >= 1. */

/* Scalars of Alg. 2 and App. A (host memory). */
typedef struct {
    float sigma_w2;       /* data-noise variance sigma_w^2 (> 0)             */
    float sigma2;         /* proximal parameter sigma^2 of eq. prox (> 0)    */
    float rho;            /* Mann relaxation, in (0, 1)                      */
    float beta;           /* surrogate interval factor of App. A (> 1)       */
    float mu_init_scale;  /* s_mu: mu_l starts at s_mu A^H y_l (> 0)         */
    const float* upsilon; /* HOST [n_agents] agent weights, summing to 1     */
    int32_t n_agents;     /* L (forward agents only) or L + 1 (with prior)   */
    int32_t r_update;     /* CLAMP_R_QUADRATIC or CLAMP_R_EXACT               */
} clamp_params;

/* r-update of the forward agent.  CLAMP_R_QUADRATIC: the quadratic surrogate
 * of App. A (r' anchored, clipped to [r', xi], uses beta).  CLAMP_R_EXACT: the
 * exact proximal map of the EM surrogate (eq. surrogate-prox, Sec. III-B),
 * argmin_{r>0} log r + s/r + (r - v)^2 / (2 sigma^2) per voxel: the positive
 * root of r^3 - v r^2 + sigma^2 r - sigma^2 s with the smallest objective,
 * solved in float64 (beta unused). */
#define CLAMP_R_QUADRATIC 0
#define CLAMP_R_EXACT 1

/* Per-look state of the forward agents (device memory, caller-owned).
 *   mu      complex64 [L][n]   posterior means mu_l (eq. mu2).
 *   resid   complex64 [L][nz][P] D(a)(y_l - A mu_l) in the compact layout.
 *   r       float32 [n_agents][n]  agent outputs; r[l] (l < L) is also look
 *           l's surrogate anchor r'_l, and slice L (when present) is the prior's.
 *   y_pupil complex64 [L][nz][P] D(a) y_l in the compact layout, or NULL.
 *           clamp_fwd_init fills it; clamp_fwd_refresh rebuilds resid from it.
 *   ahy2    double [L] ||A^H y_l||^2 (= ||D(a) y_l||^2), or NULL.
 *           clamp_fwd_init fills it; clamp_fwd_agent then reports the
 *           mu-residual of eq. residual.
 * With the 3D operator (range_support K >= 1) resid and y_pupil are
 * [L][K][P]. */
typedef struct {
    void* mu;
    void* resid;
    float* r;
    void* y_pupil;
    double* ahy2;
} clamp_fwd_state;

/* Builds device tables for `nscenes` scenes: FFT twiddles (computed in
 * float64, rounded to float32), pupil tables and tile counts.  Allocates
 * device memory on the current device (CLAMP_ENOMEM on failure,
 * CLAMP_EDEVICE without a usable device).  *out is owned by the caller and
 * released with clamp_plan_destroy.  CLAMP_EUNSUPPORTED for an nx or ny
 * outside the supported set; CLAMP_EINVAL for an empty pupil. */
clamp_status clamp_plan_create(const clamp_scene* scenes, int32_t nscenes,
                               clamp_plan** out);

/* Releases the plan's device tables.  NULL is accepted. */
clamp_status clamp_plan_destroy(clamp_plan* plan);

/* Bytes of workspace the calls below need for any scene of the plan. */
clamp_status clamp_plan_workspace_size(const clamp_plan* plan, size_t* bytes);

/* Host query: pupil samples per slice P, band columns B (columns with at
 * least one pupil sample) and alpha = P / (nx ny) (Sec. III-B). */
clamp_status clamp_plan_pupil_info(const clamp_plan* plan, int32_t scene,
                                   int32_t* P, int32_t* B, double* alpha);

/* Host query: writes the P positions u*nx + v of the compact layout into the
 * HOST array idx[P]. */
clamp_status clamp_plan_pupil_index(const clamp_plan* plan, int32_t scene,
                                    int32_t* idx);

/* Aperture operator of eq. A on nbatch stacked volumes:
 * in, out complex64 [nbatch][nz][ny][nx] (full grids; CLAMP_FWD writes zeros
 * outside the pupil, CLAMP_ADJ reads only pupil samples).  in and out must
 * not overlap.  nbatch >= 0 (0 enqueues nothing). */
clamp_status clamp_aperture_op(const clamp_plan* plan, int32_t scene, int32_t dir,
                               const void* in, void* out, int32_t nbatch,
                               void* workspace, void* hip_stream);

/* Initialisation of Alg. 2 from the looks y_full complex64 [L][nz][ny][nx]
 * (only pupil samples are read):
 *   b_l = A^H y_l;  r0 = (1/L) sum_l |b_l|^2, floored at 1e-12 mean(r0);
 *   mu_l = s_mu b_l;  resid_l = (1 - s_mu) D(a) y_l  (exact, as A A^H = D(a));
 *   state->r[j] = r0 and w[j] = r0 for every agent j < n_agents;
 *   state->y_pupil = D(a) y_l and state->ahy2[l] = ||A^H y_l||^2 where those
 *   pointers are not NULL. */
clamp_status clamp_fwd_init(const clamp_plan* plan, int32_t scene,
                            const clamp_params* params, const void* y_full,
                            clamp_fwd_state* state, float* w,
                            void* workspace, void* hip_stream);

/* One application of every forward agent (Alg. 2, the per-look loop body;
 * Sec. III-B; App. A), all looks in parallel:
 *   c = sigma_w^2 r' / (alpha r' + sigma_w^2) with r' = r[l];
 *   d = A^H resid / sigma_w^2 - omega mu, omega = 1/(r' + sigma_w^2/alpha);
 *   gamma = ||d||^2 / (||A d||^2 / sigma_w^2 + sum omega |d|^2) (0 if d = 0);
 *   mu += gamma d;  resid -= gamma D(a) F d;
 *   r[l] = surrogate prox at v = w[l] with s = c + |mu|^2 (params->r_update:
 *   the quadratic surrogate of App. A with beta, or the exact prox).
 * w: float32 [L][n] (the forward agents' slices of the Mann state).
 * diag: device double [L + 1][8].  Row l < L, look l:
 *   {gamma, ||d||^2, ||A d||^2, h before, h after, mu-residual,
 *    sum omega |d|^2, ||resid||^2 after},
 *   where h = ||resid||^2 / (2 sigma_w^2) + sum omega |mu|^2 / 2 is the
 *   objective of the mu-step (eq. mu-objective) less the constant
 *   ||(1 - a) y_l||^2 / (2 sigma_w^2), so h before - h after = gamma ||d||^2 / 2;
 *   and the mu-residual is the look's term of eq. residual in its
 *   noise-floored form, ||d|| / ||A^H y_l / sigma_w^2|| with the d of this
 *   step (0 when state->ahy2 is NULL).
 *   Row L: {mu-residual of eq. residual (the mean of the looks' terms),
 *   sum_l h before, sum_l h after, 0, 0, 0, 0, 0}.
 * fault: device uint32, OR-ed with CLAMP_FAULT_* bits (never cleared). */
clamp_status clamp_fwd_agent(const clamp_plan* plan, int32_t scene,
                             const clamp_params* params, clamp_fwd_state* state,
                             const float* w, double* diag, uint32_t* fault,
                             void* workspace, void* hip_stream);

/* One application of every forward agent with the Mann step of Alg. 1 fused
 * into its last pass: the forward agents as clamp_fwd_agent, then (Alg. 1)
 * x = 2 r - w, x_bar = sum_j upsilon_j x_j, w <- w + 2 rho (x_bar - r) over
 * all n_agents agents, w_bar = sum_j upsilon_j w_j of the updated w, and
 * conv_err (device double [1]) = ||r - G(w)|| / ||G(w)|| with G built from
 * the w passed in (eq. mace-convergence-error).
 * The prior agent reads only its own w, so Alg. 2's order (forward agents,
 * prior, Mann step) is kept when the caller applies the prior before this
 * call: with n_agents = L + 1, state->r slice L must already hold H(w[L]).
 * Representation of the Mann state, which lets the pass read each look once:
 *   w     float32 [n_agents][n]: slice l < L holds u_l = w_l - 2 rho x_bar,
 *         slice L (with a prior) holds the prior agent's w_{L+1} itself;
 *   xbar  float32 [n]: x_bar of the previous call (zeros after
 *         clamp_fwd_init, which makes u_l = w_l); the call replaces it.
 * The Mann state of look l is u_l + 2 rho x_bar.  wbar: float32 [n] out.
 * diag and fault as clamp_fwd_agent; w is read and written. */
clamp_status clamp_fwd_agent_mace(const clamp_plan* plan, int32_t scene,
                                  const clamp_params* params, clamp_fwd_state* state,
                                  float* w, float* xbar, float* wbar, double* diag,
                                  double* conv_err, uint32_t* fault,
                                  void* workspace, void* hip_stream);

/* The Mann state of clamp_fwd_agent_mace's representation, written out:
 * out[l] = w[l] + 2 rho xbar for the looks l < L, out[L] = w[L] (the prior
 * agent's, when n_agents = L + 1).  w, out: float32 [n_agents][n], not
 * overlapping; xbar: float32 [n]. */
clamp_status clamp_mace_state(const clamp_plan* plan, int32_t scene, const clamp_params* params,
                              const float* w, const float* xbar, float* out, void* hip_stream);

/* Residual refresh: resid_l = y_pupil_l - D(a) F mu_l, recomputed from the
 * data (Alg. 2 defines the residual by mu; the agent updates it by the
 * recurrence resid -= gamma D(a) F d, whose float32 rounding accumulates over
 * iterations).  Needs state->y_pupil (CLAMP_EINVAL otherwise); reads mu,
 * writes resid. */
clamp_status clamp_fwd_refresh(const clamp_plan* plan, int32_t scene, clamp_fwd_state* state,
                               void* workspace, void* hip_stream);

/* Fixed prior agent: out = periodic separable 3D Gaussian smoothing of in
 * (float32 [n] each; standard deviation sigma_vox voxels, 7 taps per axis,
 * taps normalised to sum 1).  in and out must not overlap; in must be
 * 16-byte aligned (the x pass reads it in float4 units), as any device
 * allocation and any agent slice w + j n of a stack is; CLAMP_EINVAL
 * otherwise. */
clamp_status clamp_prior_gauss(const clamp_plan* plan, int32_t scene, float sigma_vox,
                               const float* in, float* out,
                               void* workspace, void* hip_stream);

/* Comparison regularizers of Sec. V as prior agents (the prior slot of
 * Alg. 2), each the proximal map of its regularizer on the image in (float32
 * [n]) into out (float32 [n], not overlapping in).  The paper names them
 * without formulas or weights; this library reads them as follows.
 *
 * l_{2,1} (l2 in cross-range, l1 in range): R(r) = sum_z ||r[z, :, :]||_2
 * over the range slices; out = argmin_r tau R(r) + ||r - in||^2 / 2, which
 * scales each slice by max(0, 1 - tau / ||in_z||_2).  tau >= 0 (the weight
 * times the proximal parameter). */
clamp_status clamp_prior_l21(const clamp_plan* plan, int32_t scene, float tau,
                             const float* in, float* out, void* workspace, void* hip_stream);

/* Isotropic total variation: TV(r) = sum_voxels |grad r| with forward
 * differences along z, y, x (a difference leaving the volume is zero);
 * out approximates argmin_r lam TV(r) + ||r - in||^2 / 2 by `iters` steps of
 * Chambolle's dual projection iteration from p = 0 (step 1/12):
 * p <- (p + g / 12) / (1 + |g| / 12) with g = grad(div p - in / lam), then
 * out = in - lam div p (div the negative adjoint of grad).  lam > 0,
 * 0 <= iters <= 100000. */
clamp_status clamp_prior_tv(const clamp_plan* plan, int32_t scene, float lam, int32_t iters,
                            const float* in, float* out, void* workspace, void* hip_stream);

/* Mann step of Alg. 1 over n_agents stacked images (float32 [n_agents][n]):
 *   x = 2 r - w;  w <- w + 2 rho (sum_j upsilon_j x_j - r);
 *   wbar (float32 [n]) = sum_j upsilon_j w_j of the updated w;
 *   conv_err (device double [1]) = ||r - G(w)|| / ||G(w)|| with G built from
 *   the w passed in (eq. mace-convergence-error). */
clamp_status clamp_mace_step(const clamp_plan* plan, int32_t scene,
                             const clamp_params* params, float* w, const float* r,
                             float* wbar, double* conv_err,
                             void* workspace, void* hip_stream);

/* clamp_mace_step for callers that cannot allocate or pass a workspace
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * allocation): the same Mann step, with its reduction scratch in a 1 MiB
 * array the library holds in device memory on each GPU it runs on (resolved
 * on the first call on a device, kept until the process ends).  Volumes of
 * at most 2^25 voxels (e.g. 512 x 512 x 128); larger ones return
 * CLAMP_ESHAPE.  The plan's device must be current (CLAMP_EDEVICE
 * otherwise).  Allocates nothing.  Every call on one GPU shares that GPU's
 * scratch: calls that overlap in time on one GPU (different streams) race. */
clamp_status clamp_mace_step_noalloc(const clamp_plan* plan, int32_t scene,
                                     const clamp_params* params, float* w, const float* r,
                                     float* wbar, double* conv_err, void* hip_stream);

/* ------------------------------------------------------------------------
 * Batches: every scene of a plan advanced together, one CLAMP iteration per
 * clamp_batch_step.  Each stage runs as persistent launches over device work
 * queues of (scene, look, row group or column tile) items; the FFT passes
 * launch once per FFT length present, the other stages once for all scenes.
 * The interval factor of App. A is beta_k = 1 + 2 / ln(k + 1) for iteration k
 * = (device iteration counter) + 1, read on the device, so a step has no
 * changing host arguments: clamp_batch_capture records one step in a HIP
 * graph and clamp_batch_replay launches it repeatedly.
 * ------------------------------------------------------------------------ */
typedef struct clamp_batch clamp_batch;

/* One scene of a batch (device pointers, caller-owned; the same arrays the
 * single-scene calls take).  params.beta is ignored (see above).
 * xbar selects the form of the Mann step for the whole batch (every scene
 * has one, or none does; CLAMP_EINVAL otherwise):
 *   NULL      the Mann step as its own pass after the prior agents
 *             (clamp_fwd_agent, clamp_prior_gauss, clamp_mace_step);
 *   non-NULL  float32 [n]: the Mann step fused into the update pass, with w
 *             and xbar in clamp_fwd_agent_mace's representation (zeros in
 *             xbar after clamp_fwd_init; w_bar = r0 then) and the prior
 *             agents applied first (clamp_prior_gauss, clamp_fwd_agent_mace).
 * A scene with a prior (n_agents = L + 1) needs ny a multiple of 8 and nx of
 * 32 (CLAMP_EUNSUPPORTED otherwise). */
typedef struct {
    clamp_params params;    /* n_agents = L or L + 1, at most 40 in a batch;  */
                            /* r_update CLAMP_R_QUADRATIC (else EUNSUPPORTED) */
    clamp_fwd_state state;  /* mu, resid, r (r: float32 [n_agents][n])        */
    float* w;               /* float32 [n_agents][n]                          */
    float* wbar;            /* float32 [n]                                    */
    double* diag;           /* double [L + 1][8], as clamp_fwd_agent          */
    float prior_sigma;      /* Gaussian prior width when n_agents = L + 1     */
    float* xbar;            /* NULL, or float32 [n] (see above)               */
} clamp_batch_scene;

/* Workspace bytes of a batch over every scene of the plan (the scenes'
 * single-call workspaces laid end to end). */
clamp_status clamp_batch_workspace_size(const clamp_plan* plan, size_t* bytes);

/* Creates a batch over all nscenes scenes of the plan.  scenes: HOST array
 * [nscenes].  fault: device uint32; conv_err: device double [nscenes] (the
 * convergence error of each scene's last step).  Allocates device queues and
 * tables; the iteration counter starts at 0.  *out is released with
 * clamp_batch_destroy. */
clamp_status clamp_batch_create(const clamp_plan* plan, const clamp_batch_scene* scenes, uint32_t* fault,
                                double* conv_err, void* workspace, clamp_batch** out);
clamp_status clamp_batch_destroy(clamp_batch* batch);

/* Sets the device iteration counter (iterations already done) on the stream. */
clamp_status clamp_batch_set_iteration(clamp_batch* batch, int32_t done, void* hip_stream);

/* One CLAMP iteration of every scene: forward agents, prior agents of the
 * scenes that have one, Mann step, then the counter advances (with xbar:
 * prior agents, then the forward agents with the Mann step fused in). */
clamp_status clamp_batch_step(clamp_batch* batch, void* hip_stream);

/* Grid sizes of the row and column passes in blocks per compute unit, each
 * block walking the queue with a grid-size stride; 0 = one block per work
 * item (the default for rows; columns default to 4 per CU). */
clamp_status clamp_batch_set_tiles(clamp_batch* batch, int32_t row_blocks_per_cu, int32_t col_blocks_per_cu);

/* Times the passes that only write the workspace (inverse and forward column
 * passes, gradient row pass) for grid sizes {one block per item, 2, 4, 8, 16
 * per CU} on the current state, keeps the fastest, and reports them
 * (HOST int32 [2]: rows, columns; may be NULL).
 * Synchronises the stream. */
clamp_status clamp_batch_autotune(clamp_batch* batch, void* hip_stream, int32_t* chosen);

/* Records one clamp_batch_step into a HIP graph (the stream must not be the
 * NULL stream), replacing any earlier recording. */
clamp_status clamp_batch_capture(clamp_batch* batch, void* hip_stream);

/* Launches the recorded graph `iters` times on the stream. */
clamp_status clamp_batch_replay(clamp_batch* batch, int32_t iters, void* hip_stream);

/* ------------------------------------------------------------------------
 * Learned prior agent: a residual 3D CNN denoiser (the learned stand-in for
 * the paper's deep prior agent, Sec. III-C).  8 convolutions of 3x3x3 taps
 * with biases and zero padding, channels 1 -> 32 (x6) -> 32 -> 1, ReLU after
 * the first seven, output H(x) = x + N(x); BF16 weights and activations with
 * FP32 accumulation on the matrix cores, trained with Adam on the mean
 * squared error.
 *
 * Parameters (float32, CLAMP_CNN_PARAMS values): for each layer l = 0..7,
 * W_l[27][Cin_l][Cout_l] then b_l[Cout_l], with tap t = 9 (dz+1) + 3 (dy+1) +
 * (dx+1) for offsets in {-1, 0, 1}; the layer computes
 *   y[v][co] = b[co] + sum_t sum_ci x[v + off(t)][ci] W[t][ci][co].
 * Volumes are float32 [nvol][nz][ny][nx] with nx a multiple of 32.
 * ------------------------------------------------------------------------ */
#define CLAMP_CNN_PARAMS 167841
typedef struct clamp_cnn clamp_cnn;

/* Allocates device parameters (zero), Adam moments and BF16 copies on the
 * current device (CLAMP_EDEVICE without one, CLAMP_ENOMEM when allocation
 * fails).  Destroy frees them; call it only after every call using the
 * object has completed on the device. */
clamp_status clamp_cnn_create(clamp_cnn** out);
clamp_status clamp_cnn_destroy(clamp_cnn* cnn);
/* Copies HOST parameters in (and resets the Adam state and step count) or
 * out.  Both are synchronous device copies: finish the work of other streams
 * that uses the object first.  set_params rejects non-finite values with
 * CLAMP_EINVAL (nothing is changed). */
clamp_status clamp_cnn_set_params(clamp_cnn* cnn, const float* params);
clamp_status clamp_cnn_get_params(const clamp_cnn* cnn, float* params);
/* Workspace bytes for apply (train = 0) or gradient (train = 1) calls on
 * nvol volumes of nz x ny x nx.  Errors shared by the sized calls:
 * CLAMP_EINVAL for non-positive sizes or NULL arguments, CLAMP_ESHAPE when nx
 * is not a multiple of 32 or nvol nz ny nx >= 2^31. */
clamp_status clamp_cnn_workspace_size(int32_t nvol, int32_t nz, int32_t ny, int32_t nx, int32_t train,
                                      size_t* bytes);
/* out = H(x) per volume (device float32 arrays).  normalize != 0 applies the
 * scale-free form out = x + m N(x / m) with m the mean of all nvol volumes. */
clamp_status clamp_cnn_apply(clamp_cnn* cnn, const float* x, float* out, int32_t nvol, int32_t nz, int32_t ny,
                             int32_t nx, int32_t normalize, void* workspace, void* hip_stream);
/* Mean squared error of H(x) against target over the batch into *loss
 * (device double) and its gradient with respect to every parameter into
 * grad (device float32 [CLAMP_CNN_PARAMS]; NULL keeps it inside the object
 * for clamp_cnn_adam_step). */
clamp_status clamp_cnn_grad(clamp_cnn* cnn, const float* x, const float* target, int32_t nvol, int32_t nz,
                            int32_t ny, int32_t nx, double* loss, float* grad, void* workspace, void* hip_stream);
/* One Adam step (beta1 0.9, beta2 0.999, eps 1e-8, bias-corrected) with the
 * gradient of the last clamp_cnn_grad call that kept it inside the object.
 * The gradient is first clipped in norm to 3 times a running average of the
 * past (clipped) norms (weight 0.05 per step; the first step is not clipped),
 * and a gradient with a non-finite norm leaves parameters, moments and the
 * running norm unchanged (the step count of the bias correction still
 * advances).  clamp_cnn_set_params resets the running norm and the Adam
 * state. */
clamp_status clamp_cnn_adam_step(clamp_cnn* cnn, float lr, void* hip_stream);

/* ------------------------------------------------------------------------
 * U-Net prior agent (the paper's deep prior architecture, Sec. III-C): three
 * encoder blocks of two 3x3x3 convolutions, each followed by batch
 * normalisation and ReLU, with 2x2x2 max pooling after each block; three
 * decoder blocks, each opening with a 2x2x2 stride-2 transposed convolution
 * whose output is added to the encoder output of the same level, then two
 * convolutions with batch normalisation and ReLU; a final 3x3x3 convolution
 * to one channel; output H(x) = x + N(x).  Every level is 32 channels wide.
 * The convolutions followed by batch normalisation have no bias.  BF16
 * weights and activations with FP32 accumulation on the matrix cores.
 *
 * Parameters (float32, CLAMP_UNET_PARAMS values): for each of the 12
 * batch-normalised convolutions (encoder blocks 1, 2, 3, then decoder blocks
 * 3, 2, 1, two each) W[27][Cin][32] (Cin = 1 for the first, else 32; taps as
 * for the CNN), gamma[32], beta[32]; for each transposed convolution
 * (decoder blocks 3, 2, 1) W[8][32][32] with sub-position s = 4a + 2b + c of
 * output voxel (2z+a, 2y+b, 2x+c), then b[32]; the final W[27][32][1], b[1].
 * Running statistics (float32, CLAMP_UNET_STATS values): per batch
 * normalisation mean[32] then variance[32].  Apply uses evaluation mode: the
 * running statistics, folded into the convolutions (eps 1e-5).
 * Volumes are float32 [nvol][nz][ny][nx] with nz and ny multiples of 8 and
 * nx a multiple of 128 (the third level's rows are 32-voxel tiles).
 * ------------------------------------------------------------------------ */
#define CLAMP_UNET_PARAMS 331297
#define CLAMP_UNET_STATS (12 * 2 * 32)
typedef struct clamp_unet clamp_unet;

/* Allocates device parameters (zero), running statistics (mean 0, variance
 * 1) and evaluation weights on the current device (CLAMP_EDEVICE without
 * one, CLAMP_ENOMEM when allocation fails).  Destroy frees them; call it
 * only after every call using the object has completed on the device. */
clamp_status clamp_unet_create(clamp_unet** out);
clamp_status clamp_unet_destroy(clamp_unet* unet);
/* Copies HOST parameters and running statistics (NULL: mean 0, variance 1)
 * in, and rebuilds the evaluation weights, or copies either out (NULL skips
 * it).  Synchronous device copies: finish the work of other streams that
 * uses the object first.  set_params rejects non-finite values and negative
 * variances with CLAMP_EINVAL (nothing is changed). */
clamp_status clamp_unet_set_params(clamp_unet* unet, const float* params, const float* stats);
clamp_status clamp_unet_get_params(const clamp_unet* unet, float* params, float* stats);
/* Workspace bytes for apply (train = 0) or gradient (train = 1) calls on
 * nvol volumes of nz x ny x nx.  Errors shared by the sized calls:
 * CLAMP_EINVAL for non-positive sizes or NULL arguments, CLAMP_ESHAPE when nz
 * or ny is not a multiple of 8, nx not a multiple of 128, or nvol nz ny nx >=
 * 2^31. */
clamp_status clamp_unet_workspace_size(int32_t nvol, int32_t nz, int32_t ny, int32_t nx, int32_t train,
                                       size_t* bytes);
/* out = H(x) per volume (device float32 arrays), evaluation mode.
 * normalize != 0 applies the scale-free form out = x + m N(x / m) with m the
 * mean of all nvol volumes.  x and out must not overlap (CLAMP_EINVAL). */
clamp_status clamp_unet_apply(clamp_unet* unet, const float* x, float* out, int32_t nvol, int32_t nz, int32_t ny,
                              int32_t nx, int32_t normalize, void* workspace, void* hip_stream);
/* Training mode: mean squared error of H(x) against target over the batch
 * into *loss (device double), with batch normalisation on the batch
 * statistics (biased variance), and its gradient with respect to every
 * parameter into grad (device float32 [CLAMP_UNET_PARAMS]; NULL keeps it
 * inside the object for clamp_unet_adam_step).  Updates the running
 * statistics (momentum 0.1, unbiased variance). */
clamp_status clamp_unet_grad(clamp_unet* unet, const float* x, const float* target, int32_t nvol, int32_t nz,
                             int32_t ny, int32_t nx, double* loss, float* grad, void* workspace, void* hip_stream);
/* One Adam step with gradient-norm clipping, as clamp_cnn_adam_step, with
 * the gradient of the last clamp_unet_grad call that kept it inside the
 * object.  clamp_unet_set_params resets the Adam state. */
clamp_status clamp_unet_adam_step(clamp_unet* unet, float lr, void* hip_stream);

/* Optional per-stage timing (for benchmarks).  While enabled, every call
 * that takes a stream records a pair of HIP events on that stream around
 * each of its stages; clamp_plan_get_timing waits for the recorded events,
 * writes the summed milliseconds and launch counts of each stage
 * (HOST arrays of CLAMP_STAGES entries, see clamp_stage_name) and forgets
 * the records.  Enabling timing makes the plan unsafe to share between
 * threads.  Creating events can fail with CLAMP_EDEVICE. */
#define CLAMP_STAGES 15
clamp_status clamp_plan_set_timing(clamp_plan* plan, int32_t enable);
/* Timing of the stages whose bit is set in stage_mask only (bit s = stage s;
 * 0 turns timing off, all CLAMP_STAGES bits equal clamp_plan_set_timing(1)):
 * a benchmark can time its dominant stage with two events per call instead
 * of a pair around every stage.  CLAMP_EINVAL for bits at or past
 * CLAMP_STAGES. */
clamp_status clamp_plan_set_timing_stages(clamp_plan* plan, uint32_t stage_mask);
clamp_status clamp_plan_get_timing(clamp_plan* plan, double* total_ms, int32_t* launches);
/* Name of a timing stage ("" outside [0, CLAMP_STAGES)). */
const char* clamp_stage_name(int32_t stage);

/* Message for the calling thread's last non-OK status ("" if none). */
const char* clamp_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* CLAMP_H */
