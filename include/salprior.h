/*
 * salprior -- C-ABI of the MI355X (gfx950) saliency -> Kalman prior -> MRF weight path.
 *
 * The method follows Akamine, Fukuchi, Kimura, Takagi, "Fully automatic extraction of
 * salient objects from videos in near real-time" (arXiv:1008.0502):
 *   - the saliency map of each frame from intensity, colour-opponent, orientation and
 *     motion features (Section 3; GPU steps in Section 7.2: pixel-wise features,
 *     Gaussian pyramids, normalisation by global and local extrema, weighted sum);
 *   - the saliency-based prior with a near-zero prior on the frame edge (Section 5);
 *   - the Kalman update of the prior from the previous frame (Section 6);
 *   - the unary (t-link) and pairwise (n-link) capacities of the MRF whose minimum cut
 *     gives the segmentation (Section 4, Eqs. 1-4).  The cut itself is not part of
 *     this library.
 *
 * Conventions for every call:
 *   - All image/map pointers are DEVICE pointers on the context's GPU, row-major,
 *     tightly packed, owned by the caller, and must stay valid until the work
 *     enqueued on the context's HIP stream has run.  RGB frames are uint8 [H][W][3].
 *   - Calls enqueue asynchronously on the context's stream and never synchronise
 *     (saliency_backward copies a few scalars host->device first).  Device faults
 *     surface at the caller's next synchronisation.
 *   - Return 0 on success or a negative SP_E* code; sp_last_error() (per host thread)
 *     then describes the failure.  No C++ exception crosses this interface.  A failed
 *     call leaves the context usable.
 */
#ifndef SALPRIOR_H
#define SALPRIOR_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SP_OK 0
#define SP_EINVAL (-1) /* bad argument (NULL, non-finite or out-of-range parameter) */
#define SP_ESHAPE (-2) /* frame too small / too large for the requested pyramid */
#define SP_ENOMEM (-3) /* device allocation failed */
#define SP_EHIP (-4)   /* a HIP runtime call failed; the message names it */
#define SP_ESTATE (-5) /* call not valid in the context's state (e.g. no tape) */

#define SP_NCHANNELS 8 /* I, RG, BY, O0, O45, O90, O135, M */
#define SP_MAX_LEVELS 12

typedef struct sp_ctx sp_ctx;
typedef struct sp_batch sp_batch;

/* Parameters.  sp_default_params() fills the defaults noted below. */
typedef struct sp_params {
  int32_t depth;       /* pyramid depth D; <= 0: floor(log2(min(H, W))) - 1 */
  int32_t n_centers;   /* number of centre levels, 1..4 (default 2: {1, 2}) */
  int32_t centers[4];
  int32_t n_deltas;    /* number of centre-surround offsets, 1..4 (default 2: {2, 3}) */
  int32_t deltas[4];   /* pairs (c, c + delta) whose surround exceeds D are dropped */
  float weights[8];    /* channel weights of the saliency sum, order as SP_NCHANNELS (1) */
  double q;            /* Kalman process variance Q = sigma_2^2 of Section 6 (1e-3) */
  double r;            /* Kalman observation-side variance R = sigma_1^2 (1e-1) */
  float eps;           /* near-zero prior: border value and clamp of q (1e-4) */
  int32_t border;      /* width of the border ring whose prior is eps (1) */
  float lambda;        /* contrast weight of the pairwise capacity (1) */
  float potts;         /* constant of the generalised Potts prior (0) */
  int32_t lm_block;    /* block edge of the local maxima in N(.): must be 8 */
  float flat_tol;      /* a map whose range is <= flat_tol normalises to 0 (1e-5) */
  float gabor_lambda;  /* Gabor wavelength in pixels (4) */
  float gabor_sigma;   /* Gabor envelope sigma (2) */
  int32_t gabor_radius;/* Gabor kernel radius, 1..8 (6: a 13x13 kernel) */
  int32_t record_tape; /* >0: frames the adjoint tape can hold (0: no tape) */
  /* Variants of the prior.  A context that records a tape must keep the defaults. */
  int32_t f_mode;      /* prediction f of Section 6 from the previous segmentation (or, without
                          one, from the previous prior): 0 = 5x5 binomial blur (default);
                          1 = distance transform, f = exp(-d^2 / (2 dt_sigma^2)) with d the
                          Euclidean distance to the nearest object pixel (the stand-in object
                          is prior > 1/2); f = 0 when there is no object pixel */
  float dt_sigma;      /* f_mode 1: decay length in pixels, 0 < dt_sigma <= 4 (2) */
  double ssm_q;        /* stochastic saliency map (Section 3): with ssm_r > 0 the observation */
  double ssm_r;        /* is taken from a per-pixel Kalman filter of S with process variance
                          ssm_q >= 0 and observation variance ssm_r (0, 0: off) */
  /* Colour likelihood of the t-links (sp_colour_likelihood). */
  int32_t gmm_components; /* Gaussians per label, 0..4 (3; 0: the call is unavailable) */
  int32_t gmm_iters;   /* EM iterations after the start, 0..100 (10) */
  float gmm_reg;       /* added to every covariance diagonal, colours in [0, 1] (1e-4) */
} sp_params;

/* Geometry of a context, as derived by sp_create. */
typedef struct sp_geometry {
  int32_t H, W;          /* level-0 size */
  int32_t depth;         /* D */
  int32_t top;           /* deepest level any pair uses */
  int32_t c_min, c_max;  /* smallest and largest centre level with a pair */
  int32_t n_pairs;
  int32_t pair_c[16], pair_s[16];
  int32_t level_h[SP_MAX_LEVELS + 1], level_w[SP_MAX_LEVELS + 1];
  int32_t Hc, Wc;        /* size of the saliency map = level c_max */
} sp_geometry;

/* Fills p with the defaults listed in sp_params.  p must not be NULL. */
void sp_default_params(sp_params* p);

/* Creates a context for H x W frames on the current HIP device, enqueuing on
 * hip_stream (a hipStream_t; NULL = the default stream).  Validates p against H and W
 * and allocates every buffer the context will use (scratch, pyramid, Kalman state,
 * tape); no later call allocates device memory.  *out receives the context. */
int sp_create(const sp_params* p, int32_t H, int32_t W, void* hip_stream, sp_ctx** out);

/* Frees everything the context owns (after synchronising its stream).  NULL is a no-op. */
int sp_destroy(sp_ctx* ctx);

/* Changes the stream later calls enqueue on. */
int sp_set_stream(sp_ctx* ctx, void* hip_stream);

/* Copies the context's geometry to *out. */
int sp_get_geometry(const sp_ctx* ctx, sp_geometry* out);

/* Replaces the channel weights and the Kalman variances (finite, q >= 0, r >= 0,
 * q + r > 0).  Takes effect from the next call; the gain sequence restarts only on
 * sp_reset.  After recorded steps it invalidates the tape (saliency_backward then
 * fails with SP_ESTATE until sp_reset). */
int sp_set_weights(sp_ctx* ctx, const float* weights8, double q, double r);

/* Starts a new clip: the next prior_update is step t = 0 (prior = observation) and the
 * tape is emptied. */
int sp_reset(sp_ctx* ctx);

/* Step index the next prior_update will run (frames updated since sp_reset). */
int64_t sp_step_index(const sp_ctx* ctx);

/* Generation of the recorded clip: a counter that sp_reset, sp_set_weights and
 * sp_set_state each advance (-1 for a NULL context).  A caller that runs the forward
 * clip, then later the adjoint, compares the value taken after the forward with the
 * value before the backward: a change means the tape was restarted or no longer
 * matches the weights and variances it was recorded with. */
int64_t sp_tape_generation(const sp_ctx* ctx);

/* Saliency map of one frame (Section 3; Section 7.2).
 *   rgb_t    [H][W][3] uint8, frame t.
 *   rgb_prev [H][W][3] uint8, frame t-1, or NULL (first frame: the motion feature is 0).
 *   S_out    [Hc][Wc] float: S = sum_k w_k C_k.
 *   C_out    [8][Hc][Wc] float conspicuity maps, or NULL.
 * When the context records a tape, the checkpoint of this frame's pyramid level c_min
 * and S are stored for the adjoint. */
int saliency_forward(sp_ctx* ctx, const uint8_t* rgb_t, const uint8_t* rgb_prev, float* S_out, float* C_out);

/* Kalman prior update (Section 6) from a saliency map (Section 5).
 *   S          [Hc][Wc] float, normally the S_out of saliency_forward for this frame.
 *   seg_prev   [H][W] uint8 labels {0,1} of the previous frame (the caller's graph cut),
 *              or NULL: the previous prior stands in for it.
 *   prior_out  [H][W] float receives p-hat(A_{x,t} = 1); may be NULL (the context keeps
 *              its own copy as the Kalman state).
 * q_t = clamp(upsample(S / max S), eps, 1 - eps) with q = eps on the border ring and
 * q = 0.5 when max S <= flat_tol; t = 0: prior = q_0; t >= 1: f = G * prev,
 * prior = f + K_t (q_t - f), K_t = (P_{t-1} + Q) / (P_{t-1} + Q + R), P_t = R K_t,
 * prior = eps on the border ring.  Advances the step index. */
int prior_update(sp_ctx* ctx, const float* S, const uint8_t* seg_prev, float* prior_out);

/* Starts a clip from manual labels (Section 4's manual-label prior; the first frame of
 * the "Manual" comparison of Section 8.1) instead of a saliency observation:
 *   labels     [H][W] uint8: 1 = object, 0 = background, any other value = no label.
 *   prior_out  [H][W] float or NULL receives p(A_x = 1): 1, eps and 0.5 respectively.
 * The prior becomes the Kalman state of step 0 with variance R (no border ring), so the
 * next prior_update is step 1.  Resets the clip first (like sp_reset). */
int sp_manual_prior(sp_ctx* ctx, const uint8_t* labels, float* prior_out);

/* The stochastic saliency map of the last prior_update (ssm_r > 0): *mean receives a
 * device pointer to the per-pixel means [Hc][Wc] (valid until the next update), *var
 * the variance shared by every pixel.  SP_ESTATE when the map is off or no update has
 * run since the reset. */
int sp_stochastic_saliency(const sp_ctx* ctx, const float** mean, double* var);

/* MRF capacities (Section 4, Eqs. 1-4) of one frame and its prior.
 *   rgb_t        [H][W][3] uint8.
 *   prior        [H][W] float p(A_x = 1).
 *   unary_out    [2][H][W] float: U0 = -ln(1 - min(p, 1-eps)) (cost of label 0,
 *                background) and U1 = -ln max(p, eps) (cost of label 1, object).
 *   pairwise_out [4][H][W] float: capacity between (y, x) and its E, S, SE, SW
 *                neighbour, potts + lambda * exp(-beta ||dC||^2) / ||dx||, 0 outside.
 *   beta_out     [1] float or NULL: beta = 1 / (2 mean ||dC||^2) over all 8-neighbour
 *                pairs (0 for a constant frame). */
int mrf_weights(sp_ctx* ctx, const uint8_t* rgb_t, const float* prior, float* unary_out, float* pairwise_out,
                float* beta_out);

/* Colour likelihood of the t-links (Section 4: psi_1(D | A_x) = -log p(C_x | A_x), p a
 * Gaussian mixture over RGB fitted by EM; Section 5: every pixel is a sample weighted by
 * the prior; Section 8.1: M = 3).  For each label it fits a mixture of
 * p->gmm_components Gaussians (full covariances, colours RGB / 255) by weighted EM -- the
 * object's samples weighted by prior, the background's by 1 - prior -- starting from the
 * label's weighted mean and covariance with the means spread along the covariance's
 * leading eigenvector, for p->gmm_iters iterations (covariances + gmm_reg I), then adds
 * psi_1 of each label to its unary cost.  A label whose weight vanishes adds nothing.
 *   rgb_t        [H][W][3] uint8.
 *   prior        [H][W] float p(A_x = 1).
 *   unary_inout  [2][H][W] float: U0 += psi_1(C | A = 0), U1 += psi_1(C | A = 1) (pass
 *                zeros to receive psi_1 alone, or mrf_weights' unary_out to get both terms).
 *   gmm_out      [2][M][10] float or NULL: per label and component the weight, mean (3)
 *                and covariance (xx, xy, xz, yy, yz, zz); zeros for dropped components.
 * SP_ESTATE when the context was created with gmm_components = 0. */
int sp_colour_likelihood(sp_ctx* ctx, const uint8_t* rgb_t, const float* prior, float* unary_inout, float* gmm_out);

/* Minimum cut of the MRF (Section 4: the MAP labelling is the minimum s-t cut of the graph
 * of Eqs. 2-4), the segmentation that closes the loop of Section 6 when passed as the next
 * frame's seg_prev.  An sp_cut holds the residual graph of H x W frames (44 bytes per
 * pixel, allocated by sp_cut_create, freed by sp_cut_destroy; NULL is a no-op there) and
 * enqueues on hip_stream (NULL = the default stream).
 *   unary     [2][H][W] float: U0 (cost of the background), U1 (cost of the object).
 *   pairwise  [4][H][W] float: the E, S, SE, SW n-link capacities of mrf_weights.
 *   scale     > 0: capacities become integers q = rint(c * scale) (FP32, half to even),
 *             clamped to [0, 2^24], so the flow is exact.
 *   labels    [H][W] uint8 receives 1 (object: source side) or 0 (background).
 *   flow_out  [1] int64 (device) or NULL receives the maximum flow = the cut's cost in
 *             the integer capacities.
 * The source side is the object: a background pixel pays U0, an object pixel U1, and each
 * 8-neighbour pair with different labels its capacity.  Among all minimum cuts the one
 * with the largest object is returned (a pixel is background exactly when it can still
 * reach the sink in the residual graph of a maximum flow), so the labelling is unique.
 * Push-relabel with exact global relabelling on the GPU; sp_mincut synchronises the stream
 * between its rounds.  SP_ESTATE if it has not converged after 65536 push rounds. */
typedef struct sp_cut sp_cut;
int sp_cut_create(int32_t H, int32_t W, void* hip_stream, sp_cut** out);
int sp_cut_destroy(sp_cut* cut);
int sp_mincut(sp_cut* cut, const float* unary, const float* pairwise, float scale, uint8_t* labels,
              int64_t* flow_out);

/* The whole per-frame path in one call, with fewer kernel launches than the three
 * calls above: saliency_forward, then prior_update on S_out, then (when unary_out and
 * pairwise_out are both given) mrf_weights on the new prior.  The pairwise capacities
 * are computed in the feature pass and the unary ones in the prior pass.  Arguments
 * as in those calls (S_out required; C_out, seg_prev, prior_out, unary_out,
 * pairwise_out, beta_out optional).  Records the tape like the separate calls. */
int sp_step(sp_ctx* ctx, const uint8_t* rgb_t, const uint8_t* rgb_prev, const uint8_t* seg_prev, float* S_out,
            float* C_out, float* prior_out, float* unary_out, float* pairwise_out, float* beta_out);

/* Adjoint of the clip recorded since sp_reset (requires record_tape >= T and exactly T
 * prior updates since the reset).
 *   grad_prior [T][H][W] float: dL/d prior_t for every recorded step.
 *   grad_w [8], grad_q [1], grad_r [1] float (device): dL/dw, dL/dQ, dL/dR.
 * The conspicuity maps are recomputed from the checkpointed pyramid level c_min. */
int saliency_backward(sp_ctx* ctx, const float* grad_prior, int32_t T, float* grad_w, float* grad_q,
                      float* grad_r);

/* Pixel-level adjoint: dL/d frame for every frame of the clip, through the saliency model
 * (N(.), the across-scale sum, centre-surround, the Gabor maps, the pyramid and the level-0
 * features of Section 3 / Section 7.2); the motion feature also carries gradient to the
 * previous frame.  Run saliency_backward for the clip first: this call continues from its
 * dL/dS of every frame.  The frames' maps are recomputed from the frames.
 *   frames       [T][H][W][3] uint8 (device): the clip the forward ran, in order.
 *   grad_frames  [T][H][W][3] float (device): receives dL/d(frame value), per unit of the
 *                0..255 scale (the frames taken as real numbers).
 * Non-differentiable points: the chromatic mask and colour maximum are held fixed; the
 * global minimum and maximum and each 8x8 block maximum of an N(.) input take the gradient
 * at the first row-major position within 2^-20 of the map's range of the extreme; a map at
 * or below flat_tol passes none; the derivative of a centre-surround |D| is 0 where |D| is
 * at most 2^-16 of the pair's largest |value| (below FP32's resolution of the maps; flat
 * regions of both levels make D vanish identically) and sign(D) elsewhere; the feature
 * branches are decided on the frame bytes (2R - G - B > 0 and its like, min(R, G) > B,
 * R <= G for the min, the sign of the byte-sum difference for the motion, 0 on a tie);
 * max(0, .) passes nothing at 0.
 * SP_ESTATE unless saliency_backward of these T steps ran last on this tape. */
int saliency_backward_frames(sp_ctx* ctx, const uint8_t* frames, int32_t T, float* grad_frames);

/* Fitting loss helper: loss = mean over [T][H][W] of (prior - mask)^2 and its gradient.
 *   prior [T][H][W] float, mask [T][H][W] uint8 {0,1}, loss [1] float,
 *   grad_prior [T][H][W] float or NULL. */
int sp_mse_mask_loss(sp_ctx* ctx, const float* prior, const uint8_t* mask, int32_t T, float* loss,
                     float* grad_prior);

/* Checkpoint / resume of the Kalman state: the prior of the last step plus the step
 * index and variance.  sp_state_size gives the byte size; buffers are device memory. */
int sp_state_size(const sp_ctx* ctx, size_t* bytes);
int sp_get_state(sp_ctx* ctx, void* dev_buf, size_t bytes);
int sp_set_state(sp_ctx* ctx, const void* dev_buf, size_t bytes);

/* Batched form: n independent streams of possibly different sizes, one frame each per
 * step, every phase of the step in one launch over all streams, the step captured once
 * in a HIP graph and replayed.  Each stream keeps its Kalman state on the device.
 *   H[n], W[n]: host arrays.  p: shared parameters.  With p->record_tape = T > 0 every
 *   stream records an adjoint tape of up to T steps (sp_batch_backward); a step beyond
 *   the tape fails with SP_ESTATE until sp_batch_reset.
 *   flags: SP_BATCH_MRF also computes every stream's MRF capacities each step into
 *   buffers the batch owns (read them with sp_batch_outputs); see also SP_BATCH_CONSP. */
#define SP_BATCH_MRF 1
/* SP_BATCH_CONSP also keeps every stream's 8 conspicuity maps of the last step (read
 * them with sp_batch_consp). */
#define SP_BATCH_CONSP 2
int sp_batch_create(const sp_params* p, int32_t n, const int32_t* H, const int32_t* W, int32_t flags,
                    void* hip_stream, sp_batch** out);

/* One step.  rgb_ptrs: DEVICE array of n device pointers to this step's frames, read by
 * the step's first launch when it runs (the array must stay valid until then; the frames
 * until the next step has run, which reads them as the previous frames).  prior_ptrs:
 * DEVICE array of n device pointers receiving the priors, or NULL (then read them with
 * sp_batch_prior). */
int sp_batch_step(sp_batch* b, const uint8_t* const* rgb_ptrs, float* const* prior_ptrs);

/* n consecutive steps in one graph launch: the same kernels, in the same order and with the
 * same results, as n calls of sp_batch_step(b, rgb_tables[k], NULL), without the idle time
 * the device spends between two graph launches.  rgb_tables: HOST array of n (1..1024)
 * DEVICE frame tables as in sp_batch_step (each must stay valid until its step has run).
 * The graph is captured on the first call with a given n and kept; later calls re-point
 * the steps whose table changed.  A tape (record_tape > 0) must have room for all n steps
 * (else SP_ESTATE and no step runs).  Read the priors with sp_batch_prior afterwards. */
int sp_batch_steps(sp_batch* b, int32_t n, const uint8_t* const* const* rgb_tables);

/* Device pointer to stream i's current prior (valid until the next step). */
int sp_batch_prior(sp_batch* b, int32_t i, const float** prior);
/* Device pointers to stream i's saliency map [Hc][Wc] and, with SP_BATCH_MRF, its
 * unary [2][H][W], pairwise [4][H][W] capacities and beta [1] of the last step (any
 * output pointer may be NULL; the MRF ones are NULL without SP_BATCH_MRF). */
int sp_batch_outputs(sp_batch* b, int32_t i, const float** S, const float** unary, const float** pairwise,
                     const float** beta);
/* Device pointer to stream i's conspicuity maps [8][Hc][Wc] of the last step (NULL
 * without SP_BATCH_CONSP). */
int sp_batch_consp(sp_batch* b, int32_t i, const float** C);
int sp_batch_reset(sp_batch* b);
int sp_batch_destroy(sp_batch* b);

/* Channel weights w[8] and Kalman variances q, r (host values) shared by every stream
 * of the batch.  Steps already recorded used the old values, so a tape holding any
 * steps becomes invalid for sp_batch_backward until sp_batch_reset.  Synchronises. */
int sp_batch_set_weights(sp_batch* b, const float* w, double q, double r);
/* Steps run since the last reset (-1 for NULL), and a counter bumped by every reset,
 * autotune and weight change (a caller holding a recorded clip can tell whether the
 * tape still holds it). */
int64_t sp_batch_step_index(const sp_batch* b);
int64_t sp_batch_tape_generation(const sp_batch* b);

/* Batched form of the adjoint (record_tape > 0).  The clip of every stream is the steps
 * since the last sp_batch_reset; the recursion and its adjoint follow Section 6 as in
 * saliency_backward, for each stream on its own.
 *   sp_batch_tape_prior: device pointer to stream i's recorded priors [cap][H][W] (row t
 *     holds the prior of step t).
 *   sp_batch_mse_mask_loss: for every stream i, loss[i] = mean over [T][H][W] of
 *     (prior - mask_i)^2 on its first T recorded priors (T <= steps recorded).
 *     masks: HOST array of n device pointers, mask_i [T][H][W] uint8 in {0,1}.
 *     loss: device [n] float.  grad_prior: HOST array of n device pointers receiving
 *     dL_i/dprior [T][H][W] float, or NULL.
 *   sp_batch_backward: gradients of every stream's loss L_i, given grad_prior (HOST array
 *     of n device pointers, [T][H][W] float each, dL_i/dprior_t), for exactly T = the
 *     steps recorded since the reset.  grad_w: device [n][8], grad_q, grad_r: device [n].
 *     The conspicuity maps are recomputed from every stream's checkpointed level c_min,
 *     a few frames of every stream per launch.
 * The host arrays are read during the call; the device buffers must stay valid until
 * the stream reaches the call's launches.  The tables the calls upload are staged in
 * pinned host memory; refilling a stage waits for its previous upload. */
int sp_batch_tape_prior(sp_batch* b, int32_t i, const float** prior);
int sp_batch_mse_mask_loss(sp_batch* b, const uint8_t* const* masks, int32_t T, float* loss,
                           float* const* grad_prior);
int sp_batch_backward(sp_batch* b, const float* const* grad_prior, int32_t T, float* grad_w, float* grad_q,
                      float* grad_r);

/* Measurement hook: while enabled, every kernel launch of the context is bracketed by
 * a pair of HIP events recorded on the context's stream (one pair per launch, up to
 * 65536 pairs).  sp_profile_read synchronises the stream and returns, per kernel kind
 * 0..SP_NKINDS-1, the summed device time in ms and the number of launches since the
 * last read (arrays of length n >= SP_NKINDS), then clears the record. */
#define SP_NKINDS 29
int sp_profile_enable(sp_ctx* ctx, int32_t enable);
int sp_profile_read(sp_ctx* ctx, int32_t n, float* total_ms, int32_t* launches);
/* The same measurement hook for a batch: while enabled, sp_batch_step launches the
 * step's phases one by one (the same kernels as the graph) bracketed by events. */
int sp_batch_profile_enable(sp_batch* b, int32_t enable);
int sp_batch_profile_read(sp_batch* b, int32_t n, float* total_ms, int32_t* launches);
/* Measurement hook for HBM byte counters: copies `bytes` (a positive multiple of 16, at
 * most 2 GiB) from device buffer src to device buffer dst on the given stream, with one
 * of the access forms the kernels use: mode 0 = a 4-byte load and store per lane, 1 = a
 * 16-byte load and store per lane, 2 = 4-byte direct global-to-LDS loads, then 4-byte
 * stores from LDS.  A counter run over it reads against a known byte count. */
int sp_calibration_copy(const void* src, void* dst, size_t bytes, int32_t mode, void* hip_stream);

/* Name of the kernel behind kind k (static string; "" if out of range). */
const char* sp_kernel_name(int32_t k);

/* Autotuner.  Times the candidate launch shapes of the batch -- the width (16, 32 or 64
 * pixels) of the level-0 update tiles per resolution, and the XCD-aware order of the
 * job tables on or off -- over `steps` eager steps each on the given frames (device
 * array of n device pointers, as in sp_batch_step), keeps the fastest, records the
 * choice per resolution for batches and contexts created later in this process, and
 * resets the batch.  The candidates compute identical results.  report (may be NULL)
 * receives a text summary.  Synchronises. */
int sp_batch_autotune(sp_batch* b, const uint8_t* const* rgb_ptrs, int32_t steps, char* report, size_t report_len);
/* The same for one context, timing the fused step on rgb_t (rgb_prev may be NULL);
 * resets the context. */
int sp_autotune(sp_ctx* ctx, const uint8_t* rgb_t, const uint8_t* rgb_prev, int32_t steps, char* report,
                size_t report_len);

/* Forces the launch shapes the autotuner would otherwise choose: the width (16, 32 or
 * 64) of the level-0 update tiles, the XCD-aware job order (0/1) and the channels per
 * across-scale workgroup (1, 2, 4 or 8; rejected when the LDS of that many channels
 * exceeds the limit for the geometry).  Every choice computes identical results.  The
 * context form synchronises its stream; the batch form drops the captured graph, which
 * is captured again at the next step. */
int sp_set_tune(sp_ctx* ctx, int32_t kalman_tw, int32_t xcd_order, int32_t channels);
int sp_batch_set_tune(sp_batch* b, int32_t kalman_tw, int32_t xcd_order, int32_t channels);
/* Forgets every autotuner choice recorded in this process (contexts and batches created
 * later start from the defaults: tile width 32, no XCD order, 2 channels). */
int sp_tune_cache_clear(void);

/* Allocation-free form of saliency_forward, for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc).  It needs no context: it validates p against H and W like sp_create, lays
 * the stream's pyramid, maps, partials and job table out in a device array the library
 * holds for each GPU from its load until the process ends (SP_NOALLOC_MAX_BYTES), and
 * computes S_out and C_out (optional) of one frame exactly as saliency_forward of a
 * context with the same parameters does (same kernels, same launch shapes).  Arguments
 * as in saliency_forward; hip_stream is a hipStream_t (NULL = the default stream).
 * It calls no allocation routine.  It copies its job table into the array and waits for
 * that copy (and so for earlier work on hip_stream) before enqueuing the kernels.  Every
 * call on one GPU uses that GPU's one array: calls that overlap on a GPU (other host
 * threads, other streams) race and must be serialised by the caller.  Nothing in the
 * array needs to start at zero: each call writes what it reads.  A frame whose layout
 * exceeds the array fails with SP_ESHAPE (the message gives the bytes it needs). */
#define SP_NOALLOC_MAX_BYTES (64u << 20)
int sp_saliency_noalloc(const sp_params* p, int32_t H, int32_t W, const uint8_t* rgb_t, const uint8_t* rgb_prev,
                        float* S_out, float* C_out, void* hip_stream);

/* Description of the last error on this host thread ("" if none). */
const char* sp_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* SALPRIOR_H */
