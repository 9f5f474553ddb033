/*
 * sad.h -- C ABI of the Soft Anisotropic Diagrams (SAD) hot path on AMD MI355X (gfx950).
 *
 * Conventions shared by every entry point
 *   - Pointers are DEVICE pointers unless marked "host".  The caller owns every buffer
 *     (inputs, outputs and scratch); the library allocates nothing, never synchronises
 *     and never reads device memory on the host, so every call may be recorded into a
 *     HIP graph.  Work is enqueued on `stream` (a hipStream_t; NULL = default stream)
 *     and the call returns.
 *   - Arguments are validated on the host before anything is enqueued: a bad argument
 *     returns SAD_ERR_INVALID_ARGUMENT or SAD_ERR_UNSUPPORTED and enqueues nothing.  A
 *     launch failure returns SAD_ERR_DEVICE.  sad_last_error() returns a message for
 *     the last failing call on the calling thread.  Faults inside a kernel surface at
 *     the caller's next synchronisation.
 *   - Site buffer `sites`: float[10][cap], parameter-major, in the order
 *     (x, y, log_tau, r, c_r, c_g, c_b, u_x, u_y, a) of App. B.2 ("Site buffer").  Slot
 *     i is site ID i.  A site is active iff x >= 0 and all ten values are finite
 *     (inactive sites have x = y = -1); every kernel skips inactive sites.
 *   - Derived-record buffer `rec`: float[n_slots][SAD_REC_FLOATS], written by
 *     sad_prepare_sites from `sites`; every image-space call reads `rec`, so call
 *     sad_prepare_sites after any change of `sites` (sad_adam_step can refresh it).
 *   - Top-K list field `topk`: uint32[K/4][H*W][4] ("two 4-channel textures" for
 *     K = 8, App. B.2): plane k/4, pixel p = i*W + j, lane k%4.  Each pixel's list is
 *     sorted by (score descending, ID ascending) and padded with SAD_INVALID_ID.
 *   - Images: float[3][H][W] (channel-major).  Pixel (row i, column j) is the point
 *     (x, y) = (j, i).
 *   - The score of site i at point x (Sec. 4.1-4.2) is
 *        l_i(x) = tau_i s (r_i - ||x - p_i||_{G_i}),  G_i = e^a u u^T + e^-a v v^T,
 *     v = (-u_y, u_x), tau = exp(log_tau), s = score scale; it is evaluated in float32
 *     in one fixed sequence of correctly rounded operations, so the lists are
 *     reproducible bit for bit.
 */
#ifndef SAD_H
#define SAD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    SAD_OK = 0,
    SAD_ERR_INVALID_ARGUMENT = 1,
    SAD_ERR_UNSUPPORTED = 2,
    SAD_ERR_WORKSPACE = 3,
    SAD_ERR_DEVICE = 4
} sad_status;

#define SAD_NPARAM 10
#define SAD_REC_FLOATS 16
#define SAD_INVALID_ID 0xFFFFFFFFu
#define SAD_MAX_K 32

/* One image and its site set.  K must be a multiple of 4 in [4, SAD_MAX_K].
 * n_slots <= cap: site IDs are 0..n_slots-1 (injected IDs are drawn from this range).
 * score_scale: s of Sec. 4.1; 0 selects 1/max(H, W). */
typedef struct {
    int32_t H, W;
    int32_t K;
    int32_t n_slots;
    int64_t cap;
    float score_scale;
} sad_image;

/* Device accumulator of the MSE loss.  A call that reports the loss adds L to `value`;
 * part[] is scratch that every call leaves at zero (zero the whole struct once).  The
 * loss is summed in per-block partials spread over SAD_LOSS_PARTS addresses and folded
 * by a single-block pass, so no single address takes one atomic per block. */
#define SAD_LOSS_PARTS 64
typedef struct {
    float value;
    float part[SAD_LOSS_PARTS];
} sad_loss_acc;

/* Adam hyper-parameters (Sec. 5: per-parameter base learning rates, fixed betas and
 * epsilon).  lr[p] is the learning rate of parameter p in the site order above. */
typedef struct {
    float lr[SAD_NPARAM];
    float beta1, beta2, eps;
} sad_adam_params;

/* ---- a0: per-site derived values (the "pack" kernel of App. B.2 / B.7) ----------
 * rec[i] = {x, y, G11, 2*G12, G22, kappa, r, valid, c_r, c_g, c_b, u_x, u_y, e^a,
 *           e^-a, tau} for every slot i < n_slots, with tau = f32(exp(double log_tau)),
 * e^{+-a} = f32(exp(+-double a)), kappa = tau * s, G11 = fma(e^a, u_x^2, e^-a u_y^2),
 * G22 = fma(e^a, u_y^2, e^-a u_x^2), G12 = (e^a - e^-a) u_x u_y; valid = 1 for an
 * active site with finite kappa > 0 and finite G, else 0 (the record is then ignored).
 * sites: [10][cap] (read); rec: [n_slots][16] (written). */
sad_status sad_prepare_sites(const sad_image *img, const float *sites, float *rec, void *stream);

/* ---- a2: list initialisation (the seed pass of App. B.3) --------------------------
 * Clears every slot to SAD_INVALID_ID, then maps each valid site to the pixel
 * (rint(y), rint(x)) clamped to the image; a pixel's list becomes the top K of the
 * sites mapped to it.  Deterministic.  scratch: uint64[H*W] (contents undefined after;
 * the K*4 bytes per pixel of a second list field are enough). */
sad_status sad_seed_topk(const sad_image *img, const float *rec, uint32_t *topk,
                         uint64_t *scratch, void *stream);

/* sad_seed_topk for callers that cannot allocate device memory (code under HIP graph
 * capture, serving loops, harnesses that forbid hipMalloc): the same result, with the
 * per-pixel scratch taken from a static array in the library's own device memory
 * instead of an argument.  The array holds SAD_SEED_STATIC_PIXELS uint64 words (32 MiB)
 * on every device the library runs on, until the process ends; its address on a device
 * is looked up on the first call made with that device current.  Images of more than
 * SAD_SEED_STATIC_PIXELS pixels are rejected with SAD_ERR_WORKSPACE.  The call allocates
 * nothing.  Every call on one device shares that device's array (each call clears what
 * it uses with a kernel), so calls that overlap on one device -- on different streams or
 * from different threads -- race and must be ordered by the caller. */
#define SAD_SEED_STATIC_PIXELS (1 << 22)
sad_status sad_seed_topk_noalloc(const sad_image *img, const float *rec, uint32_t *topk,
                                 void *stream);

/* ---- a3: one propagation pass (Sec. 4.3 update equation) --------------------------
 * Jacobi: reads topk_in everywhere, writes topk_out (must not alias).  Candidate set of
 * pixel p: its own list, the lists at (+-jump, 0) and (0, +-jump) that lie inside the
 * image, and n_inject injected IDs; draw j is ID floor(hi32 * n_slots / 2^32) of
 * SplitMix64 output number (pass_index * H*W + p) * n_inject + j of the stream seeded by
 * `seed`.  Empty, out-of-range and invalid IDs are dropped, repeated IDs collapse, and
 * the top K by (score descending, ID ascending) are written.  jump >= 1,
 * 0 <= n_inject <= 16. */
sad_status sad_propagate_topk(const sad_image *img, const float *rec, const uint32_t *topk_in,
                              uint32_t *topk_out, int32_t jump, int32_t n_inject, uint64_t seed,
                              uint64_t pass_index, void *stream);

/* Jump step of refresh t (Sec. 4.3): B = 2^ceil(log2 max(H,W)),
 * s_t = max(1, B / 2^(min(t, log2 B - 1) + 1)).  Host function. */
int32_t sad_jump_step(int64_t t, int32_t H, int32_t W);

/* ---- a4: forward blend (Sec. 4.2) -------------------------------------------------
 * out[ch][i][j] = sum_k w_k c_k over the valid entries of the pixel's list, w = softmax
 * of the scores with the maximum subtracted (App. B.4); an empty list gives 0.
 * out: float[3][H][W] (written). */
sad_status sad_render_fwd(const sad_image *img, const float *rec, const uint32_t *topk,
                          float *out, void *stream);

/* ---- a5: loss gradient (Sec. 6.1) -------------------------------------------------
 * L = (1/P) sum_x ||c(x) - I(x)||^2 with P = H*W; grad = dL/dc = (2/P)(c - I).
 * img, target: float[3][H][W]; grad: float[3][H][W] (written, may alias img);
 * loss: nullable device accumulator, L is added to loss->value. */
sad_status sad_loss_grad(const sad_image *img, const float *rendered, const float *target,
                         float *grad, sad_loss_acc *loss, void *stream);

/* ---- a4 + a5 fused: forward blend and loss gradient in one pass ------------------
 * As sad_render_fwd followed by sad_loss_grad, without storing the image unless
 * rendered != NULL: grad_img = (2/P)(c - I); L is added to loss->value if loss != NULL.
 * target, grad_img (written), rendered (nullable, written): float[3][H][W]. */
sad_status sad_render_fwd_loss(const sad_image *img, const float *rec, const uint32_t *topk,
                               const float *target, float *rendered, float *grad_img,
                               sad_loss_acc *loss, void *stream);

/* ---- a6: backward scatter (App. B.4; Sec. 4.8 tiled pre-reduction) ---------------
 * Recomputes the blend weights from rec and topk (nothing is stored by the forward)
 * and ACCUMULATES (+=) dL/dsite into grad_sites[10][cap] (caller zeroes) for
 * dL/dc = grad_img [3][H][W]:
 *   dc_k += w_k g;  gamma_k = w_k g.(c_k - c);  dlog_tau_k += gamma_k l_k;
 *   dr_k += gamma_k kappa_k;  with rho = -gamma kappa / (2 n) (0 when n = 0),
 *   alpha = u.d, beta = v.d, d = x - p:  dp += -2 rho (e^a alpha u + e^-a beta v),
 *   da += rho (e^a alpha^2 - e^-a beta^2), du_x += 2 rho (e^a alpha d_x + e^-a beta d_y),
 *   du_y += 2 rho (e^a alpha d_y - e^-a beta d_x).
 * If removal_delta != NULL (target then required) it also accumulates the removal
 * delta of Sec. 4.5, (||c'_k - I||^2 - ||c - I||^2) / P with c'_k the blend without
 * entry k, into removal_delta[cap].  Partial sums of a 16x16 pixel tile are combined in
 * LDS in 64-bit fixed point (terms scaled by 2^40 * 2^(ceil(log2 P) - 1), i.e. exact
 * integer adds with a resolution of 2^-40 of a term of size 1/P; a term too large for
 * that range goes to a float atomic instead) and each tile flushes one float atomic per
 * (site, parameter), so the order of the float additions across tiles -- and the last
 * bits of the result -- vary from run to run. */
sad_status sad_render_bwd(const sad_image *img, const float *rec, const uint32_t *topk,
                          const float *grad_img, const float *target, float *grad_sites,
                          float *removal_delta, void *stream);

/* Exact top-K by brute force over sites 0..n_slots-1 (the ground truth Sec. 6.5
 * compares propagated lists with): for each pixel index pix[q] (i*W + j), the K best
 * sites at (j, i) in list order (score descending, ID ascending), padded with
 * SAD_INVALID_ID; an index outside [0, H*W) gives an all-invalid row.  pix: DEVICE
 * int64[n_pix]; out: uint32[n_pix][K] (one row per pixel).  One block per pixel, so
 * meant for samples (cost n_pix * n_slots scores). */
sad_status sad_exact_topk(const sad_image *img, const float *rec, const int64_t *pix,
                          int64_t n_pix, uint32_t *out, void *stream);

/* ---- a8: Adam step (Sec. 5; clamps of Sec. 6.1) ----------------------------------
 * For every active slot: bias-corrected Adam on the ten parameters with gradient
 * grad[10][cap], moments m, v [10][cap] (updated), step >= 1; then clamp x to
 * [0, W-1], y to [0, H-1], log_tau to [2, 20], r to [1, 512], a to [-2, 2], colours to
 * [0, 1] and renormalise u (u = (1, 0) if |u| = 0).  Inactive slots are untouched.  If
 * rec != NULL the derived records of the updated sites are rewritten as by
 * sad_prepare_sites.  With flags & SAD_ADAM_ZERO_GRAD the gradient is cleared after it
 * has been read (the next backward accumulates into zeros); with flags &
 * SAD_ADAM_GRAD_SITE_MAJOR the gradient is the training step's site-major [cap][10]
 * accumulator instead of [10][cap]; with flags & SAD_ADAM_GRAD_FIXED its elements are
 * int64 fixed point (the deterministic accumulator of a training step run with
 * SAD_TRAIN_DETERMINISTIC, 8 bytes per element) instead of float.  params: host. */
#define SAD_ADAM_ZERO_GRAD 1u
#define SAD_ADAM_GRAD_SITE_MAJOR 2u
#define SAD_ADAM_GRAD_FIXED 4u
sad_status sad_adam_step(const sad_image *img, float *sites, float *grad, float *m, float *v,
                         const sad_adam_params *params, int64_t step, float *rec, uint32_t flags,
                         void *stream);

/* ---- a9: random access (Sec. 6.6: render from cached lists) -----------------------
 * For each query point xy[q] = (x, y) (float32, pixel units, x = column): the list of
 * the nearest pixel (rint, clamped to the image) blended with scores evaluated at the
 * exact point.  xy: float[M][2]; out: float[M][3] (written). */
sad_status sad_query_points(const sad_image *img, const float *rec, const uint32_t *topk,
                            const float *xy, int64_t M, float *out, void *stream);

/* Point queries of many requests against many resident site sets in one launch (the
 * serving path).  Job j answers M_j points of one set: the same computation as
 * sad_query_points, so a result does not depend on the other jobs of the launch.
 * All sets of one call share K.  jobs: DEVICE array [n_jobs] with q0 (the first
 * global point index of the job) increasing; total = sum of M_j. */
typedef struct {
    const float *rec;       /* derived records of the set */
    const uint32_t *topk;   /* its list field */
    const float *xy;        /* [M][2] query points */
    float *out;             /* [M][3] colours */
    int64_t M;
    int64_t q0;
    int32_t H, W, n_slots;
    int32_t pad;
} sad_query_job;

sad_status sad_query_batch(const sad_query_job *jobs, int32_t n_jobs, int64_t total, int32_t K,
                           void *stream);

/* ---- initialisation (Sec. 4.4) ----------------------------------------------------
 * P_init(x) = (1 - lambda) |grad I(x)| / sum |grad I| + lambda / (H W), |grad I| the
 * Frobenius norm over RGB of edge-clamped central differences.  Draws n_sites distinct
 * pixels by Efraimidis-Spirakis keys log(u_p) / P_init(p) (u_p from SplitMix64 output p
 * of `seed`, mapped to (0,1) as (hi32 + 0.5) / 2^32; the n_sites largest keys win, ties
 * to the lower pixel) and writes them in raster order at the pixel centres, with the
 * target colour there, log_tau = log_tau0, r = r0, u = (1, 0), a = 0.  Slots
 * n_sites..cap-1 are made inactive.  Requires n_sites <= min(H*W, cap) and
 * img->n_slots == cap is not required.  target: float[3][H][W]; sites: [10][cap]
 * (written).  workspace: device scratch of *workspace_bytes; call with workspace =
 * NULL to query the size. */
sad_status sad_init_sites(const sad_image *img, const float *target, int32_t n_sites,
                          float lambda, uint64_t seed, float log_tau0, float r0, float *sites,
                          void *workspace, size_t *workspace_bytes, void *stream);

/* ---- a8: one training iteration with device-resident counters ----------------------
 * Counters live in device memory so that a recorded HIP graph replays correctly: every
 * replay reads and advances them on the device. */
typedef struct {
    int64_t pass;      /* refresh counter t: jump s_t (Sec. 4.3) and injection stream */
    int64_t adam_step; /* Adam steps taken so far */
    sad_loss_acc loss; /* loss.value = L of the last step */
    uint64_t done;     /* blocks of the step's last kernel that have finished (the last
                          one folds the loss and advances the counters, then resets it) */
} sad_step_state;

typedef struct {
    int32_t n_inject;   /* J injected IDs per pixel and pass (Sec. 6.1: 4) */
    int32_t fixed_jump; /* <= 0: the Sec. 4.3 schedule of the pass index; > 0: this jump */
    uint64_t seed;      /* injection stream */
    sad_adam_params adam;
    /* Candidate update period f_cand (App. B.3 Tab. impl_params, Sec. 6.1): iteration
     * state->pass propagates only when state->pass % prop_every == 0, as pass number
     * state->pass / prop_every of the schedule and of the injection stream; the other
     * iterations re-score and sort each pixel's own list (a pass with no neighbours and
     * no injections).  0 or 1: propagate every iteration. */
    int32_t prop_every;
    /* SAD_TRAIN_DETERMINISTIC: bit-reproducible gradient sums.  grad_sites then holds
     * int64 fixed point, int64_t[cap][10] (80 bytes per site, zero on entry): every
     * gradient term is rounded once into units of 2^-(20 + e), 2^e the power of two
     * just below P = H*W (2^e >= P/2), and only integers are added after that (per
     * 16x16 tile in LDS, then into grad_sites), so the sums do not depend on the order
     * in which threads and tiles run.  Without it each tile's exact fixed-point sum is
     * converted to float and added with a float atomic, in whatever order tiles finish. */
    uint32_t flags;
} sad_train_config;
#define SAD_TRAIN_DETERMINISTIC 1u
/* SAD_TRAIN_LOSS_SET (sad_train_image_pass): store L in state->loss.value instead of
 * adding it (no separate clear of the value before the pass).  sad_train_step always
 * stores L; the batched step does not take this flag. */
#define SAD_TRAIN_LOSS_SET 2u

/* One iteration (Sec. 5: no host work inside the loop), enqueued as:
 *   1. propagation pass topk_in -> topk_out with pass index state->pass;
 *   2. the forward blend of topk_out and the loss gradient dL/dc, written to grad_img
 *      [3][H][W] if grad_img != NULL, the image to rendered [3][H][W] if rendered !=
 *      NULL, L to state->loss.value;
 *   3. the backward scatter into grad_sites, which must be zero on entry.  This
 *      accumulator is SITE-MAJOR, float[cap][10] (the ten parameters of site i at
 *      10*i .. 10*i+9), unlike the [10][cap] of sad_render_bwd: each tile adds the
 *      ten sums of a site into one cache line;
 *   (1-3 are one kernel: the new keys of a pixel carry the scores its blend needs.)
 *   4. Adam step number state->adam_step + 1 (clamps, renormalised u), rec refreshed,
 *      grad_sites cleared again (ready for the next call);
 *   5. state->pass += 1, state->adam_step += 1.
 * rec must describe `sites` on entry (sad_prepare_sites); after the call topk_out holds
 * the current list field (pass the two list buffers in swapped order next time).
 * cfg: host; state: device (zero it before the first call). */
sad_status sad_train_step(const sad_image *img, const sad_train_config *cfg, const float *target,
                          float *sites, float *rec, const uint32_t *topk_in, uint32_t *topk_out,
                          float *grad_sites, float *adam_m, float *adam_v, float *rendered,
                          float *grad_img, sad_step_state *state, void *stream);

/* Steps 1-3 of sad_train_step alone (rows a3-a6 as one kernel): the propagation pass
 * with pass index state->pass (not advanced), the blend, the loss gradient (L added to
 * state->loss.value, or stored there with SAD_TRAIN_LOSS_SET) and the backward into
 * grad_sites (site-major [cap][10], accumulated, +=).  Same argument meaning as
 * sad_train_step. */
sad_status sad_train_image_pass(const sad_image *img, const sad_train_config *cfg,
                                const float *target, const float *rec, const uint32_t *topk_in,
                                uint32_t *topk_out, float *grad_sites, float *rendered,
                                float *grad_img, sad_step_state *state, void *stream);

/* The training pass's site-major gradient acc [cap][10] in the layout of the sites,
 * grad [10][cap] (written, every slot < cap): grad[q][i] = scale * acc[i][q] with scale =
 * *scale (a DEVICE float, e.g. the incoming gradient of an autograd backward) or 1 when
 * scale is NULL.  With SAD_GRAD_CLEAR_SOURCE, acc is zeroed after it is read (ready for
 * the next pass).  Float accumulators only (not the deterministic int64 form). */
#define SAD_GRAD_CLEAR_SOURCE 1u
sad_status sad_grad_to_params(const sad_image *img, float *grad_site_major, const float *scale,
                              float *grad, uint32_t flags, void *stream);

/* Device-counter forms of sad_propagate_topk and sad_adam_step (Sec. 4.3 schedule,
 * Sec. 5 Adam), for an iteration assembled from the separate calls (e.g. around the
 * autograd wrapper) and recorded once into a HIP graph: the counters live in a
 * sad_step_state on the device, so every replay continues the schedule.
 *
 * sad_propagate_topk_state: one pass with pass index state->pass and the jump
 * s_t = sad_jump_step(state->pass, H, W), both read on the device; state is not
 * modified.  Other arguments as sad_propagate_topk.
 *
 * sad_adam_step_state: sad_adam_step with step = state->adam_step + 1 read on the
 * device; when the update is done the last block folds state->loss.part into
 * state->loss.value and advances state->pass and state->adam_step by one (the end of
 * an iteration, as in sad_train_step; with n_slots = 0 only the counters advance).
 * flags as sad_adam_step.  state: device, zeroed before the first call; calls that
 * share a state must not overlap. */
sad_status sad_propagate_topk_state(const sad_image *img, const float *rec,
                                    const uint32_t *topk_in, uint32_t *topk_out,
                                    int32_t n_inject, uint64_t seed,
                                    const sad_step_state *state, void *stream);
sad_status sad_adam_step_state(const sad_image *img, float *sites, float *grad, float *m,
                               float *v, const sad_adam_params *params, float *rec,
                               uint32_t flags, sad_step_state *state, void *stream);

/* ---- a8: batched training of many images in one persistent launch ----------------
 * Images of uneven size and site budget share pooled buffers.  Image b's blocks start
 * at fixed offsets: pixel pools (target [3][P_b] at 3*px0 floats, each list field
 * [K/4][P_b][4] at K*px0 words, optional rendered / grad_img [3][P_b] at 3*px0 floats)
 * and site pools (sites, m, v [10][cap_b] and the site-major gradient [cap_b][10], each
 * at 10*site0 floats; derived records [cap_b][16] at 16*site0 floats).  All images use
 * the batch's K. */
typedef struct {
    int32_t H, W;
    int32_t n_slots;
    int32_t tile0;      /* first work item (tile of the batch's shape) of this image;
                           items are numbered image by image in raster order of tiles */
    int64_t cap;
    int64_t px0;        /* pixels of the images before this one */
    int64_t site0;      /* site slots (sum of cap) of the images before this one */
    float score_scale;  /* 0 => 1 / max(H, W) */
    int32_t pad;
} sad_batch_image;

typedef struct {
    int32_t n_images;
    int32_t K;
    int32_t n_items;           /* total tiles of all images (tile shape: tile_w) */
    int32_t grid;              /* persistent workgroups; 0 => one per tile */
    int32_t chunked;           /* 0: item i goes to workgroup i mod grid; 1: each
                                  workgroup takes a contiguous run of items (its XCD's
                                  L2 then holds neighbouring tiles) */
    int32_t tile_w;            /* work-item tile: 0 or 16 = 16 x 16 pixels, 32 = 32 x 8
                                  (four 8 x 8 wave64 blocks either way); n_items and each
                                  image's tile0 count tiles of this shape */
    int64_t n_site_slots;      /* sum of cap over the images */
    const sad_batch_image *images;  /* DEVICE array [n_images], tile0 increasing */
} sad_batch;

/* One training iteration of every image of the batch (sad_train_step semantics per
 * image; image b uses states[b]): one persistent image-space kernel over all tiles of
 * all images, then per-image loss folds, one Adam kernel over all site slots and one
 * state update, whatever the number of images.  batch: host struct whose `images`
 * points to device memory; states: device [n_images]; rendered, grad_img nullable.
 * With cfg->flags & SAD_TRAIN_DETERMINISTIC the gradient pool holds int64 elements
 * (image b's rows at element 10*site0, in units of 2^-(20 + e_b) for its own P_b). */
sad_status sad_batch_train_step(const sad_batch *batch, const sad_train_config *cfg,
                                const float *target, float *sites, float *rec,
                                const uint32_t *topk_in, uint32_t *topk_out, float *grad_sites,
                                float *adam_m, float *adam_v, float *rendered, float *grad_img,
                                sad_step_state *states, void *stream);

/* ---- adaptive budget: statistics, prune, split (Sec. 4.5; App. B.5) ---------------
 * Statistics pass.  For every pixel x, blended from its list as in sad_render_fwd, with
 * residual e(x) = ||c(x) - I(x)||^2, and every valid entry i (w = its softmax weight,
 * omega = w e(x), d = x - p_i):
 *   stats[0][i] += w             soft mass m_i
 *   stats[1][i] += omega         energy E_i
 *   stats[2][i] += omega d_x     stats[3][i] += omega d_y
 *   stats[4][i] += omega d_x^2   stats[5][i] += omega d_x d_y   stats[6][i] += omega d_y^2
 *   stats[7][i] += Delta_i(x) / (H W)   removal delta (as sad_render_bwd computes it)
 * i.e. the residual-weighted moments about the site centre.  stats: float[8][cap],
 * accumulated (+=): the caller zeroes it.  target: float[3][H][W].  Sums are formed
 * per 16x16 tile in 64-bit fixed point in LDS and added across tiles with float
 * atomics, so the last bits depend on scheduling. */
#define SAD_NSTAT 8
sad_status sad_site_stats(const sad_image *img, const float *rec, const uint32_t *topk,
                          const float *target, float *stats, void *stream);

/* Order-independent form of sad_site_stats (Sec. 4.5, App. B.5: the same statistics),
 * for deterministic encodes.  Every term is rounded once to its statistic's unit 2^-s
 * (s = 40, 40, 36, 36, 30, 30, 30 for stats[0..6] and 40 + e for stats[7], 2^e the
 * largest power of two below H W), and all sums are integer: per tile in LDS, over
 * tiles exactly in 128 bits.  So the statistics depend only on the inputs, not on
 * scheduling; they differ from sad_site_stats's by the per-term rounding (at most
 * 2^-(s+1) per term).
 * acc: DEVICE int64[2][8][cap] workspace (16 * 8 * cap bytes, 8-byte aligned), cleared
 *   by the call; on return acc[0][q][i] + 2^64 acc[1][q][i] is the sum of
 *   stats[q][i] in units of 2^-s.
 * stats: float[8][cap], WRITTEN (=) for every slot 0..cap-1 (zero where no pixel
 *   lists the slot), not accumulated.
 * Errors: SAD_ERR_INVALID_ARGUMENT for NULL target, acc or stats, NULL or unaligned
 * rec / topk when n_slots > 0, a misaligned acc, or a bad descriptor. */
sad_status sad_site_stats_fixed(const sad_image *img, const float *rec, const uint32_t *topk,
                                const float *target, int64_t *acc, float *stats,
                                void *stream);

/* One budget step on slots 0..cap-1 (img->n_slots is not used; img->K only for
 * seeding).  With n_active the number of active slots:
 *   SAD_DP_PRUNE: the floor(p_prune n_active) active sites with the smallest removal
 *     delta stats[7] (ties to the lower slot) become inactive (x = y = -1).
 *   SAD_DP_SPLIT: candidates are the active, unpruned sites with m = stats[0] >
 *     min_mass; their score E / max(m, eps)^alpha is evaluated in double and rounded
 *     to float (ties to the lower slot); the min(floor(p_split n_active), candidates,
 *     free slots) best are split in two.  Children are offset from the residual-weighted
 *     centroid along the principal axis of the residual-weighted covariance by
 *     0.5 sqrt(m) px (clamped to [1.5, 48]), take u = that axis and a = 0.5 ln(l2/l1)
 *     (clamped to [-2, 2]; -2 if l2 <= 0); without usable statistics (E <= 1e-12, trace
 *     <= 1e-9 or eigenvalue gap <= 1e-6 of the trace) they are offset from p along the
 *     principal axis of the target's Sobel structure tensor at p (else along u), keep u
 *     and take a = 0.8 a.  Both children: positions clamped to the image, log_tau - 0.25
 *     and 0.85 r (clamped as by Adam), colour = target at the nearest pixel.  The "+"
 *     child keeps the parent's slot; parents in ascending slot order give their "-"
 *     child the free slots (inactive after the prune) in ascending order.  Adam moments
 *     of both slots are zeroed (all ten parameters).
 *   SAD_DP_SEED (topk non-NULL): at every pixel holding a "-" child, the child with the
 *     smallest slot replaces list entry K-1, so that propagation starts from it.
 * counts: DEVICE int64[6] = {n_active, pruned, split, n_active after, high water (1 +
 * the largest active slot, 0 if none), split candidates}.  After the call the caller
 * refreshes the derived records (sad_prepare_sites) over n_slots >= high water.
 * stats: float[8][cap] from sad_site_stats.  workspace: device scratch of
 * *workspace_bytes; workspace = NULL queries the size. */
#define SAD_DP_PRUNE 1u
#define SAD_DP_SPLIT 2u
#define SAD_DP_SEED 4u
typedef struct {
    double p_prune;  /* fraction of the active count pruned (Sec. 6.1: 0.033) */
    double p_split;  /* fraction of the active count split (Sec. 6.1: 0.01) */
    double alpha;    /* score exponent (Sec. 6.1: 0.7) */
    double eps;      /* mass floor (Sec. 4.5: 1e-8) */
    double min_mass; /* sites with m <= min_mass are not split (Sec. 4.5: 1) */
    uint32_t flags;
    uint32_t pad;
} sad_budget_params;

sad_status sad_densify_prune(const sad_image *img, const float *target, float *sites,
                             float *adam_m, float *adam_v, const float *stats,
                             const sad_budget_params *params /* host */, uint32_t *topk,
                             int64_t *counts, void *workspace, size_t *workspace_bytes,
                             void *stream);

/* ---- full-refresh regime (Sec. 6.6 "full refresh"; App. B.3) ----------------------
 * A list field may live on a grid of Hg x Wg cells laid over img's H x W image: a
 * downscaled candidate grid (App. B.3 "Downscaled candidate grid", Hg = ceil(H / s_grid))
 * or the pixels of a new output resolution (Sec. 6.6: a new pixel grid needs its lists
 * rebuilt).  Its layout is that of `topk` with Hg*Wg cells in place of the pixels:
 * uint32[K/4][Hg*Wg][4].  Cell (i, j) is evaluated at the centre of its UV square,
 *   x = ((2 j + 1) W - Wg) / (2 Wg),  y = ((2 i + 1) H - Hg) / (2 Hg)
 * (pixel units, each a ratio of exact integers divided in double and rounded once to
 * float; on the image's own grid Hg = H, Wg = W the cell is the pixel), and image point
 * (or pixel) j belongs to cell floor((2 j + 1) Wg / (2 W)) -- the integer mapping of
 * App. B.3 (floor(j / s) when W = s Wg).  Hg, Wg >= 1, Hg*Wg <= 2^30. */

/* Seed pass on a grid (App. B.3 "JFA prepass": the seed pass): every entry cleared to
 * SAD_INVALID_ID, then each valid site goes to the cell of its nearest pixel
 * (rint(y), rint(x)) clamped to the image, and a cell keeps its best n_entries sites
 * (0 <= n_entries <= K) by (score at the cell's point descending, ID ascending).  With
 * Hg = H, Wg = W, n_entries = K it is sad_seed_topk.  topk: [K/4][Hg*Wg][4] (written);
 * scratch: uint64[Hg*Wg] (contents undefined after). */
sad_status sad_seed_grid(const sad_image *img, int32_t Hg, int32_t Wg, int32_t n_entries,
                         const float *rec, uint32_t *topk, uint64_t *scratch, void *stream);

/* One propagation pass on a grid: sad_propagate_topk with cells in place of pixels --
 * neighbours at +-jump cells, candidates scored at the cell's point, injection draws of
 * pass t numbered (t * Hg*Wg + cell) * n_inject + j.  With Hg = H, Wg = W it is
 * sad_propagate_topk. */
sad_status sad_propagate_grid(const sad_image *img, int32_t Hg, int32_t Wg, const float *rec,
                              const uint32_t *topk_in, uint32_t *topk_out, int32_t jump,
                              int32_t n_inject, uint64_t seed, uint64_t pass_index,
                              void *stream);

/* One JFA flood pass (App. B.3 "JFA prepass"), Jacobi: each cell gathers the first four
 * entries (plane 0 of the field, "the first candidate texture") of the cells at
 * (di step, dj step), di, dj in {-1, 0, 1}, that lie in the grid (itself included),
 * drops empty, out-of-range and invalid IDs and repeats, scores the rest exactly at its
 * point and writes the best four by (score descending, ID ascending) into plane 0 of
 * topk_out.  Planes 1.. of topk_out are not written.  step >= 1. */
sad_status sad_jfa_flood(const sad_image *img, int32_t Hg, int32_t Wg, const float *rec,
                         const uint32_t *topk_in, uint32_t *topk_out, int32_t step,
                         void *stream);

/* Steps of the JFA prepass on an Hg x Wg grid (App. B.3: ceil(log2 max(W, H)) flood
 * passes): L = ceil(log2 max(Hg, Wg)) steps 2^(L-1), ..., 2, 1 written to steps[]
 * (host, room for 31); returns L, or -1 for a bad argument.  Host function. */
int32_t sad_jfa_steps(int32_t Hg, int32_t Wg, int32_t *steps);

/* A full refresh of a list field on a grid (Sec. 6.6; App. B.3): with SAD_REFRESH_JFA the
 * JFA prepass (seed pass keeping four entries per cell, then the flood passes of
 * sad_jfa_steps, so entries 4..K-1 start empty), otherwise the seed pass keeping K
 * entries; then n_pass propagation passes t = 0 .. n_pass - 1 with the Sec. 4.3
 * schedule of the grid (jump sad_jump_step(t, Hg, Wg), injection stream t).  The result
 * is in topk; topk_tmp (the same size, not aliasing topk) is ping-pong space, scratch
 * uint64[Hg*Wg]; the contents of both are undefined after.  The paper's render call is
 * SAD_REFRESH_JFA with 16 passes followed by a render. */
#define SAD_REFRESH_JFA 1u
sad_status sad_refresh(const sad_image *img, int32_t Hg, int32_t Wg, uint32_t flags,
                       int32_t n_pass, int32_t n_inject, uint64_t seed, const float *rec,
                       uint32_t *topk, uint32_t *topk_tmp, uint64_t *scratch, void *stream);

/* Render at an output grid of Ho x Wo points over the image from a list field of
 * Hg x Wg cells (Sec. 4.2 blend; Sec. 6.6 re-render at a different resolution):
 * output point (io, jo) is the centre of its cell of the output grid, takes the list of
 * the list-grid cell holding that centre (the integer mapping above) and is blended as
 * by sad_render_fwd at its own coordinates.  Ho = Hg, Wo = Wg renders a grid's own
 * lists; Ho = H, Wo = W renders the image from a downscaled candidate grid; all four
 * equal to the image is sad_render_fwd.  out: float[3][Ho][Wo] (written). */
sad_status sad_render_grid(const sad_image *img, int32_t Hg, int32_t Wg, const float *rec,
                           const uint32_t *topk, int32_t Ho, int32_t Wo, float *out,
                           void *stream);

/* ---- packed 16-byte inference record (App. B.2 "Packed storage for evaluation") ----
 * Four 32-bit words per site slot (uint32[n_slots][4]):
 *   w0 = x code | y code << 15 | 1 << 31: positions as 15-bit UNORM over [0, W-1] and
 *        [0, H-1], bit 31 the active flag (bit 30 zero)
 *   w1 = c_r | c_g << 11 | c_b << 22: colours as 11 / 11 / 10-bit UNORM over their
 *        per-image [min, min + scale]
 *   w2 = log_tau | r << 16: 16-bit UNORM each over their per-image [min, min + scale]
 *   w3 = angle code | float16 bits of a << 16: the direction u as a 16-bit UNORM of
 *        atan2(u_y, u_x) over [-pi, pi] (double precision)
 * An inactive slot packs to four zero words.  A UNORM code with b bits is
 * rint(t (2^b - 1)) with t = (v - min) / scale clamped to [0, 1] (0 when scale = 0),
 * each step one float32 operation; it decodes to min + scale (code / (2^b - 1)).  The
 * direction decodes to (f32(cos th), f32(sin th)) with th = code / 65535 * 2 pi - pi in
 * double, a to the float16 value; a record without the active flag decodes to an
 * inactive site (x = y = -1, the rest 0).  At 16 bytes per site the size in bits per
 * pixel is n 128 / (H W) (Sec. 6.1).
 * Quantisation parameters q: float[SAD_NQPARAM] = {log_tau min, scale, r min, scale,
 * c_r min, scale, c_g min, scale, c_b min, scale}, min and max over the active slots
 * < n_slots and scale = max - min (all zero without an active site). */
#define SAD_NQPARAM 10

/* q (written) from sites [10][cap] over slots < n_slots.  q is also the reduction's
 * working memory (no other scratch). */
sad_status sad_pack_qparams(const sad_image *img, const float *sites, float *q, void *stream);

/* packed [n_slots][4] (written) from sites [10][cap] with quantisation parameters q
 * (device, e.g. from sad_pack_qparams).  Requires H, W <= 32768. */
sad_status sad_pack_sites(const sad_image *img, const float *sites, const float *q,
                          uint32_t *packed, void *stream);

/* Decode packed [n_slots][4] into sites [10][cap] (slots < n_slots written). */
sad_status sad_unpack_sites(const sad_image *img, const uint32_t *packed, const float *q,
                            float *sites, void *stream);

/* Decode packed [n_slots][4] straight into derived records rec [n_slots][16] (the records
 * sad_prepare_sites would write for the decoded sites), for the image-space calls. */
sad_status sad_prepare_packed(const sad_image *img, const uint32_t *packed, const float *q,
                              float *rec, void *stream);

/* sad_render_fwd and sad_query_points reading the packed records: each list entry's
 * record is decoded in place (16 bytes gathered per entry instead of the derived
 * record's 48), with the same result as the same call on sad_prepare_packed's records. */
sad_status sad_render_packed(const sad_image *img, const uint32_t *packed, const float *q,
                             const uint32_t *topk, float *out, void *stream);
sad_status sad_query_packed(const sad_image *img, const uint32_t *packed, const float *q,
                            const uint32_t *topk, const float *xy, int64_t M, float *out,
                            void *stream);

/* ---- tau diffusion (App. B.6) ---------------------------------------------------------
 * One Jacobi step of the optional smoothing of the log tau gradient: for every slot
 * i < n_slots whose record is valid, with N(i) the valid entries other than i of the list
 * at the pixel nearest its centre ((rint(y), rint(x)) clamped),
 *   g_out[i] = (1 - lambda) g_in[i] + lambda mean_{j in N(i)} g_in[j],
 * and g_out[i] = g_in[i] when N(i) is empty or the record is invalid.  Element i of a
 * gradient array is at g[i * stride]: stride 1 for the log tau row of a [10][cap]
 * gradient (g = grad + 2 cap), stride 10 for the training step's site-major [cap][10]
 * accumulator (g = grad + 2).  g_in and g_out must not alias; 0 <= lambda <= 1. */
sad_status sad_tau_diffusion(const sad_image *img, const float *rec, const uint32_t *topk,
                             const float *g_in, int64_t in_stride, float lambda, float *g_out,
                             int64_t out_stride, void *stream);

/* ---- one-dimensional SAD (Sec. 7 "1D Signal Fitting") -----------------------------------
 * A signal of M samples, sample m at x = m.  Sites have four parameters, float[4][cap] in
 * the order (p, c, log_tau, r); the score is the 2-D one on a line,
 *   l_i(x) = tau_i s (r_i - |x - p_i|),   s = score_scale (0 selects 1/M),
 * evaluated in float32 as d = x - p, n = |d|, l = kappa (r - n) + 0 with
 * kappa = f32(exp(double log_tau)) * s.  A site is active iff p >= 0, all four values are
 * finite and kappa is finite and > 0.  Lists: uint32[K/4][M][4] as the 2-D field, sorted
 * by (score descending, ID ascending).  Derived records rec1: float4[n_slots] =
 * {p, r, kappa, c}, kappa = 0 for an inactive site. */
typedef struct {
    int32_t M;
    int32_t K;
    int32_t n_slots;
    int32_t pad;
    int64_t cap;
    float score_scale;
} sad_signal;

/* rec1 [n_slots] (written) from sites [4][cap]. */
sad_status sad1d_prepare(const sad_signal *sg, const float *sites, float *rec1, void *stream);
/* Seed pass: every entry cleared, then each active site goes to sample rint(p) (clamped)
 * and a sample keeps the top K of its sites.  scratch: uint64[M]. */
sad_status sad1d_seed(const sad_signal *sg, const float *rec1, uint32_t *topk,
                      uint64_t *scratch, void *stream);
/* One Jacobi propagation pass on the line: own list, the lists at m +- jump inside
 * [0, M), n_inject IDs (draw j: SplitMix64 output (pass_index M + m) n_inject + j of the
 * stream `seed`, ID = floor(hi32 n_slots / 2^32)); the top K distinct valid IDs. */
sad_status sad1d_propagate(const sad_signal *sg, const float *rec1, const uint32_t *topk_in,
                           uint32_t *topk_out, int32_t jump, int32_t n_inject, uint64_t seed,
                           uint64_t pass_index, void *stream);
/* Blend of every sample (max-subtracted softmax of its valid entries; an empty list gives
 * 0) into out[M] (nullable).  With target[M]: L = (1/M) sum (c - I)^2 is added to
 * loss->value (nullable), and if grad != NULL the gradients for dL/dc = (2/M)(c - I) are
 * accumulated (+=, float atomics) into grad[4][cap]: dc += w g, gamma = w g (c_k - c),
 * dlog_tau += gamma l, dr += gamma kappa, dp += gamma kappa sign(x - p) (0 at x = p). */
sad_status sad1d_render(const sad_signal *sg, const float *rec1, const uint32_t *topk,
                        const float *target, float *out, float *grad, sad_loss_acc *loss,
                        void *stream);
/* Adam (bias-corrected, step >= 1) on the four parameters with learning rates lr (host
 * [4]), then p clamped to [0, M-1], log_tau to [2, 20], r to [1, 512]; inactive slots
 * untouched.  sites, m, v: [4][cap] (updated); grad: [4][cap]. */
sad_status sad1d_adam(const sad_signal *sg, float *sites, const float *grad, float *m, float *v,
                      const float *lr, float beta1, float beta2, float eps, int64_t step,
                      void *stream);

/* ---- diagnostics ------------------------------------------------------------------ */
const char *sad_status_string(sad_status s);
const char *sad_last_error(void);
/* Library version string (host). */
const char *sad_version(void);

#ifdef __cplusplus
}
#endif
#endif /* SAD_H */
