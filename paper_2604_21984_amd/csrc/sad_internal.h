// sad_internal.h -- launchers shared between translation units (no validation here:
// callers have checked their arguments).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "sad.h"

namespace sad {

// One propagation pass.  If pass_dev != NULL the pass index is *pass_dev (device) and,
// when jump <= 0, the jump is the schedule step of that index; otherwise pass / jump.
void launch_propagate(const sad_image *img, const float *rec, const uint32_t *in, uint32_t *out,
                      int32_t jump, int32_t n_inject, uint64_t seed, uint64_t pass,
                      const int64_t *pass_dev, hipStream_t st);
// Seed pass (App. B.3) on a grid of Hg x Wg cells over img's H x W image: every entry
// of topk [K/4][Hg*Wg][4] cleared, then each cell keeps its best n_entries sites (the
// sites whose nearest pixel lies in it), scored at the cell's point.  scratch:
// uint64[Hg*Wg].
struct SeedGrid {
    int H, W, Hg, Wg;
};
void launch_seed(const sad_image *img, int32_t Hg, int32_t Wg, int32_t n_entries,
                 const float *rec, uint32_t *topk, uint64_t *scratch, hipStream_t st);
// The same pass on a list field of Hg x Wg cells over img's image, each cell scored at
// its centre (App. B.3); Hg = H, Wg = W is launch_propagate.
void launch_propagate_grid(const sad_image *img, int32_t Hg, int32_t Wg, const float *rec,
                           const uint32_t *in, uint32_t *out, int32_t jump, int32_t n_inject,
                           uint64_t seed, uint64_t pass, const int64_t *pass_dev, hipStream_t st);
void launch_fwd(const sad_image *img, const float *rec, const uint32_t *topk, float *out,
                hipStream_t st);
void launch_loss_grad(const sad_image *img, const float *rendered, const float *target,
                      float *grad, sad_loss_acc *loss, bool overwrite, hipStream_t st);
// Fold loss->part into loss->value (added, or written if overwrite) and clear part[].
void launch_loss_fold(sad_loss_acc *loss, bool overwrite, hipStream_t st);
// Forward blend fused with the loss gradient; rendered may be NULL.
void launch_fwd_loss(const sad_image *img, const float *rec, const uint32_t *topk,
                     const float *target, float *rendered, float *grad_img, sad_loss_acc *loss,
                     bool overwrite, hipStream_t st);
void launch_bwd(const sad_image *img, const float *rec, const uint32_t *topk, const float *grad_img,
                const float *target, float *grad_sites, float *removal_delta, hipStream_t st);
// Adam; if step_dev != NULL the step is *step_dev + 1 (device), else `step`.  If
// zero_grad, the gradient is cleared after it has been read (ready for the next step).
// The gradient is [10][cap], or [cap][10] with grad_site_major (the training step's).
// If fin != NULL the last block also folds fin's loss partials and advances its
// counters (the end of a training iteration).  Nothing is launched if n_slots == 0.
// With grad_fixed the gradient elements are int64 in units of det_grad_unit(H * W) (the
// deterministic accumulator of the training step).
void launch_adam(const sad_image *img, float s, float *sites, float *grad, float *m, float *v,
                 const sad_adam_params *p, int64_t step, const int64_t *step_dev, float *rec,
                 bool zero_grad, bool grad_site_major, sad_step_state *fin, hipStream_t st,
                 bool grad_fixed = false);
void launch_fill_f32(float *p, int64_t n, float v, hipStream_t st);
// state->pass += 1 and state->adam_step += 1 (one thread).
void launch_state_advance(sad_step_state *state, hipStream_t st);

// Radix select over unsigned 64-bit codes (8 passes of 8 bits, most significant
// first).  On entry st->prefix = st->mask = 0 and st->want = the rank wanted (1 = the
// largest), all on the device; on exit st->prefix is the want-th largest code T and
// st->want the number of codes equal to T still to take.  hist: 256 zeroed counters,
// left zeroed.
struct SelState {
    uint64_t prefix;
    uint64_t mask;
    uint32_t want;
    uint32_t pad;
};
void launch_radix_select(const uint64_t *code, int64_t n, SelState *st, uint32_t *hist,
                         hipStream_t s);
// Exclusive prefix sum of n uint32 flags, in place; btot: scan_blocks(n) counters.
int64_t scan_blocks(int64_t n);
void launch_excl_scan(uint32_t *f, int64_t n, uint32_t *btot, hipStream_t s);

// Device-side jump schedule (Sec. 4.3), same formula as sad_jump_step.
__host__ __device__ inline int32_t jump_of(int64_t t, int32_t H, int32_t W) {
    const int m = H > W ? H : W;
    int lb = 0;
    while ((1LL << lb) < m) ++lb;
    const int64_t B = 1LL << lb;
    int64_t e = t < (int64_t)(lb - 1) ? t : (int64_t)(lb - 1);
    if (e < 0) e = 0;
    const int64_t s = B >> (e + 1);
    return (int32_t)(s > 1 ? s : 1);
}

}  // namespace sad
