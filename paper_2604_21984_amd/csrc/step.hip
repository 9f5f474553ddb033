// step.hip -- one training iteration with device-resident counters (graph-replayable).
#include "sad_device.h"
#include "sad_host.h"
#include "sad_internal.h"

namespace sad {

__global__ void k_state_advance(sad_step_state *__restrict__ s) {
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        s->pass += 1;
        s->adam_step += 1;
    }
}

}  // namespace sad

using namespace sad;

extern "C" sad_status sad_train_step(const sad_image *img, const sad_train_config *cfg,
                                     const float *target, float *sites, float *rec,
                                     const uint32_t *topk_in, uint32_t *topk_out, float *grad_sites,
                                     float *adam_m, float *adam_v, float *rendered, float *grad_img,
                                     sad_step_state *state, void *stream) {
    float s;
    SAD_TRY(check_image(img, &s));
    SAD_REQUIRE(cfg && state, SAD_ERR_INVALID_ARGUMENT, "sad_train_step: cfg / state is NULL");
    SAD_REQUIRE(target && sites && rec && topk_in && topk_out && grad_sites && adam_m && adam_v &&
                    grad_img,
                SAD_ERR_INVALID_ARGUMENT, "sad_train_step: NULL pointer");
    SAD_REQUIRE(topk_in != topk_out, SAD_ERR_INVALID_ARGUMENT,
                "sad_train_step: topk_in and topk_out must not alias");
    SAD_REQUIRE(aligned16(rec) && aligned16(topk_in) && aligned16(topk_out),
                SAD_ERR_INVALID_ARGUMENT, "sad_train_step: rec / lists not 16-byte aligned");
    SAD_REQUIRE(cfg->n_inject >= 0 && cfg->n_inject <= 16, SAD_ERR_INVALID_ARGUMENT,
                "sad_train_step: n_inject must be in [0, 16]");
    hipStream_t st = as_stream(stream);
    launch_propagate(img, rec, topk_in, topk_out, cfg->fixed_jump > 0 ? cfg->fixed_jump : 0,
                     cfg->n_inject, cfg->seed, 0, &state->pass, st);
    launch_fwd_loss(img, rec, topk_out, target, rendered, grad_img, &state->loss, true, st);
    launch_bwd(img, rec, topk_out, grad_img, nullptr, grad_sites, nullptr, st);
    launch_adam(img, s, sites, grad_sites, adam_m, adam_v, &cfg->adam, 1, &state->adam_step, rec,
                true, st);
    hipLaunchKernelGGL(k_state_advance, dim3(1), dim3(64), 0, st, state);
    return check_launch("sad_train_step");
}
