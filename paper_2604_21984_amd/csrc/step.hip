// step.hip -- one training iteration with device-resident counters (graph-replayable).
//
// The image-space work of an iteration is one kernel: per pixel, the propagation pass
// produces the new sorted keys; their exact scores are the logits of the blend, so the
// forward, the loss gradient and the backward contributions follow in registers without
// reading the list or the gradient image back; the tile's contributions meet in the
// fixed-point LDS table and are flushed once per (site, parameter).  Adam follows as a
// per-site kernel (it needs every tile's contribution).
#include "sad_device.h"
#include "sad_host.h"
#include "sad_internal.h"
#include "sad_kernels.h"

namespace sad {

template <int K, bool kDet>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(K == 16 ? 4 : 1, 8))) void k_train(PropArgs pa, ImgArgs a, FixScale fx,
                                               const float4 *__restrict__ rec,
                                               const uint4 *__restrict__ lin,
                                               uint4 *__restrict__ lout,
                                               const float *__restrict__ tgt,
                                               float *__restrict__ rendered,
                                               float *__restrict__ gimg,
                                               sad_loss_acc *__restrict__ loss,
                                               float *__restrict__ grad) {
    // The propagation's candidate queue and the backward's accumulators are used in
    // turn, so they share one LDS buffer (ten 64-bit channels: no removal delta here).
    constexpr int kQ = QueueDepth<K>::v;
    constexpr int kWords = (kQ > 20 ? kQ : 20) * 256;
    static_assert(kWords >= 10 * 2 * kHashSlots, "accumulators must fit");
    __shared__ __align__(16) uint32_t lds[kWords];
    __shared__ uint32_t hkey[kHashSlots];
    __shared__ uint32_t occ[kHashSlots + 1];
    uint32_t(*queue)[256] = reinterpret_cast<uint32_t(*)[256]>(lds);
    unsigned long long(*hacc)[kHashSlots] = reinterpret_cast<unsigned long long(*)[kHashSlots]>(lds);
    const int tile = xcd_tile(blockIdx.x, a.n_blocks);
    const TilePix px = tile_pixel(tile, a.tiles_x);
    const bool in = px.i < a.H && px.j < a.W;
    const int64_t P = (int64_t)a.H * a.W, p = (int64_t)px.i * a.W + px.j;
    uint64_t keys[K];
    if (in) {
        prop_pixel<K>(pa, rec, lin, px, queue, keys);
#pragma unroll
        for (int g = 0; g < K / 4; ++g)
            lout[(int64_t)g * P + p] = make_uint4(key_id(keys[4 * g]), key_id(keys[4 * g + 1]),
                                                  key_id(keys[4 * g + 2]), key_id(keys[4 * g + 3]));
    }
    __syncthreads();  // the queue is free: clear the accumulators in its place
    bwd_tile_init<10>(hkey, hacc);
    __syncthreads();
    float sq = 0.f;
    if (in) {
        const float X = (float)px.j, Y = (float)px.i;
        PixelBlend<K> b;
        blend_keys<K, true>(rec, keys, b, lane_rot() % K);
        float g[3];
#pragma unroll
        for (int ch = 0; ch < 3; ++ch) {
            const float d = b.c[ch] - tgt[ch * P + p];
            g[ch] = 2.0f * a.inv_P * d;
            sq = fmaf(d, d, sq);
            if (gimg) gimg[ch * P + p] = g[ch];
            if (rendered) rendered[ch * P + p] = b.c[ch];
        }
        bwd_pixel<K, false, true, kDet>(rec, b, X, Y, g[0], g[1], g[2], 0.f, 0.f, 0.f, hkey,
                                        hacc, fx, a.inv_P, a.cap, grad, nullptr);
    }
    const float tot = block_sum(sq);  // contains the barrier the flush needs
    if (threadIdx.x == 0) atomic_add_f32(&loss->part[blockIdx.x % SAD_LOSS_PARTS], tot * a.inv_P);
    bwd_flush<false, true, kDet>(hkey, hacc, fx, a.cap, grad, nullptr, occ);
}

// grad[q][i] = scale * acc[i][q] for every slot i < cap (scale = *scale_dev, or 1), and
// with clear the source row is zeroed after it has been read.
__global__ __launch_bounds__(256) void k_grad_to_params(float *__restrict__ acc,
                                                        const float *__restrict__ scale_dev,
                                                        float *__restrict__ grad, int64_t cap,
                                                        int clear) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= cap) return;
    const float sc = scale_dev ? *scale_dev : 1.0f;
    float v[SAD_NPARAM];
#pragma unroll
    for (int q = 0; q < SAD_NPARAM; ++q) v[q] = acc[i * SAD_NPARAM + q];
#pragma unroll
    for (int q = 0; q < SAD_NPARAM; ++q) grad[q * cap + i] = sc * v[q];
    if (clear) {
#pragma unroll
        for (int q = 0; q < SAD_NPARAM; ++q) acc[i * SAD_NPARAM + q] = 0.0f;
    }
}

__global__ void k_state_advance(sad_step_state *__restrict__ s) {
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        s->pass += 1;
        s->adam_step += 1;
    }
}

}  // namespace sad

using namespace sad;

void sad::launch_state_advance(sad_step_state *state, hipStream_t st) {
    hipLaunchKernelGGL(k_state_advance, dim3(1), dim3(64), 0, st, state);
}

static sad_status image_pass(const sad_image *img, const sad_train_config *cfg,
                             const float *target, const float *rec, const uint32_t *topk_in,
                             uint32_t *topk_out, float *grad_sites, float *rendered,
                             float *grad_img, sad_step_state *state, bool overwrite_loss,
                             bool fold, hipStream_t st) {
    SAD_TRY(check_image(img, nullptr));
    SAD_REQUIRE(cfg && state, SAD_ERR_INVALID_ARGUMENT, "training pass: cfg / state is NULL");
    SAD_REQUIRE(target && rec && topk_in && topk_out && grad_sites, SAD_ERR_INVALID_ARGUMENT,
                "training pass: NULL pointer");
    SAD_REQUIRE(topk_in != topk_out, SAD_ERR_INVALID_ARGUMENT,
                "training pass: topk_in and topk_out must not alias");
    SAD_REQUIRE(aligned16(rec) && aligned16(topk_in) && aligned16(topk_out),
                SAD_ERR_INVALID_ARGUMENT, "training pass: rec / lists not 16-byte aligned");
    SAD_REQUIRE(cfg->n_inject >= 0 && cfg->n_inject <= 16, SAD_ERR_INVALID_ARGUMENT,
                "training pass: n_inject must be in [0, 16]");
    SAD_REQUIRE(cfg->prop_every >= 0 && cfg->prop_every <= 1024, SAD_ERR_INVALID_ARGUMENT,
                "training pass: prop_every must be in [0, 1024]");
    SAD_REQUIRE((cfg->flags & ~(SAD_TRAIN_DETERMINISTIC | SAD_TRAIN_LOSS_SET)) == 0,
                SAD_ERR_INVALID_ARGUMENT, "training pass: unknown flags 0x%x", cfg->flags);
    overwrite_loss = overwrite_loss || (cfg->flags & SAD_TRAIN_LOSS_SET) != 0;
    if (img->n_slots == 0) {  // no sites: empty lists, colour 0, nothing to update
        launch_propagate(img, rec, topk_in, topk_out, 1, 0, 0, 0, nullptr, st);
        if (grad_img)
            launch_fwd_loss(img, rec, topk_out, target, rendered, grad_img, &state->loss,
                            overwrite_loss, st);
        else if (rendered)
            launch_fill_f32(rendered, 3ll * img->H * img->W, 0.f, st);
        return check_launch("training pass");
    }
    PropArgs pa;
    pa.H = img->H;
    pa.W = img->W;
    pa.n_slots = img->n_slots;
    pa.jump = cfg->fixed_jump > 0 ? cfg->fixed_jump : 0;
    pa.J = cfg->n_inject;
    pa.every = cfg->prop_every;
    pa.tiles_x = tiles_x(img);
    pa.n_blocks = n_tiles(img);
    pa.seed = cfg->seed;
    pa.pass = 0;
    pa.pass_dev = &state->pass;
    ImgArgs a;
    a.H = img->H;
    a.W = img->W;
    a.n_slots = img->n_slots;
    a.tiles_x = pa.tiles_x;
    a.n_blocks = pa.n_blocks;
    a.cap = img->cap;
    a.inv_P = (float)(1.0 / ((double)img->H * img->W));
    const FixScale fx = fix_scale((int64_t)img->H * img->W);
    const float4 *r4 = reinterpret_cast<const float4 *>(rec);
    const uint4 *li = reinterpret_cast<const uint4 *>(topk_in);
    uint4 *lo = reinterpret_cast<uint4 *>(topk_out);
    const bool det = (cfg->flags & SAD_TRAIN_DETERMINISTIC) != 0;
#define SAD_TRAIN_CASE(KK)                                                                    \
    case KK:                                                                                  \
        if (det)                                                                              \
            hipLaunchKernelGGL((k_train<KK, true>), dim3(a.n_blocks), dim3(256), 0, st, pa, a, fx, \
                               r4, li, lo, target, rendered, grad_img, &state->loss,          \
                               grad_sites);                                                   \
        else                                                                                  \
            hipLaunchKernelGGL((k_train<KK, false>), dim3(a.n_blocks), dim3(256), 0, st, pa, a,   \
                               fx, r4, li, lo, target, rendered, grad_img, &state->loss,      \
                               grad_sites);                                                   \
        break;
    switch (img->K) {
        SAD_TRAIN_CASE(4)
        SAD_TRAIN_CASE(8)
        SAD_TRAIN_CASE(12)
        SAD_TRAIN_CASE(16)
        SAD_TRAIN_CASE(20)
        SAD_TRAIN_CASE(24)
        SAD_TRAIN_CASE(28)
        SAD_TRAIN_CASE(32)
        default: break;
    }
#undef SAD_TRAIN_CASE
    if (fold) launch_loss_fold(&state->loss, overwrite_loss, st);
    return check_launch("training pass");
}

extern "C" sad_status sad_train_image_pass(const sad_image *img, const sad_train_config *cfg,
                                           const float *target, const float *rec,
                                           const uint32_t *topk_in, uint32_t *topk_out,
                                           float *grad_sites, float *rendered, float *grad_img,
                                           sad_step_state *state, void *stream) {
    return image_pass(img, cfg, target, rec, topk_in, topk_out, grad_sites, rendered, grad_img,
                      state, false, true, as_stream(stream));
}

extern "C" sad_status sad_train_step(const sad_image *img, const sad_train_config *cfg,
                                     const float *target, float *sites, float *rec,
                                     const uint32_t *topk_in, uint32_t *topk_out, float *grad_sites,
                                     float *adam_m, float *adam_v, float *rendered, float *grad_img,
                                     sad_step_state *state, void *stream) {
    float s;
    SAD_TRY(check_image(img, &s));
    SAD_REQUIRE(sites && adam_m && adam_v, SAD_ERR_INVALID_ARGUMENT, "sad_train_step: NULL pointer");
    hipStream_t st = as_stream(stream);
    if (img->n_slots == 0) {  // nothing to optimise: fold the loss, advance the counters
        SAD_TRY(image_pass(img, cfg, target, rec, topk_in, topk_out, grad_sites, rendered,
                           grad_img, state, true, true, st));
        launch_state_advance(state, st);
        return check_launch("sad_train_step");
    }
    // the image pass leaves its loss partials; the last Adam block folds them and
    // advances the counters (two kernels per iteration)
    SAD_TRY(image_pass(img, cfg, target, rec, topk_in, topk_out, grad_sites, rendered, grad_img,
                       state, true, false, st));
    launch_adam(img, s, sites, grad_sites, adam_m, adam_v, &cfg->adam, 1, &state->adam_step, rec,
                true, true, state, st, (cfg->flags & SAD_TRAIN_DETERMINISTIC) != 0);
    return check_launch("sad_train_step");
}

extern "C" sad_status sad_grad_to_params(const sad_image *img, float *grad_site_major,
                                         const float *scale, float *grad, uint32_t flags,
                                         void *stream) {
    SAD_TRY(check_image(img, nullptr));
    SAD_REQUIRE(grad_site_major && grad, SAD_ERR_INVALID_ARGUMENT,
                "sad_grad_to_params: NULL pointer");
    SAD_REQUIRE(grad_site_major != grad, SAD_ERR_INVALID_ARGUMENT,
                "sad_grad_to_params: source and destination must not alias");
    SAD_REQUIRE((flags & ~SAD_GRAD_CLEAR_SOURCE) == 0, SAD_ERR_INVALID_ARGUMENT,
                "sad_grad_to_params: unknown flags 0x%x", flags);
    if (img->cap == 0) return SAD_OK;
    hipLaunchKernelGGL(k_grad_to_params, dim3((unsigned)((img->cap + 255) / 256)), dim3(256), 0,
                       as_stream(stream), grad_site_major, scale, grad, img->cap,
                       (flags & SAD_GRAD_CLEAR_SOURCE) ? 1 : 0);
    return check_launch("sad_grad_to_params");
}
