// batch.hip -- one training iteration of many images of uneven size in one persistent
// launch over (image, 16x16 tile) work items, plus per-image loss folds, one Adam
// launch over every site slot and one state update.
#include "sad_device.h"
#include "sad_host.h"
#include "sad_internal.h"
#include "sad_kernels.h"
#include "sad_sites.h"

namespace sad {

// Largest b with key(b) <= x over a non-decreasing device array (b in [0, n)).
template <typename F>
__device__ __forceinline__ int upper_index(int n, int64_t x, F key) {
    int lo = 0, hi = n - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (key(mid) <= x)
            lo = mid;
        else
            hi = mid - 1;
    }
    return lo;
}

__device__ __forceinline__ FixScale fix_scale_dev(int64_t P) {
    const int e = fix_exponent(P);
    FixScale fx;
    fx.to_fix = ldexp(1.0, 32 + e);
    fx.from_fix = ldexp(1.0, -(32 + e));
    fx.limit = (float)ldexp(1.0, 15 - e);
    fx.to_det = ldexp(1.0, 40 + e - kGlobShift);
    fx.pre = ldexpf(1.0f, 32 + e);
    fx.pre_det = ldexpf(1.0f, 40 + e - kGlobShift);
    fx.post = ldexpf(1.0f, -(32 + e));
    return fx;
}

struct BatchArgs {
    int n_images, n_items, chunked, J, fixed_jump, every;
    uint64_t seed;
    const sad_batch_image *images;
};

// One (image, tile) work item: propagate, render, loss gradient and backward of its 256
// pixels, flushed into the image's site-major gradient.  The queue and the accumulators
// share one LDS buffer (used in turn, as in the single-image training kernel).
template <int K, bool kDet, int TW>
__device__ __forceinline__ void batch_item(const BatchArgs &ba, int item,
                                           const float4 *__restrict__ rec,
                                           const uint4 *__restrict__ lin,
                                           uint4 *__restrict__ lout,
                                           const float *__restrict__ tgt,
                                           float *__restrict__ rendered, float *__restrict__ gimg,
                                           sad_step_state *__restrict__ states,
                                           float *__restrict__ grad, uint32_t *lds,
                                           uint32_t *hkey, uint32_t *occ) {
    uint32_t(*queue)[256] = reinterpret_cast<uint32_t(*)[256]>(lds);
    unsigned long long(*hacc)[kHashSlots] = reinterpret_cast<unsigned long long(*)[kHashSlots]>(lds);
    // the item, and so the image, is the same for the whole block: keep its
    // descriptor in scalar registers
    const int b = __builtin_amdgcn_readfirstlane(
        upper_index(ba.n_images, item, [&](int k) { return (int64_t)ba.images[k].tile0; }));
    sad_batch_image im = ba.images[b];
    im.H = __builtin_amdgcn_readfirstlane(im.H);
    im.W = __builtin_amdgcn_readfirstlane(im.W);
    im.n_slots = __builtin_amdgcn_readfirstlane(im.n_slots);
    im.tile0 = __builtin_amdgcn_readfirstlane(im.tile0);
    im.cap = ((int64_t)__builtin_amdgcn_readfirstlane((int)(im.cap >> 32)) << 32) |
             (uint32_t)__builtin_amdgcn_readfirstlane((int)im.cap);
    im.px0 = ((int64_t)__builtin_amdgcn_readfirstlane((int)(im.px0 >> 32)) << 32) |
             (uint32_t)__builtin_amdgcn_readfirstlane((int)im.px0);
    im.site0 = ((int64_t)__builtin_amdgcn_readfirstlane((int)(im.site0 >> 32)) << 32) |
               (uint32_t)__builtin_amdgcn_readfirstlane((int)im.site0);
    const int tiles_x = (im.W + TW - 1) / TW;
    const TilePix px = tile_pixel_w<TW>(item - im.tile0, tiles_x);
    const int64_t P = (int64_t)im.H * im.W;
    PropArgs pa;
    pa.H = im.H;
    pa.W = im.W;
    pa.n_slots = im.n_slots;
    pa.jump = ba.fixed_jump > 0 ? ba.fixed_jump : 0;
    pa.J = ba.J;
    pa.every = ba.every;
    pa.tiles_x = tiles_x;
    pa.n_blocks = 0;
    pa.seed = ba.seed;
    pa.pass = 0;
    pa.pass_dev = &states[b].pass;
    const float inv_P = (float)(1.0 / (double)P);
    const FixScale fx = fix_scale_dev(P);
    const float4 *r4 = rec + 4 * im.site0;
    const uint4 *li = lin + (int64_t)(K / 4) * im.px0;
    uint4 *lo = lout + (int64_t)(K / 4) * im.px0;
    const float *tg = tgt + 3 * im.px0;
    // the image's gradient rows (int64 elements in the deterministic mode)
    float *gr = kDet ? reinterpret_cast<float *>(reinterpret_cast<long long *>(grad) + 10 * im.site0)
                     : grad + 10 * im.site0;

    const bool live = im.n_slots > 0 && px.i < im.H && px.j < im.W;
    const int64_t p = (int64_t)px.i * im.W + px.j;
    uint64_t keys[K];
    if (live) {
        prop_pixel<K>(pa, r4, li, px, queue, keys);
#pragma unroll
        for (int g = 0; g < K / 4; ++g)
            lo[(int64_t)g * P + p] = make_uint4(key_id(keys[4 * g]), key_id(keys[4 * g + 1]),
                                                key_id(keys[4 * g + 2]),
                                                key_id(keys[4 * g + 3]));
    }
    __syncthreads();  // the queue is free: clear the accumulators in its place
    bwd_tile_init<10>(hkey, hacc);
    __syncthreads();
    float sq = 0.f;
    if (live) {
        const float X = (float)px.j, Y = (float)px.i;
        PixelBlend<K> bl;
        blend_keys<K, true>(r4, keys, bl, lane_rot() % K);
        float g[3];
#pragma unroll
        for (int ch = 0; ch < 3; ++ch) {
            const float d = bl.c[ch] - tg[ch * P + p];
            g[ch] = 2.0f * inv_P * d;
            sq = fmaf(d, d, sq);
            if (gimg) gimg[3 * im.px0 + ch * P + p] = g[ch];
            if (rendered) rendered[3 * im.px0 + ch * P + p] = bl.c[ch];
        }
        bwd_pixel<K, false, true, kDet>(r4, bl, X, Y, g[0], g[1], g[2], 0.f, 0.f, 0.f, hkey,
                                        hacc, fx, inv_P, im.cap, gr, nullptr);
    } else if (im.n_slots == 0 && px.i < im.H && px.j < im.W) {
        // no sites: empty list, colour 0
#pragma unroll
        for (int g = 0; g < K / 4; ++g)
            lo[(int64_t)g * P + p] = make_uint4(SAD_INVALID_ID, SAD_INVALID_ID, SAD_INVALID_ID,
                                                SAD_INVALID_ID);
#pragma unroll
        for (int ch = 0; ch < 3; ++ch) {
            const float d = -tg[ch * P + p];
            sq = fmaf(d, d, sq);
            if (gimg) gimg[3 * im.px0 + ch * P + p] = 2.0f * inv_P * d;
            if (rendered) rendered[3 * im.px0 + ch * P + p] = 0.f;
        }
    }
    const float tot = block_sum(sq);  // includes a barrier
    if (threadIdx.x == 0)
        atomic_add_f32(&states[b].loss.part[item % SAD_LOSS_PARTS], tot * inv_P);
    bwd_flush<false, true, kDet>(hkey, hacc, fx, im.cap, gr, nullptr, occ);
}

template <int K>
constexpr int batch_lds_words() {
    return (QueueDepth<K>::v > 20 ? QueueDepth<K>::v : 20) * 256;
}

// Persistent form: gridDim.x blocks walk the items in contiguous runs (block -> XCD-local
// range) or round robin.  The loop costs registers: for K <= 8 the kernel is held to 128
// VGPRs (four waves per SIMD, no spill); larger K would spill under that cap and is left
// uncapped.
template <int K, bool kDet, int TW>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(K <= 8 ? 4 : 1, 8))) void k_batch_train(
    BatchArgs ba, const float4 *__restrict__ rec, const uint4 *__restrict__ lin,
    uint4 *__restrict__ lout, const float *__restrict__ tgt, float *__restrict__ rendered,
    float *__restrict__ gimg, sad_step_state *__restrict__ states, float *__restrict__ grad) {
    __shared__ __align__(16) uint32_t lds[batch_lds_words<K>()];
    __shared__ uint32_t hkey[kHashSlots];
    __shared__ uint32_t occ[kHashSlots + 1];
    const int G = gridDim.x;
    int first, step, last;
    if (ba.chunked) {
        const int b = xcd_tile(blockIdx.x, G);
        const int per = (ba.n_items + G - 1) / G;
        first = b * per;
        last = min(first + per, ba.n_items);
        step = 1;
    } else {
        first = blockIdx.x;
        last = ba.n_items;
        step = G;
    }
    for (int item = first; item < last; item += step) {
        batch_item<K, kDet, TW>(ba, item, rec, lin, lout, tgt, rendered, gimg, states, grad, lds,
                                hkey, occ);
        __syncthreads();  // the next item re-initialises the table
    }
}

// One block per item (no loop), items remapped so that each XCD takes a contiguous run
// of them (neighbouring tiles of an image share that XCD's L2).
template <int K, bool kDet, int TW>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(K == 16 ? 4 : 1, 8))) void k_batch_train_1(
    BatchArgs ba, const float4 *__restrict__ rec, const uint4 *__restrict__ lin,
    uint4 *__restrict__ lout, const float *__restrict__ tgt, float *__restrict__ rendered,
    float *__restrict__ gimg, sad_step_state *__restrict__ states, float *__restrict__ grad) {
    __shared__ __align__(16) uint32_t lds[batch_lds_words<K>()];
    __shared__ uint32_t hkey[kHashSlots];
    __shared__ uint32_t occ[kHashSlots + 1];
    batch_item<K, kDet, TW>(ba, xcd_tile(blockIdx.x, gridDim.x), rec, lin, lout, tgt, rendered,
                            gimg, states, grad, lds, hkey, occ);
}

__global__ __launch_bounds__(64) void k_batch_loss_fold(sad_step_state *__restrict__ states) {
    sad_loss_acc *loss = &states[blockIdx.x].loss;
    const int i = threadIdx.x;
    float v = i < SAD_LOSS_PARTS ? loss->part[i] : 0.f;
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    if (i < SAD_LOSS_PARTS) loss->part[i] = 0.f;
    if (i == 0) loss->value = v;
}

__device__ __forceinline__ void batch_adam_slot(int n_images,
                                                const sad_batch_image *__restrict__ imgs,
                                                int64_t gi, float *__restrict__ sites,
                                                float *__restrict__ grad, float *__restrict__ m,
                                                float *__restrict__ v, float4 *__restrict__ rec,
                                                const sad_step_state *__restrict__ states,
                                                const AdamArgs &A) {
    const int b = upper_index(n_images, gi, [&](int k) { return imgs[k].site0; });
    const sad_batch_image im = imgs[b];
    const int64_t i = gi - im.site0;
    if (i >= im.n_slots) return;  // slots beyond n_slots are not sites
    const float s = im.score_scale != 0.0f ? im.score_scale
                                           : 1.0f / (float)(im.H > im.W ? im.H : im.W);
    const int64_t o = 10 * im.site0;
    float *g = A.grad_fixed ? reinterpret_cast<float *>(reinterpret_cast<long long *>(grad) + o)
                            : grad + o;
    AdamArgs Ai = A;
    Ai.grad_from = det_grad_unit((int64_t)im.H * im.W);
    adam_site(sites + o, g, m + o, v + o, im.cap, i, im.H, im.W, Ai, &states[b].adam_step, s,
              rec + 4 * im.site0);
}

// Adam over every site slot of the batch.  (The loss fold and the counter update stay
// separate one-block kernels here: a finishing block would need one same-address atomic
// per Adam block, thousands for a large batch.)
__global__ __launch_bounds__(256) void k_batch_adam(int n_images, const sad_batch_image *__restrict__ imgs,
                                                    int64_t n_slots_total, float *__restrict__ sites,
                                                    float *__restrict__ grad, float *__restrict__ m,
                                                    float *__restrict__ v, float4 *__restrict__ rec,
                                                    const sad_step_state *__restrict__ states,
                                                    AdamArgs A) {
    const int64_t gi = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (gi < n_slots_total) batch_adam_slot(n_images, imgs, gi, sites, grad, m, v, rec, states, A);
}

__global__ __launch_bounds__(256) void k_batch_advance(sad_step_state *__restrict__ states, int n) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b < n) {
        states[b].pass += 1;
        states[b].adam_step += 1;
    }
}

}  // namespace sad

using namespace sad;

extern "C" sad_status sad_batch_train_step(const sad_batch *batch, const sad_train_config *cfg,
                                           const float *target, float *sites, float *rec,
                                           const uint32_t *topk_in, uint32_t *topk_out,
                                           float *grad_sites, float *adam_m, float *adam_v,
                                           float *rendered, float *grad_img,
                                           sad_step_state *states, void *stream) {
    SAD_REQUIRE(batch && cfg && states, SAD_ERR_INVALID_ARGUMENT, "sad_batch_train_step: NULL argument");
    SAD_REQUIRE(batch->n_images >= 1 && batch->images, SAD_ERR_INVALID_ARGUMENT,
                "sad_batch_train_step: empty batch");
    SAD_REQUIRE(batch->K >= 4 && batch->K <= SAD_MAX_K && (batch->K & 3) == 0, SAD_ERR_UNSUPPORTED,
                "sad_batch_train_step: K = %d unsupported", batch->K);
    SAD_REQUIRE(batch->n_items >= 1 && batch->n_site_slots >= 0, SAD_ERR_INVALID_ARGUMENT,
                "sad_batch_train_step: bad item / slot counts");
    SAD_REQUIRE(target && sites && rec && topk_in && topk_out && grad_sites && adam_m && adam_v,
                SAD_ERR_INVALID_ARGUMENT, "sad_batch_train_step: NULL pointer");
    SAD_REQUIRE(topk_in != topk_out, SAD_ERR_INVALID_ARGUMENT,
                "sad_batch_train_step: topk_in and topk_out must not alias");
    SAD_REQUIRE(aligned16(rec) && aligned16(topk_in) && aligned16(topk_out),
                SAD_ERR_INVALID_ARGUMENT, "sad_batch_train_step: rec / lists not 16-byte aligned");
    SAD_REQUIRE(cfg->n_inject >= 0 && cfg->n_inject <= 16, SAD_ERR_INVALID_ARGUMENT,
                "sad_batch_train_step: n_inject must be in [0, 16]");
    SAD_REQUIRE(cfg->prop_every >= 0 && cfg->prop_every <= 1024, SAD_ERR_INVALID_ARGUMENT,
                "training pass: prop_every must be in [0, 1024]");
    SAD_REQUIRE((cfg->flags & ~SAD_TRAIN_DETERMINISTIC) == 0, SAD_ERR_INVALID_ARGUMENT,
                "sad_batch_train_step: unknown flags 0x%x", cfg->flags);
    SAD_REQUIRE(batch->tile_w == 0 || batch->tile_w == 16 || batch->tile_w == 32,
                SAD_ERR_UNSUPPORTED, "sad_batch_train_step: tile width %d (16 or 32)",
                batch->tile_w);
    const bool det = (cfg->flags & SAD_TRAIN_DETERMINISTIC) != 0;
    const bool wide = batch->tile_w == 32;
    hipStream_t st = as_stream(stream);
    BatchArgs ba;
    ba.n_images = batch->n_images;
    ba.n_items = batch->n_items;
    ba.chunked = batch->chunked;
    ba.J = cfg->n_inject;
    ba.fixed_jump = cfg->fixed_jump;
    ba.every = cfg->prop_every;
    ba.seed = cfg->seed;
    ba.images = batch->images;
    const int grid = batch->grid > 0 ? (batch->grid < batch->n_items ? batch->grid : batch->n_items)
                                     : batch->n_items;
    const float4 *r4 = reinterpret_cast<const float4 *>(rec);
    const uint4 *li = reinterpret_cast<const uint4 *>(topk_in);
    uint4 *lo = reinterpret_cast<uint4 *>(topk_out);
#define SAD_BATCH_LAUNCH(KK, DET, TW)                                                          \
    if (batch->grid > 0 && grid < batch->n_items)                                              \
        hipLaunchKernelGGL((k_batch_train<KK, DET, TW>), dim3(grid), dim3(256), 0, st, ba, r4,   \
                           li, lo, target, rendered, grad_img, states, grad_sites);           \
    else                                                                                       \
        hipLaunchKernelGGL((k_batch_train_1<KK, DET, TW>), dim3(ba.n_items), dim3(256), 0, st,   \
                           ba, r4, li, lo, target, rendered, grad_img, states, grad_sites);
#define SAD_BATCH_CASE(KK)                                                                     \
    case KK:                                                                                   \
        if (det) {                                                                             \
            if (wide) {                                                                        \
                SAD_BATCH_LAUNCH(KK, true, 32)                                                 \
            } else {                                                                           \
                SAD_BATCH_LAUNCH(KK, true, 16)                                                 \
            }                                                                                  \
        } else {                                                                               \
            if (wide) {                                                                        \
                SAD_BATCH_LAUNCH(KK, false, 32)                                                \
            } else {                                                                           \
                SAD_BATCH_LAUNCH(KK, false, 16)                                                \
            }                                                                                  \
        }                                                                                      \
        break;
    switch (batch->K) {
        SAD_BATCH_CASE(4)
        SAD_BATCH_CASE(8)
        SAD_BATCH_CASE(12)
        SAD_BATCH_CASE(16)
        SAD_BATCH_CASE(20)
        SAD_BATCH_CASE(24)
        SAD_BATCH_CASE(28)
        SAD_BATCH_CASE(32)
        default: break;
    }
#undef SAD_BATCH_CASE
#undef SAD_BATCH_LAUNCH
    AdamArgs A;
    for (int p = 0; p < SAD_NPARAM; ++p) A.lr[p] = cfg->adam.lr[p];
    A.b1 = cfg->adam.beta1;
    A.b2 = cfg->adam.beta2;
    A.eps = cfg->adam.eps;
    A.c1 = A.c2 = 1.0f;  // formed on the device from each image's step
    A.zero_grad = 1;
    A.grad_site_major = 1;
    A.grad_fixed = det ? 1 : 0;
    A.grad_from = 0.0;  // set per image on the device
    hipLaunchKernelGGL(k_batch_loss_fold, dim3(batch->n_images), dim3(64), 0, st, states);
    if (batch->n_site_slots > 0)
        hipLaunchKernelGGL(k_batch_adam, dim3((unsigned)((batch->n_site_slots + 255) / 256)),
                           dim3(256), 0, st, batch->n_images, batch->images, batch->n_site_slots,
                           sites, grad_sites, adam_m, adam_v, reinterpret_cast<float4 *>(rec),
                           states, A);
    hipLaunchKernelGGL(k_batch_advance, dim3((batch->n_images + 255) / 256), dim3(256), 0, st,
                       states, batch->n_images);
    return check_launch("sad_batch_train_step");
}
