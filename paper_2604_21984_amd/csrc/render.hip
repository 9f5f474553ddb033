// render.hip -- forward blend (Sec. 4.2), loss gradient (Sec. 6.1), backward scatter
// with per-tile LDS pre-reduction (App. B.4, Sec. 4.8), point queries (Sec. 6.6).
#include <cmath>

#include "sad_device.h"
#include "sad_host.h"
#include "sad_internal.h"
#include "sad_kernels.h"

namespace sad {

template <int K>
__global__ __launch_bounds__(256) void k_fwd(ImgArgs a, const float4 *__restrict__ rec,
                                             const uint4 *__restrict__ topk,
                                             float *__restrict__ out) {
    const int tile = xcd_tile(blockIdx.x, a.n_blocks);
    const TilePix px = tile_pixel(tile, a.tiles_x);
    if (px.i >= a.H || px.j >= a.W) return;
    const int64_t P = (int64_t)a.H * a.W, p = (int64_t)px.i * a.W + px.j;
    PixelBlend<K> b;
    blend<K, false>(rec, (uint32_t)a.n_slots, topk, P, p, (float)px.j, (float)px.i, b,
                    lane_rot() % K);
    out[p] = b.c[0];
    out[P + p] = b.c[1];
    out[2 * P + p] = b.c[2];
}

// dL/dc = (2/P)(c - I); loss += (1/P) sum (c - I)^2.  Grid-stride over a bounded
// number of blocks, one atomic per block (a single address takes every block's atomic).
__global__ __launch_bounds__(256) void k_loss_grad(const float *__restrict__ img,
                                                   const float *__restrict__ tgt,
                                                   float *__restrict__ grad, int64_t n3,
                                                   float inv_P, sad_loss_acc *__restrict__ loss) {
    float sq = 0.f;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n3;
         i += (int64_t)gridDim.x * blockDim.x) {
        const float d = img[i] - tgt[i];
        grad[i] = 2.0f * inv_P * d;
        sq = fmaf(d, d, sq);
    }
    if (!loss) return;
    const float t = block_sum(sq);
    if (threadIdx.x == 0) atomic_add_f32(&loss->part[blockIdx.x % SAD_LOSS_PARTS], t * inv_P);
}

// Fold the partials into value (added, or written if `overwrite`) and clear them.
__global__ __launch_bounds__(64) void k_loss_fold(sad_loss_acc *__restrict__ loss, int overwrite) {
    const int i = threadIdx.x;
    float v = i < SAD_LOSS_PARTS ? loss->part[i] : 0.f;
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    if (i < SAD_LOSS_PARTS) loss->part[i] = 0.f;
    if (i == 0) loss->value = overwrite ? v : loss->value + v;
}

// Forward blend fused with the loss gradient (training step): writes dL/dc and,
// optionally, the rendered image; one loss atomic per block.
template <int K>
__global__ __launch_bounds__(256) void k_fwd_loss(ImgArgs a, const float4 *__restrict__ rec,
                                                  const uint4 *__restrict__ topk,
                                                  const float *__restrict__ tgt,
                                                  float *__restrict__ out,
                                                  float *__restrict__ gimg,
                                                  sad_loss_acc *__restrict__ loss) {
    const int tile = xcd_tile(blockIdx.x, a.n_blocks);
    const TilePix px = tile_pixel(tile, a.tiles_x);
    float sq = 0.f;
    if (px.i < a.H && px.j < a.W) {
        const int64_t P = (int64_t)a.H * a.W, p = (int64_t)px.i * a.W + px.j;
        PixelBlend<K> b;
        blend<K, false>(rec, (uint32_t)a.n_slots, topk, P, p, (float)px.j, (float)px.i, b,
                        lane_rot() % K);
#pragma unroll
        for (int ch = 0; ch < 3; ++ch) {
            const float d = b.c[ch] - tgt[ch * P + p];
            gimg[ch * P + p] = 2.0f * a.inv_P * d;
            if (out) out[ch * P + p] = b.c[ch];
            sq = fmaf(d, d, sq);
        }
    }
    if (!loss) return;
    const float t = block_sum(sq);
    if (threadIdx.x == 0) atomic_add_f32(&loss->part[blockIdx.x % SAD_LOSS_PARTS], t * a.inv_P);
}

template <int K, bool kRD>
__global__ __launch_bounds__(256) void k_bwd(ImgArgs a, FixScale fx, const float4 *__restrict__ rec,
                                             const uint4 *__restrict__ topk,
                                             const float *__restrict__ gimg,
                                             const float *__restrict__ tgt,
                                             float *__restrict__ grad, float *__restrict__ rdel) {
    __shared__ uint32_t hkey[kHashSlots];
    __shared__ uint32_t occ[kHashSlots + 1];
    __shared__ unsigned long long hacc[kAcc][kHashSlots];
    bwd_tile_init(hkey, hacc);
    __syncthreads();

    const int tile = xcd_tile(blockIdx.x, a.n_blocks);
    const TilePix px = tile_pixel(tile, a.tiles_x);
    if (px.i < a.H && px.j < a.W) {
        const int64_t P = (int64_t)a.H * a.W, p = (int64_t)px.i * a.W + px.j;
        const float X = (float)px.j, Y = (float)px.i;
        PixelBlend<K> b;
        blend<K, true>(rec, (uint32_t)a.n_slots, topk, P, p, X, Y, b, lane_rot() % K);
        const float I0 = kRD ? tgt[p] : 0.f, I1 = kRD ? tgt[P + p] : 0.f;
        const float I2 = kRD ? tgt[2 * P + p] : 0.f;
        bwd_pixel<K, kRD>(rec, b, X, Y, gimg[p], gimg[P + p], gimg[2 * P + p], I0, I1, I2,
                          hkey, hacc, fx, a.inv_P, a.cap, grad, rdel);
    }
    __syncthreads();
    bwd_flush<kRD>(hkey, hacc, fx, a.cap, grad, rdel, occ);
}

// ---- point queries ----------------------------------------------------------------
template <int K>
__global__ __launch_bounds__(256) void k_query(ImgArgs a, const float4 *__restrict__ rec,
                                               const uint4 *__restrict__ topk,
                                               const float2 *__restrict__ xy, int64_t M,
                                               float *__restrict__ out) {
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= M) return;
    const float2 pt = xy[q];
    const float fi = rintf(pt.y), fj = rintf(pt.x);
    const int ii = !(fi > 0.f) ? 0 : (fi > (float)(a.H - 1) ? a.H - 1 : (int)fi);
    const int jj = !(fj > 0.f) ? 0 : (fj > (float)(a.W - 1) ? a.W - 1 : (int)fj);
    const int64_t P = (int64_t)a.H * a.W, p = (int64_t)ii * a.W + jj;
    PixelBlend<K> b;
    blend<K, false>(rec, (uint32_t)a.n_slots, topk, P, p, pt.x, pt.y, b);
    out[3 * q] = b.c[0];
    out[3 * q + 1] = b.c[1];
    out[3 * q + 2] = b.c[2];
}

// Serving: one thread per point over all jobs; the job is found by binary search on q0.
template <int K>
__global__ __launch_bounds__(256) void k_query_batch(const sad_query_job *__restrict__ jobs,
                                                     int n_jobs, int64_t total) {
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= total) return;
    int lo = 0, hi = n_jobs - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (jobs[mid].q0 <= g)
            lo = mid;
        else
            hi = mid - 1;
    }
    const sad_query_job jb = jobs[lo];
    const int64_t q = g - jb.q0;
    if (q < 0 || q >= jb.M) return;
    const float2 pt = reinterpret_cast<const float2 *>(jb.xy)[q];
    const float fi = rintf(pt.y), fj = rintf(pt.x);
    const int ii = !(fi > 0.f) ? 0 : (fi > (float)(jb.H - 1) ? jb.H - 1 : (int)fi);
    const int jj = !(fj > 0.f) ? 0 : (fj > (float)(jb.W - 1) ? jb.W - 1 : (int)fj);
    const int64_t P = (int64_t)jb.H * jb.W, p = (int64_t)ii * jb.W + jj;
    float c0 = 0.f, c1 = 0.f, c2 = 0.f;
    if (jb.n_slots > 0) {
        PixelBlend<K> b;
        blend<K, false>(reinterpret_cast<const float4 *>(jb.rec), (uint32_t)jb.n_slots,
                        reinterpret_cast<const uint4 *>(jb.topk), P, p, pt.x, pt.y, b);
        c0 = b.c[0];
        c1 = b.c[1];
        c2 = b.c[2];
    }
    jb.out[3 * q] = c0;
    jb.out[3 * q + 1] = c1;
    jb.out[3 * q + 2] = c2;
}

__global__ __launch_bounds__(256) void k_fill(float *__restrict__ p, int64_t n, float v) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}


}  // namespace sad

using namespace sad;

void sad::launch_fwd(const sad_image *img, const float *rec, const uint32_t *topk, float *out,
                     hipStream_t st) {
    const ImgArgs a = img_args(img);
    if (img->n_slots == 0) {
        launch_fill_f32(out, 3ll * img->H * img->W, 0.0f, st);
        return;
    }
    const float4 *r4 = reinterpret_cast<const float4 *>(rec);
    const uint4 *l4 = reinterpret_cast<const uint4 *>(topk);
    SAD_K_SWITCH(img->K, hipLaunchKernelGGL(k_fwd<KK>, dim3(a.n_blocks), dim3(256), 0, st, a, r4,
                                            l4, out));
}

void sad::launch_loss_fold(sad_loss_acc *loss, bool overwrite, hipStream_t st) {
    hipLaunchKernelGGL(k_loss_fold, dim3(1), dim3(64), 0, st, loss, overwrite ? 1 : 0);
}

void sad::launch_loss_grad(const sad_image *img, const float *rendered, const float *target,
                           float *grad, sad_loss_acc *loss, bool overwrite, hipStream_t st) {
    const int64_t n3 = 3ll * img->H * img->W;
    int64_t nb = (n3 + 256 * 8 - 1) / (256 * 8);
    if (nb > 512) nb = 512;
    if (nb < 1) nb = 1;
    hipLaunchKernelGGL(k_loss_grad, dim3((unsigned)nb), dim3(256), 0, st, rendered, target, grad, n3,
                       (float)(1.0 / ((double)img->H * img->W)), loss);
    if (loss) launch_loss_fold(loss, overwrite, st);
}

void sad::launch_fwd_loss(const sad_image *img, const float *rec, const uint32_t *topk,
                          const float *target, float *rendered, float *grad_img,
                          sad_loss_acc *loss, bool overwrite, hipStream_t st) {
    if (img->n_slots == 0) {  // colour 0 everywhere; the loss kernel reads the zeros in place
        if (rendered) launch_fill_f32(rendered, 3ll * img->H * img->W, 0.0f, st);
        launch_fill_f32(grad_img, 3ll * img->H * img->W, 0.0f, st);
        launch_loss_grad(img, grad_img, target, grad_img, loss, overwrite, st);
        return;
    }
    const ImgArgs a = img_args(img);
    const float4 *r4 = reinterpret_cast<const float4 *>(rec);
    const uint4 *l4 = reinterpret_cast<const uint4 *>(topk);
    SAD_K_SWITCH(img->K, hipLaunchKernelGGL(k_fwd_loss<KK>, dim3(a.n_blocks), dim3(256), 0, st, a,
                                            r4, l4, target, rendered, grad_img, loss));
    if (loss) launch_loss_fold(loss, overwrite, st);
}

void sad::launch_bwd(const sad_image *img, const float *rec, const uint32_t *topk,
                     const float *grad_img, const float *target, float *grad_sites,
                     float *removal_delta, hipStream_t st) {
    if (img->n_slots == 0) return;
    const ImgArgs a = img_args(img);
    const FixScale fx = fix_scale((int64_t)img->H * img->W);
    const float4 *r4 = reinterpret_cast<const float4 *>(rec);
    const uint4 *l4 = reinterpret_cast<const uint4 *>(topk);
    if (removal_delta) {
        SAD_K_SWITCH(img->K, hipLaunchKernelGGL((k_bwd<KK, true>), dim3(a.n_blocks), dim3(256), 0,
                                                st, a, fx, r4, l4, grad_img, target, grad_sites,
                                                removal_delta));
    } else {
        SAD_K_SWITCH(img->K, hipLaunchKernelGGL((k_bwd<KK, false>), dim3(a.n_blocks), dim3(256), 0,
                                                st, a, fx, r4, l4, grad_img, target, grad_sites,
                                                removal_delta));
    }
}

void sad::launch_fill_f32(float *p, int64_t n, float v, hipStream_t st) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_fill, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, p, n, v);
}

extern "C" sad_status sad_render_fwd(const sad_image *img, const float *rec, const uint32_t *topk,
                                     float *out, void *stream) {
    SAD_TRY(check_image(img, nullptr));
    SAD_REQUIRE(topk && out, SAD_ERR_INVALID_ARGUMENT, "sad_render_fwd: NULL pointer");
    SAD_REQUIRE(aligned16(topk), SAD_ERR_INVALID_ARGUMENT, "sad_render_fwd: topk not 16-byte aligned");
    SAD_REQUIRE(img->n_slots == 0 || (rec && aligned16(rec)), SAD_ERR_INVALID_ARGUMENT,
                "sad_render_fwd: bad rec");
    launch_fwd(img, rec, topk, out, as_stream(stream));
    return check_launch("sad_render_fwd");
}

extern "C" sad_status sad_loss_grad(const sad_image *img, const float *rendered,
                                    const float *target, float *grad, sad_loss_acc *loss,
                                    void *stream) {
    SAD_TRY(check_image(img, nullptr));
    SAD_REQUIRE(rendered && target && grad, SAD_ERR_INVALID_ARGUMENT, "sad_loss_grad: NULL pointer");
    launch_loss_grad(img, rendered, target, grad, loss, false, as_stream(stream));
    return check_launch("sad_loss_grad");
}

extern "C" sad_status sad_render_fwd_loss(const sad_image *img, const float *rec,
                                          const uint32_t *topk, const float *target,
                                          float *rendered, float *grad_img, sad_loss_acc *loss,
                                          void *stream) {
    SAD_TRY(check_image(img, nullptr));
    SAD_REQUIRE(topk && target && grad_img, SAD_ERR_INVALID_ARGUMENT,
                "sad_render_fwd_loss: NULL pointer");
    SAD_REQUIRE(aligned16(topk), SAD_ERR_INVALID_ARGUMENT,
                "sad_render_fwd_loss: topk not 16-byte aligned");
    SAD_REQUIRE(img->n_slots == 0 || (rec && aligned16(rec)), SAD_ERR_INVALID_ARGUMENT,
                "sad_render_fwd_loss: bad rec");
    launch_fwd_loss(img, rec, topk, target, rendered, grad_img, loss, false, as_stream(stream));
    return check_launch("sad_render_fwd_loss");
}

extern "C" sad_status sad_render_bwd(const sad_image *img, const float *rec, const uint32_t *topk,
                                     const float *grad_img, const float *target, float *grad_sites,
                                     float *removal_delta, void *stream) {
    SAD_TRY(check_image(img, nullptr));
    SAD_REQUIRE(topk && grad_img && grad_sites, SAD_ERR_INVALID_ARGUMENT,
                "sad_render_bwd: NULL pointer");
    SAD_REQUIRE(!removal_delta || target, SAD_ERR_INVALID_ARGUMENT,
                "sad_render_bwd: removal_delta requires target");
    SAD_REQUIRE(aligned16(topk), SAD_ERR_INVALID_ARGUMENT, "sad_render_bwd: topk not 16-byte aligned");
    SAD_REQUIRE(img->n_slots == 0 || (rec && aligned16(rec)), SAD_ERR_INVALID_ARGUMENT,
                "sad_render_bwd: bad rec");
    launch_bwd(img, rec, topk, grad_img, target, grad_sites, removal_delta, as_stream(stream));
    return check_launch("sad_render_bwd");
}

extern "C" sad_status sad_query_points(const sad_image *img, const float *rec, const uint32_t *topk,
                                       const float *xy, int64_t M, float *out, void *stream) {
    SAD_TRY(check_image(img, nullptr));
    SAD_REQUIRE(M >= 0, SAD_ERR_INVALID_ARGUMENT, "sad_query_points: M < 0");
    if (M == 0) return SAD_OK;
    SAD_REQUIRE(topk && xy && out, SAD_ERR_INVALID_ARGUMENT, "sad_query_points: NULL pointer");
    SAD_REQUIRE(aligned16(topk) && (reinterpret_cast<uintptr_t>(xy) & 7u) == 0,
                SAD_ERR_INVALID_ARGUMENT, "sad_query_points: misaligned pointer");
    SAD_REQUIRE(M <= ((int64_t)1 << 31) * 255, SAD_ERR_INVALID_ARGUMENT, "sad_query_points: M too large");
    hipStream_t st = as_stream(stream);
    if (img->n_slots == 0) {
        launch_fill_f32(out, 3 * M, 0.0f, st);
        return check_launch("sad_query_points");
    }
    SAD_REQUIRE(rec && aligned16(rec), SAD_ERR_INVALID_ARGUMENT, "sad_query_points: bad rec");
    const ImgArgs a = img_args(img);
    const float4 *r4 = reinterpret_cast<const float4 *>(rec);
    const uint4 *l4 = reinterpret_cast<const uint4 *>(topk);
    const float2 *p2 = reinterpret_cast<const float2 *>(xy);
    const unsigned nb = (unsigned)((M + 255) / 256);
    SAD_K_SWITCH(img->K, hipLaunchKernelGGL(k_query<KK>, dim3(nb), dim3(256), 0, st, a, r4, l4, p2, M,
                                            out));
    return check_launch("sad_query_points");
}

extern "C" sad_status sad_query_batch(const sad_query_job *jobs, int32_t n_jobs, int64_t total,
                                      int32_t K, void *stream) {
    SAD_REQUIRE(n_jobs >= 0 && total >= 0, SAD_ERR_INVALID_ARGUMENT, "sad_query_batch: negative count");
    if (n_jobs == 0 || total == 0) return SAD_OK;
    SAD_REQUIRE(jobs, SAD_ERR_INVALID_ARGUMENT, "sad_query_batch: jobs is NULL");
    SAD_REQUIRE(K >= 4 && K <= SAD_MAX_K && (K & 3) == 0, SAD_ERR_UNSUPPORTED,
                "sad_query_batch: K = %d unsupported", K);
    SAD_REQUIRE(total <= ((int64_t)1 << 31) * 255, SAD_ERR_INVALID_ARGUMENT, "sad_query_batch: too many points");
    const unsigned nb = (unsigned)((total + 255) / 256);
    hipStream_t st = as_stream(stream);
    SAD_K_SWITCH(K, hipLaunchKernelGGL(k_query_batch<KK>, dim3(nb), dim3(256), 0, st, jobs, n_jobs, total));
    return check_launch("sad_query_batch");
}
