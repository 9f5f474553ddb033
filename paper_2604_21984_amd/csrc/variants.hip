// variants.hip -- the paper's variants of the method: tau diffusion (App. B.6, a per-site
// Jacobi smoothing of the log tau gradient over each site's candidate list) and the
// one-dimensional SAD (Sec. 7 "1D Signal Fitting": the same soft partition on a line).
#include <cmath>

#include "sad_device.h"
#include "sad_host.h"
#include "sad_internal.h"
#include "sad_kernels.h"

namespace sad {

// ---- tau diffusion ---------------------------------------------------------------------
// Site i (valid record) reads the list of the pixel nearest its centre, averages g_in
// over the valid entries other than itself and mixes: g_out = (1 - lambda) g_in +
// lambda mean; without such entries (or for an invalid record) g_out = g_in.  Element i
// of a gradient array is at g[i * stride].
__global__ __launch_bounds__(256) void k_tau_diffusion(int H, int W, int n, const float4 *__restrict__ rec,
                                                       const uint4 *__restrict__ topk, int K,
                                                       const float *__restrict__ g_in,
                                                       int64_t in_stride, float lambda,
                                                       float *__restrict__ g_out,
                                                       int64_t out_stride) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float gi = g_in[i * in_stride];
    const float4 q0 = rec[4 * i], q1 = rec[4 * i + 1];
    float res = gi;
    if (q1.w != 0.0f) {
        const float fi = rintf(q0.y), fj = rintf(q0.x);
        const int ii = fi < 0.f ? 0 : (fi > (float)(H - 1) ? H - 1 : (int)fi);
        const int jj = fj < 0.f ? 0 : (fj > (float)(W - 1) ? W - 1 : (int)fj);
        const int64_t P = (int64_t)H * W, p = (int64_t)ii * W + jj;
        float sum = 0.0f;
        int cnt = 0;
        for (int g = 0; g < K / 4; ++g) {
            const uint4 v = topk[(int64_t)g * P + p];
            const uint32_t id[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                const uint32_t j = id[c];
                if (j >= (uint32_t)n || (int64_t)j == i) continue;
                if (rec[4 * (size_t)j + 1].w == 0.0f) continue;
                sum += g_in[(int64_t)j * in_stride];
                ++cnt;
            }
        }
        if (cnt) res = fmaf(lambda, sum / (float)cnt, (1.0f - lambda) * gi);
    }
    g_out[i * out_stride] = res;
}

// ---- one-dimensional SAD ---------------------------------------------------------------
// Derived record of a 1-D site: {p, r, kappa, c}, kappa = f32(exp(double log_tau)) * s,
// and kappa = 0 marks an inactive or invalid site (kappa must be finite and > 0).
__global__ __launch_bounds__(256) void k1_prepare(const float *__restrict__ sites, int64_t cap,
                                                  int n, float s, float4 *__restrict__ rec) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float p = sites[i], c = sites[cap + i], lt = sites[2 * cap + i], r = sites[3 * cap + i];
    float kappa = 0.0f;
    if (p >= 0.0f && isfinite(p) && isfinite(c) && isfinite(lt) && isfinite(r)) {
        kappa = __fmul_rn((float)exp((double)lt), s);
        if (!(kappa > 0.0f) || !isfinite(kappa)) kappa = 0.0f;
    }
    rec[i] = make_float4(p, r, kappa, c);
}

// l = kappa (r - |X - p|) + 0, each step one correctly rounded float32 operation.
__device__ __forceinline__ float score1(const float4 q, float X) {
    const float n = fabsf(__fsub_rn(X, q.x));
    return __fadd_rn(__fmul_rn(q.z, __fsub_rn(q.y, n)), 0.0f);
}

__device__ __forceinline__ uint64_t key1(const float4 *__restrict__ rec, uint32_t ns, uint32_t id,
                                         float X) {
    if (id >= ns) return 0ull;
    const float4 q = rec[id];
    return q.z > 0.0f ? make_key(score1(q, X), id) : 0ull;
}

__global__ __launch_bounds__(256) void k_fill_planes1(uint32_t *__restrict__ p, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = SAD_INVALID_ID;
}

__global__ __launch_bounds__(256) void k1_fill(uint64_t *__restrict__ p, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0ull;
}

__device__ __forceinline__ int seed_sample(float p, int M) {
    const float f = rintf(p);
    return f > (float)(M - 1) ? M - 1 : (f < 0.f ? 0 : (int)f);
}

__device__ __forceinline__ bool placed1(const uint32_t *__restrict__ topk, int64_t M, int m, int round,
                                        uint32_t i) {
    for (int k = 0; k < round; ++k)
        if (topk[((int64_t)(k >> 2) * M + m) * 4 + (k & 3)] == i) return true;
    return false;
}

// Round r of the 1-D seed pass: bids with a 64-bit atomic max, then the winner of each
// sample takes entry r (as the 2-D seed pass).
__global__ __launch_bounds__(256) void k1_seed_bid(const float4 *__restrict__ rec, int n, int M,
                                                   int round, const uint32_t *__restrict__ topk,
                                                   unsigned long long *__restrict__ best) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float4 q = rec[i];
    if (!(q.z > 0.0f)) return;
    const int m = seed_sample(q.x, M);
    if (placed1(topk, M, m, round, (uint32_t)i)) return;
    atomicMax(best + m, (unsigned long long)make_key(score1(q, (float)m), (uint32_t)i));
}

__global__ __launch_bounds__(256) void k1_seed_take(const float4 *__restrict__ rec, int n, int M,
                                                    int round, uint32_t *__restrict__ topk,
                                                    unsigned long long *__restrict__ best) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float4 q = rec[i];
    if (!(q.z > 0.0f)) return;
    const int m = seed_sample(q.x, M);
    if (placed1(topk, M, m, round, (uint32_t)i)) return;
    if (best[m] == (unsigned long long)make_key(score1(q, (float)m), (uint32_t)i)) {
        topk[((int64_t)(round >> 2) * M + m) * 4 + (round & 3)] = (uint32_t)i;
        best[m] = 0ull;
    }
}

// One Jacobi pass on the line: own list, the lists at m +- jump inside [0, M), and J
// injected IDs (SplitMix64 output (pass M + m) J + j, ID = hi32 n_slots / 2^32); the top
// K distinct IDs by (score descending, ID ascending).
template <int K>
__global__ __launch_bounds__(256) void k1_prop(int M, int n_slots, const float4 *__restrict__ rec,
                                               const uint4 *__restrict__ lin,
                                               uint4 *__restrict__ lout, int jump, int J,
                                               uint64_t seed, uint64_t pass) {
    const int m = blockIdx.x * blockDim.x + threadIdx.x;
    if (m >= M) return;
    const float X = (float)m;
    const uint32_t ns = (uint32_t)n_slots;
    uint64_t keys[K];
#pragma unroll
    for (int k = 0; k < K; ++k) keys[k] = 0ull;
    const int src[3] = {m, m + jump, m - jump};
#pragma unroll 1
    for (int a = 0; a < 3; ++a) {
        if (src[a] < 0 || src[a] >= M) continue;
#pragma unroll
        for (int g = 0; g < K / 4; ++g) {
            const uint4 v = lin[(int64_t)g * M + src[a]];
            insert_key<K>(keys, key1(rec, ns, v.x, X));
            insert_key<K>(keys, key1(rec, ns, v.y, X));
            insert_key<K>(keys, key1(rec, ns, v.z, X));
            insert_key<K>(keys, key1(rec, ns, v.w, X));
        }
    }
    const uint64_t k0 = (pass * (uint64_t)M + (uint64_t)m) * (uint64_t)J;
#pragma unroll 1
    for (int j = 0; j < J; ++j) {
        const uint64_t hi = splitmix64(seed, k0 + (uint64_t)j) >> 32;
        insert_key<K>(keys, key1(rec, ns, (uint32_t)((hi * (uint64_t)ns) >> 32), X));
    }
#pragma unroll
    for (int g = 0; g < K / 4; ++g)
        lout[(int64_t)g * M + m] = make_uint4(key_id(keys[4 * g]), key_id(keys[4 * g + 1]),
                                              key_id(keys[4 * g + 2]), key_id(keys[4 * g + 3]));
}

// Blend of every sample, and with a target its loss (added to loss->part, folded
// separately) and the gradients for dL/dc = (2/M)(c - I) accumulated into grad[4][cap]:
// dc += w g; gamma = w g (c_k - c); dlog_tau += gamma l; dr += gamma kappa;
// dp += gamma kappa sign(x - p) (0 at x = p).  c_k - c is formed relative to the best
// entry, as in the 2-D backward.
template <int K>
__global__ __launch_bounds__(256) void k1_render(int M, int n_slots, int64_t cap,
                                                 const float4 *__restrict__ rec,
                                                 const uint4 *__restrict__ topk,
                                                 const float *__restrict__ target,
                                                 float *__restrict__ out, float *__restrict__ grad,
                                                 sad_loss_acc *__restrict__ loss, FixScale fx) {
    // The 256 samples of a block share few sites: their gradient terms meet in a block
    // table keyed by site ID (64-bit fixed point in units of 2^-(40 + e), 2^e ~ M / 2:
    // finer than the image table's unit, since a 1-D site's gradient is a sum of few
    // small terms; a term below 2^51 units converts exactly and 256 of them stay below
    // 2^59), flushed with one float atomic per (site, parameter); a term the table
    // cannot take goes straight to global memory.
    __shared__ uint32_t hkey[kHashSlots];
    __shared__ unsigned long long hacc[4][kHashSlots];
    const bool tab = grad != nullptr;   // the same for the whole launch
    if (tab) {
        hkey[threadIdx.x] = SAD_INVALID_ID;
#pragma unroll
        for (int q = 0; q < 4; ++q) hacc[q][threadIdx.x] = 0ull;
        __syncthreads();
    }
    const int m = blockIdx.x * blockDim.x + threadIdx.x;
    float sq = 0.0f;
    if (m < M) {
        const float X = (float)m;
        const uint32_t ns = (uint32_t)n_slots;
        uint32_t id[K];
        float l[K], col[K];
        bool ok[K];
        float mx = -INFINITY;
        int nv = 0;
#pragma unroll
        for (int g = 0; g < K / 4; ++g) {
            const uint4 v = topk[(int64_t)g * M + m];
            id[4 * g] = v.x;
            id[4 * g + 1] = v.y;
            id[4 * g + 2] = v.z;
            id[4 * g + 3] = v.w;
        }
#pragma unroll
        for (int k = 0; k < K; ++k) {
            const uint32_t idc = id[k] < ns ? id[k] : 0u;
            const float4 q = ns ? rec[idc] : make_float4(0.f, 0.f, 0.f, 0.f);
            ok[k] = id[k] < ns && q.z > 0.0f;
            l[k] = score1(q, X);
            col[k] = q.w;
            id[k] = idc;
            if (ok[k]) {
                mx = fmaxf(mx, l[k]);
                ++nv;
            }
        }
        int r = 0;
#pragma unroll
        for (int k = K - 1; k >= 0; --k)
            if (ok[k] && l[k] == mx) r = k;
        float cr = 0.0f;
#pragma unroll
        for (int k = 0; k < K; ++k)
            if (k == r) cr = col[k];
        float e[K], S = 0.0f, d = 0.0f;
#pragma unroll
        for (int k = 0; k < K; ++k) {
            e[k] = ok[k] ? __expf(l[k] - mx) : 0.0f;
            S += e[k];
            d = fmaf(e[k], col[k] - cr, d);
        }
        const float inv = nv ? 1.0f / S : 0.0f;
        const float dc = d * inv;             // c - c_r
        const float c = nv ? cr + dc : 0.0f;
        if (out) out[m] = c;
        if (target) {
            const float res = c - target[m];
            sq = res * res;
            if (grad) {
                // dL/dc pre-scaled by 2^(40 + e): every term below arrives in table units
                const float gm = (2.0f * res / (float)M) * fx.pre;
#pragma unroll
                for (int k = 0; k < K; ++k) {
                    const float w = e[k] * inv;
                    // all four terms are multiples of w: weight 0 adds exactly 0
                    if (!ok[k] || w == 0.0f) continue;
                    const float4 q = rec[id[k]];
                    const float gam = w * gm * ((col[k] - cr) - dc);
                    const float dx = X - q.x;
                    const float sg = dx > 0.0f ? 1.0f : (dx < 0.0f ? -1.0f : 0.0f);
                    const float t[4] = {gam * q.z * sg, w * gm, gam * l[k], gam * q.z};
                    const int slot = hash_slot(hkey, id[k]);
                    const float asum = fabsf(t[0]) + fabsf(t[1]) + fabsf(t[2]) + fabsf(t[3]);
                    if (slot >= 0 && asum < 0x1p51f) {
#pragma unroll
                        for (int c = 0; c < 4; ++c) atomicAdd(&hacc[c][slot], rint_i64(t[c]));
                    } else {
#pragma unroll
                        for (int c = 0; c < 4; ++c)
                            if (t[c] != 0.0f) atomic_add_f32(grad + c * cap + id[k], t[c] * fx.post);
                    }
                }
            }
        }
    }
    if (tab) {
        __syncthreads();
        const uint32_t sid = hkey[threadIdx.x];
        if (sid != SAD_INVALID_ID) {
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                const unsigned long long u = hacc[c][threadIdx.x];
                if (u) atomic_add_f32(grad + c * cap + sid, from_fixed(u, fx.from_fix));
            }
        }
    }
    if (!loss || !target) return;
    const float t = block_sum(sq);
    if (threadIdx.x == 0) atomic_add_f32(&loss->part[blockIdx.x % SAD_LOSS_PARTS], t / (float)M);
}

// Adam on the four parameters (bias-corrected, step t >= 1), then p in [0, M-1], log_tau
// in [2, 20], r in [1, 512]; inactive slots untouched.
__global__ __launch_bounds__(256) void k1_adam(float *__restrict__ sites, const float *__restrict__ grad,
                                               float *__restrict__ mom, float *__restrict__ vel,
                                               int64_t cap, int n, int M, float4 lr, float b1,
                                               float b2, float eps, int64_t t) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    float x[4];
    bool act = true;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        x[q] = sites[q * cap + i];
        act = act && isfinite(x[q]);
    }
    if (!act || !(x[0] >= 0.0f)) return;
    const float bc1 = (float)(1.0 - pow((double)b1, (double)t));
    const float bc2 = (float)(1.0 - pow((double)b2, (double)t));
    const float lrs[4] = {lr.x, lr.y, lr.z, lr.w};
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int64_t o = q * cap + i;
        const float g = grad[o];
        const float mq = b1 * mom[o] + (1.0f - b1) * g;
        const float vq = b2 * vel[o] + (1.0f - b2) * g * g;
        mom[o] = mq;
        vel[o] = vq;
        x[q] -= lrs[q] * (mq / bc1) / (sqrtf(vq / bc2) + eps);
    }
    x[0] = fminf(fmaxf(x[0], 0.0f), (float)(M - 1));
    x[2] = fminf(fmaxf(x[2], 2.0f), 20.0f);
    x[3] = fminf(fmaxf(x[3], 1.0f), 512.0f);
#pragma unroll
    for (int q = 0; q < 4; ++q) sites[q * cap + i] = x[q];
}

__global__ __launch_bounds__(64) void k1_loss_fold(sad_loss_acc *__restrict__ loss) {
    const int i = threadIdx.x;
    float v = i < SAD_LOSS_PARTS ? loss->part[i] : 0.f;
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    if (i < SAD_LOSS_PARTS) loss->part[i] = 0.f;
    if (i == 0) loss->value += v;
}

static unsigned nblk(int64_t n) { return (unsigned)((n + 255) / 256); }

static sad_status check_signal(const sad_signal *sg, float *s_eff) {
    SAD_REQUIRE(sg, SAD_ERR_INVALID_ARGUMENT, "signal descriptor is NULL");
    SAD_REQUIRE(sg->M >= 1 && sg->M <= (1 << 30), SAD_ERR_INVALID_ARGUMENT, "bad sample count %d",
                sg->M);
    SAD_REQUIRE(sg->K >= 4 && sg->K <= SAD_MAX_K && (sg->K & 3) == 0, SAD_ERR_UNSUPPORTED,
                "K = %d unsupported (multiple of 4 in [4, %d])", sg->K, SAD_MAX_K);
    SAD_REQUIRE(sg->n_slots >= 0 && sg->cap >= sg->n_slots && sg->cap <= ((int64_t)1 << 31),
                SAD_ERR_INVALID_ARGUMENT, "bad slot counts n_slots = %d, cap = %lld", sg->n_slots,
                (long long)sg->cap);
    float s = sg->score_scale == 0.0f ? 1.0f / (float)sg->M : sg->score_scale;
    SAD_REQUIRE(s > 0.0f && s < 3.0e38f, SAD_ERR_INVALID_ARGUMENT, "bad score scale %g",
                (double)sg->score_scale);
    if (s_eff) *s_eff = s;
    return SAD_OK;
}

}  // namespace sad

using namespace sad;

extern "C" sad_status sad_tau_diffusion(const sad_image *img, const float *rec,
                                        const uint32_t *topk, const float *g_in,
                                        int64_t in_stride, float lambda, float *g_out,
                                        int64_t out_stride, void *stream) {
    SAD_TRY(check_image(img, nullptr));
    if (img->n_slots == 0) return SAD_OK;
    SAD_REQUIRE(rec && topk && g_in && g_out, SAD_ERR_INVALID_ARGUMENT,
                "sad_tau_diffusion: NULL pointer");
    SAD_REQUIRE(aligned16(rec) && aligned16(topk), SAD_ERR_INVALID_ARGUMENT,
                "sad_tau_diffusion: rec / topk not 16-byte aligned");
    SAD_REQUIRE(in_stride >= 1 && out_stride >= 1, SAD_ERR_INVALID_ARGUMENT,
                "sad_tau_diffusion: strides must be >= 1");
    SAD_REQUIRE(g_in != g_out, SAD_ERR_INVALID_ARGUMENT,
                "sad_tau_diffusion: g_in and g_out must not alias (Jacobi step)");
    SAD_REQUIRE(lambda >= 0.0f && lambda <= 1.0f, SAD_ERR_INVALID_ARGUMENT,
                "sad_tau_diffusion: lambda must be in [0, 1]");
    hipLaunchKernelGGL(k_tau_diffusion, dim3(nblk(img->n_slots)), dim3(256), 0, as_stream(stream),
                       img->H, img->W, img->n_slots, reinterpret_cast<const float4 *>(rec),
                       reinterpret_cast<const uint4 *>(topk), img->K, g_in, in_stride, lambda,
                       g_out, out_stride);
    return check_launch("sad_tau_diffusion");
}

extern "C" sad_status sad1d_prepare(const sad_signal *sg, const float *sites, float *rec,
                                    void *stream) {
    float s;
    SAD_TRY(check_signal(sg, &s));
    if (sg->n_slots == 0) return SAD_OK;
    SAD_REQUIRE(sites && rec && aligned16(rec), SAD_ERR_INVALID_ARGUMENT,
                "sad1d_prepare: NULL pointer or rec not 16-byte aligned");
    hipLaunchKernelGGL(k1_prepare, dim3(nblk(sg->n_slots)), dim3(256), 0, as_stream(stream), sites,
                       sg->cap, sg->n_slots, s, reinterpret_cast<float4 *>(rec));
    return check_launch("sad1d_prepare");
}

extern "C" sad_status sad1d_seed(const sad_signal *sg, const float *rec, uint32_t *topk,
                                 uint64_t *scratch, void *stream) {
    SAD_TRY(check_signal(sg, nullptr));
    SAD_REQUIRE(topk && scratch && (rec || sg->n_slots == 0), SAD_ERR_INVALID_ARGUMENT,
                "sad1d_seed: NULL pointer");
    hipStream_t st = as_stream(stream);
    const int64_t nl = (int64_t)sg->M * sg->K;
    hipLaunchKernelGGL(k_fill_planes1, dim3(nblk(nl)), dim3(256), 0, st, topk, nl);
    const int n = sg->n_slots;
    if (n > 0) {
        hipLaunchKernelGGL(k1_fill, dim3(nblk(sg->M)), dim3(256), 0, st, scratch, (int64_t)sg->M);
        const float4 *r4 = reinterpret_cast<const float4 *>(rec);
        auto *best = reinterpret_cast<unsigned long long *>(scratch);
        for (int round = 0; round < sg->K; ++round) {
            hipLaunchKernelGGL(k1_seed_bid, dim3(nblk(n)), dim3(256), 0, st, r4, n, sg->M, round,
                               topk, best);
            hipLaunchKernelGGL(k1_seed_take, dim3(nblk(n)), dim3(256), 0, st, r4, n, sg->M, round,
                               topk, best);
        }
    }
    return check_launch("sad1d_seed");
}

extern "C" sad_status sad1d_propagate(const sad_signal *sg, const float *rec,
                                      const uint32_t *topk_in, uint32_t *topk_out, int32_t jump,
                                      int32_t n_inject, uint64_t seed, uint64_t pass_index,
                                      void *stream) {
    SAD_TRY(check_signal(sg, nullptr));
    SAD_REQUIRE(topk_in && topk_out && topk_in != topk_out, SAD_ERR_INVALID_ARGUMENT,
                "sad1d_propagate: NULL or aliasing lists (Jacobi pass)");
    SAD_REQUIRE(aligned16(topk_in) && aligned16(topk_out), SAD_ERR_INVALID_ARGUMENT,
                "sad1d_propagate: lists must be 16-byte aligned");
    SAD_REQUIRE(jump >= 1 && jump <= (1 << 30) && n_inject >= 0 && n_inject <= 16,
                SAD_ERR_INVALID_ARGUMENT,
                "sad1d_propagate: 1 <= jump <= 2^30 and 0 <= n_inject <= 16");
    hipStream_t st = as_stream(stream);
    if (sg->n_slots == 0) {
        const int64_t nl = (int64_t)sg->M * sg->K;
        hipLaunchKernelGGL(k_fill_planes1, dim3(nblk(nl)), dim3(256), 0, st, topk_out, nl);
        return check_launch("sad1d_propagate");
    }
    SAD_REQUIRE(rec && aligned16(rec), SAD_ERR_INVALID_ARGUMENT,
                "sad1d_propagate: rec NULL or not 16-byte aligned");
    const float4 *r4 = reinterpret_cast<const float4 *>(rec);
    const uint4 *li = reinterpret_cast<const uint4 *>(topk_in);
    uint4 *lo = reinterpret_cast<uint4 *>(topk_out);
    SAD_K_SWITCH(sg->K, hipLaunchKernelGGL((k1_prop<KK>), dim3(nblk(sg->M)), dim3(256), 0, st,
                                           sg->M, sg->n_slots, r4, li, lo, jump, n_inject, seed,
                                           pass_index));
    return check_launch("sad1d_propagate");
}

extern "C" sad_status sad1d_render(const sad_signal *sg, const float *rec, const uint32_t *topk,
                                   const float *target, float *out, float *grad,
                                   sad_loss_acc *loss, void *stream) {
    SAD_TRY(check_signal(sg, nullptr));
    SAD_REQUIRE(topk && aligned16(topk), SAD_ERR_INVALID_ARGUMENT,
                "sad1d_render: topk NULL or not 16-byte aligned");
    SAD_REQUIRE(target || (!grad && !loss), SAD_ERR_INVALID_ARGUMENT,
                "sad1d_render: grad and loss need the target");
    hipStream_t st = as_stream(stream);
    SAD_REQUIRE(sg->n_slots == 0 || (rec && aligned16(rec)), SAD_ERR_INVALID_ARGUMENT,
                "sad1d_render: rec NULL or not 16-byte aligned");
    const float4 *r4 = reinterpret_cast<const float4 *>(rec);
    const uint4 *t4 = reinterpret_cast<const uint4 *>(topk);
    const int ns = sg->n_slots;
    const bool g = grad && ns > 0;
    FixScale fx = fix_scale(sg->M);   // the 1-D table's finer unit 2^-(40 + e)
    const int e = fix_exponent(sg->M);
    fx.pre = std::ldexp(1.0f, 40 + e);
    fx.post = std::ldexp(1.0f, -(40 + e));
    fx.from_fix = std::ldexp(1.0, -(40 + e));
    SAD_K_SWITCH(sg->K, hipLaunchKernelGGL((k1_render<KK>), dim3(nblk(sg->M)), dim3(256), 0, st,
                                           sg->M, ns, sg->cap, r4, t4, target, out,
                                           g ? grad : nullptr, loss, fx));
    if (loss) hipLaunchKernelGGL(k1_loss_fold, dim3(1), dim3(64), 0, st, loss);
    return check_launch("sad1d_render");
}

extern "C" sad_status sad1d_adam(const sad_signal *sg, float *sites, const float *grad, float *m,
                                 float *v, const float *lr /* host [4] */, float beta1,
                                 float beta2, float eps, int64_t step, void *stream) {
    SAD_TRY(check_signal(sg, nullptr));
    SAD_REQUIRE(step >= 1, SAD_ERR_INVALID_ARGUMENT, "sad1d_adam: step must be >= 1");
    if (sg->n_slots == 0) return SAD_OK;
    SAD_REQUIRE(sites && grad && m && v && lr, SAD_ERR_INVALID_ARGUMENT,
                "sad1d_adam: NULL pointer");
    const float4 lr4 = make_float4(lr[0], lr[1], lr[2], lr[3]);
    hipLaunchKernelGGL(k1_adam, dim3(nblk(sg->n_slots)), dim3(256), 0, as_stream(stream), sites,
                       grad, m, v, sg->cap, sg->n_slots, sg->M, lr4, beta1, beta2, eps, step);
    return check_launch("sad1d_adam");
}
