// render.hip -- forward blend (Sec. 4.2), loss gradient (Sec. 6.1), backward scatter
// with per-tile LDS pre-reduction (App. B.4, Sec. 4.8), point queries (Sec. 6.6).
#include <cmath>

#include "sad_device.h"
#include "sad_host.h"
#include "sad_internal.h"

namespace sad {

struct ImgArgs {
    int H, W, n_slots, tiles_x, n_blocks;
    int64_t cap;
    float inv_P;
};

// Valid entries of one pixel's list with their scores (K registers each).
template <int K>
struct PixelBlend {
    uint32_t id[K];
    float l[K];
    float e[K];
    bool ok[K];
    float S, c[3];
    int nv;
};

// Gather and score the list of pixel p at point (X, Y); max-subtracted softmax; colour.
// Rotate ids[] left by `rot` (0 <= rot < 8) with three conditional stages.  Used by the
// backward so that neighbouring lanes work on different ranks of their (similar) lists
// in the same instruction, which spreads their LDS atomics over different sites.
template <int K>
__device__ __forceinline__ void rotate_ids(uint32_t (&ids)[K], int rot) {
#pragma unroll
    for (int st = 1; st < 8 && st < K; st <<= 1) {
        const bool c = (rot & st) != 0;
        uint32_t t[K];
#pragma unroll
        for (int j = 0; j < K; ++j) t[j] = c ? ids[(j + st) % K] : ids[j];
#pragma unroll
        for (int j = 0; j < K; ++j) ids[j] = t[j];
    }
}

template <int K, bool kNeedN>
__device__ __forceinline__ void blend(const float4 *__restrict__ rec, uint32_t ns,
                                      const uint4 *__restrict__ topk, int64_t P, int64_t p,
                                      float X, float Y, PixelBlend<K> &b, float (*col)[3],
                                      float *nrm, int rot = 0) {
    float m = -INFINITY;
    b.nv = 0;
    uint32_t ids[K];
#pragma unroll
    for (int g = 0; g < K / 4; ++g) {
        const uint4 v = topk[(int64_t)g * P + p];
        ids[4 * g] = v.x;
        ids[4 * g + 1] = v.y;
        ids[4 * g + 2] = v.z;
        ids[4 * g + 3] = v.w;
    }
    if (rot) rotate_ids<K>(ids, rot);
#pragma unroll
    for (int g = 0; g < K / 4; ++g) {
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            const int k = 4 * g + t;
            const uint32_t id = ids[k];
            const bool in_range = id < ns;
            const uint32_t idc = in_range ? id : 0u;
            const float4 q0 = rec[4 * (size_t)idc], q1 = rec[4 * (size_t)idc + 1];
            const float4 q2 = rec[4 * (size_t)idc + 2];
            b.id[k] = idc;
            b.ok[k] = in_range && q1.w != 0.0f;
            float n;
            b.l[k] = score(q0, q1, X, Y, &n);
            if (kNeedN) nrm[k] = n;
            col[k][0] = q2.x;
            col[k][1] = q2.y;
            col[k][2] = q2.z;
            if (b.ok[k]) {
                m = fmaxf(m, b.l[k]);
                ++b.nv;
            }
        }
    }
    b.S = 0.f;
    b.c[0] = b.c[1] = b.c[2] = 0.f;
#pragma unroll
    for (int k = 0; k < K; ++k) {
        b.e[k] = b.ok[k] ? __expf(b.l[k] - m) : 0.0f;
        b.S += b.e[k];
        b.c[0] = fmaf(b.e[k], col[k][0], b.c[0]);
        b.c[1] = fmaf(b.e[k], col[k][1], b.c[1]);
        b.c[2] = fmaf(b.e[k], col[k][2], b.c[2]);
    }
    if (b.nv) {
        const float inv = __builtin_amdgcn_rcpf(b.S);
        b.c[0] *= inv;
        b.c[1] *= inv;
        b.c[2] *= inv;
    }
}

template <int K>
__global__ __launch_bounds__(256) void k_fwd(ImgArgs a, const float4 *__restrict__ rec,
                                             const uint4 *__restrict__ topk,
                                             float *__restrict__ out) {
    const int tile = xcd_tile(blockIdx.x, a.n_blocks);
    const TilePix px = tile_pixel(tile, a.tiles_x);
    if (px.i >= a.H || px.j >= a.W) return;
    const int64_t P = (int64_t)a.H * a.W, p = (int64_t)px.i * a.W + px.j;
    PixelBlend<K> b;
    float col[K][3];
    blend<K, false>(rec, (uint32_t)a.n_slots, topk, P, p, (float)px.j, (float)px.i, b, col,
                    nullptr);
    out[p] = b.c[0];
    out[P + p] = b.c[1];
    out[2 * P + p] = b.c[2];
}

// dL/dc = (2/P)(c - I); loss += (1/P) sum (c - I)^2.  Grid-stride over a bounded
// number of blocks, one atomic per block (a single address takes every block's atomic).
__device__ __forceinline__ float block_sum(float v) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    __shared__ float part[4];
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = v;
    __syncthreads();
    const float r = (part[0] + part[1]) + (part[2] + part[3]);
    __syncthreads();
    return r;
}

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
        float col[K][3];
        blend<K, false>(rec, (uint32_t)a.n_slots, topk, P, p, (float)px.j, (float)px.i, b, col,
                        nullptr);
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

// ---- backward ---------------------------------------------------------------------
// Per-tile hash table in LDS keyed by site ID (multiplicative hash, linear probing of
// at most 8 slots, CAS insert; Sec. 4.8, Alg. hash_grad, App. B.4).  Each (pixel,
// entry) contribution is added into its slot's accumulators.  On gfx950 LDS float
// atomics are slow even without address conflicts while integer atomics are fast, so
// the accumulators are 64-bit fixed point: a term v becomes rint(v * 2^40 * 2^e) with
// 2^e ~ P/2 (every term carries the 1/P of dL/dc).  Terms with |v| 2^e >= 2^15 go to
// a float global atomic instead, so a tile sum (<= 256 terms per slot) stays below
// 2^63.  After the tile, each occupied slot is flushed with one float global atomic
// per parameter.
constexpr int kHashSlots = 256;
constexpr int kProbes = 8;
constexpr int kAcc = 11;  // 10 parameters + removal delta

struct FixScale {
    double to_fix;     // 2^(40 + e)
    double from_fix;   // 2^-(40 + e)
    float limit;       // |v| must be below 2^(15 - e)
};

__device__ __forceinline__ unsigned long long to_fixed(float v, double scale) {
    const double x = rint((double)v * scale);
    const double hi = floor(x * 0x1p-32);
    const double lo = fma(hi, -0x1p32, x);  // exact, in [0, 2^32)
    return ((unsigned long long)(uint32_t)(int32_t)hi << 32) | (uint32_t)lo;
}

__device__ __forceinline__ float from_fixed(unsigned long long u, double inv_scale) {
    const double hi = (double)(int32_t)(uint32_t)(u >> 32);
    const double lo = (double)(uint32_t)u;
    return (float)(fma(hi, 0x1p32, lo) * inv_scale);
}

__device__ __forceinline__ int hash_slot(uint32_t *__restrict__ hkey, uint32_t id) {
    const uint32_t h = (id * 2654435761u) >> 24;
#pragma unroll 1
    for (int pr = 0; pr < kProbes; ++pr) {
        const uint32_t s = (h + pr) & (kHashSlots - 1);
        uint32_t k = hkey[s];
        if (k == id) return (int)s;
        if (k == SAD_INVALID_ID) {
            k = atomicCAS(&hkey[s], SAD_INVALID_ID, id);
            if (k == SAD_INVALID_ID || k == id) return (int)s;
        }
    }
    return -1;
}

template <int K, bool kRD>
__global__ __launch_bounds__(256) void k_bwd(ImgArgs a, FixScale fx, const float4 *__restrict__ rec,
                                             const uint4 *__restrict__ topk,
                                             const float *__restrict__ gimg,
                                             const float *__restrict__ tgt,
                                             float *__restrict__ grad, float *__restrict__ rdel) {
    __shared__ uint32_t hkey[kHashSlots];
    __shared__ unsigned long long hacc[kAcc][kHashSlots];
    const int t = threadIdx.x;
    hkey[t] = SAD_INVALID_ID;
#pragma unroll
    for (int q = 0; q < kAcc; ++q) hacc[q][t] = 0ull;
    __syncthreads();

    const int tile = xcd_tile(blockIdx.x, a.n_blocks);
    const TilePix px = tile_pixel(tile, a.tiles_x);
    if (px.i < a.H && px.j < a.W) {
        const int64_t P = (int64_t)a.H * a.W, p = (int64_t)px.i * a.W + px.j;
        const float X = (float)px.j, Y = (float)px.i;
        PixelBlend<K> b;
        float col[K][3];
        float nrm[K];
        const int lane = t & 63;
        const int rot = ((lane & 7) + 3 * (lane >> 3)) & 7;
        blend<K, true>(rec, (uint32_t)a.n_slots, topk, P, p, X, Y, b, col, nrm, rot % K);
        if (b.nv) {
            const float g0 = gimg[p], g1 = gimg[P + p], g2 = gimg[2 * P + p];
            const float invS = __builtin_amdgcn_rcpf(b.S);
            // Reference entry r: the largest score (e_r = 1).  Differences are formed
            // relative to it, so that nothing cancels when one weight is close to 1:
            //   c_k - c = (c_k - c_r) - dc_r,  dc_r = sum_j w_j (c_j - c_r).
            int r = 0;
            float mx = -INFINITY;
#pragma unroll
            for (int k = 0; k < K; ++k)
                if (b.ok[k] && b.l[k] > mx) {
                    mx = b.l[k];
                    r = k;
                }
            float cr0 = 0.f, cr1 = 0.f, cr2 = 0.f;
#pragma unroll
            for (int k = 0; k < K; ++k)
                if (k == r) {
                    cr0 = col[k][0];
                    cr1 = col[k][1];
                    cr2 = col[k][2];
                }
            float dc0 = 0.f, dc1 = 0.f, dc2 = 0.f;
#pragma unroll
            for (int k = 0; k < K; ++k) {
                const float w = b.e[k] * invS;  // 0 for invalid entries
                dc0 = fmaf(w, col[k][0] - cr0, dc0);
                dc1 = fmaf(w, col[k][1] - cr1, dc1);
                dc2 = fmaf(w, col[k][2] - cr2, dc2);
            }
            // removal delta (Sec. 4.5): Delta = (c' - c) . ((c' - c) + 2 (c - I))
            float e0 = 0.f, e1 = 0.f, e2 = 0.f;      // c - I
            float dr0 = 0.f, dr1 = 0.f, dr2 = 0.f;   // c'_r - c for the reference entry
            if (kRD) {
                e0 = b.c[0] - tgt[p];
                e1 = b.c[1] - tgt[P + p];
                e2 = b.c[2] - tgt[2 * P + p];
                if (b.nv > 1) {
                    float m2 = -INFINITY;
#pragma unroll
                    for (int k = 0; k < K; ++k)
                        if (b.ok[k] && k != r) m2 = fmaxf(m2, b.l[k]);
                    float S2 = 0.f, n0 = 0.f, n1 = 0.f, n2 = 0.f;
#pragma unroll
                    for (int k = 0; k < K; ++k) {
                        if (!b.ok[k] || k == r) continue;
                        const float ee = __expf(b.l[k] - m2);
                        S2 += ee;
                        n0 = fmaf(ee, col[k][0] - cr0, n0);
                        n1 = fmaf(ee, col[k][1] - cr1, n1);
                        n2 = fmaf(ee, col[k][2] - cr2, n2);
                    }
                    const float inv2 = __builtin_amdgcn_rcpf(S2);
                    dr0 = n0 * inv2 - dc0;
                    dr1 = n1 * inv2 - dc1;
                    dr2 = n2 * inv2 - dc2;
                } else {  // no other entry: the pixel would render 0
                    dr0 = -b.c[0];
                    dr1 = -b.c[1];
                    dr2 = -b.c[2];
                }
            }
#pragma unroll
            for (int k = 0; k < K; ++k) {
                if (!b.ok[k]) continue;
                const uint32_t id = b.id[k];
                const float4 q0 = rec[4 * (size_t)id], q1 = rec[4 * (size_t)id + 1];
                const float4 q2 = rec[4 * (size_t)id + 2], q3 = rec[4 * (size_t)id + 3];
                const float w = b.e[k] * invS;
                const float d0 = (col[k][0] - cr0) - dc0;  // c_k - c
                const float d1 = (col[k][1] - cr1) - dc1;
                const float d2 = (col[k][2] - cr2) - dc2;
                float acc[kAcc];
                acc[4] = w * g0;
                acc[5] = w * g1;
                acc[6] = w * g2;
                const float gam = w * (g0 * d0 + g1 * d1 + g2 * d2);
                acc[2] = gam * b.l[k];
                acc[3] = gam * q1.y;
                const float n = nrm[k];
                acc[0] = acc[1] = acc[7] = acc[8] = acc[9] = 0.f;
                if (n > 0.f) {
                    const float rho = -0.5f * gam * q1.y * __builtin_amdgcn_rcpf(n);
                    const float ux = q2.w, uy = q3.x, ep = q3.y, em = q3.z;
                    const float dx = X - q0.x, dy = Y - q0.y;
                    const float al = ux * dx + uy * dy, be = ux * dy - uy * dx;
                    const float A = ep * al, B = em * be;
                    acc[0] = -2.0f * rho * (A * ux - B * uy);
                    acc[1] = -2.0f * rho * (A * uy + B * ux);
                    acc[9] = rho * (A * al - B * be);
                    acc[7] = 2.0f * rho * (A * dx + B * dy);
                    acc[8] = 2.0f * rho * (A * dy - B * dx);
                }
                acc[10] = 0.f;
                if (kRD) {
                    float p0, p1, p2;  // c'_k - c
                    if (k == r) {
                        p0 = dr0;
                        p1 = dr1;
                        p2 = dr2;
                    } else {  // c' - c = -w / (1 - w) (c_k - c), with w <= 1/2 here
                        const float f = -w * __builtin_amdgcn_rcpf(1.0f - w);
                        p0 = f * d0;
                        p1 = f * d1;
                        p2 = f * d2;
                    }
                    acc[10] = (p0 * (p0 + 2.0f * e0) + p1 * (p1 + 2.0f * e1) +
                               p2 * (p2 + 2.0f * e2)) * a.inv_P;
                }
                const int slot = hash_slot(hkey, id);
                constexpr int nq = kRD ? kAcc : 10;
#pragma unroll
                for (int q = 0; q < nq; ++q) {
                    float *dst = q < 10 ? grad + q * a.cap + id : rdel + id;
                    if (slot >= 0 && fabsf(acc[q]) < fx.limit)
                        atomicAdd(&hacc[q][slot], to_fixed(acc[q], fx.to_fix));
                    else if (acc[q] != 0.0f)
                        atomic_add_f32(dst, acc[q]);
                }
            }
        }
    }
    __syncthreads();
    const uint32_t id = hkey[t];
    if (id != SAD_INVALID_ID) {
        constexpr int nq = kRD ? kAcc : 10;
#pragma unroll
        for (int q = 0; q < nq; ++q) {
            const unsigned long long u = hacc[q][t];
            if (u) atomic_add_f32(q < 10 ? grad + q * a.cap + id : rdel + id,
                                  from_fixed(u, fx.from_fix));
        }
    }
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
    float col[K][3];
    blend<K, false>(rec, (uint32_t)a.n_slots, topk, P, p, pt.x, pt.y, b, col, nullptr);
    out[3 * q] = b.c[0];
    out[3 * q + 1] = b.c[1];
    out[3 * q + 2] = b.c[2];
}

__global__ __launch_bounds__(256) void k_fill(float *__restrict__ p, int64_t n, float v) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

static ImgArgs img_args(const sad_image *img) {
    ImgArgs a;
    a.H = img->H;
    a.W = img->W;
    a.n_slots = img->n_slots;
    a.tiles_x = tiles_x(img);
    a.n_blocks = n_tiles(img);
    a.cap = img->cap;
    a.inv_P = 1.0f / (float)((double)img->H * img->W);
    return a;
}

#define SAD_K_SWITCH(KV, CALL)                           \
    switch (KV) {                                        \
        case 4: { constexpr int KK = 4; CALL; } break;   \
        case 8: { constexpr int KK = 8; CALL; } break;   \
        case 12: { constexpr int KK = 12; CALL; } break; \
        case 16: { constexpr int KK = 16; CALL; } break; \
        case 20: { constexpr int KK = 20; CALL; } break; \
        case 24: { constexpr int KK = 24; CALL; } break; \
        case 28: { constexpr int KK = 28; CALL; } break; \
        case 32: { constexpr int KK = 32; CALL; } break; \
        default: break;                                  \
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
    const int64_t P = (int64_t)img->H * img->W;
    int e = 0;
    while ((int64_t)1 << (e + 1) < P) ++e;  // 2^e ~ P / 2
    FixScale fx;
    fx.to_fix = std::ldexp(1.0, 40 + e);
    fx.from_fix = std::ldexp(1.0, -(40 + e));
    fx.limit = (float)std::ldexp(1.0, 15 - e);
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
