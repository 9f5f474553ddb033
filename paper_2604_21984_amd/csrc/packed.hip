// packed.hip -- the packed 16-byte inference record (App. B.2 "Packed storage for
// evaluation"): per-image quantisation parameters, packing, decoding to sites or straight
// to derived records, and rendering / point queries that read the packed records.
#include <cmath>

#include "sad_device.h"
#include "sad_host.h"
#include "sad_internal.h"
#include "sad_kernels.h"
#include "sad_sites.h"

namespace sad {

constexpr double kPi = 3.14159265358979323846264338327950288;

// Quantisation parameters: {log_tau min, scale, r min, scale, c_r min, scale, c_g min,
// scale, c_b min, scale}; read once per thread (uniform, cached).
struct PackQ {
    float v[SAD_NQPARAM];
};
__device__ __forceinline__ PackQ load_q(const float *__restrict__ q) {
    PackQ p;
#pragma unroll
    for (int k = 0; k < SAD_NQPARAM; ++k) p.v[k] = q[k];
    return p;
}

// The five quantised parameters in q order.
__device__ __forceinline__ int qpar(int k) { return k == 0 ? 2 : (k == 1 ? 3 : 3 + k - 1); }

// UNORM code of v over [mn, mn + sc] with `bits` bits: t = (v - mn) / sc clamped to
// [0, 1] (0 when sc = 0), code = rint(t (2^bits - 1)); each step one float32 operation.
__device__ __forceinline__ uint32_t unorm_code(float v, float mn, float sc, int bits) {
    const float maxq = (float)((1u << bits) - 1u);
    float t = sc > 0.0f ? __fdiv_rn(__fsub_rn(v, mn), sc) : 0.0f;
    if (!(t > 0.0f)) t = 0.0f;
    if (t > 1.0f) t = 1.0f;
    return (uint32_t)rintf(__fmul_rn(t, maxq));
}

// Decoded value of a UNORM code: mn + sc (code / (2^bits - 1)).
__device__ __forceinline__ float unorm_value(uint32_t code, float mn, float sc, int bits) {
    const float maxq = (float)((1u << bits) - 1u);
    return __fadd_rn(mn, __fmul_rn(sc, __fdiv_rn((float)code, maxq)));
}

__device__ __forceinline__ bool site_active(const float (&v)[SAD_NPARAM]) {
    bool act = v[0] >= 0.0f;
#pragma unroll
    for (int p = 0; p < SAD_NPARAM; ++p) act = act && isfinite(v[p]);
    return act;
}

// The four words of a site's record (an inactive site packs to zeros):
//   w0 = x code (15 bits over [0, W-1]) | y code << 15 (over [0, H-1]) | 1 << 31
//   w1 = c_r (11 bits) | c_g << 11 (11 bits) | c_b << 22 (10 bits)
//   w2 = log_tau (16 bits) | r << 16 (16 bits)
//   w3 = angle code of u (16-bit UNORM of atan2(u_y, u_x) over [-pi, pi]) | float16 a << 16
__device__ __forceinline__ uint4 pack_record(const float (&v)[SAD_NPARAM], const PackQ &q, int H,
                                             int W) {
    if (!site_active(v)) return make_uint4(0u, 0u, 0u, 0u);
    uint4 w;
    w.x = unorm_code(v[0], 0.0f, (float)(W - 1), 15) |
          (unorm_code(v[1], 0.0f, (float)(H - 1), 15) << 15) | 0x80000000u;
    w.y = unorm_code(v[4], q.v[4], q.v[5], 11) | (unorm_code(v[5], q.v[6], q.v[7], 11) << 11) |
          (unorm_code(v[6], q.v[8], q.v[9], 10) << 22);
    w.z = unorm_code(v[2], q.v[0], q.v[1], 16) | (unorm_code(v[3], q.v[2], q.v[3], 16) << 16);
    const double th = atan2((double)v[8], (double)v[7]);
    const double t = (th + kPi) / (2.0 * kPi);
    const uint32_t ang = (uint32_t)rint(t * 65535.0);
    const _Float16 ah = (_Float16)v[9];
    w.w = ang | ((uint32_t)__builtin_bit_cast(uint16_t, ah) << 16);
    return w;
}

// Parameters decoded from a record; without the active flag x = y = -1 and the rest 0.
__device__ __forceinline__ void unpack_record(uint4 w, const PackQ &q, int H, int W,
                                              float (&v)[SAD_NPARAM]) {
#pragma unroll
    for (int p = 0; p < SAD_NPARAM; ++p) v[p] = 0.0f;
    v[0] = v[1] = -1.0f;
    if (!(w.x & 0x80000000u)) return;
    v[0] = unorm_value(w.x & 0x7FFFu, 0.0f, (float)(W - 1), 15);
    v[1] = unorm_value((w.x >> 15) & 0x7FFFu, 0.0f, (float)(H - 1), 15);
    v[4] = unorm_value(w.y & 0x7FFu, q.v[4], q.v[5], 11);
    v[5] = unorm_value((w.y >> 11) & 0x7FFu, q.v[6], q.v[7], 11);
    v[6] = unorm_value(w.y >> 22, q.v[8], q.v[9], 10);
    v[2] = unorm_value(w.z & 0xFFFFu, q.v[0], q.v[1], 16);
    v[3] = unorm_value(w.z >> 16, q.v[2], q.v[3], 16);
    const double th = (double)(w.w & 0xFFFFu) / 65535.0 * (2.0 * kPi) - kPi;
    v[7] = (float)cos(th);
    v[8] = (float)sin(th);
    v[9] = (float)__builtin_bit_cast(_Float16, (uint16_t)(w.w >> 16));
}

// Order-preserving map of a float to uint32 (for min / max with integer atomics).
__device__ __forceinline__ uint32_t ordered(float f) {
    const uint32_t b = __float_as_uint(f);
    return b ^ ((uint32_t)((int32_t)b >> 31) | 0x80000000u);
}
__device__ __forceinline__ float unordered(uint32_t o) {
    return __uint_as_float((o & 0x80000000u) ? (o ^ 0x80000000u) : ~o);
}

// The quantisation parameters are reduced in place in the caller's q[10]: while the
// reduction runs, word 2k holds the ordered minimum and word 2k + 1 the ordered maximum
// of parameter k; the last kernel turns them into (min, max - min).
__global__ __launch_bounds__(64) void k_q_init(uint32_t *__restrict__ qw) {
    const int k = threadIdx.x;
    if (k < SAD_NQPARAM) qw[k] = (k & 1) ? 0u : 0xFFFFFFFFu;
}

__global__ __launch_bounds__(256) void k_q_reduce(const float *__restrict__ sites, int64_t cap,
                                                  int n, uint32_t *__restrict__ qw) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    float v[SAD_NPARAM];
    bool act = false;
    if (i < n) {
#pragma unroll
        for (int p = 0; p < SAD_NPARAM; ++p) v[p] = sites[p * cap + i];
        act = site_active(v);
    }
#pragma unroll
    for (int k = 0; k < SAD_NQPARAM / 2; ++k) {
        uint32_t mn = act ? ordered(v[qpar(k)]) : 0xFFFFFFFFu;
        uint32_t mx = act ? ordered(v[qpar(k)]) : 0u;
        for (int o = 32; o > 0; o >>= 1) {
            mn = min(mn, (uint32_t)__shfl_xor((int)mn, o));
            mx = max(mx, (uint32_t)__shfl_xor((int)mx, o));
        }
        if ((threadIdx.x & 63) == 0) {
            if (mn != 0xFFFFFFFFu) atomicMin(&qw[2 * k], mn);
            if (mx != 0u) atomicMax(&qw[2 * k + 1], mx);
        }
    }
}

__global__ __launch_bounds__(64) void k_q_finish(uint32_t *__restrict__ qw) {
    const int k = threadIdx.x;
    if (k >= SAD_NQPARAM / 2) return;
    const uint32_t omn = qw[2 * k], omx = qw[2 * k + 1];
    float mn = 0.0f, sc = 0.0f;
    if (omn != 0xFFFFFFFFu) {  // at least one active site
        mn = unordered(omn);
        sc = __fsub_rn(unordered(omx), mn);
    }
    float *q = reinterpret_cast<float *>(qw);
    q[2 * k] = mn;
    q[2 * k + 1] = sc;
}

__global__ __launch_bounds__(256) void k_pack(const float *__restrict__ sites, int64_t cap, int n,
                                              int H, int W, const float *__restrict__ qp,
                                              uint4 *__restrict__ packed) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const PackQ q = load_q(qp);
    float v[SAD_NPARAM];
#pragma unroll
    for (int p = 0; p < SAD_NPARAM; ++p) v[p] = sites[p * cap + i];
    packed[i] = pack_record(v, q, H, W);
}

__global__ __launch_bounds__(256) void k_unpack(const uint4 *__restrict__ packed, int n, int H,
                                                int W, const float *__restrict__ qp,
                                                float *__restrict__ sites, int64_t cap) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    float v[SAD_NPARAM];
    unpack_record(packed[i], load_q(qp), H, W, v);
#pragma unroll
    for (int p = 0; p < SAD_NPARAM; ++p) sites[p * cap + i] = v[p];
}

__global__ __launch_bounds__(256) void k_unpack_prepare(const uint4 *__restrict__ packed, int n,
                                                        int H, int W, const float *__restrict__ qp,
                                                        float s, float4 *__restrict__ rec) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    float v[SAD_NPARAM];
    unpack_record(packed[i], load_q(qp), H, W, v);
    record_of(v, i, s, rec);
}

// Record source of the blend that decodes each entry's packed record in place.
struct PackedSrc {
    const uint4 *__restrict__ packed;
    PackQ q;
    int H, W;
    float s;
    __device__ __forceinline__ void fetch(uint32_t id, float4 &q0, float4 &q1, float4 &q2) const {
        float v[SAD_NPARAM];
        unpack_record(packed[id], q, H, W, v);
        float4 q3;
        derive(v, s, q0, q1, q2, q3);
    }
};

template <int K>
__global__ __launch_bounds__(256) void k_fwd_packed(ImgArgs a, const uint4 *__restrict__ packed,
                                                    const float *__restrict__ qp, float s,
                                                    const uint4 *__restrict__ topk,
                                                    float *__restrict__ out) {
    const int tile = xcd_tile(blockIdx.x, a.n_blocks);
    const TilePix px = tile_pixel(tile, a.tiles_x);
    if (px.i >= a.H || px.j >= a.W) return;
    const PackedSrc src{packed, load_q(qp), a.H, a.W, s};
    const int64_t P = (int64_t)a.H * a.W, p = (int64_t)px.i * a.W + px.j;
    PixelBlend<K> b;
    blend_src<K, false>(src, (uint32_t)a.n_slots, topk, P, p, (float)px.j, (float)px.i, b,
                        lane_rot() % K);
    out[p] = b.c[0];
    out[P + p] = b.c[1];
    out[2 * P + p] = b.c[2];
}

template <int K>
__global__ __launch_bounds__(256) void k_query_packed(ImgArgs a, const uint4 *__restrict__ packed,
                                                      const float *__restrict__ qp, float s,
                                                      const uint4 *__restrict__ topk,
                                                      const float2 *__restrict__ xy, int64_t M,
                                                      float *__restrict__ out) {
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= M) return;
    const PackedSrc src{packed, load_q(qp), a.H, a.W, s};
    const float2 pt = xy[q];
    const float fi = rintf(pt.y), fj = rintf(pt.x);
    const int ii = !(fi > 0.f) ? 0 : (fi > (float)(a.H - 1) ? a.H - 1 : (int)fi);
    const int jj = !(fj > 0.f) ? 0 : (fj > (float)(a.W - 1) ? a.W - 1 : (int)fj);
    const int64_t P = (int64_t)a.H * a.W, p = (int64_t)ii * a.W + jj;
    PixelBlend<K> b;
    blend_src<K, false>(src, (uint32_t)a.n_slots, topk, P, p, pt.x, pt.y, b);
    out[3 * q] = b.c[0];
    out[3 * q + 1] = b.c[1];
    out[3 * q + 2] = b.c[2];
}

static unsigned blocks_of(int64_t n) { return (unsigned)((n + 255) / 256); }

}  // namespace sad

using namespace sad;

extern "C" sad_status sad_pack_qparams(const sad_image *img, const float *sites, float *q,
                                       void *stream) {
    SAD_TRY(check_image(img, nullptr));
    SAD_REQUIRE(q && (sites || img->n_slots == 0), SAD_ERR_INVALID_ARGUMENT,
                "sad_pack_qparams: NULL pointer");
    SAD_REQUIRE((reinterpret_cast<uintptr_t>(q) & 3u) == 0, SAD_ERR_INVALID_ARGUMENT,
                "sad_pack_qparams: q not 4-byte aligned");
    hipStream_t st = as_stream(stream);
    uint32_t *qw = reinterpret_cast<uint32_t *>(q);
    hipLaunchKernelGGL(k_q_init, dim3(1), dim3(64), 0, st, qw);
    if (img->n_slots > 0)
        hipLaunchKernelGGL(k_q_reduce, dim3(blocks_of(img->n_slots)), dim3(256), 0, st, sites,
                           img->cap, img->n_slots, qw);
    hipLaunchKernelGGL(k_q_finish, dim3(1), dim3(64), 0, st, qw);
    return check_launch("sad_pack_qparams");
}

extern "C" sad_status sad_pack_sites(const sad_image *img, const float *sites, const float *q,
                                     uint32_t *packed, void *stream) {
    SAD_TRY(check_image(img, nullptr));
    if (img->n_slots == 0) return SAD_OK;
    SAD_REQUIRE(sites && q && packed, SAD_ERR_INVALID_ARGUMENT, "sad_pack_sites: NULL pointer");
    SAD_REQUIRE(aligned16(packed), SAD_ERR_INVALID_ARGUMENT,
                "sad_pack_sites: packed not 16-byte aligned");
    SAD_REQUIRE(img->H <= 32768 && img->W <= 32768, SAD_ERR_UNSUPPORTED,
                "sad_pack_sites: positions are 15-bit codes (H, W <= 32768)");
    hipLaunchKernelGGL(k_pack, dim3(blocks_of(img->n_slots)), dim3(256), 0, as_stream(stream),
                       sites, img->cap, img->n_slots, img->H, img->W, q,
                       reinterpret_cast<uint4 *>(packed));
    return check_launch("sad_pack_sites");
}

extern "C" sad_status sad_unpack_sites(const sad_image *img, const uint32_t *packed,
                                       const float *q, float *sites, void *stream) {
    SAD_TRY(check_image(img, nullptr));
    if (img->n_slots == 0) return SAD_OK;
    SAD_REQUIRE(sites && q && packed, SAD_ERR_INVALID_ARGUMENT, "sad_unpack_sites: NULL pointer");
    SAD_REQUIRE(aligned16(packed), SAD_ERR_INVALID_ARGUMENT,
                "sad_unpack_sites: packed not 16-byte aligned");
    hipLaunchKernelGGL(k_unpack, dim3(blocks_of(img->n_slots)), dim3(256), 0, as_stream(stream),
                       reinterpret_cast<const uint4 *>(packed), img->n_slots, img->H, img->W, q,
                       sites, img->cap);
    return check_launch("sad_unpack_sites");
}

extern "C" sad_status sad_prepare_packed(const sad_image *img, const uint32_t *packed,
                                         const float *q, float *rec, void *stream) {
    float s;
    SAD_TRY(check_image(img, &s));
    if (img->n_slots == 0) return SAD_OK;
    SAD_REQUIRE(rec && q && packed, SAD_ERR_INVALID_ARGUMENT, "sad_prepare_packed: NULL pointer");
    SAD_REQUIRE(aligned16(packed) && aligned16(rec), SAD_ERR_INVALID_ARGUMENT,
                "sad_prepare_packed: packed / rec not 16-byte aligned");
    hipLaunchKernelGGL(k_unpack_prepare, dim3(blocks_of(img->n_slots)), dim3(256), 0,
                       as_stream(stream), reinterpret_cast<const uint4 *>(packed), img->n_slots,
                       img->H, img->W, q, s, reinterpret_cast<float4 *>(rec));
    return check_launch("sad_prepare_packed");
}

extern "C" sad_status sad_render_packed(const sad_image *img, const uint32_t *packed,
                                        const float *q, const uint32_t *topk, float *out,
                                        void *stream) {
    float s;
    SAD_TRY(check_image(img, &s));
    SAD_REQUIRE(topk && out, SAD_ERR_INVALID_ARGUMENT, "sad_render_packed: NULL pointer");
    SAD_REQUIRE(aligned16(topk), SAD_ERR_INVALID_ARGUMENT,
                "sad_render_packed: topk not 16-byte aligned");
    hipStream_t st = as_stream(stream);
    if (img->n_slots == 0) {
        launch_fill_f32(out, 3 * (int64_t)img->H * img->W, 0.0f, st);
        return check_launch("sad_render_packed");
    }
    SAD_REQUIRE(packed && q && aligned16(packed), SAD_ERR_INVALID_ARGUMENT,
                "sad_render_packed: packed NULL or not 16-byte aligned, or q NULL");
    const ImgArgs a = img_args(img);
    const uint4 *pk = reinterpret_cast<const uint4 *>(packed);
    const uint4 *t4 = reinterpret_cast<const uint4 *>(topk);
    SAD_K_SWITCH(img->K, hipLaunchKernelGGL((k_fwd_packed<KK>), dim3(a.n_blocks), dim3(256), 0, st,
                                            a, pk, q, s, t4, out));
    return check_launch("sad_render_packed");
}

extern "C" sad_status sad_query_packed(const sad_image *img, const uint32_t *packed,
                                       const float *q, const uint32_t *topk, const float *xy,
                                       int64_t M, float *out, void *stream) {
    float s;
    SAD_TRY(check_image(img, &s));
    SAD_REQUIRE(M >= 0, SAD_ERR_INVALID_ARGUMENT, "sad_query_packed: negative M");
    if (M == 0) return SAD_OK;
    SAD_REQUIRE(topk && xy && out, SAD_ERR_INVALID_ARGUMENT, "sad_query_packed: NULL pointer");
    SAD_REQUIRE(aligned16(topk) && (reinterpret_cast<uintptr_t>(xy) & 7u) == 0,
                SAD_ERR_INVALID_ARGUMENT, "sad_query_packed: topk / xy misaligned");
    hipStream_t st = as_stream(stream);
    if (img->n_slots == 0) {
        launch_fill_f32(out, 3 * M, 0.0f, st);
        return check_launch("sad_query_packed");
    }
    SAD_REQUIRE(packed && q && aligned16(packed), SAD_ERR_INVALID_ARGUMENT,
                "sad_query_packed: packed NULL or not 16-byte aligned, or q NULL");
    const ImgArgs a = img_args(img);
    const uint4 *pk = reinterpret_cast<const uint4 *>(packed);
    const uint4 *t4 = reinterpret_cast<const uint4 *>(topk);
    const float2 *p2 = reinterpret_cast<const float2 *>(xy);
    SAD_K_SWITCH(img->K, hipLaunchKernelGGL((k_query_packed<KK>), dim3(blocks_of(M)), dim3(256), 0,
                                            st, a, pk, q, s, t4, p2, M, out));
    return check_launch("sad_query_packed");
}
