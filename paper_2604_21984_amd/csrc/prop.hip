// prop.hip -- one Jacobi propagation pass of the per-pixel top-K list field (Sec. 4.3).
#include "sad_device.h"
#include "sad_host.h"
#include "sad_internal.h"
#include "sad_kernels.h"

namespace sad {

// a.H x a.W is the grid the list field lives on; with kGrid it is a candidate grid over
// an Hi x Wi image and each cell is scored at its centre (App. B.3), otherwise the grid
// is the image and each pixel is scored at itself.
template <int K, bool kGrid>
__global__ __launch_bounds__(256) void k_prop(PropArgs a, int Hi, int Wi,
                                              const float4 *__restrict__ rec,
                                              const uint4 *__restrict__ lin,
                                              uint4 *__restrict__ lout) {
    __shared__ uint32_t queue[QueueDepth<K>::v][256];
    const int tile = xcd_tile(blockIdx.x, a.n_blocks);
    const TilePix px = tile_pixel(tile, a.tiles_x);
    if (px.i >= a.H || px.j >= a.W) return;  // no block barriers below
    uint64_t keys[K];
    if (kGrid)
        prop_pixel<K>(a, rec, lin, px, queue, keys, grid_point(px.j, Wi, a.W),
                      grid_point(px.i, Hi, a.H));
    else
        prop_pixel<K>(a, rec, lin, px, queue, keys);
    const int64_t P = (int64_t)a.H * a.W;
    const int64_t p = (int64_t)px.i * a.W + px.j;
#pragma unroll
    for (int g = 0; g < K / 4; ++g)
        lout[(int64_t)g * P + p] = make_uint4(key_id(keys[4 * g]), key_id(keys[4 * g + 1]),
                                              key_id(keys[4 * g + 2]), key_id(keys[4 * g + 3]));
}

template <int K>
static void launch_prop(const PropArgs &a, int Hi, int Wi, const float4 *rec, const uint4 *lin,
                        uint4 *lout, hipStream_t st) {
    if (Hi == a.H && Wi == a.W)
        hipLaunchKernelGGL((k_prop<K, false>), dim3(a.n_blocks), dim3(256), 0, st, a, Hi, Wi, rec,
                           lin, lout);
    else
        hipLaunchKernelGGL((k_prop<K, true>), dim3(a.n_blocks), dim3(256), 0, st, a, Hi, Wi, rec,
                           lin, lout);
}

__global__ __launch_bounds__(256) void k_fill_list(uint32_t *__restrict__ p, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = SAD_INVALID_ID;
}

// Exact top-K of one pixel per block by brute force: each of the 128 threads keeps the
// best K of a strided share of the sites (keys are unique: one ID, one key), then a
// pairwise tree of merges of sorted lists in LDS.
constexpr int kExactThreads = 128;

template <int K>
__global__ __launch_bounds__(kExactThreads) void k_exact(int H, int W, int n_slots,
                                                         const float4 *__restrict__ rec,
                                                         const int64_t *__restrict__ pix,
                                                         uint32_t *__restrict__ out) {
    __shared__ uint64_t lk[kExactThreads][K];
    const int t = threadIdx.x;
    const int64_t P = (int64_t)H * W;
    const int64_t p = pix[blockIdx.x];
    uint64_t keys[K];
#pragma unroll
    for (int k = 0; k < K; ++k) keys[k] = 0ull;
    if (p >= 0 && p < P) {
        const float X = (float)(p % W), Y = (float)(p / W);
        for (int i = t; i < n_slots; i += kExactThreads) {
            const float4 q0 = rec[4 * (size_t)i], q1 = rec[4 * (size_t)i + 1];
            if (q1.w == 0.0f) continue;
            insert_key<K>(keys, make_key(score(q0, q1, X, Y), (uint32_t)i));
        }
    }
#pragma unroll
    for (int k = 0; k < K; ++k) lk[t][k] = keys[k];
    __syncthreads();
    for (int s = kExactThreads / 2; s >= 1; s >>= 1) {
        if (t < s) {
            uint64_t m[K];
            int ia = 0, ib = 0;
#pragma unroll
            for (int k = 0; k < K; ++k) {
                const uint64_t a = ia < K ? lk[t][ia] : 0ull;
                const uint64_t b = ib < K ? lk[t + s][ib] : 0ull;
                const bool ta = a >= b;
                m[k] = ta ? a : b;
                ia += ta ? 1 : 0;
                ib += ta ? 0 : 1;
            }
#pragma unroll
            for (int k = 0; k < K; ++k) lk[t][k] = m[k];
        }
        __syncthreads();
    }
    if (t < K) {
        const uint64_t k = lk[0][t];
        out[(int64_t)blockIdx.x * K + t] = k ? key_id(k) : SAD_INVALID_ID;
    }
}

}  // namespace sad

using namespace sad;

extern "C" int32_t sad_jump_step(int64_t t, int32_t H, int32_t W) { return jump_of(t, H, W); }

void sad::launch_propagate(const sad_image *img, const float *rec, const uint32_t *in,
                           uint32_t *out, int32_t jump, int32_t n_inject, uint64_t seed,
                           uint64_t pass, const int64_t *pass_dev, hipStream_t st) {
    launch_propagate_grid(img, img->H, img->W, rec, in, out, jump, n_inject, seed, pass, pass_dev,
                          st);
}

void sad::launch_propagate_grid(const sad_image *img, int32_t Hg, int32_t Wg, const float *rec,
                                const uint32_t *in, uint32_t *out, int32_t jump, int32_t n_inject,
                                uint64_t seed, uint64_t pass, const int64_t *pass_dev,
                                hipStream_t st) {
    const int64_t P = (int64_t)Hg * Wg;
    if (img->n_slots == 0) {
        const int64_t n = P * img->K;
        hipLaunchKernelGGL(k_fill_list, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, out, n);
        return;
    }
    PropArgs a;
    a.H = Hg;
    a.W = Wg;
    a.n_slots = img->n_slots;
    a.jump = jump;
    a.J = n_inject;
    a.every = 1;
    a.tiles_x = (Wg + 15) / 16;
    a.n_blocks = a.tiles_x * ((Hg + 15) / 16);
    a.seed = seed;
    a.pass = pass;
    a.pass_dev = pass_dev;
    const float4 *r4 = reinterpret_cast<const float4 *>(rec);
    const uint4 *li = reinterpret_cast<const uint4 *>(in);
    uint4 *lo = reinterpret_cast<uint4 *>(out);
    const int Hi = img->H, Wi = img->W;
    switch (img->K) {
        case 4: launch_prop<4>(a, Hi, Wi, r4, li, lo, st); break;
        case 8: launch_prop<8>(a, Hi, Wi, r4, li, lo, st); break;
        case 12: launch_prop<12>(a, Hi, Wi, r4, li, lo, st); break;
        case 16: launch_prop<16>(a, Hi, Wi, r4, li, lo, st); break;
        case 20: launch_prop<20>(a, Hi, Wi, r4, li, lo, st); break;
        case 24: launch_prop<24>(a, Hi, Wi, r4, li, lo, st); break;
        case 28: launch_prop<28>(a, Hi, Wi, r4, li, lo, st); break;
        case 32: launch_prop<32>(a, Hi, Wi, r4, li, lo, st); break;
        default: break;
    }
}

extern "C" sad_status sad_exact_topk(const sad_image *img, const float *rec, const int64_t *pix,
                                     int64_t n_pix, uint32_t *out, void *stream) {
    SAD_TRY(check_image(img, nullptr));
    SAD_REQUIRE(n_pix >= 0 && n_pix <= 0x7FFFFFFF, SAD_ERR_INVALID_ARGUMENT,
                "sad_exact_topk: bad pixel count");
    if (n_pix == 0) return SAD_OK;
    SAD_REQUIRE(pix && out, SAD_ERR_INVALID_ARGUMENT, "sad_exact_topk: NULL pointer");
    SAD_REQUIRE(img->n_slots == 0 || (rec && aligned16(rec)), SAD_ERR_INVALID_ARGUMENT,
                "sad_exact_topk: rec NULL or not 16-byte aligned");
    hipStream_t st = as_stream(stream);
    const dim3 g((unsigned)n_pix), b(kExactThreads);
    const float4 *r4 = reinterpret_cast<const float4 *>(rec);
    switch (img->K) {
#define SAD_EXACT_CASE(KK)                                                                    \
    case KK:                                                                                  \
        hipLaunchKernelGGL(k_exact<KK>, g, b, 0, st, img->H, img->W, img->n_slots, r4, pix, out); \
        break;
        SAD_EXACT_CASE(4) SAD_EXACT_CASE(8) SAD_EXACT_CASE(12) SAD_EXACT_CASE(16)
        SAD_EXACT_CASE(20) SAD_EXACT_CASE(24) SAD_EXACT_CASE(28) SAD_EXACT_CASE(32)
#undef SAD_EXACT_CASE
        default: break;
    }
    return check_launch("sad_exact_topk");
}

extern "C" sad_status sad_propagate_topk_state(const sad_image *img, const float *rec,
                                               const uint32_t *topk_in, uint32_t *topk_out,
                                               int32_t n_inject, uint64_t seed,
                                               const sad_step_state *state, void *stream) {
    SAD_TRY(check_image(img, nullptr));
    SAD_REQUIRE(state, SAD_ERR_INVALID_ARGUMENT, "sad_propagate_topk_state: state is NULL");
    SAD_REQUIRE(topk_in && topk_out, SAD_ERR_INVALID_ARGUMENT,
                "sad_propagate_topk_state: NULL list");
    SAD_REQUIRE(topk_in != topk_out, SAD_ERR_INVALID_ARGUMENT,
                "sad_propagate_topk_state: topk_in and topk_out must not alias (Jacobi pass)");
    SAD_REQUIRE(aligned16(topk_in) && aligned16(topk_out), SAD_ERR_INVALID_ARGUMENT,
                "sad_propagate_topk_state: lists must be 16-byte aligned");
    SAD_REQUIRE(n_inject >= 0 && n_inject <= 16, SAD_ERR_INVALID_ARGUMENT,
                "sad_propagate_topk_state: n_inject must be in [0, 16]");
    SAD_REQUIRE(img->n_slots == 0 || (rec && aligned16(rec)), SAD_ERR_INVALID_ARGUMENT,
                "sad_propagate_topk_state: rec NULL or not 16-byte aligned");
    launch_propagate(img, rec, topk_in, topk_out, 0, n_inject, seed, 0, &state->pass,
                     as_stream(stream));
    return check_launch("sad_propagate_topk_state");
}

extern "C" sad_status sad_propagate_topk(const sad_image *img, const float *rec,
                                         const uint32_t *topk_in, uint32_t *topk_out,
                                         int32_t jump, int32_t n_inject, uint64_t seed,
                                         uint64_t pass_index, void *stream) {
    SAD_TRY(check_image(img, nullptr));
    SAD_REQUIRE(topk_in && topk_out, SAD_ERR_INVALID_ARGUMENT, "sad_propagate_topk: NULL list");
    SAD_REQUIRE(topk_in != topk_out, SAD_ERR_INVALID_ARGUMENT,
                "sad_propagate_topk: topk_in and topk_out must not alias (Jacobi pass)");
    SAD_REQUIRE(aligned16(topk_in) && aligned16(topk_out), SAD_ERR_INVALID_ARGUMENT,
                "sad_propagate_topk: lists must be 16-byte aligned");
    SAD_REQUIRE(jump >= 1, SAD_ERR_INVALID_ARGUMENT, "sad_propagate_topk: jump must be >= 1");
    SAD_REQUIRE(n_inject >= 0 && n_inject <= 16, SAD_ERR_INVALID_ARGUMENT,
                "sad_propagate_topk: n_inject must be in [0, 16]");
    SAD_REQUIRE(img->n_slots == 0 || (rec && aligned16(rec)), SAD_ERR_INVALID_ARGUMENT,
                "sad_propagate_topk: rec NULL or not 16-byte aligned");
    launch_propagate(img, rec, topk_in, topk_out, jump, n_inject, seed, pass_index, nullptr,
                     as_stream(stream));
    return check_launch("sad_propagate_topk");
}
