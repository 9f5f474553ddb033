// prop.hip -- one Jacobi propagation pass of the per-pixel top-K list field (Sec. 4.3).
#include "sad_device.h"
#include "sad_host.h"
#include "sad_internal.h"

namespace sad {

struct PropArgs {
    int H, W, n_slots, jump, J, tiles_x, n_blocks;
    uint64_t seed, pass;
    const int64_t *pass_dev;  // device pass index (graph-replayable), or NULL
};

// One thread per pixel, 16x16 tiles (four 8x8 wave64 blocks).
//  1. The pixel's own list is scored exactly and sorted (Batcher network); the K-th
//     key is the admission threshold.
//  2. Every other candidate (the four lists at +-jump inside the image, then the J
//     injected IDs) is first screened cheaply: an ID already kept is a repeat (equal
//     key, never inserted); otherwise the score is estimated with the hardware square
//     root (<= 1 ulp) and rejected if it is below the threshold by more than a bound on
//     the estimate's error.  The bound: with |n_a - n| <= 2^-22 n, the float32 score
//     differs from the exact sequence by at most 2^-21 (kappa (|r| + n) + |l|); the
//     test uses 2^-19 of that sum.
//  3. Survivors are queued in LDS and scored exactly before the queue could overflow
//     and at the end, then bubbled into the sorted key array.
// A candidate is only ever discarded when its exact key is below the K-th key, so the
// result is the exact top K of the candidate set, as in the plain definition.
template <int K>
struct QueueDepth {
    static constexpr int v = K + 8;  // room for one whole list (or 4 injections) after a check
};

template <int K>
__global__ __launch_bounds__(256) void k_prop(PropArgs a, const float4 *__restrict__ rec,
                                              const uint4 *__restrict__ lin,
                                              uint4 *__restrict__ lout) {
    constexpr int Q = QueueDepth<K>::v;
    __shared__ uint32_t queue[Q][256];
    const int tile = xcd_tile(blockIdx.x, a.n_blocks);
    const TilePix px = tile_pixel(tile, a.tiles_x);
    if (px.i >= a.H || px.j >= a.W) return;  // no block barriers below
    const int tid = threadIdx.x;
    const int64_t P = (int64_t)a.H * a.W;
    const int64_t p = (int64_t)px.i * a.W + px.j;
    const float X = (float)px.j, Y = (float)px.i;
    const uint32_t ns = (uint32_t)a.n_slots;
    const uint64_t pass = a.pass_dev ? (uint64_t)*a.pass_dev : a.pass;
    const int s = (a.pass_dev && a.jump <= 0) ? jump_of((int64_t)pass, a.H, a.W) : a.jump;

    auto exact_key = [&](uint32_t id) __attribute__((always_inline)) -> uint64_t {
        const bool in_range = id < ns;
        const uint32_t idc = in_range ? id : 0u;
        const float4 q0 = rec[4 * (size_t)idc], q1 = rec[4 * (size_t)idc + 1];
        return (in_range && q1.w != 0.0f) ? make_key(score(q0, q1, X, Y), id) : 0ull;
    };

    // 1. own list
    uint64_t keys[K];
#pragma unroll
    for (int g = 0; g < K / 4; ++g) {
        const uint4 v = lin[(int64_t)g * P + p];
        keys[4 * g] = exact_key(v.x);
        keys[4 * g + 1] = exact_key(v.y);
        keys[4 * g + 2] = exact_key(v.z);
        keys[4 * g + 3] = exact_key(v.w);
    }
    sort_keys_desc<K>(keys);
    bool rep = false;
#pragma unroll
    for (int k = 1; k < K; ++k) rep = rep || (keys[k] != 0ull && keys[k] == keys[k - 1]);
    if (rep) {  // a repeated ID in the input list: rebuild as a set
        uint64_t t[K];
#pragma unroll
        for (int k = 0; k < K; ++k) {
            t[k] = keys[k];
            keys[k] = 0ull;
        }
#pragma unroll
        for (int k = 0; k < K; ++k) insert_key<K>(keys, t[k]);
    }
    float kth = keys[K - 1] ? key_score(keys[K - 1]) : -INFINITY;
    int qn = 0;

    auto screen = [&](uint32_t id) __attribute__((always_inline)) {
        const bool in_range = id < ns;
        const uint32_t idc = in_range ? id : 0u;
        const float4 q0 = rec[4 * (size_t)idc], q1 = rec[4 * (size_t)idc + 1];
        const uint32_t nid = ~id;
        bool kept = false;
#pragma unroll
        for (int k = 0; k < K; ++k) kept = kept || ((uint32_t)keys[k] == nid);
        const float na = __builtin_amdgcn_sqrtf(quad(q0, q1, X, Y));
        const float la = q1.y * (q1.z - na);
        const float bound = fmaf(q1.y, fabsf(q1.z) + na, fabsf(la)) * 0x1p-19f;
        const bool maybe = in_range && q1.w != 0.0f && !kept &&
                           (keys[K - 1] == 0ull || la + bound >= kth);
        if (maybe) queue[qn++][tid] = id;
    };
    auto drain_if = [&](int room) __attribute__((always_inline)) {
        if (__any(qn > Q - room)) {
            for (int i = 0; i < Q; ++i) {
                if (!__any(i < qn)) break;
                if (i < qn) insert_key<K>(keys, exact_key(queue[i][tid]));
            }
            qn = 0;
            kth = keys[K - 1] ? key_score(keys[K - 1]) : -INFINITY;
        }
    };

    // 2. screen the other candidates: the four lists at +-jump, then the injections
#pragma unroll 1
    for (int nb = 0; nb < 4; ++nb) {
        const int di = nb == 2 ? s : (nb == 3 ? -s : 0);
        const int dj = nb == 0 ? s : (nb == 1 ? -s : 0);
        const int ii = px.i + di, jj = px.j + dj;
        drain_if(K);
        if (ii >= 0 && ii < a.H && jj >= 0 && jj < a.W) {
            const int64_t q = (int64_t)ii * a.W + jj;
#pragma unroll
            for (int g = 0; g < K / 4; ++g) {
                const uint4 v = lin[(int64_t)g * P + q];
                screen(v.x);
                screen(v.y);
                screen(v.z);
                screen(v.w);
            }
        }
    }
    const uint64_t k0 = (pass * (uint64_t)P + (uint64_t)p) * (uint64_t)a.J;
#pragma unroll 1
    for (int j = 0; j < a.J; j += 4) {
        drain_if(4);
#pragma unroll
        for (int jj = 0; jj < 4; ++jj)
            if (j + jj < a.J) {
                const uint64_t hi = splitmix64(a.seed, k0 + (uint64_t)(j + jj)) >> 32;
                screen((uint32_t)((hi * (uint64_t)ns) >> 32));
            }
    }
    // 3. remaining survivors
    drain_if(Q + 1);
#pragma unroll
    for (int g = 0; g < K / 4; ++g)
        lout[(int64_t)g * P + p] = make_uint4(key_id(keys[4 * g]), key_id(keys[4 * g + 1]),
                                              key_id(keys[4 * g + 2]), key_id(keys[4 * g + 3]));
}

template <int K>
static void launch_prop(const PropArgs &a, const float4 *rec, const uint4 *lin, uint4 *lout,
                        hipStream_t st) {
    hipLaunchKernelGGL(k_prop<K>, dim3(a.n_blocks), dim3(256), 0, st, a, rec, lin, lout);
}

__global__ __launch_bounds__(256) void k_fill_list(uint32_t *__restrict__ p, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = SAD_INVALID_ID;
}

}  // namespace sad

using namespace sad;

extern "C" int32_t sad_jump_step(int64_t t, int32_t H, int32_t W) { return jump_of(t, H, W); }

void sad::launch_propagate(const sad_image *img, const float *rec, const uint32_t *in,
                           uint32_t *out, int32_t jump, int32_t n_inject, uint64_t seed,
                           uint64_t pass, const int64_t *pass_dev, hipStream_t st) {
    const int64_t P = (int64_t)img->H * img->W;
    if (img->n_slots == 0) {
        const int64_t n = P * img->K;
        hipLaunchKernelGGL(k_fill_list, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, out, n);
        return;
    }
    PropArgs a;
    a.H = img->H;
    a.W = img->W;
    a.n_slots = img->n_slots;
    a.jump = jump;
    a.J = n_inject;
    a.tiles_x = tiles_x(img);
    a.n_blocks = n_tiles(img);
    a.seed = seed;
    a.pass = pass;
    a.pass_dev = pass_dev;
    const float4 *r4 = reinterpret_cast<const float4 *>(rec);
    const uint4 *li = reinterpret_cast<const uint4 *>(in);
    uint4 *lo = reinterpret_cast<uint4 *>(out);
    switch (img->K) {
        case 4: launch_prop<4>(a, r4, li, lo, st); break;
        case 8: launch_prop<8>(a, r4, li, lo, st); break;
        case 12: launch_prop<12>(a, r4, li, lo, st); break;
        case 16: launch_prop<16>(a, r4, li, lo, st); break;
        case 20: launch_prop<20>(a, r4, li, lo, st); break;
        case 24: launch_prop<24>(a, r4, li, lo, st); break;
        case 28: launch_prop<28>(a, r4, li, lo, st); break;
        case 32: launch_prop<32>(a, r4, li, lo, st); break;
        default: break;
    }
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
