// sad_kernels.h -- per-pixel device routines shared by the kernels: propagation of one
// pixel's list (Sec. 4.3), the soft blend (Sec. 4.2) and the backward contributions
// with the per-tile fixed-point LDS table (App. B.4, Sec. 4.8).
#pragma once

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

inline ImgArgs img_args(const sad_image *img) {
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

// Valid entries of one pixel's list with their scores (K registers each).
template <int K>
struct PixelBlend {
    uint32_t id[K];
    float l[K];
    float e[K];
    bool ok[K];
    float S, c[3];
    int nv;
    int r;                // reference entry (largest score), when requested
    float cr[3], dc[3];   // its colour and sum_k w_k (c_k - c_r)
};

// Rotate ids[] left by `rot` (0 <= rot < 8) with three conditional stages.  The
// image-space kernels take a pixel's entries in an order rotated by the lane's
// position in its 8x8 block (lane_rot), so that neighbouring lanes, whose sorted lists
// are nearly the same, work on different sites in the same instruction: the
// backward's LDS atomics then go to different slots instead of all to the best site's.
// Every image-space kernel uses the same rotation, so their sums are formed in the
// same order.
template <int K, typename T>
__device__ __forceinline__ void rotate_ids(T (&ids)[K], int rot) {
#pragma unroll
    for (int st = 1; st < 8 && st < K; st <<= 1) {
        const bool c = (rot & st) != 0;
        T t[K];
#pragma unroll
        for (int j = 0; j < K; ++j) t[j] = c ? ids[(j + st) % K] : ids[j];
#pragma unroll
        for (int j = 0; j < K; ++j) ids[j] = t[j];
    }
}

__device__ __forceinline__ int lane_rot() {
    const int lane = threadIdx.x & 63;
    return ((lane & 7) + 3 * (lane >> 3)) & 7;
}

// Softmax and colour of a pixel whose entries have been gathered: the max-subtracted
// weights (App. B.4), c = sum_k w_k c_k, and with kRef the reference entry r (the
// first entry with the largest score), its colour c_r and dc = sum_k w_k (c_k - c_r),
// which the backward needs to form c_k - c without cancellation.
template <int K, bool kRef>
__device__ __forceinline__ void finish_blend(PixelBlend<K> &b, const float (*col)[3], float m) {
    b.r = 0;
    b.cr[0] = b.cr[1] = b.cr[2] = 0.f;
    if (kRef) {
        float mx = -INFINITY;
#pragma unroll
        for (int k = 0; k < K; ++k)
            if (b.ok[k] && b.l[k] > mx) {
                mx = b.l[k];
                b.r = k;
            }
#pragma unroll
        for (int k = 0; k < K; ++k)
            if (k == b.r) {
                b.cr[0] = col[k][0];
                b.cr[1] = col[k][1];
                b.cr[2] = col[k][2];
            }
    }
    b.S = 0.f;
    float c0 = 0.f, c1 = 0.f, c2 = 0.f, d0 = 0.f, d1 = 0.f, d2 = 0.f;
#pragma unroll
    for (int k = 0; k < K; ++k) {
        b.e[k] = b.ok[k] ? __expf(b.l[k] - m) : 0.0f;
        b.S += b.e[k];
        c0 = fmaf(b.e[k], col[k][0], c0);
        c1 = fmaf(b.e[k], col[k][1], c1);
        c2 = fmaf(b.e[k], col[k][2], c2);
        if (kRef) {
            d0 = fmaf(b.e[k], col[k][0] - b.cr[0], d0);
            d1 = fmaf(b.e[k], col[k][1] - b.cr[1], d1);
            d2 = fmaf(b.e[k], col[k][2] - b.cr[2], d2);
        }
    }
    const float inv = b.nv ? __builtin_amdgcn_rcpf(b.S) : 0.f;
    b.c[0] = c0 * inv;
    b.c[1] = c1 * inv;
    b.c[2] = c2 * inv;
    b.dc[0] = d0 * inv;
    b.dc[1] = d1 * inv;
    b.dc[2] = d2 * inv;
}

// Where the blend gathers a site's record from: the derived records (RecSrc), or a
// source that builds q0..q2 another way (the packed records' decoder).
struct RecSrc {
    const float4 *__restrict__ rec;
    __device__ __forceinline__ void fetch(uint32_t id, float4 &q0, float4 &q1, float4 &q2) const {
        q0 = rec[4 * (size_t)id];
        q1 = rec[4 * (size_t)id + 1];
        q2 = rec[4 * (size_t)id + 2];
    }
};

// Whether the blend fetches a group of entries' records before scoring any of them
// (derived records only: the packed source decodes in its fetch, and a group of decoded
// records does not fit the registers).
template <class Src>
struct GroupFetch {
    static constexpr bool v = false;
};
template <>
struct GroupFetch<RecSrc> {
    static constexpr bool v = true;
};

// Gather and score the list of pixel p at point (X, Y); max-subtracted softmax; colour.
// The entries are taken in the order rotated by `rot`.  Without the reference terms and
// for K <= 16, the records of a group of entries (all of them up to K = 8, four at a time
// up to 16) are in registers before any score is formed, so a wave waits for one memory
// round trip per group: random point queries, whose lanes gather unrelated records, run
// ~1.6x faster (2^20 points at 2048^2: 116 -> 74 us at K = 8, 352 -> 217 us at K = 16).
template <int K, bool kRef, class Src>
__device__ __forceinline__ void blend_src(const Src &src, uint32_t ns,
                                          const uint4 *__restrict__ topk, int64_t P, int64_t p,
                                          float X, float Y, PixelBlend<K> &b, int rot = 0) {
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
    float col[K][3];
    constexpr int G = (GroupFetch<Src>::v && !kRef) ? (K <= 8 ? K : (K <= 16 ? 4 : 1)) : 1;
    if constexpr (G == 1) {
#pragma unroll
        for (int k = 0; k < K; ++k) {
            const uint32_t id = ids[k];
            const bool in_range = id < ns;
            const uint32_t idc = in_range ? id : 0u;
            float4 q0, q1, q2;
            src.fetch(idc, q0, q1, q2);
            b.id[k] = idc;
            b.ok[k] = in_range && q1.w != 0.0f;
            b.l[k] = score(q0, q1, X, Y);
            col[k][0] = q2.x;
            col[k][1] = q2.y;
            col[k][2] = q2.z;
            if (b.ok[k]) {
                m = fmaxf(m, b.l[k]);
                ++b.nv;
            }
        }
        finish_blend<K, kRef>(b, col, m);
        return;
    }
#pragma unroll
    for (int g0 = 0; g0 < K; g0 += G) {
        float4 q0[G], q1[G], q2[G];
#pragma unroll
        for (int k = 0; k < G; ++k) {
            const uint32_t id = ids[g0 + k];
            src.fetch(id < ns ? id : 0u, q0[k], q1[k], q2[k]);
        }
        // the group's records all in registers here: one wait for the group
#pragma unroll
        for (int k = 0; k < G; ++k)
            asm volatile("" ::"v"(q0[k].x), "v"(q0[k].y), "v"(q0[k].z), "v"(q0[k].w),
                         "v"(q1[k].x), "v"(q1[k].y), "v"(q1[k].z), "v"(q1[k].w),
                         "v"(q2[k].x), "v"(q2[k].y), "v"(q2[k].z));
#pragma unroll
        for (int k = 0; k < G; ++k) {
            const int kk = g0 + k;
            const uint32_t id = ids[kk];
            const bool in_range = id < ns;
            b.id[kk] = in_range ? id : 0u;
            b.ok[kk] = in_range && q1[k].w != 0.0f;
            b.l[kk] = score(q0[k], q1[k], X, Y);
            col[kk][0] = q2[k].x;
            col[kk][1] = q2[k].y;
            col[kk][2] = q2[k].z;
            if (b.ok[kk]) {
                m = fmaxf(m, b.l[kk]);
                ++b.nv;
            }
        }
    }
    finish_blend<K, kRef>(b, col, m);
}

template <int K, bool kRef>
__device__ __forceinline__ void blend(const float4 *__restrict__ rec, uint32_t ns,
                                      const uint4 *__restrict__ topk, int64_t P, int64_t p,
                                      float X, float Y, PixelBlend<K> &b, int rot = 0) {
    blend_src<K, kRef>(RecSrc{rec}, ns, topk, P, p, X, Y, b, rot);
}

// The blend of a pixel from its freshly propagated keys (sorted descending, so entry 0
// holds the maximum score): the scores are the keys' own exact float32 scores.  The
// entries are taken in the order rotated by `rot`, as blend() does with its list.
template <int K, bool kRef>
__device__ __forceinline__ void blend_keys(const float4 *__restrict__ rec, const uint64_t (&sorted)[K],
                                           PixelBlend<K> &b, int rot = 0) {
    b.nv = 0;
    const float m = sorted[0] ? key_score(sorted[0]) : 0.0f;
    uint64_t keys[K];
#pragma unroll
    for (int k = 0; k < K; ++k) keys[k] = sorted[k];
    if (rot) rotate_ids<K>(keys, rot);
    float col[K][3];
#pragma unroll
    for (int k = 0; k < K; ++k) {
        b.ok[k] = keys[k] != 0ull;
        const uint32_t id = b.ok[k] ? key_id(keys[k]) : 0u;
        b.id[k] = id;
        b.l[k] = b.ok[k] ? key_score(keys[k]) : 0.0f;
        const float4 q2 = rec[4 * (size_t)id + 2];
        col[k][0] = q2.x;
        col[k][1] = q2.y;
        col[k][2] = q2.z;
        b.nv += b.ok[k] ? 1 : 0;
    }
    finish_blend<K, kRef>(b, col, m);
}

__device__ __forceinline__ float block_sum(float v) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    __shared__ float part[4];
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = v;
    __syncthreads();
    const float r = (part[0] + part[1]) + (part[2] + part[3]);
    __syncthreads();
    return r;
}

// ---- propagation ------------------------------------------------------------------
struct PropArgs {
    int H, W, n_slots, jump, J, tiles_x, n_blocks;
    int every;                // candidate update period (<= 1: every iteration)
    uint64_t seed, pass;
    const int64_t *pass_dev;  // device iteration index (graph-replayable), or NULL
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

// Exact keys of NC candidate IDs at pixel centre (X, Y) into out[].  The NC record
// loads are issued before any score is formed, so a wave waits for one memory round
// trip per group rather than one per candidate.  An ID >= ns or a site marked invalid
// gives the empty key 0.
template <int NC>
__device__ __forceinline__ void exact_keys(const float4 *__restrict__ rec, uint32_t ns, float X,
                                           float Y, const uint32_t (&id)[NC], uint64_t *out) {
    float4 q0[NC], q1[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) {
        const uint32_t idc = id[c] < ns ? id[c] : 0u;
        q0[c] = rec[4 * (size_t)idc];
        q1[c] = rec[4 * (size_t)idc + 1];
    }
#pragma unroll
    for (int c = 0; c < NC; ++c) {
        const uint64_t k = make_key(score(q0[c], q1[c], X, Y), id[c]);
        out[c] = ((id[c] < ns) & (q1[c].w != 0.0f)) ? k : 0ull;
    }
}

// The new list of pixel (px.i, px.j) into keys[] (sorted, 0 = empty).  Lanes of pixels
// outside the image must not call it (it votes across the wave, so call it from a
// branch that those lanes skip).  queue: the kernel's LDS queue, Q x 256 words.
// (X, Y) is the point the candidates are scored at: the pixel itself on the image's own
// grid, the cell's centre on a candidate grid (a.H x a.W cells then).
template <int K>
__device__ __forceinline__ void prop_pixel(const PropArgs &a, const float4 *__restrict__ rec,
                                           const uint4 *__restrict__ lin, TilePix px,
                                           uint32_t (*queue)[256], uint64_t (&keys)[K],
                                           float X, float Y) {
    constexpr int Q = QueueDepth<K>::v;
    const int tid = threadIdx.x;
    const int64_t P = (int64_t)a.H * a.W;
    const int64_t p = (int64_t)px.i * a.W + px.j;
    const uint32_t ns = (uint32_t)a.n_slots;
    const uint64_t it = a.pass_dev ? (uint64_t)*a.pass_dev : a.pass;
    // with an update period f, iteration it is pass it / f, and only every f-th
    // iteration looks at neighbours and injections (the same for the whole launch)
    const bool full = a.every <= 1 || it % (uint64_t)a.every == 0;
    const uint64_t pass = a.every <= 1 ? it : it / (uint64_t)a.every;
    const int s = (a.pass_dev && a.jump <= 0) ? jump_of((int64_t)pass, a.H, a.W) : a.jump;

    // 1. own list
    {
        uint4 ol[K / 4];
#pragma unroll
        for (int g = 0; g < K / 4; ++g) ol[g] = lin[(int64_t)g * P + p];
#pragma unroll
        for (int g = 0; g < K / 4; ++g) {
            const uint32_t id[4] = {ol[g].x, ol[g].y, ol[g].z, ol[g].w};
            exact_keys<4>(rec, ns, X, Y, id, &keys[4 * g]);
        }
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

    // Screen four candidates: drop IDs already in the list and out-of-range IDs, then
    // estimate each remaining score with the hardware square root and queue the ID
    // unless the estimate is below the K-th score by more than its error bound.  The
    // four record loads go out together; a dropped ID reads record 0, which all such
    // lanes of the wave share, so the gather only fetches records of new IDs.
    auto screen4 = [&](uint4 v) __attribute__((always_inline)) {
        const uint32_t id[4] = {v.x, v.y, v.z, v.w};
        uint32_t idc[4];
        bool ok[4];
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            // (the empty asm keeps ~id as a value, so each test below is one compare
            // instead of an xor and a compare with -1)
            uint32_t nid = ~id[c];
            asm("" : "+v"(nid));
            bool kept = false;
#pragma unroll
            for (int k = 0; k < K; ++k) kept |= ((uint32_t)keys[k] == nid);
            ok[c] = (id[c] < ns) & !kept;
            idc[c] = ok[c] ? id[c] : 0u;
        }
        float4 q0[4], q1[4];
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            q0[c] = rec[4 * (size_t)idc[c]];
            q1[c] = rec[4 * (size_t)idc[c] + 1];
        }
        const bool open = keys[K - 1] == 0ull;
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            const float na = __builtin_amdgcn_sqrtf(quad(q0[c], q1[c], X, Y));
            const float la = q1[c].y * (q1[c].z - na);
            const float bound = fmaf(q1[c].y, fabsf(q1[c].z) + na, fabsf(la)) * 0x1p-19f;
            const bool maybe = ok[c] & (q1[c].w != 0.0f) & (open | (la + bound >= kth));
            if (maybe) queue[qn++][tid] = id[c];
        }
    };
    auto drain_if = [&](int room) __attribute__((always_inline)) {
        if (__any(qn > Q - room)) {
            for (int i = 0; i < Q; i += 2) {
                if (!__any(i < qn)) break;
                const uint32_t id[2] = {i < qn ? queue[i][tid] : SAD_INVALID_ID,
                                        i + 1 < qn ? queue[i + 1][tid] : SAD_INVALID_ID};
                uint64_t nk[2];
                exact_keys<2>(rec, ns, X, Y, id, nk);
                insert_key<K>(keys, nk[0]);
                insert_key<K>(keys, nk[1]);
            }
            qn = 0;
            kth = keys[K - 1] ? key_score(keys[K - 1]) : -INFINITY;
        }
    };

    // 2. screen the other candidates: the four lists at +-jump, then the injections
#pragma unroll 1
    for (int nb = 0; nb < (full ? 4 : 0); ++nb) {
        const int di = nb == 2 ? s : (nb == 3 ? -s : 0);
        const int dj = nb == 0 ? s : (nb == 1 ? -s : 0);
        const int ii = px.i + di, jj = px.j + dj;
        drain_if(K);
        if (ii >= 0 && ii < a.H && jj >= 0 && jj < a.W) {
            const int64_t q = (int64_t)ii * a.W + jj;
            uint4 nl[K / 4];
#pragma unroll
            for (int g = 0; g < K / 4; ++g) nl[g] = lin[(int64_t)g * P + q];
#pragma unroll
            for (int g = 0; g < K / 4; ++g) screen4(nl[g]);
        }
    }
    const uint64_t k0 = (pass * (uint64_t)P + (uint64_t)p) * (uint64_t)a.J;
#pragma unroll 1
    for (int j = 0; j < (full ? a.J : 0); j += 4) {
        drain_if(4);
        uint32_t inj[4];
#pragma unroll
        for (int jj = 0; jj < 4; ++jj) {
            const uint64_t hi = splitmix64(a.seed, k0 + (uint64_t)(j + jj)) >> 32;
            inj[jj] = j + jj < a.J ? (uint32_t)((hi * (uint64_t)ns) >> 32) : SAD_INVALID_ID;
        }
        screen4(make_uint4(inj[0], inj[1], inj[2], inj[3]));
    }
    // 3. remaining survivors
    drain_if(Q + 1);
}

template <int K>
__device__ __forceinline__ void prop_pixel(const PropArgs &a, const float4 *__restrict__ rec,
                                           const uint4 *__restrict__ lin, TilePix px,
                                           uint32_t (*queue)[256], uint64_t (&keys)[K]) {
    prop_pixel<K>(a, rec, lin, px, queue, keys, (float)px.j, (float)px.i);
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

// Address of gradient element (parameter q, site id): parameter-major [10][cap] (the
// layout of sad_render_bwd's output) or site-major [cap][10] (the training step's own
// accumulator: the ten sums of one site share a cache line, so the flush's atomics of a
// (tile, site) pair coalesce into one or two line requests).
template <bool kSiteMajor>
__device__ __forceinline__ float *grad_at(float *grad, int q, uint32_t id, int64_t cap) {
    return kSiteMajor ? grad + (int64_t)id * SAD_NPARAM + q : grad + q * cap + id;
}

struct FixScale {
    double to_fix;     // 2^(32 + e): the tile table's unit is 2^-(32 + e)
    double from_fix;   // 2^-(32 + e)
    float limit;       // |v| must be below 2^(15 - e)
    double to_det;     // 2^(20 + e): the deterministic mode's unit is 2^-(20 + e)
    // The backward forms its terms from a pre-scaled dL/dc (every gradient term is
    // linear in dL/dc, so scaling it by a power of two scales each term exactly): a
    // term v arrives as x = v / unit, |x| < 2^47 when the term is in range, and its
    // fixed-point integer is rint(x) (rint_i64).
    float pre;         // 2^(32 + e)
    float pre_det;     // 2^(40 + e - kGlobShift)
    float post;        // 2^-(32 + e): back from x to v (float fallback)
};

// |x| bound of a pre-scaled term that the tile table takes (a tile slot then sums at
// most 256 terms below 2^47: far from 2^63).
constexpr float kHiLimit = 0x1p47f;

// rint(x) (ties to even) of a float with |x| < 2^51 as a 64-bit two's complement
// integer: in double, x + 1.5 2^52 lies in [2^52, 2^53), where neighbouring doubles are
// 1 apart, so the add rounds x to an integer and the sum's encoding is the encoding of
// 1.5 2^52 plus that integer.  A conversion, a double add and a 64-bit subtract.
__device__ __forceinline__ unsigned long long rint_i64(float x) {
    const double d = (double)x + 0x1.8p52;
    return (unsigned long long)__double_as_longlong(d) - 0x4338000000000000ull;
}

// Deterministic gradient sums (training steps with SAD_TRAIN_DETERMINISTIC): every
// term is rounded once into units of det_grad_unit(P) (2^kGlobShift times the default
// tile resolution) and from there on only integers are added: in the LDS tile table,
// by the flush into the int64 global accumulator, and directly for the terms that
// bypass the table.  The sums therefore depend neither on the order in which tiles
// finish nor on which terms found a table slot.  Range: |sum| < 2^63 holds for
// |gradient| < 2^(43 - e) (> 10^7 for a 4096 x 4096 image).

__device__ __forceinline__ long long *grad64_at(float *grad, int q, uint32_t id, int64_t cap,
                                                bool site_major) {
    long long *g = reinterpret_cast<long long *>(grad);
    return site_major ? g + (int64_t)id * SAD_NPARAM + q : g + q * cap + id;
}

// A pre-scaled term x (in the deterministic unit) straight into the deterministic
// accumulator: rint(x), clamped to the int64 range.
__device__ __forceinline__ void det_add_x(long long *dst, float xs) {
    double x = rint((double)xs);
    x = fmin(fmax(x, -0x1p62), 0x1p62);
    atomicAdd(reinterpret_cast<unsigned long long *>(dst), (unsigned long long)(long long)x);
}

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

// Contributions of one pixel (its blend b, with the reference terms) to the site
// gradients for dL/dc = (g0, g1, g2), added into the tile table (hkey, hacc) or, if
// the table is full or a term is out of fixed-point range, straight to global memory.
// With kRD also the removal delta against the target colour (I0, I1, I2).  Each
// entry's record is gathered again here (colour, metric, direction) rather than kept
// in registers from the blend.
template <int K, bool kRD, bool kSiteMajor = false, bool kDet = false>
__device__ __forceinline__ void bwd_pixel(const float4 *__restrict__ rec, const PixelBlend<K> &b,
                                          float X, float Y, float g0, float g1, float g2,
                                          float I0, float I1, float I2,
                                          uint32_t *__restrict__ hkey,
                                          unsigned long long (*hacc)[kHashSlots],
                                          const FixScale &fx, float inv_P, int64_t cap,
                                          float *__restrict__ grad, float *__restrict__ rdel) {
    static_assert(!(kRD && kDet), "the deterministic mode has no removal-delta channel");
    if (!b.nv) return;
    const float invS = __builtin_amdgcn_rcpf(b.S);
    // c_k - c = (c_k - c_r) - dc with dc = sum_j w_j (c_j - c_r), r the reference entry
    // (largest score, e_r = 1): nothing cancels when one weight is close to 1.
    const int r = b.r;
    const float cr0 = b.cr[0], cr1 = b.cr[1], cr2 = b.cr[2];
    const float dc0 = b.dc[0], dc1 = b.dc[1], dc2 = b.dc[2];
    // removal delta (Sec. 4.5): Delta = (c' - c) . ((c' - c) + 2 (c - I))
    float e0 = 0.f, e1 = 0.f, e2 = 0.f;      // c - I
    float dr0 = 0.f, dr1 = 0.f, dr2 = 0.f;   // c'_r - c for the reference entry
    if (kRD) {
        e0 = b.c[0] - I0;
        e1 = b.c[1] - I1;
        e2 = b.c[2] - I2;
        if (b.nv > 1) {
            float m2 = -INFINITY;
#pragma unroll
            for (int k = 0; k < K; ++k)
                if (b.ok[k] && k != r) m2 = fmaxf(m2, b.l[k]);
            float S2 = 0.f, n0 = 0.f, n1 = 0.f, n2 = 0.f;
#pragma unroll
            for (int k = 0; k < K; ++k) {
                if (!b.ok[k] || k == r) continue;
                const float4 q2 = rec[4 * (size_t)b.id[k] + 2];
                const float ee = __expf(b.l[k] - m2);
                S2 += ee;
                n0 = fmaf(ee, q2.x - cr0, n0);
                n1 = fmaf(ee, q2.y - cr1, n1);
                n2 = fmaf(ee, q2.z - cr2, n2);
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
    // Every gradient term is linear in dL/dc: form them from dL/dc pre-scaled so that
    // each term arrives in table units (rint_i64).
    const float pre = kDet ? fx.pre_det : fx.pre;
    const float gs0 = g0 * pre, gs1 = g1 * pre, gs2 = g2 * pre;
    // Entries are visited one at a time from the front of shifting copies of the
    // per-entry arrays (a rolled loop without dynamic register indexing), which keeps
    // one entry's records in flight and the register footprint small.
    uint32_t ids[K];
    float ls[K], ws[K];
#pragma unroll
    for (int k = 0; k < K; ++k) {
        ws[k] = b.e[k] * invS;
        // every term of an entry is a multiple of its weight (the removal delta of a
        // non-reference entry too): an entry whose weight is 0 adds exactly 0, so it
        // takes no table slot and no atomics (up to K = 8: at K = 16 the extra test
        // costs more in the register-capped kernel than it saves)
        ids[k] = (b.ok[k] && (K > 8 || ws[k] != 0.0f)) ? b.id[k] : SAD_INVALID_ID;
        ls[k] = b.l[k];
    }
#pragma unroll 1
    for (int k = 0; k < K; ++k) {
        const uint32_t id = ids[0];
        const float lk = ls[0], w = ws[0];
#pragma unroll
        for (int j = 0; j + 1 < K; ++j) {
            ids[j] = ids[j + 1];
            ls[j] = ls[j + 1];
            ws[j] = ws[j + 1];
        }
        if (id == SAD_INVALID_ID) continue;
        const float4 q0 = rec[4 * (size_t)id], q1 = rec[4 * (size_t)id + 1];
        const float4 q2 = rec[4 * (size_t)id + 2], q3 = rec[4 * (size_t)id + 3];
        const float d0 = (q2.x - cr0) - dc0;  // c_k - c
        const float d1 = (q2.y - cr1) - dc1;
        const float d2 = (q2.z - cr2) - dc2;
        float acc[kAcc];
        acc[4] = w * gs0;
        acc[5] = w * gs1;
        acc[6] = w * gs2;
        const float gam = w * fmaf(gs0, d0, fmaf(gs1, d1, gs2 * d2));
        acc[2] = gam * lk;
        acc[3] = gam * q1.y;
        {
            // n by the hardware square root (a gradient term needs no correctly rounded
            // n); a select, not a branch, for n = 0, so that the gathers of q2.w and q3
            // are not deferred behind it
            const float dx = X - q0.x, dy = Y - q0.y;
            const float t = fmaf(q0.w, dy, q0.z * dx);
            const float n = __builtin_amdgcn_sqrtf(fmaxf(fmaf(t, dx, q1.x * dy * dy), 0.0f));
            const float rho = n > 0.f ? -0.5f * gam * q1.y * __builtin_amdgcn_rcpf(n) : 0.f;
            const float ux = q2.w, uy = q3.x, ep = q3.y, em = q3.z;
            const float al = fmaf(ux, dx, uy * dy), be = fmaf(ux, dy, -(uy * dx));
            const float A = ep * al, B = em * be;
            const float r2 = 2.0f * rho;
            acc[0] = -r2 * fmaf(A, ux, -(B * uy));
            acc[1] = -r2 * fmaf(A, uy, B * ux);
            acc[9] = rho * fmaf(A, al, -(B * be));
            acc[7] = r2 * fmaf(A, dx, B * dy);
            acc[8] = r2 * fmaf(A, dy, -(B * dx));
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
                       p2 * (p2 + 2.0f * e2)) * (inv_P * pre);
        }
        const int slot = hash_slot(hkey, id);
        constexpr int nq = kRD ? kAcc : 10;
        // One range test per entry: the table takes all of the entry's terms when their
        // absolute sum is in range (a NaN fails the test and reaches global memory), else
        // every non-zero term goes to global memory.  Every term is added to the table
        // (zero when it goes global), so the adds are straight-line code.
        float asum = fabsf(acc[0]);
#pragma unroll
        for (int q = 1; q < nq; ++q) asum += fabsf(acc[q]);
        const bool in = slot >= 0 && asum < kHiLimit;
        const int sl = slot >= 0 ? slot : 0;
#pragma unroll
        for (int q = 0; q < nq; ++q) {
            // select the float, then convert: the empty asm keeps the compiler from
            // moving the select after the conversion (two 32-bit selects instead of one)
            float x = in ? acc[q] : 0.0f;
            asm("" : "+v"(x));
            atomicAdd(&hacc[q][sl], rint_i64(x));
        }
        if (!in) {
#pragma unroll
            for (int q = 0; q < nq; ++q) {
                if (acc[q] == 0.0f) continue;
                if (kDet && q < 10)
                    det_add_x(grad64_at(grad, q, id, cap, kSiteMajor), acc[q]);
                else
                    atomic_add_f32(q < 10 ? grad_at<kSiteMajor>(grad, q, id, cap) : rdel + id,
                                   acc[q] * fx.post);
            }
        }
    }
}

// Clear the tile table (one slot per thread of a 256-thread block).
template <int NQ = kAcc>
__device__ __forceinline__ void bwd_tile_init(uint32_t *__restrict__ hkey,
                                              unsigned long long (*hacc)[kHashSlots]) {
    const int t = threadIdx.x;
    hkey[t] = SAD_INVALID_ID;
#pragma unroll
    for (int q = 0; q < NQ; ++q) hacc[q][t] = 0ull;
}

// Flush the tile table: one float global atomic per occupied (site, parameter).  The
// occupied slots are first listed compactly; thread i then takes (slot i / nq, parameter
// i % nq), so that consecutive lanes add into consecutive parameters of one site (one
// cache line in the site-major layout).  Every thread of the block must call it.
// occ: LDS scratch of kHashSlots + 1 words (the list and its length).
template <bool kRD, bool kSiteMajor = false, bool kDet = false>
__device__ __forceinline__ void bwd_flush(const uint32_t *__restrict__ hkey,
                                          unsigned long long (*hacc)[kHashSlots],
                                          const FixScale &fx, int64_t cap,
                                          float *__restrict__ grad, float *__restrict__ rdel,
                                          uint32_t *__restrict__ occ) {
    static_assert(!(kRD && kDet), "the deterministic mode has no removal-delta channel");
    const int t = threadIdx.x;
    uint32_t &n_occ = occ[kHashSlots];
    if (t == 0) n_occ = 0;
    __syncthreads();
    if (hkey[t] != SAD_INVALID_ID) occ[atomicAdd(&n_occ, 1u)] = (uint32_t)t;
    __syncthreads();
    constexpr int nq = kRD ? kAcc : 10;
    const int n = (int)n_occ * nq;
    for (int i = t; i < n; i += kHashSlots) {
        const int j = i / nq, q = i - j * nq;
        const int sl = occ[j];
        const uint32_t id = hkey[sl];
        const unsigned long long u = hacc[q][sl];
        if (!u) continue;
        if (kDet && !(kRD && q == 10)) {  // already in the accumulator's units
            atomicAdd(reinterpret_cast<unsigned long long *>(
                          grad64_at(grad, q, id, cap, kSiteMajor)),
                      u);
            continue;
        }
        float *dst = (kRD && q == 10) ? rdel + id
                     : (kSiteMajor ? grad + (int64_t)id * SAD_NPARAM + q : grad + q * cap + id);
        atomic_add_f32(dst, from_fixed(u, fx.from_fix));
    }
}

// Fixed-point scale for an image of P pixels: 2^(40 + e) with 2^e ~ P / 2.
inline FixScale fix_scale(int64_t P) {
    const int e = fix_exponent(P);
    FixScale fx;
    fx.to_fix = std::ldexp(1.0, 32 + e);
    fx.from_fix = std::ldexp(1.0, -(32 + e));
    fx.limit = (float)std::ldexp(1.0, 15 - e);
    fx.to_det = std::ldexp(1.0, 40 + e - kGlobShift);
    fx.pre = std::ldexp(1.0f, 32 + e);
    fx.pre_det = std::ldexp(1.0f, 40 + e - kGlobShift);
    fx.post = std::ldexp(1.0f, -(32 + e));
    return fx;
}

}  // namespace sad
