// sad_device.h -- device-side building blocks shared by the gfx950 kernels.
//
// Score (Sec. 4.1-4.2), list keys, the injection generator and tile mapping.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "sad.h"

namespace sad {

// Derived record layout (SAD_REC_FLOATS = 16 floats = 64 bytes = four float4):
//   q0 = {x, y, G11, 2*G12}   q1 = {G22, kappa, r, valid}
//   q2 = {c_r, c_g, c_b, u_x} q3 = {u_y, e^a, e^-a, tau}
// The propagation pass reads q0..q1, the forward q0..q2, the backward all four.
constexpr int kRecQ = 4;

// Quadratic form q = d^T G d of the score (first half of score()).
__device__ __forceinline__ float quad(const float4 q0, const float4 q1, float X, float Y) {
    const float dx = __fsub_rn(X, q0.x);
    const float dy = __fsub_rn(Y, q0.y);
    const float t = __fmaf_rn(q0.w, dy, __fmul_rn(q0.z, dx));
    return fmaxf(__fmaf_rn(t, dx, __fmul_rn(__fmul_rn(q1.x, dy), dy)), 0.0f);
}

// l = kappa (r - ||x - p||_G), evaluated in float32 as
//   t = fma(2 G12, dy, G11 dx); q = fma(t, dx, (G22 dy) dy); q = max(q, 0);
//   n = sqrt(q); l = kappa (r - n) + 0
// with every operation correctly rounded (explicit _rn intrinsics; the TU is also
// compiled without contraction).  The square root is sqrtf, which the compiler expands
// to the hardware estimate plus an fma test of its two neighbours, i.e. correctly
// rounded; __fsqrt_rn compiles to the bare estimate (1 ulp) on this target and would
// let scores drift by an ulp from the reference sequence.  The trailing "+ 0" maps -0
// to +0.
__device__ __forceinline__ float score(const float4 q0, const float4 q1, float X, float Y,
                                       float *n_out = nullptr) {
    const float dx = __fsub_rn(X, q0.x);
    const float dy = __fsub_rn(Y, q0.y);
    const float t = __fmaf_rn(q0.w, dy, __fmul_rn(q0.z, dx));
    float q = __fmaf_rn(t, dx, __fmul_rn(__fmul_rn(q1.x, dy), dy));
    q = fmaxf(q, 0.0f);
    const float n = sqrtf(q);
    if (n_out) *n_out = n;
    return __fadd_rn(__fmul_rn(q1.y, __fsub_rn(q1.z, n)), 0.0f);
}

// Fixed-point scales of the backward for an image of P pixels, 2^e ~ P / 2 (every
// gradient term carries the 1/P of dL/dc): the LDS tile table counts in 2^-(40 + e),
// the deterministic global accumulator in det_grad_unit(P) = 2^-(40 + e - kGlobShift).
constexpr int kGlobShift = 20;
__host__ __device__ inline int fix_exponent(int64_t P) {
    int e = 0;
    while ((int64_t)1 << (e + 1) < P) ++e;
    return e;
}
__host__ __device__ inline double det_grad_unit(int64_t P) {
    return ldexp(1.0, -(40 + fix_exponent(P) - kGlobShift));
}

// Total order (score descending, ID ascending) as one unsigned 64-bit key: the high
// word is the score's bits made monotone, the low word ~ID.  Key 0 is "empty" (no
// finite or infinite score maps to 0) and ~0 of an empty key's low word is the
// sentinel 0xFFFFFFFF.
__device__ __forceinline__ uint64_t make_key(float l, uint32_t id) {
    const uint32_t b = __float_as_uint(l);
    const uint32_t o = b ^ ((uint32_t)((int32_t)b >> 31) | 0x80000000u);
    return ((uint64_t)o << 32) | (uint32_t)(~id);
}
__device__ __forceinline__ uint32_t key_id(uint64_t k) { return ~(uint32_t)k; }
__device__ __forceinline__ float key_score(uint64_t k) {
    const uint32_t o = (uint32_t)(k >> 32);
    const uint32_t b = (o & 0x80000000u) ? (o ^ 0x80000000u) : ~o;
    return __uint_as_float(b);
}

// Insert candidate key c into keys[0..K-1] (descending, unique, 0 = empty): bubble it
// down; an equal key is a repeated ID and is dropped.
template <int K>
__device__ __forceinline__ void insert_key(uint64_t (&keys)[K], uint64_t c) {
    if (c > keys[K - 1]) {
#pragma unroll
        for (int j = 0; j < K; ++j) {
            const uint64_t kj = keys[j];
            const bool gt = c > kj;
            const bool eq = c == kj;
            keys[j] = gt ? c : kj;
            c = gt ? kj : (eq ? 0ull : c);
        }
    }
}

// Sort keys[] descending with Batcher's odd-even merge network (Knuth TAOCP vol. 3,
// 5.3.4); K is padded to the next power of two with empty (zero) keys.
template <int K>
struct Pow2 {
    static constexpr int v = K <= 4 ? 4 : K <= 8 ? 8 : K <= 16 ? 16 : 32;
};

template <int N>
__device__ __forceinline__ void ce_desc(uint64_t (&a)[N], int x, int y) {
    const uint64_t ax = a[x], ay = a[y];
    const bool sw = ax < ay;
    a[x] = sw ? ay : ax;
    a[y] = sw ? ax : ay;
}

template <int K>
__device__ __forceinline__ void sort_keys_desc(uint64_t (&keys)[K]) {
    constexpr int N = Pow2<K>::v;
    uint64_t a[N];
#pragma unroll
    for (int i = 0; i < N; ++i) a[i] = i < K ? keys[i] : 0ull;
#pragma unroll
    for (int p = 1; p < N; p <<= 1)
#pragma unroll
        for (int k = p; k >= 1; k >>= 1)
#pragma unroll
            for (int j = k % p; j + k < N; j += 2 * k)
#pragma unroll
                for (int i = 0; i < k; ++i)
                    if (i < N - j - k && (i + j) / (2 * p) == (i + j + k) / (2 * p))
                        ce_desc<N>(a, i + j, i + j + k);
#pragma unroll
    for (int i = 0; i < K; ++i) keys[i] = a[i];
}

// SplitMix64 (Steele, Lea, Flood 2014): output number k of the stream seeded by seed.
__device__ __forceinline__ uint64_t splitmix64(uint64_t seed, uint64_t k) {
    uint64_t z = seed + (k + 1ull) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// Evaluation grids (App. B.3 "Downscaled candidate grid").  A list field may live on a
// grid of n_grid cells along an axis of n_img pixels.  Cell j is evaluated at the centre
// of its UV interval, (j + 1/2) / n_grid, which in pixel units (pixel j at coordinate j)
// is ((2 j + 1) n_img - n_grid) / (2 n_grid): a ratio of exact integers divided in
// double and rounded once to float; on the image's own grid it is j exactly.
__host__ __device__ __forceinline__ float grid_point(int j, int n_img, int n_grid) {
    if (n_img == n_grid) return (float)j;
    const double num = (double)(2 * (int64_t)j + 1) * (double)n_img - (double)n_grid;
    return (float)(num / (2.0 * (double)n_grid));
}
// The integer map from an axis of n_from points to n_to cells: point j lies in the cell
// whose UV interval holds its UV centre, floor((2 j + 1) n_to / (2 n_from)); for
// n_from = s n_to that is floor(j / s), and the identity when the two are equal.
__host__ __device__ __forceinline__ int cell_of(int j, int n_from, int n_to) {
    return (int)(((2 * (int64_t)j + 1) * (int64_t)n_to) / (2 * (int64_t)n_from));
}

// Workgroups are handed to the eight XCDs round-robin (block b runs on XCD b % 8).
// Remap so that each XCD works through one contiguous range of tiles: neighbouring
// tiles then share that XCD's L2 (site records and neighbour lists).
__device__ __forceinline__ int xcd_tile(int bid, int nblk) {
    constexpr int X = 8;
    const int q = nblk / X, r = nblk % X;
    const int xcd = bid % X, k = bid / X;
    const int base = xcd < r ? xcd * (q + 1) : r * (q + 1) + (xcd - r) * q;
    return base + k;
}

// 16x16-pixel tile of 256 threads: four wave64s, each an 8x8 block.
struct TilePix {
    int i, j;
};
__device__ __forceinline__ TilePix tile_pixel(int tile, int tiles_x) {
    const int ty = tile / tiles_x, tx = tile - ty * tiles_x;
    const int t = threadIdx.x;
    const int w = t >> 6, l = t & 63;
    TilePix p;
    p.i = ty * 16 + (w >> 1) * 8 + (l >> 3);
    p.j = tx * 16 + (w & 1) * 8 + (l & 7);
    return p;
}

// The same for a tile TW pixels wide and 256 / TW tall, still four 8x8 wave64 blocks
// (TW = 16: 2 x 2 blocks, tile_pixel's mapping; TW = 32: 4 x 1 blocks).
template <int TW>
__device__ __forceinline__ TilePix tile_pixel_w(int tile, int tiles_x) {
    static_assert(TW == 16 || TW == 32, "tiles are 16 x 16 or 32 x 8");
    constexpr int TH = 256 / TW, WX = TW / 8;
    const int ty = tile / tiles_x, tx = tile - ty * tiles_x;
    const int t = threadIdx.x;
    const int w = t >> 6, l = t & 63;
    TilePix p;
    p.i = ty * TH + (w / WX) * 8 + (l >> 3);
    p.j = tx * TW + (w % WX) * 8 + (l & 7);
    return p;
}

__device__ __forceinline__ void atomic_add_f32(float *p, float v) { unsafeAtomicAdd(p, v); }

}  // namespace sad
