// budget.hip -- adaptive budget on the GPU (Sec. 4.5, App. B.5): the per-site
// statistics pass, and one prune / split step with list seeding.
//
// Statistics: one 256-thread block per 16x16 tile, the per-tile LDS hash of the
// backward keyed by site ID, eight 64-bit fixed-point accumulators per slot (a scale
// per statistic), one float global atomic per occupied (site, statistic) at the end.
//
// Budget step: per-slot kernels and two radix selections over 64-bit keys
// (value bits made monotone << 32 | ~slot, so ties go to the lower slot):
//   count active + prune keys -> select -> prune, split keys, candidates -> select ->
//   parent / free flags -> two exclusive scans -> free list -> split -> seed -> counts.
// The split geometry is evaluated per parent in double.
#include <cmath>

#include "sad_device.h"
#include "sad_host.h"
#include "sad_internal.h"
#include "sad_kernels.h"

namespace sad {

// ---- statistics ---------------------------------------------------------------------
constexpr int kNStat = SAD_NSTAT;

// Fixed-point scale 2^s of each statistic.  A tile adds at most 256 terms into one
// slot, so terms with |v| < 2^(54 - s) keep the 64-bit sum below 2^62; larger terms go
// straight to a float global atomic.  The removal delta carries 1/P and uses 2^(40+e),
// 2^e ~ P / 2, as the backward does.
struct StatScale {
    double to[kNStat];
    double from[kNStat];
    float limit[kNStat];
};

static StatScale stat_scale(int64_t P) {
    int e = 0;
    while ((int64_t)1 << (e + 1) < P) ++e;
    const int ex[kNStat] = {40, 40, 36, 36, 30, 30, 30, 40 + e};
    StatScale sc;
    for (int q = 0; q < kNStat; ++q) {
        sc.to[q] = std::ldexp(1.0, ex[q]);
        sc.from[q] = std::ldexp(1.0, -ex[q]);
        sc.limit[q] = (float)std::ldexp(1.0, 54 - ex[q]);
    }
    return sc;
}

// Exact 128-bit sum in two 64-bit planes: lo accumulates modulo 2^64 and hi takes each
// add's carry out of lo plus the sign extension of the term, so hi * 2^64 + lo is the
// integer sum of the terms whatever the order of the adds.
__device__ __forceinline__ void wide_add(unsigned long long *__restrict__ lo,
                                         unsigned long long *__restrict__ hi, int64_t idx,
                                         long long u) {
    const unsigned long long old = atomicAdd(lo + idx, (unsigned long long)u);
    const long long hd = (old + (unsigned long long)u < old ? 1 : 0) + (u < 0 ? -1 : 0);
    if (hd) atomicAdd(hi + idx, (unsigned long long)hd);
}

// A term in units of 2^-s, rounded once (clamped to +-2^62; below the LDS limit this is
// the same integer to_fixed forms).
__device__ __forceinline__ long long fixed_term(float v, double to) {
    double x = rint((double)v * to);
    x = fmin(fmax(x, -0x1p62), 0x1p62);
    return (long long)x;
}

// kFixed: every term is rounded once to its statistic's unit and every sum is an
// integer (tile sums in LDS, the sum over tiles exact in acc = lo[8][cap], hi[8][cap]),
// so the sums do not depend on the order in which tiles and lanes add.
// Register budgets: four waves per SIMD up to K = 8 (K = 8 needs 132 registers
// uncapped, three waves; capped 128 and 5 spilled: 12 % less time at 2048x2048) and
// two for K = 12..16 (K = 16 needs 262 uncapped, one wave; capped 254 and 6 spilled:
// 42 % less time at 2048x2048) -- more waves to hide the record gathers.
template <int K, bool kFixed>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(K <= 8 ? 4 : (K <= 16 ? 2 : 1), 8))) void k_stats(ImgArgs a, StatScale sc,
                                               const float4 *__restrict__ rec,
                                               const uint4 *__restrict__ topk,
                                               const float *__restrict__ tgt,
                                               float *__restrict__ stats,
                                               unsigned long long *__restrict__ acc) {
    unsigned long long *acc_hi = acc + (int64_t)kNStat * a.cap;
    __shared__ uint32_t hkey[kHashSlots];
    __shared__ unsigned long long hacc[kNStat][kHashSlots];
    const int t = threadIdx.x;
    hkey[t] = SAD_INVALID_ID;
#pragma unroll
    for (int q = 0; q < kNStat; ++q) hacc[q][t] = 0ull;
    __syncthreads();

    const int tile = xcd_tile(blockIdx.x, a.n_blocks);
    const TilePix px = tile_pixel(tile, a.tiles_x);
    if (px.i < a.H && px.j < a.W) {
        const int64_t P = (int64_t)a.H * a.W, p = (int64_t)px.i * a.W + px.j;
        const float X = (float)px.j, Y = (float)px.i;
        PixelBlend<K> b;
        blend<K, true>(rec, (uint32_t)a.n_slots, topk, P, p, X, Y, b, lane_rot() % K);
        if (b.nv) {
            const float invS = __builtin_amdgcn_rcpf(b.S);
            const float e0 = b.c[0] - tgt[p], e1 = b.c[1] - tgt[P + p], e2 = b.c[2] - tgt[2 * P + p];
            const float err = e0 * e0 + e1 * e1 + e2 * e2;
            // removal delta with the reference entry r (largest score), as in the
            // backward: c'_k - c = -w_k / (1 - w_k) (c_k - c) for k != r, and c'_r from
            // the softmax of the others
            const int r = b.r;
            const float cr0 = b.cr[0], cr1 = b.cr[1], cr2 = b.cr[2];
            const float dc0 = b.dc[0], dc1 = b.dc[1], dc2 = b.dc[2];
            float dr0, dr1, dr2;
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
            } else {
                dr0 = -b.c[0];
                dr1 = -b.c[1];
                dr2 = -b.c[2];
            }
#pragma unroll
            for (int k = 0; k < K; ++k) {
                const float w = b.e[k] * invS;
                // every statistic of an entry is a multiple of its weight (the removal
                // delta of a non-reference entry too): weight 0 adds exactly 0
                if (!b.ok[k] || w == 0.0f) continue;
                const uint32_t id = b.id[k];
                const float4 q0 = rec[4 * (size_t)id];
                const float4 q2 = rec[4 * (size_t)id + 2];
                const float om = w * err;
                const float dx = X - q0.x, dy = Y - q0.y;
                float p0, p1, p2;
                if (k == r) {
                    p0 = dr0;
                    p1 = dr1;
                    p2 = dr2;
                } else {
                    const float f = -w * __builtin_amdgcn_rcpf(1.0f - w);
                    p0 = f * ((q2.x - cr0) - dc0);
                    p1 = f * ((q2.y - cr1) - dc1);
                    p2 = f * ((q2.z - cr2) - dc2);
                }
                float v[kNStat];
                v[0] = w;
                v[1] = om;
                v[2] = om * dx;
                v[3] = om * dy;
                v[4] = v[2] * dx;
                v[5] = v[2] * dy;
                v[6] = v[3] * dy;
                v[7] = (p0 * (p0 + 2.0f * e0) + p1 * (p1 + 2.0f * e1) + p2 * (p2 + 2.0f * e2)) *
                       a.inv_P;
                const int slot = hash_slot(hkey, id);
#pragma unroll
                for (int q = 0; q < kNStat; ++q) {
                    if (slot >= 0 && fabsf(v[q]) < sc.limit[q])
                        atomicAdd(&hacc[q][slot], to_fixed(v[q], sc.to[q]));
                    else if (v[q] != 0.0f) {
                        if (kFixed)
                            wide_add(acc, acc_hi, q * a.cap + id, fixed_term(v[q], sc.to[q]));
                        else
                            atomic_add_f32(stats + q * a.cap + id, v[q]);
                    }
                }
            }
        }
    }
    __syncthreads();
    const uint32_t id = hkey[t];
    if (id == SAD_INVALID_ID) return;
#pragma unroll
    for (int q = 0; q < kNStat; ++q) {
        const unsigned long long u = hacc[q][t];
        if (!u) continue;
        if (kFixed)  // a tile sum is below 2^62 in magnitude: one signed 64-bit term
            wide_add(acc, acc_hi, q * a.cap + id, (long long)u);
        else
            atomic_add_f32(stats + q * a.cap + id, from_fixed(u, sc.from[q]));
    }
}

__global__ __launch_bounds__(256) void k_zero_u64(unsigned long long *__restrict__ p, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0ull;
}

// stats[q][i] = (hi * 2^64 + lo) * 2^-s_q, rounded to float (through double: the same
// exact sum always gives the same float).  With lo read as signed, the sum is
// (hi + [lo < 0]) * 2^64 + lo_signed; a sum that fits in 64 bits (high part 0) is
// converted from the signed low word directly, so small negative sums do not cancel
// against 2^64 (unsigned lo just below 2^64 would round to a multiple of 2^12 units).
__global__ __launch_bounds__(256) void k_stats_out(StatScale sc, const unsigned long long *__restrict__ acc,
                                                  int64_t cap, float *__restrict__ stats) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= kNStat * cap) return;
    const int q = (int)(i / cap);
    const long long lo = (long long)acc[i];
    const long long hi = (long long)acc[kNStat * cap + i] + (lo < 0 ? 1 : 0);
    const double sum = hi == 0 ? (double)lo : fma((double)hi, 0x1p64, (double)lo);
    stats[i] = (float)(sum * sc.from[q]);
}

// ---- budget step --------------------------------------------------------------------
struct DPState {
    SelState sp, ss;                 // prune / split selections
    unsigned long long n_active, n_cand, want_p, want_s, hw;
};

__device__ __forceinline__ bool slot_active(const float *__restrict__ sites, int64_t cap,
                                            int64_t i) {
    bool fin = true;
#pragma unroll
    for (int q = 0; q < SAD_NPARAM; ++q) fin = fin && isfinite(sites[q * cap + i]);
    return fin && sites[i] >= 0.0f;
}

__device__ __forceinline__ uint32_t ord_f32(float f) {
    const uint32_t b = __float_as_uint(f);
    return b ^ ((uint32_t)((int32_t)b >> 31) | 0x80000000u);
}
// larger value first, then lower slot
__device__ __forceinline__ uint64_t key_desc(float v, int64_t i) {
    return ((uint64_t)ord_f32(v) << 32) | (uint32_t)(~(uint32_t)i);
}
// smaller value first, then lower slot
__device__ __forceinline__ uint64_t key_asc(float v, int64_t i) {
    return ((uint64_t)(~ord_f32(v)) << 32) | (uint32_t)(~(uint32_t)i);
}

// Sum of a per-thread count over the block, added to *dst by one thread.
__device__ __forceinline__ void block_count_add(uint32_t c, unsigned long long *dst) {
    for (int o = 32; o > 0; o >>= 1) c += __shfl_xor(c, o);
    __shared__ uint32_t part[4];
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = c;
    __syncthreads();
    if (threadIdx.x == 0) {
        const uint32_t s = part[0] + part[1] + part[2] + part[3];
        if (s) atomicAdd(dst, (unsigned long long)s);
    }
}

__global__ __launch_bounds__(256) void k_dp_begin(DPState *st, uint32_t *hist) {
    if (threadIdx.x == 0) {
        st->sp.prefix = st->sp.mask = 0;
        st->ss.prefix = st->ss.mask = 0;
        st->sp.want = st->ss.want = 1;
        st->sp.pad = st->ss.pad = 0;
        st->n_active = st->n_cand = st->want_p = st->want_s = st->hw = 0;
    }
    hist[threadIdx.x] = 0u;
}

__global__ __launch_bounds__(256) void k_dp_count(const float *__restrict__ sites, int64_t cap,
                                                  const float *__restrict__ stats,
                                                  uint64_t *__restrict__ key_p,
                                                  DPState *__restrict__ st) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    uint32_t c = 0;
    if (i < cap) {
        const bool act = slot_active(sites, cap, i);
        key_p[i] = act ? key_asc(stats[7 * cap + i], i) : 0ull;
        c = act ? 1u : 0u;
    }
    block_count_add(c, &st->n_active);
}

__global__ void k_dp_want_prune(DPState *st, double p_prune, int on) {
    const unsigned long long n = st->n_active;
    unsigned long long w = on ? (unsigned long long)floor(p_prune * (double)n) : 0ull;
    if (w > n) w = n;
    st->want_p = w;
    st->sp.want = w ? (uint32_t)w : 1u;
}

__global__ __launch_bounds__(256) void k_dp_prune(float *__restrict__ sites, int64_t cap,
                                                  const float *__restrict__ stats,
                                                  const uint64_t *__restrict__ key_p,
                                                  uint64_t *__restrict__ key_s,
                                                  DPState *__restrict__ st, double alpha,
                                                  double eps, double min_mass) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    uint32_t c = 0;
    if (i < cap) {
        const uint64_t kp = key_p[i];
        const bool pruned = st->want_p && kp && kp >= st->sp.prefix;
        if (pruned) {
            sites[i] = -1.0f;
            sites[cap + i] = -1.0f;
        }
        uint64_t ks = 0ull;
        const double m = (double)stats[i];
        if (kp && !pruned && m > min_mass) {
            const double sc = (double)stats[cap + i] / pow(m > eps ? m : eps, alpha);
            ks = key_desc((float)sc, i);
            c = 1u;
        }
        key_s[i] = ks;
    }
    block_count_add(c, &st->n_cand);
}

__global__ void k_dp_want_split(DPState *st, int64_t cap, double p_split, int on) {
    const unsigned long long n = st->n_active;
    const unsigned long long n_free = (unsigned long long)cap - n + st->want_p;
    unsigned long long w = on ? (unsigned long long)floor(p_split * (double)n) : 0ull;
    if (w > st->n_cand) w = st->n_cand;
    if (w > n_free) w = n_free;
    st->want_s = w;
    st->ss.want = w ? (uint32_t)w : 1u;
}

__device__ __forceinline__ bool is_parent(const uint64_t *__restrict__ key_s, int64_t i,
                                          const DPState *__restrict__ st) {
    const uint64_t k = key_s[i];
    return st->want_s && k && k >= st->ss.prefix;
}

__global__ __launch_bounds__(256) void k_dp_flags(const float *__restrict__ sites, int64_t cap,
                                                  const uint64_t *__restrict__ key_s,
                                                  const DPState *__restrict__ st,
                                                  uint32_t *__restrict__ fpar,
                                                  uint32_t *__restrict__ ffree) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= cap) return;
    fpar[i] = is_parent(key_s, i, st) ? 1u : 0u;
    ffree[i] = slot_active(sites, cap, i) ? 0u : 1u;
}

__global__ __launch_bounds__(256) void k_dp_free_list(const float *__restrict__ sites,
                                                      int64_t cap,
                                                      const uint32_t *__restrict__ rfree,
                                                      const DPState *__restrict__ st,
                                                      uint32_t *__restrict__ free_list) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= cap) return;
    const uint32_t r = rfree[i];
    if (r < st->want_s && !slot_active(sites, cap, i)) free_list[r] = (uint32_t)i;
}

__device__ __forceinline__ double clampd(double v, double lo, double hi) {
    return v < lo ? lo : (v > hi ? hi : v);
}

__device__ __forceinline__ int64_t nearest_pixel(int H, int W, double x, double y) {
    const double fi = rint(y), fj = rint(x);
    const int64_t i = fi > 0 ? (fi > H - 1 ? H - 1 : (int64_t)fi) : 0;
    const int64_t j = fj > 0 ? (fj > W - 1 ? W - 1 : (int64_t)fj) : 0;
    return i * W + j;
}

// Principal axis of [[a, b], [b, c]] (eigenvalues l1 >= l2, unit eigenvector of l1 with
// its first non-zero component positive); false when the trace is <= 1e-9 or the
// eigenvalue gap 2 disc is <= 2e-6 of the trace.
__device__ __forceinline__ bool principal_axis(double a, double b, double c, double &ex,
                                               double &ey, double &l1, double &l2) {
    const double h = 0.5 * (a - c), tr = a + c;
    const double disc = sqrt(h * h + b * b);
    if (!(tr > 1e-9) || !(disc > 1e-6 * tr)) return false;
    l1 = 0.5 * tr + disc;
    l2 = 0.5 * tr - disc;
    double vx, vy;
    if (a >= c) {
        vx = l1 - c;
        vy = b;
    } else {
        vx = b;
        vy = l1 - a;
    }
    const double nv = sqrt(vx * vx + vy * vy);
    vx /= nv;
    vy /= nv;
    if (vx < 0 || (vx == 0 && vy < 0)) {
        vx = -vx;
        vy = -vy;
    }
    ex = vx;
    ey = vy;
    return true;
}

__global__ __launch_bounds__(256) void k_dp_split(float *__restrict__ sites, int64_t cap,
                                                  float *__restrict__ am, float *__restrict__ av,
                                                  const float *__restrict__ stats,
                                                  const float *__restrict__ tgt, int H, int W,
                                                  const uint64_t *__restrict__ key_s,
                                                  const uint32_t *__restrict__ rpar,
                                                  const uint32_t *__restrict__ free_list,
                                                  const DPState *__restrict__ st) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= cap || !is_parent(key_s, i, st)) return;
    const int64_t c = free_list[rpar[i]];
    const int64_t P = (int64_t)H * W;
    float par[SAD_NPARAM];
#pragma unroll
    for (int q = 0; q < SAD_NPARAM; ++q) par[q] = sites[q * cap + i];
    const double m = stats[i], E = stats[cap + i];
    const double delta = clampd(0.5 * sqrt(m), 1.5, 48.0);
    const double px = par[0], py = par[1];
    double cx = px, cy = py, ex = 0, ey = 0, l1 = 0, l2 = 0;
    double ux = par[7], uy = par[8], a = par[9];
    bool have = false;
    if (E > 1e-12) {
        const double mx = (double)stats[2 * cap + i] / E, my = (double)stats[3 * cap + i] / E;
        const double cxx = (double)stats[4 * cap + i] / E - mx * mx;
        const double cxy = (double)stats[5 * cap + i] / E - mx * my;
        const double cyy = (double)stats[6 * cap + i] / E - my * my;
        if (principal_axis(cxx, cxy, cyy, ex, ey, l1, l2)) {
            have = true;
            cx = px + mx;
            cy = py + my;
            ux = ex;
            uy = ey;
            a = l2 > 0 ? clampd(0.5 * log(l2 / l1), -2.0, 2.0) : -2.0;
        }
    }
    if (!have) {  // Sobel structure tensor of the target at the site's pixel
        const int64_t q = nearest_pixel(H, W, px, py);
        const int64_t y = q / W, x = q - y * W;
        const int64_t ym = y > 0 ? y - 1 : 0, yp = y + 1 < H ? y + 1 : H - 1;
        const int64_t xm = x > 0 ? x - 1 : 0, xp = x + 1 < W ? x + 1 : W - 1;
        double txx = 0, txy = 0, tyy = 0;
        for (int ch = 0; ch < 3; ++ch) {
            const float *I = tgt + ch * P;
            auto T = [&](int64_t r, int64_t cc) { return (double)I[r * W + cc]; };
            const double gx = (T(ym, xp) + 2.0 * T(y, xp) + T(yp, xp)) -
                              (T(ym, xm) + 2.0 * T(y, xm) + T(yp, xm));
            const double gy = (T(yp, xm) + 2.0 * T(yp, x) + T(yp, xp)) -
                              (T(ym, xm) + 2.0 * T(ym, x) + T(ym, xp));
            txx += gx * gx;
            txy += gx * gy;
            tyy += gy * gy;
        }
        if (!principal_axis(txx, txy, tyy, ex, ey, l1, l2)) {
            const double nu = sqrt(ux * ux + uy * uy);
            if (nu > 0) {
                ex = ux / nu;
                ey = uy / nu;
            } else {
                ex = 1.0;
                ey = 0.0;
            }
        }
        a = 0.8 * a;
    }
    const double lt = clampd((double)par[2] - 0.25, 2.0, 20.0);
    const double rr = clampd(0.85 * (double)par[3], 1.0, 512.0);
#pragma unroll
    for (int kid = 0; kid < 2; ++kid) {
        const int64_t s = kid == 0 ? i : c;
        const double sg = kid == 0 ? 1.0 : -1.0;
        const float x = (float)clampd(cx + sg * delta * ex, 0.0, (double)(W - 1));
        const float y = (float)clampd(cy + sg * delta * ey, 0.0, (double)(H - 1));
        const int64_t q = nearest_pixel(H, W, (double)x, (double)y);
        const float o[SAD_NPARAM] = {x, y, (float)lt, (float)rr, tgt[q], tgt[P + q], tgt[2 * P + q],
                                     (float)ux, (float)uy, (float)a};
#pragma unroll
        for (int p = 0; p < SAD_NPARAM; ++p) {
            sites[p * cap + s] = o[p];
            if (am) am[p * cap + s] = 0.0f;
            if (av) av[p * cap + s] = 0.0f;
        }
    }
}

// Seeding, two kernels: first every "-" child clears entry K-1 at its pixel, then each
// writes its slot with atomicMin, so the smallest slot wins (SAD_INVALID_ID is the
// largest value).
__global__ __launch_bounds__(256) void k_dp_seed(const float *__restrict__ sites, int64_t cap,
                                                 const uint64_t *__restrict__ key_s,
                                                 const uint32_t *__restrict__ rpar,
                                                 const uint32_t *__restrict__ free_list,
                                                 const DPState *__restrict__ st, int H, int W,
                                                 int K, uint32_t *__restrict__ topk, int phase) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= cap || !is_parent(key_s, i, st)) return;
    const uint32_t c = free_list[rpar[i]];
    const int64_t q = nearest_pixel(H, W, (double)sites[c], (double)sites[cap + c]);
    const int64_t P = (int64_t)H * W;
    uint32_t *e = topk + ((int64_t)(K / 4 - 1) * P + q) * 4 + 3;
    if (phase == 0)
        *e = SAD_INVALID_ID;
    else
        atomicMin(e, c);
}

__global__ __launch_bounds__(256) void k_dp_hw(const float *__restrict__ sites, int64_t cap,
                                               DPState *__restrict__ st) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    unsigned long long h = (i < cap && slot_active(sites, cap, i)) ? (unsigned long long)(i + 1) : 0ull;
    for (int o = 32; o > 0; o >>= 1) {
        const unsigned long long g = __shfl_xor(h, o);
        h = g > h ? g : h;
    }
    if ((threadIdx.x & 63) == 0 && h) atomicMax(&st->hw, h);
}

__global__ void k_dp_counts(const DPState *__restrict__ st, int64_t *__restrict__ counts) {
    counts[0] = (int64_t)st->n_active;
    counts[1] = (int64_t)st->want_p;
    counts[2] = (int64_t)st->want_s;
    counts[3] = (int64_t)(st->n_active - st->want_p + st->want_s);
    counts[4] = (int64_t)st->hw;
    counts[5] = (int64_t)st->n_cand;
}

static size_t align_up(size_t x) { return (x + 255) & ~(size_t)255; }

}  // namespace sad

using namespace sad;

extern "C" sad_status sad_site_stats(const sad_image *img, const float *rec, const uint32_t *topk,
                                     const float *target, float *stats, void *stream) {
    SAD_TRY(check_image(img, nullptr));
    SAD_REQUIRE(stats && target, SAD_ERR_INVALID_ARGUMENT, "sad_site_stats: NULL pointer");
    if (img->n_slots == 0) return SAD_OK;
    SAD_REQUIRE(rec && topk, SAD_ERR_INVALID_ARGUMENT, "sad_site_stats: NULL pointer");
    SAD_REQUIRE(aligned16(rec) && aligned16(topk), SAD_ERR_INVALID_ARGUMENT,
                "sad_site_stats: rec and topk must be 16-byte aligned");
    const ImgArgs a = img_args(img);
    const StatScale sc = stat_scale((int64_t)img->H * img->W);
    hipStream_t st = as_stream(stream);
    const float4 *r4 = reinterpret_cast<const float4 *>(rec);
    const uint4 *l4 = reinterpret_cast<const uint4 *>(topk);
    SAD_K_SWITCH(img->K, hipLaunchKernelGGL((k_stats<KK, false>), dim3(a.n_blocks), dim3(256), 0,
                                            st, a, sc, r4, l4, target, stats, nullptr));
    return check_launch("sad_site_stats");
}

extern "C" sad_status sad_site_stats_fixed(const sad_image *img, const float *rec,
                                           const uint32_t *topk, const float *target,
                                           int64_t *acc, float *stats, void *stream) {
    SAD_TRY(check_image(img, nullptr));
    SAD_REQUIRE(stats && target && acc, SAD_ERR_INVALID_ARGUMENT,
                "sad_site_stats_fixed: NULL pointer");
    SAD_REQUIRE(((uintptr_t)acc & 7) == 0, SAD_ERR_INVALID_ARGUMENT,
                "sad_site_stats_fixed: acc must be 8-byte aligned");
    if (img->n_slots > 0)
        SAD_REQUIRE(rec && topk && aligned16(rec) && aligned16(topk), SAD_ERR_INVALID_ARGUMENT,
                    "sad_site_stats_fixed: rec and topk must be non-NULL and 16-byte aligned");
    const ImgArgs a = img_args(img);
    const StatScale sc = stat_scale((int64_t)img->H * img->W);
    hipStream_t st = as_stream(stream);
    unsigned long long *acc64 = reinterpret_cast<unsigned long long *>(acc);
    const int64_t n = 2ll * kNStat * img->cap, n_out = (int64_t)kNStat * img->cap;
    if (n > 0)
        hipLaunchKernelGGL(k_zero_u64, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, acc64,
                           n);
    if (img->n_slots > 0) {
        const float4 *r4 = reinterpret_cast<const float4 *>(rec);
        const uint4 *l4 = reinterpret_cast<const uint4 *>(topk);
        SAD_K_SWITCH(img->K, hipLaunchKernelGGL((k_stats<KK, true>), dim3(a.n_blocks), dim3(256),
                                                0, st, a, sc, r4, l4, target, stats, acc64));
    }
    if (n_out > 0)
        hipLaunchKernelGGL(k_stats_out, dim3((unsigned)((n_out + 255) / 256)), dim3(256), 0, st,
                           sc, acc64, (int64_t)img->cap, stats);
    return check_launch("sad_site_stats_fixed");
}

extern "C" sad_status sad_densify_prune(const sad_image *img, const float *target, float *sites,
                                        float *adam_m, float *adam_v, const float *stats,
                                        const sad_budget_params *prm, uint32_t *topk,
                                        int64_t *counts, void *workspace,
                                        size_t *workspace_bytes, void *stream) {
    SAD_TRY(check_image(img, nullptr));
    SAD_REQUIRE(workspace_bytes, SAD_ERR_INVALID_ARGUMENT,
                "sad_densify_prune: workspace_bytes is NULL");
    const int64_t cap = img->cap;
    const int64_t nbs = scan_blocks(cap > 0 ? cap : 1);
    const size_t off_st = 0;
    const size_t off_hist = align_up(off_st + sizeof(DPState));
    const size_t off_kp = align_up(off_hist + 256 * 4);
    const size_t off_ks = align_up(off_kp + 8 * (size_t)cap);
    const size_t off_rp = align_up(off_ks + 8 * (size_t)cap);
    const size_t off_rf = align_up(off_rp + 4 * (size_t)cap);
    const size_t off_fl = align_up(off_rf + 4 * (size_t)cap);
    const size_t off_bt = align_up(off_fl + 4 * (size_t)cap);
    const size_t need = align_up(off_bt + 4 * (size_t)nbs);
    if (!workspace) {
        *workspace_bytes = need;
        return SAD_OK;
    }
    SAD_REQUIRE(*workspace_bytes >= need, SAD_ERR_WORKSPACE,
                "sad_densify_prune: workspace too small (%zu < %zu)", *workspace_bytes, need);
    SAD_REQUIRE(prm, SAD_ERR_INVALID_ARGUMENT, "sad_densify_prune: params is NULL");
    SAD_REQUIRE(target && sites && stats && counts, SAD_ERR_INVALID_ARGUMENT,
                "sad_densify_prune: NULL pointer");
    SAD_REQUIRE((prm->flags & ~(SAD_DP_PRUNE | SAD_DP_SPLIT | SAD_DP_SEED)) == 0,
                SAD_ERR_INVALID_ARGUMENT, "sad_densify_prune: unknown flags 0x%x", prm->flags);
    SAD_REQUIRE(prm->p_prune >= 0.0 && prm->p_prune <= 1.0 && prm->p_split >= 0.0 &&
                    prm->p_split <= 1.0,
                SAD_ERR_INVALID_ARGUMENT, "sad_densify_prune: fractions must be in [0, 1]");
    SAD_REQUIRE(prm->alpha >= 0.0 && prm->eps > 0.0 && prm->min_mass == prm->min_mass,
                SAD_ERR_INVALID_ARGUMENT, "sad_densify_prune: bad alpha / eps / min_mass");
    SAD_REQUIRE(!(prm->flags & SAD_DP_SEED) || (topk && aligned16(topk)),
                SAD_ERR_INVALID_ARGUMENT,
                "sad_densify_prune: seeding needs a 16-byte aligned topk");
    hipStream_t st = as_stream(stream);
    char *ws = static_cast<char *>(workspace);
    DPState *dp = reinterpret_cast<DPState *>(ws + off_st);
    uint32_t *hist = reinterpret_cast<uint32_t *>(ws + off_hist);
    uint64_t *key_p = reinterpret_cast<uint64_t *>(ws + off_kp);
    uint64_t *key_s = reinterpret_cast<uint64_t *>(ws + off_ks);
    uint32_t *rpar = reinterpret_cast<uint32_t *>(ws + off_rp);
    uint32_t *rfree = reinterpret_cast<uint32_t *>(ws + off_rf);
    uint32_t *flist = reinterpret_cast<uint32_t *>(ws + off_fl);
    uint32_t *btot = reinterpret_cast<uint32_t *>(ws + off_bt);
    const unsigned nb = (unsigned)((cap + 255) / 256);
    hipLaunchKernelGGL(k_dp_begin, dim3(1), dim3(256), 0, st, dp, hist);
    if (cap == 0) {
        hipLaunchKernelGGL(k_dp_counts, dim3(1), dim3(1), 0, st, dp, counts);
        return check_launch("sad_densify_prune");
    }
    hipLaunchKernelGGL(k_dp_count, dim3(nb), dim3(256), 0, st, sites, cap, stats, key_p, dp);
    hipLaunchKernelGGL(k_dp_want_prune, dim3(1), dim3(1), 0, st, dp, prm->p_prune,
                       (prm->flags & SAD_DP_PRUNE) ? 1 : 0);
    launch_radix_select(key_p, cap, &dp->sp, hist, st);
    hipLaunchKernelGGL(k_dp_prune, dim3(nb), dim3(256), 0, st, sites, cap, stats, key_p, key_s, dp,
                       prm->alpha, prm->eps, prm->min_mass);
    hipLaunchKernelGGL(k_dp_want_split, dim3(1), dim3(1), 0, st, dp, cap, prm->p_split,
                       (prm->flags & SAD_DP_SPLIT) ? 1 : 0);
    launch_radix_select(key_s, cap, &dp->ss, hist, st);
    hipLaunchKernelGGL(k_dp_flags, dim3(nb), dim3(256), 0, st, sites, cap, key_s, dp, rpar, rfree);
    launch_excl_scan(rpar, cap, btot, st);
    launch_excl_scan(rfree, cap, btot, st);
    hipLaunchKernelGGL(k_dp_free_list, dim3(nb), dim3(256), 0, st, sites, cap, rfree, dp, flist);
    hipLaunchKernelGGL(k_dp_split, dim3(nb), dim3(256), 0, st, sites, cap, adam_m, adam_v, stats,
                       target, img->H, img->W, key_s, rpar, flist, dp);
    if (prm->flags & SAD_DP_SEED) {
        for (int phase = 0; phase < 2; ++phase)
            hipLaunchKernelGGL(k_dp_seed, dim3(nb), dim3(256), 0, st, sites, cap, key_s, rpar, flist,
                               dp, img->H, img->W, img->K, topk, phase);
    }
    hipLaunchKernelGGL(k_dp_hw, dim3(nb), dim3(256), 0, st, sites, cap, dp);
    hipLaunchKernelGGL(k_dp_counts, dim3(1), dim3(1), 0, st, dp, counts);
    return check_launch("sad_densify_prune");
}
