// sad_sites.h -- per-site device routines: the derived record (Sec. 4.1) and the Adam
// update with the clamps of Sec. 6.1.
#pragma once

#include <cmath>

#include "sad_device.h"

namespace sad {

// Derived record of a site with parameters v[] (Sec. 4.1: G = e^a u u^T + e^-a v v^T,
// v = (-u_y, u_x); tau = exp(log_tau); kappa = tau * s), as the four float4 q0..q3 of
// the record layout.  Transcendentals in double, rounded once.
__device__ __forceinline__ void derive(const float (&v)[SAD_NPARAM], float s, float4 &q0,
                                       float4 &q1, float4 &q2, float4 &q3) {
    bool finite = true;
#pragma unroll
    for (int p = 0; p < SAD_NPARAM; ++p) finite = finite && isfinite(v[p]);
    const float x = v[0], y = v[1], lt = v[2], r = v[3], ux = v[7], uy = v[8], a = v[9];
    q0 = make_float4(x, y, 0.f, 0.f);
    q1 = make_float4(0.f, 0.f, r, 0.f);
    q2 = make_float4(v[4], v[5], v[6], ux);
    q3 = make_float4(uy, 0.f, 0.f, 0.f);
    if (finite && x >= 0.0f) {
        const float tau = (float)exp((double)lt);
        const float ep = (float)exp((double)a);
        const float em = (float)exp(-(double)a);
        const float kappa = __fmul_rn(tau, s);
        const float uxx = __fmul_rn(ux, ux), uyy = __fmul_rn(uy, uy), uxy = __fmul_rn(ux, uy);
        const float g11 = __fmaf_rn(ep, uxx, __fmul_rn(em, uyy));
        const float g22 = __fmaf_rn(ep, uyy, __fmul_rn(em, uxx));
        const float g12 = __fmul_rn(__fsub_rn(ep, em), uxy);
        const float g12x2 = __fmul_rn(2.0f, g12);
        const bool ok = kappa > 0.0f && isfinite(kappa) && isfinite(g11) && isfinite(g22) &&
                        isfinite(g12x2);
        q0.z = g11;
        q0.w = g12x2;
        q1.x = g22;
        q1.y = kappa;
        q1.w = ok ? 1.0f : 0.0f;
        q3.y = ep;
        q3.z = em;
        q3.w = tau;
    }
}

// Derived record of slot i written to rec[i].
__device__ __forceinline__ void record_of(const float (&v)[SAD_NPARAM], int64_t i, float s,
                                          float4 *__restrict__ rec) {
    float4 q0, q1, q2, q3;
    derive(v, s, q0, q1, q2, q3);
    rec[4 * i + 0] = q0;
    rec[4 * i + 1] = q1;
    rec[4 * i + 2] = q2;
    rec[4 * i + 3] = q3;
}

__device__ __forceinline__ void write_record(const float *__restrict__ sites, int64_t cap,
                                             int64_t i, float s, float4 *__restrict__ rec) {
    float v[SAD_NPARAM];
#pragma unroll
    for (int p = 0; p < SAD_NPARAM; ++p) v[p] = sites[p * cap + i];
    record_of(v, i, s, rec);
}

// ---- end of a training iteration ---------------------------------------------------
// Called by every thread of every block of the iteration's last kernel after its own
// work: the last block to arrive folds the loss partials of each state in st[0..n)
// into its value (written), clears them and advances pass and adam_step; the block
// counter lives in st[0].done and is reset by that block, so the kernel can be replayed
// from a graph.  Every block reads the counters before it arrives here.
__device__ __forceinline__ void finish_iteration(sad_step_state *__restrict__ st, int n) {
    __shared__ int last;
    __syncthreads();
    if (threadIdx.x == 0) {
        __threadfence();
        last = atomicAdd(reinterpret_cast<unsigned long long *>(&st[0].done), 1ull) ==
               (unsigned long long)(gridDim.x - 1);
    }
    __syncthreads();
    if (!last) return;
    __threadfence();
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    for (int b = w; b < n; b += blockDim.x >> 6) {  // one wave per state
        sad_loss_acc *loss = &st[b].loss;
        float v = lane < SAD_LOSS_PARTS ? loss->part[lane] : 0.f;
        for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
        if (lane < SAD_LOSS_PARTS) loss->part[lane] = 0.f;
        if (lane == 0) {
            loss->value = v;
            st[b].pass += 1;
            st[b].adam_step += 1;
        }
    }
    if (threadIdx.x == 0) st[0].done = 0ull;
}

// ---- Adam (Sec. 5; clamps of Sec. 6.1) ----------------------------------------------
struct AdamArgs {
    float lr[SAD_NPARAM];
    float b1, b2, eps, c1, c2;  // c1 = 1 - b1^t, c2 = 1 - b2^t (host step)
    int zero_grad;              // clear the gradient after reading it
    int grad_site_major;        // gradient [cap][10] (training step) instead of [10][cap]
    int grad_fixed;             // gradient elements are int64 fixed point (deterministic
                                // sums) worth grad_from each, instead of float
    double grad_from;
};

// Adam on slot i of one image's [10][cap] buffers (site order of App. B.2), then clamps
// and renormalised u; inactive slots are left untouched.  The gradient is [10][cap] or,
// with A.grad_site_major, [cap][10]; kFixed: int64 elements worth A.grad_from each.
// step_dev, if set, holds the number of steps taken so far.  Every operand is loaded
// before anything depends on one (the activity test included), so the loads share one
// memory latency, and the double pow of a device-side step overlaps it.
template <bool kFixed>
__device__ __forceinline__ void adam_site_impl(float *__restrict__ sites,
                                               float *__restrict__ grad,
                                               float *__restrict__ m, float *__restrict__ v,
                                               int64_t cap, int64_t i, int H, int W,
                                               const AdamArgs &A, const int64_t *step_dev,
                                               float s, float4 *__restrict__ rec) {
    const int64_t gs = A.grad_site_major ? 1 : cap;             // parameter stride
    const int64_t g0 = A.grad_site_major ? i * SAD_NPARAM : i;  // first element of site i
    long long *g64 = reinterpret_cast<long long *>(grad);
    float g[SAD_NPARAM], m0[SAD_NPARAM], v0[SAD_NPARAM], x0[SAD_NPARAM];
#pragma unroll
    for (int p = 0; p < SAD_NPARAM; ++p) {
        const int64_t o = p * cap + i;
        g[p] = kFixed ? (float)((double)g64[g0 + p * gs] * A.grad_from) : grad[g0 + p * gs];
        m0[p] = m[o];
        v0[p] = v[o];
        x0[p] = sites[o];
    }
    if (A.zero_grad)
#pragma unroll
        for (int p = 0; p < SAD_NPARAM; ++p) {
            if (kFixed)
                g64[g0 + p * gs] = 0;
            else
                grad[g0 + p * gs] = 0.0f;
        }
    if (!(x0[0] >= 0.0f)) {  // inactive slot: parameters untouched
        if (rec) record_of(x0, i, s, rec);
        return;
    }
    float c1 = A.c1, c2 = A.c2;
    if (step_dev) {
        const double t = (double)(*step_dev + 1);
        c1 = (float)(1.0 - pow((double)A.b1, t));
        c2 = (float)(1.0 - pow((double)A.b2, t));
    }
    const float lo[SAD_NPARAM] = {0.f, 0.f, 2.f, 1.f, 0.f, 0.f, 0.f, -INFINITY, -INFINITY, -2.f};
    const float hi[SAD_NPARAM] = {(float)(W - 1), (float)(H - 1), 20.f, 512.f, 1.f, 1.f, 1.f,
                                  INFINITY, INFINITY, 2.f};
    // One division per site for each bias correction and the hardware square root and
    // reciprocal (1 ulp) per parameter: the update differs from the exactly rounded
    // quotients by a few ulps of the step, far below the parity tolerance, and a site's
    // chain of dependent instructions (one wave per SIMD at typical site counts) is
    // much shorter than with ten IEEE divisions and square roots per quotient.
    const float ic1 = 1.0f / c1, ic2 = 1.0f / c2;
    float th[SAD_NPARAM];
#pragma unroll
    for (int p = 0; p < SAD_NPARAM; ++p) {
        const int64_t o = p * cap + i;
        const float mm = A.b1 * m0[p] + (1.0f - A.b1) * g[p];
        const float vv = A.b2 * v0[p] + (1.0f - A.b2) * g[p] * g[p];
        m[o] = mm;
        v[o] = vv;
        const float mh = mm * ic1, vh = vv * ic2;
        const float den = __builtin_amdgcn_sqrtf(vh) + A.eps;
        float x = x0[p] - A.lr[p] * mh * __builtin_amdgcn_rcpf(den);
        x = fminf(fmaxf(x, lo[p]), hi[p]);
        th[p] = x;
    }
    const float nu = sqrtf(th[7] * th[7] + th[8] * th[8]);
    if (nu > 0.f) {
        const float inu = 1.0f / nu;
        th[7] *= inu;
        th[8] *= inu;
    } else {
        th[7] = 1.f;
        th[8] = 0.f;
    }
#pragma unroll
    for (int p = 0; p < SAD_NPARAM; ++p) sites[p * cap + i] = th[p];
    if (rec) record_of(th, i, s, rec);  // from the registers, not re-read
}

__device__ __forceinline__ void adam_site(float *__restrict__ sites, float *__restrict__ grad,
                                          float *__restrict__ m, float *__restrict__ v,
                                          int64_t cap, int64_t i, int H, int W, const AdamArgs &A,
                                          const int64_t *step_dev, float s,
                                          float4 *__restrict__ rec) {
    if (A.grad_fixed)  // uniform: one straight-line copy per gradient type
        adam_site_impl<true>(sites, grad, m, v, cap, i, H, W, A, step_dev, s, rec);
    else
        adam_site_impl<false>(sites, grad, m, v, cap, i, H, W, A, step_dev, s, rec);
}

}  // namespace sad
