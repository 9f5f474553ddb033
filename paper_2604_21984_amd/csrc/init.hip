// init.hip -- gradient-weighted site initialisation (Sec. 4.4) on the GPU.
//
// 1. |grad I| per pixel (double), summed with a fixed reduction tree (run-to-run
//    deterministic).
// 2. Efraimidis-Spirakis key log(u_p) / P_init(p) per pixel (double), as an unsigned
//    64-bit order-preserving code.
// 3. Radix select (8 passes of 8 bits, most significant first) finds the n-th largest
//    code T and how many codes equal to T are still needed.
// 4. Selection flags (code > T, or code == T among the first `need` in raster order),
//    exclusive scan -> slot of each winner; winners are written in raster order.
#include <cmath>

#include "sad_device.h"
#include "sad_host.h"
#include "sad_internal.h"

namespace sad {

constexpr int kScanItems = 4;
constexpr int kScanBlock = 256 * kScanItems;

__device__ __forceinline__ double grad_mag(const float *__restrict__ I, int H, int W, int i, int j) {
    const int64_t P = (int64_t)H * W;
    const int jp = j + 1 < W ? j + 1 : W - 1, jm = j > 0 ? j - 1 : 0;
    const int ip = i + 1 < H ? i + 1 : H - 1, im = i > 0 ? i - 1 : 0;
    double acc = 0.0;
    for (int ch = 0; ch < 3; ++ch) {
        const float *c = I + ch * P;
        const double gx = 0.5 * ((double)c[(int64_t)i * W + jp] - (double)c[(int64_t)i * W + jm]);
        const double gy = 0.5 * ((double)c[(int64_t)ip * W + j] - (double)c[(int64_t)im * W + j]);
        acc += gx * gx + gy * gy;
    }
    return sqrt(acc);
}

__device__ __forceinline__ double block_sum_d(double v) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    __shared__ double part[4];
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = v;
    __syncthreads();
    const double r = (part[0] + part[1]) + (part[2] + part[3]);
    __syncthreads();
    return r;
}

__global__ __launch_bounds__(256) void k_gm_partial(const float *__restrict__ I, int H, int W,
                                                    double *__restrict__ partial) {
    const int64_t P = (int64_t)H * W;
    const int64_t base = (int64_t)blockIdx.x * kScanBlock;
    double acc = 0.0;
    for (int r = 0; r < kScanItems; ++r) {
        const int64_t p = base + (int64_t)r * 256 + threadIdx.x;
        if (p < P) acc += grad_mag(I, H, W, (int)(p / W), (int)(p % W));
    }
    const double s = block_sum_d(acc);
    if (threadIdx.x == 0) partial[blockIdx.x] = s;
}

__global__ __launch_bounds__(256) void k_sum_partials(const double *__restrict__ partial, int nb,
                                                      double *__restrict__ total) {
    double acc = 0.0;
    for (int b = threadIdx.x; b < nb; b += 256) acc += partial[b];
    const double s = block_sum_d(acc);
    if (threadIdx.x == 0) *total = s;
}

__device__ __forceinline__ uint64_t order_f64(double v) {
    const uint64_t b = (uint64_t)__double_as_longlong(v);
    return b ^ ((b >> 63) ? ~0ull : 0x8000000000000000ull);
}

__global__ __launch_bounds__(256) void k_keys(const float *__restrict__ I, int H, int W, double lam,
                                              uint64_t seed, const double *__restrict__ Gsum,
                                              uint64_t *__restrict__ code) {
    const int64_t P = (int64_t)H * W;
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= P) return;
    const double G = *Gsum;
    const double gm = grad_mag(I, H, W, (int)(p / W), (int)(p % W));
    const double pr = lam / (double)P + (G > 0.0 ? (1.0 - lam) * gm / G : 0.0);
    const double u = ((double)(splitmix64(seed, (uint64_t)p) >> 32) + 0.5) / 4294967296.0;
    const double key = pr > 0.0 ? log(u) / pr : -INFINITY;
    code[p] = order_f64(key);
}

__global__ void k_sel_init(SelState *st, uint32_t n) {
    st->prefix = 0;
    st->mask = 0;
    st->want = n;
}

__global__ __launch_bounds__(256) void k_sel_hist(const uint64_t *__restrict__ code, int64_t P,
                                                  int shift, const SelState *__restrict__ st,
                                                  uint32_t *__restrict__ hist) {
    __shared__ uint32_t h[256];
    h[threadIdx.x] = 0;
    __syncthreads();
    const uint64_t prefix = st->prefix, mask = st->mask;
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < P;
         p += (int64_t)gridDim.x * blockDim.x) {
        const uint64_t c = code[p];
        if ((c & mask) == prefix) atomicAdd(&h[(c >> shift) & 255u], 1u);
    }
    __syncthreads();
    if (h[threadIdx.x]) atomicAdd(&hist[threadIdx.x], h[threadIdx.x]);
}

// Pick the digit holding the want-th largest code (single thread); clear hist.
__global__ void k_sel_pick(SelState *st, uint32_t *hist, int shift) {
    if (threadIdx.x != 0) return;
    uint32_t want = st->want, cum = 0;
    int d = 0;
    for (int b = 255; b >= 0; --b) {
        if (cum + hist[b] >= want) {
            d = b;
            break;
        }
        cum += hist[b];
    }
    st->want = want - cum;
    st->prefix |= (uint64_t)d << shift;
    st->mask |= (uint64_t)255 << shift;
    for (int b = 0; b < 256; ++b) hist[b] = 0;
}

// flags[p] = 1 where code == T (used to rank ties), 0 elsewhere
__global__ __launch_bounds__(256) void k_eq_flags(const uint64_t *__restrict__ code, int64_t P,
                                                  const SelState *__restrict__ st,
                                                  uint32_t *__restrict__ f) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p < P) f[p] = code[p] == st->prefix ? 1u : 0u;
}

// flags[p] = selected?  (tie rank from the exclusive scan of the equality flags)
__global__ __launch_bounds__(256) void k_sel_flags(const uint64_t *__restrict__ code, int64_t P,
                                                   const SelState *__restrict__ st,
                                                   uint32_t *__restrict__ f) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= P) return;
    const uint64_t c = code[p], T = st->prefix;
    f[p] = (c > T || (c == T && f[p] < st->want)) ? 1u : 0u;
}

// ---- exclusive scan of uint32 flags (in place), three kernels ----------------------
__device__ __forceinline__ uint32_t block_excl_scan(uint32_t v, uint32_t *total) {
    // wave-level inclusive scan
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    uint32_t x = v;
    for (int o = 1; o < 64; o <<= 1) {
        const uint32_t y = __shfl_up(x, o);
        if (lane >= o) x += y;
    }
    __shared__ uint32_t wsum[4];
    if (lane == 63) wsum[w] = x;
    __syncthreads();
    uint32_t off = 0;
    for (int k = 0; k < w; ++k) off += wsum[k];
    *total = wsum[0] + wsum[1] + wsum[2] + wsum[3];
    __syncthreads();
    return off + x - v;
}

__global__ __launch_bounds__(256) void k_scan_tot(const uint32_t *__restrict__ f, int64_t P,
                                                  uint32_t *__restrict__ btot) {
    const int64_t base = (int64_t)blockIdx.x * kScanBlock + (int64_t)threadIdx.x * kScanItems;
    uint32_t s = 0;
    for (int r = 0; r < kScanItems; ++r)
        if (base + r < P) s += f[base + r];
    uint32_t tot;
    block_excl_scan(s, &tot);
    if (threadIdx.x == 0) btot[blockIdx.x] = tot;
}

__global__ __launch_bounds__(256) void k_scan_btot(uint32_t *__restrict__ btot, int nb) {
    uint32_t carry = 0;
    for (int b0 = 0; b0 < nb; b0 += 256) {
        const int b = b0 + threadIdx.x;
        const uint32_t v = b < nb ? btot[b] : 0u;
        uint32_t tot;
        const uint32_t ex = block_excl_scan(v, &tot);
        if (b < nb) btot[b] = carry + ex;
        carry += tot;
    }
}

__global__ __launch_bounds__(256) void k_scan_apply(uint32_t *__restrict__ f, int64_t P,
                                                    const uint32_t *__restrict__ btot) {
    const int64_t base = (int64_t)blockIdx.x * kScanBlock + (int64_t)threadIdx.x * kScanItems;
    uint32_t v[kScanItems], s = 0;
    for (int r = 0; r < kScanItems; ++r) {
        v[r] = base + r < P ? f[base + r] : 0u;
        s += v[r];
    }
    uint32_t tot;
    uint32_t run = block_excl_scan(s, &tot) + btot[blockIdx.x];
    for (int r = 0; r < kScanItems; ++r) {
        if (base + r < P) f[base + r] = run;
        run += v[r];
    }
}

// Winners: code > T or (code == T and tie rank < want); slot = exclusive scan of winners.
__global__ __launch_bounds__(256) void k_write_sites(const float *__restrict__ I, int H, int W,
                                                     const uint64_t *__restrict__ code,
                                                     const uint32_t *__restrict__ slot,
                                                     const uint32_t *__restrict__ win,
                                                     float log_tau0, float r0,
                                                     float *__restrict__ sites, int64_t cap) {
    const int64_t P = (int64_t)H * W;
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= P) return;
    // a pixel won iff the exclusive scan steps at p
    const uint32_t s0 = slot[p];
    const uint32_t s1 = p + 1 < P ? slot[p + 1] : *win;
    if (s1 == s0) return;
    const int64_t k = s0;
    if (k >= cap) return;
    const float v[SAD_NPARAM] = {(float)(p % W), (float)(p / W), log_tau0, r0, I[p], I[P + p],
                                 I[2 * P + p], 1.0f, 0.0f, 0.0f};
    for (int q = 0; q < SAD_NPARAM; ++q) sites[q * cap + k] = v[q];
}

__global__ __launch_bounds__(256) void k_clear_slots(float *__restrict__ sites, int64_t cap,
                                                     int64_t from) {
    const int64_t i = from + (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= cap) return;
    for (int q = 0; q < SAD_NPARAM; ++q) sites[q * cap + i] = (q < 2) ? -1.0f : 0.0f;
}

__global__ void k_total(const uint32_t *__restrict__ f, const uint32_t *__restrict__ flags_last,
                        int64_t P, uint32_t *__restrict__ out) {
    // total winners = exclusive-scan value at P-1 + flag at P-1
    *out = f[P - 1] + *flags_last;
}
__global__ void k_zero_u32(uint32_t *__restrict__ p, int n) {
    for (int i = threadIdx.x; i < n; i += blockDim.x) p[i] = 0u;
}
__global__ void k_copy1(const uint32_t *__restrict__ a, uint32_t *__restrict__ b) { *b = *a; }

static size_t align_up(size_t x) { return (x + 255) & ~(size_t)255; }

void launch_radix_select(const uint64_t *code, int64_t n, SelState *st, uint32_t *hist,
                         hipStream_t s) {
    const int64_t nb = (n + 255) / 256;
    const unsigned nbh = (unsigned)(nb < 1024 ? (nb > 0 ? nb : 1) : 1024);
    for (int d = 7; d >= 0; --d) {
        hipLaunchKernelGGL(k_sel_hist, dim3(nbh), dim3(256), 0, s, code, n, 8 * d, st, hist);
        hipLaunchKernelGGL(k_sel_pick, dim3(1), dim3(64), 0, s, st, hist, 8 * d);
    }
}

int64_t scan_blocks(int64_t n) { return (n + kScanBlock - 1) / kScanBlock; }

void launch_excl_scan(uint32_t *f, int64_t n, uint32_t *btot, hipStream_t s) {
    const int64_t nb = scan_blocks(n);
    hipLaunchKernelGGL(k_scan_tot, dim3((unsigned)nb), dim3(256), 0, s, f, n, btot);
    hipLaunchKernelGGL(k_scan_btot, dim3(1), dim3(256), 0, s, btot, (int)nb);
    hipLaunchKernelGGL(k_scan_apply, dim3((unsigned)nb), dim3(256), 0, s, f, n, btot);
}

}  // namespace sad

using namespace sad;

extern "C" sad_status sad_init_sites(const sad_image *img, const float *target, int32_t n_sites,
                                     float lambda, uint64_t seed, float log_tau0, float r0,
                                     float *sites, void *workspace, size_t *workspace_bytes,
                                     void *stream) {
    SAD_TRY(check_image(img, nullptr));
    SAD_REQUIRE(workspace_bytes, SAD_ERR_INVALID_ARGUMENT, "sad_init_sites: workspace_bytes is NULL");
    const int64_t P = (int64_t)img->H * img->W;
    const int64_t nb_scan = (P + kScanBlock - 1) / kScanBlock;
    const size_t off_code = 0;
    const size_t off_flag = align_up(off_code + 8 * (size_t)P);
    const size_t off_btot = align_up(off_flag + 4 * (size_t)P);
    const size_t off_part = align_up(off_btot + 4 * (size_t)nb_scan);
    const size_t off_G = align_up(off_part + 8 * (size_t)nb_scan);
    const size_t off_st = align_up(off_G + 8);
    const size_t off_hist = align_up(off_st + sizeof(SelState));
    const size_t off_misc = align_up(off_hist + 256 * 4);
    const size_t need = align_up(off_misc + 16);
    if (!workspace) {
        *workspace_bytes = need;
        return SAD_OK;
    }
    SAD_REQUIRE(*workspace_bytes >= need, SAD_ERR_WORKSPACE,
                "sad_init_sites: workspace too small (%zu < %zu)", *workspace_bytes, need);
    SAD_REQUIRE(target && sites, SAD_ERR_INVALID_ARGUMENT, "sad_init_sites: NULL pointer");
    SAD_REQUIRE(n_sites >= 0 && n_sites <= P && n_sites <= img->cap, SAD_ERR_INVALID_ARGUMENT,
                "sad_init_sites: n_sites must be in [0, min(H*W, cap)]");
    SAD_REQUIRE(lambda >= 0.f && lambda <= 1.f, SAD_ERR_INVALID_ARGUMENT,
                "sad_init_sites: lambda must be in [0, 1]");
    hipStream_t st = as_stream(stream);
    char *ws = static_cast<char *>(workspace);
    uint64_t *code = reinterpret_cast<uint64_t *>(ws + off_code);
    uint32_t *flag = reinterpret_cast<uint32_t *>(ws + off_flag);
    uint32_t *btot = reinterpret_cast<uint32_t *>(ws + off_btot);
    double *part = reinterpret_cast<double *>(ws + off_part);
    double *G = reinterpret_cast<double *>(ws + off_G);
    SelState *sel = reinterpret_cast<SelState *>(ws + off_st);
    uint32_t *hist = reinterpret_cast<uint32_t *>(ws + off_hist);
    uint32_t *misc = reinterpret_cast<uint32_t *>(ws + off_misc);
    const unsigned nbP = (unsigned)((P + 255) / 256);

    auto scan = [&](uint32_t *f) { launch_excl_scan(f, P, btot, st); };
    if (n_sites > 0) {
        hipLaunchKernelGGL(k_gm_partial, dim3((unsigned)nb_scan), dim3(256), 0, st, target, img->H,
                           img->W, part);
        hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(256), 0, st, part, (int)nb_scan, G);
        hipLaunchKernelGGL(k_keys, dim3(nbP), dim3(256), 0, st, target, img->H, img->W,
                           (double)lambda, seed, G, code);
        hipLaunchKernelGGL(k_sel_init, dim3(1), dim3(1), 0, st, sel, (uint32_t)n_sites);
        hipLaunchKernelGGL(k_zero_u32, dim3(1), dim3(256), 0, st, hist, 256);
        launch_radix_select(code, P, sel, hist, st);
        hipLaunchKernelGGL(k_eq_flags, dim3(nbP), dim3(256), 0, st, code, P, sel, flag);
        scan(flag);
        hipLaunchKernelGGL(k_sel_flags, dim3(nbP), dim3(256), 0, st, code, P, sel, flag);
        hipLaunchKernelGGL(k_copy1, dim3(1), dim3(1), 0, st, flag + (P - 1), misc);
        scan(flag);
        hipLaunchKernelGGL(k_total, dim3(1), dim3(1), 0, st, flag, misc, P, misc + 1);
        hipLaunchKernelGGL(k_write_sites, dim3(nbP), dim3(256), 0, st, target, img->H, img->W, code,
                           flag, misc + 1, log_tau0, r0, sites, img->cap);
        SAD_TRY(check_launch("sad_init_sites"));
    }
    if (img->cap > n_sites) {
        const int64_t nclr = img->cap - n_sites;
        hipLaunchKernelGGL(k_clear_slots, dim3((unsigned)((nclr + 255) / 256)), dim3(256), 0, st,
                           sites, img->cap, (int64_t)n_sites);
    }
    return check_launch("sad_init_sites");
}
