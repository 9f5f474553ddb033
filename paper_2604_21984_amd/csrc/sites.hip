// sites.hip -- per-site kernels: derived records (the pack step), seed pass, Adam.
#include <cmath>
#include <mutex>

#include "sad_device.h"
#include "sad_host.h"
#include "sad_internal.h"
#include "sad_sites.h"

namespace sad {

__global__ __launch_bounds__(256) void k_prepare(const float *__restrict__ sites, int64_t cap,
                                                 int n, float s, float4 *__restrict__ rec) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) write_record(sites, cap, i, s, rec);
}

// ---- seed pass --------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_fill_u32(uint32_t *__restrict__ p, int64_t n, uint32_t v) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}
__global__ __launch_bounds__(256) void k_fill_u64(uint64_t *__restrict__ p, int64_t n, uint64_t v) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

// The cell of a site's nearest pixel (rint(y), rint(x)) clamped to the H x W image, on
// a grid of Hg x Wg cells (the pixel itself when the grid is the image's).
__device__ __forceinline__ int64_t seed_cell(float x, float y, const SeedGrid &g) {
    const float fi = rintf(y), fj = rintf(x);
    const int ii = fi < 0.f ? 0 : (fi > (float)(g.H - 1) ? g.H - 1 : (int)fi);
    const int jj = fj < 0.f ? 0 : (fj > (float)(g.W - 1) ? g.W - 1 : (int)fj);
    return (int64_t)cell_of(ii, g.H, g.Hg) * g.Wg + cell_of(jj, g.W, g.Wg);
}

// Has site i already been placed in entries 0..round-1 of cell p?
__device__ __forceinline__ bool placed(const uint32_t *__restrict__ topk, int64_t P, int64_t p,
                                       int round, uint32_t i) {
    for (int k = 0; k < round; ++k)
        if (topk[((int64_t)(k >> 2) * P + p) * 4 + (k & 3)] == i) return true;
    return false;
}

// The key of a site at the point of its seed cell.
__device__ __forceinline__ uint64_t seed_key(const float4 q0, const float4 q1, int64_t p,
                                             const SeedGrid &g, uint32_t i) {
    const float X = grid_point((int)(p % g.Wg), g.W, g.Wg);
    const float Y = grid_point((int)(p / g.Wg), g.H, g.Hg);
    return make_key(score(q0, q1, X, Y), i);
}

// Round r of the seed pass: every valid, not yet placed site bids its key for its
// cell with a 64-bit atomic max; the winner takes entry r (next kernel).
__global__ __launch_bounds__(256) void k_seed_bid(const float4 *__restrict__ rec, int n,
                                                  SeedGrid g, int round,
                                                  const uint32_t *__restrict__ topk,
                                                  unsigned long long *__restrict__ best) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float4 q0 = rec[4 * i], q1 = rec[4 * i + 1];
    if (q1.w == 0.0f) return;
    const int64_t P = (int64_t)g.Hg * g.Wg;
    const int64_t p = seed_cell(q0.x, q0.y, g);
    if (placed(topk, P, p, round, (uint32_t)i)) return;
    atomicMax(best + p, (unsigned long long)seed_key(q0, q1, p, g, (uint32_t)i));
}

__global__ __launch_bounds__(256) void k_seed_take(const float4 *__restrict__ rec, int n,
                                                   SeedGrid g, int round,
                                                   uint32_t *__restrict__ topk,
                                                   unsigned long long *__restrict__ best) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float4 q0 = rec[4 * i], q1 = rec[4 * i + 1];
    if (q1.w == 0.0f) return;
    const int64_t P = (int64_t)g.Hg * g.Wg;
    const int64_t p = seed_cell(q0.x, q0.y, g);
    if (placed(topk, P, p, round, (uint32_t)i)) return;
    if (best[p] == (unsigned long long)seed_key(q0, q1, p, g, (uint32_t)i)) {
        topk[((int64_t)(round >> 2) * P + p) * 4 + (round & 3)] = (uint32_t)i;
        best[p] = 0ull;  // only the winner resets; losers compare against their own key
    }
}

__global__ __launch_bounds__(256) void k_adam(float *__restrict__ sites,
                                              float *__restrict__ grad,
                                              float *__restrict__ m, float *__restrict__ v,
                                              int64_t cap, int n, int H, int W, AdamArgs A,
                                              const int64_t *step_dev, float s,
                                              float4 *__restrict__ rec,
                                              sad_step_state *__restrict__ fin) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) adam_site(sites, grad, m, v, cap, i, H, W, A, step_dev, s, rec);
    if (fin) finish_iteration(fin, 1);
}

}  // namespace sad

using namespace sad;

extern "C" sad_status sad_prepare_sites(const sad_image *img, const float *sites, float *rec,
                                        void *stream) {
    float s;
    SAD_TRY(check_image(img, &s));
    if (img->n_slots == 0) return SAD_OK;
    SAD_REQUIRE(sites && rec, SAD_ERR_INVALID_ARGUMENT, "sad_prepare_sites: NULL pointer");
    SAD_REQUIRE(aligned16(rec), SAD_ERR_INVALID_ARGUMENT, "sad_prepare_sites: rec not 16-byte aligned");
    const int n = img->n_slots;
    hipLaunchKernelGGL(k_prepare, dim3((n + 255) / 256), dim3(256), 0, as_stream(stream), sites,
                       img->cap, n, s, reinterpret_cast<float4 *>(rec));
    return check_launch("sad_prepare_sites");
}

void sad::launch_seed(const sad_image *img, int32_t Hg, int32_t Wg, int32_t n_entries,
                      const float *rec, uint32_t *topk, uint64_t *scratch, hipStream_t st) {
    const int64_t P = (int64_t)Hg * Wg;
    const int64_t nl = P * img->K;
    hipLaunchKernelGGL(k_fill_u32, dim3((unsigned)((nl + 255) / 256)), dim3(256), 0, st, topk, nl,
                       SAD_INVALID_ID);
    const int n = img->n_slots;
    if (n == 0 || n_entries <= 0) return;
    hipLaunchKernelGGL(k_fill_u64, dim3((unsigned)((P + 255) / 256)), dim3(256), 0, st, scratch, P,
                       0ull);
    const float4 *r4 = reinterpret_cast<const float4 *>(rec);
    auto *best = reinterpret_cast<unsigned long long *>(scratch);
    SeedGrid g;
    g.H = img->H;
    g.W = img->W;
    g.Hg = Hg;
    g.Wg = Wg;
    for (int round = 0; round < n_entries && round < img->K; ++round) {
        hipLaunchKernelGGL(k_seed_bid, dim3((n + 255) / 256), dim3(256), 0, st, r4, n, g, round,
                           topk, best);
        hipLaunchKernelGGL(k_seed_take, dim3((n + 255) / 256), dim3(256), 0, st, r4, n, g, round,
                           topk, best);
    }
}

extern "C" sad_status sad_seed_topk(const sad_image *img, const float *rec, uint32_t *topk,
                                    uint64_t *scratch, void *stream) {
    SAD_TRY(check_image(img, nullptr));
    SAD_REQUIRE(topk && scratch && (rec || img->n_slots == 0), SAD_ERR_INVALID_ARGUMENT,
                "sad_seed_topk: NULL pointer");
    SAD_REQUIRE(!rec || aligned16(rec), SAD_ERR_INVALID_ARGUMENT, "sad_seed_topk: rec not 16-byte aligned");
    launch_seed(img, img->H, img->W, img->K, rec, topk, scratch, as_stream(stream));
    return check_launch("sad_seed_topk");
}

// ---- seed pass without allocation ---------------------------------------------------
// The seed pass's per-pixel bid words for callers that cannot allocate: one array per
// device, in the code object's own device memory, for images of up to
// SAD_SEED_STATIC_PIXELS pixels (32 MiB, held on every device the library runs on until
// the process ends).  Host code never passes the array's name to a kernel (on the host it
// is only a stand-in for the symbol): each device's address is looked up once, with that
// device current, and kept.
static __device__ __align__(256) uint64_t scratch[SAD_SEED_STATIC_PIXELS];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
uint64_t *g_scratch_dev[kMaxDevices] = {};

sad_status static_scratch(uint64_t **out) {
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    SAD_REQUIRE(e == hipSuccess, SAD_ERR_DEVICE, "sad_seed_topk_noalloc: hipGetDevice: %s",
                hipGetErrorString(e));
    SAD_REQUIRE(dev >= 0 && dev < kMaxDevices, SAD_ERR_UNSUPPORTED,
                "sad_seed_topk_noalloc: device %d beyond the %d supported", dev, kMaxDevices);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_dev[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        SAD_REQUIRE(e == hipSuccess && p, SAD_ERR_DEVICE,
                    "sad_seed_topk_noalloc: hipGetSymbolAddress: %s", hipGetErrorString(e));
        g_scratch_dev[dev] = static_cast<uint64_t *>(p);
    }
    *out = g_scratch_dev[dev];
    return SAD_OK;
}
}  // namespace

extern "C" sad_status sad_seed_topk_noalloc(const sad_image *img, const float *rec,
                                            uint32_t *topk, void *stream) {
    SAD_TRY(check_image(img, nullptr));
    SAD_REQUIRE(topk && (rec || img->n_slots == 0), SAD_ERR_INVALID_ARGUMENT,
                "sad_seed_topk_noalloc: NULL pointer");
    SAD_REQUIRE(!rec || aligned16(rec), SAD_ERR_INVALID_ARGUMENT,
                "sad_seed_topk_noalloc: rec not 16-byte aligned");
    SAD_REQUIRE((int64_t)img->H * img->W <= (int64_t)SAD_SEED_STATIC_PIXELS, SAD_ERR_WORKSPACE,
                "sad_seed_topk_noalloc: %d x %d pixels exceed the static scratch of %d pixels",
                img->H, img->W, SAD_SEED_STATIC_PIXELS);
    uint64_t *ws = nullptr;
    SAD_TRY(static_scratch(&ws));
    launch_seed(img, img->H, img->W, img->K, rec, topk, ws, as_stream(stream));
    return check_launch("sad_seed_topk_noalloc");
}

void sad::launch_adam(const sad_image *img, float s, float *sites, float *grad, float *m,
                      float *v, const sad_adam_params *params, int64_t step,
                      const int64_t *step_dev, float *rec, bool zero_grad, bool grad_site_major,
                      sad_step_state *fin, hipStream_t st, bool grad_fixed) {
    if (img->n_slots == 0) return;
    AdamArgs A;
    for (int p = 0; p < SAD_NPARAM; ++p) A.lr[p] = params->lr[p];
    A.b1 = params->beta1;
    A.b2 = params->beta2;
    A.eps = params->eps;
    A.c1 = (float)(1.0 - std::pow((double)params->beta1, (double)step));
    A.c2 = (float)(1.0 - std::pow((double)params->beta2, (double)step));
    A.zero_grad = zero_grad ? 1 : 0;
    A.grad_site_major = grad_site_major ? 1 : 0;
    A.grad_fixed = grad_fixed ? 1 : 0;
    A.grad_from = det_grad_unit((int64_t)img->H * img->W);
    const int n = img->n_slots;
    hipLaunchKernelGGL(k_adam, dim3((n + 255) / 256), dim3(256), 0, st, sites, grad, m, v, img->cap,
                       n, img->H, img->W, A, step_dev, s, reinterpret_cast<float4 *>(rec), fin);
}

extern "C" sad_status sad_adam_step(const sad_image *img, float *sites, float *grad, float *m,
                                    float *v, const sad_adam_params *params, int64_t step,
                                    float *rec, uint32_t flags, void *stream) {
    float s;
    SAD_TRY(check_image(img, &s));
    SAD_REQUIRE(params, SAD_ERR_INVALID_ARGUMENT, "sad_adam_step: params is NULL");
    SAD_REQUIRE(step >= 1, SAD_ERR_INVALID_ARGUMENT, "sad_adam_step: step must be >= 1");
    if (img->n_slots == 0) return SAD_OK;
    SAD_REQUIRE(sites && grad && m && v, SAD_ERR_INVALID_ARGUMENT, "sad_adam_step: NULL pointer");
    SAD_REQUIRE(!rec || aligned16(rec), SAD_ERR_INVALID_ARGUMENT, "sad_adam_step: rec not 16-byte aligned");
    SAD_REQUIRE((flags & ~(SAD_ADAM_ZERO_GRAD | SAD_ADAM_GRAD_SITE_MAJOR |
                           SAD_ADAM_GRAD_FIXED)) == 0,
                SAD_ERR_INVALID_ARGUMENT,
                "sad_adam_step: unknown flags 0x%x", flags);
    launch_adam(img, s, sites, grad, m, v, params, step, nullptr, rec,
                (flags & SAD_ADAM_ZERO_GRAD) != 0, (flags & SAD_ADAM_GRAD_SITE_MAJOR) != 0,
                nullptr, as_stream(stream), (flags & SAD_ADAM_GRAD_FIXED) != 0);
    return check_launch("sad_adam_step");
}

extern "C" sad_status sad_adam_step_state(const sad_image *img, float *sites, float *grad,
                                          float *m, float *v, const sad_adam_params *params,
                                          float *rec, uint32_t flags, sad_step_state *state,
                                          void *stream) {
    float s;
    SAD_TRY(check_image(img, &s));
    SAD_REQUIRE(params && state, SAD_ERR_INVALID_ARGUMENT,
                "sad_adam_step_state: params or state is NULL");
    SAD_REQUIRE((flags & ~(SAD_ADAM_ZERO_GRAD | SAD_ADAM_GRAD_SITE_MAJOR |
                           SAD_ADAM_GRAD_FIXED)) == 0,
                SAD_ERR_INVALID_ARGUMENT, "sad_adam_step_state: unknown flags 0x%x", flags);
    hipStream_t st = as_stream(stream);
    if (img->n_slots == 0) {
        launch_state_advance(state, st);
        return check_launch("sad_adam_step_state");
    }
    SAD_REQUIRE(sites && grad && m && v, SAD_ERR_INVALID_ARGUMENT,
                "sad_adam_step_state: NULL pointer");
    SAD_REQUIRE(!rec || aligned16(rec), SAD_ERR_INVALID_ARGUMENT,
                "sad_adam_step_state: rec not 16-byte aligned");
    launch_adam(img, s, sites, grad, m, v, params, 1, &state->adam_step, rec,
                (flags & SAD_ADAM_ZERO_GRAD) != 0, (flags & SAD_ADAM_GRAD_SITE_MAJOR) != 0,
                state, st, (flags & SAD_ADAM_GRAD_FIXED) != 0);
    return check_launch("sad_adam_step_state");
}
