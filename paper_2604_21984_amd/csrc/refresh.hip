// refresh.hip -- the full-refresh regime (Sec. 6.6; App. B.3): list fields on a grid of
// cells other than the image's pixels (a downscaled candidate grid, or the pixels of a
// new output resolution), the JFA flood prepass, a full refresh (seed or JFA prepass,
// then propagation passes) and rendering from a grid's lists.
#include "sad_device.h"
#include "sad_host.h"
#include "sad_internal.h"
#include "sad_kernels.h"

namespace sad {

struct GridArgs {
    int H, W;        // image
    int Hg, Wg;      // cells of the list field
    int n_slots, tiles_x, n_blocks;
};

inline GridArgs grid_args(const sad_image *img, int Hg, int Wg) {
    GridArgs g;
    g.H = img->H;
    g.W = img->W;
    g.Hg = Hg;
    g.Wg = Wg;
    g.n_slots = img->n_slots;
    g.tiles_x = (Wg + 15) / 16;
    g.n_blocks = g.tiles_x * ((Hg + 15) / 16);
    return g;
}

// One JFA flood pass (App. B.3), Jacobi: cell (i, j) takes the first four entries (the
// first candidate texture, plane 0 of the field) of the cells (i + di step, j + dj step),
// di, dj in {-1, 0, 1}, that lie in the grid (itself included), scores them exactly at
// its centre and writes the best four distinct IDs by (score descending, ID ascending)
// into plane 0 of out.  Planes 1.. of out are not touched.
// The cell's own four entries are scored exactly first; every other candidate is
// screened as in the propagation pass (an ID already kept is a repeat; otherwise the
// score is estimated with the hardware square root and dropped when it lies below the
// fourth key by more than the estimate's error bound), and only survivors are scored
// exactly and inserted, so the result is the exact best four of the candidate set.
__global__ __launch_bounds__(256) void k_jfa_flood(GridArgs g, int step,
                                                   const float4 *__restrict__ rec,
                                                   const uint4 *__restrict__ lin,
                                                   uint4 *__restrict__ lout) {
    const int tile = xcd_tile(blockIdx.x, g.n_blocks);
    const TilePix px = tile_pixel(tile, g.tiles_x);
    if (px.i >= g.Hg || px.j >= g.Wg) return;
    const float X = grid_point(px.j, g.W, g.Wg), Y = grid_point(px.i, g.H, g.Hg);
    const uint32_t ns = (uint32_t)g.n_slots;
    uint64_t keys[4] = {0ull, 0ull, 0ull, 0ull};
    {
        const uint4 v = lin[(int64_t)px.i * g.Wg + px.j];
        const uint32_t id[4] = {v.x, v.y, v.z, v.w};
        uint64_t nk[4];
        exact_keys<4>(rec, ns, X, Y, id, nk);
#pragma unroll
        for (int c = 0; c < 4; ++c) insert_key<4>(keys, nk[c]);
    }
#pragma unroll 1
    for (int nb = 0; nb < 9; ++nb) {
        if (nb == 4) continue;  // the cell itself, taken above
        const int ii = px.i + (nb / 3 - 1) * step, jj = px.j + (nb % 3 - 1) * step;
        if (ii < 0 || ii >= g.Hg || jj < 0 || jj >= g.Wg) continue;
        const uint4 v = lin[(int64_t)ii * g.Wg + jj];
        const uint32_t id[4] = {v.x, v.y, v.z, v.w};
        bool ok[4];
        uint32_t idc[4];
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            const uint32_t nid = ~id[c];
            bool kept = false;
#pragma unroll
            for (int k = 0; k < 4; ++k) kept |= ((uint32_t)keys[k] == nid);
            ok[c] = (id[c] < ns) & !kept;
            idc[c] = ok[c] ? id[c] : 0u;
        }
        float4 q0[4], q1[4];
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            q0[c] = rec[4 * (size_t)idc[c]];
            q1[c] = rec[4 * (size_t)idc[c] + 1];
        }
        const float kth = keys[3] ? key_score(keys[3]) : -INFINITY;
        const bool open = keys[3] == 0ull;
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            const float na = __builtin_amdgcn_sqrtf(quad(q0[c], q1[c], X, Y));
            const float la = q1[c].y * (q1[c].z - na);
            const float bound = fmaf(q1[c].y, fabsf(q1[c].z) + na, fabsf(la)) * 0x1p-19f;
            if (ok[c] & (q1[c].w != 0.0f) & (open | (la + bound >= kth)))
                insert_key<4>(keys, make_key(score(q0[c], q1[c], X, Y), id[c]));
        }
    }
    lout[(int64_t)px.i * g.Wg + px.j] =
        make_uint4(key_id(keys[0]), key_id(keys[1]), key_id(keys[2]), key_id(keys[3]));
}

// Blend on an output grid of Ho x Wo points over the image (Sec. 6.6: rendering a new
// pixel grid) from a list field of Hg x Wg cells: output point (io, jo) sits at the
// centre of its cell of the output grid and takes the list of the list-grid cell that
// holds that centre.  out: float[3][Ho][Wo].
template <int K>
__global__ __launch_bounds__(256) void k_fwd_grid(GridArgs g, int Ho, int Wo, int tiles_xo,
                                                  int n_blocks_o, const float4 *__restrict__ rec,
                                                  const uint4 *__restrict__ topk,
                                                  float *__restrict__ out) {
    const int tile = xcd_tile(blockIdx.x, n_blocks_o);
    const TilePix px = tile_pixel(tile, tiles_xo);
    if (px.i >= Ho || px.j >= Wo) return;
    const float X = grid_point(px.j, g.W, Wo), Y = grid_point(px.i, g.H, Ho);
    const int64_t Pg = (int64_t)g.Hg * g.Wg;
    const int64_t c = (int64_t)cell_of(px.i, Ho, g.Hg) * g.Wg + cell_of(px.j, Wo, g.Wg);
    PixelBlend<K> b;
    blend<K, false>(rec, (uint32_t)g.n_slots, topk, Pg, c, X, Y, b, lane_rot() % K);
    const int64_t Po = (int64_t)Ho * Wo, o = (int64_t)px.i * Wo + px.j;
    out[o] = b.c[0];
    out[Po + o] = b.c[1];
    out[2 * Po + o] = b.c[2];
}

__global__ __launch_bounds__(256) void k_fill_planes(uint32_t *__restrict__ p, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = SAD_INVALID_ID;
}

static sad_status check_grid(const char *what, int32_t Hg, int32_t Wg) {
    SAD_REQUIRE(Hg >= 1 && Wg >= 1 && (int64_t)Hg * Wg <= ((int64_t)1 << 30),
                SAD_ERR_INVALID_ARGUMENT, "%s: bad grid %d x %d", what, Hg, Wg);
    return SAD_OK;
}

static int jfa_steps(int32_t Hg, int32_t Wg, int32_t *steps) {
    const int m = Hg > Wg ? Hg : Wg;
    int L = 0;
    while ((1LL << L) < m) ++L;
    for (int k = 0; k < L; ++k) steps[k] = 1 << (L - 1 - k);
    return L;
}

static void launch_flood(const GridArgs &g, const float *rec, const uint32_t *in, uint32_t *out,
                         int step, hipStream_t st) {
    hipLaunchKernelGGL(k_jfa_flood, dim3(g.n_blocks), dim3(256), 0, st, g, step,
                       reinterpret_cast<const float4 *>(rec), reinterpret_cast<const uint4 *>(in),
                       reinterpret_cast<uint4 *>(out));
}

static void fill_invalid(uint32_t *p, int64_t n, hipStream_t st) {
    if (n > 0)
        hipLaunchKernelGGL(k_fill_planes, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, p, n);
}

}  // namespace sad

using namespace sad;

extern "C" int32_t sad_jfa_steps(int32_t Hg, int32_t Wg, int32_t *steps) {
    if (Hg < 1 || Wg < 1 || !steps) return -1;
    return jfa_steps(Hg, Wg, steps);
}

extern "C" sad_status sad_seed_grid(const sad_image *img, int32_t Hg, int32_t Wg,
                                    int32_t n_entries, const float *rec, uint32_t *topk,
                                    uint64_t *scratch, void *stream) {
    SAD_TRY(check_image(img, nullptr));
    SAD_TRY(check_grid("sad_seed_grid", Hg, Wg));
    SAD_REQUIRE(n_entries >= 0 && n_entries <= img->K, SAD_ERR_INVALID_ARGUMENT,
                "sad_seed_grid: n_entries must be in [0, K]");
    SAD_REQUIRE(topk && scratch && (rec || img->n_slots == 0), SAD_ERR_INVALID_ARGUMENT,
                "sad_seed_grid: NULL pointer");
    SAD_REQUIRE(!rec || aligned16(rec), SAD_ERR_INVALID_ARGUMENT,
                "sad_seed_grid: rec not 16-byte aligned");
    launch_seed(img, Hg, Wg, n_entries, rec, topk, scratch, as_stream(stream));
    return check_launch("sad_seed_grid");
}

extern "C" sad_status sad_propagate_grid(const sad_image *img, int32_t Hg, int32_t Wg,
                                         const float *rec, const uint32_t *topk_in,
                                         uint32_t *topk_out, int32_t jump, int32_t n_inject,
                                         uint64_t seed, uint64_t pass_index, void *stream) {
    SAD_TRY(check_image(img, nullptr));
    SAD_TRY(check_grid("sad_propagate_grid", Hg, Wg));
    SAD_REQUIRE(topk_in && topk_out, SAD_ERR_INVALID_ARGUMENT, "sad_propagate_grid: NULL list");
    SAD_REQUIRE(topk_in != topk_out, SAD_ERR_INVALID_ARGUMENT,
                "sad_propagate_grid: topk_in and topk_out must not alias (Jacobi pass)");
    SAD_REQUIRE(aligned16(topk_in) && aligned16(topk_out), SAD_ERR_INVALID_ARGUMENT,
                "sad_propagate_grid: lists must be 16-byte aligned");
    SAD_REQUIRE(jump >= 1, SAD_ERR_INVALID_ARGUMENT, "sad_propagate_grid: jump must be >= 1");
    SAD_REQUIRE(n_inject >= 0 && n_inject <= 16, SAD_ERR_INVALID_ARGUMENT,
                "sad_propagate_grid: n_inject must be in [0, 16]");
    SAD_REQUIRE(img->n_slots == 0 || (rec && aligned16(rec)), SAD_ERR_INVALID_ARGUMENT,
                "sad_propagate_grid: rec NULL or not 16-byte aligned");
    launch_propagate_grid(img, Hg, Wg, rec, topk_in, topk_out, jump, n_inject, seed, pass_index,
                          nullptr, as_stream(stream));
    return check_launch("sad_propagate_grid");
}

extern "C" sad_status sad_jfa_flood(const sad_image *img, int32_t Hg, int32_t Wg,
                                    const float *rec, const uint32_t *topk_in,
                                    uint32_t *topk_out, int32_t step, void *stream) {
    SAD_TRY(check_image(img, nullptr));
    SAD_TRY(check_grid("sad_jfa_flood", Hg, Wg));
    SAD_REQUIRE(topk_in && topk_out, SAD_ERR_INVALID_ARGUMENT, "sad_jfa_flood: NULL list");
    SAD_REQUIRE(topk_in != topk_out, SAD_ERR_INVALID_ARGUMENT,
                "sad_jfa_flood: topk_in and topk_out must not alias (Jacobi pass)");
    SAD_REQUIRE(aligned16(topk_in) && aligned16(topk_out), SAD_ERR_INVALID_ARGUMENT,
                "sad_jfa_flood: lists must be 16-byte aligned");
    SAD_REQUIRE(step >= 1, SAD_ERR_INVALID_ARGUMENT, "sad_jfa_flood: step must be >= 1");
    hipStream_t st = as_stream(stream);
    if (img->n_slots == 0) {  // no site: every first entry is empty
        fill_invalid(topk_out, (int64_t)Hg * Wg * 4, st);
        return check_launch("sad_jfa_flood");
    }
    SAD_REQUIRE(rec && aligned16(rec), SAD_ERR_INVALID_ARGUMENT,
                "sad_jfa_flood: rec NULL or not 16-byte aligned");
    launch_flood(grid_args(img, Hg, Wg), rec, topk_in, topk_out, step, st);
    return check_launch("sad_jfa_flood");
}

extern "C" sad_status sad_refresh(const sad_image *img, int32_t Hg, int32_t Wg, uint32_t flags,
                                  int32_t n_pass, int32_t n_inject, uint64_t seed,
                                  const float *rec, uint32_t *topk, uint32_t *topk_tmp,
                                  uint64_t *scratch, void *stream) {
    SAD_TRY(check_image(img, nullptr));
    SAD_TRY(check_grid("sad_refresh", Hg, Wg));
    SAD_REQUIRE(n_pass >= 0 && n_pass <= 4096, SAD_ERR_INVALID_ARGUMENT,
                "sad_refresh: n_pass must be in [0, 4096]");
    SAD_REQUIRE(n_inject >= 0 && n_inject <= 16, SAD_ERR_INVALID_ARGUMENT,
                "sad_refresh: n_inject must be in [0, 16]");
    SAD_REQUIRE((flags & ~SAD_REFRESH_JFA) == 0, SAD_ERR_INVALID_ARGUMENT,
                "sad_refresh: unknown flags 0x%x", flags);
    SAD_REQUIRE(topk && topk_tmp && scratch, SAD_ERR_INVALID_ARGUMENT, "sad_refresh: NULL pointer");
    SAD_REQUIRE(topk != topk_tmp, SAD_ERR_INVALID_ARGUMENT,
                "sad_refresh: topk and topk_tmp must be different buffers");
    SAD_REQUIRE(aligned16(topk) && aligned16(topk_tmp), SAD_ERR_INVALID_ARGUMENT,
                "sad_refresh: lists must be 16-byte aligned");
    SAD_REQUIRE(img->n_slots == 0 || (rec && aligned16(rec)), SAD_ERR_INVALID_ARGUMENT,
                "sad_refresh: rec NULL or not 16-byte aligned");
    hipStream_t st = as_stream(stream);
    const int64_t P = (int64_t)Hg * Wg;
    if (img->n_slots == 0) {
        fill_invalid(topk, P * img->K, st);
        return check_launch("sad_refresh");
    }
    const bool jfa = (flags & SAD_REFRESH_JFA) != 0;
    int32_t steps[32];
    const int L = jfa ? jfa_steps(Hg, Wg, steps) : 0;
    // Ping-pong between the two buffers, seeding the one that makes the last pass land
    // in topk.
    uint32_t *cur = ((L + n_pass) % 2 == 0) ? topk : topk_tmp;
    uint32_t *nxt = cur == topk ? topk_tmp : topk;
    launch_seed(img, Hg, Wg, jfa ? 4 : img->K, rec, cur, scratch, st);
    if (L > 0) {
        // the floods write plane 0 only: the other buffer's later planes start empty
        fill_invalid(nxt + P * 4, P * (img->K - 4), st);
        const GridArgs g = grid_args(img, Hg, Wg);
        for (int k = 0; k < L; ++k) {
            launch_flood(g, rec, cur, nxt, steps[k], st);
            uint32_t *t = cur;
            cur = nxt;
            nxt = t;
        }
    }
    for (int t = 0; t < n_pass; ++t) {
        launch_propagate_grid(img, Hg, Wg, rec, cur, nxt, jump_of(t, Hg, Wg), n_inject, seed,
                              (uint64_t)t, nullptr, st);
        uint32_t *tmp = cur;
        cur = nxt;
        nxt = tmp;
    }
    return check_launch("sad_refresh");
}

extern "C" sad_status sad_render_grid(const sad_image *img, int32_t Hg, int32_t Wg,
                                      const float *rec, const uint32_t *topk, int32_t Ho,
                                      int32_t Wo, float *out, void *stream) {
    SAD_TRY(check_image(img, nullptr));
    SAD_TRY(check_grid("sad_render_grid", Hg, Wg));
    SAD_TRY(check_grid("sad_render_grid (output)", Ho, Wo));
    SAD_REQUIRE(topk && out, SAD_ERR_INVALID_ARGUMENT, "sad_render_grid: NULL pointer");
    SAD_REQUIRE(aligned16(topk), SAD_ERR_INVALID_ARGUMENT,
                "sad_render_grid: topk must be 16-byte aligned");
    SAD_REQUIRE(img->n_slots == 0 || (rec && aligned16(rec)), SAD_ERR_INVALID_ARGUMENT,
                "sad_render_grid: rec NULL or not 16-byte aligned");
    hipStream_t st = as_stream(stream);
    const int64_t Po = (int64_t)Ho * Wo;
    if (img->n_slots == 0) {  // every list is empty: the image is black
        launch_fill_f32(out, 3 * Po, 0.0f, st);
        return check_launch("sad_render_grid");
    }
    const GridArgs g = grid_args(img, Hg, Wg);
    const int txo = (Wo + 15) / 16, nbo = txo * ((Ho + 15) / 16);
    const float4 *r4 = reinterpret_cast<const float4 *>(rec);
    const uint4 *t4 = reinterpret_cast<const uint4 *>(topk);
    SAD_K_SWITCH(img->K, hipLaunchKernelGGL((k_fwd_grid<KK>), dim3(nbo), dim3(256), 0, st, g, Ho,
                                            Wo, txo, nbo, r4, t4, out));
    return check_launch("sad_render_grid");
}
