/*
 * sad_oracle.c -- plain, slow CPU oracle for the Soft Anisotropic Diagrams hot path.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the reference the GPU library is checked
 * against.  Only the test suite, the smoke check and the benchmark's CPU-baseline leg
 * may load it.  The GPU library never includes, links or calls anything here, and
 * nothing here includes the GPU library's headers.
 *
 * Precision policy
 *   - The per-site score l_i(x) is the quantity that decides integers (which sites
 *     enter a top-K list).  The paper keeps sites in float32 (App. B.2, "Site
 *     buffer"), so scores are evaluated in float32 in one fixed sequence of
 *     correctly rounded operations (see score_f32 below); the two transcendentals
 *     per site are evaluated in double and rounded once to float.
 *   - Everything else (softmax blend, loss, gradients, removal delta, Adam,
 *     initialisation keys) is evaluated in double.  Blend and gradients take the
 *     float32 scores as their logits, so that the weights belong to the same scores
 *     that chose the list; an all-double mode (SCORE_F64) exists for
 *     finite-difference checks.
 *
 * Layouts (all host memory)
 *   sites  : float[10][cap], parameter-major, order (x, y, log_tau, r, c_r, c_g, c_b,
 *            u_x, u_y, a) as in App. B.2 "Site buffer".  A site is active iff x >= 0
 *            and all ten values are finite.
 *   lists  : uint32[H*W][K], pixel-major, one row of K site IDs per pixel (row-major
 *            pixels, pixel id = i*W + j), 0xFFFFFFFF = empty slot.
 *   images : double or float [3][H][W].
 * Pixel (row i, column j) is evaluated at the point x = (j, i).
 *
 * Parity status of each function is stated in its comment; the pins live in tests/.
 *
 * Threads: loops whose iterations are independent pixels (top-K, seed, propagation,
 * blend, queries) are split over OpenMP threads; each pixel's result does not depend
 * on the split.  The backward sums each thread's pixels into its own buffer and adds
 * the buffers in thread order (double precision; the order of additions depends on the
 * thread count only).  ora_set_threads(1) runs everything on one core.
 */
#include <math.h>
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORA_INVALID 0xFFFFFFFFu
#define ORA_PI 3.14159265358979323846264338327950288
enum { P_X, P_Y, P_LOGTAU, P_R, P_CR, P_CG, P_CB, P_UX, P_UY, P_A, NPARAM };

/* ------------------------------------------------------------------------------ */
/* Per-site quantities (Sec. 4.1, "Site Representation")                            */
/* ------------------------------------------------------------------------------ */

typedef struct {
    int valid;
    float x, y, log_tau, r, c[3], ux, uy, a;
    /* float32 derived values (canonical) */
    float tau, ep, em, kappa, g11, g12, g22;
} site_t;

static float prm(const float *sites, int64_t cap, int p, int64_t i) { return sites[(int64_t)p * cap + i]; }

/* Sec. 4.1: G = e^a u u^T + e^-a v v^T with v the 90-degree rotation (-u_y, u_x) of u,
 * so det G = |u|^4 and the eigenvalues along u and v are e^a |u|^2 and e^-a |u|^2.
 * tau = exp(log_tau) (Sec. 4.1 list of parameters); kappa = tau * s folds the
 * resolution scale s of d_mix into the temperature.  The three metric entries are
 * formed in float32 in a fixed order. */
static site_t site_load(const float *sites, int64_t cap, int64_t i, float s)
{
    site_t t;
    memset(&t, 0, sizeof t);
    t.x = prm(sites, cap, P_X, i);       t.y = prm(sites, cap, P_Y, i);
    t.log_tau = prm(sites, cap, P_LOGTAU, i);
    t.r = prm(sites, cap, P_R, i);
    t.c[0] = prm(sites, cap, P_CR, i);   t.c[1] = prm(sites, cap, P_CG, i);
    t.c[2] = prm(sites, cap, P_CB, i);
    t.ux = prm(sites, cap, P_UX, i);     t.uy = prm(sites, cap, P_UY, i);
    t.a = prm(sites, cap, P_A, i);
    int finite = 1;
    for (int p = 0; p < NPARAM; ++p) finite &= isfinite(prm(sites, cap, p, i)) ? 1 : 0;
    /* App. B.2: an inactive site has x < 0, and every kernel skips it. */
    t.valid = finite && t.x >= 0.0f;
    if (!t.valid) return t;
    t.tau = (float)exp((double)t.log_tau);
    t.ep = (float)exp((double)t.a);
    t.em = (float)exp(-(double)t.a);
    t.kappa = t.tau * s;
    float uxx = t.ux * t.ux, uyy = t.uy * t.uy, uxy = t.ux * t.uy;
    t.g11 = fmaf(t.ep, uxx, t.em * uyy);
    t.g22 = fmaf(t.ep, uyy, t.em * uxx);
    t.g12 = (t.ep - t.em) * uxy;
    if (!(t.kappa > 0.0f) || !isfinite(t.kappa) || !isfinite(t.g11) || !isfinite(t.g12) ||
        !isfinite(t.g22))
        t.valid = 0;
    return t;
}

/* Exposed for pins: derived[i] = {valid, tau, e^a, e^-a, kappa, G11, G12, G22}. */
void ora_site_derived(const float *sites, int64_t cap, int64_t n, float s, float *out)
{
    for (int64_t i = 0; i < n; ++i) {
        site_t t = site_load(sites, cap, i, s);
        float *o = out + 8 * i;
        o[0] = (float)t.valid; o[1] = t.tau; o[2] = t.ep; o[3] = t.em; o[4] = t.kappa;
        o[5] = t.g11; o[6] = t.g12; o[7] = t.g22;
    }
}

/* Sec. 4.1-4.2: l_i(x) = -tau_i d_mix(x,i) = tau_i s (r_i - ||x - p_i||_{G_i}).
 * Canonical float32 sequence (every step correctly rounded, no contraction):
 *   dx = X - p_x, dy = Y - p_y
 *   t  = fma(2 G12, dy, G11 dx)          -> G11 dx + 2 G12 dy
 *   q  = fma(t, dx, (G22 dy) dy)          -> d^T G d
 *   q  = max(q, 0);  n = sqrt(q);  l = kappa (r - n);  l = l + 0  (signed zero -> +0)
 * The list order is (l descending, ID ascending). */
static float score_f32(const site_t *t, float X, float Y)
{
    float dx = X - t->x, dy = Y - t->y;
    float tt = fmaf(2.0f * t->g12, dy, t->g11 * dx);
    float q = fmaf(tt, dx, (t->g22 * dy) * dy);
    if (!(q > 0.0f)) q = 0.0f;
    float n = sqrtf(q);
    float l = t->kappa * (t->r - n);
    return l + 0.0f;
}

/* The same score entirely in double (finite-difference checks only). */
static double score_f64(const site_t *t, double s, double X, double Y, double *n_out)
{
    double dx = X - (double)t->x, dy = Y - (double)t->y;
    double ux = t->ux, uy = t->uy;
    double ep = exp((double)t->a), em = exp(-(double)t->a);
    double al = ux * dx + uy * dy;    /* u . d */
    double be = -uy * dx + ux * dy;   /* v . d, v = (-u_y, u_x) */
    double q = ep * al * al + em * be * be;
    double n = sqrt(q > 0 ? q : 0);
    if (n_out) *n_out = n;
    return exp((double)t->log_tau) * s * ((double)t->r - n);
}

float ora_score(const float *sites, int64_t cap, int64_t id, float s, float X, float Y)
{
    site_t t = site_load(sites, cap, id, s);
    return t.valid ? score_f32(&t, X, Y) : -INFINITY;
}

double ora_score_f64(const float *sites, int64_t cap, int64_t id, double s, double X, double Y)
{
    site_t t = site_load(sites, cap, id, (float)s);
    return t.valid ? score_f64(&t, s, X, Y, NULL) : -INFINITY;
}

/* ------------------------------------------------------------------------------ */
/* Top-K selection (Sec. 4.3 update equation; storage Sec. 4.6)                     */
/* ------------------------------------------------------------------------------ */

typedef struct { float l; uint32_t id; } cand_t;

/* (l descending, ID ascending): a strict total order on distinct IDs. */
static int cand_cmp(const void *pa, const void *pb)
{
    const cand_t *a = (const cand_t *)pa, *b = (const cand_t *)pb;
    if (a->l > b->l) return -1;
    if (a->l < b->l) return 1;
    if (a->id < b->id) return -1;
    if (a->id > b->id) return 1;
    return 0;
}

/* Sort candidates, drop repeated IDs (a set union in the update equation), keep the
 * first K, pad with the empty sentinel. */
static void select_topk(cand_t *c, int nc, int K, uint32_t *out)
{
    qsort(c, (size_t)nc, sizeof(cand_t), cand_cmp);
    int k = 0;
    for (int i = 0; i < nc && k < K; ++i) {
        if (i > 0 && c[i].id == c[i - 1].id) continue;
        out[k++] = c[i].id;
    }
    for (; k < K; ++k) out[k] = ORA_INVALID;
}

/* Exact top-K over every active site, for the pixels listed in pix (or all pixels if
 * pix is NULL).  out: [npix][K].  Parity: pinned (k-d tree k-NN in the isotropic case,
 * brute force by definition). */
void ora_brute_topk(int H, int W, int K, float s, const float *sites, int64_t cap, int64_t n,
                    const int64_t *pix, int64_t npix, uint32_t *out)
{
    site_t *st = (site_t *)malloc(sizeof(site_t) * (size_t)(n > 0 ? n : 1));
    for (int64_t i = 0; i < n; ++i) st[i] = site_load(sites, cap, i, s);
    int64_t total = pix ? npix : (int64_t)H * W;
#pragma omp parallel
    {
        cand_t *c = (cand_t *)malloc(sizeof(cand_t) * (size_t)(n > 0 ? n : 1));
#pragma omp for schedule(dynamic, 64)
        for (int64_t q = 0; q < total; ++q) {
            int64_t p = pix ? pix[q] : q;
            float X = (float)(p % W), Y = (float)(p / W);
            int nc = 0;
            for (int64_t i = 0; i < n; ++i)
                if (st[i].valid) { c[nc].l = score_f32(&st[i], X, Y); c[nc].id = (uint32_t)i; ++nc; }
            select_topk(c, nc, K, out + q * K);
        }
        free(c);
    }
    free(st);
}

/* Initial lists (the seed pass of App. B.3): each active site is mapped to the pixel
 * nearest its centre, (rint(p_y), rint(p_x)) clamped to the image, and each pixel's
 * list is the top-K of the sites mapped to it.  Parity: pinned (brute force). */
void ora_seed(int H, int W, int K, float s, const float *sites, int64_t cap, int64_t n,
              uint32_t *lists)
{
    int64_t P = (int64_t)H * W;
    for (int64_t p = 0; p < P * K; ++p) lists[p] = ORA_INVALID;
    /* bucket sites by pixel (counting pass, then fill) */
    int64_t *cnt = (int64_t *)calloc((size_t)P + 1, sizeof(int64_t));
    int64_t *where = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
    site_t *st = (site_t *)malloc(sizeof(site_t) * (size_t)(n > 0 ? n : 1));
    for (int64_t i = 0; i < n; ++i) {
        st[i] = site_load(sites, cap, i, s);
        where[i] = -1;
        if (!st[i].valid) continue;
        float fi = rintf(st[i].y), fj = rintf(st[i].x);
        int64_t ii = fi < 0 ? 0 : (fi > (float)(H - 1) ? H - 1 : (int64_t)fi);
        int64_t jj = fj < 0 ? 0 : (fj > (float)(W - 1) ? W - 1 : (int64_t)fj);
        where[i] = ii * W + jj;
        cnt[where[i]]++;
    }
    /* brute force per occupied pixel: gather its sites */
#pragma omp parallel
    {
        cand_t *c = (cand_t *)malloc(sizeof(cand_t) * (size_t)(n > 0 ? n : 1));
#pragma omp for schedule(dynamic, 256)
        for (int64_t p = 0; p < P; ++p) {
            if (!cnt[p]) continue;
            float X = (float)(p % W), Y = (float)(p / W);
            int nc = 0;
            for (int64_t i = 0; i < n; ++i)
                if (where[i] == p) { c[nc].l = score_f32(&st[i], X, Y); c[nc].id = (uint32_t)i; ++nc; }
            select_topk(c, nc, K, lists + p * K);
        }
        free(c);
    }
    free(cnt); free(where); free(st);
}

/* ------------------------------------------------------------------------------ */
/* Jump schedule and stochastic injection (Sec. 4.3; App. B.3 "Step encoding")      */
/* ------------------------------------------------------------------------------ */

/* Sec. 4.3: B = 2^ceil(log2 max(H,W)), s_t = max(1, B / 2^(min(t, log2 B - 1) + 1)). */
int ora_jump(int64_t t, int H, int W)
{
    int m = H > W ? H : W;
    int lb = 0;
    while ((1LL << lb) < m) ++lb;               /* lb = ceil(log2 m) */
    int64_t B = 1LL << lb;
    int64_t e = t < (int64_t)(lb - 1) ? t : (int64_t)(lb - 1);
    if (e < 0) e = 0;                           /* B = 1 (1x1 image): step 1 */
    int64_t st = B >> (e + 1);
    return (int)(st > 1 ? st : 1);
}

/* SplitMix64 (Steele, Lea, Flood, OOPSLA 2014): output number k (0-based) of the stream
 * seeded with `seed` is mix(seed + (k+1) * 0x9E3779B97F4A7C15), with the published
 * finaliser mix(z) = z3 where z1 = (z ^ z>>30) * 0xBF58476D1CE4E5B9,
 * z2 = (z1 ^ z1>>27) * 0x94D049BB133111EB, z3 = z2 ^ z2>>31. */
uint64_t ora_splitmix64(uint64_t seed, uint64_t k)
{
    uint64_t z = seed + (k + 1) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

/* Injected candidate j of pass t at pixel p: counter k = (t*P + p)*J + j, ID =
 * floor(hi32 * n_slots / 2^32).  (The paper seeds an xorshift with step index and pixel
 * ID; a stateless counter generator gives the same role with a reproducible stream.) */
uint32_t ora_inject_id(uint64_t seed, uint64_t t, int64_t P, int64_t p, int J, int j,
                       uint32_t n_slots)
{
    uint64_t k = ((uint64_t)t * (uint64_t)P + (uint64_t)p) * (uint64_t)J + (uint64_t)j;
    uint64_t hi = ora_splitmix64(seed, k) >> 32;
    return (uint32_t)((hi * (uint64_t)n_slots) >> 32);
}

/* ------------------------------------------------------------------------------ */
/* Evaluation grids (App. B.3 "Downscaled candidate grid")                          */
/* ------------------------------------------------------------------------------ */

/* A list field may live on a grid of Hg x Wg cells laid over the H x W image (the
 * image's own pixels are the grid Hg = H, Wg = W).  Cell (i', j') is evaluated at the
 * centre of its square in UV space, ((j' + 1/2)/Wg, (i' + 1/2)/Hg); with pixel j at
 * x = j (UV u <-> x = u W - 1/2) that is x = ((2 j' + 1) W - Wg) / (2 Wg): a ratio of
 * exact integers, divided in double and rounded once to float.  For Wg = W it is j'
 * exactly.  Parity: pinned (integer centres on the image's own grid; the mean of the
 * s covered pixel coordinates when W = s Wg; the closed form of a 2x finer grid). */
static float grid_coord(int64_t j, int n_img, int n_grid)
{
    double num = (double)(2 * j + 1) * (double)n_img - (double)n_grid;
    return (float)(num / (2.0 * (double)n_grid));
}

/* The integer map from image pixels to cells: pixel j lies in the cell whose UV
 * interval holds the pixel's centre, floor((2 j + 1) Wg / (2 W)); when W = s Wg that is
 * floor(j / s), the integer mapping (no interpolation) of App. B.3. */
static int64_t cell_of(int64_t j, int n_img, int n_grid)
{
    return ((2 * j + 1) * (int64_t)n_grid) / (2 * (int64_t)n_img);
}

/* Exposed for pins: xy[Hg*Wg][2] = the points of every cell; cell[H*W] = the cell of
 * every image pixel (row-major cell index i' Wg + j'). */
void ora_grid_points(int H, int W, int Hg, int Wg, float *xy, int64_t *cell)
{
    if (xy)
        for (int64_t i = 0; i < Hg; ++i)
            for (int64_t j = 0; j < Wg; ++j) {
                xy[2 * (i * Wg + j)] = grid_coord(j, W, Wg);
                xy[2 * (i * Wg + j) + 1] = grid_coord(i, H, Hg);
            }
    if (cell)
        for (int64_t i = 0; i < H; ++i)
            for (int64_t j = 0; j < W; ++j)
                cell[i * W + j] = cell_of(i, H, Hg) * Wg + cell_of(j, W, Wg);
}

/* One propagation pass on a grid (the body of ora_prop_pass; ora_prop_pass is the
 * image's own grid).  Lists are [Hg*Wg][K]; neighbours at +-jump cells; candidates are
 * scored at the cell's point; injection counters use P = Hg Wg and the cell index. */
static void prop_pass_impl(int H, int W, int Hg, int Wg, int K, float s, const float *sites,
                           int64_t cap, int64_t n, const uint32_t *in, uint32_t *out, int jump,
                           int J, uint64_t seed, uint64_t t, const int64_t *pix, int64_t npix)
{
    int64_t P = (int64_t)Hg * Wg;
    site_t *st = (site_t *)malloc(sizeof(site_t) * (size_t)(n > 0 ? n : 1));
    for (int64_t i = 0; i < n; ++i) st[i] = site_load(sites, cap, i, s);
    int64_t total = pix ? npix : P;
#pragma omp parallel
    {
    cand_t *c = (cand_t *)malloc(sizeof(cand_t) * (size_t)(5 * K + J + 1));
#pragma omp for schedule(dynamic, 256)
    for (int64_t q = 0; q < total; ++q) {
        int64_t p = pix ? pix[q] : q;
        int64_t i = p / Wg, j = p % Wg;
        float X = grid_coord(j, W, Wg), Y = grid_coord(i, H, Hg);
        int64_t src[5]; int ns = 0;
        src[ns++] = p;
        if (j + jump < Wg) src[ns++] = p + jump;
        if (j - jump >= 0) src[ns++] = p - jump;
        if (i + jump < Hg) src[ns++] = p + (int64_t)jump * Wg;
        if (i - jump >= 0) src[ns++] = p - (int64_t)jump * Wg;
        int nc = 0;
        for (int a = 0; a < ns; ++a)
            for (int k = 0; k < K; ++k) {
                uint32_t id = in[src[a] * K + k];
                if (id == ORA_INVALID || (int64_t)id >= n || !st[id].valid) continue;
                c[nc].l = score_f32(&st[id], X, Y); c[nc].id = id; ++nc;
            }
        for (int jj = 0; jj < J; ++jj) {
            uint32_t id = n > 0 ? ora_inject_id(seed, t, P, p, J, jj, (uint32_t)n) : ORA_INVALID;
            if (id == ORA_INVALID || (int64_t)id >= n || !st[id].valid) continue;
            c[nc].l = score_f32(&st[id], X, Y); c[nc].id = id; ++nc;
        }
        select_topk(c, nc, K, out + q * K);
    }
    free(c);
    }
    free(st);
}

/* One propagation pass (Sec. 4.3 update equation), Jacobi: every pixel reads the
 * previous field `in` and writes `out`.  Candidates: the pixel's own list, the lists
 * at (+-jump, 0) and (0, +-jump) that lie inside the image, and J injected IDs.  IDs
 * that are empty, out of range or inactive are dropped; the rest are scored with the
 * current sites and the top K of the set are kept.  If pix != NULL only those pixels
 * are computed (out is then [npix][K]).  Parity: pinned by invariants
 * (sortedness, uniqueness, monotonicity, convergence to brute force, dilation). */
void ora_prop_pass(int H, int W, int K, float s, const float *sites, int64_t cap, int64_t n,
                   const uint32_t *in, uint32_t *out, int jump, int J, uint64_t seed,
                   uint64_t t, const int64_t *pix, int64_t npix)
{
    prop_pass_impl(H, W, H, W, K, s, sites, cap, n, in, out, jump, J, seed, t, pix, npix);
}

/* The same pass on a candidate grid of Hg x Wg cells (App. B.3): lists [Hg*Wg][K].
 * Parity: pinned (equals ora_prop_pass on the image's own grid; converges to the exact
 * top K at the cell points when K >= active sites; invariants as ora_prop_pass). */
void ora_prop_pass_grid(int H, int W, int Hg, int Wg, int K, float s, const float *sites,
                        int64_t cap, int64_t n, const uint32_t *in, uint32_t *out, int jump,
                        int J, uint64_t seed, uint64_t t)
{
    prop_pass_impl(H, W, Hg, Wg, K, s, sites, cap, n, in, out, jump, J, seed, t, NULL, 0);
}

/* ------------------------------------------------------------------------------ */
/* Full refresh: seed pass and JFA flood prepass (App. B.3 "JFA prepass")            */
/* ------------------------------------------------------------------------------ */

/* Seed pass on a grid: every slot cleared; each active site goes to the cell of its
 * nearest image pixel ((rint(p_y), rint(p_x)) clamped, then cell_of), and each cell
 * keeps the best n_entries (<= K) of its sites by (score at the cell point descending,
 * ID ascending).  On the image's own grid with n_entries = K this is ora_seed; the JFA
 * prepass seeds n_entries = 4 (the first candidate texture).  Parity: pinned (equals
 * ora_seed on the image grid; brute force over the sites of each cell). */
void ora_seed_grid(int H, int W, int Hg, int Wg, int K, int n_entries, float s,
                   const float *sites, int64_t cap, int64_t n, uint32_t *lists)
{
    int64_t P = (int64_t)Hg * Wg;
    for (int64_t p = 0; p < P * K; ++p) lists[p] = ORA_INVALID;
    if (n_entries > K) n_entries = K;
    int64_t *where = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
    site_t *st = (site_t *)malloc(sizeof(site_t) * (size_t)(n > 0 ? n : 1));
    char *busy = (char *)calloc((size_t)P, 1);
    for (int64_t i = 0; i < n; ++i) {
        st[i] = site_load(sites, cap, i, s);
        where[i] = -1;
        if (!st[i].valid) continue;
        float fi = rintf(st[i].y), fj = rintf(st[i].x);
        int64_t ii = fi < 0 ? 0 : (fi > (float)(H - 1) ? H - 1 : (int64_t)fi);
        int64_t jj = fj < 0 ? 0 : (fj > (float)(W - 1) ? W - 1 : (int64_t)fj);
        where[i] = cell_of(ii, H, Hg) * Wg + cell_of(jj, W, Wg);
        busy[where[i]] = 1;
    }
    cand_t *c = (cand_t *)malloc(sizeof(cand_t) * (size_t)(n > 0 ? n : 1));
    uint32_t *tmp = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)K);
    for (int64_t p = 0; p < P; ++p) {
        if (!busy[p]) continue;
        float X = grid_coord(p % Wg, W, Wg), Y = grid_coord(p / Wg, H, Hg);
        int nc = 0;
        for (int64_t i = 0; i < n; ++i)
            if (where[i] == p) { c[nc].l = score_f32(&st[i], X, Y); c[nc].id = (uint32_t)i; ++nc; }
        select_topk(c, nc, n_entries, tmp);
        for (int k = 0; k < n_entries; ++k) lists[p * K + k] = tmp[k];
    }
    free(c); free(tmp); free(busy); free(where); free(st);
}

/* Steps of the JFA prepass on an Hg x Wg grid: L = ceil(log2 max(Hg, Wg)) flood passes
 * with steps 2^(L-1), ..., 2, 1 (App. B.3: a seed pass and ceil(log2 max(W, H)) flood
 * passes).  Writes up to 31 steps into steps[]; returns L. */
int ora_jfa_steps(int Hg, int Wg, int *steps)
{
    int m = Hg > Wg ? Hg : Wg;
    int L = 0;
    while ((1LL << L) < m) ++L;
    for (int k = 0; k < L; ++k) steps[k] = 1 << (L - 1 - k);
    return L;
}

/* One JFA flood pass (App. B.3), Jacobi: cell p gathers the first four entries (the
 * first candidate texture) of the cells at (dx, dy) step with dx, dy in {-1, 0, 1}
 * inside the grid (its own included), drops empty, out-of-range and inactive IDs and
 * repeats, scores the rest at its point and writes the best four, by (score
 * descending, ID ascending), into entries 0..3 of out; entries 4..K-1 of out are not
 * written.  Parity: pinned (a single site floods every cell; with at most four active
 * sites the prepass ends with the exact lists; per-entry scores never fall pass to pass;
 * never above the exact top 4; the diagonal neighbours matter). */
void ora_jfa_flood(int H, int W, int Hg, int Wg, int K, float s, const float *sites,
                   int64_t cap, int64_t n, const uint32_t *in, uint32_t *out, int step)
{
    int64_t P = (int64_t)Hg * Wg;
    site_t *st = (site_t *)malloc(sizeof(site_t) * (size_t)(n > 0 ? n : 1));
    for (int64_t i = 0; i < n; ++i) st[i] = site_load(sites, cap, i, s);
#pragma omp parallel for schedule(dynamic, 256)
    for (int64_t p = 0; p < P; ++p) {
        int64_t i = p / Wg, j = p % Wg;
        float X = grid_coord(j, W, Wg), Y = grid_coord(i, H, Hg);
        cand_t c[36];
        int nc = 0;
        for (int di = -1; di <= 1; ++di)
            for (int dj = -1; dj <= 1; ++dj) {
                int64_t ii = i + (int64_t)di * step, jj = j + (int64_t)dj * step;
                if (ii < 0 || ii >= Hg || jj < 0 || jj >= Wg) continue;
                for (int k = 0; k < 4; ++k) {
                    uint32_t id = in[(ii * Wg + jj) * K + k];
                    if (id == ORA_INVALID || (int64_t)id >= n || !st[id].valid) continue;
                    c[nc].l = score_f32(&st[id], X, Y); c[nc].id = id; ++nc;
                }
            }
        select_topk(c, nc, 4, out + p * K);
    }
    free(st);
}

/* The JFA prepass of a full refresh (App. B.3): seed pass with four entries per cell,
 * then the flood passes of ora_jfa_steps; lists [Hg*Wg][K] (entries 4..K-1 empty). */
void ora_jfa_prepass(int H, int W, int Hg, int Wg, int K, float s, const float *sites,
                     int64_t cap, int64_t n, uint32_t *lists)
{
    int64_t P = (int64_t)Hg * Wg;
    uint32_t *tmp = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)(P * K));
    ora_seed_grid(H, W, Hg, Wg, K, 4, s, sites, cap, n, lists);
    memcpy(tmp, lists, sizeof(uint32_t) * (size_t)(P * K));
    int steps[32];
    int L = ora_jfa_steps(Hg, Wg, steps);
    for (int k = 0; k < L; ++k) {
        ora_jfa_flood(H, W, Hg, Wg, K, s, sites, cap, n, lists, tmp, steps[k]);
        memcpy(lists, tmp, sizeof(uint32_t) * (size_t)(P * K));
    }
    free(tmp);
}

/* A full refresh of a list field (Sec. 6.6 "full refresh"; App. B.3): the JFA prepass
 * (jfa != 0) or the plain seed pass with K entries, then n_pass propagation passes with
 * the Sec. 4.3 schedule of the grid, pass t = 0 .. n_pass - 1 (jump ora_jump(t, Hg, Wg),
 * injection stream t).  lists [Hg*Wg][K] (written). */
void ora_refresh(int H, int W, int Hg, int Wg, int K, float s, const float *sites,
                 int64_t cap, int64_t n, int jfa, int n_pass, int J, uint64_t seed,
                 uint32_t *lists)
{
    int64_t P = (int64_t)Hg * Wg;
    if (jfa)
        ora_jfa_prepass(H, W, Hg, Wg, K, s, sites, cap, n, lists);
    else
        ora_seed_grid(H, W, Hg, Wg, K, K, s, sites, cap, n, lists);
    uint32_t *tmp = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)(P * K));
    for (int t = 0; t < n_pass; ++t) {
        prop_pass_impl(H, W, Hg, Wg, K, s, sites, cap, n, lists, tmp, ora_jump(t, Hg, Wg), J,
                       seed, (uint64_t)t, NULL, 0);
        memcpy(lists, tmp, sizeof(uint32_t) * (size_t)(P * K));
    }
    free(tmp);
}

/* ------------------------------------------------------------------------------ */
/* Soft blend (Sec. 4.2), loss (Sec. 6.1) and gradients (App. B.4)                   */
/* ------------------------------------------------------------------------------ */

enum { SCORE_F32 = 0, SCORE_F64 = 1 };

typedef struct {
    int nv;                 /* valid entries */
    int idx[64];            /* site ids of the valid entries, list order */
    double l[64], n[64];    /* logit and metric norm */
    double w[64], e[64];    /* softmax weights, exp(l - max) */
    double S, c[3];         /* sum of e, colour */
} pix_t;

/* Sec. 4.2: w_i = exp(l_i) / sum_j exp(l_j) over the valid entries of C(x) (computed
 * with the maximum subtracted, App. B.4), c(x) = sum_i w_i c_i.  An empty list gives
 * colour 0.  K <= 64. */
static void blend_pixel(const site_t *st, int64_t n, const uint32_t *list, int K, double X,
                        double Y, float s, int mode, pix_t *px)
{
    px->nv = 0; px->S = 0; px->c[0] = px->c[1] = px->c[2] = 0;
    for (int k = 0; k < K; ++k) {
        uint32_t id = list[k];
        if (id == ORA_INVALID || (int64_t)id >= n || !st[id].valid) continue;
        int v = px->nv++;
        px->idx[v] = (int)id;
        double nn;
        double l64 = score_f64(&st[id], (double)s, X, Y, &nn);
        px->n[v] = nn;
        px->l[v] = mode == SCORE_F64 ? l64 : (double)score_f32(&st[id], (float)X, (float)Y);
    }
    if (!px->nv) return;
    double m = px->l[0];
    for (int v = 1; v < px->nv; ++v) if (px->l[v] > m) m = px->l[v];
    for (int v = 0; v < px->nv; ++v) { px->e[v] = exp(px->l[v] - m); px->S += px->e[v]; }
    for (int v = 0; v < px->nv; ++v) {
        px->w[v] = px->e[v] / px->S;
        for (int ch = 0; ch < 3; ++ch) px->c[ch] += px->w[v] * (double)st[px->idx[v]].c[ch];
    }
}

/* Render every pixel from its list.  out: double[3][H][W].  Parity: pinned (partition
 * of unity, convexity, K = N full softmax, hard Apollonius limit, scale invariance). */
void ora_render(int H, int W, int K, float s, const float *sites, int64_t cap, int64_t n,
                const uint32_t *lists, int mode, double *out)
{
    int64_t P = (int64_t)H * W;
    site_t *st = (site_t *)malloc(sizeof(site_t) * (size_t)(n > 0 ? n : 1));
    for (int64_t i = 0; i < n; ++i) st[i] = site_load(sites, cap, i, s);
#pragma omp parallel for schedule(dynamic, 256)
    for (int64_t p = 0; p < P; ++p) {
        pix_t px;
        blend_pixel(st, n, lists + p * K, K, (double)(p % W), (double)(p / W), s, mode, &px);
        for (int ch = 0; ch < 3; ++ch) out[ch * P + p] = px.c[ch];
    }
    free(st);
}

/* Sec. 4.2 evaluated at arbitrary points (random access, Sec. 6.6): the list is the
 * one stored at the nearest pixel (rint, clamped), the scores are taken at the exact
 * query point.  xy: float[M][2] in pixel units (x = column, y = row); out:
 * double[M][3].  Parity: pinned (equals ora_render at integer points). */
void ora_query(int H, int W, int K, float s, const float *sites, int64_t cap, int64_t n,
               const uint32_t *lists, const float *xy, int64_t M, double *out)
{
    site_t *st = (site_t *)malloc(sizeof(site_t) * (size_t)(n > 0 ? n : 1));
    for (int64_t i = 0; i < n; ++i) st[i] = site_load(sites, cap, i, s);
#pragma omp parallel for schedule(dynamic, 256)
    for (int64_t m = 0; m < M; ++m) {
        pix_t px;
        float x = xy[2 * m], y = xy[2 * m + 1];
        float fi = rintf(y), fj = rintf(x);
        int64_t ii = !(fi > 0) ? 0 : (fi > (float)(H - 1) ? H - 1 : (int64_t)fi);
        int64_t jj = !(fj > 0) ? 0 : (fj > (float)(W - 1) ? W - 1 : (int64_t)fj);
        blend_pixel(st, n, lists + (ii * W + jj) * K, K, (double)x, (double)y, s, SCORE_F32, &px);
        for (int ch = 0; ch < 3; ++ch) out[3 * m + ch] = px.c[ch];
    }
    free(st);
}

/* Sec. 4.2 at arbitrary points with a list given per point: out[m] = the blend of
 * lists[m] at xy[m] (the decode of a list field built on a new grid, Sec. 6.6: each
 * output point of the grid takes its own cell's list).  lists: [M][K]; xy: float[M][2];
 * out: double[M][3].  Parity: pinned (equals ora_render on the image's own grid). */
void ora_blend_points(int K, float s, const float *sites, int64_t cap, int64_t n,
                      const uint32_t *lists, const float *xy, int64_t M, double *out)
{
    site_t *st = (site_t *)malloc(sizeof(site_t) * (size_t)(n > 0 ? n : 1));
    for (int64_t i = 0; i < n; ++i) st[i] = site_load(sites, cap, i, s);
#pragma omp parallel for schedule(dynamic, 256)
    for (int64_t m = 0; m < M; ++m) {
        pix_t px;
        blend_pixel(st, n, lists + m * K, K, (double)xy[2 * m], (double)xy[2 * m + 1], s,
                    SCORE_F32, &px);
        for (int ch = 0; ch < 3; ++ch) out[3 * m + ch] = px.c[ch];
    }
    free(st);
}

/* ------------------------------------------------------------------------------ */
/* Packed 16-byte inference record (App. B.2 "Packed storage for evaluation";        */
/* Sec. 6.1 BPP accounting)                                                          */
/* ------------------------------------------------------------------------------ */

/* IEEE 754 binary32 -> binary16, round to nearest, ties to even (overflow to inf, NaN
 * kept a NaN, subnormal halves rounded at their own spacing).  Written from the
 * formats' definitions.  Parity: pinned (numpy's float16 conversion). */
uint16_t ora_f32_to_f16(float f)
{
    uint32_t b;
    memcpy(&b, &f, 4);
    uint16_t sign = (uint16_t)((b >> 16) & 0x8000u);
    uint32_t ex = (b >> 23) & 0xFFu, man = b & 0x7FFFFFu;
    if (ex == 0xFFu) return (uint16_t)(sign | 0x7C00u | (man ? 0x200u : 0u));
    int e = (int)ex - 127 + 15;                      /* biased half exponent */
    if (e >= 31) return (uint16_t)(sign | 0x7C00u);  /* overflow */
    uint32_t full, shift;
    if (e <= 0) {                                    /* subnormal half (or zero) */
        if (e < -10) return sign;                    /* below half the smallest subnormal */
        full = man | 0x800000u;                      /* the implicit one */
        shift = (uint32_t)(14 - e);                  /* 13 + (1 - e) */
        uint32_t q = full >> shift, rem = full & ((1u << shift) - 1u), half = 1u << (shift - 1);
        if (rem > half || (rem == half && (q & 1u))) ++q;
        return (uint16_t)(sign | q);                 /* a carry into 0x400 is the smallest normal */
    }
    uint32_t q = man >> 13, rem = man & 0x1FFFu;
    uint32_t h = ((uint32_t)e << 10) | q;
    if (rem > 0x1000u || (rem == 0x1000u && (q & 1u))) ++h;   /* may carry into the exponent */
    return (uint16_t)(sign | h);
}

/* binary16 -> binary32 (exact). */
float ora_f16_to_f32(uint16_t h)
{
    uint32_t sign = ((uint32_t)h & 0x8000u) << 16, ex = ((uint32_t)h >> 10) & 0x1Fu,
             man = (uint32_t)h & 0x3FFu, b;
    if (ex == 0x1Fu) b = sign | 0x7F800000u | (man << 13);
    else if (ex) b = sign | ((ex - 15 + 127) << 23) | (man << 13);
    else if (!man) b = sign;
    else {                                           /* subnormal: normalise */
        int e = -1;
        do { man <<= 1; ++e; } while (!(man & 0x400u));
        b = sign | ((uint32_t)(127 - 15 - e) << 23) | ((man & 0x3FFu) << 13);
    }
    float f;
    memcpy(&f, &b, 4);
    return f;
}

/* Per-image quantisation parameters of the packed record: q = {log_tau min, scale,
 * r min, scale, c_r min, scale, c_g min, scale, c_b min, scale} with min and max over
 * the active sites and scale = max - min (all 0 without active sites). */
void ora_pack_qparams(const float *sites, int64_t cap, int64_t n, float *q)
{
    static const int par[5] = {P_LOGTAU, P_R, P_CR, P_CG, P_CB};
    float mn[5], mx[5];
    int any = 0;
    for (int k = 0; k < 5; ++k) { mn[k] = INFINITY; mx[k] = -INFINITY; }
    for (int64_t i = 0; i < n; ++i) {
        int act = prm(sites, cap, P_X, i) >= 0.0f;
        for (int p = 0; p < NPARAM; ++p) act &= isfinite(prm(sites, cap, p, i)) ? 1 : 0;
        if (!act) continue;
        any = 1;
        for (int k = 0; k < 5; ++k) {
            float v = prm(sites, cap, par[k], i);
            if (v < mn[k]) mn[k] = v;
            if (v > mx[k]) mx[k] = v;
        }
    }
    for (int k = 0; k < 5; ++k) {
        q[2 * k] = any ? mn[k] : 0.0f;
        q[2 * k + 1] = any ? mx[k] - mn[k] : 0.0f;
    }
}

/* UNORM code of v with `bits` bits over [mn, mn + sc]: t = (v - mn) / sc clamped to
 * [0, 1] (0 if sc = 0), code = rint(t (2^bits - 1)); every step one float32 operation. */
static uint32_t unorm_code(float v, float mn, float sc, int bits)
{
    float maxq = (float)((1u << bits) - 1u);
    float t = sc > 0.0f ? (v - mn) / sc : 0.0f;
    if (!(t > 0.0f)) t = 0.0f;
    if (t > 1.0f) t = 1.0f;
    return (uint32_t)rintf(t * maxq);
}

/* Decoded value of a UNORM code: mn + sc (code / (2^bits - 1)). */
static float unorm_value(uint32_t code, float mn, float sc, int bits)
{
    float maxq = (float)((1u << bits) - 1u);
    return mn + sc * ((float)code / maxq);
}

/* Angle code of the direction u over [-pi, pi] (16-bit UNORM): theta = atan2(u_y, u_x)
 * in double, code = rint((theta + pi) / (2 pi) (2^16 - 1)). */
static uint32_t angle_code(float ux, float uy)
{
    double th = atan2((double)uy, (double)ux);
    double t = (th + ORA_PI) / (2.0 * ORA_PI);
    return (uint32_t)rint(t * 65535.0);
}

/* App. B.2 packed record of every slot < n: four 32-bit words
 *   w0 = x code (15-bit UNORM over [0, W-1]) | y code << 15 (over [0, H-1]) | 1 << 31
 *        (the active flag; bit 30 is 0)
 *   w1 = c_r code (11 bits) | c_g code << 11 (11 bits) | c_b code << 22 (10 bits)
 *   w2 = log_tau code (16 bits) | r code << 16 (16 bits)
 *   w3 = angle code of u (16 bits) | float16 bits of a << 16
 * with the per-image min / scale of q for log_tau, r and the colours; an inactive slot
 * packs to four zero words.  packed: uint32[n][4].  Parity: pinned (hand-derived words
 * of edge values; round-trip error bounds; numpy float16). */
void ora_pack_sites(int H, int W, const float *sites, int64_t cap, int64_t n, const float *q,
                    uint32_t *packed)
{
    for (int64_t i = 0; i < n; ++i) {
        uint32_t *w = packed + 4 * i;
        w[0] = w[1] = w[2] = w[3] = 0;
        int act = prm(sites, cap, P_X, i) >= 0.0f;
        for (int p = 0; p < NPARAM; ++p) act &= isfinite(prm(sites, cap, p, i)) ? 1 : 0;
        if (!act) continue;
        float x = prm(sites, cap, P_X, i), y = prm(sites, cap, P_Y, i);
        uint32_t qx = unorm_code(x, 0.0f, (float)(W - 1), 15);
        uint32_t qy = unorm_code(y, 0.0f, (float)(H - 1), 15);
        w[0] = qx | (qy << 15) | 0x80000000u;
        w[1] = unorm_code(prm(sites, cap, P_CR, i), q[4], q[5], 11) |
               (unorm_code(prm(sites, cap, P_CG, i), q[6], q[7], 11) << 11) |
               (unorm_code(prm(sites, cap, P_CB, i), q[8], q[9], 10) << 22);
        w[2] = unorm_code(prm(sites, cap, P_LOGTAU, i), q[0], q[1], 16) |
               (unorm_code(prm(sites, cap, P_R, i), q[2], q[3], 16) << 16);
        w[3] = angle_code(prm(sites, cap, P_UX, i), prm(sites, cap, P_UY, i)) |
               ((uint32_t)ora_f32_to_f16(prm(sites, cap, P_A, i)) << 16);
    }
}

/* Decode of ora_pack_sites into float32 sites [10][cap] (slots < n): each UNORM as
 * unorm_value (positions over [0, W-1] and [0, H-1]); u = (cos theta, sin theta) with
 * theta = code / (2^16 - 1) 2 pi - pi in double, each rounded once to float; a from its
 * float16 bits.  A record without the active flag decodes to an inactive site
 * (x = y = -1, the rest 0). */
void ora_unpack_sites(int H, int W, const uint32_t *packed, int64_t n, const float *q,
                      float *sites, int64_t cap)
{
    for (int64_t i = 0; i < n; ++i) {
        const uint32_t *w = packed + 4 * i;
        float v[NPARAM] = {-1.0f, -1.0f, 0, 0, 0, 0, 0, 0, 0, 0};
        if (w[0] & 0x80000000u) {
            v[P_X] = unorm_value(w[0] & 0x7FFFu, 0.0f, (float)(W - 1), 15);
            v[P_Y] = unorm_value((w[0] >> 15) & 0x7FFFu, 0.0f, (float)(H - 1), 15);
            v[P_CR] = unorm_value(w[1] & 0x7FFu, q[4], q[5], 11);
            v[P_CG] = unorm_value((w[1] >> 11) & 0x7FFu, q[6], q[7], 11);
            v[P_CB] = unorm_value(w[1] >> 22, q[8], q[9], 10);
            v[P_LOGTAU] = unorm_value(w[2] & 0xFFFFu, q[0], q[1], 16);
            v[P_R] = unorm_value(w[2] >> 16, q[2], q[3], 16);
            double th = (double)(w[3] & 0xFFFFu) / 65535.0 * (2.0 * ORA_PI) - ORA_PI;
            v[P_UX] = (float)cos(th);
            v[P_UY] = (float)sin(th);
            v[P_A] = ora_f16_to_f32((uint16_t)(w[3] >> 16));
        }
        for (int p = 0; p < NPARAM; ++p) sites[(int64_t)p * cap + i] = v[p];
    }
}

/* ------------------------------------------------------------------------------ */
/* Tau diffusion (App. B.6)                                                          */
/* ------------------------------------------------------------------------------ */

/* One Jacobi step of log tau gradient smoothing: for every active, valid site i < n,
 * with N(i) = the valid sites other than i in the candidate list of the pixel nearest
 * its centre ((rint(p_y), rint(p_x)) clamped),
 *   g_out[i] = (1 - lambda) g_in[i] + lambda mean_{j in N(i)} g_in[j],
 * and g_out[i] = g_in[i] when N(i) is empty or the site is inactive.  All reads are of
 * g_in (Jacobi).  g_in, g_out: double[n].  Parity: pinned (lambda = 0 is the identity,
 * lambda = 1 the neighbour mean, a constant field is fixed, a hand-worked example). */
void ora_tau_diffusion(int H, int W, int K, float s, const float *sites, int64_t cap, int64_t n,
                       const uint32_t *lists, const double *g_in, double lambda, double *g_out)
{
    site_t *st = (site_t *)malloc(sizeof(site_t) * (size_t)(n > 0 ? n : 1));
    for (int64_t i = 0; i < n; ++i) st[i] = site_load(sites, cap, i, s);
    for (int64_t i = 0; i < n; ++i) {
        g_out[i] = g_in[i];
        if (!st[i].valid) continue;
        float fi = rintf(st[i].y), fj = rintf(st[i].x);
        int64_t ii = fi < 0 ? 0 : (fi > (float)(H - 1) ? H - 1 : (int64_t)fi);
        int64_t jj = fj < 0 ? 0 : (fj > (float)(W - 1) ? W - 1 : (int64_t)fj);
        const uint32_t *l = lists + (ii * W + jj) * K;
        double sum = 0;
        int cnt = 0;
        for (int k = 0; k < K; ++k) {
            uint32_t id = l[k];
            if (id == ORA_INVALID || (int64_t)id >= n || (int64_t)id == i || !st[id].valid) continue;
            sum += g_in[id];
            ++cnt;
        }
        if (cnt) g_out[i] = (1.0 - lambda) * g_in[i] + lambda * (sum / cnt);
    }
    free(st);
}

/* ------------------------------------------------------------------------------ */
/* One-dimensional SAD (Sec. 7 "1D Signal Fitting")                                  */
/* ------------------------------------------------------------------------------ */

/* A 1-D signal of M samples, sample m at x = m.  Each site has four parameters, stored
 * float[4][cap] in the order (p, c, log_tau, r): position, value, log-temperature and
 * radius.  The soft partition is the 2-D one on a line: the score is
 *   l_i(x) = tau_i s (r_i - |x - p_i|)
 * (the metric is the absolute value), s = 1/M unless given, and a sample blends the
 * values of its top-K list by the softmax of the scores.  Canonical float32 score:
 * d = X - p, n = |d|, l = kappa (r - n) + 0 with kappa = f32(exp(double log_tau)) * s.
 * A site is active iff p >= 0 and all four values are finite (and kappa finite > 0). */
enum { Q_P, Q_C, Q_LOGTAU, Q_R, NPARAM1 };

typedef struct { int valid; float p, c, log_tau, r, kappa; } site1_t;

static site1_t site1_load(const float *sites, int64_t cap, int64_t i, float s)
{
    site1_t t;
    t.p = sites[Q_P * cap + i]; t.c = sites[Q_C * cap + i];
    t.log_tau = sites[Q_LOGTAU * cap + i]; t.r = sites[Q_R * cap + i];
    t.valid = t.p >= 0.0f && isfinite(t.p) && isfinite(t.c) && isfinite(t.log_tau) && isfinite(t.r);
    t.kappa = 0.0f;
    if (t.valid) {
        t.kappa = (float)exp((double)t.log_tau) * s;
        if (!(t.kappa > 0.0f) || !isfinite(t.kappa)) t.valid = 0;
    }
    return t;
}

static float score1_f32(const site1_t *t, float X)
{
    float n = fabsf(X - t->p);
    float l = t->kappa * (t->r - n);
    return l + 0.0f;
}

/* Exact top-K of every sample over the active sites (l descending, ID ascending).
 * out: [M][K].  Parity: pinned (sorted distance in the equal-tau, equal-r case). */
void ora1d_brute_topk(int M, int K, float s, const float *sites, int64_t cap, int64_t n,
                      uint32_t *out)
{
    site1_t *st = (site1_t *)malloc(sizeof(site1_t) * (size_t)(n > 0 ? n : 1));
    cand_t *c = (cand_t *)malloc(sizeof(cand_t) * (size_t)(n > 0 ? n : 1));
    for (int64_t i = 0; i < n; ++i) st[i] = site1_load(sites, cap, i, s);
    for (int64_t m = 0; m < M; ++m) {
        int nc = 0;
        for (int64_t i = 0; i < n; ++i)
            if (st[i].valid) { c[nc].l = score1_f32(&st[i], (float)m); c[nc].id = (uint32_t)i; ++nc; }
        select_topk(c, nc, K, out + m * K);
    }
    free(c); free(st);
}

/* Seed pass: each active site goes to sample rint(p) clamped to [0, M-1]; a sample keeps
 * the top K of its sites.  Parity: pinned (brute force per sample). */
void ora1d_seed(int M, int K, float s, const float *sites, int64_t cap, int64_t n,
                uint32_t *lists)
{
    for (int64_t q = 0; q < (int64_t)M * K; ++q) lists[q] = ORA_INVALID;
    site1_t *st = (site1_t *)malloc(sizeof(site1_t) * (size_t)(n > 0 ? n : 1));
    int64_t *where = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
    cand_t *c = (cand_t *)malloc(sizeof(cand_t) * (size_t)(n > 0 ? n : 1));
    for (int64_t i = 0; i < n; ++i) {
        st[i] = site1_load(sites, cap, i, s);
        where[i] = -1;
        if (!st[i].valid) continue;
        float f = rintf(st[i].p);
        where[i] = f > (float)(M - 1) ? M - 1 : (int64_t)f;
    }
    for (int64_t m = 0; m < M; ++m) {
        int nc = 0;
        for (int64_t i = 0; i < n; ++i)
            if (where[i] == m) { c[nc].l = score1_f32(&st[i], (float)m); c[nc].id = (uint32_t)i; ++nc; }
        if (nc) select_topk(c, nc, K, lists + m * K);
    }
    free(c); free(where); free(st);
}

/* One propagation pass on the line (Sec. 4.3 update equation in 1-D), Jacobi:
 * candidates = own list, the lists at m +- jump inside [0, M), and J injected IDs (draw
 * j: SplitMix64 output (t M + m) J + j, ID = hi32 n_slots / 2^32).  Parity: pinned
 * (converges to brute force when K >= active sites; monotone per entry; single-site
 * dilation by {0, +-s_t}). */
void ora1d_prop_pass(int M, int K, float s, const float *sites, int64_t cap, int64_t n,
                     const uint32_t *in, uint32_t *out, int jump, int J, uint64_t seed,
                     uint64_t t)
{
    site1_t *st = (site1_t *)malloc(sizeof(site1_t) * (size_t)(n > 0 ? n : 1));
    cand_t *c = (cand_t *)malloc(sizeof(cand_t) * (size_t)(3 * K + J + 1));
    for (int64_t i = 0; i < n; ++i) st[i] = site1_load(sites, cap, i, s);
    for (int64_t m = 0; m < M; ++m) {
        int64_t src[3]; int ns = 0;
        src[ns++] = m;
        if (m + jump < M) src[ns++] = m + jump;
        if (m - jump >= 0) src[ns++] = m - jump;
        int nc = 0;
        for (int a = 0; a < ns; ++a)
            for (int k = 0; k < K; ++k) {
                uint32_t id = in[src[a] * K + k];
                if (id == ORA_INVALID || (int64_t)id >= n || !st[id].valid) continue;
                c[nc].l = score1_f32(&st[id], (float)m); c[nc].id = id; ++nc;
            }
        for (int j = 0; j < J; ++j) {
            uint32_t id = n > 0 ? ora_inject_id(seed, t, M, m, J, j, (uint32_t)n) : ORA_INVALID;
            if (id == ORA_INVALID || (int64_t)id >= n || !st[id].valid) continue;
            c[nc].l = score1_f32(&st[id], (float)m); c[nc].id = id; ++nc;
        }
        select_topk(c, nc, K, out + m * K);
    }
    free(c); free(st);
}

/* Blend of every sample (softmax of the valid entries' scores, max subtracted; an empty
 * list gives 0), its loss L = (1/M) sum (c - I)^2 against target[M] (returned, if target
 * != NULL) and, if grad != NULL, the gradients for dL/dc = (2/M)(c - I), accumulated
 * into grad[4][cap] (+=):
 *   dc_k += w_k g;  gamma_k = w_k g (c_k - c);  dlog_tau_k += gamma_k l_k;
 *   dr_k += gamma_k kappa_k;  dp_k += gamma_k kappa_k sign(x - p_k)  (0 at x = p_k).
 * gabs (nullable, [4][cap]) accumulates |term|.  mode SCORE_F64 scores in double
 * (finite differences).  out: double[M] (nullable).  Parity: pinned (K = N full softmax,
 * hard limit, central finite differences, sum identities). */
double ora1d_render_loss_bwd(int M, int K, float s, const float *sites, int64_t cap, int64_t n,
                             const uint32_t *lists, const float *target, int mode, double *out,
                             double *grad, double *gabs)
{
    site1_t *st = (site1_t *)malloc(sizeof(site1_t) * (size_t)(n > 0 ? n : 1));
    for (int64_t i = 0; i < n; ++i) st[i] = site1_load(sites, cap, i, s);
    double L = 0;
    for (int64_t m = 0; m < M; ++m) {
        double X = (double)m;
        int idx[64], nv = 0;
        double l[64], e[64], S = 0, c = 0, mx = -INFINITY;
        for (int k = 0; k < K; ++k) {
            uint32_t id = lists[m * K + k];
            if (id == ORA_INVALID || (int64_t)id >= n || !st[id].valid) continue;
            const site1_t *t = &st[id];
            idx[nv] = (int)id;
            l[nv] = mode == SCORE_F64
                        ? exp((double)t->log_tau) * (double)s * ((double)t->r - fabs(X - (double)t->p))
                        : (double)score1_f32(t, (float)m);
            if (l[nv] > mx) mx = l[nv];
            ++nv;
        }
        for (int v = 0; v < nv; ++v) { e[v] = exp(l[v] - mx); S += e[v]; }
        for (int v = 0; v < nv; ++v) c += e[v] / S * (double)st[idx[v]].c;
        if (out) out[m] = c;
        if (!target) continue;
        double d = c - (double)target[m];
        L += d * d;
        if (!grad) continue;
        double g = 2.0 * d / (double)M;
        for (int v = 0; v < nv; ++v) {
            const site1_t *t = &st[idx[v]];
            int64_t id = idx[v];
            double w = e[v] / S;
            double gam = w * g * ((double)t->c - c);
            double kap = exp((double)t->log_tau) * (double)s;
            double dx = X - (double)t->p;
            double sg = dx > 0 ? 1.0 : (dx < 0 ? -1.0 : 0.0);
            double term[4] = {gam * kap * sg, w * g, gam * l[v], gam * kap};
            for (int q = 0; q < 4; ++q) {
                grad[q * cap + id] += term[q];
                if (gabs) gabs[q * cap + id] += fabs(term[q]);
            }
        }
    }
    free(st);
    return target ? L / (double)M : 0.0;
}

/* Adam on the four parameters (Kingma & Ba, bias-corrected, as ora_adam) followed by the
 * clamps p in [0, M-1], log_tau in [2, 20], r in [1, 512]; inactive slots untouched.
 * sites, m, v: double[4][cap] in place; grad: double[4][cap]; lr: double[4].  Parity:
 * pinned (torch.optim.Adam). */
void ora1d_adam(int M, double *sites, const double *grad, double *m, double *v, int64_t cap,
                int64_t n, const double *lr, double b1, double b2, double eps, int64_t t)
{
    for (int64_t i = 0; i < n; ++i) {
        int act = sites[Q_P * cap + i] >= 0.0;
        for (int q = 0; q < NPARAM1; ++q) act &= isfinite(sites[q * cap + i]) ? 1 : 0;
        if (!act) continue;
        for (int q = 0; q < NPARAM1; ++q) {
            int64_t o = q * cap + i;
            m[o] = b1 * m[o] + (1 - b1) * grad[o];
            v[o] = b2 * v[o] + (1 - b2) * grad[o] * grad[o];
            double mh = m[o] / (1 - pow(b1, (double)t)), vh = v[o] / (1 - pow(b2, (double)t));
            sites[o] -= lr[q] * mh / (sqrt(vh) + eps);
        }
        double *p = &sites[Q_P * cap + i], *lt = &sites[Q_LOGTAU * cap + i], *r = &sites[Q_R * cap + i];
        *p = *p < 0 ? 0 : (*p > M - 1 ? M - 1 : *p);
        *lt = *lt < 2 ? 2 : (*lt > 20 ? 20 : *lt);
        *r = *r < 1 ? 1 : (*r > 512 ? 512 : *r);
    }
}

/* Sec. 6.1: L = E_x ||c(x) - I(x)||^2 = (1/P) sum_x sum_ch (c - I)^2 with P = H W;
 * dL/dc(x) = (2/P)(c(x) - I(x)).  Returns L. */
double ora_loss_grad(int H, int W, const double *img, const float *target, double *grad)
{
    int64_t P = (int64_t)H * W;
    double L = 0;
    for (int64_t i = 0; i < 3 * P; ++i) {
        double d = img[i] - (double)target[i];
        L += d * d;
        if (grad) grad[i] = 2.0 * d / (double)P;
    }
    return L / (double)P;
}

/* Gradients of the loss w.r.t. every site parameter (App. B.4 lists position, log tau,
 * r, colour, anisotropy direction and a; the formulas are derived here):
 *   dL/dc_k        += w_k g
 *   gamma_k         = w_k g . (c_k - c)            (= dL/dl_k)
 *   dL/dlog_tau_k  += gamma_k l_k                   (dl/dlog_tau = l)
 *   dL/dr_k        += gamma_k tau_k s
 *   rho_k           = -gamma_k tau_k s / (2 n_k)   (= dL/dq_k), 0 if n_k = 0
 *   with alpha = u.d, beta = v.d, d = x - p, v = (-u_y, u_x):
 *   dL/dp          += -2 rho (e^a alpha u + e^-a beta v)
 *   dL/da          += rho (e^a alpha^2 - e^-a beta^2)
 *   dL/du_x        += 2 rho (e^a alpha d_x + e^-a beta d_y)
 *   dL/du_y        += 2 rho (e^a alpha d_y - e^-a beta d_x)
 * grad_img: double[3][H][W] = dL/dc(x).  grad: double[10][cap], accumulated (+=).
 * If target and rdelta are non-NULL, also accumulates the removal delta of Sec. 4.5
 * (see removal_delta below) divided by P into rdelta[cap].  If gabs is non-NULL it
 * accumulates the absolute values of the per-pixel terms of every sum ([10][cap]): the
 * scale against which the rounding of a float32 evaluation of that sum is measured.
 * Parity: pinned (central finite differences in SCORE_F64 mode; shift and colour sum
 * identities; removal delta against re-rendering without the site). */
static void acc2(double *grad, double *gabs, int64_t o, double v)
{
    grad[o] += v;
    if (gabs) gabs[o] += fabs(v);
}

/* Sec. 4.5 removal delta of every entry of one blended pixel: c' = the colour with
 * entry v removed and the remaining weights renormalised, Delta_v = ||c' - I||^2 -
 * ||c - I||^2.  c' is formed as the softmax of the other entries (their maximum
 * subtracted), which equals (c - w_v c_v) / (1 - w_v) but does not cancel when w_v -> 1.
 * With no other valid entry c' = 0 (an empty list renders 0). */
static void removal_delta_pixel(const pix_t *px, const site_t *st, const float *target,
                                int64_t P, int64_t p, double *out)
{
    double base = 0;
    for (int ch = 0; ch < 3; ++ch) {
        double d = px->c[ch] - (double)target[ch * P + p];
        base += d * d;
    }
    for (int v = 0; v < px->nv; ++v) {
        double cp[3] = {0, 0, 0};
        double m = -INFINITY;
        for (int u = 0; u < px->nv; ++u) if (u != v && px->l[u] > m) m = px->l[u];
        if (px->nv > 1) {
            double S = 0;
            for (int u = 0; u < px->nv; ++u) {
                if (u == v) continue;
                double e = exp(px->l[u] - m);
                S += e;
                for (int ch = 0; ch < 3; ++ch) cp[ch] += e * (double)st[px->idx[u]].c[ch];
            }
            for (int ch = 0; ch < 3; ++ch) cp[ch] /= S;
        }
        double rem = 0;
        for (int ch = 0; ch < 3; ++ch) {
            double d = cp[ch] - (double)target[ch * P + p];
            rem += d * d;
        }
        out[v] = rem - base;
    }
}

void ora_render_bwd(int H, int W, int K, float s, const float *sites, int64_t cap, int64_t n,
                    const uint32_t *lists, const double *grad_img, const float *target,
                    int mode, double *grad, double *rdelta, double *gabs)
{
    int64_t P = (int64_t)H * W;
    site_t *st = (site_t *)malloc(sizeof(site_t) * (size_t)(n > 0 ? n : 1));
    for (int64_t i = 0; i < n; ++i) st[i] = site_load(sites, cap, i, s);
    int nt = omp_get_max_threads();
    /* per-thread sums: thread 0 adds into the caller's buffers, the others into their
     * own, added in thread order at the end */
    double **tg = (double **)calloc((size_t)nt, sizeof(double *));
    double **ta = (double **)calloc((size_t)nt, sizeof(double *));
    double **tr = (double **)calloc((size_t)nt, sizeof(double *));
    for (int th = 1; th < nt; ++th) {
        tg[th] = (double *)calloc((size_t)(NPARAM * cap), sizeof(double));
        if (gabs) ta[th] = (double *)calloc((size_t)(NPARAM * cap), sizeof(double));
        if (rdelta) tr[th] = (double *)calloc((size_t)cap, sizeof(double));
    }
    tg[0] = grad; ta[0] = gabs; tr[0] = rdelta;
#pragma omp parallel num_threads(nt)
    {
    const int th = omp_get_thread_num();
    double *grad_t = tg[th], *gabs_t = ta[th], *rdelta_t = tr[th];
#pragma omp for schedule(static)
    for (int64_t p = 0; p < P; ++p) {
        pix_t px;
        double *grad = grad_t, *gabs = gabs_t, *rdelta = rdelta_t;
        double X = (double)(p % W), Y = (double)(p / W);
        blend_pixel(st, n, lists + p * K, K, X, Y, s, mode, &px);
        if (!px.nv) continue;
        double g[3];
        for (int ch = 0; ch < 3; ++ch) g[ch] = grad_img[ch * P + p];
        for (int v = 0; v < px.nv; ++v) {
            const site_t *t = &st[px.idx[v]];
            int64_t id = px.idx[v];
            double w = px.w[v];
            double gam = 0;
            for (int ch = 0; ch < 3; ++ch) {
                acc2(grad, gabs, (P_CR + ch) * cap + id, w * g[ch]);
                gam += w * g[ch] * ((double)t->c[ch] - px.c[ch]);
            }
            double kap = exp((double)t->log_tau) * (double)s;
            acc2(grad, gabs, P_LOGTAU * cap + id, gam * px.l[v]);
            acc2(grad, gabs, P_R * cap + id, gam * kap);
            double nn = px.n[v];
            if (nn > 0) {
                double rho = -gam * kap / (2.0 * nn);
                double ux = t->ux, uy = t->uy;
                double dx = X - (double)t->x, dy = Y - (double)t->y;
                double ep = exp((double)t->a), em = exp(-(double)t->a);
                double al = ux * dx + uy * dy, be = -uy * dx + ux * dy;
                acc2(grad, gabs, P_X * cap + id, -2.0 * rho * (ep * al * ux + em * be * (-uy)));
                acc2(grad, gabs, P_Y * cap + id, -2.0 * rho * (ep * al * uy + em * be * ux));
                acc2(grad, gabs, P_A * cap + id, rho * (ep * al * al - em * be * be));
                acc2(grad, gabs, P_UX * cap + id, 2.0 * rho * (ep * al * dx + em * be * dy));
                acc2(grad, gabs, P_UY * cap + id, 2.0 * rho * (ep * al * dy - em * be * dx));
            }
        }
        if (target && rdelta) {
            double dl[64];
            removal_delta_pixel(&px, st, target, P, p, dl);
            for (int v = 0; v < px.nv; ++v) rdelta[px.idx[v]] += dl[v] / (double)P;
        }
    }
    }
    for (int th = 1; th < nt; ++th) {
        for (int64_t o = 0; o < NPARAM * cap; ++o) grad[o] += tg[th][o];
        if (gabs) for (int64_t o = 0; o < NPARAM * cap; ++o) gabs[o] += ta[th][o];
        if (rdelta) for (int64_t o = 0; o < cap; ++o) rdelta[o] += tr[th][o];
        free(tg[th]); free(ta[th]); free(tr[th]);
    }
    free(tg); free(ta); free(tr);
    free(st);
}

/* Number of OpenMP threads of the loops above (1 = a single core); returns the number
 * in force before the call.  n <= 0 only queries it. */
int ora_set_threads(int n)
{
    int old = omp_get_max_threads();
    if (n > 0) omp_set_num_threads(n);
    return old;
}

/* ------------------------------------------------------------------------------ */
/* Adam with clamps (Sec. 5; Sec. 6.1 clamp ranges; Sec. 4.1 renormalisation of u)  */
/* ------------------------------------------------------------------------------ */

/* Textbook Adam (Kingma and Ba 2015), bias-corrected, per-parameter learning rates
 * lr[10]; step t counts from 1.  Afterwards: x in [0, W-1], y in [0, H-1],
 * log_tau in [2, 20], r in [1, 512], a in [-2, 2], colours in [0, 1], u renormalised
 * (u = (1, 0) if |u| = 0).  Inactive sites are left untouched.  State in double.
 * sites: double[10][cap] updated in place; m, v: double[10][cap]. */
void ora_adam(int H, int W, double *sites, const double *grad, double *m, double *v,
              int64_t cap, int64_t n, const double *lr, double b1, double b2, double eps,
              int64_t t)
{
    double c1 = 1.0 - pow(b1, (double)t), c2 = 1.0 - pow(b2, (double)t);
    for (int64_t i = 0; i < n; ++i) {
        if (!(sites[P_X * cap + i] >= 0.0)) continue;
        for (int p = 0; p < NPARAM; ++p) {
            int64_t o = (int64_t)p * cap + i;
            double g = grad[o];
            m[o] = b1 * m[o] + (1.0 - b1) * g;
            v[o] = b2 * v[o] + (1.0 - b2) * g * g;
            double mh = m[o] / c1, vh = v[o] / c2;
            sites[o] -= lr[p] * mh / (sqrt(vh) + eps);
        }
        double lo[NPARAM] = {0, 0, 2, 1, 0, 0, 0, -INFINITY, -INFINITY, -2};
        double hi[NPARAM] = {(double)(W - 1), (double)(H - 1), 20, 512, 1, 1, 1, INFINITY,
                             INFINITY, 2};
        for (int p = 0; p < NPARAM; ++p) {
            double *x = &sites[(int64_t)p * cap + i];
            if (*x < lo[p]) *x = lo[p];
            if (*x > hi[p]) *x = hi[p];
        }
        double ux = sites[P_UX * cap + i], uy = sites[P_UY * cap + i];
        double nu = sqrt(ux * ux + uy * uy);
        if (nu > 0) { sites[P_UX * cap + i] = ux / nu; sites[P_UY * cap + i] = uy / nu; }
        else { sites[P_UX * cap + i] = 1; sites[P_UY * cap + i] = 0; }
    }
}

/* ------------------------------------------------------------------------------ */
/* Gradient-weighted initialisation (Sec. 4.4)                                        */
/* ------------------------------------------------------------------------------ */

/* P_init(x) = (1 - lambda) |grad I(x)| / sum |grad I| + lambda / (H W), with
 * |grad I| the Frobenius norm over RGB of central differences (edge-clamped).  N
 * distinct pixels are drawn with probability proportional to P_init by the
 * Efraimidis-Spirakis method (2006): pixel p gets key log(u_p) / P_init(p), u_p in
 * (0,1) from SplitMix64 output number p of `seed`; the N largest keys win (ties to the
 * lower pixel index).  Sites are written in increasing pixel order at the pixel
 * centre, with the target colour there and the fixed defaults log_tau0, r0, u = (1,0),
 * a = 0.  Slots n..cap-1 are set inactive (x = y = -1).  Returns the number of sites
 * written.  keys_out (nullable) receives the H*W keys.  Parity: pinned (closed forms
 * for the gradient map, N = H W, lambda = 1, selection without replacement). */
static int key_cmp_desc(const void *pa, const void *pb)
{
    const double *a = (const double *)pa, *b = (const double *)pb;
    if (a[0] > b[0]) return -1;
    if (a[0] < b[0]) return 1;
    return a[1] < b[1] ? -1 : (a[1] > b[1] ? 1 : 0);
}

int64_t ora_init_sites(int H, int W, const float *target, int64_t N, double lambda,
                       uint64_t seed, float log_tau0, float r0, float *sites, int64_t cap,
                       double *keys_out)
{
    int64_t P = (int64_t)H * W;
    if (N > P) N = P;
    if (N > cap) N = cap;
    double *gm = (double *)malloc(sizeof(double) * (size_t)P);
    double G = 0;
    for (int64_t i = 0; i < H; ++i)
        for (int64_t j = 0; j < W; ++j) {
            int64_t jp = j + 1 < W ? j + 1 : W - 1, jm = j > 0 ? j - 1 : 0;
            int64_t ip = i + 1 < H ? i + 1 : H - 1, im = i > 0 ? i - 1 : 0;
            double acc = 0;
            for (int ch = 0; ch < 3; ++ch) {
                const float *I = target + ch * P;
                double gx = 0.5 * ((double)I[i * W + jp] - (double)I[i * W + jm]);
                double gy = 0.5 * ((double)I[ip * W + j] - (double)I[im * W + j]);
                acc += gx * gx + gy * gy;
            }
            gm[i * W + j] = sqrt(acc);
            G += gm[i * W + j];
        }
    double *kp = (double *)malloc(sizeof(double) * 2 * (size_t)P);
    for (int64_t p = 0; p < P; ++p) {
        double pr = lambda / (double)P + (G > 0 ? (1.0 - lambda) * gm[p] / G : 0.0);
        double u = ((double)(ora_splitmix64(seed, (uint64_t)p) >> 32) + 0.5) / 4294967296.0;
        double key = pr > 0 ? log(u) / pr : -INFINITY;
        kp[2 * p] = key; kp[2 * p + 1] = (double)p;
        if (keys_out) keys_out[p] = key;
    }
    qsort(kp, (size_t)P, 2 * sizeof(double), key_cmp_desc);
    /* mark winners, then write them in raster order */
    unsigned char *win = (unsigned char *)calloc((size_t)P, 1);
    for (int64_t q = 0; q < N; ++q) win[(int64_t)kp[2 * q + 1]] = 1;
    int64_t k = 0;
    for (int64_t p = 0; p < P; ++p) {
        if (!win[p]) continue;
        float vals[NPARAM] = {(float)(p % W), (float)(p / W), log_tau0, r0,
                              target[p], target[P + p], target[2 * P + p], 1.0f, 0.0f, 0.0f};
        for (int q = 0; q < NPARAM; ++q) sites[(int64_t)q * cap + k] = vals[q];
        ++k;
    }
    for (int64_t i = k; i < cap; ++i)
        for (int q = 0; q < NPARAM; ++q)
            sites[(int64_t)q * cap + i] = (q == P_X || q == P_Y) ? -1.0f : 0.0f;
    free(gm); free(kp); free(win);
    return k;
}

/* ------------------------------------------------------------------------------ */
/* Adaptive budget: statistics, densify, prune (Sec. 4.5; App. B.5)                  */
/* ------------------------------------------------------------------------------ */

enum { ST_M, ST_E, ST_SX, ST_SY, ST_SXX, ST_SXY, ST_SYY, ST_RD, NSTAT };

/* Statistics pass (App. B.5 "Densification scores"; Sec. 4.5 responsibilities).  For
 * every pixel x with a non-empty list, blended as in ora_render (weights w from the
 * float32 scores), with residual e(x) = ||c(x) - I(x)||^2, and every valid entry i:
 *   m_i  += w_i(x)                       soft mass
 *   E_i  += w_i(x) e(x)                  energy
 *   with omega = w_i(x) e(x) and d = x - p_i:
 *   S_x  += omega d_x      S_y  += omega d_y
 *   S_xx += omega d_x^2    S_xy += omega d_x d_y    S_yy += omega d_y^2
 *   R_i  += Delta_i(x) / P               removal delta, as in ora_render_bwd
 * The moments are weighted by the residual (the split uses a residual-weighted
 * centroid and covariance) and taken about the site centre p_i; the covariance does
 * not depend on that origin.  stats: double[8][cap] in the order (m, E, S_x, S_y,
 * S_xx, S_xy, S_yy, R), accumulated (+=).  sabs (nullable) accumulates the absolute
 * values of the terms; ssens (nullable) a sensitivity scale: each term's size per unit
 * of colour error (w sqrt(e) |f(d)| for the residual terms, w for the mass, (sqrt(e) +
 * 1) / P for the removal delta).  Both measure what the float32 evaluation of a sum
 * can be expected to get wrong.  Parity: pinned (mass is a partition of
 * unity, energy sums to the loss, one-site moments against a weighted covariance
 * from a library routine, removal delta against ora_render_bwd). */
static void acc3(double *stats, double *sabs, double *ssens, int64_t o, double v, double sens)
{
    stats[o] += v;
    if (sabs) sabs[o] += fabs(v);
    if (ssens) ssens[o] += sens;
}

void ora_site_stats(int H, int W, int K, float s, const float *sites, int64_t cap, int64_t n,
                    const uint32_t *lists, const float *target, double *stats, double *sabs,
                    double *ssens)
{
    int64_t P = (int64_t)H * W;
    site_t *st = (site_t *)malloc(sizeof(site_t) * (size_t)(n > 0 ? n : 1));
    for (int64_t i = 0; i < n; ++i) st[i] = site_load(sites, cap, i, s);
    pix_t px;
    double dl[64];
    for (int64_t p = 0; p < P; ++p) {
        double X = (double)(p % W), Y = (double)(p / W);
        blend_pixel(st, n, lists + p * K, K, X, Y, s, SCORE_F32, &px);
        if (!px.nv) continue;
        double e = 0;
        for (int ch = 0; ch < 3; ++ch) {
            double d = px.c[ch] - (double)target[ch * P + p];
            e += d * d;
        }
        removal_delta_pixel(&px, st, target, P, p, dl);
        /* sensitivity scale of the residual terms: |d e / d c| |dc| ~ 2 sqrt(e) |dc| */
        double se = sqrt(e);
        for (int v = 0; v < px.nv; ++v) {
            int64_t id = px.idx[v];
            double w = px.w[v], om = w * e, ws = w * se;
            double dx = X - (double)st[id].x, dy = Y - (double)st[id].y;
            double ax = fabs(dx), ay = fabs(dy);
            acc3(stats, sabs, ssens, ST_M * cap + id, w, w);
            acc3(stats, sabs, ssens, ST_E * cap + id, om, ws);
            acc3(stats, sabs, ssens, ST_SX * cap + id, om * dx, ws * ax);
            acc3(stats, sabs, ssens, ST_SY * cap + id, om * dy, ws * ay);
            acc3(stats, sabs, ssens, ST_SXX * cap + id, om * dx * dx, ws * ax * ax);
            acc3(stats, sabs, ssens, ST_SXY * cap + id, om * dx * dy, ws * ax * ay);
            acc3(stats, sabs, ssens, ST_SYY * cap + id, om * dy * dy, ws * ay * ay);
            acc3(stats, sabs, ssens, ST_RD * cap + id, dl[v] / (double)P, (se + 1.0) / (double)P);
        }
    }
    free(st);
}

/* Principal axis of the symmetric 2x2 matrix [[a, b], [b, c]]: eigenvalues
 * l1 >= l2 and the unit eigenvector of l1, signed so that its first non-zero
 * component is positive.  Returns 0 (no axis) unless the trace exceeds 1e-9 and the
 * eigenvalue gap 2 disc exceeds 2e-6 of the trace. */
static int principal_axis(double a, double b, double c, double *ex, double *ey, double *l1,
                          double *l2)
{
    double h = 0.5 * (a - c), tr = a + c;
    double disc = sqrt(h * h + b * b);
    if (!(tr > 1e-9) || !(disc > 1e-6 * tr)) return 0;
    *l1 = 0.5 * tr + disc;
    *l2 = 0.5 * tr - disc;
    double vx, vy;
    if (a >= c) { vx = *l1 - c; vy = b; }
    else        { vx = b; vy = *l1 - a; }
    double nv = sqrt(vx * vx + vy * vy);
    vx /= nv; vy /= nv;
    if (vx < 0 || (vx == 0 && vy < 0)) { vx = -vx; vy = -vy; }
    *ex = vx; *ey = vy;
    return 1;
}

static double clampd(double v, double lo, double hi) { return v < lo ? lo : (v > hi ? hi : v); }

static int64_t nearest_pixel(int H, int W, double x, double y)
{
    double fi = rint(y), fj = rint(x);
    int64_t i = fi > 0 ? (fi > H - 1 ? H - 1 : (int64_t)fi) : 0;
    int64_t j = fj > 0 ? (fj > W - 1 ? W - 1 : (int64_t)fj) : 0;
    return i * W + j;
}

/* Split of one site (Sec. 4.5, App. B.5 "Split kernel").  par: the parent's ten
 * parameters; stat: its (m, E, S_x, S_y, S_xx, S_xy, S_yy).  Writes the two children.
 *   offset delta = 0.5 sqrt(m) pixels, clamped to [1.5, 48]
 *   with statistics (E > 1e-12 and a principal axis of the residual-weighted
 *   covariance C = S../E - mu mu^T, mu = (S_x, S_y) / E): children at p + mu +- delta e1,
 *   u = e1 and a = 0.5 ln(l2 / l1) clamped to [-2, 2] (the det-1 metric whose level
 *   sets have the covariance's aspect ratio and long axis along e1; a = -2 if l2 <= 0)
 *   without: e1 = principal axis of the Sobel structure tensor of the target at the
 *   site's pixel (summed over channels, edges clamped), else u; children at
 *   p +- delta e1, u unchanged, a = 0.8 a
 *   both: positions clamped to the image, log_tau - 0.25 in [2, 20], 0.85 r in
 *   [1, 512], colour = target at the child's nearest pixel.
 * Child "+" keeps the parent's slot, child "-" takes a free slot. */
static void split_site(int H, int W, const float *target, const float *par,
                       const float *stat, float *ca, float *cb)
{
    int64_t P = (int64_t)H * W;
    double m = stat[ST_M], E = stat[ST_E];
    double delta = clampd(0.5 * sqrt(m), 1.5, 48.0);
    double px = par[P_X], py = par[P_Y];
    double cx = px, cy = py, ex = 0, ey = 0, l1, l2;
    double ux = par[P_UX], uy = par[P_UY], a = par[P_A];
    int have = 0;
    if (E > 1e-12) {
        double mx = (double)stat[ST_SX] / E, my = (double)stat[ST_SY] / E;
        double cxx = (double)stat[ST_SXX] / E - mx * mx;
        double cxy = (double)stat[ST_SXY] / E - mx * my;
        double cyy = (double)stat[ST_SYY] / E - my * my;
        if (principal_axis(cxx, cxy, cyy, &ex, &ey, &l1, &l2)) {
            have = 1;
            cx = px + mx;
            cy = py + my;
            ux = ex;
            uy = ey;
            a = l2 > 0 ? clampd(0.5 * log(l2 / l1), -2.0, 2.0) : -2.0;
        }
    }
    if (!have) {
        int64_t q = nearest_pixel(H, W, px, py);
        int64_t i = q / W, j = q % W;
        int64_t im = i > 0 ? i - 1 : 0, ip = i + 1 < H ? i + 1 : H - 1;
        int64_t jm = j > 0 ? j - 1 : 0, jp = j + 1 < W ? j + 1 : W - 1;
        double txx = 0, txy = 0, tyy = 0;
        for (int ch = 0; ch < 3; ++ch) {
            const float *I = target + ch * P;
#define T_(r, c) ((double)I[(r) * W + (c)])
            double gx = (T_(im, jp) + 2.0 * T_(i, jp) + T_(ip, jp)) -
                        (T_(im, jm) + 2.0 * T_(i, jm) + T_(ip, jm));
            double gy = (T_(ip, jm) + 2.0 * T_(ip, j) + T_(ip, jp)) -
                        (T_(im, jm) + 2.0 * T_(im, j) + T_(im, jp));
#undef T_
            txx += gx * gx;
            txy += gx * gy;
            tyy += gy * gy;
        }
        if (!principal_axis(txx, txy, tyy, &ex, &ey, &l1, &l2)) {
            double nu = sqrt(ux * ux + uy * uy);
            if (nu > 0) { ex = ux / nu; ey = uy / nu; }
            else        { ex = 1.0; ey = 0.0; }
        }
        a = 0.8 * a;
    }
    float *kids[2] = {ca, cb};
    for (int c = 0; c < 2; ++c) {
        float *o = kids[c];
        double sg = c == 0 ? 1.0 : -1.0;
        for (int q = 0; q < NPARAM; ++q) o[q] = par[q];
        o[P_X] = (float)clampd(cx + sg * delta * ex, 0.0, (double)(W - 1));
        o[P_Y] = (float)clampd(cy + sg * delta * ey, 0.0, (double)(H - 1));
        o[P_LOGTAU] = (float)clampd((double)par[P_LOGTAU] - 0.25, 2.0, 20.0);
        o[P_R] = (float)clampd(0.85 * (double)par[P_R], 1.0, 512.0);
        int64_t q = nearest_pixel(H, W, (double)o[P_X], (double)o[P_Y]);
        for (int ch = 0; ch < 3; ++ch) o[P_CR + ch] = target[ch * P + q];
        o[P_UX] = (float)ux;
        o[P_UY] = (float)uy;
        o[P_A] = (float)a;
    }
}

typedef struct { float key; int64_t id; } rank_t;

static int rank_cmp_desc(const void *pa, const void *pb)
{
    const rank_t *a = (const rank_t *)pa, *b = (const rank_t *)pb;
    if (a->key > b->key) return -1;
    if (a->key < b->key) return 1;
    return a->id < b->id ? -1 : (a->id > b->id ? 1 : 0);
}

static int rank_cmp_asc(const void *pa, const void *pb)
{
    const rank_t *a = (const rank_t *)pa, *b = (const rank_t *)pb;
    if (a->key < b->key) return -1;
    if (a->key > b->key) return 1;
    return a->id < b->id ? -1 : (a->id > b->id ? 1 : 0);
}

static int site_active(const float *sites, int64_t cap, int64_t i)
{
    for (int q = 0; q < NPARAM; ++q)
        if (!isfinite(sites[(int64_t)q * cap + i])) return 0;
    return sites[i] >= 0.0f;
}

/* One budget step (Sec. 4.5 "Adaptive Budget"; App. B.5), on slots 0..cap-1.
 *   n_active = number of active slots.
 *   prune (flags & 1): the floor(p_prune n_active) active sites with the smallest
 *     removal delta R (float32, ties to the lower ID) become inactive (x = y = -1).
 *   split (flags & 2): candidates are the active, unpruned sites with m > min_mass;
 *     score s = E / max(m, eps)^alpha (double, rounded to float32; ties to the lower
 *     ID); the min(floor(p_split n_active), candidates, free slots) best are split
 *     (split_site).  Parents in ascending ID order take the free slots (inactive after
 *     the prune) in ascending order for their second child.  Adam moments m, v of
 *     both children's slots are zeroed (all ten parameters).
 *   seed (flags & 4, lists non-NULL): the new child with the smallest ID at each pixel
 *     replaces entry K-1 of that pixel's list, so that propagation starts from it.
 * stats: float[8][cap] (ora_site_stats order; m, E, moments and R are read).
 * counts[6] = {n_active, n_pruned, n_split, n_active after, high water (1 + largest
 * active slot, 0 if none), split candidates}.  Parity: pinned (selections against a
 * sort, closed-form split geometry, fallback axis of a ramp, clamps, slot order). */
void ora_densify_prune(int H, int W, int K, const float *target, float *sites, int64_t cap,
                       float *adam_m, float *adam_v, const float *stats, double p_prune,
                       double p_split, double alpha, double eps, double min_mass, int flags,
                       uint32_t *lists, int64_t *counts)
{
    int64_t P = (int64_t)H * W;
    unsigned char *act = (unsigned char *)malloc((size_t)cap + 1);
    rank_t *rk = (rank_t *)malloc(sizeof(rank_t) * (size_t)(cap + 1));
    int64_t n_act = 0;
    for (int64_t i = 0; i < cap; ++i) { act[i] = (unsigned char)site_active(sites, cap, i); n_act += act[i]; }
    /* prune */
    int64_t n_p = (flags & 1) ? (int64_t)floor(p_prune * (double)n_act) : 0;
    int64_t nr = 0;
    for (int64_t i = 0; i < cap; ++i)
        if (act[i]) { rk[nr].key = stats[ST_RD * cap + i]; rk[nr].id = i; ++nr; }
    qsort(rk, (size_t)nr, sizeof(rank_t), rank_cmp_asc);
    if (n_p > nr) n_p = nr;
    for (int64_t q = 0; q < n_p; ++q) {
        int64_t i = rk[q].id;
        act[i] = 2; /* pruned in this call */
        sites[P_X * cap + i] = -1.0f;
        sites[P_Y * cap + i] = -1.0f;
    }
    /* split */
    int64_t n_cand = 0;
    for (int64_t i = 0; i < cap; ++i) {
        if (act[i] != 1) continue;
        double m = stats[ST_M * cap + i];
        if (!(m > min_mass)) continue;
        double sc = (double)stats[ST_E * cap + i] / pow(m > eps ? m : eps, alpha);
        rk[n_cand].key = (float)sc;
        rk[n_cand].id = i;
        ++n_cand;
    }
    int64_t n_free = cap - (n_act - n_p);
    int64_t n_s = 0;
    if (flags & 2) {
        n_s = (int64_t)floor(p_split * (double)n_act);
        if (n_s > n_cand) n_s = n_cand;
        if (n_s > n_free) n_s = n_free;
    }
    qsort(rk, (size_t)n_cand, sizeof(rank_t), rank_cmp_desc);
    unsigned char *par = (unsigned char *)calloc((size_t)cap + 1, 1);
    for (int64_t q = 0; q < n_s; ++q) par[rk[q].id] = 1;
    int64_t *child = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n_s + 1));
    int64_t j = 0;
    for (int64_t i = 0; i < cap && j < n_s; ++i)
        if (act[i] != 1) child[j++] = i;
    float pa[NPARAM], ca[NPARAM], cb[NPARAM], stv[NSTAT];
    uint32_t *seed = NULL;
    if ((flags & 4) && lists) {
        seed = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)P);
        for (int64_t p = 0; p < P; ++p) seed[p] = ORA_INVALID;
    }
    j = 0;
    for (int64_t i = 0; i < cap; ++i) {
        if (!par[i]) continue;
        int64_t c = child[j++];
        for (int q = 0; q < NPARAM; ++q) pa[q] = sites[(int64_t)q * cap + i];
        for (int q = 0; q < NSTAT; ++q) stv[q] = stats[(int64_t)q * cap + i];
        split_site(H, W, target, pa, stv, ca, cb);
        for (int q = 0; q < NPARAM; ++q) {
            sites[(int64_t)q * cap + i] = ca[q];
            sites[(int64_t)q * cap + c] = cb[q];
            if (adam_m) { adam_m[(int64_t)q * cap + i] = 0.0f; adam_m[(int64_t)q * cap + c] = 0.0f; }
            if (adam_v) { adam_v[(int64_t)q * cap + i] = 0.0f; adam_v[(int64_t)q * cap + c] = 0.0f; }
        }
        if (seed) {
            int64_t q = nearest_pixel(H, W, (double)cb[P_X], (double)cb[P_Y]);
            if ((uint32_t)c < seed[q]) seed[q] = (uint32_t)c;
        }
    }
    if (seed) {
        for (int64_t p = 0; p < P; ++p)
            if (seed[p] != ORA_INVALID) lists[p * K + (K - 1)] = seed[p];
        free(seed);
    }
    int64_t hw = 0;
    for (int64_t i = 0; i < cap; ++i) if (site_active(sites, cap, i)) hw = i + 1;
    counts[0] = n_act;
    counts[1] = n_p;
    counts[2] = n_s;
    counts[3] = n_act - n_p + n_s;
    counts[4] = hw;
    counts[5] = n_cand;
    free(act); free(rk); free(par); free(child);
}
