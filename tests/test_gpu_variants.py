"""GPU parity of the paper's variants against the CPU oracle: tau diffusion (App. B.6)
and the one-dimensional SAD (Sec. 7 "1D Signal Fitting": seed pass, propagation, blend,
loss, gradients, Adam).

Lists bit-exact; values within 1e-5 max-abs; gradients per parameter row
|d| <= 1e-4 (|g| + 1e-3 max|g|) + 1e-5 sum|terms| (the float32 sum of the per-sample
terms, as the 2-D rule); the smoothed gradient and Adam against the float64 oracle within
a few float32 roundings."""
import numpy as np
import pytest
import torch

import oracle as O
import synth
from _helpers import rows_to_planar, planar_to_rows

pytestmark = pytest.mark.gpu
DEV = "cuda"


@pytest.fixture(scope="module")
def S():
    import paper_2604_21984_amd._lib as S
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return S


def _t(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


# ---- tau diffusion ----------------------------------------------------------------------

@pytest.mark.parametrize("lam", [0.0, 0.3, 1.0])
@pytest.mark.parametrize("site_major", [False, True])
def test_tau_diffusion_matches_oracle(S, lam, site_major):
    H, W, K, N = 60, 90, 8, 700
    sites = synth.random_sites(3, H, W, N, cap=N + 5, anisotropic=True, log_tau_range=(2, 5),
                               r_range=(1, 3))
    sites[0:2, [4, 50]] = -1.0
    s = O.default_scale(H, W)
    lists = O.refresh(H, W, H, W, K, s, sites, N, True, 10, 4, 1)
    cap = sites.shape[1]
    img = S.image(H, W, K, N, cap)
    rec = torch.empty(N * 16, dtype=torch.float32, device=DEV)
    S.prepare_sites(img, _t(sites), rec)
    topk = _t(rows_to_planar(lists, H, W, K))
    g = np.random.default_rng(4).normal(0, 1e-3, N).astype(np.float32)
    if site_major:   # the training step's [cap][10] accumulator: log tau at 10 i + 2
        gin = torch.zeros((cap, 10), dtype=torch.float32, device=DEV)
        gin[:N, 2] = _t(g)
        gout = torch.full_like(gin, 7.0)
        S.tau_diffusion(img, rec, topk, gin.view(-1)[2:], 10, lam, gout.view(-1)[2:], 10)
        got = gout[:N, 2]
        untouched = torch.cat([gout[:, :2].reshape(-1), gout[:, 3:].reshape(-1)])
    else:            # a [10][cap] gradient: the log tau row
        gin = torch.zeros((10, cap), dtype=torch.float32, device=DEV)
        gin[2, :N] = _t(g)
        gout = torch.full_like(gin, 7.0)
        S.tau_diffusion(img, rec, topk, gin[2], 1, lam, gout[2], 1)
        got = gout[2, :N]
        untouched = torch.cat([gout[:2].reshape(-1), gout[3:].reshape(-1)])
    torch.cuda.synchronize()
    ref = O.tau_diffusion(H, W, K, s, sites, N, lists, g.astype(np.float64), lam)
    got = got.cpu().numpy().astype(np.float64)
    if lam == 0.0:
        assert np.array_equal(got, g.astype(np.float64))
    err = np.abs(got - ref)
    assert np.all(err <= 4e-7 * (np.abs(g) + np.abs(g).max())), float(err.max())
    assert bool((untouched == 7.0).all())
    with pytest.raises(S.SadError):
        S.tau_diffusion(img, rec, topk, gin.view(-1), 1, lam, gin.view(-1), 1)


# ---- one-dimensional SAD ----------------------------------------------------------------

class Sig:
    def __init__(self, S, M, K, sites, n):
        self.S, self.M, self.K, self.n = S, M, K, n
        self.sg = S.signal(M, K, n, sites.shape[1])
        self.sites = _t(sites)
        self.rec = torch.empty(max(n, 1) * 4, dtype=torch.float32, device=DEV)
        S.prepare1d(self.sg, self.sites, self.rec)

    def field(self):
        return torch.empty((self.K // 4, self.M, 4), dtype=torch.int32, device=DEV)


def _rows1(f, M, K):
    return planar_to_rows(f.cpu().numpy(), 1, M, K)


@pytest.mark.parametrize("M,n,K,J", [(300, 40, 4, 2), (5000, 600, 8, 4), (777, 900, 16, 3),
                                     (64, 3, 8, 1), (1 << 20, 1 << 16, 8, 4)])
def test_1d_seed_and_propagation_lockstep_bit_exact(S, M, n, K, J):
    sites = synth.sites1d(5 + K, M, n, cap=n + 3)
    sites[0, 1] = -1.0
    sites[3, 2] = np.inf
    s = O.scale1d(M)
    g = Sig(S, M, K, sites, n)
    f, f2 = g.field(), g.field()
    scratch = torch.empty(M, dtype=torch.int64, device=DEV)
    S.seed1d(g.sg, g.rec, f, scratch)
    torch.cuda.synchronize()
    cur = O.seed1d(M, K, s, sites, n)
    assert np.array_equal(_rows1(f, M, K), cur)
    for t in range(12):
        jmp = O.jump(t, 1, M)
        fin = _t(rows_to_planar(cur, 1, M, K))
        S.propagate1d(g.sg, g.rec, fin, f2, jmp, J, 99, t)
        torch.cuda.synchronize()
        ref = O.prop_pass1d(M, K, s, sites, n, cur, jmp, J, 99, t)
        assert np.array_equal(_rows1(f2, M, K), ref), f"pass {t}"
        cur = ref
    if n <= K:
        assert np.array_equal(cur, O.brute_topk1d(M, K, s, sites, n))


@pytest.mark.parametrize("M,n,K", [(400, 50, 4), (6000, 700, 8), (999, 300, 16),
                                   (777, 900, 16), (1 << 20, 1 << 16, 8)])
def test_1d_render_loss_gradients(S, M, n, K):
    """Colours, loss and gradients against the oracle; (777, 900, 16) holds more sites
    per block than the block table's 256 slots (terms overflow to global atomics), and
    (2^20, 2^16, 8) is the size the benchmark times."""
    sites = synth.sites1d(11 + K, M, n)
    sites[0, 3] = -1.0
    s = O.scale1d(M)
    target = synth.signal1d(12, M)
    lists = O.seed1d(M, K, s, sites, n)
    for t in range(14):
        lists = O.prop_pass1d(M, K, s, sites, n, lists, O.jump(t, 1, M), 3, 5, t)
    g = Sig(S, M, K, sites, n)
    topk = _t(rows_to_planar(lists, 1, M, K))
    out = torch.empty(M, dtype=torch.float32, device=DEV)
    grad = torch.zeros((4, n), dtype=torch.float32, device=DEV)
    loss = S.loss_acc(DEV)
    S.render1d(g.sg, g.rec, topk, _t(target), out, grad, loss)
    torch.cuda.synchronize()
    col, L, gref, gabs = O.render1d(M, K, s, sites, n, lists, target=target, grad=True,
                                    abs_sum=True)
    assert float(np.abs(out.cpu().numpy() - col).max()) <= 1e-5
    assert abs(float(loss[0]) - L) <= 1e-5 * L
    gg = grad.cpu().numpy().astype(np.float64)
    for q in range(4):
        tol = 1e-4 * (np.abs(gref[q]) + 1e-3 * np.abs(gref[q]).max()) + 1e-5 * gabs[q]
        err = np.abs(gg[q] - gref[q])
        assert np.all(err <= tol), (q, float((err / tol).max()))


def test_1d_adam_matches_oracle(S):
    M, n, cap = 500, 40, 43
    sites = synth.sites1d(21, M, n, cap=cap)
    sites[0, 0], sites[2, 1], sites[3, 2] = 0.01, 19.995, 1.001
    g = Sig(S, M, 8, sites, n)
    lr = [0.1, 0.01, 0.05, 0.1]
    m = torch.zeros((4, cap), dtype=torch.float32, device=DEV)
    v = torch.zeros_like(m)
    sd = np.array(sites, dtype=np.float64)
    md, vd = np.zeros_like(sd), np.zeros_like(sd)
    rng = np.random.default_rng(22)
    for t in range(1, 6):
        gr = rng.normal(0, 1, (4, cap)).astype(np.float32)
        gr[0, 0], gr[2, 1], gr[3, 2] = 1.0, -1.0, 1.0
        S.adam1d(g.sg, g.sites, _t(gr), m, v, lr, t)
        O.adam1d(M, sd, gr.astype(np.float64), md, vd, n, np.array(lr), 0.9, 0.999, 1e-8, t)
    torch.cuda.synchronize()
    got = g.sites.cpu().numpy().astype(np.float64)
    # float32 arithmetic against float64: a few roundings of each parameter and step
    tol = 4e-7 * np.abs(sd) + 1e-6 * np.array(lr)[:, None]
    assert np.all(np.abs(got[:, :n] - sd[:, :n]) <= tol[:, :n])
    assert got[0, 0] == 0 and got[2, 1] == 20 and got[3, 2] == 1
    assert np.all(got[:, n:] == sites[:, n:])


def test_1d_fit_reduces_loss(S):
    """A whole 1-D encode on the GPU: 300 iterations of pass + render/gradient + Adam."""
    M, n, K, J = 20000, 800, 8, 4
    target = _t(synth.signal1d(31, M))
    sites = synth.sites1d(32, M, n, log_tau_range=(4.0, 4.0), r_range=(1.0, 1.0))
    g = Sig(S, M, K, sites, n)
    a, b = g.field(), g.field()
    S.seed1d(g.sg, g.rec, a, torch.empty(M, dtype=torch.int64, device=DEV))
    grad = torch.zeros((4, n), dtype=torch.float32, device=DEV)
    m, v = torch.zeros_like(grad), torch.zeros_like(grad)
    losses = []
    for t in range(300):
        S.propagate1d(g.sg, g.rec, a, b, O.jump(t, 1, M), J, 7, t)
        a, b = b, a
        loss = S.loss_acc(DEV)
        grad.zero_()
        S.render1d(g.sg, g.rec, a, target, None, grad, loss)
        S.adam1d(g.sg, g.sites, grad, m, v, [1.0, 0.01, 0.01, 0.1], t + 1)
        S.prepare1d(g.sg, g.sites, g.rec)
        if t in (0, 299):
            losses.append(float(loss[0]))
    assert losses[1] < 0.5 * losses[0], losses
