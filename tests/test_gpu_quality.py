"""GPU: brute-force exact top-K against the oracle (bit-exact), and the convergence
measurement of the propagated field (Sec. 6.5) on a small domain."""
import numpy as np
import pytest
import torch

import oracle as O
import synth

pytestmark = pytest.mark.gpu
DEV = "cuda"


@pytest.fixture(scope="module")
def S():
    from paper_2604_21984_amd import _lib
    return _lib


@pytest.mark.parametrize("H,W,N,K", [(40, 56, 300, 4), (64, 48, 700, 8), (33, 70, 129, 16),
                                     (20, 20, 45, 32), (16, 24, 5, 8)])
def test_exact_topk_bit_exact(S, H, W, N, K):
    sites = synth.random_sites(N + K, H, W, N, anisotropic=True, log_tau_range=(2.0, 5.0),
                               r_range=(1.0, 20.0))
    sites[:, N - 1] = sites[:, 1]        # a duplicate: equal scores, ID order decides
    sites[0, N // 2] = -1.0              # an inactive site
    sites[1, N // 2] = -1.0
    s = O.default_scale(H, W)
    rng = np.random.default_rng(N)
    pix = np.concatenate([rng.choice(H * W, 150, replace=True), [0, H * W - 1, -3, H * W]])
    ref = O.brute_topk(H, W, K, s, sites, N, pix=np.clip(pix, 0, H * W - 1))
    ref[pix < 0] = O.INVALID
    ref[pix >= H * W] = O.INVALID
    img = S.image(H, W, K, N, N)
    rec = torch.empty(N * S.REC_FLOATS, dtype=torch.float32, device=DEV)
    S.prepare_sites(img, torch.from_numpy(sites).to(DEV), rec)
    out = torch.empty((len(pix), K), dtype=torch.int32, device=DEV)
    S.exact_topk(img, rec, torch.from_numpy(pix.astype(np.int64)).to(DEV), out)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(out.cpu().numpy().view(np.uint32), ref)


def test_convergence_measurement_against_oracle(S):
    from paper_2604_21984_amd import quality as Q
    H, W, N, K = 128, 160, 1200, 8
    sites = synth.cell_sites(2, H, W, N)
    res = Q.convergence(sites, H, W, K=K, passes=(4, 8, 12), n_pix=256, seed=5)
    # the same pixels against the oracle's brute force
    pix = np.sort(np.random.default_rng(5).choice(H * W, 256, replace=False))
    ref = O.brute_topk(H, W, K, O.default_scale(H, W), sites, N, pix=pix)
    img = S.image(H, W, K, N, N)
    rec = torch.empty(N * S.REC_FLOATS, dtype=torch.float32, device=DEV)
    S.prepare_sites(img, torch.from_numpy(sites).to(DEV), rec)
    out = torch.empty((256, K), dtype=torch.int32, device=DEV)
    S.exact_topk(img, rec, torch.from_numpy(pix.astype(np.int64)).to(DEV), out)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(out.cpu().numpy().view(np.uint32), ref)
    assert set(res) == {4, 8, 12}
    em = [res[t][0] for t in (4, 8, 12)]
    rc = [res[t][1] for t in (4, 8, 12)]
    assert rc[2] >= 0.95 and em[2] >= 0.7, res
    assert rc[0] <= rc[2] + 1e-12
