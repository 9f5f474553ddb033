"""Quality of the propagated top-K field against the exact top-K (Sec. 6.5).

A list field is built from the seed pass (or the JFA prepass) and n propagation passes
(the jump schedule of Sec. 4.3, J injections per pass), and compared at sampled pixels
with the exact top-K from ``sad_exact_topk``: "exact match" is the fraction of pixels
whose K-set equals the exact one, "recall" the mean fraction of the exact K found.
"""
import numpy as np
import torch

from . import _lib as S


def set_agreement(approx, exact):
    """(exact-match fraction, recall) of two [n, K] uint32 arrays of lists."""
    inv = 0xFFFFFFFF
    match, rec_sum = 0, 0.0
    for a, e in zip(approx, exact):
        ea = set(int(x) for x in e if x != inv)
        aa = set(int(x) for x in a if x != inv)
        match += ea == aa
        rec_sum += len(ea & aa) / len(ea) if ea else 1.0
    n = max(len(exact), 1)
    return match / n, rec_sum / n


def _rows(lists, pix, H, W, K):
    """Rows of the planar field [K/4, H*W, 4] at the pixels pix -> [n, K] uint32."""
    a = lists.view(K // 4, H * W, 4)[:, pix].permute(1, 0, 2).reshape(len(pix), K)
    return a.cpu().numpy().view(np.uint32)


def convergence(sites, H, W, K=8, J=4, passes=(8, 12, 16), n_pix=256, seed=0, device="cuda",
                jfa=False):
    """Exact match and recall after each number of passes in `passes` for one site set
    (float32 [10, N] host array).  The field starts from the seed pass, or with jfa=True
    from the JFA prepass of a full refresh (App. B.3: seed pass keeping four entries,
    then the flood passes)."""
    N = sites.shape[1]
    img = S.image(H, W, K, N, N)
    sd = torch.from_numpy(np.ascontiguousarray(sites)).to(device)
    rec = torch.empty(N * S.REC_FLOATS, dtype=torch.float32, device=device)
    S.prepare_sites(img, sd, rec)
    a = torch.empty((K // 4, H, W, 4), dtype=torch.int32, device=device)
    b = torch.empty_like(a)
    if jfa:
        scratch = torch.empty(H * W, dtype=torch.int64, device=device)
        S.refresh(img, H, W, rec, a, b, scratch, 0, J, seed ^ 0x5EED, jfa=True)
    else:
        S.seed_topk(img, rec, a, b)
    pix = np.sort(np.random.default_rng(seed).choice(H * W, n_pix, replace=False))
    pix_d = torch.from_numpy(pix.astype(np.int64)).to(device)
    exact = torch.empty((n_pix, K), dtype=torch.int32, device=device)
    S.exact_topk(img, rec, pix_d, exact)
    ex = exact.cpu().numpy().view(np.uint32)
    out = {}
    for t in range(max(passes)):
        S.propagate_topk(img, rec, a, b, S.jump_step(t, H, W), J, seed ^ 0x5EED, t)
        a, b = b, a
        if t + 1 in passes:
            out[t + 1] = set_agreement(_rows(a, pix, H, W, K), ex)
    return out
