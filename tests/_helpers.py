"""Test helpers: layout conversion between the GPU list field and the oracle's
pixel-major lists, and the tolerance rules of the parity tests."""
import numpy as np

INVALID = 0xFFFFFFFF


def planar_to_rows(topk, H, W, K):
    """[K/4, H, W, 4] int32 (GPU) -> [H*W, K] uint32 (oracle)."""
    a = np.asarray(topk).astype(np.int64) & 0xFFFFFFFF
    a = a.reshape(K // 4, H * W, 4).transpose(1, 0, 2).reshape(H * W, K)
    return a.astype(np.uint32)


def rows_to_planar(rows, H, W, K):
    """[H*W, K] uint32 -> [K/4, H, W, 4] int32."""
    a = np.asarray(rows, dtype=np.uint32).reshape(H * W, K // 4, 4).transpose(1, 0, 2)
    return np.ascontiguousarray(a.reshape(K // 4, H, W, 4)).view(np.int32)


# parameter groups of the gradient tolerance: position, log tau, r, colour, u, a
GROUPS = [(0, 2), (2, 3), (3, 4), (4, 7), (7, 9), (9, 10)]


# A float32 sum of n terms, in any order, is off by at most (n - 1) 2^-24 sum|terms|;
# with the rounding of each term's own evaluation this stays below 1e-5 sum|terms| for
# the tile sizes used here.
COND = 1e-5


def grad_report(got, ref, absum=None, rel=1e-4, floor=1e-3):
    """Per group: |got - ref| <= rel (|ref| + floor max_group |ref|) + COND * absum,
    absum being the oracle's sum of absolute per-pixel terms (the conditioning of each
    sum; 0 if not given).  Returns the worst ratio (<= 1 passes) and a description of
    the worst entry of each group."""
    worst, lines = 0.0, []
    for a, b in GROUPS:
        r = np.asarray(ref[a:b], np.float64)
        g = np.asarray(got[a:b], np.float64)
        scale = rel * (np.abs(r) + floor * max(np.abs(r).max(), 1e-30))
        if absum is not None:
            scale = scale + COND * np.asarray(absum[a:b], np.float64)
        ratio = np.abs(g - r) / scale
        j = np.unravel_index(int(np.argmax(ratio)), ratio.shape)
        worst = max(worst, float(ratio[j]))
        lines.append(f"params {a}..{b - 1}: worst {ratio[j]:.3g} at param {a + j[0]} site {j[1]} "
                     f"ref {r[j]:.4e} got {g[j]:.4e} (group max {np.abs(r).max():.3e})")
    return worst, "\n".join(lines)


def grad_close(got, ref, absum=None, rel=1e-4, floor=1e-3):
    return grad_report(got, ref, absum, rel, floor)[0]


def grad_check(got, ref, absum, label):
    """The gradient parity rule of the tests (grad_report with the conditioning term),
    and beside it the worst ratio under the plain per-group rule without that term.
    Prints both (and appends them to the JSON-lines file named by SAD_PARITY_LOG, if
    set); returns (widened, plain, description of the widened worst entries)."""
    import json
    import os
    w, rep = grad_report(got, ref, absum)
    plain, _ = grad_report(got, ref, None)
    print(f"PARITY {label}: widened {w:.3g} plain {plain:.3g}", flush=True)
    path = os.environ.get("SAD_PARITY_LOG")
    if path:
        with open(path, "a") as f:
            f.write(json.dumps({"case": label, "widened": w, "plain": plain}) + "\n")
    return w, plain, rep
