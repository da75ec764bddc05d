"""Helpers shared by the GPU parity tests: comparison of edge sets with the
parity bands, and label agreement.  They only compare; neither side of a
comparison is computed here."""
import numpy as np

RADIUS_BAND = 1e-5      # pairs with |d - r| <= band may differ (FP32 vs FP64 distance)
TIE_BAND = 1e-5         # candidates within band of a saturated point's K-th distance


def pair_keys(src, dst, n):
    return np.asarray(src, np.int64) * n + np.asarray(dst, np.int64)


def kth_distance(emb, lo, hi, d2, k_max):
    """Per point: the distance of its k_max-th nearest neighbour within r (inf if unsaturated)."""
    n = emb.shape[0]
    qi = np.concatenate([lo, hi])
    qd = np.concatenate([d2, d2])
    order = np.lexsort((qd, qi))
    qi, qd = qi[order], qd[order]
    cnt = np.bincount(qi, minlength=n)
    start = np.zeros(n + 1, np.int64)
    start[1:] = np.cumsum(cnt)
    kth = np.full(n, np.inf)
    sat = cnt > k_max
    kth[sat] = np.sqrt(qd[start[:-1][sat] + k_max - 1])
    return kth


def compare_edges(emb, gsrc, gdst, osrc, odst, radius, k_max, lo, hi, d2, band=None):
    """Returns (n_diff_total, n_diff_outside_bands, details).  `band` widens both
    bands (default RADIUS_BAND and TIE_BAND)."""
    n = emb.shape[0]
    e = np.asarray(emb, np.float64)
    g = pair_keys(gsrc, gdst, n)
    o = pair_keys(osrc, odst, n)
    diff = np.setxor1d(g, o)
    if diff.size == 0:
        return 0, 0, []
    a, b = diff // n, diff % n
    d = np.sqrt(((e[a] - e[b]) ** 2).sum(axis=1))
    kth = kth_distance(e, lo, hi, d2, k_max)
    rb = RADIUS_BAND if band is None else band
    tb = TIE_BAND if band is None else band
    in_band = (np.abs(d - radius) <= rb) | (np.abs(d - kth[a]) <= tb) | (np.abs(d - kth[b]) <= tb)
    bad = ~in_band
    details = [(int(x), int(y), float(z), bool(x * n + y in set(g.tolist()))) for x, y, z in
               zip(a[bad][:10], b[bad][:10], d[bad][:10])]
    return int(diff.size), int(bad.sum()), details


def label_agreement(la, lb, min_hits=3):
    """Hit-level agreement and exact-match Jaccard of candidates with >= min_hits hits."""
    la, lb = np.asarray(la), np.asarray(lb)
    hit = float(np.mean(canonical(la) == canonical(lb))) if la.size else 1.0

    def cands(lab):
        out = {}
        for i, v in enumerate(lab.tolist()):
            out.setdefault(v, []).append(i)
        return {tuple(v) for v in out.values() if len(v) >= min_hits}

    ca, cb = cands(la), cands(lb)
    union = ca | cb
    jac = len(ca & cb) / len(union) if union else 1.0
    return hit, jac


def canonical(labels):
    """Relabel to min-id form (identity for labels already in that form)."""
    labels = np.asarray(labels, np.int64)
    first = {}
    out = np.empty_like(labels)
    for i, v in enumerate(labels.tolist()):
        out[i] = first.setdefault(v, i)
    return out
