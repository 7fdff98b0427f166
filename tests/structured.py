"""Helpers on the structured band layout (row i, slot s = (s_1..s_d) in C order over
2p+1 per direction, column j_k = i_k - p + s_k): dense expansion for tiny spaces and
the error metrics used by the parity tests."""
import numpy as np


def row_multi(n, rows):
    rows = np.asarray(rows, dtype=np.int64)
    idx = []
    rem = rows.copy()
    for nk in reversed(n):
        idx.append(rem % nk)
        rem //= nk
    return idx[::-1]


def columns(n, p, rows):
    """[len(rows), S^d] flat column index of every slot (-1 where outside the space)."""
    d = len(n)
    S = 2 * p + 1
    idx = row_multi(n, rows)
    s = np.array(np.unravel_index(np.arange(S ** d), [S] * d))      # [d, SD]
    col = np.zeros((len(idx[0]), S ** d), dtype=np.int64)
    ok = np.ones_like(col, dtype=bool)
    for k in range(d):
        jk = idx[k][:, None] - p + s[k][None, :]
        ok &= (jk >= 0) & (jk < n[k])
        col = col * n[k] + jk
    return np.where(ok, col, -1)


def to_dense(vals, n, p):
    """Dense [N, N] matrix from structured rows [N, S^d] (all rows, C order)."""
    N = int(np.prod(n))
    cols = columns(n, p, np.arange(N))
    D = np.zeros((N, N))
    r, s = np.nonzero(cols >= 0)
    D[r, cols[r, s]] = vals[r, s]
    return D


def from_dense(D, n, p, rows=None):
    N = int(np.prod(n))
    rows = np.arange(N) if rows is None else np.asarray(rows)
    cols = columns(n, p, rows)
    out = np.zeros(cols.shape)
    ok = cols >= 0
    rr = np.broadcast_to(np.arange(len(rows))[:, None], cols.shape)
    out[ok] = D[rows[rr[ok]], cols[ok]]
    return out


def row_scaled_error(got, want):
    """max over rows and slots of |got - want| / max_s' |want[row, s']| (rows of zeros skipped)."""
    got = np.asarray(got, dtype=np.float64)
    want = np.asarray(want, dtype=np.float64)
    scale = np.abs(want).max(axis=1, keepdims=True)
    scale[scale == 0] = 1.0
    return float((np.abs(got - want) / scale).max())


def entry_relative_error(got, want, floor=0.0):
    """max |got - want| / |want| over entries with |want| > floor (0/0 skipped)."""
    got = np.asarray(got, dtype=np.float64)
    want = np.asarray(want, dtype=np.float64)
    m = np.abs(want) > floor
    if not m.any():
        return 0.0
    return float((np.abs(got[m] - want[m]) / np.abs(want[m])).max())


def point_offsets(n, p, rows):
    """[len(rows), (p+1)^d] flat grid offsets of the points owned by each row: row i owns
    grid point (i_k (p+1) + q_k)_k of the C-ordered [n_k (p+1)] grid, q in C order."""
    d = len(n)
    Q = p + 1
    idx = row_multi(n, rows)
    qs = np.array(np.unravel_index(np.arange(Q ** d), [Q] * d))       # [d, QD]
    off = np.zeros((len(idx[0]), Q ** d), dtype=np.int64)
    for k in range(d):
        off = off * (n[k] * Q) + (idx[k][:, None] * Q + qs[k][None, :])
    return off


def sample_rows(n, p, count, seed):
    """Deterministic row sample that covers every boundary class: rows whose index in
    each direction is drawn from the first and last 2p+1 indices and a few interior
    ones, plus uniformly random rows; sorted, unique."""
    rng = np.random.default_rng(seed)
    d = len(n)
    cand = []
    for nk in n:
        edge = list(range(min(nk, 2 * p + 1))) + list(range(max(0, nk - 2 * p - 1), nk))
        inner = list(rng.integers(0, nk, size=4))
        cand.append(np.unique(np.array(edge + inner)))
    picks = np.stack([rng.choice(c, size=count) for c in cand])           # [d, count]
    flat = np.zeros(count, dtype=np.int64)
    for k in range(d):
        flat = flat * n[k] + picks[k]
    corners = np.array(np.meshgrid(*[[0, nk - 1] for nk in n], indexing="ij")).reshape(d, -1)
    cflat = np.zeros(corners.shape[1], dtype=np.int64)
    for k in range(d):
        cflat = cflat * n[k] + corners[k]
    total = int(np.prod(n))
    rand = rng.integers(0, total, size=count // 2)
    return np.unique(np.concatenate([flat, cflat, rand]))
