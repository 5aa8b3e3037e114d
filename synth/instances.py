"""Seeded synthetic instances of the per-day DODE non-negative least-squares problem.

Every array here is an *input*: the static link/OD incidence pattern, the lag
ratios of each cluster's assignment matrix, the planted demand, the observed
link counts and the per-epoch row permutations.  Nothing in this module runs any
step of the SPGD solver (no residual, gradient, step or projection); the
observation model x = rho q* + noise is data synthesis, done with dense-block
BLAS products or, for small cases, element loops in a fixed order.

Shapes follow the paper's discretisation (section "Tensor representation",
Table "DODE framework variable vectorization"): per day the OD vector is
q[t][p] (interval-major, OD-minor), the link vector is x[h][a].  The
assignment matrix of cluster c is stored as lag-band blocks: entry
rho[(t+l)*L + a, t*P + p] = W_c[l][t][nz] where nz indexes the (a, p) pair in
the incidence pattern (CSR, rows = links, sorted columns).  Blocks with
t + l >= H are absent (midnight spill-over dropped, section "Estimate the
dynamic OD demand").
"""
from __future__ import annotations

from dataclasses import dataclass, field
import math

import numpy as np

BASE_SEED = 190109266

# Synthetic workloads: sizes, densities and SPGD hyper-parameters of the five
# benchmark configurations.  The Sacramento network and its PeMS / NPMRDS data
# are not available; these seeded corridors stand in for them.
CONFIGS = {
    1: dict(P=4, L=6, T=12, K=3, sizes=(7,), inc=0.5, pattern="bernoulli",
            demand="uniform50", noise="add1", x_dtype="f64",
            optimizer="fixed", epochs=200, batch_rows=8192, eta=None),
    2: dict(P=50, L=200, T=288, K=6, sizes=(365,), inc=0.10, pattern="corridor",
            demand="gamma", noise="mult5", x_dtype="f32",
            optimizer="adagrad", epochs=300, batch_rows=8192, eta=5.0, day_tile=32),
    3: dict(P=150, L=500, T=288, K=6, sizes=(400, 250, 150, 120, 80, 50, 30, 15),
            inc=0.08, pattern="corridor", demand="gamma", noise="mult5", x_dtype="f32",
            optimizer="adagrad", epochs=300, batch_rows=8192, eta=5.0),
    5: dict(P=400, L=1500, T=288, K=6,
            sizes=(300, 200, 150, 110, 90, 70, 50, 40, 30, 25, 20, 10),
            inc=0.08, pattern="corridor", demand="gamma", noise="mult5", x_dtype="f32",
            optimizer="adagrad", epochs=300, batch_rows=8192, eta=5.0),
}


@dataclass
class Instance:
    P: int
    L: int
    T: int
    H: int
    K: int
    sizes: tuple
    day_cluster: np.ndarray      # int32 [D]
    row_ptr: np.ndarray          # int32 [L+1]   incidence pattern, CSR by link
    col_idx: np.ndarray          # int32 [nnz]   OD index of each pattern entry
    W: list                      # per cluster float64 [K][T][nnz] lag-band values
    qstar: np.ndarray            # float64 [D][T][P] planted demand
    x0: object                   # float64 [D][H][L] noiseless observations (None for large instances)
    x: np.ndarray                # [D][H][L] observations (float64 or float32)
    seed: int
    meta: dict = field(default_factory=dict)

    @property
    def D(self) -> int:
        return int(self.day_cluster.shape[0])

    @property
    def C(self) -> int:
        return len(self.sizes)

    @property
    def nnz(self) -> int:
        return int(self.col_idx.shape[0])

    def row_of_nz(self) -> np.ndarray:
        return np.repeat(np.arange(self.L, dtype=np.int32), np.diff(self.row_ptr))

    def dense_blocks(self, c: int) -> np.ndarray:
        """[K][T][L][P] dense copy of cluster c's lag blocks (small instances only)."""
        B = np.zeros((self.K, self.T, self.L, self.P))
        rows = self.row_of_nz()
        B[:, :, rows, self.col_idx] = self.W[c]
        return B

    def days_of(self, c: int) -> np.ndarray:
        return np.nonzero(self.day_cluster == c)[0].astype(np.int32)


@dataclass
class RouteInstance:
    """Path-level description for the route-choice parameterisation.

    Path k serves OD path_od[k] and crosses links pair_link[pair_ptr[k]:pair_ptr[k+1]];
    R[c][l][t][m] is the lag ratio of path-link pair m (normalised over l).  The
    OD-level pattern (row_ptr, col_idx) is the union of the path incidences, and
    pair_nz[m] is the pattern entry that pair m feeds.
    """
    P: int
    L: int
    T: int
    H: int
    K: int
    n_paths: int
    path_od: np.ndarray          # int32 [n_paths]
    pair_ptr: np.ndarray         # int32 [n_paths+1]
    pair_link: np.ndarray        # int32 [n_pairs]
    pair_nz: np.ndarray          # int32 [n_pairs]
    row_ptr: np.ndarray          # int32 [L+1]
    col_idx: np.ndarray          # int32 [nnz]
    R: list                      # per cluster float64 [K][T][n_pairs]
    pi_true: list                # per cluster float64 [n_paths] true route proportions
    z0: list                     # per cluster float64 [n_paths] starting logits
    qstar: np.ndarray
    x: np.ndarray
    day_cluster: np.ndarray
    sizes: tuple
    seed: int

    @property
    def n_pairs(self) -> int:
        return int(self.pair_link.shape[0])

    @property
    def nnz(self) -> int:
        return int(self.col_idx.shape[0])

    @property
    def D(self) -> int:
        return int(self.day_cluster.shape[0])


def chunk_h_blocks(L: int, H: int, batch_rows: int) -> int:
    """Whole interval blocks per minibatch: floor(b / L), at least 1, at most H."""
    return int(min(H, max(1, batch_rows // L)))


def _pattern_csr(S: np.ndarray):
    L = S.shape[0]
    row_ptr = np.zeros(L + 1, dtype=np.int32)
    row_ptr[1:] = np.cumsum(S.sum(axis=1))
    _, cols = np.nonzero(S)
    return row_ptr, cols.astype(np.int32)


def _incidence(rng, L, P, inc, pattern):
    if pattern == "bernoulli":
        S = rng.random((L, P)) < inc
        while True:
            empty = np.nonzero(~S.any(axis=0))[0]
            if empty.size == 0:
                break
            S[:, empty] = rng.random((L, empty.size)) < inc
        return S
    if pattern == "corridor":
        # Four corridor-directions of L/4 consecutive links; each OD takes a
        # contiguous route of round(inc*L) links in one of them.  ODs sorted by
        # (corridor, origin).
        ncor = 4 if L >= 4 else 1
        seg = L // ncor
        m = max(1, int(round(inc * L)))
        if m > seg:
            raise ValueError("route longer than a corridor")
        cor = rng.integers(0, ncor, size=P)
        org = rng.integers(0, seg - m + 1, size=P)
        order = np.lexsort((org, cor))
        cor, org = cor[order], org[order]
        S = np.zeros((L, P), dtype=bool)
        for p in range(P):
            s0 = cor[p] * seg + org[p]
            S[s0:s0 + m, p] = True
        return S
    raise ValueError(pattern)


def _lag_ratios(rng, K, T, H, n):
    """[K][T][n] ratios: U(0,1) per lag, normalised over the K lags, then lags
    that land past the last interval are dropped (their mass leaves the day).
    The draws are taken in [T][n][K] order, a slab of intervals at a time (the
    same stream as one draw of the whole array)."""
    W = np.empty((K, T, n))
    step = max(1, (1 << 22) // max(1, n * K))
    for t0 in range(0, T, step):
        t1 = min(T, t0 + step)
        w = rng.random((t1 - t0, n, K))
        w /= w.sum(axis=2, keepdims=True)
        W[:, t0:t1, :] = w.transpose(2, 0, 1)
    for l in range(K):
        if H - l < T:
            W[l, max(H - l, 0):, :] = 0.0
    return W


def _profile(T):
    tau = np.arange(T) * (24.0 / T)
    prof = 0.2 + np.exp(-(tau - 8.0) ** 2 / 2.0) + 0.9 * np.exp(-(tau - 17.5) ** 2 / (2 * 1.25 ** 2))
    return prof / prof.mean()


class _BandCSR:
    """Row-compressed layout of the full (H*L) x (T*P) band matrix of one pattern,
    columns sorted within each row.  Built once per pattern; `src` maps each
    CSR slot to its flat [K][T][nnz] value."""

    def __init__(self, P, L, T, H, K, row_ptr, col_idx):
        row_ptr = np.asarray(row_ptr, dtype=np.int64)
        col_idx = np.asarray(col_idx, dtype=np.int64)
        nnz = col_idx.shape[0]
        deg = np.diff(row_ptr)
        # row (h, a) holds the departure intervals t = h-l inside [0, T) in
        # increasing order, each with the pattern entries of link a
        t_lo = np.maximum(np.arange(H) - (K - 1), 0)
        t_hi = np.minimum(np.arange(H), T - 1)
        nt = np.maximum(t_hi - t_lo + 1, 0)
        lens = (nt[:, None] * deg[None, :]).ravel()
        indptr = np.zeros(H * L + 1, dtype=np.int64)
        np.cumsum(lens, out=indptr[1:])
        indices = np.empty(indptr[-1], dtype=np.int32)
        src = np.empty(indptr[-1], dtype=np.int64)
        # inside row block h (all L links, nt intervals each), pattern entry j
        # of link a at its t-th interval sits at nt*row_ptr[a] + t*deg[a] + (j - row_ptr[a])
        J = np.arange(nnz, dtype=np.int64)
        A = np.repeat(np.arange(L, dtype=np.int64), deg)
        rel = {}
        for h in range(H):
            n_t = int(nt[h])
            if n_t == 0:
                continue
            if n_t not in rel:
                ti = np.arange(n_t, dtype=np.int64)[:, None]
                rel[n_t] = (n_t * row_ptr[A] + ti * deg[A] + (J - row_ptr[A])[None, :]).ravel()
            tt = np.arange(t_lo[h], t_hi[h] + 1, dtype=np.int64)[:, None]
            pos = indptr[h * L] + rel[n_t]
            indices[pos] = (tt * P + col_idx[None, :]).ravel()
            src[pos] = ((h - tt) * T * nnz + tt * nnz + J[None, :]).ravel()
        self.indptr, self.indices, self.src = indptr, indices, src
        self.shape = (H * L, T * P)

    def product(self, Wc, Q):
        """[n][H][L] link counts of the days in Q ([n][T][P]); days are split
        over threads (each row's sum runs in the same order for any split)."""
        import scipy.sparse as sp
        from concurrent.futures import ThreadPoolExecutor
        M = sp.csr_matrix((Wc.ravel()[self.src], self.indices, self.indptr), shape=self.shape)
        n = Q.shape[0]
        Qt = np.ascontiguousarray(Q.reshape(n, -1).T)
        Y = np.empty((n, self.shape[0]))
        step = 16
        chunks = [(d, min(n, d + step)) for d in range(0, n, step)]

        def one(ab):
            a, b = ab
            Y[a:b] = (M @ np.ascontiguousarray(Qt[:, a:b])).T

        with ThreadPoolExecutor(max_workers=min(16, len(chunks))) as ex:
            list(ex.map(one, chunks))
        return Y


def _observe(P, L, T, H, K, row_ptr, col_idx, Wc, Q, band=None):
    """Noiseless link counts of the days in Q ([n][T][P]) under one cluster's blocks."""
    n = Q.shape[0]
    if K * T * L * P > 2_000_000:
        band = band or _BandCSR(P, L, T, H, K, row_ptr, col_idx)
        return band.product(Wc, Q).reshape(n, H, L)
    X0 = np.zeros((n, H, L))
    rows = np.repeat(np.arange(L), np.diff(row_ptr))
    for l in range(K):
        for t in range(min(T, H - l)):
            # fixed-order element loop over the pattern entries
            contrib = Wc[l, t][None, :] * Q[:, t, col_idx]                # [n][nnz]
            for j in range(rows.shape[0]):
                X0[:, t + l, rows[j]] += contrib[:, j]
    return X0


def make_instance(P, L, T, K, sizes, inc, pattern="corridor", demand="gamma", noise="mult5",
                  x_dtype="f32", seed=BASE_SEED, H=None, planted_zero_frac=0.0, keep_x0=False,
                  progress=None, **_ignored):
    """Seeded synthetic instance; `progress(msg)`, when given, is called after
    each generation stage (large instances take minutes)."""
    H = T if H is None else H
    rng = np.random.Generator(np.random.PCG64(seed))
    S = _incidence(rng, L, P, inc, pattern)
    row_ptr, col_idx = _pattern_csr(S)
    nnz = col_idx.shape[0]
    C = len(sizes)
    W = [_lag_ratios(rng, K, T, H, nnz) for _ in range(C)]
    if progress:
        progress(f"lag ratios of {C} clusters ({nnz} pattern entries)")
    D = int(sum(sizes))
    day_cluster = np.repeat(np.arange(C, dtype=np.int32), sizes)
    if demand == "uniform50":
        qstar = rng.uniform(0.0, 50.0, size=(D, T, P))
    elif demand == "gamma":
        qstar = rng.standard_gamma(2.0, size=(D, T, P), dtype=np.float32).astype(np.float64)
        qstar *= 10.0 * _profile(T)[None, :, None]
    else:
        raise ValueError(demand)
    if planted_zero_frac > 0:
        qstar[rng.random(qstar.shape) < planted_zero_frac] = 0.0
    big = K * T * L * P > 2_000_000
    band = _BandCSR(P, L, T, H, K, row_ptr, col_idx) if big else None
    if progress and big:
        progress("band matrix layout")
    keep = keep_x0 or not big
    x0 = np.empty((D, H, L)) if keep else None
    x = np.empty((D, H, L), dtype=np.float32 if x_dtype == "f32" else np.float64)
    for c in range(C):
        d = np.nonzero(day_cluster == c)[0]
        x0c = _observe(P, L, T, H, K, row_ptr, col_idx, W[c], qstar[d], band)
        if keep:
            x0[d] = x0c
        # observation noise, drawn cluster by cluster
        if noise == "add1":
            x0c += rng.standard_normal(x0c.shape)
        elif noise == "mult5":
            x0c *= 1.0 + 0.05 * rng.standard_normal(x0c.shape, dtype=np.float32)
        elif noise != "none":
            raise ValueError(noise)
        np.maximum(x0c, 0.0, out=x0c)
        x[d] = x0c
        del x0c
        if progress:
            progress(f"observations of cluster {c + 1}/{C}")
    return Instance(P=P, L=L, T=T, H=H, K=K, sizes=tuple(int(s) for s in sizes),
                    day_cluster=day_cluster, row_ptr=row_ptr, col_idx=col_idx, W=W,
                    qstar=qstar, x0=x0, x=x, seed=seed,
                    meta=dict(inc=inc, pattern=pattern, demand=demand, noise=noise))


def make_config(cid: int, sizes=None, pattern=None, seed=None, progress=None) -> Instance:
    """Instance for one benchmark configuration (optionally with fewer days or
    the Bernoulli stress pattern).  Seed = 190109266 + 100 * config id."""
    cfg = dict(CONFIGS[cid])
    if sizes is not None:
        cfg["sizes"] = tuple(sizes)
    if pattern is not None:
        cfg["pattern"] = pattern
    s = BASE_SEED + 100 * cid if seed is None else seed
    inst = make_instance(seed=s, progress=progress, **cfg)
    inst.meta.update(config=cid, epochs=cfg["epochs"], batch_rows=cfg["batch_rows"],
                     optimizer=cfg["optimizer"], eta=cfg["eta"])
    return inst


def make_perms(seed: int, E: int, C: int, H: int) -> np.ndarray:
    """int32 [E][C][H]: one Fisher-Yates shuffle of the H interval blocks per (epoch, cluster)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    out = np.empty((E, C, H), dtype=np.int32)
    for e in range(E):
        for c in range(C):
            out[e, c] = rng.permutation(H)
    return out


def make_row_perms(seed: int, E: int, n_rows: int) -> np.ndarray:
    """int32 [E][n_rows]: row-level shuffles for the paper-literal row minibatches."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return np.stack([rng.permutation(n_rows) for _ in range(E)]).astype(np.int32)


def make_route_instance(P=4, L=6, T=12, K=3, n_paths=150, sizes=(7,), link_prob=0.5,
                        seed=BASE_SEED + 400, noise="add1") -> RouteInstance:
    """Route-choice workload: n_paths candidate paths spread over the P ODs, each
    with a Bernoulli(link_prob) non-empty link set and its own lag ratios.  True
    route proportions are Dirichlet(1) per OD; starting logits are N(0,1)."""
    H = T
    rng = np.random.Generator(np.random.PCG64(seed))
    path_od = np.repeat(np.arange(P, dtype=np.int32), [len(a) for a in np.array_split(np.arange(n_paths), P)])
    links = []
    for k in range(n_paths):
        while True:
            m = rng.random(L) < link_prob
            if m.any():
                break
        links.append(np.nonzero(m)[0].astype(np.int32))
    pair_ptr = np.zeros(n_paths + 1, dtype=np.int32)
    pair_ptr[1:] = np.cumsum([len(a) for a in links])
    pair_link = np.concatenate(links).astype(np.int32)
    pair_path = np.repeat(np.arange(n_paths), np.diff(pair_ptr))
    S = np.zeros((L, P), dtype=bool)
    S[pair_link, path_od[pair_path]] = True
    row_ptr, col_idx = _pattern_csr(S)
    nzmap = -np.ones((L, P), dtype=np.int64)
    rows = np.repeat(np.arange(L), np.diff(row_ptr))
    nzmap[rows, col_idx] = np.arange(col_idx.shape[0])
    pair_nz = nzmap[pair_link, path_od[pair_path]].astype(np.int32)
    C = len(sizes)
    R = [_lag_ratios(rng, K, T, H, pair_link.shape[0]) for _ in range(C)]
    pi_true, z0 = [], []
    for c in range(C):
        pi = np.empty(n_paths)
        for p in range(P):
            ks = np.nonzero(path_od == p)[0]
            pi[ks] = rng.dirichlet(np.ones(ks.size))
        pi_true.append(pi)
        z0.append(rng.standard_normal(n_paths))
    D = int(sum(sizes))
    day_cluster = np.repeat(np.arange(C, dtype=np.int32), sizes)
    qstar = rng.uniform(0.0, 50.0, size=(D, T, P))
    x = np.empty((D, H, L))
    for c in range(C):
        # true assignment of cluster c: path ratios weighted by true proportions
        Wc = np.zeros((K, T, col_idx.shape[0]))
        np.add.at(Wc, (slice(None), slice(None), pair_nz), R[c] * pi_true[c][pair_path][None, None, :])
        d = np.nonzero(day_cluster == c)[0]
        x[d] = _observe(P, L, T, H, K, row_ptr, col_idx, Wc, qstar[d])
    if noise == "add1":
        x = np.maximum(0.0, x + rng.standard_normal(x.shape))
    return RouteInstance(P=P, L=L, T=T, H=H, K=K, n_paths=n_paths, path_od=path_od,
                         pair_ptr=pair_ptr, pair_link=pair_link, pair_nz=pair_nz,
                         row_ptr=row_ptr, col_idx=col_idx, R=R, pi_true=pi_true, z0=z0,
                         qstar=qstar, x=x, day_cluster=day_cluster, sizes=tuple(sizes), seed=seed)


@dataclass
class SpeedInstance:
    """Corridor network with ordered routes and per-day link speeds (for the
    dynamic assignment ratios of paths)."""
    L: int
    H: int
    dt: float                 # minutes per interval
    path_ptr: np.ndarray      # [n_paths+1] int32
    path_link: np.ndarray     # [n_pairs] int32, links of each path in traversal order
    link_len: np.ndarray      # [L] miles
    speed: np.ndarray         # [D][L][H] float32, miles per minute
    day_cluster: np.ndarray   # [D] int32
    sizes: tuple
    seed: int


def make_speed_instance(L=500, P=150, H=288, sizes=(400, 250, 150, 120, 80, 50, 30, 15),
                        inc=0.08, dt=5.0, seed=BASE_SEED + 600, progress=None) -> SpeedInstance:
    """Routes of the corridor pattern (each OD one path: round(inc*L) consecutive
    links of one of 4 corridor-directions, in driving order), link lengths
    U(0.15, 0.35) mi, free-flow speed 65 mph, and per-day speeds
    v = vff * (1 - depth_c * congestion(t)) * (1 + 0.05 N(0,1)) clipped to
    [5, 80] mph.  The congestion profile has AM and PM peaks; its depth depends
    on the cluster (deep weekday-like patterns down to shallow weekend-like
    ones) and on the corridor-direction (AM peak inbound, PM outbound)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    ncor = 4
    seg = L // ncor
    m = max(1, int(round(inc * L)))
    cor = rng.integers(0, ncor, size=P)
    org = rng.integers(0, seg - m + 1, size=P)
    order = np.lexsort((org, cor))
    cor, org = cor[order], org[order]
    path_link = np.concatenate([cor[p] * seg + org[p] + np.arange(m) for p in range(P)]).astype(np.int32)
    path_ptr = (np.arange(P + 1) * m).astype(np.int32)
    link_len = rng.uniform(0.15, 0.35, size=L)
    C = len(sizes)
    D = int(sum(sizes))
    day_cluster = np.repeat(np.arange(C, dtype=np.int32), sizes)
    tau = (np.arange(H) + 0.5) * dt / 60.0                          # hour of day
    am = np.exp(-(tau - 8.0) ** 2 / 2.0)
    pm = np.exp(-(tau - 17.5) ** 2 / (2 * 1.25 ** 2))
    depth = np.linspace(0.6, 0.1, C)                                 # per cluster
    link_cor = np.arange(L) // seg
    inbound = (link_cor % 2 == 0)[:, None]                           # [L][1]
    vff = 65.0 / 60.0                                                # miles per minute
    speed = np.empty((D, L, H), dtype=np.float32)
    for c in range(C):
        prof = np.where(inbound, am[None, :] + 0.4 * pm[None, :], 0.4 * am[None, :] + pm[None, :])
        base = vff * (1.0 - depth[c] * prof)                          # [L][H]
        for d in np.nonzero(day_cluster == c)[0]:
            v = base * (1.0 + 0.05 * rng.standard_normal((L, H)))
            speed[d] = np.clip(v, 5.0 / 60.0, 80.0 / 60.0)
        if progress:
            progress(f"speeds of cluster {c + 1}/{C}")
    return SpeedInstance(L=L, H=H, dt=dt, path_ptr=path_ptr, path_link=path_link,
                         link_len=link_len, speed=speed, day_cluster=day_cluster,
                         sizes=tuple(sizes), seed=seed)


@dataclass
class ChoiceInstance:
    """Corridor network with alternative routes per OD and per-day link speeds
    (for route portions from mean path costs and the assignment matrix they
    give).  Path k serves OD path_od[k] and crosses links
    path_link[path_ptr[k]:path_ptr[k+1]] in driving order; the OD-level pattern
    (row_ptr, col_idx) is the union of the path incidences, and pair_nz[m] is
    the pattern entry that pair m feeds."""
    P: int
    L: int
    T: int
    H: int
    K: int
    dt: float                 # minutes per interval
    path_od: np.ndarray       # [n_paths] int32
    path_ptr: np.ndarray      # [n_paths+1] int32
    path_link: np.ndarray     # [n_pairs] int32
    pair_nz: np.ndarray       # [n_pairs] int32
    row_ptr: np.ndarray       # [L+1] int32
    col_idx: np.ndarray       # [nnz] int32
    link_len: np.ndarray      # [L] miles
    speed: np.ndarray         # [D][L][H] float32, miles per minute
    day_cluster: np.ndarray   # [D] int32
    sizes: tuple
    seed: int

    @property
    def n_paths(self) -> int:
        return int(self.path_od.shape[0])

    @property
    def n_pairs(self) -> int:
        return int(self.path_link.shape[0])

    @property
    def nnz(self) -> int:
        return int(self.col_idx.shape[0])


def make_choice_instance(L=500, P=150, H=288, K=6, sizes=(400, 250, 150, 120, 80, 50, 30, 15),
                         m=20, dt=5.0, ragged=False, seed=BASE_SEED + 700,
                         progress=None) -> ChoiceInstance:
    """Each of 4 corridor-directions has a freeway and a parallel arterial of
    L//8 links each (link i of one beside link i of the other).  OD p spans m
    consecutive link positions of one corridor-direction and has three routes:
    all freeway, all arterial, and freeway for the first half then arterial
    (with ragged=True each OD keeps a random non-empty subset of them, and m
    varies per OD in [m/2, m]).  Link lengths U(0.15, 0.35) mi (arterial links
    1.1x); free-flow speed 65 mph on freeways, 35 mph on arterials; per-day
    speeds v = vff * (1 - depth * congestion(t)) * (1 + 0.05 N(0,1)) clipped
    to [5, 80] mph, with AM/PM peaks by direction, the freeway depth per
    cluster from 0.7 down to 0.1 and the arterial depth 0.3 of it."""
    rng = np.random.Generator(np.random.PCG64(seed))
    ncor = 4
    seg = L // (2 * ncor)
    if seg < m:
        raise ValueError("corridor shorter than a route")
    fw = lambda c, i: c * seg + i                     # freeway link i of corridor c
    art = lambda c, i: ncor * seg + c * seg + i       # arterial link i of corridor c
    cor = rng.integers(0, ncor, size=P)
    path_od, links = [], []
    for p in range(P):
        mp = int(rng.integers((m + 1) // 2, m + 1)) if ragged else m
        o = int(rng.integers(0, seg - mp + 1))
        idx = np.arange(o, o + mp)
        h = mp // 2
        alts = [fw(cor[p], idx), art(cor[p], idx),
                np.concatenate([fw(cor[p], idx[:h]), art(cor[p], idx[h:])])]
        keep = [0, 1, 2]
        if ragged:
            while True:
                keep = [i for i in range(3) if rng.random() < 0.6]
                if keep:
                    break
        for i in keep:
            path_od.append(p)
            links.append(np.asarray(alts[i], dtype=np.int32))
    path_od = np.asarray(path_od, dtype=np.int32)
    path_ptr = np.zeros(len(links) + 1, dtype=np.int32)
    path_ptr[1:] = np.cumsum([len(a) for a in links])
    path_link = np.concatenate(links).astype(np.int32)
    pair_path = np.repeat(np.arange(len(links)), np.diff(path_ptr))
    S = np.zeros((L, P), dtype=bool)
    S[path_link, path_od[pair_path]] = True
    row_ptr, col_idx = _pattern_csr(S)
    nzmap = -np.ones((L, P), dtype=np.int64)
    rows = np.repeat(np.arange(L), np.diff(row_ptr))
    nzmap[rows, col_idx] = np.arange(col_idx.shape[0])
    pair_nz = nzmap[path_link, path_od[pair_path]].astype(np.int32)
    is_art = np.arange(L) >= ncor * seg
    link_len = rng.uniform(0.15, 0.35, size=L) * np.where(is_art, 1.1, 1.0)
    C = len(sizes)
    D = int(sum(sizes))
    day_cluster = np.repeat(np.arange(C, dtype=np.int32), sizes)
    tau = (np.arange(H) + 0.5) * dt / 60.0                          # hour of day
    am = np.exp(-(tau - 8.0) ** 2 / 2.0)
    pm = np.exp(-(tau - 17.5) ** 2 / (2 * 1.25 ** 2))
    depth = np.linspace(0.7, 0.1, C)
    inbound = ((np.arange(L) % (ncor * seg)) // seg % 2 == 0)[:, None]
    prof = np.where(inbound, am[None, :] + 0.4 * pm[None, :], 0.4 * am[None, :] + pm[None, :])
    vff = np.where(is_art, 35.0, 65.0)[:, None] / 60.0               # miles per minute
    dscale = np.where(is_art, 0.3, 1.0)[:, None]
    speed = np.empty((D, L, H), dtype=np.float32)
    for c in range(C):
        base = vff * (1.0 - depth[c] * dscale * prof)
        for d in np.nonzero(day_cluster == c)[0]:
            v = base * (1.0 + 0.05 * rng.standard_normal((L, H)))
            speed[d] = np.clip(v, 5.0 / 60.0, 80.0 / 60.0)
        if progress:
            progress(f"speeds of cluster {c + 1}/{C}")
    return ChoiceInstance(P=P, L=L, T=H, H=H, K=K, dt=dt, path_od=path_od, path_ptr=path_ptr,
                          path_link=path_link, pair_nz=pair_nz, row_ptr=row_ptr, col_idx=col_idx,
                          link_len=link_len, speed=speed, day_cluster=day_cluster,
                          sizes=tuple(sizes), seed=seed)


def make_dense_instance(n, m=None, seed=BASE_SEED + 800, epochs=0, chunk=8192):
    """The efficiency experiment's random NNLS: B [m][n] (m = n by default)
    with U(0,1) entries, x* with U(0,1) entries, y = B x* (FP64), and `epochs`
    row permutations [E][m].  Returns (B, y, xstar, perms)."""
    m = n if m is None else m
    rng = np.random.Generator(np.random.PCG64(seed + n))
    B = rng.uniform(0.0, 1.0, size=(m, n))
    xstar = rng.uniform(0.0, 1.0, size=n)
    y = B @ xstar
    prng = np.random.Generator(np.random.PCG64(seed + n + 1))
    perms = np.stack([prng.permutation(m) for _ in range(epochs)]).astype(np.int32) if epochs else \
        np.zeros((0, m), dtype=np.int32)
    return B, y, xstar, perms
