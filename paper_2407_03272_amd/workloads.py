"""Seeded synthetic inputs shaped like the paper's workloads.

This module only builds inputs: sparse matrices in CSR form (int32 row
pointers and column indices, float64 values, columns sorted within each row,
diagonal stored explicitly) and right-hand sides.  It holds none of the
solver's arithmetic, so both the CPU oracle tests and the GPU path can draw
the same inputs from it.

Workloads (paper context in brackets):

* ``poisson_dirichlet`` -- 5-point (2D) / 7-point (3D) Dirichlet Laplacians
  on a regular grid, diagonal 2d and off-diagonals -1.  These are SPD
  stiffness matrices of the kind the experiments on SPD systems use
  (Section 4.3); the paper's own SuiteSparse matrices are not available, so
  these stand in for them.
* ``chung_lu_laplacian`` -- singular graph Laplacian L = Deg - A of a
  power-law random graph (Section 4.2 defines L(G); the SNAP graphs used
  there are not available, so a Chung-Lu graph with exponent 2.5 and mean
  degree 16 stands in for them).
* ``sdd_system`` -- the strictly diagonally dominant system of Section 4.1,
  Q = (n+1) I - 1 1^T with b = 1, whose solution is x* = 1.
* ``random_spd`` / ``random_laplacian`` -- tiny irregular systems for tests.
* ``fe_p1_system`` -- P1 finite-element stiffness matrices on jittered 2D/3D
  grids with lognormal coefficients and a lumped reaction term (SPD).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np
import scipy.sparse as sp


@dataclass
class CsrSystem:
    """A linear system Q x = b with Q in CSR form (see module docstring)."""

    rowptr: np.ndarray            # int32[n+1]
    colidx: np.ndarray            # int32[nnz]
    vals: np.ndarray              # float64[nnz]
    b: np.ndarray                 # float64[n] (or float64[n, k] row-interleaved)
    xstar: np.ndarray | None = None
    name: str = ""
    meta: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return int(self.rowptr.shape[0] - 1)

    @property
    def nnz(self) -> int:
        return int(self.colidx.shape[0])

    def scipy(self) -> sp.csr_matrix:
        return sp.csr_matrix((self.vals, self.colidx, self.rowptr), shape=(self.n, self.n))


def _csr_from_dense_cols(cols: np.ndarray, vals: np.ndarray):
    """Pack an (n, w) table of column indices (-1 = absent) into CSR."""
    mask = cols >= 0
    counts = mask.sum(axis=1)
    rowptr = np.zeros(cols.shape[0] + 1, dtype=np.int64)
    np.cumsum(counts, out=rowptr[1:])
    colidx = cols[mask].astype(np.int32)
    v = vals[mask].astype(np.float64)
    return rowptr.astype(np.int32), colidx, v


def poisson_dirichlet(shape: tuple[int, ...]):
    """CSR of the Dirichlet Laplacian on the interior grid ``shape``.

    2D: 5-point stencil, diagonal 4.  3D: 7-point stencil, diagonal 6.
    Off-diagonals are -1.  Unknown (i0, i1[, i2]) has index
    i0 + s0*(i1 + s1*i2) (first axis fastest).  Columns come out sorted.
    Returns (rowptr, colidx, vals).
    """
    d = len(shape)
    if d not in (2, 3):
        raise ValueError("shape must be 2D or 3D")
    n = int(np.prod(shape))
    idx = np.arange(n, dtype=np.int64)
    coords = []
    rem = idx.copy()
    for s in shape:
        coords.append(rem % s)
        rem //= s
    strides = [1]
    for s in shape[:-1]:
        strides.append(strides[-1] * s)
    # neighbour offsets in increasing column order: -stride_{d-1} ... -1, 0, +1 ... +stride_{d-1}
    offs = []
    for a in reversed(range(d)):
        offs.append((a, -1))
    offs.append((None, 0))
    for a in range(d):
        offs.append((a, +1))
    cols = np.full((n, 2 * d + 1), -1, dtype=np.int64)
    vals = np.zeros((n, 2 * d + 1), dtype=np.float64)
    for k, (a, sgn) in enumerate(offs):
        if a is None:
            cols[:, k] = idx
            vals[:, k] = 2.0 * d
        else:
            ok = (coords[a] + sgn >= 0) & (coords[a] + sgn < shape[a])
            cols[ok, k] = idx[ok] + sgn * strides[a]
            vals[ok, k] = -1.0
    return _csr_from_dense_cols(cols, vals)


def poisson_apply(shape: tuple[int, ...], x: np.ndarray) -> np.ndarray:
    """b = Q x for the Dirichlet Laplacian of ``poisson_dirichlet``, computed on the grid.

    Used only to manufacture right-hand sides b = Q x* for a chosen x*.
    """
    d = len(shape)
    g = x.reshape(tuple(reversed(shape)))  # C order: last grid axis is fastest
    out = 2.0 * d * g
    for ax in range(d):
        sl_lo = [slice(None)] * d
        sl_hi = [slice(None)] * d
        sl_lo[ax] = slice(0, -1)
        sl_hi[ax] = slice(1, None)
        out[tuple(sl_lo)] -= g[tuple(sl_hi)]
        out[tuple(sl_hi)] -= g[tuple(sl_lo)]
    return out.reshape(-1)


def poisson_system(shape: tuple[int, ...], seed: int, nrhs: int = 1, name: str = "") -> CsrSystem:
    """Dirichlet Laplacian with x* ~ N(0,1) (seeded, numpy PCG64) and b = Q x*."""
    rowptr, colidx, vals = poisson_dirichlet(shape)
    n = rowptr.shape[0] - 1
    rng = np.random.default_rng(seed)
    if nrhs == 1:
        xs = rng.standard_normal(n)
        b = poisson_apply(shape, xs)
    else:
        xs = rng.standard_normal((n, nrhs))
        b = np.stack([poisson_apply(shape, np.ascontiguousarray(xs[:, j])) for j in range(nrhs)], axis=1)
    return CsrSystem(rowptr, colidx, vals, b, xs, name or f"poisson{'x'.join(map(str, shape))}",
                     {"shape": tuple(shape), "seed": seed})


def poisson2d_64(seed: int = 1001) -> CsrSystem:
    """2D 5-point Dirichlet Poisson on the 64x64 interior grid: n=4096, nnz=20224."""
    return poisson_system((64, 64), seed, name="poisson2d_64x64")


def poisson3d_128(seed: int = 1002) -> CsrSystem:
    """3D 7-point Dirichlet Laplacian on 128^3: n=2,097,152, nnz=14,581,760."""
    return poisson_system((128, 128, 128), seed, name="laplace3d_128")


# ----------------------------------------------------------------------------
# Section 4.1: strictly diagonally dominant system
# ----------------------------------------------------------------------------

def sdd_system(n: int) -> CsrSystem:
    """Q = (n+1) I - 1 1^T (diagonal n, off-diagonal -1), b = 1, x* = 1 (Section 4.1)."""
    rowptr = (np.arange(n + 1, dtype=np.int64) * n).astype(np.int32)
    colidx = np.tile(np.arange(n, dtype=np.int32), n)
    vals = np.full(n * n, -1.0)
    vals[np.arange(n) * n + np.arange(n)] = float(n)
    return CsrSystem(rowptr, colidx, vals, np.ones(n), np.ones(n), f"sdd{n}", {"n": n})


# ----------------------------------------------------------------------------
# Section 4.2: graph Laplacians (Chung-Lu stand-in for the SNAP graphs)
# ----------------------------------------------------------------------------

def _laplacian_from_edges(n: int, u: np.ndarray, v: np.ndarray):
    """CSR of L = Deg - A for the simple undirected graph with edge list (u, v), u != v, no duplicates."""
    rows = np.concatenate([u, v, np.arange(n)])
    cols = np.concatenate([v, u, np.arange(n)])
    deg = np.bincount(np.concatenate([u, v]), minlength=n).astype(np.float64)
    data = np.concatenate([-np.ones(2 * u.shape[0]), deg])
    A = sp.csr_matrix((data, (rows, cols)), shape=(n, n))
    A.sort_indices()
    return A.indptr.astype(np.int32), A.indices.astype(np.int32), A.data.astype(np.float64)


def _inverse_cdf(cdf: np.ndarray, r: np.ndarray) -> np.ndarray:
    """searchsorted(cdf, r, side="right") for each r, done on the sorted draws (the same indices, far
    fewer cache misses than searching draws in random order)."""
    order = np.argsort(r)
    out = np.empty(r.shape[0], dtype=np.int64)
    out[order] = np.searchsorted(cdf, r[order], side="right")
    return out


def chung_lu_edges(n: int, mean_degree: float = 16.0, gamma: float = 2.5, seed: int = 1003,
                   offset: float = 1.0):
    """Chung-Lu random graph with power-law expected degrees.

    Expected degrees w_i ~ (i + offset)^(-1/(gamma-1)), scaled to the target mean
    and capped at sqrt(sum w).  n*mean/2 edges are drawn with both endpoints
    chosen with probability proportional to w; self-loops and duplicate edges
    are dropped.  Vertices are relabelled by a seeded random permutation.
    Returns (u, v) with u < v.
    """
    rng = np.random.default_rng(seed)
    i = np.arange(n, dtype=np.float64)
    w = (i + offset) ** (-1.0 / (gamma - 1.0))
    w *= mean_degree * n / w.sum()
    cap = math.sqrt(w.sum())
    w = np.minimum(w, cap)
    cdf = np.cumsum(w)
    cdf /= cdf[-1]
    m = int(round(n * mean_degree / 2))
    a = _inverse_cdf(cdf, rng.random(m))
    c = _inverse_cdf(cdf, rng.random(m))
    np.minimum(a, n - 1, out=a)
    np.minimum(c, n - 1, out=c)
    keep = a != c
    a, c = a[keep], c[keep]
    lo, hi = np.minimum(a, c), np.maximum(a, c)
    key = np.unique(lo * n + hi)
    lo, hi = key // n, key % n
    perm = rng.permutation(n)
    pu, pv = perm[lo], perm[hi]
    return np.minimum(pu, pv), np.maximum(pu, pv)


def mean_zero_per_component(n: int, u: np.ndarray, v: np.ndarray, b: np.ndarray) -> np.ndarray:
    """Project b to the range of the Laplacian: mean zero on each connected component, 0 on isolated vertices."""
    from scipy.sparse.csgraph import connected_components

    A = sp.coo_matrix((np.ones(u.shape[0]), (u, v)), shape=(n, n)).tocsr()
    ncomp, lab = connected_components(A, directed=False)
    sums = np.bincount(lab, weights=b, minlength=ncomp)
    cnt = np.bincount(lab, minlength=ncomp)
    out = b - (sums / cnt)[lab]
    out[cnt[lab] == 1] = 0.0
    return out


def chung_lu_laplacian(n: int = 1 << 22, mean_degree: float = 16.0, gamma: float = 2.5,
                       seed: int = 1003, b_seed: int = 1013, nrhs: int = 1) -> CsrSystem:
    """Singular Laplacian of a Chung-Lu graph with b ~ N(0,1) projected into range(L)."""
    u, v = chung_lu_edges(n, mean_degree, gamma, seed)
    rowptr, colidx, vals = _laplacian_from_edges(n, u, v)
    rng = np.random.default_rng(b_seed)
    if nrhs == 1:
        b = mean_zero_per_component(n, u, v, rng.standard_normal(n))
    else:
        raw = rng.standard_normal((n, nrhs))
        b = np.stack([mean_zero_per_component(n, u, v, np.ascontiguousarray(raw[:, j]))
                      for j in range(nrhs)], axis=1)
    deg = np.diff(rowptr) - 1
    return CsrSystem(rowptr, colidx, vals, b, None, f"chunglu_n{n}",
                     {"n": n, "edges": int(u.shape[0]), "mean_degree": float(2 * u.shape[0] / n),
                      "max_degree": int(deg.max()), "isolated": int((deg == 0).sum()),
                      "seed": seed, "b_seed": b_seed})


# ----------------------------------------------------------------------------
# small irregular systems for tests
# ----------------------------------------------------------------------------

def random_laplacian(n: int, p_edge: float, seed: int, weighted: bool = False):
    """Erdos-Renyi graph Laplacian (possibly disconnected). Returns (rowptr, colidx, vals, u, v)."""
    rng = np.random.default_rng(seed)
    iu, ju = np.triu_indices(n, 1)
    keep = rng.random(iu.shape[0]) < p_edge
    u, v = iu[keep].astype(np.int64), ju[keep].astype(np.int64)
    if not weighted:
        rowptr, colidx, vals = _laplacian_from_edges(n, u, v)
        return rowptr, colidx, vals, u, v
    w = rng.uniform(0.1, 2.0, size=u.shape[0])
    rows = np.concatenate([u, v, np.arange(n)])
    cols = np.concatenate([v, u, np.arange(n)])
    deg = np.bincount(u, weights=w, minlength=n) + np.bincount(v, weights=w, minlength=n)
    data = np.concatenate([-w, -w, deg])
    A = sp.csr_matrix((data, (rows, cols)), shape=(n, n))
    A.sort_indices()
    return A.indptr.astype(np.int32), A.indices.astype(np.int32), A.data.astype(np.float64), u, v


def random_spd(n: int, density: float, seed: int, shift: float = 0.1):
    """Sparse SPD matrix: weighted graph Laplacian plus a positive diagonal shift. Returns (rowptr, colidx, vals)."""
    rowptr, colidx, vals, _, _ = random_laplacian(n, density, seed, weighted=True)
    rng = np.random.default_rng(seed + 7)
    A = sp.csr_matrix((vals, colidx, rowptr), shape=(n, n))
    A = (A + sp.diags(shift + rng.random(n))).tocsr()
    A.sort_indices()
    return A.indptr.astype(np.int32), A.indices.astype(np.int32), A.data.astype(np.float64)


def rhs_in_range(rowptr, colidx, vals, seed: int, nrhs: int = 1) -> np.ndarray:
    """b = Q z for z ~ N(0,1): consistent for any symmetric Q (used for singular test systems)."""
    n = rowptr.shape[0] - 1
    A = sp.csr_matrix((vals, colidx, rowptr), shape=(n, n))
    rng = np.random.default_rng(seed)
    z = rng.standard_normal((n, nrhs)) if nrhs > 1 else rng.standard_normal(n)
    return np.asarray(A @ z)


# ----------------------------------------------------------------------------
# P1 finite-element stiffness systems (batched workload)
# ----------------------------------------------------------------------------

def _grid_simplices(m: int, dim: int) -> np.ndarray:
    """Simplices of the regular grid with m nodes per side: 2 triangles per square (2D),
    6 Kuhn tetrahedra per cube (3D).  Node (i0, i1[, i2]) has index i0 + m*(i1 + m*i2)."""
    if dim == 2:
        i, j = np.meshgrid(np.arange(m - 1), np.arange(m - 1), indexing="ij")
        i, j = i.ravel(), j.ravel()
        n00 = i + m * j
        n10 = n00 + 1
        n01 = n00 + m
        n11 = n01 + 1
        return np.concatenate([np.stack([n00, n10, n11], 1), np.stack([n00, n11, n01], 1)])
    i, j, k = np.meshgrid(np.arange(m - 1), np.arange(m - 1), np.arange(m - 1), indexing="ij")
    base = (i + m * (j + m * k)).ravel()
    step = [1, m, m * m]
    tets = []
    import itertools
    for p in itertools.permutations(range(3)):   # Kuhn: one tetrahedron per axis order
        v0 = base
        v1 = v0 + step[p[0]]
        v2 = v1 + step[p[1]]
        v3 = v2 + step[p[2]]
        tets.append(np.stack([v0, v1, v2, v3], 1))
    return np.concatenate(tets)


def fe_p1_system(n_target: int, dim: int, seed: int, nrhs: int = 8, jitter: float | None = None,
                 reaction_factor: float = 10.0) -> CsrSystem:
    """SPD P1 stiffness system on a jittered grid of the unit square (dim 2) or cube (dim 3).

    m = round(n_target^(1/dim)) nodes per side, every node an unknown (natural boundary condition).
    Interior nodes are moved uniformly by up to jitter*h per coordinate (0.2 in 2D, 0.1 in 3D), redrawn
    until every element has positive volume.  Per-element diffusion kappa_e = exp(Z), Z ~ N(0,1); a lumped
    reaction term c_r = reaction_factor * mean(kappa_e) times the lumped mass makes the matrix SPD.
    nrhs right-hand sides ~ N(0,1), row-interleaved (n x nrhs).
    """
    rng = np.random.default_rng(seed)
    m = max(2, int(round(n_target ** (1.0 / dim))))
    n = m ** dim
    h = 1.0 / (m - 1)
    jit = (0.2 if dim == 2 else 0.1) if jitter is None else jitter
    coords = [np.arange(n) // (m ** k) % m for k in range(dim)]
    X = np.stack([c * h for c in coords], 1)
    interior = np.all([(c > 0) & (c < m - 1) for c in coords], axis=0)
    T = _grid_simplices(m, dim)
    ones = np.ones((T.shape[0], dim + 1, 1))
    ref_sign = np.sign(np.linalg.det(np.concatenate([ones, X[T]], axis=2)))   # orientation of each grid simplex
    for _ in range(20):
        Xj = X.copy()
        Xj[interior] += rng.uniform(-jit * h, jit * h, size=(int(interior.sum()), dim))
        A = np.concatenate([ones, Xj[T]], axis=2)
        det = np.linalg.det(A)
        if np.all(np.sign(det) == ref_sign):          # no element inverted or degenerate
            break
    else:
        raise RuntimeError("could not jitter the grid without inverting an element")
    vol = np.abs(det) / (1.0 if dim == 1 else (2.0 if dim == 2 else 6.0))
    grads = np.linalg.inv(A)[:, 1:, :]                 # (E, dim, dim+1): gradient of each barycentric function
    kappa = np.exp(rng.standard_normal(T.shape[0]))
    Ke = (kappa * vol)[:, None, None] * (grads.transpose(0, 2, 1) @ grads)
    rows = np.repeat(T, dim + 1, axis=1).ravel()
    cols = np.tile(T, (1, dim + 1)).ravel()
    K = sp.coo_matrix((Ke.ravel(), (rows, cols)), shape=(n, n)).tocsr()
    lumped = np.bincount(T.ravel(), weights=np.repeat(vol / (dim + 1), dim + 1), minlength=n)
    K = (K + sp.diags(reaction_factor * kappa.mean() * lumped)).tocsr()
    K.sum_duplicates()
    K.sort_indices()
    b = rng.standard_normal((n, nrhs)) if nrhs > 1 else rng.standard_normal(n)
    return CsrSystem(K.indptr.astype(np.int32), K.indices.astype(np.int32), K.data.astype(np.float64), b, None,
                     f"fe{dim}d_n{n}", {"dim": dim, "m": m, "n": n, "seed": seed})


def fe_batch_specs(nsys: int = 512, n_lo: float = 1e3, n_hi: float = 2e5, seed: int = 1004):
    """(n_target, dim, seed) of each batch member: sizes log-uniform in [n_lo, n_hi], dimension 2 or 3 with
    probability 1/2 each, one seed per system."""
    rng = np.random.default_rng(seed)
    sizes = np.exp(rng.uniform(np.log(n_lo), np.log(n_hi), nsys))
    dims = rng.integers(2, 4, nsys)
    seeds = rng.integers(0, 2 ** 31 - 1, nsys)
    return [(int(sizes[k]), int(dims[k]), int(seeds[k])) for k in range(nsys)]


def _fe_from_spec(args):
    n, d, sd, nrhs = args
    return fe_p1_system(n, d, sd, nrhs=nrhs)


def fe_batch(nsys: int = 512, n_lo: float = 1e3, n_hi: float = 2e5, seed: int = 1004, nrhs: int = 8,
             workers: int = 1):
    """The batch members of fe_batch_specs, built in order (in `workers` processes when > 1)."""
    specs = [(n, d, sd, nrhs) for n, d, sd in fe_batch_specs(nsys, n_lo, n_hi, seed)]
    if workers <= 1:
        return [_fe_from_spec(a) for a in specs]
    from concurrent.futures import ProcessPoolExecutor
    with ProcessPoolExecutor(max_workers=workers) as ex:
        return list(ex.map(_fe_from_spec, specs, chunksize=4))


def serve_trace(nreq: int, seed: int = 1005, rate: float = 200.0, fe_pool: int | None = None, workers: int = 8):
    """Request trace of the serving workload: Poisson arrivals at `rate` per second; 70% P1
    finite-element systems drawn from the batch generator's distribution (sizes log-uniform in
    [1e3, 2e5], 2D or 3D, lognormal coefficients), each request its own independent draw (seed
    derived from `seed`; with `fe_pool` set, draws from the first `fe_pool` members of the batch
    instead); 30% 3D 7-point Dirichlet Laplacians with m ~ U{16..100} per side; one right-hand side
    each, N(0,1); tolerance 1e-6 or 1e-8 with probability 1/2 each."""
    from concurrent.futures import ProcessPoolExecutor
    rng = np.random.default_rng(seed)
    arr = np.cumsum(rng.exponential(1.0 / rate, nreq))
    kind = rng.random(nreq) < 0.7
    ms = rng.integers(16, 101, nreq)
    tols = np.where(rng.random(nreq) < 0.5, 1e-6, 1e-8)
    bseeds = rng.integers(0, 2 ** 31 - 1, nreq)
    if fe_pool is None:
        specs = fe_batch_specs(nreq, 1e3, 2e5, seed + 1)    # one independent system per request index
        fe_idx = np.arange(nreq)
    else:
        fe_idx = rng.integers(0, fe_pool, nreq)
        specs = fe_batch_specs(512, 1e3, 2e5, 1004)
    need = sorted(set(int(k) for k, f in zip(fe_idx, kind) if f))
    with ProcessPoolExecutor(max_workers=max(1, workers)) as ex:
        fe_sys = dict(zip(need, ex.map(_fe_from_spec, [(*specs[k], 1) for k in need], chunksize=2)))
    lap = {m: poisson_dirichlet((m, m, m)) for m in sorted(set(int(m) for m, f in zip(ms, kind) if not f))}
    reqs = []
    for i in range(nreq):
        r = np.random.default_rng(int(bseeds[i]))
        if kind[i]:
            s = fe_sys[int(fe_idx[i])]
            rowptr, colidx, vals = s.rowptr, s.colidx, s.vals
        else:
            rowptr, colidx, vals = lap[int(ms[i])]
        b = r.standard_normal(len(rowptr) - 1)
        reqs.append(dict(t=float(arr[i]), sys=CsrSystem(rowptr, colidx, vals, b), b=b, tol=float(tols[i]),
                         fe=bool(kind[i])))
    return reqs
