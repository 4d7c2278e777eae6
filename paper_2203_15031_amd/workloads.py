"""Seeded synthetic workloads for SPMESL.

This module only draws data: a population precision matrix Omega with a
given graph structure and n Gaussian samples X ~ N(0, Omega^{-1}).  It holds
none of the estimator's arithmetic, so both the HIP path and the CPU oracle
take their inputs from here.

Every generator is deterministic in its seed (numpy PCG64 via
``np.random.default_rng``).  X is returned row-major, shape (n, p), float64.

Structures
----------
* ``ar_cov``        Sigma_ij = rho^|i-j| (a tridiagonal precision matrix).
* ``block_ar_cov``  block-diagonal with AR(1) covariance blocks.
* ``erdos_renyi``   random graph, edge probability q, weights +-U[a, b],
                    diagonal shifted to a minimum eigenvalue, unit variance.
* ``hub``           consecutive groups; the first node of a group is a hub
                    joined to the rest with one positive weight.
* ``scale_free_tree`` Barabasi-Albert tree (m = 1), weights +-U[a, b],
                    diagonally dominant precision; sampled through its
                    fill-free Cholesky factor (leaves first).
* The four networks of the paper's simulation study (Section 4.1): AR(1)
  with 0.48 off-diagonals, AR(4) with 0.6^|i-j|, and scale-free and hub
  networks built from subnetworks of 100 nodes.

The named workloads (``WORKLOADS``) are the ones the tests and the
benchmark use; their penalty is lambda0 = sqrt(2 log p / n) (one states its
own) and their tolerance 1e-8.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

__all__ = [
    "Workload", "WORKLOADS", "workload", "generate", "generate_batch",
    "ar_cov", "block_ar_cov", "erdos_renyi_precision", "hub_precision",
    "sample_from_cov", "sample_from_precision", "scale_free_tree_sample",
    "paper_network", "orthogonal_pairs_design", "exact_covariance_design", "star_band_design",
    "sparse_regression",
]


def _rng(seed):
    return np.random.default_rng(seed)


# --------------------------------------------------------------------------
# covariance / precision builders
# --------------------------------------------------------------------------

def ar_cov(p: int, rho: float) -> np.ndarray:
    """Sigma_ij = rho^|i-j| (p x p)."""
    idx = np.arange(p)
    return rho ** np.abs(idx[:, None] - idx[None, :])


def block_ar_cov(nblocks: int, bsize: int, rho: float) -> list[np.ndarray]:
    """The diagonal blocks of a block-diagonal AR(1) covariance."""
    return [ar_cov(bsize, rho) for _ in range(nblocks)]


def erdos_renyi_precision(p: int, q: float, wlo: float, whi: float,
                          min_eig: float, rng) -> np.ndarray:
    """Erdos-Renyi precision matrix.

    Edges on i<j with probability q, weights of random sign and magnitude
    U[wlo, whi]; the diagonal is shifted so that the smallest eigenvalue is
    ``min_eig``; finally Omega <- D^{-1} Omega D^{-1} with D = diag(Omega^{-1})^{-1/2}
    so that the implied covariance has a unit diagonal.
    """
    mask = np.triu(rng.random((p, p)) < q, 1)
    w = rng.uniform(wlo, whi, size=(p, p)) * rng.choice([-1.0, 1.0], size=(p, p))
    A = np.where(mask, w, 0.0)
    A = A + A.T
    lam_min = np.linalg.eigvalsh(A)[0]
    Om = A + (min_eig - lam_min) * np.eye(p)
    return _unit_variance(Om)


def _unit_variance(Om: np.ndarray) -> np.ndarray:
    Sig = np.linalg.inv(Om)
    d = np.sqrt(np.diag(Sig))
    return Om * d[:, None] * d[None, :]


def hub_precision(p: int, group: int, weight: float, min_eig: float):
    """Hub precision matrix as a list of diagonal blocks.

    Nodes are cut into consecutive groups of ``group`` (the last may be
    shorter); node 0 of a group is the hub, joined to every other member
    with ``weight``.  Omega = weight*A + (|lambda_min(weight*A)| + min_eig) I,
    then rescaled to unit variance.  Returns the list of blocks.
    """
    blocks = []
    start = 0
    while start < p:
        m = min(group, p - start)
        A = np.zeros((m, m))
        A[0, 1:] = weight
        A[1:, 0] = weight
        if m > 1:
            lam_min = np.linalg.eigvalsh(A)[0]
        else:
            lam_min = 0.0
        Om = A + (abs(lam_min) + min_eig) * np.eye(m)
        blocks.append(_unit_variance(Om))
        start += m
    return blocks


# --------------------------------------------------------------------------
# samplers
# --------------------------------------------------------------------------

def sample_from_cov(n: int, Sigma_blocks, rng, centre: bool = True) -> np.ndarray:
    """X ~ N(0, blockdiag(Sigma_blocks)) with X = Z L^T, Sigma = L L^T."""
    if isinstance(Sigma_blocks, np.ndarray):
        Sigma_blocks = [Sigma_blocks]
    p = sum(b.shape[0] for b in Sigma_blocks)
    Z = rng.standard_normal((n, p))
    X = np.empty((n, p))
    s = 0
    for b in Sigma_blocks:
        m = b.shape[0]
        L = np.linalg.cholesky(b)
        X[:, s:s + m] = Z[:, s:s + m] @ L.T
        s += m
    if centre:
        X -= X.mean(axis=0, keepdims=True)
    return X


def sample_from_precision(n: int, Omega_blocks, rng, centre: bool = False) -> np.ndarray:
    """X ~ N(0, Omega^{-1}) with Omega = L L^T: X = Z L^{-1} (rows x = L^{-T} z)."""
    import scipy.linalg as sla
    if isinstance(Omega_blocks, np.ndarray):
        Omega_blocks = [Omega_blocks]
    p = sum(b.shape[0] for b in Omega_blocks)
    Z = rng.standard_normal((n, p))
    X = np.empty((n, p))
    s = 0
    for b in Omega_blocks:
        m = b.shape[0]
        L = np.linalg.cholesky(b)
        # rows: L^T x = z  ->  X^T = L^{-T} Z^T
        X[:, s:s + m] = sla.solve_triangular(L, Z[:, s:s + m].T, lower=True, trans="T").T
        s += m
    if centre:
        X -= X.mean(axis=0, keepdims=True)
    return X


def scale_free_tree_sample(n: int, p: int, wlo: float, whi: float, diag_add: float,
                           rng, unit_variance: bool = True):
    """Barabasi-Albert tree (m = 1) precision, sampled without forming it densely.

    Node t >= 2 attaches to one earlier node chosen with probability
    proportional to its degree (nodes 0 and 1 start joined).  Edge weights
    have random sign and magnitude U[wlo, whi]; omega_ii = sum_j |omega_ij| +
    diag_add.  With parents always earlier than children, the Cholesky factor
    of Omega in leaves-first (reverse) order has no fill, so sampling and the
    unit-variance rescale are O(n p).

    Returns (X, parent, weight, diag): the tree and the precision entries
    before the unit-variance rescale, which scales column i of X by
    1/sqrt(Sigma_ii).
    """
    parent = np.full(p, -1, dtype=np.int64)
    # degree-proportional choice via the repeated-endpoint list
    ends = np.empty(2 * p, dtype=np.int64)
    ne = 0
    if p >= 2:
        parent[1] = 0
        ends[0], ends[1] = 0, 1
        ne = 2
    u = rng.random(p)
    for t in range(2, p):
        j = ends[int(u[t] * ne)]
        parent[t] = j
        ends[ne] = j
        ends[ne + 1] = t
        ne += 2
    w = rng.uniform(wlo, whi, size=p) * rng.choice([-1.0, 1.0], size=p)
    w[0] = 0.0
    absum = np.zeros(p)
    for t in range(1, p):
        absum[t] += abs(w[t])
        absum[parent[t]] += abs(w[t])
    diag = absum + diag_add
    # Cholesky Omega = L L^T eliminating t = p-1 .. 0 (children first).
    Ldiag = np.zeros(p)
    Lpar = np.zeros(p)          # L[parent[t], t]
    dd = diag.copy()
    for t in range(p - 1, -1, -1):
        Ldiag[t] = math.sqrt(dd[t])
        if parent[t] >= 0:
            Lpar[t] = w[t] / Ldiag[t]
            dd[parent[t]] -= Lpar[t] ** 2
    # x = L^{-T} z: row t of L^T x = z is L_tt x_t + L[par,t] x_par = z_t,
    # solved root first (parents have smaller indices).
    Z = rng.standard_normal((n, p))
    X = np.empty((n, p))
    for t in range(p):
        if parent[t] >= 0:
            X[:, t] = (Z[:, t] - Lpar[t] * X[:, parent[t]]) / Ldiag[t]
        else:
            X[:, t] = Z[:, t] / Ldiag[t]
    if unit_variance:
        # Sigma_tt = ||L^{-1} e_t||^2; L^{-1} e_t lives on the path t -> root.
        var = np.empty(p)
        for t in range(p):
            y = 1.0 / Ldiag[t]
            acc = y * y
            v = t
            while parent[v] >= 0:
                m = parent[v]
                y = -Lpar[v] * y / Ldiag[m]
                acc += y * y
                v = m
            var[t] = acc
        X /= np.sqrt(var)[None, :]
    return X, parent, w, diag


def paper_network(kind: str, p: int, rng) -> np.ndarray:
    """The precision matrices of the paper's simulation study (Section 4.1).

    kind: "ar1" (omega_ii = 1, omega_{i,i+-1} = 0.48), "ar4"
    (0.6^|i-j| for |i-j| <= 4), "sf" (a growing random tree, each new node
    attached to an earlier one chosen uniformly) or "hub" (10 hubs per 100
    nodes, each non-hub joined to 1-3 of them).  "sf" and "hub" are built as
    p/100 subnetworks of 100 nodes with off-diagonal magnitudes raised to at
    least 0.1, through the steps: U([-1,-0.5] U [0.5,1]) weights, row
    division by 1.5 x the row's absolute sum, symmetrisation, unit diagonal.
    Those steps give a positive definite matrix for the scale-free trees
    drawn here (nodes of small degree); the hub subnetworks are not positive
    definite after them, and their diagonal is raised until the smallest
    eigenvalue is 0.1 (the same guard would apply to a scale-free draw).
    """
    if kind == "ar1":
        Om = np.eye(p)
        i = np.arange(p - 1)
        Om[i, i + 1] = Om[i + 1, i] = 0.48
        return Om
    if kind == "ar4":
        idx = np.arange(p)
        d = np.abs(idx[:, None] - idx[None, :])
        return np.where(d <= 4, 0.6 ** d, 0.0)
    if kind not in ("sf", "hub"):
        raise ValueError(kind)
    if p % 100:
        raise ValueError("p must be a multiple of 100 for the subnetwork networks")
    Om = np.zeros((p, p))
    for s in range(0, p, 100):
        E = _tree_edges(100, rng) if kind == "sf" else _hub_edges(100, rng)
        T = subnetwork_precision(E, 100, rng)
        # not positive definite when a node has many neighbours of small
        # degree (a hub row sums to about 5): raise the diagonal until the
        # smallest eigenvalue is 0.1
        ev = np.linalg.eigvalsh(T).min()
        if ev < 0.1:
            T += (0.1 - ev) * np.eye(100)
        Om[s:s + 100, s:s + 100] = T
    return Om


def subnetwork_precision(edges, m: int, rng) -> np.ndarray:
    """Steps (i)-(iv) of Section 4.1 on one subnetwork, then the floor of 0.1
    on the nonzero off-diagonal magnitudes."""
    T = np.eye(m)
    for (a, b) in edges:
        mag = rng.uniform(0.5, 1.0)
        T[a, b] = T[b, a] = mag * rng.choice([-1.0, 1.0])
    off = T - np.diag(np.diag(T))
    rs = 1.5 * np.abs(off).sum(axis=1)
    rs[rs == 0] = 1.0
    T = off / rs[:, None]
    T = (T + T.T) / 2
    small = (T != 0) & (np.abs(T) < 0.1)
    T[small] = np.sign(T[small]) * 0.1
    np.fill_diagonal(T, 1.0)
    return T


def _tree_edges(m_nodes: int, rng, power: float = 0.0):
    # growing tree from one edge: node t attaches to an earlier node j with
    # probability proportional to degree(j)^power (0: uniform; 1: the linear
    # preferential attachment of the Barabasi-Albert model)
    edges = [(0, 1)]
    deg = np.zeros(m_nodes)
    deg[0] = deg[1] = 1
    for t in range(2, m_nodes):
        w = deg[:t] ** power
        j = rng.choice(t, p=w / w.sum())
        edges.append((j, t))
        deg[j] += 1
        deg[t] += 1
    return edges


def _hub_edges(m_nodes: int, rng):
    hubs = rng.choice(m_nodes, size=10, replace=False)
    others = np.setdiff1d(np.arange(m_nodes), hubs)
    edges = set()
    # each non-hub joins 1-3 hubs, one with probability 0.8, two with 0.18,
    # three with 0.02 (mean 1.22): about 110 edges per 100 nodes, the edge
    # count the paper's hub networks have at p = 500 (551); hubs then average
    # degree 11
    for v in others:
        k = int(rng.choice(3, p=[0.8, 0.18, 0.02])) + 1
        for h in rng.choice(hubs, size=k, replace=False):
            edges.add((min(h, v), max(h, v)))
    return sorted(edges)


def orthogonal_pairs_design(n: int, rs, rng) -> np.ndarray:
    """X whose sample correlation is block-diagonal with 2x2 blocks [[1,r],[r,1]].

    Column pairs (2i, 2i+1) have exact sample correlation rs[i] and distinct
    pairs are exactly uncorrelated (columns from an orthonormal basis of the
    centred space).  Requires n > 2 len(rs).
    """
    m = len(rs)
    p = 2 * m
    if n <= p:
        raise ValueError("need n > p")
    Z = rng.standard_normal((n, p))
    Z -= Z.mean(axis=0, keepdims=True)
    Q, _ = np.linalg.qr(Z)
    X = np.empty((n, p))
    for i, r in enumerate(rs):
        q1, q2 = Q[:, 2 * i], Q[:, 2 * i + 1]
        X[:, 2 * i] = q1 * math.sqrt(n)
        X[:, 2 * i + 1] = (r * q1 + math.sqrt(1 - r * r) * q2) * math.sqrt(n)
    return X


def exact_covariance_design(n: int, S: np.ndarray, rng) -> np.ndarray:
    """X (n x p) with centred columns whose sample covariance X^T X / n is S exactly.

    S must be symmetric positive definite.  X = sqrt(n) Q L^T with S = L L^T
    and Q an orthonormal basis of n-vectors orthogonal to the all-ones
    vector (so the columns are centred).  Requires n > p.
    """
    p = S.shape[0]
    if n <= p:
        raise ValueError("need n > p")
    Z = rng.standard_normal((n, p))
    Z -= Z.mean(axis=0, keepdims=True)
    Q, _ = np.linalg.qr(Z)
    L = np.linalg.cholesky(S)
    return math.sqrt(n) * (Q @ L.T)


def star_band_design(n: int = 200, arms: int = 40, lambda0: float = 0.15, gap: float = 3e-5,
                     pairs=(0.6, -0.5, 0.7, 0.4, -0.65), seed: int = 6) -> np.ndarray:
    """A design whose first variable has `arms` exactly uncorrelated partners,
    each at sample correlation lambda0 - gap, followed by independent pairs
    with the given correlations.

    At penalty lambda0 the first column's regression stays at beta = 0 and
    sigma = 1, with all `arms` gradients |s_j1| = lambda0 - gap just below its
    threshold.  Requires arms (lambda0 - gap)^2 < 1 (positive definite).
    """
    r = lambda0 - gap
    m = 1 + arms
    p = m + 2 * len(pairs)
    S = np.eye(p)
    S[0, 1:m] = r
    S[1:m, 0] = r
    for i, c in enumerate(pairs):
        a = m + 2 * i
        S[a, a + 1] = S[a + 1, a] = c
    return exact_covariance_design(n, S, _rng(seed))


# --------------------------------------------------------------------------
# the named workloads
# --------------------------------------------------------------------------

def sparse_regression(n: int = 250, p: int = 500, sigmas=(3.0, 5.0), seed: int = 5):
    """The regression example of Section 3 (the one behind Fig. 2): y = X beta
    + sigma eps with beta = (2 x 5, -1 x 5, 0 x (p - 10)), eps ~ N(0, I), one
    response per noise level sigma, all on one design.  The paper does not
    say how X is drawn; here its entries are iid N(0, 1).

    Returns X (n x p), Y (n x len(sigmas)) and beta (p)."""
    rng = _rng(seed)
    beta = np.zeros(p)
    beta[:5] = 2.0
    beta[5:10] = -1.0
    X = rng.standard_normal((n, p))
    E = rng.standard_normal((n, len(sigmas)))
    Y = (X @ beta)[:, None] + E * np.asarray(sigmas, dtype=np.float64)[None, :]
    return X, np.ascontiguousarray(Y), beta


@dataclass(frozen=True)
class Workload:
    name: str
    n: int
    p: int
    seed: int
    structure: str
    tol: float = 1e-8
    batch: int = 1
    extra: dict = field(default_factory=dict)

    @property
    def lambda0(self) -> float:
        """sqrt(2 log p / n), the penalty the workload is specified with
        (unless it states its own)."""
        if "lambda0" in self.extra:
            return float(self.extra["lambda0"])
        return math.sqrt(2.0 * math.log(self.p) / self.n)


WORKLOADS = {
    "ar1_n100_p200": Workload("ar1_n100_p200", 100, 200, 0, "ar_cov(0.5), centred"),
    "er_n200_p1000": Workload("er_n200_p1000", 200, 1000, 1,
                              "ER(0.01), +-U[0.25,0.5], min eig 0.1, unit variance"),
    "blockar_n400_p5000": Workload("blockar_n400_p5000", 400, 5000, 2,
                                   "50 blocks of 100, AR(1) rho=0.6 covariance"),
    "hub_batch64": Workload("hub_batch64", 0, 0, 3,
                            "64 datasets, p~U{256..4096}, n=ceil(p/2), hubs of 20, weight 0.3",
                            batch=64),
    "sf_n1000_p20000": Workload("sf_n1000_p20000", 1000, 20000, 4,
                                "Barabasi-Albert tree, +-U[0.2,0.4], diag dominant + 0.1"),
    # every column's support has 130-190 coordinates at this small penalty:
    # the case of working sets beyond the 128 an LDS tier holds
    "dense_n1500_p300": Workload("dense_n1500_p300", 1500, 300, 9, "ar_cov(0.3), centred, lambda0 = 0.015",
                                 extra={"lambda0": 0.015}),
}


def workload(name: str) -> Workload:
    return WORKLOADS[name]


def generate(name: str, n: int | None = None, p: int | None = None) -> np.ndarray:
    """Draw X (n x p, row-major float64) for a named workload.

    n and p default to the workload's; passing smaller values draws the same
    structure at a reduced size (tests use this for quick cases).
    """
    w = WORKLOADS[name]
    n = w.n if n is None else n
    p = w.p if p is None else p
    rng = _rng(w.seed)
    if name == "ar1_n100_p200":
        return sample_from_cov(n, ar_cov(p, 0.5), rng, centre=True)
    if name == "er_n200_p1000":
        Om = erdos_renyi_precision(p, 0.01, 0.25, 0.5, 0.1, rng)
        return sample_from_precision(n, Om, rng)
    if name == "blockar_n400_p5000":
        bs = 100 if p >= 100 else p
        nb = p // bs
        blocks = block_ar_cov(nb, bs, 0.6)
        if nb * bs < p:
            blocks.append(ar_cov(p - nb * bs, 0.6))
        return sample_from_cov(n, blocks, rng, centre=False)
    if name == "sf_n1000_p20000":
        X, *_ = scale_free_tree_sample(n, p, 0.2, 0.4, 0.1, rng)
        return X
    if name == "dense_n1500_p300":
        return sample_from_cov(n, ar_cov(p, 0.3), rng, centre=True)
    raise ValueError(f"{name} is a batch workload; use generate_batch")


def generate_replicas(name: str, count: int) -> list[np.ndarray]:
    """`count` independent data sets of a named single-set workload: the
    workload's own X first, then draws of the same structure and size from
    seeds spawned from the workload's seed."""
    w = WORKLOADS[name]
    out = [generate(name)]
    for ss in np.random.SeedSequence(w.seed).spawn(count - 1):
        rng = np.random.default_rng(ss)
        if name == "blockar_n400_p5000":
            out.append(sample_from_cov(w.n, block_ar_cov(w.p // 100, 100, 0.6), rng, centre=False))
        else:
            raise ValueError(f"no replicas defined for {name}")
    return out


def batch_shapes(count: int = 64, seed: int = 3, pmin: int = 256, pmax: int = 4096):
    """(n_i, p_i) of the batched hub workload: p ~ U{pmin..pmax}, n = ceil(p/2)."""
    rng = _rng(seed)
    ps = rng.integers(pmin, pmax + 1, size=count)
    return [(int(math.ceil(pi / 2)), int(pi)) for pi in ps]


def generate_batch(count: int = 64, seed: int = 3, pmin: int = 256, pmax: int = 4096):
    """The batched hub workload: a list of X_i (n_i x p_i)."""
    shapes = batch_shapes(count, seed, pmin, pmax)
    children = np.random.SeedSequence(seed).spawn(count)
    out = []
    for (n, p), ss in zip(shapes, children):
        rng = np.random.default_rng(ss)
        blocks = hub_precision(p, 20, 0.3, 0.1)
        out.append(sample_from_precision(n, blocks, rng))
    return out
