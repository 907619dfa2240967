"""QGGMRF prior with a depth-modulated scale (Sec. 2, "Prior model", Eqs. (14)-(17)).

    cost(x) = sum over cliques {s, r} of b_sr * rho(x_s - x_r)
    rho(D)  = |D|^p / (p sg^p) * u^(q-p) / (1 + u^(q-p)),   u = |D| / (T sg)
    sg      = sigma0 * sqrt(m_s m_r),
    m_s     = 1 + (m - 1) * (depth_s / max depth)^a.

Readings (the clique set and b_sr come from a cited work that is not part of
the paper): the cliques are the pairs of 8-neighbours, each unordered pair
counted once; b_sr is proportional to the inverse index distance and scaled so
that an interior voxel's eight weights sum to one (edge 1/(4 + 2 sqrt 2),
diagonal that over sqrt 2); missing neighbours at the border are dropped;
depth_s is the voxel-centre depth and the maximum depth the deepest centre.
The threshold T of Eq. (15) is called T_q in code that also handles travel
times.

For the separable surrogate the potential is bounded at the current difference
D' by the quadratic through rho(D') with the same slope (the symmetric bound of
QGGMRF): b_sr rho(D) <= B_sr D^2 + const, B_sr = b_sr * rho'(D') / (2 D').
"""
from __future__ import annotations

import numpy as np

B_EDGE = 1.0 / (4.0 + 2.0 * np.sqrt(2.0))
B_DIAG = B_EDGE / np.sqrt(2.0)
# (d_row, d_col) from s to r, one of each unordered neighbour pair
OFFSETS = ((0, 1, B_EDGE), (1, 0, B_EDGE), (1, -1, B_DIAG), (1, 1, B_DIAG))


def depth_modulation(grid, m: float, a: float) -> np.ndarray:
    """m_s of Eq. (17) for every row (voxel-centre depth / deepest centre depth)."""
    depth = grid.z0 + (np.arange(grid.nz) + 0.5) * grid.dz
    return 1.0 + (m - 1.0) * (depth / depth[-1]) ** a


def cliques(grid, prior):
    """All neighbour pairs: flat indices s, r, weight b_sr and scale sigma_g (Eq. (16))."""
    nz, nx = grid.nz, grid.nx
    ms = depth_modulation(grid, prior.m, prior.a)
    rows, cols = np.meshgrid(np.arange(nz), np.arange(nx), indexing="ij")
    S, R, Bw, Sg = [], [], [], []
    for dr, dc, bw in OFFSETS:
        r2, c2 = rows + dr, cols + dc
        ok = (r2 >= 0) & (r2 < nz) & (c2 >= 0) & (c2 < nx)
        s_idx = (rows * nx + cols)[ok]
        r_idx = (r2 * nx + c2)[ok]
        S.append(s_idx)
        R.append(r_idx)
        Bw.append(np.full(s_idx.shape, bw))
        Sg.append(prior.sigma0 * np.sqrt(ms[rows[ok]] * ms[r2[ok]]))
    return np.concatenate(S), np.concatenate(R), np.concatenate(Bw), np.concatenate(Sg)


def rho(delta, sg, prior):
    """Potential of Eq. (15)."""
    p, q, T = prior.p, prior.q, prior.T
    a = np.abs(delta)
    u = a / (T * sg)
    uq = u ** (q - p)
    return a ** p / (p * sg ** p) * uq / (1.0 + uq)


def rho_prime(delta, sg, prior):
    """d rho / d delta, written out from Eq. (15)."""
    p, q, T = prior.p, prior.q, prior.T
    a = np.abs(delta)
    u = a / (T * sg)
    uq = u ** (q - p)
    return np.sign(delta) * a ** (p - 1) / sg ** p * uq * (q / p + uq) / (1.0 + uq) ** 2


def half_curvature(delta, sg, prior):
    """rho'(delta) / (2 delta), finite at delta = 0 when q = 2.

    a^(p-2) u^(q-p) = a^(q-2) (T sg)^(p-q), so with q = 2 no factor is singular;
    the limit at delta -> 0 is 1 / (p sg^2 T^(2-p)).
    """
    p, q, T = prior.p, prior.q, prior.T
    a = np.abs(delta)
    u = a / (T * sg)
    uq = u ** (q - p)
    lead = a ** (q - 2.0) * (T * sg) ** (p - q) / (2.0 * sg ** p)
    return lead * (q / p + uq) / (1.0 + uq) ** 2


def cost(x, grid, prior) -> float:
    """Prior term of Eq. (18): sum over cliques of b_sr rho(x_s - x_r)."""
    xf = np.asarray(x, float).reshape(-1)
    s, r, bw, sg = cliques(grid, prior)
    return float(np.sum(bw * rho(xf[s] - xf[r], sg, prior)))


def gradient(x, grid, prior) -> np.ndarray:
    """Gradient of the prior term, image-shaped."""
    xf = np.asarray(x, float).reshape(-1)
    s, r, bw, sg = cliques(grid, prior)
    d = bw * rho_prime(xf[s] - xf[r], sg, prior)
    n = xf.size
    gr = np.bincount(s, weights=d, minlength=n) - np.bincount(r, weights=d, minlength=n)
    return gr.reshape(np.shape(x))


def surrogate(x, grid, prior):
    """Per-voxel (slope, curvature) of the separable prior surrogate at x.

    With B_sr = b_sr rho'(D)/(2D) at D = x_s - x_r, the pair term is bounded by
    B_sr (x_s - x_r)^2 and, splitting it between both voxels,
    by 2 B_sr ((x_s - (x_s' + x_r')/2)^2 + (x_r - (x_s' + x_r')/2)^2).
    Voxel s then gets slope sum_r 2 B_sr (x_s - x_r) and curvature sum_r 4 B_sr.
    """
    xf = np.asarray(x, float).reshape(-1)
    s, r, bw, sg = cliques(grid, prior)
    delta = xf[s] - xf[r]
    Bsr = bw * half_curvature(delta, sg, prior)
    n = xf.size
    slope = (np.bincount(s, weights=2 * Bsr * delta, minlength=n)
             - np.bincount(r, weights=2 * Bsr * delta, minlength=n))
    curv = np.bincount(s, weights=4 * Bsr, minlength=n) + np.bincount(r, weights=4 * Bsr, minlength=n)
    return slope.reshape(np.shape(x)), curv.reshape(np.shape(x))


def icd_terms(x, grid, prior, v: int):
    """Slope and curvature of the one-voxel prior surrogate at voxel v.

    With the neighbours held fixed the pair term of voxel v is bounded by
    B_sr (x_v - x_r)^2: slope sum_r 2 B_sr (x_v - x_r), curvature sum_r 2 B_sr.
    """
    nz, nx = grid.nz, grid.nx
    ms = depth_modulation(grid, prior.m, prior.a)
    xf = np.asarray(x, float).reshape(-1)
    rv, cv = divmod(v, nx)
    slope = 0.0
    curv = 0.0
    for dr, dc, bw in OFFSETS:
        for sgn in (1, -1):
            r2, c2 = rv + sgn * dr, cv + sgn * dc
            if 0 <= r2 < nz and 0 <= c2 < nx:
                sg = prior.sigma0 * np.sqrt(ms[rv] * ms[r2])
                delta = xf[v] - xf[r2 * nx + c2]
                B = bw * half_curvature(delta, sg, prior)
                slope += 2 * B * delta
                curv += 2 * B
    return slope, curv
