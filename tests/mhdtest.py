"""Small numpy helpers shared by the tests (assembly of global arrays from patches,
discrete divergence of the face field, conserved sums, linear-wave initial data)."""
from __future__ import annotations

import math

import numpy as np

import refmath as rm
from paper_2508_09568_amd import workloads as W


def global_interior(U, L, grid):
    """Owned cells/faces of a regular patch grid as one (8, Z, Y, X) array."""
    Px, Py, Pz = grid
    n = L.dims[0]
    nz, ny, nx = int(n[2]), int(n[1]), int(n[0])
    G = np.zeros((8, Pz * nz, Py * ny, Px * nx))
    for pz in range(Pz):
        for py in range(Py):
            for px in range(Px):
                p = px + Px * (py + Py * pz)
                G[:, pz * nz:(pz + 1) * nz, py * ny:(py + 1) * ny, px * nx:(px + 1) * nx] = \
                    L.interior(U, p)
    return G


def div_b(U, L, dx):
    """Discrete divergence of the face field per interior cell (guards must be filled):
    sum_d (B_d[c + e_d] - B_d[c]) / dx_d over active directions."""
    out = []
    g = L.g
    for p in range(L.P):
        V = L.view(U, p)
        n = L.dims[p]
        sl = [slice(g, g + int(n[d])) if n[d] > 1 else slice(0, 1) for d in range(3)]
        s = np.zeros(tuple(int(n[d]) for d in (2, 1, 0)))
        for d in range(3):
            if n[d] <= 1:
                continue
            up = list(sl)
            up[d] = slice(g + 1, g + 1 + int(n[d]))
            B = V[5 + d]
            s += (B[up[2], up[1], up[0]] - B[sl[2], sl[1], sl[0]]) / dx[p][d]
        out.append(s)
    return out


def sums(U, L):
    """Interior sums of the 8 fields (pairwise numpy summation)."""
    return np.array([sum(L.interior(U, p)[m].sum() for p in range(L.P)) for m in range(8)])


def linear_wave_1d(N, family, amp=1e-6, gamma=5.0 / 3.0, g=3):
    """1D periodic linear MHD wave of one family ('fast'/'alfven'/'slow' right-going,
    'entropy' on a background flow u0 = 1): q = q0 + amp r sin(2 pi x), r a right
    eigenvector of the primitive Jacobian from numpy.linalg.eig."""
    u0 = 1.0 if family == "entropy" else 0.0
    q0 = np.array([1.0, u0, 0.0, 0.0, 1.0 / gamma, 1.0, math.sqrt(2.0), 0.5])
    lam, R = rm.wave_eigensystem(q0, gamma)
    idx = {"fast": 6, "alfven": 5, "slow": 4, "entropy": 3}[family]
    r7 = R[:, idx]
    r = np.array([r7[0], r7[1], r7[2], r7[3], r7[4], 0.0, r7[5], r7[6]])
    r /= np.abs(r).max()
    L = W.Layout([[N, 1, 1]], g)
    U = np.zeros(L.total)
    V = L.view(U, 0)
    x = (np.arange(N + 2 * g) - g + 0.5) / N
    s = np.sin(2 * math.pi * x)
    for i in range(N + 2 * g):
        q = q0 + amp * r * s[i]
        V[:, 0, 0, i] = rm.prim_to_cons(q, gamma)
    nbr = W.grid_neighbours((1, 1, 1), (True, True, True))
    period = 1.0 / abs(lam[idx])
    return L, U, np.array([[1.0 / N, 1.0, 1.0]]), nbr, period


def linear_wave_2d(N, family="fast", amp=1e-6, gamma=5.0 / 3.0, g=3, patches=2):
    """Same wave travelling along the grid diagonal of the periodic unit square
    (wavelength 1/sqrt 2); the in-plane face field comes from a vector potential so the
    discrete divergence vanishes."""
    u0 = 1.0 if family == "entropy" else 0.0
    qn = np.array([1.0, u0, 0.0, 0.0, 1.0 / gamma, 1.0, math.sqrt(2.0), 0.5])
    lam, R = rm.wave_eigensystem(qn, gamma)
    idx = {"fast": 6, "alfven": 5, "slow": 4, "entropy": 3}[family]
    r7 = R[:, idx]
    r = np.array([r7[0], r7[1], r7[2], r7[3], r7[4], 0.0, r7[5], r7[6]])
    r /= np.abs(r).max()
    nx_, ny_ = 1 / math.sqrt(2), 1 / math.sqrt(2)
    k = 2 * math.pi * math.sqrt(2)            # along s = n.x

    def prim(x, y):
        s = nx_ * x + ny_ * y
        ex = (slice(None),) + (None,) * np.ndim(s)
        q = qn[ex] + amp * r[ex] * np.sin(k * s)[None]
        # rotate (n, t, z) -> (x, y, z) for velocity and field
        rho, un, ut, w, p, bn, bt, bz = q
        return np.array([rho, un * nx_ - ut * ny_, un * ny_ + ut * nx_, w, p,
                         bn * nx_ - bt * ny_, bn * ny_ + bt * nx_, bz])

    def Az(x, y):
        s = nx_ * x + ny_ * y
        bn, bt0, rb = qn[5], qn[6], r[6]
        return bn * (nx_ * y - ny_ * x) - bt0 * s + amp * rb * np.cos(k * s) / k

    m = N // patches
    L = W.Layout(np.tile([m, m, 1], (patches * patches, 1)), g)
    U = np.zeros(L.total)
    h = 1.0 / N
    for py in range(patches):
        for px in range(patches):
            V = L.view(U, px + patches * py)
            i = np.arange(m + 2 * g) - g
            xc = (px * m + i + 0.5) * h
            yc = (py * m + i + 0.5) * h
            YY, XX = np.meshgrid(yc, xc, indexing="ij")
            q = prim(XX, YY)
            V[:, 0] = rm.prim_to_cons(q, gamma)
            xl, yl = XX - 0.5 * h, YY - 0.5 * h    # lower faces
            V[5, 0] = (Az(xl, YY + 0.5 * h) - Az(xl, YY - 0.5 * h)) / h
            V[6, 0] = -(Az(XX + 0.5 * h, yl) - Az(XX - 0.5 * h, yl)) / h
    nbr = W.grid_neighbours((patches, patches, 1), (True, True, True))
    dx = np.tile([h, h, 1.0], (L.P, 1))
    period = (1 / math.sqrt(2)) / abs(lam[idx])
    return L, U, dx, nbr, period


def cyclic_permute(U, L, dx, grid, times=1):
    """Map a problem on a regular patch grid under the axis cycle x -> y -> z -> x
    (components and face fields are renamed, dims, spacings and the patch grid
    rotate).  Returns (U, layout, dx, grid)."""
    for _ in range(times):
        Px, Py, Pz = grid
        ngrid = (Pz, Px, Py)
        dims = L.dims[:, [2, 0, 1]]
        L2 = W.Layout(dims, L.g)
        out = np.empty_like(U)
        dx2 = np.empty_like(dx)
        for pz in range(Pz):
            for py in range(Py):
                for px in range(Px):
                    p = px + Px * (py + Py * pz)
                    q = pz + ngrid[0] * (px + ngrid[1] * py)
                    V = L.view(U, p)
                    V2 = L2.view(out, q)
                    # new (z', y', x') indices = old (y, x, z)
                    for m_new, m_old in ((0, 0), (1, 3), (2, 1), (3, 2), (4, 4), (5, 7),
                                         (6, 5), (7, 6)):
                        V2[m_new] = np.transpose(V[m_old], (1, 2, 0))
                    dx2[q] = dx[p][[2, 0, 1]]
        U, L, dx, grid = out, L2, dx2, ngrid
    return U, L, dx, grid
