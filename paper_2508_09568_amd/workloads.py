"""Seeded synthetic inputs for the MHD bunch update.

Shared by the tests, the smoke check and the benchmark.  The module holds no
arithmetic of the update itself: it lays out patches (padded boxes with guard zones,
field-major, x fastest), builds neighbour tables and evaluates initial conditions,
turning primitive fields into the conserved state through the definition of total
energy E = p/(gamma-1) + rho|u|^2/2 + |B|^2/2 (code units, mu_0 = 1).

Problems (sizes and parameters as the paper's validation and performance sections
describe them; the turbulence initial field is this project's own seeded recipe
because the paper does not give one):
  sod            -- 1D shock tube, outflow, gamma 1.4
  orszag_tang    -- 2D periodic vortex on 8x8 patches of 32^2, gamma 5/3
  turbulence     -- 3D periodic supersonic velocity field, 16^3 patches of 32^3
  uneven         -- 3600 patches of 16^3..48^3 sampling the turbulence field
  adjoint_case   -- 64^3 periodic, linear fast wave + seeded noise
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

RHO, MX, MY, MZ, EN, BX, BY, BZ = range(8)


# ----------------------------------------------------------------------------- layout

@dataclass
class Layout:
    """Patch table of a bunch: interior dims per patch, guard width, element offsets."""
    dims: np.ndarray          # (P, 3) int32, 1 = collapsed direction
    g: int

    def __post_init__(self):
        self.dims = np.ascontiguousarray(np.asarray(self.dims, dtype=np.int32).reshape(-1, 3))

    @property
    def P(self) -> int:
        return int(self.dims.shape[0])

    @property
    def N(self) -> np.ndarray:
        return np.where(self.dims > 1, self.dims + 2 * self.g, 1).astype(np.int64)

    @property
    def Nc(self) -> np.ndarray:
        N = self.N
        return N[:, 0] * N[:, 1] * N[:, 2]

    @property
    def base(self) -> np.ndarray:
        """Element offset of each patch (and the total at the end)."""
        return np.concatenate([[0], np.cumsum(8 * self.Nc)]).astype(np.int64)

    @property
    def total(self) -> int:
        return int(self.base[-1])

    @property
    def interior_cells(self) -> int:
        return int(np.prod(self.dims.astype(np.int64), axis=1).sum())

    def view(self, U, p):
        """(8, Nz, Ny, Nx) view of patch p of the flat array U."""
        b = self.base
        Nx, Ny, Nz = (int(v) for v in self.N[p])
        return U[b[p]:b[p + 1]].reshape(8, Nz, Ny, Nx)

    def interior(self, U, p):
        """(8, nz, ny, nx) view of the owned cells/faces of patch p."""
        V = self.view(U, p)
        g = self.g
        sl = []
        for d in (2, 1, 0):
            sl.append(slice(g, g + int(self.dims[p, d])) if self.dims[p, d] > 1 else slice(0, 1))
        return V[:, sl[0], sl[1], sl[2]]


def grid_neighbours(grid, periodic):
    """27-entry neighbour table for a regular grid of patches, patch id =
    ix + Px*(iy + Py*iz); entry (ox+1)+3(oy+1)+9(oz+1); -1 marks a domain boundary."""
    Px, Py, Pz = grid
    ids = np.arange(Px * Py * Pz, dtype=np.int32).reshape(Pz, Py, Px)
    nbr = np.full((Px * Py * Pz, 27), -1, dtype=np.int32)
    for iz in range(Pz):
        for iy in range(Py):
            for ix in range(Px):
                p = ids[iz, iy, ix]
                for oz in (-1, 0, 1):
                    for oy in (-1, 0, 1):
                        for ox in (-1, 0, 1):
                            c, ok = [], True
                            for i, o, n, per in ((ix, ox, Px, periodic[0]), (iy, oy, Py, periodic[1]),
                                                 (iz, oz, Pz, periodic[2])):
                                j = i + o
                                if j < 0 or j >= n:
                                    if per:
                                        j %= n
                                    else:
                                        ok = False
                                c.append(j)
                            if ok:
                                nbr[p, (ox + 1) + 3 * (oy + 1) + 9 * (oz + 1)] = ids[c[2], c[1], c[0]]
    return nbr


@dataclass
class Workload:
    name: str
    layout: Layout
    U: np.ndarray             # flat float64 state, guards filled
    dx: np.ndarray            # (P, 3) cell sizes
    gamma: float
    nbr: np.ndarray | None = None   # (P, 27) or None (guards frozen)
    cfl: float = 0.4
    t_end: float | None = None
    nsteps: int | None = None
    meta: dict = field(default_factory=dict)


def _conserved(rho, u, v, w, p, bcx, bcy, bcz, gamma):
    """Total energy from primitive fields (energy relation of the paper's §2.1)."""
    return (p / (gamma - 1.0) + 0.5 * rho * (u * u + v * v + w * w)
            + 0.5 * (bcx * bcx + bcy * bcy + bcz * bcz))


def _centres(origin, i0, n, h):
    """Cell-centre coordinates origin + (i - g + 1/2) h for padded indices i0."""
    return origin + (i0 + 0.5) * h


# ------------------------------------------------------------------------- problems

def sod(n=128, patches=1, g=3, gamma=1.4):
    """Sod shock tube on [0,1]: (rho, p) = (1, 1) for x < 1/2, (0.125, 0.1) beyond;
    u = B = 0; zero-gradient outflow at both ends; t_end = 0.2."""
    assert n % patches == 0
    m = n // patches
    L = Layout(np.tile([m, 1, 1], (patches, 1)), g)
    U = np.zeros(L.total)
    h = 1.0 / n
    for p in range(patches):
        V = L.view(U, p)
        x = (p * m + np.arange(m + 2 * g) - g + 0.5) * h
        left = x < 0.5
        rho = np.where(left, 1.0, 0.125)
        pr = np.where(left, 1.0, 0.1)
        V[RHO, 0, 0, :] = rho
        V[EN, 0, 0, :] = pr / (gamma - 1.0)
    dx = np.tile([h, 1.0, 1.0], (patches, 1))
    nbr = grid_neighbours((patches, 1, 1), (False, False, False))
    return Workload("sod", L, U, dx, gamma, nbr, cfl=0.4, t_end=0.2)


def orszag_tang(N=256, patch=32, g=3, gamma=5.0 / 3.0, t_end=0.5):
    """Orszag-Tang vortex on the periodic unit square: rho = 25/(36 pi),
    p = 5/(12 pi), u = (-sin 2 pi y, sin 2 pi x, 0),
    B = (-sin 2 pi y, sin 4 pi x, 0)/sqrt(4 pi) sampled at face centres."""
    assert N % patch == 0
    Pg = N // patch
    L = Layout(np.tile([patch, patch, 1], (Pg * Pg, 1)), g)
    U = np.zeros(L.total)
    h = 1.0 / N
    r0, p0, s = 25.0 / (36.0 * math.pi), 5.0 / (12.0 * math.pi), 1.0 / math.sqrt(4.0 * math.pi)
    tp = 2.0 * math.pi
    for py in range(Pg):
        for px in range(Pg):
            p = px + Pg * py
            V = L.view(U, p)
            i = np.arange(patch + 2 * g) - g
            xc = (px * patch + i + 0.5) * h
            yc = (py * patch + i + 0.5) * h
            yy, xx = np.meshgrid(yc, xc, indexing="ij")
            u = -np.sin(tp * yy)
            v = np.sin(tp * xx)
            bcx, bcy = -s * np.sin(tp * yy), s * np.sin(2 * tp * xx)
            V[RHO, 0] = r0
            V[MX, 0] = r0 * u
            V[MY, 0] = r0 * v
            V[EN, 0] = _conserved(r0, u, v, 0.0, p0, bcx, bcy, 0.0, gamma)
            # Bx on lower x faces (x_{i-1/2}, y_j); By on lower y faces (x_i, y_{j-1/2})
            V[BX, 0] = -s * np.sin(tp * yy)
            V[BY, 0] = s * np.sin(2 * tp * xx)
    dx = np.tile([h, h, 1.0], (L.P, 1))
    nbr = grid_neighbours((Pg, Pg, 1), (True, True, True))
    return Workload("orszag_tang", L, U, dx, gamma, nbr, cfl=0.4, t_end=t_end)


# -------------------------------------------------------- seeded turbulent velocity

KMAX = 8


def turbulence_modes(seed=3, mach=4.0, kmax=KMAX):
    """Fourier amplitudes a[c, kx, ky, kz] (indices offset by kmax) of a real random
    velocity field: i.i.d. complex Gaussian per Cartesian component with
    <|a_k|^2> ~ |k|^-2 for integer 1 <= |k| <= kmax, Hermitian-symmetrised, scaled to a
    3D rms |v| of `mach` (sound speed 1)."""
    rng = np.random.default_rng(seed)
    n = 2 * kmax + 1
    re = rng.standard_normal((3, n, n, n))
    im = rng.standard_normal((3, n, n, n))
    a = (re + 1j * im) / math.sqrt(2.0)
    k = np.arange(-kmax, kmax + 1)
    kk = np.sqrt(k[:, None, None] ** 2 + k[None, :, None] ** 2 + k[None, None, :] ** 2)
    mask = (kk >= 1.0) & (kk <= kmax)
    amp = np.where(mask, 1.0 / np.where(kk > 0, kk, 1.0), 0.0)
    a = a * amp[None]
    a = (a + np.conj(a[:, ::-1, ::-1, ::-1])) / math.sqrt(2.0)   # a(-k) = conj a(k)
    a *= mach / math.sqrt(np.sum(np.abs(a) ** 2))                  # Parseval: <|v|^2>
    return a


def eval_modes(a, xs, ys, zs, kmax=KMAX, device="cpu"):
    """Evaluate v_c(x, y, z) = sum_k a[c,k] exp(2 pi i k.x) on the tensor-product points
    xs (B, nx), ys (B, ny), zs (B, nz) for a batch of B patches; returns a float64
    torch tensor (B, 3, nz, ny, nx)."""
    import torch
    k = torch.arange(-kmax, kmax + 1, dtype=torch.float64, device=device)
    A = torch.as_tensor(a, dtype=torch.complex128, device=device)          # (3, a, b, c)

    def ph(x):
        x = torch.as_tensor(x, dtype=torch.float64, device=device)
        return torch.exp(2j * math.pi * k[None, :, None] * x[:, None, :])  # (B, 17, n)

    X, Y, Z = ph(xs), ph(ys), ph(zs)
    # contract kz, then ky, then kx (separable sums)
    T = torch.einsum("sabc,pck->psabk", A, Z)
    T = torch.einsum("psabk,pbj->psajk", T, Y)
    T = torch.einsum("psajk,pai->pskji", T, X)
    return T.real.contiguous()


def _fill_turbulent(L, U, origins, h, a, gamma, b0, device="cpu", chunk=256):
    """Fill every patch with rho = 1, p = 1/gamma, B = (b0, 0, 0) and the seeded
    velocity field evaluated at its padded cell centres (guards included)."""
    import torch
    g = L.g
    p0 = 1.0 / gamma
    out = torch.as_tensor(U) if not isinstance(U, torch.Tensor) else U
    dims = L.dims
    base = L.base
    order = np.argsort(dims[:, 0], kind="stable")
    # batch patches of equal size
    for n in np.unique(dims[:, 0]):
        idx = np.nonzero(dims[:, 0] == n)[0]
        m = int(n) + 2 * g
        i = np.arange(m) - g + 0.5
        for s in range(0, len(idx), chunk):
            ids = idx[s:s + chunk]
            o = origins[ids]
            hh = h[ids][:, None]
            xs = o[:, 0:1] + i[None, :] * hh
            ys = o[:, 1:2] + i[None, :] * hh
            zs = o[:, 2:3] + i[None, :] * hh
            vel = eval_modes(a, xs, ys, zs, device=device)                 # (B,3,m,m,m)
            B = vel.shape[0]
            blk = torch.zeros((B, 8, m, m, m), dtype=torch.float64, device=device)
            blk[:, RHO] = 1.0
            blk[:, MX:MZ + 1] = vel
            ke = 0.5 * (vel * vel).sum(dim=1)
            blk[:, EN] = p0 / (gamma - 1.0) + ke + 0.5 * b0 * b0
            blk[:, BX] = b0
            blk = blk.reshape(B, -1)
            for t, p in enumerate(ids):
                out[int(base[p]):int(base[p + 1])] = blk[t].to(out.device, out.dtype)
    del order
    return out


def turbulence(N=512, patch=32, g=3, seed=3, gamma=5.0 / 3.0, mach=4.0, b0=0.2, nsteps=10,
               device="cpu", dtype=None, grid=None):
    """Decaying supersonic MHD turbulence on the periodic unit cube, N^3 cells as
    (N/patch)^3 patches of patch^3; rho = 1, p = 1/gamma (sound speed 1),
    B = (b0, 0, 0); velocity = seeded random field (turbulence_modes), rms Mach `mach`.

    With `grid` = (gx, gy, gz) only that sub-block of patches (a corner of the domain,
    same cell size) is generated, for small test cases.  Returns a Workload whose U is
    a torch tensor on `device` (dtype float64 unless `dtype` is given)."""
    import torch
    assert N % patch == 0
    Pg = N // patch
    gx, gy, gz = grid if grid is not None else (Pg, Pg, Pg)
    L = Layout(np.tile([patch, patch, patch], (gx * gy * gz, 1)), g)
    h = 1.0 / N
    iz, iy, ix = np.meshgrid(np.arange(gz), np.arange(gy), np.arange(gx), indexing="ij")
    origins = np.stack([ix.ravel(), iy.ravel(), iz.ravel()], axis=1) * (patch * h)
    hs = np.full(L.P, h)
    U = torch.zeros(L.total, dtype=dtype or torch.float64, device=device)
    a = turbulence_modes(seed, mach)
    _fill_turbulent(L, U, origins, hs, a, gamma, b0, device=device)
    dx = np.full((L.P, 3), h)
    periodic = (gx == Pg, gy == Pg, gz == Pg)
    nbr = grid_neighbours((gx, gy, gz), periodic)
    return Workload("turbulence", L, U, dx, gamma, nbr, cfl=0.4, nsteps=nsteps,
                    meta={"N": N, "patch": patch, "seed": seed, "grid": (gx, gy, gz)})


UNEVEN_MIX = ((16, 2000), (24, 1000), (32, 500), (48, 100))


def uneven(mix=UNEVEN_MIX, g=3, seed=4, field_seed=3, gamma=5.0 / 3.0, mach=4.0, b0=0.2,
           nsteps=10, device="cpu", dtype=None):
    """Uneven bunch: patches of several sizes, each covering one of the 16^3 slots of
    the unit cube (slot drawn with `seed`) at its own resolution h = 1/(16 n), holding
    the turbulence field sampled at its cell centres, guards included (frozen guards:
    no exchange).  Patch order is shuffled with the same seed."""
    import torch
    rng = np.random.default_rng(seed)
    sizes = np.concatenate([np.full(c, n, dtype=np.int32) for n, c in mix])
    sizes = sizes[rng.permutation(len(sizes))]
    slots = rng.integers(0, 16, size=(len(sizes), 3))
    L = Layout(np.stack([sizes, sizes, sizes], axis=1), g)
    h = 1.0 / (16.0 * sizes)
    origins = slots / 16.0
    U = torch.zeros(L.total, dtype=dtype or torch.float64, device=device)
    a = turbulence_modes(field_seed, mach)
    _fill_turbulent(L, U, origins, h, a, gamma, b0, device=device)
    dx = np.stack([h, h, h], axis=1)
    return Workload("uneven", L, U, dx, gamma, None, cfl=0.4, nsteps=nsteps,
                    meta={"mix": mix, "seed": seed})


def adjoint_case(noise_seed=5, N=64, patch=32, g=3, gamma=5.0 / 3.0, amp=1e-3, noise=1e-4,
                 nsteps=20):
    """64^3 periodic box as 2^3 patches of 32^3; background rho = 1, p = 0.6,
    B = (1, 0, 0) (sound speed 1); longitudinal wave along x with
    (drho, du, dp) = amp (rho, c, gamma p) sin 2 pi x; then i.i.d. N(0, noise^2) added to
    all 8 conserved fields at every owned cell and face (seeded); guards filled by
    periodic copy is left to the caller (neighbour table returned)."""
    Pg = N // patch
    L = Layout(np.tile([patch, patch, patch], (Pg ** 3, 1)), g)
    U = np.zeros(L.total)
    h = 1.0 / N
    r0, p0, c0 = 1.0, 0.6, math.sqrt(gamma * 0.6 / 1.0)
    rng = np.random.default_rng(noise_seed)
    for p in range(L.P):
        px, py, pz = p % Pg, (p // Pg) % Pg, p // (Pg * Pg)
        V = L.view(U, p)
        m = patch + 2 * g
        x = (px * patch + np.arange(m) - g + 0.5) * h
        sx = np.sin(2 * math.pi * x)[None, None, :] * np.ones((m, m, 1))
        rho = r0 * (1 + amp * sx)
        u = amp * c0 * sx
        pr = p0 + amp * gamma * p0 * sx
        V[RHO] = rho
        V[MX] = rho * u
        V[EN] = _conserved(rho, u, 0.0, 0.0, pr, 1.0, 0.0, 0.0, gamma)
        V[BX] = 1.0
    for p in range(L.P):
        I = L.interior(U, p)
        I += noise * rng.standard_normal(I.shape)
    dx = np.full((L.P, 3), h)
    nbr = grid_neighbours((Pg, Pg, Pg), (True, True, True))
    return Workload("adjoint", L, U, dx, gamma, nbr, cfl=0.4, nsteps=nsteps)
