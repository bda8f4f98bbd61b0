"""Seeded synthetic Oseen systems on a staggered (MAC) grid.

This module only builds inputs: the sparse matrix C, the right-hand side b and
geometric metadata.  It contains none of the domain-decomposition method's
arithmetic and is shared, as data, by the CPU oracle and the GPU path.

Problem (paper, section 1, the Navier-Stokes equations and the block 2x2
Picard/Oseen form C = [D E^T; -E 0]): one Picard step of the steady
incompressible Navier-Stokes equations on [-1,1]^2,

    -nu Lap u + (w . grad) u + grad p = f,   div u = 0,

with a frozen, divergence-free wind w = (-d psi/dy, d psi/dx), a lid velocity
u = 1 on y = 1 and no-slip on the other walls.  The paper's experiments use
IFISS Q2-Q1 finite elements on a leaky lid-driven cavity (section 5); those
matrices are not available, so this finite-volume MAC discretisation stands in
for them, with the paper's range of viscosities and grid stretching.

Discretisation:
  * n x n cells; widths uniform (2/n) or geometric towards every wall with
    ratio r per cell: h_k = h_0 r^k from each wall, k = 0..n/2-1, mirrored,
    h_0 = (r-1)/(r^(n/2)-1) so that each half sums to 1.
  * unknowns: u on interior vertical faces ((n-1) n), v on interior
    horizontal faces (n (n-1)), p at cell centres (n^2 - 1: cell (0,0) is
    pinned to remove the hydrostatic mode).  Order: all u (x fastest), all v
    (x fastest), all p (x fastest, cell (0,0) skipped), i.e. velocity block
    first as in the paper's block form.  N = 3n^2 - 2n - 1.
  * every equation is multiplied by its control-volume area (finite-volume
    scaling), so the gradient block is exactly the transpose of the negated
    divergence block.
  * viscous fluxes nu * length / distance, with distance Delta/2 to a wall
    ghost for tangential velocities;
  * convection in central, skew-symmetric form: the off-diagonal entry for
    the neighbour across face f is F_f/2, F_f the outward face flux computed
    from the stream function as psi(end) - psi(start); the convective
    diagonal is zero, so the convection matrix is exactly skew-symmetric.
    Optionally (scheme="hybrid") a face whose Peclet number |F_f| / a_f
    exceeds 2 is differenced upwind instead: its viscous coefficient a_f is
    raised to |F_f|/2, which adds a symmetric, diagonally dominant
    (artificial diffusion) part and leaves the skew part unchanged.
  * b: velocity rows = control-volume area * f with f ~ N(0,1) drawn from
    numpy.random.default_rng(seed), plus the lid's Dirichlet contribution;
    pressure rows = 0.
"""
from __future__ import annotations

import numpy as np


# --------------------------------------------------------------------------
# grids and winds
# --------------------------------------------------------------------------

def cell_widths(n: int, stretch: float | None = None) -> np.ndarray:
    """Cell widths on [-1, 1]: uniform 2/n, or geometric towards both walls."""
    if n < 2:
        raise ValueError("need n >= 2 cells")
    if stretch is None or stretch == 1.0:
        return np.full(n, 2.0 / n)
    if n % 2:
        raise ValueError("stretched grids need an even n")
    r = float(stretch)
    half = n // 2
    h0 = (r - 1.0) / (r ** half - 1.0)
    h = h0 * r ** np.arange(half, dtype=np.float64)
    return np.concatenate([h, h[::-1]])


def face_coords(widths: np.ndarray) -> np.ndarray:
    x = np.empty(widths.size + 1)
    x[0] = -1.0
    x[1:] = -1.0 + np.cumsum(widths)
    x[-1] = 1.0
    return x


class Wind:
    """Stream function psi = s * (1-x^2)(1-y^2) * (c0 + c1 x + c2 y + c3 x y).

    The default (c = (1,0,0,0), s = 1) gives w = (2y(1-x^2), -2x(1-y^2)).
    psi vanishes on the boundary, so the wind has no normal component there.
    """

    def __init__(self, coeffs=(1.0, 0.0, 0.0, 0.0), scale: float = 1.0):
        self.c = tuple(float(v) for v in coeffs)
        self.s = float(scale)

    def psi(self, x, y):
        c0, c1, c2, c3 = self.c
        return self.s * (1.0 - x * x) * (1.0 - y * y) * (c0 + c1 * x + c2 * y + c3 * x * y)

    def velocity(self, x, y):
        """w = (-d psi/dy, d psi/dx), evaluated analytically."""
        c0, c1, c2, c3 = self.c
        bx = 1.0 - x * x
        by = 1.0 - y * y
        m = c0 + c1 * x + c2 * y + c3 * x * y
        dpsi_dx = self.s * (-2.0 * x * by * m + bx * by * (c1 + c3 * y))
        dpsi_dy = self.s * (-2.0 * y * bx * m + bx * by * (c2 + c3 * x))
        return -dpsi_dy, dpsi_dx

    @staticmethod
    def random_modes(rng: np.random.Generator, max_speed: float = 2.0) -> "Wind":
        """Seeded combination of the four recirculating modes, scaled so that
        the largest speed on a 101 x 101 sample of the square is max_speed."""
        c = rng.standard_normal(4)
        w = Wind(c, 1.0)
        t = np.linspace(-1.0, 1.0, 101)
        X, Y = np.meshgrid(t, t, indexing="xy")
        wx, wy = w.velocity(X, Y)
        vmax = float(np.sqrt(wx * wx + wy * wy).max())
        return Wind(c, max_speed / vmax if vmax > 0 else 1.0)


    def cv_fluxes(self, g):
        """Outward face fluxes of every velocity control volume, exact for
        the stream function: psi(end) - psi(start) along each face."""
        return _stream_fluxes(self.psi, g)


class FaceWind:
    """A discrete wind given by face velocities (a previous Picard iterate):
    u on the interior vertical faces (array (n, n-1), [j, i-1]) and v on the
    interior horizontal faces ((n-1, n), [j-1, i]), zero on the walls.
    Control-volume face fluxes interpolate these linearly: a face through a
    cell centre takes the mean of the cell's two face velocities times the
    face length, and a face along a grid line takes the two half-faces'
    velocities times their half-lengths."""

    def __init__(self, u, v):
        self.u = np.asarray(u, dtype=np.float64)
        self.v = np.asarray(v, dtype=np.float64)

    @staticmethod
    def from_solution(x, n):
        """The velocity part of a solution vector in the generator's order."""
        nu_ = (n - 1) * n
        return FaceWind(np.asarray(x[:nu_]).reshape(n, n - 1), np.asarray(x[nu_:2 * nu_]).reshape(n - 1, n))

    def cv_fluxes(self, g):
        n, dx, dy = g["n"], g["dx"], g["dy"]
        if self.u.shape != (n, n - 1) or self.v.shape != (n - 1, n):
            raise ValueError("face velocities do not match the grid")
        Up = np.zeros((n, n + 1))     # Up[j, i] = u on vertical face i of row j
        Up[:, 1:n] = self.u
        Vp = np.zeros((n + 1, n))     # Vp[j, i] = v on horizontal face j of column i
        Vp[1:n, :] = self.v
        I, J = g["uI"], g["uJ"]
        f = {}
        f["uE"] = 0.5 * (Up[J, I] + Up[J, I + 1]) * dy[J]
        f["uW"] = -0.5 * (Up[J, I - 1] + Up[J, I]) * dy[J]
        f["uN"] = 0.5 * (Vp[J + 1, I - 1] * dx[I - 1] + Vp[J + 1, I] * dx[I])
        f["uS"] = -0.5 * (Vp[J, I - 1] * dx[I - 1] + Vp[J, I] * dx[I])
        I2, J2 = g["vI"], g["vJ"]
        f["vN"] = 0.5 * (Vp[J2, I2] + Vp[J2 + 1, I2]) * dx[I2]
        f["vS"] = -0.5 * (Vp[J2 - 1, I2] + Vp[J2, I2]) * dx[I2]
        f["vE"] = 0.5 * (Up[J2 - 1, I2 + 1] * dy[J2 - 1] + Up[J2, I2 + 1] * dy[J2])
        f["vW"] = -0.5 * (Up[J2 - 1, I2] * dy[J2 - 1] + Up[J2, I2] * dy[J2])
        return f


def _stream_fluxes(psi, g):
    X, Y, xc, yc = g["X"], g["Y"], g["xc"], g["yc"]
    I, J = g["uI"], g["uJ"]
    I2, J2 = g["vI"], g["vJ"]
    return {
        "uE": psi(xc[I], Y[J]) - psi(xc[I], Y[J + 1]),
        "uW": psi(xc[I - 1], Y[J + 1]) - psi(xc[I - 1], Y[J]),
        "uN": psi(xc[I], Y[J + 1]) - psi(xc[I - 1], Y[J + 1]),
        "uS": psi(xc[I - 1], Y[J]) - psi(xc[I], Y[J]),
        "vN": psi(X[I2 + 1], yc[J2]) - psi(X[I2], yc[J2]),
        "vS": psi(X[I2], yc[J2 - 1]) - psi(X[I2 + 1], yc[J2 - 1]),
        "vE": psi(X[I2 + 1], yc[J2 - 1]) - psi(X[I2 + 1], yc[J2]),
        "vW": psi(X[I2], yc[J2]) - psi(X[I2], yc[J2 - 1]),
    }


# --------------------------------------------------------------------------
# assembly
# --------------------------------------------------------------------------

class _Coo:
    def __init__(self):
        self.r, self.c, self.v = [], [], []

    def add(self, rows, cols, vals, mask=None):
        rows = np.asarray(rows)
        cols = np.broadcast_to(np.asarray(cols), rows.shape)
        vals = np.broadcast_to(np.asarray(vals, dtype=np.float64), rows.shape)
        if mask is not None:
            m = np.broadcast_to(np.asarray(mask, dtype=bool), rows.shape)
            rows, cols, vals = rows[m], cols[m], vals[m]
        self.r.append(rows.ravel().astype(np.int64))
        self.c.append(cols.ravel().astype(np.int64))
        self.v.append(vals.ravel().copy())

    def to_csr(self, N):
        r = np.concatenate(self.r)
        c = np.concatenate(self.c)
        v = np.concatenate(self.v)
        key = r * N + c
        order = np.argsort(key, kind="stable")
        key, v = key[order], v[order]
        uk, first = np.unique(key, return_index=True)
        if uk.size != key.size:
            raise AssertionError("duplicate entries in assembly")
        rows = (uk // N).astype(np.int64)
        cols = (uk % N).astype(np.int32)
        rowptr = np.zeros(N + 1, dtype=np.int64)
        np.add.at(rowptr, rows + 1, 1)
        rowptr = np.cumsum(rowptr).astype(np.int32)
        return rowptr, cols, v[first]


def make_oseen_mac(n: int, nu: float, wind: Wind | FaceWind | None = None, stretch: float | None = None,
                   seed: int | None = 0, lid: float = 1.0, forcing=None, scheme: str = "central"):
    """Assemble C (CSR, int32 indices, float64 values), b and metadata.

    wind: a stream-function Wind (default Wind()) or a FaceWind (discrete
          face velocities, e.g. the previous Picard iterate).  The sparsity
          pattern does not depend on the wind.
    forcing: None -> f ~ N(0,1) per velocity unknown from default_rng(seed);
             callable (fu(x,y), fv(x,y)) -> point values at the unknowns.
    scheme: "central" (skew-symmetric convection) or "hybrid" (central on a
            face whose Peclet number |F_f| / a_f is at most 2, first-order
            upwind beyond: the viscous coefficient a_f of the face is replaced
            by max(a_f, |F_f|/2)).
    """
    if scheme not in ("central", "hybrid"):
        raise ValueError(scheme)
    hyb = scheme == "hybrid"
    wind = wind or Wind()
    dx = cell_widths(n, stretch)
    dy = dx.copy()
    X = face_coords(dx)
    Y = face_coords(dy)
    xc = 0.5 * (X[:-1] + X[1:])
    yc = 0.5 * (Y[:-1] + Y[1:])
    uI, uJ = np.meshgrid(np.arange(1, n), np.arange(n), indexing="xy")
    vI, vJ = np.meshgrid(np.arange(n), np.arange(1, n), indexing="xy")
    flux = wind.cv_fluxes(dict(n=n, dx=dx, dy=dy, X=X, Y=Y, xc=xc, yc=yc, uI=uI, uJ=uJ, vI=vI, vJ=vJ))

    nu_ = (n - 1) * n
    nv_ = n * (n - 1)
    npr = n * n - 1
    N = nu_ + nv_ + npr

    def U(i, j):  # i = 1..n-1, j = 0..n-1
        return j * (n - 1) + (i - 1)

    def V(i, j):  # i = 0..n-1, j = 1..n-1
        return nu_ + (j - 1) * n + i

    def P(i, j):  # cell (i, j) != (0, 0)
        return nu_ + nv_ + j * n + i - 1

    coo = _Coo()
    b = np.zeros(N)

    # ---------------- u momentum ----------------
    I, J = np.meshgrid(np.arange(1, n), np.arange(n), indexing="xy")  # shape (n, n-1)
    rows = U(I, J)
    wu = xc[I] - xc[I - 1]          # CV width
    hu = dy[J]                      # CV height
    diag = np.zeros(I.shape)
    bu = np.zeros(I.shape)
    lidv = np.zeros(I.shape)
    # east neighbour u(i+1, j), face at xc[i]
    a = nu * hu / dx[I]
    F = flux["uE"]
    if hyb:
        a = np.maximum(a, 0.5 * np.abs(F))
    inner = I + 1 <= n - 1
    coo.add(rows, U(np.minimum(I + 1, n - 1), J), -a + 0.5 * F, inner)
    diag += a
    # west neighbour u(i-1, j), face at xc[i-1]
    a = nu * hu / dx[I - 1]
    F = flux["uW"]
    if hyb:
        a = np.maximum(a, 0.5 * np.abs(F))
    inner = I - 1 >= 1
    coo.add(rows, U(np.maximum(I - 1, 1), J), -a + 0.5 * F, inner)
    diag += a
    # north neighbour u(i, j+1), face at Y[j+1]
    top = J + 1 == n
    dist = np.where(top, 0.5 * dy[J], yc[np.minimum(J + 1, n - 1)] - yc[J])
    a = nu * wu / dist
    F = flux["uN"]
    if hyb:
        a = np.maximum(a, 0.5 * np.abs(F))
    coo.add(rows, U(I, np.minimum(J + 1, n - 1)), -a + 0.5 * F, ~top)
    diag += a
    lidv = np.where(top, lid, 0.0)
    bu += (a - 0.5 * F) * lidv
    # south neighbour u(i, j-1), face at Y[j]
    bot = J == 0
    dist = np.where(bot, 0.5 * dy[J], yc[J] - yc[np.maximum(J - 1, 0)])
    a = nu * wu / dist
    F = flux["uS"]
    if hyb:
        a = np.maximum(a, 0.5 * np.abs(F))
    coo.add(rows, U(I, np.maximum(J - 1, 0)), -a + 0.5 * F, ~bot)
    diag += a
    coo.add(rows, rows, diag)
    # pressure gradient: +dy (p(i,j) - p(i-1,j))
    coo.add(rows, P(I, J), hu, ~((I == 0) & (J == 0)))
    coo.add(rows, P(np.maximum(I - 1, 0), J), -hu, ~((I - 1 == 0) & (J == 0)))
    areas_u = wu * hu
    xu, yu = X[I], yc[J]

    # ---------------- v momentum ----------------
    I2, J2 = np.meshgrid(np.arange(n), np.arange(1, n), indexing="xy")  # shape (n-1, n)
    rows2 = V(I2, J2)
    wv = dx[I2]
    hv = yc[J2] - yc[J2 - 1]
    diag2 = np.zeros(I2.shape)
    # north v(i, j+1), face at yc[j]
    a = nu * wv / dy[J2]
    F = flux["vN"]
    if hyb:
        a = np.maximum(a, 0.5 * np.abs(F))
    coo.add(rows2, V(I2, np.minimum(J2 + 1, n - 1)), -a + 0.5 * F, J2 + 1 <= n - 1)
    diag2 += a
    # south v(i, j-1), face at yc[j-1]
    a = nu * wv / dy[J2 - 1]
    F = flux["vS"]
    if hyb:
        a = np.maximum(a, 0.5 * np.abs(F))
    coo.add(rows2, V(I2, np.maximum(J2 - 1, 1)), -a + 0.5 * F, J2 - 1 >= 1)
    diag2 += a
    # east v(i+1, j), face at X[i+1]
    right = I2 + 1 == n
    dist = np.where(right, 0.5 * dx[I2], xc[np.minimum(I2 + 1, n - 1)] - xc[I2])
    a = nu * hv / dist
    F = flux["vE"]
    if hyb:
        a = np.maximum(a, 0.5 * np.abs(F))
    coo.add(rows2, V(np.minimum(I2 + 1, n - 1), J2), -a + 0.5 * F, ~right)
    diag2 += a
    # west v(i-1, j), face at X[i]
    left = I2 == 0
    dist = np.where(left, 0.5 * dx[I2], xc[I2] - xc[np.maximum(I2 - 1, 0)])
    a = nu * hv / dist
    F = flux["vW"]
    if hyb:
        a = np.maximum(a, 0.5 * np.abs(F))
    coo.add(rows2, V(np.maximum(I2 - 1, 0), J2), -a + 0.5 * F, ~left)
    diag2 += a
    coo.add(rows2, rows2, diag2)
    # pressure gradient: +dx (p(i,j) - p(i,j-1))
    coo.add(rows2, P(I2, J2), wv, ~((I2 == 0) & (J2 == 0)))
    coo.add(rows2, P(I2, J2 - 1), -wv, ~((I2 == 0) & (J2 - 1 == 0)))
    areas_v = wv * hv
    xv, yv = xc[I2], Y[J2]

    # ---------------- continuity: divergence ----------------
    Ic, Jc = np.meshgrid(np.arange(n), np.arange(n), indexing="xy")
    keep = ~((Ic == 0) & (Jc == 0))
    Ic, Jc = Ic[keep], Jc[keep]
    prow = P(Ic, Jc)
    m = Ic + 1 <= n - 1
    coo.add(prow[m], U(Ic[m] + 1, Jc[m]), dy[Jc[m]])            # + dy u_east
    m = Ic >= 1
    coo.add(prow[m], U(Ic[m], Jc[m]), -dy[Jc[m]])               # - dy u_west
    m = Jc + 1 <= n - 1
    coo.add(prow[m], V(Ic[m], Jc[m] + 1), dx[Ic[m]])            # + dx v_north
    m = Jc >= 1
    coo.add(prow[m], V(Ic[m], Jc[m]), -dx[Ic[m]])               # - dx v_south

    rowptr, colidx, vals = coo.to_csr(N)

    # ---------------- right-hand side ----------------
    if forcing is None:
        rng = np.random.default_rng(seed)
        f = rng.standard_normal(nu_ + nv_)
        fu = f[:nu_].reshape(I.shape)
        fv = f[nu_:].reshape(I2.shape)
    else:
        fu_fn, fv_fn = forcing
        fu = fu_fn(xu, yu)
        fv = fv_fn(xv, yv)
    b[rows.ravel()] = (areas_u * fu + bu).ravel()
    b[rows2.ravel()] = (areas_v * fv).ravel()

    meta = dict(n=n, nu=nu, N=N, n_u=nu_, n_v=nv_, n_p=npr, dx=dx, dy=dy, X=X, Y=Y,
                xc=xc, yc=yc, stretch=stretch, seed=seed, wind=wind,
                xu=xu.ravel(), yu=yu.ravel(), xv=xv.ravel(), yv=yv.ravel(),
                area_u=areas_u.ravel(), area_v=areas_v.ravel())
    return rowptr, colidx, vals, b, meta


def unknown_positions(meta):
    """(x, y, kind) of every unknown: kind 0 = u, 1 = v, 2 = p."""
    n = meta["n"]
    xc, yc = meta["xc"], meta["yc"]
    Pi, Pj = np.meshgrid(np.arange(n), np.arange(n), indexing="xy")
    keep = ~((Pi == 0) & (Pj == 0))
    x = np.concatenate([meta["xu"], meta["xv"], xc[Pi[keep]]])
    y = np.concatenate([meta["yu"], meta["yv"], yc[Pj[keep]]])
    kind = np.concatenate([np.zeros(meta["n_u"], np.int8), np.ones(meta["n_v"], np.int8),
                           np.full(meta["n_p"], 2, np.int8)])
    return x, y, kind
