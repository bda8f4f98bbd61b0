"""Pins of the seeded MAC Oseen generator (input side, no method arithmetic)."""
import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spl

from workloads.mac_oseen import Wind, cell_widths, make_oseen_mac, unknown_positions


@pytest.mark.parametrize("n", [2, 4, 7, 16, 40])
def test_sizes_closed_form(n):
    rp, ci, v, b, meta = make_oseen_mac(n, 0.1, seed=3)
    assert meta["N"] == 3 * n * n - 2 * n - 1
    assert len(v) == 18 * n * n - 26 * n
    assert rp[-1] == len(v) and rp.dtype == np.int32 and ci.dtype == np.int32
    for i in range(meta["N"]):  # sorted, unique columns per row
        c = ci[rp[i]:rp[i + 1]]
        assert np.all(np.diff(c) > 0)


def test_convection_exactly_skew_and_viscous_symmetric():
    n = 12
    rp, ci, v, b, meta = make_oseen_mac(n, 0.0, stretch=1.07, seed=1)
    C = sp.csr_matrix((v, ci, rp)).toarray()
    nv = meta["n_u"] + meta["n_v"]
    A = C[:nv, :nv]
    assert np.abs(A + A.T).max() == 0.0
    assert np.abs(np.diag(A)).max() == 0.0
    rp, ci, v, b, meta = make_oseen_mac(n, 0.3, wind=Wind((0, 0, 0, 0)), stretch=1.07, seed=1)
    C = sp.csr_matrix((v, ci, rp)).toarray()
    A = C[:nv, :nv]
    assert np.abs(A - A.T).max() == 0.0
    assert np.all(np.linalg.eigvalsh(A) > 0)


def test_gradient_is_negated_divergence_transpose():
    rp, ci, v, b, meta = make_oseen_mac(10, 0.05, stretch=1.1, seed=2)
    C = sp.csr_matrix((v, ci, rp)).toarray()
    nv = meta["n_u"] + meta["n_v"]
    assert np.abs(C[:nv, nv:] + C[nv:, :nv].T).max() == 0.0
    assert np.abs(C[nv:, nv:]).max() == 0.0
    assert np.all(b[nv:] == 0.0)


def test_stretched_widths():
    w = cell_widths(64, 1.05)
    assert abs(w.sum() - 2.0) < 1e-14
    assert np.allclose(w[1:32] / w[:31], 1.05, rtol=0, atol=1e-12)
    assert np.array_equal(w, w[::-1])
    assert np.allclose(cell_widths(8), 0.25)


def test_face_fluxes_divergence_free():
    """Sum of outward stream-function fluxes of each u control volume is zero
    to rounding, i.e. the discrete wind is divergence free."""
    n = 20
    wind = Wind((0.3, -1.1, 0.7, 0.4), 1.7)
    X = -1 + np.concatenate([[0], np.cumsum(cell_widths(n, 1.03))])
    xc = 0.5 * (X[1:] + X[:-1])
    psi = wind.psi
    worst = 0.0
    for i in range(1, n):
        for j in range(n):
            fe = psi(xc[i], X[j]) - psi(xc[i], X[j + 1])
            fw = psi(xc[i - 1], X[j + 1]) - psi(xc[i - 1], X[j])
            fn = psi(xc[i], X[j + 1]) - psi(xc[i - 1], X[j + 1])
            fs = psi(xc[i - 1], X[j]) - psi(xc[i], X[j])
            worst = max(worst, abs(fe + fw + fn + fs))
    assert worst < 1e-15


def test_wind_is_velocity_of_stream_function():
    wind = Wind((0.3, -1.1, 0.7, 0.4), 1.7)
    x, y, h = 0.31, -0.57, 1e-6
    wx, wy = wind.velocity(x, y)
    assert abs(wx + (wind.psi(x, y + h) - wind.psi(x, y - h)) / (2 * h)) < 1e-8
    assert abs(wy - (wind.psi(x + h, y) - wind.psi(x - h, y)) / (2 * h)) < 1e-8
    d = Wind()
    assert np.allclose(d.velocity(0.5, 0.25), (2 * 0.25 * (1 - 0.25), -2 * 0.5 * (1 - 0.0625)))


def _mms_error(n, nu):
    """Manufactured solution psi* = (1-x^2)^2 (1-y^2)^2, u* = psi*_y,
    v* = -psi*_x, p* = x y, lid off; returns max nodal velocity error."""
    def us(x, y):
        return (1 - x * x) ** 2 * 2 * (1 - y * y) * (-2 * y)

    def vs(x, y):
        return -((1 - y * y) ** 2 * 2 * (1 - x * x) * (-2 * x))

    # derivatives written out by hand
    def lap_u(x, y):
        # u* = -4 y (1-x^2)^2 (1-y^2)
        uxx = -4 * y * (1 - y * y) * (12 * x * x - 4)
        uyy = -4 * (1 - x * x) ** 2 * (-6 * y)
        return uxx + uyy

    def lap_v(x, y):
        # v* = 4 x (1-y^2)^2 (1-x^2)
        vxx = 4 * (1 - y * y) ** 2 * (-6 * x)
        vyy = 4 * x * (1 - x * x) * (12 * y * y - 4)
        return vxx + vyy

    def ux(x, y):
        return -4 * y * (1 - y * y) * 2 * (1 - x * x) * (-2 * x)

    def uy(x, y):
        return -4 * (1 - x * x) ** 2 * (1 - 3 * y * y)

    def vx(x, y):
        return 4 * (1 - y * y) ** 2 * (1 - 3 * x * x)

    def vy(x, y):
        return 4 * x * (1 - x * x) * 2 * (1 - y * y) * (-2 * y)

    w = Wind()

    def fu(x, y):
        wx, wy = w.velocity(x, y)
        return -nu * lap_u(x, y) + wx * ux(x, y) + wy * uy(x, y) + y

    def fv(x, y):
        wx, wy = w.velocity(x, y)
        return -nu * lap_v(x, y) + wx * vx(x, y) + wy * vy(x, y) + x

    rp, ci, v, b, meta = make_oseen_mac(n, nu, wind=w, lid=0.0, forcing=(fu, fv))
    C = sp.csc_matrix(sp.csr_matrix((v, ci, rp)))
    sol = spl.splu(C).solve(b)
    X, Y, kind = unknown_positions(meta)
    ex = np.where(kind == 0, us(X, Y), np.where(kind == 1, vs(X, Y), 0.0))
    nv = meta["n_u"] + meta["n_v"]
    return np.abs(sol[:nv] - ex[:nv]).max()


def test_manufactured_solution_second_order():
    e = [_mms_error(n, 0.1) for n in (16, 32, 64)]
    assert e[2] < 5e-3
    assert e[0] / e[1] > 3.4 and e[1] / e[2] > 3.6


def test_rhs_seeded():
    b1 = make_oseen_mac(8, 0.1, seed=5)[3]
    b2 = make_oseen_mac(8, 0.1, seed=5)[3]
    b3 = make_oseen_mac(8, 0.1, seed=6)[3]
    assert np.array_equal(b1, b2) and not np.array_equal(b1, b3)


def test_hybrid_scheme_is_central_below_peclet_two_and_upwind_above():
    """The hybrid option: where every face Peclet number |F_f|/a_f is at most 2
    the matrix equals the central one; at high Peclet numbers every
    convective off-diagonal entry is the upwind one, -max(-F_f, 0), so the
    velocity block's off-diagonal entries are <= 0 and its symmetric part is
    positive semidefinite (diagonally dominant)."""
    import scipy.sparse as sp
    rp, ci, v, _, meta = make_oseen_mac(8, 1.0, seed=1)
    rp2, ci2, v2, _, _ = make_oseen_mac(8, 1.0, seed=1, scheme="hybrid")
    assert np.array_equal(rp, rp2) and np.array_equal(ci, ci2) and np.array_equal(v, v2)
    rpc, cic, vc, _, meta = make_oseen_mac(16, 1e-4, seed=1)
    rph, cih, vh, _, _ = make_oseen_mac(16, 1e-4, seed=1, scheme="hybrid")
    assert np.array_equal(cic, cih)
    nvel = meta["n_u"] + meta["n_v"]
    A = sp.csr_matrix((vh, cih, rph), shape=(meta["N"], meta["N"]))[:nvel, :nvel].toarray()
    off = A - np.diag(np.diag(A))
    assert off.max() <= 0.0
    Sym = 0.5 * (A + A.T)
    assert np.linalg.eigvalsh(Sym).min() > -1e-12 * np.abs(Sym).max()
    Ac = sp.csr_matrix((vc, cic, rpc), shape=(meta["N"], meta["N"]))[:nvel, :nvel].toarray()
    assert np.abs(Ac - A).max() > 0.0
    # hybrid minus central is symmetric (added diffusion), the skew parts agree
    Dd = A - Ac
    assert np.abs(Dd - Dd.T).max() <= 1e-15 * np.abs(A).max()
