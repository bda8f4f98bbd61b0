"""Pins of the Picard outer loop (section 1: the Oseen system is one Picard
linearisation of the steady Navier-Stokes equations) and of the discrete
wind it feeds back into the generator."""
import numpy as np
import pytest
import scipy.sparse as sp

from oracle.picard import assemble, ns_residual, picard
from workloads.mac_oseen import FaceWind, Wind, make_oseen_mac

ZERO = (lambda x, y: 0.0 * x, lambda x, y: 0.0 * y)


def _C(n, nu, wind, stretch=None):
    rp, ci, v, b, meta = make_oseen_mac(n, nu, wind=wind, stretch=stretch, seed=1)
    return sp.csr_matrix((v, ci, rp), shape=(meta["N"], meta["N"])), b, meta, rp, ci


def _rand_wind(n, seed):
    rng = np.random.default_rng(seed)
    return FaceWind(rng.standard_normal((n, n - 1)), rng.standard_normal((n - 1, n)))


def test_pattern_does_not_depend_on_the_wind():
    """The partition can be reused across Picard steps: same rowptr/colidx."""
    _, _, _, rp0, ci0 = _C(12, 0.05, FaceWind(np.zeros((12, 11)), np.zeros((11, 12))), 1.05)
    _, _, _, rp1, ci1 = _C(12, 0.05, _rand_wind(12, 3), 1.05)
    assert np.array_equal(rp0, rp1) and np.array_equal(ci0, ci1)


def test_face_wind_convection_is_skew_and_linear():
    n, nu = 12, 0.05
    C0, b0, meta, _, _ = _C(n, nu, FaceWind(np.zeros((n, n - 1)), np.zeros((n - 1, n))), 1.05)
    w1, w2 = _rand_wind(n, 1), _rand_wind(n, 2)
    K1 = (_C(n, nu, w1, 1.05)[0] - C0).toarray()
    K2 = (_C(n, nu, w2, 1.05)[0] - C0).toarray()
    K12 = (_C(n, nu, FaceWind(w1.u + 2 * w2.u, w1.v + 2 * w2.v), 1.05)[0] - C0).toarray()
    nvel = meta["n_u"] + meta["n_v"]
    for K in (K1, K2):
        assert np.abs(K + K.T).max() <= 1e-13 * np.abs(K).max()    # skew-symmetric convection
        assert not K[nvel:, :].any() and not K[:, nvel:].any()      # velocity block only
        assert np.abs(K).max() > 0
    assert np.abs(K12 - (K1 + 2 * K2)).max() <= 1e-12 * np.abs(K12).max()


def _face_average_wind(w, n, stretch=None):
    """Face velocities of a stream-function wind: the exact mean over each face."""
    _, _, _, _, meta = make_oseen_mac(n, 0.1, stretch=stretch, seed=0)
    X, Y = meta["X"], meta["Y"]
    u = np.zeros((n, n - 1))
    v = np.zeros((n - 1, n))
    for j in range(n):
        for i in range(1, n):
            u[j, i - 1] = (w.psi(X[i], Y[j]) - w.psi(X[i], Y[j + 1])) / (Y[j + 1] - Y[j])
    for j in range(1, n):
        for i in range(n):
            v[j - 1, i] = (w.psi(X[i + 1], Y[j]) - w.psi(X[i], Y[j])) / (X[i + 1] - X[i])
    return FaceWind(u, v)


def test_face_wind_fluxes_converge_to_the_stream_fluxes():
    """Face velocities sampled from a smooth stream function give CV fluxes
    that approach the exact ones at second order (ratio ~4 per halving);
    a wrong interpolation index would stall at first order or worse."""
    w = Wind((1.0, 0.5, -0.3, 0.2))
    errs = []
    for n in (16, 32, 64):
        Cs = _C(n, 0.1, w)[0]
        Cf = _C(n, 0.1, _face_average_wind(w, n))[0]
        # convective entries are F/2 with F = O(h), so compare relative to h
        errs.append(np.abs((Cs - Cf).toarray()).max() * n)
    assert errs[0] / errs[1] > 3.0 and errs[1] / errs[2] > 3.0, errs


def test_picard_fixed_point_solves_navier_stokes():
    """The Picard limit equals the root of the discrete steady Navier-Stokes
    equations found by a different method (scipy's hybrid Powell root finder
    on the residual), on an 8x8 lid-driven cavity."""
    from scipy.optimize import root
    n, nu = 8, 0.05
    pr = picard(n, nu, m=2, sz=8, tol=1e-12, maxit=60, lin_tol=1e-13, forcing=ZERO)
    assert pr.converged
    N = len(pr.x)

    def F(x):
        rp, ci, v, b, meta = assemble(n, nu, x, forcing=ZERO)
        return sp.csr_matrix((v, ci, rp), shape=(N, N)) @ x - b

    sol = root(F, np.zeros(N), method="hybr", tol=1e-13)
    assert sol.success
    assert np.linalg.norm(sol.x - pr.x) <= 1e-8 * np.linalg.norm(sol.x)
    assert ns_residual(n, nu, pr.x, forcing=ZERO) <= 1e-12


def test_picard_converges_on_the_lid_driven_cavity():
    pr = picard(16, 0.01, m=4, sz=24, tol=1e-8, forcing=ZERO)
    assert pr.converged and len(pr.residuals) <= 25
    assert pr.residuals[-1] <= 1e-8
    # the first step is the Stokes problem (zero wind): the residual of x_0 = 0 is 1
    assert pr.residuals[0] == pytest.approx(1.0)
