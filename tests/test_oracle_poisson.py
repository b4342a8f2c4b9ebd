"""Pins of the Poisson solver (Eq. poisson solved by red-black SOR with
Chebyshev acceleration, Sec. II.C) against an exact spectral solve, a
brute-force site loop and the discrete identity sum rho grad psi = 0."""
import numpy as np
import pytest

from oracle import poisson

RNG = np.random.default_rng(1)


def fft_solve(b):
    """Exact periodic solution of the 7-point problem via numpy.fft: the
    operator is diagonal in Fourier space with eigenvalue
    -(6 - 2 cos kx - 2 cos ky - 2 cos kz); mean(psi) = 0."""
    Z, Y, X = b.shape
    kz = 2 * np.pi * np.fft.fftfreq(Z)[:, None, None]
    ky = 2 * np.pi * np.fft.fftfreq(Y)[None, :, None]
    kx = 2 * np.pi * np.fft.fftfreq(X)[None, None, :]
    lam = -(6.0 - 2 * np.cos(kx) - 2 * np.cos(ky) - 2 * np.cos(kz))
    lam[0, 0, 0] = 1.0
    ph = np.fft.fftn(b) / lam
    ph[0, 0, 0] = 0.0
    return np.real(np.fft.ifftn(ph))


def random_rhs(shape):
    rho = RNG.normal(size=shape)
    return poisson.rhs_from_charge(rho, 0.341)


def test_laplacian_matches_fourier_symbol():
    b = random_rhs((6, 8, 10))
    psi = fft_solve(b)
    assert np.allclose(poisson.laplacian(psi), b, atol=1e-12 * np.abs(b).max())


@pytest.mark.parametrize("shape", [(8, 8, 8), (12, 6, 10), (16, 16, 32)])
def test_sor_converges_to_spectral_solution(shape):
    b = random_rhs(shape)
    psi, it, rr = poisson.sor_red_black_chebyshev(b, np.zeros(shape), 1e-12, 20000)
    assert rr <= 1e-12
    exact = fft_solve(b)
    assert abs(psi.mean()) < 1e-14
    assert np.max(np.abs(psi - exact)) <= 1e-9 * np.max(np.abs(exact))
    assert poisson.relative_residual(exact, b) < 1e-13


def test_sor_warm_start_from_solution_takes_no_iteration():
    b = random_rhs((8, 8, 8))
    exact = fft_solve(b)
    psi, it, rr = poisson.sor_red_black_chebyshev(b, exact, 1e-10, 100)
    assert it == 0 and rr <= 1e-10


def test_zero_rhs_gives_zero_potential():
    b = np.zeros((4, 4, 4))
    psi, it, rr = poisson.sor_red_black_chebyshev(b, RNG.normal(size=(4, 4, 4)), 1e-10, 10)
    assert it == 0 and not psi.any()


def test_not_converged_raises():
    b = random_rhs((16, 16, 16))
    with pytest.raises(poisson.NotConverged):
        poisson.sor_red_black_chebyshev(b, np.zeros_like(b), 1e-12, 2)


def _brute_force_sweeps(b, psi0, rho_j, iterations):
    """Site-by-site loops: red sites (x+y+z even) in any order, then black,
    each with the relaxation factor of the Chebyshev schedule."""
    Z, Y, X = b.shape
    psi = psi0.copy()
    omega = 1.0
    for it in range(iterations):
        for half, parity in enumerate((0, 1)):
            new = psi.copy()
            for z in range(Z):
                for y in range(Y):
                    for x in range(X):
                        if (x + y + z) % 2 != parity:
                            continue
                        s = (psi[(z + 1) % Z, y, x] + psi[(z - 1) % Z, y, x]
                             + psi[z, (y + 1) % Y, x] + psi[z, (y - 1) % Y, x]
                             + psi[z, y, (x + 1) % X] + psi[z, y, (x - 1) % X])
                        new[z, y, x] = (1 - omega) * psi[z, y, x] + omega * (s - b[z, y, x]) / 6.0
            psi = new
            if it == 0 and half == 0:
                omega = 1.0 / (1.0 - rho_j ** 2 / 2.0)
            else:
                omega = 1.0 / (1.0 - rho_j ** 2 * omega / 4.0)
    return psi


def test_iterates_match_site_loops():
    shape = (4, 6, 4)
    b = random_rhs(shape)
    psi0 = RNG.normal(size=shape) * 0.1
    rj = poisson.jacobi_radius(shape)
    for k in (1, 2, 5):
        vec, _, _ = poisson.sor_red_black_chebyshev(b, psi0, 0.0, 0, rho_j=rj, iterations=k)
        ref = _brute_force_sweeps(b, psi0, rj, k)
        assert np.allclose(vec, ref, rtol=1e-13, atol=1e-15)


def test_jacobi_radius_is_largest_nontrivial_eigenvalue():
    """Enumerate the Jacobi eigenvalues (cos kx + cos ky + cos kz) / 3 of the
    periodic operator and take the largest magnitude below 1 once the two
    unit modes (constant, checkerboard) are set aside."""
    for shape in [(8, 8, 8), (16, 8, 32), (10, 12, 6)]:
        Z, Y, X = shape
        ev = []
        for a in range(Z):
            for bb in range(Y):
                for c in range(X):
                    v = (np.cos(2 * np.pi * a / Z) + np.cos(2 * np.pi * bb / Y)
                         + np.cos(2 * np.pi * c / X)) / 3.0
                    if abs(abs(v) - 1.0) > 1e-12:
                        ev.append(abs(v))
        assert poisson.jacobi_radius(shape) == pytest.approx(max(ev), rel=1e-14)


def test_chebyshev_beats_gauss_seidel():
    """With the Jacobi radius the accelerated solver needs far fewer sweeps
    than plain red-black Gauss-Seidel (rho_J = 0 gives omega = 1 throughout)."""
    b = random_rhs((16, 16, 16))
    _, it_cheb, _ = poisson.sor_red_black_chebyshev(b, np.zeros_like(b), 1e-8, 5000)
    _, it_gs, _ = poisson.sor_red_black_chebyshev(b, np.zeros_like(b), 1e-8, 5000, rho_j=0.0)
    assert it_cheb * 3 < it_gs


def test_force_balance_of_field_and_charge():
    """With E = -grad_h psi (central) and A_h psi = -rho / eps on the periodic
    box, sum_r rho E = 0 exactly: the electrostatic forces on all charges
    cancel, so momentum is conserved."""
    shape = (8, 10, 12)
    rho = RNG.normal(size=shape)
    rho -= rho.mean()
    eps = 0.341
    psi = fft_solve(poisson.rhs_from_charge(rho, eps))
    E = poisson.electric_field(psi, (0.0, 0.0, 0.0))
    total = (rho[None] * E).sum(axis=(1, 2, 3))
    assert np.max(np.abs(total)) < 1e-12 * np.abs(rho).sum() * np.abs(E).max()
    # and for the iterative solution to its tolerance
    psi2, _, _ = poisson.sor_red_black_chebyshev(poisson.rhs_from_charge(rho, eps),
                                                 np.zeros(shape), 1e-10, 10000)
    E2 = poisson.electric_field(psi2, (0.0, 0.0, 0.0))
    assert np.max(np.abs((rho[None] * E2).sum(axis=(1, 2, 3)))) < 1e-8 * np.abs(rho).sum() * np.abs(E2).max()


def test_field_sign_points_down_the_potential():
    """A positive point charge gives a potential maximum and a field pointing
    away from it (E = -grad psi), with eps from the Bjerrum length."""
    shape = (16, 16, 16)
    rho = np.zeros(shape)
    rho[8, 8, 8] = 1.0
    psi = fft_solve(poisson.rhs_from_charge(rho, 0.341))
    assert psi[8, 8, 8] == psi.max()
    E = poisson.electric_field(psi, (0.0, 0.0, 0.0))
    assert E[0, 8, 8, 9] > 0 and E[0, 8, 8, 7] < 0
    assert E[2, 9, 8, 8] > 0 and E[2, 7, 8, 8] < 0
