"""Pins of the D3Q19 tables and of the local collision pieces against closed
forms and invariants that the paper's equations fix (Sec. II.C)."""
import itertools

import numpy as np
import pytest

from oracle import d3q19 as L
from oracle import lb

RNG = np.random.default_rng(0)


def test_velocity_set_structure():
    c = L.C
    assert c.shape == (19, 3)
    assert len({tuple(v) for v in c}) == 19
    norms = (c * c).sum(axis=1)
    assert (norms == 0).sum() == 1 and (norms == 1).sum() == 6 and (norms == 2).sum() == 12
    for p in range(19):
        assert np.all(c[L.OPP[p]] == -c[p])


def test_weight_isotropy():
    """Moments of the weights fix them: sum w = 1, sum w c c = vT2 I,
    sum w c c c c = vT2^2 (d d + d d + d d), odd moments vanish."""
    w, c = L.W, L.C.astype(float)
    assert np.isclose(w.sum(), 1.0, atol=1e-15)
    assert np.allclose(np.einsum("p,pa->a", w, c), 0.0, atol=1e-15)
    assert np.allclose(np.einsum("p,pa,pb->ab", w, c, c), L.VT2 * np.eye(3), atol=1e-15)
    assert np.allclose(np.einsum("p,pa,pb,pc->abc", w, c, c, c), 0.0, atol=1e-15)
    d = np.eye(3)
    iso = (np.einsum("ab,cd->abcd", d, d) + np.einsum("ac,bd->abcd", d, d)
           + np.einsum("ad,bc->abcd", d, d))
    assert np.allclose(np.einsum("p,pa,pb,pc,pd->abcd", w, c, c, c, c), L.VT2 ** 2 * iso, atol=1e-15)
    assert L.VT2 == pytest.approx(1.0 / 3.0)


def test_equilibrium_moments():
    """sum f_eq = n, sum c f_eq = n u, sum c c f_eq = n (vT2 I + u u)."""
    n = RNG.uniform(0.5, 1.5, size=(4,))
    u = RNG.uniform(-0.1, 0.1, size=(3, 4))
    feq = lb.equilibrium(n, u)
    c = L.C.astype(float)
    assert np.allclose(feq.sum(axis=0), n, rtol=1e-14)
    assert np.allclose(np.einsum("pa,pk->ak", c, feq), n * u, rtol=1e-13, atol=1e-16)
    second = np.einsum("pa,pb,pk->abk", c, c, feq)
    want = n * (L.VT2 * np.eye(3)[:, :, None] + u[:, None] * u[None, :])
    assert np.allclose(second, want, rtol=1e-13, atol=1e-16)


def test_forcing_moments():
    """sum S = 0, sum c S = n phi, sum c c S = n (u phi + phi u)."""
    n = RNG.uniform(0.01, 1.5, size=(5,))
    u = RNG.uniform(-0.1, 0.1, size=(3, 5))
    phi = RNG.uniform(-0.05, 0.05, size=(3, 5))
    S = lb.forcing(n, u, phi)
    c = L.C.astype(float)
    assert np.allclose(S.sum(axis=0), 0.0, atol=1e-16)
    assert np.allclose(np.einsum("pa,pk->ak", c, S), n * phi, rtol=1e-13, atol=1e-17)
    second = np.einsum("pa,pb,pk->abk", c, c, S)
    want = n * (u[:, None] * phi[None, :] + phi[:, None] * u[None, :])
    assert np.allclose(second, want, rtol=1e-12, atol=1e-17)


def test_drag_closed_form_solves_implicit_definition():
    """The closed form must satisfy u^a = j^a / n^a + Phi^a / 2 with
    Phi^a = G^a + Phi_drag^a(u) and Phi_drag taken literally from Eq. Fidef."""
    S, K = 3, 7
    n = RNG.uniform(0.005, 1.2, size=(S, K))
    j = RNG.uniform(-0.02, 0.02, size=(S, 3, K))
    G = RNG.uniform(-0.03, 0.03, size=(S, 3, K))
    wd = np.array([0.7, 1.3, 2.1])
    u, phi = lb.species_velocities(n, j, G, wd)
    drag = lb.drag_force(n, u, wd)
    assert np.allclose(phi, G + drag, rtol=1e-13, atol=1e-17)
    assert np.allclose(u, j / n[:, None] + phi / 2.0, rtol=1e-13, atol=1e-17)


def test_drag_conserves_momentum_for_equal_rates():
    S, K = 3, 5
    n = RNG.uniform(0.005, 1.2, size=(S, K))
    u = RNG.uniform(-0.1, 0.1, size=(S, 3, K))
    drag = lb.drag_force(n, u, np.ones(3) * 0.9)
    assert np.allclose((n[:, None] * drag).sum(axis=0), 0.0, atol=1e-16)


@pytest.mark.parametrize("tau", [1.0, 0.8, 1.7])
def test_collision_conserves_mass_and_adds_force(tau):
    """Collision keeps every species' mass and adds n Phi to its momentum;
    at tau = 1 it returns f_eq + S / 2."""
    shape = (2, 2, 2)
    f = RNG.uniform(0.0, 0.1, size=(3, 19) + shape)
    f[0] *= 10.0
    G = RNG.uniform(-0.01, 0.01, size=(3, 3) + shape)
    fluid = np.ones(shape, dtype=bool)
    taus = np.array([tau, tau, tau])
    fs, u, phi = lb.collide(f, G, taus, np.ones(3), fluid)
    n, j = lb.moments(f)
    n2, j2 = lb.moments(fs)
    assert np.allclose(n2, n, rtol=1e-14)
    assert np.allclose(j2, j + n[:, None] * phi, rtol=1e-12, atol=1e-16)
    if tau == 1.0:
        for s in range(3):
            want = lb.equilibrium(n[s], u[s]) + 0.5 * lb.forcing(n[s], u[s], phi[s])
            assert np.allclose(fs[s], want, rtol=1e-13, atol=1e-17)


def test_streaming_moves_each_population_along_its_velocity():
    """Brute force on a 4^3 periodic box: a single non-zero population f_p at
    r lands at r + c_p, for every p and several r."""
    shape = (4, 4, 4)
    solid = np.zeros(shape, dtype=bool)
    for p in range(19):
        for r in [(0, 0, 0), (3, 1, 2), (1, 3, 3)]:
            f = np.zeros((1, 19) + shape)
            f[0, p, r[2], r[1], r[0]] = 1.0
            out = lb.stream(f, solid)
            dest = tuple((np.array(r) + L.C[p]) % 4)
            assert out[0, p, dest[2], dest[1], dest[0]] == 1.0
            assert out.sum() == 1.0


def test_bounce_back_returns_population_reversed():
    """A population pointing into a solid site comes back at the same site
    with the opposite velocity (halfway bounce-back)."""
    shape = (4, 4, 4)
    solid = np.zeros(shape, dtype=bool)
    solid[2, 1, 1] = True                        # z=2, y=1, x=1
    f = np.zeros((1, 19) + shape)
    p = 5                                        # +z
    f[0, p, 1, 1, 1] = 1.0                       # at (x=1, y=1, z=1) heading to z=2
    out = lb.stream(f, solid)
    assert out[0, L.OPP[p], 1, 1, 1] == 1.0
    assert out.sum() == 1.0


def test_streaming_conserves_mass_with_random_walls():
    shape = (6, 4, 8)
    solid = RNG.uniform(size=shape) < 0.3
    f = RNG.uniform(size=(3, 19) + shape) * (~solid)[None, None]
    m0 = f.sum(axis=(1, 2, 3, 4))
    for _ in range(20):
        f = lb.stream(f, solid)
    assert np.allclose(f.sum(axis=(1, 2, 3, 4)), m0, rtol=1e-14)
