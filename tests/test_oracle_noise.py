"""Pins of the thermal fluctuations (Sec. II.C, the stochastic term Delta of
Eq. kernelf2; Sec. II.B, the Langevin noise of the beads): the counter-based
generator reproduces the published known-answer vectors, its normals have
unit variance, the D3Q19 mode basis is orthonormal under the paper's scalar
product with the density, current and momentum-flux modes where the paper
puts them, Delta conserves mass and momentum and drives every other mode
with variance m n omega (2 - omega), the fluctuating lattice reaches
equipartition <j_x^2> = n k_B T, a bead in a resting fluid reaches the
stationary variance of its discrete Langevin map, and fluid + bead momentum
stays exact with the noise on."""
import os

import numpy as np
import pytest

from oracle import d3q19 as L
from oracle import lb, md, noise, step

HERE = os.path.dirname(os.path.abspath(__file__))


def test_philox_known_answer_vectors():
    rows = [l.split() for l in open(os.path.join(HERE, "golden", "philox_kat.txt"))
            if l.strip() and not l.startswith("#")]
    assert len(rows) == 3
    for r in rows:
        w = np.array([int(x, 16) for x in r], dtype=np.uint64).astype(np.uint32)
        assert np.array_equal(noise.philox4x32_10(w[:4], w[4:6]), w[6:10]), r


def test_normals_have_zero_mean_and_unit_variance():
    ctr = np.stack([np.arange(100000), np.full(100000, 7), np.zeros(100000), np.zeros(100000)],
                   axis=-1).astype(np.uint32)
    z = noise.normals(noise.philox4x32_10(ctr, noise.seed_key(12345))).ravel()
    n = z.size
    assert abs(z.mean()) < 4.0 / np.sqrt(n)
    assert abs(z.var() - 1.0) < 4.0 * np.sqrt(2.0 / n)
    assert abs((z ** 4).mean() - 3.0) < 0.05                     # Gaussian kurtosis
    u = noise.uniform(np.array([0, 0xFFFFFFFF], dtype=np.uint32))
    assert 0.0 < u[0] < 1e-9 and 1.0 - 1e-9 < u[1] < 1.0


def test_mode_basis_is_orthonormal_with_hydrodynamic_modes_first():
    chi = noise.mode_basis()
    gram = (L.W[None, :] * chi) @ chi.T
    assert np.allclose(gram, np.eye(L.Q), atol=1e-14)
    c = L.C.astype(np.float64)
    assert np.allclose(chi[0], 1.0)
    assert np.allclose(chi[1:4], c.T / np.sqrt(L.VT2))
    # modes 0 and 4..9 span exactly the quadratic polynomials (momentum flux)
    quad = np.array([np.ones(L.Q)] + [c[:, a] * c[:, b] for a in range(3) for b in range(a, 3)])
    assert np.linalg.matrix_rank(np.vstack([quad, chi[[0, 4, 5, 6, 7, 8, 9]]])) == 7


def test_delta_conserves_mass_and_momentum_and_drives_modes_at_the_stated_variance():
    shape = (40, 30, 20)
    n = np.full(shape, 0.7)
    omega, kT = 0.8, 2e-3
    d = noise.lattice_noise(n, omega, kT, species=1, step=3, seed=99)
    c = L.C.astype(np.float64)
    assert np.abs(d.sum(axis=0)).max() < 1e-16
    assert np.abs(np.einsum("pk,p...->k...", c, d)).max() < 1e-16
    modes = np.einsum("kp,p...->k...", noise.mode_basis(), d).reshape(L.Q, -1)
    var = (kT / L.VT2) * 0.7 * omega * (2.0 - omega)
    assert np.abs(modes[:4]).max() < 1e-16
    m = modes.shape[1]
    for k in range(4, L.Q):
        assert abs(modes[k].var() / var - 1.0) < 4.0 * np.sqrt(2.0 / m), k
        assert abs(modes[k].mean()) < 4.0 * np.sqrt(var / m), k
    # species, step and seed give independent streams
    d2 = noise.lattice_noise(n, omega, kT, species=2, step=3, seed=99)
    d3 = noise.lattice_noise(n, omega, kT, species=1, step=4, seed=99)
    d4 = noise.lattice_noise(n, omega, kT, species=1, step=3, seed=100)
    for other in (d2, d3, d4):
        r = np.corrcoef(d[1].ravel(), other[1].ravel())[0, 1]
        assert abs(r) < 4.0 / np.sqrt(d[1].size)


def test_fluctuating_lattice_reaches_equipartition():
    """Three independent species (no drag, no charges) on a periodic box at
    k_B T = 1e-3: the site momentum of each species fluctuates with
    <j_x^2> = n k_B T (1 - 1 / N_sites) (the total momentum stays zero),
    whatever its density, at tau = 1 and tau = 0.8."""
    shape = (6, 6, 6)
    kT = 1e-3
    dens = (1.0, 0.5, 0.25)
    n0 = np.stack([np.full(shape, v) for v in dens])
    p = step.Params(valence=(0.0, 0.0, 0.0), tau=(1.0, 0.8, 1.0), omega_drag=(0.0, 0.0, 0.0),
                    kT=kT, fluctuations=True, seed=2026)
    sim = step.Simulation(p, np.zeros(shape, dtype=bool), np.zeros(shape), n0)
    sim.run(100)
    acc = np.zeros(3)
    steps = 1500
    for _ in range(steps):
        sim.step()
        _, j = lb.moments(sim.f)
        acc += (j ** 2).mean(axis=(1, 2, 3, 4))
    acc /= steps
    expect = np.array(dens) * kT * (1.0 - 1.0 / np.prod(shape))
    print(acc / expect)
    assert np.all(np.abs(acc / expect - 1.0) < 0.04), acc / expect
    assert np.allclose(sim.mass(), n0.sum(axis=(1, 2, 3)), rtol=1e-13)
    assert np.abs(sim.momentum()).max() < 1e-12


def test_bead_in_resting_fluid_reaches_the_discrete_langevin_variance():
    """A bead coupled by friction gamma to a fluid so dense that it stays at
    rest, with the noise of variance 2 gamma k_B T / h per substep: its
    velocity follows V' = (1 - a) V + (h / M) xi, a = gamma h / M, whose
    stationary variance per component is 2 k_B T / (M (2 - a)) (k_B T / M
    as h -> 0).  Every impulse the bead receives goes to the fluid."""
    shape = (4, 4, 4)
    dens = 1e9
    n = np.stack([np.full(shape, dens), np.full(shape, 1e-3 * dens), np.full(shape, 1e-3 * dens)])
    j = np.zeros((3, 3) + shape)
    E = np.zeros((3,) + shape)
    fluid = np.ones(shape, dtype=bool)
    M, gamma, n_sub, kT = 2.0, 5.0, 5, 0.2
    poly = dict(M=M, q=np.zeros(1), k_fene=0.0, R0=1e3, eps=0.0, sigma=1.0, gamma=gamma,
                n_sub=n_sub)
    R = np.array([[1.3, 2.2, 0.7]])
    V = np.zeros((1, 3))
    h = 1.0 / n_sub
    a = gamma * h / M
    samples = []
    for t in range(3000):
        V0 = V.copy()
        R, V, K = md.md_substeps(R, V, n, j, E, fluid, np.zeros((0, 3)), poly,
                                 thermal=(77, t, kT))
        assert np.allclose(K.sum(axis=(0, 2, 3, 4)), -M * (V - V0)[0], rtol=1e-9, atol=1e-15)
        if t >= 20:
            samples.append(V[0].copy())
    v = np.array(samples)
    expect = 2.0 * kT / (M * (2.0 - a))
    # correlation time of the map: 1 / a substeps, far below a lattice step
    assert np.all(np.abs(v.var(axis=0) / expect - 1.0) < 0.06), v.var(axis=0) / expect
    assert np.all(np.abs(v.mean(axis=0)) < 4.0 * np.sqrt(expect / len(v)))


def test_fluid_plus_bead_momentum_is_exact_with_noise():
    shape = (8, 8, 12)
    rng = np.random.default_rng(5)
    n0 = np.stack([np.ones(shape), 0.1 * (1 + 0.05 * rng.uniform(-1, 1, shape)),
                   0.1 * (1 + 0.05 * rng.uniform(-1, 1, shape))])
    R = np.array([[3.0, 4.0, 5.0], [3.95, 4.1, 5.1], [4.9, 4.3, 5.0]])
    poly = step.polymer_params(3, q=-0.3)
    p = step.Params(poisson_tol=1e-12, kT=1e-3, fluctuations=True, seed=4)
    sim = step.Simulation(p, np.zeros(shape, dtype=bool), np.zeros(shape), n0,
                          beads=(R, np.zeros_like(R), poly))

    def total():
        return sim.momentum() + poly["M"] * sim.V.sum(axis=0)
    P0 = total()
    m0 = sim.mass()
    sim.run(5)
    assert np.allclose(total(), P0, atol=1e-12)
    assert np.allclose(sim.mass(), m0, rtol=1e-13)
    assert np.abs(sim.V).max() > 1e-4            # the noise moved the beads
