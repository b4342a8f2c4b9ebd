"""Thermal fluctuations: the stochastic term Delta of the lattice kinetic
equation (Eq. kernelf2 and the Delta equation of Sec. II.C) and the
Langevin noise on the beads (Sec. II.B), with the counter-based random
numbers both are drawn from.

Random numbers.  Philox4x32-10 (Salmon, Moraes, Dror and Shaw, "Parallel
random numbers: as easy as 1, 2, 3", SC 2011): a 128-bit counter and a
64-bit key give four 32-bit words through ten rounds; each round multiplies
two counter words by the constants 0xD2511F53 and 0xCD9E8D57, keeps the
high and low halves of the products, and mixes the high halves with the
other two words and the key, which is bumped by the Weyl constants
0x9E3779B9 and 0xBB67AE85 between rounds.  A word x gives the uniform
u = (x + 1/2) / 2^32 in (0, 1); two uniforms give two standard normals by
the Box-Muller transform, sqrt(-2 ln u1) (cos 2 pi u2, sin 2 pi u2), so one
call gives four normals (words 0, 1 and 2, 3).

Keys and counters (the library uses the same definition):
  key       (seed mod 2^32, seed div 2^32) of the 64-bit seed;
  lattice   species a, site r (linear index (z ny + y) nx + x), step t
            (the number of steps completed before this one): calls
            j = 0..3 with counter (r, t, 4 a + j, 0), normals 4 j .. 4 j + 3;
            the first 15 of the 16 are N_4 .. N_18;
  beads     bead i, step t, substep s: counter (i, t, s, 1), normals 0..2
            are the x, y, z components.

Readings taken (listed with the others in the design notes):
  * the mode basis {chi_k}: the 19 polynomials of the lattice velocities
    1; c_x, c_y, c_z; c^2 - 1; 3 c_x^2 - c^2; c_y^2 - c_z^2; c_x c_y; c_y c_z;
    c_x c_z; (3 c^2 - 5) c_x, (3 c^2 - 5) c_y, (3 c^2 - 5) c_z;
    (c_y^2 - c_z^2) c_x, (c_z^2 - c_x^2) c_y, (c_x^2 - c_y^2) c_z;
    3 c^4 - 6 c^2 + 1; (2 c^2 - 3)(3 c_x^2 - c^2); (2 c^2 - 3)(c_y^2 - c_z^2),
    each divided by its norm sqrt(sum_p w_p chi_kp^2), which makes them
    orthonormal under sum_p w_p chi_kp chi_lp (the paper's scalar product):
    k = 0 density, 1-3 current, 4-9 momentum flux, 10-18 non-hydrodynamic;
  * Delta_p = sqrt(m n omega (2 - omega)) w_p sum_{k=4}^{18} chi_kp N_k with
    n the species' density at the site before the collision (clamped at 0)
    and the thermal mass m = k_B T / v_T^2 (k_B T = m v_T^2); Delta is added
    to the post-collision populations of fluid sites;
  * bead noise: xi_i ~ N(0, 2 gamma k_B T / h) per component and substep h
    (the fluctuation-dissipation theorem of Sec. II.B for the total
    friction gamma), acting on the bead together with the friction; the
    fluid receives the opposite impulse, shared among the species by their
    number fractions like the friction, so fluid + bead momentum stays
    exact.
"""
import numpy as np

from . import d3q19 as L

_M0 = np.uint64(0xD2511F53)
_M1 = np.uint64(0xCD9E8D57)
_W0 = np.uint64(0x9E3779B9)
_W1 = np.uint64(0xBB67AE85)
_LO = np.uint64(0xFFFFFFFF)
_S32 = np.uint64(32)


def philox4x32_10(counter, key):
    """Philox4x32-10 of counters [..., 4] and keys [..., 2] (uint32,
    broadcast against each other); returns uint32 [..., 4]."""
    ctr = np.asarray(counter, dtype=np.uint64)
    k = np.asarray(key, dtype=np.uint64)
    c0, c1, c2, c3 = (ctr[..., i] for i in range(4))
    k0, k1 = k[..., 0], k[..., 1]
    for rnd in range(10):
        if rnd:
            k0 = (k0 + _W0) & _LO
            k1 = (k1 + _W1) & _LO
        p0 = _M0 * c0                      # both factors < 2^32: exact in 64 bits
        p1 = _M1 * c2
        c0, c1, c2, c3 = ((p1 >> _S32) ^ c1 ^ k0, p1 & _LO, (p0 >> _S32) ^ c3 ^ k1, p0 & _LO)
    return np.stack([c0, c1, c2, c3], axis=-1).astype(np.uint32)


def seed_key(seed):
    seed = int(seed) & 0xFFFFFFFFFFFFFFFF
    return np.array([seed & 0xFFFFFFFF, seed >> 32], dtype=np.uint32)


def uniform(words):
    """(x + 1/2) / 2^32 of uint32 words, in (0, 1)."""
    return (np.asarray(words, dtype=np.float64) + 0.5) * (1.0 / 4294967296.0)


def normals(words):
    """Four standard normals per Philox output [..., 4] by Box-Muller on the
    word pairs (0, 1) and (2, 3)."""
    u = uniform(words)
    r01 = np.sqrt(-2.0 * np.log(u[..., 0]))
    r23 = np.sqrt(-2.0 * np.log(u[..., 2]))
    return np.stack([r01 * np.cos(2.0 * np.pi * u[..., 1]), r01 * np.sin(2.0 * np.pi * u[..., 1]),
                     r23 * np.cos(2.0 * np.pi * u[..., 3]), r23 * np.sin(2.0 * np.pi * u[..., 3])],
                    axis=-1)


def mode_basis():
    """chi [19, 19]: row k is mode k over the populations p, orthonormal
    under sum_p w_p chi_kp chi_lp."""
    c = L.C.astype(np.float64)
    cx, cy, cz = c[:, 0], c[:, 1], c[:, 2]
    c2 = cx * cx + cy * cy + cz * cz
    rows = [np.ones(L.Q), cx, cy, cz,
            c2 - 1.0, 3.0 * cx * cx - c2, cy * cy - cz * cz, cx * cy, cy * cz, cx * cz,
            (3.0 * c2 - 5.0) * cx, (3.0 * c2 - 5.0) * cy, (3.0 * c2 - 5.0) * cz,
            (cy * cy - cz * cz) * cx, (cz * cz - cx * cx) * cy, (cx * cx - cy * cy) * cz,
            3.0 * c2 * c2 - 6.0 * c2 + 1.0, (2.0 * c2 - 3.0) * (3.0 * cx * cx - c2),
            (2.0 * c2 - 3.0) * (cy * cy - cz * cz)]
    chi = np.array(rows)
    return chi / np.sqrt((L.W[None, :] * chi * chi).sum(axis=1))[:, None]


def lattice_normals(shape, species, step, seed):
    """N_4 .. N_18 at every site of a box [Z, Y, X] for one species and step:
    returns [15, Z, Y, X]."""
    nsite = int(np.prod(shape))
    r = np.arange(nsite, dtype=np.uint64)
    out = np.empty((16, nsite))
    key = seed_key(seed)
    for j in range(4):
        ctr = np.stack([r, np.full(nsite, step, np.uint64), np.full(nsite, 4 * species + j, np.uint64),
                        np.zeros(nsite, np.uint64)], axis=-1)
        out[4 * j:4 * j + 4] = normals(philox4x32_10(ctr, key)).T
    return out[:15].reshape((15,) + tuple(shape))


def lattice_noise(n, omega, kT, species, step, seed):
    """Delta_p of one species at every site: n [Z, Y, X] its density before
    the collision; returns [19, Z, Y, X]."""
    chi = mode_basis()
    m = kT / L.VT2
    amp = np.sqrt(m * np.maximum(n, 0.0) * omega * (2.0 - omega))
    N = lattice_normals(n.shape, species, step, seed)                     # [15, ...]
    proj = np.einsum("kp,k...->p...", chi[4:], N)                         # sum_k chi_kp N_k
    return L.W.reshape((L.Q,) + (1,) * n.ndim) * amp[None] * proj


def bead_normals(n_beads, step, substep, seed):
    """Standard normals [N, 3] of the beads' noise at one substep."""
    i = np.arange(n_beads, dtype=np.uint64)
    ctr = np.stack([i, np.full(n_beads, step, np.uint64), np.full(n_beads, substep, np.uint64),
                    np.ones(n_beads, np.uint64)], axis=-1)
    return normals(philox4x32_10(ctr, seed_key(seed)))[:, :3]
