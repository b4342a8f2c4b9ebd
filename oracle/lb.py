"""Multi-component lattice-Boltzmann kernel: moments, equilibrium, forcing,
inter-species drag, BGK collision and streaming with bounce-back walls.

Sources in the paper (Sec. II.A and II.C):
  * moments n^a = sum_p f_p, n^a u^a = sum_p c_p f_p   (moment equations of Sec. II.C)
  * equilibrium f_eq (Eq. kernelf)
  * propagation f_p(r + c_p, t + 1) = f_p(r, t) + Omega_p  (propagation scheme)
  * Omega = -omega_visc (f - f_eq) + S (+ Delta, the noise, off here)  (Eq. kernelf2)
  * forcing S (Eq. kernelg), added "partially to the currents" (Guo scheme)
  * drag Phi_drag (Eq. Fidef)

Readings taken where the text is ambiguous (each is listed in the design notes):
  * f_eq is evaluated with the species' own velocity u^a, not with u^a - u
    (with u^a - u the total first moment would vanish, so momentum could not
    be carried at all);
  * Guo forcing: the velocity entering f_eq and S is shifted by half the force,
    u^a = j^a / n^a + Phi^a / 2, and S is scaled by (1 - omega/2);
  * the drag depends on u^a, which with the half-force shift is implicit; for
    equal masses sum_b (n^b/n)(u^a - u^b) = u^a - ubar with ubar the
    number-weighted mean, and the implicit system has the closed form
    implemented in `species_velocities`;
  * walls: halfway bounce-back on every link that points into a solid site;
    all three axes are periodic.

Arrays: populations f[species, p, z, y, x]; vectors v[..., 3, z, y, x] hold
(x, y, z) components.  Everything is float64.
"""
import numpy as np

from . import d3q19 as L


def moments(f):
    """Zeroth and first moments of the populations.

    f: [S, 19, Z, Y, X] -> n [S, Z, Y, X], j [S, 3, Z, Y, X] with
    n^a = sum_p f^a_p and j^a = n^a u^a = sum_p c_p f^a_p.
    """
    n = f.sum(axis=1)
    j = np.einsum("pk,spzyx->skzyx", L.C.astype(np.float64), f)
    return n, j


def equilibrium(n, u):
    """Second-order Hermite equilibrium of Eq. kernelf for one species.

    n: [...], u: [3, ...] (the species velocity).  Returns [19, ...]:
      f_eq_p = w_p n [1 + c.u / vT2 + ((c.u)^2 - vT2 u.u) / (2 vT2^2)].
    """
    cu = np.einsum("pk,k...->p...", L.C.astype(np.float64), u)
    uu = (u * u).sum(axis=0)
    w = L.W.reshape((L.Q,) + (1,) * n.ndim)
    return w * n * (1.0 + cu / L.VT2 + (cu * cu - L.VT2 * uu) / (2.0 * L.VT2 ** 2))


def forcing(n, u, phi):
    """Forcing term S of Eq. kernelg for one species.

    n: [...], u, phi: [3, ...] (velocity and force per particle).  Returns
      S_p = w_p n [c.phi / vT2 + ((c.u)(c.phi) - vT2 phi.u) / vT2^2].
    """
    cf = np.einsum("pk,k...->p...", L.C.astype(np.float64), phi)
    cu = np.einsum("pk,k...->p...", L.C.astype(np.float64), u)
    fu = (phi * u).sum(axis=0)
    w = L.W.reshape((L.Q,) + (1,) * n.ndim)
    return w * n * (cf / L.VT2 + (cu * cf - L.VT2 * fu) / L.VT2 ** 2)


def drag_force(n, u, omega_drag):
    """Inter-species drag of Eq. Fidef with unit masses, written out literally.

    n: [S, ...], u: [S, 3, ...], omega_drag: [S].  Returns [S, 3, ...]:
      Phi_drag^a = - omega_drag^a sum_b (n^b / n) (u^a - u^b),  n = sum_b n^b.
    """
    S = n.shape[0]
    ntot = n.sum(axis=0)
    out = np.zeros_like(u)
    for a in range(S):
        acc = np.zeros_like(u[a])
        for b in range(S):
            acc += (n[b] / ntot) * (u[a] - u[b])
        out[a] = -omega_drag[a] * acc
    return out


def species_velocities(n, j, G, omega_drag):
    """Solve the implicit half-force velocity shift including the drag.

    With Guo forcing the velocity used in f_eq and S is
        u^a = j^a / n^a + Phi^a / 2,   Phi^a = G^a + Phi_drag^a(u),
    where G^a is every force per particle except the drag.  For unit masses
    Phi_drag^a = -omega_drag^a (u^a - ubar), ubar = sum_b x^b u^b, x^b = n^b / n.
    Writing a^a = omega_drag^a / 2 and b^a = j^a / n^a + G^a / 2 gives
        u^a  = (b^a + a^a ubar) / (1 + a^a),
        ubar = sum_a x^a b^a / (1 + a^a)  /  sum_a x^a / (1 + a^a).

    n: [S, ...] (all > 0), j, G: [S, 3, ...].  Returns (u, Phi) with Phi the
    total force per particle, both [S, 3, ...].
    """
    S = n.shape[0]
    ntot = n.sum(axis=0)
    x = n / ntot
    a = np.asarray(omega_drag, dtype=np.float64) / 2.0
    b = j / n[:, None] + G / 2.0
    num = np.zeros_like(b[0])
    den = np.zeros_like(ntot)
    for s in range(S):
        num += x[s] * b[s] / (1.0 + a[s])
        den += x[s] / (1.0 + a[s])
    ubar = num / den
    u = np.empty_like(b)
    phi = np.empty_like(b)
    for s in range(S):
        u[s] = (b[s] + a[s] * ubar) / (1.0 + a[s])
        phi[s] = G[s] - 2.0 * a[s] * (u[s] - ubar)
    return u, phi


def collide(f, G, tau, omega_drag, fluid, noise=None):
    """BGK collision with Guo forcing at the fluid sites (Eqs. kernelf2, kernelg).

    f: [S, 19, Z, Y, X] pre-collision populations; G: [S, 3, Z, Y, X] force
    per particle excluding the drag; tau: [S] relaxation times
    (omega_visc = 1 / tau); fluid: bool [Z, Y, X]; noise: optional
    [S, 19, Z, Y, X] stochastic term Delta of Eq. kernelf2.
    Returns f* = f - omega (f - f_eq(n, u)) + (1 - omega/2) S(n, u, Phi)
    (+ Delta) at fluid sites and zero at solid sites, plus (u, Phi).
    """
    S = f.shape[0]
    n, j = moments(f)
    nsafe = np.where(fluid[None], n, 1.0)
    u, phi = species_velocities(nsafe, np.where(fluid[None, None], j, 0.0),
                                np.where(fluid[None, None], G, 0.0), omega_drag)
    out = np.zeros_like(f)
    for s in range(S):
        omega = 1.0 / tau[s]
        feq = equilibrium(nsafe[s], u[s])
        src = forcing(nsafe[s], u[s], phi[s])
        out[s] = f[s] - omega * (f[s] - feq) + (1.0 - 0.5 * omega) * src
        if noise is not None:
            out[s] += noise[s]
    out *= fluid[None, None]
    return out, u, phi


def stream(fstar, solid):
    """Propagation with halfway bounce-back; periodic in x, y and z.

    f_p(r, t+1) = f*_p(r - c_p)      if r - c_p is a fluid site,
                = f*_opp(p)(r)        otherwise (the population that left r
                                      along -c_p towards the wall returns),
    and populations of solid sites are zero.
    """
    fluid = ~solid
    out = np.zeros_like(fstar)
    for p in range(L.Q):
        cx, cy, cz = (int(v) for v in L.C[p])
        shift = (cz, cy, cx)
        pulled = np.roll(fstar[:, p], shift, axis=(-3, -2, -1))
        src_solid = np.roll(solid, shift, axis=(-3, -2, -1))
        out[:, p] = np.where(src_solid[None], fstar[:, L.OPP[p]], pulled)
    out *= fluid[None, None]
    return out


def init_equilibrium(n0, solid):
    """Populations at rest: f_p = w_p n0 on fluid sites, zero on solid sites.

    n0: [S, Z, Y, X] initial densities.  (Step-0 initialisation of the
    algorithm of Fig. 1: populations are set and moments computed from them.)
    """
    f = L.W[None, :, None, None, None] * n0[:, None]
    return f * (~solid)[None, None]
