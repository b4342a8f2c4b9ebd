"""Poisson equation for the electrostatic potential (Eq. poisson) and its
solution by red-black successive over-relaxation with Chebyshev acceleration
(Sec. II.C, last paragraphs; the SOR routine of the cited Numerical Recipes).

Readings taken (the paper names the method but not its discretisation):
  * 7-point Laplacian A_h on the whole periodic box with uniform permittivity,
    solid sites included (wall charges sit on boundary solid sites);
  * the periodic problem needs a neutral right-hand side, so the mean of the
    charge density is removed and the gauge is fixed by mean(psi) = 0;
  * right-hand side b = -(rho_e - mean(rho_e)) / eps, A_h psi = b;
  * red sites are those with x + y + z even, updated first; every box side
    must be even so that the colouring is consistent across the periodic
    faces;
  * Chebyshev schedule: omega = 1 for the first half sweep, then
    omega = 1 / (1 - rho_J^2 / 2), then omega <- 1 / (1 - rho_J^2 omega / 4)
    after every half sweep, restarted for every solve;
  * rho_J is the spectral radius of the Jacobi iteration on the mean-free
    subspace; for the periodic 7-point operator its eigenvalues are
    (cos kx + cos ky + cos kz) / 3 and the largest one below 1 (the constant
    mode is the null space; its red-black partner, the checkerboard, is
    annihilated by the red-black ordering) is (2 + cos(2 pi / N_max)) / 3;
  * stop when ||b - A_h psi||_2 / ||b||_2 <= tol, checked after every full
    iteration (red + black); b == 0 gives psi = 0.
"""
import numpy as np


def laplacian(psi):
    """7-point periodic Laplacian (sum of the six neighbours minus 6 psi)."""
    out = -6.0 * psi
    for ax in (-3, -2, -1):
        out = out + np.roll(psi, 1, axis=ax) + np.roll(psi, -1, axis=ax)
    return out


def neighbour_sum(psi):
    s = np.zeros_like(psi)
    for ax in (-3, -2, -1):
        s = s + np.roll(psi, 1, axis=ax) + np.roll(psi, -1, axis=ax)
    return s


def rhs_from_charge(rho_e, eps):
    """b = -(rho_e - mean rho_e) / eps, so that A_h psi = b approximates
    laplacian(psi) = -rho_e / eps on the periodic box."""
    return -(rho_e - rho_e.mean()) / eps


def relative_residual(psi, b):
    """||b - A_h psi||_2 / ||b||_2 in float64 (0 if b is zero and psi solves it)."""
    r = b - laplacian(psi)
    bn = np.sqrt((b * b).sum())
    rn = np.sqrt((r * r).sum())
    if bn == 0.0:
        return 0.0 if rn == 0.0 else np.inf
    return rn / bn


def jacobi_radius(shape):
    """Largest Jacobi eigenvalue below 1 of the periodic 7-point operator."""
    nmax = max(shape)
    return (2.0 + np.cos(2.0 * np.pi / nmax)) / 3.0


def red_mask(shape):
    z, y, x = np.indices(shape)
    return (x + y + z) % 2 == 0


class NotConverged(RuntimeError):
    pass


def sor_red_black_chebyshev(b, psi0, tol, max_iter, rho_j=None, iterations=None):
    """Red-black SOR with Chebyshev acceleration.

    b, psi0: [Z, Y, X] float64.  Runs until the relative residual is <= tol
    (checked before the first iteration and after every full iteration), or,
    if `iterations` is given, exactly that many full iterations with no test.
    Returns (psi, iterations_done, relative_residual).  The mean of psi is
    removed after convergence (not when `iterations` is given, so that
    iterates can be compared one by one).
    Raises NotConverged when max_iter full iterations do not reach tol.
    """
    shape = b.shape
    assert all(n % 2 == 0 for n in shape), "red-black ordering needs even sides"
    if rho_j is None:
        rho_j = jacobi_radius(shape)
    red = red_mask(shape)
    black = ~red
    psi = np.array(psi0, dtype=np.float64, copy=True)

    if iterations is None:
        if not np.any(b):
            return np.zeros_like(b), 0, 0.0
        rr = relative_residual(psi, b)
        if rr <= tol:
            return psi - psi.mean(), 0, rr
        n_max = max_iter
    else:
        n_max = iterations

    omega = 1.0
    done = 0
    for it in range(n_max):
        for half, colour in enumerate((red, black)):
            gs = (neighbour_sum(psi) - b) / 6.0
            psi = np.where(colour, psi + omega * (gs - psi), psi)
            if it == 0 and half == 0:
                omega = 1.0 / (1.0 - 0.5 * rho_j * rho_j)
            else:
                omega = 1.0 / (1.0 - 0.25 * rho_j * rho_j * omega)
        done = it + 1
        if iterations is None:
            rr = relative_residual(psi, b)
            if rr <= tol:
                return psi - psi.mean(), done, rr
    if iterations is not None:
        return psi, done, relative_residual(psi, b)
    raise NotConverged(f"red-black SOR did not reach {tol} in {max_iter} iterations "
                       f"(residual {relative_residual(psi, b):.3e})")


def electric_field(psi, E_ext):
    """E = -grad_h psi (central differences, periodic) + E_ext.

    Returns [3, Z, Y, X] with (x, y, z) components."""
    E = np.empty((3,) + psi.shape)
    for k, ax in enumerate((-1, -2, -3)):
        E[k] = -(np.roll(psi, -1, axis=ax) - np.roll(psi, 1, axis=ax)) / 2.0 + E_ext[k]
    return E


# ---------------------------------------------------------------------------
# Insulating walls (the Neumann condition after Eq. poisson): the potential
# lives on the fluid sites only; across a face between a fluid site and a
# solid site the normal derivative is fixed by the wall's surface charge,
# -grad psi . n = Sigma / eps with n the normal pointing into the fluid.
# Readings taken:
#   * finite volumes on the lattice cells: for a fluid site r,
#       sum over fluid face neighbours (psi_nb - psi_r)
#         = -(rho_r + sum over its wall faces Sigma_f) / eps,
#     i.e. each wall face's flux Sigma_f / eps enters the balance of the
#     fluid cell it bounds;
#   * the surface charge of a face is that of its solid site divided over
#     the solid site's fluid face neighbours: Sigma_f = q_w / k_w (a charged
#     solid site with no fluid face neighbour is an error);
#   * the periodic fluid domain with zero-flux walls leaves psi defined up
#     to a constant: the fluid mean of the charge is removed and the fluid
#     mean of psi is set to zero;
#   * the field at a fluid site is the central difference with the ghost
#     value psi_r + Sigma_f / eps in place of a solid face neighbour (the
#     face's prescribed flux), and zero at solid sites.
# ---------------------------------------------------------------------------
_FACES = ((-1, 1), (-1, -1), (-2, 1), (-2, -1), (-3, 1), (-3, -1))   # (axis, shift)


def open_faces(fluid):
    """Number of fluid face neighbours of every site."""
    k = np.zeros(fluid.shape)
    for ax, sh in _FACES:
        k += np.roll(fluid, sh, axis=ax)
    return k


def face_charge(wall_q, solid):
    """Sigma_f of the faces of every solid site: q_w / k_w (0 elsewhere)."""
    k = open_faces(~solid)
    charged = solid & (wall_q != 0.0)
    if np.any(charged & (k == 0)):
        raise ValueError("a charged solid site has no fluid face neighbour")
    return np.where(charged, wall_q / np.where(k > 0, k, 1.0), 0.0)


def neumann_laplacian(psi, fluid):
    """sum over fluid face neighbours of (psi_nb - psi_r) at fluid sites, 0
    at solid sites."""
    out = np.zeros_like(psi)
    for ax, sh in _FACES:
        nb_fluid = np.roll(fluid, sh, axis=ax)
        out += np.where(nb_fluid, np.roll(psi, sh, axis=ax) - psi, 0.0)
    return np.where(fluid, out, 0.0)


def neumann_rhs(rho, wall_q, solid, eps):
    """b with A_N psi = b: b = -(rho + s - mean_fluid(rho + s)) / eps at fluid
    sites, s = the surface charge of the site's wall faces; 0 at solid
    sites.  rho: charge density of the fluid sites (values on solid sites
    are ignored)."""
    fluid = ~solid
    sig = face_charge(wall_q, solid)
    s = np.zeros_like(rho)
    for ax, sh in _FACES:
        s += np.roll(sig, sh, axis=ax)
    tot = np.where(fluid, rho + s, 0.0)
    mean = tot.sum() / fluid.sum()
    return np.where(fluid, -(tot - mean) / eps, 0.0)


def neumann_relative_residual(psi, b, fluid):
    r = np.where(fluid, b - neumann_laplacian(psi, fluid), 0.0)
    bn = np.sqrt((b * b).sum())
    rn = np.sqrt((r * r).sum())
    if bn == 0.0:
        return 0.0 if rn == 0.0 else np.inf
    return rn / bn


def sor_neumann(b, psi0, fluid, tol, max_iter, rho_j=None, iterations=None):
    """Red-black SOR with the Chebyshev schedule of sor_red_black_chebyshev on
    the fluid sites: psi_r <- psi_r + omega ((sum over fluid face neighbours
    psi_nb - b_r) / k_r - psi_r), k_r the number of fluid face neighbours.
    Stops when the relative residual over the fluid is <= tol (tested before
    the first and after every full iteration); removes the fluid mean of psi.
    Returns (psi, iterations, residual); psi is 0 on solid sites."""
    shape = b.shape
    assert all(n % 2 == 0 for n in shape), "red-black ordering needs even sides"
    k = open_faces(fluid)
    if np.any(fluid & (k == 0)):
        raise ValueError("a fluid site has no fluid face neighbour")
    if rho_j is None:
        rho_j = jacobi_radius(shape)
    red = red_mask(shape) & fluid
    black = ~red_mask(shape) & fluid
    psi = np.where(fluid, np.array(psi0, dtype=np.float64), 0.0)
    kk = np.where(fluid, k, 1.0)

    def gauge(p):
        return np.where(fluid, p - p[fluid].mean(), 0.0)

    if iterations is None:
        if not np.any(b):
            return np.zeros_like(b), 0, 0.0
        rr = neumann_relative_residual(psi, b, fluid)
        if rr <= tol:
            return gauge(psi), 0, rr
        n_max = max_iter
    else:
        n_max = iterations
    omega = 1.0
    done = 0
    for it in range(n_max):
        for half, colour in enumerate((red, black)):
            nbsum = np.zeros_like(psi)
            for ax, sh in _FACES:
                nbsum += np.where(np.roll(fluid, sh, axis=ax), np.roll(psi, sh, axis=ax), 0.0)
            gs = (nbsum - b) / kk
            psi = np.where(colour, psi + omega * (gs - psi), psi)
            if it == 0 and half == 0:
                omega = 1.0 / (1.0 - 0.5 * rho_j * rho_j)
            else:
                omega = 1.0 / (1.0 - 0.25 * rho_j * rho_j * omega)
        done = it + 1
        if iterations is None:
            rr = neumann_relative_residual(psi, b, fluid)
            if rr <= tol:
                return gauge(psi), done, rr
    if iterations is not None:
        return psi, done, neumann_relative_residual(psi, b, fluid)
    raise NotConverged(f"Neumann SOR did not reach {tol} in {max_iter} iterations")


def electric_field_neumann(psi, solid, wall_q, eps, E_ext):
    """E = -grad_h psi + E_ext at fluid sites, the central difference taking
    psi_r + Sigma_f / eps for a solid face neighbour; zero at solid sites."""
    fluid = ~solid
    sig = face_charge(wall_q, solid)
    E = np.zeros((3,) + psi.shape)
    for k, ax in enumerate((-1, -2, -3)):
        up = np.where(np.roll(fluid, -1, axis=ax), np.roll(psi, -1, axis=ax),
                      psi + np.roll(sig, -1, axis=ax) / eps)
        dn = np.where(np.roll(fluid, 1, axis=ax), np.roll(psi, 1, axis=ax),
                      psi + np.roll(sig, 1, axis=ax) / eps)
        E[k] = np.where(fluid, -(up - dn) / 2.0 + E_ext[k], 0.0)
    return E
