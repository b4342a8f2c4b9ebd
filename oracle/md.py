"""Bead-spring polymer: Langevin beads coupled to the fluid species by friction
(Sec. II.B) and the interpolation / extrapolation kernel that joins the
Lagrangian beads with the lattice (Sec. II.C, last paragraph).

Readings taken (listed with the others in the design notes):
  * kernel: trilinear over the 8 lattice nodes around a bead (nodes sit at
    integer coordinates); for the fluid velocity and composition, and for the
    spreading of the friction back onto the fluid, the weights are
    renormalised over the fluid corners; the electric field and the bead charge
    use the plain weights (the potential exists on every site);
  * friction from species a on bead i:  phi_i^a = gamma x^a(R_i) (u^a(R_i) - V_i),
    with x^a = n^a / n the local number fraction, so that the three species
    together exert gamma (ubar - V_i); the fluid receives the opposite impulse
    as a force density spread with the same weights;
  * coupling kernel: the trilinear kernel above, or (poly["coupling"] ==
    "theta") the occupation cube theta_i of Eq. totalforcefluid, the nodes
    within the cube of side sigma around the bead, each with the same
    weight, renormalised over the fluid nodes of the cube so that
    sum_r theta_i(r) = 1 (the friction the fluid receives then equals the
    bead's); it replaces the trilinear weights for the fluid velocity and
    composition at the bead and for the spreading of the friction, while
    the bead charge and the field keep the trilinear weights;
  * fluid fields seen by the beads over the MD substeps of one lattice step:
    densities from the populations at time t, and node velocities
    (j^a + K^a) / n^a, where j^a is the momentum of the populations at time t
    and K^a the momentum the beads have already handed to species a at that
    node in the earlier substeps of the same step.  The exchange is thus
    resolved at the substep, which keeps a stiff chain with strong friction
    stable (with the nodes frozen for the whole subcycle, the fluid would get
    the full exchange at once and overshoot whenever gamma times the kernel's
    self-weight exceeds the local fluid density by a factor of about two);
  * conservative forces: FENE bonds between chain neighbours,
    U = -k R0^2 / 2 ln(1 - (r / R0)^2), a purely repulsive WCA between all
    pairs; or, with poly["bond"] == "harmonic", the bonds of Eq.
    polymermodel, U = k (r - l_bond)^2 / 2, and the WCA only between beads
    more than one apart along the chain (|i - j| > 1); the same WCA between
    a bead and the centres of boundary solid sites,
    and the electric force q_i E(R_i) with E = -grad psi + E_ext (the text's
    "+ q_i grad psi" is read as the usual -q_i grad psi), interpolated once
    per lattice step at the position R_i(t) where the bead's charge was
    deposited for that step's Poisson solve (the paper solves Eq. poisson
    once per lattice step for the forces on the fluid and on the molecule,
    Sec. II.C, then subcycles the molecule): deposit and interpolation then
    use the same weights, so the electrostatic forces on ions, walls and
    beads sum to zero and a bead never feels its own deposited charge, which
    sampling the frozen field along the substeps would make it do;
  * integrator: n_sub substeps of h = 1 / n_sub per lattice step,
    V += h (F + sum_a phi^a) / M, then R += h V (semi-implicit Euler);
  * thermal noise (optional): xi ~ N(0, 2 gamma k_B T / h) per component and
    substep from the counter-based generator of noise.py, added to the
    friction of each species in proportion to its number fraction,
    phi^a += x^a xi, so that the bead receives the whole xi and the fluid
    the opposite impulse.
Positions are unwrapped; lattice indices and pair separations use the periodic
box (minimum image).
"""
import numpy as np

from . import d3q19 as L
from . import noise

WCA_CUT = 2.0 ** (1.0 / 6.0)


def trilinear(R, shape):
    """Trilinear corner nodes and weights.

    R: [N, 3] positions (x, y, z); shape: (Z, Y, X).  Returns
    idx [N, 8, 3] integer (x, y, z) node indices wrapped into the box and
    w [N, 8] weights; corner k has offsets ((k>>0)&1, (k>>1)&1, (k>>2)&1).
    """
    Z, Y, X = shape
    box = np.array([X, Y, Z])
    i0 = np.floor(R).astype(np.int64)
    d = R - i0
    N = R.shape[0]
    idx = np.empty((N, 8, 3), dtype=np.int64)
    w = np.empty((N, 8))
    for k in range(8):
        o = np.array([(k >> 0) & 1, (k >> 1) & 1, (k >> 2) & 1])
        idx[:, k] = np.mod(i0 + o, box)
        wk = np.ones(N)
        for a in range(3):
            wk = wk * (d[:, a] if o[a] else (1.0 - d[:, a]))
        w[:, k] = wk
    return idx, w


def theta_weights(R, shape, sigma):
    """Occupation cube of Eq. totalforcefluid: theta_i(r) = 1 for the
    lattice nodes r with R_i - sigma/2 < r <= R_i + sigma/2 in every axis
    (the cube of side sigma around the bead), 0 elsewhere.  For
    1 <= sigma <= 2 these nodes are among the 8 corners of the bead's cell:
    returns the corner indices of `trilinear` and the indicator [N, 8]."""
    idx, _ = trilinear(R, shape)
    i0 = np.floor(R)
    w = np.ones((R.shape[0], 8))
    for k in range(8):
        for a in range(3):
            node = i0[:, a] + ((k >> a) & 1)
            inside = (node - R[:, a] > -0.5 * sigma) & (node - R[:, a] <= 0.5 * sigma)
            w[:, k] *= inside
    return idx, w


def gather(field, idx):
    """field [..., Z, Y, X] at nodes idx [N, 8, 3] -> [..., N, 8]."""
    return field[..., idx[..., 2], idx[..., 1], idx[..., 0]]


def minimum_image(d, box):
    return d - box * np.round(d / box)


def fene_energy(R, box, k, R0):
    d = minimum_image(R[1:] - R[:-1], box)
    r2 = (d * d).sum(axis=1)
    return float(np.sum(-0.5 * k * R0 * R0 * np.log(1.0 - r2 / (R0 * R0))))


def fene_forces(R, box, k, R0):
    """-grad of the FENE energy over the chain bonds (i, i+1)."""
    F = np.zeros_like(R)
    d = minimum_image(R[1:] - R[:-1], box)      # from i to i+1
    r2 = (d * d).sum(axis=1)
    if np.any(r2 >= R0 * R0):
        raise FloatingPointError("FENE bond stretched beyond R0")
    coef = k / (1.0 - r2 / (R0 * R0))          # force on i is +coef * d
    F[:-1] += coef[:, None] * d
    F[1:] -= coef[:, None] * d
    return F


def harmonic_energy(R, box, k, l):
    d = minimum_image(R[1:] - R[:-1], box)
    r = np.sqrt((d * d).sum(axis=1))
    return float(np.sum(0.5 * k * (r - l) ** 2))


def harmonic_forces(R, box, k, l):
    """-grad of the harmonic bond energy over the chain bonds (i, i+1)."""
    F = np.zeros_like(R)
    d = minimum_image(R[1:] - R[:-1], box)      # from i to i+1
    r = np.sqrt((d * d).sum(axis=1))
    coef = k * (r - l) / r                      # force on i is +coef * d
    F[:-1] += coef[:, None] * d
    F[1:] -= coef[:, None] * d
    return F


def wca_energy(R, box, eps, sigma, skip_bonded=False):
    N = R.shape[0]
    e = 0.0
    for i in range(N):
        for j in range(i + 1, N):
            if skip_bonded and j == i + 1:
                continue
            d = minimum_image(R[j] - R[i], box)
            r = np.sqrt((d * d).sum())
            if r < WCA_CUT * sigma:
                sr6 = (sigma / r) ** 6
                e += 4.0 * eps * (sr6 * sr6 - sr6) + eps
    return e


def wca_pair_forces(R, box, eps, sigma, skip_bonded=False):
    """Repulsive WCA between every pair of beads (minimum image); with
    skip_bonded not between chain neighbours."""
    d = minimum_image(R[:, None, :] - R[None, :, :], box)   # R_i - R_j
    r2 = (d * d).sum(axis=2)
    np.fill_diagonal(r2, np.inf)
    if skip_bonded:
        i = np.arange(R.shape[0] - 1)
        r2[i, i + 1] = np.inf
        r2[i + 1, i] = np.inf
    inside = r2 < (WCA_CUT * sigma) ** 2
    sr2 = np.where(inside, sigma * sigma / np.where(inside, r2, 1.0), 0.0)
    sr6 = sr2 ** 3
    coef = np.where(inside, 24.0 * eps * (2.0 * sr6 * sr6 - sr6) / np.where(inside, r2, 1.0), 0.0)
    return (coef[:, :, None] * d).sum(axis=1)


def wall_sites(solid):
    """Boundary solid sites: solid sites with at least one fluid site among
    their 18 D3Q19 neighbours.  Returns [M, 3] (x, y, z) coordinates."""
    fluid = ~solid
    near_fluid = np.zeros_like(solid)
    for p in range(1, L.Q):
        cx, cy, cz = (int(v) for v in L.C[p])
        near_fluid |= np.roll(fluid, (-cz, -cy, -cx), axis=(-3, -2, -1))
    zz, yy, xx = np.nonzero(solid & near_fluid)
    return np.stack([xx, yy, zz], axis=1).astype(np.float64)


def wall_forces(R, walls, box, eps, sigma):
    """WCA between each bead and every boundary solid site centre."""
    F = np.zeros_like(R)
    if walls.shape[0] == 0:
        return F
    for i in range(R.shape[0]):
        d = minimum_image(R[i][None, :] - walls, box)
        r2 = (d * d).sum(axis=1)
        inside = r2 < (WCA_CUT * sigma) ** 2
        if not np.any(inside):
            continue
        r2i = r2[inside]
        sr6 = (sigma * sigma / r2i) ** 3
        coef = 24.0 * eps * (2.0 * sr6 * sr6 - sr6) / r2i
        F[i] += (coef[:, None] * d[inside]).sum(axis=0)
    return F


def wall_energy(R, walls, box, eps, sigma):
    e = 0.0
    for i in range(R.shape[0]):
        d = minimum_image(R[i][None, :] - walls, box)
        r = np.sqrt((d * d).sum(axis=1))
        r = r[r < WCA_CUT * sigma]
        sr6 = (sigma / r) ** 6
        e += float(np.sum(4.0 * eps * (sr6 * sr6 - sr6) + eps))
    return e


def deposit_charge(R, q, shape, fluid=None):
    """Bead charge on the lattice: sum_i q_i W(r - R_i), plain trilinear
    weights, or with `fluid` the weights renormalised over the fluid corners
    (insulating walls: the solid holds no potential)."""
    rho = np.zeros(shape)
    idx, w = trilinear(R, shape)
    if fluid is not None:
        fl = gather(fluid, idx).astype(np.float64)
        w = w * fl / (w * fl).sum(axis=1, keepdims=True)
    np.add.at(rho, (idx[..., 2], idx[..., 1], idx[..., 0]), q[:, None] * w)
    return rho


def md_substeps(R, V, n, j, E, fluid, walls, poly, thermal=None, field_on_fluid=False):
    """Advance the beads over one lattice step and spread the friction.

    R, V: [N, 3]; n: [S, Z, Y, X] and j: [S, 3, Z, Y, X] from the populations
    at time t; E: [3, Z, Y, X] nodal field including E_ext; fluid: bool
    [Z, Y, X]; walls: [M, 3] boundary site centres; poly: dict with keys
    M, q [N], k_fene, R0, eps, sigma, gamma, n_sub (and optionally bond =
    "harmonic" with k_bond, l_bond).

    thermal: optional (seed, step, kT) switching on the bead noise of this
    lattice step.  field_on_fluid: interpolate the field with the weights
    renormalised over the fluid corners (insulating walls, where the bead
    charge is deposited with those weights too).

    Returns (R, V, K) with K [S, 3, Z, Y, X] the force density on each species
    accumulated over the substeps (the fluid's share of the friction).
    """
    shape = n.shape[1:]
    Z, Y, X = shape
    box = np.array([X, Y, Z], dtype=np.float64)
    S = n.shape[0]
    h = 1.0 / poly["n_sub"]
    gamma = poly["gamma"]
    M = poly["M"]
    q = np.asarray(poly["q"], dtype=np.float64)
    ntot = n.sum(axis=0)
    K = np.zeros((S, 3) + shape)
    R = np.array(R, dtype=np.float64, copy=True)
    V = np.array(V, dtype=np.float64, copy=True)
    # electric force with the plain weights at the positions of the deposit
    idx0, w0 = trilinear(R, shape)
    if field_on_fluid:
        fl0 = gather(fluid, idx0).astype(np.float64)
        w0 = w0 * fl0 / (w0 * fl0).sum(axis=1, keepdims=True)
    F_el = q[:, None] * (w0[None] * gather(E, idx0)).sum(axis=-1).T           # [N, 3]
    theta = poly.get("coupling", "trilinear") == "theta"
    for sub in range(poly["n_sub"]):
        if theta:
            idx, w = theta_weights(R, shape, poly["sigma"])
        else:
            idx, w = trilinear(R, shape)
        fl = gather(fluid, idx).astype(np.float64)
        wsum = (w * fl).sum(axis=1)
        if np.any(wsum <= 0.0):
            raise FloatingPointError("bead with no fluid corner")
        wt = w * fl / wsum[:, None]
        nc = gather(n, idx)                                   # [S, N, 8]
        nsafe = np.where(fl[None] > 0, nc, 1.0)
        # node momentum: populations at time t plus what the beads have
        # given to the species during the earlier substeps of this step
        jc = gather(j + K, idx)                               # [S, 3, N, 8]
        u_b = (wt[None, None] * jc / nsafe[:, None]).sum(axis=-1)        # [S, 3, N]
        ntc = np.where(fl > 0, gather(ntot, idx), 1.0)
        x_b = (wt[None] * nc / ntc[None]).sum(axis=-1)                    # [S, N]

        harmonic = poly.get("bond", "fene") == "harmonic"
        if harmonic:
            F = harmonic_forces(R, box, poly["k_bond"], poly["l_bond"])
        else:
            F = fene_forces(R, box, poly["k_fene"], poly["R0"])
        F += wca_pair_forces(R, box, poly["eps"], poly["sigma"], skip_bonded=harmonic)
        F += wall_forces(R, walls, box, poly["eps"], poly["sigma"])
        F += F_el

        phi = gamma * x_b[:, :, None] * (np.transpose(u_b, (0, 2, 1)) - V[None])   # [S, N, 3]
        if thermal is not None:
            seed, tstep, kT = thermal
            xi = np.sqrt(2.0 * gamma * kT / h) * noise.bead_normals(R.shape[0], tstep, sub, seed)
            phi = phi + x_b[:, :, None] * xi[None]
        V = V + h * (F + phi.sum(axis=0)) / M
        R = R + h * V
        for s in range(S):
            for c in range(3):
                np.add.at(K[s, c], (idx[..., 2], idx[..., 1], idx[..., 0]),
                          -h * phi[s][:, c][:, None] * wt)
    return R, V, K
