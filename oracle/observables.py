"""Pore observables of the translocation study (Sec. IV): the ionic current
through a plane of the pore (Sec. IV.B, from which the conductance G = I /
Delta V follows) and the time at which each bead passes a plane, e.g. the
pore's mid-plane (Sec. IV.C).

Test infrastructure: a plain float64 reference used only by the tests, the
smoke check and the benchmark's CPU baseline, never by the library.

Definitions (the paper measures both but gives no formula; the readings are
listed in the design notes):
  * plane flux: the particles of a species that one propagation step carried
    across the link plane between z and z + 1 (z + 1 taken periodically),
    counted +1 in +z and -1 in -z.  A population crosses when it streams
    from a fluid site on one side to a fluid site on the other; a population
    aimed at a solid site is bounced back and stays.  The charge current is
    sum_a z^a times the species flux.
  * bead crossing: a bead crosses the plane z = z_plane (or one of its
    periodic images z_plane + k L_z) in a step when floor((Z - z_plane) / L_z)
    differs between its z coordinate Z before and after the step; per bead
    the first and last such step (steps counted from 1; -1 if none) and the
    net count (+1 for a crossing in +z, -1 in -z).
"""
import numpy as np

from . import d3q19 as L


def plane_flux(f, solid, z):
    """Species fluxes across the link plane between z and z + 1.

    f: populations of time t AFTER propagation, [S, 19, Z, Y, X] (as kept by
    `step.Simulation`); solid: bool [Z, Y, X].  A population f_p(r) at a fluid
    site r whose source r - c_p is fluid arrived by streaming from r - c_p; it
    crossed the plane if r - c_p and r lie on opposite sides of it.
    Returns [S] float64.
    """
    nz = solid.shape[0]
    zu = (z + 1) % nz
    out = np.zeros(f.shape[0])
    for p in range(L.Q):
        cx, cy, cz = (int(v) for v in L.C[p])
        if cz == 0:
            continue
        # destination plane of the crossing populations, and their source plane
        dest = zu if cz == 1 else z
        src = z if cz == 1 else zu
        sign = 1.0 if cz == 1 else -1.0
        # source of (x, y) on the destination plane: (x - cx, y - cy) on src
        src_solid = np.roll(solid[src], (cy, cx), axis=(0, 1))
        open_link = ~solid[dest] & ~src_solid
        out += sign * np.where(open_link[None], f[:, p, dest], 0.0).sum(axis=(1, 2))
    return out


def charge_current(flux, valence):
    """sum_a z^a flux^a: the charge carried across the plane per step."""
    return float(np.dot(np.asarray(valence, dtype=np.float64), flux))


def bead_crossings(z_hist, z_plane, Lz):
    """First / last crossing step and net count per bead.

    z_hist: [T + 1, N] bead z coordinates at steps 0 .. T (unwrapped).
    Returns (first [N], last [N], net [N]) int arrays.
    """
    z_hist = np.asarray(z_hist, dtype=np.float64)
    k = np.floor((z_hist - z_plane) / Lz)
    n = z_hist.shape[1]
    first = np.full(n, -1, dtype=np.int64)
    last = np.full(n, -1, dtype=np.int64)
    net = np.zeros(n, dtype=np.int64)
    for t in range(1, z_hist.shape[0]):
        for i in range(n):
            if k[t, i] != k[t - 1, i]:
                if first[i] < 0:
                    first[i] = t
                last[i] = t
                net[i] += 1 if k[t, i] > k[t - 1, i] else -1
    return first, last, net
