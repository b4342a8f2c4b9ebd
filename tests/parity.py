"""Error measures used by the GPU-vs-oracle tests.

Densities: max over sites of |n_gpu - n_ref| / n_ref (fluid sites).
Velocities: max |u_gpu - u_ref| / max |u_ref| per species (a pointwise
relative error is meaningless where the flow vanishes).
Potential: max |psi_gpu - psi_ref| / max |psi_ref|.
"""
import numpy as np


def density_error(n_gpu, n_ref, fluid):
    return float(np.max(np.abs(n_gpu - n_ref)[..., fluid] / np.abs(n_ref)[..., fluid]))


def velocity_error(u_gpu, u_ref, fluid):
    scale = np.max(np.abs(u_ref[..., fluid]))
    if scale == 0.0:
        return float(np.max(np.abs(u_gpu[..., fluid])))
    return float(np.max(np.abs(u_gpu - u_ref)[..., fluid]) / scale)


def field_error(a, b):
    scale = np.max(np.abs(b))
    return float(np.max(np.abs(a - b)) / scale) if scale > 0 else float(np.max(np.abs(a)))


def bf16_round(a):
    """Round to the nearest bfloat16 (ties to even), returned as float64: the
    top 16 bits of the float32 pattern after adding half an ulp of bfloat16."""
    f = np.ascontiguousarray(a, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def rel_l2(a, b):
    """||a - b|| / ||b||."""
    nb = float(np.linalg.norm(np.ravel(b)))
    return float(np.linalg.norm(np.ravel(a) - np.ravel(b))) / (nb if nb > 0 else 1.0)
