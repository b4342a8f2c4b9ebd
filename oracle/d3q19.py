"""D3Q19 velocity set and weights (Sec. II.C, "Discretization procedure").

One rest velocity, six of length 1 along the axes and twelve of length sqrt(2)
along the face diagonals; lattice spacing and time step are 1.  The weights are
the standard D3Q19 Gaussian weights 1/3, 1/18, 1/36 and the thermal velocity
squared is v_T^2 = 1/3 (the lattice sound speed).

Vectors are stored as (cx, cy, cz).  Fields are stored with x fastest, i.e. an
array index [z, y, x].  The ordering below is the population order used by
the library's public headers; the oracle defines it independently.
"""
import numpy as np

C = np.array([
    [0, 0, 0],
    [1, 0, 0], [-1, 0, 0], [0, 1, 0], [0, -1, 0], [0, 0, 1], [0, 0, -1],
    [1, 1, 0], [-1, -1, 0], [1, -1, 0], [-1, 1, 0],
    [1, 0, 1], [-1, 0, -1], [1, 0, -1], [-1, 0, 1],
    [0, 1, 1], [0, -1, -1], [0, 1, -1], [0, -1, 1],
], dtype=np.int64)

Q = 19

W = np.array([1.0 / 3.0] + [1.0 / 18.0] * 6 + [1.0 / 36.0] * 12, dtype=np.float64)

# thermal velocity squared of the lattice, v_T^2 (Eq. kernelf)
VT2 = 1.0 / 3.0


def _opposite():
    opp = np.empty(Q, dtype=np.int64)
    for p in range(Q):
        matches = [q for q in range(Q) if np.all(C[q] == -C[p])]
        assert len(matches) == 1
        opp[p] = matches[0]
    return opp


OPP = _opposite()
