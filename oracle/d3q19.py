"""D3Q19 lattice constants (oracle side; test infrastructure only).

The paper uses the D3Q19 discretization with q = 19 PDFs per node
(Sect. 2 and Sect. 4). It does not list the velocity order or the weights;
this order is a reading (rest, the six axis directions, then the twelve
face diagonals, each followed by its opposite), and the weights are the
standard D3Q19 ones: 1/3, 1/18 and 1/36.
"""

import numpy as np

#: lattice velocities c_q, q = 0..18
C = np.array([
    (0, 0, 0),
    (1, 0, 0), (-1, 0, 0),
    (0, 1, 0), (0, -1, 0),
    (0, 0, 1), (0, 0, -1),
    (1, 1, 0), (-1, -1, 0),
    (1, -1, 0), (-1, 1, 0),
    (1, 0, 1), (-1, 0, -1),
    (1, 0, -1), (-1, 0, 1),
    (0, 1, 1), (0, -1, -1),
    (0, 1, -1), (0, -1, 1),
], dtype=np.int64)

Q = 19

#: weights, each one IEEE division
W = [1.0 / 3.0] + [1.0 / 18.0] * 6 + [1.0 / 36.0] * 12


def _opposite():
    out = []
    for q in range(Q):
        hits = [k for k in range(Q) if all(C[k] == -C[q])]
        assert len(hits) == 1
        out.append(hits[0])
    return out


#: index of the direction opposite to q (c_OPP[q] = -c_q)
OPP = _opposite()
