"""Independent helpers for the oracle pins (test code only).

Nothing here is shared with the oracle's arithmetic: the golden tables are
read from the paper's transcription, J is evaluated from the shape-function
gradients of Appendix A (not from the edge-vector blends the oracle uses), and
the Bernstein collocation matrix is built from the definition in Section 3.1.
"""
import os
import re
from fractions import Fraction
from itertools import permutations, product

import numpy as np

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")

# Fig. 3 node positions (half-steps) -- typed in again here from the figure's
# description so that an ordering mistake in the oracle is caught.
FIG3 = {
    1: (0, 0, 0), 2: (2, 0, 0), 3: (2, 2, 0), 4: (0, 2, 0),
    5: (0, 0, 2), 6: (2, 0, 2), 7: (2, 2, 2), 8: (0, 2, 2),
}
# edge midpoints 9..20 between corner pairs, faces 21..26, centre 27
FIG3_EDGES = [(1, 2), (2, 3), (3, 4), (4, 1), (1, 5), (2, 6), (3, 7), (4, 8),
              (5, 6), (6, 7), (7, 8), (8, 5)]
for _i, (_p, _q) in enumerate(FIG3_EDGES):
    FIG3[9 + _i] = tuple((a + b) // 2 for a, b in zip(FIG3[_p], FIG3[_q]))
FIG3[21] = (1, 1, 0)   # zeta = 0
FIG3[22] = (1, 0, 1)   # eta = 0
FIG3[23] = (2, 1, 1)   # xi = 1
FIG3[24] = (1, 2, 1)   # eta = 1
FIG3[25] = (0, 1, 1)   # xi = 0
FIG3[26] = (1, 1, 2)   # zeta = 1
FIG3[27] = (1, 1, 1)
NODES = [FIG3[a] for a in range(1, 28)]


def read_table(name, nrows, ncols, first_row=1):
    """Parse a transcribed table into a Fraction matrix."""
    M = [[Fraction(0)] * ncols for _ in range(nrows)]
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.split("#", 1)[0].strip()
            if not line:
                continue
            row, rest = line.split(":", 1)
            r = int(row) - first_row
            for tok in rest.split():
                cols, val = tok.split(":")
                v = Fraction(val)
                if "-" in cols:
                    a, b = (int(x) for x in cols.split("-"))
                else:
                    a = b = int(cols)
                for c in range(a, b + 1):
                    M[r][c - 1] = v
    return M


def read_figure(name):
    """Points (8,3) and the 'expect' lines of a figure fixture."""
    pts, expect = [], {}
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            m = re.match(r"#\s*expect:\s*(\S+)\s*(.*)", line)
            if m:
                expect[m.group(1)] = m.group(2).split()
                continue
            line = line.split("#", 1)[0].strip()
            if line:
                pts.append([float(x) for x in line.split()])
    return np.array(pts), expect


def bernstein(k, t):
    return [(1 - t) ** 2, 2 * t * (1 - t), t * t][k]


def collocation_matrix():
    """A_{alpha beta} = B_beta(xi_alpha), Section 3.2, exact."""
    pts = [tuple(Fraction(c, 2) for c in n) for n in NODES]
    return [[bernstein(nb[0], p[0]) * bernstein(nb[1], p[1]) * bernstein(nb[2], p[2])
             for nb in NODES] for p in pts]


def shape_gradients(xi, eta, zeta):
    """d L_k / d(xi, eta, zeta) for the 8 shape functions of Appendix A."""
    one = 1
    L = [((one - xi), (one - eta), (one - zeta)), (xi, (one - eta), (one - zeta)),
         (xi, eta, (one - zeta)), ((one - xi), eta, (one - zeta)),
         ((one - xi), (one - eta), zeta), (xi, (one - eta), zeta),
         (xi, eta, zeta), ((one - xi), eta, zeta)]
    sign = [(-1, -1, -1), (1, -1, -1), (1, 1, -1), (-1, 1, -1),
            (-1, -1, 1), (1, -1, 1), (1, 1, 1), (-1, 1, 1)]
    out = []
    for (fx, fy, fz), (sx, sy, sz) in zip(L, sign):
        out.append((sx * fy * fz, sy * fx * fz, sz * fx * fy))
    return out


def jacobian_shape(P, xi, eta, zeta):
    """J = det(dx/dxi) from the shape-function gradients (works on Fractions)."""
    G = shape_gradients(xi, eta, zeta)
    Jm = [[sum(G[k][j] * P[k][i] for k in range(8)) for j in range(3)] for i in range(3)]
    return (Jm[0][0] * (Jm[1][1] * Jm[2][2] - Jm[1][2] * Jm[2][1])
            - Jm[0][1] * (Jm[1][0] * Jm[2][2] - Jm[1][2] * Jm[2][0])
            + Jm[0][2] * (Jm[1][0] * Jm[2][1] - Jm[1][1] * Jm[2][0]))


def jacobian_grid(P, m):
    """J (float64) on the (m+1)^3 uniform grid of [0,1]^3, vectorised."""
    t = np.linspace(0.0, 1.0, m + 1)
    xi, eta, zeta = np.meshgrid(t, t, t, indexing="ij")
    xi, eta, zeta = xi.ravel(), eta.ravel(), zeta.ravel()
    G = shape_gradients(xi, eta, zeta)
    P = np.asarray(P, dtype=np.float64)
    D = np.zeros((xi.size, 3, 3))
    for k in range(8):
        for j in range(3):
            D[:, :, j] += np.outer(G[k][j], P[k])
    return np.linalg.det(D)


def cube_symmetries():
    """The 48 symmetries of [0,1]^3 as (axis permutation, flips, det sign)."""
    out = []
    for perm in permutations(range(3)):
        psign = np.linalg.det(np.eye(3)[list(perm)])
        for flips in product((0, 1), repeat=3):
            out.append((perm, flips, int(round(psign)) * (-1) ** sum(flips)))
    return out


def apply_symmetry(points, sym):
    """Relabel the 8 nodes so that the new map is x(sigma(xi)).  Returns the new
    points and the Fig. 3 index map alpha -> sigma(alpha) (0-based)."""
    perm, flips, _ = sym

    def sigma(pos, top):  # pos in {0..top}^3
        q = [pos[perm[d]] for d in range(3)]
        return tuple(top - q[d] if flips[d] else q[d] for d in range(3))

    corners = [tuple(c // 2 for c in NODES[k]) for k in range(8)]
    new = [points[corners.index(sigma(corners[k], 1))] for k in range(8)]
    amap = [NODES.index(sigma(NODES[a], 2)) for a in range(27)]
    return np.array(new), amap
