"""P1 finite elements on a structured triangle mesh of the unit square.

Test infrastructure only (see ``oracle/__init__.py``).

Paper passages followed: Sec. 2 weak form and semi-discretisation
(Eq. acoustic_ode, M u'' + C u' + K u = f with a(u,v) = int c grad u . grad v);
Sec. 4 (Eq. randODEchapt2: M deterministic, K carries the random speed) and
Sec. 6 setup (unit square, u = 0 on all four sides).

Readings (the paper is silent): the mesh is n x n square cells, nodes
(i/n, j/n) numbered i + (n+1) j, each cell cut along its diagonal from (i,j)
to (i+1,j+1); consistent P1 mass; the coefficient is constant per element,
taken at the element centroid.
"""

import numpy as np
import scipy.sparse as sp


class StructuredMesh:
    """n x n cells on [0,1]^2, two triangles per cell."""

    def __init__(self, n):
        self.n = n
        self.nn = (n + 1) * (n + 1)
        i, j = np.meshgrid(np.arange(n + 1), np.arange(n + 1), indexing="xy")
        self.x = (i.ravel() / n).astype(np.float64)
        self.y = (j.ravel() / n).astype(np.float64)
        tris = []
        for cj in range(n):
            for ci in range(n):
                v00 = ci + (n + 1) * cj
                v10, v01 = v00 + 1, v00 + n + 1
                v11 = v01 + 1
                tris.append((v00, v10, v11))
                tris.append((v00, v11, v01))
        self.tris = np.array(tris, dtype=np.int64)
        self.cx = self.x[self.tris].mean(axis=1)
        self.cy = self.y[self.tris].mean(axis=1)
        bnd = (self.x == 0) | (self.x == 1) | (self.y == 0) | (self.y == 1)
        self.free = np.nonzero(~bnd)[0]


def element_matrices(px, py):
    """Local P1 stiffness (unit coefficient) and consistent mass of one triangle."""
    area = 0.5 * ((px[1] - px[0]) * (py[2] - py[0])
                  - (px[2] - px[0]) * (py[1] - py[0]))
    # gradients of the barycentric coordinates: rotated opposite edges / 2A
    bx = np.array([py[1] - py[2], py[2] - py[0], py[0] - py[1]]) / (2 * area)
    by = np.array([px[2] - px[1], px[0] - px[2], px[1] - px[0]]) / (2 * area)
    ke = area * (np.outer(bx, bx) + np.outer(by, by))
    me = area / 12.0 * (np.ones((3, 3)) + np.eye(3))
    return ke, me


def assemble(mesh, coef):
    """Global stiffness matrices K_k = sum_e coef[k, e] K_e and mass M.

    coef has shape (nk, ne).  Returns (list of K_k, M) as CSR over all nodes;
    duplicate (row, col) pairs of the element scatter are summed.
    """
    ne = len(mesh.tris)
    ke = np.zeros((ne, 3, 3))
    me = np.zeros((ne, 3, 3))
    for e, t in enumerate(mesh.tris):
        ke[e], me[e] = element_matrices(mesh.x[t], mesh.y[t])
    rows = np.repeat(mesh.tris, 3, axis=1).ravel()
    cols = np.tile(mesh.tris, (1, 3)).ravel()
    shape = (mesh.nn, mesh.nn)
    K = [sp.csr_matrix(((coef[k][:, None, None] * ke).ravel(), (rows, cols)),
                       shape=shape) for k in range(coef.shape[0])]
    M = sp.csr_matrix((me.ravel(), (rows, cols)), shape=shape)
    return K, M
