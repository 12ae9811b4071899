"""Structured hex8 grid, boundary conditions and load (Sec. 3.1, Tab. geometries).

The paper uses structured grids of geometrically cubic trilinear hexahedra and
removes constrained DOFs before any residual norm.  The workloads here use the
cantilever setting: the x = 0 face fully clamped and a unit downward (-z) load
spread over the bottom edge of the free end (x = L, z = 0).  A distributed load
is converted to consistent nodal forces by tributary length, so the interior
nodes of the edge carry -1/ny and the two end nodes -1/(2 ny); the total is -1.

Numbering (x fastest): element e = ex + nx (ey + ny ez); node
n = i + (nx+1)(j + (ny+1) k); DOF 3n + c.
"""
import numpy as np

from .ke import LOCAL


class Grid:
    def __init__(self, nx, ny, nz):
        self.nx, self.ny, self.nz = int(nx), int(ny), int(nz)
        self.NX, self.NY, self.NZ = self.nx + 1, self.ny + 1, self.nz + 1
        self.n_elem = self.nx * self.ny * self.nz
        self.n_nodes = self.NX * self.NY * self.NZ
        self.n_dof = 3 * self.n_nodes

    def node(self, i, j, k):
        return i + self.NX * (j + self.NY * k)

    def node_ijk(self, n):
        i = n % self.NX
        j = (n // self.NX) % self.NY
        k = n // (self.NX * self.NY)
        return i, j, k

    def elem_nodes(self):
        """(n_elem, 8) node ids of every element in local order a = i + 2j + 4k."""
        ex, ey, ez = np.meshgrid(np.arange(self.nx), np.arange(self.ny),
                                 np.arange(self.nz), indexing="ij")
        ex = ex.transpose(2, 1, 0).ravel()   # x fastest
        ey = ey.transpose(2, 1, 0).ravel()
        ez = ez.transpose(2, 1, 0).ravel()
        cols = [self.node(ex + i, ey + j, ez + k) for (i, j, k) in LOCAL]
        return np.stack(cols, axis=1)

    def elem_dofs(self):
        """(n_elem, 24) global DOFs of every element, local DOF 3a + c."""
        en = self.elem_nodes()
        return (3 * en[:, :, None] + np.arange(3)[None, None, :]).reshape(self.n_elem, 24)

    def node_coords(self):
        n = np.arange(self.n_nodes)
        i, j, k = self.node_ijk(n)
        return np.stack([i, j, k], axis=1).astype(float)

    def clamped_nodes(self):
        """Nodes on the x = 0 face (all three DOFs fixed)."""
        return self.node_ijk(np.arange(self.n_nodes))[0] == 0

    def free_dofs(self):
        """Boolean mask over the n_dof DOFs: True where the DOF is free."""
        return np.repeat(~self.clamped_nodes(), 3)

    def n_free(self):
        return int(self.free_dofs().sum())

    def edge_load(self):
        """Unit -z load on the edge x = L, z = 0, consistent nodal forces by
        tributary length (total force (0, 0, -1))."""
        f = np.zeros(self.n_dof)
        for j in range(self.NY):
            w = 1.0 / self.ny
            if j == 0 or j == self.ny:
                w *= 0.5
            f[3 * self.node(self.nx, j, 0) + 2] -= w
        return f
