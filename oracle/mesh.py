"""Uniform mesh of square elements, skeleton (trace) numbering and boundary data.

Sec. 2.2.2: the hybrid unknown lives on the skeleton, one nodal value per
(face, ordinate, face node).  Boundary data enter through the projection P_M g
onto the trace space (the definition of the space V_h^g); with collocated LGL
face quadrature the discrete projection is nodal interpolation, so the
trace value on a domain-inflow DOF is g evaluated at the face node.

Numbering:
  element e = j n_x + i (x fastest), lower-left corner (x0 + i h, y0 + j h);
  vertical face  V(i, j) = j (n_x+1) + i,            i = 0..n_x, j < n_y;
  horizontal face H(i, j) = (n_x+1) n_y + j n_x + i,  j = 0..n_y, i < n_x;
  element (i, j) has W = V(i,j), E = V(i+1,j), S = H(i,j), N = H(i,j+1);
  trace DOF = (F N_a + k)(p+1) + jn, jn along increasing x or y.
"""
import numpy as np


class Mesh:
    def __init__(self, n_x, n_y, h, x0=0.0, y0=0.0):
        self.n_x, self.n_y, self.h, self.x0, self.y0 = int(n_x), int(n_y), float(h), float(x0), float(y0)
        self.E = self.n_x * self.n_y
        self.n_vfaces = (self.n_x + 1) * self.n_y
        self.n_faces = self.n_vfaces + self.n_x * (self.n_y + 1)

    def vface(self, i, j):
        return j * (self.n_x + 1) + i

    def hface(self, i, j):
        return self.n_vfaces + j * self.n_x + i

    def element_faces(self, e):
        i, j = e % self.n_x, e // self.n_x
        return [self.vface(i, j), self.vface(i + 1, j), self.hface(i, j), self.hface(i, j + 1)]

    def n_trace(self, disc):
        return self.n_faces * disc.n_a * disc.q

    def trace_dof(self, disc, F, k, jn):
        return (F * disc.n_a + k) * disc.q + jn

    def element_dofs(self, disc):
        """(in_dofs [E, m], out_dofs [E, m]): global trace DOF of each local index."""
        ind = np.empty((self.E, disc.m), dtype=np.int64)
        outd = np.empty((self.E, disc.m), dtype=np.int64)
        for e in range(self.E):
            faces = self.element_faces(e)
            for iota, (f, k, j, nd, row) in enumerate(disc.in_tab):
                ind[e, iota] = self.trace_dof(disc, faces[f], k, j)
            for o, (f, k, j, nd, row) in enumerate(disc.out_tab):
                outd[e, o] = self.trace_dof(disc, faces[f], k, j)
        return ind, outd

    def face_geometry(self, disc, F):
        """(x[q], y[q], outward domain normal or None) of the nodes of face F."""
        t = 0.5 * (disc.xi + 1.0) * self.h
        if F < self.n_vfaces:
            j, i = divmod(F, self.n_x + 1)
            x = np.full(disc.q, self.x0 + i * self.h)
            y = self.y0 + j * self.h + t
            nrm = (-1.0, 0.0) if i == 0 else ((1.0, 0.0) if i == self.n_x else None)
        else:
            j, i = divmod(F - self.n_vfaces, self.n_x)
            x = self.x0 + i * self.h + t
            y = np.full(disc.q, self.y0 + j * self.h)
            nrm = (0.0, -1.0) if j == 0 else ((0.0, 1.0) if j == self.n_y else None)
        return x, y, nrm

    def inflow_mask(self, disc):
        """Boolean [n_trace]: DOFs on the domain boundary with s . n_domain < 0."""
        mask = np.zeros(self.n_trace(disc), dtype=bool)
        for F in range(self.n_faces):
            _, _, nrm = self.face_geometry(disc, F)
            if nrm is None:
                continue
            for k in range(disc.n_a):
                if disc.s[k, 0] * nrm[0] + disc.s[k, 1] * nrm[1] < 0:
                    base = self.trace_dof(disc, F, k, 0)
                    mask[base:base + disc.q] = True
        return mask

    def boundary_vector(self, disc, g):
        """b[n_trace] = g(x, y, theta_k) on domain-inflow DOFs, 0 elsewhere.

        g is a callable g(x_array, y_array, theta) -> array.
        """
        b = np.zeros(self.n_trace(disc))
        for F in range(self.n_faces):
            x, y, nrm = self.face_geometry(disc, F)
            if nrm is None:
                continue
            for k in range(disc.n_a):
                if disc.s[k, 0] * nrm[0] + disc.s[k, 1] * nrm[1] < 0:
                    base = self.trace_dof(disc, F, k, 0)
                    b[base:base + disc.q] = g(x, y, disc.theta[k])
        return b

    def node_coords(self, disc):
        """Physical coordinates X, Y [E, nn] of the element LGL nodes (nd = b q + a)."""
        t = 0.5 * (disc.xi + 1.0) * self.h
        X = np.empty((self.E, disc.nn))
        Y = np.empty((self.E, disc.nn))
        for e in range(self.E):
            i, j = e % self.n_x, e // self.n_x
            for b in range(disc.q):
                for a in range(disc.q):
                    X[e, b * disc.q + a] = self.x0 + i * self.h + t[a]
                    Y[e, b * disc.q + a] = self.y0 + j * self.h + t[b]
        return X, Y

    def boundary_vector_sides(self, disc, g_side):
        """b from per-side data g_side[4, n_a] (sides W, E, S, N), constant
        along each side: b = g_side[side, k] on the domain-inflow DOFs of that
        side, 0 elsewhere."""
        g_side = np.asarray(g_side, dtype=np.float64)
        b = np.zeros(self.n_trace(disc))
        for F in range(self.n_faces):
            _, _, nrm = self.face_geometry(disc, F)
            if nrm is None:
                continue
            side = {(-1.0, 0.0): 0, (1.0, 0.0): 1, (0.0, -1.0): 2, (0.0, 1.0): 3}[nrm]
            for k in range(disc.n_a):
                if disc.s[k, 0] * nrm[0] + disc.s[k, 1] * nrm[1] < 0:
                    base = self.trace_dof(disc, F, k, 0)
                    b[base:base + disc.q] = g_side[side, k]
        return b
