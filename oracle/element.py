"""Element matrices of the lowest-order hexahedral Nedelec space (Sec. 2).

On a cube T of side h with local coordinates (xi, eta, zeta) in [0,1]^3, the space
ND(T) of eq. (nedlec form) has the 12 basis functions dual to the edge averages of
eq. (NDdof).  For the x-edge at (eta, zeta) = (a, b) in {0,1}^2 the basis function is
(psi_a(eta) psi_b(zeta), 0, 0) with psi_0(t) = 1 - t, psi_1(t) = t (its tangential
average is 1 on that edge and 0 on the 11 others); y- and z-edges are the cyclic
analogues.

Local edge order: index 4 d + (a + 2 b) for direction d, where (a, b) are the
offsets along the two other axes in increasing axis order
(x-edges: (eta, zeta); y-edges: (xi, zeta); z-edges: (xi, eta)).

The curl of an ND(T) field has constant normal component on each of the 6 faces;
its value times the face area is the circulation of the field around the face
(Stokes), i.e. h times a signed sum of four edge values.  The face fields form the
lowest-order Raviart-Thomas space of T, whose 1-D mass along the face normal is
m = [[1/3, 1/6], [1/6, 1/3]].
"""
import numpy as np

M2 = np.array([[1.0 / 3.0, 1.0 / 6.0], [1.0 / 6.0, 1.0 / 3.0]])


def local_edge(d, a, b):
    return 4 * d + a + 2 * b


def face_circulation():
    """6 x 12 integer matrix: circulation (divided by h) of each face.

    Faces in order x-face xi=0, xi=1, y-face eta=0, 1, z-face zeta=0, 1.
    The x-face at xi0 is traversed with the right-hand rule around +x:
    +z(xi0, eta=1) - z(xi0, eta=0) - y(xi0, zeta=1) + y(xi0, zeta=0); the y- and
    z-faces follow cyclically.
    """
    D = np.zeros((6, 12))
    for f in range(2):
        # x-face xi = f: y-edges indexed (xi, zeta), z-edges (xi, eta)
        D[f, local_edge(2, f, 1)] += 1
        D[f, local_edge(2, f, 0)] -= 1
        D[f, local_edge(1, f, 1)] -= 1
        D[f, local_edge(1, f, 0)] += 1
        # y-face eta = f: x-edges (eta, zeta), z-edges (xi, eta)
        D[2 + f, local_edge(0, f, 1)] += 1
        D[2 + f, local_edge(0, f, 0)] -= 1
        D[2 + f, local_edge(2, 1, f)] -= 1
        D[2 + f, local_edge(2, 0, f)] += 1
        # z-face zeta = f: y-edges (xi, zeta), x-edges (eta, zeta)
        D[4 + f, local_edge(1, 1, f)] += 1
        D[4 + f, local_edge(1, 0, f)] -= 1
        D[4 + f, local_edge(0, 1, f)] -= 1
        D[4 + f, local_edge(0, 0, f)] += 1
    return D


def mass_matrix(h):
    """M_T[e, e'] = int_T phi_e . phi_e' = h^3 blockdiag(M4, M4, M4), M4 = m (x) m."""
    M4 = np.kron(M2, M2)
    M = np.zeros((12, 12))
    for d in range(3):
        M[4 * d:4 * d + 4, 4 * d:4 * d + 4] = M4
    return h ** 3 * M


def curl_matrix(h):
    """K_T[e, e'] = int_T curl phi_e . curl phi_e' = h D^T blockdiag(m, m, m) D."""
    D = face_circulation()
    Mf = np.zeros((6, 6))
    for f in range(3):
        Mf[2 * f:2 * f + 2, 2 * f:2 * f + 2] = M2
    return h * D.T @ Mf @ D


def element_matrix(h, alpha):
    """Element matrix of a_T(w, v) = alpha (curl w, curl v)_T + (w, v)_T (eq. def bilinear form)."""
    return alpha * curl_matrix(h) + mass_matrix(h)
