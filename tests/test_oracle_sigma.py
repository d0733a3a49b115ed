"""The sigma-transformed formulation (Sec. 3.1: K = J J^T / det J with
d = eta + h, nabla^sigma = (d_x, d_y, d_sigma)) discretises the same weak form
as the physical one under the change of variables (x, y, z) -> (x, y, sigma).
With the sigma-layered map of the oracle (straight triangles, z = -h +
sigma (eta + h), eta interpolated at order P) both give the same element
matrices: assembled here directly from the paper's K tensor at the same
cubature, they equal the oracle's physical-form element matrices."""
import numpy as np
import pytest

from oracle import mesh as M
from oracle.operator import LevelGeometry, StiffnessOperator, element_node_xyz
from oracle.refelem import ref
from paper_2009_00705_amd import workloads as W


@pytest.mark.parametrize("P,L", [(3, 2), (4, 1)])
def test_sigma_form_element_matrices_equal_the_physical_ones(P, L):
    h = 1.0
    m = W.box_mesh(2, L, depth=h)
    num = M.Numbering(m, P)
    xy = M.unique_xy_2d(m, num)
    eta = 0.1 * np.sin(xy[:, 0]) * np.cos(xy[:, 1])
    Ae = StiffnessOperator(num, LevelGeometry(P, P, element_node_xyz(m, num, eta))).element_matrices()
    re = ref(P)
    B, Dr, Ds = re.tri_eval(re.cr, re.cs)          # triangle basis at the triangle points
    Bz, Dz = re.line_eval(re.zq)                    # vertical basis at the Gauss points
    X2 = M.node_xy_2d(m, num)                       # (nt, Np_tri, 2), affine triangles
    for e in range(num.n_elem):
        t, layer = divmod(e, L)
        X = X2[t]
        J2 = np.array([[Dr[0] @ X[:, 0], Ds[0] @ X[:, 0]], [Dr[0] @ X[:, 1], Ds[0] @ X[:, 1]]])
        Ji = np.linalg.inv(J2)                      # (r_x r_y; s_x s_y)
        et = eta[num.map2d[t]]
        ex = (Dr @ et) * Ji[0, 0] + (Ds @ et) * Ji[1, 0]
        ey = (Dr @ et) * Ji[0, 1] + (Ds @ et) * Ji[1, 1]
        d = B @ et + h
        A = np.zeros((re.np, re.np))
        for k in range(P + 1):
            sig = (layer + (1 + re.zq[k]) / 2) / L
            for q in range(re.nq_tri):
                # gradients of the prism basis in (x, y, sigma)
                gx = np.kron(Bz[k], Dr[q] * Ji[0, 0] + Ds[q] * Ji[1, 0])
                gy = np.kron(Bz[k], Dr[q] * Ji[0, 1] + Ds[q] * Ji[1, 1])
                gs = np.kron(Dz[k] * 2 * L, B[q])
                Kq = np.array([[d[q], 0.0, -sig * ex[q]],
                               [0.0, d[q], -sig * ey[q]],
                               [-sig * ex[q], -sig * ey[q], (1 + sig ** 2 * (ex[q] ** 2 + ey[q] ** 2)) / d[q]]])
                Gr = np.stack([gx, gy, gs])
                w = re.zw[k] * re.cw[q] * abs(np.linalg.det(J2)) / (2 * L)
                A += w * Gr.T @ Kq @ Gr
        np.testing.assert_allclose(A, Ae[e], atol=1e-12 * np.abs(Ae[e]).max())
