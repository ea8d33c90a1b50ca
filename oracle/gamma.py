"""Euclidean Dirac matrices in the chiral basis (oracle).

The paper fixes no basis.  Reading taken: gamma_k = [[0, -i sigma_k],
[i sigma_k, 0]] (k = 1, 2, 3), gamma_4 = [[0, 1], [1, 0]], so that
gamma_5 = gamma_1 gamma_2 gamma_3 gamma_4 = diag(1, 1, -1, -1).  The spectrum of
H_W does not depend on this choice.  Index 0..3 of ``gammas()`` is x, y, z, t.
"""
import numpy as np

_s1 = np.array([[0, 1], [1, 0]], dtype=np.complex128)
_s2 = np.array([[0, -1j], [1j, 0]], dtype=np.complex128)
_s3 = np.array([[1, 0], [0, -1]], dtype=np.complex128)
_z2 = np.zeros((2, 2), dtype=np.complex128)
_i2 = np.eye(2, dtype=np.complex128)


def gammas():
    """[4][4][4] complex128: gamma_1 .. gamma_4 in the chiral basis."""
    out = []
    for s in (_s1, _s2, _s3):
        out.append(np.block([[_z2, -1j * s], [1j * s, _z2]]))
    out.append(np.block([[_z2, _i2], [_i2, _z2]]))
    return np.array(out)


def gamma5():
    g = gammas()
    return g[0] @ g[1] @ g[2] @ g[3]
