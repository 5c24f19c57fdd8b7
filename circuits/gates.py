"""Gate matrices (complex128) under the conventions of this package.

Single-qubit gates act on column vectors (|0>, |1>).  Two-qubit matrices are
indexed row = 2*o1 + o2 (first listed qubit is the high bit of the 2-bit row
index), columns likewise for the inputs.
"""
import numpy as np

_S2 = 1.0 / np.sqrt(2.0)

H = _S2 * np.array([[1, 1], [1, -1]], dtype=np.complex128)
# RX(pi/2)
SQRT_X = _S2 * np.array([[1, -1j], [-1j, 1]], dtype=np.complex128)
# RY(pi/2)
SQRT_Y = _S2 * np.array([[1, -1], [1, 1]], dtype=np.complex128)
# exp(-i pi W / 4), W = (X + Y)/sqrt(2)
SQRT_W = _S2 * np.array([[1, -np.exp(1j * np.pi / 4)],
                         [np.exp(-1j * np.pi / 4), 1]], dtype=np.complex128)

CZ = np.diag([1, 1, 1, -1]).astype(np.complex128)


def z_phase(theta):
    """diag(1, e^{i theta})."""
    return np.diag([1.0, np.exp(1j * theta)]).astype(np.complex128)


def cphase(phi):
    """diag(1, 1, 1, e^{i phi})."""
    return np.diag([1.0, 1.0, 1.0, np.exp(1j * phi)]).astype(np.complex128)


def fsim(theta, phi):
    c, s = np.cos(theta), np.sin(theta)
    return np.array([[1, 0, 0, 0],
                     [0, c, -1j * s, 0],
                     [0, -1j * s, c, 0],
                     [0, 0, 0, np.exp(-1j * phi)]], dtype=np.complex128)


def haar_su2(rng):
    """Haar-random SU(2): a normalised complex 2-vector (a, b) from four
    standard normals gives [[a, -conj(b)], [b, conj(a)]]."""
    v = rng.standard_normal(4)
    v /= np.linalg.norm(v)
    a = v[0] + 1j * v[1]
    b = v[2] + 1j * v[3]
    return np.array([[a, -np.conj(b)], [b, np.conj(a)]], dtype=np.complex128)


def haar_su4(rng):
    """Haar-random SU(4): QR of a complex Ginibre matrix with the diagonal
    phases of R moved into Q (Mezzadri 2007), then scaled to unit determinant."""
    z = (rng.standard_normal((4, 4)) + 1j * rng.standard_normal((4, 4))) / np.sqrt(2)
    q, r = np.linalg.qr(z)
    d = np.diag(r)
    q = q * (d / np.abs(d))[None, :]
    det = np.linalg.det(q)
    q = q / det ** 0.25
    return q.astype(np.complex128)
