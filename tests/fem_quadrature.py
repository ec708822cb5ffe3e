"""Brute-force P1 weak forms by Gauss-Legendre quadrature (numpy).

Used only to pin the oracle: the oracle evaluates the mass, stiffness and
advection forms of eq. sde1 / fde1 with closed-form three-point stencils; here
the same integrals are computed cell by cell by quadrature over the P1 basis
functions, written independently of those stencils.
"""
import numpy as np

_GX, _GW = np.polynomial.legendre.leggauss(4)  # exact for degree <= 7
_S = 0.5 * (_GX + 1.0)
_W = 0.5 * _GW


def _cells(nx):
    e = np.arange(nx)
    return e, (e + 1) % nx


def mass(L, f):
    nx = len(f)
    h = L / nx
    out = np.zeros(nx)
    left, right = _cells(nx)
    for s, w in zip(_S, _W):
        fq = f[left] * (1 - s) + f[right] * s
        np.add.at(out, left, w * h * fq * (1 - s))
        np.add.at(out, right, w * h * fq * s)
    return out


def stiff(L, f):
    nx = len(f)
    h = L / nx
    out = np.zeros(nx)
    left, right = _cells(nx)
    for s, w in zip(_S, _W):
        fx = (f[right] - f[left]) / h
        np.add.at(out, left, w * h * fx * (-1.0 / h))
        np.add.at(out, right, w * h * fx * (1.0 / h))
    return out


def advect(L, v, f):
    """(f d_x v, phi_i) - (f v, d_x phi_i) for P1 f, v, by quadrature."""
    nx = len(f)
    h = L / nx
    out = np.zeros(nx)
    left, right = _cells(nx)
    for s, w in zip(_S, _W):
        fq = f[left] * (1 - s) + f[right] * s
        vq = v[left] * (1 - s) + v[right] * s
        vx = (v[right] - v[left]) / h
        np.add.at(out, left, w * h * (fq * vx * (1 - s) - fq * vq * (-1.0 / h)))
        np.add.at(out, right, w * h * (fq * vx * s - fq * vq * (1.0 / h)))
    return out


def dense(op, nx):
    """Dense matrix of a linear operator on R^nx."""
    A = np.zeros((nx, nx))
    for j in range(nx):
        e = np.zeros(nx)
        e[j] = 1.0
        A[:, j] = op(e)
    return A
