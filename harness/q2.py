"""Reference-element tables for Q2 velocity and P1-discontinuous pressure.

Section 2 and section 3 fix the element pair (Q2 / P1disc); the concrete
basis and quadrature are this project's choice: tensor-product Lagrange
polynomials on the nodes {-1, 0, 1} per axis, the pressure basis {1, xi, eta,
zeta} on the reference cube [-1, 1]^3, and the 3x3x3 Gauss rule, which
integrates every product that appears exactly on axis-aligned voxels.
Local node k of an element sits at lattice offset (k % 3, (k // 3) % 3, k // 9)
(xi fastest).
"""
import numpy as np

NODES_1D = np.array([-1.0, 0.0, 1.0])
GAUSS_1D = np.array([-np.sqrt(0.6), 0.0, np.sqrt(0.6)])
WEIGHTS_1D = np.array([5.0 / 9.0, 8.0 / 9.0, 5.0 / 9.0])


def lagrange_1d(t):
    """Values and derivatives of the three quadratic Lagrange polynomials at t."""
    t = np.asarray(t, dtype=np.float64)
    val = np.stack([0.5 * t * (t - 1.0), 1.0 - t * t, 0.5 * t * (t + 1.0)], axis=-1)
    der = np.stack([t - 0.5, -2.0 * t, t + 0.5], axis=-1)
    return val, der


def local_offsets():
    k = np.arange(27)
    return np.stack([k % 3, (k // 3) % 3, k // 9], axis=1)


def quadrature_points():
    """27 Gauss points (xi fastest) and their weights."""
    g = GAUSS_1D
    w = WEIGHTS_1D
    pts = np.array([(g[i], g[j], g[k]) for k in range(3) for j in range(3) for i in range(3)])
    wts = np.array([w[i] * w[j] * w[k] for k in range(3) for j in range(3) for i in range(3)])
    return pts, wts


def q2_tables(points):
    """phi[q, a] and dphi[q, a, dir] (reference derivatives) at the given points."""
    off = local_offsets()
    vx, dx = lagrange_1d(points[:, 0])
    vy, dy = lagrange_1d(points[:, 1])
    vz, dz = lagrange_1d(points[:, 2])
    ax, ay, az = off[:, 0], off[:, 1], off[:, 2]
    phi = vx[:, ax] * vy[:, ay] * vz[:, az]
    dphi = np.stack([dx[:, ax] * vy[:, ay] * vz[:, az],
                     vx[:, ax] * dy[:, ay] * vz[:, az],
                     vx[:, ax] * vy[:, ay] * dz[:, az]], axis=-1)
    return phi, dphi


def p1_tables(points):
    """psi[q, m] for the P1disc modes {1, xi, eta, zeta}."""
    ones = np.ones(points.shape[0])
    return np.stack([ones, points[:, 0], points[:, 1], points[:, 2]], axis=1)
