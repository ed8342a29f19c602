"""Hemisphere direction rules for the angular quadrature of the fast spectral
method (Sec. 4.4.1, 3D case).  TEST INFRASTRUCTURE ONLY (see package doc).

The angular integral over e in S^2_+ of the kernel's Fourier factors is even in
e, so any rule on the half sphere whose weights sum to 2*pi (the hemisphere
area) integrates it.  Three rules are provided; each returns (dirs[M,3],
weights[M]) in float64.
"""
import math

import numpy as np


def icosa6():
    """The six axes of the regular icosahedron, weight pi/3 each (an exact
    antipodal 5-design).  Representatives (0,1,g),(0,-1,g),(1,g,0),(-1,g,0),
    (g,0,1),(-g,0,1), g the golden ratio, normalised."""
    g = (1.0 + math.sqrt(5.0)) / 2.0
    raw = np.array([[0.0, 1.0, g], [0.0, -1.0, g], [1.0, g, 0.0],
                    [-1.0, g, 0.0], [g, 0.0, 1.0], [-g, 0.0, 1.0]])
    dirs = raw / math.sqrt(1.0 + g * g)
    return dirs, np.full(6, math.pi / 3.0)


def product(a1: int, a2: int):
    """The (theta_p, phi_q) product grid of the 3D fast method with a1*a2
    points: theta_p = (p + 1/2) pi / a1, phi_q = q pi / a2 (p < a1, q < a2),
    weights proportional to sin(theta_p) and renormalised to sum to 2 pi
    (the area element the printed rule omits)."""
    th = (np.arange(a1) + 0.5) * math.pi / a1
    ph = np.arange(a2) * math.pi / a2
    T, P = np.meshgrid(th, ph, indexing="ij")
    T = T.ravel()
    P = P.ravel()
    dirs = np.stack([np.sin(T) * np.cos(P), np.sin(T) * np.sin(P), np.cos(T)], axis=1)
    w = np.sin(T)
    w = w * (2.0 * math.pi / w.sum())
    return dirs, w


def spiral(m: int):
    """Equal-weight golden-spiral rule on the upper hemisphere: z_p = (p+1/2)/m
    (equal-area bands), azimuth 2 pi p / golden ratio, weight 2 pi / m."""
    p = np.arange(m, dtype=np.float64)
    z = (p + 0.5) / m
    g = (1.0 + math.sqrt(5.0)) / 2.0
    az = 2.0 * math.pi * p / g
    s = np.sqrt(1.0 - z * z)
    dirs = np.stack([s * np.cos(az), s * np.sin(az), z], axis=1)
    return dirs, np.full(m, 2.0 * math.pi / m)
