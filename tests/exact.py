"""Exact rational geometry used to pin the oracle (independent of both the
oracle and the HIP library): the volume of the unit cube below a plane by
inclusion-exclusion over the cube's vertices, evaluated in rational arithmetic."""
from fractions import Fraction as Fr
from itertools import product
from math import factorial


def volume(m, alpha):
    """|{x in [0,1]^3 : m.x <= alpha}| for rational m (any signs, not all zero)."""
    m = [Fr(v) for v in m]
    a = Fr(alpha)
    # reflect negative components: m_i x_i = m_i + |m_i| (1 - x_i)
    for i in range(3):
        if m[i] < 0:
            a -= m[i]
            m[i] = -m[i]
    nz = [v for v in m if v != 0]
    k = len(nz)
    if k == 0:
        return Fr(1) if a >= 0 else Fr(0)
    den = Fr(factorial(k))
    for v in nz:
        den *= v
    tot = Fr(0)
    for bits in product((0, 1), repeat=k):
        s = a - sum(b * v for b, v in zip(bits, nz))
        if s > 0:
            tot += (-1) ** sum(bits) * s ** k
    return tot / den


def dvolume(m, alpha):
    """dV/dalpha of volume(m, alpha), exactly (rational). The interface area inside
    the cube is this value times |m|_2, since moving the plane by d(alpha) moves it a
    distance d(alpha)/|m|_2."""
    m = [Fr(v) for v in m]
    a = Fr(alpha)
    for i in range(3):
        if m[i] < 0:
            a -= m[i]
            m[i] = -m[i]
    nz = [v for v in m if v != 0]
    k = len(nz)
    den = Fr(factorial(k))
    for v in nz:
        den *= v
    tot = Fr(0)
    for bits in product((0, 1), repeat=k):
        s = a - sum(b * v for b, v in zip(bits, nz))
        if s > 0:
            tot += (-1) ** sum(bits) * k * s ** (k - 1)
    return tot / den


def plane_block(n, x0, nd=3):
    """Exact volume fractions of the half-space n.(x - x0) <= 0 on the 3x3x3 block of
    unit cells with offsets -1..1 around the central cell [0,1]^3 (float array [dz][dy][dx]).
    For nd == 2 all three z planes equal the central one."""
    import numpy as np
    out = np.zeros((3, 3, 3))
    for dz in (-1, 0, 1):
        for dy in (-1, 0, 1):
            for dx in (-1, 0, 1):
                o = (dx, dy, 0 if nd == 2 else dz)
                a = sum(Fr(n[i]) * (Fr(x0[i]) - o[i]) for i in range(3))
                out[dz + 1, dy + 1, dx + 1] = float(volume(n, a))
    return out
