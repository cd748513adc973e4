"""Exact helix in a sector's local frame, written from circle geometry (uses
asin, unlike the tracker's series form), for the closed-form pins.

State at plane x0: (y, z, snp, tgl, qpt); signed curvature C = kB * qpt with
kB = -c * B (a positive charge turns clockwise seen from +z for B along +z);
sin(phi) grows linearly in x with slope C; z grows with the transverse arc
length with slope tgl.
"""
import numpy as np

C_LIGHT = 0.299792458e-2


def kB(bz=0.5):
    return -C_LIGHT * bz


def at(state, x0, x, bz=0.5):
    """Exact (y, z, snp) at plane x (vectorised over x)."""
    y0, z0, snp0, tgl, qpt = [float(v) for v in state]
    x = np.asarray(x, np.float64)
    c = kB(bz) * qpt
    phi0 = np.arcsin(snp0)
    if c == 0.0:
        y = y0 + (x - x0) * np.tan(phi0)
        s = (x - x0) / np.cos(phi0)
        return y, z0 + tgl * s, np.full_like(x, snp0)
    snp = snp0 + c * (x - x0)
    phi = np.arcsin(snp)
    yc = y0 + np.cos(phi0) / c
    y = yc - np.cos(phi) / c
    s = (phi - phi0) / c
    return y, z0 + tgl * s, snp


def exact_arc(state, x0, x, bz=0.5):
    """Transverse arc length from x0 to x."""
    _, _, snp0, _, qpt = state
    c = kB(bz) * qpt
    phi0 = np.arcsin(snp0)
    if c == 0.0:
        return (x - x0) / np.cos(phi0)
    return (np.arcsin(snp0 + c * (x - x0)) - phi0) / c
