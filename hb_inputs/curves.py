"""Curve inclusions for the HB integrator (Sec. 3.2, domain with a sound-hard inclusion):
a closed curve C discretised into N_s straight segments, given by their
centres r^s_i, lengths w_i and the slowness n(r^s_i) of the medium there.
Geometry only; none of the integrator's arithmetic."""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np


@dataclass
class Curve:
    centres: np.ndarray    # (N_s, 2) segment centres
    w: np.ndarray          # (N_s,) segment lengths
    slowness: np.ndarray   # (N_s,) n at the segment centres
    name: str = ""

    @property
    def Ns(self) -> int:
        return int(self.w.shape[0])


def circle(prob, centre, radius, ns, name=None) -> Curve:
    """The polygon of ns equal chords inscribed in the circle |r - centre| =
    radius (vertices at angles 2 pi k / ns): segment centres are the chord
    midpoints, lengths 2 radius sin(pi / ns)."""
    if prob.dim != 2:
        raise ValueError("curve inclusions are 2D")
    c = np.asarray(centre, np.float64)
    mid = (np.arange(ns, dtype=np.float64) + 0.5) * (2.0 * math.pi / ns)
    rm = radius * math.cos(math.pi / ns)
    P = c + rm * np.stack([np.cos(mid), np.sin(mid)], axis=1)
    w = np.full(ns, 2.0 * radius * math.sin(math.pi / ns))
    n = np.ascontiguousarray(prob.meta["medium"].slowness(P), dtype=np.float64)
    return Curve(centres=np.ascontiguousarray(P), w=w, slowness=n,
                 name=name or f"circle-c{tuple(c)}-r{radius}-ns{ns}")


def _polyline(prob, pts, w_target, name):
    """Straight segments of length <= w_target along the open polyline pts
    (each side split evenly)."""
    P = np.asarray(pts, np.float64)
    cs, ws = [], []
    for a, b in zip(P[:-1], P[1:]):
        L = float(np.linalg.norm(b - a))
        k = max(1, int(math.ceil(L / w_target)))
        t = (np.arange(k) + 0.5) / k
        cs.append(a[None, :] + t[:, None] * (b - a)[None, :])
        ws.append(np.full(k, L / k))
    C = np.ascontiguousarray(np.concatenate(cs))
    n = np.ascontiguousarray(prob.meta["medium"].slowness(C), dtype=np.float64)
    return Curve(centres=C, w=np.concatenate(ws), slowness=n, name=name)


def segment_length(prob, ppw):
    """w = 2 pi / (omega n_max ppw): ppw segments per shortest local
    wavelength (Sec. 5, inclusion examples)."""
    return 2.0 * math.pi / (prob.omega * float(np.max(prob.slowness)) * ppw)


def open_square(prob, centre, side, ppw, name=None) -> Curve:
    """The outline of the square of this side centred at `centre` without
    its top side (an open curve; Sec. 5, 2D examples with inclusion), cut
    into segments of ppw per shortest wavelength."""
    if prob.dim != 2:
        raise ValueError("curve inclusions are 2D")
    cx, cy = centre
    a = side / 2.0
    pts = [(cx - a, cy + a), (cx - a, cy - a), (cx + a, cy - a), (cx + a, cy + a)]
    return _polyline(prob, pts, segment_length(prob, ppw),
                     name or f"open-square-c{tuple(centre)}-s{side}-ppw{ppw}")
