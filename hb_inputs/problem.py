"""The HB integrator problem statement (Sec. 3.1): a regular cell grid on a
box, the angular frequency, the number of HB terms, the tabulated
ingredients and the slowness at the cell centres."""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Optional

import numpy as np

from .tables import tabulate


@dataclass
class HBProblem:
    dim: int
    ncell: tuple            # cells per axis
    origin: tuple           # lower corner of the cell grid
    h: float                # cell size
    omega: float            # angular frequency
    nterms: int             # 1 (N=0) or 2 (N=1)
    nI: int                 # Chebyshev nodes per axis per table box
    nbox: tuple             # table boxes per axis
    box_origin: tuple
    box_size: float
    tau2: np.ndarray        # (NT, NT)
    v0: np.ndarray
    v1: Optional[np.ndarray]
    slowness: np.ndarray    # (N_v,) at cell centres, natural order
    name: str = ""
    meta: dict = field(default_factory=dict)

    @property
    def Nv(self) -> int:
        return int(np.prod(self.ncell[: self.dim]))

    @property
    def NT(self) -> int:
        return int(self.tau2.shape[0])

    def centres(self, idx=None) -> np.ndarray:
        """Cell centres, natural index i = x + nx*(y + ny*z)."""
        if idx is None:
            idx = np.arange(self.Nv)
        idx = np.asarray(idx, dtype=np.int64)
        out = np.empty(idx.shape + (self.dim,))
        rem = idx.copy()
        for ax in range(self.dim):
            k = rem % self.ncell[ax]
            rem //= self.ncell[ax]
            out[..., ax] = self.origin[ax] + (k + 0.5) * self.h
        return out


def make_problem(medium, dim, ncell, omega, nI, nbox=None, nterms=2,
                 origin=None, extent=1.0, name="") -> HBProblem:
    """Cells of size extent/ncell[0] on [origin, origin + extent]^d with the
    table region equal to the cell region split into ``nbox`` boxes."""
    ncell = tuple(int(c) for c in ncell)
    if len(ncell) != dim:
        raise ValueError("ncell must have dim entries")
    if origin is None:
        origin = (0.0,) * dim
    if nbox is None:
        nbox = (1,) * dim
    h = extent / ncell[0]
    ext = [c * h for c in ncell]
    box_size = max(ext[ax] / nbox[ax] for ax in range(dim))
    tau2, v0, v1 = tabulate(medium, dim, nI, nbox, origin, box_size)
    prob = HBProblem(dim=dim, ncell=ncell, origin=tuple(origin), h=h,
                     omega=float(omega), nterms=nterms, nI=nI,
                     nbox=tuple(nbox), box_origin=tuple(origin),
                     box_size=box_size, tau2=tau2, v0=v0,
                     v1=v1 if nterms == 2 else None,
                     slowness=np.zeros(0), name=name)
    prob.slowness = np.ascontiguousarray(medium.slowness(prob.centres()))
    prob.meta["medium"] = medium
    return prob
