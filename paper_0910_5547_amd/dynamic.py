"""A dynamic hierarchy driven through the C ABI: the steps on either side of the per-patch
update that the paper keeps on the host (Sec. 3), with the flagging on the GPU.

Every `every` root steps the hierarchy is rebuilt from the root up: the refinement flags
of level l (amr_flag_cells, GPU) are clustered on the host into level l+1 boxes
(amr_cluster_flags), a table for levels 0..l+1 is created, and its arena is filled from
the hierarchy being replaced (amr_regrid_fill: cells the old hierarchy holds are copied,
the rest prolonged from the new level below).  Between rebuilds the hierarchy advances by
subcycled root steps (amr_cfl_dt + amr_hydro_advance).
"""
from __future__ import annotations

import torch

from . import amr as A
from . import workloads as W


class DynamicHierarchy:
    """A hierarchy over a fixed root level (brick-aligned patches), refined up to
    `max_level` levels where |d rho| / min rho > eps between face neighbours.

    Faces of new patches on the root domain's boundary take the boundary condition of
    that side of the domain (`domain_bc`, faces -x, +x, -y, +y, -z, +z); the others are
    EXTERNAL.  The root patches' own faces are kept as given."""

    def __init__(self, ps_root, U_root, max_level, eps, every=4, brick=8, block=32, domain_bc=None, cfl=0.8,
                 t0=0.0, **table_kw):
        assert int(ps_root.level.max()) == 0
        self.root = ps_root
        self.max_level, self.eps, self.every = max_level, eps, every
        self.brick, self.block, self.cfl = brick, block, cfl
        self.kw = dict(table_kw)
        self.domain = tuple(int(x) for x in (ps_root.lo + ps_root.n).max(axis=0))
        self.domain_bc = list(domain_bc) if domain_bc is not None else [W.BC_OUTFLOW] * 6
        self.ps = ps_root
        self.T = A.Table(ps_root, **self.kw)
        self.U = self.T.upload(U_root)
        self.steps = 0
        self.t = float(t0)  # the time of U_root
        self.rebuilds = 0

    def _patchset(self, boxes_by_level):
        """Root patches followed by the boxes of each finer level, in one new arena."""
        r = self.root
        n = [list(r.n[p]) for p in range(r.npatch)]
        lo = [list(r.lo[p]) for p in range(r.npatch)]
        bc = [list(r.bc[p]) for p in range(r.npatch)]
        lev = [0] * r.npatch
        for l, boxes in enumerate(boxes_by_level, start=1):
            N = [self.domain[d] << l for d in range(3)]
            for b in boxes:
                blo, bn = [int(x) for x in b[:3]], [int(x) for x in b[3:]]
                f = [W.BC_EXTERNAL] * 6
                for d in range(r.ndim):
                    if blo[d] == 0:
                        f[2 * d] = self.domain_bc[2 * d]
                    if blo[d] + bn[d] == N[d]:
                        f[2 * d + 1] = self.domain_bc[2 * d + 1]
                n.append(bn)
                lo.append(blo)
                bc.append(f)
                lev.append(l)
        return W.make_patchset(r.ndim, n, r.ng, bc, level=lev, lo=lo, gamma=r.gamma, theta=r.theta, dx0=r.dx0,
                               nvar=r.nvar)

    def rebuild(self):
        """Rebuild every level above the root from the current state."""
        old_T, old_U = self.T, self.U
        cur_T, cur_U, cur_ps = old_T, old_U, self.ps
        boxes = []
        for l in range(self.max_level):
            if l > int(cur_ps.level.max()):
                break
            ncell = A.amr_table_cells(cur_T.h, l)
            flags = torch.zeros(ncell, dtype=torch.uint8, device=cur_U.device)
            A.amr_flag_cells(cur_T.h, cur_U, l, self.eps, flags)
            torch.cuda.synchronize()
            b = A.amr_cluster_flags(cur_T.descs, cur_ps.ndim, self.domain, l, flags.cpu().numpy(), self.brick,
                                    self.block)
            if len(b) == 0:
                break
            boxes.append(b)
            ps = self._patchset(boxes)
            T = A.Table(ps, **self.kw)
            try:
                U = torch.zeros(int(A.amr_table_arena_elems(T.h)), dtype=torch.float64, device=cur_U.device)
                A.amr_regrid_fill(old_T.h, old_U, T.h, U)
            except BaseException:
                T.close()
                if cur_T is not old_T:
                    cur_T.close()
                raise
            if cur_T is not old_T:
                cur_T.close()
            cur_T, cur_U, cur_ps = T, U, ps
        if cur_T is old_T:  # nothing to refine: drop the finer levels
            if int(self.ps.level.max()) == 0:
                return
            ps = self._patchset([])
            T = A.Table(ps, **self.kw)
            try:
                U = torch.zeros(int(A.amr_table_arena_elems(T.h)), dtype=torch.float64, device=old_U.device)
                A.amr_regrid_fill(old_T.h, old_U, T.h, U)
            except BaseException:
                T.close()
                raise
            cur_T, cur_U, cur_ps = T, U, ps
        old_T.close()
        self.T, self.U, self.ps = cur_T, cur_U, cur_ps
        self.rebuilds += 1

    def advance(self, t_end, max_steps=100000):
        """Root steps until t_end (the last one clipped), rebuilding every `every` steps."""
        while self.t < t_end and max_steps > 0:
            if self.steps % self.every == 0:
                self.rebuild()
            dt = A.amr_cfl_dt(self.T.h, self.U, self.cfl, -1, self.T.dt, host=True)
            if self.t + dt > t_end:
                dt = t_end - self.t
                self.T.dt.fill_(dt)
            A.amr_hydro_advance(self.T.h, self.U, self.T.dt)
            self.t += dt
            self.steps += 1
            max_steps -= 1
        torch.cuda.synchronize()
        st = self.T.status()
        if st != A.AMR_OK:
            raise RuntimeError(A.amr_status_string(st))

    def host_state(self):
        return self.ps, self.U.cpu().numpy()

    def close(self):
        self.T.close()
