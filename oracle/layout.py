"""Point layout of the nonoverlapping decomposition (oracle).

Section 3 of the paper introduces, per subdomain s, interior points x_i^s,
boundary points x_b^s and interface points x_Gamma^s, and one auxiliary
unknown u_Gamma per interface point shared by the neighbouring subdomains.
The paper does not fix where the points sit; this layout takes the reading:

* the rectangle is split into nsub_x x nsub_y equal boxes, s = sy*nsub_x + sx;
* interior points: cell-centred q_x x q_y grid in each box (row-major, y outer);
* every box edge carries points at the midpoints t_k = (k + 1/2)/m of m equal
  pieces, so no point sits on a box corner; an edge on the outer boundary
  carries m_bdry_edge Dirichlet points, an edge between two boxes carries
  m_ifc_edge interface points;
* each interface point is shared by exactly two subdomains and gets exactly
  one unknown and one flux-continuity row;
* interface numbering: all vertical interface edges (row-major: edge row y
  outer, x inner), then all horizontal interface edges, points along an edge
  in increasing coordinate;
* per subdomain the edges are visited bottom, right, top, left; boundary
  rows and interface rows of K^s follow that order.
"""
from __future__ import annotations

import dataclasses

import numpy as np

# Outward unit normals of the bottom, right, top and left edge of a box.
EDGE_NORMALS = ((0.0, -1.0), (1.0, 0.0), (0.0, 1.0), (-1.0, 0.0))


@dataclasses.dataclass
class Subdomain:
    sx: int
    sy: int
    xa: float          # lower-left corner
    ya: float
    hx: float          # box size
    hy: float
    interior: np.ndarray    # (q_x*q_y, 2)
    boundary: np.ndarray    # (mb_s, 2)
    interface: np.ndarray   # (k_s, 2)
    normals: np.ndarray     # (k_s, 2) outward normal of this box at each interface point
    gidx: np.ndarray        # (k_s,) global interface index of each local interface point

    @property
    def center(self):
        return (self.xa + 0.5 * self.hx, self.ya + 0.5 * self.hy)


@dataclasses.dataclass
class Layout:
    subs: list
    n_interface: int
    interface_points: np.ndarray   # (nG, 2) in global numbering

    def boundary_points(self):
        """All boundary points, subdomain-major, in local row order."""
        return np.concatenate([s.boundary for s in self.subs]) if self.subs else np.zeros((0, 2))

    def interior_points(self):
        return np.concatenate([s.interior for s in self.subs])


def _edge_points(p0, p1, m):
    t = (np.arange(m) + 0.5) / m
    return np.stack([p0[0] + t * (p1[0] - p0[0]), p0[1] + t * (p1[1] - p0[1])], axis=1)


def build_layout(problem) -> Layout:
    nx, ny = problem.nsub_x, problem.nsub_y
    hx = (problem.x1 - problem.x0) / nx
    hy = (problem.y1 - problem.y0) / ny
    mg, mb = problem.m_ifc_edge, problem.m_bdry_edge

    def xline(i):
        return problem.x0 + i * hx

    def yline(j):
        return problem.y0 + j * hy

    # Global interface edges and their points.
    n_v = (nx - 1) * ny
    vbase, hbase = {}, {}
    pts = []
    for j in range(ny):
        for i in range(1, nx):
            vbase[(i, j)] = len(pts) * mg
            pts.append(_edge_points((xline(i), yline(j)), (xline(i), yline(j + 1)), mg))
    for j in range(1, ny):
        for i in range(nx):
            hbase[(i, j)] = len(pts) * mg
            pts.append(_edge_points((xline(i), yline(j)), (xline(i + 1), yline(j)), mg))
    n_edges = len(pts)
    assert n_edges == n_v + nx * (ny - 1)
    ipts = np.concatenate(pts) if pts else np.zeros((0, 2))

    subs = []
    for sy in range(ny):
        for sx in range(nx):
            xa, ya = xline(sx), yline(sy)
            xb_, yb_ = xline(sx + 1), yline(sy + 1)
            tx = (np.arange(problem.q_x) + 0.5) / problem.q_x
            ty = (np.arange(problem.q_y) + 0.5) / problem.q_y
            X, Y = np.meshgrid(xa + tx * hx, ya + ty * hy)
            interior = np.stack([X.ravel(), Y.ravel()], axis=1)
            # (corner0, corner1, exterior?, global base if interface)
            edges = [
                ((xa, ya), (xb_, ya), sy == 0, None if sy == 0 else hbase[(sx, sy)]),
                ((xb_, ya), (xb_, yb_), sx == nx - 1, None if sx == nx - 1 else vbase[(sx + 1, sy)]),
                ((xa, yb_), (xb_, yb_), sy == ny - 1, None if sy == ny - 1 else hbase[(sx, sy + 1)]),
                ((xa, ya), (xa, yb_), sx == 0, None if sx == 0 else vbase[(sx, sy)]),
            ]
            bnd, ifc, nrm, gid = [], [], [], []
            for e, (p0, p1, exterior, base) in enumerate(edges):
                if exterior:
                    bnd.append(_edge_points(p0, p1, mb))
                else:
                    idx = base + np.arange(mg)
                    ifc.append(ipts[idx])
                    gid.append(idx)
                    nrm.append(np.tile(np.array(EDGE_NORMALS[e]), (mg, 1)))
            subs.append(Subdomain(
                sx=sx, sy=sy, xa=xa, ya=ya, hx=hx, hy=hy, interior=interior,
                boundary=np.concatenate(bnd) if bnd else np.zeros((0, 2)),
                interface=np.concatenate(ifc) if ifc else np.zeros((0, 2)),
                normals=np.concatenate(nrm) if nrm else np.zeros((0, 2)),
                gidx=np.concatenate(gid).astype(np.int64) if gid else np.zeros(0, np.int64)))
    return Layout(subs=subs, n_interface=n_edges * mg, interface_points=ipts)


def owner_subdomain(problem, x, y):
    """Subdomain holding each point: half-open boxes, the last box closed."""
    sx = np.floor((np.asarray(x) - problem.x0) * problem.nsub_x / (problem.x1 - problem.x0)).astype(np.int64)
    sy = np.floor((np.asarray(y) - problem.y0) * problem.nsub_y / (problem.y1 - problem.y0)).astype(np.int64)
    sx = np.clip(sx, 0, problem.nsub_x - 1)
    sy = np.clip(sy, 0, problem.nsub_y - 1)
    return sy * problem.nsub_x + sx
