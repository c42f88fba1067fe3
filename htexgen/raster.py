"""Raster-order query batches: a software rasterizer (numpy, float64) that
renders a mesh's intrinsic triangles through a pinhole camera and emits one
query per covered pixel, in scanline order, as a fragment stage would see
them: the visible triangle's halfedge h, its perspective-correct
barycentric (u, v) and the screen-space derivatives of (u, v) (for an
isotropic footprint or anisotropic filtering).

The triangles are an input (three 3D points per halfedge, in the order
v0, v1, v2 with (u, v, w) = (1, 0, 0) at v2, (0, 1, 0) at v0 and
(0, 0, 1) at v1); this module only projects, tests coverage and resolves
visibility.  Derivatives are the differences of the triangle's (u, v)
plane equations one pixel to the right and one pixel down, as a GPU's
screen derivatives are.
"""
from __future__ import annotations

import dataclasses

import numpy as np


@dataclasses.dataclass
class Camera:
    eye: np.ndarray        # [3]
    target: np.ndarray     # [3]
    up: np.ndarray         # [3]
    fov_y: float           # vertical field of view, radians
    width: int
    height: int

    def basis(self):
        f = self.target - self.eye
        f = f / np.linalg.norm(f)
        r = np.cross(f, self.up)
        r = r / np.linalg.norm(r)
        u = np.cross(r, f)
        return r, u, f

    def project(self, p):
        """Pixel coordinates (x right, y down; pixel (i, j) covers
        [i, i+1) x [j, j+1)) and view depth of points p [..., 3]."""
        r, u, f = self.basis()
        d = p - self.eye
        z = d @ f
        t = np.tan(0.5 * self.fov_y)
        aspect = self.width / self.height
        ndc_x = (d @ r) / (z * t * aspect)
        ndc_y = (d @ u) / (z * t)
        x = (ndc_x + 1.0) * 0.5 * self.width
        y = (1.0 - ndc_y) * 0.5 * self.height
        return x, y, z


def sphere_view(width=3840, height=2160, distance=2.3, fov_y_deg=40.0):
    """A camera looking at the unit sphere's centre from `distance`: at 2.3
    and a 40 degree vertical field of view the sphere spans the frame's
    height and most of its width (its silhouette, where footprints turn
    anisotropic, is in view), and about a quarter of its faces face the
    camera."""
    d = np.array([0.31, 0.42, 1.45])
    return Camera(eye=d / np.linalg.norm(d) * distance, target=np.zeros(3),
                  up=np.array([0.0, 1.0, 0.0]), fov_y=np.deg2rad(fov_y_deg), width=width,
                  height=height)


@dataclasses.dataclass
class Frame:
    h: np.ndarray       # int32 [Q] visible halfedge per covered pixel
    u: np.ndarray       # float32 [Q]
    v: np.ndarray       # float32 [Q]
    jac: np.ndarray     # float32 [Q, 4] = du/dx, dv/dx, du/dy, dv/dy
    pixel: np.ndarray   # int64 [Q] = y * width + x (scanline order)
    depth: np.ndarray   # float64 [Q]

    @property
    def Q(self):
        return len(self.h)

    def footprint(self) -> np.ndarray:
        """Isotropic footprint (OpenGL's LOD scale): the longer of the two
        derivative vectors, in barycentric = quad units."""
        j = self.jac.astype(np.float64)
        px = np.hypot(j[:, 0], j[:, 1])
        py = np.hypot(j[:, 2], j[:, 3])
        return np.maximum(px, py).astype(np.float32)


def _persp_bary(cam, P, X, Y):
    """Perspective-correct barycentric weights of pixel points (X, Y) in
    triangles P [n, 3, 3]: solve for the point of the triangle's plane on
    the pixel's ray, in float64.  Returns (a0, a1, a2) per row."""
    r, up, f = cam.basis()
    t = np.tan(0.5 * cam.fov_y)
    aspect = cam.width / cam.height
    ndc_x = 2.0 * X / cam.width - 1.0
    ndc_y = 1.0 - 2.0 * Y / cam.height
    D = (f[None, :] + (ndc_x * t * aspect)[:, None] * r[None, :] +
         (ndc_y * t)[:, None] * up[None, :])                  # ray directions
    e1 = P[:, 0] - P[:, 2]
    e2 = P[:, 1] - P[:, 2]
    s = cam.eye[None, :] - P[:, 2]
    # eye + tau D = P2 + a0 e1 + a1 e2  (Cramer's rule)
    n = np.cross(e1, e2)
    det = -np.einsum("ij,ij->i", D, n)
    a0 = -np.einsum("ij,ij->i", D, np.cross(s, e2)) / det
    a1 = -np.einsum("ij,ij->i", D, np.cross(e1, s)) / det
    return a0, a1, 1.0 - a0 - a1


def rasterize(tri: np.ndarray, cam: Camera, chunk: int = 1 << 16) -> Frame:
    """Render intrinsic triangles tri [H, 3, 3] (v0, v1, v2 per halfedge).
    Front faces only (counter-clockwise on screen seen from the camera);
    pixel centres at (i + 1/2, j + 1/2); nearest triangle wins, ties to the
    smaller halfedge."""
    H = len(tri)
    W_, H_ = cam.width, cam.height
    v0, v1, v2 = tri[:, 0], tri[:, 1], tri[:, 2]
    x0, y0, z0 = cam.project(v0)
    x1, y1, z1 = cam.project(v1)
    x2, y2, z2 = cam.project(v2)
    area = (x0 - x2) * (y1 - y2) - (x1 - x2) * (y0 - y2)
    front = (area < 0) & (z0 > 0) & (z1 > 0) & (z2 > 0)   # y points down
    # pixels whose centre (i + 1/2, j + 1/2) lies in the triangle's box
    big = 1 << 30
    xmin = np.ceil(np.clip(np.minimum(np.minimum(x0, x1), x2), -big, big) - 0.5).astype(np.int64)
    xmax = np.floor(np.clip(np.maximum(np.maximum(x0, x1), x2), -big, big) - 0.5).astype(np.int64)
    ymin = np.ceil(np.clip(np.minimum(np.minimum(y0, y1), y2), -big, big) - 0.5).astype(np.int64)
    ymax = np.floor(np.clip(np.maximum(np.maximum(y0, y1), y2), -big, big) - 0.5).astype(np.int64)
    xmin = np.clip(xmin, 0, W_)
    ymin = np.clip(ymin, 0, H_)
    xmax = np.clip(xmax, -1, W_ - 1)
    ymax = np.clip(ymax, -1, H_ - 1)
    nx = np.maximum(xmax - xmin + 1, 0)
    ny = np.maximum(ymax - ymin + 1, 0)
    cand = np.where(front, nx * ny, 0)
    best_depth = np.full(W_ * H_, np.inf)
    best_h = np.full(W_ * H_, -1, dtype=np.int64)
    idx = np.nonzero(cand)[0]
    # chunks of triangles holding about `chunk` * 16 candidate pixels each
    csum = np.cumsum(cand[idx])
    cuts = np.searchsorted(csum, np.arange(chunk * 16, csum[-1] if len(csum) else 0,
                                           chunk * 16), side="right")
    bounds = [0] + [int(c) for c in cuts] + [len(idx)]
    for a, b in zip(bounds[:-1], bounds[1:]):
        t = idx[a:b]
        cnt = cand[t]
        if cnt.sum() == 0:
            continue
        tt = np.repeat(t, cnt)
        k = np.arange(cnt.sum()) - np.repeat(np.cumsum(cnt) - cnt, cnt)
        px = xmin[tt] + k % nx[tt]
        py = ymin[tt] + k // nx[tt]
        cx = px + 0.5
        cy = py + 0.5
        # edge functions: a front face has negative area with y down, so a
        # centre is covered when all three are <= 0 (pixels exactly on a
        # shared edge go to both triangles; visibility then keeps one)
        ax, ay = x0[tt], y0[tt]
        bx, by = x1[tt], y1[tt]
        qx, qy = x2[tt], y2[tt]
        w0 = (bx - cx) * (qy - cy) - (qx - cx) * (by - cy)
        w1 = (qx - cx) * (ay - cy) - (ax - cx) * (qy - cy)
        w2 = (ax - cx) * (by - cy) - (bx - cx) * (ay - cy)
        inside = ((w0 <= 0) & (w1 <= 0) & (w2 <= 0))
        tt, px, py, cx, cy = tt[inside], px[inside], py[inside], cx[inside], cy[inside]
        if len(tt) == 0:
            continue
        P = tri[tt]
        a0, a1, a2 = _persp_bary(cam, P, cx, cy)
        pt = a0[:, None] * P[:, 0] + a1[:, None] * P[:, 1] + a2[:, None] * P[:, 2]
        depth = (pt - cam.eye) @ cam.basis()[2]
        pix = py * W_ + px
        # nearest per pixel within the chunk, then against the frame
        order = np.lexsort((tt, depth, pix))
        pix_s, d_s, t_s = pix[order], depth[order], tt[order]
        firsts = np.r_[True, pix_s[1:] != pix_s[:-1]]
        pix_s, d_s, t_s = pix_s[firsts], d_s[firsts], t_s[firsts]
        better = (d_s < best_depth[pix_s]) | ((d_s == best_depth[pix_s]) & (t_s < best_h[pix_s]))
        best_depth[pix_s[better]] = d_s[better]
        best_h[pix_s[better]] = t_s[better]
    pix = np.nonzero(best_h >= 0)[0]
    h = best_h[pix]
    px = (pix % W_).astype(np.float64)
    py = (pix // W_).astype(np.float64)
    P = tri[h]
    out_u = np.empty(len(pix))
    out_v = np.empty(len(pix))
    jac = np.empty((len(pix), 4))
    for s in range(0, len(pix), 1 << 20):
        sl = slice(s, s + (1 << 20))
        Ps = P[sl]
        a0, a1, a2 = _persp_bary(cam, Ps, px[sl] + 0.5, py[sl] + 0.5)
        b0, b1, b2 = _persp_bary(cam, Ps, px[sl] + 1.5, py[sl] + 0.5)
        c0, c1, c2 = _persp_bary(cam, Ps, px[sl] + 0.5, py[sl] + 1.5)
        # (u, v) weigh v2 and v0
        out_u[sl], out_v[sl] = a2, a0
        jac[sl, 0], jac[sl, 1] = b2 - a2, b0 - a0
        jac[sl, 2], jac[sl, 3] = c2 - a2, c0 - a0
    return Frame(h=h.astype(np.int32), u=out_u.astype(np.float32), v=out_v.astype(np.float32),
                 jac=jac.astype(np.float32), pixel=pix.astype(np.int64),
                 depth=best_depth[pix])
