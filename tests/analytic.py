"""Closed-form references used to pin the oracle (test code, FP64).

* Exact pixel coverage of projected triangles (box pixel filter): the pixel
  integral of eq. first for piecewise-constant radiance is an area, computed by
  convex polygon clipping (Sutherland-Hodgman).
* Lambert's closed form for the irradiance from a uniform polygonal emitter
  (the analytic irradiance line of work the thesis cites as Arvo 1994):
  E(x) = L_e/2 * sum_i Theta_i * (n . Gamma_i), with Gamma_i the unit normal of
  the plane through x and polygon edge i, Theta_i the angle it subtends.

Neither module shares code with the oracle or the HIP path; derivatives are
taken by central differences of these exact, smooth functions.
"""
from __future__ import annotations

import math

import numpy as np


def clip_polygon(poly, a, b, c):
    """Keep the part of polygon (list of 2D points) with a*x + b*y + c >= 0."""
    out = []
    n = len(poly)
    for i in range(n):
        p, q = poly[i], poly[(i + 1) % n]
        fp = a * p[0] + b * p[1] + c
        fq = a * q[0] + b * q[1] + c
        if fp >= 0:
            out.append(p)
        if (fp >= 0) != (fq >= 0):
            t = fp / (fp - fq)
            out.append((p[0] + t * (q[0] - p[0]), p[1] + t * (q[1] - p[1])))
    return out


def poly_area(poly):
    s = 0.0
    for i in range(len(poly)):
        p, q = poly[i], poly[(i + 1) % len(poly)]
        s += p[0] * q[1] - q[0] * p[1]
    return 0.5 * s


def ccw(poly):
    return poly if poly_area(poly) >= 0 else poly[::-1]


def clip_convex(poly, clipper):
    """Intersection of a polygon with a convex CCW clipper polygon."""
    for i in range(len(clipper)):
        if not poly:
            return []
        p, q = clipper[i], clipper[(i + 1) % len(clipper)]
        # left of p->q: (q-p) x (x-p) >= 0
        a = -(q[1] - p[1])
        b = q[0] - p[0]
        c = -(a * p[0] + b * p[1])
        poly = clip_polygon(poly, a, b, c)
    return poly


def box_clip_area(poly, x0, y0, x1, y1):
    poly = clip_polygon(poly, 1, 0, -x0)
    if poly:
        poly = clip_polygon(poly, -1, 0, x1)
    if poly:
        poly = clip_polygon(poly, 0, 1, -y0)
    if poly:
        poly = clip_polygon(poly, 0, -1, y1)
    return abs(poly_area(poly)) if len(poly) >= 3 else 0.0


# ---------------------------------------------------------------------------
# pinhole camera (definition: look-at frame, d = f + ndc_x*asp*t*r + ndc_y*t*u,
# screen in pixels with y down)
# ---------------------------------------------------------------------------

def camera_frame(pos, look, up):
    pos, look, up = (np.asarray(v, np.float64) for v in (pos, look, up))
    f = look - pos
    f /= np.linalg.norm(f)
    r = np.cross(f, up)
    r /= np.linalg.norm(r)
    u = np.cross(r, f)
    return pos, f, r, u


def project(P, cam9, fov_deg, W, H):
    c, f, r, u = camera_frame(cam9[0:3], cam9[3:6], cam9[6:9])
    t = math.tan(math.radians(fov_deg) / 2)
    q = np.asarray(P, np.float64) - c
    z = q @ f
    sx = W / 2 * (1 + (q @ r) / (z * (W / H) * t))
    sy = H / 2 * (1 - (q @ u) / (z * t))
    return np.stack([sx, sy], -1)


def screen_ray(sx, sy, cam9, fov_deg, W, H):
    c, f, r, u = camera_frame(cam9[0:3], cam9[3:6], cam9[6:9])
    t = math.tan(math.radians(fov_deg) / 2)
    nx = 2 * sx / W - 1
    ny = 1 - 2 * sy / H
    d = f[None] + np.outer(nx * (W / H) * t, r) + np.outer(ny * t, u)
    return c, d


# ---------------------------------------------------------------------------
# exact image of two emissive triangles over a constant background
# ---------------------------------------------------------------------------

def two_triangle_image(verts, emission, background, cam9, fov, W, H, window=None):
    """Exact box-filtered image (pixel integrals) for two non-intersecting
    triangles with constant two-sided emission."""
    verts = np.asarray(verts, np.float64).reshape(2, 3, 3)
    x0, y0, x1, y1 = window if window is not None else (0, 0, W, H)
    s = [ccw([tuple(p) for p in project(verts[i], cam9, fov, W, H)]) for i in range(2)]
    inter = clip_convex(s[0], s[1])
    front = 0
    if len(inter) >= 3:
        # depth order from a point inside the overlap
        cx = sum(p[0] for p in inter) / len(inter)
        cy = sum(p[1] for p in inter) / len(inter)
        o, d = screen_ray(np.array([cx]), np.array([cy]), cam9, fov, W, H)
        depth = []
        for i in range(2):
            a, b, c = verts[i]
            n = np.cross(b - a, c - a)
            depth.append(((a - o) @ n) / (d[0] @ n))
        front = 0 if depth[0] < depth[1] else 1
    back = 1 - front
    img = np.full((y1 - y0, x1 - x0), float(background))
    allp = np.concatenate([np.array(s[0]), np.array(s[1])])
    bx0 = max(x0, int(math.floor(allp[:, 0].min())))
    bx1 = min(x1, int(math.ceil(allp[:, 0].max())))
    by0 = max(y0, int(math.floor(allp[:, 1].min())))
    by1 = min(y1, int(math.ceil(allp[:, 1].max())))
    for py in range(by0, by1):
        for px in range(bx0, bx1):
            af = box_clip_area(s[front], px, py, px + 1, py + 1)
            ab = box_clip_area(s[back], px, py, px + 1, py + 1)
            afb = box_clip_area(inter, px, py, px + 1, py + 1) if len(inter) >= 3 else 0.0
            img[py - y0, px - x0] = (background * (1 - af - ab + afb) + emission[front] * af
                                     + emission[back] * (ab - afb))
    return img


def near_clip(poly3d, cam9, near):
    """Part of a planar 3D polygon at camera-space depth >= near
    (Sutherland-Hodgman against the near plane)."""
    c, f, _, _ = camera_frame(cam9[0:3], cam9[3:6], cam9[6:9])
    pts = [np.asarray(p, np.float64) for p in poly3d]
    out = []
    for i in range(len(pts)):
        p, q = pts[i], pts[(i + 1) % len(pts)]
        dp, dq = (p - c) @ f - near, (q - c) @ f - near
        if dp >= 0:
            out.append(p)
        if (dp >= 0) != (dq >= 0):
            out.append(p + (q - p) * (dp / (dp - dq)))
    return out


def near_clipped_two_triangle_image(verts, emission, background, cam9, fov, W, H, near, window=None):
    """Exact box-filtered image of two non-intersecting emissive triangles
    (constant two-sided emission) when geometry nearer than `near` (camera-
    space depth) is invisible: each triangle is clipped against the near plane
    in 3D, then its visible polygon is projected. The clipped polygon's new
    side lies on the near plane and must project outside the window (it is not
    a mesh edge)."""
    verts = np.asarray(verts, np.float64).reshape(2, 3, 3)
    x0, y0, x1, y1 = window if window is not None else (0, 0, W, H)
    polys3 = [near_clip(verts[i], cam9, near) for i in range(2)]
    s = [ccw([tuple(p) for p in project(np.array(polys3[i]), cam9, fov, W, H)]) if len(polys3[i]) >= 3 else []
         for i in range(2)]
    inter = clip_convex(s[0], s[1]) if s[0] and s[1] else []
    front = 0
    if len(inter) >= 3:
        cx = sum(p[0] for p in inter) / len(inter)
        cy = sum(p[1] for p in inter) / len(inter)
        o, d = screen_ray(np.array([cx]), np.array([cy]), cam9, fov, W, H)
        depth = []
        for i in range(2):
            a, b, c = verts[i]
            n = np.cross(b - a, c - a)
            depth.append(((a - o) @ n) / (d[0] @ n))
        front = 0 if depth[0] < depth[1] else 1
    back = 1 - front
    img = np.full((y1 - y0, x1 - x0), float(background))
    for py in range(y0, y1):
        for px in range(x0, x1):
            af = box_clip_area(s[front], px, py, px + 1, py + 1) if s[front] else 0.0
            ab = box_clip_area(s[back], px, py, px + 1, py + 1) if s[back] else 0.0
            afb = box_clip_area(inter, px, py, px + 1, py + 1) if len(inter) >= 3 else 0.0
            img[py - y0, px - x0] = (background * (1 - af - ab + afb) + emission[front] * af
                                     + emission[back] * (ab - afb))
    return img


# ---------------------------------------------------------------------------
# Lambert: irradiance from a uniform planar polygon
# ---------------------------------------------------------------------------

def polygon_irradiance(x, n, poly, Le):
    """Irradiance at x (normal n) from a planar polygon (k x 3, any winding)
    of constant radiance Le, fully visible and above x's tangent plane."""
    if len(poly) < 3:
        return 0.0
    E = 0.0
    k = len(poly)
    for i in range(k):
        a = poly[i] - x
        b = poly[(i + 1) % k] - x
        cr = np.cross(a, b)
        ln = np.linalg.norm(cr)
        if ln == 0:
            continue
        theta = math.atan2(ln, float(a @ b))
        E += theta * float(n @ (cr / ln))
    return abs(0.5 * Le * E)


def shadowed_irradiance(x, n, light, occ, Le):
    """Irradiance at x from a convex planar light polygon partly hidden by a
    triangle occluder lying strictly between x and the light's plane."""
    light = np.asarray(light, np.float64)
    occ = np.asarray(occ, np.float64)
    ln = np.cross(light[1] - light[0], light[2] - light[0])
    ln /= np.linalg.norm(ln)
    d0 = ln @ light[0]
    # project occluder vertices from x onto the light plane
    proj = []
    for q in occ:
        t = (d0 - ln @ x) / (ln @ (q - x))
        proj.append(x + (q - x) * t)
    proj = np.array(proj)
    # 2D coordinates in the light plane
    e1 = light[1] - light[0]
    e1 /= np.linalg.norm(e1)
    e2 = np.cross(ln, e1)
    to2 = lambda P: [(float((p - light[0]) @ e1), float((p - light[0]) @ e2)) for p in P]
    L2 = ccw(to2(light))
    S2 = ccw(to2(proj))
    I2 = clip_convex(S2, L2)
    full = polygon_irradiance(x, n, light, Le)
    if len(I2) < 3:
        return full
    I3 = np.array([light[0] + e1 * p[0] + e2 * p[1] for p in I2])
    return full - polygon_irradiance(x, n, I3, Le)
