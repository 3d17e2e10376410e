"""Brute-force per-pixel ray casting (test helper, FP64, no snapping).

An independent check of the oracle's visibility: every pixel-centre ray of a frame is
intersected with every triangle by the Moller-Trumbore test (Moller & Trumbore,
"Fast, minimum storage ray-triangle intersection", JGT 1997), keeping front faces
only, and the nearest hit wins.  It uses the unsnapped FP64 geometry, so it agrees
with the rasterizer's answer everywhere except within the sub-pixel snapping band of
a projected edge and where two surfaces are almost at the same depth; ``edge_dist``
reports the first so tests can exclude it.
"""
from __future__ import annotations

import numpy as np


def frame_triangles(batch, f):
    """View-space vertices [T,3,3], vertex normals [T,3,3] (view space), scene-local
    triangle IDs [T] and object index [T] of the visible objects of frame f."""
    s = int(batch.frame_scene[f])
    V = batch.view[f].astype(np.float64)
    R_v, t_v = V[:, :3], V[:, 3]
    tris, nrms, ids, objs = [], [], [], []
    base = 0
    for o in range(batch.scene_object_begin[s], batch.scene_object_begin[s + 1]):
        mesh = batch.meshes[batch.object_mesh[o]]
        P = batch.object_pose[o].astype(np.float64)
        if batch.object_visible[o]:
            world = mesh.pos.astype(np.float64) @ P[:, :3].T + P[:, 3]
            eye = world @ R_v.T + t_v
            n = mesh.nrm.astype(np.float64) @ (R_v @ P[:, :3]).T
            n /= np.linalg.norm(n, axis=1, keepdims=True)
            tris.append(eye[mesh.idx])
            nrms.append(n[mesh.idx])
            ids.append(base + np.arange(mesh.n_tris))
            objs.append(np.full(mesh.n_tris, o))
        base += mesh.n_tris
    if not tris:
        z = np.zeros((0, 3, 3))
        return z, z, np.zeros(0, np.int64), np.zeros(0, np.int64)
    return np.concatenate(tris), np.concatenate(nrms), np.concatenate(ids), np.concatenate(objs)


def pixel_rays(batch, f):
    W, H = int(batch.width[f]), int(batch.height[f])
    fx, fy, cx, cy = batch.intr[f].astype(np.float64)
    j, i = np.mgrid[0:H, 0:W]
    r = np.stack([(i + 0.5 - cx) / fx, -(j + 0.5 - cy) / fy, -np.ones_like(i, float)], -1)
    return r.reshape(-1, 3)


def cast(batch, f, chunk: int = 128):
    """Nearest front-facing hit per pixel.

    Returns dict(tri [P] (-1 = miss), obj [P], depth [P] (eye depth), depth2 [P]
    (second-nearest hit, +inf), bary [P,3] (weights of the triangle's 3 vertices),
    normal [P,3] (interpolated unit view-space normal))."""
    T, N, ids, objs = frame_triangles(batch, f)
    r = pixel_rays(batch, f)
    P = r.shape[0]
    best = np.full(P, np.inf)
    second = np.full(P, np.inf)
    tri = np.full(P, -1, np.int64)
    bu = np.zeros(P)
    bv = np.zeros(P)
    for k0 in range(0, T.shape[0], chunk):
        v0, v1, v2 = T[k0:k0 + chunk, 0], T[k0:k0 + chunk, 1], T[k0:k0 + chunk, 2]
        e1, e2 = v1 - v0, v2 - v0
        pvec = np.cross(r[:, None, :], e2[None])                # [P,k,3]
        det = np.einsum("pkc,kc->pk", pvec, e1)
        front = det > 0
        inv = np.where(front, 1.0 / np.where(front, det, 1.0), 0.0)
        tvec = -v0[None]                                         # origin at the eye
        u = np.einsum("pkc,pkc->pk", np.broadcast_to(tvec, pvec.shape), pvec) * inv
        q = np.cross(np.broadcast_to(tvec, pvec.shape), e1[None])
        v = np.einsum("pc,pkc->pk", r, q) * inv
        t = np.einsum("kc,pkc->pk", e2, q) * inv
        hit = front & (u >= 0) & (v >= 0) & (u + v <= 1) & (t > 0)
        t = np.where(hit, t, np.inf)
        for kk in range(t.shape[1]):
            tk = t[:, kk]
            closer = tk < best
            second = np.where(closer, best, np.minimum(second, tk))
            best = np.where(closer, tk, best)
            tri = np.where(closer, k0 + kk, tri)
            bu = np.where(closer, u[:, kk], bu)
            bv = np.where(closer, v[:, kk], bv)
    hitp = tri >= 0
    bary = np.stack([1 - bu - bv, bu, bv], -1)
    nrm = np.zeros((P, 3))
    if hitp.any():
        nn = np.einsum("pk,pkc->pc", bary[hitp], N[tri[hitp]])
        nrm[hitp] = nn / np.linalg.norm(nn, axis=1, keepdims=True)
    return dict(tri=np.where(hitp, ids[np.maximum(tri, 0)], -1), obj=np.where(hitp, objs[np.maximum(tri, 0)], -1),
                depth=np.where(hitp, best, 0.0), depth2=second, bary=bary, normal=nrm)


def edge_dist(batch, f, chunk: int = 512):
    """Distance in pixels from every pixel centre to the nearest projected edge of a
    front-facing triangle in front of the camera (unsnapped projection)."""
    T, _, _, _ = frame_triangles(batch, f)
    W, H = int(batch.width[f]), int(batch.height[f])
    fx, fy, cx, cy = batch.intr[f].astype(np.float64)
    j, i = np.mgrid[0:H, 0:W]
    pc = np.stack([i + 0.5, j + 0.5], -1).reshape(-1, 2)
    dist = np.full(pc.shape[0], np.inf)
    if T.shape[0] == 0:
        return dist
    w = -T[..., 2]
    ok = np.all(w > 1e-6, axis=1)
    T, w = T[ok], w[ok]
    s = np.stack([fx * T[..., 0] / w + cx, -fy * T[..., 1] / w + cy], -1)  # [T,3,2]
    cr = (s[:, 1, 0] - s[:, 0, 0]) * (s[:, 2, 1] - s[:, 0, 1]) - (s[:, 1, 1] - s[:, 0, 1]) * (s[:, 2, 0] - s[:, 0, 0])
    s = s[cr < 0]  # front faces are clockwise on a y-down screen
    a = np.concatenate([s[:, 0], s[:, 1], s[:, 2]])
    b = np.concatenate([s[:, 1], s[:, 2], s[:, 0]])
    for k0 in range(0, a.shape[0], chunk):
        A, B = a[k0:k0 + chunk], b[k0:k0 + chunk]
        d = B - A
        L2 = np.maximum((d * d).sum(-1), 1e-300)
        rel = pc[:, None, :] - A[None]
        tt = np.clip((rel * d[None]).sum(-1) / L2, 0, 1)
        proj = A[None] + tt[..., None] * d[None]
        dd = np.sqrt(((pc[:, None, :] - proj) ** 2).sum(-1))
        dist = np.minimum(dist, dd.min(1))
    return dist
