"""Scene preparation for the oracle: per-triangle planes and face grouping.

Test infrastructure: see the package docstring.

A face is a maximal set of triangles that lie in one plane and share one
material.  Candidate paths are ordered lists of scene primitives (paper
Sec. II-B); the image method depends only on the planes (and materials) that a
list visits, so primitives are identified by face.  Grouping rule: unit normal
n = (e1 x e2)/|e1 x e2| made canonical by flipping it so that its first
component with |n_i| > 1e-6 is positive; offset c = n . v0; two triangles share
a face when material, rint(n * 2^30) and rint(c * 2^30) all agree.  Faces are
numbered in order of their first triangle.
"""
from __future__ import annotations

import numpy as np

from .consts import PLANE_QUANT


def tri_vertices(V, F):
    V = np.asarray(V, dtype=np.float64)
    F = np.asarray(F, dtype=np.int64)
    return V[F[:, 0]], V[F[:, 1]], V[F[:, 2]]


def canonical_planes(V, F):
    """Canonical unit normals (nt, 3) and offsets (nt,) per triangle."""
    v0, v1, v2 = tri_vertices(V, F)
    n = np.cross(v1 - v0, v2 - v0)
    n = n / np.linalg.norm(n, axis=1, keepdims=True)
    big = np.abs(n) > 1e-6
    first = np.argmax(big, axis=1)
    sgn = np.sign(n[np.arange(n.shape[0]), first])
    n = n * sgn[:, None]
    c = np.einsum("ij,ij->i", n, v0)
    return n, c


def face_ids(V, F, tri_mat):
    """Face id per triangle (numbered by first appearance) and the number of faces."""
    n, c = canonical_planes(V, F)
    q = np.concatenate([np.asarray(tri_mat, dtype=np.int64)[:, None],
                        np.rint(n * PLANE_QUANT).astype(np.int64),
                        np.rint(c * PLANE_QUANT).astype(np.int64)[:, None]], axis=1)
    ids = np.empty(q.shape[0], dtype=np.int32)
    seen = {}
    for k, row in enumerate(map(tuple, q)):
        if row not in seen:
            seen[row] = len(seen)
        ids[k] = seen[row]
    return ids, len(seen)


class Geometry:
    """Float64 view of a scene used by every oracle module."""

    def __init__(self, scene):
        self.V = np.asarray(scene.V, dtype=np.float64)
        self.F = np.asarray(scene.F, dtype=np.int32)
        self.tri_mat = np.asarray(scene.tri_mat, dtype=np.int32)
        self.materials = np.asarray(scene.materials, dtype=np.float64)
        self.freq = float(scene.freq_hz)
        self.face, self.nfaces = face_ids(self.V, self.F, self.tri_mat)
        self.normal, self.offset = canonical_planes(self.V, self.F)
        v0, v1, v2 = tri_vertices(self.V, self.F)
        self.v0, self.v1, self.v2 = v0, v1, v2
        first = np.full(self.nfaces, -1, dtype=np.int64)
        for k in range(self.F.shape[0] - 1, -1, -1):
            first[self.face[k]] = k
        self.face_first_tri = first
        self.face_normal = self.normal[first]
        self.face_point = v0[first]
        self.face_mat = self.tri_mat[first]
        order = np.argsort(self.face, kind="stable")
        bounds = np.cumsum(np.bincount(self.face, minlength=self.nfaces))[:-1]
        self.face_tris = np.split(order, bounds)
