"""Voxel meshes with Q2 node lattices, boundary tags and part hierarchies.

Numbering: active voxels (elements) and used lattice nodes are both numbered
lexicographically with x fastest.  An element at voxel (ix, iy, iz) owns the
27 lattice nodes (2ix + a, 2iy + b, 2iz + c), a, b, c in {0, 1, 2}, in local
order a + 3b + 9c.  Coordinates: x = (lattice a) * h / 2 etc.
"""
import numpy as np
from scipy import ndimage

from .q2 import local_offsets

# face id -> (axis, side)   side 0 = low face, 1 = high face
FACES = [(0, 0), (0, 1), (1, 0), (1, 1), (2, 0), (2, 1)]


class VoxelMesh:
    def __init__(self, active, h):
        active = np.asarray(active, dtype=bool)
        self.nx, self.ny, self.nz = active.shape
        self.h = float(h)
        self.active = active
        # element list, x fastest: iterate A[iz, iy, ix] in C order
        iz, iy, ix = np.nonzero(active.transpose(2, 1, 0))
        self.elem_ijk = np.stack([ix, iy, iz], axis=1).astype(np.int64)
        self.n_elem = self.elem_ijk.shape[0]
        self.Lx, self.Ly, self.Lz = 2 * self.nx + 1, 2 * self.ny + 1, 2 * self.nz + 1
        off = local_offsets()
        lat = 2 * self.elem_ijk[:, None, :] + off[None, :, :]            # (E, 27, 3)
        lid = lat[..., 0] + self.Lx * (lat[..., 1] + self.Ly * lat[..., 2])
        used, inv = np.unique(lid.ravel(), return_inverse=True)
        self.node_lattice_id = used
        self.n_nodes = used.shape[0]
        self.elem_node = inv.reshape(self.n_elem, 27).astype(np.int32)
        a = used % self.Lx
        b = (used // self.Lx) % self.Ly
        c = used // (self.Lx * self.Ly)
        self.node_lat = np.stack([a, b, c], axis=1)
        self.node_xyz = self.node_lat * (0.5 * self.h)

    def elem_index_grid(self):
        g = -np.ones((self.nx, self.ny, self.nz), dtype=np.int64)
        g[self.elem_ijk[:, 0], self.elem_ijk[:, 1], self.elem_ijk[:, 2]] = np.arange(self.n_elem)
        return g

    def boundary_faces(self):
        """(element, face id) pairs whose neighbour voxel is absent or outside the grid."""
        shape = np.array([self.nx, self.ny, self.nz])
        out = []
        for f, (axis, side) in enumerate(FACES):
            nb = self.elem_ijk.copy()
            nb[:, axis] += 1 if side else -1
            inside = np.all((nb >= 0) & (nb < shape), axis=1)
            nb_active = np.zeros(self.n_elem, dtype=bool)
            nb_active[inside] = self.active[nb[inside, 0], nb[inside, 1], nb[inside, 2]]
            for e in np.nonzero(~nb_active)[0]:
                out.append((int(e), f))
        return out

    def face_nodes(self, e, f):
        axis, side = FACES[f]
        off = local_offsets()
        sel = off[:, axis] == (2 if side else 0)
        return self.elem_node[e, sel]


def axis_segments(n, rng=None, frac3=0.0):
    """Split range(n) into consecutive segments of length 2 (some 3): segment id per index."""
    seg = np.empty(n, dtype=np.int64)
    pos, s = 0, 0
    while pos < n:
        ln = 2
        if rng is not None and frac3 > 0 and rng.random() < frac3:
            ln = 3
        ln = min(ln, n - pos)
        if n - pos - ln == 1:          # never leave a segment of length one behind
            ln += 1
        seg[pos:pos + ln] = s
        pos += ln
        s += 1
    return seg


def part_hierarchy(mesh, seg_x, seg_y, seg_z, levels):
    """Level-1 parts from per-axis voxel segments; coarser levels group block coordinates 2x2x2.

    Returns elem_part (level-1 part per element), n_parts (levels-1 entries) and
    part_parent (levels-2 arrays).  Part ids are compacted in lexicographic
    order of block coordinates (x fastest); blocks without an active voxel are
    dropped.
    """
    ijk = mesh.elem_ijk
    bx, by, bz = seg_x[ijk[:, 0]], seg_y[ijk[:, 1]], seg_z[ijk[:, 2]]
    nbx, nby = seg_x.max() + 1, seg_y.max() + 1

    def compact(cx, cy, cz, sx, sy):
        key = cx + sx * (cy + sy * cz)
        uniq, inv = np.unique(key, return_inverse=True)
        return uniq, inv

    n_parts, part_parent = [], []
    if levels < 2:
        return np.zeros(mesh.n_elem, dtype=np.int32), [1], []
    uniq, elem_part = compact(bx, by, bz, nbx, nby)
    n_parts.append(len(uniq))
    # block coordinates of each level-1 part
    pcx, pcy, pcz = uniq % nbx, (uniq // nbx) % nby, uniq // (nbx * nby)
    sx, sy = nbx, nby
    for _ in range(levels - 2):
        cx, cy, cz = pcx // 2, pcy // 2, pcz // 2
        sx, sy = (sx + 1) // 2, (sy + 1) // 2
        uq, inv = compact(cx, cy, cz, sx, sy)
        part_parent.append(inv.astype(np.int32))
        n_parts.append(len(uq))
        pcx, pcy, pcz = uq % sx, (uq // sx) % sy, uq // (sx * sy)
    return elem_part.astype(np.int32), n_parts, part_parent


def die_voxels(nx, ny, nz, rng, target=0.20, tol=0.02):
    """Seeded die-like voxel channel: a box with cylinder and box obstacles.

    Obstacles (cylinders along y or z with radius 1.5-4 voxels and a seeded
    length, and boxes of 2-6 voxels per side) stay clear of the first and last
    two x-slabs and are added until the masked fraction lies in
    [target - tol, target + tol].  Only the face-connected component that
    touches both x-ends is kept.
    """
    active = np.ones((nx, ny, nz), dtype=bool)
    total = active.size
    cx, cy, cz = np.meshgrid(np.arange(nx) + 0.5, np.arange(ny) + 0.5, np.arange(nz) + 0.5, indexing="ij")
    tries = 0
    while (1.0 - active.mean()) < target - tol and tries < 10000:
        tries += 1
        m = np.zeros_like(active)
        if rng.random() < 0.5:
            r = rng.uniform(1.5, 4.0)
            x0 = rng.uniform(2 + r, nx - 2 - r) if nx - 4 > 2 * r else nx / 2
            if rng.random() < 0.5:      # axis y
                c2 = rng.uniform(0, nz)
                lo = rng.uniform(0, ny * 0.5)
                hi = lo + rng.uniform(0.5, 1.0) * ny
                m = ((cx - x0) ** 2 + (cz - c2) ** 2 <= r * r) & (cy >= lo) & (cy <= hi)
            else:                       # axis z
                c2 = rng.uniform(0, ny)
                lo = rng.uniform(0, nz * 0.5)
                hi = lo + rng.uniform(0.5, 1.0) * nz
                m = ((cx - x0) ** 2 + (cy - c2) ** 2 <= r * r) & (cz >= lo) & (cz <= hi)
        else:
            sx, sy, sz = rng.integers(2, 7, size=3)
            x0 = rng.integers(2, max(3, nx - 2 - sx + 1))
            y0 = rng.integers(0, max(1, ny - sy + 1))
            z0 = rng.integers(0, max(1, nz - sz + 1))
            m[x0:x0 + sx, y0:y0 + sy, z0:z0 + sz] = True
        m[:2] = False
        m[nx - 2:] = False
        trial = active & ~m
        if (1.0 - trial.mean()) > target + tol:
            continue
        active = trial
    lab, _ = ndimage.label(active)
    left = set(np.unique(lab[0])) - {0}
    right = set(np.unique(lab[-1])) - {0}
    keep = sorted(left & right)
    if not keep:
        raise RuntimeError("die generator: no channel connects both x-ends")
    sizes = [(lab == k).sum() for k in keep]
    active = lab == keep[int(np.argmax(sizes))]
    assert active.sum() <= total
    return active
