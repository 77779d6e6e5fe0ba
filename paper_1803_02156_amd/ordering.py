"""Row orders for lattice Hamiltonians, passed to ``chebfd_matrix_build(order=...)``.

A fused Chebyshev step gathers, for every row, the block-vector rows of its
lattice neighbours.  In the natural order (x fastest, then y, then z) the
z-neighbours of a site are Nx Ny sites away, so on a large lattice they have
left the cache before they are gathered again and the block vector U is read
from memory about three times per step instead of once.  The orders here
shorten those distances without changing the matrix (a symmetric permutation,
like the sigma sort of SELL-C-sigma itself):

* the lattice is cut into ``parts`` boxes (one per L2 domain: the step kernel
  hands each of the eight XCDs of the device one contiguous eighth of the
  rows), and
* inside a box, sites are taken in pencils of px x py sites swept along z, so a
  site's z-neighbours are px py sites away instead of a whole lattice plane
  (measured on the 128x128x64 lattice: HBM reads of a step 1.94 x the
  algorithmic bytes in the natural order, 1.36 x with 8 x 4 pencils), or in
  y-slabs swept z-plane by z-plane.

With the default 4 x 4 pencils (4 orbitals) a z-neighbour is 64 rows away and
84 % of the entries lie within three 32-row tiles of their row, which lets the
FP64 step stage the gathered block in LDS (the window kernel; 8 x 4 pencils put
z-neighbours 128 rows away, outside that window).

Orbitals of a site stay consecutive (row = orbitals * site + orbital).
"""
from __future__ import annotations

import numpy as np


def _split(dims, parts):
    """Factor `parts` (a power of two) over the three extents, largest extent first."""
    split = [1, 1, 1]
    ext = list(dims)
    p = parts
    while p > 1:
        k = int(np.argmax([e / s if e % (2 * s) == 0 else 0 for e, s in zip(ext, split)]))
        if ext[k] % (2 * split[k]) != 0:
            return None
        split[k] *= 2
        p //= 2
    return tuple(split)


def pencil_groups(npx: int, npy: int, sweeps: int):
    """Shape (gx, gy), gx gy = sweeps, of the block of pencils that the sweep ranges of
    one box take at the same time, or None when no such block tiles the npx x npy
    pencils.  A gather that leaves its pencil in x or y finds its row in L2 when the
    neighbour pencil is in the same block; the faces on the block's edge miss, a
    share of 1 / gx of the x faces and 1 / gy of the y faces: the shape minimising
    1 / gx + 1 / gy (wider in x on ties) is taken."""
    best = None
    for gx in range(1, sweeps + 1):
        if sweeps % gx:
            continue
        gy = sweeps // gx
        if npx % gx or npy % gy:
            continue
        cost = 1.0 / gx + 1.0 / gy
        if best is None or cost < best[0] - 1e-12 or (abs(cost - best[0]) <= 1e-12 and gx > best[1]):
            best = (cost, gx, gy)
    return None if best is None else (best[1], best[2])


def lattice_row_order(Nx: int, Ny: int, Nz: int, orbitals: int = 4, parts: int = 8, slab: int = 8,
                      pencil=(4, 4), sweeps: int = 32):
    """Row order (int32 permutation of 0..n-1, order[k] = original row placed k-th) for a
    lattice with site index x + Nx (y + Ny z) and row orbitals * site + orbital.

    Inside a box, pencils of px x py sites (``pencil``, default 4 x 4) are swept
    along z, so that z-neighbours are px py sites apart and x/y-neighbours are in
    the same or an adjacent pencil; with ``pencil=None``, or when px, py do not
    divide the box extents, y-slabs of ``slab`` lines are swept z-plane by z-plane
    instead.  Falls back to fewer boxes when the extents do not split evenly, and
    to slabs of the full box width when ``slab`` does not divide it.

    ``sweeps``: the window step kernel splits each box's rows into this many
    contiguous ranges, swept side by side by the workgroups of one XCD (32 CUs
    per XCD).  When it divides the number of pencils of a box, the ranges take
    a block of gx x gy pencils at a time (``pencil_groups``; 8 x 4 for 32
    ranges where the box allows it): the pencils next to a pencil in x and y are
    then mostly swept at the same time by other workgroups of the same XCD, and
    the gathers that leave a workgroup's LDS window find their rows in L2.
    When no block shape fits, pencil p goes to range p % sweeps (position
    p // sweeps).  ``sweeps=1`` keeps the pencils in x-fastest order."""
    dims = (int(Nx), int(Ny), int(Nz))
    split = None
    while parts >= 1 and split is None:
        split = _split(dims, parts)
        if split is None:
            parts //= 2
    px, py, pz = split
    bx, by, bz = Nx // px, Ny // py, Nz // pz
    sy = slab if (slab >= 1 and by % slab == 0) else by
    x, y, z = np.meshgrid(np.arange(Nx), np.arange(Ny), np.arange(Nz), indexing="ij")
    x, y, z = x.ravel(), y.ravel(), z.ravel()
    site = x + Nx * (y + Ny * z)
    box = (x // bx) + px * ((y // by) + py * (z // bz))
    ly = y % by
    # lexsort: the last key is the primary one
    if pencil is not None and bx % pencil[0] == 0 and by % pencil[1] == 0:
        # pencils of px x py sites swept along z: z-neighbours px py sites apart
        px, py = pencil
        lx = x % bx
        npx, npen = bx // px, (bx // px) * (by // py)
        ipx, ipy = lx // px, ly // py                      # pencil coordinates in the box
        npy = by // py
        pen = ipx + npx * ipy                               # pencil index in the box, x fastest
        grp = pencil_groups(npx, npy, sweeps) if sweeps > 1 and npen % sweeps == 0 else None
        if grp is not None:
            # the sweeps side by side take a gx x gy block of pencils at a time: range
            # r = (ipx % gx) + gx (ipy % gy), position = block index (x fastest)
            gx, gy = grp
            r = ipx % gx + gx * (ipy % gy)
            blk = ipx // gx + (npx // gx) * (ipy // gy)
            pen = r * (npen // sweeps) + blk
        elif sweeps > 1 and npen % sweeps == 0:
            pen = (pen % sweeps) * (npen // sweeps) + pen // sweeps
        key = np.lexsort((lx % px, ly % py, z % bz, pen, box))
    else:
        key = np.lexsort((x % bx, ly, z % bz, ly // sy, box))
    sites = site[key]
    rows = (orbitals * sites[:, None] + np.arange(orbitals)[None, :]).ravel()
    return rows.astype(np.int32)
