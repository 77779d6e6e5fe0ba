"""Lattice row orders for matrix ingest (host only)."""
import numpy as np
import pytest

from paper_1803_02156_amd.ordering import lattice_row_order


@pytest.mark.parametrize("dims,parts,slab", [((64, 64, 32), 8, 8), ((16, 16, 8), 8, 4), ((6, 5, 4), 8, 8),
                                             ((12, 8, 10), 4, 2), ((3, 3, 3), 8, 8)])
def test_is_a_permutation_with_orbitals_together(dims, parts, slab):
    n = 4 * int(np.prod(dims))
    o = lattice_row_order(*dims, parts=parts, slab=slab)
    assert o.dtype == np.int32 and o.shape == (n,)
    assert np.array_equal(np.sort(o), np.arange(n))
    q = o.reshape(-1, 4)
    assert np.all(q % 4 == np.arange(4)) and np.all(q // 4 == (q[:, :1] // 4))


def test_neighbour_distances_shrink():
    Nx, Ny, Nz = 64, 64, 32
    o = lattice_row_order(Nx, Ny, Nz)
    pos = np.empty(o.size, dtype=np.int64)
    pos[o] = np.arange(o.size)
    s = np.arange(Nx * Ny * Nz)
    x, y, z = s % Nx, (s // Nx) % Ny, s // (Nx * Ny)
    zn = x + Nx * (y + Ny * ((z + 1) % Nz))
    d_new = np.abs(pos[4 * zn] - pos[4 * s])
    d_old = 4 * Nx * Ny
    # within a box and slab the z-neighbour is one slab plane away (box_x * 8 sites)
    assert np.median(d_new) <= 4 * 32 * 8 < d_old
    # the boxes are contiguous eighths
    box_rows = o.size // 8
    sites_of = o.reshape(8, box_rows)[:, ::4] // 4
    for b in range(8):
        xs, ys, zs = sites_of[b] % Nx, (sites_of[b] // Nx) % Ny, sites_of[b] // (Nx * Ny)
        assert np.ptp(xs) < 64 and (np.ptp(xs) + 1) * (np.ptp(ys) + 1) * (np.ptp(zs) + 1) == box_rows // 4


def test_pencil_order_keeps_z_neighbours_close():
    Nx, Ny, Nz = 128, 128, 64
    s = np.arange(Nx * Ny * Nz)
    x, y, z = s % Nx, (s // Nx) % Ny, s // (Nx * Ny)
    zn = x + Nx * (y + Ny * ((z + 1) % Nz))
    for pencil in ((4, 4), (8, 4)):                        # default 4 x 4
        o = lattice_row_order(Nx, Ny, Nz, pencil=pencil)
        pos = np.empty(o.size, dtype=np.int64)
        pos[o] = np.arange(o.size)
        d = np.abs(pos[4 * zn] - pos[4 * s])
        assert np.median(d) == 4 * pencil[0] * pencil[1]
    assert np.array_equal(lattice_row_order(Nx, Ny, Nz), lattice_row_order(Nx, Ny, Nz, pencil=(4, 4)))
    o2 = lattice_row_order(6, 5, 4)                        # pencils do not divide: slabs
    assert np.array_equal(np.sort(o2), np.arange(o2.size))


def test_pencils_interleaved_over_sweeps():
    """With sweeps = 32, a site's x- or y-neighbour in another pencil of the same
    box sits in another sweep range at nearly the same offset: the ranges, swept
    side by side, reach both rows at about the same time.  (128x128x64: boxes of
    32 x 64 x 64 sites, 128 pencils of 4096 rows per box, 4 per range.)"""
    Nx, Ny, Nz = 128, 128, 64
    n_rows = 4 * Nx * Ny * Nz
    box_rows, span = n_rows // 8, n_rows // (8 * 32)
    s = np.arange(Nx * Ny * Nz)
    x, y, z = s % Nx, (s // Nx) % Ny, s // (Nx * Ny)
    nbrs = ((x + 1) % Nx + Nx * (y + Ny * z), x + Nx * ((y + 1) % Ny + Ny * z))
    # sweeps = 32, y: pencil rows r -> r + 1 with r % 4 == 3 (3 of the 15 inside a box) wrap to the
    # next position.  sweeps = 1 (x-fastest pencils, 4 to a range): x-neighbour pencils share a
    # range, 4084 rows apart; y-neighbour pencils (8 on) happen to sit two ranges on, aligned.
    for sweeps, bounds in ((32, ((1.0, 1.0), (0.79, 0.81))), (1, ((0.0, 0.0), (1.0, 1.0)))):
        o = lattice_row_order(Nx, Ny, Nz, sweeps=sweeps)
        pos = np.empty(o.size, dtype=np.int64)
        pos[o] = np.arange(o.size)
        for nb, (lo, hi) in zip(nbrs, bounds):
            a, b = pos[4 * s], pos[4 * nb]
            far = (a // box_rows == b // box_rows) & (np.abs(a - b) > 96)   # same box, outside the window
            close = np.mean(np.abs(a[far] % span - b[far] % span) <= 64)
            assert lo <= close <= hi, (sweeps, close)


def test_pencil_groups_shape():
    from paper_1803_02156_amd.ordering import pencil_groups
    assert pencil_groups(16, 32, 32) == (8, 4)
    assert pencil_groups(8, 16, 32) == (8, 4)
    assert pencil_groups(4, 8, 32) == (4, 8)
    assert pencil_groups(32, 1, 32) == (32, 1)
    assert pencil_groups(3, 5, 32) is None


def test_grouped_sweeps_take_neighbour_pencils_together():
    """Boxes of 16 x 16 pencils: the 32 ranges take 8 x 4 pencil blocks at a time,
    so fewer x/y neighbours outside the LDS window are swept at another time than
    with the plain deal (32 pencils of two pencil rows)."""
    import paper_1803_02156_amd.ordering as O
    Nx, Ny, Nz = 128, 256, 32
    s = np.arange(Nx * Ny * Nz)
    x, y, z = s % Nx, (s // Nx) % Ny, s // (Nx * Ny)
    nbrs = ((x + 1) % Nx + Nx * (y + Ny * z), x + Nx * ((y + 1) % Ny + Ny * z))

    def not_together(o):
        n_rows = o.size
        box_rows, span = n_rows // 8, n_rows // (8 * 32)
        pos = np.empty(o.size, dtype=np.int64)
        pos[o] = np.arange(o.size)
        out = 0.0
        for nb in nbrs:
            a, b = pos[4 * s], pos[4 * nb]
            far = np.abs(a - b) > 96
            together = (a // box_rows == b // box_rows) & (np.abs(a % span - b % span) <= 64)
            out += np.mean(far & ~together)
        return out
    grouped = not_together(O.lattice_row_order(Nx, Ny, Nz))
    saved = O.pencil_groups
    try:
        O.pencil_groups = lambda *a: None
        plain = not_together(O.lattice_row_order(Nx, Ny, Nz))
    finally:
        O.pencil_groups = saved
    assert grouped < 0.75 * plain, (grouped, plain)


@pytest.mark.parametrize("dims", [(64, 64, 32), (128, 128, 64)])
def test_window_halo_holds_the_lattice_neighbours(dims):
    """The window step kernel reads a gathered row from LDS when its permuted index
    lies within h tiles of the row's tile: h = 3 for 32-row tiles, h = 1 for
    64-row tiles.  In the default lattice order (4 x 4 pencils of 4 orbitals,
    z-neighbours 64 rows apart) both windows must hold at least 700 of 1000
    entries of a Topi row (the kernel's selection threshold), and the one-tile
    window of 64-row tiles as many as the three-tile window of 32-row tiles:
    every z-neighbour is inside, only x/y-neighbours in other pencils are not."""
    from topi import topi_csr
    Nx, Ny, Nz = dims
    rowptr, col, _ = topi_csr(Nx, Ny, Nz, m=1.0, W=1.0, seed=1)
    o = lattice_row_order(Nx, Ny, Nz)
    iperm = np.empty(o.size, dtype=np.int64)
    iperm[o] = np.arange(o.size)
    rows = np.repeat(np.arange(o.size), np.diff(rowptr))
    pr, pc = iperm[rows], iperm[col]
    share = {}
    for tr, h in ((32, 3), (64, 1)):
        t0 = pr // tr * tr
        share[tr] = np.count_nonzero((pc >= t0 - h * tr) & (pc < t0 + (h + 1) * tr)) * 1000 // len(col)
        assert share[tr] >= 700, (tr, share[tr])
    assert share[64] >= share[32] - 5, share
    # z-neighbours (4 x 4 x 4 = 64 rows apart in a pencil) are always inside the 64-row window
    s = np.arange(Nx * Ny * Nz)
    x, y, z = s % Nx, (s // Nx) % Ny, s // (Nx * Ny)
    zn = x + Nx * (y + Ny * ((z + 1) % Nz))
    same_box = (z + 1) % (Nz // 2 if Nz % 2 == 0 else Nz) != 0
    d = np.abs(iperm[4 * zn] // 64 - iperm[4 * s] // 64)
    assert np.all(d[same_box] <= 1)
