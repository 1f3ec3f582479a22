"""Pins of the oracle's Esirkepov deposit, whole step and tile sort.

Deposit:
  * discrete continuity (rho1 - rho0)/dt + div J = 0 to roundoff, orders
    1..3, 2D and 3D, including grids smaller than the stencil (it wraps
    onto itself);
  * order 1, particle staying inside one cell: the current equals the exact
    charge flux of the unit-cube cloud through each face along the straight
    path, integrated numerically in time (an independent route);
  * order 1, 1D motion crossing a node: the textbook split of the flux
    between the two edges;
  * 3D with one cell along y reproduces the 2D Jx and Jz; the 2D
    out-of-plane Jy equals the y-line sum of the 3D Jy of a particle moving
    in y;
  * grid sum of J equals q w v / dV.
Whole step: Gauss's law residual div E - rho is constant to roundoff.
Sort: equals Python's stable ``sorted`` and every key names the tile of
the particle's cell.
"""
import math

import numpy as np
import pytest

import oracle
from pic_inputs import SimpleSpecies

ORDERS = (1, 2, 3)


def _sp(x, u, w, q=-1.0, m=1.0):
    return SimpleSpecies(q, m, np.ascontiguousarray(x, dtype=np.float64),
                         np.ascontiguousarray(u, dtype=np.float64),
                         np.ascontiguousarray(w, dtype=np.float64))


def _continuity(dim, n, order, dx, npart, seed, maxstep=0.9):
    dt = 0.7
    g = oracle.make_grid(dim, n, dx, dt, order)
    N = n[0] * n[1] * n[2]
    rng = np.random.default_rng(seed)
    x0 = rng.uniform(0, 1, (3, npart)) * np.array(n)[:, None]
    dxp = rng.uniform(-maxstep, maxstep, (3, npart))
    if dim == 2:
        x0[1] = 0.0
        dxp[1] = 0.0
    x1 = x0 + dxp
    w = rng.uniform(0.5, 2.0, npart)
    q = -1.0
    J = np.zeros((3, N))
    for p in range(npart):
        oracle.deposit(g, J, q, w[p], x0[:, p], x1[:, p], 0.3)
    x1w = np.array([[oracle.wrap(x1[d, p], n[d]) if not (dim == 2 and d == 1) else 0.0
                     for p in range(npart)] for d in range(3)])
    u = np.zeros((3, npart))
    r0 = oracle.rho(g, [_sp(x0, u, w, q)], N)
    r1 = oracle.rho(g, [_sp(x1w, u, w, q)], N)
    dj = oracle.div_j(g, J, N)
    res = (r1 - r0) / dt + dj
    scale = np.max(np.abs(dj)) + np.max(np.abs(r0)) / dt
    return np.max(np.abs(res)) / scale, J


@pytest.mark.parametrize("order", ORDERS)
@pytest.mark.parametrize("dim", (2, 3))
def test_continuity_roundoff(order, dim):
    n = (7, 6, 5) if dim == 3 else (7, 1, 5)
    err, _ = _continuity(dim, n, order, (1.0, 1.0, 1.0), 40, 21 + order)
    assert err < 1e-14


@pytest.mark.parametrize("order", ORDERS)
def test_continuity_tiny_wrapping_grid_and_anisotropic_cells(order):
    err, _ = _continuity(3, (3, 2, 4), order, (0.7, 1.2, 1.0), 20, 31 + order)
    assert err < 1e-14
    err, _ = _continuity(2, (3, 1, 2), order, (1.1, 1.0, 0.9), 20, 41 + order)
    assert err < 1e-14


def _cube_flux(x0, x1, dt, axis, face, j, k, nq=4000):
    """Exact flux of a unit-cube cloud (unit charge) through the face
    x_axis = face + 1/2 restricted to the transverse cell (j, k), integrated
    over the straight path x0 -> x1 by the midpoint rule (the integrand is
    piecewise smooth; the test paths keep it polynomial)."""
    t = (np.arange(nq) + 0.5) / nq
    pos = x0[:, None] + (x1 - x0)[:, None] * t[None, :]
    oth = [d for d in range(3) if d != axis]
    over = np.abs(pos[axis] - (face + 0.5)) < 0.5
    ov = lambda p, c: np.clip(1.0 - np.abs(p - c), 0.0, None)
    trans = ov(pos[oth[0]], j) * ov(pos[oth[1]], k)
    v = (x1[axis] - x0[axis]) / dt
    return v * np.mean(over * trans)


def test_order1_equals_exact_cloud_flux_inside_a_cell():
    n = (6, 6, 6)
    dt = 0.5
    g = oracle.make_grid(3, n, (1, 1, 1), dt, 1)
    N = 216
    rng = np.random.default_rng(51)
    for _ in range(6):
        c = rng.integers(1, 4, 3).astype(float)
        a = c + rng.uniform(0.05, 0.45, 3)
        b = c + rng.uniform(0.55, 0.95, 3)
        x0, x1 = (a, b) if rng.uniform() < 0.5 else (b, a)
        J = np.zeros((3, N))
        oracle.deposit(g, J, 1.0, 1.0, x0, x1, 0.0)
        Jr = J.reshape(3, n[2], n[1], n[0])
        for axis in range(3):
            for f0 in range(n[0]):
                for p in range(n[1]):
                    for r in range(n[2]):
                        idx = [f0, p, r] if axis == 0 else ([p, f0, r] if axis == 1 else [p, r, f0])
                        face = idx[axis]
                        jj, kk = [idx[d] for d in range(3) if d != axis]
                        ref = _cube_flux(x0, x1, dt, axis, face, jj, kk)
                        got = Jr[axis, idx[2], idx[1], idx[0]]
                        assert abs(got - ref) < 2e-6, (axis, idx, got, ref)


def test_order1_1d_crossing_split():
    n = (8, 4, 4)
    dt = 0.5
    g = oracle.make_grid(3, n, (1, 1, 1), dt, 1)
    J = np.zeros((3, 128))
    x0 = np.array([2.7, 1.0, 1.0])   # on nodes transversally: weight 1 at (1, 1)
    x1 = np.array([3.2, 1.0, 1.0])
    oracle.deposit(g, J, 1.0, 1.0, x0, x1, 0.0)
    Jr = J.reshape(3, 4, 4, 8)
    # path 2.7 -> 3.0 inside cell [2, 3] and 3.0 -> 3.2 inside [3, 4]
    assert abs(Jr[0, 1, 1, 2] - 0.3 / dt) < 1e-15
    assert abs(Jr[0, 1, 1, 3] - 0.2 / dt) < 1e-15
    Jr[0, 1, 1, 2] = Jr[0, 1, 1, 3] = 0.0
    assert np.max(np.abs(Jr)) == 0.0


@pytest.mark.parametrize("order", ORDERS)
def test_3d_one_y_cell_matches_2d_in_plane_current(order):
    n = (6, 1, 5)
    g3 = oracle.make_grid(3, n, (1, 1, 1), 0.6, order)
    g2 = oracle.make_grid(2, n, (1, 1, 1), 0.6, order)
    rng = np.random.default_rng(61)
    J3 = np.zeros((3, 30)); J2 = np.zeros((3, 30))
    for _ in range(10):
        x0 = np.array([rng.uniform(0, 6), 0.0, rng.uniform(0, 5)])
        x1 = x0 + np.array([rng.uniform(-0.9, 0.9), 0.0, rng.uniform(-0.9, 0.9)])
        oracle.deposit(g3, J3, -1.0, 1.3, x0, x1, 0.0)
        oracle.deposit(g2, J2, -1.0, 1.3, x0, x1, 0.0)
    assert np.max(np.abs(J3[0] - J2[0])) < 1e-14
    assert np.max(np.abs(J3[2] - J2[2])) < 1e-14


@pytest.mark.parametrize("order", ORDERS)
def test_2d_out_of_plane_current_is_y_line_sum_of_3d(order):
    n3 = (6, 16, 5)
    dt = 0.6
    g3 = oracle.make_grid(3, n3, (1, 1, 1), dt, order)
    g2 = oracle.make_grid(2, (6, 1, 5), (1, 1, 1), dt, order)
    rng = np.random.default_rng(71 + order)
    for _ in range(5):
        x0 = np.array([rng.uniform(0, 6), 8.3, rng.uniform(0, 5)])
        d = rng.uniform(-0.8, 0.8, 3)
        x1 = x0 + d
        J3 = np.zeros((3, 6 * 16 * 5)); J2 = np.zeros((3, 30))
        oracle.deposit(g3, J3, -1.0, 0.7, x0, x1, 0.0)
        vy = d[1] / dt
        oracle.deposit(g2, J2, -1.0, 0.7, np.array([x0[0], 0, x0[2]]), np.array([x1[0], 0, x1[2]]), vy)
        line = J3[1].reshape(5, 16, 6).sum(axis=1).reshape(-1)
        assert np.max(np.abs(line - J2[1])) < 1e-14


@pytest.mark.parametrize("order", ORDERS)
def test_grid_sum_of_current(order):
    n = (8, 7, 6)
    dt = 0.55
    dx = (1.0, 0.8, 1.25)
    g = oracle.make_grid(3, n, dx, dt, order)
    rng = np.random.default_rng(81)
    J = np.zeros((3, 336))
    tot = np.zeros(3)
    for _ in range(10):
        x0 = rng.uniform(0, 1, 3) * np.array(n)
        d = rng.uniform(-0.9, 0.9, 3)
        w = rng.uniform(0.5, 2)
        oracle.deposit(g, J, -1.0, w, x0, x0 + d, 0.0)
        tot += -1.0 * w * d * np.array(dx) / dt / (dx[0] * dx[1] * dx[2])
    assert np.allclose(J.sum(axis=1), tot, rtol=1e-13, atol=1e-15)


@pytest.mark.parametrize("order", ORDERS)
@pytest.mark.parametrize("dim", (2, 3))
def test_whole_step_gauss_law_residual_constant(order, dim):
    from pic_inputs import uniform_box
    wl = uniform_box((6, 5, 4), 3, 0.05, 0.05, order, 9001, "cpu", tile=(2, 2, 2),
                     fields="fourier", dim=dim)
    box = wl.boxes[0]
    g = oracle.make_grid(box.dim, box.n, box.dx, box.dt, box.order)
    sp = wl.species[0].numpy()
    sp.u[:] *= 20.0          # hot, so particles cross cells
    E = np.ascontiguousarray(wl.E[0].numpy()); B = np.ascontiguousarray(wl.B[0].numpy())
    J = np.zeros_like(E)
    N = box.ncells

    def gauss():
        divE = oracle.div_j(g, E, N)     # same discrete divergence on nodes
        return divE - oracle.rho(g, [sp], N)

    r0 = gauss()
    for _ in range(4):
        oracle.pic_step(g, E, B, J, [sp])
    assert np.max(np.abs(gauss() - r0)) < 1e-13 * max(1.0, np.max(np.abs(r0)))


def test_wrap_rule():
    assert oracle.wrap(32.25, 32.0) == 0.25
    assert oracle.wrap(-0.25, 32.0) == 31.75
    assert oracle.wrap(-1e-300, 32.0) == 0.0       # rounds to L -> the point 0
    assert oracle.wrap(31.5, 32.0) == 31.5


def test_stable_sort_and_keys():
    from pic_inputs import uniform_box
    wl = uniform_box((10, 9, 7), 2, 0.01, 0.3, 1, 77, "cpu", tile=(4, 4, 4))
    box = wl.boxes[0]
    sp = wl.species[0].numpy()
    rng = np.random.default_rng(3)
    perm0 = rng.permutation(sp.x.shape[1])
    sp = _sp(sp.x[:, perm0], sp.u[:, perm0], sp.w[perm0])
    g = oracle.make_grid(3, box.n, box.dx, box.dt, 1)
    key = oracle.tile_keys(g, box.tile, sp)
    nt = [-(-box.n[d] // box.tile[d]) for d in range(3)]
    for p in range(0, sp.x.shape[1], 7):
        t = key[p]
        tx, ty, tz = t % nt[0], (t // nt[0]) % nt[1], t // (nt[0] * nt[1])
        for d, td in zip(range(3), (tx, ty, tz)):
            c = math.floor(sp.x[d, p])
            assert td * box.tile[d] <= c < (td + 1) * box.tile[d]
    perm, count, offset = oracle.stable_sort(key, nt[0] * nt[1] * nt[2])
    ref = sorted(range(len(key)), key=lambda i: key[i])
    assert list(perm) == ref
    assert offset[-1] == len(key) and (np.diff(offset) == count).all()
    assert np.array_equal(count, np.bincount(key, minlength=len(count)))


def _cells_in_tile(sp, box):
    c = np.floor(sp.x).astype(np.int64) % np.array(box.n)[:, None]
    t = np.array(box.tile)[:, None]
    return c // t, c % t


def test_cell_order_keys():
    """The within-tile cell order: its tile part is the tile id, equal keys
    mean equal cells (so a stable sort makes each cell's particles
    contiguous), and two different cells of one class that share a row along
    an axis differ by a multiple of 4 along it (the layout's promise that
    consecutive cells never deposit onto one LDS node)."""
    from pic_inputs import uniform_box
    wl = uniform_box((16, 12, 9), 3, 0.01, 0.3, 1, 79, "cpu", tile=(8, 4, 8))
    box = wl.boxes[0]
    sp = wl.species[0].numpy()
    g = oracle.make_grid(3, box.n, box.dx, box.dt, 1)
    cbits = 8                                   # 8 * 4 * 8 = 256 cells per tile
    key = oracle.cell_order_keys(g, box.tile, cbits, sp)
    assert np.array_equal(key >> (cbits + 2), oracle.tile_keys(g, box.tile, sp))
    tiles, local = _cells_in_tile(sp, box)
    cell = np.floor(sp.x).astype(np.int64)
    ids = {}
    for p in range(key.shape[0]):
        ids.setdefault(int(key[p]), set()).add(tuple(cell[:, p]))
    assert all(len(v) == 1 for v in ids.values())
    assert len(ids) == len({tuple(cell[:, p]) for p in range(key.shape[0])})
    cls = (key >> cbits) & 3
    n = key.shape[0]
    for p in range(0, n, 5):
        same = (key >> (cbits + 2) == key[p] >> (cbits + 2)) & (cls == cls[p]) & (key != key[p])
        for d in range(3):
            o = [e for e in range(3) if e != d]
            row = same & (local[o[0]] == local[o[0], p]) & (local[o[1]] == local[o[1], p])
            dd = np.abs(local[d, row] - local[d, p])
            assert (dd % 4 == 0).all() and (dd >= 4).all()
    perm = oracle.stable_perm(key)
    assert list(perm) == sorted(range(n), key=lambda i: (key[i], i))
    k = key[perm]
    change = np.nonzero(np.diff(k))[0]
    seen = set()
    for run in np.split(np.arange(n), change + 1):
        c = tuple(cell[:, perm[run[0]]])
        assert c not in seen
        seen.add(c)


def test_cell_order_keys_2d_brute():
    """2D: every cell of a 8x8 box with 4x4 tiles, one particle each; keys
    enumerate (tile, class, cell) exactly, checked cell by cell."""
    n = (8, 1, 8)
    xs, zs = np.meshgrid(np.arange(8) + 0.5, np.arange(8) + 0.5, indexing="ij")
    x = np.zeros((3, 64))
    x[0] = xs.ravel()
    x[2] = zs.ravel()
    sp = _sp(x, np.zeros((3, 64)), np.ones(64))
    g = oracle.make_grid(2, n, (1.0, 1.0, 1.0), 0.5, 1)
    key = oracle.cell_order_keys(g, (4, 1, 4), 4, sp)
    for p in range(64):
        cx, cz = int(x[0, p]), int(x[2, p])
        tile = cx // 4 + 2 * (cz // 4)
        lx, lz = cx % 4, cz % 4
        assert key[p] >> 6 == tile
        assert (key[p] >> 4) & 3 == (lx + lz) % 4
        assert key[p] & 15 == lx + 4 * lz
    assert len(set(key.tolist())) == 64


def test_quad_order():
    """Whole groups of four first: the result is a permutation that keeps
    the tile grouping of the cell order; inside each tile every aligned group
    of four of the first part shares one cell, the second part holds fewer
    than four particles of any cell, and each part keeps the cell order
    (checked against the stable cell-order permutation)."""
    from pic_inputs import uniform_box
    wl = uniform_box((16, 8, 8), 4, 0.01, 0.3, 1, 81, "cpu", tile=(8, 8, 8))
    box = wl.boxes[0]
    sp = wl.species[0].numpy()
    rng = np.random.default_rng(11)
    keep = np.sort(rng.choice(sp.x.shape[1], size=sp.x.shape[1] * 3 // 4, replace=False))
    x = sp.x[:, keep] + rng.uniform(-0.45, 0.45, size=(3, keep.size))   # drifted cells
    x = np.mod(x, np.array(box.n, float)[:, None])
    sp = _sp(x, sp.u[:, keep], sp.w[keep])
    g = oracle.make_grid(3, box.n, box.dx, box.dt, 1)
    cbits = 9
    key = oracle.cell_order_keys(g, box.tile, cbits, sp)
    base = oracle.stable_perm(key)
    perm = oracle.quad_order(key, cbits)
    n = key.shape[0]
    assert sorted(perm.tolist()) == list(range(n))
    tiles = key >> (cbits + 2)
    assert np.array_equal(tiles[perm], tiles[base])
    rank_in_base = np.empty(n, np.int64)
    rank_in_base[base] = np.arange(n)
    for t in np.unique(tiles):
        seg = perm[tiles[perm] == t]
        counts = {}
        for i in seg:
            counts[key[i]] = counts.get(key[i], 0) + 1
        whole = sum(c - c % 4 for c in counts.values())
        first, second = seg[:whole], seg[whole:]
        for q in range(0, whole, 4):
            assert len(set(key[first[q:q + 4]].tolist())) == 1
        rest = {}
        for i in second:
            rest[key[i]] = rest.get(key[i], 0) + 1
        assert all(v < 4 and v == counts[k] % 4 for k, v in rest.items())
        assert (np.diff(rank_in_base[first]) > 0).all()
        assert (np.diff(rank_in_base[second]) > 0).all()


def test_tile_cell_keys():
    """Cell order without classes: the tile part is the tile id, equal keys
    mean equal cells, and within a tile the keys enumerate the cells x
    fastest (checked on every cell of a 2-tile box)."""
    n = (8, 4, 8)
    g = oracle.make_grid(3, n, (1.0, 1.0, 1.0), 0.5, 1)
    cells = np.stack(np.meshgrid(*[np.arange(k) for k in n], indexing="ij")).reshape(3, -1)
    x = cells + 0.25
    sp = _sp(x, np.zeros_like(x), np.ones(x.shape[1]))
    key = oracle.tile_cell_keys(g, (8, 4, 4), 7, sp)
    assert np.array_equal(key >> 7, oracle.tile_keys(g, (8, 4, 4), sp))
    assert len(set(key.tolist())) == x.shape[1]
    order = np.argsort(key, kind="stable")
    first_tile = order[:128]
    c = cells[:, first_tile]
    assert np.array_equal(c[0], np.tile(np.arange(8), 16))
    assert np.array_equal(c[1], np.tile(np.repeat(np.arange(4), 8), 4))
    assert np.array_equal(c[2], np.repeat(np.arange(4), 32))
