"""The AA access pattern of LBM_VARIANT_AA, checked on the CPU on small lattices: the index rules
of csrc/lbm_aa.hip (which slot each node reads and writes in even and odd steps, bounce-back at
walls) written out here in the same form, applied with an arbitrary node-local map in place of the
collision, must (1) give every node the populations that pull streaming with half-way bounce-back
gives it (Eq. LBE), step after step, and (2) touch every storage location from one node only within
a step, so that the in-place update has no race.  The GPU tests check the kernels themselves
against the oracle; this pins the access pattern they implement."""
import numpy as np
import pytest

CX = [0, 1, 0, -1, 0, 1, -1, -1, 1]
CY = [0, 0, 1, 0, -1, 1, 1, -1, -1]
OPP = [0, 3, 4, 1, 2, 7, 8, 5, 6]


def _neighbour(x, y, dx, dy, nx, ny, walls):
    xn, yn = (x + dx) % nx, y + dy
    if yn < 0 or yn >= ny:
        if walls:
            return None
        yn %= ny
    return xn, yn


def _pull(fs, nx, ny, walls):
    """Pull streaming of post-collision populations fs[i][y][x] with half-way bounce-back."""
    f = np.empty_like(fs)
    for y in range(ny):
        for x in range(nx):
            for i in range(9):
                s = _neighbour(x, y, -CX[i], -CY[i], nx, ny, walls)
                f[i, y, x] = fs[i, s[1], s[0]] if s is not None else fs[OPP[i], y, x]
    return f


def _aa_read(x, y, i, odd, nx, ny, walls):
    if not odd:
        return (i, y, x)
    s = _neighbour(x, y, -CX[i], -CY[i], nx, ny, walls)
    return (OPP[i], s[1], s[0]) if s is not None else (i, y, x)


def _aa_write(x, y, i, odd, nx, ny, walls):
    if not odd:
        return (OPP[i], y, x)
    d = _neighbour(x, y, CX[i], CY[i], nx, ny, walls)
    return (i, d[1], d[0]) if d is not None else (OPP[i], y, x)


@pytest.mark.parametrize("walls", [False, True], ids=["periodic", "walls"])
@pytest.mark.parametrize("nx,ny", [(7, 5), (4, 3), (1, 2), (3, 1)])
def test_aa_pattern_is_pull_streaming_without_races(walls, nx, ny):
    rng = np.random.default_rng(nx * 10 + ny + (100 if walls else 0))
    steps = 5
    f = rng.random((9, ny, nx))          # f_i(x, 0), the natural layout of the AA buffer
    maps = [(rng.random((9, ny, nx)) + 0.5, rng.random((9, ny, nx))) for _ in range(steps)]
    A = f.copy()
    ref = f.copy()
    for t in range(steps):
        odd = t % 2 == 1
        a, b = maps[t]
        # reference: collide the current populations with the node-local map, then pull
        ref = _pull(ref * a + b, nx, ny, walls)
        # AA: each node reads its populations, applies the same map and writes them back
        readers, writers = {}, {}
        out = A.copy()
        for y in range(ny):
            for x in range(nx):
                g = np.empty(9)
                for i in range(9):
                    loc = _aa_read(x, y, i, odd, nx, ny, walls)
                    readers.setdefault(loc, set()).add((x, y))
                    g[i] = A[loc]
                o = g * a[:, y, x] + b[:, y, x]
                for i in range(9):
                    loc = _aa_write(x, y, i, odd, nx, ny, walls)
                    assert loc not in writers, ("two writers", t, loc)
                    writers[loc] = (x, y)
                    out[loc] = o[i]
        # a location written in this step is read, if at all, only by the node that writes it
        for loc, w in writers.items():
            assert readers.get(loc, {w}) <= {w}, ("read by another node", t, loc)
        A = out
        # the populations at time t + 1, gathered from the AA buffer in the next step's layout
        g = np.empty_like(A)
        for y in range(ny):
            for x in range(nx):
                for i in range(9):
                    g[i, y, x] = A[_aa_read(x, y, i, (t + 1) % 2 == 1, nx, ny, walls)]
        np.testing.assert_array_equal(g, ref)
