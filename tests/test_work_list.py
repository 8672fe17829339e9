"""The host-built 2D work list (lbm_ms_work_list, no GPU needed), on several masks and every 2D
launch shape, fixed and packed: every fluid node is the own node of exactly one tile; no tile
has more own nodes than lanes or rows than its moment tile; each tile's halo lists exactly the
fluid axis neighbours of its own nodes that are not its own (y periodic, x bounded); tiles come
in row-band order.  The GPU parity tests cannot see a node updated twice (it would write the same
value twice), so these invariants are checked here."""

import numpy as np
import pytest

from paper_1809_01600_amd import inputs, lbm_ms


def _masks():
    rng = np.random.default_rng(40)
    out = [("random 0.5", (rng.random((37, 150)) < 0.5).astype(np.uint8)),
           ("random 0.2", (rng.random((64, 64)) < 0.2).astype(np.uint8)),
           ("all fluid", np.zeros((29, 70), dtype=np.uint8)),
           ("short", (rng.random((3, 130)) < 0.3).astype(np.uint8))]
    c = inputs.porous_2d(n=256, seed=5)
    out.append(("disks 256", np.ascontiguousarray(c.mask()[0])))
    return out


@pytest.mark.parametrize("name,solid", _masks(), ids=lambda v: v if isinstance(v, str) else "")
@pytest.mark.parametrize("lat", ["D2Q9", "D2Q5"])
def test_work_list_invariants(name, solid, lat):
    ny, nx = solid.shape
    fluid = solid == 0
    for ty, rows in lbm_ms.tile_options(lbm_ms.LATTICES[lat]):
        tiles, ent = lbm_ms.work_list(lat, solid, ty, rows)
        rt = rows if rows > 0 else ty
        owner = np.full((ny, nx), -1, dtype=np.int64)
        count = np.zeros((ny, nx), dtype=np.int64)
        for t, (x0, y0, inst, _, oo, on, ho, hn) in enumerate(tiles):
            assert inst == 0 and 0 < on <= 32 * ty and ho == oo + on
            own = set()
            for e in ent[oo:oo + on]:
                cx, cy = int(e & 255), int(e >> 8)
                assert 1 <= cx <= 64 and 1 <= cy <= rt
                x, y = x0 + cx - 1, y0 + cy - 1
                assert x < nx and y < ny and fluid[y, x]
                count[y, x] += 1
                owner[y, x] = t
                own.add((cx, cy))
            want = set()
            for cx, cy in own:
                for dx, dy in ((1, 0), (-1, 0), (0, 1), (0, -1)):
                    hx, hy = cx + dx, cy + dy
                    gx, gy = x0 + hx - 1, (y0 + hy - 1) % ny
                    if 0 <= gx < nx and fluid[gy, gx] and (hx, hy) not in own:
                        want.add((hx, hy))
            got = [(int(e & 255), int(e >> 8)) for e in ent[ho:ho + hn]]
            assert len(got) == len(set(got)) and set(got) == want, (ty, rows, t)
        assert np.array_equal(count, fluid.astype(np.int64)), (ty, rows)
        order = [(int(y0), int(x0)) for x0, y0, *_ in tiles]
        if rows > 0:
            assert order == sorted(order)
        else:  # fixed tiles: row bands, then strips (split parts stay together)
            assert [(y // ty, x) for y, x in order] == sorted((y // ty, x) for y, x in order)


def test_packed_tiles_fill_the_lanes():
    """Packed tiles never split, so on the benchmark's kind of geometry they need fewer
    workgroups than fixed 64 x 8 tiles for the same nodes."""
    solid = np.ascontiguousarray(inputs.porous_2d(n=512, seed=2).mask()[0])
    fixed, _ = lbm_ms.work_list("D2Q9", solid, 8, 0)
    packed, _ = lbm_ms.work_list("D2Q9", solid, 8, 12)
    assert fixed[:, 5].sum() == packed[:, 5].sum()
    assert len(packed) < 0.8 * len(fixed)
    assert packed[:, 5].mean() > 1.25 * fixed[:, 5].mean()


def test_rejects_3d_and_unknown_shapes():
    solid = np.zeros((8, 70), dtype=np.uint8)
    with pytest.raises(lbm_ms.LbmMsError):
        lbm_ms.work_list("D3Q19", solid, 8, 0)
    with pytest.raises(lbm_ms.LbmMsError):
        lbm_ms.work_list("D2Q9", solid, 8, 5)
