"""The room an S-BKI insert reserves in the map before it knows how many class
blocks it will allocate (host logic of the insert, checked here on the CPU).

The insert reserves, per class, min(targets, 27 x the class's (class, block)
slots) new class blocks: a row reaches voxels only in its own block and the 26
around it (reach R <= B), so a class's rows touch at most 27 blocks per block
they occupy, and never more blocks than the targets (the 27-neighbourhoods of
all occupied blocks).  The class blocks an insert into an empty map needs are
the (block, class) pairs that receive a non-zero sum of Eq. (7).  Here those
pairs come from the oracle's map (every voxel whose alpha_k exceeds alpha0),
the slots and targets from the oracle's training rows, and the bound must hold
on every scene; the checks also guard the bound's two halves separately.
"""
import numpy as np
import pytest

import oracle
import scenes


def _rows(sc):
    p = sc.params
    xs, ys = [], []
    for s in sc.scans:
        tx, ty, _ = oracle.training_set(s.xyz, s.label, s.origin, p.free_step, p.K, p.free_class)
        xs.append(tx)
        ys.append(ty)
    return np.concatenate(xs), np.concatenate(ys)


def _blocks(ijk, B):
    return np.floor_divide(ijk, B)


def _bound_and_actual(sc):
    p = sc.params
    B = p.block_size
    tx, ty = _rows(sc)
    rb = _blocks(oracle.voxel_coords(tx, p.res), B)            # row blocks
    slots = {(int(c), tuple(b)) for c, b in zip(ty, rb.tolist())}
    per_class = {}
    for c, _ in slots:
        per_class[c] = per_class.get(c, 0) + 1
    occupied = {b for _, b in slots}
    targets = {(b[0] + dx, b[1] + dy, b[2] + dz) for b in occupied
               for dx in (-1, 0, 1) for dy in (-1, 0, 1) for dz in (-1, 0, 1)}
    n_t = len(targets)
    bound = sum(min(n_t, 27 * n) for n in per_class.values())
    # (block, class) pairs with a non-zero sum in a fresh map
    om = oracle.OracleMap.from_params(p)
    for s in sc.scans:
        om.insert_scan(s.xyz, s.label, s.origin, p.free_step, p.free_class)
    ijk, alpha, _, _ = om.export()
    a0 = np.float64(np.float32(p.alpha0))
    vb = _blocks(ijk, B)
    pairs = set()
    for k in range(p.K):
        hit = alpha[:, k] > a0
        pairs |= {(k, tuple(b)) for b in vb[hit].tolist()}
    per_class_pairs = {}
    for k, _ in pairs:
        per_class_pairs[k] = per_class_pairs.get(k, 0) + 1
    return bound, len(pairs), per_class, per_class_pairs, n_t, pairs, targets


@pytest.mark.parametrize("make", [
    lambda: scenes.make_config(0),
    lambda: scenes.random_points_scene(11, 600, K=5, extent=1.2, res=0.1, l=0.3,
                                       free_step=0.2, block_size=4, origin=(1.0, -0.5, 0.4)),
    # reach equal to the block size (R = 2 at B = 2, R = 4 at B = 4): the widest
    # reach the insert accepts (it refuses R > B, where rows pass the 26 blocks)
    lambda: scenes.random_points_scene(12, 400, K=3, extent=0.8, res=0.2, l=0.45,
                                       free_step=0.0, block_size=2),
    lambda: scenes.random_points_scene(13, 300, K=4, extent=1.0, res=0.1, l=0.44,
                                       free_step=0.3, block_size=4, origin=(0.2, 0.1, -0.6)),
])
def test_reserved_class_blocks_bound_the_allocation(make):
    sc = make()
    p = sc.params
    reach = int(np.ceil(np.float64(np.float32(p.l)) / np.float64(np.float32(p.res)) + 0.5)) - 1
    assert reach <= p.block_size   # (a shape the insert accepts)
    bound, actual, per_class, per_class_pairs, n_t, pairs, targets = _bound_and_actual(sc)
    assert actual > 0
    assert actual <= bound
    for k, n in per_class_pairs.items():
        assert n <= min(n_t, 27 * per_class.get(k, 0)), k   # no class outgrows its own share
    # every allocated block is a target (the neighbourhood of an occupied block)
    assert {b for _, b in pairs} <= targets
